"""Thin ctypes binding of libsf.so (include/sf.h): the same calls, with
argument marshalling only.  Every step of an SF operation runs in the HIP
kernels of the library; PyTorch only provides device memory and streams.

If libsf.so is missing, :func:`lib` raises -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsf.so")

# enums of sf.h
SF_F64, SF_F32, SF_I32, SF_I64, SF_F64_I32, SF_F16, SF_BF16 = 0, 1, 2, 3, 4, 5, 6
SF_REPLACE, SF_SUM, SF_MAX, SF_MIN, SF_MAXLOC, SF_MINLOC, SF_PROD = 0, 1, 2, 3, 4, 5, 6
SF_REDUCE_AUTO, SF_REDUCE_ATOMIC, SF_REDUCE_DETERMINISTIC = 0, 1, 2
SF_COPY_VALUES, SF_USE_POINTER, SF_OWN_POINTER = 0, 1, 2
SF_KIND_BCAST, SF_KIND_REDUCE, SF_KIND_FETCH_AND_OP = 0, 1, 2
SF_PATTERN_GENERIC, SF_PATTERN_CONTIGUOUS, SF_PATTERN_3D = 0, 1, 2
ERRORS = {0: "SF_OK", -1: "SF_ERR_ARG", -2: "SF_ERR_DUP_LEAF", -3: "SF_ERR_NOT_SETUP",
          -4: "SF_ERR_UNSUPPORTED", -5: "SF_ERR_HIP", -6: "SF_ERR_OOM", -7: "SF_ERR_MISMATCH",
          -8: "SF_ERR_BUSY", -9: "SF_ERR_SCRATCH"}
SF_NOALLOC_SCRATCH_BYTES = 64 << 20
OPS = {"replace": SF_REPLACE, "sum": SF_SUM, "max": SF_MAX, "min": SF_MIN, "maxloc": SF_MAXLOC,
       "minloc": SF_MINLOC, "prod": SF_PROD}
MODES = {"auto": SF_REDUCE_AUTO, "atomic": SF_REDUCE_ATOMIC, "deterministic": SF_REDUCE_DETERMINISTIC}
ELEM_SIZE = {SF_F64: 8, SF_F32: 4, SF_I32: 4, SF_I64: 8, SF_F64_I32: 16, SF_F16: 2, SF_BF16: 2}

EXPORTS = [
    "sf_create", "sf_setup", "sf_set_reduce_mode", "sf_bcast_begin", "sf_bcast_end",
    "sf_reduce_begin", "sf_reduce_end", "sf_reduce_begin_noalloc", "sf_fetch_and_op_begin", "sf_fetch_and_op_end",
    "sf_get_multi_sf", "sf_gather_begin", "sf_gather_end", "sf_scatter_begin", "sf_scatter_end",
    "sf_csr_create", "sf_csr_transpose", "sf_csr_spmv", "sf_csr_destroy", "sf_spmv", "sf_spmv_transpose",
    "sf_get_graph", "sf_create_embedded_root_sf", "sf_create_embedded_leaf_sf", "sf_compose", "sf_compose_inverse",
    "sf_batch_create", "sf_batch_launch", "sf_batch_launch_separate", "sf_batch_graph_capture",
    "sf_batch_graph_launch", "sf_batch_autotune", "sf_batch_get_config", "sf_batch_set_config",
    "sf_batch_destroy", "sf_get_info", "sf_get_segment", "sf_error_string", "sf_last_hip_error",
    "sf_destroy",
]


class SfError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = ERRORS.get(code, str(code))
        if code == -5:
            msg += f" (hipError {lib().sf_last_hip_error()})"
        super().__init__(f"{where}: {msg}")

    def __reduce__(self):
        return (SfError, (self.code, str(self)))


class SfNode(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("index", ctypes.c_int64)]


class SfUnit(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("bs", ctypes.c_int32)]


class SfSetupOpts(ctypes.Structure):
    _fields_ = [("reduce_mode", ctypes.c_int32), ("use_patterns", ctypes.c_int32),
                ("analyze_only", ctypes.c_int32), ("partition", ctypes.c_int32),
                ("hot_path", ctypes.c_int32)]


class SfPattern(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("start", ctypes.c_int32), ("dx", ctypes.c_int32),
                ("dy", ctypes.c_int32), ("dz", ctypes.c_int32), ("sy", ctypes.c_int32),
                ("sz", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SfSegmentInfo(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("nleaves", ctypes.c_int64), ("root", SfPattern),
                ("leaf", SfPattern)]


class SfInfo(ctypes.Structure):
    _fields_ = [("nroots", ctypes.c_int64), ("nleaves", ctypes.c_int64), ("leafspace", ctypes.c_int64),
                ("nsegments", ctypes.c_int64), ("nroots_touched", ctypes.c_int64),
                ("max_degree", ctypes.c_int64), ("has_dup_roots", ctypes.c_int32),
                ("reduce_mode", ctypes.c_int32), ("nhot", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("hot_roots", ctypes.c_int64)]


class SfBatchItem(ctypes.Structure):
    _fields_ = [("sf", ctypes.c_void_p), ("unit", SfUnit), ("kind", ctypes.c_int32),
                ("op", ctypes.c_int32), ("rootdata", ctypes.c_void_p), ("leafdata", ctypes.c_void_p),
                ("leafupdate", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libsf.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is missing: build it with `python -m paper_2102_13018_amd.build`")
        L = ctypes.CDLL(_SO)
        p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.sf_create.argtypes = [i64, i64, p, i32, p, i32, ctypes.POINTER(p)]
        L.sf_setup.argtypes = [p, ctypes.POINTER(SfSetupOpts)]
        L.sf_set_reduce_mode.argtypes = [p, i32]
        for name in ("sf_bcast_begin", "sf_bcast_end", "sf_reduce_begin", "sf_reduce_end",
                     "sf_reduce_begin_noalloc"):
            getattr(L, name).argtypes = [p, SfUnit, p, p, i32, p]
        for name in ("sf_fetch_and_op_begin", "sf_fetch_and_op_end"):
            getattr(L, name).argtypes = [p, SfUnit, p, p, p, i32, p]
        L.sf_get_graph.argtypes = [p, p, p]
        L.sf_create_embedded_root_sf.argtypes = [p, i64, p, ctypes.POINTER(p)]
        L.sf_create_embedded_leaf_sf.argtypes = [p, i64, p, ctypes.POINTER(p)]
        L.sf_compose.argtypes = [p, p, ctypes.POINTER(p)]
        L.sf_compose_inverse.argtypes = [p, p, ctypes.POINTER(p)]
        L.sf_get_multi_sf.argtypes = [p, ctypes.POINTER(p)]
        for name in ("sf_gather_begin", "sf_gather_end", "sf_scatter_begin", "sf_scatter_end"):
            getattr(L, name).argtypes = [p, SfUnit, p, p, p]
        L.sf_csr_create.argtypes = [i64, i64, p, p, p, ctypes.POINTER(p)]
        L.sf_csr_transpose.argtypes = [p, ctypes.POINTER(p)]
        L.sf_csr_spmv.argtypes = [p, p, p, i32, p]
        L.sf_csr_destroy.argtypes = [ctypes.POINTER(p)]
        L.sf_spmv.argtypes = [p, p, p, p, p, p, p, p]
        L.sf_spmv_transpose.argtypes = [p, p, p, p, p, p, p]
        L.sf_batch_create.argtypes = [i32, ctypes.POINTER(SfBatchItem), ctypes.POINTER(p)]
        L.sf_batch_launch.argtypes = [p, p]
        L.sf_batch_launch_separate.argtypes = [p, p]
        L.sf_batch_graph_capture.argtypes = [p, i32, p]
        L.sf_batch_graph_launch.argtypes = [p, p]
        L.sf_batch_autotune.argtypes = [p, ctypes.c_char_p, p]
        L.sf_batch_get_config.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.sf_batch_set_config.argtypes = [p, i32, i32]
        L.sf_batch_destroy.argtypes = [ctypes.POINTER(p)]
        L.sf_get_info.argtypes = [p, ctypes.POINTER(SfInfo)]
        L.sf_get_segment.argtypes = [p, i64, ctypes.POINTER(SfSegmentInfo)]
        L.sf_error_string.argtypes = [ctypes.c_int]
        L.sf_error_string.restype = ctypes.c_char_p
        L.sf_last_hip_error.argtypes = []
        L.sf_destroy.argtypes = [ctypes.POINTER(p)]
        for name in EXPORTS:
            if name != "sf_error_string":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc, where):
    if rc != 0:
        raise SfError(rc, where)


def _ptr(x):
    """Device address of a torch tensor, or an int address."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


_UNIT_TORCH = {SF_F64: "torch.float64", SF_F32: "torch.float32", SF_I32: "torch.int32", SF_I64: "torch.int64",
               SF_F16: "torch.float16", SF_BF16: "torch.bfloat16"}


def check_buffer(x, nunits, unit, what):
    """Raise SfError(SF_ERR_ARG) unless a tensor argument can hold ``nunits``
    units: a contiguous device tensor of at least that many bytes whose dtype
    is the unit's (or a byte tensor carrying raw units, e.g. MAXLOC pairs).
    Integer addresses are passed through unchecked."""
    if x is None or isinstance(x, int):
        return
    if not getattr(x, "is_cuda", False):
        raise SfError(-1, f"{what}: not a device tensor")
    if not x.is_contiguous():
        raise SfError(-1, f"{what}: not contiguous")
    need = int(nunits) * int(unit.bs) * ELEM_SIZE[int(unit.dtype)]
    have = int(x.numel()) * int(x.element_size())
    if have < need:
        raise SfError(-1, f"{what}: {have} bytes, the unit needs {need}")
    dt = str(x.dtype)
    if dt not in ("torch.uint8", "torch.int8") and dt != _UNIT_TORCH.get(int(unit.dtype)):
        raise SfError(-1, f"{what}: dtype {dt} does not match the unit")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def unit_of(t, dtype=None, bs=None):
    """sf_unit of a torch tensor: dtype from the tensor, bs = elements per row.
    MAXLOC pairs are passed explicitly (dtype=SF_F64_I32)."""
    import torch
    if dtype is None:
        dtype = {torch.float64: SF_F64, torch.float32: SF_F32, torch.int32: SF_I32,
                 torch.int64: SF_I64, torch.float16: SF_F16, torch.bfloat16: SF_BF16}[t.dtype]
    if bs is None:
        bs = 1 if t.dim() <= 1 else int(np.prod(t.shape[1:]))
    return SfUnit(dtype, bs)


class StarForest:
    """One device's share of a star forest (PetscSF, Section 3.1).

    ``iroot[i]`` is the root of leaf i, ``ilocal[i]`` its slot (None for a
    contiguous leaf space), ``ranks[i]`` its segment label (None = one
    segment)."""

    def __init__(self, nroots, iroot, ilocal=None, ranks=None):
        iroot = np.ascontiguousarray(iroot, dtype=np.int64)
        n = iroot.size
        nodes = np.zeros((n, 2), dtype=np.int64)
        nodes[:, 1] = iroot
        if ranks is not None:
            nodes[:, 0] = np.asarray(ranks, dtype=np.int64)
        il = None if ilocal is None else np.ascontiguousarray(ilocal, dtype=np.int64)
        h = ctypes.c_void_p()
        rc = lib().sf_create(int(nroots), n,
                             None if il is None else il.ctypes.data_as(ctypes.c_void_p), SF_COPY_VALUES,
                             nodes.ctypes.data_as(ctypes.c_void_p), SF_COPY_VALUES, ctypes.byref(h))
        check(rc, "sf_create")
        self.h = h
        self.nroots = int(nroots)
        self.nleaves = n
        self.leafspace = n if il is None else (int(il.max()) + 1 if n else 0)

    def setup(self, reduce_mode="auto", use_patterns=True, analyze_only=False, partition="auto",
              hot_path="auto"):
        onoff = {"auto": 0, True: 1, False: 2, "on": 1, "off": 2}
        o = SfSetupOpts(MODES.get(reduce_mode, reduce_mode), int(bool(use_patterns)),
                        int(bool(analyze_only)), onoff[partition], onoff[hot_path])
        check(lib().sf_setup(self.h, ctypes.byref(o)), "sf_setup")
        return self

    def set_reduce_mode(self, mode):
        check(lib().sf_set_reduce_mode(self.h, MODES.get(mode, mode)), "sf_set_reduce_mode")

    # ------------------------------------------------------------ begin/end
    def _check(self, unit, root, leaf, upd=None):
        check_buffer(root, self.nroots, unit, "rootdata")
        check_buffer(leaf, self.leafspace, unit, "leafdata")
        check_buffer(upd, self.leafspace, unit, "leafupdate")

    def bcast_begin(self, unit, root, leaf, op="replace", stream=None):
        self._check(unit, root, leaf)
        check(lib().sf_bcast_begin(self.h, unit, _ptr(root), _ptr(leaf), OPS.get(op, op), _stream(stream)),
              "sf_bcast_begin")

    def bcast_end(self, unit, root, leaf, op="replace", stream=None):
        check(lib().sf_bcast_end(self.h, unit, _ptr(root), _ptr(leaf), OPS.get(op, op), _stream(stream)),
              "sf_bcast_end")

    def reduce_begin(self, unit, leaf, root, op="sum", stream=None):
        self._check(unit, root, leaf)
        check(lib().sf_reduce_begin(self.h, unit, _ptr(leaf), _ptr(root), OPS.get(op, op), _stream(stream)),
              "sf_reduce_begin")

    def reduce_begin_noalloc(self, unit, leaf, root, op="sum", stream=None):
        self._check(unit, root, leaf)
        check(lib().sf_reduce_begin_noalloc(self.h, unit, _ptr(leaf), _ptr(root), OPS.get(op, op),
                                            _stream(stream)), "sf_reduce_begin_noalloc")

    def reduce_end(self, unit, leaf, root, op="sum", stream=None):
        check(lib().sf_reduce_end(self.h, unit, _ptr(leaf), _ptr(root), OPS.get(op, op), _stream(stream)),
              "sf_reduce_end")

    def fetch_and_op_begin(self, unit, root, leaf, leafupdate, op="sum", stream=None):
        self._check(unit, root, leaf, leafupdate)
        check(lib().sf_fetch_and_op_begin(self.h, unit, _ptr(root), _ptr(leaf), _ptr(leafupdate),
                                          OPS.get(op, op), _stream(stream)), "sf_fetch_and_op_begin")

    def fetch_and_op_end(self, unit, root, leaf, leafupdate, op="sum", stream=None):
        check(lib().sf_fetch_and_op_end(self.h, unit, _ptr(root), _ptr(leaf), _ptr(leafupdate),
                                        OPS.get(op, op), _stream(stream)), "sf_fetch_and_op_end")

    # ------------------------------------------------- begin + end helpers
    def bcast(self, root, leaf, op="replace", unit=None, stream=None):
        unit = unit or unit_of(root)
        self.bcast_begin(unit, root, leaf, op, stream)
        self.bcast_end(unit, root, leaf, op, stream)
        return leaf

    def reduce(self, leaf, root, op="sum", unit=None, stream=None):
        unit = unit or unit_of(root)
        self.reduce_begin(unit, leaf, root, op, stream)
        self.reduce_end(unit, leaf, root, op, stream)
        return root

    def fetch_and_op(self, root, leaf, leafupdate, op="sum", unit=None, stream=None):
        unit = unit or unit_of(root)
        self.fetch_and_op_begin(unit, root, leaf, leafupdate, op, stream)
        self.fetch_and_op_end(unit, root, leaf, leafupdate, op, stream)
        return root, leafupdate

    # -------------------------------------------------------- composition
    @classmethod
    def _wrap(cls, h):
        """A StarForest around a new handle from the library (owned)."""
        sf = cls.__new__(cls)
        sf.h = h
        inf = SfInfo()
        lib().sf_get_info(h, ctypes.byref(inf))  # (not set up: sizes are still filled in)
        sf.nroots, sf.nleaves, sf.leafspace = int(inf.nroots), int(inf.nleaves), int(inf.leafspace)
        return sf

    def graph(self):
        """(ilocal, iroot, ranks) of the SF as given to sf_create."""
        il = np.zeros(self.nleaves, np.int64)
        nodes = np.zeros((self.nleaves, 2), np.int64)
        check(lib().sf_get_graph(self.h, il.ctypes.data_as(ctypes.c_void_p), nodes.ctypes.data_as(ctypes.c_void_p)),
              "sf_get_graph")
        return il, nodes[:, 1].copy(), nodes[:, 0].copy()

    def embedded_root_sf(self, roots):
        r = np.ascontiguousarray(roots, np.int64)
        h = ctypes.c_void_p()
        check(lib().sf_create_embedded_root_sf(self.h, r.size, r.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)),
              "sf_create_embedded_root_sf")
        return StarForest._wrap(h)

    def embedded_leaf_sf(self, leaves):
        r = np.ascontiguousarray(leaves, np.int64)
        h = ctypes.c_void_p()
        check(lib().sf_create_embedded_leaf_sf(self.h, r.size, r.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)),
              "sf_create_embedded_leaf_sf")
        return StarForest._wrap(h)

    def compose(self, b):
        h = ctypes.c_void_p()
        check(lib().sf_compose(self.h, b.h, ctypes.byref(h)), "sf_compose")
        return StarForest._wrap(h)

    def compose_inverse(self, b):
        h = ctypes.c_void_p()
        check(lib().sf_compose_inverse(self.h, b.h, ctypes.byref(h)), "sf_compose_inverse")
        return StarForest._wrap(h)

    # ------------------------------------------ multi-SF, Gather, Scatter
    def multi_sf(self):
        """The multi-SF (a StarForest view of a handle this SF owns)."""
        h = ctypes.c_void_p()
        check(lib().sf_get_multi_sf(self.h, ctypes.byref(h)), "sf_get_multi_sf")
        m = StarForest.__new__(StarForest)
        m.h, m.nroots, m.nleaves, m.leafspace, m._owner = h, self.nleaves, self.nleaves, self.leafspace, self
        return m

    def gather(self, leaf, multiroot, unit=None, stream=None):
        unit = unit or unit_of(leaf)
        check_buffer(leaf, self.leafspace, unit, "leafdata")
        check_buffer(multiroot, self.nleaves, unit, "multirootdata")
        check(lib().sf_gather_begin(self.h, unit, _ptr(leaf), _ptr(multiroot), _stream(stream)), "sf_gather_begin")
        check(lib().sf_gather_end(self.h, unit, _ptr(leaf), _ptr(multiroot), _stream(stream)), "sf_gather_end")
        return multiroot

    def scatter(self, multiroot, leaf, unit=None, stream=None):
        unit = unit or unit_of(leaf)
        check_buffer(leaf, self.leafspace, unit, "leafdata")
        check_buffer(multiroot, self.nleaves, unit, "multirootdata")
        check(lib().sf_scatter_begin(self.h, unit, _ptr(multiroot), _ptr(leaf), _stream(stream)),
              "sf_scatter_begin")
        check(lib().sf_scatter_end(self.h, unit, _ptr(multiroot), _ptr(leaf), _stream(stream)), "sf_scatter_end")
        return leaf

    # ---------------------------------------------------------- inspection
    def info(self):
        inf = SfInfo()
        check(lib().sf_get_info(self.h, ctypes.byref(inf)), "sf_get_info")
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def segment(self, s):
        seg = SfSegmentInfo()
        check(lib().sf_get_segment(self.h, int(s), ctypes.byref(seg)), "sf_get_segment")
        return {"rank": seg.rank, "nleaves": seg.nleaves, "root": seg.root.as_dict(),
                "leaf": seg.leaf.as_dict()}

    def destroy(self):
        if getattr(self, "_owner", None) is not None:  # a multi-SF: its owner frees it
            return
        if getattr(self, "h", None) and self.h.value:
            lib().sf_destroy(ctypes.byref(self.h))

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Csr:
    """A CSR matrix of f64 values on the device (sf_csr_*): the diagonal or
    off-diagonal block of a row-distributed matrix (Section 4.1)."""

    def __init__(self, nrows, ncols, rowptr, colidx, values, _handle=None):
        self.nrows, self.ncols = int(nrows), int(ncols)
        if _handle is not None:
            self.h = _handle
            return
        rp = np.ascontiguousarray(rowptr, np.int64)
        ci = np.ascontiguousarray(colidx, np.int32)
        va = np.ascontiguousarray(values, np.float64)
        h = ctypes.c_void_p()
        check(lib().sf_csr_create(self.nrows, self.ncols, rp.ctypes.data_as(ctypes.c_void_p),
                                  ci.ctypes.data_as(ctypes.c_void_p), va.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(h)), "sf_csr_create")
        self.h = h

    def transpose(self):
        h = ctypes.c_void_p()
        check(lib().sf_csr_transpose(self.h, ctypes.byref(h)), "sf_csr_transpose")
        return Csr(self.ncols, self.nrows, None, None, None, _handle=h)

    def spmv(self, x, y, accumulate=False, stream=None):
        check_buffer(x, self.ncols, SfUnit(SF_F64, 1), "x")
        check_buffer(y, self.nrows, SfUnit(SF_F64, 1), "y")
        check(lib().sf_csr_spmv(self.h, _ptr(x), _ptr(y), int(bool(accumulate)), _stream(stream)), "sf_csr_spmv")
        return y

    def destroy(self):
        if getattr(self, "h", None) and self.h.value:
            lib().sf_csr_destroy(ctypes.byref(self.h))

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def spmv(sf, A, B, x, lvec, y, stream=None, comm_stream=None):
    """y = A x + B lvec with lvec = SFBcast(x) overlapped with A x (sf_spmv):
    the Bcast on comm_stream, the products on stream."""
    u = SfUnit(SF_F64, 1)
    check_buffer(x, sf.nroots, u, "x")
    check_buffer(lvec, sf.leafspace, u, "lvec")
    check_buffer(y, A.nrows, u, "y")
    check(lib().sf_spmv(sf.h, A.h, B.h, _ptr(x), _ptr(lvec), _ptr(y), _stream(stream), _stream(comm_stream)),
          "sf_spmv")
    return y


def spmv_transpose(sf, At, Bt, x, lvec, y, stream=None):
    """y = A^T x + SFReduce_SUM(B^T x) (sf_spmv_transpose)."""
    u = SfUnit(SF_F64, 1)
    check_buffer(x, At.ncols, u, "x")
    check_buffer(lvec, sf.leafspace, u, "lvec")
    check_buffer(y, sf.nroots, u, "y")
    check(lib().sf_spmv_transpose(sf.h, At.h, Bt.h, _ptr(x), _ptr(lvec), _ptr(y), _stream(stream)),
          "sf_spmv_transpose")
    return y


class Batch:
    """A batch of SF operations run in one kernel launch (sf_batch_*).
    items: list of (StarForest, unit, kind, op, root_tensor, leaf_tensor) or,
    for kind "fetch_and_op", (..., root, leaf, leafupdate)."""

    def __init__(self, items):
        arr = (SfBatchItem * len(items))()
        self._keep = []
        for k, item in enumerate(items):
            sf, unit, kind, op, root, leaf = item[:6]
            upd = item[6] if len(item) > 6 else None
            sf._check(unit, root, leaf, upd)
            kind = {"bcast": SF_KIND_BCAST, "reduce": SF_KIND_REDUCE,
                    "fetch_and_op": SF_KIND_FETCH_AND_OP}.get(kind, kind)
            arr[k] = SfBatchItem(sf.h.value, unit, kind, OPS.get(op, op), _ptr(root), _ptr(leaf), _ptr(upd))
            self._keep.append((sf, root, leaf, upd))
        h = ctypes.c_void_p()
        check(lib().sf_batch_create(len(items), arr, ctypes.byref(h)), "sf_batch_create")
        self.h = h

    def launch(self, stream=None):
        check(lib().sf_batch_launch(self.h, _stream(stream)), "sf_batch_launch")

    def launch_separate(self, stream=None):
        check(lib().sf_batch_launch_separate(self.h, _stream(stream)), "sf_batch_launch_separate")

    def graph_capture(self, mode=0, stream=None):
        check(lib().sf_batch_graph_capture(self.h, int(mode), _stream(stream)), "sf_batch_graph_capture")

    def graph_launch(self, stream=None):
        check(lib().sf_batch_graph_launch(self.h, _stream(stream)), "sf_batch_graph_launch")

    def autotune(self, cache_path=None, stream=None):
        cp = None if cache_path is None else str(cache_path).encode()
        check(lib().sf_batch_autotune(self.h, cp, _stream(stream)), "sf_batch_autotune")

    def config(self):
        lpt, tile, nt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        check(lib().sf_batch_get_config(self.h, ctypes.byref(lpt), ctypes.byref(tile), ctypes.byref(nt)),
              "sf_batch_get_config")
        return lpt.value, tile.value, nt.value

    def set_config(self, lpt, tile):
        check(lib().sf_batch_set_config(self.h, int(lpt), int(tile)), "sf_batch_set_config")

    def destroy(self):
        if getattr(self, "h", None) and self.h.value:
            lib().sf_batch_destroy(ctypes.byref(self.h))

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
