"""CPU oracle for the star-forest (SF) operations -- TEST INFRASTRUCTURE ONLY.

Plain definitions of SFBcast, SFReduce and SFFetchAndOp (paper Section 3.2),
written in C (``sf_oracle.c``) and called here through ctypes on NumPy
arrays.  Only the tests, the package smoke check and the benchmark's CPU
baseline use this package; the product path never imports it, and it shares
no code with the GPU library.

Data are NumPy arrays of units: shape ``[n]`` (bs = 1) or ``[n, bs]``, with
dtype float64 / float32 / int32 / int64 / float16, :data:`BF16` (bfloat16
bit patterns), or :data:`PAIR` (the MAXLOC / MINLOC unit
``{double v; int32 i; int32 pad}``, 16-byte extent).

Every wrapper is functional: it copies its data arguments and returns new
arrays, so a test can keep the inputs.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

PAIR = np.dtype([("v", "<f8"), ("i", "<i4"), ("pad", "<i4")])
# bfloat16 units: NumPy has no such type, so their 16-bit patterns travel in
# a one-field structured dtype (binary16 units are plain np.float16)
BF16 = np.dtype([("bf16", "<u2")])

# enum values of sf_oracle.h
_DT = {np.dtype(np.float64): 0, np.dtype(np.float32): 1, np.dtype(np.int32): 2,
       np.dtype(np.int64): 3, PAIR: 4, np.dtype(np.float16): 5, BF16: 6}
REPLACE, SUM, MAX, MIN, MAXLOC, MINLOC, PROD = 0, 1, 2, 3, 4, 5, 6
OPS = {"replace": REPLACE, "sum": SUM, "max": MAX, "min": MIN, "maxloc": MAXLOC, "minloc": MINLOC, "prod": PROD}
PW_TOPDOWN, PW_BOTTOMUP = 0, 1

_lib = None


_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force=True):
    """Compile liboracle.so (sequential) and liboracle_omp.so (the same
    definitions plus their OpenMP variants, for the CPU baseline) with gcc:
    no fast-math, no FP contraction."""
    flags = ["-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared"]
    for so, src, extra in ((_SO, "sf_oracle.c", []), (_SO_OMP, "sf_oracle_omp.c", ["-fopenmp"])):
        if force or not os.path.exists(so):
            subprocess.check_call(["gcc", *flags, *extra, "-o", so + ".tmp", os.path.join(_HERE, src), "-lm"])
            os.replace(so + ".tmp", so)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, p, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        L.orc_bcast.argtypes = [i64, i64, p, p, ci, ci, ci, p, p]
        L.orc_reduce.argtypes = [i64, i64, p, p, ci, ci, ci, p, p, ci]
        L.orc_fetch_and_op.argtypes = [i64, i64, p, p, ci, ci, ci, p, p, p]
        for f in (L.orc_bcast, L.orc_reduce, L.orc_fetch_and_op):
            f.restype = ci
        L.orc_csr_spmv.argtypes = [i64, p, p, p, p, p, ci]
        L.orc_csr_spmv_t.argtypes = [i64, i64, p, p, p, p, p, ci]
        L.orc_csr_spmv.restype = L.orc_csr_spmv_t.restype = ci
        L.orc_multi_sf.argtypes = [i64, i64, p, p, p]
        L.orc_gather.argtypes = [i64, p, p, ci, ci, p, p]
        L.orc_scatter.argtypes = [i64, p, p, ci, ci, p, p]
        for f in (L.orc_multi_sf, L.orc_gather, L.orc_scatter):
            f.restype = ci
        L.orc_pairwise_f64.argtypes = [p, i64, ci]
        L.orc_pairwise_f64.restype = ctypes.c_double
        L.orc_pairwise_f32.argtypes = [p, i64, ci]
        L.orc_pairwise_f32.restype = ctypes.c_float
        for f in (L.orc_to_f16, L.orc_to_bf16):
            f.argtypes, f.restype = [ctypes.c_double], ctypes.c_uint16
        for f in (L.orc_from_f16, L.orc_from_bf16):
            f.argtypes, f.restype = [ctypes.c_uint16], ctypes.c_double
        _lib = L
    return _lib


_lib_omp = None


def lib_omp():
    """The OpenMP build (CPU baseline only)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_SO_OMP):
            build()
        L = ctypes.CDLL(_SO_OMP)
        i64, p, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        L.orc_bcast_omp.argtypes = [i64, i64, p, p, ci, ci, ci, p, p]
        L.orc_reduce_omp.argtypes = [i64, i64, p, p, ci, ci, ci, p, p]
        L.orc_fetch_and_op_omp.argtypes = [i64, i64, p, p, ci, ci, ci, p, p, p]
        for f in (L.orc_bcast_omp, L.orc_reduce_omp, L.orc_fetch_and_op_omp, L.orc_omp_threads):
            f.restype = ci
        L.orc_omp_threads.argtypes = []
        _lib_omp = L
    return _lib_omp


def omp_threads():
    """Threads the OpenMP variants run on (OMP_NUM_THREADS, else the host's)."""
    return int(lib_omp().orc_omp_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph(nroots, iroot, ilocal):
    iroot = np.ascontiguousarray(iroot, dtype=np.int64)
    ilocal = None if ilocal is None else np.ascontiguousarray(ilocal, dtype=np.int64)
    if ilocal is not None and ilocal.shape != iroot.shape:
        raise ValueError("ilocal and iroot differ in length")
    return int(nroots), iroot, ilocal


def _unit(a):
    a = np.asarray(a)
    if a.dtype not in _DT:
        raise TypeError(f"unsupported unit dtype {a.dtype}")
    bs = 1 if a.ndim == 1 else int(np.prod(a.shape[1:]))
    return _DT[a.dtype], bs


def _op(op):
    return OPS[op] if isinstance(op, str) else int(op)


def bcast(nroots, iroot, ilocal, rootdata, leafdata, op="replace"):
    """Return a copy of ``leafdata`` after SFBcast(rootdata -> leafdata, op)."""
    nroots, iroot, ilocal = _graph(nroots, iroot, ilocal)
    root = np.ascontiguousarray(rootdata)
    leaf = np.array(leafdata, copy=True, order="C")
    dt, bs = _unit(root)
    assert _unit(leaf) == (dt, bs) and root.shape[0] == nroots
    if iroot.size and (ilocal.max() if ilocal is not None else iroot.size - 1) >= leaf.shape[0]:
        raise ValueError("leaf buffer smaller than the leaf space")
    rc = lib().orc_bcast(nroots, iroot.size, _ptr(ilocal), _ptr(iroot), dt, bs, _op(op),
                         _ptr(root), _ptr(leaf))
    if rc:
        raise ValueError("oracle rejected the arguments")
    return leaf


def reduce(nroots, iroot, ilocal, leafdata, rootdata, op="sum", pw_form=PW_TOPDOWN):
    """Return a copy of ``rootdata`` after SFReduce(leafdata -> rootdata, op)."""
    nroots, iroot, ilocal = _graph(nroots, iroot, ilocal)
    leaf = np.ascontiguousarray(leafdata)
    root = np.array(rootdata, copy=True, order="C")
    dt, bs = _unit(root)
    assert _unit(leaf) == (dt, bs) and root.shape[0] == nroots
    if iroot.size and (ilocal.max() if ilocal is not None else iroot.size - 1) >= leaf.shape[0]:
        raise ValueError("leaf buffer smaller than the leaf space")
    rc = lib().orc_reduce(nroots, iroot.size, _ptr(ilocal), _ptr(iroot), dt, bs, _op(op),
                          _ptr(leaf), _ptr(root), pw_form)
    if rc:
        raise ValueError("oracle rejected the arguments")
    return root


def fetch_and_op(nroots, iroot, ilocal, rootdata, leafdata, leafupdate, op="sum"):
    """Return (root, leafupdate) after SFFetchAndOp in leaf order."""
    nroots, iroot, ilocal = _graph(nroots, iroot, ilocal)
    leaf = np.ascontiguousarray(leafdata)
    root = np.array(rootdata, copy=True, order="C")
    upd = np.array(leafupdate, copy=True, order="C")
    dt, bs = _unit(root)
    assert _unit(leaf) == (dt, bs) == _unit(upd) and root.shape[0] == nroots
    rc = lib().orc_fetch_and_op(nroots, iroot.size, _ptr(ilocal), _ptr(iroot), dt, bs, _op(op),
                                _ptr(root), _ptr(leaf), _ptr(upd))
    if rc:
        raise ValueError("oracle rejected the arguments")
    return root, upd


def multi_sf(nroots, iroot, ilocal):
    """The multi-SF (Section 3.2, item 2): the new root of every leaf, as an
    int64 array over leaf indices; there are nleaves new roots."""
    nroots, iroot, ilocal = _graph(nroots, iroot, ilocal)
    m = np.zeros(iroot.size, np.int64)
    if lib().orc_multi_sf(nroots, iroot.size, _ptr(ilocal), _ptr(iroot), _ptr(m)):
        raise ValueError("oracle rejected the arguments")
    return m


def gather(nroots, iroot, ilocal, leafdata, multirootdata):
    """Return a copy of ``multirootdata`` after SFGather(leafdata)."""
    m = multi_sf(nroots, iroot, ilocal)
    _, iroot, ilocal = _graph(nroots, iroot, ilocal)
    leaf = np.ascontiguousarray(leafdata)
    mr = np.array(multirootdata, copy=True, order="C")
    dt, bs = _unit(leaf)
    assert _unit(mr) == (dt, bs) and mr.shape[0] >= iroot.size
    if lib().orc_gather(iroot.size, _ptr(ilocal), _ptr(m), dt, bs, _ptr(leaf), _ptr(mr)):
        raise ValueError("oracle rejected the arguments")
    return mr


def scatter(nroots, iroot, ilocal, multirootdata, leafdata):
    """Return a copy of ``leafdata`` after SFScatter(multirootdata)."""
    m = multi_sf(nroots, iroot, ilocal)
    _, iroot, ilocal = _graph(nroots, iroot, ilocal)
    mr = np.ascontiguousarray(multirootdata)
    leaf = np.array(leafdata, copy=True, order="C")
    dt, bs = _unit(leaf)
    assert _unit(mr) == (dt, bs) and mr.shape[0] >= iroot.size
    if lib().orc_scatter(iroot.size, _ptr(ilocal), _ptr(m), dt, bs, _ptr(mr), _ptr(leaf)):
        raise ValueError("oracle rejected the arguments")
    return leaf


def csr_spmv(rowptr, colidx, values, x, y=None, transpose=False, ncols=None):
    """y = A x (or A^T x) for A in CSR (f64), plus y when given; returns a
    new array."""
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    colidx = np.ascontiguousarray(colidx, np.int32)
    values = np.ascontiguousarray(values, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    nrows = rowptr.size - 1
    acc = y is not None
    if transpose:
        ncols = int(ncols if ncols is not None else (colidx.max() + 1 if colidx.size else 0))
        out = np.array(y, np.float64, copy=True) if acc else np.zeros(ncols)
        rc = lib().orc_csr_spmv_t(nrows, ncols, _ptr(rowptr), _ptr(colidx), _ptr(values), _ptr(x), _ptr(out),
                                  int(acc))
    else:
        out = np.array(y, np.float64, copy=True) if acc else np.zeros(nrows)
        rc = lib().orc_csr_spmv(nrows, _ptr(rowptr), _ptr(colidx), _ptr(values), _ptr(x), _ptr(out), int(acc))
    if rc:
        raise ValueError("oracle rejected the arguments")
    return out


def spmv_split(nroots, iroot, A, B, x):
    """Section 4.1: y = M x with M = [A B] split by columns: lvec =
    Bcast(x) over the ghost SF (leaf j <- root iroot[j]), y = A x + B lvec.
    A, B are (rowptr, colidx, values); returns (y, lvec)."""
    lvec = bcast(nroots, iroot, None, np.asarray(x, np.float64), np.zeros(len(iroot)))
    y = csr_spmv(*A, x)
    return csr_spmv(*B, lvec, y), lvec


def spmv_split_transpose(nroots, iroot, A, B, x):
    """y = M^T x: y = A^T x, lvec = B^T x, then Reduce SUM (lvec -> y)."""
    y = csr_spmv(*A, x, transpose=True, ncols=nroots)
    lvec = csr_spmv(*B, x, transpose=True, ncols=len(iroot))
    return reduce(nroots, iroot, None, lvec, y, "sum"), lvec


def pairwise(x, form=PW_TOPDOWN):
    """Canonical pairwise sum of a 1-D float64/float32 array."""
    x = np.ascontiguousarray(x)
    if x.dtype == np.float64:
        return np.float64(lib().orc_pairwise_f64(_ptr(x), x.size, form))
    if x.dtype == np.float32:
        return np.float32(lib().orc_pairwise_f32(_ptr(x), x.size, form))
    raise TypeError(x.dtype)


# ------------------------------------------------ OpenMP variants (baseline)
def bcast_omp(nroots, iroot, ilocal, rootdata, leafdata, op="replace"):
    """bcast() on several host threads; identical results."""
    nroots, iroot, ilocal = _graph(nroots, iroot, ilocal)
    root = np.ascontiguousarray(rootdata)
    leaf = np.array(leafdata, copy=True, order="C")
    dt, bs = _unit(root)
    assert _unit(leaf) == (dt, bs) and root.shape[0] == nroots
    rc = lib_omp().orc_bcast_omp(nroots, iroot.size, _ptr(ilocal), _ptr(iroot), dt, bs, _op(op),
                                 _ptr(root), _ptr(leaf))
    if rc:
        raise ValueError("oracle rejected the arguments")
    return leaf


def reduce_omp(nroots, iroot, ilocal, leafdata, rootdata, op="sum"):
    """reduce() on several host threads (roots split among them); identical results."""
    nroots, iroot, ilocal = _graph(nroots, iroot, ilocal)
    leaf = np.ascontiguousarray(leafdata)
    root = np.array(rootdata, copy=True, order="C")
    dt, bs = _unit(root)
    assert _unit(leaf) == (dt, bs) and root.shape[0] == nroots
    rc = lib_omp().orc_reduce_omp(nroots, iroot.size, _ptr(ilocal), _ptr(iroot), dt, bs, _op(op),
                                  _ptr(leaf), _ptr(root))
    if rc:
        raise ValueError("oracle rejected the arguments")
    return root


def fetch_and_op_omp(nroots, iroot, ilocal, rootdata, leafdata, leafupdate, op="sum"):
    """fetch_and_op() on several host threads (roots split among them, each
    root's leaves in leaf order); identical results."""
    nroots, iroot, ilocal = _graph(nroots, iroot, ilocal)
    leaf = np.ascontiguousarray(leafdata)
    root = np.array(rootdata, copy=True, order="C")
    upd = np.array(leafupdate, copy=True, order="C")
    dt, bs = _unit(root)
    assert _unit(leaf) == (dt, bs) == _unit(upd) and root.shape[0] == nroots
    rc = lib_omp().orc_fetch_and_op_omp(nroots, iroot.size, _ptr(ilocal), _ptr(iroot), dt, bs, _op(op),
                                        _ptr(root), _ptr(leaf), _ptr(upd))
    if rc:
        raise ValueError("oracle rejected the arguments")
    return root, upd


# ------------------------------------------------ composition (Section 3.3)
# Graphs as (nroots, iroot, ilocal, ranks) with ilocal an int64 array of
# slots; pure Python over the edges (small cases).
def compose(a, b):
    """AB = a then b: a's leaf slots are b's roots; a leaf of b on root m
    joins a's root r when a has a leaf at slot m on root r."""
    na, ira, ila, _ = a
    _, irb, ilb, rkb = b
    root_at = {int(s): int(r) for s, r in zip(ila, ira)}
    keep = [k for k in range(len(irb)) if int(irb[k]) in root_at]
    return (na, np.array([root_at[int(irb[k])] for k in keep], np.int64), np.array([ilb[k] for k in keep], np.int64),
            np.array([rkb[k] for k in keep], np.int64))


def compose_inverse(a, b):
    """a and b share a leaf space, b's roots have at most one leaf: b's root
    m, whose leaf sits at slot l, joins a's root r when a has a leaf at l."""
    na, ira, ila, rka = a
    nb, irb, ilb, _ = b
    at = {int(s): (int(r), int(q)) for s, r, q in zip(ila, ira, rka)}
    slot_of_root = {}
    for s, r in zip(ilb, irb):
        assert int(r) not in slot_of_root, "b's roots must have degree <= 1"
        slot_of_root[int(r)] = int(s)
    keep = [m for m in range(nb) if m in slot_of_root and slot_of_root[m] in at]
    return (na, np.array([at[slot_of_root[m]][0] for m in keep], np.int64), np.array(keep, np.int64),
            np.array([at[slot_of_root[m]][1] for m in keep], np.int64))


def embedded_root(sf, roots):
    """Only the edges whose root is selected (no renumbering)."""
    n, ir, il, rk = sf
    sel = set(int(r) for r in roots)
    keep = [k for k in range(len(ir)) if int(ir[k]) in sel]
    return n, ir[keep], il[keep], rk[keep]


def embedded_leaf(sf, slots):
    """Only the edges whose leaf slot is selected (no renumbering)."""
    n, ir, il, rk = sf
    sel = set(int(s) for s in slots)
    keep = [k for k in range(len(ir)) if int(il[k]) in sel]
    return n, ir[keep], il[keep], rk[keep]


def to_f16(x):
    """Bit pattern of x rounded to binary16 (nearest, ties to even)."""
    return int(lib().orc_to_f16(float(x)))


def to_bf16(x):
    """Bit pattern of x rounded to bfloat16 (nearest, ties to even)."""
    return int(lib().orc_to_bf16(float(x)))


def from_f16(h):
    return float(lib().orc_from_f16(int(h)))


def from_bf16(h):
    return float(lib().orc_from_bf16(int(h)))
