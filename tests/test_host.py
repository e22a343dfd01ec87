"""CPU tests of the library's host side: the C ABI loads and exports every
call that include/sf.h declares; graph validation and error codes; setup
analysis (segments, pattern detection of Section 5.2, duplicate roots,
degree classes) through ``analyze_only`` -- no device is touched."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "sf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(sf_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_exports():
    assert sorted(S.EXPORTS) == header_functions()


def test_library_exports_every_declared_symbol():
    L = S.lib()
    for name in header_functions():
        assert hasattr(L, name), name


def test_error_strings():
    L = S.lib()
    for code in S.ERRORS:
        assert L.sf_error_string(code)
    assert L.sf_error_string(0) == b"success"


def create(nroots, iroot, ilocal=None, ranks=None):
    return S.StarForest(nroots, iroot, ilocal, ranks)


def test_validation_errors():
    with pytest.raises(S.SfError) as e:
        create(3, [0, 3])
    assert e.value.code == -1
    with pytest.raises(S.SfError) as e:
        create(3, [0, -1])
    assert e.value.code == -1
    with pytest.raises(S.SfError) as e:
        create(3, [0, 1], ilocal=[2, 2])
    assert e.value.code == -2          # SF_ERR_DUP_LEAF: stars are disjoint
    with pytest.raises(S.SfError) as e:
        create(3, [0, 1], ilocal=[0, -4])
    assert e.value.code == -1
    with pytest.raises(S.SfError) as e:
        create(-1, [])
    assert e.value.code == -1
    # OWN_POINTER is not supported
    h = ctypes.c_void_p()
    nodes = np.zeros((1, 2), np.int64)
    rc = S.lib().sf_create(1, 1, None, S.SF_OWN_POINTER, nodes.ctypes.data_as(ctypes.c_void_p),
                           S.SF_COPY_VALUES, ctypes.byref(h))
    assert rc == -4


def test_operations_before_setup_are_rejected():
    sf = create(3, [0, 1, 1])
    with pytest.raises(S.SfError) as e:
        sf.bcast_begin(S.SfUnit(S.SF_F64, 1), 0x1000, 0x2000, "replace", 0)
    assert e.value.code == -3
    sf.setup(analyze_only=True)    # analysis only: still no device plan
    with pytest.raises(S.SfError) as e:
        sf.reduce_begin(S.SfUnit(S.SF_F64, 1), 0x1000, 0x2000, "sum", 0)
    assert e.value.code == -3
    with pytest.raises(S.SfError) as e:
        sf.bcast_end(S.SfUnit(S.SF_F64, 1), 0x1000, 0x2000, "replace", 0)
    assert e.value.code == -7      # end without begin


def test_fig2_analysis():
    g = inputs.fig2()
    sf = create(g.nroots, g.iroot, g.ilocal, g.ranks).setup(analyze_only=True)
    info = sf.info()
    assert info["leafspace"] == 11 and info["nsegments"] == 3
    assert info["has_dup_roots"] == 1 and info["max_degree"] == 3
    assert info["nroots_touched"] == 7
    seg = [sf.segment(s) for s in range(3)]
    assert [s["nleaves"] for s in seg] == [4, 3, 3]
    assert seg[0]["leaf"]["kind"] == S.SF_PATTERN_CONTIGUOUS          # slots 0..3
    assert seg[1]["leaf"]["kind"] == S.SF_PATTERN_GENERIC             # slots 4, 5, 7


def brute_indices(p, n):
    """Enumerate start + i + sy*j + sz*k of a pattern in t order (Section 5.2)."""
    if p["kind"] == S.SF_PATTERN_CONTIGUOUS:
        return [p["start"] + t for t in range(n)]
    out = []
    for k in range(p["dz"]):
        for j in range(p["dy"]):
            for i in range(p["dx"]):
                out.append(p["start"] + i + p["sy"] * j + p["sz"] * k)
    return out


@pytest.mark.parametrize("n", [4, 7, 16])
def test_halo_patterns_detected(n):
    g = inputs.halo3d(n)
    sf = create(g.nroots, g.iroot, None, g.ranks).setup(analyze_only=True)
    info = sf.info()
    assert info["nsegments"] == 26
    start = 0
    for s in range(26):
        seg = sf.segment(s)
        m = seg["nleaves"]
        assert seg["leaf"]["kind"] == S.SF_PATTERN_CONTIGUOUS and seg["leaf"]["start"] == start
        assert seg["root"]["kind"] != S.SF_PATTERN_GENERIC, (s, seg)
        assert brute_indices(seg["root"], m) == g.iroot[start:start + m].tolist()
        start += m
    # degrees: faces 1, edges 3, corners 7
    deg = np.bincount(g.iroot, minlength=g.nroots)
    assert info["max_degree"] == 7 and deg.max() == 7


def test_pattern_detection_cases():
    def one_segment(idx, nroots=None):
        idx = np.asarray(idx, dtype=np.int64)
        nroots = nroots or int(idx.max()) + 1
        sf = create(nroots, idx).setup(analyze_only=True)
        return sf.segment(0)["root"]
    # contiguous
    p = one_segment(np.arange(10, 50), 60)
    assert p["kind"] == S.SF_PATTERN_CONTIGUOUS and p["start"] == 10
    # strided: dx = 1
    p = one_segment(np.arange(0, 300, 3))
    assert p["kind"] == S.SF_PATTERN_3D and p["dx"] == 1 and p["sy"] == 3
    # 3-D sub-block of a 10 x 8 x 6 box: start (2,1,1), size (4,3,2)
    X, Y = 10, 8
    blk = [2 + X * 1 + X * Y * 1 + i + X * j + X * Y * k for k in range(2) for j in range(3) for i in range(4)]
    p = one_segment(blk, X * Y * 6)
    assert (p["kind"], p["dx"], p["dy"], p["dz"], p["sy"], p["sz"]) == (S.SF_PATTERN_3D, 4, 3, 2, X, X * Y)
    assert brute_indices(p, len(blk)) == blk
    # near miss: one index perturbed -> generic
    bad = list(blk)
    bad[13] += 1
    assert one_segment(bad, X * Y * 6)["kind"] == S.SF_PATTERN_GENERIC
    # random -> generic
    rng = np.random.default_rng(0)
    assert one_segment(rng.integers(0, 1000, 500), 1000)["kind"] == S.SF_PATTERN_GENERIC


def test_generic_path_when_patterns_off():
    g = inputs.halo3d(6)
    sf = create(g.nroots, g.iroot, None, g.ranks).setup(use_patterns=False, analyze_only=True)
    assert sf.info()["nsegments"] == 26     # segments are still reported


def test_hot_roots_of_zipf_graph():
    g = inputs.spmv_ghost(seed=3, nroots=20000, nleaves=400000)
    sf = create(g.nroots, g.iroot, None, g.ranks).setup(analyze_only=True)
    info = sf.info()
    deg = np.bincount(g.iroot, minlength=g.nroots)
    assert info["max_degree"] == deg.max()
    assert info["nroots_touched"] == int((deg > 0).sum())
    # LDS-aggregation candidates: roots of degree >= 64, at most 8192, by degree
    assert info["nhot"] == min(8192, int((deg >= 64).sum())) and info["nhot"] > 0
    assert info["nsegments"] == 64


def test_empty_graph_analysis():
    sf = create(0, []).setup(analyze_only=True)
    info = sf.info()
    assert info["nleaves"] == 0 and info["nroots_touched"] == 0 and info["has_dup_roots"] == 0


@pytest.mark.parametrize("case", ["zipf", "holes", "halo", "one_root"])
def test_partitioned_plan_self_checks(case):
    """Setup with the partitioned path forced on builds its windows, per-window
    root and chunk descriptors and pass-A tiles on the host, and checks them
    (offsets inside their window, the slot map a permutation); a failed check
    is SF_ERR_ARG."""
    if case == "zipf":
        g = inputs.spmv_ghost(seed=3, nroots=20000, nleaves=300001)
    elif case == "holes":
        g = inputs.single_sf(seed=11, nroots=5000, nleaves=70001, leafspace=90001)
    elif case == "halo":
        g = inputs.halo3d(13)
    else:
        n = 200003
        g = inputs.Graph(2, np.full(n, 1, np.int64), None, np.zeros(n, np.int64), n)
    sf = create(g.nroots, g.iroot, g.ilocal, g.ranks).setup(partition="on", analyze_only=True)
    assert sf.info()["nleaves"] == g.nleaves


def test_index_width_limits():
    """Device indices are int32 (nroots, leaf space < 2^31): larger SFs are
    rejected at create with SF_ERR_ARG before anything is allocated."""
    L = S.lib()
    h = ctypes.c_void_p()
    nodes = np.zeros((1, 2), np.int64)
    p = nodes.ctypes.data_as(ctypes.c_void_p)
    assert L.sf_create(2**31, 1, None, S.SF_COPY_VALUES, p, S.SF_COPY_VALUES, ctypes.byref(h)) == -1
    assert L.sf_create(1, 2**31, None, S.SF_COPY_VALUES, p, S.SF_COPY_VALUES, ctypes.byref(h)) == -1
    big = np.array([2**31 - 1], np.int64)
    assert L.sf_create(1, 1, big.ctypes.data_as(ctypes.c_void_p), S.SF_COPY_VALUES, p, S.SF_COPY_VALUES,
                       ctypes.byref(h)) == -1
    ok = np.array([2**20], np.int64)   # a large slot inside the limit is accepted
    assert L.sf_create(1, 1, ok.ctypes.data_as(ctypes.c_void_p), S.SF_COPY_VALUES, p, S.SF_COPY_VALUES,
                       ctypes.byref(h)) == 0
    assert L.sf_destroy(ctypes.byref(h)) == 0


def test_bench_traffic_bookkeeping():
    """The benchmark's HBM counters are keyed on the built library's device
    code: the hash is stable, read from the .hip_fatbin section, and the
    committed counters are either for this build or reported as absent."""
    import importlib.util
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    h = bench.device_code_hash()
    assert h is not None and re.fullmatch(r"[0-9a-f]{16}", h)
    assert bench.device_code_hash() == h
    assert bench.measured_traffic("no_such_op") is None
    with open(os.path.join(root, "profiles", "hbm_traffic.json")) as f:
        d = json.load(f)
    t = bench.measured_traffic("fetch_and_op_i64_det")
    if d.get("_device_code_hash") == h:
        ops = d["ops"]["fetch_and_op_i64_det"]
        assert t == int(ops["fetch_bytes"] + ops["write_bytes"]) and t > 0
    else:
        assert t is None


class _FakeTensor:
    """Stands in for a torch tensor in the binding's argument checks (no GPU)."""

    def __init__(self, numel, esize, dtype, cuda=True, contiguous=True):
        self._n, self._e, self.dtype, self.is_cuda, self._c = numel, esize, dtype, cuda, contiguous

    def numel(self):
        return self._n

    def element_size(self):
        return self._e

    def is_contiguous(self):
        return self._c


def test_binding_checks_tensor_arguments():
    """Tensor arguments are checked before any call into the library: device,
    contiguity, size in bytes against the units the SF needs, dtype against
    the unit (byte tensors carry raw units)."""
    u = S.SfUnit(S.SF_F64, 2)
    ok = _FakeTensor(100 * 2, 8, "torch.float64")
    S.check_buffer(ok, 100, u, "x")
    S.check_buffer(_FakeTensor(1600, 1, "torch.uint8"), 100, u, "x")     # raw bytes
    S.check_buffer(0x1000, 100, u, "x")                                   # an address: unchecked
    bad = [_FakeTensor(200, 8, "torch.float64", cuda=False),               # host memory
           _FakeTensor(200, 8, "torch.float64", contiguous=False),         # strided view
           _FakeTensor(199, 8, "torch.float64"),                           # one element short
           _FakeTensor(1599, 1, "torch.uint8"),                            # one byte short
           _FakeTensor(400, 4, "torch.float32")]                           # wrong dtype
    for t in bad:
        with pytest.raises(S.SfError) as e:
            S.check_buffer(t, 100, u, "x")
        assert e.value.code == -1
    # through the StarForest calls: rejected before the library sees them
    sf = create(3, [0, 1, 1])
    small = _FakeTensor(2, 8, "torch.float64")
    with pytest.raises(S.SfError) as e:
        sf.reduce_begin(S.SfUnit(S.SF_F64, 1), small, ok, "sum", 0)   # 3 leaf slots needed
    assert e.value.code == -1 and "leafdata" in str(e.value)
    with pytest.raises(S.SfError) as e:
        sf.fetch_and_op_begin(S.SfUnit(S.SF_F64, 1), ok, ok, small, "sum", 0)
    assert e.value.code == -1 and "leafupdate" in str(e.value)
