"""GPU parity of the hot-root path of the partitioned Reduce / FetchAndOp:
the leaves of the roots of highest degree stay in leaf order (per-tile
group values combined per root) while the other roots take the windows.
Results must equal the oracle's exactly wherever they are deterministic --
and equal the same SF set up without the hot path -- and meet the atomic bar
otherwise."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S
from helpers import (atomic_sum_tolerance, check_fetch_chain, check_fetch_chain_fp, dev, first_diff, host,
                     same_bits, unit)

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check(got, want, what):
    if not same_bits(got, want):
        idx, a, b = first_diff(got, want)
        raise AssertionError(f"{what}: differs at {idx.tolist()}: got {a} want {b}")


def make(g, mode, hot="on", part="on"):
    return S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode=mode, partition=part, hot_path=hot)


def reduce_on(sf, leaf, root, op):
    l, r = dev(leaf), dev(root)
    sf.reduce(l, r, op, unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root)


def fetch_on(sf, root, leaf, upd):
    r, l, u = dev(root), dev(leaf), dev(upd)
    sf.fetch_and_op(r, l, u, "sum", unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root), host(u, upd)


@pytest.fixture(scope="module")
def zipf():
    # 37 pass-A tiles (a ragged last one); the top root has ~1200 leaves per
    # tile (groups across 64-entry blocks and thread strides)
    return inputs.spmv_ghost(seed=3, nroots=20000, nleaves=300001)


def test_hot_path_is_planned(zipf):
    info = make(zipf, "deterministic").info()
    assert info["hot_roots"] > 0
    assert make(zipf, "deterministic", hot="off").info()["hot_roots"] == 0
    assert make(zipf, "deterministic", hot="auto").info()["hot_roots"] == 0  # opt-in


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int32, np.int64])
@pytest.mark.parametrize("op", ["sum", "max", "min"])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_hot_reduce(zipf, dtype, op, mode):
    g = zipf
    rng = np.random.default_rng(1000)
    integer = np.dtype(dtype).kind == "i"
    leaf = inputs.unit_data(rng, g.leafspace, 1, dtype, "full" if integer else "normal")
    root = inputs.unit_data(rng, g.nroots, 1, dtype, "full" if integer else "normal")
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, op)
    got = reduce_on(make(g, mode), leaf, root, op)
    what = f"hot {mode} {op} {np.dtype(dtype)}"
    if mode == "atomic" and op == "sum" and not integer:
        ok, worst = atomic_sum_tolerance(got, want, root, leaf, g.iroot, 1e-12 if dtype == np.float64 else 1e-5)
        assert ok, (what, worst)
    else:
        check(got, want, what)
        check(got, reduce_on(make(g, mode, hot="off"), leaf, root, op), what + " vs hot off")


@pytest.mark.parametrize("dtype,bs", [(np.float64, 2), (np.int32, 3), (np.float32, 4), (np.int64, 2)])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_hot_reduce_units(dtype, bs, mode):
    g = inputs.spmv_ghost(seed=21, nroots=3001, nleaves=120011)
    rng = np.random.default_rng(1001 + bs)
    integer = np.dtype(dtype).kind == "i"
    leaf = inputs.unit_data(rng, g.leafspace, bs, dtype, "full" if integer else "normal")
    root = inputs.unit_data(rng, g.nroots, bs, dtype, "full" if integer else "normal")
    for op in ("max", "sum"):
        want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, op)
        got = reduce_on(make(g, mode), leaf, root, op)
        if op == "sum" and not integer:
            if mode == "atomic":
                ok, worst = atomic_sum_tolerance(got, want, root, leaf, g.iroot,
                                                 1e-12 if dtype == np.float64 else 1e-5)
                assert ok, worst
                continue
        check(got, want, f"units {np.dtype(dtype)} x {bs} {op} {mode}")


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_hot_fetch_det(zipf, dtype):
    g = zipf
    rng = np.random.default_rng(1002)
    root0 = inputs.unit_data(rng, g.nroots, 1, dtype, "full")
    leaf = inputs.unit_data(rng, g.leafspace, 1, dtype, "full")
    upd0 = np.zeros(g.leafspace, dtype)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, leaf, upd0)
    r, u = fetch_on(make(g, "deterministic"), root0, leaf, upd0)
    check(r, wr, "hot fetch roots")
    check(u, wu, "hot fetch leafupdate")


@pytest.mark.parametrize("dtype,bs", [(np.int32, 2), (np.int32, 3), (np.int64, 2)])
def test_hot_fetch_det_units(dtype, bs):
    g = inputs.spmv_ghost(seed=22, nroots=3001, nleaves=120011)
    rng = np.random.default_rng(1003 + bs)
    root0 = inputs.unit_data(rng, g.nroots, bs, dtype, "full")
    leaf = inputs.unit_data(rng, g.leafspace, bs, dtype, "full")
    upd0 = np.zeros((g.leafspace, bs), dtype)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, leaf, upd0)
    r, u = fetch_on(make(g, "deterministic"), root0, leaf, upd0)
    check(r, wr, f"hot fetch roots x {bs}")
    check(u, wu, f"hot fetch leafupdate x {bs}")


def test_hot_fetch_atomic_int(zipf):
    g = zipf
    rng = np.random.default_rng(1004)
    root0 = rng.integers(0, 100, g.nroots).astype(np.int64)
    leaf = rng.integers(0, 100, g.leafspace).astype(np.int64)
    r, u = fetch_on(make(g, "atomic"), root0, leaf, np.zeros(g.leafspace, np.int64))
    check_fetch_chain(g.iroot, np.arange(g.nleaves), root0, leaf, u, r)


@pytest.mark.parametrize("dtype,rtol", [(np.float64, 1e-12), (np.float32, 1e-5)])
@pytest.mark.parametrize("hot", ["on", "off"])
def test_fetch_float_atomic_chain(zipf, dtype, rtol, hot):
    """Atomic FP FetchAndOp: the fetched values of every root form a chain
    of partial sums, within the atomic-sum tolerance."""
    g = zipf
    rng = np.random.default_rng(1005)
    root0 = rng.standard_normal(g.nroots).astype(dtype)
    leaf = (1.0 + rng.random(g.leafspace)).astype(dtype)  # in [1, 2): no reordering by rounding
    r, u = fetch_on(make(g, "atomic", hot=hot), root0, leaf, np.zeros(g.leafspace, dtype))
    check_fetch_chain_fp(g.iroot, np.arange(g.nleaves), root0, leaf, u, r, rtol)


def test_hot_permuted_slots():
    """ilocal a subset of a larger leaf space (leaf order still the segment
    order): the hot phase gathers and scatters through the slot list."""
    g = inputs.single_sf(seed=23, nroots=300, nleaves=70001, leafspace=90001)
    g.ranks = np.zeros(g.nleaves, np.int64)
    rng = np.random.default_rng(1006)
    assert make(g, "deterministic").info()["hot_roots"] > 0
    leaf = rng.integers(-1000, 1000, (g.leafspace, 2)).astype(np.int32)
    root = rng.integers(-1000, 1000, (g.nroots, 2)).astype(np.int32)
    check(reduce_on(make(g, "deterministic"), leaf, root, "sum"),
          oracle.reduce(g.nroots, g.iroot, g.ilocal, leaf, root, "sum"), "holes reduce")
    ri = rng.integers(0, 100, g.nroots).astype(np.int64)
    li = rng.integers(0, 100, g.leafspace).astype(np.int64)
    u0 = np.full(g.leafspace, -5, np.int64)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, g.ilocal, ri, li, u0)
    r, u = fetch_on(make(g, "deterministic"), ri, li, u0)
    check(r, wr, "holes fetch roots")
    check(u, wu, "holes fetch leafupdate (holes untouched)")


def test_hot_every_leaf_hot():
    """Four roots take every leaf: every tile's 8192 entries are hot (the
    largest hot phase) and no window is cold."""
    n = 8192 * 5 + 77
    rng = np.random.default_rng(1007)
    iroot = rng.integers(0, 4, n).astype(np.int64)
    g = inputs.Graph(6, iroot, None, np.zeros(n, np.int64), n)
    sf = make(g, "deterministic")
    assert sf.info()["hot_roots"] == 4
    leaf = rng.integers(-2**62, 2**62, n).astype(np.int64)
    root = rng.integers(-2**62, 2**62, 6).astype(np.int64)
    check(reduce_on(sf, leaf, root, "sum"), oracle.reduce(6, iroot, None, leaf, root, "sum"), "all hot reduce")
    check(reduce_on(sf, leaf, root, "max"), oracle.reduce(6, iroot, None, leaf, root, "max"), "all hot max")
    wr, wu = oracle.fetch_and_op(6, iroot, None, root, leaf, np.zeros(n, np.int64))
    r, u = fetch_on(sf, root, leaf, np.zeros(n, np.int64))
    check(r, wr, "all hot fetch roots")
    check(u, wu, "all hot fetch leafupdate")


def test_hot_off_when_segments_interleave():
    """Segment labels that are not in leaf order make the processing order
    differ from leaf order: no hot path, same results."""
    g = inputs.spmv_ghost(seed=24, nroots=2000, nleaves=100003)
    rng = np.random.default_rng(1008)
    g.ranks = rng.integers(0, 5, g.nleaves).astype(np.int64)
    sf = make(g, "deterministic")
    assert sf.info()["hot_roots"] == 0
    leaf = rng.integers(0, 100, g.leafspace).astype(np.int32)
    root = rng.integers(0, 100, g.nroots).astype(np.int32)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root, leaf, np.zeros(g.leafspace, np.int32))
    r, u = fetch_on(sf, root, leaf, np.zeros(g.leafspace, np.int32))
    check(r, wr, "interleaved fetch roots")
    check(u, wu, "interleaved fetch leafupdate")


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_hot_random_graphs(seed):
    """Random Zipf exponents and sizes: every hot op against the oracle."""
    rng = np.random.default_rng(seed)
    s = float(rng.uniform(0.7, 1.6))
    L = int(rng.integers(70000, 400000))
    R = int(rng.integers(500, 40000))
    g = inputs.spmv_ghost(seed=seed, nroots=R, nleaves=L, zipf_s=s)
    leaf = inputs.unit_data(rng, g.leafspace, 1, np.int64, "full")
    root = inputs.unit_data(rng, g.nroots, 1, np.int64, "full")
    for mode in ("deterministic", "atomic"):
        sf = make(g, mode)
        for op in ("sum", "max", "min"):
            check(reduce_on(sf, leaf, root, op), oracle.reduce(g.nroots, g.iroot, None, leaf, root, op),
                  f"seed {seed} {mode} {op}")
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root, leaf, np.zeros(g.leafspace, np.int64))
    r, u = fetch_on(make(g, "deterministic"), root, leaf, np.zeros(g.leafspace, np.int64))
    check(r, wr, f"seed {seed} fetch roots")
    check(u, wu, f"seed {seed} fetch leafupdate")
