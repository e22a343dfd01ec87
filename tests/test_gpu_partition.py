"""GPU parity of the partitioned deterministic path (pass A into bucket-major
scratch, pass B per window on its XCD): forced on at test sizes, it must give
the oracle's bits exactly like the direct path."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S
from helpers import dev, host, same_bits, first_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_reduce(g, leaf, root, op, part, offset=0):
    sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode="deterministic", partition=part)
    l, r = dev(leaf, offset), dev(root)
    from helpers import unit
    sf.reduce(l, r, op, unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root)


def run_fetch(g, root, leaf, upd, part):
    sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode="deterministic", partition=part)
    from helpers import unit
    r, l, u = dev(root), dev(leaf), dev(upd)
    sf.fetch_and_op(r, l, u, "sum", unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root), host(u, upd)


def check(got, want, what):
    if not same_bits(got, want):
        idx, a, b = first_diff(got, want)
        raise AssertionError(f"{what}: differs at {idx.tolist()}: got {a} want {b}")


@pytest.fixture(scope="module")
def zipf():
    return inputs.spmv_ghost(seed=3, nroots=20000, nleaves=300001)


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int32, np.int64])
@pytest.mark.parametrize("op", ["sum", "max", "min"])
def test_partition_reduce(zipf, dtype, op):
    g = zipf
    rng = np.random.default_rng(800)
    kind = "full" if np.dtype(dtype).kind == "i" else "normal"
    leaf = inputs.unit_data(rng, g.leafspace, 1, dtype, kind)
    root = inputs.unit_data(rng, g.nroots, 1, dtype, kind)
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, op)
    check(run_reduce(g, leaf, root, op, "on"), want, f"partition {op} {np.dtype(dtype)}")


@pytest.mark.parametrize("ties", [False, True])
def test_partition_maxloc(zipf, ties):
    g = zipf
    rng = np.random.default_rng(801)
    leaf = inputs.maxloc_leaves(rng, g.leafspace, ties)
    root = inputs.maxloc_roots(rng, g.nroots, ties)
    root["pad"] = 9
    got = run_reduce(g, leaf, root, "maxloc", "on")
    check(got, oracle.reduce(g.nroots, g.iroot, None, leaf, root, "maxloc"), "partition maxloc")
    assert (got["pad"] == 9).all()


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_partition_fetch(zipf, dtype):
    g = zipf
    rng = np.random.default_rng(802)
    root0 = rng.integers(0, 100, g.nroots).astype(dtype)
    leaf = rng.integers(0, 100, g.nleaves).astype(dtype)
    upd0 = np.zeros(g.nleaves, dtype)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, leaf, upd0)
    r, u = run_fetch(g, root0, leaf, upd0, "on")
    check(r, wr, "partition fetch roots")
    check(u, wu, "partition fetch leafupdate")


def test_partition_multi_sf(zipf):
    g = zipf
    deg = np.bincount(g.iroot, minlength=g.nroots).astype(np.int64)
    root0 = np.concatenate([[0], np.cumsum(deg)[:-1]]).astype(np.int64)
    r, u = run_fetch(g, root0, np.ones(g.nleaves, np.int64), np.zeros(g.nleaves, np.int64), "on")
    assert np.array_equal(r, root0 + deg)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, np.ones(g.nleaves, np.int64),
                                 np.zeros(g.nleaves, np.int64))
    check(u, wu, "multi-sf")


def test_partition_holes_and_permuted_slots():
    """ilocal a random subset of a larger leaf space: pass A gathers through
    the slot list, pass C writes only connected slots."""
    g = inputs.single_sf(seed=11, nroots=5000, nleaves=70001, leafspace=90001)
    rng = np.random.default_rng(803)
    leaf = rng.standard_normal((g.leafspace, 3))
    root = rng.standard_normal((g.nroots, 3))
    check(run_reduce(g, leaf, root, "sum", "on"), oracle.reduce(g.nroots, g.iroot, g.ilocal, leaf, root), "holes")
    ri = rng.integers(0, 100, g.nroots).astype(np.int32)
    li = rng.integers(0, 100, g.leafspace).astype(np.int32)
    u0 = np.full(g.leafspace, -5, np.int32)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, g.ilocal, ri, li, u0)
    r, u = run_fetch(g, ri, li, u0, "on")
    check(r, wr, "holes fetch roots")
    check(u, wu, "holes fetch leafupdate (holes untouched)")


@pytest.mark.parametrize("dtype,bs", [(np.float32, 16), (np.int32, 5), (np.float64, 3)])
def test_partition_units(dtype, bs):
    g = inputs.spmv_ghost(seed=12, nroots=4001, nleaves=90007)
    rng = np.random.default_rng(804 + bs)
    leaf = inputs.unit_data(rng, g.leafspace, bs, dtype)
    root = inputs.unit_data(rng, g.nroots, bs, dtype)
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root)
    check(run_reduce(g, leaf, root, "sum", "on"), want, f"units {bs}")
    off = np.dtype(dtype).itemsize        # element-aligned, not unit-aligned
    check(run_reduce(g, leaf, root, "sum", "on", offset=off), want, f"units {bs} offset {off}")


def test_partition_halo_and_single_root():
    g = inputs.halo3d(13)
    rng = np.random.default_rng(805)
    leaf = rng.standard_normal((g.leafspace, 3))
    root = rng.standard_normal((g.nroots, 3))
    check(run_reduce(g, leaf, root, "sum", "on"), oracle.reduce(g.nroots, g.iroot, None, leaf, root), "halo")
    n = 200003
    g1 = inputs.Graph(2, np.full(n, 1, np.int64), None, np.zeros(n, np.int64), n)
    leaf = rng.standard_normal(n)
    root = rng.standard_normal(2)
    check(run_reduce(g1, leaf, root, "sum", "on"), oracle.reduce(2, g1.iroot, None, leaf, root), "one root")


def test_partition_matches_direct_bitwise(zipf):
    g = zipf
    rng = np.random.default_rng(806)
    leaf = rng.standard_normal(g.nleaves).astype(np.float32)
    root = rng.standard_normal(g.nroots).astype(np.float32)
    a = run_reduce(g, leaf, root, "sum", "on")
    b = run_reduce(g, leaf, root, "sum", "off")
    assert same_bits(a, b)
