"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (default setup options: the partitioned path for the large
SFs), plus the direct atomic kernels with partitioning switched off.  The C oracle handles
these sizes in seconds, so outputs are compared element by element: bit-exact
for REPLACE / MAX / MAXLOC / integer work / the deterministic sum, within the
stated tolerance for the atomic FP sum."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S
from helpers import atomic_sum_tolerance, check_fetch_chain, dev, first_diff, host, same_bits, unit

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def same(got, want, what):
    if not same_bits(got, want):
        idx, a, b = first_diff(got, want)
        raise AssertionError(f"{what}: differs at {idx.tolist()}: got {a} want {b}")


def run(sf, kind, a, b, op):
    da, db = dev(a), dev(b)
    if kind == "bcast":
        sf.bcast(da, db, op, unit=unit(a))
    else:
        sf.reduce(da, db, op, unit=unit(b))
    torch.cuda.synchronize()
    return host(db, b)


@pytest.fixture(scope="module")
def spmv():
    return inputs.spmv_ghost(seed=3)


@pytest.mark.parametrize("part", ["auto", "off"])
def test_spmv_ghost_full_atomic(spmv, part):
    """Atomic mode at full size: partitioned (default) and the direct
    persistent atomic kernels (partitioning off)."""
    g = spmv
    rng = np.random.default_rng(1005)
    sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="atomic", partition=part)
    root = rng.standard_normal(g.nroots)
    leaf = rng.standard_normal(g.nleaves)
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, "sum")
    ok, worst = atomic_sum_tolerance(run(sf, "reduce", leaf, root, "sum"), want, root, leaf, g.iroot, 1e-12)
    assert ok, worst
    same(run(sf, "reduce", leaf, root, "min"), oracle.reduce(g.nroots, g.iroot, None, leaf, root, "min"),
         f"reduce min atomic ({part})")
    l32, r32 = leaf.astype(np.float32), root.astype(np.float32)
    w32 = oracle.reduce(g.nroots, g.iroot, None, l32, r32, "sum")
    ok, worst = atomic_sum_tolerance(run(sf, "reduce", l32, r32, "sum"), w32, r32, l32, g.iroot, 1e-5)
    assert ok, worst
    r0 = rng.integers(0, 100, g.nroots).astype(np.int64)
    lf = rng.integers(0, 100, g.nleaves).astype(np.int64)
    r, l, u = dev(r0), dev(lf), dev(np.zeros(g.nleaves, np.int64))
    sf.fetch_and_op(r, l, u, "sum", unit=S.SfUnit(S.SF_I64, 1))
    torch.cuda.synchronize()
    check_fetch_chain(g.iroot, np.arange(g.nleaves), r0, lf, host(u, lf), host(r, r0))


def test_spmv_ghost_full(spmv):
    g = spmv
    rng = np.random.default_rng(1000)
    sf_det = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="deterministic")
    sf_atom = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="atomic")
    root = rng.standard_normal(g.nroots)
    leaf = rng.standard_normal(g.nleaves)
    same(run(sf_det, "bcast", root, leaf, "replace"), oracle.bcast(g.nroots, g.iroot, None, root, leaf), "bcast")
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, "sum")
    same(run(sf_det, "reduce", leaf, root, "sum"), want, "reduce sum f64 deterministic (partitioned)")
    ok, worst = atomic_sum_tolerance(run(sf_atom, "reduce", leaf, root, "sum"), want, root, leaf, g.iroot, 1e-12)
    assert ok, worst
    same(run(sf_atom, "reduce", leaf, root, "max"), oracle.reduce(g.nroots, g.iroot, None, leaf, root, "max"),
         "reduce max atomic")
    l32, r32 = leaf.astype(np.float32), root.astype(np.float32)
    same(run(sf_det, "reduce", l32, r32, "sum"), oracle.reduce(g.nroots, g.iroot, None, l32, r32, "sum"),
         "reduce sum f32 deterministic")


@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_spmv_ghost_full_maxloc(spmv, mode):
    g = spmv
    rng = np.random.default_rng(1001)
    sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode=mode)
    leaf = inputs.maxloc_leaves(rng, g.nleaves, ties=True)
    root = inputs.maxloc_roots(rng, g.nroots, ties=True)
    same(run(sf, "reduce", leaf, root, "maxloc"), oracle.reduce(g.nroots, g.iroot, None, leaf, root, "maxloc"),
         f"maxloc {mode}")


@pytest.fixture(scope="module")
def deep_root():
    """One root of ~17.06M leaves among five: 66.6K level-0 chunk results, so
    three levels above level 0 (261, 2, 1 results); the other roots take
    about 3.4K leaves each (one level above level 0)."""
    n = (1 << 24) + 300000
    rng = np.random.default_rng(1010)
    iroot = np.where(rng.random(n) < 0.999, 2, rng.integers(0, 5, n)).astype(np.int64)
    return inputs.Graph(5, iroot, None, np.zeros(n, np.int64), n)


@pytest.mark.parametrize("part", ["on", "off"])
def test_deep_root_levels(deep_root, part):
    """Three chunk levels above level 0 give the oracle's bits, on the
    partitioned and the direct deterministic paths."""
    g = deep_root
    rng = np.random.default_rng(1011)
    sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="deterministic", partition=part)
    leaf = rng.standard_normal(g.nleaves)
    root = rng.standard_normal(g.nroots)
    same(run(sf, "reduce", leaf, root, "sum"), oracle.reduce(g.nroots, g.iroot, None, leaf, root, "sum"),
         f"deep root sum ({part})")
    lp = inputs.maxloc_leaves(rng, g.nleaves, ties=True)
    rp = inputs.maxloc_roots(rng, g.nroots, ties=True)
    same(run(sf, "reduce", lp, rp, "maxloc"), oracle.reduce(g.nroots, g.iroot, None, lp, rp, "maxloc"),
         f"deep root maxloc ({part})")


def test_spmv_ghost_full_fetch_and_op(spmv):
    g = spmv
    deg = np.bincount(g.iroot, minlength=g.nroots).astype(np.int64)
    root0 = np.concatenate([[0], np.cumsum(deg)[:-1]]).astype(np.int64)
    ones = np.ones(g.nleaves, np.int64)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, ones, np.zeros(g.nleaves, np.int64))
    for mode in ("deterministic", "atomic"):
        sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode=mode)
        r, l, u = dev(root0), dev(ones), dev(np.zeros(g.nleaves, np.int64))
        sf.fetch_and_op(r, l, u, "sum", unit=S.SfUnit(S.SF_I64, 1))
        torch.cuda.synchronize()
        r, u = host(r, root0), host(u, ones)
        same(r, wr, f"fetch roots {mode}")
        if mode == "deterministic":
            same(u, wu, "fetch leafupdate deterministic")
        else:
            assert np.array_equal(np.sort(u), np.arange(g.nleaves))
            check_fetch_chain(g.iroot, np.arange(g.nleaves), root0, ones, u, r)


@pytest.mark.parametrize("bs", [1, 3])
def test_halo_256_full(bs):
    g = inputs.halo3d(256)
    rng = np.random.default_rng(1002 + bs)
    root = rng.standard_normal((g.nroots, bs))
    leaf = rng.standard_normal((g.nleaves, bs))
    want_b = oracle.bcast(g.nroots, g.iroot, None, root, leaf)
    want_r = oracle.reduce(g.nroots, g.iroot, None, leaf, root)
    for pat in (True, False):
        sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="deterministic", use_patterns=pat)
        same(run(sf, "bcast", root, leaf, "replace"), want_b, f"halo bcast patterns={pat}")
        same(run(sf, "reduce", leaf, root, "sum"), want_r, f"halo reduce patterns={pat}")


def test_batch_mix_full():
    items = inputs.batch_mix(seed=4)
    keep, bitems, wants = [], [], []
    for it in items:
        g = it["graph"]
        rng = np.random.default_rng(it["seed"])
        sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="atomic")
        root = inputs.unit_data(rng, g.nroots, it["bs"], it["dtype"])
        leaf = inputs.unit_data(rng, g.nleaves, it["bs"], it["dtype"])
        troot, tleaf = torch.from_numpy(root).cuda(), torch.from_numpy(leaf).cuda()
        if it["kind"] == "bcast":
            wants.append(oracle.bcast(g.nroots, g.iroot, None, root, leaf))
        else:
            wants.append(oracle.reduce(g.nroots, g.iroot, None, leaf, root))
        keep.append((it, g, root, leaf, troot, tleaf))
        bitems.append((sf, S.unit_of(troot), it["kind"], it["op"], troot, tleaf))
    batch = S.Batch(bitems)
    batch.launch()
    torch.cuda.synchronize()
    for (it, g, root, leaf, troot, tleaf), want in zip(keep, wants):
        if it["kind"] == "bcast":
            same(tleaf.cpu().numpy(), want, "batch bcast")
        elif np.dtype(it["dtype"]).kind == "i":
            same(troot.cpu().numpy(), want, "batch reduce int")
        else:
            rtol = 1e-12 if np.dtype(it["dtype"]) == np.float64 else 1e-5
            ok, worst = atomic_sum_tolerance(troot.cpu().numpy(), want, root, leaf, g.iroot, rtol)
            assert ok, worst


def test_knn_full_fp32x16():
    g = inputs.knn_graph(seed=5)
    rng = np.random.default_rng(1004)
    sf = S.StarForest(g.nroots, g.iroot, None, None).setup(reduce_mode="deterministic")
    root = rng.standard_normal((g.nroots, 16)).astype(np.float32)
    leaf = rng.standard_normal((g.nleaves, 16)).astype(np.float32)
    same(run(sf, "bcast", root, leaf, "replace"), oracle.bcast(g.nroots, g.iroot, None, root, leaf), "knn bcast")
    same(run(sf, "reduce", leaf, np.zeros_like(root), "sum"),
         oracle.reduce(g.nroots, g.iroot, None, leaf, np.zeros_like(root), "sum"), "knn reduce (adjoint of bcast)")
