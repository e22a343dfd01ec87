"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the
same seeded inputs.  Bit-exact for REPLACE, MAX/MIN/MAXLOC, integer work and
the deterministic FP sum; the atomic FP sum within
|got - oracle| <= rtol * (|root0| + sum|x|), rtol 1e-12 (f64) / 1e-5 (f32)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S
from helpers import PAIR, atomic_sum_tolerance, check_fetch_chain, dev, first_diff, host, same_bits, unit

pytestmark = pytest.mark.gpu

RTOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


@pytest.fixture(autouse=True, scope="module")
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def make_sf(g, mode="auto", use_patterns=True):
    return S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode=mode, use_patterns=use_patterns)


def gpu_bcast(sf, root, leaf, op="replace", offset=0):
    r, l = dev(root), dev(leaf, offset)
    sf.bcast(r, l, op, unit=unit(root))
    torch.cuda.synchronize()
    return host(l, leaf)


def gpu_reduce(sf, leaf, root, op="sum", offset=0):
    l, r = dev(leaf, offset), dev(root)
    sf.reduce(l, r, op, unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root)


def gpu_fetch(sf, root, leaf, upd):
    r, l, u = dev(root), dev(leaf), dev(upd)
    sf.fetch_and_op(r, l, u, "sum", unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root), host(u, upd)


def assert_same(got, want, what):
    if not same_bits(got, want):
        idx, a, b = first_diff(got, want)
        raise AssertionError(f"{what}: differs at {idx.tolist()}: got {a} want {b}")


def reduce_checked(g, leaf, root, op, mode, what):
    """Run a Reduce on the GPU in ``mode`` and compare with the oracle."""
    sf = make_sf(g, mode)
    got = gpu_reduce(sf, leaf, root, op)
    want = oracle.reduce(g.nroots, g.iroot, g.ilocal, leaf, root, op)
    exact = not (op == "sum" and np.asarray(root).dtype.kind == "f" and mode != "deterministic"
                 and sf.info()["has_dup_roots"])
    if exact:
        assert_same(got, want, what)
    else:
        slots = g.ilocal if g.ilocal is not None else np.arange(g.nleaves)
        ok, worst = atomic_sum_tolerance(got, want, root, np.asarray(leaf)[slots], g.iroot,
                                         RTOL[np.asarray(root).dtype])
        assert ok, f"{what}: atomic sum off by {worst:.3g} relative"
    return got


# ----------------------------------------------------------------- Fig. 2
@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int32, np.int64])
def test_fig2(dtype):
    g = inputs.fig2()
    root = (10 * np.arange(9)).astype(dtype)
    out = gpu_bcast(make_sf(g), root, np.full(11, -1, dtype))
    assert out.tolist() == [50, 30, 30, 20, 70, 0, -1, 80, 0, 30, 60]
    leaf = (np.arange(11) + 1).astype(dtype)
    for mode in ("auto", "atomic", "deterministic"):
        out = gpu_reduce(make_sf(g, mode), leaf, np.zeros(9, dtype))
        assert out.tolist() == [15, 0, 4, 15, 0, 1, 11, 5, 8], mode


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_fig2_multi_sf(dtype):
    g = inputs.fig2()
    root0 = np.array([0, 2, 2, 3, 6, 6, 7, 8, 9], dtype)
    r, u = gpu_fetch(make_sf(g, "deterministic"), root0, np.ones(11, dtype), np.full(11, -1, dtype))
    assert r.tolist() == [2, 2, 3, 6, 6, 7, 8, 9, 10]
    assert u.tolist() == [6, 3, 4, 2, 8, 0, -1, 9, 1, 5, 7]
    r, u = gpu_fetch(make_sf(g, "atomic"), root0, np.ones(11, dtype), np.full(11, -1, dtype))
    assert r.tolist() == [2, 2, 3, 6, 6, 7, 8, 9, 10]
    assert sorted(u[g.ilocal].tolist()) == list(range(10)) and u[6] == -1


# ------------------------------------------------------ single uniform SF
def test_single_sf_full_size():
    g = inputs.single_sf(seed=1)
    rng = np.random.default_rng(101)
    root = rng.standard_normal(g.nroots)
    leaf = rng.standard_normal(g.leafspace)
    assert_same(gpu_bcast(make_sf(g), root, leaf), oracle.bcast(g.nroots, g.iroot, g.ilocal, root, leaf),
                "bcast replace")
    for mode in ("deterministic", "atomic"):
        reduce_checked(g, leaf, root, "sum", mode, f"reduce sum {mode}")
        reduce_checked(g, leaf, root, "max", mode, f"reduce max {mode}")
    ri = rng.integers(0, 100, g.nroots).astype(np.int32)
    li = rng.integers(0, 100, g.leafspace).astype(np.int32)
    upd0 = np.full(g.leafspace, -7, np.int32)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, g.ilocal, ri, li, upd0, "sum")
    r, u = gpu_fetch(make_sf(g, "deterministic"), ri, li, upd0)
    assert_same(r, wr, "fetch det roots")
    assert_same(u, wu, "fetch det leafupdate")
    r, u = gpu_fetch(make_sf(g, "atomic"), ri, li, upd0)
    check_fetch_chain(g.iroot, g.ilocal, ri, li, u, r)
    holes = np.setdiff1d(np.arange(g.leafspace), g.ilocal)
    assert (u[holes] == -7).all()


# --------------------------------------------------------------- 3-D halo
@pytest.mark.parametrize("n", [8, 17])
@pytest.mark.parametrize("bs", [1, 3])
@pytest.mark.parametrize("use_patterns", [True, False])
def test_halo(n, bs, use_patterns):
    g = inputs.halo3d(n)
    rng = np.random.default_rng(200 + n)
    root = rng.standard_normal((g.nroots, bs))
    leaf = rng.standard_normal((g.leafspace, bs))
    sf = make_sf(g, "auto", use_patterns)
    assert_same(gpu_bcast(sf, root, leaf), oracle.bcast(g.nroots, g.iroot, None, root, leaf), "halo bcast")
    for mode in ("deterministic", "atomic"):
        sfm = make_sf(g, mode, use_patterns)
        got = gpu_reduce(sfm, leaf, root, "sum")
        want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, "sum")
        if mode == "deterministic":
            assert_same(got, want, "halo reduce det")
        else:
            ok, worst = atomic_sum_tolerance(got, want, root, leaf, g.iroot, 1e-12)
            assert ok, worst


@pytest.mark.parametrize("use_patterns", [True, False])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_halo_reduce_split_every_op(use_patterns, mode):
    """The halo's roots are single-leaf except on the box's edges (3 or 7
    leaves): for units of more than 8 bytes the Reduce splits into a pattern
    (or index) stream for the single-leaf roots and register trees for the
    others, in both modes, for every op -- the oracle's bits exactly (the
    split has no atomics); 8-byte units keep the root-sorted trees."""
    g = inputs.halo3d(21)
    rng = np.random.default_rng(210)
    sf = make_sf(g, mode, use_patterns)
    for dtype, bs in ((np.float64, 1), (np.float32, 3), (np.int32, 2), (np.int64, 1)):
        kind = "full" if np.dtype(dtype).kind == "i" else "normal"
        root = inputs.unit_data(rng, g.nroots, bs, dtype, kind)
        leaf = inputs.unit_data(rng, g.leafspace, bs, dtype, kind)
        for op in ("sum", "max", "min"):
            got = gpu_reduce(sf, leaf, root, op)
            want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, op)
            if (mode == "atomic" and op == "sum" and np.dtype(dtype).kind == "f"
                    and np.dtype(dtype).itemsize * bs <= 8):  # no split: native atomics
                ok, worst = atomic_sum_tolerance(got, want, root, leaf, g.iroot, RTOL[np.dtype(dtype)])
                assert ok, worst
            else:
                assert_same(got, want, f"halo split {op} {np.dtype(dtype)} x {bs}")
    lp = inputs.maxloc_leaves(rng, g.leafspace, ties=True)
    rp = inputs.maxloc_roots(rng, g.nroots, ties=True)
    assert_same(gpu_reduce(sf, lp, rp, "maxloc"), oracle.reduce(g.nroots, g.iroot, None, lp, rp, "maxloc"),
                "halo split maxloc")


# ------------------------------------------------------------ Zipf graph
@pytest.fixture(scope="module")
def zipf():
    return inputs.spmv_ghost(seed=3, nroots=20000, nleaves=300001)


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int32, np.int64])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_zipf_reduce_sum(zipf, dtype, mode):
    g = zipf
    rng = np.random.default_rng(300)
    kind = "full" if np.dtype(dtype).kind == "i" else "normal"
    leaf = inputs.unit_data(rng, g.leafspace, 1, dtype, kind)
    root = inputs.unit_data(rng, g.nroots, 1, dtype, kind)
    reduce_checked(g, leaf, root, "sum", mode, f"zipf sum {np.dtype(dtype)} {mode}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int32])
@pytest.mark.parametrize("op", ["max", "min"])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_zipf_reduce_maxmin(zipf, dtype, op, mode):
    g = zipf
    rng = np.random.default_rng(301)
    leaf = inputs.unit_data(rng, g.leafspace, 1, dtype)
    root = inputs.unit_data(rng, g.nroots, 1, dtype)
    if np.dtype(dtype).kind == "f":   # signed zeros take part: -0 < +0
        leaf[::97] = 0.0
        leaf[::89] = -0.0
        root[::31] = -0.0
    reduce_checked(g, leaf, root, op, mode, f"zipf {op} {mode}")


@pytest.mark.parametrize("ties", [False, True])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_zipf_maxloc(zipf, ties, mode):
    g = zipf
    rng = np.random.default_rng(302)
    leaf = inputs.maxloc_leaves(rng, g.leafspace, ties)
    root = inputs.maxloc_roots(rng, g.nroots, ties)
    leaf["pad"] = 12345
    root["pad"] = -777
    got = reduce_checked(g, leaf, root, "maxloc", mode, f"maxloc ties={ties} {mode}")
    assert (got["pad"] == -777).all()


def test_zipf_bcast_and_replace(zipf):
    g = zipf
    rng = np.random.default_rng(303)
    root = rng.standard_normal((g.nroots, 2))
    leaf = rng.standard_normal((g.leafspace, 2))
    assert_same(gpu_bcast(make_sf(g), root, leaf), oracle.bcast(g.nroots, g.iroot, None, root, leaf), "bcast")
    for op in ("sum", "max", "min"):
        assert_same(gpu_bcast(make_sf(g), root, leaf, op), oracle.bcast(g.nroots, g.iroot, None, root, leaf, op),
                    f"bcast {op}")
    reduce_checked(g, leaf, root, "replace", "deterministic", "reduce replace")


@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_zipf_fetch_multi_sf(zipf, mode):
    g = zipf
    deg = np.bincount(g.iroot, minlength=g.nroots).astype(np.int64)
    root0 = np.concatenate([[0], np.cumsum(deg)[:-1]]).astype(np.int64)
    ones = np.ones(g.nleaves, np.int64)
    r, u = gpu_fetch(make_sf(g, mode), root0, ones, np.zeros(g.nleaves, np.int64))
    assert np.array_equal(r, root0 + deg)
    assert np.array_equal(np.sort(u), np.arange(g.nleaves))     # multi-SF: a permutation
    if mode == "deterministic":
        wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, ones, np.zeros(g.nleaves, np.int64))
        assert_same(u, wu, "multi-sf leafupdate")
    else:
        check_fetch_chain(g.iroot, np.arange(g.nleaves), root0, ones, u, r)


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_zipf_fetch_u100(zipf, dtype, mode):
    g = zipf
    rng = np.random.default_rng(304)
    root0 = rng.integers(0, 100, g.nroots).astype(dtype)
    leaf = rng.integers(0, 100, g.nleaves).astype(dtype)
    upd0 = np.zeros(g.nleaves, dtype)
    r, u = gpu_fetch(make_sf(g, mode), root0, leaf, upd0)
    if mode == "deterministic":
        wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, leaf, upd0)
        assert_same(r, wr, "fetch roots")
        assert_same(u, wu, "fetch leafupdate")
    else:
        check_fetch_chain(g.iroot, np.arange(g.nleaves), root0, leaf, u, r)


def test_fetch_float_atomic(zipf):
    g = zipf
    rng = np.random.default_rng(305)
    root0 = rng.standard_normal(g.nroots)
    leaf = np.abs(rng.standard_normal(g.nleaves))
    r, u = gpu_fetch(make_sf(g, "atomic"), root0, leaf, np.zeros(g.nleaves))
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root0, "sum")
    ok, worst = atomic_sum_tolerance(r, want, root0, leaf, g.iroot, 1e-12)
    assert ok, worst
    # every fetched value lies between the root's start and final value
    lo, hi = root0[g.iroot], r[g.iroot]
    assert np.all(u >= lo - 1e-9 * np.abs(hi)) and np.all(u <= hi + 1e-9 * np.abs(hi))


# ------------------------------------------------------------- edge cases
def test_empty_graph():
    g = inputs.Graph(5, np.zeros(0, np.int64), None, np.zeros(0, np.int64), 0)
    sf = make_sf(g)
    root = np.arange(5, dtype=np.float64)
    leaf = np.zeros(1)
    assert_same(gpu_bcast(sf, root, leaf), leaf, "empty bcast")
    assert_same(gpu_reduce(sf, leaf, root), root, "empty reduce")


def test_one_root_takes_every_leaf():
    n = 100003   # several chunk levels, ragged at every level
    g = inputs.Graph(3, np.full(n, 1, np.int64), None, np.zeros(n, np.int64), n)
    rng = np.random.default_rng(400)
    leaf = rng.standard_normal(n)
    root = rng.standard_normal(3)
    for mode in ("deterministic", "atomic"):
        reduce_checked(g, leaf, root, "sum", mode, f"one root {mode}")
    r, u = gpu_fetch(make_sf(g, "deterministic"), np.arange(3, dtype=np.int64), np.ones(n, np.int64),
                     np.zeros(n, np.int64))
    assert r.tolist() == [0, 1 + n, 2] and np.array_equal(u, 1 + np.arange(n))


@pytest.mark.parametrize("dtype,bs", [(np.float32, 16), (np.int32, 5), (np.float64, 3), (np.int64, 7)])
def test_unit_shapes(dtype, bs):
    g = inputs.spmv_ghost(seed=9, nroots=3001, nleaves=40007)
    rng = np.random.default_rng(500 + bs)
    root = inputs.unit_data(rng, g.nroots, bs, dtype)
    leaf = inputs.unit_data(rng, g.leafspace, bs, dtype)
    assert_same(gpu_bcast(make_sf(g), root, leaf), oracle.bcast(g.nroots, g.iroot, None, root, leaf), "bcast")
    reduce_checked(g, leaf, root, "sum", "deterministic", "reduce det")
    reduce_checked(g, leaf, root, "sum", "atomic", "reduce atomic")
    if np.dtype(dtype).kind == "i":
        # the direct deterministic FetchAndOp with units of several elements:
        # a 40K-leaf Zipf SF (below the partitioning threshold, and forced
        # off) has roots of degree above 32 (chunk sums and root scans)
        assert np.bincount(g.iroot).max() > 32
        ri = inputs.unit_data(rng, g.nroots, bs, dtype, "full")
        li = inputs.unit_data(rng, g.leafspace, bs, dtype, "full")
        u0 = np.zeros_like(li)
        wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, ri, li, u0)
        sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode="deterministic", partition="off")
        r, u = gpu_fetch(sf, ri, li, u0)
        assert_same(r, wr, "fetch det roots")
        assert_same(u, wu, "fetch det leafupdate")


def test_misaligned_buffers():
    """Units of 16 bytes whose buffer starts 4 bytes into an allocation:
    the move falls back to narrower words, results stay exact."""
    g = inputs.single_sf(seed=7, nroots=999, nleaves=5001, leafspace=6007)
    rng = np.random.default_rng(600)
    root = rng.standard_normal((g.nroots, 4)).astype(np.float32)
    leaf = rng.standard_normal((g.leafspace, 4)).astype(np.float32)
    assert_same(gpu_bcast(make_sf(g), root, leaf, offset=4), oracle.bcast(g.nroots, g.iroot, g.ilocal, root, leaf),
                "misaligned bcast")
    assert_same(gpu_reduce(make_sf(g, "deterministic"), leaf, root, offset=4),
                oracle.reduce(g.nroots, g.iroot, g.ilocal, leaf, root), "misaligned reduce")


def test_begin_end_protocol():
    g = inputs.single_sf(seed=8, nroots=100, nleaves=500, leafspace=600)
    sf = make_sf(g)
    root, leaf = dev(np.zeros(100)), dev(np.zeros(600))
    u = S.SfUnit(S.SF_F64, 1)
    sf.bcast_begin(u, root, leaf)
    with pytest.raises(S.SfError) as e:      # same op on the same buffers while pending
        sf.bcast_begin(u, root, leaf)
    assert e.value.code == -8
    with pytest.raises(S.SfError) as e:      # end with a different op
        sf.bcast_end(u, root, leaf, "sum")
    assert e.value.code == -7
    sf.bcast_end(u, root, leaf)
    with pytest.raises(S.SfError) as e:      # MAXLOC needs pair units
        sf.reduce(leaf, root, "maxloc", unit=u)
    assert e.value.code == -4
    torch.cuda.synchronize()


def test_determinism_across_runs(zipf):
    g = zipf
    rng = np.random.default_rng(700)
    leaf = rng.standard_normal(g.nleaves).astype(np.float32)
    root = rng.standard_normal(g.nroots).astype(np.float32)
    sf = make_sf(g, "deterministic")
    a = gpu_reduce(sf, leaf, root)
    b = gpu_reduce(sf, leaf, root)
    assert same_bits(a, b)


def test_contiguous_segments_copy_and_ping_pong():
    """Every segment contiguous on both sides (Section 5.2's no-pack case):
    Bcast REPLACE is a device copy per segment; the ping-pong of Table 1's
    test (Bcast then Reduce REPLACE on a one-to-one SF) restores the roots."""
    n = 1000
    # two segments: leaves 0..599 <- roots 400..999, leaves 600..999 <- roots 0..399
    iroot = np.concatenate([np.arange(400, 1000), np.arange(0, 400)])
    ranks = np.concatenate([np.zeros(600, np.int64), np.ones(400, np.int64)])
    g = inputs.Graph(n, iroot, None, ranks, n)
    rng = np.random.default_rng(900)
    for dtype, bs in [(np.float64, 1), (np.float32, 3), (np.int32, 1)]:
        root = inputs.unit_data(rng, n, bs, dtype)
        leaf = inputs.unit_data(rng, n, bs, dtype)
        sf = make_sf(g)
        assert sf.segment(0)["root"]["kind"] == S.SF_PATTERN_CONTIGUOUS
        got = gpu_bcast(sf, root, leaf)
        assert_same(got, oracle.bcast(n, iroot, None, root, leaf), "contiguous bcast")
        back = gpu_reduce(sf, got, np.zeros_like(root), "replace")
        assert_same(back, root, "ping-pong round trip")


@pytest.mark.parametrize("op", ["replace", "maxloc"])
def test_bcast_pair_units(op):
    """Bcast of MAXLOC pairs (16-byte units) on an SF with holes: value and
    index as the oracle's, the leaves' padding and the holes untouched."""
    g = inputs.single_sf(seed=47, nroots=3000, nleaves=20000, leafspace=24000)
    rng = np.random.default_rng(48)
    root = inputs.maxloc_roots(rng, g.nroots, ties=True)
    root["i"] = rng.integers(0, 50, g.nroots)
    leaf = inputs.maxloc_leaves(rng, g.leafspace, ties=True)
    leaf["i"] = rng.integers(0, 50, g.leafspace)
    leaf["pad"] = 77
    got = gpu_bcast(make_sf(g), root, leaf, op)
    assert_same(got, oracle.bcast(g.nroots, g.iroot, g.ilocal, root, leaf, op), f"pair bcast {op}")
    assert (got["pad"] == 77).all()
