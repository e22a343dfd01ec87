"""GPU parity of the partitioned path (pass A into window-major scratch,
pass B per window from LDS): forced on at test sizes, the deterministic mode
must give the oracle's bits exactly like the direct path, and the atomic
mode must meet the atomic bar (order-free results exact, FP sums within
tolerance, FetchAndOp a valid prefix chain)."""
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


@pytest.mark.parametrize("dtype,bs", [(np.float32, 2), (np.float32, 3), (np.int32, 4), (np.float64, 2),
                                      (np.int64, 2)])
@pytest.mark.parametrize("op", ["sum", "max", "min"])
@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_partition_units(dtype, bs, op, mode):
    """Units of several elements (8, 12 and 16 bytes: both unit-size classes
    of the partitioned path), element-aligned as well as unit-aligned."""
    from helpers import atomic_sum_tolerance
    g = inputs.spmv_ghost(seed=12, nroots=4001, nleaves=90007)
    rng = np.random.default_rng(804 + bs)
    integer = np.dtype(dtype).kind == "i"
    leaf = inputs.unit_data(rng, g.leafspace, bs, dtype, "full" if integer else "normal")
    root = inputs.unit_data(rng, g.nroots, bs, dtype, "full" if integer else "normal")
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, op)
    off = np.dtype(dtype).itemsize        # element-aligned, not unit-aligned
    for o in (0, off):
        sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode=mode, partition="on")
        from helpers import unit
        l, r = dev(leaf, o), dev(root)
        sf.reduce(l, r, op, unit=unit(root))
        torch.cuda.synchronize()
        got = host(r, root)
        what = f"units {np.dtype(dtype)} x {bs} {op} {mode} offset {o}"
        if mode == "atomic" and op == "sum" and not integer:
            ok, worst = atomic_sum_tolerance(got, want, root, leaf, g.iroot, 1e-12 if dtype == np.float64 else 1e-5)
            assert ok, (what, worst)
        else:
            check(got, want, what)


@pytest.mark.parametrize("dtype,bs", [(np.float32, 16), (np.int32, 5), (np.float64, 3)])
def test_partition_oversize_units_fall_back(dtype, bs):
    """Units above 16 bytes take the direct path even with partitioning on."""
    g = inputs.spmv_ghost(seed=12, nroots=4001, nleaves=90007)
    rng = np.random.default_rng(804 + bs)
    leaf = inputs.unit_data(rng, g.leafspace, bs, dtype)
    root = inputs.unit_data(rng, g.nroots, bs, dtype)
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root)
    check(run_reduce(g, leaf, root, "sum", "on"), want, f"units {bs}")


def test_partition_halo_and_single_root():
    g = inputs.halo3d(13)
    rng = np.random.default_rng(805)
    leaf = rng.standard_normal((g.leafspace, 2))
    root = rng.standard_normal((g.nroots, 2))
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


# ------------------------------------------------------------ atomic mode
# With reduce_mode="atomic" the partitioned path keeps the per-window work of
# the deterministic one, and the chunks of a large root meet at the root
# through native atomics (reduce) or returning atomic adds (FetchAndOp).

def run_reduce_mode(g, leaf, root, op, mode, part="on"):
    sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode=mode, partition=part)
    from helpers import unit
    l, r = dev(leaf), dev(root)
    sf.reduce(l, r, op, unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root)


def run_fetch_mode(g, root, leaf, upd, mode, part="on"):
    sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup(reduce_mode=mode, partition=part)
    from helpers import unit
    r, l, u = dev(root), dev(leaf), dev(upd)
    sf.fetch_and_op(r, l, u, "sum", unit=unit(root))
    torch.cuda.synchronize()
    return host(r, root), host(u, upd)


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.int32, np.int64])
@pytest.mark.parametrize("op", ["sum", "max", "min"])
def test_partition_atomic_reduce(zipf, dtype, op):
    from helpers import atomic_sum_tolerance
    g = zipf
    rng = np.random.default_rng(810)
    kind = "full" if np.dtype(dtype).kind == "i" else "normal"
    leaf = inputs.unit_data(rng, g.leafspace, 1, dtype, kind)
    root = inputs.unit_data(rng, g.nroots, 1, dtype, kind)
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root, op)
    got = run_reduce_mode(g, leaf, root, op, "atomic")
    if op == "sum" and np.dtype(dtype).kind == "f":
        rtol = 1e-12 if dtype == np.float64 else 1e-5
        ok, worst = atomic_sum_tolerance(got, want, root, leaf, g.iroot, rtol)
        assert ok, f"atomic partition sum {np.dtype(dtype)}: {worst:.3g}"
        untouched = np.bincount(g.iroot, minlength=g.nroots) == 0
        assert same_bits(got[untouched], root[untouched])
    else:   # integer sums wrap in any order; MAX/MIN are order-free
        check(got, want, f"atomic partition {op} {np.dtype(dtype)}")


@pytest.mark.parametrize("dtype", [np.int32, np.int64, np.float64])
def test_partition_atomic_fetch_chain(zipf, dtype):
    """Integer-valued data (also in float64, where every partial sum is
    exact): the fetched values of each root form a prefix chain and the
    final roots are exact."""
    from helpers import check_fetch_chain
    g = zipf
    rng = np.random.default_rng(811)
    root0 = rng.integers(0, 100, g.nroots).astype(dtype)
    leaf = rng.integers(0, 100, g.nleaves).astype(dtype)
    r, u = run_fetch_mode(g, root0, leaf, np.zeros(g.nleaves, dtype), "atomic")
    check_fetch_chain(g.iroot, np.arange(g.nleaves), root0, leaf, u, r)


def test_partition_atomic_fetch_float(zipf):
    from helpers import atomic_sum_tolerance
    g = zipf
    rng = np.random.default_rng(812)
    root0 = rng.standard_normal(g.nroots)
    leaf = np.abs(rng.standard_normal(g.nleaves))
    r, u = run_fetch_mode(g, root0, leaf, np.zeros(g.nleaves), "atomic")
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root0, "sum")
    ok, worst = atomic_sum_tolerance(r, want, root0, leaf, g.iroot, 1e-12)
    assert ok, worst
    lo, hi = root0[g.iroot], r[g.iroot]
    assert np.all(u >= lo - 1e-9 * np.abs(hi)) and np.all(u <= hi + 1e-9 * np.abs(hi))
    # float32: same checks at its own tolerance
    r32, u32 = run_fetch_mode(g, root0.astype(np.float32), leaf.astype(np.float32),
                              np.zeros(g.nleaves, np.float32), "atomic")
    want32 = oracle.reduce(g.nroots, g.iroot, None, leaf.astype(np.float32), root0.astype(np.float32), "sum")
    ok, worst = atomic_sum_tolerance(r32, want32, root0.astype(np.float32), leaf.astype(np.float32), g.iroot, 1e-5)
    assert ok, worst


def test_partition_atomic_holes_and_units():
    from helpers import atomic_sum_tolerance, check_fetch_chain
    g = inputs.single_sf(seed=14, nroots=5000, nleaves=70001, leafspace=90001)
    rng = np.random.default_rng(813)
    leaf = rng.standard_normal((g.leafspace, 2))
    root = rng.standard_normal((g.nroots, 2))
    want = oracle.reduce(g.nroots, g.iroot, g.ilocal, leaf, root)
    got = run_reduce_mode(g, leaf, root, "sum", "atomic")
    slots = g.ilocal
    ok, worst = atomic_sum_tolerance(got, want, root, leaf[slots], g.iroot, 1e-12)
    assert ok, worst
    li = inputs.unit_data(rng, g.leafspace, 3, np.int32, "full")
    ri = inputs.unit_data(rng, g.nroots, 3, np.int32, "full")
    check(run_reduce_mode(g, li, ri, "max", "atomic"), oracle.reduce(g.nroots, g.iroot, g.ilocal, li, ri, "max"),
          "atomic max bs 3 with holes")
    r0 = rng.integers(0, 100, g.nroots).astype(np.int64)
    lf = rng.integers(0, 100, g.leafspace).astype(np.int64)
    u0 = np.full(g.leafspace, -5, np.int64)
    r, u = run_fetch_mode(g, r0, lf, u0, "atomic")
    holes = np.ones(g.leafspace, bool)
    holes[slots] = False
    assert (u[holes] == -5).all(), "holes untouched"
    check_fetch_chain(g.iroot, slots, r0, lf, u, r)


def test_partition_atomic_single_root():
    """Every leaf on one root: all chunks meet at one address."""
    n = 200003
    g1 = inputs.Graph(2, np.full(n, 1, np.int64), None, np.zeros(n, np.int64), n)
    rng = np.random.default_rng(814)
    leaf = rng.integers(-1000, 1000, n).astype(np.int64)
    root = np.array([7, 11], np.int64)
    check(run_reduce_mode(g1, leaf, root, "sum", "atomic"), oracle.reduce(2, g1.iroot, None, leaf, root), "one root")
    from helpers import check_fetch_chain
    ones = np.ones(n, np.int64)
    r, u = run_fetch_mode(g1, root, ones, np.zeros(n, np.int64), "atomic")
    check_fetch_chain(g1.iroot, np.arange(n), root, ones, u, r)


@pytest.mark.parametrize("dtype,bs", [(np.int32, 2), (np.int32, 3), (np.int64, 2)])
def test_partition_fetch_units(zipf, dtype, bs):
    """FetchAndOp on multi-element units through both unit-size classes
    (8 and 12 / 16 bytes): deterministic bit-exact, atomic a valid chain
    per element."""
    from helpers import check_fetch_chain
    g = zipf
    rng = np.random.default_rng(815 + bs)
    root0 = rng.integers(0, 100, (g.nroots, bs)).astype(dtype)
    leaf = rng.integers(0, 100, (g.nleaves, bs)).astype(dtype)
    upd0 = np.zeros((g.nleaves, bs), dtype)
    wr, wu = oracle.fetch_and_op(g.nroots, g.iroot, None, root0, leaf, upd0)
    r, u = run_fetch_mode(g, root0, leaf, upd0, "deterministic")
    check(r, wr, f"fetch det roots bs {bs}")
    check(u, wu, f"fetch det leafupdate bs {bs}")
    r, u = run_fetch_mode(g, root0, leaf, upd0, "atomic")
    for c in range(bs):
        check_fetch_chain(g.iroot, np.arange(g.nleaves), root0[:, c], leaf[:, c], u[:, c], r[:, c])


@pytest.mark.parametrize("mode", ["deterministic", "atomic"])
def test_partition_graph_capture(zipf, mode):
    """Partitioned Reduce and FetchAndOp captured into a HIP graph after one
    eager call of each: three replays, each after eager work that resets the
    inputs and synchronises; before the second, an eager call with a wider
    unit grows the SF's scratch (the captured graph keeps its buffer).  Every
    replay must give the oracle's result (the atomic bar in atomic mode)."""
    from helpers import atomic_sum_tolerance, check_fetch_chain
    g = zipf
    rng = np.random.default_rng(816)
    sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode=mode, partition="on")
    leaf = rng.standard_normal(g.nleaves)
    root0 = rng.standard_normal(g.nroots)
    want = oracle.reduce(g.nroots, g.iroot, None, leaf, root0, "sum")
    froot0 = rng.integers(0, 100, g.nroots).astype(np.int64)
    fleaf = rng.integers(0, 100, g.nleaves).astype(np.int64)
    fwr, fwu = oracle.fetch_and_op(g.nroots, g.iroot, None, froot0, fleaf, np.zeros(g.nleaves, np.int64))
    dl, dr0, dr = dev(leaf), dev(root0), dev(root0)
    dfl, dfr0, dfr, dfu = dev(fleaf), dev(froot0), dev(froot0), dev(np.zeros(g.nleaves, np.int64))
    u64, ui64 = S.SfUnit(S.SF_F64, 1), S.SfUnit(S.SF_I64, 1)

    def run():
        sf.reduce(dl, dr, "sum", unit=u64)
        sf.fetch_and_op(dfr, dfl, dfu, "sum", unit=ui64)

    def check_all(what):
        r, fr, fu = host(dr, root0), host(dfr, froot0), host(dfu, fleaf)
        if mode == "deterministic":
            check(r, want, f"{what}: reduce")
            check(fr, fwr, f"{what}: fetch roots")
            check(fu, fwu, f"{what}: fetch leafupdate")
        else:
            ok, worst = atomic_sum_tolerance(r, want, root0, leaf, g.iroot, 1e-12)
            assert ok, f"{what}: reduce {worst:.3g}"
            check_fetch_chain(g.iroot, np.arange(g.nleaves), froot0, fleaf, fu, fr)

    run()  # eager: allocates scratch, sets kernel attributes
    torch.cuda.synchronize()
    check_all("eager")
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        run()
    wide = rng.standard_normal((g.nleaves, 2))
    wroot = rng.standard_normal((g.nroots, 2))
    for rep in range(3):
        dr.copy_(dr0)
        dfr.copy_(dfr0)
        dfu.zero_()
        if rep == 1:  # grows the scratch: 16-byte units
            dw, dwr = dev(wide), dev(wroot)
            sf.reduce(dw, dwr, "sum", unit=S.SfUnit(S.SF_F64, 2))
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        check_all(f"replay {rep}")


def test_graph_capture_pairs_and_bcast(zipf):
    """MAXLOC / MINLOC through the partitioned path (12-byte scratch units)
    and Bcast REPLACE (two blocks per tile) captured into a HIP graph after
    one eager call each; three replays, each after eager work that resets the
    outputs and synchronises, each checked against the oracle."""
    from helpers import PAIR
    g = zipf
    rng = np.random.default_rng(817)
    sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="deterministic", partition="on")
    lp = inputs.maxloc_leaves(rng, g.leafspace, ties=True)
    rp = inputs.maxloc_roots(rng, g.nroots, ties=True)
    want_max = oracle.reduce(g.nroots, g.iroot, None, lp, rp, "maxloc")
    want_min = oracle.reduce(g.nroots, g.iroot, None, lp, rp, "minloc")
    root = rng.standard_normal(g.nroots)
    want_b = oracle.bcast(g.nroots, g.iroot, None, root, np.zeros(g.leafspace), "replace")
    dl, dr0, dmax, dmin = dev(lp), dev(rp), dev(rp), dev(rp)
    db_root, db_leaf = dev(root), dev(np.zeros(g.leafspace))
    up, u64 = S.SfUnit(S.SF_F64_I32, 1), S.SfUnit(S.SF_F64, 1)

    def run():
        sf.reduce(dl, dmax, "maxloc", unit=up)
        sf.reduce(dl, dmin, "minloc", unit=up)
        sf.bcast(db_root, db_leaf, "replace", unit=u64)

    def check_all(what):
        check(host(dmax, rp), want_max, f"{what}: maxloc")
        check(host(dmin, rp), want_min, f"{what}: minloc")
        check(host(db_leaf, want_b), want_b, f"{what}: bcast")

    run()
    torch.cuda.synchronize()
    check_all("eager")
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        run()
    for rep in range(3):
        dmax.copy_(dr0)
        dmin.copy_(dr0)
        db_leaf.zero_()
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        check_all(f"replay {rep}")
