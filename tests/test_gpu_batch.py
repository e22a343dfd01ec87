"""GPU tests of the batched path: many uneven SF operations in one persistent
launch, the per-SF launches, HIP-graph replays of both, and the autotuner's
candidates -- all against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S
from helpers import atomic_sum_tolerance, check_fetch_chain, check_fetch_chain_fp, same_bits

pytestmark = pytest.mark.gpu

TDT = {np.dtype(np.float64): (torch.float64, S.SF_F64), np.dtype(np.float32): (torch.float32, S.SF_F32),
       np.dtype(np.int32): (torch.int32, S.SF_I32)}


@pytest.fixture(scope="module")
def batch_case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    items = inputs.batch_mix(seed=4, count=24, lmin=10, lmax=3e4)
    case = []
    for k, it in enumerate(items):
        g = it["graph"]
        rng = np.random.default_rng(it["seed"])
        mode = "deterministic" if k % 2 else "atomic"
        kind = "fetch_and_op" if k % 3 == 2 else it["kind"]  # every third item a FetchAndOp
        sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode=mode)
        root = inputs.unit_data(rng, g.nroots, it["bs"], it["dtype"])
        leaf = inputs.unit_data(rng, g.nleaves, it["bs"], it["dtype"])
        upd = None
        if kind == "bcast":
            want = oracle.bcast(g.nroots, g.iroot, None, root, leaf)
        elif kind == "reduce":
            want = oracle.reduce(g.nroots, g.iroot, None, leaf, root)
        else:
            if np.dtype(it["dtype"]).kind == "i":
                root = inputs.unit_data(rng, g.nroots, it["bs"], it["dtype"], "u100")
                leaf = inputs.unit_data(rng, g.nleaves, it["bs"], it["dtype"], "u100")
            else:  # bounded away from 0: the atomic chain check needs no reordering by rounding
                leaf = (1.0 + rng.random(leaf.shape)).astype(it["dtype"])
            upd = np.zeros_like(leaf)
            want = oracle.fetch_and_op(g.nroots, g.iroot, None, root, leaf, upd)
        tt, sd = TDT[it["dtype"]]
        troot = torch.from_numpy(root).cuda()
        tleaf = torch.from_numpy(leaf).cuda()
        tupd = None if upd is None else torch.from_numpy(upd).cuda()
        case.append(dict(it=it, kind=kind, g=g, sf=sf, mode=mode, root=root, leaf=leaf, upd=upd, want=want,
                         troot=troot, tleaf=tleaf, tupd=tupd, unit=S.SfUnit(sd, it["bs"])))
    batch = S.Batch([(c["sf"], c["unit"], c["kind"], "sum" if c["kind"] == "fetch_and_op" else c["it"]["op"],
                      c["troot"], c["tleaf"], c["tupd"]) for c in case])
    assert sum(c["kind"] == "fetch_and_op" for c in case) >= 8
    return case, batch


def reset(case):
    for c in case:
        c["troot"].copy_(torch.from_numpy(c["root"]))
        c["tleaf"].copy_(torch.from_numpy(c["leaf"]))
        if c["tupd"] is not None:
            c["tupd"].zero_()


def check_fetch(c, what):
    it, g = c["it"], c["g"]
    r, u = c["troot"].cpu().numpy(), c["tupd"].cpu().numpy()
    wr, wu = c["want"]
    integer = np.dtype(it["dtype"]).kind == "i"
    if integer and c["mode"] == "deterministic":
        assert same_bits(r, wr) and same_bits(u, wu), f"{what}: fetch-and-op in leaf order"
        return
    bs = it["bs"]
    for e in range(bs):  # each element of the unit is its own chain
        col = (lambda a: a if bs == 1 else a.reshape(-1, bs)[:, e])
        if integer:
            check_fetch_chain(g.iroot, np.arange(g.nleaves), col(c["root"]), col(c["leaf"]), col(u), col(r))
        else:
            rtol = 1e-12 if np.dtype(it["dtype"]) == np.float64 else 1e-5
            check_fetch_chain_fp(g.iroot, np.arange(g.nleaves), col(c["root"]), col(c["leaf"]), col(u), col(r), rtol)


def check(case, what):
    torch.cuda.synchronize()
    for k, c in enumerate(case):
        it, g = c["it"], c["g"]
        if c["kind"] == "fetch_and_op":
            check_fetch(c, f"{what}: item {k} ({c['mode']} {np.dtype(it['dtype'])} x {it['bs']})")
            continue
        if c["kind"] == "bcast":
            got = c["tleaf"].cpu().numpy()
            assert same_bits(got, c["want"]), f"{what}: item {k} bcast"
            continue
        got = c["troot"].cpu().numpy()
        exact = np.dtype(it["dtype"]).kind == "i" or c["mode"] == "deterministic" or g.iroot.size == 0
        if exact:
            assert same_bits(got, c["want"]), f"{what}: item {k} reduce {c['mode']} {it['dtype']}"
        else:
            rtol = 1e-12 if np.dtype(it["dtype"]) == np.float64 else 1e-5
            ok, worst = atomic_sum_tolerance(got, c["want"], c["root"], c["leaf"], g.iroot, rtol)
            assert ok, f"{what}: item {k} atomic sum {worst}"


def test_batch_persistent(batch_case):
    case, batch = batch_case
    reset(case)
    batch.launch()
    check(case, "persistent")


def test_batch_separate(batch_case):
    case, batch = batch_case
    reset(case)
    batch.launch_separate()
    check(case, "separate")


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_graph_replays(batch_case, mode):
    case, batch = batch_case
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    batch.graph_capture(mode, stream)
    for rep in range(3):
        reset(case)                       # eager work between replays
        torch.cuda.synchronize()
        batch.graph_launch(stream)
        stream.synchronize()
        check(case, f"graph mode {mode} replay {rep}")


def test_autotune_candidates_agree(batch_case, tmp_path):
    case, batch = batch_case
    results = []
    for lpt, tile in [(1, 1024), (4, 2048), (8, 8192), (2, 4096)]:
        batch.set_config(lpt, tile)
        reset(case)
        batch.launch()
        check(case, f"config {lpt}x{tile}")
        # deterministic items: Reduce, and FetchAndOp on integers (floating
        # point FetchAndOp takes atomics in every mode)
        results.append([c["troot"].cpu().numpy().copy() for c in case
                        if c["mode"] == "deterministic" and (c["kind"] == "reduce" or (
                            c["kind"] == "fetch_and_op" and np.dtype(c["it"]["dtype"]).kind == "i"))])
    for r in results[1:]:
        assert all(same_bits(a, b) for a, b in zip(results[0], r))
    cache = tmp_path / "tune.txt"
    batch.autotune(str(cache))
    first = batch.config()
    assert cache.read_text().count("\n") == 1
    batch.set_config(1, 1024)
    batch.autotune(str(cache))          # cache hit: same choice, no new line
    assert batch.config()[:2] == first[:2] and cache.read_text().count("\n") == 1
    reset(case)
    batch.launch()
    check(case, "autotuned")


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_graph_with_partitioned_item(mode):
    """A batch holding a large SF that takes the partitioned path (atomic
    mode) beside a small Bcast, captured before either SF has run: the
    capture allocates the scratch the per-item launches need beforehand;
    three replays with eager resets and synchronisation between them."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(950 + mode)
    gz = inputs.spmv_ghost(seed=3, nroots=20000, nleaves=300001)
    sfz = S.StarForest(gz.nroots, gz.iroot, None, gz.ranks).setup(reduce_mode="atomic", partition="on")
    rz, lz = rng.standard_normal(gz.nroots), rng.standard_normal(gz.nleaves)
    wz = oracle.reduce(gz.nroots, gz.iroot, None, lz, rz)
    gb = inputs.single_sf(seed=951, nroots=3000, nleaves=9000, leafspace=9500)
    sfb = S.StarForest(gb.nroots, gb.iroot, gb.ilocal, gb.ranks).setup()
    rb, lb = rng.standard_normal((gb.nroots, 2)), rng.standard_normal((gb.leafspace, 2))
    wb = oracle.bcast(gb.nroots, gb.iroot, gb.ilocal, rb, lb)
    t = [torch.from_numpy(a).cuda() for a in (rz, lz, rb, lb)]
    u1, u2 = S.SfUnit(S.SF_F64, 1), S.SfUnit(S.SF_F64, 2)
    batch = S.Batch([(sfz, u1, "reduce", "sum", t[0], t[1]), (sfb, u2, "bcast", "replace", t[2], t[3])])
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    batch.graph_capture(mode, stream)
    for rep in range(3):
        t[0].copy_(torch.from_numpy(rz))
        t[3].copy_(torch.from_numpy(lb))
        torch.cuda.synchronize()
        batch.graph_launch(stream)
        stream.synchronize()
        ok, worst = atomic_sum_tolerance(t[0].cpu().numpy(), wz, rz, lz, gz.iroot, 1e-12)
        assert ok, f"mode {mode} replay {rep}: partitioned item {worst:.3g}"
        assert same_bits(t[3].cpu().numpy(), wb), f"mode {mode} replay {rep}: bcast item"


def test_batch_deterministic_wave_items():
    """Deterministic Reduce and FetchAndOp items whose roots have 40..256
    leaves (one wavefront per root) and, for FetchAndOp, up to ~4000 (the
    wavefront walks the root 64 leaves at a time); units of 2 and 3
    elements, f32 / f64 / int64; the persistent launch and graph replays
    against the oracle bit for bit."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(960)
    specs = [(np.float32, 2, 300, 30000), (np.float64, 3, 200, 20000), (np.int64, 2, 20, 40000),
             (np.int32, 3, 150, 30000)]
    case = []
    for k, (dt, bs, R, L) in enumerate(specs):
        iroot = rng.integers(0, R, L).astype(np.int64)
        g = inputs.Graph(R, iroot, None, np.zeros(L, np.int64), L)
        deg = np.bincount(iroot, minlength=R)
        assert deg.max() > 32
        sf = S.StarForest(R, iroot).setup(reduce_mode="deterministic")
        integer = np.dtype(dt).kind == "i"
        root = inputs.unit_data(rng, R, bs, dt, "full" if integer else "normal")
        leaf = inputs.unit_data(rng, L, bs, dt, "full" if integer else "normal")
        if integer:
            upd0 = np.zeros_like(leaf)
            want = oracle.fetch_and_op(R, iroot, None, root, leaf, upd0)
            kind = "fetch_and_op"
        else:
            assert deg.max() <= 256
            want = oracle.reduce(R, iroot, None, leaf, root)
            kind = "reduce"
        t = dict(root=torch.from_numpy(root).cuda(), leaf=torch.from_numpy(leaf).cuda(),
                 upd=torch.from_numpy(np.zeros_like(leaf)).cuda() if integer else None)
        sd = {np.dtype(np.float32): S.SF_F32, np.dtype(np.float64): S.SF_F64, np.dtype(np.int64): S.SF_I64,
              np.dtype(np.int32): S.SF_I32}[np.dtype(dt)]
        case.append(dict(sf=sf, kind=kind, unit=S.SfUnit(sd, bs), root=root, want=want, t=t))
    batch = S.Batch([(c["sf"], c["unit"], c["kind"], "sum", c["t"]["root"], c["t"]["leaf"], c["t"]["upd"])
                     for c in case])

    def verify(what):
        torch.cuda.synchronize()
        for k, c in enumerate(case):
            got = c["t"]["root"].cpu().numpy()
            if c["kind"] == "reduce":
                assert same_bits(got, c["want"]), f"{what}: reduce item {k}"
            else:
                assert same_bits(got, c["want"][0]), f"{what}: fetch item {k} roots"
                assert same_bits(c["t"]["upd"].cpu().numpy(), c["want"][1]), f"{what}: fetch item {k} leafupdate"

    def reset_all():
        for c in case:
            c["t"]["root"].copy_(torch.from_numpy(c["root"]))
            if c["t"]["upd"] is not None:
                c["t"]["upd"].zero_()

    reset_all()
    batch.launch()
    verify("persistent")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    batch.graph_capture(0, stream)
    for rep in range(3):
        reset_all()
        torch.cuda.synchronize()
        batch.graph_launch(stream)
        stream.synchronize()
        verify(f"replay {rep}")


def test_batch_rejects_items_set_up_again():
    """Setting an item's SF up again frees the device plan the batch points
    into: every later use of the batch fails, and nothing is launched."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = inputs.single_sf(seed=961, nroots=500, nleaves=3000, leafspace=3000)
    sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup()
    root = torch.zeros(g.nroots, dtype=torch.float64, device="cuda")
    leaf = torch.zeros(g.leafspace, dtype=torch.float64, device="cuda")
    batch = S.Batch([(sf, S.SfUnit(S.SF_F64, 1), "reduce", "sum", root, leaf)])
    batch.launch()
    torch.cuda.synchronize()
    sf.setup(reduce_mode="atomic")
    for call in (lambda: batch.launch(), lambda: batch.launch_separate(), lambda: batch.set_config(4, 1024),
                 lambda: batch.graph_capture(0, torch.cuda.Stream()), lambda: batch.autotune(None)):
        with pytest.raises(S.SfError, match="SF_ERR_NOT_SETUP"):
            call()
