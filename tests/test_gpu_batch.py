"""GPU tests of the batched path: many uneven SF operations in one persistent
launch, the per-SF launches, HIP-graph replays of both, and the autotuner's
candidates -- all against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S
from helpers import atomic_sum_tolerance, same_bits

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
        sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode=mode)
        root = inputs.unit_data(rng, g.nroots, it["bs"], it["dtype"])
        leaf = inputs.unit_data(rng, g.nleaves, it["bs"], it["dtype"])
        if it["kind"] == "bcast":
            want = oracle.bcast(g.nroots, g.iroot, None, root, leaf)
        else:
            want = oracle.reduce(g.nroots, g.iroot, None, leaf, root)
        tt, sd = TDT[it["dtype"]]
        troot = torch.from_numpy(root).cuda()
        tleaf = torch.from_numpy(leaf).cuda()
        case.append(dict(it=it, g=g, sf=sf, mode=mode, root=root, leaf=leaf, want=want, troot=troot, tleaf=tleaf,
                         unit=S.SfUnit(sd, it["bs"])))
    batch = S.Batch([(c["sf"], c["unit"], c["it"]["kind"], c["it"]["op"], c["troot"], c["tleaf"]) for c in case])
    return case, batch


def reset(case):
    for c in case:
        c["troot"].copy_(torch.from_numpy(c["root"]))
        c["tleaf"].copy_(torch.from_numpy(c["leaf"]))


def check(case, what):
    torch.cuda.synchronize()
    for k, c in enumerate(case):
        it, g = c["it"], c["g"]
        if it["kind"] == "bcast":
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
        results.append([c["troot"].cpu().numpy().copy() for c in case if c["mode"] == "deterministic"])
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
