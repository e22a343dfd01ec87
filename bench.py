#!/usr/bin/env python3
"""Benchmark of the star-forest hot path on one MI355X.

Workload: the unstructured SpMV-ghost SF (paper Section 4.1) at full size --
nroots = 2,000,000, nleaves = 16,000,000, Zipf(1.1) root in-degree, 64
neighbour segments -- with every operation of the hot path on it:
SFBcast REPLACE (fp64), SFReduce SUM on the atomic and on the deterministic
path (fp64, fp32), SFReduce MAX (fp64), MAXLOC (fp64,int32), SFFetchAndOp
SUM (int64, multi-SF construction).  One step runs all of them once on data
already resident in HBM.

value = algorithmic bytes of a step (unit data + indices; roots counted once
per distinct touched root) / measured time of a step, in GB/s.

Unless ``--no-rows`` is given, more is measured after the timed loop and
reported beside it: each op after a cache-evicting write, a device copy
ceiling, the direct atomic kernels (partitioning off), the 3-D halo pattern
path vs the generic index path, the batched single launch vs per-SF
launches (eager and graph-replayed), and the differentiable gather/scatter
chain.  ``--profile-op NAME`` runs single ops (for rocprofv3 counters).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def device_code_hash():
    """Hash of the library's device code (the .hip_fatbin section of
    libsf.so; the whole file if that section is not found): HBM counters
    taken on other kernels are stale.  Builds are reproducible, so an edit of
    host code or comments keeps the hash."""
    import hashlib
    import struct
    path = os.path.join(ROOT, "paper_2102_13018_amd", "libsf.so")
    try:
        with open(path, "rb") as fh:
            b = fh.read()
    except OSError:
        return None
    data = b
    if b[:4] == b"\x7fELF" and b[4] == 2:  # 64-bit ELF: find the section
        shoff, = struct.unpack_from("<Q", b, 0x28)
        shentsize, shnum, shstrndx = struct.unpack_from("<HHH", b, 0x3A)
        secs = [struct.unpack_from("<IIQQQQIIQQ", b, shoff + i * shentsize) for i in range(shnum)]
        names = secs[shstrndx][4]
        for sec in secs:
            end = b.index(b"\0", names + sec[0])
            if b[names + sec[0]:end] == b".hip_fatbin":
                data = b[sec[4]:sec[4] + sec[5]]
                break
    return hashlib.sha256(data).hexdigest()[:16]


def measured_traffic(op):
    """HBM bytes per launch of `op` (all of its kernel dispatches) from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy), or None when the summary is missing or was taken on a
    different device code."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    ops = d.get("ops", {})
    h = device_code_hash()
    if h is None or d.get("_device_code_hash") != h or op not in ops:
        return None
    return int(ops[op]["fetch_bytes"] + ops[op]["write_bytes"])


def _dispatches(path):
    """(kernel name, counter value) per dispatch of a rocprofv3 counter CSV,
    in dispatch order."""
    import csv
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            acc.setdefault(d, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
    return [tuple(acc[d]) for d in sorted(acc)]


def _op_launches(disp, launches):
    """The dispatches of the op: the library's (sfi::) dispatches at the end of
    the run form `launches` identical launches; returns one launch's kernels
    (name, total counter value over the launches)."""
    lib = [d for d in disp if "sfi::" in d[0]]
    for per in range(1, len(lib) // launches + 1):
        tail = lib[len(lib) - per * launches:]
        names = [n for n, _ in tail]
        if all(names[i] == names[i % per] for i in range(len(names))):
            out = {}
            for n, v in tail:
                out[n] = out.get(n, 0.0) + v
            return out
    raise ValueError("no repeated launch pattern in the counter dispatches")


def pmc_summary(pmc_dir, launches, copy_bytes):
    """profiles/hbm_traffic.json and profiles/spmv_ghost_hbm_counters.md from
    rocprofv3 counter runs laid out as <pmc_dir>/<op>/<FETCH_SIZE|WRITE_SIZE>/
    pmc_counter_collection.csv (one `--profile-op <op>` run per counter).
    FETCH_SIZE and WRITE_SIZE are read in KiB and scaled by what they count
    for the run's largest plain device copy of copy_bytes."""
    ops, scale = {}, {}
    for op in sorted(os.listdir(pmc_dir)):
        vals = {}
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            path = os.path.join(pmc_dir, op, ctr, "pmc_counter_collection.csv")
            disp = _dispatches(path)
            copy = max(v for n, v in disp if "copyBuffer" in n)
            f = copy_bytes / (copy * 1024.0)
            per = {n: v * 1024.0 * f / launches for n, v in _op_launches(disp, launches).items()}
            vals[ctr] = (per, f)
        kernels = {n: {"fetch_bytes": vals["FETCH_SIZE"][0][n], "write_bytes": vals["WRITE_SIZE"][0].get(n, 0.0)}
                   for n in vals["FETCH_SIZE"][0]}
        ops[op] = {"fetch_bytes": sum(k["fetch_bytes"] for k in kernels.values()),
                   "write_bytes": sum(k["write_bytes"] for k in kernels.values()), "kernels": kernels}
        scale[op] = {"fetch": vals["FETCH_SIZE"][1], "write": vals["WRITE_SIZE"][1]}
    d = {"_device_code_hash": device_code_hash(), "_scale": scale, "ops": ops}
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json"), "w") as f:
        json.dump(d, f, indent=1)
    return d


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-rows", action="store_true",
                   help="time the step only: skip cold-cache times, copy ceiling, direct atomic and small / halo / batch / "
                        "autograd rows")
    p.add_argument("--only-row", default=None, choices=["small", "halo", "batch", "autograd", "spmv"],
                   help="run one row alone (for a profiler) and print its JSON")
    p.add_argument("--profile-op", default=None, help="comma-separated ops to run alone (steps times), for a profiler")
    p.add_argument("--copy-bytes", type=int, default=0, help="run a plain device copy of this size (counter scale)")
    p.add_argument("--pmc-summary", default=None,
                   help="write profiles/hbm_traffic.json from rocprofv3 FETCH_SIZE / WRITE_SIZE runs in this "
                        "directory (<op>/<counter>/pmc_counter_collection.csv; --steps + --warmup launches per op, "
                        "--copy-bytes the copy that scales the counters); needs no GPU")
    p.add_argument("--partition-sweep", action="store_true",
                   help="time Reduce SUM f64 and FetchAndOp SUM int64 with partitioning off / on / auto on "
                        "Zipf and uniform SFs of 2^16..2^22 leaves (the automatic threshold's evidence)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Op:
    def __init__(self, name, fn, nbytes, kernels):
        self.name, self.fn, self.nbytes, self.kernels = name, fn, nbytes, kernels
        self.times = []


def build_spmv_ops(torch, S, inputs, g):
    """The ops of one step on the SpMV-ghost SF, with their algorithmic bytes."""
    dev = torch.device("cuda")
    rng = np.random.default_rng(1234)
    L, R = g.nleaves, g.nroots
    deg = np.bincount(g.iroot, minlength=R)
    Rt = int((deg > 0).sum())
    idx = 4 * L                                     # iremote (ilocal is NULL)
    t0 = time.time()
    sf = S.StarForest(R, g.iroot, None, g.ranks).setup(reduce_mode="atomic")
    setup_s = time.time() - t0
    log(f"setup of {L} leaves: {setup_s:.2f} s, info {sf.info()}")
    # the direct persistent atomic kernels (partitioning off), timed beside the step
    sfd = S.StarForest(R, g.iroot, None, g.ranks).setup(reduce_mode="atomic", partition="off")

    xr64 = torch.from_numpy(rng.standard_normal(R)).to(dev)
    xl64 = torch.from_numpy(rng.standard_normal(L)).to(dev)
    yl64 = torch.empty(L, dtype=torch.float64, device=dev)
    xr32 = xr64.float()
    xl32 = xl64.float()
    pair = np.dtype([("v", "<f8"), ("i", "<i4"), ("pad", "<i4")])
    lp = inputs.maxloc_leaves(rng, L)
    rp = inputs.maxloc_roots(rng, R)
    lpair = torch.from_numpy(lp.view(np.uint8)).to(dev)
    rpair = torch.from_numpy(rp.view(np.uint8)).to(dev)
    root0 = np.concatenate([[0], np.cumsum(deg)[:-1]]).astype(np.int64)
    fr = torch.from_numpy(root0).to(dev)
    fl = torch.ones(L, dtype=torch.int64, device=dev)
    fu = torch.empty(L, dtype=torch.int64, device=dev)
    u64, u32 = S.SfUnit(S.SF_F64, 1), S.SfUnit(S.SF_F32, 1)
    upair, ui64 = S.SfUnit(S.SF_F64_I32, 1), S.SfUnit(S.SF_I64, 1)

    def red(mode, leaf, root, op, unit, on=sf):
        def f():
            on.set_reduce_mode(mode)
            on.reduce(leaf, root, op, unit=unit)
        return f

    def fop(mode, on=sf):
        def f():
            on.set_reduce_mode(mode)
            on.fetch_and_op(fr, fl, fu, "sum", unit=ui64)
        return f

    b8 = lambda u: L * u + Rt * u + idx            # Bcast
    r8 = lambda u: L * u + 2 * Rt * u + idx        # Reduce
    f8 = lambda u: 2 * L * u + 2 * Rt * u + idx    # FetchAndOp
    ops = [
        Op("bcast_replace_f64", lambda: sf.bcast(xr64, yl64, "replace", unit=u64), b8(8), "k_bcast_move"),
        Op("reduce_sum_f64_atomic", red("atomic", xl64, xr64, "sum", u64), r8(8), "k_sp_move + k_sp_reduce<atomic>"),
        Op("reduce_sum_f64_det", red("deterministic", xl64, xr64, "sum", u64), r8(8),
           "k_sp_move + k_sp_reduce + k_det_chunk"),
        Op("reduce_sum_f32_det", red("deterministic", xl32, xr32, "sum", u32), r8(4),
           "k_sp_move + k_sp_reduce + k_det_chunk"),
        Op("reduce_max_f64_atomic", red("atomic", xl64, xr64, "max", u64), r8(8), "k_sp_move + k_sp_reduce<atomic>"),
        Op("reduce_maxloc_det", red("deterministic", lpair, rpair, "maxloc", upair), r8(16),
           "k_sp_move + k_sp_reduce + k_det_chunk"),
        Op("fetch_and_op_i64_det", fop("deterministic"), f8(8),
           "k_sp_move + k_sp_fop<det> + k_sp_span_scan + k_sp_move<add bases>"),
        Op("fetch_and_op_i64_atomic", fop("atomic"), f8(8), "k_sp_move + k_sp_fop<atomic> + k_sp_move"),
    ]
    direct = [
        Op("reduce_sum_f64_atomic_direct", red("atomic", xl64, xr64, "sum", u64, sfd), r8(8), "k_reduce_atomic"),
        Op("reduce_max_f64_atomic_direct", red("atomic", xl64, xr64, "max", u64, sfd), r8(8), "k_reduce_atomic"),
        Op("fetch_and_op_i64_atomic_direct", fop("atomic", sfd), f8(8), "k_fop_atomic_hot"),
    ]
    data = dict(xr64=xr64, xl64=xl64, deg=deg, Rt=Rt, setup_s=setup_s)
    return sf, ops, direct, data


class CacheFlush:
    """Evicts an op's data from the L2s and the 256 MB Infinity Cache before
    it runs.  kind "read" reads a 1 GiB buffer (a reduction): the caches then
    hold clean lines of that buffer and none of the op's data.  kind "write"
    overwrites the buffer instead, which also leaves up to 256 MB of dirty
    lines that the op pays to write back -- time that belongs to the flush,
    reported beside the headline."""

    def __init__(self, torch, kind="read"):
        self.torch, self.kind = torch, kind
        self.buf = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        self.buf.fill_(1.0)
        self.acc = torch.empty((), dtype=torch.float64, device="cuda")

    def __call__(self):
        if self.kind == "read":
            self.torch.sum(self.buf, dim=0, out=self.acc)
        else:
            self.buf.fill_(1.0)


def time_ops(torch, ops, steps, warmup, flush=None):
    """Warm up, then time exactly `steps` steps; every op is bracketed by
    events on the current stream (the stream the library launches on).  With
    `flush` (a CacheFlush), the caches are flushed before every op, outside
    its events: L2 and the Infinity Cache hold none of the op's data when it
    starts (cold)."""
    for _ in range(warmup):
        for op in ops:
            if flush is not None:
                flush()
            op.fn()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in ops]
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        for k, op in enumerate(ops):
            if flush is not None:
                flush()
            ev[s][k][0].record()
            op.fn()
            ev[s][k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s in range(steps):
        for k, op in enumerate(ops):
            op.times.append(ev[s][k][0].elapsed_time(ev[s][k][1]))
    return wall


def cold_write_flush(torch, ops, steps, warmup, step_bytes):
    """The step with a 1 GiB write before every op: the op also writes back
    the flush's dirty lines that the Infinity Cache still holds."""
    for o in ops:
        o.times = []
    fl = CacheFlush(torch, "write")
    time_ops(torch, ops, steps, warmup, flush=fl)
    del fl
    dev_ms = float(np.mean([sum(o.times[s] for o in ops) for s in range(steps)]))
    return {"cache": "cold, flushed by a 1 GiB write (dirty lines left in the Infinity Cache)",
            "value": round(step_bytes / dev_ms / 1e6, 1), "ms_per_step": round(dev_ms, 3),
            "ops": {o.name: round(float(np.median(o.times)) * 1e3, 1) for o in ops}}


def warm_ops(torch, ops, steps, warmup):
    """The step's ops back to back without flushes (the Infinity Cache keeps
    what the previous op left): a labelled side row."""
    for o in ops:
        o.times = []
    wall = time_ops(torch, ops, steps, warmup)
    out = {}
    for o in ops:
        med = float(np.median(o.times))
        out[o.name] = {"us": round(med * 1e3, 1), "GBps": round(o.nbytes / med / 1e6, 1),
                       "frac_peak": round(o.nbytes / med / 1e6 / HBM_PEAK_GBS, 4)}
    step_bytes = sum(o.nbytes for o in ops)
    return {"cache": "warm (ops back to back, no flush)", "value": round(step_bytes / (wall / steps) / 1e9, 1),
            "ms_per_step": round(wall * 1e3 / steps, 3), "ops": out}


def copy_ceiling(torch, nbytes=1 << 31):
    """Measured device-to-device copy rate (read + write bytes / time)."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(5):
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del a, b
    return round(2 * nbytes / float(np.min(ts)) / 1e6, 1)


def cpu_baseline(g, budget_s=8.0):
    """The oracle, as it stands, on the same SF: Bcast, Reduce SUM and
    FetchAndOp, in two builds -- the OpenMP variants (leaves split among the
    threads for Bcast, roots for Reduce and FetchAndOp, each root's leaves in
    leaf order: the same bits) on every host thread it is given, and the
    sequential definitions on one.  Each leg runs whole rounds of the three
    ops until its budget is spent; reports algorithmic bytes / time."""
    import oracle
    rng = np.random.default_rng(99)
    L, R = g.nleaves, g.nroots
    deg = np.bincount(g.iroot, minlength=R)
    Rt = int((deg > 0).sum())
    xr = rng.standard_normal(R)
    xl = rng.standard_normal(L)
    root0 = np.concatenate([[0], np.cumsum(deg)[:-1]]).astype(np.int64)
    ones, zeros = np.ones(L, np.int64), np.zeros(L, np.int64)
    nb = {"bcast": L * 8 + Rt * 8 + 4 * L, "reduce": L * 8 + 2 * Rt * 8 + 4 * L,
          "fetch": 2 * L * 8 + 2 * Rt * 8 + 4 * L}

    def leg(bcast, reduce, fetch):
        jobs = [("bcast_replace_f64", lambda: bcast(R, g.iroot, None, xr, xl), nb["bcast"]),
                ("reduce_sum_f64", lambda: reduce(R, g.iroot, None, xl, xr), nb["reduce"]),
                ("fetch_and_op_i64", lambda: fetch(R, g.iroot, None, root0, ones, zeros), nb["fetch"])]
        tot_b, tot_t, rounds = 0, 0.0, 0
        while tot_t < budget_s:
            for name, fn, n in jobs:
                t0 = time.perf_counter()
                fn()
                tot_t += time.perf_counter() - t0
                tot_b += n
            rounds += 1
        return round(tot_b / tot_t / 1e9, 4), rounds, tot_t

    threads = oracle.omp_threads()
    v_omp, r_omp, t_omp = leg(oracle.bcast_omp, oracle.reduce_omp, oracle.fetch_and_op_omp)
    v_seq, r_seq, t_seq = leg(oracle.bcast, oracle.reduce, oracle.fetch_and_op)
    ops = "(bcast_replace_f64, reduce_sum_f64, fetch_and_op_i64)"
    return {"value": v_omp, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{r_omp} rounds of {ops} on the full spmv_ghost SF, OpenMP oracle on {threads} threads, "
                      f"{t_omp:.1f} s",
            "sequential": {"value": v_seq, "unit": "GB/s", "cores": 1,
                           "sample": f"{r_seq} rounds of {ops}, sequential C oracle, {t_seq:.1f} s"},
            "cpu": cpu_model(), "host_threads": os.cpu_count()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def graph_time_us(torch, fn, reps=20):
    """Device time per call of a short op: `reps` calls captured in one HIP
    graph (no host gaps between kernels), replayed and timed with events."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(5):
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e3 / reps)
    return float(np.median(times))


def small_row(torch, S, inputs, steps):
    """The 16K-leaf SF with holes (Fig. 2's kind at test scale): 4096 roots,
    16384 leaves on a random subset of 20000 slots.  Launch-bound, so each op
    is timed as 20 graph-captured calls."""
    g = inputs.single_sf(seed=1)
    dev = torch.device("cuda")
    rng = np.random.default_rng(6)
    deg = np.bincount(g.iroot, minlength=g.nroots)
    Rt = int((deg > 0).sum())
    L = g.nleaves
    idx = 8 * L  # iremote and ilocal (a random subset: no pattern)
    root = torch.from_numpy(rng.standard_normal(g.nroots)).to(dev)
    leaf = torch.from_numpy(rng.standard_normal(g.leafspace)).to(dev)
    ri = torch.from_numpy(rng.integers(0, 100, g.nroots).astype(np.int32)).to(dev)
    li = torch.from_numpy(rng.integers(0, 100, g.leafspace).astype(np.int32)).to(dev)
    ui = torch.zeros(g.leafspace, dtype=torch.int32, device=dev)
    f64, i32 = S.SfUnit(S.SF_F64, 1), S.SfUnit(S.SF_I32, 1)
    sf = S.StarForest(g.nroots, g.iroot, g.ilocal, g.ranks).setup()
    cases = {
        "bcast_replace_f64": (lambda: sf.bcast(root, leaf, "replace", unit=f64), L * 8 + Rt * 8 + idx),
        "reduce_sum_f64": (lambda: sf.reduce(leaf, root, "sum", unit=f64), L * 8 + 2 * Rt * 8 + idx),
        "reduce_max_f64": (lambda: sf.reduce(leaf, root, "max", unit=f64), L * 8 + 2 * Rt * 8 + idx),
        "fetch_and_op_i32": (lambda: sf.fetch_and_op(ri, li, ui, "sum", unit=i32), 2 * L * 4 + 2 * Rt * 4 + idx),
    }
    out = {}
    for name, (fn, nb) in cases.items():
        us = graph_time_us(torch, fn)
        out[name] = {"us": round(us, 2), "alg_MB": round(nb / 1e6, 3), "GBps": round(nb / us / 1e3, 1)}
    return {"workload": "single_sf(nroots=4096, nleaves=16384, leafspace=20000)",
            "timing": "20 calls per HIP graph", "ops": out}


def halo_row(torch, S, inputs, steps):
    """Periodic 256^3 halo: pattern path vs generic index path.  The ops are a
    few microseconds long, so each is timed as 20 graph-captured calls."""
    g = inputs.halo3d(256)
    dev = torch.device("cuda")
    rng = np.random.default_rng(5)
    deg = np.bincount(g.iroot, minlength=g.nroots)
    Rt = int((deg > 0).sum())
    out = {}
    for bs in (1, 3):
        root = torch.from_numpy(rng.standard_normal((g.nroots, bs))).to(dev)
        leaf = torch.empty((g.nleaves, bs), dtype=torch.float64, device=dev)
        u = S.SfUnit(S.SF_F64, bs)
        for pat in (True, False):
            sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="deterministic", use_patterns=pat)
            idx = 0 if pat else 4 * g.nleaves
            for kind in ("bcast", "reduce"):
                fn = (lambda: sf.bcast(root, leaf, "replace", unit=u)) if kind == "bcast" else \
                    (lambda: sf.reduce(leaf, root, "sum", unit=u))
                nb = g.nleaves * 8 * bs + (1 if kind == "bcast" else 2) * Rt * 8 * bs + idx
                us = graph_time_us(torch, fn)
                out[f"{kind}_bs{bs}_{'pattern' if pat else 'generic'}"] = {
                    "us": round(us, 2), "alg_MB": round(nb / 1e6, 2), "GBps": round(nb / us / 1e3, 1)}
    return {"workload": "halo3d(n=256, 26 segments, 396296 ghost leaves)", "timing": "20 calls per HIP graph",
            "ops": out}


def batch_row(torch, S, inputs, steps):
    items = inputs.batch_mix(seed=4)
    dev = torch.device("cuda")
    bitems, keep, nbytes = [], [], 0
    tdt = {np.dtype(np.float64): (torch.float64, S.SF_F64, 8), np.dtype(np.float32): (torch.float32, S.SF_F32, 4),
           np.dtype(np.int32): (torch.int32, S.SF_I32, 4)}
    for it in items:
        g = it["graph"]
        rng = np.random.default_rng(it["seed"])
        tt, sd, es = tdt[it["dtype"]]
        bs = it["bs"]
        sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode="auto")
        root = torch.from_numpy(inputs.unit_data(rng, g.nroots, bs, it["dtype"])).to(dev)
        leaf = torch.from_numpy(inputs.unit_data(rng, g.nleaves, bs, it["dtype"])).to(dev)
        deg = np.bincount(g.iroot, minlength=g.nroots)
        Rt = int((deg > 0).sum())
        u = es * bs
        nbytes += g.nleaves * u + (1 if it["kind"] == "bcast" else 2) * Rt * u + 4 * g.nleaves
        bitems.append((sf, S.SfUnit(sd, bs), it["kind"], it["op"], root, leaf))
        keep.append(sf)
    batch = S.Batch(bitems)
    batch.autotune(None)
    cfg = batch.config()
    stream = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(stream):
        batch.graph_capture(0, stream)
        res_graph_persist = Op("graph_one_launch", lambda: batch.graph_launch(stream), nbytes, "")
        torch.cuda.synchronize()
        for name, fn in (("one_launch", lambda: batch.launch(stream)),
                         ("separate", lambda: batch.launch_separate(stream))):
            op = Op(name, fn, nbytes, "")
            time_ops(torch, [op], steps, 3)
            res[name] = op
        time_ops(torch, [res_graph_persist], steps, 3)
        res["graph_one_launch"] = res_graph_persist
        batch.graph_capture(1, stream)
        op = Op("graph_separate", lambda: batch.graph_launch(stream), nbytes, "")
        time_ops(torch, [op], steps, 3)
        res["graph_separate"] = op
    # host wall time of one launch-to-sync, median over reps
    wall = {}
    for name, fn in (("one_launch", lambda: batch.launch(stream)), ("separate", lambda: batch.launch_separate(stream))):
        ts = []
        for _ in range(10):
            t0 = time.perf_counter()
            fn()
            stream.synchronize()
            ts.append(time.perf_counter() - t0)
        wall[name] = round(float(np.median(ts)) * 1e6, 1)
    out = {k: {"us": round(float(np.median(v.times)) * 1e3, 1),
               "GBps": round(nbytes / float(np.median(v.times)) / 1e6, 1)} for k, v in res.items()}
    return {"workload": f"batch_mix(64 SFs, {sum(i['graph'].nleaves for i in items)} leaves)",
            "alg_bytes": nbytes, "autotuned": {"lpt": cfg[0], "tile": cfg[1], "tiles": cfg[2]},
            "device": out, "host_wall_us": wall}


def autograd_row(torch, S, inputs, steps, g=None):
    from paper_2102_13018_amd import autograd as A
    g = g if g is not None else inputs.knn_graph(seed=5)
    dev = torch.device("cuda")
    rng = np.random.default_rng(6)
    sf = S.StarForest(g.nroots, g.iroot, None, None).setup(reduce_mode="deterministic")
    h = torch.from_numpy(rng.standard_normal((g.nroots, 16)).astype(np.float32)).to(dev).requires_grad_(True)
    a = [torch.from_numpy((rng.standard_normal(g.nleaves) / np.sqrt(8)).astype(np.float32)).to(dev)
         for _ in range(3)]
    G = torch.from_numpy(rng.standard_normal((g.nroots, 16)).astype(np.float32)).to(dev)
    deg = np.bincount(g.iroot, minlength=g.nroots)
    Rt = int((deg > 0).sum())
    L = g.nleaves

    def step():
        loss = A.chain_loss(sf, h, a, G, checkpoint=True)
        loss.backward()
        h.grad = None

    op = Op("chain", step, 0, "")
    time_ops(torch, [op], max(3, steps // 4), 2)
    # per-layer SF traffic: forward Bcast + Reduce, backward Reduce + Bcast,
    # plus the checkpoint recompute of the forward pair
    u = 64
    bc = L * u + Rt * u + 4 * L
    rd = L * u + 2 * Rt * u + 4 * L
    sf_bytes = 3 * (2 * (bc + rd) + (bc + rd))
    ms = float(np.median(op.times))
    return {"workload": f"knn(npoints={g.nroots}, k=8) fp32 x16, 3-layer checkpointed chain",
            "step_us": round(ms * 1e3, 1), "sf_alg_bytes": sf_bytes,
            "sf_GBps_lower_bound": round(sf_bytes / ms / 1e6, 1)}


def build_knn_ops(torch, S, g):
    """The differentiable gather/scatter workload's two SF ops alone: SFBcast
    REPLACE and the deterministic SFReduce SUM of fp32 x 16 units (64 bytes)
    on the 1M-point k-NN graph (8M leaves, in-degree 0..20)."""
    dev = torch.device("cuda")
    rng = np.random.default_rng(7)
    L, R = g.nleaves, g.nroots
    deg = np.bincount(g.iroot, minlength=R)
    Rt = int((deg > 0).sum())
    sf = S.StarForest(R, g.iroot, None, None).setup(reduce_mode="deterministic")
    root = torch.from_numpy(rng.standard_normal((R, 16)).astype(np.float32)).to(dev)
    leaf = torch.from_numpy(rng.standard_normal((L, 16)).astype(np.float32)).to(dev)
    leaf_out = torch.empty_like(leaf)
    root_acc = root.clone()
    u = S.SfUnit(S.SF_F32, 16)
    ub = 64
    ops = [Op("knn_bcast_f32x16", lambda: sf.bcast(root, leaf_out, "replace", unit=u), L * ub + Rt * ub + 4 * L,
              "k_bcast_move"),
           Op("knn_reduce_sum_f32x16_det", lambda: sf.reduce(leaf, root_acc, "sum", unit=u),
              L * ub + 2 * Rt * ub + 4 * L, "k_det_small_all")]
    return sf, ops, (root, leaf, leaf_out, root_acc)


def knn_row(torch, S, g, steps, flush, copy_gbps):
    """Each op alone, cold (flush before every run), with its roofline."""
    sf, ops, keep = build_knn_ops(torch, S, g)
    time_ops(torch, ops, steps, 2, flush=flush)
    out = {}
    for o in ops:
        avg = float(np.mean(o.times))
        ach = o.nbytes / avg / 1e6
        out[o.name] = {"us": round(float(np.median(o.times)) * 1e3, 1), "avg_us": round(avg * 1e3, 1),
                       "alg_MB": round(o.nbytes / 1e6, 1), "GBps": round(ach, 1),
                       "frac_peak": round(ach / HBM_PEAK_GBS, 4),
                       "frac_copy_ceiling": round(ach / copy_gbps, 4) if copy_gbps else None,
                       "kernel": o.kernels, "traffic": measured_traffic(o.name)}
    return {"workload": f"knn(npoints={g.nroots}, k=8) fp32 x16 (64-byte units), each op alone",
            "cache": "cold (1 GiB read before every op)", "ops": out}


def spmv_row(torch, S, inputs, steps):
    """Section 4.1's SpMV on one rank's share of a split matrix (1M rows, A
    15 entries per row, B 4 per row over a 250K-entry ghost vector): y = A x
    + B lvec with SFBcast(x -> lvec) on a second stream overlapped with A x,
    against the same three steps serialised on one stream; and y = M^T x."""
    d = inputs.split_matrix(seed=7)
    dev = torch.device("cuda")
    sf = S.StarForest(d["n"], d["iroot"]).setup()
    A = S.Csr(d["n"], d["n"], *d["A"])
    B = S.Csr(d["n"], d["m"], *d["B"])
    At, Bt = A.transpose(), B.transpose()
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.standard_normal(d["n"])).to(dev)
    lvec = torch.zeros(d["m"], dtype=torch.float64, device=dev)
    y = torch.zeros(d["n"], dtype=torch.float64, device=dev)
    comm = torch.cuda.Stream()
    u = S.SfUnit(S.SF_F64, 1)

    def serial():
        sf.bcast(x, lvec, "replace", unit=u)
        A.spmv(x, y)
        B.spmv(lvec, y, accumulate=True)

    ops = [Op("overlapped", lambda: S.spmv(sf, A, B, x, lvec, y, comm_stream=comm), 0, "sf_spmv"),
           Op("serial", serial, 0, "bcast; A x; B lvec"),
           Op("transpose", lambda: S.spmv_transpose(sf, At, Bt, x, lvec, y), 0, "sf_spmv_transpose"),
           Op("bcast_alone", lambda: sf.bcast(x, lvec, "replace", unit=u), 0, "k_bcast_move")]
    time_ops(torch, ops, steps, 3)
    out = {o.name: round(float(np.median(o.times)) * 1e3, 1) for o in ops}
    nnz = int(d["A"][0][-1] + d["B"][0][-1])
    # matrix bytes (8-byte values, 4-byte columns, 8-byte row offsets) and
    # the vectors read and written once
    mbytes = 12 * nnz + 16 * (d["n"] + 1) + 8 * (2 * d["n"] + 2 * d["m"])
    return {"workload": d["meta"]["name"], "us": out, "overlap_saving_us": round(out["serial"] - out["overlapped"], 1),
            "matrix_vector_MB": round(mbytes / 1e6, 1),
            "overlapped_GBps": round(mbytes / out["overlapped"] / 1e3, 1)}


def partition_sweep(torch, S, inputs, steps):
    """Median device time (us) of Reduce SUM f64 and FetchAndOp SUM int64 in
    both modes, with the partitioned path off, on and automatic, on Zipf SFs
    (nroots = nleaves / 8) and on SFs with uniform roots of mean degree 2 and
    8, of 2^16..2^22 leaves."""
    out = {}
    for fam in ("zipf", "uniform2", "uniform8"):
        for lg in range(16, 23):
            L = 1 << lg
            if fam == "zipf":
                g = inputs.spmv_ghost(seed=3, nroots=max(1, L // 8), nleaves=L)
            else:
                R = max(1, L // int(fam[7:]))
                iroot = np.random.default_rng(lg).integers(0, R, L).astype(np.int64)
                g = inputs.Graph(R, iroot, None, np.zeros(L, np.int64), L)
            rng = np.random.default_rng(1)
            leaf = torch.from_numpy(rng.standard_normal(L)).cuda()
            root = torch.from_numpy(rng.standard_normal(g.nroots)).cuda()
            li = torch.ones(L, dtype=torch.int64, device="cuda")
            ri = torch.zeros(g.nroots, dtype=torch.int64, device="cuda")
            ui = torch.zeros(L, dtype=torch.int64, device="cuda")
            row = {}
            for part in ("off", "on", "auto"):
                for mode in ("deterministic", "atomic"):
                    sf = S.StarForest(g.nroots, g.iroot, None, g.ranks).setup(reduce_mode=mode, partition=part)
                    ops = [Op("reduce", lambda: sf.reduce(leaf, root, "sum", unit=S.SfUnit(S.SF_F64, 1)), 0, ""),
                           Op("fetch", lambda: sf.fetch_and_op(ri, li, ui, "sum", unit=S.SfUnit(S.SF_I64, 1)), 0, "")]
                    time_ops(torch, ops, steps, 3)
                    for o in ops:
                        row[f"{o.name}_{mode[:3]}_{part}"] = round(float(np.median(o.times)) * 1e3, 1)
            out[f"{fam} 2^{lg}"] = row
            log(f"{fam} 2^{lg}: {row}")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.pmc_summary:
        d = pmc_summary(args.pmc_summary, args.steps + args.warmup, args.copy_bytes)
        for op, v in d["ops"].items():
            log(f"{op:32s} fetch {v['fetch_bytes'] / 1e6:8.1f} MB  write {v['write_bytes'] / 1e6:8.1f} MB")
        return
    import torch
    from paper_2102_13018_amd import inputs
    from paper_2102_13018_amd import sf as S
    S.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_bytes:
        # a plain device copy of known size: the scale of the HBM counters
        n = args.copy_bytes // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied 3 x {args.copy_bytes} bytes")
        del a, b
        if not args.profile_op:
            return

    if args.partition_sweep:
        print(json.dumps({"partition_sweep": partition_sweep(torch, S, inputs, args.steps)}), flush=True)
        return

    if args.only_row:
        fn = {"small": small_row, "halo": halo_row, "batch": batch_row, "autograd": autograd_row,
              "spmv": spmv_row}[args.only_row]
        print(json.dumps({args.only_row: fn(torch, S, inputs, args.steps)}), flush=True)
        return

    t0 = time.time()
    g = inputs.spmv_ghost(seed=3)
    log(f"generated spmv_ghost in {time.time() - t0:.1f} s")
    sf, ops, direct, data = build_spmv_ops(torch, S, inputs, g)
    if args.profile_op:
        names = args.profile_op.split(",")
        pick = [o for o in ops + direct if o.name in names]
        if len(pick) < len(names):
            gk = inputs.knn_graph(seed=5)
            _, kops, keep = build_knn_ops(torch, S, gk)
            pick += [o for o in kops if o.name in names]
        assert len(pick) == len(names), f"unknown op in {args.profile_op}"
        time_ops(torch, pick, args.steps, args.warmup)
        for o in pick:
            log(f"{o.name}: median {np.median(o.times) * 1e3:.1f} us over {len(o.times)} launches")
        return

    # the step, cold: the 256 MB Infinity Cache and the L2s are flushed by a
    # 1 GiB read before every op (outside the op's events)
    flush = CacheFlush(torch, "read")
    torch.cuda.synchronize()
    wall = time_ops(torch, ops, args.steps, args.warmup, flush=flush)
    step_bytes = sum(o.nbytes for o in ops)
    dev_ms = float(np.mean([sum(o.times[s] for o in ops) for s in range(args.steps)]))
    value = step_bytes / dev_ms / 1e6
    per_op = {}
    for o in ops:
        med = float(np.median(o.times))
        per_op[o.name] = {"us": round(med * 1e3, 1), "alg_MB": round(o.nbytes / 1e6, 1),
                          "GBps": round(o.nbytes / med / 1e6, 1),
                          "frac_peak": round(o.nbytes / med / 1e6 / HBM_PEAK_GBS, 4)}
        log(f"{o.name:28s} {med * 1e3:9.1f} us  {o.nbytes / med / 1e6:8.1f} GB/s (cold)")
    copy_gbps = copy_ceiling(torch)
    # dominant op: the largest share of step time; one launch of it is one
    # begin/end pair, i.e. the sequence of kernels named in "kernel"
    dom = max(ops, key=lambda o: float(np.mean(o.times)))
    avg_ms = float(np.mean(dom.times))
    achieved = dom.nbytes / avg_ms / 1e6
    roofline = {"bound": "hbm", "kernel": dom.kernels, "op": dom.name,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom.name),
                "alg_bytes_per_launch": dom.nbytes, "avg_launch_us": round(avg_ms * 1e3, 1),
                "cache": "cold", "copy_ceiling_GBps": copy_gbps,
                "frac_of_copy_ceiling": round(achieved / copy_gbps, 4)}
    out = {"metric": "effective HBM GB/s (unit data + indices) for SFBcast/SFReduce vs peak; batched vs per-SF time",
           "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(dev_ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "spmv_ghost(nroots=2000000, nleaves=16000000, zipf=1.1, 64 segments, seed=3)",
                      "ops_per_step": [o.name for o in ops], "step_alg_bytes": step_bytes,
                      "cache": "cold: a 1 GiB read flushes L2 and the Infinity Cache before every op; "
                               "ms_per_step sums the ops' event times, the flushes lie outside them "
                               "(warm numbers: ops_warm; after a 1 GiB write instead: ops_cold_write_flush)",
                      "wall_ms_per_step_with_flushes": round(wall * 1e3 / args.steps, 3),
                      "setup_s": round(data["setup_s"], 2), "parallelism": "single-gpu"},
           "ops": per_op, "roofline": roofline, "copy_ceiling_GBps": copy_gbps,
           "value_vs_copy_ceiling": round(value / copy_gbps, 4)}
    if not args.no_rows:
        # beside the step (after it, so that a profile of `--no-rows` sees the
        # step's kernels only): the warm step, the direct atomic kernels, and
        # the small / halo / batch / k-NN / autograd rows
        out["ops_warm"] = warm_ops(torch, ops, args.steps, args.warmup)
        out["ops_cold_write_flush"] = cold_write_flush(torch, ops, args.steps, args.warmup, step_bytes)
        time_ops(torch, direct, max(5, args.steps // 2), 2)
        direct_row = {}
        for o in direct:
            med = float(np.median(o.times))
            direct_row[o.name] = {"us": round(med * 1e3, 1), "GBps": round(o.nbytes / med / 1e6, 1),
                                  "kernel": o.kernels, "traffic": measured_traffic(o.name)}
            log(f"{o.name:28s} {med * 1e3:9.1f} us  {o.nbytes / med / 1e6:8.1f} GB/s")
        out["row_direct_atomic"] = direct_row
        del sf, ops, direct, data
        for name, fn in (("small", small_row), ("halo", halo_row), ("batch", batch_row), ("spmv", spmv_row)):
            try:
                out[f"row_{name}"] = fn(torch, S, inputs, args.steps)
            except Exception as e:  # a row that cannot run is reported, not hidden
                out[f"row_{name}"] = {"error": repr(e)}
            log(f"row {name}: {out[f'row_{name}']}")
        gk = None
        try:
            gk = inputs.knn_graph(seed=5)
            out["row_knn"] = knn_row(torch, S, gk, args.steps, flush, copy_gbps)
        except Exception as e:
            out["row_knn"] = {"error": repr(e)}
        log(f"row knn: {out['row_knn']}")
        try:
            out["row_autograd"] = autograd_row(torch, S, inputs, args.steps, gk)
        except Exception as e:
            out["row_autograd"] = {"error": repr(e)}
        log(f"row autograd: {out['row_autograd']}")
    del flush
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
