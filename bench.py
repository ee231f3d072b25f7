"""Benchmark of the iFCTN-TC PAM sweep on one MI355X.

A step is one full PAM sweep (every factor block of eq. (updateG), the
reconstruction and the X step of eq. (updateX), with the stop-test
reductions) over the video144 workload: the largest single-GPU
configuration, an order-4 144x176x3x50 colour-video-shaped tensor, planted
iFCTN R=5 + a smoothly translated texture, 5% uniform sampling, rho = 0.1.
Inputs are resident in HBM before the timed region.

Prints one JSON line with sweeps/s, the roofline of the dominant kernel
class and of every class (HIP events on the job's stream), the precision
comparison (bfloat16 + float32 refinement against float32 at equal RSE) on
the image-, traffic- and video-shaped workloads, the served mix, the
rank-grid tuning batches, a secondary image-shaped (256x256x31) leg and the
CPU oracle baseline (single thread and all host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="video144")
    ap.add_argument("--secondary", default="msi256", help="a second workload timed the same way ('' = none)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"],
                    help="bf16 = bfloat16 X streaming + float32 refinement sweeps (BF16_REFINE)")
    ap.add_argument("--refine", type=int, default=30, help="float32 refinement sweeps of the bf16 path")
    ap.add_argument("--no-compare", action="store_true", help="skip the bf16-vs-fp32 equal-RSE comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-mix leg")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-precision", default="bf16", choices=["fp32", "bf16"])
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-streams", type=int, default=16)
    ap.add_argument("--serve-round", type=int, default=10)
    ap.add_argument("--serve-sequential", type=int, default=32,
                    help="requests of the mix also run alone, one after another (0 = skip)")
    ap.add_argument("--serve-sustained-rate", type=float, default=30.0,
                    help="arrival rate (requests/s) of a second, shorter served run at a load the server keeps up with")
    ap.add_argument("--serve-sustained-requests", type=int, default=128)
    ap.add_argument("--ranks", default="",
                    help="edge ranks R[a][b], a < b, row by row (e.g. 36,9,9), replacing the workload's; "
                         "initial factors are drawn for them")
    ap.add_argument("--no-tuning", action="store_true", help="skip the rank-grid tuning leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", default=None, metavar="WORKLOAD",
                    help="only run the CPU oracle baseline on this workload and print its JSON")
    ap.add_argument("--cpu-seed", type=int, default=0)
    ap.add_argument("--route", default="auto", choices=["auto", "percolumn", "gamma"],
                    help="factor-block route: auto (the library's default), the per-column Gram-weight "
                         "route only, or the Gamma route wherever it fits")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (scale for the HBM byte counters)")
    return ap.parse_args()


HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6


def measured_traffic(workload, precision):
    """HBM bytes per contraction launch from the committed counter summary, or None.

    The summary (profiles/contract_<workload>_traffic.txt) holds FETCH_SIZE
    and WRITE_SIZE per dispatch, already scaled by a plain copy of known size;
    it counts only while the kernel sources are the ones the counters were
    taken on."""
    path = os.path.join(ROOT, "profiles", f"contract_{workload}_traffic.txt")
    if precision != "fp32" or not os.path.exists(path):
        return None
    TRAFFIC_FILE = path
    rec = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("bench:"):
                for kv in line.split()[1:]:
                    k, _, v = kv.partition("=")
                    rec[k] = v
    from paper_2511_16358_amd.profsum import kernel_source_digest
    if rec.get("kernel_sources_sha256") != kernel_source_digest():
        return None
    return float(rec["hbm_bytes_per_launch"])


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "copies": 5}), flush=True)


def algorithmic_bytes(dims, esz, mask_frac):
    """Minimum HBM bytes per launch class for one sweep of the fused pipeline.

    contraction (mode k): read X once                      -> nX * esz
    fused X step (mode 0 of the next sweep, or the final
    X-step launch): read X, read the 1-bit mask, write the
    unobserved entries                                      -> nX * (esz + 1/8 + (1-p) esz)
    """
    nX = int(np.prod(dims))
    read = nX * esz
    upd = nX * (esz + 1.0 / 8.0 + (1.0 - mask_frac) * esz)
    return nX, read, upd


def contraction_bytes(n_con, n_fused, read, upd):
    """Algorithmic bytes of n_con contraction launches of which n_fused carry
    the X step: a fused launch reads X once for both, so it moves `upd`
    bytes and the others `read`."""
    return (n_con - n_fused) * read + n_fused * upd


_FORK_FN = None


def _fork_call(item):
    return _FORK_FN(item)


def fork_map(nproc):
    """A map over the columns of one factor block on nproc forked worker
    processes (they inherit the block's operands; only the solved columns
    travel back).  Timing wrapper only: the oracle's arithmetic is unchanged."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")

    def m(fn, items):
        global _FORK_FN
        _FORK_FN = fn
        items = list(items)
        with ctx.Pool(min(nproc, max(1, len(items)))) as pool:
            return pool.map(_fork_call, items, chunksize=max(1, len(items) // (4 * nproc)))
    return m


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, seed, budget_s=10.0):
    """The FP64 oracle as it stands, on a bounded sample of the workload: PAM
    sweeps single-threaded (numpy/BLAS on one thread), then with its
    per-column solves mapped over the host's cores by forked processes (at
    most 16, the CPU share of one GPU on the box).  Runs in a process of its
    own that never touches the GPU (started by bench.py after the GPU work)."""
    from threadpoolctl import threadpool_limits
    import oracle
    from paper_2511_16358_amd import workloads as W
    p = W.problem(name, seed, lambda d, r, G: oracle.reconstruct(G, d))
    O64 = p.O.astype(np.float64)
    nproc = min(16, len(os.sched_getaffinity(0)))

    def run(map_columns):
        X = oracle.initial_x(O64, p.mask)
        G = {k: v.copy() for k, v in p.G0.items()}
        t0 = time.perf_counter()
        n = 0
        while n == 0 or (time.perf_counter() - t0 < budget_s and n < 40):
            X, G, _ = oracle.pam_sweep(X, G, O64, p.mask, p.dims, p.rho, map_columns=map_columns)
            n += 1
        return n, time.perf_counter() - t0

    with threadpool_limits(limits=1):
        n1, t1 = run(map)
        nn, tn = run(fork_map(nproc))
    return {"value": round(nn / tn, 3), "unit": "sweeps/s", "cores": nproc, "kind": "oracle",
            "sample": f"{nn} PAM sweeps of {name} (same workload, seed {seed}), float64 numpy, per-column "
                      f"solves on {nproc} processes, {tn:.1f} s; single thread: {n1} sweeps in {t1:.1f} s",
            "single_thread": {"value": round(n1 / t1, 3), "unit": "sweeps/s", "cores": 1,
                              "sample": f"{n1} sweeps, {t1:.1f} s"},
            "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}


def cpu_baseline_child(name, seed):
    """cpu_baseline in a child process (the oracle never runs in the process
    that holds the GPU); returns its JSON result."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", name, "--cpu-seed",
                        str(seed)], capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def timed_run(ifctn, torch, p, precision, steps, warmup, refine=0):
    """Warm-up, then `steps` sweeps timed with events on the job's stream
    (the last `refine` of them after promotion for the bf16 path).
    Returns (ms, RSE, job)."""
    job = ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks, rho=p.rho, precision=precision)
    stream = torch.cuda.current_stream()
    if warmup:
        # warm-up on a scratch job so the timed job starts from X^0
        wj = ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks, rho=p.rho, precision=precision)
        wj.sweep(warmup, stats=True)
        wj.close()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    if precision == ifctn.IFCTN_BF16_REFINE:
        job.sweep(steps - refine, stats=False)
        job.promote()
        job.sweep(refine, stats=False)
    else:
        job.sweep(steps, stats=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    X = job.x().cpu().numpy().astype(np.float64)
    rse = float(np.linalg.norm((X - p.X_true).ravel()) / np.linalg.norm(p.X_true.astype(np.float64).ravel()))
    return ev0.elapsed_time(ev1), rse, job


def precision_comparison(ifctn, torch, p, steps, refine):
    """Equal-RSE comparison: the FP32 path and the bf16 path (steps - refine
    bfloat16 sweeps + refine float32 sweeps) over the same sweep count."""
    ms32, rse32, j = timed_run(ifctn, torch, p, ifctn.IFCTN_FP32, steps, 3)
    j.close()
    msb, rseb, j = timed_run(ifctn, torch, p, ifctn.IFCTN_BF16_REFINE, steps, 3, refine)
    j.close()
    return {"sweeps": steps,
            "fp32": {"sweeps_per_s": round(steps / (ms32 / 1e3), 2), "rse": rse32},
            "bf16_refine": {"sweeps_per_s": round(steps / (msb / 1e3), 2), "rse": rseb,
                            "bf16_sweeps": steps - refine, "fp32_refine_sweeps": refine},
            "equal_rse": bool(rseb <= 1.01 * rse32),
            "speedup_bf16_over_fp32": round(ms32 / msb, 4)}


def served_inputs(ifctn, torch, specs):
    """Device tensors of the served mix: planted part assembled by the library,
    unit max, N(0, 0.01^2) noise and Bernoulli masks from torch's device
    generator (seeded per request), initial factors from numpy."""
    from paper_2511_16358_amd import workloads as W
    out = []
    for sp in specs:
        core = ifctn.assemble(sp.dims, sp.ranks, sp.planted)                 # float32 on the device
        g = torch.Generator(device="cuda")
        g.manual_seed(sp.seed)
        X = core / core.abs().max()
        X = X + W.SERVED["noise"] * torch.randn(sp.dims, device="cuda", generator=g)
        mask = (torch.rand(sp.dims, device="cuda", generator=g) < sp.keep).to(torch.uint8)
        O = torch.where(mask.bool(), X, torch.zeros((), device="cuda"))
        obs = X[mask.bool()].double()
        rms = float(torch.sqrt((obs * obs).mean())) if obs.numel() else 1.0
        G0 = W.initial_factors(np.random.default_rng(sp.seed + 1), sp.dims, sp.ranks, rms)
        out.append((O.contiguous(), mask.contiguous(), G0))
    torch.cuda.synchronize()
    return out


def serve_mix(ifctn, torch, args, n=None, rate=None, sequential=True):
    """The served mix: requests submitted at their Poisson arrival times to a
    continuous-batching server; latency = completion - submission."""
    from paper_2511_16358_amd import workloads as W
    n = args.serve_requests if n is None else n
    rate = W.SERVED["rate"] if rate is None else rate
    specs = W.served_requests(n, seed=0, rate=rate)
    t_gen = time.perf_counter()
    inputs = served_inputs(ifctn, torch, specs)
    t_gen = time.perf_counter() - t_gen
    prec = ifctn.IFCTN_BF16_REFINE if args.serve_precision == "bf16" else ifctn.IFCTN_FP32
    refine = 30 if prec == ifctn.IFCTN_BF16_REFINE else 0
    srv = ifctn.Server(int(args.serve_budget_gb * (1 << 30)), max_active=args.serve_slots,
                       num_streams=args.serve_streams, sweeps_per_round=args.serve_round)
    done = {}
    t0 = time.perf_counter()
    for q, (sp, (O, M, G0)) in enumerate(zip(specs, inputs)):
        while time.perf_counter() - t0 < sp.arrival:
            for c in srv.poll(64):
                done[c["tag"]] = c
            time.sleep(0.0002)
        srv.submit(O, M, G0, sp.dims, sp.ranks, W.SERVED["t_max"], eps=W.SERVED["eps"], precision=prec,
                   refine_sweeps=refine, tag=q, sync=False)
    while len(done) < len(specs):
        for c in srv.poll(64, wait_ms=200):
            done[c["tag"]] = c
    wall = time.perf_counter() - t0
    srv.close()
    # the first requests of the mix again, alone and one after another through
    # ifctn_complete (same precision, refinement, t_max and eps): the rate
    # without the server's overlap of jobs
    seq = None
    nseq = min(args.serve_sequential, len(specs)) if sequential else 0
    if nseq > 0:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        seq_sweeps = 0
        for sp, (O, M, G0) in zip(specs[:nseq], inputs[:nseq]):
            _, st = ifctn.complete(O, M, G0, sp.dims, sp.ranks, W.SERVED["t_max"], eps=W.SERVED["eps"],
                                   precision=prec, refine_sweeps=refine)
            seq_sweeps += st["sweeps_done"]
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t1
        seq = {"requests": nseq, "sweeps": int(seq_sweeps), "wall_s": round(t_seq, 3),
               "sweeps_per_s": round(seq_sweeps / t_seq, 1)}
    bad = [c for c in done.values() if c["status"] != ifctn.IFCTN_OK]
    lat = np.array([c["t_done"] - c["t_submit"] for c in done.values()])
    queue = np.array([c["t_admit"] - c["t_submit"] for c in done.values()])
    sweeps = sum(c["stats"]["sweeps_done"] for c in done.values())
    first = min(c["t_submit"] for c in done.values())
    last = max(c["t_done"] for c in done.values())
    nX = np.array([np.prod(sp.dims) for sp in specs], dtype=np.float64)
    return {"requests": len(specs), "failed": len(bad),
            "p50_latency_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
            "p99_latency_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
            "mean_queue_ms": round(1e3 * float(queue.mean()), 2),
            "aggregate_sweeps_per_s": round(sweeps / (last - first), 1),
            "entry_sweeps_per_s": round(float(sum(nX[c["tag"]] * c["stats"]["sweeps_done"]
                                                  for c in done.values())) / (last - first), 1),
            "converged": int(sum(c["stats"]["converged"] for c in done.values())),
            "makespan_s": round(last - first, 3), "wall_s": round(wall, 3),
            "arrival_window_s": round(specs[-1].arrival, 3),
            "mean_entries": int(nX.mean()),
            "precision": args.serve_precision + ("+30 fp32 refine" if refine else ""),
            "server": {"hbm_budget_gb": args.serve_budget_gb, "slots": args.serve_slots,
                       "streams": args.serve_streams, "sweeps_per_round": args.serve_round},
            "input_generation_s": round(t_gen, 2),
            "sequential": seq,
            "served_over_sequential": (round((sweeps / (last - first)) / seq["sweeps_per_s"], 3)
                                       if seq else None),
            "mix": f"{len(specs)} requests, Poisson arrivals at {rate:g}/s, orders 3-5, modes 16-256 (<= 4,194,304 entries), "
                   "R in 2..6, sampling 5/10/30%, planted iFCTN N(0,1) unit max + N(0,0.01^2), "
                   "t_max 100, eps 1e-5"}


def rank_grid_run(ifctn, torch, p, grids, t_max=1000, eps=1e-5, precision=None):
    """One tensor, many rank matrices, submitted together to a server (the
    observed tensor and mask are shared device buffers); wall time from the
    first submission to the last completion, RSE of every rank."""
    prec = ifctn.IFCTN_FP32 if precision is None else precision
    from paper_2511_16358_amd import workloads as W
    O = torch.as_tensor(p.O).cuda()
    M = torch.as_tensor(p.mask).cuda()
    G0s = [W.initial_factors_for(p, r, seed=100 + q) for q, r in enumerate(grids)]
    need = sum(ifctn.workspace_bytes(p.dims, r, prec) for r in grids)
    srv = ifctn.Server(int(need * 1.2) + (64 << 20), max_active=len(grids), num_streams=min(16, len(grids)),
                       sweeps_per_round=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, (r, G0) in enumerate(zip(grids, G0s)):
        srv.submit(O, M, G0, p.dims, r, t_max, eps=eps, precision=prec, tag=q, sync=False)
    done = {}
    while len(done) < len(grids):
        for c in srv.poll(64, wait_ms=100):
            done[c["tag"]] = c
    wall = time.perf_counter() - t0
    truth = np.linalg.norm(p.X_true.astype(np.float64).ravel())
    rows = []
    for q, r in enumerate(grids):
        c = done[q]
        X = c["X"].cpu().numpy().astype(np.float64)
        rse = float(np.linalg.norm((X - p.X_true).ravel()) / truth)
        up = [int(r[a][b]) for a in range(len(p.dims)) for b in range(a + 1, len(p.dims))]
        rows.append({"ranks_upper": up, "rse": round(rse, 6), "sweeps": c["stats"]["sweeps_done"],
                     "converged": c["stats"]["converged"]})
    srv.close()
    best = min(rows, key=lambda x: x["rse"])
    return {"wall_s": round(wall, 3), "jobs": len(grids), "best": best, "grid": rows}


def tuning(ifctn, torch):
    """Rank selection as a served batch: the synthetic 20^4 Tucker-(5,5,5,5)
    tensor of Sec. 5 at 80% and 90% missing entries over uniform ranks 2..8,
    and the image-shaped tensor over the image rank grid (values up to 8)."""
    from paper_2511_16358_amd import workloads as W
    out = {}
    for miss in (0.8, 0.9):
        p = W.tucker_problem(seed=0, missing=miss)
        out[f"tucker20_rm{int(miss * 100)}"] = rank_grid_run(ifctn, torch, p, W.rank_grid_uniform(4))
    d = W.draw("msi256", 0)
    core = ifctn.assemble(d.dims, d.ranks, d.planted, precision=ifctn.IFCTN_FP64).cpu().numpy()
    p = W.finish(d, core)
    out["msi256_grid"] = rank_grid_run(ifctn, torch, p, W.rank_grid_msi())
    out["note"] = ("t_max 1000, eps 1e-5, rho 0.1 (the paper's settings); wall time covers the whole grid, "
                   "as the paper's reported times include tuning")
    return out


def load_workload(ifctn, W, name):
    """Synthetic input of a workload, its planted part assembled by the library."""
    d = W.draw(name, 0)
    core = ifctn.assemble(d.dims, d.ranks, d.planted, precision=ifctn.IFCTN_FP64).cpu().numpy()
    return W.finish(d, core)


def time_sweeps(ifctn, torch, p, prec, steps, warmup):
    """Warm-up, then exactly `steps` sweeps timed with events on the job's
    stream; then the same count again with per-kernel events.  Returns the
    timing, the per-class figures, the statistics and the job."""
    Oin = p.O.astype(np.float64) if prec == ifctn.IFCTN_FP64 else p.O
    job = ifctn.Job(Oin, p.mask, p.G0, p.dims, p.ranks, rho=p.rho, precision=prec)
    stream = torch.cuda.current_stream()
    job.sweep(warmup, stats=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    job.sweep(steps, stats=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    st = job.sweep(0, stats=True)
    job.timing(True)
    job.sweep(steps, stats=False)
    per = {}
    for name, kc in (("contract", ifctn.KC_CONTRACT), ("solve", ifctn.KC_SOLVE),
                     ("update", ifctn.KC_UPDATE), ("gram", ifctn.KC_GRAM), ("urow", ifctn.KC_UROW)):
        ms, n = job.timing_query(kc)
        per[name] = {"total_ms": ms, "launches": n, "avg_us": 1e3 * ms / max(n, 1)}
    job.timing(False)
    return gpu_ms, wall, per, st, job


def empty_launch_us(torch, n=64):
    """Average duration of a one-element fill kernel with events on the
    current stream: the floor of one dependent launch."""
    x = torch.zeros(1, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(8):
        x.fill_(1.0)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        x.fill_(2.0)
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / n * 1e3


def rooflines(ifctn, p, per, steps, esz, empty_us):
    """Roofline of every kernel class of the sweep (see the design notes):
    contraction -- HBM bytes (N reads of X per sweep, the fused X step on
    mode 0) against 8 TB/s; Gamma build -- FP64 multiply-adds of Gamma_k on
    the matrix cores against 78.6 TFLOP/s; solve -- a chain of N - 1
    dependent sub-block steps per launch, FP64 flops against 78.6 TFLOP/s
    and microseconds per step above the empty-launch floor."""
    mask_frac = float(p.mask.mean())
    nX, rd, upd = algorithmic_bytes(p.dims, esz, mask_frac)
    N = len(p.dims)
    out = {}
    n_con = per["contract"]["launches"]
    if n_con:
        con_bytes = contraction_bytes(n_con, max(0, steps - 1), rd, upd)
        gbs = con_bytes / (per["contract"]["total_ms"] * 1e-3) / 1e9
        out["contract"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                           "algorithmic_bytes_per_launch": round(con_bytes / n_con),
                           "kernel": "k_contract_rows / k_contract_cols (mode-k contraction, fused X step on mode 0)",
                           "avg_us": round(per["contract"]["avg_us"], 2)}
    plan = ifctn.plan_blocks(p.dims, p.ranks)
    g_fma = sum(f for r, f in plan if r == ifctn.ROUTE_GAMMA)
    if per["gram"]["launches"] and g_fma > 0:
        flops = 2.0 * g_fma * steps
        tfs = flops / (per["gram"]["total_ms"] * 1e-3) / 1e12
        out["gram"] = {"bound": "mfma", "achieved": round(tfs, 4), "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                       "frac": round(tfs / FP64_MFMA_PEAK_TFS, 5), "traffic": None,
                       "algorithmic_flops_per_launch": round(flops / per["gram"]["launches"]),
                       "kernel": "k_gamma (Gamma_k = Z_k^T Z_k on v_mfma_f64_16x16x4f64)",
                       "avg_us": round(per["gram"]["avg_us"], 2)}
    if per["solve"]["launches"]:
        # per column and sub-block: the H and b contraction chains and the
        # LDL^T; per sub-block: the column count of its block
        fl = 0.0
        for k in range(N):
            Ik = p.dims[k]
            for i in range(N):
                if i == k:
                    continue
                R = int(p.ranks[k][i])
                fl += Ik * (2.0 * R ** 3 / 3.0 + 2.0 * R * R)
            if plan[k][0] == ifctn.ROUTE_GAMMA:
                npk = [int(p.ranks[k][m]) * (int(p.ranks[k][m]) + 1) // 2 for m in range(N) if m != k]
                P = int(np.prod(npk))
                Rp = int(np.prod([int(p.ranks[k][m]) for m in range(N) if m != k]))
                fl += (N - 1) * Ik * 2.0 * (P + Rp)
        flops = fl * steps
        tfs = flops / (per["solve"]["total_ms"] * 1e-3) / 1e12
        avg = per["solve"]["avg_us"]
        out["solve"] = {"bound": "alu", "achieved": round(tfs, 5), "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": round(tfs / FP64_MFMA_PEAK_TFS, 6), "traffic": None,
                        "latency": {"avg_us": round(avg, 2), "dependent_steps_per_launch": N - 1,
                                    "empty_launch_us": round(empty_us, 2),
                                    "us_per_step_above_floor": round((avg - empty_us) / (N - 1), 2)},
                        "kernel": "k_solve_gamma / k_solve (per-column proximal LS, Gauss-Seidel over i)",
                        "avg_us": round(avg, 2)}
    return out


def main():
    args = parse()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.cpu_baseline_only, args.cpu_seed)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(one job's sweep runs on one GPU; the multi-GPU mode for these workloads is "
              f"independent jobs per GPU)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    from paper_2511_16358_amd import ifctn
    from paper_2511_16358_amd import workloads as W

    if args.route != "auto":
        ifctn.set_option("gamma", 0 if args.route == "percolumn" else 2)
    prec = {"fp32": ifctn.IFCTN_FP32, "fp64": ifctn.IFCTN_FP64, "bf16": ifctn.IFCTN_BF16_REFINE}[args.precision]
    esz = {"fp32": 4, "fp64": 8, "bf16": 2}[args.precision]

    p = load_workload(ifctn, W, args.workload)
    if args.ranks:
        up = [int(v) for v in args.ranks.split(",")]
        N = len(p.dims)
        if len(up) != N * (N - 1) // 2:
            sys.exit(f"--ranks needs {N * (N - 1) // 2} values for an order-{N} workload")
        r = np.zeros((N, N), dtype=np.int64)
        it = iter(up)
        for a in range(N):
            for b in range(a + 1, N):
                r[a][b] = r[b][a] = next(it)
        p = W.Problem(p.name, p.dims, r, p.O, p.mask, p.X_true, W.initial_factors_for(p, r, seed=1), p.rho,
                      p.sweeps, p.meta)
    gpu_ms, wall, per, st, job = time_sweeps(ifctn, torch, p, prec, args.steps, args.warmup)
    ms_per_step = gpu_ms / args.steps
    sweeps_per_s = args.steps / (gpu_ms / 1e3)
    empty_us = empty_launch_us(torch)
    classes = rooflines(ifctn, p, per, args.steps, esz, empty_us)
    traffic = measured_traffic(args.workload, args.precision)
    if traffic is not None and "contract" in classes:
        classes["contract"]["traffic"] = round(traffic)
    dominant = max((k for k in per if k in classes), key=lambda k: per[k]["total_ms"])
    roof = dict(classes[dominant])
    Xdev = job.x()
    Xf = Xdev.cpu().numpy().astype(np.float64)
    rse = float(np.linalg.norm((Xf - p.X_true).ravel()) / np.linalg.norm(p.X_true.astype(np.float64).ravel()))
    job.close()

    secondary = None
    if args.secondary:
        p2 = load_workload(ifctn, W, args.secondary)
        ms2, _, per2, _, job2 = time_sweeps(ifctn, torch, p2, prec, args.steps, args.warmup)
        Xd2 = job2.x()
        image = None
        if len(p2.dims) == 3 and args.secondary == "msi256":
            mp, mss, _, _ = ifctn.image_metrics(Xd2.float(), p2.X_true)
            image = {"mpsnr_db": round(mp, 3), "mssim": round(mss, 4)}
        job2.close()
        c2 = rooflines(ifctn, p2, per2, args.steps, esz, empty_us)
        t2 = measured_traffic(args.secondary, args.precision)
        if t2 is not None and "contract" in c2:
            c2["contract"]["traffic"] = round(t2)
        secondary = {"workload": f"{args.secondary}: {W.DESCRIPTIONS[args.secondary]}",
                     "value": round(args.steps / (ms2 / 1e3), 2), "unit": "sweeps/s",
                     "ms_per_step": round(ms2 / args.steps, 5), "roofline_classes": c2,
                     "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in per2.items()},
                     "image_metrics_after_timed_sweeps": image}

    cmp = None
    if not args.no_compare and args.precision != "fp64":
        cmp = {}
        for name in ("video144", "traffic214", "msi256"):
            pc = p if name == args.workload else load_workload(ifctn, W, name)
            cmp[name] = precision_comparison(ifctn, torch, pc, W.CONFIGS[name][2], args.refine)

    served = None
    if not args.no_serve:
        served = serve_mix(ifctn, torch, args)
        if args.serve_sustained_requests > 0:
            sus = serve_mix(ifctn, torch, args, n=args.serve_sustained_requests, rate=args.serve_sustained_rate,
                            sequential=False)
            served["sustained_load"] = {k: sus[k] for k in ("requests", "failed", "p50_latency_ms", "p99_latency_ms",
                                                            "mean_queue_ms", "aggregate_sweeps_per_s", "makespan_s",
                                                            "arrival_window_s", "mix")}

    tune = None
    if not args.no_tuning:
        tune = tuning(ifctn, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_child(args.workload, 0)

    out = {
        "metric": "PAM sweeps/sec",
        "value": round(sweeps_per_s, 2),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W.DESCRIPTIONS[args.workload]}",
                   "dims": list(p.dims), "rank": int(p.ranks[0][1]),
                   "ranks_upper": [int(p.ranks[a][b]) for a in range(len(p.dims)) for b in range(a + 1, len(p.dims))],
                   "rho": p.rho,
                   "precision": f"{args.precision} X streaming ({'float64' if args.precision == 'fp64' else 'float32'} arithmetic), "
                                "fp64 Gram/LDL^T/factors/reductions",
                   "routes": [["per-column", "phased", "gamma", "large-rank"][r]
                              for r, _ in ifctn.plan_blocks(p.dims, p.ranks)],
                   "parallelism": "single GPU"},
        "roofline": roof,
        "roofline_classes": classes,
        "dominant_kernel_class": dominant,
        "cpu_baseline": cpu,
        "precision_comparison": cmp,
        "secondary": secondary,
        "serving": served,
        "tuning": tune,
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in per.items()},
        "rse_after_timed_sweeps": rse,
        "objective": st["objective"],
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
