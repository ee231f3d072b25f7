"""Benchmark of the iFCTN-TC PAM sweep on one MI355X.

A step is one full PAM sweep (every factor block of eq. (updateG), the
reconstruction and the X step of eq. (updateX), with the stop-test
reductions) over the msi256 workload: 256x256x31 multispectral-image-shaped
tensor, planted iFCTN R=6 + Gaussian bumps + noise, 10% uniform sampling,
rho = 0.1.  Inputs are resident in HBM before the timed region.

Prints one JSON line with sweeps/s, the roofline of the dominant kernel
(HIP events on the job's stream) and the CPU oracle baseline.
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

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="msi256")
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
    ap.add_argument("--no-tuning", action="store_true", help="skip the rank-grid tuning leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=0, help="oracle sweeps (0 = auto, ~10-30 s)")
    ap.add_argument("--route", default="auto", choices=["auto", "percolumn", "gamma"],
                    help="factor-block route: auto (the library's default), the per-column Gram-weight "
                         "route only, or the Gamma route wherever it fits")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (scale for the HBM byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contract_msi256_traffic.txt")


def measured_traffic(workload, precision):
    """HBM bytes per contraction launch from the committed counter summary, or None.

    The summary holds FETCH_SIZE and WRITE_SIZE per dispatch, already scaled by
    a plain copy of known size; it counts only while the kernel sources are the
    ones the counters were taken on."""
    if workload != "msi256" or precision != "fp32" or not os.path.exists(TRAFFIC_FILE):
        return None
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


def cpu_baseline(name, seed, sweeps_req):
    """The FP64 oracle (single thread) on a bounded sample of the workload."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import oracle
    from paper_2511_16358_amd import workloads as W
    p = W.problem(name, seed, lambda d, r, G: oracle.reconstruct(G, d))
    O64 = p.O.astype(np.float64)
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    if ctx:
        ctx.__enter__()
    try:
        X = oracle.initial_x(O64, p.mask)
        G = {k: v.copy() for k, v in p.G0.items()}
        t0 = time.perf_counter()
        X, G, _ = oracle.pam_sweep(X, G, O64, p.mask, p.dims, p.rho)
        t1 = time.perf_counter()
        n = sweeps_req or max(1, min(40, int(15.0 / max(t1 - t0, 1e-3))))
        for _ in range(n - 1):
            X, G, _ = oracle.pam_sweep(X, G, O64, p.mask, p.dims, p.rho)
        dt = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    return {"value": n / dt, "unit": "sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} PAM sweeps of {name} (same workload, seed {seed}), float64 numpy, "
                      f"single thread, {dt:.1f} s"}


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


def serve_mix(ifctn, torch, args):
    """The served mix: requests submitted at their Poisson arrival times to a
    continuous-batching server; latency = completion - submission."""
    from paper_2511_16358_amd import workloads as W
    specs = W.served_requests(args.serve_requests, seed=0)
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
    nseq = min(args.serve_sequential, len(specs))
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
            "mix": f"{len(specs)} requests, Poisson arrivals at 200/s, orders 3-5, modes 16-256 (<= 4,194,304 entries), "
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


def main():
    args = parse()
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

    # synthetic input: planted part assembled by the library itself
    d = W.draw(args.workload, 0)
    core = ifctn.assemble(d.dims, d.ranks, d.planted, precision=ifctn.IFCTN_FP64).cpu().numpy()
    p = W.finish(d, core)
    Oin = p.O.astype(np.float64) if prec == ifctn.IFCTN_FP64 else p.O
    job = ifctn.Job(Oin, p.mask, p.G0, p.dims, p.ranks, rho=p.rho, precision=prec)
    stream = torch.cuda.current_stream()

    job.sweep(args.warmup, stats=True)
    torch.cuda.synchronize()

    # timed region: exactly K sweeps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    job.sweep(args.steps, stats=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    sweeps_per_s = args.steps / (gpu_ms / 1e3)
    st = job.sweep(0, stats=True)

    # second pass with per-kernel events (same K) for the roofline
    job.timing(True)
    job.sweep(args.steps, stats=False)
    per = {}
    for name, kc in (("contract", ifctn.KC_CONTRACT), ("solve", ifctn.KC_SOLVE),
                     ("update", ifctn.KC_UPDATE), ("gram", ifctn.KC_GRAM)):
        ms, n = job.timing_query(kc)
        per[name] = {"total_ms": ms, "launches": n, "avg_us": 1e3 * ms / max(n, 1)}
    job.timing(False)

    mask_frac = float(p.mask.mean())
    nX, rd, upd = algorithmic_bytes(p.dims, esz, mask_frac)
    # contraction launches: N per sweep; the first of each sweep after the
    # first also carries the previous sweep's X step
    N = len(p.dims)
    n_con = per["contract"]["launches"]
    n_fused = max(0, args.steps - 1)
    con_bytes = contraction_bytes(n_con, n_fused, rd, upd)
    dominant = max(per, key=lambda k: per[k]["total_ms"])
    con_gbs = con_bytes / (per["contract"]["total_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, args.precision)
    roof = {"bound": "hbm", "achieved": round(con_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(con_gbs / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "algorithmic_bytes_per_launch": round(con_bytes / max(n_con, 1)),
            "kernel": "k_contract (mode-k contraction, fused X step on mode 0)",
            "avg_us": round(per["contract"]["avg_us"], 2)}

    Xdev = job.x()
    Xf = Xdev.cpu().numpy().astype(np.float64)
    rse = float(np.linalg.norm((Xf - p.X_true).ravel()) / np.linalg.norm(p.X_true.astype(np.float64).ravel()))
    image = None
    if len(p.dims) == 3 and args.workload == "msi256":
        mp, ms, _, _ = ifctn.image_metrics(Xdev.float(), p.X_true)
        image = {"mpsnr_db": round(mp, 3), "mssim": round(ms, 4)}
    job.close()

    cmp = None
    if not args.no_compare and args.precision != "fp64":
        cmp = precision_comparison(ifctn, torch, p, W.CONFIGS[args.workload][2], args.refine)

    served = None
    if not args.no_serve:
        served = serve_mix(ifctn, torch, args)

    tune = None
    if not args.no_tuning:
        tune = tuning(ifctn, torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, 0, args.cpu_sweeps)

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
                   "dims": list(p.dims), "rank": int(p.ranks[0][1]), "rho": p.rho,
                   "precision": f"{args.precision} X streaming ({'float64' if args.precision == 'fp64' else 'float32'} arithmetic), "
                                "fp64 Gram/LDL^T/factors/reductions",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "precision_comparison": cmp,
        "serving": served,
        "tuning": tune,
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in per.items()},
        "dominant_kernel_class": dominant,
        "rse_after_timed_sweeps": rse,
        "image_metrics_after_timed_sweeps": image,
        "objective": st["objective"],
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
