#!/usr/bin/env python3
"""MOCCA iterations per second for one-step three-material spectral CT on one
MI355X: 512^2 material maps, 720 views x 1024 bins fan beam, 120 energy bins,
four overlapping windows, block-diagonal SPC, clipped curvature (the "large"
workload of synth.problem).

    python bench.py [--steps K] [--warmup W] [--gpus 1]

One step = one MOCCA iteration (forward projection of fbar, per-ray spectral
model + step lengths + dual step, back-projection fused with the primal step),
with every input resident on the device.  Prints one JSON line with the
iteration rate, the projector rates, a roofline entry for the dominant kernel
(its average duration measured here with events on the library's stream) and
the FP64 oracle timed on the host as a CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MOCCA iter/s + projector GRays/s at 512^2 x4 windows; batched solves/s; p50/p99"

# MI355X: 256 CUs x 64 lanes x 2.4 GHz of non-packed VALU issue; HBM3E 8 TB/s.
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit (lane operations, an FMA counts one): what the
# method computes, counted for a generic evaluation of each step.
#   exact chord length of one (ray, pixel) pair ~ 12 (clipping the line to
#     the pixel square); forward projection adds 3 FMA (15 per nonzero of X),
#     back-projection of [q; S] 9 FMA (21; diagonal SPC [q; h] 6 -> 18).
#   one (ray, energy) pair of the energy loop ~ 45; per-ray tail (step
#     lengths, Hessian, eigen-clip, 4x4 dual solve) ~ 600; per pixel (3x3
#     solve, update, extrapolation) ~ 80.
#   window curvature (no curvature sums, no eigen-clip): ~ 23 per (ray,
#     energy) pair and ~ 60 per ray.
# The library's trapezoid form of the chord takes 5 operations (2 FP64 FMA
# for the signed distance, |.|-subtract, clamp), so its kernels execute
# fewer operations per nonzero than these counts (14 instead of 21 in the
# back-projection).
OPS = {"fp_nnz": 15, "bp_nnz_block": 21, "bp_nnz_diag": 18, "energy_clip": 45, "energy_window": 23,
       "tail_clip": 600, "tail_window": 60, "pixel": 80}
# Algorithmic HBM bytes per iteration (FP32): per ray c 4 + y in/out 8 + rho 1
# + p write/read 6 + qS write/read 18 words; per pixel f, fbar read and written 12.
BYTES_PER_RAY = 4 * 37
BYTES_PER_PIXEL = 4 * 12

KERNEL_NAMES = {0: "k_forward<3>", 1: "k_spectral_dual", 2: "k_back_primal"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large", choices=["tiny", "medium", "large"])
    ap.add_argument("--precond", default="block", choices=["block", "diag"])
    ap.add_argument("--curvature", default="clip", choices=["clip", "window"])
    ap.add_argument("--fp64-small", type=int, default=0)
    ap.add_argument("--energy-sums", default="auto", choices=["auto", "vector"],
                    help="vector: the spectral step's energy sums as per-ray vector FMAs instead of the "
                         "matrix-core contraction the plan picks where it applies")
    ap.add_argument("--lam", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3, help="whole oracle iterations timed for the CPU baseline")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--legs", default="single,batched,serving",
                    help="comma list of single (the 512^2 iteration rate), batched, serving, convergence; a run "
                         "without 'single' prints only the other legs")
    ap.add_argument("--conv-workloads", default="medium:500,large:1000",
                    help="workload:iterations pairs of the convergence leg")
    ap.add_argument("--batch-iters", type=int, default=100,
                    help="iterations per slice of the batched leg (0 skips it)")
    ap.add_argument("--batch-per-size", type=int, default=6, help="slices per size in the batched mix")
    ap.add_argument("--serve-requests", type=int, default=32, help="requests of the serving leg (0 skips it)")
    ap.add_argument("--serve-rates", default="4,64",
                    help="comma list of Poisson arrival rates (1/s) of the serving leg: a light one and one that "
                         "saturates the one-slot loop")
    ap.add_argument("--serve-tick", type=int, default=5, help="iterations between admissions and retirements")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times) to calibrate HBM byte counters")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}), flush=True)


DEFAULT_LAM = {"tiny": 3e-7, "medium": 3e-7, "large": 2e-8}


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1801_06263_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != source_hash():
        return None
    return ent.get("bytes_per_launch")


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pr, lam, precond, curvature, n_iter):
    """The FP64 oracle's MOCCA iteration on the full scan, timed on one host
    core: the system matrix X is built once (timed separately), then n_iter
    whole iterations from f = 0 are timed."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import model, mocca, projector

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        X = projector.system_matrix(pr.geom)
        t_build = time.perf_counter() - t0
        chat = model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec)
        c = synth.poisson_counts(chat, pr.seed)
        rho = np.asarray(X.sum(axis=1)).ravel()
        st = mocca.initial_state(3, X.shape[1], X.shape[0], 4)
        t0 = time.perf_counter()
        for _ in range(n_iter):
            st = mocca.mocca_step(X, rho, st, c, pr.spec, lam, precond, curvature)
        t_iter = (time.perf_counter() - t0) / n_iter
    nnz = X.nnz
    del X
    sample = (f"{n_iter} whole MOCCA iterations from f = 0 on the full {pr.geom.n}^2, {pr.geom.n_views} x "
              f"{pr.geom.n_bins} scan ({pr.spec.n_energy} energies), {t_iter:.2f} s each; the CSR system matrix "
              f"({nnz} nonzeros) built once beforehand in {t_build:.1f} s (not in the rate)")
    return {"value": round(1.0 / t_iter, 5), "unit": "iter/s", "cores": 1, "kind": "oracle", "sample": sample,
            "x_build_s": round(t_build, 1), "s_per_iteration": round(t_iter, 3), "host_cpu": host_cpu(),
            "host_nproc": os.cpu_count()}


def library_counts(plan, pr):
    """Poisson counts at the phantom from the library's own counts model."""
    import numpy as np
    import torch

    import synth
    g = pr.geom
    p = plan.forward_project(torch.as_tensor(pr.f_true.astype(np.float32)).cuda())
    chat = plan.spectral_model(p, torch.zeros(4, g.n_views, g.n_bins, device="cuda"))["chat"]
    c = synth.poisson_counts(chat.double().cpu().numpy(), pr.seed).astype(np.float32)
    return torch.from_numpy(c).cuda()


BATCH_LAM = 2e-8


def batched_leg(n_iter: int, per_size: int):
    """Batched solves/s: the mixed-size slices (128^2 .. 512^2, views 1.4 n,
    bins 2 n) each solved for n_iter iterations, as one batch (one launch
    per stage for all slices, graph replay, tuned launch shapes) and as the
    plain loop that runs each scan alone with osscir_mocca_iterate, one after
    the other, on the same stream.  Both give bit-identical maps."""
    import torch

    import synth
    from paper_1801_06263_amd import Batch, Params, Plan

    mix = synth.batch_mix(per_size)
    plans, counts = {}, []
    for pr in mix:
        n = pr.geom.n
        if n not in plans:
            plans[n] = Plan(pr.geom, pr.spec)
        counts.append(library_counts(plans[n], pr))
    params = Params(BATCH_LAM, "block", "clip", True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # the plain per-scan loop
    seq = [plans[pr.geom.n].new_state(c) for pr, c in zip(mix, counts)]
    warm = plans[mix[0].geom.n].new_state(counts[0])
    plans[mix[0].geom.n].mocca_iterate(warm, params, 2)
    torch.cuda.synchronize()
    ev[0].record()
    for pr, st in zip(mix, seq):
        plans[pr.geom.n].mocca_iterate(st, params, n_iter)
    ev[1].record()
    torch.cuda.synchronize()
    t_seq = ev[0].elapsed_time(ev[1]) * 1e-3
    # the batch: tune, capture the graph on a throw-away iteration, rebind fresh states
    b = Batch(params, len(mix))
    tmp = [plans[pr.geom.n].new_state(c) for pr, c in zip(mix, counts)]
    for i, (pr, st) in enumerate(zip(mix, tmp)):
        b.set_slot(i, plans[pr.geom.n], st, BATCH_LAM)
    t_tune = time.perf_counter()
    cfg = b.tune(2)
    t_tune = time.perf_counter() - t_tune
    b.iterate(1, use_graph=True)
    del tmp
    states = [plans[pr.geom.n].new_state(c) for pr, c in zip(mix, counts)]
    for i, (pr, st) in enumerate(zip(mix, states)):
        b.set_slot(i, plans[pr.geom.n], st, BATCH_LAM, max_iter=n_iter)
    b.iterate(0)  # uploads the new slot table outside the timed region
    torch.cuda.synchronize()
    ev[2].record()
    b.iterate(n_iter, use_graph=True)
    ev[3].record()
    torch.cuda.synchronize()
    t_batch = ev[2].elapsed_time(ev[3]) * 1e-3
    status = b.status()
    done = all(status[i][0] == 2 and status[i][1] == n_iter for i in range(len(mix)))
    equal = all(torch.equal(a.f, z.f) and torch.equal(a.y, z.y) for a, z in zip(states, seq))
    finite = all(bool(torch.isfinite(st.f).all().item()) for st in states)
    sizes = sorted(plans)
    return {
        "solves_per_s": round(len(mix) / t_batch, 3),
        "sequential_solves_per_s": round(len(mix) / t_seq, 3),
        "speedup_vs_sequential": round(t_seq / t_batch, 3),
        "ms_per_batched_iteration": round(t_batch * 1e3 / n_iter, 3),
        "ms_per_sequential_sweep": round(t_seq * 1e3 / n_iter, 3),
        "iterations_per_solve": n_iter,
        "slices": f"{len(mix)}: {per_size} each of " + "/".join(f"{n}^2" for n in sizes)
                  + " (views 1.4 n, bins 2 n, 120 energies, I0 1e6)",
        "lambda": BATCH_LAM, "graph": True, "tuned_config": cfg, "tune_s": round(t_tune, 2),
        "all_done_at_budget": done, "bitwise_equal_to_sequential": equal, "state_finite": finite,
    }


CONV_GRIDS = {
    "block": (5e-9, 1e-8, 2e-8, 5e-8, 1e-7, 2e-7, 3e-7, 5e-7),
    "mupc": (3e-7, 1e-6, 2e-6, 5e-6, 1e-5, 2e-5, 5e-5),
    "diag": (1e-9, 1e-8, 3e-8, 1e-7, 3e-7, 1e-6),
    # block SPC with nested loops: k inner steps per expansion point, the
    # same number of steps in all (each step costs one single-loop iteration)
    "nested2": (2e-8, 5e-8, 1e-7, 2e-7, 5e-7, 1e-6, 2e-6, 5e-6),
    "nested4": (2e-8, 5e-8, 1e-7, 2e-7, 5e-7, 1e-6, 2e-6, 5e-6, 1e-5),
    "nested8": (5e-8, 1e-7, 2e-7, 5e-7, 1e-6, 2e-6, 5e-6, 1e-5, 2e-5),
    # mu-PC with the same nesting, for a like-for-like comparison
    "mupc_nested4": (1e-6, 2e-6, 5e-6, 1e-5, 2e-5, 5e-5, 1e-4, 2e-4),
}


def convergence_leg(spec_str: str):
    """D_TPL(c, chat(f_n)) per iteration (the paper's Fig. 3 quantity) for
    block-diagonal SPC, mu-PC (diagonal SPC in the orthonormal material
    basis), diagonal SPC, block SPC with nested loops (2, 4 or 8 inner
    steps per expansion point) and mu-PC with 4, each over a lambda grid, clipped curvature; the
    best lambda per method is the one with the lowest final D_TPL."""
    import numpy as np
    import torch

    import synth
    from paper_1801_06263_amd import Params, Plan
    from paper_1801_06263_amd.osscir import mu_pc_spectral

    out = {}
    for item in spec_str.split(","):
        wl, n_iter = item.split(":")
        n_iter = int(n_iter)
        pr = synth.problem(wl)
        plan = Plan(pr.geom, pr.spec)
        c = library_counts(plan, pr)
        spec_t, _ = mu_pc_spectral(pr.spec)
        plan_t = Plan(pr.geom, spec_t)
        g = pr.geom
        floor = float(plan.dtpl(torch.as_tensor(pr.f_true.astype(np.float32)).cuda(), c).item())
        res = {"iterations": n_iter, "dtpl_at_truth": floor,
               "dtpl_at_zero": float(plan.dtpl(torch.zeros(3, g.n, g.n, device="cuda"), c).item())}
        marks = [m for m in (1, 10, 30, 100, 300, 1000, 2000) if m <= n_iter]
        for method, lams in CONV_GRIDS.items():
            finals, curves = [], {}
            for lam in lams:
                pl = plan_t if method.startswith("mupc") else plan
                st = pl.new_state(c)
                if "nested" in method:
                    k = int(method.split("nested")[1])
                    pre = "diag" if method.startswith("mupc") else "block"
                    _, d = pl.mocca_iterate_nested(st, Params(lam, pre, "clip", True), n_iter // k, k, dtpl=True)
                    d = d.double().cpu().numpy()
                else:
                    prm = Params(lam, "diag" if method == "mupc" else method, "clip", True)
                    d = pl.mocca_iterate(st, prm, n_iter, dtpl=True).double().cpu().numpy()
                fin = float(d[-1]) if np.isfinite(d[-1]) else float("inf")
                finals.append(fin)
                curves[lam] = {m: (float(d[m - 1]) if np.isfinite(d[m - 1]) else None) for m in marks}
            k = int(np.argmin(finals))
            res[method] = {"lambda_grid": list(lams), "final_dtpl": finals, "best_lambda": lams[k],
                           "best_curve": curves[lams[k]]}
            print(f"[bench] convergence {wl} {method}: best lambda {lams[k]:.1e}, final {finals[k]:.4e}",
                  file=sys.stderr, flush=True)
        out[wl] = res
        plan.close()
        plan_t.close()
    return out


SERVE_TOL = 1e-4


def serving_leg(n_requests: int, rate: float, per_tick: int, batch_cfg=None, seed: int = 4242):
    """Poisson arrivals (rate per second) of reconstruction requests, each a
    slice of the mixed-size scans (128^2 .. 512^2 uniformly) with its own
    phantom, an iteration budget uniform in [100, 1000] and the relative
    change stop 1e-4.  Served twice on the same arrival times: continuous
    batching (32 slots, 64 GB HBM budget, graph replay, tuned launch shapes)
    and the plain one-scan-at-a-time loop (one slot, first come first
    served).  Latency = completion - arrival; solves/s = requests /
    makespan.  Results are compared bit for bit."""
    import numpy as np
    import torch

    import synth
    from paper_1801_06263_amd import Params, Plan
    from paper_1801_06263_amd.serve import Request, Server, latency_summary

    rng = np.random.default_rng(seed)
    tmp_plans = {}
    reqs, t = [], 0.0
    for i in range(n_requests):
        size = int(rng.choice(synth.BATCH_SIZES))
        pr = synth.batch_slice(size, 1000 + i)
        if size not in tmp_plans:
            tmp_plans[size] = (pr.geom, pr.spec, Plan(pr.geom, pr.spec))
        c = library_counts(tmp_plans[size][2], pr).cpu().numpy()
        t += float(rng.exponential(1.0 / rate))
        reqs.append(Request(i, pr.geom, pr.spec, c, BATCH_LAM, max_iter=int(rng.integers(100, 1001)), tol=SERVE_TOL,
                            arrival=t))
    scans = [(g, sp) for g, sp, _ in tmp_plans.values()]
    for _, _, p in tmp_plans.values():
        p.close()
    modes = Params(BATCH_LAM, "block", "clip", True)
    out, finals = {}, {}
    for name, slots in (("batched", 32), ("sequential", 1)):
        srv = Server(modes, max_slots=slots, hbm_budget=64 << 30, iters_per_tick=per_tick)
        if batch_cfg and slots > 1:
            srv.batch.set_config(**batch_cfg)
        for g, sp in scans:
            srv.preload_plan(g, sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.run(reqs)
        makespan = time.perf_counter() - t0
        summ = latency_summary(res, makespan)
        summ["slots"] = slots
        summ["peak_hbm_gb"] = round(srv.peak_used / 1e9, 3)
        summ["ticks"] = srv.ticks
        out[name] = summ
        finals[name] = {r.rid: r for r in res}
        srv.close()
        print(f"[bench] serving {name}: {summ}", file=sys.stderr, flush=True)
    b, q = finals["batched"], finals["sequential"]
    equal = all(torch.equal(b[i].f, q[i].f) and b[i].iters == q[i].iters for i in b)
    it = np.array([r.iters for r in b.values()])
    return {
        "arrival_rate_per_s": rate, "requests": n_requests, "iters_per_tick": per_tick,
        "stop_rule": f"budget uniform [100, 1000] or relative change <= {SERVE_TOL}",
        "iterations_per_request": {"min": int(it.min()), "median": int(np.median(it)), "max": int(it.max())},
        "stopped_by_tolerance": int(sum(1 for r in b.values() if r.rel_change <= SERVE_TOL)),
        "batched": out["batched"], "sequential": out["sequential"],
        "solves_per_s_speedup": round(out["batched"]["solves_per_s"] / out["sequential"]["solves_per_s"], 3),
        "p99_latency_ratio_seq_over_batched": round(out["sequential"]["p99_latency_s"]
                                                    / out["batched"]["p99_latency_s"], 3),
        "bitwise_equal_batched_vs_sequential": equal,
    }


def serving_rates(args, cfg):
    """The serving leg at each arrival rate of --serve-rates (same requests
    and arrival draws, scaled to the rate)."""
    out = {}
    for rate in [float(r) for r in args.serve_rates.split(",") if r]:
        print(f"[bench] serving leg: {args.serve_requests} requests at {rate}/s", file=sys.stderr, flush=True)
        out[f"{rate:g}_per_s"] = serving_leg(args.serve_requests, rate, args.serve_tick, cfg)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (--gpus {args.gpus} asked): the library runs a scan on one GPU; "
              "independent slices would shard across GPUs with no exchange, which is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import torch

    import synth
    from paper_1801_06263_amd import Params, Plan

    torch.cuda.set_device(0)
    legs = set(args.legs.split(","))
    if "single" not in legs:
        line = {}
        if "batched" in legs:
            line["batched"] = batched_leg(args.batch_iters, args.batch_per_size)
        if "serving" in legs:
            cfg = line.get("batched", {}).get("tuned_config")
            line["serving"] = serving_rates(args, cfg)
        if "convergence" in legs:
            line["convergence"] = convergence_leg(args.conv_workloads)
        print(json.dumps(line), flush=True)
        if args.json_out:
            with open(args.json_out, "w") as fh:
                fh.write(json.dumps(line) + "\n")
        return
    pr = synth.problem(args.workload)
    geom = pr.geom
    lam = args.lam if args.lam is not None else DEFAULT_LAM[args.workload]
    t_setup = time.perf_counter()
    plan = Plan(geom, pr.spec)
    if args.energy_sums == "vector":
        plan.set_energy_sums(False)
    V, D, N = geom.n_views, geom.n_bins, geom.n
    L = V * D
    # synthetic measured counts from the library's own counts model at the phantom
    f_true = torch.as_tensor(pr.f_true.astype(np.float32)).cuda()
    p_true = plan.forward_project(f_true)
    chat = plan.spectral_model(p_true, torch.zeros(4, V, D, device="cuda"))["chat"]
    c = synth.poisson_counts(chat.double().cpu().numpy(), pr.seed).astype(np.float32)
    state = plan.new_state(torch.from_numpy(c).cuda())
    params = Params(lam, args.precond, args.curvature, bool(args.fp64_small))
    nnz = int(plan.ray_nnz().sum().item())
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] {args.workload}: {N}^2, {V}x{D} rays, {pr.spec.n_energy} energies, nnz(X)={nnz}, "
          f"setup {t_setup:.1f}s; warmup {args.warmup}, timed {args.steps}", file=sys.stderr, flush=True)

    # warmup, then the timed region: K whole iterations
    plan.mocca_iterate(state, params, args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    plan.mocca_iterate(state, params, args.steps)
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    finite = bool(torch.isfinite(state.f).all().item() and torch.isfinite(state.y).all().item())
    print(f"[bench] {ms_per_step:.3f} ms/iteration ({t_wall:.2f}s wall for {args.steps}), state finite={finite}",
          file=sys.stderr, flush=True)
    # the spread over repeated runs: median of 5 runs of 100 iterations
    runs = []
    for _ in range(5):
        e0.record()
        plan.mocca_iterate(state, params, 100)
        e1.record()
        torch.cuda.synchronize()
        runs.append(100.0 / (e0.elapsed_time(e1) * 1e-3))
    runs.sort()

    # per-kernel durations: the same iterations stage by stage, events on the library's stream
    stage_ms = [0.0, 0.0, 0.0]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(args.steps):
        ev[0].record()
        for s in range(3):
            plan.mocca_stage(state, params, s)
            ev[s + 1].record()
        torch.cuda.synchronize()
        for s in range(3):
            stage_ms[s] += ev[s].elapsed_time(ev[s + 1])
    stage_ms = [t / args.steps for t in stage_ms]

    # projector rates: 3-channel forward projection, 9-channel back-projection
    q9 = torch.randn(9, V, D, device="cuda")
    fp_out = torch.empty(3, V, D, device="cuda")
    bp_out = torch.empty(9, N, N, device="cuda")
    plan.forward_project(state.fbar, out=fp_out)
    plan.back_project(q9, out=bp_out)
    a0, a1, a2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    a0.record()
    for _ in range(args.steps):
        plan.forward_project(state.fbar, out=fp_out)
    a1.record()
    for _ in range(args.steps):
        plan.back_project(q9, out=bp_out)
    a2.record()
    torch.cuda.synchronize()
    fp_ms = a0.elapsed_time(a1) / args.steps
    bp_ms = a1.elapsed_time(a2) / args.steps

    # roofline of the dominant kernel
    I = pr.spec.n_energy
    clip = args.curvature == "clip"
    ops = [
        OPS["fp_nnz"] * nnz,
        (OPS["energy_clip" if clip else "energy_window"] * I + OPS["tail_clip" if clip else "tail_window"]) * L,
        OPS["bp_nnz_block" if args.precond == "block" else "bp_nnz_diag"] * nnz + OPS["pixel"] * N * N,
    ]
    dom = max(range(3), key=lambda s: stage_ms[s])
    achieved = ops[dom] / (stage_ms[dom] * 1e-3) / 1e12
    traffic = measured_traffic(KERNEL_NAMES[dom], args.workload)
    hbm_bytes = BYTES_PER_RAY * L + BYTES_PER_PIXEL * N * N
    line = {
        "metric": METRIC,
        "value": round(1000.0 / ms_per_step, 3),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N}^2 maps x3 materials, fan beam {V} views x {D} bins, "
                               f"{I} energies, 4 overlapping windows",
                   "precond": args.precond, "curvature": args.curvature, "lambda": lam,
                   "fp64_small": bool(args.fp64_small), "energy_sums": args.energy_sums, "nnz_X": nnz},
        "projector": {"fp_grays_s": round(L / (fp_ms * 1e-3) / 1e9, 3), "fp_ms_3ch": round(fp_ms, 4),
                      "bp_grays_s": round(L / (bp_ms * 1e-3) / 1e9, 3), "bp_ms_9ch": round(bp_ms, 4)},
        "stages_ms": {KERNEL_NAMES[s]: round(stage_ms[s], 4) for s in range(3)},
        "runs_5x100_iter_s": {"median": round(runs[2], 1), "min": round(runs[0], 1), "max": round(runs[4], 1)},
        "roofline": {"bound": "alu", "kernel": KERNEL_NAMES[dom], "achieved": round(achieved, 3),
                     "peak": round(PEAK_VALU_TOPS, 2), "unit": "Top/s", "frac": round(achieved / PEAK_VALU_TOPS, 4),
                     "traffic": traffic},
        "hbm": {"algorithmic_bytes_per_step": hbm_bytes,
                "achieved_gbs": round(hbm_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                "frac": round(hbm_bytes / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 5)},
        "state_finite": finite,
    }
    if "batched" in legs and args.batch_iters > 0:
        print(f"[bench] batched leg: {args.batch_per_size} slices per size, {args.batch_iters} iterations each",
              file=sys.stderr, flush=True)
        line["batched"] = batched_leg(args.batch_iters, args.batch_per_size)
        print(f"[bench] batched: {line['batched']}", file=sys.stderr, flush=True)
    if "serving" in legs and args.serve_requests > 0:
        cfg = line.get("batched", {}).get("tuned_config")
        line["serving"] = serving_rates(args, cfg)
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: {args.cpu_iters} oracle iterations on the full scan", file=sys.stderr,
              flush=True)
        line["cpu_baseline"] = cpu_baseline(pr, lam, args.precond, args.curvature, args.cpu_iters)
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as fh:
            fh.write(out + "\n")


if __name__ == "__main__":
    main()
