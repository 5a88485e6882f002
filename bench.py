"""Benchmark: Gauss-Newton CP decomposition steps on one MI355X.

Workload: dense 400 x 400 x 400 FP32 tensor with an exact rank-100 CP structure (i.i.d. N(0,1)
planted factors), rank-100 decomposition from an N(0,1) initial guess. One timed step is one
Gauss-Newton iteration (all-mode MTTKRP, Grams, gradient, preconditioned CG with eps_cg = 1e-3
and at most 20 iterations, factor update) followed by the direct relative residual that the
stopping test reads. Inputs are resident in HBM before timing starts.

Further legs (reported beside the headline value): MTTKRP TFLOP/s per mode in FP32 and FP64;
time to relative residual 1e-8 with FP64 storage against the mixed FP32 -> FP64 run; 64 uneven
problems advanced together on HIP streams; an 80^4 order-4 rank-64 tensor stored in bfloat16,
split bfloat16, FP32 and FP64 (MTTKRP time and error, GN step time, per-step residual error
against the FP64-storage run); the CPU oracle on a bounded sample of the headline workload.

Prints one JSON line. Run: python bench.py [--steps K] [--warmup W]
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

PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
METRIC = "GN steps/sec + MTTKRP TFLOP/s at 400^3 R=100; time-to-residual 1e-8 mixed vs FP64"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=400)
    ap.add_argument("--rank", type=int, default=100)
    ap.add_argument("--mttkrp-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-target", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-streams", type=int, default=8)
    ap.add_argument("--no-order4", action="store_true",
                    help="skip the 80^4 R=64 bfloat16 / split-bfloat16 leg")
    ap.add_argument("--profile-bf16", action="store_true",
                    help="only run 3 cp_mttkrp calls per mode on the 80^4 R=64 tensor in bfloat16 "
                         "and split bfloat16 (for counter runs)")
    ap.add_argument("--trajectory", type=int, default=0, metavar="STEPS",
                    help="only run STEPS plain Gauss-Newton steps from the seeded start of the "
                         "headline workload, FP32 and FP64 storage, printing each step's damping, "
                         "CG iterations, gradient and update norms and residual, then exit")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the HBM copy bandwidth and the FP32, FP64 and bf16 matrix-"
                         "core rates of this GPU (libcppeaks.so) and print them as JSON")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only time the oracle's MTTKRP, GN step, ALS sweep and residual at "
                         "300^3 R=50 and 400^3 R=100 on the host and print them as JSON")
    ap.add_argument("--profile-batched", action="store_true",
                    help="only run the 64-problem batched workload as a batch program replayed "
                         "from one graph: --warmup then --steps batch steps (for kernel traces)")
    ap.add_argument("--profile-step", action="store_true",
                    help="only run the headline loop (--warmup then --steps Gauss-Newton steps with "
                         "their residuals and run restarts) and exit (for kernel traces)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run each single-mode MTTKRP and one device copy of X of known size "
                         "(the workload the rocprofv3 counter runs are taken on), then exit")
    return ap.parse_args()


def make_inputs(s, R, dtype):
    import torch

    from workloads import gaussian_factors, planted_tensor, seed_for
    rng = np.random.default_rng(seed_for(3, 0))
    B = gaussian_factors((s, s, s), R, rng)
    X = planted_tensor(B)
    A0 = gaussian_factors((s, s, s), R, np.random.default_rng(seed_for(3, 0, init=True)))
    Xd = torch.from_numpy(X.astype(dtype)).cuda()
    return X, A0, Xd


def event_time(fn, reps, stream):
    """Average duration of fn() measured with HIP events on the library's stream."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / 1e3 / reps


def event_samples(fn, reps, stream):
    """Per-call durations (s) of fn(), each bracketed by its own pair of HIP events."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        fn()
        ev[i + 1].record(stream)
    ev[-1].synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(reps)]


def warm_gpu(P, Xd, A, seconds=0.5):
    """Untimed MTTKRP calls over every mode for about `seconds`, so that the kernel timings that
    follow see the clocks of a busy GPU: right after start-up the same kernel runs 5 to 10%
    slower for tens of milliseconds."""
    import torch
    ws = P.Workspace()
    Ms = [torch.empty((Xd.shape[n], A[0].shape[1]), dtype=Xd.dtype, device="cuda")
          for n in range(Xd.dim())]
    t0 = time.perf_counter()
    calls = 0
    while time.perf_counter() - t0 < seconds:
        for n in range(Xd.dim()):
            P.mttkrp(Xd, A, n, out=Ms[n], ws=ws)
        calls += Xd.dim()
        torch.cuda.synchronize()
    return calls


def mttkrp_times(P, Xd, A, reps, stream):
    """Per mode: median and mean duration of one cp_mttkrp call (factor preparation, main kernel,
    partial-tile reduction), and median and mean duration of its main kernel alone, from HIP
    events that cp_mttkrp_marked records on the stream right around that kernel's launch. The
    modes are timed round-robin, call by call, so that every mode sees the same clock state."""
    import torch
    ws = P.Workspace()
    R = A[0].shape[1]
    modes = range(Xd.dim())
    Ms = [torch.empty((Xd.shape[n], R), dtype=Xd.dtype, device="cuda") for n in modes]
    for n in modes:
        for _ in range(3):
            P.mttkrp(Xd, A, n, out=Ms[n], ws=ws)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    rec = [[(ev(), ev(), ev(), ev()) for _ in range(reps)] for _ in modes]
    for per_mode in rec:          # creates the HIP events
        for es in per_mode:
            for e in es:
                e.record(stream)
    torch.cuda.synchronize()
    for k in range(reps):
        for n in modes:
            c0, k0, k1, c1 = rec[n][k]
            c0.record(stream)
            P.mttkrp(Xd, A, n, out=Ms[n], ws=ws, marks=(k0, k1))
            c1.record(stream)
    torch.cuda.synchronize()
    out = {}
    for n in modes:
        ts = [c0.elapsed_time(c1) / 1e3 for c0, _, _, c1 in rec[n]]
        tk = [k0.elapsed_time(k1) / 1e3 for _, k0, k1, _ in rec[n]]
        out[n] = (float(np.median(ts)), float(np.mean(ts)), float(np.median(tk)),
                  float(np.mean(tk)))
    return out


# HBM traffic of the single-mode MTTKRP at 400^3 R=100 FP32, from two rocprofv3 counter runs
# (FETCH_SIZE, then WRITE_SIZE) of `bench.py --profile-kernels`, each divided by what the same
# counter reads for a device copy of X (256 MB read + 256 MB written), so 1.0 = exact bytes.
# Valid only for the kernel source it was taken on.
MTTKRP_TRAFFIC = {
    "source_sha256": "a4dda4356460f1a14b3437309d61ef80f22cd13bd2fb94bb9c5a99e4bb91c436",
    "bytes_per_launch": 319149006,   # mean over the three modes of the main kernel
}


def order4_leg(P, torch, reps, stream):
    """80^4 order-4 tensor, rank 64, log-uniform column norms, noise 1e-3: MTTKRP per mode and
    GN steps with the tensor stored in bfloat16, split bfloat16, FP32 and FP64 (factors FP32,
    FP64 for FP64 storage), and the per-step error of each against the FP64-storage run."""
    from workloads import make_problem
    dims, R = (80, 80, 80, 80), 64
    p = make_problem(dims, R, workload=4, problem=0, kind="lognorm", noise=1e-3)
    X64 = torch.from_numpy(p.x).cuda()
    X32 = X64.float()
    forms = {"bf16": P.to_bf16(X32), "bf16x3": P.to_bf16(X32, split=True), "f32": X32, "f64": X64}
    xbytes = {"bf16": 2, "bf16x3": 4, "f32": 4, "f64": 8}
    # start: the planted factors with 10% relative elementwise perturbation (an N(0,1) start is
    # scaled far off the column norms of up to 100 and sends the first steps away)
    rng = np.random.default_rng(4500)
    A32 = [torch.tensor(b * (1.0 + 0.1 * rng.standard_normal(b.shape)), dtype=torch.float32,
                        device="cuda") for b in p.planted]
    A64 = [a.double() for a in A32]
    flops = 2.0 * float(np.prod(dims)) * R
    ws = P.Workspace()
    M64 = [P.mttkrp(X64, A64, n, ws=ws) for n in range(4)]
    out = {}
    for name, X in forms.items():
        A = A64 if name == "f64" else A32
        modes = {}
        for n in range(4):
            M = torch.empty((dims[n], R), dtype=A[0].dtype, device="cuda")
            for _ in range(3):
                P.mttkrp(X, A, n, out=M, ws=ws)
            ts = event_samples(lambda: P.mttkrp(X, A, n, out=M, ws=ws), reps, stream)
            t = float(np.median(ts))
            err = float(torch.linalg.norm(M.double() - M64[n]) / torch.linalg.norm(M64[n]))
            modes[f"mode{n}"] = dict(median_ms=t * 1e3, tflops=flops / t / 1e12,
                                     x_read_gbs=float(np.prod(dims)) * xbytes[name] / t / 1e9,
                                     rel_err_vs_fp64_storage=err)
        # all four modes at one point (cp_mttkrp_all): FP32/FP64 storage takes modes 0..2 from
        # one pass over X (dimension tree + outer-mode contraction) and mode 3 from a second;
        # the bfloat16 forms take one pass per mode
        Ms = [torch.empty((dims[n], R), dtype=A[0].dtype, device="cuda") for n in range(4)]
        for _ in range(3):
            P.mttkrp_all(X, A, out=Ms, ws=ws)
        ta = float(np.median(event_samples(lambda: P.mttkrp_all(X, A, out=Ms, ws=ws), reps,
                                           stream)))
        modes["all"] = dict(median_ms=ta * 1e3, passes_over_x=2 if name in ("f32", "f64") else 4,
                            sum_of_single_mode_ms=sum(modes[f"mode{n}"]["median_ms"]
                                                      for n in range(4)),
                            rel_err_vs_fp64_storage=max(
                                float(torch.linalg.norm(Ms[n].double() - M64[n])
                                      / torch.linalg.norm(M64[n])) for n in range(4)))
        del Ms
        # GN steps from the same start and damping schedule; the first eight steps' direct
        # residual against the FP64 master tensor, and the step time (20 CG iterations)
        Ag = [a.clone() for a in A]
        gn = P.GaussNewton(X, Ag, P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
        traj = []
        for _ in range(8):
            gn.step()
            r = P.residual(X64, [a.double() for a in gn.A], ws=ws).cpu()
            traj.append(float(r[0] / r[1]))
        # each timed step starts from the same factors (restored outside the events), so every
        # sample is the same work: 20 CG iterations from the start point
        At = [a.clone() for a in A]
        sb = P.stats_buffer(X64.device)
        ws2 = P.Workspace()
        samples = []
        for k in range(7):
            for a, a0 in zip(At, A):
                a.copy_(a0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.gn_step(X, At, 1e-4, 0.0, 20, stats=sb, ws=ws2)
            e1.record(stream)
            e1.synchronize()
            if k >= 2:
                samples.append(e0.elapsed_time(e1))
        sst = P.read_stats(sb)
        out[name] = dict(mttkrp=modes, gn_step_20cg_ms=float(np.median(samples)),
                         gn_step_cg_iters=sst["cg_iters"], gn_step_status=sst["status"],
                         residual_first_steps=traj)
        del Ag, gn, At
    # time to relative residual 2e-3 (twice the noise level) from the same start: FP64 storage
    # alone, and the precision ladder bfloat16 -> split bfloat16 -> FP64
    target = 2e-3
    # untimed runs first, so that the timed ones reuse cached workspace allocations
    P.gn_to_target(X64, [a.clone() for a in A64], target, max_steps=40)
    P.gn_ladder_to_target([forms["bf16"], forms["bf16x3"], X64], [a.clone() for a in A32], target,
                          max_steps=40)
    Af = [a.clone() for a in A64]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, h64 = P.gn_to_target(X64, Af, target, P.GNConfig(cg_tol=1e-3, cg_maxiter=20), max_steps=40)
    t64 = time.perf_counter() - t0
    Al = [a.clone() for a in A32]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Alad, hl = P.gn_ladder_to_target([forms["bf16"], forms["bf16x3"], X64], Al, target,
                                     P.GNConfig(cg_tol=1e-3, cg_maxiter=20), max_steps=40)
    tl = time.perf_counter() - t0
    rl = P.residual(X64, [a.double() for a in Alad], ws=ws).cpu()
    ladder = dict(target=target, fp64_seconds=t64, fp64_steps=len(h64), fp64_residual=h64[-1],
                  ladder_seconds=tl, ladder_steps=[(k, r, ok) for k, r, ok in hl],
                  ladder_residual=float(rl[0] / rl[1]), speedup=t64 / tl)
    log(f"[bench] 80^4 time to residual {target}: FP64 {t64 * 1e3:.1f} ms in {len(h64)} steps; ladder "
        f"{tl * 1e3:.1f} ms, steps " + " ".join(f"{k}{'' if ok else '(rejected)'}" for k, _, ok in hl))
    for name in out:
        out[name]["residual_err_vs_fp64_per_step"] = [
            abs(a - b) / b for a, b in zip(out[name]["residual_first_steps"], out["f64"]["residual_first_steps"])]
    log("[bench] 80^4 R=64 MTTKRP per mode (ms): " + "; ".join(
        f"{k} " + " ".join(f"{v['mttkrp'][f'mode{n}']['median_ms']:.4f}" for n in range(4)) for k, v in out.items()))
    log("[bench] 80^4 R=64 all-mode MTTKRP (ms, against the sum of single modes): " + "; ".join(
        f"{k} {v['mttkrp']['all']['median_ms']:.4f} ({v['mttkrp']['all']['sum_of_single_mode_ms']:.4f})"
        for k, v in out.items()))
    log("[bench] 80^4 MTTKRP rel. error vs FP64 storage (mode 0): " + ", ".join(
        f"{k} {v['mttkrp']['mode0']['rel_err_vs_fp64_storage']:.2e}" for k, v in out.items()))
    del X64, X32, forms, M64
    log("[bench] 80^4 GN residual after 8 steps: " + ", ".join(
        f"{k} {v['residual_first_steps'][-1]:.3e}" for k, v in out.items()))
    return dict(workload="dense 80^4 tensor, rank-64 CP with N(0,1) factors whose columns are "
                         "scaled log-uniformly over [1,100], noise 1e-3; rank-64 GN-CG from the "
                         "planted factors with 10% relative perturbation",
                time_to_target=ladder,
                hbm_peak_gbs=PEAK_HBM_GBS, **out)


def gn_vs_als_leg(P, torch, stream, steps=50):
    """Workload 2 (300^3, R = 50, pairwise column cosine 0.9, noise 1e-6, FP64): 50 Gauss-Newton
    steps (eps_cg 1e-3, at most 20 CG iterations, the damping schedule) against ALS sweeps from
    the same start (Section 5's comparison), each step followed by the direct residual into a
    device history (no host synchronisation inside the timed loops). Reported at equal steps
    (50 sweeps) and at equal wall time (the ALS sweeps that fit in the GN run's time)."""
    from workloads import make_problem
    p = make_problem((300, 300, 300), 50, workload=2, kind="congruent", noise=1e-6)
    X = torch.tensor(p.x, dtype=torch.float64, device="cuda")

    def run(opt, n):
        hist = torch.empty((n, 2), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(n):
            opt.step()
            P.residual(X, opt.A, out=hist[k], ws=opt.ws)
        e1.record(stream)
        e1.synchronize()
        h = hist.cpu().numpy()
        return e0.elapsed_time(e1) / 1e3, [float(a / b) for a, b in h]

    fresh = lambda: [torch.tensor(a, device="cuda") for a in p.init]   # noqa: E731
    # untimed runs first: workspace allocation and code loading stay outside the timed loops
    run(P.GaussNewton(X, fresh(), P.GNConfig(cg_tol=1e-3, cg_maxiter=20)), 2)
    run(P.ALS(X, fresh()), 2)
    gn = P.GaussNewton(X, fresh(), P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
    t_gn, h_gn = run(gn, steps)
    t_als1, _ = run(P.ALS(X, fresh()), 5)
    n_eq = max(steps, int(t_gn / (t_als1 / 5)))
    t_als, h_als = run(P.ALS(X, fresh()), n_eq)
    per_sweep = t_als / n_eq
    k_eq = min(n_eq, max(1, int(t_gn / per_sweep)))
    log(f"[bench] 300^3 R=50 congruent: {steps} GN steps {t_gn * 1e3:.1f} ms -> residual "
        f"{h_gn[-1]:.3e}; ALS {steps} sweeps -> {h_als[steps - 1]:.3e}, {k_eq} sweeps in the same "
        f"time -> {h_als[k_eq - 1]:.3e}")
    return {"workload": "dense 300^3 FP64 tensor, rank-50 CP with pairwise column cosine 0.9 in "
                        "every mode, noise 1e-6; rank 50 from an N(0,1) start",
            "gn_steps": steps, "gn_seconds": t_gn, "gn_residuals": h_gn,
            "als_sweep_ms": per_sweep * 1e3, "als_residuals_first_50": h_als[:steps],
            "equal_steps": {"gn": h_gn[-1], "als": h_als[steps - 1]},
            "equal_time": {"seconds": t_gn, "als_sweeps": k_eq, "gn": h_gn[-1],
                           "als": h_als[k_eq - 1]},
            "note": "residual = direct relative residual after each step or sweep, read from a "
                    "device history; the timed loops include those residual passes"}


def objective_leg(P, torch, Xd, A0, stream, reps=10):
    """The differentiable objective at 400^3, R = 100 (FP32): forward + backward of
    cp_objective, in the direct form (residual pass forward, gradient backward) and the fused
    form (gradient and f by the expansion in the forward, the backward only scales)."""
    out = {}
    for method in ("direct", "fused"):
        A = [torch.tensor(a, dtype=torch.float32, device="cuda", requires_grad=True) for a in A0]

        def fb():
            for a in A:
                a.grad = None
            P.cp_objective(Xd, A, method=method).backward()
        for _ in range(3):
            fb()
        t = event_time(fb, reps, stream)
        out[method] = {"fwd_bwd_ms": t * 1e3, "per_s": 1.0 / t}
    log(f"[bench] objective forward+backward at 400^3 R=100: direct {out['direct']['fwd_bwd_ms']:.3f}"
        f" ms, fused {out['fused']['fwd_bwd_ms']:.3f} ms")
    out["note"] = ("cp_objective forward + backward, HIP events; fused: f by the expansion "
                   "(cancels near an exact fit), the gradient bits of the direct form")
    return out


def high_rank_leg(P, torch, stream):
    """Section 5's high-rank regime at s = 150, R = 200 (R above every mode size), FP64: one
    Gauss-Newton step, one ALS sweep and the direct residual, HIP-event timed."""
    from workloads import make_problem
    p = make_problem((150, 150, 150), 200, workload=0, problem=200, noise=1e-2)
    X = torch.tensor(p.x, dtype=torch.float64, device="cuda")
    gn = P.GaussNewton(X, [torch.tensor(a, device="cuda") for a in p.init],
                       P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
    for _ in range(2):
        gn.step()
    t_gn = event_time(gn.step, 5, stream)
    cg_iters = gn.stats()["cg_iters"]
    als = P.ALS(X, [torch.tensor(a, device="cuda") for a in p.init], 1e-2)
    als.step()
    t_als = event_time(als.step, 5, stream)
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    P.residual(X, gn.A, out=out, ws=gn.ws)
    t_res = event_time(lambda: P.residual(X, gn.A, out=out, ws=gn.ws), 5, stream)
    log(f"[bench] 150^3 R=200 FP64: GN step {t_gn * 1e3:.3f} ms ({cg_iters} CG its last step), "
        f"ALS sweep {t_als * 1e3:.3f} ms, direct residual {t_res * 1e3:.3f} ms")
    # above R = 208 the inverse, the Cholesky factor and CG work on tiles in global memory
    p3 = make_problem((150, 150, 150), 300, workload=0, problem=300, noise=1e-2)
    X3 = torch.tensor(p3.x, dtype=torch.float64, device="cuda")
    gn3 = P.GaussNewton(X3, [torch.tensor(a, device="cuda") for a in p3.init],
                        P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
    gn3.step()
    t_gn3 = event_time(gn3.step, 3, stream)
    its3 = gn3.stats()["cg_iters"]
    als3 = P.ALS(X3, [torch.tensor(a, device="cuda") for a in p3.init], 1e-2)
    als3.step()
    t_als3 = event_time(als3.step, 3, stream)
    log(f"[bench] 150^3 R=300 FP64: GN step {t_gn3 * 1e3:.3f} ms ({its3} CG its last step), "
        f"ALS sweep {t_als3 * 1e3:.3f} ms")
    del X3, gn3, als3
    return {"workload": "dense 150^3 FP64 tensor, rank-200 CP with N(0,1) factors, noise 1e-2; "
                        "rank 200 > s (Section 5's high-rank regime)",
            "gn_step_ms": t_gn * 1e3, "gn_cg_iters_last": cg_iters, "als_sweep_ms": t_als * 1e3,
            "residual_ms": t_res * 1e3,
            "rank_300": {"workload": "the same shape at rank 300 (above 208: blocked inverse, "
                                     "Cholesky and CG in global memory)",
                         "gn_step_ms": t_gn3 * 1e3, "gn_cg_iters_last": its3,
                         "als_sweep_ms": t_als3 * 1e3}}


def measure_peaks(torch):
    """HBM stream-copy bandwidth (1 GiB read + 1 GiB written per launch; three launch shapes, the
    best is reported) and register-only MFMA loops (16x16x4 FP32, 16x16x4 FP64, 16x16x32 bf16;
    1024 workgroups of four wavefronts), from libcppeaks.so; the best of three runs of 10
    launches each."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_1910_12331_amd", "libcppeaks.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1910_12331_amd.build`")
    lib = C.CDLL(path)
    lib.cpk_copy_gbs.restype = C.c_double
    lib.cpk_copy_gbs.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int]
    lib.cpk_mfma_tflops.restype = C.c_double
    lib.cpk_mfma_tflops.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    torch.cuda.synchronize()
    copies = {f"{b}x256_v{v}": max(lib.cpk_copy_gbs(src.data_ptr(), dst.data_ptr(), n, 10, b, v)
                                   for _ in range(3))
              for b, v in ((1024, 0), (65536, 0), (65536, 2))}
    copy = max(copies.values())
    del src, dst
    out = torch.empty(4096, dtype=torch.float64, device="cuda")
    rates = {}
    for kind, name, iters in ((0, "fp32_16x16x4", 4000), (1, "fp64_16x16x4", 4000),
                              (2, "bf16_16x16x32", 8000)):
        rates[name] = max(lib.cpk_mfma_tflops(kind, out.data_ptr(), 1024, 256, iters, 10)
                          for _ in range(3))
    log(f"[peaks] copy {copy:.0f} GB/s; MFMA TFLOP/s " +
        ", ".join(f"{k} {v:.1f}" for k, v in rates.items()))
    return {"hbm_copy_gbs": copy, "hbm_copy_configs_gbs": copies, "mfma_tflops": rates,
            "vendor": {"hbm_gbs": PEAK_HBM_GBS, "fp32_tflops": PEAK_FP32_MFMA_TFLOPS,
                       "fp64_tflops": PEAK_FP64_MFMA_TFLOPS, "bf16_tflops": 2500.0},
            "note": "copy: 2 x bytes / time; MFMA: register-only loops, 32 (FP64: 16) "
                    "independent accumulators per wavefront"}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            return max(int(i.get("num_threads", 1)) for i in info), \
                ", ".join(sorted({f"{i.get('internal_api')} {i.get('version')}" for i in info}))
    except Exception:
        pass
    return os.cpu_count(), "unknown"


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X64, A0, gpu_iters, seconds):
    """The oracle (NumPy/SciPy FP64 on the FP32-rounded inputs) doing the work of the timed GPU
    steps: each step is the oracle's Gauss-Newton step with the CG iteration count the GPU step
    took (eps_cg = 0 and that count as the cap), plus its direct residual. The residual, a sum of
    squared differences over the tensor, is timed on one slab of a tenth of mode 0 and scaled by
    ten; the steps run in the timed window's order until about `seconds` have passed."""
    import oracle as O
    Xh = X64.astype(np.float32).astype(np.float64)
    Ah = [a.astype(np.float32).astype(np.float64) for a in A0]
    O.mttkrp(Xh, Ah, 0)                       # warm-up (BLAS threads, page-in)
    sched = O.LambdaSchedule()
    n_cpu, t_steps = 0, 0.0
    while t_steps < seconds and n_cpu < len(gpu_iters):
        t0 = time.perf_counter()
        Ah, _ = O.gn_step(Xh, Ah, sched.value, 0.0, int(gpu_iters[n_cpu]))
        t_steps += time.perf_counter() - t0
        sched.advance()
        n_cpu += 1
    slab = Xh.shape[0] // 10
    t0 = time.perf_counter()
    O.residual(Xh[:slab], [Ah[0][:slab]] + Ah[1:])
    t_res = (time.perf_counter() - t0) * Xh.shape[0] / slab
    per_step = t_steps / n_cpu + t_res
    cores, blas = blas_threads()
    return dict(value=1.0 / per_step, unit="GN steps/s", cores=cores, kind="oracle",
                sample=f"{n_cpu} oracle GN steps with the timed GPU steps' CG iteration counts "
                       f"({t_steps:.1f} s) + the oracle's direct residual on a {slab}-row slab of "
                       f"mode 0 scaled by {Xh.shape[0] / slab:g} ({t_res:.1f} s per step); "
                       f"FP64 on the FP32-rounded inputs",
                step_seconds=t_steps / n_cpu, residual_seconds=t_res, cpu=cpu_model(), blas=blas)


def cpu_table(shapes=((300, 50), (400, 100)), runs=10, warm=3):
    """Oracle timings on the host for the operations of one Gauss-Newton step and one ALS sweep
    (FP64, seeded inputs of each shape with N(0,1) planted factors and start): single-mode
    MTTKRP, a GN step with exactly 20 CG iterations and with eps_cg = 1e-3 (at most 20), an ALS
    sweep, and the direct residual (on a slab of a tenth of mode 0, scaled). `warm` untimed runs,
    then median and mean over `runs` (the residual: 3 runs)."""
    import oracle as O
    from workloads import make_problem
    out = dict(cpu=cpu_model(), threads=blas_threads()[0], blas=blas_threads()[1],
               nproc=os.cpu_count(), shapes={})
    for s, R in shapes:
        p = make_problem((s, s, s), R, workload=3, problem=s)
        X, A = p.x.astype(np.float32).astype(np.float64), [a.astype(np.float32).astype(np.float64)
                                                            for a in p.init]
        row = {}

        def timeit(name, fn, n=runs, w=warm):
            for _ in range(w):
                fn()
            ts = []
            for _ in range(n):
                t0 = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - t0)
            row[name] = dict(median_s=float(np.median(ts)), mean_s=float(np.mean(ts)), runs=n)
            log(f"[cpu-table] {s}^3 R={R} {name}: median {np.median(ts):.4f} s over {n}")

        for n in range(3):
            timeit(f"mttkrp_mode{n}", lambda n=n: O.mttkrp(X, A, n))
        timeit("gn_step_20cg", lambda: O.gn_step(X, A, 1e-4, 0.0, 20))
        its = O.gn_step(X, A, 1e-4, 1e-3, 20)[1].cg_iters
        timeit("gn_step_eps1e-3", lambda: O.gn_step(X, A, 1e-4, 1e-3, 20))
        row["gn_step_eps1e-3"]["cg_iters"] = its
        timeit("als_sweep", lambda: O.als_sweep(X, A))
        slab = s // 10
        timeit("residual_slab", lambda: O.residual(X[:slab], [A[0][:slab]] + A[1:]), n=3, w=1)
        row["residual_scaled_s"] = row["residual_slab"]["median_s"] * s / slab
        out["shapes"][f"{s}^3 R={R}"] = row
    return out


def headline_runs(P, torch, Xd, A0, warmup, steps, target=1e-6):
    """The timed loop. A step is one Gauss-Newton iteration (Algorithm 1 body: eps_cg 1e-3, at
    most 20 CG iterations, the damping schedule) followed by the direct relative residual that
    its stopping test reads on the host. Runs go from the seeded start until the residual reaches
    the FP32 floor target (1e-6, where the mixed-precision driver leaves FP32 storage); the next
    step then starts a new run from the same start (factors copied back, schedule reset). Past
    that floor the FP32 gradient is rounding noise, and a step taken there leaves the converged
    point. Returns (ms per step, residuals of the timed steps, runs completed in the timed
    window, the optimizer, the start factors, target)."""
    A_start = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in A0]
    gn = P.GaussNewton(Xd, [a.clone() for a in A_start], P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
    state = dict(runs=0)

    def step():
        gn.step()
        r = gn.residual()
        if r <= target or not np.isfinite(r):
            for a, a0 in zip(gn.A, A_start):
                a.copy_(a0)
            gn.schedule = P.DampingSchedule()
            state["runs"] += 1
        return r

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    runs_before = state["runs"]
    res = []
    t0 = time.perf_counter()
    for _ in range(steps):
        res.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed / steps * 1e3, res, state["runs"] - runs_before, gn, A_start, target


def trajectory_table(P, torch, Xd, X64, A0, steps):
    """Plain Gauss-Newton steps (damping schedule, eps_cg 1e-3, <= 20 CG iterations) from the
    seeded start with FP32 and with FP64 storage; one JSON line per step with the damping, the
    CG iteration count, sum ||G(n)||, the update norm, the factor norm and the relative residual.
    Stops a run at a non-finite residual."""
    X64d = torch.from_numpy(X64).cuda()
    for name, X, dt in (("f32", Xd, torch.float32), ("f64", X64d, torch.float64)):
        opt = P.GaussNewton(X, [torch.tensor(a, dtype=dt, device="cuda") for a in A0],
                            P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
        for k in range(steps):
            lam = opt.schedule.value
            opt.step()
            st = opt.stats()
            r = opt.residual()
            print(json.dumps(dict(storage=name, step=k, lam=lam, cg_iters=st["cg_iters"],
                                  grad_norm_sum=st["grad_norm_sum"],
                                  update_norm=st["update_norm"],
                                  factor_norm=sum(float(torch.linalg.norm(a.double()))
                                                  for a in opt.A),
                                  residual=r)), flush=True)
            if not np.isfinite(r):
                break
    del X64d


def kernel_source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_1910_12331_amd", "csrc", "mttkrp.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported. The decomposition "
              "runs on a single MI355X; no multi-GPU path is implemented.", file=sys.stderr)
        sys.exit(2)
    if args.cpu_table:
        print(json.dumps(cpu_table()), flush=True)
        return
    import torch

    import paper_1910_12331_amd as P
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    P._lib.load()
    s, R = args.size, args.rank
    dev_name = torch.cuda.get_device_name(0)
    if args.peaks:
        print(json.dumps(measure_peaks(torch)), flush=True)
        return
    if args.profile_bf16:
        from workloads import make_problem
        p4 = make_problem((80, 80, 80, 80), 64, workload=4, problem=0, kind="lognorm", noise=1e-3)
        X4 = torch.tensor(p4.x, dtype=torch.float32, device="cuda")
        A4 = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p4.init]
        warm_gpu(P, X4, A4)
        ws = P.Workspace()
        for Xq in (P.to_bf16(X4), P.to_bf16(X4, split=True)):
            for n in range(4):
                for _ in range(3):
                    P.mttkrp(Xq, A4, n, ws=ws)
        torch.cuda.synchronize()
        print(json.dumps({"profile_bf16": "0.5 s of untimed FP32 cp_mttkrp calls, then 3 x "
                                          "cp_mttkrp per mode, 80^4 R=64, bfloat16 and split"}),
              flush=True)
        return
    if args.profile_batched:
        from workloads import batched_problems
        devs = [(torch.tensor(q.x, dtype=torch.float32, device="cuda"),
                 [torch.tensor(a, dtype=torch.float32, device="cuda") for a in q.init])
                for q in batched_problems(64)]
        bgn = P.BatchedGaussNewton(devs, P.GNConfig(cg_tol=1e-3, cg_maxiter=20), graphs=True,
                                   fused=True)
        for _ in range(args.warmup):
            bgn.step()
        bgn.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bgn.step()
            bgn.synchronize()
        ms = (time.perf_counter() - t0) / max(1, args.steps) * 1e3
        print(json.dumps({"profile_batched": f"{args.warmup} + {args.steps} batch steps of 64 "
                          "problems, batch program replayed from one graph",
                          "ms_per_batch_step": ms}), flush=True)
        del bgn, devs
        shutdown()
        return
    log(f"[bench] device {dev_name}; building {s}^3 rank-{R} planted FP32 tensor")
    X64, A0, Xd = make_inputs(s, R, np.float32)
    stream = torch.cuda.current_stream()

    A = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in A0]
    if args.trajectory:
        trajectory_table(P, torch, Xd, X64, A0, args.trajectory)
        return
    if args.profile_step:
        ms, res, runs, _, _, _ = headline_runs(P, torch, Xd, A0, args.warmup, args.steps)
        print(json.dumps({"profile_step": f"{args.warmup} + {args.steps} GN steps with residuals",
                          "ms_per_step": ms, "runs_completed": runs}), flush=True)
        return
    if args.profile_kernels:
        warm_gpu(P, Xd, A)
        ws = P.Workspace()
        for n in range(3):
            M = torch.empty((s, R), dtype=torch.float32, device="cuda")
            for _ in range(3):
                P.mttkrp(Xd, A, n, out=M, ws=ws)
        Xc = Xd.clone()
        torch.cuda.synchronize()
        print(json.dumps({"profile_kernels": f"0.5 s of untimed cp_mttkrp calls over the modes, then "
                                             f"3 x cp_mttkrp per mode, {s}^3 R={R} FP32; one copy of "
                                             f"{Xd.numel() * 4} bytes"}), flush=True)
        del Xc
        return

    # ---- dominant kernel: single-mode MTTKRP (2 s^3 R flops per call), HIP events, after an
    # untimed warm-up of the GPU
    flops = 2.0 * s ** 3 * R
    warm_gpu(P, Xd, A)
    mt32 = mttkrp_times(P, Xd, A, args.mttkrp_reps, stream)
    mt = {n: v[0] for n, v in mt32.items()}
    mt_tf = {n: flops / t / 1e12 for n, t in mt.items()}
    mean_t = sum(v[3] for v in mt32.values()) / 3        # main kernel alone, mean over modes
    mean_call = sum(v[1] for v in mt32.values()) / 3     # whole cp_mttkrp call
    log(f"[bench] MTTKRP FP32 per-mode median ms per call {[round(t * 1e3, 4) for t in mt.values()]}"
        f", TFLOP/s {[round(v, 1) for v in mt_tf.values()]}; main kernel median ms "
        f"{[round(v[2] * 1e3, 4) for v in mt32.values()]}")
    X64d = torch.from_numpy(X64).cuda()
    A64m = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in A0]
    mt64 = mttkrp_times(P, X64d, A64m, args.mttkrp_reps, stream)
    log(f"[bench] MTTKRP FP64 per-mode median ms {[round(v[0] * 1e3, 4) for v in mt64.values()]}")

    # all-mode MTTKRP as a GN step runs it (modes 0 and 1 from one dimension-tree pass)
    def all_mode_time(Xt, At):
        out_ = [torch.empty((s, R), dtype=At[0].dtype, device="cuda") for _ in range(3)]
        ws_ = P.Workspace()
        for _ in range(3):
            P.mttkrp_all(Xt, At, out=out_, ws=ws_)
        return float(np.median(event_samples(lambda: P.mttkrp_all(Xt, At, out=out_, ws=ws_),
                                             args.mttkrp_reps, stream)))
    tall32 = all_mode_time(Xd, A)
    tall64 = all_mode_time(X64d, A64m)
    del X64d, A64m
    log(f"[bench] all-mode MTTKRP median ms: FP32 {tall32 * 1e3:.4f}, FP64 {tall64 * 1e3:.4f}")

    # launch floor: an event-timed one-element fill kernel
    one = torch.zeros(1, device="cuda")
    floor = event_time(lambda: one.fill_(1.0), 200, stream)

    # ---- ALS sweep (comparison method)
    Aals = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in A0]
    ws_als = P.Workspace()
    for _ in range(2):
        P.als_sweep(Xd, Aals, 0.0, ws=ws_als)
    als_t = event_time(lambda: P.als_sweep(Xd, Aals, 0.0, ws=ws_als), 5, stream)

    # ---- GN step with Armijo step control (Section 5): f at the start point and at every trial
    # point is part of the step, so it also yields the residual of the new point
    Aarm = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in A0]
    garm = P.GaussNewton(Xd, Aarm, P.GNConfig(cg_tol=1e-3, cg_maxiter=20, line_search=P.Armijo()))
    for _ in range(2):
        garm.step()
    arm_t = event_time(garm.step, 5, stream)
    arm_st = garm.stats()
    del garm, Aarm
    log(f"[bench] GN step with Armijo control: {arm_t * 1e3:.3f} ms "
        f"(last step: {arm_st['ls_trials']} trial(s), alpha {arm_st['ls_alpha']})")

    high_rank = high_rank_leg(P, torch, stream)
    gn_vs_als = gn_vs_als_leg(P, torch, stream)
    objective = objective_leg(P, torch, Xd, A0, stream)

    # ---- GN steps: warmup, then K timed steps (headline_runs)
    ms_step, res_timed, runs_in_window, gn, A_start, target = headline_runs(
        P, torch, Xd, A0, args.warmup, args.steps)
    r_now = res_timed[-1]
    log(f"[bench] GN step + residual: {ms_step:.3f} ms; residuals of the timed steps "
        + " ".join(f"{r:.2e}" for r in res_timed))

    # CG iterations of the timed steps: the kernels are deterministic, so an untimed replay of
    # the same runs reads them step by step (its residuals must equal the timed ones bitwise).
    gr = P.GaussNewton(Xd, [a.clone() for a in A_start], P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
    iters, replay_res = [], []
    for k in range(args.warmup + args.steps):
        gr.step()
        r = gr.residual()
        if k >= args.warmup:
            iters.append(gr.stats()["cg_iters"])
            replay_res.append(r)
        if r <= target or not np.isfinite(r):
            for a, a0 in zip(gr.A, A_start):
                a.copy_(a0)
            gr.schedule = P.DampingSchedule()
    del gr
    r0_ = P.residual(Xd, A_start, ws=gn.ws).cpu()
    r_start = float(r0_[0] / r0_[1])
    finite = bool(np.all(np.isfinite(res_timed)))
    valid = finite and replay_res == res_timed and max(res_timed) < 10.0 * r_start
    if not valid:
        log("[bench] WARNING: a timed step left the converging runs")
    trajectory = dict(start_residual=r_start, target=target, residuals=res_timed,
                      runs_completed_in_timed_window=runs_in_window,
                      replay_equals_timed_run=replay_res == res_timed, valid=valid,
                      note="relative residual after each timed step; a run restarts from the "
                           "seeded start once its residual is <= target. valid: all finite, "
                           "bitwise equal to an untimed replay, none above 10x the start")

    # ---- GN step with exactly 20 CG iterations (eps_cg = 0), FP32 and FP64
    A20 = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in A0]
    ws20 = P.Workspace()
    sb = P.stats_buffer(Xd.device)
    for _ in range(2):
        P.gn_step(Xd, A20, 1e-4, 0.0, 20, stats=sb, ws=ws20)
    t20 = event_time(lambda: P.gn_step(Xd, A20, 1e-4, 0.0, 20, stats=sb, ws=ws20), 5, stream)
    s20 = P.read_stats(sb)
    if s20["status"] != 0 or s20["cg_iters"] != 20:
        log(f"[bench] WARNING: the 20-iteration step timing ended with status {s20['status']}, "
            f"{s20['cg_iters']} CG iterations")
    t0cg = event_time(lambda: P.gn_step(Xd, A20, 1e-4, 0.0, 0, stats=sb, ws=ws20), 5, stream)
    # the same with the preconditioner applied by Cholesky triangular solves (Section 3.3)
    P.gn_step(Xd, A20, 1e-4, 0.0, 20, stats=sb, ws=ws20, preconditioner="cholesky")
    t20c = event_time(lambda: P.gn_step(Xd, A20, 1e-4, 0.0, 20, stats=sb, ws=ws20,
                                        preconditioner="cholesky"), 3, stream)
    log(f"[bench] GN step with 20 CG iterations: {t20 * 1e3:.3f} ms with the explicit inverse, "
        f"{t20c * 1e3:.3f} ms with Cholesky triangular solves")
    resid = torch.empty(2, dtype=torch.float64, device="cuda")
    res_t = event_time(lambda: P.residual(Xd, gn.A, out=resid, ws=gn.ws), 10, stream)

    # ---- time to relative residual 1e-8, FP64 storage (the FP32 rounding floor is ~3e-8)
    ttt = None
    if not args.no_time_to_target:
        X64d = torch.from_numpy(X64).cuda()
        A20 = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in A0]
        for _ in range(2):
            P.gn_step(X64d, A20, 1e-4, 0.0, 20, stats=sb, ws=ws20)
        t20_64 = event_time(lambda: P.gn_step(X64d, A20, 1e-4, 0.0, 20, stats=sb, ws=ws20), 3, stream)
        del A20
        A64 = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in A0]
        # one untimed step of each driver first, so that the timed runs reuse cached workspace
        # allocations instead of allocating inside the timed region
        X32d = X64d.float()
        P.gn_to_target(X64d, [a.clone() for a in A64], 1e-8, max_steps=1)
        P.gn_mixed_to_target(X32d, X64d, [torch.tensor(a, dtype=torch.float32, device="cuda")
                                          for a in A0], 1.0, 1.0, max_steps=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g64, h64 = P.gn_to_target(X64d, A64, 1e-8, P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
        fp64_s = time.perf_counter() - t0
        # mixed: FP32 storage until its residual is <= 1e-6 (or stalls near the FP32 rounding
        # floor), then FP64 from the same factors and damping schedule
        A32 = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in A0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hmx = P.gn_mixed_to_target(X32d, X64d, A32, 1e-8, 1e-6,
                                      P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
        mixed_s = time.perf_counter() - t0
        n32 = sum(1 for p_, _ in hmx if p_ == "torch.float32")
        # FP64 with Armijo control (Section 5): f at the accepted point gives the residual
        Aar = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in A0]
        arm_cfg = P.GNConfig(cg_tol=1e-3, cg_maxiter=20, line_search=P.Armijo())
        P.gn_to_target(X64d, [a.clone() for a in Aar], 1e-8, arm_cfg, max_steps=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, har = P.gn_to_target(X64d, Aar, 1e-8, P.GNConfig(cg_tol=1e-3, cg_maxiter=20,
                                                           line_search=P.Armijo()))
        armijo_s = time.perf_counter() - t0
        del Aar
        log(f"[bench] time to 1e-8 with Armijo control (FP64): {armijo_s:.3f} s in {len(har)} "
            f"steps (r={har[-1]:.2e})")
        # precision ladder with the bfloat16 rungs: bfloat16 -> split bfloat16 -> FP32 -> FP64
        # storage of the same tensor (conversions made before the timed region; one untimed run
        # first so that the timed one reuses cached workspace allocations)
        Xb, Xs = P.to_bf16(X32d), P.to_bf16(X32d, split=True)
        lad_cfg = P.GNConfig(cg_tol=1e-3, cg_maxiter=20)
        P.gn_ladder_to_target([Xb, Xs, X32d, X64d], [torch.tensor(a, dtype=torch.float32,
                                                                 device="cuda") for a in A0],
                              1e-8, lad_cfg)
        Alad = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in A0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hlad = P.gn_ladder_to_target([Xb, Xs, X32d, X64d], Alad, 1e-8, lad_cfg)
        ladder_s = time.perf_counter() - t0
        del Xb, Xs, Alad
        lad_rungs = {}
        for name, _, acc in hlad:
            lad_rungs[name] = lad_rungs.get(name, 0) + 1
        log(f"[bench] time to 1e-8 with the bfloat16 ladder: {ladder_s:.3f} s, steps per rung "
            f"{lad_rungs} (r={hlad[-1][1]:.2e})")
        ttt = dict(fp64_seconds=fp64_s, fp64_steps=len(h64), fp64_residual=h64[-1],
                   fp64_armijo_seconds=armijo_s, fp64_armijo_steps=len(har),
                   fp64_armijo_residual=har[-1],
                   mixed_seconds=mixed_s, mixed_steps_fp32=n32, mixed_steps_fp64=len(hmx) - n32,
                   mixed_residual=hmx[-1][1], speedup=fp64_s / mixed_s,
                   ladder_bf16_seconds=ladder_s, ladder_bf16_steps_per_rung=lad_rungs,
                   ladder_bf16_residual=hlad[-1][1],
                   ladder_note="bfloat16 -> split bfloat16 -> FP32 -> FP64 storage "
                               "(gn_ladder_to_target: a rung is left when a step raises the "
                               "residual or the residual nears the rung's floor)",
                   fp64_gn_step_20cg_ms=t20_64 * 1e3)
        log(f"[bench] time to 1e-8: FP64 {fp64_s:.3f} s in {len(h64)} steps (r={h64[-1]:.2e}); "
            f"mixed {mixed_s:.3f} s in {n32} FP32 + {len(hmx) - n32} FP64 steps (r={hmx[-1][1]:.2e})")
        del X32d, A32
        del X64d, A64, g64

    # ---- workload 5: 64 independent FP32 problems (modes U{60..200}, rank U{8,16,32,64}),
    # one GN step each per batched step, spread over HIP streams
    batched = None
    if not args.no_batched:
        from workloads import batched_problems
        probs = batched_problems(64)
        devs = [(torch.tensor(p_.x, dtype=torch.float32, device="cuda"),
                 [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p_.init]) for p_ in probs]
        res = {}
        # sweep-based autotuner over (streams, graph replay) for this batch's shape bucket; its
        # pick is then timed like the fixed configurations below
        tune = P.autotune_batched(devs, P.GNConfig(cg_tol=1e-3, cg_maxiter=20),
                                  stream_counts=(1, 2, 4, 8, 16), steps=3)
        hz = P.device_clock_hz()
        bs = args.batched_streams
        configs = [(1, False, False, False, None), (bs, False, False, False, None),
                   (bs, True, False, False, None), (bs, False, True, False, None),
                   (bs, True, True, False, None), (1, False, True, True, None),
                   (1, True, True, True, None)]
        tk = (tune.n_streams, tune.graphs, tune.batch_cg, tune.fused, tune.tiles)
        if tk not in configs:
            configs.append(tk)

        def cname(ns, g, b, f, t=None):
            if f:
                name = "program" + ("_graph" if g else "")
            else:
                name = f"streams_{ns}" + ("_graphs" if g else "") + ("_batchcg" if b else "")
            return name if t is None else name + "_tiles_{}_{}_{}".format(*t)
        for ns, graphs, bcg, fus, tls in configs:
            cur = [(X_, [a.clone() for a in A_]) for X_, A_ in devs]
            torch.cuda.synchronize()
            bgn = P.BatchedGaussNewton(cur, P.GNConfig(cg_tol=1e-3, cg_maxiter=20), n_streams=ns,
                                       graphs=graphs, batch_cg=bcg, fused=fus, tiles=tls)
            for _ in range(2):
                bgn.step()
            bgn.synchronize()
            # per-problem step latency from device timestamps (the device clock written by a
            # one-thread kernel on the problem's stream right before and after its step; not
            # part of the single graph of a batched-CG step or of a batch program)
            stamped = not (graphs and bcg) and not fus
            stamps = torch.zeros((5, 2 * len(devs)), dtype=torch.int64, device="cuda")
            t0 = time.perf_counter()
            for k in range(5):
                bgn.step(stamps=stamps[k] if stamped else None)
                bgn.synchronize()
            el = time.perf_counter() - t0
            rec = dict(problem_steps_per_s=64 * 5 / el)
            if stamped:
                ticks = stamps.view(5, len(devs), 2).cpu().numpy()
                per = ((ticks[:, :, 1] - ticks[:, :, 0]) / hz * 1e3).ravel()
                rec.update(step_ms_p50=float(np.percentile(per, 50)),
                           step_ms_p99=float(np.percentile(per, 99)))
            res[cname(ns, graphs, bcg, fus, tls)] = rec
            del bgn, cur
        kt = cname(*tk)
        res["autotuned"] = dict(choice=kt, problem_steps_per_s=res[kt]["problem_steps_per_s"],
                                sweep_problem_steps_per_s={
                                    cname(*k): v for k, v in tune.table.items()},
                                tile_sweep_problem_steps_per_s={
                                    "tiles_{}_{}_{}".format(*t): v
                                    for t, v in tune.tile_table.items()},
                                note="sweep: 3 steps per configuration without per-problem "
                                     "events, then MTTKRP tile shapes (min items per wavefront, "
                                     "workgroups per CU, FP32 row tile in 16-row blocks; 0 = "
                                     "default) on the best configuration; "
                                     "problem_steps_per_s: the timed loop of the fixed "
                                     "configurations")
        log(f"[bench] batched autotuner picks {kt}: {res[kt]['problem_steps_per_s']:.0f} "
            f"problem-steps/s in the same timed loop")
        batched = dict(workload="64 FP32 problems, modes U{60..200}, rank U{8,16,32,64}, noise 1e-4",
                       note="_graphs: each problem's GN step and damping update replayed from a "
                            "captured HIP graph; _batchcg: CG of all problems in shared launches "
                            "(with _graphs: the whole batch step as one graph); program: the batch "
                            "program (every part of the step in shared launches, one stream; "
                            "_graph: replayed from one captured graph); "
                            "step_ms_p50/p99: per-problem step latency from "
                            f"device timestamps ({hz} Hz clock), 5 batch steps", **res)
        kb, kg = cname(bs, False, False, False), cname(bs, True, False, False)
        kc, kcg = cname(bs, False, True, False), cname(bs, True, True, False)
        kp, kpg = cname(1, False, True, True), cname(1, True, True, True)
        log(f"[bench] batched workload: batch program {res[kpg]['problem_steps_per_s']:.0f} "
            f"problem-steps/s from one graph, {res[kp]['problem_steps_per_s']:.0f} eagerly; "
            f"{res[kcg]['problem_steps_per_s']:.0f} on "
            f"{bs} streams with batched CG and one graph per batch step, "
            f"{res[kc]['problem_steps_per_s']:.0f} with batched CG eagerly, "
            f"{res[kg]['problem_steps_per_s']:.0f} with per-problem graphs, "
            f"{res[kb]['problem_steps_per_s']:.0f} eager, "
            f"{res['streams_1']['problem_steps_per_s']:.0f} on one stream; per-problem step "
            f"p50 {res[kc]['step_ms_p50']:.3f} ms, p99 {res[kc]['step_ms_p99']:.3f} ms (batched CG)")
        del devs

    # ---- order-4 workload in bfloat16 / split bfloat16 / FP32 / FP64 storage
    order4 = None if args.no_order4 else order4_leg(P, torch, args.mttkrp_reps, stream)

    # ---- CPU baseline: the oracle on host cores, bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(X64, A0, iters, args.cpu_seconds)
        log(f"[bench] CPU oracle: {cpu['value']:.4f} GN steps/s on {cpu['cores']} threads "
            f"({cpu['sample']})")

    traffic = None
    if MTTKRP_TRAFFIC is not None and MTTKRP_TRAFFIC["source_sha256"] == kernel_source_hash():
        traffic = MTTKRP_TRAFFIC["bytes_per_launch"]
    out = {
        "metric": METRIC,
        "value": 1e3 / ms_step,
        "unit": "GN steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dense {s}x{s}x{s} FP32 tensor, exact rank-{R} CP with N(0,1) "
                               f"factors; GN-CG rank {R}, eps_cg 1e-3, <=20 CG its, varying lambda "
                               f"1e-4..1e-10 (mu 2); step = GN step + direct residual at the new "
                               f"point, the step kept only if f decreases",
                   "dims": [s, s, s], "rank": R, "device": dev_name},
        "roofline": {"bound": "mfma", "achieved": flops / mean_t / 1e12,
                     "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / mean_t / 1e12 / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": traffic,
                     "kernel": "k_mttkrp, the main kernel of cp_mttkrp, FP32 single mode: HIP "
                               "events recorded on its stream around its launch (mean over modes "
                               "and calls)",
                     "per_call": {"achieved": flops / mean_call / 1e12,
                                  "frac": flops / mean_call / 1e12 / PEAK_FP32_MFMA_TFLOPS,
                                  "note": "whole cp_mttkrp call: factor preparation, main "
                                          "kernel, partial-tile reduction"}},
        "mttkrp_fp32": {f"mode{n}": {"median_ms": v[0] * 1e3, "mean_ms": v[1] * 1e3,
                                     "tflops_median": flops / v[0] / 1e12,
                                     "kernel_median_ms": v[2] * 1e3, "kernel_mean_ms": v[3] * 1e3}
                        for n, v in mt32.items()},
        "mttkrp_fp64": {f"mode{n}": {"median_ms": v[0] * 1e3, "mean_ms": v[1] * 1e3,
                                     "tflops_median": flops / v[0] / 1e12,
                                     "frac_fp64_peak": flops / v[0] / 1e12 / PEAK_FP64_MFMA_TFLOPS,
                                     "kernel_median_ms": v[2] * 1e3,
                                     "kernel_frac_fp64_peak":
                                         flops / v[2] / 1e12 / PEAK_FP64_MFMA_TFLOPS}
                        for n, v in mt64.items()},
        "mttkrp_all_modes": {
            "fp32_median_ms": tall32 * 1e3, "fp64_median_ms": tall64 * 1e3,
            "note": "one cp_mttkrp_all call; tree_tflops counts the dimension tree's 4 s^3 R flops "
                    "(two bottleneck contractions), per_mode_equivalent_tflops three separate "
                    "MTTKRPs (6 s^3 R)",
            "fp32_tree_tflops": 4.0 * s ** 3 * R / tall32 / 1e12,
            "fp32_per_mode_equivalent_tflops": 6.0 * s ** 3 * R / tall32 / 1e12,
            "fp64_tree_tflops": 4.0 * s ** 3 * R / tall64 / 1e12,
            "fp64_per_mode_equivalent_tflops": 6.0 * s ** 3 * R / tall64 / 1e12},
        "gn_step_20cg_ms": t20 * 1e3,
        "gn_steps_per_s_20cg": 1.0 / t20,
        "cg_iteration_ms": (t20 - t0cg) / 20 * 1e3,
        "gn_step_20cg_cholesky_precond_ms": t20c * 1e3,
        "launch_floor_ms": floor * 1e3,
        "residual_ms": res_t * 1e3,
        "als_sweep_ms": als_t * 1e3,
        "gn_armijo_step_ms": arm_t * 1e3,
        "gn_armijo_last": {"trials": arm_st["ls_trials"], "alpha": arm_st["ls_alpha"],
                           "note": "GN step with Armijo control (c 1e-4, shrink 0.5, <=10 trials), "
                                   "f at the start and trial points included"},
        "high_rank_150_r200_fp64": high_rank,
        "gn_vs_als_300_r50_congruent_fp64": gn_vs_als,
        "objective_fwd_bwd_400_r100_fp32": objective,
        "cg_iters_mean": float(np.mean(iters)),
        "cg_iters": iters,
        "residual_after": r_now,
        "trajectory": trajectory,
        "time_to_1e-8": ttt,
        "batched": batched,
        "order4_bf16": order4,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def shutdown():
    """Release device memory and finish GPU work before interpreter exit, so that nothing is left
    for exit-time destructors (see the note on profiler teardown in the design notes)."""
    import torch
    if torch.cuda.is_available():
        import paper_1910_12331_amd as P
        P.api.release_default_workspace()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
    shutdown()
