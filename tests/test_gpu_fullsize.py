"""The 400^3 rank-100 FP32 workload that bench.py times, checked at full size: one Gauss-Newton
step against the oracle's step, the direct residual against a closed form that needs no pass
over a reconstructed tensor, and the runs the benchmark times reaching their FP32 floor target.

The oracle runs in FP64 on the FP32-rounded inputs. The GPU forms the MTTKRPs in FP32 and all
of CG in FP64, so its step differs from the oracle's by the CG response to the FP32 rounding of
M. That bound is measured on the oracle itself: its update under a perturbation of G of the
FP32 MTTKRP's error bound (2e-5 of ||M(n)||, the bound the MTTKRP tests hold the kernel to),
times 10, plus the FP32 rounding of the returned factors.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1910_12331_amd as P  # noqa: E402

U32 = 2.0 ** -24
MTTKRP_FP32_BOUND = 2e-5


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P._lib.load()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def c3():
    """The benchmark's inputs: planted N(0,1) factors B, X = [[B]] built in FP64 and stored in
    FP32, and the N(0,1) start A0 (rounded to FP32 as the device holds it)."""
    p = make_problem((400, 400, 400), 100, workload=3)
    x32 = p.x.astype(np.float32)
    return dict(B=p.planted, X64=p.x, X32=x32,
                A0=[a.astype(np.float32).astype(np.float64) for a in p.init])


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(arrs, dt=torch.float32):
    return [torch.tensor(a, dtype=dt, device="cuda") for a in arrs]


def host(ts):
    return [t.double().cpu().numpy() for t in ts]


def test_fp32_gn_step_full_size_matches_oracle(c3):
    """One Gauss-Newton step (eps_cg = 1e-3, at most 20 CG iterations, lambda = 1e-4) at
    400^3, R = 100 in FP32 storage, from the benchmark's start, against the oracle's step."""
    lam, eps, maxiter = 1e-4, 1e-3, 20
    Xh = c3["X32"].astype(np.float64)
    Ah = c3["A0"]
    S = O.grams(Ah)
    Gam = O.gamma_set(S)
    M = [O.mttkrp(Xh, Ah, n) for n in range(3)]
    G = [Ah[n] @ Gam[n][n] - M[n] for n in range(3)]
    ref = O.pcg(G, Ah, lam, eps, maxiter, Gam)
    # the CG stop test must not be borderline: every iteration's residual sum at least 1% away
    # from the threshold, so that the FP32 gradient cannot change the iteration count
    for h in ref.history:
        assert abs(h["res_norm_sum"] / (eps * ref.grad_norm_sum) - 1.0) > 0.01
    # the oracle's response to a perturbation of G at the FP32 MTTKRP bound
    rng = np.random.default_rng(5)
    Gp = []
    for g, m in zip(G, M):
        e = rng.standard_normal(g.shape)
        Gp.append(g + MTTKRP_FP32_BOUND * np.linalg.norm(m) * e / np.linalg.norm(e))
    refp = O.pcg(Gp, Ah, lam, eps, maxiter, Gam)
    assert refp.iters == ref.iters
    v_ref = O.flatten_factors(ref.V)
    spread = rel(O.flatten_factors(refp.V), v_ref)
    new_ref = [a + v for a, v in zip(Ah, ref.V)]
    a_norm = np.linalg.norm(O.flatten_factors(new_ref))
    tol = 10.0 * spread + 4.0 * U32 * a_norm / np.linalg.norm(v_ref)

    Xd = torch.from_numpy(c3["X32"]).cuda()
    Ad = dev(Ah)
    st = P.read_stats(P.gn_step(Xd, Ad, lam, eps, maxiter))
    del Xd
    assert st["status"] == 0
    assert st["cg_iters"] == ref.iters
    v_gpu = O.flatten_factors([a - b for a, b in zip(host(Ad), Ah)])
    err = rel(v_gpu, v_ref)
    assert err < tol, (err, tol, spread)
    assert abs(st["grad_norm_sum"] - ref.grad_norm_sum) <= 10 * MTTKRP_FP32_BOUND * ref.grad_norm_sum
    un = float(np.linalg.norm(v_ref))
    assert abs(st["update_norm"] - un) <= tol * un


def closed_form_residual(B, X64, X32, A):
    """||X32 - [[A]]||_F and ||X32||_F with X32 = [[B]] + d (d the FP32 rounding of the planted
    tensor, exact in FP64), without forming [[A]]:
      ||[[B]] - [[A]]||^2 = sum(*_m B(m)^T B(m)) - 2 sum(*_m B(m)^T A(m)) + sum(*_m A(m)^T A(m))
    (inner products of CP tensors are Hadamard products of the factor cross-Grams), and
      ||X32 - [[A]]||^2 = ||[[B]] - [[A]]||^2 + 2 <d, X64> - 2 <d, [[A]]> + ||d||^2,
    with <d, [[A]]> = <MTTKRP(d, A, 0), A(0)> (Section 2.2's contraction)."""
    def had(L, Rm):
        out = np.ones((L[0].shape[1], Rm[0].shape[1]))
        for a, b in zip(L, Rm):
            out = out * (a.T @ b)
        return float(np.sum(out))
    d = X32.astype(np.float64) - X64
    dx = float(np.sum(d * X64))
    dd = float(np.sum(d * d))
    da = float(np.sum(O.mttkrp(d, A, 0) * A[0]))
    bb = had(B, B)
    num2 = bb - 2.0 * had(B, A) + had(A, A) + 2.0 * dx - 2.0 * da + dd
    return math.sqrt(num2), math.sqrt(bb + 2.0 * dx + dd)


@pytest.mark.parametrize("where", ["start", "near_solution"])
def test_fp32_residual_full_size_closed_form(c3, where):
    """The direct residual at 400^3, R = 100 in FP32 against the closed form, at the benchmark's
    start (relative residual about 1) and at the planted factors with a 1e-3 relative
    perturbation. The kernel rebuilds [[A]] in FP32 (products of R + N terms per entry) and sums
    the squared differences in FP32 within a tile and in FP64 across tiles: the bound is
    1e-5 of the residual plus 2e-6 of ||X|| for the reconstruction rounding."""
    if where == "start":
        A = c3["A0"]
    else:
        rng = np.random.default_rng(17)
        A = [(b * (1 + 1e-3 * rng.standard_normal(b.shape))).astype(np.float32).astype(np.float64)
             for b in c3["B"]]
    num_ref, xn_ref = closed_form_residual(c3["B"], c3["X64"], c3["X32"], A)
    Xd = torch.from_numpy(c3["X32"]).cuda()
    out = P.residual(Xd, dev(A)).cpu().numpy()
    del Xd
    assert abs(out[1] - xn_ref) <= 1e-6 * xn_ref
    assert abs(out[0] - num_ref) <= 1e-5 * num_ref + 2e-6 * xn_ref, (out[0], num_ref)


def test_fp32_run_reaches_floor_target(c3):
    """The benchmark's runs at full size: plain Gauss-Newton steps from the seeded start, with
    the damping schedule, reach a relative residual <= 1e-6 (the FP32 floor target at which the
    benchmark starts a new run and the mixed-precision driver leaves FP32 storage) within 30
    steps; every residual on the way is finite and below 10x the start."""
    Xd = torch.from_numpy(c3["X32"]).cuda()
    opt = P.GaussNewton(Xd, dev(c3["A0"]), P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
    r0 = P.residual(Xd, opt.A).cpu().numpy()
    start = r0[0] / r0[1]
    hist = []
    while opt.steps < 30:
        opt.step()
        assert opt.stats()["status"] == 0
        hist.append(opt.residual())
        assert math.isfinite(hist[-1]) and hist[-1] < 10 * start, hist
        if hist[-1] <= 1e-6:
            break
    del Xd
    assert hist[-1] <= 1e-6, hist


def planted_small():
    """A planted rank-5 tensor with 1e-2 noise and an N(0,1) start where, under the default
    damping schedule, the first four full steps decrease f and the next ones overshoot (checked
    on the oracle below, with every trial at least 10% of f away from its threshold)."""
    return make_problem((20, 18, 22), 5, workload=0, problem=7, noise=1e-2)


def test_carried_objective_is_bitwise_the_evaluated_one():
    """CP_LS_F0_GIVEN: a search that takes f(A) from the previous call's stats gives the same
    factors and stats bit for bit as one that evaluates f(A) again (it is the same kernel on the
    same factors), through accepted and rejected steps, FP64 and FP32."""
    p = planted_small()
    for dt in (torch.float64, torch.float32):
        Xd = dev([p.x], dt)[0]
        runs = []
        for carry in (False, True):
            cfg = P.GNConfig(cg_tol=1e-3, cg_maxiter=20,
                             line_search=P.Armijo(max_trials=1, carry_objective=carry))
            opt = P.GaussNewton(Xd, dev(p.init, dt), cfg)
            out = []
            for _ in range(6):
                opt.step()
                s = opt.stats()
                out.append((s["ls_f0"], s["ls_f"], s["ls_accepted"], s["ls_x_norm"],
                            s["cg_iters"], s["update_norm"]))
            runs.append((out, [a.clone() for a in opt.A]))
        assert runs[0][0] == runs[1][0]
        assert {r[2] for r in runs[0][0]} == {0, 1}, "need both accepted and rejected steps"
        for a, b in zip(runs[0][1], runs[1][1]):
            assert torch.equal(a, b)


def test_carried_objective_matches_oracle_f0():
    """The oracle's Armijo step with one trial, given f0 from its previous step, decides like
    the GPU's search with the carried objective over a run with acceptances and rejections
    (FP64, default damping schedule)."""
    p = planted_small()
    Xd = dev([p.x], torch.float64)[0]
    opt = P.GaussNewton(Xd, dev(p.init, torch.float64),
                        P.GNConfig(cg_tol=1e-3, cg_maxiter=20, line_search=P.Acceptance()))
    sched = O.LambdaSchedule()
    Ah, f0 = p.init, None
    decisions = []
    for _ in range(6):
        ref = O.gn_step_armijo(p.x, Ah, sched.value, 1e-3, 20, max_trials=1, f0=f0)
        if ref.trials:
            ft = O.objective(p.x, [a + v for a, v in zip(Ah, ref.V)])
            assert abs(ft - (ref.f0 + 1e-4 * ref.gv)) > 0.1 * ref.f0
        opt.step()
        s = opt.stats()
        assert s["ls_accepted"] == int(ref.accepted)
        assert abs(s["ls_f"] - ref.f) <= 1e-12 * ref.f0
        decisions.append(ref.accepted)
        Ah, f0 = ref.A, ref.f
        sched.advance()
        assert rel(O.flatten_factors(host(opt.A)), O.flatten_factors(Ah)) < 1e-12
    assert decisions == [True, True, True, True, False, False]
