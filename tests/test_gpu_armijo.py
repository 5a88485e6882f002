"""GPU parity of the Gauss-Newton step with Armijo step-size control (Section 5) through the C ABI
(cp_gn_step_armijo), against the FP64 oracle's gn_step_armijo on the same seeded inputs. The
accepted step size and the number of objective evaluations are integers decided by floating
point: every case first checks on the oracle that each trial's objective lies well away from its
Armijo threshold, so that both sides must take the same decisions."""
import numpy as np
import pytest

import oracle as O
from workloads import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1910_12331_amd as P  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P._lib.load()
    yield
    torch.cuda.synchronize()


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_start(dims, rank, scale, seed):
    """A Gaussian tensor and a Gaussian start at a small scale, where the full Gauss-Newton step
    overshoots and the search has to shrink the step."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(dims)
    return X, [scale * rng.standard_normal((s, rank)) for s in dims]


def dev(arrs, dt):
    return [torch.tensor(a, dtype=dt, device="cuda") for a in arrs]


def host(ts):
    return [t.double().cpu().numpy() for t in ts]


def trial_margins(X, A, ref, c, shrink):
    """(f(A + alpha V) - threshold) / f(A) for every trial the oracle made."""
    out, alpha = [], 1.0
    for _ in range(ref.trials):
        ft = O.objective(X, [a + alpha * v for a, v in zip(A, ref.V)])
        out.append((ft - (ref.f0 + c * alpha * ref.gv)) / ref.f0)
        alpha *= shrink
    return out


def armijo_compare(X, A, dt, lam, cg_tol, maxiter, c=1e-4, shrink=0.5, max_trials=10, tol=None,
                   margin=1e-3, damping="identity", precond="inverse"):
    if dt == torch.float32:   # the oracle sees the FP32-rounded inputs
        X = X.astype(np.float32).astype(np.float64)
        A = [a.astype(np.float32).astype(np.float64) for a in A]
    ref = O.gn_step_armijo(X, A, lam, cg_tol, maxiter, damping, c=c, shrink=shrink,
                           max_trials=max_trials, precond=precond)
    if tol is None:
        if dt == torch.float64:
            # 10x the oracle's own spread when its input factors move by 1e-15 relative
            rng = np.random.default_rng(1)
            A2 = [a * (1 + 1e-15 * rng.standard_normal(a.shape)) for a in A]
            ref2 = O.gn_step_armijo(X, A2, lam, cg_tol, maxiter, damping, c=c, shrink=shrink,
                                    max_trials=max_trials, precond=precond)
            sv = rel(O.flatten_factors([b - a for a, b in zip(A2, ref2.A)]),
                     O.flatten_factors([b - a for a, b in zip(A, ref.A)])) if ref.accepted else 0.0
            sg = abs(ref2.gv - ref.gv) / abs(ref.gv) if ref.gv != 0.0 else 0.0
            spread = max(sv, sg, abs(ref2.f - ref.f) / ref.f0)
            tol = max(1e-12, 10 * spread)
        else:
            tol = 2e-3
    assert all(abs(m) > margin for m in trial_margins(X, A, ref, c, shrink))
    Xd, Ad = dev([X], dt)[0], dev(A, dt)
    st, ls = P.gn_step_armijo(Xd, Ad, lam, cg_tol, maxiter, c, shrink, max_trials,
                              damping=damping, preconditioner=precond)
    st, ls = P.read_stats(st), P.read_armijo_stats(ls)
    assert st["status"] == 0
    assert ls["accepted"] == int(ref.accepted) and ls["trials"] == ref.trials
    assert ls["alpha"] == ref.alpha
    assert abs(ls["f0"] - ref.f0) <= 1e-12 * ref.f0 if dt == torch.float64 else \
        abs(ls["f0"] - ref.f0) <= 1e-6 * ref.f0
    assert abs(ls["gv"] - ref.gv) <= tol * abs(ref.gv)
    assert abs(ls["f"] - ref.f) <= tol * ref.f0
    # the FP32 residual kernel sums squares in FP32 within a tile, in FP64 across tiles
    xtol = 1e-12 if dt == torch.float64 else 1e-6
    assert abs(ls["x_norm"] - np.linalg.norm(X)) <= xtol * np.linalg.norm(X)
    got = host(Ad)
    step = [g - a for g, a in zip(got, A)]
    want = [o - a for o, a in zip(ref.A, A)]
    if ref.accepted:
        assert rel(np.concatenate([s.ravel() for s in step]),
                   np.concatenate([w.ravel() for w in want])) < tol
        un = ref.alpha * np.sqrt(sum(float(np.sum(v * v)) for v in ref.V))
        assert abs(st["update_norm"] - un) <= tol * un
    else:
        for g, a in zip(got, A):
            assert np.array_equal(g, a)
        assert st["update_norm"] == 0.0
    return ref, ls


@pytest.mark.parametrize("dims,rank,scale,seed,alpha", [
    ((6, 5, 7), 4, 0.3, 3, 0.125),
    ((37, 29, 45), 12, 0.3, 2, 0.5),          # several 16-row tiles, ragged tails
    ((9, 11, 7, 13), 5, 0.3, 2, 0.25),         # order 4
    ((30, 26, 35), 70, 0.3, 1, 0.5),           # R = 70 > every mode size
    ((33, 17, 21), 20, 0.2, 4, 0.25),
])
def test_armijo_step_fp64(dims, rank, scale, seed, alpha):
    X, A = small_start(dims, rank, scale, seed)
    ref, ls = armijo_compare(X, A, torch.float64, 1e-6, 1e-6, 50)
    assert ref.alpha == alpha and ls["f"] < ls["f0"]


@pytest.mark.parametrize("dims,rank,scale,seed,alpha", [((30, 26, 35), 150, 0.3, 1, 0.5),
                                                        ((40, 30, 36), 200, 0.2, 3, 0.25)])
def test_armijo_step_high_rank_fp64(dims, rank, scale, seed, alpha):
    """Above R = 128 (13 register blocks of 16 columns at R = 200); the oracle's own spread under
    a 1e-15 input perturbation is about 3e-13 here."""
    X, A = small_start(dims, rank, scale, seed)
    ref, _ = armijo_compare(X, A, torch.float64, 1e-6, 1e-3, 50)
    assert ref.alpha == alpha


@pytest.mark.parametrize("dims,rank,scale,seed", [((37, 29, 45), 12, 0.3, 2),
                                                  ((9, 11, 7, 13), 5, 0.3, 2),
                                                  ((30, 26, 35), 70, 0.1, 1)])
def test_armijo_step_fp32(dims, rank, scale, seed):
    # a fixed number of CG iterations (eps_cg = 0), so that both sides stop at the same one
    X, A = small_start(dims, rank, scale, seed)
    ref, ls = armijo_compare(X, A, torch.float32, 1e-6, 0.0, 12)
    assert ref.accepted and ref.alpha < 1.0


@pytest.mark.parametrize("damping,precond", [("diagonal", "inverse"), ("identity", "cholesky"),
                                             ("diagonal", "cholesky")])
def test_armijo_with_damping_and_preconditioner_forms(damping, precond):
    """The search composes with diagonal damping and the triangular-solve preconditioner."""
    X, A = small_start((37, 29, 45), 12, 0.3, 2)
    ref, ls = armijo_compare(X, A, torch.float64, 1e-6, 1e-6, 50, damping=damping,
                             precond=precond)
    assert ref.accepted and ls["f"] < ls["f0"]


def test_armijo_sufficient_decrease_constant_decides():
    """With c = 0.4 the same start takes a smaller step than with c = 1e-4."""
    X, A = small_start((6, 5, 7), 4, 0.3, 3)
    ref, _ = armijo_compare(X, A, torch.float64, 1e-6, 1e-6, 50, c=0.4)
    assert ref.alpha == 0.0625


def test_armijo_other_shrink_factor():
    X, A = small_start((37, 29, 45), 12, 0.3, 2)
    ref, _ = armijo_compare(X, A, torch.float64, 1e-6, 1e-6, 50, shrink=0.3)
    assert ref.accepted and ref.alpha < 1.0


def test_armijo_full_step_is_the_plain_step_bitwise():
    """Near the planted solution alpha = 1 passes at the first trial: the factors and the update
    norm are the ones cp_gn_step writes, bit for bit (FP64 and FP32)."""
    p = make_problem((50, 45, 40), 8, workload=0, problem=8, noise=1e-4)
    rng = np.random.default_rng(7)
    A0 = [b + 1e-3 * rng.standard_normal(b.shape) for b in p.planted]
    for dt in (torch.float64, torch.float32):
        Xd = dev([p.x], dt)[0]
        Aa, Ag = dev(A0, dt), dev(A0, dt)
        st_a, ls = P.gn_step_armijo(Xd, Aa, 1e-6, 1e-3, 20)
        st_g = P.gn_step(Xd, Ag, 1e-6, 1e-3, 20)
        ls = P.read_armijo_stats(ls)
        assert ls["accepted"] == 1 and ls["trials"] == 1 and ls["alpha"] == 1.0
        for a, g in zip(Aa, Ag):
            assert torch.equal(a, g)
        assert P.read_stats(st_a) == P.read_stats(st_g)
        # f at the returned point is the direct residual there
        r = P.residual(Xd, Aa).cpu().numpy()
        assert abs(ls["f"] - 0.5 * r[0] ** 2) <= 1e-10 * ls["f0"]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_armijo_without_direction_or_passing_trial_keeps_factors(dt):
    X, A = small_start((37, 29, 45), 12, 0.3, 2)
    # cg_maxiter = 0: V = 0 is no descent direction, no trial runs
    armijo_compare(X, A, dt, 1e-6, 1e-6, 0, margin=0.0)
    # one trial allowed and alpha = 1 fails: the factors are restored bit for bit
    ref, ls = armijo_compare(X, A, dt, 1e-6, 0.0, 12, max_trials=1)
    assert not ref.accepted and ls["trials"] == 1
    # no trial allowed
    ref, ls = armijo_compare(X, A, dt, 1e-6, 0.0, 12, max_trials=0, margin=0.0)
    assert ls["trials"] == 0 and ls["accepted"] == 0


def test_armijo_bf16_tensor_properties():
    """bfloat16 storage: the reported values satisfy the Armijo condition, and f0 and f are the
    objective of the bfloat16 tensor at the start and returned factors (oracle in FP64)."""
    from workloads.synth import bf16_planes, bf16_values
    X, A = small_start((40, 36, 44), 10, 0.2, 5)
    for split in (False, True):
        planes = bf16_planes(X, split)
        Xv = bf16_values(planes, split)
        Xd = P.to_bf16(torch.tensor(X, dtype=torch.float32, device="cuda"), split=split)
        Ad = dev(A, torch.float32)
        A32 = [a.astype(np.float32).astype(np.float64) for a in A]
        _, ls = P.gn_step_armijo(Xd, Ad, 1e-6, 0.0, 12)
        ls = P.read_armijo_stats(ls)
        assert ls["accepted"] == 1 and ls["alpha"] < 1.0
        assert ls["f"] <= ls["f0"] + 1e-4 * ls["alpha"] * ls["gv"]
        assert abs(ls["f0"] - O.objective(Xv, A32)) <= 1e-5 * ls["f0"]
        assert abs(ls["f"] - O.objective(Xv, host(Ad))) <= 1e-5 * ls["f0"]


def test_armijo_descends_where_plain_gauss_newton_explodes():
    """Section 5 uses Armijo's condition to make Gauss-Newton converge more often: from a start
    where the plain step increases f by orders of magnitude, every Armijo step decreases it."""
    X, A = small_start((20, 18, 22), 6, 0.05, 0)
    Xd = dev([X], torch.float64)[0]
    plain = dev(A, torch.float64)
    P.gn_step(Xd, plain, 1e-6, 1e-6, 50)
    f_start = O.objective(X, A)
    assert O.objective(X, host(plain)) > 1e3 * f_start
    cfg = P.GNConfig(cg_tol=1e-6, cg_maxiter=50, schedule=P.ConstantDamping(1e-6),
                     line_search=P.Armijo())
    opt = P.GaussNewton(Xd, dev(A, torch.float64), cfg)
    fs = [f_start]
    for _ in range(8):
        opt.step()
        s = opt.stats()
        assert s["ls_accepted"] == 1
        assert s["ls_f"] < s["ls_f0"] and abs(s["ls_f0"] - fs[-1]) <= 1e-10 * fs[-1]
        fs.append(s["ls_f"])
    assert fs[-1] < 0.95 * fs[0]


def test_armijo_full_size_matches_plain_step():
    """At 400^3, R = 100 (FP32 storage, the throughput workload) near the planted solution, the
    search accepts alpha = 1 and the result is cp_gn_step's bit for bit."""
    p = make_problem((400, 400, 400), 100, workload=1)
    rng = np.random.default_rng(11)
    A0 = [b + 1e-2 * rng.standard_normal(b.shape) for b in p.planted]
    Xd = dev([p.x], torch.float32)[0]
    Aa, Ag = dev(A0, torch.float32), dev(A0, torch.float32)
    _, ls = P.gn_step_armijo(Xd, Aa, 1e-4, 1e-3, 20)
    P.gn_step(Xd, Ag, 1e-4, 1e-3, 20)
    ls = P.read_armijo_stats(ls)
    assert ls["accepted"] == 1 and ls["alpha"] == 1.0 and ls["f"] < ls["f0"]
    for a, g in zip(Aa, Ag):
        assert torch.equal(a, g)
