"""Pins for the FP64 oracle: each check is fixed by the paper or by mathematics, not by the
oracle's own formulas (brute force, closed forms, invariants, textbook routines, a hand-worked
example). CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from workloads import make_problem, planted_tensor, gaussian_factors, congruent_factors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def factors(dims, rank, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((s, rank)) for s in dims]


# ---------------------------------------------------------------- hand-worked example
def test_golden_hand_worked_2x2x2():
    g = json.load(open(os.path.join(GOLDEN, "mttkrp_2x2x2_rank1.json")))
    X = np.array(g["X"], dtype=float)
    A = [np.array(a, dtype=float) for a in g["A"]]
    for n in range(3):
        assert np.array_equal(O.mttkrp(X, A, n), np.array(g["M"][n], dtype=float))
    num, den = O.residual(X, A)
    assert num * num == pytest.approx(g["residual_sq"], rel=1e-15)
    assert den * den == pytest.approx(g["x_norm_sq"], rel=1e-15)
    assert np.allclose(O.gradient(X, A)[0], np.array(g["G1"], dtype=float), rtol=0, atol=1e-13)


# ---------------------------------------------------------------- MTTKRP
@pytest.mark.parametrize("dims,rank", [((4, 3, 2), 2), ((3, 4, 2, 5), 3), ((5, 3), 2),
                                       ((1, 3, 2), 2), ((3, 1, 4), 3), ((2, 2, 2, 2, 2), 2)])
def test_mttkrp_brute_force(dims, rank):
    X = rnd(dims, 1)
    A = factors(dims, rank, 2)
    for n in range(len(dims)):
        assert rel(O.mttkrp(X, A, n), O.mttkrp_loops(X, A, n)) < 1e-14


@pytest.mark.parametrize("dims,rank,R2", [((30, 20, 25), 4, 6), ((9, 7, 8, 6), 3, 5), ((12, 17), 3, 4)])
def test_mttkrp_planted_closed_form(dims, rank, R2):
    """X = [[B]] gives M(n) = B(n) (Hadamard_{m != n} B(m)^T A(m)) (eq. (1) with the Gram form
    of eq. (2) applied to the cross products); also pins the generator against full()."""
    B = factors(dims, rank, 3)
    A = factors(dims, R2, 4)
    X = planted_tensor(B)
    assert rel(X, O.full(B)) < 1e-14
    for n in range(len(dims)):
        cross = np.ones((rank, R2))
        for m in range(len(dims)):
            if m != n:
                cross *= B[m].T @ A[m]
        assert rel(O.mttkrp(X, A, n), B[n] @ cross) < 1e-13


def test_full_brute_force():
    A = factors((3, 4, 2), 3, 5)
    X = O.full(A)
    for i in range(3):
        for j in range(4):
            for k in range(2):
                ref = sum(A[0][i, r] * A[1][j, r] * A[2][k, r] for r in range(3))
                assert X[i, j, k] == pytest.approx(ref, rel=1e-14, abs=1e-14)


# ---------------------------------------------------------------- Jacobian, gradient
def test_jacobian_columns_are_exact_differences():
    """The residual is linear in every single factor entry, so a central difference in one
    entry reproduces that column of J (eq. (4)) up to rounding."""
    dims, rank = (3, 2, 4), 2
    A = factors(dims, rank, 6)
    X = rnd(dims, 7)
    J = O.jacobian(A)
    v = O.flatten_factors(A)
    h = 0.5
    for col in range(v.size):
        vp, vm = v.copy(), v.copy()
        vp[col] += h
        vm[col] -= h
        rp = (X - O.full(O.unflatten_factors(vp, dims, rank))).ravel()
        rm = (X - O.full(O.unflatten_factors(vm, dims, rank))).ravel()
        assert np.allclose((rp - rm) / (2 * h), J[:, col], atol=1e-13, rtol=0)


@pytest.mark.parametrize("dims,rank", [((3, 4, 2), 2), ((2, 3, 2, 3), 2), ((4, 3), 3)])
def test_gradient_equals_JT_r(dims, rank):
    A = factors(dims, rank, 8)
    X = rnd(dims, 9)
    J = O.jacobian(A)
    r = (X - O.full(A)).ravel()
    g = O.flatten_factors(O.gradient(X, A))
    assert rel(g, J.T @ r) < 1e-13


def test_gradient_finite_differences():
    dims, rank = (4, 3, 5), 3
    A = factors(dims, rank, 10)
    X = rnd(dims, 11)
    g = O.flatten_factors(O.gradient(X, A))
    v = O.flatten_factors(A)
    h = 1e-5
    fd = np.empty_like(v)
    for i in range(v.size):
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        fd[i] = (O.objective(X, O.unflatten_factors(vp, dims, rank))
                 - O.objective(X, O.unflatten_factors(vm, dims, rank))) / (2 * h)
    assert rel(g, fd) < 1e-8


def test_gradient_zero_at_planted_solution():
    p = make_problem((20, 15, 18), 4, workload=0, problem=3)
    G = O.gradient(p.x, p.planted)
    M = [O.mttkrp(p.x, p.planted, n) for n in range(3)]
    for g, m in zip(G, M):
        assert np.linalg.norm(g) / np.linalg.norm(m) < 1e-13


# ---------------------------------------------------------------- J^T J
@pytest.mark.parametrize("dims,rank,lam", [((3, 4, 2), 2, 0.0), ((2, 3, 2, 3), 2, 0.3),
                                           ((4, 3), 3, 1e-2), ((2, 2, 3), 3, 0.0)])
def test_jtj_matvec_explicit_J(dims, rank, lam):
    A = factors(dims, rank, 12)
    W = factors(dims, rank, 13)
    H = O.jtj_dense(A)
    q = O.flatten_factors(O.jtj_matvec(A, W, lam))
    w = O.flatten_factors(W)
    assert rel(q, H @ w + lam * w) < 1e-13


def test_jtj_diagonal_blocks_are_gamma_kron_identity():
    """H(n,n) = Gamma(n,n) (x) I (Section 3.3); H(n,p) from eq. (5) with Gamma(n,p) of eq. (6)."""
    dims, rank = (3, 4, 2), 3
    A = factors(dims, rank, 14)
    H = O.jtj_dense(A)
    S = O.grams(A)
    offs = np.cumsum([0] + [s * rank for s in dims])
    for n in range(3):
        for p in range(3):
            blk = H[offs[n]:offs[n + 1], offs[p]:offs[p + 1]].reshape(dims[n], rank, dims[p], rank)
            gam = O.gamma(S, n, p)
            for k in range(dims[n]):
                for r in range(rank):
                    for l in range(dims[p]):
                        for z in range(rank):
                            if n == p:
                                ref = (k == l) * gam[r, z]
                            else:
                                ref = A[n][k, z] * A[p][l, r] * gam[r, z]
                            assert blk[k, r, l, z] == pytest.approx(ref, abs=1e-12)


def test_gamma_empty_product_is_all_ones():
    A = factors((4, 5), 3, 15)
    S = O.grams(A)
    assert np.array_equal(O.gamma(S, 0, 1), np.ones((3, 3)))
    assert np.array_equal(O.gamma(S, 0, 0), S[1])


def test_jtj_sum_of_mttkrp_identity():
    """J W = -Y with Y = sum_p [[A(1)..W(p)..A(N)]] (eq. (4)), and (J^T v)(n) = -MTTKRP_n(v),
    so (J^T J W)(n) = MTTKRP_n(Y): a medium-size check that never forms J."""
    dims, rank = (9, 7, 8), 3
    A = factors(dims, rank, 16)
    W = factors(dims, rank, 17)
    Y = sum(O.full([W[m] if m == p else A[m] for m in range(3)]) for p in range(3))
    Q = O.jtj_matvec(A, W, 0.0)
    for n in range(3):
        assert rel(Q[n], O.mttkrp(Y, A, n)) < 1e-13


def test_jtj_scaling_directions_null_and_symmetry():
    dims, rank = (5, 4, 6), 3
    A = factors(dims, rank, 18)
    for r in range(rank):
        D = [np.zeros_like(a) for a in A]
        D[0][:, r] = A[0][:, r]
        D[1][:, r] = -A[1][:, r]
        Q = O.jtj_matvec(A, D, 0.0)
        assert max(np.linalg.norm(q) for q in Q) < 1e-12 * max(np.linalg.norm(a) for a in A) ** 5
    U = factors(dims, rank, 19)
    W = factors(dims, rank, 20)
    HU, HW = O.jtj_matvec(A, U, 0.1), O.jtj_matvec(A, W, 0.1)
    lhs = sum(np.sum(u * h) for u, h in zip(U, HW))
    rhs = sum(np.sum(h * w) for h, w in zip(HU, W))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    assert sum(np.sum(w * h) for w, h in zip(W, HW)) > 0


# ---------------------------------------------------------------- PCG
def _dense_pcg(H, P, g, k):
    """Textbook PCG on explicit matrices, k iterations, started from zero."""
    x = np.zeros_like(g)
    r = -g
    z = P @ r
    w = z.copy()
    rz = r @ z
    for _ in range(k):
        q = H @ w
        a = rz / (w @ q)
        x = x + a * w
        r = r - a * q
        z = P @ r
        rz2 = r @ z
        w = z + (rz2 / rz) * w
        rz = rz2
    return x


def _block_precond(H, dims, rank, lam):
    n = H.shape[0]
    P = np.zeros((n, n))
    offs = np.cumsum([0] + [s * rank for s in dims])
    for m in range(len(dims)):
        sl = slice(offs[m], offs[m + 1])
        P[sl, sl] = np.linalg.inv(H[sl, sl] + lam * np.eye(offs[m + 1] - offs[m]))
    return P


@pytest.mark.parametrize("k", [1, 3, 7])
def test_pcg_fixed_iterations_match_dense(k):
    dims, rank, lam = (3, 4, 3), 2, 0.05
    A = factors(dims, rank, 21)
    X = rnd(dims, 22)
    G = O.gradient(X, A)
    res = O.pcg(G, A, lam, eps_cg=0.0, maxiter=k)
    assert res.iters == k
    H = O.jtj_dense(A) + lam * np.eye(sum(dims) * rank)
    P = _block_precond(O.jtj_dense(A), dims, rank, lam)
    ref = _dense_pcg(H, P, O.flatten_factors(G), k)
    assert rel(O.flatten_factors(res.V), ref) < 1e-11


def test_pcg_converged_equals_dense_solve_and_lm_step():
    dims, rank, lam = (3, 2, 4), 2, 0.1
    A = factors(dims, rank, 23)
    X = rnd(dims, 24)
    G = O.gradient(X, A)
    n = sum(dims) * rank
    res = O.pcg(G, A, lam, eps_cg=1e-14, maxiter=10 * n)
    H = O.jtj_dense(A) + lam * np.eye(n)
    ref = np.linalg.solve(H, -O.flatten_factors(G))
    assert rel(O.flatten_factors(res.V), ref) < 1e-10
    newA, st = O.gn_step(X, A, lam, eps_cg=1e-14, maxiter=10 * n)
    assert rel(O.flatten_factors(newA), O.flatten_factors(A) + ref) < 1e-10


def test_pcg_zero_gradient_takes_no_iteration():
    A = factors((4, 3, 5), 2, 25)
    G = [np.zeros_like(a) for a in A]
    res = O.pcg(G, A, 1e-3)
    assert res.iters == 0 and all(np.count_nonzero(v) == 0 for v in res.V)


def test_pcg_singular_gamma_without_damping_raises():
    a = rnd((5, 1), 26)
    A = [np.hstack([a, a]), rnd((4, 2), 27), rnd((3, 2), 28)]
    A[1][:, 1] = A[1][:, 0]
    A[2][:, 1] = A[2][:, 0]
    with pytest.raises(O.OracleError):
        O.preconditioner(O.gamma_set(O.grams(A)), 0.0)


def test_gn_fast_local_convergence_near_solution():
    p = make_problem((12, 10, 11), 3, workload=0, problem=4)
    rng = np.random.default_rng(0)
    A = [b + 1e-3 * rng.standard_normal(b.shape) for b in p.planted]
    r = []
    for _ in range(4):
        num, den = O.residual(p.x, A)
        r.append(num / den)
        A, _ = O.gn_step(p.x, A, 1e-6, eps_cg=1e-10, maxiter=500)
    # quadratic decrease (Gauss-Newton on a zero-residual problem), down to rounding
    assert r[1] < r[0] ** 2 and r[2] < 1e3 * r[1] ** 2 and r[3] < 1e-14


# ---------------------------------------------------------------- lambda schedule
def test_lambda_schedule_state_machine():
    s = O.LambdaSchedule(lam0=8.0, lo=1.0, hi=8.0, mu=2.0)
    seq = [s.value] + [s.advance() for _ in range(10)]
    assert seq == [8, 4, 2, 1, 2, 4, 8, 4, 2, 1, 2]


# ---------------------------------------------------------------- ALS
def test_als_mode_update_is_least_squares_minimiser():
    dims, rank = (5, 4, 6), 2
    X = rnd(dims, 29)
    A = factors(dims, rank, 30)
    new = O.als_sweep(X, A)
    # mode 0 uses A[1], A[2]; solve min ||X_(0) - A0 P^T|| by lstsq with P built by loops
    P = np.zeros((dims[1] * dims[2], rank))
    for j in range(dims[1]):
        for k in range(dims[2]):
            P[j * dims[2] + k] = A[1][j] * A[2][k]
    ref = np.linalg.lstsq(P, X.reshape(dims[0], -1).T, rcond=None)[0].T
    assert rel(new[0], ref) < 1e-12


def test_als_residual_monotone():
    p = make_problem((15, 12, 14), 4, workload=0, problem=5, noise=1e-2)
    A = p.init
    last = math.inf
    for _ in range(30):
        num, _ = O.residual(p.x, A)
        assert num <= last * (1 + 1e-12)
        last = num
        A = O.als_sweep(p.x, A)


def test_als_rank1_exact_in_one_sweep():
    B = factors((6, 5, 7), 1, 31)
    X = O.full(B)
    A = O.als_sweep(X, factors((6, 5, 7), 1, 32))
    num, den = O.residual(X, A)
    assert num / den < 1e-14


# ---------------------------------------------------------------- residual
def test_residual_at_planted_and_expansion():
    p = make_problem((10, 9, 8), 3, workload=0, problem=6)
    num, den = O.residual(p.x, p.planted)
    assert num / den < 1e-15
    A = factors((10, 9, 8), 3, 33)
    num, den = O.residual(p.x, A)
    e2, _ = O.residual_expansion(p.x, A)
    assert e2 == pytest.approx(num * num, rel=1e-10)


# ---------------------------------------------------------------- congruence generator
def test_congruent_factors_cosines():
    rng = np.random.default_rng(0)
    A = congruent_factors((50, 40), 6, rng, 0.9)
    for a in A:
        c = a.T @ a
        d = np.sqrt(np.diag(c))
        cos = c / np.outer(d, d)
        assert np.allclose(cos[~np.eye(6, dtype=bool)], 0.9, atol=1e-12)


# ---------------------------------------------------------------- end to end (small config)
def _factor_match(A, B):
    """Mean over components of the product of |cosines| after a greedy permutation match."""
    R = A[0].shape[1]
    C = np.ones((R, R))
    for a, b in zip(A, B):
        an = a / np.linalg.norm(a, axis=0)
        bn = b / np.linalg.norm(b, axis=0)
        C *= np.abs(an.T @ bn)
    used, score = set(), 0.0
    for i in np.argsort(-C.max(axis=1)):
        j = max((j for j in range(R) if j not in used), key=lambda j: C[i, j])
        used.add(j)
        score += C[i, j]
    return score / R


def test_gn_recovers_planted_config1():
    p = make_problem((40, 40, 40), 5, workload=1)
    A, hist, r = O.gn(p.x, p.init, O.LambdaSchedule(1e-4, 1e-10, 1e-4, 2.0), 1e-3, 20, 1e-10, 200)
    assert r <= 1e-10
    assert _factor_match(A, p.planted) >= 1 - 1e-8


def test_pcg_stop_rule_sum_of_frobenius_norms():
    """CG stops at the first iterate with sum_n ||R(n)||_F <= eps_cg sum_n ||G(n)||_F
    (Algorithm 2 loop condition), tracked here with the explicit dense iteration."""
    dims, rank, lam = (4, 3, 3), 2, 1e-3
    A = factors(dims, rank, 40)
    X = rnd(dims, 41)
    G = O.gradient(X, A)
    H = O.jtj_dense(A) + lam * np.eye(sum(dims) * rank)
    P = _block_precond(O.jtj_dense(A), dims, rank, lam)
    g = O.flatten_factors(G)
    gsum = sum(np.linalg.norm(x) for x in G)
    offs = np.cumsum([0] + [s * rank for s in dims])
    eps = 1e-2
    k_stop = None
    for k in range(1, 200):
        x = _dense_pcg(H, P, g, k)
        r = -g - H @ x
        rs = sum(np.linalg.norm(r[offs[m]:offs[m + 1]]) for m in range(3))
        if rs <= eps * gsum:
            k_stop = k
            break
    res = O.pcg(G, A, lam, eps_cg=eps, maxiter=1000)
    assert res.iters == k_stop


def test_als_sweep_is_gauss_seidel_least_squares():
    dims, rank = (4, 5, 3), 2
    X = rnd(dims, 42)
    A = factors(dims, rank, 43)
    ref = [a.copy() for a in A]
    for n in range(3):
        others = [m for m in range(3) if m != n]
        P = np.zeros((dims[others[0]] * dims[others[1]], rank))
        for i in range(dims[others[0]]):
            for j in range(dims[others[1]]):
                P[i * dims[others[1]] + j] = ref[others[0]][i] * ref[others[1]][j]
        Xn = np.moveaxis(X, n, 0).reshape(dims[n], -1)
        ref[n] = np.linalg.lstsq(P, Xn.T, rcond=None)[0].T
    new = O.als_sweep(X, A)
    for a, b in zip(new, ref):
        assert rel(a, b) < 1e-12


# ------------------------------------------------------------------ diagonal damping (Section 3.2)
def test_diagonal_damping_is_diag_of_explicit_jtj():
    """D = diag(J^T J) taken from the explicit Jacobian equals the damping matrix built from
    Gamma(n,n); the damped product equals (H + lam diag(H)) w."""
    dims, rank, lam = (4, 3, 5), 3, 0.3
    A = factors(dims, rank, 41)
    W = factors(dims, rank, 42)
    H = O.jtj_dense(A)
    Gam = O.gamma_set(O.grams(A))
    dflat = np.concatenate([np.tile(np.diag(O.damping_matrix(Gam, n, "diagonal")), dims[n])
                            for n in range(3)])
    assert rel(dflat, np.diag(H)) < 1e-14
    q = O.flatten_factors(O.jtj_matvec(A, W, lam, damping="diagonal"))
    w = O.flatten_factors(W)
    assert rel(q, H @ w + lam * np.diag(H) * w) < 1e-13


def test_diagonal_damping_pcg_converges_to_dense_solve():
    dims, rank, lam = (3, 4, 2), 2, 0.05
    A = factors(dims, rank, 43)
    X = rnd(dims, 44)
    G = O.gradient(X, A)
    n = sum(dims) * rank
    res = O.pcg(G, A, lam, eps_cg=1e-14, maxiter=10 * n, damping="diagonal")
    H = O.jtj_dense(A)
    ref = np.linalg.solve(H + lam * np.diag(np.diag(H)), -O.flatten_factors(G))
    assert rel(O.flatten_factors(res.V), ref) < 1e-10
    # the preconditioner is the inverse of the damped diagonal block
    Gam = O.gamma_set(O.grams(A))
    P = O.preconditioner(Gam, lam, "diagonal")
    blk = Gam[1][1] + lam * np.diag(np.diag(Gam[1][1]))
    assert rel(P[1] @ blk, np.eye(rank)) < 1e-12


def test_diagonal_damping_scale_invariance_of_the_damping_term():
    """Scaling column r of A(m), m != n, by c scales Gamma(n,n)[r,r] and the damping entry of
    mode n alike (unlike lam I): the diagonal term follows the problem's own scaling."""
    A = factors((4, 3, 5), 2, 45)
    B = [a.copy() for a in A]
    B[1][:, 0] *= 3.0
    G1, G2 = O.gamma_set(O.grams(A)), O.gamma_set(O.grams(B))
    d1, d2 = O.damping_matrix(G1, 0, "diagonal"), O.damping_matrix(G2, 0, "diagonal")
    assert abs(d2[0, 0] - 9.0 * d1[0, 0]) <= 1e-12 * d2[0, 0] and abs(d2[1, 1] - d1[1, 1]) < 1e-14


# ---------------------------------------------------------------- Armijo step control
def _objective_einsum(X, A):
    """f of eq. (3) for an order-3 tensor, the reconstruction written as one einsum (not the
    oracle's component-by-component sum)."""
    d = X - np.einsum("ir,jr,kr->ijk", *A)
    return 0.5 * float(np.sum(d * d))


def _small_start(seed, scale):
    rng = np.random.default_rng(seed)
    dims, R = (6, 5, 7), 4
    X = rng.standard_normal(dims)
    return X, [scale * rng.standard_normal((s, R)) for s in dims]


@pytest.mark.parametrize("c,expect_alpha", [(1e-4, 0.125), (0.4, 0.0625)])
def test_armijo_choice_by_brute_force(c, expect_alpha):
    # a start at a small scale, where the full Gauss-Newton step overshoots
    X, A = _small_start(3, 0.3)
    res = O.gn_step_armijo(X, A, 1e-6, eps_cg=1e-6, maxiter=50, c=c)
    # <G, V> is the derivative of alpha -> f(A + alpha V) at 0: central differences
    h = 1e-6
    fp = _objective_einsum(X, [a + h * v for a, v in zip(A, res.V)])
    fm = _objective_einsum(X, [a - h * v for a, v in zip(A, res.V)])
    gfd = (fp - fm) / (2 * h)
    assert gfd < 0 and abs(res.gv - gfd) < 1e-7 * abs(gfd)
    # the first of 1, 1/2, 1/4, ... meeting the sufficient-decrease condition, each trial kept
    # well away from its threshold so that the choice is unambiguous
    f0 = _objective_einsum(X, A)
    alpha, k = 1.0, 0
    while True:
        ft = _objective_einsum(X, [a + alpha * v for a, v in zip(A, res.V)])
        thr = f0 + c * alpha * gfd
        assert abs(ft - thr) > 1e-3 * f0
        k += 1
        if ft <= thr:
            break
        alpha *= 0.5
    assert alpha == expect_alpha            # the c term decides between the two cases
    assert res.accepted and res.alpha == alpha and res.trials == k
    assert abs(res.f0 - f0) < 1e-12 * f0 and abs(res.f - ft) < 1e-12 * f0 and res.f < f0
    for a, v, out in zip(A, res.V, res.A):
        assert np.array_equal(out, a + alpha * v)


def test_armijo_descends_where_the_full_step_explodes():
    X, A = _small_start(0, 0.05)
    res = O.gn_step_armijo(X, A, 1e-6, eps_cg=1e-6, maxiter=50)
    full_step = _objective_einsum(X, [a + v for a, v in zip(A, res.V)])
    assert full_step > 1e6 * res.f0                    # plain Gauss-Newton diverges here
    assert res.accepted and res.alpha < 0.01 and res.f < res.f0


def test_armijo_full_step_near_solution_is_the_gn_step():
    p = make_problem((12, 10, 11), 3, workload=0, problem=4)
    rng = np.random.default_rng(5)
    A = [b + 1e-3 * rng.standard_normal(b.shape) for b in p.planted]
    res = O.gn_step_armijo(p.x, A, 1e-6, eps_cg=1e-10, maxiter=500)
    ref, _ = O.gn_step(p.x, A, 1e-6, eps_cg=1e-10, maxiter=500)
    assert res.accepted and res.alpha == 1.0 and res.trials == 1
    assert all(np.array_equal(a, b) for a, b in zip(res.A, ref))
    assert res.f < 1e-6 * res.f0                       # quadratic convergence region


def test_armijo_without_descent_direction_or_passing_trial_keeps_factors():
    X, A = _small_start(3, 0.3)
    none = O.gn_step_armijo(X, A, 1e-6, maxiter=0)     # V = 0: <G, V> = 0 is no descent
    assert not none.accepted and none.alpha == 0.0 and none.trials == 0
    one = O.gn_step_armijo(X, A, 1e-6, eps_cg=1e-6, maxiter=50, max_trials=1)   # alpha = 1 fails
    assert not one.accepted and one.alpha == 0.0 and one.trials == 1 and one.f == one.f0
    for res in (none, one):
        assert all(np.array_equal(a, b) for a, b in zip(res.A, A))


# ---------------------------------------------------------------- Cholesky preconditioner
@pytest.mark.parametrize("k", [1, 3, 7])
@pytest.mark.parametrize("damping", ["identity", "diagonal"])
def test_pcg_cholesky_preconditioner_matches_dense(k, damping):
    """The preconditioner applied by triangular solves (Section 3.3's alternative) gives the
    iterates of textbook dense PCG with the block-diagonal preconditioner."""
    dims, rank, lam = (3, 4, 3), 2, 0.05
    A = factors(dims, rank, 23)
    X = rnd(dims, 24)
    G = O.gradient(X, A)
    res = O.pcg(G, A, lam, eps_cg=0.0, maxiter=k, damping=damping, precond="cholesky")
    assert res.iters == k
    J = O.jtj_dense(A)
    D = np.diag(np.diag(J)) if damping == "diagonal" else np.eye(J.shape[0])
    H = J + lam * D
    n = H.shape[0]
    P = np.zeros((n, n))
    offs = np.cumsum([0] + [s * rank for s in dims])
    for m in range(len(dims)):
        sl = slice(offs[m], offs[m + 1])
        P[sl, sl] = np.linalg.inv(J[sl, sl] + lam * D[sl, sl])   # the diagonal block of H
    ref = _dense_pcg(H, P, O.flatten_factors(G), k)
    assert rel(O.flatten_factors(res.V), ref) < 1e-11


def test_cholesky_apply_is_a_solve():
    rng = np.random.default_rng(25)
    B = rng.standard_normal((6, 6))
    M = B @ B.T + 6 * np.eye(6)
    L = O.cholesky_factors([[M]], 0.0)[0]
    assert np.allclose(L, np.tril(L)) and rel(L @ L.T, M) < 1e-15
    Rn = rng.standard_normal((9, 6))
    assert rel(O.cholesky_apply(L, Rn), np.linalg.solve(M, Rn.T).T) < 1e-14
