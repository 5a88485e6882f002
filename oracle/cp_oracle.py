"""Plain FP64 CPU oracle for Gauss-Newton (preconditioned implicit CG) and ALS CP decomposition.

TEST INFRASTRUCTURE. This module is the reference that the GPU library is checked against.
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does. It shares no code with the GPU library: it is NumPy/SciPy only and
imports nothing from the GPU package.

It follows N. Singh, L. Ma, H. Yang, E. Solomonik, "Comparison of Accuracy and Scalability of
Gauss-Newton and Alternating Least Squares for CP Decomposition" (arXiv:1910.12331). Equation
numbers refer to that paper: (1) the Khatri-Rao product P^(n), (2) the Hadamard product of Grams
Gamma^(n), (3) the objective f, (4) the Jacobian tensor, (5) the blocks of J^T J, (6) the
generalised Gamma^(n,p), (7) the implicit matrix-vector contraction. Algorithm 1 is CP-GN,
Algorithm 2 is CP-CG.

Conventions: a tensor is a C-order float64 ndarray of shape (s_1, ..., s_N); a factor list holds
N arrays A[n] of shape (s_n, R). Everything is computed in float64 in the order the paper
states it; library primitives (matmul, einsum, Cholesky) serve as single steps.

Readings of the paper that are not literal (each is listed in the design notes as well):
  * Algorithm 2 divides beta by sum <W,Q>; the standard preconditioned-CG ratio
    sum <R_new,Z_new> / sum <R_old,Z_old> is used instead (the literal ratio does not converge).
  * The varying-lambda schedule (Section 3.2) gives no constants; they are parameters here.
  * The relative residual (Section 5) is evaluated directly, as ||X - [[A]]||_F / ||X||_F.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

__all__ = [
    "full", "unfold", "khatri_rao", "mttkrp", "mttkrp_loops", "grams", "gamma", "gamma_set",
    "objective", "gradient", "jtj_matvec", "preconditioner", "pcg", "PCGResult", "gn_step",
    "GNStepStats", "LambdaSchedule", "als_sweep", "residual", "residual_expansion", "gn", "als",
    "jacobian", "jtj_dense", "flatten_factors", "unflatten_factors", "OracleError",
    "damping_matrix", "gn_step_armijo", "ArmijoResult", "cholesky_factors", "cholesky_apply",
    "block_norm_sum",
]


class OracleError(RuntimeError):
    """Raised where the method has no defined result (singular normal equations, breakdown)."""


# --------------------------------------------------------------------------------------------
# CP model and MTTKRP (Section 2.2)
# --------------------------------------------------------------------------------------------

def full(A):
    """Reconstruction [[A(1),...,A(N)]] = sum_r a_r(1) o ... o a_r(N)  (Section 2.2).

    Written as the sum over components of outer products, one component at a time.
    """
    dims = [a.shape[0] for a in A]
    rank = A[0].shape[1]
    out = np.zeros(dims)
    for r in range(rank):
        term = A[0][:, r]
        for a in A[1:]:
            term = np.multiply.outer(term, a[:, r])
        out += term
    return out


def unfold(X, n):
    """Mode-n matricization X_(n) of shape (s_n, prod_{m != n} s_m)  (Section 2.1).

    The column index runs over the remaining modes in increasing mode order with the last
    mode fastest, which is the ordering the Khatri-Rao product of eq. (1) produces.
    """
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def khatri_rao(mats):
    """Column-wise Kronecker product A(1) (.) A(2) (.) ... : column r is a_r(1) kron a_r(2) ...
    (Section 2.1). The first matrix's row index varies slowest."""
    rank = mats[0].shape[1]
    out = np.ones((1, rank))
    for m in mats:
        out = np.einsum("ir,jr->ijr", out, m).reshape(-1, rank)
    return out


def mttkrp(X, A, n):
    """M(n) = X_(n) P(n), with P(n) the Khatri-Rao product of all factors but A(n), eq. (1)."""
    others = [A[m] for m in range(len(A)) if m != n]
    return unfold(X, n) @ khatri_rao(others)


def mttkrp_loops(X, A, n):
    """Element-wise MTTKRP by explicit loops (tiny inputs only):
    M[k, r] = sum over all indices i with i_n = k of X[i] * prod_{m != n} A(m)[i_m, r]."""
    rank = A[0].shape[1]
    M = np.zeros((X.shape[n], rank))
    for idx in itertools.product(*[range(s) for s in X.shape]):
        for r in range(rank):
            prod = X[idx]
            for m, im in enumerate(idx):
                if m != n:
                    prod *= A[m][im, r]
            M[idx[n], r] += prod
    return M


# --------------------------------------------------------------------------------------------
# Grams and Gamma matrices, eqs. (2) and (6)
# --------------------------------------------------------------------------------------------

def grams(A):
    """S(i) = A(i)^T A(i) for every mode (Section 2.2)."""
    return [a.T @ a for a in A]


def gamma(S, n, p):
    """Gamma(n,p) = Hadamard product of S(m) over m not in {n, p}, eq. (6).

    With n == p this is Gamma(n) of eq. (2). An empty product (N = 2, n != p) is the all-ones
    matrix, the identity of the Hadamard product.
    """
    rank = S[0].shape[0]
    out = np.ones((rank, rank))
    for m in range(len(S)):
        if m != n and m != p:
            out = out * S[m]
    return out


def gamma_set(S):
    N = len(S)
    return [[gamma(S, n, p) for p in range(N)] for n in range(N)]


# --------------------------------------------------------------------------------------------
# Objective, gradient, J^T J (Section 3)
# --------------------------------------------------------------------------------------------

def objective(X, A):
    """f = 1/2 ||X - [[A]]||_F^2, eq. (3)."""
    d = X - full(A)
    return 0.5 * float(np.sum(d * d))


def gradient(X, A):
    """G(n) = A(n) Gamma(n,n) - M(n) for every mode, all at the same point (Algorithm 1)."""
    N = len(A)
    S = grams(A)
    return [A[n] @ gamma(S, n, n) - mttkrp(X, A, n) for n in range(N)]


def damping_matrix(Gam, n, damping="identity"):
    """The damping matrix D of mode n's block in (J^T J + lam D) (Section 3.2): the identity, or
    for damping == "diagonal" the diagonal of J^T J, whose block (n, n) is Gamma(n,n) (x) I by
    eq. (5), so every row of mode n is scaled by diag(Gamma(n,n))."""
    R = Gam[n][n].shape[0]
    if damping == "identity":
        return np.eye(R)
    if damping == "diagonal":
        return np.diag(np.diag(Gam[n][n]))
    raise ValueError(damping)


def jtj_matvec(A, W, lam=0.0, Gam=None, damping="identity"):
    """Q(n) = lam W(n) D(n) + sum_p (J^T J)(n,p) W(p): the damped Gauss-Newton matrix applied to
    W block by block (Algorithm 2, eq. (7)), with D(n) the damping matrix (identity, or the
    diagonal of J^T J).

    By eq. (5) the (n, n) block acts as W(n) Gamma(n,n). For p != n the block maps W(p) to the
    rows sum_{l,z} A(n)[k,z] A(p)[l,r] Gamma(n,p)[r,z] W(p)[l,z]; summing over l first gives
    A(n) (Gamma(n,p) * (W(p)^T A(p))), * the elementwise product (Gamma(n,p) is symmetric).
    """
    N = len(A)
    if Gam is None:
        Gam = gamma_set(grams(A))
    Q = []
    for n in range(N):
        q = lam * (W[n] @ damping_matrix(Gam, n, damping)) + W[n] @ Gam[n][n]
        for p in range(N):
            if p != n:
                q = q + A[n] @ (Gam[n][p] * (W[p].T @ A[p]))
        Q.append(q)
    return Q


def preconditioner(Gam, lam, damping="identity"):
    """P_inv(n) = (Gamma(n,n) + lam D(n))^-1 for every mode, built from a Cholesky factor
    (Algorithm 2, Section 3.3). Raises OracleError when the shifted matrix is not SPD."""
    out = []
    for n in range(len(Gam)):
        g = Gam[n][n] + lam * damping_matrix(Gam, n, damping)
        try:
            c = scipy.linalg.cho_factor(g, lower=True)
        except np.linalg.LinAlgError as e:
            raise OracleError(f"Gamma({n},{n}) + lambda I is not positive definite") from e
        out.append(scipy.linalg.cho_solve(c, np.eye(g.shape[0])))
    return out


def cholesky_factors(Gam, lam, damping="identity"):
    """Lower Cholesky factors L(n) of Gamma(n,n) + lam D(n), for the preconditioner applied by
    triangular solves (the alternative Section 3.3 describes and sets aside for its parallel
    depth). Raises OracleError when the shifted matrix is not SPD."""
    out = []
    for n in range(len(Gam)):
        g = Gam[n][n] + lam * damping_matrix(Gam, n, damping)
        try:
            out.append(scipy.linalg.cholesky(g, lower=True))
        except np.linalg.LinAlgError as e:
            raise OracleError(f"Gamma({n},{n}) + lambda I is not positive definite") from e
    return out


def cholesky_apply(L, Rn):
    """Z = R (L L^T)^-1 row by row: the forward solve L y = r^T, then the back solve L^T z = y."""
    y = scipy.linalg.solve_triangular(L, Rn.T, lower=True)
    return scipy.linalg.solve_triangular(L.T, y, lower=False).T


def _fro(m):
    return math.sqrt(float(np.sum(m * m)))


def _inner(a, b):
    return float(np.sum(a * b))


@dataclass
class PCGResult:
    V: list
    iters: int
    res_norm_sum: float      # sum_n ||R(n)||_F at exit
    grad_norm_sum: float     # sum_n ||G(n)||_F
    alpha_last: float = 0.0
    beta_last: float = 0.0
    history: list = field(default_factory=list)


def block_norm_sum(blocks):
    """sum_n ||B(n)||_F over the per-mode blocks: the norm Algorithms 1 and 2 use in their stop
    tests (a sum of per-mode Frobenius norms, not one 2-norm of the stacked vector)."""
    return sum(_fro(b) for b in blocks)


def pcg(G, A, lam, eps_cg=1e-3, maxiter=20, Gam=None, damping="identity", precond="inverse"):
    """Preconditioned CG for (J^T J + lam D) V = -G, D the identity or (damping == "diagonal")
    the diagonal of J^T J: the linear solve inside each step of Algorithm 1, with the block
    preconditioner (Gamma(n,n) + lam D(n))^-1 and the stop test of Algorithm 2.

    The iteration is the textbook preconditioned conjugate-gradient recurrence (Y. Saad,
    "Iterative Methods for Sparse Linear Systems", 2nd ed., SIAM 2003, Algorithm 9.1), run on the
    unknowns stacked into one vector x of length sum_n s_n R, starting from x = 0: the operator is
    eq. (7)'s product (jtj_matvec), the preconditioner acts block by block, and the inner
    products are plain dot products of the stacked vectors. Its direction coefficient is the
    textbook ratio of successive <r, z>; the printed Algorithm 2 divides by <W, Q> there instead,
    which is read as a typo (that ratio does not converge). Iteration stops when the sum of the
    per-mode residual norms is at most eps_cg times that of the gradient, or after maxiter
    iterations. A non-positive curvature <p, H p> raises OracleError.

    precond="cholesky" applies the same preconditioner by triangular solves with the Cholesky
    factor of Gamma(n,n) + lam D(n) (Section 3.3's alternative) instead of its explicit inverse.
    """
    N = len(A)
    dims = [a.shape[0] for a in A]
    rank = A[0].shape[1]
    if Gam is None:
        Gam = gamma_set(grams(A))
    if precond == "inverse":
        P = preconditioner(Gam, lam, damping)
        blockwise = lambda n, rn: rn @ P[n]   # noqa: E731
    elif precond == "cholesky":
        Lf = cholesky_factors(Gam, lam, damping)
        blockwise = lambda n, rn: cholesky_apply(Lf[n], rn)   # noqa: E731
    else:
        raise ValueError(precond)

    def split(v):
        return unflatten_factors(v, dims, rank)

    def op(v):          # y = (J^T J + lam D) v
        return flatten_factors(jtj_matvec(A, split(v), lam, Gam, damping))

    def prec(v):        # z = M^-1 v, one block per mode
        return flatten_factors([blockwise(n, b) for n, b in enumerate(split(v))])

    b = -flatten_factors(G)
    x = np.zeros_like(b)
    r = b.copy()                      # r0 = b - H x0 with x0 = 0
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    gsum = block_norm_sum(G)
    rsum = block_norm_sum(split(r))
    it, alpha, beta, hist = 0, 0.0, 0.0, []
    while rsum > eps_cg * gsum and it < maxiter:
        hp = op(p)
        curv = float(p @ hp)
        if not curv > 0.0:
            raise OracleError("CG breakdown: <p, H p> <= 0")
        alpha = rz / curv
        x = x + alpha * p
        r = r - alpha * hp
        z = prec(r)
        rz_next = float(r @ z)
        beta = rz_next / rz
        p = z + beta * p
        rz = rz_next
        rsum = block_norm_sum(split(r))
        it += 1
        hist.append(dict(alpha=alpha, beta=beta, res_norm_sum=rsum))
    return PCGResult(V=split(x), iters=it, res_norm_sum=rsum, grad_norm_sum=gsum,
                     alpha_last=alpha, beta_last=beta, history=hist)


@dataclass
class GNStepStats:
    cg_iters: int
    grad_norm_sum: float
    cg_res_norm_sum: float
    alpha_last: float
    beta_last: float
    lam: float
    update_norm: float


def gn_step(X, A, lam, eps_cg=1e-3, maxiter=20, damping="identity", precond="inverse"):
    """One loop body of Algorithm 1 (CP-GN): all M(n) at the current point, Gamma(n,p),
    G(n) = A(n) Gamma(n,n) - M(n), V = CP-CG(G, A, Gamma, eps_cg, lam), A(n) += V(n).

    Returns (new factors, GNStepStats). The input list is not modified.
    """
    N = len(A)
    S = grams(A)
    Gam = gamma_set(S)
    M = [mttkrp(X, A, n) for n in range(N)]
    G = [A[n] @ Gam[n][n] - M[n] for n in range(N)]
    res = pcg(G, A, lam, eps_cg, maxiter, Gam, damping, precond)
    newA = [A[n] + res.V[n] for n in range(N)]
    upd = math.sqrt(sum(float(np.sum(v * v)) for v in res.V))
    return newA, GNStepStats(cg_iters=res.iters, grad_norm_sum=res.grad_norm_sum,
                             cg_res_norm_sum=res.res_norm_sum, alpha_last=res.alpha_last,
                             beta_last=res.beta_last, lam=lam, update_norm=upd)


@dataclass
class ArmijoResult:
    A: list                # factors after the step (the input ones if no step size was accepted)
    alpha: float           # accepted step size (0 if none)
    trials: int            # objective evaluations made
    accepted: bool
    f0: float              # f at the start point, eq. (3)
    f: float               # f at the returned point
    gv: float              # directional derivative sum_n <G(n), V(n)> along the GN direction
    V: list                # the Gauss-Newton direction
    stats: GNStepStats


def gn_step_armijo(X, A, lam, eps_cg=1e-3, maxiter=20, damping="identity", c=1e-4, shrink=0.5,
                   max_trials=10, precond="inverse", f0=None):
    """Gauss-Newton step with Armijo step-size control (the variant Section 5 uses for the
    matrix-multiplication tensors): the direction V of Algorithm 1, then the step sizes
    alpha = 1, shrink, shrink^2, ... (at most max_trials of them) are tried in that order and the
    first one with f(A + alpha V) <= f(A) + c alpha <G, V> is taken (Armijo's sufficient-decrease
    condition; f is eq. (3), G its gradient). The paper gives no constants: c, shrink and
    max_trials are parameters. If <G, V> is not negative (no descent, e.g. V = 0) or no trial
    passes, the factors are returned unchanged with accepted = False. f0, when given, is f(A)
    (known from a previous evaluation at this point) and is not evaluated again."""
    N = len(A)
    S = grams(A)
    Gam = gamma_set(S)
    M = [mttkrp(X, A, n) for n in range(N)]
    G = [A[n] @ Gam[n][n] - M[n] for n in range(N)]
    res = pcg(G, A, lam, eps_cg, maxiter, Gam, damping, precond)
    if f0 is None:
        f0 = objective(X, A)
    gv = sum(_inner(G[n], res.V[n]) for n in range(N))
    alpha, trials, accepted, f, out = 1.0, 0, False, f0, [a.copy() for a in A]
    if gv < 0.0 and math.isfinite(f0):
        while trials < max_trials:
            trial = [A[n] + alpha * res.V[n] for n in range(N)]
            ft = objective(X, trial)
            trials += 1
            if ft <= f0 + c * alpha * gv:
                accepted, f, out = True, ft, trial
                break
            alpha *= shrink
    if not accepted:
        alpha = 0.0
    upd = alpha * math.sqrt(sum(float(np.sum(v * v)) for v in res.V))
    st = GNStepStats(cg_iters=res.iters, grad_norm_sum=res.grad_norm_sum,
                     cg_res_norm_sum=res.res_norm_sum, alpha_last=res.alpha_last,
                     beta_last=res.beta_last, lam=lam, update_norm=upd)
    return ArmijoResult(A=out, alpha=alpha, trials=trials, accepted=accepted, f0=f0, f=f, gv=gv,
                        V=res.V, stats=st)


class LambdaSchedule:
    """Varying damping of Section 3.2: start at the upper threshold, divide by mu each step
    until the lower threshold is reached, then multiply by mu until the upper threshold is
    reached, and repeat. ``value`` is the lambda for the current step; ``advance`` moves on."""

    def __init__(self, lam0=1e-4, lo=1e-10, hi=1e-4, mu=2.0):
        if not (mu > 1.0 and 0.0 < lo <= hi):
            raise ValueError("need mu > 1 and 0 < lo <= hi")
        self.value = float(lam0)
        self.lo, self.hi, self.mu = float(lo), float(hi), float(mu)
        self.down = True

    def advance(self):
        if self.down:
            self.value /= self.mu
            if self.value <= self.lo:
                self.down = False
        else:
            self.value *= self.mu
            if self.value >= self.hi:
                self.down = True
        return self.value

    def state(self):
        return dict(value=self.value, down=self.down, lo=self.lo, hi=self.hi, mu=self.mu)


# --------------------------------------------------------------------------------------------
# ALS (Section 2.2)
# --------------------------------------------------------------------------------------------

def als_sweep(X, A, lam=0.0):
    """One CP-ALS sweep, modes in increasing order (Gauss-Seidel): Gamma(n) from the current
    Grams, M(n) with the latest factors, A(n) = M(n) (Gamma(n) + lam I)^-1 by a Cholesky solve
    of the normal equations. Returns new factors; raises OracleError if Gamma(n)+lam I is not
    SPD."""
    A = [a.copy() for a in A]
    N = len(A)
    for n in range(N):
        S = grams(A)
        g = gamma(S, n, n) + lam * np.eye(A[n].shape[1])
        M = mttkrp(X, A, n)
        try:
            c = scipy.linalg.cho_factor(g, lower=True)
        except np.linalg.LinAlgError as e:
            raise OracleError(f"Gamma({n}) + lambda I is not positive definite") from e
        A[n] = scipy.linalg.cho_solve(c, M.T).T
    return A


# --------------------------------------------------------------------------------------------
# Residual (Section 5)
# --------------------------------------------------------------------------------------------

def residual(X, A):
    """Direct relative residual r = ||X - [[A]]||_F / ||X||_F (Section 5); fitness = 1 - r.

    Returns (||X - [[A]]||_F, ||X||_F). The squares are summed with math.fsum."""
    d = (X - full(A)).ravel()
    x = X.ravel()
    return math.sqrt(math.fsum(d * d)), math.sqrt(math.fsum(x * x))


def residual_expansion(X, A):
    """||X - [[A]]||^2 by the expansion ||X||^2 - 2 <M(1), A(1)> + sum_{r,z} prod_m S(m)[r,z].
    Cancels catastrophically near an exact fit; kept only to characterise that form."""
    S = grams(A)
    had = np.ones_like(S[0])
    for s in S:
        had = had * s
    xx = float(np.sum(X * X))
    cross = float(np.sum(mttkrp(X, A, 0) * A[0]))
    return xx - 2.0 * cross + float(np.sum(had)), math.sqrt(xx)


# --------------------------------------------------------------------------------------------
# Drivers (Algorithm 1 outer loop; ALS loop)
# --------------------------------------------------------------------------------------------

def gn(X, A0, schedule=None, eps_cg=1e-3, maxiter=20, target=1e-10, maxsteps=200, log=None,
       damping="identity"):
    """Algorithm 1 driver: GN steps until the direct relative residual <= target or maxsteps.
    lambda for step k is the schedule's value at step k (advanced after every step)."""
    sched = schedule or LambdaSchedule()
    A = [a.copy() for a in A0]
    hist = []
    for step in range(maxsteps):
        num, den = residual(X, A)
        if num / den <= target:
            break
        A, st = gn_step(X, A, sched.value, eps_cg, maxiter, damping)
        sched.advance()
        rec = dict(step=step, lam=st.lam, cg_iters=st.cg_iters, grad_norm_sum=st.grad_norm_sum)
        hist.append(rec)
        if log is not None:
            log(rec)
    num, den = residual(X, A)
    return A, hist, num / den


def als(X, A0, lam=0.0, target=1e-10, maxsweeps=500):
    A = [a.copy() for a in A0]
    hist = []
    for sweep in range(maxsweeps):
        num, den = residual(X, A)
        hist.append(num / den)
        if num / den <= target:
            break
        A = als_sweep(X, A, lam)
    num, den = residual(X, A)
    return A, hist, num / den


# --------------------------------------------------------------------------------------------
# Brute force for tiny inputs: explicit Jacobian, eq. (4)
# --------------------------------------------------------------------------------------------

def flatten_factors(A):
    return np.concatenate([a.ravel() for a in A])


def unflatten_factors(v, dims, rank):
    out, off = [], 0
    for s in dims:
        out.append(v[off:off + s * rank].reshape(s, rank))
        off += s * rank
    return out


def jacobian(A):
    """Explicit Jacobian of the residual X - [[A]] with respect to all factor entries, eq. (4):
    j(n)[i_1..i_N, k, r] = -(prod_{m != n} A(m)[i_m, r]) delta(i_n, k).
    Rows run over tensor entries in C order, columns over (n, k, r) in factor order."""
    dims = [a.shape[0] for a in A]
    rank = A[0].shape[1]
    ncols = sum(dims) * rank
    rows = int(np.prod(dims))
    J = np.zeros((rows, ncols))
    offs = np.cumsum([0] + [s * rank for s in dims])
    for row, idx in enumerate(itertools.product(*[range(s) for s in dims])):
        for n, k in enumerate(idx):
            for r in range(rank):
                prod = 1.0
                for m, im in enumerate(idx):
                    if m != n:
                        prod *= A[m][im, r]
                J[row, offs[n] + k * rank + r] = -prod
    return J


def jtj_dense(A):
    J = jacobian(A)
    return J.T @ J
