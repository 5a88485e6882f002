"""Parity of the HIP library (through its C ABI) with the FP64 oracle on identical seeded inputs.

Tolerances are normwise relative errors ||gpu - ref||_F / ||ref||_F:
  * FP64 paths: 1e-12 per call.
  * FP32 paths: the oracle runs in FP64 on the FP32-rounded inputs. MTTKRP 2e-5; quantities
    that cancel (gradient, residual) are measured against the size of the terms that cancel.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import make_problem, planted_tensor

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1910_12331_amd as P  # noqa: E402

TOL = {torch.float64: 1e-12, torch.float32: 2e-5}


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rnd_factors(dims, rank, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal((s, rank)) for s in dims]


def to_dev(arrs, dt):
    return [torch.tensor(a, dtype=dt, device="cuda").contiguous() for a in arrs]


def rounded(arrs, dt):
    """What the device sees, in float64 (FP32 inputs are rounded first)."""
    if dt == torch.float32:
        return [np.asarray(a, dtype=np.float32).astype(np.float64) for a in arrs]
    return [np.asarray(a, dtype=np.float64) for a in arrs]


def host(ts):
    return [t.double().cpu().numpy() for t in ts]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P._lib.load()
    yield
    torch.cuda.synchronize()


# ------------------------------------------------------------------------------------ MTTKRP
MTTKRP_CASES = [
    ((40, 40, 40), 5), ((37, 29, 51), 7), ((9, 7, 8, 6), 3), ((13, 17), 4), ((64, 48, 32), 16),
    ((30, 20, 25), 50), ((24, 20, 18), 100), ((12, 10, 9), 130), ((1, 5, 3), 2), ((5, 1, 3), 2),
    ((6, 5, 7, 3, 4), 9), ((70, 3, 66), 33), ((230, 17, 12), 20), ((20, 9, 7, 32), 12),
    ((9, 5, 6, 4, 8), 7), ((6, 4, 3, 5, 2, 12), 5), ((40, 2, 3, 2, 2, 2, 2, 16), 5),
]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank", MTTKRP_CASES, ids=[f"{d}-R{r}" for d, r in MTTKRP_CASES])
def test_mttkrp_matches_oracle(dims, rank, dt):
    rng = np.random.default_rng(sum(dims) + rank)
    X = rng.standard_normal(dims)
    A = rnd_factors(dims, rank, 7 + rank)
    Xh, Ah = rounded([X], dt)[0], rounded(A, dt)
    Xd, Ad = to_dev([X], dt)[0], to_dev(A, dt)
    for n in range(len(dims)):
        M = P.mttkrp(Xd, Ad, n)
        ref = O.mttkrp(Xh, Ah, n)
        assert rel(host([M])[0], ref) < TOL[dt], (n, rel(host([M])[0], ref))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank", MTTKRP_CASES, ids=[f"{d}-R{r}" for d, r in MTTKRP_CASES])
def test_mttkrp_all_matches_oracle(dims, rank, dt):
    """All-mode MTTKRP in one call (order 3: the dimension tree when the inner mode allows
    vector loads, else one pass per mode) against the oracle's per-mode definition."""
    rng = np.random.default_rng(sum(dims) + rank + 1)
    X = rng.standard_normal(dims)
    A = rnd_factors(dims, rank, 9 + rank)
    Xh, Ah = rounded([X], dt)[0], rounded(A, dt)
    Ms = P.mttkrp_all(to_dev([X], dt)[0], to_dev(A, dt))
    for n, M in enumerate(Ms):
        ref = O.mttkrp(Xh, Ah, n)
        assert rel(host([M])[0], ref) < TOL[dt], (n, rel(host([M])[0], ref))


TILE_SHAPES = [P.Tiles(4), P.Tiles(64, 1), P.Tiles(1, 8), P.Tiles(row_block=2),
               P.Tiles(row_block=4), P.Tiles(row_block=5), P.Tiles(8, 4, 2)]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank", [((150, 37, 60), 20), ((45, 33, 28, 20), 9),
                                       ((70, 3, 66), 33)])
def test_mttkrp_tile_shapes_match_oracle(dims, rank, dt):
    """Every MTTKRP tile shape (cp_set_tuning: items per wavefront, workgroups per compute unit,
    FP32 row tile) computes the contraction of Section 2.2: single-mode and all-mode calls
    against the oracle, on modes of several row tiles with a ragged tail, with and without
    vector loads (a last mode of 66); the defaults set explicitly give the default's bits, and
    the thread's setting is restored afterwards."""
    rng = np.random.default_rng(sum(dims) + rank + 5)
    X = rng.standard_normal(dims)
    A = rnd_factors(dims, rank, 11 + rank)
    Xh, Ah = rounded([X], dt)[0], rounded(A, dt)
    Xd, Ad = to_dev([X], dt)[0], to_dev(A, dt)
    N = len(dims)
    base = [P.mttkrp(Xd, Ad, n) for n in range(N)]
    with P.tiles(P.Tiles(16, 2, 0)):
        for n in range(N):
            assert torch.equal(P.mttkrp(Xd, Ad, n), base[n]), n
    refs = [O.mttkrp(Xh, Ah, n) for n in range(N)]
    for t in TILE_SHAPES:
        with P.tiles(t):
            for n in range(N):
                M = host([P.mttkrp(Xd, Ad, n)])[0]
                assert rel(M, refs[n]) < TOL[dt], (t, n, rel(M, refs[n]))
            for n, M in enumerate(P.mttkrp_all(Xd, Ad)):
                M = host([M])[0]
                assert rel(M, refs[n]) < TOL[dt], (t, "all", n, rel(M, refs[n]))
    assert P.get_tiles() == P.Tiles()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims", [(40, 1, 32), (40, 1, 20), (33, 2, 48), (40, 1, 1, 32),
                                  (20, 9, 7, 32)])
def test_mttkrp_all_tree_with_more_splits_than_items(dims, dt):
    """Dimension tree (mode 0 with vector loads) where the contraction has fewer items than
    wavefronts (middle modes of 1 or 2): a wavefront without items between two that share an
    outer index writes no partial, and the reduction must not read its slot. The workspace is
    filled with NaN first, so a stale slot (or an unwritten Pm row of order 4) would show."""
    rank = 5
    rng = np.random.default_rng(sum(dims) + 77)
    X = rng.standard_normal(dims)
    A = rnd_factors(dims, rank, 78)
    Xh, Ah = rounded([X], dt)[0], rounded(A, dt)
    Xd, Ad = to_dev([X], dt)[0], to_dev(A, dt)
    for t in [None, P.Tiles(1, 8)]:
        with P.tiles(t):
            ws = P.Workspace()
            ws.get(P.api._problem(Xd, rank), P._lib.OP_MTTKRP_ALL, Xd.device)
            ws._buf.fill_(255)   # all-ones bytes: NaN in FP32 and FP64
            Ms = P.mttkrp_all(Xd, Ad, ws=ws)
        for n, M in enumerate(Ms):
            M = host([M])[0]
            ref = O.mttkrp(Xh, Ah, n)
            assert np.isfinite(M).all() and rel(M, ref) < TOL[dt], (t, n, rel(M, ref))


def test_mttkrp_all_400_fp32_closed_form():
    """The bench's all-mode launch shape (400^3, R = 100, FP32, dimension tree for modes 0 and 1)
    against the planted closed form on every output."""
    rng = np.random.default_rng(3001)
    B = [rng.standard_normal((400, 100)).astype(np.float32).astype(np.float64) for _ in range(3)]
    X = planted_tensor(B).astype(np.float32)
    A = [rng.standard_normal((400, 100)).astype(np.float32).astype(np.float64) for _ in range(3)]
    Xd = torch.from_numpy(X).cuda()
    del X
    Ms = P.mttkrp_all(Xd, to_dev(A, torch.float32))
    for n in range(3):
        cross = np.ones((100, 100))
        for m in range(3):
            if m != n:
                cross *= B[m].T @ A[m]
        assert rel(host([Ms[n]])[0], B[n] @ cross) < 2e-5


def test_mttkrp_config2_full_size_fp64():
    """300^3, R = 50, congruent factors + noise (FP64), every mode against the oracle."""
    p = make_problem((300, 300, 300), 50, workload=2, kind="congruent", noise=1e-6)
    Xd = to_dev([p.x], torch.float64)[0]
    Ad = to_dev(p.init, torch.float64)
    for n in range(3):
        M = P.mttkrp(Xd, Ad, n)
        assert rel(host([M])[0], O.mttkrp(p.x, p.init, n)) < 1e-12


@pytest.mark.parametrize("tiles", [P.Tiles(4, 1, 4), P.Tiles(64, 4, 2)],
                         ids=["4items-1wg-64rows", "64items-4wg-32rows"])
def test_mttkrp_400_fp32_closed_form_tile_shapes(tiles):
    """The bench's 400^3 R = 100 FP32 shape under other MTTKRP tile shapes (single-mode and
    all-mode calls, several launches' worth of splits and row tiles) against the planted closed
    form M(n) = B(n) (Hadamard_{m != n} B(m)^T A(m)) in FP64."""
    rng = np.random.default_rng(3002)
    B = [rng.standard_normal((400, 100)).astype(np.float32).astype(np.float64) for _ in range(3)]
    X = planted_tensor(B).astype(np.float32)
    A = [rng.standard_normal((400, 100)).astype(np.float32).astype(np.float64) for _ in range(3)]
    Xd = torch.from_numpy(X).cuda()
    del X
    Ad = to_dev(A, torch.float32)
    refs = []
    for n in range(3):
        cross = np.ones((100, 100))
        for m in range(3):
            if m != n:
                cross *= B[m].T @ A[m]
        refs.append(B[n] @ cross)
    with P.tiles(tiles):
        for n in range(3):
            assert rel(host([P.mttkrp(Xd, Ad, n)])[0], refs[n]) < 2e-5, n
        for n, M in enumerate(P.mttkrp_all(Xd, Ad)):
            assert rel(host([M])[0], refs[n]) < 2e-5, ("all", n)


def test_mttkrp_400_fp32_closed_form():
    """400^3, R = 100 FP32 planted tensor: M(n) = B(n) (Hadamard_{m != n} B(m)^T A(m)) holds at
    any size; checked against that closed form (FP64) on the FP32-rounded factors."""
    rng = np.random.default_rng(3000)
    B = [rng.standard_normal((400, 100)).astype(np.float32).astype(np.float64) for _ in range(3)]
    X = planted_tensor(B).astype(np.float32)
    A = [rng.standard_normal((400, 100)).astype(np.float32).astype(np.float64) for _ in range(3)]
    Xd = torch.from_numpy(X).cuda()
    del X
    Ad = to_dev(A, torch.float32)
    for n in range(3):
        cross = np.ones((100, 100))
        for m in range(3):
            if m != n:
                cross *= B[m].T @ A[m]
        ref = B[n] @ cross
        M = P.mttkrp(Xd, Ad, n)
        # X itself is rounded to FP32 (relative 6e-8 per entry) on top of the FP32 contraction
        assert rel(host([M])[0], ref) < 2e-5
        # cp_mttkrp_marked (the bench's roofline timing): same bits, and the bracketed main
        # kernel lies inside the HIP-event time of the whole call
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for e in ev:
            e.record()
        ev[0].record()
        M2 = P.mttkrp(Xd, Ad, n, marks=(ev[1], ev[2]))
        ev[3].record()
        ev[3].synchronize()
        assert torch.equal(M2, M)
        t_kernel, t_call = ev[1].elapsed_time(ev[2]), ev[0].elapsed_time(ev[3])
        assert 0.0 < t_kernel <= t_call, (t_kernel, t_call)


# ------------------------------------------------------------------------------------ gradient
GRAD_CASES = [((40, 40, 40), 5), ((23, 18, 31), 6), ((9, 7, 8, 6), 3), ((11, 13), 4),
              ((30, 25, 20), 50), ((20, 9, 7, 32), 12), ((9, 5, 6, 4, 8), 7),
              ((40, 2, 3, 2, 2, 2, 2, 16), 5)]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank", GRAD_CASES, ids=[f"{d}-R{r}" for d, r in GRAD_CASES])
def test_gradient_matches_oracle(dims, rank, dt):
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-2)
    Xh, Ah = rounded([p.x], dt)[0], rounded(p.init, dt)
    G, gsum = P.gn_gradient(to_dev([p.x], dt)[0], to_dev(p.init, dt))
    ref = O.gradient(Xh, Ah)
    S = O.grams(Ah)
    scale = [np.linalg.norm(Ah[n] @ O.gamma(S, n, n)) + np.linalg.norm(O.mttkrp(Xh, Ah, n))
             for n in range(len(dims))]
    for n, (g, r) in enumerate(zip(host(G), ref)):
        err = np.linalg.norm(g - r) / scale[n]
        assert err < TOL[dt], (n, err)
    refsum = sum(np.linalg.norm(r) for r in ref)
    assert abs(float(gsum.item()) - refsum) / refsum < (1e-12 if dt == torch.float64 else 1e-4)


def test_gradient_config2_fp64():
    p = make_problem((300, 300, 300), 50, workload=2, kind="congruent", noise=1e-6)
    G, _ = P.gn_gradient(to_dev([p.x], torch.float64)[0], to_dev(p.init, torch.float64))
    for g, r in zip(host(G), O.gradient(p.x, p.init)):
        assert rel(g, r) < 1e-12


# ------------------------------------------------------------------------------------ J^T J
@pytest.mark.parametrize("dims,rank,lam", [((3, 4, 2), 2, 0.0), ((2, 3, 2, 3), 2, 0.3),
                                           ((4, 3), 3, 1e-2), ((5, 4, 6), 3, 1e-4)])
def test_jtj_matvec_explicit_jacobian(dims, rank, lam):
    A = rnd_factors(dims, rank, 11)
    W = rnd_factors(dims, rank, 12)
    Q = P.jtj_matvec(to_dev(A, torch.float64), to_dev(W, torch.float64), lam)
    H = O.jtj_dense(A)
    w = O.flatten_factors(W)
    assert rel(O.flatten_factors(host(Q)), H @ w + lam * w) < 1e-12


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank,lam", [((40, 40, 40), 5, 1e-4), ((300, 300, 300), 50, 1e-3),
                                           ((400, 400, 400), 100, 1e-4), ((17, 9, 12, 8), 7, 0.0)])
def test_jtj_matvec_matches_oracle(dims, rank, lam, dt):
    A = rounded(rnd_factors(dims, rank, 13), dt)
    W = rounded(rnd_factors(dims, rank, 14), dt)
    Q = P.jtj_matvec(to_dev(A, dt), to_dev(W, dt), lam)
    ref = O.jtj_matvec(A, W, lam)
    tol = 1e-12 if dt == torch.float64 else 1e-6   # FP64 inside; only the output is rounded
    assert rel(O.flatten_factors(host(Q)), O.flatten_factors(ref)) < tol


# ------------------------------------------------------------------------------------ GN step
def oracle_sensitivity(Xh, Ah, lam, eps, maxiter, seed=1, damping="identity", precond="inverse"):
    """Change of the oracle's GN update when its input factors move by 1e-15 relative: the
    rounding-level spread that any implementation with another summation order inherits
    (large once CG iterates past its rounding floor and loses orthogonality)."""
    rng = np.random.default_rng(seed)
    A2 = [a * (1 + 1e-15 * rng.standard_normal(a.shape)) for a in Ah]
    v1 = O.flatten_factors([b - a for a, b in
                            zip(Ah, O.gn_step(Xh, Ah, lam, eps, maxiter, damping, precond)[0])])
    v2 = O.flatten_factors([b - a for a, b in
                            zip(A2, O.gn_step(Xh, A2, lam, eps, maxiter, damping, precond)[0])])
    return float(np.linalg.norm(v1 - v2) / max(np.linalg.norm(v1), 1e-300))


def gn_compare(p, dt, lam, eps, maxiter, tol_v, damping="identity", precond="inverse"):
    Xh, Ah = rounded([p.x], dt)[0], rounded(p.init, dt)
    if tol_v == "sensitivity":
        tol_v = max(1e-12, 10 * oracle_sensitivity(Xh, Ah, lam, eps, maxiter, damping=damping,
                                                   precond=precond))
    Ad = to_dev(p.init, dt)
    st = P.read_stats(P.gn_step(to_dev([p.x], dt)[0], Ad, lam, eps, maxiter, damping=damping,
                                preconditioner=precond))
    newA, ref = O.gn_step(Xh, Ah, lam, eps, maxiter, damping, precond)
    assert st["status"] == 0
    assert st["cg_iters"] == ref.cg_iters
    V = [a - b for a, b in zip(host(Ad), Ah)]
    Vref = [a - b for a, b in zip(newA, Ah)]
    err = rel(O.flatten_factors(V), O.flatten_factors(Vref))
    assert err < tol_v, err
    assert abs(st["grad_norm_sum"] - ref.grad_norm_sum) <= tol_v * ref.grad_norm_sum
    return st, ref


def als_sensitivity_tol(Xh, Ah, lam, seed=2):
    """max(1e-12, 10x the change of the oracle's sweep when its input factors move by 1e-15
    relative): the rounding-level spread of a sweep whose later modes solve with Gamma(n) of
    large condition number."""
    rng = np.random.default_rng(seed)
    ref = O.als_sweep(Xh, Ah, lam)
    ref2 = O.als_sweep(Xh, [a * (1 + 1e-15 * rng.standard_normal(a.shape)) for a in Ah], lam)
    return max(1e-12, 10 * max(rel(r2, r) for r2, r in zip(ref2, ref)))


@pytest.mark.parametrize("maxiter", [0, 1, 5, 10])
def test_gn_step_fixed_iterations_fp64(maxiter):
    p = make_problem((40, 40, 40), 5, workload=1)
    gn_compare(p, torch.float64, 1e-4, 0.0, maxiter, 1e-12)


@pytest.mark.parametrize("maxiter", [0, 1, 5])
@pytest.mark.parametrize("dims", [(24, 10, 9, 16), (9, 5, 6, 4, 8)])
def test_gn_step_fixed_iterations_dimension_tree_orders_4_5_fp64(dims, maxiter):
    """Orders 4 and 5 with the last mode a multiple of 4: the gradient's modes 0 .. N-2 come
    from one pass over X (dimension tree and the outer-mode contraction)."""
    p = make_problem(dims, 6, workload=1)
    gn_compare(p, torch.float64, 1e-4, 0.0, maxiter, 1e-12)


@pytest.mark.parametrize("maxiter", [0, 1, 5, 10])
def test_gn_step_diagonal_damping_fixed_iterations_fp64(maxiter):
    """lam diag(J^T J) damping (Section 3.2) in the CG product and the preconditioner."""
    p = make_problem((40, 40, 40), 5, workload=1)
    gn_compare(p, torch.float64, 1e-2, 0.0, maxiter, 1e-12, damping="diagonal")


@pytest.mark.parametrize("damping", ["identity", "diagonal"])
@pytest.mark.parametrize("dims,rank", [((80, 80, 80), 120), ((60, 50, 70), 150),
                                       ((150, 150, 150), 200)])
def test_gn_step_high_rank_rank_exceeds_mode_size(dims, rank, damping):
    """The high-rank regime of Section 5 (s = 80, R = 120 and s = 150, R = 200, both above the
    mode sizes): each Gram has rank s < R, the damped systems stay SPD. Above R = 128 the inverse
    and the CG operand rows take 9 to 13 register blocks of 16 columns. CG with the tolerance
    test, both damping forms, FP64."""
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-2)
    gn_compare(p, torch.float64, 1e-2, 1e-3, 20, "sensitivity", damping=damping)


@pytest.mark.parametrize("damping", ["identity", "diagonal"])
@pytest.mark.parametrize("dims,rank", [((30, 28, 26), 230), ((40, 36, 24, 6), 300)])
def test_gn_step_rank_above_208(dims, rank, damping):
    """Ranks above 208 (Section 5's Cyclops runs go to R = 2000): the preconditioner inverse is
    blocked Gauss-Jordan in global memory and CG runs from the generic product kernels. CG with
    the tolerance test, both damping forms, FP64, against the oracle's step."""
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-2)
    gn_compare(p, torch.float64, 1e-2, 1e-3, 20, "sensitivity", damping=damping)


@pytest.mark.parametrize("maxiter", [0, 1, 7])
def test_gn_step_rank_above_208_fixed_iterations(maxiter):
    """R = 257 (17 blocks of 16 columns, the last one ragged) with exactly 0, 1 and 7 CG
    iterations (eps_cg = 0) against the oracle's step."""
    p = make_problem((20, 18, 22), 257, workload=0, problem=7, noise=1e-2)
    gn_compare(p, torch.float64, 5e-2, 0.0, maxiter, "sensitivity")


@pytest.mark.parametrize("dims,rank", [((60, 50, 70), 150), ((150, 150, 150), 200),
                                       ((30, 28, 26), 230), ((40, 36, 24, 6), 300)])
def test_als_sweep_high_rank(dims, rank):
    """ALS above R = 128 (each mode takes its own pass over X; the Cholesky factor has 13
    register blocks at R = 200, and above R = 208 it is blocked in global memory with the
    substitutions one block column per launch), held to 10x the oracle's own spread under a
    1e-15 input perturbation."""
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-2)
    Ad = to_dev(p.init, torch.float64)
    status = P.als_sweep(to_dev([p.x], torch.float64)[0], Ad, 1e-2)
    assert int(status.item()) == 0
    ref = O.als_sweep(p.x, p.init, 1e-2)
    rng = np.random.default_rng(2)
    ref2 = O.als_sweep(p.x, [a * (1 + 1e-15 * rng.standard_normal(a.shape)) for a in p.init], 1e-2)
    for a, r, r2 in zip(host(Ad), ref, ref2):
        assert rel(a, r) < max(1e-12, 10 * rel(r2, r))


def test_gn_step_past_cg_rounding_floor_fp64():
    """20 CG iterations with eps_cg = 0 run past convergence; the bar is 10x the oracle's own
    spread under a 1e-15 perturbation of its input."""
    p = make_problem((40, 40, 40), 5, workload=1)
    gn_compare(p, torch.float64, 1e-4, 0.0, 20, "sensitivity")


# R = 128 takes the per-operation CG kernels (its R x R tiles exceed the fused kernels' LDS).
@pytest.mark.parametrize("dims,rank,lam", [((40, 40, 40), 5, 1e-4), ((23, 18, 31), 6, 1e-2),
                                           ((9, 7, 8, 6), 3, 1e-3), ((11, 13), 4, 1e-3),
                                           ((60, 50, 40), 20, 1e-4), ((130, 120, 110), 100, 1e-2),
                                           ((150, 140, 136), 128, 1e-2)])
def test_gn_step_cg_tolerance_fp64(dims, rank, lam):
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-3)
    gn_compare(p, torch.float64, lam, 1e-3, 50, "sensitivity")


def test_gn_step_config2_fp64():
    p = make_problem((300, 300, 300), 50, workload=2, kind="congruent", noise=1e-6)
    st, ref = gn_compare(p, torch.float64, 1e-4, 1e-3, 20, "sensitivity")
    assert st["cg_iters"] >= 1


def test_gn_step_fp32():
    p = make_problem((40, 40, 40), 5, workload=1)
    gn_compare(p, torch.float32, 1e-4, 0.0, 10, 1e-4)


# ----------------------------------------------------- preconditioner by triangular solves
@pytest.mark.parametrize("maxiter", [0, 1, 5, 10])
def test_gn_step_cholesky_preconditioner_fixed_iterations_fp64(maxiter):
    """CP_GN_CHOL_PRECOND: the Cholesky factor of Gamma(n,n) + lambda I and a forward and a back
    triangular solve per CG application (Section 3.3's alternative to the explicit inverse)."""
    p = make_problem((40, 40, 40), 5, workload=1)
    gn_compare(p, torch.float64, 1e-4, 0.0, maxiter, 1e-12, precond="cholesky")


@pytest.mark.parametrize("dims,rank,lam,damping", [
    ((23, 18, 31), 6, 1e-2, "identity"), ((9, 7, 8, 6), 3, 1e-3, "identity"),
    ((11, 13), 4, 1e-3, "diagonal"), ((130, 120, 110), 100, 1e-2, "identity"),
    ((150, 140, 136), 128, 1e-2, "diagonal"), ((70, 65, 67), 33, 1e-3, "identity")])
def test_gn_step_cholesky_preconditioner_cg_tolerance_fp64(dims, rank, lam, damping):
    """Several 64-row blocks with ragged tails, orders 2 to 4, R up to 128 (the 64 KB LDS limit
    of the solve kernel), odd R, both damping forms."""
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-3)
    gn_compare(p, torch.float64, lam, 1e-3, 50, "sensitivity", damping=damping, precond="cholesky")


def test_gn_step_cholesky_preconditioner_fp32():
    p = make_problem((40, 40, 40), 5, workload=1)
    gn_compare(p, torch.float32, 1e-4, 0.0, 10, 1e-4, precond="cholesky")


def test_cholesky_and_inverse_preconditioners_agree_on_gpu():
    """Both forms apply the same operator: the steps agree to rounding. Bound: 10x the sum of the
    oracle's own difference between the two forms and its spread under 1e-15 input
    perturbations (at least 1e-12)."""
    p = make_problem((60, 50, 40), 20, workload=0, problem=20, noise=1e-3)
    ref = [O.flatten_factors([b - a for a, b in
                              zip(p.init, O.gn_step(p.x, p.init, 1e-3, 1e-3, 20, "identity", pc)[0])])
           for pc in ("inverse", "cholesky")]
    forms = float(np.linalg.norm(ref[1] - ref[0]) / np.linalg.norm(ref[0]))
    tol = max(1e-12, 10 * (forms + oracle_sensitivity(p.x, p.init, 1e-3, 1e-3, 20)))
    X = to_dev([p.x], torch.float64)[0]
    out = []
    for pc in ("inverse", "cholesky"):
        Ad = to_dev(p.init, torch.float64)
        st = P.read_stats(P.gn_step(X, Ad, 1e-3, 1e-3, 20, preconditioner=pc))
        out.append((st, [a - b for a, b in zip(host(Ad), p.init)]))
    assert out[0][0]["cg_iters"] == out[1][0]["cg_iters"]
    assert rel(O.flatten_factors(out[1][1]), O.flatten_factors(out[0][1])) < tol


def test_gn_step_cholesky_preconditioner_not_spd_leaves_factors():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((6, 1))
    A = [np.hstack([a, a]), rng.standard_normal((5, 2)), rng.standard_normal((4, 2))]
    A[1][:, 1] = A[1][:, 0]
    A[2][:, 1] = A[2][:, 0]
    Ad = to_dev(A, torch.float64)
    before = host(Ad)
    st = P.read_stats(P.gn_step(to_dev([rng.standard_normal((6, 5, 4))], torch.float64)[0], Ad,
                                0.0, 1e-3, 20, preconditioner="cholesky"))
    assert st["status"] == P._lib.CP_ENOTSPD
    for x, y in zip(host(Ad), before):
        assert np.array_equal(x, y)


def test_gn_step_zero_gradient_no_iteration():
    X = torch.zeros((8, 9, 10), dtype=torch.float64, device="cuda")
    A = [torch.zeros((s, 3), dtype=torch.float64, device="cuda") for s in (8, 9, 10)]
    st = P.read_stats(P.gn_step(X, A, 1e-3, 1e-3, 20))
    assert st["status"] == 0 and st["cg_iters"] == 0 and st["update_norm"] == 0.0
    assert all(float(a.abs().max()) == 0.0 for a in A)


def test_gn_step_not_spd_leaves_factors():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((6, 1))
    A = [np.hstack([a, a]), rng.standard_normal((5, 2)), rng.standard_normal((4, 2))]
    A[1][:, 1] = A[1][:, 0]
    A[2][:, 1] = A[2][:, 0]
    Ad = to_dev(A, torch.float64)
    before = host(Ad)
    st = P.read_stats(P.gn_step(to_dev([rng.standard_normal((6, 5, 4))], torch.float64)[0], Ad,
                                0.0, 1e-3, 20))
    assert st["status"] == P._lib.CP_ENOTSPD
    for x, y in zip(host(Ad), before):
        assert np.array_equal(x, y)


def test_gn_step_bitwise_deterministic():
    p = make_problem((50, 45, 40), 12, workload=0, problem=9, noise=1e-3)
    outs = []
    for _ in range(2):
        Ad = to_dev(p.init, torch.float64)
        P.gn_step(to_dev([p.x], torch.float64)[0], Ad, 1e-3, 1e-3, 20)
        outs.append(host(Ad))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


# ------------------------------------------------------------------------------------ ALS
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank,lam", [((40, 40, 40), 5, 0.0), ((23, 18, 31), 6, 1e-2),
                                           ((9, 7, 8, 6), 3, 0.0), ((30, 25, 20), 50, 1e-3)])
def test_als_sweep_matches_oracle(dims, rank, lam, dt):
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-2)
    Xh, Ah = rounded([p.x], dt)[0], rounded(p.init, dt)
    Ad = to_dev(p.init, dt)
    status = P.als_sweep(to_dev([p.x], dt)[0], Ad, lam)
    assert int(status.item()) == 0
    ref = O.als_sweep(Xh, Ah, lam)
    tol = 1e-12 if dt == torch.float64 else 1e-4
    for a, r in zip(host(Ad), ref):
        assert rel(a, r) < tol


def test_als_with_step_decay_regularization_matches_oracle():
    """ALS with lambda = 0.01 halved every 2 sweeps (the schedule of Section 5, compressed):
    each sweep against the oracle's sweep with the same lambda."""
    p = make_problem((30, 26, 34), 6, workload=0, problem=6, noise=1e-2)
    X = to_dev([p.x], torch.float64)[0]
    opt = P.ALS(X, to_dev(p.init, torch.float64), schedule=P.StepDecay(1e-2, 0.5, 2))
    ref = [a.copy() for a in p.init]
    for k in range(5):
        lam = 1e-2 * 0.5 ** (k // 2)
        assert opt.schedule.value == lam
        assert int(opt.step().item()) == 0
        tol = als_sensitivity_tol(p.x, ref, lam)
        ref = O.als_sweep(p.x, ref, lam)
        for a, r in zip(host(opt.A), ref):
            assert rel(a, r) < tol


def test_als_sweep_config2_fp64():
    """After the first mode the congruent data make the Grams ill-conditioned (cond ~1e9-1e11),
    so later modes are held to 10x the oracle's own spread under a 1e-15 input perturbation."""
    p = make_problem((300, 300, 300), 50, workload=2, kind="congruent", noise=1e-6)
    Ad = to_dev(p.init, torch.float64)
    P.als_sweep(to_dev([p.x], torch.float64)[0], Ad, 0.0)
    ref = O.als_sweep(p.x, p.init)
    rng = np.random.default_rng(1)
    ref2 = O.als_sweep(p.x, [a * (1 + 1e-15 * rng.standard_normal(a.shape)) for a in p.init])
    for a, r, r2 in zip(host(Ad), ref, ref2):
        assert rel(a, r) < max(1e-12, 10 * rel(r2, r))


# ------------------------------------------------------------------------------------ residual
# R = 130, 200, 208: the MFMA kernel with 9 to 13 column blocks (one 16-row sub-tile per
# wavefront); R = 230: the scalar kernel.
RES_CASES = [((40, 40, 40), 5), ((37, 29, 51), 7), ((9, 7, 8, 6), 3), ((13, 17), 4),
             ((12, 10, 9), 130), ((24, 20, 18), 100), ((23, 19, 41), 200),
             ((9, 11, 7, 13), 208), ((14, 12, 10), 230)]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank", RES_CASES, ids=[f"{d}-R{r}" for d, r in RES_CASES])
def test_residual_matches_oracle(dims, rank, dt):
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-1)
    Xh, Ah = rounded([p.x], dt)[0], rounded(p.init, dt)
    out = P.residual(to_dev([p.x], dt)[0], to_dev(p.init, dt)).cpu().numpy()
    num, den = O.residual(Xh, Ah)
    tol = 1e-12 if dt == torch.float64 else 1e-5
    assert abs(out[0] - num) / num < tol and abs(out[1] - den) / den < tol
    ex = P.residual(to_dev([p.x], dt)[0], to_dev(p.init, dt), method=1).cpu().numpy()
    e2, _ = O.residual_expansion(Xh, Ah)
    assert abs(ex[0] ** 2 - e2) / (den * den + abs(e2)) < (1e-12 if dt == torch.float64 else 1e-5)


def test_residual_at_planted_solution_fp64():
    p = make_problem((60, 50, 40), 8, workload=0, problem=1)
    out = P.residual(to_dev([p.x], torch.float64)[0], to_dev(p.planted, torch.float64)).cpu().numpy()
    assert out[0] / out[1] < 1e-14


# ------------------------------------------------------------------------------------ end to end
def test_gn_end_to_end_config1():
    p = make_problem((40, 40, 40), 5, workload=1)
    X = to_dev([p.x], torch.float64)[0]
    Ad = to_dev(p.init, torch.float64)
    opt = P.GaussNewton(X, Ad, P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
    r = opt.residual()
    for _ in range(200):
        if r <= 1e-10:
            break
        opt.step()
        assert opt.stats()["status"] == 0
        r = opt.residual()
    assert r <= 1e-10
    _, hist, rref = O.gn(p.x, p.init, O.LambdaSchedule(1e-4, 1e-10, 1e-4, 2.0), 1e-3, 20, 1e-10, 200)
    assert rref <= 1e-10 and abs(opt.steps - len(hist)) <= 3
    num, den = O.residual(p.x, host(Ad))
    assert num / den <= 1e-10


def test_als_end_to_end_config1_monotone():
    p = make_problem((40, 40, 40), 5, workload=1)
    X = to_dev([p.x], torch.float64)[0]
    Ad = to_dev(p.init, torch.float64)
    opt = P.ALS(X, Ad)
    last = math.inf
    for _ in range(300):
        r = opt.residual()
        assert r <= last * (1 + 1e-9)
        last = r
        if r <= 1e-10:
            break
        opt.step()
    assert last <= 1e-10


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_als_sweep_dimension_tree_and_per_mode_paths_match_oracle(dt):
    """Order 3: with the ALS workspace (room for T = X x_3 A(3)) modes 1 and 2 come from T; with
    the smaller workspace of the other operations each mode takes its own pass over X. Both
    sweeps match the oracle."""
    import ctypes as C
    from paper_1910_12331_amd import _lib as L
    from paper_1910_12331_amd import api
    p = make_problem((36, 28, 44), 9, workload=0, problem=9, noise=1e-2)
    Xh, Ah = rounded([p.x], dt)[0], rounded(p.init, dt)
    ref = O.als_sweep(Xh, Ah, 1e-3)
    X = to_dev([p.x], dt)[0]
    prob = api._problem(X, 9)
    sizes = []
    for op in (L.OP_ALS_SWEEP, L.OP_GN_STEP):
        n = C.c_size_t(0)
        assert L.load().cp_workspace_bytes(C.byref(prob), op, C.byref(n)) == 0
        sizes.append(int(n.value))
    assert sizes[0] > sizes[1]
    ws = torch.empty(sizes[0] + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    tol = 1e-12 if dt == torch.float64 else 1e-4
    for nbytes in sizes:
        Ad = to_dev(p.init, dt)
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        rc = L.load().cp_als_sweep(C.byref(prob), X.data_ptr(), api._ptrs(Ad), 1e-3, status.data_ptr(),
                                   base, nbytes, api._stream())
        assert rc == 0
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        for a, r in zip(host(Ad), ref):
            assert rel(a, r) < tol, nbytes


# ------------------------------------------------------------------ the largest order (8) and 7
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("dims,rank", [((3, 2, 4, 2, 3, 2, 2, 3), 3), ((2, 3, 2, 2, 3, 2, 2, 2), 17),
                                       ((4, 3, 2, 3, 2, 3, 2), 5)])
def test_highest_orders_every_entry_point(dims, rank, dt):
    """Orders 7 and 8 (CP_MAX_ORDER), mode sizes 2 to 4 (ragged 16-row tiles), R = 17 over two
    column blocks: MTTKRP per mode and all modes, the gradient, J^T J, a GN step with a fixed CG
    iteration count, an ALS sweep and the direct residual against the oracle (on the rounded
    inputs for FP32)."""
    f64 = dt == torch.float64
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-1)
    Xh, Ah = rounded([p.x], dt)[0], rounded(p.init, dt)
    X = to_dev([p.x], dt)[0]
    A = to_dev(p.init, dt)
    tm = 1e-12 if f64 else 2e-5
    for n in range(len(dims)):
        assert rel(P.mttkrp(X, A, n).double().cpu().numpy(), O.mttkrp(Xh, Ah, n)) < tm
    for n, m in enumerate(P.mttkrp_all(X, A)):
        assert rel(m.double().cpu().numpy(), O.mttkrp(Xh, Ah, n)) < tm
    G, _ = P.gn_gradient(X, A)
    for g, gr in zip(G, O.gradient(Xh, Ah)):
        assert rel(g.double().cpu().numpy(), gr) < (1e-12 if f64 else 1e-4)
    W = [np.random.default_rng(7).standard_normal(a.shape) for a in p.init]
    Wh = rounded(W, dt)
    Q = P.jtj_matvec(A, to_dev(W, dt), 1e-2)
    for q, qr in zip(Q, O.jtj_matvec(Ah, Wh, 1e-2)):
        assert rel(q.double().cpu().numpy(), qr) < (1e-12 if f64 else 1e-6)
    gn_compare(p, dt, 1e-3, 0.0, 5, "sensitivity" if f64 else 1e-4)
    Aals = to_dev(p.init, dt)
    assert int(P.als_sweep(X, Aals, 1e-3).item()) == 0
    ta = als_sensitivity_tol(Xh, Ah, 1e-3) if f64 else 1e-4
    for a, r in zip(host(Aals), O.als_sweep(Xh, Ah, 1e-3)):
        assert rel(a, r) < ta
    out = P.residual(X, A).cpu().numpy()
    num, den = O.residual(Xh, Ah)
    tr = 1e-12 if f64 else 1e-5
    assert abs(out[0] - num) / num < tr and abs(out[1] - den) / den < tr


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_mode_longer_than_one_row_tile_grid(dt):
    """2.2 million rows in mode 0: 68750 (FP64) and 34375 (FP32) row tiles per single-mode launch,
    137500 and 68750 in the order-3 tree pass, so the launches run in chunks of at most 65535 row
    tiles. MTTKRP of every mode, the all-mode call, the residual and a GN step against the
    oracle."""
    dims, R = (2_200_000, 3, 4), 4
    p = make_problem(dims, R, workload=0, problem=41, noise=1e-2)
    Xh, Ah = rounded([p.x], dt)[0], rounded(p.init, dt)
    X = to_dev([p.x], dt)[0]
    A = to_dev(p.init, dt)
    tol = 1e-12 if dt == torch.float64 else 2e-5
    for n in range(3):
        assert rel(P.mttkrp(X, A, n).double().cpu().numpy(), O.mttkrp(Xh, Ah, n)) < tol
    for n, m in enumerate(P.mttkrp_all(X, A)):
        assert rel(m.double().cpu().numpy(), O.mttkrp(Xh, Ah, n)) < tol
    out = P.residual(X, A).cpu().numpy()
    num, den = O.residual(Xh, Ah)
    assert abs(out[0] - num) / num < (1e-12 if dt == torch.float64 else 1e-5)
    gn_compare(p, dt, 1e-3, 0.0, 3, "sensitivity" if dt == torch.float64 else 1e-4)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_als_sweep_not_spd_leaves_factors(dt):
    """A zero column in every factor but mode 0's makes Gamma(0) singular with an exact zero
    pivot: the Cholesky factorization reports CP_ENOTSPD and the sweep leaves every factor as it
    was (the later modes are skipped too)."""
    p = make_problem((30, 20, 25), 6, workload=0, problem=6, noise=1e-2)
    A = [a.copy() for a in p.init]
    A[1][:, 2] = 0.0
    A[2][:, 2] = 0.0
    Ad = to_dev(A, dt)
    before = [a.clone() for a in Ad]
    status = P.als_sweep(to_dev([p.x], dt)[0], Ad, 0.0)
    assert int(status.item()) == P._lib.CP_ENOTSPD
    for a, b in zip(Ad, before):
        assert torch.equal(a, b)
