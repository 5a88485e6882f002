"""GPU tests of the bfloat16 tensor forms (x_dtype CP_BF16 and the split CP_BF16X3) through
the C ABI, against the FP64 oracle on the values the bfloat16 storage represents.

Error bound. The stored tensor is exact (the oracle takes hi, or hi + lo, in FP64). The library
forms each Khatri-Rao entry K = A(q)[k, r] * P_o[r] in FP32 (P_o, the outer modes' row, rounded
once to FP32) and rounds it to bfloat16 (relative error <= 2^-8; <= 2^-16 for its hi + lo split),
drops the lo*lo product in the split form (<= 2^-16 (1 + 2^-8)^2 relative to |X||K|), and sums in
FP32: 32 products per matrix instruction into an accumulator that runs over the L items of one
wavefront, then the fixed four-wavefront sum; the partial tiles are added in FP64. Elementwise,
with Mabs = MTTKRP(|X|, |A|):
    |M_gpu - M| <= gamma * Mabs,  gamma = u_f + 2 (L + 48) 2^-24,
u_f = 2^-8 (single plane) or 1.1 * 2^-15 (split); L is computed from the launch geometry below.
A dropped term or a wrong operand layout exceeds it by orders of magnitude.
"""
import numpy as np
import pytest

import oracle as O
from workloads import bf16_planes, bf16_values, make_problem

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


def dev_x(planes, split):
    t = torch.from_numpy(np.ascontiguousarray(planes).view(np.int16)).view(torch.bfloat16).cuda()
    return P.SplitBF16Tensor(t) if split else t


def dev_f(arrs):
    return [torch.tensor(a, dtype=torch.float32, device="cuda") for a in arrs]


def f32(arrs):
    return [np.asarray(a, dtype=np.float32).astype(np.float64) for a in arrs]


def items_per_wavefront(dims, mode):
    """Largest number of (outer index, 32-wide inner chunk) items one wavefront accumulates:
    row tiles of 80 rows (64 for the last mode), one resident workgroup per compute unit (256)
    split over the tiles, four wavefronts per workgroup (eight for the last mode), at least two
    items per wavefront."""
    N = len(dims)
    caseB = mode == N - 1
    q = N - 2 if caseB else N - 1
    J = dims[mode]
    outer = int(np.prod(dims)) // J // dims[q]
    nitems = outer * ((dims[q] + 31) // 32)
    rt = -(-J // (64 if caseB else 80))
    w = 8 if caseB else 4
    sw = max(1, min(256 // rt, -(-nitems // (2 * w)), 1024))
    return -(-nitems // (w * sw))


def gamma(dims, mode, split):
    L = items_per_wavefront(dims, mode)
    return (1.1 * 2.0 ** -15 if split else 2.0 ** -8) + 2 * (L + 48) * 2.0 ** -24


def stored(p, split):
    planes = bf16_planes(p.x, split)
    return planes, bf16_values(planes, split)


# ------------------------------------------------------------------ storage conversion
@pytest.mark.parametrize("split", [False, True])
def test_to_bf16_bit_exact(split):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(100_003).astype(np.float32) * np.float32(100.0)
    x[:6] = [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, -0.0, 3.0e-39]
    out = P.to_bf16(torch.tensor(x, device="cuda"), split=split)
    got = (out.planes if split else out).cpu().view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, bf16_planes(x, split))


# ------------------------------------------------------------------ MTTKRP
SHAPES = [
    ((24, 20, 16, 32), 64),   # order 4, vector loads in both cases
    ((37, 29, 45), 20),       # inner size 45 and last mode 45: scalar-load paths
    ((33, 26, 40), 80),       # R = 80: two launches of four column blocks
    ((96, 96, 96), 16),       # several row tiles and items per wavefront, ragged tiles
    ((50, 47), 7),            # order 2
    ((6, 5, 7, 4, 8), 5),     # order 5
    ((20, 18, 16), 130),      # R = 130: three launches (4 + 4 + 1 column blocks)
]


@pytest.mark.parametrize("split", [False, True], ids=["bf16", "bf16x3"])
@pytest.mark.parametrize("dims,rank", SHAPES)
def test_mttkrp_within_bound(dims, rank, split):
    p = make_problem(dims, rank, workload=4, problem=rank, kind="lognorm", noise=1e-3)
    planes, xv = stored(p, split)
    A = f32(p.init)
    X = dev_x(planes, split)
    Ad = dev_f(A)
    absA = [np.abs(a) for a in A]
    for n in range(len(dims)):
        M = P.mttkrp(X, Ad, n).double().cpu().numpy()
        ref = O.mttkrp(xv, A, n)
        bound = gamma(dims, n, split) * O.mttkrp(np.abs(xv), absA, n) + 1e-30
        ratio = float(np.max(np.abs(M - ref) / bound))
        assert ratio <= 1.0, (n, ratio)


@pytest.mark.parametrize("split", [False, True], ids=["bf16", "bf16x3"])
@pytest.mark.parametrize("dims,rank", [((28, 22, 24, 16), 20), ((40, 33, 32), 24),
                                       ((6, 5, 7, 4, 8), 5), ((30, 1, 1, 32), 9),
                                       ((28, 22, 24, 18), 20)])
def test_mttkrp_all_within_bound(dims, rank, split):
    """All modes at one point (one pass per mode for a bfloat16 tensor), orders 3 to 5, middle
    modes of 1, a last mode that rules out vector loads. The workspace is filled with NaN first,
    so a partial or table entry left unwritten would show."""
    p = make_problem(dims, rank, workload=4, problem=21, kind="lognorm", noise=1e-3)
    planes, xv = stored(p, split)
    A = f32(p.init)
    absA = [np.abs(a) for a in A]
    X = dev_x(planes, split)
    ws = P.Workspace()
    ws.get(P.api._problem(X, rank), P._lib.OP_MTTKRP_ALL, X.device)
    ws._buf.fill_(255)
    Ms = P.mttkrp_all(X, dev_f(A), ws=ws)
    for n, M in enumerate(Ms):
        ref = O.mttkrp(xv, A, n)
        bound = gamma(dims, n, split) * O.mttkrp(np.abs(xv), absA, n) + 1e-30
        assert np.all(np.abs(M.double().cpu().numpy() - ref) <= bound), n


@pytest.mark.parametrize("split", [False, True], ids=["bf16", "bf16x3"])
def test_mttkrp_full_size_sampled_rows(split):
    """80^4, R = 64, log-uniform column norms, noise 1e-3 (the benchmark's launch shape): rows
    of every mode's MTTKRP against the oracle on the one-row slices."""
    dims, rank = (80, 80, 80, 80), 64
    p = make_problem(dims, rank, workload=4, problem=0, kind="lognorm", noise=1e-3)
    planes, xv = stored(p, split)
    A = f32(p.init)
    X = dev_x(planes, split)
    Ad = dev_f(A)
    for n in range(4):
        M = P.mttkrp(X, Ad, n).double().cpu().numpy()
        for j in (0, 37, 79):
            xs = np.take(xv, [j], axis=n)
            As = [a[j:j + 1] if m == n else a for m, a in enumerate(A)]
            ref = O.mttkrp(xs, As, n)[0]
            bound = gamma(dims, n, split) * O.mttkrp(np.abs(xs), [np.abs(a) for a in As], n)[0]
            assert np.all(np.abs(M[j] - ref) <= bound), (n, j)
    torch.cuda.synchronize()


def test_mttkrp_split_is_more_accurate():
    """Normwise, the split form is at least 30x closer to the oracle than the single plane on the
    same tensor values (both represent the same rounded-to-16-bit tensor here)."""
    dims, rank = (40, 36, 48), 32
    p = make_problem(dims, rank, workload=4, problem=9, kind="lognorm", noise=1e-3)
    planes = bf16_planes(p.x, True)
    xv = bf16_values(planes[0], False)           # a tensor exactly representable in one plane
    split_planes = np.stack([planes[0], np.zeros_like(planes[0])])
    A = f32(p.init)
    Ad = dev_f(A)
    ref = O.mttkrp(xv, A, 0)
    e1 = np.linalg.norm(P.mttkrp(dev_x(planes[0], False), Ad, 0).double().cpu().numpy() - ref)
    e3 = np.linalg.norm(P.mttkrp(dev_x(split_planes, True), Ad, 0).double().cpu().numpy() - ref)
    assert e3 * 30 < e1


# ------------------------------------------------------------------ residual, gradient, step
@pytest.mark.parametrize("split", [False, True], ids=["bf16", "bf16x3"])
def test_residual_matches_oracle(split):
    dims, rank = (30, 26, 22, 20), 12
    p = make_problem(dims, rank, workload=4, problem=3, kind="lognorm", noise=1e-3)
    planes, xv = stored(p, split)
    A = f32(p.init)
    num, den = O.residual(xv, A)
    out = P.residual(dev_x(planes, split), dev_f(A)).cpu().numpy()
    assert abs(out[0] - num) / num < 1e-5 and abs(out[1] - den) / den < 1e-6
    # the expansion's cross term 2 <M(1), A(1)> comes from the bfloat16 MTTKRP: its error is at
    # most 2 gamma <Mabs, |A(1)|>, which is at most 2 gamma (||X||^2 + ||[[A]]||^2); relative to
    # ||X||^2 + |squared residual| that is below 4 gamma
    ex = P.residual(dev_x(planes, split), dev_f(A), method=1).cpu().numpy()
    e2, _ = O.residual_expansion(xv, A)
    assert abs(ex[0] ** 2 - e2) / (den * den + abs(e2)) < 4 * gamma(dims, 0, split) + 1e-5


@pytest.mark.parametrize("split", [False, True], ids=["bf16", "bf16x3"])
@pytest.mark.parametrize("dims", [(24, 22, 20, 18), (24, 22, 20, 16)])
def test_gradient_vs_fp64_master(dims, split):
    """Error of the GPU gradient against the FP64 oracle on the FP64 master tensor, within the
    bound that storage rounding plus the MTTKRP bound give: elementwise
    |G_gpu - G| <= MTTKRP(|X_stored - X|, |A|) + gamma MTTKRP(|X_stored|, |A|) + 2^-23 |G_gpu|.
    Last modes of 18 and 16 (scalar and vector loads along the inner index)."""
    rank = 16
    p = make_problem(dims, rank, workload=4, problem=5, kind="lognorm", noise=1e-3)
    planes, xv = stored(p, split)
    A = f32(p.init)
    absA = [np.abs(a) for a in A]
    G, _ = P.gn_gradient(dev_x(planes, split), dev_f(A))
    ref = O.gradient(p.x, A)
    dx = np.abs(xv - p.x)
    for n in range(4):
        g = G[n].double().cpu().numpy()
        bound = (O.mttkrp(dx, absA, n) + gamma(dims, n, split) * O.mttkrp(np.abs(xv), absA, n)
                 + 2.0 ** -23 * np.abs(g) + 1e-30)
        assert np.all(np.abs(g - ref[n]) <= bound), n


@pytest.mark.parametrize("split", [False, True], ids=["bf16", "bf16x3"])
def test_gn_step_matches_oracle_on_stored_tensor(split):
    """One Gauss-Newton step (fixed CG iteration count) on the bfloat16 tensor against the FP64
    oracle's step on the values it stores: the gradient error (gamma relative, see above) carries
    through the linear CG iteration, so the update agrees to a small multiple of gamma."""
    dims, rank = (20, 18, 16, 24), 8
    p = make_problem(dims, rank, workload=4, problem=2, kind="lognorm", noise=1e-3)
    planes, xv = stored(p, split)
    A = f32(p.init)
    Ad = dev_f(A)
    st = P.gn_step(dev_x(planes, split), Ad, 1e-4, 0.0, 5)
    s = P.read_stats(st)
    assert s["status"] == 0 and s["cg_iters"] == 5
    ref, _ = O.gn_step(xv, A, 1e-4, 0.0, 5)
    tol = 40 * max(gamma(dims, n, split) for n in range(4))
    for a, r, a0 in zip(Ad, ref, A):
        upd = a.double().cpu().numpy() - a0
        assert np.linalg.norm(upd - (r - a0)) <= tol * np.linalg.norm(r - a0) + 1e-6 * np.linalg.norm(a0)


@pytest.mark.parametrize("split", [False, True], ids=["bf16", "bf16x3"])
def test_als_sweep_matches_oracle_on_stored_tensor(split):
    """One ALS sweep (Section 2.2) on the bfloat16 tensor against the oracle's sweep on the values
    it stores. Mode n's update M(n) (Gamma(n) + lam I)^-1 inherits the MTTKRP error: relative
    error <= kappa_n gamma ||Mabs(n)|| / ||M(n)|| (kappa_n the condition number of
    Gamma(n) + lam I); the three modes of a sweep feed each other, so the test allows the sum
    over modes of those terms, times 2."""
    dims, rank, lam = (36, 30, 40), 4, 1e-3
    p = make_problem(dims, rank, workload=4, problem=11, noise=1e-2)
    planes, xv = stored(p, split)
    A = f32(p.init)
    Ad = dev_f(A)
    st = P.als_sweep(dev_x(planes, split), Ad, lam)
    assert int(st.item()) == 0
    ref = O.als_sweep(xv, A, lam)
    # the bound's ingredients, along the oracle's own sweep
    cur = [a.copy() for a in A]
    budget = 0.0
    for n in range(3):
        S = [c.T @ c for c in cur]
        G = np.ones((rank, rank))
        for m in range(3):
            if m != n:
                G = G * S[m]
        kappa = np.linalg.cond(G + lam * np.eye(rank))
        M = O.mttkrp(xv, cur, n)
        Mabs = O.mttkrp(np.abs(xv), [np.abs(c) for c in cur], n)
        budget += kappa * gamma(dims, n, split) * np.linalg.norm(Mabs) / np.linalg.norm(M)
        cur[n] = ref[n]
    for a, r in zip(Ad, ref):
        assert rel(a.double().cpu().numpy(), r) <= 2 * budget


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_precision_ladder_reaches_target():
    """The ladder bfloat16 -> split bfloat16 -> FP64 from a perturbed planted start reaches a
    residual target twice the noise level on the FP64 tensor; accepted steps on the lower rungs
    never raise the residual, and the run ends on a rung able to certify the target."""
    dims, rank, target = (40, 36, 32, 40), 16, 2e-3
    p = make_problem(dims, rank, workload=4, problem=31, kind="lognorm", noise=1e-3)
    rng = np.random.default_rng(4531)
    A0 = [b * (1.0 + 0.1 * rng.standard_normal(b.shape)) for b in p.planted]
    X64 = torch.tensor(p.x, device="cuda")
    X32 = X64.float()
    rungs = [P.to_bf16(X32), P.to_bf16(X32, split=True), X64]
    A, hist = P.gn_ladder_to_target(rungs, dev_f(A0), target, max_steps=40)
    num, den = O.residual(p.x, [a.double().cpu().numpy() for a in A])
    assert num / den <= target * (1 + 1e-9)
    assert hist[-1][0] in ("bf16x3", "torch.float64") and hist[-1][2]
    last = {}
    for name, r, ok in hist:
        if ok and name != "torch.float64" and name in last:
            assert r <= last[name]
        if ok:
            last[name] = r
