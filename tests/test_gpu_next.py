"""GPU tests of the layers above the kernels: the differentiable CP objective and the
mixed-precision Gauss-Newton driver. Each call goes through the C ABI of libcpgn.so and is
compared with the FP64 oracle (or with properties that hold at any size)."""
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


def dev(arrs, dt, grad=False):
    return [torch.tensor(a, dtype=dt, device="cuda", requires_grad=grad) for a in arrs]


# ------------------------------------------------------------------ differentiable objective
@pytest.mark.parametrize("dims,rank", [((12, 10, 8), 3), ((9, 7, 8, 6), 4), ((11, 13), 5)])
def test_objective_and_gradient_match_oracle(dims, rank):
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-1)
    X = dev([p.x], torch.float64)[0]
    A = dev(p.init, torch.float64, grad=True)
    f = P.cp_objective(X, A)
    f.backward()
    assert abs(float(f.detach()) - O.objective(p.x, p.init)) <= 1e-12 * O.objective(p.x, p.init)
    for a, g in zip(A, O.gradient(p.x, p.init)):
        assert rel(a.grad.cpu().numpy(), g) < 1e-12


def test_objective_gradcheck_fp64():
    """Finite differences of the library's own forward agree with its backward (12x10x8, R=3)."""
    p = make_problem((12, 10, 8), 3, workload=0, problem=3, noise=1e-1)
    X = dev([p.x], torch.float64)[0]
    A = tuple(dev(p.init, torch.float64, grad=True))
    assert torch.autograd.gradcheck(lambda *a: P.cp_objective(X, a), A, eps=1e-6, atol=1e-6,
                                    rtol=1e-6)


def test_objective_chain_rule_and_fp32():
    """A scalar multiple of f scales the gradient; FP32 against the oracle on rounded inputs."""
    p = make_problem((30, 25, 20), 6, workload=0, problem=6, noise=1e-2)
    xs = p.x.astype(np.float32).astype(np.float64)
    As = [a.astype(np.float32).astype(np.float64) for a in p.init]
    X = dev([p.x], torch.float32)[0]
    A = dev(p.init, torch.float32, grad=True)
    (3.0 * P.cp_objective(X, A)).backward()
    for a, g in zip(A, O.gradient(xs, As)):
        assert rel(a.grad.double().cpu().numpy(), 3.0 * g) < 1e-4


@pytest.mark.parametrize("dims,rank", [((12, 10, 8), 3), ((9, 7, 8, 6), 4), ((37, 29, 45), 20)])
def test_fused_objective_matches_oracle_and_direct_gradient(dims, rank):
    """method="fused" (cp_objective_gradient): the same gradient bits as the direct form's
    backward (the same kernels), and f by the expansion within its cancellation bound: the
    FP64 rounding of ||X||^2, 2 <M, A> and sum prod S, 64 u (||X||^2 + 2 |<M, A>| + sum prod S)
    in absolute terms, here with a residual of about 0.1 of ||X||."""
    p = make_problem(dims, rank, workload=0, problem=rank, noise=1e-1)
    X = dev([p.x], torch.float64)[0]
    A1 = dev(p.init, torch.float64, grad=True)
    A2 = dev(p.init, torch.float64, grad=True)
    f1 = P.cp_objective(X, A1, method="fused")
    f1.backward()
    P.cp_objective(X, A2).backward()
    for a, b in zip(A1, A2):
        assert torch.equal(a.grad, b.grad)
    ref = O.objective(p.x, p.init)
    M0 = O.mttkrp(p.x, p.init, 0)
    S = O.grams(p.init)
    had = np.ones_like(S[0])
    for sm in S:
        had = had * sm
    scale = float(np.sum(p.x * p.x)) + 2 * abs(float(np.sum(M0 * p.init[0]))) + abs(float(np.sum(had)))
    assert abs(float(f1.detach()) - ref) <= 0.5 * 64 * 2.0 ** -53 * scale


def test_fused_objective_gradcheck_fp64():
    p = make_problem((12, 10, 8), 3, workload=0, problem=3, noise=1e-1)
    X = dev([p.x], torch.float64)[0]
    A = tuple(dev(p.init, torch.float64, grad=True))
    assert torch.autograd.gradcheck(lambda *a: P.cp_objective(X, a, method="fused"), A, eps=1e-6,
                                    atol=1e-6, rtol=1e-6)


def test_objective_rejects_gradient_of_x():
    p = make_problem((6, 5, 4), 2, workload=0, problem=2)
    X = torch.tensor(p.x, dtype=torch.float64, device="cuda", requires_grad=True)
    A = dev(p.init, torch.float64, grad=True)
    f = P.cp_objective(X, A)
    with pytest.raises(RuntimeError):
        f.backward()


# ------------------------------------------------------------------ mixed-precision driver
def test_mixed_precision_driver_reaches_target_below_fp32_floor():
    """Workload 1 (40^3, R=5, exact): FP32 steps until the FP32 residual is <= 1e-6, then FP64
    steps to 1e-10, which FP32 storage alone cannot reach."""
    p = make_problem((40, 40, 40), 5, workload=1)
    X64 = torch.tensor(p.x, device="cuda")
    X32 = X64.float()
    A = dev(p.init, torch.float32)
    Af, hist = P.gn_mixed_to_target(X32, X64, A, 1e-10, 1e-6)
    kinds = [k for k, _ in hist]
    assert kinds[0] == "torch.float32" and kinds[-1] == "torch.float64"
    assert kinds == sorted(kinds, key=lambda k: k != "torch.float32")   # one switch
    assert hist[-1][1] <= 1e-10
    assert all(a.dtype == torch.float64 for a in Af)
    # the final residual is the oracle's for the returned factors
    num, den = O.residual(p.x, [a.cpu().numpy() for a in Af])
    assert abs(num / den - hist[-1][1]) <= 1e-13 + 1e-6 * num / den


def test_gn_to_target_matches_oracle_step_count():
    p = make_problem((40, 40, 40), 5, workload=1)
    X = torch.tensor(p.x, device="cuda")
    opt, hist = P.gn_to_target(X, dev(p.init, torch.float64), 1e-10)
    _, ohist, _ = O.gn(p.x, p.init, O.LambdaSchedule(1e-4, 1e-10, 1e-4, 2.0), 1e-3, 20, 1e-10, 200)
    assert hist[-1] <= 1e-10
    assert abs(len(hist) - len(ohist)) <= 3


# ------------------------------------------------------------------ batched problems (workload 5)
def test_batched_streams_match_single_stream_runs():
    """Problems advanced on three streams end bitwise where sequential single-stream runs end,
    and each first step matches the oracle."""
    from workloads import batched_problems
    probs = batched_problems(5)
    devs = [(torch.tensor(p.x, dtype=torch.float32, device="cuda"),
             [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]) for p in probs]
    seq = []
    for X, A in devs:
        A2 = [a.clone() for a in A]
        g = P.GaussNewton(X, A2)
        for _ in range(2):
            g.step()
        seq.append(A2)
    torch.cuda.synchronize()
    b = P.BatchedGaussNewton(devs, n_streams=3)
    b.step()
    b.synchronize()
    # first step against the oracle on the FP32-rounded inputs
    for p, opt in zip(probs[:2], b.opts[:2]):
        xs = p.x.astype(np.float32).astype(np.float64)
        As = [a.astype(np.float32).astype(np.float64) for a in p.init]
        its = opt.stats()["cg_iters"]   # same iteration count, so no tie at the stop threshold
        ref, _ = O.gn_step(xs, As, 1e-4, 0.0, its)
        for a, r in zip(opt.A, ref):
            assert rel(a.double().cpu().numpy(), r) < 1e-4
    ev = b.step(timed=True)
    b.synchronize()
    assert len(ev) == len(probs) and all(e0.elapsed_time(e1) > 0 for e0, e1 in ev)
    for opt, A2 in zip(b.opts, seq):
        for a, a2 in zip(opt.A, A2):
            assert torch.equal(a, a2)


def test_device_timestamps_bracket_batched_steps():
    """cp_device_timestamp around each problem's step on its stream: the clock rate is positive,
    every step's end stamp is after its start, the stamps of problems on one stream are ordered
    as the steps were enqueued, each step's device duration is no longer than the HIP-event time
    around the same step (plus 20 us for the stamp kernels), and the stamped run ends where an
    unstamped one does."""
    from workloads import batched_problems
    probs = batched_problems(4)
    mk = lambda: [(torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                   [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]) for p in probs]
    hz = P.device_clock_hz()
    assert hz > 0
    plain = P.BatchedGaussNewton(mk(), n_streams=2)
    b = P.BatchedGaussNewton(mk(), n_streams=2)
    stamps = torch.zeros(2 * len(probs), dtype=torch.int64, device="cuda")
    plain.step()
    ev = b.step(timed=True, stamps=stamps)
    plain.synchronize()
    b.synchronize()
    t = stamps.view(len(probs), 2).cpu().numpy()
    assert (t[:, 1] > t[:, 0]).all()
    for i in range(2, len(probs)):   # problems i - 2 and i share a stream
        assert t[i, 0] >= t[i - 2, 1]
    for (e0, e1), (s0, s1) in zip(ev, t):
        dev_ms = (s1 - s0) / hz * 1e3
        assert 0.0 < dev_ms <= e0.elapsed_time(e1) + 0.02
    for op, ob in zip(plain.opts, b.opts):
        for a, c in zip(op.A, ob.A):
            assert torch.equal(a, c)


def test_batched_cg_steps_match_per_problem_steps():
    """Steps split in begin / batched CG / end (cp_gn_step_begin, cp_gn_cg_batch, cp_gn_step_end)
    give bitwise the factors and stats of each problem's own cp_gn_step over three steps, for
    uneven problems (modes 60..200, ranks 8..64, so the batch runs with the largest rank's column
    blocks), and the first step matches the oracle."""
    from workloads import batched_problems
    probs = batched_problems(6)
    mk = lambda: [(torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                   [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]) for p in probs]
    ref = [P.GaussNewton(X, A) for X, A in mk()]
    bat = P.BatchedGaussNewton(mk(), n_streams=3, batch_cg=True)
    for k in range(3):
        for g in ref:
            g.step()
        bat.step()
        bat.synchronize()
        torch.cuda.synchronize()
        for g, ob in zip(ref, bat.opts):
            assert g.stats() == ob.stats(), k
            for a, b in zip(g.A, ob.A):
                assert torch.equal(a, b), k
        if k == 0:
            for p, ob in zip(probs[:2], bat.opts[:2]):
                xs = p.x.astype(np.float32).astype(np.float64)
                As = [a.astype(np.float32).astype(np.float64) for a in p.init]
                its = ob.stats()["cg_iters"]
                r, _ = O.gn_step(xs, As, 1e-4, 0.0, its)
                for a, b in zip(ob.A, r):
                    assert rel(a.double().cpu().numpy(), b) < 1e-4


def test_batched_cg_single_problem_matches_gn_step_fp64():
    """One FP64 problem through begin / batch of one / end equals cp_gn_step bitwise (factors and
    stats), with the host damping and with the device damping."""
    p = make_problem((30, 25, 20), 7, workload=1, problem=3)
    X = torch.tensor(p.x, device="cuda")
    for devlam in (False, True):
        A1 = [torch.tensor(a, device="cuda") for a in p.init]
        A2 = [a.clone() for a in A1]
        s1 = P.gn_step(X, A1, 3e-3, 1e-3, 20)
        if devlam:
            lam = torch.tensor([3e-3], dtype=torch.float64, device="cuda")
            st = P.gn_step_begin(X, A2, lam_dev=lam, cg_tol=1e-3, cg_maxiter=20)
        else:
            st = P.gn_step_begin(X, A2, lam=3e-3, cg_tol=1e-3, cg_maxiter=20)
        P.gn_cg_batch([st], 20)
        s2 = P.gn_step_end(st)
        torch.cuda.synchronize()
        assert P.read_stats(s1) == P.read_stats(s2)
        for a, b in zip(A1, A2):
            assert torch.equal(a, b)


def test_batched_cg_graph_replays_match_eager():
    """The whole batched step captured as one graph (all streams) and replayed three times, with
    eager work between replays, gives bitwise the eager batched iterates and schedules."""
    from workloads import batched_problems
    probs = batched_problems(5)
    mk = lambda: [(torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                   [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]) for p in probs]
    eager = P.BatchedGaussNewton(mk(), n_streams=2, batch_cg=True)
    graph = P.BatchedGaussNewton(mk(), n_streams=2, batch_cg=True, graphs=True)
    for k in range(3):
        eager.step()
        eager.synchronize()
        graph.step()
        graph.synchronize()
        _ = graph.residuals()
        torch.cuda.synchronize()
        for oe, og in zip(eager.opts, graph.opts):
            assert og.schedule.value == oe.schedule.value
            for a, b in zip(oe.A, og.A):
                assert torch.equal(a, b), k


@pytest.mark.parametrize("dt", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batch_program_steps_match_per_problem_steps(dt):
    """The batch program (cp_gn_batch_create / cp_gn_batch_step: every part of the step in shared
    launches) gives bitwise the factors, stats and device damping schedules of each problem's own
    cp_gn_step over three steps, for uneven problems (modes 60..200 with and without vector
    loads, ranks 8..64), and the first step matches the oracle."""
    from workloads import batched_problems
    probs = batched_problems(7)
    mk = lambda: [(torch.tensor(p.x, dtype=dt, device="cuda"),
                   [torch.tensor(a, dtype=dt, device="cuda") for a in p.init]) for p in probs]
    ref = [P.GaussNewton(X, A) for X, A in mk()]
    bat = P.BatchedGaussNewton(mk(), fused=True)
    assert bat.program is not None
    for k in range(3):
        for g in ref:
            g.step()
        bat.step()
        bat.synchronize()
        torch.cuda.synchronize()
        for g, ob in zip(ref, bat.opts):
            assert g.stats() == ob.stats(), k
            assert ob.schedule.value == g.schedule.value, k
            for a, b in zip(g.A, ob.A):
                assert torch.equal(a, b), k
        if k == 0:
            for p, ob in zip(probs[:2], bat.opts[:2]):
                xs = p.x.astype(np.float32).astype(np.float64) if dt == torch.float32 else p.x
                As = [a.astype(np.float32).astype(np.float64) if dt == torch.float32 else a
                      for a in p.init]
                r, _ = O.gn_step(xs, As, 1e-4, 0.0, ob.stats()["cg_iters"])
                for a, b in zip(ob.A, r):
                    assert rel(a.double().cpu().numpy(), b) < (1e-4 if dt == torch.float32 else 1e-9)


def test_batched_runs_under_tile_shape_match_single_problem_runs():
    """Batch runners given an MTTKRP tile shape (the batch program replayed from one graph, and
    eager steps on three streams) give bitwise the factors and stats of each problem's own steps
    under the same shape (api.tiles), the first step matches the oracle, and the calling thread's
    shape is the default again outside the runners."""
    from workloads import batched_problems
    probs = batched_problems(5)
    T = P.Tiles(8, 4, 2)
    mk = lambda: [(torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                   [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init])
                  for p in probs]
    with P.tiles(T):
        ref = [P.GaussNewton(X, A) for X, A in mk()]
    bat = P.BatchedGaussNewton(mk(), fused=True, graphs=True, tiles=T)
    eag = P.BatchedGaussNewton(mk(), n_streams=3, tiles=T)
    assert P.get_tiles() == P.Tiles()
    for k in range(3):
        with P.tiles(T):
            for g in ref:
                g.step()
        bat.step()
        eag.step()
        bat.synchronize()
        eag.synchronize()
        torch.cuda.synchronize()
        assert P.get_tiles() == P.Tiles()
        for g, ob, oe in zip(ref, bat.opts, eag.opts):
            assert g.stats() == ob.stats() == oe.stats(), k
            for a, b, c in zip(g.A, ob.A, oe.A):
                assert torch.equal(a, b) and torch.equal(a, c), k
        if k == 0:
            for p, ob in zip(probs[:2], bat.opts[:2]):
                xs = p.x.astype(np.float32).astype(np.float64)
                As = [a.astype(np.float32).astype(np.float64) for a in p.init]
                r, _ = O.gn_step(xs, As, 1e-4, 0.0, ob.stats()["cg_iters"])
                for a, b in zip(ob.A, r):
                    assert rel(a.double().cpu().numpy(), b) < 1e-4


def test_batch_program_mixed_orders_dtypes_diagonal_damping():
    """One batch program over problems of orders 3 and 4, FP32 and FP64, ranks 5 to 40, with the
    diagonal damping: the launches of different kernel instantiations share levels, and every
    problem still gives bitwise the factors and stats of its own steps (two steps)."""
    rng = np.random.default_rng(11)
    shapes = [((23, 19, 31), 5, torch.float32), ((12, 9, 11, 8), 7, torch.float64),
              ((40, 36, 20), 40, torch.float64), ((10, 13, 8, 9), 12, torch.float32),
              ((64, 30, 17), 20, torch.float32), ((25, 25, 25), 33, torch.float64)]
    data = [(rng.standard_normal(sh), [rng.standard_normal((n, R)) for n in sh], dt)
            for sh, R, dt in shapes]
    mk = lambda: [(torch.tensor(x, dtype=dt, device="cuda"),
                   [torch.tensor(a, dtype=dt, device="cuda") for a in A]) for x, A, dt in data]
    cfg = P.GNConfig(cg_tol=1e-3, cg_maxiter=20, damping="diagonal")
    ref = [P.GaussNewton(X, A, cfg) for X, A in mk()]
    bat = P.BatchedGaussNewton(mk(), cfg, fused=True)
    for k in range(2):
        for g in ref:
            g.step()
        bat.step()
        bat.synchronize()
        torch.cuda.synchronize()
        for g, ob in zip(ref, bat.opts):
            assert g.stats() == ob.stats(), k
            for a, b in zip(g.A, ob.A):
                assert torch.equal(a, b), k


def test_batch_program_graph_replays_match_eager():
    """The batch program captured as one graph and replayed three times, with eager work between
    the replays, gives bitwise the eager program's iterates and schedules."""
    from workloads import batched_problems
    probs = batched_problems(5)
    mk = lambda: [(torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                   [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]) for p in probs]
    eager = P.BatchedGaussNewton(mk(), fused=True)
    graph = P.BatchedGaussNewton(mk(), fused=True, graphs=True)
    for k in range(3):
        eager.step()
        eager.synchronize()
        graph.step()
        graph.synchronize()
        _ = graph.residuals()
        torch.cuda.synchronize()
        for oe, og in zip(eager.opts, graph.opts):
            assert og.schedule.value == oe.schedule.value
            assert og.stats() == oe.stats()
            for a, b in zip(oe.A, og.A):
                assert torch.equal(a, b), k


def test_batch_program_many_problems_split_into_groups():
    """More problems than one batched launch holds (130 > 128 members): the program splits its
    launches and the CG batches, and every problem still matches its own step bitwise."""
    rng = np.random.default_rng(5)
    shapes = [(6 + i % 5, 5 + i % 3, 7 + i % 4) for i in range(130)]
    data = [(rng.standard_normal(sh), [rng.standard_normal((n, 3)) for n in sh]) for sh in shapes]
    mk = lambda: [(torch.tensor(x, dtype=torch.float64, device="cuda"),
                   [torch.tensor(a, dtype=torch.float64, device="cuda") for a in A]) for x, A in data]
    ref = [P.GaussNewton(X, A) for X, A in mk()]
    bat = P.BatchedGaussNewton(mk(), fused=True)
    for g in ref:
        g.step()
    bat.step()
    bat.synchronize()
    torch.cuda.synchronize()
    for g, ob in zip(ref, bat.opts):
        assert g.stats() == ob.stats()
        for a, b in zip(g.A, ob.A):
            assert torch.equal(a, b)


# ------------------------------------------------------------------ graph-replayable steps
def test_device_damping_schedule_matches_host():
    """cp_damping_advance gives bitwise the host schedule's sequence (both directions)."""
    sched = P.DampingSchedule(1e-4, 1e-10, 1e-4, 2.0)
    state = sched.to_device("cuda")
    for _ in range(90):
        P.damping_advance(state)
        sched.advance()
        v = state.cpu().tolist()
        assert v[0] == sched.value and (v[4] != 0.0) == sched.decreasing


def test_gn_step_devlam_matches_gn_step():
    p = make_problem((30, 26, 22), 6, workload=0, problem=6, noise=1e-2)
    X = torch.tensor(p.x, device="cuda")
    A1, A2 = dev(p.init, torch.float64), dev(p.init, torch.float64)
    for lam, damping in ((1e-3, "identity"), (2.5e-4, "diagonal")):
        P.gn_step(X, A1, lam, 1e-3, 20, damping=damping)
        P.gn_step_devlam(X, A2, torch.tensor([lam], dtype=torch.float64, device="cuda"), 1e-3, 20,
                         damping=damping)
        for a, b in zip(A1, A2):
            assert torch.equal(a, b)


def test_gn_step_devlam_rejects_negative_lambda_on_device():
    p = make_problem((12, 10, 8), 3, workload=0, problem=3, noise=1e-2)
    X = torch.tensor(p.x, device="cuda")
    A = dev(p.init, torch.float64)
    st = P.gn_step_devlam(X, A, torch.tensor([-1.0], dtype=torch.float64, device="cuda"))
    assert P.read_stats(st)["status"] == -1   # CP_EINVAL
    for a, a0 in zip(A, p.init):
        assert np.array_equal(a.cpu().numpy(), a0)


def test_batched_graph_replays_match_eager_steps():
    """Each problem's captured step (GN step + device damping update) replayed three times, with
    eager work and synchronisations between replays, gives bitwise the eager batched iterates."""
    from workloads import batched_problems
    probs = batched_problems(5)
    mk = lambda: [(torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                   [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]) for p in probs]
    eager = P.BatchedGaussNewton(mk(), n_streams=3)
    graph = P.BatchedGaussNewton(mk(), n_streams=3, graphs=True)
    for k in range(3):
        eager.step()
        eager.synchronize()
        graph.step()
        graph.synchronize()
        _ = graph.residuals()          # eager library work on the same streams between replays
        torch.cuda.synchronize()
        for oe, og in zip(eager.opts, graph.opts):
            assert og.schedule.value == oe.schedule.value
            for a, b in zip(oe.A, og.A):
                assert torch.equal(a, b), k


def test_autotuned_batched_run_matches_single_stream():
    """The autotuner leaves the caller's factors untouched, picks one of the candidates, and the
    tuned runner gives the single-stream eager iterates bit for bit."""
    rng = np.random.default_rng(3)
    probs = []
    for i in range(6):
        dims, R = tuple(int(v) for v in rng.integers(20, 60, 3)), int(rng.choice([4, 8, 16]))
        p = make_problem(dims, R, workload=5, problem=i, noise=1e-3)
        probs.append((torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                      [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]))
    before = [[a.clone() for a in A] for _, A in probs]
    cfg = P.GNConfig(cg_tol=1e-3, cg_maxiter=20)
    tune = P.autotune_batched(probs, cfg, stream_counts=(1, 4), steps=2, cache={})
    key = (tune.n_streams, tune.graphs, tune.batch_cg, tune.fused)
    assert key in tune.table and len(tune.table) == 10
    # the tile sweep: the default and 8 shapes, one field at a time
    assert len(tune.tile_table) == 9 and P.Tiles() in tune.tile_table
    assert tune.tiles is None or tune.tiles in tune.tile_table
    assert P.get_tiles() == P.Tiles()
    for (_, A), B in zip(probs, before):
        assert all(torch.equal(a, b) for a, b in zip(A, B))
    tuned = [(X, [a.clone() for a in A]) for X, A in probs]
    bgn = P.BatchedGaussNewton(tuned, cfg, n_streams=tune.n_streams, graphs=tune.graphs,
                               batch_cg=tune.batch_cg, fused=tune.fused, tiles=tune.tiles)
    for _ in range(3):
        bgn.step()
    bgn.synchronize()
    for (X, A), (_, At) in zip(probs, tuned):
        ref = [a.clone() for a in A]
        with P.tiles(tune.tiles):
            opt = P.GaussNewton(X, ref, P.GNConfig(cg_tol=1e-3, cg_maxiter=20))
            for _ in range(3):
                opt.step()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(At, ref))


def test_batched_graph_replays_with_cholesky_preconditioner_match_eager():
    """Graph replay of the step with the triangular-solve preconditioner (its solve kernel holds
    130 KB of LDS) gives the eager iterates bit for bit."""
    probs = []
    for i, (dims, R) in enumerate([((40, 36, 44), 8), ((70, 50, 66), 16)]):
        p = make_problem(dims, R, workload=5, problem=10 + i, noise=1e-3)
        probs.append((torch.tensor(p.x, dtype=torch.float32, device="cuda"),
                      [torch.tensor(a, dtype=torch.float32, device="cuda") for a in p.init]))
    cfg = P.GNConfig(cg_tol=1e-3, cg_maxiter=20, preconditioner="cholesky")
    runs = []
    for graphs in (False, True):
        cur = [(X, [a.clone() for a in A]) for X, A in probs]
        bgn = P.BatchedGaussNewton(cur, cfg, n_streams=2, graphs=graphs)
        for _ in range(3):
            bgn.step()
            bgn.synchronize()
            torch.cuda.synchronize()
        runs.append(cur)
    for (_, Ae), (_, Ag) in zip(*runs):
        assert all(torch.equal(a, b) for a, b in zip(Ae, Ag))


@pytest.mark.parametrize("variant", ["cholesky", "armijo"])
def test_gn_to_target_with_variants(variant):
    """A full run to 1e-10 with the triangular-solve preconditioner (the same iterates up to
    rounding: the plain run's number of steps to within 2), or with Armijo control (the residual
    never rises; from this start it avoids the plain run's overshoots and needs 14 steps
    instead of 21)."""
    p = make_problem((40, 40, 40), 5, workload=1)
    X = torch.tensor(p.x, device="cuda")
    runs = {}
    for name in ("plain", variant):
        A = [torch.tensor(a, device="cuda") for a in p.init]
        cfg = P.GNConfig(cg_tol=1e-3, cg_maxiter=20,
                         preconditioner="cholesky" if name == "cholesky" else "inverse",
                         line_search=P.Armijo() if name == "armijo" else None)
        opt, hist = P.gn_to_target(X, A, 1e-10, cfg, max_steps=200)
        assert hist[-1] <= 1e-10 and opt.stats()["status"] == 0
        if name == "armijo":   # every accepted Armijo step lowers f, so the residual falls
            assert all(b <= a * (1 + 1e-9) for a, b in zip(hist, hist[1:]))
        runs[name] = len(hist)
    if variant == "cholesky":
        assert abs(runs[variant] - runs["plain"]) <= 2
