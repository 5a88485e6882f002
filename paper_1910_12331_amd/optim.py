"""Optimizer objects with a step() member, as the paper structures its ALS and Gauss-Newton
drivers (Section 4): each step() is one ALS sweep or one Gauss-Newton iteration, executed by
libcpgn.so on the GPU."""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field, replace

import torch

from . import api


class DampingSchedule:
    """Varying Tikhonov damping of Section 3.2: begin at the upper threshold, divide by mu after
    every step until the lower threshold is reached, then multiply by mu until the upper one is
    reached again, and so on. `value` is the damping for the coming step."""

    def __init__(self, start=1e-4, lower=1e-10, upper=1e-4, mu=2.0):
        if not (mu > 1.0 and 0.0 < lower <= upper):
            raise ValueError("need mu > 1 and 0 < lower <= upper")
        self.value, self.lower, self.upper, self.mu = float(start), float(lower), float(upper), float(mu)
        self.decreasing = True

    def advance(self) -> float:
        if self.decreasing:
            self.value = self.value / self.mu
            if self.value <= self.lower:
                self.decreasing = False
        else:
            self.value = self.value * self.mu
            if self.value >= self.upper:
                self.decreasing = True
        return self.value

    def state_dict(self):
        return dict(value=self.value, lower=self.lower, upper=self.upper, mu=self.mu,
                    decreasing=self.decreasing)

    def to_device(self, device) -> torch.Tensor:
        """The state as the float64[5] device array that cp_damping_advance advances."""
        return torch.tensor([self.value, self.lower, self.upper, self.mu,
                             1.0 if self.decreasing else 0.0], dtype=torch.float64, device=device)

    def load_device(self, state):
        """Take the state back from its device array (or from the same five values on the
        host)."""
        v = state.cpu().tolist() if isinstance(state, torch.Tensor) else list(state)
        self.value, self.lower, self.upper, self.mu = v[0], v[1], v[2], v[3]
        self.decreasing = v[4] != 0.0

    def load_state_dict(self, d):
        self.value, self.lower, self.upper, self.mu = d["value"], d["lower"], d["upper"], d["mu"]
        self.decreasing = d["decreasing"]


class ConstantDamping:
    """A fixed damping lambda (Section 5 runs Gauss-Newton with Armijo's condition at a constant
    lambda); the same interface as DampingSchedule."""

    def __init__(self, value: float):
        if not value >= 0.0:
            raise ValueError("need lambda >= 0")
        self.value = float(value)

    def advance(self) -> float:
        return self.value

    def state_dict(self):
        return dict(value=self.value)

    def load_state_dict(self, d):
        self.value = d["value"]


@dataclass
class Armijo:
    """Armijo step-size control (Section 5): step sizes 1, shrink, shrink^2, ... (at most
    max_trials) until f(A + alpha V) <= f(A) + c alpha <G, V>. With max_trials = 1 this is the
    accept-or-reject rule of a damped Gauss-Newton iteration: a step that does not decrease f
    enough leaves the factors as they were.

    carry_objective: after the first step, f at the current point is the one the previous
    search evaluated (the optimizer is the only writer of its factors), so each step costs one
    residual pass per trial and none at the start."""
    c: float = 1e-4
    shrink: float = 0.5
    max_trials: int = 10
    carry_objective: bool = True


def Acceptance(c: float = 1e-4) -> Armijo:
    """The full Gauss-Newton step, taken only if f(A + V) <= f(A) + c <G, V> (one trial)."""
    return Armijo(c=c, shrink=0.5, max_trials=1, carry_objective=True)


@dataclass
class GNConfig:
    cg_tol: float = 1e-3
    cg_maxiter: int = 20
    schedule: DampingSchedule | ConstantDamping | None = None
    damping: str = "identity"       # or "diagonal": lam diag(J^T J) (Section 3.2)
    line_search: Armijo | None = None
    preconditioner: str = "inverse"  # or "cholesky": triangular solves (Section 3.3), R <= 128


class GaussNewton:
    """Algorithm 1 (CP-GN). Factors are updated in place on the device."""

    def __init__(self, X: torch.Tensor, A, config: GNConfig | None = None):
        self.X, self.A = X, list(A)
        self.cfg = config or GNConfig()
        self.schedule = self.cfg.schedule or DampingSchedule()
        self.ws = api.Workspace()
        self.stats_buf = api.stats_buffer(X.device)
        self.ls_buf = api.armijo_stats_buffer(X.device) if self.cfg.line_search else None
        self.steps = 0
        self._f_known = False    # ls_buf holds f at the current factors

    def reset_objective(self):
        """Call after changing the factors outside step(): the next search evaluates f anew."""
        self._f_known = False

    def step(self) -> torch.Tensor:
        ls = self.cfg.line_search
        if ls is None:
            api.gn_step(self.X, self.A, self.schedule.value, self.cfg.cg_tol, self.cfg.cg_maxiter,
                        stats=self.stats_buf, ws=self.ws, damping=self.cfg.damping,
                        preconditioner=self.cfg.preconditioner)
        else:
            api.gn_step_armijo(self.X, self.A, self.schedule.value, self.cfg.cg_tol,
                               self.cfg.cg_maxiter, ls.c, ls.shrink, ls.max_trials,
                               stats=self.stats_buf, ls_stats=self.ls_buf, ws=self.ws,
                               damping=self.cfg.damping, preconditioner=self.cfg.preconditioner,
                               f0_given=ls.carry_objective and self._f_known)
            self._f_known = True
        self.schedule.advance()
        self.steps += 1
        return self.stats_buf

    def stats(self) -> dict:
        out = api.read_stats(self.stats_buf)
        if self.ls_buf is not None:
            out.update({"ls_" + k: v for k, v in api.read_armijo_stats(self.ls_buf).items()})
        return out

    def residual(self) -> float:
        """Direct relative residual ||X - [[A]]|| / ||X|| at the current factors. After an Armijo
        step it is read from the search's own evaluation at the returned point (the same direct
        residual kernel), without another pass over X."""
        if self.ls_buf is not None and self._f_known:
            s = api.read_armijo_stats(self.ls_buf)
            return math.sqrt(2.0 * max(s["f"], 0.0)) / s["x_norm"]
        r = api.residual(self.X, self.A, ws=self.ws).cpu()
        return float(r[0] / r[1])


class StepDecay:
    """A regularization that starts at `start` and is multiplied by `factor` after every `every`
    sweeps: Section 5 runs ALS on the matrix-multiplication tensors with lambda = 0.01 halved
    every 100 iterations. `value` is the lambda for the coming sweep."""

    def __init__(self, start: float = 1e-2, factor: float = 0.5, every: int = 100):
        if not (start >= 0.0 and 0.0 < factor and every >= 1):
            raise ValueError("need start >= 0, factor > 0 and every >= 1")
        self.value, self.factor, self.every, self.count = float(start), float(factor), int(every), 0

    def advance(self) -> float:
        self.count += 1
        if self.count % self.every == 0:
            self.value = self.value * self.factor
        return self.value


class ALS:
    """Alternating least squares sweeps (Section 2.2), with a fixed Tikhonov lambda or a
    schedule with `value` and `advance()` (e.g. StepDecay)."""

    def __init__(self, X: torch.Tensor, A, lam: float = 0.0, schedule=None):
        self.X, self.A, self.lam = X, list(A), float(lam)
        self.schedule = schedule
        self.ws = api.Workspace()
        self.status = torch.zeros(1, dtype=torch.int32, device=X.device)
        self.steps = 0

    def step(self) -> torch.Tensor:
        lam = self.schedule.value if self.schedule is not None else self.lam
        api.als_sweep(self.X, self.A, lam, status=self.status, ws=self.ws)
        if self.schedule is not None:
            self.schedule.advance()
        self.steps += 1
        return self.status

    def residual(self) -> float:
        r = api.residual(self.X, self.A, ws=self.ws).cpu()
        return float(r[0] / r[1])


def gn_to_target(X, A, target, config: GNConfig | None = None, max_steps: int = 300):
    """Gauss-Newton steps on (X, A) until the direct relative residual is <= target or
    max_steps steps were taken. The residual is read after every step (one host
    synchronisation per step). Returns (optimizer, list of per-step residuals)."""
    opt = GaussNewton(X, A, config)
    hist = []
    while opt.steps < max_steps:
        opt.step()
        hist.append(opt.residual())
        if hist[-1] <= target:
            break
    return opt, hist


def gn_mixed_to_target(X_low, X_high, A, target, switch_residual: float = 1e-6,
                       config: GNConfig | None = None, max_steps: int = 300):
    """Mixed-precision Gauss-Newton run to a residual target below the low precision's floor.

    Steps run on X_low (e.g. FP32 storage, half the bytes and twice the matrix-core rate of
    FP64) until its relative residual is <= switch_residual, or stops halving once below 1e-4
    (the storage rounding floor is near); the factors are then cast to X_high's precision and
    the same damping schedule continues on X_high until the residual is <= target. X_low and
    X_high hold the same tensor. Returns (factors, history of (precision, residual))."""
    cfg = config or GNConfig()
    sched = cfg.schedule or DampingSchedule()
    low_cfg = replace(cfg, schedule=sched)
    opt = GaussNewton(X_low, A, low_cfg)
    hist = []
    prev = float("inf")
    while opt.steps < max_steps:
        opt.step()
        r = opt.residual()
        hist.append((str(X_low.dtype), r))
        if r <= target or r <= switch_residual or (r < 1e-4 and r > 0.5 * prev):
            break
        prev = r
    if hist and hist[-1][1] <= target:
        return opt.A, hist
    A_high = [a.to(api.factor_dtype(X_high)) for a in opt.A]
    high = GaussNewton(X_high, A_high, replace(cfg, schedule=sched))
    while opt.steps + high.steps < max_steps:
        high.step()
        r = high.residual()
        hist.append((str(X_high.dtype), r))
        if r <= target:
            break
    return high.A, hist


# Relative residual at which each storage form is taken to be at its rounding floor: about the
# relative accuracy of its MTTKRP (bfloat16 3e-3, split bfloat16 5e-6, FP32 5e-7 measured at
# 80^4), times a margin; FP64 has none.
_RUNG_FLOOR = {"bf16": 1e-2, "bf16x3": 3e-5, "torch.float32": 1e-6, "torch.float64": 0.0}


def _rung_name(X) -> str:
    if isinstance(X, api.SplitBF16Tensor):
        return "bf16x3"
    if X.dtype == torch.bfloat16:
        return "bf16"
    return str(X.dtype)


def gn_ladder_to_target(rungs, A, target, config: GNConfig | None = None, max_steps: int = 300):
    """Gauss-Newton over a ladder of storage precisions of one tensor, lowest first (e.g. a
    bfloat16 tensor, its split form, FP64). One damping schedule runs through all rungs.

    After each step the direct residual is read on the current rung. A step that raises it is
    rejected (factors and damping state restored) and the run moves up a rung; so does an accepted
    step whose residual is below the rung's floor (_RUNG_FLOOR), or above half the previous one
    while within 100x of that floor. A lower rung ends the run only if its floor is at most a tenth
    of the target (its residual, measured on its own rounded tensor, then certifies the target).
    The top rung takes every step until the residual is <= target or max_steps steps were taken.
    Returns (factors, history of (rung, residual, accepted))."""
    cfg = config or GNConfig()
    sched = cfg.schedule or DampingSchedule()
    A = list(A)
    hist = []
    steps = 0
    prev = float("inf")
    for i, X in enumerate(rungs):
        top = i == len(rungs) - 1
        name = _rung_name(X)
        floor = _RUNG_FLOOR.get(name, 0.0)
        A = [a.to(api.factor_dtype(X)) for a in A]
        opt = GaussNewton(X, A, replace(cfg, schedule=sched))
        if i > 0:
            prev = opt.residual()
        while steps < max_steps:
            keep = [a.clone() for a in opt.A]
            state = sched.state_dict()
            opt.step()
            steps += 1
            r = opt.residual()
            if not top and not (r <= prev):      # rejected (also catches NaN)
                for a, k in zip(opt.A, keep):
                    a.copy_(k)
                sched.load_state_dict(state)
                hist.append((name, r, False))
                break
            hist.append((name, r, True))
            if r <= target and (top or floor <= 0.1 * target):
                return opt.A, hist
            if r <= target:          # this rung cannot certify the target: move up
                prev = r
                break
            if not top and (r <= floor or (r > 0.5 * prev and r < 100.0 * floor)):
                prev = r
                break
            prev = r
        A = opt.A
        if steps >= max_steps:
            break
    return A, hist


class BatchedGaussNewton:
    """Independent Gauss-Newton decompositions advanced together (many random restarts or
    many small tensors). Problem i runs on HIP stream i % n_streams with its own workspace and
    damping schedule, so small problems overlap on the GPU; each problem's iterates are the ones
    a single-stream run produces (the kernels are deterministic). All streams have the default
    priority.

    With graphs=True one Gauss-Newton step of each problem, together with its damping update
    (read and advanced on the device), is captured once as a HIP graph and replayed per step: the
    host then issues one graph launch per problem instead of every kernel launch of the step.

    With batch_cg=True the CG iterations of all problems share launches (cp_gn_cg_batch): each
    problem's step begins on its stream (gradient and preconditioner), the streams join, CG runs
    for the whole batch on the current stream (three launches per iteration instead of three per
    iteration and problem), and the streams fork again for the updates. The iterates are bitwise
    those of the per-problem steps. With graphs=True as well, the whole batch step (all streams)
    is captured as one graph.

    With fused=True (implies batch_cg) every part of the step shares launches: a batch program
    (api.GNBatchProgram, cp_gn_batch_create) records each problem's launches before and after CG
    once, and a step runs one launch per kernel and position in the step for all problems, on
    the current stream, with the damping schedules advanced on the device. Same iterates again;
    with graphs=True the program's launches are captured as one graph.

    tiles (api.Tiles) sets the MTTKRP tile shape of every launch the runner makes (workspaces,
    eager steps, captured graphs and the batch program); the iterates then agree with the
    default shape's to rounding, and bitwise with single-problem runs under the same shape."""

    def __init__(self, problems, config: GNConfig | None = None, n_streams: int = 8,
                 graphs: bool = False, batch_cg: bool = False, fused: bool = False,
                 tiles: api.Tiles | None = None):
        self.tiles = tiles
        with api.tiles(tiles):
            self._init(problems, config, n_streams, graphs, batch_cg, fused)

    def _init(self, problems, config, n_streams, graphs, batch_cg, fused):
        cfg = config or GNConfig()
        if graphs and cfg.line_search is not None:
            raise ValueError("graph replay covers the plain Gauss-Newton step only")
        batch_cg = batch_cg or fused
        if batch_cg and (cfg.line_search is not None or cfg.preconditioner != "inverse"):
            raise ValueError("batched CG covers the plain step with the explicit inverse")
        self.batch_cg = batch_cg
        self.fused = fused
        self.program = None
        self.cfg = cfg
        torch.cuda.current_stream().synchronize()   # inputs were written on the current stream
        self.streams = [torch.cuda.Stream() for _ in range(max(1, n_streams))]
        self.opts = []
        for i, (X, A) in enumerate(problems):
            with torch.cuda.stream(self.streams[i % len(self.streams)]):
                self.opts.append(GaussNewton(X, A, replace(cfg, schedule=None)))
        self.graphs = None
        self.batch_graph = None
        if fused:
            self._build_program(graphs)
        elif graphs and batch_cg:
            self._capture_batch()
        elif graphs:
            self._capture()

    def _device_states(self):
        """The problems' damping states as rows of one device array (one copy reads them all)."""
        self.lam_all = torch.stack([opt.schedule.to_device(opt.X.device) for opt in self.opts])
        self.lam_state = [self.lam_all[i] for i in range(len(self.opts))]

    def _build_program(self, graphs: bool):
        self._device_states()
        torch.cuda.synchronize()
        self.program = api.GNBatchProgram(
            [(opt.X, opt.A, opt.ws, opt.stats_buf, st) for opt, st in zip(self.opts, self.lam_state)],
            cg_tol=self.cfg.cg_tol, cg_maxiter=self.cfg.cg_maxiter, damping=self.cfg.damping)
        self.graphs = []   # the schedules live on the device (see synchronize)
        if graphs:
            cap = torch.cuda.Stream()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                self.program.step()
            self.batch_graph = g
            torch.cuda.synchronize()

    def _batch_step(self, lam_states=None, stamps=None):
        """Enqueue one batched step of every problem: begin on each problem's stream, CG of all
        on the current stream, end on each problem's stream (events fork and join the streams)."""
        main = torch.cuda.current_stream()
        fork = torch.cuda.Event()
        fork.record(main)
        begun = []
        for i, opt in enumerate(self.opts):
            s = self.streams[i % len(self.streams)]
            s.wait_event(fork)
            with torch.cuda.stream(s):
                if stamps is not None:
                    api.device_timestamp(stamps, 2 * i)
                if lam_states is not None:
                    begun.append(api.gn_step_begin(opt.X, opt.A, lam_dev=lam_states[i][0:1],
                                                   cg_tol=self.cfg.cg_tol,
                                                   cg_maxiter=self.cfg.cg_maxiter, ws=opt.ws,
                                                   damping=self.cfg.damping))
                else:
                    begun.append(api.gn_step_begin(opt.X, opt.A, lam=opt.schedule.value,
                                                   cg_tol=self.cfg.cg_tol,
                                                   cg_maxiter=self.cfg.cg_maxiter, ws=opt.ws,
                                                   damping=self.cfg.damping))
        for s in self.streams[:len(self.opts)]:
            join = torch.cuda.Event()
            join.record(s)
            main.wait_event(join)
        for k in range(0, len(begun), api.L.MAX_CG_BATCH):
            api.gn_cg_batch(begun[k:k + api.L.MAX_CG_BATCH], self.cfg.cg_maxiter)
        fork2 = torch.cuda.Event()
        fork2.record(main)
        for i, opt in enumerate(self.opts):
            s = self.streams[i % len(self.streams)]
            s.wait_event(fork2)
            with torch.cuda.stream(s):
                api.gn_step_end(begun[i], stats=opt.stats_buf)
                if lam_states is not None:
                    api.damping_advance(lam_states[i])
                if stamps is not None:
                    api.device_timestamp(stamps, 2 * i + 1)
        for s in self.streams[:len(self.opts)]:
            join = torch.cuda.Event()
            join.record(s)
            main.wait_event(join)

    def _capture_batch(self):
        self._device_states()
        for opt in self.opts:
            prob = api._problem(opt.X, int(opt.A[0].shape[1]))
            api._ws(prob, api.L.OP_GN_STEP, opt.X.device, opt.ws)
        torch.cuda.synchronize()
        cap = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cap):
            self._batch_step(lam_states=self.lam_state)
        self.batch_graph = g
        self.graphs = []   # the per-problem schedules live on the device (see synchronize)
        torch.cuda.synchronize()

    def _capture(self):
        self._device_states()
        self.graphs = []
        for i, opt in enumerate(self.opts):
            s = self.streams[i % len(self.streams)]
            state = self.lam_state[i]
            # allocate the workspace before capture (nothing may be allocated inside it)
            prob = api._problem(opt.X, int(opt.A[0].shape[1]))
            api._ws(prob, api.L.OP_GN_STEP, opt.X.device, opt.ws)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                api.gn_step_devlam(opt.X, opt.A, state[0:1], self.cfg.cg_tol, self.cfg.cg_maxiter,
                                   stats=opt.stats_buf, ws=opt.ws, damping=self.cfg.damping,
                                   preconditioner=self.cfg.preconditioner)
                api.damping_advance(state)
            self.graphs.append(g)
        torch.cuda.synchronize()

    def step(self, timed: bool = False, stamps: torch.Tensor | None = None):
        """One Gauss-Newton step of every problem. With timed=True returns one (start, end) pair
        of HIP events per problem, recorded on its stream around its step. With stamps (device
        int64, 2 per problem) the device clock is written to stamps[2 i] and stamps[2 i + 1] by
        kernels enqueued on problem i's stream right before and after its step
        (api.device_timestamp; ticks of api.device_clock_hz())."""
        with api.tiles(self.tiles):
            return self._step(timed, stamps)

    def _step(self, timed, stamps):
        if self.batch_cg:
            if timed:
                raise ValueError("a batched step has one span per problem: use stamps")
            if self.fused and stamps is not None:
                raise ValueError("stamps are not part of a batch program")
            if self.batch_graph is not None:
                if stamps is not None:
                    raise ValueError("stamps are not part of the captured batch graph")
                self.batch_graph.replay()
            elif self.program is not None:
                self.program.step()
            else:
                self._batch_step(stamps=stamps)
            for opt in self.opts:
                if self.batch_graph is None and self.program is None:
                    opt.schedule.advance()
                opt.steps += 1
            return []
        events = []
        for i, opt in enumerate(self.opts):
            s = self.streams[i % len(self.streams)]
            with torch.cuda.stream(s):
                if timed:
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(s)
                if stamps is not None:
                    api.device_timestamp(stamps, 2 * i)
                if self.graphs is not None:
                    self.graphs[i].replay()
                    opt.steps += 1
                else:
                    opt.step()
                if stamps is not None:
                    api.device_timestamp(stamps, 2 * i + 1)
                if timed:
                    e1.record(s)
                    events.append((e0, e1))
        return events

    def synchronize(self):
        torch.cuda.current_stream().synchronize()
        for s in self.streams:
            s.synchronize()
        if self.graphs is not None:   # keep the host schedules in step with the device ones
            for opt, row in zip(self.opts, self.lam_all.cpu().tolist()):
                opt.schedule.load_device(row)

    def residuals(self):
        out = []
        with api.tiles(self.tiles):
            for i, opt in enumerate(self.opts):
                with torch.cuda.stream(self.streams[i % len(self.streams)]):
                    out.append(opt.residual())
        return out


@dataclass
class BatchedTuning:
    """The configuration chosen for a batch: HIP streams, graph replay, batched CG, the batch
    program and the MTTKRP tile shape (None: the default), the throughput it measured, the launch
    sweep (problem-steps/s per (n_streams, graphs, batch_cg, fused), default tiles) and the tile
    sweep (problem-steps/s per api.Tiles, chosen launch configuration)."""
    n_streams: int
    graphs: bool
    problem_steps_per_s: float
    table: dict
    batch_cg: bool = False
    fused: bool = False
    tiles: api.Tiles | None = None
    tile_table: dict = field(default_factory=dict)


# MTTKRP tile shapes the autotuner tries, one field at a time from the default (16 items per
# wavefront, 2 workgroups per CU, automatic row tile)
TILE_CANDIDATES = (("min_items", (4, 8, 32, 64)), ("wg_per_cu", (1, 4)), ("row_block", (2, 4)))
# a tile shape replaces the best one so far only when it is this much faster (timing noise of a
# few-step sweep)
TILE_MARGIN = 1.03


_TUNING_CACHE: dict = {}


def _pow2_ceil(v: int) -> int:
    return 1 << max(0, int(v) - 1).bit_length()


def batch_key(problems) -> tuple:
    """Shape bucket of a batch of (X, A) problems: the count, the storage type, and the ranks and
    largest mode sizes rounded up to powers of two, so that batches of similar shapes share a
    tuning."""
    ranks = sorted(_pow2_ceil(int(A[0].shape[1])) for _, A in problems)
    sizes = sorted(_pow2_ceil(max(int(s) for s in X.shape)) for X, _ in problems)
    dtypes = sorted({str(getattr(X, "dtype", type(X).__name__)) for X, _ in problems})
    return (len(problems), tuple(dtypes), tuple(ranks), tuple(sizes))


def _time_batched(problems, config, n_streams, graphs, steps, batch_cg=False,
                  fused=False, tiles=None) -> float:
    cur = [(X, [a.clone() for a in A]) for X, A in problems]   # the caller's factors stay as is
    torch.cuda.synchronize()
    bgn = BatchedGaussNewton(cur, config, n_streams=n_streams, graphs=graphs, batch_cg=batch_cg,
                             fused=fused, tiles=tiles)
    bgn.step()
    bgn.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bgn.step()
    bgn.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def autotune_batched(problems, config: GNConfig | None = None, stream_counts=(1, 2, 4, 8, 16),
                     graphs=(False, True), steps: int = 3, timer=None, cache=_TUNING_CACHE,
                     batch_cg=(False, True), fused=(False, True), tile_sweep: bool = True):
    """Sweep-based tuning of the batched runner: every (n_streams, graphs, batch_cg, fused)
    configuration runs `steps` Gauss-Newton steps of the whole batch on copies of its factors,
    timed by the wall clock, and the fastest is returned (the first one on a tie). batch_cg=True
    (CG of all problems in shared launches) is swept only where it applies (plain step,
    explicit-inverse preconditioner, ranks <= 128); fused=True (the whole step as a batch
    program, on one stream: n_streams 1) where that applies as well and no tensor is stored in
    bfloat16. The launch configurations do not change the iterates (the kernels are
    deterministic and the batched launches give the per-problem bits), only the throughput.

    With tile_sweep (FP32/FP64 tensors only) the chosen configuration is then timed under other
    MTTKRP tile shapes (api.Tiles), one field of TILE_CANDIDATES at a time starting from the
    default; a shape is kept when it beats the best so far by TILE_MARGIN. The tile shape changes
    the order of the MTTKRP's partial sums, so iterates under the chosen shape agree with the
    default's to rounding. The result is cached per batch_key, so a batch of a shape seen before
    is not timed again."""
    key = batch_key(problems)
    if cache is not None and key in cache:
        return cache[key]
    cfg = config or GNConfig()
    can_batch = (cfg.line_search is None and cfg.preconditioner == "inverse"
                 and max(int(A[0].shape[1]) for _, A in problems) <= 128)
    can_fuse = can_batch and all(isinstance(X, torch.Tensor) for X, _ in problems)
    timer = timer or _time_batched
    table = {}
    for g in graphs:
        for f in fused:
            if f and can_fuse:
                table[(1, bool(g), True, True)] = len(problems) * steps / timer(
                    problems, config, 1, g, steps, True, True)
    for ns in stream_counts:
        for g in graphs:
            for b in batch_cg:
                if b and not can_batch:
                    continue
                table[(int(ns), bool(g), bool(b), False)] = len(problems) * steps / timer(
                    problems, config, ns, g, steps, bool(b), False)
    best = max(table, key=table.get)
    rate = table[best]
    chosen = None
    tile_table = {}
    if tile_sweep and all(isinstance(X, torch.Tensor) and X.dtype in (torch.float32, torch.float64)
                          for X, _ in problems):
        cur = api.Tiles()
        tile_table[cur] = rate
        for name, values in TILE_CANDIDATES:
            base = cur
            for v in values:
                t = base._replace(**{name: v})
                if t in tile_table:
                    continue
                tile_table[t] = len(problems) * steps / timer(
                    problems, config, best[0], best[1], steps, best[2], best[3], tiles=t)
                if tile_table[t] > tile_table[cur] * TILE_MARGIN:
                    cur = t
        if cur != api.Tiles():
            chosen, rate = cur, tile_table[cur]
    out = BatchedTuning(n_streams=best[0], graphs=best[1], problem_steps_per_s=rate,
                        table=table, batch_cg=best[2], fused=best[3], tiles=chosen,
                        tile_table=tile_table)
    if cache is not None:
        cache[key] = out
    return out
