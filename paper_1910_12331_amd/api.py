"""Python entry points over the libcpgn.so C ABI.

Tensors are torch tensors resident on the GPU; this module only checks them, hands their
device pointers and the current HIP stream to the library, and allocates the workspace with
torch. Every step of the computation runs in the library's HIP kernels; there is no CPU
fallback, and a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import contextlib
from typing import NamedTuple, Sequence

import torch

from . import _lib as L

_DT = {torch.float64: L.CP_F64, torch.float32: L.CP_F32}


class SplitBF16Tensor:
    """A tensor stored as two bfloat16 planes whose sum is the tensor (x_dtype CP_BF16X3):
    `planes` has shape (2, *dims), hi plane first. Its MTTKRP takes three bf16 products per term
    (hi*hi + hi*lo + lo*hi) and is accurate to about 2^-16 relative. Build one from FP32 with
    to_bf16(X, split=True)."""

    dtype = "bf16x3"

    def __init__(self, planes: torch.Tensor):
        if planes.dtype != torch.bfloat16 or planes.dim() < 2 or planes.shape[0] != 2:
            raise ValueError("planes must be a (2, *dims) bfloat16 tensor")
        self.planes = planes
        self.shape = tuple(planes.shape[1:])
        self.device = planes.device
        self.is_cuda = planes.is_cuda

    def is_contiguous(self) -> bool:
        return self.planes.is_contiguous()

    def data_ptr(self) -> int:
        return self.planes.data_ptr()

    def dim(self) -> int:
        return len(self.shape)

    def to_float(self) -> torch.Tensor:
        """hi + lo in FP32 (exact for planes made from FP32 values)."""
        return self.planes[0].float() + self.planes[1].float()


def factor_dtype(X) -> torch.dtype:
    """dtype of the factor matrices that go with tensor X: FP32 for the bfloat16 forms."""
    if isinstance(X, SplitBF16Tensor) or X.dtype == torch.bfloat16:
        return torch.float32
    return X.dtype


def to_bf16(X: torch.Tensor, split: bool = False):
    """Round an FP32 GPU tensor to bfloat16 (nearest even) with the library's conversion kernel.
    split=True also keeps the rounding remainder as a second bfloat16 plane and returns a
    SplitBF16Tensor; otherwise a bfloat16 tensor of X's shape."""
    _dev(X, "X", torch.float32)
    n = X.numel()
    out = torch.empty(((2,) if split else ()) + tuple(X.shape), dtype=torch.bfloat16, device=X.device)
    _check(L.load().cp_tensor_to_bf16(X.data_ptr(), n, 1 if split else 0, out.data_ptr(), _stream()),
           "cp_tensor_to_bf16")
    return SplitBF16Tensor(out) if split else out


class CpError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {L.status_string(code)} (code {code})")
        self.code = code


def _check(rc: int, where: str):
    if rc != L.CP_OK:
        raise CpError(rc, where)


def _problem(X, rank: int) -> L.CpProblem:
    if isinstance(X, SplitBF16Tensor):
        xd, fd = L.CP_BF16X3, L.CP_F32
    elif X.dtype == torch.bfloat16:
        xd, fd = L.CP_BF16, L.CP_F32
    elif X.dtype in _DT:
        xd = fd = _DT[X.dtype]
    else:
        raise TypeError(f"unsupported tensor dtype {X.dtype}")
    if X.dim() < 2 or X.dim() > L.MAX_ORDER:
        raise ValueError("tensor order must be between 2 and 8")
    p = L.CpProblem()
    p.order = X.dim()
    p.rank = int(rank)
    for i, s in enumerate(X.shape):
        p.dims[i] = int(s)
    p.x_dtype, p.f_dtype = xd, fd
    return p


def _problem_from_factors(A: Sequence[torch.Tensor]) -> L.CpProblem:
    p = L.CpProblem()
    p.order = len(A)
    p.rank = int(A[0].shape[1])
    for i, a in enumerate(A):
        p.dims[i] = int(a.shape[0])
    p.x_dtype = p.f_dtype = _DT[A[0].dtype]
    return p


def _dev(t: torch.Tensor, name: str, dtype=None, shape=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _ptrs(ts: Sequence[torch.Tensor]):
    arr = L.PTRS()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


def _factors(A, X_or_dims, dtype, rank, name="A"):
    dims = X_or_dims
    if len(A) != len(dims):
        raise ValueError(f"{name} must hold one matrix per mode")
    for n, a in enumerate(A):
        _dev(a, f"{name}[{n}]", dtype, (dims[n], rank))
    return A


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Workspace:
    """Caches one device workspace per (problem, op); grows on demand."""

    def __init__(self):
        self._buf = None

    def get(self, prob: L.CpProblem, op: int, device) -> tuple[int, int]:
        n = C.c_size_t(0)
        _check(L.load().cp_workspace_bytes(C.byref(prob), op, C.byref(n)), "cp_workspace_bytes")
        need = int(n.value) + 256
        if self._buf is None or self._buf.numel() < need or self._buf.device != device:
            self._buf = torch.empty(need, dtype=torch.uint8, device=device)
        base = self._buf.data_ptr()
        aligned = (base + 255) // 256 * 256
        return aligned, int(n.value)


_default_ws = Workspace()


def release_default_workspace():
    """Drop the module-level workspace (for a clean shutdown: device memory is then released
    before interpreter exit instead of by exit-time destructors)."""
    _default_ws._buf = None


def _ws(prob, op, device, ws):
    return (ws or _default_ws).get(prob, op, device)


def mttkrp(X: torch.Tensor, A: Sequence[torch.Tensor], mode: int, out=None, ws=None,
           marks=None):
    """M = X_(mode) P^(mode) (Section 2.2, eq. (1)); returns a dims[mode] x R tensor.
    marks: optional (begin, end) pair of torch.cuda.Event (enable_timing=True, recorded once
    before so that the HIP events exist), recorded around the main MTTKRP kernel only
    (cp_mttkrp_marked): begin.elapsed_time(end) is that kernel's duration."""
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    if out is None:
        out = torch.empty((X.shape[mode], R), dtype=factor_dtype(X), device=X.device)
    _dev(out, "out", factor_dtype(X), (X.shape[mode], R))
    w, nb = _ws(prob, L.OP_MTTKRP, X.device, ws)
    lib = L.load()
    if marks is None:
        _check(lib.cp_mttkrp(C.byref(prob), X.data_ptr(), _ptrs(A), int(mode), out.data_ptr(), w,
                             nb, _stream()), "cp_mttkrp")
    else:
        ev0, ev1 = marks
        if not ev0.cuda_event or not ev1.cuda_event:
            raise ValueError("mttkrp marks: record each event once before passing it")
        _check(lib.cp_mttkrp_marked(C.byref(prob), X.data_ptr(), _ptrs(A), int(mode),
                                    out.data_ptr(), w, nb, _stream(), C.c_void_p(ev0.cuda_event),
                                    C.c_void_p(ev1.cuda_event)), "cp_mttkrp_marked")
    return out


def mttkrp_all(X, A: Sequence[torch.Tensor], out=None, ws=None):
    """M(n) for every mode at one point (FP32/FP64 order >= 3 with the last mode a multiple of
    4: modes 0 .. N-2 from one pass over X through a dimension tree). Returns the list of
    dims[n] x R tensors."""
    _dev(X, "X")
    R = int(A[0].shape[1])
    fd = factor_dtype(X)
    _factors(A, X.shape, fd, R)
    prob = _problem(X, R)
    if out is None:
        out = [torch.empty((s, R), dtype=fd, device=X.device) for s in X.shape]
    _factors(out, X.shape, fd, R, "out")
    w, nb = _ws(prob, L.OP_MTTKRP_ALL, X.device, ws)
    _check(L.load().cp_mttkrp_all(C.byref(prob), X.data_ptr(), _ptrs(A), _ptrs(out), w, nb,
                                  _stream()), "cp_mttkrp_all")
    return out


def gn_gradient(X: torch.Tensor, A: Sequence[torch.Tensor], ws=None):
    """G(n) = A(n) Gamma(n,n) - M(n) for every mode (Algorithm 1). Returns (G list, sum ||G||)."""
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    G = [torch.empty_like(a) for a in A]
    gsum = torch.empty(1, dtype=torch.float64, device=X.device)
    w, nb = _ws(prob, L.OP_GN_GRADIENT, X.device, ws)
    _check(L.load().cp_gn_gradient(C.byref(prob), X.data_ptr(), _ptrs(A), _ptrs(G), gsum.data_ptr(),
                                   w, nb, _stream()), "cp_gn_gradient")
    return G, gsum


def objective_gradient(X: torch.Tensor, A: Sequence[torch.Tensor], ws=None):
    """G(n) = A(n) Gamma(n,n) - M(n) for every mode and [||X - [[A]]||_F, ||X||_F] by the expansion
    from the same MTTKRP and Grams (cp_objective_gradient). Returns (G list, device float64[2])."""
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    G = [torch.empty_like(a) for a in A]
    res = torch.empty(2, dtype=torch.float64, device=X.device)
    w, nb = _ws(prob, L.OP_GN_GRADIENT, X.device, ws)
    _check(L.load().cp_objective_gradient(C.byref(prob), X.data_ptr(), _ptrs(A), _ptrs(G),
                                          res.data_ptr(), w, nb, _stream()),
           "cp_objective_gradient")
    return G, res


def jtj_matvec(A: Sequence[torch.Tensor], W: Sequence[torch.Tensor], lam: float = 0.0, ws=None):
    """Q = (J^T J + lam I) W through the implicit contractions of eq. (7)."""
    R = int(A[0].shape[1])
    dims = [a.shape[0] for a in A]
    _factors(A, dims, A[0].dtype, R)
    _factors(W, dims, A[0].dtype, R, "W")
    prob = _problem_from_factors(A)
    Q = [torch.empty_like(w) for w in W]
    w, nb = _ws(prob, L.OP_GN_JTJ_MATVEC, A[0].device, ws)
    _check(L.load().cp_gn_jtj_matvec(C.byref(prob), _ptrs(A), _ptrs(W), float(lam), _ptrs(Q), w, nb,
                                     _stream()), "cp_gn_jtj_matvec")
    return Q


STATS_FIELDS = ("status", "cg_iters", "grad_norm_sum", "cg_res_norm_sum", "alpha_last",
                "beta_last", "update_norm")


def stats_buffer(device) -> torch.Tensor:
    return torch.zeros(C.sizeof(L.CpGnStats), dtype=torch.uint8, device=device)


def read_stats(buf: torch.Tensor) -> dict:
    raw = bytes(buf.cpu().numpy().tobytes())
    s = L.CpGnStats.from_buffer_copy(raw)
    return {f: getattr(s, f) for f in STATS_FIELDS}


def _gn_flags(damping: str, preconditioner: str) -> int:
    if damping not in ("identity", "diagonal"):
        raise ValueError("damping must be 'identity' or 'diagonal'")
    if preconditioner not in ("inverse", "cholesky"):
        raise ValueError("preconditioner must be 'inverse' or 'cholesky'")
    return ((L.GN_DIAG_DAMPING if damping == "diagonal" else 0)
            | (L.GN_CHOL_PRECOND if preconditioner == "cholesky" else 0))


def gn_step(X: torch.Tensor, A: Sequence[torch.Tensor], lam: float, cg_tol: float = 1e-3,
            cg_maxiter: int = 20, stats=None, ws=None, damping: str = "identity",
            preconditioner: str = "inverse"):
    """One Algorithm 1 step in place on A; returns the device stats buffer (cp_gn_stats).
    damping: "identity" (lam I) or "diagonal" (lam diag(J^T J), Section 3.2).
    preconditioner: "inverse" (explicit inverse, Section 3.3) or "cholesky" (triangular solves
    with the Cholesky factor, R <= 128)."""
    if damping not in ("identity", "diagonal"):
        raise ValueError("damping must be 'identity' or 'diagonal'")
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    prm = L.CpGnParams(float(lam), float(cg_tol), int(cg_maxiter),
                       _gn_flags(damping, preconditioner))
    if stats is None:
        stats = stats_buffer(X.device)
    w, nb = _ws(prob, L.OP_GN_STEP, X.device, ws)
    _check(L.load().cp_gn_step(C.byref(prob), X.data_ptr(), _ptrs(A), C.byref(prm), stats.data_ptr(),
                               w, nb, _stream()), "cp_gn_step")
    return stats


def gn_step_noalloc(X: torch.Tensor, A: Sequence[torch.Tensor], lam: float, cg_tol: float = 1e-3,
                    cg_maxiter: int = 20, stats=None, damping: str = "identity",
                    preconditioner: str = "inverse"):
    """gn_step with the library's built-in device scratch as workspace (cp_gn_step_noalloc): no
    device memory is allocated for the call (pass `stats` to allocate nothing at all). Calls that
    overlap on one GPU share that scratch and must not run concurrently."""
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    prm = L.CpGnParams(float(lam), float(cg_tol), int(cg_maxiter),
                       _gn_flags(damping, preconditioner))
    if stats is None:
        stats = stats_buffer(X.device)
    _check(L.load().cp_gn_step_noalloc(C.byref(prob), X.data_ptr(), _ptrs(A), C.byref(prm),
                                       stats.data_ptr(), _stream()), "cp_gn_step_noalloc")
    return stats


ARMIJO_FIELDS = ("alpha", "f0", "f", "gv", "x_norm", "trials", "accepted")


def armijo_stats_buffer(device) -> torch.Tensor:
    return torch.zeros(C.sizeof(L.CpArmijoStats), dtype=torch.uint8, device=device)


def read_armijo_stats(buf: torch.Tensor) -> dict:
    s = L.CpArmijoStats.from_buffer_copy(bytes(buf.cpu().numpy().tobytes()))
    return {f: getattr(s, f) for f in ARMIJO_FIELDS}


def gn_step_armijo(X: torch.Tensor, A: Sequence[torch.Tensor], lam: float, cg_tol: float = 1e-3,
                   cg_maxiter: int = 20, c: float = 1e-4, shrink: float = 0.5,
                   max_trials: int = 10, stats=None, ls_stats=None, ws=None,
                   damping: str = "identity", preconditioner: str = "inverse",
                   f0_given: bool = False):
    """Gauss-Newton step with Armijo step-size control (Section 5), in place on A: the direction
    of gn_step, then the first of alpha = 1, shrink, shrink^2, ... (at most max_trials) with
    f(A + alpha V) <= f(A) + c alpha <G, V>. Returns (stats buffer, Armijo stats buffer), both on
    the device (read_stats, read_armijo_stats). f0_given=True takes f(A) from ls_stats as the
    previous call on these same factors left it (CP_LS_F0_GIVEN) instead of a residual pass."""
    if damping not in ("identity", "diagonal"):
        raise ValueError("damping must be 'identity' or 'diagonal'")
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    prm = L.CpGnParams(float(lam), float(cg_tol), int(cg_maxiter),
                       _gn_flags(damping, preconditioner))
    ls = L.CpArmijoParams(float(c), float(shrink), int(max_trials),
                          L.LS_F0_GIVEN if f0_given else 0)
    if stats is None:
        stats = stats_buffer(X.device)
    if ls_stats is None:
        if f0_given:
            raise ValueError("f0_given needs the ls_stats buffer of the previous step")
        ls_stats = armijo_stats_buffer(X.device)
    w, nb = _ws(prob, L.OP_GN_STEP, X.device, ws)
    _check(L.load().cp_gn_step_armijo(C.byref(prob), X.data_ptr(), _ptrs(A), C.byref(prm),
                                      C.byref(ls), stats.data_ptr(), ls_stats.data_ptr(), w, nb,
                                      _stream()), "cp_gn_step_armijo")
    return stats, ls_stats


def gn_step_devlam(X, A: Sequence[torch.Tensor], lam_dev: torch.Tensor, cg_tol: float = 1e-3,
                   cg_maxiter: int = 20, stats=None, ws=None, damping: str = "identity",
                   preconditioner: str = "inverse"):
    """gn_step with the damping read from device memory (lam_dev: a one-element float64 GPU
    tensor) when the step runs, so that a captured graph of the step follows a changing lambda."""
    if damping not in ("identity", "diagonal"):
        raise ValueError("damping must be 'identity' or 'diagonal'")
    _dev(X, "X")
    _dev(lam_dev, "lam_dev", torch.float64)
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    prm = L.CpGnParams(0.0, float(cg_tol), int(cg_maxiter),
                       _gn_flags(damping, preconditioner))
    if stats is None:
        stats = stats_buffer(X.device)
    w, nb = _ws(prob, L.OP_GN_STEP, X.device, ws)
    _check(L.load().cp_gn_step_devlam(C.byref(prob), X.data_ptr(), _ptrs(A), C.byref(prm),
                                      lam_dev.data_ptr(), stats.data_ptr(), w, nb, _stream()),
           "cp_gn_step_devlam")
    return stats


class BegunStep(NamedTuple):
    """A Gauss-Newton step whose part before CG is enqueued (gn_step_begin): the problem, its
    workspace (pointer and size) and the factors the step updates."""
    prob: object
    ws_ptr: int
    ws_bytes: int
    A: list


def gn_step_begin(X, A: Sequence[torch.Tensor], lam: float | None = None, lam_dev=None,
                  cg_tol: float = 1e-3, cg_maxiter: int = 20, ws=None,
                  damping: str = "identity") -> BegunStep:
    """The part of a Gauss-Newton step before CG on the current stream (cp_gn_step_begin), with
    the damping lam (host) or lam_dev (a one-element float64 GPU tensor read when it runs)."""
    if damping not in ("identity", "diagonal"):
        raise ValueError("damping must be 'identity' or 'diagonal'")
    if (lam is None) == (lam_dev is None):
        raise ValueError("give exactly one of lam and lam_dev")
    _dev(X, "X")
    if lam_dev is not None:
        _dev(lam_dev, "lam_dev", torch.float64)
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    prm = L.CpGnParams(float(lam) if lam is not None else 0.0, float(cg_tol), int(cg_maxiter),
                       _gn_flags(damping, "inverse"))
    w, nb = _ws(prob, L.OP_GN_STEP, X.device, ws)
    _check(L.load().cp_gn_step_begin(C.byref(prob), X.data_ptr(), _ptrs(A), C.byref(prm),
                                     lam_dev.data_ptr() if lam_dev is not None else None, w, nb,
                                     _stream()), "cp_gn_step_begin")
    return BegunStep(prob, w, nb, list(A))


def gn_cg_batch(steps: Sequence[BegunStep], cg_maxiter: int = 20):
    """CG of every begun step in shared launches on the current stream (cp_gn_cg_batch)."""
    n = len(steps)
    if not 1 <= n <= L.MAX_CG_BATCH:
        raise ValueError(f"1 to {L.MAX_CG_BATCH} steps per batch")
    probs = (L.CpProblem * n)(*[s.prob for s in steps])
    wss = (C.c_void_p * n)(*[s.ws_ptr for s in steps])
    nbs = (C.c_size_t * n)(*[s.ws_bytes for s in steps])
    _check(L.load().cp_gn_cg_batch(n, probs, wss, nbs, int(cg_maxiter), _stream()),
           "cp_gn_cg_batch")


def gn_step_end(step: BegunStep, stats=None):
    """A += V and the step's stats for one begun step, on the current stream (cp_gn_step_end)."""
    if stats is None:
        stats = stats_buffer(step.A[0].device)
    _check(L.load().cp_gn_step_end(C.byref(step.prob), _ptrs(step.A), stats.data_ptr(),
                                   step.ws_ptr, step.ws_bytes, _stream()), "cp_gn_step_end")
    return stats


class GNBatchProgram:
    """One Gauss-Newton step of many problems in shared launches (cp_gn_batch_create /
    cp_gn_batch_step): each problem's launches before and after CG are recorded once, and a step
    runs one launch per kernel and position in the step for the whole batch, with the CG of all
    problems in between. Each problem's factors, stats and damping come out bitwise as from
    gn_step_begin / gn_cg_batch / gn_step_end.

    problems: sequence of (X, A, ws, stats, lam_state): ws a Workspace, stats a stats_buffer,
    lam_state a float64[5] damping state on the device (read as lambda and advanced after each
    step) or None (then lam is used). The tensors must stay alive and unmoved while the program
    is used; the program keeps references to them."""

    def __init__(self, problems, lam: float = 0.0, cg_tol: float = 1e-3, cg_maxiter: int = 20,
                 damping: str = "identity"):
        n = len(problems)
        if n < 1:
            raise ValueError("at least one problem")
        self._keep = []
        probs = (L.CpProblem * n)()
        Xs = (C.c_void_p * n)()
        As = (C.c_void_p * (n * L.MAX_ORDER))()
        lams = (C.c_void_p * n)()
        states = (C.c_void_p * n)()
        stats = (C.c_void_p * n)()
        wss = (C.c_void_p * n)()
        nbs = (C.c_size_t * n)()
        for i, (X, A, ws, st, lam_state) in enumerate(problems):
            _dev(X, "X")
            R = int(A[0].shape[1])
            _factors(A, X.shape, factor_dtype(X), R)
            probs[i] = _problem(X, R)
            Xs[i] = X.data_ptr()
            for m, a in enumerate(A):
                As[i * L.MAX_ORDER + m] = a.data_ptr()
            if lam_state is not None:
                _dev(lam_state, "lam_state", torch.float64, (5,))
                lams[i] = states[i] = lam_state.data_ptr()
            stats[i] = st.data_ptr()
            wss[i], nbs[i] = ws.get(probs[i], L.OP_GN_STEP, X.device)
            self._keep.append((X, list(A), ws, st, lam_state))
        prm = L.CpGnParams(float(lam), float(cg_tol), int(cg_maxiter), _gn_flags(damping, "inverse"))
        lib = L.load()
        need = C.c_size_t(0)
        handle = C.c_void_p(None)
        args = [n, probs, Xs, As, C.byref(prm), lams, states, stats, wss, nbs]
        rc = lib.cp_gn_batch_create(*args, None, 0, C.byref(need), C.byref(handle))
        if rc != L.CP_EWORKSPACE:
            _check(rc, "cp_gn_batch_create")
        self.table = torch.empty(int(need.value) + 16, dtype=torch.uint8, device=problems[0][0].device)
        base = (self.table.data_ptr() + 15) // 16 * 16
        _check(lib.cp_gn_batch_create(*args, base, int(need.value), C.byref(need), C.byref(handle)),
               "cp_gn_batch_create")
        self._handle = handle
        self._lib = lib

    def step(self):
        """Enqueue one Gauss-Newton step of every problem on the current stream."""
        _check(self._lib.cp_gn_batch_step(self._handle, _stream()), "cp_gn_batch_step")

    def close(self):
        if self._handle is not None and self._handle.value:
            self._lib.cp_gn_batch_destroy(self._handle)
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def damping_advance(state: torch.Tensor):
    """Advance a device damping state {lambda, lower, upper, mu, decreasing} (float64[5]) once."""
    _dev(state, "state", torch.float64, (5,))
    _check(L.load().cp_damping_advance(state.data_ptr(), _stream()), "cp_damping_advance")
    return state


def device_timestamp(buf: torch.Tensor, index: int):
    """Enqueue on the current stream a write of the device clock to buf[index] (device int64)."""
    _dev(buf, "buf", torch.int64)
    if not 0 <= index < buf.numel():
        raise IndexError(index)
    ptr = buf.data_ptr() + index * 8
    _check(L.load().cp_device_timestamp(ptr, _stream()), "cp_device_timestamp")


def device_clock_hz() -> int:
    """Rate of the clock that device_timestamp writes (ticks per second)."""
    hz = C.c_int64(0)
    _check(L.load().cp_device_clock_hz(C.byref(hz)), "cp_device_clock_hz")
    return int(hz.value)


class Tiles(NamedTuple):
    """MTTKRP tile shape (cp_tuning): least items per wavefront, workgroups per compute unit a
    launch aims for, FP32 row tile in 16-row blocks (2, 4 or 5). 0 takes the default
    (16, 2, automatic)."""
    min_items: int = 0
    wg_per_cu: int = 0
    row_block: int = 0


def set_tiles(t: Tiles | None):
    """Set the calling thread's MTTKRP tile shape for the calls made from it afterwards
    (cp_set_tuning); None restores the defaults."""
    lib = L.load()
    if t is None:
        _check(lib.cp_set_tuning(None), "cp_set_tuning")
        return
    ct = L.CpTuning(int(t.min_items), int(t.wg_per_cu), int(t.row_block), 0)
    _check(lib.cp_set_tuning(C.byref(ct)), "cp_set_tuning")


def get_tiles() -> Tiles:
    """The calling thread's MTTKRP tile shape (cp_get_tuning; zeros are defaults)."""
    ct = L.CpTuning()
    _check(L.load().cp_get_tuning(C.byref(ct)), "cp_get_tuning")
    return Tiles(ct.mttkrp_min_items, ct.mttkrp_wg_per_cu, ct.mttkrp_row_block)


@contextlib.contextmanager
def tiles(t: Tiles | None):
    """Run a block under MTTKRP tile shape t (None: leave the current one) and restore the
    previous shape afterwards."""
    if t is None:
        yield
        return
    prev = get_tiles()
    set_tiles(t)
    try:
        yield
    finally:
        set_tiles(prev)


def als_sweep(X: torch.Tensor, A: Sequence[torch.Tensor], lam: float = 0.0, status=None, ws=None):
    """One ALS sweep in place on A (Section 2.2); returns the device int32 status."""
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
    w, nb = _ws(prob, L.OP_ALS_SWEEP, X.device, ws)
    _check(L.load().cp_als_sweep(C.byref(prob), X.data_ptr(), _ptrs(A), float(lam), status.data_ptr(),
                                 w, nb, _stream()), "cp_als_sweep")
    return status


def residual(X: torch.Tensor, A: Sequence[torch.Tensor], method: int = L.RESIDUAL_DIRECT, out=None,
             ws=None):
    """Device tensor [||X - [[A]]||_F, ||X||_F] (Section 5)."""
    _dev(X, "X")
    R = int(A[0].shape[1])
    _factors(A, X.shape, factor_dtype(X), R)
    prob = _problem(X, R)
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=X.device)
    w, nb = _ws(prob, L.OP_RESIDUAL, X.device, ws)
    _check(L.load().cp_residual(C.byref(prob), X.data_ptr(), _ptrs(A), int(method), out.data_ptr(),
                                w, nb, _stream()), "cp_residual")
    return out
