"""cp_gn_step_noalloc (the Gauss-Newton step on the library's built-in device scratch, for
callers that cannot allocate) against cp_gn_step with a caller workspace, through the C ABI: two
calls in a row on the same scratch, the second with a smaller problem, so that it runs over the
first call's leftovers. The two entry points run the same kernels on the same inputs, so the
factors and the stats must agree bit for bit (stronger than the 1e-12 FP64 parity bar)."""
import ctypes as C

import numpy as np
import pytest

from workloads import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1910_12331_amd as P  # noqa: E402
from paper_1910_12331_amd import _lib as L  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P._lib.load()
    yield
    torch.cuda.synchronize()


def abi_step(X, A, lam, eps, maxiter, noalloc):
    """One step through the raw C ABI; returns (factors after the step, stats bytes)."""
    lib = L.load()
    prob = P.api._problem(X, int(A[0].shape[1]))
    prm = L.CpGnParams(lam, eps, maxiter, 0)
    stats = P.stats_buffer(X.device)
    A = [a.clone() for a in A]
    ptrs = P.api._ptrs(A)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = lib.cp_gn_step_noalloc(C.byref(prob), X.data_ptr(), ptrs, C.byref(prm),
                                    stats.data_ptr(), stream)
    else:
        n = C.c_size_t(0)
        assert lib.cp_workspace_bytes(C.byref(prob), L.OP_GN_STEP, C.byref(n)) == 0
        ws = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=X.device)
        base = (ws.data_ptr() + 255) // 256 * 256
        rc = lib.cp_gn_step(C.byref(prob), X.data_ptr(), ptrs, C.byref(prm), stats.data_ptr(),
                            base, n.value, stream)
    assert rc == L.CP_OK, L.status_string(rc)
    torch.cuda.synchronize()
    return A, stats.cpu()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_noalloc_step_matches_workspace_step_twice(dt):
    big = make_problem((300, 300, 300), 50, workload=2, kind="congruent", noise=1e-6)
    small = make_problem((40, 40, 40), 5, workload=1)
    for p in (big, small):             # the second call is smaller and meets the first's leftovers
        X = torch.tensor(p.x, dtype=dt, device="cuda")
        A = [torch.tensor(a, dtype=dt, device="cuda") for a in p.init]
        got, st_got = abi_step(X, A, 1e-4, 1e-3, 20, noalloc=True)
        ref, st_ref = abi_step(X, A, 1e-4, 1e-3, 20, noalloc=False)
        assert torch.equal(st_got, st_ref)
        s = P.read_stats(st_got)
        assert s["status"] == 0 and s["cg_iters"] >= 1
        for g, r in zip(got, ref):
            assert torch.equal(g, r)
            rel = float(torch.linalg.norm((g - r).double()) / torch.linalg.norm(r.double()))
            assert rel <= 1e-12


def test_noalloc_binding_runs_a_gauss_newton_run():
    """The Python binding over the entry point: a run on workload 1 to a relative residual of
    1e-10 takes the same steps as the workspace form."""
    p = make_problem((40, 40, 40), 5, workload=1)
    X = torch.tensor(p.x, device="cuda")
    A1 = [torch.tensor(a, device="cuda") for a in p.init]
    A2 = [torch.tensor(a, device="cuda") for a in p.init]
    sched = P.DampingSchedule()
    sb1, sb2 = P.stats_buffer(X.device), P.stats_buffer(X.device)
    ws = P.Workspace()
    for _ in range(40):
        P.gn_step_noalloc(X, A1, sched.value, 1e-3, 20, stats=sb1)
        P.gn_step(X, A2, sched.value, 1e-3, 20, stats=sb2, ws=ws)
        sched.advance()
        assert torch.equal(sb1, sb2)
        r = P.residual(X, A1, ws=ws).cpu()
        if float(r[0] / r[1]) <= 1e-10:
            break
    assert float(r[0] / r[1]) <= 1e-10
    for a, b in zip(A1, A2):
        assert torch.equal(a, b)
