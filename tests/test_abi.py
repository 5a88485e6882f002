"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every symbol the
public header declares, its structs have the header's layout, and argument errors are
reported before anything is enqueued. Also the host-side damping schedule."""
import ctypes as C
import os
import re
import subprocess
import threading

import pytest

import oracle as O
from paper_1910_12331_amd import _lib as L
from paper_1910_12331_amd.optim import DampingSchedule

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpgn.h")


@pytest.fixture(scope="module")
def lib():
    return L.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cp_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (cp_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "cpgn.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(cp_problem), offsetof(cp_problem, dims),'
        " offsetof(cp_problem, x_dtype), offsetof(cp_problem, f_dtype), sizeof(cp_gn_params));\n"
        'printf("%zu %zu %zu\\n", sizeof(cp_gn_stats), offsetof(cp_gn_stats, grad_norm_sum),'
        " offsetof(cp_gn_stats, update_norm));\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(cp_armijo_params), offsetof(cp_armijo_params,'
        ' max_trials), sizeof(cp_armijo_stats), offsetof(cp_armijo_stats, x_norm),'
        " offsetof(cp_armijo_stats, accepted));\n"
        'printf("%zu %zu %zu\\n", sizeof(cp_tuning), offsetof(cp_tuning, mttkrp_row_block),'
        " offsetof(cp_tuning, reserved));\n"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    a = list(map(int, lines[0].split()))
    b = list(map(int, lines[1].split()))
    assert a == [C.sizeof(L.CpProblem), L.CpProblem.dims.offset, L.CpProblem.x_dtype.offset,
                 L.CpProblem.f_dtype.offset, C.sizeof(L.CpGnParams)]
    assert b == [C.sizeof(L.CpGnStats), L.CpGnStats.grad_norm_sum.offset,
                 L.CpGnStats.update_norm.offset]
    c = list(map(int, lines[2].split()))
    assert c == [C.sizeof(L.CpArmijoParams), L.CpArmijoParams.max_trials.offset,
                 C.sizeof(L.CpArmijoStats), L.CpArmijoStats.x_norm.offset,
                 L.CpArmijoStats.accepted.offset]
    d = list(map(int, lines[3].split()))
    assert d == [C.sizeof(L.CpTuning), L.CpTuning.mttkrp_row_block.offset,
                 L.CpTuning.reserved.offset]


def prob(dims=(8, 9, 10), rank=5, dt=L.CP_F64):
    p = L.CpProblem()
    p.order = len(dims)
    p.rank = rank
    for i, s in enumerate(dims):
        p.dims[i] = s
    p.x_dtype = p.f_dtype = dt
    return p


def ws_bytes(lib, p, op=L.OP_GN_STEP):
    n = C.c_size_t(0)
    rc = lib.cp_workspace_bytes(C.byref(p), op, C.byref(n))
    return rc, n.value


def test_workspace_queries(lib):
    rc, n = ws_bytes(lib, prob())
    assert rc == 0 and n > 0 and n % 256 == 0
    for op in range(7):
        assert ws_bytes(lib, prob(), op)[0] == 0
    assert ws_bytes(lib, prob(), 17)[0] == L.CP_EINVAL
    big = ws_bytes(lib, prob((400, 400, 400), 100, L.CP_F32))[1]
    assert big < 64 << 20   # the workspace stays small next to the tensor


def test_tuning_validation_and_workspace_sizes(lib):
    """cp_set_tuning checks its fields, keeps the setting per thread and resets on NULL; the
    MTTKRP partial tiles in the workspace follow the split it sets (host planning only)."""
    p = prob((400, 400, 400), 100, L.CP_F32)
    base = ws_bytes(lib, p)[1]
    got = L.CpTuning()
    try:
        for bad in [(-1, 0, 0, 0), (4097, 0, 0, 0), (0, 9, 0, 0), (0, -1, 0, 0), (0, 0, 3, 0),
                    (0, 0, 1, 0), (0, 0, 0, 1)]:
            assert lib.cp_set_tuning(C.byref(L.CpTuning(*bad))) == L.CP_EINVAL, bad
        assert lib.cp_get_tuning(C.byref(got)) == 0
        assert (got.mttkrp_min_items, got.mttkrp_wg_per_cu, got.mttkrp_row_block) == (0, 0, 0)
        assert lib.cp_get_tuning(None) == L.CP_EINVAL
        assert lib.cp_set_tuning(C.byref(L.CpTuning(8, 4, 2, 0))) == 0
        assert lib.cp_get_tuning(C.byref(got)) == 0
        assert (got.mttkrp_min_items, got.mttkrp_wg_per_cu, got.mttkrp_row_block) == (8, 4, 2)
        # twice the workgroups per launch: more partial tiles than the default split
        assert ws_bytes(lib, p)[1] > base
        assert lib.cp_set_tuning(C.byref(L.CpTuning(4096, 1, 0, 0))) == 0
        assert ws_bytes(lib, p)[1] <= base
        # the setting belongs to the thread that made it
        seen = []
        t = threading.Thread(target=lambda: seen.append(ws_bytes(lib, p)[1]))
        t.start()
        t.join()
        assert seen == [base]
        assert lib.cp_set_tuning(C.byref(L.CpTuning(16, 2, 0, 0))) == 0   # the defaults
        assert ws_bytes(lib, p)[1] == base
    finally:
        assert lib.cp_set_tuning(None) == 0
    assert ws_bytes(lib, p)[1] == base


@pytest.mark.parametrize("mut,code", [
    (lambda p: setattr(p, "order", 1), L.CP_EINVAL),
    (lambda p: setattr(p, "order", 9), L.CP_EINVAL),
    (lambda p: setattr(p, "rank", 0), L.CP_EINVAL),
    (lambda p: p.dims.__setitem__(1, 0), L.CP_EINVAL),
    (lambda p: setattr(p, "f_dtype", L.CP_F32), L.CP_EUNSUPPORTED),
    (lambda p: (setattr(p, "x_dtype", 2), setattr(p, "f_dtype", 2)), L.CP_EUNSUPPORTED),
    (lambda p: (setattr(p, "x_dtype", L.CP_BF16X3), setattr(p, "f_dtype", L.CP_F64)), L.CP_EUNSUPPORTED),
    (lambda p: (setattr(p, "x_dtype", 4), setattr(p, "f_dtype", L.CP_F32)), L.CP_EUNSUPPORTED),
    (lambda p: (setattr(p, "x_dtype", L.CP_BF16), setattr(p, "f_dtype", L.CP_F32)), L.CP_OK),
    (lambda p: (setattr(p, "x_dtype", L.CP_BF16X3), setattr(p, "f_dtype", L.CP_F32)), L.CP_OK),
])
def test_problem_validation(lib, mut, code):
    p = prob()
    mut(p)
    assert ws_bytes(lib, p)[0] == code


def fake_ptrs(n=3):
    a = L.PTRS()
    for i in range(n):
        a[i] = 0x1000 * (i + 1)
    return a


def test_call_validation_without_launch(lib):
    p = prob()
    _, need = ws_bytes(lib, p)
    X, M, ws = C.c_void_p(0x10000), C.c_void_p(0x20000), C.c_void_p(0x40000)
    A = fake_ptrs()
    # bad mode, null tensor, null factor, small / misaligned / null workspace
    assert lib.cp_mttkrp(C.byref(p), X, A, 3, M, ws, need, None) == L.CP_EINVAL
    assert lib.cp_mttkrp(C.byref(p), X, A, -1, M, ws, need, None) == L.CP_EINVAL
    assert lib.cp_mttkrp(C.byref(p), None, A, 0, M, ws, need, None) == L.CP_EINVAL
    A0 = fake_ptrs()
    A0[1] = 0
    assert lib.cp_mttkrp(C.byref(p), X, A0, 0, M, ws, need, None) == L.CP_EINVAL
    assert lib.cp_mttkrp(C.byref(p), X, A, 0, M, ws, need - 1, None) == L.CP_EWORKSPACE
    assert lib.cp_mttkrp(C.byref(p), X, A, 0, M, C.c_void_p(0x40010), need, None) == L.CP_EINVAL
    assert lib.cp_mttkrp(C.byref(p), X, A, 0, M, None, need, None) == L.CP_EINVAL
    # the marked form validates the same way before recording anything
    assert lib.cp_mttkrp_marked(C.byref(p), X, A, 3, M, ws, need, None, None, None) == L.CP_EINVAL
    assert lib.cp_mttkrp_marked(C.byref(p), None, A, 0, M, ws, need, None, None,
                                None) == L.CP_EINVAL
    assert lib.cp_mttkrp_marked(C.byref(p), X, A, 0, M, ws, need - 1, None, None,
                                None) == L.CP_EWORKSPACE
    # all-mode MTTKRP: null output pointer, null tensor, small workspace
    Ms = fake_ptrs()
    Ms[2] = 0
    assert lib.cp_mttkrp_all(C.byref(p), X, A, Ms, ws, need, None) == L.CP_EINVAL
    assert lib.cp_mttkrp_all(C.byref(p), None, A, fake_ptrs(), ws, need, None) == L.CP_EINVAL
    assert lib.cp_mttkrp_all(C.byref(p), X, A, fake_ptrs(), ws, need - 1, None) == L.CP_EWORKSPACE
    # device damping: null pointers
    good0 = L.CpGnParams(0.0, 1e-3, 20, 0)
    assert lib.cp_gn_step_devlam(C.byref(p), X, A, C.byref(good0), None, C.c_void_p(0x50000), ws,
                                 need, None) == L.CP_EINVAL
    assert lib.cp_damping_advance(None, None) == L.CP_EINVAL
    assert lib.cp_device_timestamp(None, None) == L.CP_EINVAL
    # split step: batch size and null arrays are rejected before any launch
    wsa = (C.c_void_p * 1)(ws)
    nba = (C.c_size_t * 1)(need)
    assert lib.cp_gn_cg_batch(0, C.byref(p), wsa, nba, 20, None) == L.CP_EINVAL
    assert lib.cp_gn_cg_batch(L.MAX_CG_BATCH + 1, C.byref(p), wsa, nba, 20, None) == L.CP_EINVAL
    assert lib.cp_gn_cg_batch(1, C.byref(p), None, nba, 20, None) == L.CP_EINVAL
    assert lib.cp_gn_cg_batch(1, C.byref(p), wsa, nba, -1, None) == L.CP_EINVAL
    assert lib.cp_gn_step_begin(C.byref(p), None, A, C.byref(good0), None, ws, need, None) == L.CP_EINVAL
    assert lib.cp_gn_step_end(C.byref(p), A, None, ws, need, None) == L.CP_EINVAL
    assert lib.cp_device_clock_hz(None) == L.CP_EINVAL
    # batch program: argument checks, then the table-size query (recording only, no launch)
    n2 = 2
    probs2 = (L.CpProblem * n2)(p, p)
    X2 = (C.c_void_p * n2)(0x10000, 0x11000)
    A2 = (C.c_void_p * (n2 * L.MAX_ORDER))(*([0x1000, 0x2000, 0x3000] + [0] * (L.MAX_ORDER - 3)) * 2)
    st2 = (C.c_void_p * n2)(0x50000, 0x51000)
    ws2 = (C.c_void_p * n2)(0x40000, 0x40000 + (need + 4095) // 4096 * 4096)
    nb2 = (C.c_size_t * n2)(need, need)
    needed, h = C.c_size_t(0), C.c_void_p(None)
    args = lambda cnt, prm=good0, st=st2: [cnt, probs2, X2, A2, C.byref(prm), None, None, st, ws2,
                                          nb2, None, 0, C.byref(needed), C.byref(h)]
    assert lib.cp_gn_batch_create(*args(0)) == L.CP_EINVAL
    assert lib.cp_gn_batch_create(*args(n2, st=None)) == L.CP_EINVAL
    chol = L.CpGnParams(0.0, 1e-3, 20, L.GN_CHOL_PRECOND)
    assert lib.cp_gn_batch_create(*args(n2, prm=chol)) == L.CP_EUNSUPPORTED
    assert lib.cp_gn_batch_create(*args(n2)) == L.CP_EWORKSPACE and needed.value > 0
    assert not h.value   # nothing created
    assert lib.cp_gn_batch_step(None, None) == L.CP_EINVAL
    big = L.CpProblem(p.order, 130, p.dims, p.x_dtype, p.f_dtype)
    probs3 = (L.CpProblem * n2)(big, big)
    assert lib.cp_gn_batch_create(n2, probs3, X2, A2, C.byref(good0), None, None, st2, ws2, nb2,
                                  None, 0, C.byref(needed), C.byref(h)) == L.CP_EUNSUPPORTED
    # storage conversion: negative count, null pointers
    assert lib.cp_tensor_to_bf16(X, -1, 0, M, None) == L.CP_EINVAL
    assert lib.cp_tensor_to_bf16(None, 10, 0, M, None) == L.CP_EINVAL
    assert lib.cp_tensor_to_bf16(X, 10, 1, None, None) == L.CP_EINVAL
    assert lib.cp_tensor_to_bf16(None, 0, 0, None, None) == L.CP_OK
    # Gauss-Newton parameters
    st = C.c_void_p(0x50000)
    for prm in [L.CpGnParams(-1.0, 1e-3, 20, 0), L.CpGnParams(1e-3, -1.0, 20, 0),
                L.CpGnParams(1e-3, 1e-3, -1, 0), L.CpGnParams(1e-3, 1e-3, 20, 4),
                L.CpGnParams(float("nan"), 1e-3, 20, 0)]:
        assert lib.cp_gn_step(C.byref(p), X, A, C.byref(prm), st, ws, need, None) == L.CP_EINVAL
    good = L.CpGnParams(1e-3, 1e-3, 20, 0)
    assert lib.cp_gn_step(C.byref(p), X, A, C.byref(good), None, ws, need, None) == L.CP_EINVAL
    assert lib.cp_gn_step(C.byref(p), X, A, C.byref(good), st, ws, need // 2, None) == L.CP_EWORKSPACE
    # Armijo step control: null search parameters or stats, constants out of range
    ls_st = C.c_void_p(0x70000)
    ok_ls = L.CpArmijoParams(1e-4, 0.5, 10, 0)
    assert lib.cp_gn_step_armijo(C.byref(p), X, A, C.byref(good), None, st, ls_st, ws, need,
                                 None) == L.CP_EINVAL
    assert lib.cp_gn_step_armijo(C.byref(p), X, A, C.byref(good), C.byref(ok_ls), st, None, ws,
                                 need, None) == L.CP_EINVAL
    assert lib.cp_gn_step_armijo(C.byref(p), X, A, C.byref(good), C.byref(ok_ls), None, ls_st, ws,
                                 need, None) == L.CP_EINVAL
    for bad in [L.CpArmijoParams(0.0, 0.5, 10, 0), L.CpArmijoParams(1.0, 0.5, 10, 0),
                L.CpArmijoParams(1e-4, 0.0, 10, 0), L.CpArmijoParams(1e-4, 1.0, 10, 0),
                L.CpArmijoParams(float("nan"), 0.5, 10, 0), L.CpArmijoParams(1e-4, 0.5, -1, 0),
                L.CpArmijoParams(1e-4, 0.5, 65, 0), L.CpArmijoParams(1e-4, 0.5, 10, 2)]:
        assert lib.cp_gn_step_armijo(C.byref(p), X, A, C.byref(good), C.byref(bad), st, ls_st, ws,
                                     need, None) == L.CP_EINVAL
    assert lib.cp_gn_step_armijo(C.byref(p), X, A, C.byref(L.CpGnParams(-1.0, 1e-3, 20, 0)),
                                 C.byref(ok_ls), st, ls_st, ws, need, None) == L.CP_EINVAL
    assert lib.cp_gn_step_armijo(C.byref(p), X, A, C.byref(good), C.byref(ok_ls), st, ls_st, ws,
                                 need // 2, None) == L.CP_EWORKSPACE
    assert lib.cp_als_sweep(C.byref(p), X, A, -1.0, None, ws, need, None) == L.CP_EINVAL
    assert lib.cp_residual(C.byref(p), X, A, 2, C.c_void_p(0x60000), ws, need, None) == L.CP_EINVAL
    assert lib.cp_residual(C.byref(p), X, A, 0, None, ws, need, None) == L.CP_EINVAL
    assert lib.cp_gn_jtj_matvec(C.byref(p), A, A, -1.0, A, ws, need, None) == L.CP_EINVAL
    assert lib.cp_gn_gradient(C.byref(p), X, A, L.PTRS(), None, ws, need, None) == L.CP_EINVAL
    # the triangular-solve preconditioner keeps its operands in 64 KB of LDS: R <= 128
    pc = prob(rank=129)
    _, need3 = ws_bytes(lib, pc)
    chol = L.CpGnParams(1e-3, 1e-3, 20, L.GN_CHOL_PRECOND)
    assert lib.cp_gn_step(C.byref(pc), X, A, C.byref(chol), st, ws, need3, None) == L.CP_EUNSUPPORTED
    assert lib.cp_gn_step_armijo(C.byref(pc), X, A, C.byref(chol), C.byref(ok_ls), st, ls_st, ws,
                                 need3, None) == L.CP_EUNSUPPORTED


def test_status_strings(lib):
    for code in range(0, -8, -1):
        assert len(L.status_string(code)) > 0
    assert L.status_string(-99) == "unknown status"


def test_damping_schedule_matches_oracle_definition():
    a = DampingSchedule(1e-4, 1e-10, 1e-4, 2.0)
    b = O.LambdaSchedule(1e-4, 1e-10, 1e-4, 2.0)
    for _ in range(100):
        assert a.value == b.value
        a.advance()
        b.advance()
    s = DampingSchedule(1.0, 0.25, 1.0, 2.0)
    seq = [s.value] + [s.advance() for _ in range(6)]
    assert seq == [1.0, 0.5, 0.25, 0.5, 1.0, 0.5, 0.25]


def test_gn_flag_constant_matches_header():
    text = open(os.path.join(ROOT, "include", "cpgn.h")).read()
    m = re.search(r"#define\s+CP_GN_DIAG_DAMPING\s+(\d+)u", text)
    assert m and int(m.group(1)) == L.GN_DIAG_DAMPING
    m = re.search(r"#define\s+CP_GN_CHOL_PRECOND\s+(\d+)u", text)
    assert m and int(m.group(1)) == L.GN_CHOL_PRECOND


def test_mode_longer_than_one_row_tile_grid_is_planned(lib):
    """A 2.2-million-row mode needs more than 65535 MTTKRP row tiles (the grid-y limit) in FP64
    and FP32: the launches are split into chunks of row tiles, so the plan accepts it."""
    n = C.c_size_t(0)
    for dt in (L.CP_F64, L.CP_F32):
        p = prob(dims=(2_200_000, 3, 4), rank=4, dt=dt)
        for op in range(7):
            assert lib.cp_workspace_bytes(C.byref(p), op, C.byref(n)) == L.CP_OK


def test_noalloc_step_rejects_problems_beyond_its_scratch(lib):
    """cp_gn_step_noalloc checks the problem against its built-in 64 MiB scratch before it
    touches the device: a 1000^3 rank-208 FP64 step (about 289 MiB of workspace) is refused with
    CP_ESCRATCH, and null pointers with CP_EINVAL."""
    p = L.CpProblem()
    p.order, p.rank = 3, 208
    for i in range(3):
        p.dims[i] = 1000
    p.x_dtype = p.f_dtype = L.CP_F64
    n = C.c_size_t(0)
    assert lib.cp_workspace_bytes(C.byref(p), L.OP_GN_STEP, C.byref(n)) == L.CP_OK
    assert n.value > L.NOALLOC_SCRATCH_BYTES
    good = L.CpGnParams(1e-4, 1e-3, 20, 0)
    X, st = C.c_void_p(0x10000), C.c_void_p(0x50000)
    assert lib.cp_gn_step_noalloc(C.byref(p), X, fake_ptrs(), C.byref(good), st, None) == L.CP_ESCRATCH
    assert "scratch" in L.status_string(L.CP_ESCRATCH)
    q = prob()
    assert lib.cp_gn_step_noalloc(C.byref(q), None, fake_ptrs(), C.byref(good), st, None) == L.CP_EINVAL
    assert lib.cp_gn_step_noalloc(C.byref(q), X, fake_ptrs(), None, st, None) == L.CP_EINVAL
    A0 = fake_ptrs()
    A0[1] = 0
    assert lib.cp_gn_step_noalloc(C.byref(q), X, A0, C.byref(good), st, None) == L.CP_EINVAL
