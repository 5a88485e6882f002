// C ABI of libcpgn.so: argument validation, workspace carving and launch sequencing for
// Gauss-Newton (Algorithms 1 and 2 of Singh, Ma, Yang, Solomonik, arXiv:1910.12331) and
// ALS (Section 2.2). Every call enqueues on the caller's stream and returns; FP64 CG scalars
// stay on the device, so a whole Gauss-Newton step runs without a host synchronisation.
#include <math.h>
#include <string.h>

#include <mutex>

#include "batch.h"

#include <vector>

namespace cpgn {

// Launchers defined in the other translation units.
void launch_gram2(const Dims&, const double*, const double*, double*, int, const CgState*, hipStream_t);
void launch_gamma(const Dims&, const double*, double*, hipStream_t);
void launch_ycore(const Dims&, const double*, const double*, double*, const CgState*, hipStream_t);
int rowmm_blocks(const Dims&);
void launch_to64(const Dims&, const PerMode<const void*>&, int, double*, hipStream_t);
void launch_fin_grad(const Dims&, int, const double*, CgState*, double, double*, hipStream_t);
void launch_state_reset(CgState*, hipStream_t);
void launch_gn_apply(const Dims&, double*, const double*, const PerMode<void*>&, int, double*,
                     const CgState*, hipStream_t);
void launch_gn_stats(const Dims&, int, const double*, const CgState*, cp_gn_stats*, hipStream_t);
void launch_status_out(const CgState*, int32_t*, hipStream_t);
void launch_timestamp(int64_t*, hipStream_t);
int spd_inv_supported(int);
int launch_spd_inv(int, const double*, int64_t, double, double*, int64_t, int, int, CgState*,
                   hipStream_t, bool diag_damping = false, const double* lam_dev = nullptr,
                   double* tmp = nullptr);
int als_supported(int);
int launch_als_solve_big(int R, int64_t s, const double* G, int64_t g_stride, double lambda,
                         double* L, int64_t l_stride, double* Dinv, double* stage, int mode,
                         const double* M, double* Y, double* A64, void* Aout, int dtype,
                         CgState* st, hipStream_t hs);
void launch_cgw_zero(const Dims&, double*, const CgState*, hipStream_t);
void launch_cgw_check(const Dims&, const double*, const double*, CgState*, int, bool,
                      hipStream_t);
void launch_cgw_dir(const Dims&, const double*, double*, const CgState*, int, hipStream_t);
void launch_cgw_damp(const Dims&, const double*, double*, const double*, double, const double*,
                     bool, double*, const CgState*, hipStream_t);
void launch_cgw_alpha(const Dims&, const double*, CgState*, int, hipStream_t);
void launch_cgw_update(const Dims&, double*, double*, const double*, const double*, double*,
                       const CgState*, hipStream_t);
int launch_spd_chol(int, const double*, int64_t, double, double*, int64_t, int, int, CgState*,
                    hipStream_t, bool diag_damping, const double* lam_dev);
void launch_damping_advance(double*, hipStream_t);
void launch_ls_gv(const Dims&, const double*, const double*, double*, CgState*, hipStream_t);
void launch_ls_init(int, const double*, CgState*, hipStream_t);
void launch_ls_init_given(const cp_armijo_stats*, CgState*, hipStream_t);
void launch_ls_trial(const Dims&, const double*, const double*, const PerMode<void*>&, int, void*,
                     const CgState*, hipStream_t);
void launch_ls_check(int, const double*, CgState*, double, double, hipStream_t);
void launch_ls_final(const Dims&, const double*, const double*, const PerMode<void*>&, int,
                     double*, const CgState*, cp_armijo_stats*, hipStream_t);
int launch_residual_direct(const Plan&, const void*, void*, double*, hipStream_t,
                           const int32_t* skip = nullptr, int* nblocks = nullptr);
int launch_sumsq(const Plan&, const void*, double*, hipStream_t, int*);
void launch_fin_residual_expansion(const Dims&, int, const double*, const double*, const double*,
                                   const double*, double*, hipStream_t);
int launch_prepare_factors_src(const Plan&, const void* const*, int, void*, hipStream_t, bool,
                               unsigned krp_modes = ~0u);
size_t cg_slot_bytes(const Plan&);
int launch_cg(const Plan&, const Dims&, const double*, const double*, const double*, double*,
              double*, double*, double*, double*, double*, double*, double*, void*, CgState*,
              double, int, bool, hipStream_t, const double* lam_dev = nullptr, bool chol = false);
size_t cg_args_bytes();
void launch_cg_store(const Plan& p, const Dims& d, const double* A64, const double* gam,
                     const double* pinv, double* V, double* R0, double* R1, double* Z, double* W0,
                     double* W1, double* Q, double* B, void* slots, CgState* st, double lambda,
                     bool diag_damping, const double* lam_dev, void* dst, hipStream_t s);
int launch_cg_batch(int count, const Plan* plans, void* const* args, int maxiter, hipStream_t s);

void launch_rowmm(const Dims&, const RowMM&, const CgState*, hipStream_t);
int launch_chol_tiles(int, const double*, int64_t, double, double*, int64_t, double*, int64_t, int,
                      int, CgState*, hipStream_t);
int launch_chol_rows(int, int64_t, const double*, const double*, const double*, void*, int,
                     const CgState*, hipStream_t);
int64_t ttm_rows(const Plan&);
int launch_ttm_last(const Plan&, const void*, void*, void*, hipStream_t);
void launch_ttm_contract(const Plan&, const void*, const double*, int, double*, hipStream_t);

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// MTTKRP tile shape of the plans made on this host thread (cp_set_tuning; zeros: defaults).
static thread_local cp_tuning t_tuning = {0, 0, 0, 0};

int make_plan(const cp_problem* prob, Plan* p) {
  if (!prob || !p) return CP_EINVAL;
  if (prob->order < 2 || prob->order > kMaxOrder || prob->rank < 1) return CP_EINVAL;
  const bool native = prob->x_dtype == prob->f_dtype &&
                      (prob->x_dtype == CP_F64 || prob->x_dtype == CP_F32);
  const bool bf16 = prob->f_dtype == CP_F32 &&
                    (prob->x_dtype == CP_BF16 || prob->x_dtype == CP_BF16X3);
  if (!native && !bf16) return CP_EUNSUPPORTED;
  *p = Plan{};
  if (t_tuning.mttkrp_min_items) p->mt_min_items = t_tuning.mttkrp_min_items;
  if (t_tuning.mttkrp_wg_per_cu) p->mt_wg_per_cu = t_tuning.mttkrp_wg_per_cu;
  p->mt_row_block = t_tuning.mttkrp_row_block;
  p->N = prob->order;
  p->R = prob->rank;
  if (p->R > (1 << 20)) return CP_EINVAL;
  p->Rp = (p->R + 15) / 16 * 16;
  p->NBt = p->Rp / 16;
  p->dtype = prob->f_dtype;
  p->xk = prob->x_dtype == CP_BF16 ? 1 : prob->x_dtype == CP_BF16X3 ? 2 : 0;
  p->esz = p->dtype == CP_F64 ? 8 : 4;
  p->total = 1;
  for (int n = 0; n < p->N; ++n) {
    const int64_t s = prob->dims[n];
    if (s < 1) return CP_EINVAL;
    if (p->total > ((int64_t)1 << 50) / s) return CP_EINVAL;
    p->s[n] = s;
    p->total *= s;
    p->sum_s += s;
    p->max_s = s > p->max_s ? s : p->max_s;
  }
  p->qc_last = (p->s[p->N - 1] + 15) / 16;
  p->qc_prev = (p->s[p->N - 2] + 15) / 16;
  int64_t part = p->qc_last * 16 * p->Rp;   // residual's packed last factor reuses this region
  int64_t p1 = 0;
  int64_t krp = 0;
  // Dimension tree for modes 0 .. N-2: order 3 always; higher orders while the tree partials
  // and Pm (FP64, one row per outer index) take at most a quarter of X's bytes
  const int64_t n_outer_idx = p->total / (p->s[0] * p->s[p->N - 1]);
  if (p->xk == 0 && p->N == 3) p->tree = true;
  if (p->xk == 0 && p->N >= 4) {
    const MttkrpGeom g = mttkrp_geom(*p, 0, true, true);
    const double extra = (double)g.RT * g.O * g.HS * p->Rp * p->esz + (double)n_outer_idx * p->R * 8;
    p->tree = extra <= 0.25 * (double)p->total * p->esz;
  }
  for (int n = 0; n < p->N && p->xk != 0; ++n) {
    const MttkrpGeom g = mttkrp_geom_bf16(*p, n);
    const int64_t e = g.SW * g.RT * g.rows_per_tile * p->Rp;
    part = e > part ? e : part;
    krp += g.O * p->Rp;
  }
  for (int n = 0; n < p->N && p->xk == 0; ++n) {
    for (int v = 0; v < 4; ++v) {   // geometry of every launch form (vector loads, tree)
      const bool dt = v >= 2;
      if (dt && !(n == 0 && p->tree)) continue;
      const MttkrpGeom g = mttkrp_geom(*p, n, (v & 1) == 1, dt);
      const int64_t e = g.SW * g.RT * g.rows_per_tile * p->Rp;
      part = e > part ? e : part;
      if (dt) {
        const int64_t e1 = g.RT * g.O * g.HS * p->Rp;
        p1 = e1 > p1 ? e1 : p1;
      }
    }
  }
  p->part_elems = part;
  const int64_t RR = (int64_t)p->R * p->R;
  const size_t vec = (size_t)p->sum_s * p->R * 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  p->off_apad = take((size_t)p->sum_s * p->Rp * p->esz);
  // packed inner factors: 16-row chunks in the compute precision, or FP32 32-row chunks for
  // a bfloat16 tensor
  const size_t fl = p->xk ? (size_t)(p->s[p->N - 1] + 31) / 32 * p->NBt * 2048
                          : (size_t)p->qc_last * p->NBt * 256 * p->esz;
  const size_t fp = p->xk ? (size_t)(p->s[p->N - 2] + 31) / 32 * p->NBt * 2048
                          : (size_t)p->qc_prev * p->NBt * 256 * p->esz;
  p->off_fpk_last = take(fl);
  p->off_fpk_prev = take(fp);
  p->off_part = take((size_t)part * p->esz);
  p->off_p1 = take((size_t)p1 * p->esz);
  p->off_m64 = take(vec);
  p->off_a64 = take(vec);
  p->off_s = take((size_t)p->N * RR * 8);
  p->off_gam = take((size_t)p->N * p->N * RR * 8);
  p->off_pinv = take((size_t)p->N * RR * 8);
  p->off_dinv = take((size_t)p->N * ((p->R + 15) / 16) * 256 * 8);
  p->off_g = take(vec);
  p->off_v = take(vec);
  p->off_r = take(vec);
  p->off_z = take(vec);
  p->off_w = take(vec);
  p->off_q = take(vec);
  p->off_bp = take((size_t)p->N * RR * 8);
  p->off_y = take((size_t)p->N * RR * 8);
  p->off_red = take((size_t)3 * p->N * kRedSlots * 8);
  p->off_state = take(sizeof(CgState));
  p->off_w1 = take(vec);
  p->off_r1 = take(vec);
  p->off_slots = take(cg_slot_bytes(*p));
  p->off_cgargs = take(cg_args_bytes());
  p->off_krp = take((size_t)krp * 4);
  if (p->tree && p->N >= 4) p->off_pm = take((size_t)n_outer_idx * p->R * 8);
  p->bytes = off;
  // the T pass launches one grid row per row tile of s0 s1 (at most 65535); the contraction of
  // T keeps one output row's R values in one workgroup's lanes (R <= 128)
  if (p->N == 3 && p->xk == 0 && p->R <= 128 &&
      ttm_rows(*p) / (16 * (p->dtype == CP_F64 ? 2 : 4)) <= 65535)
    p->t_bytes = align256((size_t)ttm_rows(*p) * p->Rp * p->esz);
  return CP_OK;
}

Dims make_dims(const Plan& p) {
  Dims d{};
  d.N = p.N;
  d.R = p.R;
  d.Rp = p.Rp;
  d.off[0] = 0;
  for (int n = 0; n < p.N; ++n) {
    d.s[n] = p.s[n];
    d.off[n + 1] = d.off[n] + p.s[n];
  }
  return d;
}

// Pointers into a carved workspace.
struct Ws {
  char* base;
  double *m64, *a64, *S, *gam, *pinv, *g, *v, *r, *z, *w, *q, *bp, *y, *red_dot, *red_nrm,
      *red_wq;
  CgState* st;
};

static Ws carve(const Plan& p, void* ws) {
  Ws w{};
  w.base = (char*)ws;
  w.m64 = (double*)(w.base + p.off_m64);
  w.a64 = (double*)(w.base + p.off_a64);
  w.S = (double*)(w.base + p.off_s);
  w.gam = (double*)(w.base + p.off_gam);
  w.pinv = (double*)(w.base + p.off_pinv);
  w.g = (double*)(w.base + p.off_g);
  w.v = (double*)(w.base + p.off_v);
  w.r = (double*)(w.base + p.off_r);
  w.z = (double*)(w.base + p.off_z);
  w.w = (double*)(w.base + p.off_w);
  w.q = (double*)(w.base + p.off_q);
  w.bp = (double*)(w.base + p.off_bp);
  w.y = (double*)(w.base + p.off_y);
  w.red_dot = (double*)(w.base + p.off_red);
  w.red_nrm = w.red_dot + (size_t)p.N * kRedSlots;
  w.red_wq = w.red_nrm + (size_t)p.N * kRedSlots;
  w.st = (CgState*)(w.base + p.off_state);
  return w;
}

static int check_ws(const Plan& p, void* ws, size_t ws_bytes) {
  if (!ws) return CP_EINVAL;
  if ((uintptr_t)ws % 256 != 0) return CP_EINVAL;
  if (ws_bytes < p.bytes) return CP_EWORKSPACE;
  return CP_OK;
}

static int check_ptrs(const Plan& p, const void* const* A) {
  if (!A) return CP_EINVAL;
  for (int n = 0; n < p.N; ++n)
    if (!A[n]) return CP_EINVAL;
  return CP_OK;
}

static int hip_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CP_OK : CP_EHIP;
}

// Gradient of Algorithm 1 into w.g (and R = -G into w.r); fills the per-mode norm partials and
// resets the CG state (gsum, eps). Requires prepared factors (Apad, Fpk, A64).
static void gradient_core(const Plan& p, const Dims& d, const void* X, const Ws& w, double eps,
                          const PerMode<void*>& cast_g, double* gsum_out, hipStream_t st) {
  launch_gram2(d, w.a64, w.a64, w.S, -1, nullptr, st);
  launch_gamma(d, w.S, w.gam, st);
  // modes 0 .. N-2 (the dimension tree: one pass over X where it applies), then mode N-1
  double* m64[kMaxOrder];
  void* mout[kMaxOrder] = {};
  int64_t off = 0;
  for (int n = 0; n < p.N; ++n) {
    m64[n] = w.m64 + off * p.R;
    off += p.s[n];
  }
  launch_mttkrp_lead(p, X, w.base, m64, mout, st);
  launch_mttkrp(p, X, p.N - 1, w.base, m64[p.N - 1], nullptr, st);
  const int64_t RR = (int64_t)p.R * p.R;
  RowMM a{};
  a.in = w.m64;
  a.cin = -1.0;
  a.l1 = w.a64;
  a.t1 = w.gam;
  a.t1_stride = (int64_t)(p.N + 1) * RR;
  a.out = w.g;
  a.out2 = w.r;
  a.out2_scale = -1.0;
  a.red_nrm = w.red_nrm;
  a.cast_out = cast_g;
  a.cast_dtype = p.dtype;
  a.mode_only = -1;
  launch_rowmm(d, a, nullptr, st);
  launch_fin_grad(d, rowmm_blocks(d), w.red_nrm, w.st, eps, gsum_out, st);
}

// Q = lambda W + sum_p MatVec (eq. (7)) on FP64 packed vectors; writes <W,Q> partials.
static void matvec_core(const Plan& p, const Dims& d, const Ws& w, const double* W, double lambda,
                        double* Q, const PerMode<void*>& cast_q, bool use_state, hipStream_t st) {
  const int64_t RR = (int64_t)p.R * p.R;
  const CgState* cs = use_state ? w.st : nullptr;
  launch_gram2(d, w.a64, W, w.bp, -1, cs, st);
  launch_ycore(d, w.gam, w.bp, w.y, cs, st);
  RowMM a{};
  a.in = W;
  a.cin = lambda;
  a.l1 = W;
  a.t1 = w.gam;
  a.t1_stride = (int64_t)(p.N + 1) * RR;
  a.l2 = w.a64;
  a.t2 = w.y;
  a.t2_stride = RR;
  a.out = Q;
  a.dotw = W;
  a.red_dot = w.red_dot;
  a.cast_out = cast_q;
  a.cast_dtype = p.dtype;
  a.mode_only = -1;
  launch_rowmm(d, a, cs, st);
}

}  // namespace cpgn

using namespace cpgn;

extern "C" {

int cp_abi_version(void) { return CP_ABI_VERSION; }

int cp_set_tuning(const cp_tuning* t) {
  if (!t) {
    t_tuning = cp_tuning{0, 0, 0, 0};
    return CP_OK;
  }
  if (t->mttkrp_min_items < 0 || t->mttkrp_min_items > 4096) return CP_EINVAL;
  if (t->mttkrp_wg_per_cu < 0 || t->mttkrp_wg_per_cu > 8) return CP_EINVAL;
  if (t->mttkrp_row_block != 0 && t->mttkrp_row_block != 2 && t->mttkrp_row_block != 4 &&
      t->mttkrp_row_block != 5)
    return CP_EINVAL;
  if (t->reserved != 0) return CP_EINVAL;
  t_tuning = *t;
  return CP_OK;
}

int cp_get_tuning(cp_tuning* t) {
  if (!t) return CP_EINVAL;
  *t = t_tuning;
  return CP_OK;
}

const char* cp_status_string(int s) {
  switch (s) {
    case CP_OK: return "ok";
    case CP_EINVAL: return "invalid argument";
    case CP_EUNSUPPORTED: return "unsupported dtype combination or size";
    case CP_EWORKSPACE: return "workspace too small";
    case CP_EHIP: return "HIP launch error";
    case CP_ENOTSPD: return "matrix not symmetric positive definite (Cholesky pivot <= 0)";
    case CP_EBREAKDOWN: return "CG breakdown (sum <W,Q> <= 0)";
    case CP_ENONFINITE: return "non-finite value";
    case CP_ESCRATCH: return "problem needs more than the built-in scratch buffer (64 MiB)";
    default: return "unknown status";
  }
}

int cp_workspace_bytes(const cp_problem* prob, int op, size_t* bytes) {
  if (!bytes) return CP_EINVAL;
  if (op < CP_OP_MTTKRP || op > CP_OP_MTTKRP_ALL) return CP_EINVAL;
  Plan p;
  const int rc = make_plan(prob, &p);
  if (rc) return rc;
  *bytes = p.bytes + (op == CP_OP_ALS_SWEEP ? p.t_bytes : 0);
  return CP_OK;
}

int cp_mttkrp_marked(const cp_problem* prob, const void* X, const void* const* A, int mode,
                     void* M, void* ws, size_t ws_bytes, void* stream, void* kernel_begin,
                     void* kernel_end) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X || !M || mode < 0 || mode >= p.N) return CP_EINVAL;
  if ((rc = check_ptrs(p, A)) || (rc = check_ws(p, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  KernelMarks mk;
  mk.before = (hipEvent_t)kernel_begin;
  mk.after = (hipEvent_t)kernel_end;
  launch_prepare_factors_src(p, A, p.dtype, ws, st, false, 1u << mode);
  launch_mttkrp(p, X, mode, ws, nullptr, M, st, mk);
  return hip_status();
}

int cp_mttkrp(const cp_problem* prob, const void* X, const void* const* A, int mode, void* M,
              void* ws, size_t ws_bytes, void* stream) {
  return cp_mttkrp_marked(prob, X, A, mode, M, ws, ws_bytes, stream, nullptr, nullptr);
}

int cp_mttkrp_all(const cp_problem* prob, const void* X, const void* const* A, void* const* M,
                  void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X) return CP_EINVAL;
  if ((rc = check_ptrs(p, A)) || (rc = check_ptrs(p, (const void* const*)M)) ||
      (rc = check_ws(p, ws, ws_bytes)))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  launch_prepare_factors_src(p, A, p.dtype, ws, st, false);
  // modes 0 .. N-2 (the dimension tree: one pass over X where it applies), then mode N-1
  double* m64[kMaxOrder] = {};
  int rc2 = launch_mttkrp_lead(p, X, ws, m64, M, st);
  if (!rc2) rc2 = launch_mttkrp(p, X, p.N - 1, ws, nullptr, M[p.N - 1], st);
  if (rc2) return rc2;
  return hip_status();
}

int cp_gn_gradient(const cp_problem* prob, const void* X, const void* const* A, void* const* G,
                   double* grad_norm_sum_dev, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X) return CP_EINVAL;
  if ((rc = check_ptrs(p, A)) || (rc = check_ptrs(p, (const void* const*)G)) ||
      (rc = check_ws(p, ws, ws_bytes)))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  launch_prepare_factors_src(p, A, p.dtype, ws, st, true);
  PerMode<void*> cg{};
  for (int n = 0; n < p.N; ++n) cg.p[n] = G[n];
  gradient_core(p, d, X, w, 0.0, cg, grad_norm_sum_dev, st);
  return hip_status();
}

int cp_objective_gradient(const cp_problem* prob, const void* X, const void* const* A,
                          void* const* G, double* res_dev, void* ws, size_t ws_bytes,
                          void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X || !res_dev) return CP_EINVAL;
  if ((rc = check_ptrs(p, A)) || (rc = check_ptrs(p, (const void* const*)G)) ||
      (rc = check_ws(p, ws, ws_bytes)))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  launch_prepare_factors_src(p, A, p.dtype, ws, st, true);
  PerMode<void*> cg{};
  for (int n = 0; n < p.N; ++n) cg.p[n] = G[n];
  gradient_core(p, d, X, w, 0.0, cg, nullptr, st);
  // ||X - [[A]]||^2 = ||X||^2 - 2 <M(0), A(0)> + sum_{r,z} prod_m S(m)[r,z] from the same M(0)
  // and Grams: one more pass over X, for ||X||^2, with no matrix work
  int nblocks = 0;
  launch_sumsq(p, X, w.red_dot, st, &nblocks);
  launch_fin_residual_expansion(d, nblocks, w.red_dot, w.m64, w.a64, w.S, res_dev, st);
  return hip_status();
}

int cp_gn_jtj_matvec(const cp_problem* prob, const void* const* A, const void* const* W,
                     double lambda, void* const* Q, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!(lambda >= 0.0) || !isfinite(lambda)) return CP_EINVAL;
  if ((rc = check_ptrs(p, A)) || (rc = check_ptrs(p, W)) ||
      (rc = check_ptrs(p, (const void* const*)Q)) || (rc = check_ws(p, ws, ws_bytes)))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  PerMode<const void*> src{};
  for (int n = 0; n < p.N; ++n) src.p[n] = A[n];
  launch_to64(d, src, p.dtype, w.a64, st);
  for (int n = 0; n < p.N; ++n) src.p[n] = W[n];
  launch_to64(d, src, p.dtype, w.w, st);
  launch_gram2(d, w.a64, w.a64, w.S, -1, nullptr, st);
  launch_gamma(d, w.S, w.gam, st);
  PerMode<void*> cq{};
  for (int n = 0; n < p.N; ++n) cq.p[n] = Q[n];
  matvec_core(p, d, w, w.w, lambda, w.q, cq, false, st);
  return hip_status();
}

// One Gauss-Newton step; the damping is prm->lambda, or *lam_dev read on the device.
// One Gauss-Newton step: the direction V of Algorithm 1, then either the full step A += V or,
// with ls, the Armijo search along V (Section 5).
// Checks of the Gauss-Newton parameters shared by every step entry point.
static int gn_params_ok(const Plan& p, const cp_gn_params* prm, const double* lam_dev) {
  if (!lam_dev && (!(prm->lambda >= 0.0) || !isfinite(prm->lambda))) return CP_EINVAL;
  if (!(prm->cg_tol >= 0.0) || !isfinite(prm->cg_tol) || prm->cg_maxiter < 0 ||
      (prm->flags & ~(CP_GN_DIAG_DAMPING | CP_GN_CHOL_PRECOND)) != 0)
    return CP_EINVAL;
  if (!spd_inv_supported(p.R)) return CP_EUNSUPPORTED;
  if ((prm->flags & CP_GN_CHOL_PRECOND) && p.R > 128) return CP_EUNSUPPORTED;
  return CP_OK;
}

// The part of a step before CG: prepared factors, gradient (Algorithm 1), preconditioner.
static void gn_pre_cg(const Plan& p, const Dims& d, const Ws& w, const void* X, void* const* A,
                      const cp_gn_params* prm, const double* lam_dev, void* ws, hipStream_t st) {
  const int64_t RR = (int64_t)p.R * p.R;
  const double lam = lam_dev ? 0.0 : prm->lambda;
  launch_prepare_factors_src(p, (const void* const*)A, p.dtype, ws, st, true);
  PerMode<void*> none{};
  gradient_core(p, d, X, w, prm->cg_tol, none, nullptr, st);
  // Preconditioner P_inv(n) = (Gamma(n,n) + lambda I)^-1.
  const bool diag = (prm->flags & CP_GN_DIAG_DAMPING) != 0;
  if (prm->flags & CP_GN_CHOL_PRECOND)   // Cholesky factors, applied by triangular solves in CG
    launch_spd_chol(p.R, w.gam, (int64_t)(p.N + 1) * RR, lam, w.pinv, RR, 0, p.N, w.st, st, diag,
                    lam_dev);
  else   // (above kMaxGnRank the inverse works in global memory, with Y's buffer as scratch)
    launch_spd_inv(p.R, w.gam, (int64_t)(p.N + 1) * RR, lam, w.pinv, RR, 0, p.N, w.st, st, diag,
                   lam_dev, w.y);
}

// CG of Algorithm 2 for R > kMaxGnRank (the fixed-rank CG kernels hold operand rows of up to
// kMaxGnRank values in registers): the same iteration from the generic product kernels, with
// the scalars on the device (see the k_cgw_* kernels).
static void cg_wide(const Plan& p, const Dims& d, const Ws& w, double lam, const double* lam_dev,
                    bool diag, int maxiter, hipStream_t st) {
  const int64_t RR = (int64_t)p.R * p.R;
  launch_cgw_zero(d, w.v, w.st, st);
  RowMM z{};   // Z = R P_inv and the partials of <Z, R>
  z.l1 = w.r;
  z.t1 = w.pinv;
  z.t1_stride = RR;
  z.out = w.z;
  z.dotw = w.r;
  z.red_dot = w.red_dot;
  z.mode_only = -1;
  RowMM q{};   // Q0 = W Gamma(n,n) + A(n) Y(n)^T, eq. (7)
  q.l1 = w.w;
  q.t1 = w.gam;
  q.t1_stride = (int64_t)(p.N + 1) * RR;
  q.l2 = w.a64;
  q.t2 = w.y;
  q.t2_stride = RR;
  q.out = w.q;
  q.mode_only = -1;
  launch_rowmm(d, z, w.st, st);
  for (int it = 0; it < maxiter; ++it) {
    launch_cgw_check(d, w.red_dot, w.red_nrm, w.st, it, false, st);
    launch_cgw_dir(d, w.z, w.w, w.st, it, st);
    launch_gram2(d, w.a64, w.w, w.bp, -1, w.st, st);
    launch_ycore(d, w.gam, w.bp, w.y, w.st, st);
    launch_rowmm(d, q, w.st, st);
    launch_cgw_damp(d, w.w, w.q, w.gam, lam, lam_dev, diag, w.red_wq, w.st, st);
    launch_cgw_alpha(d, w.red_wq, w.st, it, st);
    launch_cgw_update(d, w.v, w.r, w.w, w.q, w.red_nrm, w.st, st);
    launch_rowmm(d, z, w.st, st);
  }
  launch_cgw_check(d, w.red_dot, w.red_nrm, w.st, maxiter, true, st);
}

static int gn_step_impl(const cp_problem* prob, const void* X, void* const* A,
                        const cp_gn_params* prm, const double* lam_dev, cp_gn_stats* stats,
                        void* ws, size_t ws_bytes, void* stream,
                        const cp_armijo_params* ls = nullptr, cp_armijo_stats* ls_stats = nullptr) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X || !prm || !stats) return CP_EINVAL;
  if (ls && (!ls_stats || !(ls->c > 0.0 && ls->c < 1.0) ||
             !(ls->shrink > 0.0 && ls->shrink < 1.0) || ls->max_trials < 0 ||
             ls->max_trials > 64 || (ls->flags & ~CP_LS_F0_GIVEN) != 0))
    return CP_EINVAL;
  if ((rc = gn_params_ok(p, prm, lam_dev))) return rc;
  if ((rc = check_ptrs(p, (const void* const*)A)) || (rc = check_ws(p, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  const int nb = rowmm_blocks(d);
  const double lam = lam_dev ? 0.0 : prm->lambda;
  const bool diag = (prm->flags & CP_GN_DIAG_DAMPING) != 0;
  const bool chol = (prm->flags & CP_GN_CHOL_PRECOND) != 0;
  gn_pre_cg(p, d, w, X, A, prm, lam_dev, ws, st);
  // CG: three launches per iteration, scalars kept on the device.
  if (p.R > kMaxGnRank)
    cg_wide(p, d, w, lam, lam_dev, diag, prm->cg_maxiter, st);
  else
    launch_cg(p, d, w.a64, w.gam, w.pinv, w.v, w.r, (double*)(w.base + p.off_r1), w.z, w.w,
              (double*)(w.base + p.off_w1), w.q, w.bp, w.base + p.off_slots, w.st, lam,
              prm->cg_maxiter, diag, st, lam_dev, chol);
  PerMode<void*> aout{};
  for (int n = 0; n < p.N; ++n) aout.p[n] = A[n];
  if (!ls) {
    launch_gn_apply(d, w.a64, w.v, aout, p.dtype, w.red_nrm, w.st, st);
    launch_gn_stats(d, nb, w.red_nrm, w.st, stats, st);
    return hip_status();
  }
  // Armijo search along V: the slope <G, V>, f at the start point (the padded factor copies still
  // hold it; or the previous search's f), then max_trials trial points, each skipped on the
  // device once one has passed.
  launch_ls_gv(d, w.g, w.v, w.red_dot, w.st, st);
  int rb = 0;
  if (ls->flags & CP_LS_F0_GIVEN) {
    launch_ls_init_given(ls_stats, w.st, st);
  } else {
    launch_residual_direct(p, X, ws, nullptr, st, nullptr, &rb);
    launch_ls_init(rb, w.red_dot, w.st, st);
  }
  const int32_t* done = &w.st->ls_done;
  for (int k = 0; k < ls->max_trials; ++k) {
    launch_ls_trial(d, w.a64, w.v, aout, p.dtype, w.base + p.off_apad, w.st, st);
    launch_residual_direct(p, X, ws, nullptr, st, done, &rb);
    launch_ls_check(rb, w.red_dot, w.st, ls->c, ls->shrink, st);
  }
  launch_ls_final(d, w.a64, w.v, aout, p.dtype, w.red_nrm, w.st, ls_stats, st);
  launch_gn_stats(d, nb, w.red_nrm, w.st, stats, st);
  return hip_status();
}

int cp_gn_step(const cp_problem* prob, const void* X, void* const* A, const cp_gn_params* prm,
               cp_gn_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  return gn_step_impl(prob, X, A, prm, nullptr, stats, ws, ws_bytes, stream);
}

int cp_gn_step_devlam(const cp_problem* prob, const void* X, void* const* A,
                      const cp_gn_params* prm, const double* lambda_dev, cp_gn_stats* stats,
                      void* ws, size_t ws_bytes, void* stream) {
  if (!lambda_dev) return CP_EINVAL;
  return gn_step_impl(prob, X, A, prm, lambda_dev, stats, ws, ws_bytes, stream);
}

int cp_gn_step_begin(const cp_problem* prob, const void* X, void* const* A,
                     const cp_gn_params* prm, const double* lambda_dev, void* ws, size_t ws_bytes,
                     void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X || !prm) return CP_EINVAL;
  if ((rc = gn_params_ok(p, prm, lambda_dev))) return rc;
  if (p.R > 128 || (prm->flags & CP_GN_CHOL_PRECOND)) return CP_EUNSUPPORTED;
  if ((rc = check_ptrs(p, (const void* const*)A)) || (rc = check_ws(p, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  gn_pre_cg(p, d, w, X, A, prm, lambda_dev, ws, st);
  launch_cg_store(p, d, w.a64, w.gam, w.pinv, w.v, w.r, (double*)(w.base + p.off_r1), w.z, w.w,
                  (double*)(w.base + p.off_w1), w.q, w.bp, w.base + p.off_slots, w.st,
                  lambda_dev ? 0.0 : prm->lambda, (prm->flags & CP_GN_DIAG_DAMPING) != 0,
                  lambda_dev, w.base + p.off_cgargs, st);
  return hip_status();
}

int cp_gn_cg_batch(int count, const cp_problem* probs, void* const* ws, const size_t* ws_bytes,
                   int cg_maxiter, void* stream) {
  if (count < 1 || count > CP_MAX_CG_BATCH || !probs || !ws || !ws_bytes || cg_maxiter < 0)
    return CP_EINVAL;
  std::vector<Plan> plans((size_t)count);
  std::vector<void*> args((size_t)count);
  for (int i = 0; i < count; ++i) {
    int rc = make_plan(&probs[i], &plans[i]);
    if (rc) return rc;
    if (plans[i].R > 128) return CP_EUNSUPPORTED;
    if ((rc = check_ws(plans[i], ws[i], ws_bytes[i]))) return rc;
    args[i] = (char*)ws[i] + plans[i].off_cgargs;
  }
  launch_cg_batch(count, plans.data(), args.data(), cg_maxiter, (hipStream_t)stream);
  return hip_status();
}

int cp_gn_step_end(const cp_problem* prob, void* const* A, cp_gn_stats* stats, void* ws,
                   size_t ws_bytes, void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!stats) return CP_EINVAL;
  if ((rc = check_ptrs(p, (const void* const*)A)) || (rc = check_ws(p, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  PerMode<void*> aout{};
  for (int n = 0; n < p.N; ++n) aout.p[n] = A[n];
  launch_gn_apply(d, w.a64, w.v, aout, p.dtype, w.red_nrm, w.st, st);
  launch_gn_stats(d, rowmm_blocks(d), w.red_nrm, w.st, stats, st);
  return hip_status();
}

}  // extern "C"

// Workspace of cp_gn_step_noalloc: one copy per GPU, resident until the process ends. Host code
// never uses the array's name as an address: kernels get the device address that
// hipGetSymbolAddress returns for the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[CP_NOALLOC_SCRATCH_BYTES];
static constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

static int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return CP_EHIP;
  if (dev < 0 || dev >= kMaxScratchDevices) return CP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CP_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CP_OK;
}

extern "C" {

int cp_gn_step_noalloc(const cp_problem* prob, const void* X, void* const* A,
                       const cp_gn_params* prm, cp_gn_stats* stats, void* stream) {
  size_t need = 0;
  int rc = cp_workspace_bytes(prob, CP_OP_GN_STEP, &need);
  if (rc) return rc;
  if (need > CP_NOALLOC_SCRATCH_BYTES) return CP_ESCRATCH;
  if (!X || !prm || !stats) return CP_EINVAL;
  Plan p;
  if ((rc = make_plan(prob, &p)) || (rc = check_ptrs(p, (const void* const*)A))) return rc;
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return gn_step_impl(prob, X, A, prm, nullptr, stats, ws, CP_NOALLOC_SCRATCH_BYTES, stream);
}

int cp_gn_step_armijo(const cp_problem* prob, const void* X, void* const* A,
                      const cp_gn_params* prm, const cp_armijo_params* ls, cp_gn_stats* stats,
                      cp_armijo_stats* ls_stats, void* ws, size_t ws_bytes, void* stream) {
  if (!ls) return CP_EINVAL;
  return gn_step_impl(prob, X, A, prm, nullptr, stats, ws, ws_bytes, stream, ls, ls_stats);
}

int cp_damping_advance(double* state_dev, void* stream) {
  if (!state_dev) return CP_EINVAL;
  launch_damping_advance(state_dev, (hipStream_t)stream);
  return hip_status();
}

int cp_device_timestamp(int64_t* dst_dev, void* stream) {
  if (!dst_dev) return CP_EINVAL;
  launch_timestamp(dst_dev, (hipStream_t)stream);
  return hip_status();
}

int cp_device_clock_hz(int64_t* hz) {
  if (!hz) return CP_EINVAL;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return CP_EHIP;
  *hz = (int64_t)khz * 1000;
  return CP_OK;
}

int cp_als_sweep(const cp_problem* prob, const void* X, void* const* A, double lambda,
                 int32_t* status_dev, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X || !(lambda >= 0.0) || !isfinite(lambda)) return CP_EINVAL;
  if (!als_supported(p.R)) return CP_EUNSUPPORTED;
  if ((rc = check_ptrs(p, (const void* const*)A)) || (rc = check_ws(p, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  const int64_t RR = (int64_t)p.R * p.R;
  launch_state_reset(w.st, st);
  launch_prepare_factors_src(p, (const void* const*)A, p.dtype, ws, st, true, 1u);
  launch_gram2(d, w.a64, w.a64, w.S, -1, nullptr, st);
  // Order 3 with room for T (the ALS workspace query includes it): modes 0 and 1 share
  // T = X x_3 A(2) (Section 2.2, dimension tree), since A(2) changes only at the end of the
  // sweep; M(0) and M(1) are then O(s0 s1 R) contractions of T with the latest factors.
  const bool tree = p.t_bytes > 0 && ws_bytes >= p.bytes + p.t_bytes;
  void* Tbuf = w.base + p.bytes;
  if (tree) launch_ttm_last(p, X, ws, Tbuf, st);
  int64_t off = 0;
  for (int n = 0; n < p.N; ++n) {
    launch_gamma(d, w.S, w.gam, st);
    double* m64n = w.m64 + off * p.R;
    if (tree && n < 2)
      launch_ttm_contract(p, Tbuf, w.a64 + (n == 0 ? p.s[0] * p.R : 0), n, m64n, st);
    else
      launch_mttkrp(p, X, n, ws, m64n, nullptr, st);
    // A(n) = M(n) (Gamma(n) + lambda I)^-1: FP64 Cholesky factor L, then Y L^T = M(n) and
    // A(n) L = Y by substitution (skipped, factors unchanged, when a pivot is not positive)
    double* dinv = (double*)(w.base + p.off_dinv);
    const int64_t dstride = (int64_t)((p.R + 15) / 16) * 256;
    if (p.R > kMaxGnRank) {   // L in global memory, tiles streamed (the Y and CG buffers as scratch)
      launch_als_solve_big(p.R, p.s[n], w.gam, (int64_t)(p.N + 1) * RR, lambda, w.pinv, RR,
                           dinv + n * dstride, w.y, n, m64n, w.z, w.v, A[n], p.dtype, w.st, st);
    } else {
      launch_chol_tiles(p.R, w.gam, (int64_t)(p.N + 1) * RR, lambda, w.pinv, RR, dinv, dstride,
                        n, 1, w.st, st);
      launch_chol_rows(p.R, p.s[n], m64n, w.pinv + n * RR, dinv + n * dstride, A[n], p.dtype,
                       w.st, st);
    }
    // refresh the padded/packed copies, the FP64 copy and the Gram of the updated mode
    launch_prepare_factors_src(p, (const void* const*)A, p.dtype, ws, st, true, 1u << (n + 1));
    launch_gram2(d, w.a64, w.a64, w.S, n, nullptr, st);
    off += p.s[n];
  }
  if (status_dev) launch_status_out(w.st, status_dev, st);
  return hip_status();
}

int cp_residual(const cp_problem* prob, const void* X, const void* const* A, int method,
                double* out_dev, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int rc = make_plan(prob, &p);
  if (rc) return rc;
  if (!X || !out_dev) return CP_EINVAL;
  if (method != CP_RESIDUAL_DIRECT && method != CP_RESIDUAL_EXPANSION) return CP_EINVAL;
  if ((rc = check_ptrs(p, A)) || (rc = check_ws(p, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Dims d = make_dims(p);
  const Ws w = carve(p, ws);
  launch_prepare_factors_src(p, A, p.dtype, ws, st, method == CP_RESIDUAL_EXPANSION,
                             method == CP_RESIDUAL_EXPANSION ? 1u : 0u);
  if (method == CP_RESIDUAL_DIRECT) {
    launch_residual_direct(p, X, ws, out_dev, st);
  } else {
    launch_mttkrp(p, X, 0, ws, w.m64, nullptr, st);
    launch_gram2(d, w.a64, w.a64, w.S, -1, nullptr, st);
    int nblocks = 0;
    launch_sumsq(p, X, w.red_dot, st, &nblocks);
    launch_fin_residual_expansion(d, nblocks, w.red_dot, w.m64, w.a64, w.S, out_dev, st);
  }
  return hip_status();
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Batch program: the launches of one Gauss-Newton step of many problems, recorded per problem
// once and run as one launch per (kernel, position in the step) for the whole batch.
// ---------------------------------------------------------------------------------------------
namespace cpgn {

thread_local std::vector<BatchRec>* t_batch_rec = nullptr;

// One batched launch: the members' records are in the device table at tab.blk[i].
struct BatchLaunch {
  void (*launch)(const BatchTab&, unsigned, size_t, hipStream_t) = nullptr;
  BatchTab tab{};
  unsigned blocks = 0;
  size_t lds = 0;
};

// Records the launches that `fn` makes on the calling thread (none runs).
template <class F>
static std::vector<BatchRec> record(F&& fn) {
  std::vector<BatchRec> recs;
  t_batch_rec = &recs;
  fn();
  t_batch_rec = nullptr;
  return recs;
}

// Level-synchronous schedule of per-problem chains: the j-th launches of all chains form level
// j; within a level, launches of the same kernel are merged (at most kMaxBatch members each).
// A chain's launch j + 1 runs after its launch j because levels are enqueued in order on one
// stream. Member records are appended to `bytes` (16-byte aligned); blk[] holds offsets into it
// until the table's device address is known.
static std::vector<BatchLaunch> schedule(const std::vector<std::vector<BatchRec>>& chains,
                                         std::vector<unsigned char>& bytes) {
  std::vector<BatchLaunch> out;
  size_t depth = 0;
  for (const auto& c : chains) depth = c.size() > depth ? c.size() : depth;
  for (size_t j = 0; j < depth; ++j) {
    std::vector<int> todo;
    for (int i = 0; i < (int)chains.size(); ++i)
      if (j < chains[i].size()) todo.push_back(i);
    while (!todo.empty()) {
      const BatchRec& head = chains[todo[0]][j];
      BatchLaunch L;
      L.launch = head.launch;
      std::vector<int> rest;
      for (int i : todo) {
        const BatchRec& r = chains[i][j];
        if (r.launch != head.launch || L.tab.n == kMaxBatch) {
          rest.push_back(i);
          continue;
        }
        const size_t at = (bytes.size() + 15) / 16 * 16;
        bytes.resize(at + r.blk.size());
        memcpy(bytes.data() + at, r.blk.data(), r.blk.size());
        L.tab.blk[L.tab.n] = (const unsigned char*)(uintptr_t)at;
        L.tab.off[L.tab.n] = (int)L.blocks;
        L.blocks += r.blocks;
        L.lds = r.lds > L.lds ? r.lds : L.lds;
        ++L.tab.n;
      }
      L.tab.off[L.tab.n] = (int)L.blocks;
      out.push_back(L);
      todo.swap(rest);
    }
  }
  return out;
}

}  // namespace cpgn

struct cp_gn_batch {
  std::vector<cpgn::BatchLaunch> pre, post;
  std::vector<cpgn::Plan> plans;
  std::vector<void*> cgargs;
  int cg_maxiter = 0;
};

extern "C" {

int cp_gn_batch_create(int count, const cp_problem* probs, const void* const* X, void* const* A,
                       const cp_gn_params* prm, double* const* lambda_dev,
                       double* const* damping_state, cp_gn_stats* const* stats,
                       void* const* ws, const size_t* ws_bytes, void* table, size_t table_bytes,
                       size_t* table_needed, cp_gn_batch** out) {
  if (count < 1 || !probs || !X || !A || !prm || !stats || !ws || !ws_bytes || !table_needed ||
      !out)
    return CP_EINVAL;
  if (prm->flags & CP_GN_CHOL_PRECOND) return CP_EUNSUPPORTED;
  std::vector<Plan> plans((size_t)count);
  for (int i = 0; i < count; ++i) {
    Plan& p = plans[i];
    int rc = make_plan(&probs[i], &p);
    if (rc) return rc;
    const double* lam = lambda_dev ? lambda_dev[i] : nullptr;
    if (!X[i] || !stats[i]) return CP_EINVAL;
    if ((rc = gn_params_ok(p, prm, lam))) return rc;
    if (p.R > 128 || p.xk != 0) return CP_EUNSUPPORTED;
    if ((rc = check_ptrs(p, (const void* const*)(A + (size_t)i * CP_MAX_ORDER))) ||
        (rc = check_ws(p, ws[i], ws_bytes[i])))
      return rc;
  }
  // Record each problem's launches: before CG (cp_gn_step_begin), after CG (cp_gn_step_end and
  // the damping update). Nothing is launched while recording.
  std::vector<std::vector<BatchRec>> pre((size_t)count), post((size_t)count);
  std::vector<void*> cgargs((size_t)count);
  const hipStream_t none = nullptr;
  for (int i = 0; i < count; ++i) {
    const Plan& p = plans[i];
    const Dims d = make_dims(p);
    const Ws w = carve(p, ws[i]);
    void* const* Ai = A + (size_t)i * CP_MAX_ORDER;
    const double* lam = lambda_dev ? lambda_dev[i] : nullptr;
    pre[i] = record([&] {
      gn_pre_cg(p, d, w, X[i], Ai, prm, lam, ws[i], none);
      launch_cg_store(p, d, w.a64, w.gam, w.pinv, w.v, w.r, (double*)(w.base + p.off_r1), w.z,
                      w.w, (double*)(w.base + p.off_w1), w.q, w.bp, w.base + p.off_slots, w.st,
                      lam ? 0.0 : prm->lambda, (prm->flags & CP_GN_DIAG_DAMPING) != 0, lam,
                      w.base + p.off_cgargs, none);
    });
    post[i] = record([&] {
      PerMode<void*> aout{};
      for (int n = 0; n < p.N; ++n) aout.p[n] = Ai[n];
      launch_gn_apply(d, w.a64, w.v, aout, p.dtype, w.red_nrm, w.st, none);
      launch_gn_stats(d, rowmm_blocks(d), w.red_nrm, w.st, stats[i], none);
      if (damping_state && damping_state[i]) launch_damping_advance(damping_state[i], none);
    });
    cgargs[i] = w.base + p.off_cgargs;
  }
  std::vector<unsigned char> bytes;
  std::vector<BatchLaunch> lpre = schedule(pre, bytes), lpost = schedule(post, bytes);
  *table_needed = bytes.size();
  if (!table || table_bytes < bytes.size() || ((uintptr_t)table % 16) != 0) return CP_EWORKSPACE;
  for (auto* ls : {&lpre, &lpost})
    for (BatchLaunch& L : *ls)
      for (int k = 0; k < L.tab.n; ++k)
        L.tab.blk[k] = (const unsigned char*)table + (uintptr_t)L.tab.blk[k];
  if (hipMemcpy(table, bytes.data(), bytes.size(), hipMemcpyHostToDevice) != hipSuccess)
    return hip_status();
  cp_gn_batch* b = new cp_gn_batch;
  b->pre = std::move(lpre);
  b->post = std::move(lpost);
  b->plans = std::move(plans);
  b->cgargs = std::move(cgargs);
  b->cg_maxiter = prm->cg_maxiter;
  *out = b;
  return CP_OK;
}

int cp_gn_batch_step(cp_gn_batch* b, void* stream) {
  if (!b) return CP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  for (const BatchLaunch& L : b->pre) L.launch(L.tab, L.blocks, L.lds, st);
  const int count = (int)b->plans.size();
  for (int k = 0; k < count; k += kMaxCgBatch) {
    const int n = count - k < kMaxCgBatch ? count - k : kMaxCgBatch;
    launch_cg_batch(n, b->plans.data() + k, b->cgargs.data() + k, b->cg_maxiter, st);
  }
  for (const BatchLaunch& L : b->post) L.launch(L.tab, L.blocks, L.lds, st);
  return hip_status();
}

int cp_gn_batch_destroy(cp_gn_batch* b) {
  delete b;
  return CP_OK;
}

}  // extern "C"
