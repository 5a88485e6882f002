// FP64 kernels for the small dense parts of one Gauss-Newton step and one ALS sweep
// (Singh, Ma, Yang, Solomonik, arXiv:1910.12331): Grams S = A^T A and the Hadamard products
// Gamma(n,p) of eqs. (2) and (6); row-block times R x R products (gradient of Algorithm 1,
// the implicit J^T J product of eq. (7), the preconditioner apply of Algorithm 2); the CG
// vector recurrences with device-resident FP64 scalars; the explicit inverse
// (Gamma(n,n) + lambda I)^-1 of the Gauss-Newton preconditioner (Section 3.3), by Gauss-Jordan
// elimination without pivoting, and the register Cholesky factor of the triangular-solve
// preconditioner. The ALS solve is in chol.hip.
//
// Packed layout: the per-mode [s_n, R] matrices of one kind (factors, gradient, CG vectors)
// are stored back to back as one [sum_n s_n, R] FP64 array; Dims::off[n] is mode n's first
// row. Every reduction writes one partial per workgroup and is finished by a single
// workgroup in a fixed order, so results do not depend on scheduling.
#include "batch.h"

namespace cpgn {

// ------------------------------------------------------------------------------------------
// Deterministic block reduction of two doubles (fixed tree over 256 threads).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[256], sb[256];
  const int t = threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) {
      sa[t] += sa[t + w];
      sb[t] += sb[t + w];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  __syncthreads();
}

__device__ __forceinline__ bool state_done(const CgState* st) {
  return *(volatile const int32_t*)&st->done != 0;
}

// Gam[n][p] = Hadamard product of S(m) over m not in {n, p} (all-ones when empty), eq. (6).
struct KGamma {
  struct Args {
    Dims d;
    const double* S;
    double* Gam;
  };
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3 gdim) {
    const Dims& d = a.d;
    const double* __restrict__ S = a.S;
    double* __restrict__ Gam = a.Gam;
    const int R = d.R, N = d.N;
    const int64_t RR = (int64_t)R * R;
    const int64_t total = (int64_t)N * N * RR;
    for (int64_t idx = bid.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gdim.x * blockDim.x) {
      const int64_t e = idx % RR;
      const int np = (int)(idx / RR);
      const int n = np / N, p = np % N;
      double v = 1.0;
      for (int m = 0; m < N; ++m)
        if (m != n && m != p) v *= S[m * RR + e];
      Gam[idx] = v;
    }
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

__global__ __launch_bounds__(256) void k_gamma(KGamma::Args a) { KGamma::run(a, CPGN_BID, CPGN_GDIM); }

void KGamma::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_gamma, grid, dim3(kThreads), lds, s, a);
}

// Y(n)[r][z] = sum_{p != n} Gam[n][p][r][z] * B(p)[r][z]  (the R x R core of eq. (7)).
__global__ void k_ycore(Dims d, const double* __restrict__ Gam, const double* __restrict__ B,
                        double* __restrict__ Y, const CgState* st) {
  if (st && state_done(st)) return;
  const int R = d.R, N = d.N;
  const int64_t RR = (int64_t)R * R;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)N * RR;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(idx / RR);
    const int64_t e = idx - n * RR;
    double v = 0.0;
    for (int p = 0; p < N; ++p)
      if (p != n) v += Gam[((int64_t)n * N + p) * RR + e] * B[p * RR + e];
    Y[idx] = v;
  }
}

// ------------------------------------------------------------------------------------------
// Row-block times small matrices, all modes in one launch (grid.y = mode):
//   Out(n)[k][r] = cin * In(n)[k][r] + sum_z L1(n)[k][z] T1(n)[z][r] + sum_z L2(n)[k][z] T2(n)[r][z]
// T1/T2 are per-mode R x R matrices at T + n * t_stride (t_stride = 0 shares one matrix).
// Optional: Out2 = out2_scale * Out; a copy of Out in the caller's precision (per-mode
// pointers); per-workgroup partials of <Out(n), D(n)> and ||Out(n)||^2.
// ------------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_rowmm(Dims d, RowMM a, const CgState* st) {
  if (st && (state_done(st) || (a.skip_if_status && st->status != 0))) return;
  const int n = a.mode_only >= 0 ? a.mode_only : blockIdx.y;
  const int R = d.R;
  const int64_t rows = d.s[n];
  const int64_t base = d.off[n] * R;
  const double* T1 = a.t1 ? a.t1 + n * a.t1_stride : nullptr;
  const double* T2 = a.t2 ? a.t2 + n * a.t2_stride : nullptr;
  double dot = 0.0, nrm = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * R;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / R;
    const int r = (int)(e - k * R);
    const int64_t at = base + e;
    double v = a.in ? a.cin * a.in[at] : 0.0;
    if (T1) {
      const double* L = a.l1 + base + k * R;
      double s = 0.0;
      for (int z = 0; z < R; ++z) s += L[z] * T1[(int64_t)z * R + r];
      v += s;
    }
    if (T2) {
      const double* L = a.l2 + base + k * R;
      const double* Tr = T2 + (int64_t)r * R;
      double s = 0.0;
      for (int z = 0; z < R; ++z) s += L[z] * Tr[z];
      v += s;
    }
    if (a.out) a.out[at] = v;
    if (a.out2) a.out2[at] = a.out2_scale * v;
    if (a.cast_out.p[n]) {
      if (a.cast_dtype == CP_F64) ((double*)a.cast_out.p[n])[e] = v;
      else ((float*)a.cast_out.p[n])[e] = (float)v;
    }
    if (a.dotw) dot += v * a.dotw[at];
    nrm += v * v;
  }
  if (a.red_dot || a.red_nrm) {
    block_sum2(dot, nrm);
    if (threadIdx.x == 0) {
      if (a.red_dot) a.red_dot[n * kRedSlots + blockIdx.x] = dot;
      if (a.red_nrm) a.red_nrm[n * kRedSlots + blockIdx.x] = nrm;
    }
  }
}

// Per-mode conversion of caller buffers to packed FP64.
__global__ void k_to64(Dims d, PerMode<const void*> src, int dtype, double* __restrict__ dst) {
  const int n = blockIdx.y;
  const int64_t cnt = d.s[n] * d.R, base = d.off[n] * d.R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[base + e] = dtype == CP_F64 ? ((const double*)src.p[n])[e]
                                    : (double)((const float*)src.p[n])[e];
}

// ------------------------------------------------------------------------------------------
// Scalar finishing steps (one workgroup). Partials are summed in index order.
// ------------------------------------------------------------------------------------------
__device__ double sum_slots(const double* red, int nblocks) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) a += red[i];
  block_sum2(a, b);
  return a;
}

// Gradient norms: gsum = sum_n sqrt(sum_b nrm[n][b]); resets the CG state.
struct KFinGrad {
  struct Args {
    int N, nblocks;
    const double* red_nrm;
    CgState* st;
    double eps;
    double* gsum_out;
  };
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3, dim3) {
    double g = 0.0;
    for (int n = 0; n < a.N; ++n) g += sqrt(sum_slots(a.red_nrm + n * kRedSlots, a.nblocks));
    if (threadIdx.x == 0) {
      CgState* st = a.st;
      st->gsum = g;
      st->rsum = g;
      st->eps = a.eps;
      st->alpha = 0.0;
      st->beta = 0.0;
      st->rz = 0.0;
      st->upd2 = 0.0;
      st->iters = 0;
      st->status = isfinite(g) ? CP_OK : CP_ENONFINITE;
      st->done = st->status != CP_OK ? 1 : 0;
      if (a.gsum_out) *a.gsum_out = g;
    }
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

__global__ __launch_bounds__(256) void k_fin_grad(KFinGrad::Args a) {
  KFinGrad::run(a, CPGN_BID, CPGN_GDIM);
}

void KFinGrad::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_fin_grad, grid, dim3(kThreads), lds, s, a);
}

__global__ void k_state_reset(CgState* st) {
  if (threadIdx.x == 0) {
    st->gsum = st->rsum = st->alpha = st->beta = st->rz = st->upd2 = 0.0;
    st->eps = 0.0;
    st->iters = 0;
    st->status = CP_OK;
    st->done = 0;
  }
}

// A64 += V (when the step did not fail), write the caller's factors, ||V||, and the stats.
struct KGnApply {
  struct Args {
    Dims d;
    double* A64;
    const double* V;
    PerMode<void*> Aout;
    int dtype;
    double* red_nrm;
    const CgState* st;
  };
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3 gdim) {
    const Dims& d = a.d;
    double* __restrict__ A64 = a.A64;
    const double* __restrict__ V = a.V;
    const int n = bid.y;
    const bool ok = a.st->status == CP_OK;
    const int64_t base = d.off[n] * d.R, cnt = d.s[n] * d.R;
    double nrm = 0.0, dummy = 0.0;
    for (int64_t e = bid.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (int64_t)gdim.x * blockDim.x) {
      const double v = ok ? V[base + e] : 0.0;
      nrm += v * v;
      if (ok) {
        const double x = A64[base + e] + v;
        A64[base + e] = x;
        if (a.dtype == CP_F64) ((double*)a.Aout.p[n])[e] = x;
        else ((float*)a.Aout.p[n])[e] = (float)x;
      }
    }
    block_sum2(nrm, dummy);
    if (threadIdx.x == 0) a.red_nrm[n * kRedSlots + bid.x] = nrm;
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

__global__ __launch_bounds__(256) void k_gn_apply(KGnApply::Args a) {
  KGnApply::run(a, CPGN_BID, CPGN_GDIM);
}

void KGnApply::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_gn_apply, grid, dim3(kThreads), lds, s, a);
}

struct KGnStats {
  struct Args {
    int N, nblocks;
    const double* red_nrm;
    const CgState* st;
    cp_gn_stats* out;
  };
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3, dim3) {
    double u = 0.0;
    for (int n = 0; n < a.N; ++n) u += sum_slots(a.red_nrm + n * kRedSlots, a.nblocks);
    if (threadIdx.x == 0) {
      const CgState* st = a.st;
      cp_gn_stats* out = a.out;
      out->status = st->status;
      out->cg_iters = st->iters;
      out->grad_norm_sum = st->gsum;
      out->cg_res_norm_sum = st->rsum;
      out->alpha_last = st->alpha;
      out->beta_last = st->beta;
      out->update_norm = sqrt(u);
    }
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

__global__ __launch_bounds__(256) void k_gn_stats(KGnStats::Args a) {
  KGnStats::run(a, CPGN_BID, CPGN_GDIM);
}

void KGnStats::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_gn_stats, grid, dim3(kThreads), lds, s, a);
}

// ------------------------------------------------------------------------------------------
// Armijo step-size control (Section 5): after the direction V of Algorithm 1 is known, the step
// sizes alpha = 1, shrink, shrink^2, ... are tried in order and the first one with
// f(A + alpha V) <= f(A) + c alpha <G, V> is taken; f is eq. (3), G its gradient. Every trial is
// launched; once one has passed (ls_done) the remaining launches return at once, so the search
// needs no host synchronisation.
// ------------------------------------------------------------------------------------------

// Partials of <G, V> over the packed gradient and direction.
__global__ __launch_bounds__(256) void k_ls_dot(int64_t cnt, const double* __restrict__ G,
                                                const double* __restrict__ V, double* red) {
  double s = 0.0, dummy = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x)
    s = fma(G[e], V[e], s);
  block_sum2(s, dummy);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

__global__ void k_ls_gv(int nblocks, const double* red, CgState* st) {
  const double gv = sum_slots(red, nblocks);
  if (threadIdx.x == 0) st->ls_gv = gv;
}

__device__ void ls_start(CgState* st, double f0, double xn) {
  st->ls_f0 = f0;
  st->ls_xn = xn;
  st->ls_f = f0;
  st->ls_alpha = 1.0;
  st->ls_trials = 0;
  st->ls_accepted = 0;
  const double gv = st->ls_gv;
  st->ls_done = (st->status != CP_OK || !(gv < 0.0) || !isfinite(f0)) ? 1 : 0;
}

// Start of the search from the residual partials at the start point (slots [0] = squared
// differences, [kRedSlots] = squares of X). No trial runs when CG failed, when V is not a
// descent direction (<G, V> >= 0, e.g. V = 0) or when f is not finite.
__global__ void k_ls_init(int nblocks, const double* red, CgState* st) {
  const double d2 = sum_slots(red, nblocks);
  const double x2 = sum_slots(red + kRedSlots, nblocks);
  if (threadIdx.x == 0) ls_start(st, 0.5 * d2, sqrt(x2));
}

// Start of the search with f at the start point and ||X|| taken from the stats of the previous
// search on the same factors (f at the point it returned), instead of a residual pass.
__global__ void k_ls_init_given(const cp_armijo_stats* prev, CgState* st) {
  if (threadIdx.x == 0) ls_start(st, prev->f, prev->x_norm);
}

// Trial point A + alpha V: the caller's factors (f_dtype) and the padded compute-precision
// copies the residual reads (columns below R; the zero padding is left as it is).
template <typename T>
__global__ __launch_bounds__(256) void k_ls_trial(Dims d, const double* __restrict__ A64,
                                                  const double* __restrict__ V,
                                                  PerMode<void*> Aout, int dtype, T* apad,
                                                  const CgState* st) {
  if (st->ls_done) return;
  const int n = blockIdx.y;
  const double alpha = st->ls_alpha;
  const int64_t base = d.off[n] * d.R, cnt = d.s[n] * d.R;
  T* ap = apad + d.off[n] * d.Rp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double a = A64[base + e] + alpha * V[base + e];
    const int64_t row = e / d.R, col = e - row * d.R;
    ap[row * d.Rp + col] = (T)a;
    if (dtype == CP_F64) ((double*)Aout.p[n])[e] = a;
    else ((float*)Aout.p[n])[e] = (float)a;
  }
}

// Armijo test of the current trial from its residual partials; on failure the step size shrinks.
__global__ void k_ls_check(int nblocks, const double* red, CgState* st, double c, double shrink) {
  if (st->ls_done) return;
  const double d2 = sum_slots(red, nblocks);
  if (threadIdx.x == 0) {
    const double f = 0.5 * d2;
    const double alpha = st->ls_alpha;
    st->ls_trials += 1;
    if (f <= st->ls_f0 + c * alpha * st->ls_gv) {
      st->ls_f = f;
      st->ls_accepted = 1;
      st->ls_done = 1;
    } else {
      st->ls_alpha = alpha * shrink;
    }
  }
}

// End of the search: without an accepted step the caller's factors are restored from the FP64
// copy of the start point (exact, it was read from them); partials of ||alpha V||^2 for the stats.
__global__ __launch_bounds__(256) void k_ls_final(Dims d, const double* __restrict__ A64,
                                                  const double* __restrict__ V,
                                                  PerMode<void*> Aout, int dtype, double* red_nrm,
                                                  const CgState* st) {
  const int n = blockIdx.y;
  const bool acc = st->ls_accepted != 0;
  const bool restore = !acc && st->ls_trials > 0;
  const double alpha = acc ? st->ls_alpha : 0.0;
  const int64_t base = d.off[n] * d.R, cnt = d.s[n] * d.R;
  double nrm = 0.0, dummy = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = alpha * V[base + e];
    nrm += v * v;
    if (restore) {
      const double a = A64[base + e];
      if (dtype == CP_F64) ((double*)Aout.p[n])[e] = a;
      else ((float*)Aout.p[n])[e] = (float)a;
    }
  }
  block_sum2(nrm, dummy);
  if (threadIdx.x == 0) red_nrm[n * kRedSlots + blockIdx.x] = nrm;
}

__global__ void k_ls_stats(const CgState* st, cp_armijo_stats* out) {
  if (threadIdx.x != 0) return;
  const bool acc = st->ls_accepted != 0;
  out->alpha = acc ? st->ls_alpha : 0.0;
  out->f0 = st->ls_f0;
  out->f = st->ls_f;
  out->gv = st->ls_gv;
  out->x_norm = st->ls_xn;
  out->trials = st->ls_trials;
  out->accepted = acc ? 1 : 0;
}

__global__ void k_timestamp(int64_t* out) {
  if (threadIdx.x == 0) *out = (int64_t)wall_clock64();
}

__global__ void k_status_out(const CgState* st, int32_t* out) {
  if (threadIdx.x == 0) *out = st->status;
}

// ------------------------------------------------------------------------------------------
// P = (G + lambda I)^-1 for an R x R SPD matrix (R <= 208), one workgroup per matrix, FP64.
// In-place Gauss-Jordan inversion without pivoting: for an SPD matrix its pivots are the
// Cholesky pivots (the diagonals of the successive Schur complements), so "pivot > 0" is the
// same positive-definiteness test, and R steps give the inverse directly. Thread (ty, tx) of
// the TDY x TDX grid keeps the entries (ty + TDY ai, tx + TDX bk) of the identity-padded matrix
// in registers; each step publishes the pivot row r and column c through double-buffered LDS
// (one barrier), applies a_ik -= (c_i / p) r_k to every entry, and sets the pivot row to r / p,
// the pivot column to -c / p and the pivot to 1 / p (the Gauss-Jordan update).
// A non-positive or non-finite pivot records CP_ENOTSPD and marks the state done. With lam_dev
// the damping is read from device memory (a negative or non-finite value records CP_EINVAL).
template <int NBY, int NBX, int TDY, int TDX>
__global__ __launch_bounds__(TDY * TDX) void k_spd_inv(int R, const double* __restrict__ Gin,
                                                   int64_t g_stride, double lambda,
                                                   const double* __restrict__ lam_dev,
                                                   double* __restrict__ Pout, int64_t p_stride,
                                                   int first_mode, CgState* st, int diag_damping) {
  constexpr int RPY = TDY * NBY, RPX = TDX * NBX;
  __shared__ double colbuf[2][RPY], rowbuf[2][RPX];
  __shared__ int sbad;
  const int n = first_mode + blockIdx.x;
  const double* G = Gin + n * g_stride;
  double* P = Pout + n * p_stride;
  const int t = threadIdx.x, tx = t % TDX, ty = t / TDX;
  if (lam_dev) lambda = *lam_dev;
  if (t == 0) {
    sbad = st->status != CP_OK;   // one read: another workgroup may set it meanwhile
    if (!sbad && (!(lambda >= 0.0) || !isfinite(lambda))) {
      st->status = CP_EINVAL;
      st->done = 1;
      sbad = 1;
    }
  }
  __syncthreads();
  if (sbad) return;
  double a[NBY][NBX];
#pragma unroll
  for (int ai = 0; ai < NBY; ++ai)
#pragma unroll
    for (int bk = 0; bk < NBX; ++bk) {
      const int i = ty + TDY * ai, k = tx + TDX * bk;
      // lambda I, or lambda diag(G); G is read only inside the R x R block
      a[ai][bk] = (i < R && k < R)
                      ? G[i * R + k] + (i == k ? (diag_damping ? lambda * G[i * R + i] : lambda) : 0.0)
                      : (i == k ? 1.0 : 0.0);
    }
  // Pivot j = TDY jb + jt: its row lives in register row jb of thread row jt, its column in
  // register column jb TDY / TDX of thread column j % TDX (TDX is a multiple of TDY, so that
  // register column is the same for the whole block jb). Unrolling jb makes every register index
  // a constant: no selects over the register blocks.
#pragma unroll
  for (int jb = 0; jb < NBY; ++jb) {
    constexpr int kRatio = TDX / TDY;
    const int jbx = jb / kRatio;
    for (int jt = 0; jt < TDY; ++jt) {
      const int j = jb * TDY + jt;
      if (j >= R) break;   // uniform
      const int b = j & 1, jtx = j % TDX;
      if (ty == jt) {
#pragma unroll
        for (int bk = 0; bk < NBX; ++bk) rowbuf[b][tx + TDX * bk] = a[jb][bk];
      }
      if (tx == jtx) {
#pragma unroll
        for (int ai = 0; ai < NBY; ++ai) colbuf[b][ty + TDY * ai] = a[ai][jbx];
      }
      __syncthreads();
      const double piv = rowbuf[b][j];
      if (!(piv > 0.0) || !isfinite(piv)) {   // same value in every thread: uniform exit
        if (t == 0) {
          st->status = CP_ENOTSPD;
          st->done = 1;
        }
        return;
      }
      const double rp = 1.0 / piv;
      double u[NBY], v[NBX];
#pragma unroll
      for (int q = 0; q < NBY; ++q) u[q] = colbuf[b][ty + TDY * q] * rp;
#pragma unroll
      for (int q = 0; q < NBX; ++q) v[q] = rowbuf[b][tx + TDX * q];
      // One FMA per entry; it leaves 0 in the pivot row and column, which their owners then
      // set to r_k / p, -c_i / p and 1 / p.
#pragma unroll
      for (int ai = 0; ai < NBY; ++ai)
#pragma unroll
        for (int bk = 0; bk < NBX; ++bk) a[ai][bk] -= u[ai] * v[bk];
      if (ty == jt) {
#pragma unroll
        for (int bk = 0; bk < NBX; ++bk) a[jb][bk] = v[bk] * rp;
      }
      if (tx == jtx) {
#pragma unroll
        for (int ai = 0; ai < NBY; ++ai) a[ai][jbx] = -u[ai];
      }
      if (ty == jt && tx == jtx) a[jb][jbx] = rp;
    }
  }
#pragma unroll
  for (int ai = 0; ai < NBY; ++ai)
#pragma unroll
    for (int bk = 0; bk < NBX; ++bk) {
      const int i = ty + TDY * ai, k = tx + TDX * bk;
      if (i < R && k < R) P[i * R + k] = a[ai][bk];
    }
}

// ------------------------------------------------------------------------------------------
// Lower Cholesky factor L of G + lambda I (or G + lambda diag(G)), R <= 128, for the
// preconditioner applied by triangular solves (the alternative to the explicit inverse that
// Section 3.3 describes). Same thread layout as k_spd_inv: thread (ty, tx) keeps the entries
// (ty + TD ai, tx + TD bk) in registers. Step j publishes column j through double-buffered LDS
// (one barrier), sets L[j][j] = sqrt(p), L[i][j] = c_i / sqrt(p) below it, and updates the
// trailing block a_ik -= c_i c_k / p (right-looking Cholesky); the divisions are products with
// 1 / p and 1 / sqrt(p), formed once per step. Entries above the diagonal are
// written as 0. A non-positive or non-finite pivot records CP_ENOTSPD and marks the state done.
// ------------------------------------------------------------------------------------------
template <int NBK, int TD>
__global__ __launch_bounds__(TD * TD) void k_spd_chol(int R, const double* __restrict__ Gin,
                                                  int64_t g_stride, double lambda,
                                                  const double* __restrict__ lam_dev,
                                                  double* __restrict__ Lout, int64_t l_stride,
                                                  int first_mode, CgState* st, int diag_damping) {
  constexpr int RP = TD * NBK;
  __shared__ double colbuf[2][RP];
  __shared__ int sbad;
  const int n = first_mode + blockIdx.x;
  const double* G = Gin + n * g_stride;
  double* L = Lout + n * l_stride;
  const int t = threadIdx.x, tx = t % TD, ty = t / TD;
  if (lam_dev) lambda = *lam_dev;
  if (t == 0) {
    sbad = st->status != CP_OK;
    if (!sbad && (!(lambda >= 0.0) || !isfinite(lambda))) {
      st->status = CP_EINVAL;
      st->done = 1;
      sbad = 1;
    }
  }
  __syncthreads();
  if (sbad) return;
  double a[NBK][NBK];
#pragma unroll
  for (int ai = 0; ai < NBK; ++ai)
#pragma unroll
    for (int bk = 0; bk < NBK; ++bk) {
      const int i = ty + TD * ai, k = tx + TD * bk;
      a[ai][bk] = (i < R && k < R)
                      ? G[i * R + k] + (i == k ? (diag_damping ? lambda * G[i * R + i] : lambda) : 0.0)
                      : (i == k ? 1.0 : 0.0);
    }
  // Pivot j = TD jb + jt: its column is register column jb of thread column jt; unrolling jb
  // makes every register index a constant.
#pragma unroll
  for (int jb = 0; jb < NBK; ++jb) {
    for (int jt = 0; jt < TD; ++jt) {
      const int j = jb * TD + jt;
      if (j >= R) break;   // uniform
      const int b = j & 1;
      if (tx == jt) {
#pragma unroll
        for (int ai = 0; ai < NBK; ++ai) colbuf[b][ty + TD * ai] = a[ai][jb];
      }
      __syncthreads();
      const double piv = colbuf[b][j];
      if (!(piv > 0.0) || !isfinite(piv)) {   // same value in every thread: uniform exit
        if (t == 0) {
          st->status = CP_ENOTSPD;
          st->done = 1;
        }
        return;
      }
      const double d = sqrt(piv), rp = 1.0 / piv, rd = 1.0 / d;
      double u[NBK], v[NBK];
#pragma unroll
      for (int q = 0; q < NBK; ++q) {
        const int i = ty + TD * q, k = tx + TD * q;
        u[q] = i > j ? colbuf[b][i] * rp : 0.0;
        v[q] = k > j ? colbuf[b][k] : 0.0;
      }
#pragma unroll
      for (int ai = 0; ai < NBK; ++ai)
#pragma unroll
        for (int bk = 0; bk < NBK; ++bk) a[ai][bk] -= u[ai] * v[bk];
      if (tx == jt) {   // column j of L: rows below the pivot, and the pivot itself
#pragma unroll
        for (int ai = 0; ai < NBK; ++ai) {
          const int i = ty + TD * ai;
          if (i > j) a[ai][jb] = colbuf[b][i] * rd;
          else if (i == j) a[ai][jb] = d;
        }
      }
    }
  }
#pragma unroll
  for (int ai = 0; ai < NBK; ++ai)
#pragma unroll
    for (int bk = 0; bk < NBK; ++bk) {
      const int i = ty + TD * ai, k = tx + TD * bk;
      if (i < R && k < R) L[i * R + k] = k <= i ? a[ai][bk] : 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// Direct residual ||X - [[A]]||_F^2 and ||X||_F^2 (Section 5). The reconstruction tile
// Xt[o][k] = sum_r KRP(o, r) A(N)[k, r] (o runs over all modes but the last) is built on the
// matrix cores: the Khatri-Rao rows of a 16*MB-row tile stay in registers as A operands, the
// last factor is streamed in a packed B-operand layout, and each reconstructed 16x16 tile is
// compared with X in FP64.
// ------------------------------------------------------------------------------------------
struct ResArgs {
  const void* X;
  const void* apad[kMaxOrder];  // [s_m][Rp] compute precision
  const void* bpk;              // [K/16][RS][64]: A(N)[16kb + lane%16][(lane/16) RS + s]
  int64_t O, K, KB;
  int64_t s[kMaxOrder];
  int N, Rp;
  int64_t xplane;               // split bfloat16 tensor: elements between the hi and lo planes
  double* red;                  // [2][kRedSlots]
  const int32_t* skip;          // when set and nonzero the kernels do nothing (a finished search)
};

// Entry e of X in the compute precision T. XK: 0 = stored as T; 1 = bfloat16; 2 = two
// bfloat16 planes whose sum is the tensor (lo plane at X + plane).
template <typename T, int XK>
__device__ __forceinline__ T x_at(const void* X, int64_t e, int64_t plane) {
  if constexpr (XK == 0) {
    return ((const T*)X)[e];
  } else {
    const uint16_t* h = (const uint16_t*)X;
    float v = bf16_to_float(h[e]);
    if constexpr (XK == 2) v += bf16_to_float(h[plane + e]);
    return (T)v;
  }
}

// Four consecutive entries e..e+3 of X (e a multiple of 4, X 16-byte aligned for XK = 0 and
// 8-byte aligned otherwise).
template <typename T, int XK>
__device__ __forceinline__ void x_at4(const void* X, int64_t e, int64_t plane, T (&out)[4]) {
  if constexpr (XK == 0) {
    typedef T tv4 __attribute__((ext_vector_type(4)));
    const tv4 w = *(const tv4*)((const T*)X + e);
#pragma unroll
    for (int v = 0; v < 4; ++v) out[v] = w[v];
  } else {
    const uint16_t* h = (const uint16_t*)X;
    const uint2 w = *(const uint2*)(h + e);
    float f[4] = {bf16_to_float(w.x & 0xffffu), bf16_to_float(w.x >> 16),
                  bf16_to_float(w.y & 0xffffu), bf16_to_float(w.y >> 16)};
    if constexpr (XK == 2) {
      const uint2 l = *(const uint2*)(h + plane + e);
      f[0] += bf16_to_float(l.x & 0xffffu);
      f[1] += bf16_to_float(l.x >> 16);
      f[2] += bf16_to_float(l.y & 0xffffu);
      f[3] += bf16_to_float(l.y >> 16);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) out[v] = (T)f[v];
  }
}

// Direct residual (Section 5): ||X - [[A]]||^2 and ||X||^2 in one pass over X. X is viewed as
// [O][K] with K = s_N; the reconstruction is the product of the Khatri-Rao rows of the first N-1
// factors (O x R, built in registers) with A(N)^T, on the matrix cores.
// A workgroup owns a group of four 16 MB-row tiles (one per wavefront) and walks the 16-column
// blocks kb of its item range [b I / B, (b+1) I / B) over (group, kb) items in group-major
// order, so that the load is balanced to one item. The B fragment of column block kb (the
// packed last factor) is shared by the four wavefronts through LDS: each thread loads one
// 1/256 share for the next item while the current one is multiplied, and a barrier per item
// publishes it. X values of the next item are requested before the current item's products
// (ping-pong registers); the Khatri-Rao rows are rebuilt only when the group changes.
template <typename T> struct ResCfg;
template <> struct ResCfg<float> { static constexpr int MB = 3, OCC = 2; };
template <> struct ResCfg<double> { static constexpr int MB = 2, OCC = 1; };
// Sub-tiles per wavefront: one above 8 column blocks (R > 128), where the Khatri-Rao rows alone
// take 4 NBR registers per sub-tile and lane.
template <typename T> constexpr int res_mb(int nbr) { return nbr > 8 ? 1 : ResCfg<T>::MB; }

template <typename T, int MB>
struct ResX {
  T x[MB][4];
};

// FP32 multiplies with the operands swapped (the B fragment as A operand, the Khatri-Rao rows
// as B operand), which leaves lane 16 g + m with reconstructed entries (row m, columns 4 g + v):
// four consecutive columns of one X row, read with one 16-byte load when K is a multiple of 4
// (VX). FP64 keeps the direct form (its accumulator layout strides rows by 4).
template <typename T, int NBR, bool VX, int XK>
__global__ __launch_bounds__(256, ResCfg<T>::OCC) void k_residual(ResArgs a) {
  constexpr int MB = res_mb<T>(NBR);
  constexpr bool SWAP = sizeof(T) == 4;
  constexpr int RS = 4 * NBR;          // MFMA steps (R padded to 16 NBR, 4 per step)
  constexpr int BSH = RS * kWave / 256;   // B elements per thread per item (= NBR)
  typedef typename Mfma<T>::v4 v4;
  __shared__ T bs[2][RS * kWave];
  struct ResB {
    T v[BSH];
  };
  if (a.skip && *a.skip) return;   // uniform over the grid
  const int t = threadIdx.x, lane = t & 63, g = lane >> 4, m = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const void* X = a.X;
  const T* B = (const T*)a.bpk;
  const int64_t ntiles = (a.O + 16 * MB - 1) / (16 * MB);
  const int64_t ngroups = (ntiles + 3) / 4;
  const int64_t nitems = ngroups * a.KB;
  const int64_t i0 = blockIdx.x * nitems / gridDim.x, i1 = (blockIdx.x + 1) * nitems / gridDim.x;
  double d2 = 0.0, x2 = 0.0;
  if (i0 < i1) {
    const int64_t last = a.O * a.K - 1;
    const int64_t lane_row = (int64_t)Mfma<T>::out_row(lane, 0) * a.K + m;
    const int dv = Mfma<T>::out_row(0, 1);   // row step between accumulator elements
    T ar[MB][RS];
    ResB bn;
    ResX<T, MB> xa, xb;
    int64_t grp = i0 / a.KB, kb = i0 - grp * a.KB;   // item being multiplied
    int64_t gn = grp, kbn = kb;                      // item being prefetched
    int64_t built = -1;

    auto load_b = [&](ResB& bn, int64_t kk) {
#pragma unroll
      for (int j = 0; j < BSH; ++j) bn.v[j] = B[kk * RS * kWave + t + 256 * j];
    };
    auto store_b = [&](const ResB& bn, int buf) {
#pragma unroll
      for (int j = 0; j < BSH; ++j) bs[buf][t + 256 * j] = bn.v[j];
    };
    // X of item (gg, kk) for this wavefront's tile; every load is issued from a clamped offset
    // (out-of-range values are skipped where consumed).
    auto load_x = [&](ResX<T, MB>& xr, int64_t gg, int64_t kk) {
      const int64_t tile = gg * 4 + wv;
      if constexpr (SWAP) {
        // entries (row 16 mb + m, columns 4 g + v) of the tile
        const int64_t off0 = (tile * 16 * MB + m) * a.K + kk * 16 + 4 * g;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int64_t off = off0 + (int64_t)(16 * mb) * a.K;
          if constexpr (VX) {
            x_at4<T, XK>(X, off < last - 3 ? off : last - 3, a.xplane, xr.x[mb]);
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              xr.x[mb][v] = x_at<T, XK>(X, off + v < last ? off + v : last, a.xplane);
          }
        }
      } else {
        const int64_t off0 = tile * 16 * MB * a.K + kk * 16 + lane_row;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t off = off0 + (int64_t)(16 * mb + dv * v) * a.K;
            xr.x[mb][v] = x_at<T, XK>(X, off < last ? off : last, a.xplane);
          }
      }
    };
    auto advance = [&](int64_t& gg, int64_t& kk) {
      if (++kk == a.KB) {
        kk = 0;
        ++gg;
      }
    };
    // Khatri-Rao rows of this wavefront's tile: lane (g, m) holds, for row 16 mb + m, the
    // contiguous k-range [g RS, (g+1) RS) of the padded factor rows (16-byte loads). The first
    // factor's rows for all sub-tiles are requested together; each further factor multiplies in.
    auto build = [&](int64_t gg) {
      constexpr int VW = 16 / (int)sizeof(T);
      typedef T tvw __attribute__((ext_vector_type(VW)));
      const int64_t tile = gg * 4 + wv;
      // Mixed-radix digits of row tile*16MB + r: the tile's first row is split once (wave-
      // uniform), each lane then adds its offset r = 16 mb + m < 64 digit by digit with small
      // 32-bit carries. Rows past O read factor row 0; the epilogue skips them.
      int64_t brem = tile * 16 * MB;
      uint32_t carry[MB];
      bool in[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        carry[mb] = 16 * mb + m;
        in[mb] = brem + 16 * mb + m < a.O;
      }
      for (int q = a.N - 2; q >= 0; --q) {
        const int64_t sq = a.s[q];
        const uint32_t bd = (uint32_t)(brem % sq);
        brem /= sq;
        const uint32_t s32 = (uint32_t)sq;
        const bool first = q == a.N - 2;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const uint32_t tq = bd + carry[mb];
          const uint32_t idx = in[mb] ? tq % s32 : 0u;
          carry[mb] = tq / s32;
          const T* row = (const T*)a.apad[q] + (int64_t)idx * a.Rp + g * RS;
          if (first) {   // loaded straight into the operand registers
#pragma unroll
            for (int s = 0; s < RS; s += VW) {
              const tvw w = *(const tvw*)(row + s);
#pragma unroll
              for (int u = 0; u < VW; ++u) ar[mb][s + u] = w[u];
            }
          } else {
#pragma unroll
            for (int s = 0; s < RS; s += VW) {
              const tvw w = *(const tvw*)(row + s);
#pragma unroll
              for (int u = 0; u < VW; ++u) ar[mb][s + u] *= w[u];
            }
            // one sub-tile's factor row in flight at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    };
    auto consume = [&](const ResX<T, MB>& xr, int buf, int64_t gg, int64_t kk) {
      const int64_t tile = gg * 4 + wv;
      v4 acc[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[mb] = v4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const T b = bs[buf][s * kWave + lane];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[mb] = SWAP ? Mfma<T>::mac(b, ar[mb][s], acc[mb]) : Mfma<T>::mac(ar[mb][s], b, acc[mb]);
      }
      if ((tile + 1) * 16 * MB <= a.O && (kk + 1) * 16 <= a.K) {
        // Full tile: the 16 squares of this lane are summed in the tensor precision (exact
        // differences near a fit), then added to the FP64 totals.
        T dsq = T(0), xsq = T(0);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T x = xr.x[mb][v];
            const T df = x - acc[mb][v];
            dsq = fma(df, df, dsq);
            xsq = fma(x, x, xsq);
          }
        d2 += (double)dsq;
        x2 += (double)xsq;
      } else {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t o = tile * 16 * MB + 16 * mb + (SWAP ? m : Mfma<T>::out_row(lane, v));
            const int64_t col = kk * 16 + (SWAP ? 4 * g + v : m);
            const bool ok = o < a.O && col < a.K;
            const double x = ok ? (double)xr.x[mb][v] : 0.0;
            const double df = x - (ok ? (double)acc[mb][v] : 0.0);
            d2 = fma(df, df, d2);
            x2 = fma(x, x, x2);
          }
      }
    };
    // One item: request the next one (its B share and X values; past the range the current item
    // again, unused), multiply the current one with the B fragment in LDS slot buf, publish the
    // next B fragment in the other slot.
    auto step = [&](ResX<T, MB>& cur, ResX<T, MB>& nxt, int buf, int64_t i) {
      const bool more = i + 1 < i1;
      load_b(bn, more ? kbn : kb);
      load_x(nxt, more ? gn : grp, more ? kbn : kb);
      advance(gn, kbn);
      if (grp != built) {
        build(grp);
        built = grp;
      }
      consume(cur, buf, grp, kb);
      advance(grp, kb);
      store_b(bn, buf ^ 1);
      __syncthreads();
    };

    load_b(bn, kbn);
    load_x(xa, gn, kbn);
    advance(gn, kbn);
    store_b(bn, 0);
    __syncthreads();
    int64_t i = i0;
    while (true) {
      step(xa, xb, 0, i);
      if (++i >= i1) break;
      step(xb, xa, 1, i);
      if (++i >= i1) break;
    }
  }
  block_sum2(d2, x2);
  if (threadIdx.x == 0) {
    a.red[blockIdx.x] = d2;
    a.red[kRedSlots + blockIdx.x] = x2;
  }
}

// Pack the last factor for the residual's B fragments: bpk[kb][s][lane] = A[16kb + m][g RS + s]
// (lane group g owns the contiguous k-range [g RS, (g+1) RS) of the contraction).
template <typename T>
__global__ void k_pack_last(const T* __restrict__ apad_last, int64_t K, int Rp, int64_t KB,
                            T* __restrict__ bpk, const int32_t* skip) {
  if (skip && *skip) return;
  const int RS = Rp / 4;
  const int64_t total = KB * RS * kWave;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int lane = (int)(e % kWave);
    const int64_t rest = e / kWave;
    const int s = (int)(rest % RS);
    const int64_t kb = rest / RS;
    const int64_t k = 16 * kb + (lane & 15);
    bpk[e] = k < K ? apad_last[k * Rp + (lane >> 4) * RS + s] : T(0);
  }
}

// Fallback for R > 208: one thread per tensor entry, scalar FP64 reconstruction.
template <typename T, int XK>
__global__ void k_residual_scalar(ResArgs a, int R) {
  if (a.skip && *a.skip) return;
  double d2 = 0.0, x2 = 0.0;
  const int64_t total = a.O * a.K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t idx[kMaxOrder];
    int64_t rem = e;
    for (int q = a.N - 1; q >= 0; --q) {
      idx[q] = rem % a.s[q];
      rem /= a.s[q];
    }
    double xt = 0.0;
    for (int r = 0; r < R; ++r) {
      double p = 1.0;
      for (int q = 0; q < a.N; ++q) p *= (double)((const T*)a.apad[q])[idx[q] * a.Rp + r];
      xt += p;
    }
    const double x = (double)x_at<T, XK>(a.X, e, a.xplane);
    d2 += (x - xt) * (x - xt);
    x2 += x * x;
  }
  block_sum2(d2, x2);
  if (threadIdx.x == 0) {
    a.red[blockIdx.x] = d2;
    a.red[kRedSlots + blockIdx.x] = x2;
  }
}

// sum of squares of X (for the expansion form).
template <typename T, int XK>
__global__ void k_sumsq(const void* __restrict__ X, int64_t total, double* red) {
  double x2 = 0.0, dummy = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)x_at<T, XK>(X, e, total);
    x2 += x * x;
  }
  block_sum2(x2, dummy);
  if (threadIdx.x == 0) red[kRedSlots + blockIdx.x] = x2;
}

__global__ void k_fin_residual_direct(int nblocks, const double* red, double* out) {
  const double d2 = sum_slots(red, nblocks);
  const double x2 = sum_slots(red + kRedSlots, nblocks);
  if (threadIdx.x == 0) {
    out[0] = sqrt(d2);
    out[1] = sqrt(x2);
  }
}

// ||X||^2 - 2 <M(1), A(1)> + sum_{r,z} prod_m S(m)[r][z]; a negative value is clamped to 0.
__global__ void k_fin_residual_expansion(Dims d, int nblocks, const double* red,
                                         const double* M0, const double* A64, const double* S,
                                         double* out) {
  const double x2 = sum_slots(red + kRedSlots, nblocks);
  double cross = 0.0, had = 0.0;
  const int64_t n0 = d.s[0] * d.R;
  for (int64_t e = threadIdx.x; e < n0; e += blockDim.x) cross += M0[e] * A64[e];
  const int64_t RR = (int64_t)d.R * d.R;
  for (int64_t e = threadIdx.x; e < RR; e += blockDim.x) {
    double p = 1.0;
    for (int m = 0; m < d.N; ++m) p *= S[m * RR + e];
    had += p;
  }
  block_sum2(cross, had);
  if (threadIdx.x == 0) {
    const double r2 = x2 - 2.0 * cross + had;
    out[0] = sqrt(r2 > 0.0 ? r2 : 0.0);
    out[1] = sqrt(x2);
  }
}

// ------------------------------------------------------------------------------------------
// Host launchers used by the API layer
// ------------------------------------------------------------------------------------------
int grid1(int64_t n, int cap) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

void launch_gram_mfma(const Dims&, const double*, const double*, double*, int, const CgState*,
                      hipStream_t);
void launch_rowmm_mfma(const Dims&, const RowMM&, const CgState*, hipStream_t);
int rowmm_mfma_blocks(const Dims&);

void launch_gram2(const Dims& d, const double* X, const double* Y, double* C, int mode_only,
                  const CgState* st, hipStream_t s) {
  launch_gram_mfma(d, X, Y, C, mode_only, st, s);
}

void launch_gamma(const Dims& d, const double* S, double* Gam, hipStream_t s) {
  dispatch<KGamma>(dim3(grid1((int64_t)d.N * d.N * d.R * d.R, 256)), 0, s, {d, S, Gam});
}

void launch_ycore(const Dims& d, const double* Gam, const double* B, double* Y, const CgState* st,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_ycore, dim3(grid1((int64_t)d.N * d.R * d.R, 256)), dim3(256), 0, s, d, Gam,
                     B, Y, st);
}

int rowmm_blocks(const Dims& d) {
  if (d.R <= 128) return rowmm_mfma_blocks(d);
  int64_t mx = 0;
  for (int n = 0; n < d.N; ++n) mx = d.s[n] > mx ? d.s[n] : mx;
  return grid1(mx * d.R, 256);
}

void launch_rowmm(const Dims& d, const RowMM& a, const CgState* st, hipStream_t s) {
  if (d.R <= 128) {
    launch_rowmm_mfma(d, a, st, s);
    return;
  }
  dim3 grid(rowmm_blocks(d), a.mode_only >= 0 ? 1 : d.N);
  hipLaunchKernelGGL(k_rowmm, grid, dim3(256), 0, s, d, a, st);
}

void launch_to64(const Dims& d, const PerMode<const void*>& src, int dtype, double* dst,
                 hipStream_t s) {
  dim3 grid(rowmm_blocks(d), d.N);
  hipLaunchKernelGGL(k_to64, grid, dim3(256), 0, s, d, src, dtype, dst);
}

void launch_fin_grad(const Dims& d, int nblocks, const double* red_nrm, CgState* st, double eps,
                     double* gsum_out, hipStream_t s) {
  dispatch<KFinGrad>(dim3(1), 0, s, {d.N, nblocks, red_nrm, st, eps, gsum_out});
}

void launch_state_reset(CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st);
}

void launch_gn_apply(const Dims& d, double* A64, const double* V, const PerMode<void*>& Aout,
                     int dtype, double* red_nrm, const CgState* st, hipStream_t s) {
  dim3 grid(rowmm_blocks(d), d.N);
  dispatch<KGnApply>(grid, 0, s, {d, A64, V, Aout, dtype, red_nrm, st});
}

void launch_gn_stats(const Dims& d, int nblocks, const double* red_nrm, const CgState* st,
                     cp_gn_stats* out, hipStream_t s) {
  dispatch<KGnStats>(dim3(1), 0, s, {d.N, nblocks, red_nrm, st, out});
}

// Damping schedule of Section 3.2 on the device: state = {value, lower, upper, mu, decreasing}.
// One thread; the same IEEE operations as the host schedule, so both give the same sequence.
struct KDampingAdvance {
  struct Args {
    double* state;
  };
  static constexpr int kThreads = 64, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3, dim3) {
    if (threadIdx.x != 0) return;
    double* state = a.state;
    double v = state[0];
    const double lower = state[1], upper = state[2], mu = state[3];
    bool dec = state[4] != 0.0;
    if (dec) {
      v = v / mu;
      if (v <= lower) dec = false;
    } else {
      v = v * mu;
      if (v >= upper) dec = true;
    }
    state[0] = v;
    state[4] = dec ? 1.0 : 0.0;
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

__global__ __launch_bounds__(64) void k_damping_advance(KDampingAdvance::Args a) {
  KDampingAdvance::run(a, CPGN_BID, CPGN_GDIM);
}

void KDampingAdvance::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_damping_advance, grid, dim3(kThreads), lds, s, a);
}

void launch_damping_advance(double* state, hipStream_t s) {
  dispatch<KDampingAdvance>(dim3(1), 0, s, {state});
}

void launch_timestamp(int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_timestamp, dim3(1), dim3(64), 0, s, out);
}

void launch_status_out(const CgState* st, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, s, st, out);
}

// GN and ALS need R <= kMaxGnRank (the inverse is register-resident in one workgroup).
// Any rank: up to kMaxGnRank the Gauss-Newton inverse and the ALS Cholesky factor are register-
// or LDS-resident in one workgroup, above it they are blocked in global memory.
int spd_inv_supported(int R) { return R >= 1; }
int als_supported(int R) { return R >= 1; }

int launch_spd_inv_big(int R, const double* G, int64_t g_stride, double lambda, double* P,
                       int64_t p_stride, int first_mode, int count, CgState* st, hipStream_t s,
                       bool diag_damping, const double* lam_dev, double* tmp);

#ifndef CPGN_SPD_TD
#define CPGN_SPD_TD 32
#endif
int launch_spd_inv_blk(int R, const double* G, int64_t g_stride, double lambda, double* P,
                       int64_t p_stride, int first_mode, int count, CgState* st, hipStream_t s,
                       bool diag_damping, const double* lam_dev);

int launch_spd_inv(int R, const double* G, int64_t g_stride, double lambda, double* P,
                   int64_t p_stride, int first_mode, int count, CgState* st, hipStream_t s,
                   bool diag_damping, const double* lam_dev, double* tmp) {
  if (R > kMaxGnRank) {
    if (!tmp) return (int)hipErrorInvalidValue;
    return launch_spd_inv_big(R, G, g_stride, lambda, P, p_stride, first_mode, count, st, s,
                              diag_damping, lam_dev, tmp);
  }
  // R <= 128: Gauss-Jordan blocked by 16 x 16 tiles on the FP64 matrix cores (chol.hip)
  if (R <= 128)
    return launch_spd_inv_blk(R, G, g_stride, lambda, P, p_stride, first_mode, count, st, s,
                              diag_damping, lam_dev);
  // Thread grid TD x TD, each thread an NBK x NBK block. 32 x 32 (1024 threads) measured faster
  // than 16 x 16 at R = 50, 100 and 128 (the same arithmetic, so the same bits).
  constexpr int TD = CPGN_SPD_TD;
  if (R > 128) {
    // 16 x 32 threads (two wavefronts per SIMD), each a block of up to 13 x 7 entries, without
    // scratch or accumulation registers (a 16 x 16 grid of 13 x 13 blocks spilled to AGPRs and
    // took 544 us at R = 200).
    switch ((R + 15) / 16) {
#define CPGN_SPD16(k)                                                                         \
  case k:                                                                                     \
    hipLaunchKernelGGL((k_spd_inv<k, (k + 1) / 2, 16, 32>), dim3(count), dim3(512), 0, s, R, G, \
                       g_stride, lambda, lam_dev, P, p_stride, first_mode, st,               \
                       diag_damping ? 1 : 0);                                                 \
    break;
      CPGN_SPD16(9) CPGN_SPD16(10) CPGN_SPD16(11) CPGN_SPD16(12) CPGN_SPD16(13)
#undef CPGN_SPD16
      default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
  }
  const int nbk = (R + TD - 1) / TD;
  switch (nbk) {
#define CPGN_SPD(k)                                                                           \
  case k:                                                                                     \
    hipLaunchKernelGGL((k_spd_inv<k, k, TD, TD>), dim3(count), dim3(TD * TD), 0, s, R, G,   \
                       g_stride, lambda, lam_dev, P, p_stride, first_mode, st,               \
                       diag_damping ? 1 : 0);                                                 \
    break;
    CPGN_SPD(1) CPGN_SPD(2) CPGN_SPD(3) CPGN_SPD(4)
#if CPGN_SPD_TD == 16
    CPGN_SPD(5) CPGN_SPD(6) CPGN_SPD(7) CPGN_SPD(8)
#endif
#undef CPGN_SPD
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// Cholesky factors of all modes' G + lambda I in one launch (R <= 128; 32 x 32 threads).
int launch_spd_chol(int R, const double* G, int64_t g_stride, double lambda, double* L,
                    int64_t l_stride, int first_mode, int count, CgState* st, hipStream_t s,
                    bool diag_damping, const double* lam_dev) {
  switch ((R + 31) / 32) {
#define CPGN_CHOL(k)                                                                          \
  case k:                                                                                     \
    hipLaunchKernelGGL((k_spd_chol<k, 32>), dim3(count), dim3(1024), 0, s, R, G, g_stride,    \
                       lambda, lam_dev, L, l_stride, first_mode, st, diag_damping ? 1 : 0);   \
    break;
    CPGN_CHOL(1) CPGN_CHOL(2) CPGN_CHOL(3) CPGN_CHOL(4)
#undef CPGN_CHOL
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <typename T, int XK>
static int launch_residual_t(const Plan& p, const void* X, char* ws, double* out, hipStream_t s,
                             const int32_t* skip, int* nblocks) {
  const int MB = res_mb<T>(p.NBt);
  ResArgs a{};
  a.X = X;
  a.skip = skip;
  a.xplane = p.total;
  int64_t off = 0;
  for (int m = 0; m < p.N; ++m) {
    a.apad[m] = ws + p.off_apad + off * p.esz;
    a.s[m] = p.s[m];
    off += p.s[m] * p.Rp;
  }
  a.N = p.N;
  a.Rp = p.Rp;
  a.K = p.s[p.N - 1];
  a.O = p.total / a.K;
  a.KB = (a.K + 15) / 16;
  a.red = (double*)(ws + p.off_red);
  if (p.R <= kMaxGnRank) {
    // the packed last factor reuses the MTTKRP partial region
    a.bpk = ws + p.off_part;
    hipLaunchKernelGGL(k_pack_last<T>, dim3(grid1(a.KB * p.Rp / 4 * kWave, 1024)), dim3(256), 0,
                       s, (const T*)a.apad[p.N - 1], a.K, p.Rp, a.KB, (T*)(ws + p.off_part),
                       skip);
    const int64_t items = ((a.O + 16 * MB - 1) / (16 * MB) + 3) / 4 * a.KB;
    int64_t blocks = items;
    if (blocks > ResCfg<T>::OCC * kNumCU) blocks = ResCfg<T>::OCC * kNumCU;   // one resident round
    const bool vx = a.K % 4 == 0 && ((uintptr_t)X % (XK ? 8 : 16)) == 0;
    switch (p.NBt) {
#define CPGN_RES(k)                                                                         \
  case k:                                                                                   \
    if (vx) hipLaunchKernelGGL((k_residual<T, k, true, XK>), dim3(blocks), dim3(256), 0, s, a); \
    else hipLaunchKernelGGL((k_residual<T, k, false, XK>), dim3(blocks), dim3(256), 0, s, a);   \
    break;
      CPGN_RES(1) CPGN_RES(2) CPGN_RES(3) CPGN_RES(4) CPGN_RES(5) CPGN_RES(6) CPGN_RES(7)
      CPGN_RES(8) CPGN_RES(9) CPGN_RES(10) CPGN_RES(11) CPGN_RES(12) CPGN_RES(13)
#undef CPGN_RES
      default: break;
    }
    if (out)
      hipLaunchKernelGGL(k_fin_residual_direct, dim3(1), dim3(256), 0, s, (int)blocks, a.red, out);
    if (nblocks) *nblocks = (int)blocks;
  } else {
    const int blocks = grid1(p.total, kRedSlots);
    hipLaunchKernelGGL((k_residual_scalar<T, XK>), dim3(blocks), dim3(256), 0, s, a, p.R);
    if (out) hipLaunchKernelGGL(k_fin_residual_direct, dim3(1), dim3(256), 0, s, blocks, a.red, out);
    if (nblocks) *nblocks = blocks;
  }
  return (int)hipGetLastError();
}

// Direct residual: out = {||X - [[A]]||, ||X||}. With out null only the partial sums of squares
// are left in the reduction slots (nblocks of each); with skip set the launches do nothing once
// *skip is nonzero on the device.
int launch_residual_direct(const Plan& p, const void* X, void* ws, double* out, hipStream_t s,
                           const int32_t* skip, int* nblocks) {
  char* w = (char*)ws;
  if (p.xk == 1) return launch_residual_t<float, 1>(p, X, w, out, s, skip, nblocks);
  if (p.xk == 2) return launch_residual_t<float, 2>(p, X, w, out, s, skip, nblocks);
  if (p.dtype == CP_F32) return launch_residual_t<float, 0>(p, X, w, out, s, skip, nblocks);
  return launch_residual_t<double, 0>(p, X, w, out, s, skip, nblocks);
}

int launch_sumsq(const Plan& p, const void* X, double* red, hipStream_t s, int* nblocks) {
  const int blocks = grid1(p.total, kRedSlots);
  if (p.xk == 1)
    hipLaunchKernelGGL((k_sumsq<float, 1>), dim3(blocks), dim3(256), 0, s, X, p.total, red);
  else if (p.xk == 2)
    hipLaunchKernelGGL((k_sumsq<float, 2>), dim3(blocks), dim3(256), 0, s, X, p.total, red);
  else if (p.dtype == CP_F32)
    hipLaunchKernelGGL((k_sumsq<float, 0>), dim3(blocks), dim3(256), 0, s, X, p.total, red);
  else
    hipLaunchKernelGGL((k_sumsq<double, 0>), dim3(blocks), dim3(256), 0, s, X, p.total, red);
  *nblocks = blocks;
  return (int)hipGetLastError();
}

void launch_fin_residual_expansion(const Dims& d, int nblocks, const double* red, const double* M0,
                                   const double* A64, const double* S, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_residual_expansion, dim3(1), dim3(256), 0, s, d, nblocks, red, M0, A64,
                     S, out);
}

void launch_ls_gv(const Dims& d, const double* G, const double* V, double* red, CgState* st,
                  hipStream_t s) {
  const int64_t cnt = d.off[d.N] * d.R;
  const int blocks = grid1(cnt, kRedSlots);
  hipLaunchKernelGGL(k_ls_dot, dim3(blocks), dim3(256), 0, s, cnt, G, V, red);
  hipLaunchKernelGGL(k_ls_gv, dim3(1), dim3(256), 0, s, blocks, red, st);
}

void launch_ls_init(int nblocks, const double* red, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_ls_init, dim3(1), dim3(256), 0, s, nblocks, red, st);
}

void launch_ls_init_given(const cp_armijo_stats* prev, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_ls_init_given, dim3(1), dim3(64), 0, s, prev, st);
}

void launch_ls_trial(const Dims& d, const double* A64, const double* V, const PerMode<void*>& Aout,
                     int dtype, void* apad, const CgState* st, hipStream_t s) {
  dim3 grid(rowmm_blocks(d), d.N);
  if (dtype == CP_F64)
    hipLaunchKernelGGL(k_ls_trial<double>, grid, dim3(256), 0, s, d, A64, V, Aout, dtype,
                       (double*)apad, st);
  else
    hipLaunchKernelGGL(k_ls_trial<float>, grid, dim3(256), 0, s, d, A64, V, Aout, dtype,
                       (float*)apad, st);
}

void launch_ls_check(int nblocks, const double* red, CgState* st, double c, double shrink,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_ls_check, dim3(1), dim3(256), 0, s, nblocks, red, st, c, shrink);
}

void launch_ls_final(const Dims& d, const double* A64, const double* V, const PerMode<void*>& Aout,
                     int dtype, double* red_nrm, const CgState* st, cp_armijo_stats* out,
                     hipStream_t s) {
  dim3 grid(rowmm_blocks(d), d.N);
  hipLaunchKernelGGL(k_ls_final, grid, dim3(256), 0, s, d, A64, V, Aout, dtype, red_nrm, st);
  hipLaunchKernelGGL(k_ls_stats, dim3(1), dim3(64), 0, s, st, out);
}

}  // namespace cpgn

namespace cpgn {

// ---------------------------------------------------------------------------------------------
// CG of Algorithm 2 for R > kMaxGnRank, composed from the generic product kernels (Grams, the
// R x R core of eq. (7), row products) and the small kernels below; all scalars stay on the
// device, and every kernel returns at once when the state is done, as in the fixed-rank CG. Per
// iteration: check (rho = <R,Z>, the stop test, beta), W = Z + beta W, Q = (J^T J + lambda D) W,
// alpha = rho / <W,Q>, V += alpha W and R -= alpha Q, Z = R P_inv. Partial sums are per block and
// mode, added in a fixed order.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cgw_zero(Dims d, double* __restrict__ V,
                                                  const CgState* st) {
  if (state_done(st)) return;
  const int n = blockIdx.y;
  const int64_t base = d.off[n] * d.R, cnt = d.s[n] * d.R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x)
    V[base + e] = 0.0;
}

// Before iteration `it` (it iterations done): rho = sum <R,Z>, rsum = sum_n ||R(n)|| (gsum before
// the first iteration, R = -G), the stop test, beta = rho / rho_old.
__global__ __launch_bounds__(256) void k_cgw_check(int N, int nblocks, const double* red_rz,
                                                   const double* red_rr, CgState* st, int it,
                                                   int final_check) {
  if (state_done(st)) return;
  double rho = 0.0, rsum = 0.0;
  for (int n = 0; n < N; ++n) rho += sum_slots(red_rz + n * kRedSlots, nblocks);
  if (it == 0) {
    rsum = st->gsum;
  } else {
    for (int n = 0; n < N; ++n) rsum += sqrt(sum_slots(red_rr + n * kRedSlots, nblocks));
  }
  if (threadIdx.x != 0) return;
  const double beta = it == 0 ? 0.0 : rho / st->rho[(it + 1) & 1];
  bool stop = false;
  int status = CP_OK;
  if (!isfinite(rho) || !isfinite(rsum)) {
    status = CP_ENONFINITE;
    stop = true;
  } else if (!(rsum > st->eps * st->gsum)) {
    stop = true;
  }
  st->rho[it & 1] = rho;
  st->rz = rho;
  st->rsum = rsum;
  st->iters = it;
  if (it > 0) st->beta = beta;
  if (stop || final_check) {
    st->status = status;
    st->done = 1;
  }
}

// W = Z + beta W (beta = 0 before the first iteration).
__global__ __launch_bounds__(256) void k_cgw_dir(Dims d, const double* __restrict__ Z,
                                                 double* __restrict__ W, const CgState* st,
                                                 int it) {
  if (state_done(st)) return;
  const double beta = it == 0 ? 0.0 : st->beta;
  const int n = blockIdx.y;
  const int64_t base = d.off[n] * d.R, cnt = d.s[n] * d.R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x)
    W[base + e] = it == 0 ? Z[base + e] : __fma_rn(beta, W[base + e], Z[base + e]);
}

// Q = lambda_c W + Q0 (lambda_c = lambda, or lambda Gamma(n,n)[c][c] for the diagonal damping)
// and the partials of <W, Q>.
__global__ __launch_bounds__(256) void k_cgw_damp(Dims d, const double* __restrict__ W,
                                                  double* __restrict__ Q,
                                                  const double* __restrict__ gam, double lambda,
                                                  const double* __restrict__ lam_dev, int diag,
                                                  double* red_wq, const CgState* st) {
  if (state_done(st)) return;
  const int n = blockIdx.y, R = d.R, N = d.N;
  const double lam = lam_dev ? *lam_dev : lambda;
  const double* Gnn = gam + (int64_t)n * (N + 1) * R * R;
  const int64_t base = d.off[n] * R, cnt = d.s[n] * R;
  double dot = 0.0, dummy = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % R);
    const double lc = diag ? lam * Gnn[(int64_t)c * (R + 1)] : lam;
    const double w = W[base + e];
    const double q = __fma_rn(lc, w, Q[base + e]);
    Q[base + e] = q;
    dot += w * q;
  }
  block_sum2(dot, dummy);
  if (threadIdx.x == 0) red_wq[n * kRedSlots + blockIdx.x] = dot;
}

// alpha = rho / sum <W, Q>; a non-positive or non-finite denominator stops CG with a status.
__global__ __launch_bounds__(256) void k_cgw_alpha(int N, int nblocks, const double* red_wq,
                                                   CgState* st, int it) {
  if (state_done(st)) return;
  double wq = 0.0;
  for (int n = 0; n < N; ++n) wq += sum_slots(red_wq + n * kRedSlots, nblocks);
  if (threadIdx.x != 0) return;
  int status = CP_OK;
  if (!isfinite(wq)) status = CP_ENONFINITE;
  else if (!(wq > 0.0)) status = CP_EBREAKDOWN;
  if (status != CP_OK) {
    st->status = status;
    st->done = 1;
    return;
  }
  st->alpha = st->rho[it & 1] / wq;
}

// V += alpha W, R -= alpha Q, and the partials of ||R||^2.
__global__ __launch_bounds__(256) void k_cgw_update(Dims d, double* __restrict__ V,
                                                    double* __restrict__ Rv,
                                                    const double* __restrict__ W,
                                                    const double* __restrict__ Q, double* red_rr,
                                                    const CgState* st) {
  if (state_done(st)) return;
  const double alpha = st->alpha;
  const int n = blockIdx.y;
  const int64_t base = d.off[n] * d.R, cnt = d.s[n] * d.R;
  double nrm = 0.0, dummy = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    V[base + e] = __fma_rn(alpha, W[base + e], V[base + e]);
    const double r = __fma_rn(-alpha, Q[base + e], Rv[base + e]);
    Rv[base + e] = r;
    nrm += r * r;
  }
  block_sum2(nrm, dummy);
  if (threadIdx.x == 0) red_rr[n * kRedSlots + blockIdx.x] = nrm;
}

void launch_cgw_zero(const Dims& d, double* V, const CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cgw_zero, dim3(rowmm_blocks(d), d.N), dim3(256), 0, s, d, V, st);
}
void launch_cgw_check(const Dims& d, const double* red_rz, const double* red_rr, CgState* st,
                      int it, bool final_check, hipStream_t s) {
  hipLaunchKernelGGL(k_cgw_check, dim3(1), dim3(256), 0, s, d.N, rowmm_blocks(d), red_rz, red_rr,
                     st, it, final_check ? 1 : 0);
}
void launch_cgw_dir(const Dims& d, const double* Z, double* W, const CgState* st, int it,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_cgw_dir, dim3(rowmm_blocks(d), d.N), dim3(256), 0, s, d, Z, W, st, it);
}
void launch_cgw_damp(const Dims& d, const double* W, double* Q, const double* gam, double lambda,
                     const double* lam_dev, bool diag, double* red_wq, const CgState* st,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_cgw_damp, dim3(rowmm_blocks(d), d.N), dim3(256), 0, s, d, W, Q, gam,
                     lambda, lam_dev, diag ? 1 : 0, red_wq, st);
}
void launch_cgw_alpha(const Dims& d, const double* red_wq, CgState* st, int it, hipStream_t s) {
  hipLaunchKernelGGL(k_cgw_alpha, dim3(1), dim3(256), 0, s, d.N, rowmm_blocks(d), red_wq, st, it);
}
void launch_cgw_update(const Dims& d, double* V, double* Rv, const double* W, const double* Q,
                       double* red_rr, const CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cgw_update, dim3(rowmm_blocks(d), d.N), dim3(256), 0, s, d, V, Rv, W, Q,
                     red_rr, st);
}

}  // namespace cpgn
