// Algorithm 2 (CP-CG) of Singh, Ma, Yang, Solomonik (arXiv:1910.12331) as three fused kernels
// per iteration (all vectors FP64, packed [sum_n s_n, R]):
//   k_cg_proj    W = Z + beta W_old (into the other W buffer) and B(p) = A(p)^T W(p) in 16x16
//                tiles of the R x R result; a tile sums over all rows of its mode (no partials).
//   k_cg_matvec  Y(n) = sum_{p != n} Gamma(n,p) * B(p) staged in LDS, then
//                Q(n) = lambda W(n) + W(n) Gamma(n,n) + A(n) Y(n)^T (eq. (7)) for a block of rows,
//                <W,Q> per block; the last block to finish forms alpha = rho / sum <W,Q>.
//   k_cg_update  V += alpha W, R -= alpha Q, Z = R P_inv(n), <R,Z> and ||R(n)||^2 per block; the
//                last block forms beta = rho_new / rho and the stop test
//                sum_n ||R(n)||_F <= eps_cg sum_n ||G(n)||_F.
// The CG scalars stay in device memory; a kernel that finds the state done returns at once, so
// the host enqueues cg_maxiter iterations without synchronising. "Last block" reductions add the
// per-block partials in block order, so results do not depend on scheduling.
#include "cpgn_internal.h"

namespace cpgn {

constexpr int kRowBlk = 16;       // rows per block in the row kernels
constexpr int kTile = 16;         // B(p) tile edge
constexpr int kChunk = 64;        // rows staged per LDS chunk in k_cg_proj
constexpr int kMaxR = 128;

struct CgArgs {
  Dims d;
  const double* A64;
  const double* gam;      // Gamma[n][p]
  const double* pinv;     // P_inv[n]
  double* V;
  double* Rv;             // -G on entry
  double* Z;
  double* W[2];           // ping-pong W buffers
  double* Q;
  double* B;
  double* slot_dot;       // [nrowblk]
  double* slot_nrm;       // [nrowblk]
  unsigned* counter;      // last-block counters [2]
  CgState* st;
  double lambda;
  int nrowblk;
  int rb_off[kMaxOrder + 1];
};

__device__ __forceinline__ void bsum2(double& a, double& b) {
  __shared__ double sa[256], sb[256];
  const int t = threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
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

__device__ __forceinline__ void rowblk(const CgArgs& a, int task, int& n, int64_t& k0) {
  n = 0;
  while (task >= a.rb_off[n + 1]) ++n;
  k0 = (int64_t)(task - a.rb_off[n]) * kRowBlk;
}

// True in every thread of the block that finished last (its partial is already written).
__device__ __forceinline__ bool last_block(unsigned* counter) {
  __shared__ int is_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    is_last = prev == gridDim.x * gridDim.y - 1;
    if (is_last) *counter = 0u;   // ready for the next use
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last != 0;
}

__device__ __forceinline__ double sum_slots(const double* s, int n) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += s[i];
  bsum2(a, b);
  return a;
}

// acc[kk] += sum_z L[kk][z] T[z][r] for the kRowBlk rows staged in LDS (L: [kRowBlk][R]) and the
// R x R matrix T staged in LDS with row stride R + 1. Thread t owns column r = t % 128 and rows
// h*8 .. h*8+7, h = t / 128.
__device__ __forceinline__ void rowblock_times(const double* L, const double* T, int R,
                                               double acc[8]) {
  const int r = threadIdx.x & 127, h = threadIdx.x >> 7;
  if (r >= R) return;
  const double* Lh = L + h * 8 * R;
#pragma unroll 4
  for (int z = 0; z < R; ++z) {
    const double tv = T[z * (R + 1) + r];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc[kk] += Lh[kk * R + z] * tv;
  }
}


// Stage an R x R matrix into LDS with row stride R + 1 (optionally transposed), eight loads
// in flight per thread so that the copy costs about one memory latency.
__device__ __forceinline__ void stage_rr(double* T, const double* src, int R, bool transpose) {
  const int RR = R * R;
  for (int e0 = threadIdx.x; e0 < RR; e0 += 256 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      v[u] = e < RR ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      if (e < RR) {
        const int i = e / R, j = e - i * R;
        if (transpose) T[j * (R + 1) + i] = v[u];
        else T[i * (R + 1) + j] = v[u];
      }
    }
  }
}

// T[z][r] = Y(n)[r][z] = sum_{p != n} Gamma(n,p)[r][z] B(p)[r][z], batched like stage_rr.
__device__ __forceinline__ void stage_y(double* T, const double* gam, const double* B, int n,
                                        int N, int R) {
  const int RR = R * R;
  for (int e0 = threadIdx.x; e0 < RR; e0 += 256 * 4) {
    double y[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = 0; p < N; ++p) {
      if (p == n) continue;
      double g[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * 256;
        g[u] = e < RR ? gam[((int64_t)n * N + p) * RR + e] : 0.0;
        b[u] = e < RR ? B[(int64_t)p * RR + e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] += g[u] * b[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * 256;
      if (e < RR) {
        const int r = e / R, z = e - r * R;
        T[z * (R + 1) + r] = y[u];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Initialisation: V = 0, W_0 = 0, Z = R P_inv (R = -G), rho = sum <R,Z>, stop test.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cg_init(CgArgs a) {
  if (a.st->done) return;
  extern __shared__ double sm[];
  const int R = a.d.R, t = threadIdx.x;
  double* L = sm;                       // [kRowBlk][R]
  double* T = sm + kRowBlk * R;         // [R][R + 1]
  int n;
  int64_t k0;
  rowblk(a, blockIdx.x, n, k0);
  const int64_t rows = a.d.s[n] - k0 < kRowBlk ? a.d.s[n] - k0 : kRowBlk;
  const int64_t base = (a.d.off[n] + k0) * R;
  stage_rr(T, a.pinv + (int64_t)n * R * R, R, false);
  for (int e = t; e < kRowBlk * R; e += 256) {
    const bool in = e / R < rows;
    L[e] = in ? a.Rv[base + e] : 0.0;
    if (in) {
      a.V[base + e] = 0.0;
      a.W[0][base + e] = 0.0;
    }
  }
  __syncthreads();
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  rowblock_times(L, T, R, acc);
  const int r = t & 127, h = t >> 7;
  double dot = 0.0, dummy = 0.0;
  if (r < R) {
    for (int kk = 0; kk < 8; ++kk) {
      const int row = h * 8 + kk;
      if (row < rows) {
        a.Z[base + row * R + r] = acc[kk];
        dot += acc[kk] * L[row * R + r];
      }
    }
  }
  bsum2(dot, dummy);
  if (t == 0) a.slot_dot[blockIdx.x] = dot;
  if (last_block(&a.counter[0])) {
    const double rho = sum_slots(a.slot_dot, a.nrowblk);
    if (t == 0) {
      CgState* st = a.st;
      st->rz = rho;
      st->beta = 0.0;
      if (!isfinite(rho)) {
        st->status = CP_ENONFINITE;
        st->done = 1;
      } else if (!(st->rsum > st->eps * st->gsum)) {
        st->done = 1;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// W = Z + beta W_old (stored by the tiles with row-tile 0) and B(p) = A(p)^T W(p).
// grid: N * TB * TB blocks.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cg_proj(CgArgs a, int it) {
  if (a.st->done) return;
  __shared__ double as[kChunk][kTile + 1], wsm[kChunk][kTile + 1];
  const int R = a.d.R, t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int TB = (R + kTile - 1) / kTile;
  const int p = blockIdx.x / (TB * TB), rt = (blockIdx.x / TB) % TB, zt = blockIdx.x % TB;
  const int r0 = rt * kTile, z0 = zt * kTile;
  const int64_t s = a.d.s[p], base = a.d.off[p] * R;
  const double beta = a.st->beta;
  const double* Wold = a.W[it & 1];
  double* Wnew = a.W[(it + 1) & 1];
  double acc = 0.0;
  for (int64_t c0 = 0; c0 < s; c0 += kChunk) {
    double av[4], zv[4], wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + u * 256, kk = e >> 4, cc = e & 15;
      const int64_t k = c0 + kk;
      const int rc = r0 + cc, zc = z0 + cc;
      const bool ina = k < s && rc < R, inw = k < s && zc < R;
      av[u] = ina ? a.A64[base + k * R + rc] : 0.0;
      zv[u] = inw ? a.Z[base + k * R + zc] : 0.0;
      wv[u] = inw ? Wold[base + k * R + zc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + u * 256, kk = e >> 4, cc = e & 15;
      const int64_t k = c0 + kk;
      const int zc = z0 + cc;
      const double w = zv[u] + beta * wv[u];
      if (rt == 0 && k < s && zc < R) Wnew[base + k * R + zc] = w;
      as[kk][cc] = av[u];
      wsm[kk][cc] = w;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kChunk; ++kk) acc += as[kk][ty] * wsm[kk][tx];
    __syncthreads();
  }
  if (r0 + ty < R && z0 + tx < R) a.B[(int64_t)p * R * R + (int64_t)(r0 + ty) * R + z0 + tx] = acc;
}

// ---------------------------------------------------------------------------------------------
// Q = lambda W + W Gamma(n,n) + A Y(n)^T for a block of rows; alpha in the last block.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cg_matvec(CgArgs a, int it) {
  if (a.st->done) return;
  extern __shared__ double sm[];
  const int R = a.d.R, N = a.d.N, t = threadIdx.x;
  const int64_t RR = (int64_t)R * R;
  double* Lw = sm;                      // [kRowBlk][R]
  double* La = sm + kRowBlk * R;        // [kRowBlk][R]
  double* T = sm + 2 * kRowBlk * R;     // [R][R + 1]
  int n;
  int64_t k0;
  rowblk(a, blockIdx.x, n, k0);
  const int64_t rows = a.d.s[n] - k0 < kRowBlk ? a.d.s[n] - k0 : kRowBlk;
  const int64_t base = (a.d.off[n] + k0) * R;
  const double* W = a.W[(it + 1) & 1];
  for (int e = t; e < kRowBlk * R; e += 256) {
    const bool in = e / R < rows;
    Lw[e] = in ? W[base + e] : 0.0;
    La[e] = in ? a.A64[base + e] : 0.0;
  }
  stage_rr(T, a.gam + (int64_t)n * (N + 1) * RR, R, false);   // Gamma(n,n)
  __syncthreads();
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  rowblock_times(Lw, T, R, acc);
  __syncthreads();
  stage_y(T, a.gam, a.B, n, N, R);   // T[z][r] = Y(n)[r][z]
  __syncthreads();
  rowblock_times(La, T, R, acc);
  const int r = t & 127, h = t >> 7;
  double dot = 0.0, dummy = 0.0;
  if (r < R) {
    for (int kk = 0; kk < 8; ++kk) {
      const int row = h * 8 + kk;
      if (row < rows) {
        const double w = Lw[row * R + r];
        const double q = acc[kk] + a.lambda * w;
        a.Q[base + row * R + r] = q;
        dot += w * q;
      }
    }
  }
  bsum2(dot, dummy);
  if (t == 0) a.slot_dot[blockIdx.x] = dot;
  if (last_block(&a.counter[0])) {
    const double wq = sum_slots(a.slot_dot, a.nrowblk);
    if (t == 0) {
      CgState* st = a.st;
      if (!isfinite(wq)) {
        st->status = CP_ENONFINITE;
        st->done = 1;
      } else if (!(wq > 0.0)) {
        st->status = CP_EBREAKDOWN;
        st->done = 1;
      } else {
        st->alpha = st->rz / wq;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// V += alpha W, R -= alpha Q, Z = R P_inv; beta and the stop test in the last block.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cg_update(CgArgs a, int it) {
  if (a.st->done) return;
  extern __shared__ double sm[];
  const int R = a.d.R, N = a.d.N, t = threadIdx.x;
  double* L = sm;                       // [kRowBlk][R]
  double* T = sm + kRowBlk * R;         // [R][R + 1]
  int n;
  int64_t k0;
  rowblk(a, blockIdx.x, n, k0);
  const int64_t rows = a.d.s[n] - k0 < kRowBlk ? a.d.s[n] - k0 : kRowBlk;
  const int64_t base = (a.d.off[n] + k0) * R;
  const double alpha = a.st->alpha;
  const double* W = a.W[(it + 1) & 1];
  stage_rr(T, a.pinv + (int64_t)n * R * R, R, false);
  double nrm = 0.0;
  for (int e = t; e < kRowBlk * R; e += 256) {
    double rv = 0.0;
    if (e / R < rows) {
      a.V[base + e] += alpha * W[base + e];
      rv = a.Rv[base + e] - alpha * a.Q[base + e];
      a.Rv[base + e] = rv;
      nrm += rv * rv;
    }
    L[e] = rv;
  }
  __syncthreads();
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  rowblock_times(L, T, R, acc);
  const int r = t & 127, h = t >> 7;
  double dot = 0.0;
  if (r < R) {
    for (int kk = 0; kk < 8; ++kk) {
      const int row = h * 8 + kk;
      if (row < rows) {
        a.Z[base + row * R + r] = acc[kk];
        dot += acc[kk] * L[row * R + r];
      }
    }
  }
  bsum2(dot, nrm);
  if (t == 0) {
    a.slot_dot[blockIdx.x] = dot;
    a.slot_nrm[blockIdx.x] = nrm;
  }
  if (last_block(&a.counter[1])) {
    const double rz = sum_slots(a.slot_dot, a.nrowblk);
    double rs = 0.0;
    for (int m = 0; m < N; ++m) rs += sqrt(sum_slots(a.slot_nrm + a.rb_off[m], a.rb_off[m + 1] - a.rb_off[m]));
    if (t == 0) {
      CgState* st = a.st;
      st->beta = rz / st->rz;
      st->rz = rz;
      st->rsum = rs;
      st->iters += 1;
      if (!isfinite(rz) || !isfinite(rs)) {
        st->status = CP_ENONFINITE;
        st->done = 1;
      } else if (!(rs > st->eps * st->gsum)) {
        st->done = 1;
      }
    }
  }
}

__global__ void k_counter_reset(unsigned* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0u;
}

size_t cg_slot_bytes(const Plan& p) {
  int64_t nb = 0;
  for (int n = 0; n < p.N; ++n) nb += (p.s[n] + kRowBlk - 1) / kRowBlk;
  return (size_t)(2 * nb) * sizeof(double) + 256;
}

int cg_supported(const Plan& p) {
  const size_t lds = (size_t)(2 * kRowBlk * p.R + (size_t)p.R * (p.R + 1)) * sizeof(double);
  return p.R <= kMaxR && lds <= 150 * 1024;
}

// Enqueues the initialisation and cg_maxiter iterations.
int launch_cg(const Plan& p, const Dims& d, const double* A64, const double* gam,
              const double* pinv, double* V, double* Rv, double* Z, double* W0, double* W1,
              double* Q, double* B, void* slots, CgState* st, double lambda, int maxiter,
              hipStream_t s) {
  CgArgs a{};
  a.d = d;
  a.A64 = A64;
  a.gam = gam;
  a.pinv = pinv;
  a.V = V;
  a.Rv = Rv;
  a.Z = Z;
  a.W[0] = W0;
  a.W[1] = W1;
  a.Q = Q;
  a.B = B;
  a.st = st;
  a.lambda = lambda;
  a.rb_off[0] = 0;
  for (int n = 0; n < p.N; ++n)
    a.rb_off[n + 1] = a.rb_off[n] + (int)((p.s[n] + kRowBlk - 1) / kRowBlk);
  a.nrowblk = a.rb_off[p.N];
  a.slot_dot = (double*)slots;
  a.slot_nrm = a.slot_dot + a.nrowblk;
  a.counter = (unsigned*)((char*)slots + cg_slot_bytes(p) - 256);
  const int R = p.R, TB = (R + kTile - 1) / kTile;
  const size_t lds1 = (size_t)(kRowBlk * R + R * (R + 1)) * sizeof(double);
  const size_t lds2 = (size_t)(2 * kRowBlk * R + R * (R + 1)) * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_cg_init, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void*)k_cg_matvec, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void*)k_cg_update, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL(k_counter_reset, dim3(1), dim3(64), 0, s, a.counter);
  hipLaunchKernelGGL(k_cg_init, dim3(a.nrowblk), dim3(256), lds1, s, a);
  for (int it = 0; it < maxiter; ++it) {
    hipLaunchKernelGGL(k_cg_proj, dim3(p.N * TB * TB), dim3(256), 0, s, a, it);
    hipLaunchKernelGGL(k_cg_matvec, dim3(a.nrowblk), dim3(256), lds2, s, a, it);
    hipLaunchKernelGGL(k_cg_update, dim3(a.nrowblk), dim3(256), lds1, s, a, it);
  }
  return (int)hipGetLastError();
}

}  // namespace cpgn
