// FP64 Cholesky factorization of an ALS normal-equation matrix and the triangular solves that
// apply it to the rows of M (Section 2.2: A(n) = M(n) (Gamma(n) + lambda I)^-1).
//
//   k_chol_tiles  L L^T = G + lambda I for R <= 208, one workgroup of eight wavefronts per matrix.
//                 Right-looking and blocked by 16 x 16 tiles: the lower-triangle tiles live in
//                 registers in the FP64 MFMA accumulator layout, spread over the wavefronts. Step
//                 k factors the diagonal tile (one wavefront, in registers, values exchanged by
//                 lane permutes), solves the tiles below it against that factor (by substitution
//                 across the 16 lanes of a row group) and subtracts the outer products of that
//                 panel from the trailing tiles on the matrix cores: two workgroup barriers per
//                 16 columns instead of one per pivot.
//   k_chol_rows   A = M (L L^T)^-1 for 16 rows per wavefront: Y L^T = M by forward substitution,
//                 then A L = Y by back substitution, 16 columns at a time, with the 16 x 16
//                 diagonal blocks applied through their inverses (as blocked triangular solvers
//                 do), so every step is a product on the FP64 matrix cores. Wavefronts share
//                 nothing but L, which a workgroup stages in LDS when it fits (R <= 128).
//                 k_chol_tiles forms those 16 x 16 inverses by the same substitution on the
//                 identity, beside the panel of each step.
#include "batch.h"
#include "mfma64.h"

namespace cpgn {

constexpr int kCholWaves = 8;
constexpr int kCholMaxNT = (kMaxGnRank + 15) / 16;
constexpr int kCholMaxSlots = (kCholMaxNT * (kCholMaxNT + 1) / 2 + kCholWaves - 1) / kCholWaves;

// Orders the LDS accesses of one wavefront (its lanes exchange values through LDS).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lower-triangle tile t = I (I + 1) / 2 + J -> (I, J).
__host__ __device__ constexpr int tile_row(int t) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  return i;
}
__host__ __device__ constexpr int tile_col(int t) { return t - tile_row(t) * (tile_row(t) + 1) / 2; }

// Entry (r, c) of G + lambda I, extended by the identity past R.
__device__ __forceinline__ double shifted(const double* G, int R, double lambda, int r, int c) {
  if (r < R && c < R) return G[r * R + c] + (r == c ? lambda : 0.0);
  return r == c ? 1.0 : 0.0;
}

// The kernels below run once per launch over short dependency chains, so their code is kept
// compact (runtime loops): fully unrolled variants spent most of their time fetching
// instructions.

// Forward substitution across the 16 lanes of each row group: rows of T (rows g + 4 v, column
// m) become X with X L^T = T for a 16 x 16 lower-triangular L, given lmc(c) = L[m][c] and
// rdl = 1 / L[m][m].
template <typename LF>
__device__ __forceinline__ void row_forward16(dv4& T, LF lmc, double rdl, int g, int m) {
  // branch-free: the four exchanges of a step are issued together, the updates are selects
#pragma unroll 1
  for (int c = 0; c < 16; ++c) {
    const double l = lmc(c);
    double xb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) xb[v] = __shfl(T[v] * rdl, 16 * g + c);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double upd = T[v] - xb[v] * l;
      T[v] = m > c ? upd : (m == c ? xb[v] : T[v]);
    }
  }
}

// Right-looking Cholesky of one 16 x 16 tile held by a wavefront in the accumulator layout
// (lane (g, m): rows g + 4 v, column m). Pivot c: p = T[c][c] from its lane, column c of the
// lane's rows and the entry T[m][c] for the lane's column from their owners; the trailing
// entries lose c_i c_j / p, column c becomes c_i / sqrt(p) and the pivot sqrt(p). Returns false
// (same in every lane) for a non-positive or non-finite pivot. Entries above the diagonal are
// set to 0.
__device__ __forceinline__ bool tile_cholesky(dv4& D, int g, int m) {
  const int mv = m >> 2;
#pragma unroll 1
  for (int c = 0; c < 16; ++c) {
    const int vc = c >> 2;
    const double dvc = vc == 0 ? D[0] : vc == 1 ? D[1] : vc == 2 ? D[2] : D[3];
    double ci[4], cjv[4];
    const double p = __shfl(dvc, 16 * (c & 3) + c);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      ci[v] = __shfl(D[v], 16 * g + c);
      cjv[v] = __shfl(D[v], 16 * (m & 3) + c);
    }
    if (!(p > 0.0) || !isfinite(p)) return false;   // the same value in every lane
    const double d = sqrt(p), rp = 1.0 / p, rd = d * rp;
    const double cj = mv == 0 ? cjv[0] : mv == 1 ? cjv[1] : mv == 2 ? cjv[2] : cjv[3];
    const double cjr = cj * rp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = g + 4 * v;
      const double upd = D[v] - ci[v] * cjr;
      const double col = i > c ? ci[v] * rd : (i == c ? d : D[v]);
      D[v] = m > c ? (i > c ? upd : D[v]) : (m == c ? col : D[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) D[v] = m > g + 4 * v ? 0.0 : D[v];
  return true;
}

// grid: one workgroup per matrix (modes first_mode, first_mode + 1, ...), 512 threads. Tile t of
// the lower triangle belongs to wavefront t % 8, register slot t / 8; lane (g, m) = (lane / 16,
// lane % 16) holds rows g + 4 v, column m of its tiles (the MFMA accumulator layout). Step k:
// (a) the owner of tile (k, k) factors it in registers and publishes it in LDS; (b) the owners
// of the tiles below it solve them against it (X L_kk^T = T) and publish them; (c) every tile
// right of column k and on or below the diagonal loses the product of its two panel tiles. L is
// written once all steps are done. A non-positive or non-finite pivot records CP_ENOTSPD, marks
// the state done and writes nothing. Entries of L above the diagonal are not written.
template <int SLOTS>
__global__ __launch_bounds__(kCholWaves * 64) void k_chol_tiles(int R, const double* __restrict__ Gin,
                                                              int64_t g_stride, double lambda,
                                                              double* __restrict__ Lout,
                                                              int64_t l_stride,
                                                              double* __restrict__ Dout,
                                                              int64_t d_stride, int first_mode,
                                                              CgState* st) {
  __shared__ double dg[16][17];                        // L_kk of the current step
  __shared__ double pan[2][kCholMaxNT][16][17];        // the solved panel of a step
  __shared__ int sbad;
  const int n = first_mode + blockIdx.x;
  const double* G = Gin + n * g_stride;
  double* L = Lout + n * l_stride;
  double* Dinv = Dout + n * d_stride;
  const int NT = (R + 15) >> 4, NTT = NT * (NT + 1) / 2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  if (threadIdx.x == 0) sbad = st->status != CP_OK;
  __syncthreads();
  if (sbad) return;

  dv4 T[SLOTS];
  int TI[SLOTS], TJ[SLOTS];
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) {
    const int t = w + kCholWaves * i;
    TI[i] = t < NTT ? tile_row(t) : -1;
    TJ[i] = t < NTT ? t - TI[i] * (TI[i] + 1) / 2 : -1;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      T[i][v] = t < NTT ? shifted(G, R, lambda, 16 * TI[i] + g + 4 * v, 16 * TJ[i] + m) : 0.0;
  }

  for (int k = 0; k < NT; ++k) {
    const int b = k & 1;
    const int tkk = k * (k + 1) / 2 + k;
    if (w == tkk % kCholWaves) {                                             // (a)
      const int slot = tkk / kCholWaves;
      dv4 D = T[0];
#pragma unroll
      for (int i = 1; i < SLOTS; ++i)
        if (i == slot) D = T[i];
      const bool ok = tile_cholesky(D, g, m);
#pragma unroll
      for (int i = 0; i < SLOTS; ++i)
        if (i == slot) T[i] = D;
#pragma unroll
      for (int v = 0; v < 4; ++v) dg[g + 4 * v][m] = D[v];
      if (!ok && lane == 0) {
        st->status = CP_ENOTSPD;
        st->done = 1;
        sbad = 1;
      }
    }
    __syncthreads();
    if (sbad) return;
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) {                                        // (b)
      if (TJ[i] == k && TI[i] > k) {
        row_forward16(T[i], [&](int c) { return dg[m][c]; }, 1.0 / dg[m][m], g, m);
#pragma unroll
        for (int v = 0; v < 4; ++v) pan[b][TI[i]][g + 4 * v][m] = T[i][v];
      }
    }
    if (w == (tkk + 1) % kCholWaves) {   // L_kk^-T: the same substitution on the identity
      dv4 E;
#pragma unroll
      for (int v = 0; v < 4; ++v) E[v] = g + 4 * v == m ? 1.0 : 0.0;
      row_forward16(E, [&](int c) { return dg[m][c]; }, 1.0 / dg[m][m], g, m);
#pragma unroll
      for (int v = 0; v < 4; ++v) Dinv[k * 256 + (g + 4 * v) * 16 + m] = E[v];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) {                                        // (c)
      if (TJ[i] > k) {
        const int I = TI[i], J = TJ[i];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int q = 4 * q4 + g;
          T[i] = mfma64(-pan[b][I][m][q], pan[b][J][m][q], T[i]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) {
    if (TI[i] < 0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * TI[i] + g + 4 * v, c = 16 * TJ[i] + m;
      if (r < R && c < R && c <= r) L[r * R + c] = T[i][v];
    }
  }
}

// Entry (i, j) of L, extended by the identity past R (only i >= j is read).
template <bool LDSL>
__device__ __forceinline__ double lget(const double* __restrict__ L, const double* Lt, int R, int i,
                                       int j) {
  if (LDSL) {
    const int I = i >> 4, J = j >> 4;
    return Lt[(I * (I + 1) / 2 + J) * 272 + (i & 15) * 17 + (j & 15)];
  }
  if (i < R && j < R) return L[i * R + j];
  return i == j ? 1.0 : 0.0;
}

// grid: ceil(s / 64) workgroups of four wavefronts; wavefront w of workgroup b owns rows
// 64 b + 16 w .. + 15 of the mode. Each 16-column block of the forward solve Y L^T = M is the
// product (M_k - sum_{j<k} Y_j L_kj^T) L_kk^-T, and of the back solve A L = Y the product
// (Y_k - sum_{j>k} A_j L_jk) L_kk^-1: blocked substitution in which the 16 x 16 diagonal blocks
// act through their inverses (Dinv: L_kk^-T, one 16 x 16 block per k, row-major), so that every
// step is a chain of FP64 MFMAs. Dynamic LDS: 4 x 16 x (16 NT + 1) doubles for the rows, plus,
// when LDSL, the NT (NT + 1) / 2 lower tiles of L and the NT blocks of Dinv at 16 x 17 doubles
// each. Skipped when the state records a failure (the factors keep their values). Writes A in
// the caller's dtype.
template <int NT, bool LDSL>
__global__ __launch_bounds__(256) void k_chol_rows(int R, int64_t s, const double* __restrict__ M,
                                                   const double* __restrict__ L,
                                                   const double* __restrict__ Dinv,
                                                   void* __restrict__ Aout, int dtype,
                                                   const CgState* st) {
  constexpr int RP = 16 * NT, YS = RP + 1, NTT = NT * (NT + 1) / 2;
  extern __shared__ double smem[];
  if (st->status != CP_OK) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, m = lane & 15;
  double* Y = smem + w * 16 * YS;
  double* Lt = smem + 4 * 16 * YS;
  double* Dt = Lt + NTT * 272;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + 16 * w;
  if (LDSL) {   // thread t stages entry (t / 16, t % 16) of every tile: all loads in flight
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    double v[NTT + NT];
#pragma unroll
    for (int t = 0; t < NTT; ++t) {
      const int i = 16 * tile_row(t) + r, j = 16 * tile_col(t) + c;
      v[t] = (i < R && j < R) ? L[i * R + j] : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) v[NTT + k] = Dinv[k * 256 + threadIdx.x];
#pragma unroll
    for (int t = 0; t < NTT + NT; ++t) Lt[t * 272 + r * 17 + c] = v[t];
  }
  {   // the wavefront's 16 rows of M, zero past R and past the mode
    double v[RP / 4];
#pragma unroll
    for (int q = 0; q < RP / 4; ++q) {
      const int e = lane + 64 * q, r = e / RP, c = e - r * RP;
      const int64_t row = row0 + r;
      v[q] = (row < s && c < R) ? M[row * R + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < RP / 4; ++q) {
      const int e = lane + 64 * q, r = e / RP, c = e - r * RP;
      Y[r * YS + c] = v[q];
    }
  }
  if (LDSL) __syncthreads();
  else wave_lds_sync();
  // Dinv block k entry (a, b) = (L_kk^-T)[a][b]
  auto dget = [&](int k, int a, int b) {
    return LDSL ? Dt[k * 272 + a * 17 + b] : Dinv[k * 256 + a * 16 + b];
  };
  // forward: Y L^T = M, block by block
#pragma unroll 1
  for (int k = 0; k < NT; ++k) {
    dv4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = Y[(g + 4 * v) * YS + 16 * k + m];
#pragma unroll 1
    for (int jb = 0; jb < k; ++jb) {
      double a[4], bv[4];
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int q = 16 * jb + 4 * q4 + g;
        a[q4] = Y[m * YS + q];
        bv[q4] = lget<LDSL>(L, Lt, R, 16 * k + m, q);
      }
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) acc = mfma64(-a[q4], bv[q4], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Y[(g + 4 * v) * YS + 16 * k + m] = acc[v];
    wave_lds_sync();
    dv4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4)
      y = mfma64(Y[m * YS + 16 * k + 4 * q4 + g], dget(k, 4 * q4 + g, m), y);
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) Y[(g + 4 * v) * YS + 16 * k + m] = y[v];
    wave_lds_sync();
  }
  // back: A L = Y, last block first (A overwrites Y block by block)
#pragma unroll 1
  for (int k = NT - 1; k >= 0; --k) {
    dv4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = Y[(g + 4 * v) * YS + 16 * k + m];
#pragma unroll 1
    for (int jb = k + 1; jb < NT; ++jb) {
      double a[4], bv[4];
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int q = 16 * jb + 4 * q4 + g;
        a[q4] = Y[m * YS + q];
        bv[q4] = lget<LDSL>(L, Lt, R, q, 16 * k + m);
      }
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) acc = mfma64(-a[q4], bv[q4], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Y[(g + 4 * v) * YS + 16 * k + m] = acc[v];
    wave_lds_sync();
    dv4 a = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4)
      a = mfma64(Y[m * YS + 16 * k + 4 * q4 + g], dget(k, m, 4 * q4 + g), a);
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) Y[(g + 4 * v) * YS + 16 * k + m] = a[v];
    wave_lds_sync();
  }
  for (int e = lane; e < 16 * R; e += 64) {
    const int r = e / R, c = e - r * R;
    const int64_t row = row0 + r;
    if (row < s) {
      if (dtype == CP_F64) ((double*)Aout)[row * R + c] = Y[r * YS + c];
      else ((float*)Aout)[row * R + c] = (float)Y[r * YS + c];
    }
  }
}

// ------------------------------------------------------------------------------------------
// P = (G + lambda I)^-1 (or G + lambda diag(G)) for R <= 128, one workgroup of 16 wavefronts
// per matrix: Gauss-Jordan elimination without pivoting, blocked by 16 x 16 tiles. For an SPD
// matrix the pivots are those of its Cholesky factorization, so "pivot > 0" tests positive
// definiteness. The identity-padded matrix (RP = 16 NT rows) lives in LDS. Block step k:
//   (a) one wavefront inverts the diagonal tile D = M_kk in place by 16 scalar Gauss-Jordan
//       steps in registers (row and column of each pivot exchanged by lane permutes); for
//       k > 0 it does so during step k - 1, right after updating that tile in (c);
//   (b) M_kj <- D^-1 M_kj for j != k (the pivot block row);
//   (c) M_ij <- M_ij - M_ik M_kj for i, j != k, and M_ik <- -M_ik D^-1 (the pivot block
//       column, written after a barrier, once every product has read the old M_ik);
// (b) and (c) are 16 x 16 x 16 products on the FP64 matrix cores. Four workgroup barriers per
// 16 pivots instead of one per pivot. A non-positive or non-finite pivot records CP_ENOTSPD.
constexpr int kInvWaves = 16;

// Value of lane c of each quad of lanes (DPP quad permutation), for a double.
template <int C>
__device__ __forceinline__ double quad_bcast(double x) {
  const int2 v = __builtin_bit_cast(int2, x);
  const int lo = __builtin_amdgcn_mov_dpp(v.x, C * 0x55, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(v.y, C * 0x55, 0xF, 0xF, false);
  return __builtin_bit_cast(double, int2{lo, hi});
}

// Value of lane l (uniform) of a double.
__device__ __forceinline__ double read_lane(double x, int l) {
  const int2 v = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, int2{__builtin_amdgcn_readlane(v.x, l),
                                         __builtin_amdgcn_readlane(v.y, l)});
}

template <int NT>
__device__ __forceinline__ void spd_inv_blk_body(int R, const double* __restrict__ Gin,
                                                 int64_t g_stride, double lambda,
                                                 const double* __restrict__ lam_dev,
                                                 double* __restrict__ Pout, int64_t p_stride,
                                                 int first_mode, CgState* st, int diag_damping,
                                                 dim3 bid) {
  constexpr int RP = 16 * NT, LD = RP + 1;   // odd row stride: column reads hit distinct banks
  extern __shared__ double M[];               // [RP][LD]
  __shared__ int sbad;
  const int n = first_mode + bid.x;
  const double* G = Gin + n * g_stride;
  double* P = Pout + n * p_stride;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, g = lane >> 4, m = lane & 15;
  // every load of the matrix is issued before the first is used (one round trip)
  constexpr int kInit = (RP * RP + kInvWaves * 64 - 1) / (kInvWaves * 64);
  double gv[kInit];
#pragma unroll
  for (int u = 0; u < kInit; ++u) {
    const int e = t + u * kInvWaves * 64, i = e / RP, k = e - i * RP;
    const bool ok = e < RP * RP && i < R && k < R;
    const double x = G[ok ? i * R + k : 0];
    gv[u] = ok ? x : 0.0;
  }
  if (lam_dev) lambda = *lam_dev;
  if (t == 0) {
    sbad = st->status != CP_OK;   // one read: another workgroup may set it meanwhile
    if (!sbad && (!(lambda >= 0.0) || !isfinite(lambda))) {
      st->status = CP_EINVAL;
      st->done = 1;
      sbad = 1;
    }
  }
#pragma unroll
  for (int u = 0; u < kInit; ++u) {
    const int e = t + u * kInvWaves * 64, i = e / RP, k = e - i * RP;
    if (e < RP * RP) {
      // lambda I or lambda diag(G) inside the R x R block, the identity past it
      const double v = i < R && k < R ? gv[u] + (i == k ? (diag_damping ? lambda * gv[u] : lambda) : 0.0)
                                      : (i == k ? 1.0 : 0.0);
      M[i * LD + k] = v;
    }
  }
  __syncthreads();
  if (sbad) return;
  auto tile = [&](int I, int J) { return M + (16 * I) * LD + 16 * J; };
  // C += op(A) B over one 16 x 16 x 16 tile product: A operand A[m][4 q + g] (scaled by sa),
  // B operand B[4 q + g][m]; C[g + 4 v][m] in element v.
  auto tprod = [&](const double* A, const double* B, double sa, dv4 c) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      c = mfma64(sa * A[m * LD + 4 * q + g], B[(4 * q + g) * LD + m], c);
    return c;
  };
  auto tload = [&](const double* T) {
    dv4 c;
#pragma unroll
    for (int v = 0; v < 4; ++v) c[v] = T[(g + 4 * v) * LD + m];
    return c;
  };
  auto tstore = [&](double* T, dv4 c) {
#pragma unroll
    for (int v = 0; v < 4; ++v) T[(g + 4 * v) * LD + m] = c[v];
  };
  // Wavefront 0 inverts a diagonal tile in place: lane l holds entries (r, 4 (l % 4) + e),
  // r = l / 4; the row and column of each pivot are exchanged by lane permutes.
  auto pivot_inv = [&](double* D) {
    const int r = lane >> 2, cq = 4 * (lane & 3);
    double a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = D[r * LD + cq + e];
    bool bad = false;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      double rowp[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) rowp[e] = __shfl(a[e], 4 * p + (lane & 3));
      // column p: entry (r, p) sits in lane 4 r + p / 4 of this lane's quad (a quad broadcast);
      // the pivot in lane 4 p + p / 4 (uniform)
      const double ap = a[p & 3];
      double colp;
      switch (p >> 2) {
        case 0: colp = quad_bcast<0>(ap); break;
        case 1: colp = quad_bcast<1>(ap); break;
        case 2: colp = quad_bcast<2>(ap); break;
        default: colp = quad_bcast<3>(ap); break;
      }
      const double piv = read_lane(ap, 4 * p + (p >> 2));
      bad = bad || !(piv > 0.0) || !isfinite(piv);
      // 1 / piv: the hardware reciprocal refined by one Newton step for f(x) = 1/x - piv
      const double r0 = __builtin_amdgcn_rcp(piv);
      const double rp = __fma_rn(r0, __fma_rn(-piv, r0, 1.0), r0);
      const double u = colp * rp;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = cq + e;
        const double upd = a[e] - u * rowp[e];
        a[e] = r == p ? (c == p ? rp : rowp[e] * rp) : (c == p ? -u : upd);
      }
    }
    if (bad && lane == 0) sbad = 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) D[r * LD + cq + e] = a[e];
  };
  if (wv == 0) pivot_inv(tile(0, 0));
  __syncthreads();
  constexpr int NM = NT > 1 ? NT - 1 : 1;
#pragma unroll 1
  for (int k = 0; k < NT; ++k) {
    if (sbad) {   // same value in every thread: uniform exit
      if (t == 0) {
        st->status = CP_ENOTSPD;
        st->done = 1;
      }
      return;
    }
    const double* Dk = tile(k, k);   // (a) already inverted
    // (b) the pivot block row, one tile per wavefront
    for (int j = wv; j < NT - 1; j += kInvWaves) {
      const int jj = j < k ? j : j + 1;
      const dv4 c = tprod(Dk, tile(k, jj), 1.0, dv4{0.0, 0.0, 0.0, 0.0});
      tstore(tile(k, jj), c);
    }
    __syncthreads();
    // (c) wavefront 0 updates the next diagonal tile and inverts it (the next step's (a));
    // wavefronts 1.. form the pivot block column in registers and update the other trailing
    // tiles.
    dv4 colt = {0.0, 0.0, 0.0, 0.0};
    const int ic = wv - 1 < k ? wv - 1 : wv;
    const bool has_col = wv >= 1 && wv <= NT - 1;
    if (wv == 0) {
      if (k + 1 < NT) {
        double* T = tile(k + 1, k + 1);
        tstore(T, tprod(tile(k + 1, k), tile(k, k + 1), -1.0, tload(T)));
        pivot_inv(T);
      }
    } else {
      if (has_col) colt = tprod(tile(ic, k), Dk, -1.0, colt);
      const int un = k + 1 < NT ? k * NM + k : -1;   // the next diagonal tile, done above
      for (int u = wv - 1; u < (NT - 1) * (NT - 1); u += kInvWaves - 1) {
        if (u == un) continue;
        const int i = u / NM, j = u - i * NM;
        const int ii = i < k ? i : i + 1, jj = j < k ? j : j + 1;
        double* T = tile(ii, jj);
        tstore(T, tprod(tile(ii, k), tile(k, jj), -1.0, tload(T)));
      }
    }
    __syncthreads();
    if (has_col) tstore(tile(ic, k), colt);
    __syncthreads();
  }
  for (int e = t; e < R * R; e += kInvWaves * 64) {
    const int i = e / R, k = e - i * R;
    P[e] = M[i * LD + k];
  }
}

template <int NT>
struct KSpdInvBlk {
  struct Args {
    int R;
    const double* G;
    int64_t g_stride;
    double lambda;
    const double* lam_dev;
    double* P;
    int64_t p_stride;
    int first_mode;
    CgState* st;
    int diag_damping;
  };
  static constexpr int kThreads = kInvWaves * 64, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3) {
    spd_inv_blk_body<NT>(a.R, a.G, a.g_stride, a.lambda, a.lam_dev, a.P, a.p_stride,
                         a.first_mode, a.st, a.diag_damping, bid);
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

template <int NT>
__global__ __launch_bounds__(kInvWaves * 64) void k_spd_inv_blk(typename KSpdInvBlk<NT>::Args a) {
  KSpdInvBlk<NT>::run(a, CPGN_BID, CPGN_GDIM);
}

template <int NT>
void KSpdInvBlk<NT>::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL((k_spd_inv_blk<NT>), grid, dim3(kThreads), lds, s, a);
}

int launch_spd_inv_blk(int R, const double* G, int64_t g_stride, double lambda, double* P,
                       int64_t p_stride, int first_mode, int count, CgState* st, hipStream_t s,
                       bool diag_damping, const double* lam_dev) {
  const int NT = (R + 15) / 16;
  const size_t lds = (size_t)16 * NT * (16 * NT + 1) * sizeof(double);
  switch (NT) {
#define CPGN_INV(k)                                                                             \
  case k:                                                                                       \
    dispatch<KSpdInvBlk<k>>(dim3(count), lds, s,                                                \
                            {R, G, g_stride, lambda, lam_dev, P, p_stride, first_mode, st,       \
                             diag_damping ? 1 : 0});                                             \
    break;
    CPGN_INV(1) CPGN_INV(2) CPGN_INV(3) CPGN_INV(4) CPGN_INV(5) CPGN_INV(6) CPGN_INV(7)
    CPGN_INV(8)
#undef CPGN_INV
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_chol_tiles(int R, const double* G, int64_t g_stride, double lambda, double* L,
                      int64_t l_stride, double* Dinv, int64_t d_stride, int first_mode, int count,
                      CgState* st, hipStream_t s) {
  if (R < 1 || R > kMaxGnRank) return (int)hipErrorInvalidValue;
  const int NT = (R + 15) / 16, NTT = NT * (NT + 1) / 2;
  const int slots = (NTT + kCholWaves - 1) / kCholWaves;
#define CPGN_CHOLT(k)                                                                          \
  if (slots <= k) {                                                                          \
    hipLaunchKernelGGL(k_chol_tiles<k>, dim3(count), dim3(kCholWaves * 64), 0, s, R, G,      \
                       g_stride, lambda, L, l_stride, Dinv, d_stride, first_mode, st);       \
    return (int)hipGetLastError();                                                           \
  }
  CPGN_CHOLT(1) CPGN_CHOLT(2) CPGN_CHOLT(4) CPGN_CHOLT(6) CPGN_CHOLT(9) CPGN_CHOLT(kCholMaxSlots)
#undef CPGN_CHOLT
  return (int)hipErrorInvalidValue;
}

int launch_chol_rows(int R, int64_t s, const double* M, const double* L, const double* Dinv,
                     void* A, int dtype, const CgState* st, hipStream_t stream) {
  if (R < 1 || R > kMaxGnRank || s < 1) return (int)hipErrorInvalidValue;
  const int NT = (R + 15) / 16;
  const dim3 grid((unsigned)((s + 63) / 64));
  switch (NT) {
#define CPGN_CHOLR(k)                                                                           \
  case k: {                                                                                    \
    constexpr bool lds = k <= 8;                                                               \
    const size_t bytes =                                                                       \
        (size_t)(4 * 16 * (16 * k + 1) + (lds ? (k * (k + 1) / 2 + k) * 272 : 0)) * sizeof(double); \
    hipLaunchKernelGGL((k_chol_rows<k, lds>), grid, dim3(256), bytes, stream, R, s, M, L, Dinv,  \
                       A, dtype, st);                                                          \
    break;                                                                                     \
  }
    CPGN_CHOLR(1) CPGN_CHOLR(2) CPGN_CHOLR(3) CPGN_CHOLR(4) CPGN_CHOLR(5) CPGN_CHOLR(6)
    CPGN_CHOLR(7) CPGN_CHOLR(8) CPGN_CHOLR(9) CPGN_CHOLR(10) CPGN_CHOLR(11) CPGN_CHOLR(12)
    CPGN_CHOLR(13)
#undef CPGN_CHOLR
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}


// ---------------------------------------------------------------------------------------------
// SPD inverse for R > kMaxGnRank (the matrix no longer fits a workgroup's registers or LDS):
// Gauss-Jordan in place on P = G(n,n) + lambda D in global memory, blocked by 16 x 16 tiles, two
// launches per block step k (K = ceil(R / 16) steps). With M = [[D, B], [C, E]] (block k first),
// one step gives [[D^-1, D^-1 B], [-C D^-1, E - C D^-1 B]]:
//   k_inv_big_row   one workgroup per tile j of block row k (and mode): inverts D (16 x 16 in LDS,
//                   Gauss-Jordan on pivots that must be positive, else CP_ENOTSPD), writes the
//                   new row tile D^-1 P[k][j] (j != k), saves the old column tile C[j] = P[j][k]
//                   and, for j = k, D^-1 to a buffer.
//   k_inv_big_rest  one workgroup per tile (i, j), i != k: P[i][j] -= C[i] P[k][j] (j != k, the
//                   new row), P[i][k] = -C[i] D^-1; and P[k][k] = D^-1.
// tmp holds, per mode, C (K x 16 x 16) and D^-1 (16 x 16).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_inv_big_init(int R, const double* __restrict__ G,
                                                      int64_t g_stride, double lambda,
                                                      const double* __restrict__ lam_dev,
                                                      double* __restrict__ P, int64_t p_stride,
                                                      int first_mode, int diag_damping) {
  const int n = first_mode + blockIdx.y;
  const double lam = lam_dev ? *lam_dev : lambda;
  const double* Gn = G + n * g_stride;
  double* Pn = P + n * p_stride;
  const int64_t RR = (int64_t)R * R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < RR;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R, j = e - i * R;
    double v = Gn[e];
    if (i == j) v += diag_damping ? lam * v : lam;
    Pn[e] = v;
  }
}

// Inverse of the diagonal tile of block k into Ds (LDS, [16][17]); 256 threads, thread (r, c).
// Rows and columns past R hold the identity. Returns false (uniformly) on a pivot that is not
// positive and finite.
__device__ __forceinline__ bool inv_diag_tile(const double* Pn, int R, int k, double (*Ds)[17]) {
  __shared__ int bad;
  const int t = threadIdx.x, r = t >> 4, c = t & 15;
  const int gi = 16 * k + r, gj = 16 * k + c;
  Ds[r][c] = (gi < R && gj < R) ? Pn[(int64_t)gi * R + gj] : (r == c ? 1.0 : 0.0);
  if (t == 0) bad = 0;
  __syncthreads();
  for (int p = 0; p < 16; ++p) {
    const double piv = Ds[p][p];
    const double prow = Ds[p][c], fcol = Ds[r][p];
    __syncthreads();
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (t == 0) bad = 1;
    } else {
      const double rp = (c == p ? 1.0 : prow) / piv;   // row p of the in-place inverse
      if (r == p) Ds[r][c] = rp;
      else Ds[r][c] = (c == p ? 0.0 : Ds[r][c]) - fcol * rp;
    }
    __syncthreads();
  }
  return bad == 0;
}

__global__ __launch_bounds__(256) void k_inv_big_row(int R, double* __restrict__ P,
                                                     int64_t p_stride, int first_mode, int k,
                                                     double* __restrict__ tmp, int64_t t_stride,
                                                     CgState* st) {
  __shared__ double Ds[16][17];
  __shared__ double T[16][17];
  if (st && st->status != CP_OK) return;   // an earlier step failed: the result is not used
  const int n = first_mode + blockIdx.y, j = blockIdx.x;
  const int K = (R + 15) / 16;
  double* Pn = P + n * p_stride;
  double* C = tmp + n * t_stride;          // [K][16][16]
  double* Dinv = C + (int64_t)K * 256;     // [16][16]
  const int t = threadIdx.x, r = t >> 4, c = t & 15;
  const bool ok = inv_diag_tile(Pn, R, k, Ds);
  if (!ok) {
    if (j == 0 && t == 0 && st) {
      st->status = CP_ENOTSPD;
      st->done = 1;
    }
    return;
  }
  if (j == k) {
    Dinv[r * 16 + c] = Ds[r][c];
    return;
  }
  // column tile j of block column k (old values) and row tile (k, j) of P
  const int gi = 16 * j + r, gk = 16 * k + c;
  C[(int64_t)j * 256 + t] = (gi < R && gk < R) ? Pn[(int64_t)gi * R + gk] : 0.0;
  const int rk = 16 * k + r, cj = 16 * j + c;
  T[r][c] = (rk < R && cj < R) ? Pn[(int64_t)rk * R + cj] : 0.0;
  __syncthreads();
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) v = fma(Ds[r][q], T[q][c], v);
  if (rk < R && cj < R) Pn[(int64_t)rk * R + cj] = v;
}

__global__ __launch_bounds__(256) void k_inv_big_rest(int R, double* __restrict__ P,
                                                      int64_t p_stride, int first_mode, int k,
                                                      const double* __restrict__ tmp,
                                                      int64_t t_stride, const CgState* st) {
  __shared__ double Ci[16][17];
  __shared__ double Rk[16][17];
  if (st && st->status != CP_OK) return;
  const int K = (R + 15) / 16;
  const int n = first_mode + blockIdx.z, i = blockIdx.y, j = blockIdx.x;
  double* Pn = P + n * p_stride;
  const double* C = tmp + n * t_stride;
  const double* Dinv = C + (int64_t)K * 256;
  const int t = threadIdx.x, r = t >> 4, c = t & 15;
  const int gi = 16 * i + r, gj = 16 * j + c;
  if (i == k) {
    if (j == k && gi < R && gj < R) Pn[(int64_t)gi * R + gj] = Dinv[t];
    return;
  }
  Ci[r][c] = C[(int64_t)i * 256 + t];
  if (j == k) {
    Rk[r][c] = Dinv[t];
  } else {
    const int rk = 16 * k + r;
    Rk[r][c] = (rk < R && gj < R) ? Pn[(int64_t)rk * R + gj] : 0.0;
  }
  __syncthreads();
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) v = fma(Ci[r][q], Rk[q][c], v);
  if (gi < R && gj < R) {
    const int64_t e = (int64_t)gi * R + gj;
    Pn[e] = j == k ? -v : Pn[e] - v;
  }
}

// Workspace of launch_spd_inv_big per mode (doubles).
int64_t spd_inv_big_tmp(int R) { return (int64_t)((R + 15) / 16) * 256 + 256; }

int launch_spd_inv_big(int R, const double* G, int64_t g_stride, double lambda, double* P,
                       int64_t p_stride, int first_mode, int count, CgState* st, hipStream_t s,
                       bool diag_damping, const double* lam_dev, double* tmp) {
  const int K = (R + 15) / 16;
  const int64_t ts = spd_inv_big_tmp(R);
  const int64_t RR = (int64_t)R * R;
  int g = (int)((RR + 255) / 256);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_inv_big_init, dim3(g, count), dim3(256), 0, s, R, G, g_stride, lambda,
                     lam_dev, P, p_stride, first_mode, diag_damping ? 1 : 0);
  for (int k = 0; k < K; ++k) {
    hipLaunchKernelGGL(k_inv_big_row, dim3(K, count), dim3(256), 0, s, R, P, p_stride,
                       first_mode, k, tmp, ts, st);
    hipLaunchKernelGGL(k_inv_big_rest, dim3(K, K, count), dim3(256), 0, s, R, P, p_stride,
                       first_mode, k, tmp, ts, st);
  }
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// ALS solve for R > kMaxGnRank: A(n) = M (L L^T)^-1 with L L^T = Gamma(n) + lambda I, all in
// global memory, blocked by 16 x 16 tiles (K = ceil(R / 16)).
//   Cholesky, right-looking, two launches per block column k:
//     k_cholb_panel  one workgroup per tile row i >= k: factors the diagonal tile A_kk = L_kk
//                    L_kk^T in LDS (pivots must be positive, else CP_ENOTSPD) and inverts L_kk;
//                    row k stores L_kk (staged) and L_kk^-1, rows i > k store L_ik = A_ik L_kk^-T.
//     k_cholb_trail  one workgroup per tile (i, j), k < j <= i: A_ij -= L_ik L_jk^T; and the
//                    staged L_kk into place.
//   Substitution, one launch per block column: Y L^T = M forward (Y_k = (M_k - sum_{j<k} Y_j
//   L_kj^T) L_kk^-T), then A L = Y backward (A_k = (Y_k - sum_{j>k} A_j L_jk) L_kk^-1); 16 rows
//   x 16 columns per workgroup. Skipped (factors unchanged) when the factorization failed.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cholb_init(int R, const double* __restrict__ G,
                                                    int64_t g_stride, double lambda,
                                                    double* __restrict__ L, int64_t l_stride,
                                                    int mode) {
  const double* Gn = G + mode * g_stride;
  double* Ln = L + mode * l_stride;
  const int64_t RR = (int64_t)R * R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < RR;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R, j = e - i * R;
    Ln[e] = Gn[e] + (i == j ? lambda : 0.0);
  }
}

__global__ __launch_bounds__(256) void k_cholb_panel(int R, double* __restrict__ L,
                                                     int64_t l_stride, int mode, int k,
                                                     double* __restrict__ stage,
                                                     double* __restrict__ Dinv, CgState* st) {
  __shared__ double A[16][17], X[16][17], T[16][17];
  __shared__ int bad;
  if (st->status != CP_OK) return;
  double* Ln = L + mode * l_stride;
  const int i = k + blockIdx.x;
  const int t = threadIdx.x, r = t >> 4, c = t & 15;
  const int gr = 16 * k + r, gc = 16 * k + c;
  A[r][c] = (gr < R && gc < R) ? Ln[(int64_t)gr * R + gc] : (r == c ? 1.0 : 0.0);
  X[r][c] = 0.0;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int p = 0; p < 16; ++p) {   // A_kk = L L^T, column p at a time (lower triangle)
    const double d = A[p][p];
    if (!(d > 0.0) || !isfinite(d)) {
      if (t == 0) bad = 1;
      break;
    }
    const double l = sqrt(d);
    const double arp = A[r][p], acp = A[c][p];
    __syncthreads();
    if (c == p && r >= p) A[r][p] = r == p ? l : arp / l;
    else if (r > p && c > p && c <= r) A[r][c] -= (arp / l) * (acp / l);
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (blockIdx.x == 0 && t == 0) st->status = CP_ENOTSPD;
    return;
  }
  for (int p = 0; p < 16; ++p) {   // X = L_kk^-1 (lower), row p from rows < p
    if (r == p && c <= p) {
      double v = c == p ? 1.0 : 0.0;
      for (int q = c; q < p; ++q) v -= A[p][q] * X[q][c];
      X[p][c] = v / A[p][p];
    }
    __syncthreads();
  }
  if (i == k) {
    stage[t] = c <= r ? A[r][c] : 0.0;
    Dinv[(int64_t)k * 256 + t] = X[r][c];
    return;
  }
  const int ir = 16 * i + r;
  T[r][c] = (ir < R && gc < R) ? Ln[(int64_t)ir * R + gc] : 0.0;
  __syncthreads();
  double v = 0.0;   // L_ik = A_ik L_kk^-T: sum_q A_ik[r][q] X[c][q]
#pragma unroll
  for (int q = 0; q < 16; ++q) v = fma(T[r][q], X[c][q], v);
  if (ir < R && gc < R) Ln[(int64_t)ir * R + gc] = v;
}

__global__ __launch_bounds__(256) void k_cholb_trail(int R, double* __restrict__ L,
                                                     int64_t l_stride, int mode, int k,
                                                     const double* __restrict__ stage,
                                                     const CgState* st) {
  __shared__ double Li[16][17], Lj[16][17];
  if (st->status != CP_OK) return;
  const int i = blockIdx.y, j = blockIdx.x;
  double* Ln = L + mode * l_stride;
  const int t = threadIdx.x, r = t >> 4, c = t & 15;
  if (i == k && j == k) {
    const int gr = 16 * k + r, gc = 16 * k + c;
    if (gr < R && gc < R) Ln[(int64_t)gr * R + gc] = stage[t];
    return;
  }
  if (!(j > k && j <= i)) return;
  const int ir = 16 * i + r, jr = 16 * j + r, kc = 16 * k + c;
  Li[r][c] = (ir < R && kc < R) ? Ln[(int64_t)ir * R + kc] : 0.0;
  Lj[r][c] = (jr < R && kc < R) ? Ln[(int64_t)jr * R + kc] : 0.0;
  __syncthreads();
  double v = 0.0;   // (L_ik L_jk^T)[r][c] = sum_q L_ik[r][q] L_jk[c][q]
#pragma unroll
  for (int q = 0; q < 16; ++q) v = fma(Li[r][q], Lj[c][q], v);
  const int gc = 16 * j + c;
  if (ir < R && gc < R) Ln[(int64_t)ir * R + gc] -= v;
}

// Forward (back = 0) or backward (back = 1) substitution for block column k over 16 rows of the
// mode per workgroup. fwd: In = M, Out = Y; back: In = Y, Out = A (FP64) and Acast.
__global__ __launch_bounds__(256) void k_cholb_solve(int R, int64_t s, const double* __restrict__ In,
                                                     const double* __restrict__ L,
                                                     const double* __restrict__ Dinv, int k,
                                                     int back, double* __restrict__ Out,
                                                     void* __restrict__ Acast, int dtype,
                                                     const CgState* st) {
  __shared__ double U[16][17], D[16][17];
  if (st->status != CP_OK) return;
  const int t = threadIdx.x, r = t >> 4, c = t & 15;
  const int64_t row = (int64_t)blockIdx.x * 16 + r;
  const int col = 16 * k + c;
  D[r][c] = Dinv[(int64_t)k * 256 + t];
  double u = 0.0;
  if (row < s && col < R) {
    u = In[row * R + col];
    const double* Orow = Out + row * R;
    if (!back) {
      for (int q = 0; q < 16 * k; ++q) u -= Orow[q] * L[(int64_t)col * R + q];
    } else {
      for (int q = 16 * (k + 1); q < R; ++q) u -= Orow[q] * L[(int64_t)q * R + col];
    }
  }
  U[r][c] = u;
  __syncthreads();
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q)   // fwd: Y_k = U L_kk^-T; back: A_k = U L_kk^-1
    v = fma(U[r][q], back ? D[q][c] : D[c][q], v);
  if (row < s && col < R) {
    Out[row * R + col] = v;
    if (back) {
      if (dtype == CP_F64) ((double*)Acast)[row * R + col] = v;
      else ((float*)Acast)[row * R + col] = (float)v;
    }
  }
}

// A = M (G_n + lambda I)^-1 for one mode n, R > kMaxGnRank. L: R x R per mode (l_stride),
// Dinv: K x 256 doubles, stage: 256 doubles, Y and A64: s x R doubles of scratch.
int launch_als_solve_big(int R, int64_t s, const double* G, int64_t g_stride, double lambda,
                         double* L, int64_t l_stride, double* Dinv, double* stage, int mode,
                         const double* M, double* Y, double* A64, void* Aout, int dtype,
                         CgState* st, hipStream_t hs) {
  const int K = (R + 15) / 16;
  const int64_t RR = (int64_t)R * R;
  int g = (int)((RR + 255) / 256);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_cholb_init, dim3(g), dim3(256), 0, hs, R, G, g_stride, lambda, L,
                     l_stride, mode);
  double* Ln = L + mode * l_stride;
  for (int k = 0; k < K; ++k) {
    hipLaunchKernelGGL(k_cholb_panel, dim3(K - k), dim3(256), 0, hs, R, L, l_stride, mode, k,
                       stage, Dinv, st);
    hipLaunchKernelGGL(k_cholb_trail, dim3(K, K), dim3(256), 0, hs, R, L, l_stride, mode, k,
                       stage, (const CgState*)st);
  }
  const dim3 rows((unsigned)((s + 15) / 16));
  for (int k = 0; k < K; ++k)
    hipLaunchKernelGGL(k_cholb_solve, rows, dim3(256), 0, hs, R, s, M, (const double*)Ln,
                       (const double*)Dinv, k, 0, Y, nullptr, dtype, (const CgState*)st);
  for (int k = K - 1; k >= 0; --k)
    hipLaunchKernelGGL(k_cholb_solve, rows, dim3(256), 0, hs, R, s, (const double*)Y,
                       (const double*)Ln, (const double*)Dinv, k, 1, A64, Aout, dtype,
                       (const CgState*)st);
  return (int)hipGetLastError();
}

}  // namespace cpgn
