// Algorithm 2 (CP-CG) of Singh, Ma, Yang, Solomonik (arXiv:1910.12331): preconditioned CG on
// (J^T J + lambda I) V = -G with the block preconditioner (Gamma(n,n) + lambda I)^-1 of
// Section 3.3, as three launches per iteration. All vectors are FP64, packed [sum_n s_n, R] by
// mode.
//
//   k_cg_proj    rho = sum <R,Z> and the stop test sum_n ||R(n)||_F <= eps sum_n ||G(n)||_F from
//                the previous launch's per-block partials; beta = rho / rho_old;
//                W = Z + beta W_old; B(p) = A(p)^T W(p), one 16 x 16 tile of B(p) per workgroup
//                (the sum over all s_p rows stays inside the workgroup).
//   k_cg_matvec  Q(n) = lambda W(n) D(n) + W(n) Gamma(n,n) + A(n) Y(n)^T (D = I, or the diagonal
//                of J^T J, diag(Gamma(n,n)), for diagonal damping) with
//                Y(n) = sum_{p != n} Gamma(n,p) * B(p) (eq. (7) contracted in factored form),
//                for a 64-row x 16-column block; per-block <W,Q>.
//   k_cg_update  alpha = rho / sum <W,Q> from the matvec partials; V += alpha W;
//                R_new = R - alpha Q; Z = R_new P_inv(n) for the block; per-block <R_new,Z> and
//                ||R_new||^2 (per mode).
//
// Every workgroup of a launch reduces the previous launch's partials itself, in one fixed order,
// so all of them obtain bitwise the same alpha, beta and stop decision without atomics or a
// second pass; the result does not depend on scheduling. A launch that finds the state done
// returns at once, so the host enqueues cg_maxiter iterations without synchronising. Vectors
// that a launch reads in full rows while other workgroups of the same launch write them (R, W)
// are double-buffered by iteration parity.
//
// The row x (R x R) products run on the 16x16x4 FP64 matrix instruction. Lane l = 16 g + m of a
// wavefront owns row m of a 16-row tile and the contiguous k-range [g K/4, (g+1) K/4) of the
// contraction (K = R padded to 16 KB): its operands are loaded straight from memory into
// registers, all in one batch, while the shared 16-column slice of the R x R operand goes
// through LDS.
#include "batch.h"
#include "mfma64.h"

namespace cpgn {

constexpr int kCgRows = 64;     // rows per workgroup in init / matvec / update (4 wavefronts)
constexpr int kProjWaves = 8;   // wavefronts per B(p) tile in k_cg_proj

struct CgArgs {
  Dims d;
  const double* A64;
  const double* gam;      // Gamma[n][p], R x R each
  const double* pinv;     // P_inv[n]
  double* V;
  double* Rv[2];          // residual, double-buffered; Rv[0] = -G on entry
  double* Z;
  double* W[2];           // search direction, double-buffered
  double* Q;
  double* B;              // B(p) = A(p)^T W(p), [N][R][R]
  double* slot_wq;        // per-block partials [nslot]
  double* slot_rz;
  double* slot_nrm;
  CgState* st;
  double lambda;
  const double* lam_dev;  // when set, the damping is read from here (device memory)
  int diag_damping;       // damping lambda diag(Gamma(n,n)) instead of lambda I
  int TB;                 // 16-column tiles of R
  int nslot;              // row blocks x TB
  int rb_off[kMaxOrder + 1];
};

// Sums of per-block partials, identical in every thread of the workgroup. The slots are staged
// in LDS (1024 at a time); each sum is split into 8 contiguous pieces added sequentially by 8
// threads, and the 8 piece sums are added in order by one thread. This has a shorter critical
// path than a cross-lane butterfly (each xor step is a dependent LDS round trip) and a fixed
// order, so every workgroup gets the same bits; one barrier hands the results to all threads.
//   slot_sums<1>: sum of s0[0..nslot) (unused: a butterfly serves one value as well).
//   slot_sums<2>: sum of s0, and the sums of s1 over each mode's slot range [rb_off[n] TB,
//                 rb_off[n+1] TB) (slot order is mode-major).
template <int K>
__device__ __forceinline__ void slot_sums(const CgArgs& a, const double* s0, const double* s1,
                                          double (&out)[1 + kMaxOrder]) {
  constexpr int kChunkSlots = 1024, kPieces = 8;
  __shared__ double l0[kChunkSlots], l1[K == 2 ? kChunkSlots : 1];
  __shared__ double piece[1 + kMaxOrder][kPieces];
  __shared__ double res[1 + kMaxOrder];
  const int t = threadIdx.x;
  const int nsum = K == 2 ? 1 + a.d.N : 1;
  const int q = t / kPieces, pc = t - q * kPieces;   // sum q, piece pc
  int lo_n = 0, hi_n = a.nslot;
  if (K == 2 && q >= 1 && q < nsum) {
    lo_n = a.rb_off[q - 1] * a.TB;
    hi_n = a.rb_off[q] * a.TB;
  }
  double acc = 0.0;
  for (int c0 = 0; c0 < a.nslot; c0 += kChunkSlots) {
    const int cn = a.nslot - c0 < kChunkSlots ? a.nslot - c0 : kChunkSlots;
    for (int i = t; i < cn; i += blockDim.x) {
      l0[i] = s0[c0 + i];
      if (K == 2) l1[i] = s1[c0 + i];
    }
    __syncthreads();
    if (q < nsum) {
      const int lo = lo_n - c0 > 0 ? lo_n - c0 : 0, hi = hi_n - c0 < cn ? hi_n - c0 : cn;
      if (lo < hi) {
        const int len = hi - lo, per = (len + kPieces - 1) / kPieces;
        const int b0 = lo + pc * per, b1 = b0 + per < hi ? b0 + per : hi;
        const double* src = q == 0 ? l0 : l1;
        for (int i = b0; i < b1; ++i) acc += src[i];
      }
    }
    __syncthreads();
  }
  if (q < nsum) piece[q][pc] = acc;
  __syncthreads();
  if (t < nsum) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < kPieces; ++i) r += piece[t][i];
    res[t] = r;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 1 + kMaxOrder; ++i) out[i] = i < nsum ? res[i] : 0.0;
}

// rho = sum <R,Z> and rsum = sum_n sqrt(sum ||R(n)||^2) from the previous init / update launch.
__device__ __forceinline__ void reduce_rz(const CgArgs& a, double& rho, double& rsum) {
  double v[1 + kMaxOrder];
  slot_sums<2>(a, a.slot_rz, a.slot_nrm, v);
  rho = v[0];
  rsum = 0.0;
#pragma unroll
  for (int n = 0; n < kMaxOrder; ++n)
    if (n < a.d.N) rsum += sqrt(v[1 + n]);
}

// True in every thread of the workgroup when CG has stopped. One thread reads the flag (another
// workgroup of the same launch may be setting it) and the barrier hands its value to all, so
// the early return is uniform; a stopped launch returns before loading anything else.
__device__ __forceinline__ bool cg_stopped(const CgState* st) {
  __shared__ int sdone;
  if (threadIdx.x == 0) sdone = __builtin_nontemporal_load(&st->done);
  __syncthreads();
  return sdone != 0;
}

// Records the CG state before iteration `it` (it iterations done) and decides whether to stop.
// Called by every workgroup with identical inputs; workgroup 0 writes.
__device__ __forceinline__ bool cg_check(const CgArgs& a, int it, double rho, double rho_old,
                                         double rsum, double gsum, double eps, double& beta,
                                         bool writer) {
  beta = it == 0 ? 0.0 : rho / rho_old;
  bool stop = false;
  int status = CP_OK;
  if (!isfinite(rho) || !isfinite(rsum)) {
    status = CP_ENONFINITE;
    stop = true;
  } else if (!(rsum > eps * gsum)) {
    stop = true;
  }
  if (writer && threadIdx.x == 0) {
    CgState* st = a.st;
    st->rho[it & 1] = rho;
    st->rz = rho;
    st->rsum = rsum;
    st->iters = it;
    if (it > 0) st->beta = beta;
    if (stop) {
      st->status = status;
      st->done = 1;
    }
  }
  return stop;
}

// ---------------------------------------------------------------------------------------------
// k_cg_update<KB, INIT>: one 64 x 16 block of Z = R_new P_inv(n), plus V and R for that block.
// INIT: CG initialisation (alpha = 0, V = 0, R = -G unchanged, so R_new = R and Rv is not
// rewritten). Otherwise alpha = rho / sum <W,Q> from k_cg_matvec's partials.
// grid: nslot workgroups of 256 threads; block b covers row block b / TB, columns 16 (b % TB).
// ---------------------------------------------------------------------------------------------
// CHOL: the preconditioner is applied afterwards by k_cg_trsv (triangular solves); this kernel
// then writes V, R_new and the norm partials only.
template <int KB, bool INIT, bool EVEN, bool CHOL>
__device__ __forceinline__ void cg_update_body(const CgArgs& a, int it, int bid) {
  constexpr int KQ = 4 * KB;    // MFMA steps (k values per lane)
  constexpr int KP = 16 * KB;   // padded contraction length
  __shared__ double Ps[slice_elems(KP)];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, m = lane & 15, g = lane >> 4;
  const int R = a.d.R;
  const int rb = bid / a.TB, ct = bid - rb * a.TB, c0 = ct * 16;
  int n = 0;
  while (rb >= a.rb_off[n + 1]) ++n;
  const int64_t s = a.d.s[n];
  const int64_t k0 = (int64_t)(rb - a.rb_off[n]) * kCgRows + wv * 16;   // first row of the tile
  const int64_t rbase = a.d.off[n];
  const double* Rin = a.Rv[it & 1];
  double* Rout = a.Rv[(it + 1) & 1];
  const double* W = a.W[(it + 1) & 1];
  if (cg_stopped(a.st)) return;
  const double rho = INIT ? 0.0 : a.st->rho[it & 1];

  // Operand rows: row k0 + m, k = kstep(j, g).
  const bool rowok = k0 + m < s;
  double ro[KQ], qo[KQ];
  load_oprow<KQ, EVEN>(ro, Rin + (rbase + k0 + m) * R, rowok, R, g);
  if (!INIT) load_oprow<KQ, EVEN>(qo, a.Q + (rbase + k0 + m) * R, rowok, R, g);
  // P_inv(n)[:, c0:c0+16] into LDS (k-major, 16 contiguous columns per k).
  const double* P = a.pinv + (int64_t)n * R * R;
  double ps[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int e = t + 256 * i, k = e >> 4, c = e & 15;
    ps[i] = (!CHOL && k < R && c0 + c < R) ? P[(int64_t)k * R + c0 + c] : 0.0;
  }
  // This lane's outputs: rows k0 + g + 4v, column c0 + m.
  const bool colok = c0 + m < R;
  double rd[4], qd[4], vd[4], wd[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = k0 + g + 4 * v;
    const bool ok = colok && row < s;
    const int64_t e = (rbase + row) * R + c0 + m;
    rd[v] = ok ? Rin[e] : 0.0;
    qd[v] = !INIT && ok ? a.Q[e] : 0.0;
    vd[v] = !INIT && ok ? a.V[e] : 0.0;
    wd[v] = !INIT && ok ? W[e] : 0.0;
  }
  double wq = 0.0;
  if (!INIT) {   // one value: a butterfly is as short as the sequential pieces
    double v1[1] = {0.0};
    for (int i = t; i < a.nslot; i += 256) v1[0] += a.slot_wq[i];
    block_sum(v1);
    wq = v1[0];
  }
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int e = t + 256 * i;
    Ps[sidx(e >> 4, e & 15)] = ps[i];
  }
  double alpha = 0.0;
  if (!INIT) {
    int status = CP_OK;
    if (!isfinite(wq)) status = CP_ENONFINITE;
    else if (!(wq > 0.0)) status = CP_EBREAKDOWN;
    if (status != CP_OK) {
      if (bid == 0 && t == 0) {
        a.st->status = status;
        a.st->done = 1;
      }
      return;
    }
    alpha = rho / wq;
    if (bid == 0 && t == 0) a.st->alpha = alpha;
#pragma unroll
    for (int j = 0; j < KQ; ++j) ro[j] = __fma_rn(-alpha, qo[j], ro[j]);
  }
  __syncthreads();
  dv4 acc = {0.0, 0.0, 0.0, 0.0};
  if constexpr (!CHOL) {
#pragma unroll
    for (int j = 0; j < KQ; ++j)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ro[j], Ps[sidx(kstep(j, g), m)], acc, 0, 0, 0);
  }
  double dot = 0.0, nrm = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = k0 + g + 4 * v;
    if (colok && row < s) {
      const int64_t e = (rbase + row) * R + c0 + m;
      const double rn = INIT ? rd[v] : __fma_rn(-alpha, qd[v], rd[v]);
      if (INIT) {
        a.V[e] = 0.0;
      } else {
        a.V[e] = __fma_rn(alpha, wd[v], vd[v]);
        Rout[e] = rn;
      }
      if constexpr (!CHOL) {
        a.Z[e] = acc[v];
        dot += acc[v] * rn;
      }
      nrm += rn * rn;
    }
  }
  double v2[2] = {dot, nrm};
  block_sum(v2);
  if (t == 0) {
    if constexpr (!CHOL) a.slot_rz[bid] = v2[0];
    a.slot_nrm[bid] = v2[1];
  }
}

template <int KB, bool INIT, bool EVEN, bool CHOL>
__global__ __launch_bounds__(256) void k_cg_update(CgArgs a, int it) {
  cg_update_body<KB, INIT, EVEN, CHOL>(a, it, blockIdx.x);
}

// ---------------------------------------------------------------------------------------------
// k_cg_trsv: Z = R (L L^T)^-1 for one 64-row block of a mode, L the lower Cholesky factor of
// Gamma(n,n) + lambda D (stored in a.pinv). One wavefront; lane k solves row k: the forward solve
// L y = r^T, then the back solve L^T z = y, each entry (r_i - sum_j L_ij y_j) / L_ii with the sum
// split over eight accumulators. The lower triangle of L (packed by rows, 66 KB at R = 128) and y
// (column-major [i][lane], 64 KB, no bank conflicts) sit in LDS, so the sums read LDS only; the
// 130 KB fit gfx950's 160 KB of LDS per workgroup. The block's <R, Z> goes to its first
// column-tile slot and 0 to the others (the slot layout of k_cg_update). R <= 128. R_new is
// Rv[(it + 1) & 1], or Rv[0] for the initialisation.
// ---------------------------------------------------------------------------------------------
template <bool INIT>
__global__ __launch_bounds__(64) void k_cg_trsv(CgArgs a, int it) {
  __shared__ double Ys[128 * 64];
  __shared__ double Lp[128 * 129 / 2];
  const int R = a.d.R, t = threadIdx.x;
  const int rb = blockIdx.x;
  int n = 0;
  while (rb >= a.rb_off[n + 1]) ++n;
  const int64_t s = a.d.s[n];
  const int64_t k0 = (int64_t)(rb - a.rb_off[n]) * kCgRows;
  const int rows = (int)(s - k0 < kCgRows ? s - k0 : kCgRows);
  const double* Rin = INIT ? a.Rv[0] : a.Rv[(it + 1) & 1];
  // No workgroup of this launch writes the flag, so every lane reads the same value (the
  // workgroup is one wavefront: the early exit is uniform).
  if (__builtin_amdgcn_readfirstlane(__builtin_nontemporal_load(&a.st->done)) != 0) return;
  const double* L = a.pinv + (int64_t)n * R * R;
  for (int i0 = 0; i0 < R; i0 += 4) {   // rows i0..i0+3 of L's lower triangle: 8 loads in flight
    double v[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = i0 + u, j = t + 64 * h;
        v[u][h] = (i < R && j <= i) ? L[(int64_t)i * R + j] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = i0 + u, j = t + 64 * h;
        if (i < R && j <= i) Lp[i * (i + 1) / 2 + j] = v[u][h];
      }
  }
  const int64_t row = (a.d.off[n] + k0 + (t < rows ? t : 0)) * R;
  for (int i0 = 0; i0 < R; i0 += 8) {   // this lane's row of R into Ys (rows past the mode: 0)
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (t < rows && i0 + u < R) ? Rin[row + i0 + u] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < R) Ys[(i0 + u) * 64 + t] = v[u];
  }
  __syncthreads();
  double dot = 0.0;
  if (t < rows) {
    for (int i = 0; i < R; ++i) {   // forward: L y = r
      const double* Li = Lp + i * (i + 1) / 2;
      double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int j = 0;
      for (; j + 7 < i; j += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = fma(Li[j + u], Ys[(j + u) * 64 + t], acc[u]);
      }
      for (; j < i; ++j) acc[0] = fma(Li[j], Ys[j * 64 + t], acc[0]);
      const double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                         ((acc[4] + acc[5]) + (acc[6] + acc[7]));
      Ys[i * 64 + t] = (Ys[i * 64 + t] - sum) / Li[i];
    }
    for (int i = R - 1; i >= 0; --i) {   // back: L^T z = y (column i of L below the diagonal)
      double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int j = i + 1;
      for (; j + 7 < R; j += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          acc[u] = fma(Lp[(j + u) * (j + u + 1) / 2 + i], Ys[(j + u) * 64 + t], acc[u]);
      }
      for (; j < R; ++j) acc[0] = fma(Lp[j * (j + 1) / 2 + i], Ys[j * 64 + t], acc[0]);
      const double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                         ((acc[4] + acc[5]) + (acc[6] + acc[7]));
      Ys[i * 64 + t] = (Ys[i * 64 + t] - sum) / Lp[i * (i + 1) / 2 + i];
    }
    for (int i0 = 0; i0 < R; i0 += 8) {   // Z and this row's <R, Z>
      double rv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) rv[u] = i0 + u < R ? Rin[row + i0 + u] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < R) {
          const double z = Ys[(i0 + u) * 64 + t];
          a.Z[row + i0 + u] = z;
          dot = fma(z, rv[u], dot);
        }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) dot += __shfl_xor(dot, o);   // same bits in every lane
  if (t == 0)
    for (int c = 0; c < a.TB; ++c) a.slot_rz[rb * a.TB + c] = c == 0 ? dot : 0.0;
}

// ---------------------------------------------------------------------------------------------
// k_cg_proj: stop test and beta, W = Z + beta W_old (stored by the row-tile-0 workgroups), and
// one 16 x 16 tile of B(p) = A(p)^T W(p). grid: N * TB * TB workgroups of 512 threads; the
// eight wavefronts split the rows of mode p and their partial tiles are added in order.
// ---------------------------------------------------------------------------------------------
constexpr int kProjSteps = 16;   // 4-row MFMA steps loaded per batch and wavefront

struct ProjBatch {
  double av[kProjSteps], zv[kProjSteps], wo[kProjSteps];
};

__device__ __forceinline__ void proj_load(ProjBatch& b, const CgArgs& a, const double* Wold, int it,
                                          int64_t qb, int64_t q1, int64_t s, int64_t base, int R,
                                          int r0, int z0, int m, int g, bool rok, bool zok) {
#pragma unroll
  for (int j = 0; j < kProjSteps; ++j) {
    const int64_t k = (qb + j) * 4 + g;
    const bool ok = qb + j < q1 && k < s;
    const int64_t row = (base + k) * R;
    b.av[j] = ok && rok ? a.A64[row + r0 + m] : 0.0;
    b.zv[j] = ok && zok ? a.Z[row + z0 + m] : 0.0;
    b.wo[j] = ok && zok && it > 0 ? Wold[row + z0 + m] : 0.0;
  }
}

__device__ __forceinline__ void cg_proj_body(const CgArgs& a, int it, int bid) {
  __shared__ double part[kProjWaves][64][4];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, m = lane & 15, g = lane >> 4;
  const int R = a.d.R, TB = a.TB;
  const int p = bid / (TB * TB), rt = (bid / TB) % TB, zt = bid % TB;
  const int r0 = rt * 16, z0 = zt * 16;
  const int64_t s = a.d.s[p], base = a.d.off[p];
  const double* Wold = a.W[it & 1];
  double* Wnew = a.W[(it + 1) & 1];
  // Wavefront wv takes the 4-row steps [q0, q1) of this mode's rows.
  const int64_t nsteps = (s + 3) / 4;
  const int64_t per = (nsteps + kProjWaves - 1) / kProjWaves;
  const int64_t q0 = wv * per, q1 = q0 + per < nsteps ? q0 + per : nsteps;
  const bool rok = r0 + m < R, zok = z0 + m < R;
  const bool store_w = rt == 0 && zok;
  if (cg_stopped(a.st)) return;
  // The first batch of rows is requested before the scalars it waits for.
  ProjBatch b;
  proj_load(b, a, Wold, it, q0, q1, s, base, R, r0, z0, m, g, rok, zok);
  const double gsum = a.st->gsum, eps = a.st->eps, rho_old = a.st->rho[(it + 1) & 1];
  double rho, rsum, beta;
  reduce_rz(a, rho, rsum);
  if (cg_check(a, it, rho, rho_old, rsum, gsum, eps, beta, bid == 0)) return;

  dv4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t qb = q0; qb < q1; qb += kProjSteps) {
    if (qb != q0) proj_load(b, a, Wold, it, qb, q1, s, base, R, r0, z0, m, g, rok, zok);
#pragma unroll
    for (int j = 0; j < kProjSteps; ++j) {
      const double w = it > 0 ? __fma_rn(beta, b.wo[j], b.zv[j]) : b.zv[j];
      const int64_t k = (qb + j) * 4 + g;
      if (store_w && qb + j < q1 && k < s) Wnew[(base + k) * R + z0 + m] = w;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(b.av[j], w, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) part[wv][lane][v] = acc[v];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double bsum = 0.0;
      for (int w = 0; w < kProjWaves; ++w) bsum += part[w][lane][v];
      const int r = r0 + g + 4 * v, z = z0 + m;
      if (r < R && z < R) a.B[(int64_t)p * R * R + (int64_t)r * R + z] = bsum;
    }
  }
}

__global__ __launch_bounds__(512) void k_cg_proj(CgArgs a, int it) { cg_proj_body(a, it, blockIdx.x); }

// ---------------------------------------------------------------------------------------------
// k_cg_matvec<KB>: one 64 x 16 block of Q(n) = lambda W + W Gamma(n,n) + A Y(n)^T and its
// partial <W,Q>. grid: nslot workgroups of 256 threads.
// ---------------------------------------------------------------------------------------------
template <int KB, bool EVEN>
__device__ __forceinline__ void cg_matvec_body(const CgArgs& a, int it, int bid) {
  constexpr int KQ = 4 * KB;
  constexpr int KP = 16 * KB;
  __shared__ double Gs[slice_elems(KP)];   // Gamma(n,n)[k][c0 + c]
  __shared__ double Ys[slice_elems(KP)];   // Y(n)[c0 + c][k]
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, m = lane & 15, g = lane >> 4;
  const int R = a.d.R, N = a.d.N;
  const int64_t RR = (int64_t)R * R;
  const int rb = bid / a.TB, ct = bid - rb * a.TB, c0 = ct * 16;
  int n = 0;
  while (rb >= a.rb_off[n + 1]) ++n;
  const int64_t s = a.d.s[n];
  const int64_t k0 = (int64_t)(rb - a.rb_off[n]) * kCgRows + wv * 16;
  const int64_t rbase = a.d.off[n];
  const double* W = a.W[(it + 1) & 1];
  if (cg_stopped(a.st)) return;

  const bool rowok = k0 + m < s;
  double wo[KQ], ao[KQ];
  load_oprow<KQ, EVEN>(wo, W + (rbase + k0 + m) * R, rowok, R, g);
  load_oprow<KQ, EVEN>(ao, a.A64 + (rbase + k0 + m) * R, rowok, R, g);
  // Shared slices, element e -> (c = e / KP, k = e % KP): contiguous in k in memory.
  const double* Gnn = a.gam + (int64_t)n * (N + 1) * RR;
  double gs[KB], ys[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int e = t + 256 * i, c = e / KP, k = e - c * KP;
    const bool ok = k < R && c0 + c < R;
    gs[i] = ok ? Gnn[(int64_t)(c0 + c) * R + k] : 0.0;   // Gamma(n,n) is symmetric
    ys[i] = 0.0;
  }
  // Y(n) slice: the other modes q != n in ascending order, two per batch of loads.
  for (int qi = 0; qi < N - 1; qi += 2) {
    const int q1 = qi < n ? qi : qi + 1;
    const bool two = qi + 1 < N - 1;
    const int q2 = two ? (qi + 1 < n ? qi + 1 : qi + 2) : q1;
    const double* g1 = a.gam + ((int64_t)n * N + q1) * RR;
    const double* b1 = a.B + (int64_t)q1 * RR;
    const double* g2 = a.gam + ((int64_t)n * N + q2) * RR;
    const double* b2 = a.B + (int64_t)q2 * RR;
    double gv1[KB], bv1[KB], gv2[KB], bv2[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      const int e = t + 256 * i, c = e / KP, k = e - c * KP;
      const bool ok = k < R && c0 + c < R;
      const int64_t off = (int64_t)(c0 + c) * R + k;
      gv1[i] = ok ? g1[off] : 0.0;
      bv1[i] = ok ? b1[off] : 0.0;
      gv2[i] = ok && two ? g2[off] : 0.0;
      bv2[i] = ok && two ? b2[off] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      ys[i] = __fma_rn(gv1[i], bv1[i], ys[i]);
      if (two) ys[i] = __fma_rn(gv2[i], bv2[i], ys[i]);
    }
  }
  const bool colok = c0 + m < R;
  double wd[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = k0 + g + 4 * v;
    wd[v] = colok && row < s ? W[(rbase + row) * R + c0 + m] : 0.0;
  }
  // damping of this lane's column: lambda, or lambda Gamma(n,n)[c][c] (diagonal of J^T J)
  const double lam = a.lam_dev ? *a.lam_dev : a.lambda;
  const double lam_c = a.diag_damping && colok ? lam * Gnn[(int64_t)(c0 + m) * (R + 1)] : lam;
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int e = t + 256 * i, c = e / KP, k = e - c * KP;
    Gs[sidx(k, c)] = gs[i];
    Ys[sidx(k, c)] = ys[i];
  }
  __syncthreads();
  dv4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < KQ; ++j)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wo[j], Gs[sidx(kstep(j, g), m)], acc, 0, 0, 0);
#pragma unroll
  for (int j = 0; j < KQ; ++j)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ao[j], Ys[sidx(kstep(j, g), m)], acc, 0, 0, 0);
  double dot = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = k0 + g + 4 * v;
    if (colok && row < s) {
      const double q = __fma_rn(lam_c, wd[v], acc[v]);
      a.Q[(rbase + row) * R + c0 + m] = q;
      dot += wd[v] * q;
    }
  }
  double v1[1] = {dot};
  block_sum(v1);
  if (t == 0) a.slot_wq[bid] = v1[0];
}

template <int KB, bool EVEN>
__global__ __launch_bounds__(256) void k_cg_matvec(CgArgs a, int it) {
  cg_matvec_body<KB, EVEN>(a, it, blockIdx.x);
}

// After the last enqueued iteration: the state for cg_maxiter completed iterations.
__device__ __forceinline__ void cg_final_body(const CgArgs& a, int maxiter) {
  if (cg_stopped(a.st)) return;
  const double gsum = a.st->gsum, eps = a.st->eps, rho_old = a.st->rho[(maxiter + 1) & 1];
  double rho, rsum, beta;
  reduce_rz(a, rho, rsum);
  cg_check(a, maxiter, rho, rho_old, rsum, gsum, eps, beta, true);
  if (threadIdx.x == 0) a.st->done = 1;
}

__global__ __launch_bounds__(512) void k_cg_final(CgArgs a, int maxiter) { cg_final_body(a, maxiter); }

int cg_tiles(const Plan& p) { return (p.R + 15) / 16; }

int cg_row_blocks(const Plan& p) {
  int nb = 0;
  for (int n = 0; n < p.N; ++n) nb += (int)((p.s[n] + kCgRows - 1) / kCgRows);
  return nb;
}

size_t cg_slot_bytes(const Plan& p) {
  return (size_t)3 * cg_row_blocks(p) * cg_tiles(p) * sizeof(double);
}

template <int KB, bool EVEN, bool CHOL>
static void launch_kb(const CgArgs& a, int N, int maxiter, hipStream_t s) {
  const int nrb = a.rb_off[N];
  hipLaunchKernelGGL((k_cg_update<KB, true, EVEN, CHOL>), dim3(a.nslot), dim3(256), 0, s, a, 0);
  if (CHOL) hipLaunchKernelGGL(k_cg_trsv<true>, dim3(nrb), dim3(64), 0, s, a, 0);
  for (int it = 0; it < maxiter; ++it) {
    hipLaunchKernelGGL(k_cg_proj, dim3(N * a.TB * a.TB), dim3(512), 0, s, a, it);
    hipLaunchKernelGGL((k_cg_matvec<KB, EVEN>), dim3(a.nslot), dim3(256), 0, s, a, it);
    hipLaunchKernelGGL((k_cg_update<KB, false, EVEN, CHOL>), dim3(a.nslot), dim3(256), 0, s, a,
                       it);
    if (CHOL) hipLaunchKernelGGL(k_cg_trsv<false>, dim3(nrb), dim3(64), 0, s, a, it);
  }
  hipLaunchKernelGGL(k_cg_final, dim3(1), dim3(512), 0, s, a, maxiter);
}

template <int KB>
static void launch_kb(const CgArgs& a, int N, int maxiter, hipStream_t s, bool chol) {
  if (chol) {
    if constexpr (KB <= 8) {
      if (a.d.R % 2 == 0) launch_kb<KB, true, true>(a, N, maxiter, s);
      else launch_kb<KB, false, true>(a, N, maxiter, s);
    }
    return;
  }
  if (a.d.R % 2 == 0) launch_kb<KB, true, false>(a, N, maxiter, s);
  else launch_kb<KB, false, false>(a, N, maxiter, s);
}

static CgArgs make_cg_args(const Plan& p, const Dims& d, const double* A64, const double* gam,
                           const double* pinv, double* V, double* R0, double* R1, double* Z,
                           double* W0, double* W1, double* Q, double* B, void* slots, CgState* st,
                           double lambda, bool diag_damping, const double* lam_dev) {
  CgArgs a{};
  a.d = d;
  a.A64 = A64;
  a.gam = gam;
  a.pinv = pinv;
  a.V = V;
  a.Rv[0] = R0;
  a.Rv[1] = R1;
  a.Z = Z;
  a.W[0] = W0;
  a.W[1] = W1;
  a.Q = Q;
  a.B = B;
  a.st = st;
  a.lambda = lambda;
  a.lam_dev = lam_dev;
  a.diag_damping = diag_damping ? 1 : 0;
  a.TB = cg_tiles(p);
  a.rb_off[0] = 0;
  for (int n = 0; n < p.N; ++n)
    a.rb_off[n + 1] = a.rb_off[n] + (int)((p.s[n] + kCgRows - 1) / kCgRows);
  a.nslot = a.rb_off[p.N] * a.TB;
  a.slot_wq = (double*)slots;
  a.slot_rz = a.slot_wq + a.nslot;
  a.slot_nrm = a.slot_rz + a.nslot;
  return a;
}

// Enqueues CG initialisation, cg_maxiter iterations and the final state. R = -G must be in R0.
int launch_cg(const Plan& p, const Dims& d, const double* A64, const double* gam,
              const double* pinv, double* V, double* R0, double* R1, double* Z, double* W0,
              double* W1, double* Q, double* B, void* slots, CgState* st, double lambda,
              int maxiter, bool diag_damping, hipStream_t s, const double* lam_dev, bool chol) {
  if (chol && p.R > 128) return (int)hipErrorInvalidValue;
  const CgArgs a = make_cg_args(p, d, A64, gam, pinv, V, R0, R1, Z, W0, W1, Q, B, slots, st,
                                lambda, diag_damping, lam_dev);
  switch (a.TB) {
    case 1: launch_kb<1>(a, p.N, maxiter, s, chol); break;
    case 2: launch_kb<2>(a, p.N, maxiter, s, chol); break;
    case 3: launch_kb<3>(a, p.N, maxiter, s, chol); break;
    case 4: launch_kb<4>(a, p.N, maxiter, s, chol); break;
    case 5: launch_kb<5>(a, p.N, maxiter, s, chol); break;
    case 6: launch_kb<6>(a, p.N, maxiter, s, chol); break;
    case 7: launch_kb<7>(a, p.N, maxiter, s, chol); break;
    case 8: launch_kb<8>(a, p.N, maxiter, s, chol); break;
    // 128 < R <= 208: operand rows of up to 52 doubles per lane (no scratch; part in AGPRs)
    case 9: launch_kb<9>(a, p.N, maxiter, s, chol); break;
    case 10: launch_kb<10>(a, p.N, maxiter, s, chol); break;
    case 11: launch_kb<11>(a, p.N, maxiter, s, chol); break;
    case 12: launch_kb<12>(a, p.N, maxiter, s, chol); break;
    case 13: launch_kb<13>(a, p.N, maxiter, s, chol); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Batched CG: the iterations of many independent problems in shared launches. Each problem's
// CgArgs sits in its own workspace (written by launch_cg_store when its step begins); a launch
// covers the workgroups of every problem back to back, and workgroup b finds its problem q as the
// one with off[q] <= b < off[q + 1]. Every problem runs the bodies above on its own state, with
// the column-block count of the largest rank in the batch (extra blocks are zero: the results
// are bitwise those of the problem's own launches); a problem whose CG has stopped returns at
// once, as in its own launches.
// ---------------------------------------------------------------------------------------------
struct CgBatch {
  const CgArgs* args[kMaxCgBatch];
  int off[kMaxCgBatch + 1];    // workgroups before each problem: update and matvec launches
  int offp[kMaxCgBatch + 1];   // the same for the projection launch
  int n;
};

struct KCgStore {
  struct Args {
    CgArgs a;
    CgArgs* dst;
  };
  static constexpr int kThreads = 64, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& x, dim3, dim3) {
    if (threadIdx.x == 0) *x.dst = x.a;
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& x);
};

__global__ __launch_bounds__(64) void k_cg_store(KCgStore::Args x) {
  KCgStore::run(x, CPGN_BID, CPGN_GDIM);
}

void KCgStore::direct(dim3 grid, size_t lds, hipStream_t s, const Args& x) {
  hipLaunchKernelGGL(k_cg_store, grid, dim3(kThreads), lds, s, x);
}

size_t cg_args_bytes() { return sizeof(CgArgs); }

void launch_cg_store(const Plan& p, const Dims& d, const double* A64, const double* gam,
                     const double* pinv, double* V, double* R0, double* R1, double* Z, double* W0,
                     double* W1, double* Q, double* B, void* slots, CgState* st, double lambda,
                     bool diag_damping, const double* lam_dev, void* dst, hipStream_t s) {
  const CgArgs a = make_cg_args(p, d, A64, gam, pinv, V, R0, R1, Z, W0, W1, Q, B, slots, st,
                                lambda, diag_damping, lam_dev);
  dispatch<KCgStore>(dim3(1), 0, s, {a, (CgArgs*)dst});
}

// Problem of this workgroup and its workgroup index within that problem (uniform).
__device__ __forceinline__ int batch_find(const int* off, int n, int& local) {
  __shared__ int sq;
  for (int q = threadIdx.x; q < n; q += blockDim.x)
    if (off[q] <= (int)blockIdx.x && (int)blockIdx.x < off[q + 1]) sq = q;
  __syncthreads();
  const int q = sq;
  local = (int)blockIdx.x - off[q];
  return q;
}

template <int KB, bool INIT, bool EVEN>
__global__ __launch_bounds__(256) void k_cg_update_batch(CgBatch b, int it) {
  int bid;
  const int q = batch_find(b.off, b.n, bid);
  cg_update_body<KB, INIT, EVEN, false>(*b.args[q], it, bid);
}

__global__ __launch_bounds__(512) void k_cg_proj_batch(CgBatch b, int it) {
  int bid;
  const int q = batch_find(b.offp, b.n, bid);
  cg_proj_body(*b.args[q], it, bid);
}

template <int KB, bool EVEN>
__global__ __launch_bounds__(256) void k_cg_matvec_batch(CgBatch b, int it) {
  int bid;
  const int q = batch_find(b.off, b.n, bid);
  cg_matvec_body<KB, EVEN>(*b.args[q], it, bid);
}

__global__ __launch_bounds__(512) void k_cg_final_batch(CgBatch b, int maxiter) {
  cg_final_body(*b.args[blockIdx.x], maxiter);
}

template <int KB, bool EVEN>
static void launch_batch_kb(const CgBatch& b, int maxiter, hipStream_t s) {
  const dim3 gu((unsigned)b.off[b.n]), gp((unsigned)b.offp[b.n]);
  hipLaunchKernelGGL((k_cg_update_batch<KB, true, EVEN>), gu, dim3(256), 0, s, b, 0);
  for (int it = 0; it < maxiter; ++it) {
    hipLaunchKernelGGL(k_cg_proj_batch, gp, dim3(512), 0, s, b, it);
    hipLaunchKernelGGL((k_cg_matvec_batch<KB, EVEN>), gu, dim3(256), 0, s, b, it);
    hipLaunchKernelGGL((k_cg_update_batch<KB, false, EVEN>), gu, dim3(256), 0, s, b, it);
  }
  hipLaunchKernelGGL(k_cg_final_batch, dim3((unsigned)b.n), dim3(512), 0, s, b, maxiter);
}

// plans[i], args[i] (device CgArgs written by launch_cg_store) of count <= kMaxCgBatch problems,
// all with R <= 128 and the explicit-inverse preconditioner.
int launch_cg_batch(int count, const Plan* plans, void* const* args, int maxiter, hipStream_t s) {
  if (count < 1 || count > kMaxCgBatch) return (int)hipErrorInvalidValue;
  CgBatch b{};
  b.n = count;
  int tb = 1;
  bool even = true;
  for (int i = 0; i < count; ++i) {
    const Plan& p = plans[i];
    const int t = cg_tiles(p);
    tb = t > tb ? t : tb;
    even = even && p.R % 2 == 0;
    b.args[i] = (const CgArgs*)args[i];
    b.off[i + 1] = b.off[i] + cg_row_blocks(p) * t;
    b.offp[i + 1] = b.offp[i] + p.N * t * t;
  }
  switch (tb) {
#define CPGN_CGB(k)                                                                  \
  case k:                                                                            \
    if (even) launch_batch_kb<k, true>(b, maxiter, s);                               \
    else launch_batch_kb<k, false>(b, maxiter, s);                                   \
    break;
    CPGN_CGB(1) CPGN_CGB(2) CPGN_CGB(3) CPGN_CGB(4) CPGN_CGB(5) CPGN_CGB(6) CPGN_CGB(7)
    CPGN_CGB(8)
#undef CPGN_CGB
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // namespace cpgn
