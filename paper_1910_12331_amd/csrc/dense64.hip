// FP64 matrix-core kernels for the small dense products of a Gauss-Newton step:
//   k_gram_mfma   C(n) = X(n)^T Y(n) (Grams S(n) = A(n)^T A(n), Section 2.2, and the
//                 B(p) = A(p)^T W(p) of eq. (7)), one 16 x 16 tile per workgroup.
//   k_rowmm_mfma  Out(n) = c In(n) + L1(n) T1(n) + L2(n) T2(n)^T for 64-row x 16-column blocks
//                 (the gradient G = A Gamma(n,n) - M of Algorithm 1, the ALS solve
//                 M P_inv(n), and the rows of the implicit product of eq. (7)), with per-block
//                 partial sums of <Out, D> and ||Out||^2 for the scalar reductions.
#include "batch.h"
#include "mfma64.h"

namespace cpgn {

constexpr int kGramWaves = 8;
constexpr int kGramSteps = 16;   // 4-row MFMA steps loaded per batch and wavefront

// grid: (TB * TB, 1, number of modes), 512 threads. The eight wavefronts split the rows of the
// mode; their partial tiles are added in wavefront order.
__device__ __forceinline__ void gram_body(const Dims& d, const double* __restrict__ Xp,
                                          const double* __restrict__ Yp, double* __restrict__ C,
                                          int mode_only, const CgState* st, dim3 bid) {
  if (st && st->done) return;   // written only by earlier launches
  __shared__ double part[kGramWaves][64][4];
  const int n = mode_only >= 0 ? mode_only : bid.z;
  const int R = d.R, TB = (R + 15) / 16;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, m = lane & 15, g = lane >> 4;
  const int r0 = 16 * (bid.x / TB), z0 = 16 * (bid.x % TB);
  const int64_t s = d.s[n], base = d.off[n];
  const int64_t nsteps = (s + 3) / 4;
  const int64_t per = (nsteps + kGramWaves - 1) / kGramWaves;
  const int64_t q0 = wv * per, q1 = q0 + per < nsteps ? q0 + per : nsteps;
  const bool rok = r0 + m < R, zok = z0 + m < R;
  dv4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t qb = q0; qb < q1; qb += kGramSteps) {
    double xv[kGramSteps], yv[kGramSteps];
#pragma unroll
    for (int j = 0; j < kGramSteps; ++j) {
      const int64_t k = (qb + j) * 4 + g;
      const bool ok = qb + j < q1 && k < s;
      const int64_t row = (base + k) * R;
      xv[j] = ok && rok ? Xp[row + r0 + m] : 0.0;
      yv[j] = ok && zok ? Yp[row + z0 + m] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kGramSteps; ++j) acc = mfma64(xv[j], yv[j], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) part[wv][lane][v] = acc[v];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double c = 0.0;
      for (int w = 0; w < kGramWaves; ++w) c += part[w][lane][v];
      const int r = r0 + g + 4 * v, z = z0 + m;
      if (r < R && z < R) C[((int64_t)n * R + r) * R + z] = c;
    }
  }
}

struct KGram {
  struct Args {
    Dims d;
    const double* X;
    const double* Y;
    double* C;
    int mode_only;
    const CgState* st;
  };
  static constexpr int kThreads = 512, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3) {
    gram_body(a.d, a.X, a.Y, a.C, a.mode_only, a.st, bid);
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

__global__ __launch_bounds__(512) void k_gram_mfma(KGram::Args a) { KGram::run(a, CPGN_BID, CPGN_GDIM); }

void KGram::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_gram_mfma, grid, dim3(kThreads), lds, s, a);
}

void launch_gram_mfma(const Dims& d, const double* X, const double* Y, double* C, int mode_only,
                      const CgState* st, hipStream_t s) {
  const int TB = (d.R + 15) / 16;
  dim3 grid(TB * TB, 1, mode_only >= 0 ? 1 : d.N);
  dispatch<KGram>(grid, 0, s, {d, X, Y, C, mode_only, st});
}

// ---------------------------------------------------------------------------------------------
// grid: (nbx, modes) with nbx a multiple of TB; block x covers column tile x % TB and the row
// blocks x / TB, x / TB + nbx / TB, ... of its mode, so that nbx partial-sum slots per mode
// suffice for any number of rows.
// ---------------------------------------------------------------------------------------------
template <int KB, bool EVEN>
__device__ __forceinline__ void rowmm_body(const Dims& d, const RowMM& a, const CgState* st,
                                           dim3 bid, dim3 gdim) {
  constexpr int KQ = 4 * KB;
  constexpr int KP = 16 * KB;
  __shared__ double T1s[slice_elems(KP)];   // T1(n)[k][c0 + c]
  __shared__ double T2s[slice_elems(KP)];   // T2(n)[c0 + c][k]
  if (st && (st->done || (a.skip_if_status && st->status != 0))) return;   // earlier launches
  const int n = a.mode_only >= 0 ? a.mode_only : bid.y;
  const int R = d.R, TB = (R + 15) / 16;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, m = lane & 15, g = lane >> 4;
  const int ct = bid.x % TB, c0 = ct * 16;
  const int64_t s = d.s[n], base = d.off[n];
  const int64_t nrb = (s + 63) / 64, rstride = gdim.x / TB;
  const double* T1 = a.t1 ? a.t1 + n * a.t1_stride : nullptr;
  const double* T2 = a.t2 ? a.t2 + n * a.t2_stride : nullptr;
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int e = t + 256 * i;
    {   // T1 slice, element e -> (k = e / 16, c = e % 16): 16 contiguous columns per k
      const int k = e >> 4, c = e & 15;
      T1s[sidx(k, c)] = (T1 && k < R && c0 + c < R) ? T1[(int64_t)k * R + c0 + c] : 0.0;
    }
    {   // T2 slice, element e -> (c = e / KP, k = e % KP): contiguous in k
      const int c = e / KP, k = e - c * KP;
      T2s[sidx(k, c)] = (T2 && k < R && c0 + c < R) ? T2[(int64_t)(c0 + c) * R + k] : 0.0;
    }
  }
  __syncthreads();
  const bool colok = c0 + m < R;
  double dot = 0.0, nrm = 0.0;
  for (int64_t rb = bid.x / TB; rb < nrb; rb += rstride) {
    const int64_t k0 = rb * 64 + wv * 16;
    const bool rowok = k0 + m < s;
    dv4 acc = {0.0, 0.0, 0.0, 0.0};
    if (T1) {
      double lo[KQ];
      load_oprow<KQ, EVEN>(lo, a.l1 + (base + k0 + m) * R, rowok, R, g);
#pragma unroll
      for (int j = 0; j < KQ; ++j) acc = mfma64(lo[j], T1s[sidx(kstep(j, g), m)], acc);
    }
    if (T2) {
      double lo[KQ];
      load_oprow<KQ, EVEN>(lo, a.l2 + (base + k0 + m) * R, rowok, R, g);
#pragma unroll
      for (int j = 0; j < KQ; ++j) acc = mfma64(lo[j], T2s[sidx(kstep(j, g), m)], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = k0 + g + 4 * v;
      if (colok && row < s) {
        const int64_t e = row * R + c0 + m, at = base * R + e;
        double val = acc[v];
        if (a.in) val = __fma_rn(a.cin, a.in[at], val);
        if (a.out) a.out[at] = val;
        if (a.out2) a.out2[at] = a.out2_scale * val;
        if (a.cast_out.p[n]) {
          if (a.cast_dtype == CP_F64) ((double*)a.cast_out.p[n])[e] = val;
          else ((float*)a.cast_out.p[n])[e] = (float)val;
        }
        if (a.dotw) dot += val * a.dotw[at];
        nrm += val * val;
      }
    }
  }
  if (a.red_dot || a.red_nrm) {
    double v2[2] = {dot, nrm};
    block_sum(v2);
    if (t == 0) {
      if (a.red_dot) a.red_dot[n * kRedSlots + bid.x] = v2[0];
      if (a.red_nrm) a.red_nrm[n * kRedSlots + bid.x] = v2[1];
    }
  }
}

template <int KB, bool EVEN>
struct KRowmm {
  struct Args {
    Dims d;
    RowMM a;
    const CgState* st;
  };
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& x, dim3 bid, dim3 gdim) {
    rowmm_body<KB, EVEN>(x.d, x.a, x.st, bid, gdim);
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& x);
};

template <int KB, bool EVEN>
__global__ __launch_bounds__(256) void k_rowmm_mfma(typename KRowmm<KB, EVEN>::Args x) {
  KRowmm<KB, EVEN>::run(x, CPGN_BID, CPGN_GDIM);
}

template <int KB, bool EVEN>
void KRowmm<KB, EVEN>::direct(dim3 grid, size_t lds, hipStream_t s, const Args& x) {
  hipLaunchKernelGGL((k_rowmm_mfma<KB, EVEN>), grid, dim3(kThreads), lds, s, x);
}

// Partial-sum slots per mode used by k_rowmm_mfma: TB column tiles x up to kRedSlots / TB row
// blocks (row blocks beyond that are strided over the same workgroups).
int rowmm_mfma_blocks(const Dims& d) {
  const int TB = (d.R + 15) / 16;
  int64_t nrb = 0;
  for (int n = 0; n < d.N; ++n) nrb = (d.s[n] + 63) / 64 > nrb ? (d.s[n] + 63) / 64 : nrb;
  const int64_t cap = kRedSlots / TB;
  return (int)(TB * (nrb < cap ? nrb : cap));
}

template <int KB>
static void launch_rowmm_kb(const Dims& d, const RowMM& a, const CgState* st, hipStream_t s) {
  dim3 grid(rowmm_mfma_blocks(d), a.mode_only >= 0 ? 1 : d.N);
  if (d.R % 2 == 0) dispatch<KRowmm<KB, true>>(grid, 0, s, {d, a, st});
  else dispatch<KRowmm<KB, false>>(grid, 0, s, {d, a, st});
}

// R <= 128 only.
void launch_rowmm_mfma(const Dims& d, const RowMM& a, const CgState* st, hipStream_t s) {
  switch ((d.R + 15) / 16) {
    case 1: launch_rowmm_kb<1>(d, a, st, s); break;
    case 2: launch_rowmm_kb<2>(d, a, st, s); break;
    case 3: launch_rowmm_kb<3>(d, a, st, s); break;
    case 4: launch_rowmm_kb<4>(d, a, st, s); break;
    case 5: launch_rowmm_kb<5>(d, a, st, s); break;
    case 6: launch_rowmm_kb<6>(d, a, st, s); break;
    case 7: launch_rowmm_kb<7>(d, a, st, s); break;
    case 8: launch_rowmm_kb<8>(d, a, st, s); break;
    default: break;
  }
}

}  // namespace cpgn
