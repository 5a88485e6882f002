// Dense MTTKRP on the gfx950 matrix cores (Section 2.2 of Singh, Ma, Yang, Solomonik,
// arXiv:1910.12331): M(n)[j,r] = sum over i with i_n = j of X[i] * prod_{m != n} A(m)[i_m, r].
//
// Formulation. View C-order X as [L, J, Rr] (L = prod of the dims before mode n, J = s_n,
// Rr = prod of the dims after it). The contraction runs over every index but i_n; it is split
// into an "inner" mode q whose factor is packed for the MFMA B operand, and the remaining
// "outer" modes whose Khatri-Rao row KRP_outer(o, :) is formed once per outer index o and
// multiplied into the packed inner factor on the fly:
//   case A (n < N-1): q = N-1, the contraction index runs contiguously along X rows; lanes
//     cover 16 output rows j and each lane loads 4 consecutive inner elements with one vector
//     load (the 4 substeps of 4 MFMAs consume them, so the contraction order inside a
//     16-element chunk is permuted consistently in A and B).
//   case B (n = N-1): q = N-2 and the output rows are the contiguous index; each lane loads
//     MB consecutive output rows (one per 16-row block) per inner index.
// Every wavefront owns a tile of 16*MB output rows and an equal share of the flattened
// (outer index, inner chunk) items; its FP32/FP64 accumulators stay in registers. The four
// wavefronts of a workgroup are summed through LDS in a fixed order and each workgroup writes
// one partial tile; a second kernel adds the partials in a fixed order in FP64, so results
// are bitwise reproducible.
#include "cpgn_internal.h"

namespace cpgn {

template <typename T> struct MttkrpCfg;
template <> struct MttkrpCfg<float> { static constexpr int MB = 4; };   // 64 output rows
template <> struct MttkrpCfg<double> { static constexpr int MB = 2; };  // 32 output rows

struct MttkrpArgs {
  const void* X;
  const void* apad[kMaxOrder];  // padded factors [s_m][Rp], compute precision
  const void* fpk;              // packed inner factor [QC][NBt][64 lanes][4]
  void* part;                   // partial tiles [split_wgs][Jpad][Rp]
  int64_t J, Jpad, s_in, QC, nitems, Rr, nbo;
  int64_t outer_size[kMaxOrder];
  int outer_mode[kMaxOrder];
  int n_outer;
  int Rp, NBt, cb0;
  int nsplit;                   // wavefronts along the contraction split (= 4 * gridDim.x)
};

template <typename T, int MB> struct VecLoad;
template <> struct VecLoad<float, 4> {
  typedef float v __attribute__((ext_vector_type(4)));
};
template <> struct VecLoad<double, 2> {
  typedef double v __attribute__((ext_vector_type(2)));
};

template <typename T, bool CASE_B, int NB, bool VEC>
__global__ __launch_bounds__(256, 2) void k_mttkrp(MttkrpArgs a) {
  constexpr int MB = MttkrpCfg<T>::MB;
  typedef typename Mfma<T>::v4 v4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4, m = lane & 15;
  const int split = blockIdx.x * 4 + wave;
  const int64_t j0 = (int64_t)blockIdx.y * 16 * MB;
  const int64_t it0 = a.nitems * split / a.nsplit;
  const int64_t it1 = a.nitems * (split + 1) / a.nsplit;
  const T* __restrict__ X = (const T*)a.X;
  const v4* __restrict__ F = (const v4*)a.fpk;

  v4 acc[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[i][nb] = v4{0, 0, 0, 0};

  T kro[NB];
  int64_t o_cur = -1, base = 0;
  for (int64_t it = it0; it < it1; ++it) {
    const int64_t o = it / a.QC;
    const int64_t chunk = it - o * a.QC;
    if (o != o_cur) {
      o_cur = o;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) kro[nb] = T(1);
      int64_t rem = o;
      for (int d = a.n_outer - 1; d >= 0; --d) {
        const int64_t sz = a.outer_size[d];
        const int64_t idx = rem % sz;
        rem /= sz;
        const T* row = (const T*)a.apad[a.outer_mode[d]] + idx * a.Rp + 16 * a.cb0 + m;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) kro[nb] *= row[16 * nb];
      }
      if (!CASE_B) {
        const int64_t aa = o / a.nbo, bo = o - aa * a.nbo;
        base = aa * a.J * a.Rr + bo * a.s_in;
      } else {
        base = o * a.s_in * a.J;
      }
    }
    T b[4][NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const v4 f = F[(chunk * a.NBt + a.cb0 + nb) * kWave + lane];
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t][nb] = f[t] * kro[nb];
    }
    const int64_t in0 = chunk * 16 + 4 * g;
    if (!CASE_B) {
      v4 xv[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int64_t j = j0 + 16 * mb + m;
        const T* p = X + base + j * a.Rr + in0;
        if (VEC) {
          xv[mb] = (j < a.J && in0 < a.s_in) ? *(const v4*)p : v4{0, 0, 0, 0};
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) xv[mb][t] = (j < a.J && in0 + t < a.s_in) ? p[t] : T(0);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = Mfma<T>::mac(xv[mb][t], b[t][nb], acc[mb][nb]);
    } else {
      const int64_t jb = j0 + MB * m;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t inn = in0 + t;
        const T* p = X + base + inn * a.J + jb;
        T xv[MB];
        if (VEC) {
          typedef typename VecLoad<T, MB>::v vv;
          vv w = (inn < a.s_in && jb < a.J) ? *(const vv*)p : vv{};
#pragma unroll
          for (int v = 0; v < MB; ++v) xv[v] = w[v];
        } else {
#pragma unroll
          for (int v = 0; v < MB; ++v) xv[v] = (inn < a.s_in && jb + v < a.J) ? p[v] : T(0);
        }
#pragma unroll
        for (int v = 0; v < MB; ++v)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[v][nb] = Mfma<T>::mac(xv[v], b[t][nb], acc[v][nb]);
      }
    }
  }

  // Fixed-order sum of the four wavefronts: (w0 + w2) + (w1 + w3).
  __shared__ v4 red[2][MB * NB][kWave];
  if (wave >= 2) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) red[wave - 2][mb * NB + nb][lane] = acc[mb][nb];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] += red[wave][mb * NB + nb][lane];
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) red[0][mb * NB + nb][lane] = acc[mb][nb];
  }
  __syncthreads();
  if (wave == 0) {
    T* P = (T*)a.part + (int64_t)blockIdx.x * a.Jpad * a.Rp;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const v4 tot = acc[mb][nb] + red[0][mb * NB + nb][lane];
        const int col = 16 * (a.cb0 + nb) + m;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = Mfma<T>::out_row(lane, v);
          const int64_t row = CASE_B ? (j0 + (int64_t)MB * i + mb) : (j0 + 16 * mb + i);
          P[row * a.Rp + col] = tot[v];
        }
      }
  }
}

// M[j, r] = sum over partial tiles, in FP64, fixed order. Writes the FP64 result and/or a copy
// in the caller's precision.
template <typename T>
__global__ void k_mttkrp_reduce(const T* __restrict__ part, int nparts, int64_t Jpad, int Rp,
                                int64_t J, int R, double* __restrict__ m64, void* mout,
                                int mout_dtype) {
  const int64_t n = J * R;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx / R;
    const int r = (int)(idx - j * R);
    double s = 0.0;
    const T* p = part + j * Rp + r;
    for (int q = 0; q < nparts; ++q) s += (double)p[(int64_t)q * Jpad * Rp];
    if (m64) m64[idx] = s;
    if (mout) {
      if (mout_dtype == CP_F64) ((double*)mout)[idx] = s;
      else ((float*)mout)[idx] = (float)s;
    }
  }
}

// Padded factor copies [s_m][Rp] in the compute precision, optional FP64 copies [s_m][R], and
// the packed B-operand layout of modes N-1 and N-2:
//   fpk[chunk][cb][lane][t] = A(q)[16*chunk + 4*(lane/16) + t][16*cb + lane%16]  (0 outside).
struct PrepArgs {
  const void* src[kMaxOrder];
  int src_dtype;
  void* apad[kMaxOrder];
  double* a64[kMaxOrder];
  void* fpk_last;
  void* fpk_prev;
  int64_t s[kMaxOrder];
  int64_t seg[kMaxOrder + 3];   // cumulative segment starts: modes' apad, then the two packs
  int N, R, Rp, NBt;
  int64_t qc_last, qc_prev;
};

template <typename T>
__device__ __forceinline__ double src_at(const PrepArgs& a, int mode, int64_t i, int r) {
  return a.src_dtype == CP_F64 ? ((const double*)a.src[mode])[i * a.R + r]
                               : (double)((const float*)a.src[mode])[i * a.R + r];
}

template <typename T>
__global__ void k_prepare(PrepArgs a) {
  const int64_t total = a.seg[a.N + 2];
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < a.seg[a.N]) {
      int mode = 0;
      while (idx >= a.seg[mode + 1]) ++mode;
      const int64_t e = idx - a.seg[mode];
      const int64_t i = e / a.Rp;
      const int c = (int)(e - i * a.Rp);
      const double v = c < a.R ? src_at<T>(a, mode, i, c) : 0.0;
      ((T*)a.apad[mode])[e] = (T)v;
      if (a.a64[mode] && c < a.R) a.a64[mode][i * a.R + c] = v;
    } else {
      const bool last = idx < a.seg[a.N + 1];
      const int q = last ? a.N - 1 : a.N - 2;
      const int64_t e = idx - (last ? a.seg[a.N] : a.seg[a.N + 1]);
      const int t = (int)(e & 3);
      const int lane = (int)((e >> 2) & 63);
      const int64_t rest = e >> 8;
      const int cb = (int)(rest % a.NBt);
      const int64_t chunk = rest / a.NBt;
      const int64_t row = 16 * chunk + 4 * (lane >> 4) + t;
      const int col = 16 * cb + (lane & 15);
      const double v = (row < a.s[q] && col < a.R) ? src_at<T>(a, q, row, col) : 0.0;
      ((T*)(last ? a.fpk_last : a.fpk_prev))[e] = (T)v;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------
static int grid_for(int64_t n, int block = 256, int cap = 8192) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int mttkrp_splits(const Plan& p, int mode, int* row_tiles, int* split_wgs, int* rows_per_tile) {
  const int MB = p.dtype == CP_F32 ? MttkrpCfg<float>::MB : MttkrpCfg<double>::MB;
  const int rpt = 16 * MB;
  const int64_t J = p.s[mode];
  const int64_t RT = (J + rpt - 1) / rpt;
  const int CG = (p.NBt + 7) / 8;
  const bool caseB = mode == p.N - 1;
  const int q = caseB ? p.N - 2 : p.N - 1;
  const int64_t QC = (p.s[q] + 15) / 16;
  const int64_t nitems = (p.total / J / p.s[q]) * QC;
  // aim for about two wavefronts per SIMD on 256 CUs, each with a handful of items
  int64_t sw = (2048 + 4 * RT * CG - 1) / (4 * RT * CG);
  const int64_t max_sw = (nitems + 7) / 8;
  if (sw > max_sw) sw = max_sw;
  if (sw > kRedSlots) sw = kRedSlots;
  if (sw < 1) sw = 1;
  *row_tiles = (int)RT;
  *split_wgs = (int)sw;
  *rows_per_tile = rpt;
  return 0;
}

template <typename T, bool CASE_B, bool VEC>
static void launch_nb(int NB, dim3 grid, hipStream_t st, const MttkrpArgs& a) {
  switch (NB) {
#define CPGN_NB(k) \
  case k: hipLaunchKernelGGL((k_mttkrp<T, CASE_B, k, VEC>), grid, dim3(256), 0, st, a); break;
    CPGN_NB(1) CPGN_NB(2) CPGN_NB(3) CPGN_NB(4) CPGN_NB(5) CPGN_NB(6) CPGN_NB(7) CPGN_NB(8)
#undef CPGN_NB
    default: break;
  }
}

template <typename T>
static int launch_mttkrp_t(const Plan& p, const void* X, int mode, char* ws, double* m64,
                           void* mout, hipStream_t st) {
  constexpr int MB = MttkrpCfg<T>::MB;
  int RT, SW, rpt;
  mttkrp_splits(p, mode, &RT, &SW, &rpt);
  const bool caseB = mode == p.N - 1;
  const int q = caseB ? p.N - 2 : p.N - 1;
  MttkrpArgs a{};
  a.X = X;
  int64_t off = 0;
  for (int m = 0; m < p.N; ++m) {
    a.apad[m] = ws + p.off_apad + off * p.esz;
    off += p.s[m] * p.Rp;
  }
  a.fpk = ws + (caseB ? p.off_fpk_prev : p.off_fpk_last);
  a.part = ws + p.off_part;
  a.J = p.s[mode];
  a.Jpad = (int64_t)RT * rpt;
  a.s_in = p.s[q];
  a.QC = (p.s[q] + 15) / 16;
  a.nitems = (p.total / a.J / a.s_in) * a.QC;
  a.Rr = 1;
  for (int m = mode + 1; m < p.N; ++m) a.Rr *= p.s[m];
  a.nbo = caseB ? 1 : a.Rr / a.s_in;
  a.n_outer = 0;
  for (int m = 0; m < p.N; ++m) {
    if (m == mode || m == q) continue;
    a.outer_mode[a.n_outer] = m;
    a.outer_size[a.n_outer] = p.s[m];
    ++a.n_outer;
  }
  a.Rp = p.Rp;
  a.NBt = p.NBt;
  a.nsplit = 4 * SW;
  const bool aligned = ((uintptr_t)X % 16) == 0;
  const bool vec = aligned && (caseB ? (a.J % MB == 0) : (a.s_in % 4 == 0));
  for (int cb0 = 0; cb0 < p.NBt; cb0 += 8) {
    const int NB = p.NBt - cb0 < 8 ? p.NBt - cb0 : 8;
    a.cb0 = cb0;
    dim3 grid(SW, RT);
    if (caseB) {
      if (vec) launch_nb<T, true, true>(NB, grid, st, a);
      else launch_nb<T, true, false>(NB, grid, st, a);
    } else {
      if (vec) launch_nb<T, false, true>(NB, grid, st, a);
      else launch_nb<T, false, false>(NB, grid, st, a);
    }
  }
  hipLaunchKernelGGL(k_mttkrp_reduce<T>, dim3(grid_for(a.J * p.R)), dim3(256), 0, st,
                     (const T*)a.part, SW, a.Jpad, p.Rp, a.J, p.R, m64, mout, p.dtype);
  return (int)hipGetLastError();
}

int launch_mttkrp(const Plan& p, const void* X, int mode, void* ws, double* m64, void* mout,
                  hipStream_t st) {
  if (p.dtype == CP_F32) return launch_mttkrp_t<float>(p, X, mode, (char*)ws, m64, mout, st);
  return launch_mttkrp_t<double>(p, X, mode, (char*)ws, m64, mout, st);
}

// Source factors may be the caller's buffers (compute precision) or FP64 copies.
int launch_prepare_factors_src(const Plan& p, const void* const* src, int src_dtype, void* wsv,
                               hipStream_t st, bool also_a64) {
  char* ws = (char*)wsv;
  PrepArgs a{};
  a.src_dtype = src_dtype;
  a.N = p.N;
  a.R = p.R;
  a.Rp = p.Rp;
  a.NBt = p.NBt;
  a.qc_last = p.qc_last;
  a.qc_prev = p.qc_prev;
  int64_t off = 0, a64off = 0;
  a.seg[0] = 0;
  for (int m = 0; m < p.N; ++m) {
    a.src[m] = src[m];
    a.s[m] = p.s[m];
    a.apad[m] = ws + p.off_apad + off * p.esz;
    a.a64[m] = also_a64 ? (double*)(ws + p.off_a64) + a64off : nullptr;
    off += p.s[m] * p.Rp;
    a64off += p.s[m] * p.R;
    a.seg[m + 1] = off;
  }
  a.fpk_last = ws + p.off_fpk_last;
  a.fpk_prev = ws + p.off_fpk_prev;
  a.seg[p.N + 1] = a.seg[p.N] + p.qc_last * p.NBt * 256;
  a.seg[p.N + 2] = a.seg[p.N + 1] + p.qc_prev * p.NBt * 256;
  const int grid = grid_for(a.seg[p.N + 2]);
  if (p.dtype == CP_F32) hipLaunchKernelGGL(k_prepare<float>, dim3(grid), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_prepare<double>, dim3(grid), dim3(256), 0, st, a);
  return (int)hipGetLastError();
}

int launch_prepare_factors(const Plan& p, const void* const* A, void* ws, hipStream_t st,
                           bool also_a64) {
  return launch_prepare_factors_src(p, A, p.dtype, ws, st, also_a64);
}

}  // namespace cpgn
