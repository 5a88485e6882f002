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
#include "batch.h"

namespace cpgn {


struct MttkrpArgs {
  const void* X;
  const void* apad[kMaxOrder];  // padded factors [s_m][Rp], compute precision
  const void* fpk;              // packed inner factor [QC][NBt][64 lanes][4]
  const void* wfac;             // padded factor of the output mode (dimension-tree weights)
  void* p1;                     // dimension-tree partials [RT][O][HS][Rp]
  void* part;                   // partial tiles [split_wgs][Jpad][Rp]
  int64_t J, Jpad, s_in, QC, nitems, Rr, nbo, O, HS;
  int64_t outer_size[kMaxOrder];
  int outer_mode[kMaxOrder];
  int n_outer;
  int Rp, NBt, cb0;
  int nsplit;                   // wavefronts along the contraction split (= 4 * gridDim.x)
  int dt;                       // also emit the outer mode's MTTKRP partials (order 3)
  int64_t rt0;                  // first row tile of this launch (grid y holds at most 65535)
};

template <typename T, int MB> struct VecLoad;
template <> struct VecLoad<float, 4> {
  typedef float v __attribute__((ext_vector_type(4)));
};
template <> struct VecLoad<double, 2> {
  typedef double v __attribute__((ext_vector_type(2)));
};


// X fragments of one item. Case A: one 4-vector per 16-row block (4 contraction substeps);
// case B: MB consecutive output rows per contraction substep.
template <typename T, bool CASE_B, int MB> struct XFrag;
template <typename T, int MB> struct XFrag<T, false, MB> {
  struct type { typename Mfma<T>::v4 v[MB]; };
  static __device__ __forceinline__ T get(const type& x, int mb, int t) { return x.v[mb][t]; }
};
template <typename T, int MB> struct XFrag<T, true, MB> {
  struct type { T v[4][MB]; };
  static __device__ __forceinline__ T get(const type& x, int mb, int t) { return x.v[t][mb]; }
};

template <bool CASE_B>
__device__ __forceinline__ int64_t outer_base(const MttkrpArgs& a, int64_t o) {
  if (CASE_B) return o * a.s_in * a.J;
  const int64_t aa = o / a.nbo, bo = o - aa * a.nbo;
  return aa * a.J * a.Rr + bo * a.s_in;
}

// Khatri-Rao row of the outer modes at outer index o, for this lane's columns.
template <typename T, int NB>
__device__ __forceinline__ void outer_row(const MttkrpArgs& a, int64_t o, int m, T (&kro)[NB]) {
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
}

template <typename T, int NB>
__device__ __forceinline__ void load_f(const typename Mfma<T>::v4* __restrict__ F,
                                       const MttkrpArgs& a, int64_t chunk, int lane,
                                       typename Mfma<T>::v4 (&f)[NB]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) f[nb] = F[(chunk * a.NBt + a.cb0 + nb) * kWave + lane];
}

// Branch-free loads (out-of-range lanes read a clamped in-bounds address and select 0), so
// the compiler can keep several items' loads in flight across the MFMA sequence.
template <typename T, bool CASE_B, int MB, bool VEC>
__device__ __forceinline__ void load_x(const T* __restrict__ X, const MttkrpArgs& a, int64_t base,
                                       int64_t chunk, int64_t j0, int g, int m,
                                       typename XFrag<T, CASE_B, MB>::type& x) {
  typedef typename Mfma<T>::v4 v4;
  const int64_t in0 = chunk * 16 + 4 * g;
  if constexpr (!CASE_B) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int64_t j = j0 + 16 * mb + m;
      if constexpr (VEC) {
        const bool ok = j < a.J && in0 < a.s_in;
        const v4 w = *(const v4*)(X + (ok ? base + j * a.Rr + in0 : 0));
#pragma unroll
        for (int t = 0; t < 4; ++t) x.v[mb][t] = ok ? w[t] : T(0);
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bool ok = j < a.J && in0 + t < a.s_in;
          const T w = X[ok ? base + j * a.Rr + in0 + t : 0];
          x.v[mb][t] = ok ? w : T(0);
        }
      }
    }
  } else {
    const int64_t jb = j0 + MB * m;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t inn = in0 + t;
      if constexpr (VEC) {
        typedef typename VecLoad<T, MB>::v vv;
        const bool ok = inn < a.s_in && jb < a.J;
        const vv w = *(const vv*)(X + (ok ? base + inn * a.J + jb : 0));
#pragma unroll
        for (int v = 0; v < MB; ++v) x.v[t][v] = ok ? w[v] : T(0);
      } else {
#pragma unroll
        for (int v = 0; v < MB; ++v) {
          const bool ok = inn < a.s_in && jb + v < a.J;
          const T w = X[ok ? base + inn * a.J + jb + v : 0];
          x.v[t][v] = ok ? w : T(0);
        }
      }
    }
  }
}

// Loads of one item: packed inner factor and X fragment.
template <typename T, bool CASE_B, int MB, int NB> struct ItemBuf {
  typename Mfma<T>::v4 f[NB];
  typename XFrag<T, CASE_B, MB>::type x;
};

// Split index (within a row tile) of the wavefront that owns item t: largest w with
// floor(nitems * w / S) <= t.
__host__ __device__ __forceinline__ int64_t owner_split(int64_t t, int64_t nitems, int64_t S) {
  return ((t + 1) * S - 1) / nitems;
}

template <typename T, bool CASE_B, int MB, int NB, bool VEC, bool DT>
__device__ __forceinline__ void mttkrp_body(const MttkrpArgs& a, dim3 bid) {
  // FP64 with many column blocks keeps a single F buffer (registers); F is L2-resident.
  constexpr bool PF = sizeof(T) == 4 || NB <= 4;
  typedef typename Mfma<T>::v4 v4;
  typedef ItemBuf<T, CASE_B, MB, NB> Buf;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, m = lane & 15;
  const int split = bid.x * 4 + wave;
  const int64_t rt = a.rt0 + bid.y;
  const int64_t j0 = rt * 16 * MB;
  const int64_t it0 = a.nitems * split / a.nsplit;
  const int64_t it1 = a.nitems * (split + 1) / a.nsplit;
  const T* __restrict__ X = (const T*)a.X;
  const v4* __restrict__ F = (const v4*)a.fpk;

  // acc: this wavefront's share of M(n).
  // Plain form: the B operand is the packed inner factor times the outer Khatri-Rao row kro of
  //   the current outer index (kept in registers, refreshed when the index changes).
  // Dimension-tree form (DT): tacc accumulates T = X x_q A(q) for one outer index o; when o
  //   changes it is folded into acc with kro and, weighted by A(n), summed over the rows into
  //   the outer mode's partial M(o).
  v4 acc[MB][NB];
  v4 tacc[DT ? MB : 1][DT ? NB : 1];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[i][nb] = v4{0, 0, 0, 0};
  if constexpr (DT) {
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) tacc[i][nb] = v4{0, 0, 0, 0};
  }
  T kro[NB];

  // Two item buffers in ping-pong: the loads of the next item are in flight while the MFMAs of
  // the current one run, and no register copy forces them to complete early.
  auto issue = [&](Buf& b, int64_t chunk, int64_t base) {
    if constexpr (PF) load_f<T, NB>(F, a, chunk, lane, b.f);
    load_x<T, CASE_B, MB, VEC>(X, a, base, chunk, j0, g, m, b.x);
  };
  auto consume = [&](Buf& b, int64_t chunk) {
    if constexpr (!PF) load_f<T, NB>(F, a, chunk, lane, b.f);
    // B operands of all four substeps are formed before the first product, so no multiply
    // waits on (or stalls) the matrix instructions reading the previous substep's operands.
    T bt4[4][NB];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bt4[t][nb] = DT ? b.f[nb][t] : b.f[nb][t] * kro[nb];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T* bt = bt4[t];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const T x = XFrag<T, CASE_B, MB>::get(b.x, mb, t);
          if constexpr (DT) tacc[mb][nb] = Mfma<T>::mac(x, bt[nb], tacc[mb][nb]);
          else acc[mb][nb] = Mfma<T>::mac(x, bt[nb], acc[mb][nb]);
        }
    }
  };
  // Output row held by element v of block mb in this lane.
  auto row_of = [&](int mb, int v) -> int64_t {
    const int i = Mfma<T>::out_row(lane, v);
    return CASE_B ? j0 + (int64_t)MB * i + mb : j0 + 16 * mb + i;
  };
  // DT: fold tacc of outer index o into acc and into the outer mode's partial.
  auto flush = [&](int64_t o) {
    if constexpr (DT) {
      const T* W = (const T*)a.wfac + 16 * a.cb0 + m;
      const int64_t h = split - owner_split(o * a.QC, a.nitems, a.nsplit);
      T* P1 = (T*)a.p1 + (((rt * a.O + o) * a.HS + h) * a.Rp) + 16 * a.cb0 + m;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        T sum = T(0);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t row = row_of(mb, v);
            const T w = W[(row < a.J ? row : 0) * a.Rp + 16 * nb];
            const T tv = tacc[mb][nb][v];
            sum += tv * (row < a.J ? w : T(0));
            acc[mb][nb][v] += tv * kro[nb];
          }
        sum += __shfl_xor(sum, 16);
        sum += __shfl_xor(sum, 32);
        if (g == 0) P1[16 * nb] = sum;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) tacc[mb][nb] = v4{0, 0, 0, 0};
      }
    }
  };

  // Item position (outer index o, inner chunk, X offset of (o, chunk 0)), advanced without
  // divisions so that the loop body has no branches besides its own back-edge and the rare,
  // uniform flush.
  struct Pos {
    int64_t o, chunk, bo, base;
  };
  auto advance = [&](Pos q) {
    q.chunk += 1;
    const bool wrap = q.chunk == a.QC;
    q.chunk = wrap ? 0 : q.chunk;
    q.o += wrap ? 1 : 0;
    if constexpr (CASE_B) {
      q.base += wrap ? a.s_in * a.J : 0;
    } else {
      q.bo += wrap ? 1 : 0;
      q.base += wrap ? a.s_in : 0;
      const bool carry = q.bo == a.nbo;
      q.bo = carry ? 0 : q.bo;
      q.base += carry ? (a.J - 1) * a.Rr : 0;
    }
    return q;
  };

  Buf b0, b1;
  Pos p0{0, 0, 0, 0};
  if (it0 < it1) {
    p0.o = it0 / a.QC;
    p0.chunk = it0 - p0.o * a.QC;
    if constexpr (CASE_B) {
      p0.base = p0.o * a.s_in * a.J;
    } else {
      const int64_t aa = p0.o / a.nbo;
      p0.bo = p0.o - aa * a.nbo;
      p0.base = aa * a.J * a.Rr + p0.bo * a.s_in;
    }
    outer_row<T, NB>(a, p0.o, m, kro);
    issue(b0, p0.chunk, p0.base);
  }
  // The item after the last one is replaced by the last one (a harmless re-load), so every
  // iteration issues the same loads; the outer-index change is a rare, uniform branch.
  for (int64_t it = it0; it < it1; it += 2) {
    Pos p1 = advance(p0);
    const bool last0 = it + 1 >= it1;
    if (last0) p1 = p0;
    issue(b1, p1.chunk, p1.base);
    consume(b0, p0.chunk);
    if (last0 || p1.o != p0.o) {
      flush(p0.o);
      if (!last0) outer_row<T, NB>(a, p1.o, m, kro);
    }
    if (last0) break;
    Pos p2 = advance(p1);
    const bool last1 = it + 2 >= it1;
    if (last1) p2 = p1;
    issue(b0, p2.chunk, p2.base);
    consume(b1, p1.chunk);
    if (last1 || p2.o != p1.o) {
      flush(p1.o);
      if (!last1) outer_row<T, NB>(a, p2.o, m, kro);
    }
    p0 = p2;
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
    T* P = (T*)a.part + (int64_t)bid.x * a.Jpad * a.Rp;
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

// Plain form: one accumulator set, two wavefronts per SIMD. Dimension-tree form: two
// accumulator sets, on 32-row tiles in FP32 and 16-row tiles in FP64 (whose accumulators take
// twice the registers), also two wavefronts per SIMD.
template <typename T, bool CASE_B, int MB, int NB, bool VEC>
__global__ __launch_bounds__(256, 2) void k_mttkrp(MttkrpArgs a) {
  mttkrp_body<T, CASE_B, MB, NB, VEC, false>(a, CPGN_BID);
}

template <typename T, int MB, int NB>
__global__ __launch_bounds__(256, 2) void k_mttkrp_tree(MttkrpArgs a) {
  mttkrp_body<T, false, MB, NB, true, true>(a, CPGN_BID);
}

template <typename T, bool CASE_B, int MB, int NB, bool VEC>
struct KMttkrp {
  using Args = MttkrpArgs;
  static constexpr int kThreads = 256, kMinBlocks = 2;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3) {
    mttkrp_body<T, CASE_B, MB, NB, VEC, false>(a, bid);
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
    hipLaunchKernelGGL((k_mttkrp<T, CASE_B, MB, NB, VEC>), grid, dim3(kThreads), lds, s, a);
  }
};

template <typename T, int MB, int NB>
struct KMttkrpTree {
  using Args = MttkrpArgs;
  static constexpr int kThreads = 256, kMinBlocks = 2;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3) {
    mttkrp_body<T, false, MB, NB, true, true>(a, bid);
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
    hipLaunchKernelGGL((k_mttkrp_tree<T, MB, NB>), grid, dim3(kThreads), lds, s, a);
  }
};

// M[j, r] = sum over partial tiles, in FP64, in a fixed order. A workgroup of 16 wavefronts owns
// 64 consecutive outputs (flattened over j, r < R; one coalesced load per tile and wavefront);
// wavefront w adds the tiles p = w, w + 16, w + 32, ... in order, and the 16 wavefront sums are
// added in a fixed tree. Writes the FP64 result and/or a copy in the caller's precision.
constexpr int kRedWaves = 16;

template <typename T>
__device__ __forceinline__ void mttkrp_reduce_body(const T* __restrict__ part, int nparts,
                                                   int64_t Jpad, int Rp, int64_t J, int R,
                                                   double* __restrict__ m64, void* mout,
                                                   int mout_dtype, dim3 bid) {
  __shared__ double sh[kRedWaves][kWave];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = J * R;
  const int64_t idx = (int64_t)bid.x * kWave + lane;
  const bool ok = idx < n;
  const int64_t j = ok ? idx / R : 0;
  const int r = ok ? (int)(idx - j * R) : 0;
  const T* p = part + j * Rp + r;
  const int64_t stride = Jpad * Rp;
  double s = 0.0;
#pragma unroll 8
  for (int k = w; k < nparts; k += kRedWaves) s += (double)p[(int64_t)k * stride];
  sh[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    double t[kRedWaves];
#pragma unroll
    for (int i = 0; i < kRedWaves; ++i) t[i] = sh[i][lane];
#pragma unroll
    for (int h = kRedWaves / 2; h >= 1; h /= 2)
#pragma unroll
      for (int i = 0; i < h; ++i) t[i] += t[i + h];
    if (ok) {
      if (m64) m64[idx] = t[0];
      if (mout) {
        if (mout_dtype == CP_F64) ((double*)mout)[idx] = t[0];
        else ((float*)mout)[idx] = (float)t[0];
      }
    }
  }
}

template <typename T>
struct KMttReduce {
  struct Args {
    const T* part;
    int nparts;
    int64_t Jpad;
    int Rp;
    int64_t J;
    int R;
    double* m64;
    void* mout;
    int mout_dtype;
  };
  static constexpr int kThreads = 1024, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3) {
    mttkrp_reduce_body<T>(a.part, a.nparts, a.Jpad, a.Rp, a.J, a.R, a.m64, a.mout, a.mout_dtype,
                          bid);
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

template <typename T>
__global__ __launch_bounds__(1024) void k_mttkrp_reduce(typename KMttReduce<T>::Args a) {
  KMttReduce<T>::run(a, CPGN_BID, CPGN_GDIM);
}

template <typename T>
void KMttReduce<T>::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_mttkrp_reduce<T>, grid, dim3(kThreads), lds, s, a);
}

static unsigned reduce_grid(int64_t J, int R) { return (unsigned)((J * R + kWave - 1) / kWave); }

// Padded factor copies [s_m][Rp] in the compute precision, optional FP64 copies [s_m][R], and
// the packed B-operand layout of modes N-1 and N-2:
//   fpk[chunk][cb][lane][t] = A(q)[16*chunk + 4*(lane/16) + t][16*cb + lane%16]  (0 outside).
// For a bfloat16 tensor (xk != 0) the packs hold FP32 values in chunks of 32 rows, 8 per lane,
// A(q)[32*chunk + 8*(lane/16) + t][16*cb + lane%16], and each mode's outer Khatri-Rao rows
// krp_n[o][r] = prod over outer modes m of A(m)[i_m(o)][r] are written in FP32 (outer modes: all
// but n and its inner mode, ascending, the last one fastest).
struct PrepArgs {
  const void* src[kMaxOrder];
  int src_dtype;
  void* apad[kMaxOrder];
  double* a64[kMaxOrder];
  void* fpk_last;
  void* fpk_prev;
  float* krp;
  int64_t s[kMaxOrder];
  int64_t seg[kMaxOrder + 4];   // cumulative segment starts: modes' apad, the two packs, tables
  int64_t krp_seg[kMaxOrder + 1];   // table elements enumerated per mode (0 for skipped modes)
  int64_t krp_dst[kMaxOrder];       // element offset of each mode's table
  int small32;                      // every outer index and mode size fits in 32 bits
  int N, R, Rp, NBt, xk;
  int64_t qc_last, qc_prev;
  int64_t fplane_last, fplane_prev;   // FP32 elements of each pack (bfloat16 tensor forms)
};

template <typename T>
__device__ __forceinline__ double src_at(const PrepArgs& a, int mode, int64_t i, int r) {
  return a.src_dtype == CP_F64 ? ((const double*)a.src[mode])[i * a.R + r]
                               : (double)((const float*)a.src[mode])[i * a.R + r];
}

// I: index type of the element arithmetic (32-bit when every index fits, which makes the
// divisions by Rp and NBt several times cheaper; same values either way).
template <typename T, typename I>
__device__ __forceinline__ void prepare_impl(const PrepArgs& a, dim3 bid, dim3 gdim) {
  const int64_t total = a.seg[a.N + 3];
  for (int64_t idx = bid.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gdim.x * blockDim.x) {
    if (idx < a.seg[a.N]) {
      int mode = 0;
      while (idx >= a.seg[mode + 1]) ++mode;
      const int64_t e = idx - a.seg[mode];
      const int64_t i = (int64_t)((I)e / (I)a.Rp);
      const int c = (int)(e - i * a.Rp);
      const double v = c < a.R ? src_at<T>(a, mode, i, c) : 0.0;
      ((T*)a.apad[mode])[e] = (T)v;
      if (a.a64[mode] && c < a.R) a.a64[mode][i * a.R + c] = v;
    } else if (idx < a.seg[a.N + 2]) {
      const bool last = idx < a.seg[a.N + 1];
      const int q = last ? a.N - 1 : a.N - 2;
      const int64_t e = idx - (last ? a.seg[a.N] : a.seg[a.N + 1]);
      if (a.xk == 0) {
        const int t = (int)(e & 3);
        const int lane = (int)((e >> 2) & 63);
        const int64_t rest = e >> 8;
        const int64_t chunk = (int64_t)((I)rest / (I)a.NBt);
        const int cb = (int)(rest - chunk * a.NBt);
        const int64_t row = 16 * chunk + 4 * (lane >> 4) + t;
        const int col = 16 * cb + (lane & 15);
        const double v = (row < a.s[q] && col < a.R) ? src_at<T>(a, q, row, col) : 0.0;
        ((T*)(last ? a.fpk_last : a.fpk_prev))[e] = (T)v;
      } else {
        const int t = (int)(e & 7);
        const int lane = (int)((e >> 3) & 63);
        const int64_t rest = e >> 9;
        const int64_t chunk = (int64_t)((I)rest / (I)a.NBt);
        const int cb = (int)(rest - chunk * a.NBt);
        const int64_t row = 32 * chunk + 8 * (lane >> 4) + t;
        const int col = 16 * cb + (lane & 15);
        const float v = (row < a.s[q] && col < a.R) ? (float)src_at<T>(a, q, row, col) : 0.0f;
        ((float*)(last ? a.fpk_last : a.fpk_prev))[e] = v;
      }
    } else {
      const int64_t e0 = idx - a.seg[a.N + 2];
      int n = 0;
      while (e0 >= a.krp_seg[n + 1]) ++n;
      const int64_t e = e0 - a.krp_seg[n];
      const int q = n == a.N - 1 ? a.N - 2 : a.N - 1;
      const int64_t o = (int64_t)((I)e / (I)a.Rp);
      const int c = (int)(e - o * a.Rp);
      double v = c < a.R ? 1.0 : 0.0;
      if (a.small32) {
        uint32_t rem = (uint32_t)o;
        for (int m = a.N - 1; m >= 0 && c < a.R; --m) {
          if (m == n || m == q) continue;
          const uint32_t sm = (uint32_t)a.s[m];
          const uint32_t im = rem % sm;
          rem /= sm;
          v *= (double)(float)src_at<T>(a, m, im, c);
        }
      } else {
        int64_t rem = o;
        for (int m = a.N - 1; m >= 0 && c < a.R; --m) {
          if (m == n || m == q) continue;
          const int64_t im = rem % a.s[m];
          rem /= a.s[m];
          v *= (double)(float)src_at<T>(a, m, im, c);
        }
      }
      a.krp[a.krp_dst[n] + e] = (float)v;
    }
  }
}

template <typename T>
__device__ __forceinline__ void prepare_body(const PrepArgs& a, dim3 bid, dim3 gdim) {
  if (a.seg[a.N + 3] < ((int64_t)1 << 31)) prepare_impl<T, uint32_t>(a, bid, gdim);
  else prepare_impl<T, int64_t>(a, bid, gdim);
}

template <typename T>
struct KPrepare {
  using Args = PrepArgs;
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3 gdim) {
    prepare_body<T>(a, bid, gdim);
  }
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

template <typename T>
__global__ __launch_bounds__(256) void k_prepare(PrepArgs a) {
  prepare_body<T>(a, CPGN_BID, CPGN_GDIM);
}

template <typename T>
void KPrepare<T>::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_prepare<T>, grid, dim3(kThreads), lds, s, a);
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

MttkrpGeom mttkrp_geom(const Plan& p, int mode, bool vec_ok, bool dt) {
  MttkrpGeom g{};
  const bool caseB = mode == p.N - 1;
  const int q = caseB ? p.N - 2 : p.N - 1;
  const int64_t J = p.s[mode];
  g.MB = dt ? (p.dtype == CP_F64 ? 1 : 2) : (p.dtype == CP_F64 ? 2 : 4);
  // FP32, contraction along X rows: 80-row tiles where they pad the mode less than 64-row ones
  // (s = 400: 5 tiles and no padding rows, against 7 tiles of which 48 rows are padding), or
  // the tile the plan's tuning names (32, 64 or 80 rows)
  if (!dt && p.dtype == CP_F32 && !caseB && vec_ok && p.xk == 0) {
    if (p.mt_row_block != 0) g.MB = p.mt_row_block;
    else if ((J + 79) / 80 * 80 < (J + 63) / 64 * 64) g.MB = 5;
  }
  g.rows_per_tile = 16 * g.MB;
  g.RT = (J + g.rows_per_tile - 1) / g.rows_per_tile;
  g.QC = (p.s[q] + 15) / 16;
  g.O = p.total / J / p.s[q];
  g.nitems = g.O * g.QC;
  // One resident round of 4-wave workgroups: two per CU (<= 256 registers per lane), but at
  // least 16 items per wavefront: with fewer, the first loads of a workgroup, its reduction
  // through LDS and its partial tile cost more than its products (small modes; many such
  // problems then share launches in a batch program). Both figures come from the plan's tuning.
  const int64_t wgs = (int64_t)kNumCU * p.mt_wg_per_cu;
  int64_t sw = wgs / g.RT;
  const int64_t per_wg = 4 * (int64_t)p.mt_min_items;
  const int64_t max_sw = (g.nitems + per_wg - 1) / per_wg;
  if (sw > max_sw) sw = max_sw;
  if (sw > kRedSlots) sw = kRedSlots;
  if (sw < 1) sw = 1;
  g.SW = sw;
  const int64_t S = 4 * sw;
  g.HS = (g.QC * S + g.nitems - 1) / g.nitems + 1;
  return g;
}

template <typename T, bool CASE_B, int MB, bool VEC>
static void launch_nb(int NB, dim3 grid, hipStream_t st, const MttkrpArgs& a) {
  switch (NB) {
#define CPGN_NB(k)                                                                         \
  case k:                                                                                  \
    dispatch<KMttkrp<T, CASE_B, MB, k, VEC>>(grid, 0, st, a);                          \
    break;
    CPGN_NB(1) CPGN_NB(2) CPGN_NB(3) CPGN_NB(4) CPGN_NB(5) CPGN_NB(6) CPGN_NB(7) CPGN_NB(8)
#undef CPGN_NB
    default: break;
  }
}

template <typename T, int MB>
static void launch_tree_nb(int NB, dim3 grid, hipStream_t st, const MttkrpArgs& a) {
  switch (NB) {
#define CPGN_NB(k)                                                                      \
  case k: dispatch<KMttkrpTree<T, MB, k>>(grid, 0, st, a); break;
    CPGN_NB(1) CPGN_NB(2) CPGN_NB(3) CPGN_NB(4) CPGN_NB(5) CPGN_NB(6) CPGN_NB(7) CPGN_NB(8)
#undef CPGN_NB
    default: break;
  }
}

template <typename T>
static void launch_variant(bool caseB, bool vec, int MB, int NB, dim3 grid, hipStream_t st,
                           const MttkrpArgs& a) {
  if (a.dt) {   // order-3 dimension tree: mode 0 with vector loads only
    launch_tree_nb<T, sizeof(T) == 8 ? 1 : 2>(NB, grid, st, a);
    return;
  }
  if constexpr (sizeof(T) == 8) {
    if (caseB) {
      if (vec) launch_nb<T, true, 2, true>(NB, grid, st, a);
      else launch_nb<T, true, 2, false>(NB, grid, st, a);
    } else {
      if (vec) launch_nb<T, false, 2, true>(NB, grid, st, a);
      else launch_nb<T, false, 2, false>(NB, grid, st, a);
    }
  } else {
    if (caseB) {
      if (vec) launch_nb<T, true, 4, true>(NB, grid, st, a);
      else launch_nb<T, true, 4, false>(NB, grid, st, a);
    } else if (!vec) {
      launch_nb<T, false, 4, false>(NB, grid, st, a);
    } else if (MB == 5) {
      launch_nb<T, false, 5, true>(NB, grid, st, a);
    } else if (MB == 2) {
      launch_nb<T, false, 2, true>(NB, grid, st, a);
    } else {
      launch_nb<T, false, 4, true>(NB, grid, st, a);
    }
  }
}

// M(o)[o][r] = sum over row tiles and over the wavefronts that shared o (fixed order).
template <typename T>
struct KDtReduce {
  struct Args {
    const T* p1;
    int64_t RT, O, HS;
    int Rp, R;
    int64_t QC, nitems, S;
    double* m64;
    void* mout;
    int mout_dtype;
  };
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3 gdim);
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

template <typename T>
__device__ __forceinline__ void KDtReduce<T>::run(const Args& a, dim3 bid, dim3 gdim) {
  const T* __restrict__ p1 = a.p1;
  const int64_t RT = a.RT, O = a.O, HS = a.HS, QC = a.QC, nitems = a.nitems, S = a.S;
  const int Rp = a.Rp, R = a.R;
  double* __restrict__ m64 = a.m64;
  void* mout = a.mout;
  const int mout_dtype = a.mout_dtype;
  const int64_t n = O * R;
  for (int64_t idx = bid.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gdim.x * blockDim.x) {
    const int64_t o = idx / R;
    const int r = (int)(idx - o * R);
    const int64_t w0 = owner_split(o * QC, nitems, S);
    const int64_t h_n = owner_split((o + 1) * QC - 1, nitems, S) - w0 + 1;
    // Terms k = rt h_n + h in order; each batch of 8 is loaded before it is added, so the loads
    // of a batch are in flight together (same sum, same order as one term at a time). Slot h
    // belongs to split w0 + h. Only with more splits than items can a split between two owners
    // of o be empty; it never writes its slot, so such terms are skipped (uniform test).
    const int64_t K = RT * h_n;
    const bool may_be_empty = S > nitems;
    double s = 0.0;
    for (int64_t k0 = 0; k0 < K; k0 += 8) {
      T v[8];
      bool use[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        // K = row tiles x slots < 2^31 (both index the partial buffer): 32-bit division
        const int k = (int)(k0 + u < K ? k0 + u : K - 1);
        const int rt = k / (int)h_n, h = k - rt * (int)h_n;
        use[u] = k0 + u < K;
        if (may_be_empty) {
          const int64_t w = w0 + h;
          use[u] = use[u] && nitems * w / S < nitems * (w + 1) / S;
        }
        v[u] = p1[(((int64_t)rt * O + o) * HS + h) * Rp + r];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (use[u]) s += (double)v[u];
    }
    if (m64) m64[idx] = s;
    if (mout) {
      if (mout_dtype == CP_F64) ((double*)mout)[idx] = s;
      else ((float*)mout)[idx] = (float)s;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dt_reduce(typename KDtReduce<T>::Args a) {
  KDtReduce<T>::run(a, CPGN_BID, CPGN_GDIM);
}

template <typename T>
void KDtReduce<T>::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_dt_reduce<T>, grid, dim3(kThreads), lds, s, a);
}

static bool vec_ok(const Plan& p, int mode, const void* X) {
  const bool caseB = mode == p.N - 1;
  const int q = caseB ? p.N - 2 : p.N - 1;
  const int vw = p.dtype == CP_F64 ? 2 : 4;
  return ((uintptr_t)X % 16) == 0 && (caseB ? (p.s[mode] % vw == 0) : (p.s[q] % 4 == 0));
}

template <typename T>
static int launch_mttkrp_t(const Plan& p, const void* X, int mode, char* ws, double* m64,
                           void* mout, bool dt, double* m64_outer, void* mout_outer,
                           hipStream_t st, KernelMarks mk = {}) {
  const bool vec = vec_ok(p, mode, X);
  const MttkrpGeom G = mttkrp_geom(p, mode, vec, dt);
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
  a.wfac = a.apad[mode];
  a.p1 = ws + p.off_p1;
  a.J = p.s[mode];
  a.Jpad = G.RT * G.rows_per_tile;
  a.s_in = p.s[q];
  a.QC = G.QC;
  a.nitems = G.nitems;
  a.O = G.O;
  a.HS = G.HS;
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
  a.nsplit = (int)(4 * G.SW);
  a.dt = dt ? 1 : 0;
  if (mk.before) {
    const hipError_t e = hipEventRecord(mk.before, st);
    if (e != hipSuccess) return (int)e;
  }
  for (int cb0 = 0; cb0 < p.NBt; cb0 += 8) {
    const int NB = p.NBt - cb0 < 8 ? p.NBt - cb0 : 8;
    a.cb0 = cb0;
    for (int64_t rt0 = 0; rt0 < G.RT; rt0 += kMaxGridY) {   // row tiles in chunks of grid y
      a.rt0 = rt0;
      const int64_t nrt = G.RT - rt0 < kMaxGridY ? G.RT - rt0 : kMaxGridY;
      launch_variant<T>(caseB, vec, G.MB, NB, dim3((unsigned)G.SW, (unsigned)nrt), st, a);
    }
  }
  if (mk.after) {
    const hipError_t e = hipEventRecord(mk.after, st);
    if (e != hipSuccess) return (int)e;
  }
  dispatch<KMttReduce<T>>(dim3(reduce_grid(a.J, p.R)), 0, st,
                          {(const T*)a.part, (int)G.SW, a.Jpad, p.Rp, a.J, p.R, m64, mout, p.dtype});
  if (dt)
    dispatch<KDtReduce<T>>(dim3(grid_for(G.O * p.R)), 0, st,
                           {(const T*)a.p1, G.RT, G.O, G.HS, p.Rp, p.R, G.QC, G.nitems,
                            (int64_t)a.nsplit, m64_outer, mout_outer, p.dtype});
  return (int)hipGetLastError();
}

void launch_mttkrp_reduce_f32(const float* part, int nparts, int64_t Jpad, int Rp, int64_t J,
                              int R, double* m64, void* mout, int mout_dtype, hipStream_t st) {
  dispatch<KMttReduce<float>>(dim3(reduce_grid(J, R)), 0, st,
                              {part, nparts, Jpad, Rp, J, R, m64, mout, mout_dtype});
}

int launch_mttkrp_bf16(const Plan& p, const void* X, int mode, void* ws, double* m64, void* mout,
                       hipStream_t st, KernelMarks mk);

// Order 3: T = X x_3 A(2) as the [s0 s1][Rp] matrix (compute precision), for the ALS dimension
// tree. It is the mode-0 MTTKRP of X viewed as the two-way tensor [s0 s1, s2]: one workgroup per
// row tile sums all inner chunks, so each tile of T is written once and no reduction follows.
template <typename T>
static int launch_ttm_last_t(const Plan& p, const void* X, char* ws, void* Tout, hipStream_t st) {
  const int MB = p.dtype == CP_F64 ? 2 : 4;
  const int64_t J = p.s[0] * p.s[1], s_in = p.s[2];
  const bool vec = ((uintptr_t)X % 16) == 0 && s_in % 4 == 0;
  MttkrpArgs a{};
  a.X = X;
  a.fpk = ws + p.off_fpk_last;
  a.part = Tout;
  a.J = J;
  a.s_in = s_in;
  a.QC = (s_in + 15) / 16;
  a.nitems = a.QC;
  a.O = 1;
  a.Rr = s_in;
  a.nbo = 1;
  a.n_outer = 0;
  a.Rp = p.Rp;
  a.NBt = p.NBt;
  a.nsplit = 4;
  a.dt = 0;
  const int64_t RT = (J + 16 * MB - 1) / (16 * MB);
  a.Jpad = RT * 16 * MB;
  for (int cb0 = 0; cb0 < p.NBt; cb0 += 8) {
    const int NB = p.NBt - cb0 < 8 ? p.NBt - cb0 : 8;
    a.cb0 = cb0;
    launch_variant<T>(false, vec, MB, NB, dim3(1, (unsigned)RT), st, a);
  }
  return (int)hipGetLastError();
}

// Rows of T padded to whole tiles (the T buffer holds ttm_rows(p) x Rp elements).
int64_t ttm_rows(const Plan& p) {
  const int64_t rows = 16 * (p.dtype == CP_F64 ? 2 : 4);
  return (p.s[0] * p.s[1] + rows - 1) / rows * rows;
}

int launch_ttm_last(const Plan& p, const void* X, void* ws, void* T, hipStream_t st) {
  if (p.dtype == CP_F32) return launch_ttm_last_t<float>(p, X, (char*)ws, T, st);
  return launch_ttm_last_t<double>(p, X, (char*)ws, T, st);
}

// M(n) for n = 0 or 1 from T = X x_3 A(2): M(0)[i0][r] = sum_i1 T[i0 s1 + i1][r] F[i1][r],
// M(1)[i1][r] = sum_i0 T[i0 s1 + i1][r] F[i0][r], F the other mode's FP64 factor. One workgroup
// per output row: lane r of group g adds the terms b = g, g + 8, ... in order in FP64 (each
// step a coalesced read of one T row segment), and the 8 group sums are added in a fixed tree.
constexpr int kTtmGroups = 8;

template <typename T>
__global__ __launch_bounds__(1024) void k_ttm_contract(const T* __restrict__ Tm,
                                                       const double* __restrict__ F,
                                                       int64_t n_loop, int64_t stride_out,
                                                       int64_t stride_loop, int R,
                                                       double* __restrict__ out) {
  __shared__ double part[kTtmGroups][128];
  const int r = threadIdx.x & 127, g = threadIdx.x >> 7;
  const int64_t i = blockIdx.x;
  double acc = 0.0;
  if (r < R) {
    const T* base = Tm + i * stride_out + r;
#pragma unroll 4
    for (int64_t b = g; b < n_loop; b += kTtmGroups)
      acc = fma((double)base[b * stride_loop], F[b * R + r], acc);
  }
  part[g][r] = acc;
  __syncthreads();
  if (g == 0 && r < R) {
    double t[kTtmGroups];
#pragma unroll
    for (int q = 0; q < kTtmGroups; ++q) t[q] = part[q][r];
#pragma unroll
    for (int h = kTtmGroups / 2; h >= 1; h /= 2)
#pragma unroll
      for (int q = 0; q < h; ++q) t[q] += t[q + h];
    out[i * R + r] = t[0];
  }
}

// R <= 128 (the rank limit of the ALS sweep).
void launch_ttm_contract(const Plan& p, const void* T, const double* F, int mode, double* out,
                         hipStream_t st) {
  const int64_t s1Rp = p.s[1] * p.Rp;
  const int64_t n_out = mode == 0 ? p.s[0] : p.s[1];
  const int64_t n_loop = mode == 0 ? p.s[1] : p.s[0];
  const int64_t so = mode == 0 ? s1Rp : p.Rp, sl = mode == 0 ? p.Rp : s1Rp;
  if (p.dtype == CP_F32)
    hipLaunchKernelGGL(k_ttm_contract<float>, dim3((unsigned)n_out), dim3(1024), 0, st,
                       (const float*)T, F, n_loop, so, sl, p.R, out);
  else
    hipLaunchKernelGGL(k_ttm_contract<double>, dim3((unsigned)n_out), dim3(1024), 0, st,
                       (const double*)T, F, n_loop, so, sl, p.R, out);
}

int launch_mttkrp(const Plan& p, const void* X, int mode, void* ws, double* m64, void* mout,
                  hipStream_t st, KernelMarks mk) {
  if (p.xk != 0) return launch_mttkrp_bf16(p, X, mode, ws, m64, mout, st, mk);
  if (p.dtype == CP_F32)
    return launch_mttkrp_t<float>(p, X, mode, (char*)ws, m64, mout, false, nullptr, nullptr, st,
                                  mk);
  return launch_mttkrp_t<double>(p, X, mode, (char*)ws, m64, mout, false, nullptr, nullptr, st,
                                 mk);
}

// Order >= 4 dimension tree, second half: the tree pass leaves, for every outer index o =
// (i_1, ..., i_{N-2}) (row-major), Pm[o][r] = sum over i_0, i_{N-1} of X A(0) A(N-1) in FP64.
// Outer mode m's MTTKRP is then M(m)[i, r] = sum over the o with o_m = i of Pm[o][r] times the
// other outer factors' entries: one thread per output element, terms in increasing o.
struct KOuterContract {
  struct Args {
    const double* pm;                 // [O][R]
    int64_t O;
    int R, Rp, n_outer, dtype;        // dtype of apad and of mout
    int64_t size[kMaxOrder];          // outer sizes s_1 .. s_{N-2}
    int64_t first[kMaxOrder + 1];     // output elements before outer mode d (prefix of s_d R)
    const void* apad[kMaxOrder];      // padded factors of the outer modes [s][Rp]
    double* m64[kMaxOrder];           // FP64 outputs [s][R] (may be null)
    void* mout[kMaxOrder];            // compute-precision outputs [s][R] (may be null)
  };
  static constexpr int kThreads = 256, kMinBlocks = 1;
  static __device__ __forceinline__ void run(const Args& a, dim3 bid, dim3 gdim);
  static void direct(dim3 grid, size_t lds, hipStream_t s, const Args& a);
};

__device__ __forceinline__ void KOuterContract::run(const Args& a, dim3 bid, dim3 gdim) {
  const int64_t total = a.first[a.n_outer];
  for (int64_t idx = bid.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gdim.x * blockDim.x) {
    int d = 0;
    while (idx >= a.first[d + 1]) ++d;
    const int64_t e = idx - a.first[d];
    const int64_t i = e / a.R;
    const int r = (int)(e - i * a.R);
    int64_t stride = 1;   // distance between consecutive i_d in o
    for (int k = a.n_outer - 1; k > d; --k) stride *= a.size[k];
    const int64_t outer = a.O / (a.size[d] * stride);
    double s = 0.0;
    for (int64_t hi = 0; hi < outer; ++hi)
      for (int64_t lo = 0; lo < stride; ++lo) {
        const int64_t o = (hi * a.size[d] + i) * stride + lo;
        double w = 1.0;
        int64_t rem = o;
        for (int k = a.n_outer - 1; k >= 0; --k) {
          const int64_t ik = rem % a.size[k];
          rem /= a.size[k];
          if (k == d) continue;
          w *= a.dtype == CP_F64 ? ((const double*)a.apad[k])[ik * a.Rp + r]
                                 : (double)((const float*)a.apad[k])[ik * a.Rp + r];
        }
        s += a.pm[o * a.R + r] * w;
      }
    if (a.m64[d]) a.m64[d][e] = s;
    if (a.mout[d]) {
      if (a.dtype == CP_F64) ((double*)a.mout[d])[e] = s;
      else ((float*)a.mout[d])[e] = (float)s;
    }
  }
}

__global__ __launch_bounds__(256) void k_outer_contract(KOuterContract::Args a) {
  KOuterContract::run(a, CPGN_BID, CPGN_GDIM);
}

void KOuterContract::direct(dim3 grid, size_t lds, hipStream_t s, const Args& a) {
  hipLaunchKernelGGL(k_outer_contract, grid, dim3(kThreads), lds, s, a);
}

// Modes 0 .. N-2 at one point. With the dimension tree (FP32/FP64 storage, vector loads along
// the last mode, and Plan::tree) one pass over X gives M(0) and the outer modes' partials: for
// order 3 these are M(1) itself, for higher orders Pm, contracted by k_outer_contract. Otherwise
// one pass per mode. Each mode's result goes to its FP64 buffer and/or its caller-precision
// buffer (either may be null).
int launch_mttkrp_lead(const Plan& p, const void* X, void* ws, double* const* m64,
                       void* const* mout, hipStream_t st) {
  if (!p.tree || p.xk != 0 || !vec_ok(p, 0, X)) {
    for (int n = 0; n + 1 < p.N; ++n) {
      const int rc = launch_mttkrp(p, X, n, ws, m64[n], mout[n], st);
      if (rc) return rc;
    }
    return CP_OK;
  }
  double* pm = p.N == 3 ? m64[1] : (double*)((char*)ws + p.off_pm);
  void* pm_out = p.N == 3 ? mout[1] : nullptr;
  int rc = p.dtype == CP_F32
               ? launch_mttkrp_t<float>(p, X, 0, (char*)ws, m64[0], mout[0], true, pm, pm_out, st)
               : launch_mttkrp_t<double>(p, X, 0, (char*)ws, m64[0], mout[0], true, pm, pm_out,
                                         st);
  if (rc || p.N == 3) return rc;
  KOuterContract::Args a{};
  a.pm = pm;
  a.O = p.total / (p.s[0] * p.s[p.N - 1]);
  a.R = p.R;
  a.Rp = p.Rp;
  a.n_outer = p.N - 2;
  a.dtype = p.dtype;
  int64_t off = p.s[0];
  a.first[0] = 0;
  for (int d = 0; d < a.n_outer; ++d) {
    const int m = d + 1;
    a.size[d] = p.s[m];
    a.first[d + 1] = a.first[d] + p.s[m] * p.R;
    a.apad[d] = (char*)ws + p.off_apad + off * p.Rp * p.esz;
    off += p.s[m];
    a.m64[d] = m64[m];
    a.mout[d] = mout[m];
  }
  dispatch<KOuterContract>(dim3(grid_for(a.first[a.n_outer])), 0, st, a);
  return (int)hipGetLastError();
}

// Source factors may be the caller's buffers (compute precision) or FP64 copies.
int launch_prepare_factors_src(const Plan& p, const void* const* src, int src_dtype, void* wsv,
                               hipStream_t st, bool also_a64, unsigned krp_modes) {
  char* ws = (char*)wsv;
  PrepArgs a{};
  a.src_dtype = src_dtype;
  a.N = p.N;
  a.R = p.R;
  a.Rp = p.Rp;
  a.NBt = p.NBt;
  a.xk = p.xk;
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
  if (p.xk == 0) {
    a.seg[p.N + 1] = a.seg[p.N] + p.qc_last * p.NBt * 256;
    a.seg[p.N + 2] = a.seg[p.N + 1] + p.qc_prev * p.NBt * 256;
    a.seg[p.N + 3] = a.seg[p.N + 2];
  } else {
    a.fplane_last = (p.s[p.N - 1] + 31) / 32 * p.NBt * 512;
    a.fplane_prev = (p.s[p.N - 2] + 31) / 32 * p.NBt * 512;
    a.seg[p.N + 1] = a.seg[p.N] + a.fplane_last;
    a.seg[p.N + 2] = a.seg[p.N + 1] + a.fplane_prev;
    a.krp = (float*)(ws + p.off_krp);
    a.krp_seg[0] = 0;
    a.small32 = 1;
    int64_t dst = 0;
    for (int n = 0; n < p.N; ++n) {
      const int q = n == p.N - 1 ? p.N - 2 : p.N - 1;
      const int64_t O = p.total / p.s[n] / p.s[q];
      if (O >= ((int64_t)1 << 32) || p.s[n] >= ((int64_t)1 << 32)) a.small32 = 0;
      a.krp_dst[n] = dst;
      dst += O * p.Rp;
      a.krp_seg[n + 1] = a.krp_seg[n] + (((krp_modes >> n) & 1u) ? O * p.Rp : 0);
    }
    a.seg[p.N + 3] = a.seg[p.N + 2] + a.krp_seg[p.N];
  }
  const int grid = grid_for(a.seg[p.N + 3]);
  if (p.dtype == CP_F32) dispatch<KPrepare<float>>(dim3(grid), 0, st, a);
  else dispatch<KPrepare<double>>(dim3(grid), 0, st, a);
  return (int)hipGetLastError();
}

int launch_prepare_factors(const Plan& p, const void* const* A, void* ws, hipStream_t st,
                           bool also_a64) {
  return launch_prepare_factors_src(p, A, p.dtype, ws, st, also_a64, ~0u);
}

}  // namespace cpgn
