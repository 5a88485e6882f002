// Reduced-precision MTTKRP (the contraction of Section 2.2) on the gfx950 bf16 matrix cores:
// X stored in bfloat16, as one plane or as the two-plane split X = X_hi + X_lo; factors in
// FP32; every product is accumulated in FP32.
//
// Formulation. As in the FP32/FP64 kernels, the contraction is split into an inner mode q,
// whose factor is the MFMA B operand, and outer modes whose Khatri-Rao row is fixed per outer
// index o:  M(n)[j, r] = sum_{o, k} X[o, j, k] K[o, k, r],  K[o, k, r] = A(q)[k, r] P_o[r],
// with P_o the FP32 Khatri-Rao row of the outer modes (precomputed per o in the workspace).
// Each B operand entry K is formed in FP32 from the inner factor (staged in LDS) and P_o and
// rounded to bfloat16 once; in the split form it is split as K = K_hi + K_lo like X, and each
// tile takes the three products X_lo K_hi + X_hi K_lo + X_hi K_hi (the dropped X_lo K_lo term
// and the remainder of K's split are O(2^-16) relative). The products accumulate directly in
// FP32 registers; nothing else touches the accumulators until the end.
//   case A (n < N-1): q = N-1, the inner index is contiguous along X rows; lane (m, g) loads
//     the 8 inner elements [32 c + 8 g, +8) of output row 16 mb + m with one 16-byte load.
//   case B (n = N-1): q = N-2, the output index is contiguous; lane (m, g) loads 4 consecutive
//     output rows 4 m + mb for each of its 8 inner indices (8-byte loads) and regroups them
//     into one A operand per row block.
// Wavefronts own a contiguous range of (outer index, inner chunk) items of one row tile and keep
// the loads of the next items in flight in a ring of register buffers; the wavefronts of a
// workgroup are summed in LDS in a fixed order into one partial tile, and the partial tiles are
// added in FP64 in a fixed order, so the results are bitwise reproducible.
#include "cpgn_internal.h"

namespace cpgn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f8 __attribute__((ext_vector_type(8)));

constexpr int kBfNB = 4;              // column blocks of 16 per launch

constexpr int kBfLdsF = 64 * 1024;    // largest inner factor staged in LDS (bytes)

struct Bf16Args {
  const uint16_t* X;            // hi plane (or the only plane)
  int64_t xplane;               // elements between the hi and lo planes (split form)
  const f8* fpk;                // packed inner factor [QC][NBt][64 lanes] x 8 floats
  const float* krp;             // outer Khatri-Rao rows [O][Rp], FP32
  float* part;                  // partial tiles [SW][Jpad][Rp]
  int64_t J, Jpad, s_in, QC, nitems, Rr, nbo;
  int Rp, NBt, cb0, nb;         // nb: column blocks of this launch (<= kBfNB)
  int nsplit;                   // wavefronts along the item split (= waves per workgroup x gridDim.x)
  int flds;                     // inner factor staged in LDS (else read per item)
  int64_t rt0;                  // first row tile of this launch (grid y holds at most 65535)
};

// Tile and launch shape per case (measured at 80^4 R=64): case A keeps one wavefront per SIMD
// with a deep ring of in-flight items; case B, whose items need more regrouping work, runs two
// wavefronts per SIMD with a shallower ring. One workgroup per CU in both.
template <bool CASE_B> struct BfTile {
  static constexpr int MB = CASE_B ? 4 : 5;       // 16-row blocks per wavefront tile
  static constexpr int W = CASE_B ? 8 : 4;        // wavefronts per workgroup
  static constexpr int D1 = CASE_B ? 2 : 4;       // ring depth, single plane
  static constexpr int D3 = CASE_B ? 2 : 3;       // ring depth, split form
};

__device__ __forceinline__ f4 mfma_bf16(uint4 a, uint4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <bool CASE_B, int NP, bool FLDS, int NB>
struct BfBuf {
  static constexpr int MB = BfTile<CASE_B>::MB;
  uint4 x[NP][MB];             // A operands (8 bf16 of one output row) per plane and row block
  float kr[NB];                // outer Khatri-Rao row of the item's outer index (lane's columns)
  f8 f[FLDS ? 1 : NB];         // inner factor rows when the factor is not staged in LDS
};

// Eight FP32 values rounded to bfloat16 (nearest even) and packed as an MFMA operand; with a
// remainder plane, lo = bf16(v - hi) as well.
__device__ __forceinline__ uint4 pack_bf16(const f8& v) {
  uint32_t d[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    d[i] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{v[2 * i], v[2 * i + 1]}, bf16x2));
  return uint4{d[0], d[1], d[2], d[3]};
}
__device__ __forceinline__ f8 unpack_bf16(uint4 h) {
  const uint32_t d[4] = {h.x, h.y, h.z, h.w};
  f8 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __builtin_bit_cast(float, d[i] << 16);
    v[2 * i + 1] = __builtin_bit_cast(float, d[i] & 0xffff0000u);
  }
  return v;
}

// X fragment of one item. Every load is issued unconditionally from an in-bounds address: an
// inner index past s_in is clamped into the same row (the packed factor is zero there, so it
// contributes nothing for finite X), and an output row past J reads row J-1 (its result lands in
// a padding row of the partial tile that is never read). Without per-lane selects the loads stay
// branch-free, and the wait counts before each multiply cover only the item being consumed.
template <bool CASE_B, int NP, bool VEC, typename Buf>
__device__ __forceinline__ void bf_load_x(const Bf16Args& a, int64_t base, int64_t chunk,
                                          int64_t j0, int g, int m, Buf& b) {
  constexpr int MB = BfTile<CASE_B>::MB;
  const int64_t in0 = chunk * 32 + 8 * g;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const uint16_t* X = a.X + p * a.xplane + base;
    if constexpr (!CASE_B) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        int64_t j = j0 + 16 * mb + m;
        j = j < a.J ? j : a.J - 1;
        if constexpr (VEC) {
          const int64_t i = in0 < a.s_in ? in0 : a.s_in - 8;
          b.x[p][mb] = *(const uint4*)(X + j * a.Rr + i);
        } else {
          u16x8 h;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int64_t i = in0 + t < a.s_in ? in0 + t : a.s_in - 1;
            h[t] = X[j * a.Rr + i];
          }
          b.x[p][mb] = __builtin_bit_cast(uint4, h);
        }
      }
    } else {
      const int64_t jb = j0 + 4 * m;
      uint32_t lo16[8][2], hi16[8][2];   // dword d of the 4-row group: rows 2d (lo), 2d+1 (hi)
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int64_t inn = in0 + kk < a.s_in ? in0 + kk : a.s_in - 1;
        uint2 w;
        if constexpr (VEC) {
          w = *(const uint2*)(X + inn * a.J + (jb < a.J ? jb : a.J - 4));
        } else {
          u16x4 h;
#pragma unroll
          for (int v = 0; v < 4; ++v) h[v] = X[inn * a.J + (jb + v < a.J ? jb + v : a.J - 1)];
          w = __builtin_bit_cast(uint2, h);
        }
        lo16[kk][0] = w.x & 0xffffu;
        hi16[kk][0] = w.x >> 16;
        lo16[kk][1] = w.y & 0xffffu;
        hi16[kk][1] = w.y >> 16;
      }
      // row block mb = output rows jb + mb: 8 inner values, two per dword
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        uint32_t d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t e0 = (mb & 1) ? hi16[2 * q][mb >> 1] : lo16[2 * q][mb >> 1];
          const uint32_t e1 = (mb & 1) ? hi16[2 * q + 1][mb >> 1] : lo16[2 * q + 1][mb >> 1];
          d[q] = e0 | (e1 << 16);
        }
        b.x[p][mb] = uint4{d[0], d[1], d[2], d[3]};
      }
    }
  }
}

template <bool CASE_B, int NB, bool X3, bool VEC, bool FLDS>
__global__ __launch_bounds__(BfTile<CASE_B>::W * 64, 1) void k_mttkrp_bf16(Bf16Args a) {
  constexpr int MB = BfTile<CASE_B>::MB;
  constexpr int kBfWaves = BfTile<CASE_B>::W;
  constexpr int kBfThreads = kBfWaves * 64;
  constexpr int NP = X3 ? 2 : 1;
  typedef BfBuf<CASE_B, NP, FLDS, NB> Buf;
  extern __shared__ uint4 smem[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, m = lane & 15;
  const int split = blockIdx.x * kBfWaves + wave;
  const int64_t j0 = (a.rt0 + blockIdx.y) * 16 * MB;
  const int64_t it0 = a.nitems * split / a.nsplit;
  const int64_t it1 = a.nitems * (split + 1) / a.nsplit;

  // Stage the packed inner factor of this launch's column blocks as sF[chunk][nb][half][lane]:
  // each lane's 8 floats in two 16-byte halves, so that a wavefront's read of one half covers
  // 1 KB of consecutive LDS (no bank conflicts).
  uint4* sF = smem;
  if constexpr (FLDS) {
    const int64_t n = a.QC * NB * kWave;
    for (int64_t e = threadIdx.x; e < n; e += kBfThreads) {
      const int l = (int)(e % kWave);
      const int64_t r = e / kWave;
      const int nb = (int)(r % NB);
      const int64_t c = r / NB;
      const f8 v = a.fpk[(c * a.NBt + a.cb0 + nb) * kWave + l];
      sF[(2 * r) * kWave + l] = __builtin_bit_cast(uint4, f4{v[0], v[1], v[2], v[3]});
      sF[(2 * r + 1) * kWave + l] = __builtin_bit_cast(uint4, f4{v[4], v[5], v[6], v[7]});
    }
    __syncthreads();
  }

  f4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0, 0, 0, 0};

  auto issue = [&](Buf& b, int64_t o, int64_t chunk, int64_t base) {
    bf_load_x<CASE_B, NP, VEC>(a, base, chunk, j0, g, m, b);
    const float* kr = a.krp + o * a.Rp + 16 * a.cb0 + m;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b.kr[nb] = kr[16 * nb];
    if constexpr (!FLDS) {
      const f8* f = a.fpk + (chunk * a.NBt + a.cb0) * kWave + lane;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b.f[nb] = f[nb * kWave];
    }
  };
  auto consume = [&](const Buf& b, int64_t chunk) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      f8 fv;
      if constexpr (FLDS) {
        const f4 h0 = __builtin_bit_cast(f4, sF[(2 * (chunk * NB + nb)) * kWave + lane]);
        const f4 h1 = __builtin_bit_cast(f4, sF[(2 * (chunk * NB + nb) + 1) * kWave + lane]);
        fv = f8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
      } else {
        fv = b.f[nb];
      }
      const f8 kv = fv * b.kr[nb];   // Khatri-Rao entries of this lane's 8 inner rows, FP32
      const uint4 khi = pack_bf16(kv);
      uint4 klo;
      if constexpr (X3) klo = pack_bf16(kv - unpack_bf16(khi));   // exact difference
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        if constexpr (X3) {
          acc[mb][nb] = mfma_bf16(b.x[1][mb], khi, acc[mb][nb]);
          acc[mb][nb] = mfma_bf16(b.x[0][mb], klo, acc[mb][nb]);
        }
        acc[mb][nb] = mfma_bf16(b.x[0][mb], khi, acc[mb][nb]);
      }
    }
  };

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

  // Ring of D item buffers: the loads of the next D - 1 items are in flight while the current
  // one is multiplied (one wavefront per SIMD, so the in-flight bytes come from depth rather
  // than from other wavefronts). Items past the range repeat the last one (harmless re-loads,
  // never multiplied).
  constexpr int D = !FLDS ? 2 : X3 ? BfTile<CASE_B>::D3 : BfTile<CASE_B>::D1;
  Buf buf[D];
  Pos pos[D];
  if (it0 < it1) {
    Pos q{0, 0, 0, 0};
    q.o = it0 / a.QC;
    q.chunk = it0 - q.o * a.QC;
    if constexpr (CASE_B) {
      q.base = q.o * a.s_in * a.J;
    } else {
      const int64_t aa = q.o / a.nbo;
      q.bo = q.o - aa * a.nbo;
      q.base = aa * a.J * a.Rr + q.bo * a.s_in;
    }
    Pos nx = q;                 // next position to issue
    int64_t inx = it0;          // its item index
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {
      pos[k] = nx;
      issue(buf[k], nx.o, nx.chunk, nx.base);
      if (inx + 1 < it1) {
        nx = advance(nx);
        ++inx;
      }
    }
    for (int64_t it = it0; it < it1; it += D) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int ki = (k + D - 1) % D;   // buffer of item it + k + D - 1
        pos[ki] = nx;
        issue(buf[ki], nx.o, nx.chunk, nx.base);
        if (inx + 1 < it1) {
          nx = advance(nx);
          ++inx;
        }
        if (it + k < it1) consume(buf[k], pos[k].chunk);
      }
    }
  }

  // Fixed-order sum of the wavefronts through LDS (the staged factor is dead once every
  // wavefront has passed the first barrier): at level h, wavefront w < h adds wavefront w + h,
  // two source wavefronts per round through two LDS slots.
  f4* red = (f4*)smem;   // [2][MB * NB][64]
  for (int h = kBfWaves / 2; h >= 1; h /= 2) {
    for (int r0 = 0; r0 < h; r0 += 2) {
      __syncthreads();
      if (wave >= h + r0 && wave < h + r0 + 2) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            red[((wave - h - r0) * MB * NB + mb * NB + nb) * kWave + lane] = acc[mb][nb];
      }
      __syncthreads();
      if (wave >= r0 && wave < r0 + 2 && wave < h) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] += red[((wave - r0) * MB * NB + mb * NB + nb) * kWave + lane];
      }
    }
  }
  if (wave == 0) {
    float* P = a.part + (int64_t)blockIdx.x * a.Jpad * a.Rp;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const f4 tot = acc[mb][nb];
        const int col = 16 * (a.cb0 + nb) + m;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 4 * g + v;   // accumulator row of element v
          const int64_t row = CASE_B ? j0 + 4 * i + mb : j0 + 16 * mb + i;
          P[row * a.Rp + col] = tot[v];
        }
      }
  }
}

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------
void launch_mttkrp_reduce_f32(const float* part, int nparts, int64_t Jpad, int Rp, int64_t J,
                              int R, double* m64, void* mout, int mout_dtype, hipStream_t st);

MttkrpGeom mttkrp_geom_bf16(const Plan& p, int mode) {
  MttkrpGeom g{};
  const bool caseB = mode == p.N - 1;
  const int q = caseB ? p.N - 2 : p.N - 1;
  const int64_t J = p.s[mode];
  g.MB = caseB ? BfTile<true>::MB : BfTile<false>::MB;
  const int waves = caseB ? BfTile<true>::W : BfTile<false>::W;
  g.rows_per_tile = 16 * g.MB;
  g.RT = (J + g.rows_per_tile - 1) / g.rows_per_tile;
  g.QC = (p.s[q] + 31) / 32;
  g.O = p.total / J / p.s[q];
  g.nitems = g.O * g.QC;
  const int64_t wgs = kNumCU;   // one resident round: one workgroup per CU
  int64_t sw = wgs / g.RT;
  const int64_t max_sw = (g.nitems + 2 * waves - 1) / (2 * waves);
  if (sw > max_sw) sw = max_sw;
  if (sw > kRedSlots) sw = kRedSlots;
  if (sw < 1) sw = 1;
  g.SW = sw;
  g.HS = 0;
  return g;
}

static bool bf_vec_ok(const Plan& p, int mode, const void* X) {
  if (mode == p.N - 1) return ((uintptr_t)X % 8) == 0 && p.s[mode] % 4 == 0;
  return ((uintptr_t)X % 16) == 0 && p.s[p.N - 1] % 8 == 0;
}

template <bool CASE_B, bool X3, bool VEC>
static void bf_launch_nb(int NB, dim3 grid, size_t lds, hipStream_t st, const Bf16Args& a) {
  switch (NB) {
#define CPGN_NB(k)                                                                            \
  case k:                                                                                     \
    if (a.flds)                                                                               \
      hipLaunchKernelGGL((k_mttkrp_bf16<CASE_B, k, X3, VEC, true>), grid,                  \
                         dim3(BfTile<CASE_B>::W * 64), lds, st, a);                             \
    else                                                                                      \
      hipLaunchKernelGGL((k_mttkrp_bf16<CASE_B, k, X3, VEC, false>), grid,                 \
                         dim3(BfTile<CASE_B>::W * 64), lds, st, a);                             \
    break;
    CPGN_NB(1) CPGN_NB(2) CPGN_NB(3) CPGN_NB(4)
#undef CPGN_NB
    default: break;
  }
}

template <bool CASE_B>
static void bf_launch(bool x3, bool vec, int NB, dim3 grid, size_t lds, hipStream_t st,
                      const Bf16Args& a) {
  if (x3) {
    if (vec) bf_launch_nb<CASE_B, true, true>(NB, grid, lds, st, a);
    else bf_launch_nb<CASE_B, true, false>(NB, grid, lds, st, a);
  } else {
    if (vec) bf_launch_nb<CASE_B, false, true>(NB, grid, lds, st, a);
    else bf_launch_nb<CASE_B, false, false>(NB, grid, lds, st, a);
  }
}

// Element offset of mode n's outer Khatri-Rao table in the workspace region (FP32 [O_n][Rp]).
int64_t bf16_krp_offset(const Plan& p, int mode) {
  int64_t off = 0;
  for (int n = 0; n < mode; ++n) {
    const int q = n == p.N - 1 ? p.N - 2 : p.N - 1;
    off += p.total / p.s[n] / p.s[q] * p.Rp;
  }
  return off;
}

int launch_mttkrp_bf16(const Plan& p, const void* X, int mode, void* wsv, double* m64, void* mout,
                       hipStream_t st, KernelMarks mk) {
  char* ws = (char*)wsv;
  const bool caseB = mode == p.N - 1;
  const int q = caseB ? p.N - 2 : p.N - 1;
  const bool x3 = p.xk == 2;
  const bool vec = bf_vec_ok(p, mode, X);
  const MttkrpGeom G = mttkrp_geom_bf16(p, mode);
  Bf16Args a{};
  a.X = (const uint16_t*)X;
  a.xplane = p.total;
  a.fpk = (const f8*)(ws + (caseB ? p.off_fpk_prev : p.off_fpk_last));
  a.krp = (const float*)(ws + p.off_krp) + bf16_krp_offset(p, mode);
  a.part = (float*)(ws + p.off_part);
  a.J = p.s[mode];
  a.Jpad = G.RT * G.rows_per_tile;
  a.s_in = p.s[q];
  a.QC = G.QC;
  a.nitems = G.nitems;
  a.Rr = 1;
  for (int m = mode + 1; m < p.N; ++m) a.Rr *= p.s[m];
  a.nbo = caseB ? 1 : a.Rr / a.s_in;
  a.Rp = p.Rp;
  a.NBt = p.NBt;
  a.nsplit = (int)((caseB ? BfTile<true>::W : BfTile<false>::W) * G.SW);
  if (mk.before) {
    const hipError_t e = hipEventRecord(mk.before, st);
    if (e != hipSuccess) return (int)e;
  }
  for (int cb0 = 0; cb0 < p.NBt; cb0 += kBfNB) {
    const int NB = p.NBt - cb0 < kBfNB ? p.NBt - cb0 : kBfNB;
    a.cb0 = cb0;
    a.nb = NB;
    const size_t fbytes = (size_t)G.QC * NB * kWave * 32;
    const size_t rbytes = (size_t)2 * G.MB * NB * kWave * 16;
    a.flds = fbytes <= (size_t)kBfLdsF ? 1 : 0;
    const size_t lds = a.flds && fbytes > rbytes ? fbytes : rbytes;
    for (int64_t rt0 = 0; rt0 < G.RT; rt0 += kMaxGridY) {   // row tiles in chunks of grid y
      a.rt0 = rt0;
      const int64_t nrt = G.RT - rt0 < kMaxGridY ? G.RT - rt0 : kMaxGridY;
      const dim3 grid((unsigned)G.SW, (unsigned)nrt);
      if (caseB) bf_launch<true>(x3, vec, NB, grid, lds, st, a);
      else bf_launch<false>(x3, vec, NB, grid, lds, st, a);
    }
  }
  if (mk.after) {
    const hipError_t e = hipEventRecord(mk.after, st);
    if (e != hipSuccess) return (int)e;
  }
  launch_mttkrp_reduce_f32(a.part, (int)G.SW, a.Jpad, p.Rp, a.J, p.R, m64, mout, CP_F32, st);
  return (int)hipGetLastError();
}

__global__ void k_to_bf16(const float* __restrict__ X, int64_t n, int split,
                          uint16_t* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float x = X[e];
    const uint16_t hi = to_bf16_rne(x);
    out[e] = hi;
    if (split) out[n + e] = to_bf16_rne(x - bf16_to_float(hi));
  }
}

}  // namespace cpgn

extern "C" int cp_tensor_to_bf16(const float* X, int64_t n, int split, void* out, void* stream) {
  if (n < 0 || (n > 0 && (!X || !out))) return CP_EINVAL;
  if (n == 0) return CP_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(cpgn::k_to_bf16, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     X, n, split, (uint16_t*)out);
  return hipGetLastError() == hipSuccess ? CP_OK : CP_EHIP;
}
