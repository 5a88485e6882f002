// FP64 matrix-core building blocks shared by the dense kernels (gfx950, 64-lane wavefronts).
//
// A 16x16x4 FP64 MFMA takes lane l = 16 g + m's A value A[m][g] and B value B[g][m] and leaves
// D[g + 4 v][m] in element v of the lane's accumulator. For a row x (R x R) product the lane owns
// row m of a 16-row tile; the contraction index of step j for lane group g is
// kstep(j, g) = 8 (j / 2) + 2 g + (j % 2), so each pair of steps reads two adjacent k of the
// row (one 16-byte load). The 16-column slice of the R x R operand sits in LDS as [k][16] with
// one padding row after every pair of rows, so that the four lane groups read alternate bank
// halves.
#pragma once

#include "cpgn_internal.h"

namespace cpgn {

typedef double dv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dv4 mfma64(double a, double b, dv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int kstep(int j, int g) { return 8 * (j >> 1) + 2 * g + (j & 1); }

__device__ __forceinline__ int sidx(int k, int c) { return (k + (k >> 1)) * 16 + c; }

constexpr int slice_elems(int KP) { return (KP + KP / 2) * 16; }

// Operand row r[0..KQ) of lane group g: elements kstep(j, g) of `row` (zero past R or when the
// row is outside the mode). EVEN: R is even, so each pair is one aligned 16-byte load.
template <int KQ, bool EVEN>
__device__ __forceinline__ void load_oprow(double (&r)[KQ], const double* row, bool rowok, int R,
                                           int g) {
#pragma unroll
  for (int j = 0; j < KQ; j += 2) {
    const int k = kstep(j, g);
    if (EVEN) {
      double2 v = make_double2(0.0, 0.0);
      if (rowok && k < R) v = *reinterpret_cast<const double2*>(row + k);
      r[j] = v.x;
      r[j + 1] = v.y;
    } else {
      r[j] = rowok && k < R ? row[k] : 0.0;
      r[j + 1] = rowok && k + 1 < R ? row[k + 1] : 0.0;
    }
  }
}

// Sum of v[0..NV) over the workgroup; every thread receives the same bits. Lanes combine by an
// xor butterfly (each pairwise sum is formed identically in both partners), then wavefront
// partials are added in wavefront order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[16][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i)
    for (int o = 32; o >= 1; o >>= 1) v[i] += __shfl_xor(v[i], o);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wv][i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w][i];
    v[i] = s;
  }
  __syncthreads();
}

}  // namespace cpgn
