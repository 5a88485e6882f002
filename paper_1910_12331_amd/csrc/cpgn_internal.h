// Internal declarations shared by the HIP translation units of libcpgn.so.
// Target: AMD Instinct MI355X (gfx950, CDNA4), 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/cpgn.h"

namespace cpgn {

constexpr int kWave = 64;
constexpr int kMaxOrder = CP_MAX_ORDER;
constexpr int kRedSlots = 1024;   // max blocks contributing to one deterministic reduction
// Largest rank of the Gauss-Newton step and the ALS sweep: their R x R inverse and the CG
// kernels' operand rows are held in registers, 16 columns per block, at most 13 blocks.
constexpr int kMaxGnRank = 208;
// Largest grid y (and z) dimension of a launch.
constexpr int64_t kMaxGridY = 65535;
constexpr int kMaxCgBatch = 128;   // problems per batched CG launch (their table is a kernel argument)
constexpr int kNumCU = 256;       // compute units of an MI355X (8 XCDs x 32)

// ------------------------------------------------------------------------------------------
// Matrix-core traits. Lane l of a wavefront supplies A[l%16][l/16] and B[l/16][l%16] to a
// 16x16x4 MFMA; the accumulator layout differs between the FP32 and FP64 instructions
// (checked on gfx950): FP32 lane l, element v holds D[4*(l/16)+v][l%16]; FP64 lane l,
// element v holds D[(l/16)+4*v][l%16].
// ------------------------------------------------------------------------------------------
template <typename T> struct Mfma;

template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  typedef float v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  typedef double v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// ------------------------------------------------------------------------------------------
// Problem geometry and workspace plan (host side)
// ------------------------------------------------------------------------------------------
struct Plan {
  int N = 0, R = 0, Rp = 0, NBt = 0;   // order, rank, rank padded to 16, column blocks of 16
  int dtype = 0;                       // CP_F64 or CP_F32 (compute precision of X and factors)
  int xk = 0;                          // X storage: 0 = dtype, 1 = bfloat16, 2 = split bfloat16
  size_t esz = 0;                      // bytes per element of the compute precision
  int64_t s[kMaxOrder] = {0};
  int64_t total = 0;                   // prod s
  int64_t sum_s = 0;                   // sum s
  int64_t max_s = 0;
  int64_t qc_last = 0, qc_prev = 0;    // 16-row chunks of modes N-1 and N-2
  int64_t part_elems = 0;              // MTTKRP partial buffer (elements of compute precision)
  // byte offsets into the workspace
  size_t off_apad = 0, off_fpk_last = 0, off_fpk_prev = 0, off_part = 0, off_p1 = 0;
  size_t off_m64 = 0, off_a64 = 0, off_s = 0, off_gam = 0, off_pinv = 0, off_dinv = 0;
  size_t off_g = 0, off_v = 0, off_r = 0, off_z = 0, off_w = 0, off_q = 0;
  size_t off_bp = 0, off_y = 0, off_red = 0, off_state = 0, off_w1 = 0, off_r1 = 0;
  size_t off_slots = 0;
  size_t off_cgargs = 0;                // the CG kernel arguments, for batched CG launches
  size_t off_krp = 0;                  // outer Khatri-Rao tables of the bfloat16 MTTKRP
  size_t bytes = 0;
  size_t t_bytes = 0;                  // ALS dimension tree (order 3): T = X x_3 A(2), after `bytes`
  // Dimension tree for modes 0 .. N-2 (FP32/FP64 storage): order 3 always, higher orders while
  // its partials (and the FP64 outer-mode product Pm at off_pm) stay small next to X
  bool tree = false;
  size_t off_pm = 0;
  // MTTKRP tile shape (cp_tuning of the calling thread when the plan was made)
  int mt_min_items = 16;               // least items per wavefront
  int mt_wg_per_cu = 2;                // workgroups per compute unit a launch aims for
  int mt_row_block = 0;                // FP32 row tile in 16-row blocks (0: automatic)
};

// Device-resident CG state (FP64 scalars never leave the device during a step).
struct CgState {
  double rz;         // sum <R,Z>
  double gsum;       // sum ||G(n)||_F
  double rsum;       // sum ||R(n)||_F
  double alpha, beta;
  double eps;        // eps_cg
  double upd2;       // sum ||V||^2
  int32_t done;      // 1 once CG has stopped (converged, failed or not started)
  int32_t status;    // CP_OK or a device status code
  int32_t iters;
  int32_t pad;
  double rho[2];     // sum <R,Z> of the last two CG iterations (by iteration parity)
  // Armijo step-size control (Section 5): f = 1/2 ||X - [[A]]||^2 (eq. (3)) at the start point,
  // the directional derivative <G, V>, the current trial step size and its objective value.
  double ls_f0, ls_xn, ls_gv, ls_alpha, ls_f;   // ls_xn = ||X||_F
  int32_t ls_done;      // 1 once a step size passed or the search cannot start (no trial runs)
  int32_t ls_trials;    // objective evaluations made
  int32_t ls_accepted;
  int32_t ls_pad;
};

// Per-mode pointer bundles passed by value to kernels.
template <typename P> struct PerMode {
  P p[kMaxOrder];
};

struct Dims {
  int N, R, Rp;
  int64_t s[kMaxOrder];
  int64_t off[kMaxOrder + 1];   // row offsets of each mode in packed [sum_s, R] arrays
};

// Row-block times small matrices (see k_rowmm in dense.hip).
struct RowMM {
  const double* in;  double cin;
  const double* l1;  const double* t1;  int64_t t1_stride;
  const double* l2;  const double* t2;  int64_t t2_stride;
  double* out;
  double* out2;      double out2_scale;
  const double* dotw;                 // D for <Out, D>
  double* red_dot;                    // [N][kRedSlots]
  double* red_nrm;                    // [N][kRedSlots]
  PerMode<void*> cast_out;            // optional copy in caller precision
  int cast_dtype;
  int mode_only;                      // -1: all modes (grid.y = N)
  int skip_if_status;                 // skip when the state records a failure
};

int make_plan(const cp_problem* prob, Plan* plan);
Dims make_dims(const Plan& p);

// Launch helpers (return hipError_t as int).
int launch_prepare_factors(const Plan& p, const void* const* A, void* ws, hipStream_t st,
                           bool also_a64);
// Events recorded on the stream right before the first and after the last launch of the main
// MTTKRP kernel (not the factor preparation or the partial-tile reduction); either may be null.
struct KernelMarks {
  hipEvent_t before = nullptr, after = nullptr;
};
int launch_mttkrp(const Plan& p, const void* X, int mode, void* ws, double* m64_out,
                  void* m_out_fdtype, hipStream_t st, KernelMarks mk = {});
// Work decomposition of one MTTKRP launch (shared by the workspace plan and the launcher).
struct MttkrpGeom {
  int MB;                 // 16-row blocks per wavefront tile
  int rows_per_tile;
  int64_t RT;             // row tiles
  int64_t SW;             // workgroups per row tile (4 wavefronts each split the items)
  int64_t QC, O, nitems;  // inner chunks, outer indices, items = O * QC
  int64_t HS;             // max wavefronts sharing one outer index within a row tile
};
MttkrpGeom mttkrp_geom(const Plan& p, int mode, bool vec_ok, bool dt);
MttkrpGeom mttkrp_geom_bf16(const Plan& p, int mode);

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__host__ __device__ __forceinline__ uint16_t to_bf16_rne(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_float(uint32_t h) {
  return __builtin_bit_cast(float, h << 16);
}
int launch_mttkrp_lead(const Plan& p, const void* X, void* ws, double* const* m64,
                       void* const* mout, hipStream_t st);

}  // namespace cpgn
