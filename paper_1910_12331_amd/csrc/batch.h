// Batched launches: the launches of one Gauss-Newton step are recorded per problem once, and one
// launch per (kernel, position in the step) then runs the workgroups of every problem of a batch.
//
// A batchable kernel K provides
//   K::Args      its arguments as one struct (trivially copyable),
//   K::kThreads  its workgroup size,
//   K::run(a, bid, gdim)   the kernel body for workgroup `bid` of a grid `gdim` (device),
//   K::direct(grid, lds, stream, a)   the ordinary launch of the kernel (host).
// dispatch<K>() launches K directly, or, while a recorder is installed on the calling host
// thread, appends the launch (grid, dynamic LDS, argument bytes) to it instead. A recorded
// launch is later run by k_batched<K>, which finds its member from a table of workgroup offsets
// (a kernel argument), reads that member's grid and arguments from device memory and runs the
// same body, so each member computes exactly what its direct launch computes.
#pragma once

#include <string.h>

#include <vector>

#include "cpgn_internal.h"

namespace cpgn {

constexpr int kMaxBatch = 128;   // members of one batched launch

// This workgroup's index and the grid, for a direct launch of a kernel body.
#define CPGN_BID dim3(blockIdx.x, blockIdx.y, blockIdx.z)
#define CPGN_GDIM dim3(gridDim.x, gridDim.y, gridDim.z)

// Kernel argument of a batched launch. blk[i] points to member i's record in device memory:
// its grid (x, y, z) in the first 16 bytes, then its K::Args.
struct BatchTab {
  const unsigned char* blk[kMaxBatch];
  int off[kMaxBatch + 1];   // workgroups before each member
  int n;
};

constexpr size_t kBatchHeader = 16;

// Member of this workgroup (uniform) and the workgroup's index within that member's grid.
__device__ __forceinline__ int batch_member(const BatchTab& t, int& local) {
  __shared__ int sq;
  for (int q = threadIdx.x; q < t.n; q += blockDim.x)
    if (t.off[q] <= (int)blockIdx.x && (int)blockIdx.x < t.off[q + 1]) sq = q;
  __syncthreads();
  const int q = sq;
  local = (int)blockIdx.x - t.off[q];
  return q;
}

// (The widest MTTKRP tiles cannot keep two workgroups per CU here: the compiler's occupancy
// note for them is expected.)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wpass-failed"
// The arguments are read in place through a no-alias pointer (the table is never written while
// kernels run), so the compiler keeps uniform reads scalar and reorders them freely around the
// body's stores; a private copy would put any array indexed at run time in scratch memory.
template <class K>
__device__ __forceinline__ void batched_run(const typename K::Args* __restrict__ a, dim3 bid,
                                            dim3 gdim) {
  K::run(*a, bid, gdim);
}

template <class K>
__global__ __launch_bounds__(K::kThreads, K::kMinBlocks) void k_batched(BatchTab t) {
  int local;
  const int q = __builtin_amdgcn_readfirstlane(batch_member(t, local));
  const unsigned char* blk = t.blk[q];
  const uint32_t* g = (const uint32_t*)blk;
  const uint32_t gx = g[0], gy = g[1], gz = g[2];
  const uint32_t l = (uint32_t)local;
  batched_run<K>((const typename K::Args*)(blk + kBatchHeader),
                 dim3(l % gx, (l / gx) % gy, l / (gx * gy)), dim3(gx, gy, gz));
}
#pragma clang diagnostic pop

// A recorded launch.
struct BatchRec {
  void (*launch)(const BatchTab&, unsigned blocks, size_t lds, hipStream_t);   // also the key
  std::vector<unsigned char> blk;   // header + arguments, as copied to device memory
  unsigned blocks = 0;
  size_t lds = 0;
};

// The recorder of the calling host thread (null: launches run directly).
extern thread_local std::vector<BatchRec>* t_batch_rec;

template <class K>
void batch_launch(const BatchTab& t, unsigned blocks, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_batched<K>, dim3(blocks), dim3(K::kThreads), lds, s, t);
}

template <class K>
void dispatch(dim3 grid, size_t lds, hipStream_t s, const typename K::Args& a) {
  if (t_batch_rec) {
    BatchRec r;
    r.launch = &batch_launch<K>;
    r.blocks = grid.x * grid.y * grid.z;
    r.lds = lds;
    r.blk.assign(kBatchHeader + sizeof(a), 0);
    const uint32_t g[3] = {grid.x, grid.y, grid.z};
    memcpy(r.blk.data(), g, sizeof(g));
    memcpy(r.blk.data() + kBatchHeader, &a, sizeof(a));
    t_batch_rec->push_back(std::move(r));
    return;
  }
  K::direct(grid, lds, s, a);
}

}  // namespace cpgn
