// Persistent execution of ragged (and uniform) plans of the projection-form operators
// (matern_cov_apply / matern_sample): one launch per dimensionality runs every level tile and
// coarse block of every instance, taking work items from a queue in device memory.
//
// The tile and coarse bodies are those of the level kernels (lowpass.h), so a plan gives the
// same results as single calls with the same schedule.  Dependencies: an item of step j of an
// instance waits until step j-1 of that instance has finished every tile; memory written by
// the producing tiles is made visible with an agent-scope release (every thread, before the
// tile is counted done) and an agent-scope acquire (every thread, after the wait), since the
// producer and the consumer may sit on different XCDs with separate L2 caches.
#include "internal.h"
#include "tiles.h"
#include "kcommon.h"
#include "lowpass.h"

namespace es {
namespace {

template <int D, int L>
struct PTiles {
  static constexpr Shape3 dn = shape_of(K_LP_DOWN, D, kPVariant, L);
  static constexpr Shape3 up = shape_of(K_LP_UP, D, kPVariant, L);
  using Down = LpDownSmem<D, L, dn.a, dn.b, dn.c>;
  using Up = LpUpSmem<D, L, up.a, up.b, up.c>;
};

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

// LDS of the persistent kernel of one (dimensionality, taps): its largest body.
template <int D, int L>
constexpr size_t persist_lds() {
  return cmax(cmax(sizeof(typename PTiles<D, L>::Down), sizeof(typename PTiles<D, L>::Up)),
              sizeof(float) * (size_t)coarse_lds_floats(kPCoarseMax));
}

DEVI void run_copy(const PStep* st, int tile) {
  const int64_t n = st->task.bs_in0;
  const int64_t b = (int64_t)tile * kPCopyChunk;
  const int64_t e = min(n, b + kPCopyChunk);
  const float* src = st->task.in0;
  float* dst = st->task.out0;
  if ((n & 3) == 0) {
    for (int64_t i = b + 4 * threadIdx.x; i < e; i += 4 * kPThreads) gst4(dst + i, gld4(src + i));
  } else {
    for (int64_t i = b + threadIdx.x; i < e; i += kPThreads) gst(dst + i, gld(src + i));
  }
}

// One kernel per (dimensionality, taps): a kernel holding the bodies of every filter length
// needs more than twice the registers of its largest body (one wave per SIMD), while one per
// filter length keeps the occupancy of the level kernels.
template <int D, int L>
__global__ void __launch_bounds__(kPThreads, 4) k_persist(PArgs a) {
  using T = PTiles<D, L>;
  __shared__ __attribute__((aligned(16))) char smem[persist_lds<D, L>()];
  __shared__ int s_item;
  int32_t* ctr = a.counters;
  const Filter& f = a.f;
  // the queue of this XCD: every tile of an instance runs on one XCD, so a consumer finds its
  // producers' stores in the L2 it shares with them, and level arrays are written once (no cache
  // holds a line of them from before it was written)
  const int q = (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15) % a.nq;  // XCC_ID[3:0]
  const int qe = a.qbegin[q + 1];
  // Thread 0's work of one iteration -- counting the previous item done, then taking the next --
  // is one block followed by a barrier.  (With the count at the end of the body and the take at
  // its start, the compiler joined the two thread-0 blocks across the loop's back edge into a
  // structure in which the other threads went back to the barrier without thread 0 and re-read
  // the same item forever.)
  int prev = -1, prev_n = 0, pending = 0;
  if (threadIdx.x == 0) pending = a.qbegin[q] + atomicAdd(ctr + q, 1);
  for (;;) {
    if (threadIdx.x == 0) {
      if (prev >= 0) atomicAdd(ctr + kPDone + prev, prev_n);
      s_item = pending;
      pending = a.qbegin[q] + atomicAdd(ctr + q, 1);  // the next item, taken while this one runs
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= qe) break;
    const PItem item = a.items[it];
    const PStep* st = a.steps + item.step;
    const int wait = st->wait;
    if (wait >= 0) {
      if (threadIdx.x == 0) {
        if (a.spin_limit < 0) {  // the host forces every wait to give up (tests of the error path)
          atomicOr(ctr + kPMaxQueues, 1);
        } else {
          const int need = st->wait_count;
          int spins = 0;
          while (__hip_atomic_load(ctr + kPDone + wait, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (++spins > a.spin_limit) {  // bounded: record the give-up and go on (results invalid)
              atomicOr(ctr + kPMaxQueues, 1);
              break;
            }
            __builtin_amdgcn_s_sleep(8);
          }
        }
      }
      __syncthreads();
    }
    const int kind = st->kind;
    const int t0 = item.tile0, nt = item.ntile;
    if (kind == P_LP_DOWN) {
      const Task t = st->task;
      for (int k = 0; k < nt; ++k) {
        if (k) __syncthreads();  // the previous tile's last LDS reads are done
        lp_down_tile<D, L, T::dn.a, T::dn.b, T::dn.c, kPThreads, true>(t, t0 + k, f,
                                                                        *reinterpret_cast<typename T::Down*>(smem));
      }
    } else if (kind == P_LP_UP) {
      const Task t = st->task;
      for (int k = 0; k < nt; ++k) {
        if (k) __syncthreads();
        lp_up_tile<D, L, T::up.a, T::up.b, T::up.c, kPThreads, true>(t, t0 + k, f,
                                                                      *reinterpret_cast<typename T::Up*>(smem));
      }
    } else if (kind == P_COARSE) {
      lp_coarse_block<D, L, kPCoarseMax, kPThreads>(&st->tail, 0, f, reinterpret_cast<float*>(smem));
    } else {
      for (int k = 0; k < nt; ++k) run_copy(st, t0 + k);
    }
    // every store of the item has reached the L2 before the item is counted done
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    prev = item.step;
    prev_n = nt;
  }
}

__global__ void __launch_bounds__(256) k_zero_ints(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

}  // namespace

template <int D>
hipError_t launch_persist_d(int taps, const PArgs& a, int grid, hipStream_t s) {
  switch (taps) {
    case 2: hipLaunchKernelGGL((k_persist<D, 2>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_persist<D, 4>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_persist<D, 6>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_persist<D, 8>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    case 10: hipLaunchKernelGGL((k_persist<D, 10>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    case 12: hipLaunchKernelGGL((k_persist<D, 12>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    case 14: hipLaunchKernelGGL((k_persist<D, 14>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_persist<D, 16>), dim3(grid), dim3(kPThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_persist(int ndim, int taps, const PArgs& args, int grid, hipStream_t s) {
  switch (ndim) {
    case 1: return launch_persist_d<1>(taps, args, grid, s);
    case 2: return launch_persist_d<2>(taps, args, grid, s);
    case 3: return launch_persist_d<3>(taps, args, grid, s);
  }
  return hipErrorInvalidValue;
}

template <int D>
hipError_t occupancy_d(int taps, int* per_cu) {
  switch (taps) {
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 2>, kPThreads, 0);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 4>, kPThreads, 0);
    case 6: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 6>, kPThreads, 0);
    case 8: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 8>, kPThreads, 0);
    case 10: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 10>, kPThreads, 0);
    case 12: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 12>, kPThreads, 0);
    case 14: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 14>, kPThreads, 0);
    case 16: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_persist<D, 16>, kPThreads, 0);
  }
  return hipErrorInvalidValue;
}

int persist_resident_groups(int ndim, int taps) {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  hipError_t e = hipErrorInvalidValue;
  switch (ndim) {
    case 1: e = occupancy_d<1>(taps, &per_cu); break;
    case 2: e = occupancy_d<2>(taps, &per_cu); break;
    case 3: e = occupancy_d<3>(taps, &per_cu); break;
  }
  if (e != hipSuccess || per_cu < 1) return 0;
  return per_cu * prop.multiProcessorCount;
}

hipError_t launch_zero_ints(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t grid = (n + 255) / 256;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)grid), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace es
