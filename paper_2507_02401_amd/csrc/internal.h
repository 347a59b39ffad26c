// Internal declarations shared by the host planner (api.cpp) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/eswave.h"

namespace es {

constexpr int kMaxTaps = 16;  // db8

// Filter taps in FP32, passed to kernels by value (kernel-argument SGPRs).
struct Filter {
  float h[kMaxTaps];  // low-pass (scaling) filter
  float g[kMaxTaps];  // high-pass g[t] = (-1)^t h[L-1-t]
};

// Work of one instance group for one kernel launch.  A group is `batch` instances with the
// same geometry whose arrays sit `bs_*` elements apart.  Dims are padded to three:
// 1-D (1,1,n), 2-D (1,n0,n1), 3-D (n0,n1,n2); the last dim is contiguous and the strides
// of dims 0 and 1 are given per array (elements).
//
// Field use per kernel kind:
//   LP_DOWN   a_out = A a_in                     in0 = a_in,  out0 = a_out
//   LP_UP     out = alpha*same + beta*(A^T z)     in0 = z, in1 = same, out0 = out
//   FB_DOWN   one full analysis level             in0 = a_in, out0 = coeff (detail bands, x alpha),
//                                                 out1 = next approximation (x beta)
//   FB_UP     one full synthesis level            in0 = approximation (x beta), in1 = coeff
//                                                 (detail bands, x alpha), out0 = result
//   LP_UP2    two low-pass synthesis levels:      in0 = z2 (level i+2), in1 = a1 (level i+1),
//             out = alpha*same + beta*A^T z1,    in2 = same (level i), out0 = out;
//             z1 = gamma*a1 + delta*A^T z2        b = level-i block (2-D only)
// `b` is the full-resolution block of the level (input of analysis, output of synthesis).
struct Task {
  const float* in0;
  const float* in1;
  const float* in2;
  float* out0;
  float* out1;
  int64_t bs_in0, bs_in1, bs_in2, bs_out0, bs_out1;  // per-instance strides
  int32_t st_in0[2], st_in1[2], st_out0[2], st_out1[2];  // strides of dims 0 and 1
  float alpha, beta, gamma, delta;
  int32_t batch;
  int32_t b[3];
  int32_t ntile[3];
  int32_t tiles_per_inst;
  int32_t tile_begin;  // first work-group index of this task within the launch
  int32_t flags;       // kNorm*: squared-norm mode of the full-bank analysis kernels
};
// Squared-norm mode (FB_DOWN / FB_DOWN_S / full-bank coarse analysis): the weighted coefficients
// are summed as squares instead of stored; each work-group writes its partial sum, a compensated
// FP32 pair (leading part, remainder), to ((float2*)out0)[work-group index within the task]
// (tail: ((float2*)out)[instance]).
constexpr int32_t kNormSq = 1;   // detail bands are summed, not stored
constexpr int32_t kNormLL = 2;   // the approximation output is final: summed, not stored

// Launch arguments: tasks either inline (count == 1) or in a device table.
struct TaskArgs {
  const Task* table;  // device table of `count` tasks, or null: the single task is t0
  int32_t count;
  int32_t total_wg;   // work-groups that carry work (grid is padded to a multiple of 8)
  int32_t vec;        // 1: every staged row is 16-byte aligned and a multiple of 4 floats
  int32_t reverse;    // 1: walk the tiles in reverse order (cache reuse between launches)
  Task t0;
};

// Tail: all coarse levels of one instance in one work-group (LDS resident).
// kind: 1 = full analysis (adjoint), 2 = full synthesis (apply), 3 = low-pass projection
//       form (cov / sample).  (Kind 0, a first low-pass version, was removed.)
struct TailTask {
  const float* in;   // LP: a_T (contiguous block b); FBA: a_T; FBS: coeff (strided)
  float* out;        // LP: z_T in place of a_T, or y when T == 0; FBA: coeff; FBS: a_T or x
  int64_t bs_in, bs_out;
  int32_t st_in[2], st_out[2];
  int32_t batch;
  int32_t b[3];      // block at the tail's first level T
  int32_t nlev;      // levels handled inside the tail
  int32_t flags;     // kNormSq: full-bank analysis sums squares (partial per instance to out)
  // LP:   coef[0] = alpha for the output (w_1 if T == 0 else c_T), coef[1 + j] = c_{T+1+j};
  //       the last level's z is c_{m-1} a_{m-1}.
  // FB:   coef[j] = weight of the detail bands of tail level j (j = 0 finest), coef[nlev] =
  //       approximation weight.
  float coef[32];
  int32_t tile_begin;
  int32_t pad2_;
};

struct TailArgs {
  const TailTask* table;  // device table, or null: the single task is t0
  int32_t count;
  int32_t total_wg;
  TailTask t0;
};

enum KernelKind {
  K_LP_DOWN = 0,
  K_LP_UP = 1,
  K_FB_DOWN = 2,
  K_FB_UP = 3,
  K_LP_UP2 = 4,
  K_FB_DOWN_S = 5,  // 3-D full analysis level, streamed along axis 0 (same Task fields as FB_DOWN)
  K_FB_UP_S = 6,    // 3-D full synthesis level, streamed along axis 0 (same Task fields as FB_UP)
  K_LP_DOWN_S = 7,  // low-pass analysis level, streamed along axis 1 (2-D) or axis 0 (3-D) (same Task fields as LP_DOWN)
  K_LP_UP_S = 8     // 3-D low-pass synthesis level, streamed along axis 0 (same Task fields as LP_UP)
};
inline bool kind_is_analysis(int k) {
  return k == K_LP_DOWN || k == K_FB_DOWN || k == K_FB_DOWN_S || k == K_LP_DOWN_S;
}

// Tile shape selection: each (kind, ndim, taps) has wide (0), narrow (1) and medium (2) tiles.
constexpr int kNumVariants = 3;
struct TileShape {
  int t[3];  // output tile in the kernel's tiling space (half-res for analysis kinds,
             // full-res for synthesis kinds); padded dims are 1
};

// Launchers (kernels.hip).  All return hipError_t of the launch.
hipError_t launch_level(int kind, int ndim, int taps, int variant, const TaskArgs& args, int grid,
                        const Filter& f, hipStream_t stream);
hipError_t launch_tail(int kind, int ndim, int taps, const TailArgs& args, int grid, size_t lds_bytes,
                       const Filter& f, hipStream_t stream);
// Largest block (floats) the low-pass coarse-level kernel (tail kind 3) holds in LDS: the small
// instantiation (32 KB of LDS) and the large one (128 KB: one work-group per CU), used when a call
// has so few instances that its level kernels could not fill the chip anyway.
constexpr int kCoarseMaxBlock = 4096;
constexpr int kCoarseMaxBlockBig = 16384;
// Largest block (floats) the full-bank coarse-level kernels (tail kinds 1, 2) hold in LDS.
constexpr int kFbCoarseMaxBlock = 8192;

// ------------------------------------------------------------------------------------------
// Persistent plan execution (persist.hip).  A plan's steps -- every level launch and coarse block
// of every instance, as its frozen schedule lists them -- become a step table, and their tiles a
// list of work items in an order the host chooses.  One launch per (dimensionality, taps) runs
// them all: each work-group takes the next item of its XCD's queue, waits until the
// step its step depends on (the previous step of the same instance) has finished all its
// tiles, runs the tile, and counts it done.  Items are listed so that every step's dependency
// comes earlier in the list: a work-group only waits for items that running work-groups have
// already taken, so the queue always drains.  Every wait is bounded: past `spin_limit` polls it
// sets the error word and goes on (the results are then invalid; the host reports ES_EDEVICE).
enum PKind { P_LP_DOWN = 0, P_LP_UP = 1, P_COARSE = 2, P_COPY = 3 };

struct PStep {
  Task task;          // P_LP_DOWN / P_LP_UP: batch 1, tile_begin 0; P_COPY: in0 -> out0, bs_in0 floats
  TailTask tail;      // P_COARSE: batch 1, the instance's coarse block
  int32_t kind;       // PKind
  int32_t L;          // taps
  int32_t wait;       // step whose completion this step needs (-1: none)
  int32_t wait_count; // tiles of that step
  int32_t ntiles;     // tiles of this step
  int32_t inst;       // instance (host bookkeeping)
  int32_t pad_[2];
};

struct PItem {
  int32_t step;
  int32_t tile0;   // tiles tile0 .. tile0 + ntile - 1 of the step, run in order by one work-group
  int32_t ntile;
  int32_t pad_;
};

// Items are split into one queue per XCD: every instance is assigned to one queue, and a
// work-group takes items only from the queue of the XCD it runs on, so all tiles of an instance
// run on one XCD and its level arrays stay in that XCD's L2.  counters[q]: next item of queue q;
// counters[kPMaxQueues]: error word; counters[kPDone + j]: finished tiles of step j.
constexpr int kPMaxQueues = 8;
constexpr int kPDone = kPMaxQueues + 1;
constexpr int kPCopyChunk = 16384;  // floats per copy tile
// Largest block the persistent kernels' coarse step holds in LDS (half the level kernels' small
// class: the coarse body then needs no more LDS than the 2-D tile bodies).
constexpr int kPCoarseMax = 2048;

struct PArgs {
  const PItem* items;
  const PStep* steps;
  int32_t* counters;
  int32_t nq;                         // queues (XCDs)
  int32_t spin_limit;
  int32_t qbegin[kPMaxQueues + 1];    // queue q holds items [qbegin[q], qbegin[q + 1])
  Filter f;                           // the launch's filter (one launch per dimensionality and taps)
};

// Work-group size of the persistent kernels and the tile variants they are built with.
constexpr int kPThreads = 256;
constexpr int kPVariant = 2;
hipError_t launch_persist(int ndim, int taps, const PArgs& args, int grid, hipStream_t stream);
// Work-groups of the persistent kernel of (ndim, taps) that fit on the device at once.
int persist_resident_groups(int ndim, int taps);
hipError_t launch_zero_ints(int32_t* p, int64_t n, hipStream_t stream);

// Plain reference path: one launch per 1-D pass.
struct PlainPass {
  const float* src;
  float* dst;
  int32_t b[3];        // leading block being transformed
  int32_t st_src[2], st_dst[2];
  int32_t axis;        // 0..2 in padded coordinates
  int32_t synth;       // 0 analysis, 1 synthesis
  int32_t scale_mode;  // 0 none, 1 scale outputs (analysis), 2 scale inputs (synthesis)
  int32_t ndim;
  float w;             // weight of the detail part of the block
};
hipError_t launch_plain_pass(const PlainPass& p, int taps, const Filter& f, hipStream_t stream);
hipError_t launch_block_copy(const float* src, float* dst, const int b[3], const int st_src[2],
                             const int st_dst[2], hipStream_t stream);
hipError_t launch_copy(const float* src, float* dst, int64_t n, hipStream_t stream);

// Copies n floats whatever n and the pointers' alignment: the multiple-of-4 prefix with 16-byte
// vectors when both pointers are 16-byte aligned, everything else element by element (launch_copy
// alone requires n % 4 == 0 and aligned pointers).
inline hipError_t launch_copy_any(const float* src, float* dst, int64_t n, hipStream_t stream) {
  const bool aligned = (((uintptr_t)src | (uintptr_t)dst) & 15) == 0;
  const int64_t head = aligned ? (n & ~(int64_t)3) : 0;
  hipError_t e = head > 0 ? launch_copy(src, dst, head, stream) : hipSuccess;
  for (int64_t done = head; e == hipSuccess && done < n;) {
    const int64_t c = n - done < ((int64_t)1 << 30) ? n - done : ((int64_t)1 << 30);
    const int b[3] = {1, 1, (int)c}, z[2] = {0, 0};
    e = launch_block_copy(src + done, dst + done, b, z, z, stream);
    done += c;
  }
  return e;
}

// Squared-norm finalisation: out[b] = sum over segments k of partials[off_k + b*per_k + t],
// t < per_k (compensated pairs, in units of pairs), in a fixed order (deterministic), rounded to
// FP32.  kMaxNormSegs segments at most.
constexpr int kMaxNormSegs = 40;
struct NormSegs {
  int64_t off[kMaxNormSegs];
  int32_t per[kMaxNormSegs];
  int32_t count;
};
hipError_t launch_norm_finalize(const float2* partials, const NormSegs& segs, float* out, int64_t batch,
                                hipStream_t stream);
// Sum of squares of each of `batch` contiguous instances of n floats (identity transform).
hipError_t launch_sumsq(const float* x, int64_t n, int64_t batch, float* out, hipStream_t stream);

// LP_UP (2-D, vector path) with the solver epilogue: args.t0.in2 = mask, t0.gamma its coefficient,
// t0.out1 = one float per work-group (sum of same * out).  Tile variant as for K_LP_UP.
hipError_t launch_lp_up_cge(int taps, int variant, const TaskArgs& args, int grid, const Filter& f,
                            hipStream_t stream);

// matern_cov_apply whose last launch is the 2-D vector-path synthesis with the solver epilogue:
//   y = (scale * w_1 + gamma * mask) x + scale * A^T z_1,
// and partials[b * per + k] = the k-th work-group's sum of x * y over instance b (per = the
// launch's tiles per instance, written to *per).  Returns ES_EUNSUPPORTED, enqueueing nothing,
// when the geometry's schedule does not end in such a launch (then run the steps separately).
es_status cov_apply_masked_dot(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                               const float* x, float* y, void* ws, size_t ws_bytes, const float* mask, float gamma,
                               float scale, float* partials, int64_t partials_cap, int64_t* per, hipStream_t stream);
// Largest `per` cov_apply_masked_dot can produce for this grid (0 when it never applies).
int64_t cov_dot_partials_max(int ndim, const int64_t* shape);

// Host filter derivation (filters.cpp).
bool daubechies_filter(int order, double* h_out);

// Host error reporting shared by the exported entry points (api.cpp): sets the thread-local
// message returned by es_last_error() and returns st; the gfx950 check of the current device.
es_status report_error(es_status st, const char* msg);
es_status device_check();

}  // namespace es
