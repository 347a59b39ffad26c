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
// are summed as squares instead of stored; each work-group writes its partial sum (double) to
// ((double*)out0)[work-group index within the task] (tail: ((double*)out)[instance]).
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
  K_LP_DOWN_S = 7   // 2-D low-pass analysis level, streamed along axis 1 (same Task fields as LP_DOWN)
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

// Squared-norm finalisation: out[b] = sum over segments k of partials[off_k + b*per_k + t],
// t < per_k, in a fixed order (deterministic).  kMaxNormSegs segments at most.
constexpr int kMaxNormSegs = 40;
struct NormSegs {
  int64_t off[kMaxNormSegs];
  int32_t per[kMaxNormSegs];
  int32_t count;
};
hipError_t launch_norm_finalize(const double* partials, const NormSegs& segs, double* out, int64_t batch,
                                hipStream_t stream);
// Sum of squares of each of `batch` contiguous instances of n floats (identity transform).
hipError_t launch_sumsq(const float* x, int64_t n, int64_t batch, double* out, hipStream_t stream);

// Host filter derivation (filters.cpp).
bool daubechies_filter(int order, double* h_out);

// Host error reporting shared by the exported entry points (api.cpp): sets the thread-local
// message returned by es_last_error() and returns st; the gfx950 check of the current device.
es_status report_error(es_status st, const char* msg);
es_status device_check();

}  // namespace es
