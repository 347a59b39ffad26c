// Non-periodic realisation of E_s^* = W^{-1} D W (Sec. 4): the fast wavelet transform that the
// paper evaluates with MATLAB's routines, whose default boundary handling is half-point symmetric
// extension and whose band lengths l(i) shrink per level and are kept in a book-keeping matrix.
//
// One analysis step of a length-n axis mirrors the signal about its ends, repeating the end
// samples (x_ext[-1-j] = x[j], x_ext[n+j] = x[n-1-j]; period 2n), and keeps
//   a[k] = sum_t h[t] x_ext[2k + t - (L-2)],   k < l = floor((n + L - 1) / 2),
// and the same with g[t] = (-1)^t h[L-1-t] for the detail band.  The step is redundant (2l >= n)
// and not orthogonal; its left inverse keeps the central n samples of the upsampled, filtered
// bands:
//   x[i] = sum_k h[i + L - 2 - 2k] a[k] + g[i + L - 2 - 2k] d[k],   0 <= k < l.
// With S_a, S_d the two halves of that synthesis and A, B the two analysis halves,
// S_a A + S_d B = I on every length-n signal, and a d-dimensional level is the tensor product of
// the steps along every axis (the all-low band's synthesis S_a^{(d)} after A^{(d)}, plus 2^d - 1
// detail terms that sum to I - S_a^{(d)} A^{(d)}).  With detail level i weighted
// w_i = 2^{-2s(m-i)} and the approximation weighted 1 (= w_m), the operator therefore has the
// projection form of the periodic case with A^T replaced by S_a:
//   W^{-1} D W = w_1 I + sum_{i=1}^{m-1} c_i S_a^i A^i,   c_i = w_{i+1} - w_i,
// evaluated by the Horner recurrence
//   a_i = A a_{i-1} (a_0 = x),  z_{m-1} = c_{m-1} a_{m-1},  z_i = c_i a_i + S_a z_{i+1},
//   y = w_1 x + S_a z_1.
// Only all-low bands are formed; level m is never visited.
//
// Kernels (one work-group = one output tile, 256 threads):
//   k_sym_down  a_out = A a_in: the tile's input window (2T + L - 2 per axis) is staged in LDS
//               through per-axis tables of reflected indices, then filtered axis 2, 1, 0.
//   k_sym_up    out = alpha * same + beta * S_a z: the window of z (U/2 + L/2 - 1 per axis,
//               starting at half the tile origin) is staged with zeros outside [0, l), then
//               filtered axis 2, 1, 0; the last pass writes the combination to global memory.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/eswave.h"
#include "internal.h"
#include "kcommon.h"

namespace es {

namespace {

// Position j of the half-point symmetric extension of a length-n axis, as an index into [0, n).
DEVI int sym_ix(int j, int n) {
  const int p = 2 * n;
  j %= p;
  if (j < 0) j += p;
  return j < n ? j : p - 1 - j;
}

typedef float f2v_t __attribute__((ext_vector_type(2)));
DEVI float2 gld2(const float* p) {
  const f2v_t v = *(const GAS f2v_t*)p;
  return make_float2(v.x, v.y);
}

struct SymTask {
  const float* in;    // down: a_{i-1}; up: the coarser array z
  const float* same;  // up: the array combined with weight alpha (may equal out)
  float* out;
  int64_t bs_in, bs_same, bs_out;  // per-instance strides in floats (contiguous instances)
  int32_t ni[3];                   // padded dims of `in` (1-D: (1,1,n), 2-D: (1,n0,n1))
  int32_t no[3];                   // padded dims of `out` (and `same`)
  int32_t si[2];                   // strides (floats) of axes 0 and 1 of `in`
  int32_t so[2];                   // strides of axes 0 and 1 of `out` and `same`
  int32_t nt[3];                   // tiles per axis
  int32_t tiles_per_inst;
  int32_t zshift;                  // synthesis: the z window starts zshift samples before o/2
  float alpha, beta;               // synthesis: same == nullptr drops the alpha term
};

// Sign-correct integer division rounding down / up (b > 0).
DEVI int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
DEVI int ceil_div(int a, int b) { return -floor_div(-a, b); }

// Calls f(p) for every position p in [lo, hi] of the half-point symmetric extension of a length-n
// axis that reflects to sample j: p = j + 2n t and p = -1 - j + 2n t.
template <class F>
DEVI void for_images(int j, int n, int lo, int hi, F f) {
  const int P = 2 * n;
  for (int t = ceil_div(lo - j, P), te = floor_div(hi - j, P); t <= te; ++t) f(j + P * t);
  const int q = -1 - j;
  for (int t = ceil_div(lo - q, P), te = floor_div(hi - q, P); t <= te; ++t) f(q + P * t);
}

// Output tile (T0, T1, T2) of one analysis level; input window I_k = 2 T_k + L - 2 starting at
// 2 o_k - (L - 2) (o_k the tile's first output).  The staged rows are filtered along axis 2 with
// the periodic kernels' in-place row pass (16-byte LDS windows, results written back over the
// staging buffer as rows of T2), then along axes 1 and 0.
// ZX: the signal is extended by zeros instead of by reflection -- the transpose S_a^T of the
// synthesis's low-pass half (used by the transposed operator).
template <int D, int L, int T0, int T1, int T2, int NT, bool ZX>
__global__ void __launch_bounds__(NT) k_sym_down(SymTask t, Filter f) {
  constexpr int I0 = D >= 3 ? 2 * T0 + L - 2 : 1;
  constexpr int I1 = D >= 2 ? 2 * T1 + L - 2 : 1;
  constexpr int I2 = 2 * T2 + L - 2;
  constexpr int I2P = (I2 + 3) & ~3;
  constexpr int NROW = I0 * I1;
  constexpr int NB = D >= 3 ? I0 * T1 * T2 : 1;
  constexpr int P1 = D >= 3 ? 2 : 4, P0 = 2;
  // the window start 2 o_2 - (L - 2) is SH floats past a 16-byte boundary (T2 even)
  constexpr int SH = (L - 2) & 3 ? 4 - ((L - 2) & 3) : 0;
  constexpr int NVL = (SH + I2 + 3) / 4;  // 16-byte groups loaded per row
  constexpr int NLD = NROW * NVL, ITL = (NLD + NT - 1) / NT;
  static_assert(T2 % 4 == 0 && (D < 2 || T1 % P1 == 0) && (D < 3 || T0 % P0 == 0), "tile shape");
  static_assert(NROW * T2 + NB <= NROW * I2P, "axis-1 results must fit past the axis-2 rows");
  __shared__ __attribute__((aligned(16))) float s_in[NROW * I2P];
  // 3-D: the axis-1 results go past the axis-2 rows in the staging buffer (the axis-1 pass reads
  // only those rows), which keeps the 16-tap tile within half of the CU's LDS
  float* const s_b = s_in + NROW * T2;
  __shared__ int s_row[NROW], s_x2[I2];

  const int wg = blockIdx.x;
  const int inst = wg / t.tiles_per_inst;
  int rem = wg - inst * t.tiles_per_inst;
  const int c2 = rem % t.nt[2];
  rem /= t.nt[2];
  const int c1 = rem % t.nt[1], c0 = rem / t.nt[1];
  const float* src = t.in + inst * t.bs_in;
  float* dst = t.out + inst * t.bs_out;
  const int n0 = t.ni[0], n1 = t.ni[1], n2 = t.ni[2];
  const int m0 = t.no[0], m1 = t.no[1], m2 = t.no[2];
  const int o0 = T0 * c0, o1 = T1 * c1, o2 = T2 * c2;  // first output of the tile on each axis

  // staged row r = (i0, i1): offset of its reflected source row; along axis 2 the window runs
  // from base2, through a table of reflected columns only where it reaches past an end
  for (int r = threadIdx.x; r < NROW; r += NT) {
    const int i1 = r % I1, i0 = r / I1;
    const int j0 = 2 * o0 - (L - 2) + i0, j1 = 2 * o1 - (L - 2) + i1;
    if constexpr (ZX) {  // -1: a row outside the signal (zeros)
      const bool ok = (D < 3 || (j0 >= 0 && j0 < n0)) && (D < 2 || (j1 >= 0 && j1 < n1));
      s_row[r] = ok ? (D >= 3 ? j0 * t.si[0] : 0) + (D >= 2 ? j1 * t.si[1] : 0) : -1;
    } else {
      s_row[r] = (D >= 3 ? sym_ix(j0, n0) * t.si[0] : 0) + (D >= 2 ? sym_ix(j1, n1) * t.si[1] : 0);
    }
  }
  const int base2 = 2 * o2 - (L - 2), a2 = base2 - SH;
  // rows start at multiples of 4 floats (and so do instances): 16-byte loads inside the row
  const bool vec = ((t.si[0] | t.si[1] | t.bs_in) & 3) == 0 && a2 >= 0 && a2 + 4 * NVL <= n2;
  const bool inner = base2 >= 0 && base2 + I2 <= n2;
  if (!inner)
    for (int i = threadIdx.x; i < I2; i += NT) {
      const int j = base2 + i;
      s_x2[i] = ZX ? (j >= 0 && j < n2 ? j : -1) : sym_ix(j, n2);
    }
  __syncthreads();
  if (vec) {
    // 16-byte loads from the aligned start a2 (row offsets are multiples of 4), all issued before
    // the first LDS store; group v of a row lands at LDS positions 4v - SH .. 4v - SH + 3
    float4 v[ITL];
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, NLD - 1);
      const int r = q / NVL, g = q - r * NVL;
      v[it] = !ZX || s_row[r] >= 0 ? gld4(src + s_row[r] + a2 + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int q = int(threadIdx.x) + it * NT;
      if (q < NLD) {
        const int r = q / NVL, g = q - r * NVL;
        float* row = s_in + r * I2P;
        if constexpr (SH == 0) {
          *reinterpret_cast<float4*>(row + 4 * g) = v[it];
        } else {
          if (g > 0) *reinterpret_cast<float2*>(row + 4 * g - 2) = make_float2(v[it].x, v[it].y);
          if (4 * g + 2 <= I2P) *reinterpret_cast<float2*>(row + 4 * g) = make_float2(v[it].z, v[it].w);
        }
      }
    }
  } else {
    gather_to_lds<NT, 8>(
        NROW * I2,
        [&](int e) {
          const int r = e / I2, i2 = e - r * I2;
          const int c = inner ? base2 + i2 : s_x2[i2];
          return !ZX || (s_row[r] >= 0 && c >= 0) ? gld(src + s_row[r] + c) : 0.f;
        },
        [&](int e, float x) {
          const int r = e / I2;
          s_in[r * I2P + e - r * I2] = x;
        });
  }
  __syncthreads();

  // axis 2: (NROW, I2) -> (NROW, T2), written back over the staging buffer
  row_pass_inplace<L, 4, NROW, T2, I2P, NT, false>(s_in, f);

  if constexpr (D == 1) {
    for (int k = threadIdx.x; k < T2; k += NT) {
      const int g2 = o2 + k;
      if (g2 < m2) gst(dst + g2, s_in[k]);
    }
  } else if constexpr (D == 2) {
    analysis_pass<L, P1, false, true, NT>(
        T2, T1 / P1, f,
        [&](int c, int j0, float* w) {
#pragma unroll
          for (int j = 0; j < 2 * P1 + L - 2; ++j) w[j] = s_in[(j0 + j) * T2 + c];
        },
        [&](int c, int k, float lo, float) {
          const int g1 = o1 + k, g2 = o2 + c;
          if (g1 < m1 && g2 < m2) gst(dst + g1 * t.so[1] + g2, lo);
        });
  } else {
    analysis_pass<L, P1, false, true, NT>(
        I0 * T2, T1 / P1, f,
        [&](int l, int j0, float* w) {
          const int c = l % T2, i0 = l / T2;
#pragma unroll
          for (int j = 0; j < 2 * P1 + L - 2; ++j) w[j] = s_in[(i0 * I1 + j0 + j) * T2 + c];
        },
        [&](int l, int k, float lo, float) {
          const int c = l % T2, i0 = l / T2;
          s_b[(i0 * T1 + k) * T2 + c] = lo;
        });
    __syncthreads();
    analysis_pass<L, P0, false, true, NT>(
        T1 * T2, T0 / P0, f,
        [&](int l, int j0, float* w) {
#pragma unroll
          for (int j = 0; j < 2 * P0 + L - 2; ++j) w[j] = s_b[(j0 + j) * T1 * T2 + l];
        },
        [&](int l, int k, float lo, float) {
          const int c = l % T2, k1 = l / T2;
          const int g0 = o0 + k, g1 = o1 + k1, g2 = o2 + c;
          if (g0 < m0 && g1 < m1 && g2 < m2) gst(dst + g0 * t.so[0] + g1 * t.so[1] + g2, lo);
        });
  }
}

// Output tile (U0, U1, U2) (even) of one synthesis level; z window J_k = U_k/2 + L/2 - 1 starting
// at U_k c_k / 2: output i = U_k c_k + 2q + e reads z[U_k c_k/2 + q + L/2 - 1 - j] with tap
// h[2j + e], j < L/2 (the index i + L - 2 - 2k of the left inverse).
template <int D, int L, int U0, int U1, int U2, int NT>
__global__ void __launch_bounds__(NT) k_sym_up(SymTask t, Filter f) {
  constexpr int H = L / 2;
  constexpr int J0 = D >= 3 ? U0 / 2 + H - 1 : 1;
  constexpr int J1 = D >= 2 ? U1 / 2 + H - 1 : 1;
  constexpr int J2 = U2 / 2 + H - 1;
  constexpr int J2P = J2 | 1;
  constexpr int U2P = D == 2 ? U2 + 4 : U2 + 1;  // 2-D: rows of whole 16-byte groups for the last pass
  constexpr int NZ = J0 * J1 * J2;
  constexpr int P2 = 4, P1 = D >= 3 ? 2 : 4, P0 = 2;
  static_assert(U2 % (2 * P2) == 0 && (D < 2 || U1 % (2 * P1) == 0) && (D < 3 || U0 % (2 * P0) == 0), "tile shape");
  __shared__ float s_z[J0 * J1 * J2P];
  __shared__ float s_a[J0 * J1 * U2P];
  __shared__ float s_b[D >= 3 ? J0 * U1 * U2 : 1];
  __shared__ int s_x0[J0], s_x1[J1], s_x2[J2];

  const int wg = blockIdx.x;
  const int inst = wg / t.tiles_per_inst;
  int rem = wg - inst * t.tiles_per_inst;
  const int c2 = rem % t.nt[2];
  rem /= t.nt[2];
  const int c1 = rem % t.nt[1], c0 = rem / t.nt[1];
  const float* z = t.in + inst * t.bs_in;
  // may equal out: each output reads only its own slot; null (the extended synthesis of the
  // transposed operator): no alpha term
  const bool has_same = t.same != nullptr;
  const float* same = has_same ? t.same + inst * t.bs_same : nullptr;
  float* out = t.out + inst * t.bs_out;
  const int l0 = t.ni[0], l1 = t.ni[1], l2 = t.ni[2];
  const int m0 = t.no[0], m1 = t.no[1], m2 = t.no[2];
  const int o0 = U0 * c0, o1 = U1 * c1, o2 = U2 * c2;  // first output of the tile on each axis
  const int zs = t.zshift;
  const int r0 = o0 / 2 - zs, r1 = o1 / 2 - zs, r2 = o2 / 2 - zs;  // first z sample of the window

  // 2-D tiles whose columns lie inside a row length divisible by 4: the last pass gives each lane
  // four adjacent columns of one output row pair (16-byte LDS reads, loads and stores), and the
  // lane's `same` values are loaded first so that their latency overlaps the staging of z
  constexpr int C4 = U2 / 4, NT2 = C4 * (U1 / 2);
  const int so0 = t.so[0], so1 = t.so[1];
  const bool fast = D == 2 && ((so1 | t.bs_out | t.bs_same) & 3) == 0 && o2 + U2 <= m2;
  float4 xs0 = make_float4(0.f, 0.f, 0.f, 0.f), xs1 = xs0;
  if constexpr (D == 2) {
    static_assert(NT2 <= NT, "one task per lane");
    if (fast && has_same && threadIdx.x < NT2) {
      const int c4 = threadIdx.x % C4, ch = threadIdx.x / C4;
      const int g1 = o1 + 2 * ch, g2 = o2 + 4 * c4;
      if (g1 < m1) xs0 = gld4(same + g1 * so1 + g2);
      if (g1 + 1 < m1) xs1 = gld4(same + (g1 + 1) * so1 + g2);
    }
  }

  auto inz = [](int k, int l) { return k >= 0 && k < l; };
  for (int i = threadIdx.x; i < J2; i += NT) s_x2[i] = inz(r2 + i, l2) ? r2 + i : -1;
  for (int i = threadIdx.x; i < J1; i += NT) s_x1[i] = D >= 2 ? (inz(r1 + i, l1) ? (r1 + i) * t.si[1] : -1) : 0;
  for (int i = threadIdx.x; i < J0; i += NT) s_x0[i] = D >= 3 ? (inz(r0 + i, l0) ? (r0 + i) * t.si[0] : -1) : 0;
  __syncthreads();
  gather_to_lds<NT, 4>(
      NZ,
      [&](int e) {
        const int x2 = s_x2[e % J2], r = e / J2;
        const int x1 = s_x1[r % J1], x0 = s_x0[r / J1];
        return (x0 >= 0 && x1 >= 0 && x2 >= 0) ? gld(z + x0 + x1 + x2) : 0.f;
      },
      [&](int e, float v) { s_z[(e / J2) * J2P + e % J2] = v; });
  __syncthreads();

  // axis 2: (J0 J1 rows, J2) -> (J0 J1 rows, U2)
  synthesis_pass<L, P2, false, true, NT>(
      J0 * J1, U2 / 2 / P2, f,
      [&](int l, int j0, float* lo, float*) {
#pragma unroll
        for (int j = 0; j < P2 + H - 1; ++j) lo[j] = s_z[l * J2P + j0 + j];
      },
      [&](int l, int p, float e0, float e1) {
        s_a[l * U2P + p] = e0;
        s_a[l * U2P + p + 1] = e1;
      });
  __syncthreads();

  const float alpha = t.alpha, beta = t.beta;
  if constexpr (D == 1) {
    for (int p = threadIdx.x; p < U2; p += NT) {
      const int g2 = o2 + p;
      if (g2 < m2) gst(out + g2, fmaf(alpha, has_same ? gld(same + g2) : 0.f, beta * s_a[p]));
    }
  } else if constexpr (D == 2) {
    if (fast) {
      if (threadIdx.x < NT2) {
        // the arithmetic of synthesis_pass per output (oldest window sample first)
        const int c4 = threadIdx.x % C4, ch = threadIdx.x / C4;
        float4 lo[H];
#pragma unroll
        for (int j = 0; j < H; ++j) lo[j] = *reinterpret_cast<const float4*>(s_a + (ch + j) * U2P + 4 * c4);
        float4 e0 = make_float4(0.f, 0.f, 0.f, 0.f), e1 = e0;
#pragma unroll
        for (int j = H - 1; j >= 0; --j) {
          const float4 v = lo[H - 1 - j];
          e0.x = fmaf(f.h[2 * j], v.x, e0.x); e1.x = fmaf(f.h[2 * j + 1], v.x, e1.x);
          e0.y = fmaf(f.h[2 * j], v.y, e0.y); e1.y = fmaf(f.h[2 * j + 1], v.y, e1.y);
          e0.z = fmaf(f.h[2 * j], v.z, e0.z); e1.z = fmaf(f.h[2 * j + 1], v.z, e1.z);
          e0.w = fmaf(f.h[2 * j], v.w, e0.w); e1.w = fmaf(f.h[2 * j + 1], v.w, e1.w);
        }
        const int g1 = o1 + 2 * ch, g2 = o2 + 4 * c4;
        if (g1 < m1)
          gst4(out + g1 * so1 + g2, make_float4(fmaf(alpha, xs0.x, beta * e0.x), fmaf(alpha, xs0.y, beta * e0.y),
                                               fmaf(alpha, xs0.z, beta * e0.z), fmaf(alpha, xs0.w, beta * e0.w)));
        if (g1 + 1 < m1)
          gst4(out + (g1 + 1) * so1 + g2, make_float4(fmaf(alpha, xs1.x, beta * e1.x), fmaf(alpha, xs1.y, beta * e1.y),
                                                     fmaf(alpha, xs1.z, beta * e1.z), fmaf(alpha, xs1.w, beta * e1.w)));
      }
      return;
    }
    synthesis_pass<L, P1, false, true, NT>(
        U2, U1 / 2 / P1, f,
        [&](int c, int j0, float* lo, float*) {
#pragma unroll
          for (int j = 0; j < P1 + H - 1; ++j) lo[j] = s_a[(j0 + j) * U2P + c];
        },
        [&](int c, int p, float e0, float e1) {
          const int g1 = o1 + p, g2 = o2 + c;
          if (g2 < m2) {
            if (g1 < m1) {
              const int o = g1 * so1 + g2;
              gst(out + o, fmaf(alpha, has_same ? gld(same + o) : 0.f, beta * e0));
            }
            if (g1 + 1 < m1) {
              const int o = (g1 + 1) * so1 + g2;
              gst(out + o, fmaf(alpha, has_same ? gld(same + o) : 0.f, beta * e1));
            }
          }
        });
  } else {
    // axis 1: lines (i0, c): (J0, J1, U2) -> (J0, U1, U2)
    synthesis_pass<L, P1, false, true, NT>(
        J0 * U2, U1 / 2 / P1, f,
        [&](int l, int j0, float* lo, float*) {
          const int c = l % U2, i0 = l / U2;
#pragma unroll
          for (int j = 0; j < P1 + H - 1; ++j) lo[j] = s_a[(i0 * J1 + j0 + j) * U2P + c];
        },
        [&](int l, int p, float e0, float e1) {
          const int c = l % U2, i0 = l / U2;
          s_b[(i0 * U1 + p) * U2 + c] = e0;
          s_b[(i0 * U1 + p + 1) * U2 + c] = e1;
        });
    __syncthreads();
    // axis 0: lines (p1, c): (J0, U1, U2) -> (U0, U1, U2)
    synthesis_pass<L, P0, false, true, NT>(
        U1 * U2, U0 / 2 / P0, f,
        [&](int l, int j0, float* lo, float*) {
#pragma unroll
          for (int j = 0; j < P0 + H - 1; ++j) lo[j] = s_b[(j0 + j) * U1 * U2 + l];
        },
        [&](int l, int p, float e0, float e1) {
          const int c = l % U2, p1 = l / U2;
          const int g1 = o1 + p1, g2 = o2 + c;
          if (g1 < m1 && g2 < m2) {
            const int g0 = o0 + p;
            if (g0 < m0) {
              const int o = g0 * so0 + g1 * so1 + g2;
              gst(out + o, fmaf(alpha, has_same ? gld(same + o) : 0.f, beta * e0));
            }
            if (g0 + 1 < m0) {
              const int o = (g0 + 1) * so0 + g1 * so1 + g2;
              gst(out + o, fmaf(alpha, has_same ? gld(same + o) : 0.f, beta * e1));
            }
          }
        });
  }
}

// ---------------------------------------------------------------------------------------
// Tile shapes per (dimensionality, taps).

struct SymTiles {
  int t[3];  // analysis output tile
  int u[3];  // synthesis output tile
};

constexpr int kSymThreads = 256;
// 3-D analysis tiles of up to 12 taps: 512 threads (measured faster; the 14- and 16-tap tiles keep
// 256, their registers would not fit the 512-thread bound)
constexpr int kSym3Threads = 512;

SymTiles sym_tiles(int D, int L) {
  if (D == 1) return {{1, 1, 256}, {1, 1, 512}};
  if (D == 2) return {{1, 16, 48}, {1, 32, 64}};  // 48 columns: 11 tiles cover 519 (the 1024^2 db8 level 1)
  if (L <= 4) return {{4, 8, 16}, {8, 8, 32}};
  if (L <= 8) return {{4, 4, 16}, {8, 8, 32}};
  if (L <= 12) return {{2, 4, 16}, {8, 8, 32}};
  // 14 and 16 taps: larger tiles (measured) -- the filter halo is most of a small tile
  if (L <= 14) return {{4, 4, 16}, {8, 8, 32}};
  return {{4, 8, 16}, {8, 8, 32}};
}

// Fold of the transposed operator's extended synthesis (A^T = fold o zero-padded synthesis onto
// the extension): out[j] = alpha * same[j] + beta * sum of v over every extension position that
// reflects to j, per present axis over [-(L - 2), 2 l - 1] (v's index p + (L - 2)).
// Division of a non-negative 31-bit x by a fixed d in [1, 2^31] as a multiply-high, an add and a
// shift (Granlund and Montgomery's method with a 33-bit multiplier whose top bit is the add):
// with s = ceil(log2 d) and m = floor(2^32 (2^s - d) / d) + 1, floor(x / d) = (mulhi(x, m) + x) >> s.
struct FoldDiv {
  uint32_t m, s;
};

inline FoldDiv make_fold_div(uint32_t d) {
  uint32_t s = 0;
  while ((uint64_t(1) << s) < d) ++s;
  return {(uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1), s};
}

DEVI int fold_div(int x, FoldDiv q) { return (int)((__umulhi((uint32_t)x, q.m) + (uint32_t)x) >> q.s); }

struct SymFold {
  const float* v;
  const float* same;  // may equal out
  float* out;
  int64_t bs_v, bs_out, total;  // per-instance strides; batch * outputs per instance
  int32_t sv[2], so[2];         // strides of axes 0 and 1 of v and of out / same
  int32_t no[3];                // output dims (padded)
  int32_t nl[3];                // coefficient lengths l (padded)
  int32_t ext;                  // L - 2
  int32_t present[3];           // 1 for the axes of the grid
  // Rows (j0, j1) with another image along axis 0 or 1 ("edge rows"): j_a outside the interior
  // [alo[a], ahi[a]) of axis a; every row when axis 2 is shorter than L - 1.  ce1 = edge positions
  // of axis 1, erows = edge rows per instance.
  int32_t alo[2], ahi[2], ce1, erows;
  FoldDiv dn1, dn2, drpi;       // dividers by no[1], no[2] and no[0] * no[1]
  FoldDiv dce1, derows;         // dividers by ce1 and erows
  int32_t gmain;                // work-groups of the interior rows (set at the launch)
  float alpha, beta;
};

// Images of j along one axis.  For n >= L - 1 the extension range holds at most one position of
// each family: j itself, -1 - j near the start, 2n - 1 - j near the end (`simple`); shorter axes
// enumerate both families.
template <class F>
DEVI void visit_images(int j, int n, int lo, int hi, bool simple, F f) {
  if (simple) {
    f(j);
    if (-1 - j >= lo) f(-1 - j);
    if (2 * n - 1 - j <= hi) f(2 * n - 1 - j);
  } else {
    for_images(j, n, lo, hi, f);
  }
}

// Outputs per work-group pass of the fold: four per thread.
constexpr int kFoldPass = 4 * 256;

// Rows of the fold per work-group pass: whole output rows (instance, j0, j1) filling up to
// kFoldPass outputs, at least one (long rows are walked in passes).
inline __host__ __device__ int fold_rows_per_block(int n2) { return n2 >= kFoldPass ? 1 : kFoldPass / n2; }

// Fold on a 3-D grid (every axis extended), interior rows: rpb output rows per work-group blk of
// nblk (strided over the rows), threads along the rows' outputs; the rows an edge row has in its
// place are skipped.  Four outputs per thread and pass: every output's own position j and its
// same[] term are loaded unconditionally first (eight loads in flight), then the at most two
// axis-2 images of outputs near the ends of their row.
DEVI void fold_interior(const SymFold& F, int blk, int nblk) {
  const int n2 = F.no[2];
  const int rows = (int)(F.total / n2);  // the host keeps the row count below 2^31
  const int lo2 = -F.ext, hi2 = 2 * F.nl[2] - 1;
  const int rpi = F.no[0] * F.no[1];  // rows per instance
  const int rpb = fold_rows_per_block(n2);
  for (int64_t rb0 = (int64_t)blk * rpb; rb0 < rows; rb0 += (int64_t)nblk * rpb) {
    const int rb = (int)rb0;
    const int span = min(rpb, rows - rb) * n2;  // outputs of this block's rows
    constexpr int U = 4;
    for (int base = threadIdx.x; base < span; base += U * 256) {
      float acc[U], sv[U];
      int64_t oo[U];
      int j2s[U];
      bool st[U];
      const float* row[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = min(base + u * 256, span - 1);  // lanes past the end repeat the last output
        const int dr = fold_div(e, F.dn2), j2 = e - dr * n2;
        const int r = rb + dr;
        const int inst = fold_div(r, F.drpi), rr = r - inst * rpi;
        const int j0 = fold_div(rr, F.dn1), j1 = rr - j0 * F.no[1];
        j2s[u] = j2;
        st[u] = base + u * 256 < span && j0 >= F.alo[0] && j0 < F.ahi[0] && j1 >= F.alo[1] && j1 < F.ahi[1];
        row[u] = F.v + inst * F.bs_v + (j0 + F.ext) * F.sv[0] + (j1 + F.ext) * F.sv[1] + F.ext;
        oo[u] = inst * F.bs_out + (int64_t)j0 * F.so[0] + (int64_t)j1 * F.so[1] + j2;
        acc[u] = gld(row[u] + j2);
        sv[u] = F.same ? gld(F.same + oo[u]) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j2 = j2s[u], pa = -1 - j2, pb = 2 * n2 - 1 - j2;
        const bool ia = pa >= lo2, ib = pb <= hi2;
        if (ia || ib) {
          const float xa = gld(row[u] + (ia ? pa : j2)), xb = gld(row[u] + (ib ? pb : j2));
          acc[u] += (ia ? xa : 0.f) + (ib ? xb : 0.f);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (st[u]) gst(F.out + oo[u], fmaf(F.alpha, sv[u], F.beta * acc[u]));
    }
  }
}

// Fold, edge rows (see SymFold): every image of every output, rpb rows per work-group blk of nblk.
DEVI void fold_edges(const SymFold& F, int blk, int nblk) {
  const int n0 = F.no[0], n1 = F.no[1], n2 = F.no[2];
  const int rows = (int)(F.total / ((int64_t)n0 * n1 * n2)) * F.erows;
  int lo[3], hi[3];
  bool simple[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = F.present[a] ? -F.ext : 0;
    hi[a] = F.present[a] ? 2 * F.nl[a] - 1 : 0;
    simple[a] = !F.present[a] || F.no[a] >= F.ext + 1;
  }
  const int c0rows = (F.alo[0] + n0 - F.ahi[0]) * n1;  // edge rows with j0 at an edge of axis 0
  const int rpb = fold_rows_per_block(n2);
  for (int64_t rb0 = (int64_t)blk * rpb; rb0 < rows; rb0 += (int64_t)nblk * rpb) {
    const int rb = (int)rb0;
    const int span = min(rpb, rows - rb) * n2;
    for (int e = threadIdx.x; e < span; e += 256) {
      const int dr = fold_div(e, F.dn2), j2 = e - dr * n2;
      const int r = rb + dr;
      const int inst = fold_div(r, F.derows), s = r - inst * F.erows;
      int j0, j1;
      if (s < c0rows) {
        const int k = fold_div(s, F.dn1);
        j1 = s - k * n1;
        j0 = k < F.alo[0] ? k : F.ahi[0] + (k - F.alo[0]);
      } else {
        const int t = s - c0rows, k0 = fold_div(t, F.dce1), k1 = t - k0 * F.ce1;
        j0 = F.alo[0] + k0;
        j1 = k1 < F.alo[1] ? k1 : F.ahi[1] + (k1 - F.alo[1]);
      }
      const float* v = F.v + inst * F.bs_v;
      const int64_t o = inst * F.bs_out + (int64_t)j0 * F.so[0] + (int64_t)j1 * F.so[1] + j2;
      const int e0 = F.present[0] ? F.ext : 0, e1 = F.present[1] ? F.ext : 0, e2 = F.present[2] ? F.ext : 0;
      float acc = 0.f;
      if (simple[0] && simple[1] && simple[2]) {
        // at most three images per axis (j, -1 - j, 2n - 1 - j): all 27 combinations loaded at once,
        // a missing image replaced by j and masked
        const int jv[3] = {j0, j1, j2};
        int p[3][3];
        bool ok[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int j = jv[a], pa = -1 - j, pb = 2 * F.no[a] - 1 - j;
          ok[a][0] = true;
          ok[a][1] = F.present[a] && pa >= lo[a];
          ok[a][2] = F.present[a] && pb <= hi[a];
          p[a][0] = j;
          p[a][1] = ok[a][1] ? pa : j;
          p[a][2] = ok[a][2] ? pb : j;
        }
        float x[27];
#pragma unroll
        for (int i = 0; i < 27; ++i)
          x[i] = gld(v + (p[0][i / 9] + e0) * F.sv[0] + (p[1][i / 3 % 3] + e1) * F.sv[1] + e2 + p[2][i % 3]);
#pragma unroll
        for (int i = 0; i < 27; ++i) acc += (ok[0][i / 9] && ok[1][i / 3 % 3] && ok[2][i % 3]) ? x[i] : 0.f;
      } else {  // an axis shorter than L - 1: every image family, looped
        visit_images(j0, n0, lo[0], hi[0], simple[0], [&](int p0) {
          visit_images(j1, n1, lo[1], hi[1], simple[1], [&](int p1) {
            const float* rw = v + (p0 + e0) * F.sv[0] + (p1 + e1) * F.sv[1] + e2;
            visit_images(j2, n2, lo[2], hi[2], simple[2], [&](int p2) { acc += gld(rw + p2); });
          });
        });
      }
      gst(F.out + o, fmaf(F.alpha, F.same ? gld(F.same + o) : 0.f, F.beta * acc));
    }
  }
}

// One launch per level: work-groups [0, gmain) take the interior rows, the rest the edge rows.
__global__ void __launch_bounds__(256) k_sym_fold(SymFold F) {
  const int b = blockIdx.x;
  if (b < F.gmain)
    fold_interior(F, b, F.gmain);
  else
    fold_edges(F, b - F.gmain, gridDim.x - F.gmain);
}

// Boundary shell of the transposed operator on 1-D and 2-D grids.  On [0, n) the extended
// synthesis equals the forward synthesis S, so per axis the folded synthesis is S + C, where C adds
// at a position j the synthesis at every other image of j (nonzero only within L - 2 of an edge, or
// everywhere on an axis shorter than L - 1: the shell).  On a 2-D grid (axis 1 = rows, axis 2 =
// columns) A^T u = S1 S2 u + S1 (C2 u) + C1 ((S2 + C2) u): the forward up-level gives the first
// term; two kernels add the others, times beta.  k_sym_shell_prep evaluates, per instance,
//   Y = (S2 + C2) u  on the rows of u that the axis-1 images read (rows [0, rt) and [rb, l1)),
//   W = C2 u         at the shell columns, on every row of u;
// k_sym_shell then adds, at every shell position (j1, j2) once,
//   beta * ( [j2 in shell] sum_k1 h1(j1, k1) W[k1][j2] + [j1 in shell] sum_{p1 != j1} sum_k1 h1(p1, k1) Y[k1][j2] ).
// The synthesis at position p takes k = floor(p / 2) + i, i < L / 2, with filter index
// L - 2 + (p & 1) - 2 i; a k outside [0, l) contributes nothing.
struct SymShell {
  const float* u;
  float* out;
  float* Y;                // rows of (S2 + C2) u, pitch n[1]
  float* W;                // C2 u at the shell columns, pitch m2
  int64_t bs_u, bs_out, bs_Y, bs_W;
  int32_t su, so;          // axis-1 strides of u and out
  int32_t n[2], l[2];      // axes 1 and 2: output (level j - 1) and input (level j) lengths
  int32_t e0[2], e1[2];    // interior range [e0, e1) per axis: positions without another image
  int32_t simple[2];       // axis at least L - 1 long: at most one image of each family
  int32_t rt, rb, nY, m2;  // rows of u kept in Y: [0, rt) and [rb, l1); shell columns
  int32_t per_prep, per_shell, slab0;  // items per instance
  int32_t batch;           // instances of this launch (items below 2^31)
  int32_t D;               // 1 or 2 (a 1-D grid has one row of weight 1 along axis 1)
  int32_t ext;             // L - 2
  float beta;
};

// One synthesis sum of the line `row` (length l) at extension position p.
template <int L>
DEVI float shell_taps(const float* row, int l, int p, int stride, const Filter& f) {
  constexpr int H = L / 2;
  const int kb = floor_div(p, 2);
  const bool odd = p & 1;
  float x[H];
#pragma unroll
  for (int i = 0; i < H; ++i) x[i] = gld(row + (int64_t)min(max(kb + i, 0), l - 1) * stride);
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = kb + i;
    const float w = odd ? f.h[L - 1 - 2 * i] : f.h[L - 2 - 2 * i];
    acc = fmaf(w, (k >= 0 && k < l) ? x[i] : 0.f, acc);
  }
  return acc;
}

template <int L>
__global__ void __launch_bounds__(256) k_sym_shell_prep(SymShell S, Filter f) {
  const int lo2 = -S.ext, hi2 = 2 * S.l[1] - 1;
  const int total = S.batch * S.per_prep, nYc = S.nY * S.n[1];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int inst = idx / S.per_prep;
    int r = idx - inst * S.per_prep;
    const float* u = S.u + inst * S.bs_u;
    if (r < nYc) {  // Y: every image of column j2 (j2 itself included)
      const int y = r / S.n[1], j2 = r - y * S.n[1];
      const int k1 = y < S.rt ? y : S.rb + (y - S.rt);
      const float* row = u + (int64_t)k1 * S.su;
      float acc = 0.f;
      visit_images(j2, S.n[1], lo2, hi2, S.simple[1], [&](int p2) { acc += shell_taps<L>(row, S.l[1], p2, 1, f); });
      gst(S.Y + inst * S.bs_Y + r, acc);
    } else {        // W: the images of shell column j2 other than j2
      r -= nYc;
      const int k1 = r / S.m2, e = r - k1 * S.m2;
      const int j2 = e < S.e0[1] ? e : S.e1[1] + (e - S.e0[1]);
      const float* row = u + (int64_t)k1 * S.su;
      float acc = 0.f;
      visit_images(j2, S.n[1], lo2, hi2, S.simple[1], [&](int p2) {
        if (p2 != j2) acc += shell_taps<L>(row, S.l[1], p2, 1, f);
      });
      gst(S.W + inst * S.bs_W + r, acc);
    }
  }
}

template <int L, int D>
__global__ void __launch_bounds__(256) k_sym_shell(SymShell S, Filter f) {
  const int lo1 = -S.ext, hi1 = 2 * S.l[0] - 1;
  const int total = S.batch * S.per_shell;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int inst = idx / S.per_shell;
    int r = idx - inst * S.per_shell;
    int j1, j2;
    bool edge1, edge2;
    if (r < S.slab0) {  // axis-1 coordinate in the shell
      const int t1 = r / S.n[1];
      j2 = r - t1 * S.n[1];
      j1 = t1 < S.e0[0] ? t1 : S.e1[0] + (t1 - S.e0[0]);
      edge1 = true;
      edge2 = j2 < S.e0[1] || j2 >= S.e1[1];
    } else {            // interior axis-1 coordinate, axis-2 coordinate in the shell
      r -= S.slab0;
      const int t1 = r / S.m2, t2 = r - t1 * S.m2;
      j1 = S.e0[0] + t1;
      j2 = t2 < S.e0[1] ? t2 : S.e1[1] + (t2 - S.e0[1]);
      edge1 = false;
      edge2 = true;
    }
    float* o = S.out + (int64_t)inst * S.bs_out + (int64_t)j1 * S.so + j2;
    float corr = 0.f;
    if (edge2) {  // S1 (C2 u) at column j2
      const int e = j2 < S.e0[1] ? j2 : S.e0[1] + (j2 - S.e1[1]);
      const float* col = S.W + inst * S.bs_W + e;
      corr = D == 2 ? shell_taps<L>(col, S.l[0], j1, S.m2, f) : gld(col);
    }
    if (D == 2 && edge1) {  // C1 ((S2 + C2) u): the images of row j1 other than j1
      const float* Yc = S.Y + inst * S.bs_Y + j2;
      visit_images(j1, S.n[0], lo1, hi1, S.simple[0], [&](int p1) {
        if (p1 == j1) return;
        constexpr int H = L / 2;
        const int kb = floor_div(p1, 2);
        const bool odd = p1 & 1;
        float x[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
          const int k = min(max(kb + i, 0), S.l[0] - 1);
          const int y = k < S.rt ? k : (k >= S.rb ? S.rt + (k - S.rb) : 0);  // rows p1 reads are kept
          x[i] = gld(Yc + (int64_t)y * S.n[1]);
        }
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < H; ++i) {
          const int k = kb + i;
          const float w = odd ? f.h[L - 1 - 2 * i] : f.h[L - 2 - 2 * i];
          acc = fmaf(w, (k >= 0 && k < S.l[0]) ? x[i] : 0.f, acc);
        }
        corr += acc;
      });
    }
    gst(o, fmaf(S.beta, corr, gld(o)));
  }
}

hipError_t launch_sym_shell(int L, const SymShell& S, bool prep, unsigned grid, const Filter& f, hipStream_t s) {
  const bool two = S.D == 2;
  switch (L) {
#define ES_SHELL_CASE(LL)                                                                   \
  case LL:                                                                                  \
    if (prep) hipLaunchKernelGGL((k_sym_shell_prep<LL>), dim3(grid), dim3(256), 0, s, S, f); \
    else if (two) hipLaunchKernelGGL((k_sym_shell<LL, 2>), dim3(grid), dim3(256), 0, s, S, f); \
    else hipLaunchKernelGGL((k_sym_shell<LL, 1>), dim3(grid), dim3(256), 0, s, S, f);       \
    break;
    ES_SHELL_CASE(2) ES_SHELL_CASE(4) ES_SHELL_CASE(6) ES_SHELL_CASE(8)
    ES_SHELL_CASE(10) ES_SHELL_CASE(12) ES_SHELL_CASE(14) ES_SHELL_CASE(16)
#undef ES_SHELL_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int D, int L, bool ZX>
hipError_t launch_sym_level(bool up, const SymTask& t, int64_t grid, const Filter& f, hipStream_t s) {
  if constexpr (D == 1) {
    if (up) hipLaunchKernelGGL((k_sym_up<1, L, 1, 1, 512, kSymThreads>), dim3((unsigned)grid), dim3(kSymThreads), 0, s, t, f);
    else hipLaunchKernelGGL((k_sym_down<1, L, 1, 1, 256, kSymThreads, ZX>), dim3((unsigned)grid), dim3(kSymThreads), 0, s, t, f);
  } else if constexpr (D == 2) {
    if (up) hipLaunchKernelGGL((k_sym_up<2, L, 1, 32, 64, kSymThreads>), dim3((unsigned)grid), dim3(kSymThreads), 0, s, t, f);
    else hipLaunchKernelGGL((k_sym_down<2, L, 1, 16, 48, kSymThreads, ZX>), dim3((unsigned)grid), dim3(kSymThreads), 0, s, t, f);
  } else {
    if (up) {
      hipLaunchKernelGGL((k_sym_up<3, L, 8, 8, 32, kSymThreads>), dim3((unsigned)grid), dim3(kSymThreads), 0, s, t, f);
    } else if constexpr (L <= 4) {
      hipLaunchKernelGGL((k_sym_down<3, L, 4, 8, 16, kSym3Threads, ZX>), dim3((unsigned)grid), dim3(kSym3Threads), 0, s, t, f);
    } else if constexpr (L <= 8) {
      hipLaunchKernelGGL((k_sym_down<3, L, 4, 4, 16, kSym3Threads, ZX>), dim3((unsigned)grid), dim3(kSym3Threads), 0, s, t, f);
    } else if constexpr (L <= 12) {
      hipLaunchKernelGGL((k_sym_down<3, L, 2, 4, 16, kSym3Threads, ZX>), dim3((unsigned)grid), dim3(kSym3Threads), 0, s, t, f);
    } else if constexpr (L <= 14) {
      hipLaunchKernelGGL((k_sym_down<3, L, 4, 4, 16, kSymThreads, ZX>), dim3((unsigned)grid), dim3(kSymThreads), 0, s, t, f);
    } else {
      hipLaunchKernelGGL((k_sym_down<3, L, 4, 8, 16, kSymThreads, ZX>), dim3((unsigned)grid), dim3(kSymThreads), 0, s, t, f);
    }
  }
  return hipGetLastError();
}

template <int L>
hipError_t launch_sym_taps(int D, bool up, bool zx, const SymTask& t, int64_t grid, const Filter& f, hipStream_t s) {
  if (zx) {
    if (D == 1) return launch_sym_level<1, L, true>(up, t, grid, f, s);
    if (D == 2) return launch_sym_level<2, L, true>(up, t, grid, f, s);
    return launch_sym_level<3, L, true>(up, t, grid, f, s);
  }
  if (D == 1) return launch_sym_level<1, L, false>(up, t, grid, f, s);
  if (D == 2) return launch_sym_level<2, L, false>(up, t, grid, f, s);
  return launch_sym_level<3, L, false>(up, t, grid, f, s);
}

hipError_t launch_sym(int D, int L, bool up, bool zx, const SymTask& t, int64_t grid, const Filter& f, hipStream_t s) {
  switch (L) {
    case 2: return launch_sym_taps<2>(D, up, zx, t, grid, f, s);
    case 4: return launch_sym_taps<4>(D, up, zx, t, grid, f, s);
    case 6: return launch_sym_taps<6>(D, up, zx, t, grid, f, s);
    case 8: return launch_sym_taps<8>(D, up, zx, t, grid, f, s);
    case 10: return launch_sym_taps<10>(D, up, zx, t, grid, f, s);
    case 12: return launch_sym_taps<12>(D, up, zx, t, grid, f, s);
    case 14: return launch_sym_taps<14>(D, up, zx, t, grid, f, s);
    default: return launch_sym_taps<16>(D, up, zx, t, grid, f, s);
  }
}

// ---------------------------------------------------------------------------------------
// Host: geometry, level lengths, workspace and the launch sequence.

constexpr int kSymMaxLevels = 30;

struct SymGeo {
  int D, L, m;
  double s;
  int dims[kSymMaxLevels + 1][3];  // padded dims of a_0 (= x) .. a_m
  int64_t size(int i) const { return (int64_t)dims[i][0] * dims[i][1] * dims[i][2]; }
  // Row pitch of level i: the caller's arrays (level 0, and y) are contiguous; the level arrays in
  // the workspace start every row at a multiple of 4 floats, so that interior tiles of every level
  // take the 16-byte paths.
  int pitch(int i) const { return i == 0 ? dims[0][2] : (dims[i][2] + 3) & ~3; }
  int64_t stored(int i) const { return (int64_t)dims[i][0] * dims[i][1] * pitch(i); }
};

es_status sym_einval(const char* fmt, long long a = 0, long long b = 0) {
  char buf[200];
  snprintf(buf, sizeof buf, fmt, a, b);
  return report_error(ES_EINVAL, buf);
}

int64_t sym_len(int64_t n, int L) { return (n + L - 1) / 2; }

es_status sym_geo(int ndim, const int64_t* shape, int order, int levels, double s, SymGeo* g) {
  if (ndim < 1 || ndim > 3) return sym_einval("ndim must be 1, 2 or 3 (got %lld)", ndim);
  if (!shape) return sym_einval("shape is NULL");
  if (order < 1 || order > 8) return sym_einval("order must be in 1..8 (got %lld)", order);
  if (levels < 0 || levels > kSymMaxLevels) return sym_einval("levels must be in 0..%lld (got %lld)", kSymMaxLevels, levels);
  if (!std::isfinite(s)) return sym_einval("s must be finite");
  g->D = ndim;
  g->L = 2 * order;
  g->m = levels;
  g->s = s;
  int64_t n[3] = {1, 1, 1};
  for (int k = 0; k < ndim; ++k) {
    if (shape[k] < 1 || shape[k] > (1ll << 30)) return sym_einval("shape[%lld] must be in 1..2^30 (got %lld)", k, shape[k]);
    n[3 - ndim + k] = shape[k];
  }
  for (int i = 0; i <= levels; ++i) {
    int64_t prod = 1;
    for (int a = 0; a < 3; ++a) {
      const int64_t v = i == 0 || a < 3 - ndim ? n[a] : sym_len(g->dims[i - 1][a], g->L);
      g->dims[i][a] = (int)v;
      prod *= v;
    }
    if (prod > 0x7fffffffll || g->stored(i) > 0x7fffffffll)
      return sym_einval("level %lld holds more than 2^31-1 elements per instance", i);
  }
  return ES_OK;
}

int64_t align64f(int64_t v) { return (v + 63) & ~(int64_t)63; }


bool sym_filter(int L, Filter* f) {
  double h[kMaxTaps];
  if (!daubechies_filter(L / 2, h)) return false;
  for (int t = 0; t < kMaxTaps; ++t) f->h[t] = f->g[t] = 0.f;
  for (int t = 0; t < L; ++t) {
    f->h[t] = (float)h[t];
    f->g[t] = (float)((t & 1) ? -h[L - 1 - t] : h[L - 1 - t]);
  }
  return true;
}

struct SymLaunch {
  int kind;  // 0 analysis level, 1 synthesis level, 2 fold, 3 boundary shell (transposed operator)
  bool zx;   // analysis with zero extension (S_a^T)
  SymTask t;
  SymFold fold;
  SymShell shell;
  int64_t grid;
};

// Boundary shell of the transposed up-level j on 1-D and 2-D grids (see k_sym_shell): lengths,
// interior ranges, kept rows and per-instance item counts; scratch = Y then W (floats).
SymShell sym_shell(const SymGeo& g, int j, int64_t batch, const float* u, float* out, float beta, float* scratch) {
  SymShell S{};
  S.u = u;
  S.out = out;
  S.bs_u = g.stored(j);
  S.bs_out = g.stored(j - 1);
  S.su = g.pitch(j);
  S.so = g.pitch(j - 1);
  S.D = g.D;
  S.ext = g.L - 2;
  S.beta = beta;
  const int H = g.L / 2;
  for (int a = 0; a < 2; ++a) {
    const int ax = a + 1;  // grid axes 1 and 2
    S.n[a] = g.dims[j - 1][ax];
    S.l[a] = g.dims[j][ax];
    const bool present = ax >= 3 - g.D;
    if (!present) {  // one position, no other image
      S.e0[a] = 0;
      S.e1[a] = 1;
      S.simple[a] = 1;
      continue;
    }
    const int n = S.n[a], l = S.l[a];
    S.simple[a] = n >= g.L - 1;
    if (S.simple[a]) {
      // -1 - j lies in the extension for j <= L - 3, 2n - 1 - j for j >= 2n - 2l
      S.e0[a] = g.L - 2;
      S.e1[a] = std::max(S.e0[a], std::min(n, 2 * n - 2 * l));
    } else {
      S.e0[a] = S.e1[a] = 0;  // every position may have several images
    }
  }
  if (g.D == 2) {
    // rows of u the axis-1 images read: -(L-2) <= p1 <= -1 reads k1 <= L/2 - 2, n1 <= p1 reads
    // k1 >= n1 / 2; a short axis keeps every row
    const int l1 = S.l[0];
    S.rt = S.simple[0] ? std::min(l1, H - 1) : l1;
    S.rb = S.simple[0] ? std::max(S.rt, std::min(l1, S.n[0] / 2)) : l1;
    S.nY = S.rt + (l1 - S.rb);
  } else {
    S.rt = S.rb = 1;
    S.nY = 0;
  }
  S.m2 = S.n[1] - (S.e1[1] - S.e0[1]);
  const int in1 = S.e1[0] - S.e0[0];
  S.slab0 = (S.n[0] - in1) * S.n[1];
  S.per_shell = S.slab0 + in1 * S.m2;
  S.per_prep = S.nY * S.n[1] + S.l[0] * S.m2;
  S.bs_Y = (int64_t)S.nY * S.n[1];
  S.bs_W = (int64_t)S.l[0] * S.m2;
  if (scratch) {
    S.Y = scratch;
    S.W = scratch + align64f(batch * S.bs_Y);
  }
  S.batch = (int32_t)std::min<int64_t>(batch, 0x7fffffff);
  return S;
}

// Scratch floats of the shell of level j (0 where the level has no shell pass).
int64_t sym_shell_floats(const SymGeo& g, int j, int64_t batch) {
  const SymShell S = sym_shell(g, j, batch, nullptr, nullptr, 0.f, nullptr);
  return align64f(batch * S.bs_Y) + align64f(batch * S.bs_W);
}

// Sets the tile counts of `t` for output dims `no` and tile `tile`; returns the grid.
int64_t sym_tiling(SymTask& t, const int tile[3], int64_t batch) {
  int64_t per = 1;
  for (int a = 0; a < 3; ++a) {
    t.nt[a] = (t.no[a] + tile[a] - 1) / tile[a];
    per *= t.nt[a];
  }
  t.tiles_per_inst = (int32_t)per;
  return per * batch;
}

// The transposed operator's extended synthesis of level i: every present axis runs over the
// extension positions -(L - 2) .. 2 l_i - 1, rows padded to a multiple of 4 floats.
struct ExtDims {
  int d[3], pitch;
  int64_t stored() const { return (int64_t)d[0] * d[1] * pitch; }
};
ExtDims ext_dims(const SymGeo& g, int i) {
  ExtDims e;
  for (int a = 0; a < 3; ++a) e.d[a] = a < 3 - g.D ? 1 : 2 * g.dims[i][a] + g.L - 2;
  e.pitch = (e.d[2] + 3) & ~3;
  return e;
}

// Floats of workspace: a_1 .. a_{m-1} of every instance (each level 256-byte aligned), and for
// the transposed operator after them the extended synthesis of the finest level (3-D grids) or the
// boundary-shell scratch of the largest level (1-D and 2-D grids).
int64_t sym_ws_floats(const SymGeo& g, int64_t batch, bool transpose) {
  int64_t tot = 0;
  for (int i = 1; i < g.m; ++i) tot += align64f(batch * g.stored(i));
  if (transpose && g.m >= 2 && g.D == 3) tot += align64f(batch * ext_dims(g, 1).stored());
  if (transpose && g.D <= 2) {  // the boundary-shell scratch, one level at a time
    int64_t sh = 0;
    for (int j = 1; j < g.m; ++j) sh = std::max(sh, sym_shell_floats(g, j, batch));
    tot += sh;
  }
  return tot;
}

// Launch sequence.  Forward (x -> y = W^{-1} D W x): a_i = A a_{i-1}, then
// z_{j-1} = c_{j-1} a_{j-1} + S_a z_j (y = w_1 x + S_a z_1), z over a in place.
// Transposed (x -> y = (W^{-1} D W)^T x = w_1 x + sum_i c_i (A^T)^i (S_a^T)^i x): b_i = S_a^T b_{i-1}
// (zero-extended analysis), then u_{j-1} = c_{j-1} b_{j-1} + A^T u_j with A^T = fold o extended
// synthesis (y = w_1 x + A^T u_1).
es_status sym_schedule(const SymGeo& g, int64_t batch, const float* x, float* y, float* ws, bool transpose,
                       std::vector<SymLaunch>* out) {
  out->clear();
  const SymTiles tl = sym_tiles(g.D, g.L);
  std::vector<float*> lev(g.m + 1, nullptr);
  lev[0] = const_cast<float*>(x);
  int64_t off = 0;
  for (int i = 1; i < g.m; ++i) {
    lev[i] = ws + off;
    off += align64f(batch * g.stored(i));
  }
  float* vext = ws + off;  // transposed operator only: extended level (3-D) or shell scratch
  auto strides = [&](int i, int32_t st[2]) {
    st[1] = g.pitch(i);
    st[0] = g.dims[i][1] * g.pitch(i);
  };
  // weights: w[i] of detail level i (1..m), w[m] = 1 = approximation weight
  std::vector<double> w(g.m + 1, 1.0);
  for (int i = 1; i <= g.m; ++i) w[i] = std::exp2(-2.0 * g.s * (double)(g.m - i));
  for (int i = 1; i < g.m; ++i) {
    SymLaunch l{};
    l.kind = 0;
    l.zx = transpose;
    l.t.in = lev[i - 1];
    l.t.out = lev[i];
    l.t.same = nullptr;
    l.t.bs_in = g.stored(i - 1);
    l.t.bs_out = g.stored(i);
    for (int a = 0; a < 3; ++a) {
      l.t.ni[a] = g.dims[i - 1][a];
      l.t.no[a] = g.dims[i][a];
    }
    strides(i - 1, l.t.si);
    strides(i, l.t.so);
    l.grid = sym_tiling(l.t, tl.t, batch);
    out->push_back(l);
  }
  for (int j = g.m - 1; j >= 1; --j) {
    const double alpha = j == 1 ? w[1] : w[j] - w[j - 1];
    const double beta = j == g.m - 1 ? w[g.m] - w[g.m - 1] : 1.0;
    float* dst = j == 1 ? y : lev[j - 1];
    if (!transpose) {
      // z_{j-1} = c_{j-1} a_{j-1} + S_a z_j  (y = w_1 x + S_a z_1); z_{m-1} = c_{m-1} a_{m-1}
      SymLaunch l{};
      l.kind = 1;
      l.t.in = lev[j];
      l.t.same = lev[j - 1];
      l.t.out = dst;
      l.t.bs_in = g.stored(j);
      l.t.bs_same = g.stored(j - 1);
      l.t.bs_out = g.stored(j - 1);  // y has the layout of x
      l.t.alpha = (float)alpha;
      l.t.beta = (float)beta;
      for (int a = 0; a < 3; ++a) {
        l.t.ni[a] = g.dims[j][a];
        l.t.no[a] = g.dims[j - 1][a];
      }
      strides(j, l.t.si);
      strides(j - 1, l.t.so);
      l.grid = sym_tiling(l.t, tl.u, batch);
      out->push_back(l);
      continue;
    }
    if (g.D <= 2) {
      // transposed, 1-D and 2-D: the forward up-level (u_{j-1} = c_{j-1} b_{j-1} + beta S u_j on
      // [0, n)), then the boundary shell adds beta times the extension images
      SymLaunch l{};
      l.kind = 1;
      l.t.in = lev[j];
      l.t.same = lev[j - 1];
      l.t.out = dst;
      l.t.bs_in = g.stored(j);
      l.t.bs_same = g.stored(j - 1);
      l.t.bs_out = g.stored(j - 1);
      l.t.alpha = (float)alpha;
      l.t.beta = (float)beta;
      for (int a = 0; a < 3; ++a) {
        l.t.ni[a] = g.dims[j][a];
        l.t.no[a] = g.dims[j - 1][a];
      }
      strides(j, l.t.si);
      strides(j - 1, l.t.so);
      l.grid = sym_tiling(l.t, tl.u, batch);
      out->push_back(l);
      SymLaunch sl{};
      sl.kind = 3;
      sl.shell = sym_shell(g, j, batch, lev[j], dst, (float)beta, vext);
      sl.grid = 0;  // sized at the launch
      out->push_back(sl);
      continue;
    }
    // transposed, 3-D: v = beta * (zero-padded synthesis of u_j onto the extension), then
    // u_{j-1} = c_{j-1} b_{j-1} + fold(v)
    const ExtDims E = ext_dims(g, j);
    SymLaunch l{};
    l.kind = 1;
    l.t.in = lev[j];
    l.t.same = nullptr;
    l.t.out = vext;
    l.t.bs_in = g.stored(j);
    l.t.bs_out = E.stored();
    l.t.zshift = g.L / 2 - 1;
    l.t.alpha = 0.f;
    l.t.beta = (float)beta;
    for (int a = 0; a < 3; ++a) {
      l.t.ni[a] = g.dims[j][a];
      l.t.no[a] = E.d[a];
    }
    strides(j, l.t.si);
    l.t.so[1] = E.pitch;
    l.t.so[0] = E.d[1] * E.pitch;
    l.grid = sym_tiling(l.t, tl.u, batch);
    out->push_back(l);
    SymLaunch fl{};
    fl.kind = 2;
    SymFold& F = fl.fold;
    F.v = vext;
    F.same = lev[j - 1];
    F.out = dst;
    F.bs_v = E.stored();
    F.bs_out = g.stored(j - 1);
    F.total = batch * g.size(j - 1);
    F.sv[1] = E.pitch;
    F.sv[0] = E.d[1] * E.pitch;
    strides(j - 1, F.so);
    for (int a = 0; a < 3; ++a) {
      F.no[a] = g.dims[j - 1][a];
      F.nl[a] = g.dims[j][a];
      F.present[a] = a >= 3 - g.D;
    }
    F.ext = g.L - 2;
    // interior of axes 0 and 1: no image at -1 - j (j >= L - 2) nor at 2n - 1 - j (j < 2n - 2l)
    for (int a = 0; a < 2; ++a) {
      const int n = F.no[a], lo = std::min(F.ext, n);
      const bool simple = n >= F.ext + 1;
      F.alo[a] = simple ? lo : n;
      F.ahi[a] = simple ? std::max(std::min(2 * n - 2 * F.nl[a], n), lo) : n;
    }
    if (F.no[2] < F.ext + 1) F.alo[0] = F.ahi[0] = F.no[0];  // short axis 2: every row is an edge row
    F.ce1 = F.alo[1] + F.no[1] - F.ahi[1];
    F.erows = (F.alo[0] + F.no[0] - F.ahi[0]) * F.no[1] + (F.ahi[0] - F.alo[0]) * F.ce1;
    F.dn1 = make_fold_div(F.no[1]);
    F.dn2 = make_fold_div(F.no[2]);
    F.drpi = make_fold_div(F.no[0] * F.no[1]);
    F.dce1 = make_fold_div(std::max(F.ce1, 1));
    F.derows = make_fold_div(std::max(F.erows, 1));
    F.alpha = (float)alpha;
    F.beta = 1.f;
    fl.grid = 0;  // 2-D grid, see the launch
    out->push_back(fl);
  }
  for (const SymLaunch& l : *out)
    if (l.grid > 0x7fffffffll) return sym_einval("a level needs more than 2^31-1 work-groups (%lld)", l.grid);
  return ES_OK;
}

es_status sym_run(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s, const float* x,
                  float* y, void* ws, size_t ws_bytes, void* stream, bool transpose) {
  SymGeo g;
  es_status st = sym_geo(ndim, shape, order, levels, s, &g);
  if (st != ES_OK) return st;
  if (batch < 0) return sym_einval("batch must be >= 0");
  if (batch == 0) return ES_OK;
  const int64_t N = g.size(0);
  if (N > INT64_MAX / 4 / batch) return sym_einval("batch * size overflows");
  if (transpose && g.D == 3 && g.m >= 2 && ext_dims(g, 1).stored() > 0x7fffffffll)
    return sym_einval("the extended level holds more than 2^31-1 elements per instance");
  if (transpose && g.D == 3 && batch * (N / g.dims[0][2]) > 0x7fffffffll)
    return sym_einval("the transposed operator handles at most 2^31-1 rows per call");
  if (transpose && g.D <= 2 && N > 0x3fffffffll)
    return sym_einval("the transposed operator handles at most 2^30 samples per instance on 1-D and 2-D grids");
  if (!x || !y) return sym_einval("input and output pointers must be non-NULL");
  if (((uintptr_t)x & 15) || ((uintptr_t)y & 15)) return sym_einval("input and output must be 16-byte aligned");
  const size_t io = (size_t)(batch * N) * sizeof(float);
  const char *px = (const char*)x, *py = (const char*)y;
  if (px < py + io && py < px + io) return sym_einval("input and output overlap");
  const size_t need = (size_t)sym_ws_floats(g, batch, transpose) * sizeof(float);
  if (need) {
    if (!ws) return report_error(ES_EWORKSPACE, "workspace required (es_sym_workspace_bytes), got NULL");
    if (ws_bytes < need) {
      char buf[160];
      snprintf(buf, sizeof buf, "workspace of %zu bytes required, got %zu", need, ws_bytes);
      return report_error(ES_EWORKSPACE, buf);
    }
    if ((uintptr_t)ws & 255) return sym_einval("workspace must be 256-byte aligned");
    const char* pw = (const char*)ws;
    if ((pw < px + io && px < pw + need) || (pw < py + io && py < pw + need))
      return sym_einval("workspace overlaps input or output");
  }
  std::vector<SymLaunch> seq;
  if ((st = sym_schedule(g, batch, x, y, (float*)ws, transpose, &seq)) != ES_OK) return st;
  Filter f;
  if (!sym_filter(g.L, &f)) return report_error(ES_EUNSUPPORTED, "filter derivation failed");
  if ((st = device_check()) != ES_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  hipError_t he;
  if (g.m <= 1) {  // every weight is 1: the identity
    if ((he = launch_copy_any(x, y, batch * N, hs)) != hipSuccess) return report_error(ES_EDEVICE, hipGetErrorString(he));
    return ES_OK;
  }
  for (const SymLaunch& l : seq) {
    if (l.kind == 2) {
      // interior rows and edge rows (disjoint outputs) in one launch: whole output rows per
      // work-group (at most 2^20 groups per part, strided)
      SymFold F = l.fold;
      const int64_t rows = F.total / F.no[2], inst = rows / ((int64_t)F.no[0] * F.no[1]);
      const int64_t rpb = fold_rows_per_block(F.no[2]);
      const int64_t irows = inst * ((int64_t)F.no[0] * F.no[1] - F.erows), erows = inst * F.erows;
      F.gmain = irows > 0 ? (int32_t)std::min<int64_t>((rows + rpb - 1) / rpb, 1 << 20) : 0;
      const int64_t gedge = erows > 0 ? std::min<int64_t>((erows + rpb - 1) / rpb, 1 << 20) : 0;
      he = hipSuccess;
      if (F.gmain + gedge > 0) {
        hipLaunchKernelGGL(k_sym_fold, dim3((unsigned)(F.gmain + gedge)), dim3(256), 0, hs, F);
        he = hipGetLastError();
      }
    } else if (l.kind == 3) {
      // preparation, then the shell, per chunk of instances with fewer than 2^31 items (32-bit
      // indices in the kernels; each item count per instance is below 2^31 by the size check)
      he = hipSuccess;
      for (int pass = 0; pass < 2 && he == hipSuccess; ++pass) {
        const int64_t per = pass == 0 ? l.shell.per_prep : l.shell.per_shell;
        if (per == 0) continue;
        const int64_t chunk = std::max<int64_t>(1, 0x7fffffffll / per);
        for (int64_t i0 = 0; i0 < batch && he == hipSuccess; i0 += chunk) {
          SymShell S = l.shell;
          const int64_t nb = std::min(chunk, batch - i0);
          S.u += i0 * S.bs_u;
          S.out += i0 * S.bs_out;
          S.Y += i0 * S.bs_Y;
          S.W += i0 * S.bs_W;
          S.batch = (int32_t)nb;
          const unsigned grid = (unsigned)std::min<int64_t>((nb * per + 255) / 256, 16384);
          he = launch_sym_shell(g.L, S, pass == 0, grid, f, hs);
        }
      }
    } else {
      he = launch_sym(g.D, g.L, l.kind == 1, l.zx, l.t, l.grid, f, hs);
    }
    if (he != hipSuccess) return report_error(ES_EDEVICE, hipGetErrorString(he));
  }
  return ES_OK;
}

}  // namespace

}  // namespace es

using namespace es;

extern "C" {

size_t es_sym_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels) {
  SymGeo g;
  if (sym_geo(ndim, shape, order, levels, 0.0, &g) != ES_OK || batch <= 0) return 0;
  return (size_t)sym_ws_floats(g, batch, false) * sizeof(float);
}

size_t es_sym_transpose_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels) {
  SymGeo g;
  if (sym_geo(ndim, shape, order, levels, 0.0, &g) != ES_OK || batch <= 0) return 0;
  return (size_t)sym_ws_floats(g, batch, true) * sizeof(float);
}

es_status es_sym_band_lengths(int64_t n, int order, int levels, int64_t* lengths) {
  if (!lengths) return sym_einval("lengths is NULL");
  SymGeo g;
  es_status st = sym_geo(1, &n, order, levels, 0.0, &g);
  if (st != ES_OK) return st;
  for (int i = 1; i <= levels; ++i) lengths[i - 1] = g.dims[i][2];
  return ES_OK;
}

es_status es_sym_cov_apply(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                           const float* x, float* y, void* ws, size_t ws_bytes, void* stream) {
  return sym_run(ndim, shape, batch, order, levels, s, x, y, ws, ws_bytes, stream, false);
}

es_status es_sym_cov_apply_transpose(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                                     const float* y, float* x, void* ws, size_t ws_bytes, void* stream) {
  return sym_run(ndim, shape, batch, order, levels, s, y, x, ws, ws_bytes, stream, true);
}

}  // extern "C"
