// gfx950 kernels of the wavelet E_s^* / Matern-prior path.
//
// Notation: L taps, h low-pass, g[t] = (-1)^t h[L-1-t] high-pass.  One periodic analysis step
// along an axis of even length n is a[k] = sum_t h[t] x[(2k+t) mod n],
// d[k] = sum_t g[t] x[(2k+t) mod n]; synthesis is its transpose.  (Sec. 4: the discrete
// wavelet transform W and E_s^* X = W^{-1}(D (W X)).)
//
// Level kernels (one launch per level, every instance of a batch in the same launch):
//   LP_DOWN  a_i = A a_{i-1}                    low-pass only, every axis in one kernel
//   LP_UP    out = alpha*same + beta*A^T z      low-pass-only synthesis fused with the
//                                               projection-form recurrence (see api.cpp)
//   FB_DOWN  one full analysis level: 2^d bands, detail bands scaled, LL to the next level
//   FB_UP    one full synthesis level: LL + scaled detail bands -> finer approximation
// A work-group owns one output tile.  It stages the periodic input region (tile plus filter
// halo) in LDS with 16-byte loads, filters the contiguous axis first and the strided axes
// after, keeping each thread's filter window in registers, and writes the last pass straight
// to global memory with lanes along the contiguous axis (coalesced).
//
// Tail kernels: once a level's block fits in LDS, one work-group per instance runs every
// remaining level (down, scale and up) without leaving LDS.
//
// Plain kernels: one launch per 1-D pass over the whole level block, for comparison.
#include "internal.h"
#include "tiles.h"
#include "kcommon.h"
#include "lowpass.h"

namespace es {

template <int D, int L, int T0, int T1, int T2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_lp_down(TaskArgs args, Filter f) {
  __shared__ LpDownSmem<D, L, T0, T1, T2> sm;
  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  lp_down_tile<D, L, T0, T1, T2, NT, VEC>(t, wg, f, sm);
}

// ---------------------------------------------------------------------------------------
// LP_DOWN_S (2-D): a_out = A a_in, streamed along axis 1 (body: lp_down_stream).  A work-group
// owns a strip of T2 output columns and a run of R output rows; input rows are read once per
// run (plus L - 2 at its start) and filtered along axis 2 once, instead of once per tile row.
template <int L, int R, int T2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_lp_down_s(TaskArgs args, Filter f) {
  __shared__ LpDownStreamSmem<L, R, T2, kStreamRows> sm;
  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  lp_down_stream<L, R, T2, kStreamRows, NT, VEC>(t, wg, f, sm);
}

template <int D, int L, int U0, int U1, int U2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_lp_up(TaskArgs args, Filter f) {
  __shared__ LpUpSmem<D, L, U0, U1, U2> sm;
  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  lp_up_tile<D, L, U0, U1, U2, NT, VEC>(t, wg, f, sm);
}

// LP_UP with the conjugate-gradient solver's epilogue (2-D vector path): out = (alpha + gamma m)
// same + beta A^T z, and each work-group's sum of same * out (see lp_up_tile).
template <int L, int U1, int U2, int NT>
__global__ void __launch_bounds__(NT) k_lp_up_cge(TaskArgs args, Filter f) {
  __shared__ LpUpSmem<2, L, 1, U1, U2> sm;
  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  lp_up_tile<2, L, 1, U1, U2, NT, true, true>(t, wg, f, sm);
}

// ---------------------------------------------------------------------------------------
// LP_UP2 (2-D): two synthesis levels of the projection form in one kernel,
//   z1  = gamma*a1 + delta*A^T z2   (level i+1, only on the halo region this tile needs)
//   out = alpha*same + beta*A^T z1  (level i, the tile)
// so z1 never travels through HBM.  The level-(i+1) region starts HP (>= L/2-1, a multiple
// of 4) samples before the tile's half-resolution origin; the level-(i+2) region is loaded
// from a 4-aligned start OFF2 samples before the first value the synthesis reads.

template <int L, int U1, int U2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_lp_up2(TaskArgs args, Filter f) {
  constexpr int H = L / 2;
  constexpr int HP = ((H - 1) + 3) & ~3;
  constexpr int K1 = U1 / 2 + HP, K2 = U2 / 2 + HP;  // level-(i+1) region
  constexpr int Q1 = K1 / 2 + H - 1;                 // level-(i+2) rows
  constexpr int OFF2 = ((-(HP / 2) - (H - 1)) % 4 + 4) % 4;
  constexpr int Q2 = K2 / 2 + H - 1;
  constexpr int Q2P = (Q2 + OFF2 + 3) & ~3;
  constexpr int NV2 = Q2P / 4;
  constexpr int OFF1 = HP - (H - 1);                 // tile origin inside the level-(i+1) region
  constexpr int P2 = 4, P1 = 4;                      // level i+1 -> i passes
  constexpr int P2a = (K2 / 2) % 4 == 0 ? 4 : 2;     // level i+2 -> i+1 passes
  constexpr int P1a = (K1 / 2) % 4 == 0 ? 4 : 2;
  static_assert(U1 % 16 == 0 && U2 % 16 == 0, "tile sides must be multiples of 16");
  static_assert((K2 / 2) % P2a == 0 && (K1 / 2) % P1a == 0, "region must split into whole chunks");
  __shared__ __attribute__((aligned(16))) float s_z2[Q1 * Q2P];
  __shared__ float s_r2[Q1 * K2];
  __shared__ float s_z1[K1 * K2];
  __shared__ float s_t[K1 * U2];
  __shared__ int s_row2[Q1];
  __shared__ int s_col2[NV2];
  __shared__ int s_row1[K1];
  __shared__ int s_col1[K2];

  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ z2 = t.in0 + tl.inst * t.bs_in0;
  const float* __restrict__ a1 = t.in1 + tl.inst * t.bs_in1;
  const float* same = t.in2 + tl.inst * t.bs_in2;
  float* out = t.out0 + tl.inst * t.bs_out0;
  const int b1 = t.b[1], b2 = t.b[2];
  const int p1 = b1 >> 1, p2 = b2 >> 1;  // level i+1
  const int q1 = p1 >> 1, q2 = p2 >> 1;  // level i+2
  const int R1 = tl.c1 * (U1 / 2) - HP, R2 = tl.c2 * (U2 / 2) - HP;
  const int S1 = R1 / 2 - (H - 1), S2 = R2 / 2 - (H - 1) - OFF2;

  for (int i = threadIdx.x; i < Q1; i += NT) s_row2[i] = pmod(S1 + i, q1) * q2;
  for (int i = threadIdx.x; i < NV2; i += NT) s_col2[i] = VEC ? pmod(S2 + 4 * i, q2) : S2 + 4 * i;
  for (int i = threadIdx.x; i < K1; i += NT) s_row1[i] = pmod(R1 + i, p1) * p2;
  for (int i = threadIdx.x; i < K2; i += NT) s_col1[i] = pmod(R2 + i, p2);
  __syncthreads();
  stage_rows<NT, Q1, NV2, VEC>(z2, s_row2, s_col2, s_z2, Q2P, q2);
  __syncthreads();

  // level i+2 -> i+1 along the contiguous dim: (Q1, Q2) -> (Q1, K2)
  synthesis_pass<L, P2a, false, false, NT>(
      Q1, K2 / 2 / P2a, f,
      [&](int l, int j0, float* lo, float*) {
        const float* p = s_z2 + l * Q2P + OFF2 + j0;
#pragma unroll
        for (int j = 0; j < P2a + H - 1; ++j) lo[j] = p[j];
      },
      [&](int l, int p, float e0, float e1) {
        s_r2[l * K2 + p] = e0;
        s_r2[l * K2 + p + 1] = e1;
      });
  __syncthreads();
  // level i+2 -> i+1 along rows, combined with gamma * a1: (Q1, K2) -> (K1, K2)
  const float gamma = t.gamma, delta = t.delta;
  synthesis_pass<L, P1a, false, true, NT>(
      K2, K1 / 2 / P1a, f,
      [&](int c, int j0, float* lo, float*) {
#pragma unroll
        for (int j = 0; j < P1a + H - 1; ++j) lo[j] = s_r2[(j0 + j) * K2 + c];
      },
      [&](int c, int p, float e0, float e1) {
        const int col = s_col1[c];
        s_z1[p * K2 + c] = fmaf(gamma, gld(a1 + s_row1[p] + col), delta * e0);
        s_z1[(p + 1) * K2 + c] = fmaf(gamma, gld(a1 + s_row1[p + 1] + col), delta * e1);
      });
  __syncthreads();
  // level i+1 -> i along the contiguous dim: (K1, K2) -> (K1, U2)
  synthesis_pass<L, P2, false, false, NT>(
      K1, U2 / 2 / P2, f,
      [&](int l, int j0, float* lo, float*) {
        const float* p = s_z1 + l * K2 + OFF1 + j0;
#pragma unroll
        for (int j = 0; j < P2 + H - 1; ++j) lo[j] = p[j];
      },
      [&](int l, int p, float e0, float e1) {
        s_t[l * U2 + p] = e0;
        s_t[l * U2 + p + 1] = e1;
      });
  __syncthreads();
  // level i+1 -> i along rows: (K1, U2) -> (U1, U2), out = alpha*same + beta*value
  const float alpha = t.alpha, beta = t.beta;
  synthesis_pass<L, P1, false, true, NT>(
      U2, U1 / 2 / P1, f,
      [&](int c, int j0, float* lo, float*) {
#pragma unroll
        for (int j = 0; j < P1 + H - 1; ++j) lo[j] = s_t[(OFF1 + j0 + j) * U2 + c];
      },
      [&](int c, int p, float e0, float e1) {
        const int g1 = tl.c1 * U1 + p, g2 = tl.c2 * U2 + c;
        if (g1 < b1 && g2 < b2) {
          const int o = g1 * b2 + g2;
          const float s0 = gld(same + o), s1 = gld(same + o + b2);
          gst(out + o, fmaf(alpha, s0, beta * e0));
          gst(out + o + b2, fmaf(alpha, s1, beta * e1));
        }
      });
}

// ---------------------------------------------------------------------------------------
// Streamed 3-D full-bank levels.  A work-group owns an in-plane tile (axes 1, 2) and a run of
// R output slices along axis 0, and visits the input slices the run needs in order: each slice
// is staged (with its in-plane halo) and filtered in-plane once, and the axis-0 filter combines
// the filtered slices in running sums each thread keeps in registers for its in-plane positions.
// Axis-0 halos are neither re-read nor recomputed except at the start of a run, and the in-plane
// halo is the 2-D one.  The axes are filtered in the order 2, 1, 0
// with the same arithmetic as the plain 3-D tiles, so both give identical results.

// FB_DOWN_S: in-plane tile T1 x T2 per band, R output slices.  Iteration p filters input slices
// 2p and 2p+1 of the work-group's run (staged with the in-plane halo) along axis 2 into a buffer
// of their own.  After one barrier the next pair is staged over the first buffer while every
// thread filters one column of both slices along axis 1 and adds the results to the axis-0 sums
// it keeps in registers for those positions; a second barrier ends the iteration.  Output slice
// k takes input slices 2k .. 2k+L-1 in that order, so after iteration p output p-(H-1) is
// complete; the sums then shift by one output.
template <int L, int R, int T1, int T2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_fb_down_s(TaskArgs args, Filter f) {
  constexpr int H = L / 2;
  constexpr int I1 = 2 * T1 + L - 2, I2 = 2 * T2 + L - 2;
  constexpr int I2P = (I2 + 3) & ~3, NV = I2P / 4;
  constexpr int T2x = 2 * T2;
  constexpr int P1 = 2 * T1 * T2 / NT;  // axis-1 outputs per band of one thread (one column)
  constexpr int W1 = 2 * P1 + L - 2;
  constexpr int QT = 2 * P1;            // in-plane positions per thread: rows [lo P1 | hi P1]
  constexpr int NP = R + H - 1;         // iterations
  static_assert(P1 >= 1 && P1 * NT == 2 * T1 * T2 && T1 % P1 == 0, "one axis-1 task per thread");
  __shared__ __attribute__((aligned(16))) float s_in[2 * I1 * I2P];
  __shared__ __attribute__((aligned(16))) float s_r[2 * I1 * T2x];  // rows (e, i1): [lo T2 | hi T2]
  __shared__ int s_row[I1];
  __shared__ int s_col[NV];

  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ src = t.in0 + tl.inst * t.bs_in0;
  float* __restrict__ coef = t.out0 + tl.inst * t.bs_out0;
  float* __restrict__ ll = t.out1 + tl.inst * t.bs_out1;
  const int b0 = t.b[0], b1 = t.b[1], b2 = t.b[2];
  const int h0 = b0 >> 1, h1 = b1 >> 1, h2 = b2 >> 1;
  const int k0 = R * tl.c0, o1 = 2 * T1 * tl.c1, o2 = 2 * T2 * tl.c2;
  const float alpha = t.alpha, beta = t.beta;
  const int c = threadIdx.x % T2x, kc = threadIdx.x / T2x;  // this thread's column and row chunk
  const int e2 = c >= T2, g2 = T2 * tl.c2 + c - e2 * T2;

  for (int i = threadIdx.x; i < I1; i += NT) s_row[i] = pmod(o1 + i, b1) * t.st_in0[1];
  for (int i = threadIdx.x; i < NV; i += NT) s_col[i] = VEC ? pmod(o2 + 4 * i, b2) : o2 + 4 * i;
  __syncthreads();

  // vector path: a pair's 16-byte loads are issued one iteration before it is staged, so their
  // latency overlaps the filtering of the pair before (row length I2P = 4 NV: LDS slot = load
  // index)
  constexpr int NLD = 2 * I1 * NV, ITL = (NLD + NT - 1) / NT;
  float4 pf[VEC ? ITL : 1];
  // each thread's load offsets within a slice do not change along the run: computed once
  static_assert(ITL <= 32, "one bit per load in the masks");
  int loff[VEC ? ITL : 1];
  unsigned lsec = 0;  // bit it: load it reads the second slice of the pair
  if constexpr (VEC) {
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, NLD - 1);
      const int e = q >= I1 * NV, r = q - e * I1 * NV;
      loff[it] = s_row[r / NV] + s_col[r % NV];
      lsec |= unsigned(e) << it;
    }
  }
  auto load_pair = [&](int p) {
    const float* sl0 = src + pmod(2 * (k0 + p), b0) * t.st_in0[0];
    const float* sl1 = src + pmod(2 * (k0 + p) + 1, b0) * t.st_in0[0];
#pragma unroll
    for (int it = 0; it < ITL; ++it) pf[it] = gld4(((lsec >> it) & 1 ? sl1 : sl0) + loff[it]);
  };
  auto stage_pair = [&](int p) {
    if constexpr (VEC) {
      float4* d4 = reinterpret_cast<float4*>(s_in);
#pragma unroll
      for (int it = 0; it < ITL; ++it) d4[min(int(threadIdx.x) + it * NT, NLD - 1)] = pf[it];
    } else {
#pragma unroll
      for (int e = 0; e < 2; ++e)
        stage_rows<NT, I1, NV, false>(src + pmod(2 * (k0 + p) + e, b0) * t.st_in0[0], s_row, s_col,
                                      s_in + e * I1 * I2P, I2P, b2);
    }
  };
  if constexpr (VEC) load_pair(0);
  stage_pair(0);
  __syncthreads();
  if constexpr (VEC) {
    if (NP > 1) load_pair(1);
  }

  float alo[H][QT], ahi[H][QT];
#pragma unroll
  for (int j = 0; j < H; ++j)
#pragma unroll
    for (int u = 0; u < QT; ++u) alo[j][u] = ahi[j][u] = 0.f;
  KSum nsq;  // squared-norm mode: this thread's compensated sum

  for (int p = 0; p < NP; ++p) {
    row_pass_to<L, 4, 2 * I1, T2, I2P, NT>(s_in, s_r, f);  // rows (e, i1) -> [lo T2 | hi T2]
    __syncthreads();
    if (p + 1 < NP) {
      stage_pair(p + 1);
      if constexpr (VEC) {
        if (p + 2 < NP) load_pair(p + 2);
      }
    }
    // axis 1 of both slices at column c, output rows P1 kc .. P1 kc + P1 - 1 of each band
    float x[2][QT];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      float win[W1];
#pragma unroll
      for (int j = 0; j < W1; ++j) win[j] = s_r[(e * I1 + 2 * P1 * kc + j) * T2x + c];
#pragma unroll
      for (int q = 0; q < P1; ++q) {
        float lo = 0.f, hi = 0.f;
#pragma unroll
        for (int tt = 0; tt < L; ++tt) {
          lo = fmaf(f.h[tt], win[2 * q + tt], lo);
          hi = fmaf(f.g[tt], win[2 * q + tt], hi);
        }
        x[e][q] = lo;
        x[e][P1 + q] = hi;
      }
    }
#pragma unroll
    for (int u = 0; u < QT; ++u) {
      const float x0 = x[0][u], x1 = x[1][u];
#pragma unroll
      for (int j = 0; j < H; ++j) {  // output p - j takes taps 2j, 2j+1
        alo[j][u] = fmaf(f.h[2 * j], x0, alo[j][u]);
        ahi[j][u] = fmaf(f.g[2 * j], x0, ahi[j][u]);
        alo[j][u] = fmaf(f.h[2 * j + 1], x1, alo[j][u]);
        ahi[j][u] = fmaf(f.g[2 * j + 1], x1, ahi[j][u]);
      }
    }
    const int g0 = k0 + p - (H - 1);  // output completed by this iteration
    if (p >= H - 1 && g0 < h0 && g2 < h2) {
#pragma unroll
      for (int u = 0; u < QT; ++u) {
        const int e1 = u >= P1;
        const int g1 = T1 * tl.c1 + P1 * kc + u - e1 * P1;
        if (g1 < h1) {
          // band (e0, e1, e2) at half-res position (g0, g1, g2)
          const float lo = alo[H - 1][u], hi = ahi[H - 1][u];
          if ((e1 | e2) == 0) {
            if (t.flags & kNormLL) nsq.add((beta * lo) * (beta * lo));
            else gst(ll + g0 * t.st_out1[0] + g1 * t.st_out1[1] + g2, beta * lo);
          } else if (t.flags & kNormSq) {
            nsq.add((alpha * lo) * (alpha * lo));
          } else {
            gst(coef + g0 * t.st_out0[0] + (e1 * h1 + g1) * t.st_out0[1] + e2 * h2 + g2, alpha * lo);
          }
          if (t.flags & kNormSq) nsq.add((alpha * hi) * (alpha * hi));
          else gst(coef + (h0 + g0) * t.st_out0[0] + (e1 * h1 + g1) * t.st_out0[1] + e2 * h2 + g2, alpha * hi);
        }
      }
    }
#pragma unroll
    for (int j = H - 1; j > 0; --j)
#pragma unroll
      for (int u = 0; u < QT; ++u) {
        alo[j][u] = alo[j - 1][u];
        ahi[j][u] = ahi[j - 1][u];
      }
#pragma unroll
    for (int u = 0; u < QT; ++u) alo[0][u] = ahi[0][u] = 0.f;
    __syncthreads();
  }
  if (t.flags & kNormSq) store_wg_sum<NT>(nsq, reinterpret_cast<float2*>(t.out0) + (wg - t.tile_begin));
}

// FB_UP_S: full-res output tile U1 x U2 in-plane, R output slices (R even).  Output pair Q (full-
// res slices 2Q, 2Q+1) takes the half-res slices Q-(H-1) .. Q of the low (e0 = 0) and high
// (e0 = 1) bands along axis 0.  Iteration p stages half-res slices 2p, 2p+1 of the run (8 bands
// each, in-plane halo), synthesises them in-plane into a low and a high plane, and adds them to
// the axis-0 sums each thread keeps in registers for its in-plane positions: slice r adds to
// pairs r .. r+H-1, and pair r is complete once slice r is in.
template <int L, int R, int U1, int U2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_fb_up_s(TaskArgs args, Filter f) {
  constexpr int H = L / 2;
  constexpr int J1 = U1 / 2 + H - 1, J2 = U2 / 2 + H - 1;
  constexpr int OFF = (4 - ((H - 1) & 3)) & 3;
  constexpr int J2P = (J2 + OFF + 3) & ~3, NV = J2P / 4;
  constexpr int NR = 4 * J1;         // staged rows of one slice: (e0, e1, j1), each holding both e2 halves
  constexpr int PLN = U1 * U2;        // one full-res in-plane plane
  constexpr int P2 = 4, P1 = U1 / 2 % 4 == 0 ? 4 : 2;
  constexpr int NS = R / 2 + H - 1;   // half-res slices the run needs
  constexpr int NP = (NS + 1) / 2;    // iterations
  constexpr int QT = PLN / NT;        // in-plane positions per thread
  static_assert(R % 2 == 0, "R must be even");
  static_assert(PLN % NT == 0, "positions must divide evenly among the threads");
  __shared__ __attribute__((aligned(16))) float s_in[2 * NR * 2 * J2P];
  __shared__ float s_a[2 * NR * U2];
  __shared__ float s_pl[4 * PLN];  // (slice e, band e0) planes
  __shared__ int s_rowc[2 * J1];   // in-plane row offsets into in1 for (e1, j1)
  __shared__ int s_rowl[2 * J1];   // in-plane row offsets into in0 for j1 (used when e1 = 0)
  __shared__ int s_col[2 * NV];

  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ ap = t.in0 + tl.inst * t.bs_in0;
  const float* __restrict__ cp = t.in1 + tl.inst * t.bs_in1;
  float* __restrict__ out = t.out0 + tl.inst * t.bs_out0;
  const int b0 = t.b[0], b1 = t.b[1], b2 = t.b[2];
  const int h0 = b0 >> 1, h1 = b1 >> 1, h2 = b2 >> 1;
  const int q0 = tl.c0 * (R / 2);  // first output pair (half-res index)
  const int r1 = tl.c1 * (U1 / 2) - (H - 1), r2 = tl.c2 * (U2 / 2) - (H - 1) - OFF;
  const float alpha = t.alpha, beta = t.beta;

  for (int i = threadIdx.x; i < 2 * J1; i += NT) {
    const int e1 = i / J1, j1 = i - e1 * J1;
    s_rowc[i] = (e1 * h1 + pmod(r1 + j1, h1)) * t.st_in1[1];
    s_rowl[i] = pmod(r1 + j1, h1) * t.st_in0[1];
  }
  for (int i = threadIdx.x; i < 2 * NV; i += NT) {
    const int e2 = i / NV, v = i - e2 * NV;
    s_col[i] = VEC ? pmod(r2 + 4 * v, h2) + e2 * h2 : r2 + 4 * v;
  }
  __syncthreads();

  // vector path: the next pair's loads are issued before this pair is filtered
  // (row length J2P = 4 NV: LDS slot = load index)
  constexpr int NL1 = NR * 2 * NV, NLD = 2 * NL1, ITL = (NLD + NT - 1) / NT;
  float4 pf[VEC ? ITL : 1];
  // each thread's load offsets within a slice do not change along the run: computed once
  static_assert(ITL <= 32, "one bit per load in the masks");
  int loff[VEC ? ITL : 1];
  unsigned lsec = 0, lll = 0;  // bit it: load it reads the pair's second slice / the band in0
  if constexpr (VEC) {
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, NLD - 1);
      const int e = q >= NL1, qq = q - e * NL1;
      const int v = qq % NV, re = qq / NV;  // re = row * 2 + e2
      const int e2 = re & 1, row = re >> 1;
      const int e0 = row / (2 * J1), rr = row - e0 * 2 * J1;  // rr = e1 * J1 + j1
      const bool isll = e0 == 0 && e2 == 0 && rr < J1;
      loff[it] = isll ? s_rowl[rr] + s_col[v] : e0 * h0 * t.st_in1[0] + s_rowc[rr] + s_col[e2 * NV + v];
      lsec |= unsigned(e) << it;
      lll |= unsigned(isll) << it;
    }
  }
  auto load_pair = [&](int p) {
    const int s0 = pmod(q0 - (H - 1) + 2 * p, h0), s1 = pmod(q0 - (H - 1) + 2 * p + 1, h0);
    const float* a0 = ap + s0 * t.st_in0[0];
    const float* a1 = ap + s1 * t.st_in0[0];
    const float* c0 = cp + s0 * t.st_in1[0];
    const float* c1 = cp + s1 * t.st_in1[0];
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const bool sec = (lsec >> it) & 1, isll = (lll >> it) & 1;
      float4 x = gld4((isll ? (sec ? a1 : a0) : (sec ? c1 : c0)) + loff[it]);
      const float sc = isll ? beta : alpha;
      x.x *= sc; x.y *= sc; x.z *= sc; x.w *= sc;
      pf[it] = x;
    }
  };
  if constexpr (VEC) load_pair(0);

  float ac0[H][QT], ac1[H][QT];  // pair r + j: full-res slices 2(r+j) and 2(r+j)+1
#pragma unroll
  for (int j = 0; j < H; ++j)
#pragma unroll
    for (int u = 0; u < QT; ++u) ac0[j][u] = ac1[j][u] = 0.f;

  for (int p = 0; p < NP; ++p) {
    // stage: per slice, rows (e0, e1, j1) x (e2, J2P); band (0,0,0) from in0 (x beta), the rest
    // from in1 (x alpha)
    if constexpr (VEC) {
      float4* d4 = reinterpret_cast<float4*>(s_in);
#pragma unroll
      for (int it = 0; it < ITL; ++it) d4[min(int(threadIdx.x) + it * NT, NLD - 1)] = pf[it];
      __syncthreads();
      load_pair(min(p + 1, NP - 1));
    } else {
      constexpr int N1 = NR * 2 * J2P;
      for (int q = threadIdx.x; q < 2 * N1; q += NT) {
        const int e = q >= N1, qq = q - e * N1;
        const int r0g = pmod(q0 - (H - 1) + 2 * p + e, h0);
        const int c = qq % J2P, re = qq / J2P;
        const int e2 = re & 1, row = re >> 1;
        const int e0 = row / (2 * J1), rr = row - e0 * 2 * J1;
        const int col = pmod(r2 + c, h2);
        const bool isll = e0 == 0 && e2 == 0 && rr < J1;
        const float v = isll ? beta * gld(ap + r0g * t.st_in0[0] + s_rowl[rr] + col)
                             : alpha * gld(cp + (e0 * h0 + r0g) * t.st_in1[0] + s_rowc[rr] + e2 * h2 + col);
        s_in[q] = v;
      }
      __syncthreads();
    }
    // in-plane axis 2: every staged row (e, e0, e1, j1) -> U2 full-res values
    synthesis_pass<L, P2, true, false, NT>(
        2 * NR, U2 / 2 / P2, f,
        [&](int l, int j0, float* lo, float* hi) {  // rows of J2P floats (a multiple of 4)
          lds_window<P2 + H - 1, OFF>(s_in + (2 * l) * J2P + j0, lo);
          lds_window<P2 + H - 1, OFF>(s_in + (2 * l + 1) * J2P + j0, hi);
        },
        [&](int l, int pp, float e0, float e1) {
          s_a[l * U2 + pp] = e0;
          s_a[l * U2 + pp + 1] = e1;
        });
    __syncthreads();
    // in-plane axis 1: lines (e, e0, column) -> U1 full-res rows of plane (e, e0)
    synthesis_pass<L, P1, true, true, NT>(
        4 * U2, U1 / 2 / P1, f,
        [&](int l, int j0, float* lo, float* hi) {
          const int ee = l / U2, c = l - ee * U2;  // ee = e * 2 + e0
          const float* base = s_a + ee * 2 * J1 * U2 + c;
#pragma unroll
          for (int j = 0; j < P1 + H - 1; ++j) {
            lo[j] = base[(j0 + j) * U2];
            hi[j] = base[(J1 + j0 + j) * U2];
          }
        },
        [&](int l, int pp, float v0, float v1) {
          const int ee = l / U2, c = l - ee * U2;
          s_pl[ee * PLN + pp * U2 + c] = v0;
          s_pl[ee * PLN + (pp + 1) * U2 + c] = v1;
        });
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 2; ++e) {
#pragma unroll
      for (int u = 0; u < QT; ++u) {
        const int pos = threadIdx.x + u * NT;
        const float lo = s_pl[(2 * e) * PLN + pos], hi = s_pl[(2 * e + 1) * PLN + pos];
#pragma unroll
        for (int j = 0; j < H; ++j) {  // same per-term order as synthesis_pass
          ac0[j][u] = fmaf(f.h[2 * j], lo, ac0[j][u]);
          ac1[j][u] = fmaf(f.h[2 * j + 1], lo, ac1[j][u]);
          ac0[j][u] = fmaf(f.g[2 * j], hi, ac0[j][u]);
          ac1[j][u] = fmaf(f.g[2 * j + 1], hi, ac1[j][u]);
        }
      }
      const int rel = 2 * p + e - (H - 1);  // pair completed by this slice, relative to q0
      if (rel >= 0 && rel < R / 2 && 2 * (q0 + rel) < b0) {
        const int g0 = 2 * (q0 + rel);
#pragma unroll
        for (int u = 0; u < QT; ++u) {
          const int pos = threadIdx.x + u * NT;
          const int p1 = pos / U2, c = pos - p1 * U2;
          const int g1 = tl.c1 * U1 + p1, g2 = tl.c2 * U2 + c;
          if (g1 < b1 && g2 < b2) {
            const int o = g0 * t.st_out0[0] + g1 * t.st_out0[1] + g2;
            gst(out + o, ac0[0][u]);
            gst(out + o + t.st_out0[0], ac1[0][u]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < H - 1; ++j)
#pragma unroll
        for (int u = 0; u < QT; ++u) {
          ac0[j][u] = ac0[j + 1][u];
          ac1[j][u] = ac1[j + 1][u];
        }
#pragma unroll
      for (int u = 0; u < QT; ++u) ac0[H - 1][u] = ac1[H - 1][u] = 0.f;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Streamed 3-D low-pass levels (projection form).  A work-group owns an in-plane tile and a run
// of R output slices along axis 0, as the streamed full-bank kernels do, but keeps the axis order
// of the plain 3-D low-pass tiles (axis 2, then 0, then 1): every staged slice is filtered along
// axis 2 once; the axis-0 filter is a running sum each thread keeps in registers for its
// positions of the axis-2-filtered plane (halo rows of axis 1 included); a completed output slice
// goes through LDS for the axis-1 filter.  Per output the taps are summed in the plain tiles'
// order, so both families give identical bits.

// LP_DOWN_S (3-D): a_out = A a_in; in-plane half-res tile T1 x T2, R output slices.  Iteration p
// stages input slices 2p and 2p+1 of the run; output slice k takes input slices 2k .. 2k+L-1.
template <int L, int R, int T1, int T2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_lp_down_s3(TaskArgs args, Filter f) {
  constexpr int H = L / 2;
  constexpr int I1 = 2 * T1 + L - 2, I2 = 2 * T2 + L - 2;
  constexpr int I2P = (I2 + 3) & ~3, NV = I2P / 4;
  constexpr int NPOS = I1 * T2;             // positions of one axis-2-filtered slice
  constexpr int QA = (NPOS + NT - 1) / NT;  // of them per thread
  constexpr int NP = R + H - 1;             // iterations
  constexpr int P1 = 4;
  static_assert(T1 % P1 == 0 && T2 % 4 == 0, "tile shape");
  __shared__ __attribute__((aligned(16))) float s_in[2 * I1 * I2P];
  __shared__ float s_r[2 * NPOS];  // the pair's slices filtered along axis 2
  __shared__ float s_b[NPOS];      // a completed output slice (axes 2 and 0 done)
  __shared__ int s_row[I1];
  __shared__ int s_col[NV];

  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ src = t.in0 + tl.inst * t.bs_in0;
  float* __restrict__ dst = t.out0 + tl.inst * t.bs_out0;
  const int b0 = t.b[0], b1 = t.b[1], b2 = t.b[2];
  const int n0o = b0 >> 1, n1o = b1 >> 1, n2o = b2 >> 1;
  const int k0 = R * tl.c0, o1 = 2 * T1 * tl.c1, o2 = 2 * T2 * tl.c2;

  for (int i = threadIdx.x; i < I1; i += NT) s_row[i] = pmod(o1 + i, b1) * t.st_in0[1];
  for (int i = threadIdx.x; i < NV; i += NT) s_col[i] = VEC ? pmod(o2 + 4 * i, b2) : o2 + 4 * i;
  __syncthreads();

  // vector path: a pair's 16-byte loads are issued one iteration before it is staged; each
  // thread's load offsets within a slice are computed once (LDS slot = load index)
  constexpr int NLD = 2 * I1 * NV, ITL = (NLD + NT - 1) / NT;
  static_assert(ITL <= 32, "one bit per load in the mask");
  float4 pf[VEC ? ITL : 1];
  int loff[VEC ? ITL : 1];
  unsigned lsec = 0;  // bit it: load it reads the second slice of the pair
  if constexpr (VEC) {
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, NLD - 1);
      const int e = q >= I1 * NV, r = q - e * I1 * NV;
      loff[it] = s_row[r / NV] + s_col[r % NV];
      lsec |= unsigned(e) << it;
    }
  }
  auto load_pair = [&](int p) {
    const float* sl0 = src + pmod(2 * (k0 + p), b0) * t.st_in0[0];
    const float* sl1 = src + pmod(2 * (k0 + p) + 1, b0) * t.st_in0[0];
#pragma unroll
    for (int it = 0; it < ITL; ++it) pf[it] = gld4(((lsec >> it) & 1 ? sl1 : sl0) + loff[it]);
  };
  if constexpr (VEC) load_pair(0);

  float acc[H][QA];
#pragma unroll
  for (int j = 0; j < H; ++j)
#pragma unroll
    for (int u = 0; u < QA; ++u) acc[j][u] = 0.f;

  for (int p = 0; p < NP; ++p) {
    if constexpr (VEC) {
      float4* d4 = reinterpret_cast<float4*>(s_in);
#pragma unroll
      for (int it = 0; it < ITL; ++it) d4[min(int(threadIdx.x) + it * NT, NLD - 1)] = pf[it];
      __syncthreads();
      if (p + 1 < NP) load_pair(p + 1);
    } else {
#pragma unroll
      for (int e = 0; e < 2; ++e)
        stage_rows<NT, I1, NV, false>(src + pmod(2 * (k0 + p) + e, b0) * t.st_in0[0], s_row, s_col,
                                      s_in + e * I1 * I2P, I2P, b2);
      __syncthreads();
    }
    row_pass_to<L, 4, 2 * I1, T2, I2P, NT, false>(s_in, s_r, f);  // rows (e, i1) -> T2
    __syncthreads();
    // axis 0: output p - j takes taps 2j (slice 2p) and 2j + 1 (slice 2p + 1)
#pragma unroll
    for (int u = 0; u < QA; ++u) {
      const int q = threadIdx.x + u * NT;
      if (NPOS % NT == 0 || q < NPOS) {
        const float x0 = s_r[q], x1 = s_r[NPOS + q];
#pragma unroll
        for (int j = 0; j < H; ++j) {
          acc[j][u] = fmaf(f.h[2 * j], x0, acc[j][u]);
          acc[j][u] = fmaf(f.h[2 * j + 1], x1, acc[j][u]);
        }
      }
    }
    const int g0 = k0 + p - (H - 1);  // output slice completed by this iteration
    if (p >= H - 1 && g0 < n0o) {
#pragma unroll
      for (int u = 0; u < QA; ++u) {
        const int q = threadIdx.x + u * NT;
        if (NPOS % NT == 0 || q < NPOS) s_b[q] = acc[H - 1][u];
      }
      __syncthreads();
      // axis 1: (I1, T2) -> (T1, T2), lines are columns
      analysis_pass<L, P1, false, true, NT>(
          T2, T1 / P1, f,
          [&](int c, int j0, float* w) {
#pragma unroll
            for (int j = 0; j < 2 * P1 + L - 2; ++j) w[j] = s_b[(j0 + j) * T2 + c];
          },
          [&](int c, int k, float lo, float) {
            const int g1 = T1 * tl.c1 + k, g2 = T2 * tl.c2 + c;
            if (g1 < n1o && g2 < n2o) gst(dst + (g0 * n1o + g1) * n2o + g2, lo);
          });
    }
#pragma unroll
    for (int j = H - 1; j > 0; --j)
#pragma unroll
      for (int u = 0; u < QA; ++u) acc[j][u] = acc[j - 1][u];
#pragma unroll
    for (int u = 0; u < QA; ++u) acc[0][u] = 0.f;
  }
}

// LP_UP_S (3-D): out = alpha * same + beta * A^T z; full-res in-plane tile U1 x U2, R output
// slices (R even).  Output pair Q (full-res slices 2Q, 2Q+1) takes half-res slices Q-(H-1) .. Q;
// iteration p stages half-res slices 2p, 2p+1 of the run, slice r adds to pairs r .. r+H-1 and
// pair r is complete once slice r is in.
template <int L, int R, int U1, int U2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_lp_up_s3(TaskArgs args, Filter f) {
  constexpr int H = L / 2;
  constexpr int J1 = U1 / 2 + H - 1, J2 = U2 / 2 + H - 1;
  constexpr int OFF = (4 - ((H - 1) & 3)) & 3;
  constexpr int J2P = (J2 + OFF + 3) & ~3, NV = J2P / 4;
  constexpr int NPOS = J1 * U2;             // positions of one axis-2-synthesised slice
  constexpr int QA = (NPOS + NT - 1) / NT;  // of them per thread
  constexpr int NS = R / 2 + H - 1;         // half-res slices the run needs
  constexpr int NP = (NS + 1) / 2;          // iterations
  constexpr int P2 = 4, P1 = U1 / 2 % 4 == 0 ? 4 : 2;
  static_assert(R % 2 == 0 && U2 % 8 == 0 && (U1 / 2) % P1 == 0, "tile shape");
  __shared__ __attribute__((aligned(16))) float s_in[2 * J1 * J2P];
  __shared__ float s_a[2 * NPOS];     // the pair's slices synthesised along axis 2
  __shared__ float s_b[2][2 * NPOS];  // up to two completed output pairs: planes 2Q, 2Q+1
  __shared__ int s_row[J1];
  __shared__ int s_col[NV];

  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ z = t.in0 + tl.inst * t.bs_in0;
  const float* same = t.in1 + tl.inst * t.bs_in1;  // may alias out (in-place z over a)
  float* out = t.out0 + tl.inst * t.bs_out0;
  const int b0 = t.b[0], b1 = t.b[1], b2 = t.b[2];
  const int h0 = b0 >> 1, h1 = b1 >> 1, h2 = b2 >> 1;  // z dims
  const int q0 = tl.c0 * (R / 2);                      // first output pair (half-res index)
  const int r1 = tl.c1 * (U1 / 2) - (H - 1), r2 = tl.c2 * (U2 / 2) - (H - 1) - OFF;
  const float alpha = t.alpha, beta = t.beta;

  for (int i = threadIdx.x; i < J1; i += NT) s_row[i] = pmod(r1 + i, h1) * h2;
  for (int i = threadIdx.x; i < NV; i += NT) s_col[i] = VEC ? pmod(r2 + 4 * i, h2) : r2 + 4 * i;
  __syncthreads();

  constexpr int NLD = 2 * J1 * NV, ITL = (NLD + NT - 1) / NT;
  static_assert(ITL <= 32, "one bit per load in the mask");
  float4 pf[VEC ? ITL : 1];
  int loff[VEC ? ITL : 1];
  unsigned lsec = 0;  // bit it: load it reads the second slice of the pair
  if constexpr (VEC) {
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, NLD - 1);
      const int e = q >= J1 * NV, r = q - e * J1 * NV;
      loff[it] = s_row[r / NV] + s_col[r % NV];
      lsec |= unsigned(e) << it;
    }
  }
  const int slice = h1 * h2;
  auto load_pair = [&](int p) {
    const float* sl0 = z + pmod(q0 - (H - 1) + 2 * p, h0) * slice;
    const float* sl1 = z + pmod(q0 - (H - 1) + 2 * p + 1, h0) * slice;
#pragma unroll
    for (int it = 0; it < ITL; ++it) pf[it] = gld4(((lsec >> it) & 1 ? sl1 : sl0) + loff[it]);
  };
  if constexpr (VEC) load_pair(0);

  float ac0[H][QA], ac1[H][QA];  // pair r + j: full-res slices 2(r+j) and 2(r+j)+1
#pragma unroll
  for (int j = 0; j < H; ++j)
#pragma unroll
    for (int u = 0; u < QA; ++u) ac0[j][u] = ac1[j][u] = 0.f;

  for (int p = 0; p < NP; ++p) {
    if constexpr (VEC) {
      float4* d4 = reinterpret_cast<float4*>(s_in);
#pragma unroll
      for (int it = 0; it < ITL; ++it) d4[min(int(threadIdx.x) + it * NT, NLD - 1)] = pf[it];
      __syncthreads();
      if (p + 1 < NP) load_pair(p + 1);
    } else {
#pragma unroll
      for (int e = 0; e < 2; ++e)
        stage_rows<NT, J1, NV, false>(z + pmod(q0 - (H - 1) + 2 * p + e, h0) * slice, s_row, s_col,
                                      s_in + e * J1 * J2P, J2P, h2);
      __syncthreads();
    }
    // axis 2: rows (e, j1) -> U2 full-res values
    synthesis_pass<L, P2, false, false, NT>(
        2 * J1, U2 / 2 / P2, f,
        [&](int l, int j0, float* lo, float*) {
          const float* ptr = s_in + l * J2P + OFF + j0;
#pragma unroll
          for (int j = 0; j < P2 + H - 1; ++j) lo[j] = ptr[j];
        },
        [&](int l, int pp, float e0, float e1) {
          s_a[l * U2 + pp] = e0;
          s_a[l * U2 + pp + 1] = e1;
        });
    __syncthreads();
    // axis 0: slice 2p + e adds to pairs (2p + e) - (H-1) + j, oldest slice first
    int ncomp = 0, gq0 = 0, gq1 = 0;  // completed pairs of this iteration (at most one per slice)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
#pragma unroll
      for (int u = 0; u < QA; ++u) {
        const int q = threadIdx.x + u * NT;
        if (NPOS % NT == 0 || q < NPOS) {
          const float x = s_a[e * NPOS + q];
#pragma unroll
          for (int j = 0; j < H; ++j) {  // same per-term order as synthesis_pass
            ac0[j][u] = fmaf(f.h[2 * j], x, ac0[j][u]);
            ac1[j][u] = fmaf(f.h[2 * j + 1], x, ac1[j][u]);
          }
        }
      }
      const int rel = 2 * p + e - (H - 1);  // pair completed by this slice, relative to q0
      if (rel >= 0 && rel < R / 2 && 2 * (q0 + rel) < b0) {
#pragma unroll
        for (int u = 0; u < QA; ++u) {
          const int q = threadIdx.x + u * NT;
          if (NPOS % NT == 0 || q < NPOS) {
            s_b[ncomp][q] = ac0[0][u];
            s_b[ncomp][NPOS + q] = ac1[0][u];
          }
        }
        if (ncomp == 0) gq0 = q0 + rel;
        else gq1 = q0 + rel;
        ++ncomp;
      }
#pragma unroll
      for (int j = 0; j < H - 1; ++j)
#pragma unroll
        for (int u = 0; u < QA; ++u) {
          ac0[j][u] = ac0[j + 1][u];
          ac1[j][u] = ac1[j + 1][u];
        }
#pragma unroll
      for (int u = 0; u < QA; ++u) ac0[H - 1][u] = ac1[H - 1][u] = 0.f;
    }
    if (ncomp > 0) {
      __syncthreads();
      // axis 1 of the completed pairs: lines (pair m, plane, column) -> U1 full-res rows
      synthesis_pass<L, P1, false, true, NT>(
          ncomp * 2 * U2, U1 / 2 / P1, f,
          [&](int l, int j0, float* lo, float*) {
            const int m = l / (2 * U2), rem = l - m * 2 * U2, pl = rem / U2, c = rem - pl * U2;
            const float* base = &s_b[m][pl * NPOS + c];
#pragma unroll
            for (int j = 0; j < P1 + H - 1; ++j) lo[j] = base[(j0 + j) * U2];
          },
          [&](int l, int pp, float v0, float v1) {
            const int m = l / (2 * U2), rem = l - m * 2 * U2, pl = rem / U2, c = rem - pl * U2;
            const int g0 = 2 * (m ? gq1 : gq0) + pl, g1 = tl.c1 * U1 + pp, g2 = tl.c2 * U2 + c;
            if (g0 < b0 && g1 < b1 && g2 < b2) {
              const int o = (g0 * b1 + g1) * b2 + g2;
              const float s0 = gld(same + o), s1 = gld(same + o + b2);
              gst(out + o, fmaf(alpha, s0, beta * v0));
              gst(out + o + b2, fmaf(alpha, s1, beta * v1));
            }
          });
    }
  }
}

// ---------------------------------------------------------------------------------------
// FB_DOWN: one full analysis level on a (T0,T1,T2) tile of every band.
// Bands go to out0 (packed coefficient array, strides st_out0, detail bands x alpha) except
// the all-low band, which goes to out1 (next level's approximation, strides st_out1, x beta).

template <int D, int L, int T0, int T1, int T2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_fb_down(TaskArgs args, Filter f) {
  using G = DownGeom<D, L, T0, T1, T2>;
  constexpr int P2 = 4, P1 = 4, P0 = 2;
  constexpr int T2x = 2 * T2;  // [lo | hi] along the contiguous dim
  __shared__ __attribute__((aligned(16))) float s_in[G::NROW * G::I2P];
  __shared__ float s_b[D >= 3 ? G::I0 * 2 * T1 * T2x : 1];
  __shared__ int s_row[G::NROW];
  __shared__ int s_col[G::NV];

  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ src = t.in0 + tl.inst * t.bs_in0;
  float* __restrict__ coef = t.out0 + tl.inst * t.bs_out0;
  float* __restrict__ ll = t.out1 + tl.inst * t.bs_out1;
  const int b0 = t.b[0], b1 = t.b[1], b2 = t.b[2];
  const int o0 = 2 * T0 * tl.c0, o1 = 2 * T1 * tl.c1, o2 = 2 * T2 * tl.c2;

  for (int i = threadIdx.x; i < G::NROW; i += NT) {
    const int i1 = i % G::I1, i0 = i / G::I1;
    s_row[i] = (D >= 3 ? pmod(o0 + i0, b0) * t.st_in0[0] : 0) + (D >= 2 ? pmod(o1 + i1, b1) * t.st_in0[1] : 0);
  }
  for (int i = threadIdx.x; i < G::NV; i += NT) s_col[i] = VEC ? pmod(o2 + 4 * i, b2) : o2 + 4 * i;
  __syncthreads();
  stage_rows<NT, G::NROW, G::NV, VEC>(src, s_row, s_col, s_in, G::I2P, b2);
  __syncthreads();

  float* s_a = s_in;  // (NROW, [lo T2 | hi T2]) written over the staging buffer
  row_pass_inplace<L, P2, G::NROW, T2, G::I2P, NT, true>(s_in, f);

  const int n0h = b0 >> 1, n1h = b1 >> 1, n2h = b2 >> 1;
  const float alpha = t.alpha, beta = t.beta;
  KSum nsq;  // squared-norm mode: this thread's compensated sum
  // write one coefficient of band (e0,e1,e2) at half-res position (g0,g1,g2)
  auto emit = [&](int e0, int e1, int e2, int g0, int g1, int g2, float v) {
    if (g0 >= (D >= 3 ? n0h : 1) || g1 >= (D >= 2 ? n1h : 1) || g2 >= n2h) return;
    if ((e0 | e1 | e2) == 0) {
      if (t.flags & kNormLL) nsq.add((beta * v) * (beta * v));
      else gst(ll + (D >= 3 ? g0 * t.st_out1[0] : 0) + (D >= 2 ? g1 * t.st_out1[1] : 0) + g2, beta * v);
    } else if (t.flags & kNormSq) {
      nsq.add((alpha * v) * (alpha * v));
    } else {
      const int r0 = e0 * n0h + g0, r1 = e1 * n1h + g1, r2 = e2 * n2h + g2;
      gst(coef + (D >= 3 ? r0 * t.st_out0[0] : 0) + (D >= 2 ? r1 * t.st_out0[1] : 0) + r2, alpha * v);
    }
  };

  if constexpr (D == 1) {
    for (int c = threadIdx.x; c < T2x; c += NT) {
      const int e2 = c >= T2, k = c - e2 * T2;
      emit(0, 0, e2, 0, 0, T2 * tl.c2 + k, s_a[c]);
    }
  } else if constexpr (D == 2) {
    analysis_pass<L, P1, true, true, NT>(
        T2x, T1 / P1, f,
        [&](int c, int j0, float* w) {
#pragma unroll
          for (int j = 0; j < 2 * P1 + L - 2; ++j) w[j] = s_a[(j0 + j) * T2x + c];
        },
        [&](int c, int k, float lo, float hi) {
          const int e2 = c >= T2, g2 = T2 * tl.c2 + c - e2 * T2, g1 = T1 * tl.c1 + k;
          emit(0, 0, e2, 0, g1, g2, lo);
          emit(0, 1, e2, 0, g1, g2, hi);
        });
  } else {
    // axis 1 then axis 0 (the order of the streamed kernel, so both give identical bits)
    constexpr int T1x = 2 * T1;
    analysis_pass<L, P1, true, true, NT>(
        G::I0 * T2x, T1 / P1, f,
        [&](int l, int j0, float* w) {
          const int c = l % T2x, i0 = l / T2x;
#pragma unroll
          for (int j = 0; j < 2 * P1 + L - 2; ++j) w[j] = s_a[(i0 * G::I1 + j0 + j) * T2x + c];
        },
        [&](int l, int k, float lo, float hi) {
          const int c = l % T2x, i0 = l / T2x;
          s_b[(i0 * T1x + k) * T2x + c] = lo;
          s_b[(i0 * T1x + T1 + k) * T2x + c] = hi;
        });
    __syncthreads();
    analysis_pass<L, P0, true, true, NT>(
        T1x * T2x, T0 / P0, f,
        [&](int l, int j0, float* w) {
#pragma unroll
          for (int j = 0; j < 2 * P0 + L - 2; ++j) w[j] = s_b[(j0 + j) * T1x * T2x + l];
        },
        [&](int l, int k, float lo, float hi) {
          const int c = l % T2x, k1x = l / T2x;
          const int e2 = c >= T2, e1 = k1x >= T1;
          const int g2 = T2 * tl.c2 + c - e2 * T2, g1 = T1 * tl.c1 + k1x - e1 * T1, g0 = T0 * tl.c0 + k;
          emit(0, e1, e2, g0, g1, g2, lo);
          emit(1, e1, e2, g0, g1, g2, hi);
        });
  }
  if (t.flags & kNormSq) store_wg_sum<NT>(nsq, reinterpret_cast<float2*>(t.out0) + (wg - t.tile_begin));
}

// ---------------------------------------------------------------------------------------
// FB_UP: one full synthesis level on a (U0,U1,U2) full-resolution tile.
// in0: approximation of the level (strides st_in0, x beta); in1: packed coefficient array
// (strides st_in1; detail bands x alpha); out0: finer approximation (strides st_out0).

template <int D, int L, int U0, int U1, int U2, int NT, bool VEC>
__global__ void __launch_bounds__(NT) k_fb_up(TaskArgs args, Filter f) {
  using G = UpGeom<D, L, U0, U1, U2>;
  constexpr int H = G::H;
  constexpr int P2 = 4, P1 = 4, P0 = 2;
  constexpr int NB = 1 << D;           // bands
  constexpr int NRB = G::NROW * NB / 2;  // staged rows: (e0, j0, e1, j1) for both e2
  // LDS rows: index ((e0*J0 + j0)*2*J1 + e1*J1 + j1) * 2 + e2, each J2P long
  __shared__ __attribute__((aligned(16))) float s_in[NRB * 2 * G::J2P];
  __shared__ float s_a[NRB * U2];
  __shared__ float s_b[D >= 3 ? 2 * G::J0 * U1 * U2 : 1];
  __shared__ int s_rowc[NRB];  // offset into in1 of staged row r (band rows of e0,e1)
  __shared__ int s_rowl[NRB];  // offset into in0 when e0 = e1 = 0, else -1
  __shared__ int s_col[2 * G::NV];

  const int wg = logical_wg(args.total_wg, args.reverse);
  if (wg < 0) return;
  const Task t = pick_task<Task>(args, wg);
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ ap = t.in0 + tl.inst * t.bs_in0;
  const float* __restrict__ cp = t.in1 + tl.inst * t.bs_in1;
  float* __restrict__ out = t.out0 + tl.inst * t.bs_out0;
  const int b0 = t.b[0], b1 = t.b[1], b2 = t.b[2];
  const int h0 = b0 >> 1, h1 = b1 >> 1, h2 = b2 >> 1;
  const int r0 = tl.c0 * (U0 / 2) - (H - 1), r1 = tl.c1 * (U1 / 2) - (H - 1);
  const int r2 = tl.c2 * (U2 / 2) - (H - 1) - G::OFF;
  constexpr int E0 = D >= 3 ? 2 : 1, E1 = D >= 2 ? 2 : 1;

  for (int i = threadIdx.x; i < NRB; i += NT) {
    int rem = i;
    const int j1 = rem % G::J1; rem /= G::J1;
    const int e1 = rem % E1; rem /= E1;
    const int j0 = rem % G::J0; rem /= G::J0;
    const int e0 = rem;
    const int q0 = pmod(r0 + j0, D >= 3 ? h0 : 1), q1 = pmod(r1 + j1, D >= 2 ? h1 : 1);
    s_rowc[i] = (D >= 3 ? (e0 * h0 + q0) * t.st_in1[0] : 0) + (D >= 2 ? (e1 * h1 + q1) * t.st_in1[1] : 0);
    s_rowl[i] = (e0 | e1) ? -1 : (D >= 3 ? q0 * t.st_in0[0] : 0) + (D >= 2 ? q1 * t.st_in0[1] : 0);
  }
  for (int i = threadIdx.x; i < 2 * G::NV; i += NT) {
    const int e2 = i / G::NV, v = i % G::NV;
    s_col[i] = VEC ? pmod(r2 + 4 * v, h2) + e2 * h2 : r2 + 4 * v;
  }
  __syncthreads();
  {
    const float alpha = t.alpha, beta = t.beta;
    if constexpr (VEC) {
      constexpr int n = NRB * 2 * G::NV;
      constexpr int IT = (n + NT - 1) / NT;
      float4* d4 = reinterpret_cast<float4*>(s_in);
      float4 r[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int q = min(int(threadIdx.x) + it * NT, n - 1);
        const int v = q % G::NV, re = q / G::NV;  // re = row*2 + e2
        const int e2 = re & 1, row = re >> 1;
        const bool ll = e2 == 0 && s_rowl[row] >= 0;
        const float* p = ll ? ap + s_rowl[row] + s_col[v] : cp + s_rowc[row] + s_col[e2 * G::NV + v];
        float4 x = gld4(p);
        const float sc = ll ? beta : alpha;
        x.x *= sc; x.y *= sc; x.z *= sc; x.w *= sc;
        r[it] = x;
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int q = min(int(threadIdx.x) + it * NT, n - 1);
        d4[(q / G::NV) * (G::J2P / 4) + q % G::NV] = r[it];
      }
    } else {
      const int n = NRB * 2 * G::J2P;
      for (int q = threadIdx.x; q < n; q += NT) {
        const int c = q % G::J2P, re = q / G::J2P;
        const int e2 = re & 1, row = re >> 1;
        const int col = pmod(r2 + c, h2);
        float v;
        if (e2 == 0 && s_rowl[row] >= 0) v = beta * gld(ap + s_rowl[row] + col);
        else v = alpha * gld(cp + s_rowc[row] + e2 * h2 + col);
        s_in[re * G::J2P + c] = v;
      }
    }
  }
  __syncthreads();

  synthesis_pass<L, P2, true, false, NT>(
      NRB, U2 / 2 / P2, f,
      [&](int l, int j0, float* lo, float* hi) {  // rows of J2P floats (a multiple of 4)
        lds_window<P2 + H - 1, G::OFF>(s_in + (2 * l) * G::J2P + j0, lo);
        lds_window<P2 + H - 1, G::OFF>(s_in + (2 * l + 1) * G::J2P + j0, hi);
      },
      [&](int l, int p, float e0, float e1) {
        s_a[l * U2 + p] = e0;
        s_a[l * U2 + p + 1] = e1;
      });
  __syncthreads();

  if constexpr (D == 1) {
    for (int p = threadIdx.x; p < U2; p += NT) {
      const int g2 = tl.c2 * U2 + p;
      if (g2 < b2) gst(out + g2, s_a[p]);
    }
  } else if constexpr (D == 2) {
    // rows of s_a: (e1, j1); lines are columns c
    synthesis_pass<L, P1, true, true, NT>(
        U2, U1 / 2 / P1, f,
        [&](int c, int j0, float* lo, float* hi) {
#pragma unroll
          for (int j = 0; j < P1 + H - 1; ++j) {
            lo[j] = s_a[(j0 + j) * U2 + c];
            hi[j] = s_a[(G::J1 + j0 + j) * U2 + c];
          }
        },
        [&](int c, int p, float e0, float e1) {
          const int g1 = tl.c1 * U1 + p, g2 = tl.c2 * U2 + c;
          if (g1 < b1 && g2 < b2) {
            gst(out + g1 * t.st_out0[1] + g2, e0);
            gst(out + (g1 + 1) * t.st_out0[1] + g2, e1);
          }
        });
  } else {
    // s_a rows: (e0, j0, e1, j1); axis 1 first -> s_b rows (e0, j0, p1), then axis 0 (the
    // order of the streamed kernel, so both give identical bits)
    constexpr int R1 = 2 * G::J1;  // (e1, j1)
    synthesis_pass<L, P1, true, true, NT>(
        2 * G::J0 * U2, U1 / 2 / P1, f,
        [&](int l, int j0, float* lo, float* hi) {
          const int c = l % U2, r = l / U2;  // r = e0 * J0 + j0
#pragma unroll
          for (int j = 0; j < P1 + H - 1; ++j) {
            lo[j] = s_a[(r * R1 + j0 + j) * U2 + c];
            hi[j] = s_a[(r * R1 + G::J1 + j0 + j) * U2 + c];
          }
        },
        [&](int l, int p, float e0, float e1) {
          const int c = l % U2, r = l / U2;
          s_b[(r * U1 + p) * U2 + c] = e0;
          s_b[(r * U1 + p + 1) * U2 + c] = e1;
        });
    __syncthreads();
    synthesis_pass<L, P0, true, true, NT>(
        U1 * U2, U0 / 2 / P0, f,
        [&](int l, int j0, float* lo, float* hi) {
#pragma unroll
          for (int j = 0; j < P0 + H - 1; ++j) {
            lo[j] = s_b[(j0 + j) * U1 * U2 + l];
            hi[j] = s_b[(G::J0 + j0 + j) * U1 * U2 + l];
          }
        },
        [&](int l, int p, float e0, float e1) {
          const int c = l % U2, p1 = l / U2;
          const int g0 = tl.c0 * U0 + p, g1 = tl.c1 * U1 + p1, g2 = tl.c2 * U2 + c;
          if (g0 < b0 && g1 < b1 && g2 < b2) {
            const int o = g0 * t.st_out0[0] + g1 * t.st_out0[1] + g2;
            gst(out + o, e0);
            gst(out + o + t.st_out0[0], e1);
          }
        });
  }
}

template <int D, int L, int CMAX>
__global__ void __launch_bounds__(kCoarseThreads) k_lp_coarse(TailArgs args, Filter f) {
  __shared__ __attribute__((aligned(16))) float sm[coarse_lds_floats(CMAX)];
  const int wg = logical_wg(args.total_wg);
  if (wg < 0) return;
  int ti = 0;
  if (args.table != nullptr) {
    int lo = 0, hi = args.count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (args.table[mid].tile_begin <= wg) lo = mid;
      else hi = mid - 1;
    }
    ti = lo;
  }
  const TailTask* tp = args.table != nullptr ? args.table + ti : &args.t0;
  lp_coarse_block<D, L, CMAX, kCoarseThreads>(tp, wg - tp->tile_begin, f, sm);
}

// ---------------------------------------------------------------------------------------
// FB_COARSE: the coarse levels of the full filter bank for one instance in one work-group.
// The packed pyramid of a block of at most kFbCoarseMax floats lives in a static LDS array
// (two copies for ping-pong), addressed by integer offsets; level j works on the leading
// sub-block (n_k >> j per axis).  SYN = false: analysis of levels T+1..m from a_T (contiguous
// input) into the packed coefficient block (strided output, detail bands weighted).
// SYN = true: synthesis from the packed block (strided input, weighted) down to a_T.

constexpr int kFbCoarseMax = kFbCoarseMaxBlock;

template <int L, bool SHORT>
DEVI void fbc_analysis_w(float* sm, int src, int dst, int S0, int S1, int b0, int b1, int b2, int ax, const Filter& f) {
  const int n = ax == 0 ? b0 : (ax == 1 ? b1 : b2), half = n >> 1;
  const int o0 = ax == 0 ? half : b0, o1 = ax == 1 ? half : b1, o2 = ax == 2 ? half : b2;
  const int l1 = ilog2_or_neg(o1), l2 = ilog2_or_neg(o2);
  const int step = ax == 0 ? S0 : (ax == 1 ? S1 : 1);
  const int total = o0 * o1 * o2;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, o1, o2, l1, l2, c0, c1, c2);
    const int k = ax == 0 ? c0 : (ax == 1 ? c1 : c2);
    const int other = (ax == 0 ? 0 : c0 * S0) + (ax == 1 ? 0 : c1 * S1) + (ax == 2 ? 0 : c2);
    float lo = 0.f, hi = 0.f;
    if (!SHORT) {  // n >= L: an index wraps at most once
#pragma unroll
      for (int t = 0; t < L; ++t) {
        const int i = 2 * k + t;
        const float x = sm[src + other + (i >= n ? i - n : i) * step];
        lo = fmaf(f.h[t], x, lo);
        hi = fmaf(f.g[t], x, hi);
      }
    } else {
#pragma unroll
      for (int t = 0; t < L; ++t) {
        const float x = sm[src + other + ((2 * k + t) % n) * step];
        lo = fmaf(f.h[t], x, lo);
        hi = fmaf(f.g[t], x, hi);
      }
    }
    sm[dst + other + k * step] = lo;
    sm[dst + other + (half + k) * step] = hi;
  }
}

template <int L, bool SHORT>
DEVI void fbc_synthesis_w(float* sm, int src, int dst, int S0, int S1, int b0, int b1, int b2, int ax, const Filter& f) {
  const int n = ax == 0 ? b0 : (ax == 1 ? b1 : b2), half = n >> 1;
  const int l1 = ilog2_or_neg(b1), l2 = ilog2_or_neg(b2);
  const int step = ax == 0 ? S0 : (ax == 1 ? S1 : 1);
  const int total = b0 * b1 * b2;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, b1, b2, l1, l2, c0, c1, c2);
    const int p = ax == 0 ? c0 : (ax == 1 ? c1 : c2);
    const int other = (ax == 0 ? 0 : c0 * S0) + (ax == 1 ? 0 : c1 * S1) + (ax == 2 ? 0 : c2);
    const int par = p & 1, q = p >> 1;
    float acc = 0.f;
    if (!SHORT) {  // half >= L/2: an index wraps at most once
#pragma unroll
      for (int j = 0; j < L / 2; ++j) {
        const int k = q - j < 0 ? q - j + half : q - j;
        acc = fmaf(par ? f.h[2 * j + 1] : f.h[2 * j], sm[src + other + k * step], acc);
        acc = fmaf(par ? f.g[2 * j + 1] : f.g[2 * j], sm[src + other + (half + k) * step], acc);
      }
    } else {
#pragma unroll
      for (int j = 0; j < L / 2; ++j) {
        const int k = pmod(q - j, half);
        acc = fmaf(par ? f.h[2 * j + 1] : f.h[2 * j], sm[src + other + k * step], acc);
        acc = fmaf(par ? f.g[2 * j + 1] : f.g[2 * j], sm[src + other + (half + k) * step], acc);
      }
    }
    sm[dst + other + p * step] = acc;
  }
}

// Register-window versions (as coarse_analysis_v / coarse_synthesis_v, for the strided packed
// layout of the full bank: low half at k, high half at half + k along the axis).
template <int L>
DEVI void fbc_analysis_v(float* sm, int src, int dst, int S0, int S1, int b0, int b1, int b2, int ax, const Filter& f) {
  constexpr int PO = 4, WN = 2 * PO + L - 2, W4 = (WN + 3) / 4;
  const int n = ax == 0 ? b0 : (ax == 1 ? b1 : b2), half = n >> 1;
  const int p0 = ax == 0 ? half / PO : b0, p1 = ax == 1 ? half / PO : b1, p2 = ax == 2 ? half / PO : b2;
  const int l1 = ilog2_or_neg(p1), l2 = ilog2_or_neg(p2);
  const int step = ax == 0 ? S0 : (ax == 1 ? S1 : 1);
  const int total = p0 * p1 * p2;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, p1, p2, l1, l2, c0, c1, c2);
    const int k0 = PO * (ax == 0 ? c0 : (ax == 1 ? c1 : c2));
    const int other = (ax == 0 ? 0 : c0 * S0) + (ax == 1 ? 0 : c1 * S1) + (ax == 2 ? 0 : c2);
    float win[4 * W4];
    if (ax == 2) {
#pragma unroll
      for (int v = 0; v < W4; ++v) {
        int i = 2 * k0 + 4 * v;
        i = i >= n ? i - n : i;
        const float4 x = *reinterpret_cast<const float4*>(sm + src + other + i);
        win[4 * v] = x.x; win[4 * v + 1] = x.y; win[4 * v + 2] = x.z; win[4 * v + 3] = x.w;
      }
    } else {
      const int a0 = src + other + 2 * k0 * step, a0w = a0 - n * step, wrap = n - 2 * k0;
#pragma unroll
      for (int j = 0; j < WN; ++j) win[j] = sm[(j >= wrap ? a0w : a0) + j * step];
    }
#pragma unroll
    for (int q = 0; q < PO; ++q) {
      float lo = 0.f, hi = 0.f;
#pragma unroll
      for (int t = 0; t < L; ++t) {
        lo = fmaf(f.h[t], win[2 * q + t], lo);
        hi = fmaf(f.g[t], win[2 * q + t], hi);
      }
      sm[dst + other + (k0 + q) * step] = lo;
      sm[dst + other + (half + k0 + q) * step] = hi;
    }
  }
}

template <int L>
DEVI void fbc_synthesis_v(float* sm, int src, int dst, int S0, int S1, int b0, int b1, int b2, int ax, const Filter& f) {
  constexpr int H = L / 2, PO = 8, A = (H - 1 + 3) & ~3, WN = A + 4, W4 = WN / 4;
  const int n = ax == 0 ? b0 : (ax == 1 ? b1 : b2), half = n >> 1;
  const int p0 = ax == 0 ? b0 / PO : b0, p1 = ax == 1 ? b1 / PO : b1, p2 = ax == 2 ? b2 / PO : b2;
  const int l1 = ilog2_or_neg(p1), l2 = ilog2_or_neg(p2);
  const int step = ax == 0 ? S0 : (ax == 1 ? S1 : 1);
  const int total = p0 * p1 * p2;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, p1, p2, l1, l2, c0, c1, c2);
    const int q0 = (PO / 2) * (ax == 0 ? c0 : (ax == 1 ? c1 : c2));
    const int other = (ax == 0 ? 0 : c0 * S0) + (ax == 1 ? 0 : c1 * S1) + (ax == 2 ? 0 : c2);
    float lo[WN], hi[WN];
    if (ax == 2) {
#pragma unroll
      for (int v = 0; v < W4; ++v) {
        int k = q0 - A + 4 * v;
        k = k < 0 ? k + half : k;
        const float4 x = *reinterpret_cast<const float4*>(sm + src + other + k);
        const float4 y = *reinterpret_cast<const float4*>(sm + src + other + half + k);
        lo[4 * v] = x.x; lo[4 * v + 1] = x.y; lo[4 * v + 2] = x.z; lo[4 * v + 3] = x.w;
        hi[4 * v] = y.x; hi[4 * v + 1] = y.y; hi[4 * v + 2] = y.z; hi[4 * v + 3] = y.w;
      }
    } else {
      const int a0 = src + other + (q0 - A) * step, a0w = a0 + half * step, hs = half * step;
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int a = (q0 - A + j < 0 ? a0w : a0) + j * step;
        lo[j] = sm[a];
        hi[j] = sm[a + hs];
      }
    }
#pragma unroll
    for (int r = 0; r < PO; ++r) {
      const int par = r & 1, qq = r >> 1;  // output 2 (q0 + qq) + par
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        acc = fmaf(f.h[2 * j + par], lo[A + qq - j], acc);
        acc = fmaf(f.g[2 * j + par], hi[A + qq - j], acc);
      }
      sm[dst + other + (2 * q0 + r) * step] = acc;
    }
  }
}

template <int L>
DEVI void fbc_analysis(float* sm, int src, int dst, int S0, int S1, int b0, int b1, int b2, int ax, const Filter& f) {
  const int n = ax == 0 ? b0 : (ax == 1 ? b1 : b2);
  if (n >= L && (n >> 1) % 4 == 0 && (ax != 2 || (src % 4 == 0 && S1 % 4 == 0 && S0 % 4 == 0)))
    fbc_analysis_v<L>(sm, src, dst, S0, S1, b0, b1, b2, ax, f);
  else if (n >= L) fbc_analysis_w<L, false>(sm, src, dst, S0, S1, b0, b1, b2, ax, f);
  else fbc_analysis_w<L, true>(sm, src, dst, S0, S1, b0, b1, b2, ax, f);
}
template <int L>
DEVI void fbc_synthesis(float* sm, int src, int dst, int S0, int S1, int b0, int b1, int b2, int ax, const Filter& f) {
  const int half = (ax == 0 ? b0 : (ax == 1 ? b1 : b2)) >> 1;
  if (half >= L / 2 && half % 4 == 0 && (ax != 2 || (src % 4 == 0 && S1 % 4 == 0 && S0 % 4 == 0)))
    fbc_synthesis_v<L>(sm, src, dst, S0, S1, b0, b1, b2, ax, f);
  else if (half >= L / 2) fbc_synthesis_w<L, false>(sm, src, dst, S0, S1, b0, b1, b2, ax, f);
  else fbc_synthesis_w<L, true>(sm, src, dst, S0, S1, b0, b1, b2, ax, f);
}

// Weight of the packed-pyramid element at (c0,c1,c2) of a coarse block: detail of coarse
// level j -> coef[j]; approximation (inside the block >> nlev) -> coef[nlev].
DEVI float fbc_weight(const float* coef, int nlev, int n0, int n1, int n2, int c0, int c1, int c2, int D) {
  int j = 0;
  while (j < nlev) {
    const int sh = j + 1;
    const bool inside = (c2 < (n2 >> sh)) && (D < 2 || c1 < (n1 >> sh)) && (D < 3 || c0 < (n0 >> sh));
    if (!inside) break;
    ++j;
  }
  return coef[j];
}

template <int D, int L, bool SYN>
__global__ void __launch_bounds__(kFbCoarseThreads) k_fb_coarse(TailArgs args, Filter f) {
  __shared__ __attribute__((aligned(16))) float sm[2 * kFbCoarseMax];
  const int wg = logical_wg(args.total_wg);
  if (wg < 0) return;
  int ti = 0;
  if (args.table != nullptr) {
    int lo = 0, hi = args.count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (args.table[mid].tile_begin <= wg) lo = mid;
      else hi = mid - 1;
    }
    ti = lo;
  }
  const TailTask* tp = args.table != nullptr ? args.table + ti : &args.t0;
  const int inst = wg - tp->tile_begin;
  const float* in = tp->in + inst * tp->bs_in;
  float* out = tp->out + inst * tp->bs_out;
  const int n0 = tp->b[0], n1 = tp->b[1], n2 = tp->b[2];
  const int B = n0 * n1 * n2, S0 = n1 * n2, S1 = n2;
  const int l1 = ilog2_or_neg(n1), l2 = ilog2_or_neg(n2);
  const int nl = tp->nlev;
  const int in0 = tp->st_in[0], in1 = tp->st_in[1], out0 = tp->st_out[0], out1 = tp->st_out[1];
  constexpr int CUR = 0, TMP = kFbCoarseMax;
  auto copy_back = [&](int b0, int b1, int b2) {  // TMP sub-block -> CUR
    const int t1 = ilog2_or_neg(b1), t2 = ilog2_or_neg(b2);
    for (int e = threadIdx.x; e < b0 * b1 * b2; e += blockDim.x) {
      int c0, c1, c2;
      split3(e, b1, b2, t1, t2, c0, c1, c2);
      const int o = c0 * S0 + c1 * S1 + c2;
      sm[CUR + o] = sm[TMP + o];
    }
  };
  constexpr int U = kFbCoarseMax / kFbCoarseThreads;
  if (!SYN) {
    gather_to_lds<kFbCoarseThreads, U>(
        B, [&](int e) { return gld(in + e); }, [&](int e, float v) { sm[CUR + e] = v; });
    __syncthreads();
    for (int j = 0; j < nl; ++j) {
      const int b0 = D >= 3 ? n0 >> j : 1, b1 = D >= 2 ? n1 >> j : 1, b2 = n2 >> j;
      // dim 2: CUR -> TMP, dim 1: TMP -> CUR, dim 0: CUR -> TMP
      fbc_analysis<L>(sm, CUR, TMP, S0, S1, b0, b1, b2, 2, f);
      __syncthreads();
      bool in_tmp = true;
      if (D >= 2) {
        fbc_analysis<L>(sm, TMP, CUR, S0, S1, b0, b1, b2, 1, f);
        __syncthreads();
        in_tmp = false;
        if (D >= 3) {
          fbc_analysis<L>(sm, CUR, TMP, S0, S1, b0, b1, b2, 0, f);
          __syncthreads();
          in_tmp = true;
        }
      }
      if (in_tmp) {
        copy_back(b0, b1, b2);
        __syncthreads();
      }
    }
    const bool norm = (tp->flags & kNormSq) != 0;
    KSum nsq;
    for (int e = threadIdx.x; e < B; e += blockDim.x) {
      int c0, c1, c2;
      split3(e, n1, n2, l1, l2, c0, c1, c2);
      const float w = fbc_weight(tp->coef, nl, n0, n1, n2, c0, c1, c2, D);
      const float v = w * sm[CUR + e];
      if (norm) nsq.add(v * v);
      else gst(out + (D >= 3 ? c0 * out0 : 0) + (D >= 2 ? c1 * out1 : 0) + c2, v);
    }
    if (norm) store_wg_sum<kFbCoarseThreads>(nsq, reinterpret_cast<float2*>(tp->out) + inst);
  } else {
    gather_to_lds<kFbCoarseThreads, U>(
        B,
        [&](int e) {
          int c0, c1, c2;
          split3(e, n1, n2, l1, l2, c0, c1, c2);
          return gld(in + (D >= 3 ? c0 * in0 : 0) + (D >= 2 ? c1 * in1 : 0) + c2);
        },
        [&](int e, float v) {
          int c0, c1, c2;
          split3(e, n1, n2, l1, l2, c0, c1, c2);
          sm[CUR + e] = fbc_weight(tp->coef, nl, n0, n1, n2, c0, c1, c2, D) * v;
        });
    __syncthreads();
    for (int j = nl - 1; j >= 0; --j) {
      const int b0 = D >= 3 ? n0 >> j : 1, b1 = D >= 2 ? n1 >> j : 1, b2 = n2 >> j;
      // dim 0 (3-D), dim 1, dim 2, ping-pong starting from CUR
      int a = CUR, bb = TMP;
      if (D >= 3) {
        fbc_synthesis<L>(sm, a, bb, S0, S1, b0, b1, b2, 0, f);
        __syncthreads();
        const int t = a; a = bb; bb = t;
      }
      if (D >= 2) {
        fbc_synthesis<L>(sm, a, bb, S0, S1, b0, b1, b2, 1, f);
        __syncthreads();
        const int t = a; a = bb; bb = t;
      }
      fbc_synthesis<L>(sm, a, bb, S0, S1, b0, b1, b2, 2, f);
      __syncthreads();
      if (bb != CUR) {
        copy_back(b0, b1, b2);
        __syncthreads();
      }
    }
    for (int e = threadIdx.x; e < B; e += blockDim.x) {
      int c0, c1, c2;
      split3(e, n1, n2, l1, l2, c0, c1, c2);
      gst(out + (D >= 3 ? c0 * out0 : 0) + (D >= 2 ? c1 * out1 : 0) + c2, sm[CUR + e]);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Plain reference kernels: one thread per output pair of one 1-D pass over the level block.

template <int L>
__global__ void __launch_bounds__(256) k_plain_pass(PlainPass p, Filter f) {
  const int ax = p.axis;
  const int n = p.b[ax], half = n >> 1;
  int hb[3] = {p.b[0], p.b[1], p.b[2]};
  hb[ax] = half;
  const int64_t total = (int64_t)hb[0] * hb[1] * hb[2];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int c2 = (int)(e % hb[2]);
  int64_t r = e / hb[2];
  int c1 = (int)(r % hb[1]);
  int c0 = (int)(r / hb[1]);
  int c[3] = {c0, c1, c2};
  const int k = c[ax];
  c[ax] = 0;
  const int ss = ax == 0 ? p.st_src[0] : (ax == 1 ? p.st_src[1] : 1);
  const int ds = ax == 0 ? p.st_dst[0] : (ax == 1 ? p.st_dst[1] : 1);
  const float* src = p.src + (int64_t)c[0] * p.st_src[0] + (int64_t)c[1] * p.st_src[1] + c[2];
  float* dst = p.dst + (int64_t)c[0] * p.st_dst[0] + (int64_t)c[1] * p.st_dst[1] + c[2];
  // an element is "low" when it lies in the all-low sub-block of the level block
  auto low_other = [&]() {
    for (int a = 0; a < 3; ++a) {
      if (a == ax) continue;
      if (a < 3 - p.ndim) continue;
      const int ca = a == 0 ? c0 : (a == 1 ? c1 : c2);
      if (ca >= (p.b[a] >> 1)) return false;
    }
    return true;
  };
  if (!p.synth) {
    float lo = 0.f, hi = 0.f;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const float x = src[(int64_t)((2 * k + t) % n) * ss];
      lo = fmaf(f.h[t], x, lo);
      hi = fmaf(f.g[t], x, hi);
    }
    if (p.scale_mode == 1) {
      if (!low_other()) lo *= p.w;
      hi *= p.w;
    }
    dst[(int64_t)k * ds] = lo;
    dst[(int64_t)(half + k) * ds] = hi;
  } else {
    const bool lo_scaled = (p.scale_mode == 2) && !low_other();
    const float wl = lo_scaled ? p.w : 1.f, wh = (p.scale_mode == 2) ? p.w : 1.f;
    float x0 = 0.f, x1 = 0.f;  // outputs 2k and 2k+1
#pragma unroll
    for (int t = 0; t < L; ++t) {
      // output q = 2k + e receives h[t] lo[j] + g[t] hi[j] for 2j + t == q (mod n)
      const int e0 = 2 * k - t, e1 = 2 * k + 1 - t;
      if ((e0 & 1) == 0) {
        const int j = pmod(e0 >> 1, half);
        x0 = fmaf(f.h[t], wl * src[(int64_t)j * ss], x0);
        x0 = fmaf(f.g[t], wh * src[(int64_t)(half + j) * ss], x0);
      } else {
        const int j = pmod((e1) >> 1, half);
        x1 = fmaf(f.h[t], wl * src[(int64_t)j * ss], x1);
        x1 = fmaf(f.g[t], wh * src[(int64_t)(half + j) * ss], x1);
      }
    }
    dst[(int64_t)(2 * k) * ds] = x0;
    dst[(int64_t)(2 * k + 1) * ds] = x1;
  }
}

__global__ void __launch_bounds__(256) k_block_copy(const float* src, float* dst, int b0, int b1, int b2, int s0,
                                                     int s1, int d0, int d1) {
  const int64_t total = (int64_t)b0 * b1 * b2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int c2 = (int)(e % b2);
  const int64_t r = e / b2;
  const int c1 = (int)(r % b1), c0 = (int)(r / b1);
  dst[(int64_t)c0 * d0 + (int64_t)c1 * d1 + c2] = src[(int64_t)c0 * s0 + (int64_t)c1 * s1 + c2];
}

__global__ void __launch_bounds__(256) k_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------------------
// Tile shapes and launch dispatch.

namespace {

// (kind, ndim, variant, taps) -> tile.  Variant 0 = wide, 1 = narrow (thin or small blocks).
// Analysis kinds: half-res output tile per band; synthesis kinds: full-res output tile.
// Squared-norm finalisation: one work-group per instance, segments in order, each segment's
// partials (compensated pairs) strided over the threads, then the work-group sum (fixed order:
// deterministic); the instance's norm is the rounded sum.
__global__ void __launch_bounds__(256) k_norm_finalize(const float2* __restrict__ partials, NormSegs segs,
                                                       float* __restrict__ out) {
  __shared__ float2 sum;
  const int b = blockIdx.x;
  KSum acc;
  for (int k = 0; k < segs.count; ++k) {
    const float2* p = partials + segs.off[k] + (int64_t)b * segs.per[k];
    for (int i = threadIdx.x; i < segs.per[k]; i += 256) {
      const float2 v = p[i];
      acc.merge(v.x, v.y);
    }
  }
  store_wg_sum<256>(acc, &sum);
  if (threadIdx.x == 0) out[b] = sum.x;
}

// Sum of squares of each instance (levels = 0: the transform is the identity).
__global__ void __launch_bounds__(256) k_sumsq(const float* __restrict__ x, int64_t n, float* __restrict__ out) {
  __shared__ float2 sum;
  const float* p = x + (int64_t)blockIdx.x * n;
  KSum acc;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const float v = gld(p + i);
    acc.add(v * v);
  }
  store_wg_sum<256>(acc, &sum);
  if (threadIdx.x == 0) out[blockIdx.x] = sum.x;
}


#define ES_TILE(K, D, V, L) shape_of(K, D, V, L).a, shape_of(K, D, V, L).b, shape_of(K, D, V, L).c

template <int K, int D, int L, int V, bool VEC>
hipError_t launch_kind(const TaskArgs& a, int grid, const Filter& f, hipStream_t s) {
  if constexpr (K == K_LP_DOWN)
    hipLaunchKernelGGL((k_lp_down<D, L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_LP_UP)
    hipLaunchKernelGGL((k_lp_up<D, L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_FB_DOWN)
    hipLaunchKernelGGL((k_fb_down<D, L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_LP_DOWN_S && D == 3)
    hipLaunchKernelGGL((k_lp_down_s3<L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_LP_DOWN_S)
    hipLaunchKernelGGL((k_lp_down_s<L, shape_of(K, 2, V, L).b, shape_of(K, 2, V, L).c, kThreads, VEC>), dim3(grid),
                       dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_LP_UP_S)
    hipLaunchKernelGGL((k_lp_up_s3<L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_FB_DOWN_S)
    hipLaunchKernelGGL((k_fb_down_s<L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_FB_UP_S)
    hipLaunchKernelGGL((k_fb_up_s<L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  else if constexpr (K == K_LP_UP2)
    hipLaunchKernelGGL((k_lp_up2<L, shape_of(K, 2, V, L).b, shape_of(K, 2, V, L).c, kThreads, VEC>), dim3(grid),
                       dim3(kThreads), 0, s, a, f);
  else
    hipLaunchKernelGGL((k_fb_up<D, L, ES_TILE(K, D, V, L), kThreads, VEC>), dim3(grid), dim3(kThreads), 0, s, a, f);
  return hipGetLastError();
}

template <int K, int D, int L>
hipError_t launch_kdl(int variant, bool vec, const TaskArgs& a, int grid, const Filter& f, hipStream_t s) {
  if (variant == 0) return vec ? launch_kind<K, D, L, 0, true>(a, grid, f, s) : launch_kind<K, D, L, 0, false>(a, grid, f, s);
  if (variant == 2) return vec ? launch_kind<K, D, L, 2, true>(a, grid, f, s) : launch_kind<K, D, L, 2, false>(a, grid, f, s);
  return vec ? launch_kind<K, D, L, 1, true>(a, grid, f, s) : launch_kind<K, D, L, 1, false>(a, grid, f, s);
}

template <int K, int D>
hipError_t launch_kd(int taps, int variant, bool vec, const TaskArgs& a, int grid, const Filter& f, hipStream_t s) {
  switch (taps) {
    case 2: return launch_kdl<K, D, 2>(variant, vec, a, grid, f, s);
    case 4: return launch_kdl<K, D, 4>(variant, vec, a, grid, f, s);
    case 6: return launch_kdl<K, D, 6>(variant, vec, a, grid, f, s);
    case 8: return launch_kdl<K, D, 8>(variant, vec, a, grid, f, s);
    case 10: return launch_kdl<K, D, 10>(variant, vec, a, grid, f, s);
    case 12: return launch_kdl<K, D, 12>(variant, vec, a, grid, f, s);
    case 14: return launch_kdl<K, D, 14>(variant, vec, a, grid, f, s);
    case 16: return launch_kdl<K, D, 16>(variant, vec, a, grid, f, s);
  }
  return hipErrorInvalidValue;
}

template <int K>
hipError_t launch_k(int ndim, int taps, int variant, bool vec, const TaskArgs& a, int grid, const Filter& f,
                    hipStream_t s) {
  switch (ndim) {
    case 1: return launch_kd<K, 1>(taps, variant, vec, a, grid, f, s);
    case 2: return launch_kd<K, 2>(taps, variant, vec, a, grid, f, s);
    case 3: return launch_kd<K, 3>(taps, variant, vec, a, grid, f, s);
  }
  return hipErrorInvalidValue;
}

template <int D, int L>
hipError_t launch_tail_dl(int kind, const TailArgs& a, int grid, size_t lds, const Filter& f, hipStream_t s) {
  switch (kind) {
    case 1: hipLaunchKernelGGL((k_fb_coarse<D, L, false>), dim3(grid), dim3(kFbCoarseThreads), 0, s, a, f); break;
    case 2: hipLaunchKernelGGL((k_fb_coarse<D, L, true>), dim3(grid), dim3(kFbCoarseThreads), 0, s, a, f); break;
    case 3:
      if (lds > sizeof(float) * (size_t)coarse_lds_floats(kCoarseMaxBlock))
        hipLaunchKernelGGL((k_lp_coarse<D, L, kCoarseMaxBlockBig>), dim3(grid), dim3(kCoarseThreads), 0, s, a, f);
      else
        hipLaunchKernelGGL((k_lp_coarse<D, L, kCoarseMaxBlock>), dim3(grid), dim3(kCoarseThreads), 0, s, a, f);
      break;
    default: return hipErrorInvalidValue;  // kind 0 (first low-pass tail) was removed
  }
  return hipGetLastError();
}

template <int D>
hipError_t launch_tail_d(int kind, int taps, const TailArgs& a, int grid, size_t lds, const Filter& f,
                         hipStream_t s) {
  switch (taps) {
    case 2: return launch_tail_dl<D, 2>(kind, a, grid, lds, f, s);
    case 4: return launch_tail_dl<D, 4>(kind, a, grid, lds, f, s);
    case 6: return launch_tail_dl<D, 6>(kind, a, grid, lds, f, s);
    case 8: return launch_tail_dl<D, 8>(kind, a, grid, lds, f, s);
    case 10: return launch_tail_dl<D, 10>(kind, a, grid, lds, f, s);
    case 12: return launch_tail_dl<D, 12>(kind, a, grid, lds, f, s);
    case 14: return launch_tail_dl<D, 14>(kind, a, grid, lds, f, s);
    case 16: return launch_tail_dl<D, 16>(kind, a, grid, lds, f, s);
  }
  return hipErrorInvalidValue;
}

template <int L>
hipError_t launch_plain_l(const PlainPass& p, const Filter& f, hipStream_t s) {
  int hb[3] = {p.b[0], p.b[1], p.b[2]};
  hb[p.axis] >>= 1;
  const int64_t total = (int64_t)hb[0] * hb[1] * hb[2];
  const int64_t grid = (total + 255) / 256;
  hipLaunchKernelGGL((k_plain_pass<L>), dim3((unsigned)grid), dim3(256), 0, s, p, f);
  return hipGetLastError();
}

template <int L, int V>
hipError_t launch_cge_lv(const TaskArgs& a, int grid, const Filter& f, hipStream_t s) {
  hipLaunchKernelGGL((k_lp_up_cge<L, shape_of(K_LP_UP, 2, V, L).b, shape_of(K_LP_UP, 2, V, L).c, kThreads>), dim3(grid),
                     dim3(kThreads), 0, s, a, f);
  return hipGetLastError();
}

template <int L>
hipError_t launch_cge_l(int variant, const TaskArgs& a, int grid, const Filter& f, hipStream_t s) {
  if (variant == 0) return launch_cge_lv<L, 0>(a, grid, f, s);
  if (variant == 2) return launch_cge_lv<L, 2>(a, grid, f, s);
  return launch_cge_lv<L, 1>(a, grid, f, s);
}

}  // namespace

hipError_t launch_lp_up_cge(int taps, int variant, const TaskArgs& a, int grid, const Filter& f, hipStream_t s) {
  switch (taps) {
    case 2: return launch_cge_l<2>(variant, a, grid, f, s);
    case 4: return launch_cge_l<4>(variant, a, grid, f, s);
    case 6: return launch_cge_l<6>(variant, a, grid, f, s);
    case 8: return launch_cge_l<8>(variant, a, grid, f, s);
    case 10: return launch_cge_l<10>(variant, a, grid, f, s);
    case 12: return launch_cge_l<12>(variant, a, grid, f, s);
    case 14: return launch_cge_l<14>(variant, a, grid, f, s);
    case 16: return launch_cge_l<16>(variant, a, grid, f, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_level(int kind, int ndim, int taps, int variant, const TaskArgs& args, int grid, const Filter& f,
                        hipStream_t stream) {
  // the vector path needs 16-byte rows; the host decides per launch (all tasks agree)
  const bool vec = args.vec != 0;
  switch (kind) {
    case K_LP_DOWN: return launch_k<K_LP_DOWN>(ndim, taps, variant, vec, args, grid, f, stream);
    case K_LP_UP: return launch_k<K_LP_UP>(ndim, taps, variant, vec, args, grid, f, stream);
    case K_FB_DOWN: return launch_k<K_FB_DOWN>(ndim, taps, variant, vec, args, grid, f, stream);
    case K_FB_UP: return launch_k<K_FB_UP>(ndim, taps, variant, vec, args, grid, f, stream);
    case K_LP_UP2:
      if (ndim != 2) return hipErrorInvalidValue;
      return launch_kd<K_LP_UP2, 2>(taps, variant, vec, args, grid, f, stream);
    case K_LP_DOWN_S:
      if (ndim == 3) return launch_kd<K_LP_DOWN_S, 3>(taps, variant, vec, args, grid, f, stream);
      if (ndim != 2) return hipErrorInvalidValue;
      return launch_kd<K_LP_DOWN_S, 2>(taps, variant, vec, args, grid, f, stream);
    case K_LP_UP_S:
      if (ndim != 3) return hipErrorInvalidValue;
      return launch_kd<K_LP_UP_S, 3>(taps, variant, vec, args, grid, f, stream);
    case K_FB_DOWN_S:
      if (ndim != 3) return hipErrorInvalidValue;
      return launch_kd<K_FB_DOWN_S, 3>(taps, variant, vec, args, grid, f, stream);
    case K_FB_UP_S:
      if (ndim != 3) return hipErrorInvalidValue;
      return launch_kd<K_FB_UP_S, 3>(taps, variant, vec, args, grid, f, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tail(int kind, int ndim, int taps, const TailArgs& args, int grid, size_t lds_bytes,
                       const Filter& f, hipStream_t stream) {
  switch (ndim) {
    case 1: return launch_tail_d<1>(kind, taps, args, grid, lds_bytes, f, stream);
    case 2: return launch_tail_d<2>(kind, taps, args, grid, lds_bytes, f, stream);
    case 3: return launch_tail_d<3>(kind, taps, args, grid, lds_bytes, f, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_plain_pass(const PlainPass& p, int taps, const Filter& f, hipStream_t s) {
  switch (taps) {
    case 2: return launch_plain_l<2>(p, f, s);
    case 4: return launch_plain_l<4>(p, f, s);
    case 6: return launch_plain_l<6>(p, f, s);
    case 8: return launch_plain_l<8>(p, f, s);
    case 10: return launch_plain_l<10>(p, f, s);
    case 12: return launch_plain_l<12>(p, f, s);
    case 14: return launch_plain_l<14>(p, f, s);
    case 16: return launch_plain_l<16>(p, f, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_block_copy(const float* src, float* dst, const int b[3], const int st_src[2], const int st_dst[2],
                             hipStream_t s) {
  const int64_t total = (int64_t)b[0] * b[1] * b[2];
  hipLaunchKernelGGL(k_block_copy, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, b[0], b[1], b[2],
                     st_src[0], st_src[1], st_dst[0], st_dst[1]);
  return hipGetLastError();
}

hipError_t launch_norm_finalize(const float2* partials, const NormSegs& segs, float* out, int64_t batch,
                                hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norm_finalize, dim3((unsigned)batch), dim3(256), 0, s, partials, segs, out);
  return hipGetLastError();
}

hipError_t launch_sumsq(const float* x, int64_t n, int64_t batch, float* out, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sumsq, dim3((unsigned)batch), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, int64_t n, hipStream_t s) {
  // n is a multiple of 4 and both pointers 16-byte aligned (checked by the caller)
  const int64_t n4 = n / 4;
  int64_t grid = (n4 + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<const float4*>(src),
                     reinterpret_cast<float4*>(dst), n4);
  return hipGetLastError();
}

}  // namespace es
