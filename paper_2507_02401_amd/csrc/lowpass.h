// Low-pass (projection-form) tile and coarse-level bodies: the work of one work-group, used by
// the level kernels (one launch per level) and by the persistent plan kernel alike, so that
// both give identical results.
#pragma once

#include "kcommon.h"
#include "tiles.h"

namespace es {

// ---------------------------------------------------------------------------------------
// LP_DOWN: a_out = A a_in on a (T0,T1,T2) tile of the half-resolution output.

// LDS of one LP_DOWN tile.
template <int D, int L, int T0, int T1, int T2>
struct LpDownSmem {
  using G = DownGeom<D, L, T0, T1, T2>;
  alignas(16) float s_in[G::NROW * G::I2P];
  float s_b[D >= 3 ? T0 * G::I1 * T2 : 1];
  int s_row[G::NROW];
  int s_col[G::NV];
};

// One LP_DOWN tile: work-group index `wg` of task `t` (decoded with the task's tile counts).
template <int D, int L, int T0, int T1, int T2, int NT, bool VEC>
DEVI void lp_down_tile(const Task& t, int wg, const Filter& f, LpDownSmem<D, L, T0, T1, T2>& sm) {
  using G = DownGeom<D, L, T0, T1, T2>;
  constexpr int P2 = 4, P1 = 4, P0 = 2;
  float* s_in = sm.s_in;
  float* s_b = sm.s_b;
  int* s_row = sm.s_row;
  int* s_col = sm.s_col;
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ src = t.in0 + tl.inst * t.bs_in0;
  float* __restrict__ dst = t.out0 + tl.inst * t.bs_out0;
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

  // contiguous dim: (NROW, I2) -> (NROW, T2); results go through registers so that s_a can
  // reuse the staging buffer (smaller LDS footprint, more resident work-groups)
  float* s_a = s_in;
  row_pass_inplace<L, P2, G::NROW, T2, G::I2P, NT, false>(s_in, f);

  const int n1o = b1 >> 1, n2o = b2 >> 1, n0o = b0 >> 1;
  if constexpr (D == 1) {
    // already the output: (1, T2)
    for (int k = threadIdx.x; k < T2; k += NT) {
      const int g2 = T2 * tl.c2 + k;
      if (g2 < n2o) gst(dst + g2, s_a[k]);
    }
  } else if constexpr (D == 2) {
    analysis_pass<L, P1, false, true, NT>(
        T2, T1 / P1, f,
        [&](int c, int j0, float* w) {
#pragma unroll
          for (int j = 0; j < 2 * P1 + L - 2; ++j) w[j] = s_a[(j0 + j) * T2 + c];
        },
        [&](int c, int k, float lo, float) {
          const int g1 = T1 * tl.c1 + k, g2 = T2 * tl.c2 + c;
          if (g1 < n1o && g2 < n2o) gst(dst + g1 * n2o + g2, lo);
        });
  } else {
    // dim 0: (I0, I1, T2) -> (T0, I1, T2), lines are (i1, c)
    analysis_pass<L, P0, false, true, NT>(
        G::I1 * T2, T0 / P0, f,
        [&](int l, int j0, float* w) {
#pragma unroll
          for (int j = 0; j < 2 * P0 + L - 2; ++j) w[j] = s_a[(j0 + j) * G::I1 * T2 + l];
        },
        [&](int l, int k, float lo, float) { s_b[k * G::I1 * T2 + l] = lo; });
    __syncthreads();
    // dim 1: (T0, I1, T2) -> (T0, T1, T2), lines are (k0, c)
    analysis_pass<L, P1, false, true, NT>(
        T0 * T2, T1 / P1, f,
        [&](int l, int j0, float* w) {
          const int c = l % T2, k0 = l / T2;
#pragma unroll
          for (int j = 0; j < 2 * P1 + L - 2; ++j) w[j] = s_b[(k0 * G::I1 + j0 + j) * T2 + c];
        },
        [&](int l, int k, float lo, float) {
          const int c = l % T2, k0 = l / T2;
          const int g0 = T0 * tl.c0 + k0, g1 = T1 * tl.c1 + k, g2 = T2 * tl.c2 + c;
          if (g0 < n0o && g1 < n1o && g2 < n2o) gst(dst + (g0 * n1o + g1) * n2o + g2, lo);
        });
  }
}

// ---------------------------------------------------------------------------------------
// LP_DOWN streamed along axis 1 (2-D): a_out = A a_in for a strip of T2 output columns and a
// run of R output rows per work-group.  The run's input rows are visited in chunks of CR = 2 RB
// rows; each row is filtered along axis 2 exactly once, into a ring holding the last W = CR + L - 2
// filtered rows (the rows that RB output rows read), and RB output rows are formed per chunk from
// the ring along axis 1.  Every ring row but the last is also written W rows further on (a
// mirror), so a window of up to W consecutive ring rows never wraps and is read at fixed offsets.
// The next chunk's 16-byte loads are in flight while the current chunk is filtered.  The
// arithmetic per output is that of lp_down_tile (axis 2, then axis 1, taps in order), so both
// give identical results.
template <int L, int R, int T2, int RB>
struct LpDownStreamGeom {
  static constexpr int CR = 2 * RB;                          // input rows per chunk
  static constexpr int W = CR + L - 2;                       // ring rows the outputs of a chunk read
  static constexpr int NRING = 2 * W - 1;                    // with the mirror
  static constexpr int NC = (2 * R + L - 2 + CR - 1) / CR;   // chunks of a run
  static constexpr int I2 = 2 * T2 + L - 2;
  static constexpr int I2P = (I2 + 3) & ~3;
  static constexpr int NV = I2P / 4;
};

template <int L, int R, int T2, int RB>
struct LpDownStreamSmem {
  using G = LpDownStreamGeom<L, R, T2, RB>;
  alignas(16) float s_in[G::CR * G::I2P];
  alignas(16) float s_ring[G::NRING * T2];
  int s_row[G::NC * G::CR];
  int s_col[G::NV];
};

template <int L, int R, int T2, int RB, int NT, bool VEC>
DEVI void lp_down_stream(const Task& t, int wg, const Filter& f, LpDownStreamSmem<L, R, T2, RB>& sm) {
  using G = LpDownStreamGeom<L, R, T2, RB>;
  constexpr int CR = G::CR, W = G::W, NC = G::NC, I2P = G::I2P, NV = G::NV;
  constexpr int P = 4, NCH = T2 / P;              // axis-2 pass: P outputs per task
  constexpr int CPT = NT / T2 > 0 ? NT / T2 : 1;  // axis-1 pass: tasks per column
  constexpr int RPT = RB / CPT;                   // output rows per axis-1 task
  constexpr int WC = 2 * RPT + L - 2;             // ring rows one axis-1 task reads
  static_assert(T2 % P == 0 && RB % CPT == 0 && RPT >= 1 && WC <= W, "tile shape");
  float* s_in = sm.s_in;
  float* s_ring = sm.s_ring;
  int* s_row = sm.s_row;
  int* s_col = sm.s_col;
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ src = t.in0 + tl.inst * t.bs_in0;
  float* __restrict__ dst = t.out0 + tl.inst * t.bs_out0;
  const int b1 = t.b[1], b2 = t.b[2];
  const int h1 = b1 >> 1, h2 = b2 >> 1;
  const int k0 = R * tl.c1, o2 = 2 * T2 * tl.c2;
  for (int i = threadIdx.x; i < NC * CR; i += NT) s_row[i] = pmod(2 * k0 + i, b1) * t.st_in0[1];
  for (int i = threadIdx.x; i < NV; i += NT) s_col[i] = VEC ? pmod(o2 + 4 * i, b2) : o2 + 4 * i;
  __syncthreads();

  constexpr int NLD = CR * NV, ITL = (NLD + NT - 1) / NT;
  float4 pf[VEC ? ITL : 1];
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int it = 0; it < ITL; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, NLD - 1);
      pf[it] = gld4(src + s_row[c * CR + q / NV] + s_col[q % NV]);
    }
  };
  if constexpr (VEC) load_chunk(0);

  for (int c = 0; c < NC; ++c) {
    if constexpr (VEC) {
      float4* d4 = reinterpret_cast<float4*>(s_in);  // row length I2P = 4 NV: LDS slot = load index
#pragma unroll
      for (int it = 0; it < ITL; ++it) d4[min(int(threadIdx.x) + it * NT, NLD - 1)] = pf[it];
      __syncthreads();
      if (c + 1 < NC) load_chunk(c + 1);
    } else {
      stage_rows<NT, CR, NV, false>(src, s_row + c * CR, s_col, s_in, I2P, b2);
      __syncthreads();
    }
    // axis 2: the chunk's rows into their ring slots (and mirrors)
    const int sb = (c * CR) % W;
    for (int task = threadIdx.x; task < CR * NCH; task += NT) {
      const int ch = task % NCH, r = task / NCH;
      constexpr int WN = 2 * P + L - 2, W4 = (WN + 3) / 4;
      const float4* p4 = reinterpret_cast<const float4*>(s_in + r * I2P + 2 * P * ch);
      float win[4 * W4];
#pragma unroll
      for (int v = 0; v < W4; ++v) {
        const float4 x = p4[v];
        win[4 * v] = x.x; win[4 * v + 1] = x.y; win[4 * v + 2] = x.z; win[4 * v + 3] = x.w;
      }
      float a[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        a[q] = 0.f;
#pragma unroll
        for (int tt = 0; tt < L; ++tt) a[q] = fmaf(f.h[tt], win[2 * q + tt], a[q]);
      }
      const float4 o = make_float4(a[0], a[1], a[2], a[3]);
      const int slot = sb + r >= W ? sb + r - W : sb + r;
      *reinterpret_cast<float4*>(s_ring + slot * T2 + P * ch) = o;
      if (slot < W - 1) *reinterpret_cast<float4*>(s_ring + (slot + W) * T2 + P * ch) = o;
    }
    __syncthreads();
    // axis 1: output rows kb .. kb + RB - 1 of the run (input rows 2 kb .. 2 kb + W - 1)
    const int kb = RB * c - (L / 2 - 1);
    if (kb + RB > 0) {
      for (int task = threadIdx.x; task < T2 * CPT; task += NT) {
        const int col = task % T2, part = task / T2;
        const int kp = kb + RPT * part;
        const float* rp = s_ring + pmod(2 * kp, W) * T2 + col;
        float win[WC];
#pragma unroll
        for (int j = 0; j < WC; ++j) win[j] = rp[j * T2];
        const int g2 = T2 * tl.c2 + col;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          float a = 0.f;
#pragma unroll
          for (int tt = 0; tt < L; ++tt) a = fmaf(f.h[tt], win[2 * r + tt], a);
          const int k = kp + r;
          if (k >= 0 && k < R && k0 + k < h1 && g2 < h2) gst(dst + (k0 + k) * h2 + g2, a);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// LP_UP: out = alpha*same + beta*(A^T z) on a (U0,U1,U2) full-resolution tile.

// LDS of one LP_UP tile.
template <int D, int L, int U0, int U1, int U2>
struct LpUpSmem {
  using G = UpGeom<D, L, U0, U1, U2>;
  alignas(16) float s_in[G::NROW * G::J2P];
  alignas(16) float s_a[G::NROW * U2];
  float s_b[D >= 3 ? U0 * G::J1 * U2 : 1];
  int s_row[G::NROW];
  int s_col[G::NV];
};

// One LP_UP tile: work-group index `wg` of task `t`.
// CGE (2-D vector path only; the conjugate-gradient solver's operator step): the output is
// out = (alpha + gamma * m) * same + beta * (A^T z) with m = in2 (a per-element mask), and the
// work-group's compensated sum of same * out goes to out1[wg - tile_begin] (one float).
template <int D, int L, int U0, int U1, int U2, int NT, bool VEC, bool CGE = false>
DEVI void lp_up_tile(const Task& t, int wg, const Filter& f, LpUpSmem<D, L, U0, U1, U2>& sm) {
  using G = UpGeom<D, L, U0, U1, U2>;
  constexpr int H = G::H;
  constexpr int P2 = 4, P1 = 4, P0 = 2;
  float* s_in = sm.s_in;
  float* s_a = sm.s_a;
  float* s_b = sm.s_b;
  int* s_row = sm.s_row;
  int* s_col = sm.s_col;
  const Tile tl = decode_tile(t, wg);
  const float* __restrict__ z = t.in0 + tl.inst * t.bs_in0;
  const float* same = t.in1 + tl.inst * t.bs_in1;  // may alias out (in-place z over a)
  float* out = t.out0 + tl.inst * t.bs_out0;
  const int b0 = t.b[0], b1 = t.b[1], b2 = t.b[2];
  const int h0 = b0 >> 1, h1 = b1 >> 1, h2 = b2 >> 1;  // z dims
  const int r0 = tl.c0 * (U0 / 2) - (H - 1), r1 = tl.c1 * (U1 / 2) - (H - 1);
  const int r2 = tl.c2 * (U2 / 2) - (H - 1) - G::OFF;

  // 2-D vector path: the last pass gives each lane 4 adjacent columns and PQ row pairs; the
  // lane's `same` values are loaded first, so that their latency overlaps the staging and
  // filtering of z (same has no halo: each work-group reads and writes only its own tile)
  constexpr int C4 = U2 / 4, PQ = 2;
  constexpr bool FAST2 = D == 2 && VEC && (U1 / 2) % PQ == 0;
  constexpr int NT2 = C4 * (U1 / 2 / PQ), IT2 = (NT2 + NT - 1) / NT;
  static_assert(!CGE || FAST2, "the solver epilogue exists on the 2-D vector path only");
  float4 xs[FAST2 ? IT2 : 1][FAST2 ? 2 * PQ : 1];
  float4 ms[CGE ? IT2 : 1][CGE ? 2 * PQ : 1];
  const float* mask = CGE && t.in2 ? t.in2 + tl.inst * t.bs_in2 : nullptr;  // the same for the whole launch
  if constexpr (FAST2) {
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int task = threadIdx.x + it * NT;
      const int c4 = task % C4, ch = task / C4;
      const int g2 = tl.c2 * U2 + 4 * c4;
#pragma unroll
      for (int r = 0; r < 2 * PQ; ++r) {
        const int g1 = tl.c1 * U1 + 2 * PQ * ch + r;
        const bool in = task < NT2 && g1 < b1 && g2 < b2;
        xs[it][r] = in ? gld4(same + g1 * b2 + g2) : make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (CGE) ms[it][r] = in && mask ? gld4(mask + g1 * b2 + g2) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }
  KSum cg_acc;

  for (int i = threadIdx.x; i < G::NROW; i += NT) {
    const int i1 = i % G::J1, i0 = i / G::J1;
    s_row[i] = (D >= 3 ? pmod(r0 + i0, h0) * (h1 * h2) : 0) + (D >= 2 ? pmod(r1 + i1, h1) * h2 : 0);
  }
  for (int i = threadIdx.x; i < G::NV; i += NT) s_col[i] = VEC ? pmod(r2 + 4 * i, h2) : r2 + 4 * i;
  __syncthreads();
  stage_rows<NT, G::NROW, G::NV, VEC>(z, s_row, s_col, s_in, G::J2P, h2);
  __syncthreads();

  // contiguous dim: (NROW, J2) -> (NROW, U2)
  synthesis_pass<L, P2, false, false, NT>(
      G::NROW, U2 / 2 / P2, f,
      [&](int l, int j0, float* lo, float*) {
        const float* p = s_in + l * G::J2P + G::OFF + j0;
#pragma unroll
        for (int j = 0; j < P2 + H - 1; ++j) lo[j] = p[j];
      },
      [&](int l, int p, float e0, float e1) {
        s_a[l * U2 + p] = e0;
        s_a[l * U2 + p + 1] = e1;
      });
  __syncthreads();

  const float alpha = t.alpha, beta = t.beta;
  if constexpr (D == 1) {
    for (int p = threadIdx.x; p < U2; p += NT) {
      const int g2 = tl.c2 * U2 + p;
      if (g2 < b2) gst(out + g2, fmaf(alpha, gld(same + g2), beta * s_a[p]));
    }
  } else if constexpr (FAST2) {
    // axis 1 with 4 columns per lane: float4 LDS reads, float4 global stores; per output the
    // arithmetic of synthesis_pass (oldest window sample first)
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int task = threadIdx.x + it * NT;
      if (task < NT2) {
        const int c4 = task % C4, ch = task / C4;
        const int g2 = tl.c2 * U2 + 4 * c4;
        float4 lo[PQ + H - 1];
#pragma unroll
        for (int j = 0; j < PQ + H - 1; ++j) lo[j] = *reinterpret_cast<const float4*>(s_a + (PQ * ch + j) * U2 + 4 * c4);
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          float4 e0 = make_float4(0.f, 0.f, 0.f, 0.f), e1 = e0;
#pragma unroll
          for (int j = H - 1; j >= 0; --j) {
            const float4 v = lo[q + H - 1 - j];
            e0.x = fmaf(f.h[2 * j], v.x, e0.x); e1.x = fmaf(f.h[2 * j + 1], v.x, e1.x);
            e0.y = fmaf(f.h[2 * j], v.y, e0.y); e1.y = fmaf(f.h[2 * j + 1], v.y, e1.y);
            e0.z = fmaf(f.h[2 * j], v.z, e0.z); e1.z = fmaf(f.h[2 * j + 1], v.z, e1.z);
            e0.w = fmaf(f.h[2 * j], v.w, e0.w); e1.w = fmaf(f.h[2 * j + 1], v.w, e1.w);
          }
          const int g1 = tl.c1 * U1 + 2 * (PQ * ch + q);
          if (g1 < b1 && g2 < b2) {
            const float4 s0 = xs[it][2 * q], s1 = xs[it][2 * q + 1];
            if constexpr (CGE) {
              const float gm = t.gamma;
              const float4 m0 = ms[it][2 * q], m1 = ms[it][2 * q + 1];
              const float4 y0 = make_float4(
                  fmaf(fmaf(gm, m0.x, alpha), s0.x, beta * e0.x), fmaf(fmaf(gm, m0.y, alpha), s0.y, beta * e0.y),
                  fmaf(fmaf(gm, m0.z, alpha), s0.z, beta * e0.z), fmaf(fmaf(gm, m0.w, alpha), s0.w, beta * e0.w));
              const float4 y1 = make_float4(
                  fmaf(fmaf(gm, m1.x, alpha), s1.x, beta * e1.x), fmaf(fmaf(gm, m1.y, alpha), s1.y, beta * e1.y),
                  fmaf(fmaf(gm, m1.z, alpha), s1.z, beta * e1.z), fmaf(fmaf(gm, m1.w, alpha), s1.w, beta * e1.w));
              gst4(out + g1 * b2 + g2, y0);
              gst4(out + (g1 + 1) * b2 + g2, y1);
              cg_acc.add(s0.x * y0.x); cg_acc.add(s0.y * y0.y); cg_acc.add(s0.z * y0.z); cg_acc.add(s0.w * y0.w);
              cg_acc.add(s1.x * y1.x); cg_acc.add(s1.y * y1.y); cg_acc.add(s1.z * y1.z); cg_acc.add(s1.w * y1.w);
            } else {
              const float4 y0 = make_float4(fmaf(alpha, s0.x, beta * e0.x), fmaf(alpha, s0.y, beta * e0.y),
                                            fmaf(alpha, s0.z, beta * e0.z), fmaf(alpha, s0.w, beta * e0.w));
              const float4 y1 = make_float4(fmaf(alpha, s1.x, beta * e1.x), fmaf(alpha, s1.y, beta * e1.y),
                                            fmaf(alpha, s1.z, beta * e1.z), fmaf(alpha, s1.w, beta * e1.w));
              gst4(out + g1 * b2 + g2, y0);
              gst4(out + (g1 + 1) * b2 + g2, y1);
            }
          }
        }
      }
    }
  } else if constexpr (D == 2) {
    synthesis_pass<L, P1, false, true, NT>(
        U2, U1 / 2 / P1, f,
        [&](int c, int j0, float* lo, float*) {
#pragma unroll
          for (int j = 0; j < P1 + H - 1; ++j) lo[j] = s_a[(j0 + j) * U2 + c];
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
  } else {
    // dim 0: (J0, J1, U2) -> (U0, J1, U2)
    synthesis_pass<L, P0, false, true, NT>(
        G::J1 * U2, U0 / 2 / P0, f,
        [&](int l, int j0, float* lo, float*) {
#pragma unroll
          for (int j = 0; j < P0 + H - 1; ++j) lo[j] = s_a[(j0 + j) * G::J1 * U2 + l];
        },
        [&](int l, int p, float e0, float e1) {
          s_b[p * G::J1 * U2 + l] = e0;
          s_b[(p + 1) * G::J1 * U2 + l] = e1;
        });
    __syncthreads();
    synthesis_pass<L, P1, false, true, NT>(
        U0 * U2, U1 / 2 / P1, f,
        [&](int l, int j0, float* lo, float*) {
          const int c = l % U2, p0 = l / U2;
#pragma unroll
          for (int j = 0; j < P1 + H - 1; ++j) lo[j] = s_b[(p0 * G::J1 + j0 + j) * U2 + c];
        },
        [&](int l, int p, float e0, float e1) {
          const int c = l % U2, p0 = l / U2;
          const int g0 = tl.c0 * U0 + p0, g1 = tl.c1 * U1 + p, g2 = tl.c2 * U2 + c;
          if (g0 < b0 && g1 < b1 && g2 < b2) {
            const int o = (g0 * b1 + g1) * b2 + g2;
            const float s0 = gld(same + o), s1 = gld(same + o + b2);
            gst(out + o, fmaf(alpha, s0, beta * e0));
            gst(out + o + b2, fmaf(alpha, s1, beta * e1));
          }
        });
  }
  if constexpr (CGE) {
    __shared__ float2 cg_sum;
    store_wg_sum<NT>(cg_acc, &cg_sum);  // every thread; thread 0 holds the pair
    if (threadIdx.x == 0) gst(t.out1 + (wg - t.tile_begin), cg_sum.x + cg_sum.y);
  }
}

// ---------------------------------------------------------------------------------------
// LP_COARSE: the coarse levels of the projection form for one instance in one work-group.
// Input a_T (a contiguous block of at most CMAX floats), output z_T in place (or y when
// T = 0).  Everything between the load and the store stays in a static LDS array addressed by
// integer offsets: A_0 = a_T, A_1 = a_{T+1}, ..., A_K, then two half-size temporaries.
//   down:  A_{j+1} = A A_j                       (separable, contiguous axis first)
//   top:   A_K *= c_{T+K}
//   up:    A_j = coef_j A_j + A^T A_{j+1}        (j = K-1 .. 0; coef_0 is the output weight)
// Axes at least L long wrap with one compare; shorter ones use the modulo (periodic folding).


template <int L, bool SHORT>
DEVI void coarse_analysis_w(float* sm, int src, int dst, int n0, int n1, int n2, int ax, const Filter& f) {
  // sm[src] holds an (n0, n1, n2) block; writes the low half along ax, (.., n_ax/2, ..), to sm[dst]
  const int n = ax == 0 ? n0 : (ax == 1 ? n1 : n2);
  const int o0 = ax == 0 ? n0 >> 1 : n0, o1 = ax == 1 ? n1 >> 1 : n1, o2 = ax == 2 ? n2 >> 1 : n2;
  const int l1 = ilog2_or_neg(o1), l2 = ilog2_or_neg(o2);
  const int step = ax == 0 ? n1 * n2 : (ax == 1 ? n2 : 1);
  const int total = o0 * o1 * o2;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, o1, o2, l1, l2, c0, c1, c2);
    const int k = ax == 0 ? c0 : (ax == 1 ? c1 : c2);
    const int base = src + (ax == 0 ? 0 : c0 * n1 * n2) + (ax == 1 ? 0 : c1 * n2) + (ax == 2 ? 0 : c2);
    float acc = 0.f;
    if (!SHORT) {  // n >= L: an index wraps at most once
#pragma unroll
      for (int t = 0; t < L; ++t) {
        const int i = 2 * k + t;
        acc = fmaf(f.h[t], sm[base + (i >= n ? i - n : i) * step], acc);
      }
    } else {
#pragma unroll
      for (int t = 0; t < L; ++t) acc = fmaf(f.h[t], sm[base + ((2 * k + t) % n) * step], acc);
    }
    sm[dst + e] = acc;
  }
}

template <int L, bool SHORT>
DEVI void coarse_synthesis_w(float* sm, int src, int dst, int n0, int n1, int n2, int ax, const Filter& f, bool combine,
                             float alpha) {
  // sm[src] holds the low half along ax of an (n0, n1, n2) block; writes the full block to
  // sm[dst] (dst = alpha*dst + value when combine)
  const int n = ax == 0 ? n0 : (ax == 1 ? n1 : n2), half = n >> 1;
  const int h0 = ax == 0 ? half : n0, h1 = ax == 1 ? half : n1, h2 = ax == 2 ? half : n2;
  const int step = ax == 0 ? h1 * h2 : (ax == 1 ? h2 : 1);
  const int total = n0 * n1 * n2;
  const int l1 = ilog2_or_neg(n1), l2 = ilog2_or_neg(n2);
  (void)h0;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, n1, n2, l1, l2, c0, c1, c2);
    const int p = ax == 0 ? c0 : (ax == 1 ? c1 : c2);
    const int base = src + (ax == 0 ? 0 : c0 * h1 * h2) + (ax == 1 ? 0 : c1 * h2) + (ax == 2 ? 0 : c2);
    const int par = p & 1, q = p >> 1;
    float acc = 0.f;
    if (!SHORT) {  // half >= L/2: an index wraps at most once
#pragma unroll
      for (int j = 0; j < L / 2; ++j) {
        const int k = q - j;
        acc = fmaf(par ? f.h[2 * j + 1] : f.h[2 * j], sm[base + (k < 0 ? k + half : k) * step], acc);
      }
    } else {
#pragma unroll
      for (int j = 0; j < L / 2; ++j)
        acc = fmaf(par ? f.h[2 * j + 1] : f.h[2 * j], sm[base + pmod(q - j, half) * step], acc);
    }
    sm[dst + e] = combine ? fmaf(alpha, sm[dst + e], acc) : acc;
  }
}

// Register-window versions: a thread computes PO consecutive outputs along the filtered axis
// from one window of inputs (each input read once per window, its wrap resolved once), with
// the per-output arithmetic of the versions above.  Along the contiguous axis the window is
// read as 16-byte vectors (start and length multiples of 4, so a vector never straddles the
// wrap); along the strided axes lanes run along the contiguous axis (conflict-free LDS).
// Preconditions (checked by the dispatchers): the axis is at least L long (analysis) or its
// half at least L/2 (synthesis), the outputs per line are a multiple of PO, and for the
// contiguous axis the block offset is a multiple of 4.
template <int L>
DEVI void coarse_analysis_v(float* sm, int src, int dst, int n0, int n1, int n2, int ax, const Filter& f) {
  constexpr int PO = 4, WN = 2 * PO + L - 2, W4 = (WN + 3) / 4;
  const int n = ax == 0 ? n0 : (ax == 1 ? n1 : n2);
  const int o0 = ax == 0 ? n0 >> 1 : n0, o1 = ax == 1 ? n1 >> 1 : n1, o2 = ax == 2 ? n2 >> 1 : n2;
  // item space: the filtered axis counted in chunks of PO outputs
  const int p0 = ax == 0 ? o0 / PO : o0, p1 = ax == 1 ? o1 / PO : o1, p2 = ax == 2 ? o2 / PO : o2;
  const int l1 = ilog2_or_neg(p1), l2 = ilog2_or_neg(p2);
  const int step = ax == 0 ? n1 * n2 : (ax == 1 ? n2 : 1);
  const int ostep = ax == 0 ? o1 * o2 : (ax == 1 ? o2 : 1);
  const int total = p0 * p1 * p2;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, p1, p2, l1, l2, c0, c1, c2);
    const int k0 = PO * (ax == 0 ? c0 : (ax == 1 ? c1 : c2));
    const int base = src + (ax == 0 ? 0 : c0 * n1 * n2) + (ax == 1 ? 0 : c1 * n2) + (ax == 2 ? 0 : c2);
    float win[4 * W4];
    if (ax == 2) {
#pragma unroll
      for (int v = 0; v < W4; ++v) {
        int i = 2 * k0 + 4 * v;
        i = i >= n ? i - n : i;
        const float4 x = *reinterpret_cast<const float4*>(sm + base + i);
        win[4 * v] = x.x; win[4 * v + 1] = x.y; win[4 * v + 2] = x.z; win[4 * v + 3] = x.w;
      }
    } else {
      const int a0 = base + 2 * k0 * step, a0w = a0 - n * step, wrap = n - 2 * k0;
#pragma unroll
      for (int j = 0; j < WN; ++j) win[j] = sm[(j >= wrap ? a0w : a0) + j * step];
    }
    const int ob = dst + (ax == 0 ? k0 : c0) * o1 * o2 + (ax == 1 ? k0 : c1) * o2 + (ax == 2 ? k0 : c2);
#pragma unroll
    for (int q = 0; q < PO; ++q) {
      float acc = 0.f;
#pragma unroll
      for (int t = 0; t < L; ++t) acc = fmaf(f.h[t], win[2 * q + t], acc);
      sm[ob + q * ostep] = acc;
    }
  }
}

template <int L>
DEVI void coarse_synthesis_v(float* sm, int src, int dst, int n0, int n1, int n2, int ax, const Filter& f, bool combine,
                             float alpha) {
  // PO = 8 full-res outputs (4 half-res positions q0 .. q0+3) per thread; the window holds the
  // half-res samples q0 - A .. q0 + 3 with A = L/2 - 1 rounded up to a multiple of 4
  constexpr int H = L / 2, PO = 8, A = (H - 1 + 3) & ~3, WN = A + 4, W4 = WN / 4;
  const int n = ax == 0 ? n0 : (ax == 1 ? n1 : n2), half = n >> 1;
  const int h1 = ax == 1 ? half : n1, h2 = ax == 2 ? half : n2;
  const int p0 = ax == 0 ? n0 / PO : n0, p1 = ax == 1 ? n1 / PO : n1, p2 = ax == 2 ? n2 / PO : n2;
  const int l1 = ilog2_or_neg(p1), l2 = ilog2_or_neg(p2);
  const int step = ax == 0 ? h1 * h2 : (ax == 1 ? h2 : 1);
  const int ostep = ax == 0 ? n1 * n2 : (ax == 1 ? n2 : 1);
  const int total = p0 * p1 * p2;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c0, c1, c2;
    split3(e, p1, p2, l1, l2, c0, c1, c2);
    const int q0 = (PO / 2) * (ax == 0 ? c0 : (ax == 1 ? c1 : c2));
    const int base = src + (ax == 0 ? 0 : c0 * h1 * h2) + (ax == 1 ? 0 : c1 * h2) + (ax == 2 ? 0 : c2);
    float win[WN];
    if (ax == 2) {
#pragma unroll
      for (int v = 0; v < W4; ++v) {
        int k = q0 - A + 4 * v;
        k = k < 0 ? k + half : k;
        const float4 x = *reinterpret_cast<const float4*>(sm + base + k);
        win[4 * v] = x.x; win[4 * v + 1] = x.y; win[4 * v + 2] = x.z; win[4 * v + 3] = x.w;
      }
    } else {
      const int a0 = base + (q0 - A) * step, a0w = a0 + half * step;
#pragma unroll
      for (int j = 0; j < WN; ++j) win[j] = sm[(q0 - A + j < 0 ? a0w : a0) + j * step];
    }
    const int p00 = 2 * q0;
    const int ob = dst + (ax == 0 ? p00 : c0) * n1 * n2 + (ax == 1 ? p00 : c1) * n2 + (ax == 2 ? p00 : c2);
#pragma unroll
    for (int r = 0; r < PO; ++r) {
      const int par = r & 1, qq = r >> 1;  // output 2 (q0 + qq) + par
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < H; ++j) acc = fmaf(f.h[2 * j + par], win[A + qq - j], acc);
      const int o = ob + r * ostep;
      sm[o] = combine ? fmaf(alpha, sm[o], acc) : acc;
    }
  }
}

// Uniform dispatch: register-window version where its preconditions hold, else one output per
// thread with single-wrap or modulo (axis shorter than the filter: periodic folding) indexing.
template <int L>
DEVI void coarse_analysis(float* sm, int src, int dst, int n0, int n1, int n2, int ax, const Filter& f) {
  const int n = ax == 0 ? n0 : (ax == 1 ? n1 : n2);
  if (n >= L && (n >> 1) % 4 == 0 && (ax != 2 || src % 4 == 0)) coarse_analysis_v<L>(sm, src, dst, n0, n1, n2, ax, f);
  else if (n >= L) coarse_analysis_w<L, false>(sm, src, dst, n0, n1, n2, ax, f);
  else coarse_analysis_w<L, true>(sm, src, dst, n0, n1, n2, ax, f);
}
template <int L>
DEVI void coarse_synthesis(float* sm, int src, int dst, int n0, int n1, int n2, int ax, const Filter& f, bool combine,
                           float alpha) {
  const int half = (ax == 0 ? n0 : (ax == 1 ? n1 : n2)) >> 1;
  if (half >= L / 2 && half % 4 == 0 && (ax != 2 || src % 4 == 0))
    coarse_synthesis_v<L>(sm, src, dst, n0, n1, n2, ax, f, combine, alpha);
  else if (half >= L / 2) coarse_synthesis_w<L, false>(sm, src, dst, n0, n1, n2, ax, f, combine, alpha);
  else coarse_synthesis_w<L, true>(sm, src, dst, n0, n1, n2, ax, f, combine, alpha);
}


// Every coarse level of instance `inst` of tail task `tp` in one work-group of NT threads; `sm`
// holds coarse_lds_floats(CMAX) floats of LDS (16-byte aligned).
template <int D, int L, int CMAX, int NT>
DEVI void lp_coarse_block(const TailTask* tp, int inst, const Filter& f, float* sm) {
  const float* in = tp->in + inst * tp->bs_in;
  float* out = tp->out + inst * tp->bs_out;
  const int K = tp->nlev;
  const int m0 = tp->b[0], m1 = tp->b[1], m2 = tp->b[2];
  const int B = m0 * m1 * m2;
  // offsets of A_0 .. A_K, then the temporaries
  int tmpA = 0;
  for (int j = 0; j <= K; ++j) tmpA += B >> (D * j);
  const int tmpB = tmpA + (B >> 1);
  gather_to_lds<NT, CMAX / NT>(
      B, [&](int e) { return gld(in + e); }, [&](int e, float v) { sm[e] = v; });
  __syncthreads();
  int off = 0;
  for (int j = 0; j < K; ++j) {
    const int a0 = D >= 3 ? m0 >> j : 1, a1 = D >= 2 ? m1 >> j : 1, a2 = m2 >> j;
    const int nxt = off + a0 * a1 * a2;
    if (D == 1) {
      coarse_analysis<L>(sm, off, nxt, a0, a1, a2, 2, f);
    } else if (D == 2) {
      coarse_analysis<L>(sm, off, tmpA, a0, a1, a2, 2, f);
      __syncthreads();
      coarse_analysis<L>(sm, tmpA, nxt, a0, a1, a2 >> 1, 1, f);
    } else {
      coarse_analysis<L>(sm, off, tmpA, a0, a1, a2, 2, f);
      __syncthreads();
      coarse_analysis<L>(sm, tmpA, tmpB, a0, a1, a2 >> 1, 1, f);
      __syncthreads();
      coarse_analysis<L>(sm, tmpB, nxt, a0, a1 >> 1, a2 >> 1, 0, f);
    }
    __syncthreads();
    off = nxt;
  }
  {
    const int sz = B >> (D * K);
    const float ck = tp->coef[K];
    for (int e = threadIdx.x; e < sz; e += blockDim.x) sm[off + e] *= ck;
  }
  __syncthreads();
  for (int j = K - 1; j >= 0; --j) {
    const int a0 = D >= 3 ? m0 >> j : 1, a1 = D >= 2 ? m1 >> j : 1, a2 = m2 >> j;  // output block
    const int cur = off - a0 * a1 * a2;  // A_j precedes A_{j+1}
    const float alpha = tp->coef[j];
    if (D == 1) {
      coarse_synthesis<L>(sm, off, cur, a0, a1, a2, 2, f, true, alpha);
    } else if (D == 2) {
      // contiguous axis first: (a1/2, a2/2) -> (a1/2, a2) in tmpA, then rows -> A_j
      coarse_synthesis<L>(sm, off, tmpA, a0, a1 >> 1, a2, 2, f, false, 0.f);
      __syncthreads();
      coarse_synthesis<L>(sm, tmpA, cur, a0, a1, a2, 1, f, true, alpha);
    } else {
      coarse_synthesis<L>(sm, off, tmpA, a0 >> 1, a1 >> 1, a2, 2, f, false, 0.f);
      __syncthreads();
      coarse_synthesis<L>(sm, tmpA, tmpB, a0 >> 1, a1, a2, 1, f, false, 0.f);
      __syncthreads();
      coarse_synthesis<L>(sm, tmpB, cur, a0, a1, a2, 0, f, true, alpha);
    }
    __syncthreads();
    off = cur;
  }
  for (int e = threadIdx.x; e < B; e += blockDim.x) gst(out + e, sm[e]);
}

}  // namespace es
