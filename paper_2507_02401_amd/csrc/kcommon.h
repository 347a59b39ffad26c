// Device helpers shared by every kernel of the library: global-memory accessors, LDS staging,
// work-group to tile mapping and the register-window filter passes.
#pragma once

#include "internal.h"

namespace es {


#define DEVI __device__ __forceinline__

DEVI int pmod(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Global-memory accessors.  Array pointers reach the kernels through the task tables, so the
// compiler cannot tell that they address global memory and would emit flat instructions
// (which also occupy the LDS counter and serialise against LDS traffic).  These casts to
// the global address space make every access a global_load / global_store.
#define GAS __attribute__((address_space(1)))
DEVI float gld(const float* p) { return *(const GAS float*)p; }
typedef float f4v __attribute__((ext_vector_type(4)));
DEVI float4 gld4(const float* p) {
  const f4v v = *(const GAS f4v*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
DEVI void gst(float* p, float v) { *(GAS float*)p = v; }
DEVI void gst4(float* p, float4 v) {
  f4v w;
  w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
  *(GAS f4v*)p = w;
}

// Load n (at most U * NT) elements into LDS with every load of a thread issued before the
// first LDS store, so that one work-group keeps U loads per thread in flight.  src(e) gives
// the element's value (a global load), dst(e) its LDS slot.
template <int NT, int U, class Src, class Dst>
DEVI void gather_to_lds(int n, Src src, Dst dst) {
  for (int base = threadIdx.x; base < n; base += U * NT) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT;
      v[u] = e < n ? src(e) : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT;
      if (e < n) dst(e, v[u]);
    }
  }
}

// Error-free sum of two floats (Knuth's TwoSum): s + e == a + b exactly, s = fl(a + b).
DEVI void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated FP32 accumulation (Neumaier's variant of Kahan summation): s + c holds the sum.
struct KSum {
  float s = 0.f, c = 0.f;
  DEVI void add(float v) {
    const float t = s + v;
    c += fabsf(s) >= fabsf(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  // adds another compensated sum: the two leading parts exactly, the compensations plainly
  DEVI void merge(float os, float oc) {
    float t, e;
    two_sum(s, os, t, e);
    s = t;
    c += oc + e;
  }
  DEVI float value() const { return s + c; }
};

// Sum of one compensated sum per thread over the work-group, in a fixed order (pairwise over
// the lanes of each wave, then the waves in index order); thread 0 stores it as a pair
// (leading part, remainder), normalised so that the leading part is the rounded sum.  Every
// thread of the work-group must call it.
template <int NT>
DEVI void store_wg_sum(KSum v, float2* dst) {
  __shared__ float2 part[NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float os = __shfl_down(v.s, o, 64), oc = __shfl_down(v.c, o, 64);
    v.merge(os, oc);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = make_float2(v.s, v.c);
  __syncthreads();
  if (threadIdx.x == 0) {
    KSum t = {part[0].x, part[0].y};
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) t.merge(part[i].x, part[i].y);
    float hi, lo;
    two_sum(t.s, t.c, hi, lo);
    *dst = make_float2(hi, lo);
  }
}

// ---------------------------------------------------------------------------------------
// Work-group -> task/tile mapping.
//
// The hardware hands work-group i to XCD i mod 8.  Remapping gives each XCD a contiguous run
// of logical tiles, so tiles that share filter halos share an L2.
DEVI int logical_wg(int total_wg, int reverse = 0) {
  const int grid = gridDim.x;  // padded to a multiple of 8 by the host
  const int per = grid >> 3;
  const int i = blockIdx.x;
  const int l = (i & 7) * per + (i >> 3);
  if (l >= total_wg) return -1;
  return reverse ? total_wg - 1 - l : l;
}

template <class T, class A>
DEVI T pick_task(const A& args, int wg) {
  if (args.table == nullptr) return args.t0;
  int lo = 0, hi = args.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (args.table[mid].tile_begin <= wg) lo = mid;
    else hi = mid - 1;
  }
  return args.table[lo];
}

struct Tile {
  int inst, c0, c1, c2;
};

DEVI Tile decode_tile(const Task& t, int wg) {
  const int local = wg - t.tile_begin;
  Tile r;
  r.inst = local / t.tiles_per_inst;
  int rem = local - r.inst * t.tiles_per_inst;
  r.c2 = rem % t.ntile[2];
  rem /= t.ntile[2];
  r.c1 = rem % t.ntile[1];
  r.c0 = rem / t.ntile[1];
  return r;
}

// ---------------------------------------------------------------------------------------
// Register-window filter passes over lines of an LDS array.
//
// analysis_pass: line l, chunk ch: window samples s[j] = In(l, 2*P*ch + j), j < 2P+L-2;
// outputs k = P*ch + q:  lo = sum_t h[t] s[2q+t],  hi = sum_t g[t] s[2q+t].
// synthesis_pass: window samples lo/hi In(l, P*ch + j), j < P+L/2-1; outputs p = 2(P*ch+q)+e:
//   x = sum_{j<L/2} h[2j+e] lo[q+L/2-1-j] + g[2j+e] hi[q+L/2-1-j],
// summed from the oldest window sample (j = L/2-1) to the newest (j = 0), the order in which a
// kernel streaming along the axis receives them.
// LINES_FAST puts consecutive lanes on consecutive lines (strided passes: lines are columns
// and LDS accesses are conflict-free); otherwise consecutive lanes take consecutive chunks
// of one line (contiguous pass).

template <int L, int P, bool FB, bool LINES_FAST, int NT, class In, class Out>
DEVI void analysis_pass(int nlines, int nch, const Filter& f, In in, Out out) {
  constexpr int W = 2 * P + L - 2;
  const int ntask = nlines * nch;
  for (int task = threadIdx.x; task < ntask; task += NT) {
    int l, ch;
    if (LINES_FAST) { l = task % nlines; ch = task / nlines; }
    else { ch = task % nch; l = task / nch; }
    float win[W + 3];
    in(l, 2 * P * ch, win);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      float lo = 0.f, hi = 0.f;
#pragma unroll
      for (int t = 0; t < L; ++t) {
        lo = fmaf(f.h[t], win[2 * q + t], lo);
        if (FB) hi = fmaf(f.g[t], win[2 * q + t], hi);
      }
      out(l, P * ch + q, lo, hi);
    }
  }
}

template <int L, int P, bool FB, bool LINES_FAST, int NT, class In, class Out>
DEVI void synthesis_pass(int nlines, int nch, const Filter& f, In in, Out out) {
  constexpr int H = L / 2;
  constexpr int W = P + H - 1;
  const int ntask = nlines * nch;
  for (int task = threadIdx.x; task < ntask; task += NT) {
    int l, ch;
    if (LINES_FAST) { l = task % nlines; ch = task / nlines; }
    else { ch = task % nch; l = task / nch; }
    float lo[W], hi[FB ? W : 1];
    in(l, P * ch, lo, hi);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      float e0 = 0.f, e1 = 0.f;
#pragma unroll
      for (int j = H - 1; j >= 0; --j) {
        const float a = lo[q + H - 1 - j];
        e0 = fmaf(f.h[2 * j], a, e0);
        e1 = fmaf(f.h[2 * j + 1], a, e1);
        if (FB) {
          const float d = hi[q + H - 1 - j];
          e0 = fmaf(f.g[2 * j], d, e0);
          e1 = fmaf(f.g[2 * j + 1], d, e1);
        }
      }
      out(l, 2 * (P * ch + q), e0, e1);
    }
  }
}

// N consecutive floats starting OFFS (< 4) past a 16-byte aligned LDS address, read as whole
// 16-byte vectors: lanes whose windows start 16 bytes apart then read without bank conflicts.
// The vectors cover at most 3 floats past the window, which the caller's row must hold.
template <int N, int OFFS>
DEVI void lds_window(const float* base16, float* w) {
  static_assert(OFFS >= 0 && OFFS < 4, "offset inside the first vector");
  constexpr int W4 = (OFFS + N + 3) / 4;
  const float4* p = reinterpret_cast<const float4*>(base16);
  float t[4 * W4];
#pragma unroll
  for (int v = 0; v < W4; ++v) {
    const float4 x = p[v];
    t[4 * v] = x.x; t[4 * v + 1] = x.y; t[4 * v + 2] = x.z; t[4 * v + 3] = x.w;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) w[j] = t[OFFS + j];
}

// Contiguous-dim analysis of NROW staged rows, results written back over the staging buffer
// as rows of T2 (FB: [lo T2 | hi T2]) floats.  Each task is P consecutive outputs of one row;
// a thread holds its results in registers across the barrier that frees the buffer.
template <int L, int P, int NROW, int T2, int I2P, int NT, bool FB>
DEVI void row_pass_inplace(float* s_in, const Filter& f) {
  constexpr int NCH = T2 / P;
  constexpr int NTASK = NROW * NCH;
  constexpr int IT = (NTASK + NT - 1) / NT;
  constexpr int W = 2 * P + L - 2;
  constexpr int W4 = (W + 3) / 4;
  constexpr int OUTW = FB ? 2 * T2 : T2;
  static_assert(NROW * OUTW <= NROW * I2P, "row results must fit in the staging buffer");
  float lo[IT][P], hi[FB ? IT : 1][P];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int task = threadIdx.x + it * NT;
    if (task < NTASK) {
      const int ch = task % NCH, l = task / NCH;
      const float4* p = reinterpret_cast<const float4*>(s_in + l * I2P + 2 * P * ch);
      float win[4 * W4];
#pragma unroll
      for (int v = 0; v < W4; ++v) {
        const float4 x = p[v];
        win[4 * v] = x.x; win[4 * v + 1] = x.y; win[4 * v + 2] = x.z; win[4 * v + 3] = x.w;
      }
#pragma unroll
      for (int q = 0; q < P; ++q) {
        float a = 0.f, d = 0.f;
#pragma unroll
        for (int t = 0; t < L; ++t) {
          a = fmaf(f.h[t], win[2 * q + t], a);
          if (FB) d = fmaf(f.g[t], win[2 * q + t], d);
        }
        lo[it][q] = a;
        if (FB) hi[it][q] = d;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int task = threadIdx.x + it * NT;
    if (task < NTASK) {
      const int ch = task % NCH, l = task / NCH;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        s_in[l * OUTW + P * ch + q] = lo[it][q];
        if (FB) s_in[l * OUTW + T2 + P * ch + q] = hi[FB ? it : 0][q];
      }
    }
  }
  __syncthreads();
}

// Contiguous-dim analysis of NROW staged rows of `src` into `dst`, as rows of 2 T2 floats
// [lo T2 | hi T2] (FB) or of T2 low-pass floats.  Each task is P consecutive outputs of one row,
// the taps summed in the order of row_pass_inplace.  No barrier: the caller orders the reads of
// `src` and the writes of `dst` against the other threads.
template <int L, int P, int NROW, int T2, int I2P, int NT, bool FB = true>
DEVI void row_pass_to(const float* src, float* dst, const Filter& f) {
  constexpr int NCH = T2 / P;
  constexpr int NTASK = NROW * NCH;
  constexpr int W = 2 * P + L - 2;
  constexpr int W4 = (W + 3) / 4;
  static_assert(P == 4 && T2 % 4 == 0 && I2P % 4 == 0, "16-byte windows and stores");
  for (int task = threadIdx.x; task < NTASK; task += NT) {
    const int ch = task % NCH, l = task / NCH;
    const float4* p = reinterpret_cast<const float4*>(src + l * I2P + 2 * P * ch);
    float win[4 * W4];
#pragma unroll
    for (int v = 0; v < W4; ++v) {
      const float4 x = p[v];
      win[4 * v] = x.x; win[4 * v + 1] = x.y; win[4 * v + 2] = x.z; win[4 * v + 3] = x.w;
    }
    float lo[P], hi[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      float a = 0.f, d = 0.f;
#pragma unroll
      for (int t = 0; t < L; ++t) {
        a = fmaf(f.h[t], win[2 * q + t], a);
        if (FB) d = fmaf(f.g[t], win[2 * q + t], d);
      }
      lo[q] = a;
      hi[q] = d;
    }
    float4* o = reinterpret_cast<float4*>(dst + l * (FB ? 2 * T2 : T2) + P * ch);
    o[0] = make_float4(lo[0], lo[1], lo[2], lo[3]);
    if (FB) o[T2 / 4] = make_float4(hi[0], hi[1], hi[2], hi[3]);
  }
}

// ---------------------------------------------------------------------------------------
// Geometry of a level kernel instantiation.
//
// Analysis kinds tile the half-resolution output: T_k outputs per dim, input region
// I_k = 2 T_k + L - 2 starting at 2 T_k c_k.  Synthesis kinds tile the full-resolution output:
// U_k outputs (even), half-resolution input region J_k = U_k/2 + L/2 - 1 starting at
// c_k U_k/2 - (L/2 - 1).  Dims below 3-D are padded with extent 1 and skipped.

template <int D, int L, int T0, int T1, int T2>
struct DownGeom {
  static constexpr int I0 = D >= 3 ? 2 * T0 + L - 2 : 1;
  static constexpr int I1 = D >= 2 ? 2 * T1 + L - 2 : 1;
  static constexpr int I2 = 2 * T2 + L - 2;
  static constexpr int I2P = (I2 + 3) & ~3;
  static constexpr int NV = I2P / 4;
  static constexpr int NROW = I0 * I1;
};

template <int D, int L, int U0, int U1, int U2>
struct UpGeom {
  static constexpr int H = L / 2;
  static constexpr int J0 = D >= 3 ? U0 / 2 + H - 1 : 1;
  static constexpr int J1 = D >= 2 ? U1 / 2 + H - 1 : 1;
  static constexpr int J2 = U2 / 2 + H - 1;
  // the contiguous dim is loaded from a 4-aligned start, OFF samples before the region
  static constexpr int OFF = (4 - ((H - 1) & 3)) & 3;
  static constexpr int J2P = (J2 + OFF + 3) & ~3;
  static constexpr int NV = J2P / 4;
  static constexpr int NROW = J0 * J1;
};

// Stage a periodic region into LDS: rows given by a row-offset table, 16-byte columns by a
// column table (element offsets), both already reduced modulo the block.  The trip count is
// a compile-time constant: every load of a thread is issued before the first LDS store, so a
// work-group keeps all of its global loads in flight at once.
template <int NT, int NROWS, int NV, bool VEC>
DEVI void stage_rows(const float* __restrict__ src, const int* s_row, const int* s_col, float* lds, int lds_row,
                     int b2) {
  if constexpr (VEC) {
    constexpr int N = NROWS * NV;
    constexpr int IT = (N + NT - 1) / NT;
    float4* d4 = reinterpret_cast<float4*>(lds);
    float4 r[IT];
    // no guard inside the unrolled loops: indices past the end are clamped to the last
    // element (a duplicate load and an identical duplicate store), so the compiler can issue
    // every load before the first LDS store
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, N - 1);
      r[it] = gld4(src + s_row[q / NV] + s_col[q % NV]);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int q = min(int(threadIdx.x) + it * NT, N - 1);
      d4[(q / NV) * (lds_row >> 2) + q % NV] = r[it];
    }
  } else {
    constexpr int N = NROWS * NV * 4;
    for (int q = threadIdx.x; q < N; q += NT) {
      const int e = q & 3, v = (q >> 2) % NV, r = (q >> 2) / NV;
      const int col = pmod(s_col[v] + e, b2);  // s_col holds the unreduced aligned start here
      lds[r * lds_row + 4 * v + e] = gld(src + s_row[r] + col);
    }
  }
}

// Index decomposition of a flat element index over (o0, o1, o2); shifts when o1, o2 are
// powers of two (the common case), divisions otherwise.
DEVI void split3(int e, int o1, int o2, int l1, int l2, int& c0, int& c1, int& c2) {
  if (l1 >= 0 && l2 >= 0) {
    c2 = e & (o2 - 1);
    const int r = e >> l2;
    c1 = r & (o1 - 1);
    c0 = r >> l1;
  } else {
    c2 = e % o2;
    const int r = e / o2;
    c1 = r % o1;
    c0 = r / o1;
  }
}

DEVI int ilog2_or_neg(int v) { return (v & (v - 1)) == 0 ? 31 - __builtin_clz(v) : -1; }

}  // namespace es
