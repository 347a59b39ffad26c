// Matrix-free Tikhonov / MAP solver around the wavelet prior: preconditioned conjugate gradients
// on the normal equations of J(x) = 1/2 ||M x - p||^2 + alpha/2 ||x||^2_{H^s} (Sec. 3: the
// Tikhonov functional and the linear equation of its minimiser; Sec. 4: the wavelet form of the
// Sobolev operators and the remark that iterative solvers such as conjugate gradients apply to
// it), i.e.
//     (M + alpha Gamma^2) x = M p,   Gamma^2 = W^T D_{-2s} W,   M = diag(mask),
// preconditioned with W^T D_{2s} W (the covariance: the inverse of the penalty term up to the
// factor 1/alpha, which CG's iterates do not depend on).
//
// Every step runs on the device: the two operator applications per iteration are the library's
// matern_cov_apply (smoothness -s and +s), the vector updates are fused element-wise kernels
// that also produce per-work-group partial inner products, and one work-group per instance
// reduces those partials in a fixed order and updates the instance's CG scalars.  All sums are
// FP32 with compensation (Neumaier) per thread and pairwise trees across threads; results are
// deterministic.  The host looks at the residuals only every `check_every` iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <vector>

#include "../../include/eswave.h"
#include "internal.h"
#include "kcommon.h"

namespace es {
namespace {

constexpr int kCgThreads = 256;
constexpr int kCgChunk = 4096;  // elements of one instance per work-group of the element-wise kernels

// Per-instance CG scalars (device).
struct CgScal {
  float bn;      // ||b||
  float rz;      // r . z
  float a;       // step length of this iteration (0 once converged)
  float beta;    // direction update of this iteration (0 once converged)
  float rel;     // ||r|| / ||b||
  float active;  // 1 while rel > rtol at the start of the iteration
  float pad_[2];
};

// Sum of one value per thread over the work-group, pairwise (fixed order); thread 0 gets it.
DEVI float wg_sum(float v) {
  __shared__ float part[kCgThreads / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = v;
  __syncthreads();
  float t = 0.f;
  if (threadIdx.x == 0) t = (part[0] + part[1]) + (part[2] + part[3]);
  __syncthreads();
  return t;
}

// Sums of two values per thread over the work-group, pairwise (fixed order); thread 0 gets them.
DEVI float2 wg_sum2(float v, float u) {
  __shared__ float2 part2[kCgThreads / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_down(v, o, 64);
    u += __shfl_down(u, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part2[w] = make_float2(v, u);
  __syncthreads();
  float2 t = make_float2(0.f, 0.f);
  if (threadIdx.x == 0)
    t = make_float2((part2[0].x + part2[1].x) + (part2[2].x + part2[3].x),
                    (part2[0].y + part2[1].y) + (part2[2].y + part2[3].y));
  __syncthreads();
  return t;
}

// Work-group -> (instance, chunk) of the element-wise kernels.
struct Span {
  int64_t inst, lo, hi;  // elements [lo, hi) of instance inst
};
DEVI Span span_of(int64_t n, int per) {
  Span sp;
  sp.inst = blockIdx.x / per;
  sp.lo = (int64_t)(blockIdx.x % per) * kCgChunk;
  sp.hi = min(n, sp.lo + kCgChunk);
  return sp;
}

// Element-wise loop over one chunk; vectors of four where the instance size allows.
template <class F>
DEVI void for_chunk(const Span& sp, int64_t n, F f) {
  const int64_t base = sp.inst * n;
  if ((n & 3) == 0) {
    for (int64_t i = sp.lo + 4 * threadIdx.x; i < sp.hi; i += 4 * kCgThreads) f(base + i, 4);
  } else {
    for (int64_t i = sp.lo + threadIdx.x; i < sp.hi; i += kCgThreads) f(base + i, 1);
  }
}

// r = mask * p, x = 0; partial r . r
__global__ void __launch_bounds__(kCgThreads) k_cg_init(int64_t n, int per, const float* __restrict__ p,
                                                        const float* __restrict__ mask, float* __restrict__ x,
                                                        float* __restrict__ r, float* __restrict__ part) {
  const Span sp = span_of(n, per);
  KSum acc;
  for_chunk(sp, n, [&](int64_t i, int w) {
    for (int k = 0; k < w; ++k) {
      const float v = gld(mask + i + k) * gld(p + i + k);
      gst(r + i + k, v);
      gst(x + i + k, 0.f);
      acc.add(v * v);
    }
  });
  const float t = wg_sum(acc.value());
  if (threadIdx.x == 0) gst(part + blockIdx.x, t);
}

// partial a . b (and, when dst is given, dst = b: the first direction d = z)
__global__ void __launch_bounds__(kCgThreads) k_cg_dot(int64_t n, int per, const float* __restrict__ a,
                                                       const float* __restrict__ b, float* __restrict__ dst,
                                                       float* __restrict__ part) {
  const Span sp = span_of(n, per);
  KSum acc;
  for_chunk(sp, n, [&](int64_t i, int w) {
    if (w == 4) {
      const float4 u = gld4(a + i), v = gld4(b + i);
      if (dst) gst4(dst + i, v);
      acc.add(u.x * v.x);
      acc.add(u.y * v.y);
      acc.add(u.z * v.z);
      acc.add(u.w * v.w);
    } else {
      const float v = gld(b + i);
      if (dst) gst(dst + i, v);
      acc.add(gld(a + i) * v);
    }
  });
  const float t = wg_sum(acc.value());
  if (threadIdx.x == 0) gst(part + blockIdx.x, t);
}

// ad = alpha * ad + mask * d (ad holds W^T D_{-2s} W d on entry); partial d . ad
__global__ void __launch_bounds__(kCgThreads) k_cg_apply(int64_t n, int per, float alpha, const float* __restrict__ mask,
                                                         const float* __restrict__ d, float* __restrict__ ad,
                                                         float* __restrict__ part) {
  const Span sp = span_of(n, per);
  KSum acc;
  for_chunk(sp, n, [&](int64_t i, int w) {
    if (w == 4) {
      const float4 m = gld4(mask + i), dv = gld4(d + i), g = gld4(ad + i);
      const float4 o = make_float4(fmaf(m.x, dv.x, alpha * g.x), fmaf(m.y, dv.y, alpha * g.y),
                                   fmaf(m.z, dv.z, alpha * g.z), fmaf(m.w, dv.w, alpha * g.w));
      gst4(ad + i, o);
      acc.add(dv.x * o.x);
      acc.add(dv.y * o.y);
      acc.add(dv.z * o.z);
      acc.add(dv.w * o.w);
    } else {
      const float dv = gld(d + i);
      const float o = fmaf(gld(mask + i), dv, alpha * gld(ad + i));
      gst(ad + i, o);
      acc.add(dv * o);
    }
  });
  const float t = wg_sum(acc.value());
  if (threadIdx.x == 0) gst(part + blockIdx.x, t);
}

// r -= a ad; partial r . r  (x += a d waits for the direction pass, which reads d anyway)
__global__ void __launch_bounds__(kCgThreads) k_cg_step(int64_t n, int per, const CgScal* __restrict__ sc,
                                                        float* __restrict__ r, const float* __restrict__ ad,
                                                        float* __restrict__ part) {
  const Span sp = span_of(n, per);
  const float a = sc[sp.inst].a;
  KSum acc;
  for_chunk(sp, n, [&](int64_t i, int w) {
    if (w == 4) {
      const float4 rv = gld4(r + i), g = gld4(ad + i);
      const float4 rn = make_float4(fmaf(-a, g.x, rv.x), fmaf(-a, g.y, rv.y), fmaf(-a, g.z, rv.z), fmaf(-a, g.w, rv.w));
      gst4(r + i, rn);
      acc.add(rn.x * rn.x);
      acc.add(rn.y * rn.y);
      acc.add(rn.z * rn.z);
      acc.add(rn.w * rn.w);
    } else {
      const float rn = fmaf(-a, gld(ad + i), gld(r + i));
      gst(r + i, rn);
      acc.add(rn * rn);
    }
  });
  const float t = wg_sum(acc.value());
  if (threadIdx.x == 0) gst(part + blockIdx.x, t);
}

// x += a d (this iteration's step), then d = beta d + z
__global__ void __launch_bounds__(kCgThreads) k_cg_dir(int64_t n, int per, const CgScal* __restrict__ sc,
                                                       float* __restrict__ x, float* __restrict__ d,
                                                       const float* __restrict__ z) {
  const Span sp = span_of(n, per);
  const float a = sc[sp.inst].a, beta = sc[sp.inst].beta;
  for_chunk(sp, n, [&](int64_t i, int w) {
    if (w == 4) {
      const float4 xv = gld4(x + i), dv = gld4(d + i), zv = gld4(z + i);
      gst4(x + i, make_float4(fmaf(a, dv.x, xv.x), fmaf(a, dv.y, xv.y), fmaf(a, dv.z, xv.z), fmaf(a, dv.w, xv.w)));
      gst4(d + i, make_float4(fmaf(beta, dv.x, zv.x), fmaf(beta, dv.y, zv.y), fmaf(beta, dv.z, zv.z),
                              fmaf(beta, dv.w, zv.w)));
    } else {
      const float dv = gld(d + i);
      gst(x + i, fmaf(a, dv, gld(x + i)));
      gst(d + i, fmaf(beta, dv, gld(z + i)));
    }
  });
}

enum CgFinal { F_INIT = 0, F_RZ0 = 1, F_A = 2, F_RR = 3, F_BETA = 4 };

// One work-group per instance: the sum of its `per` partials, in a fixed order, and the scalar
// update of step `kind`.
__global__ void __launch_bounds__(kCgThreads) k_cg_final(int kind, int per, const float* __restrict__ part,
                                                         CgScal* __restrict__ sc, float rtol) {
  const int64_t inst = blockIdx.x;
  KSum acc;
  for (int k = threadIdx.x; k < per; k += kCgThreads) acc.add(part[inst * per + k]);
  const float sum = wg_sum(acc.value());
  if (threadIdx.x != 0) return;
  CgScal c = sc[inst];
  switch (kind) {
    case F_INIT:
      c.bn = sqrtf(sum);
      c.rel = c.bn > 0.f ? 1.f : 0.f;
      c.active = c.rel > rtol ? 1.f : 0.f;
      c.a = c.beta = 0.f;
      break;
    case F_RZ0: c.rz = sum; break;
    case F_A: c.a = (c.active != 0.f && sum > 0.f) ? c.rz / sum : 0.f; break;
    case F_RR: c.rel = c.bn > 0.f ? sqrtf(sum) / c.bn : 0.f; break;
    default:  // F_BETA: sum = r . z of the new residual
      c.beta = (c.active != 0.f && c.rz > 0.f) ? sum / c.rz : 0.f;
      c.rz = sum;
      c.active = c.rel > rtol ? c.active : 0.f;  // converged instances stay frozen
      break;
  }
  sc[inst] = c;
}

// ---- GMRES on (E_s^* K^* K + alpha I) x = E_s^* K^* p (K = diag(mask)) ----------------------
constexpr int kGmMaxBasis = 64;  // largest restart length
// Vectors of the basis are batch * n floats, `vs` floats apart.  Per-instance coefficients
// (inner products, norms, least-squares solutions) are device arrays indexed inst * ld + j.

// out = (sq ? m * m : m) * v
__global__ void __launch_bounds__(kCgThreads) k_gm_mask(int64_t n, int per, int sq, const float* __restrict__ mask,
                                                        const float* __restrict__ v, float* __restrict__ out) {
  const Span sp = span_of(n, per);
  for_chunk(sp, n, [&](int64_t i, int w) {
    if (w == 4) {
      float4 m = gld4(mask + i);
      const float4 x = gld4(v + i);
      if (sq) m = make_float4(m.x * m.x, m.y * m.y, m.z * m.z, m.w * m.w);
      gst4(out + i, make_float4(m.x * x.x, m.y * x.y, m.z * x.z, m.w * x.w));
    } else {
      const float m = gld(mask + i);
      gst(out + i, (sq ? m * m : m) * gld(v + i));
    }
  });
}

// out = a x + b y + c z (a null vector contributes nothing); partial ||out||^2 when part is given.
// out may be one of x, y, z (each element is read, then written, by the same thread).
__global__ void __launch_bounds__(kCgThreads) k_gm_lin3(int64_t n, int per, float a, const float* x, float b,
                                                        const float* y, float c, const float* z, float* out,
                                                        float* __restrict__ part) {
  const Span sp = span_of(n, per);
  KSum acc;
  auto l4 = [](const float* q, int64_t i) { return q ? gld4(q + i) : make_float4(0.f, 0.f, 0.f, 0.f); };
  for_chunk(sp, n, [&](int64_t i, int w) {
    if (w == 4) {  // every vector's three loads issued before the arithmetic
      const float4 xv = l4(x, i), yv = l4(y, i), zv = l4(z, i);
      const float4 o = make_float4(fmaf(c, zv.x, fmaf(b, yv.x, a * xv.x)), fmaf(c, zv.y, fmaf(b, yv.y, a * xv.y)),
                                   fmaf(c, zv.z, fmaf(b, yv.z, a * xv.z)), fmaf(c, zv.w, fmaf(b, yv.w, a * xv.w)));
      gst4(out + i, o);
      acc.add(o.x * o.x);
      acc.add(o.y * o.y);
      acc.add(o.z * o.z);
      acc.add(o.w * o.w);
    } else {
      const float o = fmaf(c, z ? gld(z + i) : 0.f, fmaf(b, y ? gld(y + i) : 0.f, x ? a * gld(x + i) : 0.f));
      gst(out + i, o);
      acc.add(o * o);
    }
  });
  if (part) {
    const float t = wg_sum(acc.value());
    if (threadIdx.x == 0) gst(part + blockIdx.x, t);
  } else {
    (void)acc;
  }
}

// Over this work-group's chunk, for j < nv: part[j * nblk + blk] = <v_j, w> and
// part[(nv + j) * nblk + blk] = <v_j, u> (u = v_{nv-1}, the newest basis vector: the new column of
// the basis's Gram matrix).  The chunks of w and u are read once, into registers (16-byte loads
// when the instance size is a multiple of 4); each product is summed within the wave per basis
// vector and across the four waves, in a fixed order, once at the end.
constexpr int kGmPer = kCgChunk / kCgThreads;  // elements of a chunk per thread
__global__ void __launch_bounds__(kCgThreads) k_gm_dots(int64_t n, int per, int nv, const float* __restrict__ V,
                                                        int64_t vs, const float* __restrict__ w,
                                                        float* __restrict__ part) {
  __shared__ float2 wp[kCgThreads / 64][kGmMaxBasis + 1];
  const Span sp = span_of(n, per);
  const int64_t base = sp.inst * n;
  const float* u = V + (int64_t)(nv - 1) * vs + base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto wave_store = [&](int j, KSum& aw, KSum& au) {
    float x = aw.value(), y = au.value();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      x += __shfl_down(x, o, 64);
      y += __shfl_down(y, o, 64);
    }
    if (lane == 0) wp[wave][j] = make_float2(x, y);
  };
  if ((n & 3) == 0) {
    constexpr int G = kGmPer / 4;  // float4 groups per thread
    float4 wv[G], uv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = sp.lo + 4 * threadIdx.x + (int64_t)g * 4 * kCgThreads;
      const bool in = i < sp.hi;
      wv[g] = in ? gld4(w + base + i) : make_float4(0.f, 0.f, 0.f, 0.f);
      uv[g] = in ? gld4(u + i) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int j = 0; j < nv; ++j) {
      const float* v = V + j * vs + base;
      float4 xv[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int64_t i = sp.lo + 4 * threadIdx.x + (int64_t)g * 4 * kCgThreads;
        xv[g] = i < sp.hi ? gld4(v + i) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      KSum aw, au;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        aw.add(xv[g].x * wv[g].x);
        aw.add(xv[g].y * wv[g].y);
        aw.add(xv[g].z * wv[g].z);
        aw.add(xv[g].w * wv[g].w);
        au.add(xv[g].x * uv[g].x);
        au.add(xv[g].y * uv[g].y);
        au.add(xv[g].z * uv[g].z);
        au.add(xv[g].w * uv[g].w);
      }
      wave_store(j, aw, au);
    }
  } else {
    float wv[kGmPer], uv[kGmPer];
#pragma unroll
    for (int k = 0; k < kGmPer; ++k) {
      const int64_t i = sp.lo + threadIdx.x + (int64_t)k * kCgThreads;
      wv[k] = i < sp.hi ? gld(w + base + i) : 0.f;
      uv[k] = i < sp.hi ? gld(u + i) : 0.f;
    }
    for (int j = 0; j < nv; ++j) {
      const float* v = V + j * vs + base;
      KSum aw, au;
#pragma unroll
      for (int k = 0; k < kGmPer; ++k) {
        const int64_t i = sp.lo + threadIdx.x + (int64_t)k * kCgThreads;
        if (i < sp.hi) {
          const float x = gld(v + i);
          aw.add(x * wv[k]);
          au.add(x * uv[k]);
        }
      }
      wave_store(j, aw, au);
    }
  }
  __syncthreads();
  const int nblk = gridDim.x;
  for (int q = threadIdx.x; q < 2 * nv; q += kCgThreads) {
    const int j = q >> 1;
    const bool second = q & 1;
    auto pick = [&](int wv_) { return second ? wp[wv_][j].y : wp[wv_][j].x; };
    const float t = (pick(0) + pick(1)) + (pick(2) + pick(3));
    gst(part + (int64_t)(second ? nv + j : j) * nblk + blockIdx.x, t);
  }
}

// Coefficients of step k (one work-group of 64 threads per instance): the new Gram column
// G[j][k] = G[k][j] = <v_j, v_k> enters the instance's (m+1) x (m+1) Gram matrix, and
// c = 2 h - G h (j, i <= k) with h = V^T w: the two classical Gram-Schmidt passes of CGS2, the
// second written through the Gram matrix (exact when the first subtraction is).
__global__ void __launch_bounds__(64) k_gm_coef(int k, const float* __restrict__ hg, int ldg, float* __restrict__ G,
                                                int ldG, float* __restrict__ c, int ldc) {
  const int inst = blockIdx.x, j = threadIdx.x;
  const float* h = hg + inst * ldg;        // h[0..k], then the Gram column [k+1 .. 2k+1]
  float* Gi = G + (int64_t)inst * ldG * ldG;
  if (j <= k) {
    const float gj = h[k + 1 + j];
    Gi[j * ldG + k] = gj;
    Gi[k * ldG + j] = gj;
  }
  __syncthreads();
  if (j <= k) {
    float acc = 0.f;
    for (int i = 0; i <= k; ++i) acc = fmaf(Gi[j * ldG + i], h[i], acc);
    c[inst * ldc + j] = 2.f * h[j] - acc;
  }
}

// dst[inst * ld + j] = sum of instance inst's `per` partials of vector j, in a fixed order;
// grid (batch, nv)
__global__ void __launch_bounds__(kCgThreads) k_gm_final(int per, int nblk, const float* __restrict__ part,
                                                         float* __restrict__ dst, int ld) {
  const int inst = blockIdx.x, j = blockIdx.y;
  KSum acc;
  for (int k = threadIdx.x; k < per; k += kCgThreads) acc.add(part[(int64_t)j * nblk + (int64_t)inst * per + k]);
  const float sum = wg_sum(acc.value());
  if (threadIdx.x == 0) dst[inst * ld + j] = sum;
}

// w -= sum_j h[inst * ld + j] v_j (j < nv); partial ||w||^2 when part is given
__global__ void __launch_bounds__(kCgThreads) k_gm_sub(int64_t n, int per, int nv, const float* __restrict__ V,
                                                       int64_t vs, const float* __restrict__ h, int ld,
                                                       float* __restrict__ w, float* __restrict__ part) {
  const Span sp = span_of(n, per);
  const int64_t base = sp.inst * n;
  __shared__ float hs[kGmMaxBasis + 1];
  for (int j = threadIdx.x; j < nv; j += kCgThreads) hs[j] = h[sp.inst * ld + j];
  __syncthreads();
  KSum acc;
  if ((n & 3) == 0) {
    for (int64_t i = sp.lo + 4 * threadIdx.x; i < sp.hi; i += 4 * kCgThreads) {
      float4 o = gld4(w + base + i);
      for (int j = 0; j < nv; ++j) {
        const float4 x = gld4(V + j * vs + base + i);
        const float hj = -hs[j];
        o = make_float4(fmaf(hj, x.x, o.x), fmaf(hj, x.y, o.y), fmaf(hj, x.z, o.z), fmaf(hj, x.w, o.w));
      }
      gst4(w + base + i, o);
      acc.add(o.x * o.x);
      acc.add(o.y * o.y);
      acc.add(o.z * o.z);
      acc.add(o.w * o.w);
    }
  } else {
    for (int64_t i = sp.lo + threadIdx.x; i < sp.hi; i += kCgThreads) {
      float o = gld(w + base + i);
      for (int j = 0; j < nv; ++j) o = fmaf(-hs[j], gld(V + j * vs + base + i), o);
      gst(w + base + i, o);
      acc.add(o * o);
    }
  }
  if (part) {
    const float t = wg_sum(acc.value());
    if (threadIdx.x == 0) gst(part + blockIdx.x, t);
  }
}

// v = w / sqrt(nrm2[inst]), or 0 when the norm is 0 (an exhausted or zero instance); with a mask,
// also t = mask^2 v (the next operator application's input)
__global__ void __launch_bounds__(kCgThreads) k_gm_scale(int64_t n, int per, const float* __restrict__ nrm2,
                                                         const float* __restrict__ w, float* __restrict__ v,
                                                         const float* __restrict__ mask, float* __restrict__ t) {
  const Span sp = span_of(n, per);
  const float q = nrm2[sp.inst];
  const float sc = q > 0.f ? 1.f / sqrtf(q) : 0.f;
  for_chunk(sp, n, [&](int64_t i, int wdt) {
    if (wdt == 4) {
      const float4 x = gld4(w + i);
      const float4 o = make_float4(sc * x.x, sc * x.y, sc * x.z, sc * x.w);
      gst4(v + i, o);
      if (mask) {
        const float4 m = gld4(mask + i);
        gst4(t + i, make_float4(m.x * m.x * o.x, m.y * m.y * o.y, m.z * m.z * o.z, m.w * m.w * o.w));
      }
    } else {
      const float o = sc * gld(w + i);
      gst(v + i, o);
      if (mask) {
        const float m = gld(mask + i);
        gst(t + i, m * m * o);
      }
    }
  });
}

// x += sum_j y[inst * ld + j] v_j (j < nv)
__global__ void __launch_bounds__(kCgThreads) k_gm_combine(int64_t n, int per, int nv, const float* __restrict__ V,
                                                           int64_t vs, const float* __restrict__ y, int ld,
                                                           float* __restrict__ x) {
  const Span sp = span_of(n, per);
  const int64_t base = sp.inst * n;
  __shared__ float ys[kGmMaxBasis + 1];
  for (int j = threadIdx.x; j < nv; j += kCgThreads) ys[j] = y[sp.inst * ld + j];
  __syncthreads();
  if ((n & 3) == 0) {
    for (int64_t i = sp.lo + 4 * threadIdx.x; i < sp.hi; i += 4 * kCgThreads) {
      float4 o = gld4(x + base + i);
      for (int j = 0; j < nv; ++j) {
        const float4 v = gld4(V + j * vs + base + i);
        o = make_float4(fmaf(ys[j], v.x, o.x), fmaf(ys[j], v.y, o.y), fmaf(ys[j], v.z, o.z), fmaf(ys[j], v.w, o.w));
      }
      gst4(x + base + i, o);
    }
  } else {
    for (int64_t i = sp.lo + threadIdx.x; i < sp.hi; i += kCgThreads) {
      float o = gld(x + base + i);
      for (int j = 0; j < nv; ++j) o = fmaf(ys[j], gld(V + j * vs + base + i), o);
      gst(x + base + i, o);
    }
  }
}

int64_t cg_parts(int64_t n) { return (n + kCgChunk - 1) / kCgChunk; }
size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct GmLayout {
  size_t V, b, w, t, part, hg, c, G, nrm, y, cov, total;
  int64_t vs;  // floats between basis vectors
};

GmLayout gm_layout(int64_t n, int64_t batch, int m, size_t cov_bytes, int64_t per) {
  GmLayout L;
  const size_t vec = a256((size_t)(n * batch) * sizeof(float));
  L.vs = (int64_t)(vec / sizeof(float));
  L.V = 0;
  L.b = L.V + vec * (size_t)(m + 1);
  L.w = L.b + vec;
  L.t = L.w + vec;
  L.part = L.t + vec;
  L.hg = L.part + a256((size_t)(2 * (m + 1) * per * batch) * sizeof(float));
  L.c = L.hg + a256((size_t)(batch * 2 * (m + 1)) * sizeof(float));
  L.G = L.c + a256((size_t)(batch * (m + 1)) * sizeof(float));
  L.nrm = L.G + a256((size_t)(batch * (m + 1) * (m + 1)) * sizeof(float));
  L.y = L.nrm + a256((size_t)batch * sizeof(float));
  L.cov = L.y + a256((size_t)(batch * (m + 1)) * sizeof(float));
  L.total = L.cov + cov_bytes;
  return L;
}


struct CgLayout {
  size_t r, z, d, ad, part, scal, cov, total;
};

CgLayout cg_layout(int64_t n, int64_t batch, size_t cov_bytes, int64_t parts) {
  CgLayout L;
  const size_t vec = a256((size_t)(n * batch) * sizeof(float));
  L.r = 0;
  L.z = L.r + vec;
  L.d = L.z + vec;
  L.ad = L.d + vec;
  L.part = L.ad + vec;
  L.scal = L.part + a256((size_t)(parts * batch) * sizeof(float));
  L.cov = L.scal + a256((size_t)batch * sizeof(CgScal));
  L.total = L.cov + cov_bytes;
  return L;
}

}  // namespace
}  // namespace es

using namespace es;

extern "C" {

size_t es_tikhonov_pcg_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels) {
  if (batch < 1 || ndim < 1 || ndim > 3 || !shape) return 0;
  int64_t n = 1;
  for (int k = 0; k < ndim; ++k) n *= shape[k];
  const size_t cov = es_workspace_bytes(ndim, shape, batch, order, levels, ES_OP_COV);
  return cg_layout(n, batch, cov, std::max(cg_parts(n), cov_dot_partials_max(ndim, shape))).total;
}

es_status es_tikhonov_pcg(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s, double alpha,
                          const float* p, const float* mask, float* x, int32_t max_iter, double rtol,
                          int32_t check_every, int32_t* iterations, float* rel_residual, void* ws, size_t ws_bytes,
                          void* stream) {
  char msg[256];
  if (ndim < 1 || ndim > 3 || !shape) return report_error(ES_EINVAL, "ndim must be 1..3 and shape non-NULL");
  if (batch < 0) return report_error(ES_EINVAL, "batch must be >= 0");
  if (!(alpha > 0) || !std::isfinite(alpha)) return report_error(ES_EINVAL, "alpha must be positive and finite");
  if (!(rtol >= 0) || !std::isfinite(rtol)) return report_error(ES_EINVAL, "rtol must be finite and >= 0");
  if (max_iter < 0) return report_error(ES_EINVAL, "max_iter must be >= 0");
  if (check_every < 1) check_every = 1;
  if (iterations) *iterations = 0;
  if (batch == 0) return ES_OK;
  if (batch > 0x7fffffffll) return report_error(ES_EINVAL, "batch too large");
  int64_t n = 1;
  for (int k = 0; k < ndim; ++k) {
    if (shape[k] < 1) return report_error(ES_EINVAL, "shape entries must be positive");
    n *= shape[k];
  }
  const int64_t per = cg_parts(n);
  if (per * batch > 0x7fffffffll) return report_error(ES_EINVAL, "problem too large");
  // validates the operator arguments (order, levels, divisibility) through the workspace query
  const size_t cov = es_workspace_bytes(ndim, shape, batch, order, levels, ES_OP_COV);
  if (cov == 0 && levels > 1) return report_error(ES_EINVAL, "invalid operator arguments (order, levels, shape)");
  // partial sums: per-chunk (element-wise kernels) or per-tile (the fused operator steps)
  const int64_t parts = std::max(per, cov_dot_partials_max(ndim, shape));
  const CgLayout L = cg_layout(n, batch, cov, parts);
  if (!p || !mask || !x || !rel_residual) return report_error(ES_EINVAL, "p, mask, x and rel_residual must be non-NULL");
  if (((uintptr_t)p | (uintptr_t)mask | (uintptr_t)x) & 15) return report_error(ES_EINVAL, "p, mask and x must be 16-byte aligned");
  if (!ws || ws_bytes < L.total) {
    snprintf(msg, sizeof msg, "workspace of %zu bytes required", L.total);
    return report_error(ES_EWORKSPACE, msg);
  }
  if ((uintptr_t)ws & 255) return report_error(ES_EINVAL, "workspace must be 256-byte aligned");
  const size_t vb = (size_t)(n * batch) * sizeof(float);
  auto ov = [](const void* a, size_t na, const void* b, size_t nb) {
    return (const char*)a < (const char*)b + nb && (const char*)b < (const char*)a + na;
  };
  if (ov(x, vb, p, vb) || ov(x, vb, mask, vb) || ov(ws, L.total, x, vb) || ov(ws, L.total, p, vb) ||
      ov(ws, L.total, mask, vb))
    return report_error(ES_EINVAL, "x must not overlap p, mask or the workspace; the workspace must not overlap p or mask");
  es_status st = device_check();
  if (st != ES_OK) return st;

  char* w = (char*)ws;
  float* r = (float*)(w + L.r);
  float* z = (float*)(w + L.z);
  float* d = (float*)(w + L.d);
  float* ad = (float*)(w + L.ad);
  float* part = (float*)(w + L.part);
  CgScal* sc = (CgScal*)(w + L.scal);
  void* cws = cov ? (void*)(w + L.cov) : nullptr;
  const hipStream_t hs = (hipStream_t)stream;
  const dim3 grid((unsigned)(per * batch)), blk(kCgThreads);
  const float frtol = (float)rtol;
  auto ok = [&](const char* what) -> es_status {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return ES_OK;
    snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
    return report_error(ES_EDEVICE, msg);
  };
  auto final_ = [&](int kind, int64_t nparts) -> es_status {
    hipLaunchKernelGGL(k_cg_final, dim3((unsigned)batch), blk, 0, hs, kind, (int)nparts, part, sc, frtol);
    return ok("CG scalar update launch");
  };
  // Fused operator steps (2-D grids whose operator ends in the vector-path synthesis): the last
  // kernel of the operator also forms the mask term and the per-tile inner products, so the
  // separate update / inner-product passes over the vectors disappear.  Falls back to the
  // separate kernels when the schedule does not allow it.
  const char* fz = getenv("ESWAVE_CG_FUSED");  // 0: always the separate kernels (comparison)
  bool fused = cov_dot_partials_max(ndim, shape) > 0 && !(fz && *fz == '0');
  // out = scale * op(in) + gamma * mask * in, and part = per-tile sums of in * out
  auto cov_dot = [&](const float* in, float* out, double sm, const float* msk, float scale, int64_t* np) -> es_status {
    const es_status r = cov_apply_masked_dot(ndim, shape, batch, order, levels, sm, in, out, cws, cov, msk, 1.f, scale,
                                             part, parts * batch, np, hs);
    if (r == ES_EUNSUPPORTED) fused = false;
    return r;
  };
  auto cov_apply = [&](const float* in, float* out, double sm) -> es_status {
    return matern_cov_apply(ndim, shape, batch, order, levels, sm, in, out, cws, cov, stream);
  };

  // r = b = M p, x = 0, ||b||; z = P r, d = z, rz = r . z
  hipLaunchKernelGGL(k_cg_init, grid, blk, 0, hs, n, (int)per, p, mask, x, r, part);
  if ((st = ok("CG init launch")) != ES_OK || (st = final_(F_INIT, per)) != ES_OK) return st;
  if ((st = cov_apply(r, z, s)) != ES_OK) return st;
  hipLaunchKernelGGL(k_cg_dot, grid, blk, 0, hs, n, (int)per, r, z, d, part);
  if ((st = ok("CG dot launch")) != ES_OK || (st = final_(F_RZ0, per)) != ES_OK) return st;

  std::vector<CgScal> host((size_t)batch);
  int it = 0;
  bool done = false;
  while (it < max_iter && !done) {
    // ad = alpha Gamma^2 d + M d, a = rz / (d . ad)
    int64_t np = per;
    st = fused ? cov_dot(d, ad, -s, mask, (float)alpha, &np) : ES_EUNSUPPORTED;
    if (st == ES_EUNSUPPORTED) {
      np = per;
      if ((st = cov_apply(d, ad, -s)) != ES_OK) return st;
      hipLaunchKernelGGL(k_cg_apply, grid, blk, 0, hs, n, (int)per, (float)alpha, mask, d, ad, part);
      st = ok("CG operator update launch");
    }
    if (st != ES_OK || (st = final_(F_A, np)) != ES_OK) return st;
    // r -= a ad, rel = ||r|| / ||b||
    hipLaunchKernelGGL(k_cg_step, grid, blk, 0, hs, n, (int)per, sc, r, ad, part);
    if ((st = ok("CG step launch")) != ES_OK || (st = final_(F_RR, per)) != ES_OK) return st;
    // z = P r, beta = (r . z) / rz, d = z + beta d
    np = per;
    st = fused ? cov_dot(r, z, s, nullptr, 1.f, &np) : ES_EUNSUPPORTED;
    if (st == ES_EUNSUPPORTED) {
      np = per;
      if ((st = cov_apply(r, z, s)) != ES_OK) return st;
      hipLaunchKernelGGL(k_cg_dot, grid, blk, 0, hs, n, (int)per, r, z, (float*)nullptr, part);
      st = ok("CG dot launch");
    }
    if (st != ES_OK || (st = final_(F_BETA, np)) != ES_OK) return st;
    // x += a d, d = z + beta d
    hipLaunchKernelGGL(k_cg_dir, grid, blk, 0, hs, n, (int)per, sc, x, d, z);
    if ((st = ok("CG direction launch")) != ES_OK) return st;
    ++it;
    if (it % check_every == 0 || it == max_iter) {
      hipError_t e = hipMemcpyAsync(host.data(), sc, host.size() * sizeof(CgScal), hipMemcpyDeviceToHost, hs);
      if (e == hipSuccess) e = hipStreamSynchronize(hs);
      if (e != hipSuccess) {
        snprintf(msg, sizeof msg, "CG residual read: %s", hipGetErrorString(e));
        return report_error(ES_EDEVICE, msg);
      }
      done = true;
      for (const CgScal& c : host) done = done && !(c.rel > frtol);
    }
  }
  hipError_t e = hipMemcpyAsync(host.data(), sc, host.size() * sizeof(CgScal), hipMemcpyDeviceToHost, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) {
    snprintf(msg, sizeof msg, "CG residual read: %s", hipGetErrorString(e));
    return report_error(ES_EDEVICE, msg);
  }
  for (int64_t b = 0; b < batch; ++b) rel_residual[b] = host[(size_t)b].rel;
  if (iterations) *iterations = it;
  return ES_OK;
}


size_t es_tikhonov_gmres_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, int order, int levels,
                                         int32_t restart) {
  if (batch < 1 || ndim < 1 || ndim > 3 || !shape || restart < 1 || restart > kGmMaxBasis) return 0;
  int64_t n = 1;
  for (int k = 0; k < ndim; ++k) n *= shape[k];
  const size_t cov = es_workspace_bytes(ndim, shape, batch, order, levels, ES_OP_COV);
  return gm_layout(n, batch, restart, cov, cg_parts(n)).total;
}

es_status es_tikhonov_gmres(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                            double alpha, const float* p, const float* mask, float* x, int32_t restart,
                            int32_t max_iter, double rtol, int32_t* iterations, float* rel_residual, void* ws,
                            size_t ws_bytes, void* stream) {
  char msg[256];
  if (ndim < 1 || ndim > 3 || !shape) return report_error(ES_EINVAL, "ndim must be 1..3 and shape non-NULL");
  if (batch < 0) return report_error(ES_EINVAL, "batch must be >= 0");
  if (!(alpha > 0) || !std::isfinite(alpha)) return report_error(ES_EINVAL, "alpha must be positive and finite");
  if (!(rtol >= 0) || !std::isfinite(rtol)) return report_error(ES_EINVAL, "rtol must be finite and >= 0");
  if (max_iter < 0) return report_error(ES_EINVAL, "max_iter must be >= 0");
  if (restart < 1 || restart > kGmMaxBasis) return report_error(ES_EINVAL, "restart must be 1..64");
  if (iterations) *iterations = 0;
  if (batch == 0) return ES_OK;
  if (batch > 0x7fffffffll) return report_error(ES_EINVAL, "batch too large");
  int64_t n = 1;
  for (int k = 0; k < ndim; ++k) {
    if (shape[k] < 1) return report_error(ES_EINVAL, "shape entries must be positive");
    n *= shape[k];
  }
  const int64_t per = cg_parts(n);
  if (per * batch > 0x7fffffffll) return report_error(ES_EINVAL, "problem too large");
  const size_t cov = es_workspace_bytes(ndim, shape, batch, order, levels, ES_OP_COV);
  if (cov == 0 && levels > 1) return report_error(ES_EINVAL, "invalid operator arguments (order, levels, shape)");
  const int m = restart;
  const GmLayout L = gm_layout(n, batch, m, cov, per);
  if (!p || !mask || !x || !rel_residual) return report_error(ES_EINVAL, "p, mask, x and rel_residual must be non-NULL");
  if (((uintptr_t)p | (uintptr_t)mask | (uintptr_t)x) & 15) return report_error(ES_EINVAL, "p, mask and x must be 16-byte aligned");
  if (!ws || ws_bytes < L.total) {
    snprintf(msg, sizeof msg, "workspace of %zu bytes required", L.total);
    return report_error(ES_EWORKSPACE, msg);
  }
  if ((uintptr_t)ws & 255) return report_error(ES_EINVAL, "workspace must be 256-byte aligned");
  const size_t vb = (size_t)(n * batch) * sizeof(float);
  auto ov = [](const void* a, size_t na, const void* b, size_t nb) {
    return (const char*)a < (const char*)b + nb && (const char*)b < (const char*)a + na;
  };
  if (ov(x, vb, p, vb) || ov(x, vb, mask, vb) || ov(ws, L.total, x, vb) || ov(ws, L.total, p, vb) ||
      ov(ws, L.total, mask, vb))
    return report_error(ES_EINVAL, "x must not overlap p, mask or the workspace; the workspace must not overlap p or mask");
  es_status st = device_check();
  if (st != ES_OK) return st;

  char* wsc = (char*)ws;
  float* V = (float*)(wsc + L.V);
  float* bv = (float*)(wsc + L.b);
  float* w = (float*)(wsc + L.w);
  float* t = (float*)(wsc + L.t);
  float* part = (float*)(wsc + L.part);
  float* hg = (float*)(wsc + L.hg);
  float* cd = (float*)(wsc + L.c);
  float* Gd = (float*)(wsc + L.G);
  float* nrm = (float*)(wsc + L.nrm);
  float* yd = (float*)(wsc + L.y);
  void* cws = cov ? (void*)(wsc + L.cov) : nullptr;
  const int64_t vs = L.vs;
  const int ld = m + 1;
  const hipStream_t hs = (hipStream_t)stream;
  const dim3 grid((unsigned)(per * batch)), blk(kCgThreads);
  const int nblk = (int)(per * batch);
  auto ok = [&](const char* what) -> es_status {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return ES_OK;
    snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
    return report_error(ES_EDEVICE, msg);
  };
  auto to_host = [&](void* dst, const void* src, size_t bytes) -> es_status {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e == hipSuccess) return ES_OK;
    snprintf(msg, sizeof msg, "GMRES coefficient read: %s", hipGetErrorString(e));
    return report_error(ES_EDEVICE, msg);
  };
  // per-instance sums of `nv` partial arrays into dst[inst * ldd + j]
  auto final_ = [&](int nv, float* dst, int ldd) -> es_status {
    hipLaunchKernelGGL(k_gm_final, dim3((unsigned)batch, (unsigned)nv), blk, 0, hs, (int)per, nblk, part, dst, ldd);
    return ok("GMRES reduction launch");
  };
  // out = A v = E_s^*(mask^2 v) + alpha v, or out = b - A v (residual); premasked: t already holds
  // mask^2 v (written with the basis vector)
  auto apply_a = [&](const float* v, float* out, bool residual, float* nparts, bool premasked) -> es_status {
    if (!premasked) hipLaunchKernelGGL(k_gm_mask, grid, blk, 0, hs, n, (int)per, 1, mask, v, t);
    es_status r = ok("GMRES mask launch");
    if (r == ES_OK) r = matern_cov_apply(ndim, shape, batch, order, levels, s, t, out, cws, cov, stream);
    if (r != ES_OK) return r;
    if (residual)
      hipLaunchKernelGGL(k_gm_lin3, grid, blk, 0, hs, n, (int)per, 1.f, (const float*)bv, -1.f, (const float*)out,
                         (float)-alpha, v, out, nparts);
    else
      hipLaunchKernelGGL(k_gm_lin3, grid, blk, 0, hs, n, (int)per, 1.f, (const float*)out, (float)alpha, v,
                         0.f, (const float*)nullptr, out, nparts);
    return ok("GMRES update launch");
  };
  // host copies of the coefficients and the FP64 least-squares state per instance: R (upper
  // triangle of the rotated Hessenberg matrix, column-major m x m), rotations, right side g,
  // ||b||, the current residual norm, whether the instance still takes steps, its steps this cycle
  std::vector<float> hb, hn, yh;
  std::vector<double> R, cs, sn, g, bn, beta;
  std::vector<char> active;
  std::vector<int> kk;
  try {
    hb.resize((size_t)batch * ld);
    hn.resize((size_t)batch);
    yh.assign((size_t)batch * ld, 0.f);
    R.resize((size_t)batch * m * m);
    cs.resize((size_t)batch * m);
    sn.resize((size_t)batch * m);
    g.resize((size_t)batch * ld);
    bn.resize((size_t)batch);
    beta.resize((size_t)batch);
    active.resize((size_t)batch);
    kk.resize((size_t)batch);
  } catch (const std::bad_alloc&) {
    return report_error(ES_ENOMEM, "host memory for the GMRES coefficients of every instance");
  }

  // b = E_s^*(mask p), x = 0, v_0 = b / ||b||
  hipLaunchKernelGGL(k_gm_mask, grid, blk, 0, hs, n, (int)per, 0, mask, p, t);
  if ((st = ok("GMRES mask launch")) != ES_OK) return st;
  if ((st = matern_cov_apply(ndim, shape, batch, order, levels, s, t, bv, cws, cov, stream)) != ES_OK) return st;
  hipLaunchKernelGGL(k_gm_lin3, grid, blk, 0, hs, n, (int)per, 0.f, (const float*)nullptr, 0.f,
                     (const float*)nullptr, 0.f, (const float*)nullptr, x, (float*)nullptr);
  hipLaunchKernelGGL(k_gm_lin3, grid, blk, 0, hs, n, (int)per, 1.f, (const float*)bv, 0.f, (const float*)nullptr,
                     0.f, (const float*)nullptr, w, part);
  if ((st = ok("GMRES init launch")) != ES_OK || (st = final_(1, nrm, 1)) != ES_OK) return st;
  hipLaunchKernelGGL(k_gm_scale, grid, blk, 0, hs, n, (int)per, nrm, w, V, mask, t);
  if ((st = ok("GMRES scale launch")) != ES_OK || (st = to_host(hn.data(), nrm, hn.size() * sizeof(float))) != ES_OK)
    return st;

  for (int64_t b = 0; b < batch; ++b) {
    bn[b] = beta[b] = std::sqrt((double)hn[b]);
    active[b] = bn[b] > 0 && 1.0 > rtol;
  }
  int it = 0;
  auto any_active = [&]() {
    for (char a : active)
      if (a) return true;
    return false;
  };
  while (any_active() && it < max_iter) {
    for (int64_t b = 0; b < batch; ++b) {
      std::fill(g.begin() + b * ld, g.begin() + (b + 1) * ld, 0.0);
      g[b * ld] = beta[b];
      kk[b] = 0;
    }
    int K = 0;  // Arnoldi steps of this cycle
    while (K < m && it < max_iter && any_active()) {
      const int k = K;
      const float* vk = V + k * vs;
      if ((st = apply_a(vk, w, false, nullptr, true)) != ES_OK) return st;
      // Gram-Schmidt against v_0 .. v_k: one pass of inner products (with w and with v_k), the
      // CGS2 coefficients from the Gram matrix, one update pass
      hipLaunchKernelGGL(k_gm_dots, grid, blk, 0, hs, n, (int)per, k + 1, (const float*)V, vs, (const float*)w, part);
      if ((st = ok("GMRES inner-product launch")) != ES_OK || (st = final_(2 * (k + 1), hg, 2 * ld)) != ES_OK) return st;
      hipLaunchKernelGGL(k_gm_coef, dim3((unsigned)batch), dim3(64), 0, hs, k, (const float*)hg, 2 * ld, Gd, ld, cd,
                         ld);
      if ((st = ok("GMRES coefficient launch")) != ES_OK) return st;
      hipLaunchKernelGGL(k_gm_sub, grid, blk, 0, hs, n, (int)per, k + 1, (const float*)V, vs, (const float*)cd, ld, w,
                         part);
      if ((st = ok("GMRES update launch")) != ES_OK || (st = final_(1, nrm, 1)) != ES_OK) return st;
      hipLaunchKernelGGL(k_gm_scale, grid, blk, 0, hs, n, (int)per, (const float*)nrm, (const float*)w,
                         V + (k + 1) * vs, mask, t);
      if ((st = ok("GMRES scale launch")) != ES_OK) return st;
      if ((st = to_host(hb.data(), cd, hb.size() * sizeof(float))) != ES_OK ||
          (st = to_host(hn.data(), nrm, hn.size() * sizeof(float))) != ES_OK)
        return st;
      ++it;
      ++K;
      for (int64_t b = 0; b < batch; ++b) {
        if (!active[b]) continue;
        double col[kGmMaxBasis + 1];
        for (int j = 0; j <= k; ++j) col[j] = (double)hb[b * ld + j];
        col[k + 1] = std::sqrt((double)hn[b]);
        double* c = cs.data() + b * m;
        double* sv = sn.data() + b * m;
        for (int i = 0; i < k; ++i) {  // earlier rotations
          const double u = col[i], v = col[i + 1];
          col[i] = c[i] * u + sv[i] * v;
          col[i + 1] = -sv[i] * u + c[i] * v;
        }
        const double r = std::hypot(col[k], col[k + 1]);
        c[k] = r > 0 ? col[k] / r : 1.0;
        sv[k] = r > 0 ? col[k + 1] / r : 0.0;
        col[k] = r;
        double* gb = g.data() + b * ld;
        gb[k + 1] = -sv[k] * gb[k];
        gb[k] = c[k] * gb[k];
        for (int j = 0; j <= k; ++j) R[(size_t)b * m * m + (size_t)k * m + j] = col[j];
        kk[b] = k + 1;
        if (!(std::fabs(gb[k + 1]) / bn[b] > rtol) || r == 0) active[b] = 0;
      }
    }
    // x += V y, y = R^{-1} g over each instance's steps of this cycle
    for (int64_t b = 0; b < batch; ++b) {
      const int nk = kk[b];
      const double* Rb = R.data() + (size_t)b * m * m;
      double yv[kGmMaxBasis];
      for (int i = nk - 1; i >= 0; --i) {
        double v = g[b * ld + i];
        for (int j = i + 1; j < nk; ++j) v -= Rb[(size_t)j * m + i] * yv[j];
        yv[i] = Rb[(size_t)i * m + i] != 0 ? v / Rb[(size_t)i * m + i] : 0.0;
      }
      for (int j = 0; j < ld; ++j) yh[b * ld + j] = j < nk ? (float)yv[j] : 0.f;
    }
    hipError_t e = hipMemcpyAsync(yd, yh.data(), yh.size() * sizeof(float), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) {
      snprintf(msg, sizeof msg, "GMRES coefficient write: %s", hipGetErrorString(e));
      return report_error(ES_EDEVICE, msg);
    }
    hipLaunchKernelGGL(k_gm_combine, grid, blk, 0, hs, n, (int)per, K, (const float*)V, vs, (const float*)yd, ld, x);
    if ((st = ok("GMRES combine launch")) != ES_OK) return st;
    if (!any_active() || it >= max_iter) break;
    // restart from the true residual r = b - A x: v_0 = r / ||r||
    if ((st = apply_a(x, w, true, part, false)) != ES_OK || (st = final_(1, nrm, 1)) != ES_OK) return st;
    hipLaunchKernelGGL(k_gm_scale, grid, blk, 0, hs, n, (int)per, (const float*)nrm, (const float*)w, V, mask, t);
    if ((st = ok("GMRES scale launch")) != ES_OK || (st = to_host(hn.data(), nrm, hn.size() * sizeof(float))) != ES_OK)
      return st;
    for (int64_t b = 0; b < batch; ++b) {
      beta[b] = std::sqrt((double)hn[b]);
      if (active[b] && !(beta[b] / bn[b] > rtol)) active[b] = 0;
    }
  }
  // true relative residual of the final iterate
  if ((st = apply_a(x, w, true, part, false)) != ES_OK || (st = final_(1, nrm, 1)) != ES_OK) return st;
  if ((st = to_host(hn.data(), nrm, hn.size() * sizeof(float))) != ES_OK) return st;
  for (int64_t b = 0; b < batch; ++b)
    rel_residual[b] = bn[b] > 0 ? (float)(std::sqrt((double)hn[b]) / bn[b]) : 0.f;
  if (iterations) *iterations = it;
  return ES_OK;
}

}  // extern "C"
