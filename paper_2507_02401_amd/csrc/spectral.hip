// Fourier realisation of the adjoint embedding (Sec. 4, Implementation): y = ifft(B . fft(x)) with B the Bessel
// potential (1 + 4 pi^2 |xi|^2)^(-s) sampled on the FFT grid of a periodic box of side `period`.
//
// The transforms are hipFFT's (real-to-complex forward, complex-to-real inverse, one plan pair per
// geometry, cached); the multiplication by B and the 1/N of the inverse transform are one
// hand-written pass over the half spectrum.  B is formed in registers from the element's
// frequency, so no table is read.  The library may overwrite the input of an out-of-place
// transform, so the forward transform reads a copy of x made in y (skipped when x == y).

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "../../include/eswave.h"
#include "internal.h"

namespace es {

namespace {

// z holds rows of h2 = n2/2 + 1 complex values (the non-negative frequencies of the last axis);
// row r of the batch has leading-axis indices i1 = r mod n1, i0 = (r / n1) mod n0 (padded dims:
// 1 for absent axes).  Each work-group takes 256 >> SH consecutive rows at a time; within a row
// the threads stride by 1 << SH.  |frequency| of index i on an n-point axis is min(i, n - i).
__global__ void __launch_bounds__(256) k_fourier_scale(float2* __restrict__ z, int64_t rows, int n0, int n1, int h2,
                                                       int sh, float c, float neg_s, float inv_n) {
  const int rpw = 256 >> sh;
  const int lr = threadIdx.x >> sh;
  const int j0 = threadIdx.x & ((1 << sh) - 1);
  for (int64_t r0 = (int64_t)blockIdx.x * rpw; r0 < rows; r0 += (int64_t)gridDim.x * rpw) {
    const int64_t r = r0 + lr;
    if (r >= rows) continue;
    const int64_t q1 = r / n1;
    const int i1 = (int)(r - q1 * n1);
    const int i0 = (int)(q1 % n0);
    const float a1 = (float)min(i1, n1 - i1), a0 = (float)min(i0, n0 - i0);
    const float qrow = fmaf(a0, a0, a1 * a1);
    float2* __restrict__ row = z + r * h2;
    for (int j = j0; j < h2; j += 1 << sh) {
      const float fj = (float)j;
      const float q = fmaf(fj, fj, qrow);
      const float b = exp2f(neg_s * log2f(fmaf(c, q, 1.f))) * inv_n;
      float2 v = row[j];
      v.x *= b;
      v.y *= b;
      row[j] = v;
    }
  }
}

__global__ void __launch_bounds__(256) k_copy_floats(const float* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t n4 = n / 4;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  float4* d4 = reinterpret_cast<float4*>(dst);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
    d4[i] = s4[i];
  const int64_t t = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

struct PlanKey {
  int dev, ndim;
  int64_t n[3], batch;
  bool operator<(const PlanKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (ndim != o.ndim) return ndim < o.ndim;
    for (int k = 0; k < 3; ++k)
      if (n[k] != o.n[k]) return n[k] < o.n[k];
    return batch < o.batch;
  }
};

struct PlanPair {
  hipfftHandle fwd = 0, inv = 0;
  size_t work = 0;  // work-area bytes (the larger of the two plans)
};

std::mutex g_mu;  // guards the cache and every use of a cached plan (stream and work area are plan state)
std::map<PlanKey, PlanPair>& cache() {
  static auto* m = new std::map<PlanKey, PlanPair>();  // plans live until es_fft_release_plans()
  return *m;
}

const char* fft_name(hipfftResult r) {
  switch (r) {
    case HIPFFT_SUCCESS: return "HIPFFT_SUCCESS";
    case HIPFFT_INVALID_PLAN: return "HIPFFT_INVALID_PLAN";
    case HIPFFT_ALLOC_FAILED: return "HIPFFT_ALLOC_FAILED";
    case HIPFFT_INVALID_VALUE: return "HIPFFT_INVALID_VALUE";
    case HIPFFT_INTERNAL_ERROR: return "HIPFFT_INTERNAL_ERROR";
    case HIPFFT_EXEC_FAILED: return "HIPFFT_EXEC_FAILED";
    case HIPFFT_SETUP_FAILED: return "HIPFFT_SETUP_FAILED";
    case HIPFFT_INVALID_SIZE: return "HIPFFT_INVALID_SIZE";
    default: return "hipFFT error";
  }
}

es_status fft_fail(hipfftResult r, const char* where) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s (%d)", where, fft_name(r), (int)r);
  return report_error(r == HIPFFT_ALLOC_FAILED ? ES_ENOMEM : ES_EDEVICE, buf);
}

es_status einval(const char* msg) { return report_error(ES_EINVAL, msg); }

struct FftGeo {
  int ndim;
  int64_t n[3];  // the grid as given (ndim entries)
  int64_t N;     // voxels per instance
  int64_t h_last;  // n_last / 2 + 1
  int64_t spec_per;  // complex values per instance
};

es_status fft_geo(int ndim, const int64_t* shape, int64_t batch, FftGeo* g) {
  if (ndim < 1 || ndim > 3) return einval("ndim must be 1, 2 or 3");
  if (!shape) return einval("shape is NULL");
  if (batch < 0) return einval("batch must be >= 0");
  g->ndim = ndim;
  g->N = 1;
  for (int k = 0; k < ndim; ++k) {
    if (shape[k] < 2 || shape[k] > (1ll << 30)) return einval("every side must be in 2..2^30");
    g->n[k] = shape[k];
    g->N *= shape[k];
    if (g->N > 0x7fffffffll) return einval("an instance may hold at most 2^31-1 elements");
  }
  g->h_last = g->n[ndim - 1] / 2 + 1;
  g->spec_per = g->N / g->n[ndim - 1] * g->h_last;
  if (batch > 0 && g->spec_per > (int64_t)(0x7fffffffffffll / batch)) return einval("batch * size overflows");
  return ES_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Creates (or finds) the plan pair; caller holds g_mu.
es_status get_plans(const FftGeo& g, int64_t batch, PlanPair** out) {
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return report_error(ES_EDEVICE, hipGetErrorString(he));
  PlanKey key{dev, g.ndim, {0, 0, 0}, batch};
  for (int k = 0; k < g.ndim; ++k) key.n[k] = g.n[k];
  auto it = cache().find(key);
  if (it != cache().end()) {
    *out = &it->second;
    return ES_OK;
  }
  PlanPair pp;
  long long n[3], inem[3], onem[3];
  for (int k = 0; k < g.ndim; ++k) n[k] = inem[k] = onem[k] = g.n[k];
  onem[g.ndim - 1] = g.h_last;
  size_t wf = 0, wi = 0;
  hipfftResult r;
  if ((r = hipfftCreate(&pp.fwd)) != HIPFFT_SUCCESS) return fft_fail(r, "hipfftCreate");
  if ((r = hipfftCreate(&pp.inv)) != HIPFFT_SUCCESS) {
    hipfftDestroy(pp.fwd);
    return fft_fail(r, "hipfftCreate");
  }
  r = hipfftSetAutoAllocation(pp.fwd, 0);
  if (r == HIPFFT_SUCCESS) r = hipfftSetAutoAllocation(pp.inv, 0);
  if (r == HIPFFT_SUCCESS)
    r = hipfftMakePlanMany64(pp.fwd, g.ndim, n, inem, 1, g.N, onem, 1, g.spec_per, HIPFFT_R2C, batch, &wf);
  if (r == HIPFFT_SUCCESS)
    r = hipfftMakePlanMany64(pp.inv, g.ndim, n, onem, 1, g.spec_per, inem, 1, g.N, HIPFFT_C2R, batch, &wi);
  if (r != HIPFFT_SUCCESS) {
    hipfftDestroy(pp.fwd);
    hipfftDestroy(pp.inv);
    return fft_fail(r, "hipfftMakePlanMany64");
  }
  pp.work = wf > wi ? wf : wi;
  *out = &cache().emplace(key, pp).first->second;
  return ES_OK;
}

size_t spectrum_bytes(const FftGeo& g, int64_t batch) { return align256((size_t)(batch * g.spec_per) * 8); }

}  // namespace

}  // namespace es

using namespace es;

extern "C" {

es_status es_fft_workspace_bytes(int ndim, const int64_t* shape, int64_t batch, size_t* bytes) {
  if (!bytes) return einval("bytes is NULL");
  *bytes = 0;
  FftGeo g;
  es_status st = fft_geo(ndim, shape, batch, &g);
  if (st != ES_OK || batch == 0) return st;
  if ((st = device_check()) != ES_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  PlanPair* pp = nullptr;
  if ((st = get_plans(g, batch, &pp)) != ES_OK) return st;
  *bytes = spectrum_bytes(g, batch) + align256(pp->work);
  return ES_OK;
}

es_status es_fft_cov_apply(int ndim, const int64_t* shape, int64_t batch, double s, double period, const float* x,
                           float* y, void* ws, size_t ws_bytes, void* stream) {
  FftGeo g;
  es_status st = fft_geo(ndim, shape, batch, &g);
  if (st != ES_OK) return st;
  if (!std::isfinite(s)) return einval("s must be finite");
  if (!(period > 0) || !std::isfinite(period)) return einval("period must be finite and positive");
  if (batch == 0) return ES_OK;
  if (!x || !y) return einval("input and output pointers must be non-NULL");
  if (((uintptr_t)x & 15) || ((uintptr_t)y & 15)) return einval("input and output must be 16-byte aligned");
  const size_t io = (size_t)(batch * g.N) * sizeof(float);
  const char* px = (const char*)x;
  const char* py = (const char*)y;
  if (px != py && px < py + io && py < px + io) return einval("input and output overlap (only x == y is allowed)");
  if ((st = device_check()) != ES_OK) return st;
  hipStream_t hs = (hipStream_t)stream;

  std::lock_guard<std::mutex> lk(g_mu);
  PlanPair* pp = nullptr;
  if ((st = get_plans(g, batch, &pp)) != ES_OK) return st;
  const size_t spec = spectrum_bytes(g, batch);
  const size_t need = spec + align256(pp->work);
  if (!ws) return report_error(ES_EWORKSPACE, "workspace required (es_fft_workspace_bytes), got NULL");
  if (ws_bytes < need) {
    char buf[160];
    snprintf(buf, sizeof buf, "workspace of %zu bytes required, got %zu", need, ws_bytes);
    return report_error(ES_EWORKSPACE, buf);
  }
  if ((uintptr_t)ws & 255) return einval("workspace must be 256-byte aligned");
  const char* pw = (const char*)ws;
  if ((pw < px + io && px < pw + need) || (pw < py + io && py < pw + need))
    return einval("workspace overlaps input or output");

  float2* z = (float2*)ws;
  void* work = pp->work ? (void*)((char*)ws + spec) : nullptr;
  const int64_t n_all = batch * g.N;
  hipError_t he;
  if (x != y) {
    int64_t grid = (n_all / 4 + 255) / 256;
    grid = grid < 1 ? 1 : grid > 8192 ? 8192 : grid;
    hipLaunchKernelGGL(k_copy_floats, dim3((unsigned)grid), dim3(256), 0, hs, x, y, n_all);
    if ((he = hipGetLastError()) != hipSuccess) return report_error(ES_EDEVICE, hipGetErrorString(he));
  }
  hipfftResult r;
  if ((r = hipfftSetStream(pp->fwd, hs)) != HIPFFT_SUCCESS) return fft_fail(r, "hipfftSetStream");
  if ((r = hipfftSetWorkArea(pp->fwd, work)) != HIPFFT_SUCCESS) return fft_fail(r, "hipfftSetWorkArea");
  if ((r = hipfftExecR2C(pp->fwd, (hipfftReal*)y, (hipfftComplex*)z)) != HIPFFT_SUCCESS)
    return fft_fail(r, "hipfftExecR2C");

  // padded leading dims of the half spectrum: rows = batch * n0 * n1, h2 complex per row
  const int n0 = g.ndim == 3 ? (int)g.n[0] : 1;
  const int n1 = g.ndim >= 2 ? (int)g.n[g.ndim - 2] : 1;
  const int h2 = (int)g.h_last;
  const int64_t rows = batch * (g.N / g.n[g.ndim - 1]);
  int sh = 0;
  while ((1 << sh) < h2 && sh < 8) ++sh;
  const int rpw = 256 >> sh;
  int64_t grid = (rows + rpw - 1) / rpw;
  grid = grid > (1 << 20) ? (1 << 20) : grid;
  const double c = 4.0 * M_PI * M_PI / (period * period);
  hipLaunchKernelGGL(k_fourier_scale, dim3((unsigned)grid), dim3(256), 0, hs, z, rows, n0, n1, h2, sh, (float)c,
                     (float)(-s), (float)(1.0 / (double)g.N));
  if ((he = hipGetLastError()) != hipSuccess) return report_error(ES_EDEVICE, hipGetErrorString(he));

  if ((r = hipfftSetStream(pp->inv, hs)) != HIPFFT_SUCCESS) return fft_fail(r, "hipfftSetStream");
  if ((r = hipfftSetWorkArea(pp->inv, work)) != HIPFFT_SUCCESS) return fft_fail(r, "hipfftSetWorkArea");
  if ((r = hipfftExecC2R(pp->inv, (hipfftComplex*)z, (hipfftReal*)y)) != HIPFFT_SUCCESS)
    return fft_fail(r, "hipfftExecC2R");
  return ES_OK;
}

es_status es_fft_release_plans(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (cache().empty()) return ES_OK;
  int cur = 0;
  hipError_t he = hipGetDevice(&cur);
  if (he != hipSuccess) return report_error(ES_EDEVICE, hipGetErrorString(he));
  // work already enqueued with a plan must finish before its device memory is released
  for (auto it = cache().begin(); it != cache().end();) {
    const int dev = it->first.dev;
    if ((he = hipSetDevice(dev)) != hipSuccess || (he = hipDeviceSynchronize()) != hipSuccess) break;
    for (; it != cache().end() && it->first.dev == dev; it = cache().erase(it)) {
      hipfftDestroy(it->second.fwd);
      hipfftDestroy(it->second.inv);
    }
  }
  (void)hipSetDevice(cur);
  if (he != hipSuccess) return report_error(ES_EDEVICE, hipGetErrorString(he));
  return ES_OK;
}

}  // extern "C"
