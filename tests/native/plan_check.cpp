// Host-only driver of the plan planner and its table checks, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_plan_native.py (CPU only; no device call).
//
// Reads plans from stdin, one per block:
//   plan <op> <count>
//   <ndim> <n0> <n1> <n2> <order> <levels> <s>      (count lines; unused sides are 1)
// For each plan it builds the host plan (es_plan_create_host), lays the instances out as a
// caller would (every array 256-byte aligned, inputs, outputs and workspace apart), fills the
// tables for those addresses (es_plan_fill_host, which checks every launch's footprint against
// them), does it again for a second layout, and checks that a misaligned input, an undersized
// workspace and an input overlapping an output are refused.  Prints "ok <plans> <work-groups>".
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "eswave.h"
#include "internal.h"

// The launchers live in the HIP kernels; the host-only paths never reach them.
namespace es {
hipError_t launch_level(int, int, int, int, const TaskArgs&, int, const Filter&, hipStream_t) { abort(); }
hipError_t launch_lp_up_cge(int, int, const TaskArgs&, int, const Filter&, hipStream_t) { abort(); }
hipError_t launch_tail(int, int, int, const TailArgs&, int, size_t, const Filter&, hipStream_t) { abort(); }
hipError_t launch_plain_pass(const PlainPass&, int, const Filter&, hipStream_t) { abort(); }
hipError_t launch_block_copy(const float*, float*, const int*, const int*, const int*, hipStream_t) { abort(); }
hipError_t launch_copy(const float*, float*, int64_t, hipStream_t) { abort(); }
hipError_t launch_norm_finalize(const float2*, const NormSegs&, float*, int64_t, hipStream_t) { abort(); }
hipError_t launch_sumsq(const float*, int64_t, int64_t, float*, hipStream_t) { abort(); }
hipError_t launch_persist(int, int, const PArgs&, int, hipStream_t) { abort(); }
int persist_resident_groups(int, int) { abort(); }
hipError_t launch_zero_ints(int32_t*, int64_t, hipStream_t) { abort(); }
}  // namespace es

static uint64_t up256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

static int fill(es_plan* p, const std::vector<es_desc>& d, uint64_t base, uint64_t gap, int skew) {
  const int n = (int)d.size();
  std::vector<uint64_t> in(n), out(n);
  uint64_t cur = base;
  for (int k = 0; k < n; ++k) {
    uint64_t N = 1;
    for (int a = 0; a < d[k].ndim; ++a) N *= (uint64_t)d[k].shape[a];
    in[k] = cur;
    cur = up256(cur + 4 * N) + gap;
    out[k] = cur;
    cur = up256(cur + 4 * N) + gap;
  }
  if (skew) std::swap(in, out);  // outputs below inputs
  const size_t ws_bytes = es_plan_workspace_bytes(p);
  const uint64_t ws = up256(cur + 4096);
  int st = es_plan_fill_host(p, in.data(), out.data(), ws, ws_bytes);
  if (st != ES_OK) {
    fprintf(stderr, "fill failed: %s\n", es_last_error());
    return 1;
  }
  // refusals: misaligned input, short workspace, input overlapping an output
  if (n > 0) {
    std::vector<uint64_t> bad = in;
    bad[n - 1] += 4;
    if (es_plan_fill_host(p, bad.data(), out.data(), ws, ws_bytes) != ES_EINVAL) {
      fprintf(stderr, "misaligned input accepted\n");
      return 1;
    }
    if (ws_bytes && es_plan_fill_host(p, in.data(), out.data(), ws, ws_bytes - 4) != ES_EWORKSPACE) {
      fprintf(stderr, "short workspace accepted\n");
      return 1;
    }
    bad = in;
    bad[0] = out[0] + 256;
    uint64_t N0 = 1;
    for (int a = 0; a < d[0].ndim; ++a) N0 *= (uint64_t)d[0].shape[a];
    if (N0 * 4 > 256 && es_plan_fill_host(p, bad.data(), out.data(), ws, ws_bytes) != ES_EINVAL) {
      fprintf(stderr, "overlapping input accepted\n");
      return 1;
    }
    // the good layout again (the last call must leave valid tables)
    if (es_plan_fill_host(p, in.data(), out.data(), ws, ws_bytes) != ES_OK) return 1;
  }
  return 0;
}

int main() {
  char word[32];
  int plans = 0;
  long long wgs = 0;
  while (scanf("%31s", word) == 1) {
    if (strcmp(word, "plan") != 0) {
      fprintf(stderr, "bad input\n");
      return 2;
    }
    int op = 0, count = 0;
    if (scanf("%d %d", &op, &count) != 2) return 2;
    std::vector<es_desc> d(count);
    for (int k = 0; k < count; ++k) {
      long long n0, n1, n2;
      if (scanf("%d %lld %lld %lld %d %d %lf", &d[k].ndim, &n0, &n1, &n2, &d[k].order, &d[k].levels, &d[k].s) != 7)
        return 2;
      d[k].shape[0] = n0;
      d[k].shape[1] = n1;
      d[k].shape[2] = n2;
      d[k].reserved = 0;
    }
    es_plan* p = nullptr;
    if (es_plan_create_host(d.data(), count, op, &p) != ES_OK) {
      fprintf(stderr, "plan %d: create failed: %s\n", plans, es_last_error());
      return 1;
    }
    if (fill(p, d, (uint64_t)1 << 32, 0, 0) || fill(p, d, (uint64_t)3 << 40, 4096, 1)) {
      fprintf(stderr, "plan %d (op %d, %d instances) failed\n", plans, op, count);
      es_plan_destroy(p);
      return 1;
    }
    wgs += es_plan_work_groups(p);
    es_plan_destroy(p);
    ++plans;
  }
  printf("ok %d %lld\n", plans, wgs);
  return 0;
}
