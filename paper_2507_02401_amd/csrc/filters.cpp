// Daubechies extremal-phase filters, derived on the host at first use.
//
// The paper (Sec. 4, MRA paragraph and Def. 4.1) requires a compactly supported orthonormal
// scaling function of regularity r and leaves the family open; dbN is used.  Its low-pass
// filter follows from the spectral factorisation
//   |m0(w)|^2 = cos^{2N}(w/2) P(sin^2(w/2)),   P(y) = sum_{k<N} C(N-1+k, k) y^k :
// every root y of P maps to a reciprocal pair z, 1/z through y = (2 - z - 1/z)/4 and the
// extremal-phase (minimum-phase) choice keeps |z| < 1, so that
//   H(z) = c (1 + z^{-1})^N prod (1 - z_k z^{-1}),   h[t] = coefficient of z^{-t},
// normalised to sum_t h[t] = sqrt(2).  Roots are found with the Durand-Kerner iteration and
// polished with Newton steps, all in long double complex arithmetic.
#include <cmath>
#include <complex>
#include <mutex>
#include <vector>

#include "internal.h"

namespace es {
namespace {

using cld = std::complex<long double>;

cld horner(const std::vector<long double>& a, cld x) {  // a: highest degree first
  cld r = 0;
  for (long double c : a) r = r * x + c;
  return r;
}

cld horner_deriv(const std::vector<long double>& a, cld x) {
  cld r = 0;
  int deg = (int)a.size() - 1;
  for (int i = 0; i < deg; ++i) r = r * x + a[i] * (long double)(deg - i);
  return r;
}

std::vector<cld> poly_roots(const std::vector<long double>& a) {
  int deg = (int)a.size() - 1;
  std::vector<cld> r(deg);
  if (deg <= 0) return r;
  std::vector<long double> mon(a.size());
  for (size_t i = 0; i < a.size(); ++i) mon[i] = a[i] / a[0];
  cld seed(0.4L, 0.9L), p = 1;
  for (int k = 0; k < deg; ++k) { r[k] = p; p *= seed; }
  for (int it = 0; it < 2000; ++it) {
    long double moved = 0;
    for (int i = 0; i < deg; ++i) {
      cld den = 1;
      for (int j = 0; j < deg; ++j)
        if (j != i) den *= (r[i] - r[j]);
      cld step = horner(mon, r[i]) / den;
      r[i] -= step;
      moved = std::max(moved, std::abs(step));
    }
    if (moved < 1e-30L) break;
  }
  for (int i = 0; i < deg; ++i)
    for (int it = 0; it < 5; ++it) {
      cld d = horner_deriv(mon, r[i]);
      if (std::abs(d) == 0) break;
      r[i] -= horner(mon, r[i]) / d;
    }
  return r;
}

bool derive(int order, double* out) {
  const int n = order;
  std::vector<long double> P(n);  // highest degree first
  for (int k = 0; k < n; ++k) {
    long double c = 1;  // C(n-1+k, k)
    for (int j = 1; j <= k; ++j) c = c * (long double)(n - 1 + j) / (long double)j;
    P[n - 1 - k] = c;
  }
  std::vector<cld> ys = poly_roots(P);
  std::vector<cld> poly(1, cld(1));
  auto mul = [&](cld a0, cld a1) {  // poly *= (a0 + a1 w)
    std::vector<cld> q(poly.size() + 1, cld(0));
    for (size_t i = 0; i < poly.size(); ++i) { q[i] += poly[i] * a0; q[i + 1] += poly[i] * a1; }
    poly.swap(q);
  };
  for (int i = 0; i < n; ++i) mul(1, 1);
  for (cld y : ys) {
    cld b = 2.0L - 4.0L * y;
    cld disc = std::sqrt(b * b - 4.0L);
    cld z1 = (b + disc) / 2.0L, z2 = (b - disc) / 2.0L;
    mul(1, -(std::abs(z1) < 1 ? z1 : z2));
  }
  long double sum = 0;
  for (auto& c : poly) sum += c.real();
  const long double scale = std::sqrt(2.0L) / sum;
  for (int t = 0; t < 2 * n; ++t) out[t] = (double)(poly[t].real() * scale);
  // self-check: orthonormality of even shifts and the sum rule
  for (int l = 0; l < n; ++l) {
    long double dot = 0;
    for (int t = 0; t + 2 * l < 2 * n; ++t) dot += (long double)out[t] * out[t + 2 * l];
    if (std::fabs(dot - (l == 0 ? 1.0L : 0.0L)) > 1e-14L) return false;
  }
  return true;
}

struct Cache {
  std::once_flag once;
  bool ok[9] = {};
  double h[9][kMaxTaps] = {};
};
Cache& cache() {
  static Cache c;
  return c;
}

}  // namespace

bool daubechies_filter(int order, double* h_out) {
  if (order < 1 || order > 8) return false;
  Cache& c = cache();
  std::call_once(c.once, [&] {
    for (int o = 1; o <= 8; ++o) c.ok[o] = derive(o, c.h[o]);
  });
  if (!c.ok[order]) return false;
  for (int t = 0; t < 2 * order; ++t) h_out[t] = c.h[order][t];
  return true;
}

}  // namespace es
