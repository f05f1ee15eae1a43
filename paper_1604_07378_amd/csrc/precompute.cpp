// Material tables and the stiffness rule of section 4.1 (Eq. stiffness):
// k is the slope of the least-squares line through the stress profile
// f(s) = a'(s) + 2 b'(s) + c'(s) (dPsi/ds1 at s2 = s3 = 1) on [lo, hi],
// k = 12 / L^3 * integral_lo^hi (s - mid) f(s) ds, with L = hi - lo.
#include <cmath>

#include "host.hpp"

namespace qn {

void spline_tables(Material& m) {
  // a'' is linear between knots; integrate exactly from s = 1 (knot 2), where
  // a(1) = a'(1) = 0, outwards in both directions.
  const int ref = 2;
  m.a0[ref] = 0.0;
  m.a1[ref] = 0.0;
  for (int j = ref; j < kSplineKnots - 1; ++j) {
    const double dx = spline_knot(j + 1) - spline_knot(j);
    const double c0 = m.d2[j], c1 = m.d2[j + 1];
    m.a1[j + 1] = m.a1[j] + dx * 0.5 * (c0 + c1);
    m.a0[j + 1] = m.a0[j] + m.a1[j] * dx + dx * dx * (2.0 * c0 + c1) / 6.0;
  }
  for (int j = ref; j > 0; --j) {
    const double dx = spline_knot(j) - spline_knot(j - 1);
    const double c0 = m.d2[j - 1], c1 = m.d2[j];
    m.a1[j - 1] = m.a1[j] - dx * 0.5 * (c0 + c1);
    m.a0[j - 1] = m.a0[j] - m.a1[j] * dx + dx * dx * (c0 + 2.0 * c1) / 6.0;
  }
}

namespace {

// a'(s) of the spline (quadratic on each knot interval, linear outside).
double spline_da(const Material& m, double s) {
  if (s <= spline_knot(0)) return m.a1[0] + m.d2[0] * (s - spline_knot(0));
  if (s >= spline_knot(7)) return m.a1[7] + m.d2[7] * (s - spline_knot(7));
  int j = (int)((s - 0.2) / 0.4);
  if (j > 6) j = 6;
  if (j < 0) j = 0;
  const double x = s - spline_knot(j);
  const double slope = (m.d2[j + 1] - m.d2[j]) / 0.4;
  return m.a1[j] + m.d2[j] * x + 0.5 * slope * x * x;
}

// Antiderivatives F(s) of (s - mid) * g(s) for the closed-form integrands.
double anti_lin(double s, double mid) {           // g(s) = s - 1
  return s * s * s / 3.0 - (mid + 1.0) * s * s / 2.0 + mid * s;
}

}  // namespace

double stiffness_fit(const Material& m, double lo, double hi) {
  const double L = hi - lo, mid = 0.5 * (lo + hi);
  const double scale = 12.0 / (L * L * L);
  // Mooney-Rivlin's stress profile is the Neo-Hookean one with shear
  // modulus mu + 2 mu2: f(s) = (mu + 2 mu2)(s - 1/s) + lam log(s) / s
  const double mu = m.type == MOONEY_RIVLIN ? m.mu + 2.0 * m.mu2 : m.mu, lam = m.lam;
  switch (m.type) {
    case NEOHOOKEAN:
    case MOONEY_RIVLIN: {
      // f(s) = mu s - mu / s + lam log(s) / s
      auto F = [&](double s) {
        const double ls = std::log(s);
        return mu * (s * s * s / 3.0 - mid * s * s / 2.0) - mu * (s - mid * ls) +
               lam * (s * ls - s - mid * 0.5 * ls * ls);
      };
      return scale * (F(hi) - F(lo));
    }
    case STVK: {
      // f(s) = (mu + lam/2)(s^3 - s)
      auto F = [&](double s) {
        return s * s * s * s * s / 5.0 - s * s * s / 3.0 - mid * (s * s * s * s / 4.0 - s * s / 2.0);
      };
      return scale * (mu + 0.5 * lam) * (F(hi) - F(lo));
    }
    case COROTATED:
      // f(s) = (2 mu + lam)(s - 1)
      return scale * (2.0 * mu + lam) * (anti_lin(hi, mid) - anti_lin(lo, mid));
    case POLYNOMIAL: {
      // f(s) = 4 mu (s - 1)^3; with u = s - 1: (s - mid) = u + (1 - mid)
      auto F = [&](double s) {
        const double u = s - 1.0;
        return u * u * u * u * u / 5.0 + (1.0 - mid) * u * u * u * u / 4.0;
      };
      return scale * 4.0 * mu * (F(hi) - F(lo));
    }
    case SPLINE: {
      // f(s) = a'(s) + lam (s - 1); (s - mid) a'(s) is a cubic on every knot
      // interval, so Simpson's rule on each piece is exact.
      double cuts[kSplineKnots + 2];
      int nc = 0;
      cuts[nc++] = lo;
      for (int j = 0; j < kSplineKnots; ++j)
        if (spline_knot(j) > lo && spline_knot(j) < hi) cuts[nc++] = spline_knot(j);
      cuts[nc++] = hi;
      double acc = 0.0;
      for (int i = 0; i + 1 < nc; ++i) {
        const double a = cuts[i], b = cuts[i + 1], c = 0.5 * (a + b);
        acc += (b - a) / 6.0 *
               ((a - mid) * spline_da(m, a) + 4.0 * (c - mid) * spline_da(m, c) + (b - mid) * spline_da(m, b));
      }
      return scale * acc + scale * lam * (anti_lin(hi, mid) - anti_lin(lo, mid));
    }
  }
  return 0.0;
}

}  // namespace qn
