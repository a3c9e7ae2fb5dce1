// Host FP64 cosmology for the time-integration factors and the initial-condition amplitude:
// E(a), linear growth D(a) and f(a) (Sec. 2.2), kick and drift integrals of the leapfrog
// (Sec. 2.3.3 "timestep"), BBKS transfer function and sigma_8 normalisation (Sec. 2.3.2).
// Quadrature: adaptive Gauss-Legendre with nodes found by Newton iteration on P_n.
#include <cmath>
#include <functional>
#include <vector>

#include "cosmo.h"

namespace cube {
namespace {

struct GL {
  std::vector<double> x, w;
  explicit GL(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double p3 = p2;
          p2 = p1;
          p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        const double pp = n * (z * p1 - p2) / (z * z - 1.0);
        const double dz = p1 / pp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) {
          x[i] = z;
          w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
          break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
      }
    }
  }
  double apply(const std::function<double(double)>& f, double a, double b) const {
    const double h = 0.5 * (b - a), m = 0.5 * (b + a);
    double s = 0.0;
    for (size_t i = 0; i < x.size(); ++i) s += w[i] * f(m + h * x[i]);
    return s * h;
  }
};

const GL& gl20() {
  static const GL g(20);
  return g;
}

// Adaptive bisection: accept when two half-interval rules agree with the whole-interval rule to
// the relative tolerance or to the absolute floor `atol` (needed where the integral cancels).
double adapt(const std::function<double(double)>& f, double a, double b, double whole, double rtol, double atol,
             int depth) {
  const double m = 0.5 * (a + b);
  const double l = gl20().apply(f, a, m), r = gl20().apply(f, m, b);
  const double err = std::fabs(l + r - whole);
  if (depth >= 30 || err <= rtol * std::fabs(l + r) || err <= atol) return l + r;
  return adapt(f, a, m, l, rtol, 0.5 * atol, depth + 1) + adapt(f, m, b, r, rtol, 0.5 * atol, depth + 1);
}

double integrate(const std::function<double(double)>& f, double a, double b, double rtol = 1e-13,
                 double atol = 0.0) {
  if (a == b) return 0.0;
  const double whole = gl20().apply(f, a, b);
  const double floor_abs = atol > 0.0 ? atol : 1e-15 * std::fabs(whole);
  return adapt(f, a, b, whole, rtol, floor_abs, 0);
}

double tophat(double x) {
  if (std::fabs(x) < 1e-3) return 1.0 - x * x / 10.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

}  // namespace

double Cosmo::E(double a) const { return std::sqrt(om / (a * a * a) + ok / (a * a) + ol); }

double Cosmo::growth_unnorm(double a) const {
  auto f = [this](double x) {
    const double xe = x * E(x);
    return 1.0 / (xe * xe * xe);
  };
  // split near zero where the integrand behaves as x^{3/2}
  return E(a) * (integrate(f, 0.0, a * 1e-3) + integrate(f, a * 1e-3, a));
}

double Cosmo::f(double a) const {
  auto g = [this](double x) {
    const double xe = x * E(x);
    return 1.0 / (xe * xe * xe);
  };
  const double I = integrate(g, 0.0, a * 1e-3) + integrate(g, a * 1e-3, a);
  const double e = E(a);
  const double dlnE = -(3.0 * om / (a * a * a) + 2.0 * ok / (a * a)) / (2.0 * e * e);
  return dlnE + 1.0 / (a * a * e * e * e * I);
}

double Cosmo::kick(double a0, double a1) const {
  return integrate([this](double x) { return 1.0 / (x * x * E(x)); }, a0, a1);
}

double Cosmo::drift(double a0, double a1) const {
  return integrate([this](double x) { return 1.0 / (x * x * x * E(x)); }, a0, a1);
}

double Cosmo::transfer(double k) const {
  const double q = k / (om * h);
  if (q <= 0.0) return 1.0;
  const double t1 = std::log1p(2.34 * q) / (2.34 * q);
  const double poly = 1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) + std::pow(6.71 * q, 4);
  return t1 * std::pow(poly, -0.25);
}

double Cosmo::pk_shape(double k) const {
  const double t = transfer(k);
  return amp * std::pow(k, ns) * t * t;
}

double Cosmo::pk(double k, double a) const {
  const double d = D(a);
  return pk_shape(k) * d * d;
}

void Cosmo::init() {
  ok = 1.0 - om - ol;
  d_norm = growth_unnorm(1.0);
  // sigma^2(8 Mpc/h) of the shape k^ns T^2, integrated in ln k over pieces
  const double r = 8.0;
  auto integrand = [this, r](double lnk) {
    const double k = std::exp(lnk);
    const double t = transfer(k);
    const double w = tophat(k * r);
    return k * k * k * std::pow(k, ns) * t * t * w * w;
  };
  const double lo = std::log(1e-6), hi = std::log(300.0);
  const int pieces = 200;
  double rough = 0.0;
  for (int i = 0; i < pieces; ++i) {
    const double a0 = lo + (hi - lo) * i / pieces, a1 = lo + (hi - lo) * (i + 1) / pieces;
    rough += std::fabs(gl20().apply(integrand, a0, a1));
  }
  double s = 0.0;
  for (int i = 0; i < pieces; ++i) {
    const double a0 = lo + (hi - lo) * i / pieces, a1 = lo + (hi - lo) * (i + 1) / pieces;
    s += integrate(integrand, a0, a1, 1e-12, 1e-15 * rough / pieces);
  }
  s /= 2.0 * M_PI * M_PI;
  amp = sigma8 * sigma8 / s;
}

}  // namespace cube
