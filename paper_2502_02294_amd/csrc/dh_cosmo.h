// Host FP64 background cosmology of the library (flat LambdaCDM without radiation): E(a),
// t(a) and its inverse in closed form, the linear growth factor (Heath integral) and rate,
// and the sigma_8 normalisation of the BBKS spectrum, by composite Simpson quadrature.
#pragma once

#include <cmath>

namespace dh {

struct Cosmo {
  double om, ol;

  double E(double a) const { return std::sqrt(om / (a * a * a) + ol); }
  double t_of_a(double a) const {
    return 2.0 / (3.0 * std::sqrt(ol)) * std::asinh(std::sqrt(ol / om) * std::pow(a, 1.5));
  }
  double a_of_t(double t) const {
    return std::cbrt(om / ol) * std::pow(std::sinh(1.5 * std::sqrt(ol) * t), 2.0 / 3.0);
  }
  // int_0^a da' / (a' E(a'))^3 with a' = s^2 (smooth integrand), Simpson on s
  double heath(double a) const {
    const int m = 4000;
    const double s1 = std::sqrt(a), hs = s1 / m;
    auto f = [&](double s) {
      if (s == 0.0) return 0.0;
      const double ap = s * s;
      const double x = ap * E(ap);
      return 2.0 * s / (x * x * x);
    };
    double acc = f(0.0) + f(s1);
    for (int i = 1; i < m; ++i) acc += (i & 1 ? 4.0 : 2.0) * f(i * hs);
    return acc * hs / 3.0;
  }
  double growth_u(double a) const { return 2.5 * om * E(a) * heath(a); }
  double growth(double a) const { return growth_u(a) / growth_u(1.0); }
  double growth_rate(double a) const {
    const double e2 = E(a) * E(a);
    return -1.5 * om / (a * a * a * e2) + 2.5 * om / (a * a * e2 * growth_u(a));
  }
};

inline double bbks(double q) {
  return std::log(1.0 + 2.34 * q) / (2.34 * q) *
         std::pow(1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) +
                      std::pow(6.71 * q, 4),
                  -0.25);
}

// A with sigma(8 Mpc/h) = sigma8 for P(k) = A k^n_s T(k/(om h))^2; Simpson in ln k
inline double spectrum_amplitude(double om, double h, double n_s, double sigma8) {
  const double lo = std::log(1e-7), hi = std::log(1e4);
  const int m = 400000;
  const double dl = (hi - lo) / m;
  auto f = [&](double lk) {
    const double k = std::exp(lk);
    const double t = bbks(k / (om * h));
    const double x = 8.0 * k;
    const double w = x < 1e-4 ? 1.0 - x * x / 10.0 : 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
    return k * k * k * std::pow(k, n_s) * t * t * w * w;
  };
  double acc = f(lo) + f(hi);
  for (int i = 1; i < m; ++i) acc += (i & 1 ? 4.0 : 2.0) * f(lo + i * dl);
  const double s2 = acc * dl / 3.0 / (2.0 * M_PI * M_PI);
  return sigma8 * sigma8 / s2;
}

}  // namespace dh
