// Host FP64 background cosmology of the library (flat LambdaCDM without radiation): E(a),
// t(a) and its inverse in closed form, the linear growth factor (Heath integral) and rate,
// and the sigma_8 normalisation of the BBKS spectrum, by composite Simpson quadrature.
#pragma once

#include <cmath>
#include <vector>

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

// The Heath integral I(a) = int_0^a da' / (a' E(a'))^3 tabulated on s = sqrt(a) (a smooth
// integrand in s), with cubic Hermite interpolation from the exact derivative
// dI/ds = 2 s / (s^2 E(s^2))^3: for the per-step growth functions of the FastPM factors,
// which would otherwise need a fresh quadrature at every step.
struct HeathTable {
  double hs = 0.0;
  std::vector<double> I, dI;
  void build(const Cosmo& c, double a_max, int m = 2048) {
    const double smax = std::sqrt(a_max);
    hs = smax / m;
    auto f = [&](double s) {
      if (s == 0.0) return 0.0;
      const double ap = s * s;
      const double x = ap * c.E(ap);
      return 2.0 * s / (x * x * x);
    };
    I.assign(m + 1, 0.0);
    dI.assign(m + 1, 0.0);
    for (int k = 0; k <= m; ++k) {
      dI[k] = f(k * hs);
      if (k == 0) continue;
      const int sub = 16;   // Simpson over [s_{k-1}, s_k]
      const double h = hs / sub, s0 = (k - 1) * hs;
      double acc = f(s0) + f(s0 + hs);
      for (int i = 1; i < sub; ++i) acc += (i & 1 ? 4.0 : 2.0) * f(s0 + i * h);
      I[k] = I[k - 1] + acc * h / 3.0;
    }
  }
  bool covers(double a) const {
    return !I.empty() && a >= 0.0 && std::sqrt(a) <= hs * (static_cast<double>(I.size()) - 1);
  }
  double operator()(double a) const {
    const double s = std::sqrt(a);
    const int m = static_cast<int>(I.size()) - 1;
    int k = static_cast<int>(s / hs);
    if (k >= m) k = m - 1;
    const double t = s / hs - k, t2 = t * t, t3 = t2 * t;
    return (2 * t3 - 3 * t2 + 1) * I[k] + (t3 - 2 * t2 + t) * hs * dI[k] +
           (-2 * t3 + 3 * t2) * I[k + 1] + (t3 - t2) * hs * dI[k + 1];
  }
};

// Kick and drift factors of one kick-drift-kick step a0 -> a_half -> a1 that are exact for
// the linear growing mode (the modified KDK of FastPM): with the growth factor D, the
// momentum function G = a^2 dD/dt = a^2 E f D and the force function F = dG/dt = (3 Om / 2a) D
// (the linear growth equation), opening kick (G(a_half) - G(a0)) / F(a0), drift
// (D(a1) - D(a0)) / G(a_half), closing kick (G(a1) - G(a_half)) / F(a1).  The normalisation
// of D cancels; D_u = (5 Om / 2) E I from the table.
inline void fastpm_factors(const Cosmo& c, const HeathTable& T, double a0, double ah, double a1,
                           double* k_open, double* drift, double* k_close) {
  auto du = [&](double a) { return 2.5 * c.om * c.E(a) * (T.covers(a) ? T(a) : c.heath(a)); };
  auto gm = [&](double a) {
    const double e2 = c.E(a) * c.E(a), d = du(a);
    const double f = -1.5 * c.om / (a * a * a * e2) + 2.5 * c.om / (a * a * e2 * d);
    return a * a * c.E(a) * f * d;
  };
  auto fo = [&](double a) { return 1.5 * c.om * du(a) / a; };
  const double g0 = gm(a0), gh = gm(ah), g1 = gm(a1);
  *k_open = (gh - g0) / fo(a0);
  *drift = (du(a1) - du(a0)) / gh;
  *k_close = (g1 - gh) / fo(a1);
}

inline double bbks(double q) {
  return std::log(1.0 + 2.34 * q) / (2.34 * q) *
         std::pow(1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) +
                      std::pow(6.71 * q, 4),
                  -0.25);
}

// Eisenstein & Hu (1998) transfer function without the baryon oscillations, of k in h/Mpc
// (Sec. 2.1 sets the initial spectrum with the Eisenstein & Hu fitting formulae): the
// k-independent constants of its effective shape Gamma(k) = om h (alpha + (1 - alpha) /
// (1 + (0.43 k h s)^4)) and q = k theta^2 / Gamma, T = L / (L + C q^2), L = ln(2 e + 1.8 q),
// C = 14.2 + 731 / (1 + 62.5 q); s = 44.5 ln(9.83 / w_m) / sqrt(1 + 10 w_b^(3/4)) Mpc,
// alpha = 1 - 0.328 ln(431 w_m) f_b + 0.38 ln(22.3 w_m) f_b^2, theta = T_cmb / 2.7 K.
struct EhShape {
  double theta2, alpha, ks;   // ks = 0.43 h s: Gamma's cut-off in k [h/Mpc]^-1
  double omh;
};
inline EhShape eh_shape(double om, double ob, double h) {
  EhShape e;
  const double wm = om * h * h, wb = ob * h * h, fb = ob / om;
  const double s = 44.5 * std::log(9.83 / wm) / std::sqrt(1.0 + 10.0 * std::pow(wb, 0.75));
  e.alpha = 1.0 - 0.328 * std::log(431.0 * wm) * fb + 0.38 * std::log(22.3 * wm) * fb * fb;
  e.ks = 0.43 * h * s;
  e.theta2 = (2.7255 / 2.7) * (2.7255 / 2.7);
  e.omh = om * h;
  return e;
}
inline double eh_transfer(double k, const EhShape& e) {
  const double ks4 = std::pow(k * e.ks, 4);
  const double gamma = e.omh * (e.alpha + (1.0 - e.alpha) / (1.0 + ks4));
  const double q = k * e.theta2 / gamma;
  const double l = std::log(2.0 * M_E + 1.8 * q);
  const double c = 14.2 + 731.0 / (1.0 + 62.5 * q);
  return l / (l + c * q * q);
}

// A with sigma(8 Mpc/h) = sigma8 for P(k) = A k^n_s T(k)^2 (BBKS of k/(om h), or Eisenstein &
// Hu when eh); Simpson in ln k
inline double spectrum_amplitude(double om, double h, double n_s, double sigma8, bool eh = false,
                                 double ob = 0.05) {
  const double lo = std::log(1e-7), hi = std::log(1e4);
  const int m = 400000;
  const double dl = (hi - lo) / m;
  const EhShape es = eh_shape(om, ob, h);
  auto f = [&](double lk) {
    const double k = std::exp(lk);
    const double t = eh ? eh_transfer(k, es) : bbks(k / (om * h));
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
