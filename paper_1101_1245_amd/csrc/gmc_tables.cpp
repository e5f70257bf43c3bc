// gmc_tables.cpp -- double-precision construction of the FP32 tables read by
// the transport kernels: photon attenuation partials (Sec. II.A, Eq. 2),
// restricted stopping power and hard-event cross sections (Sec. II.B, Eqs.
// 5-6), transport mean free path for the multiple-scattering step
// (Sec. II.B.2), the screening inversion used by the angular sampler, and the
// Woodcock majorants (Eq. 3 and Sec. II.B.3).
//
// The physics is the effective-element model of the library's design notes:
// free-electron Klein-Nishina Compton scattering, a Z^4/E^3 photoelectric
// term, a threshold-shaped pair term, the Bethe collision stopping power
// without density effect, Moller hard collisions, a complete-screening
// bremsstrahlung cross section and screened-Rutherford elastic scattering.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gmc_tables.hpp"

namespace gmc {
namespace {

constexpr double kElectronRest = 0.51099895;       // MeV
constexpr double kElectronRadius = 2.8179403262e-13;  // cm
constexpr double kAvogadro = 6.02214076e23;
constexpr double kFine = 1.0 / 137.035999084;
constexpr double kPi = 3.14159265358979323846;
// Photoelectric calibration: water's Z^4/E^3 term meets Klein-Nishina at 26 keV.
constexpr double kPhotoConst = 1.9522732685184204e-31;  // cm^2
constexpr double kPairConst = 2.0;
constexpr double kTfRadius = 0.885;   // Thomas-Fermi radius in units of a0 Z^-1/3

struct Kin {
  double t, tau, gam, beta2, pc, beta;
  explicit Kin(double kinetic) : t(kinetic) {
    tau = t / kElectronRest;
    gam = tau + 1.0;
    beta2 = 1.0 - 1.0 / (gam * gam);
    pc = std::sqrt(t * (t + 2.0 * kElectronRest));
    beta = pc / (t + kElectronRest);
  }
};

class MaterialModel {
 public:
  explicit MaterialModel(const gmc_material& m) : za_(m.z_over_a), z_(m.z_eff), i_(m.i_ev * 1e-6) {
    const double a_eff = z_ / za_;
    x0_ = 716.4 * a_eff / (z_ * (z_ + 1.0) * std::log(287.0 / std::sqrt(z_)));
    electrons_per_gram_ = kAvogadro * za_;
  }

  // --- photons, cm^2/g ---
  double compton(double e) const {
    const double k = e / kElectronRest;
    const double l = std::log1p(2.0 * k);
    const double d = 1.0 + 2.0 * k;
    const double s = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / d - l / k) + l / (2.0 * k) - (1.0 + 3.0 * k) / (d * d);
    return electrons_per_gram_ * 2.0 * kPi * kElectronRadius * kElectronRadius * s;
  }
  double photo(double e) const {
    const double k = e / kElectronRest;
    return electrons_per_gram_ * kPhotoConst * z_ * z_ * z_ / (k * k * k);
  }
  double pair(double e) const {
    const double k = e / kElectronRest;
    if (k <= 2.0) return 0.0;
    const double f = 1.0 - 2.0 / k;
    return electrons_per_gram_ * (z_ + 1.0) * kFine * kElectronRadius * kElectronRadius * kPairConst *
           std::log(k / 2.0) * f * f * f;
  }

  // --- electrons ---
  // Bethe collision stopping power, MeV cm^2/g (no density effect).
  double stopping_col(double t) const {
    const Kin q(t);
    const double ir = i_ / kElectronRest;
    const double fm = 1.0 - q.beta2 + (q.tau * q.tau / 8.0 - (2.0 * q.tau + 1.0) * std::log(2.0)) / (q.gam * q.gam);
    return bethe_pref() / q.beta2 * (std::log(q.tau * q.tau * (q.tau + 2.0) / (2.0 * ir * ir)) + fm);
  }
  // Moller: number and energy of collisions transferring eps*T, eps in [kcut/T, 1/2].
  double moller_sigma(double t, double kcut) const {
    if (t <= 2.0 * kcut) return 0.0;
    const Kin q(t);
    const double e0 = kcut / t;
    const double r = q.tau / q.gam;
    const double c = (2.0 * q.tau + 1.0) / (q.gam * q.gam);
    const double integral = (1.0 / e0 - 2.0) + (2.0 - 1.0 / (1.0 - e0)) + r * r * (0.5 - e0) - c * std::log((1.0 - e0) / e0);
    return bethe_pref() / (q.beta2 * t) * integral;
  }
  double moller_hard_loss(double t, double kcut) const {
    if (t <= 2.0 * kcut) return 0.0;
    const Kin q(t);
    const double e0 = kcut / t;
    const double r = q.tau / q.gam;
    const double c = (2.0 * q.tau + 1.0) / (q.gam * q.gam);
    const double i1 = std::log(0.5 / e0);                                          // int eps/eps^2
    const double i2 = (2.0 + std::log(0.5)) - (1.0 / (1.0 - e0) + std::log(1.0 - e0));  // int eps/(1-eps)^2
    const double i3 = 0.5 * (0.25 - e0 * e0);                                      // int eps
    const double i4 = std::log(2.0 * (1.0 - e0));                                  // int 1/(1-eps)
    return bethe_pref() / q.beta2 * (i1 + i2 + r * r * i3 - c * i4);
  }
  // Complete-screening bremsstrahlung: number of photons above kc and energy
  // radiated below min(kc, T), per g/cm^2.
  double brems_sigma(double t, double kc) const {
    if (t <= kc) return 0.0;
    const double e = t + kElectronRest;
    return ((4.0 / 3.0) * std::log(t / kc) - (4.0 / 3.0) * (t - kc) / e + (t * t - kc * kc) / (2.0 * e * e)) / x0_;
  }
  double brems_soft_loss(double t, double kc) const {
    const double k = std::min(kc, t);
    const double e = t + kElectronRest;
    return ((4.0 / 3.0) * k - (2.0 / 3.0) * k * k / e + k * k * k / (3.0 * e * e)) / x0_;
  }
  // Restricted total stopping power L(E, K_cut) of Eq. 6.
  double restricted_loss(double t, double kcut, double kc) const {
    return stopping_col(t) - moller_hard_loss(t, kcut) + brems_soft_loss(t, kc);
  }
  // Screened-Rutherford inverse transport mean free path, cm^2/g.
  double inv_transport_mfp(double t) const {
    const Kin q(t);
    const double s = kFine * kElectronRest / q.pc * std::cbrt(z_) / kTfRadius;
    const double eta = 0.25 * s * s * (1.13 + 3.76 * (kFine * z_ / q.beta) * (kFine * z_ / q.beta));
    const double m = kElectronRest / (q.beta * q.pc);
    return 2.0 * kPi * kElectronRadius * kElectronRadius * electrons_per_gram_ * (z_ + 1.0) * m * m *
           (std::log1p(1.0 / eta) - 1.0 / (1.0 + eta));
  }

 private:
  double bethe_pref() const {
    return 2.0 * kPi * kAvogadro * kElectronRadius * kElectronRadius * kElectronRest * za_;
  }
  double za_, z_, i_, x0_, electrons_per_gram_;
};

double grid_energy(int i) {
  return kEmin * std::exp((double)i * std::log(kEmax / kEmin) / (double)(kNE - 1));
}

// First moment of 1 - cos for the screened-Rutherford shape with screening a.
double wentzel_moment(double a) {
  if (a > 50.0) {
    const double x = 1.0 / a;
    double s = 0.0, p = 1.0;
    for (int n = 1; n <= 14; ++n) {
      s += ((n % 2) ? 1.0 : -1.0) * p / (double)(n * (n + 1));
      p *= x;
    }
    return 2.0 * s;
  }
  return 2.0 * a * ((1.0 + a) * std::log1p(1.0 / a) - 1.0);
}

// ln A for a first moment g1, by Newton's method on ln A with a bracketing
// fallback (the moment rises monotonically with A).
double solve_ln_screening(double g1) {
  double lo = -80.0, hi = 40.0;
  double x = std::log(g1 / (1.0 - g1));   // ln A ~ logit(G1) - ln 3 near isotropy, close enough to start
  if (x < lo || x > hi) x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double a = std::exp(x);
    const double f = wentzel_moment(a) - g1;
    if (f > 0) hi = x; else lo = x;
    if (hi - lo < 1e-15) break;
    // derivative of the moment with respect to ln A, numerically
    const double h = 1e-6;
    const double df = (wentzel_moment(std::exp(x + h)) - wentzel_moment(std::exp(x - h))) / (2.0 * h);
    double xn = df > 0 ? x - f / df : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) < 1e-14) { x = xn; break; }
    x = xn;
  }
  return x;
}

}  // namespace

void build_tables(const gmc_material* mats, int n_mat, double kcut, double kc, HostTables* out) {
  out->n_mat = n_mat;
  out->ph.assign((size_t)n_mat * kNE, float4{0, 0, 0, 0});
  out->el.assign((size_t)n_mat * kNE, float4{0, 0, 0, 0});
  for (int m = 0; m < n_mat; ++m) {
    const MaterialModel mm(mats[m]);
    for (int i = 0; i < kNE; ++i) {
      const double e = grid_energy(i);
      const double c = mm.compton(e), p = mm.photo(e), q = mm.pair(e);
      out->ph[(size_t)m * kNE + i] = float4{(float)c, (float)(c + p), (float)(c + p + q), 0.0f};
      out->el[(size_t)m * kNE + i] = float4{(float)mm.restricted_loss(e, kcut, kc), (float)mm.moller_sigma(e, kcut),
                                            (float)mm.brems_sigma(e, kc), (float)mm.inv_transport_mfp(e)};
    }
  }
  // ln A at evenly spaced logit(G1) from G1 = 1e-12 to the isotropic threshold
  out->ms_y0 = std::log(1e-12 / (1.0 - 1e-12));
  const double y1 = std::log(0.9999 / (1.0 - 0.9999));
  out->ms_dy = (y1 - out->ms_y0) / (double)(kNms - 1);
  out->ms.resize(kNms);
  for (int i = 0; i < kNms; ++i) {
    const double y = out->ms_y0 + out->ms_dy * i;
    const double g1 = 1.0 / (1.0 + std::exp(-y));
    out->ms[i] = (float)solve_ln_screening(g1);
  }
}

void build_majorants(const HostTables& t, const double* rho_max, double margin, float* maj_g, float* maj_e) {
  double running = 0.0;
  for (int i = 0; i < kNE - 1; ++i) {
    double mu = 0.0, sg = 0.0;
    for (int m = 0; m < t.n_mat; ++m) {
      const double r = rho_max[m];
      if (!(r > 0.0)) continue;
      const float4 a = t.ph[(size_t)m * kNE + i], b = t.ph[(size_t)m * kNE + i + 1];
      mu = std::max(mu, r * std::max((double)a.z, (double)b.z));
      const float4 c = t.el[(size_t)m * kNE + i], d = t.el[(size_t)m * kNE + i + 1];
      sg = std::max(sg, r * std::max((double)c.y + (double)c.z, (double)d.y + (double)d.z));
    }
    running = std::max(running, sg);
    maj_g[i] = (float)(margin * mu);
    maj_e[i] = (float)(margin * running);
  }
  maj_g[kNE - 1] = maj_g[kNE - 2];
  maj_e[kNE - 1] = maj_e[kNE - 2];
}

}  // namespace gmc
