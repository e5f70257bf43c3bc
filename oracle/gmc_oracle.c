/*
 * gmc_oracle.c -- plain FP64 CPU oracle for the coupled photon-electron
 * transport of Hissoiny et al. (GPUMCD), Sec. II.A (photons) and Sec. II.B
 * (electrons), with the statistics of Sec. II.D.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library.  Everything is evaluated from closed forms in double
 * precision, one history at a time, depth first, single-threaded; there is no
 * tabulation except the majorant grid that the Woodcock scheme of Sec. II.A
 * (Eq. 3) needs.
 *
 * Where the paper relies on material that is not reproduced in it (PEGS4
 * data, the EGSnrc and PENELOPE sampling routines, the Kawrakow-Bielajew
 * multiple-scattering data), the physics model is re-specified from closed
 * forms; each such substitution is marked "[reading]" below and is listed
 * with its justification in the design notes of the repository.
 */
#include "gmc_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Physical constants (CODATA 2018).                                   */
#define MC2    0.51099895          /* electron rest energy, MeV */
#define RE     2.8179403262e-13    /* classical electron radius, cm */
#define NAV    6.02214076e23       /* Avogadro, 1/mol */
#define ALPHA  (1.0 / 137.035999084)
#define TWOPI  6.283185307179586476925286766559
#define PI     3.141592653589793238462643383280
/* 2 pi N_A r_e^2 m c^2, MeV cm^2 / mol */
#define K2     (TWOPI * NAV * RE * RE * MC2)
/* [reading] photoelectric constant: water's photoelectric and Compton
 * coefficients (Z/A 0.55509, Z 7.42) cross at 26 keV. */
#define C_PE   1.9522732685184204e-31
/* [reading] pair-term constant multiplying the threshold-shaped log. */
#define C_PAIR 2.0
/* Screening constant of the Thomas-Fermi radius, a_TF = 0.885 a_0 Z^-1/3. */
#define TF_C   0.885

/* Majorant grid: log-spaced nodes on [1 keV, 32 MeV]. */
#define NE     1024
#define EMIN   1.0e-3
#define EMAX   32.0
#define MAJ_MARGIN 1.001
/* [reading] multiple scattering is taken as isotropic at or above this G1. */
#define G1_ISO 0.9999

/* [reading] the electron voxel skin as a fraction of the smallest voxel width
 * (1e-4); tests may change it to show that the dose does not depend on it. */
static double g_skin_fraction = 1e-4;
void orc_set_skin_fraction(double f) { if (f > 0.0 && f < 0.5) g_skin_fraction = f; }

/* ------------------------------------------------------------------ */
/* Philox4x32-10 and Philox4x64-10 (Salmon et al., SC'11).            */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B97F4A7C15ull; k1 += 0xBB67AE8584CAA73Bull; }
    __uint128_t p0 = (__uint128_t)0xD2E7470EE14C6C93ull * c0;
    __uint128_t p1 = (__uint128_t)0xCA5A826395121157ull * c2;
    uint64_t n0 = (uint64_t)(p1 >> 64) ^ c1 ^ k0;
    uint64_t n1 = (uint64_t)p1;
    uint64_t n2 = (uint64_t)(p0 >> 64) ^ c3 ^ k1;
    uint64_t n3 = (uint64_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 64-bit finalizer of splitmix64: gives each child particle its own stream
 * path without drawing from the parent's stream.  The input is offset by the
 * splitmix64 increment so that the root path 0 is not a fixed point. */
static uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27; z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

uint64_t orc_child_path(uint64_t parent_path, uint32_t parent_n, uint32_t child_idx) {
  return mix64((parent_path ^ (((uint64_t)parent_n << 2) | (uint64_t)child_idx)) + 0x9E3779B97F4A7C15ull);
}

/* One particle's stream: counter = (n >> 2, path lo, path hi, history),
 * key = (seed lo, seed hi ^ beam).  Word n of the stream is word (n & 3) of
 * that block. */
typedef struct {
  uint32_t key[2];
  uint32_t hist;
  uint64_t path;
  uint32_t n;
  uint32_t blk[4];
  uint32_t blk_id;
  int have;
} stream_t;

static void stream_init(stream_t* s, const uint32_t key[2], uint32_t hist, uint64_t path, uint32_t n) {
  s->key[0] = key[0]; s->key[1] = key[1];
  s->hist = hist; s->path = path; s->n = n; s->have = 0;
}

/* Every photon event and every electron step starts at the next block
 * boundary of the particle's stream. */
static void stream_align(stream_t* s) { s->n = (s->n + 3u) & ~3u; }

static uint32_t stream_word(stream_t* s) {
  uint32_t id = s->n >> 2;
  if (!s->have || s->blk_id != id) {
    uint32_t ctr[4] = { id, (uint32_t)s->path, (uint32_t)(s->path >> 32), s->hist };
    orc_philox4x32(ctr, s->key, s->blk);
    s->blk_id = id; s->have = 1;
  }
  uint32_t w = s->blk[s->n & 3u];
  s->n++;
  return w;
}

/* Uniform in (0,1): the top 24 bits with the lowest forced to 1, i.e. an odd
 * multiple of 2^-24.  Such values are exact in binary32 and binary64, and
 * neither 0 nor 1 occurs (the zeta of Eq. 1 must avoid ln 0). */
static double word_to_u(uint32_t w) { return (double)((w >> 8) | 1u) * 0x1p-24; }
static double next_u(stream_t* s) { return word_to_u(stream_word(s)); }

static void make_key(uint64_t seed, uint32_t beam, uint32_t key[2]) {
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32) ^ beam;
}

void orc_stream_words(uint64_t seed, uint32_t beam, uint32_t hist, uint64_t path,
                      uint32_t n0, int count, uint32_t* words, double* uniforms) {
  uint32_t key[2]; make_key(seed, beam, key);
  stream_t s; stream_init(&s, key, hist, path, n0);
  for (int i = 0; i < count; ++i) {
    uint32_t w = stream_word(&s);
    if (words) words[i] = w;
    if (uniforms) uniforms[i] = word_to_u(w);
  }
}

/* ------------------------------------------------------------------ */
/* Materials and closed-form cross sections.                          */
typedef struct {
  double za, z, i_mev;   /* Z/A, Z_eff, I */
  double x0;             /* radiation length, g/cm^2 */
} mat_t;

static void mat_init(mat_t* m, const orc_material* in) {
  m->za = in->z_over_a; m->z = in->z_eff; m->i_mev = in->i_ev * 1e-6;
  double a = m->z / m->za;  /* effective atomic mass */
  m->x0 = 716.4 * a / (m->z * (m->z + 1.0) * log(287.0 / sqrt(m->z)));
}

/* Total Klein-Nishina cross section per electron (cm^2), k = E / mc^2
 * (Compton on free electrons, Sec. II.A). */
static double sigma_kn(double k) {
  double a = log1p(2.0 * k);
  double b = 1.0 + 2.0 * k;
  return TWOPI * RE * RE *
         ((1.0 + k) / (k * k) * (2.0 * (1.0 + k) / b - a / k) + a / (2.0 * k) -
          (1.0 + 3.0 * k) / (b * b));
}

/* Eq. 2: mu/rho = (N_A / A) sigma, here per unit density (cm^2/g). */
static double mu_compton(const mat_t* m, double e) { return NAV * m->za * sigma_kn(e / MC2); }

/* [reading] K-shell photoelectric term with a per-atom Z^4 E^-3 law
 * (Sec. II.A: all electrons from the K shell, no relaxation). */
static double mu_photo(const mat_t* m, double e) {
  double k = e / MC2;
  return NAV * m->za * C_PE * m->z * m->z * m->z / (k * k * k);
}

/* [reading] pair term (Sec. II.A): Z(Z+1)/A scaling with a threshold-shaped
 * logarithm, zero at and below 2 mc^2. */
static double mu_pair(const mat_t* m, double e) {
  double k = e / MC2;
  if (k <= 2.0) return 0.0;
  double t = 1.0 - 2.0 / k;
  return NAV * m->za * (m->z + 1.0) * ALPHA * RE * RE * C_PAIR * log(0.5 * k) * t * t * t;
}

static double mu_total(const mat_t* m, double e) {
  return mu_compton(m, e) + mu_photo(m, e) + mu_pair(m, e);
}

/* Collision stopping power (Bethe formula for electrons, density effect
 * omitted), MeV cm^2/g: the S of Eq. 5. */
static double s_col(const mat_t* m, double t) {
  double tau = t / MC2, g = tau + 1.0;
  double b2 = 1.0 - 1.0 / (g * g);
  double ir = m->i_mev / MC2;
  double f = 1.0 - b2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * log(2.0)) / (g * g);
  return K2 * m->za / b2 * (log(tau * tau * (tau + 2.0) / (2.0 * ir * ir)) + f);
}

/* Moller cross section for energy transfers eps*T with eps in [kcut/T, 1/2]
 * (Sec. II.B.1, free electrons, no spin effects), cm^2/g. */
static double sig_moller(const mat_t* m, double t, double kcut) {
  if (t <= 2.0 * kcut) return 0.0;
  double tau = t / MC2, g = tau + 1.0;
  double b2 = 1.0 - 1.0 / (g * g);
  double e0 = kcut / t, r = tau / g;
  double c = (2.0 * tau + 1.0) / (g * g);
  return K2 * m->za / (b2 * t) *
         (1.0 / e0 - 1.0 / (1.0 - e0) + r * r * (0.5 - e0) - c * log((1.0 - e0) / e0));
}

/* Energy lost per unit path to Moller transfers above kcut, MeV cm^2/g. */
static double eloss_moller_hard(const mat_t* m, double t, double kcut) {
  if (t <= 2.0 * kcut) return 0.0;
  double tau = t / MC2, g = tau + 1.0;
  double b2 = 1.0 - 1.0 / (g * g);
  double e0 = kcut / t, r = tau / g;
  double c = (2.0 * tau + 1.0) / (g * g);
  return K2 * m->za / b2 *
         (log(1.0 / (2.0 * e0)) + 2.0 - log(2.0) - 1.0 / (1.0 - e0) - log(1.0 - e0) +
          r * r * (0.125 - 0.5 * e0 * e0) - c * log(2.0 * (1.0 - e0)));
}

/* Restricted collision stopping power: Eq. 6 for the collision part. */
static double l_col(const mat_t* m, double t, double kcut) {
  return s_col(m, t) - eloss_moller_hard(m, t, kcut);
}

/* [reading] bremsstrahlung: complete-screening cross section
 * dSigma/dk = (1/X0)(1/k)(4/3 - 4y/3 + y^2), y = k/E, E total energy. */
static double sig_brems(const mat_t* m, double t, double kc) {
  if (t <= kc) return 0.0;
  double e = t + MC2;
  return ((4.0 / 3.0) * log(t / kc) - (4.0 / 3.0) * (t - kc) / e + (t * t - kc * kc) / (2.0 * e * e)) / m->x0;
}

static double rad_loss_below(const mat_t* m, double t, double kk) {
  double e = t + MC2;
  return ((4.0 / 3.0) * kk - (2.0 / 3.0) * kk * kk / e + kk * kk * kk / (3.0 * e * e)) / m->x0;
}

static double l_rad(const mat_t* m, double t, double kc) { return rad_loss_below(m, t, t < kc ? t : kc); }
static double s_rad(const mat_t* m, double t) { return rad_loss_below(m, t, t); }

/* Total restricted stopping power L(E, K_cut) of Eq. 6. */
static double l_total(const mat_t* m, double t, double kcut, double kc) {
  return l_col(m, t, kcut) + l_rad(m, t, kc);
}

/* [reading] multiple scattering (Sec. II.B.2): screened-Rutherford (Wentzel)
 * elastic scattering with Moliere's screening parameter. */
static double screening_eta(const mat_t* m, double t) {
  double pc = sqrt(t * (t + 2.0 * MC2));
  double beta = pc / (t + MC2);
  double a = ALPHA * MC2 / pc * cbrt(m->z) / TF_C;
  double az = ALPHA * m->z / beta;
  return 0.25 * a * a * (1.13 + 3.76 * az * az);
}

/* Inverse transport mean free path per unit density (cm^2/g). */
static double inv_lambda1(const mat_t* m, double t) {
  double pc = sqrt(t * (t + 2.0 * MC2));
  double beta = pc / (t + MC2);
  double eta = screening_eta(m, t);
  double q = MC2 / (beta * pc);
  return TWOPI * RE * RE * NAV * m->za * (m->z + 1.0) * q * q * (log1p(1.0 / eta) - 1.0 / (1.0 + eta));
}

int orc_xs(const orc_material* in, int which, const double* e, int n, double kcut, double kc, double* out) {
  mat_t m; mat_init(&m, in);
  for (int i = 0; i < n; ++i) {
    double x = e[i], v;
    switch (which) {
      case 0: v = mu_compton(&m, x); break;
      case 1: v = mu_photo(&m, x); break;
      case 2: v = mu_pair(&m, x); break;
      case 3: v = s_col(&m, x); break;
      case 4: v = sig_moller(&m, x, kcut); break;
      case 5: v = eloss_moller_hard(&m, x, kcut); break;
      case 6: v = l_col(&m, x, kcut); break;
      case 7: v = sig_brems(&m, x, kc); break;
      case 8: v = l_rad(&m, x, kc); break;
      case 9: v = s_rad(&m, x); break;
      case 10: v = l_total(&m, x, kcut, kc); break;
      case 11: v = inv_lambda1(&m, x); break;
      case 12: v = screening_eta(&m, x); break;
      default: return -1;
    }
    out[i] = v;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Direction change by polar cos(theta) and azimuth phi about d.       */
static void rotate(const double d[3], double cost, double phi, double out[3]) {
  if (cost > 1.0) cost = 1.0;
  if (cost < -1.0) cost = -1.0;
  double sint = sqrt((1.0 - cost) * (1.0 + cost));
  double cp = cos(phi), sp = sin(phi);
  double u = d[0], v = d[1], w = d[2];
  double rho2 = u * u + v * v;
  double nu, nv, nw;
  if (rho2 > 1e-20) {
    double r = sqrt(rho2);
    nu = u * cost + sint * (u * w * cp - v * sp) / r;
    nv = v * cost + sint * (v * w * cp + u * sp) / r;
    nw = w * cost - r * sint * cp;
  } else {
    nu = sint * cp;
    nv = sint * sp;
    nw = (w >= 0.0) ? cost : -cost;
  }
  double inv = 1.0 / sqrt(nu * nu + nv * nv + nw * nw);
  out[0] = nu * inv; out[1] = nv * inv; out[2] = nw * inv;
}

void orc_rotate(const double d[3], double cost, double phi, double out[3]) { rotate(d, cost, phi, out); }

/* ------------------------------------------------------------------ */
/* Samplers.  Each consumes uniforms from the particle's own stream in a
 * fixed order; the HIP path follows the same order.                  */

/* Compton (Sec. II.A) [reading: the Everett direct method is not given, so the
 * Klein-Nishina epsilon = E'/E is drawn by composition-rejection]:
 * 1/eps with weight ln(1/eps0), eps with weight (1-eps0^2)/2, accepted with
 * 1 - eps sin^2(theta)/(1+eps^2).  Three uniforms per trial. */
static void sample_kn(double k, stream_t* s, double* eps_out, double* cost_out) {
  double eps0 = 1.0 / (1.0 + 2.0 * k);
  double a1 = log1p(2.0 * k);
  double a2 = 0.5 * (1.0 - eps0 * eps0);
  for (;;) {
    double u1 = next_u(s), u2 = next_u(s), u3 = next_u(s);
    double eps;
    if (u1 * (a1 + a2) < a1) eps = exp(-a1 * u2);
    else eps = sqrt(eps0 * eps0 + (1.0 - eps0 * eps0) * u2);
    double t = (1.0 - eps) / (k * eps);
    double sin2 = t * (2.0 - t);
    double g = 1.0 - eps * sin2 / (1.0 + eps * eps);
    if (u3 <= g) { *eps_out = eps; *cost_out = 1.0 - t; return; }
  }
}

/* Photoelectron polar angle from the Sauter K-shell distribution (Sec. II.A).
 * With nu = 1 - cos(theta), A = 1/beta - 1 and B = beta g (g-1)(g-2)/2, the
 * density is proportional to (2 - nu) nu/(A+nu)^3 [1/(A+nu) + B]; nu is
 * drawn from nu/(A+nu)^3 on [0, 2] by inversion and accepted with
 * (2-nu)(1/(A+nu) + B) / (2/A + 2 max(B, 0)).  Two uniforms per trial. */
static double sample_sauter(double t, stream_t* s) {
  double g = 1.0 + t / MC2;
  double beta = sqrt(t * (t + 2.0 * MC2)) / (t + MC2);
  double a = 1.0 / (g * g * beta * (1.0 + beta));   /* = 1/beta - 1 */
  double b = 0.5 * beta * g * (g - 1.0) * (g - 2.0);
  double mx = 2.0 / a + 2.0 * (b > 0.0 ? b : 0.0);
  for (;;) {
    double u1 = next_u(s), u2 = next_u(s);
    double q = 2.0 * sqrt(u1) / (a + 2.0);
    double nu = q * a / (1.0 - q);
    double f = (2.0 - nu) * (1.0 / (a + nu) + b);
    if (u2 * mx <= f) return 1.0 - nu;
  }
}

/* [reading] pair-electron polar angle: p(cos theta) ~ (1 - beta cos theta)^-2,
 * inverted in closed form.  One uniform. */
static double pair_cos(double t, double u) {
  double g = 1.0 + t / MC2;
  double beta = sqrt(t * (t + 2.0 * MC2)) / (t + MC2);
  double omb = 1.0 / (g * g * (1.0 + beta));           /* 1 - beta */
  return (2.0 * u - 1.0 + beta) / (omb + 2.0 * beta * u);
}

/* Moller energy fraction eps in [kcut/T, 1/2] (Sec. II.B.1): mixture of
 * 1/eps^2 (weight 1/eps0 - 2) and a flat part (weight 5(1/2 - eps0)),
 * accepted with h(eps)/(1 + 5 eps^2) where eps^-2 h(eps) is the bracket of
 * the Moller cross section.  Three uniforms per trial. */
static double sample_moller(double t, double kcut, stream_t* s) {
  double tau = t / MC2, g = tau + 1.0;
  double e0 = kcut / t;
  double r2 = (tau / g) * (tau / g);
  double c = (2.0 * tau + 1.0) / (g * g);
  double w1 = 1.0 / e0 - 2.0, w2 = 5.0 * (0.5 - e0);
  for (;;) {
    double u1 = next_u(s), u2 = next_u(s), u3 = next_u(s);
    double eps;
    if (u1 * (w1 + w2) < w1) eps = 1.0 / (1.0 / e0 - u2 * (1.0 / e0 - 2.0));
    else eps = e0 + u2 * (0.5 - e0);
    double q = eps / (1.0 - eps);
    double h = 1.0 + q * q + r2 * eps * eps - c * q;
    if (u3 * (1.0 + 5.0 * eps * eps) <= h) return eps;
  }
}

/* Bremsstrahlung photon energy k in [kc, T] (Sec. II.B.1): log-uniform
 * proposal accepted with (4/3 - 4y/3 + y^2)/(4/3).  Two uniforms per trial. */
static double sample_brems(double t, double kc, stream_t* s) {
  double e = t + MC2;
  double lr = log(t / kc);
  for (;;) {
    double u1 = next_u(s), u2 = next_u(s);
    double k = kc * exp(u1 * lr);
    double y = k / e;
    if (u2 * (4.0 / 3.0) <= 4.0 / 3.0 - (4.0 / 3.0) * y + y * y) return k;
  }
}

/* Mean of 1 - cos(theta) for the screened-Rutherford shape with screening A:
 * 2A[(1+A) ln(1+1/A) - 1]; a series in 1/A is used for large A. */
static double wentzel_g1(double a) {
  if (a > 100.0) {
    double x = 1.0 / a, sum = 0.0, p = 1.0;
    for (int n = 1; n <= 12; ++n) {
      sum += ((n & 1) ? 1.0 : -1.0) * p / (double)(n * (n + 1));
      p *= x;
    }
    return 2.0 * sum;
  }
  return 2.0 * a * ((1.0 + a) * log1p(1.0 / a) - 1.0);
}

/* Screening A such that the per-step mean of 1 - cos(theta) equals G1, by
 * bisection on ln A (the mean rises monotonically with A). */
double orc_ms_screening_A(double g1) {
  double lo = -700.0, hi = 700.0;
  for (int it = 0; it < 64; ++it) {   /* 1400 / 2^64: ln A to ~1e-16 */
    double mid = 0.5 * (lo + hi);
    if (wentzel_g1(exp(mid)) < g1) lo = mid; else hi = mid;
  }
  return exp(0.5 * (lo + hi));
}

/* Polar cosine for a step with first-moment parameter G1 = 1 - exp(-s/lambda_1):
 * w = 1 - cos(theta) = 2 A u / (1 + A - u).  One uniform. */
static double wentzel_cos(double g1, double u) {
  if (!(g1 > 0.0)) return 1.0;
  if (g1 >= G1_ISO) return 1.0 - 2.0 * u;
  double a = orc_ms_screening_A(g1);
  return 1.0 - 2.0 * a * u / (1.0 + a - u);
}

int orc_sample(int which, double p1, double p2, uint64_t seed, int count, double* out, double* out2) {
  uint32_t key[2]; make_key(seed, 0, key);
  stream_t s; stream_init(&s, key, 0, 0, 0);
  for (int i = 0; i < count; ++i) {
    switch (which) {
      case 0: { double e, c; sample_kn(p1 / MC2, &s, &e, &c); out[i] = e; if (out2) out2[i] = c; break; }
      case 1: out[i] = sample_sauter(p1, &s); break;
      case 2: out[i] = pair_cos(p1, next_u(&s)); break;
      case 3: out[i] = sample_moller(p1, p2, &s); break;
      case 4: out[i] = sample_brems(p1, p2, &s); break;
      case 5: out[i] = wentzel_cos(p1, next_u(&s)); break;
      default: return -1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Event kinematics.  Each takes the incoming particle's energy and direction,
 * draws from its stream in a fixed order and returns the outgoing particles;
 * the transport below calls exactly these, and orc_event exposes them to the
 * tests, which check them against the conservation laws they must obey.    */

/* Compton (Sec. II.A): scattered photon (e1, d1) and recoil electron (t, dt);
 * the electron's direction is that of the momentum the photon gave up,
 * E d - E1 d1 (units of MeV/c), so momentum is conserved exactly and
 * |E d - E1 d1| = sqrt(t (t + 2 mc^2)) is the Compton relation. */
static void compton_event(double e, const double d[3], stream_t* s, double* e1, double d1[3], double* t,
                          double dt[3]) {
  double eps, cost;
  sample_kn(e / MC2, s, &eps, &cost);
  double phi = TWOPI * next_u(s);
  rotate(d, cost, phi, d1);
  *e1 = eps * e;
  *t = e - *e1;
  double pe[3] = { e * d[0] - *e1 * d1[0], e * d[1] - *e1 * d1[1], e * d[2] - *e1 * d1[2] };
  double n2 = pe[0] * pe[0] + pe[1] * pe[1] + pe[2] * pe[2];
  double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  dt[0] = pe[0] * inv; dt[1] = pe[1] * inv; dt[2] = pe[2] * inv;
}

/* Photoelectric (Sec. II.A): one electron with the whole photon energy
 * (binding neglected) in the Sauter direction. */
static void photo_event(double e, const double d[3], stream_t* s, double de[3]) {
  double cost = sample_sauter(e, s);
  double phi = TWOPI * next_u(s);
  rotate(d, cost, phi, de);
}

/* [reading] pair production without positron transport (Sec. II.A): two
 * electrons share e - 2 mc^2 uniformly, each at its own (1 - beta cos)^-2
 * angle, at opposite azimuths. */
static void pair_event(double e, const double d[3], stream_t* s, double* t1, double d1[3], double* t2,
                       double d2[3]) {
  double avail = e - 2.0 * MC2;
  *t1 = next_u(s) * avail;
  *t2 = avail - *t1;
  double c1 = pair_cos(*t1, next_u(s));
  double c2 = pair_cos(*t2, next_u(s));
  double phi = TWOPI * next_u(s);
  rotate(d, c1, phi, d1);
  rotate(d, c2, phi + PI, d2);
}

/* Moller (Sec. II.B.1): binary collision of an electron of kinetic energy t
 * with a free electron at rest; the delta ray (w, dd) and the primary
 * (t - w, dp) leave at the two-body angles cos^2 = T'(T + 2 mc^2) /
 * (T (T' + 2 mc^2)) of each outgoing kinetic energy T', at opposite
 * azimuths, so that their momenta add up to the incoming one. */
static void moller_event(double t, const double d[3], double kcut, stream_t* s, double* w, double dd[3],
                         double* tp, double dp[3]) {
  double eps = sample_moller(t, kcut, s);
  *w = eps * t;
  *tp = t - *w;
  double cd = sqrt(*w * (t + 2.0 * MC2) / (t * (*w + 2.0 * MC2)));
  double cpp = sqrt(*tp * (t + 2.0 * MC2) / (t * (*tp + 2.0 * MC2)));
  double phi = TWOPI * next_u(s);
  rotate(d, cd, phi, dd);
  rotate(d, cpp, phi + PI, dp);
}

/* [reading] bremsstrahlung (Sec. II.B.1): photon energy k from the
 * complete-screening spectrum, emitted at the polar angle mc^2 / E (E the
 * electron's total energy) with a uniform azimuth; the electron keeps its
 * direction and loses k. */
static void brems_event(double t, const double d[3], double kc, stream_t* s, double* k, double dg[3]) {
  *k = sample_brems(t, kc, s);
  double phi = TWOPI * next_u(s);
  rotate(d, cos(MC2 / (t + MC2)), phi, dg);
}

int orc_event(int which, double e, double p2, const double d[3], uint64_t seed, int count, double* out) {
  uint32_t key[2]; make_key(seed, 0, key);
  for (int i = 0; i < count; ++i) {
    stream_t s; stream_init(&s, key, (uint32_t)i, 0, 0);
    double* o = out + 8 * (size_t)i;
    double ea = 0.0, eb = 0.0, da[3] = { 0, 0, 0 }, db[3] = { 0, 0, 0 };
    switch (which) {
      case 0: compton_event(e, d, &s, &ea, da, &eb, db); break;
      case 1: ea = e; photo_event(e, d, &s, da); break;
      case 2: if (e <= 2.0 * MC2) return -1; pair_event(e, d, &s, &ea, da, &eb, db); break;
      case 3: if (e <= 2.0 * p2) return -1; moller_event(e, d, p2, &s, &ea, da, &eb, db); break;
      case 4: if (e <= p2) return -1; brems_event(e, d, p2, &s, &ea, da); eb = e - ea; memcpy(db, d, sizeof db); break;
      default: return -1;
    }
    o[0] = ea; o[1] = da[0]; o[2] = da[1]; o[3] = da[2];
    o[4] = eb; o[5] = db[0]; o[6] = db[1]; o[7] = db[2];
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Majorants for the Woodcock scheme (Eq. 3; Sec. II.B.3 for electrons).
 * [reading] mu_hat is piecewise constant per grid bin: 1.001 times the largest
 * rho_max(m) mu_m at either bin edge over the materials present.  Sigma_hat is
 * the running maximum over lower bins of the same construction for the hard
 * electron cross section, so that it bounds the cross section at every energy
 * below the step-start energy (this makes the monotonicity assumption of
 * Sec. II.B.3 unnecessary). */
int orc_grid_size(void) { return NE; }

static double grid_e(int i) { return EMIN * exp((double)i * log(EMAX / EMIN) / (double)(NE - 1)); }

static int ebin(double e) {
  double f = (log(e) - log(EMIN)) * (double)(NE - 1) / log(EMAX / EMIN);
  int i = (int)floor(f);
  if (i < 0) i = 0;
  if (i > NE - 2) i = NE - 2;
  return i;
}

static void resolve_cuts(const orc_physics* p, double* kcut, double* kc) {
  *kcut = p->kcut > 0 ? p->kcut : p->ecut;
  *kc = p->kc > 0 ? p->kc : p->pcut;
}

static int build_majorants(const mat_t* mats, int n_mat, const orc_phantom* ph, double kcut, double kc,
                           double* mu_hat, double* sig_hat) {
  double* rmax = (double*)calloc((size_t)n_mat, sizeof(double));
  if (!rmax) return -2;
  size_t nv = (size_t)ph->nx * ph->ny * ph->nz;
  for (size_t v = 0; v < nv; ++v) {
    int m = ph->mat[v];
    if (ph->rho[v] > rmax[m]) rmax[m] = ph->rho[v];
  }
  double run = 0.0;
  for (int i = 0; i < NE - 1; ++i) {
    double ea = grid_e(i), eb = grid_e(i + 1);
    double mu = 0.0, sg = 0.0;
    for (int m = 0; m < n_mat; ++m) {
      if (!(rmax[m] > 0.0)) continue;
      double a = rmax[m] * mu_total(&mats[m], ea), b = rmax[m] * mu_total(&mats[m], eb);
      if (a > mu) mu = a;
      if (b > mu) mu = b;
      double c = rmax[m] * (sig_moller(&mats[m], ea, kcut) + sig_brems(&mats[m], ea, kc));
      double d = rmax[m] * (sig_moller(&mats[m], eb, kcut) + sig_brems(&mats[m], eb, kc));
      if (c > sg) sg = c;
      if (d > sg) sg = d;
    }
    if (sg > run) run = sg;
    mu_hat[i] = MAJ_MARGIN * mu;
    sig_hat[i] = MAJ_MARGIN * run;
  }
  mu_hat[NE - 1] = mu_hat[NE - 2];
  sig_hat[NE - 1] = sig_hat[NE - 2];
  free(rmax);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Transport.                                                          */
typedef struct { double s, c; } ksum_t;   /* Neumaier compensated sum */
static void kadd(ksum_t* k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x; else k->c += (x - t) + k->s;
  k->s = t;
}
static double kval(const ksum_t* k) { return k->s + k->c; }

typedef struct {
  double x[3], d[3], e;
  uint64_t path;
  uint32_t n;
  int type;          /* 0 photon, 1 electron */
} part_t;

typedef struct {
  const orc_phantom* ph;
  mat_t* mats;
  double ecut, pcut, kcut, kc, esmax;
  int mode;
  double mu_hat[NE], sig_hat[NE];
  double lx, ly, lz, skin;
  uint32_t key[2];
  uint32_t hist;
  double* tmp;
  size_t* touched; size_t n_touched, cap_touched;
  part_t* stack; size_t sp, cap;
  ksum_t e_in, e_dep, e_esc, e_sink;
  orc_stats st;
  /* first-event recording */
  int record_first;
  double first_xyz[3];
  uint32_t first_n;
  int first_hit;
  /* path-limited electron tracks (test modes 3 and 4) */
  double path_left;
  int track_done;
} ctx_t;

static int inside(const ctx_t* c, const double* x) {
  return x[0] >= 0.0 && x[0] < c->lx && x[1] >= 0.0 && x[1] < c->ly && x[2] >= 0.0 && x[2] < c->lz;
}

/* Voxel containing x: floor(x / dx) per axis; a point on a face belongs to
 * the voxel on its high side. */
static size_t voxel_of(const ctx_t* c, const double* x, int* ix, int* iy, int* iz) {
  const orc_phantom* p = c->ph;
  int i = (int)floor(x[0] / p->dx), j = (int)floor(x[1] / p->dy), k = (int)floor(x[2] / p->dz);
  if (i < 0) i = 0;
  if (i >= p->nx) i = p->nx - 1;
  if (j < 0) j = 0;
  if (j >= p->ny) j = p->ny - 1;
  if (k < 0) k = 0;
  if (k >= p->nz) k = p->nz - 1;
  if (ix) { *ix = i; *iy = j; *iz = k; }
  return ((size_t)k * p->ny + j) * p->nx + i;
}

/* [reading] Voxel of an electron: each coordinate is first advanced by a skin
 * of 1e-4 voxel widths in the direction of travel, so a point that a hinge
 * leaves a hair short of a face it is moving towards already belongs to the
 * voxel beyond it.  Forward-peaked deflections pile such shortfalls up near
 * zero; without the skin the step count would depend on how finely the
 * arithmetic resolves them.  Returns 0 when the advanced point is outside the
 * phantom (the electron escapes). */
static int electron_voxel(const ctx_t* c, const double* x, const double* d, int* ix, int* iy, int* iz, size_t* v) {
  const orc_phantom* p = c->ph;
  double ext[3] = { c->lx, c->ly, c->lz };
  double del[3] = { p->dx, p->dy, p->dz };
  int n[3] = { p->nx, p->ny, p->nz };
  int idx[3];
  for (int a = 0; a < 3; ++a) {
    double q = x[a] + (d[a] > 0.0 ? c->skin : (d[a] < 0.0 ? -c->skin : 0.0));
    if (!(q >= 0.0 && q < ext[a])) return 0;
    int i = (int)floor(q / del[a]);
    if (i < 0) i = 0;
    if (i >= n[a]) i = n[a] - 1;
    idx[a] = i;
  }
  *ix = idx[0]; *iy = idx[1]; *iz = idx[2];
  *v = ((size_t)idx[2] * p->ny + idx[1]) * p->nx + idx[0];
  return 1;
}

/* d_vox of Eq. 4: distance along d to the boundary of voxel (i, j, k). */
static double dist_boundary(const ctx_t* c, const double* x, const double* d, int i, int j, int k) {
  const orc_phantom* p = c->ph;
  double t = INFINITY;
  int idx[3] = { i, j, k };
  double del[3] = { p->dx, p->dy, p->dz };
  for (int a = 0; a < 3; ++a) {
    double ta;
    if (d[a] > 0.0) ta = ((idx[a] + 1) * del[a] - x[a]) / d[a];
    else if (d[a] < 0.0) ta = (idx[a] * del[a] - x[a]) / d[a];
    else continue;
    if (ta < t) t = ta;
  }
  return t < 0.0 ? 0.0 : t;
}

static void deposit(ctx_t* c, size_t v, double e) {
  if (!(e > 0.0)) return;
  if (c->tmp[v] == 0.0) {
    if (c->n_touched == c->cap_touched) {
      c->cap_touched = c->cap_touched ? 2 * c->cap_touched : 1024;
      c->touched = (size_t*)realloc(c->touched, c->cap_touched * sizeof(size_t));
    }
    c->touched[c->n_touched++] = v;
  }
  c->tmp[v] += e;
  kadd(&c->e_dep, e);
}

static void escape(ctx_t* c, double e) { kadd(&c->e_esc, e); }

/* Push a particle whose state is p, located in voxel v; below its cutoff it
 * deposits locally instead (Sec. II.A: P_cut; Sec. II.B: electron cutoff).
 * Returns 1 if the particle was pushed. */
static int push_particle(ctx_t* c, const part_t* p, size_t v) {
  double cut = p->type == 0 ? c->pcut : c->ecut;
  if (p->e < cut) { deposit(c, v, p->e); return 0; }
  if (c->sp == c->cap) {
    c->cap = c->cap ? 2 * c->cap : 256;
    c->stack = (part_t*)realloc(c->stack, c->cap * sizeof(part_t));
  }
  c->stack[c->sp++] = *p;
  return 1;
}

/* A secondary created at x in voxel v starts its own stream at word 0. */
static void spawn(ctx_t* c, int type, const double* x, const double* d, double e, uint64_t path, size_t v) {
  part_t p;
  memcpy(p.x, x, sizeof p.x);
  memcpy(p.d, d, sizeof p.d);
  p.e = e; p.path = path; p.n = 0; p.type = type;
  if (push_particle(c, &p, v)) c->st.n_secondaries++;
}

static void move(part_t* p, double s) {
  p->x[0] += s * p->d[0]; p->x[1] += s * p->d[1]; p->x[2] += s * p->d[2];
}

/* Analogue photon transport with Woodcock tracking (Sec. II.A, Eqs. 1-3).
 * Per event: free path with mu_hat, then one uniform r against the
 * cumulative (Compton, photoelectric, pair) partials, fictitious otherwise. */
static void photon_run(ctx_t* c, part_t* p) {
  stream_t s; stream_init(&s, c->key, c->hist, p->path, p->n);
  for (;;) {
    stream_align(&s);
    double e = p->e;
    double muh = c->mu_hat[ebin(e)];
    if (!(muh > 0.0)) { escape(c, e); return; }
    double dist = -log(next_u(&s)) / muh;
    move(p, dist);
    c->st.n_photon_events++;
    if (!inside(c, p->x)) { escape(c, e); return; }
    size_t v = voxel_of(c, p->x, 0, 0, 0);
    double rho = c->ph->rho[v];
    const mat_t* m = &c->mats[c->ph->mat[v]];
    double mc = rho * mu_compton(m, e), mp = rho * mu_photo(m, e), mq = rho * mu_pair(m, e);
    double mt = mc + mp + mq;
    if (mt > muh) c->st.n_majorant_violations++;
    double r = next_u(&s) * muh;
    if (r >= mt) { c->st.n_fictitious++; continue; }
    if (c->record_first) {
      memcpy(c->first_xyz, p->x, sizeof p->x);
      c->first_n = s.n; c->first_hit = 1;
      return;
    }
    if (c->mode == 1) { deposit(c, v, e); return; }
    if (r < mc) {
      /* Compton: scattered photon and a recoil electron. */
      double e1, t, d1[3], dt[3];
      compton_event(e, p->d, &s, &e1, d1, &t, dt);
      if (t >= c->ecut) spawn(c, 1, p->x, dt, t, orc_child_path(p->path, s.n, 0), v);
      else deposit(c, v, t);
      memcpy(p->d, d1, sizeof d1);
      p->e = e1;
      if (e1 < c->pcut) { deposit(c, v, e1); return; }
    } else if (r < mc + mp) {
      /* Photoelectric: one electron with the full photon energy. */
      double de[3];
      photo_event(e, p->d, &s, de);
      spawn(c, 1, p->x, de, e, orc_child_path(p->path, s.n, 0), v);
      return;
    } else {
      /* Pair: two electrons; the rest energy 2 mc^2 leaves the ledger as a
       * sink (no positrons). */
      double t1, t2, d1[3], d2[3];
      pair_event(e, p->d, &s, &t1, d1, &t2, d2);
      double avail = e - 2.0 * MC2;
      kadd(&c->e_sink, e - avail);
      spawn(c, 1, p->x, d1, t1, orc_child_path(p->path, s.n, 0), v);
      spawn(c, 1, p->x, d2, t2, orc_child_path(p->path, s.n, 1), v);
      return;
    }
  }
}

/* Class II condensed-history electron transport (Sec. II.B.3):
 * e_s = min{d_vox, e_s-max, e_hard} (Eq. 4); e_hard from the majorant
 * Sigma_hat at the step-start energy; energy loss of Eq. 8 (read with the
 * factor s); random hinge at zeta e_s where the multiple-scattering
 * deflection is applied, with the deflection energy taken before or after the
 * loss at random (a fair coin from the hinge word's lowest bit, so a step
 * without a hard event uses one 4-word block); the loss is deposited in the
 * step-start voxel; after the
 * second leg (1 - zeta) e_s a hard-event candidate is accepted with
 * Sigma(end)/Sigma_hat and split into Moller or bremsstrahlung. */
static void electron_run(ctx_t* c, part_t* p) {
  stream_t s; stream_init(&s, c->key, c->hist, p->path, p->n);
  /* test modes: 2 straight-ahead CSDA (no hard events, no deflection);
   * 3 CSDA loss and deflection without hard events; 4 deflection only */
  const int no_hard = c->mode >= 2, no_ms = c->mode == 2, no_loss = c->mode == 4;
  for (;;) {
    stream_align(&s);
    double t = p->e;
    int ix, iy, iz;
    size_t v0;
    if (!electron_voxel(c, p->x, p->d, &ix, &iy, &iz, &v0)) { escape(c, t); return; }
    if (t < c->ecut) { deposit(c, v0, t); return; }
    double rho0 = c->ph->rho[v0];
    const mat_t* m0 = &c->mats[c->ph->mat[v0]];
    c->st.n_e_steps++;
    double sh = c->sig_hat[ebin(t)];
    double uh = next_u(&s);
    double ehard = (no_hard || !(sh > 0.0)) ? INFINITY : -log(uh) / sh;
    double dv = dist_boundary(c, p->x, p->d, ix, iy, iz);
    if (dv < c->skin) dv = c->skin;
    double emax = (c->esmax > 0.0 && rho0 > 0.0) ? c->esmax / rho0 : INFINITY;
    double es = dv;
    int hard = 0;
    if (emax < es) es = emax;
    if (ehard < es) { es = ehard; hard = 1; }
    if (c->path_left < es) es = c->path_left;   /* a path-limited test track (never hard: modes 3, 4) */
    double l0 = rho0 * l_total(m0, t, c->kcut, c->kc);
    double tm = t - 0.5 * es * l0;
    if (tm < EMIN) tm = EMIN;
    double de = no_loss ? 0.0 : es * rho0 * l_total(m0, tm, c->kcut, c->kc);
    /* one word gives the hinge fraction (its top 24 bits) and the fair coin of
     * the deflection energy (its lowest bit, which the uniform does not use) */
    uint32_t wz = stream_word(&s);
    double zeta = word_to_u(wz);
    move(p, zeta * es);
    double t1 = t - de;
    if (t1 < c->ecut) { deposit(c, v0, t); return; }
    double tms = (wz & 1u) ? t1 : t;
    double ua = next_u(&s), uphi = next_u(&s);
    if (!no_ms) {
      /* Sec. II.B.2: the first moment of the deflection over the step,
       * G1 = 1 - exp(-e_s / lambda_1), lambda_1 at the chosen energy */
      double g1 = -expm1(-es * rho0 * inv_lambda1(m0, tms));
      double cost = wentzel_cos(g1, ua);
      double nd[3]; rotate(p->d, cost, TWOPI * uphi, nd);
      memcpy(p->d, nd, sizeof nd);
    }
    deposit(c, v0, de);
    p->e = t1;
    move(p, (1.0 - zeta) * es);
    if (c->path_left < INFINITY) {
      c->path_left -= es;
      if (c->path_left <= 1e-12 * es) {
        c->track_done = 1;
        return;
      }
    }
    int jx, jy, jz;
    size_t v1;
    if (!electron_voxel(c, p->x, p->d, &jx, &jy, &jz, &v1)) { escape(c, t1); return; }
    if (!hard) continue;
    double ur = next_u(&s);
    double rho1 = c->ph->rho[v1];
    const mat_t* m1 = &c->mats[c->ph->mat[v1]];
    double sm = rho1 * sig_moller(m1, t1, c->kcut);
    double sb = rho1 * sig_brems(m1, t1, c->kc);
    if (sm + sb > sh) c->st.n_majorant_violations++;
    double r = ur * sh;
    if (r < sm) {
      c->st.n_hard++;
      double w, tp, dd[3], dp[3];
      moller_event(t1, p->d, c->kcut, &s, &w, dd, &tp, dp);
      spawn(c, 1, p->x, dd, w, orc_child_path(p->path, s.n, 0), v1);
      memcpy(p->d, dp, sizeof dp);
      p->e = tp;
      if (tp < c->ecut) { deposit(c, v1, tp); return; }
    } else if (r < sm + sb) {
      c->st.n_hard++;
      double k, dg[3];
      brems_event(t1, p->d, c->kc, &s, &k, dg);
      spawn(c, 0, p->x, dg, k, orc_child_path(p->path, s.n, 0), v1);
      p->e = t1 - k;
      if (p->e < c->ecut) { deposit(c, v1, p->e); return; }
    }
  }
}

static int ctx_setup(ctx_t* c, const orc_material* mats, int n_mat, const orc_phantom* ph,
                     const orc_physics* phys, uint64_t seed, uint32_t beam) {
  memset(c, 0, sizeof *c);
  if (!mats || n_mat <= 0 || n_mat > 255 || !ph || !phys) return -1;
  if (ph->nx <= 0 || ph->ny <= 0 || ph->nz <= 0 || !(ph->dx > 0) || !(ph->dy > 0) || !(ph->dz > 0)) return -1;
  if (!(phys->ecut > 0) || !(phys->pcut > 0)) return -1;
  size_t nv = (size_t)ph->nx * ph->ny * ph->nz;
  for (size_t v = 0; v < nv; ++v)
    if (ph->mat[v] >= n_mat || !(ph->rho[v] >= 0.0f)) return -1;
  c->ph = ph;
  c->mats = (mat_t*)malloc((size_t)n_mat * sizeof(mat_t));
  for (int m = 0; m < n_mat; ++m) mat_init(&c->mats[m], &mats[m]);
  c->ecut = phys->ecut; c->pcut = phys->pcut;
  resolve_cuts(phys, &c->kcut, &c->kc);
  c->esmax = phys->esmax_gcm2;
  c->mode = phys->test_mode;
  c->lx = ph->nx * ph->dx; c->ly = ph->ny * ph->dy; c->lz = ph->nz * ph->dz;
  double dmin = ph->dx < ph->dy ? ph->dx : ph->dy;
  if (ph->dz < dmin) dmin = ph->dz;
  c->skin = g_skin_fraction * dmin;
  c->path_left = INFINITY;
  make_key(seed, beam, c->key);
  if (build_majorants(c->mats, n_mat, ph, c->kcut, c->kc, c->mu_hat, c->sig_hat)) return -2;
  c->tmp = (double*)calloc(nv, sizeof(double));
  return c->tmp ? 0 : -2;
}

static void ctx_free(ctx_t* c) {
  free(c->mats); free(c->tmp); free(c->touched); free(c->stack);
}

/* Tabulated spectrum: a histogram (weight w_j spread evenly over
 * [e_j, e_j+1)), sampled by inverting its piecewise-linear CDF with one
 * uniform.  C_j = (w_0 + ... + w_j-1) / W, summed left to right, C_n = 1;
 * u falls in the bin with C_j <= u < C_j+1. */
static double sample_tabulated(const orc_source* src, double u) {
  const int n = src->tab_n;
  double total = 0.0;
  for (int j = 0; j < n; ++j) total += src->tab_w[j];
  double s = 0.0;   /* w_0 + ... + w_j-1 */
  for (int j = 0; j < n; ++j) {
    const double c0 = s / total;
    s += src->tab_w[j];
    const double c1 = (j == n - 1) ? 1.0 : s / total;
    if (u < c1 && c1 > c0)
      return src->tab_e[j] + (u - c0) / (c1 - c0) * (src->tab_e[j + 1] - src->tab_e[j]);
  }
  return src->tab_e[n];
}

/* Source (Sec. II.C.2, initParticle): a parallel beam along +z entering at
 * z = 0, position uniform over the field rectangle, energy monoenergetic,
 * triangular (inverse CDF) or tabulated.  Consumes the first block (four
 * words) of the history's root stream; transport continues from word 4. */
static void sample_source(const orc_source* src, const uint32_t key[2], uint32_t hist, part_t* p) {
  stream_t s; stream_init(&s, key, hist, 0, 0);
  double u0 = next_u(&s), u1 = next_u(&s), u2 = next_u(&s);
  (void)next_u(&s);
  p->x[0] = src->cx + (u0 - 0.5) * src->wx;
  p->x[1] = src->cy + (u1 - 0.5) * src->wy;
  p->x[2] = 0.0;
  p->d[0] = 0.0; p->d[1] = 0.0; p->d[2] = 1.0;
  double e = src->e;
  if (src->spectrum == 1) {
    double a = src->e_lo, m = src->e_mode, b = src->e_hi;
    double fc = (m - a) / (b - a);
    e = (u2 < fc) ? a + sqrt(u2 * (b - a) * (m - a)) : b - sqrt((1.0 - u2) * (b - a) * (b - m));
  } else if (src->spectrum == 2) {
    e = sample_tabulated(src, u2);
  }
  p->e = e;
  p->path = 0;
  p->n = 4;
  p->type = src->particle == 0 ? 0 : 1;
}

static int check_source(const orc_source* src) {
  if (!src || (src->particle != 0 && src->particle != 1)) return -1;
  if (src->spectrum == 0) return (src->e > 0 && src->e <= 30.0) ? 0 : -1;
  if (src->spectrum == 1)
    return (src->e_lo > 0 && src->e_lo <= src->e_mode && src->e_mode <= src->e_hi &&
            src->e_lo < src->e_hi && src->e_hi <= 30.0) ? 0 : -1;
  if (src->spectrum == 2) {
    if (!src->tab_e || !src->tab_w || src->tab_n < 1 || src->tab_n > 4096) return -1;
    if (!(src->tab_e[0] > 0.0 && src->tab_e[src->tab_n] <= 30.0)) return -1;
    double total = 0.0;
    for (int j = 0; j < src->tab_n; ++j) {
      if (!(src->tab_e[j + 1] > src->tab_e[j]) || !(src->tab_w[j] >= 0.0) || !isfinite(src->tab_w[j])) return -1;
      total += src->tab_w[j];
    }
    return (total > 0.0 && isfinite(total)) ? 0 : -1;
  }
  return -1;
}

int orc_sample_source(const orc_source* src, uint64_t seed, uint64_t h_begin, uint64_t h_end, double* out) {
  if (check_source(src)) return -1;
  uint32_t key[2]; make_key(seed, src->beam_id, key);
  for (uint64_t h = h_begin; h < h_end; ++h) {
    part_t p;
    sample_source(src, key, (uint32_t)h, &p);
    double* o = out + 3 * (h - h_begin);
    o[0] = p.x[0]; o[1] = p.x[1]; o[2] = p.e;
  }
  return 0;
}

int orc_run(const orc_material* mats, int n_mat, const orc_phantom* ph,
            const orc_source* src, const orc_physics* phys, uint64_t seed,
            uint64_t h_begin, uint64_t h_end, uint64_t n_total,
            double* e1, double* e2, double* eb, orc_stats* st) {
  if (check_source(src)) return -1;
  if (h_end < h_begin || h_end > n_total || n_total > 0xFFFFFFFFull) return -1;
  /* mode 4 (deflection without energy loss) only ends an electron at the
   * phantom's surface; it serves path-limited tracks alone */
  if (!phys || phys->test_mode < 0 || phys->test_mode > 3) return -1;
  int nb = phys->n_batches > 0 ? phys->n_batches : 1;
  ctx_t c;
  int rc = ctx_setup(&c, mats, n_mat, ph, phys, seed, src->beam_id);
  if (rc) { ctx_free(&c); return rc; }
  size_t nv = (size_t)ph->nx * ph->ny * ph->nz;
  for (uint64_t h = h_begin; h < h_end; ++h) {
    c.hist = (uint32_t)h;
    part_t p;
    sample_source(src, c.key, c.hist, &p);
    kadd(&c.e_in, p.e);
    c.st.n_hist++;
    if (!inside(&c, p.x)) escape(&c, p.e);
    else push_particle(&c, &p, voxel_of(&c, p.x, 0, 0, 0));
    while (c.sp) {
      part_t q = c.stack[--c.sp];
      if (q.type == 0) photon_run(&c, &q); else electron_run(&c, &q);
    }
    /* History-by-history tallies for Eq. 13 and batch sums; history h
     * belongs to batch h mod K (batches interleaved over the histories). */
    size_t k = (size_t)(h % (uint64_t)nb);
    for (size_t i = 0; i < c.n_touched; ++i) {
      size_t w = c.touched[i];
      double t = c.tmp[w];
      e1[w] += t;
      if (e2) e2[w] += t * t;
      if (eb) eb[k * nv + w] += t;
      c.tmp[w] = 0.0;
    }
    c.n_touched = 0;
  }
  if (st) {
    st->e_in += kval(&c.e_in); st->e_dep += kval(&c.e_dep);
    st->e_esc += kval(&c.e_esc); st->e_sink += kval(&c.e_sink);
    st->n_hist += c.st.n_hist; st->n_photon_events += c.st.n_photon_events;
    st->n_fictitious += c.st.n_fictitious; st->n_e_steps += c.st.n_e_steps;
    st->n_hard += c.st.n_hard; st->n_secondaries += c.st.n_secondaries;
    st->n_majorant_violations += c.st.n_majorant_violations;
  }
  ctx_free(&c);
  return 0;
}

int orc_first_events(const orc_material* mats, int n_mat, const orc_phantom* ph,
                     const orc_source* src, const orc_physics* phys, uint64_t seed,
                     uint64_t h_begin, uint64_t h_end, double* xyz, uint32_t* n_used) {
  if (check_source(src) || src->particle != 0) return -1;
  ctx_t c;
  int rc = ctx_setup(&c, mats, n_mat, ph, phys, seed, src->beam_id);
  if (rc) { ctx_free(&c); return rc; }
  c.record_first = 1;
  for (uint64_t h = h_begin; h < h_end; ++h) {
    size_t i = (size_t)(h - h_begin);
    c.hist = (uint32_t)h;
    part_t p;
    sample_source(src, c.key, c.hist, &p);
    c.first_hit = 0; c.first_n = 0;
    if (inside(&c, p.x) && p.e >= c.pcut) photon_run(&c, &p);
    if (c.first_hit) {
      xyz[3 * i] = c.first_xyz[0]; xyz[3 * i + 1] = c.first_xyz[1]; xyz[3 * i + 2] = c.first_xyz[2];
    } else {
      xyz[3 * i] = xyz[3 * i + 1] = xyz[3 * i + 2] = NAN;
    }
    n_used[i] = c.first_n;
    c.n_touched = 0;
  }
  ctx_free(&c);
  return 0;
}

int orc_majorants(const orc_material* mats, int n_mat, const orc_phantom* ph,
                  const orc_physics* phys, double* mu_hat, double* sigma_hat) {
  if (!mats || n_mat <= 0 || !ph || !phys) return -1;
  mat_t* m = (mat_t*)malloc((size_t)n_mat * sizeof(mat_t));
  for (int i = 0; i < n_mat; ++i) mat_init(&m[i], &mats[i]);
  double kcut, kc; resolve_cuts(phys, &kcut, &kc);
  int rc = build_majorants(m, n_mat, ph, kcut, kc, mu_hat, sigma_hat);
  free(m);
  return rc;
}

int orc_electron_tracks(const orc_material* mats, int n_mat, const orc_phantom* ph,
                        const orc_source* src, const orc_physics* phys, uint64_t seed,
                        uint64_t h_begin, uint64_t h_end, double path_cm, double z_start, double* out) {
  if (check_source(src) || src->particle != 1) return -1;
  if (!phys || (phys->test_mode != 3 && phys->test_mode != 4) || !(path_cm > 0.0)) return -1;
  ctx_t c;
  int rc = ctx_setup(&c, mats, n_mat, ph, phys, seed, src->beam_id);
  if (rc) { ctx_free(&c); return rc; }
  for (uint64_t h = h_begin; h < h_end; ++h) {
    double* o = out + 5 * (h - h_begin);
    c.hist = (uint32_t)h;
    part_t p;
    sample_source(src, c.key, c.hist, &p);
    p.x[2] = z_start;
    c.path_left = path_cm;
    c.track_done = 0;
    if (inside(&c, p.x) && p.e >= c.ecut) electron_run(&c, &p);
    if (c.track_done) {
      o[0] = p.d[0]; o[1] = p.d[1]; o[2] = p.d[2]; o[3] = p.e; o[4] = p.x[2];
    } else {
      o[0] = o[1] = o[2] = o[3] = o[4] = NAN;
    }
    for (size_t i = 0; i < c.n_touched; ++i) c.tmp[c.touched[i]] = 0.0;
    c.n_touched = 0;
  }
  ctx_free(&c);
  return 0;
}
