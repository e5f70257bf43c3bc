/*
 * gmc_oracle.h -- plain FP64 CPU oracle for coupled photon-electron Monte Carlo
 * dose calculation in a voxelized phantom (Hissoiny et al., "GPUMCD: a new
 * GPU-oriented Monte Carlo dose calculation platform", Sec. II).
 *
 * TEST INFRASTRUCTURE.  This library exists to check the HIP transport path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant
 * generator with the HIP library: every formula here is written out again
 * from the paper (and the closed forms it relies on), in double precision,
 * single-threaded, one history at a time, depth first.
 *
 * Units: cm, g/cm^3, MeV.  Arrays are [nz][ny][nx] with x fastest.
 */
#ifndef GMC_ORACLE_H
#define GMC_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Effective-element material: electrons per gram divided by N_A (Z/A),
 * effective atomic number, mean excitation energy in eV. */
typedef struct { double z_over_a, z_eff, i_ev; } orc_material;

typedef struct {
  int nx, ny, nz;
  double dx, dy, dz;
  const float* rho;        /* g/cm^3, nx*ny*nz */
  const uint8_t* mat;      /* material index per voxel */
} orc_phantom;

typedef struct {
  int particle;            /* 0 photon, 1 electron */
  int spectrum;            /* 0 monoenergetic, 1 triangular, 2 tabulated (histogram) */
  double e, e_lo, e_mode, e_hi;
  double cx, cy, wx, wy;   /* field centre and full widths at z = 0, direction +z */
  uint32_t beam_id;        /* enters the RNG key */
  const double* tab_e;     /* tabulated: tab_n + 1 increasing bin edges, MeV */
  const double* tab_w;     /* tabulated: tab_n bin weights (>= 0, not all zero) */
  int tab_n;
} orc_source;

typedef struct {
  double ecut, pcut;       /* kinetic electron / photon transport cutoffs */
  double kcut, kc;         /* Moller and bremsstrahlung thresholds (<=0 -> ecut, pcut) */
  double esmax_gcm2;       /* user step bound in g/cm^2 (<=0 -> none) */
  int n_batches;           /* K for the batch variance estimate */
  int test_mode;           /* 0 full, 1 photon first collision, 2 electron CSDA straight-ahead,
                              3 electron CSDA loss and deflection without hard events,
                              4 electron deflection only (no energy loss, no hard events;
                              path-limited tracks only) */
} orc_physics;

typedef struct {
  double e_in, e_dep, e_esc, e_sink;     /* energy ledger, compensated sums (MeV) */
  uint64_t n_hist, n_photon_events, n_fictitious, n_e_steps, n_hard,
           n_secondaries, n_majorant_violations;
} orc_stats;

/* Counter-based generator (replaces the paper's MWC, Sec. II.C.1). */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint64_t orc_child_path(uint64_t parent_path, uint32_t parent_n, uint32_t child_idx);
void orc_stream_words(uint64_t seed, uint32_t beam, uint32_t hist, uint64_t path,
                      uint32_t n0, int count, uint32_t* words, double* uniforms);

/* Cross sections per unit density (cm^2/g) or stopping powers (MeV cm^2/g).
 * which: 0 mu_C, 1 mu_pe, 2 mu_pair, 3 S_col, 4 Sigma_Moller, 5 Moller hard
 * energy loss, 6 L_col (restricted), 7 Sigma_brems, 8 L_rad (restricted),
 * 9 S_rad, 10 L = L_col + L_rad, 11 1/lambda_1, 12 eta (screening). */
int orc_xs(const orc_material* m, int which, const double* e, int n, double kcut, double kc, double* out);

/* Draw `count` samples from one stream (seed, 0, hist 0, path 0).
 * which: 0 KN epsilon (p1 = k) [out2 = cos theta], 1 Sauter cos theta (p1 = T),
 * 2 pair-electron cos theta (p1 = T), 3 Moller epsilon (p1 = T, p2 = kcut),
 * 4 brems photon energy (p1 = T, p2 = kc), 5 Wentzel cos theta (p1 = G1). */
int orc_sample(int which, double p1, double p2, uint64_t seed, int count, double* out, double* out2);
double orc_ms_screening_A(double g1);
void orc_rotate(const double d[3], double cost, double phi, double out[3]);

/* Majorants on the shared log-energy grid: photon mu_hat and electron
 * Sigma_hat (cm^-1) for the materials present in the phantom. */
int orc_grid_size(void);
int orc_majorants(const orc_material* mats, int n_mat, const orc_phantom* ph,
                  const orc_physics* phys, double* mu_hat, double* sigma_hat);

/* Run histories [h_begin, h_end) of a beam of n_total histories.
 * e1[v] += sum_h E_vh, e2[v] += sum_h E_vh^2 (history by history, Eq. 13),
 * eb[k*nvox + v] += batch sums, history h in batch k = h mod K (nullable).
 * Accumulates into the outputs.
 * Returns 0, or a negative code for invalid input. */
int orc_run(const orc_material* mats, int n_mat, const orc_phantom* ph,
            const orc_source* src, const orc_physics* phys, uint64_t seed,
            uint64_t h_begin, uint64_t h_end, uint64_t n_total,
            double* e1, double* e2, double* eb, orc_stats* st);

/* Primaries of histories [h_begin, h_end): x, y and kinetic energy (MeV)
 * into out[3 * i .. 3 * i + 2].  Returns 0, or -1 for an invalid source. */
int orc_sample_source(const orc_source* src, uint64_t seed, uint64_t h_begin, uint64_t h_end, double* out);

/* Per-history first real photon interaction (test mode 1 semantics):
 * writes x,y,z of the first real interaction (NaN if escaped) and the
 * number of stream words consumed up to it. */
int orc_first_events(const orc_material* mats, int n_mat, const orc_phantom* ph,
                     const orc_source* src, const orc_physics* phys, uint64_t seed,
                     uint64_t h_begin, uint64_t h_end, double* xyz, uint32_t* n_used);

/* Outgoing particles of one event, `count` samples on the streams
 * (seed, 0, hist i, path 0) of an incoming particle of energy e (MeV) moving
 * along d.  which: 0 Compton (photon, recoil electron), 1 photoelectric
 * (electron), 2 pair (two electrons), 3 Moller (p2 = kcut: delta ray, primary),
 * 4 bremsstrahlung (p2 = kc: photon, electron).  out[8 i .. 8 i + 7] =
 * E_a, d_a, E_b, d_b (unused entries zero).  Returns -1 below the event's
 * threshold or for an unknown kind. */
int orc_event(int which, double e, double p2, const double d[3], uint64_t seed, int count, double* out);

/* Path-limited tracks of the primary electrons of histories [h_begin, h_end)
 * in test mode 3 or 4, started at depth z_start (instead of the phantom's
 * entrance face) along +z: each stops after path_cm of path (its last step
 * shortened to fit).  out[5 i .. 5 i + 4] = final direction, kinetic energy and
 * depth z, or NaN if the electron left the phantom or fell below the cutoff
 * first. */
int orc_electron_tracks(const orc_material* mats, int n_mat, const orc_phantom* ph,
                        const orc_source* src, const orc_physics* phys, uint64_t seed,
                        uint64_t h_begin, uint64_t h_end, double path_cm, double z_start, double* out);

/* The electron voxel skin as a fraction of the smallest voxel width (default
 * 1e-4; values outside (0, 0.5) are ignored).  Process-wide. */
void orc_set_skin_fraction(double f);

#ifdef __cplusplus
}
#endif
#endif
