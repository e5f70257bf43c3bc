/*
 * gpumcd.h -- C ABI of the MI355X (gfx950) coupled photon-electron Monte Carlo
 * dose engine.  The transport follows Hissoiny et al., "GPUMCD: a new
 * GPU-oriented Monte Carlo dose calculation platform": analogue photon
 * transport with Woodcock tracking (Sec. II.A, Eqs. 1-3), class II
 * condensed-history electrons with CSDA loss, random-hinge multiple
 * scattering and hard Moller / bremsstrahlung events (Sec. II.B, Eqs. 4-8),
 * particle arrays per type processed in alternating passes (Sec. II.C.2-3),
 * and the dose / uncertainty estimators of Sec. II.D (Eqs. 11-13).
 *
 * Conventions
 *  - Units: cm, g/cm^3, MeV.  Dose is Gy per history; sigma is the absolute
 *    one-standard-deviation uncertainty of that mean, same unit.
 *  - Volumes are [nz][ny][nx] with x fastest.  Beams enter at z = 0 along +z.
 *  - Every function returns GMC_OK (0) or a negative GMC_E* code; on error
 *    gmc_last_error() describes it.  No exception crosses the ABI.
 *  - A context is not thread safe, except that the served form's server
 *    thread works beside the caller's calls.  Blocking work runs on the
 *    context's HIP stream; gmc_run_* return after their results are complete.
 *  - Inputs are copied: the caller may free them when the call returns.
 *    Outputs go to caller-owned buffers, host or device memory according to
 *    the *_ptr_kind argument.
 *  - Determinism: the same (phantom, tables, source incl. beam_id, n, seed)
 *    gives bit-identical dose and sigma on every run and for every tuning,
 *    because every particle draws from its own counter-based stream and the
 *    tallies are integer sums.
 */
#ifndef GPUMCD_H
#define GPUMCD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GMC_OK = 0,
  GMC_EINVAL = -1,     /* invalid argument: sizes, ids, energies, cutoffs */
  GMC_ENOMEM = -2,     /* device allocation failed */
  GMC_EDEVICE = -3,    /* HIP runtime error */
  GMC_ENOTFOUND = -4,  /* unknown tables / phantom id */
  GMC_EBUSY = -5,
  GMC_EOVERFLOW = -6,  /* an integer tally could overflow, or a queue overflowed */
  GMC_EINTERNAL = -7   /* broken invariant (energy ledger, queue accounting) */
};

enum { GMC_HOST = 0, GMC_DEVICE = 1 };          /* pointer kinds */
enum { GMC_PHOTON = 0, GMC_ELECTRON = 1 };
enum { GMC_MONO = 0, GMC_TRIANGULAR = 1, GMC_TABULATED = 2 };

typedef struct gmc_context gmc_context;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * run on (e.g. torch.cuda.current_stream().cuda_stream) or NULL for a stream
 * owned by the context.  *out receives the context. */
int gmc_create(int device, void* hip_stream, gmc_context** out);
/* Free every device allocation of the context.  NULL is accepted. */
void gmc_destroy(gmc_context* ctx);
/* Text of the last error on this context; valid until the next call. */
const char* gmc_last_error(const gmc_context* ctx);

/* Effective-element material (Sec. II.A Eq. 2 uses N_A/A; the electron
 * coefficients use Z/A, Z and the mean excitation energy I). */
typedef struct { double z_over_a, z_eff, i_ev; } gmc_material;

/* Physics settings.  Cutoffs are kinetic energies (MeV): electrons below
 * ecut_mev and photons below pcut_mev deposit locally (P_cut of Sec. II.A).
 * kcut_mev (Moller, K_cut of Eq. 6) and kc_mev (bremsstrahlung) default to
 * ecut and pcut when <= 0.  esmax_gcm2 is the user step bound e_s-max of
 * Eq. 4 in g/cm^2 (<= 0: none).  n_batches is K of the batch uncertainty
 * estimate (default 32 when <= 0).  test_mode: 0 full transport; 1 photons
 * deposit their energy at their first real interaction; 2 electrons move in
 * straight lines with CSDA loss only (no hard events, no deflection).
 * majorant_margin scales the Woodcock majorants of Eq. 3 (photons) and of
 * the hard-event distance (electrons, Sec. II.B.3) over the largest
 * attenuation they bound (<= 0: 1.001; accepted in [0.01, 100]).  Below 1 the
 * majorant undercuts the real coefficient somewhere: the transport still runs
 * and every such event is counted in n_majorant_violations (the dose is then
 * biased; values below 1 exist to exercise that count). */
typedef struct {
  double ecut_mev, pcut_mev, kcut_mev, kc_mev, esmax_gcm2;
  int n_batches;
  int test_mode;
  double majorant_margin;
} gmc_physics;

/* Build the FP32 log-energy tables (cross sections, restricted stopping
 * power, transport mean free path, screening inversion) for `n_mat`
 * materials (1..8) in double precision and upload them.  *tables_id
 * receives a handle. */
int gmc_load_tables(gmc_context* ctx, const gmc_material* mats, int n_mat, const gmc_physics* phys,
                    int32_t* tables_id);

/* Upload a voxel phantom: densities (g/cm^3, >= 0, finite) and material
 * indices (< n_mat of the tables used with it), both nx*ny*nz, x fastest,
 * in host or device memory per ptr_kind (Sec. II.C.2: composition and
 * density arrays).  *phantom_id receives a handle. */
int gmc_load_phantom(gmc_context* ctx, int nx, int ny, int nz, double dx_cm, double dy_cm, double dz_cm,
                     const float* density_gcc, const uint8_t* material_id, int ptr_kind, int32_t* phantom_id);

/* Release a tables or phantom handle. */
int gmc_release(gmc_context* ctx, int32_t id);

/* Parallel beam along +z entering at z = 0 (Sec. II.C.2, initParticle):
 * position uniform over the field of full widths (wx, wy) centred at
 * (cx, cy); energy monoenergetic (e_mev), triangular on [e_lo, e_hi] with
 * mode e_mode (inverse CDF), or tabulated: a histogram of tab_n bins (1..4096)
 * with increasing edges tab_e[0..tab_n] in (0, 30] MeV and weights
 * tab_w[0..tab_n-1] (>= 0, finite, not all zero), each bin's weight spread
 * evenly over the bin, sampled by inverting the piecewise-linear CDF.  The
 * tables are host memory, read during the call (copied by gmc_submit); they
 * are ignored by the other spectra.  beam_id enters the random stream key, so
 * beamlets with different ids draw independent streams.
 * first_history numbers the beam's histories: a run of n histories
 * transports histories first_history .. first_history + n - 1, drawing their
 * random streams and falling into their batches (history h in batch
 * h mod n_batches) exactly as those histories of one larger run do
 * (first_history + n must stay below 2^32).  Shards of a beam run with
 * consecutive ranges -- on one GPU after another or on several GPUs -- thus
 * produce integer tallies whose sum is bit for bit the tally of the whole
 * run (gmc_run_beam_tally, gmc_finalize_tally).  0 for an ordinary run;
 * gmc_first_events takes explicit history numbers and ignores it. */
typedef struct {
  int particle;
  int spectrum;
  double e_mev, e_lo, e_mode, e_hi;
  double cx_cm, cy_cm, wx_cm, wy_cm;
  uint32_t beam_id;
  const double* tab_e;
  const double* tab_w;
  int tab_n;
  uint64_t first_history;
} gmc_source;

/* Per-run statistics.  Energies in MeV; the integer ledger residual (in units
 * of 2^-27 MeV) is incident - deposited - escaped - pair rest energy and is
 * zero by construction.  n_passes counts rounds (admission, electron pass,
 * photon pass).  t_photon_pass_s / t_electron_pass_s are the summed
 * durations of the pass kernels, each launch bracketed by a pair of HIP
 * events (event nodes of the graph in the batched form), over
 * n_photon_launches / n_electron_launches launches. */
typedef struct {
  double t_total_s, t_device_s;
  double e_in_mev, e_dep_mev, e_esc_mev, e_sink_mev;
  uint64_t n_hist, n_photon_events, n_fictitious, n_e_steps, n_hard, n_secondaries,
           n_majorant_violations, n_passes;
  int64_t ledger_residual_lsb;
  double t_photon_pass_s, t_electron_pass_s;
  uint64_t n_photon_launches, n_electron_launches;
  double s_rel;   /* Eq. 12: mean sigma/D over voxels with D > 0.2 D_max of the
                     (combined) dose; NaN when sigma was not requested or
                     nothing was deposited */
  double t_round_s;            /* summed durations of the persistent round kernels */
  uint64_t n_round_launches;   /* (tuning persistent), bracketed like the passes */
  uint64_t n_photon_interactions;   /* photon flights (of n_photon_events) that ended in a real
                                       Compton, photoelectric or pair interaction */
} gmc_run_stats;

/* Optional tuning of the engine.  A field <= 0 selects its default; a NULL
 * tuning selects all defaults in gmc_run_beam and the autotuner's cached
 * choice in gmc_run_beams.
 *   events_per_visit: events a particle may take per kernel visit before it
 *     is requeued (the N of the stream-compaction scheme, Sec. II.C.3;
 *     1..32768, default 64; an electron's events are its steps, a photon's
 *     its interactions, fictitious ones included);
 *   secondaries_per_visit: secondaries a particle may create per visit
 *     (2..64, default 4);
 *   chunk: primaries admitted per admission step while a particle type's
 *     array holds fewer (default 2^22, at most 2^24);
 *   wg_size: threads per workgroup of the pass kernels (64..1024, multiple
 *     of 64; default: per pass kernel, the smallest of 256, 512 and 1024 that
 *     keeps the most wavefronts resident -- each workgroup stages its own
 *     copy of the tables in LDS, so with several materials larger workgroups
 *     keep more wavefronts per compute unit);
 *   pass_items: most particles one pass launch transports (1024..2^23,
 *     default 2^23); the rest is carried to the next pass;
 *   wave_items: particles per chunk when a pass deals its particles to the
 *     wavefronts round-robin (64..1024, rounded down to a power of two;
 *     default 64);
 *   rounds_per_check: batched form only; the captured graph holds
 *     2 x rounds_per_check rounds and the host reads the particle counts
 *     once per replay (1..1024, default 4);
 *   refill_lanes: idle lanes of a wavefront (1..64, default 4) before they
 *     take new particles from the wavefront's range;
 *   energy_sort: > 0 regroups every pass's particles by energy first
 *     (highest first; a counting sort on log-energy buckets into a spare
 *     buffer of pass_items particles), the grouping of similar energies that
 *     Sec. IV.B proposes for polyenergetic beams (default 0: off: on MI355X
 *     the sort costs more than the passes gain);
 *   tail_lanes: once a wavefront has taken every particle of its share of a
 *     pass (and, in the electron pass, no parked electron waits), the
 *     particles still on its lanes are requeued for the next pass after
 *     their next event whenever at most tail_lanes lanes hold one, instead
 *     of the wavefront running on for its last few particles; only while
 *     primaries remain to be admitted (a next pass of each type follows
 *     anyway; the last passes of a job finish in place) and for shares of at
 *     least 256 particles (0: default, 64 in the electron pass and 32 in the
 *     photon pass; 1..64 both passes; -1 off);
 *   queue_items: particles that admission and the other type's outputs may
 *     put in a type's queue (its soft capacity; 64..2^25, default 8 x chunk,
 *     at least 2^23).  A queue too small for the per-visit output budget
 *     leaves neither pass able to move: such a job ends with GMC_EOVERFLOW
 *     ("both particle queues are too full") instead of running forever;
 *   persistent: > 0 runs each round as one persistent kernel instead of an
 *     electron pass and a photon pass: its wavefronts claim chunks of
 *     wave_items particles from a device work queue -- the round's
 *     electrons first, then its photons (the round's new primaries come last
 *     in each queue) -- each workgroup from a partition of the queue with a
 *     counter of its own, then from other partitions once its own is used up,
 *     each wavefront up to a cap (an even share plus one chunk) that bounds
 *     its staging, and no wavefront waits for another; workgroups of at most
 *     512 threads (wg_size is clamped to 512 for it); every
 *     workgroup holds both table blocks in LDS, so jobs with more than four
 *     materials run the passes instead (default 0; energy_sort is ignored
 *     with it);
 *   aggregate: the electron pass sums, at the end of each loop iteration,
 *     the tally additions of the wavefront's lanes that go to one address
 *     and adds the sum with one atomic (1 on, -1 off; 0, the default: on
 *     where every beam's own tally is a single slice -- per-beam doses of a
 *     batched job too large for per-beam batches -- whose pencil beams send
 *     many lanes to one address).
 * No tuning changes any result: the dose is bit-identical for every choice
 * that lets the job finish. */
typedef struct {
  int events_per_visit, secondaries_per_visit, chunk, wg_size;
  int pass_items, wave_items, rounds_per_check, refill_lanes;
  int energy_sort, tail_lanes, queue_items, persistent, aggregate;
} gmc_tuning;

/* Transport n_histories histories of one beam (the plain form: one beam per
 * sequence of alternating electron and photon passes until both particle
 * arrays are empty, Sec. II.C.2) and write the dose per history and its
 * batch uncertainty per voxel (history h in batch h mod n_batches).  seed keys the random streams.  Outputs are
 * nx*ny*nz doubles in host or device memory per out_ptr_kind; sigma and
 * stats may be NULL.  n_histories must be < 2^32 and at least n_batches. */
int gmc_run_beam(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const gmc_source* src,
                 uint64_t n_histories, uint64_t seed, double* dose_gy_per_hist, double* sigma_gy_per_hist,
                 int out_ptr_kind, const gmc_tuning* tuning, gmc_run_stats* stats);

/* The plain form's run of gmc_run_beam, returning the raw integer batch
 * tallies instead of the dose: tally[k * nvox + v] is the energy deposited in
 * voxel v by the histories of batch k (history h of the run, numbered from
 * src->first_history, in batch h mod n_batches), in units of 2^-27 MeV,
 * n_batches * nx*ny*nz uint64 values in host or device memory per
 * out_ptr_kind.  Tallies of runs over disjoint history ranges add up (as
 * integers, in any order) to the tally of one run over their union: the
 * exchange format of a beam sharded across GPUs (Sec. II.C.3's multi-GPU
 * scheme, one reduction of integer sums).  stats as for gmc_run_beam (s_rel
 * NaN). */
int gmc_run_beam_tally(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const gmc_source* src,
                       uint64_t n_histories, uint64_t seed, uint64_t* tally, int out_ptr_kind,
                       const gmc_tuning* tuning, gmc_run_stats* stats);

/* Dose per history and batch uncertainty (Sec. II.D: D = sum_k T_k / N in
 * Gy; sigma^2 = sum_k n_k^2 (m_k - m)^2 / (N^2 (K - 1)/K), Eq. 13 over K
 * batches) of integer batch tallies laid out as gmc_run_beam_tally writes
 * them, covering histories [h_begin, h_end) of a beam (N = h_end - h_begin,
 * at least n_batches; n_k the histories of batch k in that range), on the
 * phantom's voxels.  tally is host or device memory per tally_ptr_kind,
 * dose and sigma (sigma may be NULL) per out_ptr_kind; *s_rel (may be NULL)
 * receives s of Eq. 12 (NaN without sigma).  Equal tallies and ranges give
 * bit-identical results to gmc_run_beam's finalize. */
int gmc_finalize_tally(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const uint64_t* tally,
                       int tally_ptr_kind, uint64_t h_begin, uint64_t h_end, double* dose, double* sigma,
                       int out_ptr_kind, double* s_rel);

/* gmc_finalize_tally for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and results as gmc_finalize_tally with device
 * pointers: tally (n_batches * nx*ny*nz uint64, layout as gmc_run_beam_tally
 * writes it), dose and sigma (nx*ny*nz doubles each; sigma may be NULL) are
 * device memory, s_rel (may be NULL; NaN without sigma) host memory.  Equal
 * tallies and ranges give bit-identical dose, sigma and s to
 * gmc_finalize_tally.  The call allocates nothing: its work memory (the
 * histories per batch and the partial sums of s, at most 1024 batches,
 * 14.3 KB) is one array of the library's device code per GPU, held until
 * the process ends; n_batches above 1024 is refused with GMC_EINVAL.  Every
 * call on a GPU shares that GPU's array, so calls that overlap on one GPU
 * (other threads, other contexts) race and must not be made.  Runs on the
 * context stream and returns when the results are complete. */
int gmc_finalize_tally_noalloc(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const uint64_t* tally,
                               uint64_t h_begin, uint64_t h_end, double* dose, double* sigma, double* s_rel);

/* Grid size of a loaded phantom: the number of doubles every dose and sigma
 * output of a run on it holds is nx*ny*nz. */
int gmc_phantom_dims(gmc_context* ctx, int32_t phantom_id, int* nx, int* ny, int* nz);

/* Transport several beams in one job (the batched form): primaries of every
 * beam are admitted into the shared per-type particle arrays as space frees
 * up, and the rounds of alternating electron and photon passes (Sec. II.C.2)
 * run from a captured HIP graph, the host reading the particle counts once
 * per replay.  srcs[b] and n_hist[b] (b < n_beams, 1 <= n_beams <= 2^20, each
 * n_hist[b] >= 1) describe beam b; beam b draws the same random streams as
 * gmc_run_beam(srcs[b], n_hist[b], seed), so beams with distinct beam_id are
 * independent.  History h of a beam belongs to batch h mod n_batches.
 *   dose_per_beam: NULL, or a host array of n_beams pointers, each NULL or
 *     an nx*ny*nz output of beam b's dose per history of that beam
 *     (bit-identical to gmc_run_beam's dose for the same beam and seed);
 *   sigma_per_beam: NULL, or likewise beam b's batch uncertainty
 *     (bit-identical to gmc_run_beam's sigma); needs at least n_batches
 *     histories in every beam;
 *   combined_dose / combined_sigma: dose per history summed over all beams'
 *     histories (divided by their total) and its batch uncertainty;
 *     combined_dose is required, combined_sigma may be NULL.
 * With per-beam outputs the job keeps n_batches*nx*ny*nz uint64 tallies per
 * beam when they fit in half of the free device memory (batch k of the
 * combined result is then the sum of the beams' batches k); otherwise each
 * beam gets a single nx*ny*nz tally beside a combined one batched over the
 * histories of all beams in order (and sigma_per_beam is refused with
 * GMC_ENOMEM).  The combined dose is the same either way.  Output pointers
 * are host or device memory per out_ptr_kind.  The sum of n_hist must be
 * < 2^32 and at least n_batches.  The work runs on a stream owned by the
 * context, ordered after the context stream's earlier work, and the context
 * stream waits for it before the call returns. */
int gmc_run_beams(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs,
                  const uint64_t* n_hist, int n_beams, uint64_t seed, double* const* dose_per_beam,
                  double* const* sigma_per_beam, double* combined_dose, double* combined_sigma,
                  int out_ptr_kind, const gmc_tuning* tuning, gmc_run_stats* stats);

/* Autotuner of the batched form.  Picks the admission chunk, the pass size,
 * the events per visit, the workgroup size, the particles per wavefront,
 * the refill threshold, the rounds per status check and the persistent
 * round kernel against graph-replayed passes by coordinate
 * descent, starting with the admission chunk and the pass size together
 * (pass = 2 x chunk): each candidate runs the whole job when about 24 such
 * runs fit the budget, else a sample (the first histories of every beam, in
 * proportion: 5% of the job but at least 2^25 histories), and is timed on
 * the device; a change is kept when it saves at least 2%.  Choices are cached in the context per job class (grid size,
 * mean energy, electron fraction, field area, history count and material
 * count on coarse logarithmic scales); a cached class returns at once.
 * gmc_autotune tunes the job with combined outputs only; gmc_run_beams with
 * tuning NULL and per-beam outputs tunes (and caches) the job as it runs
 * it, with per-beam tallies.
 * budget_s bounds the search's wall time (<= 0: 10 s).  gmc_run_beams with
 * tuning NULL calls this first.  *out receives the choice; report may be
 * NULL. */
typedef struct {
  int trials;                 /* sample jobs run */
  int from_cache;             /* 1: the class was tuned before, nothing run */
  int complete;               /* 0: the budget ran out before every knob was tried */
  uint64_t sample_histories;
  double t_default_s;         /* sample's device time with the default tuning */
  double t_best_s;            /* with the chosen tuning */
} gmc_autotune_report;

int gmc_autotune(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs,
                 const uint64_t* n_hist, int n_beams, double budget_s, gmc_tuning* out,
                 gmc_autotune_report* report);

/* ----------------------------------------------------------- served form
 * Continuous batching of dose requests.  gmc_server_start starts a server
 * thread on the context; each request is one beam on a loaded phantom and
 * tables (which stay resident: a request only references them, and they
 * cannot be released while a request holds them).  Requests wait in
 * submission order for one of max_slots slots; a request starts as soon as
 * a slot is free and its device footprint fits beside the other slots'
 * within hbm_budget_bytes, so requests that arrive while others run are
 * admitted at once and their kernels overlap on the device.  Footprint of a
 * request: its slot's particle queues and staging plus n_batches*nx*ny*nz
 * uint64 tallies and the nx*ny*nz dose and sigma.  Each request runs the
 * batched form's engine on one beam with the autotuner's cached choice for
 * its class (defaults when none), so its dose and sigma are bit-identical
 * to gmc_run_beam's for the same phantom, tables, source, histories and
 * seed, whatever else runs beside it.  A finished request's dose and sigma
 * stay in device memory (a pool of result buffers the server reuses) until
 * gmc_poll copies them out -- device to device, or device to host -- in one
 * copy; results waiting to be polled count against hbm_budget_bytes, and
 * when a request could not start otherwise, the oldest of them moves to host
 * memory instead. */
typedef struct {
  size_t hbm_budget_bytes;    /* device memory the slots may hold; 0: 3/4 of the free memory */
  int max_slots;              /* requests on the device at once, 1..16 (0: 4) */
} gmc_server_config;

typedef struct {
  double t_queue_s;           /* submission to start on a slot */
  double t_run_s;             /* start to result ready */
  double t_latency_s;         /* submission to result ready */
  gmc_run_stats run;
} gmc_request_stats;

typedef struct {
  int running, pending, in_flight, finished_unpolled;
  size_t budget_bytes;
} gmc_server_status_t;

/* Start the server (cfg may be NULL).  GMC_EBUSY if one is running. */
int gmc_server_start(gmc_context* ctx, const gmc_server_config* cfg);
/* Queue a request; *ticket identifies it.  n_histories in [n_batches, 2^32).
 * GMC_EBUSY if its footprint can never fit in the budget. */
int gmc_submit(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const gmc_source* src,
               uint64_t n_histories, uint64_t seed, uint64_t* ticket);
/* *done = 1 once the request has finished (waiting for it when wait != 0);
 * then its dose and sigma (nx*ny*nz doubles, either may be NULL) are written
 * to host or device memory per out_ptr_kind, stats (may be NULL) filled, the
 * ticket retired, and the request's own error code returned if it failed. */
int gmc_poll(gmc_context* ctx, uint64_t ticket, int wait, int* done, double* dose, double* sigma,
             int out_ptr_kind, gmc_request_stats* stats);
/* Finish every queued and running request, then stop the thread and free
 * the slots; finished tickets stay pollable (their results move to host
 * memory). */
int gmc_server_stop(gmc_context* ctx);
int gmc_server_status(gmc_context* ctx, gmc_server_status_t* status);

/* ---------------------------------------------------------------- checks */
/* Words n0 .. n0+count-1 of the stream (seed, beam, hist, path), computed
 * on the device; out_words is host memory. */
int gmc_rng_words(gmc_context* ctx, uint64_t seed, uint32_t beam, uint32_t hist, uint64_t path, uint32_t n0,
                  int count, uint32_t* out_words);

/* Evaluate the device-resident tables by their device interpolation at n
 * energies (host arrays).  which: 0 mu_C, 1 mu_C+mu_pe, 2 mu_total (per unit
 * density, cm^2/g), 3 restricted stopping power L, 4 Sigma_Moller,
 * 5 Sigma_brems, 6 1/lambda_1 (cm^2/g or MeV cm^2/g), 7 Wentzel screening A
 * for G1 = energies[i]. */
int gmc_table_eval(gmc_context* ctx, int32_t tables_id, int which, int mat, const double* energies, int n,
                   double* out);

/* Per-history first real photon interaction of histories [h_begin, h_end)
 * of a photon beam, on the device: xyz (3 floats per history, NaN if the
 * photon escaped first) and the number of stream words used up to it. */
int gmc_first_events(gmc_context* ctx, int32_t phantom_id, int32_t tables_id, const gmc_source* src,
                     uint64_t seed, uint32_t h_begin, uint32_t h_end, float* out_xyz, uint32_t* out_nused);

/* Measure the device's 64-bit atomic-add rate, the second roof of the
 * tally path: 2^20 lanes each add 1 to 64 words of an array of
 * 2^log2_words uint64 words (10..31, up to 16 GiB), at hashed addresses (hot = 0) or on
 * word t mod hot of the first hot words (hot a power of two, at most the
 * array's size), with the instruction the tallies use; timed with HIP events
 * after a warm-up launch.  *adds_per_s receives the additions per second.
 * The array is allocated and freed by the call. */
int gmc_atomic_rate(gmc_context* ctx, int log2_words, int hot, double* adds_per_s);

#ifdef __cplusplus
}
#endif
#endif
