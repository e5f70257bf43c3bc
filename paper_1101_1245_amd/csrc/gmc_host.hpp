// gmc_host.hpp -- host-side state of the engine: table and phantom objects,
// the per-run workspace (particle queues, counters, tallies, stream and
// events), the transport engine's interface, and the context behind the
// C ABI.  Shared by gmc_engine.cpp (engine, blocking forms, autotuner),
// gmc_server.cpp (served form) and gmc_runtime.cpp (ABI entry points).
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gmc_internal.hpp"
#include "gmc_tables.hpp"
#include "gpumcd.h"

namespace gmc {

struct TablesObj {
  gmc_physics phys{};
  double kcut = 0, kc = 0;
  double margin = 1.001;         // majorant safety factor
  HostTables host;
  float4* d_ph = nullptr;
  float4* d_el = nullptr;
  float* d_ms = nullptr;
};

struct PhantomObj {
  int nx = 0, ny = 0, nz = 0;
  double dx = 0, dy = 0, dz = 0;
  uint2* d_vox = nullptr;
  std::vector<double> rho_max;   // per material index 0..255
  int max_mat = 0;
  size_t nvox() const { return (size_t)nx * ny * nz; }
};

struct MajObj {
  float* d_g = nullptr;
  float* d_e = nullptr;
};

struct QueueBuf {
  DevQueue q{};
  void* base = nullptr;
};

constexpr uint32_t kMinSoftCap = 1u << 23;
constexpr uint32_t kMaxSoftCap = 1u << 25;
constexpr uint32_t kMaxWaves = 1u << 15;
constexpr int kSortGrid = 2048;              // workgroups of the regrouping kernels
constexpr double kAutotuneBudgetS = 10.0;   // default wall-clock budget of one tuning
constexpr double kTuneTrials = 24.0;        // about how many candidates one tuning runs
constexpr uint64_t kTuneMinSample = 1ull << 25;   // 8 chunks of the largest candidate
// Idle lanes of an electron-pass wavefront, its range done, that take back
// parked electrons together (their hard events then run on that many lanes).
constexpr int kResumeLanes = 32;
// Smallest share of a pass (particles per wavefront) whose tail is requeued.
constexpr uint32_t kTailMinItems = 256u;
// Admission segments of a job with several beams of a type: at least this
// many histories each, at most kMaxAdmitSegments per type.
constexpr uint64_t kAdmitSegment = 4096u;
constexpr uint64_t kMaxAdmitSegments = 1u << 16;

// Device control block of a workspace: queue counts [type][buffer],
// admission cursor and histories per type, the last pass plans and
// admissions.  One copy of it is the host's view of a job's progress.
struct Control {
  uint32_t counts[4];
  uint32_t sched[4];            // cursor[2], total[2]
  PassPlan plan[2];
  AdmitPlan adm[2];
  ClaimType claim[2];           // the round kernel's work queue per type
  bool done() const {
    return sched[0] == sched[2] && sched[1] == sched[3] && counts[0] == 0 && counts[1] == 0 && counts[2] == 0 &&
           counts[3] == 0;
  }
};

// Everything one running job needs on the device, with the stream it runs
// on.  The context has one for the blocking forms; the server has one per
// slot.  Buffers only grow (released by ws_trim or ws_free).
struct Workspace {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  uint32_t cap = 0;              // allocated particles per queue buffer
  uint32_t cap_soft = 0;         // what admission and other-type outputs may fill
  QueueBuf qbuf[2][2];          // [type: 0 photon, 1 electron][2 buffers]
  int acc[2] = {0, 0};          // buffer of each type that accumulates
  QueueBuf stg[2];              // staging: [0] same type, [1] other type
  uint32_t stg_cap = 0;
  QueueBuf sorted;              // a work buffer regrouped by energy (when sorting)
  uint32_t sorted_cap = 0;
  uint32_t* d_sort = nullptr;   // [2][kSortBuckets]: bucket counts, bucket cursors
  Control* d_ctl = nullptr;
  Control* h_ctl = nullptr;     // pinned host copy
  unsigned long long* d_ctr = nullptr;   // [C_COUNT][kCtrSlots]
  unsigned long long* h_ctr = nullptr;   // pinned host copy
  unsigned long long* d_tally = nullptr;
  size_t tally_elems = 0;
  DevBeam* d_beams = nullptr;
  DevSource* d_sources = nullptr;
  double* d_tab = nullptr;      // the job's tabulated spectra
  size_t tab_cap = 0;
  uint32_t* d_start = nullptr;   // [2][seg_cap + 1] admission segments per type: first job-wide index
  uint32_t* d_beam_of = nullptr;   // [2][seg_cap] beam of each segment
  uint32_t* d_seg_h = nullptr;     // [2][seg_cap] index in its beam of the segment's first history
  size_t beams_cap = 0;
  size_t seg_cap = 0;
  uint32_t* d_claim = nullptr;  // [2][kMaxClaimParts] chunk counters of the round kernel's work queue
  double* d_nk = nullptr;
  double* d_srel = nullptr;     // [3 kRelBlocks + 1] work of the s reduction, s last
  double* h_srel = nullptr;     // pinned copy of s
  double* h_nk = nullptr;       // pinned batch sizes for the finalize
  double* d_dose = nullptr;
  double* d_sigma = nullptr;
  size_t out_elems = 0;
  FinalizeArgs* d_fin = nullptr;   // per-beam finalize arguments of a batched job
  double* d_fin_nk = nullptr;      // and their batch sizes
  size_t fin_cap = 0, fin_nk_cap = 0;
  std::map<std::vector<int>, int> resident;    // (kernel, block, materials) -> resident workgroups
  hipEvent_t ev0 = nullptr, ev1 = nullptr;     // around a whole job
  hipEvent_t kev0 = nullptr, kev1 = nullptr;   // around a pass launch (plain form)
  hipEvent_t ev_ctl = nullptr;                 // after a control-block copy
  std::vector<hipEvent_t> gev;                 // pairs around the passes of a captured graph
  double t_pass[3] = {0.0, 0.0, 0.0};          // summed photon pass, electron pass, round kernel durations, s
  uint64_t n_pass[3] = {0, 0, 0};
};

int wfail(Workspace* w, int code, const std::string& msg);

#define WS_TRY(w, expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::gmc::wfail(w, e_ == hipErrorOutOfMemory ? GMC_ENOMEM : GMC_EDEVICE,      \
                          std::string(#expr) + ": " + hipGetErrorString(e_));           \
  } while (0)

// stream null: the workspace creates (and owns) a non-blocking stream.
int ws_init(Workspace* w, int device, hipStream_t stream);
void ws_free(Workspace* w);
// Release the job-sized buffers (tallies, outputs); keep queues and staging.
void ws_trim(Workspace* w);
size_t ws_device_bytes(const Workspace& w);
int ws_ensure_tally(Workspace* w, size_t elems);
int ws_ensure_out(Workspace* w, size_t elems);
int ws_ensure_beams(Workspace* w, size_t n);
int ws_ensure_fin(Workspace* w, size_t n, size_t nk);
// Admission segment tables of n segments per type.
int ws_ensure_segments(Workspace* w, size_t n);

// Engine knobs (gmc_tuning with defaults filled in).
struct Tune {
  int events, secondaries, chunk, block, pass_items, wave_items, rounds, refill;
  int sort;            // 1: energy regrouping before every pass
  int tail_g, tail_e;  // tail requeue lanes of the photon / electron pass (0: off)
  int queue;           // soft queue capacity (0: from the chunk)
  int persistent;      // 1: one persistent round kernel per round
  int aggregate;       // 1 on, -1 off, 0 where every beam's tally a is a single slice
};
Tune resolve_tuning(const gmc_tuning* t);
gmc_tuning default_tuning();

// Queue capacity (allocated and soft) and staging slots the engine uses for a tuning.
void queue_sizes(Workspace* w, const Tune& tu, int n_mat, uint32_t* cap, uint32_t* cap_soft, uint32_t* stg);
// Whether a tuning runs rounds as the persistent kernel for n_mat materials.
bool uses_round(const Tune& tu, int n_mat);

int check_source(std::string* err, const gmc_source* s);
// Highest and mean kinetic energy of a (checked) source's spectrum, MeV.
double source_emax(const gmc_source& s);
double source_emean(const gmc_source& s);
// Edges then the normalised CDF at them (C_0 = 0, C_n = 1) of a tabulated spectrum.
void tabulated_cdf(const gmc_source& s, std::vector<double>* out);
uint32_t mev_to_lsb(double e);
DevPhantom dev_phantom(const PhantomObj& p);
DevCuts dev_cuts(const TablesObj& t);
DevSource dev_source(const gmc_source& s);
DevTables dev_tables(const TablesObj& t, const MajObj& m);

// One transport job: its beams, their sources and tally targets.  Histories
// of each particle type are numbered consecutively over the beams of that
// type (start[t][j] is the first history of the j-th beam of type t).
struct Job {
  const PhantomObj* P = nullptr;
  const TablesObj* T = nullptr;
  MajObj maj;
  std::vector<DevBeam> beams;
  std::vector<DevSource> sources;
  std::vector<double> tab;            // tabulated spectra: per such beam, edges then normalised CDF
  std::vector<size_t> tab_off;        // per beam: offset in tab (tabulated beams only)
  // admission segments per type: segment j covers job-wide indices
  // [start[j], start[j+1]), histories seg_h[j] ... of beam beam_of[j]
  std::vector<uint32_t> start[2], beam_of[2], seg_h[2];
  uint32_t total[2] = {0, 0};
};

// How a job tallies (the plain form and the served form use kCombined with
// one beam).
enum TallyMode {
  kCombined,       // one tally [K][nvox] batched over all histories: no per-beam doses
  kBeamBatched,    // a [K][nvox] tally per beam; the combined result is their sum
  kBeamPlusComb    // a [1][nvox] tally per beam plus a combined [K][nvox] one (two additions per deposit)
};

// Beams, sources and tally targets of a job in workspace w (tallies at
// w->d_tally, laid out per mode).
void build_job(Job* J, Workspace* w, const PhantomObj& P, const TablesObj& T, const MajObj& maj,
               const gmc_source* srcs, const uint64_t* n_hist, int n_beams, uint64_t seed, TallyMode mode);
size_t job_tally_elems(TallyMode mode, size_t nvox, uint32_t K, size_t n_beams);

// Workgroup size of a pass kernel: the requested one, or (requested 0) the
// smallest of 256 / 512 / 1024 threads that keeps the most wavefronts
// resident (with many materials the LDS tables, one copy per workgroup,
// limit 256-thread workgroups to half the occupancy registers allow).
int pass_block(Workspace* w, int kernel, int requested, int n_mat);
// Wavefronts of a pass grid (resident workgroups x waves per workgroup, at
// most kMaxWaves).
uint32_t pass_waves(Workspace* w, int kernel, int block, int n_mat);

struct Engine {
  Workspace* w = nullptr;
  Tune tu{};
  bool round = false;             // rounds as one persistent kernel (tu.persistent and the tables fit)
  int round_block = 0;            // its workgroup size, grid, wavefronts
  uint32_t round_blocks = 0, round_waves = 0;
  int block[2] = {0, 0};          // workgroup size of each pass kernel
  PassArgs proto{};
  AdmitArgs adm[2]{};
  uint32_t total[2] = {0, 0};
  uint32_t waves[2] = {0, 0};     // wavefronts of each pass grid
  uint32_t blocks[2] = {0, 0};
  uint32_t bud_same[2] = {0, 0}, bud_other[2] = {0, 0};
};

// Queues, staging, beam tables and counters of a job (enqueued on w->stream,
// plus small synchronous uploads).
int engine_setup(Workspace* w, Engine& E, const Job& J, const Tune& tu);
// Plain form: run to the end, host reads after admission and electron pass.
int engine_run_plain(Engine& E, uint64_t* rounds);
// Capture 2 * tu.rounds rounds (with event pairs around the passes) on
// w->stream into an executable graph.
int engine_capture(Engine& E, hipGraphExec_t* exec, int* rounds_per_replay);
// Batched form: capture, then replay until done (blocking).
int engine_run_graph(Engine& E, uint64_t* rounds);
// Enqueue a copy of the control block to w->h_ctl and record w->ev_ctl.
int enqueue_control_copy(Workspace* w);
// After a replay's control copy completed: check it and add the pass times;
// *done tells whether the job finished (a job that cannot progress any more
// returns GMC_EOVERFLOW).
int after_replay(Engine& E, int rounds_per_replay, bool* done);

// Histories per batch for interleaved batches: n_k += #{h in [h0, h0 + n) : h mod K = k}.
void add_batch_sizes(std::vector<double>& nk, uint64_t h0, uint64_t n, uint32_t K);
// Gy per tally unit (2^-27 MeV) per unit density of a voxel of P.
double dose_per_lsb(const PhantomObj& P);
// Dose and sigma of `nsum` tallies ([K][nvox] each, `stride` apart, added).
// With sync false the batch sizes go through the pinned w->h_nk and the
// call does not wait (one finalize in flight per workspace).
// `blocked`: the tally is in the library's blocked layout (else slice-major,
// as the C ABI's raw tallies are).
int finalize(Workspace* w, const PhantomObj& P, const unsigned long long* tally, uint32_t nsum, size_t stride,
             uint32_t K, const std::vector<double>& nk, uint64_t n, double* d_dose, double* d_sigma, bool ledger,
             bool sync, bool blocked = true);
// Counters -> stats (from the pinned copy when `pinned`), ledger check.
int stats_from_counters(Workspace* w, const unsigned long long* slots, gmc_run_stats* stats, uint64_t n_hist,
                        uint64_t rounds, double t_total_s, double t_device_s);
int collect_stats(Workspace* w, gmc_run_stats* stats, uint64_t n_hist, uint64_t rounds,
                  std::chrono::steady_clock::time_point t_start);

// Job class of the autotuner's cache.
std::vector<int> job_class(const PhantomObj& P, const TablesObj& T, const gmc_source* srcs, const uint64_t* n_hist,
                           int n_beams);

struct Server;

}  // namespace gmc

struct gmc_context {
  int device = 0;
  std::string err;
  std::mutex mu;   // guards the maps and the tuning cache (the server thread reads them)
  int32_t next_id = 1;
  std::map<int32_t, std::unique_ptr<gmc::TablesObj>> tables;
  std::map<int32_t, std::unique_ptr<gmc::PhantomObj>> phantoms;
  std::map<std::pair<int32_t, int32_t>, gmc::MajObj> majorants;
  std::map<std::vector<int>, gmc_tuning> tuned;   // autotuner choices per job class
  std::map<int32_t, int> refs;                     // server requests holding a tables / phantom id
  gmc::Workspace ws;                               // the blocking forms' workspace
  hipStream_t gstream = nullptr;                   // owned stream the batched form captures on
  hipEvent_t join = nullptr;
  gmc::Server* server = nullptr;                   // owned; see server_destroy
};

namespace gmc {
int cfail(gmc_context* c, int code, const std::string& msg);
// Majorants of a (phantom, tables) pair, built and uploaded once (locks c->mu).
int get_majorants(gmc_context* c, int32_t pid, int32_t tid, const PhantomObj& p, const TablesObj& t, MajObj* out,
                  std::string* err);
// Blocking run of a job in the context's workspace (the plain and batched forms).
// tally_out (single-beam plain runs): the raw [K][nvox] batch tallies are
// copied there too (host or device per tally_kind); dose may then be NULL.
int run_job(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs, const uint64_t* n_hist,
            int n_beams, uint64_t seed, double* const* dose_per_beam, double* const* sigma_per_beam, double* dose,
            double* sigma, int out_kind, const gmc_tuning* tuning, gmc_run_stats* stats, bool batched,
            uint64_t* tally_out = nullptr, int tally_kind = GMC_HOST);
// per_beam: tune the job as run with per-beam outputs (their tally layout),
// a job class of its own.
int autotune(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs, const uint64_t* n_hist,
             int n_beams, double budget_s, gmc_tuning* out, gmc_autotune_report* rep, bool per_beam = false);
// Served form (gmc_server.cpp).
void server_destroy(gmc_context* c);
}  // namespace gmc
