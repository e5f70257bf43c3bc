// gmc_runtime.cpp -- host runtime behind the C ABI of include/gpumcd.h: device
// buffers, table and phantom handles, and the transport engine.
//
// The engine runs rounds of [admit primaries -> electron pass -> compaction
// -> photon pass -> compaction] until every history is admitted and both
// particle arrays are empty (Sec. II.C.2: photons and electrons are simulated
// in alternating passes; the leftover threshold is zero, so no particle is
// ever dropped).  Pass sizes are planned on the device from device-resident
// counts.  The plain form (gmc_run_beam) reads the counts after admission and
// after the electron pass of every round and skips empty passes; the batched
// form (gmc_run_beams) captures several rounds in a HIP graph and replays it,
// reading the counts once per replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "gmc_internal.hpp"
#include "gmc_tables.hpp"
#include "gpumcd.h"

using namespace gmc;

namespace {

struct TablesObj {
  gmc_physics phys{};
  double kcut = 0, kc = 0;
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
};

struct MajObj {
  float* d_g = nullptr;
  float* d_e = nullptr;
};

struct QueueBuf {
  DevQueue q{};
  void* base = nullptr;
};

constexpr uint32_t kDefaultCap = 1u << 23;
constexpr uint32_t kMaxCap = 1u << 26;
constexpr uint32_t kMaxWaves = 1u << 15;
constexpr double kAutotuneBudgetS = 3.0;   // default wall-clock budget of one tuning

}  // namespace

struct gmc_context {
  int device = 0;
  hipStream_t stream = nullptr;     // the caller's (or an owned) stream
  bool own_stream = false;
  hipStream_t gstream = nullptr;    // owned stream the batched form captures on
  hipEvent_t join = nullptr;
  std::string err;
  int32_t next_id = 1;
  std::map<int32_t, std::unique_ptr<TablesObj>> tables;
  std::map<int32_t, std::unique_ptr<PhantomObj>> phantoms;
  std::map<std::pair<int32_t, int32_t>, MajObj> majorants;
  std::map<std::vector<int>, gmc_tuning> tuned;   // autotuner choices per job class
  // particle queues [type: 0 photon, 1 electron][2 buffers]; buffer acc[t]
  // of each type accumulates, the other one is consumed by the next pass
  uint32_t cap = 0;
  QueueBuf qbuf[2][2];
  int acc[2] = {0, 0};
  QueueBuf stg[2];                 // staging: [0] same type, [1] other type
  uint32_t stg_cap = 0;
  uint32_t* d_counts = nullptr;    // [type][buffer]
  uint32_t* d_sched = nullptr;     // admission cursor per type [2], histories per type [2]
  AdmitPlan* d_adm = nullptr;      // [2]
  PassPlan* d_plan = nullptr;      // [2]
  uint32_t* d_used = nullptr;      // [2][kMaxWaves]
  uint32_t* d_offsets = nullptr;   // [2][kMaxWaves + 1]
  unsigned long long* d_ctr = nullptr;  // [C_COUNT][kCtrSlots]
  unsigned long long* d_tally = nullptr;
  size_t tally_elems = 0;
  DevBeam* d_beams = nullptr;
  DevSource* d_sources = nullptr;
  uint32_t* d_start = nullptr;     // [2][beams_cap + 1]
  uint32_t* d_beam_of = nullptr;   // [2][beams_cap]
  size_t beams_cap = 0;
  double* d_nk = nullptr;
  double* d_dose = nullptr;
  double* d_sigma = nullptr;
  size_t out_elems = 0;
  int resident[2] = {0, 0};
  int resident_block[2] = {0, 0};
  int resident_nmat[2] = {0, 0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t kev0 = nullptr, kev1 = nullptr;   // around each pass launch (plain form)
  std::vector<hipEvent_t> gev;                 // pairs around each pass of a captured graph
  double t_pass[2] = {0.0, 0.0};               // summed pass durations, s
  uint64_t n_pass[2] = {0, 0};
};

namespace {

int fail(gmc_context* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_TRY(ctx, expr)                                                               \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, e_ == hipErrorOutOfMemory ? GMC_ENOMEM : GMC_EDEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

void free_queue(QueueBuf& b) {
  if (b.base) (void)hipFree(b.base);
  b = QueueBuf{};
}

hipError_t alloc_queue(QueueBuf& b, uint32_t cap) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, (size_t)Q_FIELDS * cap * sizeof(uint32_t));
  if (e != hipSuccess) return e;
  b.base = p;
  b.q.base = static_cast<uint32_t*>(p);
  b.q.stride = cap;
  b.q.cap = cap;
  return hipSuccess;
}

int ensure_queues(gmc_context* c, uint32_t cap) {
  if (c->cap >= cap) return GMC_OK;
  for (auto& t : c->qbuf)
    for (auto& b : t) free_queue(b);
  c->cap = 0;
  for (auto& t : c->qbuf)
    for (auto& b : t) HIP_TRY(c, alloc_queue(b, cap));
  c->cap = cap;
  return GMC_OK;
}

int ensure_staging(gmc_context* c, uint32_t slots) {
  if (c->stg_cap >= slots) return GMC_OK;
  if ((uint64_t)slots * Q_FIELDS >= (1ull << 32)) return fail(c, GMC_EOVERFLOW, "staging queue too large");
  for (auto& b : c->stg) free_queue(b);
  c->stg_cap = 0;
  for (auto& b : c->stg) HIP_TRY(c, alloc_queue(b, slots));
  c->stg_cap = slots;
  return GMC_OK;
}

int ensure_tally(gmc_context* c, size_t elems) {
  if (c->tally_elems >= elems) return GMC_OK;
  if (c->d_tally) (void)hipFree(c->d_tally);
  c->d_tally = nullptr;
  c->tally_elems = 0;
  HIP_TRY(c, hipMalloc(&c->d_tally, elems * sizeof(unsigned long long)));
  c->tally_elems = elems;
  return GMC_OK;
}

int ensure_out(gmc_context* c, size_t elems) {
  if (c->out_elems >= elems) return GMC_OK;
  if (c->d_dose) (void)hipFree(c->d_dose);
  if (c->d_sigma) (void)hipFree(c->d_sigma);
  c->d_dose = c->d_sigma = nullptr;
  c->out_elems = 0;
  HIP_TRY(c, hipMalloc(&c->d_dose, elems * sizeof(double)));
  HIP_TRY(c, hipMalloc(&c->d_sigma, elems * sizeof(double)));
  c->out_elems = elems;
  return GMC_OK;
}

int ensure_beams(gmc_context* c, size_t n) {
  if (c->beams_cap >= n) return GMC_OK;
  (void)hipFree(c->d_beams);
  (void)hipFree(c->d_sources);
  (void)hipFree(c->d_start);
  (void)hipFree(c->d_beam_of);
  c->d_beams = nullptr;
  c->d_sources = nullptr;
  c->d_start = nullptr;
  c->d_beam_of = nullptr;
  c->beams_cap = 0;
  HIP_TRY(c, hipMalloc(&c->d_beams, n * sizeof(DevBeam)));
  HIP_TRY(c, hipMalloc(&c->d_sources, n * sizeof(DevSource)));
  HIP_TRY(c, hipMalloc(&c->d_start, 2 * (n + 1) * sizeof(uint32_t)));
  HIP_TRY(c, hipMalloc(&c->d_beam_of, 2 * n * sizeof(uint32_t)));
  c->beams_cap = n;
  return GMC_OK;
}

DevPhantom dev_phantom(const PhantomObj& p) {
  DevPhantom d;
  d.vox = p.d_vox;
  d.nx = p.nx; d.ny = p.ny; d.nz = p.nz;
  d.dx = (float)p.dx; d.dy = (float)p.dy; d.dz = (float)p.dz;
  d.idx = (float)(1.0 / p.dx); d.idy = (float)(1.0 / p.dy); d.idz = (float)(1.0 / p.dz);
  d.lx = (float)(p.nx * p.dx); d.ly = (float)(p.ny * p.dy); d.lz = (float)(p.nz * p.dz);
  d.skin = (float)(1e-4 * std::min(p.dx, std::min(p.dy, p.dz)));
  return d;
}

uint32_t mev_to_lsb(double e) { return (uint32_t)std::llround(e * 134217728.0); }

DevCuts dev_cuts(const TablesObj& t) {
  DevCuts c;
  c.ecut_lsb = mev_to_lsb(t.phys.ecut_mev);
  c.pcut_lsb = mev_to_lsb(t.phys.pcut_mev);
  c.kcut2_lsb = mev_to_lsb(2.0 * t.kcut);
  c.kc_lsb = mev_to_lsb(t.kc);
  c.two_mc2_lsb = mev_to_lsb(2.0 * 0.51099895);
  c.kcut = (float)t.kcut;
  c.kc = (float)t.kc;
  c.esmax_gcm2 = t.phys.esmax_gcm2 > 0 ? (float)t.phys.esmax_gcm2 : 0.0f;
  c.emin = (float)kEmin;
  c.mode = t.phys.test_mode;
  return c;
}

DevSource dev_source(const gmc_source& s) {
  DevSource d;
  d.particle = s.particle;
  d.spectrum = s.spectrum;
  d.e_lsb = mev_to_lsb(s.e_mev);
  d.e_lo = (float)s.e_lo;
  d.e_mode = (float)s.e_mode;
  d.e_hi = (float)s.e_hi;
  d.cx = (float)s.cx_cm;
  d.cy = (float)s.cy_cm;
  d.wx = (float)s.wx_cm;
  d.wy = (float)s.wy_cm;
  return d;
}

int get_majorants(gmc_context* c, int32_t pid, int32_t tid, const PhantomObj& p, const TablesObj& t, MajObj* out) {
  auto key = std::make_pair(pid, tid);
  auto it = c->majorants.find(key);
  if (it != c->majorants.end()) { *out = it->second; return GMC_OK; }
  std::vector<float> g(kNE), e(kNE);
  build_majorants(t.host, p.rho_max.data(), g.data(), e.data());
  MajObj m;
  HIP_TRY(c, hipMalloc(&m.d_g, kNE * sizeof(float)));
  HIP_TRY(c, hipMalloc(&m.d_e, kNE * sizeof(float)));
  HIP_TRY(c, hipMemcpy(m.d_g, g.data(), kNE * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(m.d_e, e.data(), kNE * sizeof(float), hipMemcpyHostToDevice));
  c->majorants[key] = m;
  *out = m;
  return GMC_OK;
}

DevTables dev_tables(const TablesObj& t, const MajObj& m) {
  DevTables d;
  d.ph = t.d_ph; d.el = t.d_el; d.ms = t.d_ms;
  d.maj_g = m.d_g; d.maj_e = m.d_e;
  d.n_mat = t.host.n_mat;
  d.lg2_emin = (float)std::log2(kEmin);
  d.inv_h2 = (float)((kNE - 1) / std::log2(kEmax / kEmin));
  d.ms_y0 = (float)t.host.ms_y0;
  d.ms_inv_dy = (float)(1.0 / t.host.ms_dy);
  return d;
}

int check_source(gmc_context* c, const gmc_source* s) {
  if (!s) return fail(c, GMC_EINVAL, "source is NULL");
  if (s->particle != GMC_PHOTON && s->particle != GMC_ELECTRON) return fail(c, GMC_EINVAL, "bad particle type");
  if (s->spectrum == GMC_MONO) {
    if (!(s->e_mev > 0.0 && s->e_mev <= 30.0)) return fail(c, GMC_EINVAL, "energy must be in (0, 30] MeV");
  } else if (s->spectrum == GMC_TRIANGULAR) {
    if (!(s->e_lo > 0.0 && s->e_lo <= s->e_mode && s->e_mode <= s->e_hi && s->e_lo < s->e_hi && s->e_hi <= 30.0))
      return fail(c, GMC_EINVAL, "triangular spectrum needs 0 < lo <= mode <= hi <= 30, lo < hi");
  } else {
    return fail(c, GMC_EINVAL, "bad spectrum kind");
  }
  if (!(std::isfinite(s->cx_cm) && std::isfinite(s->cy_cm) && s->wx_cm >= 0.0 && s->wy_cm >= 0.0 &&
        std::isfinite(s->wx_cm) && std::isfinite(s->wy_cm)))
    return fail(c, GMC_EINVAL, "bad field geometry");
  return GMC_OK;
}

struct Tune {
  int events, secondaries, chunk, block, pass_items, wave_items, rounds, refill;
};

Tune resolve_tuning(const gmc_tuning* t) {
  Tune r{64, 4, 1 << 20, 256, 1 << 21, 64, 4, 1};
  if (t) {
    if (t->events_per_visit > 0) r.events = t->events_per_visit;
    if (t->secondaries_per_visit >= 2) r.secondaries = std::min(t->secondaries_per_visit, 64);
    if (t->chunk > 0) r.chunk = std::min(t->chunk, 1 << 24);
    if (t->wg_size >= 64 && t->wg_size <= 256 && t->wg_size % 64 == 0) r.block = t->wg_size;
    if (t->pass_items > 0) r.pass_items = std::min(std::max(t->pass_items, 1024), 1 << 23);
    if (t->wave_items > 0) r.wave_items = std::min(std::max(t->wave_items, 64), 1 << 16);
    if (t->rounds_per_check > 0) r.rounds = std::min(t->rounds_per_check, 1024);
    if (t->refill_lanes > 0) r.refill = std::min(t->refill_lanes, 64);
  }
  return r;
}

int resident_blocks(gmc_context* c, int kernel, int block, int n_mat) {
  if (c->resident[kernel] == 0 || c->resident_block[kernel] != block || c->resident_nmat[kernel] != n_mat) {
    const size_t lds = kernel == 0 ? photon_lds_bytes(n_mat) : electron_lds_bytes(n_mat);
    c->resident[kernel] = max_resident_blocks(kernel, block, lds);
    c->resident_block[kernel] = block;
    c->resident_nmat[kernel] = n_mat;
  }
  return c->resident[kernel];
}

int copy_out(gmc_context* c, double* dst, const double* src, size_t n, int kind) {
  if (!dst) return GMC_OK;
  HIP_TRY(c, hipMemcpyAsync(dst, src, n * sizeof(double),
                            kind == GMC_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream));
  return GMC_OK;
}

// ------------------------------------------------------------------ engine
// One transport job: its beams, their sources and tally targets.  Histories
// of each particle type are numbered consecutively over the beams of that
// type (start[t][j] is the first history of the j-th beam of type t).
struct Job {
  const PhantomObj* P = nullptr;
  const TablesObj* T = nullptr;
  MajObj maj;
  std::vector<DevBeam> beams;
  std::vector<DevSource> sources;
  std::vector<uint32_t> start[2], beam_of[2];
  uint32_t total[2] = {0, 0};
};

struct Engine {
  gmc_context* c = nullptr;
  Tune tu{};
  PassArgs proto{};
  AdmitArgs adm[2]{};
  uint32_t total[2] = {0, 0};
  uint32_t waves[2] = {0, 0};     // wavefronts of each pass grid
  uint32_t blocks[2] = {0, 0};
  uint32_t bud_same[2] = {0, 0}, bud_other[2] = {0, 0};
};

uint32_t* count_ptr(gmc_context* c, int type, int buf) { return c->d_counts + 2 * type + buf; }

// Record `ev` on stream s; while s is being captured, as an event record node
// appended to the captured graph after the current dependencies.
hipError_t record_event(hipStream_t s, hipEvent_t ev, bool capturing) {
  if (!capturing) return hipEventRecord(ev, s);
  hipStreamCaptureStatus status = hipStreamCaptureStatusNone;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  hipError_t e = hipStreamGetCaptureInfo_v2(s, &status, nullptr, &g, &deps, &nd);
  if (e != hipSuccess) return e;
  if (status != hipStreamCaptureStatusActive) return hipErrorIllegalState;
  hipGraphNode_t node = nullptr;
  e = hipGraphAddEventRecordNode(&node, g, deps, nd, ev);
  if (e != hipSuccess) return e;
  return hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
}

// Enqueue plan, pass and the two compactions of `type` over its accumulating
// buffer, which becomes the work buffer; the other buffer accumulates from
// then on.  The pass kernel is bracketed by the events t0 / t1 (recorded as
// graph event nodes while the stream is being captured).
int enqueue_pass(Engine& E, int type, hipEvent_t t0, hipEvent_t t1, bool capturing) {
  gmc_context* c = E.c;
  const int other = 1 - type;
  const int wi = c->acc[type];
  c->acc[type] ^= 1;
  const int ni = c->acc[type];
  PlanArgs pa;
  pa.n_work = count_ptr(c, type, wi);
  pa.n_other = count_ptr(c, other, c->acc[other]);
  pa.plan = c->d_plan + type;
  pa.cap = c->cap;
  pa.max_items = (uint32_t)E.tu.pass_items;
  pa.waves = E.waves[type];
  pa.min_per_wave = (uint32_t)E.tu.wave_items;
  pa.bud_same = E.bud_same[type];
  pa.bud_other = E.bud_other[type];
  HIP_TRY(c, launch_plan_pass(pa, c->stream));
  PassArgs a = E.proto;
  a.work = c->qbuf[type][wi].q;
  a.plan = c->d_plan + type;
  a.stg_same = c->stg[0].q;
  a.stg_other = c->stg[1].q;
  a.used_same = c->d_used;
  a.used_other = c->d_used + kMaxWaves;
  HIP_TRY(c, record_event(c->stream, t0, capturing));
  hipError_t e = type == 0 ? launch_photon_pass(a, (int)E.blocks[0], E.tu.block, c->stream)
                           : launch_electron_pass(a, (int)E.blocks[1], E.tu.block, c->stream);
  if (e != hipSuccess) return fail(c, GMC_EDEVICE, std::string("pass launch: ") + hipGetErrorString(e));
  HIP_TRY(c, record_event(c->stream, t1, capturing));
  for (int d = 0; d < 2; ++d) {
    const int dt = d == 0 ? type : other;
    const int dbuf = d == 0 ? ni : c->acc[other];
    CompactArgs ca;
    ca.stg = c->stg[d].q;
    ca.plan = c->d_plan + type;
    ca.same = d == 0;
    ca.used = d == 0 ? a.used_same : a.used_other;
    ca.waves = E.waves[type];
    ca.offsets = c->d_offsets + d * (kMaxWaves + 1);
    ca.dst = c->qbuf[dt][dbuf].q;
    ca.dst_count = count_ptr(c, dt, dbuf);
    ca.work = c->qbuf[type][wi].q;
    ca.work_count = count_ptr(c, type, wi);
    ca.ctr = c->d_ctr;
    e = launch_compact(ca, c->stream);
    if (e != hipSuccess) return fail(c, GMC_EDEVICE, std::string("compaction launch: ") + hipGetErrorString(e));
  }
  return GMC_OK;
}

int enqueue_admission(Engine& E) {
  gmc_context* c = E.c;
  AdmitPlanArgs ap;
  ap.cursor = c->d_sched;
  ap.total = c->d_sched + 2;
  ap.count0 = count_ptr(c, 0, c->acc[0]);
  ap.count1 = count_ptr(c, 1, c->acc[1]);
  ap.out = c->d_adm;
  ap.cap = c->cap;
  ap.chunk = (uint32_t)E.tu.chunk;
  HIP_TRY(c, launch_admit_plan(ap, c->stream));
  for (int t = 0; t < 2; ++t) {
    AdmitArgs a = E.adm[t];
    a.out = c->qbuf[t][c->acc[t]].q;
    HIP_TRY(c, launch_admit(a, std::min<uint32_t>((uint32_t)E.tu.chunk, E.total[t]), c->stream));
  }
  return GMC_OK;
}

struct Status {
  uint32_t counts[4];
  uint32_t sched[4];            // cursor[2], total[2]
  PassPlan plan[2];
  AdmitPlan adm[2];
  bool done() const {
    return sched[0] == sched[2] && sched[1] == sched[3] && counts[0] == 0 && counts[1] == 0 && counts[2] == 0 &&
           counts[3] == 0;
  }
};

int read_status(gmc_context* c, Status* s) {
  HIP_TRY(c, hipMemcpyAsync(s->counts, c->d_counts, sizeof(s->counts), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(s->sched, c->d_sched, sizeof(s->sched), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(s->plan, c->d_plan, sizeof(s->plan), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(s->adm, c->d_adm, sizeof(s->adm), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < 4; ++i)
    if (s->counts[i] > c->cap) return fail(c, GMC_EINTERNAL, "particle queue overflow on the device");
  return GMC_OK;
}

int stuck(gmc_context* c) {
  return fail(c, GMC_EOVERFLOW,
              "both particle queues are too full for any pass to proceed; lower the chunk or the secondaries "
              "budget");
}

// Device state of a job: queues, staging, beam tables, counters.
int engine_setup(gmc_context* c, Engine& E, const Job& J, const Tune& tu) {
  E.c = c;
  E.tu = tu;
  E.total[0] = J.total[0];
  E.total[1] = J.total[1];
  const int n_mat = J.T->host.n_mat;
  const uint64_t want = (uint64_t)tu.chunk * (uint64_t)(tu.secondaries + 1) * 2u;
  const uint32_t cap = (uint32_t)std::max<uint64_t>(kDefaultCap, std::min<uint64_t>(want, kMaxCap));
  int rc = ensure_queues(c, cap);
  if (rc) return rc;
  uint32_t stg = 0;
  for (int t = 0; t < 2; ++t) {
    E.bud_same[t] = t == 0 ? 1u : (uint32_t)tu.secondaries + 1u;
    E.bud_other[t] = (uint32_t)tu.secondaries;
    const uint32_t wpb = (uint32_t)tu.block / 64u;
    const uint32_t res = (uint32_t)resident_blocks(c, t, tu.block, n_mat);
    E.blocks[t] = std::max<uint32_t>(1u, std::min<uint32_t>(res, kMaxWaves / wpb));
    E.waves[t] = E.blocks[t] * wpb;
    const uint32_t qmax =
        std::max<uint32_t>((uint32_t)tu.wave_items, ((uint32_t)tu.pass_items + E.waves[t] - 1) / E.waves[t]);
    stg = std::max<uint32_t>(stg, E.waves[t] * qmax * std::max(E.bud_same[t], E.bud_other[t]));
  }
  rc = ensure_staging(c, stg);
  if (rc) return rc;
  const size_t nb = J.beams.size();
  rc = ensure_beams(c, nb);
  if (rc) return rc;
  HIP_TRY(c, hipMemcpy(c->d_beams, J.beams.data(), nb * sizeof(DevBeam), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->d_sources, J.sources.data(), nb * sizeof(DevSource), hipMemcpyHostToDevice));
  for (int t = 0; t < 2; ++t) {
    HIP_TRY(c, hipMemcpy(c->d_start + t * (c->beams_cap + 1), J.start[t].data(), J.start[t].size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice));
    if (!J.beam_of[t].empty())
      HIP_TRY(c, hipMemcpy(c->d_beam_of + t * c->beams_cap, J.beam_of[t].data(),
                           J.beam_of[t].size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  }
  const uint32_t sched[4] = {0u, 0u, J.total[0], J.total[1]};
  HIP_TRY(c, hipMemcpy(c->d_sched, sched, sizeof(sched), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemsetAsync(c->d_counts, 0, 4 * sizeof(uint32_t), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_ctr, 0, C_COUNT * kCtrSlots * sizeof(unsigned long long), c->stream));
  c->acc[0] = c->acc[1] = 0;
  const DevPhantom dph = dev_phantom(*J.P);
  const DevCuts cuts = dev_cuts(*J.T);
  E.proto = PassArgs{};
  E.proto.ph = dph;
  E.proto.tab = dev_tables(*J.T, J.maj);
  E.proto.cut = cuts;
  E.proto.beams = c->d_beams;
  E.proto.ctr = c->d_ctr;
  E.proto.max_events = tu.events;
  E.proto.max_secondaries = tu.secondaries;
  E.proto.refill_lanes = tu.refill;
  for (int t = 0; t < 2; ++t) {
    AdmitArgs& a = E.adm[t];
    a = AdmitArgs{};
    a.ph = dph;
    a.cut = cuts;
    a.plan = c->d_adm + t;
    a.start = c->d_start + t * (c->beams_cap + 1);
    a.beam_of = c->d_beam_of + t * c->beams_cap;
    a.nb = (uint32_t)J.beam_of[t].size();
    a.beams = c->d_beams;
    a.sources = c->d_sources;
    a.ctr = c->d_ctr;
    a.nvox = (uint32_t)((size_t)J.P->nx * J.P->ny * J.P->nz);
  }
  c->t_pass[0] = c->t_pass[1] = 0.0;
  c->n_pass[0] = c->n_pass[1] = 0;
  return GMC_OK;
}

int add_pass_time(gmc_context* c, int type, hipEvent_t t0, hipEvent_t t1) {
  float ms = 0.0f;
  HIP_TRY(c, hipEventElapsedTime(&ms, t0, t1));
  c->t_pass[type] += ms * 1e-3;
  ++c->n_pass[type];
  return GMC_OK;
}

// Plain form: counts read after admission and after the electron pass of
// every round; passes with nothing to do are skipped.  A round in which no
// primary was admitted and no pass transported anything leaves the state
// unchanged, so the next one would too: that is reported, not looped on.
int engine_run_plain(Engine& E, uint64_t* rounds) {
  gmc_context* c = E.c;
  Status st;
  bool e_prog = true, g_ran = false;
  for (;;) {
    int rc = enqueue_admission(E);
    if (rc) return rc;
    rc = read_status(c, &st);
    if (rc) return rc;
    if (g_ran) rc = add_pass_time(c, 0, c->kev0, c->kev1);
    if (rc) return rc;
    if (st.done()) break;
    const bool g_prog = g_ran && st.plan[0].m > 0;
    if (*rounds > 0 && st.adm[0].count == 0 && st.adm[1].count == 0 && !e_prog && !g_prog) return stuck(c);
    ++*rounds;
    e_prog = false;
    g_ran = false;
    if (st.counts[2 + c->acc[1]] > 0) {
      rc = enqueue_pass(E, 1, c->kev0, c->kev1, false);
      if (rc) return rc;
      rc = read_status(c, &st);
      if (rc) return rc;
      rc = add_pass_time(c, 1, c->kev0, c->kev1);
      if (rc) return rc;
      e_prog = st.plan[1].m > 0;
    }
    if (st.counts[c->acc[0]] > 0) {
      rc = enqueue_pass(E, 0, c->kev0, c->kev1, false);
      if (rc) return rc;
      g_ran = true;
    }
  }
  return GMC_OK;
}

int ensure_graph_events(gmc_context* c, size_t n) {
  while (c->gev.size() < n) {
    hipEvent_t e = nullptr;
    HIP_TRY(c, hipEventCreate(&e));
    c->gev.push_back(e);
  }
  return GMC_OK;
}

// Batched form: 2 R rounds (R = rounds_per_check) captured in one graph --
// each type's buffers swap once per round, so after an even number of rounds
// the buffer roles are back where they started -- replayed until the job is
// done, with one status read per replay.  Every pass kernel in the graph is
// bracketed by its own pair of event nodes, read after each replay.
int engine_run_graph(Engine& E, uint64_t* rounds) {
  gmc_context* c = E.c;
  const int nr = 2 * E.tu.rounds;
  int rc = ensure_graph_events(c, (size_t)4 * nr);
  if (rc) return rc;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  for (int r = 0; r < nr && rc == GMC_OK; ++r) {
    rc = enqueue_admission(E);
    if (rc == GMC_OK) rc = enqueue_pass(E, 1, c->gev[4 * r + 2], c->gev[4 * r + 3], true);
    if (rc == GMC_OK) rc = enqueue_pass(E, 0, c->gev[4 * r], c->gev[4 * r + 1], true);
  }
  const hipError_t ec = hipStreamEndCapture(c->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return fail(c, GMC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(c, GMC_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  Status st;
  for (;;) {
    e = hipGraphLaunch(exec, c->stream);
    if (e != hipSuccess) break;
    *rounds += (uint64_t)nr;
    rc = read_status(c, &st);
    if (rc) break;
    // pair i brackets the pass of type i & 1 in round i / 2
    for (int i = 0; i < 2 * nr && rc == GMC_OK; ++i) rc = add_pass_time(c, i & 1, c->gev[2 * i], c->gev[2 * i + 1]);
    if (rc || st.done()) break;
    // the last round admitted nothing and both of its passes transported
    // nothing: a fixed point
    if (st.adm[0].count == 0 && st.adm[1].count == 0 && st.plan[0].m == 0 && st.plan[1].m == 0) {
      rc = stuck(c);
      break;
    }
  }
  (void)hipGraphExecDestroy(exec);
  if (e != hipSuccess) return fail(c, GMC_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  return rc;
}

// Histories per batch for interleaved batches: n_k = #{h < n : h mod K = k}.
void add_batch_sizes(std::vector<double>& nk, uint64_t n, uint32_t K) {
  nk.resize(K, 0.0);
  for (uint32_t k = 0; k < K; ++k) nk[k] += (double)((n + K - 1 - k) / K);
}

// Dose and sigma of `nsum` tallies ([K][nvox] each, `stride` elements apart,
// added together) into device buffers (Eqs. 11-13).  nk: histories per
// batch; n: all histories.
int finalize(gmc_context* c, const PhantomObj& P, const unsigned long long* tally, uint32_t nsum, size_t stride,
             uint32_t K, const std::vector<double>& nk, uint64_t n, double* d_dose, double* d_sigma, bool ledger) {
  HIP_TRY(c, hipMemcpyAsync(c->d_nk, nk.data(), K * sizeof(double), hipMemcpyHostToDevice, c->stream));
  FinalizeArgs fa;
  fa.tally = tally;
  fa.nsum = nsum;
  fa.sum_stride = stride;
  fa.vox = P.d_vox;
  fa.nk = c->d_nk;
  fa.nvox = (uint32_t)((size_t)P.nx * P.ny * P.nz);
  fa.K = K;
  fa.n_total = (double)n;
  fa.conv = kLsbMeV * 1.602176634e-13 / (P.dx * P.dy * P.dz * 1e-3);
  fa.dose = d_dose;
  fa.sigma = d_sigma;
  fa.ctr = ledger ? c->d_ctr : nullptr;
  HIP_TRY(c, launch_finalize(fa, c->stream));
  // the batch sizes come from host memory the caller may release on return
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return GMC_OK;
}

int collect_stats(gmc_context* c, gmc_run_stats* stats, uint64_t n_hist, uint64_t rounds,
                  std::chrono::steady_clock::time_point t_start) {
  std::vector<unsigned long long> slots((size_t)C_COUNT * kCtrSlots);
  HIP_TRY(c, hipMemcpyAsync(slots.data(), c->d_ctr, slots.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float dev_ms = 0.0f;
  HIP_TRY(c, hipEventElapsedTime(&dev_ms, c->ev0, c->ev1));
  unsigned long long ctr[C_COUNT] = {};
  for (int k = 0; k < C_COUNT; ++k)
    for (int j = 0; j < kCtrSlots; ++j) ctr[k] += slots[(size_t)k * kCtrSlots + j];
  const long long resid = (long long)(ctr[C_E_IN] - ctr[C_E_DEP] - ctr[C_E_ESC] - ctr[C_E_SINK]);
  if (stats) {
    stats->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    stats->t_device_s = dev_ms * 1e-3;
    stats->e_in_mev = ctr[C_E_IN] * kLsbMeV;
    stats->e_dep_mev = ctr[C_E_DEP] * kLsbMeV;
    stats->e_esc_mev = ctr[C_E_ESC] * kLsbMeV;
    stats->e_sink_mev = ctr[C_E_SINK] * kLsbMeV;
    stats->n_hist = n_hist;
    stats->n_photon_events = ctr[C_PH_EVENTS];
    stats->n_fictitious = ctr[C_FICT];
    stats->n_e_steps = ctr[C_E_STEPS];
    stats->n_hard = ctr[C_HARD];
    stats->n_secondaries = ctr[C_SEC];
    stats->n_majorant_violations = ctr[C_VIOL];
    stats->n_passes = rounds;
    stats->ledger_residual_lsb = resid;
    stats->t_photon_pass_s = c->t_pass[0];
    stats->t_electron_pass_s = c->t_pass[1];
    stats->n_photon_launches = c->n_pass[0];
    stats->n_electron_launches = c->n_pass[1];
  }
  if (ctr[C_OVERFLOW]) return fail(c, GMC_EINTERNAL, "queue overflow detected on the device");
  if (resid != 0) return fail(c, GMC_EINTERNAL, "energy ledger does not close: residual " + std::to_string(resid));
  return GMC_OK;
}

// The batched form works on the context's own capture stream, ordered after
// the caller's stream on entry and before it on exit.
struct StreamSwap {
  gmc_context* c;
  hipStream_t user;
  bool on;
  StreamSwap(gmc_context* ctx, bool enable) : c(ctx), user(ctx->stream), on(enable) {
    if (!on) return;
    (void)hipEventRecord(c->join, user);
    (void)hipStreamWaitEvent(c->gstream, c->join, 0);
    c->stream = c->gstream;
  }
  ~StreamSwap() {
    if (!on) return;
    (void)hipEventRecord(c->join, c->gstream);
    (void)hipStreamWaitEvent(user, c->join, 0);
    c->stream = user;
  }
};

// How the batched form tallies (the plain form is kCombined with one beam).
enum TallyMode {
  kCombined,       // one tally [K][nvox] batched over all histories: no per-beam doses
  kBeamBatched,    // a [K][nvox] tally per beam; the combined result is their sum
  kBeamPlusComb    // a [1][nvox] tally per beam plus a combined [K][nvox] one (two additions per deposit)
};

// Shared by the plain and batched forms.
int run_job(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs, const uint64_t* n_hist,
            int n_beams, uint64_t seed, double* const* dose_per_beam, double* const* sigma_per_beam, double* dose,
            double* sigma, int out_kind, const gmc_tuning* tuning, gmc_run_stats* stats, bool batched) {
  const auto t_start = std::chrono::steady_clock::now();
  auto pi = c->phantoms.find(phantom_id);
  auto ti = c->tables.find(tables_id);
  if (pi == c->phantoms.end() || ti == c->tables.end()) return fail(c, GMC_ENOTFOUND, "unknown phantom or tables id");
  const PhantomObj& P = *pi->second;
  const TablesObj& T = *ti->second;
  if (n_beams < 1 || n_beams > (1 << 20) || !srcs || !n_hist) return fail(c, GMC_EINVAL, "need 1 .. 2^20 beams");
  if (!dose) return fail(c, GMC_EINVAL, "dose output is NULL");
  if (out_kind != GMC_HOST && out_kind != GMC_DEVICE) return fail(c, GMC_EINVAL, "bad out_ptr_kind");
  if (P.max_mat >= T.host.n_mat) return fail(c, GMC_EINVAL, "phantom uses a material index beyond the tables");
  const uint32_t K = (uint32_t)T.phys.n_batches;
  uint64_t n_total = 0, per_type[2] = {0, 0}, n_min = ~0ull;
  double e_sum = 0.0;
  for (int b = 0; b < n_beams; ++b) {
    const int rc = check_source(c, &srcs[b]);
    if (rc) return rc;
    if (n_hist[b] == 0) return fail(c, GMC_EINVAL, "every beam needs at least one history");
    if (n_hist[b] >= (1ull << 32)) return fail(c, GMC_EINVAL, "histories must be < 2^32");
    n_total += n_hist[b];
    n_min = std::min<uint64_t>(n_min, n_hist[b]);
    per_type[srcs[b].particle] += n_hist[b];
    const double e_max = srcs[b].spectrum == GMC_MONO ? srcs[b].e_mev : srcs[b].e_hi;
    e_sum += (double)n_hist[b] * (e_max * 134217728.0 + 1.0);
  }
  if (n_total < K) return fail(c, GMC_EINVAL, "need at least n_batches histories");
  if (n_total >= (1ull << 32)) return fail(c, GMC_EINVAL, "total histories must be < 2^32");
  if (e_sum >= 9.2e18) return fail(c, GMC_EOVERFLOW, "histories x energy would overflow the 64-bit tallies");
  (void)hipSetDevice(c->device);
  const Tune tu = resolve_tuning(tuning);
  const size_t nvox = (size_t)P.nx * P.ny * P.nz;
  const size_t NB = (size_t)n_beams;

  // tally layout: per-beam K-batched tallies when per-beam results are asked
  // for, every beam has at least K histories and they fit in half of the free
  // device memory; per-beam sigma needs them
  TallyMode mode = kCombined;
  if (batched && (dose_per_beam || sigma_per_beam)) {
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const double need = (double)NB * K * nvox * sizeof(unsigned long long);
    const double room = 0.5 * ((double)free_b + (double)c->tally_elems * sizeof(unsigned long long));
    mode = (n_min >= K && need <= room) ? kBeamBatched : kBeamPlusComb;
    if (sigma_per_beam && mode != kBeamBatched)
      return fail(c, n_min < K ? GMC_EINVAL : GMC_ENOMEM,
                  n_min < K ? "sigma per beam needs at least n_batches histories in every beam"
                            : "per-beam batched tallies do not fit in device memory");
  }
  const size_t tally_elems = mode == kCombined ? nvox * K : mode == kBeamBatched ? nvox * K * NB : nvox * (K + NB);
  int rc = ensure_tally(c, tally_elems);
  if (rc) return rc;
  rc = ensure_out(c, nvox);
  if (rc) return rc;

  Job J;
  J.P = &P;
  J.T = &T;
  rc = get_majorants(c, phantom_id, tables_id, P, T, &J.maj);
  if (rc) return rc;
  for (int t = 0; t < 2; ++t) J.start[t].push_back(0u);
  uint32_t off = 0;
  for (int b = 0; b < n_beams; ++b) {
    DevBeam db{};
    db.key0 = (uint32_t)seed;
    db.key1 = (uint32_t)(seed >> 32) ^ srcs[b].beam_id;
    db.b = DevTally{nullptr, 1u, 0u};
    if (mode == kCombined) {
      db.a = DevTally{c->d_tally, K, off};
    } else if (mode == kBeamBatched) {
      db.a = DevTally{c->d_tally + nvox * K * (size_t)b, K, 0u};
    } else {
      db.a = DevTally{c->d_tally + nvox * ((size_t)K + (size_t)b), 1u, 0u};
      db.b = DevTally{c->d_tally, K, off};
    }
    J.beams.push_back(db);
    J.sources.push_back(dev_source(srcs[b]));
    const int t = srcs[b].particle;
    J.beam_of[t].push_back((uint32_t)b);
    J.start[t].push_back(J.start[t].back() + (uint32_t)n_hist[b]);
    off += (uint32_t)n_hist[b];
  }
  J.total[0] = (uint32_t)per_type[0];
  J.total[1] = (uint32_t)per_type[1];

  StreamSwap swap(c, batched);
  HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  HIP_TRY(c, launch_fill_u64(c->d_tally, tally_elems, 0ull, c->stream));
  Engine E;
  rc = engine_setup(c, E, J, tu);
  if (rc) return rc;
  uint64_t rounds = 0;
  rc = batched ? engine_run_graph(E, &rounds) : engine_run_plain(E, &rounds);
  if (rc) return rc;

  // combined result (and the ledger's deposited total)
  std::vector<double> nk;
  if (mode == kBeamBatched) {
    for (int b = 0; b < n_beams; ++b) add_batch_sizes(nk, n_hist[b], K);
  } else {
    add_batch_sizes(nk, n_total, K);
  }
  double* d_out = out_kind == GMC_DEVICE ? dose : c->d_dose;
  double* s_out = sigma ? (out_kind == GMC_DEVICE ? sigma : c->d_sigma) : nullptr;
  rc = mode == kBeamBatched ? finalize(c, P, c->d_tally, (uint32_t)NB, nvox * K, K, nk, n_total, d_out, s_out, true)
                            : finalize(c, P, c->d_tally, 1u, 0u, K, nk, n_total, d_out, s_out, true);
  if (rc) return rc;
  if (out_kind == GMC_HOST) {
    rc = copy_out(c, dose, c->d_dose, nvox, GMC_HOST);
    if (rc) return rc;
    if (sigma) rc = copy_out(c, sigma, c->d_sigma, nvox, GMC_HOST);
    if (rc) return rc;
  }
  // per-beam results
  if (mode != kCombined) {
    for (int b = 0; b < n_beams; ++b) {
      double* want_d = dose_per_beam ? dose_per_beam[b] : nullptr;
      double* want_s = sigma_per_beam ? sigma_per_beam[b] : nullptr;
      if (!want_d && !want_s) continue;
      // the dose is always computed; it lands in scratch when not wanted
      double* dd = out_kind == GMC_DEVICE && want_d ? want_d : c->d_dose;
      double* ds = want_s ? (out_kind == GMC_DEVICE ? want_s : c->d_sigma) : nullptr;
      const uint32_t kb = mode == kBeamBatched ? K : 1u;
      const unsigned long long* tb = c->d_tally + (mode == kBeamBatched ? nvox * K * (size_t)b : nvox * ((size_t)K + b));
      std::vector<double> nkb;
      add_batch_sizes(nkb, n_hist[b], kb);
      rc = finalize(c, P, tb, 1u, 0u, kb, nkb, n_hist[b], dd, ds, false);
      if (rc) return rc;
      if (out_kind == GMC_HOST) {
        if (want_d) rc = copy_out(c, want_d, c->d_dose, nvox, GMC_HOST);
        if (rc == GMC_OK && want_s) rc = copy_out(c, want_s, c->d_sigma, nvox, GMC_HOST);
        if (rc) return rc;
      }
    }
  }
  return collect_stats(c, stats, n_total, rounds, t_start);
}

// ---------------------------------------------------------------- autotuner
// Job class for the autotuner's cache: grid size, beam energy, particle mix,
// field area and material count, each on a coarse (mostly logarithmic) scale.
std::vector<int> job_class(const PhantomObj& P, const TablesObj& T, const gmc_source* srcs, const uint64_t* n_hist,
                           int n_beams) {
  double n = 0, e = 0, fe = 0, area = 0;
  for (int b = 0; b < n_beams; ++b) {
    const double w = (double)n_hist[b];
    n += w;
    e += w * (srcs[b].spectrum == GMC_MONO ? srcs[b].e_mev : srcs[b].e_mode);
    fe += srcs[b].particle == GMC_ELECTRON ? w : 0.0;
    area += w * srcs[b].wx_cm * srcs[b].wy_cm;
  }
  const double nvox = (double)P.nx * P.ny * P.nz;
  return {(int)std::lround(std::log2(nvox)), (int)std::lround(2.0 * std::log2(e / n)), (int)std::lround(4.0 * fe / n),
          (int)std::lround(std::log2(area / n + 0.01)), (int)std::lround(std::log2(n)), T.host.n_mat};
}

gmc_tuning default_tuning() {
  const Tune d = resolve_tuning(nullptr);
  gmc_tuning t;
  t.events_per_visit = d.events;
  t.secondaries_per_visit = d.secondaries;
  t.chunk = d.chunk;
  t.wg_size = d.block;
  t.pass_items = d.pass_items;
  t.wave_items = d.wave_items;
  t.rounds_per_check = d.rounds;
  t.refill_lanes = d.refill;
  return t;
}

// Coordinate descent over the engine's knobs on a sample of the job (the
// first histories of every beam, in proportion, about 5% of the job and at
// least 2^20 histories), each candidate timed on the device from the
// admission to the finalize; a change is kept when it saves at least 2%.
int autotune(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs, const uint64_t* n_hist,
             int n_beams, double budget_s, gmc_tuning* out, gmc_autotune_report* rep) {
  auto pi = c->phantoms.find(phantom_id);
  auto ti = c->tables.find(tables_id);
  if (pi == c->phantoms.end() || ti == c->tables.end()) return fail(c, GMC_ENOTFOUND, "unknown phantom or tables id");
  if (n_beams < 1 || !srcs || !n_hist || !out) return fail(c, GMC_EINVAL, "bad autotune arguments");
  const PhantomObj& P = *pi->second;
  const TablesObj& T = *ti->second;
  uint64_t n_total = 0;
  for (int b = 0; b < n_beams; ++b) {
    if (n_hist[b] == 0) return fail(c, GMC_EINVAL, "every beam needs at least one history");
    n_total += n_hist[b];
  }
  if (n_total >= (1ull << 32)) return fail(c, GMC_EINVAL, "total histories must be < 2^32");
  const std::vector<int> key = job_class(P, T, srcs, n_hist, n_beams);
  gmc_autotune_report r{};
  auto hit = c->tuned.find(key);
  if (hit != c->tuned.end()) {
    *out = hit->second;
    r.from_cache = 1;
    if (rep) *rep = r;
    return GMC_OK;
  }
  const uint64_t want = std::min<uint64_t>(n_total, std::max<uint64_t>(1ull << 20, n_total / 20));
  const double f = (double)want / (double)n_total;
  std::vector<uint64_t> ns(n_beams);
  uint64_t n_sample = 0;
  for (int b = 0; b < n_beams; ++b) {
    ns[b] = std::max<uint64_t>(1, (uint64_t)std::llround(f * (double)n_hist[b]));
    n_sample += ns[b];
  }
  if (n_sample < (uint64_t)T.phys.n_batches || n_sample >= (1ull << 32))
    return fail(c, GMC_EINVAL, "job too small or too large to tune");
  int rc = ensure_out(c, (size_t)P.nx * P.ny * P.nz);
  if (rc) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  auto trial = [&](const gmc_tuning& t, double* sec) -> int {
    gmc_run_stats st{};
    const int e = run_job(c, phantom_id, tables_id, srcs, ns.data(), n_beams, 0x5eedull, nullptr, nullptr, c->d_dose,
                          nullptr, GMC_DEVICE, &t, &st, true);
    ++r.trials;
    *sec = st.t_device_s;
    return e;
  };
  gmc_tuning best = default_tuning();
  double t_best = 0.0;
  rc = trial(best, &t_best);   // first run warms the buffers; time again
  if (rc == GMC_OK) rc = trial(best, &t_best);
  if (rc) return rc;
  r.t_default_s = t_best;
  struct Dim { int gmc_tuning::*field; std::vector<int> values; };
  const std::vector<Dim> dims = {
      {&gmc_tuning::chunk, {1 << 18, 1 << 19, 1 << 20, 1 << 21, 1 << 22}},
      {&gmc_tuning::pass_items, {1 << 20, 1 << 21, 1 << 22}},
      {&gmc_tuning::events_per_visit, {16, 32, 64, 128}},
      {&gmc_tuning::wg_size, {128, 256}},
      {&gmc_tuning::wave_items, {64, 128, 256}},
      {&gmc_tuning::refill_lanes, {1, 4, 8}},
      {&gmc_tuning::rounds_per_check, {2, 4, 8}},
  };
  bool out_of_time = false;
  for (const Dim& d : dims) {
    const int cur = best.*(d.field);
    for (int v : d.values) {
      if (v == cur) continue;
      if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > budget_s) {
        out_of_time = true;
        break;
      }
      gmc_tuning cand = best;
      cand.*(d.field) = v;
      double t = 0.0;
      rc = trial(cand, &t);
      if (rc) return rc;
      if (t < 0.98 * t_best) {
        t_best = t;
        best = cand;
      }
    }
    if (out_of_time) break;
  }
  r.t_best_s = t_best;
  r.sample_histories = n_sample;
  r.complete = out_of_time ? 0 : 1;
  c->tuned[key] = best;
  *out = best;
  if (rep) *rep = r;
  return GMC_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

int gmc_create(int device, void* hip_stream, gmc_context** out) {
  if (!out) return GMC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GMC_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return GMC_EDEVICE;
  auto* c = new gmc_context();
  c->device = device;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return GMC_EDEVICE; }
    c->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&c->d_counts, 4 * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&c->d_sched, 4 * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&c->d_adm, 2 * sizeof(AdmitPlan)) != hipSuccess ||
      hipMalloc(&c->d_plan, 2 * sizeof(PassPlan)) != hipSuccess ||
      hipMalloc(&c->d_ctr, C_COUNT * kCtrSlots * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_nk, kMaxBatches * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_used, 2 * kMaxWaves * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&c->d_offsets, 2 * (kMaxWaves + 1) * sizeof(uint32_t)) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreate(&c->kev0) != hipSuccess || hipEventCreate(&c->kev1) != hipSuccess) {
    gmc_destroy(c);
    return GMC_ENOMEM;
  }
  *out = c;
  return GMC_OK;
}

void gmc_destroy(gmc_context* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->gstream) (void)hipStreamSynchronize(c->gstream);
  for (auto& kv : c->tables) {
    (void)hipFree(kv.second->d_ph);
    (void)hipFree(kv.second->d_el);
    (void)hipFree(kv.second->d_ms);
  }
  for (auto& kv : c->phantoms) (void)hipFree(kv.second->d_vox);
  for (auto& kv : c->majorants) {
    (void)hipFree(kv.second.d_g);
    (void)hipFree(kv.second.d_e);
  }
  for (auto& t : c->qbuf)
    for (auto& b : t) free_queue(b);
  for (auto& b : c->stg) free_queue(b);
  for (void* p : {(void*)c->d_used, (void*)c->d_offsets, (void*)c->d_sched, (void*)c->d_adm, (void*)c->d_plan,
                  (void*)c->d_counts, (void*)c->d_ctr, (void*)c->d_tally, (void*)c->d_beams, (void*)c->d_sources,
                  (void*)c->d_start, (void*)c->d_beam_of, (void*)c->d_nk, (void*)c->d_dose, (void*)c->d_sigma})
    if (p) (void)hipFree(p);
  for (hipEvent_t e : {c->ev0, c->ev1, c->kev0, c->kev1, c->join})
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->gev) (void)hipEventDestroy(e);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* gmc_last_error(const gmc_context* c) { return c ? c->err.c_str() : "no context"; }

int gmc_load_tables(gmc_context* c, const gmc_material* mats, int n_mat, const gmc_physics* phys,
                    int32_t* tables_id) {
  if (!c) return GMC_EINVAL;
  if (!mats || !phys || !tables_id || n_mat < 1 || n_mat > kMaxMat)
    return fail(c, GMC_EINVAL, "need 1..8 materials, physics and an id pointer");
  for (int m = 0; m < n_mat; ++m)
    if (!(mats[m].z_over_a > 0 && mats[m].z_eff >= 1.0 && mats[m].i_ev > 0))
      return fail(c, GMC_EINVAL, "material " + std::to_string(m) + " has a non-positive Z/A, Z or I");
  if (!(phys->ecut_mev >= 2 * kEmin && phys->ecut_mev < 30.0 && phys->pcut_mev >= kEmin && phys->pcut_mev < 30.0))
    return fail(c, GMC_EINVAL, "cutoffs must lie in [0.002, 30) MeV (electrons) and [0.001, 30) MeV (photons)");
  if (phys->test_mode < 0 || phys->test_mode > 2) return fail(c, GMC_EINVAL, "test_mode must be 0, 1 or 2");
  if (phys->n_batches > kMaxBatches) return fail(c, GMC_EINVAL, "n_batches must be <= 1024");
  (void)hipSetDevice(c->device);
  auto t = std::make_unique<TablesObj>();
  t->phys = *phys;
  if (t->phys.n_batches <= 0) t->phys.n_batches = 32;
  t->kcut = phys->kcut_mev > 0 ? phys->kcut_mev : phys->ecut_mev;
  t->kc = phys->kc_mev > 0 ? phys->kc_mev : phys->pcut_mev;
  if (!(t->kcut >= kEmin && t->kc >= kEmin)) return fail(c, GMC_EINVAL, "kcut and kc must be >= 0.001 MeV");
  build_tables(mats, n_mat, t->kcut, t->kc, &t->host);
  const size_t nb = (size_t)n_mat * kNE * sizeof(float4);
  HIP_TRY(c, hipMalloc(&t->d_ph, nb));
  HIP_TRY(c, hipMalloc(&t->d_el, nb));
  HIP_TRY(c, hipMalloc(&t->d_ms, kNms * sizeof(float)));
  HIP_TRY(c, hipMemcpy(t->d_ph, t->host.ph.data(), nb, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(t->d_el, t->host.el.data(), nb, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(t->d_ms, t->host.ms.data(), kNms * sizeof(float), hipMemcpyHostToDevice));
  const int32_t id = c->next_id++;
  c->tables[id] = std::move(t);
  *tables_id = id;
  return GMC_OK;
}

int gmc_load_phantom(gmc_context* c, int nx, int ny, int nz, double dx, double dy, double dz,
                     const float* density, const uint8_t* material, int ptr_kind, int32_t* phantom_id) {
  if (!c) return GMC_EINVAL;
  if (!density || !material || !phantom_id) return fail(c, GMC_EINVAL, "NULL phantom array or id pointer");
  if (nx <= 0 || ny <= 0 || nz <= 0 || (double)nx * ny * nz > 2147483647.0)
    return fail(c, GMC_EINVAL, "grid must be positive with fewer than 2^31 voxels");
  if (!(dx > 0 && dy > 0 && dz > 0 && std::isfinite(dx) && std::isfinite(dy) && std::isfinite(dz)))
    return fail(c, GMC_EINVAL, "voxel sizes must be positive");
  if (ptr_kind != GMC_HOST && ptr_kind != GMC_DEVICE) return fail(c, GMC_EINVAL, "bad ptr_kind");
  (void)hipSetDevice(c->device);
  const size_t nv = (size_t)nx * ny * nz;
  std::vector<float> rho(nv);
  std::vector<uint8_t> mat(nv);
  if (ptr_kind == GMC_HOST) {
    std::memcpy(rho.data(), density, nv * sizeof(float));
    std::memcpy(mat.data(), material, nv);
  } else {
    HIP_TRY(c, hipMemcpy(rho.data(), density, nv * sizeof(float), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(mat.data(), material, nv, hipMemcpyDeviceToHost));
  }
  auto p = std::make_unique<PhantomObj>();
  p->nx = nx; p->ny = ny; p->nz = nz; p->dx = dx; p->dy = dy; p->dz = dz;
  p->rho_max.assign(256, 0.0);
  std::vector<uint2> vox(nv);
  for (size_t v = 0; v < nv; ++v) {
    const float r = rho[v];
    if (!(r >= 0.0f) || !std::isfinite(r)) return fail(c, GMC_EINVAL, "densities must be finite and >= 0");
    const int m = mat[v];
    p->rho_max[m] = std::max(p->rho_max[m], (double)r);
    p->max_mat = std::max(p->max_mat, m);
    uint32_t bits;
    std::memcpy(&bits, &r, 4);
    vox[v] = uint2{bits, (uint32_t)m};
  }
  HIP_TRY(c, hipMalloc(&p->d_vox, nv * sizeof(uint2)));
  HIP_TRY(c, hipMemcpy(p->d_vox, vox.data(), nv * sizeof(uint2), hipMemcpyHostToDevice));
  const int32_t id = c->next_id++;
  c->phantoms[id] = std::move(p);
  *phantom_id = id;
  return GMC_OK;
}

int gmc_release(gmc_context* c, int32_t id) {
  if (!c) return GMC_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  auto drop_maj = [&](bool by_phantom) {
    for (auto it = c->majorants.begin(); it != c->majorants.end();) {
      if ((by_phantom ? it->first.first : it->first.second) == id) {
        (void)hipFree(it->second.d_g);
        (void)hipFree(it->second.d_e);
        it = c->majorants.erase(it);
      } else {
        ++it;
      }
    }
  };
  auto t = c->tables.find(id);
  if (t != c->tables.end()) {
    (void)hipFree(t->second->d_ph);
    (void)hipFree(t->second->d_el);
    (void)hipFree(t->second->d_ms);
    c->tables.erase(t);
    drop_maj(false);
    return GMC_OK;
  }
  auto p = c->phantoms.find(id);
  if (p != c->phantoms.end()) {
    (void)hipFree(p->second->d_vox);
    c->phantoms.erase(p);
    drop_maj(true);
    return GMC_OK;
  }
  return fail(c, GMC_ENOTFOUND, "unknown id " + std::to_string(id));
}

int gmc_run_beam(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* src, uint64_t n_hist,
                 uint64_t seed, double* dose, double* sigma, int out_kind, const gmc_tuning* tuning,
                 gmc_run_stats* stats) {
  if (!c) return GMC_EINVAL;
  if (!src) return fail(c, GMC_EINVAL, "source is NULL");
  return run_job(c, phantom_id, tables_id, src, &n_hist, 1, seed, nullptr, nullptr, dose, sigma, out_kind, tuning,
                 stats, false);
}

int gmc_run_beams(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs,
                  const uint64_t* n_hist, int n_beams, uint64_t seed, double* const* dose_per_beam,
                  double* const* sigma_per_beam, double* combined_dose, double* combined_sigma, int out_kind,
                  const gmc_tuning* tuning, gmc_run_stats* stats) {
  if (!c) return GMC_EINVAL;
  gmc_tuning tuned;
  if (!tuning && srcs && n_hist && n_beams >= 1) {
    const int rc = autotune(c, phantom_id, tables_id, srcs, n_hist, n_beams, kAutotuneBudgetS, &tuned, nullptr);
    if (rc) return rc;
    tuning = &tuned;
  }
  return run_job(c, phantom_id, tables_id, srcs, n_hist, n_beams, seed, dose_per_beam, sigma_per_beam, combined_dose,
                 combined_sigma, out_kind, tuning, stats, true);
}

int gmc_autotune(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs,
                 const uint64_t* n_hist, int n_beams, double budget_s, gmc_tuning* out, gmc_autotune_report* report) {
  if (!c) return GMC_EINVAL;
  for (int b = 0; srcs && b < n_beams; ++b) {
    const int rc = check_source(c, &srcs[b]);
    if (rc) return rc;
  }
  return autotune(c, phantom_id, tables_id, srcs, n_hist, n_beams, budget_s > 0 ? budget_s : kAutotuneBudgetS, out,
                  report);
}

int gmc_rng_words(gmc_context* c, uint64_t seed, uint32_t beam, uint32_t hist, uint64_t path, uint32_t n0, int count,
                  uint32_t* out) {
  if (!c) return GMC_EINVAL;
  if (!out || count < 0) return fail(c, GMC_EINVAL, "bad output");
  if (count == 0) return GMC_OK;
  (void)hipSetDevice(c->device);
  uint32_t* d = nullptr;
  HIP_TRY(c, hipMalloc(&d, count * sizeof(uint32_t)));
  hipError_t e = launch_rng_words((uint32_t)seed, (uint32_t)(seed >> 32) ^ beam, hist, (uint32_t)path,
                                  (uint32_t)(path >> 32), n0, count, d, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d, count * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(c, GMC_EDEVICE, hipGetErrorString(e));
  return GMC_OK;
}

int gmc_table_eval(gmc_context* c, int32_t tables_id, int which, int mat, const double* energies, int n,
                   double* out) {
  if (!c) return GMC_EINVAL;
  auto ti = c->tables.find(tables_id);
  if (ti == c->tables.end()) return fail(c, GMC_ENOTFOUND, "unknown tables id");
  if (which < 0 || which > 7 || mat < 0 || mat >= ti->second->host.n_mat || n < 0 || (n && (!energies || !out)))
    return fail(c, GMC_EINVAL, "bad table query");
  if (n == 0) return GMC_OK;
  (void)hipSetDevice(c->device);
  std::vector<float> ef(n), of(n);
  for (int i = 0; i < n; ++i) ef[i] = (float)energies[i];
  float *de = nullptr, *dout = nullptr;
  HIP_TRY(c, hipMalloc(&de, n * sizeof(float)));
  HIP_TRY(c, hipMalloc(&dout, n * sizeof(float)));
  const MajObj none;
  const DevTables t = dev_tables(*ti->second, none);
  hipError_t e = hipMemcpyAsync(de, ef.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_table_eval(t, which, mat, de, n, dout, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(of.data(), dout, n * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(de);
  (void)hipFree(dout);
  if (e != hipSuccess) return fail(c, GMC_EDEVICE, hipGetErrorString(e));
  for (int i = 0; i < n; ++i) out[i] = of[i];
  return GMC_OK;
}

int gmc_first_events(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* src, uint64_t seed,
                     uint32_t h_begin, uint32_t h_end, float* out_xyz, uint32_t* out_nused) {
  if (!c) return GMC_EINVAL;
  auto pi = c->phantoms.find(phantom_id);
  auto ti = c->tables.find(tables_id);
  if (pi == c->phantoms.end() || ti == c->tables.end()) return fail(c, GMC_ENOTFOUND, "unknown phantom or tables id");
  int rc = check_source(c, src);
  if (rc) return rc;
  if (src->particle != GMC_PHOTON) return fail(c, GMC_EINVAL, "first events are defined for photon beams");
  if (h_end < h_begin || !out_xyz || !out_nused) return fail(c, GMC_EINVAL, "bad history range or outputs");
  const PhantomObj& P = *pi->second;
  const TablesObj& T = *ti->second;
  if (P.max_mat >= T.host.n_mat) return fail(c, GMC_EINVAL, "phantom uses a material index beyond the tables");
  const uint32_t n = h_end - h_begin;
  if (n == 0) return GMC_OK;
  (void)hipSetDevice(c->device);
  MajObj maj;
  rc = get_majorants(c, phantom_id, tables_id, P, T, &maj);
  if (rc) return rc;
  rc = ensure_beams(c, 1);
  if (rc) return rc;
  DevBeam beam{};
  beam.key0 = (uint32_t)seed;
  beam.key1 = (uint32_t)(seed >> 32) ^ src->beam_id;
  beam.a = DevTally{nullptr, 1u, 0u};
  beam.b = DevTally{nullptr, 1u, 0u};
  PassArgs a{};
  a.ph = dev_phantom(P);
  a.tab = dev_tables(T, maj);
  a.cut = dev_cuts(T);
  a.beams = c->d_beams;
  const DevSource ds = dev_source(*src);
  float* dx = nullptr;
  uint32_t* dn = nullptr;
  HIP_TRY(c, hipMemcpy(c->d_beams, &beam, sizeof(beam), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMalloc(&dx, (size_t)n * 3 * sizeof(float)));
  hipError_t e = hipMalloc(&dn, (size_t)n * sizeof(uint32_t));
  if (e == hipSuccess) e = launch_first_events(a, ds, h_begin, n, dx, dn, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_xyz, dx, (size_t)n * 3 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out_nused, dn, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(dx);
  if (dn) (void)hipFree(dn);
  if (e != hipSuccess) return fail(c, GMC_EDEVICE, hipGetErrorString(e));
  return GMC_OK;
}

}  // extern "C"
