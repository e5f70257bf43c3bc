// gmc_engine.cpp -- the transport engine on the host side: workspaces, job
// construction, the rounds of [admit primaries -> electron pass -> photon
// pass] (each pass appending its outputs to the queues; Sec. II.C.2: photons and
// electrons are simulated in alternating passes; the leftover threshold is
// zero, so no particle is ever dropped), the finalize (Sec. II.D), the
// blocking plain and batched forms and the autotuner.
//
// Pass sizes are planned on the device from device-resident counts, so a
// round needs no host read.  The plain form reads the control block after
// admission and after the electron pass of every round and skips empty
// passes; the batched form captures several rounds in a HIP graph and
// replays it, reading the control block once per replay.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "gmc_host.hpp"

namespace gmc {

int wfail(Workspace* w, int code, const std::string& msg) {
  if (w) w->err = msg;
  return code;
}

int cfail(gmc_context* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

// ---------------------------------------------------------------- workspace
namespace {

void free_queue(QueueBuf& b) {
  if (b.base) (void)hipFree(b.base);
  b = QueueBuf{};
}

hipError_t alloc_queue(QueueBuf& b, uint32_t cap, int fields) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, (size_t)fields * cap * sizeof(uint32_t));
  if (e != hipSuccess) return e;
  b.base = p;
  b.q.base = static_cast<uint32_t*>(p);
  b.q.stride = cap;
  b.q.cap = cap;
  return hipSuccess;
}

int ensure_queues(Workspace* w, uint32_t cap) {
  if (w->cap >= cap) return GMC_OK;
  for (auto& t : w->qbuf)
    for (auto& b : t) free_queue(b);
  w->cap = 0;
  for (auto& t : w->qbuf)
    for (auto& b : t) WS_TRY(w, alloc_queue(b, cap, Q_FIELDS));
  w->cap = cap;
  return GMC_OK;
}

// The regrouping buffer (one pass's items) and the sort's counters, which
// start at zero.
int ensure_sorted(Workspace* w, uint32_t cap) {
  if (!w->d_sort) WS_TRY(w, hipMalloc(&w->d_sort, 2 * kSortBuckets * sizeof(uint32_t)));
  WS_TRY(w, hipMemsetAsync(w->d_sort, 0, 2 * kSortBuckets * sizeof(uint32_t), w->stream));
  if (w->sorted_cap >= cap) return GMC_OK;
  free_queue(w->sorted);
  w->sorted_cap = 0;
  WS_TRY(w, alloc_queue(w->sorted, cap, Q_FIELDS));
  w->sorted_cap = cap;
  return GMC_OK;
}

int ensure_staging(Workspace* w, uint32_t slots) {
  if (w->stg_cap >= slots) return GMC_OK;
  if ((uint64_t)slots * kStgFields >= (1ull << 32)) return wfail(w, GMC_EOVERFLOW, "staging queue too large");
  for (auto& b : w->stg) free_queue(b);
  w->stg_cap = 0;
  for (auto& b : w->stg) WS_TRY(w, alloc_queue(b, slots, kStgFields));
  w->stg_cap = slots;
  return GMC_OK;
}

// Events that only time the pass kernels: without the system-scope fence an
// event record does not wait for the caches to be written back, which would
// add several microseconds between the kernels it separates.
hipError_t create_timing_event(hipEvent_t* e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

int ensure_graph_events(Workspace* w, size_t n) {
  while (w->gev.size() < n) {
    hipEvent_t e = nullptr;
    WS_TRY(w, create_timing_event(&e));
    w->gev.push_back(e);
  }
  return GMC_OK;
}

int resident_blocks(Workspace* w, int kernel, int block, int n_mat) {
  const std::vector<int> key{kernel, block, n_mat};
  auto it = w->resident.find(key);
  if (it != w->resident.end()) return it->second;
  const size_t lds = kernel == 0 ? photon_lds_bytes(n_mat)
                     : kernel == 1 ? electron_lds_bytes(n_mat) : round_lds_bytes(n_mat);
  const int r = max_resident_blocks(kernel, block, lds);
  w->resident[key] = r;
  return r;
}

}  // namespace

uint32_t pass_waves(Workspace* w, int kernel, int block, int n_mat) {
  const uint32_t wpb = (uint32_t)block / 64u;
  const uint32_t res = (uint32_t)resident_blocks(w, kernel, block, n_mat);
  return std::max<uint32_t>(1u, std::min<uint32_t>(res, kMaxWaves / wpb)) * wpb;
}

int pass_block(Workspace* w, int kernel, int requested, int n_mat) {
  if (requested > 0) return kernel == 2 ? std::min(requested, kRoundMaxBlock) : requested;
  int best = 256;
  uint32_t best_waves = 0;
  for (int b : {256, 512, 1024}) {
    if (kernel == 2 && b > kRoundMaxBlock) continue;
    const uint32_t waves = pass_waves(w, kernel, b, n_mat);
    if (waves > best_waves) {
      best_waves = waves;
      best = b;
    }
  }
  return best;
}

int ws_init(Workspace* w, int device, hipStream_t stream) {
  w->device = device;
  if (stream) {
    w->stream = stream;
  } else {
    WS_TRY(w, hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    w->own_stream = true;
  }
  WS_TRY(w, hipMalloc(&w->d_ctl, sizeof(Control)));
  WS_TRY(w, hipHostMalloc(&w->h_ctl, sizeof(Control), hipHostMallocDefault));
  WS_TRY(w, hipMalloc(&w->d_ctr, C_COUNT * kCtrSlots * sizeof(unsigned long long)));
  WS_TRY(w, hipHostMalloc(&w->h_ctr, C_COUNT * kCtrSlots * sizeof(unsigned long long), hipHostMallocDefault));
  WS_TRY(w, hipMalloc(&w->d_claim, 2 * kMaxClaimParts * sizeof(uint32_t)));
  WS_TRY(w, hipMalloc(&w->d_nk, kMaxBatches * sizeof(double)));
  WS_TRY(w, hipMalloc(&w->d_srel, (3 * kRelBlocks + 1) * sizeof(double)));
  WS_TRY(w, hipHostMalloc(&w->h_srel, sizeof(double), hipHostMallocDefault));
  WS_TRY(w, hipHostMalloc(&w->h_nk, kMaxBatches * sizeof(double), hipHostMallocDefault));
  WS_TRY(w, hipEventCreate(&w->ev0));
  WS_TRY(w, hipEventCreate(&w->ev1));
  WS_TRY(w, create_timing_event(&w->kev0));
  WS_TRY(w, create_timing_event(&w->kev1));
  WS_TRY(w, hipEventCreateWithFlags(&w->ev_ctl, hipEventDisableTiming));
  return GMC_OK;
}

void ws_trim(Workspace* w) {
  if (w->stream) (void)hipStreamSynchronize(w->stream);
  if (w->d_tally) (void)hipFree(w->d_tally);
  if (w->d_dose) (void)hipFree(w->d_dose);
  if (w->d_sigma) (void)hipFree(w->d_sigma);
  w->d_tally = nullptr;
  w->d_dose = w->d_sigma = nullptr;
  w->tally_elems = w->out_elems = 0;
}

void ws_free(Workspace* w) {
  if (w->stream) (void)hipStreamSynchronize(w->stream);
  ws_trim(w);
  for (auto& t : w->qbuf)
    for (auto& b : t) free_queue(b);
  for (auto& b : w->stg) free_queue(b);
  free_queue(w->sorted);
  w->cap = w->stg_cap = w->sorted_cap = 0;
  for (void* p : {(void*)w->d_ctl, (void*)w->d_ctr, (void*)w->d_beams, (void*)w->d_sort, (void*)w->d_tab,
                  (void*)w->d_sources, (void*)w->d_start, (void*)w->d_beam_of, (void*)w->d_seg_h, (void*)w->d_nk,
                  (void*)w->d_claim, (void*)w->d_fin, (void*)w->d_fin_nk})
    if (p) (void)hipFree(p);
  w->d_fin = nullptr;
  w->d_fin_nk = nullptr;
  w->fin_cap = w->fin_nk_cap = 0;
  for (void* p : {(void*)w->h_ctl, (void*)w->h_ctr, (void*)w->h_nk, (void*)w->h_srel})
    if (p) (void)hipHostFree(p);
  w->d_ctl = nullptr;
  w->h_ctl = nullptr;
  w->d_ctr = w->h_ctr = nullptr;
  w->d_beams = nullptr;
  w->d_sources = nullptr;
  w->d_start = w->d_beam_of = w->d_seg_h = nullptr;
  w->seg_cap = 0;
  w->d_sort = nullptr;
  w->d_tab = nullptr;
  w->tab_cap = 0;
  if (w->d_srel) (void)hipFree(w->d_srel);
  w->d_srel = nullptr;
  w->h_srel = nullptr;
  w->d_nk = w->h_nk = nullptr;
  w->d_claim = nullptr;
  w->beams_cap = 0;
  for (hipEvent_t e : {w->ev0, w->ev1, w->kev0, w->kev1, w->ev_ctl})
    if (e) (void)hipEventDestroy(e);
  w->ev0 = w->ev1 = w->kev0 = w->kev1 = w->ev_ctl = nullptr;
  for (hipEvent_t e : w->gev) (void)hipEventDestroy(e);
  w->gev.clear();
  if (w->own_stream && w->stream) (void)hipStreamDestroy(w->stream);
  w->stream = nullptr;
  w->own_stream = false;
}

size_t ws_device_bytes(const Workspace& w) {
  return sizeof(uint32_t) * ((size_t)Q_FIELDS * (4ull * w.cap + w.sorted_cap) + (size_t)kStgFields * 2ull * w.stg_cap) +
         w.tally_elems * sizeof(unsigned long long) + 2 * w.out_elems * sizeof(double) +
         w.beams_cap * (sizeof(DevBeam) + sizeof(DevSource)) + w.seg_cap * 6 * sizeof(uint32_t) +
         w.tab_cap * sizeof(double);
}

int ws_ensure_tally(Workspace* w, size_t elems) {
  if (w->tally_elems >= elems) return GMC_OK;
  if (w->d_tally) (void)hipFree(w->d_tally);
  w->d_tally = nullptr;
  w->tally_elems = 0;
  WS_TRY(w, hipMalloc(&w->d_tally, elems * sizeof(unsigned long long)));
  w->tally_elems = elems;
  return GMC_OK;
}

int ws_ensure_out(Workspace* w, size_t elems) {
  if (w->out_elems >= elems) return GMC_OK;
  if (w->d_dose) (void)hipFree(w->d_dose);
  if (w->d_sigma) (void)hipFree(w->d_sigma);
  w->d_dose = w->d_sigma = nullptr;
  w->out_elems = 0;
  WS_TRY(w, hipMalloc(&w->d_dose, elems * sizeof(double)));
  WS_TRY(w, hipMalloc(&w->d_sigma, elems * sizeof(double)));
  w->out_elems = elems;
  return GMC_OK;
}

int ws_ensure_beams(Workspace* w, size_t n) {
  if (w->beams_cap >= n) return GMC_OK;
  for (void* p : {(void*)w->d_beams, (void*)w->d_sources})
    if (p) (void)hipFree(p);
  w->d_beams = nullptr;
  w->d_sources = nullptr;
  w->beams_cap = 0;
  WS_TRY(w, hipMalloc(&w->d_beams, n * sizeof(DevBeam)));
  WS_TRY(w, hipMalloc(&w->d_sources, n * sizeof(DevSource)));
  w->beams_cap = n;
  return GMC_OK;
}

int ws_ensure_fin(Workspace* w, size_t n, size_t nk) {
  if (w->fin_cap < n) {
    if (w->d_fin) (void)hipFree(w->d_fin);
    w->d_fin = nullptr;
    w->fin_cap = 0;
    WS_TRY(w, hipMalloc(&w->d_fin, n * sizeof(FinalizeArgs)));
    w->fin_cap = n;
  }
  if (w->fin_nk_cap < nk) {
    if (w->d_fin_nk) (void)hipFree(w->d_fin_nk);
    w->d_fin_nk = nullptr;
    w->fin_nk_cap = 0;
    WS_TRY(w, hipMalloc(&w->d_fin_nk, nk * sizeof(double)));
    w->fin_nk_cap = nk;
  }
  return GMC_OK;
}

int ws_ensure_segments(Workspace* w, size_t n) {
  if (w->seg_cap >= n) return GMC_OK;
  for (void* p : {(void*)w->d_start, (void*)w->d_beam_of, (void*)w->d_seg_h})
    if (p) (void)hipFree(p);
  w->d_start = w->d_beam_of = w->d_seg_h = nullptr;
  w->seg_cap = 0;
  WS_TRY(w, hipMalloc(&w->d_start, 2 * (n + 1) * sizeof(uint32_t)));
  WS_TRY(w, hipMalloc(&w->d_beam_of, 2 * n * sizeof(uint32_t)));
  WS_TRY(w, hipMalloc(&w->d_seg_h, 2 * n * sizeof(uint32_t)));
  w->seg_cap = n;
  return GMC_OK;
}

// ---------------------------------------------------------------- settings
Tune resolve_tuning(const gmc_tuning* t) {
  Tune r{64, 4, 1 << 22, 0, 1 << 23, 64, 4, 4, 0, 32, 64, 0, 0, 0};
  if (t) {
    // an electron parked at a hard event keeps its visit's event count in 16 bits
    if (t->events_per_visit > 0) r.events = std::min(t->events_per_visit, 1 << 15);
    if (t->secondaries_per_visit >= 2) r.secondaries = std::min(t->secondaries_per_visit, 64);
    if (t->chunk > 0) r.chunk = std::min(t->chunk, 1 << 24);
    if (t->wg_size >= 64 && t->wg_size <= 1024 && t->wg_size % 64 == 0) r.block = t->wg_size;
    if (t->pass_items > 0) r.pass_items = std::min(std::max(t->pass_items, 1024), 1 << 23);
    if (t->wave_items > 0) {
      // a power of two in [64, 1024]
      int c = 64;
      while (c * 2 <= std::min(t->wave_items, 1024)) c *= 2;
      r.wave_items = c;
    }
    if (t->rounds_per_check > 0) r.rounds = std::min(t->rounds_per_check, 1024);
    if (t->refill_lanes > 0) r.refill = std::min(t->refill_lanes, 64);
    if (t->energy_sort > 0) r.sort = 1;
    if (t->tail_lanes < 0) r.tail_g = r.tail_e = 0;
    if (t->tail_lanes > 0) r.tail_g = r.tail_e = std::min(t->tail_lanes, 64);
    if (t->queue_items > 0) r.queue = (int)std::min<uint32_t>(std::max(t->queue_items, 64), kMaxSoftCap);
    if (t->persistent > 0) r.persistent = 1;
    r.aggregate = t->aggregate > 0 ? 1 : (t->aggregate < 0 ? -1 : 0);
  }
  return r;
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
  t.energy_sort = d.sort;
  t.tail_lanes = 0;   // the per-pass defaults
  t.queue_items = 0;
  t.persistent = d.persistent;
  t.aggregate = d.aggregate;
  return t;
}

// Queue capacity.  Soft: what admission and the outputs of the other type
// may fill -- eight admission chunks, at least 2^23 and at most 2^25
// particles.  Allocated: the soft capacity plus a full pass of this type's
// own per-visit outputs, so a pass is never shrunk by its own backlog (a
// type whose pass could only take a sliver of its queue would fall behind
// the other type feeding it).  Staging: every wavefront of the pass grid
// gets segments for its largest share of a pass times the per-visit budget.
void queue_sizes(Workspace* w, const Tune& tu, int n_mat, uint32_t* cap, uint32_t* cap_soft, uint32_t* stg) {
  const uint64_t soft = tu.queue > 0 ? (uint64_t)tu.queue
                                     : std::max<uint64_t>(kMinSoftCap, std::min<uint64_t>(8ull * (uint64_t)tu.chunk,
                                                                                          kMaxSoftCap));
  *cap_soft = (uint32_t)soft;
  *cap = (uint32_t)(soft + (uint64_t)tu.secondaries * (uint64_t)tu.pass_items);
  uint32_t s = 0;
  for (int t = 0; t < 2; ++t) {
    // largest segment per particle: photon pass, its electrons (or survivor
    // + one parked entry); electron pass, survivor + secondaries + one
    // parked entry
    const uint32_t bud = t == 0 ? std::max<uint32_t>((uint32_t)tu.secondaries, 2u) : (uint32_t)tu.secondaries + 2u;
    const uint32_t waves = pass_waves(w, t, pass_block(w, t, tu.block, n_mat), n_mat);
    // items go to wavefronts in chunks of wave_items
    const uint32_t cs = (uint32_t)tu.wave_items;
    const uint32_t chunks = ((uint32_t)tu.pass_items + cs - 1u) / cs;
    const uint32_t qmax = (chunks + waves - 1) / waves * cs;
    s = std::max<uint32_t>(s, waves * qmax * bud);
  }
  if (uses_round(tu, n_mat)) {
    // round kernel: per wavefront an electron segment (electron phase
    // survivors, secondaries and parked stack, photon phase electrons) and
    // a photon segment (bremsstrahlung, photon survivors and parked stack),
    // for claim caps of an even share of chunks plus one
    const uint32_t waves = pass_waves(w, 2, pass_block(w, 2, tu.block, n_mat), n_mat);
    const uint64_t cs = (uint64_t)tu.wave_items;
    const uint64_t cap = (((uint64_t)tu.pass_items + cs - 1u) / cs + waves - 1u) / waves * cs + cs;
    const uint64_t sec = (uint64_t)tu.secondaries;
    const uint64_t seg = std::max(cap * (sec + 2u) + cap * sec, cap * sec + 2u * cap);
    // beyond 32-bit slot indices the staging check refuses the job (GMC_EOVERFLOW)
    s = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(s, (uint64_t)waves * seg), 0xFFFFFFFFull);
  }
  *stg = s;
}

bool uses_round(const Tune& tu, int n_mat) { return tu.persistent > 0 && n_mat <= kMaxRoundMat; }

int check_source(std::string* err, const gmc_source* s) {
  auto bad = [&](const char* m) {
    *err = m;
    return GMC_EINVAL;
  };
  if (!s) return bad("source is NULL");
  if (s->particle != GMC_PHOTON && s->particle != GMC_ELECTRON) return bad("bad particle type");
  if (s->spectrum == GMC_MONO) {
    if (!(s->e_mev > 0.0 && s->e_mev <= 30.0)) return bad("energy must be in (0, 30] MeV");
  } else if (s->spectrum == GMC_TRIANGULAR) {
    if (!(s->e_lo > 0.0 && s->e_lo <= s->e_mode && s->e_mode <= s->e_hi && s->e_lo < s->e_hi && s->e_hi <= 30.0))
      return bad("triangular spectrum needs 0 < lo <= mode <= hi <= 30, lo < hi");
  } else if (s->spectrum == GMC_TABULATED) {
    if (!s->tab_e || !s->tab_w || s->tab_n < 1 || s->tab_n > 4096)
      return bad("tabulated spectrum needs 1..4096 bins and both tables");
    if (!(s->tab_e[0] > 0.0 && s->tab_e[s->tab_n] <= 30.0)) return bad("tabulated spectrum must lie in (0, 30] MeV");
    double total = 0.0;
    for (int j = 0; j < s->tab_n; ++j) {
      if (!(s->tab_e[j + 1] > s->tab_e[j])) return bad("tabulated spectrum edges must increase");
      if (!(s->tab_w[j] >= 0.0 && std::isfinite(s->tab_w[j]))) return bad("tabulated spectrum weights must be >= 0");
      total += s->tab_w[j];
    }
    if (!(total > 0.0 && std::isfinite(total))) return bad("tabulated spectrum weights sum to zero");
  } else {
    return bad("bad spectrum kind");
  }
  if (!(std::isfinite(s->cx_cm) && std::isfinite(s->cy_cm) && s->wx_cm >= 0.0 && s->wy_cm >= 0.0 &&
        std::isfinite(s->wx_cm) && std::isfinite(s->wy_cm)))
    return bad("bad field geometry");
  return GMC_OK;
}

uint32_t mev_to_lsb(double e) { return (uint32_t)std::llround(e * 134217728.0); }

double source_emax(const gmc_source& s) {
  if (s.spectrum == GMC_TRIANGULAR) return s.e_hi;
  if (s.spectrum == GMC_TABULATED) return s.tab_e[s.tab_n];
  return s.e_mev;
}

double source_emean(const gmc_source& s) {
  if (s.spectrum == GMC_TRIANGULAR) return (s.e_lo + s.e_mode + s.e_hi) / 3.0;
  if (s.spectrum == GMC_TABULATED) {
    double m = 0.0, w = 0.0;
    for (int j = 0; j < s.tab_n; ++j) {
      m += s.tab_w[j] * 0.5 * (s.tab_e[j] + s.tab_e[j + 1]);
      w += s.tab_w[j];
    }
    return m / w;
  }
  return s.e_mev;
}

// The normalised CDF is summed left to right and divided by the total, with
// C_n set to exactly 1, so that a uniform below 1 always finds a bin.
void tabulated_cdf(const gmc_source& s, std::vector<double>* out) {
  const int n = s.tab_n;
  double total = 0.0;
  for (int j = 0; j < n; ++j) total += s.tab_w[j];
  out->insert(out->end(), s.tab_e, s.tab_e + n + 1);
  double sum = 0.0;
  out->push_back(0.0);
  for (int j = 0; j < n; ++j) {
    sum += s.tab_w[j];
    out->push_back(j == n - 1 ? 1.0 : sum / total);
  }
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
  d.tab = nullptr;   // set where the job's tables are uploaded
  d.tab_n = s.spectrum == GMC_TABULATED ? (uint32_t)s.tab_n : 0u;
  d.h0 = (uint32_t)s.first_history;
  return d;
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

int get_majorants(gmc_context* c, int32_t pid, int32_t tid, const PhantomObj& p, const TablesObj& t, MajObj* out,
                  std::string* err) {
  std::lock_guard<std::mutex> lk(c->mu);
  auto key = std::make_pair(pid, tid);
  auto it = c->majorants.find(key);
  if (it != c->majorants.end()) {
    *out = it->second;
    return GMC_OK;
  }
  std::vector<float> g(kNE), e(kNE);
  build_majorants(t.host, p.rho_max.data(), t.margin, g.data(), e.data());
  MajObj m;
  hipError_t he = hipMalloc(&m.d_g, kNE * sizeof(float));
  if (he == hipSuccess) he = hipMalloc(&m.d_e, kNE * sizeof(float));
  if (he == hipSuccess) he = hipMemcpy(m.d_g, g.data(), kNE * sizeof(float), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(m.d_e, e.data(), kNE * sizeof(float), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    if (m.d_g) (void)hipFree(m.d_g);
    if (m.d_e) (void)hipFree(m.d_e);
    *err = std::string("majorant upload: ") + hipGetErrorString(he);
    return he == hipErrorOutOfMemory ? GMC_ENOMEM : GMC_EDEVICE;
  }
  c->majorants[key] = m;
  *out = m;
  return GMC_OK;
}

// ---------------------------------------------------------------------- jobs
size_t job_tally_elems(TallyMode mode, size_t nvox, uint32_t K, size_t n_beams) {
  const size_t nvp = tally_vox(nvox);
  return mode == kCombined ? nvp * K : mode == kBeamBatched ? nvp * K * n_beams : nvp * (K + n_beams);
}

void build_job(Job* J, Workspace* w, const PhantomObj& P, const TablesObj& T, const MajObj& maj,
               const gmc_source* srcs, const uint64_t* n_hist, int n_beams, uint64_t seed, TallyMode mode) {
  const size_t nvp = tally_vox(P.nvox());   // voxels of a tally target, padded to whole blocks
  const uint32_t K = (uint32_t)T.phys.n_batches;
  J->P = &P;
  J->T = &T;
  J->maj = maj;
  for (int t = 0; t < 2; ++t) {
    J->start[t].assign(1, 0u);
    J->beam_of[t].clear();
    J->seg_h[t].clear();
  }
  uint32_t off = 0;
  uint64_t per_type[2] = {0, 0};
  std::vector<int> of_type[2];
  for (int b = 0; b < n_beams; ++b) {
    DevBeam db{};
    db.key0 = (uint32_t)seed;
    db.key1 = (uint32_t)(seed >> 32) ^ srcs[b].beam_id;
    db.b = DevTally{nullptr, 1u, 0u};
    if (mode == kCombined) {
      db.a = DevTally{w->d_tally, K, off % K};
    } else if (mode == kBeamBatched) {
      db.a = DevTally{w->d_tally + nvp * K * (size_t)b, K, 0u};
    } else {
      db.a = DevTally{w->d_tally + nvp * ((size_t)K + (size_t)b), 1u, 0u};
      db.b = DevTally{w->d_tally, K, off % K};
    }
    J->beams.push_back(db);
    J->sources.push_back(dev_source(srcs[b]));
    J->tab_off.push_back(J->tab.size());
    if (srcs[b].spectrum == GMC_TABULATED) tabulated_cdf(srcs[b], &J->tab);
    const int t = srcs[b].particle;
    of_type[t].push_back(b);
    per_type[t] += n_hist[b];
    off += (uint32_t)n_hist[b];
  }
  // Admission order.  A beam's histories admitted as one block would put
  // nearly every particle in flight on that beam, and its own tally (one
  // slice when per-beam doses are kept beside the combined ones) would take
  // all their additions on the few voxels of its axis.  So each type's beams
  // are cut into segments of at least kAdmitSegment histories, ordered by the
  // fraction of its beam a segment's middle lies at: every beam is admitted
  // in proportion and the particles in flight spread over all of them.  Only
  // the order of admission changes; a history's number, stream and batch do
  // not, so neither does any result.
  for (int t = 0; t < 2; ++t) {
    struct Piece {
      double key;
      uint32_t beam, h, n;
    };
    std::vector<Piece> pieces;
    const uint64_t seg = of_type[t].size() <= 1
                             ? std::numeric_limits<uint32_t>::max()
                             : std::max<uint64_t>(kAdmitSegment, (per_type[t] + kMaxAdmitSegments - 1) / kMaxAdmitSegments);
    for (int b : of_type[t]) {
      const uint64_t n = n_hist[b];
      for (uint64_t h = 0; h < n; h += seg) {
        const uint64_t len = std::min<uint64_t>(seg, n - h);
        pieces.push_back(Piece{((double)h + 0.5 * (double)len) / (double)n, (uint32_t)b, (uint32_t)h, (uint32_t)len});
      }
    }
    std::stable_sort(pieces.begin(), pieces.end(), [](const Piece& x, const Piece& y) { return x.key < y.key; });
    for (const Piece& p : pieces) {
      J->beam_of[t].push_back(p.beam);
      J->seg_h[t].push_back(p.h);
      J->start[t].push_back(J->start[t].back() + p.n);
    }
  }
  J->total[0] = (uint32_t)per_type[0];
  J->total[1] = (uint32_t)per_type[1];
}

// -------------------------------------------------------------------- engine
namespace {

uint32_t* count_ptr(Workspace* w, int type, int buf) { return w->d_ctl->counts + 2 * type + buf; }

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

// Enqueue the plan and the pass of `type` over its accumulating buffer, which
// becomes the work buffer; the other buffer accumulates from then on (the
// pass appends its outputs to it and to the other type's accumulating
// buffer).  The pass kernel is bracketed by the events t0 / t1 (recorded as
// graph event nodes while the stream is being captured).
int enqueue_pass(Engine& E, int type, hipEvent_t t0, hipEvent_t t1, bool capturing) {
  Workspace* w = E.w;
  const int other = 1 - type;
  const int wi = w->acc[type];
  w->acc[type] ^= 1;
  const int ni = w->acc[type];
  PlanArgs pa;
  pa.n_work = count_ptr(w, type, wi);
  pa.n_new = count_ptr(w, type, ni);
  pa.n_other = count_ptr(w, other, w->acc[other]);
  pa.plan = w->d_ctl->plan + type;
  pa.cap = w->cap;
  pa.cap_other = w->cap_soft;
  pa.max_items = (uint32_t)E.tu.pass_items;
  pa.waves = E.waves[type];
  pa.chunk_log2 = 0;
  while ((1u << pa.chunk_log2) < (uint32_t)E.tu.wave_items) ++pa.chunk_log2;
  pa.bud_same = E.bud_same[type];
  pa.bud_other = E.bud_other[type];
  pa.park_slots = 1u;   // one parked entry per particle: electrons at hard events, photons at absorption
  pa.sched = w->d_ctl->sched;
  WS_TRY(w, launch_plan_pass(pa, w->stream));
  PassArgs a = E.proto;
  a.work = w->qbuf[type][wi].q;
  a.carry_src = a.work;
  if (E.tu.sort) {
    // the pass's items, regrouped by energy into the spare buffer; the
    // carry-over stays where it is
    SortArgs sa;
    sa.src = a.work;
    sa.dst = w->sorted.q;
    sa.n = &w->d_ctl->plan[type].m;
    sa.hist = w->d_sort;
    sa.cursor = w->d_sort + kSortBuckets;
    WS_TRY(w, launch_sort(sa, kSortGrid, w->stream));
    a.work = w->sorted.q;
  }
  a.plan = w->d_ctl->plan + type;
  a.stg_same = w->stg[0].q;
  a.stg_other = w->stg[1].q;
  a.dst_same = w->qbuf[type][ni].q;
  a.dst_other = w->qbuf[other][w->acc[other]].q;
  a.cnt_same = count_ptr(w, type, ni);
  a.cnt_other = count_ptr(w, other, w->acc[other]);
  a.tail_lanes = type == 0 ? E.tu.tail_g : E.tu.tail_e;
  a.tail_min = kTailMinItems;
  WS_TRY(w, record_event(w->stream, t0, capturing));
  hipError_t e = type == 0 ? launch_photon_pass(a, (int)E.blocks[0], E.block[0], w->stream)
                           : launch_electron_pass(a, (int)E.blocks[1], E.block[1], w->stream);
  if (e != hipSuccess) return wfail(w, GMC_EDEVICE, std::string("pass launch: ") + hipGetErrorString(e));
  WS_TRY(w, record_event(w->stream, t1, capturing));
  return GMC_OK;
}

// Enqueue the round plan and the persistent round kernel over both types'
// accumulating buffers, which become the work buffers (each type's other
// buffer accumulates from then on), bracketed by t0 / t1.
int enqueue_round(Engine& E, hipEvent_t t0, hipEvent_t t1, bool capturing) {
  Workspace* w = E.w;
  int wi[2], ni[2];
  for (int t = 0; t < 2; ++t) {
    wi[t] = w->acc[t];
    w->acc[t] ^= 1;
    ni[t] = w->acc[t];
  }
  uint32_t lg = 0;
  while ((1u << lg) < (uint32_t)E.tu.wave_items) ++lg;
  RoundPlanArgs pa;
  for (int t = 0; t < 2; ++t) {
    pa.n_work[t] = count_ptr(w, t, wi[t]);
    pa.n_new[t] = count_ptr(w, t, ni[t]);
  }
  pa.plan = w->d_ctl->plan;
  pa.claims = w->d_ctl->claim;
  pa.claim_ctr = w->d_claim;
  pa.cap = w->cap;
  pa.cap_soft = w->cap_soft;
  pa.max_items = (uint32_t)E.tu.pass_items;
  pa.waves = E.round_waves;
  pa.blocks = E.round_blocks;
  pa.chunk_log2 = lg;
  pa.sec = (uint32_t)E.tu.secondaries;
  pa.sched = w->d_ctl->sched;
  WS_TRY(w, launch_plan_round(pa, w->stream));
  RoundArgs r;
  r.g = E.proto;
  r.e = E.proto;
  r.g.work = r.g.carry_src = w->qbuf[0][wi[0]].q;
  r.e.work = r.e.carry_src = w->qbuf[1][wi[1]].q;
  r.g.plan = w->d_ctl->plan + 0;
  r.e.plan = w->d_ctl->plan + 1;
  r.e.stg_same = r.g.stg_other = w->stg[0].q;   // electron outputs
  r.g.stg_same = r.e.stg_other = w->stg[1].q;   // photon outputs
  r.g.dst_same = r.e.dst_other = w->qbuf[0][ni[0]].q;
  r.e.dst_same = r.g.dst_other = w->qbuf[1][ni[1]].q;
  r.g.cnt_same = r.e.cnt_other = count_ptr(w, 0, ni[0]);
  r.e.cnt_same = r.g.cnt_other = count_ptr(w, 1, ni[1]);
  r.g.tail_lanes = E.tu.tail_g;
  r.e.tail_lanes = E.tu.tail_e;
  r.g.tail_min = r.e.tail_min = kTailMinItems;
  r.claims = w->d_ctl->claim;
  r.claim_ctr = w->d_claim;
  WS_TRY(w, record_event(w->stream, t0, capturing));
  const hipError_t e = launch_round(r, (int)E.round_blocks, E.round_block, w->stream);
  if (e != hipSuccess) return wfail(w, GMC_EDEVICE, std::string("round launch: ") + hipGetErrorString(e));
  WS_TRY(w, record_event(w->stream, t1, capturing));
  return GMC_OK;
}

int enqueue_admission(Engine& E) {
  Workspace* w = E.w;
  AdmitPlanArgs ap;
  ap.cursor = w->d_ctl->sched;
  ap.total = w->d_ctl->sched + 2;
  ap.count0 = count_ptr(w, 0, w->acc[0]);
  ap.count1 = count_ptr(w, 1, w->acc[1]);
  ap.out = w->d_ctl->adm;
  ap.cap = w->cap_soft;
  ap.chunk = (uint32_t)E.tu.chunk;
  WS_TRY(w, launch_admit_plan(ap, w->stream));
  for (int t = 0; t < 2; ++t) {
    AdmitArgs a = E.adm[t];
    a.out = w->qbuf[t][w->acc[t]].q;
    WS_TRY(w, launch_admit(a, std::min<uint32_t>((uint32_t)E.tu.chunk, E.total[t]), w->stream));
  }
  return GMC_OK;
}

int check_control(Workspace* w) {
  for (int i = 0; i < 4; ++i)
    if (w->h_ctl->counts[i] > w->cap) return wfail(w, GMC_EINTERNAL, "particle queue overflow on the device");
  return GMC_OK;
}

int read_control(Workspace* w) {
  int rc = enqueue_control_copy(w);
  if (rc) return rc;
  WS_TRY(w, hipEventSynchronize(w->ev_ctl));
  return check_control(w);
}

int stuck(Workspace* w) {
  const Control& st = *w->h_ctl;
  return wfail(w, GMC_EOVERFLOW,
               "both particle queues are too full for any pass to proceed (photons " +
                   std::to_string(st.counts[0] + st.counts[1]) + ", electrons " +
                   std::to_string(st.counts[2] + st.counts[3]) + ", capacity " + std::to_string(w->cap_soft) +
                   "); lower the chunk or the secondaries budget");
}

int add_pass_time(Workspace* w, int type, hipEvent_t t0, hipEvent_t t1) {
  float ms = 0.0f;
  WS_TRY(w, hipEventElapsedTime(&ms, t0, t1));
  w->t_pass[type] += ms * 1e-3;
  ++w->n_pass[type];
  return GMC_OK;
}

}  // namespace

int enqueue_control_copy(Workspace* w) {
  WS_TRY(w, hipMemcpyAsync(w->h_ctl, w->d_ctl, sizeof(Control), hipMemcpyDeviceToHost, w->stream));
  WS_TRY(w, hipEventRecord(w->ev_ctl, w->stream));
  return GMC_OK;
}

int engine_setup(Workspace* w, Engine& E, const Job& J, const Tune& tu) {
  E.w = w;
  E.tu = tu;
  E.total[0] = J.total[0];
  E.total[1] = J.total[1];
  const int n_mat = J.T->host.n_mat;
  uint32_t cap = 0, soft = 0, stg = 0;
  queue_sizes(w, tu, n_mat, &cap, &soft, &stg);
  if ((uint64_t)cap * Q_FIELDS >= (1ull << 32)) return wfail(w, GMC_EOVERFLOW, "queue capacity too large");
  int rc = ensure_queues(w, cap);
  if (rc) return rc;
  w->cap_soft = soft;
  rc = ensure_staging(w, stg);
  if (rc) return rc;
  if (tu.sort) {
    rc = ensure_sorted(w, (uint32_t)tu.pass_items);   // a pass's items
    if (rc) return rc;
  }
  for (int t = 0; t < 2; ++t) {
    E.bud_same[t] = t == 0 ? 1u : (uint32_t)tu.secondaries + 1u;
    E.bud_other[t] = (uint32_t)tu.secondaries;
    E.block[t] = pass_block(w, t, tu.block, n_mat);
    E.waves[t] = pass_waves(w, t, E.block[t], n_mat);
    E.blocks[t] = E.waves[t] / ((uint32_t)E.block[t] / 64u);
  }
  const size_t nb = J.beams.size();
  rc = ws_ensure_beams(w, nb);
  if (rc) return rc;
  rc = ws_ensure_segments(w, std::max(J.beam_of[0].size(), J.beam_of[1].size()));
  if (rc) return rc;
  WS_TRY(w, hipMemcpy(w->d_beams, J.beams.data(), nb * sizeof(DevBeam), hipMemcpyHostToDevice));
  std::vector<DevSource> srcs = J.sources;
  if (!J.tab.empty()) {
    if (w->tab_cap < J.tab.size()) {
      if (w->d_tab) (void)hipFree(w->d_tab);
      w->d_tab = nullptr;
      w->tab_cap = 0;
      WS_TRY(w, hipMalloc(&w->d_tab, J.tab.size() * sizeof(double)));
      w->tab_cap = J.tab.size();
    }
    WS_TRY(w, hipMemcpy(w->d_tab, J.tab.data(), J.tab.size() * sizeof(double), hipMemcpyHostToDevice));
    for (size_t b = 0; b < nb; ++b)
      if (srcs[b].spectrum == GMC_TABULATED) srcs[b].tab = w->d_tab + J.tab_off[b];
  }
  WS_TRY(w, hipMemcpy(w->d_sources, srcs.data(), nb * sizeof(DevSource), hipMemcpyHostToDevice));
  for (int t = 0; t < 2; ++t) {
    WS_TRY(w, hipMemcpy(w->d_start + t * (w->seg_cap + 1), J.start[t].data(), J.start[t].size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice));
    if (!J.beam_of[t].empty()) {
      WS_TRY(w, hipMemcpy(w->d_beam_of + t * w->seg_cap, J.beam_of[t].data(),
                          J.beam_of[t].size() * sizeof(uint32_t), hipMemcpyHostToDevice));
      WS_TRY(w, hipMemcpy(w->d_seg_h + t * w->seg_cap, J.seg_h[t].data(), J.seg_h[t].size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
    }
  }
  Control ctl{};
  ctl.sched[2] = J.total[0];
  ctl.sched[3] = J.total[1];
  WS_TRY(w, hipMemcpy(w->d_ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice));
  WS_TRY(w, hipMemsetAsync(w->d_ctr, 0, C_COUNT * kCtrSlots * sizeof(unsigned long long), w->stream));
  w->acc[0] = w->acc[1] = 0;
  const DevPhantom dph = dev_phantom(*J.P);
  const DevCuts cuts = dev_cuts(*J.T);
  E.proto = PassArgs{};
  E.proto.ph = dph;
  E.proto.tab = dev_tables(*J.T, J.maj);
  E.proto.cut = cuts;
  E.proto.beams = w->d_beams;
  E.proto.n_beams = (int)J.beams.size();
  E.proto.ctr = w->d_ctr;
  E.proto.max_events = tu.events;
  E.proto.max_secondaries = tu.secondaries;
  E.proto.refill_lanes = tu.refill;
  E.proto.resume_lanes = kResumeLanes;
  bool single = true;   // every beam's own tally is one slice
  for (const DevBeam& b : J.beams) single &= b.a.K == 1u;
  E.proto.agg_a = tu.aggregate > 0 || (tu.aggregate == 0 && single) ? 1 : 0;
  // batches of the tally targets (their blocked layout's line count per
  // voxel block): the same for every beam of a job
  const uint32_t ka = J.beams.empty() ? 1u : J.beams[0].a.K, kb = J.beams.empty() ? 1u : J.beams[0].b.K;
  for (const DevBeam& b : J.beams)
    if (b.a.K != ka || b.b.K != kb) return wfail(w, GMC_EINTERNAL, "tally targets of one job differ in batches");
  E.proto.ka = ka;
  E.proto.kb = kb;
  for (int t = 0; t < 2; ++t) {
    AdmitArgs& a = E.adm[t];
    a = AdmitArgs{};
    a.ph = dph;
    a.cut = cuts;
    a.plan = w->d_ctl->adm + t;
    a.start = w->d_start + t * (w->seg_cap + 1);
    a.beam_of = w->d_beam_of + t * w->seg_cap;
    a.seg_h = w->d_seg_h + t * w->seg_cap;
    a.nb = (uint32_t)J.beam_of[t].size();
    a.beams = w->d_beams;
    a.sources = w->d_sources;
    a.ctr = w->d_ctr;
    a.ka = ka;
    a.kb = kb;
  }
  E.round = uses_round(tu, n_mat);
  if (E.round) {
    E.round_block = pass_block(w, 2, tu.block, n_mat);
    E.round_waves = pass_waves(w, 2, E.round_block, n_mat);
    E.round_blocks = E.round_waves / ((uint32_t)E.round_block / 64u);
  }
  for (int k = 0; k < 3; ++k) {
    w->t_pass[k] = 0.0;
    w->n_pass[k] = 0;
  }
  return GMC_OK;
}

// Plain form: the control block is read after admission and after the
// electron pass of every round; passes with nothing to do are skipped.  A
// round in which no primary was admitted and no pass transported anything
// leaves the state unchanged, so the next one would too: that is reported,
// not looped on.
int engine_run_plain(Engine& E, uint64_t* rounds) {
  Workspace* w = E.w;
  const Control& st = *w->h_ctl;
  if (E.round) {
    // one persistent kernel per round; the control block is read after each
    bool moved = true;
    for (;;) {
      int rc = enqueue_admission(E);
      if (rc) return rc;
      rc = read_control(w);
      if (rc) return rc;
      if (*rounds > 0) rc = add_pass_time(w, 2, w->kev0, w->kev1);
      if (rc) return rc;
      if (st.done()) break;
      if (*rounds > 0 && st.adm[0].count == 0 && st.adm[1].count == 0 && !moved) return stuck(w);
      ++*rounds;
      rc = enqueue_round(E, w->kev0, w->kev1, false);
      if (rc) return rc;
      rc = read_control(w);
      if (rc) return rc;
      moved = st.plan[0].m > 0 || st.plan[1].m > 0;
    }
    return GMC_OK;
  }
  bool e_prog = true, g_ran = false;
  for (;;) {
    int rc = enqueue_admission(E);
    if (rc) return rc;
    rc = read_control(w);
    if (rc) return rc;
    if (g_ran) rc = add_pass_time(w, 0, w->kev0, w->kev1);
    if (rc) return rc;
    if (st.done()) break;
    const bool g_prog = g_ran && st.plan[0].m > 0;
    if (*rounds > 0 && st.adm[0].count == 0 && st.adm[1].count == 0 && !e_prog && !g_prog) return stuck(w);
    ++*rounds;
    e_prog = false;
    g_ran = false;
    if (st.counts[2 + w->acc[1]] > 0) {
      rc = enqueue_pass(E, 1, w->kev0, w->kev1, false);
      if (rc) return rc;
      rc = read_control(w);
      if (rc) return rc;
      rc = add_pass_time(w, 1, w->kev0, w->kev1);
      if (rc) return rc;
      e_prog = st.plan[1].m > 0;
    }
    if (st.counts[w->acc[0]] > 0) {
      rc = enqueue_pass(E, 0, w->kev0, w->kev1, false);
      if (rc) return rc;
      g_ran = true;
    }
  }
  return GMC_OK;
}

// 2 R rounds (R = rounds_per_check) in one graph: each type's buffers swap
// once per round, so after an even number of rounds the buffer roles are
// back where they started.  Every pass kernel is bracketed by its own pair
// of event nodes.
int engine_capture(Engine& E, hipGraphExec_t* exec, int* rounds_per_replay) {
  Workspace* w = E.w;
  const int nr = 2 * E.tu.rounds;
  int rc = ensure_graph_events(w, (size_t)4 * nr);
  if (rc) return rc;
  hipGraph_t graph = nullptr;
  WS_TRY(w, hipStreamBeginCapture(w->stream, hipStreamCaptureModeThreadLocal));
  for (int r = 0; r < nr && rc == GMC_OK; ++r) {
    rc = enqueue_admission(E);
    if (E.round) {
      if (rc == GMC_OK) rc = enqueue_round(E, w->gev[4 * r], w->gev[4 * r + 1], true);
      continue;
    }
    if (rc == GMC_OK) rc = enqueue_pass(E, 1, w->gev[4 * r + 2], w->gev[4 * r + 3], true);
    if (rc == GMC_OK) rc = enqueue_pass(E, 0, w->gev[4 * r], w->gev[4 * r + 1], true);
  }
  const hipError_t ec = hipStreamEndCapture(w->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return wfail(w, GMC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
  const hipError_t e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return wfail(w, GMC_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  *rounds_per_replay = nr;
  return GMC_OK;
}

int after_replay(Engine& E, int nr, bool* done) {
  Workspace* w = E.w;
  int rc = check_control(w);
  // pair i brackets the pass of type i & 1 in round i / 2 (the round kernel: pair 2 r)
  if (E.round) {
    for (int r = 0; r < nr && rc == GMC_OK; ++r) rc = add_pass_time(w, 2, w->gev[4 * r], w->gev[4 * r + 1]);
  } else {
    for (int i = 0; i < 2 * nr && rc == GMC_OK; ++i) rc = add_pass_time(w, i & 1, w->gev[2 * i], w->gev[2 * i + 1]);
  }
  if (rc) return rc;
  const Control& st = *w->h_ctl;
  *done = st.done();
  // the last round admitted nothing and neither pass transported anything:
  // a fixed point
  if (!*done && st.adm[0].count == 0 && st.adm[1].count == 0 && st.plan[0].m == 0 && st.plan[1].m == 0)
    return stuck(w);
  return GMC_OK;
}

int engine_run_graph(Engine& E, uint64_t* rounds) {
  Workspace* w = E.w;
  hipGraphExec_t exec = nullptr;
  int nr = 0;
  int rc = engine_capture(E, &exec, &nr);
  if (rc) return rc;
  for (bool done = false; !done && rc == GMC_OK;) {
    const hipError_t e = hipGraphLaunch(exec, w->stream);
    if (e != hipSuccess) {
      rc = wfail(w, GMC_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
      break;
    }
    *rounds += (uint64_t)nr;
    rc = read_control(w);
    if (rc == GMC_OK) rc = after_replay(E, nr, &done);
  }
  (void)hipGraphExecDestroy(exec);
  return rc;
}

// ------------------------------------------------------------------ finalize
void add_batch_sizes(std::vector<double>& nk, uint64_t h0, uint64_t n, uint32_t K) {
  nk.resize(K, 0.0);
  // #{h < m : h mod K = k} = (m + K - 1 - k) / K, differenced over [h0, h0 + n)
  for (uint32_t k = 0; k < K; ++k) nk[k] += (double)((h0 + n + K - 1 - k) / K - (h0 + K - 1 - k) / K);
}

double dose_per_lsb(const PhantomObj& P) { return kLsbMeV * 1.602176634e-13 / (P.dx * P.dy * P.dz * 1e-3); }

int finalize(Workspace* w, const PhantomObj& P, const unsigned long long* tally, uint32_t nsum, size_t stride,
             uint32_t K, const std::vector<double>& nk, uint64_t n, double* d_dose, double* d_sigma, bool ledger,
             bool sync, bool blocked) {
  if (sync) {
    WS_TRY(w, hipMemcpyAsync(w->d_nk, nk.data(), K * sizeof(double), hipMemcpyHostToDevice, w->stream));
  } else {
    std::memcpy(w->h_nk, nk.data(), K * sizeof(double));
    WS_TRY(w, hipMemcpyAsync(w->d_nk, w->h_nk, K * sizeof(double), hipMemcpyHostToDevice, w->stream));
  }
  FinalizeArgs fa;
  fa.tally = tally;
  fa.nsum = nsum;
  fa.sum_stride = stride;
  fa.vox = P.d_vox;
  fa.nk = w->d_nk;
  fa.nvox = (uint32_t)P.nvox();
  fa.K = K;
  fa.n_total = (double)n;
  fa.conv = dose_per_lsb(P);
  fa.dose = d_dose;
  fa.sigma = d_sigma;
  fa.ctr = ledger ? w->d_ctr : nullptr;
  fa.blocked = blocked ? 1u : 0u;
  WS_TRY(w, launch_finalize(fa, w->stream));
  // the job's s (Eq. 12) with its combined result, read with the counters
  if (ledger) {
    w->h_srel[0] = std::numeric_limits<double>::quiet_NaN();
    if (d_sigma) {
      WS_TRY(w, launch_rel_uncertainty(d_dose, d_sigma, (uint32_t)P.nvox(), w->d_srel, w->stream));
      WS_TRY(w, hipMemcpyAsync(w->h_srel, w->d_srel + 3 * kRelBlocks, sizeof(double), hipMemcpyDeviceToHost,
                               w->stream));
    }
  }
  // nk is caller memory that may go away on return
  if (sync) WS_TRY(w, hipStreamSynchronize(w->stream));
  return GMC_OK;
}

int stats_from_counters(Workspace* w, const unsigned long long* slots, gmc_run_stats* stats, uint64_t n_hist,
                        uint64_t rounds, double t_total_s, double t_device_s) {
  unsigned long long ctr[C_COUNT] = {};
  for (int k = 0; k < C_COUNT; ++k)
    for (int j = 0; j < kCtrSlots; ++j) ctr[k] += slots[(size_t)k * kCtrSlots + j];
  const long long resid = (long long)(ctr[C_E_IN] - ctr[C_E_DEP] - ctr[C_E_ESC] - ctr[C_E_SINK]);
  if (stats) {
    stats->t_total_s = t_total_s;
    stats->t_device_s = t_device_s;
    stats->e_in_mev = ctr[C_E_IN] * kLsbMeV;
    stats->e_dep_mev = ctr[C_E_DEP] * kLsbMeV;
    stats->e_esc_mev = ctr[C_E_ESC] * kLsbMeV;
    stats->e_sink_mev = ctr[C_E_SINK] * kLsbMeV;
    stats->n_hist = n_hist;
    stats->n_photon_events = ctr[C_PH_EVENTS];
    stats->n_fictitious = ctr[C_FICT];
    stats->n_photon_interactions = ctr[C_PH_REAL];
    stats->n_e_steps = ctr[C_E_STEPS];
    stats->n_hard = ctr[C_HARD];
    stats->n_secondaries = ctr[C_SEC];
    stats->n_majorant_violations = ctr[C_VIOL];
    stats->n_passes = rounds;
    stats->ledger_residual_lsb = resid;
    stats->t_photon_pass_s = w->t_pass[0];
    stats->t_electron_pass_s = w->t_pass[1];
    stats->n_photon_launches = w->n_pass[0];
    stats->n_electron_launches = w->n_pass[1];
    stats->t_round_s = w->t_pass[2];
    stats->n_round_launches = w->n_pass[2];
    stats->s_rel = w->h_srel[0];
  }
  if (ctr[C_OVERFLOW]) return wfail(w, GMC_EINTERNAL, "queue overflow detected on the device");
  if (resid != 0) return wfail(w, GMC_EINTERNAL, "energy ledger does not close: residual " + std::to_string(resid));
  return GMC_OK;
}

int collect_stats(Workspace* w, gmc_run_stats* stats, uint64_t n_hist, uint64_t rounds,
                  std::chrono::steady_clock::time_point t_start) {
  WS_TRY(w, hipMemcpyAsync(w->h_ctr, w->d_ctr, (size_t)C_COUNT * kCtrSlots * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, w->stream));
  WS_TRY(w, hipEventRecord(w->ev1, w->stream));
  WS_TRY(w, hipStreamSynchronize(w->stream));
  float dev_ms = 0.0f;
  WS_TRY(w, hipEventElapsedTime(&dev_ms, w->ev0, w->ev1));
  const double t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return stats_from_counters(w, w->h_ctr, stats, n_hist, rounds, t_total, dev_ms * 1e-3);
}

// ------------------------------------------------------------ blocking forms
namespace {

int copy_out(Workspace* w, double* dst, const double* src, size_t n) {
  if (!dst) return GMC_OK;
  WS_TRY(w, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, w->stream));
  return GMC_OK;
}

// The batched form works on the context's own capture stream (a stream that
// may be captured, unlike the legacy default stream a caller could hand in),
// ordered after the caller's stream on entry and before it on exit.
struct StreamSwap {
  gmc_context* c;
  hipStream_t user;
  bool on;
  StreamSwap(gmc_context* ctx, bool enable) : c(ctx), user(ctx->ws.stream), on(enable) {
    if (!on) return;
    (void)hipEventRecord(c->join, user);
    (void)hipStreamWaitEvent(c->gstream, c->join, 0);
    c->ws.stream = c->gstream;
  }
  ~StreamSwap() {
    if (!on) return;
    (void)hipEventRecord(c->join, c->gstream);
    (void)hipStreamWaitEvent(user, c->join, 0);
    c->ws.stream = user;
  }
};

int run_job_ws(gmc_context* c, Workspace* w, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs,
               const uint64_t* n_hist, int n_beams, uint64_t seed, double* const* dose_per_beam,
               double* const* sigma_per_beam, double* dose, double* sigma, int out_kind, const gmc_tuning* tuning,
               gmc_run_stats* stats, bool batched, uint64_t* tally_out, int tally_kind) {
  const auto t_start = std::chrono::steady_clock::now();
  const PhantomObj* pp = nullptr;
  const TablesObj* tp = nullptr;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto pi = c->phantoms.find(phantom_id);
    auto ti = c->tables.find(tables_id);
    if (pi != c->phantoms.end()) pp = pi->second.get();
    if (ti != c->tables.end()) tp = ti->second.get();
  }
  if (!pp || !tp) return wfail(w, GMC_ENOTFOUND, "unknown phantom or tables id");
  const PhantomObj& P = *pp;
  const TablesObj& T = *tp;
  if (n_beams < 1 || n_beams > (1 << 20) || !srcs || !n_hist) return wfail(w, GMC_EINVAL, "need 1 .. 2^20 beams");
  if (!dose && !tally_out) return wfail(w, GMC_EINVAL, "dose output is NULL");
  if (out_kind != GMC_HOST && out_kind != GMC_DEVICE) return wfail(w, GMC_EINVAL, "bad out_ptr_kind");
  if (tally_out && (batched || n_beams != 1 || (tally_kind != GMC_HOST && tally_kind != GMC_DEVICE)))
    return wfail(w, GMC_EINVAL, "raw tallies are returned for one beam in the plain form, to host or device memory");
  if (P.max_mat >= T.host.n_mat) return wfail(w, GMC_EINVAL, "phantom uses a material index beyond the tables");
  const uint32_t K = (uint32_t)T.phys.n_batches;
  uint64_t n_total = 0, n_min = ~0ull;
  double e_sum = 0.0;
  for (int b = 0; b < n_beams; ++b) {
    const int rc = check_source(&w->err, &srcs[b]);
    if (rc) return rc;
    if (n_hist[b] == 0) return wfail(w, GMC_EINVAL, "every beam needs at least one history");
    if (n_hist[b] >= (1ull << 32)) return wfail(w, GMC_EINVAL, "histories must be < 2^32");
    // history numbers stay within 32 bits (their combined batch, (off + h) mod K, is
    // formed from off mod K on the device)
    if (srcs[b].first_history + n_hist[b] >= (1ull << 32))
      return wfail(w, GMC_EINVAL, "first_history + histories must stay below 2^32");
    n_total += n_hist[b];
    n_min = std::min<uint64_t>(n_min, n_hist[b]);
    const double e_max = source_emax(srcs[b]);
    e_sum += (double)n_hist[b] * (e_max * 134217728.0 + 1.0);
  }
  if (n_total < K) return wfail(w, GMC_EINVAL, "need at least n_batches histories");
  if (n_total >= (1ull << 32)) return wfail(w, GMC_EINVAL, "total histories must be < 2^32");
  if (e_sum >= 9.2e18) return wfail(w, GMC_EOVERFLOW, "histories x energy would overflow the 64-bit tallies");
  (void)hipSetDevice(c->device);
  const Tune tu = resolve_tuning(tuning);
  const size_t nvox = P.nvox();
  const size_t NB = (size_t)n_beams;

  // per-beam K-batched tallies when per-beam results are asked for, every
  // beam has at least K histories and they fit in half of the free device
  // memory; per-beam sigma needs them
  TallyMode mode = kCombined;
  if (batched && (dose_per_beam || sigma_per_beam)) {
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const double need = (double)NB * K * tally_vox(nvox) * sizeof(unsigned long long);
    const double room = 0.5 * ((double)free_b + (double)w->tally_elems * sizeof(unsigned long long));
    mode = (n_min >= K && need <= room) ? kBeamBatched : kBeamPlusComb;
    if (sigma_per_beam && mode != kBeamBatched)
      return wfail(w, n_min < K ? GMC_EINVAL : GMC_ENOMEM,
                   n_min < K ? "sigma per beam needs at least n_batches histories in every beam"
                             : "per-beam batched tallies do not fit in device memory");
  }
  const size_t tally_elems = job_tally_elems(mode, nvox, K, NB);
  int rc = ws_ensure_tally(w, tally_elems);
  if (rc) return rc;
  rc = ws_ensure_out(w, nvox);
  if (rc) return rc;
  MajObj maj;
  rc = get_majorants(c, phantom_id, tables_id, P, T, &maj, &w->err);
  if (rc) return rc;
  Job J;
  build_job(&J, w, P, T, maj, srcs, n_hist, n_beams, seed, mode);

  StreamSwap swap(c, batched && w == &c->ws);
  WS_TRY(w, hipEventRecord(w->ev0, w->stream));
  WS_TRY(w, launch_fill_u64(w->d_tally, tally_elems, 0ull, w->stream));
  Engine E;
  rc = engine_setup(w, E, J, tu);
  if (rc) return rc;
  uint64_t rounds = 0;
  rc = batched ? engine_run_graph(E, &rounds) : engine_run_plain(E, &rounds);
  if (rc) return rc;

  // combined result (and the ledger's deposited total)
  std::vector<double> nk;
  {
    // beam b's history h (numbered from its first history) is in combined
    // batch (off_b + h) mod K, off_b its offset in the combined tally
    uint64_t off = 0;
    for (int b = 0; b < n_beams; ++b) {
      add_batch_sizes(nk, (mode == kBeamBatched ? 0 : off) + srcs[b].first_history, n_hist[b], K);
      off += n_hist[b];
    }
  }
  double* d_out = out_kind == GMC_DEVICE && dose ? dose : w->d_dose;
  double* s_out = sigma ? (out_kind == GMC_DEVICE ? sigma : w->d_sigma) : nullptr;
  rc = mode == kBeamBatched
           ? finalize(w, P, w->d_tally, (uint32_t)NB, tally_vox(nvox) * K, K, nk, n_total, d_out, s_out, true, true)
           : finalize(w, P, w->d_tally, 1u, 0u, K, nk, n_total, d_out, s_out, true, true);
  if (rc) return rc;
  if (out_kind == GMC_HOST) {
    rc = copy_out(w, dose, w->d_dose, nvox);
    if (rc == GMC_OK && sigma) rc = copy_out(w, sigma, w->d_sigma, nvox);
    if (rc) return rc;
  }
  if (tally_out) {
    // the raw tally in the ABI's slice-major layout (staged on the device for a host buffer)
    const size_t bytes = nvox * K * sizeof(unsigned long long);
    unsigned long long* tmp = nullptr;
    if (tally_kind == GMC_HOST && hipMalloc(&tmp, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return wfail(w, GMC_ENOMEM, "staging buffer for the raw tally");
    }
    unsigned long long* dst = tmp ? tmp : reinterpret_cast<unsigned long long*>(tally_out);
    hipError_t e = launch_tally_to_slices(w->d_tally, dst, (uint32_t)nvox, K, w->stream);
    if (e == hipSuccess && tmp) e = hipMemcpyAsync(tally_out, tmp, bytes, hipMemcpyDeviceToHost, w->stream);
    if (e == hipSuccess && tmp) e = hipStreamSynchronize(w->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return wfail(w, GMC_EDEVICE, std::string("raw tally copy: ") + hipGetErrorString(e));
  }
  // per-beam results: into device memory all in one launch, into host memory
  // one beam at a time through the scratch outputs
  if (mode != kCombined && out_kind == GMC_DEVICE) {
    const uint32_t kb = mode == kBeamBatched ? K : 1u;
    std::vector<FinalizeArgs> list;
    std::vector<double> nks;   // kb batch sizes per listed beam
    for (int b = 0; b < n_beams; ++b) {
      double* want_d = dose_per_beam ? dose_per_beam[b] : nullptr;
      double* want_s = sigma_per_beam ? sigma_per_beam[b] : nullptr;
      if (!want_d && !want_s) continue;
      FinalizeArgs fa{};
      fa.tally = w->d_tally +
                 (mode == kBeamBatched ? tally_vox(nvox) * K * (size_t)b : tally_vox(nvox) * ((size_t)K + (size_t)b));
      fa.nsum = 1u;
      fa.sum_stride = 0u;
      fa.vox = P.d_vox;
      fa.nvox = (uint32_t)nvox;
      fa.K = kb;
      fa.n_total = (double)n_hist[b];
      fa.conv = dose_per_lsb(P);
      fa.dose = want_d;
      fa.sigma = want_s;
      fa.ctr = nullptr;
      fa.blocked = 1u;
      list.push_back(fa);
      std::vector<double> nkb;
      add_batch_sizes(nkb, srcs[b].first_history, n_hist[b], kb);
      nks.insert(nks.end(), nkb.begin(), nkb.end());
    }
    if (!list.empty()) {
      rc = ws_ensure_fin(w, list.size(), nks.size());
      if (rc) return rc;
      for (size_t i = 0; i < list.size(); ++i) list[i].nk = w->d_fin_nk + i * kb;
      WS_TRY(w, hipMemcpyAsync(w->d_fin_nk, nks.data(), nks.size() * sizeof(double), hipMemcpyHostToDevice,
                               w->stream));
      WS_TRY(w, hipMemcpyAsync(w->d_fin, list.data(), list.size() * sizeof(FinalizeArgs), hipMemcpyHostToDevice,
                               w->stream));
      WS_TRY(w, launch_finalize_many(w->d_fin, (uint32_t)list.size(), (uint32_t)nvox, kb, 1u, w->stream));
      // the argument lists are host memory of this call: wait until the device has used them
      WS_TRY(w, hipStreamSynchronize(w->stream));
    }
  } else if (mode != kCombined) {
    for (int b = 0; b < n_beams; ++b) {
      double* want_d = dose_per_beam ? dose_per_beam[b] : nullptr;
      double* want_s = sigma_per_beam ? sigma_per_beam[b] : nullptr;
      if (!want_d && !want_s) continue;
      // the dose is always computed; it lands in scratch when not wanted
      double* dd = out_kind == GMC_DEVICE && want_d ? want_d : w->d_dose;
      double* ds = want_s ? (out_kind == GMC_DEVICE ? want_s : w->d_sigma) : nullptr;
      const uint32_t kb = mode == kBeamBatched ? K : 1u;
      const unsigned long long* tb =
          w->d_tally + (mode == kBeamBatched ? tally_vox(nvox) * K * (size_t)b : tally_vox(nvox) * ((size_t)K + (size_t)b));
      std::vector<double> nkb;
      add_batch_sizes(nkb, srcs[b].first_history, n_hist[b], kb);
      rc = finalize(w, P, tb, 1u, 0u, kb, nkb, n_hist[b], dd, ds, false, true);
      if (rc) return rc;
      if (out_kind == GMC_HOST) {
        if (want_d) rc = copy_out(w, want_d, w->d_dose, nvox);
        if (rc == GMC_OK && want_s) rc = copy_out(w, want_s, w->d_sigma, nvox);
        if (rc) return rc;
        WS_TRY(w, hipStreamSynchronize(w->stream));
      }
    }
  }
  return collect_stats(w, stats, n_total, rounds, t_start);
}

}  // namespace

int run_job(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs, const uint64_t* n_hist,
            int n_beams, uint64_t seed, double* const* dose_per_beam, double* const* sigma_per_beam, double* dose,
            double* sigma, int out_kind, const gmc_tuning* tuning, gmc_run_stats* stats, bool batched,
            uint64_t* tally_out, int tally_kind) {
  const int rc = run_job_ws(c, &c->ws, phantom_id, tables_id, srcs, n_hist, n_beams, seed, dose_per_beam,
                            sigma_per_beam, dose, sigma, out_kind, tuning, stats, batched, tally_out, tally_kind);
  if (rc) c->err = c->ws.err;
  return rc;
}

// ----------------------------------------------------------------- autotuner
std::vector<int> job_class(const PhantomObj& P, const TablesObj& T, const gmc_source* srcs, const uint64_t* n_hist,
                           int n_beams) {
  double n = 0, e = 0, fe = 0, area = 0;
  for (int b = 0; b < n_beams; ++b) {
    const double w = (double)n_hist[b];
    n += w;
    e += w * source_emean(srcs[b]);
    fe += srcs[b].particle == GMC_ELECTRON ? w : 0.0;
    area += w * srcs[b].wx_cm * srcs[b].wy_cm;
  }
  const double nvox = (double)P.nvox();
  return {(int)std::lround(std::log2(nvox)), (int)std::lround(2.0 * std::log2(e / n)), (int)std::lround(4.0 * fe / n),
          (int)std::lround(std::log2(area / n + 0.01)), (int)std::lround(std::log2(n)), T.host.n_mat};
}

// Coordinate descent over the engine's knobs on a sample of the job (the
// first histories of every beam, in proportion, about 5% of the job and at
// least 2^20 histories), each candidate timed on the device from the
// admission to the finalize; a change is kept when it saves at least 2%.
int autotune(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs, const uint64_t* n_hist,
             int n_beams, double budget_s, gmc_tuning* out, gmc_autotune_report* rep, bool per_beam) {
  if (n_beams < 1 || !srcs || !n_hist || !out) return cfail(c, GMC_EINVAL, "bad autotune arguments");
  const PhantomObj* pp = nullptr;
  const TablesObj* tp = nullptr;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto pi = c->phantoms.find(phantom_id);
    auto ti = c->tables.find(tables_id);
    if (pi != c->phantoms.end()) pp = pi->second.get();
    if (ti != c->tables.end()) tp = ti->second.get();
  }
  if (!pp || !tp) return cfail(c, GMC_ENOTFOUND, "unknown phantom or tables id");
  uint64_t n_total = 0;
  for (int b = 0; b < n_beams; ++b) {
    std::string err;
    if (check_source(&err, &srcs[b])) return cfail(c, GMC_EINVAL, err);
    if (n_hist[b] == 0) return cfail(c, GMC_EINVAL, "every beam needs at least one history");
    n_total += n_hist[b];
  }
  if (n_total >= (1ull << 32)) return cfail(c, GMC_EINVAL, "total histories must be < 2^32");
  std::vector<int> key = job_class(*pp, *tp, srcs, n_hist, n_beams);
  key.push_back(per_beam ? 1 : 0);
  gmc_autotune_report r{};
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto hit = c->tuned.find(key);
    if (hit != c->tuned.end()) {
      *out = hit->second;
      r.from_cache = 1;
      if (rep) *rep = r;
      return GMC_OK;
    }
  }
  // A sample must hold several admission chunks of the largest candidate:
  // queue occupancy, and with it the pass sizes and lane fill, only settles
  // after a few rounds, and a sample too short for that ranks large passes
  // wrongly.
  const uint64_t want = std::min<uint64_t>(n_total, std::max<uint64_t>(kTuneMinSample, n_total / 20));
  const double f = (double)want / (double)n_total;
  std::vector<uint64_t> ns(n_beams);
  uint64_t n_sample = 0;
  for (int b = 0; b < n_beams; ++b) {
    ns[b] = std::max<uint64_t>(1, (uint64_t)std::llround(f * (double)n_hist[b]));
    n_sample += ns[b];
  }
  if (n_sample < (uint64_t)tp->phys.n_batches || n_sample >= (1ull << 32))
    return cfail(c, GMC_EINVAL, "job too small or too large to tune");
  int rc = ws_ensure_out(&c->ws, pp->nvox());
  if (rc) return cfail(c, rc, c->ws.err);
  const auto t0 = std::chrono::steady_clock::now();
  // with per-beam outputs every beam's dose lands in the same scratch buffer
  std::vector<double*> pb(per_beam ? (size_t)n_beams : 0u, c->ws.d_dose);
  // A candidate that needs larger queues allocates them inside its timed
  // run; run it again then, so that it is timed on its own work.
  auto trial = [&](const gmc_tuning& t, double* sec) -> int {
    for (int rep = 0; rep < 2; ++rep) {
      const uint32_t cap0 = c->ws.cap, stg0 = c->ws.stg_cap;
      gmc_run_stats st{};
      const int e = run_job(c, phantom_id, tables_id, srcs, ns.data(), n_beams, 0x5eedull,
                            per_beam ? pb.data() : nullptr, nullptr, c->ws.d_dose, nullptr, GMC_DEVICE, &t, &st,
                            true);
      ++r.trials;
      *sec = st.t_device_s;
      if (e != GMC_OK || (c->ws.cap == cap0 && c->ws.stg_cap == stg0)) return e;
    }
    return GMC_OK;
  };
  gmc_tuning best = default_tuning();
  double t_best = 0.0;
  rc = trial(best, &t_best);   // the first run sizes the buffers; time a second one
  if (rc == GMC_OK) rc = trial(best, &t_best);
  if (rc) return rc;
  // When the whole job's trials fit the budget, tune on the whole job: even
  // a sample of several chunks ranks the largest chunks and passes lower
  // than the job itself does.
  if (n_sample < n_total && t_best * ((double)n_total / (double)n_sample) * kTuneTrials <= budget_s) {
    for (int b = 0; b < n_beams; ++b) ns[b] = n_hist[b];
    n_sample = n_total;
    rc = trial(best, &t_best);
    if (rc == GMC_OK) rc = trial(best, &t_best);
    if (rc) return rc;
  }
  r.t_default_s = t_best;
  // twin: a second field set to twice the value (admission chunk and pass
  // size move together first: a pass should hold about two chunks)
  struct Dim {
    int gmc_tuning::*field;
    std::vector<int> values;
    int gmc_tuning::*twin;
  };
  const std::vector<Dim> dims = {
      {&gmc_tuning::chunk, {1 << 19, 1 << 20, 1 << 21, 1 << 22}, &gmc_tuning::pass_items},
      {&gmc_tuning::chunk, {1 << 19, 1 << 20, 1 << 21, 1 << 22}, nullptr},
      {&gmc_tuning::pass_items, {1 << 20, 1 << 21, 1 << 22, 1 << 23}, nullptr},
      {&gmc_tuning::events_per_visit, {32, 64, 128}, nullptr},
      {&gmc_tuning::wg_size, {256, 512, 1024}, nullptr},
      {&gmc_tuning::wave_items, {64, 128, 256}, nullptr},
      {&gmc_tuning::refill_lanes, {1, 4, 8, 16}, nullptr},
      {&gmc_tuning::rounds_per_check, {2, 4, 8}, nullptr},
      // the persistent round kernel against graph-replayed passes
      {&gmc_tuning::persistent, {1}, nullptr},
  };
  bool out_of_time = false;
  for (const Dim& d : dims) {
    const int cur = best.*(d.field);
    for (int v : d.values) {
      if (v == cur && (!d.twin || best.*(d.twin) == 2 * v)) continue;
      if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > budget_s) {
        out_of_time = true;
        break;
      }
      gmc_tuning cand = best;
      cand.*(d.field) = v;
      if (d.twin) cand.*(d.twin) = 2 * v;
      double t = 0.0;
      rc = trial(cand, &t);
      if (rc == GMC_EDEVICE) return rc;   // the device itself failed: stop
      if (rc) continue;                   // a candidate the job cannot run with (memory, queues): rejected
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
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->tuned[key] = best;
  }
  *out = best;
  if (rep) *rep = r;
  return GMC_OK;
}

}  // namespace gmc
