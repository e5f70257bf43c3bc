// gmc_runtime.cpp -- host runtime behind the C ABI of include/gpumcd.h: device
// buffers, table and phantom handles, and the plain transport loop that
// alternates electron and photon passes until both particle arrays are empty
// (Sec. II.C.2, with the leftover threshold fixed at zero so that no particle
// is ever dropped).
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
constexpr uint32_t kMaxWaves = 1u << 15;

}  // namespace

struct gmc_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int32_t next_id = 1;
  std::map<int32_t, std::unique_ptr<TablesObj>> tables;
  std::map<int32_t, std::unique_ptr<PhantomObj>> phantoms;
  std::map<std::pair<int32_t, int32_t>, MajObj> majorants;
  // work buffers
  uint32_t cap = 0;
  QueueBuf qbuf[2][2];           // [type: 0 photon, 1 electron][2 buffers]
  int pend_idx[2] = {0, 0};      // which buffer of each type accumulates
  uint32_t* d_counts = nullptr;  // [2] pending counts per type
  unsigned long long* d_ctr = nullptr;  // [C_COUNT][kCtrSlots]
  unsigned long long* d_tally = nullptr;
  size_t tally_elems = 0;
  DevBeam* d_beams = nullptr;
  size_t beams_cap = 0;
  double* d_nk = nullptr;
  double* d_dose = nullptr;
  double* d_sigma = nullptr;
  size_t out_elems = 0;
  QueueBuf stg[2];                 // staging: [0] same type, [1] other type
  uint32_t stg_cap = 0;
  uint32_t* d_used = nullptr;      // [2][kMaxWaves]
  uint32_t* d_offsets = nullptr;   // [2][kMaxWaves]
  int resident[2] = {0, 0};
  int resident_block[2] = {0, 0};
  int resident_nmat[2] = {0, 0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t kev0 = nullptr, kev1 = nullptr;   // around each pass launch
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

DevQueue offset_queue(const DevQueue& q, uint32_t off) {
  DevQueue r = q;
  r.base += off;
  r.cap = q.cap - off;
  return r;
}

int ensure_queues(gmc_context* c, uint32_t cap) {
  if (c->cap >= cap) return GMC_OK;
  for (auto& t : c->qbuf)
    for (auto& b : t) free_queue(b);
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
  if (c->d_beams) (void)hipFree(c->d_beams);
  c->d_beams = nullptr;
  c->beams_cap = 0;
  HIP_TRY(c, hipMalloc(&c->d_beams, n * sizeof(DevBeam)));
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

// Pending counts per type.  A count above the capacity means the device
// skipped writes (it never writes past the capacity); it is reported before
// any kernel could read the missing entries.
int read_counts(gmc_context* c, uint32_t h[2]) {
  HIP_TRY(c, hipMemcpyAsync(h, c->d_counts, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (h[0] > c->cap || h[1] > c->cap) return fail(c, GMC_EINTERNAL, "particle queue overflow on the device");
  return GMC_OK;
}

struct Tune {
  int events, secondaries, chunk, block, pass_items;
};

Tune resolve_tuning(const gmc_tuning* t) {
  Tune r{64, 4, 1 << 20, 256, 1 << 21};
  if (t) {
    if (t->events_per_visit > 0) r.events = t->events_per_visit;
    if (t->secondaries_per_visit >= 2) r.secondaries = t->secondaries_per_visit;
    if (t->chunk > 0) r.chunk = t->chunk;
    if (t->wg_size >= 64 && t->wg_size <= 256 && t->wg_size % 64 == 0) r.block = t->wg_size;
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

// Run one pass over all pending particles of `type`.  The work is cut into
// launches of at most tu.pass_items particles; in each launch wavefront w owns
// a range of q particles and private staging segments sized for the
// worst-case output of q particles (survivor plus per-visit secondary
// budget), so no particle is ever dropped.  After each launch the segments
// are compacted into the pending queues.
int run_pass(gmc_context* c, int type, const PassArgs& proto, const Tune& tu, uint32_t counts[2],
             uint64_t* n_launch) {
  const int other = 1 - type;
  const uint32_t n = counts[type];
  if (n == 0) return GMC_OK;
  // the pending buffer becomes the work buffer; the other one collects
  const int wi = c->pend_idx[type];
  c->pend_idx[type] ^= 1;
  HIP_TRY(c, hipMemsetAsync(c->d_counts + type, 0, sizeof(uint32_t), c->stream));
  counts[type] = 0;
  const uint32_t bud_same = type == 0 ? 1u : (uint32_t)tu.secondaries + 1u;
  const uint32_t bud_other = (uint32_t)tu.secondaries;
  const DevQueue work = c->qbuf[type][wi].q;
  const int res = resident_blocks(c, type, tu.block, proto.tab.n_mat);
  const uint32_t waves_full = std::min<uint32_t>((uint32_t)res * (uint32_t)(tu.block / 64), kMaxWaves);
  uint32_t off = 0;
  while (off < n) {
    uint32_t m = std::min<uint32_t>(n - off, (uint32_t)tu.pass_items);
    m = std::min(m, (c->cap - counts[type]) / bud_same);
    m = std::min(m, (c->cap - counts[other]) / bud_other);
    if (m == 0) return fail(c, GMC_EOVERFLOW, "particle queues are full; raise the capacity or lower the chunk");
    uint32_t waves = std::max<uint32_t>(1u, std::min<uint32_t>(waves_full, (m + 63u) / 64u));
    const uint32_t q = (m + waves - 1) / waves;
    waves = (m + q - 1) / q;
    const uint32_t wpb = (uint32_t)tu.block / 64u;
    const uint32_t blocks = (waves + wpb - 1) / wpb;
    const uint32_t grid_waves = blocks * wpb;
    const uint32_t seg_same = q * bud_same, seg_other = q * bud_other;
    int rc = ensure_staging(c, grid_waves * std::max(seg_same, seg_other));
    if (rc) return rc;
    PassArgs a = proto;
    a.work = offset_queue(work, off);
    a.n_work = m;
    a.per_wave = q;
    a.stg_same = c->stg[0].q;
    a.stg_other = c->stg[1].q;
    a.seg_same = seg_same;
    a.seg_other = seg_other;
    a.used_same = c->d_used;
    a.used_other = c->d_used + kMaxWaves;
    a.max_events = tu.events;
    a.max_secondaries = tu.secondaries;
    HIP_TRY(c, hipEventRecord(c->kev0, c->stream));
    hipError_t e = type == 0 ? launch_photon_pass(a, (int)blocks, tu.block, c->stream)
                             : launch_electron_pass(a, (int)blocks, tu.block, c->stream);
    if (e != hipSuccess) return fail(c, GMC_EDEVICE, std::string("pass launch: ") + hipGetErrorString(e));
    HIP_TRY(c, hipEventRecord(c->kev1, c->stream));
    ++*n_launch;
    for (int d = 0; d < 2; ++d) {
      const int dt = d == 0 ? type : other;
      CompactArgs ca;
      ca.stg = c->stg[d].q;
      ca.seg = d == 0 ? seg_same : seg_other;
      ca.used = d == 0 ? a.used_same : a.used_other;
      ca.waves = grid_waves;
      ca.offsets = c->d_offsets + d * kMaxWaves;
      ca.dst = c->qbuf[dt][c->pend_idx[dt]].q;
      ca.dst_count = c->d_counts + dt;
      ca.ctr = c->d_ctr;
      e = launch_compact(ca, c->stream);
      if (e != hipSuccess) return fail(c, GMC_EDEVICE, std::string("compaction launch: ") + hipGetErrorString(e));
    }
    rc = read_counts(c, counts);
    if (rc) return rc;
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->kev0, c->kev1));
    c->t_pass[type] += ms * 1e-3;
    ++c->n_pass[type];
    off += m;
  }
  return GMC_OK;
}

int copy_out(gmc_context* c, double* dst, const double* src, size_t n, int kind) {
  if (!dst) return GMC_OK;
  HIP_TRY(c, hipMemcpyAsync(dst, src, n * sizeof(double),
                            kind == GMC_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, c->stream));
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
  if (hipMalloc(&c->d_counts, 2 * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&c->d_ctr, C_COUNT * kCtrSlots * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_nk, kMaxBatches * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_used, 2 * kMaxWaves * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&c->d_offsets, 2 * kMaxWaves * sizeof(uint32_t)) != hipSuccess ||
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
  for (auto& kv : c->tables) {
    (void)hipFree(kv.second->d_ph); (void)hipFree(kv.second->d_el); (void)hipFree(kv.second->d_ms);
  }
  for (auto& kv : c->phantoms) (void)hipFree(kv.second->d_vox);
  for (auto& kv : c->majorants) { (void)hipFree(kv.second.d_g); (void)hipFree(kv.second.d_e); }
  for (auto& t : c->qbuf)
    for (auto& b : t) free_queue(b);
  for (auto& b : c->stg) free_queue(b);
  (void)hipFree(c->d_used); (void)hipFree(c->d_offsets);
  (void)hipFree(c->d_counts); (void)hipFree(c->d_ctr); (void)hipFree(c->d_tally); (void)hipFree(c->d_beams);
  (void)hipFree(c->d_nk); (void)hipFree(c->d_dose); (void)hipFree(c->d_sigma);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->kev0) (void)hipEventDestroy(c->kev0);
  if (c->kev1) (void)hipEventDestroy(c->kev1);
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
        (void)hipFree(it->second.d_g); (void)hipFree(it->second.d_e);
        it = c->majorants.erase(it);
      } else {
        ++it;
      }
    }
  };
  auto t = c->tables.find(id);
  if (t != c->tables.end()) {
    (void)hipFree(t->second->d_ph); (void)hipFree(t->second->d_el); (void)hipFree(t->second->d_ms);
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

int gmc_run_beam(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* src,
                 uint64_t n_hist, uint64_t seed, double* dose, double* sigma, int out_kind,
                 const gmc_tuning* tuning, gmc_run_stats* stats) {
  if (!c) return GMC_EINVAL;
  const auto t_start = std::chrono::steady_clock::now();
  auto pi = c->phantoms.find(phantom_id);
  auto ti = c->tables.find(tables_id);
  if (pi == c->phantoms.end() || ti == c->tables.end()) return fail(c, GMC_ENOTFOUND, "unknown phantom or tables id");
  const PhantomObj& P = *pi->second;
  const TablesObj& T = *ti->second;
  int rc = check_source(c, src);
  if (rc) return rc;
  if (!dose) return fail(c, GMC_EINVAL, "dose output is NULL");
  if (out_kind != GMC_HOST && out_kind != GMC_DEVICE) return fail(c, GMC_EINVAL, "bad out_ptr_kind");
  if (P.max_mat >= T.host.n_mat) return fail(c, GMC_EINVAL, "phantom uses a material index beyond the tables");
  const uint32_t K = (uint32_t)T.phys.n_batches;
  if (n_hist < K || n_hist >= (1ull << 32)) return fail(c, GMC_EINVAL, "n_histories must be in [n_batches, 2^32)");
  const double emax = src->spectrum == GMC_MONO ? src->e_mev : src->e_hi;
  if ((double)n_hist * (emax * 134217728.0 + 1.0) >= 9.2e18)
    return fail(c, GMC_EOVERFLOW, "n_histories * energy would overflow the 64-bit tallies");
  (void)hipSetDevice(c->device);
  const Tune tu = resolve_tuning(tuning);
  const size_t nvox = (size_t)P.nx * P.ny * P.nz;

  MajObj maj;
  rc = get_majorants(c, phantom_id, tables_id, P, T, &maj);
  if (rc) return rc;
  // worst-case per-visit output must fit a chunk; the queues hold the chunk many times over
  // 12 fields of a queue stay addressable with 32-bit word indices below 2^32
  const uint32_t want_cap = std::max<uint32_t>(kDefaultCap, (uint32_t)std::min<uint64_t>(
      (uint64_t)tu.chunk * (tu.secondaries + 1) * 2, 1u << 26));
  rc = ensure_queues(c, want_cap);
  if (rc) return rc;
  rc = ensure_tally(c, (size_t)K * nvox);
  if (rc) return rc;
  rc = ensure_beams(c, 1);
  if (rc) return rc;
  if (out_kind == GMC_HOST || !sigma) {
    rc = ensure_out(c, nvox);
    if (rc) return rc;
  }

  // batch sizes n_k = #{h : floor(h K / N) = k}
  std::vector<double> nk(K, 0.0);
  for (uint32_t k = 0; k < K; ++k) {
    const uint64_t lo = (k * n_hist + K - 1) / K, hi = ((k + 1) * n_hist + K - 1) / K;
    nk[k] = (double)(hi - lo);
  }
  DevBeam beam;
  beam.key0 = (uint32_t)seed;
  beam.key1 = (uint32_t)(seed >> 32) ^ src->beam_id;
  beam.nhist = (uint32_t)n_hist;
  beam.nbatch = K;
  beam.tally = c->d_tally;

  HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_beams, &beam, sizeof(beam), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_nk, nk.data(), K * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_fill_u64(c->d_tally, (size_t)K * nvox, 0ull, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_ctr, 0, C_COUNT * kCtrSlots * sizeof(unsigned long long), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_counts, 0, 2 * sizeof(uint32_t), c->stream));

  const DevPhantom dph = dev_phantom(P);
  const DevCuts cuts = dev_cuts(T);
  PassArgs proto{};
  proto.ph = dph;
  proto.tab = dev_tables(T, maj);
  proto.cut = cuts;
  proto.beams = c->d_beams;
  proto.ctr = c->d_ctr;

  SourceArgs sa{};
  sa.ph = dph;
  sa.cut = cuts;
  sa.beams = c->d_beams;
  sa.ctr = c->d_ctr;
  sa.beam = 0;
  sa.spectrum = src->spectrum;
  sa.e_lsb = mev_to_lsb(src->e_mev);
  sa.e_lo = (float)src->e_lo; sa.e_mode = (float)src->e_mode; sa.e_hi = (float)src->e_hi;
  sa.cx = (float)src->cx_cm; sa.cy = (float)src->cy_cm; sa.wx = (float)src->wx_cm; sa.wy = (float)src->wy_cm;
  sa.particle = src->particle;

  c->t_pass[0] = c->t_pass[1] = 0.0;
  c->n_pass[0] = c->n_pass[1] = 0;
  const int ptype = src->particle == GMC_PHOTON ? 0 : 1;
  uint32_t counts[2] = {0, 0};
  uint64_t admitted = 0, launches = 0;
  for (;;) {
    if (admitted < n_hist && counts[0] + counts[1] < (uint32_t)tu.chunk) {
      const uint32_t room = c->cap - counts[ptype];
      const uint32_t cnt = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(tu.chunk, n_hist - admitted), room);
      if (cnt == 0) return fail(c, GMC_EOVERFLOW, "no room to admit primaries");
      sa.out = c->qbuf[ptype][c->pend_idx[ptype]].q;
      sa.out_base = counts[ptype];
      sa.out_count = c->d_counts + ptype;
      sa.h0 = (uint32_t)admitted;
      sa.count = cnt;
      HIP_TRY(c, launch_source(sa, c->stream));
      admitted += cnt;
      counts[ptype] += cnt;
    }
    if (counts[1]) { rc = run_pass(c, 1, proto, tu, counts, &launches); if (rc) return rc; }
    if (counts[0]) { rc = run_pass(c, 0, proto, tu, counts, &launches); if (rc) return rc; }
    if (admitted == n_hist && counts[0] == 0 && counts[1] == 0) break;
  }

  FinalizeArgs fa;
  fa.tally = c->d_tally;
  fa.vox = P.d_vox;
  fa.nk = c->d_nk;
  fa.nvox = (uint32_t)nvox;
  fa.K = K;
  fa.n_total = (double)n_hist;
  fa.conv = kLsbMeV * 1.602176634e-13 / (P.dx * P.dy * P.dz * 1e-3);
  fa.dose = out_kind == GMC_DEVICE ? dose : c->d_dose;
  fa.sigma = sigma ? (out_kind == GMC_DEVICE ? sigma : c->d_sigma) : nullptr;
  fa.ctr = c->d_ctr;
  HIP_TRY(c, launch_finalize(fa, c->stream));
  if (out_kind == GMC_HOST) {
    rc = copy_out(c, dose, c->d_dose, nvox, GMC_HOST);
    if (rc) return rc;
    if (sigma) { rc = copy_out(c, sigma, c->d_sigma, nvox, GMC_HOST); if (rc) return rc; }
  }
  std::vector<unsigned long long> slots((size_t)C_COUNT * kCtrSlots);
  HIP_TRY(c, hipMemcpyAsync(slots.data(), c->d_ctr, slots.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float dev_ms = 0.0f;
  (void)hipEventElapsedTime(&dev_ms, c->ev0, c->ev1);
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
    stats->n_passes = launches;
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

int gmc_rng_words(gmc_context* c, uint64_t seed, uint32_t beam, uint32_t hist, uint64_t path, uint32_t n0,
                  int count, uint32_t* out) {
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
  MajObj none;
  DevTables t = dev_tables(*ti->second, none);
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
  beam.nhist = 1;
  beam.nbatch = 1;
  beam.tally = nullptr;
  PassArgs a{};
  a.ph = dev_phantom(P);
  a.tab = dev_tables(T, maj);
  a.cut = dev_cuts(T);
  a.beams = c->d_beams;
  SourceArgs sa{};
  sa.ph = a.ph;
  sa.cut = a.cut;
  sa.beam = 0;
  sa.h0 = h_begin;
  sa.count = n;
  sa.spectrum = src->spectrum;
  sa.e_lsb = mev_to_lsb(src->e_mev);
  sa.e_lo = (float)src->e_lo; sa.e_mode = (float)src->e_mode; sa.e_hi = (float)src->e_hi;
  sa.cx = (float)src->cx_cm; sa.cy = (float)src->cy_cm; sa.wx = (float)src->wx_cm; sa.wy = (float)src->wy_cm;
  sa.particle = 0;
  float* dx = nullptr;
  uint32_t* dn = nullptr;
  HIP_TRY(c, hipMalloc(&dx, (size_t)n * 3 * sizeof(float)));
  HIP_TRY(c, hipMalloc(&dn, (size_t)n * sizeof(uint32_t)));
  hipError_t e = hipMemcpyAsync(c->d_beams, &beam, sizeof(beam), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_first_events(a, sa, dx, dn, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out_xyz, dx, (size_t)n * 3 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out_nused, dn, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(dx);
  (void)hipFree(dn);
  if (e != hipSuccess) return fail(c, GMC_EDEVICE, hipGetErrorString(e));
  return GMC_OK;
}

}  // extern "C"
