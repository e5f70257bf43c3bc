// gmc_runtime.cpp -- entry points of the C ABI declared in include/gpumcd.h:
// context, table and phantom handles, the plain and batched forms, the
// autotuner and the device checks.  The engine is in gmc_engine.cpp, the
// served form in gmc_server.cpp.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "gmc_host.hpp"

using namespace gmc;

extern "C" {

int gmc_create(int device, void* hip_stream, gmc_context** out) {
  if (!out) return GMC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GMC_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return GMC_EDEVICE;
  // The allocation-free entry points' work memory: its address on this device.
  if (scratch_resolve(device) != hipSuccess) return GMC_EDEVICE;
  auto* c = new gmc_context();
  c->device = device;
  if (ws_init(&c->ws, device, static_cast<hipStream_t>(hip_stream)) != GMC_OK ||
      hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess) {
    gmc_destroy(c);
    return GMC_ENOMEM;
  }
  *out = c;
  return GMC_OK;
}

void gmc_destroy(gmc_context* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  server_destroy(c);
  ws_free(&c->ws);
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
  if (c->join) (void)hipEventDestroy(c->join);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  delete c;
}

const char* gmc_last_error(const gmc_context* c) { return c ? c->err.c_str() : "no context"; }

int gmc_load_tables(gmc_context* c, const gmc_material* mats, int n_mat, const gmc_physics* phys,
                    int32_t* tables_id) {
  if (!c) return GMC_EINVAL;
  if (!mats || !phys || !tables_id || n_mat < 1 || n_mat > kMaxMat)
    return cfail(c, GMC_EINVAL, "need 1..8 materials, physics and an id pointer");
  for (int m = 0; m < n_mat; ++m)
    if (!(mats[m].z_over_a > 0 && mats[m].z_eff >= 1.0 && mats[m].i_ev > 0))
      return cfail(c, GMC_EINVAL, "material " + std::to_string(m) + " has a non-positive Z/A, Z or I");
  if (!(phys->ecut_mev >= 2 * kEmin && phys->ecut_mev < 30.0 && phys->pcut_mev >= kEmin && phys->pcut_mev < 30.0))
    return cfail(c, GMC_EINVAL, "cutoffs must lie in [0.002, 30) MeV (electrons) and [0.001, 30) MeV (photons)");
  if (phys->test_mode < 0 || phys->test_mode > 2) return cfail(c, GMC_EINVAL, "test_mode must be 0, 1 or 2");
  if (phys->n_batches > kMaxBatches) return cfail(c, GMC_EINVAL, "n_batches must be <= 1024");
  if (phys->majorant_margin > 0 && !(phys->majorant_margin >= 0.01 && phys->majorant_margin <= 100.0))
    return cfail(c, GMC_EINVAL, "majorant_margin must lie in [0.01, 100] (or <= 0 for the default)");
  (void)hipSetDevice(c->device);
  auto t = std::make_unique<TablesObj>();
  t->phys = *phys;
  if (t->phys.n_batches <= 0) t->phys.n_batches = 32;
  t->kcut = phys->kcut_mev > 0 ? phys->kcut_mev : phys->ecut_mev;
  t->kc = phys->kc_mev > 0 ? phys->kc_mev : phys->pcut_mev;
  if (phys->majorant_margin > 0) t->margin = phys->majorant_margin;
  if (!(t->kcut >= kEmin && t->kc >= kEmin)) return cfail(c, GMC_EINVAL, "kcut and kc must be >= 0.001 MeV");
  build_tables(mats, n_mat, t->kcut, t->kc, &t->host);
  const size_t nb = (size_t)n_mat * kNE * sizeof(float4);
  hipError_t e = hipMalloc(&t->d_ph, nb);
  if (e == hipSuccess) e = hipMalloc(&t->d_el, nb);
  if (e == hipSuccess) e = hipMalloc(&t->d_ms, kNms * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(t->d_ph, t->host.ph.data(), nb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(t->d_el, t->host.el.data(), nb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(t->d_ms, t->host.ms.data(), kNms * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    for (void* p : {(void*)t->d_ph, (void*)t->d_el, (void*)t->d_ms})
      if (p) (void)hipFree(p);
    return cfail(c, e == hipErrorOutOfMemory ? GMC_ENOMEM : GMC_EDEVICE,
                 std::string("table upload: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(c->mu);
  const int32_t id = c->next_id++;
  c->tables[id] = std::move(t);
  *tables_id = id;
  return GMC_OK;
}

int gmc_load_phantom(gmc_context* c, int nx, int ny, int nz, double dx, double dy, double dz,
                     const float* density, const uint8_t* material, int ptr_kind, int32_t* phantom_id) {
  if (!c) return GMC_EINVAL;
  if (!density || !material || !phantom_id) return cfail(c, GMC_EINVAL, "NULL phantom array or id pointer");
  if (nx <= 0 || ny <= 0 || nz <= 0 || (double)nx * ny * nz > 2147483647.0)
    return cfail(c, GMC_EINVAL, "grid must be positive with fewer than 2^31 voxels");
  if (!(dx > 0 && dy > 0 && dz > 0 && std::isfinite(dx) && std::isfinite(dy) && std::isfinite(dz)))
    return cfail(c, GMC_EINVAL, "voxel sizes must be positive");
  if (ptr_kind != GMC_HOST && ptr_kind != GMC_DEVICE) return cfail(c, GMC_EINVAL, "bad ptr_kind");
  (void)hipSetDevice(c->device);
  const size_t nv = (size_t)nx * ny * nz;
  std::vector<float> rho(nv);
  std::vector<uint8_t> mat(nv);
  if (ptr_kind == GMC_HOST) {
    std::memcpy(rho.data(), density, nv * sizeof(float));
    std::memcpy(mat.data(), material, nv);
  } else {
    if (hipMemcpy(rho.data(), density, nv * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(mat.data(), material, nv, hipMemcpyDeviceToHost) != hipSuccess)
      return cfail(c, GMC_EDEVICE, "copy of the phantom from device memory failed");
  }
  auto p = std::make_unique<PhantomObj>();
  p->nx = nx; p->ny = ny; p->nz = nz; p->dx = dx; p->dy = dy; p->dz = dz;
  p->rho_max.assign(256, 0.0);
  std::vector<uint2> vox(nv);
  for (size_t v = 0; v < nv; ++v) {
    const float r = rho[v];
    if (!(r >= 0.0f) || !std::isfinite(r)) return cfail(c, GMC_EINVAL, "densities must be finite and >= 0");
    const int m = mat[v];
    p->rho_max[m] = std::max(p->rho_max[m], (double)r);
    p->max_mat = std::max(p->max_mat, m);
    uint32_t bits;
    std::memcpy(&bits, &r, 4);
    vox[v] = uint2{bits, (uint32_t)m};
  }
  hipError_t e = hipMalloc(&p->d_vox, nv * sizeof(uint2));
  if (e == hipSuccess) e = hipMemcpy(p->d_vox, vox.data(), nv * sizeof(uint2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (p->d_vox) (void)hipFree(p->d_vox);
    return cfail(c, e == hipErrorOutOfMemory ? GMC_ENOMEM : GMC_EDEVICE,
                 std::string("phantom upload: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(c->mu);
  const int32_t id = c->next_id++;
  c->phantoms[id] = std::move(p);
  *phantom_id = id;
  return GMC_OK;
}

int gmc_release(gmc_context* c, int32_t id) {
  if (!c) return GMC_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->ws.stream);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->refs.count(id)) return cfail(c, GMC_EBUSY, "id " + std::to_string(id) + " is used by a queued request");
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
  return cfail(c, GMC_ENOTFOUND, "unknown id " + std::to_string(id));
}

int gmc_run_beam(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* src, uint64_t n_hist,
                 uint64_t seed, double* dose, double* sigma, int out_kind, const gmc_tuning* tuning,
                 gmc_run_stats* stats) {
  if (!c) return GMC_EINVAL;
  if (!src) return cfail(c, GMC_EINVAL, "source is NULL");
  return run_job(c, phantom_id, tables_id, src, &n_hist, 1, seed, nullptr, nullptr, dose, sigma, out_kind, tuning,
                 stats, false);
}

int gmc_run_beam_tally(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* src, uint64_t n_hist,
                       uint64_t seed, uint64_t* tally, int out_kind, const gmc_tuning* tuning, gmc_run_stats* stats) {
  if (!c) return GMC_EINVAL;
  if (!src) return cfail(c, GMC_EINVAL, "source is NULL");
  if (!tally) return cfail(c, GMC_EINVAL, "tally output is NULL");
  return run_job(c, phantom_id, tables_id, src, &n_hist, 1, seed, nullptr, nullptr, nullptr, nullptr, GMC_DEVICE,
                 tuning, stats, false, tally, out_kind);
}

int gmc_finalize_tally(gmc_context* c, int32_t phantom_id, int32_t tables_id, const uint64_t* tally, int tally_kind,
                       uint64_t h_begin, uint64_t h_end, double* dose, double* sigma, int out_kind, double* s_rel) {
  if (!c) return GMC_EINVAL;
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
  if (!tally || !dose) return cfail(c, GMC_EINVAL, "tally or dose is NULL");
  if ((tally_kind != GMC_HOST && tally_kind != GMC_DEVICE) || (out_kind != GMC_HOST && out_kind != GMC_DEVICE))
    return cfail(c, GMC_EINVAL, "bad pointer kind");
  const uint32_t K = (uint32_t)tp->phys.n_batches;
  if (h_end <= h_begin || h_end > (1ull << 32) || h_end - h_begin < K)
    return cfail(c, GMC_EINVAL, "the history range must hold at least n_batches histories below 2^32");
  (void)hipSetDevice(c->device);
  Workspace* w = &c->ws;
  const size_t nvox = pp->nvox();
  int rc = ws_ensure_out(w, nvox);
  if (rc) return cfail(c, rc, w->err);
  const unsigned long long* d_tally = reinterpret_cast<const unsigned long long*>(tally);
  if (tally_kind == GMC_HOST) {
    rc = ws_ensure_tally(w, nvox * K);
    if (rc) return cfail(c, rc, w->err);
    if (hipMemcpyAsync(w->d_tally, tally, nvox * K * sizeof(unsigned long long), hipMemcpyHostToDevice,
                       w->stream) != hipSuccess)
      return cfail(c, GMC_EDEVICE, "copy of the tallies to the device failed");
    d_tally = w->d_tally;
  }
  std::vector<double> nk;
  add_batch_sizes(nk, h_begin, h_end - h_begin, K);
  double* dd = out_kind == GMC_DEVICE ? dose : w->d_dose;
  double* ds = sigma ? (out_kind == GMC_DEVICE ? sigma : w->d_sigma) : nullptr;
  rc = finalize(w, *pp, d_tally, 1u, 0u, K, nk, h_end - h_begin, dd, ds, true, true, false);
  if (rc) return cfail(c, rc, w->err);
  if (out_kind == GMC_HOST) {
    hipError_t e = hipMemcpy(dose, w->d_dose, nvox * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && sigma) e = hipMemcpy(sigma, w->d_sigma, nvox * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return cfail(c, GMC_EDEVICE, std::string("result copy: ") + hipGetErrorString(e));
  }
  if (s_rel) *s_rel = w->h_srel[0];
  return GMC_OK;
}

int gmc_finalize_tally_noalloc(gmc_context* c, int32_t phantom_id, int32_t tables_id, const uint64_t* tally,
                               uint64_t h_begin, uint64_t h_end, double* dose, double* sigma, double* s_rel) {
  if (!c) return GMC_EINVAL;
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
  if (!tally || !dose) return cfail(c, GMC_EINVAL, "tally or dose is NULL");
  const uint32_t K = (uint32_t)tp->phys.n_batches;
  if (K > (uint32_t)kMaxBatches)
    return cfail(c, GMC_EINVAL, "n_batches above the " + std::to_string(kMaxBatches) +
                                    " batches the allocation-free work area holds");
  if (h_end <= h_begin || h_end > (1ull << 32) || h_end - h_begin < K)
    return cfail(c, GMC_EINVAL, "the history range must hold at least n_batches histories below 2^32");
  if (pp->nvox() > 0xffffffffull) return cfail(c, GMC_EINVAL, "phantom too large");
  (void)hipSetDevice(c->device);
  double* work = scratch_address(c->device);
  if (!work) return cfail(c, GMC_EDEVICE, "the allocation-free work area has no address on this device");
  Workspace* w = &c->ws;
  double* nk = work;                    // [K] histories per batch
  double* rel = work + kMaxBatches;     // [3 kRelBlocks + 1] s reduction, s last
  hipError_t e = launch_batch_sizes(nk, h_begin, h_end - h_begin, K, w->stream);
  FinalizeArgs fa;
  fa.tally = reinterpret_cast<const unsigned long long*>(tally);
  fa.nsum = 1u;
  fa.sum_stride = 0u;
  fa.vox = pp->d_vox;
  fa.nk = nk;
  fa.nvox = (uint32_t)pp->nvox();
  fa.K = K;
  fa.n_total = (double)(h_end - h_begin);
  fa.conv = dose_per_lsb(*pp);
  fa.dose = dose;
  fa.sigma = sigma;
  fa.ctr = nullptr;
  fa.blocked = 0u;   // the ABI's slice-major raw tallies
  if (e == hipSuccess) e = launch_finalize(fa, w->stream);
  w->h_srel[0] = std::numeric_limits<double>::quiet_NaN();
  if (e == hipSuccess && sigma && s_rel) {
    e = launch_rel_uncertainty(dose, sigma, (uint32_t)pp->nvox(), rel, w->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(w->h_srel, rel + 3 * kRelBlocks, sizeof(double), hipMemcpyDeviceToHost, w->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(w->stream);
  if (e != hipSuccess) return cfail(c, GMC_EDEVICE, std::string("allocation-free finalize: ") + hipGetErrorString(e));
  if (s_rel) *s_rel = w->h_srel[0];
  return GMC_OK;
}

int gmc_phantom_dims(gmc_context* c, int32_t phantom_id, int* nx, int* ny, int* nz) {
  if (!c) return GMC_EINVAL;
  if (!nx || !ny || !nz) return cfail(c, GMC_EINVAL, "NULL output");
  std::lock_guard<std::mutex> lk(c->mu);
  auto pi = c->phantoms.find(phantom_id);
  if (pi == c->phantoms.end()) return cfail(c, GMC_ENOTFOUND, "unknown phantom id " + std::to_string(phantom_id));
  *nx = pi->second->nx;
  *ny = pi->second->ny;
  *nz = pi->second->nz;
  return GMC_OK;
}

int gmc_run_beams(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs,
                  const uint64_t* n_hist, int n_beams, uint64_t seed, double* const* dose_per_beam,
                  double* const* sigma_per_beam, double* combined_dose, double* combined_sigma, int out_kind,
                  const gmc_tuning* tuning, gmc_run_stats* stats) {
  if (!c) return GMC_EINVAL;
  gmc_tuning tuned;
  if (!tuning && srcs && n_hist && n_beams >= 1) {
    const int rc = autotune(c, phantom_id, tables_id, srcs, n_hist, n_beams, kAutotuneBudgetS, &tuned, nullptr,
                            dose_per_beam != nullptr || sigma_per_beam != nullptr);
    if (rc) return rc;
    tuning = &tuned;
  }
  return run_job(c, phantom_id, tables_id, srcs, n_hist, n_beams, seed, dose_per_beam, sigma_per_beam, combined_dose,
                 combined_sigma, out_kind, tuning, stats, true);
}

int gmc_autotune(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* srcs,
                 const uint64_t* n_hist, int n_beams, double budget_s, gmc_tuning* out, gmc_autotune_report* report) {
  if (!c) return GMC_EINVAL;
  return autotune(c, phantom_id, tables_id, srcs, n_hist, n_beams, budget_s > 0 ? budget_s : kAutotuneBudgetS, out,
                  report);
}

int gmc_atomic_rate(gmc_context* c, int log2_words, int hot, double* adds_per_s) {
  if (!c) return GMC_EINVAL;
  if (!adds_per_s) return cfail(c, GMC_EINVAL, "output pointer is NULL");
  if (log2_words < 10 || log2_words > 31) return cfail(c, GMC_EINVAL, "log2_words must be in [10, 31]");
  const uint64_t words = 1ull << log2_words;
  if (hot < 0 || (hot > 0 && ((hot & (hot - 1)) != 0 || (uint64_t)hot > words)))
    return cfail(c, GMC_EINVAL, "hot must be 0 or a power of two no larger than the array");
  (void)hipSetDevice(c->device);
  const hipStream_t s = c->ws.stream;
  unsigned long long* d = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.0f;
  hipError_t e = hipMalloc(&d, words * sizeof(unsigned long long));
  if (e == hipSuccess) e = launch_fill_u64(d, words, 0ull, s);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_atomic_rate(d, (uint32_t)(words - 1), (uint32_t)hot, s);   // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch_atomic_rate(d, (uint32_t)(words - 1), (uint32_t)hot, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d) (void)hipFree(d);
  if (e != hipSuccess) return cfail(c, GMC_EDEVICE, hipGetErrorString(e));
  *adds_per_s = (double)kAtomicRateAdds / (ms * 1e-3);
  return GMC_OK;
}

int gmc_rng_words(gmc_context* c, uint64_t seed, uint32_t beam, uint32_t hist, uint64_t path, uint32_t n0, int count,
                  uint32_t* out) {
  if (!c) return GMC_EINVAL;
  if (!out || count < 0) return cfail(c, GMC_EINVAL, "bad output");
  if (count == 0) return GMC_OK;
  (void)hipSetDevice(c->device);
  const hipStream_t s = c->ws.stream;
  uint32_t* d = nullptr;
  hipError_t e = hipMalloc(&d, count * sizeof(uint32_t));
  if (e == hipSuccess)
    e = launch_rng_words((uint32_t)seed, (uint32_t)(seed >> 32) ^ beam, hist, (uint32_t)path, (uint32_t)(path >> 32),
                         n0, count, d, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d, count * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (d) (void)hipFree(d);
  if (e != hipSuccess) return cfail(c, GMC_EDEVICE, hipGetErrorString(e));
  return GMC_OK;
}

int gmc_table_eval(gmc_context* c, int32_t tables_id, int which, int mat, const double* energies, int n,
                   double* out) {
  if (!c) return GMC_EINVAL;
  const TablesObj* tp = nullptr;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto ti = c->tables.find(tables_id);
    if (ti != c->tables.end()) tp = ti->second.get();
  }
  if (!tp) return cfail(c, GMC_ENOTFOUND, "unknown tables id");
  if (which < 0 || which > 7 || mat < 0 || mat >= tp->host.n_mat || n < 0 || (n && (!energies || !out)))
    return cfail(c, GMC_EINVAL, "bad table query");
  if (n == 0) return GMC_OK;
  (void)hipSetDevice(c->device);
  const hipStream_t s = c->ws.stream;
  std::vector<float> ef(n), of(n);
  for (int i = 0; i < n; ++i) ef[i] = (float)energies[i];
  float *de = nullptr, *dout = nullptr;
  const MajObj none;
  const DevTables t = dev_tables(*tp, none);
  hipError_t e = hipMalloc(&de, n * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&dout, n * sizeof(float));
  if (e == hipSuccess) e = hipMemcpyAsync(de, ef.data(), n * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_table_eval(t, which, mat, de, n, dout, s);
  if (e == hipSuccess) e = hipMemcpyAsync(of.data(), dout, n * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (de) (void)hipFree(de);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return cfail(c, GMC_EDEVICE, hipGetErrorString(e));
  for (int i = 0; i < n; ++i) out[i] = of[i];
  return GMC_OK;
}

int gmc_first_events(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* src, uint64_t seed,
                     uint32_t h_begin, uint32_t h_end, float* out_xyz, uint32_t* out_nused) {
  if (!c) return GMC_EINVAL;
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
  std::string err;
  if (check_source(&err, src)) return cfail(c, GMC_EINVAL, err);
  if (src->particle != GMC_PHOTON) return cfail(c, GMC_EINVAL, "first events are defined for photon beams");
  if (h_end < h_begin || !out_xyz || !out_nused) return cfail(c, GMC_EINVAL, "bad history range or outputs");
  if (pp->max_mat >= tp->host.n_mat) return cfail(c, GMC_EINVAL, "phantom uses a material index beyond the tables");
  const uint32_t n = h_end - h_begin;
  if (n == 0) return GMC_OK;
  (void)hipSetDevice(c->device);
  Workspace* w = &c->ws;
  MajObj maj;
  int rc = get_majorants(c, phantom_id, tables_id, *pp, *tp, &maj, &err);
  if (rc) return cfail(c, rc, err);
  rc = ws_ensure_beams(w, 1);
  if (rc) return cfail(c, rc, w->err);
  DevBeam beam{};
  beam.key0 = (uint32_t)seed;
  beam.key1 = (uint32_t)(seed >> 32) ^ src->beam_id;
  beam.a = DevTally{nullptr, 1u, 0u};
  beam.b = DevTally{nullptr, 1u, 0u};
  PassArgs a{};
  a.ka = a.kb = 1u;
  a.ph = dev_phantom(*pp);
  a.tab = dev_tables(*tp, maj);
  a.cut = dev_cuts(*tp);
  a.beams = w->d_beams;
  a.n_beams = 1;
  DevSource ds = dev_source(*src);
  float* dx = nullptr;
  uint32_t* dn = nullptr;
  double* dt = nullptr;
  hipError_t e = hipMemcpy(w->d_beams, &beam, sizeof(beam), hipMemcpyHostToDevice);
  if (e == hipSuccess && src->spectrum == GMC_TABULATED) {
    std::vector<double> tab;
    tabulated_cdf(*src, &tab);
    e = hipMalloc(&dt, tab.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(dt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    ds.tab = dt;
  }
  if (e == hipSuccess) e = hipMalloc(&dx, (size_t)n * 3 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&dn, (size_t)n * sizeof(uint32_t));
  if (e == hipSuccess) e = launch_first_events(a, ds, h_begin, n, dx, dn, w->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_xyz, dx, (size_t)n * 3 * sizeof(float), hipMemcpyDeviceToHost, w->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_nused, dn, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost, w->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(w->stream);
  if (dx) (void)hipFree(dx);
  if (dn) (void)hipFree(dn);
  if (dt) (void)hipFree(dt);
  if (e != hipSuccess) return cfail(c, GMC_EDEVICE, hipGetErrorString(e));
  return GMC_OK;
}

}  // extern "C"
