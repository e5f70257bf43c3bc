// gmc_kernels.hip -- gfx950 kernels of the coupled photon-electron transport.
//
// A pass kernel transports the particles of ONE type (Sec. II.C.2: photons and
// electrons are never simulated together, which removes the divergence of
// the photon-electron coupling).  Each wavefront owns a contiguous range of
// the work queue; a lane runs events on its particle until it dies, reaches
// the per-visit event cap (the N of Sec. II.C.3) or its per-visit secondary
// budget, and then takes the next particle of the range (lane-level refill,
// the "pool" idea of Sec. II.C.3 inside one launch).  Survivors and
// secondaries go to the wavefront's private segments of two staging queues,
// so no lane ever waits on a shared counter; when a workgroup is done, its
// wavefronts copy their segments into the accumulating queues, one atomic per
// workgroup and queue reserving the room (the stream compaction of Sec.
// II.C.3).  Rare, costly events (electron hard events, photon absorptions)
// are parked and sampled by many lanes together.
// Deposits are uint64 fixed-point atomics, so the dose is an exact integer
// sum independent of thread order.  Cross-section and stopping-power tables
// are staged in LDS by every workgroup.
#include <algorithm>
#include <mutex>

#include "gmc_device.hpp"

namespace gmc {
using namespace dev;

// ------------------------------------------------------------------ source
// Primary of history h (Sec. II.C.2, initParticle): parallel beam along +z at
// z = 0, position uniform over the field, energy monoenergetic, triangular or
// tabulated.  Uses the first block (words 0-3) of the history's root stream.
struct Primary { float x, y; uint32_t e; };

// Tabulated spectrum (a histogram): the bin j with C_j <= u < C_j+1 of the
// normalised CDF C at the edges (C_0 = 0, C_n = 1), found by bisection for
// the first edge above u, and the linear inverse inside it, in FP64.
__device__ __forceinline__ uint32_t sample_tabulated(const double* tab, uint32_t n, double u) {
  const double* edge = tab;
  const double* cdf = tab + n + 1;
  uint32_t lo = 0u, hi = n;   // cdf[lo] <= u < cdf[hi]
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cdf[mid] <= u) lo = mid; else hi = mid;
  }
  const double e = edge[lo] + (u - cdf[lo]) / (cdf[lo + 1] - cdf[lo]) * (edge[lo + 1] - edge[lo]);
  return (uint32_t)__double2uint_rn(e * 134217728.0);
}

__device__ __forceinline__ Primary sample_primary(const DevSource& a, const DevBeam& b, uint32_t h) {
  const Block blk = philox(0u, 0u, 0u, h, b.key0, b.key1);
  const float u0 = to_uniform(blk.w0), u1 = to_uniform(blk.w1), u2 = to_uniform(blk.w2);
  Primary p;
  p.x = a.cx + (u0 - 0.5f) * a.wx;
  p.y = a.cy + (u1 - 0.5f) * a.wy;
  if (a.spectrum == 1) {
    const float lo = a.e_lo, md = a.e_mode, hi = a.e_hi;
    const float fc = (md - lo) / (hi - lo);
    const float e = (u2 < fc) ? lo + sqrtf(u2 * (hi - lo) * (md - lo)) : hi - sqrtf((1.0f - u2) * (hi - lo) * (hi - md));
    p.e = to_lsb(e);
  } else if (a.spectrum == 2) {
    p.e = sample_tabulated(a.tab, a.tab_n, (double)u2);
  } else {
    p.e = a.e_lsb;
  }
  return p;
}

// History h's batch of a tally target: the sum of that batch in voxel v is
// at the returned pointer + vox_off(v, K) (the blocked layout).
__device__ __forceinline__ unsigned long long* tally_slice(const DevTally& t, uint32_t h) {
  if (!t.base) return nullptr;
  uint32_t k = h % t.K + t.off;   // (off + h) mod K with off < K: no 32-bit overflow
  if (k >= t.K) k -= t.K;
  return t.base + (size_t)k * kTallyBlock;
}
__device__ __forceinline__ size_t vox_off(uint32_t v, uint32_t K) {
  return (size_t)(v / kTallyBlock) * kTallyBlock * K + (v % kTallyBlock);
}

// Tally addition through the global address space: the tally pointers come
// from the beam table, so the compiler cannot tell their address space and
// would issue a flat atomic, which also holds the LDS counter -- every later
// table read in LDS would then wait for the atomic to be acknowledged.
__device__ __forceinline__ void tally_add(unsigned long long* p, unsigned long long v) {
  typedef __attribute__((address_space(1))) unsigned long long global_u64;
  __hip_atomic_fetch_add((global_u64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Admission sizes for both particle types: take the next histories of each
// type while its accumulating buffer holds fewer than `chunk` particles.
__global__ void k_admit_plan(AdmitPlanArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int t = 0; t < 2; ++t) {
    uint32_t* cnt = t == 0 ? a.count0 : a.count1;
    const uint32_t have = *cnt;
    const uint32_t left = a.total[t] - a.cursor[t];
    uint32_t take = 0;
    if (have < a.chunk) {
      take = min(left, a.chunk);
      take = have < a.cap ? min(take, a.cap - have) : 0u;
    }
    a.out[t].base = have;
    a.out[t].count = take;
    a.out[t].cursor = a.cursor[t];
    a.cursor[t] += take;
    *cnt = have + take;
  }
}

// Primaries of one particle type, written by index.  Primaries that start
// outside the phantom escape and sub-cutoff ones deposit where they enter;
// both are stored with zero energy, which the pass kernels skip.
__global__ void __launch_bounds__(256) k_admit(AdmitArgs a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const AdmitPlan pl = *a.plan;
  const bool valid = i < pl.count;
  const uint32_t g = pl.cursor + i;
  uint32_t j = 0;
  if (valid) {   // the segment holding index g: last j with start[j] <= g
    uint32_t lo = 0, hi = a.nb;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (a.start[mid] <= g) lo = mid; else hi = mid;
    }
    j = lo;
  }
  const uint32_t beam = valid ? a.beam_of[j] : 0u;
  uint32_t h = 0u;   // history number: the beam's first history plus its index in the beam
  Primary p{0.0f, 0.0f, 0u};
  int particle = 0;
  if (valid) {
    const DevSource src = a.sources[beam];
    particle = src.particle;
    h = g - a.start[j] + a.seg_h[j] + src.h0;
    p = sample_primary(src, a.beams[beam], h);
  }
  const bool in = valid && inside(a.ph, p.x, p.y, 0.0f);
  const uint32_t cut = particle == 0 ? a.cut.pcut_lsb : a.cut.ecut_lsb;
  const bool keep = in && p.e >= cut;
  const unsigned long long esc = (valid && !in) ? p.e : 0ull;
  if (in && !keep) {
    int ix, iy, iz;
    const int v = voxel(a.ph, p.x, p.y, 0.0f, ix, iy, iz);
    const DevBeam b = a.beams[beam];
    unsigned long long* ta = tally_slice(b.a, h);
    unsigned long long* tb = tally_slice(b.b, h);
    if (ta && p.e) tally_add(ta + vox_off((uint32_t)v, a.ka), (unsigned long long)p.e);
    if (tb && p.e) tally_add(tb + vox_off((uint32_t)v, a.kb), (unsigned long long)p.e);
  }
  if (valid) {
    const uint32_t slot = pl.base + i;
    if (slot < a.out.cap) put(a.out, slot, p.x, p.y, 0.0f, 0.0f, 0.0f, 1.0f, keep ? p.e : 0u, h, 0u, 0u, 4u, beam);
    else ctr_add(a.ctr, C_OVERFLOW, 1ull);
  }
  const unsigned long long ein = wave_sum(valid ? (unsigned long long)p.e : 0ull);
  const unsigned long long es = wave_sum(esc);
  if (lane_id() == 0) {
    if (ein) ctr_add(a.ctr, C_E_IN, ein);
    if (es) ctr_add(a.ctr, C_E_ESC, es);
  }
}

// ------------------------------------------------------------ lane state
struct Lane {
  float x, y, z, u, v, w;
  uint32_t e, beam;
  Stream s;
  unsigned long long* ta;      // this history's batch slice of tally target a
  unsigned long long* tb;      // of target b (null when the beam has none)
};

// A beam-table entry read member by member through a pointer of a given
// address space.
template <typename P>
__device__ __forceinline__ DevBeam read_beam(P p) {
  DevBeam b;
  b.key0 = p->key0;
  b.key1 = p->key1;
  b.a.base = p->a.base;
  b.a.K = p->a.K;
  b.a.off = p->a.off;
  b.b.base = p->b.base;
  b.b.K = p->b.K;
  b.b.off = p->b.off;
  return b;
}

__device__ __forceinline__ void load_lane(Lane& L, const DevQueue& q, uint32_t i, const PassArgs& a,
                                          const DevBeam* lbeams) {
  L.x = __uint_as_float(qf(q, Q_X, i)); L.y = __uint_as_float(qf(q, Q_Y, i)); L.z = __uint_as_float(qf(q, Q_Z, i));
  L.u = __uint_as_float(qf(q, Q_U, i)); L.v = __uint_as_float(qf(q, Q_V, i)); L.w = __uint_as_float(qf(q, Q_W, i));
  L.e = qf(q, Q_E, i);
  L.beam = qf(q, Q_BEAM, i);
  L.s.hist = qf(q, Q_HIST, i); L.s.plo = qf(q, Q_PLO, i); L.s.phi = qf(q, Q_PHI, i); L.s.n = qf(q, Q_N, i);
  // explicit address spaces: a merged pointer would make this a flat load,
  // which waits on both the LDS and the memory counters
  typedef __attribute__((address_space(3))) const DevBeam lds_beam;
  typedef __attribute__((address_space(1))) const DevBeam global_beam;
  const DevBeam b = a.n_beams <= kLdsBeams ? read_beam((lds_beam*)lbeams + L.beam)
                                           : read_beam((global_beam*)a.beams + L.beam);
  L.s.k0 = b.key0; L.s.k1 = b.key1;
  L.ta = tally_slice(b.a, L.s.hist);
  L.tb = tally_slice(b.b, L.s.hist);
}

__device__ __forceinline__ void store_lane(const Lane& L, const DevQueue& q, uint32_t slot) {
  put(q, slot, L.x, L.y, L.z, L.u, L.v, L.w, L.e, L.s.hist, L.s.plo, L.s.phi, L.s.n, L.beam);
}

struct Child { float u, v, w; uint32_t e, plo, phi; };

// A wavefront's share of the pass: the work queue's items m are cut into
// chunks (64 items by default) and chunk c goes to wavefront c mod W, so that every
// wavefront gets a slice of every part of the queue -- carried-over
// particles, survivors, the other type's secondaries, new primaries -- whose
// lives differ widely; contiguous shares left many wavefronts idle while a
// few finished theirs.  Loads stay coalesced within a chunk.  [next, end) is
// the wave-uniform cursor over the wavefront's own items, numbered 0..end-1.
struct WaveRange {
  uint32_t next, end, wave, waves, lg;
  // every item of the share has been handed to a lane
  __device__ __forceinline__ bool done() { return next >= end; }
  // items in the share (the tail requeue applies to large shares only)
  __device__ __forceinline__ uint32_t size() const { return end; }
  // work-queue index of the wavefront's item j
  __device__ __forceinline__ uint32_t item(uint32_t j) const {
    return (((j >> lg) * waves + wave) << lg) + (j & ((1u << lg) - 1u));
  }
};

__device__ __forceinline__ WaveRange wave_range(const PassPlan& P, uint32_t wave, uint32_t waves) {
  const uint32_t lg = P.chunk_log2;
  const uint32_t chunks = (uint32_t)(((uint64_t)P.m + (1u << lg) - 1u) >> lg);
  WaveRange r{0u, 0u, wave, waves, lg};
  if (wave < chunks) {
    const uint32_t own = (chunks - 1u - wave) / waves + 1u;
    r.end = own << lg;
    if ((chunks - 1u) % waves == wave) r.end -= (chunks << lg) - P.m;   // the last chunk may be partial
  }
  return r;
}

// A wavefront's work in the persistent round kernel: chunks of 2^lg
// consecutive work-queue items claimed one at a time from a device work
// queue.  The m items of a type are split into `parts` contiguous
// partitions, each with its own chunk counter; a wavefront claims from its
// workgroup's partition (block mod parts) first, so most claims are atomics
// on a counter only that workgroup's wavefronts share.  When that partition
// is used up the wavefront steals: its 64 lanes read 64 partitions' counters
// at once (agent-scope loads; a counter only grows, so one that reads
// exhausted is exhausted) and it claims from the first that still has a
// chunk, moving on through all partitions before it gives up.  It never
// claims more than `cap` items in all (the bound its staging segments were
// sized for); the caps add up to more than m, so every item is claimed by
// some wavefront.  No wavefront waits for another.  [next, end) are queue
// indices of the current chunk's items not yet handed out.
struct ClaimRange {
  uint32_t next, end;
  uint32_t taken, cap;        // items claimed so far, most it may claim
  uint32_t cur;               // partition of the last successful claim
  uint32_t m, parts, lg;
  bool exhausted;             // every partition found used up (or the cap reached)
  uint32_t* ctr;              // [parts] chunk counters of this type

  __device__ __forceinline__ uint32_t lo(uint32_t p) const {
    return (uint32_t)(((uint64_t)m * p) / parts);
  }
  __device__ __forceinline__ uint32_t chunks(uint32_t p) const {
    return (lo(p + 1u) - lo(p) + (1u << lg) - 1u) >> lg;
  }
  // one atomic on partition p's counter (wave-uniform p): true and the
  // chunk set when p still had one
  __device__ __forceinline__ bool take(uint32_t p) {
    uint32_t c = 0u;
    if (lane_id() == 0u) c = atomicAdd(ctr + p, 1u);
    c = __shfl(c, 0);
    const uint32_t a = lo(p), b = lo(p + 1u);
    const uint64_t first = (uint64_t)a + ((uint64_t)c << lg);
    if (first >= b) return false;
    next = (uint32_t)first;
    end = (uint32_t)min<uint64_t>(first + (1u << lg), b);
    taken += end - next;
    cur = p;
    return true;
  }
  __device__ __forceinline__ void claim() {
    if (exhausted || taken + (1u << lg) > cap) {
      exhausted = true;
      return;
    }
    if (take(cur)) return;
    // steal: scan the partitions after the current one, 64 at a time
    for (uint32_t base = 1u; base < parts; base += 64u) {
      const uint32_t off = base + lane_id();
      uint32_t p = cur + off;
      if (p >= parts) p -= parts;
      bool avail = false;
      if (off < parts) {
        const uint32_t c = __hip_atomic_load(ctr + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        avail = c < chunks(p);
      }
      unsigned long long mask = __ballot(avail);
      while (mask) {
        const int j = __ffsll((long long)mask) - 1;
        const uint32_t pj = (uint32_t)__shfl((int)p, j);
        if (take(pj)) return;
        mask &= mask - 1ull;
      }
    }
    exhausted = true;
  }
  // wave-uniform: claims the next chunk when the current one is used up
  __device__ __forceinline__ bool done() {
    if (next < end) return false;
    claim();
    return next >= end;
  }
  __device__ __forceinline__ uint32_t size() const { return taken; }
  __device__ __forceinline__ uint32_t item(uint32_t j) const { return j; }
};

__device__ __forceinline__ ClaimRange claim_range(const ClaimType& T, uint32_t* ctr, uint32_t lg, uint32_t block) {
  ClaimRange r;
  r.next = r.end = 0u;
  r.taken = 0u;
  r.cap = T.cap;
  r.m = T.m;
  r.parts = T.parts;
  r.cur = block % T.parts;
  r.lg = lg;
  r.exhausted = T.m == 0u;
  r.ctr = ctr;
  return r;
}

// Lanes without a particle take the next items of the range, in lane order,
// once at least a.refill_lanes of them are idle (one refill then pays the
// load latency for many lanes; with every lane idle it always proceeds).
// Entries with zero energy (primaries settled by the source) are skipped.
template <class R>
__device__ __forceinline__ void refill(Lane& L, bool& have, int& events, int& pushes, R& r, const PassArgs& a,
                                       const DevBeam* lbeams) {
  const unsigned long long need = __ballot(!have);
  if (need == 0 || __popcll(need) < a.refill_lanes || r.done()) return;
  if (!have) {
    const uint32_t it = r.next + (uint32_t)__popcll(need & lanes_below());
    if (it < r.end) {
      load_lane(L, a.work, r.item(it), a, lbeams);
      have = L.e != 0;
      events = 0;
      pushes = 0;
    }
  }
  const uint32_t nxt = r.next + (uint32_t)__popcll(need);
  r.next = nxt < r.end ? nxt : r.end;
}

// Write one entry into a wave segment; a slot beyond the segment (never
// expected: the per-visit budgets bound every segment) is counted, not written.
__device__ __forceinline__ bool seg_ok(const WaveSeg& g, uint32_t slot, unsigned long long* ctr) {
  if (slot < g.cap) return true;
  ctr_add(ctr, C_OVERFLOW, 1ull);
  return false;
}

__device__ __forceinline__ void deposit(const Lane& L, const PassArgs& a, int v, uint32_t e) {
  if (!e) return;
  tally_add(L.ta + vox_off((uint32_t)v, a.ka), (unsigned long long)e);
  if (L.tb) tally_add(L.tb + vox_off((uint32_t)v, a.kb), (unsigned long long)e);
}

// An electron usually takes several steps in one voxel (a boundary-limited
// step stops a hair short of the face, the next one crosses it), so the
// electron pass keeps one pending deposit per lane and adds it to the tally
// when the electron deposits elsewhere or leaves the lane.  The sum of a
// particle's deposits never exceeds its energy (< 2^32 units), and integer
// addition makes the result independent of when the additions happen.
struct Pending {
  int v = -1;
  uint32_t e = 0;
};

// A finished pending deposit whose tally-a addition waits for the end of the
// loop iteration, where the wavefront adds it aggregated (agg_a): lanes whose
// additions go to the same address are summed and their leader adds the sum
// with one atomic.  That pays where many lanes add to one address -- a
// single-slice tally of a pencil beam, all of whose histories deposit on the
// beam's axis -- and is left off where the batch slices already spread the
// addresses.
struct Deferred {
  unsigned long long* addr = nullptr;
  uint32_t e = 0;
};

__device__ __forceinline__ void flush(const Lane& L, const PassArgs& a, Pending& p, Deferred& d, bool agg) {
  if (p.e) {
    if (!agg) {
      deposit(L, a, p.v, p.e);
    } else {
      if (L.tb) tally_add(L.tb + vox_off((uint32_t)p.v, a.kb), (unsigned long long)p.e);
      if (d.e) tally_add(d.addr, (unsigned long long)d.e);   // a second one in the same iteration
      d.addr = L.ta + vox_off((uint32_t)p.v, a.ka);
      d.e = p.e;
    }
  }
  p.e = 0;
  p.v = -1;
}

__device__ __forceinline__ void deposit_later(const Lane& L, const PassArgs& a, Pending& p, int v, uint32_t e,
                                              Deferred& d, bool agg) {
  if (!e) return;
  if (v != p.v) {
    flush(L, a, p, d, agg);
    p.v = v;
  }
  p.e += e;
}

// End of a loop iteration (all lanes): the deferred additions, those to the
// first deferring lane's address summed into one atomic, the others each
// their own (one round: addresses that differ cost no extra rounds).
__device__ __forceinline__ void commit_deferred(Deferred& d) {
  const bool want = d.e != 0u;
  const unsigned long long m = __ballot(want);
  if (m == 0ull) return;
  const int leader = __ffsll((long long)m) - 1;
  const unsigned long long la = __shfl((unsigned long long)d.addr, leader);
  const bool same = want && (unsigned long long)d.addr == la;
  const unsigned long long sum = wave_sum(same ? (unsigned long long)d.e : 0ull);
  if ((int)lane_id() == leader) tally_add(d.addr, sum);
  else if (want && !same) tally_add(d.addr, (unsigned long long)d.e);
  d.e = 0u;
}

// One photon flight and interaction decision (Sec. II.A, Eqs. 1-3): free path
// with the majorant, then one uniform against the cumulative Compton,
// photoelectric, pair partials of the voxel; fictitious otherwise.
enum { PH_ESCAPE = 0, PH_FICT = 1, PH_COMPTON = 2, PH_PHOTO = 3, PH_PAIR = 4 };

__device__ __forceinline__ int photon_flight(Lane& L, const PassArgs& a, const float4* tab, const float* majg,
                                             int& v0, uint32_t& viol) {
  L.s.align();
  const float ef = (float)L.e * kLsbF;
  const TPos p = tpos(a.tab, ef);
  const float muh = majg[p.i];
  if (!(muh > 0.0f)) return PH_ESCAPE;
  const float d = fdiv(-fln(L.s.uniform()), muh);
  L.x = fmaf(d, L.u, L.x);
  L.y = fmaf(d, L.v, L.y);
  L.z = fmaf(d, L.w, L.z);
  if (!inside(a.ph, L.x, L.y, L.z)) return PH_ESCAPE;
  int ix, iy, iz;
  v0 = voxel(a.ph, L.x, L.y, L.z, ix, iy, iz);
  const uint2 vx = a.ph.vox[v0];
  const float rho = __uint_as_float(vx.x);
  const float4 c = lerp4(tab, (int)vx.y * kNE, p);
  const float mc = rho * c.x, mcp = rho * c.y;
  const float mt = (L.e > a.cut.two_mc2_lsb) ? rho * c.z : mcp;
  if (mt > muh) ++viol;
  const float r = L.s.uniform() * muh;
  if (r >= mt) return PH_FICT;
  if (r < mc) return PH_COMPTON;
  if (r < mcp) return PH_PHOTO;
  return PH_PAIR;
}

// End of a pass kernel's workgroup (every thread calls it once, after its
// wavefront's loop): particles m..n-1 of the work queue go to the front of
// the type's new queue (grid-stride over all threads), then one atomic per
// destination reserves room for the workgroup's staged entries and each
// wavefront copies its own segments.  Entries beyond a queue's capacity are
// counted, not written.
__device__ __forceinline__ void copy_entry(const DevQueue& dst, uint32_t d, const DevQueue& src, uint32_t s,
                                           unsigned long long* ctr) {
  if (d >= dst.cap) {
    ctr_add(ctr, C_OVERFLOW, 1ull);
    return;
  }
#pragma unroll
  for (int f = 0; f < Q_FIELDS; ++f) qf(dst, f, d) = qf(src, f, s);
}

__device__ __forceinline__ void append_outputs(const PassArgs& a, const PassPlan& P, const WaveSeg& gs,
                                               const WaveSeg& go) {
  __shared__ uint32_t s_used[2][16];
  __shared__ uint32_t s_base[2];
  const uint32_t carry = P.n - P.m;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < carry; i += gridDim.x * blockDim.x)
    copy_entry(a.dst_same, i, a.carry_src, P.m + i, a.ctr);
  const uint32_t wl = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t n0 = min(gs.used, gs.cap), n1 = min(go.used, go.cap);
  if (lane_id() == 0) {
    s_used[0][wl] = n0;
    s_used[1][wl] = n1;
  }
  __syncthreads();
  if (threadIdx.x < 2u) {
    uint32_t tot = 0;
    for (uint32_t w = 0; w < nw; ++w) tot += s_used[threadIdx.x][w];
    s_base[threadIdx.x] = tot ? atomicAdd(threadIdx.x == 0 ? a.cnt_same : a.cnt_other, tot) : 0u;
  }
  __syncthreads();
  uint32_t o0 = s_base[0], o1 = s_base[1];
  for (uint32_t w = 0; w < wl; ++w) {
    o0 += s_used[0][w];
    o1 += s_used[1][w];
  }
  for (uint32_t i = lane_id(); i < n0; i += 64u) copy_entry(a.dst_same, o0 + i, a.stg_same, gs.base + i, a.ctr);
  for (uint32_t i = lane_id(); i < n1; i += 64u) copy_entry(a.dst_other, o1 + i, a.stg_other, go.base + i, a.ctr);
}

// Photon absorbed in voxel v0 (Sec. II.B.2): photoelectric effect, one
// electron with the whole energy in the Sauter direction; or pair production,
// two electrons sharing E - 2 mc^2 uniformly at opposite azimuths, 2 mc^2 to
// the sink.  Electrons below the cutoff are deposited in v0; those above are
// left in c0 (and c1), nchild of them.
__device__ __forceinline__ void absorb_photon(Lane& L, const PassArgs& a, int kind, int v0, Child& c0, Child& c1,
                                              int& nchild, unsigned long long& acc_sink) {
  if (kind == PH_PHOTO) {
    const float ef = (float)L.e * kLsbF;
    const float cost = sample_sauter(ef, L.s);
    const float phi = kTwoPi * L.s.uniform();
    c0.u = L.u; c0.v = L.v; c0.w = L.w;
    rotate(c0.u, c0.v, c0.w, cost, phi);
    if (L.e >= a.cut.ecut_lsb) {
      c0.e = L.e;
      child_path(L.s.plo, L.s.phi, L.s.n, 0u, c0.plo, c0.phi);
      nchild = 1;
    } else {
      deposit(L, a, v0, L.e);
    }
    return;
  }
  const uint32_t avail = L.e - a.cut.two_mc2_lsb;
  const uint32_t t1 = min((uint32_t)fminf(L.s.uniform() * (float)avail, kMaxLsbF), avail);
  const uint32_t t2 = avail - t1;
  const float cs1 = pair_cos((float)t1 * kLsbF, L.s.uniform());
  const float cs2 = pair_cos((float)t2 * kLsbF, L.s.uniform());
  const float phi = kTwoPi * L.s.uniform();
  acc_sink += a.cut.two_mc2_lsb;
  c0.u = L.u; c0.v = L.v; c0.w = L.w;
  rotate(c0.u, c0.v, c0.w, cs1, phi);
  c1.u = L.u; c1.v = L.v; c1.w = L.w;
  rotate(c1.u, c1.v, c1.w, cs2, phi + kPi);
  if (t1 >= a.cut.ecut_lsb) {
    c0.e = t1;
    child_path(L.s.plo, L.s.phi, L.s.n, 0u, c0.plo, c0.phi);
    nchild = 1;
  } else {
    deposit(L, a, v0, t1);
  }
  if (t2 >= a.cut.ecut_lsb) {
    c1.e = t2;
    child_path(L.s.plo, L.s.phi, L.s.n, 1u, c1.plo, c1.phi);
    if (nchild == 0) c0 = c1;   // keep the pushed children contiguous
    ++nchild;
  } else {
    deposit(L, a, v0, t2);
  }
}

// Push the children of one event (nchild of c0, c1 per lane) to the wave's
// electron staging segment.
__device__ __forceinline__ void push_electrons(const Lane& L, const PassArgs& a, WaveSeg& g, int nchild,
                                               const Child& c0, const Child& c1) {
  const WaveSeg::Slots sl = g.append(nchild >= 1, nchild >= 2);
  const uint32_t hist = L.s.hist;
  if (nchild >= 1 && seg_ok(g, sl.s0, a.ctr))
    put(a.stg_other, g.base + sl.s0, L.x, L.y, L.z, c0.u, c0.v, c0.w, c0.e, hist, c0.plo, c0.phi, 0u, L.beam);
  if (nchild >= 2 && seg_ok(g, sl.s1, a.ctr))
    put(a.stg_other, g.base + sl.s1, L.x, L.y, L.z, c1.u, c1.v, c1.w, c1.e, hist, c1.plo, c1.phi, 0u, L.beam);
}

// ------------------------------------------------------------ photon pass
// One Woodcock flight per iteration (Sec. II.B.2).  Photoelectric and pair
// events end the photon: it is parked on a stack at the top of the
// wavefront's photon staging segment (with the interaction type) and the
// lane takes the next photon; once the range is done the wavefront samples
// the parked absorptions 64 at a time, so those two rarer branches do not run
// in most iterations with a few lanes each.  Each photon draws the same words
// in the same order either way.  Segment bound: each photon of the range
// leaves at most one survivor and is parked at most once, within per_wave x 2
// slots.
// Run counters a wavefront accumulates over its loop, added to the run's
// counters once at the end of the kernel.
struct WaveTotals {
  unsigned long long esc = 0, sink = 0;
  uint32_t ev = 0, fict = 0, viol = 0, sec = 0, steps = 0, hard = 0;
  uint32_t real = 0;   // photon flights that end in a real interaction
};

__device__ __forceinline__ void add_totals(const WaveTotals& t, unsigned long long* ctr) {
  const unsigned long long s_esc = wave_sum(t.esc), s_sink = wave_sum(t.sink);
  const unsigned long long s_ev = wave_sum(t.ev), s_fict = wave_sum(t.fict), s_viol = wave_sum(t.viol),
                           s_sec = wave_sum(t.sec), s_steps = wave_sum(t.steps), s_hard = wave_sum(t.hard),
                           s_real = wave_sum(t.real);
  if (lane_id() == 0) {
    if (s_esc) ctr_add(ctr, C_E_ESC, s_esc);
    if (s_sink) ctr_add(ctr, C_E_SINK, s_sink);
    if (s_ev) ctr_add(ctr, C_PH_EVENTS, s_ev);
    if (s_fict) ctr_add(ctr, C_FICT, s_fict);
    if (s_real) ctr_add(ctr, C_PH_REAL, s_real);
    if (s_viol) ctr_add(ctr, C_VIOL, s_viol);
    if (s_sec) ctr_add(ctr, C_SEC, s_sec);
    if (s_steps) ctr_add(ctr, C_E_STEPS, s_steps);
    if (s_hard) ctr_add(ctr, C_HARD, s_hard);
  }
}

// The photon transport of one wavefront over its range: photon tables in
// LDS at tab (per material) and majg (majorant), the beam table at lbeams.
template <class R>
__device__ void photon_loop(const PassArgs& a, uint32_t admitting, R& range, WaveSeg& gsame, WaveSeg& gother,
                            const float4* tab, const float* majg, const DevBeam* lbeams, WaveTotals& tot) {
  Lane L;
  bool have = false;
  int events = 0, pushes = 0;
  uint32_t npark = 0;   // parked absorptions on the stack, wave-uniform

  for (;;) {
    refill(L, have, events, pushes, range, a, lbeams);
    // a refill may bring only zero-energy entries: the wavefront goes on
    // until its range is done
    if (!__any(have)) {
      if (range.done()) break;
      continue;
    }
    int nchild = 0;
    Child c0, c1;
    bool surv = false, park = false;
    int kind = PH_ESCAPE;
    // tail of the share: with the range empty and few lanes still busy, a
    // photon that lives on after this event is requeued (while primaries
    // remain to be admitted)
    bool tail = false;
    if (a.tail_lanes > 0 && admitting && range.done() && range.size() >= a.tail_min)
      tail = (uint32_t)__popcll(__ballot(have)) <= (uint32_t)a.tail_lanes;
    if (have) {
      int v0 = 0;
      kind = photon_flight(L, a, tab, majg, v0, tot.viol);
      ++tot.ev;
      if (kind >= PH_COMPTON) ++tot.real;
      if (kind == PH_ESCAPE) {
        tot.esc += L.e;
        have = false;
      } else if (kind == PH_FICT) {
        ++tot.fict;
      } else if (a.cut.mode == 1) {
        deposit(L, a, v0, L.e);
        have = false;
      } else if (kind == PH_COMPTON) {
        // scattered photon plus recoil electron (momentum conservation)
        const float ef = (float)L.e * kLsbF;
        float eps, cost;
        sample_kn(ef / kMc2, L.s, eps, cost);
        const float phi = kTwoPi * L.s.uniform();
        float nu = L.u, nv = L.v, nw = L.w;
        rotate(nu, nv, nw, cost, phi);
        const uint32_t e1 = min(to_lsb(eps * ef), L.e);
        const uint32_t te = L.e - e1;
        if (te >= a.cut.ecut_lsb) {
          const float e1f = (float)e1 * kLsbF;
          float pu = ef * L.u - e1f * nu, pv = ef * L.v - e1f * nv, pw = ef * L.w - e1f * nw;
          const float inv = rsqrtf(pu * pu + pv * pv + pw * pw);
          c0.u = pu * inv; c0.v = pv * inv; c0.w = pw * inv;
          c0.e = te;
          child_path(L.s.plo, L.s.phi, L.s.n, 0u, c0.plo, c0.phi);
          nchild = 1;
        } else {
          deposit(L, a, v0, te);
        }
        L.u = nu; L.v = nv; L.w = nw;
        L.e = e1;
        if (e1 < a.cut.pcut_lsb) {
          deposit(L, a, v0, e1);
          have = false;
        }
      } else {
        // photoelectric absorption or pair production: parked, sampled in the wave's last phase
        park = true;
        have = false;
      }
      pushes += nchild;
      tot.sec += nchild;
      if (have) {
        ++events;
        if (tail || events >= a.max_events || pushes + 2 > a.max_secondaries) {
          surv = true;
          have = false;
        }
      }
    }
    // secondary electrons to the electron staging segment, survivors to the
    // bottom of the photon one, absorbed photons onto its stack
    push_electrons(L, a, gother, nchild, c0, c1);
    const WaveSeg::Slots ss = gsame.append(surv, false);
    if (surv && seg_ok(gsame, ss.s0, a.ctr)) store_lane(L, a.stg_same, gsame.base + ss.s0);
    const unsigned long long pm = __ballot(park);
    if (park) {
      const uint32_t k = npark + (uint32_t)__popcll(pm & lanes_below());
      if (k < gsame.cap && gsame.cap - 1u - k >= gsame.used) {
        const uint32_t slot = gsame.base + gsame.cap - 1u - k;
        store_lane(L, a.stg_same, slot);
        qf(a.stg_same, Q_AUX, slot) = (uint32_t)kind;
      } else {
        ctr_add(a.ctr, C_OVERFLOW, 1ull);
      }
    }
    npark += (uint32_t)__popcll(pm);
  }

  // last phase: the parked absorptions with every lane busy
  if (npark) __threadfence_block();   // a lane may read an entry another lane wrote
  for (uint32_t k0 = 0; k0 < npark; k0 += 64u) {
    const uint32_t k = k0 + lane_id();
    int nchild = 0;
    Child c0, c1;
    if (k < npark) {
      const uint32_t slot = gsame.base + gsame.cap - 1u - k;
      load_lane(L, a.stg_same, slot, a, lbeams);
      L.s.resume();
      const int kind = (int)qf(a.stg_same, Q_AUX, slot);
      int ix, iy, iz;
      const int v0 = voxel(a.ph, L.x, L.y, L.z, ix, iy, iz);
      absorb_photon(L, a, kind, v0, c0, c1, nchild, tot.sink);
      tot.sec += nchild;
    }
    push_electrons(L, a, gother, nchild, c0, c1);
  }
}

__global__ void __launch_bounds__(1024) k_photon_pass(PassArgs a) {
  extern __shared__ float4 smem[];
  const int nt = a.tab.n_mat * kNE;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) smem[i] = a.tab.ph[i];
  float* majg = reinterpret_cast<float*>(smem + nt);
  for (int i = threadIdx.x; i < kNE; i += blockDim.x) majg[i] = a.tab.maj_g[i];
  DevBeam* lbeams = reinterpret_cast<DevBeam*>(majg + kNE);
  if (a.n_beams <= kLdsBeams)
    for (int i = threadIdx.x; i < a.n_beams; i += blockDim.x) lbeams[i] = a.beams[i];
  __syncthreads();

  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const PassPlan P = *a.plan;
  WaveRange range = wave_range(P, wave, (gridDim.x * blockDim.x) >> 6);
  WaveSeg gsame{wave * P.seg_same, P.seg_same, 0u}, gother{wave * P.seg_other, P.seg_other, 0u};
  WaveTotals tot;
  photon_loop(a, P.admitting, range, gsame, gother, smem, majg, lbeams, tot);
  append_outputs(a, P, gsame, gother);
  add_totals(tot, a.ctr);
}

// ---------------------------------------------------------- electron pass
// Hard-event candidate at the end of a step (Sec. II.B.3): accepted with
// Sigma(end) / Sigma_hat, Sigma_hat being the majorant at the step-start
// energy, and split into Moller or bremsstrahlung.  The electron stands at
// the step's end point in voxel v1 with its energy after the step's loss;
// energy below the cutoffs is deposited in v1.  Returns whether the electron
// lives on; a secondary above its cutoff is left in c0 (ctype 0 photon, 1
// electron).
__device__ __forceinline__ bool hard_event(Lane& L, const PassArgs& a, const float4* smem, float sh, int v1,
                                           Child& c0, int& ctype, uint32_t& c_hard, uint32_t& c_viol) {
  const float t1f = (float)L.e * kLsbF;
  const float ur = L.s.uniform();
  const uint2 vy = a.ph.vox[v1];
  const float rho1 = __uint_as_float(vy.x);
  const float4 t1 = lerp4(smem, (int)vy.y * kNE, tpos(a.tab, t1f));
  const float sm = (L.e > a.cut.kcut2_lsb) ? rho1 * t1.y : 0.0f;
  const float sb = (L.e > a.cut.kc_lsb) ? rho1 * t1.z : 0.0f;
  if (sm + sb > sh) ++c_viol;
  const float r = ur * sh;
  if (r < sm) {
    // Moller: binary collision with a free electron at rest
    ++c_hard;
    const float eps = sample_moller(t1f, a.cut.kcut, L.s);
    const uint32_t wl = min(to_lsb(eps * t1f), L.e);
    const uint32_t tp = L.e - wl;
    const float wf = (float)wl * kLsbF, tpf = (float)tp * kLsbF;
    const float cd = sqrtf(fdiv(wf * (t1f + 2.0f * kMc2), t1f * (wf + 2.0f * kMc2)));
    const float cpp = sqrtf(fdiv(tpf * (t1f + 2.0f * kMc2), t1f * (tpf + 2.0f * kMc2)));
    const float phi = kTwoPi * L.s.uniform();
    c0.u = L.u; c0.v = L.v; c0.w = L.w;
    rotate(c0.u, c0.v, c0.w, cd, phi);
    rotate(L.u, L.v, L.w, cpp, phi + kPi);
    if (wl >= a.cut.ecut_lsb) {
      c0.e = wl;
      child_path(L.s.plo, L.s.phi, L.s.n, 0u, c0.plo, c0.phi);
      ctype = 1;
    } else {
      deposit(L, a, v1, wl);
    }
    L.e = tp;
  } else if (r < sm + sb) {
    // bremsstrahlung: electron direction unchanged, photon at mc^2/E
    ++c_hard;
    const float k = sample_brems(t1f, a.cut.kc, L.s);
    const float phi = kTwoPi * L.s.uniform();
    const uint32_t kl = min(to_lsb(k), L.e);
    c0.u = L.u; c0.v = L.v; c0.w = L.w;
    rotate(c0.u, c0.v, c0.w, __cosf(fdiv(kMc2, t1f + kMc2)), phi);
    if (kl >= a.cut.pcut_lsb) {
      c0.e = kl;
      child_path(L.s.plo, L.s.phi, L.s.n, 0u, c0.plo, c0.phi);
      ctype = 0;
    } else {
      deposit(L, a, v1, kl);
    }
    L.e -= kl;
  }
  if (L.e < a.cut.ecut_lsb) {
    deposit(L, a, v1, L.e);
    return false;
  }
  return true;
}

// One condensed step per iteration (Sec. II.B.3): e_s = min{d_vox, e_s-max,
// e_hard} (Eq. 4) with e_hard from the majorant at the step-start energy;
// energy loss of Eq. 8 read with the factor s; random hinge at zeta e_s with
// the deflection energy taken before or after the loss at random; the loss is
// deposited in the step-start voxel.
//
// A step that ends at a hard-event candidate parks the electron on a stack at
// the top of the wavefront's electron staging segment (with the step-start
// majorant and its visit counters), and its lane takes the next particle of
// the range.  Once the range is done, idle lanes take parked electrons back
// -- at least resume_lanes of them at a time, or all that remain when every
// lane is idle -- sample their hard events together and step on.  Sampling a
// hard event where it occurs would run the Moller and bremsstrahlung code in
// most iterations with a few lanes each.  A particle's draws and operations,
// and so the dose, are the same either way.
//
// Segment bound: each particle of the range (at most per_wave) leaves at most
// max_secondaries secondaries and one survivor at the bottom, and is parked
// at most once at a time, so a segment of per_wave x (max_secondaries + 2)
// slots holds bottom and stack without overlap.
// The electron transport of one wavefront over its range: electron tables
// in LDS at tab (per material), maje (hard-event majorant) and ms (screening),
// the beam table at lbeams.
template <class R>
__device__ void electron_loop(const PassArgs& a, uint32_t admitting, R& range, WaveSeg& gsame, WaveSeg& gother,
                              const float4* tab, const float* maje, const float* ms, const DevBeam* lbeams,
                              WaveTotals& tot) {
  Lane L;
  Pending pend;
  Deferred dfr;
  bool have = false;
  int events = 0, pushes = 0;
  uint32_t npark = 0;   // parked electrons on the stack, wave-uniform
  const float emin = a.cut.emin;

  for (;;) {
    refill(L, have, events, pushes, range, a, lbeams);
    // range done: idle lanes take back parked electrons, newest first
    bool hd = false;
    float hsh = 0.0f;
    if (npark && range.done()) {
      const unsigned long long need = __ballot(!have);
      const uint32_t nn = (uint32_t)__popcll(need);
      if (nn >= (uint32_t)a.resume_lanes || nn == 64u) {
        const uint32_t take = min(nn, npark);
        if (!have) {
          const uint32_t r = (uint32_t)__popcll(need & lanes_below());
          if (r < take) {
            const uint32_t slot = gsame.base + gsame.cap - npark + r;
            load_lane(L, a.stg_same, slot, a, lbeams);
            L.s.resume();
            hsh = __uint_as_float(qf(a.stg_same, Q_AUX, slot));
            const uint32_t cnt = qf(a.stg_same, Q_AUX2, slot);
            events = (int)(cnt & 0xffffu);
            pushes = (int)(cnt >> 16);
            pend.v = (int)qf(a.stg_same, Q_PV, slot);
            pend.e = qf(a.stg_same, Q_PE, slot);
            hd = true;
          }
        }
        npark -= take;
      }
    }
    if (!__any(have || hd)) {
      if (range.done()) break;
      continue;
    }
    if (__any(hd)) {
      int ctype = -1;
      Child c0;
      if (hd) {
        int jx, jy, jz, v1;
        if (electron_voxel(a.ph, L.x, L.y, L.z, L.u, L.v, L.w, jx, jy, jz, v1)) {   // inside when it was parked
          have = hard_event(L, a, tab, hsh, v1, c0, ctype, tot.hard, tot.viol);
        } else {
          tot.esc += L.e;
        }
        if (ctype >= 0) { ++pushes; ++tot.sec; }
      }
      // delta rays to the electron staging segment, photons to the photon one
      const WaveSeg::Slots se = gsame.append(ctype == 1, false);
      if (ctype == 1 && seg_ok(gsame, se.s0, a.ctr))
        put(a.stg_same, gsame.base + se.s0, L.x, L.y, L.z, c0.u, c0.v, c0.w, c0.e, L.s.hist, c0.plo, c0.phi, 0u, L.beam);
      const WaveSeg::Slots sg = gother.append(ctype == 0, false);
      if (ctype == 0 && seg_ok(gother, sg.s0, a.ctr))
        put(a.stg_other, gother.base + sg.s0, L.x, L.y, L.z, c0.u, c0.v, c0.w, c0.e, L.s.hist, c0.plo, c0.phi, 0u, L.beam);
    }
    bool surv = false, park = false;
    float sh = 0.0f;
    // tail of the share: with the range and the stack empty and few lanes
    // still busy, an electron that has stepped in this visit is requeued
    // rather than holding the wavefront for its last few particles -- while
    // primaries remain to be admitted, when a next pass comes anyway
    bool tail = false;
    if (a.tail_lanes > 0 && admitting && npark == 0 && range.done() && range.size() >= a.tail_min)
      tail = (uint32_t)__popcll(__ballot(have)) <= (uint32_t)a.tail_lanes;
    if (have && ((tail && events > 0) || events >= a.max_events || pushes + 1 > a.max_secondaries)) {
      // tail of the share, or visit budget spent (after a hard event): requeued
      surv = true;
      have = false;
    }
    // a resumed electron that ended at its hard event, or is requeued, adds
    // the pending deposit it brought back (idle lanes hold none)
    if (!have) flush(L, a, pend, dfr, a.agg_a);
    if (have) {
      L.s.align();
      int ix, iy, iz, v0;
      if (!electron_voxel(a.ph, L.x, L.y, L.z, L.u, L.v, L.w, ix, iy, iz, v0)) {
        tot.esc += L.e;
        have = false;
      } else {
        const uint2 vx = a.ph.vox[v0];
        const float rho0 = __uint_as_float(vx.x);
        const int base0 = (int)vx.y * kNE;
        if (L.e < a.cut.ecut_lsb) {
          deposit_later(L, a, pend, v0, L.e, dfr, a.agg_a);
          have = false;
        } else {
          ++tot.steps;
          const float tf = (float)L.e * kLsbF;
          const TPos p0 = tpos(a.tab, tf);
          sh = maje[p0.i];
          const float uh = L.s.uniform();
          const float ehard = (a.cut.mode == 2 || !(sh > 0.0f)) ? kInf : fdiv(-fln(uh), sh);
          const float dv = fmaxf(dist_boundary(a.ph, L.x, L.y, L.z, L.u, L.v, L.w, ix, iy, iz), a.ph.skin);
          const float emax = (a.cut.esmax_gcm2 > 0.0f && rho0 > 0.0f) ? fdiv(a.cut.esmax_gcm2, rho0) : kInf;
          float es = dv;
          bool hard = false;
          if (emax < es) es = emax;
          if (ehard < es) { es = ehard; hard = true; }
          const float4 t0 = lerp4(tab, base0, p0);
          const float l0 = rho0 * t0.x;
          const float tm = fmaxf(tf - 0.5f * es * l0, emin);
          const float de = es * rho0 * lerp_x(tab, base0, tpos(a.tab, tm));
          // the hinge word: fraction zeta from its top bits, deflection-energy coin from bit 0
          const uint32_t wz = L.s.word();
          const float zeta = to_uniform(wz);
          const float s1 = zeta * es;
          L.x = fmaf(s1, L.u, L.x);
          L.y = fmaf(s1, L.v, L.y);
          L.z = fmaf(s1, L.w, L.z);
          const uint32_t dl = to_lsb(de);
          if (dl >= L.e || L.e - dl < a.cut.ecut_lsb) {
            deposit_later(L, a, pend, v0, L.e, dfr, a.agg_a);
            have = false;
          } else {
            const uint32_t e1 = L.e - dl;
            const float t1f = (float)e1 * kLsbF;
            const float ua = L.s.uniform(), uphi = L.s.uniform();
            if (a.cut.mode != 2) {
              const float il = (wz & 1u) ? lerp_w(tab, base0, tpos(a.tab, t1f)) : t0.w;
              const float xx = es * rho0 * il;
              // G1 = 1 - exp(-x), by its series where the subtraction would cancel
              const float g1 = xx < 1e-3f ? xx * (1.0f - 0.5f * xx * (1.0f - xx * (1.0f / 3.0f))) : 1.0f - fexp(-xx);
              rotate_om(L.u, L.v, L.w, wentzel_om(a.tab, ms, g1, ua), kTwoPi * uphi);
            }
            deposit_later(L, a, pend, v0, dl, dfr, a.agg_a);
            L.e = e1;
            const float s2 = (1.0f - zeta) * es;
            L.x = fmaf(s2, L.u, L.x);
            L.y = fmaf(s2, L.v, L.y);
            L.z = fmaf(s2, L.w, L.z);
            int jx, jy, jz, v1;
            if (!electron_voxel(a.ph, L.x, L.y, L.z, L.u, L.v, L.w, jx, jy, jz, v1)) {
              tot.esc += L.e;
              have = false;
            } else if (hard) {
              park = true;
              have = false;
            }
          }
        }
      }
      if (have || park) {
        ++events;
        if (have && events >= a.max_events) {
          surv = true;
          have = false;
        }
      }
      // before the lane takes another particle; a parked electron keeps its
      // pending deposit (pencil beams concentrate deposits on few voxels,
      // where every extra atomic costs)
      if (!have && !park) flush(L, a, pend, dfr, a.agg_a);
    }
    {
      // survivors to the bottom of the electron staging segment, parked electrons onto its stack
      const WaveSeg::Slots se = gsame.append(surv, false);
      if (surv && seg_ok(gsame, se.s0, a.ctr)) store_lane(L, a.stg_same, gsame.base + se.s0);
      const unsigned long long pm = __ballot(park);
      if (park) {
        const uint32_t k = npark + (uint32_t)__popcll(pm & lanes_below());
        if (k < gsame.cap && gsame.cap - 1u - k >= gsame.used) {
          const uint32_t slot = gsame.base + gsame.cap - 1u - k;
          store_lane(L, a.stg_same, slot);
          qf(a.stg_same, Q_AUX, slot) = __float_as_uint(sh);
          qf(a.stg_same, Q_AUX2, slot) = (uint32_t)events | ((uint32_t)pushes << 16);
          qf(a.stg_same, Q_PV, slot) = (uint32_t)pend.v;
          qf(a.stg_same, Q_PE, slot) = pend.e;
          pend = Pending{};
        } else {
          ctr_add(a.ctr, C_OVERFLOW, 1ull);
          flush(L, a, pend, dfr, a.agg_a);
        }
      }
      npark += (uint32_t)__popcll(pm);
      // a lane that reads a parked entry may not be the lane that wrote it
      if (pm) __threadfence_block();
    }
    if (a.agg_a) commit_deferred(dfr);
  }
}

__global__ void __launch_bounds__(1024) k_electron_pass(PassArgs a) {
  extern __shared__ float4 smem[];
  const int nt = a.tab.n_mat * kNE;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) smem[i] = a.tab.el[i];
  float* maje = reinterpret_cast<float*>(smem + nt);
  float* ms = maje + kNE;
  for (int i = threadIdx.x; i < kNE; i += blockDim.x) maje[i] = a.tab.maj_e[i];
  for (int i = threadIdx.x; i < kNms; i += blockDim.x) ms[i] = a.tab.ms[i];
  DevBeam* lbeams = reinterpret_cast<DevBeam*>(ms + kNms);
  if (a.n_beams <= kLdsBeams)
    for (int i = threadIdx.x; i < a.n_beams; i += blockDim.x) lbeams[i] = a.beams[i];
  __syncthreads();

  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const PassPlan P = *a.plan;
  WaveRange range = wave_range(P, wave, (gridDim.x * blockDim.x) >> 6);
  WaveSeg gsame{wave * P.seg_same, P.seg_same, 0u}, gother{wave * P.seg_other, P.seg_other, 0u};
  WaveTotals tot;
  electron_loop(a, P.admitting, range, gsame, gother, smem, maje, ms, lbeams, tot);
  append_outputs(a, P, gsame, gother);
  add_totals(tot, a.ctr);
}

// ------------------------------------------------------------ round kernel
// End of a round kernel's workgroup: both types' carried-over particles to
// the front of their new queues, then one atomic per type reserves room for
// the workgroup's staged outputs of that type and each wavefront copies its
// segments.
__device__ __forceinline__ void append_round(const RoundArgs& r, const PassPlan& Pe, const PassPlan& Pg,
                                             const WaveSeg& se, const WaveSeg& sg) {
  __shared__ uint32_t s_used[2][16];
  __shared__ uint32_t s_base[2];
  const uint32_t ce = Pe.n - Pe.m, cg = Pg.n - Pg.m;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ce; i += gridDim.x * blockDim.x)
    copy_entry(r.e.dst_same, i, r.e.carry_src, Pe.m + i, r.e.ctr);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cg; i += gridDim.x * blockDim.x)
    copy_entry(r.g.dst_same, i, r.g.carry_src, Pg.m + i, r.g.ctr);
  const uint32_t wl = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t n0 = min(se.used, se.cap), n1 = min(sg.used, sg.cap);
  if (lane_id() == 0) {
    s_used[0][wl] = n0;
    s_used[1][wl] = n1;
  }
  __syncthreads();
  if (threadIdx.x < 2u) {
    uint32_t tot = 0;
    for (uint32_t w = 0; w < nw; ++w) tot += s_used[threadIdx.x][w];
    s_base[threadIdx.x] = tot ? atomicAdd(threadIdx.x == 0 ? r.e.cnt_same : r.g.cnt_same, tot) : 0u;
  }
  __syncthreads();
  uint32_t o0 = s_base[0], o1 = s_base[1];
  for (uint32_t w = 0; w < wl; ++w) {
    o0 += s_used[0][w];
    o1 += s_used[1][w];
  }
  for (uint32_t i = lane_id(); i < n0; i += 64u) copy_entry(r.e.dst_same, o0 + i, r.e.stg_same, se.base + i, r.e.ctr);
  for (uint32_t i = lane_id(); i < n1; i += 64u) copy_entry(r.g.dst_same, o1 + i, r.g.stg_same, sg.base + i, r.g.ctr);
}

// The persistent round kernel (the batched form's pool of persistent
// wavefronts, Sec. II.C.3): every workgroup stages both table blocks, and
// each wavefront claims chunks of the round's electrons from the device work
// queue until none is left (or its cap is reached), finishes its electrons
// and their parked hard events, then claims photons the same way.  The
// electron and photon loops are those of the pass kernels; only where their
// items come from differs.  Electron outputs of both phases go to the
// wavefront's electron segment, photon outputs to its photon segment.
__global__ void __launch_bounds__(kRoundMaxBlock) k_round(RoundArgs r) {
  extern __shared__ float4 smem[];
  const int nt = r.e.tab.n_mat * kNE;
  float4* tg = smem;
  float4* te = smem + nt;
  float* majg = reinterpret_cast<float*>(te + nt);
  float* maje = majg + kNE;
  float* ms = maje + kNE;
  DevBeam* lbeams = reinterpret_cast<DevBeam*>(ms + kNms);
  for (int i = threadIdx.x; i < nt; i += blockDim.x) {
    tg[i] = r.g.tab.ph[i];
    te[i] = r.e.tab.el[i];
  }
  for (int i = threadIdx.x; i < kNE; i += blockDim.x) {
    majg[i] = r.g.tab.maj_g[i];
    maje[i] = r.e.tab.maj_e[i];
  }
  for (int i = threadIdx.x; i < kNms; i += blockDim.x) ms[i] = r.e.tab.ms[i];
  if (r.e.n_beams <= kLdsBeams)
    for (int i = threadIdx.x; i < r.e.n_beams; i += blockDim.x) lbeams[i] = r.e.beams[i];
  __syncthreads();

  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const PassPlan Pg = *r.g.plan, Pe = *r.e.plan;
  WaveSeg se{wave * Pe.seg_same, Pe.seg_same, 0u}, sg{wave * Pg.seg_same, Pg.seg_same, 0u};
  WaveTotals tot;
  ClaimRange re = claim_range(r.claims[1], r.claim_ctr + kMaxClaimParts, Pe.chunk_log2, blockIdx.x);
  electron_loop(r.e, Pe.admitting, re, se, sg, te, maje, ms, lbeams, tot);
  ClaimRange rg = claim_range(r.claims[0], r.claim_ctr, Pg.chunk_log2, blockIdx.x);
  photon_loop(r.g, Pg.admitting, rg, sg, se, tg, majg, lbeams, tot);
  append_round(r, Pe, Pg, se, sg);
  add_totals(tot, r.e.ctr);
}

// ---------------------------------------------------------------- finalize
// Batch k of voxel v, summed over the nsum tallies being finalized together.
__device__ __forceinline__ unsigned long long batch_total(const FinalizeArgs& a, uint32_t k, uint32_t v) {
  unsigned long long t = 0;
  const size_t e = a.blocked ? vox_off(v, a.K) + (size_t)k * kTallyBlock : (size_t)k * a.nvox + v;
  for (uint32_t j = 0; j < a.nsum; ++j) t += a.tally[(size_t)j * a.sum_stride + e];
  return t;
}

// Dose per history and batch uncertainty in double precision (Sec. II.D):
// D = sum_k T_k / N converted to Gy; sigma^2 = sum_k n_k^2 (m_k - m)^2 /
// (N^2 (K-1)/K) with m_k = T_k / n_k the batch means, each term formed as
// (T_k - n_k m)^2 (the same quantity, without a division).  Both forms
// below return the voxel's deposited energy for the integer ledger, and
// give the same bits for the same batches.
//
// General form: any number of batches, nsum tallies added.
__device__ __forceinline__ unsigned long long finalize_general(const FinalizeArgs& a, uint32_t v) {
  unsigned long long s1 = 0;
  for (uint32_t k = 0; k < a.K; ++k) s1 += batch_total(a, k, v);
  const double rho = (double)__uint_as_float(a.vox[v].x);
  const double conv = rho > 0.0 ? a.conv / rho : 0.0;
  const double m = (double)s1 / a.n_total;
  if (a.dose) a.dose[v] = m * conv;
  if (a.sigma) {
    double acc = 0.0;
    for (uint32_t k = 0; k < a.K; ++k) {
      const double nk = a.nk[k];
      if (!(nk > 0.0)) continue;   // a batch without histories adds nothing
      const double d = (double)batch_total(a, k, v) - nk * m;
      acc += d * d;
    }
    const double var = a.K > 1 ? acc / (a.n_total * a.n_total * (double)(a.K - 1) / (double)a.K) : 0.0;
    a.sigma[v] = sqrt(var) * conv;
  }
  return s1;
}

// Register form, for one tally of at most KR batches: a lane issues every
// batch load of its voxel before it uses any (K loads in flight, not one at
// a time), then forms D and sigma from registers with the general form's
// operations in the same order.  The batch sizes come from LDS (nk_lds:
// kFinRegK entries, zero past K), and sigma's sum has no branch: a batch
// without histories adds +0.0 to a sum of non-negative terms, which leaves
// it as it was.
constexpr uint32_t kFinRegK = 32;
template <uint32_t KR>
__device__ __forceinline__ unsigned long long finalize_reg(const FinalizeArgs& a, uint32_t v, const double* nk_lds) {
  const size_t step = a.blocked ? kTallyBlock : a.nvox;
  const unsigned long long* p = a.tally + (a.blocked ? vox_off(v, a.K) : v);
  // batches past K (at most K of them) load batch K-1 again: in bounds,
  // straight-line code with no wait between the loads; they count as zero
  unsigned long long t[KR];
#pragma unroll
  for (uint32_t k = 0; k < KR; ++k) t[k] = p[(size_t)(k < a.K ? k : a.K - 1u) * step];
  const double rho = (double)__uint_as_float(a.vox[v].x);
  unsigned long long s1 = 0;
#pragma unroll
  for (uint32_t k = 0; k < KR; ++k) s1 += k < a.K ? t[k] : 0ull;
  const double conv = rho > 0.0 ? a.conv / rho : 0.0;
  const double m = (double)s1 / a.n_total;
  double sig = 0.0;
  if (a.sigma) {
    double acc = 0.0;
#pragma unroll
    for (uint32_t k = 0; k < KR; ++k) {
      const double nk = nk_lds[k];
      const double d = (double)t[k] - nk * m;
      const double term = d * d;
      acc += nk > 0.0 ? term : 0.0;
    }
    const double var = a.K > 1 ? acc / (a.n_total * a.n_total * (double)(a.K - 1) / (double)a.K) : 0.0;
    sig = sqrt(var) * conv;
  }
  if (a.dose) a.dose[v] = m * conv;
  if (a.sigma) a.sigma[v] = sig;
  return s1;
}

// Every thread of the workgroup calls this (the LDS fill has a barrier).
// KR: the register form's width, 0 for the general form; arguments it does
// not fit (more batches than KR, or several tallies) take the general form.
template <uint32_t KR>
__device__ __forceinline__ void finalize_voxels(const FinalizeArgs& a, uint32_t v) {
  __shared__ double nk_lds[kFinRegK];
  const bool reg = KR > 0 && a.nsum == 1u && a.K >= 1u && a.K <= KR;
  if (reg && a.sigma) {
    if (threadIdx.x < kFinRegK) nk_lds[threadIdx.x] = threadIdx.x < a.K ? a.nk[threadIdx.x] : 0.0;
    __syncthreads();
  }
  unsigned long long s1 = 0;
  if (v < a.nvox) s1 = reg ? finalize_reg<(KR > 0 ? KR : 1u)>(a, v, nk_lds) : finalize_general(a, v);
  const unsigned long long t = wave_sum(s1);
  if (lane_id() == 0 && t && a.ctr) ctr_add(a.ctr, C_E_DEP, t);
}

// One instance per width, so that each has the registers of its own width
// (a lane of the one-batch form holds two loads, not thirty-two, and the
// occupancy that hides their latency).
template <uint32_t KR>
__global__ void __launch_bounds__(256) k_finalize(FinalizeArgs a) {
  finalize_voxels<KR>(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// Many finalizes of one phantom in one launch (the beams of a batched job
// with per-beam results): workgroup row y takes finalize y of the list, with
// the same arithmetic as k_finalize.  The row's arguments are copied before
// any store or barrier, so that they are read once, as uniform scalar loads.
template <uint32_t KR>
__global__ void __launch_bounds__(256) k_finalize_many(const FinalizeArgs* __restrict__ list) {
  const FinalizeArgs a = list[blockIdx.y];
  finalize_voxels<KR>(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// Eq. 12's s: block maxima of D, then per-block sums of sigma/D and counts
// over D > 0.2 D_max, then their totals; every sum in a fixed order.
__device__ __forceinline__ double block_reduce(double v, bool take_max) {
  __shared__ double r[256];
  r[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) r[threadIdx.x] = take_max ? fmax(r[threadIdx.x], r[threadIdx.x + h])
                                                       : r[threadIdx.x] + r[threadIdx.x + h];
    __syncthreads();
  }
  const double out = r[0];
  __syncthreads();
  return out;
}

__global__ void __launch_bounds__(256) k_rel_max(const double* dose, uint32_t nvox, double* work) {
  double m = 0.0;
  for (uint32_t v = blockIdx.x * 256u + threadIdx.x; v < nvox; v += gridDim.x * 256u) m = fmax(m, dose[v]);
  m = block_reduce(m, true);
  if (threadIdx.x == 0) work[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) k_rel_sum(const double* dose, const double* sigma, uint32_t nvox, double* work) {
  double m = 0.0;
  for (int b = 0; b < kRelBlocks; ++b) m = fmax(m, work[b]);
  const double cut = 0.2 * m;
  double s = 0.0, c = 0.0;
  for (uint32_t v = blockIdx.x * 256u + threadIdx.x; v < nvox; v += gridDim.x * 256u) {
    const double d = dose[v];
    if (d > cut) {
      s += sigma[v] / d;
      c += 1.0;
    }
  }
  s = block_reduce(s, false);
  c = block_reduce(c, false);
  if (threadIdx.x == 0) {
    work[kRelBlocks + blockIdx.x] = s;
    work[2 * kRelBlocks + blockIdx.x] = c;
  }
}

__global__ void __launch_bounds__(256) k_rel_final(double* work) {
  const double s = block_reduce(work[kRelBlocks + threadIdx.x], false);
  const double c = block_reduce(work[2 * kRelBlocks + threadIdx.x], false);
  if (threadIdx.x == 0) work[3 * kRelBlocks] = c > 0.0 ? s / c : __longlong_as_double(0x7ff8000000000000ll);
}

// ------------------------------------------------------------------ checks
__global__ void k_rng_words(uint32_t key0, uint32_t key1, uint32_t hist, uint32_t plo, uint32_t phi, uint32_t n0,
                            int count, uint32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t n = n0 + (uint32_t)i;
  const Block b = philox(n >> 2, plo, phi, hist, key0, key1);
  const uint32_t j = n & 3u;
  out[i] = j == 0 ? b.w0 : (j == 1 ? b.w1 : (j == 2 ? b.w2 : b.w3));
}

__global__ void k_table_eval(DevTables t, int which, int mat, const float* e, int n, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (which == 7) {
    const float g1 = e[i];
    out[i] = screening_A(t, t.ms, g1);
    return;
  }
  const TPos p = tpos(t, e[i]);
  if (which <= 2) {
    const float4 c = lerp4(t.ph, mat * kNE, p);
    out[i] = which == 0 ? c.x : (which == 1 ? c.y : c.z);
  } else {
    const float4 c = lerp4(t.el, mat * kNE, p);
    out[i] = which == 3 ? c.x : (which == 4 ? c.y : (which == 5 ? c.z : c.w));
  }
}

// First real photon interaction of each history (checks the stream use, the
// majorant and the table lookups against the oracle history by history).
__global__ void __launch_bounds__(256) k_first_events(PassArgs a, DevSource src, uint32_t h0, uint32_t count,
                                                      float* xyz, uint32_t* nused) {
  extern __shared__ float4 smem[];
  const int nt = a.tab.n_mat * kNE;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) smem[i] = a.tab.ph[i];
  float* majg = reinterpret_cast<float*>(smem + nt);
  for (int i = threadIdx.x; i < kNE; i += blockDim.x) majg[i] = a.tab.maj_g[i];
  __syncthreads();
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t h = h0 + i;
  const DevBeam b = a.beams[0];
  const Primary pr = sample_primary(src, b, h);
  const float nan = __builtin_nanf("");
  xyz[3 * i] = nan; xyz[3 * i + 1] = nan; xyz[3 * i + 2] = nan;
  nused[i] = 0;
  if (!inside(a.ph, pr.x, pr.y, 0.0f) || pr.e < a.cut.pcut_lsb) return;
  Lane L;
  L.x = pr.x; L.y = pr.y; L.z = 0.0f; L.u = 0.0f; L.v = 0.0f; L.w = 1.0f; L.e = pr.e; L.beam = 0;
  L.s.k0 = b.key0; L.s.k1 = b.key1; L.s.hist = h; L.s.plo = 0; L.s.phi = 0; L.s.n = 4;
  L.ta = nullptr;
  L.tb = nullptr;
  uint32_t viol = 0;
  for (int guard = 0; guard < (1 << 20); ++guard) {
    int v0 = 0;
    const int kind = photon_flight(L, a, smem, majg, v0, viol);
    if (kind == PH_ESCAPE) return;
    if (kind != PH_FICT) {
      xyz[3 * i] = L.x; xyz[3 * i + 1] = L.y; xyz[3 * i + 2] = L.z;
      nused[i] = L.s.n;
      return;
    }
  }
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// -------------------------------------------------------------- planning
// Sizes of the next pass from the device-resident counts: at most max_items
// particles, and no more than the free space of both destination buffers
// admits under the worst-case per-visit output (the particles left over are
// carried to the next buffer, one slot each).
__global__ void k_plan_pass(PlanArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t n = *a.n_work;
  const uint32_t no = *a.n_other;
  uint64_t m = n < a.max_items ? n : a.max_items;
  // own outputs (carry-over + per-visit budget) must fit the allocated
  // buffer; outputs to the other type only fill it up to its soft capacity,
  // which leaves every type room for a full pass of its own outputs
  if (a.bud_same > 1) {
    const uint64_t lim = n < a.cap ? (uint64_t)(a.cap - n) / (a.bud_same - 1) : 0u;
    if (m > lim) m = lim;
  }
  if (a.bud_other > 0) {
    const uint64_t lim = no < a.cap_other ? (uint64_t)(a.cap_other - no) / a.bud_other : 0u;
    if (m > lim) m = lim;
  }
  // most items a wavefront gets (whole chunks, dealt round-robin)
  const uint64_t chunks = (m + (1u << a.chunk_log2) - 1u) >> a.chunk_log2;
  uint32_t q = (uint32_t)(((chunks + a.waves - 1) / a.waves) << a.chunk_log2);
  if (q == 0u) q = 1u << a.chunk_log2;
  PassPlan P;
  P.n = n;
  P.m = (uint32_t)m;
  *a.n_work = 0u;                 // the work buffer is consumed by this pass
  *a.n_new = n - (uint32_t)m;     // carried-over particles go to the front of the new buffer
  P.per_wave = q;
  P.chunk_log2 = a.chunk_log2;
  P.seg_same = q * (a.bud_same + a.park_slots);
  P.seg_other = q * a.bud_other;
  P.admitting = (a.sched[0] < a.sched[2] || a.sched[1] < a.sched[3]) ? 1u : 0u;
  *a.plan = P;
}

// Sizes of a round (one lane): the electrons' share first, bounded like an
// electron pass (own outputs within the allocated capacity, photons within
// the soft one), then the photons queued at the round's start, bounded so
// that the electrons they create keep the electron queue within the soft
// capacity; the claim caps (an even share of chunks plus one) and the
// segments those caps need; the claim counters are cleared.
__global__ void k_plan_round(RoundPlanArgs a) {
  // every thread of the one workgroup clears claim counters; thread 0 plans
  for (uint32_t i = threadIdx.x; i < 2u * (uint32_t)kMaxClaimParts; i += blockDim.x) a.claim_ctr[i] = 0u;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t ne = *a.n_work[1], ng = *a.n_work[0];
  const uint64_t s = a.sec;
  uint64_t me = ne < a.max_items ? ne : a.max_items;
  if (s > 0) {
    const uint64_t l1 = ne < a.cap ? (uint64_t)(a.cap - ne) / s : 0u;
    const uint64_t l2 = ng < a.cap_soft ? (uint64_t)(a.cap_soft - ng) / s : 0u;
    if (me > l1) me = l1;
    if (me > l2) me = l2;
  }
  uint64_t mg = ng < a.max_items ? ng : a.max_items;
  if (s > 0) {
    const uint64_t held = (uint64_t)ne + me * s;   // most the electron queue holds after the electron phase
    const uint64_t l3 = held < a.cap_soft ? ((uint64_t)a.cap_soft - held) / s : 0u;
    if (mg > l3) mg = l3;
  }
  const uint32_t ch = 1u << a.chunk_log2;
  const uint32_t ms[2] = {(uint32_t)mg, (uint32_t)me};
  const uint32_t ns[2] = {ng, ne};
  uint32_t caps[2];
  for (int t = 0; t < 2; ++t) {
    const uint64_t chunks = ((uint64_t)ms[t] + ch - 1u) >> a.chunk_log2;
    caps[t] = (uint32_t)(((chunks + a.waves - 1u) / a.waves + 1u) << a.chunk_log2);
    // one partition per workgroup, of at least two chunks each
    uint64_t parts = chunks >> 1;
    const uint64_t most = a.blocks < (uint32_t)kMaxClaimParts ? a.blocks : (uint32_t)kMaxClaimParts;
    if (parts > most) parts = most;
    if (parts < 1u) parts = 1u;
    ClaimType c;
    c.cap = caps[t];
    c.m = ms[t];
    c.parts = (uint32_t)parts;
    a.claims[t] = c;
    *a.n_work[t] = 0u;
    *a.n_new[t] = ns[t] - ms[t];
  }
  const uint32_t admitting = (a.sched[0] < a.sched[2] || a.sched[1] < a.sched[3]) ? 1u : 0u;
  // electron outputs: survivors, secondaries and the parked stack of the
  // electron phase, the photon phase's electrons; photon outputs:
  // bremsstrahlung of the electron phase, survivors and the parked stack of
  // the photon phase
  const uint64_t seg_e = (uint64_t)caps[1] * (s + 2u) + (uint64_t)caps[0] * s;
  const uint64_t seg_g = (uint64_t)caps[1] * s + 2ull * caps[0];
  for (int t = 0; t < 2; ++t) {
    PassPlan P;
    P.n = ns[t];
    P.m = ms[t];
    P.per_wave = caps[t];
    P.chunk_log2 = a.chunk_log2;
    P.seg_same = (uint32_t)(t == 1 ? seg_e : seg_g);
    P.seg_other = (uint32_t)(t == 1 ? seg_g : seg_e);
    P.admitting = admitting;
    a.plan[t] = P;
  }
}

// ------------------------------------------------------ energy regrouping
// Sort key: bucket 4 log2(e) + the two bits below the leading one, reversed
// so that the highest energies come first; zero-energy entries go last.
__device__ __forceinline__ uint32_t sort_key(uint32_t e) {
  if (e == 0u) return kSortBuckets - 1u;
  const uint32_t lg = 31u - (uint32_t)__clz(e);
  const uint32_t sub = lg >= 2u ? (e >> (lg - 2u)) & 3u : (e << (2u - lg)) & 3u;
  return (uint32_t)(kSortBuckets - 1) - min((lg << 2) | sub, (uint32_t)(kSortBuckets - 2));
}

// Bucket counts of all entries (grid-stride, one LDS histogram per workgroup).
__global__ void __launch_bounds__(256) k_sort_count(SortArgs a) {
  __shared__ uint32_t h[kSortBuckets];
  for (int b = threadIdx.x; b < kSortBuckets; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const uint32_t n = *a.n;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicAdd(&h[sort_key(qf(a.src, Q_E, i))], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < kSortBuckets; b += blockDim.x)
    if (h[b]) atomicAdd(a.hist + b, h[b]);
}

// Bucket starts (exclusive prefix sum in key order); the counts are cleared
// for the next sort.  One workgroup of kSortBuckets threads.
__global__ void __launch_bounds__(kSortBuckets) k_sort_offsets(SortArgs a) {
  __shared__ uint32_t c[kSortBuckets];
  const int b = threadIdx.x;
  c[b] = a.hist[b];
  __syncthreads();
  uint32_t start = 0u;
  for (int j = 0; j < b; ++j) start += c[j];
  a.cursor[b] = start;
  a.hist[b] = 0u;
}

// Every entry to its bucket: each workgroup counts a tile of entries in LDS,
// reserves room per bucket with one atomic each, and writes its entries
// there (the queue count is unchanged).
constexpr uint32_t kSortTile = 2048;
__global__ void __launch_bounds__(256) k_sort_scatter(SortArgs a) {
  __shared__ uint32_t h[kSortBuckets];
  __shared__ uint32_t base[kSortBuckets];
  const uint32_t n = *a.n;
  for (uint32_t t0 = blockIdx.x * kSortTile; t0 < n; t0 += gridDim.x * kSortTile) {
    const uint32_t t1 = min(t0 + kSortTile, n);
    for (int b = threadIdx.x; b < kSortBuckets; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    for (uint32_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) atomicAdd(&h[sort_key(qf(a.src, Q_E, i))], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < kSortBuckets; b += blockDim.x) {
      base[b] = h[b] ? atomicAdd(a.cursor + b, h[b]) : 0u;
      h[b] = 0u;
    }
    __syncthreads();
    for (uint32_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
      const uint32_t key = sort_key(qf(a.src, Q_E, i));
      const uint32_t slot = base[key] + atomicAdd(&h[key], 1u);
      for (int f = 0; f < Q_FIELDS; ++f) qf(a.dst, f, slot) = qf(a.src, f, i);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers
// Tables, majorant, (screening table,) beam table.
size_t photon_lds_bytes(int n_mat) {
  return (size_t)n_mat * kNE * sizeof(float4) + kNE * sizeof(float) + kLdsBeams * sizeof(DevBeam);
}
size_t electron_lds_bytes(int n_mat) {
  return (size_t)n_mat * kNE * sizeof(float4) + kNE * sizeof(float) + kNms * sizeof(float) +
         kLdsBeams * sizeof(DevBeam);
}

// Both table blocks and the beam table.
size_t round_lds_bytes(int n_mat) {
  return 2 * (size_t)n_mat * kNE * sizeof(float4) + 2 * kNE * sizeof(float) + kNms * sizeof(float) +
         kLdsBeams * sizeof(DevBeam);
}

// The pass kernels' dynamic-LDS limit is raised once, to what the largest
// table set needs (occupancy follows the size each launch asks for), so that
// launches -- also those recorded into a graph -- set no attributes.
static hipError_t lds_limits() {
  static const hipError_t e = [] {
    hipError_t r = hipFuncSetAttribute((const void*)k_photon_pass, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)photon_lds_bytes(kMaxMat));
    if (r == hipSuccess)
      r = hipFuncSetAttribute((const void*)k_electron_pass, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)electron_lds_bytes(kMaxMat));
    if (r == hipSuccess)
      r = hipFuncSetAttribute((const void*)k_round, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)round_lds_bytes(kMaxRoundMat));
    return r;
  }();
  return e;
}

hipError_t launch_sort(const SortArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_count, dim3(grid), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sort_offsets, dim3(1), dim3(kSortBuckets), 0, s, a);
  hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_plan_pass(const PlanArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_pass, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_admit_plan(const AdmitPlanArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_admit_plan, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_admit(const AdmitArgs& a, uint32_t max_count, hipStream_t s) {
  if (max_count == 0 || a.nb == 0) return hipSuccess;
  const uint32_t grid = (max_count + 255u) / 256u;
  hipLaunchKernelGGL(k_admit, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_photon_pass(const PassArgs& a, int grid, int block, hipStream_t s) {
  const size_t lds = photon_lds_bytes(a.tab.n_mat);
  const hipError_t e = lds_limits();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_photon_pass, dim3(grid), dim3(block), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_plan_round(const RoundPlanArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_round, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_round(const RoundArgs& a, int grid, int block, hipStream_t s) {
  if (a.e.tab.n_mat > kMaxRoundMat) return hipErrorInvalidValue;
  const size_t lds = round_lds_bytes(a.e.tab.n_mat);
  const hipError_t e = lds_limits();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_round, dim3(grid), dim3(block), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_electron_pass(const PassArgs& a, int grid, int block, hipStream_t s) {
  const size_t lds = electron_lds_bytes(a.tab.n_mat);
  const hipError_t e = lds_limits();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_electron_pass, dim3(grid), dim3(block), lds, s, a);
  return hipGetLastError();
}

// Thread i writes slice-major element i (batch i / nvox, voxel i mod nvox):
// coalesced stores, reads one line per 16 threads.
__global__ void __launch_bounds__(256) k_tally_to_slices(const unsigned long long* in, unsigned long long* out,
                                                         uint32_t nvox, uint32_t K) {
  const size_t n = (size_t)nvox * K;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)(i / nvox), v = (uint32_t)(i % nvox);
    out[i] = in[vox_off(v, K) + (size_t)k * kTallyBlock];
  }
}

hipError_t launch_tally_to_slices(const unsigned long long* blocked, unsigned long long* slices, uint32_t nvox,
                                  uint32_t K, hipStream_t s) {
  const size_t n = (size_t)nvox * K;
  if (n == 0) return hipSuccess;
  const int grid = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_tally_to_slices, dim3(grid), dim3(256), 0, s, blocked, slices, nvox, K);
  return hipGetLastError();
}

// The narrowest register form that holds K batches of one tally, else 0
// (the general form).
static uint32_t finalize_width(uint32_t K, uint32_t nsum) {
  if (nsum != 1u || K < 1u || K > kFinRegK) return 0u;
  return K == 1u ? 1u : K <= 4u ? 4u : K <= 8u ? 8u : K <= 16u ? 16u : kFinRegK;
}

template <uint32_t KR>
static void finalize_many_rows(const FinalizeArgs* d_list, uint32_t n, uint32_t nvox, hipStream_t s) {
  for (uint32_t j0 = 0; j0 < n; j0 += 65535u) {   // rows of a grid
    const uint32_t rows = std::min(n - j0, 65535u);
    hipLaunchKernelGGL(k_finalize_many<KR>, dim3((nvox + 255) / 256, rows), dim3(256), 0, s, d_list + j0);
  }
}

hipError_t launch_finalize_many(const FinalizeArgs* d_list, uint32_t n, uint32_t nvox, uint32_t K, uint32_t nsum,
                                hipStream_t s) {
  switch (finalize_width(K, nsum)) {
    case 1u: finalize_many_rows<1u>(d_list, n, nvox, s); break;
    case 4u: finalize_many_rows<4u>(d_list, n, nvox, s); break;
    case 8u: finalize_many_rows<8u>(d_list, n, nvox, s); break;
    case 16u: finalize_many_rows<16u>(d_list, n, nvox, s); break;
    case kFinRegK: finalize_many_rows<kFinRegK>(d_list, n, nvox, s); break;
    default: finalize_many_rows<0u>(d_list, n, nvox, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  const int grid = (int)((a.nvox + 255) / 256);
  switch (finalize_width(a.K, a.nsum)) {
    case 1u: hipLaunchKernelGGL(k_finalize<1u>, dim3(grid), dim3(256), 0, s, a); break;
    case 4u: hipLaunchKernelGGL(k_finalize<4u>, dim3(grid), dim3(256), 0, s, a); break;
    case 8u: hipLaunchKernelGGL(k_finalize<8u>, dim3(grid), dim3(256), 0, s, a); break;
    case 16u: hipLaunchKernelGGL(k_finalize<16u>, dim3(grid), dim3(256), 0, s, a); break;
    case kFinRegK: hipLaunchKernelGGL(k_finalize<kFinRegK>, dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_finalize<0u>, dim3(grid), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_rel_uncertainty(const double* dose, const double* sigma, uint32_t nvox, double* work,
                                  hipStream_t s) {
  static_assert(kRelBlocks == 256, "k_rel_final reduces one block of 256 partials");
  hipLaunchKernelGGL(k_rel_max, dim3(kRelBlocks), dim3(256), 0, s, dose, nvox, work);
  hipLaunchKernelGGL(k_rel_sum, dim3(kRelBlocks), dim3(256), 0, s, dose, sigma, nvox, work);
  hipLaunchKernelGGL(k_rel_final, dim3(1), dim3(256), 0, s, work);
  return hipGetLastError();
}

hipError_t launch_rng_words(uint32_t key0, uint32_t key1, uint32_t hist, uint32_t plo, uint32_t phi, uint32_t n0,
                            int count, uint32_t* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rng_words, dim3((count + 255) / 256), dim3(256), 0, s, key0, key1, hist, plo, phi, n0, count,
                     out);
  return hipGetLastError();
}

hipError_t launch_table_eval(const DevTables& t, int which, int mat, const float* e, int n, float* out,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_table_eval, dim3((n + 255) / 256), dim3(256), 0, s, t, which, mat, e, n, out);
  return hipGetLastError();
}

hipError_t launch_first_events(const PassArgs& a, const DevSource& src, uint32_t h0, uint32_t count, float* xyz,
                               uint32_t* nused, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t lds = photon_lds_bytes(a.tab.n_mat);
  const hipError_t e = hipFuncSetAttribute((const void*)k_first_events, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)photon_lds_bytes(kMaxMat));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_first_events, dim3((count + 255) / 256), dim3(256), lds, s, a, src, h0, count, xyz, nused);
  return hipGetLastError();
}

// Atomic-rate microbenchmark: lane t adds 1 to 64 words of a + (0..mask),
// at hashed addresses (a 32-bit xorshift-multiply finaliser), or (hot > 0)
// to word t mod hot, through the same global atomic as the tallies.
constexpr int kAtomicPerLane = 64;
constexpr int kAtomicBlocks = 4096;
static_assert(kAtomicRateAdds == (uint64_t)kAtomicBlocks * 256u * kAtomicPerLane, "additions per launch");
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void __launch_bounds__(256) k_atomic_rate(unsigned long long* a, uint32_t mask, uint32_t hot) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int j = 0; j < kAtomicPerLane; ++j) {
    const uint32_t i = hot ? (t & (hot - 1u)) : (mix32(t * 977u + (uint32_t)j * 131071u) & mask);
    tally_add(a + i, 1ull);
  }
}

hipError_t launch_atomic_rate(unsigned long long* a, uint32_t mask, uint32_t hot, hipStream_t s) {
  hipLaunchKernelGGL(k_atomic_rate, dim3(kAtomicBlocks), dim3(256), 0, s, a, mask, hot);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ------------------------------------------------ allocation-free finalize
// The work memory of gmc_finalize_tally_noalloc lives here instead of in
// memory the library allocates.  Host code never uses the array's name as an
// address: it takes the device address hipGetSymbolAddress returns for the
// current device, once per device, and passes that to the kernels.
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static double* g_scratch_addr[kScratchDevices] = {};

hipError_t scratch_resolve(int device) {
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_addr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* scratch_address(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_addr[device];
}

// #{h in [h0, h0 + n) : h mod K = k}, from #{h < m : h mod K = k} = (m + K - 1 - k) / K.
__global__ void k_batch_sizes(double* nk, unsigned long long h0, unsigned long long n, uint32_t K) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) nk[k] = (double)((h0 + n + K - 1 - k) / K - (h0 + K - 1 - k) / K);
}

hipError_t launch_batch_sizes(double* nk, uint64_t h0, uint64_t n, uint32_t K, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_sizes, dim3((K + 255u) / 256u), dim3(256), 0, s, nk, (unsigned long long)h0,
                     (unsigned long long)n, K);
  return hipGetLastError();
}

int max_resident_blocks(int kernel, int block, size_t lds) {
  int per_cu = 0;
  const void* fn = kernel == 0 ? (const void*)k_photon_pass
                   : kernel == 1 ? (const void*)k_electron_pass : (const void*)k_round;
  (void)lds_limits();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess || per_cu <= 0) per_cu = 1;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus <= 0) cus = 256;
  return per_cu * cus;
}

}  // namespace gmc
