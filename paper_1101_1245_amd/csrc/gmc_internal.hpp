// gmc_internal.hpp -- device-visible data layout shared by the host runtime and
// the gfx950 kernels of the transport engine.
//
// Memory layout in HBM (all linear, no textures):
//  * phantom: one uint2 per voxel {float bits of density, material index},
//    [nz][ny][nx], so a voxel costs one 8-byte gather (Sec. II.C.2 keeps
//    composition and density in two 3D textures);
//  * tables: FP32 nodes on a log-energy grid, one float4 per (material, node),
//    staged into LDS by each workgroup;
//  * particles: structure-of-arrays queues, 48 bytes per particle, two
//    buffers per particle type (one being consumed, one accumulating);
//  * tallies: uint64 fixed-point energy (2^-27 MeV) per (batch, voxel).
//
// Pass sizes live on the device: a one-lane planning kernel reads the queue
// counts and writes a PassPlan that the pass kernel reads, so
// a sequence of passes can be enqueued (or captured in a graph) without the
// host reading counts in between.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmc {

constexpr int kNE = 1024;               // log-energy nodes on [kEmin, kEmax]
constexpr double kEmin = 1.0e-3;        // MeV
constexpr double kEmax = 32.0;          // MeV (the fixed-point energy range)
constexpr int kNms = 512;               // nodes of the multiple-scattering screening table
constexpr int kMaxMat = 8;
// Tally layout inside the library: voxels in blocks of kTallyBlock, each
// batch's sums of a block on one 128-byte line, and the block's K lines
// adjacent -- the sum of batch k in voxel v at
// (v / kTallyBlock) kTallyBlock K + k kTallyBlock + v mod kTallyBlock, over
// tally_vox(nvox) voxels (the last block padded).  Batches never share a
// line, so the additions of a narrow beam's histories to its few voxels do
// not contend for one, and a voxel's batches stay within a few kilobytes.
// The raw tallies of the C ABI are slice-major ([K][nvox]) instead.
constexpr uint32_t kTallyBlock = 16;
inline size_t tally_vox(size_t nvox) { return (nvox + kTallyBlock - 1) / kTallyBlock * kTallyBlock; }
constexpr int kMaxBatches = 1024;
constexpr double kLsbMeV = 1.0 / 134217728.0;   // 2^-27 MeV per energy unit

struct DevPhantom {
  const uint2* vox;
  int nx, ny, nz;
  float dx, dy, dz;
  float idx, idy, idz;
  float lx, ly, lz;
  float skin;         // 1e-4 of the smallest voxel width
};

struct DevTables {
  const float4* ph;     // [n_mat][kNE] {mu_C, mu_C + mu_pe, mu_total, 0} per unit density, cm^2/g
  const float4* el;     // [n_mat][kNE] {L, Sigma_M, Sigma_B, 1/lambda_1} per unit density
  const float* ms;      // [kNms] ln A at evenly spaced logit(G1)
  const float* maj_g;   // [kNE] photon majorant per grid bin, cm^-1
  const float* maj_e;   // [kNE] electron hard-event majorant per grid bin, cm^-1
  int n_mat;
  float lg2_emin;       // log2(kEmin)
  float inv_h2;         // grid nodes per unit of log2 E
  float ms_y0;          // logit(G1) of the first screening node
  float ms_inv_dy;      // nodes per unit of logit(G1)
};

struct DevCuts {
  uint32_t ecut_lsb, pcut_lsb;   // transport cutoffs in energy units
  uint32_t kcut2_lsb, kc_lsb;    // Moller needs T > 2 K_cut; brems needs T > k_c
  uint32_t two_mc2_lsb;          // pair threshold and rest-energy sink
  float kcut, kc;                // MeV
  float esmax_gcm2;              // <= 0: none
  float emin;                    // lowest table energy, MeV
  int mode;                      // 0 full, 1 photon first collision, 2 electron CSDA straight-ahead
};

// Structure-of-arrays particle queue: field f of entry i is the 32-bit word
// base[f * stride + i].  Fields: position x y z and direction u v w (float
// bits), kinetic energy in 2^-27 MeV units, history index, stream path (two
// words), stream word counter, beam index.
enum QueueField { Q_X = 0, Q_Y, Q_Z, Q_U, Q_V, Q_W, Q_E, Q_HIST, Q_PLO, Q_PHI, Q_N, Q_BEAM, Q_FIELDS };
// Staging entries carry four words more for an electron parked at a
// hard-event candidate: the step-start majorant (float bits), its visit
// counters (events | pushes << 16) and its pending deposit (voxel, energy).
constexpr int Q_AUX = Q_FIELDS;
constexpr int Q_AUX2 = Q_FIELDS + 1;
constexpr int Q_PV = Q_FIELDS + 2;
constexpr int Q_PE = Q_FIELDS + 3;
constexpr int kStgFields = Q_FIELDS + 4;
struct DevQueue {
  uint32_t* base;
  uint32_t stride;
  uint32_t cap;
};

// One tally target: K batch sums per voxel in the blocked layout above, from
// base (null: no target).  History h of the beam goes to batch (off + h) mod
// K, off < K (the host reduces it); interleaved batches keep every run of consecutive histories spread over
// all K batches, so lanes working on neighbouring histories rarely add to the
// same address.
struct DevTally {
  unsigned long long* base;
  uint32_t K, off;
};

// A beam: its stream key and up to two tally targets.  Target a is the
// beam's own tally (K batches, or 1 when only its dose is needed); target b,
// when set, is a combined tally batched over all beams' histories.
struct DevBeam {
  uint32_t key0, key1;          // Philox key (seed lo, seed hi ^ beam id)
  DevTally a, b;
};
// Beams whose table the pass kernels keep in LDS (beside the physics tables):
// a particle's refill then reads its beam's key and tally slices without a
// second dependent global load.  Jobs with more beams read it from memory.
constexpr int kLdsBeams = 256;

// A beam's source, on the device for the admission kernel.
struct DevSource {
  int particle, spectrum;
  uint32_t e_lsb;               // monoenergetic energy
  float e_lo, e_mode, e_hi;     // triangular spectrum
  float cx, cy, wx, wy;
  const double* tab;            // tabulated: bin edges [tab_n + 1], then the normalised CDF at them [tab_n + 1]
  uint32_t tab_n;
  uint32_t h0;                  // number of the beam's first history (its stream and batch)
};

// Run counters (energy ledger in 2^-27 MeV units, event counts).  Each counter
// is spread over kCtrSlots words, picked by wavefront, so that the per-wave
// additions at the end of every kernel do not all hit one address; the host
// sums the slots.  C_E_DEP is the deposited total summed by the finalize.
enum CounterIndex {
  C_E_IN = 0, C_E_ESC, C_E_SINK, C_PH_EVENTS, C_FICT, C_VIOL, C_E_STEPS, C_HARD, C_SEC, C_OVERFLOW, C_E_DEP,
  C_PH_REAL, C_COUNT
};
constexpr int kCtrSlots = 256;

// Sizes of one pass, written by k_plan_pass.  The work buffer holds n
// particles; this pass transports the first m, dealt to the wavefronts in
// chunks of 2^chunk_log2 (chunk c to wavefront c mod W), at most per_wave
// each; each wavefront has staging segments of seg_same / seg_other slots.
// Particles m..n-1 are carried over to the next buffer.
struct PassPlan {
  uint32_t n, m, per_wave, seg_same, seg_other, chunk_log2;
  uint32_t admitting;   // primaries remain to be admitted: more passes of both types follow
};

// The device work queue of the persistent round kernel, per particle type:
// the round's m items split into `parts` contiguous partitions, partition p
// holding items [m p / parts, m (p+1) / parts) and a chunk counter of its
// own, and the most items one wavefront may claim.  Workgroup b claims from
// partition b mod parts first, so a claim is normally an atomic that only
// its own workgroup's wavefronts share.
constexpr int kMaxClaimParts = 4096;
struct ClaimType {
  uint32_t cap;
  uint32_t m;
  uint32_t parts;
};

struct PlanArgs {
  uint32_t* n_work;             // count of the work buffer (read, then cleared)
  uint32_t* n_new;              // count of the type's new accumulating buffer: set to the carry-over
  const uint32_t* n_other;      // count of the other type's accumulating buffer
  PassPlan* plan;
  uint32_t cap;                 // allocated queue capacity (bounds this type's own outputs)
  uint32_t cap_other;           // soft capacity the outputs to the other type must respect
  uint32_t max_items;           // most particles per pass
  uint32_t waves;               // wavefronts in the pass grid
  uint32_t chunk_log2;          // items per chunk dealt to a wavefront: 2^chunk_log2 (>= 64)
  uint32_t bud_same, bud_other; // per-visit output budgets per particle
  uint32_t park_slots;          // same-type staging slots per particle for parked electrons
  const uint32_t* sched;        // admission cursors [2] and totals [2]
};

// A pass kernel's work: each wave of the grid owns its chunks of the work
// queue (at most per_wave items), refills its lanes from them, and appends
// survivors and secondaries to its own segments of two staging queues
// (same type / other type) -- no atomics on shared counters while it
// transports.  When a workgroup is done, one atomic per destination reserves
// room for all of its waves' entries in the accumulating queues and each
// wave copies its segments there; particles the pass did not take (m..n-1)
// are copied to the front of the type's new queue.  Queue order then depends
// on which workgroups finish first; no result does (every particle carries its
// own stream and tallies are integer sums).
struct PassArgs {
  DevPhantom ph;
  DevTables tab;
  DevCuts cut;
  DevQueue work;           // items 0..m-1 of the pass
  DevQueue carry_src;      // items m..n-1, carried over (the work buffer, or the unsorted one)
  const PassPlan* plan;
  DevQueue stg_same;       // survivors and same-type secondaries
  DevQueue stg_other;      // other-type secondaries
  DevQueue dst_same;       // the type's new accumulating queue (carry-over in front)
  DevQueue dst_other;      // the other type's accumulating queue
  uint32_t* cnt_same;      // their counts
  uint32_t* cnt_other;
  const DevBeam* beams;
  int n_beams;
  unsigned long long* ctr;   // [C_COUNT][kCtrSlots]
  int max_events;
  int max_secondaries;
  int refill_lanes;          // idle lanes (1..64) that trigger a refill
  int resume_lanes;          // idle lanes (1..64) that take back parked electrons
  int tail_lanes;            // requeue the lanes' particles once the share is done and at most this many remain
  uint32_t tail_min;         // ... for shares of at least this many particles
  int agg_a;                 // electron pass: tally-a additions of a loop iteration aggregated per address
  uint32_t ka, kb;           // batches of the beams' tally targets a and b, the same for every beam
};

// The persistent round kernel: one launch per round transports the
// electrons and then the photons of the round's work queues, every
// wavefront claiming chunks of items from the device work queue (ClaimType
// per type, with its counters) instead of a fixed share.  g and e are the
// photon and electron halves as pass arguments: each reads its own work
// queue and plan; electron outputs go to staging queue 0 (e.stg_same,
// g.stg_other) and photon outputs to staging queue 1.
struct RoundArgs {
  PassArgs g, e;
  const ClaimType* claims;      // [2] photon, electron
  uint32_t* claim_ctr;          // [2][kMaxClaimParts] chunk counters (cleared by the plan)
};

// Sizes of a round: both types' plans as k_plan_pass would make them in
// sequence (electrons first; the photons transported in the round are those
// queued at its start), the per-wavefront claim caps and segments.
struct RoundPlanArgs {
  uint32_t* n_work[2];          // counts of the work buffers (read, then cleared)
  uint32_t* n_new[2];           // counts of the new accumulating buffers: set to the carry-overs
  PassPlan* plan;               // [2]
  ClaimType* claims;            // [2]
  uint32_t* claim_ctr;          // [2][kMaxClaimParts]
  uint32_t cap, cap_soft;       // allocated and soft queue capacity
  uint32_t max_items;           // most particles of a type per round
  uint32_t waves;               // wavefronts of the round grid
  uint32_t blocks;              // workgroups of the round grid
  uint32_t chunk_log2;          // items per claimed chunk: 2^chunk_log2
  uint32_t sec;                 // secondaries per visit
  const uint32_t* sched;        // admission cursors [2] and totals [2]
};

// Admission of primaries of one particle type.  The histories of all beams of
// that type are numbered consecutively (beam j of the type owns
// [start[j], start[j+1])); each admission takes the next `count` of them,
// stored from `base` on in the type's accumulating buffer.
struct AdmitPlan {
  uint32_t base, count, cursor;
};

struct AdmitPlanArgs {
  uint32_t* cursor;             // next history to admit, per type [2]
  const uint32_t* total;        // histories per type [2]
  uint32_t* count0;             // accumulating photon count
  uint32_t* count1;             // accumulating electron count
  AdmitPlan* out;               // [2]
  uint32_t cap, chunk;          // cap: the soft queue capacity
};

struct AdmitArgs {
  DevPhantom ph;
  DevCuts cut;
  DevQueue out;
  const AdmitPlan* plan;
  const uint32_t* start;        // [nb + 1] first job-wide index of each admission segment of this type
  const uint32_t* beam_of;      // [nb] beam of each segment
  const uint32_t* seg_h;        // [nb] index in its beam of each segment's first history
  uint32_t nb;                  // segments
  const DevBeam* beams;
  const DevSource* sources;     // indexed by beam
  unsigned long long* ctr;
  uint32_t ka, kb;              // as in PassArgs
};

// Energy regrouping of a work queue before its pass (the grouping of
// particles of similar energy that Sec. IV.B proposes against the divergence
// of polyenergetic beams): a counting sort on log-energy buckets, four per
// octave of the 2^-27 MeV units, highest energy first, so that the lanes of a
// chunk hold particles of similar energy and every wavefront takes its
// longest-lived particles first.  Order within a bucket is whatever the
// atomics give: no result depends on queue order.
constexpr int kSortBuckets = 128;
struct SortArgs {
  DevQueue src, dst;            // dst: room for n entries
  const uint32_t* n;            // entries to regroup: the first n of src (the pass's m)
  uint32_t* hist;               // [kSortBuckets] counts; zero before and after a sort
  uint32_t* cursor;             // [kSortBuckets] next free slot of each bucket in dst
};

struct FinalizeArgs {
  const unsigned long long* tally;  // nsum tallies sum_stride apart (added), each blocked or [K][nvox]
  uint32_t nsum;
  size_t sum_stride;                // elements between successive tallies
  const uint2* vox;
  const double* nk;                 // histories per batch
  uint32_t nvox, K;
  double n_total, conv;             // conv = LSB * J/MeV / (V * 1e-3 kg/g)
  double* dose;                     // may be null in k_finalize_many (sigma only)
  double* sigma;                    // may be null
  unsigned long long* ctr;          // [C_COUNT][kCtrSlots], gets C_E_DEP (may be null)
  uint32_t blocked;                 // 1: the library's blocked layout; 0: slice-major [K][nvox]
};

// Launchers (gmc_kernels.hip).
size_t photon_lds_bytes(int n_mat);
size_t electron_lds_bytes(int n_mat);
hipError_t launch_plan_pass(const PlanArgs& a, hipStream_t s);
hipError_t launch_photon_pass(const PassArgs& a, int grid, int block, hipStream_t s);
size_t round_lds_bytes(int n_mat);
constexpr int kMaxRoundMat = 4;        // both table blocks of more materials do not fit in LDS
hipError_t launch_plan_round(const RoundPlanArgs& a, hipStream_t s);
hipError_t launch_round(const RoundArgs& a, int grid, int block, hipStream_t s);
hipError_t launch_electron_pass(const PassArgs& a, int grid, int block, hipStream_t s);
hipError_t launch_admit_plan(const AdmitPlanArgs& a, hipStream_t s);
hipError_t launch_admit(const AdmitArgs& a, uint32_t max_count, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
// n finalizes of one phantom (nvox voxels each), their arguments at d_list in
// device memory, all with the same K and nsum (a null dose skips the dose).
hipError_t launch_finalize_many(const FinalizeArgs* d_list, uint32_t n, uint32_t nvox, uint32_t K, uint32_t nsum,
                                hipStream_t s);
// A blocked tally (nvox voxels, K batches) rewritten slice-major, [K][nvox].
hipError_t launch_tally_to_slices(const unsigned long long* blocked, unsigned long long* slices, uint32_t nvox,
                                  uint32_t K, hipStream_t s);
hipError_t launch_rng_words(uint32_t key0, uint32_t key1, uint32_t hist, uint32_t plo, uint32_t phi, uint32_t n0,
                            int count, uint32_t* out, hipStream_t s);
hipError_t launch_table_eval(const DevTables& t, int which, int mat, const float* e, int n, float* out,
                             hipStream_t s);
hipError_t launch_first_events(const PassArgs& a, const DevSource& src, uint32_t h0, uint32_t count, float* xyz,
                               uint32_t* nused, hipStream_t s);
hipError_t launch_sort(const SortArgs& a, int grid, hipStream_t s);
constexpr uint64_t kAtomicRateAdds = 4096ull * 256ull * 64ull;   // additions per microbenchmark launch
// Eq. 12's s of a dose and sigma array: mean sigma/D over voxels with
// D > 0.2 D_max, by fixed-order reductions (the same inputs give the same
// bits).  work holds kRelBlocks block maxima, sums and counts, then s.
constexpr int kRelBlocks = 256;
hipError_t launch_rel_uncertainty(const double* dose, const double* sigma, uint32_t nvox, double* work, hipStream_t s);
hipError_t launch_atomic_rate(unsigned long long* a, uint32_t mask, uint32_t hot, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s);
// kernel: 0 photon pass, 1 electron pass, 2 round kernel
int max_resident_blocks(int kernel, int block, size_t lds);

// Largest workgroup of the round kernel: it holds the electron and the photon
// loop, whose registers together exceed what a 1024-thread workgroup leaves
// each lane (128), so it is bounded at 512 threads (up to 256 registers)
// rather than spill.
constexpr int kRoundMaxBlock = 512;

// Work memory of the allocation-free finalize: a file-scope device array of
// the kernels' source, one copy per device, never freed.  It holds the
// histories per batch (kMaxBatches doubles) and then the s reduction's work
// (3 kRelBlocks + 1 doubles).
constexpr size_t kScratchDoubles = (size_t)kMaxBatches + 3 * (size_t)kRelBlocks + 1;
constexpr int kScratchDevices = 64;
// Resolve the array's address on `device` (which must be current): done once
// per device, at context creation.
hipError_t scratch_resolve(int device);
// Its address on `device` (nullptr before scratch_resolve succeeded there).
double* scratch_address(int device);
// nk[k] = histories of [h0, h0 + n) in batch k (h mod K), k < K.
hipError_t launch_batch_sizes(double* nk, uint64_t h0, uint64_t n, uint32_t K, hipStream_t s);

}  // namespace gmc
