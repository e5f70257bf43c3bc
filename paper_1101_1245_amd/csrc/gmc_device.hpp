// gmc_device.hpp -- FP32 device building blocks of the gfx950 transport kernels:
// per-particle counter-based streams, log-grid table interpolation from LDS,
// voxel geometry, direction rotation and the interaction samplers.
//
// Every sampler consumes uniforms from the particle's own stream in a fixed
// order, so a particle's trajectory depends on its state and stream only,
// never on which lane, wavefront or pass runs it.
#pragma once
#include "gmc_internal.hpp"

namespace gmc {
namespace dev {

constexpr float kMc2 = 0.51099895f;                 // MeV
constexpr float kTwoPi = 6.28318530717958648f;
constexpr float kPi = 3.14159265358979324f;
constexpr float kLsbF = 7.450580596923828125e-09f;  // 2^-27 MeV per energy unit
constexpr float kInvLsbF = 134217728.0f;            // 2^27
constexpr float kU24 = 5.9604644775390625e-08f;     // 2^-24
constexpr float kInf = __builtin_huge_valf();
constexpr float kMaxLsbF = 4294967040.0f;           // largest float below 2^32
// Multiple scattering is drawn isotropically at or above this first moment.
constexpr float kG1Iso = 0.9999f;
constexpr float kLn2 = 0.693147180559945309f;
constexpr float kLog2e = 1.44269504088896341f;

// ---------------------------------------------------------------- fast FP32 forms
// Reciprocal, quotient, natural log and exponential of the transport as the
// hardware's v_rcp_f32, v_log_f32 (log2) and v_exp_f32 (exp2), each within
// about 1 ulp, and at most one multiply.  The general forms add range scaling
// for operands beyond 2^96 and an extended-precision ln 2 product; no operand
// here comes near such ranges (denormals are flushed, uniforms lie in
// [2^-24, 1), energies in [1 keV, 32 MeV], lengths and cross sections far
// inside), so those steps would only cost instructions.
__device__ __forceinline__ float frcp(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float fln(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }

// ---------------------------------------------------------------- Philox4x32-10
struct Block { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ Block philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    // one 32x32->64 multiply each (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input exclusive or as one gfx950 v_bitop3_b32 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
  }
  return Block{c0, c1, c2, c3};
}

__device__ __forceinline__ float to_uniform(uint32_t w) { return (float)((w >> 8) | 1u) * kU24; }

// Stream path of a child: splitmix64 finalizer of the parent path mixed with
// the parent's word counter at the spawning event and the child's index.
__device__ __forceinline__ void child_path(uint32_t plo, uint32_t phi, uint32_t n, uint32_t idx, uint32_t& olo,
                                           uint32_t& ohi) {
  uint64_t z = ((uint64_t)phi << 32) | (uint64_t)plo;
  z = (z ^ (((uint64_t)n << 2) | (uint64_t)idx)) + 0x9E3779B97F4A7C15ull;
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27; z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  olo = (uint32_t)z;
  ohi = (uint32_t)(z >> 32);
}

// A particle's stream: word n is word (n & 3) of Philox4x32-10 with counter
// (n >> 2, path lo, path hi, history) and key (seed lo, seed hi ^ beam id).
// Each event starts on a block boundary (align), so the block refresh falls on
// the same draw for every lane of a wavefront.
struct Stream {
  uint32_t k0, k1, plo, phi, hist, n;
  uint32_t b0, b1, b2, b3;

  __device__ __forceinline__ void align() { n = (n + 3u) & ~3u; }
  __device__ __forceinline__ uint32_t word() {
    const uint32_t j = n & 3u;
    if (j == 0) {
      const Block b = philox(n >> 2, plo, phi, hist, k0, k1);
      b0 = b.w0; b1 = b.w1; b2 = b.w2; b3 = b.w3;
    }
    const uint32_t wd = j == 0 ? b0 : (j == 1 ? b1 : (j == 2 ? b2 : b3));
    ++n;
    return wd;
  }
  __device__ __forceinline__ float uniform() { return to_uniform(word()); }
  // After a reload between two words of a block: recompute the cached block
  // the next draws come from (a particle stored at a block boundary needs
  // nothing).
  __device__ __forceinline__ void resume() {
    if (n & 3u) {
      const Block b = philox(n >> 2, plo, phi, hist, k0, k1);
      b0 = b.w0; b1 = b.w1; b2 = b.w2; b3 = b.w3;
    }
  }
};

// ---------------------------------------------------------------- tables
struct TPos { int i; float t; };

// Position on the log-energy grid: node index i and fraction t in [0, 1].
__device__ __forceinline__ TPos tpos(const DevTables& T, float e) {
  float f = (__log2f(e) - T.lg2_emin) * T.inv_h2;
  f = fminf(fmaxf(f, 0.0f), (float)(kNE - 1));
  const int i = min((int)f, kNE - 2);
  return TPos{i, f - (float)i};
}

__device__ __forceinline__ float4 lerp4(const float4* tab, int base, TPos p) {
  const float4 a = tab[base + p.i];
  const float4 b = tab[base + p.i + 1];
  return make_float4(fmaf(p.t, b.x - a.x, a.x), fmaf(p.t, b.y - a.y, a.y), fmaf(p.t, b.z - a.z, a.z),
                     fmaf(p.t, b.w - a.w, a.w));
}

__device__ __forceinline__ float lerp_x(const float4* tab, int base, TPos p) {
  const float a = tab[base + p.i].x;
  const float b = tab[base + p.i + 1].x;
  return fmaf(p.t, b - a, a);
}

__device__ __forceinline__ float lerp_w(const float4* tab, int base, TPos p) {
  const float a = tab[base + p.i].w;
  const float b = tab[base + p.i + 1].w;
  return fmaf(p.t, b - a, a);
}

// ---------------------------------------------------------------- geometry
__device__ __forceinline__ bool inside(const DevPhantom& P, float x, float y, float z) {
  return x >= 0.0f && x < P.lx && y >= 0.0f && y < P.ly && z >= 0.0f && z < P.lz;
}

// Voxel of an inside point: floor(x / dx) per axis (a point on a face belongs
// to the voxel on its high side).
__device__ __forceinline__ int voxel(const DevPhantom& P, float x, float y, float z, int& ix, int& iy, int& iz) {
  ix = min((int)(x * P.idx), P.nx - 1);
  iy = min((int)(y * P.idy), P.ny - 1);
  iz = min((int)(z * P.idz), P.nz - 1);
  return (iz * P.ny + iy) * P.nx + ix;
}

// Voxel of an electron: each coordinate is advanced by the skin in the
// direction of travel before flooring, so a hinge endpoint left a hair short
// of the face it heads for counts as beyond it.  False when the advanced
// point is outside the phantom (the electron escapes).
__device__ __forceinline__ bool electron_voxel(const DevPhantom& P, float x, float y, float z, float u, float v,
                                               float w, int& ix, int& iy, int& iz, int& vox) {
  const float sk = P.skin;
  const float qx = x + (u > 0.0f ? sk : (u < 0.0f ? -sk : 0.0f));
  const float qy = y + (v > 0.0f ? sk : (v < 0.0f ? -sk : 0.0f));
  const float qz = z + (w > 0.0f ? sk : (w < 0.0f ? -sk : 0.0f));
  if (!(qx >= 0.0f && qx < P.lx && qy >= 0.0f && qy < P.ly && qz >= 0.0f && qz < P.lz)) return false;
  vox = voxel(P, qx, qy, qz, ix, iy, iz);
  return true;
}

// Distance along (u, v, w) to the boundary of voxel (ix, iy, iz): d_vox of Eq. 4.
__device__ __forceinline__ float dist_boundary(const DevPhantom& P, float x, float y, float z, float u, float v,
                                               float w, int ix, int iy, int iz) {
  float t = kInf;
  if (u > 0.0f) t = fminf(t, fdiv((float)(ix + 1) * P.dx - x, u));
  else if (u < 0.0f) t = fminf(t, fdiv((float)ix * P.dx - x, u));
  if (v > 0.0f) t = fminf(t, fdiv((float)(iy + 1) * P.dy - y, v));
  else if (v < 0.0f) t = fminf(t, fdiv((float)iy * P.dy - y, v));
  if (w > 0.0f) t = fminf(t, fdiv((float)(iz + 1) * P.dz - z, w));
  else if (w < 0.0f) t = fminf(t, fdiv((float)iz * P.dz - z, w));
  return fmaxf(t, 0.0f);
}

// New direction at polar cosine cost and azimuth phi about (u, v, w),
// renormalised.
// Turn (u, v, w) by the polar angle with cosine cost and sine sint about the
// old direction, azimuth phi.
__device__ __forceinline__ void rotate_cs(float& u, float& v, float& w, float cost, float sint, float phi) {
  float sp, cp;
  __sincosf(phi, &sp, &cp);
  const float rho2 = u * u + v * v;
  float nu, nv, nw;
  if (rho2 > 1e-20f) {
    const float r = sqrtf(rho2);
    const float ir = frcp(r);
    nu = u * cost + sint * (u * w * cp - v * sp) * ir;
    nv = v * cost + sint * (v * w * cp + u * sp) * ir;
    nw = w * cost - r * sint * cp;
  } else {
    nu = sint * cp;
    nv = sint * sp;
    nw = w >= 0.0f ? cost : -cost;
  }
  const float inv = rsqrtf(nu * nu + nv * nv + nw * nw);
  u = nu * inv; v = nv * inv; w = nw * inv;
}

__device__ __forceinline__ void rotate(float& u, float& v, float& w, float cost, float phi) {
  cost = fminf(fmaxf(cost, -1.0f), 1.0f);
  rotate_cs(u, v, w, cost, sqrtf((1.0f - cost) * (1.0f + cost)), phi);
}

// The same by om = 1 - cos(theta): for the small angles of a multiple-
// scattering step, cos(theta) rounded to FP32 keeps few digits of om, so the
// sine is formed from om itself, sin = sqrt(om (2 - om)).
__device__ __forceinline__ void rotate_om(float& u, float& v, float& w, float om, float phi) {
  om = fminf(fmaxf(om, 0.0f), 2.0f);
  rotate_cs(u, v, w, 1.0f - om, sqrtf(om * (2.0f - om)), phi);
}

__device__ __forceinline__ uint32_t to_lsb(float mev) {
  return (uint32_t)fminf(fmaxf(mev * kInvLsbF, 0.0f), kMaxLsbF);
}

// ---------------------------------------------------------------- samplers
// Compton (Sec. II.A): Klein-Nishina epsilon = E'/E by composition-rejection,
// 1/eps with weight ln(1/eps0) and eps with weight (1 - eps0^2)/2, accepted
// with 1 - eps sin^2/(1 + eps^2).  Three uniforms per trial.
__device__ __forceinline__ void sample_kn(float k, Stream& s, float& eps, float& cost) {
  const float eps0 = frcp(1.0f + 2.0f * k);
  const float a1 = fln(1.0f + 2.0f * k);
  const float a2 = 0.5f * (1.0f - eps0 * eps0);
  for (;;) {
    const float u1 = s.uniform(), u2 = s.uniform(), u3 = s.uniform();
    const float e = (u1 * (a1 + a2) < a1) ? fexp(-a1 * u2) : sqrtf(eps0 * eps0 + (1.0f - eps0 * eps0) * u2);
    const float t = fdiv(1.0f - e, k * e);
    const float sin2 = t * (2.0f - t);
    const float g = 1.0f - fdiv(e * sin2, 1.0f + e * e);
    if (u3 <= g) { eps = e; cost = 1.0f - t; return; }
  }
}

// Photoelectron polar cosine from the Sauter K-shell distribution (Sec. II.A):
// nu = 1 - cos from nu/(A+nu)^3 on [0, 2] by inversion, accepted with
// (2 - nu)(1/(A+nu) + B)/(2/A + 2 max(B, 0)).  Two uniforms per trial.
__device__ __forceinline__ float sample_sauter(float t, Stream& s) {
  const float g = 1.0f + t / kMc2;
  const float beta = fdiv(sqrtf(t * (t + 2.0f * kMc2)), t + kMc2);
  const float a = frcp(g * g * beta * (1.0f + beta));
  const float b = 0.5f * beta * g * (g - 1.0f) * (g - 2.0f);
  const float mx = fdiv(2.0f, a) + 2.0f * fmaxf(b, 0.0f);
  for (;;) {
    const float u1 = s.uniform(), u2 = s.uniform();
    const float q = fdiv(2.0f * sqrtf(u1), a + 2.0f);
    const float nu = fdiv(q * a, 1.0f - q);
    const float f = (2.0f - nu) * (frcp(a + nu) + b);
    if (u2 * mx <= f) return 1.0f - nu;
  }
}

// Pair electron polar cosine from (1 - beta cos)^-2 by inversion.
__device__ __forceinline__ float pair_cos(float t, float u) {
  const float g = 1.0f + t / kMc2;
  const float beta = fdiv(sqrtf(t * (t + 2.0f * kMc2)), t + kMc2);
  const float omb = frcp(g * g * (1.0f + beta));
  return fdiv(2.0f * u - 1.0f + beta, omb + 2.0f * beta * u);
}

// Moller energy fraction in [kcut/T, 1/2] (Sec. II.B.1): 1/eps^2 and flat
// components, accepted with h(eps)/(1 + 5 eps^2).  Three uniforms per trial.
__device__ __forceinline__ float sample_moller(float t, float kcut, Stream& s) {
  const float tau = t / kMc2, g = tau + 1.0f;
  const float e0 = fdiv(kcut, t);
  const float r2 = fdiv(tau, g) * fdiv(tau, g);
  const float c = fdiv(2.0f * tau + 1.0f, g * g);
  const float ie0 = frcp(e0);
  const float w1 = ie0 - 2.0f, w2 = 5.0f * (0.5f - e0);
  for (;;) {
    const float u1 = s.uniform(), u2 = s.uniform(), u3 = s.uniform();
    const float eps = (u1 * (w1 + w2) < w1) ? frcp(ie0 - u2 * (ie0 - 2.0f)) : e0 + u2 * (0.5f - e0);
    const float q = fdiv(eps, 1.0f - eps);
    const float h = 1.0f + q * q + r2 * eps * eps - c * q;
    if (u3 * (1.0f + 5.0f * eps * eps) <= h) return eps;
  }
}

// Bremsstrahlung photon energy in [kc, T] (Sec. II.B.1): log-uniform proposal
// accepted with (4/3 - 4y/3 + y^2)/(4/3), y = k/E.  Two uniforms per trial.
__device__ __forceinline__ float sample_brems(float t, float kc, Stream& s) {
  const float e = t + kMc2;
  const float lr = fln(fdiv(t, kc));
  for (;;) {
    const float u1 = s.uniform(), u2 = s.uniform();
    const float k = kc * fexp(u1 * lr);
    const float y = fdiv(k, e);
    if (u2 * (4.0f / 3.0f) <= 4.0f / 3.0f - (4.0f / 3.0f) * y + y * y) return k;
  }
}

// Screening parameter A of the step's screened-Rutherford angular shape for a
// first moment G1 (Sec. II.B.2), from the table of ln A at logit(G1).
__device__ __forceinline__ float screening_A(const DevTables& T, const float* ms, float g1) {
  const float y = fln(fdiv(g1, 1.0f - g1));
  const float f = (y - T.ms_y0) * T.ms_inv_dy;
  const int i = min(max((int)floorf(f), 0), kNms - 2);
  const float t = f - (float)i;     // outside [0, 1] extrapolates the end segment
  return fexp(fmaf(t, ms[i + 1] - ms[i], ms[i]));
}

// Polar cosine of one condensed step: w = 1 - cos = 2 A u / (1 + A - u).
// 1 - cos(theta) of a multiple-scattering step (Wentzel shape with screening
// A from G1): om = 2 A u / (1 + A - u); isotropic above the G1 limit.  The
// denominator is formed as (1 - u) + A: u is an odd multiple of 2^-24, so
// 1 - u is exact in FP32, whereas 1 + A rounds A away when A < 2^-24 (short
// steps, low density) and fattens the large-angle tail.
__device__ __forceinline__ float wentzel_om(const DevTables& T, const float* ms, float g1, float u) {
  if (!(g1 > 0.0f)) return 0.0f;
  if (g1 >= kG1Iso) return 2.0f * u;
  const float a = screening_A(T, ms, g1);
  return fdiv(2.0f * a * u, (1.0f - u) + a);
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long lanes_below() {
  const uint32_t lane = lane_id();
  return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// A wavefront's private output segment [base, base + cap) of a staging queue;
// `used` is wave-uniform.  Each lane appends 0, 1 or 2 entries; the slots
// follow lane order, so no atomic is needed.
struct WaveSeg {
  uint32_t base, cap, used;
  struct Slots { uint32_t s0, s1; };
  __device__ __forceinline__ Slots append(bool want0, bool want1) {
    const unsigned long long m0 = __ballot(want0);
    const unsigned long long m1 = __ballot(want1);
    const unsigned long long lt = lanes_below();
    const uint32_t n0 = (uint32_t)__popcll(m0);
    Slots r;
    r.s0 = used + (uint32_t)__popcll(m0 & lt);
    r.s1 = used + n0 + (uint32_t)__popcll(m1 & lt);
    used += n0 + (uint32_t)__popcll(m1);
    return r;
  }
};

__device__ __forceinline__ uint32_t& qf(const DevQueue& q, int f, uint32_t i) { return q.base[f * q.stride + i]; }

__device__ __forceinline__ void put(const DevQueue& q, uint32_t slot, float x, float y, float z, float u, float v,
                                    float w, uint32_t e, uint32_t hist, uint32_t plo, uint32_t phi, uint32_t n,
                                    uint32_t beam) {
  qf(q, Q_X, slot) = __float_as_uint(x); qf(q, Q_Y, slot) = __float_as_uint(y); qf(q, Q_Z, slot) = __float_as_uint(z);
  qf(q, Q_U, slot) = __float_as_uint(u); qf(q, Q_V, slot) = __float_as_uint(v); qf(q, Q_W, slot) = __float_as_uint(w);
  qf(q, Q_E, slot) = e; qf(q, Q_HIST, slot) = hist; qf(q, Q_PLO, slot) = plo; qf(q, Q_PHI, slot) = phi;
  qf(q, Q_N, slot) = n; qf(q, Q_BEAM, slot) = beam;
}

// Add to run counter `idx` in the slot of the calling wavefront.
__device__ __forceinline__ void ctr_add(unsigned long long* ctr, int idx, unsigned long long v) {
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  atomicAdd(&ctr[idx * kCtrSlots + (wave & (kCtrSlots - 1))], v);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, off);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off);
    v += ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

}  // namespace dev
}  // namespace gmc
