// labf_device.h -- device helpers shared by the kernel sources (wave
// primitives, the Philox normals, the alchemical schedule, periodic images).
#pragma once
#include "labf_impl.h"

#include <math.h>

namespace labf {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// box shift of each axis encoded in a list entry's image code
__device__ __forceinline__ int img_x(int code) { return (code & 3) - 1; }
__device__ __forceinline__ int img_y(int code) { return ((code >> 2) & 3) - 1; }
__device__ __forceinline__ int img_z(int code) { return ((code >> 4) & 3) - 1; }
// number of lanes below this one whose bit is set in a ballot
__device__ __forceinline__ int lanes_below(unsigned long long bal) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
  return v;
}

// load at a 32-bit byte offset from a base pointer
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, uint32_t bo) {
  return *(const T *)((const char *)base + bo);
}
// store at a 32-bit byte offset from a base pointer
template <typename T>
__device__ __forceinline__ void st_off(T *base, uint32_t bo, T v) {
  *(T *)((char *)base + bo) = v;
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// hardware reciprocal in FP32 (about 1 ulp), a true division in FP64
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, multipliers 0xD2511F53 and
// 0xCD9E8D57, key bumped by 0x9E3779B9 / 0xBB67AE85 between rounds.
__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// Four standard normals for counter (atom, step, walker, purpose): Box-Muller
// in FP64 with u1 = (a + 1) 2^-32 in (0, 1], u2 = b 2^-32.
__device__ inline void gauss4(uint64_t seed, uint32_t atom, uint32_t step, uint32_t walker,
                       uint32_t purpose, double z[4]) {
  uint32_t c0 = atom, c1 = step, c2 = walker, c3 = purpose;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double two_pi = 6.283185307179586;
  const double inv = 2.3283064365386963e-10;  // 2^-32
  const uint32_t o[4] = {c0, c1, c2, c3};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double u1 = ((double)o[2 * k] + 1.0) * inv;
    const double u2 = (double)o[2 * k + 1] * inv;
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(two_pi * u2, &sn, &cs);
    z[2 * k] = rad * cs;
    z[2 * k + 1] = rad * sn;
  }
}

// One Box-Muller pair of gauss4, bit for bit: p = 0 gives z[0], z[1], p = 1
// gives z[2], z[3] (cosine, then sine), so that lanes can share an atom's
// draws.
__device__ inline void gauss_pair(uint64_t seed, uint32_t atom, uint32_t step, uint32_t walker,
                                  uint32_t purpose, int p, double &zc, double &zs) {
  uint32_t c0 = atom, c1 = step, c2 = walker, c3 = purpose;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double two_pi = 6.283185307179586;
  const double inv = 2.3283064365386963e-10;  // 2^-32
  const double u1 = ((double)(p ? c2 : c0) + 1.0) * inv;
  const double u2 = (double)(p ? c3 : c1) * inv;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(two_pi * u2, &sn, &cs);
  zc = rad * cs;
  zs = rad * sn;
}

// The normal z[k] (k < 4) of gauss4, bit for bit.
__device__ inline double gauss_comp(uint64_t seed, uint32_t atom, uint32_t step, uint32_t walker,
                                    uint32_t purpose, int k) {
  double zc, zs;
  gauss_pair(seed, atom, step, walker, purpose, k >> 1, zc, zs);
  return (k & 1) ? zs : zc;
}


// Channel coupling c_x(lambda) and dc_x/dlambda of the alchemical schedule:
// ramp clip((lambda - s)/(e - s), 0, 1); decoupling c = 1 - ramp, coupling
// c = ramp; slope on [s, e) and at lambda = e = hi.
__device__ __forceinline__ void channel(double lam, double s0, double s1, int coupling, double hi,
                                        double &c, double &dc) {
  const double w = s1 - s0;
  double m = lam <= s0 ? 0.0 : (lam >= s1 ? 1.0 : (lam - s0) / w);
  double dm = ((lam >= s0 && lam < s1) || (lam == s1 && s1 == hi)) ? 1.0 / w : 0.0;
  c = coupling ? m : 1.0 - m;
  dc = coupling ? dm : -dm;
}

template <typename T>
__device__ __forceinline__ T wrap_pos(T x, T B, T L) {
  if (x >= B + L) x -= L;
  else if (x < B) x += L;
  return x;
}

__device__ __forceinline__ double min_image(double d, double L) {
  if (d > 0.5 * L) d -= L;
  else if (d < -0.5 * L) d += L;
  return d;
}

// XCD-aware block order: consecutive logical blocks (neighbouring clusters,
// sharing j-data) land on the same XCD and its L2.  Grid = 8 * ceil(nb / 8).
__device__ __forceinline__ int xcd_block(int nb) {
  const int per = (nb + 7) >> 3;
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}


// Adds one per lane to ctr[K] (lanes with K < 0 add nothing) with one atomic
// per distinct K in the wave; returns the lane's offset among the additions
// to its counter (old value + rank among the wave's lanes with the same K).
// Slot order keeps a wave within one or two columns.
__device__ __forceinline__ int wave_agg_add(int32_t *ctr, int64_t K) {
  const int lane = lane_id();
  unsigned long long todo = __ballot(K >= 0);
  int result = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int64_t KL = __shfl(K, leader, WAVE);
    const unsigned long long same = __ballot(K == KL) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(&ctr[KL], __popcll(same));
    base = __shfl(base, leader, WAVE);
    if (K == KL) result = base + __popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  return result;
}

}  // namespace labf
