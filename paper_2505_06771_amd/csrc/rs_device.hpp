// rs_device.hpp -- device building blocks of the batched Robotarium step on
// gfx950: counter-based stream, lane-group reductions, per-launch constants.
//
// Layout used by every kernel: a wavefront (64 lanes) is split into aligned
// groups of G lanes (G = 2, 4, 8 or 16); group g of a wavefront owns one
// environment and lane i of the group owns robot i (lanes i >= N idle but
// still take part in the group's shuffles, so every shuffle reads lanes that
// run the same control path).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr float kPiF = 3.14159265358979323846f;
constexpr double kPiD = 3.14159265358979323846;

template <typename T> __device__ __forceinline__ T pi_v();
template <> __device__ __forceinline__ float pi_v<float>() { return kPiF; }
template <> __device__ __forceinline__ double pi_v<double>() { return kPiD; }

__device__ __forceinline__ void sincos_t(float a, float *s, float *c) { sincosf(a, s, c); }
__device__ __forceinline__ void sincos_t(double a, double *s, double *c) { sincos(a, s, c); }
__device__ __forceinline__ float sqrt_t(float a) { return sqrtf(a); }
__device__ __forceinline__ double sqrt_t(double a) { return sqrt(a); }
__device__ __forceinline__ float rsqrt_t(float a) { return rsqrtf(a); }
__device__ __forceinline__ double rsqrt_t(double a) { return rsqrt(a); }

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 multiplies
// with a Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

enum : uint32_t { kAction = 0, kPolicy = 1, kPose = 2, kGoal = 3, kHeading = 4 };

__device__ __forceinline__ uint4 stream_block(uint32_t k0, uint32_t k1, uint32_t w0, uint32_t w1,
                                              uint32_t purpose, uint32_t index, uint32_t w3) {
  return philox4x32_10(make_uint4(w0, w1, (purpose << 24) | (index & 0xFFFFFFu), w3), k0, k1);
}

__device__ __forceinline__ uint32_t word(uint4 v, int k) {
  return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// 24-bit uniform in [0, 1): exact in FP32.
__device__ __forceinline__ float unit24(uint32_t r) { return (float)(r >> 8) * 5.9604644775390625e-8f; }

// ---- lane-group primitives (groups are aligned blocks of G lanes) ----------
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <int G, typename T> __device__ __forceinline__ T group_max(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}
template <int G, typename T> __device__ __forceinline__ T group_min(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
// Arg-max with deterministic tie break on the smaller id; every lane of the
// group ends with the same (value, id).
template <int G, typename T> __device__ __forceinline__ void group_argmax(T &v, int &id) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    int j = __shfl_xor(id, o, 64);
    if (w > v || (w == v && j < id)) {
      v = w;
      id = j;
    }
  }
}
template <int G, typename T> __device__ __forceinline__ void group_argmin(T &v, int &id) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    int j = __shfl_xor(id, o, 64);
    if (w < v || (w == v && j < id)) {
      v = w;
      id = j;
    }
  }
}
// Bits of the group's lanes in a wave ballot, shifted down to bit 0.
template <int G> __device__ __forceinline__ uint32_t group_bits(uint64_t ballot, int lane) {
  const int base = lane & ~(G - 1);
  const uint64_t m = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  return (uint32_t)((ballot >> base) & m);
}
template <int G> __device__ __forceinline__ bool group_all(bool pred, int lane) {
  const uint64_t m = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  return group_bits<G>(__ballot(pred), lane) == (uint32_t)m;
}
template <int G> __device__ __forceinline__ bool group_any(bool pred, int lane) {
  return group_bits<G>(__ballot(pred), lane) != 0u;
}

// Per-launch constants of the simulation, in the state precision T.
template <typename T> struct SimConst {
  T x_min, x_max, y_min, y_max;
  T dt, l, inv_l, gamma, rs2, kb, half, vmax, aspeed, kp;
  T R, L, wheel_lim;  // R <= 0: no saturation
  T inv_R, R_over_L;  // 1/R and R/L
  T goal_r;
  T tol_add;          // active-set admission threshold (normalised violation)
  T eps_z;            // relative threshold for a dependent constraint
  T eps_r;            // threshold on the multiplier step direction
  int max_steps;
  int controller;
  int qp_cap;         // 0: 8N + 32
  uint32_t key0, key1;
  // reset lattice (integer units of `grid`)
  int64_t xlo, ylo, wx, wy, sep2, xhi, yhi;
  double grid;
};

}  // namespace rs
