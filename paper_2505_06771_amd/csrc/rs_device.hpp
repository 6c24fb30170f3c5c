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

#include <type_traits>

namespace rs {

constexpr float kPiF = 3.14159265358979323846f;
constexpr double kPiD = 3.14159265358979323846;

template <typename T> __device__ __forceinline__ T pi_v();
template <> __device__ __forceinline__ float pi_v<float>() { return kPiF; }
template <> __device__ __forceinline__ double pi_v<double>() { return kPiD; }

// FP32 uses the hardware sine/cosine: headings stay in [-pi, pi], where its
// error (~1e-6) is far inside the tolerances of positions and observations.
__device__ __forceinline__ void sincos_t(float a, float *s, float *c) { __sincosf(a, s, c); }
__device__ __forceinline__ void sincos_t(double a, double *s, double *c) { sincos(a, s, c); }
// FP32 square root and reciprocal square root as the hardware instructions
// (about 1 ulp; no rescaling for denormal inputs, which the simulation's
// squared distances and speeds never are)
__device__ __forceinline__ float sqrt_t(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double sqrt_t(double a) { return sqrt(a); }
__device__ __forceinline__ float rsqrt_t(float a) { return __builtin_amdgcn_rsqf(a); }
__device__ __forceinline__ double rsqrt_t(double a) { return rsqrt(a); }

__device__ __forceinline__ float atan2_t(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double atan2_t(double y, double x) { return atan2(y, x); }

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

enum : uint32_t { kAction = 0, kPolicy = 1, kPose = 2, kGoal = 3, kHeading = 4, kNoise = 6 };

__device__ __forceinline__ uint4 stream_block(uint32_t k0, uint32_t k1, uint32_t w0, uint32_t w1,
                                              uint32_t purpose, uint32_t index, uint32_t w3) {
  return philox4x32_10(make_uint4(w0, w1, (purpose << 24) | (index & 0xFFFFFFu), w3), k0, k1);
}

__device__ __forceinline__ uint32_t word(uint4 v, int k) {
  const uint32_t lo = (k & 1) ? v.y : v.x, hi = (k & 1) ? v.w : v.z;
  return (k & 2) ? hi : lo;
}

// 24-bit uniform in [0, 1): exact in FP32 (and in FP64).
__device__ __forceinline__ float unit24(uint32_t r) { return (float)(r >> 8) * 5.9604644775390625e-8f; }
template <typename T> __device__ __forceinline__ T unit24_t(uint32_t r) {
  return (T)(r >> 8) * T(5.9604644775390625e-8);
}

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

// ---- DPP lane exchange inside a group (VALU-speed, no LDS traffic) --------
// Controls: quad_perm [1,0,3,2] = 0xB1 (lane ^ 1), quad_perm [2,3,0,1] = 0x4E
// (lane ^ 2), quad_perm [1,2,3,0] = 0x39, [3,0,1,2] = 0x93, row_ror:n =
// 0x120 + n (lane l reads lane (l - n) mod 16 of its row), row_mirror = 0x140
// (l reads 15 - l), row_half_mirror = 0x141 (l reads 7 - l within its half).
// Every control used here reads a lane of the caller's own row (and group),
// so no source is out of bounds: with bound_ctrl the move carries no old
// value to initialise.
template <int CTRL> __device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ int dpp(int v) { return dpp_i32<CTRL>(v); }
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i32<CTRL>((int)(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value held by lane (i + K) mod G of the caller's group (1 <= K < G). Every
// lane of the group must be active.
template <int G, int K, typename T> __device__ __forceinline__ T grot(T v, int lane) {
  static_assert(K >= 1 && K < G, "rotation inside the group");
  if constexpr (G == 2) {
    return dpp<0xB1>(v);
  } else if constexpr (G == 4) {
    return dpp<(K == 1 ? 0x39 : (K == 2 ? 0x4E : 0x93))>(v);
  } else if constexpr (G == 16) {
    return dpp<0x120 + (16 - K)>(v);
  } else {  // G == 8: two rotations of the 16-lane row; each lane keeps the
             // one that lands inside its own 8-lane half
    const T a = dpp<0x120 + (16 - K)>(v);  // lane (l + K) mod 16 of the row
    const T b = dpp<0x120 + (8 - K)>(v);   // lane (l + 8 + K) mod 16 of the row
    return ((lane & 7) + K < 8) ? a : b;
  }
}

// Butterfly over the group with a commutative `op`: every lane of the group
// ends with the same, bitwise identical, result.
template <int G, typename T, typename Op> __device__ __forceinline__ T gred(T v, Op op) {
  v = op(v, dpp<0xB1>(v));
  if constexpr (G >= 4) v = op(v, dpp<0x4E>(v));
  if constexpr (G >= 8) v = op(v, dpp<0x141>(v));
  if constexpr (G >= 16) v = op(v, dpp<0x140>(v));
  return v;
}
template <int G, typename T> __device__ __forceinline__ T gsum(T v) {
  return gred<G>(v, [](T a, T b) { return a + b; });
}
template <int G, typename T> __device__ __forceinline__ T gmax(T v) {
  return gred<G>(v, [](T a, T b) { return a > b ? a : b; });
}
template <int G, typename T> __device__ __forceinline__ T gmin(T v) {
  return gred<G>(v, [](T a, T b) { return a < b ? a : b; });
}

// LDS writes of the wavefront's lanes visible to its other lanes (and kept
// ahead of the reads that follow): wavefront-scope fences around a wave
// barrier, no hardware wait.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Phase clock of a wavefront (diagnostic builds only). Built with
// -DRS_PHASE_TIMERS, the fused rollout reads the shader clock at the
// boundaries of its step phases and adds the cycles of each phase to the
// wavefront's counters in LDS (one 64-bit add by the first active lane, so
// the counters take no registers from the step loop and a mark inside a
// branch still counts); without the flag every call here compiles to nothing.
enum : int {
  kPhObs = 0,     // observation rows: assembly, LDS staging, HBM stores
  kPhMlp = 1,     // policy MLP on MFMA
  kPhSample = 2,  // softmax and inverse-CDF draw
  kPhPre = 3,     // projection points, nominal command, pre-clip, bounds
  kPhQp = 4,      // certificate QP
  kPhPost = 5,    // unicycle map, Euler step, reward, termination, reset
  kPhLoop = 6,    // steps in which some env of the wavefront ran the active-set loop
  kPhTotal = 7,   // cycles of the whole step loop
  kPhases = 8
};
struct PhaseClock {
#ifdef RS_PHASE_TIMERS
  uint64_t last;
  unsigned long long *acc;  // the wavefront's kPhases counters in LDS
  int lane;
  __device__ __forceinline__ void start(unsigned long long *lds_acc, int lane_id) {
    acc = lds_acc;
    lane = lane_id;
    if (lane < kPhases) acc[lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    last = __builtin_amdgcn_s_memtime();
  }
  __device__ __forceinline__ void add(int k, unsigned long long v) {
    if (lane == __builtin_amdgcn_readfirstlane(lane))
      __hip_atomic_fetch_add(acc + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
  __device__ __forceinline__ void mark(int k) {
    const uint64_t now = __builtin_amdgcn_s_memtime();
    add(k, now - last);
    last = now;
  }
  __device__ __forceinline__ void count(int k, bool any) {
    if (any) add(k, 1ull);
  }
  __device__ __forceinline__ uint64_t last_or_zero() const { return last; }
#else
  __device__ __forceinline__ uint64_t last_or_zero() const { return 0; }
  __device__ __forceinline__ void start(unsigned long long *, int) {}
  __device__ __forceinline__ void mark(int) {}
  __device__ __forceinline__ void count(int, bool) {}
#endif
};

// Compile-time loop: f(std::integral_constant<int, K>) for K in [B, E).
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Per-launch constants of the simulation, in the state precision T.
template <typename T> struct SimConst {
  T xwl, xwh, ywl, ywh;  // walls pulled in by r_s/2: x_min + r_s/2, x_max - r_s/2, ...
  T dt, l, inv_l, gamma, rs2, kb, vmax, vmax4, aspeed, kp;
  T wstep, kv, kw;  // waypoint distance and position-controller gains
  T krho, kalpha;   // pose-controller gains (its k_beta term vanishes on move waypoints)
  T noise;          // action-noise amplitude (0: off)
  T prey_step, tag_r, tag_reward;  // Predator-Prey: prey move per step, tag radius, reward
  T R, halfL, wheel_lim;  // R <= 0: no saturation; halfL = L/2
  T inv_R, R_over_L;  // 1/R and R/L
  T goal_r;
  T tol_add;          // active-set admission threshold (normalised violation)
  T eps_z;            // relative threshold for a dependent constraint
  T eps_r;            // threshold on the multiplier step direction
  int max_steps;
  int controller;
  int scenario;       // 0 Navigation, 1 Predator-Prey (kernels are specialised on it)
  int qp_cap;         // 0: 8N + 32
  uint32_t key0, key1;
  // reset lattice (integer units of `grid`)
  int64_t xlo, ylo, wx, wy, sep2, xhi, yhi;
  double grid;
};

// Reference to the launch's SimConst in the kernel-argument segment. A field
// read through it is loaded (by a scalar load) where it is used, so constants
// needed only on cold paths (reset sampler, stream key) do not hold scalar
// registers across a step loop.
template <typename T> struct ConstRef {
  uint64_t addr;
  __device__ __forceinline__ const __attribute__((address_space(4))) SimConst<T> *get() const {
    uint64_t a = addr;
    asm volatile("" : "+s"(a));  // opaque: the load stays at the use
    return (const __attribute__((address_space(4))) SimConst<T> *)a;
  }
};
// `offset` = offsetof(kernel argument struct, its SimConst member); the
// struct must be the kernel's first parameter.
// Only in a kernel's own body: in a device function that the compiler keeps
// out of line, the kernel-argument segment pointer reads as null. Callees
// take the ConstRef their kernel formed.
template <typename T> __device__ __forceinline__ ConstRef<T> kernarg_const(size_t offset) {
  return ConstRef<T>{(uint64_t)__builtin_amdgcn_kernarg_segment_ptr() + offset};
}

}  // namespace rs
