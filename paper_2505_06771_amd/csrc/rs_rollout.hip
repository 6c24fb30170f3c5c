// rs_rollout.hip -- fused, persistent policy rollout (FP32 state, bf16 MLP on
// MFMA) and its C-ABI entry point.
//
// One launch runs all H steps: the state of every robot stays in registers,
// each wavefront owns 64/G environments (lane i of a G-lane group = robot i).
// Per step and wavefront:
//   1. observation rows (2N+4 floats) are built in registers and staged in LDS
//      packed env after env for the MLP; with a compile-time robot count each
//      lane stores its own row to HBM with 16-byte stores, otherwise the
//      staging area is copied out as one contiguous range per wavefront;
//   2. the policy runs transposed on v_mfma_f32_16x16x32_bf16: for each tile
//      of 16 robots, H1^T = W1^T X^T (K = 32 features), H2^T = W2^T H1^T,
//      logits^T = W3^T H2^T (K = 64 in two steps). The K order of layers 2-3
//      is permuted so that the accumulator registers of one layer are the
//      B operand of the next, with no LDS round trip; weights are permuted the
//      same way when they are loaded into registers at kernel start, and the
//      biases seed the accumulators;
//   3. logits go through LDS back to the robot's lane, which draws its action
//      by inverse CDF from its own counter-based uniform;
//   4. the env step (certificate QP, dynamics, reward, reset) runs as in
//      env_step.
#include "rs_internal.hpp"
#include "rs_step.hpp"

#include <cstddef>
#include <cstring>

namespace rs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx2 __attribute__((ext_vector_type(2)));

constexpr int kRollBlock = 256;
constexpr int kRollWaves = kRollBlock / 64;

#ifdef RS_PHASE_TIMERS
// Per-wavefront phase cycles of the last rollout launch (diagnostic builds):
// [wavefront][kPhases], wavefront = block * 4 + wave; launches with more
// wavefronts record the first kTimedWaves.
constexpr int kTimedWaves = 1 << 16;
__device__ unsigned long long rs_phase_cycles_dev[kTimedWaves][kPhases];
#endif

struct RolloutArgs {
  SimConst<float> C;
  int E, N, D, H;
  uint32_t env_base, t0;
  float *x, *y, *th, *gx, *gy;
  int32_t *step, *episode;
  const __bf16 *w1, *w2, *w3;
  const float *b1, *b2, *b3;
  float *obs;
  uint8_t *actions;
  float *reward;
  uint8_t *done;
  int32_t *qp_stats;            // [E][kQPStats] accumulated (STATS kernels only)
  unsigned long long *qp_fail;  // the context's failure counters
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ReLU of a bf16 pair with a packed 16-bit integer max: a bf16 with the sign
// bit set is a negative int16, so max(., 0) zeroes exactly the negative values
// (and -0). Rounding commutes with ReLU, so this equals rounding the FP32 ReLU.
__device__ __forceinline__ bf16x2 relu_bf16x2(bf16x2 p) {
  const shortx2 z = {0, 0};
  return __builtin_bit_cast(bf16x2, __builtin_elementwise_max(__builtin_bit_cast(shortx2, p), z));
}

// Eight FP32 values rounded to bf16 (round to nearest even), one
// v_cvt_pk_bf16_f32 per pair, optionally followed by the pairwise ReLU.
template <bool RELU>
__device__ __forceinline__ bf16x8 pack_bf16x8(floatx4 a, floatx4 b) {
  bf16x2 p0 = __builtin_convertvector((floatx2){a[0], a[1]}, bf16x2);
  bf16x2 p1 = __builtin_convertvector((floatx2){a[2], a[3]}, bf16x2);
  bf16x2 p2 = __builtin_convertvector((floatx2){b[0], b[1]}, bf16x2);
  bf16x2 p3 = __builtin_convertvector((floatx2){b[2], b[3]}, bf16x2);
  if constexpr (RELU) {
    p0 = relu_bf16x2(p0);
    p1 = relu_bf16x2(p1);
    p2 = relu_bf16x2(p2);
    p3 = relu_bf16x2(p3);
  }
  return __builtin_shufflevector(__builtin_shufflevector(p0, p1, 0, 1, 2, 3),
                                 __builtin_shufflevector(p2, p3, 0, 1, 2, 3), 0, 1, 2, 3, 4, 5,
                                 6, 7);
}

// Hidden index held in slot j of lane group g at k-step s of layers 2 and 3:
// the accumulator of output tile (2s + j/4), register j%4, of lane group g.
__device__ __forceinline__ int perm_hidden(int s, int g, int j) {
  return 16 * (2 * s + (j >> 2)) + 4 * g + (j & 3);
}

// NC > 0 fixes the robot count at compile time (NC <= G); NC = 0 reads it
// from the arguments. STATS: the kernel also counts the certificate's stages
// per env (qp_stats); the kernels without it carry none of that code.
// Teams of three (NC = 3) run three wavefronts per SIMD: at the paper's team
// size a launch has a third more wavefronts than 8-robot envs of the same
// robot count (one lane in four of a 4-lane group is idle), and two per SIMD
// would leave a second, partial round. That needs at most 168 VGPRs and 53 KiB
// of LDS per block: the policy weights stay in LDS and are read at each step's
// MLP, the staging and logit areas are sized to what three robots use.
// 16-lane groups (9 to 16 robots) hold more state per lane than 256 VGPRs
// take, so they run one wavefront per SIMD with the accumulation registers
// as well.
template <int G, int NC> constexpr int rollout_waves_per_simd() {
  return NC == 3 ? 3 : (G == 16 ? 1 : 2);
}

template <int G, int NC, bool PP, bool STATS>
__global__ __launch_bounds__(kRollBlock, (rollout_waves_per_simd<G, NC>())) void k_rollout(RolloutArgs A) {
  constexpr int EPW = 64 / G;
  constexpr bool kTeam3 = NC == 3;
  // staging floats per wavefront: 3-robot rows are 10 floats, and the MLP
  // reads up to 22 floats past the last one (zero weights)
  constexpr int kObsFloats = kTeam3 ? 704 : 64 * 32;
  constexpr int kLogitRows = kTeam3 ? 2 : 4;
  // teams of three: the MFMA A-operand fragments of the three layers (14 x 64
  // bf16x8) after the wavefronts' staging areas
  constexpr int kWFloats = kTeam3 ? 14 * 64 * 4 : 0;
  __shared__ QPScratch<float, G> qs[kRollBlock / G];
  __shared__ __attribute__((aligned(16))) float obs_lds[kRollWaves * kObsFloats + kWFloats];
  // logits 4g..4g+3 of robot n at [g][n], g = 0..3 (g >= 2: the padding
  // rows of the last layer, never read; written so that the four tiles of
  // the MLP are one branch-free block the scheduler can interleave; teams of
  // three keep only the rows that are read)
  __shared__ float4 logit_lds[kRollWaves][kLogitRows * 64];
  // hidden-layer biases in the accumulator layout: [layer][tile][lane group]
  __shared__ float4 bias_lds[2][4][4];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x < 32) {
    const int layer = threadIdx.x >> 4, mt = (threadIdx.x >> 2) & 3, gg = threadIdx.x & 3;
    const float *bsrc = layer ? A.b2 : A.b1;
    bias_lds[layer][mt][gg] = make_float4(bsrc[16 * mt + 4 * gg], bsrc[16 * mt + 4 * gg + 1],
                                          bsrc[16 * mt + 4 * gg + 2], bsrc[16 * mt + 4 * gg + 3]);
  }
  bf16x8 *wfrag = reinterpret_cast<bf16x8 *>(obs_lds + kRollWaves * kObsFloats);  // [14][64]
  if constexpr (kTeam3) {
    if (wave == 0) {  // the fragments are the same for every wavefront
      const int g = lane >> 4, c16 = lane & 15;
      const __bf16 zero = (__bf16)0.0f;
      constexpr int Dt = 2 * NC + 4;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        bf16x8 w1;
#pragma unroll
        for (int j = 0; j < 8; ++j) w1[j] = 8 * g + j < Dt ? A.w1[(8 * g + j) * 64 + 16 * mt + c16] : zero;
        wfrag[mt * 64 + lane] = w1;
#pragma unroll
        for (int sk = 0; sk < 2; ++sk) {
          bf16x8 w2;
#pragma unroll
          for (int j = 0; j < 8; ++j) w2[j] = A.w2[perm_hidden(sk, g, j) * 64 + 16 * mt + c16];
          wfrag[(4 + 2 * mt + sk) * 64 + lane] = w2;
        }
      }
#pragma unroll
      for (int sk = 0; sk < 2; ++sk) {
        bf16x8 w3;
#pragma unroll
        for (int j = 0; j < 8; ++j) w3[j] = c16 < 5 ? A.w3[perm_hidden(sk, g, j) * 5 + c16] : zero;
        wfrag[(12 + sk) * 64 + lane] = w3;
      }
    }
  }
  __syncthreads();  // the only block-wide barrier, before any wavefront leaves
  const int i = lane & (G - 1);
  const int grp = lane / G;
  const int e0 = (blockIdx.x * kRollWaves + wave) * EPW;
  if (e0 >= A.E) return;  // the whole wavefront leaves together
  const int e = e0 + grp;
  const int N = NC ? NC : A.N;
  const ConstRef<float> K = kernarg_const<float>(offsetof(RolloutArgs, C));
  const int D = 2 * N + 4;
  const bool env_ok = e < A.E;
  const bool on = env_ok && i < N;
  const int nenv = min(EPW, A.E - e0);
  // robot index (E * N < 2^31, checked by the entry point)
  const uint32_t r = on ? (uint32_t)(e * N + i) : 0u;

  float x = 0.f, y = 0.f, th = 0.f, gx = 0.f, gy = 0.f;
  int step = 0, episode = 0;
  if (on) { x = A.x[r]; y = A.y[r]; th = A.th[r]; gx = A.gx[r]; gy = A.gy[r]; }
  if (env_ok) { step = A.step[e]; episode = A.episode[e]; }
  float s, c;
  sincos_t(th, &s, &c);

  // ---- policy weights into registers (MFMA A-operand fragments) ----------
  const int g = lane >> 4, c16 = lane & 15;
  bf16x8 rw1f[4], rw2f[4][2], rw3f[2];  // (not for teams of three)
  floatx4 b3f;
  const __bf16 zero = (__bf16)0.0f;
#pragma unroll
  for (int mt = 0; mt < 4 && !kTeam3; ++mt) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int f = 8 * g + j;
      rw1f[mt][j] = f < D ? A.w1[f * 64 + 16 * mt + c16] : zero;
    }
#pragma unroll
    for (int sk = 0; sk < 2; ++sk)
#pragma unroll
      for (int j = 0; j < 8; ++j) rw2f[mt][sk][j] = A.w2[perm_hidden(sk, g, j) * 64 + 16 * mt + c16];
  }
#pragma unroll
  for (int sk = 0; sk < 2 && !kTeam3; ++sk)
#pragma unroll
    for (int j = 0; j < 8; ++j) rw3f[sk][j] = c16 < 5 ? A.w3[perm_hidden(sk, g, j) * 5 + c16] : zero;
#pragma unroll
  for (int j = 0; j < 4; ++j) b3f[j] = (4 * g + j) < 5 ? A.b3[4 * g + j] : 0.0f;

  // Complete the state and weight loads before the step loop. Without this
  // the first in-loop use waits on the vector-memory counter, which on this
  // architecture also counts the loop's own global stores: every step would
  // stall until its observation stores had landed.
  __builtin_amdgcn_s_waitcnt(0);

  float *obs_w = obs_lds + wave * kObsFloats;
  // the compile-time-count path stages bf16 rows of DB values (same buffer)
  __bf16 *obs_b = reinterpret_cast<__bf16 *>(obs_w);
  constexpr int DB = ((2 * NC + 4 + 7) / 8) * 8;
  static_assert(NC == 0 || 64 * DB + 8 <= 64 * 32 * 2, "bf16 staging fits");
  // Zero the wavefront's staging area once: the MLP reads eight features per
  // lane from packed rows without bounds tests, so what it reads past the
  // last row (multiplied by zero weights, or feeding columns of robots that
  // do not exist) must be finite.
  if constexpr (kTeam3) {
    for (int q = lane; q < kObsFloats / 4; q += 64)
      reinterpret_cast<float4 *>(obs_w)[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      reinterpret_cast<float4 *>(obs_w)[q * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  wave_lds_sync();
  float4 *logit_w = logit_lds[wave];
  QPScratch<float, G> *sh = &qs[threadIdx.x / G];
  const int base = lane & ~(G - 1);
  const int nfl = nenv * N * D;             // floats of this wavefront's rows
  const bool vec4 = ((N * D) & 3) == 0;
  const int row = grp * N + i;              // packed LDS row of my robot

  uint4 qblk = make_uint4(0u, 0u, 0u, 0u);  // this lane's Philox block (G >= 4)
  PhaseClock pc;
#ifdef RS_PHASE_TIMERS
  __shared__ unsigned long long phase_lds[kRollWaves][kPhases];
  pc.start(phase_lds[wave], lane);
#else
  pc.start(nullptr, lane);
#endif
  const uint64_t t_begin = pc.last_or_zero();
  for (int t = 0; t < A.H; ++t) {
    // teams of three: the lane's robot index, opaque to the compiler, so the
    // lane masks derived from it are formed anew each step rather than held
    // across the loop (which at 168 VGPRs would spill)
    int il = i;
    if constexpr (kTeam3) asm volatile("" : "+v"(il));
    // ---- 1. observation -> LDS (packed) -> HBM --------------------------
    if constexpr (NC > 0 && ((2 * NC + 4) & 3) == 0) {
      // Row assembled in registers: every lane of the group posts its (x, y)
      // to the group's LDS scratch (free between two certificate solves) and
      // reads back all NC positions with broadcast reads; slot s of the
      // neighbour block then holds robot j = s + (s >= i). The row goes to
      // the MLP's LDS staging and to HBM as 16-byte stores.
      constexpr int DC = 2 * NC + 4;
      static_assert(NC % 2 == 0 && sizeof(QPScratch<float, G>) >= NC * sizeof(float2), "");
      float rw[DC];
      rw[0] = x; rw[1] = y; rw[2] = c; rw[3] = s;
      reinterpret_cast<float2 *>(sh)[i] = make_float2(x, y);
      wave_lds_sync();
      float px_[NC], py_[NC];
#pragma unroll
      for (int q = 0; q < NC / 2; ++q) {
        const float4 v = reinterpret_cast<const float4 *>(sh)[q];
        px_[2 * q] = v.x; py_[2 * q] = v.y; px_[2 * q + 1] = v.z; py_[2 * q + 1] = v.w;
      }
#pragma unroll
      for (int S = 0; S < NC - 1; ++S) {
        rw[4 + 2 * S] = (S < il ? px_[S] : px_[S + 1]) - x;
        rw[5 + 2 * S] = (S < il ? py_[S] : py_[S + 1]) - y;
      }
      rw[DC - 2] = gx - x;
      rw[DC - 1] = gy - y;
      if (on) {
        // MLP staging in bf16 (the MLP's input precision, rounded as it would
        // round them), rows of DB values padded with zeros
        bf16x8 *o8 = reinterpret_cast<bf16x8 *>(obs_b + row * DB);
#pragma unroll
        for (int q = 0; q < DB / 8; ++q) {
          floatx4 lo4, hi4;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            lo4[j] = 8 * q + j < DC ? rw[(8 * q + j) % DC] : 0.f;
            hi4[j] = 8 * q + 4 + j < DC ? rw[(8 * q + 4 + j) % DC] : 0.f;
          }
          o8[q] = pack_bf16x8<false>(lo4, hi4);
        }
        if (A.obs) {
          float4 *g4 = reinterpret_cast<float4 *>(A.obs + ((size_t)t * A.E + e0) * (size_t)(NC * DC)) +
                       row * (DC / 4);
#pragma unroll
          for (int q = 0; q < DC / 4; ++q) {
            g4[q] = make_float4(rw[4 * q], rw[4 * q + 1], rw[4 * q + 2], rw[4 * q + 3]);
          }
        }
      }
      wave_lds_sync();
    } else {
      float *o = obs_w + row * D;
      if (on) { o[0] = x; o[1] = y; o[2] = c; o[3] = s; }
      static_for<1, G>([&](auto kc) {  // neighbour (i + K) mod G by rotation
        constexpr int K = decltype(kc)::value;
        const float xj = grot<G, K>(x, lane), yj = grot<G, K>(y, lane);
        const int j = (i + K) & (G - 1);
        if (on && j < N) {
          const int m = 4 + 2 * (j < i ? j : j - 1);
          o[m] = xj - x;
          o[m + 1] = yj - y;
        }
      });
      if (on) { o[D - 2] = gx - x; o[D - 1] = gy - y; }
      wave_lds_sync();
      if (A.obs) {
        float *dst = A.obs + ((size_t)t * A.E + e0) * (size_t)(N * D);  // wavefront-uniform
        if (vec4) {
          for (int q = lane; q < (nfl >> 2); q += 64)
            reinterpret_cast<float4 *>(dst)[q] = reinterpret_cast<const float4 *>(obs_w)[q];
        } else {
          for (int q = lane; q < (nfl >> 1); q += 64)
            reinterpret_cast<float2 *>(dst)[q] = reinterpret_cast<const float2 *>(obs_w)[q];
        }
      }
    }

    pc.mark(kPhObs);
    // ---- 2. policy MLP on MFMA, one tile of 16 robots at a time ----------
    // hidden biases (accumulator seeds): read once per step, shared by the
    // four tiles
    bf16x8 w1f[4], w2f[4][2], w3f[2];
    if constexpr (kTeam3) {
      // read at each step: the empty asm keeps the loads in the loop
      uint32_t wofs = 0;
      asm volatile("" : "+v"(wofs));
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        w1f[mt] = wfrag[mt * 64 + lane + wofs];
        w2f[mt][0] = wfrag[(4 + 2 * mt) * 64 + lane + wofs];
        w2f[mt][1] = wfrag[(5 + 2 * mt) * 64 + lane + wofs];
      }
      w3f[0] = wfrag[12 * 64 + lane + wofs];
      w3f[1] = wfrag[13 * 64 + lane + wofs];
    } else {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        w1f[mt] = rw1f[mt];
        w2f[mt][0] = rw2f[mt][0];
        w2f[mt][1] = rw2f[mt][1];
      }
      w3f[0] = rw3f[0];
      w3f[1] = rw3f[1];
    }
    floatx4 b1v[4], b2v[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const float4 p1 = bias_lds[0][mt][g], p2 = bias_lds[1][mt][g];
      b1v[mt] = (floatx4){p1.x, p1.y, p1.z, p1.w};
      b2v[mt] = (floatx4){p2.x, p2.y, p2.z, p2.w};
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int n = 16 * nt + c16;  // wave lane of the robot in this column
      const int ng = n / G, ni = n & (G - 1);
      // features 8g .. 8g+7 of robot n; past D they run into the next row
      // (finite, times zero weights); lanes of missing robots read finite
      // rows whose logits are never used
      const float *src = obs_w + (ng * N + ni) * D + 8 * g;
      bf16x8 xb;
      if constexpr (NC > 0 && ((2 * NC + 4) & 3) == 0) {
        xb = *reinterpret_cast<const bf16x8 *>(obs_b + (ng * NC + ni) * DB + 8 * g);
      } else if ((D & 3) == 0) {
        const float4 f0 = reinterpret_cast<const float4 *>(src)[0];
        const float4 f1 = reinterpret_cast<const float4 *>(src)[1];
        xb = pack_bf16x8<false>((floatx4){f0.x, f0.y, f0.z, f0.w},
                                 (floatx4){f1.x, f1.y, f1.z, f1.w});
      } else {
        floatx4 fa, fb;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const float2 f = reinterpret_cast<const float2 *>(src)[j];
          const float2 g = reinterpret_cast<const float2 *>(src)[j + 2];
          fa[2 * j] = f.x;
          fa[2 * j + 1] = f.y;
          fb[2 * j] = g.x;
          fb[2 * j + 1] = g.y;
        }
        xb = pack_bf16x8<false>(fa, fb);
      }
      floatx4 h1[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        h1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f[mt], xb, b1v[mt], 0, 0, 0);
      bf16x8 hb[2];
#pragma unroll
      for (int sk = 0; sk < 2; ++sk) hb[sk] = pack_bf16x8<true>(h1[2 * sk], h1[2 * sk + 1]);
      floatx4 h2[4];
#pragma unroll
      for (int mo = 0; mo < 4; ++mo) {
        h2[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2f[mo][0], hb[0], b2v[mo], 0, 0, 0);
        h2[mo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2f[mo][1], hb[1], h2[mo], 0, 0, 0);
      }
      bf16x8 hc[2];
#pragma unroll
      for (int sk = 0; sk < 2; ++sk) hc[sk] = pack_bf16x8<true>(h2[2 * sk], h2[2 * sk + 1]);
      floatx4 lg = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3f[0], hc[0], b3f, 0, 0, 0);
      lg = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3f[1], hc[1], lg, 0, 0, 0);
      // lane (g, c16) holds logits 4g..4g+3 of robot n
      if (!kTeam3 || g < 2) logit_w[g * 64 + n] = make_float4(lg[0], lg[1], lg[2], lg[3]);
    }
    wave_lds_sync();

    pc.mark(kPhMlp);
    // ---- 3. categorical draw in the robot's own lane ----------------------
    const float4 la = logit_w[lane], lb = logit_w[64 + lane];
    const float l5[5] = {la.x, la.y, la.z, la.w, lb.x};
    float mx = l5[0];
#pragma unroll
    for (int k = 1; k < 5; ++k) mx = fmaxf(mx, l5[k]);
    float ex[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) ex[k] = __expf(l5[k] - mx);
    const float tot = (((ex[0] + ex[1]) + ex[2]) + ex[3]) + ex[4];
    const uint32_t env_id = A.env_base + (uint32_t)e;
    // Sampling word of robot i at stream time t0 + t: word i&3 of block
    // (env_id, t0 + t, 1<<24 | i>>2, 0). With G >= 4 a lane quad holds the 4
    // robots of one block, so every 4 steps quad lane j computes the block of
    // step t + j and the others read it by DPP.
    uint32_t rbits;
    if constexpr (G >= 4) {
      const int ph = t & 3;
      if (ph == 0) {
        const auto *P = K.get();
        qblk = stream_block(P->key0, P->key1, env_id, A.t0 + (uint32_t)(t + (il & 3)), kPolicy,
                            (uint32_t)(il >> 2), 0u);
      }
      uint4 src;
      switch (ph) {
        case 0: src = make_uint4(dpp<0x00>((int)qblk.x), dpp<0x00>((int)qblk.y), dpp<0x00>((int)qblk.z), dpp<0x00>((int)qblk.w)); break;
        case 1: src = make_uint4(dpp<0x55>((int)qblk.x), dpp<0x55>((int)qblk.y), dpp<0x55>((int)qblk.z), dpp<0x55>((int)qblk.w)); break;
        case 2: src = make_uint4(dpp<0xAA>((int)qblk.x), dpp<0xAA>((int)qblk.y), dpp<0xAA>((int)qblk.z), dpp<0xAA>((int)qblk.w)); break;
        default: src = make_uint4(dpp<0xFF>((int)qblk.x), dpp<0xFF>((int)qblk.y), dpp<0xFF>((int)qblk.z), dpp<0xFF>((int)qblk.w)); break;
      }
      rbits = word(src, il & 3);
    } else {
      const auto *P = K.get();
      rbits = word(stream_block(P->key0, P->key1, env_id, A.t0 + (uint32_t)t, kPolicy,
                                (uint32_t)(i >> 2), 0u), i & 3);
    }
    const float u = unit24(rbits);
    // first k with u < C_k (C the cumulative distribution), else 4: the
    // cumulative sums do not decrease, so that is the number of k < 4 with
    // C_k <= u
    const float inv_tot = __builtin_amdgcn_rcpf(tot);
    float cdf = ex[0] * inv_tot;
    int action = u < cdf ? 0 : 1;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      cdf += ex[k] * inv_tot;
      action += u < cdf ? 0 : 1;
    }
    // per-step base pointers are uniform; the lane offsets are 32-bit
    uint8_t *act_t = A.actions + (size_t)t * (size_t)A.E * (size_t)N;
    if (on) act_t[r] = (uint8_t)action;

    pc.mark(kPhSample);
    // ---- 4. env step --------------------------------------------------------
    if (env_ok) {
      const StepOut<float> so = env_step_group<float, G, PP>(K, A.C.qp_cap, sh, lane, il, N, on, env_id,
                                                         A.t0 + (uint32_t)t, action, x, y, th, c, s, gx, gy, step,
                                                         episode, false,
#ifdef RS_PHASE_TIMERS
                                                         &pc
#else
                                                         nullptr
#endif
                                                         );
      if (il == 0) {
        (A.reward + (size_t)t * A.E)[(uint32_t)e] = so.reward;
        (A.done + (size_t)t * A.E)[(uint32_t)e] = so.done ? 1 : 0;
        if constexpr (STATS) qp_stats_add(A.qp_stats + (size_t)e * kQPStats, so.qp);
        qp_fail_count(A.qp_fail, so.qp);
      }
    }
  }
  if (on) { A.x[r] = x; A.y[r] = y; A.th[r] = th; A.gx[r] = gx; A.gy[r] = gy; }
  if (env_ok && i == 0) { A.step[e] = step; A.episode[e] = episode; }
#ifdef RS_PHASE_TIMERS
  pc.add(kPhTotal, pc.last - t_begin);
  wave_lds_sync();
  const int wid = blockIdx.x * kRollWaves + wave;
  if (lane < kPhases && wid < kTimedWaves) rs_phase_cycles_dev[wid][lane] = phase_lds[wave][lane];
#else
  (void)t_begin;
#endif
}

// Kernel for N robots: a compile-time robot count for N = 8 (8 lanes, no
// idle lane) and N = 3 (the team size of the paper's scenarios), the
// lane-group width with a run-time count otherwise.
template <bool PP, bool ST> static const void *rollout_kernel_for(int N) {
  if (N == 8) return reinterpret_cast<const void *>(&k_rollout<8, 8, PP, ST>);
  if (N == 3) return reinterpret_cast<const void *>(&k_rollout<4, 3, PP, ST>);  // the paper's teams
  switch (pow2_group(N)) {
    case 2: return reinterpret_cast<const void *>(&k_rollout<2, 0, PP, ST>);
    case 4: return reinterpret_cast<const void *>(&k_rollout<4, 0, PP, ST>);
    case 8: return reinterpret_cast<const void *>(&k_rollout<8, 0, PP, ST>);
    default: return reinterpret_cast<const void *>(&k_rollout<16, 0, PP, ST>);
  }
}
static const void *rollout_kernel(const RolloutArgs &A) {
  const bool pp = A.C.scenario == RS_SCN_PREDATOR_PREY, st = A.qp_stats != nullptr;
  if (pp) return st ? rollout_kernel_for<true, true>(A.N) : rollout_kernel_for<true, false>(A.N);
  return st ? rollout_kernel_for<false, true>(A.N) : rollout_kernel_for<false, false>(A.N);
}

static bool launch_rollout(const RolloutArgs &A, dim3 grid, hipStream_t st) {
  RolloutArgs copy = A;
  void *kargs[] = {&copy};
  return hipLaunchKernel(rollout_kernel(A), grid, dim3(kRollBlock), kargs, 0, st) == hipSuccess;
}

}  // namespace rs

using namespace rs;

extern "C" rs_status rollout(rs_ctx *ctx, const rs_params *p, const rs_batch *b,
                             const rs_policy *policy, int32_t horizon, int64_t t_global0,
                             float *obs, uint8_t *actions, float *reward, uint8_t *done,
                             int32_t *qp_stats, void *stream) {
  RS_CHECK_ARG(ctx != nullptr, "ctx is NULL");
  rs_status s = check_params(p);
  if (s != RS_OK) return s;
  RS_CHECK_ARG(b != nullptr && policy != nullptr, "batch/policy is NULL");
  RS_CHECK_ARG(p->dtype == RS_F32, "rollout runs in FP32 (dtype must be RS_F32)");
  RS_CHECK_ARG(action_driven(p->controller), "rollout samples actions: discrete, waypoint or pose controller");
  RS_CHECK_ARG(b->num_envs >= 1, "num_envs must be >= 1");
  RS_CHECK_ARG((int64_t)b->num_envs * b->robots < (int64_t)1 << 31, "num_envs * robots must be < 2^31");
  RS_CHECK_ARG(b->robots >= 2 && 2 * b->robots + 4 <= 32,
               "rollout needs 2 <= robots and 2*robots+4 <= 32 (got %d)", b->robots);
  RS_CHECK_ARG(horizon >= 1, "horizon must be >= 1");
  RS_CHECK_ARG(policy->in_dim == 2 * b->robots + 4, "policy in_dim %d != 2N+4", policy->in_dim);
  RS_CHECK_ARG(policy->w1 && policy->w2 && policy->w3 && policy->b1 && policy->b2 && policy->b3,
               "policy pointer is NULL");
  RS_CHECK_ARG(actions && reward && done, "actions/reward/done outputs are required");
  RS_CHECK_ARG(b->x && b->y && b->theta && b->goal_x && b->goal_y && b->step && b->episode,
               "state pointer is NULL");
  RS_CHECK_ARG(((uintptr_t)obs & 15) == 0, "obs must be 16-byte aligned");
  RolloutArgs A;
  std::memset(&A, 0, sizeof(A));
  A.C = make_const<float>(*p);
  A.E = b->num_envs;
  A.N = b->robots;
  A.D = 2 * b->robots + 4;
  A.H = horizon;
  A.env_base = (uint32_t)b->env_id_base;
  A.t0 = (uint32_t)t_global0;
  A.x = (float *)b->x; A.y = (float *)b->y; A.th = (float *)b->theta;
  A.gx = (float *)b->goal_x; A.gy = (float *)b->goal_y;
  A.step = b->step; A.episode = b->episode;
  A.w1 = (const __bf16 *)policy->w1; A.w2 = (const __bf16 *)policy->w2;
  A.w3 = (const __bf16 *)policy->w3;
  A.b1 = policy->b1; A.b2 = policy->b2; A.b3 = policy->b3;
  A.obs = obs; A.actions = actions; A.reward = reward; A.done = done;
  A.qp_stats = qp_stats;
  A.qp_fail = ctx->qp_fail;
  const int G = pow2_group(A.N);
  const int waves = (A.E + (64 / G) - 1) / (64 / G);
  const dim3 grid((waves + kRollWaves - 1) / kRollWaves);
  hipStream_t st = (hipStream_t)stream;

  // Replay a captured graph of this launch shape; when only scalar arguments
  // (e.g. the stream time) differ, patch the kernel node of the instantiated
  // graph instead of capturing again.
  RolloutArgs shape = A;
  shape.t0 = 0;
  GraphKey key;
  key.words.resize((sizeof(A) + sizeof(uintptr_t) - 1) / sizeof(uintptr_t) + 1, 0);
  std::memcpy(key.words.data(), &shape, sizeof(shape));
  key.words.back() = grid.x;
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (ctx->graphs.size() >= 32) {
      for (auto &kv : ctx->graphs) {
        (void)hipGraphExecDestroy(kv.second.exec);
        (void)hipGraphDestroy(kv.second.graph);
      }
      ctx->graphs.clear();
    }
    if (!ctx->capture_stream)
      RS_CHECK_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    CachedGraph cg;
    RS_CHECK_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
    const bool ok = launch_rollout(A, grid, ctx->capture_stream);
    hipError_t ce = hipStreamEndCapture(ctx->capture_stream, &cg.graph);
    if (!ok || ce != hipSuccess) {
      set_error("rollout capture failed: %s", hipGetErrorString(ce));
      return RS_ERR_DEVICE;
    }
    size_t nnodes = 1;
    hipError_t ne = hipGraphGetNodes(cg.graph, &cg.node, &nnodes);
    hipError_t ie = hipGraphInstantiate(&cg.exec, cg.graph, nullptr, nullptr, 0);
    if (ne != hipSuccess || nnodes != 1 || ie != hipSuccess) {
      set_error("rollout graph instantiate failed: %s", hipGetErrorString(ie));
      if (cg.graph) (void)hipGraphDestroy(cg.graph);
      return RS_ERR_DEVICE;
    }
    cg.args.assign(reinterpret_cast<const char *>(&A), reinterpret_cast<const char *>(&A) + sizeof(A));
    it = ctx->graphs.emplace(key, cg).first;
  } else if (std::memcmp(it->second.args.data(), &A, sizeof(A)) != 0) {
    RolloutArgs copy = A;
    void *kargs[] = {&copy};
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void *>(rollout_kernel(A));
    kp.gridDim = grid;
    kp.blockDim = dim3(kRollBlock);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    RS_CHECK_HIP(hipGraphExecKernelNodeSetParams(it->second.exec, it->second.node, &kp));
    std::memcpy(it->second.args.data(), &A, sizeof(A));
  }
  RS_CHECK_HIP(hipGraphLaunch(it->second.exec, st));
  return RS_OK;
}

extern "C" rs_status rs_phase_cycles(rs_ctx *ctx, int64_t *out, int32_t waves) {
  RS_CHECK_ARG(ctx != nullptr && out != nullptr && waves >= 1, "ctx/out/waves invalid");
#ifdef RS_PHASE_TIMERS
  RS_CHECK_ARG(waves <= kTimedWaves, "at most %d wavefronts are recorded", kTimedWaves);
  RS_CHECK_HIP(hipSetDevice(ctx->device));
  RS_CHECK_HIP(hipDeviceSynchronize());
  RS_CHECK_HIP(hipMemcpyFromSymbol(out, HIP_SYMBOL(rs_phase_cycles_dev),
                                   (size_t)waves * kPhases * sizeof(int64_t), 0,
                                   hipMemcpyDeviceToHost));
  return RS_OK;
#else
  set_error("phase timers are compiled out (build with RS_PHASE_TIMERS)");
  return RS_ERR_UNSUPPORTED;
#endif
}
