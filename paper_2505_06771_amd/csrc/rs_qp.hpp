// rs_qp.hpp -- barrier-certificate QP of one environment, solved exactly by
// the lane group that owns it.
//
// Problem (control barrier certificate of JaxRobotarium Sec. 4.1, with the
// cubic class-K pairwise rows and wall rows defined in robostep.h):
//     min |u - u_nom|^2   s.t.  -2 D_ij.u_i + 2 D_ij.u_j <= gamma h_ij^3  (i<j)
//                               lo_i <= u_i <= hi_i                     (per coordinate)
// The minimiser is the Euclidean projection of u_nom onto a polytope, hence
// unique. It is found with a dual active-set method in the style of Goldfarb
// and Idnani (1983) specialised to the identity Hessian:
//   * bound rows are unit rows, so an active bound simply fixes its coordinate;
//     the active pairwise rows S enter a Gram system restricted to the free
//     coordinates, G_S = C_S^free C_S^free^T (q x q, q small), factored by
//     Cholesky in LDS;
//   * the start point clips u_nom to the box, which is exactly the state after
//     adding every violated bound (they are mutually orthogonal);
//   * each iteration adds the most violated row (normalised violation),
//     stepping along its component z orthogonal to the active set and
//     dropping an active row whose multiplier would turn negative.
// Rows that no point of the speed box can violate (4 v_max (|Dx|+|Dy|) <= b)
// are never examined: they are implied by the box, so the solution is
// unchanged.
//
// Work split inside the group: lane i owns robot i (its u, bounds, fixed
// flags and bound multipliers) and the pairs (i, i+k mod N), k = 1..N/2
// (k = N/2 only for i < N/2), so every pair has exactly one owner and the
// violation scan costs ceil((N-1)/2) rounds. The q x q algebra is done
// identically by every lane of the group from group-uniform data.
#pragma once

#include "rs_device.hpp"

namespace rs {

template <typename T, int G> struct alignas(16) QPScratch {
  int act[2 * G];           // active pair rows: a | b << 8, a < b
  T dx[2 * G], dy[2 * G];   // D = p_a - p_b of each active row
  T lam[2 * G];             // multipliers (objective 1/2 |u - u_nom|^2)
  T rv[2 * G];              // r = G_S^-1 g
  T L[(2 * G) * (2 * G + 1) / 2];  // packed lower Cholesky factor of G_S
};

__device__ __forceinline__ int tri(int a, int b) { return (a * (a + 1)) / 2 + b; }

// Owner lane and rotation distance of pair (a, b), a < b, among N robots.
__device__ __forceinline__ void pair_owner(int a, int b, int N, int &owner, int &k) {
  const int d = b - a;
  if (2 * d <= N) {
    owner = a;
    k = d;
  } else {
    owner = b;
    k = N - d;
  }
}

// Index of pair (a, b), a < b, in lexicographic order.
__device__ __forceinline__ int pair_index(int a, int b, int N) {
  return a * (2 * N - a - 1) / 2 + (b - a - 1);
}

// min / max / |.| as single instructions (operands are never NaN here).
__device__ __forceinline__ float tmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ float tmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double tmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double tmin(double a, double b) { return __builtin_fmin(a, b); }
// clamp to [lo, hi] with lo <= hi: one median-of-three in FP32
__device__ __forceinline__ float tclamp(float x, float lo, float hi) {
  return __builtin_amdgcn_fmed3f(x, lo, hi);
}
__device__ __forceinline__ double tclamp(double x, double lo, double hi) {
  return __builtin_fmin(__builtin_fmax(x, lo), hi);
}
__device__ __forceinline__ float tabs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double tabs(double a) { return __builtin_fabs(a); }
// Quotient used by the step-length and ratio tests of the solver: in FP32 a
// reciprocal (1 ulp) times the numerator, in FP64 the correctly rounded
// division.
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
template <typename T> __device__ __forceinline__ T big_v();
template <> __device__ __forceinline__ float big_v<float>() { return 3.0e38f; }
template <> __device__ __forceinline__ double big_v<double>() { return 1.0e300; }

// Per-coordinate bounds: speed box intersected with the wall certificates of
// the projection point (walls pulled in by r_s / 2, gain c_b gamma, cubic).
template <typename T, typename CS>
__device__ __forceinline__ void wall_bounds(const CS &C, T px, T py, T &lox, T &hix,
                                            T &loy, T &hiy) {
  const T mxh = C.xwh - px, mxl = px - C.xwl;
  const T myh = C.ywh - py, myl = py - C.ywl;
  hix = tmin(C.vmax, C.kb * (mxh * mxh * mxh));
  lox = tmax(-C.vmax, -(C.kb * (mxl * mxl * mxl)));
  hiy = tmin(C.vmax, C.kb * (myh * myh * myh));
  loy = tmax(-C.vmax, -(C.kb * (myl * myl * myl)));
}

// Gram entry of active rows s, t over the free coordinates.
template <typename T>
__device__ __forceinline__ T gram_entry(int as, int bs, T dxs, T dys, int at, int bt, T dxt,
                                        T dyt, uint32_t freex, uint32_t freey) {
  T acc = T(0);
  // robot shared as the "a" (sign -) or "b" (sign +) end of each row
  const int ends_s[2] = {as, bs};
  const int ends_t[2] = {at, bt};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int r = ends_s[u];
      if (r == ends_t[v]) {
        const T sg = (u == v) ? T(4) : T(-4);
        T dd = T(0);
        if ((freex >> r) & 1u) dd += dxs * dxt;
        if ((freey >> r) & 1u) dd += dys * dyt;
        acc += sg * dd;
      }
    }
  }
  return acc;
}

// Stage of the solver that produced the command.
enum : int {
  kStBox = 0,        // no row violated at the box clip u0
  kStOneRow = 1,     // one violated row: closed-form projection
  kStTwoRows = 2,    // two violated rows on four distinct robots
  kStShared = 3,     // two or three rows through shared robots (Gram system, no bound)
  kStActiveSet = 4,  // register-resident active-set loop
  kStGeneral = 5     // general active-set solver with its rows in LDS
};

struct QPInfo {
  int status;  // 0 solved, 1 infeasible, 2 iteration cap / numerical failure
  int iters;   // active-set iterations
  int q;       // active pairwise rows at exit
  int in_lds;  // 1: the rows are in sh->act / sh->lam (general solver)
  int stage;   // kSt*: the stage that produced the command
};

// Per-env certificate statistics (the qp_stats outputs): slots 0..5 count
// solves by the stage that produced the command, slot 6 infeasible solves,
// slot 7 solves stopped by the iteration cap or a numerical failure (neither
// of the last two is counted in 0..5), slot 8 the active-set iterations of
// the solves that ran the loop.
constexpr int kQPStats = 9;
__device__ __forceinline__ int qp_stat_slot(const QPInfo &q) {
  return q.status == 1 ? 6 : (q.status == 2 ? 7 : q.stage);
}
// Adds one solve to an env's counters (one lane of the group calls it).
__device__ __forceinline__ void qp_stats_add(int32_t *q, const QPInfo &info) {
  q[qp_stat_slot(info)] += 1;
  if (info.stage >= kStActiveSet) q[8] += info.iters;
}
// Always-on failure counters of a context: [0] infeasible, [1] capped.
__device__ __forceinline__ void qp_fail_count(unsigned long long *fail, const QPInfo &info) {
  if (fail && info.status != 0) atomicAdd(fail + (info.status - 1), 1ull);
}

// General solver with the active set in LDS (any number of active rows).
// Every lane of the group must call this together (uniform control flow
// within the group). `i` is the robot index (lane in group), `on` = i < N. On
// return (ux, uy) is the command; for status 1 it is the per-coordinate
// fallback. Used when the register-resident solver below runs out of slots.
template <typename T, int G>
__device__ QPInfo qp_solve_lds(QPScratch<T, G> *sh, const SimConst<T> C, int lane, int i, int N,
                           bool on, T px, T py, T uhx, T uhy, T lox, T hix, T loy, T hiy, T &ux,
                           T &uy) {
  const int base = lane & ~(G - 1);
  const T BIG = big_v<T>();
  QPInfo info{0, 0, 0, 1, kStGeneral};

  // --- empty box: infeasible, closed-form fallback -------------------------
  const bool crossed = on && (lox > hix || loy > hiy);
  bool dead = group_any<G>(crossed, lane);

  // --- start: clip to the box; active bounds fix their coordinate ----------
  int fx = 0, fy = 0;  // +1 fixed at upper, -1 fixed at lower
  T mux = T(0), muy = T(0);
  ux = uhx;
  uy = uhy;
  if (on) {
    if (uhx > hix) { ux = hix; fx = 1; mux = uhx - hix; }
    else if (uhx < lox) { ux = lox; fx = -1; mux = lox - uhx; }
    if (uhy > hiy) { uy = hiy; fy = 1; muy = uhy - hiy; }
    else if (uhy < loy) { uy = loy; fy = -1; muy = loy - uhy; }
  }

  int q = 0;
  uint32_t own_act = 0;  // bit k: my rotation-k pair is active
  const int cap = C.qp_cap > 0 ? C.qp_cap : 8 * N + 32;
  const int K = N >> 1;

  while (!dead) {
    // --- most violated constraint ------------------------------------------
    T best = C.tol_add;
    int bid = -1;  // pair: a << 4 | b ; bound: 256 + 4 i + 2 coord + (lower)
    bool coincide = false;
    if (on) {
      if (fx == 0) {
        const T su = ux - hix, sl = lox - ux;
        if (su > best) { best = su; bid = 256 + 4 * i; }
        else if (sl > best) { best = sl; bid = 256 + 4 * i + 1; }
      }
      if (fy == 0) {
        const T su = uy - hiy, sl = loy - uy;
        if (su > best) { best = su; bid = 256 + 4 * i + 2; }
        else if (sl > best) { best = sl; bid = 256 + 4 * i + 3; }
      }
    }
    for (int k = 1; k <= K; ++k) {
      const int j = on ? (i + k >= N ? i + k - N : i + k) : 0;
      const T pxj = __shfl(px, base + j, 64), pyj = __shfl(py, base + j, 64);
      const T uxj = __shfl(ux, base + j, 64), uyj = __shfl(uy, base + j, 64);
      const bool mine = on && !(2 * k == N && i >= k) && !((own_act >> k) & 1u);
      if (mine) {
        const bool ia = i < j;
        const T dx = ia ? px - pxj : pxj - px;
        const T dy = ia ? py - pyj : pyj - py;
        const T d2 = dx * dx + dy * dy;
        const T h = d2 - C.rs2;
        const T bb = C.gamma * (h * h * h);
        if (C.vmax4 * (tabs(dx) + tabs(dy)) > bb) {
          const T dux = ia ? uxj - ux : ux - uxj;  // u_b - u_a
          const T duy = ia ? uyj - uy : uy - uyj;
          const T s = T(2) * (dx * dux + dy * duy) - bb;
          if (d2 > T(0)) {
            const T sn = s * (T(0.35355339059327373) * rsqrt_t(d2));  // s / |c|
            if (sn > best) {
              best = sn;
              bid = (ia ? i : j) << 4 | (ia ? j : i);
            }
          } else if (bb < T(0)) {
            coincide = true;
          }
        }
      }
    }
    if (group_any<G>(coincide, lane)) { dead = true; break; }
    group_argmax<G>(best, bid);
    if (bid < 0) break;  // optimal
    if (++info.iters > cap) { info.status = 2; break; }

    // --- constraint p -------------------------------------------------------
    const bool p_pair = bid < 256;
    const int pa = p_pair ? (bid >> 4) : ((bid - 256) >> 2);
    const int pb = p_pair ? (bid & 15) : 0;
    const int pk = p_pair ? 0 : (((bid - 256) >> 1) & 1);     // bound coordinate
    const int psig = p_pair ? 0 : (((bid - 256) & 1) ? -1 : 1);  // +1 upper
    T dpx = T(0), dpy = T(0), bp = T(0);
    {
      const T xa = __shfl(px, base + pa, 64), ya = __shfl(py, base + pa, 64);
      const T xb = __shfl(px, base + pb, 64), yb = __shfl(py, base + pb, 64);
      if (p_pair) {
        dpx = xa - xb;
        dpy = ya - yb;
        const T h = dpx * dpx + dpy * dpy - C.rs2;
        bp = C.gamma * (h * h * h);
      }
    }
    T lam_p = T(0);
    bool added = false;
    for (int inner = 0; inner < cap && !added; ++inner) {
      const uint32_t freex = ~group_bits<G>(__ballot(fx != 0), lane);
      const uint32_t freey = ~group_bits<G>(__ballot(fy != 0), lane);
      // Gram system of the active rows over the free coordinates
      bool chol_ok = true;
      for (int a = 0; a < q && chol_ok; ++a) {
        const int acta = sh->act[a];
        const int aa = acta & 255, ab = acta >> 8;
        const T adx = sh->dx[a], ady = sh->dy[a];
        for (int b = 0; b <= a; ++b) {
          const int actb = sh->act[b];
          T s = gram_entry<T>(aa, ab, adx, ady, actb & 255, actb >> 8, sh->dx[b], sh->dy[b], freex,
                              freey);
          for (int k2 = 0; k2 < b; ++k2) s -= sh->L[tri(a, k2)] * sh->L[tri(b, k2)];
          if (a == b) {
            if (!(s > T(0))) { chol_ok = false; break; }
            sh->L[tri(a, a)] = sqrt_t(s);
          } else {
            sh->L[tri(a, b)] = s / sh->L[tri(b, b)];
          }
        }
      }
      if (!chol_ok) { info.status = 2; break; }
      // g = C_S^free c_p, then r = G_S^-1 g (forward, backward substitution)
      for (int a = 0; a < q; ++a) {
        const int acta = sh->act[a];
        const int aa = acta & 255, ab = acta >> 8;
        T g;
        if (p_pair) {
          g = gram_entry<T>(aa, ab, sh->dx[a], sh->dy[a], pa, pb, dpx, dpy, freex, freey);
        } else {
          const T comp = pk ? sh->dy[a] : sh->dx[a];
          g = (pa == aa) ? T(-2) * comp : ((pa == ab) ? T(2) * comp : T(0));
          g *= T(psig);
        }
        for (int k2 = 0; k2 < a; ++k2) g -= sh->L[tri(a, k2)] * sh->rv[k2];
        sh->rv[a] = g / sh->L[tri(a, a)];
      }
      for (int a = q - 1; a >= 0; --a) {
        T s = sh->rv[a];
        for (int k2 = a + 1; k2 < q; ++k2) s -= sh->L[tri(k2, a)] * sh->rv[k2];
        sh->rv[a] = s / sh->L[tri(a, a)];
      }
      // (C_S^T r) and c_p at my robot
      T crx = T(0), cry = T(0);
      for (int a = 0; a < q; ++a) {
        const int acta = sh->act[a];
        const T ra = sh->rv[a];
        if (i == (acta & 255)) { crx -= T(2) * sh->dx[a] * ra; cry -= T(2) * sh->dy[a] * ra; }
        else if (i == (acta >> 8)) { crx += T(2) * sh->dx[a] * ra; cry += T(2) * sh->dy[a] * ra; }
      }
      T cpx = T(0), cpy = T(0);
      if (p_pair) {
        if (i == pa) { cpx = T(-2) * dpx; cpy = T(-2) * dpy; }
        else if (i == pb) { cpx = T(2) * dpx; cpy = T(2) * dpy; }
      } else if (i == pa) {
        if (pk) cpy = T(psig); else cpx = T(psig);
      }
      if (!on) { crx = cry = cpx = cpy = T(0); }
      const T zx = fx == 0 ? cpx - crx : T(0);
      const T zy = fy == 0 ? cpy - cry : T(0);
      const T rfx = fx != 0 ? T(fx) * (cpx - crx) : T(0);
      const T rfy = fy != 0 ? T(fy) * (cpy - cry) : T(0);
      const T zz = group_sum<G>(zx * zx + zy * zy);
      T cpn2;
      if (p_pair) {
        T sa = T(0), sb = T(0);
        if ((freex >> pa) & 1u) sa += dpx * dpx;
        if ((freey >> pa) & 1u) sa += dpy * dpy;
        if ((freex >> pb) & 1u) sb += dpx * dpx;
        if ((freey >> pb) & 1u) sb += dpy * dpy;
        cpn2 = T(4) * (sa + sb);
      } else {
        cpn2 = T(1);
      }
      // blocking step t1: active rows first (uniform), then my fixed bounds
      T t1 = BIG;
      int drop = -1;  // pair slot, or 1024 + 2 robot + coord for a bound
      for (int a = 0; a < q; ++a) {
        const T ra = sh->rv[a];
        if (ra > C.eps_r) {
          const T ratio = qdiv(sh->lam[a], ra);
          if (ratio < t1) { t1 = ratio; drop = a; }
        }
      }
      if (on && fx != 0 && rfx > C.eps_r) {
        const T ratio = qdiv(mux, rfx);
        if (ratio < t1 || (ratio == t1 && drop < 0)) { t1 = ratio; drop = 1024 + 2 * i; }
      }
      if (on && fy != 0 && rfy > C.eps_r) {
        const T ratio = qdiv(muy, rfy);
        if (ratio < t1 || (ratio == t1 && drop < 0)) { t1 = ratio; drop = 1024 + 2 * i + 1; }
      }
      group_argmin<G>(t1, drop);
      // current violation of p
      T sp;
      if (p_pair) {
        const T uxa = __shfl(ux, base + pa, 64), uya = __shfl(uy, base + pa, 64);
        const T uxb = __shfl(ux, base + pb, 64), uyb = __shfl(uy, base + pb, 64);
        sp = T(2) * (dpx * (uxb - uxa) + dpy * (uyb - uya)) - bp;
      } else {
        const T mine = pk ? (psig > 0 ? uy - hiy : loy - uy) : (psig > 0 ? ux - hix : lox - ux);
        sp = __shfl(mine, base + pa, 64);
      }
      const bool z_ok = zz > C.eps_z * cpn2;
      const T t2 = z_ok ? qdiv(sp, zz) : BIG;
      if (drop < 0 && !z_ok) { dead = true; break; }  // no step can restore p
      const bool full = z_ok && (drop < 0 || t2 <= t1);
      const T t = full ? t2 : t1;
      if (z_ok) {
        ux -= t * zx;
        uy -= t * zy;
      }
      for (int a = 0; a < q; ++a) sh->lam[a] = sh->lam[a] - t * sh->rv[a];
      if (on) {
        mux -= t * rfx;
        muy -= t * rfy;
      }
      lam_p += t;
      if (full) {
        if (p_pair) {
          if (q >= 2 * G) { info.status = 2; break; }
          sh->act[q] = pa | (pb << 8);
          sh->dx[q] = dpx;
          sh->dy[q] = dpy;
          sh->lam[q] = lam_p;
          ++q;
          int owner, kk;
          pair_owner(pa, pb, N, owner, kk);
          if (i == owner) own_act |= 1u << kk;
        } else if (i == pa) {
          if (pk) { fy = psig; muy = lam_p; uy = psig > 0 ? hiy : loy; }
          else { fx = psig; mux = lam_p; ux = psig > 0 ? hix : lox; }
        }
        added = true;
      } else if (drop >= 1024) {
        const int r = (drop - 1024) >> 1, c = (drop - 1024) & 1;
        if (i == r) {
          if (c) { fy = 0; muy = T(0); } else { fx = 0; mux = T(0); }
        }
      } else {
        const int act = sh->act[drop];
        int owner, kk;
        pair_owner(act & 255, act >> 8, N, owner, kk);
        if (i == owner) own_act &= ~(1u << kk);
        for (int a = drop; a + 1 < q; ++a) {
          sh->act[a] = sh->act[a + 1];
          sh->dx[a] = sh->dx[a + 1];
          sh->dy[a] = sh->dy[a + 1];
          sh->lam[a] = sh->lam[a + 1];
        }
        --q;
      }
      if (++info.iters > cap) { info.status = 2; break; }
    }
    if (info.status == 2 || dead) break;
  }

  if (dead) {
    info.status = 1;
    if (on) {
      ux = lox <= hix ? tmin(tmax(uhx, lox), hix) : T(0.5) * (lox + hix);
      uy = loy <= hiy ? tmin(tmax(uhy, loy), hiy) : T(0.5) * (loy + hiy);
    }
  }
  info.q = dead ? 0 : q;
  return info;
}

}  // namespace rs

namespace rs {

// ---------------------------------------------------------------------------
// Register-resident solver (the hot path). Same method as qp_solve_lds, but
//  * the active pairwise rows live in kQR group-uniform register slots, so
//    the q x q Gram/Cholesky algebra is straight-line code on registers;
//  * a lane owns the pairs (i, (i+K) mod G), K = 1..G/2 (K = G/2 only for
//    i < G/2), whose geometry (D, b, 1/|c|) is computed once per solve from
//    DPP rotations of the projection points;
//  * every cross-lane quantity (argmax with the row's data as payload, |z|^2,
//    the violation of the entering row, the blocking step) is a DPP butterfly
//    over the group: no LDS traffic at all.
// When a row must enter while all slots are taken, or the Gram system loses
// positive definiteness, the general solver restarts from scratch.
// ---------------------------------------------------------------------------
constexpr int kQR = 4;

template <typename T> struct QPActive {
  int q;
  int rows_in_lds;  // 1: the rows are in sh->act / sh->lam (active-set loops)
  int sa[kQR], sb[kQR];
  T slam[kQR];
};

template <int G, typename T>
__device__ __forceinline__ void gargmax_payload(T &v, int &id, T &p0, T &p1, T &p2) {
  auto step = [&](auto cc) {
    constexpr int CT = decltype(cc)::value;
    const T w = dpp<CT>(v), q0 = dpp<CT>(p0), q1 = dpp<CT>(p1), q2 = dpp<CT>(p2);
    const int j = dpp<CT>(id);
    if (w > v || (w == v && j < id)) { v = w; id = j; p0 = q0; p1 = q1; p2 = q2; }
  };
  step(std::integral_constant<int, 0xB1>{});
  if constexpr (G >= 4) step(std::integral_constant<int, 0x4E>{});
  if constexpr (G >= 8) step(std::integral_constant<int, 0x141>{});
  if constexpr (G >= 16) step(std::integral_constant<int, 0x140>{});
}

template <int G, typename T> __device__ __forceinline__ void gargmax(T &v, int &id) {
  auto step = [&](auto cc) {
    constexpr int CT = decltype(cc)::value;
    const T w = dpp<CT>(v);
    const int j = dpp<CT>(id);
    if (w > v || (w == v && j < id)) { v = w; id = j; }
  };
  step(std::integral_constant<int, 0xB1>{});
  if constexpr (G >= 4) step(std::integral_constant<int, 0x4E>{});
  if constexpr (G >= 8) step(std::integral_constant<int, 0x141>{});
  if constexpr (G >= 16) step(std::integral_constant<int, 0x140>{});
}

template <int G, typename T> __device__ __forceinline__ void gargmin(T &v, int &id) {
  auto step = [&](auto cc) {
    constexpr int CT = decltype(cc)::value;
    const T w = dpp<CT>(v);
    const int j = dpp<CT>(id);
    if (w < v || (w == v && j < id)) { v = w; id = j; }
  };
  step(std::integral_constant<int, 0xB1>{});
  if constexpr (G >= 4) step(std::integral_constant<int, 0x4E>{});
  if constexpr (G >= 8) step(std::integral_constant<int, 0x141>{});
  if constexpr (G >= 16) step(std::integral_constant<int, 0x140>{});
}

// Lane of the group holding the largest positive score (ties: smaller lane),
// or -1 if no lane has one. A non-negative float orders like its bit pattern
// read as an unsigned integer, so the score's bits, truncated by one byte,
// carry 255 - lane in the low byte and a single unsigned-max butterfly
// decides; the caller then reads the winner's payload from its lane.
template <int G, typename T>
__device__ __forceinline__ int group_argmax_lane(T score, bool has, int i) {
  const uint32_t key0 =
      has ? ((__float_as_uint((float)score) & 0xFFFFFF00u) | (uint32_t)(255 - i)) : 0u;
  const int key = gred<G>((int)key0, [](int a, int b) { return (uint32_t)a > (uint32_t)b ? a : b; });
  return key == 0 ? -1 : 255 - (key & 255);
}

// Owner lane and rotation of pair (a, b), a < b, under the mod-G ownership.
template <int G> __device__ __forceinline__ void pair_owner_g(int a, int b, int &owner, int &k) {
  const int d = b - a;
  if (2 * d <= G) { owner = a; k = d; }
  else { owner = b; k = G - d; }
}

// Result of the active-set loop: six values, so that it comes back in
// registers (a larger result would travel through scratch memory, and
// reading it back would wait for every outstanding store of the wavefront).
template <typename T> struct QPLoopOut {
  T ux, uy;
  int status, iters, q, in_lds;
};

// The active-set loop, kept out of line: it runs for the few environments the
// closed-form stages leave, and inlined its registers would weigh on every
// step. It rebuilds the pair geometry and the box clip from the arguments and
// starts from the box clip or, with `seed`, from the one-row solution of row
// (fpa, fpb) with multiplier fl1 (fdx, fdy = p_a - p_b). Every lane of the
// group calls it together. Only scalars cross the call. With want_rows the
// active rows and their multipliers are left in sh->act / sh->lam (as the
// general solver leaves them) for the caller to read.
template <typename T, int G>
__device__ __noinline__ QPLoopOut<T> qp_active_set(QPScratch<T, G> *sh, int lane, int i, int N,
                                                   bool on, T px, T py, T uhx, T uhy, T lox,
                                                   T hix, T loy, T hiy, bool seed, int fpa,
                                                   int fpb, T fl1, T fdx, T fdy, T rs2, T gamma,
                                                   T vmax4, T tol_add, T eps_z, T eps_r,
                                                   int qp_cap, bool want_rows) {
  constexpr int KH = G / 2;
  const T BIG = big_v<T>();
  SimConst<T> C{};
  C.rs2 = rs2;
  C.gamma = gamma;
  C.vmax4 = vmax4;
  C.tol_add = tol_add;
  C.eps_z = eps_z;
  C.eps_r = eps_r;
  C.qp_cap = qp_cap;
  // the wavefronts in this loop are the slowest of a launch: give them the
  // first claim on issue slots over the other wavefront of their SIMD
  __builtin_amdgcn_s_setprio(1);
  QPInfo info{0, 0, 0, 0, kStBox};
  bool dead = false;
  T ux, uy;
  // --- geometry of the owned pairs ------------------------------------------
  T cdx[KH], cdy[KH], cb[KH], crn[KH];
  int cpid[KH];
  static_for<1, KH + 1>([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const T pxj = grot<G, K>(px, lane), pyj = grot<G, K>(py, lane);
    const int j = (i + K) & (G - 1);
    const bool valid = on && j < N && !(2 * K == G && i >= KH);
    const bool ia = i < j;
    const T dx = ia ? px - pxj : pxj - px;
    const T dy = ia ? py - pyj : pyj - py;
    const T d2 = dx * dx + dy * dy;
    const T h = d2 - C.rs2;
    const T bb = C.gamma * (h * h * h);
    const bool cand = valid && (C.vmax4 * (tabs(dx) + tabs(dy)) > bb);
    cdx[K - 1] = dx;
    cdy[K - 1] = dy;
    cb[K - 1] = bb;
    crn[K - 1] = d2 > T(0) ? T(0.35355339059327373) * rsqrt_t(d2) : T(0);
    cpid[K - 1] = (cand && d2 > T(0)) ? ((ia ? i : j) << 4 | (ia ? j : i)) : -1;
  });
  // --- start: clip to the box; active bounds fix their coordinate ----------
  int fx = 0, fy = 0;
  T mux = T(0), muy = T(0);
  ux = uhx;
  uy = uhy;
  if (on) {
    if (uhx > hix) { ux = hix; fx = 1; mux = uhx - hix; }
    else if (uhx < lox) { ux = lox; fx = -1; mux = lox - uhx; }
    if (uhy > hiy) { uy = hiy; fy = 1; muy = uhy - hiy; }
    else if (uhy < loy) { uy = loy; fy = -1; muy = loy - uhy; }
  }

  const int cap = C.qp_cap > 0 ? C.qp_cap : 8 * N + 32;
  // Active pairwise rows: group-uniform slots (robots, multiplier) and, per
  // lane, the row's coefficients at the lane's robot (zero unless the robot is
  // one of the row's two ends). Gram entries and the products with the
  // entering row are then one butterfly sum each.
  int q = 0;
  int sa[kQR], sb[kQR];
  T slam[kQR], ccx[kQR], ccy[kQR];
  // Cholesky factor of the Gram system over the free coordinates, kept across
  // iterations: a row entering by a full step appends [w, |z|] (since
  // |z|^2 = c_p^T c_p - |L^-1 g|^2); any change of the free set or a dropped
  // row refactors.
  T L[kQR * (kQR + 1) / 2], Linv[kQR];
  bool lvalid = true;
#pragma unroll
  for (int a = 0; a < kQR; ++a) {
    sa[a] = sb[a] = -1;
    slam[a] = ccx[a] = ccy[a] = T(0);
    Linv[a] = T(0);
#pragma unroll
    for (int b = 0; b <= a; ++b) L[tri(a, b)] = T(0);
  }
  uint32_t own_act = 0;
  bool restart = false;

  if (seed) {
    // row (fpa, fpb) active with multiplier fl1; its robots' coordinates are
    // free or clipped at that multiplier, and the clipped ones are fixed with
    // the bound multiplier that makes the point stationary
    q = 1;
    sa[0] = fpa;
    sb[0] = fpb;
    slam[0] = fl1;
    lvalid = false;
    info.iters = 1;
    int owner, kk;
    pair_owner_g<G>(fpa, fpb, owner, kk);
    if (i == owner) own_act |= 1u << kk;
    ccx[0] = i == fpa ? T(-2) * fdx : (i == fpb ? T(2) * fdx : T(0));
    ccy[0] = i == fpa ? T(-2) * fdy : (i == fpb ? T(2) * fdy : T(0));
    if (on && (i == fpa || i == fpb)) {
      const T vx = uhx - fl1 * ccx[0];
      const T vy = uhy - fl1 * ccy[0];
      ux = tclamp(vx, lox, hix);
      uy = tclamp(vy, loy, hiy);
      fx = vx > hix ? 1 : (vx < lox ? -1 : 0);
      mux = vx > hix ? vx - hix : (vx < lox ? lox - vx : T(0));
      fy = vy > hiy ? 1 : (vy < loy ? -1 : 0);
      muy = vy > hiy ? vy - hiy : (vy < loy ? loy - vy : T(0));
    }
  }
  const bool run_gi = true;

  // --- active-set loop ---------------------------------------------------------
  // One flat loop. Without a pending row an iteration picks the most violated
  // row p; with one it takes a step toward satisfying p: a full step makes p
  // active, a partial step releases the blocking active row or fixed bound.
  // Unused slots hold zero coefficients and identity rows of the factor, so
  // the slot algebra runs over all kQR slots as straight-line code.
  bool pend = false;
  bool p_pair = false;
  int pa = 0, pb = 0, pk = 0, psig = 0;
  T cpx = T(0), cpy = T(0), bp = T(0), lam_p = T(0);
#pragma unroll
  for (int a = 0; a < kQR; ++a) {
    if (a >= q) {
      L[tri(a, a)] = T(1);
      Linv[a] = T(1);
    }
  }
  bool go = run_gi && !dead;
  [[maybe_unused]] bool first = true;  // FP32: the first pick may take the caller's row
  while (go) {
    if constexpr (std::is_same<T, float>::value) {
      // FP32: the caller hands over the row its closed-form stages found most
      // violated at this start: with a seed, through the group's scratch
      // (L[0..3]: row id a << 4 | b, D = p_a - p_b, b); without one, the rows
      // of a rejected guess (or four or more rows violated at u0) start at
      // u0, where the row (fpa, fpb, fdx, fdy) is the most violated one, its
      // b from the same formula as the geometry above. It enters without a scan once its
      // violation here is confirmed; otherwise (or with no row handed over)
      // the first pick scans as usual.
      if (first) {
        first = false;
        int pid = fpa >= 0 ? (fpa << 4 | fpb) : -1;
        T rdx = fdx, rdy = fdy;
        const T rd2 = fdx * fdx + fdy * fdy;
        const T rh = rd2 - C.rs2;
        T rb = C.gamma * (rh * rh * rh);
        if (seed) {
          const float4 pr = reinterpret_cast<const float4 *>(sh->L)[0];
          pid = __float_as_int(pr.x);
          rdx = pr.y;
          rdy = pr.z;
          rb = pr.w;
        }
        const int ea = pid >> 4, eb = pid & 15;
        const T sgn = i == ea ? T(-2) : (i == eb ? T(2) : T(0));
        const T ex = on ? sgn * rdx : T(0), ey = on ? sgn * rdy : T(0);
        const T v0 = gsum<G>(ex * ux + ey * uy) - rb;
        if (pid >= 0 && v0 > T(0)) {
          if (++info.iters > cap) { info.status = 2; break; }
          p_pair = true;
          pa = ea;
          pb = eb;
          pk = 0;
          psig = 0;
          cpx = ex;
          cpy = ey;
          bp = rb;
          lam_p = T(0);
          pend = true;
        }
      }
    }
    if (!pend) {
      // --- most violated constraint (argmax carries the row's data) --------
      T best = C.tol_add, bdx = T(0), bdy = T(0), bbb = T(0);
      int bid = -1;
      if (on) {
        if (fx == 0) {
          const T su = ux - hix, sl = lox - ux;
          if (su > best) { best = su; bid = 256 + 4 * i; }
          else if (sl > best) { best = sl; bid = 256 + 4 * i + 1; }
        }
        if (fy == 0) {
          const T su = uy - hiy, sl = loy - uy;
          if (su > best) { best = su; bid = 256 + 4 * i + 2; }
          else if (sl > best) { best = sl; bid = 256 + 4 * i + 3; }
        }
      }
      static_for<1, KH + 1>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        const T uxj = grot<G, K>(ux, lane), uyj = grot<G, K>(uy, lane);
        if (cpid[K - 1] >= 0 && !((own_act >> K) & 1u)) {
          const bool ia = i < ((i + K) & (G - 1));
          const T dux = ia ? uxj - ux : ux - uxj;
          const T duy = ia ? uyj - uy : uy - uyj;
          const T sn = (T(2) * (cdx[K - 1] * dux + cdy[K - 1] * duy) - cb[K - 1]) * crn[K - 1];
          if (sn > best) {
            best = sn;
            bid = cpid[K - 1];
            bdx = cdx[K - 1];
            bdy = cdy[K - 1];
            bbb = cb[K - 1];
          }
        }
      });
      gargmax_payload<G>(best, bid, bdx, bdy, bbb);
      if (bid < 0) break;  // optimal
      if (++info.iters > cap) { info.status = 2; break; }
      p_pair = bid < 256;
      pa = p_pair ? (bid >> 4) : ((bid - 256) >> 2);
      pb = p_pair ? (bid & 15) : -1;
      pk = p_pair ? 0 : (((bid - 256) >> 1) & 1);
      psig = p_pair ? 0 : (((bid - 256) & 1) ? -1 : 1);
      // entering row's coefficients at my robot
      const T sgn = i == pa ? T(-2) : (i == pb ? T(2) : T(0));
      cpx = p_pair ? sgn * bdx : ((i == pa && pk == 0) ? T(psig) : T(0));
      cpy = p_pair ? sgn * bdy : ((i == pa && pk == 1) ? T(psig) : T(0));
      if (!on) cpx = cpy = T(0);
      bp = bbb;
      lam_p = T(0);
      pend = true;
    }
    const bool frx = fx == 0, fry = fy == 0;
    // slots in use by some group of the wavefront: the algebra of the slots
    // beyond them (zero rows, identity rows of the factor) is skipped, which
    // leaves every group's values exactly as if it had run
    int qw = 0;
#pragma unroll
    for (int k = 1; k <= kQR; ++k) qw = __ballot(q >= k) ? k : qw;
    if (!lvalid) {
      // refactor the Gram system over the current free coordinates
      bool pd = true;
#pragma unroll
      for (int a = 0; a < kQR; ++a) {
        if (a < qw) {
#pragma unroll
          for (int b = 0; b <= a; ++b) {
            T sgm = gsum<G>((frx ? ccx[a] * ccx[b] : T(0)) + (fry ? ccy[a] * ccy[b] : T(0)));
#pragma unroll
            for (int k2 = 0; k2 < b; ++k2) sgm -= L[tri(a, k2)] * L[tri(b, k2)];
            if (b == a) {
              sgm = a < q ? sgm : T(1);
              pd = pd && (sgm > T(0));
              const T rs = rsqrt_t(tmax(sgm, T(1e-30)));
              L[tri(a, a)] = sgm * rs;
              Linv[a] = rs;
            } else {
              L[tri(a, b)] = sgm * Linv[b];
            }
          }
        } else {
#pragma unroll
          for (int b = 0; b < a; ++b) L[tri(a, b)] = T(0);
          L[tri(a, a)] = T(1);
          Linv[a] = T(1);
        }
      }
      if (!pd) { restart = true; break; }
      lvalid = true;
    }
    // g = C_S^free c_p, w = L^-1 g, r = L^-T w (zero on unused slots)
    T w[kQR], rv[kQR];
#pragma unroll
    for (int a = 0; a < kQR; ++a) {
      if (a < qw) {
        T g = gsum<G>((frx ? ccx[a] * cpx : T(0)) + (fry ? ccy[a] * cpy : T(0)));
#pragma unroll
        for (int k2 = 0; k2 < a; ++k2) g -= L[tri(a, k2)] * w[k2];
        w[a] = g * Linv[a];
      } else {
        w[a] = T(0);
      }
    }
#pragma unroll
    for (int a = kQR - 1; a >= 0; --a) {
      T sgm = w[a];
#pragma unroll
      for (int k2 = a + 1; k2 < kQR; ++k2) sgm -= L[tri(k2, a)] * rv[k2];
      rv[a] = sgm * Linv[a];
    }
    // C_S^T r at my robot, the primal direction z (free coordinates) and the
    // direction of my fixed bounds' multipliers
    T crx = T(0), cry = T(0);
#pragma unroll
    for (int a = 0; a < kQR; ++a) {
      crx += rv[a] * ccx[a];
      cry += rv[a] * ccy[a];
    }
    const T zx = frx ? cpx - crx : T(0);
    const T zy = fry ? cpy - cry : T(0);
    const T rfx = frx ? T(0) : T(fx) * (cpx - crx);
    const T rfy = fry ? T(0) : T(fy) * (cpy - cry);
    const T zz = gsum<G>(zx * zx + zy * zy);
    const T cpn2 = gsum<G>((frx ? cpx * cpx : T(0)) + (fry ? cpy * cpy : T(0)));
    // blocking step t1 over active rows (uniform) and my fixed bounds
    T t1 = BIG;
    int drop = -1;
#pragma unroll
    for (int a = 0; a < kQR; ++a) {
      const T ratio = qdiv(slam[a], rv[a]);
      const bool ok = a < q && rv[a] > C.eps_r && ratio < t1;
      t1 = ok ? ratio : t1;
      drop = ok ? a : drop;
    }
    {
      const T rx = qdiv(mux, rfx), ry = qdiv(muy, rfy);
      const bool okx = on && !frx && rfx > C.eps_r && (rx < t1 || (rx == t1 && drop < 0));
      t1 = okx ? rx : t1;
      drop = okx ? 1024 + 2 * i : drop;
      const bool oky = on && !fry && rfy > C.eps_r && (ry < t1 || (ry == t1 && drop < 0));
      t1 = oky ? ry : t1;
      drop = oky ? 1024 + 2 * i + 1 : drop;
    }
    gargmin<G>(t1, drop);
    // current violation of p
    T contrib = p_pair ? cpx * ux + cpy * uy : T(0);
    if (!p_pair && on && i == pa)
      contrib = pk ? (psig > 0 ? uy - hiy : loy - uy) : (psig > 0 ? ux - hix : lox - ux);
    const T sp = gsum<G>(contrib) - (p_pair ? bp : T(0));
    const bool z_ok = zz > C.eps_z * cpn2;
    const T t2 = z_ok ? qdiv(sp, zz) : BIG;
    if (drop < 0 && !z_ok) { dead = true; break; }
    const bool full = z_ok && (drop < 0 || t2 <= t1);
    const T t = full ? t2 : t1;
    if (full && p_pair && q == kQR) { restart = true; break; }  // no slot left
    const T tz = z_ok ? t : T(0);
    ux -= tz * zx;
    uy -= tz * zy;
#pragma unroll
    for (int a = 0; a < kQR; ++a) slam[a] -= a < q ? t * rv[a] : T(0);
    mux -= t * rfx;
    muy -= t * rfy;
    lam_p += t;
    if (full && p_pair) {
      // append p at slot q and extend the factor: L[q] = [w, |z|]
      const T rz = rsqrt_t(zz);
#pragma unroll
      for (int a = 0; a < kQR; ++a) {
        const bool here = a == q;
        sa[a] = here ? pa : sa[a];
        sb[a] = here ? pb : sb[a];
        slam[a] = here ? lam_p : slam[a];
        ccx[a] = here ? cpx : ccx[a];
        ccy[a] = here ? cpy : ccy[a];
#pragma unroll
        for (int k2 = 0; k2 < a; ++k2) L[tri(a, k2)] = here ? w[k2] : L[tri(a, k2)];
        L[tri(a, a)] = here ? zz * rz : L[tri(a, a)];
        Linv[a] = here ? rz : Linv[a];
      }
      ++q;
      int owner, kk;
      pair_owner_g<G>(pa, pb, owner, kk);
      if (i == owner) own_act |= 1u << kk;
    } else if (full) {
      // p is a bound: fix the coordinate
      if (i == pa) {
        if (pk) { fy = psig; muy = lam_p; uy = psig > 0 ? hiy : loy; }
        else { fx = psig; mux = lam_p; ux = psig > 0 ? hix : lox; }
      }
      lvalid = false;
    } else if (drop >= 1024) {
      const int r = (drop - 1024) >> 1, cc2 = (drop - 1024) & 1;
      if (i == r) {
        if (cc2) { fy = 0; muy = T(0); } else { fx = 0; mux = T(0); }
      }
      lvalid = false;
    } else {
      // release active row `drop`: shift the later slots down
      int owner = 0, kk = 0;
#pragma unroll
      for (int a = 0; a < kQR; ++a)
        if (a == drop) pair_owner_g<G>(sa[a], sb[a], owner, kk);
      if (i == owner) own_act &= ~(1u << kk);
#pragma unroll
      for (int a = 0; a < kQR; ++a) {
        const bool mv = a >= drop && a + 1 < q;
        const bool clr = a >= drop && !mv;
        if (a + 1 < kQR) {
          sa[a] = mv ? sa[a + 1] : (clr ? -1 : sa[a]);
          sb[a] = mv ? sb[a + 1] : (clr ? -1 : sb[a]);
          slam[a] = mv ? slam[a + 1] : (clr ? T(0) : slam[a]);
          ccx[a] = mv ? ccx[a + 1] : (clr ? T(0) : ccx[a]);
          ccy[a] = mv ? ccy[a + 1] : (clr ? T(0) : ccy[a]);
        } else if (clr) {
          sa[a] = sb[a] = -1;
          slam[a] = ccx[a] = ccy[a] = T(0);
        }
      }
      --q;
      lvalid = false;
    }
    if (full) pend = false;
    if (++info.iters > cap) { info.status = 2; break; }
  }

  QPLoopOut<T> out;
  if (restart && !dead) {
    // more active rows than register slots (or a degenerate Gram system):
    // solve again with the general solver
    const QPInfo r = qp_solve_lds<T, G>(sh, C, lane, i, N, on, px, py, uhx, uhy, lox, hix, loy,
                                        hiy, ux, uy);
    info.status = r.status;
    info.iters += r.iters;
    q = r.q;
    out.in_lds = 1;
  } else {
    out.in_lds = 0;
    if (dead) {
      info.status = 1;
      q = 0;
      if (on) {
        ux = lox <= hix ? tmin(tmax(uhx, lox), hix) : T(0.5) * (lox + hix);
        uy = loy <= hiy ? tmin(tmax(uhy, loy), hiy) : T(0.5) * (loy + hiy);
      }
    }
  }
  out.ux = ux;
  out.uy = uy;
  out.status = info.status;
  out.iters = info.iters;
  out.q = q;
  if (want_rows && !out.in_lds) {
    if (i == 0) {
#pragma unroll
      for (int a = 0; a < kQR; ++a) {
        if (a < q) {
          sh->act[a] = sa[a] | (sb[a] << 8);
          sh->lam[a] = slam[a];
        }
      }
    }
    wave_lds_fence();
  }
  __builtin_amdgcn_s_setprio(0);
  return out;
}

template <typename T, int G>
__device__ QPInfo qp_solve(QPScratch<T, G> *sh, ConstRef<T> K, int qp_cap, int lane, int i, int N,
                           bool on, T px, T py, T uhx, T uhy, T lox, T hix, T loy, T hiy, T &ux,
                           T &uy, QPActive<T> *act_out = nullptr) {
  const auto &C = *K.get();  // the solver's constants, loaded for this phase
  constexpr int KH = G / 2;
  const T BIG = big_v<T>();
  QPInfo info{0, 0, 0, 0, kStBox};

  // --- box clip u0 (every bound holds there) ---------------------------------
  ux = uhx;
  uy = uhy;
  if (on) {
    ux = uhx > hix ? hix : (uhx < lox ? lox : uhx);
    uy = uhy > hiy ? hiy : (uhy < loy ? loy : uhy);
  }

  // --- geometry of the owned pairs and their violations at u0 ---------------
  // (the partner's position and command are fetched together)
  T cdx[KH], cdy[KH], cb[KH], crn[KH], snk[KH];
  int cpid[KH];
  bool coincide = false;
  // FP32 8-lane groups take the partner's (p, u0) from one 16-byte LDS
  // exchange in the group's scratch (free here) instead of four DPP
  // rotations of two moves and a select each
  constexpr bool kLdsX = std::is_same<T, float>::value && G == 8;
  // the FP32 closed-form guesses beyond two rows (every group width alike, so
  // that results do not depend on the schedule)
  constexpr bool kGuess = std::is_same<T, float>::value;
  float4 *xq = reinterpret_cast<float4 *>(sh);
  static_assert(!kGuess || sizeof(QPScratch<T, G>) >= G * (sizeof(float4) + 3 * sizeof(float2)),
                "the exchange fits in the group's scratch");
  if constexpr (kLdsX) {
    xq[i] = make_float4(px, py, ux, uy);
    wave_lds_fence();
  }
  static_for<1, KH + 1>([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    T pxj, pyj, uxj, uyj;
    if constexpr (kLdsX) {
      const float4 v = xq[(i + K) & (G - 1)];
      pxj = v.x; pyj = v.y; uxj = v.z; uyj = v.w;
    } else {
      pxj = grot<G, K>(px, lane); pyj = grot<G, K>(py, lane);
      uxj = grot<G, K>(ux, lane); uyj = grot<G, K>(uy, lane);
    }
    const int j = (i + K) & (G - 1);
    const bool valid = on && j < N && !(2 * K == G && i >= KH);
    // D = p_i - p_j as this lane sees the pair. The row's own D runs from
    // its lower-index robot, which only flips the sign: the distance, the
    // pruning test and the violation do not see it, and it is applied when
    // the row is picked.
    const T dx = px - pxj, dy = py - pyj;
    const T d2 = dx * dx + dy * dy;
    const T h = d2 - C.rs2;
    const T bb = C.gamma * (h * h * h);
    const bool cand = valid && (C.vmax4 * (tabs(dx) + tabs(dy)) > bb);
    cdx[K - 1] = dx;
    cdy[K - 1] = dy;
    cb[K - 1] = bb;
    cpid[K - 1] = (cand && d2 > T(0)) ? (min(i, j) << 4 | max(i, j)) : -1;
    if (cand && !(d2 > T(0)) && bb < T(0)) coincide = true;
    // violation 2 D.(u_j - u_i) - b over |c| = 2 sqrt(2) |D| (a pair with
    // D = 0 is no candidate: its value is never used)
    crn[K - 1] = T(0.35355339059327373) * rsqrt_t(d2);
    const T sn = (T(2) * (dx * (uxj - ux) + dy * (uyj - uy)) - bb) * crn[K - 1];
    snk[K - 1] = cpid[K - 1] >= 0 ? sn : -BIG;
  });
  bool dead = group_any<G>(coincide || (on && (lox > hix || loy > hiy)), lane);

  // outcome of the closed-form stages: rows accepted (fq = 1 or 2), or a
  // one-row start for the active-set loop (seed)
  int fq = 0, fpa = -1, fpb = -1, fqa = -1, fqb = -1, fra = -1, frb = -1;
  T fl1 = T(0), fl2 = T(0), fl3 = T(0), fdx = T(0), fdy = T(0);
  bool seed = false;

  // --- closed-form stages --------------------------------------------------------
  // Every bound holds at the box clip u0. If at most two pairwise rows are
  // violated there, the solution is guessed in closed form and accepted when it
  // satisfies every row through the robots it moves (rows away from them keep
  // their values at u0, where only the guessed rows were violated): being the
  // minimiser over a superset of the feasible set, a feasible guess is the
  // solution.
  //  * One row p = (a, b), or two rows on four distinct robots: each row's
  //    projection onto box & {c.u <= b} is u(l) = clip(u_nom - l c), with
  //    l >= 0 the root of the non-increasing, piecewise linear
  //    phi(l) = c.u(l) - b; its breakpoints are where a coordinate of the
  //    row's two robots meets a bound.
  //  * Two rows through a shared robot: assuming no bound binds on the three
  //    robots, the multipliers solve the 2 x 2 Gram system; the guess also
  //    needs both multipliers >= 0 and the three commands inside their bounds.
  //  * FP32 only: after a rejected one-row guess, rows p and r (the row that
  //    guess violates) both active, or r alone when p's multiplier comes out
  //    negative; and for exactly three violated rows, all three active. Each
  //    solves its rows' Gram system with no bound binding and is accepted
  //    when the multipliers are >= 0, the moved robots stay inside their
  //    boxes and every other row holds: the KKT conditions of the QP.
  // A rejected one-row guess (with p active and the clipped coordinates fixed)
  // is a dual-feasible start for the active-set loop below; otherwise the loop
  // starts from u0.
  bool run_gi = !dead;
  if (!dead) {
    const T thr = C.tol_add;
    const int gbase = lane & ~(G - 1);
    T bdx = T(0), bdy = T(0), bbb = T(0);
    int bid = -1, nv = 0;
    if constexpr (kGuess) {
      // FP32: most violated row of the group by one integer key per row (the
      // score's float bits truncated by a byte, 255 - row id in the low byte:
      // a positive float orders like its bits), the maximum over the owned
      // rows, then over the group by one butterfly. The winner does not depend
      // on which lane owns which row, so it is the same for every group width.
      // Its D and b are recomputed from the two robots' projection points, by
      // the formulas of the scan (the same values the owner holds).
      uint32_t bkey = 0u;
      int nviol = 0;
      static_for<1, KH + 1>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        const bool v = snk[K - 1] > thr;
        nviol += v ? 1 : 0;
        const uint32_t k =
            v ? ((__float_as_uint((float)snk[K - 1]) & 0xFFFFFF00u) | (uint32_t)(255 - cpid[K - 1]))
              : 0u;
        bkey = k > bkey ? k : bkey;
      });
      const int key =
          gred<G>((int)bkey, [](int a, int b) { return (uint32_t)a > (uint32_t)b ? a : b; });
      nv = gsum<G>(nviol);
      bid = key == 0 ? -1 : 255 - (key & 255);
      const int ra = bid < 0 ? 0 : bid >> 4, rb = bid < 0 ? 0 : bid & 15;
      T pax, pay, pbx, pby;
      if constexpr (kLdsX) {
        const float4 va = xq[ra], vb = xq[rb];
        pax = va.x; pay = va.y; pbx = vb.x; pby = vb.y;
      } else {
        pax = __shfl(px, gbase + ra, 64); pay = __shfl(py, gbase + ra, 64);
        pbx = __shfl(px, gbase + rb, 64); pby = __shfl(py, gbase + rb, 64);
      }
      bdx = pax - pbx;
      bdy = pay - pby;
      const T d2 = bdx * bdx + bdy * bdy;
      const T h = d2 - C.rs2;
      bbb = C.gamma * (h * h * h);
    } else {
      T best = thr;
      int nviol = 0;
      static_for<1, KH + 1>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        nviol += snk[K - 1] > thr ? 1 : 0;
        if (snk[K - 1] > best) {
          best = snk[K - 1];
          bid = cpid[K - 1];
          bdx = cdx[K - 1];
          bdy = cdy[K - 1];
          bbb = cb[K - 1];
        }
      });
      // most violated row of the group: winner lane by one integer
      // butterfly, its row's data read from that lane
      const int wl = group_argmax_lane<G>(best, bid >= 0, i);
      nv = gsum<G>(nviol);
      const int src = gbase + (wl < 0 ? 0 : wl);
      bid = wl < 0 ? -1 : __shfl(bid, src, 64);
      bdx = __shfl(bdx, src, 64);
      bdy = __shfl(bdy, src, 64);
      bbb = __shfl(bbb, src, 64);
      // orient D from the row's lower-index robot (the owner is either end)
      const bool flip = wl != (bid >> 4);
      bdx = flip ? -bdx : bdx;
      bdy = flip ? -bdy : bdy;
    }
    if (bid < 0) {
      run_gi = false;  // u0 is the solution
    } else if (nv == 3 && kGuess) {
      if constexpr (kGuess) {
        // Three rows violated at u0 (FP32): guess all three
        // active with no bound binding, from their 3 x 3 Gram system, and
        // accept as the two-row stages do; otherwise the loop starts from u0.
        T sx[2] = {T(0), T(0)}, sy[2] = {T(0), T(0)}, sb[2] = {T(0), T(0)};
        int sid[2] = {-1, -1};
        static_for<0, 2>([&](auto rc) {
          constexpr int R = decltype(rc)::value;
          T b2 = thr, e2x = T(0), e2y = T(0), beta2 = T(0);
          int id2 = -1;
          static_for<1, KH + 1>([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            const int id = cpid[K - 1];
            const bool taken = id == bid || (R == 1 && id == sid[0]);
            if (!taken && snk[K - 1] > b2) {
              b2 = snk[K - 1];
              id2 = id;
              e2x = cdx[K - 1];
              e2y = cdy[K - 1];
              beta2 = cb[K - 1];
            }
          });
          const int w2 = group_argmax_lane<G>(b2, id2 >= 0, i);
          const int src = gbase + (w2 < 0 ? 0 : w2);
          id2 = w2 < 0 ? -1 : __shfl(id2, src, 64);
          e2x = __shfl(e2x, src, 64);
          e2y = __shfl(e2y, src, 64);
          beta2 = __shfl(beta2, src, 64);
          const bool flip2 = w2 != (id2 >> 4);
          sx[R] = flip2 ? -e2x : e2x;
          sy[R] = flip2 ? -e2y : e2y;
          sb[R] = beta2;
          sid[R] = id2;
        });
        const int pa = bid >> 4, pb = bid & 15;
        const int qa = sid[0] >> 4, qb = sid[0] & 15, ra = sid[1] >> 4, rb = sid[1] & 15;
        const bool all3 = sid[0] >= 0 && sid[1] >= 0;
        auto coef = [&](int a, int b, T dx, T dy, T &cx, T &cy) {
          cx = i == a ? T(-2) * dx : (i == b ? T(2) * dx : T(0));
          cy = i == a ? T(-2) * dy : (i == b ? T(2) * dy : T(0));
        };
        T c1x, c1y, c2x, c2y, c3x, c3y;
        coef(pa, pb, bdx, bdy, c1x, c1y);
        coef(qa, qb, sx[0], sy[0], c2x, c2y);
        coef(ra, rb, sx[1], sy[1], c3x, c3y);
        const T g11 = T(8) * (bdx * bdx + bdy * bdy);
        const T g22 = T(8) * (sx[0] * sx[0] + sy[0] * sy[0]);
        const T g33 = T(8) * (sx[1] * sx[1] + sy[1] * sy[1]);
        const T g12 = gsum<G>(c1x * c2x + c1y * c2y);
        const T g13 = gsum<G>(c1x * c3x + c1y * c3y);
        const T g23 = gsum<G>(c2x * c3x + c2y * c3y);
        const T h1 = gsum<G>(c1x * uhx + c1y * uhy) - bbb;
        const T h2 = gsum<G>(c2x * uhx + c2y * uhy) - sb[0];
        const T h3 = gsum<G>(c3x * uhx + c3y * uhy) - sb[1];
        // Cramer's rule on the symmetric 3 x 3 system
        const T m11 = g22 * g33 - g23 * g23, m12 = g12 * g33 - g23 * g13, m13 = g12 * g23 - g22 * g13;
        const T det = g11 * m11 - g12 * m12 + g13 * m13;
        const T idet = qdiv(T(1), det);
        const T l1 = (h1 * m11 - g12 * (h2 * g33 - g23 * h3) + g13 * (h2 * g23 - g22 * h3)) * idet;
        const T l2 = (g11 * (h2 * g33 - g23 * h3) - h1 * m12 + g13 * (g12 * h3 - h2 * g13)) * idet;
        const T l3 = (g11 * (g22 * h3 - h2 * g23) - g12 * (g12 * h3 - h2 * g13) + h1 * m13) * idet;
        bool ok3 = all3 && det > T(1e-6) * g11 * g22 * g33 && l1 >= T(0) && l2 >= T(0) && l3 >= T(0);
        const bool mv = i == pa || i == pb || i == qa || i == qb || i == ra || i == rb;
        const T vx = uhx - l1 * c1x - l2 * c2x - l3 * c3x;
        const T vy = uhy - l1 * c1y - l2 * c2y - l3 * c3y;
        const bool outb = on && mv && (vx < lox || vx > hix || vy < loy || vy > hiy);
        ok3 = ok3 && !group_any<G>(outb, lane);
        const T wx = (on && mv) ? vx : ux, wy = (on && mv) ? vy : uy;  // unmoved: u0
        float2 *xw = reinterpret_cast<float2 *>(sh) + 2 * G;
        xw[i] = make_float2(wx, wy);
        wave_lds_fence();
        bool bad3 = !ok3;
        static_for<1, KH + 1>([&](auto kc) {
          constexpr int K = decltype(kc)::value;
          const float2 v = xw[(i + K) & (G - 1)];
          const int id = cpid[K - 1];
          const T sn = (T(2) * (cdx[K - 1] * (v.x - wx) + cdy[K - 1] * (v.y - wy)) - cb[K - 1]) *
                       crn[K - 1];
          bad3 = bad3 | ((id >= 0) & (id != bid) & (id != sid[0]) & (id != sid[1]) &
                         (sn > C.tol_add));
        });
        const bool accept3 = !group_any<G>(bad3, lane);
        if (accept3) {
          ux = wx;
          uy = wy;
          fq = 3;
          fpa = pa; fpb = pb; fl1 = l1;
          fqa = qa; fqb = qb; fl2 = l2;
          fra = ra; frb = rb; fl3 = l3;
          info.stage = kStShared;
          info.iters = 3;
          run_gi = false;
        } else {
          // the loop starts at u0, where p is the most violated row
          fpa = pa; fpb = pb; fdx = bdx; fdy = bdy;
        }
      }
    } else if (nv <= 2) {
      // the other violated row, if any
      T b2 = thr, e2x = T(0), e2y = T(0), beta2 = T(0);
      int id2 = -1;
      if (nv == 2) {
        static_for<1, KH + 1>([&](auto kc) {
          constexpr int K = decltype(kc)::value;
          if (cpid[K - 1] != bid && snk[K - 1] > b2) {
            b2 = snk[K - 1];
            id2 = cpid[K - 1];
            e2x = cdx[K - 1];
            e2y = cdy[K - 1];
            beta2 = cb[K - 1];
          }
        });
        const int w2 = group_argmax_lane<G>(b2, id2 >= 0, i);
        const int src = gbase + (w2 < 0 ? 0 : w2);
        id2 = w2 < 0 ? -1 : __shfl(id2, src, 64);
        e2x = __shfl(e2x, src, 64);
        e2y = __shfl(e2y, src, 64);
        beta2 = __shfl(beta2, src, 64);
        const bool flip2 = w2 != (id2 >> 4);
        e2x = flip2 ? -e2x : e2x;
        e2y = flip2 ? -e2y : e2y;
      }
      const bool two = nv == 2 && id2 >= 0;
      const int pa = bid >> 4, pb = bid & 15;
      const int qa = two ? id2 >> 4 : pa, qb = two ? id2 & 15 : pb;
      const bool shared = two && (qa == pa || qa == pb || qb == pa || qb == pb);
      bool ok = true;
      T lam1 = T(0), lam2 = T(0);
      T nux = ux, nuy = uy;  // my command under the guess (u0 unless I move)
      // projection onto box & one half-space for each row, on its own two
      // robots; rows one after the other (a true loop keeps the registers of
      // one row) with a trip count uniform over the wavefront
      const int trips = __ballot(two && !shared) ? 2 : 1;
#pragma unroll 1
      for (int rr = 0; rr < trips; ++rr) {
        const bool r2 = rr == 1;
        const bool use = !shared && (!r2 || two);  // this group solves this row
        const int ra = r2 ? qa : pa, rb = r2 ? qb : pb;
        const T dx = r2 ? e2x : bdx, dy = r2 ? e2y : bdy;
        const T beta = r2 ? beta2 : bbb;
        // projection onto the row's hyperplane with every coordinate free: the
        // row's solution whenever it lands inside the box of both its robots
        // (each group takes it then, whatever the other groups need)
        const T cix = i == ra ? T(-2) * dx : (i == rb ? T(2) * dx : T(0));
        const T ciy = i == ra ? T(-2) * dy : (i == rb ? T(2) * dy : T(0));
        const T lamf = (gsum<G>(cix * uhx + ciy * uhy) - beta) * qdiv(T(1), T(8) * (dx * dx + dy * dy));
        const T fvx = uhx - lamf * cix, fvy = uhy - lamf * ciy;
        const bool end_ab = use && (i == ra || i == rb);
        const bool fbad = end_ab && (fvx < lox || fvx > hix || fvy < loy || fvy > hiy);
        const bool free_ok = use && lamf > T(0) && !group_any<G>(fbad, lane);
        if (__ballot(use && !free_ok) == 0) {  // every row of the wave: the free solution
          nux = end_ab ? fvx : nux;
          nuy = end_ab ? fvy : nuy;
          lam2 = r2 ? lamf : lam2;
          lam1 = r2 ? lam1 : lamf;
          continue;
        }
        const int la = gbase + ra, lb = gbase + rb;
        const T cc[4] = {T(-2) * dx, T(-2) * dy, T(2) * dx, T(2) * dy};
        const T un[4] = {__shfl(uhx, la, 64), __shfl(uhy, la, 64), __shfl(uhx, lb, 64),
                         __shfl(uhy, lb, 64)};
        const T lo[4] = {__shfl(lox, la, 64), __shfl(loy, la, 64), __shfl(lox, lb, 64),
                         __shfl(loy, lb, 64)};
        const T hi[4] = {__shfl(hix, la, 64), __shfl(hiy, la, 64), __shfl(hix, lb, 64),
                         __shfl(hiy, lb, 64)};
        auto phi = [&](T lm) {
          T acc = -beta;
#pragma unroll
          for (int k = 0; k < 4; ++k) acc += cc[k] * tclamp(un[k] - lm * cc[k], lo[k], hi[k]);
          return acc;
        };
        // the root lies between the largest breakpoint (or 0) where phi is
        // still positive, (llo, plo), and the smallest one where it is not,
        // (lhi, phi_hi): no breakpoint falls in between, so phi is linear
        // there. The eight breakpoints are shared out over the group's lanes
        // and both ends found by one butterfly (equal breakpoints give equal
        // phi). No breakpoint with phi <= 0: the row cannot be met in the box.
        T llo = T(0), plo = phi(T(0));
        T lhi = BIG, phh = T(0);
        {
          T bl = T(-1), bv = T(0);
          for (int b = i; b < 8; b += G) {
            // breakpoint b: the multiplier where coordinate k = b / 2 meets
            // its upper (b even) or lower (b odd) bound; a coordinate the row
            // does not move gives 0
            const int k = b >> 1;
            auto pick = [&](const T *v) {
              const T lo2 = (k & 1) ? v[1] : v[0], hi2 = (k & 1) ? v[3] : v[2];
              return (k & 2) ? hi2 : lo2;
            };
            const T ck = pick(cc), uk = pick(un), bk = (b & 1) ? pick(lo) : pick(hi);
            const T ek = ck != T(0) ? (uk - bk) * qdiv(T(1), ck) : T(0);
            const T pk = phi(ek);
            const bool pos = pk > T(0);
            const bool better = pos & (ek > bl);
            bl = better ? ek : bl;
            bv = better ? pk : bv;
            const bool upper = !pos & (ek < lhi);
            lhi = upper ? ek : lhi;
            phh = upper ? pk : phh;
          }
          auto merge = [&](auto c) {
            constexpr int CT = decltype(c)::value;
            const T w = dpp<CT>(bl), q = dpp<CT>(bv);
            const bool better = w > bl;
            bl = better ? w : bl;
            bv = better ? q : bv;
            const T wu = dpp<CT>(lhi), qu = dpp<CT>(phh);
            const bool lower = wu < lhi;
            lhi = lower ? wu : lhi;
            phh = lower ? qu : phh;
          };
          merge(std::integral_constant<int, 0xB1>{});
          if constexpr (G >= 4) merge(std::integral_constant<int, 0x4E>{});
          if constexpr (G >= 8) merge(std::integral_constant<int, 0x141>{});
          if constexpr (G >= 16) merge(std::integral_constant<int, 0x140>{});
          plo = bl > llo ? bv : plo;
          llo = bl > llo ? bl : llo;
        }
        ok = ok && (!use || free_ok || lhi < BIG);
        const T lam = free_ok ? lamf : llo + plo * (tmin(lhi, BIG) - llo) * qdiv(T(1), plo - phh);
        const bool ma = use && i == ra, mb = use && i == rb;
        const T ax = tclamp(un[0] - lam * cc[0], lo[0], hi[0]);
        const T ay = tclamp(un[1] - lam * cc[1], lo[1], hi[1]);
        const T bx = tclamp(un[2] - lam * cc[2], lo[2], hi[2]);
        const T by = tclamp(un[3] - lam * cc[3], lo[3], hi[3]);
        nux = free_ok ? (end_ab ? fvx : nux) : (ma ? ax : (mb ? bx : nux));
        nuy = free_ok ? (end_ab ? fvy : nuy) : (ma ? ay : (mb ? by : nuy));
        lam2 = r2 ? lam : lam2;
        lam1 = r2 ? lam1 : lam;
      }
      if (shared) {
        // two rows through a shared robot r; j is p2's other end. With no
        // bound binding on a, b, j: u = u_nom - lam1 c1 - lam2 c2 there.
        const T c1x = i == pa ? T(-2) * bdx : (i == pb ? T(2) * bdx : T(0));
        const T c1y = i == pa ? T(-2) * bdy : (i == pb ? T(2) * bdy : T(0));
        const T c2x = i == qa ? T(-2) * e2x : (i == qb ? T(2) * e2x : T(0));
        const T c2y = i == qa ? T(-2) * e2y : (i == qb ? T(2) * e2y : T(0));
        const T g11 = T(8) * (bdx * bdx + bdy * bdy);
        const T g22 = T(8) * (e2x * e2x + e2y * e2y);
        const T g12 = gsum<G>(c1x * c2x + c1y * c2y);
        const T h1 = gsum<G>(c1x * uhx + c1y * uhy) - bbb;
        const T h2 = gsum<G>(c2x * uhx + c2y * uhy) - beta2;
        const T det = g11 * g22 - g12 * g12;
        const T idet = qdiv(T(1), det);
        lam1 = (g22 * h1 - g12 * h2) * idet;
        lam2 = (g11 * h2 - g12 * h1) * idet;
        ok = det > T(1e-6) * g11 * g22 && lam1 >= T(0) && lam2 >= T(0);
        const bool mv = i == pa || i == pb || i == qa || i == qb;
        const T vx = uhx - lam1 * c1x - lam2 * c2x;
        const T vy = uhy - lam1 * c1y - lam2 * c2y;
        nux = mv ? vx : nux;
        nuy = mv ? vy : nuy;
        const bool out = mv && (vx < lox || vx > hix || vy < loy || vy > hiy);
        ok = ok && !group_any<G>(out, lane);
      }
      // check every candidate row at the guess, except the guessed ones, from
      // the geometry of the scan: a row with both ends unmoved keeps its value
      // at u0 (below the threshold), and a pruned row holds anywhere in the
      // speed box, which contains every guess
      bool bad = !ok;
      float2 *xv = reinterpret_cast<float2 *>(sh) + 2 * G;  // past the scan's exchange
      if constexpr (kLdsX) {
        xv[i] = make_float2(nux, nuy);
        wave_lds_fence();
      }
      static_for<1, KH + 1>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        T uxj, uyj;
        if constexpr (kLdsX) {
          const float2 v = xv[(i + K) & (G - 1)];
          uxj = v.x; uyj = v.y;
        } else {
          uxj = grot<G, K>(nux, lane); uyj = grot<G, K>(nuy, lane);
        }
        const int id = cpid[K - 1];
        const bool guessed = (id == bid) | (two & (id == id2));
        const T sn = (T(2) * (cdx[K - 1] * (uxj - nux) + cdy[K - 1] * (uyj - nuy)) - cb[K - 1]) *
                     crn[K - 1];
        bad = bad | ((id >= 0) & !guessed & (sn > C.tol_add));
      });
      bool accept = !group_any<G>(bad, lane);
      bool seeded = !accept && !two && ok;
      bool second = false;  // accepted on the second guess below
      bool lone = false;    // accepted with the violated row alone
      int sqa = qa, sqb = qb, spa = pa, spb = pb;
      if constexpr (kGuess) {
        // A rejected one-row guess violates some row r, which shares a robot
        // with p (only p's robots moved). Second guess: p and r both active
        // with no bound binding, from their 2 x 2 Gram system, accepted by
        // the checks of the shared-robot stage (wave-uniform branch: only
        // wavefronts with such a group pay for it). The guess's commands go
        // through the group's LDS exchange (xv).
        if (__ballot(seeded) != 0) {
          if constexpr (!kLdsX) {  // the guess's commands into the exchange
            xv[i] = make_float2(nux, nuy);
            wave_lds_fence();
          }
          T rbest = C.tol_add, rdx = T(0), rdy = T(0), rbb = T(0);
          int rid = -1;
          static_for<1, KH + 1>([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            const float2 v = xv[(i + K) & (G - 1)];
            const int id = cpid[K - 1];
            const T sn = (T(2) * (cdx[K - 1] * (v.x - nux) + cdy[K - 1] * (v.y - nuy)) - cb[K - 1]) *
                         crn[K - 1];
            if (seeded && id >= 0 && id != bid && sn > rbest) {
              rbest = sn;
              rid = id;
              rdx = cdx[K - 1];
              rdy = cdy[K - 1];
              rbb = cb[K - 1];
            }
          });
          const int wr = group_argmax_lane<G>(rbest, rid >= 0, i);
          const int src = gbase + (wr < 0 ? 0 : wr);
          rid = wr < 0 ? -1 : __shfl(rid, src, 64);
          rdx = __shfl(rdx, src, 64);
          rdy = __shfl(rdy, src, 64);
          rbb = __shfl(rbb, src, 64);
          const bool flipr = wr != (rid >> 4);
          rdx = flipr ? -rdx : rdx;
          rdy = flipr ? -rdy : rdy;
          // a seeded loop starts at this guess, where r is the most violated
          // row: handed over through the group's scratch (L[0..3])
          if (seeded && i == 0)
            reinterpret_cast<float4 *>(sh->L)[0] = make_float4(__int_as_float(rid), rdx, rdy, rbb);
          const int ra = rid >> 4, rb = rid & 15;
          const bool try2 =
              seeded && rid >= 0 && (ra == pa || ra == pb || rb == pa || rb == pb);
          const T c1x = i == pa ? T(-2) * bdx : (i == pb ? T(2) * bdx : T(0));
          const T c1y = i == pa ? T(-2) * bdy : (i == pb ? T(2) * bdy : T(0));
          const T c2x = i == ra ? T(-2) * rdx : (i == rb ? T(2) * rdx : T(0));
          const T c2y = i == ra ? T(-2) * rdy : (i == rb ? T(2) * rdy : T(0));
          const T g11 = T(8) * (bdx * bdx + bdy * bdy);
          const T g22 = T(8) * (rdx * rdx + rdy * rdy);
          const T g12 = gsum<G>(c1x * c2x + c1y * c2y);
          const T h1 = gsum<G>(c1x * uhx + c1y * uhy) - bbb;
          const T h2 = gsum<G>(c2x * uhx + c2y * uhy) - rbb;
          const T det = g11 * g22 - g12 * g12;
          const T idet = qdiv(T(1), det);
          const T m1 = (g22 * h1 - g12 * h2) * idet;
          const T m2 = (g11 * h2 - g12 * h1) * idet;
          bool ok2 = try2 && det > T(1e-6) * g11 * g22 && m1 >= T(0) && m2 >= T(0);
          const bool mv = i == pa || i == pb || i == ra || i == rb;
          const T vx = uhx - m1 * c1x - m2 * c2x;
          const T vy = uhy - m1 * c1y - m2 * c2y;
          const bool outb = on && mv && (vx < lox || vx > hix || vy < loy || vy > hiy);
          ok2 = ok2 && !group_any<G>(outb, lane);
          const T wx = (on && mv) ? vx : ux, wy = (on && mv) ? vy : uy;  // unmoved: u0
          float2 *xw = xv + G;  // past the guess's exchange
          xw[i] = make_float2(wx, wy);
          wave_lds_fence();
          bool bad2 = !ok2;
          static_for<1, KH + 1>([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            const float2 v = xw[(i + K) & (G - 1)];
            const int id = cpid[K - 1];
            const T sn = (T(2) * (cdx[K - 1] * (v.x - wx) + cdy[K - 1] * (v.y - wy)) - cb[K - 1]) *
                         crn[K - 1];
            bad2 = bad2 | ((id >= 0) & (id != bid) & (id != rid) & (sn > C.tol_add));
          });
          second = try2 && !group_any<G>(bad2, lane);
          if (second) {
            nux = wx;
            nuy = wy;
            lam1 = m1;
            lam2 = m2;
            sqa = ra;
            sqb = rb;
            accept = true;
            seeded = false;
          }
          // p's multiplier came out negative: r alone, projected with every
          // coordinate free, p then checked like every other row
          const bool try3 = try2 && !second && m1 < T(0);
          if (__ballot(try3) != 0) {
            const T lr = qdiv(h2, g22);
            const bool mv3 = i == ra || i == rb;
            const T v3x = uhx - lr * c2x, v3y = uhy - lr * c2y;
            const bool outb3 = on && mv3 && (v3x < lox || v3x > hix || v3y < loy || v3y > hiy);
            const bool ok3 = try3 && lr > T(0) && !group_any<G>(outb3, lane);
            const T w3x = (on && mv3) ? v3x : ux, w3y = (on && mv3) ? v3y : uy;
            float2 *x3 = xw + G;  // past the second guess's exchange
            x3[i] = make_float2(w3x, w3y);
            wave_lds_fence();
            bool bad3 = !ok3;
            static_for<1, KH + 1>([&](auto kc) {
              constexpr int K = decltype(kc)::value;
              const float2 v = x3[(i + K) & (G - 1)];
              const int id = cpid[K - 1];
              const T sn = (T(2) * (cdx[K - 1] * (v.x - w3x) + cdy[K - 1] * (v.y - w3y)) - cb[K - 1]) *
                           crn[K - 1];
              bad3 = bad3 | ((id >= 0) & (id != rid) & (sn > C.tol_add));
            });
            lone = try3 && !group_any<G>(bad3, lane);
            if (lone) {
              nux = w3x;
              nuy = w3y;
              lam1 = lr;
              spa = ra;
              spb = rb;
              accept = true;
              seeded = false;
            }
          }
        }
      }
      // accepted: the guess is the solution; one rejected row with ok: start
      // the loop from u(l) with p active; otherwise from u0 (unchanged)
      ux = (accept || seeded) ? nux : ux;
      uy = (accept || seeded) ? nuy : uy;
      fq = accept ? ((two || second) ? 2 : 1) : fq;
      info.stage = (two || second) ? ((shared || second) ? kStShared : kStTwoRows) : kStOneRow;
      seed = seeded;
      fpa = spa; fpb = spb; fl1 = lam1; fdx = bdx; fdy = bdy;
      fqa = sqa; fqb = sqb; fl2 = lam2;
      run_gi = !accept;
      info.iters = (two || second) ? 2 : 1;
    } else {
      if constexpr (kGuess) {
        // four or more rows violated at u0, where the loop starts: p is the
        // most violated one
        fpa = bid >> 4; fpb = bid & 15; fdx = bdx; fdy = bdy;
      }
    }
  }

  if (__builtin_expect(run_gi, 0)) {
    const QPLoopOut<T> r = qp_active_set<T, G>(sh, lane, i, N, on, px, py, uhx, uhy, lox, hix,
                                               loy, hiy, seed, fpa, fpb, fl1, fdx, fdy, C.rs2,
                                               C.gamma, C.vmax4, C.tol_add, C.eps_z, C.eps_r,
                                               qp_cap, act_out != nullptr);
    ux = r.ux;
    uy = r.uy;
    info.status = r.status;
    info.iters = r.iters;
    info.q = r.q;
    info.in_lds = r.in_lds;
    info.stage = r.in_lds ? kStGeneral : kStActiveSet;
    if (act_out) {
      act_out->q = r.q;
      act_out->rows_in_lds = 1;
    }
    return info;
  }
  if (dead) {
    info.status = 1;
    info.stage = kStBox;
    fq = 0;
    if (on) {
      ux = lox <= hix ? tmin(tmax(uhx, lox), hix) : T(0.5) * (lox + hix);
      uy = loy <= hiy ? tmin(tmax(uhy, loy), hiy) : T(0.5) * (loy + hiy);
    }
  }
  info.q = fq;
  if (act_out) {
    act_out->q = fq;
    act_out->rows_in_lds = 0;
    act_out->sa[0] = fq > 0 ? fpa : -1;
    act_out->sb[0] = fq > 0 ? fpb : -1;
    act_out->slam[0] = fq > 0 ? fl1 : T(0);
    act_out->sa[1] = fq > 1 ? fqa : -1;
    act_out->sb[1] = fq > 1 ? fqb : -1;
    act_out->slam[1] = fq > 1 ? fl2 : T(0);
    act_out->sa[2] = fq > 2 ? fra : -1;
    act_out->sb[2] = fq > 2 ? frb : -1;
    act_out->slam[2] = fq > 2 ? fl3 : T(0);
#pragma unroll
    for (int a = 3; a < kQR; ++a) {
      act_out->sa[a] = -1;
      act_out->sb[a] = -1;
      act_out->slam[a] = T(0);
    }
  }
  return info;
}

}  // namespace rs
