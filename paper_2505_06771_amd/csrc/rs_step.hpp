// rs_step.hpp -- one environment step for the lane group that owns the
// environment (lane i = robot i). Definitions follow robostep.h (JaxRobotarium
// Sec. 4.1 and the Navigation scenario of the appendix).
#pragma once

#include "rs_qp.hpp"

namespace rs {

// Discrete single-integrator moves: 0 stay, 1 +x, 2 -x, 3 +y, 4 -y.
__device__ __forceinline__ void move_dir(int a, int &dx, int &dy) {
  dx = (a == 1) - (a == 2);
  dy = (a == 3) - (a == 4);
}

__device__ __forceinline__ int drawn_action(uint32_t k0, uint32_t k1, uint32_t env_id,
                                            uint32_t t, int i) {
  const uint4 o = stream_block(k0, k1, env_id, t, kAction, (uint32_t)(i >> 2), 0u);
  return (int)(((uint64_t)word(o, i & 3) * 5ull) >> 32);
}

// Magnitude limit of the nominal command, decided on squared norms (an
// axis-aligned command of exactly v_max squares to v_max^2 and is left alone).
template <typename T, typename CS>
__device__ __forceinline__ void preclip(const CS &C, T &ux, T &uy) {
  const T n2 = ux * ux + uy * uy;
  if (n2 > C.vmax * C.vmax) {
    const T sc = C.vmax * rsqrt_t(n2);
    ux *= sc;
    uy *= sc;
  }
}

// Single-integrator command at the projection point -> unicycle (v, w), then
// GRITSBot wheel-speed saturation.
template <typename T, typename CS>
__device__ __forceinline__ void si_to_uni(const CS &C, T c, T s, T ux, T uy, T &v, T &w) {
  v = c * ux + s * uy;
  w = (c * uy - s * ux) * C.inv_l;
  if (C.R > T(0)) {
    T phr = (v + C.halfL * w) * C.inv_R;
    T phl = (v - C.halfL * w) * C.inv_R;
    phr = tclamp(phr, -C.wheel_lim, C.wheel_lim);
    phl = tclamp(phl, -C.wheel_lim, C.wheel_lim);
    v = T(0.5) * C.R * (phr + phl);
    w = C.R_over_L * (phr - phl);
  }
}

// Explicit Euler with the pre-step heading; heading wrapped to [-pi, pi]
// (|dt w| < pi, so one correction suffices).
template <typename T, typename CS>
__device__ __forceinline__ void integrate(const CS &C, T c, T s, T v, T w, T &x, T &y,
                                          T &th) {
  x += C.dt * v * c;
  y += C.dt * v * s;
  T t = th + C.dt * w;
  const T pi = pi_v<T>();
  if (t > pi) t -= T(2) * pi;
  else if (t < -pi) t += T(2) * pi;
  th = t;
}

// Lattice placement of N points with the minimum separation: every lane of
// the group draws the same candidate for robot r; lanes j < r test it against
// their own point; the first candidate nobody rejects is kept by lane r.
template <typename T, int G>
__device__ void place_points(ConstRef<T> K, uint32_t env_id, uint32_t episode, uint32_t purpose,
                             int i, int N, int lane, int64_t &X, int64_t &Y) {
  const auto *P = K.get();
  const int64_t xlo = P->xlo, ylo = P->ylo, wx = P->wx, wy = P->wy, sep2 = P->sep2;
  const int64_t xhi = P->xhi, yhi = P->yhi;
  const uint32_t key0 = P->key0, key1 = P->key1;
  X = 0;
  Y = 0;
  for (int r = 0; r < N; ++r) {
    bool placed = false;
    for (uint32_t att = 0; att < 64u && !placed; ++att) {
      const uint4 o = stream_block(key0, key1, env_id, episode, purpose, (uint32_t)r, att);
      const int64_t cx = xlo + (int64_t)(((uint64_t)o.x * (uint64_t)wx) >> 32);
      const int64_t cy = ylo + (int64_t)(((uint64_t)o.y * (uint64_t)wy) >> 32);
      const int64_t ddx = cx - X, ddy = cy - Y;
      const bool clash = (i < r) && (ddx * ddx + ddy * ddy < sep2);
      if (!group_any<G>(clash, lane)) {
        placed = true;
        if (i == r) { X = cx; Y = cy; }
      }
    }
    for (int64_t cy = ylo; cy <= yhi && !placed; cy += 500) {
      for (int64_t cx = xlo; cx <= xhi && !placed; cx += 500) {
        const int64_t ddx = cx - X, ddy = cy - Y;
        const bool clash = (i < r) && (ddx * ddx + ddy * ddy < sep2);
        if (!group_any<G>(clash, lane)) {
          placed = true;
          if (i == r) { X = cx; Y = cy; }
        }
      }
    }
    if (!placed && i == r) { X = xlo; Y = ylo; }
  }
}

// Reset sampler for the group's environment (episode `episode`). Its
// constants (lattice, separation, stream key) are loaded from the kernel
// arguments where they are used: it is the cold path of a step. With PP
// (Predator-Prey) every goal slot gets the prey: robot 0's goal point.
template <typename T, int G, bool PP = false>
__device__ void reset_env(ConstRef<T> K, uint32_t env_id, uint32_t episode, int i, int N,
                          int lane, T &x, T &y, T &th, T &gx, T &gy) {
  int64_t X, Y, GX, GY;
  place_points<T, G>(K, env_id, episode, kPose, i, N, lane, X, Y);
  place_points<T, G>(K, env_id, episode, kGoal, i, N, lane, GX, GY);
  const auto *P = K.get();
  const double grid = P->grid;
  const uint4 hb = stream_block(P->key0, P->key1, env_id, episode, kHeading, (uint32_t)(i >> 2), 0u);
  const double u = (double)(word(hb, i & 3) >> 8) * 5.9604644775390625e-8;
  th = (T)(-kPiD + 2.0 * kPiD * u);
  x = (T)((double)X * grid);
  y = (T)((double)Y * grid);
  gx = (T)((double)GX * grid);
  gy = (T)((double)GY * grid);
  if constexpr (PP) {
    const int base = lane & ~(G - 1);
    gx = __shfl(gx, base, 64);
    gy = __shfl(gy, base, 64);
  }
}

// Predator-Prey prey move (appendix, Predator Prey: the prey keeps as far as
// it can from the closest tagger). Candidates: stay, then a step of
// prey_step in direction 2 pi k / 16 for k = 0..15, clamped to the walls
// pulled in by r_s/2; the prey takes the candidate with the largest squared
// distance to the closest robot centre (x, y of the calling lanes, before
// they move), the first on ties. (qx, qy) is group-uniform in and out.
// Every lane forms all 17 candidates (group-uniform) and its robot's distance
// to each. With G >= 4 the distances go through the group's QP scratch in LDS
// (unused at this point of the step): lane i then takes the minimum over the
// robots for candidates i, i + G, ..., and one arg-max butterfly picks the
// winner; with G = 2 a group minimum per candidate is as cheap.
template <typename T, int G, typename CS>
__device__ __forceinline__ void prey_move(const CS &C, QPScratch<T, G> *sh, int i,
                                          bool on, T x, T y, T &qx, T &qy) {
  constexpr int NCAND = 17;
  constexpr double kC = 0.92387953251128674, kH = 0.70710678118654752, kS = 0.38268343236508977;
  constexpr double dir_c[16] = {1, kC, kH, kS, 0, -kS, -kH, -kC, -1, -kC, -kH, -kS, 0, kS, kH, kC};
  constexpr double dir_s[16] = {0, kS, kH, kC, 1, kC, kH, kS, 0, -kS, -kH, -kC, -1, -kC, -kH, -kS};
  const T far = T(1e30);
  const T st = C.prey_step;
  // candidate k's position (the same arithmetic wherever it is formed)
  auto cand = [&](auto kc, T &cx, T &cy) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k == 0) {
      cx = qx;
      cy = qy;
    } else {
      cx = tclamp(qx + st * T(dir_c[k - 1]), C.xwl, C.xwh);
      cy = tclamp(qy + st * T(dir_s[k - 1]), C.ywl, C.ywh);
    }
  };
  if constexpr (G == 2 || sizeof(QPScratch<T, G>) < sizeof(T) * NCAND * G) {
    T best = T(-1), bx = qx, by = qy;
    static_for<0, NCAND>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      T cx, cy;
      cand(kc, cx, cy);
      const T ex = cx - x, ey = cy - y;
      const T sc = gmin<G>(on ? ex * ex + ey * ey : far);
      const bool bt = sc > best;
      best = bt ? sc : best;
      bx = bt ? cx : bx;
      by = bt ? cy : by;
    });
    qx = bx;
    qy = by;
  } else {
    T *d = reinterpret_cast<T *>(sh);  // [candidate][robot]
    static_for<0, NCAND>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      T cx, cy;
      cand(kc, cx, cy);
      const T ex = cx - x, ey = cy - y;
      d[k * G + i] = on ? ex * ex + ey * ey : far;
    });
    wave_lds_fence();
    T best = T(-1);
    int bk = NCAND;
    for (int k = i; k < NCAND; k += G) {  // ascending: the first maximum stays
      T m = d[k * G];
#pragma unroll
      for (int j = 1; j < G; ++j) m = tmin(m, d[k * G + j]);
      const bool bt = m > best;
      best = bt ? m : best;
      bk = bt ? k : bk;
    }
    wave_lds_fence();  // the scratch is the QP's again
    // arg-max over the group, ties to the lower candidate index
    auto merge = [&](auto c) {
      constexpr int CT = decltype(c)::value;
      const T w = dpp<CT>(best);
      const int wk = dpp<CT>(bk);
      const bool bt = (w > best) | ((w == best) & (wk < bk));
      best = bt ? w : best;
      bk = bt ? wk : bk;
    };
    merge(std::integral_constant<int, 0xB1>{});
    if constexpr (G >= 4) merge(std::integral_constant<int, 0x4E>{});
    if constexpr (G >= 8) merge(std::integral_constant<int, 0x141>{});
    if constexpr (G >= 16) merge(std::integral_constant<int, 0x140>{});
    // the winner's direction, then its position formed as above
    T dc = T(0), ds = T(0);
    static_for<1, NCAND>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      dc = bk == k ? T(dir_c[k - 1]) : dc;
      ds = bk == k ? T(dir_s[k - 1]) : ds;
    });
    if (bk > 0) {
      qx = tclamp(qx + st * dc, C.xwl, C.xwh);
      qy = tclamp(qy + st * ds, C.ywl, C.ywh);
    }
  }
}

// Observation of robot i: x, y, cos th, sin th, (x_j - x_i, y_j - y_i) for
// j != i ascending, g_i - (x_i, y_i). Written to o[0 .. 2N+3]. Neighbour
// positions arrive by DPP rotations inside the group.
template <typename T, int G>
__device__ __forceinline__ void write_obs(T *o, int lane, int i, int N, bool on, T x, T y, T c,
                                          T s, T gx, T gy) {
  if (on) {
    o[0] = x;
    o[1] = y;
    o[2] = c;
    o[3] = s;
  }
  static_for<1, G>([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const T xj = grot<G, K>(x, lane), yj = grot<G, K>(y, lane);
    const int j = (i + K) & (G - 1);
    if (on && j < N) {
      const int m = 4 + 2 * (j < i ? j : j - 1);
      o[m] = xj - x;
      o[m + 1] = yj - y;
    }
  });
  if (on) {
    o[2 * N + 2] = gx - x;
    o[2 * N + 3] = gy - y;
  }
}

// Largest normalised violation of (ux, uy) against the rows (owner scan) and
// bounds; group-uniform result.
template <typename T, int G, typename CS>
__device__ T max_violation(const CS &C, int lane, int i, int N, bool on, T px, T py,
                           T ux, T uy, T lox, T hix, T loy, T hiy) {
  const int base = lane & ~(G - 1);
  T worst = T(0);
  if (on) worst = tmax(tmax(ux - hix, lox - ux), tmax(uy - hiy, loy - uy));
  for (int k = 1; k <= (N >> 1); ++k) {
    const int j = on ? (i + k >= N ? i + k - N : i + k) : 0;
    const T pxj = __shfl(px, base + j, 64), pyj = __shfl(py, base + j, 64);
    const T uxj = __shfl(ux, base + j, 64), uyj = __shfl(uy, base + j, 64);
    if (on && !(2 * k == N && i >= k)) {
      const bool ia = i < j;
      const T dx = ia ? px - pxj : pxj - px, dy = ia ? py - pyj : pyj - py;
      const T d2 = dx * dx + dy * dy, h = d2 - C.rs2;
      const T s = T(2) * (dx * (ia ? uxj - ux : ux - uxj) + dy * (ia ? uyj - uy : uy - uyj)) -
                  C.gamma * (h * h * h);
      worst = tmax(worst, d2 > T(0) ? s * (T(0.35355339059327373) * rsqrt_t(d2)) : s);
    }
  }
  return tmax(group_max<G>(worst), T(0));
}

// Result of one group step.
template <typename T> struct StepOut {
  T reward;
  bool done;
  QPInfo qp;
  T maxviol;
};

// One env step for the group (all lanes call together). State (x, y, th,
// gx, gy, c = cos th, s = sin th) is updated in place; `action` is the lane's
// action (ignored by the go-to-goal controller); `t` is the stream time of
// the step (keys the action noise). `step`/`episode` are group-uniform and
// updated. Observation of the post-step state is left to the caller (c, s
// are refreshed).
template <typename T, int G, bool PP = false>
__device__ StepOut<T> env_step_group(ConstRef<T> K, int qp_cap, QPScratch<T, G> *sh, int lane,
                                     int i, int N, bool on, uint32_t env_id, uint32_t t, int action,
                                     T &x, T &y, T &th, T &c, T &s, T &gx, T &gy, int &step,
                                     int &episode, bool want_viol, PhaseClock *pc = nullptr) {
  StepOut<T> out;
  // Constants are read from the kernel arguments phase by phase (see
  // ConstRef), so that they do not hold scalar registers across the step.
  // projection point and nominal command
  const auto &C = *K.get();
  const T px = x + C.l * c, py = y + C.l * s;
  T unx, uny;
  if (C.controller == 1) {
    unx = C.kp * (gx - px);
    uny = C.kp * (gy - py);
  } else {
    int ddx, ddy;
    move_dir(action, ddx, ddy);
    if (C.controller == 2) {
      // Waypoint wstep ahead of the centre along the move (Sec. 6.1, waypoint
      // actions), steered to by the unicycle position controller
      // v = kv rho cos(alpha), w = kw sin(alpha). The waypoint lies on a unit
      // axis d, so rho cos(alpha) = wstep d.(c, s) and sin(alpha) =
      // (c, s) x d; the stay action (d = 0) gives v = w = 0. The unicycle
      // command moves the projection point at v (c, s) + l w (-s, c).
      const T v = C.kv * C.wstep * (c * T(ddx) + s * T(ddy));
      const T w = C.kw * (c * T(ddy) - s * T(ddx));
      unx = v * c - C.l * w * s;
      uny = v * s + C.l * w * c;
    } else if (C.controller == 3) {
      // Pose waypoint wstep ahead along the unit axis d, heading along d,
      // steered to by the pose law v = k_rho rho cos(alpha), w = k_alpha
      // alpha + k_rho (sin(alpha) cos(alpha) / alpha)(alpha + k_beta beta).
      // The waypoint lies on the ray of its own heading, so beta = 0 and the
      // turn rate is k_alpha alpha + k_rho sin(alpha) cos(alpha), with
      // cos(alpha) = (c, s).d, sin(alpha) = (c, s) x d; staying (d = 0)
      // gives v = w = 0 (alpha = 0 set explicitly: the products with d = 0
      // can be signed zeros, and atan2(+0, -0) = pi).
      const T ca = c * T(ddx) + s * T(ddy), sa = c * T(ddy) - s * T(ddx);
      const T alpha = (ddx != 0 || ddy != 0) ? atan2_t(sa, ca) : T(0);
      const T v = C.krho * C.wstep * ca;
      const T w = C.kalpha * alpha + C.krho * sa * ca;
      unx = v * c - C.l * w * s;
      uny = v * s + C.l * w * c;
    } else {
      unx = C.aspeed * T(ddx);
      uny = C.aspeed * T(ddy);
    }
  }
  if (C.noise > T(0)) {
    // action noise (Sec. 7, domain randomisation): uniform in [-sigma, sigma)
    // per coordinate, words 0 and 1 of block (env_id, t, kNoise, i)
    const uint4 o = stream_block(C.key0, C.key1, env_id, t, kNoise, (uint32_t)i, 0u);
    unx += C.noise * (T(2) * unit24_t<T>(o.x) - T(1));
    uny += C.noise * (T(2) * unit24_t<T>(o.y) - T(1));
  }
  preclip(*K.get(), unx, uny);
  // Predator-Prey: the prey (held in every goal slot) moves on the pre-step
  // centres, at the same time as the robots
  T qx = gx, qy = gy;
  if constexpr (PP) {
    const int base = lane & ~(G - 1);
    qx = __shfl(gx, base, 64);
    qy = __shfl(gy, base, 64);
    prey_move<T, G>(*K.get(), sh, i, on, x, y, qx, qy);
  }
  T lox, hix, loy, hiy;
  wall_bounds(*K.get(), px, py, lox, hix, loy, hiy);
  T ux, uy;
  if (pc) pc->mark(kPhPre);
  out.qp = qp_solve<T, G>(sh, K, qp_cap, lane, i, N, on, px, py, unx, uny, lox, hix, loy, hiy, ux,
                          uy);
  if (pc) {
    pc->mark(kPhQp);
#ifdef RS_PHASE_TIMERS
    pc->count(kPhLoop, __ballot(out.qp.stage >= kStActiveSet) != 0);
#endif
  }
  out.maxviol = want_viol ? max_violation<T, G>(*K.get(), lane, i, N, on, px, py, ux, uy, lox, hix,
                                                loy, hiy)
                          : T(0);
  T v, w;
  si_to_uni(*K.get(), c, s, ux, uy, v, w);
  if (on) integrate(*K.get(), c, s, v, w, x, y, th);
  // reward and termination
  step += 1;
  const auto &Cd = *K.get();
  if constexpr (PP) {
    // tag: some centre closer than the tag radius to the moved prey
    gx = qx;
    gy = qy;
    T dist = T(0);
    if (on) {
      const T ex = x - qx, ey = y - qy;
      dist = sqrt_t(ex * ex + ey * ey);
    }
    const bool tag = group_any<G>(on && dist < Cd.tag_r, lane);
    out.reward = tag ? Cd.tag_reward : T(0);
    out.done = Cd.max_steps > 0 && step >= Cd.max_steps;
  } else {
    T dist = T(0);
    if (on) {
      const T ex = x - gx, ey = y - gy;
      dist = sqrt_t(ex * ex + ey * ey);
    }
    out.reward = -gsum<G>(dist);
    const bool near_all = group_all<G>(!on || dist < Cd.goal_r, lane);
    out.done = (Cd.goal_r > T(0) && near_all) || (Cd.max_steps > 0 && step >= Cd.max_steps);
  }
  if (out.done) {
    episode += 1;
    step = 0;
    T nx, ny, nth, ngx, ngy;
    reset_env<T, G, PP>(K, env_id, (uint32_t)episode, i, N, lane, nx, ny, nth, ngx, ngy);
    if (on) { x = nx; y = ny; th = nth; gx = ngx; gy = ngy; }
  }
  sincos_t(th, &s, &c);
  if (pc) pc->mark(kPhPost);
  return out;
}

}  // namespace rs
