/*
 * robostep_oracle.c -- plain FP64 CPU oracle of the batched Robotarium
 * environment step. TEST INFRASTRUCTURE ONLY (see robostep_oracle.h).
 *
 * Paper passages followed (JaxRobotarium, arXiv 2505.06771):
 *   Sec. 4.1 "Design"      unicycle GRITSBot model, single-integrator and
 *                          unicycle controllers, barrier-certificate QP.
 *   Appendix, Navigation   observation = own position + vector to goal,
 *                          reward = -1 x distance of robots to their goals.
 *   Appendix, Predator Prey  taggers, a prey that flees the closest tagger,
 *                          reward 10 per step with a tag.
 *   Sec. 9 "Limitations"   the simulator's QP solver differs from the testbed's;
 *                          the ground truth here is the exact minimiser.
 * The paper states none of the formulas; the readings used are stated on each
 * function below.
 */
#include "robostep_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_MAX_N 16
#define ORC_MAX_VARS (2 * ORC_MAX_N)
#define ORC_MAX_PAIRS (ORC_MAX_N * (ORC_MAX_N - 1) / 2)
#define ORC_MAX_ROWS (ORC_MAX_PAIRS + 2 * ORC_MAX_VARS)

/* Stream purposes (word 2 of the counter carries purpose << 24 | index). */
enum { PURPOSE_ACTION = 0, PURPOSE_POLICY = 1, PURPOSE_POSE = 2, PURPOSE_GOAL = 3,
       PURPOSE_HEADING = 4, PURPOSE_WEIGHTS = 5, PURPOSE_NOISE = 6 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as published by Salmon et al. (SC'11): ten rounds of two   */
/* 32x32->64 multiplies with a Weyl-sequence key schedule.                   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t prod0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void stream_block(const orc_params *p, uint32_t w0, uint32_t w1, uint32_t purpose,
                         uint32_t index, uint32_t w3, uint32_t out[4]) {
  uint32_t ctr[4] = {w0, w1, (purpose << 24) | (index & 0xFFFFFFu), w3};
  uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* 24-bit uniform in [0,1): exact in FP32 and FP64. */
static double unit_uniform(uint32_t r) { return ldexp((double)(r >> 8), -24); }

/* ------------------------------------------------------------------------ */
/* bfloat16 round-to-nearest-even of an FP64 value.                          */
/* ------------------------------------------------------------------------ */
double orc_bf16_round(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  frexp(x, &e);                 /* |x| = m 2^e, m in [0.5, 1) */
  int lsb_exp = e - 8;          /* 8 significant bits */
  if (e - 1 < -126) lsb_exp = -133; /* subnormal range of the float exponent */
  double q = nearbyint(ldexp(x, -lsb_exp)); /* default rounding: ties to even */
  double r = ldexp(q, lsb_exp);
  if (fabs(r) > 3.38953138925153547590470800371487866880e38) r = copysign(INFINITY, x);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Reset sampler (start poses uniform with a minimum separation, goals       */
/* uniform in the arena, headings uniform). Positions live on an integer     */
/* lattice of pitch `grid` inside the arena shrunk by `reset_margin`, so the */
/* separation test is exact integer arithmetic: robot i tries up to 64 draws */
/* and keeps the first at squared lattice distance >= S^2 from robots < i;   */
/* if all fail, it scans a coarse lattice (every 500 cells) row by row.      */
/* ------------------------------------------------------------------------ */
static int64_t scale_draw(uint32_t r, int64_t width) {
  return (int64_t)(((uint64_t)r * (uint64_t)width) >> 32);
}

static int separated(const int64_t *X, const int64_t *Y, int32_t count, int64_t cx, int64_t cy,
                     int64_t s2) {
  for (int32_t j = 0; j < count; ++j) {
    int64_t dx = cx - X[j], dy = cy - Y[j];
    if (dx * dx + dy * dy < s2) return 0;
  }
  return 1;
}

static void place_points(const orc_params *p, uint64_t env_id, int32_t episode, int32_t n,
                         uint32_t purpose, int64_t *X, int64_t *Y) {
  int64_t xlo = llround((p->x_min + p->reset_margin) / p->grid);
  int64_t xhi = llround((p->x_max - p->reset_margin) / p->grid);
  int64_t ylo = llround((p->y_min + p->reset_margin) / p->grid);
  int64_t yhi = llround((p->y_max - p->reset_margin) / p->grid);
  int64_t wx = xhi - xlo + 1, wy = yhi - ylo + 1;
  int64_t s = llround(p->min_sep / p->grid);
  int64_t s2 = s * s;
  for (int32_t i = 0; i < n; ++i) {
    int placed = 0;
    for (uint32_t attempt = 0; attempt < 64 && !placed; ++attempt) {
      uint32_t o[4];
      stream_block(p, (uint32_t)env_id, (uint32_t)episode, purpose, (uint32_t)i, attempt, o);
      int64_t cx = xlo + scale_draw(o[0], wx);
      int64_t cy = ylo + scale_draw(o[1], wy);
      if (separated(X, Y, i, cx, cy, s2)) {
        X[i] = cx; Y[i] = cy; placed = 1;
      }
    }
    for (int64_t cy = ylo; cy <= yhi && !placed; cy += 500) {
      for (int64_t cx = xlo; cx <= xhi && !placed; cx += 500) {
        if (separated(X, Y, i, cx, cy, s2)) {
          X[i] = cx; Y[i] = cy; placed = 1;
        }
      }
    }
    if (!placed) { X[i] = xlo; Y[i] = ylo; }
  }
}

void orc_reset_lattice(const orc_params *p, uint64_t env_id, int32_t episode, int32_t n,
                       int64_t *X, int64_t *Y, int64_t *GX, int64_t *GY, uint32_t *heading_bits) {
  place_points(p, env_id, episode, n, PURPOSE_POSE, X, Y);
  place_points(p, env_id, episode, n, PURPOSE_GOAL, GX, GY);
  for (int32_t i = 0; i < n; ++i) {
    uint32_t o[4];
    stream_block(p, (uint32_t)env_id, (uint32_t)episode, PURPOSE_HEADING, (uint32_t)(i >> 2), 0, o);
    heading_bits[i] = o[i & 3];
  }
}

void orc_reset_env(const orc_params *p, uint64_t env_id, int32_t episode, int32_t n, double *x,
                   double *y, double *th, double *gx, double *gy) {
  int64_t X[ORC_MAX_N], Y[ORC_MAX_N], GX[ORC_MAX_N], GY[ORC_MAX_N];
  uint32_t hb[ORC_MAX_N];
  orc_reset_lattice(p, env_id, episode, n, X, Y, GX, GY, hb);
  for (int32_t i = 0; i < n; ++i) {
    /* Predator-Prey: the prey is the goal sampler's first point, shared by
       every robot's goal slot */
    int32_t g = p->scenario == 1 ? 0 : i;
    x[i] = (double)X[i] * p->grid;
    y[i] = (double)Y[i] * p->grid;
    gx[i] = (double)GX[g] * p->grid;
    gy[i] = (double)GY[g] * p->grid;
    th[i] = -M_PI + 2.0 * M_PI * unit_uniform(hb[i]);
  }
}

/* ------------------------------------------------------------------------ */
/* Actions: five discrete single-integrator moves, index 0 stay, 1 +x, 2 -x, */
/* 3 +y, 4 -y; drawn as floor(5 r / 2^32).                                   */
/* ------------------------------------------------------------------------ */
int32_t orc_random_action(const orc_params *p, uint64_t env_id, int64_t t_global, int32_t i) {
  uint32_t o[4];
  stream_block(p, (uint32_t)env_id, (uint32_t)t_global, PURPOSE_ACTION, (uint32_t)(i >> 2), 0, o);
  return (int32_t)(((uint64_t)o[i & 3] * 5u) >> 32);
}

static void move_direction(int32_t a, double *dx, double *dy) {
  *dx = 0.0; *dy = 0.0;
  if (a == 1) *dx = 1.0;
  else if (a == 2) *dx = -1.0;
  else if (a == 3) *dy = 1.0;
  else if (a == 4) *dy = -1.0;
}

/* ------------------------------------------------------------------------ */
/* Constraint set of the barrier certificate.                                */
/*   pair rows (i<j): with D = p_i - p_j and h = |D|^2 - r_s^2,              */
/*       -2 D.u_i + 2 D.u_j <= gamma h^3          (cubic class-K function)   */
/*   wall rows on each coordinate of the projection point, walls pulled in   */
/*   by r_s/2, gain c_b gamma, intersected with |u_k| <= v_max:              */
/*       u_x <= min(v_max,  c_b gamma (x_max - r_s/2 - p_x)^3)               */
/*       u_x >= max(-v_max, -c_b gamma (p_x - x_min - r_s/2)^3)  (same in y) */
/* ------------------------------------------------------------------------ */
static double cube(double v) { return v * v * v; }

void orc_bounds(const orc_params *p, int32_t n, const double *px, const double *py, double *lo_x,
                double *hi_x, double *lo_y, double *hi_y) {
  double kb = p->boundary_gain_factor * p->barrier_gain;
  double half = 0.5 * p->safety_radius;
  for (int32_t i = 0; i < n; ++i) {
    hi_x[i] = fmin(p->v_max, kb * cube(p->x_max - half - px[i]));
    lo_x[i] = fmax(-p->v_max, -kb * cube(px[i] - p->x_min - half));
    hi_y[i] = fmin(p->v_max, kb * cube(p->y_max - half - py[i]));
    lo_y[i] = fmax(-p->v_max, -kb * cube(py[i] - p->y_min - half));
  }
}

/* Dense constraint matrix: rows 0..P-1 pairs (i<j, lexicographic), then for
 * each variable v (u0x, u0y, u1x, ...) an upper row (+e_v <= hi) and a lower
 * row (-e_v <= -lo). */
static int32_t build_rows(const orc_params *p, int32_t n, const double *px, const double *py,
                          double *C, double *d) {
  int32_t nv = 2 * n, row = 0;
  double lo_x[ORC_MAX_N], hi_x[ORC_MAX_N], lo_y[ORC_MAX_N], hi_y[ORC_MAX_N];
  orc_bounds(p, n, px, py, lo_x, hi_x, lo_y, hi_y);
  double rs2 = p->safety_radius * p->safety_radius;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t j = i + 1; j < n; ++j) {
      double dx = px[i] - px[j], dy = py[i] - py[j];
      double h = dx * dx + dy * dy - rs2;
      double *c = C + (size_t)row * nv;
      memset(c, 0, sizeof(double) * nv);
      c[2 * i] = -2.0 * dx; c[2 * i + 1] = -2.0 * dy;
      c[2 * j] = 2.0 * dx;  c[2 * j + 1] = 2.0 * dy;
      d[row] = p->barrier_gain * cube(h);
      ++row;
    }
  }
  for (int32_t v = 0; v < nv; ++v) {
    int32_t i = v / 2;
    double hi = (v & 1) ? hi_y[i] : hi_x[i];
    double lo = (v & 1) ? lo_y[i] : lo_x[i];
    double *c = C + (size_t)row * nv;
    memset(c, 0, sizeof(double) * nv);
    c[v] = 1.0; d[row] = hi; ++row;
    c = C + (size_t)row * nv;
    memset(c, 0, sizeof(double) * nv);
    c[v] = -1.0; d[row] = -lo; ++row;
  }
  return row;
}

static double dot(const double *a, const double *b, int32_t len) {
  double s = 0.0;
  for (int32_t k = 0; k < len; ++k) s += a[k] * b[k];
  return s;
}

/* Cholesky solve of the SPD system G r = g (q x q, row-major). Returns 0 on a
 * non-positive pivot. */
static int chol_solve(int32_t q, const double *G, const double *g, double *r) {
  double L[ORC_MAX_VARS * ORC_MAX_VARS];
  for (int32_t i = 0; i < q; ++i) {
    for (int32_t j = 0; j <= i; ++j) {
      double s = G[i * q + j];
      for (int32_t k = 0; k < j; ++k) s -= L[i * q + k] * L[j * q + k];
      if (i == j) {
        if (!(s > 0.0)) return 0;
        L[i * q + i] = sqrt(s);
      } else {
        L[i * q + j] = s / L[j * q + j];
      }
    }
  }
  double w[ORC_MAX_VARS];
  for (int32_t i = 0; i < q; ++i) {
    double s = g[i];
    for (int32_t k = 0; k < i; ++k) s -= L[i * q + k] * w[k];
    w[i] = s / L[i * q + i];
  }
  for (int32_t i = q - 1; i >= 0; --i) {
    double s = w[i];
    for (int32_t k = i + 1; k < q; ++k) s -= L[k * q + i] * r[k];
    r[i] = s / L[i * q + i];
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Exact projection min 1/2 |u - uhat|^2 s.t. C u <= d, by the dual          */
/* active-set method of Goldfarb and Idnani (Math. Prog. 27, 1983) with the  */
/* identity Hessian: start at the unconstrained minimiser, repeatedly add    */
/* the most violated constraint, moving along its component orthogonal to    */
/* the active normals and dropping an active constraint whose multiplier     */
/* would turn negative. Dense algebra; everything recomputed each iteration. */
/* Returns 0 solved, 1 infeasible, 2 iteration cap or numerical failure.     */
/* mult[k] receives the multiplier of row k (0 when inactive).               */
/* ------------------------------------------------------------------------ */
static int32_t dual_active_set(int32_t nv, int32_t m, const double *C, const double *d,
                               const double *uhat, double *u, double *mult) {
  int32_t active[ORC_MAX_VARS + 1];
  double lam[ORC_MAX_VARS + 1];
  int32_t q = 0;
  char in_set[ORC_MAX_ROWS];
  double cnorm[ORC_MAX_ROWS];
  memset(in_set, 0, sizeof(in_set));
  for (int32_t k = 0; k < m; ++k) cnorm[k] = sqrt(dot(C + (size_t)k * nv, C + (size_t)k * nv, nv));
  memcpy(u, uhat, sizeof(double) * nv);
  memset(mult, 0, sizeof(double) * m);
  const double add_tol = 1e-13;

  for (int32_t outer = 0; outer < 4 * ORC_MAX_ROWS; ++outer) {
    int32_t pidx = -1;
    double best = add_tol;
    for (int32_t k = 0; k < m; ++k) {
      if (in_set[k]) continue;
      if (cnorm[k] == 0.0) {
        if (d[k] < -add_tol) return 1; /* 0 <= d violated for every u */
        continue;
      }
      double s = (dot(C + (size_t)k * nv, u, nv) - d[k]) / cnorm[k];
      if (s > best) { best = s; pidx = k; }
    }
    if (pidx < 0) {
      memset(mult, 0, sizeof(double) * m);
      for (int32_t a = 0; a < q; ++a) mult[active[a]] = lam[a];
      return 0;
    }
    const double *cp = C + (size_t)pidx * nv;
    double lam_p = 0.0;
    int added = 0;
    for (int32_t inner = 0; inner < 4 * ORC_MAX_ROWS && !added; ++inner) {
      double r[ORC_MAX_VARS + 1], z[ORC_MAX_VARS];
      if (q > 0) {
        double G[ORC_MAX_VARS * ORC_MAX_VARS], g[ORC_MAX_VARS];
        for (int32_t a = 0; a < q; ++a) {
          g[a] = dot(C + (size_t)active[a] * nv, cp, nv);
          for (int32_t b = 0; b < q; ++b)
            G[a * q + b] = dot(C + (size_t)active[a] * nv, C + (size_t)active[b] * nv, nv);
        }
        if (!chol_solve(q, G, g, r)) return 2;
      }
      for (int32_t k = 0; k < nv; ++k) {
        double s = cp[k];
        for (int32_t a = 0; a < q; ++a) s -= r[a] * C[(size_t)active[a] * nv + k];
        z[k] = s;
      }
      double zz = dot(z, z, nv);
      double t1 = INFINITY;
      int32_t drop = -1;
      for (int32_t a = 0; a < q; ++a) {
        if (r[a] > 1e-14) {
          double ratio = lam[a] / r[a];
          if (ratio < t1) { t1 = ratio; drop = a; }
        }
      }
      double sp = dot(cp, u, nv) - d[pidx];
      double t2 = (zz > 1e-22 * cnorm[pidx] * cnorm[pidx]) ? sp / zz : INFINITY;
      if (isinf(t1) && isinf(t2)) return 1;
      if (isinf(t2)) {
        /* dependent on the active set: move the multipliers only, drop one */
        for (int32_t a = 0; a < q; ++a) lam[a] -= t1 * r[a];
        lam_p += t1;
      } else {
        double t = t1 < t2 ? t1 : t2;
        for (int32_t k = 0; k < nv; ++k) u[k] -= t * z[k];
        for (int32_t a = 0; a < q; ++a) lam[a] -= t * r[a];
        lam_p += t;
        if (t2 <= t1) {
          if (q >= ORC_MAX_VARS + 1) return 2;
          active[q] = pidx; lam[q] = lam_p; ++q;
          in_set[pidx] = 1;
          added = 1;
          continue;
        }
      }
      /* partial step: remove the blocking constraint */
      in_set[active[drop]] = 0;
      for (int32_t a = drop; a + 1 < q; ++a) { active[a] = active[a + 1]; lam[a] = lam[a + 1]; }
      --q;
    }
    if (!added) return 2;
  }
  return 2;
}

/* KKT residuals of (u, mult) for min 1/2|u-uhat|^2 s.t. C u <= d. */
static void kkt_residuals(int32_t nv, int32_t m, const double *C, const double *d,
                          const double *uhat, const double *u, const double *mult, double *out) {
  double stat = 0.0, prim = 0.0, dual = 0.0, comp = 0.0;
  for (int32_t k = 0; k < nv; ++k) {
    double s = u[k] - uhat[k];
    for (int32_t r = 0; r < m; ++r) s += mult[r] * C[(size_t)r * nv + k];
    stat = fmax(stat, fabs(s));
  }
  for (int32_t r = 0; r < m; ++r) {
    double cn = sqrt(dot(C + (size_t)r * nv, C + (size_t)r * nv, nv));
    double slack = dot(C + (size_t)r * nv, u, nv) - d[r];
    double sn = cn > 0.0 ? slack / cn : slack;
    prim = fmax(prim, sn);
    dual = fmax(dual, -mult[r]);
    if (mult[r] > 1e-12) comp = fmax(comp, fabs(sn));
  }
  out[0] = stat; out[1] = prim; out[2] = dual; out[3] = comp;
}

double orc_max_violation(const orc_params *p, int32_t n, const double *px, const double *py,
                         const double *ux, const double *uy) {
  int32_t nv = 2 * n;
  double *C = (double *)malloc(sizeof(double) * ORC_MAX_ROWS * ORC_MAX_VARS);
  double d[ORC_MAX_ROWS], u[ORC_MAX_VARS];
  int32_t m = build_rows(p, n, px, py, C, d);
  for (int32_t i = 0; i < n; ++i) { u[2 * i] = ux[i]; u[2 * i + 1] = uy[i]; }
  double worst = 0.0;
  for (int32_t r = 0; r < m; ++r) {
    double cn = sqrt(dot(C + (size_t)r * nv, C + (size_t)r * nv, nv));
    double slack = dot(C + (size_t)r * nv, u, nv) - d[r];
    double sn = cn > 0.0 ? slack / cn : slack;
    if (sn > worst) worst = sn;
  }
  free(C);
  return worst;
}

int32_t orc_barrier_certificate(const orc_params *p, int32_t n, const double *px,
                                const double *py, const double *ux_nom, const double *uy_nom,
                                double *ux, double *uy, double *lambda, double *kkt,
                                double *max_violation) {
  int32_t nv = 2 * n, npairs = n * (n - 1) / 2;
  double *C = (double *)malloc(sizeof(double) * ORC_MAX_ROWS * ORC_MAX_VARS);
  double d[ORC_MAX_ROWS], uhat[ORC_MAX_VARS], u[ORC_MAX_VARS], mult[ORC_MAX_ROWS];
  /* magnitude pre-clip of the nominal command */
  for (int32_t i = 0; i < n; ++i) {
    double vx = ux_nom[i], vy = uy_nom[i];
    double nrm = sqrt(vx * vx + vy * vy);
    if (nrm > p->v_max) { vx *= p->v_max / nrm; vy *= p->v_max / nrm; }
    uhat[2 * i] = vx; uhat[2 * i + 1] = vy;
  }
  int32_t m = build_rows(p, n, px, py, C, d);
  int32_t status = dual_active_set(nv, m, C, d, uhat, u, mult);
  if (status == 0) {
    double res[4];
    kkt_residuals(nv, m, C, d, uhat, u, mult, res);
    if (kkt) memcpy(kkt, res, sizeof(res));
    if (res[0] > 1e-9 || res[1] > 1e-9 || res[2] > 1e-12 || res[3] > 1e-9) status = 2;
  } else if (kkt) {
    kkt[0] = kkt[1] = kkt[2] = kkt[3] = NAN;
  }
  if (status == 1) {
    /* empty constraint set: closed-form fallback, the clip of the nominal
     * command to the bounds (midpoint where the bounds cross) */
    double lo_x[ORC_MAX_N], hi_x[ORC_MAX_N], lo_y[ORC_MAX_N], hi_y[ORC_MAX_N];
    orc_bounds(p, n, px, py, lo_x, hi_x, lo_y, hi_y);
    for (int32_t i = 0; i < n; ++i) {
      u[2 * i] = lo_x[i] <= hi_x[i] ? fmin(fmax(uhat[2 * i], lo_x[i]), hi_x[i])
                                    : 0.5 * (lo_x[i] + hi_x[i]);
      u[2 * i + 1] = lo_y[i] <= hi_y[i] ? fmin(fmax(uhat[2 * i + 1], lo_y[i]), hi_y[i])
                                        : 0.5 * (lo_y[i] + hi_y[i]);
    }
    memset(mult, 0, sizeof(double) * m);
  }
  for (int32_t i = 0; i < n; ++i) { ux[i] = u[2 * i]; uy[i] = u[2 * i + 1]; }
  /* multipliers of 1/2|.|^2 are half those of |.|^2 */
  if (lambda)
    for (int32_t k = 0; k < npairs; ++k) lambda[k] = 2.0 * mult[k];
  free(C);
  if (max_violation) *max_violation = orc_max_violation(p, n, px, py, ux, uy);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Projection-point map and GRITSBot wheel saturation.                       */
/*   v = cos(th) ux + sin(th) uy,  w = (-sin(th) ux + cos(th) uy) / l        */
/*   wheels phi_R,L = (v +- (L/2) w) / R clipped to +-v_max/R, mapped back.  */
/* ------------------------------------------------------------------------ */
void orc_si_to_uni(const orc_params *p, double theta, double ux, double uy, double *v, double *w) {
  double c = cos(theta), s = sin(theta);
  double vv = c * ux + s * uy;
  double ww = (-s * ux + c * uy) / p->proj_dist;
  if (p->wheel_radius > 0.0 && p->base_length > 0.0) {
    double R = p->wheel_radius, L = p->base_length;
    double lim = p->v_max / R;
    double phr = (vv + 0.5 * L * ww) / R;
    double phl = (vv - 0.5 * L * ww) / R;
    phr = fmin(fmax(phr, -lim), lim);
    phl = fmin(fmax(phl, -lim), lim);
    vv = 0.5 * R * (phr + phl);
    ww = R * (phr - phl) / L;
  }
  *v = vv;
  *w = ww;
}

/* ------------------------------------------------------------------------ */
/* Observation (per robot): x, y, cos th, sin th, then (x_j - x_i, y_j - y_i) */
/* for every other robot in ascending j, then the goal vector g_i - (x,y).   */
/* ------------------------------------------------------------------------ */
void orc_observe(int32_t n, const double *x, const double *y, const double *th, const double *gx,
                 const double *gy, double *obs) {
  int32_t dim = 2 * n + 4;
  for (int32_t i = 0; i < n; ++i) {
    double *o = obs + (size_t)i * dim;
    o[0] = x[i]; o[1] = y[i]; o[2] = cos(th[i]); o[3] = sin(th[i]);
    int32_t k = 4;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      o[k++] = x[j] - x[i];
      o[k++] = y[j] - y[i];
    }
    o[k++] = gx[i] - x[i];
    o[k++] = gy[i] - y[i];
  }
}

/* ------------------------------------------------------------------------ */
/* Waypoint actions (Sec. 6.1: a controller manager turns waypoint actions  */
/* into unicycle commands, then the barrier filters them; Appendix B: every  */
/* scenario trains on waypoints followed by a unicycle position controller). */
/* Readings: a move action a sets the waypoint waypoint_step ahead of the    */
/* robot's centre in direction dir(a), afresh at every step; the controller  */
/* is the classic turn-and-go law on the distance rho and the bearing alpha  */
/* of the waypoint relative to the heading,                                  */
/*   v = k_v rho cos(alpha),  w = k_w sin(alpha),                             */
/* idle (0, 0) at the waypoint; its unicycle command enters the barrier as   */
/* the velocity of the projection point.                                     */
/* ------------------------------------------------------------------------ */
void orc_unicycle_position(const orc_params *p, double x, double y, double theta, double wx,
                           double wy, double *v, double *w) {
  double ex = wx - x, ey = wy - y;
  double rho = sqrt(ex * ex + ey * ey);
  if (rho == 0.0) {
    *v = 0.0;
    *w = 0.0;
    return;
  }
  double alpha = atan2(ey, ex) - theta;
  *v = p->pos_gain * rho * cos(alpha);
  *w = p->ang_gain * sin(alpha);
}

/* ------------------------------------------------------------------------ */
/* Unicycle pose controller (Sec. 4.1: unicycle controllers drive robots to  */
/* desired positions or poses; Table 1 times a pose controller beside the    */
/* position one). The paper gives no law. Reading: the globally stabilising  */
/* law of Aicardi, Casalino, Bicchi and Balestrino (1995) on the polar error */
/* of the goal pose (wx, wy, wth): rho = distance to the goal position, phi  */
/* its bearing (wth when rho = 0), alpha = wrap(phi - theta) the bearing    */
/* relative to the heading, beta = wrap(phi - wth) the bearing relative to   */
/* the goal heading, wrap to (-pi, pi] by atan2 of sine and cosine;          */
/*   v = k_rho rho cos(alpha),                                               */
/*   w = k_alpha alpha + k_rho (sin(alpha) cos(alpha) / alpha)               */
/*       (alpha + k_beta beta),                                              */
/* with sin(alpha)/alpha = 1 at alpha = 0. Waypoint poses of the action      */
/* space: a move action a sets the pose waypoint_step ahead of the centre    */
/* along dir(a), heading along dir(a) (so beta = 0 there); staying sets the */
/* robot's own pose (v = w = 0).                                             */
/* ------------------------------------------------------------------------ */
static double wrap_angle(double a) { return atan2(sin(a), cos(a)); }

void orc_unicycle_pose(const orc_params *p, double x, double y, double theta, double wx,
                       double wy, double wth, double *v, double *w) {
  double ex = wx - x, ey = wy - y;
  double rho = sqrt(ex * ex + ey * ey);
  double phi = rho > 0.0 ? atan2(ey, ex) : wth;
  double alpha = wrap_angle(phi - theta);
  double beta = wrap_angle(phi - wth);
  double sinc = alpha != 0.0 ? sin(alpha) / alpha : 1.0;
  *v = p->pose_gain_rho * rho * cos(alpha);
  *w = p->pose_gain_alpha * alpha +
       p->pose_gain_rho * sinc * cos(alpha) * (alpha + p->pose_gain_beta * beta);
}

/* The projection point sits l ahead of the axle: its velocity is the
 * centre's velocity v (cos th, sin th) plus l w (-sin th, cos th). */
void orc_uni_to_si(const orc_params *p, double theta, double v, double w, double *ux,
                   double *uy) {
  double c = cos(theta), s = sin(theta), l = p->proj_dist;
  *ux = v * c - l * w * s;
  *uy = v * s + l * w * c;
}

/* ------------------------------------------------------------------------ */
/* Action noise (Sec. 7, domain randomisation: the policy trained with      */
/* action noise narrows the sim-to-real gap; the paper gives no             */
/* distribution). Reading: each coordinate of the nominal command gets an   */
/* independent uniform draw in [-sigma, sigma) from stream purpose 6,       */
/* counter (env_id, t, 6 << 24 | i, 0), words 0 (x) and 1 (y).              */
/* ------------------------------------------------------------------------ */
void orc_action_noise(const orc_params *p, uint64_t env_id, int64_t t_global, int32_t i,
                      double *nx, double *ny) {
  uint32_t o[4];
  stream_block(p, (uint32_t)env_id, (uint32_t)t_global, PURPOSE_NOISE, (uint32_t)i, 0, o);
  *nx = p->action_noise * (2.0 * unit_uniform(o[0]) - 1.0);
  *ny = p->action_noise * (2.0 * unit_uniform(o[1]) - 1.0);
}

void orc_nominal_command(const orc_params *p, int32_t n, uint64_t env_id, int64_t t_global,
                         const double *x, const double *y, const double *th, const double *gx,
                         const double *gy, const uint8_t *actions, uint8_t *actions_used,
                         double *unx, double *uny) {
  for (int32_t i = 0; i < n; ++i) {
    if (p->controller == 1) {
      double px = x[i] + p->proj_dist * cos(th[i]);
      double py = y[i] + p->proj_dist * sin(th[i]);
      unx[i] = p->kp * (gx[i] - px);
      uny[i] = p->kp * (gy[i] - py);
    } else {
      int32_t a = actions ? (int32_t)actions[i] : orc_random_action(p, env_id, t_global, i);
      if (actions_used) actions_used[i] = (uint8_t)a;
      double dx, dy;
      move_direction(a, &dx, &dy);
      if (p->controller == 2) {
        double wx = x[i] + p->waypoint_step * dx, wy = y[i] + p->waypoint_step * dy;
        double v, w;
        orc_unicycle_position(p, x[i], y[i], th[i], wx, wy, &v, &w);
        orc_uni_to_si(p, th[i], v, w, &unx[i], &uny[i]);
      } else if (p->controller == 3) {
        double wx = x[i] + p->waypoint_step * dx, wy = y[i] + p->waypoint_step * dy;
        double wth = (dx != 0.0 || dy != 0.0) ? atan2(dy, dx) : th[i];
        double v, w;
        orc_unicycle_pose(p, x[i], y[i], th[i], wx, wy, wth, &v, &w);
        orc_uni_to_si(p, th[i], v, w, &unx[i], &uny[i]);
      } else {
        unx[i] = p->action_speed * dx;
        uny[i] = p->action_speed * dy;
      }
    }
    if (p->action_noise > 0.0) {
      double nx, ny;
      orc_action_noise(p, env_id, t_global, i, &nx, &ny);
      unx[i] += nx;
      uny[i] += ny;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Predator-Prey (Appendix B: N taggers chase a faster prey; the prey takes, */
/* at every step, the move that keeps it farthest from the closest tagger;   */
/* a tag is the prey inside some tagger's radius; team reward 10 per tag).   */
/* Readings: the prey lives in every robot's goal slot (so the observation's */
/* last pair is the vector to the prey); its candidate moves are staying put */
/* and a step of prey_speed * dt in each of 16 evenly spaced directions,     */
/* each clamped to the arena pulled in by r_s/2; it takes the candidate with */
/* the largest squared distance to the closest robot centre, judged on the   */
/* centres before the robots move (both move at once), first index on ties. */
/* A step is tagged when, after both moved, some centre is closer than       */
/* tag_radius; episodes end on the step limit only.                          */
/* ------------------------------------------------------------------------ */
int32_t orc_prey_move(const orc_params *p, int32_t n, const double *x, const double *y, double qx,
                      double qy, double *nqx, double *nqy, double *scores) {
  double lox = p->x_min + 0.5 * p->safety_radius, hix = p->x_max - 0.5 * p->safety_radius;
  double loy = p->y_min + 0.5 * p->safety_radius, hiy = p->y_max - 0.5 * p->safety_radius;
  double step = p->prey_speed * p->dt;
  int32_t best = -1;
  double best_score = -1.0;
  for (int32_t k = 0; k <= 16; ++k) {
    double cx = qx, cy = qy;
    if (k > 0) {
      double a = 2.0 * M_PI * (double)(k - 1) / 16.0;
      cx = fmin(fmax(qx + step * cos(a), lox), hix);
      cy = fmin(fmax(qy + step * sin(a), loy), hiy);
    }
    double closest = INFINITY;
    for (int32_t j = 0; j < n; ++j) {
      double d2 = (cx - x[j]) * (cx - x[j]) + (cy - y[j]) * (cy - y[j]);
      if (d2 < closest) closest = d2;
    }
    if (scores) scores[k] = closest;
    if (closest > best_score) {
      best_score = closest;
      best = k;
      *nqx = cx;
      *nqy = cy;
    }
  }
  return best;
}

int32_t orc_tagged(const orc_params *p, int32_t n, const double *x, const double *y, double qx,
                   double qy) {
  for (int32_t j = 0; j < n; ++j)
    if (sqrt((x[j] - qx) * (x[j] - qx) + (y[j] - qy) * (y[j] - qy)) < p->tag_radius) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One environment step.                                                     */
/* ------------------------------------------------------------------------ */
int32_t orc_env_step(const orc_params *p, int32_t n, uint64_t env_id, int64_t t_global,
                     double *x, double *y, double *th, double *gx, double *gy, int32_t *step,
                     int32_t *episode, const uint8_t *actions, uint8_t *actions_used,
                     double *obs, double *reward, uint8_t *done, uint8_t *infeasible,
                     double *max_violation) {
  double px[ORC_MAX_N], py[ORC_MAX_N], unx[ORC_MAX_N], uny[ORC_MAX_N];
  double ux[ORC_MAX_N], uy[ORC_MAX_N];
  for (int32_t i = 0; i < n; ++i) {
    px[i] = x[i] + p->proj_dist * cos(th[i]);
    py[i] = y[i] + p->proj_dist * sin(th[i]);
  }
  orc_nominal_command(p, n, env_id, t_global, x, y, th, gx, gy, actions, actions_used, unx, uny);
  int pp = p->scenario == 1;
  double nqx = 0.0, nqy = 0.0;
  if (pp) orc_prey_move(p, n, x, y, gx[0], gy[0], &nqx, &nqy, NULL);
  double mv = 0.0;
  int32_t status = orc_barrier_certificate(p, n, px, py, unx, uny, ux, uy, NULL, NULL, &mv);
  if (infeasible) *infeasible = (uint8_t)(status == 1);
  if (max_violation) *max_violation = mv;
  for (int32_t i = 0; i < n; ++i) {
    double v, w;
    orc_si_to_uni(p, th[i], ux[i], uy[i], &v, &w);
    double c = cos(th[i]), s = sin(th[i]);
    x[i] += p->dt * v * c;
    y[i] += p->dt * v * s;
    double t = th[i] + p->dt * w;
    th[i] = atan2(sin(t), cos(t));
  }
  *step += 1;
  double r = 0.0;
  int finished;
  if (pp) {
    for (int32_t i = 0; i < n; ++i) {
      gx[i] = nqx;
      gy[i] = nqy;
    }
    r = orc_tagged(p, n, x, y, nqx, nqy) ? p->tag_reward : 0.0;
    finished = p->max_steps > 0 && *step >= p->max_steps;
  } else {
    int all_near = 1;
    for (int32_t i = 0; i < n; ++i) {
      double dist = sqrt((x[i] - gx[i]) * (x[i] - gx[i]) + (y[i] - gy[i]) * (y[i] - gy[i]));
      r -= dist;
      if (!(dist < p->goal_radius)) all_near = 0;
    }
    finished = (p->goal_radius > 0.0 && all_near) || (p->max_steps > 0 && *step >= p->max_steps);
  }
  if (reward) *reward = r;
  if (done) *done = (uint8_t)finished;
  if (finished) {
    *episode += 1;
    *step = 0;
    orc_reset_env(p, env_id, *episode, n, x, y, th, gx, gy);
  }
  if (obs) orc_observe(n, x, y, th, gx, gy, obs);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Policy: in -> 64 -> 64 -> 5 MLP, ReLU, bf16 operands, FP64 sums.          */
/* ------------------------------------------------------------------------ */
void orc_policy_logits(int32_t in_dim, const double *w1, const double *b1, const double *w2,
                       const double *b2, const double *w3, const double *b3, const double *obs,
                       double *logits) {
  double xin[64], h1[64], h2[64];
  for (int32_t k = 0; k < in_dim; ++k) xin[k] = orc_bf16_round(obs[k]);
  for (int32_t o = 0; o < 64; ++o) {
    double s = b1[o];
    for (int32_t k = 0; k < in_dim; ++k) s += xin[k] * w1[k * 64 + o];
    h1[o] = orc_bf16_round(s > 0.0 ? s : 0.0);
  }
  for (int32_t o = 0; o < 64; ++o) {
    double s = b2[o];
    for (int32_t k = 0; k < 64; ++k) s += h1[k] * w2[k * 64 + o];
    h2[o] = orc_bf16_round(s > 0.0 ? s : 0.0);
  }
  for (int32_t o = 0; o < 5; ++o) {
    double s = b3[o];
    for (int32_t k = 0; k < 64; ++k) s += h2[k] * w3[k * 5 + o];
    logits[o] = s;
  }
}

int32_t orc_sample_action(const double *logits, uint32_t r) {
  double mx = logits[0];
  for (int32_t k = 1; k < 5; ++k) mx = fmax(mx, logits[k]);
  double e[5], total = 0.0;
  for (int32_t k = 0; k < 5; ++k) { e[k] = exp(logits[k] - mx); total += e[k]; }
  double u = unit_uniform(r), cdf = 0.0;
  for (int32_t k = 0; k < 5; ++k) {
    cdf += e[k] / total;
    if (u < cdf) return k;
  }
  return 4;
}

uint32_t orc_policy_bits(const orc_params *p, uint64_t env_id, int64_t t_global, int32_t i) {
  uint32_t o[4];
  stream_block(p, (uint32_t)env_id, (uint32_t)t_global, PURPOSE_POLICY, (uint32_t)(i >> 2), 0, o);
  return o[i & 3];
}

/* ------------------------------------------------------------------------ */
/* Batched drivers, threaded over environment ranges.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_params *p;
  int32_t n, e0, e1;
  uint64_t env_id_base;
  int64_t t_global;
  double *x, *y, *th, *gx, *gy;
  int32_t *step, *episode;
  const uint8_t *actions;
  double *obs, *reward;
  uint8_t *done, *infeasible;
  /* rollout only */
  const double *w1, *b1, *w2, *b2, *w3, *b3;
  int32_t horizon, num_envs;
  uint8_t *actions_out;
  int32_t status;
} batch_job;

static void *step_range(void *arg) {
  batch_job *J = (batch_job *)arg;
  int32_t n = J->n, dim = 2 * n + 4;
  for (int32_t e = J->e0; e < J->e1; ++e) {
    size_t b = (size_t)e * n;
    int32_t st = orc_env_step(J->p, n, J->env_id_base + (uint64_t)e, J->t_global, J->x + b,
                              J->y + b, J->th + b, J->gx + b, J->gy + b, J->step + e,
                              J->episode + e, J->actions ? J->actions + b : NULL, NULL,
                              J->obs ? J->obs + b * dim : NULL, J->reward ? J->reward + e : NULL,
                              J->done ? J->done + e : NULL,
                              J->infeasible ? J->infeasible + e : NULL, NULL);
    if (st == 2) J->status = 2;
  }
  return NULL;
}

static void *rollout_range(void *arg) {
  batch_job *J = (batch_job *)arg;
  int32_t n = J->n, dim = 2 * n + 4, E = J->num_envs;
  double ob[ORC_MAX_N * (2 * ORC_MAX_N + 4)];
  uint8_t act[ORC_MAX_N];
  for (int32_t e = J->e0; e < J->e1; ++e) {
    size_t b = (size_t)e * n;
    uint64_t env_id = J->env_id_base + (uint64_t)e;
    orc_observe(n, J->x + b, J->y + b, J->th + b, J->gx + b, J->gy + b, ob);
    for (int32_t t = 0; t < J->horizon; ++t) {
      int64_t tg = J->t_global + t;
      size_t row = (size_t)t * E + e;
      if (J->obs) memcpy(J->obs + row * n * dim, ob, sizeof(double) * n * dim);
      for (int32_t i = 0; i < n; ++i) {
        double logits[5];
        orc_policy_logits(dim, J->w1, J->b1, J->w2, J->b2, J->w3, J->b3, ob + (size_t)i * dim,
                          logits);
        act[i] = (uint8_t)orc_sample_action(logits, orc_policy_bits(J->p, env_id, tg, i));
        J->actions_out[row * n + i] = act[i];
      }
      double r;
      uint8_t dn;
      int32_t st = orc_env_step(J->p, n, env_id, tg, J->x + b, J->y + b, J->th + b, J->gx + b,
                                J->gy + b, J->step + e, J->episode + e, act, NULL, ob, &r, &dn,
                                NULL, NULL);
      if (st == 2) J->status = 2;
      J->reward[row] = r;
      J->done[row] = dn;
    }
  }
  return NULL;
}

static int32_t run_threads(batch_job *proto, int32_t num_envs, int32_t nthreads,
                           void *(*fn)(void *)) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > num_envs) nthreads = num_envs > 0 ? num_envs : 1;
  batch_job jobs[256];
  pthread_t tids[256];
  if (nthreads > 256) nthreads = 256;
  for (int32_t k = 0; k < nthreads; ++k) {
    jobs[k] = *proto;
    jobs[k].e0 = (int32_t)((int64_t)num_envs * k / nthreads);
    jobs[k].e1 = (int32_t)((int64_t)num_envs * (k + 1) / nthreads);
    jobs[k].status = 0;
  }
  if (nthreads == 1) {
    fn(&jobs[0]);
  } else {
    for (int32_t k = 0; k < nthreads; ++k) pthread_create(&tids[k], NULL, fn, &jobs[k]);
    for (int32_t k = 0; k < nthreads; ++k) pthread_join(tids[k], NULL);
  }
  int32_t status = 0;
  for (int32_t k = 0; k < nthreads; ++k)
    if (jobs[k].status) status = jobs[k].status;
  return status;
}

int32_t orc_env_step_batch(const orc_params *p, int32_t n, int32_t num_envs, uint64_t env_id_base,
                           int64_t t_global, double *x, double *y, double *th, double *gx,
                           double *gy, int32_t *step, int32_t *episode, const uint8_t *actions,
                           double *obs, double *reward, uint8_t *done, uint8_t *infeasible,
                           int32_t nthreads) {
  batch_job J;
  memset(&J, 0, sizeof(J));
  J.p = p; J.n = n; J.env_id_base = env_id_base; J.t_global = t_global;
  J.x = x; J.y = y; J.th = th; J.gx = gx; J.gy = gy; J.step = step; J.episode = episode;
  J.actions = actions; J.obs = obs; J.reward = reward; J.done = done; J.infeasible = infeasible;
  return run_threads(&J, num_envs, nthreads, step_range);
}

int32_t orc_rollout(const orc_params *p, int32_t n, int32_t num_envs, uint64_t env_id_base,
                    int64_t t_global0, const double *w1, const double *b1, const double *w2,
                    const double *b2, const double *w3, const double *b3, int32_t horizon,
                    double *x, double *y, double *th, double *gx, double *gy, int32_t *step,
                    int32_t *episode, double *obs, uint8_t *actions, double *reward,
                    uint8_t *done, int32_t nthreads) {
  batch_job J;
  memset(&J, 0, sizeof(J));
  J.p = p; J.n = n; J.env_id_base = env_id_base; J.t_global = t_global0;
  J.x = x; J.y = y; J.th = th; J.gx = gx; J.gy = gy; J.step = step; J.episode = episode;
  J.obs = obs; J.reward = reward; J.done = done; J.actions_out = actions;
  J.w1 = w1; J.b1 = b1; J.w2 = w2; J.b2 = b2; J.w3 = w3; J.b3 = b3;
  J.horizon = horizon; J.num_envs = num_envs;
  return run_threads(&J, num_envs, nthreads, rollout_range);
}
