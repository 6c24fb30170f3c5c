"""Brute-force active-set enumeration for the barrier-certificate projection.

Independent pin for the oracle's QP: every subset S of pairwise rows and every
assignment of each coordinate to {free, at lower bound, at upper bound} defines
an affine set; the projection of the nominal command onto it is a KKT point of
the full problem when it is feasible and its multipliers have the right signs.
The problem is strictly convex, so exactly one such point exists when the
feasible set is nonempty. Built from the constraint definitions written out
here (pairwise cubic certificate and per-coordinate wall/speed bounds).
"""
import itertools

import numpy as np


def constraint_data(p, px, py):
    n = px.size
    nv = 2 * n
    A, b = [], []
    for i in range(n):
        for j in range(i + 1, n):
            dx, dy = px[i] - px[j], py[i] - py[j]
            h = dx * dx + dy * dy - p.safety_radius ** 2
            a = np.zeros(nv)
            a[2 * i], a[2 * i + 1] = -2 * dx, -2 * dy
            a[2 * j], a[2 * j + 1] = 2 * dx, 2 * dy
            A.append(a)
            b.append(p.barrier_gain * h ** 3)
    kb = p.boundary_gain_factor * p.barrier_gain
    half = p.safety_radius / 2
    lo, hi = np.zeros(nv), np.zeros(nv)
    for i in range(n):
        hi[2 * i] = min(p.v_max, kb * (p.x_max - half - px[i]) ** 3)
        lo[2 * i] = max(-p.v_max, -kb * (px[i] - p.x_min - half) ** 3)
        hi[2 * i + 1] = min(p.v_max, kb * (p.y_max - half - py[i]) ** 3)
        lo[2 * i + 1] = max(-p.v_max, -kb * (py[i] - p.y_min - half) ** 3)
    return np.array(A).reshape(-1, nv), np.array(b), lo, hi


def preclip(p, uxn, uyn):
    uh = np.zeros(2 * uxn.size)
    for i in range(uxn.size):
        vx, vy = uxn[i], uyn[i]
        nr = np.hypot(vx, vy)
        if nr > p.v_max:
            vx, vy = vx * p.v_max / nr, vy * p.v_max / nr
        uh[2 * i], uh[2 * i + 1] = vx, vy
    return uh


def enumerate_kkt_points(A, b, lo, hi, uh, tol=1e-9):
    nv = uh.size
    P = A.shape[0]
    found = []
    for smask in range(1 << P):
        S = [k for k in range(P) if smask >> k & 1]
        for fmask in range(1 << nv):
            F = [v for v in range(nv) if fmask >> v & 1]
            m = len(S) + len(F)
            if m > nv:
                continue
            if m == 0:
                cands = [(uh.copy(), None)]
            else:
                M = np.zeros((m, nv))
                for r, k in enumerate(S):
                    M[r] = A[k]
                for r, v in enumerate(F):
                    M[len(S) + r, v] = 1.0
                G = M @ M.T
                if np.linalg.cond(G) > 1e10:
                    continue
                Ginv = np.linalg.inv(G)
                cands = []
                for side in itertools.product((0, 1), repeat=len(F)):
                    c = np.concatenate([b[S], [hi[v] if s else lo[v] for v, s in zip(F, side)]])
                    nu = Ginv @ (M @ uh - c)
                    ok = all(nu[r] >= -tol for r in range(len(S)))
                    for r, s in enumerate(side):
                        val = nu[len(S) + r]
                        ok = ok and (val >= -tol if s else val <= tol)
                    if ok:
                        cands.append((uh - M.T @ nu, None))
            for u, _ in cands:
                if P and (A @ u - b > tol * np.maximum(1.0, np.linalg.norm(A, axis=1))).any():
                    continue
                if (u - hi > tol).any() or (lo - u > tol).any():
                    continue
                found.append(u)
    return found
