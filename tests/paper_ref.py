"""Independent statements of the paper's objectives, used to pin the oracle.

Nothing here calls the oracle's arithmetic.  The basis comes from SciPy's
Bernstein-polynomial class; every objective is written row by row from the
paper's equations (not through the stacked F matrix); the equality-constrained
QPs are solved by the null-space method with SciPy's linear algebra, a
different algorithm from the oracle's LU factorisation of the KKT matrix.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import BPoly
from scipy.linalg import lstsq, null_space


def bernstein_scipy(q: int, nv: int, tf: float):
    """P, Pdot, Pddot on t_k = k tf/(q-1) via scipy.interpolate.BPoly."""
    t = np.arange(q) * (tf / (q - 1))
    P, Pd, Pdd = (np.zeros((q, nv)) for _ in range(3))
    for i in range(nv):
        c = np.zeros((nv, 1))
        c[i, 0] = 1.0
        bp = BPoly(c, [0.0, tf])
        P[:, i] = bp(t)
        Pd[:, i] = bp.derivative(1)(t)
        Pdd[:, i] = bp.derivative(2)(t)
    return P, Pd, Pdd


def boundary_rows(P, Pd, Pdd):
    return np.stack([P[0], Pd[0], Pdd[0], P[-1], Pd[-1], Pdd[-1]])


def atan2z(y, x):
    y = np.asarray(y, dtype=float)
    x = np.asarray(x, dtype=float)
    return np.where((x == 0) & (y == 0), 0.0, np.arctan2(y, x))


def quad_parts(J, dim):
    """Hessian H and gradient at zero g of a quadratic function J (exact up to
    rounding: second differences of a quadratic are constant)."""
    J0 = J(np.zeros(dim))
    e = np.eye(dim)
    Ji = np.array([J(e[i]) for i in range(dim)])
    Jm = np.array([J(-e[i]) for i in range(dim)])
    g = (Ji - Jm) / 2.0
    H = np.zeros((dim, dim))
    for i in range(dim):
        H[i, i] = Ji[i] + Jm[i] - 2.0 * J0
        for j in range(i + 1, dim):
            H[i, j] = H[j, i] = (J(e[i] + e[j]) - Ji[i] - Ji[j] + J0)
    return H, g


def nullspace_qp(H, g, A, b):
    """argmin 0.5 x^T H x + g^T x subject to A x = b, by the null-space method."""
    xp = lstsq(A, b)[0]
    Z = null_space(A)
    Hz = Z.T @ H @ Z
    w = np.linalg.solve(Hz, -Z.T @ (H @ xp + g))
    return xp + Z @ w


class PaperProblem:
    """Objectives of Sec. III for one trajectory, written from the equations."""

    def __init__(self, pb: dict):
        self.pb = pb
        self.q, self.nv = int(pb["q"]), int(pb["nv"])
        self.P, self.Pd, self.Pdd = bernstein_scipy(self.q, self.nv, float(pb["tf"]))
        self.A = boundary_rows(self.P, self.Pd, self.Pdd)
        self.r = np.asarray(pb["r"], float)
        self.ox, self.oy = np.asarray(pb["ox"], float), np.asarray(pb["oy"], float)
        self.a = np.asarray(pb["oa"], float) + pb["rc"]
        self.b = np.asarray(pb["ob"], float) + pb["rc"]
        self.m, self.n = len(self.r), len(self.a)
        self.flags = int(pb.get("flags", 0))

    # --- constraint rows of Sec. III-C, one axis at a time -------------------
    def penalty_rows(self, xi, axis, st, l, psi):
        """Residual rows of F xi - g for one axis (0 = x, 1 = y), listed as the
        paper lists the blocks: velocity, acceleration, obstacle (i, j), slack."""
        nv, q = self.nv, self.q
        cp, cs = xi[:nv], xi[nv:]
        pos, vel, acc, sl = self.P @ cp, self.Pd @ cp, self.Pdd @ cp, self.P @ cs
        trig = np.cos if axis == 0 else np.sin
        vm, am = self.pb["vmax"], self.pb["amax"]
        rows = [vel - vm * st["dv"][l] * trig(st["av"][l]),
                acc - am * st["da"][l] * trig(st["aa"][l])]
        for i in range(self.m):
            for j in range(self.n):
                e = i * self.n + j
                centre = self.ox[j] if axis == 0 else self.oy[j]
                semi = self.a[j] if axis == 0 else self.b[j]
                rows.append(pos + self.r[i] * sl - centre - semi * st["d"][l, e] * trig(st["alpha"][l, e]))
        rows.append(sl - trig(psi))
        return np.concatenate(rows)

    def xi1_objective(self, st, l):
        """Objective of eq. (zeta_1_sepration_1) for both axes, xi = (cx, cc, cy, cs)."""
        nv, rho = self.nv, self.pb["rho"]
        psi = self.P @ st["cpsi"][l]
        lam = st["lam"][l]
        q_cs = not (self.flags & 16)

        def J(xi):
            tot = 0.0
            for axis in (0, 1):
                blk = xi[axis * 2 * nv:(axis + 1) * 2 * nv]
                tot += 0.5 * np.sum((self.Pdd @ blk[:nv]) ** 2)
                if q_cs:
                    tot += 0.5 * np.sum((self.Pdd @ blk[nv:]) ** 2)
                tot += 0.5 * rho * np.sum(self.penalty_rows(blk, axis, st, l, psi) ** 2)
            return tot - lam @ xi
        return J

    def xi1_solution(self, st, l):
        nv = self.nv
        J = self.xi1_objective(st, l)
        H, g = quad_parts(J, 4 * nv)
        Abig = np.zeros((12, 4 * nv))
        Abig[:6, :nv] = self.A
        Abig[6:, 2 * nv:3 * nv] = self.A
        bbig = np.concatenate([self.pb["bx"], self.pb["by"]])
        return nullspace_qp(H, g, Abig, bbig)

    def psi_hat(self, st, l):
        c, s = self.P @ st["cc"][l], self.P @ st["cs"][l]
        psi = self.P @ st["cpsi"][l]
        if self.flags & 4:
            return atan2z(s, c)
        return psi + atan2z(s * np.cos(psi) - c * np.sin(psi), c * np.cos(psi) + s * np.sin(psi))

    def xi2_solution(self, st, l):
        """Minimiser of eq. (compute_convex_surrogate) subject to A c_psi = b_psi."""
        rho = self.pb["rho"]
        ph = self.psi_hat(st, l)
        lp = st["lampsi"][l]

        def J(c):
            return 0.5 * np.sum((self.Pdd @ c) ** 2) - lp @ c + 0.5 * rho * np.sum((ph - self.P @ c) ** 2)
        H, g = quad_parts(J, self.nv)
        return nullspace_qp(H, g, self.A, np.asarray(self.pb["bpsi"], float))

    # --- the remaining steps of Sec. III-D, written independently -----------
    def project(self, st, l):
        """xi3, xi4 of trajectory l (eqs. zeta_2, compute_zeta_3, alpha_v,
        alpha_a, compute_dv, compute_da) from its current coefficients, with
        the readings the oracle takes: elliptic angle unless the literal flag,
        x~ from cos psi unless the slack flag, d by the ratio form, angle 0 at
        the zero vector, d_v and d_a clipped to [0, 1]."""
        P, Pd, Pdd = self.P, self.Pd, self.Pdd
        x, y = P @ st["cx"][l], P @ st["cy"][l]
        psi = P @ st["cpsi"][l]
        if self.flags & 2:
            ux, uy = P @ st["cc"][l], P @ st["cs"][l]
        else:
            ux, uy = np.cos(psi), np.sin(psi)
        for i in range(self.m):
            for j in range(self.n):
                a, b = self.a[j], self.b[j]
                xt = x + self.r[i] * ux - self.ox[j]
                yt = y + self.r[i] * uy - self.oy[j]
                al = atan2z(yt, xt) if self.flags & 1 else atan2z(a * yt, b * xt)
                ca, sa = np.cos(al), np.sin(al)
                d = (a * xt * ca + b * yt * sa) / (a * a * ca * ca + b * b * sa * sa)
                e = i * self.n + j
                st["alpha"][l, e] = al
                st["d"][l, e] = np.maximum(1.0, d)
        for (vx, vy, lim, ka, kd) in ((Pd @ st["cx"][l], Pd @ st["cy"][l], self.pb["vmax"], "av", "dv"),
                                      (Pdd @ st["cx"][l], Pdd @ st["cy"][l], self.pb["amax"], "aa", "da")):
            al = atan2z(vy, vx)
            st[ka][l] = al
            st[kd][l] = np.clip((vx * np.cos(al) + vy * np.sin(al)) / lim, 0.0, 1.0)

    def lambda_update(self, st, l):
        """eq. update_lambda_1 as the gradient step of the row-wise penalty
        (its rows are affine in xi, so the Jacobian is exact), and eq.
        update_lambda_psi with the reading's sign."""
        nv, rho = self.nv, self.pb["rho"]
        psi = self.P @ st["cpsi"][l]
        for axis in (0, 1):
            xi = np.concatenate([st["cx" if axis == 0 else "cy"][l], st["cc" if axis == 0 else "cs"][l]])
            r0 = self.penalty_rows(np.zeros(2 * nv), axis, st, l, psi)
            J = np.stack([self.penalty_rows(e, axis, st, l, psi) - r0 for e in np.eye(2 * nv)], axis=1)
            grad = J.T @ self.penalty_rows(xi, axis, st, l, psi)
            st["lam"][l, axis * 2 * nv:(axis + 1) * 2 * nv] -= rho * grad
        sign = -1.0 if self.flags & 8 else 1.0
        st["lampsi"][l] -= sign * self.pb["rho_psi"] * (self.P.T @ (psi - st["psihat"][l]))

    def am_solve(self, st, K):
        """The AM list of Sec. III-D for every trajectory, in place: the
        initial xi3, xi4, then K times xi1, xi2, xi3, xi4 and the
        multipliers."""
        B, nv = st["cx"].shape[0], self.nv
        for l in range(B):
            self.project(st, l)
        for _ in range(K):
            for l in range(B):
                xi = self.xi1_solution(st, l)
                st["cx"][l], st["cc"][l] = xi[:nv], xi[nv:2 * nv]
                st["cy"][l], st["cs"][l] = xi[2 * nv:3 * nv], xi[3 * nv:]
                ph = self.psi_hat(st, l)
                st["cpsi"][l] = self.xi2_solution(st, l)
                st["psihat"][l] = ph
                self.project(st, l)
                self.lambda_update(st, l)
