"""Oracle linear algebra: the block-bordered primal-dual KKT system of the
scenario NLP, built densely per scenario and solved through a 1x1 Schur
complement on the shared diameter.

TEST INFRASTRUCTURE ONLY (see oracle/model.py).

The system is the slack-reduced primal-dual Newton system of an interior-point
method for problem (10) (the problem statement, eqs. 8 and 10: scenarios are
coupled only through the design variable).  Per scenario omega, with unknowns
ordered [x (21N), y_c (21N), y_d (N)]:

    K_w = [[W_xx + Sigma_x + dw I,   J_c^T,     J_d^T                ],
           [J_c,                     -dc I,     0                    ],
           [J_d,                     0,         -(1/(Sigma_s+dw)+dc) ]]

The border column b_w holds the derivatives with respect to d and
k_dd = sum_w W_dd,w + Sigma_d + dw.  The Schur complement on d is
S_d = k_dd - sum_w b_w^T K_w^{-1} b_w, and by Haynsworth's inertia additivity
In(K) = sum_w In(K_w) + In(S_d).  With a design vector theta of p entries
(the general scenario NLP, eq. 8) the border is a 43N x p matrix B_w, K_dd is
p x p and the Schur complement S = K_dd - sum_w B_w^T K_w^{-1} B_w is a dense
p x p matrix whose inertia comes from its eigenvalues.

Each K_w is factorised by LAPACK's Bunch-Kaufman LDL^T (dsytrf) after a
symmetric diagonal equilibration; the inertia is read from the 1x1 and 2x2
pivot blocks (Sylvester's law of inertia), and every solve is refined against
the unscaled matrix.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg.lapack as lapack

from .model import NR, NV

ZERO_PIVOT = 1e-20  # |eigenvalue| of an equilibrated pivot block counted as zero
REFINE_TOL = 1e-10  # refinement stops at this relative residual ||r - Kx||_inf / ||r||_inf (or when it stalls)


def scenario_kkt(J: np.ndarray, H: np.ndarray, sig_x: np.ndarray, sig_s: np.ndarray,
                 dw: float, dc: float, N: int, p: int = 1):
    """Assemble K_w (43N x 43N), the border b_w (43N,), or (43N, p) for p design
    variables, and this scenario's W_dd (scalar, or (p, p)).

    J: (22N, 21N+p) scaled Jacobian; H: (21N+p, 21N+p) Hessian of the scaled
    Lagrangian; sig_x: (21N,) primal barrier diagonal; sig_s: (N,) slack
    barrier diagonal.
    """
    nx = NV * N
    eq = np.array([n * NR + r for n in range(N) for r in range(NR - 1)])
    hy = np.array([n * NR + NR - 1 for n in range(N)])
    Jc, Jd = J[eq, :nx], J[hy, :nx]
    dim = nx + len(eq) + len(hy)
    K = np.zeros((dim, dim))
    K[:nx, :nx] = H[:nx, :nx] + np.diag(sig_x + dw)
    K[nx:nx + len(eq), :nx] = Jc
    K[:nx, nx:nx + len(eq)] = Jc.T
    K[nx + len(eq):, :nx] = Jd
    K[:nx, nx + len(eq):] = Jd.T
    K[nx:nx + len(eq), nx:nx + len(eq)] = -dc * np.eye(len(eq))
    K[nx + len(eq):, nx + len(eq):] = -np.diag(1.0 / (sig_s + dw) + dc)
    if p == 1:
        b = np.concatenate([H[:nx, nx], J[eq, nx], J[hy, nx]])
        return K, b, H[nx, nx]
    B = np.concatenate([H[:nx, nx:], J[eq, nx:], J[hy, nx:]], axis=0)
    return K, B, H[nx:, nx:]


class SymFactor:
    """Equilibrated Bunch-Kaufman factorisation of one symmetric matrix."""

    def __init__(self, K: np.ndarray):
        self.K = K
        rmax = np.abs(K).max(axis=1)
        rmax[rmax == 0.0] = 1.0
        self.s = 1.0 / np.sqrt(rmax)
        Ks = self.s[:, None] * K * self.s[None, :]
        lu, ipiv, info = lapack.dsytrf(Ks, lower=1)
        if info < 0:
            raise RuntimeError(f"dsytrf argument error {info}")
        self.lu, self.ipiv = lu, ipiv
        self.inertia = self._inertia(lu, ipiv)

    @staticmethod
    def _inertia(lu, ipiv):
        n = lu.shape[0]
        pos = neg = zero = 0
        k = 0
        while k < n:
            if ipiv[k] > 0:  # 1x1 pivot block (LAPACK 1-based positive pivot)
                ev = [lu[k, k]]
                k += 1
            else:  # 2x2 pivot block
                blk = np.array([[lu[k, k], lu[k + 1, k]], [lu[k + 1, k], lu[k + 1, k + 1]]])
                ev = list(np.linalg.eigvalsh(blk))
                k += 2
            for e in ev:
                if abs(e) <= ZERO_PIVOT:
                    zero += 1
                elif e > 0:
                    pos += 1
                else:
                    neg += 1
        return pos, neg, zero

    def _raw_solve(self, r):
        x, info = lapack.dsytrs(self.lu, self.ipiv, self.s * r, lower=1)
        if info != 0:
            raise RuntimeError(f"dsytrs error {info}")
        return self.s * x

    def solve(self, r: np.ndarray, refine: int = 5) -> np.ndarray:
        x = self._raw_solve(r)
        for _ in range(refine):
            res = r - self.K @ x
            if np.abs(res).max() <= 1e-15 * max(np.abs(r).max(), 1e-300):
                break
            x = x + self._raw_solve(res)
        return x


class BorderedKKT:
    """Factorisation of the full block-bordered system via the Schur complement on
    the design variables: d (borders (43N,), kdd scalar) or a design vector of p
    entries (borders (43N, p), kdd (p, p))."""

    def __init__(self, blocks, borders, kdd):
        self.blocks = [SymFactor(K) for K in blocks]
        self.borders = borders
        self.kdd = kdd
        self.p = 1 if np.ndim(kdd) == 0 else np.shape(kdd)[0]
        if self.p == 1:
            self.v = [F.solve(b) for F, b in zip(self.blocks, borders)]
        else:  # K_w^{-1} B_w column by column
            self.v = [np.stack([F.solve(B[:, k]) for k in range(self.p)], axis=1)
                      for F, B in zip(self.blocks, borders)]
        p = n = z = 0
        for F in self.blocks:
            p, n, z = p + F.inertia[0], n + F.inertia[1], z + F.inertia[2]
        if self.p == 1:
            self.sd = kdd - sum(float(b @ v) for b, v in zip(borders, self.v))
            if abs(self.sd) <= ZERO_PIVOT * max(1.0, abs(kdd)):
                z += 1
            elif self.sd > 0:
                p += 1
            else:
                n += 1
        else:
            S = np.array(kdd, dtype=np.float64)
            for B, V in zip(borders, self.v):
                S = S - B.T @ V
            self.sd = 0.5 * (S + S.T)
            ev = np.linalg.eigvalsh(self.sd)
            tiny = ZERO_PIVOT * max(1.0, float(np.abs(kdd).max()))
            p += int((ev > tiny).sum())
            n += int((ev < -tiny).sum())
            z += int((np.abs(ev) <= tiny).sum())
        self.inertia = (p, n, z)

    def _solve_once(self, rs, rd):
        us = [F.solve(r) for F, r in zip(self.blocks, rs)]
        if self.p == 1:
            dd = (rd - sum(float(b @ u) for b, u in zip(self.borders, us))) / self.sd
            return [u - v * dd for u, v in zip(us, self.v)], dd
        rhs = np.array(rd, dtype=np.float64)
        for B, u in zip(self.borders, us):
            rhs = rhs - B.T @ u
        dd = np.linalg.solve(self.sd, rhs)
        return [u - V @ dd for u, V in zip(us, self.v)], dd

    def residual(self, xs, xd, rs, rd):
        """Residual r - Kx and the componentwise backward error
        max_i |r - Kx|_i / (|K||x| + |r|)_i of the whole bordered system."""
        if self.p > 1:
            return self._residual_p(xs, xd, rs, rd)
        res, omega = [], 0.0
        for F, b, x, r in zip(self.blocks, self.borders, xs, rs):
            rr = r - (F.K @ x + b * xd)
            den = np.abs(F.K) @ np.abs(x) + np.abs(b) * abs(xd) + np.abs(r)
            omega = max(omega, float(np.max(np.abs(rr) / np.where(den > 0, den, 1.0))))
            res.append(rr)
        resd = rd - sum(float(b @ x) for b, x in zip(self.borders, xs)) - self.kdd * xd
        dend = sum(float(np.abs(b) @ np.abs(x)) for b, x in zip(self.borders, xs)) + abs(self.kdd * xd) + abs(rd)
        omega = max(omega, abs(resd) / (dend if dend > 0 else 1.0))
        return res, resd, omega

    def _residual_p(self, xs, xd, rs, rd):
        res, omega = [], 0.0
        xd = np.asarray(xd, dtype=np.float64)
        resd = np.array(rd, dtype=np.float64) - np.asarray(self.kdd) @ xd
        dend = np.abs(np.asarray(self.kdd)) @ np.abs(xd) + np.abs(rd)
        for F, B, x, r in zip(self.blocks, self.borders, xs, rs):
            rr = r - (F.K @ x + B @ xd)
            den = np.abs(F.K) @ np.abs(x) + np.abs(B) @ np.abs(xd) + np.abs(r)
            omega = max(omega, float(np.max(np.abs(rr) / np.where(den > 0, den, 1.0))))
            res.append(rr)
            resd = resd - B.T @ x
            dend = dend + np.abs(B).T @ np.abs(x)
        omega = max(omega, float(np.max(np.abs(resd) / np.where(dend > 0, dend, 1.0))))
        return res, resd, omega

    def solve(self, rs, rd: float, refine: int = 10):
        """Solve with per-scenario right-hand sides rs (list) and the d entry rd,
        refining on the whole bordered system until the relative residual
        ||r - Kx||_inf / ||r||_inf is at most REFINE_TOL or stops improving."""
        xs, xd = self._solve_once(rs, rd)
        rn = max([float(np.abs(rd).max())] + [float(np.abs(r).max()) for r in rs])
        best = None
        for _ in range(refine):
            res, resd, omega = self.residual(xs, xd, rs, rd)
            num = max([float(np.abs(resd).max())] + [float(np.abs(r).max()) for r in res])
            rel = num / rn if rn > 0 else num
            if best is not None and not rel < best[0]:
                xs, xd = best[1], best[2]
                break
            best = (rel, xs, xd, omega)
            if rel <= REFINE_TOL:
                break
            cs, cd = self._solve_once(res, resd)
            xs, xd = [x + c for x, c in zip(xs, cs)], xd + cd
        self.last_rel, self.last_omega = best[0], best[3]
        return xs, xd

    def rel_residual(self, xs, xd, rs, rd) -> float:
        """||K x - r||_inf / ||r||_inf of the full bordered system."""
        if self.p > 1:
            res, resd, _ = self._residual_p(xs, xd, rs, rd)
            num = max([float(np.abs(resd).max())] + [float(np.abs(r).max()) for r in res])
            den = max([float(np.abs(rd).max())] + [float(np.abs(r).max()) for r in rs])
            return num / max(den, 1e-300)
        num = abs(sum(float(b @ x) for b, x in zip(self.borders, xs)) + self.kdd * xd - rd)
        den = abs(rd)
        for F, b, x, r in zip(self.blocks, self.borders, xs, rs):
            num = max(num, float(np.abs(F.K @ x + b * xd - r).max()))
            den = max(den, float(np.abs(r).max()))
        return num / max(den, 1e-300)
