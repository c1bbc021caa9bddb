"""Minimax rational approximation of x^p in relative error (Remez exchange).

The RHMC step of the paper (Sec. 2.1, the rooted system and its rational
approximation) replaces ``(M^dagger M)^(N_f/4)`` by a rational function in
partial fractions, ``r(x) = alpha0 + sum_i alpha_i / (x + beta_i)``, whose
shifted systems are then solved together by the multi-shift solver.  The
paper does not print coefficients, so they are generated here, once, on the
host, and handed to the solver as inputs (like the gauge field).

Algorithm (textbook Remez exchange for type (n, n), weight 1/f):

1. Start from 2n+2 reference points on [lo, hi], Chebyshev-clustered in log x.
2. On the reference, solve ``P(x_k) = f(x_k) (1 + (-1)^k E) Q(x_k)`` for the
   coefficients of P, monic Q and the levelled error E.  The first
   reference is solved exactly as a generalised eigenproblem in E, keeping
   the eigenvalue whose Q has no sign change on the reference (no pole in
   the interval); later references are solved by Newton's method started
   from the previous solution.
3. Scan ``e(x) = P/(Q f) - 1`` on a dense log grid, take the extremum of
   each run of equal sign and keep 2n+2 alternating ones (multi-point
   exchange); these form the next reference.
4. Stop when the extrema are levelled: ``(max|e| - |E|) / max|e| < rtol``.

Everything runs in mpmath multiprecision in the scaled variable
``u = x / sqrt(lo*hi)``.  The partial-fraction form comes from the roots of Q
(real and negative for the exponents used here) and the residues
``P(u_i)/Q'(u_i)``.
"""

from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass, field

import mpmath as mp

_DATA_DIR = os.path.join(os.path.dirname(__file__), "data")


@dataclass
class Rational:
    p: float
    n: int
    lo: float
    hi: float
    alpha0: float
    alpha: list = field(default_factory=list)
    beta: list = field(default_factory=list)
    delta: float = 0.0          # levelled relative error of the multiprecision fit
    iterations: int = 0

    def to_json(self) -> str:
        return json.dumps(asdict(self), indent=1)

    @staticmethod
    def from_json(s: str) -> "Rational":
        return Rational(**json.loads(s))

    def __call__(self, x):
        """Evaluate r(x) in float64 (x scalar or numpy array)."""
        import numpy as np

        x = np.asarray(x, dtype=np.float64)
        y = np.full_like(x, self.alpha0)
        for a, b in zip(self.alpha, self.beta):
            y = y + a / (x + b)
        return y


def _poly(c, u):
    """sum_j c[j] u^j (Horner)."""
    acc = mp.mpf(0)
    for cj in reversed(c):
        acc = acc * u + cj
    return acc


class _Remez:
    def __init__(self, p, n, lo, hi):
        self.p = mp.mpf(p)
        self.n = n
        self.lo = mp.mpf(lo)
        self.hi = mp.mpf(hi)
        self.s = mp.sqrt(self.lo * self.hi)

    def f(self, x):
        return mp.power(x, self.p)

    def err(self, x, P, Q):
        u = x / self.s
        return _poly(P, u) / (_poly(Q, u) * self.f(x)) - 1

    def initial_reference(self):
        n = self.n
        m = 2 * n + 2
        la, lb = mp.log(self.lo), mp.log(self.hi)
        pts = []
        for k in range(m):
            t = (1 - mp.cos(mp.pi * k / (m - 1))) / 2
            pts.append(mp.exp(la + t * (lb - la)))
        return pts

    def solve_reference(self, xs, guess=None):
        """Solve F_k = P(u_k) - f_k (1 + (-1)^k E) Q(u_k) = 0, k = 0..2n+1.

        Unknowns: p_0..p_n, q_0..q_{n-1} (Q monic) and E.  Newton's method,
        started from the previous reference's solution, or from the E = 0
        interpolant when there is none.
        """
        n = self.n
        m = 2 * n + 2
        us = [x / self.s for x in xs]
        fs = [self.f(x) for x in xs]
        upow = [[mp.power(u, j) for j in range(n + 1)] for u in us]
        sg = [1 if k % 2 == 0 else -1 for k in range(m)]
        if guess is None:
            z = self._pole_free_start(us, fs, upow, sg)
        else:
            P0, Q0, E0 = guess
            z = list(P0) + list(Q0[:n]) + [E0]
        tol = mp.mpf(10) ** (-(mp.mp.dps * 2 // 3))
        for _ in range(50):
            P = z[:n + 1]
            Q = z[n + 1:2 * n + 1] + [mp.mpf(1)]
            E = z[2 * n + 1]
            rows, F = [], []
            for k in range(m):
                Pk = sum(P[j] * upow[k][j] for j in range(n + 1))
                Qk = sum(Q[j] * upow[k][j] for j in range(n + 1))
                w = fs[k] * (1 + sg[k] * E)
                F.append(-(Pk - w * Qk))
                rows.append(upow[k][:n + 1] + [-w * upow[k][j] for j in range(n)]
                            + [-sg[k] * fs[k] * Qk])
            dz = mp.lu_solve(mp.matrix(rows), mp.matrix(F))
            z = [z[i] + dz[i] for i in range(m)]
            if abs(dz[m - 1]) <= tol * abs(z[m - 1]):
                break
        P = z[:n + 1]
        Q = z[n + 1:2 * n + 1] + [mp.mpf(1)]
        return P, Q, z[2 * n + 1]

    def _pole_free_start(self, us, fs, upow, sg):
        """Exact solution of the reference equations without a pole.

        With c = (p_0..p_n, q_0..q_n) the equations read (A0 + E A1) c = 0,
        a generalised eigenproblem in E.  Of its finite real eigenvalues the
        one whose Q keeps one sign on the reference is taken (a pole between
        reference points would make e unbounded).
        """
        n = self.n
        m = 2 * n + 2
        A0 = mp.matrix([upow[k][:n + 1] + [-fs[k] * upow[k][j] for j in range(n + 1)]
                        for k in range(m)])
        A1 = mp.matrix([[0] * (n + 1) + [-sg[k] * fs[k] * upow[k][j] for j in range(n + 1)]
                        for k in range(m)])
        M = mp.inverse(A0) * A1
        mu, vecs = mp.eig(M)
        best = None
        for i, mui in enumerate(mu):
            if abs(mp.im(mui)) > mp.mpf(10) ** (-(mp.mp.dps // 3)) * abs(mui) or abs(mui) == 0:
                continue
            E = -1 / mp.re(mui)
            c = [mp.re(vecs[r, i]) for r in range(m)]
            if c[m - 1] == 0:
                continue
            c = [cj / c[m - 1] for cj in c]
            Q = c[n + 1:]
            qv = [_poly(Q, u) for u in us]
            if all(q > 0 for q in qv) or all(q < 0 for q in qv):
                if best is None or abs(E) < abs(best[1]):
                    best = (c, E)
        if best is None:
            raise RuntimeError("no pole-free solution on the reference")
        c, E = best
        return c[:2 * n + 1] + [E]

    def _refine(self, la, lb, sgn, P, Q):
        """argmax of sgn*e on [exp(la), exp(lb)] by golden-section in log x."""
        g = (mp.sqrt(5) - 1) / 2
        c = lb - g * (lb - la)
        d = la + g * (lb - la)
        fc = sgn * self.err(mp.exp(c), P, Q)
        fd = sgn * self.err(mp.exp(d), P, Q)
        for _ in range(60):
            if fc > fd:
                lb, d, fd = d, c, fc
                c = lb - g * (lb - la)
                fc = sgn * self.err(mp.exp(c), P, Q)
            else:
                la, c, fc = c, d, fd
                d = la + g * (lb - la)
                fd = sgn * self.err(mp.exp(d), P, Q)
            if lb - la < mp.mpf(10) ** (-12):
                break
        return (c, fc) if fc > fd else (d, fd)

    def exchange(self, xs, P, Q, per=24):
        """New reference: alternating extrema of e found on a dense log grid.

        The grid holds the old reference plus ``per`` points per reference
        gap.  Each maximal run of equal sign contributes its largest |e|
        (refined by golden section between the neighbouring grid points).
        Surplus extrema are pruned while keeping the alternation and the
        global maximum: the smallest one goes, together with its smaller
        neighbour unless it sits at an end.
        """
        m = len(xs)
        lx = [mp.log(x) for x in xs]
        grid = []
        for k in range(m - 1):
            for j in range(per):
                grid.append(lx[k] + (lx[k + 1] - lx[k]) * j / per)
        grid.append(lx[-1])
        ev = [self.err(mp.exp(t), P, Q) for t in grid]
        runs = []  # (sign, index of max |e| in run)
        for i, e in enumerate(ev):
            sg = 1 if e > 0 else -1
            if runs and runs[-1][0] == sg:
                if abs(e) > abs(ev[runs[-1][1]]):
                    runs[-1] = (sg, i)
            else:
                runs.append((sg, i))
        ext = []
        for sg, i in runs:
            la = grid[max(i - 1, 0)]
            lb = grid[min(i + 1, len(grid) - 1)]
            t, v = self._refine(la, lb, sg, P, Q)
            if v < sg * ev[i]:
                t, v = grid[i], sg * ev[i]
            ext.append([t, v, sg])
        while len(ext) > m:
            i = min(range(len(ext)), key=lambda j: ext[j][1])
            if i == 0 or i == len(ext) - 1:
                ext.pop(i)
            else:
                j = i - 1 if ext[i - 1][1] < ext[i + 1][1] else i + 1
                for k in sorted((i, j), reverse=True):
                    ext.pop(k)
        if len(ext) < m:
            raise RuntimeError("error curve has fewer alternations than the reference needs")
        return [mp.exp(t) for t, _, _ in ext], [v for _, v, _ in ext]


def remez_relative(p, n, lo, hi, dps=None, maxiter=60, rtol=1e-9) -> Rational:
    """Best type-(n, n) approximation of x^p on [lo, hi] in relative error."""
    import math

    if not (0 < lo < hi):
        raise ValueError("need 0 < lo < hi")
    if n < 0:
        raise ValueError("need n >= 0")
    if dps is None:
        dps = int(40 + 1.2 * n * math.log10(hi / lo))
    with mp.workdps(dps):
        R = _Remez(p, n, lo, hi)
        if n == 0:
            # best constant: c * x^(-p) levelled at the two end points
            a, b = R.f(R.lo), R.f(R.hi)
            c = 2 * a * b / (a + b)
            d = abs(b - a) / (a + b)
            return Rational(float(p), 0, float(lo), float(hi), float(c), [], [], float(d), 0)
        xs = R.initial_reference()
        sol = None
        it = 0
        for it in range(1, maxiter + 1):
            P, Q, E = sol = R.solve_reference(xs, sol)
            xs, vals = R.exchange(xs, P, Q)
            emax = max(vals)
            if (emax - abs(E)) / emax < rtol:
                break
        else:
            raise RuntimeError(f"Remez did not level for p={p} n={n} on [{lo},{hi}]")
        P, Q, E = R.solve_reference(xs, sol)
        # partial fractions from the roots of Q (highest degree first for polyroots)
        roots = mp.polyroots(list(reversed(Q)), maxsteps=400, extraprec=4 * dps)
        alpha, beta = [], []
        dQ = [j * Q[j] for j in range(1, n + 1)]
        for ui in roots:
            if abs(mp.im(ui)) > mp.mpf(10) ** (-(dps // 3)) * abs(ui) or mp.re(ui) >= 0:
                raise RuntimeError(f"denominator root {ui} is not real negative")
            ur = mp.re(ui)
            alpha.append(R.s * _poly(P, ur) / _poly(dQ, ur))
            beta.append(-R.s * ur)
        order = sorted(range(n), key=lambda i: beta[i])
        alpha = [float(alpha[i]) for i in order]
        beta = [float(beta[i]) for i in order]
        alpha0 = float(P[n])
        # levelled error measured on the final extrema
        vals = [abs(R.err(x, P, Q)) for x in xs]
        delta = float(max(vals))
        return Rational(float(p), n, float(lo), float(hi), alpha0, alpha, beta, delta, it)


def _cache_name(p, n, lo, hi):
    return f"rational_p{p:+.4f}_n{n}_lo{lo:.6e}_hi{hi:.6e}.json"


def rational_coefficients(p, n, lo, hi, cache=True) -> Rational:
    """Cached coefficients for x^p on [lo, hi] with n poles."""
    path = os.path.join(_DATA_DIR, _cache_name(p, n, lo, hi))
    if cache and os.path.exists(path):
        with open(path) as fh:
            return Rational.from_json(fh.read())
    r = remez_relative(p, n, lo, hi)
    if cache:
        os.makedirs(_DATA_DIR, exist_ok=True)
        with open(path, "w") as fh:
            fh.write(r.to_json())
    return r
