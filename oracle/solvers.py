"""Krylov solvers (oracle; test infrastructure only).

Sec. 4.3: the systems (A + sigma_i) x_i = b (Eq. shifted) are solved by CG,
the method of choice for staggered fermions; the shifted solver obtains every
x_i from the Krylov space of the smallest shift, which forces a zero starting
guess and rules out restarts.  The stopping residual is relative,
||b - (A + sigma_i) x_i|| / ||b|| <= tol, for each shift.

``multishift_cg`` keeps the shifted residuals collinear with the base one,
r_i = zeta_i r, which fixes the shifted step lengths from the base CG scalars
alone (three-term recurrence of CG, requiring collinearity at every step):

    zeta_i' = zeta_i zeta_i^- a^- / (zeta_i^- a^- (1 + a s_i) + a b^- (zeta_i^- - zeta_i))
    a_i = a zeta_i' / zeta_i,           b_i = b (zeta_i' / zeta_i)^2
    x_i += a_i p_i,                     p_i = zeta_i' r' + b_i p_i

where a, b are the base CG's alpha and beta, '-' marks the previous step and
s_i = sigma_i - sigma_0 >= 0.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def vdot(u, v):
    return np.vdot(u.reshape(-1), v.reshape(-1))


def norm(u):
    return float(np.sqrt(np.real(vdot(u, u))))


@dataclass
class SolveInfo:
    iterations: int = 0
    converged: bool = False
    shift_iterations: list = field(default_factory=list)
    history: list = field(default_factory=list)


def cg(apply_A, b, sigma=0.0, tol=1e-10, maxiter=100000, x0=None):
    """Plain CG for (A + sigma) x = b, relative residual tol."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - (apply_A(x) + sigma * x) if x0 is not None else b.copy()
    p = r.copy()
    rr = np.real(vdot(r, r))
    bn = norm(b)
    info = SolveInfo()
    for k in range(maxiter):
        if np.sqrt(rr) <= tol * bn:
            info.converged = True
            break
        Ap = apply_A(p) + sigma * p
        a = rr / np.real(vdot(p, Ap))
        x = x + a * p
        r = r - a * Ap
        rr_new = np.real(vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        info.iterations = k + 1
    else:
        info.converged = np.sqrt(rr) <= tol * bn
    return x, info


def multishift_cg(apply_A, b, shifts, tol=1e-10, maxiter=100000):
    """All x_i = (A + shifts[i])^-1 b from the Krylov space of min(shifts)."""
    shifts = np.asarray(shifts, dtype=np.float64)
    ns = shifts.size
    s0 = float(shifts.min())
    off = shifts - s0
    bn = norm(b)
    x = np.zeros((ns,) + b.shape, dtype=np.complex128)
    p_s = np.repeat(b[None].astype(np.complex128), ns, axis=0)
    r = b.astype(np.complex128).copy()
    p = r.copy()
    rr = np.real(vdot(r, r))
    zeta = np.ones(ns)
    zeta_prev = np.ones(ns)
    a_prev, b_prev = 1.0, 0.0
    active = np.ones(ns, dtype=bool)
    info = SolveInfo(shift_iterations=[0] * ns)
    k = 0
    while active.any() and k < maxiter:
        Ap = apply_A(p) + s0 * p
        a = rr / np.real(vdot(p, Ap))
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            zeta_upd = zeta * zeta_prev * a_prev / (
                zeta_prev * a_prev * (1.0 + a * off) + a * b_prev * (zeta_prev - zeta))
        zeta_new = np.where(active, zeta_upd, zeta)
        a_s = a * zeta_new / zeta
        for i in np.nonzero(active)[0]:
            x[i] += a_s[i] * p_s[i]
        r = r - a * Ap
        rr_new = np.real(vdot(r, r))
        bet = rr_new / rr
        p = r + bet * p
        b_s = bet * (zeta_new / zeta) ** 2
        for i in np.nonzero(active)[0]:
            p_s[i] = zeta_new[i] * r + b_s[i] * p_s[i]
        zeta_prev, zeta = zeta, zeta_new
        a_prev, b_prev, rr = a, bet, rr_new
        k += 1
        done = np.abs(zeta) * np.sqrt(rr) <= tol * bn
        for i in np.nonzero(active & done)[0]:
            info.shift_iterations[i] = k
        active &= ~done
        info.history.append(np.sqrt(rr) / bn)
    info.iterations = k
    info.converged = not active.any()
    for i in np.nonzero(active)[0]:
        info.shift_iterations[i] = k
    return x, info


def true_residual(apply_A, b, x, sigma):
    """||b - (A + sigma) x|| / ||b|| computed from scratch in FP64."""
    return norm(b - apply_A(x) - sigma * x) / norm(b)


def dense_solve(Adense, b, sigma):
    n = Adense.shape[0]
    return np.linalg.solve(Adense + sigma * np.eye(n), b.reshape(-1)).reshape(b.shape)
