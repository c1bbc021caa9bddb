"""Pseudofermion force (oracle; test infrastructure only).

The action of one pseudofermion, S = phi^dagger r(A) phi with
r(x) = alpha0 + sum_i alpha_i / (x + beta_i) (Eq. system_r), depends on the
links through A = m^2 - D_eo D_oe (Eq. stag).  For the variation of one link
U_mu(n) -> exp(i eps T) U_mu(n) with T Hermitian and traceless (the algebra
of the momenta of Sec. 2.1),

    dS/deps = i Tr(T F_mu(n)),   F_mu(n) = TA(U_mu(n) M_mu(n)),
    TA(X) = (X - X^dagger)/2 - Tr(X - X^dagger)/6,
    M_mu(n) = sum_i alpha_i s_mu(n) *  y_i(n+mu) x_i(n)^dagger    (n even)
                                    - x_i(n+mu) y_i(n)^dagger    (n odd)

with x_i = (A + beta_i)^-1 phi on the even sites, y_i = D_oe x_i on the odd
sites and s_mu(n) = eta_mu(n) times the time-boundary sign of the hop from n
to n+mu.  Derivation: delta S = -sum_i alpha_i x_i^dagger (delta A) x_i,
delta A = -(delta D_eo) D_oe - D_eo (delta D_oe) and D_eo^dagger = -D_oe, so
delta S = sum_i alpha_i [x_i^dagger (delta D_eo) y_i - y_i^dagger (delta D_oe) x_i];
the link enters D at n (forward hop, +s U / 2) and at n+mu (backward hop,
-s U^dagger / 2), and the two terms are complex conjugates.
"""

from __future__ import annotations

import numpy as np

from . import dirac, lattice


def traceless_antihermitian(X):
    """TA(X) on the last two axes."""
    Y = 0.5 * (X - np.swapaxes(X.conj(), -1, -2))
    tr = np.trace(Y, axis1=-2, axis2=-1) / 3.0
    return Y - tr[..., None, None] * np.eye(3)


def hop_sign(L, mu, t_bc):
    """eta_mu(n) times the boundary sign of the hop n -> n + mu, shape (Lt, Lz, Ly, Lx)."""
    s = lattice.eta(L, mu).astype(np.float64)
    if mu == 3 and t_bc != 1:
        s = s.copy()
        s[L[3] - 1] *= t_bc
    return s


def force_from_solutions(U, x, y, alpha, t_bc=-1):
    """F_mu(n) for shifted solutions x[i] (even, [npole, 3, V/2]) and
    y[i] = D_oe x[i] (odd); returns complex128 [Lt, Lz, Ly, Lx, 4, 3, 3]."""
    L = dirac.lattice_of(U)
    X = lattice.embed(x, L, 0)          # [npole, Lt, Lz, Ly, Lx, 3], zero on odd sites
    Y = lattice.embed(y, L, 1)          # zero on even sites
    par = lattice.parity_field(L)
    F = np.zeros(U.shape, dtype=np.complex128)
    a = np.asarray(alpha, dtype=np.float64)
    for mu in range(4):
        ax = lattice.AXIS[mu]
        Xf = np.roll(X, -1, axis=ax)    # x(n + mu)
        Yf = np.roll(Y, -1, axis=ax)    # y(n + mu)
        even = np.einsum("i,i...a,i...b->...ab", a, Yf, X.conj())
        odd = -np.einsum("i,i...a,i...b->...ab", a, Xf, Y.conj())
        M = np.where((par == 0)[..., None, None], even, odd)
        M = M * hop_sign(L, mu, t_bc)[..., None, None]
        F[..., mu, :, :] = traceless_antihermitian(U[..., mu, :, :] @ M)
    return F


def force(U, m, alpha, beta, phi, t_bc=-1, dense=None):
    """Force of S = sum_r phi_r^dagger r(A) phi_r (phi [nrhs, 3, V/2]) with the
    shifted systems solved densely (tiny lattices)."""
    Ad = dirac.dense_A(U, m, t_bc) if dense is None else dense
    n = Ad.shape[0]
    F = np.zeros(U.shape, dtype=np.complex128)
    for p in np.asarray(phi).reshape(-1, 3, n // 3):
        x = np.stack([np.linalg.solve(Ad + b * np.eye(n), p.reshape(-1)).reshape(3, -1)
                      for b in beta])
        y = dirac.dslash(U, x, 1, t_bc)
        F += force_from_solutions(U, x, y, alpha, t_bc)
    return F


def dense_rational_action(U, m, alpha0, alpha, beta, phi, t_bc=-1):
    """sum_r Re <phi_r, r(A) phi_r> through dense solves (tiny lattices)."""
    Ad = dirac.dense_A(U, m, t_bc)
    n = Ad.shape[0]
    S = 0.0
    for p in np.asarray(phi).reshape(-1, n):
        y = alpha0 * p
        for a, b in zip(alpha, beta):
            y = y + a * np.linalg.solve(Ad + b * np.eye(n), p)
        S += float(np.real(np.vdot(p, y)))
    return S
