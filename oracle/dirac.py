"""Staggered operator (oracle; test infrastructure only).

Eq. stag with lattice spacing a = 1:

    (M psi)(n) = m psi(n) + 1/2 sum_mu eta_mu(n) [ U_mu(n) psi(n+mu)
                                                  - U_mu(n-mu)^dagger psi(n-mu) ]

D is the hopping (second) term.  It is anti-Hermitian, so
M^dagger M = m^2 - D^2, and since D only connects opposite parities its
restriction to even sites (even/odd preconditioning, Sec. 2.1) is
A = m^2 - D_eo D_oe, with D_eo the block mapping odd to even sites.

Gauge fields are ``complex128[Lt][Lz][Ly][Lx][mu][row][col]``; a hop that
wraps around the time direction is multiplied by ``t_bc``.
"""

from __future__ import annotations

import numpy as np

from . import lattice as lat


def hopping(U, psi, t_bc=-1):
    """D psi on the full lattice; psi is [..., Lt, Lz, Ly, Lx, 3]."""
    Lt, Lz, Ly, Lx = U.shape[:4]
    L = (Lx, Ly, Lz, Lt)
    out = np.zeros(np.broadcast_shapes(psi.shape), dtype=np.complex128)
    for mu in range(4):
        ax = lat.AXIS[mu]
        fwd = np.roll(psi, -1, axis=ax)        # psi(n + mu)
        bwd = np.roll(psi, +1, axis=ax)        # psi(n - mu)
        if mu == 3 and t_bc != 1:
            fwd = fwd.copy()
            bwd = bwd.copy()
            fwd[..., Lt - 1, :, :, :, :] *= t_bc   # hop from t = Lt-1 to t = 0
            bwd[..., 0, :, :, :, :] *= t_bc        # hop from t = 0 to t = Lt-1
        Umu = U[..., mu, :, :]
        # U_mu(n - mu); a link array has one more trailing axis than a field
        Uback = np.roll(Umu, +1, axis=lat.AXIS[mu] - 1)
        term = np.einsum("...ij,...j->...i", Umu, fwd) \
            - np.einsum("...ji,...j->...i", np.conj(Uback), bwd)
        out += lat.eta(L, mu)[..., None] * term
    return 0.5 * out


def lattice_of(U):
    Lt, Lz, Ly, Lx = U.shape[:4]
    return (Lx, Ly, Lz, Lt)


def dslash(U, v, out_parity, t_bc=-1):
    """D restricted to (out_parity <- 1 - out_parity) on eo vectors [..., 3, V/2].

    out_parity = 0 gives D_eo (odd input, even output), 1 gives D_oe.
    """
    L = lattice_of(U)
    full = lat.embed(v, L, 1 - out_parity)
    return lat.restrict(hopping(U, full, t_bc), L, out_parity)


def mdagm(U, m, v, t_bc=-1):
    """A v = m^2 v - D_eo D_oe v on even-site vectors [..., 3, V/2]."""
    return m * m * v - dslash(U, dslash(U, v, 1, t_bc), 0, t_bc)


def full_matrix_M(U, m, t_bc=-1):
    """Dense M on the full lattice (tiny lattices only), lex-site-major, colour-minor."""
    Lt, Lz, Ly, Lx = U.shape[:4]
    n = Lt * Lz * Ly * Lx * 3
    eye = np.eye(n, dtype=np.complex128).reshape(n, Lt, Lz, Ly, Lx, 3)
    cols = m * eye + hopping(U, eye, t_bc)
    return cols.reshape(n, n).T


def dense_A(U, m, t_bc=-1):
    """Dense even-site A (tiny lattices only); basis index c*V/2 + eo."""
    L = lattice_of(U)
    Vh = L[0] * L[1] * L[2] * L[3] // 2
    n = 3 * Vh
    eye = np.eye(n, dtype=np.complex128).reshape(n, 3, Vh)
    return mdagm(U, m, eye, t_bc).reshape(n, n).T
