"""Lattice geometry (oracle; test infrastructure only).

Conventions (Sec. 2, Eq. stag and the definition of eta below it):

* ``L = (Lx, Ly, Lz, Lt)``, directions mu = 0, 1, 2, 3 are x, y, z, t
  (the paper's nu = 1..4).
* lexicographic site index ``lex = x + Lx*(y + Ly*(z + Lz*t))``;
  parity ``(x + y + z + t) mod 2`` (0 = even); within a parity the sites are
  ordered by ``eo = lex // 2`` (a bijection because Lx is even).
* staggered phases ``eta_0 = 1``, ``eta_1 = (-1)^x``, ``eta_2 = (-1)^(x+y)``,
  ``eta_3 = (-1)^(x+y+z)``.
* fermion boundary: periodic in space; in time a hop that wraps around the
  lattice carries the sign ``t_bc`` (-1 antiperiodic, +1 periodic).

Field arrays in this oracle are full-lattice ``[..., Lt, Lz, Ly, Lx, 3]``;
even/odd vectors are ``[..., 3, V/2]``.
"""

from __future__ import annotations

import numpy as np

# array axis of a full-lattice field [..., Lt, Lz, Ly, Lx, colour] that
# carries direction mu, counted from the end
AXIS = {0: -2, 1: -3, 2: -4, 3: -5}


def check_dims(L):
    if len(L) != 4 or any(int(l) < 2 or int(l) % 2 for l in L):
        raise ValueError(f"extents must be four even numbers >= 2, got {L}")
    return tuple(int(l) for l in L)


def coordinates(L):
    """x, y, z, t as int64 arrays of shape (Lt, Lz, Ly, Lx)."""
    Lx, Ly, Lz, Lt = check_dims(L)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly),
                             np.arange(Lx), indexing="ij")
    return x, y, z, t


def lex_index(L, x, y, z, t):
    Lx, Ly, Lz, Lt = check_dims(L)
    return x + Lx * (y + Ly * (z + Lz * t))


def parity_field(L):
    x, y, z, t = coordinates(L)
    return (x + y + z + t) % 2


def eo_coordinates(L, parity):
    """Coordinates (x, y, z, t) of the sites of one parity, in eo order."""
    L = check_dims(L)
    x, y, z, t = (c.reshape(-1) for c in coordinates(L))
    lex = lex_index(L, x, y, z, t)
    sel = (x + y + z + t) % 2 == parity
    eo = lex[sel] // 2
    order = np.argsort(eo, kind="stable")
    assert np.array_equal(eo[order], np.arange(eo.size)), "lex//2 is not a bijection"
    return x[sel][order], y[sel][order], z[sel][order], t[sel][order]


def eta(L, mu):
    x, y, z, t = coordinates(L)
    if mu == 0:
        return np.ones_like(x)
    if mu == 1:
        return (-1) ** x
    if mu == 2:
        return (-1) ** (x + y)
    return (-1) ** (x + y + z)


def neighbor_table(L, parity):
    """int64[V/2][8]: eo index of n+mu (columns 0..3) and n-mu (4..7)."""
    L = check_dims(L)
    x, y, z, t = eo_coordinates(L, parity)
    c = [x, y, z, t]
    out = np.empty((x.size, 8), dtype=np.int64)
    for mu in range(4):
        for k, step in ((mu, +1), (4 + mu, -1)):
            cc = list(c)
            cc[mu] = (c[mu] + step) % L[mu]
            out[:, k] = lex_index(L, *cc) // 2
    return out


def boundary_sign_table(L, parity, t_bc):
    """int64[V/2][8]: the time-boundary sign carried by each of the 8 hops."""
    L = check_dims(L)
    x, y, z, t = eo_coordinates(L, parity)
    out = np.ones((x.size, 8), dtype=np.int64)
    out[:, 3] = np.where(t == L[3] - 1, t_bc, 1)
    out[:, 7] = np.where(t == 0, t_bc, 1)
    return out


def embed(v, L, parity):
    """Even/odd vector [..., 3, V/2] -> full-lattice field, zero elsewhere."""
    L = check_dims(L)
    Lx, Ly, Lz, Lt = L
    x, y, z, t = eo_coordinates(L, parity)
    lead = v.shape[:-2]
    full = np.zeros(lead + (Lt, Lz, Ly, Lx, 3), dtype=np.result_type(v, np.complex128))
    full[..., t, z, y, x, :] = np.swapaxes(v, -1, -2)
    return full


def restrict(psi, L, parity):
    """Full-lattice field -> even/odd vector [..., 3, V/2] of one parity."""
    L = check_dims(L)
    x, y, z, t = eo_coordinates(L, parity)
    return np.swapaxes(psi[..., t, z, y, x, :], -1, -2)
