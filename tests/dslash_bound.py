"""Rounding bound of the FP32 hopping term (test helper): each output element
is a sum of 24 products of FP32-rounded links and vectors, so its error is at
most a few units of 2^-24 times 1/2 sum over the 8 hops of |U| |psi|."""

import numpy as np

from oracle import dirac, lattice


def abs_scale(U, v, out_par):
    """1/2 sum over the 8 hops of |U| |psi| per output element (error scale)."""
    L = dirac.lattice_of(U)
    full = np.abs(lattice.embed(v, L, 1 - out_par))
    A = np.abs(U)
    out = np.zeros(full.shape)
    for mu in range(4):
        ax = lattice.AXIS[mu]
        out += np.einsum("...ij,...j->...i", A[..., mu, :, :], np.roll(full, -1, axis=ax))
        Ab = np.roll(A[..., mu, :, :], 1, axis=ax - 1)
        out += np.einsum("...ji,...j->...i", Ab, np.roll(full, 1, axis=ax))
    return 0.5 * lattice.restrict(out, L, out_par)
