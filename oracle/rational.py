"""Rational functions of A (oracle; test infrastructure only).

Sec. 2.1 (Eq. system_r): the rooted power of M^dagger M is replaced by a
rational function in partial fractions,

    r(x) = alpha0 + sum_i alpha_i / (x + beta_i),     beta_i > 0,

so that r(A) b = alpha0 b + sum_i alpha_i (A + beta_i)^-1 b needs exactly the
shifted systems of Eq. shifted.  The coefficients are inputs here; this module
only applies them, either through the multi-shift solver or exactly through a
dense eigen-decomposition on tiny lattices.
"""

from __future__ import annotations

import numpy as np

from . import solvers


def rational_apply(apply_A, b, alpha0, alpha, beta, tol=1e-10, maxiter=100000):
    """alpha0 b + sum_i alpha_i x_i, x_i from the multi-shift solver."""
    x, info = solvers.multishift_cg(apply_A, b, beta, tol=tol, maxiter=maxiter)
    y = alpha0 * b.astype(np.complex128)
    for i, a in enumerate(alpha):
        y = y + a * x[i]
    return y, x, info


def scalar_rational(x, alpha0, alpha, beta):
    y = np.full(np.shape(x), alpha0, dtype=np.float64)
    for a, c in zip(alpha, beta):
        y = y + a / (np.asarray(x, dtype=np.float64) + c)
    return y


def dense_function_apply(Adense, b, fn):
    """fn(A) b through the eigen-decomposition of the Hermitian matrix A."""
    w, V = np.linalg.eigh(Adense)
    bb = b.reshape(-1)
    return (V @ (fn(w) * (V.conj().T @ bb))).reshape(b.shape)
