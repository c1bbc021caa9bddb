"""Pseudofermion field and action (oracle; test infrastructure only).

Sec. 2.1, the Phi algorithm: from a complex Gaussian vector R the
pseudofermion field is set to phi = M^dagger R, which makes its distribution
proportional to exp(-phi^dagger (M^dagger M)^{-1} phi).  With even/odd
preconditioning only the even sites of phi enter, and since D^dagger = -D,

    phi_e = (M^dagger R)_e = m R_e - D_eo R_o,

whose covariance is m^2 + D_eo D_eo^dagger = m^2 - D_eo D_oe = A.

For the rooted (RHMC) action each pseudofermion carries A^{-1/4}
(Eq. system_r with N_f = 2 and two pseudofermions): the action is
phi^dagger r_-(A) phi with r_- ~ x^{-1/4}, and the heat bath that makes it
Gaussian is phi = r_h(A) R with r_h ~ x^{+1/8}, so that at the start of a
trajectory the action equals R^dagger R up to the two approximation errors.
"""

from __future__ import annotations

import numpy as np

from . import dirac, rational


def phi_even(U, m, R_even, R_odd, t_bc=-1):
    """phi_e = m R_e - D_eo R_o on even-site vectors [..., 3, V/2]."""
    return m * R_even - dirac.dslash(U, R_odd, 0, t_bc)


def action(apply_A, phi, alpha0, alpha, beta, tol=1e-12):
    """Re <phi, r(A) phi> with r(A) phi from the multi-shift solver."""
    y, _, info = rational.rational_apply(apply_A, phi, alpha0, alpha, beta, tol=tol)
    return float(np.real(np.vdot(phi, y))), info


def dense_action(Adense, phi, fn):
    """Re <phi, fn(A) phi> through the eigen-decomposition (tiny lattices)."""
    return float(np.real(np.vdot(phi, rational.dense_function_apply(Adense, phi, fn))))
