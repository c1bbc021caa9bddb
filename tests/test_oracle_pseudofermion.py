"""Pins of the pseudofermion oracle (CPU).

* phi_e = (M^dagger R)_e against the dense full-lattice M built column by
  column (a different route through the operator than the even/odd blocks);
* S(phi = A^{1/2} R) = R^dagger R exactly for the unrooted action
  phi^dagger A^{-1} phi, by dense linear algebra;
* the covariance of phi_e is A: the sample mean of phi^dagger A^{-1} phi over
  Gaussian R is 3 V/2 (chi-square with 3 V/2 complex degrees of freedom);
* rooted action with the workload rationals: phi = r_h(A) R, S = phi^dagger
  r_-(A) phi equals R^dagger R within the two minimax errors (and the solver
  tolerance), and matches the dense evaluation of the same rationals.
"""

import numpy as np
import pytest

import synth
from oracle import dirac, lattice, pseudofermion, rational
from synth.make_rational import rational_for


def _gauss(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


@pytest.fixture(scope="module")
def small():
    L = (4, 4, 4, 4)
    m = 0.1
    U = synth.gauge_field(L, 0.5, 31)
    return L, m, U, dirac.dense_A(U, m)


def test_phi_is_m_dagger_R_on_even_sites(small):
    L, m, U, _ = small
    rng = np.random.default_rng(5)
    V = L[0] * L[1] * L[2] * L[3]
    R = _gauss(rng, (L[3], L[2], L[1], L[0], 3))
    M = dirac.full_matrix_M(U, m)
    full = (M.conj().T @ R.reshape(-1)).reshape(R.shape)
    want = lattice.restrict(full, L, 0)
    Re = lattice.restrict(R, L, 0)
    Ro = lattice.restrict(R, L, 1)
    got = pseudofermion.phi_even(U, m, Re, Ro)
    assert got.shape == (3, V // 2)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_unrooted_action_of_sqrt_field_is_gaussian_norm(small):
    L, m, U, Ad = small
    rng = np.random.default_rng(6)
    R = _gauss(rng, (3, Ad.shape[0] // 3))
    phi = rational.dense_function_apply(Ad, R, np.sqrt)
    S = pseudofermion.dense_action(Ad, phi, lambda w: 1.0 / w)
    assert abs(S - np.vdot(R, R).real) <= 1e-11 * np.vdot(R, R).real


def test_phi_covariance_is_A(small):
    """E[phi^dagger A^-1 phi] = 3 V/2 for phi_e = m R_e - D_eo R_o."""
    L, m, U, Ad = small
    rng = np.random.default_rng(7)
    Ainv = np.linalg.inv(Ad)
    n = Ad.shape[0]
    vals = []
    for _ in range(400):
        Re = _gauss(rng, (3, n // 3))
        Ro = _gauss(rng, (3, n // 3))
        phi = pseudofermion.phi_even(U, m, Re, Ro).reshape(-1)
        vals.append(np.vdot(phi, Ainv @ phi).real)
    # chi-square with n complex dof: mean n, standard deviation sqrt(n)
    mean = np.mean(vals)
    assert abs(mean - n) <= 5 * np.sqrt(n) / np.sqrt(len(vals))


@pytest.mark.parametrize("cfg", [1, 2])
def test_rooted_heatbath_action_reproduces_gaussian_norm(cfg):
    c = synth.CONFIGS[cfg]
    L = (4, 4, 4, 4)
    m = c["m"]
    U = synth.gauge_field(L, c["eps"], 900 + cfg)
    Ad = dirac.dense_A(U, m)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    rh = rational_for(cfg, c["hb_power"])
    rm = rational_for(cfg, -0.25)
    rng = np.random.default_rng(8)
    R = _gauss(rng, (3, Ad.shape[0] // 3))
    phi, _, info = rational.rational_apply(A, R, rh.alpha0, rh.alpha, rh.beta, tol=1e-13)
    assert info.converged
    S, info = pseudofermion.action(A, phi, rm.alpha0, rm.alpha, rm.beta, tol=1e-13)
    assert info.converged
    R2 = np.vdot(R, R).real
    # |r_h(x)^2 r_-(x) - 1| <= (1 + d_h)^2 (1 + d_-) - 1 on the spectrum
    bound = (1 + rh.delta) ** 2 * (1 + rm.delta) - 1
    assert abs(S - R2) <= (bound + 1e-10) * R2
    # the same rationals evaluated densely
    fh = lambda w: rational.scalar_rational(w, rh.alpha0, rh.alpha, rh.beta)  # noqa: E731
    fm = lambda w: rational.scalar_rational(w, rm.alpha0, rm.alpha, rm.beta)  # noqa: E731
    phid = rational.dense_function_apply(Ad, R, fh)
    Sd = pseudofermion.dense_action(Ad, phid, fm)
    assert abs(S - Sd) <= 1e-10 * R2
