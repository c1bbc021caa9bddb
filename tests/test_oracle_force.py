"""Pins of the pseudofermion-force oracle (CPU, 4^4).

* central finite differences of the dense rational action along random
  algebra directions T at single links (even and odd sites, every direction,
  a time-boundary link) equal i Tr(T F) (the derivative definition itself,
  evaluated by a route that never forms M);
* gauge covariance: F[U^G, G phi] = G(n) F[U, phi] G(n)^dagger;
* F is traceless and anti-Hermitian.
"""

import numpy as np
import pytest

import synth
from oracle import dirac, force, lattice
from synth.make_rational import rational_for


def _gauss(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


def _algebra(rng):
    H = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    H = 0.5 * (H + H.conj().T)
    return H - np.trace(H) / 3 * np.eye(3)


def _expi(eps, T):
    w, V = np.linalg.eigh(T)
    return (V * np.exp(1j * eps * w)) @ V.conj().T


@pytest.fixture(scope="module")
def setup():
    L = (4, 4, 4, 4)
    m = 0.1
    U = synth.gauge_field(L, 0.5, 41)
    r = rational_for(1, -0.25)
    rng = np.random.default_rng(42)
    phi = _gauss(rng, (2, 3, 128))
    F = force.force(U, m, r.alpha, r.beta, phi)
    return L, m, U, r, phi, F


@pytest.mark.parametrize("site,mu", [((0, 0, 0, 0), 0), ((1, 0, 0, 0), 1), ((1, 2, 3, 1), 2),
                                     ((2, 1, 0, 3), 3), ((3, 0, 1, 3), 3), ((0, 1, 1, 2), 1)])
def test_force_is_derivative_of_action(setup, site, mu):
    L, m, U, r, phi, F = setup
    x, y, z, t = site
    rng = np.random.default_rng(100 + sum(site) + mu)
    T = _algebra(rng)
    eps = 1e-5
    S = []
    for sgn in (1, -1):
        Up = U.copy()
        Up[t, z, y, x, mu] = _expi(sgn * eps, T) @ U[t, z, y, x, mu]
        S.append(force.dense_rational_action(Up, m, r.alpha0, r.alpha, r.beta, phi))
    fd = (S[0] - S[1]) / (2 * eps)
    want = (1j * np.trace(T @ F[t, z, y, x, mu])).real
    assert abs(fd - want) <= 1e-6 * max(1.0, abs(want))


def test_force_gauge_covariance(setup):
    L, m, U, r, phi, F = setup
    G = synth.gauge_field(L, 1.0, 43)[..., 0, :, :]       # random SU(3) per site
    Ug = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=lattice.AXIS[mu] - 1)    # G(n + mu); matrix fields have one more trailing axis
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.swapaxes(Gf.conj(), -1, -2)
    # phi on even sites transforms with G(n): rebuild through the full field
    full = lattice.embed(phi, L, 0)
    fullg = np.einsum("...ab,...b->...a", G, full)
    phig = lattice.restrict(fullg, L, 0)
    Fg = force.force(Ug, m, r.alpha, r.beta, phig)
    want = G[..., None, :, :] @ F @ np.swapaxes(G.conj(), -1, -2)[..., None, :, :]
    assert np.abs(Fg - want).max() <= 1e-10 * np.abs(F).max()


def test_force_is_traceless_antihermitian(setup):
    F = setup[-1]
    assert np.abs(F + np.swapaxes(F.conj(), -1, -2)).max() <= 1e-14 * np.abs(F).max()
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() <= 1e-14 * np.abs(F).max()
