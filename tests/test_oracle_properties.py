"""Randomised properties of the oracle's operator (hypothesis): the
consequences of Eq. stag that must hold for every lattice shape, boundary,
gauge field and mass, checked on random small lattices and seeds beyond the
fixed cases of test_oracle_dirac.py:

* anti-Hermiticity of the hopping term between parities,
  <u_e, D_eo v_o> = -<D_oe u_e, v_o>;
* gauge covariance, D[U^G](G psi) = G D[U] psi;
* A = m^2 - D_eo D_oe is Hermitian with Rayleigh quotients in [m^2, 16 + m^2]
  (||D|| <= 4).
"""

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import synth
from oracle import dirac, lattice

extent = st.sampled_from([2, 4, 6])
shapes = st.tuples(extent, extent, extent, extent)
seeds = st.integers(min_value=0, max_value=2**31 - 1)
roughness = st.floats(min_value=0.0, max_value=3.0)
boundary = st.sampled_from([-1, 1])
SETTINGS = dict(max_examples=20, deadline=None, suppress_health_check=[HealthCheck.too_slow])


def _vec(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


@settings(**SETTINGS)
@given(L=shapes, seed=seeds, eps=roughness, t_bc=boundary)
def test_hopping_anti_hermitian(L, seed, eps, t_bc):
    U = synth.gauge_field(L, eps, seed, workers=1)
    rng = np.random.default_rng(seed + 1)
    Vh = synth.even_volume(L)
    u, v = _vec(rng, (3, Vh)), _vec(rng, (3, Vh))
    lhs = np.vdot(u, dirac.dslash(U, v, 0, t_bc))
    rhs = -np.vdot(dirac.dslash(U, u, 1, t_bc), v)
    assert abs(lhs - rhs) <= 1e-13 * (1.0 + abs(lhs))


@settings(**SETTINGS)
@given(L=shapes, seed=seeds, eps=roughness, t_bc=boundary)
def test_gauge_covariance(L, seed, eps, t_bc):
    U = synth.gauge_field(L, eps, seed, workers=1)
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(seed + 2)
    G = synth.random_su3((Lt, Lz, Ly, Lx), rng, 2.0)
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=lattice.AXIS[mu] - 1)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gf, -1, -2))
    Vh = synth.even_volume(L)
    v = _vec(rng, (3, Vh))

    def rot(w, par):
        return lattice.restrict(np.einsum("...ij,...j->...i", G, lattice.embed(w, L, par)), L, par)

    for par in (0, 1):
        lhs = dirac.dslash(UG, rot(v, 1 - par), par, t_bc)
        rhs = rot(dirac.dslash(U, v, par, t_bc), par)
        np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@settings(**SETTINGS)
@given(L=shapes, seed=seeds, eps=roughness, m=st.floats(min_value=0.0, max_value=1.0), t_bc=boundary)
def test_A_hermitian_and_bounded(L, seed, eps, m, t_bc):
    U = synth.gauge_field(L, eps, seed, workers=1)
    rng = np.random.default_rng(seed + 3)
    Vh = synth.even_volume(L)
    u, v = _vec(rng, (3, Vh)), _vec(rng, (3, Vh))
    Au, Av = dirac.mdagm(U, m, u, t_bc), dirac.mdagm(U, m, v, t_bc)
    assert abs(np.vdot(u, Av) - np.vdot(Au, v)) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Av)
    q = np.vdot(v, Av).real / np.vdot(v, v).real
    assert m * m - 1e-12 <= q <= 16.0 + m * m + 1e-12
