"""Pins of the oracle's lattice geometry and staggered operator.

Each check rests on something other than the oracle's own formula: a closed
form (free-field spectrum, plane waves), a hand-derived fixture, brute force
over tiny lattices, or a symmetry the operator of Eq. stag must have
(anti-Hermiticity, gauge covariance, translations by two sites).
"""

import itertools
import os

import numpy as np
import pytest

import synth
from oracle import dirac, lattice


def _lex(L, x, y, z, t):
    return x + L[0] * (y + L[1] * (z + L[2] * t))


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 6, 8), (6, 2, 4, 2)])
def test_eo_order_and_neighbors_brute_force(L):
    """Neighbour table against a pure-Python loop over all sites."""
    V = L[0] * L[1] * L[2] * L[3]
    for parity in (0, 1):
        tab = lattice.neighbor_table(L, parity)
        seen = {}
        for t, z, y, x in itertools.product(*(range(L[3]), range(L[2]), range(L[1]), range(L[0]))):
            if (x + y + z + t) % 2 != parity:
                continue
            eo = _lex(L, x, y, z, t) // 2
            assert eo not in seen
            seen[eo] = (x, y, z, t)
            c = [x, y, z, t]
            for mu in range(4):
                f = list(c)
                f[mu] = (c[mu] + 1) % L[mu]
                b = list(c)
                b[mu] = (c[mu] - 1) % L[mu]
                assert tab[eo, mu] == _lex(L, *f) // 2
                assert tab[eo, 4 + mu] == _lex(L, *b) // 2
        assert sorted(seen) == list(range(V // 2))
        xs = lattice.eo_coordinates(L, parity)
        for eo, c in seen.items():
            assert tuple(int(a[eo]) for a in xs) == c


def _load_delta(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "delta_unit_links_4444.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            rows.append((tuple(int(a) for a in v[:5]), tuple(int(a) for a in v[5:10]),
                         complex(float(v[10]), float(v[11]))))
    return rows


def test_delta_source_matches_hand_values(golden_dir):
    L = (4, 4, 4, 4)
    U = synth.unit_gauge(L)
    rows = _load_delta(golden_dir)
    for src in sorted({r[0] for r in rows}):
        x, y, z, t, c = src
        assert (x + y + z + t) % 2 == 1
        v = np.zeros((3, 128), dtype=np.complex128)
        v[c, _lex(L, x, y, z, t) // 2] = 1.0
        out = dirac.dslash(U, v, 0, t_bc=-1)
        expect = np.zeros_like(out)
        for s, o, val in rows:
            if s != src:
                continue
            ox, oy, oz, ot, oc = o
            expect[oc, _lex(L, ox, oy, oz, ot) // 2] = val
        assert np.array_equal(out, expect)


def _free_spectrum(L, m, t_bc):
    ps = []
    for mu in range(4):
        k = np.arange(L[mu])
        if mu == 3 and t_bc == -1:
            ps.append((2 * k + 1) * np.pi / L[mu])
        else:
            ps.append(2 * np.pi * k / L[mu])
    grids = np.meshgrid(*ps, indexing="ij")
    lam = m * m + sum(np.sin(g) ** 2 for g in grids)
    return np.sort(np.repeat(lam.reshape(-1), 3))


@pytest.mark.parametrize("L,t_bc", [((4, 4, 4, 4), -1), ((4, 4, 4, 4), 1), ((2, 4, 6, 8), -1),
                                    ((6, 4, 2, 4), -1)])
def test_free_field_spectrum(L, t_bc):
    """Unit links: spec(A) doubled = {m^2 + sum_mu sin^2 p_mu} x 3 colours."""
    m = 0.1
    A = dirac.dense_A(synth.unit_gauge(L), m, t_bc)
    w = np.linalg.eigvalsh(A)
    got = np.sort(np.concatenate([w, w]))
    np.testing.assert_allclose(got, _free_spectrum(L, m, t_bc), atol=1e-13, rtol=0)


def test_free_field_4444_eigenvalue_set():
    """4^4 antiperiodic: the distinct eigenvalues are m^2 + {1/2, 3/2, 5/2, 7/2}."""
    m = 0.1
    w = np.linalg.eigvalsh(dirac.dense_A(synth.unit_gauge((4, 4, 4, 4)), m, -1))
    vals = np.unique(np.round(w - m * m, 12))
    np.testing.assert_allclose(vals, [0.5, 1.5, 2.5, 3.5], atol=1e-12)


@pytest.mark.parametrize("L", [(8, 6, 4, 10), (16, 16, 16, 4)])
def test_plane_waves_are_eigenvectors(L):
    """A e^{ip.n} = (m^2 + sum sin^2 p) e^{ip.n} for unit links, any size."""
    m = 0.02
    U = synth.unit_gauge(L)
    x, y, z, t = lattice.eo_coordinates(L, 0)
    rng = np.random.default_rng(7)
    for _ in range(3):
        k = [int(rng.integers(0, l)) for l in L]
        p = [2 * np.pi * k[i] / L[i] for i in range(3)] + [(2 * k[3] + 1) * np.pi / L[3]]
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        chi = np.array([0.3 - 0.1j, 1.0, -0.5j])
        v = chi[:, None] * phase[None, :]
        lam = m * m + sum(np.sin(q) ** 2 for q in p)
        np.testing.assert_allclose(dirac.mdagm(U, m, v), lam * v, atol=1e-13, rtol=0)


@pytest.fixture(scope="module")
def rough():
    L = (4, 4, 4, 6)
    return L, synth.gauge_field(L, 0.8, 77)


def _rand_vec(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_anti_hermitian(rough):
    L, U = rough
    Vh = synth.even_volume(L)
    rng = np.random.default_rng(1)
    for t_bc in (-1, 1):
        u = _rand_vec(rng, (3, Vh))
        v = _rand_vec(rng, (3, Vh))
        lhs = np.vdot(u, dirac.dslash(U, v, 0, t_bc))
        rhs = -np.vdot(dirac.dslash(U, u, 1, t_bc), v)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_full_matrix_anti_hermitian_hopping(rough):
    L, U = rough
    M = dirac.full_matrix_M(U, 0.0)
    np.testing.assert_allclose(M, -M.conj().T, atol=1e-15)
    # only nearest neighbours are connected
    V = synth.volume(L)
    nnz_sites = (np.abs(M.reshape(V, 3, V, 3)).sum(axis=(1, 3)) > 0).sum(axis=1)
    assert nnz_sites.max() == 8


def test_gauge_covariance(rough):
    """D[U^G](G psi) = G D[U] psi with U^G_mu(n) = G(n) U_mu(n) G(n+mu)^dagger."""
    L, U = rough
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(3)
    G = synth.random_su3((Lt, Lz, Ly, Lx), rng, 2.0)
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=lattice.AXIS[mu] - 1)
        UG[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gf, -1, -2))
    Vh = synth.even_volume(L)
    v = _rand_vec(rng, (3, Vh))
    Gt = lambda w, par: lattice.restrict(  # noqa: E731
        np.einsum("...ij,...j->...i", G, lattice.embed(w, L, par)), L, par)
    for par in (0, 1):
        lhs = dirac.dslash(UG, Gt(v, 1 - par), par)
        rhs = Gt(dirac.dslash(U, v, par), par)
        np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_translation_by_two_commutes(rough):
    L, U = rough
    Vh = synth.even_volume(L)
    rng = np.random.default_rng(5)
    v = _rand_vec(rng, (3, Vh))
    for mu in range(3):
        ax = lattice.AXIS[mu]
        Us = np.roll(U, 2, axis=ax - 2)          # link array: two extra trailing axes
        vs = lattice.restrict(np.roll(lattice.embed(v, L, 1), 2, axis=ax), L, 1)
        lhs = dirac.dslash(Us, vs, 0)
        rhs = lattice.restrict(np.roll(lattice.embed(dirac.dslash(U, v, 0), L, 0), 2, axis=ax), L, 0)
        np.testing.assert_allclose(lhs, rhs, atol=1e-14)


def test_A_hermitian_positive_and_bounded(rough):
    L, U = rough
    m = 0.05
    A = dirac.dense_A(U, m)
    np.testing.assert_allclose(A, A.conj().T, atol=1e-15)
    w = np.linalg.eigvalsh(A)
    assert w.min() >= m * m - 1e-13
    assert w.max() <= 16 + m * m + 1e-13


def test_A_is_even_block_of_MdagM(rough):
    """A = (M^dagger M) restricted to even sites, built from the full M."""
    L, U = rough
    m = 0.3
    M = dirac.full_matrix_M(U, m)
    MM = M.conj().T @ M
    V = synth.volume(L)
    x, y, z, t = lattice.eo_coordinates(L, 0)
    lex = _lex(L, x, y, z, t)
    # basis of dense_A is c*Vh + eo; of M it is 3*lex + c
    idx = np.array([[3 * lex[e] + c for e in range(V // 2)] for c in range(3)]).reshape(-1)
    np.testing.assert_allclose(MM[np.ix_(idx, idx)], dirac.dense_A(U, m), atol=1e-13)
