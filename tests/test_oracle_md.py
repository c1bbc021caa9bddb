"""Pins of the gauge-sector and molecular-dynamics oracle (CPU).

Each pin is fixed by something other than the oracle's own formulas:

* generators: Tr(T^a T^b) = delta_ab / 2 and the su(3) structure constants
  f_123 = 1, f_458 = sqrt(3)/2, f_147 = 1/2;
* kinetic term: sum Tr(H^2) = (1/2) sum omega^2; algebra coefficients of
  i H are -omega/2; the momentum layout of the C ABI against a brute-force
  loop over sites;
* plaquette action: zero on unit links; closed form on diagonal (abelian)
  links, where each plaquette is the exponential of a lattice curl; the
  single-link configuration (6 plaquettes see the link); gauge invariance;
* gauge force: central finite differences of the action, the single-link
  closed form -2 beta TA(W), gauge covariance;
* exponential: diagonal and embedded-SU(2) closed forms; reunitarisation
  fixes SU(3) matrices and positive multiples of them;
* 2MN integrator: on a harmonic oscillator one step has trace
  2 - h^2 + lam (1 - 2 lam) h^4 / 2 (derived by hand from the shears);
  the multi-step scheme reduces to it with either force switched off;
* lattice MD: |dH| falls as delta^2, the evolution is reversible to
  rounding, the heat bath makes the initial fermion action R^dagger R.
"""

import numpy as np
import pytest

import synth
from oracle import dirac, gauge, lattice, md
from synth.make_rational import rational_for

T = gauge.generators()


def _comm(a, b):
    return a @ b - b @ a


def _algebra(rng):
    H = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    H = 0.5 * (H + H.conj().T)
    return H - np.trace(H) / 3 * np.eye(3)


def _random_su3(rng, shape):
    w = rng.standard_normal(tuple(shape) + (8,))
    return gauge.reunitarize(gauge.exp_i(1.0, gauge.mom_matrix(w)))


def _transform(U, G):
    """U'_mu(n) = G(n) U_mu(n) G(n+mu)^dagger."""
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ gauge.dagger(gauge.shift(G, mu, 1))
    return out


# ------------------------------------------------------------------ algebra
def test_generator_normalisation_and_structure_constants():
    gram = np.einsum("aij,bji->ab", T, T)
    assert np.allclose(gram, 0.5 * np.eye(8), atol=1e-15)
    assert np.allclose(_comm(T[0], T[1]), 1j * T[2], atol=1e-15)
    assert np.allclose(_comm(T[3], T[4]), 1j * (0.5 * T[2] + np.sqrt(3) / 2 * T[7]), atol=1e-15)
    assert np.allclose(_comm(T[0], T[3]), 1j * 0.5 * T[6], atol=1e-15)
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T) and abs(np.trace(T[a])) < 1e-16


def test_kinetic_and_coefficients():
    rng = np.random.default_rng(1)
    w = rng.standard_normal((5, 4, 8))
    H = gauge.mom_matrix(w)
    trh2 = np.real(np.einsum("...ij,...ji->...", H, H)).sum()
    assert abs(trh2 - 0.5 * np.sum(w ** 2)) < 1e-12
    assert abs(gauge.kinetic(w) - trh2) < 1e-12
    assert np.allclose(gauge.algebra_coefficients(1j * H), -0.5 * w, atol=1e-14)


def test_mom_layout_brute_force():
    L = (4, 2, 2, 6)
    Lx, Ly, Lz, Lt = L
    Vh = Lx * Ly * Lz * Lt // 2
    w = np.random.default_rng(2).standard_normal((8, 4, 2, Vh))
    full = gauge.mom_from_abi(w, L)
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    lex = x + Lx * (y + Ly * (z + Lz * t))
                    par = (x + y + z + t) % 2
                    for mu in range(4):
                        assert np.array_equal(full[t, z, y, x, mu], w[:, mu, par, lex // 2])
    assert np.array_equal(gauge.mom_to_abi(full), w)


# ------------------------------------------------------------------ action
def test_action_unit_links_is_zero():
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, 2, 2, 2, 4, 3, 3)).copy()
    assert gauge.gauge_action(U, 5.5) == 0.0


def test_action_abelian_closed_form():
    L = (4, 2, 2, 4)
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(3)
    th = rng.uniform(-np.pi, np.pi, (Lt, Lz, Ly, Lx, 4))
    ph = rng.uniform(-np.pi, np.pi, (Lt, Lz, Ly, Lx, 4))
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = np.exp(1j * th)
    U[..., 1, 1] = np.exp(1j * ph)
    U[..., 2, 2] = np.exp(-1j * (th + ph))
    beta = 5.3
    want = 0.0
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    n = [x, y, z, t]
                    for mu in range(4):
                        for nu in range(mu + 1, 4):
                            a = list(n); a[mu] = (a[mu] + 1) % L[mu]
                            b = list(n); b[nu] = (b[nu] + 1) % L[nu]

                            def at(f, s, d):
                                return f[s[3], s[2], s[1], s[0], d]
                            f1 = at(th, n, mu) + at(th, a, nu) - at(th, b, mu) - at(th, n, nu)
                            f2 = at(ph, n, mu) + at(ph, a, nu) - at(ph, b, mu) - at(ph, n, nu)
                            retr = np.cos(f1) + np.cos(f2) + np.cos(f1 + f2)
                            want += beta * (1 - retr / 3)
    assert abs(gauge.gauge_action(U, beta) - want) < 1e-11 * abs(want)


def _single_link(L, site, mu, W):
    Lx, Ly, Lz, Lt = L
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (Lt, Lz, Ly, Lx, 4, 3, 3)).copy()
    x, y, z, t = site
    U[t, z, y, x, mu] = W
    return U


def test_action_and_force_single_link():
    rng = np.random.default_rng(4)
    W = _random_su3(rng, ())
    L = (4, 4, 2, 4)
    beta = 5.0
    U = _single_link(L, (3, 1, 0, 3), 3, W)
    assert abs(gauge.gauge_action(U, beta) - 6 * beta * (1 - np.real(np.trace(W)) / 3)) < 1e-12
    F = gauge.gauge_force(U, beta)
    want = -2 * beta * gauge.traceless_antihermitian(W)
    assert np.allclose(F[3, 0, 1, 3, 3], want, atol=1e-13)


def test_action_gauge_invariant():
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.5, 51)
    G = _random_su3(np.random.default_rng(5), (4, 4, 4, 4))
    a, b = gauge.gauge_action(U, 5.5), gauge.gauge_action(_transform(U, G), 5.5)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("site,mu", [((0, 0, 0, 0), 0), ((3, 1, 2, 3), 3), ((1, 3, 0, 2), 1),
                                     ((2, 0, 3, 1), 2)])
def test_gauge_force_is_derivative_of_action(site, mu):
    L = (4, 4, 4, 4)
    beta = 5.3
    U = synth.gauge_field(L, 0.6, 52)
    F = gauge.gauge_force(U, beta)
    rng = np.random.default_rng(60 + mu + sum(site))
    Tdir = _algebra(rng)
    x, y, z, t = site
    eps = 1e-5
    S = []
    for sg in (1, -1):
        Up = U.copy()
        Up[t, z, y, x, mu] = gauge.exp_i(sg * eps, Tdir) @ U[t, z, y, x, mu]
        S.append(gauge.gauge_action(Up, beta))
    fd = (S[0] - S[1]) / (2 * eps)
    want = np.real(1j * np.trace(Tdir @ F[t, z, y, x, mu]))
    assert abs(fd - want) < 1e-6 * max(1.0, abs(want))
    assert np.allclose(F, -gauge.dagger(F), atol=1e-14)
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-14


def test_gauge_force_covariant():
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.5, 53)
    G = _random_su3(np.random.default_rng(6), (4, 4, 4, 4))
    F = gauge.gauge_force(U, 5.5)
    F2 = gauge.gauge_force(_transform(U, G), 5.5)
    for mu in range(4):
        assert np.allclose(F2[..., mu, :, :], G @ F[..., mu, :, :] @ gauge.dagger(G), atol=1e-12)


# ------------------------------------------------------------------ exponential
def test_exponential_closed_forms():
    rng = np.random.default_rng(7)
    d = rng.standard_normal(2)
    H = np.diag([d[0], d[1], -d[0] - d[1]]).astype(np.complex128)
    assert np.allclose(gauge.exp_i(0.3, H), np.diag(np.exp(0.3j * np.diag(H))), atol=1e-15)
    # embedded SU(2): exp(i eps w T^1) = cos(eps w/2) + i sin(eps w/2) sigma_1 on the upper block
    w, eps = 1.7, 0.4
    E = gauge.exp_i(eps, w * T[0])
    c, s = np.cos(eps * w / 2), np.sin(eps * w / 2)
    assert np.allclose(E, np.array([[c, 1j * s, 0], [1j * s, c, 0], [0, 0, 1]]), atol=1e-15)
    H = _algebra(rng)
    E = gauge.exp_i(0.7, H)
    assert np.allclose(E @ E.conj().T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(E) - 1) < 1e-14


def test_reunitarize():
    rng = np.random.default_rng(8)
    U = _random_su3(rng, (10,))
    assert np.allclose(gauge.reunitarize(U), U, atol=1e-15)
    assert np.allclose(gauge.reunitarize(2.5 * U), U, atol=1e-15)
    P = U + 1e-3 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    R = gauge.reunitarize(P)
    assert np.allclose(R @ gauge.dagger(R), np.eye(3), atol=1e-15)
    assert np.allclose(np.linalg.det(R), 1, atol=1e-15)


# ------------------------------------------------------------------ integrator
class _Oscillator:
    """q'' = -(kf + kg) q split into a 'fermion' and a 'gauge' kick."""

    def __init__(self, kf, kg):
        self.kf, self.kg = kf, kg

    def step_matrix(self, tau, n_md, gauge_steps, lam):
        cols = []
        for q0, p0 in ((1.0, 0.0), (0.0, 1.0)):
            st = [q0, p0]

            def kf(c):
                st[1] -= c * self.kf * st[0]

            def kg(c):
                st[1] -= c * self.kg * st[0]

            def dr(c):
                st[0] += c * st[1]

            md.integrate_2mn(tau, n_md, gauge_steps, lam, kf, kg, dr)
            cols.append(st)
        return np.array(cols).T


def _trace_2mn(h, lam):
    return 2 - h * h + lam * (1 - 2 * lam) * h ** 4 / 2


@pytest.mark.parametrize("h", [0.1, 0.37, 0.9])
def test_2mn_single_step_trace(h):
    lam = md.LAMBDA_2MN
    M = _Oscillator(1.0, 0.0).step_matrix(h, 1, 2, lam)   # gauge force off: plain 2MN
    assert abs(np.trace(M) - _trace_2mn(h, lam)) < 1e-14
    assert abs(np.linalg.det(M) - 1) < 1e-14
    # lam = 0 is the leapfrog Q P Q: trace 2 - h^2
    M0 = _Oscillator(1.0, 0.0).step_matrix(h, 1, 2, 0.0)
    assert abs(np.trace(M0) - (2 - h * h)) < 1e-14


@pytest.mark.parametrize("gs", [2, 4, 10])
def test_2mn_multistep_gauge_only(gs):
    lam, tau = md.LAMBDA_2MN, 0.8
    M = _Oscillator(0.0, 1.0).step_matrix(tau, 1, gs, lam)
    h = tau / gs
    theta = np.arccos(_trace_2mn(h, lam) / 2)
    assert abs(np.trace(M) - 2 * np.cos(gs * theta)) < 1e-13
    assert abs(np.linalg.det(M) - 1) < 1e-14


def test_2mn_reversible_and_second_order():
    lam = md.LAMBDA_2MN
    osc = _Oscillator(0.7, 0.6)
    M = osc.step_matrix(1.0, 4, 6, lam)
    flip = np.diag([1.0, -1.0])
    assert np.allclose(flip @ M @ flip @ M, np.eye(2), atol=1e-14)
    w = np.sqrt(1.3)
    exact = np.array([[np.cos(w), np.sin(w) / w], [-w * np.sin(w), np.cos(w)]])
    e1 = np.abs(osc.step_matrix(1.0, 4, 6, lam) - exact).max()
    e2 = np.abs(osc.step_matrix(1.0, 8, 6, lam) - exact).max()
    assert 3.2 < e1 / e2 < 4.8


# ------------------------------------------------------------------ lattice MD
@pytest.fixture(scope="module")
def md_setup():
    L = (4, 4, 4, 4)
    m, beta = 0.2, 5.3
    U = synth.gauge_field(L, 0.4, 61)
    rng = np.random.default_rng(62)
    omega = rng.standard_normal((4, 4, 4, 4, 4, 8))
    R = (rng.standard_normal((2, 3, 128)) + 1j * rng.standard_normal((2, 3, 128))) * np.sqrt(0.5)
    r_md = rational_for(1, -0.25)
    r_hb = rational_for(1, 0.125)
    phi = md.heatbath(U, m, R, r_hb)
    return L, m, beta, U, omega, R, phi, r_md, r_hb


def _dH(setup, n_md, gs, tau=0.5):
    L, m, beta, U, omega, R, phi, r_md, _ = setup
    h0 = md.hamiltonian(U, omega, phi, beta, m, r_md)
    sys = md.LatticeMD(U, omega, phi, beta, m, r_md)
    sys.integrate(tau, n_md, gs)
    h1 = md.hamiltonian(sys.U, sys.omega, phi, beta, m, r_md)
    return sum(b - a for a, b in zip(h0, h1)), sys


def test_md_energy_error_second_order(md_setup):
    d1, s1 = _dH(md_setup, 2, 4)
    d2, _ = _dH(md_setup, 4, 4)
    assert abs(d1) < 0.5
    assert 3.5 < d1 / d2 < 4.5, (d1, d2)
    # 3 fermion kicks per outer step; per inner scheme gs/2 steps of 3 gauge kicks, 2 drifts
    assert (s1.n_fermion, s1.n_gauge, s1.n_drift) == (6, 24, 16)


def test_md_reversible(md_setup):
    L, m, beta, U, omega, R, phi, r_md, _ = md_setup
    a = md.LatticeMD(U, omega, phi, beta, m, r_md)
    a.integrate(0.2, 2, 4)
    b = md.LatticeMD(a.U, -a.omega, phi, beta, m, r_md)
    b.integrate(0.2, 2, 4)
    dC, dM = md.reversibility(U, b.U, omega, b.omega)
    assert dC < 1e-13 and dM < 1e-12, (dC, dM)


def test_heatbath_action_is_gaussian_norm(md_setup):
    L, m, beta, U, omega, R, phi, r_md, r_hb = md_setup
    S = md.fermion_action(U, m, phi, r_md)
    RR = float(np.sum(np.abs(R) ** 2))
    assert abs(S / RR - 1) < 1e-4


def test_pure_gauge_md_conserves_energy():
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.4, 63)
    omega = np.random.default_rng(64).standard_normal((4, 4, 4, 4, 4, 8))
    beta = 5.5

    def run(gs):
        sys = md.LatticeMD(U, omega, np.zeros((0, 3, 128)), beta, 0.1,
                           rational_for(1, -0.25))
        sys.kick_f = lambda c: None
        sys.integrate(0.5, 1, gs)
        return (gauge.kinetic(sys.omega) + gauge.gauge_action(sys.U, beta)
                - gauge.kinetic(omega) - gauge.gauge_action(U, beta))

    a, b = run(10), run(20)
    assert abs(a) < 0.5 and 3.5 < a / b < 4.5, (a, b)


def test_trajectory_metropolis(md_setup):
    L, m, beta, U, omega, R, phi, r_md, r_hb = md_setup
    a = md.trajectory(U, omega, R, 0.0, beta, m, r_hb, r_md, r_md, 0.5, 2, 4)
    assert a["accepted"] and not np.array_equal(a["U"], U)
    assert abs(a["h0"][2] / float(np.sum(np.abs(R) ** 2)) - 1) < 1e-4
    assert abs(a["dH"] - sum(a["h1"]) + sum(a["h0"])) < 1e-9
    u = 0.5 * (1.0 + np.exp(-a["dH"])) if a["dH"] > 0 else None
    if u is not None:
        b = md.trajectory(U, omega, R, u, beta, m, r_hb, r_md, r_md, 0.5, 2, 4)
        assert not b["accepted"] and np.array_equal(b["U"], U)


def test_gauge_force_at_sampled_links_matches_whole_lattice():
    L = (4, 6, 4, 2)
    U = synth.gauge_field(L, 0.7, 71)
    F = gauge.gauge_force(U, 5.1)
    rng = np.random.default_rng(72)
    k = 60
    t, z, y, x = (rng.integers(0, n, k) for n in U.shape[:4])
    mu = rng.integers(0, 4, k)
    Fs = gauge.gauge_force_links(U, 5.1, t, z, y, x, mu)
    assert np.abs(Fs - F[t, z, y, x, mu]).max() < 1e-14
