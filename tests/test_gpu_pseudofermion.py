"""GPU parity of the pseudofermion entry points (Phi algorithm, Sec. 2.1).

* rhmc_pf_phi: phi_e = m R_e - D_eo R_o against the oracle, 1e-13 relative;
* rhmc_pf_action: Re <phi, r(A) phi> against the oracle's multi-shift action
  on 4^4 (1e-10 relative, both solves at tol 1e-12);
* the heat bath phi = r_h(A) R (x^{1/8}) followed by the action with r_-
  (x^{-1/4}) returns R^dagger R within the minimax errors plus the bound the
  per-shift tolerance gives (16^3x4 FP64 and 48^3x12 MIXED batched), a
  property that holds at any size;
* with r(x) = 1/x, phi from rhmc_pf_phi has phi^dagger A^-1 phi with mean
  3 V/2 over Gaussian R (its covariance is A).
"""

import numpy as np
import pytest

import synth
from fieldcache import workload_gauge
from oracle import dirac, pseudofermion, rational
from synth.make_rational import rational_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rh():
    import torch

    from paper_1106_5673_amd import rhmc

    rhmc.load()
    assert torch.cuda.is_available()
    return rhmc


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _gauss(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


@pytest.mark.parametrize("L,t_bc,nrhs", [((4, 4, 4, 4), -1, 1), ((8, 8, 8, 6), -1, 3),
                                         ((6, 4, 4, 8), 1, 2)])
def test_pf_phi_matches_oracle(rh, L, t_bc, nrhs):
    import torch

    m = 0.05
    U = synth.gauge_field(L, 0.6, 5000 + sum(L))
    lat = rh.rhmc_lattice_create(L, t_bc)
    g = rh.rhmc_gauge_create(lat, U)
    rng = np.random.default_rng(20)
    Re = _gauss(rng, (nrhs, 3, lat.Vh))
    Ro = _gauss(rng, (nrhs, 3, lat.Vh))
    phi = torch.empty((nrhs, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    rh.rhmc_pf_phi(g, m, _dev(Re), _dev(Ro), phi)
    want = pseudofermion.phi_even(U, m, Re, Ro, t_bc)
    got = phi.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    with pytest.raises(rh.RhmcError):
        rh.rhmc_pf_phi(g, m, phi, _dev(Ro), phi)   # phi overlapping R
    g.close()


def test_pf_action_matches_oracle(rh):
    L = (4, 4, 4, 4)
    c = synth.CONFIGS[1]
    m = c["m"]
    U = synth.gauge_field(L, c["eps"], 5100)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    r = rational_for(1, -0.25)
    rng = np.random.default_rng(21)
    phi = _gauss(rng, (2, 3, lat.Vh))
    S, st = rh.rhmc_pf_action(g, m, r.alpha0, r.alpha, r.beta, _dev(phi),
                              rh.solver_params(tol=1e-12, mode=rh.RHMC_MODE_FP64))
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for k in range(2):
        want, info = pseudofermion.action(A, phi[k], r.alpha0, r.alpha, r.beta, tol=1e-12)
        assert info.converged
        assert abs(S[k] - want) <= 1e-10 * abs(want)
    assert st["max_true_residual"] <= 1e-12
    g.close()


def _invariant_bound(rh_, rm, m, tol):
    """|S - R^dagger R| / R^dagger R allowed for S = phi^dagger r_-(A) phi,
    phi = r_h(A) R: the minimax errors, plus the per-shift solver errors
    (||x_i - x_i*|| <= tol ||b|| / (m^2 + beta_i)) carried through."""
    lo, hi = m * m, 16.0 + m * m
    rat = (1 + rh_.delta) ** 2 * (1 + rm.delta) - 1
    sh = sum(abs(a) / (lo + b) for a, b in zip(rh_.alpha, rh_.beta))
    sm = sum(abs(a) / (lo + b) for a, b in zip(rm.alpha, rm.beta))
    # phi error e <= sh tol ||R||; |S| picks 2 |<e, r_- phi>| <= 2 e lo^{-1/4} hi^{1/8} ||R||,
    # and the action solve adds sm tol ||phi||^2 <= sm tol hi^{1/4} ||R||^2
    return rat + 2 * sh * tol * lo ** -0.25 * hi ** 0.125 + sm * tol * hi ** 0.25


def test_heatbath_action_invariant_16x16x16x4_fp64(rh):
    import torch

    cfg = 2
    c = synth.CONFIGS[cfg]
    m, tol = c["m"], c["tol"]
    U = workload_gauge(cfg)
    lat = rh.rhmc_lattice_create(c["L"], -1)
    g = rh.rhmc_gauge_create(lat, np.asarray(U))
    rh_, rm = rational_for(cfg, c["hb_power"]), rational_for(cfg, -0.25)
    rng = np.random.default_rng(22)
    R = _dev(_gauss(rng, (2, 3, lat.Vh)))
    phi = torch.empty_like(R)
    prm = rh.solver_params(tol=tol, mode=rh.RHMC_MODE_FP64)
    rh.rhmc_rational_apply(g, m, rh_.alpha0, rh_.alpha, rh_.beta, R, phi, prm)
    S, _ = rh.rhmc_pf_action(g, m, rm.alpha0, rm.alpha, rm.beta, phi, prm)
    R2 = (R.abs() ** 2).sum(dim=(1, 2)).cpu().numpy()
    bound = _invariant_bound(rh_, rm, m, tol)
    assert np.all(np.abs(S - R2) <= bound * R2), (S / R2 - 1, bound)
    g.close()


def test_heatbath_action_invariant_48x48x48x12_mixed_batched(rh):
    import torch

    cfg = 5
    c = synth.CONFIGS[cfg]
    m, tol = c["m"], c["tol"]
    U = workload_gauge(cfg)
    lat = rh.rhmc_lattice_create(c["L"], -1)
    g = rh.rhmc_gauge_create(lat, np.asarray(U))
    rh_, rm = rational_for(cfg, c["hb_power"]), rational_for(cfg, -0.25)
    rng = np.random.default_rng(23)
    R = _dev(_gauss(rng, (4, 3, lat.Vh)))
    phi = torch.empty_like(R)
    prm = rh.solver_params(tol=tol, mode=rh.RHMC_MODE_MIXED, tune=1)
    st = rh.rhmc_rational_apply(g, m, rh_.alpha0, rh_.alpha, rh_.beta, R, phi, prm)
    assert st["max_true_residual"] <= tol
    S, st = rh.rhmc_pf_action(g, m, rm.alpha0, rm.alpha, rm.beta, phi, prm)
    assert st["max_true_residual"] <= tol
    R2 = (R.abs() ** 2).sum(dim=(1, 2)).cpu().numpy()
    bound = _invariant_bound(rh_, rm, m, tol)
    assert np.all(np.abs(S - R2) <= bound * R2), (S / R2 - 1, bound)
    g.close()


def test_phi_covariance_is_A(rh):
    """With r(x) = 1/x the action of phi = pf_phi(R) has mean 3 V/2."""
    import torch

    L = (8, 8, 8, 8)
    m = 0.1
    U = synth.gauge_field(L, 0.5, 5200)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    rng = np.random.default_rng(24)
    nrhs = 16
    Re = _dev(_gauss(rng, (nrhs, 3, lat.Vh)))
    Ro = _dev(_gauss(rng, (nrhs, 3, lat.Vh)))
    phi = torch.empty_like(Re)
    rh.rhmc_pf_phi(g, m, Re, Ro, phi)
    S, _ = rh.rhmc_pf_action(g, m, 0.0, [1.0], [0.0], phi,
                             rh.solver_params(tol=1e-12, mode=rh.RHMC_MODE_FP64))
    n = 3 * lat.Vh
    # chi-square with n complex degrees of freedom: mean n, standard deviation sqrt(n)
    assert abs(S.mean() - n) <= 5 * np.sqrt(n) / np.sqrt(nrhs)
    g.close()


def test_pf_invalid_arguments(rh):
    import torch

    L = (4, 4, 4, 4)
    lat = rh.rhmc_lattice_create(L)
    g = rh.rhmc_gauge_create(lat, synth.unit_gauge(L), flags=rh.RHMC_LINKS_FP32_12)
    v = torch.zeros((1, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    w = torch.zeros_like(v)
    with pytest.raises(rh.RhmcError):   # no FP64 links
        rh.rhmc_pf_phi(g, 0.1, v, w, torch.empty_like(v))
    g.close()
    g = rh.rhmc_gauge_create(lat, synth.unit_gauge(L))
    with pytest.raises(rh.RhmcError):   # negative pole
        rh.rhmc_pf_action(g, 0.1, 0.0, [1.0], [-1.0], v)
    with pytest.raises(rh.RhmcError):   # non-finite coefficient
        rh.rhmc_pf_action(g, 0.1, float("nan"), [1.0], [0.5], v)
    g.close()


def _gauge_transform(U, G, phi_even):
    """U^G_mu(n) = G(n) U_mu(n) G(n+mu)^dagger and phi -> G phi (even sites)."""
    from oracle import lattice

    L = dirac.lattice_of(U)
    Ug = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=lattice.AXIS[mu] - 1)
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.swapaxes(Gf.conj(), -1, -2)
    full = lattice.embed(phi_even, L, 0)
    phig = lattice.restrict(np.einsum("...ab,...b->...a", G, full), L, 0)
    return Ug, phig


@pytest.mark.parametrize("flags", ["fp64_12", "fp64_18", "hilo"])
def test_pf_force_matches_oracle(rh, flags):
    import torch

    from oracle import force

    L = (4, 4, 4, 4)
    c = synth.CONFIGS[1]
    m = c["m"]
    U = synth.gauge_field(L, c["eps"], 5400)
    lat = rh.rhmc_lattice_create(L, -1)
    fl = dict(fp64_12=rh.RHMC_LINKS_FP64_12 | rh.RHMC_LINKS_FP32_12,
              fp64_18=rh.RHMC_LINKS_FP64_18 | rh.RHMC_LINKS_FP32_12,
              hilo=rh.RHMC_LINKS_HILO_12)[flags]
    g = rh.rhmc_gauge_create(lat, U, flags=fl)
    r = rational_for(1, -0.25)
    rng = np.random.default_rng(25)
    phi = _gauss(rng, (2, 3, lat.Vh))
    want = force.force(U, m, r.alpha, r.beta, phi)
    scale = np.abs(want).max()
    F = torch.empty(U.shape, dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_pf_force(g, m, r.alpha0, r.alpha, r.beta, _dev(phi), F,
                          rh.solver_params(tol=1e-13, mode=rh.RHMC_MODE_FP64))
    assert st["max_true_residual"] <= 1e-13
    # hi + lo links differ from the FP64 ones by ~2^-47 relative
    tol = 1e-9 if flags != "hilo" else 1e-8
    assert np.abs(F.cpu().numpy() - want).max() <= tol * scale
    if flags == "fp64_12":
        rh.rhmc_pf_force(g, m, r.alpha0, r.alpha, r.beta, _dev(phi), F,
                         rh.solver_params(tol=1e-10, mode=rh.RHMC_MODE_MIXED))
        assert np.abs(F.cpu().numpy() - want).max() <= 1e-6 * scale
    g.close()


def test_pf_force_gauge_covariance_16x16x16x4(rh):
    """F[U^G, G phi] = G F[U, phi] G^dagger, both from the GPU (a property that
    holds at any size; the tolerance is the solver's)."""
    import torch

    cfg = 2
    c = synth.CONFIGS[cfg]
    m = c["m"]
    U = np.asarray(workload_gauge(cfg))
    G = synth.gauge_field(c["L"], 1.0, 5500)[..., 0, :, :]
    rng = np.random.default_rng(26)
    lat = rh.rhmc_lattice_create(c["L"], -1)
    phi = _gauss(rng, (2, 3, lat.Vh))
    Ug, phig = _gauge_transform(U, G, phi)
    r = rational_for(cfg, -0.25)
    prm = rh.solver_params(tol=1e-12, mode=rh.RHMC_MODE_FP64)
    out = []
    for UU, pp in ((U, phi), (Ug, phig)):
        g = rh.rhmc_gauge_create(lat, UU)
        F = torch.empty(U.shape, dtype=torch.complex128, device="cuda:0")
        rh.rhmc_pf_force(g, m, r.alpha0, r.alpha, r.beta, _dev(pp), F, prm)
        out.append(F.cpu().numpy())
        g.close()
    F0, Fg = out
    want = G[..., None, :, :] @ F0 @ np.swapaxes(G.conj(), -1, -2)[..., None, :, :]
    assert np.abs(Fg - want).max() <= 1e-7 * np.abs(F0).max()


def test_pf_force_48x48x48x12_mixed_structure(rh):
    """Full size, MIXED batched, 4 sources x 20 poles.  The oracle cannot solve
    at this size, so the checks are properties that hold at any size: F is
    traceless anti-Hermitian, and a gauge transformation that differs from 1
    only on a few sites rotates F there (F -> G F G^dagger) within the solver
    tolerance."""
    import torch

    cfg = 5
    c = synth.CONFIGS[cfg]
    m, tol = c["m"], c["tol"]
    U = np.asarray(workload_gauge(cfg))
    lat = rh.rhmc_lattice_create(c["L"], -1)
    rng = np.random.default_rng(27)
    phi = _gauss(rng, (4, 3, lat.Vh))
    r = rational_for(cfg, -0.25)
    prm = rh.solver_params(tol=tol, mode=rh.RHMC_MODE_MIXED, tune=1)
    g = rh.rhmc_gauge_create(lat, U)
    F = torch.empty(U.shape, dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_pf_force(g, m, r.alpha0, r.alpha, r.beta, _dev(phi), F, prm)
    assert st["max_true_residual"] <= tol
    g.close()
    Fh = F.cpu().numpy()
    scale = np.abs(Fh).max()
    assert np.abs(Fh + np.swapaxes(Fh.conj(), -1, -2)).max() <= 1e-14 * scale
    assert np.abs(np.trace(Fh, axis1=-2, axis2=-1)).max() <= 1e-14 * scale
    # a gauge transformation that differs from 1 on a handful of sites
    G = np.broadcast_to(np.eye(3, dtype=np.complex128), U.shape[:4] + (3, 3)).copy()
    sites = [(0, 0, 0, 0), (5, 17, 33, 47), (11, 47, 2, 9), (6, 24, 24, 24)]
    rot = synth.fields.random_su3((len(sites),), np.random.default_rng(28), 1.0)
    for (t, z, y, x), Gs in zip(sites, rot):
        G[t, z, y, x] = Gs
    Ug, phig = _gauge_transform(U, G, phi)
    g = rh.rhmc_gauge_create(lat, Ug)
    Fg = torch.empty_like(F)
    rh.rhmc_pf_force(g, m, r.alpha0, r.alpha, r.beta, _dev(phig), Fg, prm)
    g.close()
    Fgh = Fg.cpu().numpy()
    for (t, z, y, x) in sites:
        want = G[t, z, y, x] @ Fh[t, z, y, x] @ G[t, z, y, x].conj().T
        assert np.abs(Fgh[t, z, y, x] - want).max() <= 1e-6 * scale
