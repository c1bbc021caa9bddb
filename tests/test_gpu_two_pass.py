"""GPU parity of the two-pass rational apply (rhmc_solver_params.two_pass).

Pass 1 of the shared Krylov solve keeps only each step's alpha and beta,
the weights w(k) of y = alpha0 b + sum_k w(k) r(k) are rebuilt from them,
and pass 2 repeats the iteration and accumulates y (a variant of the shared
solve of Sec. 4.3 that the paper does not describe).  In exact
arithmetic this is the one-pass result, so:
* on 4^4 y matches the oracle's dense r(A) b within the solver-tolerance
  bound, and A^{-1/4} b within the minimax error;
* on larger lattices it matches the one-pass FP64 apply to rounding of the
  two summation orders (1e-11 relative), and the pseudofermion action too;
* repeated calls are bit-identical, zero sources give zero, right-hand
  sides beyond one launch batch work, and misuse is rejected.
"""

from types import SimpleNamespace

import numpy as np
import pytest

import synth
from oracle import dirac, rational, solvers
from synth.make_rational import rational_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rh():
    import torch

    from paper_1106_5673_amd import rhmc

    rhmc.load()
    assert torch.cuda.is_available()
    return rhmc


def _to(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _apply(rh, g, lat, m, r, b, **kw):
    import torch

    allow = kw.pop("allow_not_converged", False)
    y = torch.empty((b.shape[0], 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_rational_apply(g, m, r.alpha0, r.alpha, r.beta, _to(b), y, rh.solver_params(**kw),
                                allow_not_converged=allow)
    return y.cpu().numpy(), st


def test_two_pass_matches_dense_oracle(rh):
    """4^4, eps 0.5, m 0.1, 8 poles of x^-1/4, tol 1e-12."""
    c = synth.CONFIGS[1]
    L, m = c["L"], c["m"]
    U = synth.gauge_field(L, c["eps"], synth.fields.seed_gauge(1))
    b = synth.source(L, synth.fields.seed_source(1), 1)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    r = rational_for(1, -0.25)
    y, st = _apply(rh, g, lat, m, r, b, tol=1e-12, two_pass=1)
    Ad = dirac.dense_A(U, m)
    yd = rational.dense_function_apply(
        Ad, b[0], lambda w: rational.scalar_rational(w, r.alpha0, r.alpha, r.beta))
    bound = sum(abs(a) * np.linalg.cond(Ad + s * np.eye(Ad.shape[0])) * 1e-12 *
                np.linalg.norm(solvers.dense_solve(Ad, b[0], s)) for a, s in zip(r.alpha, r.beta))
    assert np.linalg.norm(y[0] - yd) <= bound + 1e-14 * np.linalg.norm(yd)
    exact = rational.dense_function_apply(Ad, b[0], lambda w: w ** -0.25)
    assert np.linalg.norm(y[0] - exact) <= (r.delta + 1e-10) * np.linalg.norm(exact)
    # per-shift recurrence residuals within tol; every shift took steps
    assert st["max_true_residual"] <= 1e-12
    assert (st["iterations"] >= 1).all() and (st["refine_iterations"] == 0).all()
    assert st["total_iterations"] == st["iterations"].max()
    g.close()


@pytest.mark.parametrize("L,eps,m,nrhs,cfg", [((6, 4, 4, 8), 0.6, 0.02, 3, 3),
                                              ((8, 8, 8, 6), 0.8, 0.005, 2, 5),
                                              ((2, 2, 2, 2), 0.5, 0.1, 1, 1)])
def test_two_pass_matches_one_pass(rh, L, eps, m, nrhs, cfg):
    U = synth.gauge_field(L, eps, 7100 + sum(L))
    b = synth.source(L, 7200 + sum(L), nrhs)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    r = rational_for(cfg, -0.25)
    y1, st1 = _apply(rh, g, lat, m, r, b, tol=1e-10, mode=rh.RHMC_MODE_FP64)
    y2, st2 = _apply(rh, g, lat, m, r, b, tol=1e-10, two_pass=1)
    y3, _ = _apply(rh, g, lat, m, r, b, tol=1e-10, two_pass=1)
    assert np.array_equal(y2, y3)
    assert st2["total_iterations"] == st1["total_iterations"]
    assert (st2["iterations"] == st1["iterations"]).all()
    for j in range(nrhs):
        rel = np.linalg.norm(y2[j] - y1[j]) / np.linalg.norm(y1[j])
        print(f"rhs {j}: |y2 - y1| / |y1| = {rel:.2e}")
        assert rel <= 1e-11
    # recurrence residuals agree with the one-pass FP64 true residuals
    assert np.allclose(st2["true_residual"], st1["true_residual"], rtol=1e-2, atol=1e-13)
    g.close()


def test_two_pass_batches_and_zero_source(rh):
    """11 right-hand sides (two launch batches), one of them zero; unsorted
    shifts; graph replay off in one call."""
    L, m = (6, 4, 4, 8), 0.02
    U = synth.gauge_field(L, 0.6, 7301)
    b = synth.source(L, 7302, 11)
    b[4] = 0
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    r0 = rational_for(3, -0.25)
    perm = np.random.default_rng(3).permutation(len(r0.beta))
    r = SimpleNamespace(alpha0=r0.alpha0, alpha=np.asarray(r0.alpha)[perm],
                        beta=np.asarray(r0.beta)[perm])
    y1, _ = _apply(rh, g, lat, m, r, b, tol=1e-10)
    y2, st2 = _apply(rh, g, lat, m, r, b, tol=1e-10, two_pass=1)
    y3, _ = _apply(rh, g, lat, m, r, b, tol=1e-10, two_pass=1, use_graph=0, block=7)
    assert not y2[4].any() and st2["iterations"][4].max() == 0
    for j in range(11):
        if j == 4:
            continue
        assert np.linalg.norm(y2[j] - y1[j]) <= 1e-11 * np.linalg.norm(y1[j])
        assert np.linalg.norm(y3[j] - y1[j]) <= 1e-11 * np.linalg.norm(y1[j])
    g.close()


def test_two_pass_pseudofermion_action(rh):
    L, m = (8, 8, 8, 6), 0.01
    U = synth.gauge_field(L, 0.7, 7401)
    phi = synth.source(L, 7402, 2)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    r = rational_for(4, -0.25)
    S1, _ = rh.rhmc_pf_action(g, m, r.alpha0, r.alpha, r.beta, _to(phi), rh.solver_params(tol=1e-10))
    S2, _ = rh.rhmc_pf_action(g, m, r.alpha0, r.alpha, r.beta, _to(phi),
                              rh.solver_params(tol=1e-10, two_pass=1))
    assert np.allclose(S2, S1, rtol=1e-11, atol=0)
    g.close()


def test_two_pass_not_converged_and_misuse(rh):
    import torch

    L, m = (4, 4, 4, 4), 0.1
    U = synth.gauge_field(L, 0.5, 7501)
    b = synth.source(L, 7502, 1)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    r = rational_for(1, -0.25)
    y, st = _apply(rh, g, lat, m, r, b, tol=1e-12, two_pass=1, maxiter=10, allow_not_converged=True)
    assert st["status"] == rh.RHMC_ERR_NOT_CONVERGED
    assert st["total_iterations"] == 10 and np.isfinite(y).all()
    with pytest.raises(rh.RhmcError) as e:
        _apply(rh, g, lat, m, r, b, two_pass=1, mode=rh.RHMC_MODE_MIXED)
    assert e.value.status == rh.RHMC_ERR_UNSUPPORTED
    with pytest.raises(rh.RhmcError) as e:
        _apply(rh, g, lat, m, r, b, two_pass=1, per_shift=1)
    assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    x = torch.empty((1, len(r.beta), 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(rh.RhmcError) as e:
        rh.rhmc_multishift_cg(g, m, r.beta, _to(b), x, rh.solver_params(two_pass=1))
    assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    Lx, Ly, Lz, Lt = L
    F = torch.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(rh.RhmcError) as e:
        rh.rhmc_pf_force(g, m, r.alpha0, r.alpha, r.beta, _to(b), F, rh.solver_params(two_pass=1))
    assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    g.close()


@pytest.mark.parametrize("case", ["one_pole", "periodic", "hilo_links"])
def test_two_pass_edge_cases(rh, case):
    """A single pole, a periodic time boundary, and an FP64 operator rebuilt
    from hi/lo FP32 links: the two-pass apply equals the one-pass apply."""
    L, m = (6, 4, 4, 8), 0.03
    t_bc = 1 if case == "periodic" else -1
    U = synth.gauge_field(L, 0.6, 7601)
    b = synth.source(L, 7602, 2)
    lat = rh.rhmc_lattice_create(L, t_bc)
    flags = rh.RHMC_LINKS_HILO_12 if case == "hilo_links" else 0
    g = rh.rhmc_gauge_create(lat, U, flags=flags)
    r0 = rational_for(3, -0.25)
    if case == "one_pole":
        r = SimpleNamespace(alpha0=0.0, alpha=np.array([1.0]), beta=np.array([0.0]))
    else:
        r = r0
    y1, st1 = _apply(rh, g, lat, m, r, b, tol=1e-10)
    y2, st2 = _apply(rh, g, lat, m, r, b, tol=1e-10, two_pass=1)
    assert st2["total_iterations"] == st1["total_iterations"]
    for j in range(2):
        assert np.linalg.norm(y2[j] - y1[j]) <= 1e-11 * np.linalg.norm(y1[j])
    if case == "one_pole":
        # y = A^-1 b: its oracle residual is within tol
        A = lambda v: dirac.mdagm(U, m, v, t_bc)  # noqa: E731
        for j in range(2):
            assert solvers.true_residual(A, b[j], y2[j], 0.0) <= 1e-10
    g.close()
