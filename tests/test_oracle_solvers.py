"""Pins of the oracle's CG, multi-shift CG and rational apply.

The solvers reach a result with a plain definition, x_i = (A + sigma_i)^-1 b
(Eq. shifted), so they are pinned against dense direct solves and dense
eigen-decompositions on tiny lattices, plus independent single-shift CG.
The rational coefficients come from the Remez generator in ``synth`` and are
pinned by the equioscillation theorem, a closed form for degree 0 and a brute
force minimax fit for degree 1.
"""

import numpy as np
import pytest

import synth
from oracle import dirac, rational, solvers
from synth.make_rational import rational_for
from synth.remez import remez_relative


@pytest.fixture(scope="module")
def c1():
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.5, 1001)
    b = synth.source(L, 2100, 1)[0]
    m = 0.1
    return U, b, m, dirac.dense_A(U, m)


def test_cg_matches_dense(c1):
    U, b, m, Ad = c1
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for sigma in (0.0, 0.37):
        x, info = solvers.cg(A, b, sigma, tol=1e-12)
        assert info.converged
        xd = solvers.dense_solve(Ad, b, sigma)
        cond = np.linalg.cond(Ad + sigma * np.eye(Ad.shape[0]))
        assert np.linalg.norm(x - xd) <= cond * 1e-12 * np.linalg.norm(xd)
        assert solvers.true_residual(A, b, x, sigma) <= 1e-12


def test_multishift_matches_dense_and_single_shift(c1):
    U, b, m, Ad = c1
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    shifts = [0.0, 0.003, 0.05, 0.8, 5.0]
    x, info = solvers.multishift_cg(A, b, shifts, tol=1e-12)
    assert info.converged
    its = info.shift_iterations
    assert all(its[i] >= its[i + 1] for i in range(len(its) - 1))  # larger shifts converge first
    for i, s in enumerate(shifts):
        xd = solvers.dense_solve(Ad, b, s)
        cond = np.linalg.cond(Ad + s * np.eye(Ad.shape[0]))
        assert np.linalg.norm(x[i] - xd) <= cond * 1e-12 * np.linalg.norm(xd)
        assert solvers.true_residual(A, b, x[i], s) <= 1.5e-12
        xs, _ = solvers.cg(A, b, s, tol=1e-13)
        assert np.linalg.norm(x[i] - xs) <= cond * 2e-12 * np.linalg.norm(xs)


def test_multishift_single_shift_is_cg(c1):
    """With one shift zeta stays 1 and the iterates are CG's."""
    U, b, m, _ = c1
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    x, info = solvers.multishift_cg(A, b, [0.2], tol=1e-9)
    xc, infoc = solvers.cg(A, b, 0.2, tol=1e-9)
    assert info.iterations == infoc.iterations
    np.testing.assert_allclose(x[0], xc, rtol=0, atol=1e-13)


def test_multishift_offsets_shift_base(c1):
    """A constant added to every shift is the same as adding it to A."""
    U, b, m, _ = c1
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    A2 = lambda v: dirac.mdagm(U, m, v) + 0.25 * v  # noqa: E731
    x1, _ = solvers.multishift_cg(A, b, [0.25, 0.5, 1.25], tol=1e-12)
    x2, _ = solvers.multishift_cg(A2, b, [0.0, 0.25, 1.0], tol=1e-12)
    np.testing.assert_allclose(x1, x2, rtol=0, atol=1e-11)


# ----------------------------------------------------------------- rational


def test_remez_degree_zero_closed_form():
    lo, hi, p = 0.01, 16.01, -0.25
    r = remez_relative(p, 0, lo, hi)
    a, b = lo ** p, hi ** p
    assert r.alpha0 == pytest.approx(2 * a * b / (a + b), rel=1e-14)
    assert r.delta == pytest.approx(abs(b - a) / (a + b), rel=1e-14)


def test_remez_degree_one_brute_force():
    """Independent minimax fit: for each beta the best (alpha0, alpha) is a
    linear program on a dense grid; beta itself is found by a 1-D search."""
    from scipy.optimize import linprog, minimize_scalar

    lo, hi, p = 0.05, 4.0, -0.25
    r = remez_relative(p, 1, lo, hi)
    x = np.geomspace(lo, hi, 3001)
    w = x ** -p

    def lp(beta):
        # variables (alpha0, alpha1, t): minimise t, |alpha0 w + alpha1 w/(x+beta) - 1| <= t
        g = np.stack([w, w / (x + beta)], axis=1)
        A = np.block([[g, -np.ones((x.size, 1))], [-g, -np.ones((x.size, 1))]])
        ub = np.concatenate([np.ones(x.size), -np.ones(x.size)])
        res = linprog([0, 0, 1], A_ub=A, b_ub=ub, bounds=[(None, None)] * 3, method="highs")
        return res.fun, res.x

    best = minimize_scalar(lambda lb: lp(np.exp(lb))[0], bounds=(np.log(1e-3), np.log(10.0)),
                           method="bounded", options=dict(xatol=1e-10))
    delta_bf, (a0, a1, _) = lp(np.exp(best.x))
    assert r.delta == pytest.approx(delta_bf, rel=1e-5)
    assert r.beta[0] == pytest.approx(np.exp(best.x), rel=1e-3)
    assert r.alpha0 == pytest.approx(a0, rel=1e-3)
    assert r.alpha[0] == pytest.approx(a1, rel=1e-3)


def _alternation(r, p, lo, hi, npts=400001):
    """Signed extrema of the relative error, one per run of equal sign.

    Runs whose extremum is far below the levelled error are rounding flicker
    at a zero crossing (FP64 evaluation of r); they are dropped and their
    neighbours of equal sign merged.
    """
    x = np.geomspace(lo, hi, npts)
    e = r(x) / x ** p - 1
    sg = np.sign(e)
    runs = np.split(np.arange(x.size), np.nonzero(np.diff(sg))[0] + 1)
    ext = [float(np.abs(e[idx]).max()) * sg[idx[0]] for idx in runs]
    ext = [v for v in ext if abs(v) > 1e-3 * r.delta]
    merged = []
    for v in ext:
        if merged and np.sign(merged[-1]) == np.sign(v):
            merged[-1] = v if abs(v) > abs(merged[-1]) else merged[-1]
        else:
            merged.append(v)
    return merged


@pytest.mark.parametrize("cfg,p", [(1, -0.25), (2, -0.25), (2, 0.25), (3, -0.25), (5, -0.25),
                                   (1, 0.125), (2, 0.125), (3, 0.125), (5, 0.125)])
def test_workload_rationals_equioscillate(cfg, p):
    """Chebyshev alternation: 2n+2 extrema of alternating sign and equal size."""
    r = rational_for(cfg, p)
    c = synth.CONFIGS[cfg]
    lo = c["m"] ** 2
    ext = _alternation(r, p, lo, 16 + lo)
    assert len(ext) == 2 * r.n + 2
    mags = np.abs(ext)
    # FP64 evaluation of the partial fractions: rounding of order eps times the
    # sum of the absolute terms over |r(x)| (large where the terms of x^{+p}
    # cancel); the extrema are exact in the Remez arithmetic
    x = np.geomspace(lo, 16 + lo, 20001)
    terms = abs(r.alpha0) + sum(abs(a) / (x + b) for a, b in zip(r.alpha, r.beta))
    slack = 16 * np.finfo(float).eps * float(np.max(terms / np.abs(r(x))))
    assert mags.max() <= r.delta * (1 + 1e-4) + slack
    assert mags.min() >= r.delta * (1 - 1e-4) - slack
    assert np.all(np.array(ext[:-1]) * np.array(ext[1:]) < 0)
    # sign structure of the partial fractions
    assert all(b > 0 for b in r.beta)
    if p < 0:
        assert all(a > 0 for a in r.alpha)
    else:
        assert r.alpha0 > 0 and all(a < 0 for a in r.alpha)


def test_rational_apply_error_bound(c1):
    """||r(A) b - A^p b|| <= delta ||A^p b||, and r_+ r_- = 1 within 2 delta."""
    U, b, m, Ad = c1
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    r = rational_for(1, -0.25)
    y, x, info = rational.rational_apply(A, b, r.alpha0, r.alpha, r.beta, tol=1e-12)
    assert info.converged
    exact = rational.dense_function_apply(Ad, b, lambda w: w ** -0.25)
    assert np.linalg.norm(y - exact) <= (r.delta + 1e-11) * np.linalg.norm(exact)
    yd = rational.dense_function_apply(Ad, b, lambda w: rational.scalar_rational(w, r.alpha0, r.alpha, r.beta))
    sol_err = sum(abs(a) * np.linalg.norm(x[i] - solvers.dense_solve(Ad, b, bb))
                  for i, (a, bb) in enumerate(zip(r.alpha, r.beta)))
    assert np.linalg.norm(y - yd) <= sol_err + 1e-14 * np.linalg.norm(yd)


def test_rational_composition_is_identity():
    """r_{+1/4}(A) r_{-1/4}(A) b = b up to 2 delta + solver error (C2 interval)."""
    L = (4, 4, 4, 4)
    m = 0.02
    U = synth.gauge_field(L, 0.5, 1002)
    b = synth.source(L, 2200, 1)[0]
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    rm = rational_for(2, -0.25)
    rp = rational_for(2, 0.25)
    y, _, _ = rational.rational_apply(A, b, rm.alpha0, rm.alpha, rm.beta, tol=1e-13)
    z, _, _ = rational.rational_apply(A, y, rp.alpha0, rp.alpha, rp.beta, tol=1e-13)
    assert np.linalg.norm(z - b) <= (rm.delta + rp.delta + 1e-10) * np.linalg.norm(b)
