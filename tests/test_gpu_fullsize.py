"""Parity at the full sizes of the named workloads, in the benchmark's launch
configuration (tuned launch variants, graphs, block length 10).

At these sizes the oracle cannot solve the systems, so the solutions are
certified by properties that hold at any size:
  * the FP64 true residual ||b - (A + sigma_i) x_i|| / ||b|| <= tol, with A the
    oracle's operator for a sample of (rhs, shift) pairs and the library's FP64
    operator for all of them; the library's FP64 operator is itself compared
    with the oracle's element by element on one full-size vector, and the
    library's outputs A x_ri used for the residuals are tied to the oracle all
    at once: sum_ri c_ri (A x_ri) from the library must equal the oracle's A
    applied to sum_ri c_ri x_ri for random complex c_ri, so (by linearity) a
    wrong output for any single pair fails with probability one, at the cost
    of one oracle application;
  * the rational apply equals alpha0 b + sum alpha_i x_i of the separately
    returned shifted solutions, and r_{+1/4}(A) r_{-1/4}(A) b = b within the two
    approximation errors plus the solver tolerance.
"""

import numpy as np
import pytest

import dslash_bound
import f32layout
import synth
from oracle import dirac, solvers
from synth.make_rational import rational_for
from fieldcache import workload_gauge

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


def _workload(rh, cfg):
    c = synth.CONFIGS[cfg]
    U = workload_gauge(cfg)
    b = synth.source(c["L"], synth.fields.seed_source(cfg), c["nrhs"])
    lat = rh.rhmc_lattice_create(c["L"], -1)
    g = rh.rhmc_gauge_create(lat, np.asarray(U))
    return c, U, b, lat, g


def _gpu_true_residuals(rh, g, m, shifts, b_dev, x_dev, U=None):
    """||b - (A + s) x|| / ||b|| for every (rhs, shift) with the FP64 library
    operator.  With U, also checks sum c_ri (A x_ri) (library) against the
    oracle's A (sum c_ri x_ri) for seeded random complex c_ri."""
    import torch

    nrhs, nshift = x_dev.shape[:2]
    out = torch.empty_like(x_dev[0])
    res = np.zeros((nrhs, nshift))
    # weights c_ri = (standard complex normal) / max|x_ri|, so every pair counts
    # alike; the two sides differ by rounding only, bounded element-wise by
    # (about 100 operations per element of A v, on terms of at most 50 max|v|,
    # both sides) 1e4 * eps * sum_ri |c_ri| max|x_ri|
    rng = np.random.default_rng(4242)
    c = rng.standard_normal((nrhs, nshift)) + 1j * rng.standard_normal((nrhs, nshift))
    xmax = torch.amax(torch.abs(x_dev), dim=(2, 3)).cpu().numpy()
    c = c / xmax
    acc_ax = torch.zeros_like(x_dev[0, 0])
    acc_x = torch.zeros_like(x_dev[0, 0])
    for r in range(nrhs):
        rh.rhmc_apply_mdagm(g, m, rh.RHMC_PREC_FP64, nshift, x_dev[r], out)
        for i, s in enumerate(shifts):
            d = b_dev[r] - out[i] - s * x_dev[r, i]
            res[r, i] = (torch.linalg.vector_norm(d) / torch.linalg.vector_norm(b_dev[r])).item()
            acc_ax += complex(c[r, i]) * out[i]
            acc_x += complex(c[r, i]) * x_dev[r, i]
    if U is not None:
        want = dirac.mdagm(U, m, acc_x.cpu().numpy())
        got = acc_ax.cpu().numpy()
        bound = 1e4 * np.finfo(np.float64).eps * float(np.sum(np.abs(c) * xmax))
        assert np.abs(got - want).max() <= bound
    return res


def _check_operator_fullsize(rh, g, U, m, v):
    """The library's FP64 A against the oracle's on one full-size vector."""
    import torch

    out = torch.empty((1, 3, v.shape[-1]), dtype=torch.complex128, device="cuda:0")
    rh.rhmc_apply_mdagm(g, m, rh.RHMC_PREC_FP64, 1, _dev(v[None]), out)
    ref = dirac.mdagm(U, m, v)
    got = out.cpu().numpy()[0]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_c2_fullsize_fp64(rh):
    """16^3x4, FP64, 15-pole x^-1/4 and x^+1/4, tol 1e-10."""
    import torch

    c, U, b, lat, g = _workload(rh, 2)
    U = np.asarray(U)
    m, tol = c["m"], c["tol"]
    rm, rp = rational_for(2, -0.25), rational_for(2, 0.25)
    prm = rh.solver_params(tol=tol, mode=rh.RHMC_MODE_FP64, tune=1)
    bd = _dev(b)
    x = torch.empty((1, 15, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_multishift_cg(g, m, rm.beta, bd, x, prm)
    xs = x.cpu().numpy()
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for i, s in enumerate(rm.beta):
        assert solvers.true_residual(A, b[0], xs[0, i], s) <= tol
    assert st["max_true_residual"] <= tol
    # rational apply = combination of the returned shifted solutions
    y = torch.empty_like(bd)
    rh.rhmc_rational_apply(g, m, rm.alpha0, rm.alpha, rm.beta, bd, y, prm)
    comb = rm.alpha0 * b[0] + np.tensordot(np.asarray(rm.alpha), xs[0], axes=1)
    yn = y.cpu().numpy()[0]
    assert np.linalg.norm(yn - comb) <= 1e-12 * np.linalg.norm(comb)
    # r_{+1/4}(A) r_{-1/4}(A) b = b
    z = torch.empty_like(bd)
    rh.rhmc_rational_apply(g, m, rp.alpha0, rp.alpha, rp.beta, y, z, prm)
    err = np.linalg.norm(z.cpu().numpy() - b) / np.linalg.norm(b)
    assert err <= rm.delta + rp.delta + 1e-8
    _check_operator_fullsize(rh, g, U, m, b[0])
    g.close()


def test_c3_fullsize_mixed(rh):
    """32^3x8, MIXED (FP32 12-real operator, FP64 reliable updates), 15 poles."""
    import torch

    c, U, b, lat, g = _workload(rh, 3)
    U = np.asarray(U)
    m, tol = c["m"], c["tol"]
    r = rational_for(3, -0.25)
    bd = _dev(b)
    x = torch.empty((1, 15, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_multishift_cg(g, m, r.beta, bd, x,
                               rh.solver_params(tol=tol, mode=rh.RHMC_MODE_MIXED, tune=1))
    xs = x.cpu().numpy()
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for i, s in enumerate(r.beta):
        assert solvers.true_residual(A, b[0], xs[0, i], s) <= tol
    # error against the FP64 solve of the same systems, per shift
    x64 = torch.empty_like(x)
    rh.rhmc_multishift_cg(g, m, r.beta, bd, x64,
                          rh.solver_params(tol=tol, mode=rh.RHMC_MODE_FP64, tune=1))
    x64 = x64.cpu().numpy()
    for i, s in enumerate(r.beta):
        kappa = (16 + m * m + s) / (m * m + s)
        rel = np.linalg.norm(xs[0, i] - x64[0, i]) / np.linalg.norm(x64[0, i])
        assert rel <= 2 * kappa * tol
    assert st["reliable_updates"] > 0
    g.close()


def test_c4_fullsize_mixed_batched(rh):
    """32^3x8, 8 pseudofermion sources x 15 shifts, MIXED, batched."""
    import torch

    c, U, b, lat, g = _workload(rh, 4)
    U = np.asarray(U)
    m, tol = c["m"], c["tol"]
    r = rational_for(4, -0.25)
    bd = _dev(b)
    x = torch.empty((8, 15, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    rh.rhmc_multishift_cg(g, m, r.beta, bd, x,
                          rh.solver_params(tol=tol, mode=rh.RHMC_MODE_MIXED, tune=1))
    res = _gpu_true_residuals(rh, g, m, r.beta, bd, x, U)
    assert res.max() <= tol * (1 + 1e-6)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for (rr, i) in ((0, 0), (7, 14), (3, 7)):
        xi = x[rr, i].cpu().numpy()
        assert solvers.true_residual(A, b[rr], xi, r.beta[i]) <= tol
    g.close()


def test_c5_hopping_kernels_fullsize(rh):
    """48^3x12, the four sources of the workload: the FP32-12 (paired vectors)
    and FP64-12 hopping launches in the library's default launch variants,
    which the bench times, against the oracle on every output element: FP32
    within its rounding bound (32 * 2^-24 of 1/2 sum |U| |psi|), FP64 to 1e-13
    of the largest element."""
    import torch

    c, U, b, lat, g = _workload(rh, 5)
    U = np.asarray(U)
    for out_par in (1, 0):
        want = dirac.dslash(U, b, out_par)
        vin = _dev(b)
        out = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, out_par, rh.RHMC_PREC_FP64, 4, vin, out)
        got = out.cpu().numpy()
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
        b32 = b.astype(np.complex64)
        vin = _dev(f32layout.pack(b32))
        out = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, out_par, rh.RHMC_PREC_FP32, 4, vin, out)
        got = f32layout.unpack(out.cpu().numpy(), 4, lat.Vh).astype(np.complex128)
        b64 = b32.astype(np.complex128)
        want = dirac.dslash(U, b64, out_par)
        bound = 32 * 2.0 ** -24 * dslash_bound.abs_scale(U, b64, out_par) + 1e-30
        err = np.abs(got - want)
        assert np.all(err <= bound), float((err / bound).max())
    g.close()


def test_c5_fullsize_mixed_batched(rh):
    """48^3x12, 4 sources x 20-pole x^-1/4, MIXED batched, tol 1e-10."""
    import torch

    c, U, b, lat, g = _workload(rh, 5)
    U = np.asarray(U)
    m, tol = c["m"], c["tol"]
    r = rational_for(5, -0.25)
    bd = _dev(b)
    x = torch.empty((4, 20, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_multishift_cg(g, m, r.beta, bd, x,
                               rh.solver_params(tol=tol, mode=rh.RHMC_MODE_MIXED, tune=1))
    assert st["max_true_residual"] <= tol
    res = _gpu_true_residuals(rh, g, m, r.beta, bd, x, U)
    assert res.max() <= tol * (1 + 1e-6)
    # the rational apply in the same configuration equals the combination
    y = torch.empty_like(bd)
    rh.rhmc_rational_apply(g, m, r.alpha0, r.alpha, r.beta, bd, y,
                           rh.solver_params(tol=tol, mode=rh.RHMC_MODE_MIXED, tune=1))
    alpha = torch.tensor(r.alpha, dtype=torch.complex128, device="cuda:0")
    comb = r.alpha0 * bd + torch.einsum("i,rick->rck", alpha, x)
    # the solves are deterministic (fixed-order reductions, same launch
    # variants), so only the summation order of the combine differs
    d = (torch.linalg.vector_norm(y - comb) / torch.linalg.vector_norm(comb)).item()
    assert d <= 1e-12
    # the oracle's operator on a sample, and the library's FP64 operator against it
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for (rr, i) in ((0, 0), (2, 19)):
        xi = x[rr, i].cpu().numpy()
        assert solvers.true_residual(A, b[rr], xi, r.beta[i]) <= tol
    _check_operator_fullsize(rh, g, U, m, b[1])
    g.close()


def test_edge_sizes(rh):
    """Empty batch rejected, 32 shifts, more right-hand sides than one group."""
    import torch

    L = (4, 4, 4, 6)
    m = 0.1
    U = synth.gauge_field(L, 0.5, 7000)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    empty = torch.empty((0, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(rh.RhmcError):
        rh.rhmc_multishift_cg(g, m, [0.1], empty,
                              torch.empty((0, 1, 3, lat.Vh), dtype=torch.complex128, device="cuda:0"))
    shifts = np.geomspace(1e-4, 50.0, 32)
    b = synth.source(L, 7001, 19)
    x = torch.empty((19, 32, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    rh.rhmc_multishift_cg(g, m, shifts, _dev(b), x, rh.solver_params(tol=1e-10, mode=rh.RHMC_MODE_MIXED))
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    xs = x.cpu().numpy()
    for rr in (0, 8, 18):
        for i in (0, 15, 31):
            assert solvers.true_residual(A, b[rr], xs[rr, i], shifts[i]) <= 1e-10
    g.close()
