"""GPU parity of the multi-shift CG and the rational apply (through the C ABI).

The solvers reach x_i = (A + sigma_i)^-1 b to a tolerance, so their outputs
are certified by the oracle: dense direct solves on tiny lattices
(||x - x_dense|| <= kappa_i * tol * ||x_dense||) and, on every lattice, the
true residual ||b - (A + sigma_i) x_i|| / ||b|| <= tol recomputed with the
oracle's FP64 operator.  Iteration counts are reported, not compared.
"""

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


def _setup(rh, L, eps, seed, nrhs, src_seed, t_bc=-1):
    U = synth.gauge_field(L, eps, seed)
    b = synth.source(L, src_seed, nrhs)
    lat = rh.rhmc_lattice_create(L, t_bc)
    g = rh.rhmc_gauge_create(lat, U)
    return U, b, lat, g


def _solve(rh, g, lat, m, shifts, b, **kw):
    import torch

    x = torch.empty((b.shape[0], len(shifts), 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    allow = kw.pop("allow_not_converged", False)
    st = rh.rhmc_multishift_cg(g, m, shifts, _to(b), x, rh.solver_params(**kw),
                               allow_not_converged=allow)
    return x.cpu().numpy(), st


def test_c1_fp64_matches_dense_solves(rh):
    """4^4, eps 0.5, m 0.1, 8-pole x^-1/4 on [m^2, 16+m^2], tol 1e-12."""
    c = synth.CONFIGS[1]
    U, b, lat, g = _setup(rh, c["L"], c["eps"], synth.fields.seed_gauge(1), 1,
                          synth.fields.seed_source(1))
    m = c["m"]
    r = rational_for(1, -0.25)
    x, st = _solve(rh, g, lat, m, r.beta, b, tol=1e-12, mode=rh.RHMC_MODE_FP64)
    Ad = dirac.dense_A(U, m)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for i, s in enumerate(r.beta):
        xd = solvers.dense_solve(Ad, b[0], s)
        kappa = np.linalg.cond(Ad + s * np.eye(Ad.shape[0]))
        assert np.linalg.norm(x[0, i] - xd) <= kappa * 1e-12 * np.linalg.norm(xd)
        assert solvers.true_residual(A, b[0], x[0, i], s) <= 1e-12
    assert st["max_true_residual"] <= 1e-12
    # the library's own FP64 true residuals agree with the oracle's
    for i, s in enumerate(r.beta):
        ores = solvers.true_residual(A, b[0], x[0, i], s)
        assert st["true_residual"][0, i] == pytest.approx(ores, rel=1e-3, abs=1e-15)
    # rational apply: y = alpha0 b + sum alpha_i x_i against the dense oracle
    import torch

    y = torch.empty((1, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    rh.rhmc_rational_apply(g, m, r.alpha0, r.alpha, r.beta, _to(b), y,
                           rh.solver_params(tol=1e-12))
    yd = rational.dense_function_apply(
        Ad, b[0], lambda w: rational.scalar_rational(w, r.alpha0, r.alpha, r.beta))
    bound = sum(abs(a) * np.linalg.cond(Ad + s * np.eye(Ad.shape[0])) * 1e-12 *
                np.linalg.norm(solvers.dense_solve(Ad, b[0], s)) for a, s in zip(r.alpha, r.beta))
    assert np.linalg.norm(y.cpu().numpy()[0] - yd) <= bound + 1e-14 * np.linalg.norm(yd)
    exact = rational.dense_function_apply(Ad, b[0], lambda w: w ** -0.25)
    assert np.linalg.norm(y.cpu().numpy()[0] - exact) <= (r.delta + 1e-10) * np.linalg.norm(exact)
    g.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
@pytest.mark.parametrize("L,nrhs", [((6, 4, 4, 8), 3), ((8, 8, 8, 6), 2), ((2, 2, 2, 2), 1)])
def test_multishift_true_residuals(rh, mode, L, nrhs):
    m = 0.05
    U, b, lat, g = _setup(rh, L, 0.7, 5000 + sum(L), nrhs, 6000)
    shifts = np.array([0.0, 1e-3, 0.02, 0.3, 1.5, 7.0])
    md = rh.RHMC_MODE_FP64 if mode == "fp64" else rh.RHMC_MODE_MIXED
    x, st = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=md)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for r in range(nrhs):
        for i, s in enumerate(shifts):
            assert solvers.true_residual(A, b[r], x[r, i], s) <= 1e-10
    # larger shifts converge no later than smaller ones
    its = st["iterations"]
    assert np.all(np.diff(its, axis=1) <= 0)
    g.close()


@pytest.mark.parametrize("block,use_graph", [(1, 1), (3, 0), (7, 1), (16, 1), (20, 0), (32, 1), (41, 0), (50, 1)])
def test_block_lengths_and_graph(rh, block, use_graph):
    L = (8, 8, 8, 6)
    m = 0.03
    U, b, lat, g = _setup(rh, L, 0.6, 5100, 2, 6100)
    shifts = np.array([0.002, 0.05, 0.9])
    for mode in (rh.RHMC_MODE_FP64, rh.RHMC_MODE_MIXED):
        x, st = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=mode, block=block,
                       use_graph=use_graph)
        A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
        for r in range(2):
            for i, s in enumerate(shifts):
                assert solvers.true_residual(A, b[r], x[r, i], s) <= 1e-10
    g.close()


def test_graph_replay_is_bit_identical_to_eager(rh):
    L = (8, 8, 8, 6)
    U, b, lat, g = _setup(rh, L, 0.6, 5200, 2, 6200)
    shifts = np.array([0.0, 0.01, 0.5])
    for mode in (rh.RHMC_MODE_FP64, rh.RHMC_MODE_MIXED):
        x1, s1 = _solve(rh, g, lat, 0.04, shifts, b, tol=1e-10, mode=mode, use_graph=1)
        x2, s2 = _solve(rh, g, lat, 0.04, shifts, b, tol=1e-10, mode=mode, use_graph=0)
        x3, s3 = _solve(rh, g, lat, 0.04, shifts, b, tol=1e-10, mode=mode, use_graph=1)
        assert np.array_equal(x1, x2) and np.array_equal(x1, x3)
        assert s1["total_iterations"] == s2["total_iterations"] == s3["total_iterations"]
    g.close()


@pytest.mark.parametrize("nrhs", [8, 11])
def test_batched_rhs(rh, nrhs):
    """Several pseudofermions at once (groups of eight share each link read)."""
    L = (4, 4, 4, 8)
    m = 0.02
    U, b, lat, g = _setup(rh, L, 0.7, 5300, nrhs, 6300)
    shifts = np.array([0.0, 0.004, 0.1, 2.0])
    x, st = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=rh.RHMC_MODE_MIXED)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for r in range(nrhs):
        for i, s in enumerate(shifts):
            assert solvers.true_residual(A, b[r], x[r, i], s) <= 1e-10
    # each right-hand side equals its own single solve to the tolerance scale
    x1, _ = _solve(rh, g, lat, m, shifts, b[3:4], tol=1e-10, mode=rh.RHMC_MODE_MIXED)
    assert np.linalg.norm(x1[0] - x[3]) <= 1e-6 * np.linalg.norm(x[3])
    g.close()


def test_unsorted_shifts_and_periodic_time(rh):
    L = (4, 4, 4, 4)
    m = 0.1
    U, b, lat, g = _setup(rh, L, 0.5, 5400, 1, 6400, t_bc=1)
    shifts = np.array([0.5, 0.0, 3.0, 0.02])
    x, _ = _solve(rh, g, lat, m, shifts, b, tol=1e-11, mode=rh.RHMC_MODE_FP64)
    Ad = dirac.dense_A(U, m, t_bc=1)
    for i, s in enumerate(shifts):
        xd = solvers.dense_solve(Ad, b[0], s)
        kappa = np.linalg.cond(Ad + s * np.eye(Ad.shape[0]))
        assert np.linalg.norm(x[0, i] - xd) <= kappa * 1e-11 * np.linalg.norm(xd)
    g.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_zero_source_gives_zero(rh, mode):
    """A zero right-hand side beside a nonzero one: done from the start (in
    MIXED mode through the FP64 phase, the switch, reliable updates and the
    true-residual check), its solutions exactly zero."""
    L = (4, 4, 4, 4)
    U, b, lat, g = _setup(rh, L, 0.5, 5500, 2, 6500)
    b[1] = 0
    md = rh.RHMC_MODE_FP64 if mode == "fp64" else rh.RHMC_MODE_MIXED
    x, st = _solve(rh, g, lat, 0.1, [0.0, 0.3], b, tol=1e-10, mode=md)
    assert np.all(x[1] == 0)
    assert st["true_residual"][1].max() == 0 and st["iterations"][1].max() == 0
    A = lambda v: dirac.mdagm(U, 0.1, v)  # noqa: E731
    assert solvers.true_residual(A, b[0], x[0, 0], 0.0) <= 1e-10
    g.close()


def test_not_converged_reports_stats(rh):
    L = (8, 8, 8, 6)
    U, b, lat, g = _setup(rh, L, 0.6, 5600, 1, 6600)
    x, st = _solve(rh, g, lat, 0.01, [0.0, 0.1], b, tol=1e-10, maxiter=20, refine=0,
                   allow_not_converged=True)
    assert st["status"] == rh.RHMC_ERR_NOT_CONVERGED
    assert st["total_iterations"] >= 20
    assert st["max_true_residual"] > 1e-10
    g.close()


def test_nonfinite_source_rejected(rh):
    L = (4, 4, 4, 4)
    U, b, lat, g = _setup(rh, L, 0.5, 5700, 1, 6700)
    b[0, 1, 3] = np.nan
    with pytest.raises(rh.RhmcError) as e:
        _solve(rh, g, lat, 0.1, [0.0], b)
    assert e.value.status == rh.RHMC_ERR_NONFINITE
    g.close()


def test_invalid_shifts_rejected(rh):
    L = (4, 4, 4, 4)
    U, b, lat, g = _setup(rh, L, 0.5, 5800, 1, 6800)
    for m, shifts in ((0.1, [-0.1]), (0.0, [0.0, 1.0]), (0.1, [np.inf])):
        with pytest.raises(rh.RhmcError) as e:
            _solve(rh, g, lat, m, shifts, b)
        assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    g.close()


def test_refinement_batch_larger_than_rhs_count(rh):
    """Regression: refining more shifts than there are right-hand sides grows
    the workspace in the middle of a call; the call must keep working."""
    L = (8, 8, 8, 6)
    m = 0.05
    U, b, lat, g = _setup(rh, L, 0.7, 5900, 1, 6900)
    shifts = np.array([0.0, 1e-3, 0.02, 0.3, 1.5, 7.0, 20.0, 50.0])
    x, st = _solve(rh, g, lat, m, shifts, b, tol=3e-12, mode=rh.RHMC_MODE_MIXED)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for i, s in enumerate(shifts):
        assert solvers.true_residual(A, b[0], x[0, i], s) <= 3e-12
    # a second, larger solve on the same gauge object after the growth
    b2 = synth.source(L, 6901, 3)
    x2, _ = _solve(rh, g, lat, m, shifts[:3], b2, tol=1e-10, mode=rh.RHMC_MODE_MIXED)
    for r in range(3):
        for i, s in enumerate(shifts[:3]):
            assert solvers.true_residual(A, b2[r], x2[r, i], s) <= 1e-10
    g.close()


def test_mixed_solve_with_hilo_links_only(rh):
    """With only the hi/lo planes stored, reliable updates and the true
    residual use the hi + lo FP64 operator; the oracle certifies every shift.
    The hi + lo operator differs from the FP64 one by ~1e-13 ||x|| (relative
    link error ~2^-47 through ||D|| <= 4), so the shifts keep ||x|| / ||b|| <=
    1 / (m^2 + 0.01) ~ 92 and that difference far below tol."""
    L = (8, 8, 8, 6)
    m = 0.03
    U = synth.gauge_field(L, 0.6, 5300)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U, flags=rh.RHMC_LINKS_HILO_12)
    b = synth.source(L, 6300, 2)
    shifts = np.array([0.01, 0.05, 0.3, 2.0])
    import torch

    x = torch.empty((2, shifts.size, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_multishift_cg(g, m, shifts, torch.from_numpy(b).to("cuda:0"), x,
                               rh.solver_params(tol=1e-10, mode=rh.RHMC_MODE_MIXED))
    assert st["reliable_updates"] > 0
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    xs = x.cpu().numpy()
    for r in range(2):
        for i, s in enumerate(shifts):
            assert solvers.true_residual(A, b[r], xs[r, i], s) <= 1e-10
    g.close()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
@pytest.mark.parametrize("L,nrhs,shifts", [((6, 4, 4, 8), 3, [0.0, 1e-3, 0.05, 0.7, 3.0]),
                                           ((8, 8, 8, 6), 2, [2e-4, 0.01, 0.5]),
                                           ((4, 4, 4, 4), 4, [0.001, 0.02, 0.1, 0.4, 1.5, 6.0])])
def test_per_shift_solver(rh, mode, L, nrhs, shifts):
    """per_shift = 1: every shifted system solved by its own CG from a zero
    start (batches of up to 8 systems, more than 8 here in the first case);
    certified by the oracle's FP64 true residual, and equal to the
    multi-shift answer within the conditioning of each shift."""
    m = 0.05
    U, b, lat, g = _setup(rh, L, 0.6, 9000 + sum(L), nrhs, 9100)
    md = rh.RHMC_MODE_FP64 if mode == "fp64" else rh.RHMC_MODE_MIXED
    x1, st1 = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=md, per_shift=1)
    x2, _ = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=md)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for r in range(nrhs):
        for i, s in enumerate(shifts):
            assert solvers.true_residual(A, b[r], x1[r, i], s) <= 1e-10
            kappa = (16.0 + m * m + s) / (m * m + s)
            err = np.linalg.norm(x1[r, i] - x2[r, i]) / np.linalg.norm(x2[r, i])
            assert err <= 2e-10 * kappa, (r, s, err)
    assert st1["max_true_residual"] <= 1e-10
    # every system reports its own iteration count; larger shifts need fewer
    it = st1["iterations"]
    assert (it > 0).all() and (it[:, -1] <= it[:, 0]).all()
    g.close()


def test_mixed_solve_with_non_su3_links(rh):
    """Links that are not SU(3): the default storage is FP32-18 + FP64-18 and
    the MIXED multi-shift solve still meets the oracle's FP64 true residual."""
    L = (6, 4, 4, 8)
    U0 = synth.gauge_field(L, 0.6, 9300)
    rng = np.random.default_rng(9301)
    U = U0 + 0.3 * (rng.standard_normal(U0.shape) + 1j * rng.standard_normal(U0.shape))
    b = synth.source(L, 9302, 2)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    m = 0.1
    shifts = [0.0, 0.01, 0.3, 2.0]
    x, st = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=rh.RHMC_MODE_MIXED)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for r in range(2):
        for i, s in enumerate(shifts):
            assert solvers.true_residual(A, b[r], x[r, i], s) <= 1e-10
    g.close()


@pytest.mark.parametrize("head,use_graph,block", [(0.0, 1, 25), (1e-3, 1, 25), (0.0, 0, 7)])
def test_mixed_fp64_head(rh, head, use_graph, block):
    """8^4, eps 0.8, m 0.005, 2 rhs, the 20-pole x^-1/4 of the 48^3x12
    workload, tol 1e-10.  The MIXED shared solve iterates in FP64 until
    ||r|| <= head ||b|| (0: the automatic 1e-2), then in FP32 with reliable
    updates.  Every shift must meet tol (oracle FP64 true residual), and the
    refinement the shifted systems need must fall below that of the same
    solve in FP32 from the first iteration (fp64_head < 0).  Graph replay and
    eager launches with an odd block length both take the switch."""
    L = (8, 8, 8, 8)
    U, b, lat, g = _setup(rh, L, 0.8, 5151, 2, 6151)
    m = 0.005
    r = rational_for(5, -0.25)
    assert len(r.beta) == 20 and synth.CONFIGS[5]["m"] == m
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    kw = dict(tol=1e-10, mode=rh.RHMC_MODE_MIXED, use_graph=use_graph, block=block)
    x, st = _solve(rh, g, lat, m, r.beta, b, fp64_head=head, **kw)
    assert 0 < st["fp64_head_iterations"] < st["total_iterations"]
    for j in range(2):
        for i, s in enumerate(r.beta):
            assert solvers.true_residual(A, b[j], x[j, i], s) <= 1e-10
    x0, st0 = _solve(rh, g, lat, m, r.beta, b, fp64_head=-1.0, **kw)
    assert st0["fp64_head_iterations"] == 0
    print(f"head {head}: FP64 iterations {st['fp64_head_iterations']} of {st['total_iterations']}, "
          f"refine {int(st['refine_iterations'].sum())} vs {int(st0['refine_iterations'].sum())} "
          f"without the FP64 phase")
    assert st["refine_iterations"].sum() < st0["refine_iterations"].sum()
    # the two solves agree to the accuracy both certify
    for j in range(2):
        for i in range(len(r.beta)):
            kappa = (16.0 + m * m + r.beta[i]) / (m * m + r.beta[i])
            assert np.linalg.norm(x[j, i] - x0[j, i]) <= 2e-10 * kappa * np.linalg.norm(x0[j, i])
    with pytest.raises(rh.RhmcError) as e:
        _solve(rh, g, lat, m, r.beta, b, mode=rh.RHMC_MODE_MIXED, fp64_head=float("nan"))
    assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    g.close()


def test_mixed_fp64_head_below_tol_is_the_fp64_solve(rh):
    """With the FP64 phase threshold below tol the phase runs to convergence:
    the MIXED call then launches exactly the kernels of the plain FP64 solve
    with the same block length (MIXED turns the default 32 into 25, a divisor
    of the 50 iterations between replacements), so with deterministic
    reductions the solutions are bit-identical."""
    L = (6, 4, 4, 8)
    U, b, lat, g = _setup(rh, L, 0.6, 5252, 3, 6252)
    m = 0.02
    shifts = rational_for(1, -0.25).beta
    x64, st64 = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=rh.RHMC_MODE_FP64, block=25)
    xm, stm = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=rh.RHMC_MODE_MIXED, fp64_head=1e-12)
    assert stm["fp64_head_iterations"] == stm["total_iterations"] == st64["total_iterations"]
    assert stm["reliable_updates"] == 0
    assert st64["refine_rounds"] == 0 and stm["refine_rounds"] == 0
    assert np.array_equal(xm, x64)
    g.close()


def test_true_residual_check_trips_without_reliable_updates(rh):
    """Failure detection: a MIXED solve of one system with residual
    replacement effectively off (and no FP64 phase, no refinement) lets the
    FP32 recursion report convergence while the true residual has stalled far
    above tol; the FP64 check must return NOT_CONVERGED with the stalled
    residual in the statistics.  With replacement every 50 iterations the same
    solve meets tol (Sec. 4.3, residual replacement)."""
    L = (8, 8, 8, 6)
    U, b, lat, g = _setup(rh, L, 0.6, 5901, 1, 6901)
    m = 0.01
    kw = dict(tol=1e-10, mode=rh.RHMC_MODE_MIXED, refine=0, fp64_head=-1.0, maxiter=20000)
    x, st = _solve(rh, g, lat, m, [0.0], b, reliable_every=10**9, allow_not_converged=True, **kw)
    print(f"no replacement: {st['total_iterations']} iterations, true residual "
          f"{st['max_true_residual']:.2e}")
    assert st["status"] == rh.RHMC_ERR_NOT_CONVERGED
    assert st["reliable_updates"] == 0
    assert st["max_true_residual"] > 1e-8
    x, st = _solve(rh, g, lat, m, [0.0], b, reliable_every=50, **kw)
    assert st["status"] == rh.RHMC_OK and st["reliable_updates"] > 0
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    assert solvers.true_residual(A, b[0], x[0, 0], 0.0) <= 1e-10
    g.close()


def test_invalid_solver_params_rejected(rh):
    L = (4, 4, 4, 4)
    U, b, lat, g = _setup(rh, L, 0.5, 5950, 1, 6950)
    bad = [dict(block=0), dict(block=51), dict(reliable_every=0), dict(maxiter=0), dict(tol=0.0),
           dict(tol=float("nan")), dict(mode=7)]
    for kw in bad:
        with pytest.raises(rh.RhmcError) as e:
            _solve(rh, g, lat, 0.1, [0.0, 0.2], b, **kw)
        assert e.value.status == rh.RHMC_ERR_INVALID_ARG, kw
    # the bounds themselves are accepted
    for kw in (dict(block=1), dict(block=50, mode=rh.RHMC_MODE_MIXED)):
        x, st = _solve(rh, g, lat, 0.1, [0.0, 0.2], b, tol=1e-10, **kw)
        assert st["max_true_residual"] <= 1e-10
    g.close()


@pytest.mark.parametrize("nrhs", [9, 16])
def test_not_converged_groups_all_written(rh, nrhs):
    """More than eight right-hand sides run as groups of eight.  A group that
    ends NOT_CONVERGED (maxiter too small) keeps its last iterates, and every
    later group is still solved: every x, y, S and stat is written and equals
    what the same group gives when solved alone."""
    import torch

    L = (8, 8, 4, 4)
    m = 0.01
    U, b, lat, g = _setup(rh, L, 0.6, 5800, nrhs, 6800)
    shifts = [0.0, 0.05]
    kw = dict(tol=1e-10, maxiter=30, refine=0)
    x = torch.full((nrhs, len(shifts), 3, lat.Vh), float("nan"), dtype=torch.complex128,
                   device="cuda:0")
    st = rh.rhmc_multishift_cg(g, m, shifts, _to(b), x, rh.solver_params(**kw),
                               allow_not_converged=True)
    assert st["status"] == rh.RHMC_ERR_NOT_CONVERGED
    xs = x.cpu().numpy()
    assert np.all(np.isfinite(xs)) and np.all(np.abs(xs).reshape(nrhs, -1).max(axis=1) > 0)
    assert np.all(st["iterations"] > 0) and np.all(np.isfinite(st["true_residual"]))
    assert np.all(st["true_residual"] > 1e-10)
    x8, st8 = _solve(rh, g, lat, m, shifts, b[8:], allow_not_converged=True, **kw)
    assert np.array_equal(xs[8:], x8)
    assert np.array_equal(st["true_residual"][8:], st8["true_residual"])

    r = rational_for(1, -0.25)
    y = torch.full((nrhs, 3, lat.Vh), float("nan"), dtype=torch.complex128, device="cuda:0")
    st = rh.rhmc_rational_apply(g, m, r.alpha0, r.alpha, r.beta, _to(b), y, rh.solver_params(**kw),
                                allow_not_converged=True)
    assert st["status"] == rh.RHMC_ERR_NOT_CONVERGED
    ys = y.cpu().numpy()
    assert np.all(np.isfinite(ys))
    y8 = torch.empty((nrhs - 8, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    rh.rhmc_rational_apply(g, m, r.alpha0, r.alpha, r.beta, _to(b[8:]), y8, rh.solver_params(**kw),
                           allow_not_converged=True)
    assert np.array_equal(ys[8:], y8.cpu().numpy())

    S, st = rh.rhmc_pf_action(g, m, r.alpha0, r.alpha, r.beta, _to(b), rh.solver_params(**kw),
                              allow_not_converged=True)
    assert st["status"] == rh.RHMC_ERR_NOT_CONVERGED
    assert np.all(np.isfinite(S)) and np.all(S > 0)
    S8, _ = rh.rhmc_pf_action(g, m, r.alpha0, r.alpha, r.beta, _to(b[8:]), rh.solver_params(**kw),
                              allow_not_converged=True)
    assert np.array_equal(S[8:], S8)
    g.close()


@pytest.mark.parametrize("reliable_every,block", [(50, 32), (30, 32), (50, 50)])
def test_mixed_replacement_cadence_is_exact(rh, reliable_every, block):
    """MIXED replaces the residual every reliable_every FP32 iterations
    exactly: the block length is the divisor of reliable_every nearest to the
    requested one (25 for 50 and 32, 30 for 30 and 32), so the count of
    replacements is the FP32 iteration count divided by reliable_every."""
    L = (8, 8, 8, 8)
    m = 0.05
    U, b, lat, g = _setup(rh, L, 0.6, 5900, 1, 6900)
    x, st = _solve(rh, g, lat, m, [0.0], b, tol=1e-10, mode=rh.RHMC_MODE_MIXED,
                   reliable_every=reliable_every, block=block, fp64_head=-1.0, refine=0)
    it = st["total_iterations"]
    assert it > 2 * reliable_every
    assert st["reliable_updates"] in (it // reliable_every - 1, it // reliable_every)
    res = solvers.true_residual(lambda v: dirac.mdagm(U, m, v), b[0], x[0, 0], 0.0)
    assert res <= 1e-10
    g.close()


def test_mixed_pairs_with_finished_and_equal_members(rh):
    """FP32 iteration vectors of several systems are stored in pairs: a pair
    whose first member is finished from the start (a zero source) must keep
    iterating its second member, and equal sources solved in different pairs
    and pair halves must give the same solutions.  Sources: 0: random, 1:
    zero, 2 and 4: copies of 0, 3: random (five systems: the last pair has an
    absent partner)."""
    L = (6, 4, 4, 8)
    m = 0.05
    U, b, lat, g = _setup(rh, L, 0.6, 5900, 5, 6900)
    b[1] = 0.0
    b[2] = b[0]
    b[4] = b[0]
    shifts = np.array([0.0, 0.01, 0.3, 2.0])
    x, st = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=rh.RHMC_MODE_MIXED)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    assert np.all(x[1] == 0)
    for r in (0, 2, 3, 4):
        for i, s in enumerate(shifts):
            assert solvers.true_residual(A, b[r], x[r, i], s) <= 1e-10, (r, i)
    for r in (2, 4):
        assert np.linalg.norm(x[r] - x[0]) <= 1e-13 * np.linalg.norm(x[0]), r
    g.close()


@pytest.mark.parametrize("nrhs", [3, 5, 8])
def test_rhs_tiled_launch_variants_in_the_solver(rh, nrhs):
    """Launch variants with an rhs tile (a class of four or eight right-hand
    sides split into two launches) keep one layout of the block partial sums:
    a MIXED solve with tiled FP32 and FP64 variants pinned reaches the
    tolerance for every system and shift, and agrees with the untiled solve to
    the tolerance scale."""
    L = (6, 4, 4, 8)
    m = 0.05
    U, b, lat, g = _setup(rh, L, 0.6, 6100, nrhs, 7100)
    shifts = np.array([0.0, 0.01, 0.3])
    x0, _ = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=rh.RHMC_MODE_MIXED)
    tiled = 96 + 36   # staged rows, two-hop batches, z-tiles of 6, rhs tile
    for prec in (rh.RHMC_PREC_FP32, rh.RHMC_PREC_FP64):
        rh.rhmc_set_dslash_variant(g, prec, nrhs, tiled)
        rh.rhmc_set_dslash_variant(g, prec, 1, 96 + 12)   # refinement systems one at a time
    x, st = _solve(rh, g, lat, m, shifts, b, tol=1e-10, mode=rh.RHMC_MODE_MIXED)
    A = lambda v: dirac.mdagm(U, m, v)  # noqa: E731
    for r in range(nrhs):
        for i, s in enumerate(shifts):
            assert solvers.true_residual(A, b[r], x[r, i], s) <= 1e-10, (r, i)
    assert np.linalg.norm(x - x0) <= 1e-7 * np.linalg.norm(x0)
    g.close()
