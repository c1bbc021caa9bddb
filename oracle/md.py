"""Molecular dynamics and the trajectory of the Phi algorithm (oracle; test
infrastructure only).

Sec. 2.1: the momenta H_mu(n) are conjugate to the links; the Hamiltonian is
sum Tr(H^2) + S_g + S_f; the equations of motion are integrated with a
symmetric symplectic scheme, and a Metropolis test on the change of the
Hamiltonian makes the update exact.  The paper's runs use the second-order
minimum-norm (2MN) scheme with the action split into a fermion and a gauge
part integrated on two time scales (multi-step).

One 2MN step of size h, for a kick P(c) (momenta, omega -= c * coefficients
of the force) and a drift Q(c) (links, U -> exp(i c H) U):

    P(lam h) Q(h/2) P((1 - 2 lam) h) Q(h/2) P(lam h)

Multi-step reading: the outer scheme, of step delta = tau / n_md, kicks with
the fermion force; each of its two drifts Q(delta/2) is replaced by
gauge_steps/2 inner 2MN steps of size delta/gauge_steps that kick with the
gauge force and drift the links.  The ratio of the fermion step to the gauge
step is then gauge_steps, and a trajectory makes n_md * gauge_steps gauge
steps.  This oracle applies every kick as written (no merging of adjacent
kicks).

Fermion action of npf pseudofermions, S_f = sum_k phi_k^dagger r(A) phi_k;
the heat bath sets phi_k = r_hb(A) R_k from complex Gaussian R_k.
"""

from __future__ import annotations

import numpy as np

from . import dirac, force, gauge, rational, solvers

# the minimum-norm value of the 2MN parameter (Omelyan, Mryglod and Folk)
LAMBDA_2MN = 0.1931833275037836


def integrate_2mn(tau, n_md, gauge_steps, lam, kick_f, kick_g, drift):
    """Multi-step 2MN scheme as described in the module docstring.  The three
    callables take the step coefficient c."""
    if n_md < 1 or gauge_steps < 2 or gauge_steps % 2:
        raise ValueError("n_md >= 1 and an even gauge_steps >= 2 are required")
    delta = tau / n_md
    h = delta / gauge_steps

    def inner():
        for _ in range(gauge_steps // 2):
            kick_g(lam * h)
            drift(0.5 * h)
            kick_g((1.0 - 2.0 * lam) * h)
            drift(0.5 * h)
            kick_g(lam * h)

    for _ in range(n_md):
        kick_f(lam * delta)
        inner()
        kick_f((1.0 - 2.0 * lam) * delta)
        inner()
        kick_f(lam * delta)


class LatticeMD:
    """Links, momenta and pseudofermions evolved by the kicks and drifts.

    U: links [Lt, Lz, Ly, Lx, 4, 3, 3]; omega: momenta [Lt, Lz, Ly, Lx, 4, 8];
    phi: pseudofermions [npf, 3, V/2]; r_md: the force's rational (alpha, beta
    used); solve: "dense" (exact, tiny lattices) or "cg" (multi-shift CG to
    cg_tol).
    """

    def __init__(self, U, omega, phi, beta, m, r_md, t_bc=-1, solve="dense", cg_tol=1e-13):
        self.U = np.array(U, dtype=np.complex128)
        self.omega = np.array(omega, dtype=np.float64)
        self.phi = np.asarray(phi, dtype=np.complex128)
        self.beta, self.m, self.t_bc = float(beta), float(m), t_bc
        self.alpha = np.asarray(r_md.alpha, dtype=np.float64)
        self.poles = np.asarray(r_md.beta, dtype=np.float64)
        self.solve, self.cg_tol = solve, cg_tol
        self.n_fermion = self.n_gauge = self.n_drift = 0

    def fermion_force(self):
        if self.solve == "dense":
            return force.force(self.U, self.m, self.alpha, self.poles, self.phi, self.t_bc)
        A = lambda v: dirac.mdagm(self.U, self.m, v, self.t_bc)  # noqa: E731
        F = np.zeros_like(self.U)
        for p in self.phi:
            x, info = solvers.multishift_cg(A, p, self.poles, tol=self.cg_tol)
            assert info.converged
            y = dirac.dslash(self.U, x, 1, self.t_bc)
            F += force.force_from_solutions(self.U, x, y, self.alpha, self.t_bc)
        return F

    def kick_f(self, c):
        self.omega -= c * gauge.algebra_coefficients(self.fermion_force())
        self.n_fermion += 1

    def kick_g(self, c):
        self.omega -= c * gauge.algebra_coefficients(gauge.gauge_force(self.U, self.beta))
        self.n_gauge += 1

    def drift(self, c):
        self.U = gauge.update_links(self.U, self.omega, c)
        self.n_drift += 1

    def integrate(self, tau, n_md, gauge_steps, lam=LAMBDA_2MN):
        integrate_2mn(tau, n_md, gauge_steps, lam, self.kick_f, self.kick_g, self.drift)


def fermion_action(U, m, phi, r, t_bc=-1, solve="dense", cg_tol=1e-13):
    """sum_k Re <phi_k, r(A) phi_k>."""
    if solve == "dense":
        return force.dense_rational_action(U, m, r.alpha0, r.alpha, r.beta, phi, t_bc)
    A = lambda v: dirac.mdagm(U, m, v, t_bc)  # noqa: E731
    S = 0.0
    for p in np.asarray(phi):
        y, _, info = rational.rational_apply(A, p, r.alpha0, r.alpha, r.beta, tol=cg_tol)
        assert info.converged
        S += float(np.real(np.vdot(p, y)))
    return S


def heatbath(U, m, R, r_hb, t_bc=-1, solve="dense", cg_tol=1e-13):
    """phi_k = r_hb(A) R_k."""
    A = lambda v: dirac.mdagm(U, m, v, t_bc)  # noqa: E731
    if solve == "dense":
        Ad = dirac.dense_A(U, m, t_bc)
        fn = lambda x: rational.scalar_rational(x, r_hb.alpha0, r_hb.alpha, r_hb.beta)  # noqa: E731
        return np.stack([rational.dense_function_apply(Ad, Rk, fn) for Rk in R])
    out = []
    for Rk in R:
        y, _, info = rational.rational_apply(A, Rk, r_hb.alpha0, r_hb.alpha, r_hb.beta, tol=cg_tol)
        assert info.converged
        out.append(y)
    return np.stack(out)


def hamiltonian(U, omega, phi, beta, m, r_act, t_bc=-1, solve="dense", cg_tol=1e-13):
    """(kinetic, gauge action, fermion action)."""
    return (gauge.kinetic(omega), gauge.gauge_action(U, beta),
            fermion_action(U, m, phi, r_act, t_bc, solve, cg_tol))


def trajectory(U, omega, R, u, beta, m, r_hb, r_act, r_md, tau, n_md, gauge_steps,
               lam=LAMBDA_2MN, t_bc=-1, solve="dense", cg_tol=1e-13):
    """One trajectory of the Phi algorithm (Sec. 2.1): heat bath of the
    pseudofermions, molecular dynamics, Metropolis test accept if
    u < exp(-dH).  Returns a dict with the parts of H before and after, dH,
    the decision, the final links (the initial ones if rejected) and the final
    momenta."""
    phi = heatbath(U, m, R, r_hb, t_bc, solve, cg_tol)
    h0 = hamiltonian(U, omega, phi, beta, m, r_act, t_bc, solve, cg_tol)
    md = LatticeMD(U, omega, phi, beta, m, r_md, t_bc, solve, cg_tol)
    md.integrate(tau, n_md, gauge_steps, lam)
    h1 = hamiltonian(md.U, md.omega, phi, beta, m, r_act, t_bc, solve, cg_tol)
    dH = sum(b - a for a, b in zip(h0, h1))
    accept = bool(u < np.exp(-dH))
    return dict(phi=phi, h0=h0, h1=h1, dH=dH, accepted=accept,
                U=md.U if accept else np.array(U), omega=md.omega)


def reversibility(U0, U2, omega0, omega2):
    """Delta C and Delta M of the reversibility test (Sec. 4.4): root mean square
    over the degrees of freedom (4 * 8 per site) of U(0) - U(2 tau) and
    H(0) + H(2 tau), with the Frobenius norm of each link matrix."""
    dof = 4 * 8 * U0[..., 0, 0, 0].size
    dC = np.sqrt(np.sum(np.abs(U0 - U2) ** 2) / dof)
    dM = np.sqrt(np.sum(np.abs(gauge.mom_matrix(omega0) + gauge.mom_matrix(omega2)) ** 2) / dof)
    return float(dC), float(dM)
