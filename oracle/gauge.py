"""Gauge sector of the molecular dynamics (oracle; test infrastructure only).

Sec. 2 and 2.1 of the paper:

* Gauge action: the plaquette (Wilson) action,
      S_g = beta * sum_n sum_{mu<nu} (1 - Re Tr P_{mu nu}(n) / 3),
      P_{mu nu}(n) = U_mu(n) U_nu(n+mu) U_mu(n+nu)^dagger U_nu(n)^dagger,
  with periodic links in every direction.
* Momenta: one traceless Hermitian H_mu(n) = sum_a omega^a T^a per link,
  T^a = lambda^a / 2 (Gell-Mann matrices), omega^a ~ N(0, 1); the kinetic
  term sum Tr(H^2) then equals (1/2) sum (omega^a)^2.
* Link update: U_mu(n) -> exp(i eps H_mu(n)) U_mu(n), followed by a
  reunitarisation in FP64 (Sec. 4.1): rows 1-2 Gram-Schmidt orthonormalised,
  row 3 the complex conjugate of their cross product.
* Forces: for U_mu(n) -> exp(i eps T) U_mu(n) an action S changes at rate
  dS/deps = i Tr(T F_mu(n)) with F traceless anti-Hermitian.  For S_g,
      F_g = -(beta/3) TA(U_mu(n) Sigma_mu(n)),
      Sigma_mu(n) = sum_{nu != mu} U_nu(n+mu) U_mu(n+nu)^dagger U_nu(n)^dagger
                                 + U_nu(n+mu-nu)^dagger U_mu(n-nu)^dagger U_nu(n-nu).
  Conservation of sum Tr(H^2) + S along dU/dtau = i H U gives the momentum
  equation d omega^a / dtau = -c^a with c^a = i Tr(T^a F) (real).

Field layouts: links U [Lt, Lz, Ly, Lx, 4, 3, 3] (as everywhere in the
oracle); momenta on the full lattice [Lt, Lz, Ly, Lx, 4, 8]; the C ABI's
momentum layout [8][4][2][V/2] (component, direction, parity, eo) is
converted by ``mom_from_abi`` / ``mom_to_abi``.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from . import lattice


def generators():
    """T^a = lambda^a / 2, a = 1..8, complex128 [8, 3, 3]."""
    T = np.zeros((8, 3, 3), dtype=np.complex128)
    T[0][0, 1] = T[0][1, 0] = 0.5
    T[1][0, 1], T[1][1, 0] = -0.5j, 0.5j
    T[2][0, 0], T[2][1, 1] = 0.5, -0.5
    T[3][0, 2] = T[3][2, 0] = 0.5
    T[4][0, 2], T[4][2, 0] = -0.5j, 0.5j
    T[5][1, 2] = T[5][2, 1] = 0.5
    T[6][1, 2], T[6][2, 1] = -0.5j, 0.5j
    s = 0.5 / np.sqrt(3.0)
    T[7][0, 0], T[7][1, 1], T[7][2, 2] = s, s, -2 * s
    return T


def dagger(X):
    return np.swapaxes(X.conj(), -1, -2)


def traceless_antihermitian(X):
    Y = 0.5 * (X - dagger(X))
    return Y - (np.trace(Y, axis1=-2, axis2=-1) / 3.0)[..., None, None] * np.eye(3)


def mom_matrix(omega):
    """H = sum_a omega^a T^a for omega [..., 8]."""
    return np.einsum("...a,aij->...ij", omega, generators())


def algebra_coefficients(F):
    """c^a = i Tr(T^a F) (real part; F anti-Hermitian makes it real)."""
    return np.real(1j * np.einsum("aij,...ji->...a", generators(), F))


def kinetic(omega):
    """sum Tr(H^2) = (1/2) sum omega^2."""
    return 0.5 * float(np.sum(np.asarray(omega, dtype=np.float64) ** 2))


def mom_from_abi(w, L):
    """[8][4][2][V/2] (component, mu, parity, eo) -> [Lt, Lz, Ly, Lx, 4, 8]."""
    Lx, Ly, Lz, Lt = lattice.check_dims(L)
    Vh = Lx * Ly * Lz * Lt // 2
    w = np.asarray(w, dtype=np.float64).reshape(8, 4, 2, Vh)
    out = np.zeros((Lt, Lz, Ly, Lx, 4, 8))
    for par in range(2):
        x, y, z, t = lattice.eo_coordinates(L, par)
        out[t, z, y, x] = np.transpose(w[:, :, par, :], (2, 1, 0))
    return out


def mom_to_abi(omega):
    """[Lt, Lz, Ly, Lx, 4, 8] -> [8][4][2][V/2]."""
    Lt, Lz, Ly, Lx = omega.shape[:4]
    L = (Lx, Ly, Lz, Lt)
    out = np.zeros((8, 4, 2, Lx * Ly * Lz * Lt // 2))
    for par in range(2):
        x, y, z, t = lattice.eo_coordinates(L, par)
        out[:, :, par, :] = np.transpose(omega[t, z, y, x], (2, 1, 0))
    return out


def shift(X, mu, k):
    """Matrix field X [Lt, Lz, Ly, Lx, 3, 3] taken at n + k*mu (periodic)."""
    return np.roll(X, -k, axis=lattice.AXIS[mu] - 1)


def plaquettes(U):
    """Re Tr P_{mu nu}(n) for mu < nu, [6, Lt, Lz, Ly, Lx] in the order
    (0,1), (0,2), (0,3), (1,2), (1,3), (2,3)."""
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu, Unu = U[..., mu, :, :], U[..., nu, :, :]
            P = Umu @ shift(Unu, mu, 1) @ dagger(shift(Umu, nu, 1)) @ dagger(Unu)
            out.append(np.real(np.trace(P, axis1=-2, axis2=-1)))
    return np.stack(out)


def gauge_action(U, beta):
    """S_g = beta * sum (1 - Re Tr P / 3)."""
    return float(beta * np.sum(1.0 - plaquettes(U) / 3.0))


def staples(U):
    """Sigma_mu(n) as defined in the module docstring, [..., 4, 3, 3]."""
    S = np.zeros_like(U)
    for mu in range(4):
        Umu = U[..., mu, :, :]
        for nu in range(4):
            if nu == mu:
                continue
            Unu = U[..., nu, :, :]
            up = shift(Unu, mu, 1) @ dagger(shift(Umu, nu, 1)) @ dagger(Unu)
            # the lower staple is the upper one's pattern taken at n - nu
            lo_at = dagger(shift(Unu, mu, 1)) @ dagger(Umu) @ Unu     # at site n' = n - nu
            S[..., mu, :, :] += up + shift(lo_at, nu, -1)
    return S


def gauge_force(U, beta):
    """F_g = -(beta/3) TA(U Sigma)."""
    return -(beta / 3.0) * traceless_antihermitian(U @ staples(U))


def reunitarize(U):
    """Rows 1-2 Gram-Schmidt orthonormalised, row 3 = conj(row1 x row2)."""
    r0 = U[..., 0, :]
    r0 = r0 / np.sqrt(np.sum(np.abs(r0) ** 2, axis=-1, keepdims=True))
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.sqrt(np.sum(np.abs(r1) ** 2, axis=-1, keepdims=True))
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def exp_i(eps, H):
    """exp(i eps H) of each 3x3 matrix (scipy's matrix exponential)."""
    return scipy.linalg.expm(1j * eps * np.asarray(H, dtype=np.complex128))


def update_links(U, omega, eps):
    """U -> reunitarize(exp(i eps H) U)."""
    return reunitarize(exp_i(eps, mom_matrix(omega)) @ U)


def gauge_force_links(U, beta, t, z, y, x, mu):
    """F_g of the links (t[k], z[k], y[k], x[k], mu[k]) only, from the same
    definition with the neighbours indexed explicitly (periodic): for large
    lattices, where only a sample of links is checked."""
    Lt, Lz, Ly, Lx = U.shape[:4]
    ext = (Lx, Ly, Lz, Lt)
    t, z, y, x, mu = (np.asarray(a, dtype=np.int64) for a in (t, z, y, x, mu))

    def link(c, d):   # U_d at coordinates c = [x, y, z, t] (arrays)
        return U[c[3] % Lt, c[2] % Lz, c[1] % Ly, c[0] % Lx, d]

    def step(c, d, s):
        c = [a.copy() for a in c]
        c[d] = c[d] + s
        return c

    n = [x, y, z, t]
    S = np.zeros((x.size, 3, 3), dtype=np.complex128)
    for k in range(x.size):
        m = int(mu[k])
        nk = [a[k:k + 1] for a in n]
        for nu in range(4):
            if nu == m:
                continue
            up = link(step(nk, m, 1), nu) @ dagger(link(step(nk, nu, 1), m)) @ dagger(link(nk, nu))
            lo_site = step(nk, nu, -1)
            lo = dagger(link(step(lo_site, m, 1), nu)) @ dagger(link(lo_site, m)) @ link(lo_site, nu)
            S[k] += (up + lo)[0]
    Ul = U[t, z, y, x, mu]
    return -(beta / 3.0) * traceless_antihermitian(Ul @ S)
