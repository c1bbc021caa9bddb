"""Seeded gauge fields and pseudofermion sources.

Conventions (shared by every consumer, so they are fixed here once):

* A lattice is ``L = (Lx, Ly, Lz, Lt)``; every extent is even.  Time is the
  fourth direction.
* Host gauge layout (canonical): ``complex128[Lt][Lz][Ly][Lx][mu][row][col]``
  with ``mu = 0..3`` for x, y, z, t, i.e. the site index is lexicographic with
  x running fastest.
* Even-site colour vectors are ``complex128[nrhs][3][V/2]``: colour-major,
  and within a colour the even sites in "eo" order, where
  ``eo = lex >> 1`` and ``lex = x + Lx*(y + Ly*(z + Lz*t))``.

Link generator (the paper's momentum distribution, Sec. 2.1): each link is
``U = exp(i*eps*H)`` with ``H = sum_a omega^a T^a``, ``T^a = lambda^a/2`` the
Gell-Mann generators and ``omega^a ~ N(0, 1)``; the exponential is taken by an
eigen-decomposition of ``H`` and the result is reunitarised in FP64 (first two
rows Gram-Schmidt orthonormalised, third row the complex conjugate of their
cross product), which makes ``det U = 1`` to rounding.  Random numbers are
drawn from ``numpy.random.Generator(PCG64(seed))`` in the order
site (lexicographic, x fastest) -> mu -> a = 1..8.

Source generator (the heat-bath distribution ``exp(-R^dagger R)`` of the Phi
algorithm, Sec. 2.1): real and imaginary parts ``N(0, 1/2)``, drawn per even
site (eo order) -> colour -> (re, im); right-hand side ``k`` uses seed
``seed + k``.
"""

from __future__ import annotations

import numpy as np

# The five workloads: lattice, link roughness eps, quark mass m, number of
# right-hand sides, number of poles, exponents p of x^p, solver tolerance and
# arithmetic mode.  hb_power is the exponent of the pseudofermion heat bath
# phi = A^{1/8} R that goes with the action phi^dagger A^{-1/4} phi.  The rational interval is [m^2, 16 + m^2] for all of them
# (the spectrum of M^dagger M on even sites lies there because ||D|| <= 4).
CONFIGS = {
    1: dict(L=(4, 4, 4, 4), eps=0.5, m=0.1, nrhs=1, npole=8, powers=(-0.25,),
            tol=1e-12, mode="fp64", hb_power=0.125),
    2: dict(L=(16, 16, 16, 4), eps=0.5, m=0.02, nrhs=1, npole=15,
            powers=(-0.25, 0.25), tol=1e-10, mode="fp64", hb_power=0.125),
    3: dict(L=(32, 32, 32, 8), eps=0.7, m=0.01, nrhs=1, npole=15,
            powers=(-0.25,), tol=1e-10, mode="mixed", hb_power=0.125),
    4: dict(L=(32, 32, 32, 8), eps=0.7, m=0.01, nrhs=8, npole=15,
            powers=(-0.25,), tol=1e-10, mode="mixed", hb_power=0.125),
    5: dict(L=(48, 48, 48, 12), eps=0.8, m=0.005, nrhs=4, npole=20,
            powers=(-0.25,), tol=1e-10, mode="mixed", hb_power=0.125),
}


# The molecular-dynamics workload of the algorithm tests of Sec. 4.4: a 4 x 16^3
# lattice at beta 5.264 and am 0.01335, two pseudofermions, rational
# approximations with 8 poles in the molecular dynamics and 15 in the
# Metropolis step (x^{-1/4}) and the heat bath (x^{+1/8}), n_md = 12 fermion
# steps with dtau_f / dtau_g = 10, trajectory length 1.  The gauge field is
# synthetic (link roughness 0.5 gives a plaquette near 0.5), not thermalised.
MD_WORKLOAD = dict(L=(16, 16, 16, 4), eps=0.5, beta=5.264, m=0.01335, npf=2, md_npole=8,
                   metro_npole=15, n_md=12, gauge_steps=10, tau=1.0, seed=1100)


def seed_gauge(cfg: int) -> int:
    return 1000 + cfg


def seed_source(cfg: int) -> int:
    return 2000 + 100 * cfg


def volume(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def even_volume(L) -> int:
    return volume(L) // 2


def _check_dims(L):
    if len(L) != 4 or any(int(l) < 2 or int(l) % 2 for l in L):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {L}")


def _gell_mann_generators() -> np.ndarray:
    """T^a = lambda^a / 2, a = 1..8, as complex128[8][3][3]."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam / 2


def _reunitarize(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _exp_i_eps_h(omega: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) for H = sum_a omega^a T^a, batched over leading axes."""
    T = _gell_mann_generators()
    lead = omega.shape[:-1]
    H = (omega.reshape(-1, 8) @ T.reshape(8, 9)).reshape(lead + (3, 3))
    w, V = np.linalg.eigh(H)
    U = (V * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(V, -1, -2))
    return _reunitarize(U)


def _exp_chunk(args):
    omega, eps = args
    return _exp_i_eps_h(omega, eps)


def _gpu_initialised() -> bool:
    import sys

    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:
        return True


def random_su3(shape, rng: np.random.Generator, eps: float) -> np.ndarray:
    """SU(3) matrices exp(i*eps*H) with Gaussian algebra components."""
    omega = rng.standard_normal(tuple(shape) + (8,))
    return _exp_i_eps_h(omega, eps)


def gauge_field(L, eps: float, seed: int, chunk: int = 1 << 16, workers=None) -> np.ndarray:
    """Seeded gauge field, complex128[Lt][Lz][Ly][Lx][4][3][3].

    All random numbers are drawn first, in the documented order; the
    exponentials are then evaluated chunk by chunk, in worker processes when
    the lattice is large (the result does not depend on the number of
    workers).  Worker processes are forked only while no GPU context exists.
    """
    _check_dims(L)
    Lx, Ly, Lz, Lt = (int(l) for l in L)
    V = Lx * Ly * Lz * Lt
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = rng.standard_normal((V, 4, 8))
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    starts = list(range(0, V, chunk))
    if workers is None:
        import os

        workers = 1 if (V < 4 * chunk or _gpu_initialised()) else min(16, os.cpu_count() or 1)
    if workers > 1:
        import concurrent.futures as cf
        import multiprocessing as mp

        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            parts = ex.map(_exp_chunk, ((omega[s0:s0 + chunk], eps) for s0 in starts))
            for s0, part in zip(starts, parts):
                out[s0:s0 + part.shape[0]] = part
    else:
        for s0 in starts:
            out[s0:s0 + chunk] = _exp_i_eps_h(omega[s0:s0 + chunk], eps)
    return out.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)


def unit_gauge(L) -> np.ndarray:
    _check_dims(L)
    Lx, Ly, Lz, Lt = (int(l) for l in L)
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def source(L, seed: int, nrhs: int = 1) -> np.ndarray:
    """Gaussian even-site sources, complex128[nrhs][3][V/2]."""
    _check_dims(L)
    Vh = even_volume(L)
    out = np.empty((nrhs, 3, Vh), dtype=np.complex128)
    for k in range(nrhs):
        rng = np.random.Generator(np.random.PCG64(seed + k))
        g = rng.standard_normal((Vh, 3, 2)) * np.sqrt(0.5)
        out[k] = (g[..., 0] + 1j * g[..., 1]).T
    return out


def momenta(L, seed: int) -> np.ndarray:
    """Gaussian momenta omega^a ~ N(0, 1) (the heat bath of Sec. 2.1), float64
    [8][4][2][V/2]: algebra component a, direction mu, parity, eo; drawn in
    that order."""
    _check_dims(L)
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((8, 4, 2, even_volume(L)))


def config_inputs(cfg: int):
    """(U, b, params) for one of the five named workloads."""
    c = CONFIGS[cfg]
    U = gauge_field(c["L"], c["eps"], seed_gauge(cfg))
    b = source(c["L"], seed_source(cfg), c["nrhs"])
    return U, b, c
