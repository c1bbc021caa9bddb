"""Plain FP64 CPU oracle for the even-odd staggered operator and its solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
load this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library; the two
meet only through the seeded inputs of ``synth``.

The oracle follows the paper's statement of the problem:

* ``lattice`` -- site indexing, even/odd ordering, neighbours, the staggered
  phases eta and the time-boundary sign (Sec. 2, below Eq. stag).
* ``dirac``   -- the hopping term D of Eq. stag, its even/odd blocks D_eo and
  D_oe, and A = M^dagger M restricted to even sites, A = m^2 - D_eo D_oe
  (even/odd preconditioning, Sec. 2.1).
* ``solvers`` -- CG and the shifted (multi-shift) CG for (A + sigma_i) x = b
  from one Krylov space with a zero start (Sec. 4.3, Eq. shifted), plus
  dense solves and true residuals used to certify results.
* ``rational`` -- r(A) b = alpha0 b + sum_i alpha_i (A + beta_i)^-1 b, the
  rational approximation of the rooted system (Sec. 2.1, Eq. system_r).
* ``pseudofermion``, ``force`` -- the pseudofermion field, action and heat
  bath of the Phi algorithm, and the derivative of the action with respect
  to the links (Sec. 2.1).
* ``gauge`` -- plaquette action and its force, momenta, the exponential link
  update and reunitarisation (Sec. 2, 2.1, 4.1).
* ``md`` -- the multi-step second-order minimum-norm integrator, the
  Hamiltonian, one trajectory with its Metropolis test, and the
  reversibility estimators (Sec. 2.1, 4.4).
"""

from . import dirac, force, gauge, lattice, md, pseudofermion, rational, solvers  # noqa: F401
