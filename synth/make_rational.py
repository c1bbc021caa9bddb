"""Write the cached rational coefficients for the five named workloads.

Run as ``python -m synth.make_rational``; each file in ``synth/data`` holds
alpha0, alpha_i, beta_i and the levelled relative error delta for x^p with
``npole`` poles on the interval [m^2, 16 + m^2].
"""

from .fields import CONFIGS
from .remez import rational_coefficients


def workload_rationals():
    seen = []
    for cfg, c in CONFIGS.items():
        lo = c["m"] ** 2
        for p in tuple(c["powers"]) + (c["hb_power"],):
            key = (p, c["npole"], lo, 16.0 + lo)
            if key not in seen:
                seen.append(key)
    return seen


def rational_for(cfg: int, p: float = -0.25):
    c = CONFIGS[cfg]
    lo = c["m"] ** 2
    return rational_coefficients(p, c["npole"], lo, 16.0 + lo)


if __name__ == "__main__":
    for p, n, lo, hi in workload_rationals():
        r = rational_coefficients(p, n, lo, hi)
        print(f"p={p:+.2f} n={n} [{lo:.3e}, {hi:.6f}] delta={r.delta:.3e} iters={r.iterations}",
              flush=True)
