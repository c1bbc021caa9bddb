"""Write the cached rational coefficients for the five named workloads and
the molecular-dynamics workload.

Run as ``python -m synth.make_rational``; each file in ``synth/data`` holds
alpha0, alpha_i, beta_i and the levelled relative error delta for x^p with
``npole`` poles on the interval [m^2, 16 + m^2].
"""

from .fields import CONFIGS, MD_WORKLOAD
from .remez import rational_coefficients


def workload_rationals():
    seen = []
    for cfg, c in CONFIGS.items():
        lo = c["m"] ** 2
        for p in tuple(c["powers"]) + (c["hb_power"],):
            key = (p, c["npole"], lo, 16.0 + lo)
            if key not in seen:
                seen.append(key)
    lo = MD_WORKLOAD["m"] ** 2
    for p, n in ((0.125, MD_WORKLOAD["metro_npole"]), (-0.25, MD_WORKLOAD["metro_npole"]),
                 (-0.25, MD_WORKLOAD["md_npole"])):
        key = (p, n, lo, 16.0 + lo)
        if key not in seen:
            seen.append(key)
    return seen


def rational_for(cfg: int, p: float = -0.25):
    c = CONFIGS[cfg]
    lo = c["m"] ** 2
    return rational_coefficients(p, c["npole"], lo, 16.0 + lo)


def md_rationals():
    """(heat bath x^{1/8}, Metropolis action x^{-1/4}, molecular-dynamics force
    x^{-1/4}) of the molecular-dynamics workload."""
    w = MD_WORKLOAD
    lo = w["m"] ** 2
    return (rational_coefficients(0.125, w["metro_npole"], lo, 16.0 + lo),
            rational_coefficients(-0.25, w["metro_npole"], lo, 16.0 + lo),
            rational_coefficients(-0.25, w["md_npole"], lo, 16.0 + lo))


if __name__ == "__main__":
    for p, n, lo, hi in workload_rationals():
        r = rational_coefficients(p, n, lo, hi)
        print(f"p={p:+.2f} n={n} [{lo:.3e}, {hi:.6f}] delta={r.delta:.3e} iters={r.iterations}",
              flush=True)
