"""Seeded gauge fields of the named workloads, generated once per machine.

The large fields take tens of seconds to generate; the generation runs in a
child process (which has no GPU context, so it may use worker processes) and
the result is kept as a .npy file in the temporary directory, loaded with
memory mapping afterwards.
"""

import os
import subprocess
import sys
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def workload_gauge(cfg: int) -> np.ndarray:
    import synth

    c = synth.CONFIGS[cfg]
    tag = "x".join(str(v) for v in c["L"])
    path = os.path.join(tempfile.gettempdir(), f"rhmc_gauge_cfg{cfg}_{tag}_eps{c['eps']}.npy")
    if not os.path.exists(path):
        tmp = path + f".{os.getpid()}.tmp.npy"
        code = (
            "import sys; sys.path.insert(0, %r)\n"
            "import numpy as np, synth\n"
            "c = synth.CONFIGS[%d]\n"
            "np.save(%r, synth.gauge_field(c['L'], c['eps'], synth.fields.seed_gauge(%d)))\n"
        ) % (ROOT, cfg, tmp, cfg)
        subprocess.run([sys.executable, "-c", code], check=True)
        os.replace(tmp, path)
    return np.load(path, mmap_mode="r")
