#!/usr/bin/env python
"""Benchmark of the staggered RHMC hot path on one MI355X.

Headline workload: 48^3 x 12 lattice, links exp(i*0.8*H), m = 0.005, four
Gaussian pseudofermion sources, the 20-pole rational approximation of x^-1/4
on [m^2, 16 + m^2], tolerance 1e-10 per shift.  One step is one call of
rhmc_rational_apply in MIXED precision with all four right-hand sides batched:
multi-shift CG (FP64 phase, then the FP32 12-real hopping term with FP64
reliable updates every 50 iterations, FP64 reductions and recurrences), FP64
true-residual check and refinement, FP64 combine.

Printed JSON line (one):
  value          effective GB/s of the FP32 12-real four-rhs hopping kernel,
                 algorithmic bytes per launch / launch time (HIP events on the
                 launching stream), the kernel the solve spends its time in
  roofline       that kernel against the 8 TB/s HBM peak
  dslash         the other hopping shapes (FP64-12 4 rhs, FP32-12 8 rhs, 1 rhs,
                 other link storages, the cache-resident 16^3 x 4 lattice)
  time_to_solution_s   the headline solve in MIXED + batched and in plain
                 FP64 on the same GPU, each phase of the MIXED solve with its
                 algorithmic bytes, and the per-shift error of the MIXED
                 solutions against the GPU's FP64 solutions
  workloads      the other configurations: 4^4 and 16^3 x 4 (FP64, errors
                 against full oracle solves), 32^3 x 8 with 1 rhs (MIXED, error
                 against the FP64 solve and oracle true residuals per shift)
                 and 32^3 x 8 with 8 rhs (MIXED batched)
  cpu_baseline   the FP64 numpy oracle on one host core (child process with
                 one thread): full solves of the 4^4 and 16^3 x 4 workloads and a
                 bounded sample of the headline one (extrapolated, labelled)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("Dslash GB/s (% HBM peak); multi-shift CG time to r≤10^-10, FP64 vs mixed+batched")
HBM_PEAK_GBPS = 8000.0
FLOPS_PER_SITE = 570   # 8 SU(3) x vector products (66) + 7 vector additions (6)
HEADLINE_CFG = 5


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def dslash_bytes_per_site(prec: str, nrhs: int) -> int:
    """Algorithmic bytes per output site of one hopping application: 8 links
    read once, the input vector read once and the output written once."""
    if prec == "fp32":
        return 8 * 48 + nrhs * (24 + 24)
    if prec == "fp32f":   # FP32-18 links: 72 B per link
        return 8 * 72 + nrhs * (24 + 24)
    if prec in ("fp64hl", "fp64c"):   # hi/lo FP32-12 planes or FP64-12 links: 96 B per link
        return 8 * 96 + nrhs * (48 + 48)
    return 8 * 144 + nrhs * (48 + 48)


def kernel_source_hash():
    """Hash of the hopping kernel's sources (kernel file and its headers)."""
    h = hashlib.sha256()
    for name in ("dslash_kernel.h", "dslash.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_1106_5673_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_tag: str, variant: int):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current hopping-kernel source in the same launch variant (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash() or rec.get("launch_variant") != variant:
        return None
    return rec.get("bytes_per_launch")


def host_description():
    """CPU model, logical CPUs and the thread settings numpy's kernels see."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
               if os.environ.get(k) is not None}
    return {"cpu_model": model, "nproc": os.cpu_count(), "threads_env": threads}


# ------------------------------------------------------------------ CPU baseline
ONE_THREAD = {"OMP_NUM_THREADS": "1", "OPENBLAS_NUM_THREADS": "1", "MKL_NUM_THREADS": "1",
              "NUMEXPR_NUM_THREADS": "1"}


def cpu_baseline_child(workdir: str):
    """The oracle, timed on one host core (run in a child process started with
    one BLAS/OpenMP thread).  Reads the GPU solutions the parent left in
    workdir, writes cpu.json there.

    * full oracle multi-shift solves of the 4^4 (8 poles, tol 1e-12) and
      16^3 x 4 (15 poles of x^-1/4 and of x^+1/4, tol 1e-10) workloads, timed,
      and the per-shift error of the GPU's FP64 solutions against them;
    * the oracle's true residual of every shift of the GPU's MIXED 32^3 x 8
      solve;
    * on the headline lattice, one D_oe application and a few multi-shift
      iterations (all 20 shifts), extrapolated to the GPU's iteration count."""
    import numpy as np

    import synth
    from oracle import dirac, solvers
    from synth.make_rational import rational_for

    out = {"host": host_description()}
    t_all, c_all = time.perf_counter(), time.process_time()

    def err_per_shift(xg, xo):
        return [float(np.linalg.norm(xg[i] - xo[i]) / np.linalg.norm(xo[i])) for i in range(xo.shape[0])]

    solves = {}
    for cfg, powers in ((1, (-0.25,)), (2, (-0.25, 0.25))):
        c = synth.CONFIGS[cfg]
        U = synth.gauge_field(c["L"], c["eps"], synth.fields.seed_gauge(cfg))
        b = synth.source(c["L"], synth.fields.seed_source(cfg), 1)
        A = lambda v: dirac.mdagm(U, c["m"], v)  # noqa: E731
        for p in powers:
            r = rational_for(cfg, p)
            t0 = time.perf_counter()
            xo, info = solvers.multishift_cg(A, b[0], np.asarray(r.beta), tol=c["tol"])
            dt = time.perf_counter() - t0
            key = f"c{cfg}_p{p:+.2f}"
            xg = np.load(os.path.join(workdir, f"{key}.npy"))[0]
            e = err_per_shift(xg, xo)
            solves[key] = {"lattice": list(c["L"]), "poles": int(len(r.beta)), "tol": c["tol"],
                           "oracle_s": round(dt, 3), "oracle_iterations": info.iterations,
                           "gpu_fp64_rel_error_per_shift": e, "max_rel_error": max(e)}
    out["oracle_solves"] = solves

    # oracle true residuals of the GPU's MIXED 32^3 x 8 solutions
    c = synth.CONFIGS[3]
    U3 = np.load(os.path.join(workdir, "c3_links.npy"))
    b3 = synth.source(c["L"], synth.fields.seed_source(3), 1)
    r3 = rational_for(3, -0.25)
    x3 = np.load(os.path.join(workdir, "c3_mixed.npy"))[0]
    t0 = time.perf_counter()
    res = [float(solvers.true_residual(lambda v: dirac.mdagm(U3, c["m"], v), b3[0], x3[i], s))
           for i, s in enumerate(r3.beta)]
    out["c3_mixed_oracle_true_residual_per_shift"] = res
    out["c3_oracle_check_s"] = round(time.perf_counter() - t0, 2)

    # bounded sample of the headline workload
    c = synth.CONFIGS[HEADLINE_CFG]
    U = np.load(os.path.join(workdir, "c5_links.npy"), mmap_mode="r")
    U = np.asarray(U)
    b = synth.source(c["L"], synth.fields.seed_source(HEADLINE_CFG), 1)
    r = rational_for(HEADLINE_CFG, -0.25)
    Vh = b.shape[-1]
    t0 = time.perf_counter()
    dirac.dslash(U, b[:1], 1)
    t_d = time.perf_counter() - t0
    iters = 3
    t1 = time.perf_counter()
    solvers.multishift_cg(lambda v: dirac.mdagm(U, c["m"], v), b[0], np.asarray(r.beta), tol=1e-10,
                          maxiter=iters)
    t_it = (time.perf_counter() - t1) / iters
    out["headline_sample"] = {"dslash_s": t_d, "seconds_per_cg_iteration_per_rhs": t_it,
                              "dslash_GBps": dslash_bytes_per_site("fp64", 1) * Vh / t_d / 1e9}
    out["wall_s"] = time.perf_counter() - t_all
    out["cpu_s"] = time.process_time() - c_all
    with open(os.path.join(workdir, "cpu.json"), "w") as fh:
        json.dump(out, fh)


def run_cpu_baseline(workdir: str, gpu_iters_c5: int, nrhs_c5: int, gpu_times: dict):
    """Runs cpu_baseline_child in a fresh process with one thread and
    assembles the cpu_baseline object of the JSON line."""
    env = dict(os.environ)
    env.update(ONE_THREAD)
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", workdir]
    log("timing the CPU oracle (one thread, child process)")
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        log(f"cpu baseline child failed: {r.stderr[-2000:]}")
        return None
    with open(os.path.join(workdir, "cpu.json")) as fh:
        cpu = json.load(fh)
    s = cpu["headline_sample"]
    c2 = cpu["oracle_solves"]["c2_p-0.25"]
    extrap = s["seconds_per_cg_iteration_per_rhs"] * gpu_iters_c5 * nrhs_c5
    return {
        "value": round(s["dslash_GBps"], 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("FP64 numpy oracle on one host core (child process, OMP/OpenBLAS/MKL threads = 1): "
                   "one D_oe application on 1 rhs of the 48^3x12 field (GB/s at 1248 B/site), "
                   "3 multi-shift CG iterations with 20 shifts on it, full multi-shift solves of the "
                   "4^4 and 16^3x4 workloads, and oracle true residuals of the GPU's 32^3x8 MIXED solution"),
        "headline_dslash_s": round(s["dslash_s"], 3),
        "headline_seconds_per_cg_iteration_per_rhs": round(s["seconds_per_cg_iteration_per_rhs"], 3),
        "headline_time_to_solution_s_extrapolated": round(extrap, 1),
        "extrapolation": f"seconds per iteration x {gpu_iters_c5} GPU iterations x {nrhs_c5} rhs",
        "full_solves": cpu["oracle_solves"],
        "c2_oracle_time_to_solution_s": c2["oracle_s"],
        "c2_gpu_fp64_time_to_solution_s": gpu_times.get("c2"),
        "c3_mixed_oracle_true_residual_per_shift": cpu["c3_mixed_oracle_true_residual_per_shift"],
        "wall_seconds": round(cpu["wall_s"], 1),
        "cpu_seconds": round(cpu["cpu_s"], 1),
        "host": cpu["host"],
    }


# ------------------------------------------------------------------ molecular dynamics
# Per link (FP64-12 links, FP64 momenta of 8 reals): the gauge-force kick
# reads every link once and the momenta once and writes the momenta; the link
# update reads link and momenta and writes the FP64-12 and FP32-12 copies.
# Flops of the kick: 13 complex 3x3 products (198 each), 19 third-row
# rebuilds (42 each), the staple sums and the momentum update.
GF_BYTES_PER_LINK = 96 + 64 + 64
GF_FLOPS_PER_LINK = 13 * 198 + 19 * 42 + 6 * 18 + 40
UP_BYTES_PER_LINK = 96 + 64 + 96 + 48
FP64_VECTOR_PEAK_GFLOPS = 78600.0


def kernel_entry(t, t_min, nbytes, nflops):
    e = {"us_median": round(t * 1e6, 2), "us_min": round(t_min * 1e6, 2),
         "GBps": round(nbytes / t / 1e9, 1), "hbm_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBPS, 4)}
    if nflops is not None:
        e["gflops"] = round(nflops / t / 1e9, 1)
        e["fp64_frac"] = round(nflops / t / 1e9 / FP64_VECTOR_PEAK_GFLOPS, 4)
    return e


def time_call(torch, fn, reps, warm=3):
    """Median and minimum of reps launches of fn, each between its own pair of
    HIP events on the current stream."""
    for _ in range(warm):
        fn()
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(s)
        fn()
        e1.record(s)
    ev[-1][1].synchronize()
    ts = sorted(e0.elapsed_time(e1) / 1e3 for e0, e1 in ev)
    return ts[len(ts) // 2], ts[0]


def time_md_kernels(rhmc, torch, dev, g, lat, L):
    """Gauge-force kick and link update on the headline lattice (50 timed
    launches each after 3 untimed)."""
    import synth

    mom = torch.from_numpy(synth.momenta(L, 4000 + HEADLINE_CFG)).to(dev)
    beta_g, eps_g = synth.MD_WORKLOAD["beta"], 0.004
    t_gf, t_gf_min = time_call(torch, lambda: rhmc.rhmc_gauge_force_kick(g, beta_g, 1e-9, mom), 50)
    t_up, t_up_min = time_call(torch, lambda: rhmc.rhmc_update_links(g, eps_g, mom), 50)
    nl = 4 * lat.V
    del mom
    return {"gauge_force_kick": kernel_entry(t_gf, t_gf_min, GF_BYTES_PER_LINK * nl, GF_FLOPS_PER_LINK * nl),
            "link_update": kernel_entry(t_up, t_up_min, UP_BYTES_PER_LINK * nl, None),
            "note": "HIP events around each launch; GB/s counts each FP64-12 link, momentum and "
                    "written storage once"}


def run_md_trajectory(rhmc, torch, dev, ntraj):
    """Trajectories of the molecular-dynamics workload of the algorithm tests
    (4 x 16^3, beta 5.264, am 0.01335, 2 pseudofermions, n_md 12,
    dtau_f/dtau_g 10): MIXED MD solves at 1e-3, FP64 heat-bath and Metropolis
    solves at 1e-9.  One untimed trajectory, then ntraj timed ones."""
    import numpy as np

    import synth
    from synth.make_rational import md_rationals

    w = synth.MD_WORKLOAD
    L = w["L"]
    r_hb, r_act, r_md = md_rationals()
    U = synth.gauge_field(L, w["eps"], w["seed"])
    lat = rhmc.rhmc_lattice_create(L, -1)
    g = rhmc.rhmc_gauge_create(lat, U)
    mdp = rhmc.MDParams(r_md, beta=w["beta"], mass=w["m"], tau=w["tau"], n_md=w["n_md"],
                        gauge_steps=w["gauge_steps"],
                        solver=rhmc.solver_params(tol=1e-3, mode=rhmc.RHMC_MODE_MIXED))
    hp = rhmc.HMCParams(mdp, r_hb, r_act, rhmc.solver_params(tol=1e-9, mode=rhmc.RHMC_MODE_FP64))
    gen = torch.Generator(device=dev)
    gen.manual_seed(w["seed"] + 7)
    rng = np.random.default_rng(w["seed"] + 8)
    times, stats = [], []
    for k in range(ntraj + 1):
        R = torch.complex(torch.randn((w["npf"], 3, lat.Vh), dtype=torch.float64, device=dev, generator=gen),
                          torch.randn((w["npf"], 3, lat.Vh), dtype=torch.float64, device=dev, generator=gen))
        R *= 0.5 ** 0.5
        mom = torch.from_numpy(synth.momenta(L, w["seed"] + 100 + k)).to(dev)
        u = float(rng.uniform())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = rhmc.rhmc_trajectory(g, hp, R, mom, u, allow_not_converged=True)
        torch.cuda.synchronize()
        if k > 0:
            times.append(time.perf_counter() - t1)
            stats.append(st)
    g.close()
    return {"lattice": list(L), "beta": w["beta"], "mass": w["m"], "npf": w["npf"], "n_md": w["n_md"],
            "gauge_steps": w["gauge_steps"], "setting": "MIXED MD solves at 1e-3, FP64 Metropolis at 1e-9",
            "s_per_trajectory": round(float(np.mean(times)), 4), "runs_s": [round(t, 4) for t in times],
            "dH": [round(s["dH"], 5) for s in stats],
            "fermion_forces": stats[-1]["md"]["fermion_forces"],
            "gauge_forces": stats[-1]["md"]["gauge_forces"],
            "link_updates": stats[-1]["md"]["link_updates"],
            "gauge_field": "synthetic, not thermalised"}


# ------------------------------------------------------------------ solve accounting
def solve_phase_bytes(Vh, nrhs, nshift, K, st, prec_body="fp32"):
    """Algorithmic HBM bytes of the phases of one shared solve, from the
    iteration counts in its stats (every shift counted active in every
    block: an upper bound for the flushes).  Per iteration and rhs: the two
    hopping applications (links once per application for all rhs, input and
    output once; the A-mode also reads p), r' = r - alpha Ap (3 vectors),
    p = r' + beta p (3 vectors); per block of K iterations and rhs: X and P of
    every shift read and written once (FP64) and the K stored residuals read
    once."""
    def per_iter(prec):
        v = 24 if prec == "fp32" else 48
        links = 8 * (48 if prec == "fp32" else 96)
        hop = 2 * links + nrhs * (2 * v + 2 * v + v)
        return Vh * (hop + nrhs * 6 * v)

    def per_block(prec):
        v = 24 if prec == "fp32" else 48
        return Vh * nrhs * (nshift * 4 * 48 + K * v)

    head = st["fp64_head_iterations"]
    body = st["total_iterations"] - head
    # FP64 true residual of one system: D_oe (FP64-12 links + x) and the
    # residual mode (links + t + x + b, writes nothing)
    check_per_sys = Vh * (2 * 8 * 96 + 48 * 4)
    refine = int(st["refine_iterations"].sum())
    return {
        "fp64_head": per_iter("fp64") * head + per_block("fp64") * (head // K),
        "body": per_iter(prec_body) * body + per_block(prec_body) * (body // K),
        "true_residuals": check_per_sys * nrhs * nshift,
        # refinement: single-shift systems, counted without sharing the links
        # between the systems of a batch (an upper bound)
        "refinement": refine * Vh * (2 * 8 * 48 + 11 * 24),
    }


def phases_entry(Vh, nrhs, nshift, K, st):
    b = solve_phase_bytes(Vh, nrhs, nshift, K, st)
    ms = {"fp64_head": st["head_ms"], "body": st["krylov_ms"], "true_residuals": st["check_ms"],
          "refinement": st["refine_ms"]}
    out = {}
    for k in ("fp64_head", "body", "true_residuals", "refinement"):
        t = ms[k] / 1e3
        out[k] = {"s": round(t, 4), "algorithmic_GB": round(b[k] / 1e9, 2),
                  "GBps": round(b[k] / t / 1e9, 1) if t > 0 else None}
    out["iterations"] = {"fp64_head": st["fp64_head_iterations"],
                         "body": st["total_iterations"] - st["fp64_head_iterations"],
                         "refinement_system_iterations": int(st["refine_iterations"].sum())}
    out["note"] = ("host clock per phase (phases end at host synchronisations); algorithmic bytes "
                   "from the iteration counts: 2 hopping applications + 2 vector updates per "
                   "iteration, X and P of every shift once per block (all shifts counted active), "
                   "2 FP64 hopping passes per true residual")
    return out


def per_shift_errors(torch, xm, x64):
    """max over rhs of ||x_mixed - x_fp64|| / ||x_fp64|| for every shift."""
    d = torch.linalg.vector_norm(xm - x64, dim=(2, 3)) / torch.linalg.vector_norm(x64, dim=(2, 3))
    return [float(v) for v in d.max(dim=0).values.cpu()]


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dslash-reps", type=int, default=200)
    ap.add_argument("--fp64-runs", type=int, default=5, help="timed plain FP64 solves (median reported)")
    ap.add_argument("--block", type=int, default=50,
                    help="block length of the headline MIXED solve (replacements every 50 iterations "
                         "need a divisor of 50; the default 32 gives 25, also timed)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline hopping kernel and solves (profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-dslash", action="store_true",
                    help="only the hopping-kernel timing and a copy of known size (counter runs)")
    ap.add_argument("--only-md", action="store_true",
                    help="only the molecular-dynamics kernels on the headline lattice and "
                         "trajectories of the 4x16^3 workload (profiler runs)")
    ap.add_argument("--md-trajectories", type=int, default=2,
                    help="timed 4x16^3 trajectories (after one untimed)")
    ap.add_argument("--cpu-baseline-child", metavar="DIR", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_baseline_child)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding is a design only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth
    from synth.make_rational import rational_for

    # every input is generated before the GPU is touched (the field generator
    # forks worker processes for large lattices)
    t0 = time.perf_counter()
    c = synth.CONFIGS[HEADLINE_CFG]
    L, m, nrhs = c["L"], c["m"], c["nrhs"]
    U = synth.gauge_field(L, c["eps"], synth.fields.seed_gauge(HEADLINE_CFG))
    b = synth.source(L, synth.fields.seed_source(HEADLINE_CFG), nrhs)
    rat = rational_for(HEADLINE_CFG, -0.25)
    extra_inputs = {}
    if not args.only_dslash and not args.no_extras and not args.only_md:
        for cfg in (1, 2, 3, 4):
            cc = synth.CONFIGS[cfg]
            extra_inputs[cfg] = (synth.gauge_field(cc["L"], cc["eps"], synth.fields.seed_gauge(cfg)),
                                 synth.source(cc["L"], synth.fields.seed_source(cfg), cc["nrhs"]))
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")
    workdir = tempfile.mkdtemp(prefix="rhmc_bench_")

    import torch

    from paper_1106_5673_amd import rhmc

    dev = torch.device("cuda:0")
    lat = rhmc.rhmc_lattice_create(L, -1)
    g = rhmc.rhmc_gauge_create(lat, U)
    Vh = lat.Vh
    bd = torch.from_numpy(b).to(dev)
    y = torch.empty_like(bd)
    torch.cuda.synchronize()
    log("gauge packed on the device")
    # average plaquette Re Tr P / 3 of the field: S_g at beta = 1 is sum (1 - Re Tr P / 3)
    plaquette = 1.0 - rhmc.rhmc_gauge_action(g, 1.0) / (6.0 * lat.V)
    if args.only_md:
        md = {"md_kernels": time_md_kernels(rhmc, torch, dev, g, lat, L),
              "md_trajectory_16x16x16x4": run_md_trajectory(rhmc, torch, dev, args.md_trajectories)}
        log("molecular-dynamics kernels and trajectories done")
        print(json.dumps({"lattice": list(L), "plaquette": round(plaquette, 6), **md}))
        return

    def time_dslash(prec, k, reps, gauge=None, vh=None, warm=20, flush=None):
        """Launch time of D_oe: the average over `reps` back-to-back launches
        between one pair of HIP events on the launching stream (the timed
        region), then the median and min of `reps` launches each bracketed by
        its own pair of events (which adds the events' own few microseconds
        to every sample).  With `flush` (a device buffer) the buffer is
        streamed through a reduction between launches, outside the events, so
        no cache holds the operands; there is no region average then."""
        gg = gauge if gauge is not None else g
        n = vh if vh is not None else Vh
        dt = torch.complex64 if prec == "fp32" else torch.complex128
        pr = rhmc.RHMC_PREC_FP32 if prec == "fp32" else rhmc.RHMC_PREC_FP64
        if vh is None and k <= nrhs:
            src = bd[:k]
        else:
            src = torch.randn((k, 3, n), dtype=torch.complex128, device=dev)
        # the ABI's storage of the set (FP32, k >= 2: pairs of vectors; k is 1
        # or even here, so the entries are the sources in that storage)
        assert k == 1 or k % 2 == 0
        vin = src.to(dt).contiguous().reshape(rhmc.vec_shape(pr, k, n))
        vout = torch.empty_like(vin)
        for _ in range(warm):
            rhmc.rhmc_dslash_eo(gg, 1, pr, k, vin, vout)
        s = torch.cuda.current_stream()
        region = None
        if flush is None:
            r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            r0.record(s)
            for _ in range(reps):
                rhmc.rhmc_dslash_eo(gg, 1, pr, k, vin, vout)
            r1.record(s)
            r1.synchronize()
            region = r0.elapsed_time(r1) / 1e3 / reps
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            if flush is not None:
                flush.max()
            e0.record(s)
            rhmc.rhmc_dslash_eo(gg, 1, pr, k, vin, vout)
            e1.record(s)
        ev[-1][1].synchronize()
        ts = sorted(e0.elapsed_time(e1) / 1e3 for e0, e1 in ev)
        return region, ts[len(ts) // 2], ts[0]

    def dentry(tm, nbytes, nsite, k):
        # tm = (region average, per-launch median, per-launch min); rates from the average
        t, tmed, tmin = tm
        return {"us_avg": round(t * 1e6, 2), "us_median": round(tmed * 1e6, 2), "us_min": round(tmin * 1e6, 2),
                "GBps": round(nbytes / t / 1e9, 1), "hbm_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBPS, 4),
                "gflops": round(FLOPS_PER_SITE * nsite * k / t / 1e9, 1)}

    # ---------------------------------------------------------------- hopping kernel
    # library default launch variants (the solver tunes its own), so that
    # counter runs of --only-dslash see the same kernels
    var32 = rhmc.rhmc_dslash_variant(g, rhmc.RHMC_PREC_FP32, nrhs)
    var64 = rhmc.rhmc_dslash_variant(g, rhmc.RHMC_PREC_FP64, nrhs)
    log(f"hopping launch variants: fp32 x{nrhs} {var32}, fp64 x{nrhs} {var64}")
    byts = dslash_bytes_per_site("fp32", nrhs) * Vh
    t32_4 = time_dslash("fp32", nrhs, args.dslash_reps)
    avg, avg_med, avg_min = t32_4
    achieved = byts / avg / 1e9
    byts64_4 = dslash_bytes_per_site("fp64c", nrhs) * Vh
    t64_4 = time_dslash("fp64", nrhs, args.dslash_reps)
    log(f"hopping fp32-12 x{nrhs}: {avg * 1e6:.1f} us ({achieved:.0f} GB/s; per-launch events: "
        f"median {avg_med * 1e6:.1f} us); fp64-12 x{nrhs}: {t64_4[0] * 1e6:.1f} us "
        f"({byts64_4 / t64_4[0] / 1e9:.0f} GB/s)")
    if args.only_dslash:
        time_dslash("fp32", 8, args.dslash_reps)
        log("hopping fp32-12 x8 timed")
        # a plain copy of known size for calibrating the HBM byte counters
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy of 256 MiB done")
        return

    dslash = {
        f"fp32_12_{nrhs}rhs": dentry(t32_4, byts, Vh, nrhs),
        f"fp64_12_{nrhs}rhs": dentry(t64_4, byts64_4, Vh, nrhs),
    }
    t8 = time_dslash("fp32", 8, args.dslash_reps)
    dslash["fp32_12_8rhs"] = dentry(t8, dslash_bytes_per_site("fp32", 8) * Vh, Vh, 8)
    t1 = time_dslash("fp32", 1, args.dslash_reps)
    dslash["fp32_12_1rhs"] = dentry(t1, dslash_bytes_per_site("fp32", 1) * Vh, Vh, 1)
    t641 = time_dslash("fp64", 1, args.dslash_reps)
    dslash["fp64_12_1rhs"] = dentry(t641, dslash_bytes_per_site("fp64c", 1) * Vh, Vh, 1)
    # the four-rhs launch with a 1 GiB buffer read between launches: no link
    # or vector can be served from the 256 MB Infinity Cache
    junk = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    _, avg_cold, avg_cold_min = time_dslash("fp32", nrhs, args.dslash_reps, flush=junk)
    del junk
    log(f"fp32-12 x8 {t8[0] * 1e6:.1f} us, x1 {t1[0] * 1e6:.1f} us; fp64-12 x1 {t641[0] * 1e6:.1f} us; "
        f"fp32-12 x{nrhs} cold cache {avg_cold * 1e6:.1f} us (per-launch median; warm: {avg_med * 1e6:.1f} us)")

    # ---------------------------------------------------------------- headline solves
    # The 48^3x12 solves use the library's default launch variants (tune = 0,
    # the library default), which come from timing every variant on this
    # lattice: tuning again inside a solve picks among variants a few per
    # cent apart, differently from run to run.  The 32^3x8 workloads below
    # tune (tune = 1).
    prm_mixed = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_MIXED, tune=0, block=args.block)
    prm_fp64 = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_FP64, tune=0)

    def step(prm, out=y):
        return rhmc.rhmc_rational_apply(g, m, rat.alpha0, rat.alpha, rat.beta, bd, out, prm)

    for w in range(args.warmup):
        st = step(prm_mixed)
        log(f"warmup {w}: {st['time_ms']:.1f} ms, {st['total_iterations']} iterations, "
            f"max true residual {st['max_true_residual']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, step_s = [], []
    for k in range(args.steps):
        ts_ = time.perf_counter()
        stats.append(step(prm_mixed))   # returns once the result is complete
        step_s.append(time.perf_counter() - ts_)
        log(f"step {k}: {stats[-1]['time_ms']:.1f} ms")
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / max(1, args.steps)
    t_mixed_med = sorted(step_s)[len(step_s) // 2] if step_s else t_mixed
    st = stats[-1] if stats else step(prm_mixed)
    K_mixed = args.block if 50 % args.block == 0 else 25

    step(prm_fp64)   # tunes the FP64 launch variants and builds the FP64 graphs (untimed)
    fp64_times = []
    for k in range(args.fp64_runs):
        torch.cuda.synchronize()
        t1_ = time.perf_counter()
        st64 = step(prm_fp64)
        torch.cuda.synchronize()
        fp64_times.append(time.perf_counter() - t1_)
        log(f"fp64 solve {k}: {fp64_times[-1] * 1e3:.1f} ms, {st64['total_iterations']} iterations")
    t_fp64 = sorted(fp64_times)[len(fp64_times) // 2]

    # the same MIXED solve with the library's default block length (32 asked,
    # 25 used so that replacements fall every 50 iterations)
    prm_b25 = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_MIXED, tune=0)
    torch.cuda.synchronize()
    t1_ = time.perf_counter()
    st25 = step(prm_b25)
    torch.cuda.synchronize()
    t_b25 = time.perf_counter() - t1_

    # per-shift error of the MIXED shifted solutions against the GPU's FP64
    # ones (the multi-shift solves behind the rational apply)
    xm = torch.empty((nrhs, len(rat.beta), 3, Vh), dtype=torch.complex128, device=dev)
    x64 = torch.empty_like(xm)
    rhmc.rhmc_multishift_cg(g, m, rat.beta, bd, xm, prm_mixed)
    rhmc.rhmc_multishift_cg(g, m, rat.beta, bd, x64, prm_fp64)
    err_c5 = per_shift_errors(torch, xm, x64)
    del xm, x64
    log(f"mixed vs fp64 per-shift error: max {max(err_c5):.2e}")

    time_to_solution = {
        "mixed_batched": round(t_mixed, 4),
        "mixed_batched_median": round(t_mixed_med, 4),
        "fp64": round(t_fp64, 4),
        "mixed_over_fp64_speedup": round(t_fp64 / t_mixed_med, 3),
        "mixed_batched_runs": [round(v, 4) for v in step_s],
        "fp64_runs": [round(v, 4) for v in sorted(fp64_times)],
        "mixed_block": K_mixed,
        "mixed_block_25_s": round(t_b25, 4),
        "iterations": {"mixed_batched": st["total_iterations"], "fp64": st64["total_iterations"]},
        "max_true_residual": {"mixed_batched": st["max_true_residual"], "fp64": st64["max_true_residual"]},
        "reliable_updates": st["reliable_updates"],
        "reliable_every": 50,
        "fp64_head_iterations": st["fp64_head_iterations"],
        "refine_iterations": int(st["refine_iterations"].sum()),
        "shifts_refined": int((st["refine_iterations"] > 0).sum()),
        "mixed_phases": phases_entry(Vh, nrhs, len(rat.beta), K_mixed, st),
        "fp64_phases": phases_entry(Vh, nrhs, len(rat.beta), 32, st64),
        "mixed_vs_gpu_fp64_rel_error_per_shift": err_c5,
        # launch variants of the solves (the library's defaults)
        "hop_variants": {"fp32": rhmc.rhmc_dslash_variant(g, rhmc.RHMC_PREC_FP32, nrhs),
                         "fp64": rhmc.rhmc_dslash_variant(g, rhmc.RHMC_PREC_FP64, nrhs)},
        "note": ("mixed: mean wall time of the timed steps (mixed_batched) and median of the "
                 "per-step host times (mixed_batched_median); fp64: median of the listed runs after "
                 "one untimed run; speedup from the two medians; per-shift error = max over rhs of ||x_mixed - x_fp64|| / ||x_fp64|| "
                 "against the GPU's FP64 multi-shift solution (both certified to 1e-10 by their "
                 "FP64 true residuals)"),
    }

    extras = {}
    workloads = {}
    gpu_times = {}
    if not args.no_extras:
        # MIXED with FP32 from the first iteration (no FP64 phase)
        prm_nh = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_MIXED, tune=0, fp64_head=-1.0,
                                    block=args.block)
        torch.cuda.synchronize()
        t1_ = time.perf_counter()
        st_nh = step(prm_nh)
        torch.cuda.synchronize()
        extras["mixed_batched_without_fp64_phase"] = {
            "s": round(time.perf_counter() - t1_, 4), "iterations": st_nh["total_iterations"],
            "refine_iterations": int(st_nh["refine_iterations"].sum()),
            "shifts_refined": int((st_nh["refine_iterations"] > 0).sum()),
            "max_true_residual": st_nh["max_true_residual"],
            "phases": phases_entry(Vh, nrhs, len(rat.beta), K_mixed, st_nh)}
        # two-pass FP64 rational apply (no shifted vectors)
        prm_tp = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_FP64, tune=0, two_pass=1)
        y_tp = torch.empty_like(y)
        torch.cuda.synchronize()
        t1_ = time.perf_counter()
        st_tp = rhmc.rhmc_rational_apply(g, m, rat.alpha0, rat.alpha, rat.beta, bd, y_tp, prm_tp)
        torch.cuda.synchronize()
        t_tp = time.perf_counter() - t1_
        y64 = torch.empty_like(y)
        step(prm_fp64, y64)
        extras["rational_apply_two_pass_fp64"] = {
            "s": round(t_tp, 4), "iterations_per_pass": st_tp["total_iterations"],
            "rel_diff_vs_one_pass_fp64": float(torch.linalg.vector_norm(y_tp - y64) / torch.linalg.vector_norm(y64))}
        del y_tp, y64
        # pseudofermion heat bath, action and force (MIXED batched)
        rh_ = rational_for(HEADLINE_CFG, c["hb_power"])
        gen = torch.Generator(device=dev)
        gen.manual_seed(3000 + HEADLINE_CFG)
        R = torch.complex(torch.randn((nrhs, 3, Vh), dtype=torch.float64, device=dev, generator=gen),
                          torch.randn((nrhs, 3, Vh), dtype=torch.float64, device=dev, generator=gen))
        R *= 0.5 ** 0.5
        phi = torch.empty_like(R)
        torch.cuda.synchronize()
        t1_ = time.perf_counter()
        rhmc.rhmc_rational_apply(g, m, rh_.alpha0, rh_.alpha, rh_.beta, R, phi, prm_mixed)
        torch.cuda.synchronize()
        t_hb = time.perf_counter() - t1_
        t1_ = time.perf_counter()
        S, _ = rhmc.rhmc_pf_action(g, m, rat.alpha0, rat.alpha, rat.beta, phi, prm_mixed)
        torch.cuda.synchronize()
        t_act = time.perf_counter() - t1_
        R2 = (R.abs() ** 2).sum(dim=(1, 2)).cpu().numpy()
        Fdev = torch.empty(tuple(reversed(L)) + (4, 3, 3), dtype=torch.complex128, device=dev)
        t1_ = time.perf_counter()
        rhmc.rhmc_pf_force(g, m, rat.alpha0, rat.alpha, rat.beta, phi, Fdev, prm_mixed)
        torch.cuda.synchronize()
        t_force = time.perf_counter() - t1_
        del Fdev, R, phi
        extras["pseudofermion"] = {"heatbath_s": round(t_hb, 4), "action_s": round(t_act, 4),
                                   "force_s": round(t_force, 4),
                                   "max_abs_S_over_RR_minus_1": float(np.max(np.abs(S / R2 - 1)))}
        # molecular-dynamics kernels on this lattice
        extras["md_kernels"] = time_md_kernels(rhmc, torch, dev, g, lat, L)
    # link storages other than the defaults, same lattice
    if not args.no_extras:
        ghl = rhmc.rhmc_gauge_create(lat, U, flags=rhmc.RHMC_LINKS_HILO_12)
        thl = time_dslash("fp64", 1, args.dslash_reps, gauge=ghl)
        ghl.close()
        dslash["fp64_hilo12_1rhs"] = dentry(thl, dslash_bytes_per_site("fp64hl", 1) * Vh, Vh, 1)
        g18 = rhmc.rhmc_gauge_create(lat, U, flags=rhmc.RHMC_LINKS_FP64_18)
        t18 = time_dslash("fp64", 1, args.dslash_reps, gauge=g18)
        g18.close()
        dslash["fp64_18_1rhs"] = dentry(t18, dslash_bytes_per_site("fp64", 1) * Vh, Vh, 1)
        gf = rhmc.rhmc_gauge_create(lat, U, flags=rhmc.RHMC_LINKS_FP32_18 | rhmc.RHMC_LINKS_FP64_12)
        tf4 = time_dslash("fp32", nrhs, args.dslash_reps, gauge=gf)
        gf.close()
        dslash[f"fp32_18_{nrhs}rhs"] = dentry(tf4, dslash_bytes_per_site("fp32f", nrhs) * Vh, Vh, nrhs)
    traffic = traffic_from_profile(f"dslash_fp32_{nrhs}rhs_{'x'.join(str(v) for v in L)}", var32)
    g.close()
    np.save(os.path.join(workdir, "c5_links.npy"), U)
    del U

    # ---------------------------------------------------------------- other workloads
    if not args.no_extras:
        # 4^4 and 16^3 x 4: FP64 multi-shift solves, kept for the oracle comparison
        for cfg, powers in ((1, (-0.25,)), (2, (-0.25, 0.25))):
            cc = synth.CONFIGS[cfg]
            Uc, bc = extra_inputs[cfg]
            latc = rhmc.rhmc_lattice_create(cc["L"], -1)
            gc = rhmc.rhmc_gauge_create(latc, Uc)
            bcd = torch.from_numpy(bc).to(dev)
            entry = {"lattice": list(cc["L"]), "mass": cc["m"], "tol": cc["tol"], "mode": "fp64"}
            for p in powers:
                rc = rational_for(cfg, p)
                prm = rhmc.solver_params(tol=cc["tol"], mode=rhmc.RHMC_MODE_FP64)
                x = torch.empty((1, len(rc.beta), 3, latc.Vh), dtype=torch.complex128, device=dev)
                rhmc.rhmc_multishift_cg(gc, cc["m"], rc.beta, bcd, x, prm)   # untimed (graphs)
                torch.cuda.synchronize()
                t1_ = time.perf_counter()
                stc = rhmc.rhmc_multishift_cg(gc, cc["m"], rc.beta, bcd, x, prm)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1_
                np.save(os.path.join(workdir, f"c{cfg}_p{p:+.2f}.npy"), x.cpu().numpy())
                entry[f"x^{p:+.2f}"] = {"poles": len(rc.beta), "time_to_solution_s": round(dt, 5),
                                        "iterations": stc["total_iterations"],
                                        "max_true_residual": stc["max_true_residual"]}
                if cfg == 2 and p < 0:
                    gpu_times["c2"] = round(dt, 5)
            if cfg == 2:
                # 1000 standalone FP64 D_oe applications (cache resident: 9.4 MB of FP64-18 links)
                g2 = rhmc.rhmc_gauge_create(latc, Uc, flags=rhmc.RHMC_LINKS_FP64_18)
                v2 = torch.randn((1, 3, latc.Vh), dtype=torch.complex128, device=dev)
                o2 = torch.empty_like(v2)
                for _ in range(20):
                    rhmc.rhmc_dslash_eo(g2, 1, rhmc.RHMC_PREC_FP64, 1, v2, o2)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(1000):
                    rhmc.rhmc_dslash_eo(g2, 1, rhmc.RHMC_PREC_FP64, 1, v2, o2)
                e1.record()
                e1.synchronize()
                t2 = e0.elapsed_time(e1) / 1e3 / 1000
                g2.close()
                entry["dslash_fp64_18_1000_applications"] = {
                    "us_per_application": round(t2 * 1e6, 3),
                    "GBps": round(dslash_bytes_per_site("fp64", 1) * latc.Vh / t2 / 1e9, 1),
                    "note": "back to back between one pair of events; 32 workgroups per launch: "
                            "launch- and cache-bound"}
            gc.close()
            workloads[f"c{cfg}_{'x'.join(str(v) for v in cc['L'])}"] = entry
        # 32^3 x 8: 1 rhs MIXED (error per shift) and 8 rhs MIXED batched
        for cfg in (3, 4):
            cc = synth.CONFIGS[cfg]
            Uc, bc = extra_inputs[cfg]
            latc = rhmc.rhmc_lattice_create(cc["L"], -1)
            gc = rhmc.rhmc_gauge_create(latc, Uc)
            bcd = torch.from_numpy(bc).to(dev)
            rc = rational_for(cfg, -0.25)
            nr = bc.shape[0]
            pm = rhmc.solver_params(tol=cc["tol"], mode=rhmc.RHMC_MODE_MIXED, tune=1, block=args.block)
            p64 = rhmc.solver_params(tol=cc["tol"], mode=rhmc.RHMC_MODE_FP64, tune=1)
            xm = torch.empty((nr, len(rc.beta), 3, latc.Vh), dtype=torch.complex128, device=dev)
            x64 = torch.empty_like(xm)
            rhmc.rhmc_multishift_cg(gc, cc["m"], rc.beta, bcd, xm, pm)   # untimed (tuning, graphs)
            torch.cuda.synchronize()
            t1_ = time.perf_counter()
            stm = rhmc.rhmc_multishift_cg(gc, cc["m"], rc.beta, bcd, xm, pm)
            torch.cuda.synchronize()
            tm = time.perf_counter() - t1_
            rhmc.rhmc_multishift_cg(gc, cc["m"], rc.beta, bcd, x64, p64)
            torch.cuda.synchronize()
            t1_ = time.perf_counter()
            st6 = rhmc.rhmc_multishift_cg(gc, cc["m"], rc.beta, bcd, x64, p64)
            torch.cuda.synchronize()
            t6 = time.perf_counter() - t1_
            yy = torch.empty_like(bcd)
            torch.cuda.synchronize()
            t1_ = time.perf_counter()
            rhmc.rhmc_rational_apply(gc, cc["m"], rc.alpha0, rc.alpha, rc.beta, bcd, yy, pm)
            torch.cuda.synchronize()
            tr = time.perf_counter() - t1_
            err = per_shift_errors(torch, xm, x64)
            if cfg == 3:
                np.save(os.path.join(workdir, "c3_mixed.npy"), xm.cpu().numpy())
                np.save(os.path.join(workdir, "c3_links.npy"), Uc)
            workloads[f"c{cfg}_{'x'.join(str(v) for v in cc['L'])}_{nr}rhs"] = {
                "lattice": list(cc["L"]), "mass": cc["m"], "nrhs": nr, "poles": len(rc.beta), "tol": cc["tol"],
                "multishift_mixed_s": round(tm, 4), "multishift_fp64_s": round(t6, 4),
                "rational_apply_mixed_s": round(tr, 4),
                "iterations": {"mixed": stm["total_iterations"], "fp64": st6["total_iterations"],
                               "fp64_head": stm["fp64_head_iterations"],
                               "refine": int(stm["refine_iterations"].sum())},
                "reliable_updates": stm["reliable_updates"],
                "max_true_residual": {"mixed": stm["max_true_residual"], "fp64": st6["max_true_residual"]},
                "mixed_vs_gpu_fp64_rel_error_per_shift": err,
                "mixed_phases": phases_entry(latc.Vh, nr, len(rc.beta), K_mixed, stm),
                "hop_variants": {"fp32": rhmc.rhmc_dslash_variant(gc, rhmc.RHMC_PREC_FP32, nr),
                                 "fp64": rhmc.rhmc_dslash_variant(gc, rhmc.RHMC_PREC_FP64, nr)}}
            del xm, x64
            gc.close()
        extras["md_trajectory_16x16x16x4"] = run_md_trajectory(rhmc, torch, dev, args.md_trajectories)

    out = {
        "metric": METRIC,
        "value": round(achieved, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "48^3x12, eps 0.8, m 0.005, 4 rhs x 20-pole x^-1/4, MIXED batched, tol 1e-10",
            "lattice": list(L), "nrhs": nrhs, "npole": len(rat.beta), "mass": m, "tol": c["tol"],
            "plaquette": round(plaquette, 6),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel": f"hopping FP32 12-real, {nrhs} rhs, launch variant {var32}, {avg * 1e6:.2f} us per "
                      f"launch (average of {args.dslash_reps} back-to-back launches between one pair of HIP "
                      f"events on the launching stream; with per-launch events: median "
                      f"{avg_med * 1e6:.2f}, min {avg_min * 1e6:.2f}), "
                      f"{byts / 1e6:.1f} MB algorithmic per launch",
            "cold_cache": {"us_median": round(avg_cold * 1e6, 2), "us_min": round(avg_cold_min * 1e6, 2),
                           "GBps": round(byts / avg_cold / 1e9, 1),
                           "warm_us_median": round(avg_med * 1e6, 2),
                           "note": "per-launch events with a 1 GiB buffer read between launches (outside "
                                   "the events); compare with the warm per-launch median"},
            "gflops": round(FLOPS_PER_SITE * Vh * nrhs / avg / 1e9, 1),
        },
        "dslash": dslash,
        "time_to_solution_s": time_to_solution,
        "workloads": workloads,
        "extras": extras,
    }
    if not args.no_cpu_baseline and not args.no_extras:
        out["cpu_baseline"] = run_cpu_baseline(workdir, st["total_iterations"], nrhs, gpu_times)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
