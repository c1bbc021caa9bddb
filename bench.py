#!/usr/bin/env python
"""Benchmark of the staggered RHMC hot path on one MI355X.

Workload (default): 48^3 x 12 lattice, links exp(i*0.8*H), m = 0.005, four
Gaussian pseudofermion sources, the 20-pole rational approximation of x^-1/4
on [m^2, 16 + m^2], tolerance 1e-10 per shift.  One step is one call of
rhmc_rational_apply in MIXED precision with all four right-hand sides batched:
multi-shift CG (FP32 12-real hopping term, FP64 reductions and recurrences,
FP64 reliable updates), FP64 true-residual check and refinement, FP64 combine.

Printed JSON line:
  value        effective GB/s of the FP32 12-real four-rhs hopping kernel (the
               kernel the solve spends its time in), algorithmic bytes per
               launch / average launch time from HIP events on its stream;
  ms_per_step  wall time of one mixed + batched solve;
  time_to_solution_s  the same solve in MIXED + batched and in plain FP64;
  roofline     the hopping kernel against the 8 TB/s HBM peak;
  md_kernels   the gauge-force kick and link update on the same lattice;
  md_trajectory_16x16x16x4  seconds per trajectory of the molecular-dynamics
               workload of the algorithm tests (4 x 16^3, beta 5.264,
               am 0.01335, 2 pseudofermions, n_md 12, dtau_f/dtau_g 10), with
               mixed MD solves and FP64 Metropolis solves, and all FP64;
  cpu_baseline the FP64 numpy oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("Dslash GB/s (% HBM peak); multi-shift CG time to r≤10^-10, FP64 vs mixed+batched")
HBM_PEAK_GBPS = 8000.0
FLOPS_PER_SITE = 570   # 8 SU(3) x vector products (66) + 7 vector additions (6)
WORKLOADS = {
    # name: (config index, description)
    "c5": (5, "48^3x12, eps 0.8, m 0.005, 4 rhs x 20-pole x^-1/4, MIXED batched, tol 1e-10"),
    "c4": (4, "32^3x8, eps 0.7, m 0.01, 8 rhs x 15-pole x^-1/4, MIXED batched, tol 1e-10"),
    "c3": (3, "32^3x8, eps 0.7, m 0.01, 1 rhs x 15-pole x^-1/4, MIXED, tol 1e-10"),
}


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
    """Hash of the hopping kernel's sources (kernel file and its header)."""
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


def cpu_baseline(U, b, m, rat, gpu_iters):
    """Time the FP64 oracle on a bounded sample of the same workload."""
    import numpy as np

    from oracle import dirac

    Vh = b.shape[-1]
    reps_d, iters = 2, 8   # about 12 s of host work on the 48^3x12 lattice
    t0, c0 = time.perf_counter(), time.process_time()
    for _ in range(reps_d):
        dirac.dslash(U, b[:1], 1)
    t_d = (time.perf_counter() - t0) / reps_d
    # a few iterations of the oracle's multi-shift CG on one rhs, all shifts
    from oracle import solvers

    t1 = time.perf_counter()
    solvers.multishift_cg(lambda v: dirac.mdagm(U, m, v), b[0], np.asarray(rat.beta),
                          tol=1e-10, maxiter=iters)
    t_it = (time.perf_counter() - t1) / iters
    beta = np.asarray(rat.beta)
    cpu_total = time.process_time() - c0
    wall_total = time.perf_counter() - t0
    gbps = dslash_bytes_per_site("fp64", 1) * Vh / t_d / 1e9
    nrhs = b.shape[0]
    return {
        "value": gbps,
        "unit": "GB/s",
        "cores": max(1, round(cpu_total / wall_total)),
        "kind": "oracle",
        "sample": (f"{reps_d} FP64 D_oe applications on 1 rhs ({t_d:.2f} s each, counted at "
                   f"{dslash_bytes_per_site('fp64', 1)} B/site) and {iters} multi-shift CG "
                   f"iterations on 1 rhs with {beta.size} shifts ({t_it:.2f} s each) of the "
                   f"same lattice and field"),
        "seconds_per_cg_iteration_per_rhs": t_it,
        "time_to_solution_s_extrapolated": t_it * gpu_iters * nrhs,
        "wall_seconds": wall_total,
        "cpu_seconds": cpu_total,
        "host": host_description(),
    }


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


# Molecular-dynamics kernels, per link (FP64-12 links, FP64 momenta of 8 reals):
# the gauge-force kick reads every link once and the momenta once and writes
# the momenta; the link update reads link and momenta and writes the FP64-12
# and FP32-12 copies.  Flops of the kick: 13 complex 3x3 products (198 each),
# 19 third-row rebuilds (42 each), the staple sums and the momentum update.
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


def run_md_workload(rhmc, torch, dev, ntraj):
    """Trajectories of the molecular-dynamics workload (Sec. 4.4 settings) in
    three precision settings: MD solves MIXED at r_md = 1e-3 with FP64
    Metropolis solves at r_metro = 1e-9 (the paper's MP_1), everything FP64 at
    1e-9 (D_1), and MP_1 with MIXED Metropolis solves (FP64 phase, then FP32,
    FP64-certified), which the paper rules out for shifted solvers.  One
    untimed trajectory, then `ntraj` timed ones."""
    import numpy as np

    import synth
    from synth.make_rational import md_rationals

    w = synth.MD_WORKLOAD
    L = w["L"]
    r_hb, r_act, r_md = md_rationals()
    U = synth.gauge_field(L, w["eps"], w["seed"])
    out = {"lattice": list(L), "beta": w["beta"], "mass": w["m"], "npf": w["npf"],
           "n_md": w["n_md"], "gauge_steps": w["gauge_steps"], "tau": w["tau"],
           "poles_md": len(r_md.beta), "poles_metropolis": len(r_act.beta),
           "gauge_field": "synthetic, not thermalised"}
    settings = {
        "MP1_mixed_md_1e-3_fp64_metropolis_1e-9": (rhmc.RHMC_MODE_MIXED, 1e-3, rhmc.RHMC_MODE_FP64),
        "D1_fp64_1e-9": (rhmc.RHMC_MODE_FP64, 1e-9, rhmc.RHMC_MODE_FP64),
        "mixed_md_1e-3_mixed_metropolis_1e-9": (rhmc.RHMC_MODE_MIXED, 1e-3, rhmc.RHMC_MODE_MIXED),
    }
    for name, (mode, md_tol, metro_mode) in settings.items():
        lat = rhmc.rhmc_lattice_create(L, -1)
        g = rhmc.rhmc_gauge_create(lat, U)
        metro = rhmc.solver_params(tol=1e-9, mode=metro_mode)
        mdp = rhmc.MDParams(r_md, beta=w["beta"], mass=w["m"], tau=w["tau"], n_md=w["n_md"],
                            gauge_steps=w["gauge_steps"],
                            solver=rhmc.solver_params(tol=md_tol, mode=mode))
        hp = rhmc.HMCParams(mdp, r_hb, r_act, metro)
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
        out[name] = {
            "s_per_trajectory": round(float(np.mean(times)), 4),
            "runs_s": [round(t, 4) for t in times],
            "dH": [round(s["dH"], 5) for s in stats],
            "accepted": [s["accepted"] for s in stats],
            "fermion_forces": stats[-1]["md"]["fermion_forces"],
            "gauge_forces": stats[-1]["md"]["gauge_forces"],
            "link_updates": stats[-1]["md"]["link_updates"],
            "md_cg_iterations": stats[-1]["md"]["cg_iterations"],
            "md_s": round(stats[-1]["md"]["time_ms"] / 1e3, 4),
        }
        log(f"trajectory {name}: {out[name]['s_per_trajectory']:.3f} s, dH {out[name]['dH']}, "
            f"MD {out[name]['md_s']:.3f} s, {out[name]['md_cg_iterations']} CG iterations in "
            f"{out[name]['fermion_forces']} force solves")
    return out


def run_md_chain(rhmc, torch, ntraj, metropolis="fp64"):
    """A Markov chain of `ntraj` trajectories of the molecular-dynamics
    workload from its synthetic start: momenta, pseudofermion sources and the
    Metropolis numbers drawn on the host (numpy PCG64, seed 123).  Over the
    second half, <exp(-dH)> must be 1 (the equality that holds at equilibrium
    for a reversible, area-preserving integrator with an exact Metropolis
    test).  `metropolis` sets the precision of the heat-bath and action solves
    at 1e-10: plain FP64, as the paper requires, or MIXED (FP64 phase, then
    FP32 with reliable updates, certified by FP64 true residuals)."""
    import numpy as np

    import synth
    from synth.make_rational import md_rationals

    w = synth.MD_WORKLOAD
    L = w["L"]
    r_hb, r_act, r_md = md_rationals()
    lat = rhmc.rhmc_lattice_create(L, -1)
    g = rhmc.rhmc_gauge_create(lat, synth.gauge_field(L, w["eps"], w["seed"]))
    mdp = rhmc.MDParams(r_md, beta=w["beta"], mass=w["m"], tau=w["tau"], n_md=w["n_md"],
                        gauge_steps=w["gauge_steps"],
                        solver=rhmc.solver_params(tol=1e-7, mode=rhmc.RHMC_MODE_MIXED))
    mode = rhmc.RHMC_MODE_MIXED if metropolis == "mixed" else rhmc.RHMC_MODE_FP64
    hp = rhmc.HMCParams(mdp, r_hb, r_act, rhmc.solver_params(tol=1e-10, mode=mode))
    rng = np.random.default_rng(123)
    rows = []
    t0 = time.perf_counter()
    for k in range(ntraj):
        R = torch.from_numpy((rng.standard_normal((w["npf"], 3, lat.Vh)) +
                              1j * rng.standard_normal((w["npf"], 3, lat.Vh))) * np.sqrt(0.5)).cuda()
        mom = torch.from_numpy(rng.standard_normal((8, 4, 2, lat.Vh))).cuda()
        st = rhmc.rhmc_trajectory(g, hp, R, mom, float(rng.uniform()), allow_not_converged=True)
        plaq = 1.0 - rhmc.rhmc_gauge_action(g, 1.0) / (6.0 * lat.V)
        rows.append((st["dH"], float(st["accepted"]), plaq))
        if k % 20 == 19:
            log(f"chain trajectory {k + 1}: plaquette {plaq:.5f}, dH {st['dH']:.4f}")
    g.close()
    a = np.array(rows)
    half = a[len(a) // 2:]
    e = np.exp(-half[:, 0])
    return {"trajectories": ntraj, "measured": len(half),
            "exp_minus_dH_mean": float(e.mean()), "exp_minus_dH_err": float(e.std() / np.sqrt(len(e))),
            "acceptance": float(half[:, 1].mean()), "plaquette": float(half[:, 2].mean()),
            "plaquette_err": float(half[:, 2].std() / np.sqrt(len(half))),
            "seconds": round(time.perf_counter() - t0, 1),
            "setting": f"MIXED MD solves at 1e-7, {metropolis.upper()} Metropolis solves at 1e-10",
            "dH": [float(v) for v in a[:, 0]]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--dslash-reps", type=int, default=200)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison solve")
    ap.add_argument("--fp64-runs", type=int, default=3, help="timed plain FP64 solves (median reported)")
    ap.add_argument("--md-tol", type=float, default=1e-7,
                    help="also time MIXED and FP64 at this looser tolerance (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--two-pass-runs", type=int, default=1,
                    help="timed two-pass FP64 rational applies (no shifted vectors)")
    ap.add_argument("--no-head-runs", type=int, default=1,
                    help="timed MIXED solves with no FP64 phase (fp64_head < 0), for comparison")
    ap.add_argument("--no-pf", action="store_true", help="skip the pseudofermion heat bath + action")
    ap.add_argument("--no-md", action="store_true",
                    help="skip the molecular-dynamics kernels and the 4x16^3 trajectories")
    ap.add_argument("--only-md", action="store_true",
                    help="only the molecular-dynamics kernels and trajectories (profiler runs)")
    ap.add_argument("--md-chain", type=int, default=0,
                    help="run a Markov chain of this many trajectories of the 4x16^3 workload "
                         "(MIXED MD solves at 1e-7, FP64 Metropolis at 1e-10) and report "
                         "<exp(-dH)>, acceptance and plaquette over its second half")
    ap.add_argument("--md-chain-metropolis", default="fp64", choices=("fp64", "mixed"),
                    help="precision of the chain's heat-bath and action solves")
    ap.add_argument("--md-trajectories", type=int, default=2,
                    help="timed trajectories per setting of the 4x16^3 workload (after one untimed)")
    ap.add_argument("--only-dslash", action="store_true",
                    help="only the hopping-kernel timing and a copy of known size (counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(see the sharding design); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth
    from synth.make_rational import rational_for

    cfg, desc = WORKLOADS[args.workload]
    c = synth.CONFIGS[cfg]
    L, m, nrhs = c["L"], c["m"], c["nrhs"]
    t0 = time.perf_counter()
    U = synth.gauge_field(L, c["eps"], synth.fields.seed_gauge(cfg))
    b = synth.source(L, synth.fields.seed_source(cfg), nrhs)
    rat = rational_for(cfg, -0.25)
    log(f"inputs for {desc} ready in {time.perf_counter() - t0:.1f} s")

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
    # average plaquette Re Tr P / 3 of the field (roughness descriptor): S_g at beta = 1 is sum (1 - Re Tr P / 3)
    plaquette = 1.0 - rhmc.rhmc_gauge_action(g, 1.0) / (6.0 * lat.V)

    def time_call(fn, reps, warm=3):
        """Median and min duration of fn's launches, each bracketed by HIP events."""
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

    def wall_call(fn, reps):
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / reps

    def md_kernel_timings():
        mom = torch.from_numpy(synth.momenta(L, 4000 + cfg)).to(dev)
        beta_g, eps_g = synth.MD_WORKLOAD["beta"], 0.004   # about half a gauge step of the MD workload
        t_gf, t_gf_min = time_call(lambda: rhmc.rhmc_gauge_force_kick(g, beta_g, 1e-9, mom), 50)
        t_up, t_up_min = time_call(lambda: rhmc.rhmc_update_links(g, eps_g, mom), 50)
        t_pl = wall_call(lambda: rhmc.rhmc_gauge_action(g, beta_g), 20)
        t_kin = wall_call(lambda: rhmc.rhmc_kinetic(g, mom), 20)
        nl = 4 * lat.V
        res = {
            "gauge_force_kick": kernel_entry(t_gf, t_gf_min, GF_BYTES_PER_LINK * nl, GF_FLOPS_PER_LINK * nl),
            "link_update": kernel_entry(t_up, t_up_min, UP_BYTES_PER_LINK * nl, None),
            "plaquette_action_call_ms": round(t_pl * 1e3, 3),
            "kinetic_call_ms": round(t_kin * 1e3, 3),
            "note": "HIP events around each launch; GB/s counts each FP64-12 link, momentum "
                    "and written storage once (neighbour links re-read from cache are not counted); "
                    "the action and kinetic calls include the read-back of one scalar",
        }
        log(f"gauge force kick {t_gf * 1e6:.0f} us ({res['gauge_force_kick']['GBps']} GB/s, "
            f"{res['gauge_force_kick']['gflops']} GFLOP/s), link update {t_up * 1e6:.0f} us "
            f"({res['link_update']['GBps']} GB/s), action {t_pl * 1e3:.2f} ms, kinetic {t_kin * 1e3:.2f} ms")
        return res

    if args.only_md:
        res = {"md_kernels": md_kernel_timings()}
        g.close()
        res["md_trajectory_16x16x16x4"] = run_md_workload(rhmc, torch, dev, args.md_trajectories)
        if args.md_chain > 0:
            res["md_chain_16x16x16x4"] = run_md_chain(rhmc, torch, args.md_chain, args.md_chain_metropolis)
        print(json.dumps(res), flush=True)
        return

    # ---------------------------------------------------------------- hopping kernel
    def time_dslash(prec, k, reps, gauge=None, vh=None, warm=20, flush=None):
        """Median and min launch time of D_oe over `reps` launches, each
        bracketed by its own pair of HIP events on the launching stream;
        with `flush` (a device buffer), the buffer is streamed through a
        reduction between launches, outside the events, so no cache holds the
        operands (reading, not writing, leaves no dirty lines to write back)."""
        gg = gauge if gauge is not None else g
        n = vh if vh is not None else Vh
        dt = torch.complex64 if prec == "fp32" else torch.complex128
        pr = rhmc.RHMC_PREC_FP32 if prec == "fp32" else rhmc.RHMC_PREC_FP64
        src = bd[:k] if vh is None else torch.randn((k, 3, n), dtype=torch.complex128, device=dev)
        vin = src.to(dt).contiguous()
        vout = torch.empty_like(vin)
        for _ in range(warm):
            rhmc.rhmc_dslash_eo(gg, 1, pr, k, vin, vout)
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for i, (e0, e1) in enumerate(ev):
            if flush is not None:
                flush.max()
            e0.record(s)
            rhmc.rhmc_dslash_eo(gg, 1, pr, k, vin, vout)
            e1.record(s)
        ev[-1][1].synchronize()
        ts = sorted(e0.elapsed_time(e1) / 1e3 for e0, e1 in ev)
        return ts[len(ts) // 2], ts[0], dslash_bytes_per_site(prec, k) * n

    # the timed hopping launches use the library's measured default launch
    # variants (the solver below tunes its own), so that counter runs of
    # --only-dslash see the same kernel
    var32 = rhmc.rhmc_dslash_variant(g, rhmc.RHMC_PREC_FP32, nrhs)
    var64 = rhmc.rhmc_dslash_variant(g, rhmc.RHMC_PREC_FP64, 1)
    log(f"hopping launch variants: fp32 x{nrhs} {var32}, fp64 x1 {var64}")
    avg, avg_min, byts = time_dslash("fp32", nrhs, args.dslash_reps)
    # the same launches with a 1 GiB buffer read between them: no link or
    # vector can be served from the 256 MB Infinity Cache
    # (not in the counter runs, which average every launch of the kernel)
    avg_cold = avg_cold_min = float("nan")
    if not args.only_dslash:
        junk = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        avg_cold, avg_cold_min, _ = time_dslash("fp32", nrhs, args.dslash_reps, flush=junk)
        del junk
        log(f"hopping fp32-12 x{nrhs} cold cache: {avg_cold * 1e6:.1f} us ({byts / avg_cold / 1e9:.0f} GB/s)")
    avg64, avg64_min, _ = time_dslash("fp64", 1, args.dslash_reps)
    byts64 = dslash_bytes_per_site("fp64c", 1) * Vh   # default storage: FP64-12 links
    avg1, avg1_min, byts1 = time_dslash("fp32", 1, args.dslash_reps)
    achieved = byts / avg / 1e9
    log(f"hopping fp32-12 x{nrhs}: {avg * 1e6:.1f} us ({achieved:.0f} GB/s); "
        f"fp64-12 x1: {avg64 * 1e6:.1f} us ({byts64 / avg64 / 1e9:.0f} GB/s); "
        f"fp32-12 x1: {avg1 * 1e6:.1f} us ({byts1 / avg1 / 1e9:.0f} GB/s)")

    if args.only_dslash:
        # a plain copy of known size for calibrating the HBM byte counters
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy of 256 MiB done")
        return

    prm_mixed = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_MIXED, tune=1)
    prm_fp64 = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_FP64, tune=1)

    def step(prm):
        return rhmc.rhmc_rational_apply(g, m, rat.alpha0, rat.alpha, rat.beta, bd, y, prm)

    for w in range(args.warmup):
        st = step(prm_mixed)
        log(f"warmup {w}: {st['time_ms']:.1f} ms, {st['total_iterations']} iterations, "
            f"max true residual {st['max_true_residual']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stats.append(step(prm_mixed))
        log(f"step {k}: {stats[-1]['time_ms']:.1f} ms")
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / max(1, args.steps)
    st = stats[-1] if stats else step(prm_mixed)

    t_fp64 = None
    st64 = None
    fp64_times = []
    if not args.no_fp64:
        step(prm_fp64)   # tunes the FP64 launch variants and builds the FP64 graphs (untimed)
        for k in range(args.fp64_runs):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st64 = step(prm_fp64)
            torch.cuda.synchronize()
            fp64_times.append(time.perf_counter() - t1)
            log(f"fp64 solve {k}: {fp64_times[-1] * 1e3:.1f} ms, {st64['total_iterations']} iterations")
        t_fp64 = sorted(fp64_times)[len(fp64_times) // 2]
    mixed_times = sorted(s_['time_ms'] / 1e3 for s_ in stats)

    # two-pass FP64 rational apply: no shifted vectors, the base solve twice
    two_pass = None
    if args.two_pass_runs > 0:
        prm_tp = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_FP64, tune=1, two_pass=1)
        y_tp = torch.empty_like(y)
        tp_times = []
        for k in range(args.two_pass_runs):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st_tp = rhmc.rhmc_rational_apply(g, m, rat.alpha0, rat.alpha, rat.beta, bd, y_tp, prm_tp)
            torch.cuda.synchronize()
            tp_times.append(time.perf_counter() - t1)
        diff = float(torch.linalg.vector_norm(y_tp - y) / torch.linalg.vector_norm(y))
        two_pass = {"s": round(sorted(tp_times)[len(tp_times) // 2], 4),
                    "runs_s": [round(v, 4) for v in tp_times],
                    "iterations_per_pass": st_tp["total_iterations"],
                    "max_recurrence_residual": st_tp["max_true_residual"],
                    # y holds the last one-pass result: FP64 unless those runs were skipped
                    "rel_diff_vs_one_pass_y": diff,
                    "one_pass_mode": "fp64" if not args.no_fp64 else "mixed_batched"}
        del y_tp
        log(f"two-pass fp64: {two_pass['s'] * 1e3:.0f} ms, |y - y_one_pass| / |y| = {diff:.1e}")

    # the same MIXED solve in FP32 from the first iteration (no FP64 phase):
    # the shifted systems then carry the FP32 rounding of the early steps and
    # need refinement
    no_head = None
    if args.no_head_runs > 0:
        prm_nh = rhmc.solver_params(tol=c["tol"], mode=rhmc.RHMC_MODE_MIXED, tune=1, fp64_head=-1.0)
        nh_times = []
        for k in range(args.no_head_runs):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st_nh = step(prm_nh)
            torch.cuda.synchronize()
            nh_times.append(time.perf_counter() - t1)
        no_head = {"s": round(sorted(nh_times)[len(nh_times) // 2], 4),
                   "runs_s": [round(v, 4) for v in nh_times],
                   "iterations": st_nh["total_iterations"],
                   "refine_iterations": int(st_nh["refine_iterations"].sum()),
                   "shifts_refined": int((st_nh["refine_iterations"] > 0).sum()),
                   "max_true_residual": st_nh["max_true_residual"]}
        log(f"mixed without the FP64 phase: {no_head['s'] * 1e3:.0f} ms, "
            f"{no_head['refine_iterations']} refinement iterations")

    # the same rational apply at a molecular-dynamics tolerance, where the
    # FP32 operator's shifted-residual gap needs little or no refinement
    md = None
    if args.md_tol > 0:
        md = {"tol": args.md_tol}
        for name, mode in (("mixed_batched", rhmc.RHMC_MODE_MIXED), ("fp64", rhmc.RHMC_MODE_FP64)):
            prm = rhmc.solver_params(tol=args.md_tol, mode=mode, tune=1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st_md = step(prm)
            torch.cuda.synchronize()
            md[name] = round(time.perf_counter() - t1, 4)
            md[name + "_iterations"] = st_md["total_iterations"]
            md[name + "_refine_iterations"] = int(st_md["refine_iterations"].sum())
            md[name + "_fp64_head_iterations"] = st_md["fp64_head_iterations"]
        log(f"tol {args.md_tol:g}: mixed {md['mixed_batched'] * 1e3:.0f} ms, fp64 {md['fp64'] * 1e3:.0f} ms")

    # pseudofermion heat bath phi = r_h(A) R (x^{+1/8}) and action phi^dagger r(A) phi
    pf = None
    if not args.no_pf:
        rh_ = rational_for(cfg, c["hb_power"])
        gen = torch.Generator(device=dev)
        gen.manual_seed(3000 + cfg)
        R = torch.complex(torch.randn((nrhs, 3, Vh), dtype=torch.float64, device=dev, generator=gen),
                          torch.randn((nrhs, 3, Vh), dtype=torch.float64, device=dev, generator=gen))
        R *= 0.5 ** 0.5
        phi = torch.empty_like(R)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rhmc.rhmc_rational_apply(g, m, rh_.alpha0, rh_.alpha, rh_.beta, R, phi, prm_mixed)
        torch.cuda.synchronize()
        t_hb = time.perf_counter() - t1
        t1 = time.perf_counter()
        S, st_pf = rhmc.rhmc_pf_action(g, m, rat.alpha0, rat.alpha, rat.beta, phi, prm_mixed)
        torch.cuda.synchronize()
        t_act = time.perf_counter() - t1
        R2 = (R.abs() ** 2).sum(dim=(1, 2)).cpu().numpy()
        Fdev = torch.empty(tuple(reversed(L)) + (4, 3, 3), dtype=torch.complex128, device=dev)
        t1 = time.perf_counter()
        rhmc.rhmc_pf_force(g, m, rat.alpha0, rat.alpha, rat.beta, phi, Fdev, prm_mixed)
        torch.cuda.synchronize()
        t_force = time.perf_counter() - t1
        del Fdev
        pf = {"heatbath_s": round(t_hb, 4), "action_s": round(t_act, 4), "force_s": round(t_force, 4),
              "max_abs_S_over_RR_minus_1": float(np.max(np.abs(S / R2 - 1))),
              "note": "MIXED batched, x^{+1/8} heat bath, x^{-1/4} action and force; "
                      "S = R^dagger R up to the minimax errors and the solver tolerance"}
        log(f"pseudofermion heat bath {t_hb * 1e3:.0f} ms, action {t_act * 1e3:.0f} ms, "
            f"force {t_force * 1e3:.0f} ms, "
            f"max |S/RR - 1| = {pf['max_abs_S_over_RR_minus_1']:.2e}")

    # molecular-dynamics kernels on this lattice (one lane per link or site)
    md_kernels = md_kernel_timings() if not args.no_md else None

    tag = f"dslash_fp32_{nrhs}rhs_{'x'.join(str(v) for v in L)}"
    traffic = traffic_from_profile(tag, var32)
    g.close()

    trajectories = None
    if not args.no_md:
        trajectories = run_md_workload(rhmc, torch, dev, args.md_trajectories)

    # FP64 operator from hi/lo links (Sec. 4.2 split) and from FP64-18 links, same lattice
    ghl = rhmc.rhmc_gauge_create(lat, U, flags=rhmc.RHMC_LINKS_HILO_12)
    thl, thl_min, _ = time_dslash("fp64", 1, args.dslash_reps, gauge=ghl)
    ghl.close()
    byts_hl = dslash_bytes_per_site("fp64hl", 1) * Vh
    g18 = rhmc.rhmc_gauge_create(lat, U, flags=rhmc.RHMC_LINKS_FP64_18)
    t18, t18_min, byts18 = time_dslash("fp64", 1, args.dslash_reps, gauge=g18)
    g18.close()
    log(f"hopping fp64 hi/lo x1: {thl * 1e6:.1f} us ({byts_hl / thl / 1e9:.0f} GB/s); "
        f"fp64-18 x1: {t18 * 1e6:.1f} us ({byts18 / t18 / 1e9:.0f} GB/s)")
    # FP32 operator from FP32-18 links (no reconstruction)
    gf = rhmc.rhmc_gauge_create(lat, U, flags=rhmc.RHMC_LINKS_FP32_18 | rhmc.RHMC_LINKS_FP64_12)
    tf1, tf1_min, _ = time_dslash("fp32", 1, args.dslash_reps, gauge=gf)
    tf4, tf4_min, _ = time_dslash("fp32", nrhs, args.dslash_reps, gauge=gf)
    gf.close()
    bf1, bf4 = dslash_bytes_per_site("fp32f", 1) * Vh, dslash_bytes_per_site("fp32f", nrhs) * Vh
    log(f"hopping fp32-18 x1: {tf1 * 1e6:.1f} us ({bf1 / tf1 / 1e9:.0f} GB/s); "
        f"x{nrhs}: {tf4 * 1e6:.1f} us ({bf4 / tf4 / 1e9:.0f} GB/s)")

    # 16^3x4 (cache resident: 9.4 MB of FP64 links): 1000 standalone FP64 D_oe
    c2 = synth.CONFIGS[2]
    lat2 = rhmc.rhmc_lattice_create(c2["L"], -1)
    g2 = rhmc.rhmc_gauge_create(lat2, synth.gauge_field(c2["L"], c2["eps"], synth.fields.seed_gauge(2)),
                                flags=rhmc.RHMC_LINKS_FP64_18)
    t2, t2_min, byts2 = time_dslash("fp64", 1, 1000, gauge=g2, vh=lat2.Vh)
    # the same 1000 launches back to back between one pair of events
    v2 = torch.randn((1, 3, lat2.Vh), dtype=torch.complex128, device=dev)
    o2 = torch.empty_like(v2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(1000):
        rhmc.rhmc_dslash_eo(g2, 1, rhmc.RHMC_PREC_FP64, 1, v2, o2)
    e1.record()
    e1.synchronize()
    t2_stream = e0.elapsed_time(e1) / 1e3 / 1000
    g2.close()
    log(f"16^3x4 fp64 x1 (cache resident): {t2 * 1e6:.2f} us per timed launch, "
        f"{t2_stream * 1e6:.2f} us back to back ({byts2 / t2_stream / 1e9:.0f} GB/s)")

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
            "workload": desc,
            "lattice": list(L),
            "nrhs": nrhs,
            "npole": len(rat.beta),
            "mass": m,
            "tol": c["tol"],
            "plaquette": round(plaquette, 6),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel": f"hopping FP32 12-real, {nrhs} rhs, launch variant {var32}, "
                      f"{avg * 1e6:.2f} us per launch (median of {args.dslash_reps}; min "
                      f"{avg_min * 1e6:.2f}), {byts / 1e6:.1f} MB algorithmic per launch",
            "cold_cache": {"us_median": round(avg_cold * 1e6, 2), "us_min": round(avg_cold_min * 1e6, 2),
                           "GBps": round(byts / avg_cold / 1e9, 1),
                           "note": "a 1 GiB buffer read between launches (outside the events)"},
            "gflops": round(FLOPS_PER_SITE * Vh * nrhs / avg / 1e9, 1),
        },
        "dslash": {
            "fp32_12_4rhs": {"us_median": round(avg * 1e6, 2), "us_min": round(avg_min * 1e6, 2),
                             "GBps": round(achieved, 1),
                             "gflops": round(FLOPS_PER_SITE * Vh * nrhs / avg / 1e9, 1)},
            "fp32_12_1rhs": {"us_median": round(avg1 * 1e6, 2), "us_min": round(avg1_min * 1e6, 2),
                             "GBps": round(byts1 / avg1 / 1e9, 1),
                             "gflops": round(FLOPS_PER_SITE * Vh / avg1 / 1e9, 1)},
            "fp64_12_1rhs": {"us_median": round(avg64 * 1e6, 2), "us_min": round(avg64_min * 1e6, 2),
                             "GBps": round(byts64 / avg64 / 1e9, 1),
                             "gflops": round(FLOPS_PER_SITE * Vh / avg64 / 1e9, 1)},
            "fp64_18_1rhs": {"us_median": round(t18 * 1e6, 2), "us_min": round(t18_min * 1e6, 2),
                             "GBps": round(byts18 / t18 / 1e9, 1),
                             "gflops": round(FLOPS_PER_SITE * Vh / t18 / 1e9, 1)},
            "fp32_18_1rhs": {"us_median": round(tf1 * 1e6, 2), "us_min": round(tf1_min * 1e6, 2),
                             "GBps": round(bf1 / tf1 / 1e9, 1),
                             "gflops": round(FLOPS_PER_SITE * Vh / tf1 / 1e9, 1)},
            f"fp32_18_{nrhs}rhs": {"us_median": round(tf4 * 1e6, 2), "us_min": round(tf4_min * 1e6, 2),
                                   "GBps": round(bf4 / tf4 / 1e9, 1),
                                   "gflops": round(FLOPS_PER_SITE * Vh * nrhs / tf4 / 1e9, 1)},
            "fp64_hilo12_1rhs": {"us_median": round(thl * 1e6, 2), "us_min": round(thl_min * 1e6, 2),
                                 "GBps": round(byts_hl / thl / 1e9, 1),
                                 "gflops": round(FLOPS_PER_SITE * Vh / thl / 1e9, 1)},
            "fp64_18_1rhs_16x16x16x4_cache_resident": {
                "us_median": round(t2 * 1e6, 3), "us_min": round(t2_min * 1e6, 3),
                "us_back_to_back": round(t2_stream * 1e6, 3),
                "GBps_back_to_back": round(byts2 / t2_stream / 1e9, 1), "launches": 1000,
                "note": "32 workgroups per launch: launch- and cache-bound"},
        },
        "time_to_solution_s": {
            "mixed_batched": round(t_mixed, 4),
            "fp64": None if t_fp64 is None else round(t_fp64, 4),
            "mixed_batched_runs": [round(v, 4) for v in mixed_times],
            "fp64_runs": [round(v, 4) for v in sorted(fp64_times)],
            "note": "mixed: mean wall time of the timed steps (library time per step listed); "
                    "fp64: median of the listed runs, after one untimed run",
        },
        "time_to_solution_md_tol_s": md,
        "iterations": {"mixed_batched": st["total_iterations"],
                       "fp64": None if st64 is None else st64["total_iterations"]},
        "max_true_residual": {"mixed_batched": st["max_true_residual"],
                              "fp64": None if st64 is None else st64["max_true_residual"]},
        "pseudofermion": pf,
        "md_kernels": md_kernels,
        "md_trajectory_16x16x16x4": trajectories,
        "reliable_updates": st["reliable_updates"],
        "refine_rounds": st["refine_rounds"],
        "refine_iterations": int(st["refine_iterations"].sum()),
        "shifts_refined": int((st["refine_iterations"] > 0).sum()),
        "fp64_head_iterations": st["fp64_head_iterations"],
        "mixed_batched_without_fp64_phase": no_head,
        "rational_apply_two_pass_fp64": two_pass,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(U, b, m, rat, st["total_iterations"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
