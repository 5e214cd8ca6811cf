#!/usr/bin/env python
"""Benchmark of the cluster-pair nonbonded path on one MI355X.

Workload: the 96,000-atom water-like box (32,000 three-site molecules, 9.86 nm cube,
seeded jittered lattice), Ewald real space (beta = 3.12/nm, rc = 1.0 nm, potential
shift), outer list rlist = 1.1 nm rebuilt every 100 steps, inner list rinner = 1.04 nm
rolling-pruned in 4 parts, positions given seeded Gaussian displacements of 0.002 nm per
step.  The whole displacement trajectory is generated on the GPU before timing, so inputs
are resident in HBM when the timed region starts.

One step = list build (grid + outer list + initial prune) when t mod 100 == 0, otherwise
one rolling prune; then the force + energy evaluation (and, for the fwd+bwd leg, the
backward pass of a force-matching loss).  The JSON line reports effective pair
interactions/s (pairs inside the cut-off) of the forward step, the fwd+bwd rate, the raw
rate, ns/day-equivalent at 2 fs, the force kernel's FP32 roofline fraction from HIP-event
kernel times, and the FP64 oracle timed on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair interactions/s & % FP32 VALU peak, fwd vs fwd+bwd, 96k-atom box"
CONFIG = "water96k_ewald"
PEAK_FP32 = 157.3e12          # MI355X FP32 vector peak (FLOP/s), counting packed FP32
PEAK_FP32_NONPACKED = 78.6e12 # without packed FP32 (one FMA per lane per cycle)
# Algorithmic FLOP per evaluated pair slot of the Ewald force+energy kernel (FMA = 2,
# add/mul = 1, rsqrt/rcp/exp2 = 1, compare/select = 0):
#   separation 3, r^2 5, rsqrt 1, r^-2 1, LJ force 5, q_i q_j 1,
#   Ewald: r 1, beta r 1, u = 1/(1 + p t) 3, P(u) 16, u P 1, exp argument 1, exp2 1,
#          erfc 1, g 3 (= 29), F/r 3, force accumulation 9, energies 9     => 66
FLOP_PER_PAIR_EWALD_E = 66
# Backward pass per evaluated pair slot (same counting), documented in the design doc.
FLOP_PER_PAIR_EWALD_BWD = 148


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(s, xs, cfg, budget_s=8.0):
    """Time the FP64 oracle (full brute-force evaluations of the box at consecutive steps'
    positions, until about budget_s seconds have passed) on the host cores.  Returns the
    seconds per evaluation, the first evaluation's energies and forces, the thread count
    and the number of evaluations."""
    import oracle
    oracle.build(force=False)
    p = oracle.params("ewald", rc=cfg["rc"], beta=cfg["beta"])
    t0 = time.perf_counter()
    first = None
    n = 0
    for x_np in xs:
        E, F, _ = oracle.forces(x_np, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
        if first is None:
            first = (E, F)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = (time.perf_counter() - t0) / n
    return dt, first[0], first[1], oracle.num_threads(), n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2006_09167_amd import _lib, systems
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2006_09167_amd.api import Context, NBError

    cfg = systems.CONFIGS[CONFIG]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log("generating %s" % CONFIG)
    s = systems.config_system(CONFIG)
    N = s.n
    K, W = args.steps, args.warmup
    T = W + K
    nstlist = cfg["nstlist"]

    # Seeded displacement trajectory, resident on the GPU before timing.
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg["seed"])
    traj = torch.empty((T, N, 3), dtype=torch.float32, device=dev)
    traj[0] = torch.from_numpy(s.x).to(dev)
    for t in range(1, T):
        traj[t] = traj[t - 1] + cfg["sigma_step"] * torch.randn((N, 3), generator=gen, device=dev)
    q = torch.from_numpy(s.q).to(dev)
    lj = torch.from_numpy(s.lj).to(dev)
    box = s.box
    if args.copy_probe_mb:
        # a plain copy kernel of known size: reads and writes copy_probe_mb MiB once
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = Context(n_types=s.n_types, coulomb="ewald", rc=cfg["rc"], rinner=cfg["rinner"],
                  rlist=cfg["rlist"], beta=cfg["beta"], nstlist=nstlist,
                  nstprune=cfg["nstprune"], atom_offsets=[0, N], device=dev)
    ctx.set_topology(s.type, s.excl_ptr, s.excl_idx)
    f = torch.empty((N, 3), dtype=torch.float32, device=dev)
    e = torch.empty((1, 2), dtype=torch.float64, device=dev)

    have_bwd = not args.no_backward
    G = None
    if have_bwd:
        # adjoint of a force-matching loss: G = 2 (F - F_ref), F_ref from parameters x1.05
        ctx.grid_build(traj[0], box)
        ctx.pairlist_build()
        f_ref, _, _ = ctx.forces(traj[0], q * 1.05, lj * 1.05, energy=True)
        f0, _, _ = ctx.forces(traj[0], q, lj, energy=True)
        G = (2.0 * (f0 - f_ref)).contiguous()
        try:
            ctx.backward(traj[0], q, lj, G)
        except NBError as err:
            log("backward unavailable: %s" % err)
            have_bwd = False
        torch.cuda.synchronize()

    def step(t, bwd=False, fused=True):
        # list build every nstlist steps; otherwise the rolling prune of one part, fused
        # into the force pass (nb_step) or as a separate call before nb_forces
        k = t % nstlist
        xt = traj[t]
        if k == 0:
            ctx.grid_build(xt, box)
            ctx.pairlist_build()
        if fused:
            ctx.step(xt, q, lj, k, energy=True, f=f, e=e)
        else:
            if k:
                ctx.prune_rolling(xt, k)
            ctx.forces(xt, q, lj, energy=True, f=f, e=e)
        if bwd:
            ctx.backward(xt, q, lj, G)

    # Statistics pass (untimed, deterministic): pair counts of every step.
    log("statistics pass over %d steps" % T)
    eff = np.zeros(T)
    comp = np.zeros(T)
    inner = np.zeros(T)
    n_entries = n_items = 0
    for t in range(T):
        step(t)
        st = ctx.stats()
        eff[t], comp[t], inner[t] = st["effective_pairs"], st["computed_pairs"], st["inner_pairs"]
        if t == 0:
            n_entries, n_items = st["n_entries"], st["n_work_items"]
            first_stats = st
    eff_timed, comp_timed = eff[W:].sum(), comp[W:].sum()

    def timed(bwd, fused=True):
        for t in range(W):
            step(t, bwd, fused)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for t in range(W, T):
            step(t, bwd, fused)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tm = ctx.get_timing()
        ctx.set_timing(False)
        return wall, tm

    log("timed forward pass: %d warmup + %d steps" % (W, K))
    wall, tm = timed(False)
    fwd_ms, fwd_calls = tm["forces"]
    log("forward: %.3f ms/step, force kernel %.1f us/launch" % (1e3 * wall / K, 1e3 * fwd_ms / max(fwd_calls, 1)))
    wall_sep, tm_sep = timed(False, fused=False)
    log("separate prune + forces calls: %.3f ms/step" % (1e3 * wall_sep / K))
    wall_fb = None
    tm_fb = None
    if have_bwd:
        log("timed fwd+bwd pass")
        wall_fb, tm_fb = timed(True)

    # Roofline of the plain force kernel: the separate-call pass launches only that flavor
    # (the fused pass adds the list-distance test of the pruned part to some launches).
    plain_ms, plain_calls = tm_sep["forces"]
    achieved = comp_timed * FLOP_PER_PAIR_EWALD_E / (plain_ms * 1e-3)
    # force + energy at one step for the CPU comparison
    result = {
        "metric": METRIC,
        "value": eff_timed / wall,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "water96k_ewald: 96,000-atom water-like box (32,000 molecules, "
                               "9.86 nm cube), Ewald real space beta=3.12/nm rc=1.0 nm, "
                               "rlist=1.1 nm every 100 steps, rinner=1.04 nm rolling prune "
                               "in 4 parts, Gaussian steps 0.002 nm",
                   "atoms": N, "nstlist": nstlist, "nstprune": cfg["nstprune"],
                   "list_entries": int(n_entries), "work_items": int(n_items)},
        "effective_pairs_per_step": float(eff[W:].mean()),
        "raw_pairs_per_s": comp_timed / wall,
        "ns_per_day_equiv": 0.1728 / (wall / K),
        "ms_per_step_separate_prune_call": 1e3 * wall_sep / K,
        "fwd_bwd_pairs_per_s": (eff_timed / wall_fb) if wall_fb else None,
        "fwd_bwd_ms_per_step": (1e3 * wall_fb / K) if wall_fb else None,
        "bwd_over_fwd_kernel": (tm_fb["backward"][0] / max(tm_fb["forces"][0], 1e-9))
        if tm_fb else None,
        "kernel_us": {k: (1e3 * v[0] / v[1] if v[1] else None)
                      for k, v in (tm_fb or tm).items()},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": None,
                     "kernel": "k_nb_fwd<Ewald, energy>",
                     "flop_per_pair": FLOP_PER_PAIR_EWALD_E,
                     "avg_launch_us": 1e3 * plain_ms / max(plain_calls, 1),
                     "fused_prune_launch_us": 1e3 * fwd_ms / max(fwd_calls, 1),
                     "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED},
        "work_efficiency": float(eff[W:].sum() / max(comp[W:].sum(), 1)),
        "list": {"outer_cluster_pairs": int(first_stats["outer_pairs"]),
                 "bb_cluster_pairs": int(first_stats["bb_pairs"]),
                 "mean_inner_cluster_pairs": float(inner[W:].mean())},
    }

    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle, one full evaluation of the box")
        tb = W  # a timed-range step
        # recompute the GPU result at step tb for the comparison (list state of that step)
        for t in range(tb + 1):
            step(t)
        torch.cuda.synchronize()
        xs = (traj[t].cpu().numpy() for t in range(tb, T))
        fe = f.cpu().numpy()
        ee = e.cpu().numpy()[0]
        dt, E, F, cores, n_eval = cpu_baseline(s, xs, cfg)
        err_f = float(np.linalg.norm(fe - F) / np.linalg.norm(F))
        err_e = [float(abs(ee[k] - E[k]) / abs(E[k])) for k in range(2)]
        result["cpu_baseline"] = {"value": float(eff[tb:tb + n_eval].mean()) / dt,
                                  "unit": "pair interactions/s",
                                  "cores": cores, "kind": "oracle",
                                  "sample": "%d FP64 brute-force force+energy evaluations of the "
                                            "96k box (all N(N-1)/2 minimum-image pairs) at steps "
                                            "%d.." % (n_eval, tb),
                                  "seconds_per_eval": dt}
        result["parity_at_step"] = {"step": tb, "force_rel_rms": err_f, "energy_rel": err_e}
        log("oracle %.2f s; GPU force rel RMS %.2e energy rel %s" % (dt, err_f, err_e))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
