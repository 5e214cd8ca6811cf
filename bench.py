#!/usr/bin/env python
"""Benchmark of the cluster-pair nonbonded path on one MI355X.

Default workload: the 96,000-atom water-like box (32,000 three-site molecules, 9.86 nm
cube, seeded jittered lattice), Ewald real space (beta = 3.12/nm, rc = 1.0 nm, potential
shift), outer list rlist = 1.1 nm rebuilt every 100 steps, inner list rinner = 1.04 nm
rolling-pruned in 4 parts, positions given seeded Gaussian displacements of 0.002 nm per
step.  --workload selects the 1.5M-atom box or the ensemble of 256 uneven replicas
instead (one JSON line each).  The whole displacement trajectory is generated on the
GPU before timing, so inputs are resident in HBM when the timed region starts.

One step = list build (grid + outer list + initial prune) when t mod nstlist == 0,
otherwise the rolling prune of one part fused into the force + energy pass (nb_step),
replayed from a HIP graph with positions updated in place (the copy of the step's
positions into the fixed buffer is inside the timed region).  The execution shape of
the pair kernel is chosen by the autotuner at the first list build (untimed).  The JSON
line reports effective pair interactions/s of that step, the eager and separate-call
variants, forward + backward, ns/day-equivalent at 2 fs (the mean step without list
builds plus 1/nstlist of a separately timed rebuild), the force kernel's FP32 roofline
fraction from HIP-event kernel times, and the FP64 oracle timed on the host (all threads
and one thread) with the per-output error of the GPU result at one step.
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
PEAK_FP32 = 157.3e12          # MI355X FP32 vector peak (FLOP/s), counting packed FP32
ARGON_SAMPLE_ATOMS = 131072   # oracle sample of the argon box at n_half = 200 (~6 s)
PEAK_FP32_NONPACKED = 78.6e12 # without packed FP32 (one FMA per lane per cycle)
# Algorithmic FLOP per evaluated pair slot of the force+energy kernels (FMA = 2,
# add/mul = 1, rsqrt/rcp/exp2 = 1, compare/select = 0):
#   common: separation 3, r^2 5, rsqrt 1, r^-2 1, LJ force 5, q_i q_j 1,
#           force accumulation 9                                            (= 25)
#   Ewald:  r 1, u = 1/(1 + (p beta) r) 3, P(u) of degree 7 14, u P 1, exp argument 1,
#           exp2 1, erfc 1, g 3 (= 25), F/r 3, energies 9 (V_C 3, V_LJ 4, 2 sums) => 62
#   RF:     force 5, energies 14 (V_C 4, its constants' residual term 3, V_LJ 4,
#           3 sums)                                                         => 44
FLOP_PER_PAIR = {"ewald": 62, "rf": 44}
# Lennard-Jones alone, forces only (the argon sweep): common 25 (no q_i q_j), F/r 1 => 25
FLOP_PER_PAIR_LJ_FORCE = 25
# Backward pass per evaluated pair slot (same counting, with the table gradient):
#   separation 3, r^2 5, rsqrt 1, r^-2 1, r^-6 and 12 c12 r^-6 3, phi_LJ 3, phi'_LJ/r 6,
#   q_i q_j 1, phi_C 1, G_i - G_j 3, u 5, phi 1, coefficient of d 7, h 9, w 3,
#   i- and j-accumulation 10, table gradient 15                                (= 77)
#   Ewald psi, psi', v: r 1, u = 1/(1 + (p beta) r) 3, P(u) 14, u P 1, exp 2, erfc 1,
#           2 beta/sqrt(pi) e 1, g 2, psi 1, psi' 6, v 2                      (= 34) => 111
#   RF psi, psi', v 8                                                                => 85
FLOP_PER_PAIR_BWD = {"ewald": 111, "rf": 85}

WORKLOADS = {
    "water96k_ewald": "96,000-atom water-like box (32,000 molecules, 9.86 nm cube), Ewald "
                      "real space beta=3.12/nm rc=1.0 nm, rlist=1.1 nm every 100 steps, "
                      "rinner=1.04 nm rolling prune in 4 parts, Gaussian steps 0.002 nm",
    "water1500k_ewald": "1,500,000-atom water-like box (500,000 molecules, 24.7 nm cube), "
                        "Ewald real space beta=2.60/nm rc=1.2 nm, rlist=1.3 nm every 80 "
                        "steps, rinner=1.24 nm rolling prune in 4 parts, Gaussian steps "
                        "0.002 nm",
    "argon157k_sweep": "157,464-atom Lennard-Jones argon box (rho = 26/nm^3, sigma = 0.3345 nm, "
                       "18.2 nm cube), cut-off swept so that 50 ... 3000 particles fall in the "
                       "half cut-off sphere, outer list rc + 0.1 nm, force-only evaluations",
    "water96k_work_efficiency": "96,000-atom water-like box (the water96k_ewald system), "
                                "outer list at 1.45 nm, census of M x N sub-cluster lists "
                                "(M, N in 1, 2, 4, 8) for cut-offs 0.9, 1.0, 1.2 nm and "
                                "buffers 0 ... 0.25 nm",
    "water96k_verlet_buffer": "96,000-atom water-like box (the water96k_ewald system), list "
                              "coverage by 8x8 and 8x4 cluster pairs at 64 radii (r_c + "
                              "0.01 k nm; timed at r_c = 0.9 nm) and the tolerance-based "
                              "Verlet buffer estimate "
                              "(0.005 kJ/mol/ps per atom, 300 K, 2 fs) for the particle and "
                              "cluster lists",
    "ensemble256_rf": "256 independent water-like replicas of 3k-24k atoms (log-uniform, "
                      "2.63M atoms in all, density 100/nm^3) in one context, reaction field "
                      "rc=0.9 nm, rlist=1.0 nm every 100 steps, rinner=0.94 nm rolling prune "
                      "in 4 parts, Gaussian steps 0.002 nm",
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def measured_traffic(workload, exec_cfg):
    """HBM bytes per launch of the plain pair kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when the summary is for another
    workload or execution shape, or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_nb_fwd_%s_counters.txt" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    src = b"".join(open(os.path.join(ROOT, "paper_2006_09167_amd", "csrc", f), "rb").read()
                   for f in ("nb_forces.hip", "nb_internal.h", "nb_erfc_coeffs.h",
                             "nb_pair_common.h"))
    if hashlib.sha256(src).hexdigest()[:16] not in text:
        return None
    shape = "%d entries per item, %s" % (exec_cfg["item_width"],
                                          {"xcd": "XCD-contiguous", "static": "static",
                                           "queue": "balanced runs + dynamic tail",
                                           "persist": "persistent rounds",
                                           "balanced": "equal-cost runs"}[exec_cfg["mode"]])
    for line in text.splitlines():
        if line.strip().startswith("HBM traffic") and shape in line:
            return float(line.split()[-2]) * 1e6
    return None


def load_workload(name):
    """Host arrays and parameters of a workload (seeded synthetic inputs)."""
    import numpy as np
    from paper_2006_09167_amd import systems
    if name == "ensemble256_rf":
        cfg = dict(systems.ENSEMBLE)
        reps = systems.ensemble_systems()
        c = systems.concat_systems(reps)
        c["lj"] = reps[0].lj
        c["parts"] = reps
        c["n_types"] = reps[0].n_types
    else:
        cfg = dict(systems.CONFIGS[name])
        s = systems.config_system(name)
        c = dict(x=s.x, q=s.q, type=s.type, excl_ptr=s.excl_ptr, excl_idx=s.excl_idx,
                 boxes=s.box[None], offsets=np.array([0, s.n], np.int64), lj=s.lj, parts=[s],
                 n_types=s.n_types)
    cfg.setdefault("beta", 0.0)
    return c, cfg


def cpu_baseline(c, cfg, x_np, budget_s=8.0):
    """Time the FP64 oracle on the host cores on a bounded sample of the workload at one
    step's positions.  Returns (seconds, fraction of the step's pair interactions the
    sample covers, description, oracle results for the parity check)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    p = oracle.params(cfg["coulomb"], rc=cfg["rc"], beta=cfg["beta"])
    offs = c["offsets"]
    N = int(offs[-1])
    if len(c["parts"]) > 1:
        # whole replicas in order until the budget is spent
        t0 = time.perf_counter()
        done, atoms, res = 0, 0, []
        for r, s in enumerate(c["parts"]):
            a0, a1 = int(offs[r]), int(offs[r + 1])
            E, F, _ = oracle.forces(x_np[a0:a1], s.q, s.type, s.lj, s.excl_ptr, s.excl_idx,
                                    s.box, p)
            res.append((r, E, F, None))
            done += 1
            atoms += a1 - a0
            if time.perf_counter() - t0 >= budget_s:
                break
        dt = time.perf_counter() - t0
        return dt, atoms / N, ("FP64 brute-force force+energy evaluations of the first %d "
                               "replicas (%d atoms); pairs credited in proportion to atoms"
                               % (done, atoms)), res
    s = c["parts"][0]
    if N <= 200000:
        t0 = time.perf_counter()
        n, first = 0, None
        while True:
            E, F, _ = oracle.forces(x_np, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
            if first is None:
                first = (E, F)
            n += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        dt = (time.perf_counter() - t0) / n
        return dt, 1.0, ("%d FP64 brute-force force+energy evaluations of the box (all "
                         "N(N-1)/2 minimum-image pairs)" % n), [(0, first[0], first[1], None)]
    # large box: the whole box through the oracle's cell grid (every force, the energies
    # and the virial, equal to the all-pairs sum to rounding)
    t0 = time.perf_counter()
    E, F, V = oracle.forces_cells(x_np, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
    dt = time.perf_counter() - t0
    return dt, 1.0, ("one FP64 force+energy+virial evaluation of the whole box through the "
                     "oracle's cell grid"), [(0, E, F, V)]


def cpu_single_thread(c, cfg, x_np, n_sel=1024):
    """The oracle on one host thread: per-atom FP64 sums over all partners for a seeded
    sample of atoms of the first system.  Returns (pair interactions/s, description)."""
    import numpy as np
    import oracle
    p = oracle.params(cfg["coulomb"], rc=cfg["rc"], beta=cfg["beta"])
    s = c["parts"][0]
    n = s.n
    a0 = int(c["offsets"][0])
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(n, size=min(n_sel, n), replace=False))
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.forces_on(sel, x_np[a0:a0 + n], s.q, s.type, s.lj, s.excl_ptr, s.excl_idx,
                         s.box, p)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    return dt, sel.size, n, ("FP64 brute-force forces (all partners) on %d seeded atoms of "
                             "the first box, one thread" % sel.size)


def host_info():
    """Logical CPUs and the CPU model of the host that ran the oracle."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def argon_sweep(args):
    """The paper's kernel-throughput experiment (Fig. 6): LJ argon, force-only evaluations
    of a frozen list for each cut-off of the sweep; raw (computed pair slots) and effective
    (pairs inside the cut-off) pair interactions per second."""
    import numpy as np
    import torch
    from paper_2006_09167_amd import systems
    from paper_2006_09167_amd.api import Context
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = systems.argon_box()
    N = s.n
    x = torch.from_numpy(s.x).to(dev)
    q = torch.zeros(N, dtype=torch.float32, device=dev)
    lj = torch.from_numpy(s.lj).to(dev)
    f = torch.empty((N, 3), dtype=torch.float32, device=dev)
    K = args.steps if args.steps is not None else 50
    W = min(args.warmup, 10)
    points, best = [], None
    for n_half in systems.ARGON["n_half"]:
        rc = systems.argon_cutoff(n_half)
        rlist = rc + systems.ARGON["buffer"]
        ctx = Context(n_types=1, coulomb="none", rc=rc, rinner=rlist, rlist=rlist,
                      atom_offsets=[0, N], device=dev)
        ctx.set_topology(s.type, s.excl_ptr, s.excl_idx)
        ctx.grid_build(x, s.box[None])
        ctx.pairlist_build()
        if args.exec == "auto":
            tuned, _ = ctx.autotune(x, q, lj, energy=False, repeats=3)
        else:
            ctx.set_exec(args.item_width, args.exec)
        ctx.forces(x, q, lj, energy=True, f=f)          # pair counts of this list
        st = ctx.stats()
        for _ in range(W):
            ctx.forces(x, q, lj, energy=False, f=f)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(K):
            ctx.forces(x, q, lj, energy=False, f=f)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / K
        tm = ctx.get_timing()
        ctx.set_timing(False)
        kern = tm["forces"][0] * 1e-3 / max(tm["forces"][1], 1)
        eff, raw = float(st["effective_pairs"]), float(st["computed_pairs"])
        pt = {"n_half": n_half, "rc": round(rc, 4), "rlist": round(rlist, 4),
              "list_entries": int(st["n_entries"]), "exec": ctx.get_exec(),
              "effective_pairs": eff, "raw_pairs": raw, "ms_per_eval": 1e3 * wall,
              "kernel_us": 1e6 * kern, "effective_pairs_per_s": eff / wall,
              "raw_pairs_per_s": raw / wall, "kernel_raw_pairs_per_s": raw / kern,
              "kernel_frac_of_peak": raw * FLOP_PER_PAIR_LJ_FORCE / kern / PEAK_FP32}
        log("n_half %4d rc %.3f: %.3f ms/eval, effective %.3g /s, raw %.3g /s (kernel %.1f us)"
            % (n_half, rc, 1e3 * wall, eff / wall, raw / wall, 1e6 * kern))
        points.append(pt)
        if best is None or pt["effective_pairs_per_s"] > best["effective_pairs_per_s"]:
            best = pt
        del ctx
    result = {
        "metric": "pair interactions/s (effective, LJ argon 157k, best point of the cut-off "
                  "sweep)",
        "value": best["effective_pairs_per_s"],
        "unit": "pair interactions/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": best["ms_per_eval"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]),
                   "atoms": N, "best_n_half": best["n_half"]},
        "sweep": points,
        "roofline": {"bound": "alu", "kernel": "k_nb_fwd<LJ only, forces>",
                     "flop_per_pair": FLOP_PER_PAIR_LJ_FORCE,
                     "achieved": best["kernel_raw_pairs_per_s"] * FLOP_PER_PAIR_LJ_FORCE / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": best["kernel_frac_of_peak"], "traffic": None,
                     "avg_launch_us": best["kernel_us"]},
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        pt = next(p for p in points if p["n_half"] == 200)
        p = oracle.params("rf", rc=pt["rc"])                       # all charges zero
        rng = np.random.default_rng(7)
        sel = np.sort(rng.choice(N, size=ARGON_SAMPLE_ATOMS, replace=False))
        t0 = time.perf_counter()
        F = oracle.forces_on(sel, s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
        dt = time.perf_counter() - t0
        # the sampled atoms' pairs: 2 * n_sample / N of the effective pairs of that cut-off
        result["cpu_baseline"] = {"value": pt["effective_pairs"] * 2.0 * sel.size / N / dt,
                                  "unit": "pair interactions/s", "cores": oracle.num_threads(),
                                  "kind": "oracle",
                                  "sample": "FP64 brute-force forces on %d seeded atoms " % sel.size +
                                            "(all partners) at n_half = 200", "seconds": dt}
        # parity of the GPU forces at that cut-off on the sampled atoms
        ctx = Context(n_types=1, coulomb="none", rc=pt["rc"], rinner=pt["rlist"],
                      rlist=pt["rlist"], atom_offsets=[0, N], device=dev)
        ctx.set_topology(s.type, s.excl_ptr, s.excl_idx)
        ctx.grid_build(x, s.box[None])
        ctx.pairlist_build()
        ctx.forces(x, q, lj, energy=False, f=f)
        fe = f.cpu().numpy()[sel]
        result["parity"] = {"n_half": 200, "sampled_atoms": int(sel.size),
                            "force_rel_rms": float(np.linalg.norm(fe - F) / np.linalg.norm(F))}
        log("oracle %.2f s; parity %s" % (dt, result["parity"]))
    print(json.dumps(result), flush=True)


EFF_CUTOFFS = (0.9, 1.0, 1.2)
EFF_BUFFERS = tuple(round(0.025 * k, 3) for k in range(11))
EFF_SETUPS = ((1, 1), (4, 2), (4, 4), (8, 4), (8, 8))
# list arithmetic of one atom pair slot: 3 coordinate differences, 3 squares, 2 additions
FLOP_PER_SLOT_CENSUS = 8


def work_efficiency_curves(args):
    """The paper's work-efficiency figure (Fig. 5): for three cut-offs and a range of
    buffers, the fraction of the pair evaluations of an M x N list that lie inside the
    cut-off, from one census of an outer list at the largest radius.  The timed quantity is
    the census kernel (8 x 8 pair slots examined per second)."""
    import numpy as np
    import torch
    from paper_2006_09167_amd import _lib, systems
    from paper_2006_09167_amd.api import Context
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = systems.config_system("water96k_ewald")
    N = s.n
    x = torch.from_numpy(s.x).to(dev)
    radii = sorted({round(rc + b, 4) for rc in EFF_CUTOFFS for b in EFF_BUFFERS})
    rlist = max(radii)
    ctx = Context(n_types=s.lj.shape[0], coulomb="rf", rc=1.0, rinner=rlist, rlist=rlist,
                  atom_offsets=[0, N], device=dev)
    ctx.set_topology(s.type, s.excl_ptr, s.excl_idx)
    ctx.grid_build(x, s.box[None])
    ctx.pairlist_build()
    st = ctx.stats()
    K = args.steps if args.steps is not None else 50
    W = min(args.warmup, 10)
    for _ in range(W):
        counts = ctx.list_census(radii)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(K):
        counts = ctx.list_census(radii)
    wall = (time.perf_counter() - t0) / K
    tm = ctx.get_timing()
    ctx.set_timing(False)
    kern = tm["census"][0] * 1e-3 / max(tm["census"][1], 1)
    slots = 64.0 * st["outer_pairs"]
    k_of = {r: i for i, r in enumerate(radii)}
    curves = {}
    for rc in EFF_CUTOFFS:
        kc = k_of[round(rc, 4)]
        cur = {"buffer_nm": list(EFF_BUFFERS)}
        for M, N_ in EFF_SETUPS:
            a, b = _lib.CENSUS_SIZES.index(M), _lib.CENSUS_SIZES.index(N_)
            cur["%dx%d" % (M, N_)] = [
                round(float(counts[0, 0, kc]) / (M * N_ * float(counts[a, b, k_of[round(rc + bb, 4)]])), 4)
                for bb in EFF_BUFFERS]
        curves["rc=%.1f" % rc] = cur
        log("rc %.1f: 1x1 %s | 8x4 %s | 8x8 %s" % (rc, cur["1x1"][::2], cur["8x4"][::2],
                                                   cur["8x8"][::2]))
    # properties that hold at any size: the 8 x 8 count at the list radius is the outer list,
    # counts grow with the radius and shrink with the sub-cluster size
    parity = {"outer_list_equals_8x8": bool(counts[3, 3, -1] == st["outer_pairs"]),
              "monotone_in_radius": bool(np.all(np.diff(counts, axis=2) >= 0)),
              "nested_sizes": bool(np.all(counts[1:] <= counts[:-1]) and
                                   np.all(counts[:, 1:] <= counts[:, :-1]))}
    achieved = slots * FLOP_PER_SLOT_CENSUS / kern
    result = {
        "metric": "census pair slots/s (8x8 cluster-pair slots of the outer list examined "
                  "for the work-efficiency curves)",
        "value": slots / wall, "unit": "pair slots/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": 1e3 * wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]),
                   "atoms": N, "rlist": rlist, "radii": len(radii),
                   "outer_cluster_pairs": int(st["outer_pairs"])},
        "curves": curves,
        "parity": parity,
        "roofline": {"bound": "alu", "kernel": "k_census", "flop_per_slot": FLOP_PER_SLOT_CENSUS,
                     "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": None,
                     "avg_launch_us": 1e6 * kern},
    }
    log("census: %.3f ms per call, kernel %.1f us, %.3g slots/s" % (1e3 * wall, 1e6 * kern,
                                                                    slots / kern))
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        g = oracle.grid_spec.build_grid(s.x, s.box[None], np.array([0, N]))
        n_cl = g["slot_atom"].size // 8
        hi = n_cl // 32                                  # the first 1/32 of the i-clusters
        t0 = time.perf_counter()
        c_or = oracle.census.census(g["slot_atom"], g["w"], s.box, radii, ci_lo=0, ci_hi=hi)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": 64.0 * float(c_or[3, 3, -1]) / dt,
                                  "unit": "pair slots/s", "cores": oracle.num_threads(),
                                  "kind": "oracle",
                                  "sample": "numpy census of the i-clusters 0..%d of %d, all "
                                            "%d radii" % (hi, n_cl, len(radii)),
                                  "seconds": dt}
        log("oracle census sample %.2f s" % dt)
    print(json.dumps(result), flush=True)


BUF_TOL = 0.005          # kJ/mol/ps per atom: the paper's default drift tolerance
BUF_T, BUF_DT = 300.0, 0.002
BUF_RIGID_MASS = 18.015  # a rigid water molecule carries each of its atoms
BUF_FREE_MASS = (15.9994, 1.008)
BUF_OH = 0.1             # nm: a hydrogen rotates about its oxygen at this distance


def verlet_buffer(args):
    """The Verlet buffer estimate (Sec. V.B) with the cluster implicit buffer measured by
    the coverage kernel: the list radius a particle list and the 8x8 / 8x4 cluster lists
    need for the same drift tolerance, at the paper's buffer-comparison setting (r_c 0.9 nm,
    list every 40 steps) and at the dual-list setting of the 96k workload (outer list every
    100 steps, rolling prune in 4 parts).  Timed: the coverage kernel."""
    import numpy as np
    import torch
    from paper_2006_09167_amd import api, systems
    from paper_2006_09167_amd.api import Context
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = systems.config_system("water96k_ewald")
    N = s.n
    x = torch.from_numpy(s.x).to(dev)
    V = float(np.prod(s.box.astype(np.float64)))
    n_o = int(np.sum(s.type == 0))
    rigid = dict(count=[n_o, N - n_o], mass=[BUF_RIGID_MASS] * 2, charge=[-0.82, 0.41],
                 type=[0, 1])
    free = dict(rigid, mass=list(BUF_FREE_MASS))
    rotor = dict(rigid, rot_len=[0.0, BUF_OH], rot_mass=list(BUF_FREE_MASS))
    mass_classes = {"rigid": rigid, "rotor": rotor, "free": free}
    K = args.steps if args.steps is not None else 20
    W = min(args.warmup, 5)
    # (name, r_c, Ewald beta, table step, mass readings, [(list, steps)])
    settings = [("paper_buffer_comparison", 0.9, 3.47, 0.01, ("rotor", "rigid", "free"),
                 [("list", 40), ("list", 10)]),
                ("dual_list_96k", 1.0, 3.12, 0.005, ("rotor", "rigid"),
                 [("outer", 100), ("inner", 4)])]
    out, timing = {}, None
    for name, rc, beta, step, readings, lists in settings:
        radii = (np.float32(rc) + np.float32(step) * np.arange(64, dtype=np.float32)).astype(np.float32)
        ctx = Context(n_types=s.lj.shape[0], coulomb="ewald", rc=rc, beta=beta,
                      rinner=float(radii[-1]), rlist=float(radii[-1]), atom_offsets=[0, N],
                      device=dev)
        ctx.set_topology(s.type, s.excl_ptr, s.excl_idx)
        ctx.grid_build(x, s.box[None])
        ctx.pairlist_build()
        st = ctx.stats()
        if timing is None:
            for _ in range(W):
                ctx.list_coverage(radii, 8, 8)
            ctx.set_timing(True)
            t0 = time.perf_counter()
            for _ in range(K):
                ctx.list_coverage(radii, 8, 8)
            wall = (time.perf_counter() - t0) / K
            tm = ctx.get_timing()
            ctx.set_timing(False)
            kern = tm["census"][0] * 1e-3 / max(tm["census"][1], 1)
            timing = dict(wall=wall, kern=kern, slots=64.0 * st["outer_pairs"],
                          rlist=float(radii[-1]), setting=name)
        cov = {"8x8": ctx.list_coverage(radii, 8, 8), "8x4": ctx.list_coverage(radii, 8, 4)}
        p = api.make_params(int(s.lj.shape[0]), "ewald", rc=rc, beta=beta)
        rc32 = float(np.float32(rc))
        res = {"rc": rc, "ewald_beta": beta, "table": "%d radii, r_c + %.3f k nm" % (64, step)}
        for lname, steps in lists:
            for reading in readings:
                classes = mass_classes[reading]
                r = {}
                for setup, table in [("1x1", None)] + list(cov.items()):
                    kw = {} if table is None else {"coverage": (radii, table)}
                    try:
                        rl, d = api.buffer_estimate(p, classes, s.lj, V, BUF_T, BUF_DT, steps,
                                                    BUF_TOL, max_buffer=float(radii[-1]) - rc32,
                                                    **kw)
                        r[setup] = {"r_list": round(rl, 4), "buffer_nm": round(rl - rc32, 4),
                                    "drift": d}
                    except RuntimeError:                 # not reached inside the table
                        r[setup] = None
                if name == "paper_buffer_comparison" and steps == 40:
                    # the same tolerance for both setups, the one the 8x4 list reaches
                    # with the paper's 0.105 nm (the table radii 0.10 and 0.11 nm)
                    same = {}
                    for b84 in (0.10, 0.11):
                        k = int(round(b84 / step))
                        d84 = api.buffer_drift(p, classes, s.lj, V, BUF_T, BUF_DT, steps,
                                               float(radii[k]),
                                               coverage=(radii, cov["8x4"]))
                        r11, _ = api.buffer_estimate(p, classes, s.lj, V, BUF_T, BUF_DT,
                                                     steps, d84, max_buffer=0.8)
                        same["8x4_%.2f" % b84] = {"drift": d84,
                                                  "1x1_buffer_nm": round(r11 - rc32, 4)}
                    r["1x1_at_the_drift_of_8x4"] = same
                res["%s_steps_%d_%s_masses" % (lname, steps, reading)] = r
                log("%s %s (%d steps, %s masses): %s" % (
                    name, lname, steps, reading,
                    {k: (v["buffer_nm"] if v and "buffer_nm" in v else v)
                     for k, v in r.items()}))
        out[name] = res
        del ctx
    kern = timing["kern"]
    achieved = timing["slots"] * FLOP_PER_SLOT_CENSUS / kern
    result = {
        "metric": "coverage pair slots/s (8x8 cluster-pair slots of the outer list classified "
                  "for the Verlet buffer estimate)",
        "value": timing["slots"] / timing["wall"], "unit": "pair slots/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": 1e3 * timing["wall"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]),
                   "atoms": N, "radii": 64, "tolerance": BUF_TOL, "temperature": BUF_T,
                   "dt_ps": BUF_DT, "timed_list_radius": timing["rlist"],
                   "timed_setting": timing["setting"],
                   "mass_readings": {"rotor": "molecule translates (18.015); H rotates about "
                                              "O at 0.1 nm with its own mass 1.008",
                                     "rigid": "18.015 for every atom (molecule translates)",
                                     "free": "O 15.9994, H 1.008 (free flight)"}},
        "buffers": out,
        "roofline": {"bound": "alu", "kernel": "k_census<0, cover>",
                     "flop_per_slot": FLOP_PER_SLOT_CENSUS, "achieved": achieved / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": None, "avg_launch_us": 1e6 * kern},
    }
    log("coverage: %.3f ms per call, kernel %.1f us" % (1e3 * timing["wall"], 1e6 * kern))
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        g = oracle.grid_spec.build_grid(s.x, s.box[None], np.array([0, N]))
        n_cl = g["slot_atom"].size // 8
        hi = n_cl // 2                                   # half of the i-clusters
        radii = (np.float32(0.9) + np.float32(0.01) * np.arange(64, dtype=np.float32)).astype(np.float32)
        t0 = time.perf_counter()
        c_or = oracle.buffer.coverage(g["slot_atom"], g["w"], s.box, radii, 8, 8, ci_lo=0,
                                      ci_hi=hi)
        dt = time.perf_counter() - t0
        n_trip = oracle.cluster_pairs(g["slot_atom"], g["w"], s.box, float(radii[-1]), 0, hi).size
        result["cpu_baseline"] = {"value": 64.0 * n_trip / dt, "unit": "pair slots/s",
                                  "cores": oracle.num_threads(), "kind": "oracle",
                                  "sample": "numpy coverage (8x8, 64 radii) of the i-clusters "
                                            "0..%d of %d" % (hi, n_cl), "seconds": dt}
        log("oracle coverage sample %.2f s" % dt)
    print(json.dumps(result), flush=True)


def prune_place(code):
    """Where nb_step prunes, from get_exec()['prune_fused'] (True, False or 'ahead')."""
    return {True: "inside the pair kernel", False: "as its own kernel before the pair kernel",
            "ahead": "as its own kernel after the pair kernel, for the next step, beside the "
                     "force reduction"}[code]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: workload's)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="water96k_ewald", choices=sorted(WORKLOADS))
    ap.add_argument("--exec", default="auto",
                    choices=["auto", "static", "xcd", "queue", "persist", "balanced"],
                    help="pair kernel execution shape (auto = autotuner at the first build)")
    ap.add_argument("--item-width", type=int, default=0,
                    help="entries per work item with a fixed --exec mode (0 = built-in rule)")
    ap.add_argument("--prune", default="fused", choices=["fused", "separate", "ahead"],
                    help="rolling prune placement with a fixed --exec mode")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2006_09167_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2006_09167_amd.api import Context, NBError
    if args.workload == "argon157k_sweep":
        argon_sweep(args)
        return
    if args.workload == "water96k_work_efficiency":
        work_efficiency_curves(args)
        return
    if args.workload == "water96k_verlet_buffer":
        verlet_buffer(args)
        return

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log("generating %s" % args.workload)
    c, cfg = load_workload(args.workload)
    N = int(c["offsets"][-1])
    S = len(c["parts"])
    K = args.steps if args.steps is not None else cfg["steps"]
    W = args.warmup
    T = W + K
    nstlist = cfg["nstlist"]
    coul = cfg["coulomb"]

    # Seeded displacement trajectory, resident on the GPU before timing.
    log("trajectory: %d steps of %d atoms" % (T, N))
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg["seed"])
    traj = torch.empty((T, N, 3), dtype=torch.float32, device=dev)
    traj[0] = torch.from_numpy(c["x"]).to(dev)
    for t in range(1, T):
        traj[t] = traj[t - 1] + cfg["sigma_step"] * torch.randn((N, 3), generator=gen, device=dev)
    q = torch.from_numpy(c["q"]).to(dev)
    lj = torch.from_numpy(c["lj"]).to(dev)
    boxes = c["boxes"]
    if args.copy_probe_mb:
        # a plain copy kernel of known size: reads and writes copy_probe_mb MiB once
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = Context(n_types=c["n_types"], coulomb=coul, rc=cfg["rc"], rinner=cfg["rinner"],
                  rlist=cfg["rlist"], beta=cfg["beta"], nstlist=nstlist,
                  nstprune=cfg["nstprune"], atom_offsets=c["offsets"], device=dev)
    ctx.set_topology(c["type"], c["excl_ptr"], c["excl_idx"])
    f = torch.empty((N, 3), dtype=torch.float32, device=dev)
    e = torch.empty((S, 2), dtype=torch.float64, device=dev)
    xbuf = traj[0].clone()                  # positions at a fixed address (graph replays)

    ctx.grid_build(traj[0], boxes)
    ctx.pairlist_build()
    tune = None
    if args.exec == "auto":
        best, trials = ctx.autotune(traj[0], q, lj, energy=True, repeats=5)
        tune = {"best": best, "trials": trials}
        log("autotune: item width %d, mode %s, prune %s"
            % (best["item_width"], best["mode"], {True: "fused", False: "separate",
                                                   "ahead": "ahead"}[best["prune_fused"]]))
    else:
        ctx.set_exec(args.item_width, args.exec,
                     prune_fused={"fused": True, "separate": False, "ahead": "ahead"}[args.prune])

    have_bwd = not args.no_backward
    G = None
    if have_bwd:
        # adjoint of a force-matching loss: G = 2 (F - F_ref), F_ref from parameters x1.05
        f_ref, _, _ = ctx.forces(traj[0], q * 1.05, lj * 1.05, energy=True)
        f0, _, _ = ctx.forces(traj[0], q, lj, energy=True)
        G = (2.0 * (f0 - f_ref)).contiguous()
        del f_ref, f0
        try:
            ctx.backward(traj[0], q, lj, G)
        except NBError as err:
            log("backward unavailable: %s" % err)
            have_bwd = False
        torch.cuda.synchronize()

    def step(t, path="graph", bwd=False):
        # list build every nstlist steps; otherwise the rolling prune of one part, fused
        # into the force pass (nb_step, eager or graph-replayed) or a separate call
        k = t % nstlist
        if path == "graph":
            xbuf.copy_(traj[t])
            xt = xbuf
        else:
            xt = traj[t]
        if k == 0:
            ctx.grid_build(xt, boxes)
            ctx.pairlist_build()
        if path == "separate":
            if k:
                ctx.prune_rolling(xt, k)
            ctx.forces(xt, q, lj, energy=True, f=f, e=e)
        else:
            ctx.step(xt, q, lj, k, energy=True, f=f, e=e, graph=(path == "graph"))
        if bwd:
            ctx.backward(xt, q, lj, G)

    # Statistics pass (untimed, deterministic): pair counts of every step.
    log("statistics pass over %d steps" % T)
    eff = np.zeros(T)
    comp = np.zeros(T)
    inner = np.zeros(T)
    first_stats = None
    for t in range(T):
        step(t, "eager")
        st = ctx.stats()
        eff[t], comp[t], inner[t] = st["effective_pairs"], st["computed_pairs"], st["inner_pairs"]
        if t == 0:
            first_stats = st
    eff_timed, comp_timed = eff[W:].sum(), comp[W:].sum()

    def timed(path, bwd=False, timing=False):
        for t in range(W):
            step(t, path, bwd)
        torch.cuda.synchronize()
        if timing:
            ctx.set_timing(True)
        t0 = time.perf_counter()
        for t in range(W, T):
            step(t, path, bwd)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tm = ctx.get_timing() if timing else None
        if timing:
            ctx.set_timing(False)
        return wall, tm

    log("timed graph-replayed step: %d warmup + %d steps" % (W, K))
    wall_graph, _ = timed("graph")
    log("graph: %.3f ms/step" % (1e3 * wall_graph / K))
    # The same steps launched one by one (positions read where they are: no copy into a
    # fixed buffer, no events); the faster of the two is the step's time.
    wall_plain, _ = timed("eager")
    log("eager step without timing events: %.3f ms/step" % (1e3 * wall_plain / K))
    graph_path = wall_graph <= wall_plain
    wall = wall_graph if graph_path else wall_plain
    wall_eager, tm_eager = timed("eager", timing=True)
    log("eager step: %.3f ms/step" % (1e3 * wall_eager / K))
    wall_sep, tm_sep = timed("separate", timing=True)
    log("separate prune + forces calls: %.3f ms/step" % (1e3 * wall_sep / K))
    wall_fb = tm_fb = None
    if have_bwd:
        log("timed fwd+bwd pass")
        wall_fb, tm_fb = timed("eager", bwd=True, timing=True)

    # The list rebuild (grid, outer list with its initial prune, work items) on its own:
    # the ns/day equivalent adds 1/nstlist of it to the step time without builds.
    torch.cuda.synchronize()
    t_build = []
    for _ in range(3):
        t0 = time.perf_counter()
        ctx.grid_build(traj[W], boxes)
        ctx.pairlist_build()
        torch.cuda.synchronize()
        t_build.append(time.perf_counter() - t0)
    build_s = sorted(t_build)[1]
    n_builds = sum(1 for t in range(W, T) if t % nstlist == 0)
    step_s = max(wall - n_builds * build_s, 0.0) / K
    amortized_s = step_s + build_s / nstlist
    log("list rebuild %.3f ms; step without builds %.4f ms, amortized %.4f ms"
        % (1e3 * build_s, 1e3 * step_s, 1e3 * amortized_s))

    # Roofline of the plain force kernel: the separate-call pass launches only that flavor
    # (the fused pass adds the list-distance test of the pruned part to some launches).
    plain_ms, plain_calls = tm_sep["forces"]
    flop = FLOP_PER_PAIR[coul]
    achieved = comp_timed * flop / (plain_ms * 1e-3)
    fused_ms, fused_calls = tm_eager["forces"]
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
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]),
                   "atoms": N, "systems": S, "nstlist": nstlist, "nstprune": cfg["nstprune"],
                   "list_entries": int(first_stats["n_entries"]),
                   "work_items": int(first_stats["n_work_items"]),
                   "exec": ctx.get_exec()},
        "step_path": ("nb_step_graph (HIP graph replay, positions copied in place" if graph_path
                      else "nb_step launched kernel by kernel (positions read in place")
        + "; rolling prune %s; the faster of graph replay and kernel-by-kernel launch)"
        % prune_place(ctx.get_exec()["prune_fused"]),
        "ms_per_step_graph": 1e3 * wall_graph / K,
        "ms_per_step_launched": 1e3 * wall_plain / K,
        "effective_pairs_per_step": float(eff[W:].mean()),
        "raw_pairs_per_s": comp_timed / wall,
        "ns_per_day_equiv": 0.1728 / amortized_s,
        "ms_list_rebuild": 1e3 * build_s,
        "ms_per_step_amortized": 1e3 * amortized_s,
        "builds_in_timed_steps": n_builds,
        "ms_per_step_eager_with_timing_events": 1e3 * wall_eager / K,
        "ms_per_step_separate_prune_call": 1e3 * wall_sep / K,
        "fwd_bwd_pairs_per_s": (eff_timed / wall_fb) if wall_fb else None,
        "fwd_bwd_raw_pairs_per_s": (comp_timed / wall_fb) if wall_fb else None,
        "fwd_bwd_ms_per_step": (1e3 * wall_fb / K) if wall_fb else None,
        "bwd_over_fwd_kernel": (tm_fb["backward"][0] / max(tm_fb["forces"][0], 1e-9))
        if tm_fb else None,
        "kernel_us": {k: (1e3 * v[0] / v[1] if v[1] else None)
                      for k, v in (tm_fb or tm_eager).items()},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": measured_traffic(args.workload, ctx.get_exec()),
                     "kernel": "k_nb_fwd<%s, energy>" % ("Ewald" if coul == "ewald" else "RF"),
                     "flop_per_pair": flop,
                     "avg_launch_us": 1e3 * plain_ms / max(plain_calls, 1),
                     "step_pass_launch_us": 1e3 * fused_ms / max(fused_calls, 1),
                     "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED},
        "roofline_backward": ({"bound": "alu", "kernel": "k_nb_bwd (with table gradient)",
                               "flop_per_pair": FLOP_PER_PAIR_BWD[coul],
                               "achieved": comp_timed * FLOP_PER_PAIR_BWD[coul]
                               / (tm_fb["backward"][0] * 1e-3) / 1e12,
                               "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                               "frac": comp_timed * FLOP_PER_PAIR_BWD[coul]
                               / (tm_fb["backward"][0] * 1e-3) / PEAK_FP32,
                               "avg_launch_us": 1e3 * tm_fb["backward"][0]
                               / max(tm_fb["backward"][1], 1)} if tm_fb else None),
        "work_efficiency": float(eff[W:].sum() / max(comp[W:].sum(), 1)),
        "list": {"outer_cluster_pairs": int(first_stats["outer_pairs"]),
                 "bb_cluster_pairs": int(first_stats["bb_pairs"]),
                 "mean_inner_cluster_pairs": float(inner[W:].mean())},
    }
    if tune:
        result["autotune"] = tune

    if not args.no_cpu_baseline:
        tb = W  # a timed-range step: recompute the GPU result with that step's list state
        log("cpu baseline: FP64 oracle on a bounded sample at step %d" % tb)
        for t in range(tb + 1):
            step(t, "eager")
        torch.cuda.synchronize()
        x_np = traj[tb].cpu().numpy()
        fe = f.cpu().numpy()
        ee = e.cpu().numpy()
        # the virial of that step too, for the per-output errors
        xv = traj[tb].clone()
        _, _, vv = ctx.forces(xv, q, lj, energy=True, virial=True)
        vv = vv.cpu().numpy()
        dt, frac, sample, res = cpu_baseline(c, cfg, x_np)
        par = {"step": tb}
        if S > 1:
            offs = c["offsets"]
            num = den = 0.0
            worst = 0.0
            for r, E, F, _ in res:
                a0, a1 = int(offs[r]), int(offs[r + 1])
                num += float(np.sum((fe[a0:a1] - F) ** 2))
                den += float(np.sum(F ** 2))
                worst = max(worst, float(np.max(np.abs(ee[r] - E) / np.abs(E))))
            par.update(force_rel_rms=math.sqrt(num / den), energy_rel_max=worst,
                       replicas=len(res))
        else:
            _, E, F, V = res[0]
            par.update(force_rel_rms=float(np.linalg.norm(fe - F) / np.linalg.norm(F)),
                       energy_rel=[float(abs(ee[0, k] - E[k]) / abs(E[k])) for k in range(2)])
            if V is not None:
                par["virial_rel_rms"] = float(np.linalg.norm(vv[0] - V) / np.linalg.norm(V))
        import oracle
        dt1, n1, n_box, sample1 = cpu_single_thread(c, cfg, x_np)
        # the sampled atoms' pairs are 2 n1 / n_box of the first box's pairs
        eff_box = float(eff[tb]) * n_box / N
        result["cpu_baseline"] = {"value": float(eff[tb]) * frac / dt,
                                  "unit": "pair interactions/s",
                                  "cores": oracle.num_threads(), "kind": "oracle",
                                  "sample": sample + " at step %d" % tb,
                                  "seconds": dt,
                                  "value_one_thread": eff_box * 2.0 * n1 / n_box / dt1,
                                  "sample_one_thread": sample1, "seconds_one_thread": dt1,
                                  "host": host_info()}
        result["parity_at_step"] = par
        log("oracle %.2f s (one thread: %.2f s); parity %s" % (dt, dt1, par))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
