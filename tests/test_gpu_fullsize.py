"""Parity at the full sizes of the benchmarked workloads, in the launch configuration the
benchmark times (autotuned execution shape, fused rolling prune):

* the 96,000-atom Ewald box: every force, both energies and the virial against the FP64
  oracle over all N(N-1)/2 minimum-image pairs, at the build and at rolling steps;
* the 1,500,000-atom Ewald box: forces on a seeded sample of atoms against the oracle's
  per-atom sums over all partners, and the list invariants (each cluster pair once,
  inner list inside the outer list) over the whole box."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import (concat, dev, energy_tolerance, keys_of, make_ctx, oracle_forces_multi,
                        oracle_params, rel_rms)
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu


def ctx_for(name, c):
    cfg = systems.CONFIGS[name]
    ctx = make_ctx(c, coulomb="ewald", rc=cfg["rc"], rinner=cfg["rinner"], rlist=cfg["rlist"],
                   beta=cfg["beta"], nstlist=cfg["nstlist"], nstprune=cfg["nstprune"])
    return ctx, cfg


def test_water96k_full_parity_at_build_and_rolling_steps():
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    ctx, cfg = ctx_for("water96k_ewald", c)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    q, lj = dev(c["q"]), dev(c["lj"])
    best, _ = ctx.autotune(x, q, lj, energy=True, repeats=2)
    print("autotuned:", best)
    p = oracle_params("ewald", cfg["rc"], cfg["beta"])
    rng = np.random.default_rng(17)
    xs = c["x"].copy()
    for t in range(0, 6):
        if t > 0:
            xs = (xs + rng.normal(0.0, cfg["sigma_step"], xs.shape)).astype(np.float32)
        f, e, v = ctx.step(dev(xs), q, lj, t, energy=True, virial=True)
        torch.cuda.synchronize()
        if t not in (0, 1, 5):
            continue
        E, F, V, A = oracle_forces_multi(c, xs, p)
        tol = energy_tolerance(E, A, True)
        err_f = rel_rms(f.cpu().numpy(), F)
        en = e.cpu().numpy()
        print("step %d: force rel RMS %.2e, energy rel %s" % (t, err_f, np.abs(en - E) / np.abs(E)))
        assert err_f <= 1e-5
        assert np.all(np.abs(en - E) <= tol)
        assert rel_rms(v.cpu().numpy(), V) <= 1e-5


@pytest.mark.timeout(420)
def test_water1500k_sampled_forces_and_list_invariants():
    s = systems.config_system("water1500k_ewald")
    print("1.5M box generated", flush=True)
    c = concat(s)
    ctx, cfg = ctx_for("water1500k_ewald", c)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    q, lj = dev(c["q"]), dev(c["lj"])
    f, e, _ = ctx.step(x, q, lj, 0, energy=True)
    torch.cuda.synchronize()
    print("1.5M box: list built, forces done", flush=True)
    rng = np.random.default_rng(23)
    sel = np.sort(rng.choice(s.n, size=512, replace=False))
    F = oracle.forces_on(sel, s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box,
                         oracle_params("ewald", cfg["rc"], cfg["beta"]))
    err = rel_rms(f.cpu().numpy()[sel], F)
    print("1.5M box: sampled force rel RMS %.2e over %d atoms" % (err, sel.size))
    assert err <= 1e-5
    assert np.all(np.isfinite(e.cpu().numpy()))
    st = ctx.stats()
    n_cl = st["n_clusters"]
    ko = keys_of(ctx.get_pairs("outer"), n_cl)
    ki = keys_of(ctx.get_pairs("inner"), n_cl)
    assert np.unique(ko).size == ko.size
    assert np.all(np.isin(ki, ko))
    assert st["outer_pairs"] == ko.size and st["inner_pairs"] == ki.size
