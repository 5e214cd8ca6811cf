"""Parity at the full sizes of the benchmarked workloads, in the launch configuration the
benchmark times (autotuned execution shape, fused rolling prune):

* the 96,000-atom Ewald box: every force, both energies and the virial against the FP64
  oracle over all N(N-1)/2 minimum-image pairs, at the build and at rolling steps;
* the 96,000-atom Ewald box backward pass (the one the forward + backward metric times:
  adjoint of a force-matching loss, table gradient on) against the oracle's backward
  pass, in the benchmark's execution shape;
* the 1,500,000-atom Ewald box: the grid slot order against the oracle's grid, every
  force, both energies and the virial against the FP64 oracle at the build and at rolling
  steps around a rebuild, and the list invariants (each cluster pair once, inner list
  inside the outer list) over the whole box."""
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


def test_water96k_queue_and_balanced_modes_match_persistent():
    """The queue mode (balanced runs plus the dynamic tail from ticket pools) and the
    balanced mode at full size, with the ahead prune, over rolling steps: the same inner
    lists as the persistent mode, outputs equal to FP32 summation-order rounding (their
    items differ), the last step within the oracle bars."""
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    q, lj = dev(c["q"]), dev(c["lj"])
    ctxs = {}
    for mode in ("persist", "queue", "balanced"):
        ctx, cfg = ctx_for("water96k_ewald", c)
        ctx.grid_build(dev(c["x"]), c["boxes"])
        ctx.pairlist_build()
        ctx.set_exec(36, mode, "ahead")
        ctxs[mode] = ctx
    rng = np.random.default_rng(23)
    xs = c["x"].copy()
    for t in range(0, 4):
        if t > 0:
            xs = (xs + rng.normal(0.0, cfg["sigma_step"], xs.shape)).astype(np.float32)
        xt = dev(xs)
        out = {m: ctx.step(xt, q, lj, t, energy=True, virial=True) for m, ctx in ctxs.items()}
        torch.cuda.synchronize()
        fa, ea, va = out["persist"]
        inner = ctxs["persist"].get_pairs("inner")
        for m in ("queue", "balanced"):
            fb, eb, vb = out[m]
            assert rel_rms(fb.cpu().numpy(), fa.cpu().numpy()) <= 1e-6, (m, t)
            assert torch.allclose(eb, ea, rtol=1e-9, atol=0), (m, t)
            assert torch.allclose(vb, va, rtol=1e-6, atol=1e-6 * va.abs().max().item()), (m, t)
            assert np.array_equal(ctxs[m].get_pairs("inner"), inner), (m, t)
    E, F, V, A = oracle_forces_multi(c, xs, oracle_params("ewald", cfg["rc"], cfg["beta"]))
    f, e, v = out["queue"]
    assert rel_rms(f.cpu().numpy(), F) <= 1e-5
    assert np.all(np.abs(e.cpu().numpy() - E) <= energy_tolerance(E, A, True))


def symmetrize(gl):
    """Split the derivative w.r.t. each off-diagonal table value evenly over its entries."""
    return 0.5 * (gl + np.transpose(gl, (1, 0, 2)))


@pytest.mark.timeout(420)
def test_water96k_backward_in_benchmark_shape():
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    ctx, cfg = ctx_for("water96k_ewald", c)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    ctx.set_exec(40, "persist", False)
    q, lj = dev(c["q"]), dev(c["lj"])
    p = oracle_params("ewald", cfg["rc"], cfg["beta"])
    rng = np.random.default_rng(31)
    xs = c["x"].copy()
    for t in range(0, 3):
        if t > 0:
            xs = (xs + rng.normal(0.0, cfg["sigma_step"], xs.shape)).astype(np.float32)
        xt = dev(xs)
        f0, _, _ = ctx.step(xt, q, lj, t, energy=False)
        f_ref, _, _ = ctx.forces(xt, q * 1.05, lj * 1.05, energy=False)
        G = (2.0 * (f0 - f_ref)).contiguous()
        gE = None if t == 0 else np.array([[0.7, -0.4]], np.float64)
        gx, gq, gl = ctx.backward(xt, q, lj, G, None if gE is None else dev(gE, torch.float64))
        torch.cuda.synchronize()
        if t == 1:
            continue
        ox, oq, ol = oracle.backward(xs, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p,
                                     G.cpu().numpy().astype(np.float64),
                                     (0.0, 0.0) if gE is None else gE[0])
        errs = [rel_rms(gx.cpu().numpy(), ox), rel_rms(gq.cpu().numpy(), oq),
                rel_rms(gl.cpu().numpy(), symmetrize(ol))]
        print("96k backward step %d: grad x / q / lj rel RMS %s" % (t, errs), flush=True)
        assert max(errs) <= 1e-4, errs


@pytest.mark.timeout(840)
def test_water1500k_every_output_at_build_and_rolling_steps():
    """Every force, both energies and the virial of the 1.5M-atom box against the FP64
    oracle (summed through its cell grid, which equals the all-pairs sum to rounding), in
    the autotuned shape, at the build (step 0), the last step of the first list (79), the
    rebuild (80) and the first rolling step after it (81); Gaussian steps of 0.002 nm
    drawn on the GPU.  Also the grid slot order and the list invariants at the build."""
    s = systems.config_system("water1500k_ewald")
    print("1.5M box generated", flush=True)
    c = concat(s)
    ctx, cfg = ctx_for("water1500k_ewald", c)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    q, lj = dev(c["q"]), dev(c["lj"])
    best, _ = ctx.autotune(x, q, lj, energy=True, repeats=2)
    print("1.5M box: autotuned", best, flush=True)
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    assert np.array_equal(ctx.get_grid(), g["slot_atom"])
    del g
    st = ctx.stats()
    n_cl = st["n_clusters"]
    ko = keys_of(ctx.get_pairs("outer"), n_cl)
    ki = keys_of(ctx.get_pairs("inner"), n_cl)
    assert np.unique(ko).size == ko.size
    assert np.all(np.isin(ki, ko))
    assert st["outer_pairs"] == ko.size and st["inner_pairs"] == ki.size
    del ko, ki
    p = oracle_params("ewald", cfg["rc"], cfg["beta"])
    gen = torch.Generator(device="cuda").manual_seed(cfg["seed"])
    nst = cfg["nstlist"]
    for t in range(0, nst + 2):
        if t > 0:
            x = x + cfg["sigma_step"] * torch.randn(x.shape, generator=gen, device="cuda")
        k = t % nst
        if k == 0 and t > 0:
            ctx.grid_build(x, c["boxes"])
            ctx.pairlist_build()
        f, e, v = ctx.step(x, q, lj, k, energy=True, virial=True)
        if t not in (0, nst - 1, nst, nst + 1):
            continue
        torch.cuda.synchronize()
        xs = x.cpu().numpy()
        E, F, V, A = oracle.forces_cells(xs, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box,
                                         p, energy_abs=True)
        err_f = rel_rms(f.cpu().numpy(), F)
        en = e.cpu().numpy()[0]
        err_e = np.abs(en - E) / np.abs(E)
        err_v = rel_rms(v.cpu().numpy()[0], V)
        print("1.5M step %d: force rel RMS %.2e, E_LJ rel %.2e, E_C rel %.2e, virial rel RMS "
              "%.2e" % (t, err_f, err_e[0], err_e[1], err_v), flush=True)
        assert err_f <= 1e-5
        assert np.all(err_e <= 1e-6)
        assert err_v <= 1e-5
