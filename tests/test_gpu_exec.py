"""Execution shapes of the pair kernel (static, XCD-contiguous, balanced runs with a
dynamic tail from ticket pools, persistent rounds, equal-cost runs per wavefront), item widths, the autotuner, the graph-replayed step and an ensemble of uneven replicas in one
context, through the C ABI on an MI355X, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import (concat, dev, energy_tolerance, keys_of, make_ctx, oracle_forces_multi,
                        oracle_params, rel_rms)
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu

EWALD = dict(coulomb="ewald", rc=1.0, rinner=1.04, rlist=1.1, beta=3.12)


def built(c, **kw):
    ctx = make_ctx(c, **kw)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    return ctx, x


def check_oracle(c, x_np, f, e, coul, rc, beta=0.0, strict=True):
    E, F, _, A = oracle_forces_multi(c, x_np, oracle_params(coul, rc, beta))
    tol = energy_tolerance(E, A, strict)
    assert rel_rms(f.cpu().numpy(), F) <= 1e-5
    e = e.cpu().numpy()
    for s in range(E.shape[0]):
        for k in range(2):
            assert abs(e[s, k] - E[s, k]) <= max(tol[s, k], 1e-9), (s, k, e[s, k], E[s, k])


@pytest.mark.parametrize("width", [8, 32, 64])
def test_modes_bitwise_equal_and_queue_relaunches(sys3k, width):
    """For one item width the modes on the per-super-cluster items give bitwise the same
    forces, energies and virial (each item writes its own partials, whichever wavefront
    computes it).  The queue mode runs on items of its own (balanced runs plus the dynamic
    tail): its launches repeat one another bitwise, which also shows that its ticket pools
    are back at zero after every launch (a pool left behind would skip runs), and it is
    within the oracle bars."""
    c = concat(sys3k)
    ctx, x = built(c, nstlist=10, nstprune=4, **EWALD)
    q, lj = dev(c["q"]), dev(c["lj"])
    ref = None
    qref = None
    for mode in ("static", "xcd", "queue", "queue", "queue", "persist", "persist", "queue",
                 "static"):
        ctx.set_exec(width, mode)
        assert ctx.get_exec() == {"item_width": width, "mode": mode, "prune_fused": True,
                                  "prune_waves": 0}
        out = ctx.forces(x, q, lj, energy=True, virial=True)
        torch.cuda.synchronize()
        if mode == "queue":
            if qref is None:
                qref = [t.clone() for t in out]
                check_oracle(c, c["x"], out[0], out[1], "ewald", 1.0, 3.12)
            else:
                for a, b in zip(qref, out):
                    assert torch.equal(a, b), mode
        elif ref is None:
            ref = [t.clone() for t in out]
            check_oracle(c, c["x"], out[0], out[1], "ewald", 1.0, 3.12)
        else:
            for a, b in zip(ref, out):
                assert torch.equal(a, b), mode
    # rounding only between the two partitions
    assert rel_rms(qref[0].cpu().numpy(), ref[0].cpu().numpy()) <= 1e-6
    assert torch.allclose(qref[1], ref[1], rtol=1e-9, atol=0)


@pytest.mark.parametrize("mode", ["queue", "persist"])
def test_fused_step_in_persistent_modes_matches_static(sys3k, mode):
    """nb_step (prune fused into the pair kernel) under the persistent modes: same inner
    lists as the static mode over a rolling cycle, and bitwise the same outputs (persist,
    same items) or the same to FP32 summation-order rounding (queue, items of its own)."""
    c = concat(sys3k)
    kw = dict(nstlist=20, nstprune=4, **EWALD)
    ctx_a, _ = built(c, **kw)
    ctx_b, _ = built(c, **kw)
    ctx_b.set_exec(0, mode)
    q, lj = dev(c["q"]), dev(c["lj"])
    rng = np.random.default_rng(3)
    x = c["x"].copy()
    for t in range(1, 9):
        x = (x + rng.normal(0, 0.01, x.shape)).astype(np.float32)
        xt = dev(x)
        fa, ea, va = ctx_a.step(xt, q, lj, t, energy=True, virial=True)
        fb, eb, vb = ctx_b.step(xt, q, lj, t, energy=True, virial=True)
        if mode == "persist":
            assert torch.equal(fa, fb) and torch.equal(ea, eb) and torch.equal(va, vb), t
        else:
            torch.cuda.synchronize()
            assert rel_rms(fb.cpu().numpy(), fa.cpu().numpy()) <= 1e-6, t
            assert torch.allclose(eb, ea, rtol=1e-9, atol=0), t
            assert torch.allclose(vb, va, rtol=1e-6, atol=1e-6 * va.abs().max().item()), t
        assert np.array_equal(ctx_a.get_pairs("inner"), ctx_b.get_pairs("inner")), t
    check_oracle(c, x, fb, eb, "ewald", 1.0, 3.12)


@pytest.mark.parametrize("mode", ["xcd", "queue", "persist", "balanced"])
def test_separate_prune_step_equals_fused(sys3k, mode):
    """nb_step with the prune as separate kernels: the same inner lists and bitwise the
    same outputs as with the prune fused into the pair kernel."""
    c = concat(sys3k)
    kw = dict(nstlist=20, nstprune=4, **EWALD)
    ctx_a, _ = built(c, **kw)
    ctx_b, _ = built(c, **kw)
    ctx_a.set_exec(16, mode, prune_fused=True)
    ctx_b.set_exec(16, mode, prune_fused=False)
    q, lj = dev(c["q"]), dev(c["lj"])
    rng = np.random.default_rng(4)
    x = c["x"].copy()
    for t in range(1, 9):
        x = (x + rng.normal(0, 0.01, x.shape)).astype(np.float32)
        xt = dev(x)
        fa, ea, va = ctx_a.step(xt, q, lj, t, energy=True, virial=True)
        fb, eb, vb = ctx_b.step(xt, q, lj, t, energy=True, virial=True, graph=(t % 2 == 0))
        torch.cuda.synchronize()
        assert torch.equal(fa, fb) and torch.equal(ea, eb) and torch.equal(va, vb), t
    assert np.array_equal(ctx_a.get_pairs("inner"), ctx_b.get_pairs("inner"))


@pytest.mark.parametrize("width", [8, 40, 64])
def test_balanced_mode_rolling_cycle(sys3k, width):
    """The balanced mode (equal-cost runs of items per wavefront) over a rolling cycle with
    the prune fused: the same inner lists as the static mode, outputs equal to FP32
    summation-order rounding, and within the oracle bars."""
    c = concat(sys3k)
    kw = dict(nstlist=20, nstprune=4, **EWALD)
    ctx_a, _ = built(c, **kw)
    ctx_b, _ = built(c, **kw)
    ctx_b.set_exec(width, "balanced")
    assert ctx_b.get_exec() == {"item_width": width, "mode": "balanced", "prune_fused": True,
                                "prune_waves": 0}
    st = ctx_b.stats()
    assert st["n_work_items"] >= st["n_superclusters"]
    q, lj = dev(c["q"]), dev(c["lj"])
    rng = np.random.default_rng(13)
    x = c["x"].copy()
    for t in range(0, 7):
        if t > 0:
            x = (x + rng.normal(0, 0.002, x.shape)).astype(np.float32)
        xt = dev(x)
        fa, ea, va = ctx_a.step(xt, q, lj, t, energy=True, virial=True)
        fb, eb, vb = ctx_b.step(xt, q, lj, t, energy=True, virial=True)
        torch.cuda.synchronize()
        assert np.array_equal(ctx_a.get_pairs("inner"), ctx_b.get_pairs("inner")), t
        assert rel_rms(fb.cpu().numpy(), fa.cpu().numpy()) <= 1e-6, t
        assert torch.allclose(eb, ea, rtol=1e-9, atol=0), t
        assert torch.allclose(vb, va, rtol=1e-6, atol=1e-6 * va.abs().max().item()), t
    check_oracle(c, x, fb, eb, "ewald", 1.0, 3.12)


def test_item_width_changes_only_rounding(sys3k):
    """Another item width re-splits the lists: outputs agree with the default to FP32
    summation-order rounding and stay within the oracle bars."""
    c = concat(sys3k)
    ctx, x = built(c, **EWALD)
    q, lj = dev(c["q"]), dev(c["lj"])
    f0, e0, _ = ctx.forces(x, q, lj)
    f0, e0 = f0.clone(), e0.clone()
    for w in (1, 5, 16, 64):
        ctx.set_exec(w, "xcd")
        f, e, _ = ctx.forces(x, q, lj)
        torch.cuda.synchronize()
        assert rel_rms(f.cpu().numpy(), f0.cpu().numpy()) <= 1e-6, w
        assert torch.allclose(e, e0, rtol=1e-9, atol=0), w
        check_oracle(c, c["x"], f, e, "ewald", 1.0, 3.12)
    st = ctx.stats()
    assert st["n_work_items"] >= st["n_superclusters"]


def test_autotune_keeps_fastest_and_stays_exact(sys3k):
    c = concat(sys3k)
    ctx, x = built(c, nstlist=10, nstprune=2, **EWALD)
    q, lj = dev(c["q"]), dev(c["lj"])
    best, trials = ctx.autotune(x, q, lj, energy=True, repeats=3)
    assert len(trials) == 47
    assert trials[40]["mode"] == "persist"          # the one-round width
    n_shape = len(trials) - 6
    assert all(t["us_per_call"] > 0 for t in trials)
    # the step trials: the two fastest shapes, three prune placements each
    by_time = sorted(trials[:n_shape], key=lambda t: t["us_per_call"])
    top = {(by_time[0]["item_width"], by_time[0]["mode"])}
    top.add(next(((t["item_width"], t["mode"]) for t in by_time[1:]
                  if (t["item_width"], t["mode"]) not in top), next(iter(top))))
    assert {(t["item_width"], t["mode"]) for t in trials[n_shape:]} == top
    step = min(trials[n_shape:], key=lambda t: t["us_per_call"])
    assert (best["item_width"], best["mode"], best["prune_fused"]) == \
        (step["item_width"], step["mode"], step["prune_fused"])
    assert ctx.get_exec() == {"item_width": best["item_width"], "mode": best["mode"],
                              "prune_fused": best["prune_fused"], "prune_waves": 0}
    f, e, _ = ctx.forces(x, q, lj)
    torch.cuda.synchronize()
    check_oracle(c, c["x"], f, e, "ewald", 1.0, 3.12)
    # the choice survives the next build
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    assert ctx.get_exec()["item_width"] == best["item_width"]


@pytest.mark.parametrize("mode,fused", [("static", True), ("queue", True), ("persist", True),
                                        ("balanced", True), ("static", False),
                                        ("queue", False), ("persist", False),
                                        ("balanced", False), ("persist", "ahead"),
                                        ("static", "ahead")])
def test_graph_step_replays_match_eager(sys3k, mode, fused):
    """nb_step_graph over two list lifetimes with positions updated in place: every replay
    (with eager work and synchronisation in between) equals the eager nb_step bitwise,
    with the rolling prune fused into the pair kernel, as its own kernel before it, or
    after it for the next step inside the force reduction's launch."""
    c = concat(sys3k)
    kw = dict(nstlist=8, nstprune=4, **EWALD)
    ctx_g, _ = built(c, **kw)
    ctx_e, _ = built(c, **kw)
    ctx_g.set_exec(0, mode, prune_fused=fused)
    ctx_e.set_exec(0, mode, prune_fused=fused)
    q, lj = dev(c["q"]), dev(c["lj"])
    xg = dev(c["x"])                                   # fixed addresses for the graph
    fg = torch.empty_like(xg)
    eg = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    vg = torch.empty((1, 3, 3), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(5)
    x = c["x"].copy()
    for t in range(16):
        k = t % 8
        if t > 0:
            x = (x + rng.normal(0, 0.004, x.shape)).astype(np.float32)
            xg.copy_(dev(x))
        if k == 0:
            for ctx in (ctx_g, ctx_e):
                ctx.grid_build(xg, c["boxes"])
                ctx.pairlist_build()
        ctx_g.step(xg, q, lj, k, energy=True, virial=True, f=fg, e=eg, vir=vg, graph=True)
        torch.cuda.synchronize()
        scratch = torch.randn(1000, device="cuda").sum()        # eager work in between
        fe, ee, ve = ctx_e.step(dev(x), q, lj, k, energy=True, virial=True)
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        assert torch.equal(fg, fe) and torch.equal(eg, ee) and torch.equal(vg, ve), t
    check_oracle(c, x, fg, eg, "ewald", 1.0, 3.12)


def test_ensemble_uneven_replicas_all_modes():
    """Sixteen water-like replicas of 3k-24k atoms (log-uniform sizes) in one context and
    one launch per kernel: per-replica energies and all forces against the oracle, in
    every execution mode."""
    reps = systems.ensemble_systems(n_replicas=16)
    c = concat(reps)
    e_cfg = systems.ENSEMBLE
    ctx, x = built(c, coulomb="rf", rc=e_cfg["rc"], rinner=e_cfg["rinner"],
                   rlist=e_cfg["rlist"], nstlist=e_cfg["nstlist"], nstprune=e_cfg["nstprune"])
    q, lj = dev(c["q"]), dev(c["lj"])
    E, F, _, A = oracle_forces_multi(c, c["x"], oracle_params("rf", e_cfg["rc"]))
    tol = energy_tolerance(E, A, True)
    ref = None
    for mode in ("static", "xcd", "queue", "persist", "balanced"):
        ctx.set_exec(0, mode)
        f, e, _ = ctx.forces(x, q, lj)
        torch.cuda.synchronize()
        if ref is None or mode in ("balanced", "queue"):      # items of their own
            if ref is None:
                ref = (f.clone(), e.clone())
            assert rel_rms(f.cpu().numpy(), F) <= 1e-5
            en = e.cpu().numpy()
            assert np.all(np.abs(en - E) <= tol), np.max(np.abs(en - E) / np.abs(E))
        else:
            assert torch.equal(f, ref[0]) and torch.equal(e, ref[1]), mode


@pytest.mark.parametrize("mode", ["persist", "xcd"])
def test_ahead_prune_step_equals_prune_then_forces(sys3k, mode):
    """The ahead prune (the paper's rolling schedule, Sec. V.E: parts pruned between force
    computations): step s computes forces with the current inner list, then prunes part
    (s + 1) mod nstprune with the step-s positions in the force reduction's launch.  So step s
    equals prune_rolling(x_{s-1}, s) followed by forces(x_s), bitwise, and the inner list
    after step s equals the oracle's with part (s + 1) mod nstprune pruned at x_s."""
    c = concat(sys3k)
    nst, npr = 20, 4
    kw = dict(nstlist=nst, nstprune=npr, **EWALD)
    ctx_a, _ = built(c, **kw)
    ctx_b, _ = built(c, **kw)
    ctx_a.set_exec(16, mode, prune_fused="ahead")
    ctx_b.set_exec(16, mode, prune_fused=False)
    assert ctx_a.get_exec()["prune_fused"] == "ahead"
    q, lj = dev(c["q"]), dev(c["lj"])
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    n_cl = g["slot_atom"].size // 8
    box = c["boxes"][0]
    outer = keys_of(ctx_a.get_pairs("outer"), n_cl)
    rng = np.random.default_rng(17)
    xs = [c["x"].copy()]
    last = {p: 0 for p in range(npr)}              # positions each part was pruned with
    for s in range(0, 9):
        if s > 0:
            xs.append((xs[-1] + rng.normal(0, 0.004, xs[-1].shape)).astype(np.float32))
            ctx_b.prune_rolling(dev(xs[s - 1]), s)
        fa, ea, _ = ctx_a.step(dev(xs[s]), q, lj, s, energy=True)
        fb, eb, _ = ctx_b.forces(dev(xs[s]), q, lj, energy=True)
        torch.cuda.synchronize()
        assert torch.equal(fa, fb) and torch.equal(ea, eb), s
        last[(s + 1) % npr] = s
        inner = np.sort(keys_of(ctx_a.get_pairs("inner"), n_cl))
        ref = []
        for p in range(npr):
            w = oracle.rewrap_with(xs[last[p]], g["k"], box)
            ref.append(oracle.inner_pairs(outer, g["slot_atom"], w, box, EWALD["rinner"], npr, p))
        assert np.array_equal(inner, np.sort(np.concatenate(ref))), s
    cc = dict(c)
    cc["x"] = xs[-1]
    check_oracle(cc, xs[-1], fa, ea, "ewald", 1.0, 3.12)
