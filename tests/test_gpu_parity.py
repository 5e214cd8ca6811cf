"""Parity of the HIP path with the FP64 oracle (run on an MI355X through the C ABI).

Bars: grid slot order and pair-list sets bit-exact (as sets, each cluster pair once);
forces within 1e-5 relative RMS and each energy within 1e-6 relative of the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from conftest import small_random_system
from gpu_common import (concat, dev, energy_tolerance, keys_of, make_ctx, oracle_forces_multi,
                        oracle_pair_keys, oracle_params, rel_rms, term_scale)
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
E_TOL = 1e-6


def build(c, **kw):
    ctx = make_ctx(c, **kw)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    return ctx, x


def check_grid(ctx, c):
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    got = ctx.get_grid()
    assert np.array_equal(ctx.get_grid_dims(), np.array(g["dims"], dtype=np.int32))
    assert got.size == g["slot_atom"].size
    assert np.array_equal(got, g["slot_atom"])
    return g


def check_lists(ctx, c, g, rlist, rinner):
    n_cl = g["slot_atom"].size // 8
    outer = ctx.get_pairs("outer")
    inner = ctx.get_pairs("inner")
    ko, ki = keys_of(outer, n_cl), keys_of(inner, n_cl)
    assert np.unique(ko).size == ko.size                    # each cluster pair exactly once
    ref_o = oracle_pair_keys(c, g, rlist)
    assert np.array_equal(np.sort(ko), ref_o)
    ref_i = np.intersect1d(ref_o, oracle_pair_keys(c, g, rinner))
    assert np.array_equal(np.sort(ki), ref_i)
    return ko, ki


def check_forces(ctx, c, x, coul, rc, beta=0.0, modifier="potshift", virial=True, eps_rf=math.inf,
                 strict=True, term_ulps=None):
    q = dev(c["q"])
    lj = dev(c["lj"])
    f, e, v = ctx.forces(x, q, lj, energy=True, virial=virial)
    torch.cuda.synchronize()
    E, F, V, A = oracle_forces_multi(c, c["x"], oracle_params(coul, rc, beta, modifier, eps_rf))
    tol = energy_tolerance(E, A, strict)
    if term_ulps is not None:          # (LJ, Coulomb) worst-case units of 2^-24 per term
        p = oracle_params(coul, rc, beta, modifier, eps_rf)
        tol = np.maximum(tol, np.asarray(term_ulps) * 2.0 ** -24 * term_scale(c, p))
    f = f.cpu().numpy()
    e = e.cpu().numpy()
    assert np.all(np.isfinite(f))
    err_f = rel_rms(f, F)
    assert err_f <= F_TOL, err_f
    for s in range(E.shape[0]):
        for k in range(2):
            if abs(E[s, k]) > 0:
                assert abs(e[s, k] - E[s, k]) <= tol[s, k], (s, k, e[s, k], E[s, k], A[s, k])
            else:
                assert abs(e[s, k]) < 1e-9
    if virial:
        v = v.cpu().numpy()
        assert rel_rms(v, V) <= 1e-5
    return f, e


# ---- grid and lists ------------------------------------------------------------------------
def test_water3k_rf_grid_lists_forces(sys3k):
    c = concat(sys3k)
    ctx, x = build(c, coulomb="rf", rc=1.0, rinner=1.0, rlist=1.0)
    g = check_grid(ctx, c)
    check_lists(ctx, c, g, 1.0, 1.0)
    check_forces(ctx, c, x, "rf", 1.0)


def test_water3k_ewald_buffered_lists_and_forces(sys3k):
    c = concat(sys3k)
    ctx, x = build(c, coulomb="ewald", rc=1.0, rinner=1.04, rlist=1.1, beta=3.12, nstlist=10,
                   nstprune=4)
    g = check_grid(ctx, c)
    check_lists(ctx, c, g, 1.1, 1.04)
    check_forces(ctx, c, x, "ewald", 1.0, 3.12)
    st = ctx.stats()
    assert st["outer_pairs"] >= st["inner_pairs"] > 0
    assert st["effective_pairs"] > 0


@pytest.mark.parametrize("seed,n,box,rl", [(1, 150, 2.4, 1.1), (2, 7, 2.3, 1.1), (3, 65, 2.25, 1.1),
                                           (4, 300, [2.3, 3.1, 2.6], 1.0), (5, 1, 2.5, 1.0),
                                           (6, 2, 2.5, 1.0), (7, 513, 3.0, 1.2)])
def test_small_random_systems(seed, n, box, rl):
    s = small_random_system(seed, n, box, n_types=3, min_dist=0.15)
    c = concat(s)
    ctx, x = build(c, coulomb="ewald", rc=0.9, rinner=min(rl, 0.95), rlist=rl, beta=3.5,
                   modifier="none", nstlist=5, nstprune=2)
    g = check_grid(ctx, c)
    check_lists(ctx, c, g, rl, min(rl, 0.95))
    check_forces(ctx, c, x, "ewald", 0.9, 3.5, modifier="none", strict=False)


def test_ensemble_with_empty_and_tiny_systems():
    reps = [small_random_system(11, 200, 2.5), small_random_system(12, 0 + 1, 2.4),
            small_random_system(13, 90, 2.3), small_random_system(14, 333, 3.2)]
    reps.insert(2, systems.System(**{**reps[1].__dict__, "x": np.zeros((0, 3), np.float32),
                                     "q": np.zeros(0, np.float32), "type": np.zeros(0, np.int32),
                                     "excl_ptr": np.zeros(1, np.int64),
                                     "excl_idx": np.zeros(0, np.int32)}))
    c = concat(reps)
    ctx, x = build(c, coulomb="rf", rc=1.0, rinner=1.05, rlist=1.1, nstlist=4, nstprune=2)
    g = check_grid(ctx, c)
    check_lists(ctx, c, g, 1.1, 1.05)
    check_forces(ctx, c, x, "rf", 1.0, strict=False)


@pytest.mark.parametrize("prune_waves", [0, 1, 2, 4, 8])
def test_rolling_prune_matches_oracle(sys3k, prune_waves):
    """Dual list: inner masks of part (t mod nstprune) are re-derived from the outer list
    with the step-t coordinates, by the prune kernel with each number of wavefronts per
    item; forces then follow the current inner list."""
    c = concat(sys3k)
    nst, npr = 20, 4
    ctx, x = build(c, coulomb="ewald", rc=1.0, rinner=1.04, rlist=1.1, beta=3.12, nstlist=nst,
                   nstprune=npr)
    ctx.set_exec(0, "static", True, prune_waves)
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    n_cl = g["slot_atom"].size // 8
    outer = keys_of(ctx.get_pairs("outer"), n_cl)
    rng = np.random.default_rng(7)
    xs = [c["x"].copy()]
    last = {p: 0 for p in range(npr)}
    for t in range(1, 7):
        xs.append((xs[-1] + rng.normal(0, 0.01, xs[-1].shape)).astype(np.float32))
        xt = dev(xs[t])
        ctx.prune_rolling(xt, t)
        last[t % npr] = t
        inner = np.sort(keys_of(ctx.get_pairs("inner"), n_cl))
        ref = []
        for p in range(npr):
            w = oracle.rewrap_with(xs[last[p]], g["k"], c["boxes"][0])
            ref.append(oracle.inner_pairs(outer, g["slot_atom"], w, c["boxes"][0], 1.04, npr, p))
        assert np.array_equal(inner, np.sort(np.concatenate(ref))), t
    cc = dict(c)
    cc["x"] = xs[-1]
    check_forces(ctx, cc, dev(xs[-1]), "ewald", 1.0, 3.12)
    with pytest.raises(Exception):
        ctx.prune_rolling(dev(xs[-1]), nst)          # the outer list has expired


def test_forces_are_deterministic(sys3k):
    c = concat(sys3k)
    ctx, x = build(c, coulomb="ewald", rc=1.0, rinner=1.04, rlist=1.1, beta=3.12)
    q, lj = dev(c["q"]), dev(c["lj"])
    f1, e1, _ = ctx.forces(x, q, lj)
    f2, e2, _ = ctx.forces(x, q, lj)
    assert torch.equal(f1, f2) and torch.equal(e1, e2)
    # accumulate flag adds into the outputs
    f3, e3, _ = ctx.forces(x, q, lj, f=f1.clone(), e=e1.clone(), accumulate=True)
    assert torch.allclose(f3, 2 * f1) and torch.allclose(e3, 2 * e1)


def test_capacity_hint_overflow_reports_error(sys3k):
    from paper_2006_09167_amd.api import NBError
    c = concat(sys3k)
    ctx = make_ctx(c, coulomb="rf", rc=1.0, rlist=1.0, capacity_hint=4)
    ctx.grid_build(dev(c["x"]), c["boxes"])
    with pytest.raises(NBError) as ei:
        ctx.pairlist_build()
    assert ei.value.status == 4
    # the default context grows its capacity instead
    ctx2 = make_ctx(c, coulomb="rf", rc=1.0, rlist=1.0)
    ctx2.grid_build(dev(c["x"]), c["boxes"])
    ctx2.pairlist_build()


def test_nonfinite_coordinates_reported(sys3k):
    from paper_2006_09167_amd.api import NBError
    c = concat(sys3k)
    x = c["x"].copy()
    x[17, 1] = np.nan
    ctx = make_ctx(c, coulomb="rf", rc=1.0, rlist=1.0)
    ctx.grid_build(dev(x), c["boxes"])
    with pytest.raises(NBError) as ei:
        ctx.pairlist_build()
    assert ei.value.status == 7


def test_bad_box_rejected(sys3k):
    from paper_2006_09167_amd.api import NBError
    c = concat(sys3k)
    ctx = make_ctx(c, coulomb="rf", rc=1.0, rlist=1.6)
    with pytest.raises(NBError) as ei:
        ctx.grid_build(dev(c["x"]), c["boxes"])       # 3.104 < 2 * 1.6
    assert ei.value.status == 2


def test_fused_step_equals_prune_then_forces(sys3k):
    """nb_step (rolling prune inside the pair kernel) gives the same inner list and bitwise
    the same forces and energies as nb_prune_rolling followed by nb_forces."""
    c = concat(sys3k)
    kw = dict(coulomb="ewald", rc=1.0, rinner=1.04, rlist=1.1, beta=3.12, nstlist=20,
              nstprune=4)
    ctx_a, _ = build(c, **kw)
    ctx_b, _ = build(c, **kw)
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    n_cl = g["slot_atom"].size // 8
    q, lj = dev(c["q"]), dev(c["lj"])
    rng = np.random.default_rng(11)
    x = c["x"].copy()
    for t in range(1, 9):
        x = (x + rng.normal(0, 0.01, x.shape)).astype(np.float32)
        xt = dev(x)
        ctx_a.prune_rolling(xt, t)
        fa, ea, va = ctx_a.forces(xt, q, lj, energy=True, virial=True)
        fb, eb, vb = ctx_b.step(xt, q, lj, t, energy=True, virial=True)
        ia = np.sort(keys_of(ctx_a.get_pairs("inner"), n_cl))
        ib = np.sort(keys_of(ctx_b.get_pairs("inner"), n_cl))
        assert np.array_equal(ia, ib), t
        assert torch.equal(fa, fb) and torch.equal(ea, eb) and torch.equal(va, vb), t
    fb, eb, _ = ctx_b.step(xt, q, lj, 0)
    fa, ea, _ = ctx_a.forces(xt, q, lj)
    assert torch.equal(fa, fb)
