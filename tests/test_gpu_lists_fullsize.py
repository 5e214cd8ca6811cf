"""The pair lists of the 96,000-atom box (the benchmarked workload) bit-exact against the
oracle's cluster-pair sets, as sets, each cluster pair once:

* at the build: the bounding-box candidates contain the outer list (Sec. V.D), the outer
  list equals the oracle's S_outer and the inner list its S_inner;
* at rolling steps 1-4 (Sec. V.E: one part per step, pruned with that step's positions),
  in five execution shapes: the prune as its own kernel with one, two, four and eight
  wavefronts per item and with the automatic choice, and the prune fused into the pair
  kernel;
* with the ahead prune (part (t + 1) mod nstprune pruned with the positions of step t,
  in the force reduction's launch) in its two unit layouts: the pair kernel's items,
  several per block at 36 entries per item (more items than blocks that fit beside the
  reduction), and whole super-cluster lists at 8 entries per item (many more items)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import concat, dev, keys_of, make_ctx
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu

# (entries per item, mode, prune fused, prune wavefronts per item)
SHAPES = [(8, "static", False, 1), (40, "persist", False, 0), (40, "xcd", False, 2),
          (16, "static", False, 4), (24, "persist", False, 8), (40, "persist", True, 0),
          (36, "persist", "ahead", 0), (8, "persist", "ahead", 0)]


@pytest.mark.timeout(600)
def test_water96k_lists_at_build_and_rolling_steps():
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    cfg = systems.CONFIGS["water96k_ewald"]
    rl, ri, npr = cfg["rlist"], cfg["rinner"], cfg["nstprune"]
    box = c["boxes"][0]
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    n_cl = g["slot_atom"].size // 8
    ctxs = []
    for w, mode, fused, pw in SHAPES:
        ctx = make_ctx(c, coulomb="ewald", rc=cfg["rc"], rinner=ri, rlist=rl, beta=cfg["beta"],
                       nstlist=cfg["nstlist"], nstprune=npr)
        ctx.grid_build(dev(c["x"]), c["boxes"])
        ctx.pairlist_build()
        ctx.set_exec(w, mode, fused, pw)
        assert ctx.get_exec()["prune_waves"] == pw
        ctxs.append(ctx)
    assert np.array_equal(ctxs[0].get_grid(), g["slot_atom"])
    st0 = ctxs[0].stats()
    ref_o = oracle.cluster_pairs(g["slot_atom"], g["w"], box, rl)
    ref_i0 = np.intersect1d(ref_o, oracle.cluster_pairs(g["slot_atom"], g["w"], box, ri))
    print("96k: outer %d, inner %d cluster pairs" % (ref_o.size, ref_i0.size), flush=True)
    bb = keys_of(ctxs[0].get_pairs("bb"), n_cl)
    assert np.unique(bb).size == bb.size
    assert np.all(np.isin(ref_o, bb))
    assert bb.size == st0["bb_pairs"]
    for ctx in ctxs:
        ko = keys_of(ctx.get_pairs("outer"), n_cl)
        assert ko.size == np.unique(ko).size
        assert np.array_equal(np.sort(ko), ref_o)
        assert np.array_equal(np.sort(keys_of(ctx.get_pairs("inner"), n_cl)), ref_i0)
    q, lj = dev(c["q"]), dev(c["lj"])
    rng = np.random.default_rng(29)
    x = c["x"].copy()
    part_keys = {p: oracle.inner_pairs(ref_o, g["slot_atom"], g["w"], box, ri, npr, p)
                 for p in range(npr)}
    ahead_keys = dict(part_keys)
    for t in range(1, 5):
        x = (x + rng.normal(0.0, cfg["sigma_step"], x.shape)).astype(np.float32)
        xt = dev(x)
        for ctx in ctxs:
            ctx.step(xt, q, lj, t, energy=False)
        torch.cuda.synchronize()
        p = t % npr
        w_t = oracle.rewrap_with(x, g["k"], box)
        part_keys[p] = oracle.inner_pairs(ref_o, g["slot_atom"], w_t, box, ri, npr, p)
        pa = (t + 1) % npr
        ahead_keys[pa] = oracle.inner_pairs(ref_o, g["slot_atom"], w_t, box, ri, npr, pa)
        ref_i = np.sort(np.concatenate([part_keys[k] for k in range(npr)]))
        ref_a = np.sort(np.concatenate([ahead_keys[k] for k in range(npr)]))
        for k, ctx in enumerate(ctxs):
            ki = np.sort(keys_of(ctx.get_pairs("inner"), n_cl))
            ref = ref_a if SHAPES[k][2] == "ahead" else ref_i
            assert np.array_equal(ki, ref), (t, SHAPES[k])
        print("96k step %d: inner %d cluster pairs in all shapes" % (t, ref_i.size), flush=True)
