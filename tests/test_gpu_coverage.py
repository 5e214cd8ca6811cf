"""Coverage of the dual list over one list lifetime on the 96,000-atom box: at checked
steps every non-excluded atom pair inside rc (minimum image, FP64 distances of the
step's positions) must belong to a cluster pair of the GPU's current inner list.

A pair inside rc can be missed only if its cluster pair left the inner list at a rolling
prune (inner buffer rinner - rc) or was never in the outer list (outer buffer rlist - rc
over up to nstlist - 1 steps of drift).  The first kind must not happen here; the second
is counted and reported (the paper sizes rlist from a drift tolerance, which is not part
of this path), and bounded."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import concat, dev, keys_of, make_ctx
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu


def required_keys(x, k_build, box, slot_of, n_cl, rc, mol):
    """Canonical cluster-pair keys of all non-excluded atom pairs with r < rc."""
    from scipy.spatial import cKDTree
    L = box.astype(np.float64)
    xp = x.astype(np.float64) - k_build * L              # build-time image, continuous
    xw = np.mod(xp, L)
    xw[xw >= L] = 0.0
    pairs = cKDTree(xw, boxsize=L).query_pairs(rc, output_type="ndarray")
    a, b = pairs[:, 0], pairs[:, 1]
    keep = mol[a] != mol[b]                               # intramolecular pairs are excluded
    a, b = a[keep], b[keep]
    s = np.rint((xp[a] - xp[b]) / L).astype(np.int64)     # image of b nearest to a: x_b + s L
    ca, cb = slot_of[a] // 8, slot_of[b] // 8
    swap = ca > cb
    ci, cj = np.where(swap, cb, ca), np.where(swap, ca, cb)
    s = np.where(swap[:, None], -s, s)
    same = (ci == cj) & np.any(s != 0, axis=1)
    if np.any(same):                                      # lexicographically positive shift
        first = np.argmax(s[same] != 0, axis=1)
        neg = s[same][np.arange(first.size), first] < 0
        s_same = s[same]
        s_same[neg] = -s_same[neg]
        s[same] = s_same
    code = (s[:, 0] + 1) * 9 + (s[:, 1] + 1) * 3 + (s[:, 2] + 1)
    return (ci * n_cl + cj) * 27 + code, a.size


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prune", [True, "ahead"])
def test_dual_list_coverage_96k(prune):
    """With the prune fused, step t prunes its part with its own positions, so the inner
    list after the step is the one it used; with the ahead prune a part is pruned one step
    before its first use, so the list checked against step t's positions is the one
    before the step."""
    cfg = systems.CONFIGS["water96k_ewald"]
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    ctx = make_ctx(c, coulomb="ewald", rc=cfg["rc"], rinner=cfg["rinner"], rlist=cfg["rlist"],
                   beta=cfg["beta"], nstlist=cfg["nstlist"], nstprune=cfg["nstprune"])
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    ctx.grid_build(dev(c["x"]), c["boxes"])
    ctx.pairlist_build()
    ctx.set_exec(0, "static", prune_fused=prune)
    assert np.array_equal(ctx.get_grid(), g["slot_atom"])
    n_cl = g["slot_atom"].size // 8
    slot_of = g["atom_slot"]
    mol = np.arange(s.n) // 3
    q, lj = dev(c["q"]), dev(c["lj"])
    rng = np.random.default_rng(99)
    x = c["x"].copy()
    check = {1, 2, 3, 4, 5, 50, 98, 99}
    report = []
    if prune == "ahead":
        ctx.step(dev(x), q, lj, 0, energy=False)         # prunes part 1 for step 1
    for t in range(1, cfg["nstlist"]):
        x = (x + rng.normal(0.0, cfg["sigma_step"], x.shape)).astype(np.float32)
        if prune == "ahead" and t in check:
            inner = np.unique(keys_of(ctx.get_pairs("inner"), n_cl))   # the list step t uses
        ctx.step(dev(x), q, lj, t, energy=False)
        if t not in check:
            continue
        if prune is True:
            inner = np.unique(keys_of(ctx.get_pairs("inner"), n_cl))
        outer = np.unique(keys_of(ctx.get_pairs("outer"), n_cl))
        need, n_pairs = required_keys(x, g["k"], c["boxes"][0], slot_of, n_cl,
                                      float(cfg["rc"]), mol)
        in_inner = np.isin(need, inner)
        in_outer = np.isin(need, outer)
        miss_inner = int(np.sum(in_outer & ~in_inner))   # dropped by a rolling prune
        miss_outer = int(np.sum(~in_outer))              # never in the outer list
        report.append((t, n_pairs, miss_inner, miss_outer))
        print("step %d: %d pairs inside rc, inner-buffer misses %d, outer-buffer misses %d"
              % (t, n_pairs, miss_inner, miss_outer))
        assert miss_inner == 0, (t, miss_inner)
        assert miss_outer <= 1e-6 * n_pairs, (t, miss_outer)
    torch.cuda.synchronize()
    assert len(report) == len(check)
