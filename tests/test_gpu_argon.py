"""Lennard-Jones-only electrostatics flavor (NB_COUL_NONE) on argon boxes, the workload of
the paper's kernel-throughput sweep (Fig. 6): grid and pair lists bit-exact against the
oracle, forces, E_LJ and virial against the FP64 oracle run with zero charges, E_C exactly
zero, and the backward pass against the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import (concat, dev, keys_of, make_ctx, oracle_forces_multi, oracle_pair_keys,
                        oracle_params, rel_rms)
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_half", [50, 400])
def test_argon_lj_only_parity(n_half):
    s = systems.argon_box(k=14, seed=11)          # 2744 atoms, 4.7 nm box
    rc = systems.argon_cutoff(n_half)             # 0.97 nm and 1.94 nm
    rlist = rc + systems.ARGON["buffer"]
    c = concat(s)
    ctx = make_ctx(c, coulomb="none", rc=rc, rinner=rlist, rlist=rlist)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    assert np.array_equal(ctx.get_grid(), g["slot_atom"])
    n_cl = g["slot_atom"].size // 8
    ko = keys_of(ctx.get_pairs("outer"), n_cl)
    assert np.unique(ko).size == ko.size
    assert np.array_equal(np.sort(ko), oracle_pair_keys(c, g, rlist))

    q, lj = dev(c["q"]), dev(c["lj"])
    f, e, v = ctx.forces(x, q, lj, energy=True, virial=True)
    torch.cuda.synchronize()
    E, F, V, A = oracle_forces_multi(c, c["x"], oracle_params("rf", rc))   # all q = 0
    f, e, v = f.cpu().numpy(), e.cpu().numpy(), v.cpu().numpy()
    assert rel_rms(f, F) <= 1e-5, rel_rms(f, F)
    # At this density the lattice sits near the LJ zero crossing: E_LJ is a near-cancellation
    # of much larger pair energies (sum |e_pair| / |E_LJ| is 23 at the shorter cut-off and
    # 84 at the longer).  Each FP32 pair energy carries the error of r^-12 from the
    # hardware reciprocal square root (up to 1 ulp, times 12: a few 1e-7 relative), so the
    # bound here is max(1e-6 |E|, 1e-7 sum |e_pair|).
    tol = max(1e-6 * abs(E[0, 0]), 1e-7 * A[0, 0])
    assert abs(e[0, 0] - E[0, 0]) <= tol, (e[0, 0], E[0, 0], A[0, 0])
    assert e[0, 1] == 0.0 and E[0, 1] == 0.0
    assert rel_rms(v, V) <= 1e-5
    st = ctx.stats()
    assert st["effective_pairs"] > 0.8 * n_half * s.n      # about n_half pairs per atom


def test_argon_lj_only_backward():
    s = systems.argon_box(k=12, seed=12)          # 1728 atoms, 4.0 nm box
    rc = systems.argon_cutoff(100)
    c = concat(s)
    ctx = make_ctx(c, coulomb="none", rc=rc, rinner=rc, rlist=rc)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    rng = np.random.default_rng(3)
    G = rng.normal(size=(s.n, 3)).astype(np.float32)
    gE = np.array([[0.4, 0.0]], np.float64)
    gx, gq, gl = ctx.backward(x, dev(c["q"]), dev(c["lj"]), dev(G), dev(gE, torch.float64))
    torch.cuda.synchronize()
    ox, oq, ol = oracle.backward(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box,
                                 oracle_params("rf", rc), G.astype(np.float64), gE[0])
    assert rel_rms(gx.cpu().numpy(), ox) <= 1e-4
    assert np.all(gq.cpu().numpy() == 0.0)
    assert rel_rms(gl.cpu().numpy(), ol) <= 1e-4
