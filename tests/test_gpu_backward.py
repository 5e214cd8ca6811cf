"""Parity of the HIP backward pass with the FP64 oracle's backward pass (same adjoint G and
dL/dE given to both), and the autograd.Function chain to per-type sigma/epsilon."""
import math

import numpy as np
import pytest
import torch

import oracle
from conftest import small_random_system
from gpu_common import concat, dev, make_ctx, oracle_params, rel_rms

pytestmark = pytest.mark.gpu

G_TOL = 1e-4


def symmetrize(gl):
    """Split the derivative w.r.t. each off-diagonal table value evenly over its entries."""
    out = gl.copy()
    T = gl.shape[0]
    for a in range(T):
        for b in range(T):
            if a != b:
                out[a, b] = 0.5 * (gl[a, b] + gl[b, a])
    return out


def run_case(s, coul, rc, rinner, rlist, beta, gE, seed=0, need_lj=True):
    c = concat(s)
    ctx = make_ctx(c, coulomb=coul, rc=rc, rinner=rinner, rlist=rlist, beta=beta)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(s.n, 3)).astype(np.float32)
    ge = np.array([gE], np.float64)
    gx, gq, gl = ctx.backward(x, dev(c["q"]), dev(c["lj"]), dev(G), dev(ge, torch.float64),
                              need_lj=need_lj)
    torch.cuda.synchronize()
    p = oracle_params(coul, rc, beta)
    ox, oq, ol = oracle.backward(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p,
                                 G.astype(np.float64), np.array(gE, np.float64))
    return (gx.cpu().numpy(), gq.cpu().numpy(), None if gl is None else gl.cpu().numpy(),
            ox, oq, symmetrize(ol))


@pytest.mark.parametrize("coul,beta", [("rf", 0.0), ("ewald", 3.12)])
def test_backward_small(coul, beta):
    s = small_random_system(31, 400, 2.8, n_types=3, min_dist=0.2)
    gx, gq, gl, ox, oq, ol = run_case(s, coul, 1.0, 1.05, 1.1, beta, (0.3, -0.7))
    assert rel_rms(gx, ox) <= G_TOL, rel_rms(gx, ox)
    assert rel_rms(gq, oq) <= G_TOL, rel_rms(gq, oq)
    assert rel_rms(gl, ol) <= G_TOL, rel_rms(gl, ol)


def test_backward_diff24k(sys24k):
    """The differentiation workload: 24k atoms, 4 LJ types, random neutral charges, RF."""
    s = sys24k
    gx, gq, gl, ox, oq, ol = run_case(s, "rf", 1.0, 1.0, 1.0, 0.0, (0.0, 0.0))
    for name, a, b in (("x", gx, ox), ("q", gq, oq), ("lj", gl, ol)):
        err = rel_rms(a, b)
        print("grad_%s rel RMS %.3e" % (name, err))
        assert err <= G_TOL, (name, err)


def test_backward_water_ewald_no_table(sys3k):
    gx, gq, gl, ox, oq, ol = run_case(sys3k, "ewald", 1.0, 1.04, 1.1, 3.12, (1.0, 1.0),
                                      need_lj=False)
    assert gl is None
    assert rel_rms(gx, ox) <= G_TOL and rel_rms(gq, oq) <= G_TOL


def test_autograd_force_matching_chain():
    """NBForces through torch autograd: loss = sum |F(theta) - F_ref|^2 with F_ref from
    parameters scaled by 1.05; gradients w.r.t. x, q, sigma, eps against the FP64 oracle
    gradient chained through the Lorentz-Berthelot rule in double precision."""
    from paper_2006_09167_amd.api import NBForces, lj_table
    s = small_random_system(41, 300, 2.6, n_types=4, min_dist=0.2)
    c = concat(s)
    ctx = make_ctx(c, coulomb="rf", rc=1.0, rinner=1.0, rlist=1.0)
    xg = dev(c["x"])
    ctx.grid_build(xg, c["boxes"])
    ctx.pairlist_build()
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(s.eps, dtype=torch.float64, device="cuda", requires_grad=True)
    x = xg.clone().requires_grad_(True)
    q = dev(c["q"]).requires_grad_(True)
    p = oracle_params("rf", 1.0)
    lj_ref = (s.lj.astype(np.float64) * 1.05).astype(np.float32)
    _, f_ref, _ = oracle.forces(s.x, (s.q * np.float32(1.05)), s.type, lj_ref, s.excl_ptr,
                                s.excl_idx, s.box, p)
    f_ref_t = torch.tensor(f_ref, dtype=torch.float32, device="cuda")
    lj = lj_table(sig, eps)
    f, e = NBForces.apply(x, q, lj, ctx)
    loss = ((f - f_ref_t) ** 2).sum()
    loss.backward()
    # oracle chain: G = 2 (F - F_ref) from the oracle forces at the float32 table
    lj32 = lj.detach().cpu().numpy()
    _, f_o, _ = oracle.forces(s.x, s.q, s.type, lj32, s.excl_ptr, s.excl_idx, s.box, p)
    G = 2.0 * (f_o - f_ref)
    ox, oq, ol = oracle.backward(s.x, s.q, s.type, lj32, s.excl_ptr, s.excl_idx, s.box, p, G)
    sig_c = torch.tensor(s.sigma, dtype=torch.float64, requires_grad=True)
    eps_c = torch.tensor(s.eps, dtype=torch.float64, requires_grad=True)
    sg = 0.5 * (sig_c[:, None] + sig_c[None, :])
    eg = torch.sqrt(eps_c[:, None] * eps_c[None, :])
    tab = torch.stack([4 * eg * sg ** 6, 4 * eg * sg ** 12], -1)
    (tab * torch.tensor(symmetrize(ol))).sum().backward()
    assert rel_rms(x.grad.cpu().numpy(), ox) <= 1e-3       # G itself carries FP32 force error
    assert rel_rms(q.grad.cpu().numpy(), oq) <= 1e-3
    assert rel_rms(sig.grad.cpu().numpy(), sig_c.grad.numpy()) <= 1e-3
    assert rel_rms(eps.grad.cpu().numpy(), eps_c.grad.numpy()) <= 1e-3


@pytest.mark.parametrize("n_types", [4, 6])
def test_backward_persistent_schedule_matches_static(sys24k, n_types):
    """The persistent schedule (a resident grid, several items per wavefront, the table
    histogram cleared between items) gives bitwise the backward pass of one wavefront per
    item.  Four types use the lane-private histograms, six the shared ones with LDS
    atomics; one entry per item makes many more items than resident wavefronts."""
    import dataclasses
    from paper_2006_09167_amd.systems import lj_table_lorentz_berthelot
    rng = np.random.default_rng(7)
    s = sys24k
    if n_types != s.n_types:
        sig = rng.uniform(0.25, 0.40, n_types)
        eps = rng.uniform(0.1, 1.0, n_types)
        s = dataclasses.replace(s, type=rng.integers(0, n_types, s.n).astype(np.int32),
                                sigma=sig, eps=eps, lj=lj_table_lorentz_berthelot(sig, eps))
    c = concat(s)
    ctx = make_ctx(c, coulomb="rf", rc=1.0, rinner=1.0, rlist=1.0)
    x = dev(c["x"])
    ctx.grid_build(x, c["boxes"])
    ctx.pairlist_build()
    G = dev(rng.normal(size=(s.n, 3)).astype(np.float32))
    ge = dev(np.array([[0.3, -0.7]], np.float64), torch.float64)
    out = {}
    for mode in ("static", "persist"):
        ctx.set_exec(1, mode)
        out[mode] = ctx.backward(x, dev(c["q"]), dev(c["lj"]), G, ge)
        torch.cuda.synchronize()
    assert ctx.stats()["n_work_items"] > 12000
    for a, b in zip(out["static"], out["persist"]):
        assert torch.equal(a, b)
