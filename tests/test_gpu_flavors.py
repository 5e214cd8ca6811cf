"""The force-only flavors of the pair kernel (no energies; with and without the virial) for
reaction-field, Ewald and Lennard-Jones-only electrostatics, through nb_forces and through
nb_step with the rolling prune fused into the pair kernel and as its own kernels, against
the FP64 oracle: forces within 1e-5 relative RMS, virial within 1e-5 relative RMS.  These
are the flavors the argon throughput sweep times and that a dynamics step without energy
output runs (Sec. V.A: separate kernels for each interaction type and for energies or not).
The masked lanes of these flavors (a cluster with itself, empty slots) reach 1/r = inf and
are removed only by the final selects, so each case also checks that every force is
finite."""
import math

import numpy as np
import pytest
import torch

from gpu_common import concat, dev, make_ctx, oracle_forces_multi, oracle_params, rel_rms
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
V_TOL = 1e-5

# (coulomb for the library, for the oracle, beta); LJ-only is the oracle with zero charges
FLAVORS = [("rf", "rf", 0.0), ("ewald", "ewald", 3.12), ("none", "rf", 0.0)]


def charges(c, coul):
    return np.zeros_like(c["q"]) if coul == "none" else c["q"]


def oracle_fv(c, x, coul, beta, rc):
    cc = dict(c)
    cc["q"] = charges(c, coul[0])
    _, F, V, _ = oracle_forces_multi(cc, x, oracle_params(coul[1], rc, beta))
    return F, V


def check(f, v, F, V, what):
    f = f.cpu().numpy()
    assert np.all(np.isfinite(f)), what
    err = rel_rms(f, F)
    assert err <= F_TOL, (what, err)
    if v is not None:
        ev = rel_rms(v.cpu().numpy(), V)
        assert ev <= V_TOL, (what, ev)
    return err


def run_flavor(c, flavor, rc, rinner, rlist, nstlist, nstprune, steps, sigma, seed,
               exec_shape=None):
    """Force-only calls at the build positions, then rolling steps through nb_step with
    the prune fused (context a) and separate (context b), each against the oracle."""
    coul, _, beta = flavor
    q = dev(charges(c, coul))
    lj = dev(c["lj"])
    ctxs = []
    for fused in (True, False):
        ctx = make_ctx(c, coulomb=coul, rc=rc, rinner=rinner, rlist=rlist, beta=beta,
                       nstlist=nstlist, nstprune=nstprune)
        x0 = dev(c["x"])
        ctx.grid_build(x0, c["boxes"])
        ctx.pairlist_build()
        w, mode = exec_shape or (0, "static")
        ctx.set_exec(w, mode, fused)
        ctxs.append(ctx)
    x = c["x"].copy()
    F, V = oracle_fv(c, x, flavor, beta, rc)
    for virial in (False, True):
        f, _, v = ctxs[0].forces(dev(x), q, lj, energy=False, virial=virial)
        torch.cuda.synchronize()
        check(f, v, F, V, (coul, "nb_forces", virial))
    rng = np.random.default_rng(seed)
    errs = []
    for t in range(1, steps + 1):
        x = (x + rng.normal(0.0, sigma, x.shape)).astype(np.float32)
        F, V = oracle_fv(c, x, flavor, beta, rc)
        xt = dev(x)
        for k, ctx in enumerate(ctxs):
            virial = (t + k) % 2 == 1
            f, _, v = ctx.step(xt, q, lj, t, energy=False, virial=virial)
            torch.cuda.synchronize()
            errs.append(check(f, v, F, V, (coul, "nb_step", "fused" if k == 0 else "separate",
                                           t, virial)))
    # both contexts kept the same inner list and give bitwise equal forces
    fa, _, _ = ctxs[0].forces(xt, q, lj, energy=False)
    fb, _, _ = ctxs[1].forces(xt, q, lj, energy=False)
    assert torch.equal(fa, fb)
    return max(errs)


@pytest.mark.parametrize("flavor", FLAVORS, ids=[f[0] for f in FLAVORS])
def test_force_only_flavors_water3k(sys3k, flavor):
    c = concat(sys3k)
    run_flavor(c, flavor, 1.0, 1.04, 1.1, nstlist=20, nstprune=4, steps=4, sigma=0.002, seed=5)


@pytest.mark.parametrize("flavor", FLAVORS, ids=[f[0] for f in FLAVORS])
def test_force_only_flavors_water96k(flavor):
    """The 96,000-atom box in the benchmark's execution shape (40 entries per item,
    persistent balanced schedule), forces of every atom against the all-pairs oracle."""
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    cfg = systems.CONFIGS["water96k_ewald"]
    err = run_flavor(c, flavor, cfg["rc"], cfg["rinner"], cfg["rlist"], cfg["nstlist"],
                     cfg["nstprune"], steps=2, sigma=cfg["sigma_step"], seed=9,
                     exec_shape=(40, "persist"))
    print("%s force-only: worst force rel RMS %.2e" % (flavor[0], err))


def test_force_only_argon_sweep_flavor():
    """The argon sweep's flavor (LJ only, no energies, no virial) on a 2744-atom argon box at
    the sweep's shortest and a mid cut-off."""
    s = systems.argon_box(k=14, seed=11)
    c = concat(s)
    lj = dev(c["lj"])
    q = dev(np.zeros(s.n, np.float32))
    for n_half in (50, 200):
        rc = systems.argon_cutoff(n_half)
        rlist = rc + systems.ARGON["buffer"]
        ctx = make_ctx(c, coulomb="none", rc=rc, rinner=rlist, rlist=rlist)
        x = dev(c["x"])
        ctx.grid_build(x, c["boxes"])
        ctx.pairlist_build()
        f, _, _ = ctx.forces(x, q, lj, energy=False, virial=False)
        torch.cuda.synchronize()
        _, F, _, _ = oracle_forces_multi(c, c["x"], oracle_params("rf", rc))
        check(f, None, F, None, ("argon", n_half))
