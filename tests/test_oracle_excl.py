"""Pins of the oracle's electrostatic corrections for excluded pairs and for each atom with
itself (a run with a long-range part: the real-space Ewald correction of PME runs and
its reaction-field counterpart, Sec. V.A), against facts that do not come from the
oracle: the limit of small beta, the Taylor expansion at small distance, the potential of
a Gaussian charge cloud by numerical quadrature, the exact cancellation for a neutral
molecule under a plain cut-off reaction field, the value at the cut-off, forces as minus
the energy gradient, the box-scaling identity of the virial, and the cell-grid sums."""
import math

import numpy as np
import pytest
from scipy import integrate

from conftest import small_random_system
from paper_2006_09167_amd.systems import System, lj_table_lorentz_berthelot

EPSFAC = float(np.float32(138.935458))


def pair(r, q=(0.7, -0.4), excluded=True, box=4.0):
    x = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]], dtype=np.float32)
    sig, ep = np.array([0.3, 0.0]), np.array([0.5, 0.0])
    ptr = np.array([0, 1, 2], np.int64) if excluded else np.zeros(3, np.int64)
    idx = np.array([1, 0], np.int32) if excluded else np.zeros(0, np.int32)
    return System(x=x, q=np.array(q, np.float32), type=np.array([0, 0], np.int32),
                  excl_ptr=ptr, excl_idx=idx, box=np.full(3, box, np.float32), sigma=sig,
                  eps=ep, lj=lj_table_lorentz_berthelot(sig, ep))


def run(o, s, **kw):
    return o.forces(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, o.params(**kw))


def delta(o, s, **kw):
    """Energies, forces and virial of the corrections alone."""
    e1, f1, v1 = run(o, s, excl_corr=True, **kw)
    e0, f0, v0 = run(o, s, excl_corr=False, **kw)
    return e1 - e0, f1 - f0, v1 - v0


def rdist(s):
    return float(np.float64(s.x[1, 0]) - np.float64(s.x[0, 0]))


def test_corrections_off_by_default(oracle_mod):
    s = pair(0.1)
    e, f, v = run(oracle_mod, s, coulomb="ewald", rc=1.0, beta=3.12)
    assert np.all(e == 0) and np.all(f == 0) and np.all(v == 0)


def test_ewald_small_beta_limit(oracle_mod):
    """As beta -> 0 the corrections vanish linearly: dE/beta -> -(K/sqrt(pi)) (sum_a q_a^2 +
    2 sum over excluded pairs inside rc of q_a q_b) (erf(x)/x -> 2/sqrt(pi)).  Random
    charges (groups of three excluded atoms, not neutral), a few dozen atoms so that both
    evaluations sum in the same order."""
    s = small_random_system(73, 40, 2.6, min_dist=0.09, excl_groups=3, charge=0.6)
    beta = float(np.float32(1e-5))
    de, df, _ = delta(oracle_mod, s, coulomb="ewald", rc=1.0, beta=beta)
    q = s.q.astype(np.float64)
    self_sum = float(np.sum(q * q))
    pair_sum, n_in = 0.0, 0
    for a in range(s.n):
        for k in range(s.excl_ptr[a], s.excl_ptr[a + 1]):
            b = int(s.excl_idx[k])
            if b > a:
                d = s.x[a].astype(np.float64) - s.x[b].astype(np.float64)
                d -= s.box * np.round(d / s.box)
                if np.dot(d, d) < 1.0:
                    pair_sum += q[a] * q[b]
                    n_in += 1
    assert n_in >= 5
    expect = -(EPSFAC / math.sqrt(math.pi)) * (self_sum + 2.0 * pair_sum)
    assert de[1] / beta == pytest.approx(expect, rel=1e-8)
    assert de[0] == 0.0
    assert np.abs(df).max() < 1e-6             # forces go as beta^3


@pytest.mark.parametrize("r", [1e-3, 2e-2])
def test_ewald_small_distance_taylor(oracle_mod, r):
    """x = beta r: erf(x)/x = (2/sqrt(pi))(1 - x^2/3 + x^4/10 - x^6/42) and
    exp(-x^2) - erf(x)/x = -2x^2/3 + 2x^4/5 - x^6/7, so for the pair
    V = -kq (2 beta/sqrt(pi))(1 - x^2/3 + x^4/10 - ...), phi = kq (2 beta^3/sqrt(pi))
    (-2/3 + 2x^2/5 - x^4/7 + ...)."""
    beta = float(np.float32(3.12))
    s = pair(r, q=(0.7, -0.4))
    rr = rdist(s)
    x = beta * rr
    kq = EPSFAC * float(np.float32(0.7)) * float(np.float32(-0.4))
    de, df, _ = delta(oracle_mod, s, coulomb="ewald", rc=1.0, beta=beta)
    selfs = -EPSFAC * beta / math.sqrt(math.pi) * (float(np.float32(0.7)) ** 2
                                                   + float(np.float32(-0.4)) ** 2)
    v = -kq * 2 * beta / math.sqrt(math.pi) * (1 - x ** 2 / 3 + x ** 4 / 10 - x ** 6 / 42)
    phi = kq * 2 * beta ** 3 / math.sqrt(math.pi) * (-2 / 3 + 2 * x ** 2 / 5 - x ** 4 / 7)
    assert de[1] - selfs == pytest.approx(v, rel=1e-9)
    # force on atom 0 is phi * (x_0 - x_1) = -phi r along x
    assert df[0, 0] == pytest.approx(-phi * rr, rel=1e-6)
    assert df[1, 0] == pytest.approx(phi * rr, rel=1e-6)


@pytest.mark.parametrize("r", [0.09, 0.1, 0.1633, 0.3, 0.7])
def test_ewald_correction_is_a_gaussian_cloud_potential(oracle_mod, r):
    """erf(beta r)/r is the potential at r of a unit charge spread as the Gaussian
    (beta/sqrt(pi))^3 exp(-beta^2 s^2); evaluated by radial quadrature."""
    beta = float(np.float32(3.12))
    s = pair(r, q=(1.0, 1.0))
    rr = rdist(s)
    rho = lambda u: (beta / math.sqrt(math.pi)) ** 3 * math.exp(-beta * beta * u * u)
    inner = integrate.quad(lambda u: rho(u) * u * u, 0, rr, epsabs=0, epsrel=1e-12)[0]
    outer = integrate.quad(lambda u: rho(u) * u, rr, np.inf, epsabs=0, epsrel=1e-12)[0]
    phi_cloud = 4 * math.pi * (inner / rr + outer)
    de, _, _ = delta(oracle_mod, s, coulomb="ewald", rc=1.0, beta=beta)
    selfs = -2.0 * EPSFAC * beta / math.sqrt(math.pi)
    assert de[1] - selfs == pytest.approx(-EPSFAC * phi_cloud, rel=1e-9)


def test_rf_plain_cutoff_neutral_molecule_cancels(oracle_mod):
    """With eps_rf = eps_r (k_rf = 0, c_rf = 1/rc) the corrections of a fully excluded
    molecule are -K c_rf (sum_{a<b} q_a q_b + 1/2 sum_a q_a^2) = -(K c_rf / 2)(sum_a q_a)^2:
    zero for a neutral molecule (here one water-like molecule and one 4-site ion pair)."""
    x = np.array([[1.0, 1.0, 1.0], [1.1, 1.0, 1.0], [0.97, 1.09, 1.0],
                  [2.5, 2.5, 2.5], [2.6, 2.5, 2.5], [2.5, 2.62, 2.5], [2.5, 2.5, 2.7]],
                 np.float32)
    q = np.array([-0.82, 0.41, 0.41, 0.5, -0.25, 0.3, -0.55], np.float32)
    groups = [[0, 1, 2], [3, 4, 5, 6]]
    ptr, idx = [0], []
    for g in groups:
        for a in g:
            idx += [b for b in g if b != a]
            ptr.append(len(idx))
    sig, ep = np.array([0.0]), np.array([0.0])
    s = System(x=x, q=q, type=np.zeros(7, np.int32), excl_ptr=np.array(ptr, np.int64),
               excl_idx=np.array(idx, np.int32), box=np.full(3, 5.0, np.float32), sigma=sig,
               eps=ep, lj=lj_table_lorentz_berthelot(sig, ep))
    de, df, _ = delta(oracle_mod, s, coulomb="rf", rc=1.0, eps_rf=1.0)
    tot = [float(np.sum(q[g].astype(np.float64))) for g in groups]
    expect = -EPSFAC * 0.5 * sum(t * t for t in tot)          # ~1e-14: float32 charges
    assert de[1] == pytest.approx(expect, abs=1e-9)
    assert np.all(df == 0)


def test_rf_infinite_dielectric_value_near_cutoff(oracle_mod):
    """eps_rf = inf: k_rf = 1/(2 rc^3), c_rf = 3/(2 rc); an excluded pair at r = rc keeps
    V = kq (1/(2 rc) - 3/(2 rc)) = -kq/rc, with force phi d = -kq d / rc^3."""
    s = pair(0.999999, q=(1.0, 1.0))
    rr = rdist(s)
    de, df, _ = delta(oracle_mod, s, coulomb="rf", rc=1.0)
    selfs = -0.5 * EPSFAC * 1.5 * 2
    assert de[1] - selfs == pytest.approx(EPSFAC * (rr * rr / 2 - 1.5), rel=1e-12)
    assert de[1] - selfs == pytest.approx(-EPSFAC, rel=1e-5)
    assert df[0, 0] == pytest.approx(EPSFAC * rr, rel=1e-12)     # phi = -kq, d = -r
    # beyond the cut-off an excluded pair keeps only the self terms
    far = pair(1.2, q=(1.0, 1.0))
    de2, df2, _ = delta(oracle_mod, far, coulomb="rf", rc=1.0)
    assert de2[1] == pytest.approx(selfs, rel=1e-12) and np.all(df2 == 0)


@pytest.mark.parametrize("coul", ["rf", "ewald"])
def test_corrected_forces_are_minus_energy_gradient(oracle_mod, coul):
    s = small_random_system(71, 45, 2.6, min_dist=0.09, excl_groups=3)
    h = 2.0 ** -14
    kw = dict(coulomb=coul, rc=1.0, beta=3.12, excl_corr=True)
    e0, f, _ = run(oracle_mod, s, **kw)
    de, df, _ = delta(oracle_mod, s, coulomb=coul, rc=1.0, beta=3.12)
    assert np.abs(df).max() > 1.0                # the corrections carry forces here
    rng = np.random.default_rng(4)
    for a in rng.choice(s.n, 6, replace=False):
        for k in range(3):
            xp, xm = s.x.copy(), s.x.copy()
            xp[a, k] = np.float32(xp[a, k] + h)
            xm[a, k] = np.float32(xm[a, k] - h)
            dx = float(np.float64(xp[a, k]) - np.float64(xm[a, k]))
            ep, _, _ = run(oracle_mod, System(**{**s.__dict__, "x": xp}), **kw)
            em, _, _ = run(oracle_mod, System(**{**s.__dict__, "x": xm}), **kw)
            fd = -(ep.sum() - em.sum()) / dx
            assert fd == pytest.approx(f[a, k], rel=1e-5, abs=1e-6 * np.abs(f).max())


@pytest.mark.parametrize("coul", ["rf", "ewald"])
def test_corrected_virial_box_scaling_identity(oracle_mod, coul):
    """dE(lambda_k x_k, lambda_k L_k)/d lambda_k at 1 equals 2 Xi_kk with the corrections
    (the self terms do not depend on positions).  Dyadic coordinates keep the scaled
    single-precision inputs exact."""
    s = small_random_system(72, 50, 3.0, dyadic=True, min_dist=0.09)
    kw = dict(coulomb=coul, rc=1.0, beta=3.12, excl_corr=True)
    _, _, v = run(oracle_mod, s, **kw)
    for k in range(3):
        vals = []
        for lam in (1.0 + 2.0 ** -12, 1.0 - 2.0 ** -12):
            sc = np.ones(3)
            sc[k] = lam
            xs = (s.x.astype(np.float64) * sc).astype(np.float32)
            bs = (s.box.astype(np.float64) * sc).astype(np.float32)
            e, _, _ = run(oracle_mod, System(**{**s.__dict__, "x": xs, "box": bs}), **kw)
            vals.append(e.sum())
        dedl = (vals[0] - vals[1]) / (2.0 ** -11)
        assert dedl == pytest.approx(2.0 * v[k, k], rel=1e-4, abs=1e-4 * np.abs(v).max())


def test_corrected_cells_equal_all_pairs(oracle_mod, sys3k):
    for kw in (dict(coulomb="ewald", rc=1.0, beta=3.12), dict(coulomb="rf", rc=1.0)):
        p = oracle_mod.params(excl_corr=True, **kw)
        args = (sys3k.x, sys3k.q, sys3k.type, sys3k.lj, sys3k.excl_ptr, sys3k.excl_idx,
                sys3k.box, p)
        e0, f0, v0 = oracle_mod.forces(*args)
        e1, f1, v1 = oracle_mod.forces_cells(*args)
        assert np.abs(f1 - f0).max() <= 1e-12 * np.abs(f0).max()
        assert np.allclose(e1, e0, rtol=1e-12) and np.allclose(v1, v0, rtol=1e-10)
        sel = np.arange(0, sys3k.n, 37)
        fo = oracle_mod.forces_on(sel, *args)
        assert np.abs(fo - f0[sel]).max() <= 1e-12 * np.abs(f0).max()
