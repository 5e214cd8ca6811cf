"""Pins of the FP64 oracle's energies, forces and virial against facts that do not
come from the oracle itself: closed forms of the potentials, numerical
quadrature of the Gaussian tail, Newton's third law, finite differences of the
energy, the box-scaling identity of the virial, and invariances."""
import math

import numpy as np
import pytest
from scipy import integrate

from conftest import small_random_system
from paper_2006_09167_amd.systems import System, lj_table_lorentz_berthelot

EPSFAC = float(np.float32(138.935458))   # the single-precision value the library receives


def two_atoms(r, t=(0, 0), q=(0.0, 0.0), sigma=(0.3166, 0.0), eps=(0.65, 0.0), box=3.0,
              excluded=False):
    x = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]], dtype=np.float32)
    sig, ep = np.array(sigma), np.array(eps)
    ptr = np.array([0, 1, 2], np.int64) if excluded else np.zeros(3, np.int64)
    idx = np.array([1, 0], np.int32) if excluded else np.zeros(0, np.int32)
    return System(x=x, q=np.array(q, np.float32), type=np.array(t, np.int32), excl_ptr=ptr,
                  excl_idx=idx, box=np.full(3, box, np.float32), sigma=sig, eps=ep,
                  lj=lj_table_lorentz_berthelot(sig, ep))


def run(o, s, **kw):
    p = o.params(**kw)
    return o.forces(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)


def rdist(s):
    return float(np.float64(s.x[1, 0]) - np.float64(s.x[0, 0]))


# ---- Lennard-Jones closed forms ------------------------------------------------------
def test_lj_minimum_is_minus_epsilon_with_zero_force(oracle_mod):
    sigma, eps = 0.3166, 0.65
    s = two_atoms(2 ** (1 / 6) * sigma)
    r = rdist(s)
    e, f, _ = run(oracle_mod, s, coulomb="rf", rc=1.0, modifier="none")
    # Exact textbook value at the float32 distance, in sigma/epsilon form.
    expect = 4 * eps * ((sigma / r) ** 12 - (sigma / r) ** 6)
    assert e[0] == pytest.approx(expect, rel=1e-6)       # c6/c12 are float32 inputs
    assert e[0] == pytest.approx(-eps, rel=1e-5)
    assert abs(f[0, 0]) < 1e-4 * 24 * eps / sigma


def test_lj_zero_at_sigma_and_shift(oracle_mod):
    sigma, eps = 0.3166, 0.65
    s = two_atoms(sigma)
    r = rdist(s)
    e, _, _ = run(oracle_mod, s, coulomb="rf", rc=1.0, modifier="none")
    assert abs(e[0]) < 1e-5 * eps + abs(4 * eps * ((sigma / r) ** 12 - (sigma / r) ** 6))
    e2, _, _ = run(oracle_mod, s, coulomb="rf", rc=1.0, modifier="potshift")
    shift = 4 * eps * ((sigma / 1.0) ** 12 - (sigma / 1.0) ** 6)
    assert e2[0] - e[0] == pytest.approx(-shift, rel=1e-5)


def test_lj_force_is_24eps_form(oracle_mod):
    sigma, eps = 0.30, 0.8
    for r in (0.28, 0.33, 0.45, 0.8):
        s = two_atoms(r, sigma=(sigma, 0.0), eps=(eps, 0.0))
        rr = rdist(s)
        _, f, _ = run(oracle_mod, s, coulomb="rf", rc=1.0)
        # F_x on atom 0 = -(dV/dr) * (x0 - x1)/r, with dV/dr = 24 eps (s^6/r^7 - 2 s^12/r^13)
        dvdr = 24 * eps * (sigma ** 6 / rr ** 7 - 2 * sigma ** 12 / rr ** 13)
        assert f[0, 0] == pytest.approx(dvdr, rel=2e-6)
        assert f[1, 0] == pytest.approx(-dvdr, rel=2e-6)


# ---- Coulomb closed forms ------------------------------------------------------------
def test_rf_with_equal_dielectrics_is_shifted_coulomb(oracle_mod):
    s = two_atoms(0.5, q=(1.0, -1.0), sigma=(0.0, 0.0), eps=(0.0, 0.0))
    r = rdist(s)
    e, f, _ = run(oracle_mod, s, coulomb="rf", rc=1.0, eps_rf=1.0)
    assert e[1] == pytest.approx(-EPSFAC * (1 / r - 1.0), rel=1e-7)
    assert f[0, 0] == pytest.approx(EPSFAC / r ** 2, rel=1e-7)   # attraction towards +x


def test_rf_infinite_dielectric_vanishes_at_cutoff(oracle_mod):
    rc = 1.0
    s = two_atoms(rc * (1 - 2e-7), q=(0.7, -0.4), sigma=(0.0, 0.0), eps=(0.0, 0.0))
    e, f, _ = run(oracle_mod, s, coulomb="rf", rc=rc, eps_rf=math.inf)
    scale = EPSFAC * 0.28
    assert abs(e[1]) < 1e-6 * scale
    assert abs(f[0, 0]) < 1e-5 * scale
    # Known value inside: V = K (1/r + r^2/(2 rc^3) - 3/(2 rc)) at r = rc/2: K (2 + 1/8 - 3/2)
    s = two_atoms(0.5, q=(1.0, 1.0), sigma=(0.0, 0.0), eps=(0.0, 0.0))
    r = rdist(s)
    e, f, _ = run(oracle_mod, s, coulomb="rf", rc=1.0, eps_rf=math.inf)
    assert e[1] == pytest.approx(EPSFAC * (1 / r + r * r / 2 - 1.5), rel=1e-7)
    assert e[1] == pytest.approx(EPSFAC * 0.625, rel=1e-6)


def _gauss_tail(x):
    """erfc(x) by numerical quadrature of 2/sqrt(pi) exp(-t^2) (not libm)."""
    val, _ = integrate.quad(lambda t: math.exp(-t * t), x, np.inf, epsabs=0, epsrel=1e-13)
    return 2.0 / math.sqrt(math.pi) * val


@pytest.mark.parametrize("r", [0.15, 0.31, 0.5, 0.77, 0.99])
def test_ewald_real_space_matches_quadrature(oracle_mod, r):
    beta, rc = 3.12, 1.0
    s = two_atoms(r, q=(0.41, -0.82), sigma=(0.0, 0.0), eps=(0.0, 0.0), box=4.0)
    rr = rdist(s)
    e, f, _ = run(oracle_mod, s, coulomb="ewald", rc=rc, beta=beta)
    bf = float(np.float32(beta))
    K = EPSFAC * float(np.float32(0.41)) * float(np.float32(-0.82))
    expect_v = K * (_gauss_tail(bf * rr) / rr - _gauss_tail(bf * rc) / rc)
    assert e[1] == pytest.approx(expect_v, rel=1e-9, abs=1e-12)
    # Force from a central difference of the quadrature energy.
    h = 1e-5
    dv = K * (_gauss_tail(bf * (rr + h)) / (rr + h) - _gauss_tail(bf * (rr - h)) / (rr - h)) / (2 * h)
    assert f[1, 0] == pytest.approx(-dv, rel=1e-6)


def test_ewald_small_beta_tends_to_coulomb(oracle_mod):
    s = two_atoms(0.4, q=(1.0, 1.0), sigma=(0.0, 0.0), eps=(0.0, 0.0))
    r = rdist(s)
    e, _, _ = run(oracle_mod, s, coulomb="ewald", rc=1.0, beta=1e-6, modifier="none")
    assert e[1] == pytest.approx(EPSFAC / r, rel=1e-5)


def test_excluded_pair_contributes_nothing(oracle_mod):
    s = two_atoms(0.3, q=(1.0, -1.0), excluded=True)
    e, f, v = run(oracle_mod, s, coulomb="rf", rc=1.0)
    assert np.all(e == 0) and np.all(f == 0) and np.all(v == 0)


def test_beyond_cutoff_and_minimum_image(oracle_mod):
    # 2.6 nm apart in a 3 nm box is 0.4 nm through the boundary.
    s = two_atoms(2.6, q=(1.0, 1.0), sigma=(0.0, 0.0), eps=(0.0, 0.0), box=3.0)
    r = 3.0 - rdist(s)
    e, f, _ = run(oracle_mod, s, coulomb="rf", rc=1.0, eps_rf=1.0)
    assert e[1] == pytest.approx(EPSFAC * (1 / r - 1.0), rel=1e-6)
    assert f[0, 0] > 0          # pushed away from the image of atom 1, at x0 - 0.4
    s = two_atoms(1.2, q=(1.0, 1.0), box=3.0)
    e, f, _ = run(oracle_mod, s, coulomb="rf", rc=1.0)
    assert np.all(e == 0) and np.all(f == 0)


# ---- Whole-system properties -----------------------------------------------------------
@pytest.mark.parametrize("coul", ["rf", "ewald"])
def test_newton_third_law(oracle_mod, sys3k, coul):
    e, f, _ = run(oracle_mod, sys3k, coulomb=coul, rc=1.0, beta=3.12)
    assert np.abs(f.sum(axis=0)).max() < 1e-10 * np.abs(f).sum()


@pytest.mark.parametrize("coul", ["rf", "ewald"])
def test_force_is_minus_energy_gradient(oracle_mod, coul):
    s = small_random_system(11, 40, 2.5, dyadic=False, min_dist=0.22)
    h = 2.0 ** -14
    e0, f, _ = run(oracle_mod, s, coulomb=coul, rc=1.0, beta=3.12)
    rng = np.random.default_rng(3)
    for a in rng.choice(s.n, 6, replace=False):
        for k in range(3):
            xp, xm = s.x.copy(), s.x.copy()
            xp[a, k] = np.float32(xp[a, k] + h)
            xm[a, k] = np.float32(xm[a, k] - h)
            dx = float(np.float64(xp[a, k]) - np.float64(xm[a, k]))
            sp = System(**{**s.__dict__, "x": xp})
            sm = System(**{**s.__dict__, "x": xm})
            ep, _, _ = run(oracle_mod, sp, coulomb=coul, rc=1.0, beta=3.12)
            em, _, _ = run(oracle_mod, sm, coulomb=coul, rc=1.0, beta=3.12)
            fd = -(ep.sum() - em.sum()) / dx
            assert fd == pytest.approx(f[a, k], rel=1e-5, abs=1e-6 * np.abs(f).max())


@pytest.mark.parametrize("coul", ["rf", "ewald"])
def test_virial_box_scaling_identity(oracle_mod, coul):
    """dE(lambda_k x_k, lambda_k L_k)/d lambda_k at 1 equals 2 Xi_kk (per axis), with a
    dyadic system so the scaled single-precision inputs are exact."""
    s = small_random_system(5, 60, 3.0, dyadic=True)
    e0, _, vir = run(oracle_mod, s, coulomb=coul, rc=1.0, beta=3.12)
    h = 2.0 ** -13
    for k in range(3):
        vals = []
        for lam in (1 + h, 1 - h):
            x = s.x.copy()
            box = s.box.copy()
            x[:, k] = x[:, k] * np.float32(lam)
            box[k] = box[k] * np.float32(lam)
            assert np.float64(x[0, k]) == np.float64(s.x[0, k]) * lam   # exact scaling
            e, _, _ = run(oracle_mod, System(**{**s.__dict__, "x": x, "box": box}),
                          coulomb=coul, rc=1.0, beta=3.12)
            vals.append(e.sum())
        dE = (vals[0] - vals[1]) / (2 * h)
        assert dE == pytest.approx(2 * vir[k, k], rel=1e-5, abs=1e-6 * abs(vir).max())
    assert np.allclose(vir, vir.T, rtol=0, atol=1e-10 * abs(vir).max())


def test_translation_and_permutation_invariance(oracle_mod, sys3k):
    s = sys3k
    e0, f0, v0 = run(oracle_mod, s, coulomb="ewald", rc=1.0, beta=3.12)
    # Whole box translated by a lattice vector: identical float32 separations modulo L.
    x = s.x.copy()
    x[::7] += s.box            # some atoms moved by one box length (periodic image)
    e1, f1, v1 = run(oracle_mod, System(**{**s.__dict__, "x": x}), coulomb="ewald", rc=1.0,
                     beta=3.12)
    assert e1 == pytest.approx(e0, rel=1e-5)          # float32 rounding of x + L
    # Permutation of the atoms (exclusions remapped).
    rng = np.random.default_rng(0)
    perm = rng.permutation(s.n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(s.n)
    ptr = [0]
    idx = []
    for new in range(s.n):
        old = perm[new]
        part = inv[s.excl_idx[s.excl_ptr[old]:s.excl_ptr[old + 1]]]
        idx.extend(part.tolist())
        ptr.append(len(idx))
    sp = System(**{**s.__dict__, "x": s.x[perm], "q": s.q[perm], "type": s.type[perm],
                   "excl_ptr": np.array(ptr, np.int64), "excl_idx": np.array(idx, np.int32)})
    e2, f2, v2 = run(oracle_mod, sp, coulomb="ewald", rc=1.0, beta=3.12)
    assert e2 == pytest.approx(e0, rel=1e-12)
    assert np.allclose(f2, f0[perm], rtol=1e-10, atol=1e-9)
    assert np.allclose(v2, v0, rtol=1e-11, atol=1e-9)


def test_forces_on_matches_full(oracle_mod, sys3k):
    s = sys3k
    p = oracle_mod.params("ewald", rc=1.0, beta=3.12)
    e, f, _ = oracle_mod.forces(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
    sel = np.array([0, 1, 2, 77, 1500, 2999])
    fs = oracle_mod.forces_on(sel, s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
    assert np.allclose(fs, f[sel], rtol=1e-10, atol=1e-9)


# ---- cell-grid evaluation against the all-pairs sum -----------------------------------
def _cells_vs_pairs(o, s, **kw):
    p = o.params(**kw)
    args = (s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
    e0, f0, v0, a0 = o.forces(*args, energy_abs=True)
    e1, f1, v1, a1 = o.forces_cells(*args, energy_abs=True)
    scale = np.abs(f0).max()
    assert np.abs(f1 - f0).max() <= 1e-12 * scale
    assert np.allclose(e1, e0, rtol=1e-12, atol=1e-12 * a0.max())
    assert np.allclose(v1, v0, rtol=1e-11, atol=1e-12 * np.abs(v0).max())
    assert np.allclose(a1, a0, rtol=1e-12)
    return e0


def test_cells_equal_all_pairs_water3k(oracle_mod, sys3k):
    # 3.104 nm box, rc 1.0: three cells per axis, every cell a neighbour of every other
    _cells_vs_pairs(oracle_mod, sys3k, coulomb="rf", rc=1.0)
    _cells_vs_pairs(oracle_mod, sys3k, coulomb="ewald", rc=1.0, beta=3.12)


def test_cells_equal_all_pairs_diff24k(oracle_mod, sys24k):
    _cells_vs_pairs(oracle_mod, sys24k, coulomb="rf", rc=1.0)      # six cells per axis


def test_cells_equal_all_pairs_water96k(oracle_mod):
    from paper_2006_09167_amd import systems
    s = systems.config_system("water96k_ewald")
    _cells_vs_pairs(oracle_mod, s, coulomb="ewald", rc=1.0, beta=3.12)


def test_cells_unwrapped_coordinates_and_small_boxes(oracle_mod):
    s = small_random_system(61, 400, [3.5, 4.1, 3.2], n_types=3)
    # move atoms by whole and partial box multiples: minimum images are unchanged
    rng = np.random.default_rng(2)
    x = s.x + (rng.integers(-3, 4, s.x.shape) * s.box).astype(np.float32)
    s2 = System(**{**s.__dict__, "x": x.astype(np.float32)})
    _cells_vs_pairs(oracle_mod, s2, coulomb="ewald", rc=1.1, beta=3.0, modifier="none")
    # below three cells per axis the all-pairs sum is used
    t = small_random_system(62, 120, 2.5)
    _cells_vs_pairs(oracle_mod, t, coulomb="rf", rc=1.0)
