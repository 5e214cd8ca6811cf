"""Pins of the oracle's Verlet buffer estimate and list coverage (Sec. V.B):
 * coverage against an enumeration written from the definition on tiny random systems, the
   particle-list identity (1 x 1 coverage is the pair count at the smaller radius) and the
   census's pair counts on the diagonal;
 * the missed-energy integral of a step potential against its closed form (Gaussian tail
   moments), and of the water potentials with a stepped uncovered fraction against a Monte
   Carlo estimate of the same definition;
 * invariants: sigma depends on T t^2 only, the drift falls with the list radius, a list
   used once has none;
and the parity of the library's host-side estimate (nb_buffer_drift / nb_buffer_estimate,
no device needed) with the oracle's."""
import itertools
import math

import numpy as np
import pytest
from scipy.special import erfc

from conftest import small_random_system

WATER_CLASSES = dict(count=[1000, 2000], mass=[18.015, 18.015], charge=[-0.82, 0.41],
                     type=[0, 1])


def grid_of(o, s):
    return o.grid_spec.build_grid(s.x, s.box[None], np.array([0, s.n]))


def coverage_by_definition(slot_atom, w, box, radii, M, N):
    L = np.asarray(box, np.float32)
    n_cl = slot_atom.size // 8
    R2 = [np.float32(np.float64(np.float32(r)) ** 2) for r in radii]
    K = len(radii)
    out = np.zeros((K, K), np.int64)
    for ci in range(n_cl):
        for cj in range(ci, n_cl):
            for s in itertools.product((-1, 0, 1), repeat=3):
                if ci == cj and s != (0, 0, 0) and not s > (0, 0, 0):
                    continue
                r2 = np.full((8, 8), np.inf, np.float32)
                for p in range(8):
                    a = slot_atom[8 * ci + p]
                    for q in range(8):
                        b = slot_atom[8 * cj + q]
                        if a < 0 or b < 0 or (ci == cj and s == (0, 0, 0) and q <= p):
                            continue
                        acc = np.float32(0)
                        for k in range(3):
                            xa = w[a, k] - L[k] if s[k] > 0 else w[a, k]
                            xb = w[b, k] - L[k] if s[k] < 0 else w[b, k]
                            d = np.float32(np.float32(xa) - np.float32(xb))
                            acc = np.float32(acc + np.float32(d * d))
                        r2[p, q] = acc
                for p in range(8):
                    for q in range(8):
                        sub = r2[(p // M) * M:(p // M + 1) * M, (q // N) * N:(q // N + 1) * N]
                        for l in range(K):
                            if not np.any(sub < R2[l]):
                                continue
                            for k in range(K):
                                if r2[p, q] < R2[k]:
                                    out[l, k] += 1
    return out


@pytest.mark.parametrize("seed,n,box,radii,M,N", [(31, 70, 2.05, [0.5, 0.8, 1.0], 8, 8),
                                                   (32, 90, 2.3, [1.0, 0.4, 0.7], 8, 4),
                                                   (33, 60, 2.2, [0.6, 0.9], 2, 4)])
def test_coverage_matches_definition(oracle_mod, seed, n, box, radii, M, N):
    s = small_random_system(seed, n, box)
    g = grid_of(oracle_mod, s)
    got = oracle_mod.buffer.coverage(g["slot_atom"], g["w"], s.box, radii, M, N)
    ref = coverage_by_definition(g["slot_atom"], g["w"], s.box, radii, M, N)
    assert np.array_equal(got, ref)


def test_coverage_identities(oracle_mod, sys3k):
    s = sys3k
    g = grid_of(oracle_mod, s)
    radii = [0.9, 0.95, 1.0, 1.05, 1.1, 1.2]
    pairs = oracle_mod.census.census(g["slot_atom"], g["w"], s.box, radii)[0, 0]
    one = oracle_mod.buffer.coverage(g["slot_atom"], g["w"], s.box, radii, 1, 1)
    K = len(radii)
    assert all(one[l, k] == pairs[min(l, k)] for l in range(K) for k in range(K))
    big = oracle_mod.buffer.coverage(g["slot_atom"], g["w"], s.box, radii, 8, 8)
    assert np.array_equal(np.diag(big), pairs)
    # a cluster list holds pairs beyond its radius, more with larger radius and cluster
    assert all(big[l, k] > pairs[l] for l in range(K - 1) for k in range(l + 1, K))
    assert np.all(np.diff(big, axis=0) >= 0) and np.all(big >= one)


def q_tail(x):
    return 0.5 * erfc(x / math.sqrt(2.0))


def phi(x):
    return math.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def test_missed_energy_step_potential_closed_form(oracle_mod):
    """V = v0 inside r_c: the inner integral is v0 times the chance to end inside r_c,
    and the outer one reduces to Gaussian tail moments of (r_c + u)^2."""
    rc, v0 = 1.0, 2.5
    for sigma, b in ((0.03, 0.0), (0.05, 0.04), (0.02, 0.05), (0.04, 0.2)):
        got = oracle_mod.buffer.missed_energy_pair(lambda r: v0, sigma, rc, rc + b)
        be = b / sigma
        A0 = phi(be) - be * q_tail(be)
        A1 = 0.5 * ((1 - be * be) * q_tail(be) + be * phi(be))
        A2 = (-be ** 3 * q_tail(be) + (be * be + 2) * phi(be)) / 3.0
        ref = 4 * math.pi * v0 * (rc * rc * sigma * A0 + 2 * rc * sigma ** 2 * A1 +
                                  sigma ** 3 * A2)
        assert abs(got - ref) <= 1e-9 * ref, (sigma, b, got, ref)


def test_missed_energy_monte_carlo(oracle_mod, sys3k):
    """The same definition sampled: r0 from the r0^2 density on [r_l, r_l + 6 sigma], a
    Gaussian change of distance, |V| where the pair ends inside r_c, weighted by U."""
    p = oracle_mod.params("ewald", rc=0.9, beta=3.47)
    lj = sys3k.lj
    V = lambda r: oracle_mod.buffer.pair_potential(r, lj[0, 0, 0], lj[0, 0, 1], 0.82 * 0.82, p)
    rc, sigma, rl = float(p.rc), 0.04, float(p.rc) + 0.02
    R = np.array([rl, rl + 0.03, rl + 0.08])
    U = lambda r0: 0.3 if r0 < rl + 0.03 else (0.7 if r0 < rl + 0.08 else 1.0)
    U.breaks = R
    got = oracle_mod.buffer.missed_energy_pair(V, sigma, rc, rl, U)
    rng = np.random.default_rng(5)
    n = 2_000_000
    hi = rl + 6 * sigma
    r0 = (rl ** 3 + rng.uniform(0, 1, n) * (hi ** 3 - rl ** 3)) ** (1 / 3)
    rt = r0 + sigma * rng.normal(size=n)
    u = np.where(r0 < rl + 0.03, 0.3, np.where(r0 < rl + 0.08, 0.7, 1.0))
    inside = rt < rc
    vals = np.zeros(n)
    vals[inside] = np.abs(np.vectorize(V)(rt[inside])) * u[inside]
    shell = 4 * math.pi / 3 * (hi ** 3 - rl ** 3)
    est, se = shell * vals.mean(), shell * vals.std() / math.sqrt(n)
    assert abs(got - est) < 5 * se, (got, est, se)


def test_drift_invariants(oracle_mod, sys3k):
    p = oracle_mod.params("ewald", rc=0.9, beta=3.47)
    V = float(np.prod(sys3k.box))
    me = lambda T, dt, steps, rl: oracle_mod.buffer.missed_energy(
        p, WATER_CLASSES, sys3k.lj, V, T, dt, steps, rl)
    a, b = me(1200.0, 0.002, 21, 0.93), me(300.0, 0.004, 21, 0.93)   # T t^2 equal
    assert abs(a - b) <= 1e-9 * a
    d = [oracle_mod.buffer.drift(p, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, 40, 0.9 + x)
         for x in (0.0, 0.02, 0.05, 0.1)]
    assert all(d[i] > d[i + 1] for i in range(3)) and d[-1] >= 0.0
    assert oracle_mod.buffer.drift(p, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, 1, 0.9) == 0.0


def test_boltzmann_constant():
    import oracle
    assert abs(oracle.buffer.KB * 300.0 - 2.4943) < 1e-4            # k_B T at 300 K, kJ/mol


def test_drift_class_split_invariance(oracle_mod, sys3k):
    """Splitting a class into two identical halves leaves the missed energy unchanged (the
    pair weights N_a N_b / V sum to the same total)."""
    p = oracle_mod.params("rf", rc=1.0)
    V = float(np.prod(sys3k.box))
    one = dict(count=[3000], mass=[18.015], charge=[0.3], type=[0])
    two = dict(count=[1500, 1500], mass=[18.015, 18.015], charge=[0.3, 0.3], type=[0, 0])
    a = oracle_mod.buffer.missed_energy(p, one, sys3k.lj, V, 300.0, 0.002, 30, 1.02)
    b = oracle_mod.buffer.missed_energy(p, two, sys3k.lj, V, 300.0, 0.002, 30, 1.02)
    assert a > 0 and abs(a - b) <= 1e-8 * a


def test_missed_energy_against_simulated_displacements(oracle_mod):
    """A uniform gas of one class moved by Gaussian free-flight displacements in 3-d: the
    energy of the pairs that start at or beyond r_l and end inside r_c, summed directly, per
    atom, against the oracle's integral.  The oracle treats the change of distance as a 1-d
    Gaussian; in 3-d the sideways part lengthens pairs by about sigma^2 / r, a few percent
    of the result at sigma / r_c = 0.03, hence the 10 % bound."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(11)
    n, L = 20000, 6.0
    x0 = rng.uniform(0, L, (n, 3))
    T, m = 300.0, 18.0
    sig_atom = 0.02
    t = sig_atom / math.sqrt(oracle_mod.buffer.KB * T / m)
    x1 = x0 + rng.normal(0.0, sig_atom, (n, 3))
    c6, c12 = 2.6e-3, 2.6e-6
    p = dict(rc=0.9, coulomb=2, modifier=1, epsfac=138.935458, eps_r=1.0)
    rc, rl = 0.9, 0.9
    tree = cKDTree(x0, boxsize=L)
    pr = tree.query_pairs(rc + 8 * math.sqrt(2) * sig_atom, output_type="ndarray")
    d0 = x0[pr[:, 0]] - x0[pr[:, 1]]
    d0 -= L * np.round(d0 / L)
    d1 = d0 + (x1[pr[:, 0]] - x0[pr[:, 0]]) - (x1[pr[:, 1]] - x0[pr[:, 1]])
    r0, r1 = np.linalg.norm(d0, axis=1), np.linalg.norm(d1, axis=1)
    miss = (r0 >= rl) & (r1 < rc)
    V = lambda r: c12 / r ** 12 - c6 / r ** 6 - (c12 / rc ** 12 - c6 / rc ** 6)
    direct = np.abs(V(r1[miss])).sum() / n
    lj = np.array([[[c6, c12]]])
    got = oracle_mod.buffer.missed_energy(p, dict(count=[n], mass=[m], charge=[0.0], type=[0]),
                                          lj, L ** 3, T, t, 2, rl)
    assert miss.sum() > 10000
    assert abs(got - direct) <= 0.1 * direct, (got, direct)


# ---- the library's host-side estimate against the oracle -------------------------------
def lib_params(coulomb, rc, beta=0.0):
    from paper_2006_09167_amd import api
    return api.make_params(2, coulomb, rc=rc, beta=beta)


@pytest.mark.parametrize("coulomb,rc,beta", [("ewald", 0.9, 3.47), ("rf", 1.0, 0.0)])
def test_library_drift_matches_oracle(oracle_mod, sys3k, coulomb, rc, beta):
    from paper_2006_09167_amd import api
    V = float(np.prod(sys3k.box))
    po = oracle_mod.params(coulomb, rc=rc, beta=beta)
    pl = lib_params(coulomb, rc, beta)
    for steps, b in ((40, 0.0), (40, 0.03), (10, 0.01), (80, 0.08)):
        rl = float(np.float32(rc)) + b
        ref = oracle_mod.buffer.drift(po, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, steps, rl)
        got = api.buffer_drift(pl, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, steps, rl)
        assert abs(got - ref) <= 1e-6 * ref, (steps, b, got, ref)


def test_library_cluster_drift_and_estimate_match_oracle(oracle_mod, sys3k):
    """With a coverage table (oracle coverage of the 3k water box) for the 8 x 8 and 8 x 4
    setups; the library's estimate is the first tabulated radius the oracle accepts."""
    from paper_2006_09167_amd import api
    s = sys3k
    g = grid_of(oracle_mod, s)
    rc = 0.9
    radii = np.float32(rc) + np.float32(0.01) * np.arange(12, dtype=np.float32)
    radii = radii.astype(np.float32)
    V = float(np.prod(s.box))
    po = oracle_mod.params("ewald", rc=rc, beta=3.47)
    pl = lib_params("ewald", rc, 3.47)
    for M, N in ((8, 8), (8, 4)):
        cov = oracle_mod.buffer.coverage(g["slot_atom"], g["w"], s.box, radii, M, N)
        for l in (0, 2, 5):
            U = oracle_mod.buffer.uncovered_fraction(radii, cov, l)
            ref = oracle_mod.buffer.drift(po, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40,
                                          float(radii[l]), U)
            got = api.buffer_drift(pl, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40,
                                   float(radii[l]), coverage=(radii, cov))
            assert abs(got - ref) <= 1e-6 * ref, (M, N, l, got, ref)
            part = api.buffer_drift(pl, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40,
                                    float(radii[l]))
            assert got < part                          # the implicit buffer lowers the drift
        tol = 0.005
        r, d = api.buffer_estimate(pl, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40, tol,
                                   coverage=(radii, cov))
        l = int(np.flatnonzero(radii == np.float32(r))[0])
        drifts = [oracle_mod.buffer.drift(po, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40,
                                          float(radii[j]),
                                          oracle_mod.buffer.uncovered_fraction(radii, cov, j))
                  for j in range(l + 1)]
        assert drifts[l] <= tol * (1 + 1e-6) and all(x > tol for x in drifts[:l])
    # particle list: bisection to 1e-6 nm
    r, d = api.buffer_estimate(pl, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40, 0.005)
    assert oracle_mod.buffer.drift(po, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40, r) <= 0.005 * (1 + 1e-6)
    assert oracle_mod.buffer.drift(po, WATER_CLASSES, s.lj, V, 300.0, 0.002, 40, r - 2e-6) > 0.005


def test_library_buffer_degenerate_inputs(sys3k):
    """Zero temperature or a list used once: nothing moves, no drift, the radius is r_c."""
    from paper_2006_09167_amd import api
    pl = lib_params("ewald", 0.9, 3.47)
    V = float(np.prod(sys3k.box))
    assert api.buffer_drift(pl, WATER_CLASSES, sys3k.lj, V, 0.0, 0.002, 40, 0.9) == 0.0
    assert api.buffer_drift(pl, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, 1, 0.9) == 0.0
    assert api.buffer_drift(pl, WATER_CLASSES, sys3k.lj, V, 300.0, 0.0, 40, 0.9) == 0.0
    r, d = api.buffer_estimate(pl, WATER_CLASSES, sys3k.lj, V, 0.0, 0.002, 40)
    assert r == float(np.float32(0.9)) and d == 0.0
    empty = dict(count=[0, 0], mass=[18.0, 18.0], charge=[0.0, 0.0], type=[0, 1])
    assert api.buffer_drift(pl, empty, sys3k.lj, V, 300.0, 0.002, 40, 0.9) == 0.0


def test_library_buffer_argument_errors(sys3k):
    from paper_2006_09167_amd import api
    pl = lib_params("ewald", 0.9, 3.47)
    V = float(np.prod(sys3k.box))
    with pytest.raises(RuntimeError):
        api.buffer_drift(pl, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, 40, 0.8)   # < rc
    with pytest.raises(RuntimeError):
        api.buffer_drift(pl, dict(WATER_CLASSES, mass=[0.0, 1.0]), sys3k.lj, V, 300.0, 0.002,
                         40, 1.0)
    radii = np.array([0.9, 0.95], np.float32)
    with pytest.raises(RuntimeError):            # radius not in the coverage table
        api.buffer_drift(pl, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, 40, 0.93,
                         coverage=(radii, np.ones((2, 2), np.int64)))
    with pytest.raises(ValueError):              # class arrays of different lengths
        api.buffer_drift(pl, dict(WATER_CLASSES, mass=[18.0]), sys3k.lj, V, 300.0, 0.002, 40, 1.0)
    with pytest.raises(ValueError):              # table for the wrong number of types
        api.buffer_drift(pl, WATER_CLASSES, sys3k.lj[:1, :1], V, 300.0, 0.002, 40, 1.0)
    with pytest.raises(ValueError):              # coverage table not square in the radii
        api.buffer_drift(pl, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, 40, 0.9,
                         coverage=(radii, np.ones((2, 3), np.int64)))
    with pytest.raises(RuntimeError):            # tolerance not reached within the range
        api.buffer_estimate(pl, WATER_CLASSES, sys3k.lj, V, 300.0, 0.002, 40, 1e-30,
                            max_buffer=0.01)


def test_missed_energy_of_simulated_free_flight_on_water(oracle_mod, sys3k):
    """The model sampled on the 3k water box: each atom moves with one Maxwell velocity for
    mass 18.015 over t = 0.08 ps; every atom pair inside r_c at t whose 8 x 8 cluster pair at
    the build held no atom pair within r_l is missed (a 1 x 1 list misses the pairs that
    were themselves beyond r_l).  The |V| of the missed pairs per atom, summed directly,
    against the oracle's integral, with the coverage table of the same build for the
    cluster list.  The integral's 1-d radial model ignores the sideways lengthening of
    pairs, so it slightly overestimates (the 8 x 8 sample: ~0.8 of it)."""
    from scipy.spatial import cKDTree
    s = sys3k
    L = s.box.astype(np.float64)
    g = grid_of(oracle_mod, s)
    w = g["w"].astype(np.float64)
    slot_atom = g["slot_atom"]
    atom_slot = np.full(s.n, -1)
    atom_slot[slot_atom[slot_atom >= 0]] = np.flatnonzero(slot_atom >= 0)
    cl_of = atom_slot // 8
    members = slot_atom.reshape(-1, 8)
    radii = (np.float32(0.9) + np.float32(0.01) * np.arange(12, dtype=np.float32)).astype(np.float32)
    rc, l, T, t, m = 0.9, 2, 300.0, 0.08, 18.015
    rl = float(radii[l])
    p = oracle_mod.params("ewald", rc=rc, beta=3.47)
    rng = np.random.default_rng(3)
    x1 = w + rng.normal(0, math.sqrt(oracle_mod.buffer.KB * T / m), (s.n, 3)) * t
    pr = cKDTree(np.mod(x1, L), boxsize=L).query_pairs(rc, output_type="ndarray")
    d1 = x1[pr[:, 0]] - x1[pr[:, 1]]
    shift = np.round(d1 / L)
    r1 = np.linalg.norm(d1 - L * shift, axis=1)
    r0 = np.linalg.norm(w[pr[:, 0]] - w[pr[:, 1]] - L * shift, axis=1)
    A, B = members[cl_of[pr[:, 0]]], members[cl_of[pr[:, 1]]]
    xa = np.where(A[..., None] >= 0, w[np.maximum(A, 0)], np.nan)
    xb = np.where(B[..., None] >= 0, w[np.maximum(B, 0)], np.nan)
    dd = xa[:, :, None, :] - xb[:, None, :, :] - (L * shift)[:, None, None, :]
    rmin = np.nanmin(np.linalg.norm(dd, axis=3).reshape(len(pr), -1), axis=1)
    lj = s.lj
    V = np.vectorize(lambda r, a, b: oracle_mod.buffer.pair_potential(
        r, lj[s.type[a], s.type[b], 0], lj[s.type[a], s.type[b], 1],
        float(s.q[a]) * float(s.q[b]), p))
    direct = {}
    for name, miss in (("1x1", r0 >= rl), ("8x8", rmin >= rl)):
        assert miss.sum() > 500
        direct[name] = np.abs(V(r1[miss], pr[miss, 0], pr[miss, 1])).sum() / s.n
    n_o = int(np.sum(s.type == 0))
    cls = dict(count=[n_o, s.n - n_o], mass=[m, m], type=[0, 1],
               charge=[float(s.q[s.type == 0][0]), float(s.q[s.type == 1][0])])
    V_box = float(np.prod(L))
    cov = oracle_mod.buffer.coverage(g["slot_atom"], g["w"], s.box, radii, 8, 8)
    est = {"1x1": oracle_mod.buffer.missed_energy(p, cls, lj, V_box, T, t, 2, rl),
           "8x8": oracle_mod.buffer.missed_energy(
               p, cls, lj, V_box, T, t, 2, rl, oracle_mod.buffer.uncovered_fraction(radii, cov, l))}
    for name in ("1x1", "8x8"):
        assert 0.7 <= direct[name] / est[name] <= 1.1, (name, direct[name], est[name])
    assert est["8x8"] < 0.1 * est["1x1"]                # the implicit buffer matters


# ---- constrained atoms rotating about their partner -------------------------------------
ROTOR_CLASSES = dict(WATER_CLASSES, rot_len=[0.0, 0.1], rot_mass=[15.9994, 1.008])


def simulated_rotor_var(rng, n, kT, t, m, d):
    """Per-axis variance of d (u(t) - u(0)) for a free rotor, by simulation of the geometry:
    u(0) uniform on the sphere, angular velocity w perpendicular to u(0) with Gaussian
    components of variance kT / (m d^2) (equipartition of m d^2 |w|^2 / 2 over the two
    perpendicular axes), u turned about w by |w| t (Rodrigues' rotation)."""
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    g = rng.normal(0.0, math.sqrt(kT / (m * d * d)), (n, 3))
    w = g - np.sum(g * u, axis=1, keepdims=True) * u        # the part perpendicular to u
    om = np.linalg.norm(w, axis=1, keepdims=True)
    k = w / om
    th = om * t
    # Rodrigues with k perpendicular to u: u cos th + (k x u) sin th
    ut = u * np.cos(th) + np.cross(k, u) * np.sin(th)
    disp = d * (ut - u)
    return disp.var(axis=0).mean(), disp


@pytest.mark.parametrize("t", [0.005, 0.04, 0.078, 0.2, 1.0])
def test_rotor_variance_against_simulated_rotation(oracle_mod, t):
    """The closed form (2/3) d^2 sqrt(2) s D(s / sqrt(2)) against the variance of simulated
    free-rotor displacements of a hydrogen 0.1 nm from its partner, from the free-flight
    regime (t = 5 fs) to the saturated one (1 ps), within 4 standard errors."""
    rng = np.random.default_rng(5)
    kT = oracle_mod.buffer.KB * 300.0
    n = 400000
    sim, disp = simulated_rotor_var(rng, n, kT, t, 1.008, 0.1)
    got = oracle_mod.buffer.displacement_var(kT, t, 1e30, 0.1, 1.008)   # rotation only
    se = disp.reshape(-1).astype(np.float64).__pow__(2).std() / math.sqrt(3 * n)
    assert abs(got - sim) <= 4 * se + 1e-12, (t, got, sim, se)


def test_rotor_variance_limits(oracle_mod):
    """Small t: free flight of the atom's own mass along the two directions perpendicular to
    the bond, (2/3) k_B T t^2 / m; large t: the fixed (2/3) d^2 of a uniformly oriented bond
    vector; no rotation: k_B T t^2 / m of the carrying mass alone."""
    kT = oracle_mod.buffer.KB * 300.0
    m, d = 1.008, 0.1
    for t in (1e-5, 1e-4):
        v = oracle_mod.buffer.displacement_var(kT, t, 1e30, d, m)
        assert abs(v - (2 / 3) * kT * t * t / m) <= 1e-6 * v
    v = oracle_mod.buffer.displacement_var(kT, 1e3, 1e30, d, m)
    assert abs(v - (2 / 3) * d * d) <= 1e-4 * v
    v = oracle_mod.buffer.displacement_var(kT, 0.05, 18.015)
    assert abs(v - kT * 0.05 ** 2 / 18.015) <= 1e-15 * v
    # the translation of the carrying mass adds
    both = oracle_mod.buffer.displacement_var(kT, 0.05, 18.015, d, m)
    assert abs(both - (kT * 0.05 ** 2 / 18.015
                       + oracle_mod.buffer.displacement_var(kT, 0.05, 1e300, d, m))) <= 1e-12


def test_rotor_drift_between_rigid_and_free(oracle_mod, sys3k):
    """The rotor reading lies between a rigid molecule (hydrogen carried by the molecular
    mass alone) and free atoms (hydrogen moving freely in all three directions with its own
    mass) for a list used for 40 steps of 2 fs."""
    p = oracle_mod.params("ewald", rc=0.9, beta=3.47)
    V = float(np.prod(sys3k.box))
    free = dict(WATER_CLASSES, mass=[15.9994, 1.008])
    args = (p, None, sys3k.lj, V, 300.0, 0.002, 40, 0.95)
    d_rigid, d_rot, d_free = (oracle_mod.buffer.drift(p, cl, *args[2:])
                              for cl in (WATER_CLASSES, ROTOR_CLASSES, free))
    assert d_rigid < d_rot < d_free, (d_rigid, d_rot, d_free)


def test_library_rotor_drift_matches_oracle(oracle_mod, sys3k):
    """nb_buffer_drift with rotating classes (its own Dawson integral) against the oracle
    (scipy's dawsn), particle list, several list ages."""
    from paper_2006_09167_amd import api
    V = float(np.prod(sys3k.box))
    po = oracle_mod.params("ewald", rc=0.9, beta=3.47)
    pl = lib_params("ewald", 0.9, 3.47)
    for steps, b in ((2, 0.0), (40, 0.0), (40, 0.05), (100, 0.1), (400, 0.2)):
        rl = float(np.float32(0.9)) + b
        ref = oracle_mod.buffer.drift(po, ROTOR_CLASSES, sys3k.lj, V, 300.0, 0.002, steps, rl)
        got = api.buffer_drift(pl, ROTOR_CLASSES, sys3k.lj, V, 300.0, 0.002, steps, rl)
        assert abs(got - ref) <= 1e-6 * ref, (steps, b, got, ref)


def test_library_rotor_argument_errors(sys3k):
    from paper_2006_09167_amd import api
    V = float(np.prod(sys3k.box))
    pl = lib_params("ewald", 0.9, 3.47)
    for bad in (dict(ROTOR_CLASSES, rot_len=[0.0, -0.1]),
                dict(ROTOR_CLASSES, rot_mass=[15.9994, 0.0]),
                dict(ROTOR_CLASSES, rot_len=[0.0, float("nan")])):
        with pytest.raises(Exception):
            api.buffer_drift(pl, bad, sys3k.lj, V, 300.0, 0.002, 40, 0.95)
