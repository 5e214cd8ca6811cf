"""Verlet buffer estimate (Sec. V.B) and the coverage of a list by M x N sub-cluster pairs,
in plain numpy / scipy.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg
of the benchmark; the product library never uses it.

Coverage: coverage(...)[l, k] = number of atom pairs closer than radii[k] that lie in an
M x N sub-cluster pair (sub-clusters as in census.py) holding an atom pair closer than
radii[l] -- the pairs within radii[k] that an M x N list at radii[l] contains.

Drift (the paper names the inputs: masses, temperature, pair potentials and the cluster
setup with its implicit buffer; the model below is the reading this oracle takes of it):
  * over a list age t an atom of mass m moves by a Gaussian of variance k_B T t^2 / m per
    axis (free flight; m is the mass that carries the atom: its own, or that of the rigid
    unit it belongs to), so the distance of a pair of classes a, b changes by a Gaussian
    of variance sigma^2 = var_a + var_b;
  * an atom constrained at distance d to a partner about which it rotates (the refinement
    for constrained atoms of Sec. V.B) adds the displacement of a free rotor: its bond
    direction u turns at a constant angular velocity w perpendicular to u, a 2-d Gaussian
    of variance k_B T / (m_own d^2) per component (equipartition of the rotational kinetic
    energy m_own d^2 |w|^2 / 2), by the angle theta = |w| t; the displacement d (u(t) - u(0))
    has the squared length 2 d^2 (1 - cos theta), a third of it along any fixed axis, and
    with |w| Rayleigh distributed E[cos theta] = 1 - sqrt(2) s D(s / sqrt(2)), s^2 =
    k_B T t^2 / (m_own d^2), D Dawson's integral; the per-axis variance
    (2/3) d^2 sqrt(2) s D(s / sqrt(2)) grows as (2/3) k_B T t^2 / m_own at first and
    levels off at (2/3) d^2, and it enters sigma^2 as a Gaussian of that variance;
  * beyond the list radius partners of class b have density N_b / V;
  * a pair not in the list at r0 >= r_l that ends at r < r_c misses |V_ab(r)|; a list holds
    the fraction 1 - U(r0) of the pairs at r0 (U = 1 for a particle list, from a coverage
    table for a cluster list);
  * E = (1/N) (1/2) sum_a sum_b N_a (N_b / V) int_{r_l} 4 pi r0^2 U(r0)
                                             int^{r_c} |V_ab(r)| g_sigma(r - r0) dr dr0,
    at the oldest use of the list t = (steps - 1) dt, and drift = E / (steps dt).
The integrals are evaluated by scipy's adaptive quadrature over 10 sigma windows; the
inner one starts no lower than r_c / 2 (missed pairs end near the cut-off; below that the
free-flight expectation of |V| would be dominated by atomic overlaps, and with the r^-12
core it has no finite value at all).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import dawsn, erfc

from . import cluster_pairs, radius_sq_f32, split_key
from .census import pair_r2

KB = 0.0083144626181532        # Boltzmann constant, kJ mol^-1 K^-1
WINDOW = 10.0                  # Gaussian widths integrated on each side


# ---------------------------------------------------------------------------------------
# Coverage of a list by M x N sub-cluster pairs.
# ---------------------------------------------------------------------------------------
def coverage(slot_atom, w, box, radii, M: int, N: int, chunk: int = 1 << 15, ci_lo: int = 0,
             ci_hi=None) -> np.ndarray:
    """[K, K] counts (module docstring), over the triples whose i-cluster lies in
    [ci_lo, ci_hi) (all by default).  Per cluster triple within the largest radius: the
    smallest r2 of each M x N sub-cluster pair decides the radii at which it is held, each
    atom pair's own r2 the radii it lies within; a 2-d count over (first held radius, first
    radius the pair is within), summed cumulatively over both indices."""
    radii = np.asarray(radii, dtype=np.float64).reshape(-1)
    K = radii.size
    R2 = np.array([radius_sq_f32(r) for r in radii], dtype=np.float32)
    order = np.argsort(R2, kind="stable")
    R2s = R2[order]
    slot_atom = np.asarray(slot_atom)
    n_cl = slot_atom.size // 8
    hist = np.zeros((K + 1, K + 1), dtype=np.int64)
    keys = cluster_pairs(slot_atom, w, box, float(radii.max()), ci_lo, ci_hi)
    ci, cj, code = split_key(keys, n_cl)
    for p0 in range(0, keys.size, chunk):
        r2 = pair_r2(slot_atom, w, box, ci[p0:p0 + chunk], cj[p0:p0 + chunk],
                     code[p0:p0 + chunk])
        P = r2.shape[0]
        sub = r2.reshape(P, 8 // M, M, 8 // N, N).min(axis=(2, 4), keepdims=True)
        sub = np.broadcast_to(sub, (P, 8 // M, M, 8 // N, N)).reshape(P, 8, 8)
        # first sorted radius index with r2 < R2 (K: none)
        k_own = np.searchsorted(R2s, r2.ravel(), side="right")
        k_sub = np.searchsorted(R2s, sub.ravel(), side="right")
        np.add.at(hist, (k_sub, k_own), 1)
    cum = hist[:K, :K].cumsum(axis=0).cumsum(axis=1)
    out = np.empty((K, K), dtype=np.int64)
    out[np.ix_(order, order)] = cum
    return out


def uncovered_fraction(cov_radii, covered, l: int):
    """U(r0) for a list at cov_radii[l]: in the shell between cov_radii[k-1] and
    cov_radii[k] (k > l) one minus the fraction of its atom pairs the list holds; 1 beyond
    the table (or in an empty shell)."""
    R = np.asarray(cov_radii, dtype=np.float64)
    C = np.asarray(covered, dtype=np.int64)

    def U(r0):
        k = int(np.searchsorted(R, r0, side="right"))     # r0 in [R[k-1], R[k])
        if k >= R.size or k <= l:
            return 1.0
        total = C[k, k] - C[k - 1, k - 1]
        held = C[l, k] - C[l, k - 1]
        return 1.0 - held / total if total > 0 else 1.0
    U.breaks = R
    return U


# ---------------------------------------------------------------------------------------
# Drift.
# ---------------------------------------------------------------------------------------
def pair_potential(r, c6, c12, qq, p) -> float:
    """LJ plus the electrostatics of the kernels, with the potential-shift modifier when
    set, at r < r_c (p: oracle.params or a dict with the same fields)."""
    g = (lambda k: getattr(p, k)) if not isinstance(p, dict) else p.__getitem__
    rc, coul, shift = g("rc"), g("coulomb"), g("modifier") == 1
    f = g("epsfac") / g("eps_r")
    v = c12 / r ** 12 - c6 / r ** 6
    if shift:
        v -= c12 / rc ** 12 - c6 / rc ** 6
    if coul == 0:                                            # reaction field
        eps_r, eps_rf = g("eps_r"), g("eps_rf")
        krf = 1.0 / (2 * rc ** 3) if math.isinf(eps_rf) else \
            (eps_rf - eps_r) / ((2 * eps_rf + eps_r) * rc ** 3)
        crf = 1.0 / rc + krf * rc ** 2
        v += f * qq * (1.0 / r + krf * r * r - crf)
    elif coul == 1:                                          # Ewald real space
        beta = g("beta")
        v += f * qq * (erfc(beta * r) / r - (erfc(beta * rc) / rc if shift else 0.0))
    return v


def missed_energy_pair(V, sigma: float, rc: float, r_list: float, U=None) -> float:
    """int_{r_l} 4 pi r0^2 U(r0) int^{r_c} |V(r)| g_sigma(r - r0) dr dr0 for one class pair."""
    if sigma <= 0.0:
        return 0.0
    lo = max(rc - WINDOW * sigma, 0.5 * rc)        # missed pairs end near the cut-off
    hi = r_list + WINDOW * sigma

    def inner(r0):
        f = lambda r: abs(V(r)) * math.exp(-0.5 * ((r - r0) / sigma) ** 2)
        val, _ = integrate.quad(f, lo, rc, limit=400, epsabs=0.0, epsrel=1e-10)
        return val / (math.sqrt(2 * math.pi) * sigma)

    pts = None
    if U is not None and getattr(U, "breaks", None) is not None:
        pts = [float(b) for b in U.breaks if r_list < b < hi] or None
    Uf = U if U is not None else (lambda r0: 1.0)
    val, _ = integrate.quad(lambda r0: 4 * math.pi * r0 * r0 * Uf(r0) * inner(r0), r_list, hi,
                            points=pts, limit=400, epsabs=0.0, epsrel=1e-9)
    return val


def displacement_var(kT: float, t: float, mass: float, rot_len: float = 0.0,
                     rot_mass: float = 0.0) -> float:
    """Per-axis variance of an atom's displacement over the time t (module docstring):
    free flight with the mass that carries it, plus, for rot_len > 0, the rotation about
    its constraint partner with its own mass rot_mass."""
    v = kT * t * t / mass
    if rot_len > 0.0:
        s = t * math.sqrt(kT / (rot_mass * rot_len * rot_len))
        v += (2.0 / 3.0) * rot_len * rot_len * math.sqrt(2.0) * s * dawsn(s / math.sqrt(2.0))
    return v


def missed_energy(p, classes: dict, lj, volume: float, temperature: float, dt: float,
                  steps: int, r_list: float, U=None) -> float:
    """Missed energy per atom after (steps - 1) dt (module docstring)."""
    t = (steps - 1) * dt
    count = np.asarray(classes["count"], dtype=np.float64)
    mass = np.asarray(classes["mass"], dtype=np.float64)
    charge = np.asarray(classes["charge"], dtype=np.float64)
    typ = np.asarray(classes["type"], dtype=np.int64)
    rot_len = np.asarray(classes.get("rot_len", np.zeros(count.size)), dtype=np.float64)
    rot_mass = np.asarray(classes.get("rot_mass", np.zeros(count.size)), dtype=np.float64)
    lj = np.asarray(lj, dtype=np.float64)
    N = count.sum()
    if t <= 0.0 or N == 0:
        return 0.0
    rc = float(p.rc) if not isinstance(p, dict) else p["rc"]
    kT = KB * temperature
    var = [displacement_var(kT, t, mass[a], rot_len[a], rot_mass[a]) for a in range(count.size)]
    total = 0.0
    for a in range(count.size):
        for b in range(count.size):
            if count[a] == 0 or count[b] == 0:
                continue
            sigma = math.sqrt(var[a] + var[b])
            c6, c12 = lj[typ[a], typ[b], 0], lj[typ[a], typ[b], 1]
            qq = charge[a] * charge[b]
            V = lambda r, c6=c6, c12=c12, qq=qq: pair_potential(r, c6, c12, qq, p)
            total += 0.5 * count[a] * (count[b] / volume) * missed_energy_pair(V, sigma, rc,
                                                                            r_list, U)
    return total / N


def drift(p, classes, lj, volume, temperature, dt, steps, r_list, U=None) -> float:
    """Energy drift per atom (kJ mol^-1 ps^-1) of a list at r_list used for `steps` steps."""
    if steps * dt <= 0:
        return 0.0
    return missed_energy(p, classes, lj, volume, temperature, dt, steps, r_list, U) / (steps * dt)
