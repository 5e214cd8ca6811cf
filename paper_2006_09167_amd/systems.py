"""Seeded synthetic inputs for the cluster-pair nonbonded path.

This module only builds input data: coordinates, charges, atom types, exclusion
lists, boxes and the per-type Lennard-Jones parameters of water-like boxes.  It
holds none of the pair-interaction arithmetic; both the HIP path and the FP64
oracle receive what it returns.

The paper measures its kernels on SPC/E water boxes and a Lennard-Jones argon
system (Sec. V.C, Figs. 6 and 7).  Those inputs are not available here, so the
boxes below are seeded stand-ins: argon on a jittered lattice at the paper's density
(argon_box), and water-like boxes with the same density (about 100 atoms/nm^3),
charge pattern and exclusion structure as three-site water:

* one O (q = -0.82 e, sigma = 0.3166 nm, epsilon = 0.65 kJ/mol) and two H
  (q = +0.41 e, no Lennard-Jones) per molecule;
* O on a jittered cubic lattice (uniform jitter of +-0.1 lattice spacings per
  axis), a seeded subset of lattice sites left vacant;
* each H 0.1 nm from its O, the first in a uniformly random direction, the
  second at 109.47 degrees from the first around a uniformly random azimuth;
* a molecule whose atoms come closer than a minimum distance to another
  molecule is re-oriented (at most 100 rounds);
* the three intramolecular pairs are excluded.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# Physical constants and model parameters (nm, kJ/mol, e).
EPSFAC = 138.935458          # 1/(4 pi eps0) in kJ mol^-1 nm e^-2
Q_O, Q_H = -0.82, 0.41
SIGMA_O, EPS_O = 0.3166, 0.65
OH_DIST = 0.1                # nm
HOH_ANGLE_DEG = 109.47


@dataclasses.dataclass
class System:
    """One periodic rectangular box of atoms (user order = molecule order)."""
    x: np.ndarray            # float32 [N,3] continuous (unwrapped) coordinates, nm
    q: np.ndarray            # float32 [N] charges, e
    type: np.ndarray         # int32 [N] LJ type index
    excl_ptr: np.ndarray     # int64 [N+1] CSR row pointers of excluded partners
    excl_idx: np.ndarray     # int32 [nnz] excluded partner atom indices (both directions)
    box: np.ndarray          # float32 [3] box edge lengths, nm
    sigma: np.ndarray        # float64 [T] per-type sigma, nm (0 = no LJ)
    eps: np.ndarray          # float64 [T] per-type epsilon, kJ/mol
    lj: np.ndarray           # float32 [T,T,2] (c6, c12) table from the combination rule
    redraws: int = 0         # number of molecule re-orientations made by the generator

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_types(self) -> int:
        return int(self.sigma.shape[0])


def lj_table_lorentz_berthelot(sigma: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """(c6, c12) per type pair: sigma_ij = (s_i+s_j)/2, eps_ij = sqrt(e_i e_j),
    c6 = 4 eps sigma^6, c12 = 4 eps sigma^12 (input preparation only)."""
    s = 0.5 * (sigma[:, None] + sigma[None, :])
    e = np.sqrt(eps[:, None] * eps[None, :])
    out = np.empty(s.shape + (2,), dtype=np.float64)
    out[..., 0] = 4.0 * e * s ** 6
    out[..., 1] = 4.0 * e * s ** 12
    return out.astype(np.float32)


# --------------------------------------------------------------------------------------
# Configurations of the workloads (sizes, cut-offs, list parameters, dynamics).
# --------------------------------------------------------------------------------------
CONFIGS: Dict[str, dict] = {
    # 1,000 molecules, 10^3 lattice, 3.104 nm box; reaction field with eps_rf = inf;
    # one evaluation, so the list needs no buffer.
    "water3k_rf": dict(n_mol=1000, k=10, box=3.104, coulomb="rf", eps_rf=math.inf,
                       rc=1.0, rlist=1.0, rinner=1.0, nstlist=1, nstprune=1,
                       steps=1, seed=1, min_contact=0.15),
    # 32,000 molecules on a 32^3 lattice with 768 vacancies, 9.86 nm box; Ewald real space
    # with beta = 3.12/nm; outer list 1.1 nm rebuilt every 100 steps, inner list 1.04 nm
    # pruned in 4 rolling parts; Gaussian displacements of 0.002 nm per step.
    "water96k_ewald": dict(n_mol=32000, k=32, box=9.86, coulomb="ewald", beta=3.12,
                           rc=1.0, rlist=1.1, rinner=1.04, nstlist=100, nstprune=4,
                           steps=500, sigma_step=0.002, seed=2, min_contact=0.15),
    # 500,000 molecules on an 80^3 lattice with 12,000 vacancies, 24.7 nm box.
    "water1500k_ewald": dict(n_mol=500000, k=80, box=24.7, coulomb="ewald", beta=2.60,
                             rc=1.2, rlist=1.3, rinner=1.24, nstlist=80, nstprune=4,
                             steps=200, sigma_step=0.002, seed=3, min_contact=0.15),
    # 8,000 molecules, 20^3 lattice, 4 LJ types on every atom, random neutral charges.
    "diff24k_rf": dict(n_mol=8000, k=20, box=6.2145, coulomb="rf", eps_rf=math.inf,
                       rc=1.0, rlist=1.0, rinner=1.0, nstlist=1, nstprune=1,
                       steps=1, seed=5, min_contact=0.20, n_types=4),
}

ENSEMBLE = dict(n_replicas=256, n_min=3000, n_max=24000, density=100.0, coulomb="rf",
                eps_rf=math.inf, rc=0.9, rlist=1.0, rinner=0.94, nstlist=100, nstprune=4,
                steps=100, sigma_step=0.002, seed=4, min_contact=0.15)


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def _orient(rng: np.random.Generator, n: int) -> np.ndarray:
    """H offsets [n,2,3] for n molecules: OH_DIST from O at the HOH angle."""
    u1 = _unit_vectors(rng, n)
    r = _unit_vectors(rng, n)
    w = r - np.sum(r * u1, axis=1, keepdims=True) * u1
    norm = np.linalg.norm(w, axis=1, keepdims=True)
    bad = norm[:, 0] < 1e-6
    while np.any(bad):                       # degenerate draw: redraw the reference vector
        r[bad] = _unit_vectors(rng, int(bad.sum()))
        w = r - np.sum(r * u1, axis=1, keepdims=True) * u1
        norm = np.linalg.norm(w, axis=1, keepdims=True)
        bad = norm[:, 0] < 1e-6
    w /= norm
    th = math.radians(HOH_ANGLE_DEG)
    u2 = math.cos(th) * u1 + math.sin(th) * w
    return OH_DIST * np.stack([u1, u2], axis=1)


def _wrapped_tree(x: np.ndarray, box: float):
    from scipy.spatial import cKDTree
    xw = np.mod(x.astype(np.float64), box)
    xw[xw >= box] = 0.0
    return cKDTree(xw, boxsize=box), xw


def _close_molecules(tree, xw: np.ndarray, mol: np.ndarray, dmin: float,
                     changed: Optional[np.ndarray] = None) -> np.ndarray:
    """Molecules with an atom closer than dmin to an atom of another molecule
    (periodic); the higher-numbered molecule of each close pair is returned.

    With ``changed`` (molecules moved since the last call, which returned exactly
    them), only pairs with an atom of a changed molecule are examined: every other
    pair kept its distance and was not close at that call, or the higher molecule
    of the pair would have been returned and changed."""
    if changed is None:
        pairs = tree.query_pairs(dmin, output_type="ndarray")
        if pairs.size == 0:
            return np.zeros(0, dtype=np.int64)
        a, b = pairs[:, 0], pairs[:, 1]
    else:
        atoms = (3 * changed[:, None] + np.arange(3)[None, :]).reshape(-1)
        hits = tree.query_ball_point(xw[atoms], dmin)
        cnt = np.fromiter((len(h) for h in hits), dtype=np.int64, count=len(hits))
        if cnt.sum() == 0:
            return np.zeros(0, dtype=np.int64)
        a = np.repeat(atoms, cnt)
        b = np.concatenate([np.asarray(h, dtype=np.int64) for h in hits if len(h)])
    ma, mb = mol[a], mol[b]
    inter = ma != mb
    return np.unique(np.maximum(ma[inter], mb[inter]))


def _best_orientation(rng: np.random.Generator, tree, x: np.ndarray, o: np.ndarray,
                      mol: np.ndarray, bad: np.ndarray, box: float,
                      n_try: int = 16) -> np.ndarray:
    """For each listed molecule, the H offsets (out of n_try seeded draws) whose H
    atoms keep the largest distance to the atoms of all other molecules (tree: the
    periodic KD-tree of the current wrapped coordinates x)."""
    nb = bad.size
    cand = np.stack([_orient(rng, nb) for _ in range(n_try)], axis=1)      # [nb, n_try, 2, 3]
    hpos = o[bad][:, None, None, :] + cand                                   # [nb, n_try, 2, 3]
    hw = np.mod(hpos.reshape(-1, 3), box)
    hw[hw >= box] = 0.0
    d, idx = tree.query(hw, k=4)
    own = mol[np.minimum(idx, x.shape[0] - 1)] == np.repeat(bad, n_try * 2)[:, None]
    d = np.where(own, np.inf, d).min(axis=1).reshape(nb, n_try, 2).min(axis=2)
    best = np.argmax(d, axis=1)
    return cand[np.arange(nb), best]


def water_box(n_mol: int, k: int, box: float, seed: int, min_contact: float = 0.15,
              n_types: Optional[int] = None) -> System:
    """A water-like box of n_mol three-site molecules on a k^3 jittered lattice.

    With ``n_types`` set, every atom instead gets one of ``n_types`` LJ types drawn
    uniformly (sigma ~ U[0.25, 0.40] nm, eps ~ U[0.1, 1.0] kJ/mol per type) and a
    charge ~ N(0, 0.4^2) made neutral by subtracting the mean.
    """
    n_sites = k ** 3
    if n_mol > n_sites:
        raise ValueError("more molecules than lattice sites")
    ss = np.random.SeedSequence(seed)
    r_lat, r_jit, r_ori, r_typ = [np.random.default_rng(s) for s in ss.spawn(4)]
    a = box / k
    sites = np.arange(n_sites)
    if n_mol < n_sites:
        vac = r_lat.choice(n_sites, size=n_sites - n_mol, replace=False)
        keep = np.ones(n_sites, dtype=bool)
        keep[vac] = False
        sites = sites[keep]
    ix, iy, iz = sites // (k * k), (sites // k) % k, sites % k
    o = (np.stack([ix, iy, iz], axis=1) + 0.5) * a
    o = o + r_jit.uniform(-0.1 * a, 0.1 * a, size=o.shape)
    h = _orient(r_ori, n_mol)
    mol = np.repeat(np.arange(n_mol), 3)

    def assemble(o_, h_):
        xx = np.empty((n_mol, 3, 3), dtype=np.float64)
        xx[:, 0] = o_
        xx[:, 1] = o_ + h_[:, 0]
        xx[:, 2] = o_ + h_[:, 1]
        return xx.reshape(-1, 3)

    x = assemble(o, h)
    redraws = 0
    bad = None
    for _ in range(100):
        tree, xw = _wrapped_tree(x, box)
        bad = _close_molecules(tree, xw, mol, min_contact, bad)
        if bad.size == 0:
            break
        redraws += int(bad.size)
        h[bad] = _best_orientation(r_ori, tree, x, o, mol, bad, box)
        x = assemble(o, h)

    n = 3 * n_mol
    if n_types is None:
        q = np.tile(np.array([Q_O, Q_H, Q_H]), n_mol)
        typ = np.tile(np.array([0, 1, 1], dtype=np.int32), n_mol)
        sigma = np.array([SIGMA_O, 0.0])
        eps = np.array([EPS_O, 0.0])
    else:
        sigma = r_typ.uniform(0.25, 0.40, size=n_types)
        eps = r_typ.uniform(0.1, 1.0, size=n_types)
        typ = r_typ.integers(0, n_types, size=n).astype(np.int32)
        q = r_typ.normal(0.0, 0.4, size=n)
        q = q - q.mean()

    # Intramolecular exclusions, both directions, partners in ascending order.
    base = (np.arange(n) // 3) * 3
    partners = np.stack([base, base + 1, base + 2], axis=1)
    partners = partners[partners != np.arange(n)[:, None]].reshape(n, 2)
    excl_ptr = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    excl_idx = partners.reshape(-1).astype(np.int32)

    return System(x=x.astype(np.float32), q=q.astype(np.float32), type=typ,
                  excl_ptr=excl_ptr, excl_idx=excl_idx,
                  box=np.full(3, box, dtype=np.float32),
                  sigma=sigma, eps=eps, lj=lj_table_lorentz_berthelot(sigma, eps),
                  redraws=redraws)


# Lennard-Jones argon for the kernel-throughput sweep of the paper's Fig. 6: 157k atoms
# at 26 atoms/nm^3 with sigma = 0.3345 nm (the paper gives no epsilon; 0.996 kJ/mol is the
# usual argon value and does not change the work).  The x axis of the figure is the number
# of particles in the half cut-off sphere, n_half = (2/3) pi rc^3 rho; the sweep takes the
# cut-off for each n_half below, the outer list 0.1 nm beyond it and no rolling prune.
ARGON = dict(k=54, density=26.0, sigma=0.3345, eps=0.996, seed=2606, jitter=0.1,
             n_half=(50, 100, 200, 400, 800, 1600, 3000), buffer=0.1)


def argon_cutoff(n_half: float, density: float = ARGON["density"]) -> float:
    """Cut-off (nm) that puts n_half particles in the half cut-off sphere."""
    return (3.0 * n_half / (2.0 * math.pi * density)) ** (1.0 / 3.0)


def argon_box(k: int = ARGON["k"], density: float = ARGON["density"], seed: int = ARGON["seed"],
              jitter: float = ARGON["jitter"]) -> System:
    """k^3 argon atoms on a cubic lattice of spacing density^(-1/3), each displaced
    uniformly by up to +-jitter lattice spacings per axis; one LJ type, no charges and
    no exclusions."""
    a = density ** (-1.0 / 3.0)
    box = k * a
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    g = np.stack(np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij"),
                 -1).reshape(-1, 3).astype(np.float64)
    x = (g + 0.5 + rng.uniform(-jitter, jitter, size=g.shape)) * a
    n = x.shape[0]
    sigma = np.array([ARGON["sigma"]])
    eps = np.array([ARGON["eps"]])
    return System(x=x.astype(np.float32), q=np.zeros(n, np.float32), type=np.zeros(n, np.int32),
                  excl_ptr=np.zeros(n + 1, np.int64), excl_idx=np.zeros(0, np.int32),
                  box=np.full(3, box, dtype=np.float32), sigma=sigma, eps=eps,
                  lj=lj_table_lorentz_berthelot(sigma, eps))


def config_system(name: str) -> System:
    c = CONFIGS[name]
    return water_box(c["n_mol"], c["k"], c["box"], c["seed"], c["min_contact"],
                     c.get("n_types"))


def ensemble_sizes(seed: int = ENSEMBLE["seed"], n_replicas: int = ENSEMBLE["n_replicas"],
                   n_min: int = ENSEMBLE["n_min"], n_max: int = ENSEMBLE["n_max"]) -> np.ndarray:
    """Replica atom counts: log-uniform in [n_min, n_max], rounded to whole molecules."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    n = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_replicas))
    return (3 * np.round(n / 3.0)).astype(np.int64)


def ensemble_systems(seed: int = ENSEMBLE["seed"], n_replicas: int = ENSEMBLE["n_replicas"],
                     density: float = ENSEMBLE["density"]) -> List[System]:
    """Independent water-like replicas of uneven size at the given atom density."""
    sizes = ensemble_sizes(seed, n_replicas)
    out = []
    for r, n_atoms in enumerate(sizes):
        n_mol = int(n_atoms) // 3
        box = (n_atoms / density) ** (1.0 / 3.0)
        k = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
        out.append(water_box(n_mol, k, box, seed * 100003 + r, ENSEMBLE["min_contact"]))
    return out


def concat_systems(systems: List[System]) -> dict:
    """Concatenate replicas into one atom array with per-system offsets (host data)."""
    offs = np.zeros(len(systems) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([s.n for s in systems])
    x = np.concatenate([s.x for s in systems])
    q = np.concatenate([s.q for s in systems])
    typ = np.concatenate([s.type for s in systems])
    ptrs, idxs, base_nnz = [np.zeros(1, dtype=np.int64)], [], 0
    for s, o in zip(systems, offs[:-1]):
        ptrs.append(s.excl_ptr[1:] + base_nnz)
        idxs.append(s.excl_idx + np.int32(o))
        base_nnz += int(s.excl_ptr[-1])
    boxes = np.stack([s.box for s in systems]).astype(np.float32)
    return dict(x=x, q=q, type=typ, excl_ptr=np.concatenate(ptrs),
                excl_idx=np.concatenate(idxs).astype(np.int32), boxes=boxes, offsets=offs)


def displacement(rng: np.random.Generator, n: int, sigma: float) -> np.ndarray:
    """One step of Gaussian displacements (float32 [n,3])."""
    return rng.normal(0.0, sigma, size=(n, 3)).astype(np.float32)
