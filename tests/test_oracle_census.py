"""Pins of the oracle's work-efficiency census (Sec. V.B, Fig. 5):
 * an enumeration written straight from the definition, over every cluster triple and
   slot pair, on tiny random systems (sub-cluster grouping, the self-cluster triangle,
   canonical shifts, M against N);
 * the atom-pair count against a double-precision periodic k-d tree (scipy), bracketed
   by the k-d tree's counts one part in 5e5 either side of the radius;
 * the atom-pair count of a uniform random gas in a periodic box against its closed form
   C(n, 2) (4 pi R^3 / 3) / V (on a torus the pair events are pairwise independent, so the
   count has variance C(n, 2) p (1 - p));
 * the 8 x 8 count against the list oracle's cluster-pair set;
 * inclusions between sub-cluster sizes and radii."""
import itertools

import numpy as np
import pytest
from scipy.spatial import cKDTree

from conftest import small_random_system


def grid_of(o, x, box):
    return o.grid_spec.build_grid(np.asarray(x, np.float32), np.asarray(box, np.float32)[None],
                                  np.array([0, len(x)]))


def census_by_definition(slot_atom, w, box, radii):
    """Every canonical (ci <= cj, shift) and every counted slot pair in it, pair by pair:
    the set of (i-sub-cluster, j-sub-cluster, shift) holding a pair inside each radius."""
    sizes = (1, 2, 4, 8)
    L = np.asarray(box, np.float32)
    n_cl = slot_atom.size // 8
    held = {(M, N, k): set() for M in sizes for N in sizes for k in range(len(radii))}
    R2 = [np.float32(np.float64(np.float32(r)) ** 2) for r in radii]
    for ci in range(n_cl):
        for cj in range(ci, n_cl):
            for s in itertools.product((-1, 0, 1), repeat=3):
                if ci == cj and s != (0, 0, 0) and not s > (0, 0, 0):
                    continue
                for p in range(8):
                    a = slot_atom[8 * ci + p]
                    if a < 0:
                        continue
                    for q in range(8):
                        b = slot_atom[8 * cj + q]
                        if b < 0 or (ci == cj and s == (0, 0, 0) and q <= p):
                            continue
                        r2 = np.float32(0)
                        for k in range(3):
                            xa = w[a, k] - L[k] if s[k] > 0 else w[a, k]
                            xb = w[b, k] - L[k] if s[k] < 0 else w[b, k]
                            d = np.float32(np.float32(xa) - np.float32(xb))
                            r2 = np.float32(r2 + np.float32(d * d))
                        for k, r2k in enumerate(R2):
                            if r2 < r2k:
                                for M in sizes:
                                    for N in sizes:
                                        held[(M, N, k)].add((ci, p // M, cj, q // N, s))
    out = np.zeros((4, 4, len(radii)), np.int64)
    for (M, N, k), st in held.items():
        out[sizes.index(M), sizes.index(N), k] = len(st)
    return out


@pytest.mark.parametrize("seed,n,box,radii", [(5, 70, 2.05, [0.5, 0.8, 1.0]),
                                                (6, 110, [2.2, 2.6, 2.1], [0.45, 0.9]),
                                                (7, 40, 2.5, [0.3, 1.2])])
def test_census_matches_definition(oracle_mod, seed, n, box, radii):
    s = small_random_system(seed, n, box)
    g = grid_of(oracle_mod, s.x, s.box)
    got = oracle_mod.census.census(g["slot_atom"], g["w"], s.box, radii)
    ref = census_by_definition(g["slot_atom"], g["w"], s.box, radii)
    assert np.array_equal(got, ref)
    assert got[0, 0, -1] > 0 and np.any(got[1:, :, -1] != got[:-1, :, -1])


def test_census_pairs_against_kdtree(oracle_mod, sys3k):
    s = sys3k
    g = grid_of(oracle_mod, s.x, s.box)
    radii = [0.35, 0.7, 0.9, 1.0, 1.2]
    got = oracle_mod.census.census(g["slot_atom"], g["w"], s.box, radii)
    L = s.box.astype(np.float64)
    tree = cKDTree(np.mod(g["w"].astype(np.float64), L), boxsize=L)
    for k, r in enumerate(radii):
        r = float(np.float32(r))
        lo = tree.count_neighbors(tree, r * (1 - 2e-6)) - s.n   # ordered pairs, self pairs
        hi = tree.count_neighbors(tree, r * (1 + 2e-6)) - s.n
        assert lo // 2 <= got[0, 0, k] <= hi // 2, (r, lo // 2, got[0, 0, k], hi // 2)
        assert hi - lo < 100


def test_census_pairs_of_uniform_gas_closed_form(oracle_mod):
    rng = np.random.default_rng(2006)
    n, Lb = 4000, 3.4
    x = rng.uniform(0.0, Lb, (n, 3)).astype(np.float32)
    box = np.full(3, Lb, np.float32)
    g = grid_of(oracle_mod, x, box)
    radii = [0.3, 0.6, 1.0, 1.3]
    got = oracle_mod.census.census(g["slot_atom"], g["w"], box, radii)
    pairs = n * (n - 1) / 2
    for k, r in enumerate(radii):
        p = 4.0 / 3.0 * np.pi * r ** 3 / Lb ** 3
        mean, sd = pairs * p, np.sqrt(pairs * p * (1 - p))
        assert abs(got[0, 0, k] - mean) < 5 * sd, (r, got[0, 0, k], mean, sd)


def test_census_8x8_is_the_cluster_pair_set(oracle_mod, sys3k):
    s = sys3k
    g = grid_of(oracle_mod, s.x, s.box)
    radii = [0.6, 1.0, 1.1]
    got = oracle_mod.census.census(g["slot_atom"], g["w"], s.box, radii)
    for k, r in enumerate(radii):
        assert got[3, 3, k] == oracle_mod.cluster_pairs(g["slot_atom"], g["w"], s.box, r).size


def test_census_inclusions(oracle_mod, sys3k):
    s = sys3k
    g = grid_of(oracle_mod, s.x, s.box)
    radii = [0.5, 0.9, 0.95, 1.05, 1.2]
    c = oracle_mod.census.census(g["slot_atom"], g["w"], s.box, radii)
    assert np.all(np.diff(c, axis=2) >= 0)                     # more held as the radius grows
    # a held sub-cluster pair lies in exactly one held pair of the doubled sub-cluster,
    # which holds one or two of them
    assert np.all(c[1:, :, :] <= c[:-1, :, :]) and np.all(c[:-1, :, :] <= 2 * c[1:, :, :])
    assert np.all(c[:, 1:, :] <= c[:, :-1, :]) and np.all(c[:, :-1, :] <= 2 * c[:, 1:, :])
    # work efficiency: 1 x 1 at zero buffer is one; larger clusters compute more
    we = oracle_mod.census.work_efficiency
    assert we(c, 1, 1, 1, 1) == 1.0
    for kl in (1, 2, 3, 4):
        e = [we(c, 1, kl, M, N) for M, N in ((1, 1), (4, 4), (8, 4), (8, 8))]
        assert all(e[i] >= e[i + 1] for i in range(3)) and 0 < e[-1] < 1
