"""Pins of the oracle's grid specification and cluster-pair sets: invariants of the
grid, an independent brute-force enumeration over (i-cluster, j-cluster, shift)
on tiny inputs, threshold cases one ulp either side of the radius, coverage of
every atom pair found by a double-precision minimum-image search, permutation
invariance and inclusion between radii."""
import itertools

import numpy as np
import pytest

from conftest import small_random_system
from paper_2006_09167_amd import systems


def grid_of(o, s):
    return o.grid_spec.build_grid(s.x, s.box[None], np.array([0, s.n]))


# ---- grid ------------------------------------------------------------------------------
def check_grid_invariants(o, x, boxes, offsets):
    g = o.grid_spec.build_grid(x, boxes, offsets)
    sa = g["slot_atom"]
    real = sa[sa >= 0]
    assert np.array_equal(np.sort(real), np.arange(int(offsets[-1])))      # each atom once
    w = g["w"]
    n_sc = g["n_sc"]
    sc_of_slot = np.arange(sa.size) // 64
    # every super-cell except the last of its column is full
    counts = (sa.reshape(n_sc, 64) >= 0).sum(axis=1)
    last_of_col = np.r_[np.flatnonzero(np.diff(g["sc_col"]) != 0), n_sc - 1]
    full = np.ones(n_sc, bool)
    full[last_of_col] = False
    assert np.all(counts[full] == 64)
    assert np.all(counts >= 1)
    # atoms sit in the column of their super-cell
    for s in range(boxes.shape[0]):
        nx, ny = g["dims"][s]
        a0, a1 = int(offsets[s]), int(offsets[s + 1])
        L = boxes[s].astype(np.float64)
        for a in range(a0, a1, max(1, (a1 - a0) // 200)):
            sl = g["atom_slot"][a]
            col = g["sc_col"][sl // 64] - g["col_base"][s]
            cx, cy = col // ny, col % ny
            # the column bounds, with a rounding margin
            assert cx * L[0] / nx - 1e-5 <= w[a, 0] <= (cx + 1) * L[0] / nx + 1e-5
            assert cy * L[1] / ny - 1e-5 <= w[a, 1] <= (cy + 1) * L[1] / ny + 1e-5
    # z order along columns, then the 2x2x2 splits inside each super-cell
    for sc in range(n_sc):
        atoms = sa[sc * 64:(sc + 1) * 64]
        cl = np.arange(64) // 8
        m = atoms >= 0
        zh, yh = cl // 4, (cl // 2) % 2
        for lo, hi, axis in ((m & (zh == 0), m & (zh == 1), 2),):
            if lo.any() and hi.any():
                assert w[atoms[lo], axis].max() <= w[atoms[hi], axis].min()
        for z in (0, 1):
            lo, hi = m & (zh == z) & (yh == 0), m & (zh == z) & (yh == 1)
            if lo.any() and hi.any():
                assert w[atoms[lo], 1].max() <= w[atoms[hi], 1].min()
            for y in (0, 1):
                base = m & (zh == z) & (yh == y)
                lo, hi = base & (cl % 2 == 0), base & (cl % 2 == 1)
                if lo.any() and hi.any():
                    assert w[atoms[lo], 0].max() <= w[atoms[hi], 0].min()
        # partial super-cells fill lower halves first
        n = int(m.sum())
        assert int((m & (zh == 0)).sum()) == min(n, 32)
    return g


def test_grid_invariants_3k(oracle_mod, sys3k):
    g = check_grid_invariants(oracle_mod, sys3k.x, sys3k.box[None], np.array([0, sys3k.n]))
    assert g["dims"] == [(4, 4)]


def test_grid_invariants_ensemble(oracle_mod):
    reps = [small_random_system(s, n, L) for s, n, L in ((1, 150, 2.4), (2, 7, 2.2), (3, 300, 3.0))]
    c = systems.concat_systems(reps)
    check_grid_invariants(oracle_mod, c["x"], c["boxes"], c["offsets"])


def test_grid_matches_plain_sort(oracle_mod):
    """The slot order equals a plain Python sort with tuple keys (tiny input)."""
    s = small_random_system(9, 150, 2.3)
    g = grid_of(oracle_mod, s)
    w = g["w"]
    nx, ny = g["dims"][0]
    cinv = (np.float32(nx / np.float64(s.box[0])), np.float32(ny / np.float64(s.box[1])))
    def col(a):
        cx = min(nx - 1, max(0, int(np.floor(np.float32(w[a, 0] * cinv[0])))))
        cy = min(ny - 1, max(0, int(np.floor(np.float32(w[a, 1] * cinv[1])))))
        return cx * ny + cy
    order = sorted(range(s.n), key=lambda a: (col(a), float(w[a, 2]), a))
    expect = []
    by_col = {}
    for a in order:
        by_col.setdefault(col(a), []).append(a)
    for c in sorted(by_col):
        atoms = by_col[c]
        for k in range(0, len(atoms), 64):
            cell = atoms[k:k + 64]
            slots = [-1] * 64
            zs = [cell[:32], cell[32:]]
            for zi, zpart in enumerate(zs):
                ys = sorted(zpart, key=lambda a: (float(w[a, 1]), a))
                for yi, ypart in enumerate([ys[:16], ys[16:]]):
                    xs = sorted(ypart, key=lambda a: (float(w[a, 0]), a))
                    for xi, xpart in enumerate([xs[:8], xs[8:]]):
                        for p, a in enumerate(xpart):
                            slots[(zi * 4 + yi * 2 + xi) * 8 + p] = a
            expect.extend(slots)
    assert np.array_equal(g["slot_atom"], np.array(expect, dtype=np.int32))


def test_wrap_is_in_box(oracle_mod):
    x = np.array([[-1e-9, 9.86 - 1e-7, 19.72], [-9.86, 4.0, 1e-30], [123.4, -55.5, 0.0]],
                 dtype=np.float32)
    box = np.full(3, 9.86, np.float32)
    k, w = oracle_mod.grid_spec.wrap(x, box)
    assert np.all(w >= -1e-6) and np.all(w <= box + 1e-6)
    assert np.allclose(x.astype(np.float64) - k * box.astype(np.float64), w, atol=1e-5)


# ---- cluster pairs ---------------------------------------------------------------------
def brute_force_triples(slot_atom, w, box, R):
    """Independent enumeration: every (ci <= cj, shift) and every atom pair in it, in
    numpy single precision following the specified sequence."""
    R2 = np.float32(np.float64(np.float32(R)) ** 2)
    L = box.astype(np.float32)
    n_cl = slot_atom.size // 8
    out = set()
    shifts = list(itertools.product((-1, 0, 1), repeat=3))
    for ci in range(n_cl):
        ai = slot_atom[ci * 8:(ci + 1) * 8]
        for cj in range(ci, n_cl):
            aj = slot_atom[cj * 8:(cj + 1) * 8]
            for s in shifts:
                if ci == cj and s != (0, 0, 0) and not (s > (0, 0, 0)):
                    continue
                P, Q = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
                ok = (ai[P] >= 0) & (aj[Q] >= 0)
                if ci == cj and s == (0, 0, 0):
                    ok &= Q > P
                if not ok.any():
                    continue
                xi = w[np.where(ai[P] >= 0, ai[P], 0)]
                xj = w[np.where(aj[Q] >= 0, aj[Q], 0)]
                r2 = np.zeros(P.shape, np.float32)
                comps = []
                for k in range(3):
                    a = xi[..., k] - L[k] if s[k] > 0 else xi[..., k]
                    b = xj[..., k] - L[k] if s[k] < 0 else xj[..., k]
                    d = (a.astype(np.float32) - b.astype(np.float32)).astype(np.float32)
                    comps.append((d * d).astype(np.float32))
                r2 = ((comps[0] + comps[1]).astype(np.float32) + comps[2]).astype(np.float32)
                if np.any(ok & (r2 < R2)):
                    code = (s[0] + 1) * 9 + (s[1] + 1) * 3 + (s[2] + 1)
                    out.add((ci * n_cl + cj) * 27 + code)
    return np.array(sorted(out), dtype=np.int64)


@pytest.mark.parametrize("seed,n,box,R", [(1, 120, 2.2, 1.0), (2, 200, 2.6, 1.1),
                                          (3, 70, 2.05, 1.0), (4, 130, [2.1, 3.3, 2.5], 0.9)])
def test_cluster_pairs_match_independent_brute_force(oracle_mod, seed, n, box, R):
    s = small_random_system(seed, n, box)
    g = grid_of(oracle_mod, s)
    keys = oracle_mod.cluster_pairs(g["slot_atom"], g["w"], s.box, R)
    ref = brute_force_triples(g["slot_atom"], g["w"], s.box, R)
    assert np.array_equal(keys, ref)
    n_cl = g["slot_atom"].size // 8
    ci, cj, code = oracle_mod.split_key(keys, n_cl)
    assert np.all(ci <= cj)
    assert np.all(code[ci == cj] >= 13)        # no lexicographically negative self shifts


def test_radius_threshold_is_strict_single_precision(oracle_mod):
    """Two atoms exactly R apart are out; one ulp closer is in."""
    box = np.full(3, 4.0, np.float32)
    slot_atom = np.array([0] + [-1] * 7 + [1] + [-1] * 7, np.int32)
    for xj, inside in ((np.float32(2.5), False),
                       (np.nextafter(np.float32(2.5), np.float32(0)), True)):
        w = np.array([[1.5, 1.0, 1.0], [xj, 1.0, 1.0]], np.float32)
        keys = oracle_mod.cluster_pairs(slot_atom, w, box, 1.0)
        assert (keys.size == 1) == inside
    # same through the periodic boundary: d = (0.25) - (3.25 - 4) = 1.0 exactly
    for xj, inside in ((np.float32(3.25), False), (np.nextafter(np.float32(3.25), np.float32(4)), True)):
        w = np.array([[0.25, 1.0, 1.0], [xj, 1.0, 1.0]], np.float32)
        keys = oracle_mod.cluster_pairs(slot_atom, w, box, 1.0)
        assert (keys.size == 1) == inside
        if inside:
            _, _, code = oracle_mod.split_key(keys, 2)
            assert code[0] == 0 * 9 + 1 * 3 + 1          # s = (-1, 0, 0): j shifted by -L


def test_every_close_atom_pair_is_covered(oracle_mod, sys3k):
    """Each atom pair closer than R (double-precision minimum image, with a margin for
    single-precision rounding) lies in a listed cluster pair with the right shift."""
    s = sys3k
    g = grid_of(oracle_mod, s)
    R = 1.0
    keys = set(oracle_mod.cluster_pairs(g["slot_atom"], g["w"], s.box, R).tolist())
    n_cl = g["slot_atom"].size // 8
    w = g["w"].astype(np.float64)
    L = s.box.astype(np.float64)
    slot = g["atom_slot"]
    rng = np.random.default_rng(0)
    for a in rng.choice(s.n, 300, replace=False):
        d = w[a] - w
        img = np.round(d / L)
        dm = d - img * L
        r = np.linalg.norm(dm, axis=1)
        for b in np.flatnonzero((r < R * (1 - 1e-5)) & (np.arange(s.n) != a)):
            i, j = (a, b) if slot[a] < slot[b] else (b, a)
            # shift of j relative to i: d_ij = w_i - (w_j + s L)  =>  s = round((w_i - w_j)/L)
            sh = np.round((w[i] - w[j]) / L).astype(int)
            ci, cj = slot[i] // 8, slot[j] // 8
            if ci == cj and tuple(sh) < (0, 0, 0):
                sh = -sh
            code = (sh[0] + 1) * 9 + (sh[1] + 1) * 3 + (sh[2] + 1)
            assert (ci * n_cl + cj) * 27 + code in keys


def test_pair_sets_invariant_under_permutation(oracle_mod):
    s = small_random_system(21, 180, 2.5)
    g = grid_of(oracle_mod, s)
    rng = np.random.default_rng(1)
    perm = rng.permutation(s.n)
    sp = systems.System(**{**s.__dict__, "x": s.x[perm]})
    gp = grid_of(oracle_mod, sp)

    def as_atom_sets(gr, relabel):
        keys = oracle_mod.cluster_pairs(gr["slot_atom"], gr["w"], s.box, 1.0)
        n_cl = gr["slot_atom"].size // 8
        ci, cj, code = oracle_mod.split_key(keys, n_cl)
        sa = gr["slot_atom"].reshape(-1, 8)
        out = set()
        for a, b, c in zip(ci, cj, code):
            A = frozenset(relabel[t] for t in sa[a] if t >= 0)
            B = frozenset(relabel[t] for t in sa[b] if t >= 0)
            out.add((A, B, int(c)))
        return out

    # the grid only depends on coordinates (no ties here), so clusters hold the same atoms
    assert as_atom_sets(g, np.arange(s.n)) == as_atom_sets(gp, perm)


def test_inner_subset_of_outer_and_monotone(oracle_mod, sys3k):
    s = sys3k
    g = grid_of(oracle_mod, s)
    outer = oracle_mod.cluster_pairs(g["slot_atom"], g["w"], s.box, 1.0)
    inner = oracle_mod.cluster_pairs(g["slot_atom"], g["w"], s.box, 0.9)
    assert np.all(np.isin(inner, outer))
    assert inner.size < outer.size
    # parts partition the inner list by owner super-cluster
    n_parts = 4
    parts = [oracle_mod.inner_pairs(outer, g["slot_atom"], g["w"], s.box, 0.9, n_parts, p)
             for p in range(n_parts)]
    assert sum(p.size for p in parts) == inner.size
    assert np.array_equal(np.sort(np.concatenate(parts)), inner)


def test_rolling_part_owner_is_the_lower_cluster(oracle_mod):
    """Rolling parts follow the owner of a cluster pair, the super-cluster of its lower
    cluster index (Sec. V.E: the list is pruned in parts, one per step; Sec. V.A: each
    pair is listed once, with the super-cluster of the lower cluster).  Three atoms in
    clusters 0, 8 and 17 (super-clusters 0, 1 and 2) form the pairs (0, 8) and (8, 17);
    the second pair belongs to super-cluster 1, so with two parts it is in part 1 and with
    three parts in part 1 (owning by the higher cluster would give parts 0 and 2)."""
    slot_atom = np.full(3 * 64, -1, np.int32)
    slot_atom[0], slot_atom[64], slot_atom[8 * 17] = 0, 1, 2
    w = np.array([[1.0, 1.0, 1.0], [1.5, 1.0, 1.0], [2.0, 1.0, 1.0]], np.float32)
    box = np.full(3, 10.0, np.float32)
    n_cl = 24
    outer = oracle_mod.cluster_pairs(slot_atom, w, box, 0.7)
    k08 = (0 * n_cl + 8) * 27 + 13
    k817 = (8 * n_cl + 17) * 27 + 13
    assert outer.tolist() == [k08, k817]
    expect = {2: {0: [k08], 1: [k817]}, 3: {0: [k08], 1: [k817], 2: []}}
    for n_parts, parts in expect.items():
        for part, keys in parts.items():
            got = oracle_mod.inner_pairs(outer, slot_atom, w, box, 0.7, n_parts, part)
            assert got.tolist() == keys, (n_parts, part)
