"""Bounding-box candidates versus the list arithmetic in single precision (Sec. V.D: the
box search feeds candidates that the atom-distance test then prunes, so every pair the
list keeps must pass the box test).

The search compares the squared box gap with the list's own squared radius; the gap takes
the periodic shift on the same side as the atom distance (x_i - L for s > 0, x_j - L for
s < 0) and rounds each step once, so it can never exceed the distance of any atom pair of
the two boxes.  These CPU tests emulate both float32 sequences on single-atom boxes with
pairs just inside rlist, in boxes up to the largest edge the library accepts (1000 nm),
where one unit in the last place of L is 6e-5 nm; and they show that the earlier form,
which added s L to the j coordinate and compared with a fixed margin, lost such pairs."""
import numpy as np
import pytest

f32 = np.float32


def list_r2(xi, xj, s, L):
    """The list's squared distance: per axis a = x_i - L (s > 0), b = x_j - L (s < 0),
    d = a - b, r2 = (dx dx + dy dy) + dz dz, every step rounded to float32."""
    a = np.where(s > 0, (xi - L).astype(f32), xi)
    b = np.where(s < 0, (xj - L).astype(f32), xj)
    d = (a - b).astype(f32)
    sq = (d * d).astype(f32)
    return ((sq[:, 0] + sq[:, 1]).astype(f32) + sq[:, 2]).astype(f32)


def bb_r2(ilo, ihi, jlo, jhi, s, L):
    """The search's squared box gap with the shift on the list's side (bb_gap / bb_d2)."""
    alo = np.where(s > 0, (ilo - L).astype(f32), ilo)
    ahi = np.where(s > 0, (ihi - L).astype(f32), ihi)
    blo = np.where(s < 0, (jlo - L).astype(f32), jlo)
    bhi = np.where(s < 0, (jhi - L).astype(f32), jhi)
    g = np.maximum(f32(0), np.maximum((blo - ahi).astype(f32), (alo - bhi).astype(f32)))
    sq = (g * g).astype(f32)
    return ((sq[:, 0] + sq[:, 1]).astype(f32) + sq[:, 2]).astype(f32)


def old_bb_r2(ilo, ihi, jlo, jhi, s, L):
    """The earlier box gap: the j box moved by s L (one rounding at the size of L)."""
    o = (s.astype(f32) * L).astype(f32)
    g = np.maximum(f32(0), np.maximum(((jlo + o).astype(f32) - ihi).astype(f32),
                                      (ilo - (jhi + o).astype(f32)).astype(f32)))
    sq = (g * g).astype(f32)
    return (sq[:, 0] + sq[:, 1] + sq[:, 2]).astype(f32)


def pairs_near_radius(L, rlist, n, seed, rel=2e-5):
    """n atom pairs (x_i, x_j, s) in [0, L)^3 whose image distance is rlist (1 - u rel),
    u uniform: just inside the list radius, across every kind of periodic shift."""
    rng = np.random.default_rng(seed)
    Lv = np.full(3, L, np.float64)
    xi = rng.uniform(0, 1, (n, 3)) * Lv
    # put half the i atoms near the upper faces, so that x_j's image crosses the boundary
    near = rng.random((n, 3)) < 0.5
    xi = np.where(near, Lv - rng.uniform(0, rlist, (n, 3)), xi)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = rlist * (1.0 - rel * rng.random(n))
    img = xi - r[:, None] * v
    s = np.floor(img / Lv).astype(np.int64)     # x_j + s L = img with x_j in [0, L)
    xj = img - s * Lv
    xi32, xj32 = xi.astype(f32), xj.astype(f32)
    ok = np.all((xj32 < f32(L)) & (xj32 >= 0) & (xi32 < f32(L)), axis=1) & np.all(np.abs(s) <= 1, 1)
    return xi32[ok], xj32[ok], s[ok]


@pytest.mark.parametrize("L", [2.5, 24.7, 300.0, 1000.0])
def test_box_test_keeps_every_listed_pair(L):
    rlist = 1.1
    R2 = f32(np.float64(f32(rlist)) ** 2)
    Lf = np.full(3, f32(L), f32)
    xi, xj, s = pairs_near_radius(L, rlist, 40000, seed=int(L * 10))
    r2 = list_r2(xi, xj, s, Lf)
    kept = r2 < R2
    assert kept.sum() > 10000
    # single-atom boxes (lo = hi = x): the tightest boxes, where the gap is the distance
    g2 = bb_r2(xi, xi, xj, xj, s, Lf)
    assert np.all(g2 <= r2)
    assert np.all(g2[kept] < R2)
    # boxes grown around each atom can only shrink the gap
    rng = np.random.default_rng(7)
    lo_i = (xi - rng.uniform(0, 0.2, xi.shape)).astype(f32)
    hi_j = (xj + rng.uniform(0, 0.2, xj.shape)).astype(f32)
    assert np.all(bb_r2(lo_i, xi, xj, hi_j, s, Lf) <= g2)


def test_earlier_box_test_lost_pairs_in_long_boxes():
    """The fixed margin rlist (1 + 1e-5) + 1e-6 nm of the earlier test did not cover the
    rounding of x_j + L at L = 1000 nm (up to 3e-5 nm): some listed pairs were rejected.
    At the benchmark box sizes it held."""
    rlist = 1.1
    R2 = f32(np.float64(f32(rlist)) ** 2)
    rbb = rlist * (1.0 + 1e-5) + 1e-6
    R2bb = f32(rbb * rbb)
    lost = {}
    for L in (24.7, 1000.0):
        Lf = np.full(3, f32(L), f32)
        xi, xj, s = pairs_near_radius(L, rlist, 40000, seed=3)
        kept = list_r2(xi, xj, s, Lf) < R2
        lost[L] = int(np.sum(old_bb_r2(xi, xi, xj, xj, s, Lf)[kept] >= R2bb))
    assert lost[24.7] == 0
    assert lost[1000.0] > 0
