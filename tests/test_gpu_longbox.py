"""Boxes far from the benchmark shapes, through the whole path (grid slot order, bounding-box
candidates, outer and inner lists bit-exact against the oracle, forces and energies against
the FP64 oracle):

* a 2.4 x 2.4 x 300 nm box whose grid is one column of ~3,000 atoms (the z sort of a column
  of 2,049-4,096 atoms in LDS) and one of ~5,000 atoms (the sort in global memory);
* a 4.8 x 1000 x 2.4 nm box, the largest edge the library accepts, with atom pairs planted
  across the periodic boundary at distances a few units in the last place inside the list
  radius, where the i-cluster sits at the top of the long axis (the case in which adding
  the box edge to a coordinate near zero rounds at the size of the edge);
* an ensemble of 130 slabs with 8,320 grid columns in all (the column count and scatter
  without the LDS histogram, above 8,192 columns).
The bounding-box candidates must contain the outer list in every case (Sec. V.D)."""
import numpy as np
import pytest

import oracle
from conftest import lattice_system
from gpu_common import concat, keys_of
from test_gpu_parity import build, check_forces, check_grid, check_lists

pytestmark = pytest.mark.gpu

f32 = np.float32


def run(c, rc, rinner, rlist, expect_dims=None):
    ctx, x = build(c, coulomb="rf", rc=rc, rinner=rinner, rlist=rlist)
    g = check_grid(ctx, c)
    if expect_dims is not None:
        assert [tuple(d) for d in ctx.get_grid_dims()] == expect_dims
    ko, _ = check_lists(ctx, c, g, rlist, rinner)
    n_cl = g["slot_atom"].size // 8
    bb = keys_of(ctx.get_pairs("bb"), n_cl)
    assert np.unique(bb).size == bb.size
    assert np.all(np.isin(ko, bb))
    # On these sparse lattices most pairs inside rc lie near it, where a shifted pair energy
    # is a small difference of its terms, and there are too few pairs for rounding errors to
    # average.  Worst case per pair, in units u = 2^-24 of the term magnitudes (term_scale):
    # LJ, the hardware 1/sqrt (<= 1 ulp, 2u) carried to r^-6 through three products gives
    # 17u, the r^-12 term twice that plus the roundings of the fused sums, 36u at most, so
    # 40u; reaction field, 2u of 1/r from the 1/sqrt and one rounding each for
    # k_rf r^2 + 1/r, the subtraction of c_rf and the accumulation, so 4u.
    check_forces(ctx, c, x, "rf", rc, strict=False, term_ulps=(40, 4))
    return ctx, g, ko


@pytest.mark.parametrize("nz,expect", [(333, 2997), (556, 5004)])
def test_one_long_column(nz, expect):
    s = lattice_system((3, 3, nz), (2.4, 2.4, 300.0), seed=nz)
    assert s.n == expect
    ctx, g, ko = run(concat(s), 1.0, 1.05, 1.1, expect_dims=[(1, 1)])
    assert ko.size > 0


def _list_r2(xi, xj, s, L):
    """The specified single-precision list distance (split shift, no contraction)."""
    a = np.where(s > 0, (xi - L).astype(f32), xi)
    b = np.where(s < 0, (xj - L).astype(f32), xj)
    d = (a - b).astype(f32)
    sq = (d * d).astype(f32)
    return f32(f32(sq[0] + sq[1]) + sq[2])


def _planted_pairs(L, rlist):
    """Two atom pairs across y = 0 / y = L: a at the top of the y axis in grid column x 0,
    b at the bottom in column x 1, b placed at the largest single-precision y that keeps the
    pair inside rlist under the list's own arithmetic (shift +1 on b's side of y)."""
    R2 = f32(np.float64(f32(rlist)) ** 2)
    Lv = np.asarray(L, f32)
    out = []
    for z in (0.3, 1.5):
        xa = np.array([2.2, L[1] - 0.3, z], f32)
        yb = f32(np.sqrt(rlist ** 2 - 0.4 ** 2) - 0.3 - 1e-3)
        s = np.array([0, 1, 0])
        xb = np.array([2.6, yb, z], f32)
        assert _list_r2(xa, xb, s, Lv) < R2
        while True:
            nxt = xb.copy()
            nxt[1] = np.nextafter(xb[1], f32(10))
            if not _list_r2(xa, nxt, s, Lv) < R2:
                break
            xb = nxt
        out += [xa, xb]
    return np.array(out, np.float64)


def test_edge_1000nm_with_planted_boundary_pairs():
    L = (4.8, 1000.0, 2.4)
    rlist = 1.1
    planted = _planted_pairs(L, rlist)
    s = lattice_system((6, 1250, 6), L, seed=77, keep=lambda x: (x[:, 1] > 3) & (x[:, 1] < 997),
                       extra=planted)
    c = concat(s)
    ctx, g, ko = run(c, 1.0, 1.05, rlist)
    nx, ny = ctx.get_grid_dims()[0]
    assert nx == 2
    # each planted pair is a cluster pair of the outer list with the i-cluster on top
    n_cl = g["slot_atom"].size // 8
    slot_of = np.empty(s.n, np.int64)
    real = g["slot_atom"] >= 0
    slot_of[g["slot_atom"][real]] = np.flatnonzero(real)
    for k in range(2):
        a, b = s.n - 4 + 2 * k, s.n - 3 + 2 * k
        ca, cb = slot_of[a] // 8, slot_of[b] // 8
        assert ca < cb
        key = (ca * n_cl + cb) * 27 + (1 * 9 + 2 * 3 + 1)     # shift (0, +1, 0)
        assert key in set(ko.tolist())


def test_ensemble_above_lds_column_limit():
    slabs = [lattice_system((32, 32, 2), (40.0, 40.0, 2.3), seed=1000 + k) for k in range(130)]
    ctx, g, ko = run(concat(slabs), 1.0, 1.05, 1.1)
    dims = ctx.get_grid_dims()
    assert int(np.sum(dims[:, 0] * dims[:, 1])) > 8192
