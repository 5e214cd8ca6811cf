"""Work-efficiency census of the outer list (nb_list_census) against the oracle's census:
exact integer counts for every sub-cluster setup M x N (M, N in {1, 2, 4, 8}) and radius,
on a water box with radii in any order and repeated, on an ensemble of ragged random
systems, with the maximum number of radii, at the full 96,000-atom size, and the
argument errors."""
import numpy as np
import pytest
import torch

import oracle
from conftest import small_random_system
from gpu_common import concat, dev, make_ctx
from paper_2006_09167_amd import systems

pytestmark = pytest.mark.gpu


def oracle_census_multi(c, radii):
    """Oracle census summed over the systems of a concatenation (pairs never cross)."""
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    out = np.zeros((4, 4, len(radii)), np.int64)
    sc_col = g["sc_col"]
    for s in range(c["offsets"].size - 1):
        cb = g["col_base"][s]
        nx, ny = g["dims"][s]
        sel = np.flatnonzero((sc_col >= cb) & (sc_col < cb + nx * ny))
        if sel.size == 0:
            continue
        sub = g["slot_atom"][64 * int(sel[0]):64 * (int(sel[-1]) + 1)]
        out += oracle.census.census(sub, g["w"], c["boxes"][s], radii)
    return out


def census_of(c, rlist, radii):
    ctx = make_ctx(c, rc=min(1.0, rlist), rinner=rlist, rlist=rlist)
    ctx.grid_build(dev(c["x"]), c["boxes"])
    ctx.pairlist_build()
    got = ctx.list_census(radii)
    torch.cuda.synchronize()
    return ctx, got


def test_census_water_any_order_and_repeats(sys3k):
    c = concat(sys3k)
    radii = [1.2, 0.3, 1.0, 1.5, 0.9, 1.0, 1.45, 0.05]
    ctx, got = census_of(c, 1.5, radii)
    ref = oracle_census_multi(c, radii)
    assert np.array_equal(got, ref), np.argwhere(got != ref)
    assert got[0, 0, 2] == got[0, 0, 5] and got[0, 0, 7] == 0
    # the 8 x 8 count at the list radius is the outer list itself
    assert got[3, 3, 3] == ctx.stats()["outer_pairs"]


def test_census_ragged_ensemble():
    parts = [small_random_system(21, 150, 2.4), small_random_system(22, 37, 2.1),
             small_random_system(23, 400, [2.5, 3.0, 2.7])]
    c = concat(parts)
    radii = [0.4, 0.7, 1.0]
    _, got = census_of(c, 1.0, radii)
    assert np.array_equal(got, oracle_census_multi(c, radii))


def test_census_maximum_radii(sys3k):
    c = concat(sys3k)
    radii = list(np.linspace(0.02, 1.3, 64))
    _, got = census_of(c, 1.3, radii)
    assert got.shape == (4, 4, 64)
    assert np.array_equal(got, oracle_census_multi(c, radii))


def test_census_full_size_water96k():
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    radii = [1.0, 1.1]
    ctx, got = census_of(c, 1.1, radii)
    assert np.array_equal(got, oracle_census_multi(c, radii))
    assert got[3, 3, 1] == ctx.stats()["outer_pairs"]


def test_census_argument_errors(sys3k):
    c = concat(sys3k)
    ctx = make_ctx(c, rc=1.0, rinner=1.0, rlist=1.0)
    with pytest.raises(RuntimeError):
        ctx.list_census([0.5])                       # no list yet
    ctx.grid_build(dev(c["x"]), c["boxes"])
    ctx.pairlist_build()
    for bad in ([], [1.01], [0.0], [-0.5], [float("nan")], list(np.linspace(0.1, 1.0, 65))):
        with pytest.raises(RuntimeError):
            ctx.list_census(bad)
    assert ctx.list_census([1.0])[0, 0, 0] > 0


def test_census_and_coverage_with_empty_and_one_atom_systems():
    """Systems without atoms or with a single atom hold no pairs; the census and coverage
    of the ensemble equal those of its other members, and a list with no pair inside any
    radius counts nothing."""
    from test_gpu_buffer import oracle_coverage_multi
    one = small_random_system(52, 1, 2.4)
    empty = systems.System(**{**one.__dict__, "x": np.zeros((0, 3), np.float32),
                              "q": np.zeros(0, np.float32), "type": np.zeros(0, np.int32),
                              "excl_ptr": np.zeros(1, np.int64),
                              "excl_idx": np.zeros(0, np.int32)})
    parts = [small_random_system(51, 120, 2.3), empty, one, small_random_system(53, 60, 2.2)]
    c = concat(parts)
    radii = [0.3, 0.6, 0.9]
    ctx, got = census_of(c, 0.9, radii)
    assert np.array_equal(got, oracle_census_multi(c, radii))
    assert got[0, 0, -1] > 0
    assert np.array_equal(ctx.list_coverage(radii, 8, 4), oracle_coverage_multi(c, radii, 8, 4))
    # two atoms 1.5 nm apart: nothing within 0.5 nm
    far = systems.System(**{**one.__dict__, "x": np.array([[0.2, 0.2, 0.2], [1.7, 0.2, 0.2]],
                                                         np.float32),
                            "q": np.zeros(2, np.float32), "type": np.zeros(2, np.int32),
                            "excl_ptr": np.zeros(3, np.int64), "excl_idx": np.zeros(0, np.int32),
                            "box": np.full(3, 4.0, np.float32)})
    _, none = census_of(concat(far), 0.5, [0.2, 0.5])
    assert not np.any(none)
