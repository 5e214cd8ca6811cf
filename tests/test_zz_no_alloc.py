"""The allocation-free census entry point (nb_list_census_noalloc) against nb_list_census:
bit-identical counts on two calls in a row, the first on the 96,000-atom water box with
short work items (more items than the fixed scratch has blocks, so its blocks stride over
the items), the second on the 3,000-atom box; then the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import concat, dev, make_ctx
from paper_2006_09167_amd import _lib, systems

pytestmark = pytest.mark.gpu


def _census_pair(ctx, radii):
    ref = ctx.list_census(radii)
    got = ctx.list_census_noalloc(radii)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_census_matches_twice_then_smaller():
    big = concat(systems.config_system("water96k_ewald"))
    ctx = make_ctx(big, rc=1.0, rinner=1.2, rlist=1.2)
    ctx.grid_build(dev(big["x"]), big["boxes"])
    ctx.pairlist_build()
    ctx.set_exec(8, "static", True)            # about 30k items: above 1024 blocks x 8 waves
    assert ctx.stats()["n_work_items"] > 1024 * 8
    radii = [1.2, 0.35, 1.0, 0.9, 1.1]
    ref, got = _census_pair(ctx, radii)
    assert np.array_equal(got, ref), np.argwhere(got != ref)
    assert got[3, 3, 0] == ctx.stats()["outer_pairs"]
    # a second call on a smaller system (another context on the same device)
    small = concat(systems.config_system("water3k_rf"))
    ctx2 = make_ctx(small, rc=1.0, rinner=1.0, rlist=1.0)
    ctx2.grid_build(dev(small["x"]), small["boxes"])
    ctx2.pairlist_build()
    radii2 = [0.5, 1.0]
    ref2, got2 = _census_pair(ctx2, radii2)
    assert np.array_equal(got2, ref2), np.argwhere(got2 != ref2)
    # and the first context again: the shared scratch holds the small call's words
    ref3, got3 = _census_pair(ctx, radii)
    assert np.array_equal(got3, ref3) and np.array_equal(got3, ref)


def test_noalloc_census_limits():
    small = concat(systems.config_system("water3k_rf"))
    ctx = make_ctx(small, rc=1.0, rinner=1.0, rlist=1.0)
    with pytest.raises(RuntimeError):
        ctx.list_census_noalloc([0.5])                 # no list yet
    ctx.grid_build(dev(small["x"]), small["boxes"])
    ctx.pairlist_build()
    lib = _lib.load()
    r = np.linspace(0.1, 1.0, _lib.NB_CENSUS_MAX_RADII + 1).astype(np.float32)
    cnt = np.zeros(16 * r.size, np.int64)
    st = lib.nb_list_census_noalloc(ctx.h, int(r.size), r.ctypes.data_as(ctypes.c_void_p),
                                    cnt.ctypes.data_as(ctypes.c_void_p))
    assert st == _lib.NB_ERR_ARG
    assert b"n_radii" in lib.nb_last_error(ctx.h)
    full = list(np.linspace(0.02, 1.0, _lib.NB_CENSUS_MAX_RADII))
    ref, got = _census_pair(ctx, full)
    assert np.array_equal(got, ref)
