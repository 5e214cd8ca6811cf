"""List coverage (nb_list_coverage) against the oracle's coverage, exact, for several
sub-cluster setups and radii in any order, on a water box, a ragged ensemble and the full
96,000-atom box; and the Verlet buffer estimate fed with the GPU coverage equal to the one
fed with the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from conftest import small_random_system
from gpu_common import concat, dev, make_ctx
from paper_2006_09167_amd import api, systems

pytestmark = pytest.mark.gpu


def oracle_coverage_multi(c, radii, M, N):
    g = oracle.grid_spec.build_grid(c["x"], c["boxes"], c["offsets"])
    K = len(radii)
    out = np.zeros((K, K), np.int64)
    sc_col = g["sc_col"]
    for s in range(c["offsets"].size - 1):
        cb = g["col_base"][s]
        nx, ny = g["dims"][s]
        sel = np.flatnonzero((sc_col >= cb) & (sc_col < cb + nx * ny))
        if sel.size == 0:
            continue
        sub = g["slot_atom"][64 * int(sel[0]):64 * (int(sel[-1]) + 1)]
        out += oracle.buffer.coverage(sub, g["w"], c["boxes"][s], radii, M, N)
    return out


def listed(c, rlist):
    ctx = make_ctx(c, rc=min(0.9, rlist), rinner=rlist, rlist=rlist)
    ctx.grid_build(dev(c["x"]), c["boxes"])
    ctx.pairlist_build()
    return ctx


@pytest.mark.parametrize("M,N", [(8, 8), (8, 4), (4, 2), (1, 1), (2, 8)])
def test_coverage_water(sys3k, M, N):
    c = concat(sys3k)
    radii = [1.1, 0.9, 1.0, 1.2, 0.95, 1.0, 0.3]
    ctx = listed(c, 1.2)
    got = ctx.list_coverage(radii, M, N)
    torch.cuda.synchronize()
    assert np.array_equal(got, oracle_coverage_multi(c, radii, M, N))


def test_coverage_ragged_ensemble():
    parts = [small_random_system(41, 150, 2.4), small_random_system(42, 37, 2.1),
             small_random_system(43, 400, [2.5, 3.0, 2.7])]
    c = concat(parts)
    radii = list(np.linspace(0.3, 1.0, 9))
    ctx = listed(c, 1.0)
    for M, N in ((8, 8), (4, 4)):
        assert np.array_equal(ctx.list_coverage(radii, M, N),
                              oracle_coverage_multi(c, radii, M, N))


def test_coverage_full_size_water96k():
    s = systems.config_system("water96k_ewald")
    c = concat(s)
    radii = [1.0, 1.04, 1.1]
    ctx = listed(c, 1.1)
    assert np.array_equal(ctx.list_coverage(radii, 8, 8), oracle_coverage_multi(c, radii, 8, 8))


def test_coverage_argument_errors(sys3k):
    c = concat(sys3k)
    ctx = listed(c, 1.0)
    for bad in ((3, 8), (8, 16), (0, 8)):
        with pytest.raises(ValueError):
            ctx.list_coverage([0.9], *bad)
    with pytest.raises(RuntimeError):
        ctx.list_coverage([1.05], 8, 8)               # above the list radius


def test_buffer_estimate_from_gpu_coverage(sys3k):
    c = concat(sys3k)
    radii = (np.float32(0.9) + np.float32(0.01) * np.arange(20, dtype=np.float32)).astype(np.float32)
    ctx = listed(c, float(radii[-1]))
    classes = dict(count=[1000, 2000], mass=[18.015, 18.015], charge=[-0.82, 0.41], type=[0, 1])
    p = api.make_params(2, "ewald", rc=0.9, beta=3.47)
    V = float(np.prod(sys3k.box))
    for M, N in ((8, 8), (8, 4)):
        cov = ctx.list_coverage(radii, M, N)
        ref = oracle_coverage_multi(c, radii, M, N)
        assert np.array_equal(cov, ref)
        a = api.buffer_estimate(p, classes, sys3k.lj, V, 300.0, 0.002, 40, coverage=(radii, cov))
        b = api.buffer_estimate(p, classes, sys3k.lj, V, 300.0, 0.002, 40, coverage=(radii, ref))
        assert a == b
        part = api.buffer_estimate(p, classes, sys3k.lj, V, 300.0, 0.002, 40)
        assert a[0] <= part[0] + 0.01               # the implicit buffer never needs more
