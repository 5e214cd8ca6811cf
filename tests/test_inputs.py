"""The seeded input generators (no method arithmetic): the argon box of the throughput
sweep has the paper's density and cut-offs that put the requested number of particles in
the half cut-off sphere."""
import math

import numpy as np
from scipy.spatial import cKDTree

from paper_2006_09167_amd import systems


def test_argon_box_density_and_layout():
    s = systems.argon_box(k=10, seed=5)
    L = float(s.box[0])
    assert s.n == 1000 and np.allclose(s.box, L)
    assert abs(s.n / L ** 3 - systems.ARGON["density"]) < 1e-3
    assert np.all(s.q == 0) and np.all(s.type == 0) and s.excl_ptr[-1] == 0
    assert s.x.min() >= 0.0 and s.x.max() < L
    a = L / 10
    d, _ = cKDTree(s.x.astype(np.float64), boxsize=L).query(s.x.astype(np.float64), k=2)
    assert d[:, 1].min() >= a * (1 - 2 * systems.ARGON["jitter"]) - 1e-6
    c6, c12 = s.lj[0, 0]
    assert abs(c12 / c6 - systems.ARGON["sigma"] ** 6) < 1e-9    # sigma^6 = c12 / c6
    # same seed, same box
    assert np.array_equal(s.x, systems.argon_box(k=10, seed=5).x)


def test_argon_cutoffs_give_half_sphere_counts():
    s = systems.argon_box(k=24, seed=6)                # 13824 atoms, 7.6 nm box
    L = float(s.box[0])
    tree = cKDTree(s.x.astype(np.float64), boxsize=L)
    for n_half in (50, 200, 800):
        rc = systems.argon_cutoff(n_half)
        assert abs(2.0 / 3.0 * math.pi * rc ** 3 * systems.ARGON["density"] - n_half) < 1e-9
        pairs = tree.count_neighbors(tree, rc) - s.n    # ordered pairs, self excluded
        # the jittered lattice's shells move the count by up to 10% at the shortest cut-off
        assert abs(pairs / 2 / s.n - n_half) < 0.1 * n_half
