import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: minutes of CPU time")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in file order, the no-allocation entry point last.
    pass


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def sys3k():
    from paper_2006_09167_amd import systems
    return systems.config_system("water3k_rf")


@pytest.fixture(scope="session")
def sys24k():
    from paper_2006_09167_amd import systems
    return systems.config_system("diff24k_rf")


def small_random_system(seed, n, box, n_types=2, dyadic=False, charge=0.5, excl_groups=3,
                        min_dist=0.12):
    """A tiny random system (test helper): n atoms in a box, random types/charges,
    exclusions inside consecutive groups of ``excl_groups`` atoms.  With ``dyadic`` the
    coordinates are multiples of 2^-6 nm so that small dyadic scalings stay exact in
    single precision."""
    from paper_2006_09167_amd.systems import System, lj_table_lorentz_berthelot
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=np.float64).reshape(-1)
    if L.size == 1:
        L = np.repeat(L, 3)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, 1, 3) * L
        if dyadic:
            p = np.floor(p * 64.0) / 64.0
        ok = True
        for o in pts:
            d = p - o
            d -= L * np.round(d / L)
            if np.linalg.norm(d) < min_dist:
                ok = False
                break
        if ok:
            pts.append(p)
    x = np.array(pts, dtype=np.float32)
    sigma = rng.uniform(0.25, 0.35, n_types)
    eps = rng.uniform(0.2, 1.0, n_types)
    typ = rng.integers(0, n_types, n).astype(np.int32)
    q = rng.normal(0, charge, n)
    q -= q.mean()
    ptr = [0]
    idx = []
    for a in range(n):
        g0 = (a // excl_groups) * excl_groups
        for b in range(g0, min(n, g0 + excl_groups)):
            if b != a:
                idx.append(b)
        ptr.append(len(idx))
    return System(x=x, q=q.astype(np.float32), type=typ, excl_ptr=np.array(ptr, np.int64),
                  excl_idx=np.array(idx, np.int32), box=L.astype(np.float32), sigma=sigma,
                  eps=eps, lj=lj_table_lorentz_berthelot(sigma, eps))


def lattice_system(dims, box, seed, jitter=0.1, n_types=2, charge=0.5, excl_groups=3,
                   keep=None, extra=None):
    """Atoms on a jittered lattice of dims = (nx, ny, nz) sites filling a box (test helper):
    site (i, j, k) at ((i + 1/2) Lx / nx, ...) plus a uniform jitter of +-jitter spacings per
    axis; ``keep`` (a function of the site positions, returning a boolean mask) drops sites;
    ``extra`` appends given positions.  Random types and neutral charges; exclusions inside
    consecutive groups of ``excl_groups`` atoms (symmetric)."""
    from paper_2006_09167_amd.systems import System, lj_table_lorentz_berthelot
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=np.float64)
    dims = np.asarray(dims)
    a = L / dims
    grid = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij"), -1).reshape(-1, 3)
    x = (grid + 0.5) * a + rng.uniform(-jitter, jitter, grid.shape) * a
    if keep is not None:
        x = x[keep(x)]
    if extra is not None:
        x = np.concatenate([x, np.asarray(extra, np.float64).reshape(-1, 3)])
    x = x.astype(np.float32)
    n = x.shape[0]
    sigma = rng.uniform(0.25, 0.35, n_types)
    eps = rng.uniform(0.2, 1.0, n_types)
    typ = rng.integers(0, n_types, n).astype(np.int32)
    q = rng.normal(0, charge, n)
    q -= q.mean()
    ptr = np.zeros(n + 1, np.int64)
    idx = []
    for i in range(n):
        g0 = (i // excl_groups) * excl_groups
        idx.extend(b for b in range(g0, min(n, g0 + excl_groups)) if b != i)
        ptr[i + 1] = len(idx)
    return System(x=x, q=q.astype(np.float32), type=typ, excl_ptr=ptr,
                  excl_idx=np.array(idx, np.int32), box=L.astype(np.float32), sigma=sigma,
                  eps=eps, lj=lj_table_lorentz_berthelot(sigma, eps))
