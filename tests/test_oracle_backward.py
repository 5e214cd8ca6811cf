"""Pins of the oracle's backward pass: central finite differences of the FP64 loss
on a frozen pair set, symmetry of the Hessian, linearity in the adjoint, the zero
adjoint, and the force-matching loss of the differentiation workload."""
import numpy as np
import pytest

from conftest import small_random_system
from paper_2006_09167_amd.systems import System


def _params(o, coul):
    return o.params(coul, rc=1.0, beta=3.12)


def linear_loss(o, s, p, G, gE, x=None, q=None, lj=None):
    """L = sum G.F + gE.E, evaluated by the FP64 forward oracle."""
    x = s.x if x is None else x
    q = s.q if q is None else q
    lj = s.lj if lj is None else lj
    e, f, _ = o.forces(x, q, s.type, lj, s.excl_ptr, s.excl_idx, s.box, p)
    return float(np.sum(G * f) + np.dot(gE, e))


def _fd(fun, arr, idx, h):
    """Central difference along one float32 entry, dividing by the exact float32 step."""
    ap, am = arr.copy(), arr.copy()
    ap[idx] = np.float32(arr[idx] + h)
    am[idx] = np.float32(arr[idx] - h)
    return (fun(ap) - fun(am)) / (np.float64(ap[idx]) - np.float64(am[idx]))


def _far_from_cutoff(s, rc=1.0, margin=1e-4):
    x = s.x.astype(np.float64)
    L = s.box.astype(np.float64)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=-1)
    return not np.any(np.abs(r - rc) < margin)


def _frozen_system(seed, n, box, **kw):
    """A small system with no pair within 1e-4 nm of the cut-off, so finite differences
    with steps below that see a frozen pair set."""
    for k in range(100):
        s = small_random_system(seed + 1000 * k, n, box, min_dist=0.22, **kw)
        if _far_from_cutoff(s):
            return s
    raise RuntimeError("no frozen-set system found")


@pytest.mark.parametrize("coul", ["rf", "ewald"])
def test_backward_matches_finite_differences(oracle_mod, coul):
    o = oracle_mod
    s = _frozen_system(7, 45, 2.6)
    p = _params(o, coul)
    rng = np.random.default_rng(2)
    G = rng.normal(size=(s.n, 3))
    gE = np.array([0.7, -1.3])
    gx, gq, gl = o.backward(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p, G, gE)
    h = 2.0 ** -16
    for a in rng.choice(s.n, 5, replace=False):
        for k in range(3):
            fd = _fd(lambda xx: linear_loss(o, s, p, G, gE, x=xx), s.x, (a, k), h)
            assert fd == pytest.approx(gx[a, k], rel=2e-5, abs=1e-6 * np.abs(gx).max())
        fd = _fd(lambda qq: linear_loss(o, s, p, G, gE, q=qq), s.q, a, 2.0 ** -14)
        assert fd == pytest.approx(gq[a], rel=1e-6, abs=1e-9 * np.abs(gq).max())
    # table entries: the table is used as given (ordered type pairs)
    T = s.lj.shape[0]
    for t1 in range(T):
        for t2 in range(T):
            for c in range(2):
                hh = float(s.lj[t1, t2, c]) * 2.0 ** -12
                fd = _fd(lambda L: linear_loss(o, s, p, G, gE, lj=L), s.lj, (t1, t2, c), hh)
                assert fd == pytest.approx(gl[t1, t2, c], rel=1e-5,
                                           abs=1e-9 * np.abs(gl[..., c]).max())


def test_hessian_symmetry_linearity_and_zero(oracle_mod):
    o = oracle_mod
    s = small_random_system(8, 60, 2.6)
    p = _params(o, "ewald")
    rng = np.random.default_rng(5)
    G1, G2 = rng.normal(size=(s.n, 3)), rng.normal(size=(s.n, 3))
    z = np.zeros(2)
    args = (s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
    g1 = o.backward(*args, G1, z)[0]
    g2 = o.backward(*args, G2, z)[0]
    # grad_x of G.F is -H G with H the (symmetric) Hessian of the energy
    assert np.sum(G2 * g1) == pytest.approx(np.sum(G1 * g2), rel=1e-10)
    g12 = o.backward(*args, 2.0 * G1 - 3.0 * G2, z)
    assert np.allclose(g12[0], 2.0 * g1 - 3.0 * g2, rtol=1e-10, atol=1e-8 * np.abs(g1).max())
    g0 = o.backward(*args, np.zeros((s.n, 3)), z)
    assert all(np.all(a == 0) for a in g0)
    # translation invariance: the Hessian maps a uniform G to zero
    gu = o.backward(*args, np.tile([1.0, -2.0, 0.5], (s.n, 1)), z)[0]
    assert np.abs(gu).max() < 1e-9 * np.abs(g1).max()


def test_force_matching_loss_gradient(oracle_mod):
    """Loss sum |F(theta) - F_ref|^2 with F_ref from parameters scaled by 1.05: the
    chain rule through G = 2 (F - F_ref) agrees with finite differences of the loss."""
    o = oracle_mod
    s = _frozen_system(13, 48, 2.5, n_types=3)
    p = _params(o, "rf")
    q_ref = (s.q * np.float32(1.05)).astype(np.float32)
    lj_ref = (s.lj * np.float32(1.05)).astype(np.float32)
    _, f_ref, _ = o.forces(s.x, q_ref, s.type, lj_ref, s.excl_ptr, s.excl_idx, s.box, p)

    def loss(x=None, q=None, lj=None):
        x = s.x if x is None else x
        q = s.q if q is None else q
        lj = s.lj if lj is None else lj
        _, f, _ = o.forces(x, q, s.type, lj, s.excl_ptr, s.excl_idx, s.box, p)
        return float(np.sum((f - f_ref) ** 2))

    _, f, _ = o.forces(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p)
    G = 2.0 * (f - f_ref)
    gx, gq, gl = o.backward(s.x, s.q, s.type, s.lj, s.excl_ptr, s.excl_idx, s.box, p, G)
    rng = np.random.default_rng(9)
    for a in rng.choice(s.n, 4, replace=False):
        k = int(rng.integers(3))
        fd = _fd(lambda xx: loss(x=xx), s.x, (a, k), 2.0 ** -17)
        assert fd == pytest.approx(gx[a, k], rel=1e-4, abs=1e-6 * np.abs(gx).max())
        fd = _fd(lambda qq: loss(q=qq), s.q, a, 2.0 ** -16)
        assert fd == pytest.approx(gq[a], rel=1e-5, abs=1e-8 * np.abs(gq).max())
    fd = _fd(lambda L: loss(lj=L), s.lj, (1, 2, 1), float(s.lj[1, 2, 1]) * 2.0 ** -12)
    assert fd == pytest.approx(gl[1, 2, 1], rel=1e-4)
