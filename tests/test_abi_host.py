"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
function include/nb.h declares, its structs match the header, and argument/state
validation returns the documented status before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2006_09167_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "nb.h")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z_]+)\s*\(", src)))


def test_header_declarations_are_exported():
    lib = _lib.load()
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layout_matches_header():
    # nb_params: 3 int32, 7 float, 2 int32, int64 -> 4*12 = 48 bytes, then 8-aligned int64
    assert ctypes.sizeof(_lib.NbParams) == 56
    assert ctypes.sizeof(_lib.NbStats) == 15 * 8


def good_params(**kw):
    p = dict(n_types=2, coulomb=_lib.NB_COUL_RF, modifier=_lib.NB_MOD_POTSHIFT, rc=1.0,
             rinner=1.0, rlist=1.1, eps_r=1.0, eps_rf=math.inf, ewald_beta=0.0,
             epsfac=138.935458, nstlist=10, nstprune=2, list_capacity_hint=0)
    p.update(kw)
    return _lib.NbParams(**p)


def create(params, offsets=(0, 10)):
    lib = _lib.load()
    offs = np.asarray(offsets, dtype=np.int64)
    h = ctypes.c_void_p()
    st = lib.nb_create(ctypes.byref(params), offs.size - 1, offs.ctypes.data_as(ctypes.c_void_p),
                       None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("bad", [
    dict(rc=0.0), dict(rc=-1.0), dict(rc=float("nan")), dict(rinner=0.9),
    dict(rlist=0.95), dict(n_types=0), dict(n_types=33), dict(coulomb=7), dict(modifier=3),
    dict(eps_r=0.0), dict(eps_rf=0.0), dict(coulomb=_lib.NB_COUL_EWALD, ewald_beta=0.0),
    dict(nstlist=0), dict(nstprune=0), dict(list_capacity_hint=-1), dict(epsfac=float("inf")),
])
def test_create_rejects_bad_parameters(bad):
    st, h = create(good_params(**bad))
    assert st == _lib.NB_ERR_ARG
    assert not h.value


def test_create_rejects_bad_offsets():
    assert create(good_params(), offsets=(1, 10))[0] == _lib.NB_ERR_ARG
    assert create(good_params(), offsets=(0, 10, 5))[0] == _lib.NB_ERR_ARG


def test_state_and_topology_errors_without_device():
    lib = _lib.load()
    st, h = create(good_params(), offsets=(0, 4))
    assert st == _lib.NB_OK and h.value
    try:
        box = np.full(3, 3.0, np.float32)
        # grid before topology, list before grid, prune/forces before list
        assert lib.nb_grid_build(h, ctypes.c_void_p(1), box.ctypes.data_as(ctypes.c_void_p)) \
            == _lib.NB_ERR_STATE
        assert lib.nb_pairlist_build(h) == _lib.NB_ERR_STATE
        assert lib.nb_prune_rolling(h, ctypes.c_void_p(1), 1) == _lib.NB_ERR_STATE
        assert lib.nb_forces(h, None, None, None, None, None, None, 0) == _lib.NB_ERR_STATE
        assert lib.nb_forces_backward(h, None, None, None, None, None, None, None, None, 0) \
            == _lib.NB_ERR_STATE
        assert b"no pair list" in lib.nb_last_error(h)
        # census: arguments checked first, then the list
        r = np.array([0.5], np.float32)
        cnt = np.zeros(16, np.int64)
        vpp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert lib.nb_list_census(h, 1, vpp(r), vpp(cnt)) == _lib.NB_ERR_STATE
        assert lib.nb_list_census(h, 0, vpp(r), vpp(cnt)) == _lib.NB_ERR_ARG
        assert lib.nb_list_census(h, _lib.NB_CENSUS_MAX_RADII + 1, vpp(r), vpp(cnt)) \
            == _lib.NB_ERR_ARG
        assert lib.nb_list_census(h, 1, None, vpp(cnt)) == _lib.NB_ERR_ARG
        assert lib.nb_list_census(None, 1, vpp(r), vpp(cnt)) == _lib.NB_ERR_ARG
        # topology validation happens before any device call
        t = np.array([0, 1, 2, 0], np.int32)                     # type 2 >= n_types
        ptr = np.zeros(5, np.int64)
        idx = np.zeros(0, np.int32)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert lib.nb_set_topology(h, vp(t), vp(ptr), vp(idx)) == _lib.NB_ERR_ARG
        t = np.array([0, 1, 1, 0], np.int32)
        ptr = np.array([0, 1, 1, 1, 1], np.int64)
        idx = np.array([7], np.int32)                            # partner out of range
        assert lib.nb_set_topology(h, vp(t), vp(ptr), vp(idx)) == _lib.NB_ERR_ARG
        ptr = np.array([0, 33, 33, 33, 33], np.int64)            # too many partners
        idx = np.zeros(33, np.int32)
        assert lib.nb_set_topology(h, vp(t), vp(ptr), vp(idx)) == _lib.NB_ERR_ARG
    finally:
        lib.nb_destroy(h)


def test_null_arguments():
    lib = _lib.load()
    assert lib.nb_create(None, 1, None, None, None) == _lib.NB_ERR_ARG
    assert lib.nb_pairlist_build(None) == _lib.NB_ERR_ARG
    assert lib.nb_get_stats(None, None) == _lib.NB_ERR_ARG
    lib.nb_destroy(None)
    for s in range(8):
        assert lib.nb_strerror(s)


def test_cross_system_exclusion_rejected():
    lib = _lib.load()
    st, h = create(good_params(), offsets=(0, 2, 4))
    assert st == _lib.NB_OK
    try:
        t = np.zeros(4, np.int32)
        ptr = np.array([0, 1, 2, 3, 4], np.int64)
        idx = np.array([1, 0, 0, 2], np.int32)                   # atom 2 excludes atom 0
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert lib.nb_set_topology(h, vp(t), vp(ptr), vp(idx)) == _lib.NB_ERR_ARG
    finally:
        lib.nb_destroy(h)


def test_exec_shape_validation_without_device():
    lib = _lib.load()
    st, h = create(good_params(), offsets=(0, 4))
    assert st == _lib.NB_OK
    try:
        assert ctypes.sizeof(_lib.NbExecConfig) == 24
        assert lib.nb_set_exec(h, -1, _lib.NB_EXEC_STATIC, 1, 0) == _lib.NB_ERR_ARG
        assert lib.nb_set_exec(h, 65, _lib.NB_EXEC_STATIC, 1, 0) == _lib.NB_ERR_ARG
        assert lib.nb_set_exec(h, 16, 5, 1, 0) == _lib.NB_ERR_ARG
        assert lib.nb_set_exec(h, 16, _lib.NB_EXEC_BALANCED, 1, 0) == _lib.NB_OK
        assert lib.nb_set_exec(h, 16, -1, 1, 0) == _lib.NB_ERR_ARG
        assert lib.nb_set_exec(h, 16, _lib.NB_EXEC_PERSIST, 1, 0) == _lib.NB_OK
        assert lib.nb_set_exec(h, 16, _lib.NB_EXEC_STATIC, 3, 0) == _lib.NB_ERR_ARG
        assert lib.nb_set_exec(h, 16, _lib.NB_EXEC_STATIC, _lib.NB_PRUNE_AHEAD, 0) == _lib.NB_OK
        assert lib.nb_set_exec(h, 16, _lib.NB_EXEC_QUEUE, 0, 0) == _lib.NB_OK
        cfg = _lib.NbExecConfig()
        assert lib.nb_get_exec(h, ctypes.byref(cfg)) == _lib.NB_OK
        assert (cfg.item_width, cfg.exec_mode, cfg.prune_fused) == (16, _lib.NB_EXEC_QUEUE, 0)
        for w, ok in [(1, True), (2, True), (4, True), (8, True), (3, False), (16, False),
                      (-1, False)]:
            assert (lib.nb_set_exec(h, 16, _lib.NB_EXEC_STATIC, 0, w) == _lib.NB_OK) == ok
        assert lib.nb_get_exec(h, ctypes.byref(cfg)) == _lib.NB_OK
        assert (cfg.exec_mode, cfg.prune_waves) == (_lib.NB_EXEC_STATIC, 8)
        n = ctypes.c_int32(0)
        best = _lib.NbExecConfig()
        assert lib.nb_autotune(h, None, None, None, 1, 3, None, 0, ctypes.byref(n),
                               ctypes.byref(best)) == _lib.NB_ERR_STATE
        assert lib.nb_step_graph(h, None, None, None, None, None, None, 0, 1) \
            == _lib.NB_ERR_STATE
        assert lib.nb_get_exec(h, None) == _lib.NB_ERR_ARG
    finally:
        lib.nb_destroy(h)


def test_asymmetric_exclusions_rejected():
    """Exclusion masks are built from each atom's own row, so the list must be symmetric:
    atom 0 lists atom 1 but atom 1 does not list atom 0."""
    lib = _lib.load()
    st, h = create(good_params(), offsets=(0, 3))
    assert st == _lib.NB_OK
    try:
        t = np.zeros(3, np.int32)
        ptr = np.array([0, 1, 2, 3], np.int64)
        idx = np.array([1, 2, 1], np.int32)          # 0->1, 1->2, 2->1: 1 lacks 0
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert lib.nb_set_topology(h, vp(t), vp(ptr), vp(idx)) == _lib.NB_ERR_ARG
        assert b"symmetric" in lib.nb_last_error(h)
    finally:
        lib.nb_destroy(h)


def test_get_pairs_argument_and_state_errors():
    lib = _lib.load()
    st, h = create(good_params(), offsets=(0, 4))
    assert st == _lib.NB_OK
    try:
        n = ctypes.c_int64(0)
        for which in (0, 1, 2):
            assert lib.nb_get_pairs(h, which, None, 0, ctypes.byref(n)) == _lib.NB_ERR_STATE
        for which in (-1, 3):
            assert lib.nb_get_pairs(h, which, None, 0, ctypes.byref(n)) == _lib.NB_ERR_ARG
    finally:
        lib.nb_destroy(h)
