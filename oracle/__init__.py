"""FP64 CPU oracle for the cluster-pair nonbonded path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark import this package; the product library never does, and the two
share no code (only the seeded input generators feed both).

Contents
  * ``nb_oracle.c`` (built here with gcc into ``_nb_oracle.so``): brute-force
    minimum-image energies, forces, virial and backward pass in FP64 (and the same
    energies, forces and virial through a cell grid for large boxes), and the
    brute-force cluster-pair sets in a fixed single-precision sequence;
  * ``grid_spec.py``: the grid / slot assignment written out with numpy;
  * this module: ctypes wrappers, the pair-list set algebra (outer list, inner
    list by rolling part) and finite-difference helpers;
  * ``census.py``: the work-efficiency census of M x N sub-cluster lists (Fig. 5);
  * ``buffer.py``: list coverage by sub-cluster pairs and the Verlet buffer estimate.

Every function cites the part of the paper it follows (see the C file header).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

from . import grid_spec  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nb_oracle.c")
_LIB = os.path.join(_HERE, "_nb_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
               "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("coulomb", ctypes.c_int32), ("modifier", ctypes.c_int32),
                ("rc", ctypes.c_double), ("eps_r", ctypes.c_double),
                ("eps_rf", ctypes.c_double), ("beta", ctypes.c_double),
                ("epsfac", ctypes.c_double), ("excl_corr", ctypes.c_int32)]


def params(coulomb: str = "rf", rc: float = 1.0, eps_r: float = 1.0, eps_rf: float = math.inf,
           beta: float = 0.0, epsfac: float = 138.935458, modifier: str = "potshift",
           excl_corr: bool = False) -> Params:
    """Oracle parameters.  Cut-offs are taken as the float32 values the GPU receives.
    excl_corr: excluded pairs inside rc and each atom with itself carry the electrostatic
    corrections of a run with a long-range part (Sec. V.A)."""
    return Params(coulomb={"rf": 0, "ewald": 1}[coulomb],
                  modifier={"none": 0, "potshift": 1}[modifier],
                  rc=float(np.float32(rc)), eps_r=float(np.float32(eps_r)),
                  eps_rf=float(np.float32(eps_rf)), beta=float(np.float32(beta)),
                  epsfac=float(np.float32(epsfac)), excl_corr=1 if excl_corr else 0)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_forces.argtypes = [i64, P, P, P, ctypes.c_int32, P, P, P, P,
                                      ctypes.POINTER(Params), P, P, P, P]
        lib.oracle_forces_cells.argtypes = [i64, P, P, P, ctypes.c_int32, P, P, P, P,
                                            ctypes.POINTER(Params), P, P, P, P]
        lib.oracle_forces_on.argtypes = [i64, P, P, P, ctypes.c_int32, P, P, P, P,
                                         ctypes.POINTER(Params), i64, P, P]
        lib.oracle_backward.argtypes = [i64, P, P, P, ctypes.c_int32, P, P, P, P,
                                        ctypes.POINTER(Params), P, P, P, P, P]
        lib.oracle_cluster_pairs.argtypes = [i64, P, P, P, ctypes.c_float, i64, i64, P, i64]
        lib.oracle_cluster_pairs.restype = i64
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (for single-thread timings)."""
    _load().oracle_set_num_threads(int(n))


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def forces(x, q, type_, lj, excl_ptr, excl_idx, box, p: Params, energy_abs: bool = False):
    """FP64 all-pairs minimum-image energies [E_LJ, E_C], forces [N,3] and virial [3,3];
    with energy_abs also the sums of |pair energy| [LJ, Coulomb]."""
    x, q, t = _c(x, np.float32), _c(q, np.float32), _c(type_, np.int32)
    lj = _c(lj, np.float32)
    ep, ei, box = _c(excl_ptr, np.int64), _c(excl_idx, np.int32), _c(box, np.float32)
    n = x.shape[0]
    f = np.zeros((n, 3), dtype=np.float64)
    e = np.zeros(2, dtype=np.float64)
    v = np.zeros(9, dtype=np.float64)
    ea = np.zeros(2, dtype=np.float64)
    rc = _load().oracle_forces(n, _ptr(x), _ptr(q), _ptr(t), lj.shape[0], _ptr(lj), _ptr(ep),
                               _ptr(ei), _ptr(box), ctypes.byref(p), _ptr(f), _ptr(e), _ptr(v),
                               _ptr(ea))
    if rc != 0:
        raise MemoryError("oracle_forces failed")
    if energy_abs:
        return e, f, v.reshape(3, 3), ea
    return e, f, v.reshape(3, 3)


def forces_cells(x, q, type_, lj, excl_ptr, excl_idx, box, p: Params, energy_abs: bool = False):
    """The results of ``forces`` summed through a cell grid (each atom against the atoms
    of its 27 neighbouring cells, cells at least rc wide): linear in N, for the boxes whose
    all-pairs sum is too slow.  Falls back to ``forces`` below three cells per axis."""
    x, q, t = _c(x, np.float32), _c(q, np.float32), _c(type_, np.int32)
    lj = _c(lj, np.float32)
    ep, ei, box = _c(excl_ptr, np.int64), _c(excl_idx, np.int32), _c(box, np.float32)
    n = x.shape[0]
    f = np.zeros((n, 3), dtype=np.float64)
    e = np.zeros(2, dtype=np.float64)
    v = np.zeros(9, dtype=np.float64)
    ea = np.zeros(2, dtype=np.float64)
    rc = _load().oracle_forces_cells(n, _ptr(x), _ptr(q), _ptr(t), lj.shape[0], _ptr(lj),
                                     _ptr(ep), _ptr(ei), _ptr(box), ctypes.byref(p), _ptr(f),
                                     _ptr(e), _ptr(v), _ptr(ea))
    if rc != 0:
        raise MemoryError("oracle_forces_cells failed")
    if energy_abs:
        return e, f, v.reshape(3, 3), ea
    return e, f, v.reshape(3, 3)


def forces_on(sel, x, q, type_, lj, excl_ptr, excl_idx, box, p: Params):
    """FP64 forces on the selected atoms only."""
    x, q, t = _c(x, np.float32), _c(q, np.float32), _c(type_, np.int32)
    lj = _c(lj, np.float32)
    ep, ei, box = _c(excl_ptr, np.int64), _c(excl_idx, np.int32), _c(box, np.float32)
    sel = _c(sel, np.int64)
    out = np.zeros((sel.shape[0], 3), dtype=np.float64)
    _load().oracle_forces_on(x.shape[0], _ptr(x), _ptr(q), _ptr(t), lj.shape[0], _ptr(lj),
                             _ptr(ep), _ptr(ei), _ptr(box), ctypes.byref(p), sel.shape[0],
                             _ptr(sel), _ptr(out))
    return out


def backward(x, q, type_, lj, excl_ptr, excl_idx, box, p: Params, G, gE=(0.0, 0.0)):
    """FP64 gradients (grad_x [N,3], grad_q [N], grad_lj [T,T,2]) of a loss with
    dL/dF = G and dL/dE = gE over the frozen pair set inside the cut-off.  The
    table gradient is per ordered type pair (t_a, t_b) with a < b; a symmetric
    table's gradient is the sum of [t1,t2] and [t2,t1] on each off-diagonal."""
    x, q, t = _c(x, np.float32), _c(q, np.float32), _c(type_, np.int32)
    lj = _c(lj, np.float32)
    ep, ei, box = _c(excl_ptr, np.int64), _c(excl_idx, np.int32), _c(box, np.float32)
    G = _c(G, np.float64)
    gE = _c(gE, np.float64)
    n, T = x.shape[0], lj.shape[0]
    gx = np.zeros((n, 3), dtype=np.float64)
    gq = np.zeros(n, dtype=np.float64)
    gl = np.zeros((T, T, 2), dtype=np.float64)
    rc = _load().oracle_backward(n, _ptr(x), _ptr(q), _ptr(t), T, _ptr(lj), _ptr(ep), _ptr(ei),
                                 _ptr(box), ctypes.byref(p), _ptr(G), _ptr(gE), _ptr(gx),
                                 _ptr(gq), _ptr(gl))
    if rc != 0:
        raise MemoryError("oracle_backward failed")
    return gx, gq, gl


# ---------------------------------------------------------------------------------------
# Cluster-pair sets (Sec. V.A, V.D, V.E).
# ---------------------------------------------------------------------------------------
def cluster_pairs(slot_atom, w, box, R: float, ci_lo: int = 0, ci_hi: Optional[int] = None):
    """Sorted unique keys (ci * n_clusters + cj) * 27 + shift_code of every canonical
    cluster pair holding an atom pair with single-precision r2 < float32(R^2).
    ``w`` are the wrapped single-precision coordinates per atom (user order)."""
    slot_atom = _c(slot_atom, np.int32)
    w, box = _c(w, np.float32), _c(box, np.float32)
    n_slots = slot_atom.shape[0]
    n_cl = n_slots // 8
    if ci_hi is None:
        ci_hi = n_cl
    R2 = np.float32(np.float64(np.float32(R)) ** 2)
    cap = 1 << 16
    while True:
        out = np.empty(cap, dtype=np.int64)
        cnt = _load().oracle_cluster_pairs(n_slots, _ptr(slot_atom), _ptr(w), _ptr(box),
                                           ctypes.c_float(R2), ci_lo, ci_hi, _ptr(out), cap)
        if cnt >= 0:
            return np.unique(out[:cnt])
        cap = int(-cnt) + 1024


def radius_sq_f32(R: float) -> np.float32:
    """The single-precision squared radius a list decision compares against."""
    return np.float32(np.float64(np.float32(R)) ** 2)


def split_key(keys: np.ndarray, n_clusters: int):
    keys = np.asarray(keys, dtype=np.int64)
    code = keys % 27
    pair = keys // 27
    return pair // n_clusters, pair % n_clusters, code


def inner_pairs(outer_keys, slot_atom, w_prune, box, r_inner, n_parts: int, part: Optional[int],
                ci_lo: int = 0, ci_hi: Optional[int] = None):
    """Members of the outer list whose owner super-cluster (min cluster // 8) is in
    ``part`` (all parts when None) and that hold an atom pair within r_inner at the
    prune positions ``w_prune`` (wrapped with the build-time image offsets)."""
    n_cl = np.asarray(slot_atom).shape[0] // 8
    close = cluster_pairs(slot_atom, w_prune, box, r_inner, ci_lo, ci_hi)
    keys = np.intersect1d(np.asarray(outer_keys, dtype=np.int64), close)
    if part is not None:
        ci, _, _ = split_key(keys, n_cl)
        keys = keys[(ci // 8) % n_parts == part]
    return keys


def rewrap_with(x: np.ndarray, k: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Positions of a later step expressed with the build-time image offsets k,
    in the same single-precision sequence as the wrap: x - k * L."""
    L = np.asarray(box, dtype=np.float32)
    return (np.asarray(x, dtype=np.float32)
            - (k.astype(np.float32) * L).astype(np.float32)).astype(np.float32)


from . import census  # noqa: E402,F401  (work-efficiency census; uses the functions above)
from . import buffer  # noqa: E402,F401  (Verlet buffer estimate and list coverage)
