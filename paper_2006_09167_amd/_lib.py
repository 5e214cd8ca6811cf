"""ctypes declarations of the C ABI in include/nb.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnbmi.so")

NB_OK, NB_ERR_ARG, NB_ERR_BOX, NB_ERR_NOMEM, NB_ERR_CAPACITY, NB_ERR_STATE, NB_ERR_HIP, \
    NB_ERR_NONFINITE = range(8)
NB_COUL_RF, NB_COUL_EWALD, NB_COUL_NONE = 0, 1, 2
NB_MOD_NONE, NB_MOD_POTSHIFT = 0, 1
NB_F_ENERGY, NB_F_VIRIAL, NB_F_ACCUMULATE, NB_F_EXCL_CORR = 1, 2, 4, 8

EXPORTS = ["nb_create", "nb_destroy", "nb_set_topology", "nb_grid_build", "nb_pairlist_build",
           "nb_prune_rolling", "nb_forces", "nb_step", "nb_forces_backward", "nb_get_grid",
           "nb_get_grid_dims", "nb_get_pairs", "nb_get_stats", "nb_set_timing", "nb_get_timing",
           "nb_strerror", "nb_last_error", "nb_step_graph", "nb_set_exec", "nb_get_exec",
           "nb_autotune", "nb_list_census", "nb_list_coverage", "nb_buffer_drift",
           "nb_buffer_estimate", "nb_list_census_noalloc"]
NB_EXEC_STATIC, NB_EXEC_XCD, NB_EXEC_QUEUE, NB_EXEC_PERSIST, NB_EXEC_BALANCED = 0, 1, 2, 3, 4
NB_PRUNE_SEPARATE, NB_PRUNE_FUSED, NB_PRUNE_AHEAD = 0, 1, 2
EXEC_MODES = {"static": NB_EXEC_STATIC, "xcd": NB_EXEC_XCD, "queue": NB_EXEC_QUEUE,
              "persist": NB_EXEC_PERSIST, "balanced": NB_EXEC_BALANCED}
(NB_T_FORCES, NB_T_FORCE_REDUCE, NB_T_PRUNE, NB_T_BACKWARD, NB_T_BACKWARD_REDUCE, NB_T_CENSUS,
 NB_T_COUNT) = range(7)
TIMING_KINDS = ["forces", "force_reduce", "prune", "backward", "backward_reduce", "census"]
NB_CENSUS_MAX_RADII = 64
CENSUS_SIZES = (1, 2, 4, 8)


class NbParams(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int32), ("coulomb", ctypes.c_int32),
                ("modifier", ctypes.c_int32), ("rc", ctypes.c_float),
                ("rinner", ctypes.c_float), ("rlist", ctypes.c_float),
                ("eps_r", ctypes.c_float), ("eps_rf", ctypes.c_float),
                ("ewald_beta", ctypes.c_float), ("epsfac", ctypes.c_float),
                ("nstlist", ctypes.c_int32), ("nstprune", ctypes.c_int32),
                ("list_capacity_hint", ctypes.c_int64)]


class NbBufferInput(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("count", ctypes.c_void_p),
                ("mass", ctypes.c_void_p), ("charge", ctypes.c_void_p),
                ("type", ctypes.c_void_p), ("lj", ctypes.c_void_p),
                ("volume", ctypes.c_double), ("temperature", ctypes.c_double),
                ("dt", ctypes.c_double), ("n_cov", ctypes.c_int32),
                ("cov_radii", ctypes.c_void_p), ("covered", ctypes.c_void_p),
                ("rot_len", ctypes.c_void_p), ("rot_mass", ctypes.c_void_p)]


class NbStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_atoms", "n_slots", "n_superclusters", "n_clusters", "n_entries", "n_work_items",
        "outer_pairs", "inner_pairs", "bb_pairs", "n_excl_rows", "effective_pairs",
        "computed_pairs", "grid_columns", "capacity_per_sc", "regrows")]


class NbExecConfig(ctypes.Structure):
    _fields_ = [("item_width", ctypes.c_int32), ("exec_mode", ctypes.c_int32),
                ("prune_fused", ctypes.c_int32), ("prune_waves", ctypes.c_int32),
                ("us_per_call", ctypes.c_double)]


_lib = None


def load():
    """Load libnbmi.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnbmi.so is not built; run `python -c \"import __graft_entry__ as g; "
                          "g.build()\"` or `python paper_2006_09167_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    st = ctypes.c_int
    sig = {
        "nb_create": ([ctypes.POINTER(NbParams), i32, P, P, ctypes.POINTER(P)], st),
        "nb_destroy": ([P], None),
        "nb_set_topology": ([P, P, P, P], st),
        "nb_grid_build": ([P, P, P], st),
        "nb_pairlist_build": ([P], st),
        "nb_prune_rolling": ([P, P, i64], st),
        "nb_forces": ([P, P, P, P, P, P, P, u32], st),
        "nb_step": ([P, P, P, P, P, P, P, u32, i64], st),
        "nb_step_graph": ([P, P, P, P, P, P, P, u32, i64], st),
        "nb_set_exec": ([P, i32, i32, i32, i32], st),
        "nb_get_exec": ([P, ctypes.POINTER(NbExecConfig)], st),
        "nb_autotune": ([P, P, P, P, u32, i32, P, i32, ctypes.POINTER(i32),
                         ctypes.POINTER(NbExecConfig)], st),
        "nb_forces_backward": ([P, P, P, P, P, P, P, P, P, u32], st),
        "nb_get_grid": ([P, P, i64, ctypes.POINTER(i64)], st),
        "nb_get_grid_dims": ([P, P], st),
        "nb_get_pairs": ([P, i32, P, i64, ctypes.POINTER(i64)], st),
        "nb_get_stats": ([P, ctypes.POINTER(NbStats)], st),
        "nb_set_timing": ([P, i32], st),
        "nb_get_timing": ([P, P, P], st),
        "nb_list_census": ([P, i32, P, P], st),
        "nb_list_census_noalloc": ([P, i32, P, P], st),
        "nb_list_coverage": ([P, i32, i32, i32, P, P], st),
        "nb_buffer_drift": ([ctypes.POINTER(NbParams), ctypes.POINTER(NbBufferInput), i32,
                             ctypes.c_double, ctypes.POINTER(ctypes.c_double)], st),
        "nb_buffer_estimate": ([ctypes.POINTER(NbParams), ctypes.POINTER(NbBufferInput), i32,
                                ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                               st),
        "nb_strerror": ([st], ctypes.c_char_p),
        "nb_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib
