"""Python binding of the cluster-pair nonbonded library (torch supplies device memory and
the stream; every step of the path runs in the HIP kernels of libnbmi.so).

    ctx = Context(n_types=2, coulomb="ewald", rc=1.0, rinner=1.04, rlist=1.1, beta=3.12,
                  nstlist=100, nstprune=4, atom_offsets=[0, N])
    ctx.set_topology(types, excl_ptr, excl_idx)
    ctx.grid_build(x, box); ctx.pairlist_build()
    f, e, vir = ctx.forces(x, q, lj, energy=True)
    ctx.prune_rolling(x, steps_since_build)
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (EXEC_MODES, NB_F_ACCUMULATE, NB_F_ENERGY, NB_F_EXCL_CORR, NB_F_VIRIAL,
                   NbExecConfig)

_MODE_NAMES = {v: k for k, v in EXEC_MODES.items()}


class NBError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_lib.load().nb_strerror(status).decode(), message))
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_params(n_types: int, coulomb: str = "rf", rc: float = 1.0,
                rinner: Optional[float] = None, rlist: Optional[float] = None,
                eps_r: float = 1.0, eps_rf: float = math.inf, beta: float = 0.0,
                epsfac: float = 138.935458, modifier: str = "potshift", nstlist: int = 1,
                nstprune: int = 1, capacity_hint: int = 0) -> _lib.NbParams:
    rinner = rc if rinner is None else rinner
    rlist = rinner if rlist is None else rlist
    return _lib.NbParams(n_types=n_types,
                         coulomb={"rf": _lib.NB_COUL_RF, "ewald": _lib.NB_COUL_EWALD,
                                  "none": _lib.NB_COUL_NONE}[coulomb],
                         modifier={"none": _lib.NB_MOD_NONE,
                                   "potshift": _lib.NB_MOD_POTSHIFT}[modifier],
                         rc=rc, rinner=rinner, rlist=rlist, eps_r=eps_r, eps_rf=eps_rf,
                         ewald_beta=beta, epsfac=epsfac, nstlist=nstlist, nstprune=nstprune,
                         list_capacity_hint=capacity_hint)


def _prune_code(prune_fused) -> int:
    """nb_exec_config.prune_fused from True / False / "ahead"."""
    if isinstance(prune_fused, str):
        if prune_fused != "ahead":
            raise ValueError("prune_fused is True, False or 'ahead'")
        return _lib.NB_PRUNE_AHEAD
    return 1 if prune_fused else 0


def _prune_name(code: int):
    return "ahead" if code == _lib.NB_PRUNE_AHEAD else bool(code)


class _BufferArgs:
    """Marshalled nb_buffer_input (keeps the arrays alive; checks the sizes the library
    reads: one entry per class in every class array, an n_types x n_types x 2 table, a
    square coverage table)."""

    def __init__(self, params, classes: dict, lj, volume, temperature, dt, coverage=None):
        self.count = np.ascontiguousarray(classes["count"], dtype=np.int64).reshape(-1)
        self.mass = np.ascontiguousarray(classes["mass"], dtype=np.float64).reshape(-1)
        self.charge = np.ascontiguousarray(classes["charge"], dtype=np.float32).reshape(-1)
        self.type = np.ascontiguousarray(classes["type"], dtype=np.int32).reshape(-1)
        n = self.count.size
        if not (self.mass.size == self.charge.size == self.type.size == n):
            raise ValueError("class arrays count, mass, charge, type differ in length")
        self.rot_len = self.rot_mass = None
        if classes.get("rot_len") is not None:
            self.rot_len = np.ascontiguousarray(classes["rot_len"], dtype=np.float64).reshape(-1)
            self.rot_mass = np.ascontiguousarray(classes["rot_mass"],
                                                 dtype=np.float64).reshape(-1)
            if not (self.rot_len.size == self.rot_mass.size == n):
                raise ValueError("class arrays rot_len, rot_mass differ in length")
        self.lj = np.ascontiguousarray(np.asarray(lj, dtype=np.float32))
        if self.lj.size != 2 * params.n_types * params.n_types:
            raise ValueError("lj must hold (c6, c12) for n_types x n_types type pairs")
        n_cov, R, C = 0, None, None
        if coverage is not None:
            R = np.ascontiguousarray(coverage[0], dtype=np.float32).reshape(-1)
            C = np.ascontiguousarray(coverage[1], dtype=np.int64)
            if C.shape != (R.size, R.size):
                raise ValueError("coverage table must be [len(radii), len(radii)]")
            n_cov = int(R.size)
        self.R, self.C = R, C
        self.s = _lib.NbBufferInput(
            n_classes=int(self.count.size), count=_np_ptr(self.count), mass=_np_ptr(self.mass),
            charge=_np_ptr(self.charge), type=_np_ptr(self.type), lj=_np_ptr(self.lj),
            volume=float(volume), temperature=float(temperature), dt=float(dt), n_cov=n_cov,
            cov_radii=_np_ptr(R) if R is not None else None,
            covered=_np_ptr(C) if C is not None else None,
            rot_len=_np_ptr(self.rot_len) if self.rot_len is not None else None,
            rot_mass=_np_ptr(self.rot_mass) if self.rot_mass is not None else None)


def buffer_drift(params, classes: dict, lj, volume: float, temperature: float, dt: float,
                 steps: int, r_list: float, coverage=None) -> float:
    """Drift (kJ/mol/ps per atom) of a list at r_list used for `steps` steps
    (nb_buffer_drift).  classes: arrays count, mass, charge, type, and optionally rot_len,
    rot_mass (atoms that rotate about a constraint partner: the distance to it and their own
    mass); coverage: (radii, covered) from Context.list_coverage, or None for a particle
    list."""
    lib = _lib.load()
    a = _BufferArgs(params, classes, lj, volume, temperature, dt, coverage)
    out = ctypes.c_double()
    st = lib.nb_buffer_drift(ctypes.byref(params), ctypes.byref(a.s), int(steps),
                             float(r_list), ctypes.byref(out))
    if st != 0:
        raise NBError(st, "nb_buffer_drift")
    return out.value


def buffer_estimate(params, classes: dict, lj, volume: float, temperature: float, dt: float,
                    steps: int, tolerance: float = 0.005, max_buffer: float = 1.0,
                    coverage=None):
    """(list radius, its drift): the smallest radius within the drift tolerance
    (nb_buffer_estimate)."""
    lib = _lib.load()
    a = _BufferArgs(params, classes, lj, volume, temperature, dt, coverage)
    r, d = ctypes.c_double(), ctypes.c_double()
    st = lib.nb_buffer_estimate(ctypes.byref(params), ctypes.byref(a.s), int(steps),
                                float(tolerance), float(max_buffer), ctypes.byref(r),
                                ctypes.byref(d))
    if st != 0:
        raise NBError(st, "nb_buffer_estimate")
    return r.value, d.value


class Context:
    """One library context (one or several boxes) on one device and stream."""

    def __init__(self, n_types: int, coulomb: str = "rf", rc: float = 1.0,
                 rinner: Optional[float] = None, rlist: Optional[float] = None,
                 eps_r: float = 1.0, eps_rf: float = math.inf, beta: float = 0.0,
                 epsfac: float = 138.935458, modifier: str = "potshift", nstlist: int = 1,
                 nstprune: int = 1, capacity_hint: int = 0,
                 atom_offsets: Sequence[int] = (0,), device=None, stream=None):
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        p = make_params(n_types, coulomb, rc, rinner, rlist, eps_r, eps_rf, beta, epsfac,
                        modifier, nstlist, nstprune, capacity_hint)
        self.params = p
        self.offsets = np.ascontiguousarray(atom_offsets, dtype=np.int64)
        self.n_sys = self.offsets.size - 1
        self.n_atoms = int(self.offsets[-1])
        self.n_types = n_types
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            st = self.lib.nb_create(ctypes.byref(p), self.n_sys, _np_ptr(self.offsets),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise NBError(st, "nb_create")
        self.h = h

    # ---- helpers ------------------------------------------------------------------------
    def _check(self, st: int, what: str):
        if st != 0:
            msg = self.lib.nb_last_error(self.h)
            raise NBError(st, "%s: %s" % (what, msg.decode() if msg else ""))

    def _dev(self, t: torch.Tensor, shape, dtype, name) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError("%s must be a tensor on %s" % (name, self.device))
        if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of shape %s (got %s %s)"
                             % (name, dtype, tuple(shape), t.dtype, tuple(t.shape)))
        return t

    def close(self):
        if getattr(self, "h", None):
            self.lib.nb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- ABI calls -----------------------------------------------------------------------
    def set_topology(self, types, excl_ptr, excl_idx):
        t = np.ascontiguousarray(types, dtype=np.int32)
        ep = np.ascontiguousarray(excl_ptr, dtype=np.int64)
        ei = np.ascontiguousarray(excl_idx, dtype=np.int32)
        if t.shape != (self.n_atoms,) or ep.shape != (self.n_atoms + 1,):
            raise ValueError("topology arrays do not match the atom count")
        self._check(self.lib.nb_set_topology(self.h, _np_ptr(t), _np_ptr(ep), _np_ptr(ei)),
                    "nb_set_topology")

    def grid_build(self, x: torch.Tensor, box):
        x = self._dev(x, (self.n_atoms, 3), torch.float32, "x")
        b = np.ascontiguousarray(np.asarray(box, dtype=np.float32).reshape(self.n_sys, 3))
        self._box = b
        self._check(self.lib.nb_grid_build(self.h, _ptr(x), _np_ptr(b)), "nb_grid_build")

    def pairlist_build(self):
        self._check(self.lib.nb_pairlist_build(self.h), "nb_pairlist_build")

    def prune_rolling(self, x: torch.Tensor, steps_since_build: int):
        x = self._dev(x, (self.n_atoms, 3), torch.float32, "x")
        self._check(self.lib.nb_prune_rolling(self.h, _ptr(x), int(steps_since_build)),
                    "nb_prune_rolling")

    def forces(self, x, q, lj, energy: bool = True, virial: bool = False, f=None, e=None,
               vir=None, accumulate: bool = False, excl_corr: bool = False):
        """Returns (f [N,3] float32, energy [S,2] float64 or None, virial [S,3,3] or None).
        excl_corr adds the electrostatic corrections of excluded pairs and self terms."""
        x = self._dev(x, (self.n_atoms, 3), torch.float32, "x")
        q = self._dev(q, (self.n_atoms,), torch.float32, "q")
        lj = self._dev(lj, (self.n_types, self.n_types, 2), torch.float32, "lj")
        if f is None:
            f = torch.empty((self.n_atoms, 3), dtype=torch.float32, device=self.device)
        flags = 0
        if energy:
            flags |= NB_F_ENERGY
            if e is None:
                e = torch.empty((self.n_sys, 2), dtype=torch.float64, device=self.device)
        if virial:
            flags |= NB_F_VIRIAL
            if vir is None:
                vir = torch.empty((self.n_sys, 3, 3), dtype=torch.float64, device=self.device)
        if accumulate:
            flags |= NB_F_ACCUMULATE
        if excl_corr:
            flags |= NB_F_EXCL_CORR
        self._check(self.lib.nb_forces(self.h, _ptr(x), _ptr(q), _ptr(lj), _ptr(f),
                                       _ptr(e) if energy else None,
                                       _ptr(vir) if virial else None, flags), "nb_forces")
        return f, (e if energy else None), (vir if virial else None)

    def step(self, x, q, lj, steps_since_build: int, energy: bool = True, virial: bool = False,
             f=None, e=None, vir=None, accumulate: bool = False, graph: bool = False,
             excl_corr: bool = False):
        """Rolling prune of part (steps_since_build mod nstprune) fused into the force pass;
        the same result as prune_rolling(x, steps_since_build) followed by forces(...).
        graph=True replays the step from a captured HIP graph (nb_step_graph): keep x, q,
        lj and the outputs at fixed addresses (update them in place) so it is reused."""
        x = self._dev(x, (self.n_atoms, 3), torch.float32, "x")
        q = self._dev(q, (self.n_atoms,), torch.float32, "q")
        lj = self._dev(lj, (self.n_types, self.n_types, 2), torch.float32, "lj")
        if f is None:
            f = torch.empty((self.n_atoms, 3), dtype=torch.float32, device=self.device)
        flags = 0
        if energy:
            flags |= NB_F_ENERGY
            if e is None:
                e = torch.empty((self.n_sys, 2), dtype=torch.float64, device=self.device)
        if virial:
            flags |= NB_F_VIRIAL
            if vir is None:
                vir = torch.empty((self.n_sys, 3, 3), dtype=torch.float64, device=self.device)
        if accumulate:
            flags |= NB_F_ACCUMULATE
        if excl_corr:
            flags |= NB_F_EXCL_CORR
        fn = self.lib.nb_step_graph if graph else self.lib.nb_step
        self._check(fn(self.h, _ptr(x), _ptr(q), _ptr(lj), _ptr(f),
                       _ptr(e) if energy else None, _ptr(vir) if virial else None,
                       flags, int(steps_since_build)), "nb_step_graph" if graph else "nb_step")
        return f, (e if energy else None), (vir if virial else None)

    def set_exec(self, item_width: int = 0, mode: str = "static", prune_fused=True,
                 prune_waves: int = 0):
        """Item width (0 = built-in rule), execution mode ('static', 'xcd', 'queue':
        balanced runs plus a dynamic tail, 'persist': rounds in cost order, 'balanced'),
        where step() prunes (True: inside the pair kernel; False: its own kernel before it;
        "ahead": after the pair kernel, in the force reduction's launch, for the next
        step's part with this step's positions), and the wavefronts per item of the prune
        kernel (0 = automatic)."""
        self._check(self.lib.nb_set_exec(self.h, int(item_width), EXEC_MODES[mode],
                                         _prune_code(prune_fused), int(prune_waves)),
                    "nb_set_exec")

    def get_exec(self) -> dict:
        out = NbExecConfig()
        self._check(self.lib.nb_get_exec(self.h, ctypes.byref(out)), "nb_get_exec")
        return {"item_width": out.item_width, "mode": _MODE_NAMES[out.exec_mode],
                "prune_fused": _prune_name(out.prune_fused), "prune_waves": int(out.prune_waves)}

    def autotune(self, x, q, lj, energy: bool = True, virial: bool = False, repeats: int = 5):
        """Time nb_forces over item widths and execution modes on the current list, then a
        rolling step with each prune placement in the two fastest shapes; keep the fastest
        step's shape and placement.  Returns (best, trials) as dicts with item_width, mode,
        prune_fused, prune_waves, us_per_call."""
        x = self._dev(x, (self.n_atoms, 3), torch.float32, "x")
        q = self._dev(q, (self.n_atoms,), torch.float32, "q")
        lj = self._dev(lj, (self.n_types, self.n_types, 2), torch.float32, "lj")
        flags = (NB_F_ENERGY if energy else 0) | (NB_F_VIRIAL if virial else 0)
        cap = 64
        trials = (NbExecConfig * cap)()
        n = ctypes.c_int32(0)
        best = NbExecConfig()
        self._check(self.lib.nb_autotune(self.h, _ptr(x), _ptr(q), _ptr(lj), flags, int(repeats),
                                         ctypes.cast(trials, ctypes.c_void_p), cap,
                                         ctypes.byref(n), ctypes.byref(best)), "nb_autotune")

        def d(t):
            return {"item_width": t.item_width, "mode": _MODE_NAMES[t.exec_mode],
                    "prune_fused": _prune_name(t.prune_fused), "us_per_call": t.us_per_call}
        return d(best), [d(trials[i]) for i in range(min(n.value, cap))]

    def backward(self, x, q, lj, grad_f, grad_energy=None, need_x=True, need_q=True,
                 need_lj=True, accumulate: bool = False):
        """Returns (grad_x [N,3] f32, grad_q [N] f32, grad_lj [T,T,2] f64), None if skipped."""
        x = self._dev(x, (self.n_atoms, 3), torch.float32, "x")
        q = self._dev(q, (self.n_atoms,), torch.float32, "q")
        lj = self._dev(lj, (self.n_types, self.n_types, 2), torch.float32, "lj")
        grad_f = self._dev(grad_f, (self.n_atoms, 3), torch.float32, "grad_f")
        if grad_energy is not None:
            grad_energy = self._dev(grad_energy, (self.n_sys, 2), torch.float64, "grad_energy")
        gx = torch.empty((self.n_atoms, 3), dtype=torch.float32, device=self.device) if need_x else None
        gq = torch.empty((self.n_atoms,), dtype=torch.float32, device=self.device) if need_q else None
        gl = torch.empty((self.n_types, self.n_types, 2), dtype=torch.float64,
                         device=self.device) if need_lj else None
        flags = NB_F_ACCUMULATE if accumulate else 0
        self._check(self.lib.nb_forces_backward(self.h, _ptr(x), _ptr(q), _ptr(lj), _ptr(grad_f),
                                                _ptr(grad_energy), _ptr(gx), _ptr(gq), _ptr(gl),
                                                flags), "nb_forces_backward")
        return gx, gq, gl

    # ---- introspection ------------------------------------------------------------------
    def get_grid(self) -> np.ndarray:
        n = ctypes.c_int64()
        self._check(self.lib.nb_get_grid(self.h, None, 0, ctypes.byref(n)), "nb_get_grid")
        out = np.empty(n.value, dtype=np.int32)
        self._check(self.lib.nb_get_grid(self.h, _np_ptr(out), n.value, ctypes.byref(n)),
                    "nb_get_grid")
        return out

    def get_grid_dims(self) -> np.ndarray:
        out = np.empty((self.n_sys, 2), dtype=np.int32)
        self._check(self.lib.nb_get_grid_dims(self.h, _np_ptr(out)), "nb_get_grid_dims")
        return out

    def get_pairs(self, which: str = "outer") -> np.ndarray:
        """Cluster-pair triples (ci, cj, shift code) of the "bb" candidates, the "outer" or
        the "inner" list (syncs)."""
        w = {"bb": 0, "outer": 1, "inner": 2}[which]
        n = ctypes.c_int64()
        self._check(self.lib.nb_get_pairs(self.h, w, None, 0, ctypes.byref(n)), "nb_get_pairs")
        out = np.empty((n.value, 3), dtype=np.int32)
        self._check(self.lib.nb_get_pairs(self.h, w, _np_ptr(out), n.value, ctypes.byref(n)),
                    "nb_get_pairs")
        return out

    def set_timing(self, enable: bool = True):
        self._check(self.lib.nb_set_timing(self.h, 1 if enable else 0), "nb_set_timing")

    def get_timing(self) -> dict:
        """{kind: (milliseconds, launches)} accumulated since the last call (syncs)."""
        ms = np.zeros(_lib.NB_T_COUNT, dtype=np.float64)
        calls = np.zeros(_lib.NB_T_COUNT, dtype=np.int64)
        self._check(self.lib.nb_get_timing(self.h, _np_ptr(ms), _np_ptr(calls)), "nb_get_timing")
        return {k: (float(ms[i]), int(calls[i])) for i, k in enumerate(_lib.TIMING_KINDS)}

    def list_census(self, radii) -> np.ndarray:
        """Work-efficiency census of the current outer list (nb_list_census): int64 array
        [4, 4, K], [a, b, k] = held pairs of sub-clusters of CENSUS_SIZES[a] i-slots and
        CENSUS_SIZES[b] j-slots with an atom pair closer than radii[k] (nm, each in
        (0, rlist]); [0, 0, k] counts atom pairs, [3, 3, k] cluster pairs (syncs)."""
        r = np.ascontiguousarray(np.asarray(radii, dtype=np.float32).reshape(-1))
        out = np.zeros((16, max(1, r.size)), dtype=np.int64)
        self._check(self.lib.nb_list_census(self.h, int(r.size), _np_ptr(r), _np_ptr(out)),
                    "nb_list_census")
        return out.reshape(4, 4, -1)

    def list_census_noalloc(self, radii) -> np.ndarray:
        """nb_list_census_noalloc: the census of list_census computed in the library's fixed
        per-device scratch (no allocation); same layout and values (syncs)."""
        r = np.ascontiguousarray(np.asarray(radii, dtype=np.float32).reshape(-1))
        out = np.zeros((16, max(1, r.size)), dtype=np.int64)
        self._check(self.lib.nb_list_census_noalloc(self.h, int(r.size), _np_ptr(r),
                                                    _np_ptr(out)), "nb_list_census_noalloc")
        return out.reshape(4, 4, -1)

    def list_coverage(self, radii, m: int = 8, n: int = 8) -> np.ndarray:
        """Coverage of the current outer list by an m x n list (nb_list_coverage): int64
        [K, K], [l, k] = atom pairs closer than radii[k] in an m x n sub-cluster pair that
        holds an atom pair closer than radii[l] (syncs)."""
        sizes = _lib.CENSUS_SIZES
        if m not in sizes or n not in sizes:
            raise ValueError("sub-cluster sizes must be 1, 2, 4 or 8")
        r = np.ascontiguousarray(np.asarray(radii, dtype=np.float32).reshape(-1))
        out = np.zeros((max(1, r.size), max(1, r.size)), dtype=np.int64)
        self._check(self.lib.nb_list_coverage(self.h, sizes.index(m), sizes.index(n), int(r.size),
                                              _np_ptr(r), _np_ptr(out)), "nb_list_coverage")
        return out

    def stats(self) -> dict:
        s = _lib.NbStats()
        self._check(self.lib.nb_get_stats(self.h, ctypes.byref(s)), "nb_get_stats")
        return {k: int(getattr(s, k)) for k, _ in _lib.NbStats._fields_}


def lj_table(sigma: torch.Tensor, eps: torch.Tensor) -> torch.Tensor:
    """(c6, c12) table [T,T,2] from per-type sigma, epsilon with the Lorentz-Berthelot rule
    (differentiable; the table itself is what the library consumes)."""
    s = 0.5 * (sigma[:, None] + sigma[None, :])
    e = torch.sqrt(eps[:, None] * eps[None, :])
    return torch.stack([4.0 * e * s ** 6, 4.0 * e * s ** 12], dim=-1).to(torch.float32)


class NBForces(torch.autograd.Function):
    """(x, q, lj) -> (forces [N,3], energies [S,2]) with the HIP backward pass over the
    frozen inner list: gradients with respect to positions, charges and the LJ table."""

    @staticmethod
    def forward(fctx, x, q, lj, nb: Context):
        f, e, _ = nb.forces(x.detach().contiguous(), q.detach().contiguous(),
                            lj.detach().contiguous(), energy=True)
        fctx.nb = nb
        fctx.save_for_backward(x, q, lj)
        return f, e

    @staticmethod
    def backward(fctx, gf, ge):
        x, q, lj = fctx.saved_tensors
        nb = fctx.nb
        gf = torch.zeros_like(x) if gf is None else gf.contiguous().to(torch.float32)
        ge = None if ge is None else ge.contiguous().to(torch.float64)
        gx, gq, gl = nb.backward(x.detach().contiguous(), q.detach().contiguous(),
                                 lj.detach().contiguous(), gf, ge,
                                 need_x=fctx.needs_input_grad[0],
                                 need_q=fctx.needs_input_grad[1],
                                 need_lj=fctx.needs_input_grad[2])
        return gx, gq, (gl.to(lj.dtype) if gl is not None else None), None
