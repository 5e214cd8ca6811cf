"""Work-efficiency census of cluster-pair lists, in plain numpy.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg
of the benchmark; the product library never uses it.

The quantity is the algorithmic work efficiency of Sec. V.B (Fig. 5): the fraction of the
atom pairs a list makes a kernel compute that lie inside the cut-off.  A list of M x N
cluster pairs (Sec. V.A: i-clusters of M atoms against j-clusters of N atoms) holds every
pair of sub-clusters with at least one atom pair closer than the list radius, and costs
M N pair evaluations per held pair; the particle list (1 x 1) holds the atom pairs
themselves.

Sub-clusters are runs of consecutive slots of the 8-atom clusters of the grid: for M in
{1, 2, 4, 8} the i-sub-clusters of cluster c are the slot groups {8c + M g, ..., 8c + M g
+ M - 1}, likewise for N on the j side.  The pairs are the canonical cluster triples
(ci, cj, s) of the list oracle (ci <= cj; for ci == cj only s = 0 or a lexicographically
positive shift, and for s = 0 only i-slot before j-slot); distances follow its fixed
single-precision sequence, so every count is an exact integer.

    census(slot_atom, w, box, radii)[a, b, k]
        = number of canonical (i-sub-cluster of SIZES[a] slots, j-sub-cluster of SIZES[b]
          slots, shift) holding an atom pair with r2 < float32(radii[k]^2)

[0, 0, k] is the number of atom pairs closer than radii[k] (each unordered pair once);
[3, 3, k] is the number of 8x8 cluster pairs.
"""
from __future__ import annotations

import numpy as np

from . import cluster_pairs, radius_sq_f32, split_key

SIZES = (1, 2, 4, 8)


def _shift_codes(code):
    code = np.asarray(code, dtype=np.int64)
    return code // 9 - 1, (code // 3) % 3 - 1, code % 3 - 1


def pair_r2(slot_atom, w, box, ci, cj, code):
    """Single-precision r2 of every slot pair of the cluster triples (ci, cj, code), shape
    (P, 8, 8) indexed [triple, i-slot, j-slot], +inf where a slot is empty or the pair is
    not counted (a cluster with itself at s = 0 keeps i-slot < j-slot).  Per axis
    a = x_i - L if s > 0, b = x_j - L if s < 0, d = a - b; r2 = (dx^2 + dy^2) + dz^2, every
    step rounded to single precision (numpy float32 arithmetic has no contraction)."""
    slot_atom = np.asarray(slot_atom, dtype=np.int64)
    w = np.asarray(w, dtype=np.float32)
    L = np.asarray(box, dtype=np.float32).reshape(3)
    ai = slot_atom[(8 * np.asarray(ci)[:, None] + np.arange(8)[None, :])]   # (P, 8)
    aj = slot_atom[(8 * np.asarray(cj)[:, None] + np.arange(8)[None, :])]
    xi = w[np.maximum(ai, 0)]                                             # (P, 8, 3)
    xj = w[np.maximum(aj, 0)]
    shifts = _shift_codes(code)
    r2 = None
    for k in range(3):
        s = shifts[k][:, None]
        a = np.where(s > 0, xi[:, :, k] - L[k], xi[:, :, k]).astype(np.float32)
        b = np.where(s < 0, xj[:, :, k] - L[k], xj[:, :, k]).astype(np.float32)
        d = (a[:, :, None] - b[:, None, :]).astype(np.float32)          # (P, 8, 8)
        dd = (d * d).astype(np.float32)
        r2 = dd if r2 is None else (r2 + dd).astype(np.float32)
    valid = (ai >= 0)[:, :, None] & (aj >= 0)[:, None, :]
    diag = (np.asarray(ci) == np.asarray(cj)) & (np.asarray(code) == 13)
    tri = np.arange(8)[:, None] < np.arange(8)[None, :]
    valid &= ~diag[:, None, None] | tri[None, :, :]
    return np.where(valid, r2, np.float32(np.inf)).astype(np.float32)


def census(slot_atom, w, box, radii, chunk: int = 1 << 16, ci_lo: int = 0,
           ci_hi=None) -> np.ndarray:
    """Counts [4, 4, K] of held M x N sub-cluster pairs per radius (module docstring), over
    the triples whose i-cluster ci lies in [ci_lo, ci_hi) (all by default).  Candidates are
    the cluster triples within the largest radius (a sub-cluster pair with an atom pair
    inside a radius lies in such a triple)."""
    radii = np.asarray(radii, dtype=np.float64).reshape(-1)
    slot_atom = np.asarray(slot_atom)
    n_cl = slot_atom.size // 8
    R2 = np.array([radius_sq_f32(r) for r in radii], dtype=np.float32)
    out = np.zeros((4, 4, radii.size), dtype=np.int64)
    if radii.size == 0 or n_cl == 0:
        return out
    keys = cluster_pairs(slot_atom, w, box, float(radii.max()), ci_lo, ci_hi)
    ci, cj, code = split_key(keys, n_cl)
    for p0 in range(0, keys.size, chunk):
        r2 = pair_r2(slot_atom, w, box, ci[p0:p0 + chunk], cj[p0:p0 + chunk],
                     code[p0:p0 + chunk])
        P = r2.shape[0]
        for k in range(radii.size):
            inside = r2 < R2[k]                                            # (P, 8, 8)
            for a, M in enumerate(SIZES):
                for b, N in enumerate(SIZES):
                    held = inside.reshape(P, 8 // M, M, 8 // N, N).any(axis=(2, 4))
                    out[a, b, k] += int(held.sum())
    return out


def work_efficiency(counts: np.ndarray, k_cut: int, k_list: int, M: int, N: int) -> float:
    """Fraction of the pair evaluations of an M x N list at radii[k_list] that lie inside
    radii[k_cut] (Sec. V.B): pairs inside the cut-off over M N held sub-cluster pairs.  The
    1 x 1 list computes exactly the atom pairs inside its radius."""
    a, b = SIZES.index(M), SIZES.index(N)
    held = counts[a, b, k_list]
    return float(counts[0, 0, k_cut]) / float(M * N * held) if held else 1.0
