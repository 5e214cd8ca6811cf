"""Grid specification written out in numpy (oracle side; test infrastructure only).

The paper's search grid (Sec. V.A, Fig. 4): a regular grid in x and y whose
z-columns are cut into cells holding a fixed number of atoms; on GPUs the
clusters are grouped eight at a time into near-cubic super-clusters by a
2x2x2 grouping on the grid.  The paper fixes no sizes, orders or tie-breaks;
the reading written out here (and to be reproduced bit for bit by the HIP
grid build) is:

1. per system, columns per axis n = max(1, floor(L / s + 1/2)) with
   s = (64 V / N)^(1/3) in double precision (one 64-atom super-cell per column
   and z-slab of a near-cubic shape);
2. wrap in single precision: k = floor(x * invL), w = x - k * L, with
   invL = float32(1 / L); column index c = clamp(floor(w * float32(n / L)), 0, n-1),
   column id = cx * ny + cy (systems one after the other);
3. order atoms by (column id, w_z, atom index) and cut each column into
   consecutive super-cells of 64 atoms (the last one partial);
4. in a super-cell the first 32 atoms (by z) form the lower z-half; each half,
   ordered by (w_y, atom index), gives its first 16 to the lower y-half; each
   quarter, ordered by (w_x, atom index), gives its first 8 to the lower x-half,
   in that order inside the cluster;
5. cluster = z-half * 4 + y-half * 2 + x-half inside the super-cell, slot =
   64 * super-cell + 8 * cluster + position; unused slots hold atom -1.
"""
from __future__ import annotations

import numpy as np


def grid_dims(n_atoms: int, box: np.ndarray) -> tuple:
    if n_atoms <= 0:
        return 1, 1
    L = box.astype(np.float64)
    s = np.cbrt(64.0 * (L[0] * L[1] * L[2]) / float(n_atoms))
    nx = max(1, int(np.floor(L[0] / s + 0.5)))
    ny = max(1, int(np.floor(L[1] / s + 0.5)))
    return nx, ny


def wrap(x: np.ndarray, box: np.ndarray):
    """Single-precision wrap of user coordinates: (k int32 [N,3], w float32 [N,3])."""
    L = box.astype(np.float32)
    invL = (1.0 / box.astype(np.float64)).astype(np.float32)
    k = np.floor((x.astype(np.float32) * invL).astype(np.float32)).astype(np.float32)
    w = (x.astype(np.float32) - (k * L).astype(np.float32)).astype(np.float32)
    return k.astype(np.int32), w


def _group_rank(group: np.ndarray, key: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Rank of each element inside its group when ordered by (key, idx)."""
    o = np.lexsort((idx, key, group))
    g = group[o]
    start = np.r_[0, np.flatnonzero(g[1:] != g[:-1]) + 1]
    first = np.repeat(start, np.diff(np.r_[start, g.size]))
    rank = np.empty_like(o)
    rank[o] = np.arange(g.size) - first
    return rank


def build_grid(x: np.ndarray, boxes: np.ndarray, offsets: np.ndarray) -> dict:
    """Slot assignment for all systems.  x float32 [N,3]; boxes float32 [S,3];
    offsets int64 [S+1].  Returns slot_atom, atom_slot, wrapped coordinates,
    image offsets, per-system grid dims and per-cluster atom counts."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    boxes = np.asarray(boxes, dtype=np.float32).reshape(-1, 3)
    offsets = np.asarray(offsets, dtype=np.int64)
    n_sys = boxes.shape[0]
    N = int(offsets[-1])
    col = np.empty(N, dtype=np.int64)
    k_all = np.empty((N, 3), dtype=np.int32)
    w_all = np.empty((N, 3), dtype=np.float32)
    dims = []
    col_base = 0
    col_base_list = []
    for s in range(n_sys):
        a0, a1 = int(offsets[s]), int(offsets[s + 1])
        nx, ny = grid_dims(a1 - a0, boxes[s])
        dims.append((nx, ny))
        col_base_list.append(col_base)
        k, w = wrap(x[a0:a1], boxes[s])
        k_all[a0:a1], w_all[a0:a1] = k, w
        cinvx = np.float32(nx / np.float64(boxes[s, 0]))
        cinvy = np.float32(ny / np.float64(boxes[s, 1]))
        cx = np.floor((w[:, 0] * cinvx).astype(np.float32)).astype(np.int64)
        cy = np.floor((w[:, 1] * cinvy).astype(np.float32)).astype(np.int64)
        cx = np.clip(cx, 0, nx - 1)
        cy = np.clip(cy, 0, ny - 1)
        col[a0:a1] = col_base + cx * ny + cy
        col_base += nx * ny
    n_cols = col_base
    idx = np.arange(N, dtype=np.int64)
    order = np.lexsort((idx, w_all[:, 2], col))
    col_s = col[order]
    counts = np.bincount(col, minlength=n_cols).astype(np.int64)
    col_start = np.r_[0, np.cumsum(counts)]
    pos_in_col = np.arange(N) - col_start[col_s]
    sc_per_col = (counts + 63) // 64
    sc_start = np.r_[0, np.cumsum(sc_per_col)]
    n_sc = int(sc_start[-1])
    sc = sc_start[col_s] + pos_in_col // 64
    zh = (pos_in_col % 64) >= 32
    atoms = order
    g1 = sc * 2 + zh
    r1 = _group_rank(g1, w_all[atoms, 1], atoms)
    yh = r1 >= 16
    g2 = g1 * 2 + yh
    r2 = _group_rank(g2, w_all[atoms, 0], atoms)
    xh = r2 >= 8
    pos = r2 % 8
    cl = zh.astype(np.int64) * 4 + yh.astype(np.int64) * 2 + xh.astype(np.int64)
    slot = sc * 64 + cl * 8 + pos
    slot_atom = np.full(n_sc * 64, -1, dtype=np.int32)
    slot_atom[slot] = atoms
    atom_slot = np.empty(N, dtype=np.int64)
    atom_slot[atoms] = slot
    cluster_count = (slot_atom.reshape(-1, 8) >= 0).sum(axis=1).astype(np.int32)
    sc_col = np.repeat(np.arange(n_cols), sc_per_col)
    return dict(slot_atom=slot_atom, atom_slot=atom_slot, w=w_all, k=k_all, dims=dims,
                col_base=np.array(col_base_list, dtype=np.int64), n_cols=n_cols,
                n_sc=n_sc, col_counts=counts, sc_per_col=sc_per_col, sc_col=sc_col,
                cluster_count=cluster_count)
