// The rolling prune of one work item (Sec. V.E), shared by the prune kernel and the force
// reduction, which can run it beside its own blocks for the next step's part.
#pragma once

#include "nb_internal.h"
#include "nb_pair_common.h"

#ifndef NB_FOR8
#define NB_FOR8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)
#endif

// OR of an 8-bit value over the 64 lanes: swap neighbours, swap pairs, mirror the half
// rows, mirror the rows (every lane then holds its 16-lane row's OR), then the four rows.
__device__ inline uint32_t wave_or(uint32_t v) {
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, true);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, true);
    return (uint32_t)(__builtin_amdgcn_readlane((int)v, 0) | __builtin_amdgcn_readlane((int)v, 16) |
                      __builtin_amdgcn_readlane((int)v, 32) | __builtin_amdgcn_readlane((int)v, 48));
}

// Rolling prune (Sec. V.E) of one work item by the whole block (kPruneWaves wavefronts;
// s_xi: 64 float4 of the calling kernel's LDS; called by every thread of the block).
// Wavefront w takes the item's entries w, w + kPruneWaves, ... in order.  Lane k of a
// wavefront loads the (j-cluster, mask word) of its k-th entry once, at the start (items
// hold at most 64 entries), and the loop reads them with readlane, so no step waits for an
// entry load; the next entries' j-clusters are in flight.  The item's 64 i-atoms are
// staged once in LDS, then held eight per lane in registers.  For every i-cluster c of an
// entry's outer mask each lane tests its pair (i-atom 8 c + ii, j-atom jj) against r_inner
// in the list arithmetic (shift split between the two sides, no contraction) and keeps the
// result as bit c of a per-lane word; one OR over the wavefront per entry gives the inner
// mask.  (Per-lane bits keep the scalar unit out of the per-cluster work: a ballot and its
// test per cluster made the kernel bound by scalar issue.)  Empty slots sit far outside
// the box, so no valid-atom masks are needed; a cluster with itself keeps ii < jj.
template <int kPruneWaves>
__device__ __forceinline__ void prune_item(const NbItem it, NbEntry* __restrict__ entries,
                                           const float4* __restrict__ xp,
                                           const NbScInfo* __restrict__ sc_info,
                                           const NbSys* __restrict__ sys, float r2_inner,
                                           float4* s_xi) {
#pragma clang fp contract(off)
    if (it.ne <= 0) return;               // (items are never empty; uniform over the block)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    const int ii = lane & 7, jj = lane >> 3;
    const int e_end = it.e0 + it.ne;
    const int e_first = it.e0 + wave;
    const int kStep = kPruneWaves;
    const int n_mine = e_first < e_end ? (e_end - e_first + kStep - 1) / kStep : 0;
    int2 mine = make_int2(0, 0);          // lane k: (cj, meta) of entry e_first + k kStep
    if (lane < n_mine)
        mine = *reinterpret_cast<const int2*>(&entries[e_first + lane * kStep]);
    // A j-cluster is loaded kAhead entries before its use; positions past the end load the
    // last one again (valid memory, never used).  The loads are in flight while the block
    // waits for the i-atoms.
    constexpr int kAhead = 3;
    float4 xq[kAhead];
    const int last = n_mine > 0 ? n_mine - 1 : 0;
#pragma unroll
    for (int a = 0; a < kAhead; ++a)
        xq[a] = xp[kClusterSize * __builtin_amdgcn_readlane(mine.x, a < last ? a : last) + jj];
    if (threadIdx.x < kScAtoms) s_xi[threadIdx.x] = xp[kScAtoms * it.sc + threadIdx.x];
    __syncthreads();
    if (n_mine == 0) return;
    const NbSys S = sys[sc_info[it.sc].sys];
    const int ci0 = kClustersPerSc * it.sc;
    // i-atom ii of cluster c in registers (no LDS wait inside the loop)
#define NB_PI(c) const float4 xi##c = s_xi[kClusterSize * c + ii];
    NB_FOR8(NB_PI)
#undef NB_PI
    for (int k = 0; k < n_mine; ++k) {
        const int2 ent = make_int2(__builtin_amdgcn_readlane(mine.x, k),
                                   __builtin_amdgcn_readlane(mine.y, k));
        float4 xj = xq[0];
#pragma unroll
        for (int a = 0; a + 1 < kAhead; ++a) xq[a] = xq[a + 1];
        const int kn = k + kAhead < last ? k + kAhead : last;
        xq[kAhead - 1] = xp[kClusterSize * __builtin_amdgcn_readlane(mine.x, kn) + jj];
        const int e = e_first + k * kStep;
        const uint32_t meta = (uint32_t)ent.y;
        const int code = meta & 31u;
        const uint32_t omask = (meta >> 8) & 0xffu;
        uint32_t hits = 0;                // bit c: this lane's pair of cluster c is inside
        if (code == kShiftZero) {
            // no shift: x_i - x_j, the same bits as the general sequence with zero shifts
#define NB_PB(c)                                                                       \
            if ((omask >> c) & 1u) {                                                   \
                const float dx = xi##c.x - xj.x;                                       \
                const float dy = xi##c.y - xj.y;                                       \
                const float dz = xi##c.z - xj.z;                                       \
                const float r2 = (dx * dx + dy * dy) + dz * dz;                        \
                hits |= (r2 < r2_inner) ? (1u << c) : 0u;                              \
            }
            NB_FOR8(NB_PB)
#undef NB_PB
            const int dc = ent.x - ci0;   // a cluster with itself: pairs ii < jj only
            if ((unsigned)dc < (unsigned)kClustersPerSc && ii >= jj) hits &= ~(1u << dc);
        } else {
            // the same separation as the list build: x_i - L for s > 0, x_j - L for s < 0
            // (a shifted entry keeps all 64 pairs, an atom and its own image included)
            const int sx = shift_x(code), sy = shift_y(code), sz = shift_z(code);
            xj.x -= (sx < 0) ? S.L[0] : 0.f;
            xj.y -= (sy < 0) ? S.L[1] : 0.f;
            xj.z -= (sz < 0) ? S.L[2] : 0.f;
            const float ox = (sx > 0) ? S.L[0] : 0.f, oy = (sy > 0) ? S.L[1] : 0.f,
                        oz = (sz > 0) ? S.L[2] : 0.f;
#define NB_PB(c)                                                                       \
            if ((omask >> c) & 1u) {                                                   \
                const float dx = (xi##c.x - ox) - xj.x;                                \
                const float dy = (xi##c.y - oy) - xj.y;                                \
                const float dz = (xi##c.z - oz) - xj.z;                                \
                const float r2 = (dx * dx + dy * dy) + dz * dz;                        \
                hits |= (r2 < r2_inner) ? (1u << c) : 0u;                              \
            }
            NB_FOR8(NB_PB)
#undef NB_PB
        }
        const uint32_t imask = wave_or(hits);
        if (lane == 0) entries[e].meta = (meta & ~(0xffu << 16)) | (imask << 16);
    }
}

