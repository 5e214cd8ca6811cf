// Cluster-pair force / energy kernel (Sec. V.A).
//
// One wavefront processes one work item: a chunk of one super-cluster's joint j-list.
// Lane l holds the pair (i-atom ii = l & 7, j-atom jj = l >> 3) of the current 8x8
// cluster pair.  The super-cluster's 64 i-atoms sit in a per-wavefront LDS table and the
// eight i-clusters' force accumulators in registers for the whole item; per j-entry the
// loop over the set bits of the interaction mask is uniform (scalar branches, no
// divergence), the interaction, exclusion and cut-off masks are 64-bit scalar masks, and
// the j-forces are reduced over the eight i-lanes with DPP adds and stored once per entry
// into the entry's own partial slot (Newton's third law: each pair once).  Energies are
// summed per entry in single precision and accumulated in double.  No atomics: every
// partial has one writer; nb_reduce.hip adds them up.
#include <algorithm>

#include "nb_internal.h"
#include "nb_pair_common.h"

namespace {

constexpr int kFwdWaves = 4;
constexpr int kFwdThreads = kFwdWaves * kWave;

// One 8x8 block of pairs (i-cluster c of the item, the current j-cluster): m is the
// scalar 64-bit mask of non-excluded lanes (lane = ii + 8 jj), xj the lane's j-atom with
// the entry's periodic shift already added, tjo 16 bytes times the j-atom's type; s_t
// holds per slot the byte offset of the i-atom's row of the LJ table s_lj (16 T type_i).
template <int COUL, bool ENERGY, bool VIRIAL>
__device__ __forceinline__ void pair_block(const float4* s_x, const int* s_t,
                                           const float4* __restrict__ s_lj,
                                           uint64_t m, float& fx, float& fy,
                                           float& fz, const float4& xj, const int tjo,
                                           const NbKParams& kp, float& fjx,
                                           float& fjy, float& fjz, float& elj, float& ec,
                                           float& eclo, float (&vir)[6], int& npair,
                                           int& nblock) {
    const float4 xv = *s_x;                            // (x_i, y_i, z_i, K q_i) of this lane
    const float dx = xv.x - xj.x, dy = xv.y - xj.y, dz = xv.z - xj.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const uint64_t act = __builtin_amdgcn_ballot_w64(r2 < kp.rc2) & m;
    if (!act) return;
    const bool on = __builtin_amdgcn_inverse_ballot_w64(act);
    // (6 c6, 12 c12, 12 shift, -) of the pair's types
    const float4 p = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_lj) +
                                                      (*s_t + tjo));
    // With energies, pairs outside the cut-off or excluded get 1/r = 0 and q_i q_j = 0
    // (every force and energy term below then vanishes; r2 itself stays finite); without,
    // the scalar force alone is masked at the end.
    const float rinv = (ENERGY && !on) ? 0.f : __builtin_amdgcn_rsqf(r2);
    const float qq = (ENERGY && !on) ? 0.f : xv.w * xj.w;   // epsfac/eps_r folded into q_i
    const float rinv2 = rinv * rinv;
    const float rinv6 = rinv2 * rinv2 * rinv2;
    const float t = fmaf(p.y, rinv6, -p.x);            // 12 c12 r^-6 - 6 c6
    const float flj = rinv6 * t;                       // F_LJ * r
    float fscal;
    if (COUL == NB_COUL_NONE) {
        fscal = flj * rinv2;
    } else if (COUL == NB_COUL_RF) {
        fscal = fmaf(flj, rinv2, qq * (rinv * rinv2 - 2.0f * kp.krf));
        if (ENERGY) {
            ec = fmaf(qq, fmaf(kp.krf, r2, rinv) - kp.crf, ec);
            // The residuals of the single-precision k_rf, c_rf are far below half an ulp of
            // the pair energy near the cut-off, where most pairs are; added to it they would
            // vanish and leave a systematic 1e-6 bias in E_C.  They get their own sum.
            eclo = fmaf(qq, fmaf(kp.krf_lo, r2, -kp.crf_lo), eclo);
        }
    } else {
        const float r = r2 * rinv;
        const float e = __builtin_amdgcn_exp2f(r2 * kp.beta2_log2e);   // exp(-beta^2 r^2)
        const float erfcv = e * erfcx_poly(r, kp.p_beta);
        const float g = fmaf(erfcv, rinv, kp.two_beta_sqrtpi * e);
        fscal = fmaf(qq, g, flj) * rinv2;
        if (ENERGY) ec = fmaf(qq, fmaf(erfcv, rinv, -kp.ewald_shift), ec);
    }
    if (!ENERGY) fscal = on ? fscal : 0.f;
    const float tx = fscal * dx, ty = fscal * dy, tz = fscal * dz;
    fx += tx;
    fy += ty;
    fz += tz;
    fjx -= tx;
    fjy -= ty;
    fjz -= tz;
    if (ENERGY) {
        // 12 V_LJ = r^-6 (12 c12 r^-6 - 12 c6) - 12 shift = r^-6 (t - 6 c6) - 12 shift,
        // summed as is and divided by 12 in double precision per item: no rounded 1/12
        // (a relative bias of 4e-8 on every repulsive term)
        elj += fmaf(rinv6, t - p.x, on ? -p.z : 0.f);
        npair += __builtin_popcountll(act);
        nblock += 1;
    }
    if (VIRIAL) {
        vir[0] = fmaf(tx, dx, vir[0]);
        vir[1] = fmaf(ty, dy, vir[1]);
        vir[2] = fmaf(tz, dz, vir[2]);
        vir[3] = fmaf(tx, dy, vir[3]);
        vir[4] = fmaf(tx, dz, vir[4]);
        vir[5] = fmaf(ty, dz, vir[5]);
    }
}

// Per-cluster code of the item's eight i-clusters (unrolled; force sums in registers).
#define NB_FOR8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

// The work of one item (one wavefront): s_x and s_t are the wavefront's 64-entry LDS
// tables of the super-cluster's atoms ((x, y, z, K q) and 16 T type, by slot), s_lj the
// block's LJ table.
template <int COUL, bool ENERGY, bool VIRIAL, bool PRUNE>
__device__ __forceinline__ void fwd_item(
    const int item, const int lane, float4* s_x, int* s_t, const float4* __restrict__ s_lj,
    const NbItem* __restrict__ items, NbEntry* __restrict__ entries,
    const uint64_t* __restrict__ excl_rows, const float4* __restrict__ xq,
    const int32_t* __restrict__ type_slot, const NbScInfo* __restrict__ sc_info,
    const NbSys* __restrict__ sys, float4* __restrict__ jpart, float4* __restrict__ ipart,
    double* __restrict__ epart, const int epart_stride, const NbKParams& kp,
    const int prune_part, const int nstprune, const float r2_inner) {
    const int T = kp.n_types;
    const NbItem it = items[item];
    const int ii = lane & 7, jj = lane >> 3;
    const int sc = it.sc, ci0 = kClustersPerSc * sc;
    const NbSys S = sys[sc_info[sc].sys];
    {
        // lane l holds slot l of the super-cluster: (8 c + ii) for c = l >> 3
        const float4 v = xq[kScAtoms * sc + lane];
        s_x[lane] = make_float4(v.x, v.y, v.z, v.w * kp.epsfac_r);
        // byte offset of the i-atom's row of the LJ table (type_slot holds 16 type)
        s_t[lane] = type_slot[kScAtoms * sc + lane] * T;
    }
    __builtin_amdgcn_wave_barrier();

#define NB_IZERO(c) float fx##c = 0.f, fy##c = 0.f, fz##c = 0.f;
    NB_FOR8(NB_IZERO)
#undef NB_IZERO

    double elj_acc = 0.0, ec_acc = 0.0;
    double vir_acc[6] = {0, 0, 0, 0, 0, 0};
    int npair = 0, nblock = 0;

    const int e_end = it.e0 + it.ne;
    // Items of the rolling part pruned in this pass (Sec. V.E; part = super-cluster mod
    // nstprune) first re-derive the inner
    // masks of all their entries from the outer masks and the current coordinates, in the
    // list arithmetic: lane (e - e0) keeps entry e's new mask (items hold at most 64
    // entries) for the force loop below, lane 0 writes it back for later passes.
    const bool do_prune = PRUNE && (sc % nstprune) == prune_part;
    uint32_t pmask = 0;
    if (do_prune) {
#pragma clang fp contract(off)
        NbEntry p1 = entries[it.e0];
        float4 y1 = xq[kClusterSize * p1.cj + jj];
        for (int e = it.e0; e < e_end; ++e) {
            const NbEntry ent = p1;
            float4 xj = y1;
            if (e + 1 < e_end) {
                p1 = entries[e + 1];
                y1 = xq[kClusterSize * p1.cj + jj];
            }
            const int code = ent.meta & 31u;
            const int sx = shift_x(code), sy = shift_y(code), sz = shift_z(code);
            xj.x -= (sx < 0) ? S.L[0] : 0.f;
            xj.y -= (sy < 0) ? S.L[1] : 0.f;
            xj.z -= (sz < 0) ? S.L[2] : 0.f;
            const float ox = (sx > 0) ? S.L[0] : 0.f, oy = (sy > 0) ? S.L[1] : 0.f,
                        oz = (sz > 0) ? S.L[2] : 0.f;
            const uint32_t omask = (ent.meta >> 8) & 0xffu;
            const bool selfp = (ent.cj >> 3) == sc && code == kShiftZero;
            const int dcp = ent.cj - ci0;
            uint32_t imask = 0;
#define NB_PB(c)                                                                       \
            if ((omask >> c) & 1u) {                                                   \
                const float4 xv = s_x[kClusterSize * c + ii];                          \
                const float dx = (xv.x - ox) - xj.x;                                   \
                const float dy = (xv.y - oy) - xj.y;                                   \
                const float dz = (xv.z - oz) - xj.z;                                   \
                const float r2 = (dx * dx + dy * dy) + dz * dz;                        \
                const uint64_t m = (selfp && dcp == c) ? 0x7f3f1f0f07030100ull : ~0ull;  \
                if (__builtin_amdgcn_ballot_w64(r2 < r2_inner) & m) imask |= 1u << c;  \
            }
            NB_FOR8(NB_PB)
#undef NB_PB
            if (lane == e - it.e0) pmask = imask;
            if (lane == 0) entries[e].meta = (ent.meta & ~(0xffu << 16)) | (imask << 16);
        }
    }
    // the next entry's j-atom loads are in flight while the current entry is computed
    float elj = 0.f, ec = 0.f, eclo = 0.f;   // single-precision sums over one entry
    // xj: the lane's j-atom with the entry's periodic shift already added
    auto do_entry = [&](const NbEntry& ent, const float4& xj, const int tjo, const int e) {
        const uint32_t mask =
            do_prune ? (uint32_t)__builtin_amdgcn_readlane((int)pmask, e - it.e0)
                     : (ent.meta >> 16) & 0xffu;
        // an entry with an empty mask runs no block and stores zero j-partials below
        const int code = ent.meta & 31u;
        const uint64_t* xrow =
            (ent.excl >= 0) ? excl_rows + (size_t)ent.excl * kClustersPerSc : nullptr;
        const bool self = (ent.cj >> 3) == sc && code == kShiftZero;
        float fjx = 0.f, fjy = 0.f, fjz = 0.f;
        float vir[6] = {0, 0, 0, 0, 0, 0};
        const int dc = ent.cj - ci0;        // the i-cluster equal to the j-cluster, if any

        // self cluster pairs keep ii < jj only (empty slots fail every distance test)
#define NB_MASK(c) (((self && dc == c) ? 0x7f3f1f0f07030100ull : ~0ull) & (xrow ? xrow[c] : ~0ull))
        {
#define NB_BLOCK(c)                                                                    \
    if ((mask >> c) & 1u)                                                              \
        pair_block<COUL, ENERGY, VIRIAL>(                                              \
            s_x + kClusterSize * c + ii, s_t + kClusterSize * c + ii, s_lj, NB_MASK(c), fx##c, \
            fy##c,                                                                     \
            fz##c, xj, tjo, kp, fjx, fjy, fjz, elj, ec, eclo, vir, npair, nblock);
            NB_FOR8(NB_BLOCK)
#undef NB_BLOCK
        }
#undef NB_MASK
        fjx = dpp_sum8(fjx);
        fjy = dpp_sum8(fjy);
        fjz = dpp_sum8(fjz);
        // every lane of a row holds the same sums: all eight store them (one 128-byte line
        // per entry, non-temporal: read once, later, by the reduction), which keeps the
        // last DPP step fused with its add
        store_stream(jpart + (size_t)ent.jpos * kClusterSize + jj, fjx, fjy, fjz, 0.f);
        if (VIRIAL) {
#pragma unroll
            for (int k = 0; k < 6; ++k) vir_acc[k] += (double)vir[k];
        }
    };
    auto load_j = [&](const NbEntry& ent, float4& xj, int& tjo) {
        xj = xq[kClusterSize * ent.cj + jj];
        tjo = type_slot[kClusterSize * ent.cj + jj];
    };
    auto flush_energy = [&]() {
        if (ENERGY) {
            elj_acc += (double)elj;
            if (COUL == NB_COUL_RF) ec_acc += (double)ec + (double)eclo;
            else if (COUL == NB_COUL_EWALD) ec_acc += (double)ec;
            elj = 0.f;
            ec = 0.f;
            eclo = 0.f;
        }
    };
    // entry e + 1 is loaded one iteration before its j-atoms, so that load never waits for
    // the entry it depends on
    NbEntry nxt = entries[it.e0];
    NbEntry nxt2 = entries[it.e0 + 1 < e_end ? it.e0 + 1 : it.e0];
    float4 xj_n;
    int tj_n;
    load_j(nxt, xj_n, tj_n);
    for (int e = it.e0; e < e_end; ++e) {
        const NbEntry ent = nxt;
        // Periodic image of the j-cluster: x_j + s L, added once per entry (the shift is
        // built from the bits of L with scalar integer operations, s in {-1, 0, 1}).  The
        // loaded coordinates are dead after this, so the next entry's loads can land in
        // the same registers.
        const int code = ent.meta & 31u;
        float4 xj = xj_n;
        xj.x += shift_value(shift_x(code), S.L[0]);
        xj.y += shift_value(shift_y(code), S.L[1]);
        xj.z += shift_value(shift_z(code), S.L[2]);
        const int tj = tj_n;
        // prefetch the next j-cluster and the entry after it (past the end the last entry
        // loads itself again: unconditional loads keep the prefetch registers in place
        // across iterations)
        nxt = nxt2;
        nxt2 = entries[e + 2 < e_end ? e + 2 : e_end - 1];
        load_j(nxt, xj_n, tj_n);
        do_entry(ent, xj, tj, e);
        flush_energy();
    }
    // i-forces: reduce over the eight j-lanes jj (stride 8) and store the item's partials.
    float4* ip = ipart + (size_t)item * kScAtoms;
#define NB_IRED(c)                                                                     \
    for (int off = 8; off < kWave; off <<= 1) {                                        \
        fx##c += __shfl_xor(fx##c, off);                                               \
        fy##c += __shfl_xor(fy##c, off);                                               \
        fz##c += __shfl_xor(fz##c, off);                                               \
    }                                                                                  \
    if (jj == 0) store_stream(&ip[kClusterSize * c + ii], fx##c, fy##c, fz##c, 0.f);
    NB_FOR8(NB_IRED)
#undef NB_IRED
    if (ENERGY || VIRIAL) {
        double v[8] = {elj_acc / 12.0, ec_acc, vir_acc[0], vir_acc[1], vir_acc[2], vir_acc[3],
                       vir_acc[4], vir_acc[5]};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) v[k] += __shfl_xor(v[k], off);
        }
        if (lane == 0) {
            // structure of arrays by the item's position in super-cluster order
#pragma unroll
            for (int k = 0; k < 8; ++k) epart[(size_t)k * epart_stride + it.pos] = v[k];
            epart[(size_t)8 * epart_stride + it.pos] = (double)npair;
            epart[(size_t)9 * epart_stride + it.pos] = 64.0 * (double)nblock;
        }
    }
}

// Block b of a grid of g blocks is dispatched to XCD b mod 8 (round robin).  Renumber
// the blocks so that each XCD takes one contiguous range of items: neighbouring
// super-clusters share j-clusters, so their coordinates stay in that XCD's L2.
__device__ inline int xcd_block(int b, int g) {
    const int x = b & (kXcds - 1), k = b / kXcds;
    const int q = g / kXcds, r = g % kXcds;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Execution modes (chosen per context, by hand or by the autotuner):
//   kExecStatic  one wavefront per item, item = 4 block + wave (rolling-part major: the
//                items processed together are four super-clusters apart);
//   kExecXcd     the same with the XCD-contiguous block numbering above;
//   kExecQueue   one resident grid; wavefront g first takes its own run of items
//                (wave_item[g] .. wave_item[g + 1], near-equal estimated cost, most of
//                the work), then shorter runs (the n_dyn runs after the n_waves own ones)
//                from ticket pool g mod kQueuePools, which holds runs p, p + kQueuePools,
//                ... and is shared by wavefronts spread over the device: those that end
//                their own run early take more.  A ticket is one atomic add by lane 0,
//                after a read of the counter, so a finished pool takes no more atomics
//                (same-address atomics serialise: waves of the whole grid taking turns
//                on the last open pools cost more than the balance they buy, measured).
//                The last block to finish (counted per group of blocks, then over the
//                groups) sets every counter back to zero, so the next launch needs no
//                clearing pass (and a captured graph none);
//   kExecPersist persistent: a grid that fills the device once, rounds of G items (G
//                wavefronts) in the order given by `order` (most pair work first),
//                wavefront g taking position g of even rounds and G - 1 - g of odd ones,
//                so the most expensive item of one round goes with the cheapest of the
//                next;
//   kExecBalanced wavefront g takes its own run of items only (no dynamic tail).
// Scalar registers are capped at 96 per wavefront: at the compiler's own choice (106 in the
// energy flavor) a SIMD holds six wavefronts of this kernel although its vector registers
// leave room for seven (measured from the wavefronts' start times; the occupancy query
// still reports seven); with the cap the seventh is resident and a dozen scalars live in
// vector-register lanes instead.
template <int COUL, bool ENERGY, bool VIRIAL, bool PRUNE>
__global__ __launch_bounds__(kFwdThreads) __attribute__((amdgpu_waves_per_eu(VIRIAL ? 3 : 4)))
__attribute__((amdgpu_num_sgpr(96))) void k_nb_fwd(
    const NbItem* __restrict__ items, NbEntry* __restrict__ entries,
    const uint64_t* __restrict__ excl_rows, const float4* __restrict__ xq,
    const int32_t* __restrict__ type_slot, const NbScInfo* __restrict__ sc_info,
    const NbSys* __restrict__ sys, const float* __restrict__ lj, float4* __restrict__ jpart,
    float4* __restrict__ ipart, double* __restrict__ epart, int epart_stride, NbKParams kp,
    int n_items, int prune_part, int nstprune, float r2_inner, int mode,
    const int32_t* __restrict__ order, int32_t* __restrict__ queue,
    const int32_t* __restrict__ wave_item, int n_waves, int n_dyn, int n_cu) {
    extern __shared__ float4 s_lj[];
    __shared__ float4 s_x_all[kFwdWaves][kScAtoms];    // per wave: (x, y, z, K q) by slot
    __shared__ int s_t_all[kFwdWaves][kScAtoms];       // per wave: type * T by slot
    const int T = kp.n_types;
    for (int i = threadIdx.x; i < T * T; i += blockDim.x) {
        const float c6 = lj[2 * i], c12 = lj[2 * i + 1];
        s_lj[i] = make_float4(6.0f * c6, 12.0f * c12,
                              (12.0f * c12) * kp.rc_m12 - (12.0f * c6) * kp.rc_m6, 0.f);
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    float4* s_x = s_x_all[wave];
    int* s_t = s_t_all[wave];
#define NB_ITEM_ARGS                                                                    \
    lane, s_x, s_t, s_lj, items, entries, excl_rows, xq, type_slot, sc_info, sys, jpart, ipart, \
        epart, epart_stride, kp, prune_part, nstprune, r2_inner
    if (mode == kExecBalanced) {
        // each wavefront its own run of items, of near-equal cost
        const int g = (int)blockIdx.x * kFwdWaves + wave;
        if (g < n_waves)
            for (int i = wave_item[g]; i < wave_item[g + 1]; ++i)
                fwd_item<COUL, ENERGY, VIRIAL, PRUNE>(i, NB_ITEM_ARGS);
        return;
    }
    if (mode == kExecQueue) {
        const int g = (int)blockIdx.x * kFwdWaves + wave;
        const int32_t* dyn_item = wave_item + n_waves;   // dynamic run k: items k .. k + 1
        int32_t* tickets = queue + kQueueTickets;
        // the wavefront's pool: its runs are p, p + kQueuePools, ... below n_dyn
        const int p = g % kQueuePools;
        const int runs_p = (n_dyn > p) ? (n_dyn - p + kQueuePools - 1) / kQueuePools : 0;
        int32_t* ticket = queue + kQueueTickets + p * kPoolStride;
        int i = (g < n_waves) ? wave_item[g] : 0, i_end = (g < n_waves) ? wave_item[g + 1] : 0;
        for (;;) {
            if (i < i_end) {            // one call site: the item's registers as in other modes
                fwd_item<COUL, ENERGY, VIRIAL, PRUNE>(i, NB_ITEM_ARGS);
                ++i;
                continue;
            }
            // read the counter first: a pool that is done takes no more atomics
            if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(
                    ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >= runs_p)
                break;
            int t = 0;
            if (lane == 0) t = atomicAdd(ticket, 1);
            t = __builtin_amdgcn_readlane(t, 0);
            if (t >= runs_p) break;
            const int k = p + kQueuePools * t;
            i = dyn_item[k];
            i_end = dyn_item[k + 1];
        }
        // every wavefront of the block has taken its last ticket: count the block done
        __shared__ int s_last;
        __syncthreads();
        // (no fences: an agent-scope fence writes back and invalidates the XCD's whole L2,
        // costing tens of microseconds over the grid; the counters are only ever touched
        // by atomics, which take effect in order at one coherent point)
        if (threadIdx.x == 0) {
            const int grp = (int)blockIdx.x % kQueuePools;
            const int grp_blocks = ((int)gridDim.x - grp + kQueuePools - 1) / kQueuePools;
            const int groups = min((int)gridDim.x, kQueuePools);
            s_last = atomicAdd(queue + kQueueDone + grp * kPoolStride, 1) == grp_blocks - 1 &&
                     atomicAdd(queue + kQueueDoneAll, 1) == groups - 1;
        }
        __syncthreads();
        if (s_last) {
            // the last block: no other wavefront of this launch touches the counters now
            for (int k = threadIdx.x; k < kQueuePools; k += blockDim.x) {
                __hip_atomic_store(tickets + k * kPoolStride, 0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(queue + kQueueDone + k * kPoolStride, 0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            if (threadIdx.x == 0)
                __hip_atomic_store(queue + kQueueDoneAll, 0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    if (mode == kExecPersist) {
        const int G = (int)gridDim.x * kFwdWaves;
        // Blocks are dispatched round robin over the CUs (block b shares its CU with
        // b +- n_cu, measured), so with positions in plain block order CU 0 would take the
        // most expensive item of every CU round and the last CU the cheapest.  Positions
        // snake instead: odd CU rounds of blocks take theirs in reverse.
        const int b = (int)blockIdx.x, r = b / n_cu, at = b - r * n_cu;
        const int m = min(n_cu, (int)gridDim.x - r * n_cu);          // blocks in round r
        const int g = (r * n_cu + ((r & 1) ? m - 1 - at : at)) * kFwdWaves + wave;
        for (int base = 0, odd = 0; base < n_items; base += G, odd ^= 1) {
            const int slot = base + (odd ? G - 1 - g : g);
            if (slot < n_items) fwd_item<COUL, ENERGY, VIRIAL, PRUNE>(order[slot], NB_ITEM_ARGS);
        }
        return;
    }
    const int b = (mode == kExecXcd) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int item = b * kFwdWaves + wave;
    if (item < n_items) fwd_item<COUL, ENERGY, VIRIAL, PRUNE>(item, NB_ITEM_ARGS);
#undef NB_ITEM_ARGS
}

inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

// Resident blocks per CU of one flavor.
template <int COUL, bool E, bool V, bool P>
int fwd_blocks_per_cu(size_t lds) {
    // resident blocks per CU of this kernel flavour for the last LJ-table size asked
    static int per_cu = 0;
    static size_t per_cu_lds = 0;
    if (per_cu == 0 || per_cu_lds != lds) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_nb_fwd<COUL, E, V, P>,
                                                         kFwdThreads, lds) != hipSuccess)
            nb = 0;
        per_cu = nb > 0 ? nb : 1;
        per_cu_lds = lds;
    }
    return per_cu;
}

template <int COUL, bool P>
int prepare_fwd_c(uint32_t flags, size_t lds) {
    const bool E = (flags & NB_F_ENERGY) != 0, V = (flags & NB_F_VIRIAL) != 0;
    if (E && V) return fwd_blocks_per_cu<COUL, true, true, P>(lds);
    if (E) return fwd_blocks_per_cu<COUL, true, false, P>(lds);
    if (V) return fwd_blocks_per_cu<COUL, false, true, P>(lds);
    return fwd_blocks_per_cu<COUL, false, false, P>(lds);
}

template <int COUL, bool E, bool V, bool P>
void launch_fwd_t(const NbDev& d, const NbKParams& kp, const float* lj, int n_items,
                  int part, int nstprune, float r2_inner, int mode, hipStream_t s) {
    const size_t lds = sizeof(float4) * (size_t)kp.n_types * kp.n_types;
    int grid = blocks(n_items, kFwdWaves);
    if (mode == kExecPersist)   // one resident grid over the device
        grid = std::min(grid, fwd_blocks_per_cu<COUL, E, V, P>(lds) * std::max(d.n_cu, 1));
    if (mode == kExecBalanced || mode == kExecQueue) grid = blocks(d.n_waves, kFwdWaves);
    hipLaunchKernelGGL((k_nb_fwd<COUL, E, V, P>), dim3(grid), dim3(kFwdThreads), lds, s,
                       d.items, d.entries, d.excl_rows, d.xq, d.type_slot, d.sc_info, d.sys,
                       lj, d.jpart, d.ipart, d.epart, d.epart_stride, kp, n_items, part,
                       nstprune, r2_inner, mode, d.item_order, d.queue, d.wave_item, d.n_waves,
                       d.n_dyn, std::max(d.n_cu, 1));
}

template <int COUL, bool P>
void launch_fwd_c(const NbDev& d, const NbKParams& kp, uint32_t flags, const float* lj,
                  int n_items, int part, int nstprune, float r2_inner, int mode, hipStream_t s) {
    const bool E = (flags & NB_F_ENERGY) != 0, V = (flags & NB_F_VIRIAL) != 0;
    if (E && V) launch_fwd_t<COUL, true, true, P>(d, kp, lj, n_items, part, nstprune, r2_inner, mode, s);
    else if (E) launch_fwd_t<COUL, true, false, P>(d, kp, lj, n_items, part, nstprune, r2_inner, mode, s);
    else if (V) launch_fwd_t<COUL, false, true, P>(d, kp, lj, n_items, part, nstprune, r2_inner, mode, s);
    else launch_fwd_t<COUL, false, false, P>(d, kp, lj, n_items, part, nstprune, r2_inner, mode, s);
}

}  // namespace

hipError_t prepare_forces(int coulomb, uint32_t flags, bool prune, int n_types,
                          int* waves_per_cu) {
    const size_t lds = sizeof(float4) * (size_t)n_types * n_types;
    int nb;
    if (coulomb == NB_COUL_RF)
        nb = prune ? prepare_fwd_c<NB_COUL_RF, true>(flags, lds)
                   : prepare_fwd_c<NB_COUL_RF, false>(flags, lds);
    else if (coulomb == NB_COUL_NONE)
        nb = prune ? prepare_fwd_c<NB_COUL_NONE, true>(flags, lds)
                   : prepare_fwd_c<NB_COUL_NONE, false>(flags, lds);
    else
        nb = prune ? prepare_fwd_c<NB_COUL_EWALD, true>(flags, lds)
                   : prepare_fwd_c<NB_COUL_EWALD, false>(flags, lds);
    if (waves_per_cu) *waves_per_cu = nb * kFwdWaves;
    return hipGetLastError();
}

hipError_t launch_forces(const NbDev& d, const NbKParams& kp, int coulomb, uint32_t flags,
                         const float* lj, int n_items, int prune_part, int nstprune,
                         float r2_inner, int mode, hipStream_t s) {
    if (n_items <= 0) return hipGetLastError();
    const bool P = prune_part >= 0;
    const float r2 = P ? r2_inner : 0.f;
    const int part = P ? prune_part : -1, np = std::max(nstprune, 1);
    if (coulomb == NB_COUL_RF) {
        if (P) launch_fwd_c<NB_COUL_RF, true>(d, kp, flags, lj, n_items, part, np, r2, mode, s);
        else launch_fwd_c<NB_COUL_RF, false>(d, kp, flags, lj, n_items, part, np, r2, mode, s);
    } else if (coulomb == NB_COUL_NONE) {
        if (P) launch_fwd_c<NB_COUL_NONE, true>(d, kp, flags, lj, n_items, part, np, r2, mode, s);
        else launch_fwd_c<NB_COUL_NONE, false>(d, kp, flags, lj, n_items, part, np, r2, mode, s);
    } else {
        if (P) launch_fwd_c<NB_COUL_EWALD, true>(d, kp, flags, lj, n_items, part, np, r2, mode, s);
        else launch_fwd_c<NB_COUL_EWALD, false>(d, kp, flags, lj, n_items, part, np, r2, mode, s);
    }
    return hipGetLastError();
}
