// Backward pass of the cluster-pair force kernel over the frozen inner list.
//
// For a loss L(F, E) with adjoint G = dL/dF and gE = dL/dE (per system: LJ, Coulomb), each
// pair inside the cut-off with separation d = x_i - x_j, phi = -V'(r)/r, contributes
//   u        = (G_i - G_j) . d
//   h        = (phi'(r)/r) u d + phi (G_i - G_j) - (gE_LJ phi_LJ + gE_C phi_C) d
//   dL/dx_i += h,  dL/dx_j -= h          (Hessian-vector product; dE/dx = -F)
//   dL/dq_i += K q_j (psi u + gE_C v),   dL/dq_j += K q_i (psi u + gE_C v)
//              with phi_C = K q_i q_j psi(r), V_C = K q_i q_j v(r), K = epsfac / eps_r
//   dL/dc12 += u 12 r^-14 + gE_LJ (r^-12 - m rc^-12)
//   dL/dc6  += u (-6 r^-8) + gE_LJ (-r^-6 + m rc^-6)     for the pair's (t_i, t_j)
// The loop structure is the forward kernel's: one wavefront per work item, lane =
// (ii, jj), i-data, i-adjoints and i-gradients in registers, j-gradients reduced over the
// i-lanes with DPP and stored once per entry, table gradients in per-lane LDS
// histograms reduced per item.  A second pass sums the partials per atom (compensated)
// and the table partials per type pair in double precision.
#include <algorithm>

#include "nb_chunk_sums.h"
#include "nb_internal.h"
#include "nb_pair_common.h"


namespace {

constexpr int kBwdWaves = 2;
constexpr int kBwdThreads = kBwdWaves * kWave;
constexpr int kPrivateHistTypes = 4;   // per-lane histograms up to this many types

struct BScal {
    float gel, gec;                // dL/dE_LJ, dL/dE_C of the item's system
    float rc_m6, rc_m12;
};

// One 8x8 block of pairs: i-atom data and accumulators as scalars (lane = ii + 8 jj).
// xj is the lane's j-atom with the entry's periodic shift already added, lj_j the LDS
// address of row 0 of the LJ table plus 16 bytes times the j-atom's type, tj16 that
// offset alone (s_ti holds 16 T type_i per slot).
template <int COUL, bool LJGRAD, bool PRIV>
__device__ __forceinline__ void bwd_block(
    const float4* s_x, const float4* s_gq, const int* s_ti, uint64_t m,
    float& ax, float& ay, float& az, float& aq, const float4& xj, const float4& gj, int tj16,
    const char* lj_j, float* __restrict__ s_hist, int lane, const NbKParams& kp,
    const BScal& bs, float& ajx, float& ajy, float& ajz, float& ajq) {
    const float4 xv = *s_x;                            // (x_i, y_i, z_i, -) of this lane
    const float dx = xv.x - xj.x, dy = xv.y - xj.y, dz = xv.z - xj.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const uint64_t act = __builtin_amdgcn_ballot_w64(r2 < kp.rc2) & m;
    if (!act) return;
    const bool on = __builtin_amdgcn_inverse_ballot_w64(act);
    const float4 gq = *s_gq;                           // (G_i, K q_i) of this lane's i-atom
    const float gxi = gq.x, gyi = gq.y, gzi = gq.z, qi = gq.w;
    const int ti16 = *s_ti;
    const float4 p = *reinterpret_cast<const float4*>(lj_j + ti16);   // (6 c6, 12 c12, shift, c6)
    // Pairs outside the cut-off or excluded get 1/r = 0 and q_i q_j = 0: the force terms
    // and their derivatives below vanish (r2 stays finite); the energy-derivative terms
    // w, g6, g12 are masked explicitly.
    const float rinv = on ? __builtin_amdgcn_rsqf(r2) : 0.f;
    const float rinv2 = rinv * rinv;
    const float rinv6 = rinv2 * rinv2 * rinv2;
    const float a = p.y * rinv6;                       // 12 c12 r^-6
    const float phi_lj = rinv6 * (a - p.x) * rinv2;
    const float dphi_lj = rinv6 * rinv2 * rinv2 * fmaf(-14.0f, a, 8.0f * p.x);
    const float qq = on ? qi * xj.w : 0.f;
    float psi, dpsi, v;
    if (COUL == NB_COUL_NONE) {
        psi = dpsi = v = 0.f;
    } else if (COUL == NB_COUL_RF) {
        psi = rinv * rinv2 - 2.0f * kp.krf;
        dpsi = -3.0f * rinv2 * rinv2 * rinv;
        v = fmaf(kp.krf, r2, rinv) - kp.crf;
    } else {
        const float r = r2 * rinv;
        const float e = __builtin_amdgcn_exp2f(r2 * kp.beta2_log2e);
        const float erfcv = e * erfcx_poly(r, kp.p_beta);
        const float te = kp.two_beta_sqrtpi * e;
        const float g = fmaf(erfcv, rinv, te);
        psi = g * rinv2;
        dpsi = fmaf(-3.0f * g, rinv2 * rinv2, -2.0f * kp.beta * kp.beta * te * rinv2);
        v = fmaf(erfcv, rinv, -kp.ewald_shift);
    }
    const float phi_c = qq * psi;
    const float gdx = gxi - gj.x, gdy = gyi - gj.y, gdz = gzi - gj.z;
    const float u = fmaf(gdx, dx, fmaf(gdy, dy, gdz * dz));
    const float phi = phi_lj + phi_c;
    const float coef = fmaf(dphi_lj + qq * dpsi, u, -fmaf(bs.gel, phi_lj, bs.gec * phi_c));
    const float hx = fmaf(coef, dx, phi * gdx);
    const float hy = fmaf(coef, dy, phi * gdy);
    const float hz = fmaf(coef, dz, phi * gdz);
    const float w = on ? fmaf(psi, u, bs.gec * v) : 0.f;
    ax += hx;
    ay += hy;
    az += hz;
    aq = fmaf(xj.w, w, aq);                  // times K after the item
    ajx -= hx;
    ajy -= hy;
    ajz -= hz;
    ajq = fmaf(qi, w, ajq);                  // qi already holds K q_i
    if (LJGRAD) {
        const float rinv12 = rinv6 * rinv6;
        float g12 = fmaf(u * 12.0f * rinv2, rinv12, bs.gel * (rinv12 - bs.rc_m12));
        float g6 = fmaf(u * -6.0f * rinv2, rinv6, bs.gel * (bs.rc_m6 - rinv6));
        g12 = on ? g12 : 0.f;
        g6 = on ? g6 : 0.f;
        const int key16 = ti16 + tj16;                // 16 (type_i T + type_j)
        if (PRIV) {
            // lane-private slots: plain read-modify-write (no LDS atomics needed)
            float2* h = reinterpret_cast<float2*>(reinterpret_cast<char*>(s_hist) +
                                                  key16 * (int)(kWave * sizeof(float2) / 16)) +
                        lane;
            float2 hv = *h;
            hv.x += g6;
            hv.y += g12;
            *h = hv;
        } else {
            atomicAdd(&s_hist[key16 >> 3], g6);
            atomicAdd(&s_hist[(key16 >> 3) + 1], g12);
        }
    }
}

#define NB_FOR8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

// The work of one item (one wavefront): s_x, s_gq, s_ti the wavefront's LDS tables of the
// super-cluster's atoms, s_hist its table-gradient histogram (zero on entry, zero again
// on return).
template <int COUL, bool LJGRAD, bool PRIV>
__device__ __forceinline__ void bwd_item(
    const int item, const int lane, float4* s_x, float4* s_gq, int* s_ti,
    const float4* __restrict__ s_lj, float* __restrict__ s_hist,
    const NbItem* __restrict__ items, const NbEntry* __restrict__ entries,
    const uint64_t* __restrict__ excl_rows, const float4* __restrict__ xq,
    const float4* __restrict__ gslot, const int32_t* __restrict__ type_slot,
    const NbScInfo* __restrict__ sc_info, const NbSys* __restrict__ sys,
    const double* __restrict__ grad_e, float4* __restrict__ jpart, float4* __restrict__ ipart,
    float* __restrict__ glj_part, int glj_stride, const NbKParams& kp) {
    const int T = kp.n_types;
    const int TT = T * T;
    const NbItem it = items[item];
    const int ii = lane & 7, jj = lane >> 3;
    const int sc = it.sc, ci0 = kClustersPerSc * sc;
    const int sysi = sc_info[sc].sys;
    const NbSys S = sys[sysi];
    BScal bs;
    bs.gel = grad_e ? (float)grad_e[2 * sysi] : 0.f;
    bs.gec = grad_e ? (float)grad_e[2 * sysi + 1] : 0.f;
    bs.rc_m6 = kp.rc_m6;
    bs.rc_m12 = kp.rc_m12;
    {
        // lane l holds slot l of the super-cluster: (8 c + ii) for c = l >> 3
        const float4 v = xq[kScAtoms * sc + lane];
        const float4 g = gslot[kScAtoms * sc + lane];
        s_x[lane] = v;
        s_gq[lane] = make_float4(g.x, g.y, g.z, v.w * kp.epsfac_r);
        s_ti[lane] = type_slot[kScAtoms * sc + lane] * T;   // type_slot holds 16 type
    }
    __builtin_amdgcn_wave_barrier();

#define NB_IZERO(c) float ax##c = 0.f, ay##c = 0.f, az##c = 0.f, aq##c = 0.f;
    NB_FOR8(NB_IZERO)
#undef NB_IZERO

    const int e_end = it.e0 + it.ne;
    NbEntry nxt = entries[it.e0];
    float4 xj_n = xq[kClusterSize * nxt.cj + jj];
    float4 gj_n = gslot[kClusterSize * nxt.cj + jj];
    int tj_n = type_slot[kClusterSize * nxt.cj + jj];
    for (int e = it.e0; e < e_end; ++e) {
        const NbEntry ent = nxt;
        float4 xj = xj_n;
        const float4 gj = gj_n;
        const int tj = tj_n;
        if (e + 1 < e_end) {
            nxt = entries[e + 1];
            xj_n = xq[kClusterSize * nxt.cj + jj];
            gj_n = gslot[kClusterSize * nxt.cj + jj];
            tj_n = type_slot[kClusterSize * nxt.cj + jj];
        }
        const uint32_t mask = (ent.meta >> 16) & 0xffu;
        float4* jp = jpart + (size_t)ent.jpos * kClusterSize;
        // An entry with an empty mask runs no block and stores zero j-partials below (no
        // early exit: a second path to the loop latch makes the compiler copy all
        // loop-carried accumulators at every entry).
        const int code = ent.meta & 31u;
        const uint64_t* xrow =
            (ent.excl >= 0) ? excl_rows + (size_t)ent.excl * kClustersPerSc : nullptr;
        const bool self = (ent.cj >> 3) == sc && code == kShiftZero;
        const int dc = ent.cj - ci0;
        float ajx = 0.f, ajy = 0.f, ajz = 0.f, ajq = 0.f;
        // empty slots sit far outside the box (no distance test passes): only exclusions
        // and, for a cluster with itself, ii < jj are masked
#define NB_MASK(c)                                                                     \
    ((xrow ? xrow[c] : ~0ull) & ((self && dc == c) ? 0x7f3f1f0f07030100ull : ~0ull))
        // Periodic image of the j-cluster: x_j + s L, added once per entry.
        {
            const int sx = shift_x(code), sy = shift_y(code), sz = shift_z(code);
            xj.x += shift_value(sx, S.L[0]);
            xj.y += shift_value(sy, S.L[1]);
            xj.z += shift_value(sz, S.L[2]);
            const int tj16 = tj;                 // type_slot holds 16 type
            const char* lj_j = reinterpret_cast<const char*>(s_lj) + tj16;
#define NB_BLOCK(c)                                                                    \
    if ((mask >> c) & 1u)                                                              \
        bwd_block<COUL, LJGRAD, PRIV>(                                                 \
            s_x + kClusterSize * c + ii, s_gq + kClusterSize * c + ii,                  \
            s_ti + kClusterSize * c + ii,                                                \
            NB_MASK(c), ax##c, ay##c, az##c, aq##c, xj, gj, tj16, lj_j, s_hist, lane, kp, bs, \
            ajx, ajy, ajz, ajq);
            NB_FOR8(NB_BLOCK)
#undef NB_BLOCK
        }
#undef NB_MASK
        ajx = dpp_sum8(ajx);
        ajy = dpp_sum8(ajy);
        ajz = dpp_sum8(ajz);
        ajq = dpp_sum8(ajq);
        store_stream(&jp[jj], ajx, ajy, ajz, ajq);   // the same sums in all eight lanes
    }
    float4* ip = ipart + (size_t)item * kScAtoms;
#define NB_IRED(c)                                                                     \
    for (int off = 8; off < kWave; off <<= 1) {                                        \
        ax##c += __shfl_xor(ax##c, off);                                               \
        ay##c += __shfl_xor(ay##c, off);                                               \
        az##c += __shfl_xor(az##c, off);                                               \
        aq##c += __shfl_xor(aq##c, off);                                               \
    }                                                                                  \
    if (jj == 0)                                                                       \
        store_stream(&ip[kClusterSize * c + ii], ax##c, ay##c, az##c, aq##c * kp.epsfac_r);
    NB_FOR8(NB_IRED)
#undef NB_IRED
    if (LJGRAD) {
        __builtin_amdgcn_wave_barrier();
        // column it.pos of the [key][rank] table partials
        for (int k = lane; k < 2 * TT; k += kWave) {
            float v = 0.f;
            if (PRIV) {
                // slot (key, lane) holds (g6, g12) at float offset 2 (key * 64 + lane) + c
                const int key = k >> 1, c = k & 1;
                for (int l = 0; l < kWave; ++l) v += s_hist[2 * (key * kWave + l) + c];
            } else {
                v = s_hist[k];
            }
            glj_part[(size_t)k * glj_stride + it.pos] = v;
        }
        // Cleared for the wavefront's next item.  The LDS operations of one wavefront
        // complete in order, so these writes follow every read above.
        const int hist_per_wave = PRIV ? 2 * TT * kWave : 2 * TT;
        for (int k = lane; k < hist_per_wave; k += kWave) s_hist[k] = 0.f;
        __builtin_amdgcn_wave_barrier();
    }
}

// Execution: one wavefront per item in item order, or (kExecPersist) a grid resident on
// the device once, taking items in rounds of the most-work-first order as the forward
// kernel's persistent mode does.
template <int COUL, bool LJGRAD, bool PRIV>
__global__ __launch_bounds__(kBwdThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_nb_bwd(
    const NbItem* __restrict__ items, const NbEntry* __restrict__ entries,
    const uint64_t* __restrict__ excl_rows, const float4* __restrict__ xq,
    const float4* __restrict__ gslot, const int32_t* __restrict__ type_slot,
    const NbScInfo* __restrict__ sc_info,
    const NbSys* __restrict__ sys, const float* __restrict__ lj,
    const double* __restrict__ grad_e, float4* __restrict__ jpart, float4* __restrict__ ipart,
    float* __restrict__ glj_part, int glj_stride, NbKParams kp, int n_items, int mode,
    const int32_t* __restrict__ order, int n_cu) {
    extern __shared__ float4 s_dyn[];
    __shared__ float4 s_x_all[kBwdWaves][kScAtoms];    // per wave: (x_i, y_i, z_i, q_i)
    __shared__ float4 s_gq_all[kBwdWaves][kScAtoms];   // per wave: (G_i, K q_i)
    __shared__ int s_ti_all[kBwdWaves][kScAtoms];      // per wave: 16 T type_i
    const int T = kp.n_types;
    const int TT = T * T;
    float4* s_lj = s_dyn;
    float* s_hist_all = reinterpret_cast<float*>(s_dyn + TT);
    const int hist_per_wave = PRIV ? 2 * TT * kWave : 2 * TT;
    for (int i = threadIdx.x; i < TT; i += blockDim.x) {
        const float c6 = lj[2 * i], c12 = lj[2 * i + 1];
        s_lj[i] = make_float4(6.0f * c6, 12.0f * c12, c12 * kp.rc_m12 - c6 * kp.rc_m6, c6);
    }
    if (LJGRAD)
        for (int i = threadIdx.x; i < hist_per_wave * kBwdWaves; i += blockDim.x) s_hist_all[i] = 0.f;
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
#define NB_ITEM_ARGS                                                                    \
    lane, s_x_all[wave], s_gq_all[wave], s_ti_all[wave], s_lj,                           \
        s_hist_all + wave * hist_per_wave, items, entries, excl_rows, xq, gslot, type_slot, \
        sc_info, sys, grad_e, jpart, ipart, glj_part, glj_stride, kp
    if (mode == kExecPersist) {
        const int G = (int)gridDim.x * kBwdWaves;
        // positions snake over the CU rounds of blocks (odd rounds reversed), as in the
        // forward kernel: blocks are dealt to the CUs round robin
        const int b = (int)blockIdx.x, r = b / n_cu, at = b - r * n_cu;
        const int m = min(n_cu, (int)gridDim.x - r * n_cu);
        const int g = (r * n_cu + ((r & 1) ? m - 1 - at : at)) * kBwdWaves + wave;
        for (int base = 0, odd = 0; base < n_items; base += G, odd ^= 1) {
            const int slot = base + (odd ? G - 1 - g : g);
            if (slot < n_items) bwd_item<COUL, LJGRAD, PRIV>(order[slot], NB_ITEM_ARGS);
        }
        return;
    }
    const int item = blockIdx.x * kBwdWaves + wave;
    if (item < n_items) bwd_item<COUL, LJGRAD, PRIV>(item, NB_ITEM_ARGS);
#undef NB_ITEM_ARGS
}

// Slot-order adjoint G from the caller's per-atom dL/dF.
__global__ void k_gather_g(NbDev d, const float* __restrict__ g, int n_slots) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n_slots) return;
    const int a = d.slot_atom[slot];
    d.gslot[slot] = (a >= 0) ? make_float4(g[3 * a], g[3 * a + 1], g[3 * a + 2], 0.f)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
}

__device__ inline void neumaier(float& s, float& c, float v) {
    const float t = s + v;
    c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
}

// One wavefront per super-cluster, as the force reduction: each lane (slot) sums with
// compensation the j-partials of its cluster's segment and then the super-cluster's item
// rows, in a fixed order, and writes dL/dx and dL/dq in the caller's atom order.
constexpr int kRedWaves = 4;
__device__ inline void reduce_bwd_sc(
    int sc, const int32_t* __restrict__ slot_atom, const int32_t* __restrict__ jseg_start,
    const float4* __restrict__ jpart, const int32_t* __restrict__ sc_istart,
    const int32_t* __restrict__ sc_icount, const float4* __restrict__ ipart,
    float* __restrict__ gx, float* __restrict__ gq, int accumulate) {
    const int lane = threadIdx.x & (kWave - 1);
    const int jj = lane & 7;
    const int cj = sc * kClustersPerSc + (lane >> 3);
    const int slot = sc * kScAtoms + lane;
    const int s0 = jseg_start[cj], s1 = jseg_start[cj + 1];
    const int i0 = sc_istart[sc], i1 = i0 + sc_icount[sc];
    float s[4] = {0, 0, 0, 0}, cmp[4] = {0, 0, 0, 0};
#pragma unroll 4
    for (int k = s0; k < s1; ++k) {
        const float4 v = jpart[(size_t)k * kClusterSize + jj];
        neumaier(s[0], cmp[0], v.x);
        neumaier(s[1], cmp[1], v.y);
        neumaier(s[2], cmp[2], v.z);
        neumaier(s[3], cmp[3], v.w);
    }
#pragma unroll 2
    for (int i = i0; i < i1; ++i) {
        const float4 v = ipart[(size_t)i * kScAtoms + lane];
        neumaier(s[0], cmp[0], v.x);
        neumaier(s[1], cmp[1], v.y);
        neumaier(s[2], cmp[2], v.z);
        neumaier(s[3], cmp[3], v.w);
    }
    const int a = slot_atom[slot];
    if (a < 0) return;
    if (gx) {
        for (int k = 0; k < 3; ++k) {
            const float r = s[k] + cmp[k];
            gx[3 * a + k] = accumulate ? gx[3 * a + k] + r : r;
        }
    }
    if (gq) {
        const float r = s[3] + cmp[3];
        gq[a] = accumulate ? gq[a] + r : r;
    }
}

// Table gradient totals: thread t of the block takes the (type pair, c6/c12) keys t,
// t + blockDim.x, ... and adds the chunk partials in order.  The table is symmetric, so
// the derivative with respect to the shared value of [t1][t2] and [t2][t1] is split
// evenly between the two entries (independent of which atom of a pair the kernel treats
// as i).
__device__ inline void glj_totals(const NbDev& d, double* __restrict__ out, int n_types,
                                  int n_chunks, int accumulate) {
    const int n_keys = 2 * n_types * n_types;
    for (int k = threadIdx.x; k < n_keys; k += blockDim.x) {
        const int c = k & 1, t1 = (k >> 1) / n_types, t2 = (k >> 1) % n_types;
        const int kt = 2 * (t2 * n_types + t1) + c;
        double sk = 0.0, st = 0.0;
        for (int q = 0; q < n_chunks; ++q) {
            sk += d.cpart[(size_t)q * kChunkVals + k];
            st += d.cpart[(size_t)q * kChunkVals + kt];
        }
        const double r = (kt != k) ? 0.5 * (sk + st) : sk;
        out[k] = accumulate ? out[k] + r : r;
    }
}

// Input-gradient reduction and the table-gradient reduction in one launch: blocks
// [0, n_gblk) reduce four super-clusters each (one wavefront per super-cluster), blocks [n_gblk,
// n_gblk + n_chunks) sum kChunkItems item ranks of the table-gradient partials each; the
// last of those to finish (a ticket in queue[3], taken after a device-scope fence) forms
// the totals and resets the ticket for the next launch.
__global__ __launch_bounds__(kRedThreads) void k_reduce_bwd_step(
    NbDev d, float* __restrict__ gx, float* __restrict__ gq, double* __restrict__ glj,
    int accumulate, int n_sc, int n_gblk, int n_types, int n_items, int n_chunks) {
    static_assert(kRedThreads == kRedWaves * kWave, "one block shape for both parts");
    if ((int)blockIdx.x >= n_gblk) {
        const int c = blockIdx.x - n_gblk;
        const int p0 = c * kChunkItems, p1 = min(n_items, p0 + kChunkItems);
        chunk_sums(d.glj_part, d.epart_stride, 2 * n_types * n_types, p0, p1,
                   d.cpart + (size_t)c * kChunkVals);
        // One release fence per block, by the thread that takes the ticket: the barrier
        // orders the block's partial stores before it.  (A device-scope fence writes the
        // XCD's L2 back; one per wavefront cost about 2 us per launch at 96k atoms.)
        __shared__ int s_last;
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            s_last = (atomicAdd(d.queue + 3, 1) == n_chunks - 1);
        }
        __syncthreads();
        if (s_last) {
            // every other block's partials, released before their tickets
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            glj_totals(d, glj, n_types, n_chunks, accumulate);
            if (threadIdx.x == 0) atomicExch(d.queue + 3, 0);
        }
        return;
    }
    const int sc = blockIdx.x * kRedWaves + (int)(threadIdx.x / kWave);
    if (sc >= n_sc) return;
    reduce_bwd_sc(sc, d.slot_atom, d.jseg_start, d.jpart, d.sc_istart, d.sc_icount, d.ipart, gx,
                  gq, accumulate);
}

// Table gradient totals when there is no item (all zero, or the outputs kept).
__global__ void k_glj_final(NbDev d, double* __restrict__ out, int n_types, int accumulate) {
    glj_totals(d, out, n_types, 0, accumulate);
}

inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

template <int COUL, bool LJGRAD, bool PRIV>
int bwd_blocks_per_cu(size_t lds) {
    // resident blocks per CU of this kernel flavour for the last LDS size asked
    static int per_cu = 0;
    static size_t per_cu_lds = 0;
    if (per_cu == 0 || per_cu_lds != lds) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_nb_bwd<COUL, LJGRAD, PRIV>,
                                                         kBwdThreads, lds) != hipSuccess)
            nb = 0;
        per_cu = nb > 0 ? nb : 1;
        per_cu_lds = lds;
    }
    return per_cu;
}

// Dynamic LDS of one flavor: the LJ table and the table-gradient histograms.
template <bool LJG, bool PRIV>
size_t bwd_lds(int n_types) {
    const int TT = n_types * n_types;
    const size_t hist = LJG ? (size_t)(PRIV ? 2 * TT * kWave : 2 * TT) * kBwdWaves : 0;
    return sizeof(float4) * TT + sizeof(float) * hist;
}

template <int COUL>
int bwd_waves_c(bool ljgrad, int n_types) {
    if (!ljgrad) return bwd_blocks_per_cu<COUL, false, false>(bwd_lds<false, false>(n_types));
    if (n_types <= kPrivateHistTypes)
        return bwd_blocks_per_cu<COUL, true, true>(bwd_lds<true, true>(n_types));
    return bwd_blocks_per_cu<COUL, true, false>(bwd_lds<true, false>(n_types));
}

template <int COUL, bool LJG, bool PRIV>
void launch_bwd_t(const NbDev& d, const NbKParams& kp, const float* lj, const double* ge,
                  int n_items, int mode, hipStream_t s) {
    const size_t lds = bwd_lds<LJG, PRIV>(kp.n_types);
    // the persistent schedule when the context runs the forward pass that way, else
    // one wavefront per item
    const int bmode = (mode == kExecPersist) ? kExecPersist : kExecStatic;
    int grid = blocks(n_items, kBwdWaves);
    if (bmode == kExecPersist)
        grid = std::min(grid, bwd_blocks_per_cu<COUL, LJG, PRIV>(lds) * std::max(d.n_cu, 1));
    hipLaunchKernelGGL((k_nb_bwd<COUL, LJG, PRIV>), dim3(grid), dim3(kBwdThreads), lds, s,
                       d.items, d.entries, d.excl_rows, d.xq, d.gslot, d.type_slot, d.sc_info,
                       d.sys, lj, ge, d.jpart, d.ipart, d.glj_part, d.epart_stride, kp, n_items,
                       bmode, d.item_order, std::max(d.n_cu, 1));
}

template <int COUL>
void launch_bwd_c(const NbDev& d, const NbKParams& kp, const float* lj, const double* ge,
                  bool ljgrad, int n_items, int mode, hipStream_t s) {
    if (!ljgrad) launch_bwd_t<COUL, false, false>(d, kp, lj, ge, n_items, mode, s);
    else if (kp.n_types <= kPrivateHistTypes) launch_bwd_t<COUL, true, true>(d, kp, lj, ge, n_items, mode, s);
    else launch_bwd_t<COUL, true, false>(d, kp, lj, ge, n_items, mode, s);
}

}  // namespace

int backward_waves_per_cu(int coulomb, bool ljgrad, int n_types) {
    const int blocks_per_cu = (coulomb == NB_COUL_RF)     ? bwd_waves_c<NB_COUL_RF>(ljgrad, n_types)
                              : (coulomb == NB_COUL_NONE) ? bwd_waves_c<NB_COUL_NONE>(ljgrad, n_types)
                                                          : bwd_waves_c<NB_COUL_EWALD>(ljgrad, n_types);
    return blocks_per_cu * kBwdWaves;
}

hipError_t launch_backward(const NbDev& d, const NbKParams& kp, int coulomb, const float* lj,
                           const float* grad_f, const double* grad_energy, bool ljgrad,
                           int n_slots, int n_items, int mode, hipStream_t s) {
    if (n_slots > 0)
        hipLaunchKernelGGL(k_gather_g, dim3(blocks(n_slots, 256)), dim3(256), 0, s, d, grad_f,
                           n_slots);
    if (n_items > 0) {
        if (coulomb == NB_COUL_RF)
            launch_bwd_c<NB_COUL_RF>(d, kp, lj, grad_energy, ljgrad, n_items, mode, s);
        else if (coulomb == NB_COUL_NONE)
            launch_bwd_c<NB_COUL_NONE>(d, kp, lj, grad_energy, ljgrad, n_items, mode, s);
        else
            launch_bwd_c<NB_COUL_EWALD>(d, kp, lj, grad_energy, ljgrad, n_items, mode, s);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_backward(const NbDev& d, float* grad_x, float* grad_q, double* grad_lj,
                                  bool accumulate, int n_slots, int n_types, int n_items,
                                  hipStream_t s) {
    const int n_sc = n_slots / kScAtoms;
    const int n_gblk = (grad_x || grad_q) ? blocks(n_sc, kRedWaves) : 0;
    const int n_chunks = grad_lj ? blocks(n_items, kChunkItems) : 0;
    if (n_gblk + n_chunks > 0)
        hipLaunchKernelGGL(k_reduce_bwd_step, dim3(n_gblk + n_chunks), dim3(kRedThreads), 0, s,
                           d, grad_x, grad_q, grad_lj, accumulate ? 1 : 0, n_sc, n_gblk,
                           n_types, n_items, n_chunks);
    if (grad_lj && n_chunks == 0)
        hipLaunchKernelGGL(k_glj_final, dim3(1), dim3(kRedThreads), 0, s, d, grad_lj, n_types,
                           accumulate ? 1 : 0);
    return hipGetLastError();
}
