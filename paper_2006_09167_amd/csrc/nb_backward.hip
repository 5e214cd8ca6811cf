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
#include "nb_erfc_coeffs.h"
#include "nb_internal.h"

namespace {

constexpr int kBwdWaves = 2;
constexpr int kBwdThreads = kBwdWaves * kWave;
constexpr int kPrivateHistTypes = 4;   // per-lane histograms up to this many types

__device__ inline float dpp_sum8(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x141, 0xF, 0xF, false));
    return v;
}

__device__ inline int shift_x(int code) { return code / 9 - 1; }
__device__ inline int shift_y(int code) { return (code / 3) % 3 - 1; }
__device__ inline int shift_z(int code) { return code % 3 - 1; }

__device__ inline float erfcx_poly(float t) {
    const float u = __builtin_amdgcn_rcpf(fmaf(NB_ERFC_P, t, 1.0f));
    float p = NB_ERFC_C8;
    p = fmaf(p, u, NB_ERFC_C7);
    p = fmaf(p, u, NB_ERFC_C6);
    p = fmaf(p, u, NB_ERFC_C5);
    p = fmaf(p, u, NB_ERFC_C4);
    p = fmaf(p, u, NB_ERFC_C3);
    p = fmaf(p, u, NB_ERFC_C2);
    p = fmaf(p, u, NB_ERFC_C1);
    p = fmaf(p, u, NB_ERFC_C0);
    return u * p;
}

struct BData {
    float x[8], y[8], z[8], q[8];
    float gx[8], gy[8], gz[8];     // adjoint G of the i-atoms
    int t[8];
};

struct BAcc {
    float x[8], y[8], z[8], q[8];  // dL/dx_i and dL/dq_i / K accumulators
};

struct BScal {
    float gel, gec;                // dL/dE_LJ, dL/dE_C of the item's system
    float rc_m6, rc_m12;
};

template <int COUL, bool LJGRAD, bool PRIV, bool SHIFTED>
__device__ __forceinline__ void entry_bwd(
    const BData& I, BAcc& A, uint32_t mask, const uint64_t (&ivalid)[8], uint64_t jvalid,
    const uint64_t* __restrict__ xrow, int cj, int ci0, int code, float4 xj, float4 gj, int tj,
    const float4* __restrict__ s_lj, float* __restrict__ s_hist, int lane, const NbKParams& kp,
    const BScal& bs, float sxi, float syi, float szi, float& ajx, float& ajy, float& ajz,
    float& ajq) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!((mask >> c) & 1u)) continue;
        uint64_t m = ivalid[c] & jvalid;
        if (xrow) m &= xrow[c];
        if (cj == ci0 + c && code == kShiftZero) m &= 0x7f3f1f0f07030100ull;
        float dx, dy, dz;
        if (SHIFTED) {
            dx = (I.x[c] - sxi) - xj.x;
            dy = (I.y[c] - syi) - xj.y;
            dz = (I.z[c] - szi) - xj.z;
        } else {
            dx = I.x[c] - xj.x;
            dy = I.y[c] - xj.y;
            dz = I.z[c] - xj.z;
        }
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const uint64_t act = __builtin_amdgcn_ballot_w64(r2 < kp.rc2) & m;
        if (!act) continue;
        const bool on = __builtin_amdgcn_inverse_ballot_w64(act);
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float rinv2 = rinv * rinv;
        const float4 p = s_lj[I.t[c] + tj];              // (6 c6, 12 c12, shift, c6)
        const float rinv6 = rinv2 * rinv2 * rinv2;
        const float a = p.y * rinv6;                       // 12 c12 r^-6
        const float phi_lj = rinv6 * (a - p.x) * rinv2;
        const float dphi_lj = rinv6 * rinv2 * rinv2 * fmaf(-14.0f, a, 8.0f * p.x);
        const float qq = I.q[c] * xj.w;
        float psi, dpsi, v;
        if (COUL == NB_COUL_RF) {
            psi = rinv * rinv2 - 2.0f * kp.krf;
            dpsi = -3.0f * rinv2 * rinv2 * rinv;
            v = fmaf(kp.krf, r2, rinv) - kp.crf;
        } else {
            const float r = r2 * rinv;
            const float e = __builtin_amdgcn_exp2f(r2 * kp.beta2_log2e);
            const float erfcv = e * erfcx_poly(kp.beta * r);
            const float te = kp.two_beta_sqrtpi * e;
            const float g = fmaf(erfcv, rinv, te);
            psi = g * rinv2;
            dpsi = fmaf(-3.0f * g, rinv2 * rinv2, -2.0f * kp.beta * kp.beta * te * rinv2);
            v = fmaf(erfcv, rinv, -kp.ewald_shift);
        }
        const float phi_c = qq * psi;
        const float gdx = I.gx[c] - gj.x, gdy = I.gy[c] - gj.y, gdz = I.gz[c] - gj.z;
        const float u = fmaf(gdx, dx, fmaf(gdy, dy, gdz * dz));
        const float phi = phi_lj + phi_c;
        const float coef = fmaf(dphi_lj + qq * dpsi, u, -fmaf(bs.gel, phi_lj, bs.gec * phi_c));
        float hx = fmaf(coef, dx, phi * gdx);
        float hy = fmaf(coef, dy, phi * gdy);
        float hz = fmaf(coef, dz, phi * gdz);
        float w = fmaf(psi, u, bs.gec * v);
        hx = on ? hx : 0.f;
        hy = on ? hy : 0.f;
        hz = on ? hz : 0.f;
        w = on ? w : 0.f;
        A.x[c] += hx;
        A.y[c] += hy;
        A.z[c] += hz;
        A.q[c] = fmaf(xj.w, w, A.q[c]);          // times K after the item
        ajx -= hx;
        ajy -= hy;
        ajz -= hz;
        ajq = fmaf(I.q[c], w, ajq);              // I.q already holds K q_i
        if (LJGRAD) {
            const float rinv12 = rinv6 * rinv6;
            float g12 = fmaf(u * 12.0f * rinv2, rinv12, bs.gel * (rinv12 - bs.rc_m12));
            float g6 = fmaf(u * -6.0f * rinv2, rinv6, bs.gel * (bs.rc_m6 - rinv6));
            g12 = on ? g12 : 0.f;
            g6 = on ? g6 : 0.f;
            const int key = I.t[c] + tj;
            if (PRIV) {
                atomicAdd(&s_hist[(2 * key) * kWave + lane], g6);
                atomicAdd(&s_hist[(2 * key + 1) * kWave + lane], g12);
            } else {
                atomicAdd(&s_hist[2 * key], g6);
                atomicAdd(&s_hist[2 * key + 1], g12);
            }
        }
    }
}

template <int COUL, bool LJGRAD, bool PRIV>
__global__ __launch_bounds__(kBwdThreads) void k_nb_bwd(NbDev d, NbKParams kp,
                                                         const float* __restrict__ lj,
                                                         const double* __restrict__ grad_e,
                                                         int n_items) {
    extern __shared__ float4 s_dyn[];
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
    const int item = blockIdx.x * kBwdWaves + wave;
    if (item >= n_items) return;
    float* s_hist = s_hist_all + wave * hist_per_wave;
    const NbItem it = d.items[item];
    const int ii = lane & 7, jj = lane >> 3;
    const int sc = it.sc, ci0 = kClustersPerSc * sc;
    const NbSys S = d.sys[it.sys];
    BScal bs;
    bs.gel = grad_e ? (float)grad_e[2 * it.sys] : 0.f;
    bs.gec = grad_e ? (float)grad_e[2 * it.sys + 1] : 0.f;
    bs.rc_m6 = kp.rc_m6;
    bs.rc_m12 = kp.rc_m12;

    BData I;
    BAcc A;
    uint64_t ivalid[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int slot = kScAtoms * sc + kClusterSize * c + ii;
        const float4 v = d.xq[slot];
        const float4 g = d.gslot[slot];
        I.x[c] = v.x;
        I.y[c] = v.y;
        I.z[c] = v.z;
        I.q[c] = v.w * kp.epsfac_r;
        I.gx[c] = g.x;
        I.gy[c] = g.y;
        I.gz[c] = g.z;
        I.t[c] = d.type_slot[slot] * T;
        const int ni = (int)d.cl_bb[2 * (ci0 + c)].w;
        ivalid[c] = ((ni >= 8) ? 0xffull : ((1ull << ni) - 1ull)) * 0x0101010101010101ull;
        A.x[c] = A.y[c] = A.z[c] = A.q[c] = 0.f;
    }

    for (int e = it.e0; e < it.e0 + it.ne; ++e) {
        const NbEntry ent = d.entries[e];
        const uint32_t mask = (ent.meta >> 16) & 0xffu;
        float4* jp = d.jpart + (size_t)ent.jpos * kClusterSize;
        if (!mask) {
            if (ii == 0) jp[jj] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        const int code = ent.meta & 31u;
        const int nj = (int)(ent.meta >> 24);
        const uint64_t jvalid = (nj >= 8) ? ~0ull : ((1ull << (8 * nj)) - 1ull);
        const uint64_t* xrow =
            (ent.excl >= 0) ? d.excl_rows + (size_t)ent.excl * kClustersPerSc : nullptr;
        const int jslot = kClusterSize * ent.cj + jj;
        float4 xj = d.xq[jslot];
        const float4 gj = d.gslot[jslot];
        const int tj = d.type_slot[jslot];
        float ajx = 0.f, ajy = 0.f, ajz = 0.f, ajq = 0.f;
        if (code == kShiftZero) {
            entry_bwd<COUL, LJGRAD, PRIV, false>(I, A, mask, ivalid, jvalid, xrow, ent.cj, ci0,
                                                  code, xj, gj, tj, s_lj, s_hist, lane, kp, bs,
                                                  0.f, 0.f, 0.f, ajx, ajy, ajz, ajq);
        } else {
            const int sx = shift_x(code), sy = shift_y(code), sz = shift_z(code);
            if (sx < 0) xj.x -= S.L[0];
            if (sy < 0) xj.y -= S.L[1];
            if (sz < 0) xj.z -= S.L[2];
            entry_bwd<COUL, LJGRAD, PRIV, true>(I, A, mask, ivalid, jvalid, xrow, ent.cj, ci0,
                                                 code, xj, gj, tj, s_lj, s_hist, lane, kp, bs,
                                                 sx > 0 ? S.L[0] : 0.f, sy > 0 ? S.L[1] : 0.f,
                                                 sz > 0 ? S.L[2] : 0.f, ajx, ajy, ajz, ajq);
        }
        ajx = dpp_sum8(ajx);
        ajy = dpp_sum8(ajy);
        ajz = dpp_sum8(ajz);
        ajq = dpp_sum8(ajq);
        if (ii == 0) jp[jj] = make_float4(ajx, ajy, ajz, ajq);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
#pragma unroll
        for (int off = 8; off < kWave; off <<= 1) {
            A.x[c] += __shfl_xor(A.x[c], off);
            A.y[c] += __shfl_xor(A.y[c], off);
            A.z[c] += __shfl_xor(A.z[c], off);
            A.q[c] += __shfl_xor(A.q[c], off);
        }
    }
    if (jj == 0) {
        float4* ip = d.ipart + (size_t)item * kScAtoms;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            ip[kClusterSize * c + ii] = make_float4(A.x[c], A.y[c], A.z[c], A.q[c] * kp.epsfac_r);
    }
    if (LJGRAD) {
        __builtin_amdgcn_wave_barrier();
        float* out = d.glj_part + (size_t)item * 2 * TT;
        for (int k = lane; k < 2 * TT; k += kWave) {
            float v = 0.f;
            if (PRIV) {
                for (int l = 0; l < kWave; ++l) v += s_hist[k * kWave + l];
            } else {
                v = s_hist[k];
            }
            out[k] = v;
        }
    }
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

__global__ void k_reduce_bwd(NbDev d, float* __restrict__ gx, float* __restrict__ gq,
                             int accumulate, int n_slots) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n_slots) return;
    const int a = d.slot_atom[slot];
    if (a < 0) return;
    const int cj = slot / kClusterSize, jj = slot % kClusterSize;
    const int sc = slot / kScAtoms, loc = slot % kScAtoms;
    float s[4] = {0, 0, 0, 0}, cmp[4] = {0, 0, 0, 0};
    for (int k = d.jseg_start[cj]; k < d.jseg_start[cj + 1]; ++k) {
        const float4 v = d.jpart[(size_t)k * kClusterSize + jj];
        neumaier(s[0], cmp[0], v.x);
        neumaier(s[1], cmp[1], v.y);
        neumaier(s[2], cmp[2], v.z);
        neumaier(s[3], cmp[3], v.w);
    }
    const int i0 = d.sc_istart[sc], i1 = i0 + d.sc_icount[sc];
    for (int i = i0; i < i1; ++i) {
        const float4 v = d.ipart[(size_t)i * kScAtoms + loc];
        neumaier(s[0], cmp[0], v.x);
        neumaier(s[1], cmp[1], v.y);
        neumaier(s[2], cmp[2], v.z);
        neumaier(s[3], cmp[3], v.w);
    }
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

// Table gradient: FP64 sum over items, one thread per (type pair, c6/c12), fixed order.
// The table is symmetric, so the derivative with respect to the shared value of
// [t1][t2] and [t2][t1] is split evenly between the two entries (independent of which
// atom of a pair the kernel treats as i).
__global__ void k_reduce_glj(NbDev d, double* __restrict__ out, int n_types, int n_items,
                             int accumulate) {
    const int n_keys = 2 * n_types * n_types;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_keys) return;
    const int c = k & 1, t1 = (k >> 1) / n_types, t2 = (k >> 1) % n_types;
    const int kt = 2 * (t2 * n_types + t1) + c;
    double s = 0.0;
    for (int i = 0; i < n_items; ++i) {
        s += (double)d.glj_part[(size_t)i * n_keys + k];
        if (kt != k) s += (double)d.glj_part[(size_t)i * n_keys + kt];
    }
    if (kt != k) s *= 0.5;
    out[k] = accumulate ? out[k] + s : s;
}

inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

template <int COUL, bool LJG, bool PRIV>
void launch_bwd_t(const NbDev& d, const NbKParams& kp, const float* lj, const double* ge,
                  int n_items, hipStream_t s) {
    const int TT = kp.n_types * kp.n_types;
    const size_t hist = LJG ? (size_t)(PRIV ? 2 * TT * kWave : 2 * TT) * kBwdWaves : 0;
    const size_t lds = sizeof(float4) * TT + sizeof(float) * hist;
    hipLaunchKernelGGL((k_nb_bwd<COUL, LJG, PRIV>), dim3(blocks(n_items, kBwdWaves)),
                       dim3(kBwdThreads), lds, s, d, kp, lj, ge, n_items);
}

template <int COUL>
void launch_bwd_c(const NbDev& d, const NbKParams& kp, const float* lj, const double* ge,
                  bool ljgrad, int n_items, hipStream_t s) {
    if (!ljgrad) launch_bwd_t<COUL, false, false>(d, kp, lj, ge, n_items, s);
    else if (kp.n_types <= kPrivateHistTypes) launch_bwd_t<COUL, true, true>(d, kp, lj, ge, n_items, s);
    else launch_bwd_t<COUL, true, false>(d, kp, lj, ge, n_items, s);
}

}  // namespace

hipError_t launch_backward(const NbDev& d, const NbKParams& kp, int coulomb, const float* lj,
                           const float* grad_f, const double* grad_energy, bool ljgrad,
                           int n_slots, int n_items, hipStream_t s) {
    if (n_slots > 0)
        hipLaunchKernelGGL(k_gather_g, dim3(blocks(n_slots, 256)), dim3(256), 0, s, d, grad_f,
                           n_slots);
    if (n_items > 0) {
        if (coulomb == NB_COUL_RF) launch_bwd_c<NB_COUL_RF>(d, kp, lj, grad_energy, ljgrad, n_items, s);
        else launch_bwd_c<NB_COUL_EWALD>(d, kp, lj, grad_energy, ljgrad, n_items, s);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_backward(const NbDev& d, float* grad_x, float* grad_q, double* grad_lj,
                                  bool accumulate, int n_slots, int n_types, int n_items,
                                  hipStream_t s) {
    if (n_slots > 0 && (grad_x || grad_q))
        hipLaunchKernelGGL(k_reduce_bwd, dim3(blocks(n_slots, 256)), dim3(256), 0, s, d, grad_x,
                           grad_q, accumulate ? 1 : 0, n_slots);
    if (grad_lj) {
        const int nk = 2 * n_types * n_types;
        hipLaunchKernelGGL(k_reduce_glj, dim3(blocks(nk, 64)), dim3(64), 0, s, d, grad_lj,
                           n_types, n_items, accumulate ? 1 : 0);
    }
    return hipGetLastError();
}
