// Electrostatic corrections of excluded atom pairs inside the cut-off and of each atom with
// itself (nb_forces flag NB_F_EXCL_CORR), for runs whose long-range part counts every pair
// of charges (Sec. V.A: for PME runs the real-space Ewald correction is computed with the
// pair kernel; force-field exclusions are enforced together with the cut-off):
//   Ewald  V = -K q_a q_b erf(beta r)/r,      phi = K q_a q_b (2 beta/sqrt(pi) e^{-beta^2 r^2}
//                                                    - erf(beta r)/r) / r^2,
//          self -K q_a^2 beta/sqrt(pi);
//   RF     V = K q_a q_b (k_rf r^2 - c_rf),   phi = -2 K q_a q_b k_rf,   self -K q_a^2 c_rf / 2;
// K = epsfac / eps_r, force on a = phi (x_a - x_b).  Excluded pairs are about 3 % of the
// pairs in a water box and never go through the pair kernel, whose timing stays as it is:
// one wavefront per super-cluster takes its 64 slots, each lane its atom's excluded
// partners (slot table of the grid build), in double precision (a few hundred thousand
// pairs at most, so the cost is small, and the corrections, which nearly cancel the self
// terms for neutral molecules, carry no single-precision rounding).  Each lane keeps its
// own atom's force (each pair is evaluated from both sides; no atomics) for the force
// reduction to add; energies and virial are summed per super-cluster and then per system
// in a fixed order.
#include "nb_internal.h"

namespace {

constexpr int kXcWaves = 4;

__device__ inline double wave_sum(double v) {
    for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

template <int COUL>
__global__ __launch_bounds__(kXcWaves * kWave) void k_excl_corr(NbDev d, NbKParams kp,
                                                                 double crf, double krf,
                                                                 int n_sc, float4* __restrict__ xcf,
                                                                 double* __restrict__ xce) {
    const int sc = blockIdx.x * kXcWaves + (int)(threadIdx.x / kWave);
    if (sc >= n_sc) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int slot = sc * kScAtoms + lane;
    const int a = d.slot_atom[slot];
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (a >= 0) {
        const float4 xa = d.xq[slot];
        const NbSys S = d.sys[d.sc_info[sc].sys];
        const double K = (double)kp.epsfac_r, beta = (double)kp.beta;
        const double rc2 = (double)kp.rc2;
        const double qa = (double)xa.w;
        for (int k = 0; k < d.max_excl; ++k) {
            const int ps = d.excl_slot[(size_t)slot * d.max_excl + k];
            if (ps < 0 || ps == slot) continue;
            const float4 xb = d.xq[ps];
            double dd[3] = {(double)xa.x - (double)xb.x, (double)xa.y - (double)xb.y,
                            (double)xa.z - (double)xb.z};
            for (int m = 0; m < 3; ++m) dd[m] -= (double)S.L[m] * rint(dd[m] / (double)S.L[m]);
            const double r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
            if (!(r2 < rc2)) continue;
            const double kq = K * qa * (double)xb.w;
            double ve, phi;
            if (COUL == NB_COUL_RF) {
                ve = kq * (krf * r2 - crf);
                phi = -2.0 * kq * krf;
            } else if (r2 > 0.0) {
                const double r = sqrt(r2);
                const double ef = erf(beta * r);
                ve = -kq * ef / r;
                phi = kq * (2.0 * beta / sqrt(M_PI) * exp(-beta * beta * r2) - ef / r) / r2;
            } else {
                ve = -kq * 2.0 * beta / sqrt(M_PI);
                phi = -kq * 4.0 * beta * beta * beta / (3.0 * sqrt(M_PI));
            }
            fx += phi * dd[0];
            fy += phi * dd[1];
            fz += phi * dd[2];
            e += 0.5 * ve;                       // each pair is seen from both atoms
            v[0] += 0.5 * phi * dd[0] * dd[0];
            v[1] += 0.5 * phi * dd[1] * dd[1];
            v[2] += 0.5 * phi * dd[2] * dd[2];
            v[3] += 0.5 * phi * dd[0] * dd[1];
            v[4] += 0.5 * phi * dd[0] * dd[2];
            v[5] += 0.5 * phi * dd[1] * dd[2];
        }
        const double kqa = K * qa * qa;
        e += (COUL == NB_COUL_RF) ? -0.5 * kqa * crf : -kqa * beta / sqrt(M_PI);
    }
    xcf[slot] = make_float4((float)fx, (float)fy, (float)fz, 0.f);
    e = wave_sum(e);
    for (int m = 0; m < 6; ++m) v[m] = wave_sum(v[m]);
    if (lane == 0) {
        const size_t st = (size_t)d.n_sc_max;
        xce[sc] = e;
        for (int m = 0; m < 6; ++m) xce[(size_t)(1 + m) * st + sc] = v[m];
    }
}

// Per system (one block each): the super-cluster partials in order, added to the energies
// and the virial the force reduction wrote (Xi = -1/2 sum d (x) phi d).
__global__ __launch_bounds__(256) void k_excl_energy(NbDev d, const double* __restrict__ xce,
                                                      double* __restrict__ energy,
                                                      double* __restrict__ virial,
                                                      uint32_t flags) {
    const int sys = blockIdx.x;
    const int s0 = d.sys_sc_start[sys], s1 = d.sys_sc_start[sys + 1];
    __shared__ double s_w[4][7];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const size_t st = (size_t)d.n_sc_max;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int sc = s0 + threadIdx.x; sc < s1; sc += blockDim.x)
        for (int m = 0; m < 7; ++m) acc[m] += xce[(size_t)m * st + sc];
    for (int m = 0; m < 7; ++m) {
        acc[m] = wave_sum(acc[m]);
        if (lane == 0) s_w[wv][m] = acc[m];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[7];
        for (int m = 0; m < 7; ++m) t[m] = s_w[0][m] + s_w[1][m] + s_w[2][m] + s_w[3][m];
        if ((flags & NB_F_ENERGY) && energy) energy[2 * sys + 1] += t[0];
        if ((flags & NB_F_VIRIAL) && virial) {
            constexpr int q1[6] = {0, 4, 8, 1, 2, 5}, q2[6] = {-1, -1, -1, 3, 6, 7};
            double* vv = virial + 9 * sys;
            for (int m = 0; m < 6; ++m) {
                vv[q1[m]] += -0.5 * t[1 + m];
                if (q2[m] >= 0) vv[q2[m]] += -0.5 * t[1 + m];
            }
        }
    }
}

}  // namespace

hipError_t launch_excl_corr(const NbDev& d, const NbKParams& kp, int coulomb, double krf,
                            double crf, int n_sc, float4* xcf, double* xce, hipStream_t s) {
    if (n_sc <= 0) return hipGetLastError();
    const dim3 grid((n_sc + kXcWaves - 1) / kXcWaves), block(kXcWaves * kWave);
    if (coulomb == NB_COUL_RF)
        hipLaunchKernelGGL(k_excl_corr<NB_COUL_RF>, grid, block, 0, s, d, kp, crf, krf, n_sc, xcf,
                           xce);
    else
        hipLaunchKernelGGL(k_excl_corr<NB_COUL_EWALD>, grid, block, 0, s, d, kp, crf, krf, n_sc,
                           xcf, xce);
    return hipGetLastError();
}

hipError_t launch_excl_energy(const NbDev& d, const double* xce, double* energy, double* virial,
                              uint32_t flags, int n_sys, hipStream_t s) {
    if (n_sys > 0 && (flags & (NB_F_ENERGY | NB_F_VIRIAL)))
        hipLaunchKernelGGL(k_excl_energy, dim3(n_sys), dim3(256), 0, s, d, xce, energy, virial,
                           flags);
    return hipGetLastError();
}
