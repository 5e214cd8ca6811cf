// Per-step gather of coordinates into slot order and the reductions after the pair
// kernel: per atom, the j-partials of the entries that reference its cluster
// (consecutive by construction) and the i-partials of its super-cluster's items, added
// with compensated (Neumaier) single-precision sums and written in the caller's atom
// order; energies, virial and pair counts per system in double precision.
#include "nb_chunk_sums.h"
#include "nb_internal.h"
#include "nb_prune_item.h"

namespace {

// Per-slot gather of user-order coordinates (and charges) into slot order, wrapped with
// the image offsets of the last grid build (kept per slot in slot_pre, the same FP32
// products the build formed, so that the loads a slot waits for are two deep: its atom
// index and offset, then the atom's coordinates).  An empty slot takes its filler
// position from slot_pre and charge 0.
__global__ void k_gather(NbDev d, const float* __restrict__ x, const float* __restrict__ q,
                         float4* __restrict__ out, int n_slots) {
#pragma clang fp contract(off)
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n_slots) return;
    const int a = d.slot_atom[slot];
    const float4 p = d.slot_pre[slot];
    float4 v = p;
    if (a >= 0) {
        v.x = x[3 * a] - p.x;
        v.y = x[3 * a + 1] - p.y;
        v.z = x[3 * a + 2] - p.z;
        v.w = q ? q[a] : 0.f;
    }
    out[slot] = v;
}

__device__ inline void neumaier(float& s, float& c, float v) {
    const float t = s + v;
    c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
}

// One wavefront per super-cluster, lane = slot within it (cluster c = l >> 3, atom jj = l &
// 7): each lane sums, with compensation, the j-partials of the entries referencing its
// cluster (a contiguous segment, in entry order) and then the i-partials of the
// super-cluster's items (in item order; one 1 KB row per item, read by the whole wavefront),
// then its exclusion correction, and writes its atom's force in the caller's order.  No
// lanes are combined, so there is no cross-lane traffic, and the order of every sum is
// fixed.  (Four wavefronts per super-cluster, each summing a quarter of every segment and
// combined through LDS, measured no faster.)
constexpr int kRedWaves = 4;
__device__ __forceinline__ void reduce_sc(
    const int sc, const int32_t* __restrict__ slot_atom, const int32_t* __restrict__ jseg_start,
    const float4* __restrict__ jpart, const int32_t* __restrict__ sc_istart,
    const int32_t* __restrict__ sc_icount, const float4* __restrict__ ipart,
    const float4* __restrict__ xcf, float* __restrict__ f, int accumulate) {
    const int lane = threadIdx.x & (kWave - 1);
    const int jj = lane & 7;
    const int cj = sc * kClustersPerSc + (lane >> 3);
    const int slot = sc * kScAtoms + lane;
    const int s0 = jseg_start[cj], s1 = jseg_start[cj + 1];
    const int i0 = sc_istart[sc], i1 = i0 + sc_icount[sc];
    float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
#pragma unroll 4
    for (int k = s0; k < s1; ++k) {
        const float4 v = jpart[(size_t)k * kClusterSize + jj];
        neumaier(sx, cx, v.x);
        neumaier(sy, cy, v.y);
        neumaier(sz, cz, v.z);
    }
#pragma unroll 2
    for (int i = i0; i < i1; ++i) {
        const float4 v = ipart[(size_t)i * kScAtoms + lane];
        neumaier(sx, cx, v.x);
        neumaier(sy, cy, v.y);
        neumaier(sz, cz, v.z);
    }
    if (xcf) {                          // exclusion corrections of this atom, if any
        const float4 v = xcf[slot];
        neumaier(sx, cx, v.x);
        neumaier(sy, cy, v.y);
        neumaier(sz, cz, v.z);
    }
    const int a = slot_atom[slot];
    if (a < 0) return;
    float rx = sx + cx, ry = sy + cy, rz = sz + cz;
    if (accumulate) {
        rx += f[3 * a];
        ry += f[3 * a + 1];
        rz += f[3 * a + 2];
    }
    f[3 * a] = rx;
    f[3 * a + 1] = ry;
    f[3 * a + 2] = rz;
}

// Per-system totals from the chunk partials, in chunk order: thread t of the block takes
// the (system, value) pairs t, t + blockDim.x, ...  Values: E_LJ, E_C, the six virial
// sums xx yy zz xy xz yz, pair count, raw pair count.
__device__ inline void energy_totals(const NbDev& d, double* __restrict__ energy,
                                     double* __restrict__ virial, uint32_t flags, int n_sys) {
    const bool accum = flags & NB_F_ACCUMULATE;
    for (int idx = threadIdx.x; idx < n_sys * kEpartStride; idx += blockDim.x) {
        const int sys = idx / kEpartStride, k = idx % kEpartStride;
        const int c0 = d.sys_chunk_start[sys], c1 = d.sys_chunk_start[sys + 1];
        double t = 0.0;
        for (int c = c0; c < c1; ++c) t += d.cpart[(size_t)c * kChunkVals + k];
        if (k < 2) {
            if ((flags & NB_F_ENERGY) && energy)
                energy[2 * sys + k] = (accum ? energy[2 * sys + k] : 0.0) + t;
        } else if (k < 8) {
            // Xi = -1/2 sum d (x) f, symmetric; value k lands at these row-major positions
            if ((flags & NB_F_VIRIAL) && virial) {
                constexpr int q1[6] = {0, 4, 8, 1, 2, 5}, q2[6] = {-1, -1, -1, 3, 6, 7};
                double* v = virial + 9 * sys;
                v[q1[k - 2]] = (accum ? v[q1[k - 2]] : 0.0) - 0.5 * t;
                if (q2[k - 2] >= 0) v[q2[k - 2]] = (accum ? v[q2[k - 2]] : 0.0) - 0.5 * t;
            }
        } else {
            d.dstat[2 * sys + (k - 8)] = t;
        }
    }
}

// The ahead rolling prune, the force reduction and the energy reduction in one launch:
// blocks [0, n_pblk) prune the lists of the next step's rolling part (prune_item, four
// wavefronts per unit; the reductions read no list data, so the two run side by side), blocks [n_pblk, n_pblk + n_fblk) reduce the forces of four super-clusters
// each (one wavefront per super-cluster), the blocks after them sum one energy chunk each;
// the last energy block to finish (a ticket in queue[2], taken after a device-scope
// fence) adds the chunk partials per system and resets the ticket for the next launch.
__global__ __launch_bounds__(kRedThreads) void k_reduce_step(NbDev d, float* __restrict__ f,
                                                             int accumulate, int n_sc,
                                                             int n_fblk, double* energy,
                                                             double* virial, uint32_t flags,
                                                             int n_sys,
                                                             const float4* __restrict__ xcf,
                                                             int n_pblk, int prune_part,
                                                             int nstprune, int item0,
                                                             int n_units, int q,
                                                             float r2_inner) {
    static_assert(kRedThreads == kRedWaves * kWave, "one block shape for all parts");
    if ((int)blockIdx.x < n_pblk) {
        // Units u = blockIdx.x, + n_pblk, ... of the part.  q == 0: unit u is the pair
        // kernel's item part_items[item0 + u] (one or two per block).  q == 1: unit u is
        // the whole list of super-cluster
        // prune_part + u nstprune, in runs of at most 64 entries per wavefront (a device
        // already full of reduction blocks: fewer, longer prune blocks stage fewer i-atoms).
        __shared__ float4 s_xi[kScAtoms];
        bool first = true;
        for (int u = blockIdx.x; u < n_units; u += n_pblk) {
            NbItem it;
            if (q == 0) {
                it = d.items[d.part_items[item0 + u]];
            } else {
                it.sc = prune_part + u * nstprune;
                it.e0 = d.sc_estart[it.sc];
                it.ne = d.sc_ecount[it.sc];
                it.pos = 0;
            }
            const int e_end = it.e0 + it.ne;
            for (int e0 = it.e0; e0 < e_end; e0 += kRedWaves * kWave) {   // one call site
                if (!first) __syncthreads();               // s_xi of the previous run read
                first = false;
                NbItem run = it;
                run.e0 = e0;
                run.ne = min(kRedWaves * kWave, e_end - e0);
                prune_item<kRedWaves>(run, d.entries, d.xq, d.sc_info, d.sys, r2_inner, s_xi);
            }
        }
        return;
    }
    const int b = (int)blockIdx.x - n_pblk;
    if (b >= n_fblk) {
        const int c = b - n_fblk;
        const int4 ch = d.chunks[c];
        chunk_sums(d.epart, d.epart_stride, kEpartStride, ch.y, ch.z,
                   d.cpart + (size_t)c * kChunkVals);
        // One release fence per block, by the thread that takes the ticket: the barrier
        // orders the block's partial stores before it.  (A device-scope fence writes the
        // XCD's L2 back; one per wavefront cost about 2 us per launch at 96k atoms.)
        __shared__ int s_last;
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            s_last = (atomicAdd(d.queue + 2, 1) == d.n_chunks - 1);
        }
        __syncthreads();
        if (s_last) {
            // every other block's partials, released before their tickets
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            energy_totals(d, energy, virial, flags, n_sys);
            if (threadIdx.x == 0) atomicExch(d.queue + 2, 0);
        }
        return;
    }
    const int sc = b * kRedWaves + (int)(threadIdx.x / kWave);
    if (sc >= n_sc) return;
    reduce_sc(sc, d.slot_atom, d.jseg_start, d.jpart, d.sc_istart, d.sc_icount, d.ipart, xcf,
              f, accumulate);
}

// Per-system totals when there is no chunk to reduce (no work items).
__global__ void k_energy_final(NbDev d, double* __restrict__ energy, double* __restrict__ virial,
                               uint32_t flags, int n_sys) {
    energy_totals(d, energy, virial, flags, n_sys);
}

inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t launch_gather(const NbDev& d, const float* x, const float* q, float4* out,
                         int n_slots, hipStream_t s) {
    if (n_slots > 0)
        hipLaunchKernelGGL(k_gather, dim3(blocks(n_slots, 256)), dim3(256), 0, s, d, x, q, out,
                           n_slots);
    return hipGetLastError();
}

// Resident blocks per CU of k_reduce_step (queried once).
static int red_blocks_per_cu() {
    static int per_cu = 0;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_reduce_step, kRedThreads, 0) !=
            hipSuccess)
            nb = 0;
        per_cu = nb > 0 ? nb : 1;
    }
    return per_cu;
}

hipError_t launch_reduce(const NbDev& d, float* f, bool accumulate, int n_slots,
                        double* energy, double* virial, uint32_t flags, int n_sys,
                        const float4* xcf, int prune_part, int nstprune, int item0,
                        int n_part_items, float r2_inner, hipStream_t s) {
    const int n_sc = n_slots / kScAtoms;
    const int n_fblk = blocks(n_sc, kRedWaves);
    const bool ev = (flags & (NB_F_ENERGY | NB_F_VIRIAL)) && n_sys > 0;
    const int n_eblk = ev ? d.n_chunks : 0;
    // Prune units: the pair kernel's items of the part, one per block while they fit the
    // device beside the reduction's blocks (a second round of a few blocks cost 2.5 us at
    // 96k atoms; up to twice as many items take two per block); on a device already full
    // of reduction blocks whole super-cluster lists, several per block (1.5M atoms: 129 us
    // for the launch against 164 with items four per block and 140 with lists in
    // quarters; whole lists at 96k: 25 us, too few blocks for the latency of each).
    int q = 0, n_units = 0, n_pblk = 0;
    if (prune_part >= 0 && n_part_items > 0) {
        const int resident = red_blocks_per_cu() * std::max(d.n_cu, 1);
        const int avail = resident - n_fblk - n_eblk;
        if (2 * avail >= n_part_items) {
            n_units = n_part_items;
            n_pblk = std::min(n_units, avail);
        } else {
            q = 1;
            n_units = (n_sc > prune_part) ? (n_sc - prune_part + nstprune - 1) / nstprune : 0;
            n_pblk = std::min(n_units, std::max(avail, (n_units + 3) / 4));
        }
    }
    if (n_pblk + n_fblk + n_eblk > 0)
        hipLaunchKernelGGL(k_reduce_step, dim3(n_pblk + n_fblk + n_eblk), dim3(kRedThreads), 0,
                           s, d, f, accumulate ? 1 : 0, n_sc, n_fblk, energy, virial, flags,
                           n_sys, xcf, n_pblk, prune_part, nstprune, item0, n_units, q,
                           r2_inner);
    if (ev && n_eblk == 0)
        hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kRedThreads), 0, s, d, energy, virial,
                           flags, n_sys);
    return hipGetLastError();
}
