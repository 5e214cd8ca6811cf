// Grid build (Sec. V.A, Fig. 4): a grid regular in x and y whose z-columns are cut into
// cells of a fixed atom count; the 64-atom cells are split 2x2x2 into 8 clusters of 8
// atoms (super-clusters of near-cubic shape).  Everything here is integer work plus
// single-precision compares; the wrap and the column index are computed in a fixed
// single-precision sequence (no fused operations) so that the slot order is reproducible.
#include "nb_internal.h"

namespace {

constexpr int kScanThreads = 1024;

__device__ inline uint32_t sortable_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void k_fill(int32_t* __restrict__ p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_d(double* __restrict__ p, int n, double v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One thread per atom: single-precision wrap k = floor(x * invL), w = x - k * L, the
// column of w, and the per-column atom count.
__global__ void k_wrap_bin(int n, const float* __restrict__ x,
                           const int32_t* __restrict__ atom_sys, const NbSys* __restrict__ sys,
                           int4* __restrict__ img, float4* __restrict__ wpos,
                           int32_t* __restrict__ col_count, int32_t* __restrict__ flags,
                           int direct_count) {
#pragma clang fp contract(off)
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const NbSys S = sys[atom_sys[a]];
    int k[3];
    float w[3];
    bool bad = false;
    for (int dim = 0; dim < 3; ++dim) {
        float v = x[3 * a + dim];
        float kf = floorf(v * S.invL[dim]);
        // Non-finite or absurdly far coordinates are reported; the atom is placed at 0.
        if (!(fabsf(kf) <= 1048576.0f)) {
            bad = true;
            v = 0.0f;
            kf = 0.0f;
        }
        const float kl = kf * S.L[dim];
        w[dim] = v - kl;
        k[dim] = (int)kf;
    }
    if (bad) atomicOr(&flags[kFlagNonFinite], 1);
    int cx = (int)floorf(w[0] * S.cinv[0]);
    int cy = (int)floorf(w[1] * S.cinv[1]);
    cx = min(max(cx, 0), S.nx - 1);
    cy = min(max(cy, 0), S.ny - 1);
    const int col = S.col_base + cx * S.ny + cy;
    img[a] = make_int4(k[0], k[1], k[2], col);
    wpos[a] = make_float4(w[0], w[1], w[2], 0.0f);
    if (direct_count) atomicAdd(&col_count[col], 1);
}

// Column counts and bucketing with block-local LDS histograms: one global atomic per
// (block, column) instead of one per atom (columns are few and hot).
constexpr int kBinThreads = 256;
constexpr int kBinAtoms = 2048;        // atoms per block
constexpr int kBinMaxCols = 8192;      // LDS histogram limit (32 KB)

__global__ __launch_bounds__(kBinThreads) void k_count_cols(int n, int n_cols,
                                                             const int4* __restrict__ img,
                                                             int32_t* __restrict__ col_count) {
    extern __shared__ int s_h[];
    for (int c = threadIdx.x; c < n_cols; c += blockDim.x) s_h[c] = 0;
    __syncthreads();
    const int a0 = blockIdx.x * kBinAtoms, a1 = min(n, a0 + kBinAtoms);
    for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) atomicAdd(&s_h[img[a].w], 1);
    __syncthreads();
    for (int c = threadIdx.x; c < n_cols; c += blockDim.x)
        if (s_h[c]) atomicAdd(&col_count[c], s_h[c]);
}

__global__ __launch_bounds__(kBinThreads) void k_col_scatter_lds(
    int n, int n_cols, const int4* __restrict__ img, const int32_t* __restrict__ col_start,
    int32_t* __restrict__ col_cursor, int32_t* __restrict__ col_atoms) {
    extern __shared__ int s_h[];
    for (int c = threadIdx.x; c < n_cols; c += blockDim.x) s_h[c] = 0;
    __syncthreads();
    const int a0 = blockIdx.x * kBinAtoms, a1 = min(n, a0 + kBinAtoms);
    constexpr int kPer = kBinAtoms / kBinThreads;
    int rank[kPer], col[kPer];
    for (int k = 0; k < kPer; ++k) {
        const int a = a0 + threadIdx.x + k * kBinThreads;
        col[k] = (a < a1) ? img[a].w : -1;
        rank[k] = (a < a1) ? atomicAdd(&s_h[col[k]], 1) : 0;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n_cols; c += blockDim.x)
        if (s_h[c]) s_h[c] = atomicAdd(&col_cursor[c], s_h[c]);
    __syncthreads();
    for (int k = 0; k < kPer; ++k) {
        const int a = a0 + threadIdx.x + k * kBinThreads;
        if (a < a1) col_atoms[col_start[col[k]] + s_h[col[k]] + rank[k]] = a;
    }
}

// Exclusive scan by one block of kScanThreads threads: each thread scans a contiguous
// segment; segment totals are scanned in LDS.  f(i) gives element i.  Returns the total.
template <typename F>
__device__ int block_scan(int n, F f, int32_t* __restrict__ out) {
    __shared__ int s_part[kScanThreads];
    const int t = threadIdx.x;
    const int seg = (n + kScanThreads - 1) / kScanThreads;
    const int b = min(n, t * seg), e = min(n, b + seg);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += f(i);
    s_part[t] = sum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int v = (t >= off) ? s_part[t - off] : 0;
        __syncthreads();
        s_part[t] += v;
        __syncthreads();
    }
    int run = s_part[t] - sum;
    for (int i = b; i < e; ++i) {
        out[i] = run;
        run += f(i);
    }
    const int total = s_part[kScanThreads - 1];
    __syncthreads();
    if (t == 0) out[n] = total;
    return total;
}

// Column and super-cell offsets, per-super-cell info and per-system super-cell ranges.
__global__ __launch_bounds__(kScanThreads) void k_scan_cols(NbDev d) {
    const int nc = d.n_cols;
    block_scan(nc, [&](int i) { return d.col_count[i]; }, d.col_start);
    const int n_sc =
        block_scan(nc, [&](int i) { return (d.col_count[i] + kScAtoms - 1) / kScAtoms; },
                   d.col_sc_start);
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        d.col_cursor[c] = 0;
        int s = 0;
        while (s + 1 < d.n_sys && d.sys[s + 1].col_base <= c) ++s;   // few systems per col
        const int local = c - d.sys[s].col_base;
        const int ny = d.sys[s].ny;
        NbScInfo info;
        info.col = c;
        info.sys = s;
        info.cx = local / ny;
        info.cy = local % ny;
        for (int sc = d.col_sc_start[c]; sc < d.col_sc_start[c + 1]; ++sc) d.sc_info[sc] = info;
    }
    for (int s = threadIdx.x; s < d.n_sys; s += blockDim.x)
        d.sys_sc_start[s] = d.col_sc_start[d.sys[s].col_base];
    if (threadIdx.x == 0) {
        d.sys_sc_start[d.n_sys] = n_sc;
        d.flags[kFlagNumSc] = n_sc;
    }
}

__global__ void k_col_scatter(int n, const int4* __restrict__ img,
                              const int32_t* __restrict__ col_start,
                              int32_t* __restrict__ col_cursor, int32_t* __restrict__ col_atoms) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int col = img[a].w;
    const int pos = atomicAdd(&col_cursor[col], 1);
    col_atoms[col_start[col] + pos] = a;
}

// One block per column: order the column's atoms by (z, atom index).  The key
// (sortable z bits, index) is unique, so the order is fixed.  A column that fits in LDS is
// sorted there by a bitonic network over the next power of two (padded with all-ones keys,
// which no atom's key reaches, so the pads end up last); a larger one ranks each atom by
// counting the smaller keys in global memory.
constexpr int kSortThreads = 256;
constexpr int kSortLds = 4096;                   // keys of a column sorted in LDS (32 KB)

__global__ __launch_bounds__(kSortThreads) void k_col_sort(
    const int32_t* __restrict__ col_start, const int32_t* __restrict__ col_count,
    const int32_t* __restrict__ col_atoms, const float4* __restrict__ wpos,
    int32_t* __restrict__ col_sorted) {
    __shared__ unsigned long long s_key[kSortLds];
    const int c = blockIdx.x;
    const int base = col_start[c], n = col_count[c];
    auto key_of = [&](int i) -> unsigned long long {
        const int a = col_atoms[base + i];
        return ((unsigned long long)sortable_bits(wpos[a].z) << 32) | (unsigned)a;
    };
    if (n <= kSortLds) {
        int P = 1;
        while (P < n) P <<= 1;
        for (int i = threadIdx.x; i < P; i += blockDim.x) s_key[i] = (i < n) ? key_of(i) : ~0ull;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < P; i += blockDim.x) {
                    const int l = i ^ j;
                    if (l > i) {
                        const unsigned long long a = s_key[i], b = s_key[l];
                        if ((a > b) == ((i & k) == 0)) {
                            s_key[i] = b;
                            s_key[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            col_sorted[base + i] = (int)(s_key[i] & 0xffffffffu);
    } else {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const unsigned long long k = key_of(i);
            int r = 0;
            for (int j = 0; j < n; ++j) r += (key_of(j) < k) ? 1 : 0;
            col_sorted[base + r] = (int)(k & 0xffffffffu);
        }
    }
}

__device__ inline bool less_key(float va, int ia, float vb, int ib) {
    return va < vb || (va == vb && ia < ib);
}

// One wavefront per super-cell: 2x2x2 split into clusters, slot maps, types, build
// coordinates by slot, cluster and super-cluster bounding boxes.
__global__ __launch_bounds__(kWave) void k_supercell(NbDev d) {
    const int sc = blockIdx.x;
    if (sc >= d.flags[kFlagNumSc]) return;
    const int lane = threadIdx.x;
    __shared__ float s_x[kWave], s_y[kWave];
    __shared__ int s_a[kWave], s_yh[kWave], s_inv[kWave];
    const NbScInfo info = d.sc_info[sc];
    const int col = info.col;
    const int local = sc - d.col_sc_start[col];
    const int m = min(kScAtoms, d.col_count[col] - kScAtoms * local);
    const int a = (lane < m) ? d.col_sorted[d.col_start[col] + kScAtoms * local + lane] : -1;
    const float4 w = (a >= 0) ? d.wpos[a] : make_float4(0.f, 0.f, 0.f, 0.f);
    s_x[lane] = w.x;
    s_y[lane] = w.y;
    s_a[lane] = a;
    s_inv[lane] = -1;
    __syncthreads();
    const int zh = lane >= 32 ? 1 : 0;
    const int h0 = zh * 32, h1 = min(m, h0 + 32);
    int yh = 0, loc = -1;
    if (a >= 0) {
        int ry = 0;
        for (int k = h0; k < h1; ++k) ry += less_key(s_y[k], s_a[k], w.y, a) ? 1 : 0;
        yh = ry >= 16 ? 1 : 0;
    }
    s_yh[lane] = yh;
    __syncthreads();
    if (a >= 0) {
        int rx = 0;
        for (int k = h0; k < h1; ++k)
            rx += (s_yh[k] == yh && less_key(s_x[k], s_a[k], w.x, a)) ? 1 : 0;
        const int xh = rx >= 8 ? 1 : 0;
        loc = (zh * 4 + yh * 2 + xh) * kClusterSize + (rx - 8 * xh);
        s_inv[loc] = lane;
    }
    __syncthreads();
    const int src = s_inv[lane];
    const int atom = (src >= 0) ? s_a[src] : -1;
    const int slot = sc * kScAtoms + lane;
    d.slot_atom[slot] = atom;
    d.type_slot[slot] = (atom >= 0) ? d.type[atom] * (int)sizeof(float4) : 0;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (atom >= 0) {
        d.atom_slot[atom] = slot;
        p = d.wpos[atom];
    }
    d.xw[slot] = p;
    const float inf = __builtin_inff();
    float lo[3] = {atom >= 0 ? p.x : inf, atom >= 0 ? p.y : inf, atom >= 0 ? p.z : inf};
    float hi[3] = {atom >= 0 ? p.x : -inf, atom >= 0 ? p.y : -inf, atom >= 0 ? p.z : -inf};
    int cnt = atom >= 0 ? 1 : 0;
    for (int off = 1; off < kClusterSize; off <<= 1) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
        }
        cnt += __shfl_xor(cnt, off);
    }
    if ((lane & 7) == 0) {
        const int c = sc * kClustersPerSc + (lane >> 3);
        d.cl_bb[2 * c] = make_float4(lo[0], lo[1], lo[2], (float)cnt);
        d.cl_bb[2 * c + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
    }
    for (int off = kClusterSize; off < kWave; off <<= 1) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
        }
        cnt += __shfl_xor(cnt, off);
    }
    if (lane == 0) {
        d.sc_bb[2 * sc] = make_float4(lo[0], lo[1], lo[2], (float)cnt);
        d.sc_bb[2 * sc + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
    }
}

// Excluded partner slots per slot (-1 padded), from the atom-level CSR list.
__global__ void k_excl_slots(NbDev d) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= d.flags[kFlagNumSc] * kScAtoms) return;
    const int a = d.slot_atom[slot];
    const int b0 = (a >= 0) ? d.excl_ptr[a] : 0;
    const int len = (a >= 0) ? d.excl_ptr[a + 1] - b0 : 0;
    for (int k = 0; k < d.max_excl; ++k) {
        const int partner = (k < len) ? d.excl_idx[b0 + k] : -1;
        d.excl_slot[(size_t)slot * d.max_excl + k] = (partner >= 0) ? d.atom_slot[partner] : -1;
    }
}

// Per cluster, the range of clusters that hold the excluded partners of its atoms
// ((2^31 - 1, -1) when none): the list's exclusion pass looks at the partners of an entry's
// i-cluster only when the j-cluster falls in that range.
__global__ void k_excl_cluster_range(NbDev d) {
    const int ci = blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= d.flags[kFlagNumSc] * kClustersPerSc) return;
    int lo = 0x7fffffff, hi = -1;
    for (int ii = 0; ii < kClusterSize; ++ii) {
        const int slot = kClusterSize * ci + ii;
        for (int k = 0; k < d.max_excl; ++k) {
            const int ps = d.excl_slot[(size_t)slot * d.max_excl + k];
            if (ps >= 0) {
                lo = min(lo, ps / kClusterSize);
                hi = max(hi, ps / kClusterSize);
            }
        }
    }
    d.cl_xrange[ci] = make_int2(lo, hi);
}

// Per slot: the image offset of its atom, (kx Lx, ky Ly, kz Lz) in FP32 as the gather
// subtracts it, or, for an empty slot, its filler position.  Empty slots (charge 0) sit on
// the lattice -D (1 + i, 1 + j, 1 + k) with spacing D = max box edge + 2 rlist + 1 nm and
// (i, j, k) the slot's base-1024 digits.  Any pair with an empty slot is then at least
// 2 rlist + 1 nm apart on some axis under every periodic shift s L (|s| <= 1), and an empty
// slot and its own image |s L| apart: with box edges up to 1000 nm the coordinates stay
// below 1025 D < 1.1e6 nm, where one ulp is at most 0.125 nm.  No distance test with an
// empty slot passes, so the pair kernels need no valid-atom masks.
__global__ void k_slot_pre(NbDev d, int n_slots) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    // slots of the super-clusters of this grid (k_supercell writes no others)
    if (slot >= n_slots || slot >= d.flags[kFlagNumSc] * kScAtoms) return;
    const int a = d.slot_atom[slot];
    const float D = d.filler_d;
    float4 v = make_float4(-D * (float)(1 + (slot & 1023)), -D * (float)(1 + ((slot >> 10) & 1023)),
                           -D * (float)(1 + (slot >> 20)), 0.f);
    if (a >= 0) {
        const int4 k = d.img[a];
        const NbSys S = d.sys[d.atom_sys[a]];
        v = make_float4((float)k.x * S.L[0], (float)k.y * S.L[1], (float)k.z * S.L[2], 0.f);
    }
    d.slot_pre[slot] = v;
}

inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t launch_grid_build(const NbDev& d, const float* x, hipStream_t s) {
    const int n = d.n_atoms;
    if (d.n_cols > 0)
        hipLaunchKernelGGL(k_fill, dim3(blocks(d.n_cols, 256)), dim3(256), 0, s, d.col_count,
                           d.n_cols, 0);
    const bool lds_bins = d.n_cols <= kBinMaxCols;
    const size_t lds = sizeof(int) * (size_t)d.n_cols;
    if (n > 0) {
        hipLaunchKernelGGL(k_wrap_bin, dim3(blocks(n, 256)), dim3(256), 0, s, n, x, d.atom_sys,
                           d.sys, d.img, d.wpos, d.col_count, d.flags, lds_bins ? 0 : 1);
        if (lds_bins)
            hipLaunchKernelGGL(k_count_cols, dim3(blocks(n, kBinAtoms)), dim3(kBinThreads), lds, s,
                               n, d.n_cols, d.img, d.col_count);
    }
    hipLaunchKernelGGL(k_scan_cols, dim3(1), dim3(kScanThreads), 0, s, d);
    if (n > 0) {
        if (lds_bins)
            hipLaunchKernelGGL(k_col_scatter_lds, dim3(blocks(n, kBinAtoms)), dim3(kBinThreads),
                               lds, s, n, d.n_cols, d.img, d.col_start, d.col_cursor,
                               d.col_atoms);
        else
            hipLaunchKernelGGL(k_col_scatter, dim3(blocks(n, 256)), dim3(256), 0, s, n, d.img,
                               d.col_start, d.col_cursor, d.col_atoms);
        hipLaunchKernelGGL(k_col_sort, dim3(d.n_cols), dim3(kSortThreads), 0, s, d.col_start,
                           d.col_count, d.col_atoms, d.wpos, d.col_sorted);
    }
    if (d.n_sc_max > 0) {
        hipLaunchKernelGGL(k_supercell, dim3(d.n_sc_max), dim3(kWave), 0, s, d);
        hipLaunchKernelGGL(k_excl_slots, dim3(blocks((int64_t)d.n_sc_max * kScAtoms, 256)),
                           dim3(256), 0, s, d);
        hipLaunchKernelGGL(k_excl_cluster_range,
                           dim3(blocks((int64_t)d.n_sc_max * kClustersPerSc, 256)), dim3(256), 0,
                           s, d);
        hipLaunchKernelGGL(k_slot_pre, dim3(blocks((int64_t)d.n_sc_max * kScAtoms, 256)),
                           dim3(256), 0, s, d, (int)(d.n_sc_max * kScAtoms));
    }
    return hipGetLastError();
}

hipError_t launch_fill(int32_t* p, int n, int32_t v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(blocks(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_d(double* p, int n, double v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_d, dim3(blocks(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
