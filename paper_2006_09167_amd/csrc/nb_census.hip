// Work-efficiency census of the outer list (Sec. V.B, Fig. 5; cluster setups of Sec. V.A
// and V.D).
//
// For each radius R_k (at most the list radius) and each sub-cluster setup M x N with M, N
// in {1, 2, 4, 8} (i-sub-clusters of M consecutive slots of an 8-atom cluster, j-sub-
// clusters of N), count the pairs of sub-clusters holding an atom pair closer than R_k.
// 1 x 1 counts the atom pairs themselves, 8 x 8 the cluster pairs.  Every sub-cluster pair
// within the list radius lies in an outer-list cluster pair, so walking the outer list at
// its build positions counts them all, with the list arithmetic (shift split between the
// two sides, no contraction) and therefore exactly.
//
// * k_census: one wavefront per work item (the item's eight i-clusters loaded once).  Per
//   cluster pair every lane takes the bin of its squared distance, the number of sorted
//   thresholds R_k^2 at or below it (a two-level count: chunk pivots, then one chunk); a
//   sub-cluster pair holds a pair closer than R_k iff the smallest bin of its lanes is <= k,
//   so folding the lane bins with min over lane-xor partners (1, 2, 4 on the i side, 8, 16,
//   32 on the j side; DPP where the partner is in the same row of 16 lanes) gives each
//   sub-cluster pair's bin, which its first lane adds to an LDS histogram per setup.  Each
//   block then writes its histogram.
// * the same walk with COVER: per lane, the bin k of its own distance and the bin l of its
//   sub-cluster pair of one chosen setup; a K x K histogram over (l, k) gives, after prefix
//   sums, the atom pairs closer than R_k that lie in a sub-cluster pair held at R_l (the
//   implicit buffer of a list at R_l, used by the Verlet buffer estimate).
// * k_census_sum / k_census_total: the block histograms summed in 64-bit (chunks of blocks,
//   then the chunks); the host turns bins into counts by prefix sums.
#include <algorithm>
#include <cfloat>
#include <mutex>

#include "nb_internal.h"
#include "nb_pair_common.h"

namespace {

constexpr int kCensusWaves = 8;
constexpr int kCensusMaxBlocks = 16384;        // beyond, blocks stride over the items
constexpr int kCoverMaxBlocks = 2048;          // coverage histograms are 16 KB per block
constexpr int kCensusSetups = 16;               // (log2 M) * 4 + log2 N
constexpr int kCensusBins = NB_CENSUS_MAX_RADII;
constexpr int kHistWords = kCensusSetups * kCensusBins;     // census histogram words
constexpr int kCoverWords = kCensusBins * kCensusBins;      // coverage histogram words

#define NB_FOR8(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

// Number of thresholds at or below v (v finite), for NCH chunks of 8 ascending thresholds
// padded with +inf.  Two levels: the last threshold of each chunk (pivots, wave-uniform, in
// scalar registers) gives the chunk g holding v's place, since every threshold of the
// chunks before g is at or below its pivot <= v and every one after is at or above a pivot
// > v; then the first seven thresholds of chunk g, read from LDS (two 16-byte reads; the
// table carries one more chunk of +inf for g = NCH), finish the count.  For finite floats
// v - t is +0 when v == t and keeps the sign of the exact difference, so t <= v iff the sign
// bit of v - t is clear: each comparison costs a subtraction, a shift and an add.
__device__ inline int below(float v, float t) { return (int)(__float_as_uint(v - t) >> 31); }

template <int NCH>
__device__ inline int bin_of(const float* piv, const float* s_thr, float v) {
    int neg = 0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) neg += below(v, piv[c]);
    const int g = NCH - neg;
    const float4 a = *reinterpret_cast<const float4*>(s_thr + 8 * g);
    const float4 b = *reinterpret_cast<const float4*>(s_thr + 8 * g + 4);
    const int m = below(v, a.x) + below(v, a.y) + below(v, a.z) + below(v, a.w) +
                  below(v, b.x) + below(v, b.y) + below(v, b.z);
    return 8 * g + 7 - m;
}

// min(v, v of the lane whose index differs in the given bit): DPP inside a row of 16 lanes
// (xor 1, 2 as quad permutations; xor 4 as the half-row mirror, which pairs each lane with
// one in the other quad: equal to xor 4 once quads hold equal values; xor 8 as a rotation
// by 8), a swizzle for xor 16 and a permute across the halves for xor 32.
template <int BIT>
__device__ inline int fold_min(int v, int lane) {
    int p;
    if constexpr (BIT == 1) p = __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false);
    else if constexpr (BIT == 2) p = __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false);
    else if constexpr (BIT == 4) p = __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
    else if constexpr (BIT == 8) p = __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false);
    else if constexpr (BIT == 16) p = __builtin_amdgcn_ds_swizzle(v, 0x401f);
    else p = __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
    return min(v, p);
}

// Histogram one 8x8 cluster pair given each lane's bin (n_radii: not inside any radius).
template <int A>
__device__ inline void census_jfold(uint32_t* hist, int bi, int lane, int n_radii) {
    const int ii = lane & 7, jj = lane >> 3;
    const bool ilead = (ii & ((1 << A) - 1)) == 0;
    int b2 = bi;
    if (ilead && b2 < n_radii) atomicAdd(&hist[(4 * A + 0) * kCensusBins + b2], 1u);
    b2 = fold_min<8>(b2, lane);
    if (ilead && (jj & 1) == 0 && b2 < n_radii)
        atomicAdd(&hist[(4 * A + 1) * kCensusBins + b2], 1u);
    b2 = fold_min<16>(b2, lane);
    if (ilead && (jj & 3) == 0 && b2 < n_radii)
        atomicAdd(&hist[(4 * A + 2) * kCensusBins + b2], 1u);
    b2 = fold_min<32>(b2, lane);
    if (ilead && jj == 0 && b2 < n_radii) atomicAdd(&hist[(4 * A + 3) * kCensusBins + b2], 1u);
}

__device__ inline void census_block(uint32_t* hist, int bin, int lane, int n_radii) {
    if (!__builtin_amdgcn_ballot_w64(bin < n_radii)) return;
    census_jfold<0>(hist, bin, lane, n_radii);
    int bi = fold_min<1>(bin, lane);
    census_jfold<1>(hist, bi, lane, n_radii);
    bi = fold_min<2>(bi, lane);
    census_jfold<2>(hist, bi, lane, n_radii);
    bi = fold_min<4>(bi, lane);
    census_jfold<3>(hist, bi, lane, n_radii);
}

// Coverage of one 8x8 cluster pair for the setup of 2^ca x 2^cb sub-clusters: each lane
// with bin k < n_radii adds one to [l][k], l the bin of its sub-cluster pair (the smallest
// lane bin in it, so l <= k): the pair lies in a sub-cluster pair held at radius l.
__device__ inline void coverage_block(uint32_t* hist, int bin, int lane, int n_radii, int ca,
                                      int cb) {
    if (!__builtin_amdgcn_ballot_w64(bin < n_radii)) return;
    int b = bin;
    if (ca >= 1) b = fold_min<1>(b, lane);
    if (ca >= 2) b = fold_min<2>(b, lane);
    if (ca >= 3) b = fold_min<4>(b, lane);
    if (cb >= 1) b = fold_min<8>(b, lane);
    if (cb >= 2) b = fold_min<16>(b, lane);
    if (cb >= 3) b = fold_min<32>(b, lane);
    if (bin < n_radii) atomicAdd(&hist[b * kCensusBins + bin], 1u);
}

template <int NCH, bool COVER>
__global__ __launch_bounds__(kCensusWaves * kWave) void k_census(
    const NbItem* __restrict__ items, const NbEntry* __restrict__ entries,
    const float4* __restrict__ xw, const float4* __restrict__ cl_bb,
    const NbScInfo* __restrict__ sc_info, const NbSys* __restrict__ sys, int n_items,
    const float* __restrict__ r2_sorted, int n_radii, int n_pad, int ca, int cb,
    uint32_t* __restrict__ block_hist) {
#pragma clang fp contract(off)
    constexpr int kWords = COVER ? kCoverWords : kHistWords;
    __shared__ uint32_t hist[kWords];
    __shared__ __attribute__((aligned(16))) float s_thr[8 * (NCH + 1)];
    for (int t = threadIdx.x; t < kWords; t += blockDim.x) hist[t] = 0u;
    for (int t = threadIdx.x; t < 8 * (NCH + 1); t += blockDim.x)
        s_thr[t] = (t < n_pad) ? r2_sorted[t] : __builtin_inff();
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    const int ii = lane & 7, jj = lane >> 3;
    const float big = FLT_MAX;                     // a pair not counted: above every radius
    float piv[NCH];                                // last threshold of each chunk of 8
#pragma unroll
    for (int c = 0; c < NCH; ++c) piv[c] = r2_sorted[8 * c + 7];
    for (int k = blockIdx.x * kCensusWaves + wave; k < n_items;
         k += gridDim.x * kCensusWaves) {
        const NbItem it = items[k];
        const NbSys S = sys[sc_info[it.sc].sys];
        const int ci0 = kClustersPerSc * it.sc;
        // build positions and atom counts of the item's i-clusters (empty slots hold zeros
        // in the build coordinates: lanes past a cluster's count are not counted)
#define NB_CI(c)                                                                          \
        const float4 xi##c = xw[kScAtoms * it.sc + kClusterSize * c + ii];                \
        const bool iv##c = ii < (int)cl_bb[2 * (ci0 + c)].w;
        NB_FOR8(NB_CI)
#undef NB_CI
        for (int e = it.e0; e < it.e0 + it.ne; ++e) {
            const NbEntry ent = entries[e];
            float4 xj = xw[kClusterSize * ent.cj + jj];
            const int code = ent.meta & 31u;
            const uint32_t omask = (ent.meta >> 8) & 0xffu;
            const bool jv = jj < (int)((ent.meta >> 24) & 15u);
            const int sx = shift_x(code), sy = shift_y(code), sz = shift_z(code);
            // a = x_i - L for s > 0, b = x_j - L for s < 0, d = a - b (exact shifts)
            xj.x -= (sx < 0) ? S.L[0] : 0.f;
            xj.y -= (sy < 0) ? S.L[1] : 0.f;
            xj.z -= (sz < 0) ? S.L[2] : 0.f;
            const float ox = (sx > 0) ? S.L[0] : 0.f, oy = (sy > 0) ? S.L[1] : 0.f,
                        oz = (sz > 0) ? S.L[2] : 0.f;
            const int dc = (code == kShiftZero) ? ent.cj - ci0 : -1;
#define NB_CB(c)                                                                          \
            if ((omask >> c) & 1u) {                                                      \
                const float dx = (xi##c.x - ox) - xj.x;                                   \
                const float dy = (xi##c.y - oy) - xj.y;                                   \
                const float dz = (xi##c.z - oz) - xj.z;                                   \
                float r2 = (dx * dx + dy * dy) + dz * dz;                                 \
                if (!(iv##c && jv) || (dc == c && ii >= jj)) r2 = big;                    \
                const int bin = bin_of<NCH>(piv, s_thr, r2);                              \
                if constexpr (COVER) coverage_block(hist, bin, lane, n_radii, ca, cb);    \
                else census_block(hist, bin, lane, n_radii);                              \
            }
            NB_FOR8(NB_CB)
#undef NB_CB
        }
    }
    __syncthreads();
    uint32_t* out = block_hist + (size_t)blockIdx.x * kWords;
    for (int t = threadIdx.x; t < kWords; t += blockDim.x) out[t] = hist[t];
}

// Two-stage sum of the block histograms (integer, so the order does not matter): stage 1
// gives each thread kSumRows block rows of one histogram word, stage 2 adds the chunks.
constexpr int kSumRows = 64;

__global__ __launch_bounds__(256) void k_census_sum(const uint32_t* __restrict__ block_hist,
                                                    int n_blocks, int words,
                                                    unsigned long long* __restrict__ part) {
    const int t = blockIdx.x * 256 + threadIdx.x;          // histogram word
    const int b0 = blockIdx.y * kSumRows;
    const int b1 = min(n_blocks, b0 + kSumRows);
    unsigned long long s = 0;
    for (int b = b0; b < b1; ++b) s += block_hist[(size_t)b * words + t];
    part[(size_t)blockIdx.y * words + t] = s;
}

__global__ __launch_bounds__(256) void k_census_total(const unsigned long long* __restrict__ part,
                                                      int n_chunks, int words,
                                                      unsigned long long* __restrict__ total) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    unsigned long long s = 0;
    for (int c = 0; c < n_chunks; ++c) s += part[(size_t)c * words + t];
    total[t] = s;
}

// Thresholds of one census call passed by value (the allocation-free variant writes them
// into its scratch with this kernel instead of a host-to-device copy).
struct NbThrTable {
    float v[NB_CENSUS_MAX_RADII];
};

__global__ void k_set_thr(NbThrTable t, float* __restrict__ out) {
    out[threadIdx.x] = t.v[threadIdx.x];
}

// Scratch of nb_list_census_noalloc: the block histograms of at most kNoAllocBlocks blocks
// (the census kernel's blocks stride over the items, so any list fits), their chunk sums,
// the totals and the thresholds.  Every word used by a call is written by that call
// before it is read, so nothing has to be cleared between calls.
constexpr int kNoAllocBlocks = 1024;
constexpr size_t kNaHistOff = 0;
constexpr size_t kNaPartOff = kNaHistOff + (size_t)kNoAllocBlocks * kHistWords * 4;
constexpr size_t kNaTotalOff = kNaPartOff + (size_t)(kNoAllocBlocks / kSumRows) * kHistWords * 8;
constexpr size_t kNaThrOff = kNaTotalOff + (size_t)kHistWords * 8;
constexpr size_t kNaBytes = kNaThrOff + (size_t)NB_CENSUS_MAX_RADII * 4;
static_assert(kNoAllocBlocks % kSumRows == 0, "whole chunks of block rows");
static_assert(kNaPartOff % 256 == 0 && kNaTotalOff % 256 == 0 && kNaThrOff % 256 == 0,
              "aligned sub-buffers");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

}  // namespace

// Device address of this device's copy of `scratch`, looked up once per device with that
// device current (each device holds its own copy at its own address; host code must use
// this address, never the symbol itself).
hipError_t census_noalloc_scratch(int device, NbCensusScratch* out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    unsigned char* base = static_cast<unsigned char*>(addr[device]);
    out->hist = reinterpret_cast<uint32_t*>(base + kNaHistOff);
    out->part = reinterpret_cast<unsigned long long*>(base + kNaPartOff);
    out->total = reinterpret_cast<unsigned long long*>(base + kNaTotalOff);
    out->thr = reinterpret_cast<float*>(base + kNaThrOff);
    out->max_blocks = kNoAllocBlocks;
    out->bytes = kNaBytes;
    return hipSuccess;
}

hipError_t launch_set_thresholds(const float* r2_sorted_host, float* thr, hipStream_t s) {
    NbThrTable t;
    for (int k = 0; k < NB_CENSUS_MAX_RADII; ++k) t.v[k] = r2_sorted_host[k];
    hipLaunchKernelGGL(k_set_thr, dim3(1), dim3(NB_CENSUS_MAX_RADII), 0, s, t, thr);
    return hipGetLastError();
}

int census_blocks(int n_items, bool cover) {
    const int need = (n_items + kCensusWaves - 1) / kCensusWaves;   // one item per wavefront
    return std::max(1, std::min(need, cover ? kCoverMaxBlocks : kCensusMaxBlocks));
}

size_t census_words(bool cover) { return cover ? kCoverWords : kHistWords; }

hipError_t launch_census(const NbDev& d, int n_items, const float* r2_sorted, int n_radii,
                         bool cover, int ca, int cb, uint32_t* block_hist, int n_blocks,
                         hipStream_t s) {
    const int n_pad = (n_radii + 7) / 8 * 8;     // r2_sorted holds +inf up to n_pad
#define NB_CENSUS_LAUNCH(NCH, COV)                                                           \
    hipLaunchKernelGGL((k_census<NCH, COV>), dim3(n_blocks), dim3(kCensusWaves * kWave), 0, \
                       s, d.items, d.entries, d.xw, d.cl_bb, d.sc_info, d.sys, n_items,     \
                       r2_sorted, n_radii, n_pad, ca, cb, block_hist)
#define NB_CENSUS_CASES(COV)                                                                 \
    switch (n_pad / 8) {                                                                     \
        case 1: NB_CENSUS_LAUNCH(1, COV); break;                                             \
        case 2: NB_CENSUS_LAUNCH(2, COV); break;                                             \
        case 3: NB_CENSUS_LAUNCH(3, COV); break;                                             \
        case 4: NB_CENSUS_LAUNCH(4, COV); break;                                             \
        case 5: NB_CENSUS_LAUNCH(5, COV); break;                                             \
        case 6: NB_CENSUS_LAUNCH(6, COV); break;                                             \
        case 7: NB_CENSUS_LAUNCH(7, COV); break;                                             \
        default: NB_CENSUS_LAUNCH(8, COV); break;                                            \
    }
    if (cover) {
        NB_CENSUS_CASES(true)
    } else {
        NB_CENSUS_CASES(false)
    }
#undef NB_CENSUS_CASES
#undef NB_CENSUS_LAUNCH
    return hipGetLastError();
}

hipError_t launch_census_sum(const uint32_t* block_hist, int n_blocks, bool cover,
                             unsigned long long* part, unsigned long long* total,
                             hipStream_t s) {
    const int words = cover ? kCoverWords : kHistWords;
    const int n_chunks = (n_blocks + kSumRows - 1) / kSumRows;
    hipLaunchKernelGGL(k_census_sum, dim3(words / 256, n_chunks), dim3(256), 0, s, block_hist,
                       n_blocks, words, part);
    hipLaunchKernelGGL(k_census_total, dim3(words / 256), dim3(256), 0, s, part, n_chunks, words,
                       total);
    return hipGetLastError();
}
