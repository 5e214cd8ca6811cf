// Pair-list build and pruning (Sec. V.A, V.D, V.E).
//
// * k_search: one wavefront per i-super-cluster walks the neighbouring grid columns
//   (with periodic shifts), tests super-cluster then cluster bounding boxes against
//   rlist, and prunes each candidate (j-cluster, i-cluster) pair on atom distances with
//   a 64-lane ballot ("warp collectives"); the outer mask keeps pairs with an atom pair
//   closer than rlist, the inner mask those closer than rinner.
// * k_compact / items: entries are copied to one array in super-cluster order and cut
//   into work items of at most W entries, of near-equal length within a super-cluster
//   (list splitting, Sec. V.F), grouped by rolling-prune part.
// * exclusion rows: 64-bit masks per (entry, i-cluster) for force-field exclusions.
// * j-partial slots: entries referencing the same j-cluster get consecutive slots of the
//   partial-force buffer, ordered by entry index (deterministic force sums).
// * k_prune: rolling prune of one part of the outer list against rinner (Sec. V.E).
//
// Atom distances for list decisions use a fixed single-precision sequence without fused
// operations: per axis a = (s > 0) ? x_i - L : x_i, b = (s < 0) ? x_j - L : x_j,
// d = a - b; r2 = (dx*dx + dy*dy) + dz*dz; inside iff r2 < R2.
#include <algorithm>

#include "nb_internal.h"
#include "nb_pair_common.h"
#include "nb_prune_item.h"

namespace {

constexpr int kScanThreads = 1024;

__device__ inline int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Squared distance of atom i and the image s of atom j in the specified sequence.
__device__ inline float list_r2(float4 xi, float4 xj, int sx, int sy, int sz, const NbSys& S) {
#pragma clang fp contract(off)
    const float ax = (sx > 0) ? xi.x - S.L[0] : xi.x;
    const float ay = (sy > 0) ? xi.y - S.L[1] : xi.y;
    const float az = (sz > 0) ? xi.z - S.L[2] : xi.z;
    const float bx = (sx < 0) ? xj.x - S.L[0] : xj.x;
    const float by = (sy < 0) ? xj.y - S.L[1] : xj.y;
    const float bz = (sz < 0) ? xj.z - S.L[2] : xj.z;
    const float dx = ax - bx, dy = ay - by, dz = az - bz;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float t = xx + yy;
    return t + zz;
}

// Gap along one axis between an i box [ilo, ihi] and a j box [jlo, jhi] whose image is
// x_j + s L, with the shift on the same side as in list_r2 (x_i - L for s > 0, x_j - L for
// s < 0).  Rounding is monotone, so every atom's shifted coordinate lies inside its box's
// shifted bounds, and the gap (b_lo - a_hi or a_lo - b_hi, one rounding) is at most the
// |a - b| of every atom pair of the two boxes.
__device__ inline float bb_gap(float ilo, float ihi, float jlo, float jhi, int s, float L) {
#pragma clang fp contract(off)
    const float alo = (s > 0) ? ilo - L : ilo, ahi = (s > 0) ? ihi - L : ihi;
    const float blo = (s < 0) ? jlo - L : jlo, bhi = (s < 0) ? jhi - L : jhi;
    return fmaxf(0.f, fmaxf(blo - ahi, alo - bhi));
}

// Squared box gap summed as list_r2 sums (no contraction).  Squares and sums of
// non-negative terms are monotone too, so bb_d2 <= list_r2 for every atom pair of the two
// boxes: compared with the list's own squared radius, the box test never rejects a pair the
// atom-distance test would keep (the bounding-box candidates are a superset of the list,
// Sec. V.D), for any box edge.
__device__ inline float bb_d2(float4 ilo, float4 ihi, float4 jlo, float4 jhi, int sx, int sy,
                              int sz, const NbSys& S) {
#pragma clang fp contract(off)
    const float gx = bb_gap(ilo.x, ihi.x, jlo.x, jhi.x, sx, S.L[0]);
    const float gy = bb_gap(ilo.y, ihi.y, jlo.y, jhi.y, sy, S.L[1]);
    const float gz = bb_gap(ilo.z, ihi.z, jlo.z, jhi.z, sz, S.L[2]);
    const float xx = gx * gx, yy = gy * gy, zz = gz * gz;
    const float t = xx + yy;
    return t + zz;
}

// Valid-lane mask of an 8x8 cluster pair (lane = ii + 8 jj): real i-atoms (ii < ni), real
// j-atoms (jj < nj) and, for a cluster with itself at s = 0, only ii < jj.
__device__ inline uint64_t pair_valid_mask(int ni, int nj, bool diag) {
    const uint64_t ibyte = (ni >= 8) ? 0xffull : ((1ull << ni) - 1ull);
    const uint64_t imask = ibyte * 0x0101010101010101ull;
    const uint64_t jmask = (nj >= 8) ? ~0ull : ((1ull << (8 * nj)) - 1ull);
    const uint64_t tri = 0x7f3f1f0f07030100ull;      // bit ii + 8 jj set iff ii < jj
    return imask & jmask & (diag ? tri : ~0ull);
}

// One block of kSearchWaves wavefronts per i-super-cluster.  The candidate j-super-clusters
// are visited column by column in batches of 64 (super-cluster, z shift) candidates; batch
// u of that sequence goes to wavefront u mod kSearchWaves, which writes its entries in its
// own cap-long region of the super-cluster's scratch (kSearchWaves cap entries); at the end
// the regions are moved together in wavefront order, so the entry order is fixed by the
// grid alone.  kRecord: only list the cluster pairs that pass the bounding-box tests, as
// records (super-cluster, j-cluster, shift code, 8-bit i-mask) in d.bb_rec (counted in
// flags[kFlagBbRecords]), and leave the list and its counters alone.
template <bool kRecord>
__global__ __launch_bounds__(kSearchWaves * kWave) void k_search(NbDev d, int cap, float r2_outer,
                                                                  float r2_inner, float rlist,
                                                                  int rec_cap) {
    const int sc = blockIdx.x;
    // the grid may be launched for the bound on the super-cluster count: the grid build's
    // own count decides, and a grid built from non-finite coordinates is not searched
    if (sc >= d.flags[kFlagNumSc] || d.flags[kFlagNonFinite]) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    const int ii = lane & 7, jj = lane >> 3;
    __shared__ float4 s_ilo[kClustersPerSc], s_ihi[kClustersPerSc];
    __shared__ float4 s_ix[kScAtoms];
    __shared__ int s_n[kSearchWaves];
    const NbScInfo info = d.sc_info[sc];
    const NbSys S = d.sys[info.sys];
    if (threadIdx.x < kClustersPerSc) {
        s_ilo[threadIdx.x] = d.cl_bb[2 * (kClustersPerSc * sc + threadIdx.x)];
        s_ihi[threadIdx.x] = d.cl_bb[2 * (kClustersPerSc * sc + threadIdx.x) + 1];
    }
    if (threadIdx.x < kScAtoms) s_ix[threadIdx.x] = d.xw[kScAtoms * sc + threadIdx.x];
    __syncthreads();
    const float4 slo = d.sc_bb[2 * sc], shi = d.sc_bb[2 * sc + 1];
    const float margin = 0.01f;   // in column widths; column ranges only need to be supersets
    const int jx0 = (int)floorf((slo.x - rlist) / S.colw[0] - margin);
    const int jx1 = (int)floorf((shi.x + rlist) / S.colw[0] + margin);
    const int jy0 = (int)floorf((slo.y - rlist) / S.colw[1] - margin);
    const int jy1 = (int)floorf((shi.y + rlist) / S.colw[1] + margin);
    const int ci0 = kClustersPerSc * sc;
    NbEntry* out = d.scratch + ((size_t)sc * kSearchWaves + wave) * cap;
    int n_out = 0;
    int bb_pairs = 0;
    int unit = 0;                         // batch number in the super-cluster's sequence
    for (int jx = jx0; jx <= jx1; ++jx) {
        const int sx = floordiv(jx, S.nx);
        if (sx < -1 || sx > 1) continue;
        const int colx = jx - sx * S.nx;
        for (int jy = jy0; jy <= jy1; ++jy) {
            const int sy = floordiv(jy, S.ny);
            if (sy < -1 || sy > 1) continue;
            const int coly = jy - sy * S.ny;
            const int jcol = S.col_base + colx * S.ny + coly;
            const int J0 = max(d.col_sc_start[jcol], sc);
            const int J1 = d.col_sc_start[jcol + 1];
            const int n_cand = (J1 > J0) ? (J1 - J0) * 3 : 0;
            for (int base = 0; base < n_cand; base += kWave, ++unit) {
                if (unit % kSearchWaves != wave) continue;
                const int k = base + lane;
                bool pass = false;
                if (k < n_cand) {
                    const int J = J0 + k / 3;
                    const int sz = k % 3 - 1;
                    const float4 jlo = d.sc_bb[2 * J], jhi = d.sc_bb[2 * J + 1];
                    pass = bb_d2(slo, shi, jlo, jhi, sx, sy, sz, S) < r2_outer;
                }
                uint64_t cand = __builtin_amdgcn_ballot_w64(pass);
                while (cand) {
                    const int t = __builtin_ctzll(cand);
                    cand &= cand - 1;
                    const int J = J0 + (base + t) / 3;
                    const int sz = (base + t) % 3 - 1;
                    const int code = (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1);
                    // 64 cluster-pair box tests: lane -> (j-cluster jj, i-cluster ii); the
                    // j-super-cluster's 64 atoms are loaded at the same time (lane l: atom l)
                    // and handed to the distance tests below by shuffles, so those wait on
                    // no load of their own
                    const int cjl = kClustersPerSc * J + jj;
                    const int cil = ci0 + ii;
                    const float4 jlo = d.cl_bb[2 * cjl], jhi = d.cl_bb[2 * cjl + 1];
                    const float4 xall = d.xw[kScAtoms * J + lane];
                    const bool canon = (cjl > cil) || (cjl == cil && code >= kShiftZero);
                    const bool ok = canon && jlo.w > 0.f && s_ilo[ii].w > 0.f &&
                                    bb_d2(s_ilo[ii], s_ihi[ii], jlo, jhi, sx, sy, sz, S) < r2_outer;
                    const uint64_t M = __builtin_amdgcn_ballot_w64(ok);
                    for (int jc = 0; jc < kClustersPerSc; ++jc) {
                        const uint32_t bbmask = (uint32_t)(M >> (8 * jc)) & 0xffu;
                        if (!bbmask) continue;
                        bb_pairs += __builtin_popcount(bbmask);
                        const int cj = kClustersPerSc * J + jc;
                        if constexpr (kRecord) {
                            if (lane == 0) {
                                const int r = atomicAdd(&d.flags[kFlagBbRecords], 1);
                                if (r < rec_cap)
                                    d.bb_rec[r] = make_int4(sc, cj, code, (int)bbmask);
                            }
                            continue;
                        }
                        // atoms in cluster jc: the box of lane 8 jc (ii = 0, jj = jc)
                        const int nj = (int)__int_as_float(
                            __builtin_amdgcn_readlane(__float_as_int(jlo.w), kClusterSize * jc));
                        const int src = kClusterSize * jc + jj;
                        const float4 xj = make_float4(__shfl(xall.x, src), __shfl(xall.y, src),
                                                      __shfl(xall.z, src), 0.f);
                        uint32_t omask = 0, imask = 0;
                        for (uint32_t bits = bbmask; bits; bits &= bits - 1) {
                            const int c = __builtin_ctz(bits);
                            const float4 xi = s_ix[kClusterSize * c + ii];
                            const float r2 = list_r2(xi, xj, sx, sy, sz, S);
                            const int ni = (int)s_ilo[c].w;
                            const uint64_t valid =
                                pair_valid_mask(ni, nj, cj == ci0 + c && code == kShiftZero);
                            const uint64_t in_o = __builtin_amdgcn_ballot_w64(r2 < r2_outer) & valid;
                            const uint64_t in_i = __builtin_amdgcn_ballot_w64(r2 < r2_inner) & valid;
                            omask |= (in_o ? 1u : 0u) << c;
                            imask |= (in_i ? 1u : 0u) << c;
                        }
                        if (omask) {
                            if (n_out < cap && lane == 0) {
                                NbEntry e;
                                e.cj = cj;
                                e.meta = (uint32_t)code | (omask << 8) | (imask << 16) |
                                         ((uint32_t)nj << 24);
                                e.excl = -1;
                                e.jpos = -1;
                                out[n_out] = e;
                            }
                            ++n_out;
                        }
                    }
                }
            }
        }
    }
    if constexpr (kRecord) return;
    if (lane == 0) {
        s_n[wave] = n_out;
        if (bb_pairs) atomicAdd(&d.flags[kFlagBbPairs], bb_pairs);
    }
    __syncthreads();
    int total = 0, before = 0;
    for (int w = 0; w < kSearchWaves; ++w) {
        const int n = s_n[w];
        if (w < wave) before += min(n, cap);
        total += n;
    }
    // Move the regions together in wavefront order: wavefront w's entries go to
    // [before, before + n) from w cap on, never after their source (before <= w cap), and
    // each 64-entry chunk is read in full before it is written, so a chunk overwrites only
    // entries already moved.  The wavefronts take turns.
    NbEntry* base = d.scratch + (size_t)sc * kSearchWaves * cap;
    for (int w = 1; w < kSearchWaves; ++w) {
        if (wave == w) {
            const int n = min(n_out, cap);
            for (int k0 = 0; k0 < n; k0 += kWave) {
                NbEntry v{};
                if (k0 + lane < n) v = base[(size_t)w * cap + k0 + lane];
                __builtin_amdgcn_wave_barrier();
                if (k0 + lane < n) base[before + k0 + lane] = v;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.sc_ecount[sc] = min(total, cap);
        if (total > cap) atomicOr(&d.flags[kFlagScOverflow], 1);
        atomicMax(&d.flags[kFlagScNeeded], total);
    }
}

// Exclusive scan of a per-super-cluster count (single block).
template <typename F>
__device__ int block_scan(int n, F f, int32_t* __restrict__ out) {
    __shared__ int s_part[kScanThreads];
    const int t = threadIdx.x;
    const int seg = (n + kScanThreads - 1) / kScanThreads;
    const int b = min(n, t * seg), e = min(n, b + seg);
    int sum = 0;
    // each thread walks its own segment: unrolled so that several of its loads are in
    // flight at once (integer sums: the order changes nothing)
#pragma unroll 8
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
#pragma unroll 8
    for (int i = b; i < e; ++i) {
        out[i] = run;
        run += f(i);
    }
    const int total = s_part[kScanThreads - 1];
    __syncthreads();
    if (t == 0) out[n] = total;
    return total;
}

// n_sc < 0: the grid build's own count (none after non-finite coordinates)
__global__ __launch_bounds__(kScanThreads) void k_scan_entries(NbDev d, int n_sc) {
    if (n_sc < 0) n_sc = d.flags[kFlagNonFinite] ? 0 : d.flags[kFlagNumSc];
    const int total = block_scan(n_sc, [&](int i) { return d.sc_ecount[i]; }, d.sc_estart);
    if (threadIdx.x == 0) d.totals[0] = total;
}

// Items per super-cluster: ceil(entries / w), scanned in rolling-part-major order so that
// each part's items are contiguous (part of super-cluster sc is sc mod nstprune).
__global__ __launch_bounds__(kScanThreads) void k_scan_items(NbDev d, int n_sc, int w,
                                                             int nparts, int32_t* tmp) {
    // permuted position k -> super-cluster: parts p hold sc = p, p + nparts, ...
    auto sc_of = [&](int k) {
        int p = 0, before = 0;
        while (p < nparts) {
            const int cnt = (n_sc > p) ? (n_sc - p + nparts - 1) / nparts : 0;
            if (k < before + cnt) break;
            before += cnt;
            ++p;
        }
        return p + nparts * (k - before);
    };
    auto n_items = [&](int k) {
        const int n = d.sc_ecount[sc_of(k)];
        return (n + w - 1) / w;
    };
    block_scan(n_sc, [&](int sc) { return (d.sc_ecount[sc] + w - 1) / w; }, d.sc_ipos);
    __syncthreads();
    const int total = block_scan(n_sc, n_items, tmp);
    __syncthreads();
    for (int k = threadIdx.x; k < n_sc; k += blockDim.x) {
        const int sc = sc_of(k);
        d.sc_istart[sc] = tmp[k];
        d.sc_icount[sc] = n_items(k);
    }
    if (threadIdx.x == 0) {
        int before = 0;
        for (int p = 0; p < nparts; ++p) {
            d.part_start[p] = (before < n_sc) ? tmp[before] : total;
            const int cnt = (n_sc > p) ? (n_sc - p + nparts - 1) / nparts : 0;
            before += cnt;
        }
        d.part_start[nparts] = total;
        d.totals[1] = total;
    }
}

// Per super-cluster: copy its entries from the search scratch (at a build only; later
// re-splits into items of another width keep the entries, whose masks the rolling prune
// has changed since), and write its work items (with write_items; their part-major order
// is the item order itself, so part_items is the identity).
__global__ __launch_bounds__(kWave) void k_compact(NbDev d, int cap, int w, int copy_entries,
                                                   int write_items) {
    const int sc = blockIdx.x;
    const int n = d.sc_ecount[sc];
    const int e0 = d.sc_estart[sc];
    if (copy_entries)
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            d.entries[e0 + k] = d.scratch[(size_t)sc * kSearchWaves * cap + k];
            d.entry_sc[e0 + k] = sc;
        }
    if (!write_items) return;
    const int i0 = d.sc_istart[sc], ni = d.sc_icount[sc];
    const int p0 = d.sc_ipos[sc];
    // ni = ceil(n / w) items of near-equal length (floor or ceil of n / ni, never above w)
    for (int k = threadIdx.x; k < ni; k += blockDim.x) {
        NbItem it;
        it.sc = sc;
        const int a = (int)((int64_t)k * n / ni), b = (int)((int64_t)(k + 1) * n / ni);
        it.e0 = e0 + a;
        it.ne = b - a;
        it.pos = p0 + k;
        d.items[i0 + k] = it;
        d.part_items[i0 + k] = i0 + k;
    }
}

// Work items for the balanced and queue execution modes: the entries (in super-cluster
// order) are dealt in contiguous runs of near-equal cost, an entry costing 2 + (set bits of
// its inner mask) (its j-cluster load, shift, partial store and reductions weigh about two
// 8 x 8 blocks in measured wavefront times), to P wavefronts (the paper's list splitting
// against kernel tails, Sec. V.F, taken to its end: no wavefront waits for another's longer
// list).  With D > 0 (queue mode) the P runs cover the first fs_permille / 1000 of the
// cost and the rest is cut into D shorter runs that wavefronts take from ticket pools once
// their own run is done, which absorbs both the cost model's error and the speed
// differences between SIMDs.  Items are the pieces of a super-cluster's list inside one
// run, cut further into near-equal pieces of at most w entries; wave_item[g] ..
// wave_item[g + 1] are the items of run g (g < P: wavefront g's own, P <= g < P + D:
// dynamic run g - P), in super-cluster order (so item index = rank).  part_items lists the
// items of each rolling part together (part p: super-clusters p, p + nparts, ...) for the
// separate prune.  One block; prefix (>= E + 1 ints) and ppos (>= n_sc ints) are scratch.
__global__ __launch_bounds__(kScanThreads) void k_balanced_items(NbDev d, int n_sc, int w,
                                                                 int nparts, int P, int D,
                                                                 int fs_permille,
                                                                 int32_t* prefix,
                                                                 int32_t* ppos) {
    const int E = d.totals[0];
    const int C = block_scan(E, [&](int i) {
        return 2 + __builtin_popcount((d.entries[i].meta >> 16) & 0xffu);
    }, prefix);
    __syncthreads();
    const int R = P + D;                                             // runs
    const int64_t Cs = (D > 0) ? (int64_t)C * fs_permille / 1000 : C;   // cost of the P runs
    for (int g = threadIdx.x; g <= R; g += blockDim.x) {
        const int64_t target = (g <= P) ? ((int64_t)g * Cs + P - 1) / P      // ceil(g Cs / P)
                                        : Cs + ((int64_t)(g - P) * (C - Cs) + D - 1) / D;
        int lo = 0, hi = E;                                          // first prefix >= target
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        d.wave_e[g] = (g == R) ? E : lo;
    }
    __syncthreads();
    // pieces of super-cluster sc: its entries cut at the wavefront boundaries inside them,
    // each run cut into ceil(len / w) near-equal items; f(first entry, entries, item index
    // within the super-cluster) for each item in order
    auto for_items = [&](int sc, auto&& f) {
        const int a = d.sc_estart[sc], b = a + d.sc_ecount[sc];
        int lo = 0, hi = R + 1;                      // first boundary above a
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (d.wave_e[mid] <= a) lo = mid + 1;
            else hi = mid;
        }
        int k = 0;
        for (int s0 = a, g = lo; s0 < b; ++g) {
            const int t = (g <= R && d.wave_e[g] < b) ? d.wave_e[g] : b;
            const int len = t - s0, ni = (len + w - 1) / w;
            for (int j = 0; j < ni; ++j) {
                const int x0 = (int)((int64_t)j * len / ni), x1 = (int)((int64_t)(j + 1) * len / ni);
                f(s0 + x0, x1 - x0, k++);
            }
            s0 = t;
        }
        return k;
    };
    for (int sc = threadIdx.x; sc < n_sc; sc += blockDim.x)
        d.sc_icount[sc] = for_items(sc, [](int, int, int) {});
    __syncthreads();
    const int total = block_scan(n_sc, [&](int sc) { return d.sc_icount[sc]; }, d.sc_istart);
    __syncthreads();
    // part-major positions: parts p hold super-clusters p, p + nparts, ...
    auto sc_of = [&](int k) {
        int p = 0, before = 0;
        while (p < nparts) {
            const int cnt = (n_sc > p) ? (n_sc - p + nparts - 1) / nparts : 0;
            if (k < before + cnt) break;
            before += cnt;
            ++p;
        }
        return p + nparts * (k - before);
    };
    block_scan(n_sc, [&](int k) { return d.sc_icount[sc_of(k)]; }, ppos);
    __syncthreads();
    for (int sc = threadIdx.x; sc < n_sc; sc += blockDim.x) {
        d.sc_ipos[sc] = d.sc_istart[sc];
        const int i0 = d.sc_istart[sc];
        // part-major position of this super-cluster's first item
        int k = 0;
        {
            const int p = sc % nparts;
            for (int q = 0; q < p; ++q) k += (n_sc > q) ? (n_sc - q + nparts - 1) / nparts : 0;
            k += sc / nparts;
        }
        const int pp = ppos[k];
        for_items(sc, [&](int e0, int ne, int j) {
            NbItem it;
            it.sc = sc;
            it.e0 = e0;
            it.ne = ne;
            it.pos = i0 + j;
            d.items[i0 + j] = it;
            d.part_items[pp + j] = i0 + j;
        });
    }
    __syncthreads();
    for (int g = threadIdx.x; g <= R; g += blockDim.x) {
        // first item starting at or after the run's first entry
        int lo = 0, hi = total;
        const int e = d.wave_e[g];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (d.items[mid].e0 < e) lo = mid + 1;
            else hi = mid;
        }
        d.wave_item[g] = (g == R) ? total : lo;
    }
    if (threadIdx.x == 0) {
        int before = 0;
        for (int p = 0; p < nparts; ++p) {
            d.part_start[p] = (before < n_sc) ? ppos[before] : total;
            before += (n_sc > p) ? (n_sc - p + nparts - 1) / nparts : 0;
        }
        d.part_start[nparts] = total;
        d.totals[1] = total;
    }
    d.sc_ipos[n_sc] = total;
}

// One thread per entry: exclusion masks (bit ii + 8 jj cleared for excluded atom pairs),
// a row only for entries with an exclusion; j-segment counts; list statistics.  Rows and
// statistics are counted per block and taken with one atomic per block each: atomics of
// every wavefront on the same three counters serialised (about 80 us at 96k atoms).
constexpr int kFinishThreads = 1024;
__global__ __launch_bounds__(kFinishThreads) void k_entry_finish(NbDev d, int n_entries) {
    constexpr int kWaves = kFinishThreads / kWave;
    __shared__ int s_rows[kWaves], s_out[kWaves], s_in[kWaves];
    __shared__ int s_base;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int n_outer = 0, n_inner = 0;
    uint64_t m[kClustersPerSc];
    bool any = false;
    NbEntry ent{};
    if (e < n_entries) {
        ent = d.entries[e];
        const int sc = d.entry_sc[e];
        const uint32_t omask = (ent.meta >> 8) & 0xffu;
        // the partner-cluster ranges of the eight i-clusters, then the partner slots of
        // those in range, each group of loads issued together
        int2 xr[kClustersPerSc];
#pragma unroll
        for (int c = 0; c < kClustersPerSc; ++c)
            xr[c] = ((omask >> c) & 1u) ? d.cl_xrange[kClustersPerSc * sc + c]
                                        : make_int2(0x7fffffff, -1);
#pragma unroll
        for (int c = 0; c < kClustersPerSc; ++c) {
            m[c] = ~0ull;
            if (ent.cj < xr[c].x || ent.cj > xr[c].y) continue;   // no partner in cj
            const int ci = kClustersPerSc * sc + c;
            for (int k = 0; k < d.max_excl; ++k) {
                int ps[kClusterSize];
#pragma unroll
                for (int ii = 0; ii < kClusterSize; ++ii)
                    ps[ii] = d.excl_slot[(size_t)(kClusterSize * ci + ii) * d.max_excl + k];
#pragma unroll
                for (int ii = 0; ii < kClusterSize; ++ii)
                    if (ps[ii] >= 0 && ps[ii] / kClusterSize == ent.cj)
                        m[c] &= ~(1ull << (ii + 8 * (ps[ii] % kClusterSize)));
            }
            any |= (m[c] != ~0ull);
        }
        atomicAdd(&d.jseg_count[ent.cj], 1);
        n_outer = __builtin_popcount(omask);
        n_inner = __builtin_popcount((ent.meta >> 16) & 0xffu);
    }
    const uint64_t need = __builtin_amdgcn_ballot_w64(any);
    for (int off = kWave / 2; off > 0; off >>= 1) {
        n_outer += __shfl_xor(n_outer, off);
        n_inner += __shfl_xor(n_inner, off);
    }
    if (lane == 0) {
        s_rows[wave] = __builtin_popcountll(need);
        s_out[wave] = n_outer;
        s_in[wave] = n_inner;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int rows = 0, outer = 0, inner = 0;
        for (int w = 0; w < kWaves; ++w) {
            const int r = s_rows[w];
            s_rows[w] = rows;               // exclusive prefix: the wavefront's first row
            rows += r;
            outer += s_out[w];
            inner += s_in[w];
        }
        s_base = rows ? atomicAdd(&d.flags[kFlagNumRows], rows) : 0;
        if (outer) atomicAdd(&d.totals[2], outer);
        if (inner) atomicAdd(&d.totals[3], inner);
    }
    __syncthreads();
    if (any) {
        const int row =
            s_base + s_rows[wave] + __builtin_popcountll(need & ((1ull << lane) - 1ull));
        for (int c = 0; c < kClustersPerSc; ++c)
            d.excl_rows[(size_t)row * kClustersPerSc + c] = m[c];
        d.entries[e].excl = row;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_jseg(NbDev d, int n_cl) {
    block_scan(n_cl, [&](int i) { return d.jseg_count[i]; }, d.jseg_start);
    for (int i = threadIdx.x; i < n_cl; i += blockDim.x) d.jseg_fill[i] = 0;
}

__global__ void k_jseg_fill(NbDev d, int n_entries) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_entries) return;
    const int cj = d.entries[e].cj;
    const int pos = atomicAdd(&d.jseg_fill[cj], 1);
    d.jseg_entries[d.jseg_start[cj] + pos] = e;
}

// One wavefront per j-cluster: slot of each referencing entry = rank by entry index.
__global__ __launch_bounds__(kWave) void k_jseg_rank(NbDev d) {
    const int cj = blockIdx.x;
    const int s0 = d.jseg_start[cj], s1 = d.jseg_start[cj + 1];
    for (int i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        const int e = d.jseg_entries[i];
        int r = 0;
        for (int j = s0; j < s1; ++j) r += (d.jseg_entries[j] < e) ? 1 : 0;
        d.entries[e].jpos = s0 + r;
    }
}

// Rolling prune (Sec. V.E) of a range of the items of one part (part_items lists each
// part's items together): one block of kPruneWaves wavefronts per item (prune_item).
template <int kPruneWaves>
__global__ __launch_bounds__(kPruneWaves * kWave) void k_prune(
    const NbItem* __restrict__ items, const int32_t* __restrict__ part_items,
    NbEntry* __restrict__ entries, const float4* __restrict__ xp,
    const NbScInfo* __restrict__ sc_info, const NbSys* __restrict__ sys, int item0,
    float r2_inner) {
    __shared__ float4 s_xi[kScAtoms];
    prune_item<kPruneWaves>(items[part_items[item0 + blockIdx.x]], entries, xp, sc_info, sys,
                            r2_inner, s_xi);
}

// Estimated cost of each item (one wavefront per item): per entry 2 + the set bits of its
// inner mask as built (an entry's j-load, shift, partial store and reductions weigh about
// two 8 x 8 blocks in measured wavefront times).
__global__ __launch_bounds__(4 * kWave) void k_item_cost(NbDev d, int n_items) {
    const int item = blockIdx.x * 4 + (int)(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    if (item >= n_items) return;
    const NbItem it = d.items[item];
    int c = 0;
    for (int k = lane; k < it.ne; k += kWave)
        c += 2 + __builtin_popcount((d.entries[it.e0 + k].meta >> 16) & 0xffu);
    for (int off = 1; off < kWave; off <<= 1) c += __shfl_xor(c, off);
    if (lane == 0) d.item_cost[item] = c;
}

// Items by decreasing cost (counting sort in one block), the order in which the
// persistent pair kernel hands them out: the longest items start first.  The order
// among items of equal cost is arbitrary; it changes no result.
__global__ __launch_bounds__(1024) void k_item_order(NbDev d, int n_items) {
    __shared__ int cnt[kMaxItemCost + 1];
    for (int c = threadIdx.x; c <= kMaxItemCost; c += blockDim.x) cnt[c] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n_items; i += blockDim.x)
        atomicAdd(&cnt[min(d.item_cost[i], kMaxItemCost)], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;                        // first position of each cost, largest first
        for (int c = kMaxItemCost; c >= 0; --c) {
            const int k = cnt[c];
            cnt[c] = run;
            run += k;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_items; i += blockDim.x)
        d.item_order[atomicAdd(&cnt[min(d.item_cost[i], kMaxItemCost)], 1)] = i;
}

inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t launch_item_order(const NbDev& d, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipGetLastError();
    hipLaunchKernelGGL(k_item_cost, dim3(blocks(n_items, 4)), dim3(4 * kWave), 0, s, d, n_items);
    hipLaunchKernelGGL(k_item_order, dim3(1), dim3(1024), 0, s, d, n_items);
    return hipGetLastError();
}

hipError_t launch_search(const NbDev& d, int n_sc, int cap, float r2_outer, float r2_inner,
                         float rlist, hipStream_t s) {
    if (n_sc > 0)
        hipLaunchKernelGGL(k_search<false>, dim3(n_sc), dim3(kSearchWaves * kWave), 0, s, d, cap,
                           r2_outer, r2_inner, rlist, 0);
    return hipGetLastError();
}

hipError_t launch_search_record(const NbDev& d, int n_sc, float r2_outer, float rlist,
                                int rec_cap, hipStream_t s) {
    if (n_sc > 0)
        hipLaunchKernelGGL(k_search<true>, dim3(n_sc), dim3(kSearchWaves * kWave), 0, s, d, 0,
                           r2_outer, r2_outer, rlist, rec_cap);
    return hipGetLastError();
}

hipError_t launch_scan_entries(const NbDev& d, int n_sc, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_entries, dim3(1), dim3(kScanThreads), 0, s, d, n_sc);
    return hipGetLastError();
}

hipError_t launch_make_items(const NbDev& d, int n_sc, int cap, int w, int nstprune,
                             bool copy_entries, int balanced_waves, int dynamic_runs,
                             int static_permille, hipStream_t s) {
    if (balanced_waves > 0) {
        if (copy_entries && n_sc > 0)
            hipLaunchKernelGGL(k_compact, dim3(n_sc), dim3(kWave), 0, s, d, cap, w, 1, 0);
        // jseg_entries (entry_cap >= E + 1) and jseg_fill (>= n_sc) serve as scratch
        hipLaunchKernelGGL(k_balanced_items, dim3(1), dim3(kScanThreads), 0, s, d, n_sc, w,
                           nstprune, balanced_waves, dynamic_runs, static_permille,
                           d.jseg_entries, d.jseg_fill);
        return hipGetLastError();
    }
    // jseg_fill doubles as the scratch of the permuted scan (n_sc + 1 <= 8 n_sc_max).
    hipLaunchKernelGGL(k_scan_items, dim3(1), dim3(kScanThreads), 0, s, d, n_sc, w, nstprune,
                       d.jseg_fill);
    if (n_sc > 0)
        hipLaunchKernelGGL(k_compact, dim3(n_sc), dim3(kWave), 0, s, d, cap, w,
                           copy_entries ? 1 : 0, 1);
    return hipGetLastError();
}

hipError_t launch_list_finish(const NbDev& d, int n_sc, int64_t n_entries, int n_cl,
                              hipStream_t s) {
    hipError_t err = launch_fill(d.jseg_count, n_cl, 0, s);
    if (err != hipSuccess) return err;
    if (n_entries > 0)
        hipLaunchKernelGGL(k_entry_finish, dim3(blocks(n_entries, kFinishThreads)),
                           dim3(kFinishThreads), 0, s, d,
                           (int)n_entries);
    hipLaunchKernelGGL(k_scan_jseg, dim3(1), dim3(kScanThreads), 0, s, d, n_cl);
    if (n_entries > 0)
        hipLaunchKernelGGL(k_jseg_fill, dim3(blocks(n_entries, 256)), dim3(256), 0, s, d,
                           (int)n_entries);
    if (n_cl > 0) hipLaunchKernelGGL(k_jseg_rank, dim3(n_cl), dim3(kWave), 0, s, d);
    (void)n_sc;
    return hipGetLastError();
}

namespace {
// Blocks of k_prune<W> resident on one CU (queried once).
template <int W>
int prune_blocks_per_cu() {
    static int per_cu = 0;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_prune<W>, W * kWave, 0) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        per_cu = nb;
    }
    return per_cu;
}
}  // namespace

// Wavefronts per item as asked, or (waves = 0) eight while the part's blocks fill the
// device at most twice over (each wavefront's walk over its entries is then short), else
// two (measured at 96k atoms, 1,400 items per part: 14.6 us with eight against 16.1 with
// four; at 1.5M atoms, 22,000 items per part: 148 us with two, 151 with four, 166 with
// eight).
hipError_t launch_prune(const NbDev& d, const float4* coords, int item0, int n_items,
                        float r2_inner, int waves, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    const int64_t cus = std::max(d.n_cu, 1);
#define NB_PRUNE_LAUNCH(W)                                                                  hipLaunchKernelGGL(k_prune<W>, dim3(n_items), dim3(W * kWave), 0, s, d.items,                                 d.part_items, d.entries, coords, d.sc_info, d.sys, item0, r2_inner)
    if (waves == 0) waves = (n_items <= 2 * prune_blocks_per_cu<8>() * cus) ? 8 : 2;
    if (waves == 8) NB_PRUNE_LAUNCH(8);
    else if (waves == 4) NB_PRUNE_LAUNCH(4);
    else if (waves == 2) NB_PRUNE_LAUNCH(2);
    else NB_PRUNE_LAUNCH(1);
#undef NB_PRUNE_LAUNCH
    return hipGetLastError();
}
