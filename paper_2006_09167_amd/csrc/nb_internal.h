// Internal declarations shared by the host layer and the HIP kernels of the
// cluster-pair nonbonded library.  Not part of the public ABI (see include/nb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "nb.h"

// ---- fixed geometry of the cluster setup (Sec. V.A: 8x8 on 64-wide AMD GPUs, 8-way
// super-clustering from a 2x2x2 grouping) ------------------------------------------------
constexpr int kClusterSize = 8;                 // atoms per cluster (i and j side)
constexpr int kClustersPerSc = 8;               // clusters per super-cluster
constexpr int kScAtoms = 64;                    // atom slots per super-cluster
constexpr int kWave = 64;                       // wavefront width on gfx950
constexpr int kSearchWaves = 4;                 // wavefronts per super-cluster in the search
constexpr int kMaxTypes = 32;                   // LJ types supported by the kernels
constexpr int kMaxExcl = 32;                    // exclusion partners per atom
constexpr int kShiftZero = 13;                  // shift code of s = (0,0,0)
constexpr int kXcds = 8;                        // accelerator complex dies of an MI355X

// Execution modes of the pair kernel (values of NB_EXEC_* in nb.h).
constexpr int kExecStatic = 0;                  // one wavefront per item, in item order
constexpr int kExecXcd = 1;                     // blocks renumbered XCD-contiguously
constexpr int kExecQueue = 2;                   // balanced runs, then a dynamic tail
constexpr int kExecPersist = 3;                 // persistent grid, fixed balanced schedule
constexpr int kExecBalanced = 4;                // one run of equal-cost items per wavefront
// where nb_step prunes (values of nb_exec_config.prune_fused)
constexpr int kPruneSeparate = 0, kPruneFused = 1, kPruneAhead = 2;
constexpr int kMaxBalancedWaves = 16384;        // runs of a balanced partition, at most
// Queue mode: the wavefronts' own runs carry this share of the estimated cost (per mille),
// the rest is cut into kQueueDynPerTwoWaves x (wavefronts) / 2 shorter runs taken from
// kQueuePools ticket pools (pool p: runs p, p + kQueuePools, ...); each counter on its own
// 128-byte line (same-address atomics serialise at about 12 ns each on this GPU).
constexpr int kQueueStaticPermille = 650;
constexpr int kQueueDynPerTwoWaves = 2;
constexpr int kQueuePools = 64;                 // pool of wavefront g: g mod kQueuePools
constexpr int kPoolStride = 32;                 // int32 words per counter
constexpr int kQueueTickets = kPoolStride;      // queue[] offsets: ticket counters,
constexpr int kQueueDone = kQueueTickets + kQueuePools * kPoolStride;   // finished blocks
constexpr int kQueueDoneAll = kQueueDone + kQueuePools * kPoolStride;   // per group, groups
constexpr int kQueueWords = kQueueDoneAll + kPoolStride;
constexpr int kMaxItemCost = 64 * 10;           // estimated cost of one item, at most

// One j-entry of a super-cluster's joint list (16 bytes, loaded with one scalar load).
//   meta bits  0..4   shift code (sx+1)*9 + (sy+1)*3 + (sz+1), image x_j + s L
//              8..15  outer interaction mask (bit c: i-cluster c of the super-cluster)
//             16..23  inner interaction mask (rolling-pruned copy of the outer mask)
//             24..27  atoms in the j-cluster (1..8)
//   excl      exclusion row (8 x 64-bit masks, one per i-cluster), -1 = no exclusions
//   jpos      slot of this entry's j-force partials in the transposed partial buffer
struct __attribute__((aligned(16))) NbEntry {
    int32_t cj;
    uint32_t meta;
    int32_t excl;
    int32_t jpos;
};

// One work item: a chunk of one super-cluster's j-list, processed by one wavefront.
// pos is the item's rank in super-cluster order (items themselves are grouped by
// rolling-prune part), so that per-system partial sums are contiguous.
struct __attribute__((aligned(16))) NbItem {
    int32_t sc;
    int32_t e0;
    int32_t ne;
    int32_t pos;
};

// Per-system grid geometry (device copy).
struct NbSys {
    float L[3];          // box edges
    float invL[3];       // float32(1 / L)
    float cinv[2];       // float32(nx / Lx), float32(ny / Ly)
    float colw[2];       // column widths Lx / nx, Ly / ny (search ranges only)
    int32_t nx, ny;      // columns per axis
    int32_t col_base;    // first global column id
    int32_t atom0, atom1;
    int32_t pad;
};

// Per-super-cluster info written by the grid build.
struct NbScInfo {
    int32_t col;         // global column id
    int32_t sys;         // system index
    int32_t cx, cy;      // column coordinates inside the system's grid
};

// Scalar pair-interaction constants passed by value to the kernels.
struct NbKParams {
    float rc2;           // cut-off squared (single precision)
    float krf, crf;      // reaction-field constants (nearest single-precision values)
    float krf_lo, crf_lo;// their rounding residuals (k_rf - krf, c_rf - crf): the energy
                         // sums q_i q_j (krf_lo r^2 - crf_lo) apart, else c_rf's rounding
                         // times the sum of q_i q_j leaves a 1e-6 relative bias in E_C
    float beta;          // Ewald splitting parameter
    float p_beta;        // p beta, p the slope of the erfc substitution u = 1/(1 + p beta r)
    float beta2_log2e;   // -beta^2 / ln 2 (exp(-beta^2 r^2) = exp2(r^2 * this))
    float two_beta_sqrtpi;  // 2 beta / sqrt(pi)
    float ewald_shift;   // erfc(beta rc)/rc under the potential-shift modifier, else 0
    float epsfac_r;      // epsfac / eps_r
    float rc_m6, rc_m12; // rc^-6, rc^-12 under the potential-shift modifier, else 0
    int32_t n_types;
};

// Device flags written by kernels and read at the next synchronising call.
enum NbFlag {
    kFlagNonFinite = 0,   // a coordinate was not finite
    kFlagScOverflow = 1,  // a super-cluster had more entries than the per-sc capacity
    kFlagScNeeded = 2,    // largest per-sc entry count seen
    kFlagNumSc = 3,       // number of super-clusters of the current grid
    kFlagNumRows = 4,     // exclusion rows allocated
    kFlagBbPairs = 5,     // cluster pairs passing the bounding-box test
    kFlagBbRecords = 6,   // records written by the recording search (nb_get_pairs, BB)
    kFlagCount = 8
};

// ---- kernel launchers (nb_grid.hip, nb_list.hip, nb_forces.hip, nb_backward.hip) -------
struct NbDev;   // device buffer set, defined below

hipError_t launch_grid_build(const NbDev& d, const float* x, hipStream_t s);
hipError_t launch_search(const NbDev& d, int n_sc, int cap, float r2_outer, float r2_inner,
                         float rlist, hipStream_t s);
// The same search recording only the cluster pairs that pass the bounding-box tests
// (d.bb_rec, at most rec_cap records, counted in flags[kFlagBbRecords]).
hipError_t launch_search_record(const NbDev& d, int n_sc, float r2_outer, float rlist,
                                int rec_cap, hipStream_t s);
hipError_t launch_scan_entries(const NbDev& d, int n_sc, hipStream_t s);
// Work items of at most w entries; balanced_waves > 0: the balanced and queue modes'
// partition of the list into that many equal-cost runs (wave_e, wave_item), the first
// static_permille / 1000 of the cost when dynamic_runs > 0, whose runs hold the rest;
// else per super-cluster.
hipError_t launch_make_items(const NbDev& d, int n_sc, int cap, int w, int nstprune,
                             bool copy_entries, int balanced_waves, int dynamic_runs,
                             int static_permille, hipStream_t s);
hipError_t launch_item_order(const NbDev& d, int n_items, hipStream_t s);
hipError_t launch_list_finish(const NbDev& d, int n_sc, int64_t n_entries, int n_cl,
                              hipStream_t s);
hipError_t launch_fill(int32_t* p, int n, int32_t v, hipStream_t s);
hipError_t launch_fill_d(double* p, int n, double v, hipStream_t s);
hipError_t launch_gather(const NbDev& d, const float* x, const float* q, float4* out,
                         int n_slots, hipStream_t s);
// waves: wavefronts per item (1, 2, 4, 8), or 0 for the most with which all the part's
// blocks are resident at once
hipError_t launch_prune(const NbDev& d, const float4* coords, int item0, int n_items,
                        float r2_inner, int waves, hipStream_t s);
// prune_part >= 0: the pair kernel also re-prunes the items of that rolling part (parts by
// super-cluster mod nstprune).
hipError_t launch_forces(const NbDev& d, const NbKParams& kp, int coulomb, uint32_t flags,
                         const float* lj, int n_items, int prune_part, int nstprune,
                         float r2_inner, int mode, hipStream_t s);
// Resolve once, outside any stream capture, the launch shape of the pair kernel flavor
// for these flags (its occupancy, used by the persistent modes); optionally returns the
// wavefronts of that flavor resident per CU.
hipError_t prepare_forces(int coulomb, uint32_t flags, bool prune, int n_types,
                          int* waves_per_cu = nullptr);
// Per-atom forces (compensated sums of the partials, written in the caller's order) and,
// with NB_F_ENERGY / NB_F_VIRIAL, the energy chunks in the same launch, then per system.
// prune_part >= 0: the same launch also prunes the lists of that rolling part's
// super-clusters (prune_part, prune_part + nstprune, ...; their items are
// part_items[item0 .. item0 + n_part_items)) against r2_inner with the gathered
// coordinates (the ahead prune)
hipError_t launch_reduce(const NbDev& d, float* f, bool accumulate, int n_slots,
                        double* energy, double* virial, uint32_t flags, int n_sys,
                        const float4* xcf, int prune_part, int nstprune, int item0,
                        int n_part_items, float r2_inner, hipStream_t s);
// Electrostatic corrections of excluded pairs inside rc and of each atom with itself
// (nb_excl.hip): per-slot forces into xcf (float4 [64 n_sc_max]) and per-super-cluster
// energy and virial partials into xce ([7][n_sc_max]: E_C, then the six virial sums
// xx yy zz xy xz yz of phi d d); then added per system to energy / virial.
hipError_t launch_excl_corr(const NbDev& d, const NbKParams& kp, int coulomb, double krf,
                            double crf, int n_sc, float4* xcf, double* xce, hipStream_t s);
hipError_t launch_excl_energy(const NbDev& d, const double* xce, double* energy, double* virial,
                              uint32_t flags, int n_sys, hipStream_t s);
// Wavefronts of the backward kernel's flavor (with or without the table gradient)
// resident per CU.
int backward_waves_per_cu(int coulomb, bool ljgrad, int n_types);
hipError_t launch_backward(const NbDev& d, const NbKParams& kp, int coulomb, const float* lj,
                           const float* grad_f, const double* grad_energy, bool ljgrad,
                           int n_slots, int n_items, int mode, hipStream_t s);
hipError_t launch_reduce_backward(const NbDev& d, float* grad_x, float* grad_q,
                                  double* grad_lj, bool accumulate, int n_slots,
                                  int n_types, int n_items, hipStream_t s);

// Work-efficiency census and coverage of the outer list at its build positions
// (nb_census.hip): r2_sorted holds the ascending squared radii followed by +inf up to a
// multiple of 8; a call uses census_blocks(n_items, cover) blocks of census_words(cover)
// histogram words each, then part (one row of words per 64 blocks) and total (words).
int census_blocks(int n_items, bool cover);
size_t census_words(bool cover);
hipError_t launch_census(const NbDev& d, int n_items, const float* r2_sorted, int n_radii,
                         bool cover, int ca, int cb, uint32_t* block_hist, int n_blocks,
                         hipStream_t s);
hipError_t launch_census_sum(const uint32_t* block_hist, int n_blocks, bool cover,
                             unsigned long long* part, unsigned long long* total,
                             hipStream_t s);

// Allocation-free census (nb_list_census_noalloc): sub-buffers of a file-scope device
// array in nb_census.hip, resolved per device.  hist holds max_blocks block histograms of
// census_words(false) words, part their chunk sums, total the summed words, thr the
// NB_CENSUS_MAX_RADII thresholds.
constexpr int kMaxDevices = 64;
struct NbCensusScratch {
    uint32_t* hist;
    unsigned long long* part;
    unsigned long long* total;
    float* thr;
    int max_blocks;
    size_t bytes;
};
hipError_t census_noalloc_scratch(int device, NbCensusScratch* out);
// Writes the NB_CENSUS_MAX_RADII thresholds of a host array into device memory by a kernel
// argument (no host-to-device copy).
hipError_t launch_set_thresholds(const float* r2_sorted_host, float* thr, hipStream_t s);

// All device arrays of a context (plain pointers; sizes in the comments).
struct NbDev {
    int32_t n_atoms = 0, n_sys = 0, n_cols = 0, n_types = 0, max_excl = 0;
    int32_t n_sc_max = 0;              // upper bound of super-clusters for the grid
    int32_t n_cu = 0;                  // compute units of the device
    float filler_d = 0.f;              // lattice spacing of the empty slots' positions (nm)
    // topology
    int32_t* type = nullptr;           // [N]
    int32_t* atom_sys = nullptr;       // [N]
    int32_t* excl_ptr = nullptr;       // [N+1]
    int32_t* excl_idx = nullptr;       // [nnz]
    NbSys* sys = nullptr;              // [n_sys]
    int32_t* sys_sc_start = nullptr;   // [n_sys+1] super-cluster range per system
    // grid
    int4* img = nullptr;               // [N] (kx, ky, kz, column)
    float4* wpos = nullptr;            // [N] wrapped build coordinates
    int32_t* col_count = nullptr;      // [n_cols]
    int32_t* col_start = nullptr;      // [n_cols+1]
    int32_t* col_sc_start = nullptr;   // [n_cols+1]
    int32_t* col_cursor = nullptr;     // [n_cols]
    int32_t* col_atoms = nullptr;      // [N] bucketed by column
    int32_t* col_sorted = nullptr;     // [N] sorted by (column, z, index)
    NbScInfo* sc_info = nullptr;       // [n_sc_max]
    int32_t* slot_atom = nullptr;      // [64 n_sc_max]
    float4* slot_pre = nullptr;        // [64 n_sc_max] per slot of the last grid build: the
                                       // image offset (kx Lx, ky Ly, kz Lz, 0) subtracted
                                       // from its atom, or an empty slot's filler position
    int32_t* atom_slot = nullptr;      // [N]
    int32_t* type_slot = nullptr;      // [64 n_sc_max] 16 type: the byte offset of the type's
                                       // entry in a row of a float4 table over types
    int32_t* excl_slot = nullptr;      // [64 n_sc_max][max_excl]
    int2* cl_xrange = nullptr;         // [8 n_sc_max] clusters holding excluded partners: [lo, hi]
    float4* cl_bb = nullptr;           // [8 n_sc_max][2] lo (w = atom count), hi
    float4* sc_bb = nullptr;           // [n_sc_max][2]
    float4* xw = nullptr;              // [64 n_sc_max] build coordinates by slot
    // per-call gathered data
    float4* xq = nullptr;              // [64 n_sc_max] (x, y, z, q) by slot
    float4* xp = nullptr;              // [64 n_sc_max] prune coordinates by slot
    float4* gslot = nullptr;           // [64 n_sc_max] adjoint dL/dF by slot
    // lists
    int32_t* sc_ecount = nullptr;      // [n_sc_max]
    int32_t* sc_estart = nullptr;      // [n_sc_max+1]
    int32_t* sc_istart = nullptr;      // [n_sc_max+1] items of a super-cluster (contiguous)
    int32_t* sc_icount = nullptr;      // [n_sc_max]
    int32_t* sc_ipos = nullptr;        // [n_sc_max+1] item ranks in super-cluster order
    NbEntry* scratch = nullptr;        // [n_sc_max * cap]
    int4* bb_rec = nullptr;            // bounding-box records (sc, cj, shift code, i-mask),
                                       // only during nb_get_pairs(which = 0)
    NbEntry* entries = nullptr;        // [entry_cap]
    int32_t* entry_sc = nullptr;       // [entry_cap]
    NbItem* items = nullptr;           // [item_cap]
    int32_t* item_cost = nullptr;      // [item_cap] estimated cost per item (k_item_cost)
    int32_t* item_order = nullptr;     // [item_cap] items by decreasing cost (queue order)
    int32_t* queue = nullptr;          // [kQueueWords] unused, unused, finished
                                       //     energy-chunk blocks, finished backward chunks,
                                       //     then the queue mode's pool counters (kept zero
                                       //     between launches by the kernels themselves)
    int32_t* part_start = nullptr;     // [nstprune+1] ranges of part_items per rolling part
    int32_t* part_items = nullptr;     // [item_cap] items grouped by rolling part
    int32_t* wave_e = nullptr;         // [kMaxBalancedWaves+1] first entry per run
    int32_t* wave_item = nullptr;      // [kMaxBalancedWaves+1] first item per run
    int32_t n_waves = 0;               // wavefronts of the balanced partition (0: none)
    int32_t n_dyn = 0;                 // dynamic runs after them (queue mode)
    // The backward pass's own items (per super-cluster, of the width whose items fit its
    // resident grid in one round), when that width differs from the forward items':
    // same layout as items, item_order, item_cost, sc_istart, sc_icount, sc_ipos,
    // part_items, part_start, totals
    NbItem* b_items = nullptr;
    int32_t* b_item_order = nullptr;
    int32_t* b_item_cost = nullptr;
    int32_t* b_sc_istart = nullptr;
    int32_t* b_sc_icount = nullptr;
    int32_t* b_sc_ipos = nullptr;
    int32_t* b_part_items = nullptr;
    int32_t* b_part_start = nullptr;
    int32_t* b_totals = nullptr;
    uint64_t* excl_rows = nullptr;     // [entry_cap][8]
    int32_t* jseg_count = nullptr;     // [8 n_sc_max]
    int32_t* jseg_start = nullptr;     // [8 n_sc_max + 1]
    int32_t* jseg_fill = nullptr;      // [8 n_sc_max]
    int32_t* jseg_entries = nullptr;   // [entry_cap]
    int32_t* totals = nullptr;         // [8]: entries, items, ...
    int32_t* flags = nullptr;          // [kFlagCount]
    // force partials
    float4* jpart = nullptr;           // [entry_cap * 8]
    int64_t entry_cap = 0;             // entries allocated
    float4* ipart = nullptr;           // [item_cap * 64]
    double* epart = nullptr;           // [kEpartStride][epart_stride] by item rank
    int32_t epart_stride = 0;
    float* glj_part = nullptr;         // [T * T * 2][epart_stride] by item rank
    int4* chunks = nullptr;            // [n_chunks] (system, first rank, end rank, 0)
    int32_t* sys_chunk_start = nullptr;// [n_sys+1]
    double* cpart = nullptr;           // [n_chunks][kChunkVals] chunk partial sums
    int32_t n_chunks = 0;
    double* dstat = nullptr;           // [n_sys][2]: effective / computed pairs, last call
    float4* xcf = nullptr;             // [64 n_sc_max] exclusion-correction forces by slot
    double* xce = nullptr;             // [7][n_sc_max] exclusion-correction energy, virial
};

constexpr int kEpartStride = 10;       // E_LJ, E_C, virial xx yy zz xy xz yz, pairs, slots
constexpr int kChunkItems = 1024;      // items per chunk of the two-stage reductions
constexpr int kChunkVals = 2 * kMaxTypes * kMaxTypes;  // values per chunk partial (max)
