// Host layer of the C ABI (include/nb.h): argument validation, device buffers, and the
// order of kernel launches for the grid build, the dual pair list and the force passes.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "nb_erfc_coeffs.h"
#include "nb_internal.h"

struct nb_ctx {
    nb_params p{};
    int32_t n_sys = 0;
    std::vector<int64_t> offs;
    hipStream_t stream = nullptr;
    int device = 0;
    NbDev d;
    std::vector<NbSys> hsys;
    bool has_topology = false, has_grid = false, has_list = false;
    int32_t n_sc = 0, n_cl = 0, n_slots = 0;
    int64_t n_entries = 0;
    int32_t n_items = 0;
    int32_t cap = 0;          // entries per super-cluster in the search scratch
    int32_t item_w = 0;       // entries per work item of the current list
    int32_t fixed_w = 0;      // item width chosen by nb_set_exec / nb_autotune (0 = rule)
    int32_t exec_mode = kExecStatic;
    int items_kind = 0;           // partition of the current items (items_kind_of)
    // the backward pass's items (see backward_items): for list generation bwd_gen and
    // flavor bwd_flavor (with table gradient or not), bwd_n of width bwd_w, in the b_*
    // arrays when bwd_own, else the forward items
    std::vector<int32_t> h_ecount;   // entries per super-cluster of the current list
    uint64_t bwd_gen = ~0ull;
    int bwd_flavor = -1, bwd_w = 0, bwd_n = 0;
    bool bwd_own = false;
    size_t a_bitems = 0, a_bsc = 0;
    // nb_step's rolling prune: kPruneFused inside the pair kernel, kPruneSeparate as its own
    // kernel before it, kPruneAhead after it in the force reduction's launch, for the next
    // step's part with this step's positions
    int prune_mode = kPruneFused;
    int32_t prune_waves = 0;  // wavefronts per item of the separate prune (0 = automatic)
    uint64_t list_gen = 0;    // bumped whenever items or launch shapes change
    // graphs of nb_step_graph: key = (part, flags, pointers, list_gen)
    struct GraphEntry {
        int part, ahead;
        uint32_t flags;
        const void* ptr[7];
        uint64_t gen;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    std::vector<int32_t> part_start;
    int32_t h_totals[8] = {};  // host copy of the device totals after the last list change
    nb_stats stats{};
    std::string err;
    // allocated element counts
    size_t a_atoms = 0, a_cols = 0, a_sc = 0, a_scratch = 0, a_entries = 0, a_items = 0;
    size_t a_excl_nnz = 0, a_chunks = 0, a_cpart = 0;
    // host copies of the item tables of the current list (see finish_items)
    std::vector<int32_t> h_sss, h_ipos, h_chunk_start;
    std::vector<int4> h_chunks;
    // opt-in kernel timing: event pairs per kind, recorded on the stream
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[NB_T_COUNT];
    std::vector<hipEvent_t> ev_free;
    double t_ms[NB_T_COUNT] = {};
    int64_t t_calls[NB_T_COUNT] = {};
    // census buffers (allocated on the first nb_list_census call)
    uint32_t* census_hist = nullptr;          // [census_hist_n] block histograms
    unsigned long long* census_part = nullptr;   // [census_part_n] chunk sums
    unsigned long long* census_total = nullptr;  // [NB_CENSUS_MAX_RADII^2] totals
    float* census_thr = nullptr;              // [NB_CENSUS_MAX_RADII]
    size_t census_hist_n = 0, census_part_n = 0;
};

namespace {

template <typename T>
hipError_t dev_alloc(T*& p, size_t n) {
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        if (e != hipSuccess) return e;
    }
    if (n == 0) n = 1;
    return hipMalloc((void**)&p, n * sizeof(T));
}

nb_status fail(nb_ctx* c, nb_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

nb_status hip_fail(nb_ctx* c, hipError_t e, const char* where) {
    return fail(c, NB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define NB_HIP(ctx, call)                                          \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);   \
    } while (0)

bool finite_pos(float v) { return isfinite(v) && v > 0.f; }

// Reaction-field constants in double precision: k_rf = (eps_rf - eps_r) / ((2 eps_rf +
// eps_r) rc^3) (1 / (2 rc^3) for eps_rf = inf), c_rf = 1/rc + k_rf rc^2.
void rf_constants(const nb_params& p, double* krf_out, double* crf_out) {
    const double rc = p.rc;
    double krf;
    if (isinf(p.eps_rf)) krf = 1.0 / (2.0 * rc * rc * rc);
    else krf = ((double)p.eps_rf - p.eps_r) / ((2.0 * p.eps_rf + p.eps_r) * rc * rc * rc);
    *krf_out = krf;
    *crf_out = 1.0 / rc + krf * rc * rc;
}

NbKParams kernel_params(const nb_params& p) {
    NbKParams k{};
    const double rc = p.rc;
    k.rc2 = (float)(rc * rc);
    double krf, crf;
    rf_constants(p, &krf, &crf);
    k.krf = (float)krf;
    k.crf = (float)crf;
    k.krf_lo = (float)(krf - (double)k.krf);
    k.crf_lo = (float)(crf - (double)k.crf);
    const double b = p.ewald_beta;
    k.beta = (float)b;
    k.p_beta = (float)((double)NB_ERFC_P * b);
    k.beta2_log2e = (float)(-b * b / log(2.0));
    k.two_beta_sqrtpi = (float)(2.0 * b / sqrt(M_PI));
    const bool shift = p.modifier == NB_MOD_POTSHIFT;
    k.ewald_shift = shift ? (float)(erfc(b * rc) / rc) : 0.f;
    k.epsfac_r = (float)((double)p.epsfac / p.eps_r);
    k.rc_m6 = shift ? (float)pow(rc, -6.0) : 0.f;
    k.rc_m12 = shift ? (float)pow(rc, -12.0) : 0.f;
    k.n_types = p.n_types;
    return k;
}

float radius_sq(float r) { return (float)((double)r * (double)r); }

nb_status sync(nb_ctx* c) {
    NB_HIP(c, hipStreamSynchronize(c->stream));
    return NB_OK;
}

template <typename T>
nb_status to_host(nb_ctx* c, T* host, const T* dev, size_t n) {
    if (n == 0) return NB_OK;
    NB_HIP(c, hipMemcpyAsync(host, dev, n * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

// Device resources of a context are allocated at its first device call, after the
// arguments of that call have been validated (creation itself touches no device).
nb_status ensure_device(nb_ctx* c) {
    if (c->device < 0) NB_HIP(c, hipGetDevice(&c->device));
    NB_HIP(c, hipSetDevice(c->device));
    if (c->d.flags) return NB_OK;
    NbDev& d = c->d;
    NB_HIP(c, dev_alloc(d.flags, kFlagCount));
    NB_HIP(c, dev_alloc(d.totals, 8));
    NB_HIP(c, dev_alloc(d.dstat, 2 * c->n_sys));
    NB_HIP(c, dev_alloc(d.sys, c->n_sys));
    NB_HIP(c, dev_alloc(d.sys_sc_start, c->n_sys + 1));
    NB_HIP(c, dev_alloc(d.part_start, c->p.nstprune + 1));
    NB_HIP(c, dev_alloc(d.queue, kQueueWords));
    NB_HIP(c, dev_alloc(d.wave_e, kMaxBalancedWaves + 1));
    NB_HIP(c, dev_alloc(d.wave_item, kMaxBalancedWaves + 1));
    NB_HIP(c, launch_fill(d.queue, kQueueWords, 0, c->stream));
    int n_cu = 0;
    NB_HIP(c, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    d.n_cu = n_cu;
    return NB_OK;
}

void drop_graphs(nb_ctx* c) {
    for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

hipEvent_t take_event(nb_ctx* c) {
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Start / stop an event pair of the given kind around the launches in between.
struct TimedSection {
    nb_ctx* c;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    TimedSection(nb_ctx* c_, int k, hipStream_t s_ = nullptr)
        : c(c_), kind(k), s(s_ ? s_ : c_->stream) {
        if (!c->timing) return;
        a = take_event(c);
        b = take_event(c);
        if (a) hipEventRecord(a, s);
    }
    ~TimedSection() {
        if (!c->timing || !a || !b) return;
        hipEventRecord(b, s);
        c->ev[kind].emplace_back(a, b);
    }
};

nb_status collect_timing(nb_ctx* c) {
    NB_HIP(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < NB_T_COUNT; ++k) {
        for (auto& pr : c->ev[k]) {
            float ms = 0.f;
            NB_HIP(c, hipEventElapsedTime(&ms, pr.first, pr.second));
            c->t_ms[k] += ms;
            c->t_calls[k] += 1;
            c->ev_free.push_back(pr.first);
            c->ev_free.push_back(pr.second);
        }
        c->ev[k].clear();
    }
    return NB_OK;
}

}  // namespace

extern "C" {

const char* nb_strerror(nb_status s) {
    switch (s) {
        case NB_OK: return "ok";
        case NB_ERR_ARG: return "invalid argument";
        case NB_ERR_BOX: return "invalid box (edges must be finite and above 2 * rlist)";
        case NB_ERR_NOMEM: return "out of memory";
        case NB_ERR_CAPACITY: return "list capacity exceeded";
        case NB_ERR_STATE: return "call out of order";
        case NB_ERR_HIP: return "HIP runtime error";
        case NB_ERR_NONFINITE: return "non-finite coordinates";
    }
    return "unknown status";
}

const char* nb_last_error(const nb_ctx* c) { return c ? c->err.c_str() : ""; }

nb_status nb_create(const nb_params* params, int32_t n_systems, const int64_t* atom_offsets,
                    void* hip_stream, nb_ctx** out) {
    if (!out) return NB_ERR_ARG;
    *out = nullptr;
    if (!params || !atom_offsets || n_systems < 1) return NB_ERR_ARG;
    const nb_params& p = *params;
    if (p.n_types < 1 || p.n_types > kMaxTypes) return NB_ERR_ARG;
    if (p.coulomb != NB_COUL_RF && p.coulomb != NB_COUL_EWALD && p.coulomb != NB_COUL_NONE)
        return NB_ERR_ARG;
    if (p.modifier != NB_MOD_NONE && p.modifier != NB_MOD_POTSHIFT) return NB_ERR_ARG;
    if (!finite_pos(p.rc) || !isfinite(p.rinner) || !isfinite(p.rlist)) return NB_ERR_ARG;
    if (p.rinner < p.rc || p.rlist < p.rinner) return NB_ERR_ARG;
    if (!finite_pos(p.eps_r) || !(p.eps_rf > 0.f) || isnan(p.eps_rf)) return NB_ERR_ARG;
    if (!isfinite(p.epsfac) || !isfinite(p.ewald_beta) || p.ewald_beta < 0.f) return NB_ERR_ARG;
    if (p.coulomb == NB_COUL_EWALD && !(p.ewald_beta > 0.f)) return NB_ERR_ARG;
    if (p.nstlist < 1 || p.nstprune < 1 || p.nstprune > 64) return NB_ERR_ARG;
    if (p.list_capacity_hint < 0 || p.list_capacity_hint > (1 << 20)) return NB_ERR_ARG;
    if (atom_offsets[0] != 0) return NB_ERR_ARG;
    for (int s = 0; s < n_systems; ++s)
        if (atom_offsets[s + 1] < atom_offsets[s]) return NB_ERR_ARG;
    if (atom_offsets[n_systems] > (int64_t)1 << 30) return NB_ERR_ARG;
    nb_ctx* c = new (std::nothrow) nb_ctx();
    if (!c) return NB_ERR_NOMEM;
    c->p = p;
    c->n_sys = n_systems;
    c->offs.assign(atom_offsets, atom_offsets + n_systems + 1);
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;   // resolved at first use
    c->d.n_atoms = (int32_t)c->offs[n_systems];
    c->d.n_sys = n_systems;
    c->d.n_types = p.n_types;
    c->cap = p.list_capacity_hint > 0 ? (int32_t)p.list_capacity_hint : 256;
    c->stats.n_atoms = c->d.n_atoms;
    c->hsys.resize(n_systems);
    *out = c;
    return NB_OK;
}

void nb_destroy(nb_ctx* c) {
    if (!c) return;
    if (c->d.flags) {
        hipSetDevice(c->device);
        hipStreamSynchronize(c->stream);
    }
    NbDev& d = c->d;
    void* ptrs[] = {d.chunks, d.sys_chunk_start, d.cpart, d.sc_ipos, d.type, d.atom_sys, d.excl_ptr, d.excl_idx, d.sys, d.sys_sc_start, d.img,
                    d.wpos, d.col_count, d.col_start, d.col_sc_start, d.col_cursor, d.col_atoms,
                    d.col_sorted, d.sc_info, d.slot_atom, d.atom_slot, d.type_slot, d.excl_slot,
                    d.cl_bb, d.sc_bb, d.xw, d.xq, d.xp, d.gslot, d.sc_ecount, d.sc_estart,
                    d.sc_istart, d.sc_icount, d.scratch, d.entries, d.entry_sc, d.items,
                    d.part_start, d.excl_rows, d.jseg_count, d.jseg_start, d.jseg_fill,
                    d.jseg_entries, d.totals, d.flags, d.jpart, d.ipart, d.epart, d.glj_part,
                    d.dstat, d.item_cost, d.item_order, d.queue, d.xcf, d.xce,
                    d.part_items, d.wave_e, d.wave_item, d.cl_xrange, d.slot_pre,
                    d.b_items, d.b_item_order, d.b_item_cost, d.b_sc_istart, d.b_sc_icount,
                    d.b_sc_ipos, d.b_part_items, d.b_part_start, d.b_totals};
    drop_graphs(c);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    for (void* q : ptrs)
        if (q) hipFree(q);
    for (void* q : {(void*)c->census_hist, (void*)c->census_part, (void*)c->census_total,
                    (void*)c->census_thr})
        if (q) hipFree(q);
    for (int k = 0; k < NB_T_COUNT; ++k)
        for (auto& pr : c->ev[k]) {
            hipEventDestroy(pr.first);
            hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : c->ev_free) hipEventDestroy(e);
    delete c;
}

nb_status nb_set_topology(nb_ctx* c, const int32_t* type, const int64_t* excl_ptr,
                          const int32_t* excl_idx) {
    if (!c) return NB_ERR_ARG;
    const int64_t n = c->d.n_atoms;
    if ((n > 0 && (!type || !excl_ptr)) || (excl_ptr && excl_ptr[0] != 0))
        return fail(c, NB_ERR_ARG, "topology arrays missing or excl_ptr[0] != 0");
    std::vector<int32_t> hsys(n), hptr(n + 1), hidx;
    int max_excl = 0;
    for (int s = 0; s < c->n_sys; ++s)
        for (int64_t a = c->offs[s]; a < c->offs[s + 1]; ++a) hsys[a] = s;
    for (int64_t a = 0; a < n; ++a) {
        if (type[a] < 0 || type[a] >= c->p.n_types)
            return fail(c, NB_ERR_ARG, "atom type out of range at atom " + std::to_string(a));
        if (excl_ptr[a + 1] < excl_ptr[a])
            return fail(c, NB_ERR_ARG, "exclusion row pointers decrease");
        const int64_t len = excl_ptr[a + 1] - excl_ptr[a];
        if (len > kMaxExcl) return fail(c, NB_ERR_ARG, "more than 32 exclusions for one atom");
        max_excl = std::max<int>(max_excl, (int)len);
        for (int64_t k = excl_ptr[a]; k < excl_ptr[a + 1]; ++k) {
            const int32_t b = excl_idx ? excl_idx[k] : -1;
            if (b < 0 || b >= n || hsys[b] != hsys[a])
                return fail(c, NB_ERR_ARG, "exclusion partner out of range or in another system");
        }
    }
    const int64_t nnz = n > 0 ? excl_ptr[n] : 0;
    if (nnz > INT32_MAX) return fail(c, NB_ERR_ARG, "too many exclusions");
    // The list is symmetric: b is a partner of a iff a is a partner of b (each side's
    // exclusion mask is built from its own row).  Self entries are ignored.
    for (int64_t a = 0; a < n; ++a)
        for (int64_t k = excl_ptr[a]; k < excl_ptr[a + 1]; ++k) {
            const int32_t b = excl_idx[k];
            for (int64_t m = excl_ptr[a]; m < k; ++m)
                if (excl_idx[m] == b)
                    return fail(c, NB_ERR_ARG, "exclusion partner " + std::to_string(b) +
                                                   " listed twice for atom " + std::to_string(a));
            if (b == a) continue;
            bool found = false;
            for (int64_t m = excl_ptr[b]; m < excl_ptr[b + 1] && !found; ++m)
                found = excl_idx[m] == a;
            if (!found)
                return fail(c, NB_ERR_ARG, "exclusions not symmetric: atom " +
                                               std::to_string(b) + " lacks partner " +
                                               std::to_string(a));
        }
    for (int64_t a = 0; a <= n; ++a) hptr[a] = n > 0 ? (int32_t)excl_ptr[a] : 0;
    NbDev& d = c->d;
    nb_status st = ensure_device(c);
    if (st != NB_OK) return st;
    NB_HIP(c, dev_alloc(d.type, n));
    NB_HIP(c, dev_alloc(d.atom_sys, n));
    NB_HIP(c, dev_alloc(d.excl_ptr, n + 1));
    NB_HIP(c, dev_alloc(d.excl_idx, nnz));
    if (n > 0) {
        NB_HIP(c, hipMemcpy(d.type, type, n * sizeof(int32_t), hipMemcpyHostToDevice));
        NB_HIP(c, hipMemcpy(d.atom_sys, hsys.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
        NB_HIP(c, hipMemcpy(d.excl_ptr, hptr.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
        if (nnz > 0)
            NB_HIP(c, hipMemcpy(d.excl_idx, excl_idx, nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    d.max_excl = max_excl;
    c->has_topology = true;
    c->has_grid = c->has_list = false;
    return NB_OK;
}

nb_status nb_grid_build(nb_ctx* c, const float* x, const float* box) {
    if (!c) return NB_ERR_ARG;
    if (!c->has_topology) return fail(c, NB_ERR_STATE, "nb_set_topology has not been called");
    if (!box || (c->d.n_atoms > 0 && !x)) return fail(c, NB_ERR_ARG, "null coordinates or box");
    const float rlist = c->p.rlist;
    int n_cols = 0;
    int64_t n_sc_max = 0;
    double max_edge = 0.0;
    for (int s = 0; s < c->n_sys; ++s) {
        NbSys S{};
        for (int k = 0; k < 3; ++k) {
            const float L = box[3 * s + k];
            if (!isfinite(L) || !(L > 2.0f * rlist))
                return fail(c, NB_ERR_BOX, "box edge " + std::to_string(k) + " of system " +
                                               std::to_string(s) + " not above 2 * rlist");
            if (L > 1000.0f) return fail(c, NB_ERR_BOX, "box edge above 1000 nm");
            max_edge = std::max(max_edge, (double)L);
            S.L[k] = L;
            S.invL[k] = (float)(1.0 / (double)L);
        }
        const int64_t na = c->offs[s + 1] - c->offs[s];
        int nx = 1, ny = 1;
        if (na > 0) {
            const double V = (double)S.L[0] * (double)S.L[1] * (double)S.L[2];
            const double size = cbrt(64.0 * V / (double)na);
            nx = std::max(1, (int)floor((double)S.L[0] / size + 0.5));
            ny = std::max(1, (int)floor((double)S.L[1] / size + 0.5));
        }
        if ((int64_t)nx * ny > (1 << 22)) return fail(c, NB_ERR_BOX, "grid too large");
        S.nx = nx;
        S.ny = ny;
        S.cinv[0] = (float)((double)nx / (double)S.L[0]);
        S.cinv[1] = (float)((double)ny / (double)S.L[1]);
        S.colw[0] = (float)((double)S.L[0] / nx);
        S.colw[1] = (float)((double)S.L[1] / ny);
        S.col_base = n_cols;
        S.atom0 = (int32_t)c->offs[s];
        S.atom1 = (int32_t)c->offs[s + 1];
        n_cols += nx * ny;
        n_sc_max += (na + kScAtoms - 1) / kScAtoms + (int64_t)nx * ny;
        c->hsys[s] = S;
    }
    if (n_sc_max * kScAtoms > INT32_MAX / 2) return fail(c, NB_ERR_ARG, "too many atoms");
    NbDev& d = c->d;
    NB_HIP(c, hipSetDevice(c->device));
    const size_t N = (size_t)d.n_atoms;
    if (N > c->a_atoms) {
        NB_HIP(c, dev_alloc(d.img, N));
        NB_HIP(c, dev_alloc(d.wpos, N));
        NB_HIP(c, dev_alloc(d.col_atoms, N));
        NB_HIP(c, dev_alloc(d.col_sorted, N));
        NB_HIP(c, dev_alloc(d.atom_slot, N));
        c->a_atoms = N;
    }
    if ((size_t)n_cols > c->a_cols || !d.col_count) {
        NB_HIP(c, dev_alloc(d.col_count, n_cols));
        NB_HIP(c, dev_alloc(d.col_start, n_cols + 1));
        NB_HIP(c, dev_alloc(d.col_sc_start, n_cols + 1));
        NB_HIP(c, dev_alloc(d.col_cursor, n_cols));
        c->a_cols = n_cols;
    }
    if ((size_t)n_sc_max > c->a_sc || !d.sc_info) {
        const size_t ns = (size_t)n_sc_max, slots = ns * kScAtoms, cl = ns * kClustersPerSc;
        NB_HIP(c, dev_alloc(d.sc_info, ns));
        NB_HIP(c, dev_alloc(d.slot_atom, slots));
        NB_HIP(c, dev_alloc(d.slot_pre, slots));
        NB_HIP(c, dev_alloc(d.type_slot, slots));
        NB_HIP(c, dev_alloc(d.cl_bb, 2 * cl));
        NB_HIP(c, dev_alloc(d.sc_bb, 2 * ns));
        NB_HIP(c, dev_alloc(d.xw, slots));
        NB_HIP(c, dev_alloc(d.xq, slots));
        NB_HIP(c, dev_alloc(d.xp, slots));
        NB_HIP(c, dev_alloc(d.gslot, slots));
        NB_HIP(c, dev_alloc(d.sc_ecount, ns));
        NB_HIP(c, dev_alloc(d.sc_estart, ns + 1));
        NB_HIP(c, dev_alloc(d.sc_istart, ns + 1));
        NB_HIP(c, dev_alloc(d.sc_icount, ns));
        NB_HIP(c, dev_alloc(d.sc_ipos, ns + 1));
        NB_HIP(c, dev_alloc(d.jseg_count, cl + 8));
        NB_HIP(c, dev_alloc(d.jseg_start, cl + 9));
        NB_HIP(c, dev_alloc(d.jseg_fill, cl + 8));
        NB_HIP(c, dev_alloc(d.xcf, slots));
        NB_HIP(c, dev_alloc(d.cl_xrange, cl));
        NB_HIP(c, dev_alloc(d.xce, 7 * ns));
        c->a_sc = ns;
        c->a_excl_nnz = 0;
    }
    if (c->a_excl_nnz < (size_t)n_sc_max * kScAtoms * std::max(1, d.max_excl) || !d.excl_slot) {
        const size_t ne = (size_t)n_sc_max * kScAtoms * std::max(1, d.max_excl);
        NB_HIP(c, dev_alloc(d.excl_slot, ne));
        c->a_excl_nnz = ne;
    }
    d.n_cols = n_cols;
    d.n_sc_max = (int32_t)n_sc_max;
    // Empty slots sit on a lattice below every box with this spacing: any two of them, or
    // one and a real atom, stay more than 2 rlist apart under every periodic shift.
    d.filler_d = (float)ceil(max_edge + 2.0 * rlist + 1.0);
    NB_HIP(c, hipMemcpyAsync(d.sys, c->hsys.data(), sizeof(NbSys) * c->n_sys,
                             hipMemcpyHostToDevice, c->stream));
    NB_HIP(c, launch_fill(d.flags, kFlagCount, 0, c->stream));
    NB_HIP(c, launch_grid_build(d, x, c->stream));
    c->has_grid = true;
    c->has_list = false;
    c->stats.grid_columns = n_cols;
    return NB_OK;
}

}  // extern "C"

namespace {

// Entries per work item: the width fixed by nb_set_exec / nb_autotune, else enough items
// to fill the device (about 8192), long lists split (Sec. V.F), between 8 and 64.
int item_width(const nb_ctx* c) {
    if (c->fixed_w > 0) return c->fixed_w;
    const int64_t target_items = 8192;
    return (int)std::min<int64_t>(64, std::max<int64_t>(8, (c->n_entries + target_items - 1) /
                                                               target_items));
}

// Item partition an execution mode runs on: 0 per super-cluster, 1 the balanced runs,
// 2 the queue mode's runs with their dynamic tail.
int items_kind_of(int exec_mode) {
    return exec_mode == kExecBalanced ? 1 : exec_mode == kExecQueue ? 2 : 0;
}

// Wavefronts of the balanced partition: those of the pair kernel's energy flavor resident
// on the whole device at once; in the queue mode also its dynamic runs (half as many,
// kQueueDynPerTwoWaves per two wavefronts), the two together within kMaxBalancedWaves.
nb_status balanced_waves(nb_ctx* c, int* waves, int* dyn) {
    int per_cu = 0;
    NB_HIP(c, prepare_forces(c->p.coulomb, NB_F_ENERGY, false, c->p.n_types, &per_cu));
    const bool queue = c->exec_mode == kExecQueue;
    const int limit = queue ? kMaxBalancedWaves * 2 / (2 + kQueueDynPerTwoWaves)
                            : kMaxBalancedWaves;
    *waves = std::min(limit, std::max(1, per_cu) * std::max(1, c->d.n_cu));
    *dyn = queue ? *waves * kQueueDynPerTwoWaves / 2 : 0;
    return NB_OK;
}

// Split the entries into items of at most W entries: per super-cluster (rolling-part major
// order), or in the balanced mode into equal-cost runs per wavefront; at a build also copy
// the entries out of the search scratch.
nb_status make_items(nb_ctx* c, int W, bool copy_entries) {
    NbDev& d = c->d;
    int waves = 0, dyn = 0;
    if (c->exec_mode == kExecBalanced || c->exec_mode == kExecQueue) {
        nb_status st = balanced_waves(c, &waves, &dyn);
        if (st != NB_OK) return st;
    }
    // per super-cluster ceil(n / W) items, plus at most one more per run boundary
    const size_t item_cap =
        (size_t)c->n_sc + (size_t)(c->n_entries / W) + 1 + (size_t)waves + (size_t)dyn;
    if (item_cap > c->a_items || !d.items) {
        const size_t ni = item_cap + item_cap / 8 + 64;
        NB_HIP(c, dev_alloc(d.items, ni));
        NB_HIP(c, dev_alloc(d.item_cost, ni));
        NB_HIP(c, dev_alloc(d.item_order, ni));
        NB_HIP(c, dev_alloc(d.ipart, ni * kScAtoms));
        NB_HIP(c, dev_alloc(d.epart, ni * kEpartStride));
        d.epart_stride = (int32_t)ni;
        NB_HIP(c, dev_alloc(d.glj_part, ni * (size_t)c->p.n_types * c->p.n_types * 2));
        NB_HIP(c, dev_alloc(d.part_items, ni));
        c->a_items = ni;
    }
    d.n_waves = waves;
    d.n_dyn = dyn;
    NB_HIP(c, launch_make_items(d, c->n_sc, c->cap, W, c->p.nstprune, copy_entries, waves,
                                dyn, kQueueStaticPermille, c->stream));
    c->item_w = W;
    c->items_kind = items_kind_of(c->exec_mode);
    return NB_OK;
}

// After make_items: item count, rolling-part ranges, the chunk tables of the two-stage
// per-system reductions and the queue order of the items.
nb_status finish_items(nb_ctx* c) {
    NbDev& d = c->d;
    // item totals, rolling-part ranges and per-system item ranks: one round trip
    c->part_start.resize(c->p.nstprune + 1);
    c->h_sss.resize(c->n_sys + 1);
    c->h_ipos.resize((size_t)c->n_sc + 1);
    NB_HIP(c, hipMemcpyAsync(c->h_totals, d.totals, sizeof(c->h_totals), hipMemcpyDeviceToHost,
                             c->stream));
    NB_HIP(c, hipMemcpyAsync(c->part_start.data(), d.part_start,
                             sizeof(int32_t) * c->part_start.size(), hipMemcpyDeviceToHost,
                             c->stream));
    NB_HIP(c, hipMemcpyAsync(c->h_sss.data(), d.sys_sc_start, sizeof(int32_t) * c->h_sss.size(),
                             hipMemcpyDeviceToHost, c->stream));
    NB_HIP(c, hipMemcpyAsync(c->h_ipos.data(), d.sc_ipos, sizeof(int32_t) * c->h_ipos.size(),
                             hipMemcpyDeviceToHost, c->stream));
    // entries per super-cluster, for the backward pass's item width (no round trip there)
    c->h_ecount.resize((size_t)c->n_sc);
    if (c->n_sc > 0)
        NB_HIP(c, hipMemcpyAsync(c->h_ecount.data(), d.sc_ecount, sizeof(int32_t) * c->n_sc,
                                 hipMemcpyDeviceToHost, c->stream));
    nb_status st = sync(c);
    if (st != NB_OK) return st;
    c->n_items = c->h_totals[1];
    // item ranks of system s are [sc_ipos[sys_sc_start[s]], sc_ipos[sys_sc_start[s+1]])
    std::vector<int4>& ch = c->h_chunks;
    std::vector<int32_t>& start = c->h_chunk_start;
    ch.clear();
    start.assign(c->n_sys + 1, 0);
    for (int s = 0; s < c->n_sys; ++s) {
        start[s] = (int32_t)ch.size();
        const int p0 = c->h_ipos[c->h_sss[s]], p1 = c->h_ipos[c->h_sss[s + 1]];
        for (int p = p0; p < p1; p += kChunkItems)
            ch.push_back(make_int4(s, p, std::min(p1, p + kChunkItems), 0));
    }
    start[c->n_sys] = (int32_t)ch.size();
    const size_t nglj = (size_t)(c->n_items + kChunkItems - 1) / kChunkItems;
    const size_t ncap = std::max(ch.size(), nglj) + 1;
    // the tables only grow: no free/allocate (and no implied device synchronisation) at a
    // rebuild of the same size
    if (ch.size() + 1 > c->a_chunks || !d.chunks) {
        const size_t n = ch.size() + ch.size() / 8 + 16;
        NB_HIP(c, dev_alloc(d.chunks, n));
        c->a_chunks = n;
    }
    if (!d.sys_chunk_start) NB_HIP(c, dev_alloc(d.sys_chunk_start, c->n_sys + 1));
    if (ncap > c->a_cpart || !d.cpart) {
        const size_t n = ncap + ncap / 8 + 16;
        NB_HIP(c, dev_alloc(d.cpart, n * kChunkVals));
        c->a_cpart = n;
    }
    // host tables live in the context until the next rebuild, after a synchronisation
    if (!ch.empty())
        NB_HIP(c, hipMemcpyAsync(d.chunks, ch.data(), ch.size() * sizeof(int4),
                                 hipMemcpyHostToDevice, c->stream));
    NB_HIP(c, hipMemcpyAsync(d.sys_chunk_start, start.data(), start.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
    d.n_chunks = (int32_t)ch.size();
    NB_HIP(c, launch_item_order(d, c->n_items, c->stream));
    c->stats.n_work_items = c->n_items;
    c->list_gen++;
    drop_graphs(c);
    return NB_OK;
}

}  // namespace

extern "C" {

nb_status nb_pairlist_build(nb_ctx* c) {
    if (!c) return NB_ERR_ARG;
    if (!c->has_grid) return fail(c, NB_ERR_STATE, "nb_grid_build has not been called");
    NB_HIP(c, hipSetDevice(c->device));
    NbDev& d = c->d;
    int32_t flags[kFlagCount];
    int32_t totals[8];
    nb_status st = NB_OK;
    const float r2o = radius_sq(c->p.rlist), r2i = radius_sq(c->p.rinner);
    // Search with the current per-super-cluster capacity over the bound on the super-cluster
    // count (the kernels read the grid build's own count), scan the entry counts, then one
    // round trip for the flags and the entry total; grow and repeat on overflow.
    const int n_sc_max = d.n_sc_max;
    for (int attempt = 0;; ++attempt) {
        const size_t need = (size_t)std::max(n_sc_max, 1) * c->cap * kSearchWaves;
        if (need > c->a_scratch) {
            NB_HIP(c, dev_alloc(d.scratch, need));
            c->a_scratch = need;
        }
        // clear the search's outputs; the grid build's count and non-finite flag stay
        NB_HIP(c, launch_fill(d.flags + kFlagScOverflow, 2, 0, c->stream));
        NB_HIP(c, launch_fill(d.flags + kFlagNumRows, kFlagCount - kFlagNumRows, 0, c->stream));
        NB_HIP(c, launch_search(d, n_sc_max, c->cap, r2o, r2i, c->p.rlist, c->stream));
        NB_HIP(c, launch_scan_entries(d, -1, c->stream));
        NB_HIP(c, hipMemcpyAsync(totals, d.totals, sizeof(totals), hipMemcpyDeviceToHost,
                                 c->stream));
        st = to_host(c, flags, d.flags, kFlagCount);   // synchronises: totals too
        if (st != NB_OK) return st;
        if (flags[kFlagNonFinite]) {
            c->has_grid = false;
            return fail(c, NB_ERR_NONFINITE,
                        "non-finite or out-of-range coordinates at grid build");
        }
        if (!flags[kFlagScOverflow]) break;
        if (c->p.list_capacity_hint > 0)
            return fail(c, NB_ERR_CAPACITY, "a super-cluster has " +
                                                std::to_string(flags[kFlagScNeeded]) +
                                                " entries, above list_capacity_hint");
        c->cap = flags[kFlagScNeeded] + flags[kFlagScNeeded] / 8 + 16;
        c->stats.regrows++;
        if (attempt > 4) return fail(c, NB_ERR_CAPACITY, "list capacity did not converge");
    }
    const int n_sc = flags[kFlagNumSc];
    c->n_sc = n_sc;
    c->n_cl = n_sc * kClustersPerSc;
    c->n_slots = n_sc * kScAtoms;
    c->stats.bb_pairs = (uint32_t)flags[kFlagBbPairs];
    const int64_t E = totals[0];
    c->n_entries = E;
    if ((size_t)E > c->a_entries || !d.entries) {
        const size_t ne = (size_t)E + E / 8 + 64;
        NB_HIP(c, dev_alloc(d.entries, ne));
        NB_HIP(c, dev_alloc(d.entry_sc, ne));
        NB_HIP(c, dev_alloc(d.excl_rows, ne * kClustersPerSc));
        NB_HIP(c, dev_alloc(d.jseg_entries, ne));
        NB_HIP(c, dev_alloc(d.jpart, ne * kClusterSize));
        c->a_entries = ne;
        d.entry_cap = (int64_t)ne;
    }
    st = make_items(c, item_width(c), true);
    if (st != NB_OK) return st;
    NB_HIP(c, launch_fill(d.totals + 2, 2, 0, c->stream));
    NB_HIP(c, launch_fill(d.flags + kFlagNumRows, 1, 0, c->stream));
    NB_HIP(c, launch_list_finish(d, n_sc, E, c->n_cl, c->stream));
    // read back with finish_items' round trip (it synchronises the stream)
    NB_HIP(c, hipMemcpyAsync(flags, d.flags, sizeof(flags), hipMemcpyDeviceToHost, c->stream));
    st = finish_items(c);
    if (st != NB_OK) return st;
    c->stats.outer_pairs = c->h_totals[2];
    c->stats.inner_pairs = c->h_totals[3];
    c->stats.n_slots = c->n_slots;
    c->stats.n_superclusters = n_sc;
    c->stats.n_clusters = c->n_cl;
    c->stats.n_entries = E;
    c->stats.n_excl_rows = flags[kFlagNumRows];
    c->stats.capacity_per_sc = c->cap;
    c->has_list = true;
    return NB_OK;
}

nb_status nb_prune_rolling(nb_ctx* c, const float* x, int64_t steps_since_build) {
    if (!c) return NB_ERR_ARG;
    if (!c->has_list) return fail(c, NB_ERR_STATE, "no pair list");
    if (steps_since_build < 0) return fail(c, NB_ERR_ARG, "negative step");
    if (steps_since_build >= c->p.nstlist)
        return fail(c, NB_ERR_STATE, "the outer list has expired (steps_since_build >= nstlist)");
    if (steps_since_build == 0) return NB_OK;
    if (!x && c->d.n_atoms > 0) return fail(c, NB_ERR_ARG, "null coordinates");
    NB_HIP(c, hipSetDevice(c->device));
    const int part = (int)(steps_since_build % c->p.nstprune);
    const int i0 = c->part_start[part], i1 = c->part_start[part + 1];
    TimedSection ts(c, NB_T_PRUNE);
    NB_HIP(c, launch_gather(c->d, x, nullptr, c->d.xp, c->n_slots, c->stream));
    NB_HIP(c, launch_prune(c->d, c->d.xp, i0, i1 - i0, radius_sq(c->p.rinner), c->prune_waves,
                           c->stream));
    return NB_OK;
}

namespace {
constexpr uint32_t kForceFlags = NB_F_ENERGY | NB_F_VIRIAL | NB_F_ACCUMULATE | NB_F_EXCL_CORR;

// prune_part >= 0: re-prune that rolling part with x before the pair kernel (inside it when
// the prune is fused); ahead_part >= 0: after the pair kernel, re-prune that part with x in
// the force reduction's launch.
nb_status forces_impl(nb_ctx* c, const float* x, const float* q, const float* lj, float* f,
                      double* energy, double* virial, uint32_t flags, int prune_part,
                      int ahead_part = -1) {
    if (flags & ~kForceFlags) return fail(c, NB_ERR_ARG, "unknown flag");
    if (c->d.n_atoms > 0 && (!x || !q || !lj || !f)) return fail(c, NB_ERR_ARG, "null array");
    if ((flags & NB_F_ENERGY) && !energy) return fail(c, NB_ERR_ARG, "energy output missing");
    if ((flags & NB_F_VIRIAL) && !virial) return fail(c, NB_ERR_ARG, "virial output missing");
    NB_HIP(c, hipSetDevice(c->device));
    NbDev& d = c->d;
    const NbKParams kp = kernel_params(c->p);
    const bool fused = prune_part >= 0 && c->prune_mode == kPruneFused;
    {
        TimedSection ts(c, NB_T_FORCE_REDUCE);
        NB_HIP(c, launch_gather(d, x, q, d.xq, c->n_slots, c->stream));
    }
    if (prune_part >= 0 && !fused) {
        // the rolling prune of the part as its own kernel on the gathered coordinates,
        // then the plain pair kernel
        const int i0 = c->part_start[prune_part], i1 = c->part_start[prune_part + 1];
        TimedSection ts(c, NB_T_PRUNE);
        NB_HIP(c, launch_prune(d, d.xq, i0, i1 - i0, radius_sq(c->p.rinner), c->prune_waves,
                               c->stream));
    }
    {
        TimedSection ts(c, NB_T_FORCES);
        NB_HIP(c, launch_forces(d, kp, c->p.coulomb, flags, lj, c->n_items,
                                fused ? prune_part : -1, c->p.nstprune,
                                radius_sq(c->p.rinner), c->exec_mode, c->stream));
    }
    // The ahead prune (the paper's rolling schedule: the next step's part is pruned between
    // force computations, Sec. V.E) runs in the force reduction's launch, beside its blocks.
    // Exclusion corrections (a kernel of their own over the excluded pairs; the pair
    // kernel above is the same with or without them)
    const bool corr = (flags & NB_F_EXCL_CORR) && c->p.coulomb != NB_COUL_NONE;
    TimedSection ts(c, NB_T_FORCE_REDUCE);
    if (corr) {
        double krf, crf;
        rf_constants(c->p, &krf, &crf);
        NB_HIP(c, launch_excl_corr(d, kp, c->p.coulomb, krf, crf, c->n_sc, d.xcf, d.xce,
                                   c->stream));
    }
    NB_HIP(c, launch_reduce(d, f, (flags & NB_F_ACCUMULATE) != 0, c->n_slots, energy, virial,
                            flags, c->n_sys, corr ? d.xcf : nullptr, ahead_part,
                            c->p.nstprune, ahead_part >= 0 ? c->part_start[ahead_part] : 0,
                            ahead_part >= 0 ? c->part_start[ahead_part + 1] -
                                                  c->part_start[ahead_part]
                                            : 0,
                            radius_sq(c->p.rinner), c->stream));
    if (corr) NB_HIP(c, launch_excl_energy(d, d.xce, energy, virial, flags, c->n_sys, c->stream));
    return NB_OK;
}
}  // namespace

nb_status nb_forces(nb_ctx* c, const float* x, const float* q, const float* lj, float* f,
                    double* energy, double* virial, uint32_t flags) {
    if (!c) return NB_ERR_ARG;
    if (!c->has_list) return fail(c, NB_ERR_STATE, "no pair list");
    return forces_impl(c, x, q, lj, f, energy, virial, flags, -1);
}

namespace {
// Rolling parts of nb_step at steps_since_build s (-1: none): with the prune before or
// inside the pair kernel, part s mod nstprune with this step's positions (none at s = 0,
// the build's prune); with the ahead prune, after the pair kernel, part (s + 1) mod
// nstprune for the next step (none when s + 1 = nstlist, a build step).
nb_status step_part(nb_ctx* c, int64_t steps_since_build, int* part, int* ahead) {
    if (!c->has_list) return fail(c, NB_ERR_STATE, "no pair list");
    if (steps_since_build < 0) return fail(c, NB_ERR_ARG, "negative step");
    if (steps_since_build >= c->p.nstlist)
        return fail(c, NB_ERR_STATE, "the outer list has expired (steps_since_build >= nstlist)");
    *part = -1;
    *ahead = -1;
    if (c->prune_mode == kPruneAhead) {
        if (steps_since_build + 1 < c->p.nstlist)
            *ahead = (int)((steps_since_build + 1) % c->p.nstprune);
    } else if (steps_since_build > 0) {
        *part = (int)(steps_since_build % c->p.nstprune);
    }
    return NB_OK;
}
}  // namespace

nb_status nb_step(nb_ctx* c, const float* x, const float* q, const float* lj, float* f,
                  double* energy, double* virial, uint32_t flags, int64_t steps_since_build) {
    if (!c) return NB_ERR_ARG;
    int part = -1, ahead = -1;
    nb_status st = step_part(c, steps_since_build, &part, &ahead);
    if (st != NB_OK) return st;
    return forces_impl(c, x, q, lj, f, energy, virial, flags, part, ahead);
}

nb_status nb_step_graph(nb_ctx* c, const float* x, const float* q, const float* lj, float* f,
                        double* energy, double* virial, uint32_t flags,
                        int64_t steps_since_build) {
    if (!c) return NB_ERR_ARG;
    int part = -1, ahead = -1;
    nb_status st = step_part(c, steps_since_build, &part, &ahead);
    if (st != NB_OK) return st;
    if (flags & ~kForceFlags) return fail(c, NB_ERR_ARG, "unknown flag");
    NB_HIP(c, hipSetDevice(c->device));
    const void* key[7] = {x, q, lj, f, energy, virial, nullptr};
    for (auto& g : c->graphs)
        if (g.part == part && g.ahead == ahead && g.flags == flags && g.gen == c->list_gen &&
            std::equal(key, key + 7, g.ptr)) {
            NB_HIP(c, hipGraphLaunch(g.exec, c->stream));
            return NB_OK;
        }
    // Capture the step's launches on a private stream (nothing runs during capture),
    // without timing events, then replay the instantiated graph on the context's stream.
    if (!c->cap_stream) NB_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    NB_HIP(c, prepare_forces(c->p.coulomb, flags, part >= 0, c->p.n_types));
    const hipStream_t user = c->stream;
    const bool timing = c->timing;
    c->stream = c->cap_stream;
    c->timing = false;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) st = forces_impl(c, x, q, lj, f, energy, virial, flags, part, ahead);
    hipGraph_t graph = nullptr;
    const hipError_t e_end = (e == hipSuccess) ? hipStreamEndCapture(c->cap_stream, &graph) : e;
    c->stream = user;
    c->timing = timing;
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
    if (st != NB_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e_end != hipSuccess) return hip_fail(c, e_end, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
    // one graph per rolling part and flag set is the steady state; bound the cache
    const size_t max_graphs = (size_t)c->p.nstprune + 4;
    if (c->graphs.size() >= max_graphs) {
        hipGraphExecDestroy(c->graphs.front().exec);
        c->graphs.erase(c->graphs.begin());
    }
    nb_ctx::GraphEntry g{};
    g.part = part;
    g.ahead = ahead;
    g.flags = flags;
    std::copy(key, key + 7, g.ptr);
    g.gen = c->list_gen;
    g.exec = exec;
    c->graphs.push_back(g);
    NB_HIP(c, hipGraphLaunch(exec, c->stream));
    return NB_OK;
}

nb_status nb_set_exec(nb_ctx* c, int32_t width, int32_t exec_mode, int32_t prune_fused,
                      int32_t prune_waves) {
    if (!c) return NB_ERR_ARG;
    if (width < 0 || width > 64) return fail(c, NB_ERR_ARG, "item width must be 0 (rule) or 1..64");
    if (exec_mode != kExecStatic && exec_mode != kExecXcd && exec_mode != kExecQueue &&
        exec_mode != kExecPersist && exec_mode != kExecBalanced)
        return fail(c, NB_ERR_ARG, "unknown execution mode");
    if (prune_fused != kPruneSeparate && prune_fused != kPruneFused && prune_fused != kPruneAhead)
        return fail(c, NB_ERR_ARG, "prune_fused is 0, 1 or 2");
    if (prune_waves != 0 && prune_waves != 1 && prune_waves != 2 && prune_waves != 4 &&
        prune_waves != 8)
        return fail(c, NB_ERR_ARG, "prune_waves is 0, 1, 2, 4 or 8");
    c->fixed_w = width;
    c->prune_waves = prune_waves;
    c->exec_mode = exec_mode;
    c->prune_mode = prune_fused;
    c->list_gen++;
    if (c->d.flags) {
        NB_HIP(c, hipSetDevice(c->device));
        drop_graphs(c);
    }
    if (c->has_list && (item_width(c) != c->item_w ||
                        c->items_kind != items_kind_of(exec_mode))) {
        nb_status st = make_items(c, item_width(c), false);
        if (st != NB_OK) return st;
        return finish_items(c);
    }
    return NB_OK;
}

nb_status nb_get_exec(nb_ctx* c, nb_exec_config* out) {
    if (!c || !out) return NB_ERR_ARG;
    out->item_width = c->has_list ? c->item_w : c->fixed_w;
    out->exec_mode = c->exec_mode;
    out->prune_fused = c->prune_mode;
    out->prune_waves = c->prune_waves;
    out->us_per_call = 0.0;
    return NB_OK;
}

nb_status nb_autotune(nb_ctx* c, const float* x, const float* q, const float* lj,
                      uint32_t flags, int32_t repeats, nb_exec_config* trials, int32_t cap,
                      int32_t* n_trials, nb_exec_config* best) {
    if (!c) return NB_ERR_ARG;
    if (!c->has_list) return fail(c, NB_ERR_STATE, "no pair list");
    if (flags & ~(uint32_t)(NB_F_ENERGY | NB_F_VIRIAL))
        return fail(c, NB_ERR_ARG, "autotune flags: NB_F_ENERGY and NB_F_VIRIAL only");
    if (repeats < 1 || repeats > 1000) return fail(c, NB_ERR_ARG, "repeats out of range");
    if (cap < 0 || (cap > 0 && !trials)) return fail(c, NB_ERR_ARG, "trial buffer");
    if (c->d.n_atoms > 0 && (!x || !q || !lj)) return fail(c, NB_ERR_ARG, "null array");
    NB_HIP(c, hipSetDevice(c->device));
    // outputs of the timed calls live in buffers of this call
    float* f = nullptr;
    double* ev = nullptr;
    NB_HIP(c, dev_alloc(f, (size_t)c->d.n_atoms * 3));
    hipError_t e = dev_alloc(ev, (size_t)c->n_sys * 11);
    if (e != hipSuccess) {
        hipFree(f);
        return hip_fail(c, e, "autotune buffers");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    const bool timing = c->timing;
    c->timing = false;
    const int widths[] = {8, 16, 24, 32, 40, 48, 56, 64};
    const int modes[] = {kExecStatic, kExecXcd, kExecQueue, kExecPersist, kExecBalanced};
    nb_exec_config win{0, 0, 1, 0, 1e300}, second{0, 0, 1, 0, 1e300};
    // the two fastest shapes (item width and mode), distinct
    auto keep_best = [&](const nb_exec_config& t) {
        const bool same_win = t.item_width == win.item_width && t.exec_mode == win.exec_mode;
        if (t.us_per_call < win.us_per_call) {
            if (!same_win) second = win;
            win = t;
        } else if (!same_win && t.us_per_call < second.us_per_call) {
            second = t;
        }
    };
    int n = 0;
    nb_status st = NB_OK;
    // median time of `repeats` calls after a warm-up; part < 0: forces only, else a step
    // that also re-prunes that rolling part (valid with any current positions), before or
    // inside the pair kernel, or after it beside the reduction with the ahead prune
    auto time_calls = [&](int part, double* us) {
        std::vector<float> ms;
        const bool ahead = part >= 0 && c->prune_mode == kPruneAhead;
        for (int r = 0; r <= repeats && st == NB_OK; ++r) {
            hipEventRecord(e0, c->stream);
            st = forces_impl(c, x, q, lj, f, ev, ev + 2 * c->n_sys, flags, ahead ? -1 : part,
                             ahead ? part : -1);
            hipEventRecord(e1, c->stream);
            if (st == NB_OK && hipEventSynchronize(e1) != hipSuccess)
                st = fail(c, NB_ERR_HIP, "autotune event");
            float t = 0.f;
            if (st == NB_OK && r > 0 && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
                ms.push_back(t);
        }
        if (st != NB_OK || ms.empty()) return false;
        std::sort(ms.begin(), ms.end());
        *us = 1e3 * ms[ms.size() / 2];
        return true;
    };
    const int prune0 = c->prune_mode;
    for (int W : widths) {
        if (st != NB_OK) break;
        c->exec_mode = kExecStatic;
        st = make_items(c, W, false);
        if (st == NB_OK) st = finish_items(c);
        for (int m : modes) {
            if (st != NB_OK) break;
            c->exec_mode = m;
            if (c->items_kind != items_kind_of(m)) {   // the balanced and queue runs
                st = make_items(c, W, false);
                if (st == NB_OK) st = finish_items(c);
                if (st != NB_OK) break;
            }
            double us = 0.0;
            if (!time_calls(-1, &us)) break;
            const nb_exec_config t{W, m, prune0, c->prune_waves, us};
            if (n < cap) trials[n] = t;
            ++n;
            keep_best(t);
        }
    }
    // One more shape: the persistent round-robin schedule at the smallest width whose
    // items all fit the resident grid in one round (per super-cluster ceil(n / W) items):
    // every wavefront then takes one item and the grid has no partial round of blocks.
    // The widths above straddle that count (measured at 96k: 7094 items of at most 36
    // entries on 7168 resident wavefronts, 82 us, against 84.6 at 40 entries).
    if (st == NB_OK) {
        int per_cu = 0;
        hipError_t he = prepare_forces(c->p.coulomb, flags, false, c->p.n_types, &per_cu);
        if (he != hipSuccess) st = hip_fail(c, he, "autotune occupancy");
        const std::vector<int32_t>& cnt = c->h_ecount;
        if (st == NB_OK) {
            const int64_t G = (int64_t)std::max(1, per_cu) * std::max(1, c->d.n_cu);
            int wfit = widths[sizeof(widths) / sizeof(widths[0]) - 1];
            for (int w = widths[0]; w < wfit; ++w) {
                int64_t items = 0;
                for (int32_t k : cnt) items += (k + w - 1) / w;
                if (items <= G) {
                    wfit = w;
                    break;
                }
            }
            c->exec_mode = kExecPersist;
            st = make_items(c, wfit, false);
            if (st == NB_OK) st = finish_items(c);
            double us = 0.0;
            if (st == NB_OK && time_calls(-1, &us)) {
                const nb_exec_config t{wfit, kExecPersist, prune0, c->prune_waves, us};
                if (n < cap) trials[n] = t;
                ++n;
                keep_best(t);
            }
        }
    }
    // Then, for the two fastest shapes, a rolling step with the prune fused into the pair
    // kernel, as its own kernel before it and as its own kernel after it beside the
    // reduction; the step time decides shape and placement together (at 96k two widths
    // tie on the pair kernel, 36 and 40 entries, while the ahead prune's share of the
    // reduction launch differs by 1.3 us between them).
    if (st == NB_OK) {
        const nb_exec_config shapes[2] = {win, second.us_per_call < 1e299 ? second : win};
        double best_step = 1e300;
        nb_exec_config chosen = win;
        for (int k = 0; k < 2 && st == NB_OK; ++k) {
            const nb_exec_config& sh = shapes[k];
            c->exec_mode = sh.exec_mode;
            st = make_items(c, sh.item_width, false);
            if (st == NB_OK) st = finish_items(c);
            for (int pf : {kPruneFused, kPruneSeparate, kPruneAhead}) {
                if (st != NB_OK) break;
                c->prune_mode = pf;
                double us = 0.0;
                if (!time_calls(c->p.nstprune > 1 ? 1 : 0, &us)) break;
                const nb_exec_config t{sh.item_width, sh.exec_mode, pf, c->prune_waves, us};
                if (n < cap) trials[n] = t;
                ++n;
                if (us < best_step) {
                    best_step = us;
                    chosen = sh;
                    chosen.prune_fused = pf;
                }
            }
        }
        win = chosen;
    }
    c->timing = timing;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(f);
    hipFree(ev);
    if (st != NB_OK) return st;
    if (n_trials) *n_trials = n;
    c->fixed_w = win.item_width;
    c->exec_mode = win.exec_mode;
    c->prune_mode = win.prune_fused;
    st = finish_items(c);          // fresh item order and no graphs of the timing calls
    if (st != NB_OK) return st;
    if (best) *best = win;
    return NB_OK;
}

namespace {
// Items of the backward pass.  Its kernel holds fewer wavefronts per SIMD than the forward
// kernel (more registers per pair), so the forward items can take it two rounds, the
// second partial; it takes per-super-cluster items of the smallest width, not below the
// forward items', whose items all fit its resident grid in one round (at 96k atoms 52
// entries against the forward's 36: 171 -> 144 us), or the forward items themselves when
// that is their width.  The width is chosen on the host from the entry counts the list
// build brought back; the items are built once per list generation and flavor, on the
// device (no wait), into arrays of their own; an item count never above the forward's,
// so the per-item partial buffers fit.
nb_status backward_items(nb_ctx* c, bool ljgrad, NbDev* db, int* n_items) {
    NbDev& d = c->d;
    const int flavor = ljgrad ? 1 : 0;
    if (c->bwd_gen != c->list_gen || c->bwd_flavor != flavor) {
        const int per_cu = backward_waves_per_cu(c->p.coulomb, ljgrad, c->p.n_types);
        const int64_t G = (int64_t)std::max(1, per_cu) * std::max(1, d.n_cu);
        const std::vector<int32_t>& cnt = c->h_ecount;
        auto items_at = [&](int w) {
            int64_t n = 0;
            for (int32_t k : cnt) n += (k + w - 1) / w;
            return n;
        };
        const int w0 = std::max(1, std::min(c->item_w, 64));
        int wb = 64;
        for (int w = w0; w < 64; ++w)
            if (items_at(w) <= G) {
                wb = w;
                break;
            }
        const bool own = !(wb == c->item_w && c->items_kind == 0);
        const int nb = (int)items_at(wb);
        if (own) {
            const size_t need = (size_t)nb + 64, nsc = (size_t)std::max(d.n_sc_max, 1) + 1;
            if (need > c->a_bitems || !d.b_items) {
                NB_HIP(c, dev_alloc(d.b_items, need));
                NB_HIP(c, dev_alloc(d.b_item_order, need));
                NB_HIP(c, dev_alloc(d.b_item_cost, need));
                NB_HIP(c, dev_alloc(d.b_part_items, need));
                c->a_bitems = need;
            }
            if (nsc > c->a_bsc || !d.b_sc_istart) {
                NB_HIP(c, dev_alloc(d.b_sc_istart, nsc));
                NB_HIP(c, dev_alloc(d.b_sc_icount, nsc));
                NB_HIP(c, dev_alloc(d.b_sc_ipos, nsc));
                c->a_bsc = nsc;
            }
            if (!d.b_part_start) NB_HIP(c, dev_alloc(d.b_part_start, c->p.nstprune + 1));
            if (!d.b_totals) NB_HIP(c, dev_alloc(d.b_totals, 8));
            NB_HIP(c, hipMemcpyAsync(d.b_totals, d.totals, 8 * sizeof(int32_t),
                                     hipMemcpyDeviceToDevice, c->stream));
        }
        c->bwd_gen = c->list_gen;
        c->bwd_flavor = flavor;
        c->bwd_w = wb;
        c->bwd_n = own ? nb : c->n_items;
        c->bwd_own = own;
        if (own) {
            NbDev t = d;
            t.items = d.b_items;
            t.item_order = d.b_item_order;
            t.item_cost = d.b_item_cost;
            t.sc_istart = d.b_sc_istart;
            t.sc_icount = d.b_sc_icount;
            t.sc_ipos = d.b_sc_ipos;
            t.part_items = d.b_part_items;
            t.part_start = d.b_part_start;
            t.totals = d.b_totals;
            NB_HIP(c, launch_make_items(t, c->n_sc, c->cap, wb, c->p.nstprune, false, 0, 0,
                                        kQueueStaticPermille, c->stream));
            NB_HIP(c, launch_item_order(t, nb, c->stream));
        }
    }
    *db = d;
    if (c->bwd_own) {
        db->items = d.b_items;
        db->item_order = d.b_item_order;
        db->item_cost = d.b_item_cost;
        db->sc_istart = d.b_sc_istart;
        db->sc_icount = d.b_sc_icount;
        db->sc_ipos = d.b_sc_ipos;
        db->part_items = d.b_part_items;
        db->part_start = d.b_part_start;
        db->totals = d.b_totals;
    }
    *n_items = c->bwd_n;
    return NB_OK;
}
}  // namespace

nb_status nb_forces_backward(nb_ctx* c, const float* x, const float* q, const float* lj,
                             const float* grad_f, const double* grad_energy, float* grad_x,
                             float* grad_q, double* grad_lj, uint32_t flags) {
    if (!c) return NB_ERR_ARG;
    if (!c->has_list) return fail(c, NB_ERR_STATE, "no pair list");
    if (flags & ~(uint32_t)NB_F_ACCUMULATE) return fail(c, NB_ERR_ARG, "unknown flag");
    if (c->d.n_atoms > 0 && (!x || !q || !lj || !grad_f))
        return fail(c, NB_ERR_ARG, "null array");
    NB_HIP(c, hipSetDevice(c->device));
    const NbKParams kp = kernel_params(c->p);
    const bool acc = (flags & NB_F_ACCUMULATE) != 0;
    NbDev d;
    int n_items = 0;
    nb_status st = backward_items(c, grad_lj != nullptr, &d, &n_items);
    if (st != NB_OK) return st;
    {
        TimedSection ts(c, NB_T_BACKWARD_REDUCE);
        NB_HIP(c, launch_gather(d, x, q, d.xq, c->n_slots, c->stream));
    }
    {
        TimedSection ts(c, NB_T_BACKWARD);
        NB_HIP(c, launch_backward(d, kp, c->p.coulomb, lj, grad_f, grad_energy, grad_lj != nullptr,
                                  c->n_slots, n_items, c->exec_mode, c->stream));
    }
    TimedSection ts(c, NB_T_BACKWARD_REDUCE);
    NB_HIP(c, launch_reduce_backward(d, grad_x, grad_q, grad_lj, acc, c->n_slots, c->p.n_types,
                                     n_items, c->stream));
    return NB_OK;
}

nb_status nb_get_grid(nb_ctx* c, int32_t* slot_atom, int64_t cap, int64_t* n_slots) {
    if (!c || !n_slots) return NB_ERR_ARG;
    if (!c->has_grid) return fail(c, NB_ERR_STATE, "no grid");
    NB_HIP(c, hipSetDevice(c->device));
    int32_t ns = 0;
    nb_status st = to_host(c, &ns, c->d.flags + kFlagNumSc, 1);
    if (st != NB_OK) return st;
    *n_slots = (int64_t)ns * kScAtoms;
    if (!slot_atom || cap < *n_slots) return NB_OK;
    return to_host(c, slot_atom, c->d.slot_atom, (size_t)*n_slots);
}

nb_status nb_get_grid_dims(nb_ctx* c, int32_t* dims) {
    if (!c || !dims) return NB_ERR_ARG;
    if (!c->has_grid) return fail(c, NB_ERR_STATE, "no grid");
    for (int s = 0; s < c->n_sys; ++s) {
        dims[2 * s] = c->hsys[s].nx;
        dims[2 * s + 1] = c->hsys[s].ny;
    }
    return NB_OK;
}

namespace {
// Cluster pairs passing the bounding-box tests of the search, recomputed on the grid of the
// current list by the search kernel in its recording mode (same kernel, same inputs).
nb_status get_bb_pairs(nb_ctx* c, int32_t* triples, int64_t cap, int64_t* count) {
    NbDev& d = c->d;
    const int rec_cap = (int)std::min<int64_t>(INT32_MAX / 2, std::max<int64_t>(1, c->stats.bb_pairs));
    NB_HIP(c, dev_alloc(d.bb_rec, (size_t)rec_cap));
    nb_status st = NB_OK;
    std::vector<int4> rec;
    int32_t n_rec = 0;
    hipError_t e = launch_fill(d.flags + kFlagBbRecords, 1, 0, c->stream);
    if (e == hipSuccess)
        e = launch_search_record(d, c->n_sc, radius_sq(c->p.rlist), c->p.rlist, rec_cap,
                                 c->stream);
    if (e != hipSuccess) st = hip_fail(c, e, "bounding-box search");
    if (st == NB_OK) st = to_host(c, &n_rec, d.flags + kFlagBbRecords, 1);
    if (st == NB_OK && n_rec > rec_cap)
        st = fail(c, NB_ERR_HIP, "bounding-box records exceed the build's count");
    if (st == NB_OK) {
        rec.resize((size_t)n_rec);
        st = to_host(c, rec.data(), d.bb_rec, rec.size());
    }
    hipFree(d.bb_rec);
    d.bb_rec = nullptr;
    if (st != NB_OK) return st;
    // records are written in completion order: sort them for a deterministic output
    std::sort(rec.begin(), rec.end(), [](const int4& a, const int4& b) {
        if (a.x != b.x) return a.x < b.x;
        if (a.y != b.y) return a.y < b.y;
        return a.z < b.z;
    });
    int64_t n = 0;
    for (const int4& r : rec) n += __builtin_popcount((uint32_t)r.w);
    *count = n;
    if (!triples || cap < n) return NB_OK;
    int64_t k = 0;
    for (const int4& r : rec)
        for (int b = 0; b < 8; ++b)
            if ((r.w >> b) & 1) {
                triples[3 * k] = r.x * kClustersPerSc + b;
                triples[3 * k + 1] = r.y;
                triples[3 * k + 2] = r.z;
                ++k;
            }
    return NB_OK;
}
}  // namespace

nb_status nb_get_pairs(nb_ctx* c, int32_t which, int32_t* triples, int64_t cap, int64_t* count) {
    if (!c || !count || which < 0 || which > 2) return NB_ERR_ARG;
    if (!c->has_list) return fail(c, NB_ERR_STATE, "no pair list");
    NB_HIP(c, hipSetDevice(c->device));
    if (which == 0) return get_bb_pairs(c, triples, cap, count);
    const size_t E = (size_t)c->n_entries;
    std::vector<NbEntry> ent(E);
    std::vector<int32_t> esc(E);
    nb_status st = to_host(c, ent.data(), c->d.entries, E);
    if (st != NB_OK) return st;
    st = to_host(c, esc.data(), c->d.entry_sc, E);
    if (st != NB_OK) return st;
    const int sh = which == 1 ? 8 : 16;
    int64_t n = 0;
    for (size_t e = 0; e < E; ++e) n += __builtin_popcount((ent[e].meta >> sh) & 0xffu);
    *count = n;
    if (!triples || cap < n) return NB_OK;
    int64_t k = 0;
    for (size_t e = 0; e < E; ++e) {
        const uint32_t m = (ent[e].meta >> sh) & 0xffu;
        for (int b = 0; b < 8; ++b)
            if ((m >> b) & 1u) {
                triples[3 * k] = esc[e] * kClustersPerSc + b;
                triples[3 * k + 1] = ent[e].cj;
                triples[3 * k + 2] = (int32_t)(ent[e].meta & 31u);
                ++k;
            }
    }
    return NB_OK;
}

nb_status nb_set_timing(nb_ctx* c, int32_t enable) {
    if (!c) return NB_ERR_ARG;
    if (c->d.flags) {
        nb_status st = collect_timing(c);
        if (st != NB_OK) return st;
    }
    for (int k = 0; k < NB_T_COUNT; ++k) {
        c->t_ms[k] = 0;
        c->t_calls[k] = 0;
    }
    c->timing = enable != 0;
    return NB_OK;
}

nb_status nb_get_timing(nb_ctx* c, double* ms, int64_t* calls) {
    if (!c || !ms || !calls) return NB_ERR_ARG;
    if (c->d.flags) {
        NB_HIP(c, hipSetDevice(c->device));
        nb_status st = collect_timing(c);
        if (st != NB_OK) return st;
    }
    for (int k = 0; k < NB_T_COUNT; ++k) {
        ms[k] = c->t_ms[k];
        calls[k] = c->t_calls[k];
        c->t_ms[k] = 0;
        c->t_calls[k] = 0;
    }
    return NB_OK;
}

namespace {

// Device buffers of one census walk: block histograms of up to max_blocks blocks, their
// chunk sums, the summed words and the thresholds.
struct CensusBufs {
    uint32_t* hist;
    unsigned long long* part;
    unsigned long long* total;
    float* thr;
    int max_blocks;
    bool thr_by_kernel;   // write the thresholds with a kernel argument (no copy) and
                          // record no timing events
};

// One census or coverage walk of the outer list: validates the radii, sorts them (ord maps a
// sorted position to the caller's index) and returns the summed histogram words in tot
// (census_words(cover) words).  Uses no heap memory of its own.
nb_status census_walk(nb_ctx* c, int32_t n_radii, const float* radii, bool cover, int ca,
                      int cb, const CensusBufs& b, int* ord, unsigned long long* tot) {
    float r2[NB_CENSUS_MAX_RADII];
    for (int k = 0; k < n_radii; ++k) r2[k] = radius_sq(radii[k]);
    // stable insertion sort of at most NB_CENSUS_MAX_RADII radii
    for (int k = 0; k < n_radii; ++k) {
        int p = k;
        while (p > 0 && r2[ord[p - 1]] > r2[k]) {
            ord[p] = ord[p - 1];
            --p;
        }
        ord[p] = k;
    }
    float r2s[NB_CENSUS_MAX_RADII];
    for (int k = 0; k < NB_CENSUS_MAX_RADII; ++k)
        r2s[k] = k < n_radii ? r2[ord[k]] : __builtin_inff();   // +inf padding
    const int n_items = c->n_items;
    const int nb = std::min(census_blocks(n_items, cover), b.max_blocks);
    if (b.thr_by_kernel)
        NB_HIP(c, launch_set_thresholds(r2s, b.thr, c->stream));
    else
        NB_HIP(c, hipMemcpyAsync(b.thr, r2s, sizeof(r2s), hipMemcpyHostToDevice, c->stream));
    if (b.thr_by_kernel) {
        NB_HIP(c, launch_census(c->d, n_items, b.thr, n_radii, cover, ca, cb, b.hist, nb,
                                c->stream));
    } else {
        TimedSection ts(c, NB_T_CENSUS);
        NB_HIP(c, launch_census(c->d, n_items, b.thr, n_radii, cover, ca, cb, b.hist, nb,
                                c->stream));
    }
    NB_HIP(c, launch_census_sum(b.hist, nb, cover, b.part, b.total, c->stream));
    return to_host(c, tot, b.total, census_words(cover));
}

nb_status census_check(nb_ctx* c, int32_t n_radii, const float* radii) {
    if (n_radii < 1 || n_radii > NB_CENSUS_MAX_RADII)
        return fail(c, NB_ERR_ARG, "n_radii outside [1, NB_CENSUS_MAX_RADII]");
    if (!c->has_list) return fail(c, NB_ERR_STATE, "no pair list");
    for (int k = 0; k < n_radii; ++k)
        if (!(radii[k] > 0.f) || !(radii[k] <= c->p.rlist))
            return fail(c, NB_ERR_ARG, "census radius outside (0, rlist]");
    NB_HIP(c, hipSetDevice(c->device));
    return NB_OK;
}

// The context's census buffers, allocated on first use and grown to the list.
nb_status census_ctx_bufs(nb_ctx* c, bool cover, CensusBufs* b) {
    const int nb = census_blocks(c->n_items, cover);
    const size_t words = census_words(cover);
    const size_t need_hist = (size_t)nb * words, need_part = (size_t)((nb + 63) / 64) * words;
    if (need_hist > c->census_hist_n) {
        NB_HIP(c, dev_alloc(c->census_hist, need_hist));
        c->census_hist_n = need_hist;
    }
    if (need_part > c->census_part_n) {
        NB_HIP(c, dev_alloc(c->census_part, need_part));
        c->census_part_n = need_part;
    }
    if (!c->census_total)
        NB_HIP(c, dev_alloc(c->census_total, (size_t)NB_CENSUS_MAX_RADII * NB_CENSUS_MAX_RADII));
    if (!c->census_thr) NB_HIP(c, dev_alloc(c->census_thr, NB_CENSUS_MAX_RADII));
    *b = CensusBufs{c->census_hist, c->census_part, c->census_total, c->census_thr, nb, false};
    return NB_OK;
}

// Census counts from the summed bins: bin b holds the sub-cluster pairs first inside the
// b-th smallest radius.
void census_counts(int32_t n_radii, const int* ord, const unsigned long long* tot,
                   int64_t* counts) {
    for (int s = 0; s < 16; ++s) {
        int64_t acc = 0;
        for (int k = 0; k < n_radii; ++k) {
            acc += (int64_t)tot[(size_t)s * NB_CENSUS_MAX_RADII + k];
            counts[(size_t)s * n_radii + ord[k]] = acc;
        }
    }
}

}  // namespace

nb_status nb_list_census(nb_ctx* c, int32_t n_radii, const float* radii, int64_t* counts) {
    if (!c) return NB_ERR_ARG;
    if (!radii || !counts) return fail(c, NB_ERR_ARG, "null radii or counts");
    nb_status st = census_check(c, n_radii, radii);
    if (st != NB_OK) return st;
    CensusBufs b;
    st = census_ctx_bufs(c, false, &b);
    if (st != NB_OK) return st;
    int ord[NB_CENSUS_MAX_RADII];
    std::vector<unsigned long long> tot(census_words(false));
    st = census_walk(c, n_radii, radii, false, 0, 0, b, ord, tot.data());
    if (st != NB_OK) return st;
    census_counts(n_radii, ord, tot.data(), counts);
    return NB_OK;
}

nb_status nb_list_census_noalloc(nb_ctx* c, int32_t n_radii, const float* radii,
                                 int64_t* counts) {
    if (!c) return NB_ERR_ARG;
    if (!radii || !counts) return fail(c, NB_ERR_ARG, "null radii or counts");
    nb_status st = census_check(c, n_radii, radii);
    if (st != NB_OK) return st;
    NbCensusScratch sc{};
    NB_HIP(c, census_noalloc_scratch(c->device, &sc));
    const CensusBufs b{sc.hist, sc.part, sc.total, sc.thr, sc.max_blocks, true};
    int ord[NB_CENSUS_MAX_RADII];
    unsigned long long tot[NB_CENSUS_MAX_RADII * 16];
    static_assert(sizeof(tot) / sizeof(tot[0]) >= 16 * NB_CENSUS_MAX_RADII, "census words");
    st = census_walk(c, n_radii, radii, false, 0, 0, b, ord, tot);
    if (st != NB_OK) return st;
    census_counts(n_radii, ord, tot, counts);
    return NB_OK;
}

nb_status nb_list_coverage(nb_ctx* c, int32_t log2_m, int32_t log2_n, int32_t n_radii,
                           const float* radii, int64_t* covered) {
    if (!c) return NB_ERR_ARG;
    if (!radii || !covered) return fail(c, NB_ERR_ARG, "null radii or covered");
    if (log2_m < 0 || log2_m > 3 || log2_n < 0 || log2_n > 3)
        return fail(c, NB_ERR_ARG, "sub-cluster sizes must be 1, 2, 4 or 8");
    nb_status st = census_check(c, n_radii, radii);
    if (st != NB_OK) return st;
    CensusBufs b;
    st = census_ctx_bufs(c, true, &b);
    if (st != NB_OK) return st;
    int ord[NB_CENSUS_MAX_RADII];
    std::vector<unsigned long long> tot(census_words(true));
    st = census_walk(c, n_radii, radii, true, log2_m, log2_n, b, ord, tot.data());
    if (st != NB_OK) return st;
    // [l][k] (sorted bins): pairs first inside radius k whose sub-cluster pair is first held
    // at radius l; two prefix sums give pairs inside R_k in sub-cluster pairs held at R_l
    std::vector<int64_t> cum((size_t)n_radii * n_radii, 0);
    for (int l = 0; l < n_radii; ++l)
        for (int k = 0; k < n_radii; ++k) {
            int64_t v = (int64_t)tot[(size_t)l * NB_CENSUS_MAX_RADII + k];
            if (l > 0) v += cum[(size_t)(l - 1) * n_radii + k];
            if (k > 0) v += cum[(size_t)l * n_radii + k - 1];
            if (l > 0 && k > 0) v -= cum[(size_t)(l - 1) * n_radii + k - 1];
            cum[(size_t)l * n_radii + k] = v;
        }
    for (int l = 0; l < n_radii; ++l)
        for (int k = 0; k < n_radii; ++k)
            covered[(size_t)ord[l] * n_radii + ord[k]] = cum[(size_t)l * n_radii + k];
    return NB_OK;
}

nb_status nb_get_stats(nb_ctx* c, nb_stats* out) {
    if (!c || !out) return NB_ERR_ARG;
    if (c->has_list) {
        NB_HIP(c, hipSetDevice(c->device));
        std::vector<double> ds(2 * (size_t)c->n_sys);
        nb_status st = to_host(c, ds.data(), c->d.dstat, ds.size());
        if (st != NB_OK) return st;
        double eff = 0, comp = 0;
        for (int s = 0; s < c->n_sys; ++s) {
            eff += ds[2 * s];
            comp += ds[2 * s + 1];
        }
        c->stats.effective_pairs = (int64_t)eff;
        c->stats.computed_pairs = (int64_t)comp;
        // inner masks change with every rolling prune: recount them
        std::vector<NbEntry> ent((size_t)c->n_entries);
        st = to_host(c, ent.data(), c->d.entries, ent.size());
        if (st != NB_OK) return st;
        int64_t inner = 0;
        for (const NbEntry& e : ent) inner += __builtin_popcount((e.meta >> 16) & 0xffu);
        c->stats.inner_pairs = inner;
    }
    *out = c->stats;
    return NB_OK;
}

}  // extern "C"
