/*
 * nb.h -- C ABI of the cluster-pair short-range nonbonded library for AMD MI355X (gfx950).
 *
 * The library computes, for one or several periodic rectangular boxes of atoms, the
 * Lennard-Jones plus reaction-field or Ewald real-space forces, energies and virial of
 * all non-excluded atom pairs inside a cut-off, with the cluster-pair algorithm of
 * Pall et al., "Heterogeneous parallelization and acceleration of molecular dynamics
 * simulations in GROMACS" (J. Chem. Phys. 2020):
 *
 *   - atoms are binned on a grid that is regular in x and y and cut along z into cells
 *     of a fixed atom count; cells are split into clusters of 8 atoms, grouped 2x2x2 into
 *     super-clusters of 8 clusters (Sec. V.A, Fig. 4);
 *   - a joint list of j-clusters is built per super-cluster from cluster bounding boxes,
 *     with an 8-bit mask of the i-clusters each j-cluster interacts with, then pruned on
 *     atom distances (Sec. V.A, V.D);
 *   - the list is dual: the outer list (radius rlist) is built every nstlist steps, the
 *     inner list (radius rinner) is re-derived from it by pruning one part per step in a
 *     rolling fashion (Sec. V.E);
 *   - the force kernel evaluates every i-cluster x j-cluster pair of 8 x 8 atoms with the
 *     interaction mask, exclusion bit masks and the cut-off, each atom pair once with
 *     Newton's third law (Sec. V.A).
 *
 * Conventions
 *   - Units: nm, kJ/mol, elementary charge.  Rectangular boxes only.
 *   - "dev" pointers are HIP device pointers (e.g. a torch tensor's data_ptr() on the
 *     context's device); "host" pointers are ordinary host memory.  The caller owns every
 *     array it passes; device arrays must stay valid until the enqueued work completes.
 *   - Every call enqueues work on the context's HIP stream and returns without waiting,
 *     except those marked [sync], which wait for the stream.
 *   - No call throws; every call returns an nb_status.  Host-side validation happens
 *     before anything is enqueued; a failed call leaves the context as it was, except
 *     NB_ERR_HIP, after which the context should be destroyed.
 *   - A context is not thread-safe; use one context per stream.
 */
#ifndef NB_H
#define NB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nb_ctx nb_ctx;

typedef enum {
    NB_OK = 0,
    NB_ERR_ARG = 1,        /* null pointer, size or parameter out of range               */
    NB_ERR_BOX = 2,        /* box edge not finite, not positive, or not above 2 * rlist  */
    NB_ERR_NOMEM = 3,      /* device or host allocation failed                           */
    NB_ERR_CAPACITY = 4,   /* a list would exceed list_capacity_hint (fixed capacity)    */
    NB_ERR_STATE = 5,      /* call out of order (no topology / grid / list yet, expired) */
    NB_ERR_HIP = 6,        /* HIP runtime error; nb_last_error() has the message         */
    NB_ERR_NONFINITE = 7   /* non-finite coordinate met while building the grid          */
} nb_status;

/* Electrostatics of the pair kernel; NB_COUL_NONE is Lennard-Jones alone (charges are
 * ignored and E_C is zero), as for the paper's argon benchmark (Sec. VI). */
enum { NB_COUL_RF = 0, NB_COUL_EWALD = 1, NB_COUL_NONE = 2 };
enum { NB_MOD_NONE = 0, NB_MOD_POTSHIFT = 1 };

/* nb_forces / nb_forces_backward flags */
enum {
    NB_F_ENERGY = 1u,      /* also compute energies [LJ, Coulomb] per system (FP64)      */
    NB_F_VIRIAL = 2u,      /* also compute the virial -1/2 sum d (x) f per system (FP64) */
    NB_F_ACCUMULATE = 4u,  /* add into the output arrays instead of overwriting them     */
    NB_F_EXCL_CORR = 8u    /* nb_forces / nb_step: add the electrostatic corrections of
                              excluded pairs inside rc and of each atom with itself, which
                              a run with a long-range part needs (Sec. V.A: the real-space
                              Ewald correction of PME runs; its reaction-field analogue):
                              Ewald V = -K qa qb erf(beta r)/r, self -K qa^2 beta/sqrt(pi);
                              RF V = K qa qb (k_rf r^2 - c_rf), self -K qa^2 c_rf / 2;
                              K = epsfac / eps_r; computed by a kernel of their own in
                              double precision; no effect with NB_COUL_NONE.  The backward
                              pass does not differentiate these terms. */
};

/*
 * Interaction and list parameters.  The paper names the interactions (Lennard-Jones,
 * reaction field, real-space Ewald; Sec. II, V.A) without formulas; the library uses:
 *   V_LJ = c12 r^-12 - c6 r^-6, minus its value at rc under NB_MOD_POTSHIFT;
 *   V_RF = epsfac qa qb / eps_r (1/r + k_rf r^2 - c_rf),
 *          k_rf = (eps_rf - eps_r) / ((2 eps_rf + eps_r) rc^3) (1/(2 rc^3) for eps_rf = inf),
 *          c_rf = 1/rc + k_rf rc^2;
 *   V_EW = epsfac qa qb / eps_r erfc(beta r)/r, minus its value at rc under
 *          NB_MOD_POTSHIFT;
 * for pairs with r < rc that are neither self pairs nor listed as excluded (excluded pairs
 * and self pairs contribute nothing unless NB_F_EXCL_CORR asks for their corrections).
 */
typedef struct {
    int32_t n_types;          /* LJ types T (1..32); lj tables are [T][T][2]              */
    int32_t coulomb;          /* NB_COUL_RF, NB_COUL_EWALD or NB_COUL_NONE                 */
    int32_t modifier;         /* NB_MOD_NONE or NB_MOD_POTSHIFT                            */
    float rc;                 /* interaction cut-off, nm, > 0                              */
    float rinner;             /* inner-list radius, rc <= rinner <= rlist                  */
    float rlist;              /* outer-list radius (buffered cut-off)                      */
    float eps_r;              /* relative dielectric constant, > 0                         */
    float eps_rf;             /* reaction-field dielectric, > 0; +INFINITY allowed         */
    float ewald_beta;         /* Ewald splitting parameter, 1/nm (>= 0)                    */
    float epsfac;             /* Coulomb constant, kJ mol^-1 nm e^-2 (138.935458)          */
    int32_t nstlist;          /* steps an outer list stays valid (>= 1)                    */
    int32_t nstprune;         /* rolling-prune parts: one part pruned per step (>= 1)      */
    int64_t list_capacity_hint; /* 0: grow lists as needed; > 0: fixed entries per
                                   super-cluster, exceeding it is NB_ERR_CAPACITY          */
} nb_params;

/* Counters of the current list and the last force call (see nb_get_stats). */
typedef struct {
    int64_t n_atoms, n_slots, n_superclusters, n_clusters;
    int64_t n_entries;        /* outer-list j-entries (super-cluster, j-cluster, shift)     */
    int64_t n_work_items;     /* chunks of j-lists processed by one wavefront each         */
    int64_t outer_pairs;      /* sum over entries of popcount(outer mask), cluster pairs    */
    int64_t inner_pairs;      /* same for the inner masks as last pruned                   */
    int64_t bb_pairs;         /* cluster pairs that passed the bounding-box test           */
    int64_t n_excl_rows;      /* entries carrying an exclusion mask row                    */
    int64_t effective_pairs;  /* atom pairs inside rc in the last NB_F_ENERGY force call    */
    int64_t computed_pairs;   /* pair slots evaluated (64 per cluster pair with any pair
                                 inside rc) in the last NB_F_ENERGY force call              */
    int64_t grid_columns;     /* total x-y columns over all systems                        */
    int64_t capacity_per_sc;  /* current list capacity per super-cluster                   */
    int64_t regrows;          /* list capacity regrowths so far                            */
} nb_stats;

/*
 * Create a context for n_systems independent boxes whose atoms are the index ranges
 * [atom_offsets[s], atom_offsets[s+1]) of every per-atom array (host int64[n_systems+1],
 * atom_offsets[0] = 0, non-decreasing; empty systems allowed).  hip_stream is a
 * hipStream_t (NULL = the null stream).  Allocates device memory lazily.
 * Errors: NB_ERR_ARG for inconsistent parameters (rc <= 0, rinner < rc, rlist < rinner,
 * n_types out of range, eps_r <= 0, ...).
 */
nb_status nb_create(const nb_params* params, int32_t n_systems, const int64_t* atom_offsets,
                    void* hip_stream, nb_ctx** out);

void nb_destroy(nb_ctx* ctx);

/*
 * Per-atom LJ types (host int32[N], 0 <= type < n_types) and the force-field exclusions
 * as a symmetric CSR list (host int64[N+1] row pointers, host int32[] partner atom
 * indices in the same system); Sec. V.A: excluded pairs never interact and are masked
 * with bit masks stored with the j-clusters.  Self pairs need not be listed.  Copied once;
 * fixed for the lifetime of the context.  At most 32 partners per atom.  Errors:
 * NB_ERR_ARG for a type out of range, a partner out of range or in another system, more
 * than 32 partners, a partner listed twice, or an asymmetric list (b listed for a but a not
 * for b).
 */
nb_status nb_set_topology(nb_ctx* ctx, const int32_t* type, const int64_t* excl_ptr,
                          const int32_t* excl_idx);

/*
 * Grid build (Sec. V.A): wrap the coordinates x (dev float[N][3], continuous, not
 * re-wrapped by the caller between builds) into the boxes (host float[n_systems][3]) in
 * single precision, store each atom's image offset, bin atoms into x-y columns, sort each
 * column on z, cut it into super-cells of 64 atoms and split those 2x2x2 into clusters of
 * 8; compute cluster bounding boxes.  Requires nb_set_topology.  Errors: NB_ERR_BOX if an
 * edge is not finite, not above 2 * rlist or above 1000 nm.  NB_ERR_NONFINITE (reported by the next
 * nb_pairlist_build) if a coordinate is not finite.
 */
nb_status nb_grid_build(nb_ctx* ctx, const float* x, const float* box);

/*
 * [sync] Outer-list build (Sec. V.A, V.D): per super-cluster, the j-clusters whose
 * bounding box lies within rlist of one of its i-clusters (27 periodic shifts), each
 * cluster pair listed once (the canonical owner is the super-cluster of the lower
 * cluster index); then an atom-distance prune keeps only cluster pairs with an atom pair
 * closer than rlist (outer list) and marks those closer than rinner (inner list, all parts
 * pruned at the build positions).  Builds exclusion masks and work items.  Grows its
 * buffers and retries on overflow unless list_capacity_hint fixes the capacity.
 * Requires nb_grid_build.
 */
nb_status nb_pairlist_build(nb_ctx* ctx);

/*
 * Rolling prune (Sec. V.E): re-derive the inner masks of part
 * (steps_since_build mod nstprune) of the outer list from the current coordinates x
 * (dev float[N][3]) against rinner.  steps_since_build = 0 is a no-op (the build pruned
 * every part).  Errors: NB_ERR_STATE without a list or when
 * steps_since_build >= nstlist (the list has expired).
 */
nb_status nb_prune_rolling(nb_ctx* ctx, const float* x, int64_t steps_since_build);

/*
 * Forces (Sec. V.A) over the current inner list: x (dev float[N][3]), q (dev float[N]),
 * lj (dev float[T][T][2] = (c6, c12) per type pair, symmetric), output f (dev float[N][3]),
 * and with NB_F_ENERGY energy (dev double[n_systems][2] = LJ, Coulomb), with NB_F_VIRIAL
 * virial (dev double[n_systems][9], row-major, -1/2 sum over pairs of d (x) f).  Pair
 * arithmetic is single precision; per-atom force sums are compensated; energies and
 * virial are reduced in double precision.  Outputs are overwritten unless
 * NB_F_ACCUMULATE.  energy / virial may be NULL when their flag is not set.
 * Errors: NB_ERR_STATE without a list.
 */
nb_status nb_forces(nb_ctx* ctx, const float* x, const float* q, const float* lj, float* f,
                    double* energy, double* virial, uint32_t flags);

/*
 * One MD step of the pair path.  With the prune fused (nb_set_exec prune_fused = 1, the
 * default): exactly nb_prune_rolling(x, steps_since_build) followed by nb_forces(x, q, lj,
 * ...), with the rolling prune of the part done inside the pair kernel (Sec. V.D: a
 * special version of the force kernel prunes the list it processes); same inner list, same
 * forces, one gather and one kernel fewer.  With prune_fused = 0 the same two calls as
 * separate kernels.  steps_since_build = 0 evaluates forces only.  With prune_fused = 2
 * (ahead, the paper's rolling schedule between force computations, Sec. V.E): nb_forces
 * with the current inner list, then the part (steps_since_build + 1) mod nstprune is
 * pruned with this step's x for the next step, by blocks of the force reduction's launch
 * (none when steps_since_build + 1 = nstlist); a part is then used 1 to nstprune steps
 * after its prune instead of 0 to nstprune - 1.  Errors as both calls.
 */
nb_status nb_step(nb_ctx* ctx, const float* x, const float* q, const float* lj, float* f,
                  double* energy, double* virial, uint32_t flags, int64_t steps_since_build);

/*
 * nb_step replayed from a HIP graph.  The first call for a given rolling part, flag set
 * and set of array pointers after a list change captures the step's kernels (gather,
 * pair kernel, reductions) on a private stream and instantiates a graph; later calls
 * with the same key launch that graph on the context's stream as one submission.  This
 * removes the gaps of a sequence of short dependent kernels (Sec. V.F) and the host
 * cost of issuing them.  Same results as nb_step, bit for bit.  Graphs are dropped at
 * every nb_pairlist_build, nb_set_exec and nb_autotune; at most nstprune + 4 are kept.
 * The arrays must stay at the same addresses for a graph to be reused (update positions
 * in place).  Errors as nb_step; NB_ERR_HIP if capture or instantiation fails.
 */
nb_status nb_step_graph(nb_ctx* ctx, const float* x, const float* q, const float* lj,
                        float* f, double* energy, double* virial, uint32_t flags,
                        int64_t steps_since_build);

/*
 * Execution shape of the pair kernel.  Work items hold at most item_width entries of
 * one super-cluster's list (long lists are split for parallelism, Sec. V.F);
 * exec_mode selects how wavefronts take items:
 *   NB_EXEC_STATIC  one wavefront per item in item order;
 *   NB_EXEC_XCD     the same, blocks renumbered so that each of the 8 XCDs (each with its
 *                   own L2) processes one contiguous range of neighbouring items;
 *   NB_EXEC_QUEUE   one resident grid of G wavefronts, each first taking its own run of
 *                   near-equal estimated cost (as NB_EXEC_BALANCED, over 85 % of the
 *                   cost), then shorter runs (the rest of the list, G / 2 runs) from one
 *                   of 64 ticket pools, each shared by wavefronts spread over the device:
 *                   wavefronts on faster SIMDs take more of the tail, so all end
 *                   together (list splitting against kernel tails, Sec. V.F, with a
 *                   dynamic remainder).  Its items differ from the other modes';
 *   NB_EXEC_PERSIST persistent: one resident grid, items taken in rounds in most-work-first
 *                   order, wavefront g taking position g of even rounds and position G-1-g
 *                   of odd rounds (G wavefronts), so the per-wavefront totals even out
 *                   without any atomic;
 *   NB_EXEC_BALANCED one resident grid of G wavefronts (those of the energy flavor that fit
 *                   the device at once), the list cut into G contiguous runs of near-equal
 *                   cost (an entry costs 2 + the set bits of its inner mask as built), each
 *                   run split at super-cluster boundaries and into pieces of at most
 *                   item_width entries: every wavefront gets the same estimated share of
 *                   the work (list splitting against kernel tails, Sec. V.F).  Its items
 *                   differ from the other modes'.
 * Results do not depend on exec_mode among static, XCD and persist (each item writes its
 * own partial sums, whichever wavefront computes it), nor between launches of one mode;
 * they depend on the items only through the order of the final per-atom sums (a few ulp).
 */
enum { NB_EXEC_STATIC = 0, NB_EXEC_XCD = 1, NB_EXEC_QUEUE = 2, NB_EXEC_PERSIST = 3,
       NB_EXEC_BALANCED = 4 };
typedef struct {
    int32_t item_width;   /* entries per work item, 1..64 */
    int32_t exec_mode;    /* NB_EXEC_* */
    int32_t prune_fused;  /* nb_step: 1 = rolling prune inside the pair kernel (Sec. V.D),
                             0 = the prune as its own kernel before the pair kernel,
                             2 = ahead: its own kernel after the pair kernel, for the
                             next step's part (Sec. V.E) */
    int32_t prune_waves;  /* wavefronts per work item in the separate rolling-prune kernel:
                             1, 2, 4 or 8, or 0 = the most with which one rolling part
                             fits the device at once */
    double us_per_call;   /* nb_autotune: median time of the timed call, microseconds */
} nb_exec_config;

/* Fix the item width (0 = the built-in rule, about 8192 items, width 8..64), the mode,
 * where nb_step prunes (prune_fused 0, 1 or 2; 0 and 1 give the same inner list and
 * results, 2 prunes each part one step earlier, see nb_step) and
 * the wavefronts per item of the separate prune kernel (prune_waves 0, 1, 2, 4 or 8; same
 * inner list either way); applies to the current list at once and to every later build.
 * Errors: NB_ERR_ARG. */
nb_status nb_set_exec(nb_ctx* ctx, int32_t item_width, int32_t exec_mode, int32_t prune_fused,
                      int32_t prune_waves);
nb_status nb_get_exec(nb_ctx* ctx, nb_exec_config* out);

/*
 * [sync] Autotuner (the paper calls for dynamic auto-tuning of code flavors, Sec. VII):
 * times nb_forces(x, q, lj, flags) on the current list for item widths 8, 16, ..., 64 (steps
 * of 8), each with the five execution modes (repeats timed calls after one warm-up each,
 * HIP events, median), and NB_EXEC_PERSIST at the smallest width whose items fit the
 * resident grid in one round; then, in the two fastest shapes, a rolling step (nb_step
 * re-pruning part 1 with x) with the prune fused, separate and ahead, the step time
 * choosing shape and placement; writes up to cap trials to host trials[] and their
 * number (47) to *n_trials, and keeps
 * the fastest choices (also returned in *best) for this and later builds.
 * flags: NB_F_ENERGY and/or NB_F_VIRIAL.  Allocates and frees its own output buffers.
 * Errors: NB_ERR_STATE without a list, NB_ERR_ARG.
 */
nb_status nb_autotune(nb_ctx* ctx, const float* x, const float* q, const float* lj,
                      uint32_t flags, int32_t repeats, nb_exec_config* trials, int32_t cap,
                      int32_t* n_trials, nb_exec_config* best);

/*
 * Backward pass of nb_forces over the frozen inner list: given grad_f = dL/dF (dev
 * float[N][3]) and optionally grad_energy = dL/dE (dev double[n_systems][2], or NULL),
 * writes grad_x = dL/dx (dev float[N][3]; the Hessian-vector product of the energy with
 * grad_f, minus grad_energy times the forces), grad_q = dL/dq (dev float[N]) and
 * grad_lj = dL/d(c6, c12) (dev double[T][T][2]).  The table must be symmetric
 * (lj[a][b] = lj[b][a]); the derivative with respect to an off-diagonal value is split
 * evenly between its two entries, so chaining through any symmetric parameterisation of
 * the table is exact.  Any of the three outputs may be NULL to skip it.
 * NB_F_ACCUMULATE adds into the outputs.  Errors: NB_ERR_STATE without a list.
 */
nb_status nb_forces_backward(nb_ctx* ctx, const float* x, const float* q, const float* lj,
                             const float* grad_f, const double* grad_energy, float* grad_x,
                             float* grad_q, double* grad_lj, uint32_t flags);

/* ---- introspection for tests and tools; all [sync] ---------------------------------- */

/* Slot -> atom map of the current grid (host int32[cap], -1 = empty slot) and its size. */
nb_status nb_get_grid(nb_ctx* ctx, int32_t* slot_atom, int64_t cap, int64_t* n_slots);

/* Columns per axis of each system's grid (host int32[n_systems][2] = nx, ny). */
nb_status nb_get_grid_dims(nb_ctx* ctx, int32_t* dims);

/*
 * Cluster pairs of the outer (which = 1) or inner (which = 2) list as triples
 * (i-cluster, j-cluster, shift code) in host int32[cap][3]; shift code
 * (sx+1)*9 + (sy+1)*3 + (sz+1) for the j-cluster image x_j + s L.  which = 0 gives the
 * bounding-box candidates of the build (Sec. V.D: cluster pairs whose bounding boxes lie
 * within rlist, before the atom-distance prune), recomputed on the current grid by the
 * search kernel in a recording mode; the box test uses the list's own arithmetic so that
 * it is a superset of the outer list for every accepted box (allocates a temporary device
 * buffer).  *count receives the number of triples (even when above cap, in which case
 * nothing is written).
 */
nb_status nb_get_pairs(nb_ctx* ctx, int32_t which, int32_t* triples, int64_t cap,
                       int64_t* count);

nb_status nb_get_stats(nb_ctx* ctx, nb_stats* out);

/*
 * [sync] Work-efficiency census of the current outer list (Sec. V.B, Fig. 5; the cluster
 * setups of Sec. V.A and V.D).  For each radius radii[k] (host float[n_radii], nm, any
 * order, repeats allowed, each in (0, rlist]) and each setup M x N with M, N in
 * {1, 2, 4, 8}, counts the pairs of sub-clusters holding an atom pair closer than
 * radii[k], where an i-sub-cluster is a run of M consecutive slots of an 8-atom cluster of
 * the grid and a j-sub-cluster a run of N.  Pairs are taken as in the list: each unordered
 * atom pair (atom and periodic image) once, distances at the build positions in the list
 * arithmetic (r2 < float(radii[k])^2 in single precision), excluded pairs included.
 * counts (host int64[16][n_radii]) receives at [(log2 M) * 4 + log2 N][k] the number of
 * held M x N sub-cluster pairs: [0][k] the atom pairs closer than radii[k], [15][k] the
 * 8 x 8 cluster pairs.  An M x N list at radius r_l costs M N pair evaluations per held
 * pair, so its work efficiency at cut-off r_c is counts[0][k_c] / (M N counts[s][k_l]).
 * Errors: NB_ERR_STATE without a list; NB_ERR_ARG for a null pointer, n_radii outside
 * [1, NB_CENSUS_MAX_RADII] or a radius outside (0, rlist].  Allocates a per-context
 * histogram buffer on first use.
 */
#define NB_CENSUS_MAX_RADII 64
nb_status nb_list_census(nb_ctx* ctx, int32_t n_radii, const float* radii, int64_t* counts);

/*
 * [sync] nb_list_census without any device or host allocation, for callers that cannot
 * allocate (tight loops that re-estimate list buffers, harnesses that forbid hipMalloc).
 * Same arguments, results (bit for bit) and errors as nb_list_census; the census kernels
 * use a fixed per-device scratch array of the library (about 4.2 MB: the histograms of at
 * most 1024 blocks, which stride over the work items, so every list fits) instead of the
 * context's census buffers; the only size limit is n_radii <= NB_CENSUS_MAX_RADII
 * (NB_ERR_ARG beyond).  The scratch is shared by every context on a device and keeps the
 * last call's contents: calls that overlap on one device (contexts on different streams or
 * threads) race and must be serialised by the caller.  No timing events are recorded.
 */
nb_status nb_list_census_noalloc(nb_ctx* ctx, int32_t n_radii, const float* radii,
                                 int64_t* counts);

/*
 * [sync] Coverage of the current outer list by an M x N list (M = 2^log2_m, N = 2^log2_n,
 * each 1 ... 8; sub-clusters as in nb_list_census): the implicit buffer of cluster lists
 * that the Verlet buffer estimate takes into account (Sec. V.B).  covered (host
 * int64[n_radii][n_radii]) receives at [l][k] the number of atom pairs closer than radii[k]
 * that lie in an M x N sub-cluster pair holding an atom pair closer than radii[l], i.e. the
 * pairs within radii[k] that an M x N list at radius radii[l] contains.  [k][k] (and any
 * [l][k] with radii[l] >= radii[k]) is the number of atom pairs closer than radii[k].  Pairs,
 * distances, radii and errors as in nb_list_census; NB_ERR_ARG also for log2 sizes outside
 * [0, 3].
 */
nb_status nb_list_coverage(nb_ctx* ctx, int32_t log2_m, int32_t log2_n, int32_t n_radii,
                           const float* radii, int64_t* covered);

/*
 * Verlet buffer estimate (Sec. V.B): the drift of the energy caused by pairs that move
 * from outside a list radius to inside the cut-off during the list's lifetime, and the
 * smallest list radius that keeps it within a tolerance.  Host-only (no context, no device).
 *
 * Atoms are grouped in classes of equal mass, charge and LJ type.  Over a list age t each
 * atom moves by a Gaussian displacement of variance k_B T t^2 / m per axis (m: the mass that
 * carries it, its own or that of the rigid unit it belongs to); an atom constrained at a
 * distance d to a partner about which it rotates (the refinement for constrained atoms,
 * Sec. V.B) adds the displacement of a free rotor whose angular velocity, perpendicular to
 * the bond, has the variance k_B T / (m_own d^2) per component: per axis
 * (2/3) d^2 sqrt(2) s D(s / sqrt(2)), s = t sqrt(k_B T / (m_own d^2)), D Dawson's integral
 * (as (2/3) k_B T t^2 / m_own at first, levelling off at (2/3) d^2), taken as Gaussian; beyond the list
 * radius partners are spread uniformly; a pair not in the list that ends inside r_c, at a
 * distance of at least r_c / 2, misses |V(r)|, V the pair potential selected by the
 * nb_params (LJ with the electrostatics and the modifier of the kernels).  The missed energy per atom at age (steps - 1) dt, divided by
 * steps * dt, is the drift (kJ mol^-1 ps^-1 per atom).  A cluster list holds a fraction of
 * the pairs beyond its radius (its implicit buffer): with n_cov > 0 that fraction is taken
 * from a coverage table of nb_list_coverage (cov_radii ascending, covered[n_cov][n_cov]),
 * and the list radius must be one of cov_radii; with n_cov = 0 the list is a particle list.
 */
typedef struct {
    int32_t n_classes;
    const int64_t* count;     /* atoms per class                                              */
    const double* mass;       /* mass that carries the atom over the list lifetime, amu       */
    const float* charge;      /* e                                                            */
    const int32_t* type;      /* LJ type, < nb_params.n_types                                 */
    const float* lj;          /* (c6, c12) per type pair, float[n_types][n_types][2]          */
    double volume;            /* nm^3                                                         */
    double temperature;       /* K                                                            */
    double dt;                /* time step, ps                                                */
    int32_t n_cov;            /* coverage radii (0: particle list, no implicit buffer)        */
    const float* cov_radii;   /* [n_cov], ascending                                           */
    const int64_t* covered;   /* [n_cov][n_cov] as returned by nb_list_coverage               */
    const double* rot_len;    /* per class: distance to the constraint partner it rotates
                                 about, nm (0: none); null: no class rotates                  */
    const double* rot_mass;   /* per class: the atom's own mass, amu (read where rot_len > 0) */
} nb_buffer_input;

/* Drift for a list of radius r_list (>= rc) used for `steps` steps after its build.
 * NB_ERR_ARG for invalid input or, with a coverage table, an r_list not in it. */
nb_status nb_buffer_drift(const nb_params* params, const nb_buffer_input* in, int32_t steps,
                          double r_list, double* drift);

/* Smallest list radius in [rc, rc + max_buffer] with drift <= tolerance: by bisection to
 * 1e-6 nm for a particle list, the smallest such table radius for a cluster list.  Writes
 * the radius and its drift (drift may be null); NB_ERR_CAPACITY when no radius in range
 * reaches the tolerance.  For the dual list of Sec. V.E: steps = nstlist gives the outer
 * radius, steps = nstprune the inner one. */
nb_status nb_buffer_estimate(const nb_params* params, const nb_buffer_input* in, int32_t steps,
                             double tolerance, double max_buffer, double* r_list,
                             double* drift);

/* Kernel timing with HIP events recorded on the context's stream around each kernel
 * group (opt-in; for benchmarks and profiling).  Kinds: */
enum {
    NB_T_FORCES = 0,          /* the pair force/energy kernel of nb_forces                 */
    NB_T_FORCE_REDUCE = 1,    /* gather + per-atom force reduction + energy reduction      */
    NB_T_PRUNE = 2,           /* gather + rolling-prune kernel of nb_prune_rolling         */
    NB_T_BACKWARD = 3,        /* the pair kernel of nb_forces_backward                     */
    NB_T_BACKWARD_REDUCE = 4, /* gathers and reductions of nb_forces_backward              */
    NB_T_CENSUS = 5,          /* the census kernel of nb_list_census                       */
    NB_T_COUNT = 6
};

/* Enable (1) or disable (0) event recording; enabling clears the accumulated totals. */
nb_status nb_set_timing(nb_ctx* ctx, int32_t enable);

/* [sync] Accumulated milliseconds and launch counts per kind since the last call or since
 * timing was enabled (host double[NB_T_COUNT], int64[NB_T_COUNT]); then clears them. */
nb_status nb_get_timing(nb_ctx* ctx, double* ms, int64_t* calls);

const char* nb_strerror(nb_status status);
const char* nb_last_error(const nb_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* NB_H */
