/*
 * FP64 brute-force oracle for the cluster-pair nonbonded path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant with the HIP path.
 *
 * What it computes, and where the paper defines it:
 *
 *  - oracle_forces: the short-range nonbonded energies, forces and virial as the
 *    plain all-pairs minimum-image sum over non-excluded pairs inside the cut-off
 *    (Sec. II: forces from positions; Sec. V.A: Lennard-Jones plus electrostatics,
 *    each pair once by Newton's third law, self and force-field exclusions never
 *    interact, real-space Ewald term for PME runs).  The cluster algorithm adds no
 *    approximation to this sum apart from arithmetic precision and pairs missed
 *    by a too-short list buffer (Sec. V.B), so the plain sum is the result.
 *    The paper names the potentials but writes no formula; the forms used are
 *    the textbook 12-6 Lennard-Jones on (c6, c12), reaction field, and the Ewald
 *    real-space erfc term, with a potential-shift modifier for LJ and Ewald.
 *
 *    With excl_corr set, excluded pairs inside the cut-off and each atom with
 *    itself add the electrostatic corrections a long-range part needs (Sec. V.A:
 *    the real-space Ewald correction of PME runs; the reaction-field analogue).
 *
 *  - oracle_forces_cells: the same sums found through a cell grid (each atom against
 *    the atoms of its 27 neighbouring cells), for boxes too large for the all-pairs
 *    loop; checked against oracle_forces.
 *
 *  - oracle_backward: gradients of a scalar loss L(F, E) with respect to the
 *    positions, the charges and the (c6, c12) table, given dL/dF and dL/dE, over
 *    the frozen set of pairs inside the cut-off (the pair list is piecewise
 *    constant in the positions and is not differentiated).
 *
 *  - oracle_cluster_pairs: the set of cluster pairs that hold at least one
 *    atom pair within a radius (Sec. V.A, Fig. 4: a j-cluster is listed for an
 *    i-cluster when one of its atoms is inside the buffered cut-off of one of the
 *    i-atoms; Sec. V.D/E: the list is pruned on particle distances against the
 *    outer and the inner cut-off).  Brute force over every atom pair, with the
 *    squared distance evaluated in a fixed IEEE single-precision sequence so the
 *    decision is reproducible bit for bit.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Pair interaction parameters (plain values; mirrored by a ctypes Structure). */
typedef struct {
    int32_t coulomb;     /* 0 = reaction field, 1 = Ewald real space        */
    int32_t modifier;    /* 0 = none, 1 = potential shift (LJ and Ewald)     */
    double rc;           /* cut-off, nm                                      */
    double eps_r;        /* relative dielectric constant                     */
    double eps_rf;       /* reaction-field dielectric; +inf allowed          */
    double beta;         /* Ewald splitting parameter, 1/nm                  */
    double epsfac;       /* Coulomb constant, kJ mol^-1 nm e^-2              */
    int32_t excl_corr;   /* 1: excluded pairs inside rc and each atom with
                            itself carry their electrostatic corrections     */
} oracle_params;

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (n >= 1), for single-thread timings. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Is b in the exclusion row of a?  Rows are short (a few partners). */
static int excluded(const int64_t* ptr, const int32_t* idx, int64_t a, int64_t b) {
    for (int64_t k = ptr[a]; k < ptr[a + 1]; ++k)
        if (idx[k] == b) return 1;
    return 0;
}

/* Minimum-image separation a - b along one axis of length L (unique when L > 2 rc). */
static double min_image(double d, double L) { return d - L * nearbyint(d / L); }

/* Reaction-field constants: k_rf = (eps_rf - eps_r) / ((2 eps_rf + eps_r) rc^3),
 * which tends to 1/(2 rc^3) as eps_rf -> inf; c_rf = 1/rc + k_rf rc^2 makes V(rc) = 0. */
static void rf_constants(const oracle_params* p, double* krf, double* crf) {
    double rc3 = p->rc * p->rc * p->rc;
    if (isinf(p->eps_rf)) *krf = 1.0 / (2.0 * rc3);
    else *krf = (p->eps_rf - p->eps_r) / ((2.0 * p->eps_rf + p->eps_r) * rc3);
    *crf = 1.0 / p->rc + (*krf) * p->rc * p->rc;
}

/*
 * One pair at distance r (> 0) with Coulomb prefactor kq = epsfac qa qb / eps_r:
 *   vlj, vc     pair energies (with the shift of the modifier)
 *   flj, fc     phi = -V'(r)/r, so that the force on a is phi * (x_a - x_b)
 *   dflj, dfc   phi'(r) / r  (used by the backward pass)
 *   ulj12, ulj6 dphi_LJ/dc12, dphi_LJ/dc6
 *   elj12, elj6 dV_LJ/dc12, dV_LJ/dc6
 *   psi, v      phi_C / kq and V_C / kq
 */
typedef struct {
    double vlj, vc, flj, fc, dflj, dfc, ulj12, ulj6, elj12, elj6, psi, v, dpsi;
} pair_terms;

static void pair_eval(const oracle_params* p, double r2, double c6, double c12, double kq,
                      double krf, double crf, pair_terms* t) {
    const double r = sqrt(r2);
    const double ir = 1.0 / r, ir2 = ir * ir, ir6 = ir2 * ir2 * ir2, ir12 = ir6 * ir6;
    const double rc = p->rc;
    const double irc6 = 1.0 / (rc * rc * rc * rc * rc * rc), irc12 = irc6 * irc6;
    const double m = (p->modifier == 1) ? 1.0 : 0.0;

    /* Lennard-Jones 12-6: V = c12 r^-12 - c6 r^-6 - m (c12 rc^-12 - c6 rc^-6). */
    t->elj12 = ir12 - m * irc12;
    t->elj6 = -(ir6 - m * irc6);
    t->vlj = c12 * t->elj12 + c6 * t->elj6;
    t->ulj12 = 12.0 * ir12 * ir2;            /* d phi / d c12 = 12 r^-14 */
    t->ulj6 = -6.0 * ir6 * ir2;              /* d phi / d c6  = -6 r^-8  */
    t->flj = c12 * t->ulj12 + c6 * t->ulj6;
    /* phi_LJ'(r)/r = (-168 c12 r^-16 + 48 c6 r^-10) */
    t->dflj = (-168.0 * c12 * ir12 * ir2 * ir2 + 48.0 * c6 * ir6 * ir2 * ir2);

    if (p->coulomb == 0) {
        /* Reaction field: V = kq (1/r + k_rf r^2 - c_rf), phi = kq (r^-3 - 2 k_rf). */
        t->v = ir + krf * r2 - crf;
        t->psi = ir * ir2 - 2.0 * krf;
        t->dpsi = -3.0 * ir2 * ir2 * ir;     /* psi'(r)/r = -3 r^-5 */
    } else {
        /* Ewald real space: V = kq (erfc(beta r)/r - m erfc(beta rc)/rc),
         * phi = kq (erfc(beta r)/r + 2 beta/sqrt(pi) exp(-beta^2 r^2)) / r^2. */
        const double b = p->beta;
        const double er = erfc(b * r);
        const double ex = 2.0 * b / sqrt(M_PI) * exp(-b * b * r2);
        const double g = er * ir + ex;                               /* g = -r dV/dr  */
        const double dg = -er * ir2 - ex * ir - 2.0 * b * b * r * ex; /* dg/dr */
        t->v = er * ir - m * erfc(b * rc) / rc;
        t->psi = g * ir2;
        t->dpsi = (dg * ir2 - 2.0 * g * ir2 * ir) * ir;              /* psi'(r)/r */
    }
    t->vc = kq * t->v;
    t->fc = kq * t->psi;
    t->dfc = kq * t->dpsi;
}

/*
 * Electrostatics of an excluded pair inside the cut-off, when the run has a long-range
 * part that counts every pair of charges (Sec. V.A: for PME runs the kernel computes the
 * real-space Ewald correction; force-field exclusions are enforced together with the
 * cut-off).  Excluded pairs have no Lennard-Jones and no 1/r term, but keep what the
 * long-range treatment assigns to every pair:
 *   Ewald:  V = -kq erf(beta r)/r                (the reciprocal-space pair energy removed)
 *           phi = -V'(r)/r = kq (2 beta/sqrt(pi) exp(-beta^2 r^2) - erf(beta r)/r) / r^2
 *   RF:     V = kq (k_rf r^2 - c_rf),  phi = -2 kq k_rf   (the reaction field of the pair)
 * At r = 0 (never reached by distinct atoms) the limits -kq 2 beta/sqrt(pi) and
 * -kq 4 beta^3/(3 sqrt(pi)) are used.  Each atom with itself adds the energy
 * self_term(kq_aa) (kq_aa = epsfac q_a^2 / eps_r) and no force:
 *   Ewald: -kq_aa beta/sqrt(pi);   RF: -kq_aa c_rf / 2.
 */
static void excl_eval(const oracle_params* p, double r2, double kq, double krf, double crf,
                      double* v, double* phi) {
    if (p->coulomb == 0) {
        *v = kq * (krf * r2 - crf);
        *phi = -2.0 * kq * krf;
        return;
    }
    const double b = p->beta;
    if (r2 == 0.0) {
        *v = -kq * 2.0 * b / sqrt(M_PI);
        *phi = -kq * 4.0 * b * b * b / (3.0 * sqrt(M_PI));
        return;
    }
    const double r = sqrt(r2);
    const double ef = erf(b * r);
    *v = -kq * ef / r;
    *phi = kq * (2.0 * b / sqrt(M_PI) * exp(-b * b * r2) - ef / r) / r2;
}

static double self_term(const oracle_params* p, double kq_aa, double crf) {
    if (!p->excl_corr) return 0.0;
    if (p->coulomb == 0) return -0.5 * kq_aa * crf;
    return -kq_aa * p->beta / sqrt(M_PI);
}

/*
 * Energies [LJ, Coulomb], forces f[n][3] and virial Xi = -1/2 sum_pairs d (x) (phi d),
 * all in FP64, over every pair a < b with (a, b) not excluded and |d_ab| < rc.
 * energy_abs (may be NULL) receives the sums of |pair energy| [LJ, Coulomb], the scale
 * against which the rounding of single-precision pair energies is judged.
 * Inputs are the single-precision values the HIP path receives.
 * Atoms outside [0, L) are fine: the minimum image takes care of them.
 */
int oracle_forces(int64_t n, const float* x, const float* q, const int32_t* type,
                  int32_t ntypes, const float* lj, const int64_t* excl_ptr,
                  const int32_t* excl_idx, const float* box, const oracle_params* p,
                  double* f, double* energy, double* virial, double* energy_abs) {
    double L[3] = {box[0], box[1], box[2]};
    double krf = 0, crf = 0;
    rf_constants(p, &krf, &crf);
    const double rc2 = p->rc * p->rc;
    const double kq0 = p->epsfac / p->eps_r;
    int nt = oracle_num_threads();
    double* fbuf = (double*)calloc((size_t)nt * (size_t)n * 3, sizeof(double));
    double* ebuf = (double*)calloc((size_t)nt * 13, sizeof(double));
    if (!fbuf || !ebuf) { free(fbuf); free(ebuf); return -1; }

#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* fl = fbuf + (size_t)tid * (size_t)n * 3;
        double* el = ebuf + (size_t)tid * 13;
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < n; ++a) {
            for (int64_t b = a + 1; b < n; ++b) {
                double d[3];
                for (int k = 0; k < 3; ++k)
                    d[k] = min_image((double)x[3 * a + k] - (double)x[3 * b + k], L[k]);
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (!(r2 < rc2)) continue;
                double phi, vlj = 0.0, vc;
                if (excluded(excl_ptr, excl_idx, a, b)) {
                    if (!p->excl_corr) continue;
                    excl_eval(p, r2, kq0 * q[a] * q[b], krf, crf, &vc, &phi);
                } else {
                    const float* c = lj + 2 * ((int64_t)type[a] * ntypes + type[b]);
                    pair_terms t;
                    pair_eval(p, r2, c[0], c[1], kq0 * q[a] * q[b], krf, crf, &t);
                    phi = t.flj + t.fc;
                    vlj = t.vlj;
                    vc = t.vc;
                }
                for (int k = 0; k < 3; ++k) {
                    fl[3 * a + k] += phi * d[k];
                    fl[3 * b + k] -= phi * d[k];
                }
                el[0] += vlj;
                el[1] += vc;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) el[2 + 3 * i + j] += -0.5 * d[i] * phi * d[j];
                el[11] += fabs(vlj);
                el[12] += fabs(vc);
            }
            const double vs = self_term(p, kq0 * q[a] * q[a], crf);
            el[1] += vs;
            el[12] += fabs(vs);
        }
    }
    /* Fixed-order reduction over threads. */
    memset(f, 0, sizeof(double) * 3 * (size_t)n);
    for (int k = 0; k < 13; ++k) {
        double s = 0;
        for (int t = 0; t < nt; ++t) s += ebuf[13 * t + k];
        if (k < 2) energy[k] = s;
        else if (k < 11) virial[k - 2] = s;
        else if (energy_abs) energy_abs[k - 11] = s;
    }
    for (int t = 0; t < nt; ++t) {
        const double* fl = fbuf + (size_t)t * (size_t)n * 3;
        for (int64_t i = 0; i < 3 * n; ++i) f[i] += fl[i];
    }
    free(fbuf);
    free(ebuf);
    return 0;
}

/*
 * Force on each of the listed atoms only (O(N) per atom): for sampled checks at
 * sizes where the full O(N^2) sum is too slow to repeat.
 */
int oracle_forces_on(int64_t n, const float* x, const float* q, const int32_t* type,
                     int32_t ntypes, const float* lj, const int64_t* excl_ptr,
                     const int32_t* excl_idx, const float* box, const oracle_params* p,
                     int64_t n_sel, const int64_t* sel, double* f_sel) {
    double L[3] = {box[0], box[1], box[2]};
    double krf = 0, crf = 0;
    rf_constants(p, &krf, &crf);
    const double rc2 = p->rc * p->rc;
    const double kq0 = p->epsfac / p->eps_r;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t a = sel[s];
        double fa[3] = {0, 0, 0};
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double d[3];
            for (int k = 0; k < 3; ++k)
                d[k] = min_image((double)x[3 * a + k] - (double)x[3 * b + k], L[k]);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc2)) continue;
            double phi;
            if (excluded(excl_ptr, excl_idx, a, b)) {
                if (!p->excl_corr) continue;
                double vc;
                excl_eval(p, r2, kq0 * q[a] * q[b], krf, crf, &vc, &phi);
            } else {
                const float* c = lj + 2 * ((int64_t)type[a] * ntypes + type[b]);
                pair_terms t;
                pair_eval(p, r2, c[0], c[1], kq0 * q[a] * q[b], krf, crf, &t);
                phi = t.flj + t.fc;
            }
            for (int k = 0; k < 3; ++k) fa[k] += phi * d[k];
        }
        for (int k = 0; k < 3; ++k) f_sel[3 * s + k] = fa[k];
    }
    return 0;
}

/*
 * The energies, forces and virial of oracle_forces, summed per atom over the atoms of
 * its 27 neighbouring cells instead of over all pairs: for boxes whose all-pairs sum is
 * too slow to repeat (1.5 million atoms).  The box is cut into nc[k] = floor(L_k / rc')
 * cells per axis (rc' = rc (1 + 1e-9), so a cell is wider than the cut-off and two atoms
 * closer than rc lie in the same or adjacent cells); atoms are binned by their FP64
 * wrapped position.  With fewer than three cells on an axis the 27 neighbours would
 * repeat, and the call returns oracle_forces.  Every pair inside rc is found from both of
 * its atoms: each atom sums its own force, and half of each pair's energies, |energies|
 * and virial.  Blocks of 256 consecutive atoms keep their partial sums, added in block
 * order afterwards, so the result does not depend on the thread count.  Tested against
 * oracle_forces (rounding-level agreement).
 */
int oracle_forces_cells(int64_t n, const float* x, const float* q, const int32_t* type,
                        int32_t ntypes, const float* lj, const int64_t* excl_ptr,
                        const int32_t* excl_idx, const float* box, const oracle_params* p,
                        double* f, double* energy, double* virial, double* energy_abs) {
    const double L[3] = {box[0], box[1], box[2]};
    int nc[3];
    for (int k = 0; k < 3; ++k) {
        nc[k] = (int)floor(L[k] / (p->rc * (1.0 + 1e-9)));
        if (nc[k] < 3)
            return oracle_forces(n, x, q, type, ntypes, lj, excl_ptr, excl_idx, box, p, f,
                                 energy, virial, energy_abs);
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t* cell_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
    int64_t* members = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    const int64_t n_blk = (n + 255) / 256;
    double* bsum = (double*)calloc((size_t)(n_blk > 0 ? n_blk : 1) * 13, sizeof(double));
    if (!cell_of || !start || !fill || !members || !bsum) {
        free(cell_of); free(start); free(fill); free(members); free(bsum);
        return -1;
    }
    /* bin: counting sort by cell, atoms in index order inside a cell */
    for (int64_t a = 0; a < n; ++a) {
        int64_t c = 0;
        for (int k = 0; k < 3; ++k) {
            const double v = (double)x[3 * a + k];
            const double w = v - L[k] * floor(v / L[k]);
            int ck = (int)floor(w / L[k] * nc[k]);
            if (ck < 0) ck = 0;
            if (ck > nc[k] - 1) ck = nc[k] - 1;
            c = c * nc[k] + ck;
        }
        cell_of[a] = c;
        start[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    for (int64_t a = 0; a < n; ++a) members[start[cell_of[a]] + fill[cell_of[a]]++] = a;

    double krf = 0, crf = 0;
    rf_constants(p, &krf, &crf);
    const double rc2 = p->rc * p->rc;
    const double kq0 = p->epsfac / p->eps_r;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t blk = 0; blk < n_blk; ++blk) {
        double* s = bsum + 13 * blk;
        const int64_t a1 = (blk + 1) * 256 < n ? (blk + 1) * 256 : n;
        for (int64_t a = blk * 256; a < a1; ++a) {
            const int64_t c = cell_of[a];
            const int cz = (int)(c % nc[2]), cy = (int)((c / nc[2]) % nc[1]),
                      cx = (int)(c / ((int64_t)nc[1] * nc[2]));
            double fa[3] = {0, 0, 0};
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int64_t nb = (((int64_t)((cx + dx + nc[0]) % nc[0]) * nc[1] +
                                             (cy + dy + nc[1]) % nc[1]) * nc[2]) +
                                           (cz + dz + nc[2]) % nc[2];
                        for (int64_t m = start[nb]; m < start[nb + 1]; ++m) {
                            const int64_t b = members[m];
                            if (b == a) continue;
                            double d[3];
                            for (int k = 0; k < 3; ++k)
                                d[k] = min_image((double)x[3 * a + k] - (double)x[3 * b + k],
                                                 L[k]);
                            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                            if (!(r2 < rc2)) continue;
                            double phi, vlj = 0.0, vc;
                            if (excluded(excl_ptr, excl_idx, a, b)) {
                                if (!p->excl_corr) continue;
                                excl_eval(p, r2, kq0 * q[a] * q[b], krf, crf, &vc, &phi);
                            } else {
                                const float* cc = lj + 2 * ((int64_t)type[a] * ntypes + type[b]);
                                pair_terms t;
                                pair_eval(p, r2, cc[0], cc[1], kq0 * q[a] * q[b], krf, crf, &t);
                                phi = t.flj + t.fc;
                                vlj = t.vlj;
                                vc = t.vc;
                            }
                            for (int k = 0; k < 3; ++k) fa[k] += phi * d[k];
                            s[0] += 0.5 * vlj;
                            s[1] += 0.5 * vc;
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j)
                                    s[2 + 3 * i + j] += -0.25 * d[i] * phi * d[j];
                            s[11] += 0.5 * fabs(vlj);
                            s[12] += 0.5 * fabs(vc);
                        }
                    }
            const double vs = self_term(p, kq0 * q[a] * q[a], crf);
            s[1] += vs;
            s[12] += fabs(vs);
            for (int k = 0; k < 3; ++k) f[3 * a + k] = fa[k];
        }
    }
    for (int k = 0; k < 13; ++k) {
        double t = 0;
        for (int64_t blk = 0; blk < n_blk; ++blk) t += bsum[13 * blk + k];
        if (k < 2) energy[k] = t;
        else if (k < 11) virial[k - 2] = t;
        else if (energy_abs) energy_abs[k - 11] = t;
    }
    free(cell_of); free(start); free(fill); free(members); free(bsum);
    return 0;
}

/*
 * Backward pass over the frozen pair set P = {a < b, not excluded, |d| < rc}.
 * Given G = dL/dF [n][3] and gE = dL/dE [2] (LJ, Coulomb), accumulates:
 *   grad_x [n][3]:   per pair, u = (G_a - G_b).d,
 *                    h = (phi'(r)/r) u d + phi (G_a - G_b) - (gE_LJ phi_LJ + gE_C phi_C) d,
 *                    grad_x_a += h, grad_x_b -= h   (dE/dx_a = -F_a contribution)
 *   grad_q [n]:      phi_C = kq0 q_a q_b psi, V_C = kq0 q_a q_b v:
 *                    grad_q_a += kq0 q_b (psi u + gE_C v), grad_q_b += kq0 q_a (psi u + gE_C v)
 *   grad_lj [T][T][2] (c6, c12) per ordered type pair (t_a, t_b) of the pair as it
 *                    appears (a < b); the caller symmetrises if the table is symmetric:
 *                    dL/dc12 += u dphi/dc12 + gE_LJ dV/dc12, dL/dc6 likewise.
 */
int oracle_backward(int64_t n, const float* x, const float* q, const int32_t* type,
                    int32_t ntypes, const float* lj, const int64_t* excl_ptr,
                    const int32_t* excl_idx, const float* box, const oracle_params* p,
                    const double* G, const double* gE, double* grad_x, double* grad_q,
                    double* grad_lj) {
    double L[3] = {box[0], box[1], box[2]};
    double krf = 0, crf = 0;
    rf_constants(p, &krf, &crf);
    const double rc2 = p->rc * p->rc;
    const double kq0 = p->epsfac / p->eps_r;
    const int nt = oracle_num_threads();
    const size_t per = (size_t)n * 4 + (size_t)ntypes * ntypes * 2;
    double* buf = (double*)calloc((size_t)nt * per, sizeof(double));
    if (!buf) return -1;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* gx = buf + (size_t)tid * per;
        double* gq = gx + (size_t)n * 3;
        double* gl = gq + (size_t)n;
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < n; ++a) {
            for (int64_t b = a + 1; b < n; ++b) {
                double d[3];
                for (int k = 0; k < 3; ++k)
                    d[k] = min_image((double)x[3 * a + k] - (double)x[3 * b + k], L[k]);
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (!(r2 < rc2)) continue;
                if (excluded(excl_ptr, excl_idx, a, b)) continue;
                const int64_t tp = (int64_t)type[a] * ntypes + type[b];
                const float* c = lj + 2 * tp;
                pair_terms t;
                pair_eval(p, r2, c[0], c[1], kq0 * q[a] * q[b], krf, crf, &t);
                double dG[3], u = 0;
                for (int k = 0; k < 3; ++k) {
                    dG[k] = G[3 * a + k] - G[3 * b + k];
                    u += dG[k] * d[k];
                }
                const double phi = t.flj + t.fc, dphi = t.dflj + t.dfc;
                const double ephi = gE[0] * t.flj + gE[1] * t.fc;
                for (int k = 0; k < 3; ++k) {
                    double h = dphi * u * d[k] + phi * dG[k] - ephi * d[k];
                    gx[3 * a + k] += h;
                    gx[3 * b + k] -= h;
                }
                const double w = t.psi * u + gE[1] * t.v;
                gq[a] += kq0 * q[b] * w;
                gq[b] += kq0 * q[a] * w;
                gl[2 * tp + 0] += u * t.ulj6 + gE[0] * t.elj6;
                gl[2 * tp + 1] += u * t.ulj12 + gE[0] * t.elj12;
            }
        }
    }
    memset(grad_x, 0, sizeof(double) * 3 * (size_t)n);
    memset(grad_q, 0, sizeof(double) * (size_t)n);
    memset(grad_lj, 0, sizeof(double) * (size_t)ntypes * ntypes * 2);
    for (int t = 0; t < nt; ++t) {
        const double* gx = buf + (size_t)t * per;
        const double* gq = gx + (size_t)n * 3;
        const double* gl = gq + (size_t)n;
        for (int64_t i = 0; i < 3 * n; ++i) grad_x[i] += gx[i];
        for (int64_t i = 0; i < n; ++i) grad_q[i] += gq[i];
        for (int64_t i = 0; i < (int64_t)ntypes * ntypes * 2; ++i) grad_lj[i] += gl[i];
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Cluster-pair sets.
 *
 * Slots are grouped eight to a cluster (cluster = slot / 8); slot_atom[s] = -1 marks an
 * empty slot.  xw holds the wrapped single-precision coordinates per atom (user order).
 *
 * A cluster pair is the triple (ci, cj, s) with ci <= cj and s in {-1,0,1}^3 a periodic
 * shift of the j-cluster, coded (sx+1)*9 + (sy+1)*3 + (sz+1) (13 = no shift).  For
 * ci == cj only s = 0 and the lexicographically positive shifts are canonical, and for
 * s = 0 only the atom pairs with the i-slot before the j-slot count.
 *
 * Distance arithmetic, in IEEE single precision without fused operations, per axis:
 *   a = (s > 0) ? x_i - L : x_i ;  b = (s < 0) ? x_j - L : x_j ;  d = a - b
 *   r2 = (dx*dx + dy*dy) + dz*dz   and the pair is inside iff r2 < R2.
 * Subtracting L on the side whose coordinate is near L keeps the shift exact.
 * ------------------------------------------------------------------------- */
/* One axis of the specified sequence (compiled without contraction: each line rounds). */
static float shifted_d(float xi, float xj, float L, int s) {
    float a = (s > 0) ? (xi - L) : xi;
    float b = (s < 0) ? (xj - L) : xj;
    return a - b;
}

static int lex_positive(int sx, int sy, int sz) {
    if (sx != 0) return sx > 0;
    if (sy != 0) return sy > 0;
    return sz > 0;
}

/*
 * All canonical triples with ci in [ci_lo, ci_hi) holding at least one atom pair
 * with r2 < R2.  Writes keys (ci * n_clusters + cj) * 27 + shift_code, unsorted and
 * possibly repeated, into out[cap]; returns the number written, or -(needed) when
 * cap is too small (nothing useful written then).
 */
int64_t oracle_cluster_pairs(int64_t n_slots, const int32_t* slot_atom, const float* xw,
                             const float* box, float R2, int64_t ci_lo, int64_t ci_hi,
                             int64_t* out, int64_t cap) {
    const int64_t n_cl = n_slots / 8;
    const float L[3] = {box[0], box[1], box[2]};
    int64_t total = 0;
    if (ci_hi > n_cl) ci_hi = n_cl;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ci = ci_lo; ci < ci_hi; ++ci) {
        /* Per i-cluster: mark the (cj, s) found, to emit each at most once per row. */
        unsigned char* seen = (unsigned char*)calloc((size_t)(n_cl - ci) * 27, 1);
        int64_t local = 0;
        for (int ii = 0; ii < 8; ++ii) {
            const int64_t p = ci * 8 + ii;
            const int32_t a = slot_atom[p];
            if (a < 0) continue;
            const float* xi = xw + 3 * (int64_t)a;
            for (int64_t qs = p + 1; qs < n_slots; ++qs) {
                const int32_t b = slot_atom[qs];
                if (b < 0) continue;
                const int64_t cj = qs / 8;
                const float* xj = xw + 3 * (int64_t)b;
                /* Per axis, the squared component of each shift.  In round-to-nearest the
                 * sum of non-negative terms is never below any term, so a shift whose
                 * component alone reaches R2 cannot give r2 < R2. */
                float sq[3][3];
                int ok[3][3], any = 1;
                for (int k = 0; k < 3 && any; ++k) {
                    any = 0;
                    for (int s = -1; s <= 1; ++s) {
                        float d = shifted_d(xi[k], xj[k], L[k], s);
                        sq[k][s + 1] = d * d;
                        ok[k][s + 1] = sq[k][s + 1] < R2;
                        any |= ok[k][s + 1];
                    }
                }
                if (!any) continue;
                for (int sx = -1; sx <= 1; ++sx) {
                    if (!ok[0][sx + 1]) continue;
                    for (int sy = -1; sy <= 1; ++sy) {
                        if (!ok[1][sy + 1]) continue;
                        for (int sz = -1; sz <= 1; ++sz) {
                            if (!ok[2][sz + 1]) continue;
                            float t = sq[0][sx + 1] + sq[1][sy + 1];
                            float r2 = t + sq[2][sz + 1];
                            if (!(r2 < R2)) continue;
                            int cx = sx, cy = sy, cz = sz;
                            /* (p, q, s) with ci == cj and s lexicographically negative is the
                             * canonical (q, p, -s); its distance is the exact negative. */
                            if (cj == ci && (sx | sy | sz) != 0 && !lex_positive(sx, sy, sz)) {
                                cx = -sx; cy = -sy; cz = -sz;
                            }
                            int code = (cx + 1) * 9 + (cy + 1) * 3 + (cz + 1);
                            unsigned char* m = &seen[(cj - ci) * 27 + code];
                            if (!*m) { *m = 1; ++local; }
                        }
                    }
                }
            }
        }
        int64_t base;
#pragma omp atomic capture
        { base = total; total += local; }
        if (base + local <= cap) {
            int64_t k = base;
            for (int64_t j = 0; j < (n_cl - ci) * 27; ++j)
                if (seen[j]) out[k++] = (ci * n_cl + ci + j / 27) * 27 + (j % 27);
        }
        free(seen);
    }
    return total <= cap ? total : -total;
}
