// Verlet buffer estimate (Sec. V.B): the list radius whose missed pair interactions stay
// below a drift tolerance, from masses, temperature and the pair potentials, and, for
// cluster lists, the implicit buffer measured by nb_list_coverage.
//
// Model (all in double precision):
//   * over a list age t each atom moves by a Gaussian displacement of variance k_B T t^2 / m
//     per axis (free flight, m the mass that carries it); an atom constrained at distance d
//     to a partner about which it rotates adds a free rotor's displacement d (u(t) - u(0)):
//     its angular velocity w, perpendicular to the bond, is a 2-d Gaussian of variance
//     k_B T / (m_own d^2) per component, the squared displacement 2 d^2 (1 - cos |w| t) has a
//     third along any axis, and over the Rayleigh-distributed |w|
//     E[cos |w| t] = 1 - sqrt(2) s D(s / sqrt(2)), s^2 = k_B T t^2 / (m_own d^2), D Dawson's
//     integral; that variance enters as a Gaussian.  The distance of a pair of classes a, b
//     then changes by a Gaussian of variance sigma^2 = var_a + var_b;
//   * beyond the list radius the partners of class b are spread with density N_b / V;
//   * a pair not in the list at distance r0 >= r_l at the build that ends at r < r_c misses
//     |V_ab(r)|; a cluster list holds the fraction 1 - U(r0) of the pairs at r0 (its
//     implicit buffer), a particle list none of them (U = 1);
//   * missed energy per atom  E = (1/N) (1/2) sum_a sum_b N_a (N_b / V)
//                                 int_{r_l} dr0 4 pi r0^2 U(r0) int^{r_c} dr |V_ab(r)| g(r - r0)
//     at the oldest use of the list, t = (steps - 1) dt, and drift = E / (steps dt).
// The integrals run over 10 sigma on either Gaussian side (the rest is below e^-50), the
// inner one from no lower than r_c / 2 (missed pairs end near the cut-off; below, the
// free-flight expectation of |V| would be dominated by atomic overlaps), on Gauss-Legendre
// panels: the outer ones split at the coverage radii (U is constant between
// them) and at most sigma / 2 wide, the inner ones at most sigma / 8 wide and split at the
// zeros of V_ab, where |V_ab| has a kink.
#include <math.h>

#include <algorithm>
#include <vector>

#include "nb.h"

namespace {

constexpr double kBoltzmann = 0.0083144626181532;   // kJ mol^-1 K^-1
constexpr double kWindow = 10.0;                     // Gaussian widths integrated

struct Rule {
    std::vector<double> x, w;                        // nodes and weights on [-1, 1]
};

// Gauss-Legendre rule by Newton's iteration on P_n (three-term recurrence).
Rule gauss_legendre(int n) {
    Rule g;
    g.x.resize(n);
    g.w.resize(n);
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        g.x[i] = x;
        g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return g;
}

const Rule& rule8() {
    static const Rule r = gauss_legendre(8);
    return r;
}
const Rule& rule16() {
    static const Rule r = gauss_legendre(16);
    return r;
}

// Dawson's integral D(x) = exp(-x^2) int_0^x exp(t^2) dt = int_0^x exp(-u (2 x - u)) du
// (u = x - t), x >= 0: 16-point Gauss-Legendre panels over u, at most 1/4 and 1/(4 x) wide,
// up to where the exponent passes 60 (the rest is below e^-60 x).
double dawson(double x) {
    if (!(x > 0.0)) return 0.0;
    double hi = x;
    if (x * x > 60.0) hi = x - sqrt(x * x - 60.0);
    const double w = std::min(0.25, 0.25 / x);
    const int np = std::max(1, (int)ceil(hi / w));
    const Rule& g = rule16();
    double sum = 0.0;
    for (int p = 0; p < np; ++p) {
        const double a = hi * p / np, b = hi * (p + 1) / np;
        const double h = 0.5 * (b - a), m = 0.5 * (a + b);
        for (size_t j = 0; j < g.x.size(); ++j) {
            const double u = m + h * g.x[j];
            sum += h * g.w[j] * exp(-u * (2.0 * x - u));
        }
    }
    return sum;
}

// Per-axis variance of the displacement of an atom of class a over the time t.
double displacement_var(const nb_buffer_input& in, int a, double kT, double t) {
    double v = kT * t * t / in.mass[a];
    if (in.rot_len && in.rot_len[a] > 0.0) {
        const double d = in.rot_len[a];
        const double s = t * sqrt(kT / (in.rot_mass[a] * d * d));
        v += (2.0 / 3.0) * d * d * M_SQRT2 * s * dawson(s / M_SQRT2);
    }
    return v;
}

// Pair potential of the kernel (LJ and the chosen electrostatics, potential-shift modifier
// when set) at r < r_c.
struct Potential {
    double c6, c12, qq, rc, f, krf, crf, beta, lj_shift, c_shift;
    int coulomb;
    double operator()(double r) const {
        const double ir = 1.0 / r, ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
        double v = c12 * ir6 * ir6 - c6 * ir6 - lj_shift;
        if (coulomb == NB_COUL_RF) v += f * qq * (ir + krf * r * r - crf);
        else if (coulomb == NB_COUL_EWALD) v += f * qq * (erfc(beta * r) * ir - c_shift);
        return v;
    }
};

Potential make_potential(const nb_params& p, double c6, double c12, double qq) {
    Potential v{};
    const double rc = p.rc;
    v.c6 = c6;
    v.c12 = c12;
    v.qq = qq;
    v.rc = rc;
    v.coulomb = p.coulomb;
    v.f = (double)p.epsfac / p.eps_r;
    v.krf = isinf(p.eps_rf) ? 1.0 / (2.0 * rc * rc * rc)
                            : ((double)p.eps_rf - p.eps_r) / ((2.0 * p.eps_rf + p.eps_r) * rc * rc * rc);
    v.crf = 1.0 / rc + v.krf * rc * rc;
    v.beta = p.ewald_beta;
    const bool shift = p.modifier == NB_MOD_POTSHIFT;
    const double irc6 = 1.0 / (rc * rc * rc * rc * rc * rc);
    v.lj_shift = shift ? c12 * irc6 * irc6 - c6 * irc6 : 0.0;
    v.c_shift = shift ? erfc(v.beta * rc) / rc : 0.0;
    return v;
}

// Uncovered fraction U(r0) for a list at radius index l of the coverage table (1 beyond
// the table or with no table).
struct Uncovered {
    int n = 0, l = -1;
    const float* R = nullptr;
    const int64_t* cov = nullptr;
    double at_shell(int k) const {   // shell (R[k-1], R[k]), k > l
        const int64_t all = cov[(size_t)k * n + k] - cov[(size_t)(k - 1) * n + k - 1];
        const int64_t held = cov[(size_t)l * n + k] - cov[(size_t)l * n + k - 1];
        if (all <= 0) return 1.0;
        // a table from nb_list_coverage has 0 <= held <= all; clamp any other input
        return std::min(1.0, std::max(0.0, 1.0 - (double)held / (double)all));
    }
};

// Missed energy per atom, steps - 1 steps after the build of a list at r_l.
double missed_energy(const nb_params& p, const nb_buffer_input& in, int steps, double r_l,
                     const Uncovered& U) {
    const double t = (steps - 1) * in.dt;
    int64_t n_all = 0;
    for (int a = 0; a < in.n_classes; ++a) n_all += in.count[a];
    if (t <= 0.0 || n_all == 0) return 0.0;
    const double rc = p.rc;
    const Rule& g8 = rule8();
    const Rule& g16 = rule16();
    double total = 0.0;
    for (int a = 0; a < in.n_classes; ++a)
        for (int b = 0; b < in.n_classes; ++b) {
            if (in.count[a] == 0 || in.count[b] == 0) continue;
            const double kT = kBoltzmann * in.temperature;
            const double sig = sqrt(displacement_var(in, a, kT, t) + displacement_var(in, b, kT, t));
            if (!(sig > 0.0)) continue;                     // nothing moves (T = 0)
            const int ta = in.type[a], tb = in.type[b];
            const float* lj = in.lj + 2 * ((size_t)ta * p.n_types + tb);
            const Potential V = make_potential(p, lj[0], lj[1], (double)in.charge[a] * in.charge[b]);
            // inner nodes: r in [max(rc - W sigma, rc / 2), rc], panels <= sigma / 8, split at
            // zeros of V
            const double lo = std::max(rc - kWindow * sig, 0.5 * rc);
            const int n_in = std::max(1, (int)ceil((rc - lo) / (sig / 8.0)));
            std::vector<double> edges;
            for (int i = 0; i <= n_in; ++i) {
                const double e = (i == n_in) ? rc : lo + (rc - lo) * i / n_in;
                if (i > 0) {
                    const double e0 = edges.back();
                    const double v0 = V(e0), v1 = V(e);
                    if (v0 * v1 < 0.0) {                    // a zero inside: bisect to it
                        double x0 = e0, x1 = e;
                        for (int it = 0; it < 200 && x1 - x0 > 1e-15 * rc; ++it) {
                            const double m = 0.5 * (x0 + x1);
                            if ((V(m) < 0.0) == (v0 < 0.0)) x0 = m;
                            else x1 = m;
                        }
                        edges.push_back(0.5 * (x0 + x1));
                    }
                }
                edges.push_back(e);
            }
            std::vector<double> rn, wv;                     // nodes, weight * |V|
            for (size_t i = 0; i + 1 < edges.size(); ++i) {
                const double h = 0.5 * (edges[i + 1] - edges[i]), m = 0.5 * (edges[i + 1] + edges[i]);
                if (h <= 0.0) continue;
                for (size_t j = 0; j < g8.x.size(); ++j) {
                    const double r = m + h * g8.x[j];
                    rn.push_back(r);
                    wv.push_back(h * g8.w[j] * fabs(V(r)));
                }
            }
            // outer panels: r0 in [r_l, r_l + W sigma], split at the coverage radii
            const double hi = r_l + kWindow * sig;
            std::vector<double> oe{r_l};
            if (U.R)
                for (int k = U.l + 1; k < U.n; ++k)
                    if (U.R[k] > r_l && U.R[k] < hi) oe.push_back(U.R[k]);
            oe.push_back(hi);
            const double norm = 1.0 / (sqrt(2.0 * M_PI) * sig);
            double I = 0.0;
            int k_shell = U.l + 1;                            // shell of the current panel
            for (size_t i = 0; i + 1 < oe.size(); ++i) {
                double u = 1.0;
                if (U.R) {
                    while (k_shell < U.n && U.R[k_shell] <= oe[i]) ++k_shell;
                    u = (k_shell < U.n) ? U.at_shell(k_shell) : 1.0;
                }
                if (u == 0.0) continue;
                const int np = std::max(1, (int)ceil((oe[i + 1] - oe[i]) / (0.5 * sig)));
                for (int q = 0; q < np; ++q) {
                    const double x0 = oe[i] + (oe[i + 1] - oe[i]) * q / np;
                    const double x1 = oe[i] + (oe[i + 1] - oe[i]) * (q + 1) / np;
                    const double h = 0.5 * (x1 - x0), m = 0.5 * (x1 + x0);
                    for (size_t j = 0; j < g16.x.size(); ++j) {
                        const double r0 = m + h * g16.x[j];
                        double J = 0.0;
                        for (size_t z = 0; z < rn.size(); ++z) {
                            const double d = (rn[z] - r0) / sig;
                            J += wv[z] * exp(-0.5 * d * d);
                        }
                        I += h * g16.w[j] * 4.0 * M_PI * r0 * r0 * u * J * norm;
                    }
                }
            }
            total += 0.5 * (double)in.count[a] * ((double)in.count[b] / in.volume) * I;
        }
    return total / (double)n_all;
}

nb_status check_input(const nb_params* p, const nb_buffer_input* in, int steps) {
    if (!p || !in || steps < 1) return NB_ERR_ARG;
    if (!(p->rc > 0.f) || p->n_types < 1) return NB_ERR_ARG;
    if (in->n_classes < 0 || (in->n_classes > 0 && (!in->count || !in->mass || !in->charge ||
                                                   !in->type || !in->lj)))
        return NB_ERR_ARG;
    if (!(in->volume > 0.0) || !(in->temperature >= 0.0) || !(in->dt >= 0.0)) return NB_ERR_ARG;
    for (int a = 0; a < in->n_classes; ++a)
        if (in->count[a] < 0 || !(in->mass[a] > 0.0) || in->type[a] < 0 ||
            in->type[a] >= p->n_types || !isfinite(in->charge[a]))
            return NB_ERR_ARG;
    if (in->rot_len)
        for (int a = 0; a < in->n_classes; ++a) {
            if (!(in->rot_len[a] >= 0.0) || !isfinite(in->rot_len[a])) return NB_ERR_ARG;
            if (in->rot_len[a] > 0.0 && (!in->rot_mass || !(in->rot_mass[a] > 0.0)))
                return NB_ERR_ARG;
        }
    if (in->n_cov < 0 || in->n_cov > NB_CENSUS_MAX_RADII) return NB_ERR_ARG;
    if (in->n_cov > 0) {
        if (!in->cov_radii || !in->covered) return NB_ERR_ARG;
        for (int k = 1; k < in->n_cov; ++k)
            if (!(in->cov_radii[k] > in->cov_radii[k - 1])) return NB_ERR_ARG;
    }
    return NB_OK;
}

// Coverage row of a list radius: the table index whose radius equals r_l.
int coverage_row(const nb_buffer_input& in, double r_l) {
    for (int k = 0; k < in.n_cov; ++k)
        if ((float)r_l == in.cov_radii[k]) return k;
    return -1;
}

}  // namespace

extern "C" {

nb_status nb_buffer_drift(const nb_params* p, const nb_buffer_input* in, int32_t steps,
                          double r_list, double* drift) {
    nb_status st = check_input(p, in, steps);
    if (st != NB_OK) return st;
    if (!drift || !(r_list >= p->rc) || !isfinite(r_list)) return NB_ERR_ARG;
    Uncovered U;
    if (in->n_cov > 0) {
        U.n = in->n_cov;
        U.R = in->cov_radii;
        U.cov = in->covered;
        U.l = coverage_row(*in, r_list);
        if (U.l < 0) return NB_ERR_ARG;           // a cluster list radius must be in the table
    }
    *drift = missed_energy(*p, *in, steps, r_list, U) / (steps * in->dt);
    if (!isfinite(*drift)) *drift = 0.0;          // steps == 1 or dt == 0: nothing moves
    return NB_OK;
}

nb_status nb_buffer_estimate(const nb_params* p, const nb_buffer_input* in, int32_t steps,
                             double tolerance, double max_buffer, double* r_list,
                             double* drift) {
    nb_status st = check_input(p, in, steps);
    if (st != NB_OK) return st;
    if (!r_list || !(tolerance > 0.0) || !(max_buffer >= 0.0)) return NB_ERR_ARG;
    const double rc = p->rc;
    double d = 0.0;
    if (in->n_cov > 0) {
        // cluster list: the smallest tabulated radius >= rc within the tolerance
        for (int k = 0; k < in->n_cov; ++k) {
            const double r = in->cov_radii[k];
            if (r < (double)(float)rc || r > rc + max_buffer) continue;
            st = nb_buffer_drift(p, in, steps, r, &d);
            if (st != NB_OK) return st;
            if (d <= tolerance) {
                *r_list = r;
                if (drift) *drift = d;
                return NB_OK;
            }
        }
        return NB_ERR_CAPACITY;                   // not reached inside the table
    }
    // particle list: bisection on the buffer (the drift falls as the radius grows)
    st = nb_buffer_drift(p, in, steps, rc, &d);
    if (st != NB_OK) return st;
    if (d <= tolerance) {
        *r_list = rc;
        if (drift) *drift = d;
        return NB_OK;
    }
    double lo = rc, hi = rc + max_buffer, dh = 0.0;
    st = nb_buffer_drift(p, in, steps, hi, &dh);
    if (st != NB_OK) return st;
    if (dh > tolerance) return NB_ERR_CAPACITY;
    while (hi - lo > 1e-6) {
        const double m = 0.5 * (lo + hi);
        double dm = 0.0;
        st = nb_buffer_drift(p, in, steps, m, &dm);
        if (st != NB_OK) return st;
        if (dm <= tolerance) {
            hi = m;
            dh = dm;
        } else {
            lo = m;
        }
    }
    *r_list = hi;
    if (drift) *drift = dh;
    return NB_OK;
}

}  // extern "C"
