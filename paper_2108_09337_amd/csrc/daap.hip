// General I/O lower bound of a DAAP statement and of a program of several
// statements (Sec. 3 and 4), host code.
//
// A statement is described by its loop nest depth l, its input accesses
// (each the set of distinct iteration variables that index it, with a
// dominator weight: 1, or 1/rho_S when the access reads the output of a
// producer statement S, Corollary of Sec. 4.2) and its number of compute
// vertices |V|.  Sec. 3.2 bounds the largest subcomputation whose dominator
// set has X vertices by
//     chi(X) = max prod_t D_t  s.t.  sum_j w_j prod_{t in access j} D_t <= X,
//                                     D_t >= 1,
// the computational intensity by rho = min_{X > M} chi(X) / (X - M) (and
// by 1/u when every compute vertex has u out-degree-one input
// predecessors), and the I/O cost by Q >= |V| / rho.  The extents D_t at
// the minimizing X_0 are the shape of an I/O-optimal tile for a fast memory
// of M elements.
//
// chi(X) is a geometric program: in y_t = ln D_t it maximizes sum_t y_t
// over the convex set h(y) = ln sum_j w_j exp(a_j . y) <= ln X, y >= 0.
// It is solved here by a logarithmic barrier with damped Newton steps (the
// barrier's duality gap, (l + 1) mu, bounds the error of ln chi); rho is
// minimized over ln X by golden-section search between the smallest
// feasible X and 2^40 M.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

namespace {

constexpr int kMaxVars = CDF_DAAP_MAX_VARS;
constexpr int kMaxAcc = CDF_DAAP_MAX_ACCESSES;

bool valid(const cdf_daap_statement_t *s) {
    if (!s || s->nvars < 1 || s->nvars > kMaxVars || s->naccesses < 1 || s->naccesses > kMaxAcc) return false;
    if (s->u < 0 || !(s->nvertices >= 0.0)) return false;
    unsigned covered = 0;
    for (int j = 0; j < s->naccesses; ++j) {
        const unsigned v = s->access_vars[j];
        if (v == 0 || (v >> s->nvars) != 0) return false;
        if (!(s->access_weight[j] > 0.0) || !std::isfinite(s->access_weight[j])) return false;
        covered |= v;
    }
    // a variable that indexes no access could grow without bound
    return covered == (1u << s->nvars) - 1u;
}

double weight_sum(const cdf_daap_statement_t *s) {
    double w = 0.0;
    for (int j = 0; j < s->naccesses; ++j) w += s->access_weight[j];
    return w;
}

struct Hval {
    double h;             // ln sum_j w_j e^{a_j . y}
    double g[kMaxVars];   // gradient
    double H[kMaxVars][kMaxVars];  // Hessian
};

void eval_h(const cdf_daap_statement_t *s, const double *y, Hval &o) {
    const int l = s->nvars, m = s->naccesses;
    double e[kMaxAcc], emax = -INFINITY;
    for (int j = 0; j < m; ++j) {
        double d = std::log(s->access_weight[j]);
        for (int t = 0; t < l; ++t)
            if (s->access_vars[j] >> t & 1u) d += y[t];
        e[j] = d;
        emax = std::max(emax, d);
    }
    double sum = 0.0, p[kMaxAcc];
    for (int j = 0; j < m; ++j) sum += (p[j] = std::exp(e[j] - emax));
    o.h = emax + std::log(sum);
    for (int j = 0; j < m; ++j) p[j] /= sum;
    for (int t = 0; t < l; ++t) {
        o.g[t] = 0.0;
        for (int j = 0; j < m; ++j)
            if (s->access_vars[j] >> t & 1u) o.g[t] += p[j];
    }
    for (int t = 0; t < l; ++t)
        for (int r = 0; r < l; ++r) {
            double v = 0.0;
            for (int j = 0; j < m; ++j)
                if ((s->access_vars[j] >> t & 1u) && (s->access_vars[j] >> r & 1u)) v += p[j];
            o.H[t][r] = v - o.g[t] * o.g[r];
        }
}

// Solves A x = b for a symmetric positive definite A (n <= 8) by Cholesky;
// false if A is not numerically positive definite.
bool spd_solve(int n, double A[kMaxVars][kMaxVars], const double *b, double *x) {
    double L[kMaxVars][kMaxVars] = {};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = A[i][j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(v > 0.0)) return false;
                L[i][i] = std::sqrt(v);
            } else {
                L[i][j] = v / L[j][j];
            }
        }
    double z[kMaxVars];
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * z[k];
        z[i] = v / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = z[i];
        for (int k = i + 1; k < n; ++k) v -= L[k][i] * x[k];
        x[i] = v / L[i][i];
    }
    return true;
}

// Dense solve of the (n x n, n <= 9) system J x = r by Gaussian elimination
// with partial pivoting; false if J is singular.
bool dense_solve(int n, double J[kMaxVars + 1][kMaxVars + 1], double *r, double *x) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(J[i][k]) > std::fabs(J[p][k])) p = i;
        if (!(std::fabs(J[p][k]) > 1e-300)) return false;
        if (p != k) {
            for (int c = 0; c < n; ++c) std::swap(J[k][c], J[p][c]);
            std::swap(r[k], r[p]);
        }
        for (int i = k + 1; i < n; ++i) {
            const double f = J[i][k] / J[k][k];
            for (int c = k; c < n; ++c) J[i][c] -= f * J[k][c];
            r[i] -= f * r[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = r[i];
        for (int c = i + 1; c < n; ++c) v -= J[i][c] * x[c];
        x[i] = v / J[i][i];
    }
    return true;
}

// Active-set polish of the barrier's point.  The barrier approaches a
// bound y_t = 0 only slowly where the objective is flat, so the optimality
// conditions are solved directly: the k variables the barrier left smallest
// are fixed at 0 (k = 0, 1, ... in turn) and Newton's method solves
//     lambda dh/dy_t = 1 (t free),  h(y) = c
// for the rest.  A solution with every free y_t >= 0 and lambda dh/dy_t >= 1
// for every fixed t (freeing it would not help) is optimal for the convex
// program; the first such one replaces the barrier's point if its objective
// is not smaller.
void polish(const cdf_daap_statement_t *s, double c, double *y) {
    const int l = s->nvars;
    int order[kMaxVars];
    for (int t = 0; t < l; ++t) order[t] = t;
    std::sort(order, order + l, [&](int a, int b) { return y[a] < y[b]; });
    double y0 = 0.0;
    for (int t = 0; t < l; ++t) y0 += y[t];
    for (int nfix = 0; nfix < l; ++nfix) {
        bool fixed[kMaxVars] = {};
        for (int q = 0; q < nfix; ++q) fixed[order[q]] = true;
        int F[kMaxVars], nf = 0;
        double z[kMaxVars];
        for (int t = 0; t < l; ++t) {
            z[t] = fixed[t] ? 0.0 : y[t];
            if (!fixed[t]) F[nf++] = t;
        }
        Hval hv;
        eval_h(s, z, hv);
        double lam = 0.0;
        for (int q = 0; q < nf; ++q) lam += 1.0 / hv.g[F[q]];
        lam /= nf;
        bool ok = false;
        for (int it = 0; it < 80; ++it) {
            eval_h(s, z, hv);
            double J[kMaxVars + 1][kMaxVars + 1] = {}, r[kMaxVars + 1], d[kMaxVars + 1];
            double res = std::fabs(hv.h - c) / std::max(1.0, std::fabs(c));
            for (int q = 0; q < nf; ++q) {
                const int t = F[q];
                r[q] = -(lam * hv.g[t] - 1.0);
                res = std::max(res, std::fabs(r[q]));
                for (int q2 = 0; q2 < nf; ++q2) J[q][q2] = lam * hv.H[t][F[q2]];
                J[q][nf] = hv.g[t];
                J[nf][q] = hv.g[t];
            }
            r[nf] = -(hv.h - c);
            if (res < 1e-14) { ok = true; break; }
            if (!dense_solve(nf + 1, J, r, d)) break;
            for (int q = 0; q < nf; ++q) z[F[q]] += d[q];
            lam += d[nf];
        }
        if (!ok || !(lam > 0.0)) continue;
        bool good = true;
        for (int q = 0; q < nf; ++q) good &= z[F[q]] >= 0.0;
        eval_h(s, z, hv);
        for (int t = 0; t < l; ++t)
            if (fixed[t]) good &= lam * hv.g[t] >= 1.0 - 1e-10;
        if (!good) continue;
        double y1 = 0.0;
        for (int t = 0; t < l; ++t) y1 += z[t];
        if (y1 >= y0 - 1e-12 * std::max(1.0, y0))
            for (int t = 0; t < l; ++t) y[t] = z[t];
        return;
    }
}

// F_mu(y) = sum y + mu (ln(c - h(y)) + sum ln y); -inf outside the domain.
double barrier(const cdf_daap_statement_t *s, const double *y, double c, double mu) {
    double f = 0.0, lg = 0.0;
    for (int t = 0; t < s->nvars; ++t) {
        if (!(y[t] > 0.0)) return -INFINITY;
        f += y[t];
        lg += std::log(y[t]);
    }
    Hval hv;
    eval_h(s, y, hv);
    if (!(c - hv.h > 0.0)) return -INFINITY;
    return f + mu * (std::log(c - hv.h) + lg);
}

// chi(X) and the extents D_t; X must exceed the weight sum.
double solve_chi(const cdf_daap_statement_t *s, double X, double *tile) {
    const int l = s->nvars;
    const double c = std::log(X);
    const double c0 = std::log(weight_sum(s));
    int maxdeg = 1;
    for (int j = 0; j < s->naccesses; ++j) maxdeg = std::max(maxdeg, __builtin_popcount(s->access_vars[j]));
    double y[kMaxVars];
    const double eps = std::min(1.0, (c - c0) / (2.0 * maxdeg));
    for (int t = 0; t < l; ++t) y[t] = eps;
    for (double mu = 1.0; mu > 1e-15; mu *= 0.125) {
        for (int it = 0; it < 100; ++it) {
            Hval hv;
            eval_h(s, y, hv);
            const double gap = c - hv.h;
            double g[kMaxVars], N[kMaxVars][kMaxVars], d[kMaxVars];
            for (int t = 0; t < l; ++t) g[t] = 1.0 - mu * hv.g[t] / gap + mu / y[t];
            // N = -Hessian of F (positive definite)
            for (int t = 0; t < l; ++t)
                for (int r = 0; r < l; ++r)
                    N[t][r] = mu * (hv.H[t][r] / gap + hv.g[t] * hv.g[r] / (gap * gap)) +
                              (t == r ? mu / (y[t] * y[t]) : 0.0);
            if (!spd_solve(l, N, g, d)) break;
            double dec = 0.0;  // Newton decrement squared
            for (int t = 0; t < l; ++t) dec += g[t] * d[t];
            if (dec < 1e-20) break;
            const double f0 = barrier(s, y, c, mu);
            double a = 1.0, yn[kMaxVars];
            for (int ls = 0; ls < 60; ++ls, a *= 0.5) {
                for (int t = 0; t < l; ++t) yn[t] = y[t] + a * d[t];
                const double f1 = barrier(s, yn, c, mu);
                if (f1 >= f0 + 0.25 * a * dec) break;
            }
            if (!(barrier(s, yn, c, mu) > -INFINITY)) break;
            for (int t = 0; t < l; ++t) y[t] = yn[t];
            if (dec < 1e-18 * (1.0 + std::fabs(f0))) break;
        }
    }
    polish(s, c, y);
    double sum = 0.0;
    for (int t = 0; t < l; ++t) {
        sum += y[t];
        if (tile) tile[t] = std::exp(y[t]);
    }
    return std::exp(sum);
}

void fill_result(const cdf_daap_statement_t *s, double M, double x0, cdf_daap_result_t *r) {
    *r = cdf_daap_result_t{};
    r->x0 = x0;
    r->chi = solve_chi(s, x0, r->tile);
    r->rho = r->chi / (x0 - M);
    if (s->u > 0) r->rho = std::min(r->rho, 1.0 / s->u);
    r->q = s->nvertices / r->rho;
    for (int j = 0; j < s->naccesses; ++j) {
        double v = s->access_weight[j];
        for (int t = 0; t < s->nvars; ++t)
            if (s->access_vars[j] >> t & 1u) v *= r->tile[t];
        r->access[j] = v;
    }
}

}  // namespace

extern "C" {

cdf_status_t cdf_daap_chi(const cdf_daap_statement_t *s, double X, double *chi, double *tile) {
    if (!valid(s) || !chi) return CDF_ERR_INVALID_ARG;
    if (!(X > weight_sum(s)) || !std::isfinite(X)) return CDF_ERR_INVALID_ARG;
    *chi = solve_chi(s, X, tile);
    return CDF_OK;
}

cdf_status_t cdf_daap_statement_bound(const cdf_daap_statement_t *s, double M, cdf_daap_result_t *r) {
    if (!valid(s) || !r || !(M > 0.0) || !std::isfinite(M)) return CDF_ERR_INVALID_ARG;
    const double lo = std::log(std::max(M, weight_sum(s)) * (1.0 + 1e-9));
    const double hi = std::log(M) + 40.0 * std::log(2.0);
    auto rho_at = [&](double lx) {
        const double x = std::exp(lx);
        return solve_chi(s, x, nullptr) / (x - M);
    };
    // golden-section search for the minimum of rho over ln X
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = lo, b = hi;
    double x1 = b - g * (b - a), x2 = a + g * (b - a);
    double f1 = rho_at(x1), f2 = rho_at(x2);
    for (int it = 0; it < 200 && b - a > 1e-12; ++it) {
        if (f1 <= f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - g * (b - a);
            f1 = rho_at(x1);
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + g * (b - a);
            f2 = rho_at(x2);
        }
    }
    fill_result(s, M, std::exp(0.5 * (a + b)), r);
    return CDF_OK;
}

cdf_status_t cdf_daap_program_bound(int nstatements, const cdf_daap_statement_t *s, double M, double *q) {
    if (nstatements < 1 || !s || !q) return CDF_ERR_INVALID_ARG;
    double total = 0.0;
    std::map<int, std::vector<double>> loads;  // array id -> loads of it by each statement alone
    for (int i = 0; i < nstatements; ++i) {
        cdf_daap_result_t r;
        const cdf_status_t st = cdf_daap_statement_bound(s + i, M, &r);
        if (st != CDF_OK) return st;
        total += r.q;
        const double nsub = s[i].nvertices / r.chi;  // subcomputations of the optimal schedule
        for (int j = 0; j < s[i].naccesses; ++j) loads[s[i].array_id[j]].push_back(r.access[j] * nsub);
    }
    // Case I: of the loads of a shared input array, at least the largest
    // single statement's remain
    for (auto &kv : loads) {
        const std::vector<double> &v = kv.second;
        if (v.size() < 2) continue;
        double sum = 0.0, mx = 0.0;
        for (double x : v) {
            sum += x;
            mx = std::max(mx, x);
        }
        total -= sum - mx;
    }
    *q = total;
    return CDF_OK;
}

}  // extern "C"
