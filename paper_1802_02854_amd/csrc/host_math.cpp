// Host-side scalar mathematics of the FTKw path: cluster geometry, bond table,
// S_Q phase factors, the Appendix-A Taylor plan, the shell coefficients of the
// contour filters (Sec. III.B) and the reweighting of Sec. III.D.
//
// Built with -ffp-contract=off: each expression below is a fixed sequence of
// IEEE double operations, which is part of the library's arithmetic contract
// (the shell coefficients seed long Lanczos runs, so they must be reproducible
// bit for bit by any implementation of the contract).
#include <algorithm>
#include <cmath>
#include <vector>
#include <cstring>
#include <limits>
#include <numeric>
#include <set>
#include <utility>

#include "ftkw_internal.h"

namespace ftk {

namespace {
long floordiv(long a, long b)
{
    long q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

// a x + b y = g = gcd(a, b) >= 0
void egcd(long a, long b, long &g, long &x, long &y)
{
    long x0 = 1, y0 = 0, x1 = 0, y1 = 1;
    while (b != 0) {
        long k = floordiv(a, b);
        long t = a - k * b;
        a = b;
        b = t;
        t = x0 - k * x1;
        x0 = x1;
        x1 = t;
        t = y0 - k * y1;
        y0 = y1;
        y1 = t;
    }
    if (a < 0) {
        a = -a;
        x0 = -x0;
        y0 = -y0;
    }
    g = a;
    x = x0;
    y = y0;
}

long posmod(long a, long b)
{
    long r = a % b;
    return r < 0 ? r + b : r;
}
}  // namespace

HoneyCluster honeycomb(int t11, int t12, int t21, int t22)
{
    long det = (long)t11 * t22 - (long)t12 * t21;
    if (det == 0) fail(FTK_EINVAL, "degenerate supercell");
    HoneyCluster cl;
    long n_cells = det < 0 ? -det : det;
    if (2 * n_cells > kMaxSites) fail(FTK_EINVAL, "supercell has more than 30 sites");
    long p, m, n;
    egcd(t11, t21, p, m, n);
    if (p == 0) fail(FTK_EINVAL, "degenerate supercell");
    long q = n_cells / p;
    long s = posmod(m * t12 + n * t22, q);
    cl.n_cells = (int)n_cells;
    cl.p = (int)p;
    cl.q = (int)q;
    cl.s = (int)s;
    auto cell_index = [&](long c1, long c2) {
        long k = floordiv(c1, p);
        c1 -= k * p;
        c2 -= k * s;
        c2 = posmod(c2, q);
        return c1 + p * c2;
    };
    const double h = std::sqrt(3.0) / 2.0;
    cl.xy.assign(4 * n_cells, 0.0);
    for (long c = 0; c < n_cells; ++c) {
        long c1 = c % p, c2 = c / p;
        double xa = 1.5 * (double)c1 + 1.5 * (double)c2;
        double ya = h * (double)(c2 - c1);
        cl.xy[4 * c + 0] = xa;
        cl.xy[4 * c + 1] = ya;
        cl.xy[4 * c + 2] = xa + 1.0;
        cl.xy[4 * c + 3] = ya;
        int A = (int)(2 * c);
        cl.bi.push_back(A), cl.bj.push_back((int)(2 * cell_index(c1 - 1, c2) + 1)), cl.gamma.push_back(0);
        cl.bi.push_back(A), cl.bj.push_back((int)(2 * cell_index(c1, c2 - 1) + 1)), cl.gamma.push_back(1);
        cl.bi.push_back(A), cl.bj.push_back(A + 1), cl.gamma.push_back(2);
    }
    std::set<std::pair<int, int>> seen;
    for (size_t b = 0; b < cl.bi.size(); ++b) {
        auto key = std::make_pair(std::min(cl.bi[b], cl.bj[b]), std::max(cl.bi[b], cl.bj[b]));
        if (!seen.insert(key).second) fail(FTK_EINVAL, "supercell too small: two bonds join the same pair of sites");
    }
    return cl;
}

static void momentum_xy(long f1, long f2, long den, double *q)
{
    const double tp3 = 2.0 * M_PI / 3.0;
    const double tps = 2.0 * M_PI / std::sqrt(3.0);
    q[0] = tp3 * ((double)(f1 + f2) / (double)den);
    q[1] = tps * ((double)(f2 - f1) / (double)den);
}

std::vector<double> honeycomb_momenta(int t11, int t12, int t21, int t22)
{
    long det = (long)t11 * t22 - (long)t12 * t21;
    if (det == 0) fail(FTK_EINVAL, "degenerate supercell");
    if (det < 0) det = -det;
    std::vector<double> out;
    static const int shifts[5] = {0, -1, 1, -2, 2};
    for (long a = 0; a < det; ++a)
        for (long b = 0; b < det; ++b) {
            if (posmod(t11 * a + t12 * b, det) || posmod(t21 * a + t22 * b, det)) continue;
            long best_r2 = 0, bf1 = 0, bf2 = 0;
            bool have = false;
            for (int i : shifts)
                for (int j : shifts) {
                    long f1 = a - i * det, f2 = b - j * det;
                    // |f1 b1 + f2 b2|^2 ~ f1^2 + f2^2 - f1 f2 (b1, b2 are 120 degrees apart)
                    long r2 = f1 * f1 + f2 * f2 - f1 * f2;
                    if (!have || r2 < best_r2) {
                        have = true;
                        best_r2 = r2;
                        bf1 = f1;
                        bf2 = f2;
                    }
                }
            double q[2];
            momentum_xy(bf1, bf2, det, q);
            out.push_back(q[0]);
            out.push_back(q[1]);
        }
    return out;
}

bool named_momentum(const std::string &name, double *q)
{
    if (name == "Gamma") return momentum_xy(0, 0, 1, q), true;
    if (name == "M") return momentum_xy(1, 1, 2, q), true;
    if (name == "K") return momentum_xy(2, 1, 3, q), true;
    if (name == "M'") return momentum_xy(1, 0, 2, q), true;
    return false;
}

// --------------------------------------------------------------------------
// Bond table of the KH Hamiltonian (Sec. V.A): per bond, with c_a = J for a
// different from the bond's gamma and J + K for a == gamma, the two-spin flip
// amplitude is (c_x - c_y)/4 for parallel spins and (c_x + c_y)/4 otherwise.
BondTable make_bond_table(const ftk_cluster &c, double K, double J)
{
    if (c.n_sites < 4 || c.n_sites > kMaxSites) fail(FTK_EINVAL, "n_sites must be in [4, 30]");
    if (c.n_bonds < 1 || c.n_bonds > kMaxBonds) fail(FTK_EINVAL, "n_bonds must be in [1, 45]");
    if (!c.bond_i || !c.bond_j || !c.bond_gamma || !c.site_xy) fail(FTK_EINVAL, "cluster arrays must not be NULL");
    if (!std::isfinite(K) || !std::isfinite(J)) fail(FTK_EINVAL, "K and J must be finite");
    BondTable t;
    t.n_sites = c.n_sites;
    t.n_bonds = c.n_bonds;
    std::set<std::pair<int, int>> seen;
    for (int b = 0; b < c.n_bonds; ++b) {
        int i = c.bond_i[b], j = c.bond_j[b], g = c.bond_gamma[b];
        if (i < 0 || j < 0 || i >= c.n_sites || j >= c.n_sites || i == j)
            fail(FTK_EINVAL, "bond endpoint out of range or repeated");
        if (g < 0 || g > 2) fail(FTK_EINVAL, "bond gamma must be 0, 1 or 2");
        if (!seen.insert({std::min(i, j), std::max(i, j)}).second) fail(FTK_EINVAL, "repeated bond");
        double cc[3] = {J, J, J};
        cc[g] = J + K;
        t.bi[b] = i;
        t.bj[b] = j;
        t.gamma[b] = (int8_t)g;
        t.ap[b] = (cc[0] - cc[1]) / 4.0;
        t.aa[b] = (cc[0] + cc[1]) / 4.0;
        // bond eigenvalues (c_z +- (c_x - c_y))/4, (-c_z + c_x + c_y)/4, (-c_z - c_x - c_y)/4
        double cx = cc[0], cy = cc[1], cz = cc[2];
        double ev[4] = {(cz + cx - cy) / 4, (cz - cx + cy) / 4, (-cz + cx + cy) / 4, (-cz - cx - cy) / 4};
        double mx = 0.0;
        for (double e : ev) mx = std::max(mx, std::fabs(e));
        t.norm_bound = t.norm_bound + mx;
    }
    t.jq = J / 4.0;
    t.kq = K / 4.0;
    for (int l = 0; l < c.n_sites; ++l)
        if (!std::isfinite(c.site_xy[2 * l]) || !std::isfinite(c.site_xy[2 * l + 1]))
            fail(FTK_EINVAL, "site_xy must be finite");
    return t;
}

void sq_coefficients(int n_sites, const double *site_xy, double qx, double qy, double *h)
{
    const double s = 0.5 / std::sqrt((double)n_sites);
    for (int l = 0; l < n_sites; ++l) {
        double th = qx * site_xy[2 * l] + qy * site_xy[2 * l + 1];
        h[2 * l] = std::cos(th) * s;
        h[2 * l + 1] = std::sin(th) * s;
    }
}

// --------------------------------------------------------------------------
// Appendix A: M_d factors e^{c (l - h)}, c = N beta / (2 M_d), each a Taylor
// series of K terms.  X solves e^X / sqrt(2 pi X) = Lambda (the recurrence of
// the appendix, iterated 200 times); l = B_H/N and |e_0| = B_H/N bound the
// spectrum of h = H/N; the series stops at the first k > X' with X'^k/k! < 1e-18.
TaylorPlan taylor_plan(int n_sites, double beta, double norm_bound, double lambda)
{
    TaylorPlan p;
    const double N = (double)n_sites;
    p.ell = norm_bound / N;
    if (beta == 0.0) return p;
    const double width = 2.0 * norm_bound / N;
    double x = lambda;
    for (int i = 0; i < 200; ++i) x = std::log(lambda) + 0.5 * std::log(2.0 * M_PI * x);
    double md = std::ceil(N * beta * width / (2.0 * x));
    p.Md = md < 1.0 ? 1 : (int)md;
    p.c = N * beta / (2.0 * (double)p.Md);
    const double xs = p.c * width;
    double tau = 1.0;
    int k = 0;
    while (true) {
        ++k;
        tau = tau * xs / (double)k;
        if (((double)k > xs && tau < 1e-18) || k >= 400) break;
    }
    p.K = k;
    return p;
}

// --------------------------------------------------------------------------
// Sec. III.B: phi^m = P_{E_m, eps, M} phi_beta with P of Eq. (dfilterP).  In
// the Lanczos basis of phi_beta every resolvent (z - H)^{-1} phi_beta becomes
// ||phi_beta|| V_n (z - T_n)^{-1} e_1, so phi^m = V_n c^m with
//   c^m = (||phi_beta|| / M) sum_j w_j y_mj,  (z_mj - T_n) y_mj = e_1,
//   w_j = eps e^{i th_j}, z_mj = E_m + w_j.
// Each system is solved by elimination without pivoting (|pivot| >= Im z > 0).
double shell_energy(double E_b, double eps, int m) { return E_b + (double)(2 * m + 1) * eps; }

namespace {

// The largest Galerkin residual over the shifts after each step k = 0..n-1 (the
// device's multi-shift recurrence); visit(k, rmax) returns true to stop.
template <class Visit>
void scan_residuals(const double *alpha, const double *beta, int n, const double *zr, const double *zi, int nz,
                    Visit &&visit)
{
    std::vector<double> dr(nz), di(nz), pr(nz, 1.0), pi(nz, 0.0);
    for (int k = 0; k < n; ++k) {
        double rmax = 0.0;
        for (int j = 0; j < nz; ++j) {
            if (k == 0) {
                dr[j] = zr[j] - alpha[0];
                di[j] = zi[j];
            } else {
                const double den = dr[j] * dr[j] + di[j] * di[j];
                const double rr = dr[j] / den, ri = -di[j] / den;
                const double fr = beta[k - 1] * rr, fi = beta[k - 1] * ri;
                const double npr = pr[j] * fr - pi[j] * fi;
                const double npi = pr[j] * fi + pi[j] * fr;
                const double b2 = beta[k - 1] * beta[k - 1];
                dr[j] = (zr[j] - alpha[k]) - b2 * rr;
                di[j] = zi[j] - b2 * ri;
                pr[j] = npr;
                pi[j] = npi;
            }
            const double r = std::sqrt((pr[j] * pr[j] + pi[j] * pi[j]) / (dr[j] * dr[j] + di[j] * di[j])) * beta[k];
            rmax = r > rmax ? r : rmax;
        }
        if (visit(k, rmax)) return;
    }
}

}  // namespace

// Residual-controlled truncation (Sec. V: CG steps cut by the largest residual
// 2-norm over the shifts).
int truncation_steps(const double *alpha, const double *beta, int n, const double *zr, const double *zi, int nz,
                     double tol)
{
    int k_stop = n;
    scan_residuals(alpha, beta, n, zr, zi, nz, [&](int k, double rmax) {
        if (rmax <= tol) {
            k_stop = k + 1;
            return true;
        }
        return false;
    });
    return k_stop;
}

// The CG-step dependence of the largest residual 2-norm (Sec. V): out[k] after
// k + 1 steps, per unit right-hand side.
void residual_history(const double *alpha, const double *beta, int n, const double *zr, const double *zi, int nz,
                      double *out)
{
    scan_residuals(alpha, beta, n, zr, zi, nz, [&](int k, double rmax) {
        out[k] = rmax;
        return false;
    });
}

namespace {

// number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots)
int sturm_count(const double *alpha, const double *beta, int n, double x)
{
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
        const double off = i ? beta[i - 1] * beta[i - 1] : 0.0;
        q = (alpha[i] - x) - (i ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;  // x on a pivot: count it as below
        if (q < 0.0) ++c;
    }
    return c;
}

// smallest x with sturm_count(x) >= k, bisected down to adjacent doubles
double bisect(const double *alpha, const double *beta, int n, int k, double lo, double hi)
{
    for (int it = 0; it < 2100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (sturm_count(alpha, beta, n, mid) >= k)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

}  // namespace

void ritz_extremes(const double *alpha, const double *beta, int n, double *lo, double *hi)
{
    // Gershgorin interval, widened so both ends are strict bounds
    double glo = alpha[0], ghi = alpha[0];
    for (int i = 0; i < n; ++i) {
        const double r = (i ? std::fabs(beta[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(beta[i]) : 0.0);
        glo = std::min(glo, alpha[i] - r);
        ghi = std::max(ghi, alpha[i] + r);
    }
    const double pad = 1e-12 * std::max(1.0, ghi - glo);
    glo -= pad;
    ghi += pad;
    *lo = bisect(alpha, beta, n, 1, glo, ghi);
    *hi = bisect(alpha, beta, n, n, glo, ghi);
}

void shell_window(const double *alpha, const double *beta, int n, int L, double margin, double *E_b, double *eps)
{
    double lo, hi;
    ritz_extremes(alpha, beta, n, &lo, &hi);
    *E_b = lo - margin;
    *eps = ((hi + margin) - *E_b) / (2.0 * (double)L);
}

void shell_coefficients(const double *alpha, const double *beta, int n, double nrm, double E_b,
                        double eps, int L, int M, double *out, const int *kn)
{
    std::vector<double> wr(M), wi(M);
    for (int j = 1; j <= M; ++j) {
        double th = 2.0 * M_PI * ((double)j - 0.5) / (double)M;
        wr[j - 1] = eps * std::cos(th);
        wi[j - 1] = eps * std::sin(th);
    }
    std::vector<double> ipr(n), ipi(n), fr(n), fi(n), yr(n), yi(n);
    std::vector<double> accr((size_t)L * n, 0.0), acci((size_t)L * n, 0.0);
    for (int m = 0; m < L; ++m) {
        const double Em = shell_energy(E_b, eps, m);
        double *ar = &accr[(size_t)m * n];
        double *ai = &acci[(size_t)m * n];
        const int nm = kn ? kn[m] : n;  // shell m from T_{nm}; zero beyond
        for (int j = 0; j < M; ++j) {
            const double zr = Em + wr[j];
            const double zi = wi[j];
            double pr = zr - alpha[0];
            double pi = zi;
            double den = pr * pr + pi * pi;
            ipr[0] = pr / den;
            ipi[0] = -pi / den;
            fr[0] = 1.0;
            fi[0] = 0.0;
            for (int k = 1; k < nm; ++k) {
                const double b = beta[k - 1];
                const double lr = b * ipr[k - 1];
                const double li = b * ipi[k - 1];
                pr = (zr - alpha[k]) - b * lr;
                pi = zi - b * li;
                den = pr * pr + pi * pi;
                ipr[k] = pr / den;
                ipi[k] = -pi / den;
                fr[k] = lr * fr[k - 1] - li * fi[k - 1];
                fi[k] = lr * fi[k - 1] + li * fr[k - 1];
            }
            yr[nm - 1] = fr[nm - 1] * ipr[nm - 1] - fi[nm - 1] * ipi[nm - 1];
            yi[nm - 1] = fr[nm - 1] * ipi[nm - 1] + fi[nm - 1] * ipr[nm - 1];
            for (int k = nm - 2; k >= 0; --k) {
                const double b = beta[k];
                const double tr = fr[k] + b * yr[k + 1];
                const double ti = fi[k] + b * yi[k + 1];
                yr[k] = tr * ipr[k] - ti * ipi[k];
                yi[k] = tr * ipi[k] + ti * ipr[k];
            }
            for (int k = 0; k < nm; ++k) {
                const double tr = wr[j] * yr[k] - wi[j] * yi[k];
                const double ti = wr[j] * yi[k] + wi[j] * yr[k];
                ar[k] = ar[k] + tr;
                ai[k] = ai[k] + ti;
            }
        }
    }
    const double s = nrm / (double)M;
    for (int m = 0; m < L; ++m)
        for (int k = 0; k < n; ++k) {
            out[2 * ((size_t)m * n + k)] = accr[(size_t)m * n + k] * s;
            out[2 * ((size_t)m * n + k) + 1] = acci[(size_t)m * n + k] * s;
        }
}

// --------------------------------------------------------------------------
// Sec. III.D, Eqs. (FRW1), (FRW2), with the sample average as a ratio of sums
// (Eq. limGAB); see ftk_reweight in ftkw.h for the exact formula.
namespace {
int pick_anchor(int na, const double *betas, double bt)
{
    int best = -1;
    for (int a = 0; a < na; ++a)
        if (betas[a] <= bt && (best < 0 || betas[a] > betas[best])) best = a;
    if (best < 0) {
        best = 0;
        for (int a = 1; a < na; ++a)
            if (betas[a] < betas[best]) best = a;
    }
    return best;
}
}  // namespace

void reweight(int nv, int na, int L, int nq, int nw, const double *betas, const double *E_m,
              const double *eps, const double *log_norm, const double *n_m, const double *g,
              const double *T, int nT, int n_bins, double *S, double *S_err, double *P)
{
    const double ninf = -std::numeric_limits<double>::infinity();
    const size_t gq = (size_t)nq * nw;  // complex entries per (s, a, m)
    int B = std::min(n_bins <= 0 ? 8 : n_bins, nv);
    std::vector<double> logw((size_t)nv * L);
    std::vector<double> num((size_t)gq), binv;
    for (int it = 0; it < nT; ++it) {
        const double bt = 1.0 / T[it];
        const int a = pick_anchor(na, betas, bt);
        double mx = ninf;
        for (int s = 0; s < nv; ++s)
            for (int m = 0; m < L; ++m) {
                double nm = n_m[((size_t)s * na + a) * L + m];
                double lw = nm > 0 ? 2.0 * log_norm[(size_t)s * na + a] + (betas[a] - bt) * E_m[(size_t)a * L + m] : ninf;
                logw[(size_t)s * L + m] = lw;
                mx = std::max(mx, lw);
            }
        // ratio over a sample range [s0, s1)
        auto ratio = [&](int s0, int s1, double *dst, size_t stride) {
            double lmx = ninf;
            for (int s = s0; s < s1; ++s)
                for (int m = 0; m < L; ++m) lmx = std::max(lmx, logw[(size_t)s * L + m]);
            std::fill(num.begin(), num.end(), 0.0);
            double den = 0.0;
            for (int s = s0; s < s1; ++s)
                for (int m = 0; m < L; ++m) {
                    double lw = logw[(size_t)s * L + m];
                    if (lw == ninf) continue;
                    double w = std::exp(lw - lmx);
                    den += w * n_m[((size_t)s * na + a) * L + m];
                    const double *gp = g + 2 * (((size_t)s * na + a) * L + m) * gq;
                    for (size_t k = 0; k < gq; ++k) num[k] += w * gp[2 * k + 1];
                }
            for (size_t k = 0; k < gq; ++k) dst[k * stride] = -num[k] / (M_PI * den);
        };
        // S[q][it][w]
        std::vector<double> full(gq);
        ratio(0, nv, full.data(), 1);
        for (int q = 0; q < nq; ++q)
            for (int w = 0; w < nw; ++w) S[((size_t)q * nT + it) * nw + w] = full[(size_t)q * nw + w];
        if (P) {
            double tot = 0.0;
            std::vector<double> wn(L, 0.0);
            for (int s = 0; s < nv; ++s)
                for (int m = 0; m < L; ++m) {
                    double lw = logw[(size_t)s * L + m];
                    if (lw == ninf) continue;
                    double v = std::exp(lw - mx) * n_m[((size_t)s * na + a) * L + m];
                    wn[m] += v;
                    tot += v;
                }
            for (int m = 0; m < L; ++m) P[(size_t)it * L + m] = wn[m] / (2.0 * eps[a] * tot);
        }
        if (S_err) {
            if (B < 2) {
                for (int q = 0; q < nq; ++q)
                    for (int w = 0; w < nw; ++w)
                        S_err[((size_t)q * nT + it) * nw + w] = std::numeric_limits<double>::quiet_NaN();
            } else {
                binv.assign((size_t)B * gq, 0.0);
                for (int b = 0; b < B; ++b) ratio(b * nv / B, (b + 1) * nv / B, &binv[(size_t)b * gq], 1);
                for (size_t k = 0; k < gq; ++k) {
                    double mean = 0.0;
                    for (int b = 0; b < B; ++b) mean += binv[(size_t)b * gq + k];
                    mean /= B;
                    double var = 0.0;
                    for (int b = 0; b < B; ++b) {
                        double d = binv[(size_t)b * gq + k] - mean;
                        var += d * d;
                    }
                    var /= (B - 1);
                    size_t q = k / nw, w = k % nw;
                    S_err[((size_t)q * nT + it) * nw + w] = std::sqrt(var) / std::sqrt((double)B);
                }
            }
        }
    }
}

// Eq. FRW1 for real static observables O[s][a][m][k]: sum W O / sum W n per T'.
void reweight_observable(int nv, int na, int L, int K, const double *betas, const double *E_m, const double *log_norm,
                         const double *n_m, const double *O, const double *T, int nT, int n_bins, double *out,
                         double *err)
{
    const double ninf = -std::numeric_limits<double>::infinity();
    const int B = std::min(n_bins <= 0 ? 8 : n_bins, nv);
    auto ratio = [&](int a, double bt, int s0, int s1, double *dst) {
        double mx = ninf;
        for (int s = s0; s < s1; ++s)
            for (int m = 0; m < L; ++m)
                if (n_m[((size_t)s * na + a) * L + m] > 0)
                    mx = std::max(mx, 2.0 * log_norm[(size_t)s * na + a] + (betas[a] - bt) * E_m[(size_t)a * L + m]);
        double den = 0.0;
        for (int k = 0; k < K; ++k) dst[k] = 0.0;
        for (int s = s0; s < s1; ++s)
            for (int m = 0; m < L; ++m) {
                const size_t i = ((size_t)s * na + a) * L + m;
                if (!(n_m[i] > 0)) continue;
                const double w =
                    std::exp(2.0 * log_norm[(size_t)s * na + a] + (betas[a] - bt) * E_m[(size_t)a * L + m] - mx);
                den += w * n_m[i];
                for (int k = 0; k < K; ++k) dst[k] += w * O[i * K + k];
            }
        for (int k = 0; k < K; ++k) dst[k] /= den;
    };
    std::vector<double> v(K), bins((size_t)B * K);
    for (int it = 0; it < nT; ++it) {
        const double bt = 1.0 / T[it];
        const int a = pick_anchor(na, betas, bt);
        ratio(a, bt, 0, nv, v.data());
        for (int k = 0; k < K; ++k) out[(size_t)k * nT + it] = v[k];
        if (!err) continue;
        for (int k = 0; k < K; ++k) err[(size_t)k * nT + it] = std::numeric_limits<double>::quiet_NaN();
        if (B < 2) continue;
        for (int b = 0; b < B; ++b) ratio(a, bt, b * nv / B, (b + 1) * nv / B, &bins[(size_t)b * K]);
        for (int k = 0; k < K; ++k) {
            double mean = 0.0, var = 0.0;
            for (int b = 0; b < B; ++b) mean += bins[(size_t)b * K + k];
            mean /= B;
            for (int b = 0; b < B; ++b) var += (bins[(size_t)b * K + k] - mean) * (bins[(size_t)b * K + k] - mean);
            err[(size_t)k * nT + it] = std::sqrt(var / (B - 1)) / std::sqrt((double)B);
        }
    }
}

// Thermodynamics from the shell data (Sec. II.A for Z at the anchor, Eq. FRW1
// with O = H and H^2); formulas in ftk_thermodynamics (ftkw.h).
namespace {
double log_sum_exp(const std::vector<double> &x)
{
    double mx = -std::numeric_limits<double>::infinity();
    for (double v : x) mx = std::max(mx, v);
    if (mx == -std::numeric_limits<double>::infinity()) return mx;
    double s = 0.0;
    for (double v : x) s += std::exp(v - mx);
    return mx + std::log(s);
}
}  // namespace

namespace {

// <H>, <H^2> and ln Z at inverse temperature bt from anchor a and samples [s0, s1)
// (Sec. II.A and Eq. FRW1 with O = H, H^2)
struct ThermoData {
    int nv, na, L;
    const double *betas, *E_m, *log_norm, *n_m, *h1, *h2;
    int n_sites;

    void moments(int a, double bt, int s0, int s1, double &e1, double &e2, double &lnZ) const
    {
        const double ninf = -std::numeric_limits<double>::infinity();
        std::vector<double> lw, l0, ln2;
        std::vector<size_t> idx;
        for (int s = s0; s < s1; ++s) {
            ln2.push_back(2.0 * log_norm[(size_t)s * na + a]);
            for (int m = 0; m < L; ++m) {
                const size_t i = ((size_t)s * na + a) * L + m;
                if (!(n_m[i] > 0)) continue;
                const double em = E_m[(size_t)a * L + m];
                lw.push_back(2.0 * log_norm[(size_t)s * na + a] + (betas[a] - bt) * em);
                l0.push_back(2.0 * log_norm[(size_t)s * na + a] + std::log(n_m[i]));
                idx.push_back(i);
            }
        }
        double mx = ninf;
        for (double v : lw) mx = std::max(mx, v);
        double den = 0.0, s1m = 0.0, s2m = 0.0;
        for (size_t k = 0; k < idx.size(); ++k) {
            const size_t i = idx[k];
            const double w = std::exp(lw[k] - mx);
            const double em = E_m[(size_t)a * L + i % L];
            den += w * n_m[i];
            s1m += w * (h1 ? h1[i] : em * n_m[i]);
            s2m += w * (h2 ? h2[i] : em * em * n_m[i]);
        }
        e1 = s1m / den;
        e2 = s2m / den;
        lnZ = (double)n_sites * std::log(2.0) + log_sum_exp(ln2) - std::log((double)(s1 - s0)) +
              (std::log(den) + mx) - log_sum_exp(l0);
    }
};

// values [nq] per target from all samples and their binned errors: f(s0, s1, out)
template <class F>
void with_bins(int nv, int n_bins, int nq, double *out, double *err, F &&f)
{
    const int B = std::min(n_bins <= 0 ? 8 : n_bins, nv);
    f(0, nv, out);
    if (!err) return;
    if (B < 2) {
        for (int j = 0; j < nq; ++j) err[j] = std::numeric_limits<double>::quiet_NaN();
        return;
    }
    std::vector<double> bins((size_t)nq * B);
    for (int b = 0; b < B; ++b) f(b * nv / B, (b + 1) * nv / B, &bins[(size_t)nq * b]);
    for (int j = 0; j < nq; ++j) {
        double mean = 0.0, var = 0.0;
        for (int b = 0; b < B; ++b) mean += bins[(size_t)nq * b + j];
        mean /= B;
        for (int b = 0; b < B; ++b) var += (bins[(size_t)nq * b + j] - mean) * (bins[(size_t)nq * b + j] - mean);
        err[j] = std::sqrt(var / (B - 1)) / std::sqrt((double)B);
    }
}

}  // namespace

void thermodynamics(int nv, int na, int L, const double *betas, const double *E_m, const double *log_norm,
                    const double *n_m, const double *h1, const double *h2, int n_sites, const double *T, int nT,
                    int n_bins, double *out, double *err)
{
    const ThermoData d{nv, na, L, betas, E_m, log_norm, n_m, h1, h2, n_sites};
    for (int it = 0; it < nT; ++it) {
        const double bt = 1.0 / T[it];
        const int a = pick_anchor(na, betas, bt);
        with_bins(nv, n_bins, 4, out + 4 * (size_t)it, err ? err + 4 * (size_t)it : nullptr,
                  [&](int s0, int s1, double *q) {
                      double e1, e2, lnZ;
                      d.moments(a, bt, s0, s1, e1, e2, lnZ);
                      q[0] = e1;
                      q[1] = bt * bt * (e2 - e1 * e1);
                      q[2] = bt * e1 + lnZ;
                      q[3] = lnZ;
                  });
    }
}

void thermo_diagnostics(int nv, int na, int L, const double *betas, const double *E_m, const double *log_norm,
                        const double *n_m, const double *h1, const double *h2, int n_sites, const double *inv_T,
                        int nT, int n_bins, double *out, double *err)
{
    const ThermoData d{nv, na, L, betas, E_m, log_norm, n_m, h1, h2, n_sites};
    for (int it = 0; it < nT; ++it) {
        const double b = inv_T[it];
        const int a1 = pick_anchor(na, betas, b), a2 = pick_anchor(na, betas, 2.0 * b);
        with_bins(nv, n_bins, 2, out + 2 * (size_t)it, err ? err + 2 * (size_t)it : nullptr,
                  [&](int s0, int s1, double *q) {
                      double e1, e2, lz1, f1, f2, lz2;
                      d.moments(a1, b, s0, s1, e1, e2, lz1);
                      d.moments(a2, 2.0 * b, s0, s1, f1, f2, lz2);
                      q[0] = e2 - e1 * e1;
                      q[1] = lz2 - 2.0 * lz1;
                  });
    }
}

double overlap_ratio(double E1, double var1, double E2, double var2)
{
    return std::fabs(E1 - E2) / (std::sqrt(var1) + std::sqrt(var2));
}

int choose_anchors(int n, const double *E, const double *var, double r_max, int max_anchors, int *anchors)
{
    int k = 0, i = 0;
    anchors[k++] = 0;
    while (k < max_anchors) {
        int j = i + 1;
        while (j < n && overlap_ratio(E[i], var[i], E[j], var[j]) <= r_max) ++j;
        if (j >= n) break;
        anchors[k++] = j;
        i = j;
    }
    return k;
}

namespace {

// xorshift64*: the annealer's own deterministic stream
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return s * 2685821657736338717ull;
    }
    int below(int n) { return (int)(next() % (uint64_t)n); }
    double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Assignment of bonds to P passes and a core set: cost = sites over the tile
// limit, summed over passes.
struct Layout {
    int N, nb, P, t, c;
    const int32_t *bi, *bj;
    std::vector<int> pass;              // bond -> pass
    std::vector<int> count;             // [P][N] bonds of pass p at site l
    std::vector<char> core;             // [N]
    std::vector<int> nsites;            // [P] sites of pass p outside the core
    int ncore = 0;

    int over(int p) const { return std::max(0, nsites[p] + ncore - t); }
    int cost() const
    {
        int c0 = 0;
        for (int p = 0; p < P; ++p) c0 += over(p);
        return c0;
    }
    void add(int b, int p, int d)
    {
        for (int l : {bi[b], bj[b]}) {
            int &k = count[(size_t)p * N + l];
            if (!core[l] && ((k == 0 && d > 0) || (k == 1 && d < 0))) nsites[p] += d;
            k += d;
        }
    }
    void set_core(int l, bool in)
    {
        core[l] = in;
        ncore += in ? 1 : -1;
        for (int p = 0; p < P; ++p)
            if (count[(size_t)p * N + l] > 0) nsites[p] += in ? -1 : 1;
    }
};

bool anneal(Layout &L, Rng &rng, long iters)
{
    int cc = L.cost();
    double temp = 2.0;
    const double cool = std::pow(0.01 / temp, 1.0 / (double)iters);
    for (long it = 0; it < iters && cc > 0; ++it, temp *= cool) {
        if (rng.below(10) < 9) {
            const int b = rng.below(L.nb), p0 = L.pass[b], p1 = rng.below(L.P);
            if (p0 == p1) continue;
            L.add(b, p0, -1);
            L.add(b, p1, +1);
            const int nc = L.cost();
            if (nc <= cc || rng.unit() < std::exp((cc - nc) / temp)) {
                L.pass[b] = p1;
                cc = nc;
            } else {
                L.add(b, p1, -1);
                L.add(b, p0, +1);
            }
        } else {
            const int a = rng.below(L.N), b = rng.below(L.N);
            if (!L.core[a] || L.core[b]) continue;
            L.set_core(a, false);
            L.set_core(b, true);
            const int nc = L.cost();
            if (nc <= cc || rng.unit() < std::exp((cc - nc) / temp)) {
                cc = nc;
            } else {
                L.set_core(b, false);
                L.set_core(a, true);
            }
        }
    }
    return cc == 0;
}

}  // namespace

int plan_layout(int n_sites, int n_bonds, const int32_t *bi, const int32_t *bj, int tile_bits, int max_core,
                int32_t *site_perm, int32_t *bond_order)
{
    const int N = n_sites;
    if (N <= tile_bits || max_core < 0 || max_core > tile_bits - 2) return 0;
    Rng rng{0x9E3779B97F4A7C15ull};
    for (int P = 1; P <= 6; ++P) {
        for (int core = max_core; core >= std::min(max_core, 4); --core) {
            for (int restart = 0; restart < 6; ++restart) {
                Layout L{N, n_bonds, P, tile_bits, core, bi, bj, std::vector<int>(n_bonds, 0),
                         std::vector<int>((size_t)P * N, 0), std::vector<char>(N, 0), std::vector<int>(P, 0)};
                // random core, bonds dealt to passes in list-order blocks
                std::vector<int> order(N);
                for (int l = 0; l < N; ++l) order[l] = l;
                for (int l = N - 1; l > 0; --l) std::swap(order[l], order[rng.below(l + 1)]);
                for (int k = 0; k < core; ++k) L.set_core(order[k], true);
                for (int b = 0; b < n_bonds; ++b) {
                    L.pass[b] = (int)((long)b * P / n_bonds);
                    L.add(b, L.pass[b], +1);
                }
                if (!anneal(L, rng, 150000)) continue;
                // core sites first; then the sites of the last pass, of the one before,
                // and so on: the last pass (the most traffic) reads the most compact
                // tiles, sites in several passes going with the latest of them
                std::vector<int> last(N, -1);
                for (int p = 0; p < P; ++p)
                    for (int l = 0; l < N; ++l)
                        if (L.count[(size_t)p * N + l] > 0) last[l] = p;
                std::vector<int> sites(N);
                for (int l = 0; l < N; ++l) sites[l] = l;
                std::stable_sort(sites.begin(), sites.end(), [&](int a, int b) {
                    if (L.core[a] != L.core[b]) return L.core[a] > L.core[b];
                    return last[a] > last[b];
                });
                for (int k = 0; k < N; ++k) site_perm[sites[k]] = k;
                int k = 0;
                for (int p = 0; p < P; ++p)
                    for (int b = 0; b < n_bonds; ++b)
                        if (L.pass[b] == p) bond_order[k++] = b;
                return P;
            }
        }
    }
    return 0;
}

}  // namespace ftk

// ---------------------------------------------------------------- peak-width fit
// Eq. asymmetricLorentzian (Sec. V.F): s(w) = gamma / (gamma^2 + x^2) (a + b sigma),
// x = w - eps, sigma = 1 / (1 + e^{c x}).  Levenberg-Marquardt on the sum of
// squared residuals with the analytic derivatives
//   ds/da = lz,  ds/db = lz sigma,  ds/dc = -lz b x sigma (1 - sigma),
//   ds/dgamma = F (x^2 - gamma^2) / D^2,
//   ds/deps = F 2 gamma x / D^2 + lz b c sigma (1 - sigma),
// with D = gamma^2 + x^2, lz = gamma / D and F = a + b sigma.
namespace ftk {

namespace {

struct LorentzPoint {
    double s, d[5];
};

LorentzPoint lorentz_point(const double *p, double w)
{
    const double a = p[0], b = p[1], c = p[2], g = p[3], e = p[4];
    const double x = w - e, D = g * g + x * x, lz = g / D;
    const double t = c * x, u = std::exp(-std::fabs(t));
    const double sig = t >= 0 ? u / (1.0 + u) : 1.0 / (1.0 + u);  // 1 / (1 + e^t) without overflow
    const double ss = u / ((1.0 + u) * (1.0 + u));                 // sigma (1 - sigma)
    const double F = a + b * sig;
    LorentzPoint r;
    r.s = lz * F;
    r.d[0] = lz;
    r.d[1] = lz * sig;
    r.d[2] = -lz * b * x * ss;
    r.d[3] = F * (x * x - g * g) / (D * D);
    r.d[4] = F * 2.0 * g * x / (D * D) + lz * b * c * ss;
    return r;
}

double lorentz_cost(const double *p, const double *w, const double *y, int n)
{
    double c = 0;
    for (int i = 0; i < n; ++i) {
        const double r = lorentz_point(p, w[i]).s - y[i];
        c += r * r;
    }
    return 0.5 * c;
}

// Solve the 5 x 5 system A x = rhs by elimination with partial pivoting; false if singular.
bool solve5(double A[5][5], double *rhs)
{
    for (int k = 0; k < 5; ++k) {
        int piv = k;
        for (int i = k + 1; i < 5; ++i)
            if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
        if (!(std::fabs(A[piv][k]) > 0)) return false;
        if (piv != k) {
            for (int j = 0; j < 5; ++j) std::swap(A[k][j], A[piv][j]);
            std::swap(rhs[k], rhs[piv]);
        }
        for (int i = k + 1; i < 5; ++i) {
            const double f = A[i][k] / A[k][k];
            for (int j = k; j < 5; ++j) A[i][j] -= f * A[k][j];
            rhs[i] -= f * rhs[k];
        }
    }
    for (int k = 4; k >= 0; --k) {
        double v = rhs[k];
        for (int j = k + 1; j < 5; ++j) v -= A[k][j] * rhs[j];
        rhs[k] = v / A[k][k];
    }
    return true;
}

}  // namespace

void asym_lorentzian_start(const double *w, const double *y, int n, double *p)
{
    int k = 0;
    for (int i = 1; i < n; ++i)
        if (y[i] > y[k]) k = i;
    const double ym = y[k], e = w[k];
    double sum = 0;
    int cnt = 0;
    for (int i = k - 1; i >= 0; --i)
        if (y[i] < 0.5 * ym) {
            sum += std::fabs(w[i] - e), ++cnt;
            break;
        }
    for (int i = k + 1; i < n; ++i)
        if (y[i] < 0.5 * ym) {
            sum += std::fabs(w[i] - e), ++cnt;
            break;
        }
    const double g = cnt ? sum / cnt : 0.25 * (w[n - 1] - w[0]);
    p[0] = 0.75 * ym * g;
    p[1] = 0.5 * ym * g;
    p[2] = 0.0;
    p[3] = g;
    p[4] = e;
}

int fit_asym_lorentzian(const double *w, const double *y, int n, int max_iter, double *p, double *cost)
{
    double f = lorentz_cost(p, w, y, n), mu = 1e-3;
    int it = 0;
    while (it < max_iter) {
        ++it;
        double A[5][5] = {}, g[5] = {};
        for (int i = 0; i < n; ++i) {
            const LorentzPoint q = lorentz_point(p, w[i]);
            const double r = q.s - y[i];
            for (int j = 0; j < 5; ++j) {
                g[j] += q.d[j] * r;
                for (int l = 0; l < 5; ++l) A[j][l] += q.d[j] * q.d[l];
            }
        }
        double dmax = 0;
        for (int j = 0; j < 5; ++j) dmax = std::max(dmax, A[j][j]);
        if (!(dmax > 0)) break;
        bool accepted = false, small = false;
        while (mu < 1e20) {
            double M[5][5], step[5];
            for (int j = 0; j < 5; ++j) {
                for (int l = 0; l < 5; ++l) M[j][l] = A[j][l];
                M[j][j] += mu * std::max(A[j][j], 1e-12 * dmax);
                step[j] = -g[j];
            }
            if (solve5(M, step)) {
                double trial[5], sn = 0, pn = 0;
                for (int j = 0; j < 5; ++j) {
                    trial[j] = p[j] + step[j];
                    sn += step[j] * step[j];
                    pn += p[j] * p[j];
                }
                const double ft = lorentz_cost(trial, w, y, n);
                if (std::isfinite(ft) && ft < f) {
                    small = (f - ft) <= 1e-15 * f || sn <= 1e-30 * pn;
                    std::memcpy(p, trial, sizeof trial);
                    f = ft;
                    mu = std::max(mu * 0.3, 1e-15);
                    accepted = true;
                    break;
                }
            }
            mu *= 10.0;
        }
        if (!accepted || small) break;
    }
    if (p[3] < 0) p[0] = -p[0], p[1] = -p[1], p[3] = -p[3];
    *cost = f;
    return it;
}

}  // namespace ftk
