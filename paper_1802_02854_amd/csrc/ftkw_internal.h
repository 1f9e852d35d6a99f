// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ftkw.h"

namespace ftk {

constexpr int kMaxSites = 30;
constexpr int kMaxBonds = 3 * kMaxSites / 2;
// largest cluster whose multi-pass H v fits the static scratch of ftk_apply_h_noalloc
constexpr int kNoAllocMaxSites = 22;

// Error carrying an ftk_status across internal layers; converted at the C-ABI.
struct Error : std::runtime_error {
    ftk_status status;
    Error(ftk_status s, const std::string &msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] inline void fail(ftk_status s, const std::string &msg) { throw Error(s, msg); }

// ---------------------------------------------------------------- clusters
struct HoneyCluster {
    int n_cells = 0, p = 0, q = 0, s = 0;
    std::vector<int32_t> bi, bj;
    std::vector<int8_t> gamma;
    std::vector<double> xy;  // [2 n_sites]
};
HoneyCluster honeycomb(int t11, int t12, int t21, int t22);
std::vector<double> honeycomb_momenta(int t11, int t12, int t21, int t22);
bool named_momentum(const std::string &name, double *q);

// ---------------------------------------------------------------- model scalars
struct BondTable {
    int n_sites = 0, n_bonds = 0;
    int32_t bi[kMaxBonds], bj[kMaxBonds];
    int8_t gamma[kMaxBonds];
    double ap[kMaxBonds], aa[kMaxBonds];
    double jq = 0, kq = 0;  // J/4, K/4
    double norm_bound = 0;  // B_H
};
BondTable make_bond_table(const ftk_cluster &c, double K, double J);

// h_l = e^{i Q.R_l} (1/2) N^{-1/2}, interleaved [2 N]
void sq_coefficients(int n_sites, const double *site_xy, double qx, double qy, double *h);

// Appendix A plan for e^{-beta H/2}
struct TaylorPlan {
    int Md = 0, K = 0;
    double c = 0, ell = 0;
};
TaylorPlan taylor_plan(int n_sites, double beta, double norm_bound, double lambda);

// Shell coefficients c^m_k: out [L][n] complex interleaved; kn (optional) gives
// shell m its own step count kn[m] <= n (T_{kn[m]}, zeros beyond).
void shell_coefficients(const double *alpha, const double *beta, int n, double nrm, double E_b,
                        double eps, int L, int M, double *out, const int *kn = nullptr);
double shell_energy(double E_b, double eps, int m);
// Site relabelling and bond order for the multi-pass H v: the fewest passes
// (segments of at most tile_bits sites that all contain the core sites
// 0..core-1), then the largest core in [4, max_core], found by annealing.
// site_perm[l] = new index of site l; bond_order[k] = old index of the bond
// listed k-th.  Returns the number of passes (0 if none <= 6).
int plan_layout(int n_sites, int n_bonds, const int32_t *bi, const int32_t *bj, int tile_bits, int max_core,
                int32_t *site_perm, int32_t *bond_order);
// message returned by ftk_last_error on this thread
void set_last_error(const std::string &msg);
// rhs_block the autotuner has recorded for (device, n_sites, n_omega) in this
// process or the tuning cache file; 0 when it has none
int tuned_rhs_block(int device, int n_sites, int n_omega);
// Smallest k in [1, n] after which every shift z = zr + i zi has Galerkin
// residual |p_{k-1}| beta_k / |d_{k-1}| <= tol (forward LDL^T recurrence of T_k,
// the arithmetic of the device's multi-shift update); n if none.
int truncation_steps(const double *alpha, const double *beta, int n, const double *zr, const double *zi, int nz,
                     double tol);
void residual_history(const double *alpha, const double *beta, int n, const double *zr, const double *zi, int nz,
                      double *out);
// extreme eigenvalues of the symmetric tridiagonal T_n (diagonal alpha[0..n-1],
// off-diagonal beta[0..n-2]) by Sturm-sequence bisection
void ritz_extremes(const double *alpha, const double *beta, int n, double *lo, double *hi);
// (E_b, eps) of L shells tiling [theta_min - margin, theta_max + margin]
void shell_window(const double *alpha, const double *beta, int n, int L, double margin, double *E_b, double *eps);

// Reweighting, see ftk_reweight.
// Eq. FRW1 for real observables O [nv][na][L][K]; out/err [K][nT]
void reweight_observable(int nv, int na, int L, int K, const double *betas, const double *E_m, const double *log_norm,
                         const double *n_m, const double *O, const double *T, int nT, int n_bins, double *out,
                         double *err);
// out/err [nT][4] = (E, C, S, ln Z) per temperature; h1/h2 may be NULL
void thermodynamics(int nv, int na, int L, const double *betas, const double *E_m, const double *log_norm,
                    const double *n_m, const double *h1, const double *h2, int n_sites, const double *T, int nT,
                    int n_bins, double *out, double *err);
void thermo_diagnostics(int nv, int na, int L, const double *betas, const double *E_m, const double *log_norm,
                        const double *n_m, const double *h1, const double *h2, int n_sites, const double *inv_T,
                        int nT, int n_bins, double *out, double *err);
double overlap_ratio(double E1, double var1, double E2, double var2);
int choose_anchors(int n, const double *E, const double *var, double r_max, int max_anchors, int *anchors);
// Least-squares fit of the asymmetric Lorentzian of Sec. V.F to (w[i], y[i]),
// i < n, from the start p[0..4] = (a, b, c, gamma, eps), overwritten with the
// result (gamma > 0).  Returns the iterations taken; *cost = 0.5 sum r^2.
int fit_asym_lorentzian(const double *w, const double *y, int n, int max_iter, double *p, double *cost);
void asym_lorentzian_start(const double *w, const double *y, int n, double *p);
void reweight(int nv, int na, int L, int nq, int nw, const double *betas, const double *E_m,
              const double *eps, const double *log_norm, const double *n_m, const double *g,
              const double *T, int nT, int n_bins, double *S, double *S_err, double *P);

}  // namespace ftk
