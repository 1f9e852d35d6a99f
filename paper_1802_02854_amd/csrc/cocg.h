// Shifted COCG with seed switching: per-sequence state and launchers (cocg.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ftk {

// Shifted COCG with seed switching (complex-symmetric Lanczos basis + per-shift
// scalar recurrences; kernels.hip).  One sequence per run.
struct CocgState {
    double invr, invi;  // inv_k = 1/b_k (1/delta_0 at k = 0)
    double ipr, ipi;    // inv_{k-1}
    double bkr, bki;    // b_k (0 at k = 0)
    double akr, aki;    // a_k
    double c2r, c2i;    // -(a_k inv_k)
    double ckr, cki;    // c_k = <chi|q_k>
    double hn, hn0;     // ||q_k||^2, ||q_0||^2
    double d0r, d0i;    // delta_0 = csqrt(chi^T chi)
    double alr, ali;    // seed alpha_{k-1}
    double ber, bei;    // seed beta_{k-1}
    double dr, di;      // seed residual scale delta_k
    double norm2;       // ||chi||^2
    double shift_re;    // real offset of every shift (E_m)
    double max_resid;   // largest residual 2-norm over the shifts after the last step
    int seed;           // index of the seed shift
    int done, steps, numeric_error;
};
struct CocgShift {
    double pr, pi;    // pi_k
    double por, poi;  // pi_{k-1}
    double Pr, Pi;    // <chi|p_{k-1}> of the shift
    double gr, gi;    // <chi|x_k> of the shift
    double res;       // residual 2-norm after the shift's last update (+inf before the first)
};
// state from the right-hand side chi and the projection vector lam (= chi for a
// spectrum); c_out[0..1] = c_0
void launch_cocg_start(uint32_t dim, const double *chi, const double *lam, double *partials, CocgState *st,
                       CocgShift *sh, int n_omega, double shift_re, double *c_out, hipStream_t s);
// step k: Wcur = w_{k-1} (chi at k = 0), Wprev = w_{k-2} (chi at k = 1, unused at
// k = 0); U (may be Wprev) receives w_k; Hw is a work vector; a_out[2k], b_out[2k] =
// a_k, b_{k+1}, c_out[2k+2] = c_{k+1}; partials holds 10 vec_grid doubles
void launch_cocg_step(const HvOp &op, const double *lam, const double *Wcur, const double *Wprev, double *U,
                      double *Hw, double *partials, CocgState *st, CocgShift *sh, const double *omega, int n_omega,
                      double eta, int k, double tol, double rtol, double seed_tol, double *a_out, double *b_out,
                      double *c_out, hipStream_t s);
void launch_cocg_finish(const CocgState *st, const CocgShift *sh, int n_omega, double *g, hipStream_t s);

}  // namespace ftk
