// Device kernels of the FTKw path and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ftkw_internal.h"

namespace ftk {

// Bond table as passed to every H-applying kernel (by value, ~1 KB).
struct HvParams {
    int n_sites;
    int n_bonds;
    uint32_t mask[kMaxBonds];  // 2^i | 2^j
    uint8_t bi[kMaxBonds];
    uint8_t bj[kMaxBonds];
    uint8_t isz[kMaxBonds];    // 1 for z bonds
    double ap[kMaxBonds];      // flip amplitude, parallel spins
    double aa[kMaxBonds];      // flip amplitude, antiparallel spins
    double jq, kq;             // J/4, K/4
};
HvParams make_hv_params(const BondTable &t);

// Per-sequence scalars of a Lanczos run kept on the device between launches.
// v_k = w_{k-1} * inv_cur with w_{-1} the start vector.
struct SeqState {
    double inv_cur;    // inv_k = 1 / beta_k (1/||start|| at k = 0)
    double inv_prev;   // inv_{k-1}
    double beta_cur;   // beta_k (0 at k = 0)
    double alpha_cur;  // alpha_k after the first reduction of step k
    double norm2;      // ||start||^2 (exact-sum rounded)
    double norm;       // ||start||
    double shift_re;   // real offset added to every omega (E_m)
    double max_resid;  // max over shifts of the Galerkin residual after the last step
    int done;          // set once beta_{k+1} <= tol (invariant subspace)
    int steps;         // completed steps
    int numeric_error; // NaN / Inf seen in a coefficient
    int pad;
};

// Per-shift state of the forward LDL^T recurrence, 6 doubles.
struct ShiftState {
    double dr, di, pr, pi, gr, gi;
};

constexpr int kBlock = 256;         // threads per block of the vector kernels
constexpr int kMaxGrid = 4096;      // blocks of the grid-stride vector kernels
constexpr int kChunk = 512;         // elements per wave in the blocked H v (64 lanes x 8)
constexpr int kTile = 8192;         // elements per workgroup tile staged in LDS (128 KiB)
constexpr int kTileThreads = 1024;  // threads of a tiled workgroup (16 waves)

int vec_grid(uint32_t dim);          // grid of the streaming kernels
int hv_grid(uint32_t dim);           // grid of the H-applying kernels (= number of partial sums)
int hv_mode(uint32_t dim);           // 0 one element per thread, 1 blocked, 2 blocked + LDS tile
void set_hv_mode(int mode);          // force a smaller mode (-1: by size), for tuning
void hv_set_attributes();            // allow the tiled kernels their 128 KiB of LDS

// w = H v (natural order, one vector)
void launch_apply_h(const HvParams &P, const double *v, double *w, hipStream_t s);

// Lanczos step, first half: u = H v_k - beta_k v_{k-1}, partial sums of Re<v_k|u>.
// Wcur holds w_{k-1}, Wprev holds w_{k-2} (may equal U: read before write per
// element); U receives u; vout (optional) receives v_k.
void launch_lanczos_a(const HvParams &P, const double *Wcur, const double *Wprev, double *U,
                      double *vout, SeqState *st, double *partials, int first_step, hipStream_t s);
// alpha_k = rounded sum of the partials; alpha[k] recorded.
void launch_finalize_alpha(SeqState *st, const double *partials, int nparts, double *alpha_out,
                           int k, hipStream_t s);
// second half: w_k = u - alpha_k v_k in place of u; partial sums of ||w_k||^2.
void launch_lanczos_b(uint32_t dim, const double *Wcur, double *U, SeqState *st,
                      double *partials, hipStream_t s);
// beta_{k+1}, inv_{k+1}, breakdown test and the multi-shift update of step k.
void launch_finalize_beta(SeqState *st, const double *partials, int nparts, double *beta_out,
                          int k, double tol, ShiftState *shifts, const double *omega, int n_omega,
                          double eta, hipStream_t s);
// g = norm2 * G for every shift of a finished sequence (complex, interleaved).
void launch_finish_green(const SeqState *st, const ShiftState *shifts, int n_omega, double *g,
                         hipStream_t s);

// partial sums of Re<a|b> (a, b interleaved complex, dim entries)
void launch_dot(uint32_t dim, const double *a, const double *b, double *partials, hipStream_t s);
// st->norm2 = sum, norm = sqrt, inv_cur = 1/norm; resets the rest of the state
void launch_start_sequence(SeqState *st, const double *partials, int nparts, double shift_re,
                           hipStream_t s);
// result[0] = rounded sum of partials
void launch_sum_partials(const double *partials, int nparts, double *result, hipStream_t s);

// chi = S^alpha_{+Q} phi; h = e^{iQ.R_l}/(2 sqrt N) per site (interleaved, n_sites entries)
struct SqParams {
    int n_sites;
    int alpha;
    double h[2 * kMaxSites];
};
// output entry x goes to chi[x * stride + offset] (block layout of a batch)
void launch_apply_sq(const SqParams &P, const double *phi, double *chi, hipStream_t s, int stride = 1,
                     int offset = 0);

// One Taylor term: tn = fma(a, t, b * (H t)); acc = acc + tn
void launch_taylor_term(const HvParams &P, const double *t, double *tn, double *acc, double a,
                        double b, hipStream_t s);

// v = v * scale (scale read from host value)
void launch_scale(uint32_t dim, double *v, double scale, hipStream_t s);
// copy
void launch_copy(uint32_t dim, const double *src, double *dst, hipStream_t s);
// complex Gaussian draws of (seed, sample)
void launch_gaussian(uint32_t dim, uint64_t seed, uint64_t sample, double *g, hipStream_t s);

// Phi[m] += sum_{k < nk} c[m][k0 + k] V[k] for m < L (coef: [L][n] complex)
void launch_accumulate(uint32_t dim, const double *V, int nk, const double *coef, int n, int k0,
                       double *Phi, int L, hipStream_t s);

// ---------------------------------------------------------------------------
// Batches of B in {2, 4, 8, 16} sequences in block layout (entry (x, r) at x*B + r);
// SeqState st[B], partial sums [grid][B], alpha/beta rows of length n_max,
// shift states [B][n_omega].
int hv_batch_grid(uint32_t dim, int B);
int vec_batch_grid(uint32_t dim, int B);
struct BatchShifts {
    double re[16];  // real offset (E_m) of each sequence's shifts
};
void launch_start_batch(int B, uint32_t dim, const double *chi, double *partials, SeqState *st,
                        const BatchShifts &shift_re, hipStream_t s);
void launch_lanczos_a_batch(int B, const HvParams &P, const double *Wcur, const double *Wprev, double *U,
                            SeqState *st, double *partials, int first, hipStream_t s);
void launch_finalize_alpha_batch(int B, SeqState *st, const double *partials, int nparts, double *alpha_out,
                                 int n_max, int k, hipStream_t s);
void launch_lanczos_b_batch(int B, uint32_t dim, const double *Wcur, double *U, SeqState *st, double *partials,
                            hipStream_t s);
void launch_finalize_beta_batch(int B, SeqState *st, const double *partials, int nparts, double *beta_out,
                                int n_max, int k, double tol, ShiftState *shifts, const double *omega, int n_omega,
                                double eta, hipStream_t s);

}  // namespace ftk
