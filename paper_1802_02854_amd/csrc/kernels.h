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
    // bond-parity vectors: bit b of par(x) = bit i_b(x) ^ bit j_b(x) is the XOR of
    // smask[l] over the set bits l of x
    uint64_t smask[kMaxSites]; // bonds touching site l
    uint64_t zmask;            // z bonds
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

constexpr int kR = 8;               // elements per thread in the blocked H v
constexpr int kBlock = 256;         // threads per block of the vector kernels
constexpr int kMaxGrid = 4096;      // blocks of the grid-stride vector kernels
constexpr int kChunk = 512;         // elements per wave in the blocked H v (64 lanes x 8)
constexpr int kTile = 8192;         // elements per workgroup tile staged in LDS (128 KiB)
constexpr int kTileThreads = 1024;  // threads of a tiled workgroup (16 waves)

// Multi-pass form of H v.  The bond list is cut into contiguous segments; pass p
// walks over tiles of 2^kPassBits elements spanned by kPassBits sites that hold
// every bond of segment p, stages each tile in LDS and applies the segment's
// bonds there.  The sites 0..core-1 belong to every pass, so tiles are read in
// runs of 2^core consecutive elements.  Partial sums travel between passes
// through a scratch vector; the accumulation order per element is the bond-list
// order, exactly as in the single-pass forms.
constexpr int kPassBits = 12;
constexpr int kPassTile = 1 << kPassBits;  // 4096 elements, 64 KiB of LDS
constexpr int kPassThreads = 512;          // 8 waves x 64 lanes x kR elements
constexpr int kMaxPasses = 6;
constexpr int kPassMinSites = 16;          // smallest N given the scratch vector of the multi-pass form
struct PassGeom {
    int b0, b1;                         // the segment: bonds [b0, b1)
    uint32_t ebit[kR];                  // x offsets of a thread's kR elements (tile bits 6..8)
    uint8_t ysite[9];                   // sites of tile bits 0..5 (lane) and 9..11 (wave)
    uint8_t esite[3];                   // sites of tile bits 6..8 (register element e)
    uint8_t hsite[kMaxSites];           // sites of the tile-index bits
    uint8_t tbi[kMaxBonds], tbj[kMaxBonds];  // tile bit positions of the segment's bond ends
    uint8_t rev;                        // tiles in descending order (set per launch)
};
struct HvPlan {
    int n_passes = 0;  // 0: no multi-pass form (N <= kPassBits or too many segments)
    int core = 0;
    PassGeom pass[kMaxPasses];
};
HvPlan make_hv_plan(const BondTable &t);

// Everything an H-applying launch needs: bond table, pass plan, scratch vector.
struct HvOp {
    HvParams P;
    HvPlan plan;
    double *scratch = nullptr;  // 2^N complex; needed by the multi-pass form
    int pass_grid = 0;          // persistent workgroups of a reducing multi-pass launch
                                // (0: set_pass_grid's value, else two per compute unit)
    int hints = -1;             // cache hints of the multi-pass form: 1 streaming, 0 cached,
                                // -1 by the launch's working set (stream_hints)
};

int vec_grid(uint32_t dim);          // grid of the streaming kernels
// 0 one element per thread, 1 blocked, 2 blocked + LDS tile, 3 multi-pass
int hv_mode(const HvOp &op);
int hv_grid(const HvOp &op);         // grid of the H-applying kernels (= number of partial sums)
int hv_grid(const HvOp &op, int B);  // per-sequence grid of a stack of B sequences (multi-pass form)
void set_hv_mode(int mode);          // force a mode if available (-1: by size), for tuning
void set_pass_grid(int grid);        // workgroups per reducing multi-pass launch (0: two per compute unit)
int pass_grid_cap(const HvOp &op);   // the workgroups a reducing multi-pass launch of op may use
void set_full_grid(int on);          // 1: passes without partial sums run one workgroup per tile
void set_hints(int mode);            // force the multi-pass cache hints (1 streaming, 0 cached, -1 per op)
int forced_hints();                 // the forced hint set, -1 when none
bool stream_hints(const HvOp &op, int B);  // the hint set a launch of B sequences of op uses
void set_fuse_finalize(int on);      // 1: the beta finalisation rides in the middle pass (3+ passes) and
                                     //    alpha in the next fused first pass
void hv_set_attributes();            // allow the tiled kernels their LDS
// Device bounds checks (built into the debug library with -DFTK_DEVICE_CHECKS):
// 1 when compiled in; out = (violations, site of the first, its index) of the
// current device since the last clear (zeros in the release build).
int device_checks_compiled();
void device_checks_read(unsigned int out[3], bool clear);
// debug build: one kernel claims entry 5 of a 4-entry buffer (site 99) and writes
// the index it was given (0) to out_dev[0]; nothing in the release build
void device_checks_selftest(uint32_t *out_dev, hipStream_t s);

// w = H v (natural order, one vector)
void launch_apply_h(const HvOp &op, const double *v, double *w, hipStream_t s);

// A stack of B independent sequences run through the multi-pass kernels in one
// grid (sequence r in blockIdx.y): sequence r's vectors start r*vs doubles after
// the pointers given, its multi-pass partial sums live at scratch + r*vs, its state
// is st[r] and its reduction partials sit r*2*grid doubles into `partials`.
// The default is one sequence using the operator's own scratch vector.
struct Stack {
    int B = 1;
    double *scratch = nullptr;
    size_t vs = 0;
};

// Lanczos step, first half: u = H v_k - beta_k v_{k-1}, partial sums of Re<v_k|u>.
// Wcur holds w_{k-1}, Wprev holds w_{k-2} (may equal U: read before write per
// element); U receives u; vout (optional) receives v_k.  A stack needs the
// multi-pass form.
void launch_lanczos_a(const HvOp &op, const double *Wcur, const double *Wprev, double *U,
                      double *vout, SeqState *st, double *partials, int first_step, hipStream_t s,
                      const Stack &sk = Stack());
// Multi-pass form with at least two passes: the second half of step k-1 runs
// inside the first pass of step k.  Step k (k >= 1) is then
//   launch_lanczos_fused_first(W = buffer of u_{k-1}, Wm2 = w_{k-2})
//       -> w_{k-1} in place of u_{k-1}, partial sums of ||w_{k-1}||^2 (hv_grid of them);
//   launch_finalize_beta(step k-1);
//   launch_lanczos_a_rest(Wcur = w_{k-1}, Wprev = w_{k-2}, U, vout) -> u_k, partials of <v_k|u_k>;
//   launch_finalize_alpha(step k);
// and after the last step the plain launch_lanczos_b + launch_finalize_beta.
bool lanczos_fusable(const HvOp &op);
// Arguments of the beta finalisation of one step (launch_finalize_beta) for B sequences.
struct FinBeta {
    SeqState *st;
    const double *partials;
    int nparts;
    double *beta_out;
    int k;
    double tol;
    ShiftState *sh;
    const double *omega;
    int n_omega;
    double eta, rtol;
    int bstride;
};
// alpha_k of the previous step finalised inside the fused first pass of the next
// one (every workgroup reduces the partial sums itself; workgroup 0 records it)
struct FinAlpha {
    const double *partials;  // 2*nparts per sequence
    int nparts;
    double *alpha_out;       // rows astride apart
    int astride;
    int k;
};
bool alpha_in_fused_pass();  // the fused first pass finalises the previous alpha
// true when launch_lanczos_a_rest can run the beta finalisation of step k-1 as one
// more workgroup column of its first (middle) pass: plans of three or more passes;
// the middle pass does not depend on beta, the last pass does
bool beta_in_middle_pass(const HvOp &op);
// a stack of B > 1 sequences (Stack) runs the multi-pass kernels whatever form
// single vectors use; it needs a plan of at least two passes and the scratch vector
bool lanczos_stackable(const HvOp &op);
void launch_lanczos_fused_first(const HvOp &op, double *W, const double *Wm2, SeqState *st, double *partials,
                                hipStream_t s, const Stack &sk = Stack(), const FinAlpha *fa = nullptr);
void launch_lanczos_a_rest(const HvOp &op, const double *Wcur, const double *Wprev, double *U, double *vout,
                           SeqState *st, double *partials, hipStream_t s, const Stack &sk = Stack(),
                           const FinBeta *fb = nullptr);
// alpha_k = rounded sum of the partials; alpha[k] recorded.  B > 1: sequences
// st[0..B), partials 2*nparts apart, alpha rows astride apart.
void launch_finalize_alpha(SeqState *st, const double *partials, int nparts, double *alpha_out,
                           int k, hipStream_t s, int B = 1, int astride = 0);
// second half: w_k = u - alpha_k v_k in place of u; partial sums of ||w_k||^2
// (vec_grid of them).  B > 1: vectors vs doubles apart, partials 2*vec_grid apart.
void launch_lanczos_b(uint32_t dim, const double *Wcur, double *U, SeqState *st,
                      double *partials, hipStream_t s, int B = 1, size_t vs = 0);
// beta_{k+1}, inv_{k+1}, breakdown test and the multi-shift update of step k.
// rtol > 0: the sequence also stops (done) once the largest Galerkin residual over
// the shifts, per unit right-hand side, is <= rtol.
// B > 1: sequences st[0..B), partials 2*nparts apart, beta rows bstride apart,
// shift states n_omega apart.
void launch_finalize_beta(SeqState *st, const double *partials, int nparts, double *beta_out,
                          int k, double tol, ShiftState *shifts, const double *omega, int n_omega,
                          double eta, hipStream_t s, double rtol = 0.0, int B = 1, int bstride = 0);
// g = norm2 * G for every shift of a finished sequence (complex, interleaved).
void launch_finish_green(const SeqState *st, const ShiftState *shifts, int n_omega, double *g,
                         hipStream_t s);

// partial sums of Re<a|b> (a, b interleaved complex, dim entries); B > 1: B pairs
// of vectors vs doubles apart, partials 2*vec_grid apart
void launch_dot(uint32_t dim, const double *a, const double *b, double *partials, hipStream_t s, int B = 1,
                size_t vs = 0);
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

// chi = A phi for A = sum_l sum_alpha c_{l alpha} S^alpha_l; h[alpha] holds c_{l alpha}/2
// per site (interleaved complex).  Natural layout.
struct SpinOpParams {
    int n_sites;
    double h[3][2 * kMaxSites];
};
void launch_apply_spin_op(const SpinOpParams &P, const double *phi, double *chi, hipStream_t s);
// chi[x * stride + offset] = lam + rho, lam - rho, lam + i rho, lam - i rho for k = 0..3
void launch_polarize(uint32_t dim, int k, const double *lam, const double *rho, double *chi, hipStream_t s,
                     int stride = 1, int offset = 0);

// One Taylor term: tn = fma(a, t, b * (H t)); acc = acc + tn
void launch_taylor_term(const HvOp &op, const double *t, double *tn, double *acc, double a,
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
constexpr int kMaxBatch = 32;  // sequences per batch: 16 in block layout, 32 as a stack
struct BatchShifts {
    double re[kMaxBatch];  // real offset (E_m) of each sequence's shifts
};
void launch_start_batch(int B, uint32_t dim, const double *chi, double *partials, SeqState *st,
                        const BatchShifts &shift_re, hipStream_t s);
// start of a stack of B sequences whose vectors are 2*dim doubles apart
void launch_start_stacked(int B, uint32_t dim, const double *chi, double *partials, SeqState *st,
                          const BatchShifts &shift_re, hipStream_t s);
void launch_lanczos_a_batch(int B, const HvParams &P, const double *Wcur, const double *Wprev, double *U,
                            SeqState *st, double *partials, int first, hipStream_t s);
void launch_finalize_alpha_batch(int B, SeqState *st, const double *partials, int nparts, double *alpha_out,
                                 int n_max, int k, hipStream_t s);
void launch_lanczos_b_batch(int B, uint32_t dim, const double *Wcur, double *U, SeqState *st, double *partials,
                            hipStream_t s);
void launch_finalize_beta_batch(int B, SeqState *st, const double *partials, int nparts, double *beta_out,
                                int n_max, int k, double tol, ShiftState *shifts, const double *omega, int n_omega,
                                double eta, hipStream_t s, double rtol = 0.0);

}  // namespace ftk
