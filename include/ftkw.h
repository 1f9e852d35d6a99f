/*
 * ftkw.h -- C-ABI of the MI355X (gfx950) implementation of the FTKw hot path:
 * finite-temperature dynamical spin structure factors of the spin-1/2
 * Kitaev-Heisenberg honeycomb model from typical pure states, contour filters
 * and shifted Krylov solves (Yamaji, Suzuki, Kawamura, arXiv:1802.02854).
 *
 * Conventions for every call
 *   - Return value: FTK_OK or a negative ftk_status; ftk_last_error() then
 *     holds a message (thread-local, valid until the next call on the thread).
 *     Arguments are validated before any device work; no C++ exception
 *     crosses this interface.
 *   - Complex numbers are complex128 stored interleaved (re, im).
 *   - A state vector of an N-site cluster has 2^N complex entries in natural
 *     basis order: index x = sum_l sigma_l 2^l with sigma_l = 0 for spin up on
 *     site l (the bit-string basis of Sec. II.A).
 *   - "_dev" pointers are device memory on the context's GPU (e.g. a torch
 *     tensor's data_ptr()); all others are host memory.  Caller arrays are read
 *     during the call only; handles are owned by the caller and released with
 *     the matching *_destroy.  Device work is queued on the context's stream;
 *     calls that return host data synchronise that stream first.
 *   - Supported sizes: 4 <= N <= 30 sites (state vectors up to 16 GiB).
 *
 * Arithmetic contract.  Lanczos recurrences amplify one-ulp differences, so
 * every vector operation uses a fixed sequence of IEEE-754 double operations
 * (stated at each call) and every inner product is the double nearest to the
 * exact sum.  Two runs, and any CPU program following the same contract, give
 * identical Krylov coefficients.
 */
#ifndef FTKW_H
#define FTKW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FTK_OK = 0,
    FTK_EINVAL = -1,     /* invalid argument */
    FTK_ENOMEM = -2,     /* device or host allocation failed / budget exceeded */
    FTK_EDEVICE = -3,    /* HIP runtime error */
    FTK_ENUMERIC = -4,   /* NaN or Inf met in a Krylov coefficient */
    FTK_EBUSY = -5,      /* server queue full */
    FTK_ENOTREADY = -6,  /* server result not ready yet */
    FTK_ECANCELED = -7   /* server request cancelled (ftk_server_cancel) */
} ftk_status;

const char *ftk_last_error(void);

/* ------------------------------------------------------------------------ */
/* Context: one GPU and one HIP stream.  hip_stream is a hipStream_t owned by
 * the caller, which must outlive the context, or NULL: the library then creates
 * a blocking stream of its own (ordered with the null stream, capturable). */
typedef struct ftk_ctx ftk_ctx;
ftk_status ftk_ctx_create(int device, void *hip_stream, ftk_ctx **out);
/* The same with the context's device memory taken from the caller's allocator
 * (e.g. a framework's caching allocator): alloc(bytes, user) returns device
 * memory of at least bytes bytes, 256-byte aligned, or NULL (FTK_ENOMEM);
 * release(p, user) gives it back.  Buffers are released only after the work
 * that uses them has been enqueued on the context's stream, so an allocator
 * that reuses memory in stream order on that stream is safe; every call of the
 * library that allocates runs the callbacks on the calling thread.  Both
 * callbacks NULL: hipMalloc / hipFree. */
typedef void *(*ftk_alloc_fn)(size_t bytes, void *user);
typedef void (*ftk_free_fn)(void *p, void *user);
ftk_status ftk_ctx_create_with_allocator(int device, void *hip_stream, ftk_alloc_fn alloc, ftk_free_fn release,
                                         void *user, ftk_ctx **out);
/* A context serves one thread at a time (its stream, byte counts and timing
 * events are not locked); use one context per thread, as the server does for
 * its workers.  Destroy every handle made on a context (Hamiltonians, states,
 * spectra, pair spectra) before the context itself. */
ftk_status ftk_ctx_destroy(ftk_ctx *ctx);
ftk_status ftk_sync(ftk_ctx *ctx);
/* Device memory currently held by the library for this context, in bytes. */
ftk_status ftk_ctx_memory(const ftk_ctx *ctx, size_t *bytes_in_use);
/* Largest ftk_ctx_memory value since the last reset (reset != 0 restarts the
 * count from the current value after reporting).  peak may be NULL. */
ftk_status ftk_ctx_peak_memory(ftk_ctx *ctx, size_t *peak, int reset);
/* Kernel timing for measurements.  While enabled, HIP events on the context's
 * stream bracket every ftk_apply_h launch ("apply_h"), the Green's-function
 * loops and the filter runs.  A Green's-function batch whose n-step loop is
 * replayed from a graph is timed as a whole ("lanczos_block": n steps of its
 * rhs_block sequences); without graphs, steps 1, 9, 17, ... of every batch are
 * timed ("lanczos_step": all launches of one step, i.e. u = H v_k - beta_k
 * v_{k-1} with <v_k|u>, w_k = u - alpha_k v_k with ||w_k||, and the scalar and
 * multi-shift updates; with the multi-pass H v the second half of a step runs
 * inside the next step, so a timed step is the second half of step k-1 and the
 * first half of step k), and the filter runs' steps likewise ("filter_step").
 * ftk_ctx_kernel_time synchronises the stream and returns the number of timed
 * launches and their mean duration in milliseconds, then forgets them. */
ftk_status ftk_ctx_set_timing(ftk_ctx *ctx, int enable);
/* Tuning knobs (process-wide).  Results are identical for every setting.
 *   "hv_variant": H v kernel form, 0 = one element per thread, 1 = 8 elements
 *       per thread, 2 = 8 elements per thread with an LDS-staged 8192-element
 *       tile, 3 = multi-pass (the bond list cut into segments, each applied
 *       inside 4096-element LDS tiles of its own site set; N >= 16 with at most
 *       6 segments, else as -1); -1 (default) takes 3 from N = 18 on when the
 *       bond list needs at most 6 segments, otherwise the largest of 0..2 the
 *       vector size allows.  A Hamiltonian of N >= 16 sites holds one scratch
 *       vector for the multi-pass form.
 *   "pass_grid": workgroups of each multi-pass launch that reduces partial
 *       sums (the last pass of a Lanczos step and the fused first pass; 0, the
 *       default: two per compute unit, each looping over 4096-element tiles).
 *       The other passes (H v, Taylor terms, the middle passes) run one
 *       workgroup per tile.
 *   "full_grid": 1 (default) as just described; 0 runs every multi-pass
 *       launch on the "pass_grid" workgroups.
 *   "stream_hints": cache hints of the multi-pass kernels.  1 = streaming:
 *       partial sums stored plainly for the next pass to read back, the fused
 *       first pass's loads and its store of w nontemporal, the first pass's
 *       tiles in descending order; 0 = cached: partial sums stored
 *       nontemporally, the fused first pass's accesses plain.  Both load the
 *       pass inputs and partial sums nontemporally.  -1 (default): the
 *       autotuner's pick where it tuned the run, else streaming when one
 *       launch's vectors (B sequences of 2^N complex entries) come to 128-512
 *       MiB, cached otherwise.  Results are identical either way.
 *   "fuse_finalize": 1 (default) runs the beta finalisation of a Lanczos half
 *       step (norm, shift update, stopping test) as one more workgroup of the
 *       next middle pass when the multi-pass plan has three or more passes
 *       (the middle pass does not depend on it), and forms alpha of a step in
 *       every workgroup of the next step's fused first pass (which needs it)
 *       instead of a kernel of its own; 0 launches both finalisations on their
 *       own.  Results are identical either way.
 *   "graphs": 1 (default) captures the n-step Lanczos loop of a batch of
 *       Green's sequences into a HIP graph replayed for every batch; 0 launches
 *       each kernel.
 *   "plain_loop": 1 runs the reference one-vector loop: no graph, and every
 *       step's alpha, beta are read back to the host before the next step.
 *   "stack_batch": layout of a batch of B > 1 Green's sequences when the
 *       Hamiltonian has a multi-pass plan with at least two segments (N >= 16):
 *       1 runs them as a stack of separate vectors through the multi-pass
 *       kernels in one grid, whatever "hv_variant" says (one more vector per
 *       sequence for its partial sums), 0 uses the
 *       block layout (entry (x, r) at x*B + r) of the batched kernels, -1
 *       (default) takes the autotuner's pick for that B, else 1.  Elsewhere the
 *       block layout is used.
 * The settings are process-wide and read by every later call: change them only
 * while no other thread is inside the library (a running server's workers
 * included). */
ftk_status ftk_set_tuning(const char *key, int value);
ftk_status ftk_ctx_kernel_time(ftk_ctx *ctx, const char *kernel, int *count, double *mean_ms);

/* ------------------------------------------------------------------------ */
/* Periodic honeycomb clusters (Sec. V, Fig. 2 caption).
 * z bonds are horizontal and x, y bonds lie on the -60 / +60 degree lines: an A
 * site at R has B neighbours at R + d_g, d_z = (1, 0), d_x = (-1/2, sqrt3/2),
 * d_y = (-1/2, -sqrt3/2).  Bravais vectors a1 = d_z - d_x, a2 = d_z - d_y; the
 * supercell is T1 = t11 a1 + t12 a2, T2 = t21 a1 + t22 a2 with |det| cells.
 * Cells are the representatives 0 <= c1 < p, 0 <= c2 < q (p = gcd(t11, t21),
 * q = |det|/p), cell index c = c1 + p c2, A site 2c, B site 2c + 1; bonds are
 * listed cell by cell as (A, B, gamma) in gamma order x, y, z, and site_xy holds
 * each site's own position.
 * Call with NULL arrays to get n_sites and n_bonds; then pass arrays of
 * n_bonds (bond_*) and 2 n_sites (site_xy) entries.  FTK_EINVAL if the
 * supercell is degenerate or so small that two bonds join the same pair. */
ftk_status ftk_honeycomb_cluster(int t11, int t12, int t21, int t22, int *n_sites, int *n_bonds,
                                 int32_t *bond_i, int32_t *bond_j, int8_t *bond_gamma,
                                 double *site_xy);
/* Momenta allowed by the supercell (e^{iQ.T1} = e^{iQ.T2} = 1), folded into the
 * first Brillouin zone, as Cartesian pairs.  NULL q_xy returns the count. */
ftk_status ftk_honeycomb_momenta(int t11, int t12, int t21, int t22, int *n_q, double *q_xy);
/* "Gamma", "M" = (b1 + b2)/2, "M'" = b1/2, "K" = (2 b1 + b2)/3 with
 * b1 = (2pi/3, -2pi/sqrt3), b2 = (2pi/3, 2pi/sqrt3). */
ftk_status ftk_named_momentum(const char *name, double *q_xy);

typedef struct {
    int n_sites;
    int n_bonds;
    const int32_t *bond_i;     /* [n_bonds] site indices in [0, n_sites) */
    const int32_t *bond_j;     /* [n_bonds] */
    const int8_t *bond_gamma;  /* [n_bonds] 0 = x, 1 = y, 2 = z */
    const double *site_xy;     /* [n_sites][2] position R_l of each site */
} ftk_cluster;

/* ------------------------------------------------------------------------ */
/* Kitaev-Heisenberg Hamiltonian (Sec. V.A, Eq. H_ij):
 *   H = sum_b [J S_i.S_j + K S_i^gamma S_j^gamma],  S = sigma/2.
 * Matrix-free: only the bond table (a few hundred bytes) goes to the device.
 * FTK_EINVAL: n_sites outside [4, 30], a bond index out of range, i == j,
 * gamma outside {0, 1, 2}, a repeated bond, non-finite K or J. */
typedef struct ftk_hamiltonian ftk_hamiltonian;
ftk_status ftk_build_hamiltonian(ftk_ctx *ctx, const ftk_cluster *cluster, double K, double J,
                                 ftk_hamiltonian **out);
ftk_status ftk_hamiltonian_destroy(ftk_hamiltonian *h);
/* Segments of the multi-pass H v for this cluster's bond list (host only):
 * n_passes (0: none), the core size (sites 0..core-1 are in every pass tile),
 * and the end of every segment in the bond list (segment_end[n_passes], may be
 * NULL; at most 6). */
ftk_status ftk_hv_plan(const ftk_cluster *c, int *n_passes, int *core, int *segment_end);
/* A relabelling of the cluster for the multi-pass H v (host only): site l
 * becomes site site_perm[l] and the k-th bond of the new list is bond
 * bond_order[k] of the old one, chosen (deterministic annealing) so that the
 * bond list cuts into the fewest segments whose sites fit a 4096-element tile
 * together with the core sites 0..c-1, and then c in [4, 6] is as large as
 * possible (tiles are read in runs of 2^c elements).  The relabelled cluster is the same
 * physical system in another basis order.  *n_passes gets that number (0 and
 * the identity when no plan of at most 6 passes exists).  Arrays [n_sites],
 * [n_bonds], caller-allocated. */
ftk_status ftk_plan_layout(const ftk_cluster *c, int *site_perm, int *bond_order, int *n_passes);
/* n_sites and B_H = sum over bonds of the largest |bond eigenvalue| (>= ||H||). */
ftk_status ftk_hamiltonian_info(const ftk_hamiltonian *h, int *n_sites, double *norm_bound);

/* w = H v for n_rhs vectors stored one after another (2^N complex each).
 * Per element x, in this order: S_all and S_z = sums of s_b = +1 (parallel
 * spins) / -1 over all bonds and over z bonds; D = fma(K/4, S_z, (J/4) S_all);
 * acc = D v[x]; then for every bond b in list order
 * acc = fma(amp_b, v[x ^ (2^i | 2^j)], acc) with amp_b = (c_x - c_y)/4 for a
 * parallel pair and (c_x + c_y)/4 otherwise, c_a = J + K [a == gamma_b];
 * real and imaginary parts separately.  v and w must not overlap. */
ftk_status ftk_apply_h(const ftk_hamiltonian *h, const double *v_dev, double *w_dev, int n_rhs);
/* The same for n_rhs vectors ld >= 2^N complex entries apart (vector r starts at
 * entry r*ld of v_dev and of w_dev); FTK_EINVAL if ld < 2^N or the spans of v
 * and w overlap. */
ftk_status ftk_apply_h_strided(const ftk_hamiltonian *h, const double *v_dev, double *w_dev, int n_rhs, int64_t ld);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): w = H v exactly as
 * ftk_apply_h computes it (same kernels, bit-identical results), with the partial
 * sums of the multi-pass form kept in a static device array of the library
 * (2^22 complex entries, 64 MiB per GPU, held until the process ends) instead of
 * the Hamiltonian's scratch vector.  The call allocates nothing, on the device or
 * through the context's allocator; v_dev and w_dev are caller-owned, n_rhs
 * vectors of 2^N complex entries one after another, not overlapping.  The first
 * call on a GPU looks the array's device address up once.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other streams,
 * other threads) race, so serialise them.  FTK_EINVAL when the Hamiltonian's
 * H v is the multi-pass form on more than 22 sites (forms that need no partial
 * sums run at any size), or for NULL/overlapping arguments. */
ftk_status ftk_apply_h_noalloc(const ftk_hamiltonian *h, const double *v_dev, double *w_dev, int n_rhs);

/* Device bounds checks (a service of the library, not of the method).  The debug
 * build libftkw_check.so (same sources, -DFTK_DEVICE_CHECKS) checks every gather and
 * scatter index of the H v kernels (global vectors and LDS tiles), of the S^alpha_Q
 * gathers and of the filter accumulation against its buffer's extent; a violation
 * is counted in a device word and the access is redirected to entry 0, so the
 * kernel ends normally.  This call waits for ctx's stream and returns compiled (1
 * in the debug build, 0 in the release build, whose counters read 0), the number
 * of violations on ctx's device since the last clear, the site code of the first
 * (1 single-element H v, 2/3 blocked/tiled partner in HBM/LDS, 4/5 own elements in
 * HBM/LDS, 6/7 multi-pass element/tile entry, 8 multi-pass LDS partner, 9 staged
 * bond constants, 10/11 batch-layout own/partner, 12 S^alpha_Q, 13 filter
 * coefficients) and its index; clear != 0 resets them.  Any output may be NULL. */
ftk_status ftk_device_checks(ftk_ctx *ctx, int *compiled, uint32_t *violations, uint32_t *first_site,
                             uint32_t *first_index, int clear);
/* Debug build only (FTK_EINVAL in the release build): one kernel claims entry 5 of
 * a 4-entry buffer at site 99 without touching memory there; the check counts it
 * (ftk_device_checks then reports it) and *redirected = the index used instead, 0. */
ftk_status ftk_device_checks_selftest(ftk_ctx *ctx, uint32_t *redirected);

/* ------------------------------------------------------------------------ */
/* Random start vector (Sec. II.A): g_x = r cos(th) + i r sin(th), r = sqrt(-2 ln u1),
 * th = 2 pi u2, with u1 = ((o1 >> 11) + 1) 2^-53 and u2 = (o2 >> 11) 2^-53 taken
 * from outputs o1 = 2x+1 and o2 = 2x+2 of the counter-form SplitMix64 stream
 * (Steele, Lea, Flood 2014: output k of a stream seeded with s is mix(s + k G),
 * G = 0x9E3779B97F4A7C15) keyed by output sample+1 of the stream seeded with
 * seed.  Writes 2^n_sites un-normalised complex draws to out_dev. */
ftk_status ftk_random_vector(ftk_ctx *ctx, uint64_t seed, uint64_t sample, int n_sites, double *out_dev);

/* Shell coefficients of the contour filters (Sec. III.B, Eq. dfilterP) from n
 * Lanczos coefficients of phi (alpha_0..alpha_{n-1}, beta_1..beta_{n-1}; beta
 * has n entries, the last unused) and norm = ||phi||: the host-side step of
 * ftk_typical_states.  out [L][n] complex:
 *   c^m = (norm/M) sum_j w_j y_mj, w_j = eps (cos th_j, sin th_j),
 *   th_j = 2 pi (j - 1/2)/M, (E_m + w_j - T_n) y_mj = e_1 solved by forward
 *   elimination and back substitution without pivoting, complex products
 *   (ac - bd, ad + bc), reciprocals (a/(aa+bb), -b/(aa+bb)), contour sum in j order. */
ftk_status ftk_filter_coefficients(const double *alpha, const double *beta, int n, double norm, double E_b,
                                   double eps, int L, int M, double *out);

/* Appendix A plan for e^{-beta H/2}: Md factors e^{c (l - H/N)}, c = N beta/(2 Md),
 * each a K-term Taylor series; l = norm_bound/N.  lambda <= 0 selects 1e8. */
ftk_status ftk_taylor_plan(int n_sites, double beta, double norm_bound, double lambda, int *Md, int *K,
                           double *c, double *ell);

/* ------------------------------------------------------------------------ */
/* Filtered typical pure states (Sec. II.A, Eq. tau, Sec. III.B, Eq. filtered).
 * For every vector s and anchor a:
 *   phi_0 = g / ||g|| with g complex Gaussian (SplitMix64 counter stream keyed
 *           by (seed, first_vector + s) and Box-Muller), or g taken from
 *           gaussian_dev[s] when given;
 *   phi_beta = e^{-beta_a H/2} phi_0 by the Taylor series of Appendix A in M_d
 *           factors (each factor renormalised; log of the norm kept);
 *   n_steps Lanczos steps from phi_beta (T_n); for every shell m < L the
 *           coefficients c^m of phi^m = P_{E_m, eps_a, M} phi_beta =
 *           (||phi_beta||/M) sum_j eps e^{i th_j} V_n (z_mj - T_n)^{-1} e_1,
 *           E_m = E_b + (2m+1) eps, th_j = 2 pi (j - 1/2)/M;
 *   phi^m accumulated on the device from regenerated Lanczos vectors, and
 *           n_m = <phi^m|phi^m>.
 * Memory: L vectors per (s, a) stay resident, plus block_steps vectors of
 * workspace (block_steps = 0 picks min(n_steps, 64)).
 * E_b = eps = NULL: each anchor's window is [theta_min - window_margin,
 * theta_max + window_margin] (L shells of width 2 eps), theta the extreme Ritz
 * values of T_n of vector 0 of the call; ftk_states_scalars reports it.
 * resid_tol > 0: each filter operator is truncated on its own (Sec. V): shell
 * m uses T_{k_m}, k_m the first step after which its M contour shifts z_mj all
 * have Galerkin residual <= resid_tol per unit right-hand side (same recurrence
 * as the Green's functions, evaluated on the host from the first pass); the
 * second pass regenerates max_m k_m vectors, and ftk_states_lanczos reports that
 * many coefficients.
 * FTK_EINVAL: M odd or < 2, L < 1, eps <= 0, beta < 0, n_steps < 1;
 * FTK_ENOMEM if the states do not fit; FTK_ENUMERIC on NaN/Inf. */
typedef struct {
    uint64_t seed;
    int first_vector;            /* index of vector 0 in the seed's stream */
    int n_vectors;
    const double *anchor_beta;   /* [n_anchors]; 0 means T = infinity */
    int n_anchors;
    const double *E_b;           /* [n_anchors] lower end of the shell grid */
    const double *eps;           /* [n_anchors] contour radius = shell half-width */
    int L;                       /* shells per anchor */
    int M;                       /* contour points, even, >= 2 */
    int n_steps;                 /* Lanczos steps of the filter (at most, see resid_tol) */
    double taylor_lambda;        /* Appendix A bound Lambda; 0 -> 1e8 */
    const double *gaussian_dev;  /* optional [n_vectors][2^N] complex draws */
    int block_steps;             /* Lanczos vectors buffered per accumulation pass */
    double window_margin;        /* used when E_b and eps are both NULL (0 -> 0.1) */
    double resid_tol;            /* 0: fixed n_steps */
    int shell_moments;           /* 1: also <phi^m|H|phi^m> and ||H phi^m||^2 (one H v per shell) */
} ftk_ts_params;

typedef struct ftk_states ftk_states;
ftk_status ftk_typical_states(const ftk_hamiltonian *h, const ftk_ts_params *p, ftk_states **out);
/* log_norm [nv][na] = log ||e^{-beta H/2} phi_0||; shell_norm2 [nv][na][L] = n_m;
 * E_m [na][L]; eps [na].  Any pointer may be NULL. */
ftk_status ftk_states_scalars(const ftk_states *st, double *log_norm, double *shell_norm2,
                              double *E_m, double *eps);
/* Per-shell moments h1 = <phi^m|H|phi^m>, h2 = <H phi^m|H phi^m> ([nv][na][L],
 * phi^m of the normalised phi_beta, exact-sum dot products); FTK_EINVAL unless
 * the states were built with shell_moments = 1. */
ftk_status ftk_states_moments(const ftk_states *st, double *h1, double *h2);
/* Shell window (E_b [na], eps [na]) the states were built on. */
ftk_status ftk_states_window(const ftk_states *st, double *E_b, double *eps);
/* Filter Lanczos coefficients alpha_0..alpha_{n-1}, beta_1..beta_n of (s, a). */
ftk_status ftk_states_lanczos(const ftk_states *st, int s, int a, double *alpha, double *beta,
                              int *n_steps);
/* Copy phi^m of (s, a) (2^N complex) to out_dev. */
ftk_status ftk_states_copy_shell(const ftk_states *st, int s, int a, int m, double *out_dev);
ftk_status ftk_states_destroy(ftk_states *st);

/* ------------------------------------------------------------------------ */
/* Equi-energy Green's functions (Sec. III.C, Eqs. GAB_TPS and SQomega_TPS):
 * for every (s, a, m, alpha, Q) with n_m > 0,
 *   chi = S^alpha_{+Q} phi^m, S^alpha_{+Q} = N^{-1/2} sum_l e^{iQ.R_l} S^alpha_l,
 *   g(omega) = <chi|(omega + i eta + E_m - H)^{-1}|chi>
 *            = ||chi||^2 [(z - T_n)^{-1}]_{00}  from n_steps Lanczos steps,
 * the 00 element accumulated per shift with the forward LDL^T recurrence
 * (d_0 = z - alpha_0, p_0 = 1; p_k = p_{k-1} beta_k / d_{k-1},
 *  d_k = z - alpha_k - beta_k^2 / d_{k-1}; G = sum_k p_k^2 / d_k), and the
 * Galerkin residual ||chi|| |p_n| kept per sequence (maximum over shifts).
 * rhs_block (1, 2, 4, 8, 16 or 32) sets how many sequences share one launch; 0
 * takes the value ftk_autotune picks for this Hamiltonian and n_omega.  32 runs
 * only as a stack of multi-pass sequences (N >= 16, see "stack_batch").
 * resid_tol > 0 truncates each sequence at the first step k <= n_steps after
 * which the largest Galerkin residual over the shifts, per unit right-hand side
 * (|p_k| beta_{k+1} / |d_k|), is <= resid_tol (Sec. V, truncation of the CG
 * steps by the largest residual 2-norm); 0 runs n_steps (or to breakdown).
 * first_shell, n_shells restrict the work to the shells m in
 * [first_shell, first_shell + n_shells) of every (s, a) (n_shells = 0: to the
 * last shell), so that a job can be cut into bounded pieces; the outputs keep
 * their full [L] shape with zeros for the shells left out.
 * solver selects the shifted Krylov method (Sec. II.B):
 *   FTK_SOLVER_LANCZOS (0): the Lanczos-Galerkin values above, i.e. shifted BiCG
 *       with the shadow vector equal to the right-hand side;
 *   FTK_SOLVER_COCG (1): shifted COCG, i.e. shifted BiCG with the shadow vector
 *       conj(chi) (z - H is complex symmetric), with seed switching (Appendix C).
 *       The basis is the complex-symmetric Lanczos basis q_k (q_j^T q_k = delta_jk):
 *       u = (H w_{k-1}) inv_k + c1 w_{k-2}, c1 = -(b_k inv_{k-1}); a_k = inv_k
 *       (w_{k-1}^T u); w_k = u + c2 w_{k-1}, c2 = -(a_k inv_k); b_{k+1} =
 *       csqrt(w_k^T w_k), inv_{k+1} = 1/b_{k+1} (complex; per element
 *       t = (Hw) inv, u = (fma(c1r, wpr, fma(-c1i, wpi, tr)), fma(c1r, wpi,
 *       fma(c1i, wpr, ti))), w = (fma(c2r, wcr, fma(-c2i, wci, ur)), fma(c2r, wci,
 *       fma(c2i, wcr, ui))), t by the same product; bilinear sums exact), with the
 *       projections c_k = <chi|q_k>.  Every shift runs the shifted COCG recurrence
 *       of the seed's CG (1/alpha_k = z_s - a_k - b_k^2 alpha_{k-1}, beta_k =
 *       b_{k+1}^2 alpha_k^2); g = <chi|x_n(z)>.  The seed starts at the first
 *       frequency and moves to the shift with the largest residual 2-norm once its
 *       own is <= seed_tol ||chi|| (0 -> 1e-12).  Any other shift whose residual
 *       is <= seed_tol ||chi|| is converged and keeps its value; the sequence ends
 *       once every shift is converged (else after n_steps, a breakdown or the
 *       resid_tol truncation).  For a complex chi the finite-n values differ from
 *       Lanczos-Galerkin; both converge to the resolvent.
 *       Sequences run one per launch (rhs_block is not used); max_resid is the
 *       largest residual 2-norm over the shifts.
 * FTK_EINVAL: eta <= 0, n_omega < 1, n_q < 1, empty alpha_mask, n_steps < 1,
 * resid_tol < 0, a shell range outside [0, L), an unknown solver, seed_tol < 0. */
enum { FTK_SOLVER_LANCZOS = 0, FTK_SOLVER_COCG = 1 };
typedef struct {
    const double *q_xy;   /* [n_q][2] */
    int n_q;
    int alpha_mask;       /* bit 0 = x, bit 1 = y, bit 2 = z */
    const double *omega;  /* [n_omega] */
    int n_omega;
    double eta;
    int n_steps;
    int rhs_block;
    double resid_tol;     /* 0: fixed n_steps */
    int first_shell;      /* 0: from shell 0 */
    int n_shells;         /* 0: to shell L - 1 */
    int solver;           /* FTK_SOLVER_LANCZOS (0) or FTK_SOLVER_COCG (1) */
    double seed_tol;      /* COCG seed switching threshold per unit right-hand side; 0 -> 1e-12 */
} ftk_spec_params;

typedef struct ftk_spectrum ftk_spectrum;
/* Autotuner: times short Green's-function runs (random start vectors, 64 steps,
 * n_omega shifts) of rhs_block in {1, 4, 16, 32}, each B > 1 in both batch layouts
 * where the stacked one applies (see "stack_batch"), on this Hamiltonian and
 * returns the fastest rhs_block with its Krylov iterations per second.  When the
 * winner runs the multi-pass kernels (one sequence, or a stack) it then times it
 * with half and twice the default persistent workgroups per reducing pass (two per
 * compute unit, or the "pass_grid" tuning value) and keeps a grid that wins by
 * 0.5 %, then with the other cache-hint set than the default rule's (see
 * "stream_hints"; unless that key forces one) and keeps it if it wins by 0.5 %;
 * results depend on neither (exact partial sums; hints and tile order only).  The
 * spectrum then uses the layout, grid and hint set that won.  Results are kept per
 * (n_sites, n_omega, device name) for the process and, when the environment
 * variable FTK_TUNE_CACHE names a file, read from and written to that JSON file.
 * Either output pointer may be NULL. */
ftk_status ftk_autotune(const ftk_hamiltonian *h, int n_omega, int *rhs_block, double *iters_per_s);
/* The layout of the autotuner's pick: 1 a stack of multi-pass sequences, 0 the
 * block layout or one sequence per launch (runs the autotuner if needed). */
ftk_status ftk_autotune_layout(const ftk_hamiltonian *h, int n_omega, int *stacked);
/* Every candidate the autotuner timed in this process for (h, n_omega), in the
 * order tried: rhs_block, layout (1 stacked), Krylov iterations per second, the
 * pass grid (0: the default) and the cache-hint set it ran with (1 streaming,
 * 0 cached; see "stream_hints"), up to max_n of them; pass_grid and hints may be
 * NULL; n = 0 when the pick came from the cache file. */
ftk_status ftk_autotune_candidates(const ftk_hamiltonian *h, int n_omega, int max_n, int *n, int *rhs_block,
                                   int *stacked, double *iters_per_s, int *pass_grid, int *hints);
ftk_status ftk_shifted_krylov_spectrum(const ftk_hamiltonian *h, const ftk_states *st,
                                       const ftk_spec_params *p, ftk_spectrum **out);
/* g [nv][na][L][n_alpha][n_q][n_omega] complex (n_alpha = set bits of the mask,
 * in x, y, z order); max_resid [nv][na][L][n_alpha][n_q].  Either may be NULL. */
ftk_status ftk_spectrum_raw(const ftk_spectrum *sp, double *g, double *max_resid);
/* Work done: Krylov steps summed over the sequences that ran (empty shells and
 * shells outside the requested range run none) and the number of those sequences. */
ftk_status ftk_spectrum_work(const ftk_spectrum *sp, int64_t *krylov_steps, int *sequences);
/* ||chi||^2 = <phi^m|S^alpha_{-Q} S^alpha_{+Q}|phi^m> of every sequence
 * [nv][na][L][n_alpha][n_q] (0 for empty shells): the static structure factor's
 * shell values for ftk_reweight_observable. */
ftk_status ftk_spectrum_norms(const ftk_spectrum *sp, double *chi2);
/* Lanczos coefficients of one sequence (alpha_0..alpha_{n-1}, beta_1..beta_n). */
ftk_status ftk_spectrum_lanczos(const ftk_spectrum *sp, int s, int a, int m, int ia, int iq,
                                double *alpha, double *beta, int *n_steps);
/* Shifted COCG runs only: the complex-symmetric Lanczos scalars of one sequence,
 * a_0..a_{n-1} and b_1..b_n (complex [n]), c_0..c_n = <chi|q_k> (complex [n+1]),
 * n_steps and the final seed index; FTK_EINVAL for a Lanczos-Galerkin spectrum. */
ftk_status ftk_spectrum_cocg(const ftk_spectrum *sp, int s, int a, int m, int ia, int iq, double *a_out,
                             double *b_out, double *c_out, int *n_steps, int *seed);
ftk_status ftk_spectrum_destroy(ftk_spectrum *sp);

/* ------------------------------------------------------------------------ */
/* One Green's-function sequence that can be stopped, saved and resumed (the
 * Lanczos recurrence of Sec. II.B with the multi-shift update of Sec. III.C; the
 * paper has no checkpoints, so this is a service of the library): the state after
 * k steps is w_{k-1}, w_{k-2} (the start vector standing in for w_{-1}), the
 * sequence scalars, alpha_0..alpha_{k-1}, beta_1..beta_k and the per-shift LDL^T
 * state (d, p, G).  Steps run in chunks on the kernels of
 * ftk_shifted_krylov_spectrum; a chunk ends with both halves of its last step,
 * and since every reduction is an exact sum rounded once, the sequence run in
 * any chunks, saved and resumed in this process or another, gives bit for bit
 * the coefficients and g of the straight run.
 *
 * create: chi_dev is the right-hand side (2^N complex, device, copied), omega
 *   [n_omega] host (copied), shifts z = omega + shift_re + i eta, at most n_max
 *   steps.  FTK_EINVAL for n_omega < 1, n_max < 1, eta <= 0 or non-finite
 *   numbers; FTK_ENUMERIC when ||chi|| is zero or not finite.
 * advance: runs up to n_steps more steps (fewer at n_max, none once the sequence
 *   ended at a breakdown); *steps (may be NULL) = steps done in all.
 *   FTK_ENUMERIC when a coefficient turned NaN/Inf.
 * read: g [n_omega] complex = ||chi||^2 [(z - T_k)^{-1}]_00 after the steps done
 *   (zeros before the first), alpha/beta [steps], steps, the largest Galerkin
 *   residual over the shifts, done (breakdown, numeric error or n_max reached).
 *   Any output may be NULL.
 * save: *bytes = the size of the state; with buf != NULL writes it there (cap
 *   bytes; FTK_EINVAL when too small).  The state is a plain byte string (header,
 *   omega, scalars, coefficients, two vectors, a checksum) for this library's
 *   build; the caller owns the buffer.
 * restore: a new sequence on h from a saved state; FTK_EINVAL for a truncated or
 *   corrupt state (bad magic or checksum) or one saved on another Hamiltonian
 *   (site count or bond table differ).  The caller destroys every sequence. */
typedef struct ftk_green_seq ftk_green_seq;
ftk_status ftk_green_seq_create(const ftk_hamiltonian *h, const double *chi_dev, const double *omega, int n_omega,
                                double eta, double shift_re, int n_max, ftk_green_seq **out);
ftk_status ftk_green_seq_advance(ftk_green_seq *q, int n_steps, int *steps);
ftk_status ftk_green_seq_read(ftk_green_seq *q, double *g, double *alpha, double *beta, int *steps,
                              double *max_resid, int *done);
ftk_status ftk_green_seq_save(ftk_green_seq *q, void *buf, size_t cap, size_t *bytes);
ftk_status ftk_green_seq_restore(const ftk_hamiltonian *h, const void *buf, size_t bytes, ftk_green_seq **out);
/* n_omega, n_max and the size of a saved state (any may be NULL). */
ftk_status ftk_green_seq_info(const ftk_green_seq *q, int *n_omega, int *n_max, size_t *state_bytes);
ftk_status ftk_green_seq_destroy(ftk_green_seq *q);

/* ------------------------------------------------------------------------ */
/* Green's functions of general operator pairs (Sec. III.B; Eq. GAB_TPS with
 * A != B): per shell and pair,
 *   G_AB(omega) = <phi^m|A^dag (omega + i eta + E_m - H)^{-1} B|phi^m>
 *              = <lam|(z - H)^{-1}|rho>,  lam = A phi^m, rho = B phi^m,
 * and G_BA with A and B exchanged.  A and B are linear spin operators
 * A = sum_l sum_alpha a_{l alpha} S^alpha_l with complex coefficients (S^alpha_{+Q}
 * is a_{l alpha} = e^{iQ.R_l}/sqrt(N) on one component; a local S^alpha_j is one
 * entry 1).  The sesquilinear form is split by the polarization identity into
 * four ordinary Green's sequences from lam + rho, lam - rho, lam + i rho,
 * lam - i rho (k = 0..3), run exactly as ftk_shifted_krylov_spectrum runs its
 * sequences (same kernels, batching, truncation), and
 *   G_AB = (g_0 - g_1 - i g_2 + i g_3) / 4,   G_BA = (g_0 - g_1 + i g_2 - i g_3) / 4,
 *   <lam|rho> = (|s_0|^2 - |s_1|^2 + i (|s_3|^2 - |s_2|^2)) / 4.
 * The pair's spectral density is -(1/(2 pi i)) (G_AB(w + i eta) - conj(G_BA(w + i eta))).
 * op_a, op_b: [n_pairs][n_sites][3] complex, interleaved (alpha = x, y, z);
 * copied at the call.  Other fields as in ftk_spec_params.
 * solver = FTK_SOLVER_COCG is shifted BiCG with the shadow vector conj(rho) as the
 * paper writes it for A != B (Sec. II.B): two shifted COCG runs per pair instead of
 * four polarization sequences, G_AB = <lam|x(z)> from the run on rho (projections
 * c_k = <lam|q_k>) and G_BA from the run on lam projected on rho; <lam|rho> =
 * c_0 delta_0 of the first run; max_resid the larger of the two runs' largest
 * residuals.  ftk_pair_cocg returns each run's scalars.  FTK_EINVAL: no pair,
 * NULL operators, non-finite coefficients or frequencies, eta <= 0, n_steps < 1,
 * bad rhs_block, resid_tol < 0, an unknown solver, seed_tol < 0. */
typedef struct {
    const double *op_a;   /* [n_pairs][n_sites][3][2] */
    const double *op_b;   /* [n_pairs][n_sites][3][2] */
    int n_pairs;
    const double *omega;  /* [n_omega] */
    int n_omega;
    double eta;
    int n_steps;
    int rhs_block;        /* 0 (autotuned), 1, 2, 4, 8, 16, 32 sequences per launch */
    double resid_tol;     /* 0: fixed n_steps */
    int solver;           /* FTK_SOLVER_LANCZOS (0) or FTK_SOLVER_COCG (1), see below */
    double seed_tol;      /* COCG seed switching threshold; 0 -> 1e-12 */
} ftk_pair_params;

typedef struct ftk_pair_spectrum ftk_pair_spectrum;
ftk_status ftk_pair_green(const ftk_hamiltonian *h, const ftk_states *st, const ftk_pair_params *p,
                          ftk_pair_spectrum **out);
/* g_ab, g_ba [nv][na][L][n_pairs][n_omega] complex; overlap [nv][na][L][n_pairs]
 * complex <A phi^m|B phi^m>; max_resid [nv][na][L][n_pairs] (largest of the four
 * sequences).  Empty shells give zeros.  Any pointer may be NULL. */
ftk_status ftk_pair_raw(const ftk_pair_spectrum *sp, double *g_ab, double *g_ba, double *overlap,
                        double *max_resid);
/* Lanczos coefficients of polarization sequence k (0..3) of pair p. */
ftk_status ftk_pair_lanczos(const ftk_pair_spectrum *sp, int s, int a, int m, int p, int k, double *alpha,
                            double *beta, int *n_steps);
/* Shifted COCG pair spectra: run k (0: on rho = B phi^m, G_AB; 1: on lam = A phi^m,
 * G_BA) of pair p, as ftk_spectrum_cocg. */
ftk_status ftk_pair_cocg(const ftk_pair_spectrum *sp, int s, int a, int m, int p, int k, double *a_out,
                         double *b_out, double *c_out, int *n_steps, int *seed);
ftk_status ftk_pair_destroy(ftk_pair_spectrum *sp);
/* Coefficients [n_sites][3] complex of S^alpha_{+Q} = N^{-1/2} sum_l e^{iQ.R_l} S^alpha_l
 * (Sec. V) for ftk_pair_params: e^{iQ.R_l}/sqrt(N) on component alpha, zero
 * elsewhere (exactly twice the per-site factors the spectrum kernels use).
 * site_xy [n_sites][2]. */
ftk_status ftk_momentum_operator(int n_sites, const double *site_xy, int alpha, double qx, double qy,
                                 double *coef);

/* ------------------------------------------------------------------------ */
/* The automatic window as a host function: extreme eigenvalues of the
 * tridiagonal T_n (alpha[0..n-1], beta[0..n-2]) by Sturm bisection, then
 * E_b = theta_min - margin and eps = (theta_max + margin - E_b) / (2 L). */
ftk_status ftk_shell_window(const double *alpha, const double *beta, int n, int L, double margin, double *E_b,
                            double *eps);

/* Eq. FRW1 for real static observables: O [nv][na][L][n_obs] holds the shell
 * values <phi^m|O_k|phi^m> (e.g. ftk_spectrum_norms summed over alpha for the
 * static structure factor); out [n_obs][n_T] = sum W O / sum W n with the
 * anchors and weights of ftk_reweight; err (optional) binned likewise. */
ftk_status ftk_reweight_observable(int n_vectors, int n_anchors, int L, int n_obs, const double *anchor_beta,
                                   const double *E_m, const double *log_norm, const double *shell_norm2,
                                   const double *O, const double *T, int n_T, int n_bins, double *out, double *err);

/* Thermodynamics from the shell data (Sec. II.A: Z(beta) = N_F E[||phi_beta||^2];
 * Eq. FRW1 with O = H, H^2), per target temperature T' with the anchor a chosen
 * as in ftk_reweight, W_sm = exp(2 log_norm_s + (beta_a - beta') E_m):
 *   E = sum W h1 / sum W n,  C = beta'^2 (sum W h2 / sum W n - E^2),
 *   ln Z = N ln 2 + ln mean_s exp(2 log_norm_s) + ln(sum W n / sum W(beta_a) n),
 *   S = beta' E + ln Z  (k_B = 1; F = -T ln Z),
 * sums over samples and shells with n_m > 0.  h1, h2 ([nv][na][L], from
 * ftk_states_moments) may be NULL: E_m n_m and E_m^2 n_m stand in.  out and err
 * (optional, binned as in ftk_reweight) are [n_T][4] = (E, C, S, ln Z). */
ftk_status ftk_thermodynamics(int n_vectors, int n_anchors, int L, const double *anchor_beta, const double *E_m,
                              const double *log_norm, const double *shell_norm2, const double *h1,
                              const double *h2, int n_sites, const double *T, int n_T, int n_bins, double *out,
                              double *err);

/* Diagnostics from the same shell data, per inverse temperature b (b >= 0):
 *   out[i][0] = <H^2> - <H>^2 at b (the squared width C/(k_B b^2) of the energy
 *               distribution, Sec. III.D);
 *   out[i][1] = ln[Z(2b)/Z(b)^2] (Sec. III.C, V.B: = -S(b*) for some b* in [b, 2b]; between
 *               -N ln 2 and -ln D, D the ground-state degeneracy; the sample scatter
 *               of the estimator scales with its square root),
 * each from the anchors ftk_thermodynamics picks for b and for 2b; err
 * (optional) binned on the same samples. */
ftk_status ftk_thermo_diagnostics(int n_vectors, int n_anchors, int L, const double *anchor_beta,
                                  const double *E_m, const double *log_norm, const double *shell_norm2,
                                  const double *h1, const double *h2, int n_sites, const double *inv_T, int n_T,
                                  int n_bins, double *out, double *err);
/* Anchor ladder (Sec. III.D): reweighting from b_a to b' works while the energy
 * distributions overlap, r = |<H>_a - <H>_b'| / (sigma_a + sigma_b') small
 * (sigma^2 = <H^2> - <H>^2).  On an ascending grid of inverse temperatures with
 * <H> and the variance there (e.g. from ftk_thermodynamics and
 * ftk_thermo_diagnostics of a hot run), the first anchor is grid point 0 and each
 * next one is the first grid point whose r with the current anchor exceeds r_max,
 * so every grid point is reweighted (from the hottest anchor at or above it, as
 * ftk_reweight does) with r <= r_max unless max_anchors runs out.  anchors
 * receives up to max_anchors grid indices, n_anchors their number. */
ftk_status ftk_choose_anchors(int n, const double *beta_grid, const double *E, const double *var, double r_max,
                              int max_anchors, int *anchors, int *n_anchors);

/* Residual-controlled truncation as a host function: the smallest k in [1, n]
 * after which every shift z has Galerkin residual |p_{k-1}| beta_k / |d_{k-1}|
 * <= tol per unit right-hand side (the device's multi-shift recurrence), n if
 * none.  alpha[0..n-1], beta[0..n-1] = beta_1..beta_n. */
ftk_status ftk_truncation_steps(const double *alpha, const double *beta, int n, const double *z_re,
                                const double *z_im, int n_z, double tol, int *k);
/* The CG-step dependence of the largest residual 2-norm over the shifts (Sec. V):
 * out[k] = max_z |p_k| beta_{k+1} / |d_k| after k + 1 steps, per unit right-hand
 * side, for k = 0..n-1.  The paper's shifted BiCG with the shadow vector equal to
 * the right-hand side has the Lanczos-Galerkin iterate at every step, so these
 * are its residual norms (the seed-switched maximum over the shifts). */
ftk_status ftk_residual_history(const double *alpha, const double *beta, int n, const double *z_re,
                                const double *z_im, int n_z, double *out);

/* Width of a spectral peak (Sec. V.F, Eq. asymmetricLorentzian): least-squares
 * fit of the asymmetric Lorentzian
 *   s(w) = gamma / (gamma^2 + (w - eps)^2) * (a + b / (1 + exp(c (w - eps))))
 * to the points (omega[i], s[i]) with lo <= omega[i] <= hi (at least 5, ascending;
 * e.g. a reweighted S(Q, omega, T') from ftk_reweight), by Levenberg-Marquardt with
 * analytic derivatives; gamma / eps measures the width of the peak.  Host arrays,
 * copied at the call.  init (optional) is the start (a, b, c, gamma, eps); NULL
 * starts from the windowed data: eps at the largest value y_max, gamma the half
 * width at half maximum (mean of the distances to the nearest points below y_max/2
 * on each side where there is one; a quarter of the window if neither side has),
 * a = 0.75 y_max gamma, b = 0.5 y_max gamma, c = 0.  params [5] receives
 * (a, b, c, gamma, eps) with gamma > 0 (gamma, a, b -> -gamma, -a, -b leaves the
 * curve unchanged); cost (optional) = 0.5 sum of squared residuals; iters
 * (optional) = iterations taken (max_iter, 0 => 1000); width_ratio (optional) =
 * gamma_f / eps_f, the peak's relative width (+infinity for a peak centred at
 * eps = 0).  FTK_EINVAL for bad
 * arguments, fewer than 5 points or no positive peak in the window; FTK_ENUMERIC if
 * the fit ends on non-finite parameters. */
ftk_status ftk_fit_asymmetric_lorentzian(const double *omega, const double *s, int n, double lo, double hi,
                                         const double *init, int max_iter, double *params, double *cost,
                                         int *iters,
                                         double *width_ratio);

/* Reweighting (Sec. III.D, Eqs. FRW1 and FRW2; sample average as in Eq. limGAB):
 *   S(Q, omega, T') = -(1/pi) Im sum_s sum_m W_sm g_sm(omega) / sum_s sum_m W_sm n_sm,
 *   W_sm = exp(2 log_norm_s + (beta_a - beta') E_m),
 * with g summed over alpha and the anchor a of each T' the one with the largest
 * beta_a <= 1/T' (the smallest beta_a if none).  Exponents are shifted by their
 * maximum.  S_stderr (optional) from n_bins contiguous sample bins:
 * std(bin ratios, ddof 1)/sqrt(n_bins) (NaN below 2 bins); P (optional) is
 * Eq. FRW2, W n / (2 eps sum W n), per shell of the anchor used.
 * Shapes: E_m [na][L], eps [na], log_norm [nv][na], shell_norm2 [nv][na][L],
 * g [nv][na][L][n_q][n_omega] complex; outputs S [n_q][n_T][n_omega],
 * P [n_T][L].  FTK_EINVAL on T <= 0 or inconsistent sizes. */
ftk_status ftk_reweight(int n_vectors, int n_anchors, int L, int n_q, int n_omega,
                        const double *anchor_beta, const double *E_m, const double *eps,
                        const double *log_norm, const double *shell_norm2, const double *g,
                        const double *T, int n_T, int n_bins, double *S_out, double *S_stderr,
                        double *P_out);
/* ftk_reweight on the handles: g summed over the spectrum's alpha components (x,
 * y, z order) and the states' own scalars and shell energies.  S [n_q][n_T][n_omega],
 * S_err and P (optional) as in ftk_reweight. */
ftk_status ftk_reweight_spectrum(const ftk_states *st, const ftk_spectrum *sp, const double *T, int n_T,
                                 int n_bins, double *S, double *S_err, double *P);

/* Eq. FRW1 for operator pairs: the complex spectral density
 *   S_AB(omega, T') = -(1/(2 pi i)) sum W (G_AB - conj(G_BA)) / sum W n,
 * computed as two ftk_reweight runs: with X = (G_AB - conj(G_BA)) / 2, Re S_AB is
 * ftk_reweight of X and Im S_AB minus ftk_reweight of i X (same anchors, weights
 * and bins).  g_ab, g_ba [nv][na][L][n_pairs][n_omega] complex (ftk_pair_raw);
 * S [n_pairs][n_T][n_omega] complex; S_err (optional) holds the binned errors of
 * the real and imaginary parts as (re, im) pairs. */
ftk_status ftk_reweight_pair(int n_vectors, int n_anchors, int L, int n_pairs, int n_omega,
                             const double *anchor_beta, const double *E_m, const double *eps,
                             const double *log_norm, const double *shell_norm2, const double *g_ab,
                             const double *g_ba, const double *T, int n_T, int n_bins, double *S, double *S_err);

/* ------------------------------------------------------------------------ */
/* Serving: independent requests, each the whole method (typical states,
 * Green's functions, reweighting) for one Hamiltonian, on one GPU.
 *
 * A request is processed one start vector at a time (vector s uses stream
 * index first_vector + s); with E_b = eps = NULL its window comes from vector 0
 * (ftk_typical_states).  The result is S [n_q][n_T][n_omega] and its binned
 * standard error (min(8, n_vectors) bins), exactly what a standalone run of the
 * same calls gives: requests never share launches, and per-request arithmetic
 * does not depend on what else runs.
 *
 * Admission: each request reserves its peak device footprint
 * (ftk_request_footprint) and starts when one of n_workers worker streams is
 * free and the reservation fits in hbm_budget; the oldest waiting request goes
 * first, younger ones that fit may start ahead of it at most 4 times.  A
 * request larger than the budget is refused at submission (FTK_ENOMEM).
 * rhs_block 0 in a request takes the autotuner's recorded value for its size,
 * else 16 up to 20 sites and 1 above; block_steps 0 takes 16.  Requests
 * cannot pass gaussian_dev.  All calls are thread-safe.
 * When the environment variable FTK_SERVE_LOG names a file at server creation,
 * every request a worker ran appends one JSON line to it: ticket, status, sizes,
 * submission time, queue wait, latency, seconds in the Hamiltonian, states,
 * Green's functions and reweighting, Krylov steps and Krylov iterations per
 * second of its Green's sequences, their algorithmic GB/s (48 B per element and
 * step), the largest Galerkin residual, reserved and measured peak device bytes. */
typedef struct ftk_server ftk_server;
typedef struct {
    int64_t completed, failed, waiting;
    int running;
    double p50_latency_s, p99_latency_s;   /* submit to result, completed requests */
    double requests_per_s;                 /* completed / (last finish - first submit) */
    size_t hbm_budget, hbm_reserved, hbm_reserved_peak;
    double max_peak_over_footprint;        /* measured device peak / reservation, max over requests */
    int64_t cancelled;                     /* requests ended by ftk_server_cancel */
} ftk_serving_stats;

/* Peak device bytes a request of this shape reserves on a 2^n_sites system. */
ftk_status ftk_request_footprint(int n_sites, const ftk_ts_params *tp, const ftk_spec_params *sp, int device,
                                 size_t *bytes);
/* hbm_budget 0 -> 90% of the free device memory; n_workers 0 -> 4 (at most 16). */
ftk_status ftk_server_create(int device, size_t hbm_budget, int n_workers, ftk_server **out);
ftk_status ftk_server_submit(ftk_server *srv, const ftk_cluster *c, double K, double J, const ftk_ts_params *tp,
                             const ftk_spec_params *sp, const double *T, int n_T, uint64_t *ticket);
/* FTK_ENOTREADY while the request waits or runs; otherwise fills the outputs
 * (any may be NULL) or returns the request's error, and forgets the ticket. */
ftk_status ftk_server_poll(ftk_server *srv, uint64_t ticket, double *S_out, double *S_stderr, double *latency_s);
/* Blocks until the request is finished or timeout_s passes (FTK_ENOTREADY). */
ftk_status ftk_server_wait(ftk_server *srv, uint64_t ticket, double timeout_s);
ftk_status ftk_server_stats(ftk_server *srv, ftk_serving_stats *out);
/* Cancels a request: a waiting one leaves the queue at once; a running one stops
 * at its next stage boundary (after the Hamiltonian, after each start vector's
 * states and after each vector's Green's functions), frees its device memory and
 * its reservation.  Its poll and wait then report FTK_ECANCELED.  FTK_EINVAL for
 * an unknown ticket or a request that has already finished. */
ftk_status ftk_server_cancel(ftk_server *srv, uint64_t ticket);
/* Reserved bytes over time (seconds since creation) at every start and end of a
 * request; *n receives the number of records, at most cap are written. */
ftk_status ftk_server_occupancy(ftk_server *srv, double *t, double *bytes, int cap, int *n);
/* Drops waiting requests, finishes running ones, frees everything. */
ftk_status ftk_server_destroy(ftk_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* FTKW_H */
