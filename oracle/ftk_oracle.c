/*
 * CPU oracle for the FTKw hot path: the vector arithmetic, in plain C loops.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this file's library.  The product
 * (paper_1802_02854_amd/) never links, imports or calls it, and this file
 * shares no code with it.
 *
 * Everything is complex128, stored interleaved (re, im) in natural basis
 * order: basis index x = sum_l sigma_l 2^l, bit l = 0 means spin up on site l
 * (the bit-string basis of Sec. II.A).
 *
 * Arithmetic contract (why it is spelled out): a Lanczos recurrence amplifies
 * a one-ulp difference in its start vector to O(1e-3) differences in the
 * finite-n Green's function after a few dozen steps, so the oracle and the GPU
 * path must perform the same IEEE operations on every vector element.  The
 * order below is the contract; it is restated in the library's header.
 *   - H v   : D(x) = fma(K/4, S_z(x), (J/4) * S_all(x)) with the integer sums
 *             S_all = sum over all bonds of s_b(x), S_z = the same over z bonds,
 *             s_b = +1 for parallel spins and -1 otherwise; acc = D(x) * v[x];
 *             then for every bond b in list order acc = fma(amp_b(x), v[x^m_b], acc),
 *             real and imaginary parts separately.
 *   - dots  : the double nearest to the exact sum (double-double accumulation,
 *             exact products through fma); any summation order gives the same
 *             double except when the exact sum lies within ~2^-100 (relative
 *             to the sum of |terms|) of a rounding boundary.
 *   - every other update is written with explicit fma() where one is meant;
 *     the file is compiled with -ffp-contract=off so nothing else fuses.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DIM(n) ((int64_t)1 << (n))
/* threads only pay off on large vectors; results do not depend on the thread count */
#define PAR_MIN 32768

/* ---------------------------------------------------------------------- */
/* correctly rounded (with overwhelming probability) sums of exact products */

static inline void two_sum(double a, double b, double *s, double *e)
{
    double t = a + b;
    double bb = t - a;
    *e = (a - (t - bb)) + (b - bb);
    *s = t;
}

static inline void fast_two_sum(double a, double b, double *s, double *e)
{
    double t = a + b;
    *e = b - (t - a);
    *s = t;
}

/* (hi, lo) += x */
static inline void dd_add_d(double *hi, double *lo, double x)
{
    double s, e;
    two_sum(*hi, x, &s, &e);
    e = e + *lo;
    fast_two_sum(s, e, hi, lo);
}

/* (hi, lo) += (bh, bl) */
static inline void dd_add_dd(double *hi, double *lo, double bh, double bl)
{
    double s, e, t, f;
    two_sum(*hi, bh, &s, &e);
    two_sum(*lo, bl, &t, &f);
    e = e + t;
    fast_two_sum(s, e, &s, &e);
    e = e + f;
    fast_two_sum(s, e, hi, lo);
}

#define CHUNK 4096

/* Re <a|b> = sum_x (a_re b_re + a_im b_im), rounded once. */
double orc_dot_re(int64_t dim, const double *a, const double *b)
{
    int64_t nch = (dim + CHUNK - 1) / CHUNK;
    int PAR = dim >= PAR_MIN;
    double *part = (double *)malloc(sizeof(double) * 2 * (size_t)nch);
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t c = 0; c < nch; ++c) {
        double hi = 0.0, lo = 0.0, err = 0.0;
        int64_t x1 = (c + 1) * CHUNK < dim ? (c + 1) * CHUNK : dim;
        for (int64_t x = c * CHUNK; x < x1; ++x) {
            double p = a[2 * x] * b[2 * x];
            err = err + fma(a[2 * x], b[2 * x], -p);
            dd_add_d(&hi, &lo, p);
            double q = a[2 * x + 1] * b[2 * x + 1];
            err = err + fma(a[2 * x + 1], b[2 * x + 1], -q);
            dd_add_d(&hi, &lo, q);
        }
        dd_add_d(&hi, &lo, err);
        part[2 * c] = hi;
        part[2 * c + 1] = lo;
    }
    double hi = 0.0, lo = 0.0;
    for (int64_t c = 0; c < nch; ++c)
        dd_add_dd(&hi, &lo, part[2 * c], part[2 * c + 1]);
    free(part);
    return hi + lo;
}

/* ---------------------------------------------------------------------- */
/* Kitaev-Heisenberg Hamiltonian, Sec. V.A: H = sum_b [J S_i.S_j + K S_i^g S_j^g].
 * Diagonal: J S^z_i S^z_j on every bond plus K S^z_i S^z_j on z bonds, i.e.
 * (J/4) S_all(x) + (K/4) S_z(x).  Off-diagonal, per bond b = (i, j): the two-spin
 * flip x -> x ^ (2^i | 2^j) has amplitude ap_b for a parallel pair and aa_b for
 * an antiparallel pair (coefficients prepared by hamiltonian.py). */

static inline double diag_of(int64_t x, int nb, const int *bi, const int *bj, const int *isz,
                             double jq, double kq)
{
    int s_all = 0, s_z = 0;
    for (int b = 0; b < nb; ++b) {
        int s = (((x >> bi[b]) ^ (x >> bj[b])) & 1) ? -1 : 1;
        s_all += s;
        if (isz[b])
            s_z += s;
    }
    return fma(kq, (double)s_z, jq * (double)s_all);
}

static inline void hv_elem(int64_t x, int nb, const int *bi, const int *bj, const int *isz,
                           double jq, double kq, const double *ap, const double *aa,
                           const double *v, double *ore, double *oim)
{
    double D = diag_of(x, nb, bi, bj, isz, jq, kq);
    double re = D * v[2 * x];
    double im = D * v[2 * x + 1];
    for (int b = 0; b < nb; ++b) {
        int par = (((x >> bi[b]) ^ (x >> bj[b])) & 1) == 0;
        double amp = par ? ap[b] : aa[b];
        int64_t y = x ^ (((int64_t)1 << bi[b]) | ((int64_t)1 << bj[b]));
        re = fma(amp, v[2 * y], re);
        im = fma(amp, v[2 * y + 1], im);
    }
    *ore = re;
    *oim = im;
}

/* w = H v */
void orc_hv(int n_sites, int nb, const int *bi, const int *bj, const int *isz,
            double jq, double kq, const double *ap, const double *aa, const double *v, double *w)
{
    int64_t dim = DIM(n_sites);
    int PAR = dim >= PAR_MIN;
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t x = 0; x < dim; ++x)
        hv_elem(x, nb, bi, bj, isz, jq, kq, ap, aa, v, &w[2 * x], &w[2 * x + 1]);
}

/* H v at selected basis indices only (for spot checks at large N) */
void orc_hv_at(int n_sites, int nb, const int *bi, const int *bj, const int *isz,
               double jq, double kq, const double *ap, const double *aa, const double *v,
               int64_t n_idx, const int64_t *idx, double *out)
{
    (void)n_sites;
    int PAR = n_idx >= 1024;
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t k = 0; k < n_idx; ++k)
        hv_elem(idx[k], nb, bi, bj, isz, jq, kq, ap, aa, v, &out[2 * k], &out[2 * k + 1]);
}

/* ---------------------------------------------------------------------- */
/* Lanczos recurrence (the Krylov basis behind every shifted solve, Sec. II.B),
 * written with unnormalised residual vectors w_k (v_{k+1} = w_k / beta_{k+1} is
 * never formed; its scale is carried as inv_{k+1} = 1/beta_{k+1}):
 *   w_{-1} = start, inv_0 = 1/||start||, beta_0 = 0
 *   u     = (H w_{k-1}) * inv_k + c1 w_{k-2},   c1 = (-beta_k) * inv_{k-1}
 *   alpha_k = inv_k * Re<w_{k-1}|u>              (= Re<v_k|u>)
 *   w_k   = u + c2 w_{k-1},                      c2 = -(alpha_k * inv_k)
 *   beta_{k+1} = ||w_k||, inv_{k+1} = 1/beta_{k+1}
 * per element: t = hv * inv_k; u = fma(c1, w_{k-2}, t) (u = t at k = 0);
 * w_k = fma(c2, w_{k-1}, u).  alpha[k] = alpha_k, beta[k] = beta_{k+1}.
 * If W is not NULL, w_{k-1} is stored in W[k] (W[0] = start).  *norm receives
 * ||start||.  Returns the number of completed steps: fewer than n when
 * beta_{k+1} <= tol (invariant subspace). */
/* The Lanczos twin below, with an optional accumulation of the filtered states:
 * with Phi != NULL each residual vector w_k, as it is formed, is added into nm
 * output vectors, Phi_m += d_{m,k} w_k (D: [nm][n] complex, d_{m,k} = c_{m,k} inv_k),
 * with the per-element operations of orc_combine in k order.  Pass 2 of the filter
 * (Sec. III.B) this way regenerates the vectors instead of storing them. */
static int lanczos_core(int n_sites, int nb, const int *bi, const int *bj, const int *isz, double jq, double kq,
                        const double *ap, const double *aa, const double *start, int n, double tol, double *alpha,
                        double *beta, double *W, double *norm, int nm, const double *D, double *Phi);

int orc_lanczos(int n_sites, int nb, const int *bi, const int *bj, const int *isz,
                double jq, double kq, const double *ap, const double *aa, const double *start, int n,
                double tol, double *alpha, double *beta, double *W, double *norm)
{
    return lanczos_core(n_sites, nb, bi, bj, isz, jq, kq, ap, aa, start, n, tol, alpha, beta, W, norm, 0, NULL,
                        NULL);
}

/* Phi [nm][2 dim] = sum_k d_{m,k} w_k over the n steps of the twin from start, without
 * storing the w_k; alpha, beta as orc_lanczos.  Returns the steps taken. */
int orc_lanczos_combine(int n_sites, int nb, const int *bi, const int *bj, const int *isz, double jq, double kq,
                        const double *ap, const double *aa, const double *start, int n, double tol, double *alpha,
                        double *beta, double *norm, int nm, const double *D, double *Phi)
{
    memset(Phi, 0, sizeof(double) * 2 * (size_t)DIM(n_sites) * (size_t)nm);
    return lanczos_core(n_sites, nb, bi, bj, isz, jq, kq, ap, aa, start, n, tol, alpha, beta, NULL, norm, nm, D,
                        Phi);
}

static int lanczos_core(int n_sites, int nb, const int *bi, const int *bj, const int *isz, double jq, double kq,
                        const double *ap, const double *aa, const double *start, int n, double tol, double *alpha,
                        double *beta, double *W, double *norm, int nm, const double *D, double *Phi)
{
    int64_t dim = DIM(n_sites);
    size_t bytes = sizeof(double) * 2 * (size_t)dim;
    double *wc = (double *)malloc(bytes);
    double *wp = (double *)calloc(2 * (size_t)dim, sizeof(double));
    double *u = (double *)malloc(bytes);
    double *hv = (double *)malloc(bytes);
    memcpy(wc, start, bytes);
    int PAR = dim >= PAR_MIN;
    double nrm = sqrt(orc_dot_re(dim, wc, wc));
    *norm = nrm;
    double inv = 1.0 / nrm, inv_prev = 0.0, b = 0.0;
    int k;
    for (k = 0; k < n; ++k) {
        if (W)
            memcpy(W + (size_t)k * 2 * (size_t)dim, wc, bytes);
        if (Phi) {
#pragma omp parallel for schedule(static) if (PAR)
            for (int64_t x = 0; x < dim; ++x) {
                const double vr = wc[2 * x], vi = wc[2 * x + 1];
                for (int m = 0; m < nm; ++m) {
                    const double cr = D[2 * ((size_t)m * n + k)], ci = D[2 * ((size_t)m * n + k) + 1];
                    double *p = Phi + (size_t)m * 2 * dim + 2 * x;
                    double re = p[0], im = p[1];
                    re = fma(cr, vr, re);
                    re = fma(-ci, vi, re);
                    im = fma(cr, vi, im);
                    im = fma(ci, vr, im);
                    p[0] = re;
                    p[1] = im;
                }
            }
        }
        orc_hv(n_sites, nb, bi, bj, isz, jq, kq, ap, aa, wc, hv);
        double c1 = (-b) * inv_prev;
#pragma omp parallel for schedule(static) if (PAR)
        for (int64_t x = 0; x < 2 * dim; ++x) {
            double t = hv[x] * inv;
            u[x] = k == 0 ? t : fma(c1, wp[x], t);
        }
        double a = inv * orc_dot_re(dim, wc, u);
        double c2 = -(a * inv);
#pragma omp parallel for schedule(static) if (PAR)
        for (int64_t x = 0; x < 2 * dim; ++x)
            u[x] = fma(c2, wc[x], u[x]); /* u now holds w_k */
        double bn = sqrt(orc_dot_re(dim, u, u));
        alpha[k] = a;
        beta[k] = bn;
        if (bn <= tol) {
            ++k;
            break;
        }
        double *t = wp;
        wp = wc;
        wc = u;
        u = t;
        inv_prev = inv;
        inv = 1.0 / bn;
        b = bn;
    }
    free(wc);
    free(wp);
    free(u);
    free(hv);
    return k;
}

/* Phi_m = sum_k d_{m,k} W[k], accumulated in k order (Eq. filtered in the
 * Krylov basis, with d_{m,k} = c_{m,k} inv_k folding the scale of the stored
 * unnormalised vectors).  W: [nk][2 dim]; C: [nm][nk] complex; Phi: [nm][2 dim]. */
void orc_combine(int n_sites, int nk, int nm, const double *V, const double *C, double *Phi)
{
    int64_t dim = DIM(n_sites);
    int PAR = dim >= 1024;
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t x = 0; x < dim; ++x) {
        for (int m = 0; m < nm; ++m) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < nk; ++k) {
                double cr = C[2 * ((size_t)m * nk + k)];
                double ci = C[2 * ((size_t)m * nk + k) + 1];
                double vr = V[(size_t)k * 2 * dim + 2 * x];
                double vi = V[(size_t)k * 2 * dim + 2 * x + 1];
                re = fma(cr, vr, re);
                re = fma(-ci, vi, re);
                im = fma(cr, vi, im);
                im = fma(ci, vr, im);
            }
            Phi[(size_t)m * 2 * dim + 2 * x] = re;
            Phi[(size_t)m * 2 * dim + 2 * x + 1] = im;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* chi = S^alpha_{+Q} phi, Sec. V: S^alpha_{+Q} = N^{-1/2} sum_l e^{iQ.R_l} S^alpha_l.
 * h[l] = e^{iQ.R_l} * (1/2) N^{-1/2} (complex, prepared by spin.py).
 * alpha: 0 = x, 1 = y, 2 = z. */
void orc_apply_sq(int n_sites, int alpha, const double *h, const double *v, double *w)
{
    int64_t dim = DIM(n_sites);
    int PAR = dim >= PAR_MIN;
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t x = 0; x < dim; ++x) {
        double re = 0.0, im = 0.0;
        if (alpha == 2) {
            double cr = 0.0, ci = 0.0;
            for (int l = 0; l < n_sites; ++l) {
                if ((x >> l) & 1) { /* spin down: S^z = -1/2 */
                    cr = cr - h[2 * l];
                    ci = ci - h[2 * l + 1];
                } else {
                    cr = cr + h[2 * l];
                    ci = ci + h[2 * l + 1];
                }
            }
            double pr = v[2 * x], pi = v[2 * x + 1];
            re = cr * pr - ci * pi;
            im = cr * pi + ci * pr;
        } else {
            for (int l = 0; l < n_sites; ++l) {
                int64_t y = x ^ ((int64_t)1 << l);
                double cr = h[2 * l], ci = h[2 * l + 1];
                if (alpha == 1) {
                    /* <down|S^y|up> = +i/2 (x has bit l set), <up|S^y|down> = -i/2 */
                    if ((x >> l) & 1) {
                        double t = cr;
                        cr = -ci;
                        ci = t;
                    } else {
                        double t = cr;
                        cr = ci;
                        ci = -t;
                    }
                }
                double pr = v[2 * y], pi = v[2 * y + 1];
                double tr = cr * pr - ci * pi;
                double ti = cr * pi + ci * pr;
                re = re + tr;
                im = im + ti;
            }
        }
        w[2 * x] = re;
        w[2 * x + 1] = im;
    }
}

/* ---------------------------------------------------------------------- */
/* One Taylor term of the imaginary-time series (Appendix A):
 *   t_new = a t + b (H t)   [a = s*l, b = -s/N for the factor s (l - H/N)]
 *   acc  += t_new
 * per element: tn = fma(a, t, b * (Ht)); acc = acc + tn. */
void orc_taylor_term(int n_sites, int nb, const int *bi, const int *bj, const int *isz,
                     double jq, double kq, const double *ap, const double *aa, const double *t, double *tn,
                     double *acc, double a, double b)
{
    int64_t dim = DIM(n_sites);
    int PAR = dim >= PAR_MIN;
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t x = 0; x < dim; ++x) {
        double ur, ui;
        hv_elem(x, nb, bi, bj, isz, jq, kq, ap, aa, t, &ur, &ui);
        double nr = fma(a, t[2 * x], b * ur);
        double ni = fma(a, t[2 * x + 1], b * ui);
        tn[2 * x] = nr;
        tn[2 * x + 1] = ni;
        acc[2 * x] = acc[2 * x] + nr;
        acc[2 * x + 1] = acc[2 * x + 1] + ni;
    }
}

/* v = v * s */
void orc_scale(int64_t n_doubles, double *v, double s)
{
    int PAR = n_doubles >= 2 * PAR_MIN;
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t x = 0; x < n_doubles; ++x)
        v[x] = v[x] * s;
}

/* ---------------------------------------------------------------------- */
/* Random start vector (Sec. II.A): i.i.d. complex Gaussian amplitudes, which
 * after normalisation are uniform on the unit sphere.  Counter-form SplitMix64
 * (Steele, Lea, Flood 2014): the k-th output (k >= 1) of a generator seeded
 * with s is mix(s + k*GOLDEN).  key = output (sample+1) of the seed's stream;
 * element x draws outputs 2x+1 and 2x+2 of the key's stream; Box-Muller. */
#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The k-th output (k >= 1) of the SplitMix64 generator seeded with s. */
uint64_t orc_splitmix64(uint64_t s, uint64_t k) { return mix64(s + GOLDEN * k); }

void orc_gaussian(uint64_t seed, uint64_t sample, int n_sites, double *g)
{
    int64_t dim = DIM(n_sites);
    uint64_t key = mix64(seed + GOLDEN * (sample + 1));
    int PAR = dim >= PAR_MIN;
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t x = 0; x < dim; ++x) {
        uint64_t u1 = mix64(key + GOLDEN * (uint64_t)(2 * x + 1));
        uint64_t u2 = mix64(key + GOLDEN * (uint64_t)(2 * x + 2));
        double d1 = (double)((u1 >> 11) + 1) * 0x1.0p-53; /* (0, 1] */
        double d2 = (double)(u2 >> 11) * 0x1.0p-53;       /* [0, 1) */
        double r = sqrt(-2.0 * log(d1));
        double th = 6.283185307179586 * d2;
        g[2 * x] = r * cos(th);
        g[2 * x + 1] = r * sin(th);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Complex-symmetric (bilinear) Lanczos: the basis of shifted COCG (Sec. II.B with
 * the shadow vector conj(rho); see cocg.py).  q_j^T q_k = delta_jk with the bilinear
 * form x^T y = sum_x x_i y_i (no conjugation).  Unnormalised residuals w_k =
 * b_{k+1} q_{k+1} with the complex scale inv_k = 1/b_k carried as a scalar:
 *   w_{-1} = start, delta0 = csqrt(start^T start), inv_0 = 1/delta0, b_0 = 0
 *   u     = (H w_{k-1}) inv_k + c1 w_{k-2},   c1 = -(b_k inv_{k-1})
 *   a_k   = inv_k (w_{k-1}^T u)
 *   w_k   = u + c2 w_{k-1},                   c2 = -(a_k inv_k)
 *   b_{k+1} = csqrt(w_k^T w_k), inv_{k+1} = 1/b_{k+1}
 *   c_k   = <lam|q_k> = inv_k <lam|w_{k-1}>,  hn_k = ||q_k||^2 = |inv_k|^2 ||w_{k-1}||^2
 * Complex products are (fma(ar, br, -(ai bi)), fma(ar, bi, ai br)); per element
 *   u = (fma(c1r, wpr, fma(-c1i, wpi, tr)), fma(c1r, wpi, fma(c1i, wpr, ti))), t = (Hw) inv,
 *   w = (fma(c2r, wcr, fma(-c2i, wci, ur)), fma(c2r, wci, fma(c2i, wcr, ui)));
 * the sums are the doubles nearest the exact sums of exact products (the imaginary part
 * of w^T w is twice the rounded sum of w_r w_i); csqrt(x + iy) of a nonzero number is
 * (t, y/(2t)) with t = sqrt((m + x)/2) when x >= 0, else (|y|/(2t), copysign(t, y)) with
 * t = sqrt((m - x)/2), m = sqrt(x x + y y); 1/(x + iy) by Smith's algorithm (cinv_c).
 * a[2k], b[2k] (complex) get a_k and b_{k+1}; c[2k] for k = 0..steps; hn[k] likewise;
 * d0 = delta0.  The run stops after step k when ||w_k|| <= tol (invariant subspace) or
 * |w_k^T w_k| <= 1e-24 ||w_k||^2 (the bilinear form vanishes).  Returns the number of
 * completed steps. */
static void dd_sum_prod(double *hi, double *lo, double *err, double a, double b)
{
    double p = a * b;
    *err = *err + fma(a, b, -p);
    dd_add_d(hi, lo, p);
}

/* exact-sum reductions of one pass: out[0..2*nsum) */
static void bl_dots(int64_t dim, int nsum, const double *w, const double *u, const double *lam, double *out)
{
    int64_t nch = (dim + CHUNK - 1) / CHUNK;
    int PAR = dim >= PAR_MIN;
    double *part = (double *)malloc(sizeof(double) * 2 * 4 * (size_t)nch);
#pragma omp parallel for schedule(static) if (PAR)
    for (int64_t c = 0; c < nch; ++c) {
        double hi[4] = {0, 0, 0, 0}, lo[4] = {0, 0, 0, 0}, er[4] = {0, 0, 0, 0};
        int64_t x1 = (c + 1) * CHUNK < dim ? (c + 1) * CHUNK : dim;
        for (int64_t x = c * CHUNK; x < x1; ++x) {
            double wr = w[2 * x], wi = w[2 * x + 1];
            if (nsum == 2) { /* w^T u */
                double ur = u[2 * x], ui = u[2 * x + 1];
                dd_sum_prod(&hi[0], &lo[0], &er[0], wr, ur);
                dd_sum_prod(&hi[0], &lo[0], &er[0], -wi, ui);
                dd_sum_prod(&hi[1], &lo[1], &er[1], wr, ui);
                dd_sum_prod(&hi[1], &lo[1], &er[1], wi, ur);
            } else { /* w^T w, sum w_r w_i, <lam|w>, ||w||^2 */
                double lr = lam[2 * x], li = lam[2 * x + 1];
                dd_sum_prod(&hi[0], &lo[0], &er[0], wr, wr);
                dd_sum_prod(&hi[0], &lo[0], &er[0], -wi, wi);
                dd_sum_prod(&hi[1], &lo[1], &er[1], wr, wi);
                dd_sum_prod(&hi[2], &lo[2], &er[2], lr, wr);
                dd_sum_prod(&hi[2], &lo[2], &er[2], li, wi);
                dd_sum_prod(&hi[3], &lo[3], &er[3], lr, wi);
                dd_sum_prod(&hi[3], &lo[3], &er[3], -li, wr);
            }
        }
        for (int j = 0; j < 4; ++j) {
            dd_add_d(&hi[j], &lo[j], er[j]);
            part[8 * c + 2 * j] = hi[j];
            part[8 * c + 2 * j + 1] = lo[j];
        }
    }
    for (int j = 0; j < 4; ++j) {
        double hi = 0.0, lo = 0.0;
        for (int64_t c = 0; c < nch; ++c)
            dd_add_dd(&hi, &lo, part[8 * c + 2 * j], part[8 * c + 2 * j + 1]);
        out[j] = hi + lo;
    }
    free(part);
}

static void csqrt_c(double x, double y, double *sr, double *si)
{
    double m = sqrt(x * x + y * y);
    if (x >= 0.0) {
        double t = sqrt((m + x) / 2.0);
        *sr = t;
        *si = y / (2.0 * t);
    } else {
        double t = sqrt((m - x) / 2.0);
        *sr = fabs(y) / (2.0 * t);
        *si = copysign(t, y);
    }
}

/* 1/(x + iy) by Smith's algorithm (R. L. Smith, CACM 5, 435, 1962): no squares, so no
 * overflow for large or tiny numbers, and exactly 1/x for a real number */
static void cinv_c(double x, double y, double *r, double *i)
{
    if (fabs(x) >= fabs(y)) {
        double t = y / x;
        double d = x + y * t;
        *r = 1.0 / d;
        *i = -t / d;
    } else {
        double t = x / y;
        double d = x * t + y;
        *r = t / d;
        *i = -1.0 / d;
    }
}

static void cmul_c(double ar, double ai, double br, double bi, double *r, double *i)
{
    *r = fma(ar, br, -(ai * bi));
    *i = fma(ar, bi, ai * br);
}

int orc_lanczos_bilinear(int n_sites, int nb, const int *bi, const int *bj, const int *isz, double jq,
                         double kq, const double *ap, const double *aa, const double *start, const double *lam,
                         int n, double tol, double *a, double *b, double *c, double *hn, double *d0)
{
    int64_t dim = DIM(n_sites);
    size_t bytes = sizeof(double) * 2 * (size_t)dim;
    double *wc = (double *)malloc(bytes);
    double *wp = (double *)calloc(2 * (size_t)dim, sizeof(double));
    double *u = (double *)malloc(bytes);
    double *hv = (double *)malloc(bytes);
    int PAR = dim >= PAR_MIN;
    memcpy(wc, start, bytes);
    double s[4];
    bl_dots(dim, 4, wc, NULL, lam, s);
    double bbr = s[0], bbi = 2.0 * s[1];
    double dr, di;
    csqrt_c(bbr, bbi, &dr, &di);
    d0[0] = dr;
    d0[1] = di;
    double invr, invi, ipr = 0.0, ipi = 0.0, bkr = 0.0, bki = 0.0;
    cinv_c(dr, di, &invr, &invi);
    cmul_c(invr, invi, s[2], s[3], &c[0], &c[1]);
    {
        double nw = 0.0, lo = 0.0, er = 0.0;
        for (int64_t x = 0; x < 2 * dim; ++x)
            dd_sum_prod(&nw, &lo, &er, wc[x], wc[x]);
        dd_add_d(&nw, &lo, er);
        hn[0] = (invr * invr + invi * invi) * (nw + lo);
    }
    int k;
    for (k = 0; k < n; ++k) {
        orc_hv(n_sites, nb, bi, bj, isz, jq, kq, ap, aa, wc, hv);
        double c1r, c1i;
        cmul_c(bkr, bki, ipr, ipi, &c1r, &c1i);
        c1r = -c1r;
        c1i = -c1i;
#pragma omp parallel for schedule(static) if (PAR)
        for (int64_t x = 0; x < dim; ++x) {
            double tr, ti;
            cmul_c(hv[2 * x], hv[2 * x + 1], invr, invi, &tr, &ti);
            if (k == 0) {
                u[2 * x] = tr;
                u[2 * x + 1] = ti;
            } else {
                double pr = wp[2 * x], pi = wp[2 * x + 1];
                u[2 * x] = fma(c1r, pr, fma(-c1i, pi, tr));
                u[2 * x + 1] = fma(c1r, pi, fma(c1i, pr, ti));
            }
        }
        double t[4];
        bl_dots(dim, 2, wc, u, NULL, t);
        double akr, aki;
        cmul_c(invr, invi, t[0], t[1], &akr, &aki);
        double c2r, c2i;
        cmul_c(akr, aki, invr, invi, &c2r, &c2i);
        c2r = -c2r;
        c2i = -c2i;
#pragma omp parallel for schedule(static) if (PAR)
        for (int64_t x = 0; x < dim; ++x) {
            double wr = wc[2 * x], wi = wc[2 * x + 1];
            double ur = u[2 * x], ui = u[2 * x + 1];
            u[2 * x] = fma(c2r, wr, fma(-c2i, wi, ur));
            u[2 * x + 1] = fma(c2r, wi, fma(c2i, wr, ui));
        }
        bl_dots(dim, 4, u, NULL, lam, s);
        double wwr = s[0], wwi = 2.0 * s[1];
        double nw = 0.0, lo = 0.0, er = 0.0;
        for (int64_t x = 0; x < 2 * dim; ++x)
            dd_sum_prod(&nw, &lo, &er, u[x], u[x]);
        dd_add_d(&nw, &lo, er);
        double nrm2 = nw + lo;
        double bnr, bni;
        csqrt_c(wwr, wwi, &bnr, &bni);
        a[2 * k] = akr;
        a[2 * k + 1] = aki;
        b[2 * k] = bnr;
        b[2 * k + 1] = bni;
        double ninvr, ninvi;
        cinv_c(bnr, bni, &ninvr, &ninvi);
        cmul_c(ninvr, ninvi, s[2], s[3], &c[2 * (k + 1)], &c[2 * (k + 1) + 1]);
        hn[k + 1] = (ninvr * ninvr + ninvi * ninvi) * nrm2;
        if (sqrt(nrm2) <= tol || sqrt(wwr * wwr + wwi * wwi) <= 1e-24 * nrm2) {
            ++k;
            break;
        }
        double *tt = wp;
        wp = wc;
        wc = u;
        u = tt;
        ipr = invr;
        ipi = invi;
        invr = ninvr;
        invi = ninvi;
        bkr = bnr;
        bki = bni;
    }
    free(wc);
    free(wp);
    free(u);
    free(hv);
    return k;
}
