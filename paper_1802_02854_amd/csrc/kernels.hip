// HIP kernels (gfx950) of the FTKw path.  Compiled with -ffp-contract=off:
// every fused multiply-add below is an explicit fma(), everything else is a
// separately rounded IEEE double operation, as the library's arithmetic
// contract requires (see ftkw.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "kernels.h"

namespace ftk {

HvParams make_hv_params(const BondTable &t)
{
    HvParams P;
    std::memset(&P, 0, sizeof(P));
    P.n_sites = t.n_sites;
    P.n_bonds = t.n_bonds;
    for (int b = 0; b < t.n_bonds; ++b) {
        P.mask[b] = (1u << t.bi[b]) | (1u << t.bj[b]);
        P.bi[b] = (uint8_t)t.bi[b];
        P.bj[b] = (uint8_t)t.bj[b];
        P.isz[b] = t.gamma[b] == 2 ? 1 : 0;
        P.ap[b] = t.ap[b];
        P.aa[b] = t.aa[b];
    }
    P.jq = t.jq;
    P.kq = t.kq;
    return P;
}

int vec_grid(uint32_t dim)
{
    uint32_t g = (dim + kBlock - 1) / kBlock;
    return (int)(g < (uint32_t)kMaxGrid ? g : (uint32_t)kMaxGrid);
}

// ---------------------------------------------------------------------------
// Exact-sum helpers: a sum of exact products carried as an unevaluated pair
// (hi, lo), rounded once at the end.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    double t = a + b;
    double bb = t - a;
    e = (a - (t - bb)) + (b - bb);
    s = t;
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e)
{
    double t = a + b;
    e = b - (t - a);
    s = t;
}

__device__ __forceinline__ void dd_add(double &hi, double &lo, double x)
{
    double s, e;
    two_sum(hi, x, s, e);
    e = e + lo;
    fast_two_sum(s, e, hi, lo);
}

__device__ __forceinline__ void dd_add_dd(double &hi, double &lo, double bh, double bl)
{
    double s, e, t, f;
    two_sum(hi, bh, s, e);
    two_sum(lo, bl, t, f);
    e = e + t;
    fast_two_sum(s, e, s, e);
    e = e + f;
    fast_two_sum(s, e, hi, lo);
}

// adds a*b exactly: the rounded product goes to (hi, lo), its error to err
__device__ __forceinline__ void acc_prod(double &hi, double &lo, double &err, double a, double b)
{
    double p = a * b;
    err = err + fma(a, b, -p);
    dd_add(hi, lo, p);
}

// Block-wide reduction of (hi, lo) pairs in a fixed order; result in thread 0.
__device__ __forceinline__ void block_reduce_dd(double &hi, double &lo)
{
    __shared__ double sh[kBlock / 64][2];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double oh = __shfl_xor(hi, off, 64);
        double ol = __shfl_xor(lo, off, 64);
        dd_add_dd(hi, lo, oh, ol);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sh[wave][0] = hi;
        sh[wave][1] = lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        hi = sh[0][0];
        lo = sh[0][1];
        for (int w = 1; w < kBlock / 64; ++w) dd_add_dd(hi, lo, sh[w][0], sh[w][1]);
    }
}

// Sum of nparts (hi, lo) partials, rounded; valid in thread 0.
__device__ __forceinline__ double reduce_partials(const double *partials, int nparts)
{
    double hi = 0.0, lo = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) dd_add_dd(hi, lo, partials[2 * i], partials[2 * i + 1]);
    block_reduce_dd(hi, lo);
    return hi + lo;
}

__device__ __forceinline__ void write_partial(double *partials, double hi, double lo, double err)
{
    dd_add(hi, lo, err);
    block_reduce_dd(hi, lo);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = hi;
        partials[2 * blockIdx.x + 1] = lo;
    }
}

// ---------------------------------------------------------------------------
// (H v)[x] by the contract: D from integer bond-parity sums, then one fma per
// bond in list order.  With SCALED, every v entry is first multiplied by `scale`
// (v_k = w_{k-1} * inv_k computed where it is read).
template <bool SCALED>
__device__ __forceinline__ void hv_at(const HvParams &P, uint32_t x, const double2 *__restrict__ v,
                                      double scale, double &re, double &im, double2 &vx)
{
    int s_all = 0, s_z = 0;
    for (int b = 0; b < P.n_bonds; ++b) {
        const int s = (((x >> P.bi[b]) ^ (x >> P.bj[b])) & 1u) ? -1 : 1;
        s_all += s;
        if (P.isz[b]) s_z += s;
    }
    const double D = fma(P.kq, (double)s_z, P.jq * (double)s_all);
    vx = v[x];
    if (SCALED) {
        vx.x = vx.x * scale;
        vx.y = vx.y * scale;
    }
    re = D * vx.x;
    im = D * vx.y;
    for (int b = 0; b < P.n_bonds; ++b) {
        const bool anti = ((x >> P.bi[b]) ^ (x >> P.bj[b])) & 1u;
        const double amp = anti ? P.aa[b] : P.ap[b];
        double2 vy = v[x ^ P.mask[b]];
        if (SCALED) {
            vy.x = vy.x * scale;
            vy.y = vy.y * scale;
        }
        re = fma(amp, vy.x, re);
        im = fma(amp, vy.y, im);
    }
}

__global__ void __launch_bounds__(kBlock) k_apply_h(HvParams P, const double2 *__restrict__ v,
                                                    double2 *__restrict__ w)
{
    const uint32_t dim = 1u << P.n_sites;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        double re, im;
        double2 vx;
        hv_at<false>(P, x, v, 1.0, re, im, vx);
        w[x] = make_double2(re, im);
    }
}

void launch_apply_h(const HvParams &P, const double *v, double *w, hipStream_t s)
{
    const uint32_t dim = 1u << P.n_sites;
    hipLaunchKernelGGL(k_apply_h, dim3(vec_grid(dim)), dim3(kBlock), 0, s, P, (const double2 *)v, (double2 *)w);
}

// ---------------------------------------------------------------------------
// Lanczos step (Sec. II.B basis): u = H v_k - beta_k v_{k-1}; alpha_k = Re<v_k|u>;
// w_k = u - alpha_k v_k; beta_{k+1} = ||w_k||; v_{k+1} = w_k / beta_{k+1} (as a
// multiplication by inv = 1/beta_{k+1}, applied where v_{k+1} is read).
__global__ void __launch_bounds__(kBlock) k_lanczos_a(HvParams P, const double2 *__restrict__ Wcur,
                                                      const double2 *Wprev, double2 *U,
                                                      double2 *__restrict__ vout, SeqState *st,
                                                      double *partials, int first)
{
    if (st->done) return;
    const uint32_t dim = 1u << P.n_sites;
    const double inv = st->inv_cur, invp = st->inv_prev, mb = -st->beta_cur;
    double hi = 0.0, lo = 0.0, err = 0.0;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        double re, im;
        double2 vx;
        hv_at<true>(P, x, Wcur, inv, re, im, vx);
        if (!first) {
            const double2 wp = Wprev[x];
            re = fma(mb, wp.x * invp, re);
            im = fma(mb, wp.y * invp, im);
        }
        U[x] = make_double2(re, im);
        if (vout) vout[x] = vx;
        acc_prod(hi, lo, err, vx.x, re);
        acc_prod(hi, lo, err, vx.y, im);
    }
    write_partial(partials, hi, lo, err);
}

__global__ void __launch_bounds__(kBlock) k_lanczos_b(uint32_t dim, const double2 *__restrict__ Wcur,
                                                      double2 *__restrict__ U, SeqState *st,
                                                      double *partials)
{
    if (st->done) return;
    const double inv = st->inv_cur, ma = -st->alpha_cur;
    double hi = 0.0, lo = 0.0, err = 0.0;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 wc = Wcur[x];
        const double vr = wc.x * inv, vi = wc.y * inv;
        const double2 u = U[x];
        const double wr = fma(ma, vr, u.x);
        const double wi = fma(ma, vi, u.y);
        U[x] = make_double2(wr, wi);
        acc_prod(hi, lo, err, wr, wr);
        acc_prod(hi, lo, err, wi, wi);
    }
    write_partial(partials, hi, lo, err);
}

__global__ void __launch_bounds__(kBlock) k_finalize_alpha(SeqState *st, const double *partials,
                                                           int nparts, double *alpha_out, int k)
{
    if (st->done) return;
    const double a = reduce_partials(partials, nparts);
    if (threadIdx.x == 0) {
        if (!isfinite(a)) st->numeric_error = 1;
        st->alpha_cur = a;
        alpha_out[k] = a;
    }
}

// Forward LDL^T recurrence of (z - T)^{-1}_{00} per shift z = omega + shift_re + i eta.
__global__ void __launch_bounds__(kBlock) k_finalize_beta(SeqState *st, const double *partials,
                                                          int nparts, double *beta_out, int k,
                                                          double tol, ShiftState *sh,
                                                          const double *omega, int n_omega,
                                                          double eta)
{
    if (st->done) return;
    __shared__ double s_bn;
    __shared__ double s_res[kBlock];
    const double ssum = reduce_partials(partials, nparts);
    if (threadIdx.x == 0) s_bn = sqrt(ssum);
    const double alpha = st->alpha_cur, bk = st->beta_cur, zoff = st->shift_re;
    __syncthreads();
    const double bn = s_bn;
    double rmax = 0.0;
    for (int j = threadIdx.x; j < n_omega; j += blockDim.x) {
        const double zr = omega[j] + zoff, zi = eta;
        ShiftState q = sh[j];
        if (k == 0) {
            q.dr = zr - alpha;
            q.di = zi;
            q.pr = 1.0;
            q.pi = 0.0;
            const double den = q.dr * q.dr + q.di * q.di;
            q.gr = q.dr / den;
            q.gi = -q.di / den;
        } else {
            const double den = q.dr * q.dr + q.di * q.di;
            const double rr = q.dr / den, ri = -q.di / den;  // 1/d_{k-1}
            const double fr = bk * rr, fi = bk * ri;         // beta_k / d_{k-1}
            const double pr = q.pr * fr - q.pi * fi;
            const double pi = q.pr * fi + q.pi * fr;
            const double b2 = bk * bk;
            q.dr = (zr - alpha) - b2 * rr;
            q.di = zi - b2 * ri;
            q.pr = pr;
            q.pi = pi;
            const double p2r = pr * pr - pi * pi, p2i = 2.0 * pr * pi;
            const double dn = q.dr * q.dr + q.di * q.di;
            q.gr = q.gr + (p2r * q.dr + p2i * q.di) / dn;
            q.gi = q.gi + (p2i * q.dr - p2r * q.di) / dn;
        }
        sh[j] = q;
        // residual after k+1 steps: |p_k| beta_{k+1} / |d_k|
        const double r = sqrt((q.pr * q.pr + q.pi * q.pi) / (q.dr * q.dr + q.di * q.di)) * bn;
        rmax = r > rmax ? r : rmax;
    }
    s_res[threadIdx.x] = rmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < blockDim.x; ++i) m = s_res[i] > m ? s_res[i] : m;
        st->max_resid = m * st->norm;
        beta_out[k] = bn;
        st->steps = k + 1;
        if (!isfinite(bn)) st->numeric_error = 1;
        if (!(bn > tol)) {
            st->done = 1;
        } else {
            st->inv_prev = st->inv_cur;
            st->inv_cur = 1.0 / bn;
            st->beta_cur = bn;
        }
    }
}

__global__ void k_finish_green(const SeqState *st, const ShiftState *sh, int n_omega, double2 *g)
{
    const double n2 = st->norm2;
    const bool any = st->steps > 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_omega; j += gridDim.x * blockDim.x) {
        const ShiftState q = sh[j];
        g[j] = any ? make_double2(n2 * q.gr, n2 * q.gi) : make_double2(0.0, 0.0);
    }
}

void launch_lanczos_a(const HvParams &P, const double *Wcur, const double *Wprev, double *U,
                      double *vout, SeqState *st, double *partials, int first_step, hipStream_t s)
{
    const uint32_t dim = 1u << P.n_sites;
    hipLaunchKernelGGL(k_lanczos_a, dim3(vec_grid(dim)), dim3(kBlock), 0, s, P, (const double2 *)Wcur,
                       (const double2 *)Wprev, (double2 *)U, (double2 *)vout, st, partials, first_step);
}

void launch_finalize_alpha(SeqState *st, const double *partials, int nparts, double *alpha_out,
                           int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kBlock), 0, s, st, partials, nparts, alpha_out, k);
}

void launch_lanczos_b(uint32_t dim, const double *Wcur, double *U, SeqState *st,
                      double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_lanczos_b, dim3(vec_grid(dim)), dim3(kBlock), 0, s, dim, (const double2 *)Wcur,
                       (double2 *)U, st, partials);
}

void launch_finalize_beta(SeqState *st, const double *partials, int nparts, double *beta_out,
                          int k, double tol, ShiftState *shifts, const double *omega, int n_omega,
                          double eta, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_beta, dim3(1), dim3(kBlock), 0, s, st, partials, nparts, beta_out, k,
                       tol, shifts, omega, n_omega, eta);
}

void launch_finish_green(const SeqState *st, const ShiftState *shifts, int n_omega, double *g,
                         hipStream_t s)
{
    int grid = (n_omega + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_finish_green, dim3(grid < 1 ? 1 : grid), dim3(kBlock), 0, s, st, shifts, n_omega,
                       (double2 *)g);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_dot(uint32_t dim, const double2 *__restrict__ a,
                                                const double2 *__restrict__ b, double *partials)
{
    double hi = 0.0, lo = 0.0, err = 0.0;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 u = a[x], v = b[x];
        acc_prod(hi, lo, err, u.x, v.x);
        acc_prod(hi, lo, err, u.y, v.y);
    }
    write_partial(partials, hi, lo, err);
}

__global__ void __launch_bounds__(kBlock) k_start_sequence(SeqState *st, const double *partials,
                                                           int nparts, double shift_re)
{
    const double s = reduce_partials(partials, nparts);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(s);
        st->norm2 = s;
        st->norm = nrm;
        st->inv_cur = nrm > 0.0 ? 1.0 / nrm : 0.0;
        st->inv_prev = 0.0;
        st->beta_cur = 0.0;
        st->alpha_cur = 0.0;
        st->shift_re = shift_re;
        st->max_resid = 0.0;
        st->done = nrm > 0.0 ? 0 : 1;
        st->steps = 0;
        st->numeric_error = isfinite(s) ? 0 : 1;
        st->pad = 0;
    }
}

__global__ void __launch_bounds__(kBlock) k_sum_partials(const double *partials, int nparts, double *result)
{
    const double s = reduce_partials(partials, nparts);
    if (threadIdx.x == 0) result[0] = s;
}

void launch_dot(uint32_t dim, const double *a, const double *b, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot, dim3(vec_grid(dim)), dim3(kBlock), 0, s, dim, (const double2 *)a,
                       (const double2 *)b, partials);
}

void launch_start_sequence(SeqState *st, const double *partials, int nparts, double shift_re,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_start_sequence, dim3(1), dim3(kBlock), 0, s, st, partials, nparts, shift_re);
}

void launch_sum_partials(const double *partials, int nparts, double *result, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partials, nparts, result);
}

// ---------------------------------------------------------------------------
// chi = S^alpha_{+Q} phi (Sec. V): x and y flip one spin, z is diagonal.
// <down|S^y|up> = +i/2 and <up|S^y|down> = -i/2 (bit 1 = spin down).
__global__ void __launch_bounds__(kBlock) k_apply_sq(SqParams P, const double2 *__restrict__ phi,
                                                     double2 *__restrict__ chi)
{
    const uint32_t dim = 1u << P.n_sites;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        if (P.alpha == 2) {
            double cr = 0.0, ci = 0.0;
            for (int l = 0; l < P.n_sites; ++l) {
                if ((x >> l) & 1u) {
                    cr = cr - P.h[2 * l];
                    ci = ci - P.h[2 * l + 1];
                } else {
                    cr = cr + P.h[2 * l];
                    ci = ci + P.h[2 * l + 1];
                }
            }
            const double2 p = phi[x];
            re = cr * p.x - ci * p.y;
            im = cr * p.y + ci * p.x;
        } else {
            for (int l = 0; l < P.n_sites; ++l) {
                double cr = P.h[2 * l], ci = P.h[2 * l + 1];
                if (P.alpha == 1) {
                    if ((x >> l) & 1u) {
                        const double t = cr;
                        cr = -ci;
                        ci = t;
                    } else {
                        const double t = cr;
                        cr = ci;
                        ci = -t;
                    }
                }
                const double2 p = phi[x ^ (1u << l)];
                const double tr = cr * p.x - ci * p.y;
                const double ti = cr * p.y + ci * p.x;
                re = re + tr;
                im = im + ti;
            }
        }
        chi[x] = make_double2(re, im);
    }
}

void launch_apply_sq(const SqParams &P, const double *phi, double *chi, hipStream_t s)
{
    const uint32_t dim = 1u << P.n_sites;
    hipLaunchKernelGGL(k_apply_sq, dim3(vec_grid(dim)), dim3(kBlock), 0, s, P, (const double2 *)phi,
                       (double2 *)chi);
}

// ---------------------------------------------------------------------------
// One term of the imaginary-time Taylor series (Appendix A).
__global__ void __launch_bounds__(kBlock) k_taylor_term(HvParams P, const double2 *__restrict__ t,
                                                        double2 *__restrict__ tn,
                                                        double2 *__restrict__ acc, double a, double b)
{
    const uint32_t dim = 1u << P.n_sites;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        double re, im;
        double2 tx;
        hv_at<false>(P, x, t, 1.0, re, im, tx);
        const double nr = fma(a, tx.x, b * re);
        const double ni = fma(a, tx.y, b * im);
        tn[x] = make_double2(nr, ni);
        const double2 c = acc[x];
        acc[x] = make_double2(c.x + nr, c.y + ni);
    }
}

void launch_taylor_term(const HvParams &P, const double *t, double *tn, double *acc, double a,
                        double b, hipStream_t s)
{
    const uint32_t dim = 1u << P.n_sites;
    hipLaunchKernelGGL(k_taylor_term, dim3(vec_grid(dim)), dim3(kBlock), 0, s, P, (const double2 *)t,
                       (double2 *)tn, (double2 *)acc, a, b);
}

__global__ void k_scale(uint32_t dim, double2 *v, double scale)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 a = v[x];
        v[x] = make_double2(a.x * scale, a.y * scale);
    }
}

__global__ void k_copy(uint32_t dim, const double2 *__restrict__ src, double2 *__restrict__ dst)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x)
        dst[x] = src[x];
}

void launch_scale(uint32_t dim, double *v, double scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(vec_grid(dim)), dim3(kBlock), 0, s, dim, (double2 *)v, scale);
}

void launch_copy(uint32_t dim, const double *src, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(vec_grid(dim)), dim3(kBlock), 0, s, dim, (const double2 *)src,
                       (double2 *)dst);
}

// ---------------------------------------------------------------------------
// Random start vectors (Sec. II.A): complex Gaussian amplitudes from the counter
// form of SplitMix64 (Steele, Lea, Flood 2014): output k >= 1 of a generator
// seeded with s is mix(s + k * golden).  Key = output (sample + 1) of the seed's
// stream; element x uses outputs 2x+1 and 2x+2 of the key's stream; Box-Muller.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void k_gaussian(uint32_t dim, uint64_t key, double2 *g)
{
    const uint64_t golden = 0x9E3779B97F4A7C15ULL;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const uint64_t u1 = mix64(key + golden * (2ull * x + 1ull));
        const uint64_t u2 = mix64(key + golden * (2ull * x + 2ull));
        const double d1 = (double)((u1 >> 11) + 1ull) * 0x1.0p-53;
        const double d2 = (double)(u2 >> 11) * 0x1.0p-53;
        const double r = sqrt(-2.0 * log(d1));
        const double th = 6.283185307179586 * d2;
        double sn, cs;
        sincos(th, &sn, &cs);
        g[x] = make_double2(r * cs, r * sn);
    }
}

void launch_gaussian(uint32_t dim, uint64_t seed, uint64_t sample, double *g, hipStream_t s)
{
    const uint64_t golden = 0x9E3779B97F4A7C15ULL;
    uint64_t z = seed + golden * (sample + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    const uint64_t key = z ^ (z >> 31);
    hipLaunchKernelGGL(k_gaussian, dim3(vec_grid(dim)), dim3(kBlock), 0, s, dim, key, (double2 *)g);
}

// ---------------------------------------------------------------------------
// Filter pass 2 (Sec. III.B, Eq. filtered): Phi_m += sum_k c_{m,k} v_k over a
// buffered block of Lanczos vectors, k in increasing order, 8 shells per thread.
constexpr int kShellTile = 8;

__global__ void __launch_bounds__(kBlock) k_accumulate(uint32_t dim, const double2 *__restrict__ V,
                                                       int nk, const double2 *__restrict__ coef,
                                                       int n, int k0, double2 *__restrict__ Phi, int L)
{
    const int m0 = blockIdx.y * kShellTile;
    const int mc = L - m0 < kShellTile ? L - m0 : kShellTile;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        double2 acc[kShellTile];
#pragma unroll
        for (int mm = 0; mm < kShellTile; ++mm)
            if (mm < mc) acc[mm] = Phi[(size_t)(m0 + mm) * dim + x];
        for (int k = 0; k < nk; ++k) {
            const double2 v = V[(size_t)k * dim + x];
#pragma unroll
            for (int mm = 0; mm < kShellTile; ++mm) {
                if (mm < mc) {
                    const double2 c = coef[(size_t)(m0 + mm) * n + k0 + k];
                    double r = acc[mm].x, i = acc[mm].y;
                    r = fma(c.x, v.x, r);
                    r = fma(-c.y, v.y, r);
                    i = fma(c.x, v.y, i);
                    i = fma(c.y, v.x, i);
                    acc[mm] = make_double2(r, i);
                }
            }
        }
#pragma unroll
        for (int mm = 0; mm < kShellTile; ++mm)
            if (mm < mc) Phi[(size_t)(m0 + mm) * dim + x] = acc[mm];
    }
}

void launch_accumulate(uint32_t dim, const double *V, int nk, const double *coef, int n, int k0,
                       double *Phi, int L, hipStream_t s)
{
    dim3 grid(vec_grid(dim), (L + kShellTile - 1) / kShellTile);
    hipLaunchKernelGGL(k_accumulate, grid, dim3(kBlock), 0, s, dim, (const double2 *)V, nk,
                       (const double2 *)coef, n, k0, (double2 *)Phi, L);
}

}  // namespace ftk
