// Shifted COCG with seed switching (the solver option of the spectrum and pair
// calls): device kernels and launchers.  Compiled with -ffp-contract=off like every
// other source: each fused multiply-add is an explicit fma().
#include <hip/hip_runtime.h>

#include <cmath>

#include "cocg.h"
#include "exact_sum.h"

namespace ftk {

// Shifted COCG with seed switching (Sec. II.B with the shadow vector conj(rho);
// the seed switching of Appendix C).  H is real symmetric, so z - H is complex
// symmetric and BiCG with the shadow conj(rho) is COCG.  The vectors are the
// complex-symmetric Lanczos basis q_k (q_j^T q_k = delta_jk, bilinear form), kept as
// unnormalised residuals w_k = b_{k+1} q_{k+1} with the complex scale inv_k = 1/b_k
// carried as a scalar:
//   u   = (H w_{k-1}) inv_k + c1 w_{k-2},  c1 = -(b_k inv_{k-1});  a_k = inv_k (w_{k-1}^T u)
//   w_k = u + c2 w_{k-1},  c2 = -(a_k inv_k);  b_{k+1} = csqrt(w_k^T w_k);  inv_{k+1} = 1/b_{k+1}
//   c_k = <lam|q_k> = inv_k <lam|w_{k-1}>,  hn_k = ||q_k||^2  (lam = chi for a spectrum;
//   for an operator pair the other operator's vector, so g = <lam|x(z)>).
// Every shift z_j runs the shifted COCG scalar recurrence of the seed's CG, whose
// coefficients are the pivots of z_s - T: 1/alpha_k = z_s - a_k - b_k^2 alpha_{k-1},
// beta_k = b_{k+1}^2 alpha_k^2, residual r_k = delta_k q_k with delta_{k+1} =
// alpha_k b_{k+1} delta_k; the seed moves to the unconverged shift with the largest
// residual once its own residual is below seed_tol ||chi||.  A shift other than the
// seed whose residual is at most seed_tol ||chi|| is converged and no longer updated
// (past convergence pi_j only grows, towards overflow once the Krylov space is
// exhausted); the run ends once every shift is converged.

// complex products of the vector updates: (fma(ar, br, -(ai bi)), fma(ar, bi, ai br))
__device__ __forceinline__ void cmul_v(double ar, double ai, double br, double bi, double &r, double &i)
{
    r = fma(ar, br, -(ai * bi));
    i = fma(ar, bi, ai * br);
}
// scalar complex arithmetic of the recurrences: plain products, Smith's division
// (R. L. Smith, CACM 5, 435, 1962)
__device__ __forceinline__ void cmul_s(double ar, double ai, double br, double bi, double &r, double &i)
{
    r = ar * br - ai * bi;
    i = ar * bi + ai * br;
}
__device__ __forceinline__ void cdiv_s(double ar, double ai, double br, double bi, double &r, double &i)
{
    if (fabs(br) >= fabs(bi)) {
        const double t = bi / br;
        const double d = br + bi * t;
        r = (ar + ai * t) / d;
        i = (ai - ar * t) / d;
    } else {
        const double t = br / bi;
        const double d = br * t + bi;
        r = (ar * t + ai) / d;
        i = (ai * t - ar) / d;
    }
}
__device__ __forceinline__ void cinv_s(double x, double y, double &r, double &i)
{
    if (fabs(x) >= fabs(y)) {
        const double t = y / x;
        const double d = x + y * t;
        r = 1.0 / d;
        i = -t / d;
    } else {
        const double t = x / y;
        const double d = x * t + y;
        r = t / d;
        i = -1.0 / d;
    }
}
// principal square root: (t, y/(2t)), t = sqrt((m + x)/2) for x >= 0, else
// (|y|/(2t), copysign(t, y)), t = sqrt((m - x)/2); m = sqrt(x x + y y)
__device__ __forceinline__ void csqrt_s(double x, double y, double &r, double &i)
{
    const double m = sqrt(x * x + y * y);
    if (x >= 0.0) {
        const double t = sqrt((m + x) / 2.0);
        r = t;
        i = y / (2.0 * t);
    } else {
        const double t = sqrt((m - x) / 2.0);
        r = fabs(y) / (2.0 * t);
        i = copysign(t, y);
    }
}

// up to 5 exact sums per block, (hi, lo) pairs in partials[(block * 5 + j) * 2]
template <int NS>
__device__ __forceinline__ void write_partials5(double *partials, double (&hi)[NS], double (&lo)[NS],
                                                double (&err)[NS])
{
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        dd_add(hi[j], lo[j], err[j]);
        block_reduce_dd<kBlock>(hi[j], lo[j]);
        if (threadIdx.x == 0) {
            partials[(blockIdx.x * 5 + j) * 2] = hi[j];
            partials[(blockIdx.x * 5 + j) * 2 + 1] = lo[j];
        }
        __syncthreads();
    }
}

// sums over w of: Re w^T w = sum (w_r^2 - w_i^2), sum w_r w_i, <lam|w> (re, im), ||w||^2
__device__ __forceinline__ void cocg_norm_sums(const double2 &w, const double2 &l, double (&hi)[5], double (&lo)[5],
                                               double (&err)[5])
{
    acc_prod(hi[0], lo[0], err[0], w.x, w.x);
    acc_prod(hi[0], lo[0], err[0], -w.y, w.y);
    acc_prod(hi[1], lo[1], err[1], w.x, w.y);
    acc_prod(hi[2], lo[2], err[2], l.x, w.x);
    acc_prod(hi[2], lo[2], err[2], l.y, w.y);
    acc_prod(hi[3], lo[3], err[3], l.x, w.y);
    acc_prod(hi[3], lo[3], err[3], -l.y, w.x);
    acc_prod(hi[4], lo[4], err[4], w.x, w.x);
    acc_prod(hi[4], lo[4], err[4], w.y, w.y);
}

__global__ void __launch_bounds__(kBlock) k_cocg_start_sums(uint32_t dim, const double2 *__restrict__ w,
                                                            const double2 *__restrict__ lam, double *partials)
{
    double hi[5] = {0, 0, 0, 0, 0}, lo[5] = {0, 0, 0, 0, 0}, err[5] = {0, 0, 0, 0, 0};
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 v = w[x];
        const double2 l = lam[x];
        cocg_norm_sums(v, l, hi, lo, err);
    }
    write_partials5<5>(partials, hi, lo, err);
}

// u = (H w_{k-1}) inv_k + c1 w_{k-2} into U (U may be Wprev: each element is read
// before it is written); partial sums of w_{k-1}^T u
__global__ void __launch_bounds__(kBlock) k_cocg_a(uint32_t dim, const double2 *__restrict__ Hw,
                                                   const double2 *__restrict__ Wcur, const double2 *Wprev,
                                                   double2 *U, const CocgState *st, double *partials, int first)
{
    if (st->done) return;
    const double ir = st->invr, ii = st->invi;
    double c1r, c1i;
    cmul_v(st->bkr, st->bki, st->ipr, st->ipi, c1r, c1i);
    c1r = -c1r;
    c1i = -c1i;
    double hi[2] = {0, 0}, lo[2] = {0, 0}, err[2] = {0, 0};
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 h = Hw[x];
        const double2 wc = Wcur[x];
        double tr, ti;
        cmul_v(h.x, h.y, ir, ii, tr, ti);
        double ur = tr, ui = ti;
        if (!first) {
            const double2 wp = Wprev[x];
            ur = fma(c1r, wp.x, fma(-c1i, wp.y, tr));
            ui = fma(c1r, wp.y, fma(c1i, wp.x, ti));
        }
        U[x] = make_double2(ur, ui);
        acc_prod(hi[0], lo[0], err[0], wc.x, ur);
        acc_prod(hi[0], lo[0], err[0], -wc.y, ui);
        acc_prod(hi[1], lo[1], err[1], wc.x, ui);
        acc_prod(hi[1], lo[1], err[1], wc.y, ur);
    }
    write_partials5<2>(partials, hi, lo, err);
}

// w_k = u + c2 w_{k-1} over U (in place); partial sums of w_k^T w_k, <lam|w_k>, ||w_k||^2
__global__ void __launch_bounds__(kBlock) k_cocg_b(uint32_t dim, double2 *__restrict__ U,
                                                   const double2 *__restrict__ Wcur,
                                                   const double2 *__restrict__ lam, const CocgState *st,
                                                   double *partials)
{
    if (st->done) return;
    const double c2r = st->c2r, c2i = st->c2i;
    double hi[5] = {0, 0, 0, 0, 0}, lo[5] = {0, 0, 0, 0, 0}, err[5] = {0, 0, 0, 0, 0};
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 u = U[x];
        const double2 wc = Wcur[x];
        const double2 l = lam[x];
        const double wr = fma(c2r, wc.x, fma(-c2i, wc.y, u.x));
        const double wi = fma(c2r, wc.y, fma(c2i, wc.x, u.y));
        const double2 w = make_double2(wr, wi);
        U[x] = w;
        cocg_norm_sums(w, l, hi, lo, err);
    }
    write_partials5<5>(partials, hi, lo, err);
}

// rounded sum j of the 5-sum partials (thread 0)
__device__ __forceinline__ double reduce_sum5(const double *partials, int nparts, int j)
{
    double hi = 0.0, lo = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock)
        dd_add_dd(hi, lo, partials[(i * 5 + j) * 2], partials[(i * 5 + j) * 2 + 1]);
    block_reduce_dd<kBlock>(hi, lo);
    __syncthreads();
    return hi + lo;
}

__global__ void __launch_bounds__(kBlock) k_cocg_fin_start(CocgState *st, CocgShift *sh, int n_omega,
                                                           const double *partials, int nparts, double shift_re,
                                                           double *c_out)
{
    __shared__ double s[5];
    for (int j = 0; j < 5; ++j) {
        const double v = reduce_sum5(partials, nparts, j);
        if (threadIdx.x == 0) s[j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n_omega; j += kBlock)
        sh[j] = CocgShift{1.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, HUGE_VAL};
    if (threadIdx.x == 0) {
        CocgState q;
        double dr, di;
        csqrt_s(s[0], 2.0 * s[1], dr, di);
        q.d0r = dr;
        q.d0i = di;
        cinv_s(dr, di, q.invr, q.invi);
        q.ipr = q.ipi = 0.0;
        q.bkr = q.bki = 0.0;
        q.akr = q.aki = 0.0;
        q.c2r = q.c2i = 0.0;
        cmul_v(q.invr, q.invi, s[2], s[3], q.ckr, q.cki);
        q.hn = (q.invr * q.invr + q.invi * q.invi) * s[4];
        q.hn0 = q.hn;
        q.alr = 1.0;
        q.ali = 0.0;
        q.ber = q.bei = 0.0;
        q.dr = dr;
        q.di = di;
        q.norm2 = s[4];
        q.shift_re = shift_re;
        q.max_resid = 0.0;
        q.seed = 0;
        q.steps = 0;
        q.numeric_error = isfinite(s[0]) && isfinite(s[1]) && isfinite(s[4]) ? 0 : 1;
        q.done = s[4] > 0.0 && !q.numeric_error ? 0 : 1;
        if (!(s[4] > 0.0)) {  // a zero right-hand side: nothing to solve, g = 0
            q.invr = q.invi = q.ckr = q.cki = q.hn = q.hn0 = 0.0;
        }
        *st = q;
        c_out[0] = q.ckr;
        c_out[1] = q.cki;
    }
}

__global__ void __launch_bounds__(kBlock) k_cocg_fin_a(CocgState *st, const double *partials, int nparts,
                                                       double *a_out, int k)
{
    if (st->done) return;
    const double s0 = reduce_sum5(partials, nparts, 0);
    const double s1 = reduce_sum5(partials, nparts, 1);
    if (threadIdx.x == 0) {
        double ar, ai;
        cmul_v(st->invr, st->invi, s0, s1, ar, ai);
        st->akr = ar;
        st->aki = ai;
        double c2r, c2i;
        cmul_v(ar, ai, st->invr, st->invi, c2r, c2i);
        st->c2r = -c2r;
        st->c2i = -c2i;
        a_out[2 * k] = ar;
        a_out[2 * k + 1] = ai;
        if (!(isfinite(ar) && isfinite(ai))) st->numeric_error = 1;
    }
}

// one step k of every shift's recurrence, the seed switch, the next basis scalars
__global__ void __launch_bounds__(kBlock) k_cocg_fin_b(CocgState *st, CocgShift *sh, const double *omega,
                                                       int n_omega, double eta, const double *partials, int nparts,
                                                       int k, double tol, double rtol, double seed_tol,
                                                       double *b_out, double *c_out)
{
    if (st->done) return;
    __shared__ double s[5];
    __shared__ double q_sc[16];
    __shared__ int s_switch;
    for (int j = 0; j < 5; ++j) {
        const double v = reduce_sum5(partials, nparts, j);
        if (threadIdx.x == 0) s[j] = v;
    }
    __syncthreads();
    const CocgState q = *st;
    const double wwr = s[0], wwi = 2.0 * s[1], nrm2 = s[4];
    double bnr, bni;
    csqrt_s(wwr, wwi, bnr, bni);
    double nir, nii;
    cinv_s(bnr, bni, nir, nii);
    const double hn1 = (nir * nir + nii * nii) * nrm2;
    // the seed: 1/alpha_k = z_s - a_k - b_k^2 alpha_{k-1}
    const int sd = q.seed;
    const double zsr = omega[sd] + q.shift_re, zsi = eta;
    double b2r, b2i, tr, ti;
    cmul_s(q.bkr, q.bki, q.bkr, q.bki, b2r, b2i);
    cmul_s(b2r, b2i, q.alr, q.ali, tr, ti);
    const double dvr = (zsr - q.akr) - tr, dvi = (zsi - q.aki) - ti;
    double anr, ani;
    cdiv_s(1.0, 0.0, dvr, dvi, anr, ani);
    double fr, fi;
    cmul_s(anr, ani, q.ber, q.bei, fr, fi);
    cdiv_s(fr, fi, q.alr, q.ali, fr, fi);  // alpha_k beta_{k-1} / alpha_{k-1}
    // delta_k c_k, then the seed coefficients of the next step
    double er, ei;
    cmul_s(q.dr, q.di, q.ckr, q.cki, er, ei);
    double bsr, bsi, a2r, a2i, ber, bei, wr, wi, dnr, dni;
    cmul_s(bnr, bni, bnr, bni, bsr, bsi);
    cmul_s(anr, ani, anr, ani, a2r, a2i);
    cmul_s(bsr, bsi, a2r, a2i, ber, bei);  // beta_k = b_{k+1}^2 alpha_k^2
    cmul_s(anr, ani, bnr, bni, wr, wi);
    cmul_s(wr, wi, q.dr, q.di, dnr, dni);  // delta_{k+1} = alpha_k b_{k+1} delta_k
    const double rs = sqrt(dnr * dnr + dni * dni) * sqrt(hn1);
    const double nrm_b = sqrt(q.hn0) * sqrt(q.d0r * q.d0r + q.d0i * q.d0i);  // ||chi||
    const double thr = seed_tol * nrm_b;
    // every running shift; largest residual and its (first) index
    double rmax = -1.0;
    int imax = 0;
    double rseed = 0.0;
    for (int j = threadIdx.x; j < n_omega; j += kBlock) {
        CocgShift p = sh[j];
        if (j != sd && p.res <= thr) {  // converged: keeps its values
            if (p.res > rmax) {
                rmax = p.res;
                imax = j;
            }
            continue;
        }
        const double sgr = (omega[j] + q.shift_re) - zsr, sgi = eta - zsi;
        double t1r, t1i, d1r, d1i, u1r, u1i, u2r, u2i;
        cmul_s(anr, ani, sgr, sgi, t1r, t1i);
        d1r = p.pr - p.por;
        d1i = p.pi - p.poi;
        cmul_s(1.0 + t1r, t1i, p.pr, p.pi, u1r, u1i);
        cmul_s(fr, fi, d1r, d1i, u2r, u2i);
        const double pnr = u1r + u2r, pni = u1i + u2i;
        double qr, qi, q2r, q2i, bjr, bji, xr, xi, ajr, aji, hr, hi2, mr, mi, vr, vi;
        cdiv_s(p.por, p.poi, p.pr, p.pi, qr, qi);
        cmul_s(qr, qi, qr, qi, q2r, q2i);
        cmul_s(q.ber, q.bei, q2r, q2i, bjr, bji);
        cdiv_s(p.pr, p.pi, pnr, pni, xr, xi);
        cmul_s(anr, ani, xr, xi, ajr, aji);
        cdiv_s(er, ei, p.pr, p.pi, hr, hi2);
        cmul_s(bjr, bji, p.Pr, p.Pi, mr, mi);
        p.Pr = hr + mr;
        p.Pi = hi2 + mi;
        cmul_s(ajr, aji, p.Pr, p.Pi, vr, vi);
        p.gr = p.gr + vr;
        p.gi = p.gi + vi;
        p.por = p.pr;
        p.poi = p.pi;
        p.pr = pnr;
        p.pi = pni;
        const double res = rs / sqrt(pnr * pnr + pni * pni);
        p.res = res;
        sh[j] = p;
        if (res > rmax) {
            rmax = res;
            imax = j;
        }
        if (j == sd) rseed = res;
    }
    // block argmax (first index on ties) and the seed's residual
    __shared__ double r_sh[kBlock / 64];
    __shared__ int i_sh[kBlock / 64];
    __shared__ double rs_sh[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double orr = __shfl_xor(rmax, off, 64);
        const int oi = __shfl_xor(imax, off, 64);
        const double os = __shfl_xor(rseed, off, 64);
        if (orr > rmax || (orr == rmax && oi < imax)) {
            rmax = orr;
            imax = oi;
        }
        rseed = os > rseed ? os : rseed;
    }
    if ((threadIdx.x & 63) == 0) {
        r_sh[threadIdx.x >> 6] = rmax;
        i_sh[threadIdx.x >> 6] = imax;
        rs_sh[threadIdx.x >> 6] = rseed;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            if (r_sh[w] > r_sh[0] || (r_sh[w] == r_sh[0] && i_sh[w] < i_sh[0])) {
                r_sh[0] = r_sh[w];
                i_sh[0] = i_sh[w];
            }
            rs_sh[0] = rs_sh[w] > rs_sh[0] ? rs_sh[w] : rs_sh[0];
        }
        CocgState n = q;
        n.alr = anr;
        n.ali = ani;
        n.ber = ber;
        n.bei = bei;
        n.dr = dnr;
        n.di = dni;
        n.max_resid = r_sh[0];
        n.steps = k + 1;
        s_switch = -1;
        const bool truncated = rtol > 0.0 && r_sh[0] <= rtol * nrm_b;
        const bool converged = rs_sh[0] <= thr && !(r_sh[0] > thr);
        if (!truncated && rs_sh[0] <= thr && r_sh[0] > thr) {
            // the new seed: alpha_k, beta_k, delta_{k+1} of shift t; every pi rebased on t
            const int t = i_sh[0];
            const CocgShift pt = sh[t];
            double xr, xi, x2r, x2i;
            cdiv_s(pt.por, pt.poi, pt.pr, pt.pi, xr, xi);
            cmul_s(n.alr, n.ali, xr, xi, n.alr, n.ali);
            cmul_s(xr, xi, xr, xi, x2r, x2i);
            cmul_s(n.ber, n.bei, x2r, x2i, n.ber, n.bei);
            cdiv_s(n.dr, n.di, pt.pr, pt.pi, n.dr, n.di);
            q_sc[0] = pt.por;
            q_sc[1] = pt.poi;
            q_sc[2] = pt.pr;
            q_sc[3] = pt.pi;
            n.seed = t;
            s_switch = t;
        }
        // the basis scalars of the next step, breakdown and truncation tests
        b_out[2 * k] = bnr;
        b_out[2 * k + 1] = bni;
        double cnr, cni;
        cmul_v(nir, nii, s[2], s[3], cnr, cni);
        c_out[2 * (k + 1)] = cnr;
        c_out[2 * (k + 1) + 1] = cni;
        if (!(isfinite(bnr) && isfinite(bni) && isfinite(nrm2))) n.numeric_error = 1;
        const bool breakdown = !(sqrt(nrm2) > tol) || !(sqrt(wwr * wwr + wwi * wwi) > 1e-24 * nrm2);
        if (breakdown || truncated || converged || n.numeric_error) {
            n.done = 1;
        } else {
            n.ipr = q.invr;
            n.ipi = q.invi;
            n.invr = nir;
            n.invi = nii;
            n.bkr = bnr;
            n.bki = bni;
            n.ckr = cnr;
            n.cki = cni;
            n.hn = hn1;
        }
        *st = n;
    }
    __syncthreads();
    if (s_switch >= 0) {
        const double o_r = q_sc[0], o_i = q_sc[1], n_r = q_sc[2], n_i = q_sc[3];
        for (int j = threadIdx.x; j < n_omega; j += kBlock) {
            CocgShift p = sh[j];
            if (!(p.res > thr)) continue;  // converged shifts are not rebased
            cdiv_s(p.por, p.poi, o_r, o_i, p.por, p.poi);
            cdiv_s(p.pr, p.pi, n_r, n_i, p.pr, p.pi);
            sh[j] = p;
        }
    }
}

__global__ void k_cocg_finish(const CocgState *st, const CocgShift *sh, int n_omega, double2 *g)
{
    const bool any = st->steps > 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_omega; j += gridDim.x * blockDim.x)
        g[j] = any ? make_double2(sh[j].gr, sh[j].gi) : make_double2(0.0, 0.0);
}

void launch_cocg_start(uint32_t dim, const double *chi, const double *lam, double *partials, CocgState *st,
                       CocgShift *sh, int n_omega, double shift_re, double *c_out, hipStream_t s)
{
    const int grid = vec_grid(dim);
    hipLaunchKernelGGL(k_cocg_start_sums, dim3(grid), dim3(kBlock), 0, s, dim, (const double2 *)chi,
                       (const double2 *)lam, partials);
    hipLaunchKernelGGL(k_cocg_fin_start, dim3(1), dim3(kBlock), 0, s, st, sh, n_omega, partials, grid, shift_re,
                       c_out);
}

void launch_cocg_step(const HvOp &op, const double *lam, const double *Wcur, const double *Wprev, double *U,
                      double *Hw, double *partials, CocgState *st, CocgShift *sh, const double *omega, int n_omega,
                      double eta, int k, double tol, double rtol, double seed_tol, double *a_out, double *b_out,
                      double *c_out, hipStream_t s)
{
    const uint32_t dim = 1u << op.P.n_sites;
    const int grid = vec_grid(dim);
    launch_apply_h(op, Wcur, Hw, s);
    hipLaunchKernelGGL(k_cocg_a, dim3(grid), dim3(kBlock), 0, s, dim, (const double2 *)Hw, (const double2 *)Wcur,
                       (const double2 *)Wprev, (double2 *)U, (const CocgState *)st, partials, k == 0 ? 1 : 0);
    hipLaunchKernelGGL(k_cocg_fin_a, dim3(1), dim3(kBlock), 0, s, st, partials, grid, a_out, k);
    hipLaunchKernelGGL(k_cocg_b, dim3(grid), dim3(kBlock), 0, s, dim, (double2 *)U, (const double2 *)Wcur,
                       (const double2 *)lam, (const CocgState *)st, partials);
    hipLaunchKernelGGL(k_cocg_fin_b, dim3(1), dim3(kBlock), 0, s, st, sh, omega, n_omega, eta, partials, grid, k, tol,
                       rtol, seed_tol, b_out, c_out);
}

void launch_cocg_finish(const CocgState *st, const CocgShift *sh, int n_omega, double *g, hipStream_t s)
{
    const int grid = (n_omega + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_cocg_finish, dim3(grid < 1 ? 1 : grid), dim3(kBlock), 0, s, st, sh, n_omega, (double2 *)g);
}

}  // namespace ftk
