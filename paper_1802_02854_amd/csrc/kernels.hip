// HIP kernels (gfx950) of the FTKw path.  Compiled with -ffp-contract=off:
// every fused multiply-add below is an explicit fma(), everything else is a
// separately rounded IEEE double operation, as the library's arithmetic
// contract requires (see ftkw.h).
//
// The matrix-free product H v is the hot spot: 3N/2 bit-flip gathers per basis
// element (36 at N = 24) against 32 bytes of HBM traffic.  Its blocked form
// gives each thread 8 elements x_e = xb + 64 e (bits 6..8 of the index), so a
// wave covers 512 consecutive elements and every gather instruction reads 1 KB
// of consecutive memory; the bond parity, amplitude choice and address are
// computed once per thread and bond and shared by the 8 elements.  In the tiled
// form a workgroup of 16 waves first stages its 8192-element tile in LDS and
// bonds whose flip mask lies inside the tile read their partners from LDS; the
// others go through L1/L2.  Tiles are handed to the 8 XCDs in contiguous ranges
// so that partner tiles differing in the low tile bits share an L2.  At large N
// the partner tiles of the single-pass forms no longer fit the caches and their
// re-reads bound the kernel; the multi-pass form (kernels.h) then reads every
// element once per pass and touches no partner outside its LDS tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "exact_sum.h"
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
        P.smask[t.bi[b]] |= 1ull << b;
        P.smask[t.bj[b]] |= 1ull << b;
        if (t.gamma[b] == 2) P.zmask |= 1ull << b;
    }
    P.jq = t.jq;
    P.kq = t.kq;
    return P;
}


// Greedy cut of the bond list into segments whose sites, with the core sites
// 0..core-1, fit a pass tile; the core size with the fewest passes wins (the
// larger core on ties: longer contiguous runs, up to 64 elements = one wave's
// load of 1 KiB).
HvPlan make_hv_plan(const BondTable &t)
{
    HvPlan best;
    const int N = t.n_sites;
    if (N <= kPassBits) return best;
    for (int core = 6; core >= 2; --core) {
        HvPlan plan;
        plan.core = core;
        std::vector<std::pair<int, int>> segs;
        std::vector<uint32_t> seg_sites;
        const uint32_t core_mask = (1u << core) - 1u;
        uint32_t sites = core_mask;
        int b0 = 0;
        for (int b = 0; b < t.n_bonds; ++b) {
            const uint32_t s2 = sites | (1u << t.bi[b]) | (1u << t.bj[b]);
            if (__builtin_popcount(s2) > kPassBits) {
                segs.push_back({b0, b});
                seg_sites.push_back(sites);
                b0 = b;
                sites = core_mask | (1u << t.bi[b]) | (1u << t.bj[b]);
            } else {
                sites = s2;
            }
        }
        segs.push_back({b0, t.n_bonds});
        seg_sites.push_back(sites);
        if ((int)segs.size() > kMaxPasses) continue;
        plan.n_passes = (int)segs.size();
        for (int p = 0; p < plan.n_passes; ++p) {
            PassGeom &g = plan.pass[p];
            std::memset(&g, 0, sizeof(g));
            g.b0 = segs[p].first;
            g.b1 = segs[p].second;
            // pad with the lowest free sites, then order the tile bits by site
            uint32_t m = seg_sites[p];
            for (int l = 0; l < N && __builtin_popcount(m) < kPassBits; ++l) m |= 1u << l;
            int tsite[kPassBits], nt = 0, nh = 0;
            int pos[kMaxSites];
            for (int l = 0; l < N; ++l) {
                if (m >> l & 1u) {
                    pos[l] = nt;
                    tsite[nt++] = l;
                } else {
                    pos[l] = -1;
                    g.hsite[nh++] = (uint8_t)l;
                }
            }
            for (int j = 0; j < 6; ++j) g.ysite[j] = (uint8_t)tsite[j];
            for (int j = 0; j < 3; ++j) g.ysite[6 + j] = (uint8_t)tsite[9 + j];
            for (int e = 0; e < kR; ++e) {
                uint32_t x = 0;
                for (int j = 0; j < 3; ++j)
                    if (e >> j & 1) x |= 1u << tsite[6 + j];
                g.ebit[e] = x;
            }
            for (int b = g.b0; b < g.b1; ++b) {
                g.tbi[b] = (uint8_t)pos[t.bi[b]];
                g.tbj[b] = (uint8_t)pos[t.bj[b]];
            }
            for (int j = 0; j < 3; ++j) g.esite[j] = (uint8_t)tsite[6 + j];
            // (tile index, lane, wave, e) -> x must be a bijection onto [0, 2^N)
            uint32_t seen = 0;
            bool ok = nt == kPassBits && nh == N - kPassBits;
            for (int j = 0; j < 9; ++j) ok = ok && !(seen >> g.ysite[j] & 1u), seen |= 1u << g.ysite[j];
            ok = ok && (g.ebit[7] & seen) == 0 && __builtin_popcount(g.ebit[7]) == 3;
            seen |= g.ebit[7];
            for (int j = 0; j < nh; ++j) ok = ok && !(seen >> g.hsite[j] & 1u), seen |= 1u << g.hsite[j];
            ok = ok && seen == (N == 32 ? ~0u : (1u << N) - 1u);
            for (int b = g.b0; b < g.b1; ++b) ok = ok && g.tbi[b] < kPassBits && g.tbj[b] < kPassBits;
            if (!ok) plan.n_passes = -1;
        }
        if (plan.n_passes < 0) continue;
        if (best.n_passes == 0 || plan.n_passes < best.n_passes) best = plan;
    }
    return best;
}

int vec_grid(uint32_t dim)
{
    uint32_t g = (dim + kBlock - 1) / kBlock;
    return (int)(g < (uint32_t)kMaxGrid ? g : (uint32_t)kMaxGrid);
}

// ---------------------------------------------------------------------------
// Device bounds checks of the debug build (-DFTK_DEVICE_CHECKS, libftkw_check.so):
// FTK_IDX(i, top, lim, site) states that indices i .. i + top of a buffer with lim
// entries are read or written.  In the debug build a violation is counted in
// g_dcheck (count, site of the first, its index) and index 0 is used instead, so
// the kernel finishes and the host reports it; the release build compiles the
// check away.  Sites: 1 single-element H v gather, 2/3 blocked and tiled gathers
// (global, LDS), 4 own elements of the blocked/tiled forms, 5 own LDS entries of
// the tiled form, 6/7 multi-pass global element and LDS tile entries, 8 multi-pass
// LDS partners, 9 bond constants staged in LDS, 10/11 batch-layout own elements
// and partners, 12 S^alpha_Q gathers, 13 filter accumulation.
#ifdef FTK_DEVICE_CHECKS
__device__ unsigned int g_dcheck[3];
__device__ __forceinline__ uint32_t dchk(uint32_t i, uint32_t top, uint32_t lim, uint32_t site)
{
    if (i < lim && top < lim - i) return i;
    if (atomicAdd(&g_dcheck[0], 1u) == 0u) {
        g_dcheck[1] = site;
        g_dcheck[2] = i;
    }
    return 0u;
}
#define FTK_IDX(i, top, lim, site) dchk((uint32_t)(i), (uint32_t)(top), (uint32_t)(lim), (site))
int device_checks_compiled() { return 1; }
// one claimed access to entries 5..5 of a 4-entry buffer (site 99): counted, redirected to 0;
// nothing is read or written at the claimed index
__global__ void k_dcheck_selftest(uint32_t *out) { out[0] = FTK_IDX(5u, 0u, 4u, 99u); }
void device_checks_selftest(uint32_t *out_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_dcheck_selftest, dim3(1), dim3(1), 0, s, out_dev);
}
void device_checks_read(unsigned int out[3], bool clear)
{
    hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_dcheck), 3 * sizeof(unsigned int));
    if (e == hipSuccess && clear) {
        const unsigned int z[3] = {0u, 0u, 0u};
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_dcheck), z, 3 * sizeof(unsigned int));
    }
    if (e != hipSuccess) out[0] = out[1] = out[2] = ~0u;
}
#else
#define FTK_IDX(i, top, lim, site) (i)
int device_checks_compiled() { return 0; }
void device_checks_selftest(uint32_t *, hipStream_t) {}
void device_checks_read(unsigned int out[3], bool) { out[0] = out[1] = out[2] = 0u; }
#endif

static int g_hv_mode = -1;  // -1: chosen by size
static int g_pass_grid = 0;  // workgroups of a multi-pass launch (0: two per compute unit)
static bool g_full_grid = true;  // passes without partial sums: one workgroup per tile
static bool g_fuse_fin = true;   // beta finalisation inside the middle pass of a step
static int g_cus = 256;      // compute units of the device (set with the kernel attributes)

void set_hv_mode(int mode) { g_hv_mode = mode; }
void set_pass_grid(int grid) { g_pass_grid = grid; }
void set_full_grid(int on) { g_full_grid = on != 0; }
static int g_hints = -1;  // forced hint set of the multi-pass form (-1: per op)
void set_hints(int mode) { g_hints = mode; }
int forced_hints() { return g_hints; }

// The streaming set where one launch's vectors (B sequences of 2^N complex entries)
// come to 128-512 MiB, about the size of the 256 MB last-level cache; the cached
// set for smaller and larger working sets (the measurements are with the sets'
// definition above).
bool stream_hints(const HvOp &op, int B)
{
    if (g_hints >= 0) return g_hints != 0;
    if (op.hints >= 0) return op.hints != 0;
    const double mib = (double)B * 16.0 * (double)(1u << op.P.n_sites) / (1024.0 * 1024.0);
    return mib >= 128.0 && mib <= 512.0;
}
void set_fuse_finalize(int on) { g_fuse_fin = on != 0; }

int hv_mode(const HvOp &op)
{
    const uint32_t dim = 1u << op.P.n_sites;
    const bool multi = op.plan.n_passes > 0 && op.scratch != nullptr;
    int best = dim >= (uint32_t)kTile ? 2 : (dim >= (uint32_t)kChunk ? 1 : 0);
    if (g_hv_mode == 3) return multi ? 3 : best;
    if (g_hv_mode >= 0) return g_hv_mode <= best ? g_hv_mode : best;
    // by size: the multi-pass form once a vector outgrows the caches (measured: also with
    // 5 passes it beats the single-kernel tiled form, 11.9 against 16.9 ms at 28 sites,
    // 48.5 against 81.8 ms at 30)
    if (multi && op.P.n_sites >= 18) return 3;
    return best;
}

int pass_grid_cap(const HvOp &op)
{
    if (op.pass_grid > 0) return op.pass_grid;
    return g_pass_grid > 0 ? g_pass_grid : 2 * g_cus;
}

int hv_grid(const HvOp &op, int B)
{
    if (B <= 1 || !lanczos_stackable(op)) return hv_grid(op);
    // the stack shares the persistent workgroups: about cap / B per sequence, at
    // most one per tile
    const uint32_t tiles = (1u << op.P.n_sites) / kPassTile;
    const uint32_t cap = (uint32_t)pass_grid_cap(op);
    const uint32_t per = (cap + (uint32_t)B - 1) / (uint32_t)B;
    return (int)(tiles < per ? tiles : per);
}

int hv_grid(const HvOp &op)
{
    const uint32_t dim = 1u << op.P.n_sites;
    switch (hv_mode(op)) {
    case 3: {
        uint32_t tiles = dim / kPassTile;
        // persistent workgroups, two per compute unit (the LDS holds two 64 KiB tiles),
        // each looping over tiles: fewer partial sums for the scalar kernels to reduce
        const uint32_t cap = (uint32_t)pass_grid_cap(op);
        return (int)(tiles < cap ? tiles : cap);
    }
    case 2: {
        uint32_t tiles = dim / kTile;
        return (int)(tiles < (uint32_t)kMaxGrid ? tiles : (uint32_t)kMaxGrid);
    }
    case 1: {
        uint32_t g = dim / (kChunk * (kBlock / 64));
        return (int)(g < 1 ? 1 : (g < (uint32_t)kMaxGrid ? g : (uint32_t)kMaxGrid));
    }
    default:
        return vec_grid(dim);
    }
}

// Streaming accesses of the multi-pass form.  Every element is touched once per
// pass; which accesses carry the nontemporal hint was chosen by measurement.
typedef double nt_double2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2 *p)
{
    const nt_double2 v = __builtin_nontemporal_load((const nt_double2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(double2 *p, double2 a)
{
    nt_double2 v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, (nt_double2 *)p);
}

// Two sets of cache hints for the multi-pass form, picked per launch (stream_hints).
// Both load the pass inputs and partial sums nontemporally.  The cached set stores
// the partial sums nontemporally and lets the fused first pass load and store
// plainly; the streaming set stores the partial sums plainly (the very next pass
// reads them back), makes the fused first pass's loads and its store of w
// nontemporal, and runs the first pass's tiles in descending order.  Measured at
// 24 sites, one sequence per launch (256 MiB per vector): 0.515 ms per Lanczos step
// cached, 0.481 ms streaming; stacks of 16 sequences at 20 sites (256 MiB) 29.3k
// against 32.5k Krylov iterations/s; at 16-18 sites (stacks of 16) and for
// stacks at 24 sites the cached set is 1-5 % faster, as it is for one 20-site
// vector (7 %).
template <bool NT>
__device__ __forceinline__ double2 ld_h(const double2 *p)
{
    if constexpr (NT) return ld_nt(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st_h(double2 *p, double2 a)
{
    if constexpr (NT) st_nt(p, a);
    else *p = a;
}

// ---------------------------------------------------------------------------
// (H v)[x] by the contract, one element: D from integer bond-parity sums, then
// one fma per bond in list order.
__device__ __forceinline__ void hv_at(const HvParams &P, uint32_t x, const double2 *__restrict__ v,
                                      double &re, double &im, double2 &vx)
{
    int s_all = 0, s_z = 0;
    for (int b = 0; b < P.n_bonds; ++b) {
        const int s = (((x >> P.bi[b]) ^ (x >> P.bj[b])) & 1u) ? -1 : 1;
        s_all += s;
        if (P.isz[b]) s_z += s;
    }
    const double D = fma(P.kq, (double)s_z, P.jq * (double)s_all);
    vx = v[x];
    re = D * vx.x;
    im = D * vx.y;
    for (int b = 0; b < P.n_bonds; ++b) {
        const bool anti = ((x >> P.bi[b]) ^ (x >> P.bj[b])) & 1u;
        const double amp = anti ? P.aa[b] : P.ap[b];
        const double2 vy = v[FTK_IDX(x ^ P.mask[b], 0, 1u << P.n_sites, 1)];
        re = fma(amp, vy.x, re);
        im = fma(amp, vy.y, im);
    }
}

// Blocked form: the 8 elements xb + 64 e (xb has bits 6..8 clear).
constexpr int kRegShift = 6;

// The bond constants of a pass segment (tile bit positions of both ends, the two
// flip amplitudes), staged once per workgroup in LDS: the bond loop then reads LDS
// only instead of kernel-argument memory behind waits on global memory.  Visible
// to the loop after the first barrier of the tile loop.
struct SegLds {
    uint32_t pq[kMaxBonds];  // tbi | tbj << 8
    double aa[kMaxBonds], ap[kMaxBonds];
};
__device__ __forceinline__ void stage_segment(SegLds &seg, const HvParams &P, const PassGeom &g)
{
    const int b = g.b0 + (int)threadIdx.x;
    if (b < g.b1) {
        const uint32_t bb = FTK_IDX(b, 0, kMaxBonds, 9);
        seg.pq[bb] = (uint32_t)g.tbi[bb] | (uint32_t)g.tbj[bb] << 8;
        seg.aa[bb] = P.aa[bb];
        seg.ap[bb] = P.ap[bb];
    }
}

template <int MR>
__device__ __forceinline__ void bond_accum(double (&re)[kR], double (&im)[kR], const double2 (&pv)[kR],
                                           double ampA, double ampB)
{
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        const double amp = (__builtin_popcount(e & MR) & 1) ? ampB : ampA;
        re[e] = fma(amp, pv[e ^ MR].x, re[e]);
        im[e] = fma(amp, pv[e ^ MR].y, im[e]);
    }
}

// The same with partners read straight from the LDS tile (src = tile + (yb ^ mrest)):
// the compiler interleaves the LDS reads with the fmas instead of holding all kR
// partners in registers.
template <int MR>
__device__ __forceinline__ void bond_accum_lds(double (&re)[kR], double (&im)[kR], const double2 *src,
                                               double ampA, double ampB)
{
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        const double amp = (__builtin_popcount(e & MR) & 1) ? ampB : ampA;
        const double2 q = src[(e ^ MR) << kRegShift];
        re[e] = fma(amp, q.x, re[e]);
        im[e] = fma(amp, q.y, im[e]);
    }
}

// The same for any register mask mr without a switch: the partner of element e is
// tile[base ^ (e << kRegShift)] with base = yb ^ (the bond's full flip mask), and
// element e takes ampB when e & mr has odd parity (bit e of sel).  One code path for
// every bond, so the accumulators stay in their registers across the bond loop
// (the eight switch cases merged their results through register copies).
__device__ __forceinline__ void bond_accum_lds_flat(double (&re)[kR], double (&im)[kR], const double2 *tile,
                                                    uint32_t base, uint32_t mr, double ampA, double ampB)
{
    uint32_t sel = 0;
    if (mr & 1u) sel ^= 0xAAu;
    if (mr & 2u) sel ^= 0xCCu;
    if (mr & 4u) sel ^= 0xF0u;
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        const double2 q = tile[base ^ ((uint32_t)e << kRegShift)];
        const double amp = ((sel >> e) & 1u) ? ampB : ampA;
        re[e] = fma(amp, q.x, re[e]);
        im[e] = fma(amp, q.y, im[e]);
    }
}

#define FTK_SWITCH_MR(mr, F, ...)            \
    switch (mr) {                            \
    case 0: F<0>(__VA_ARGS__); break;        \
    case 1: F<1>(__VA_ARGS__); break;        \
    case 2: F<2>(__VA_ARGS__); break;        \
    case 3: F<3>(__VA_ARGS__); break;        \
    case 4: F<4>(__VA_ARGS__); break;        \
    case 5: F<5>(__VA_ARGS__); break;        \
    case 6: F<6>(__VA_ARGS__); break;        \
    default: F<7>(__VA_ARGS__); break;       \
    }

// Diagonal D(x_e) for the 8 elements x_e = xb + (e << RS): D = K/4 s_z + J/4 s_all
// with s = (bonds) - 2 (antiparallel bonds), counted on the bond-parity vector.
template <int RS = kRegShift>
__device__ __forceinline__ void diag_block(const HvParams &P, uint32_t xb, double (&D)[kR])
{
    uint64_t par = 0;
    for (int l = 0; l < P.n_sites; ++l)
        if ((xb >> l) & 1u) par ^= P.smask[l];
    const int nz = __popcll(P.zmask);
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        uint64_t pe = par;
        if (e & 1) pe ^= P.smask[RS];
        if (e & 2) pe ^= P.smask[RS + 1];
        if (e & 4) pe ^= P.smask[RS + 2];
        const int s_all = P.n_bonds - 2 * __popcll(pe);
        const int s_z = nz - 2 * __popcll(pe & P.zmask);
        D[e] = fma(P.kq, (double)s_z, P.jq * (double)s_all);
    }
}

// Off-diagonal part added to (re, im) in bond-list order.  With TILED, bonds
// whose mask is below kTile read partners from the LDS copy `tile` of the
// workgroup's tile (xl = xb - tile base); the others read global memory.
template <bool TILED>
__device__ __forceinline__ void offdiag_block(const HvParams &P, uint32_t xb, uint32_t xl,
                                              const double2 *__restrict__ v, const double2 *tile,
                                              double (&re)[kR], double (&im)[kR])
{
    for (int b = 0; b < P.n_bonds; ++b) {
        const uint32_t m = P.mask[b];
        const uint32_t mrest = m & ~(7u << kRegShift);
        const int mr = (m >> kRegShift) & 7;
        const bool anti = ((xb >> P.bi[b]) ^ (xb >> P.bj[b])) & 1u;
        const double ampA = anti ? P.aa[b] : P.ap[b];
        const double ampB = anti ? P.ap[b] : P.aa[b];
        double2 pv[kR];
        if (TILED && m < (uint32_t)kTile) {
            const double2 *src = tile + FTK_IDX(xl ^ mrest, 7u << kRegShift, kTile, 3);
#pragma unroll
            for (int e = 0; e < kR; ++e) pv[e] = src[e << kRegShift];
        } else {
            const double2 *src = v + FTK_IDX(xb ^ mrest, 7u << kRegShift, 1u << P.n_sites, 2);
#pragma unroll
            for (int e = 0; e < kR; ++e) pv[e] = src[e << kRegShift];
        }
        FTK_SWITCH_MR(mr, bond_accum, re, im, pv, ampA, ampB);
    }
}

// ---------------------------------------------------------------------------
// Epilogues: what each H-applying kernel does with (H v)[x] once it has it.
// A kernel with kR elements per thread first calls load(x_e) for all of them,
// then apply(..., loaded value): every input an epilogue reads is loaded before
// any output is stored, which the compiler could not arrange itself because the
// buffers may alias (the Lanczos output overwrites w_{k-2} in place).
struct EpiApply {
    static constexpr bool kReduces = false;  // no per-workgroup partial sums
    double2 *w;
    __device__ void select(int, size_t, int) {}
    __device__ bool active() const { return true; }
    __device__ void init() {}
    __device__ double2 load(size_t) const { return make_double2(0.0, 0.0); }
    __device__ void apply(size_t x, double re, double im, const double2 &, const double2 &) { w[x] = make_double2(re, im); }
    __device__ void operator()(size_t x, double re, double im, const double2 &vx) { apply(x, re, im, vx, load(x)); }
    template <int BLOCK>
    __device__ void finish() {}
};

struct EpiTaylor {
    static constexpr bool kReduces = false;
    double2 *tn;
    double2 *acc;
    double a, b;
    __device__ void select(int, size_t, int) {}
    __device__ bool active() const { return true; }
    __device__ void init() {}
    __device__ double2 load(size_t x) const { return acc[x]; }
    __device__ void apply(size_t x, double re, double im, const double2 &tx, const double2 &c)
    {
        const double nr = fma(a, tx.x, b * re);
        const double ni = fma(a, tx.y, b * im);
        tn[x] = make_double2(nr, ni);
        acc[x] = make_double2(c.x + nr, c.y + ni);
    }
    __device__ void operator()(size_t x, double re, double im, const double2 &tx) { apply(x, re, im, tx, load(x)); }
    template <int BLOCK>
    __device__ void finish() {}
};

// one element per thread (small clusters)
template <class Epi>
__global__ void __launch_bounds__(kBlock) k_hv_simple(HvParams P, const double2 *__restrict__ v, Epi epi)
{
    if (!epi.active()) return;
    const uint32_t dim = 1u << P.n_sites;
    epi.init();
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        double re, im;
        double2 vx;
        hv_at(P, x, v, re, im, vx);
        epi(x, re, im, vx);
    }
    epi.template finish<kBlock>();
}

// 8 elements per thread, partners from global memory
template <class Epi>
__global__ void __launch_bounds__(kBlock) k_hv_blocked(HvParams P, const double2 *__restrict__ v, Epi epi)
{
    const uint32_t dim = 1u << P.n_sites;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    if (!epi.active()) return;
    epi.init();
    for (uint32_t c = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); c < dim / kChunk; c += waves) {
        const uint32_t xb = FTK_IDX(c * kChunk + lane, 7u << kRegShift, dim, 4);
        double D[kR], re[kR], im[kR];
        diag_block(P, xb, D);
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const double2 o = v[xb + (e << kRegShift)];
            re[e] = D[e] * o.x;
            im[e] = D[e] * o.y;
        }
        offdiag_block<false>(P, xb, 0, v, nullptr, re, im);
        double2 in[kR];
#pragma unroll
        for (int e = 0; e < kR; ++e) in[e] = epi.load(xb + (e << kRegShift));
#pragma unroll
        for (int e = 0; e < kR; ++e) epi.apply(xb + (e << kRegShift), re[e], im[e], v[xb + (e << kRegShift)], in[e]);
    }
    epi.template finish<kBlock>();
}

// 16 waves per workgroup, the 8192-element tile staged in LDS (128 KiB)
template <class Epi>
__global__ void __launch_bounds__(kTileThreads) k_hv_tiled(HvParams P, const double2 *__restrict__ v, Epi epi)
{
    extern __shared__ double2 tile[];
    const uint32_t dim = 1u << P.n_sites;
    const uint32_t ntiles = dim / kTile;
    const uint32_t lane = threadIdx.x & 63;
    // offset of this thread's elements in the tile
    const uint32_t xw = FTK_IDX((threadIdx.x >> 6) * kChunk + lane, 7u << kRegShift, kTile, 5);
    // XCD-aware order: workgroup i runs on XCD i % 8; give each XCD a contiguous range of tiles
    const uint32_t per_xcd = (ntiles + 7) / 8;
    if (!epi.active()) return;
    epi.init();
    for (uint32_t it = blockIdx.x; it < ntiles; it += gridDim.x) {
        uint32_t t = (it % 8) * per_xcd + it / 8;
        if (per_xcd * 8 != ntiles) t = it;  // fewer than 8 tiles or uneven: natural order
        const uint32_t base = t * kTile;
        const uint32_t xb = FTK_IDX(base + xw, 7u << kRegShift, dim, 4);
        double D[kR], re[kR], im[kR];
        __syncthreads();  // the previous tile is no longer read
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const double2 o = v[xb + (e << kRegShift)];
            tile[xw + (e << kRegShift)] = o;
            re[e] = o.x;
            im[e] = o.y;
        }
        diag_block(P, xb, D);
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            re[e] = D[e] * re[e];
            im[e] = D[e] * im[e];
        }
        __syncthreads();
        offdiag_block<true>(P, xb, xw, v, tile, re, im);
        double2 in[kR];
#pragma unroll
        for (int e = 0; e < kR; ++e) in[e] = epi.load(xb + (e << kRegShift));
#pragma unroll
        for (int e = 0; e < kR; ++e) epi.apply(xb + (e << kRegShift), re[e], im[e], tile[xw + (e << kRegShift)], in[e]);
    }
    epi.template finish<kTileThreads>();
}

// One pass of the multi-pass form over every tile of its site set.  A thread
// owns the kR elements of tile index yb + 64 e (yb = lane | wave << 9); FIRST
// starts from D v, otherwise from the partial sums in `part`; LAST hands the
// finished (H v)[x] to the epilogue, otherwise the partial sums go back to `part`.
template <class Epi, bool FIRST, bool LAST, bool SH>
__global__ void __launch_bounds__(kPassThreads, 4) k_hv_pass(HvParams P, PassGeom g, const double2 *__restrict__ v,
                                                         double2 *part, Epi epi, size_t vs)
{
    extern __shared__ double2 tile[];
    // the tile workgroups are gx = gridDim.x columns; a middle pass of a Lanczos step
    // may carry one more column that finalises beta of the previous half step
    uint32_t gx = gridDim.x;
    if constexpr (!FIRST && !LAST && Epi::kReduces) {
        if (epi.fin) {
            gx = gridDim.x - 1;
            if (blockIdx.x == gx) {
                epi.finalize_block(blockIdx.y);
                return;
            }
        }
    }
    // sequence blockIdx.y of a stacked batch (vs = 0: one sequence)
    v += blockIdx.y * vs;
    part += blockIdx.y * vs;
    epi.select(blockIdx.y, vs, 2 * gx);
    const int hbits = P.n_sites - kPassBits;
    const uint32_t ntiles = 1u << hbits;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t yb = FTK_IDX(lane | (wave << 9), 7u << kRegShift, kPassTile, 7);
    uint32_t xy = 0;
    uint64_t pxy = 0;  // bond parities of the thread's base offset
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if ((lane >> j) & 1u) xy |= 1u << g.ysite[j], pxy ^= P.smask[g.ysite[j]];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if ((wave >> j) & 1u) xy |= 1u << g.ysite[6 + j], pxy ^= P.smask[g.ysite[6 + j]];
    const uint64_t pe6 = FIRST ? P.smask[g.esite[0]] : 0, pe7 = FIRST ? P.smask[g.esite[1]] : 0,
                   pe8 = FIRST ? P.smask[g.esite[2]] : 0;
    const int nz = __popcll(P.zmask);
    if (!epi.active()) return;
    if (LAST) epi.init();
    __shared__ SegLds seg;
    stage_segment(seg, P, g);
    for (uint32_t ti = blockIdx.x; ti < ntiles; ti += gx) {
        const uint32_t t = g.rev ? ntiles - 1u - ti : ti;
        uint32_t xh = 0;
        for (int j = 0; j < hbits; ++j) xh |= ((t >> j) & 1u) << g.hsite[j];
        const uint32_t xb = xh | xy;
        double re[kR], im[kR];
        __syncthreads();  // the previous tile is no longer read
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const double2 o = ld_nt(&v[FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6)]);
            tile[yb + (e << kRegShift)] = o;
            if (FIRST) {
                re[e] = o.x;
                im[e] = o.y;
            } else {
                const double2 q = ld_nt(&part[FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6)]);
                re[e] = q.x;
                im[e] = q.y;
            }
        }
        if (FIRST) {
            // D(x) = K/4 s_z + J/4 s_all with s = (bonds) - 2 (antiparallel bonds), from
            // the bond-parity vector: tile-index part, thread part, register-element part
            uint64_t par = pxy;
            for (int j = 0; j < hbits; ++j)
                if ((t >> j) & 1u) par ^= P.smask[g.hsite[j]];
#pragma unroll
            for (int e = 0; e < kR; ++e) {
                uint64_t pe = par;
                if (e & 1) pe ^= pe6;
                if (e & 2) pe ^= pe7;
                if (e & 4) pe ^= pe8;
                const int s_all = P.n_bonds - 2 * __popcll(pe);
                const int s_z = nz - 2 * __popcll(pe & P.zmask);
                const double D = fma(P.kq, (double)s_z, P.jq * (double)s_all);
                re[e] = D * re[e];
                im[e] = D * im[e];
            }
        }
        __syncthreads();
        for (int b = g.b0; b < g.b1; ++b) {
            const uint32_t pq = seg.pq[b];
            const uint32_t pi = pq & 0xffu, pj = pq >> 8;
            const uint32_t tm = (1u << pi) | (1u << pj);
            const uint32_t mrest = tm & ~(7u << kRegShift);
            const int mr = (tm >> kRegShift) & 7;
            const bool anti = ((yb >> pi) ^ (yb >> pj)) & 1u;
            const double aa = seg.aa[b], ap = seg.ap[b];
            const double ampA = anti ? aa : ap;
            const double ampB = anti ? ap : aa;
            const uint32_t base = FTK_IDX(yb ^ mrest, 7u << kRegShift, kPassTile, 8) ^ ((uint32_t)mr << kRegShift);
            bond_accum_lds_flat(re, im, tile, base, (uint32_t)mr, ampA, ampB);
        }
        if (LAST) {
            double2 in[kR];
#pragma unroll
            for (int e = 0; e < kR; ++e) in[e] = epi.load(FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6));
#pragma unroll
            for (int e = 0; e < kR; ++e) epi.apply(FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6), re[e], im[e], tile[yb + (e << kRegShift)], in[e]);
        } else {
#pragma unroll
            for (int e = 0; e < kR; ++e) st_h<!SH>(&part[FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6)], make_double2(re[e], im[e]));
        }
    }
    if (LAST) epi.template finish<kPassThreads>();
}

// Lanczos, multi-pass form: the second half of step k-1 fused into the first
// pass of step k.  W holds u_{k-1} and receives w_{k-1} = u_{k-1} + c2 w_{k-2}
// (c2 = -(alpha_{k-1} inv_{k-1}), exactly as k_lanczos_b computes it) together
// with the partial sums of ||w_{k-1}||^2; the tile of w_{k-1} then goes through
// the first segment of bonds like any first pass.
template <bool SH>
__global__ void __launch_bounds__(kPassThreads, 4) k_hv_pass_fused(HvParams P, PassGeom g, double2 *__restrict__ W,
                                                                  const double2 *__restrict__ Wm2,
                                                                  double2 *__restrict__ part, SeqState *st,
                                                                  double *partials, size_t vs, FinAlpha fa,
                                                                  int use_fa)
{
    extern __shared__ double2 tile[];
    W += blockIdx.y * vs;
    Wm2 += blockIdx.y * vs;
    part += blockIdx.y * vs;
    st += blockIdx.y;
    partials += (size_t)blockIdx.y * 2 * gridDim.x;
    if (st->done) return;
    double a;
    if (use_fa) {
        // alpha_{k-1} = inv_{k-1} <v_{k-1}|u_{k-1}>, as k_finalize_alpha forms it, in every
        // workgroup; workgroup 0 records it
        __shared__ double s_a;
        const double d = reduce_partials<kPassThreads>(fa.partials + (size_t)blockIdx.y * 2 * fa.nparts, fa.nparts);
        if (threadIdx.x == 0) {
            s_a = st->inv_cur * d;
            if (blockIdx.x == 0) {
                if (!isfinite(s_a)) st->numeric_error = 1;
                st->alpha_cur = s_a;
                fa.alpha_out[(size_t)blockIdx.y * fa.astride + fa.k] = s_a;
            }
        }
        __syncthreads();
        a = s_a;
    } else {
        a = st->alpha_cur;
    }
    const double c2 = -(a * st->inv_cur);
    const int hbits = P.n_sites - kPassBits;
    const uint32_t ntiles = 1u << hbits;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t yb = FTK_IDX(lane | (wave << 9), 7u << kRegShift, kPassTile, 7);
    uint32_t xy = 0;
    uint64_t pxy = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if ((lane >> j) & 1u) xy |= 1u << g.ysite[j], pxy ^= P.smask[g.ysite[j]];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if ((wave >> j) & 1u) xy |= 1u << g.ysite[6 + j], pxy ^= P.smask[g.ysite[6 + j]];
    const uint64_t pe6 = P.smask[g.esite[0]], pe7 = P.smask[g.esite[1]], pe8 = P.smask[g.esite[2]];
    const int nz = __popcll(P.zmask);
    __shared__ SegLds seg;
    stage_segment(seg, P, g);
    double hi = 0.0, lo = 0.0, err = 0.0;
    for (uint32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
        const uint32_t t = g.rev ? ntiles - 1u - ti : ti;
        uint32_t xh = 0;
        uint64_t par = pxy;
        for (int j = 0; j < hbits; ++j)
            if ((t >> j) & 1u) xh |= 1u << g.hsite[j], par ^= P.smask[g.hsite[j]];
        const uint32_t xb = xh | xy;
        __syncthreads();
        // w_{k-1} to the tile (W, Wm2 and part are distinct buffers).  No global store
        // in this loop: on gfx950 loads and stores share one counter, so a store issued
        // between two elements' loads would make the second element wait for it.
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const double2 u = ld_h<SH>(&W[FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6)]);
            const double2 wp = ld_h<SH>(&Wm2[FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6)]);
            const double wr = fma(c2, wp.x, u.x);
            const double wi = fma(c2, wp.y, u.y);
            tile[yb + (e << kRegShift)] = make_double2(wr, wi);
            acc_prod(hi, lo, err, wr, wr);
            acc_prod(hi, lo, err, wi, wi);
        }
        // w_{k-1} to global memory and D w, from the thread's own tile entries
        double re[kR], im[kR];
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const double2 o = tile[yb + (e << kRegShift)];
            st_h<SH>(&W[FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6)], o);
            uint64_t pe = par;
            if (e & 1) pe ^= pe6;
            if (e & 2) pe ^= pe7;
            if (e & 4) pe ^= pe8;
            const int s_all = P.n_bonds - 2 * __popcll(pe);
            const int s_z = nz - 2 * __popcll(pe & P.zmask);
            const double D = fma(P.kq, (double)s_z, P.jq * (double)s_all);
            re[e] = D * o.x;
            im[e] = D * o.y;
        }
        __syncthreads();
        for (int b = g.b0; b < g.b1; ++b) {
            const uint32_t pq = seg.pq[b];
            const uint32_t pi = pq & 0xffu, pj = pq >> 8;
            const uint32_t tm = (1u << pi) | (1u << pj);
            const uint32_t mrest = tm & ~(7u << kRegShift);
            const int mr = (tm >> kRegShift) & 7;
            const bool anti = ((yb >> pi) ^ (yb >> pj)) & 1u;
            const double aa = seg.aa[b], ap = seg.ap[b];
            const double ampA = anti ? aa : ap;
            const double ampB = anti ? ap : aa;
            const uint32_t base = FTK_IDX(yb ^ mrest, 7u << kRegShift, kPassTile, 8) ^ ((uint32_t)mr << kRegShift);
            bond_accum_lds_flat(re, im, tile, base, (uint32_t)mr, ampA, ampB);
        }
#pragma unroll
        for (int e = 0; e < kR; ++e) part[FTK_IDX(xb | g.ebit[e], 0, 1u << P.n_sites, 6)] = make_double2(re[e], im[e]);
    }
    write_partial<kPassThreads>(partials, hi, lo, err);
}

// passes p0..n_passes-1 of the multi-pass form (the first of them starts from
// D v only when p0 = 0; the last hands its sums to the epilogue)
template <class Epi, bool SH>
static void launch_passes_h(const HvOp &op, int p0, const double *v, Epi epi, hipStream_t s, int B, double *scratch,
                            size_t vs, int fin_pass)
{
    // a pass that reduces partial sums runs as persistent workgroups (hv_grid: fewer
    // partials); every other pass gets one workgroup per 4096-element tile, which
    // streams faster
    const dim3 grid_red(hv_grid(op, B), B);
    const dim3 grid_full((1u << op.P.n_sites) / kPassTile, B);
    const int np = op.plan.n_passes;
    const size_t lds = kPassTile * sizeof(double2);
    double2 *part = (double2 *)(scratch ? scratch : op.scratch);
    const size_t vs2 = vs / 2;  // in complex entries
    for (int p = p0; p < np; ++p) {
        PassGeom g = op.plan.pass[p];
        g.rev = SH && p == 0;
        const bool first = p == 0, last = p == np - 1;
        dim3 grid = (last && Epi::kReduces) || !g_full_grid ? grid_red : grid_full;
        Epi ep = epi;
        if constexpr (Epi::kReduces) {
            // a middle pass can carry the beta finalisation as one more column
            ep.fin = (p == fin_pass && !first && !last) ? 1 : 0;
            if (ep.fin) grid.x += 1;
        }
        if (first && last)
            hipLaunchKernelGGL((k_hv_pass<Epi, true, true, SH>), grid, dim3(kPassThreads), lds, s, op.P, g,
                               (const double2 *)v, part, ep, vs2);
        else if (first)
            hipLaunchKernelGGL((k_hv_pass<Epi, true, false, SH>), grid, dim3(kPassThreads), lds, s, op.P, g,
                               (const double2 *)v, part, ep, vs2);
        else if (last)
            hipLaunchKernelGGL((k_hv_pass<Epi, false, true, SH>), grid, dim3(kPassThreads), lds, s, op.P, g,
                               (const double2 *)v, part, ep, vs2);
        else
            hipLaunchKernelGGL((k_hv_pass<Epi, false, false, SH>), grid, dim3(kPassThreads), lds, s, op.P, g,
                               (const double2 *)v, part, ep, vs2);
    }
}

template <class Epi>
static void launch_passes(const HvOp &op, int p0, const double *v, Epi epi, hipStream_t s, int B = 1,
                          double *scratch = nullptr, size_t vs = 0, int fin_pass = -1)
{
    if (stream_hints(op, B))
        launch_passes_h<Epi, true>(op, p0, v, epi, s, B, scratch, vs, fin_pass);
    else
        launch_passes_h<Epi, false>(op, p0, v, epi, s, B, scratch, vs, fin_pass);
}

template <class Epi>
void launch_hv(const HvOp &op, const double *v, Epi epi, hipStream_t s)
{
    const HvParams &P = op.P;
    const int grid = hv_grid(op);
    switch (hv_mode(op)) {
    case 3:
        launch_passes(op, 0, v, epi, s);
        break;
    case 2:
        hipLaunchKernelGGL(k_hv_tiled<Epi>, dim3(grid), dim3(kTileThreads), kTile * sizeof(double2), s, P,
                           (const double2 *)v, epi);
        break;
    case 1:
        hipLaunchKernelGGL(k_hv_blocked<Epi>, dim3(grid), dim3(kBlock), 0, s, P, (const double2 *)v, epi);
        break;
    default:
        hipLaunchKernelGGL(k_hv_simple<Epi>, dim3(grid), dim3(kBlock), 0, s, P, (const double2 *)v, epi);
    }
}

void launch_apply_h(const HvOp &op, const double *v, double *w, hipStream_t s)
{
    EpiApply e;
    e.w = (double2 *)w;
    launch_hv(op, v, e, s);
}

// ---------------------------------------------------------------------------
// Lanczos step (Sec. II.B basis) with unnormalised residuals w_k = beta_{k+1} v_{k+1}:
//   u = (H w_{k-1}) inv_k + c1 w_{k-2}, c1 = (-beta_k) inv_{k-1};  alpha_k = inv_k <w_{k-1}|u>;
//   w_k = u + c2 w_{k-1}, c2 = -(alpha_k inv_k);  beta_{k+1} = ||w_k||;  inv_{k+1} = 1/beta_{k+1}.
// The H-applying first half needs inv_k and c1 as values; they live on the device,
// so the epilogue reads them through a pointer set at launch.
template <int BLOCK>
__device__ void finalize_beta_seq(const FinBeta &f, int r);

struct EpiLanczosADev {
    static constexpr bool kReduces = true;  // the last pass writes partial sums of <v|u>
    const double2 *Wprev;
    double2 *U;
    double2 *vout;
    double *partials;
    const SeqState *st;
    int first;
    int fin;     // a middle pass also finalises beta of the previous half step (extra column)
    FinBeta fb;
    double inv, c1, hi, lo, err;
    __device__ void finalize_block(int r) const { finalize_beta_seq<kPassThreads>(fb, r); }
    // sequence r of a stacked batch: vectors vs entries apart, pstride partial doubles apart
    __device__ void select(int r, size_t vs, int pstride)
    {
        Wprev += r * vs;
        U += r * vs;
        if (vout) vout += r * vs;
        st += r;
        partials += (size_t)r * pstride;
    }
    __device__ bool active() const { return !st->done; }
    __device__ void init()
    {
        inv = st->inv_cur;
        c1 = (-st->beta_cur) * st->inv_prev;
        hi = lo = err = 0.0;
    }
    __device__ double2 load(size_t x) const { return first ? make_double2(0.0, 0.0) : Wprev[x]; }
    __device__ void apply(size_t x, double re, double im, const double2 &wc, const double2 &wp)
    {
        double ur = re * inv, ui = im * inv;
        if (!first) {
            ur = fma(c1, wp.x, ur);
            ui = fma(c1, wp.y, ui);
        }
        U[x] = make_double2(ur, ui);
        if (vout) vout[x] = wc;
        acc_prod(hi, lo, err, wc.x, ur);
        acc_prod(hi, lo, err, wc.y, ui);
    }
    __device__ void operator()(size_t x, double re, double im, const double2 &wc) { apply(x, re, im, wc, load(x)); }
    template <int BLOCK>
    __device__ void finish() { write_partial<BLOCK>(partials, hi, lo, err); }
};

void launch_lanczos_a(const HvOp &op, const double *Wcur, const double *Wprev, double *U,
                      double *vout, SeqState *st, double *partials, int first_step, hipStream_t s,
                      const Stack &sk)
{
    EpiLanczosADev e;
    e.Wprev = (const double2 *)Wprev;
    e.U = (double2 *)U;
    e.vout = (double2 *)vout;
    e.partials = partials;
    e.st = st;
    e.first = first_step;
    e.fin = 0;
    if (sk.B > 1 || sk.scratch)
        launch_passes(op, 0, Wcur, e, s, sk.B, sk.scratch, sk.vs);
    else
        launch_hv(op, Wcur, e, s);
}

bool lanczos_fusable(const HvOp &op) { return hv_mode(op) == 3 && op.plan.n_passes >= 2; }
bool lanczos_stackable(const HvOp &op) { return op.plan.n_passes >= 2 && op.scratch != nullptr; }

void launch_lanczos_fused_first(const HvOp &op, double *W, const double *Wm2, SeqState *st, double *partials,
                                hipStream_t s, const Stack &sk, const FinAlpha *fa)
{
    double *part = sk.scratch ? sk.scratch : op.scratch;
    const FinAlpha f = fa ? *fa : FinAlpha{nullptr, 0, nullptr, 0, 0};
    PassGeom g = op.plan.pass[0];
    const bool sh = stream_hints(op, sk.B);
    g.rev = sh;
    const dim3 grid(hv_grid(op, sk.B), sk.B);
    if (sh)
        hipLaunchKernelGGL(k_hv_pass_fused<true>, grid, dim3(kPassThreads), kPassTile * sizeof(double2), s, op.P, g,
                           (double2 *)W, (const double2 *)Wm2, (double2 *)part, st, partials, sk.vs / 2, f, fa ? 1 : 0);
    else
        hipLaunchKernelGGL(k_hv_pass_fused<false>, grid, dim3(kPassThreads), kPassTile * sizeof(double2), s, op.P, g,
                           (double2 *)W, (const double2 *)Wm2, (double2 *)part, st, partials, sk.vs / 2, f, fa ? 1 : 0);
}

bool alpha_in_fused_pass() { return g_fuse_fin; }

bool beta_in_middle_pass(const HvOp &op) { return g_fuse_fin && op.plan.n_passes >= 3; }

void launch_lanczos_a_rest(const HvOp &op, const double *Wcur, const double *Wprev, double *U, double *vout,
                           SeqState *st, double *partials, hipStream_t s, const Stack &sk, const FinBeta *fb)
{
    EpiLanczosADev e;
    e.Wprev = (const double2 *)Wprev;
    e.U = (double2 *)U;
    e.vout = (double2 *)vout;
    e.partials = partials;
    e.st = st;
    e.first = 0;
    e.fin = 0;
    if (fb) e.fb = *fb;
    launch_passes(op, 1, Wcur, e, s, sk.B, sk.scratch, sk.vs, fb ? 1 : -1);
}

__global__ void __launch_bounds__(kBlock) k_lanczos_b(uint32_t dim, const double2 *__restrict__ Wcur,
                                                      double2 *__restrict__ U, SeqState *st,
                                                      double *partials, size_t vs)
{
    Wcur += blockIdx.y * vs;
    U += blockIdx.y * vs;
    st += blockIdx.y;
    partials += (size_t)blockIdx.y * 2 * gridDim.x;
    if (st->done) return;
    const double c2 = -(st->alpha_cur * st->inv_cur);
    double hi = 0.0, lo = 0.0, err = 0.0;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 wc = Wcur[x];
        const double2 u = U[x];
        const double wr = fma(c2, wc.x, u.x);
        const double wi = fma(c2, wc.y, u.y);
        U[x] = make_double2(wr, wi);
        acc_prod(hi, lo, err, wr, wr);
        acc_prod(hi, lo, err, wi, wi);
    }
    write_partial<kBlock>(partials, hi, lo, err);
}

__global__ void __launch_bounds__(kBlock) k_finalize_alpha(SeqState *st, const double *partials,
                                                           int nparts, double *alpha_out, int k, int astride)
{
    // sequence blockIdx.x of a stacked batch
    st += blockIdx.x;
    partials += (size_t)blockIdx.x * 2 * nparts;
    alpha_out += (size_t)blockIdx.x * astride;
    if (st->done) return;
    const double d = reduce_partials(partials, nparts);
    if (threadIdx.x == 0) {
        const double a = st->inv_cur * d;
        if (!isfinite(a)) st->numeric_error = 1;
        st->alpha_cur = a;
        alpha_out[k] = a;
    }
}

// One step of the forward LDL^T recurrence of (z - T)^{-1}_{00} for the shift z = zr + i zi
// (App. A.3): d_k, the running product p_k and the accumulated G; alpha = alpha_k,
// bk = beta_k.
__device__ __forceinline__ void shift_update(ShiftState &q, double zr, double zi, double alpha, double bk, int k)
{
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
}

// maximum over a block of BLOCK threads; valid in thread 0
template <int BLOCK>
__device__ __forceinline__ double block_max(double v)
{
    __shared__ double sh[BLOCK / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < BLOCK / 64; ++i) m = sh[i] > m ? sh[i] : m;
    return m;
}

// beta_{k+1} = ||w_k|| from the partial sums, the forward LDL^T recurrence of
// (z - T)^{-1}_{00} per shift z = omega + shift_re + i eta, and the stopping test,
// for sequence r, by one block of BLOCK threads.
template <int BLOCK>
__device__ void finalize_beta_seq(const FinBeta &f, int r)
{
    SeqState *st = f.st + r;
    const double *partials = f.partials + (size_t)r * 2 * f.nparts;
    double *beta_out = f.beta_out + (size_t)r * f.bstride;
    ShiftState *sh = f.sh ? f.sh + (size_t)r * f.n_omega : nullptr;
    const int k = f.k;
    if (st->done) return;
    __shared__ double s_bn;
    const double ssum = reduce_partials<BLOCK>(partials, f.nparts);
    if (threadIdx.x == 0) s_bn = sqrt(ssum);
    const double alpha = st->alpha_cur, bk = st->beta_cur, zoff = st->shift_re;
    __syncthreads();
    const double bn = s_bn;
    double rmax = 0.0;
    for (int j = threadIdx.x; j < f.n_omega; j += BLOCK) {
        const double zr = f.omega[j] + zoff, zi = f.eta;
        ShiftState q = sh[j];
        shift_update(q, zr, zi, alpha, bk, k);
        sh[j] = q;
        // residual after k+1 steps: |p_k| beta_{k+1} / |d_k|
        const double rs = sqrt((q.pr * q.pr + q.pi * q.pi) / (q.dr * q.dr + q.di * q.di)) * bn;
        rmax = rs > rmax ? rs : rmax;
    }
    const double m = block_max<BLOCK>(rmax);
    if (threadIdx.x == 0) {
        st->max_resid = m * st->norm;
        beta_out[k] = bn;
        st->steps = k + 1;
        if (!isfinite(bn)) st->numeric_error = 1;
        if (!(bn > f.tol) || (f.rtol > 0.0 && m <= f.rtol)) {
            st->done = 1;  // invariant subspace, or every shift converged
        } else {
            st->inv_prev = st->inv_cur;
            st->inv_cur = 1.0 / bn;
            st->beta_cur = bn;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_finalize_beta(FinBeta f) { finalize_beta_seq<kBlock>(f, blockIdx.x); }

__global__ void k_finish_green(const SeqState *st, const ShiftState *sh, int n_omega, double2 *g)
{
    const double n2 = st->norm2;
    const bool any = st->steps > 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_omega; j += gridDim.x * blockDim.x) {
        const ShiftState q = sh[j];
        g[j] = any ? make_double2(n2 * q.gr, n2 * q.gi) : make_double2(0.0, 0.0);
    }
}

void launch_finalize_alpha(SeqState *st, const double *partials, int nparts, double *alpha_out,
                           int k, hipStream_t s, int B, int astride)
{
    hipLaunchKernelGGL(k_finalize_alpha, dim3(B), dim3(kBlock), 0, s, st, partials, nparts, alpha_out, k, astride);
}

void launch_lanczos_b(uint32_t dim, const double *Wcur, double *U, SeqState *st,
                      double *partials, hipStream_t s, int B, size_t vs)
{
    hipLaunchKernelGGL(k_lanczos_b, dim3(vec_grid(dim), B), dim3(kBlock), 0, s, dim, (const double2 *)Wcur,
                       (double2 *)U, st, partials, vs / 2);
}

void launch_finalize_beta(SeqState *st, const double *partials, int nparts, double *beta_out,
                          int k, double tol, ShiftState *shifts, const double *omega, int n_omega,
                          double eta, hipStream_t s, double rtol, int B, int bstride)
{
    const FinBeta f{st, partials, nparts, beta_out, k, tol, shifts, omega, n_omega, eta, rtol, bstride};
    hipLaunchKernelGGL(k_finalize_beta, dim3(B), dim3(kBlock), 0, s, f);
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
                                                const double2 *__restrict__ b, double *partials, size_t vs)
{
    a += blockIdx.y * vs;
    b += blockIdx.y * vs;
    partials += (size_t)blockIdx.y * 2 * gridDim.x;
    double hi = 0.0, lo = 0.0, err = 0.0;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 u = a[x], v = b[x];
        acc_prod(hi, lo, err, u.x, v.x);
        acc_prod(hi, lo, err, u.y, v.y);
    }
    write_partial<kBlock>(partials, hi, lo, err);
}

__global__ void __launch_bounds__(kBlock) k_start_sequence(SeqState *st, const double *partials,
                                                           int nparts, BatchShifts shifts)
{
    st += blockIdx.x;
    partials += (size_t)blockIdx.x * 2 * nparts;
    const double shift_re = shifts.re[blockIdx.x];
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

void launch_dot(uint32_t dim, const double *a, const double *b, double *partials, hipStream_t s, int B, size_t vs)
{
    hipLaunchKernelGGL(k_dot, dim3(vec_grid(dim), B), dim3(kBlock), 0, s, dim, (const double2 *)a,
                       (const double2 *)b, partials, vs / 2);
}

void launch_start_sequence(SeqState *st, const double *partials, int nparts, double shift_re,
                           hipStream_t s)
{
    BatchShifts sh;
    sh.re[0] = shift_re;
    hipLaunchKernelGGL(k_start_sequence, dim3(1), dim3(kBlock), 0, s, st, partials, nparts, sh);
}

void launch_start_stacked(int B, uint32_t dim, const double *chi, double *partials, SeqState *st,
                          const BatchShifts &shifts, hipStream_t s)
{
    launch_dot(dim, chi, chi, partials, s, B, 2 * (size_t)dim);
    hipLaunchKernelGGL(k_start_sequence, dim3(B), dim3(kBlock), 0, s, st, partials, vec_grid(dim), shifts);
}

void launch_sum_partials(const double *partials, int nparts, double *result, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partials, nparts, result);
}

// ---------------------------------------------------------------------------
// chi = S^alpha_{+Q} phi (Sec. V): x and y flip one spin, z is diagonal.
// <down|S^y|up> = +i/2 and <up|S^y|down> = -i/2 (bit 1 = spin down).  h holds
// the per-site factors (interleaved), the 1/2 of S = sigma/2 included.
template <class Coef>
__device__ __forceinline__ double2 sq_part(int n_sites, int alpha, const Coef &h, const double2 *__restrict__ phi,
                                           uint32_t x)
{
    double re = 0.0, im = 0.0;
    if (alpha == 2) {
        double cr = 0.0, ci = 0.0;
        for (int l = 0; l < n_sites; ++l) {
            if ((x >> l) & 1u) {
                cr = cr - h[2 * l];
                ci = ci - h[2 * l + 1];
            } else {
                cr = cr + h[2 * l];
                ci = ci + h[2 * l + 1];
            }
        }
        const double2 p = phi[x];
        re = cr * p.x - ci * p.y;
        im = cr * p.y + ci * p.x;
    } else {
        for (int l = 0; l < n_sites; ++l) {
            double cr = h[2 * l], ci = h[2 * l + 1];
            if (alpha == 1) {
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
            const double2 p = phi[FTK_IDX(x ^ (1u << l), 0, 1u << n_sites, 12)];
            const double tr = cr * p.x - ci * p.y;
            const double ti = cr * p.y + ci * p.x;
            re = re + tr;
            im = im + ti;
        }
    }
    return make_double2(re, im);
}

__global__ void __launch_bounds__(kBlock) k_apply_sq(SqParams P, const double2 *__restrict__ phi,
                                                     double2 *__restrict__ chi, int stride, int offset)
{
    const uint32_t dim = 1u << P.n_sites;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x)
        chi[(size_t)x * stride + offset] = sq_part(P.n_sites, P.alpha, P.h, phi, x);
}

void launch_apply_sq(const SqParams &P, const double *phi, double *chi, hipStream_t s, int stride, int offset)
{
    const uint32_t dim = 1u << P.n_sites;
    hipLaunchKernelGGL(k_apply_sq, dim3(vec_grid(dim)), dim3(kBlock), 0, s, P, (const double2 *)phi,
                       (double2 *)chi, stride, offset);
}

// chi = A phi for a linear spin operator (operators A, B of Sec. III.B): the three
// components formed as above, added per element in the order (x + y) + z.
__global__ void __launch_bounds__(kBlock) k_apply_spin_op(SpinOpParams P, const double2 *__restrict__ phi,
                                                          double2 *__restrict__ chi)
{
    const uint32_t dim = 1u << P.n_sites;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 a = sq_part(P.n_sites, 0, P.h[0], phi, x);
        const double2 b = sq_part(P.n_sites, 1, P.h[1], phi, x);
        const double2 c = sq_part(P.n_sites, 2, P.h[2], phi, x);
        chi[x] = make_double2((a.x + b.x) + c.x, (a.y + b.y) + c.y);
    }
}

void launch_apply_spin_op(const SpinOpParams &P, const double *phi, double *chi, hipStream_t s)
{
    const uint32_t dim = 1u << P.n_sites;
    hipLaunchKernelGGL(k_apply_spin_op, dim3(vec_grid(dim)), dim3(kBlock), 0, s, P, (const double2 *)phi,
                       (double2 *)chi);
}

// the start vectors of the polarization identity: lam + rho, lam - rho, lam + i rho,
// lam - i rho for k = 0..3
__global__ void __launch_bounds__(kBlock) k_polarize(uint32_t dim, int k, const double2 *__restrict__ lam,
                                                     const double2 *__restrict__ rho, double2 *__restrict__ chi,
                                                     int stride, int offset)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += gridDim.x * blockDim.x) {
        const double2 a = lam[x], b = rho[x];
        double2 o;
        if (k == 0)
            o = make_double2(a.x + b.x, a.y + b.y);
        else if (k == 1)
            o = make_double2(a.x - b.x, a.y - b.y);
        else if (k == 2)
            o = make_double2(a.x - b.y, a.y + b.x);
        else
            o = make_double2(a.x + b.y, a.y - b.x);
        chi[(size_t)x * stride + offset] = o;
    }
}

void launch_polarize(uint32_t dim, int k, const double *lam, const double *rho, double *chi, hipStream_t s,
                     int stride, int offset)
{
    hipLaunchKernelGGL(k_polarize, dim3(vec_grid(dim)), dim3(kBlock), 0, s, dim, k, (const double2 *)lam,
                       (const double2 *)rho, (double2 *)chi, stride, offset);
}

// ---------------------------------------------------------------------------
// One term of the imaginary-time Taylor series (Appendix A).
void launch_taylor_term(const HvOp &op, const double *t, double *tn, double *acc, double a,
                        double b, hipStream_t s)
{
    EpiTaylor e;
    e.tn = (double2 *)tn;
    e.acc = (double2 *)acc;
    e.a = a;
    e.b = b;
    launch_hv(op, t, e, s);
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
// Filter pass 2 (Sec. III.B, Eq. filtered): Phi_m += sum_k d_{m,k} W_k over a
// buffered block of Lanczos residual vectors, k in increasing order, 8 shells
// per thread.  Each workgroup takes one group of 8 shells over a strided set of
// element ranges; the ny shell groups of one element range are consecutive
// workgroups of one XCD (workgroups are dealt to the 8 XCDs round-robin by linear
// index: id = xcd + 8 (group + ny q), element block xcd + 8 q), so they read the
// range's vectors at about the same time and all but the first read come from
// that XCD's L2 instead of HBM.  A full group of 8 shells has no per-shell test,
// so the eight scalar coefficient loads of a step are issued together (measured:
// 42.6 -> 34.5 ms for 64 vectors into 128 shells at 24 sites; staging the vectors
// in LDS for 16 shell groups per workgroup read each entry from HBM once but took
// 70 ms: 128 coefficient rows in flight per workgroup overran the scalar cache).
constexpr int kShellTile = 8;

__global__ void __launch_bounds__(kBlock) k_accumulate(uint32_t dim, const double2 *__restrict__ V, int nk,
                                                       const double2 *__restrict__ coef, int n, int k0,
                                                       double2 *__restrict__ Phi, int L, int gx, int ny)
{
    const uint32_t r = blockIdx.x >> 3;
    const int m0 = (int)(r % (uint32_t)ny) * kShellTile;
    const uint32_t xblock = (blockIdx.x & 7u) + 8u * (r / (uint32_t)ny);
    const int mc = L - m0 < kShellTile ? L - m0 : kShellTile;
    const double2 *cf = coef + k0;
    for (uint32_t x = xblock * blockDim.x + threadIdx.x; x < dim; x += (uint32_t)gx * blockDim.x) {
        double2 acc[kShellTile];
#pragma unroll
        for (int mm = 0; mm < kShellTile; ++mm)
            if (mm < mc) acc[mm] = Phi[(size_t)(m0 + mm) * dim + x];
        if (mc == kShellTile) {
            for (int k = 0; k < nk; ++k) {
                const double2 v = V[(size_t)k * dim + x];
                double2 c[kShellTile];
#pragma unroll
                for (int mm = 0; mm < kShellTile; ++mm) c[mm] = cf[FTK_IDX((m0 + mm) * n + k, 0, L * n, 13)];
#pragma unroll
                for (int mm = 0; mm < kShellTile; ++mm) {
                    double re = acc[mm].x, im = acc[mm].y;
                    re = fma(c[mm].x, v.x, re);
                    re = fma(-c[mm].y, v.y, re);
                    im = fma(c[mm].x, v.y, im);
                    im = fma(c[mm].y, v.x, im);
                    acc[mm] = make_double2(re, im);
                }
            }
        } else {
            for (int k = 0; k < nk; ++k) {
                const double2 v = V[(size_t)k * dim + x];
#pragma unroll
                for (int mm = 0; mm < kShellTile; ++mm) {
                    if (mm < mc) {
                        const double2 c = cf[FTK_IDX((m0 + mm) * n + k, 0, L * n, 13)];
                        double re = acc[mm].x, im = acc[mm].y;
                        re = fma(c.x, v.x, re);
                        re = fma(-c.y, v.y, re);
                        im = fma(c.x, v.y, im);
                        im = fma(c.y, v.x, im);
                        acc[mm] = make_double2(re, im);
                    }
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
    const int gx = (vec_grid(dim) + 7) / 8 * 8;  // element blocks, a multiple of the 8 XCDs
    const int ny = (L + kShellTile - 1) / kShellTile;
    hipLaunchKernelGGL(k_accumulate, dim3(gx * ny), dim3(kBlock), 0, s, dim, (const double2 *)V, nk,
                       (const double2 *)coef, n, k0, (double2 *)Phi, L, gx, ny);
}


// ===========================================================================
// Batched Krylov sequences: B right-hand sides in block layout, entry (x, r) at
// x * B + r.  A wave covers 64/B consecutive elements of all B sequences, so
// every gather instruction again reads 1 KB of consecutive memory; each thread
// owns one sequence r and 8 elements 64/B apart.  Per-sequence arithmetic is
// exactly that of a single sequence (same operations, exact-sum reductions per
// sequence), so results do not depend on B or on the batch composition.

template <int B>
struct BatchGeom {
    static constexpr int EL = 64 / B;                                  // element lanes per wave
    static constexpr int RS = EL == 32 ? 5 : EL == 16 ? 4 : EL == 8 ? 3 : EL == 4 ? 2 : EL == 2 ? 1 : 0;
    static constexpr int CHUNK = EL * kR;                              // elements per wave
};

// per-sequence (hi, lo) sums of a block: lanes with equal lane % B combine, then
// waves in order; partials[(block * B + r) * 2 + {0, 1}]
template <int B, int BLOCK>
__device__ __forceinline__ void write_partial_batch(double *partials, double hi, double lo, double err)
{
    __shared__ double sh[BLOCK / 64][B][2];
    dd_add(hi, lo, err);
#pragma unroll
    for (int off = 32; off >= B; off >>= 1) {
        double oh = __shfl_xor(hi, off, 64);
        double ol = __shfl_xor(lo, off, 64);
        dd_add_dd(hi, lo, oh, ol);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < B) {
        sh[wave][lane][0] = hi;
        sh[wave][lane][1] = lo;
    }
    __syncthreads();
    if (threadIdx.x < B) {
        double h = sh[0][threadIdx.x][0], l = sh[0][threadIdx.x][1];
        for (int w = 1; w < BLOCK / 64; ++w) dd_add_dd(h, l, sh[w][threadIdx.x][0], sh[w][threadIdx.x][1]);
        partials[2 * (blockIdx.x * B + threadIdx.x)] = h;
        partials[2 * (blockIdx.x * B + threadIdx.x) + 1] = l;
    }
}

// sum over blocks of sequence r's partials (stride B), rounded; thread 0 of a kBlock block
__device__ __forceinline__ double reduce_partials_strided(const double *partials, int nparts, int B, int r)
{
    double hi = 0.0, lo = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x)
        dd_add_dd(hi, lo, partials[2 * (i * B + r)], partials[2 * (i * B + r) + 1]);
    block_reduce_dd<kBlock>(hi, lo);
    return hi + lo;
}

template <int B>
struct EpiLanczosABatch {
    const double2 *Wprev;
    double2 *U;
    double *partials;
    const SeqState *st;  // [B]
    int first;
    double inv, c1, hi, lo, err;
    int done;
    __device__ bool active() const { return true; }
    __device__ void init(int r)
    {
        inv = st[r].inv_cur;
        c1 = (-st[r].beta_cur) * st[r].inv_prev;
        done = st[r].done;
        hi = lo = err = 0.0;
    }
    __device__ double2 load(size_t idx) const { return (first || done) ? make_double2(0.0, 0.0) : Wprev[idx]; }
    __device__ void apply(size_t idx, double re, double im, const double2 &wc, const double2 &wp)
    {
        if (done) return;
        double ur = re * inv, ui = im * inv;
        if (!first) {
            ur = fma(c1, wp.x, ur);
            ui = fma(c1, wp.y, ui);
        }
        U[idx] = make_double2(ur, ui);
        acc_prod(hi, lo, err, wc.x, ur);
        acc_prod(hi, lo, err, wc.y, ui);
    }
    template <int BLOCK>
    __device__ void finish() { write_partial_batch<B, BLOCK>(partials, hi, lo, err); }
};

template <int B, class Epi>
__global__ void __launch_bounds__(kBlock) k_hv_batch(HvParams P, const double2 *__restrict__ v, Epi epi)
{
    using G = BatchGeom<B>;
    const uint32_t dim = 1u << P.n_sites;
    const uint32_t lane = threadIdx.x & 63;
    const int r = lane % B;
    const uint32_t el = lane / B;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    epi.init(r);
    for (uint32_t c = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); c < dim / G::CHUNK; c += waves) {
        const uint32_t xb = FTK_IDX(c * G::CHUNK + el, 7u << G::RS, dim, 10);
        double D[kR], re[kR], im[kR];
        diag_block<G::RS>(P, xb, D);
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const double2 o = v[(size_t)(xb + (e << G::RS)) * B + r];
            re[e] = D[e] * o.x;
            im[e] = D[e] * o.y;
        }
        for (int b = 0; b < P.n_bonds; ++b) {
            const uint32_t m = P.mask[b];
            const uint32_t mrest = m & ~(7u << G::RS);
            const int mr = (m >> G::RS) & 7;
            const bool anti = ((xb >> P.bi[b]) ^ (xb >> P.bj[b])) & 1u;
            const double ampA = anti ? P.aa[b] : P.ap[b];
            const double ampB = anti ? P.ap[b] : P.aa[b];
            double2 pv[kR];
            const double2 *src = v + (size_t)FTK_IDX(xb ^ mrest, 7u << G::RS, dim, 11) * B + r;
#pragma unroll
            for (int e = 0; e < kR; ++e) pv[e] = src[(size_t)(e << G::RS) * B];
            FTK_SWITCH_MR(mr, bond_accum, re, im, pv, ampA, ampB);
        }
        double2 in[kR];
#pragma unroll
        for (int e = 0; e < kR; ++e) in[e] = epi.load((size_t)(xb + (e << G::RS)) * B + r);
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const size_t idx = (size_t)(xb + (e << G::RS)) * B + r;
            epi.apply(idx, re[e], im[e], v[idx], in[e]);
        }
    }
    epi.template finish<kBlock>();
}

int hv_batch_grid(uint32_t dim, int B)
{
    const uint32_t chunk = (64 / B) * kR;
    uint32_t g = dim / (chunk * (kBlock / 64));
    return (int)(g < 1 ? 1 : (g < (uint32_t)kMaxGrid ? g : (uint32_t)kMaxGrid));
}

int vec_batch_grid(uint32_t dim, int B)
{
    const uint64_t n = (uint64_t)dim * B;
    uint64_t g = (n + kBlock - 1) / kBlock;
    return (int)(g < (uint64_t)kMaxGrid ? g : (uint64_t)kMaxGrid);
}

template <int B>
static void launch_lanczos_a_batch_t(const HvParams &P, const double *Wcur, const double *Wprev, double *U,
                                     SeqState *st, double *partials, int first, hipStream_t s)
{
    EpiLanczosABatch<B> e;
    e.Wprev = (const double2 *)Wprev;
    e.U = (double2 *)U;
    e.partials = partials;
    e.st = st;
    e.first = first;
    const uint32_t dim = 1u << P.n_sites;
    hipLaunchKernelGGL((k_hv_batch<B, EpiLanczosABatch<B>>), dim3(hv_batch_grid(dim, B)), dim3(kBlock), 0, s, P,
                       (const double2 *)Wcur, e);
}

void launch_lanczos_a_batch(int B, const HvParams &P, const double *Wcur, const double *Wprev, double *U,
                            SeqState *st, double *partials, int first, hipStream_t s)
{
    switch (B) {
    case 2: launch_lanczos_a_batch_t<2>(P, Wcur, Wprev, U, st, partials, first, s); break;
    case 4: launch_lanczos_a_batch_t<4>(P, Wcur, Wprev, U, st, partials, first, s); break;
    case 8: launch_lanczos_a_batch_t<8>(P, Wcur, Wprev, U, st, partials, first, s); break;
    case 16: launch_lanczos_a_batch_t<16>(P, Wcur, Wprev, U, st, partials, first, s); break;
    default: break;
    }
}

template <int B>
__global__ void __launch_bounds__(kBlock) k_lanczos_b_batch(uint32_t dim, const double2 *__restrict__ Wcur,
                                                            double2 *__restrict__ U, const SeqState *st,
                                                            double *partials)
{
    const int r = threadIdx.x % B;  // kBlock and the grid stride are multiples of B
    const int done = st[r].done;
    const double c2 = -(st[r].alpha_cur * st[r].inv_cur);
    double hi = 0.0, lo = 0.0, err = 0.0;
    const size_t n = (size_t)dim * B;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        if (done) continue;
        const double2 wc = Wcur[idx];
        const double2 u = U[idx];
        const double wr = fma(c2, wc.x, u.x);
        const double wi = fma(c2, wc.y, u.y);
        U[idx] = make_double2(wr, wi);
        acc_prod(hi, lo, err, wr, wr);
        acc_prod(hi, lo, err, wi, wi);
    }
    write_partial_batch<B, kBlock>(partials, hi, lo, err);
}

void launch_lanczos_b_batch(int B, uint32_t dim, const double *Wcur, double *U, SeqState *st, double *partials,
                            hipStream_t s)
{
    const dim3 g(vec_batch_grid(dim, B)), t(kBlock);
    switch (B) {
    case 2: hipLaunchKernelGGL(k_lanczos_b_batch<2>, g, t, 0, s, dim, (const double2 *)Wcur, (double2 *)U, st, partials); break;
    case 4: hipLaunchKernelGGL(k_lanczos_b_batch<4>, g, t, 0, s, dim, (const double2 *)Wcur, (double2 *)U, st, partials); break;
    case 8: hipLaunchKernelGGL(k_lanczos_b_batch<8>, g, t, 0, s, dim, (const double2 *)Wcur, (double2 *)U, st, partials); break;
    case 16: hipLaunchKernelGGL(k_lanczos_b_batch<16>, g, t, 0, s, dim, (const double2 *)Wcur, (double2 *)U, st, partials); break;
    default: break;
    }
}

__global__ void __launch_bounds__(kBlock) k_finalize_alpha_batch(SeqState *st, const double *partials, int nparts,
                                                                 int B, double *alpha_out, int n_max, int k)
{
    const int r = blockIdx.x;
    if (st[r].done) return;
    const double d = reduce_partials_strided(partials, nparts, B, r);
    if (threadIdx.x == 0) {
        const double a = st[r].inv_cur * d;
        if (!isfinite(a)) st[r].numeric_error = 1;
        st[r].alpha_cur = a;
        alpha_out[(size_t)r * n_max + k] = a;
    }
}

void launch_finalize_alpha_batch(int B, SeqState *st, const double *partials, int nparts, double *alpha_out,
                                 int n_max, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_alpha_batch, dim3(B), dim3(kBlock), 0, s, st, partials, nparts, B, alpha_out,
                       n_max, k);
}

// per sequence r: beta_{k+1}, inverse, breakdown, the multi-shift update (shifts [B][n_omega])
__global__ void __launch_bounds__(kBlock) k_finalize_beta_batch(SeqState *st, const double *partials, int nparts,
                                                                int B, double *beta_out, int n_max, int k,
                                                                double tol, ShiftState *shifts,
                                                                const double *omega, int n_omega, double eta,
                                                                double rtol)
{
    const int r = blockIdx.x;
    SeqState *q0 = st + r;
    if (q0->done) return;
    __shared__ double s_bn;
    const double ssum = reduce_partials_strided(partials, nparts, B, r);
    if (threadIdx.x == 0) s_bn = sqrt(ssum);
    const double alpha = q0->alpha_cur, bk = q0->beta_cur, zoff = q0->shift_re;
    __syncthreads();
    const double bn = s_bn;
    ShiftState *sh = shifts + (size_t)r * n_omega;
    double rmax = 0.0;
    for (int j = threadIdx.x; j < n_omega; j += blockDim.x) {
        const double zr = omega[j] + zoff, zi = eta;
        ShiftState q = sh[j];
        shift_update(q, zr, zi, alpha, bk, k);
        sh[j] = q;
        const double res = sqrt((q.pr * q.pr + q.pi * q.pi) / (q.dr * q.dr + q.di * q.di)) * bn;
        rmax = res > rmax ? res : rmax;
    }
    const double m = block_max<kBlock>(rmax);
    if (threadIdx.x == 0) {
        q0->max_resid = m * q0->norm;
        beta_out[(size_t)r * n_max + k] = bn;
        q0->steps = k + 1;
        if (!isfinite(bn)) q0->numeric_error = 1;
        if (!(bn > tol) || (rtol > 0.0 && m <= rtol)) {
            q0->done = 1;
        } else {
            q0->inv_prev = q0->inv_cur;
            q0->inv_cur = 1.0 / bn;
            q0->beta_cur = bn;
        }
    }
}

void launch_finalize_beta_batch(int B, SeqState *st, const double *partials, int nparts, double *beta_out,
                                int n_max, int k, double tol, ShiftState *shifts, const double *omega, int n_omega,
                                double eta, hipStream_t s, double rtol)
{
    hipLaunchKernelGGL(k_finalize_beta_batch, dim3(B), dim3(kBlock), 0, s, st, partials, nparts, B, beta_out, n_max,
                       k, tol, shifts, omega, n_omega, eta, rtol);
}

// norms of the B start vectors and the per-sequence reset
template <int B>
__global__ void __launch_bounds__(kBlock) k_dot_batch(uint32_t dim, const double2 *__restrict__ a, double *partials)
{
    double hi = 0.0, lo = 0.0, err = 0.0;
    const size_t n = (size_t)dim * B;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        const double2 u = a[idx];
        acc_prod(hi, lo, err, u.x, u.x);
        acc_prod(hi, lo, err, u.y, u.y);
    }
    write_partial_batch<B, kBlock>(partials, hi, lo, err);
}

__global__ void __launch_bounds__(kBlock) k_start_batch(SeqState *st, const double *partials, int nparts, int B,
                                                        BatchShifts shift_re)
{
    const int r = blockIdx.x;
    const double s = reduce_partials_strided(partials, nparts, B, r);
    if (threadIdx.x == 0) {
        SeqState *q = st + r;
        const double nrm = sqrt(s);
        q->norm2 = s;
        q->norm = nrm;
        q->inv_cur = nrm > 0.0 ? 1.0 / nrm : 0.0;
        q->inv_prev = 0.0;
        q->beta_cur = 0.0;
        q->alpha_cur = 0.0;
        q->shift_re = shift_re.re[r];
        q->max_resid = 0.0;
        q->done = nrm > 0.0 ? 0 : 1;
        q->steps = 0;
        q->numeric_error = isfinite(s) ? 0 : 1;
        q->pad = 0;
    }
}

void launch_start_batch(int B, uint32_t dim, const double *chi, double *partials, SeqState *st,
                        const BatchShifts &shift_re, hipStream_t s)
{
    const dim3 g(vec_batch_grid(dim, B)), t(kBlock);
    switch (B) {
    case 2: hipLaunchKernelGGL(k_dot_batch<2>, g, t, 0, s, dim, (const double2 *)chi, partials); break;
    case 4: hipLaunchKernelGGL(k_dot_batch<4>, g, t, 0, s, dim, (const double2 *)chi, partials); break;
    case 8: hipLaunchKernelGGL(k_dot_batch<8>, g, t, 0, s, dim, (const double2 *)chi, partials); break;
    case 16: hipLaunchKernelGGL(k_dot_batch<16>, g, t, 0, s, dim, (const double2 *)chi, partials); break;
    default: break;
    }
    hipLaunchKernelGGL(k_start_batch, dim3(B), dim3(kBlock), 0, s, st, partials, vec_batch_grid(dim, B), B,
                       shift_re);
}

template <class Epi>
static void pass_attributes()
{
    const int lds = kPassTile * sizeof(double2);
    const void *k[] = {(const void *)k_hv_pass<Epi, true, true, false>, (const void *)k_hv_pass<Epi, true, false, false>,
                       (const void *)k_hv_pass<Epi, false, true, false>, (const void *)k_hv_pass<Epi, false, false, false>,
                       (const void *)k_hv_pass<Epi, true, true, true>, (const void *)k_hv_pass<Epi, true, false, true>,
                       (const void *)k_hv_pass<Epi, false, true, true>, (const void *)k_hv_pass<Epi, false, false, true>};
    for (const void *f : k) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

void hv_set_attributes()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
        prop.multiProcessorCount > 0)
        g_cus = prop.multiProcessorCount;
    (void)hipFuncSetAttribute((const void *)k_hv_pass_fused<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kPassTile * sizeof(double2));
    (void)hipFuncSetAttribute((const void *)k_hv_pass_fused<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kPassTile * sizeof(double2));
    pass_attributes<EpiApply>();
    pass_attributes<EpiLanczosADev>();
    pass_attributes<EpiTaylor>();
    (void)hipFuncSetAttribute((const void *)k_hv_tiled<EpiApply>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kTile * sizeof(double2));
    (void)hipFuncSetAttribute((const void *)k_hv_tiled<EpiLanczosADev>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kTile * sizeof(double2));
    (void)hipFuncSetAttribute((const void *)k_hv_tiled<EpiTaylor>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kTile * sizeof(double2));
}

}  // namespace ftk
