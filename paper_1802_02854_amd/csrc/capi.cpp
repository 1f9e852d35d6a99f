// C-ABI of libftkw: contexts, Hamiltonians, filtered typical states, shifted
// Krylov spectra and reweighting.  Host orchestration of the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "cocg.h"
#include "ftkw_internal.h"
#include "kernels.h"

using namespace ftk;

namespace {

thread_local std::string g_error;
bool g_use_graphs = true;
bool g_plain_loop = false;  // comparison mode: no graph, alpha/beta read on the host every step
int g_stack_mode = -1;      // batches of Green's sequences: -1 stacked when possible/tuned, 0 block layout, 1 stacked

#define HIP_CHECK(call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            fail(e_ == hipErrorOutOfMemory ? FTK_ENOMEM : FTK_EDEVICE,                       \
                 std::string(#call) + ": " + hipGetErrorString(e_));                         \
    } while (0)

template <class F>
ftk_status guard(F &&f)
{
    try {
        f();
        return FTK_OK;
    } catch (const Error &e) {
        g_error = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        g_error = "host allocation failed";
        return FTK_ENOMEM;
    } catch (const std::exception &e) {
        g_error = e.what();
        return FTK_EDEVICE;
    } catch (...) {
        g_error = "unknown error";
        return FTK_EDEVICE;
    }
}

void need(bool ok, const char *msg)
{
    if (!ok) fail(FTK_EINVAL, msg);
}

}  // namespace

// ---------------------------------------------------------------------------
struct ftk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;  // created here when the caller passed the null stream
    ftk_alloc_fn alloc_fn = nullptr;  // caller's allocator (both or neither)
    ftk_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;
    size_t bytes = 0;
    size_t peak = 0;  // high-water mark of bytes since the last reset
    bool timing = false;
    std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> events;

    // brackets the launches made by f with events when timing is on
    template <class F>
    void timed(const char *name, bool sample, F &&f)
    {
        if (!(timing && sample)) {
            f();
            return;
        }
        hipEvent_t a, b;
        HIP_CHECK(hipEventCreate(&a));
        HIP_CHECK(hipEventCreate(&b));
        HIP_CHECK(hipEventRecord(a, stream));
        f();
        HIP_CHECK(hipEventRecord(b, stream));
        events[name].push_back({a, b});
    }
    void clear_events()
    {
        for (auto &kv : events)
            for (auto &e : kv.second) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
        events.clear();
    }
    ~ftk_ctx()
    {
        clear_events();
        if (own_stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

// Device allocation tied to a context's byte count.
struct DevBuf {
    ftk_ctx *ctx = nullptr;
    void *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(ftk_ctx *c, size_t bytes) : ctx(c), n(bytes)
    {
        if (bytes == 0) return;
        HIP_CHECK(hipSetDevice(c->device));
        if (c->alloc_fn) {
            p = c->alloc_fn(bytes, c->alloc_user);
            if (!p) fail(FTK_ENOMEM, "caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                fail(FTK_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
            }
        }
        c->bytes += bytes;
        c->peak = std::max(c->peak, c->bytes);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            ctx = o.ctx;
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release()
    {
        if (p) {
            if (ctx->free_fn)
                ctx->free_fn(p, ctx->alloc_user);
            else
                (void)hipFree(p);
            ctx->bytes -= n;
        }
        p = nullptr;
        n = 0;
    }
    double *d() const { return (double *)p; }
};

}  // namespace

struct ftk_hamiltonian {
    ftk_ctx *ctx = nullptr;
    BondTable table;
    HvOp op;        // bond table, multi-pass plan and its scratch vector
    DevBuf scratch;
    std::vector<double> site_xy;
    int n_sites = 0;
    uint32_t dim = 0;
};

namespace {

// Device workspace for Lanczos runs on one Hamiltonian.
struct Krylov {
    const ftk_hamiltonian *h;
    ftk_ctx *ctx;
    hipStream_t s;
    uint32_t dim;
    int nparts;
    int nparts_hv;
    DevBuf partials, partials_b, state, alpha, beta, scalar;  // partials_b: norms of fused steps
    int n_max;
    Krylov(const ftk_hamiltonian *H, int n_steps_max, int n_states)
        : h(H), ctx(H->ctx), s(H->ctx->stream), dim(H->dim), nparts(vec_grid(H->dim)), nparts_hv(hv_grid(H->op)),
          partials(H->ctx, sizeof(double) * 2 * kMaxGrid * 16), partials_b(H->ctx, sizeof(double) * 2 * kMaxGrid * 16),
          state(H->ctx, sizeof(SeqState) * (size_t)std::max(1, n_states)),
          alpha(H->ctx, sizeof(double) * (size_t)std::max(1, n_steps_max) * std::max(1, n_states)),
          beta(H->ctx, sizeof(double) * (size_t)std::max(1, n_steps_max) * std::max(1, n_states)),
          scalar(H->ctx, sizeof(double) * 8), n_max(n_steps_max)
    {
    }
    SeqState *st(int i) const { return (SeqState *)state.p + i; }
    double *al(int i) const { return alpha.d() + (size_t)i * n_max; }
    double *be(int i) const { return beta.d() + (size_t)i * n_max; }

    // rounded Re<a|b> brought back to the host
    double dot(const double *a, const double *b)
    {
        launch_dot(dim, a, b, partials.d(), s);
        launch_sum_partials(partials.d(), nparts, scalar.d(), s);
        double r;
        HIP_CHECK(hipMemcpyAsync(&r, scalar.p, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        return r;
    }

    // n Lanczos steps of sequence i started from `start` (w_{-1}); buffers W0, W1
    // alternate; Vbuf (optional) receives v_k for k in [k0, k0 + nb) and the
    // callback flushes it; shifts (optional) get the per-step update.
    template <class Flush>
    void run(int i, const double *start, double *W0, double *W1, int n, double shift_re,
             ShiftState *shifts, const double *omega, int n_omega, double eta, double *Vbuf,
             int nb, Flush &&flush)
    {
        launch_dot(dim, start, start, partials.d(), s);
        launch_start_sequence(st(i), partials.d(), nparts, shift_re, s);
        const double tol = 1e-12 * h->table.norm_bound;
        double *W[2] = {W0, W1};
        const bool fuse = lanczos_fusable(h->op) && !g_plain_loop;
        const bool fa_on = fuse && alpha_in_fused_pass();
        double *pa = partials.d(), *pb = fa_on ? partials_b.d() : partials.d();
        int k0 = 0;
        for (int k = 0; k < n; ++k) {
            // w_k goes to W[k % 2]; v_k comes from w_{k-1}, v_{k-1} from w_{k-2}
            const double *cur = k == 0 ? start : W[(k - 1) % 2];
            const double *prv = k == 1 ? start : W[k % 2];
            double *out = W[k % 2];
            double *vout = Vbuf ? Vbuf + (size_t)(k - k0) * 2 * dim : nullptr;
            ctx->timed("filter_step", (k & 7) == 1, [&] {
                if (fuse && k > 0) {
                    // second half of step k-1 inside the first pass of step k (which also
                    // finalises alpha_{k-1}); its beta finalisation rides in the middle pass
                    // when there is one.  alpha partials in pa, norm partials in pb.
                    const FinAlpha fa{pa, nparts_hv, al(i), 0, k - 1};
                    launch_lanczos_fused_first(h->op, W[(k - 1) % 2], prv, st(i), pb, s, Stack(),
                                               fa_on ? &fa : nullptr);
                    const FinBeta fb{st(i), pb, nparts_hv, be(i), k - 1, tol, shifts, omega, n_omega, eta, 0.0, 0};
                    const bool mid = beta_in_middle_pass(h->op);
                    if (!mid)
                        launch_finalize_beta(st(i), pb, nparts_hv, be(i), k - 1, tol, shifts, omega, n_omega, eta, s);
                    launch_lanczos_a_rest(h->op, cur, prv, out, vout, st(i), pa, s, Stack(), mid ? &fb : nullptr);
                    if (!fa_on) launch_finalize_alpha(st(i), pa, nparts_hv, al(i), k, s);
                } else {
                    launch_lanczos_a(h->op, cur, prv, out, vout, st(i), partials.d(), k == 0, s);
                    if (!(fuse && fa_on)) launch_finalize_alpha(st(i), partials.d(), nparts_hv, al(i), k, s);
                    if (!fuse) {
                        launch_lanczos_b(dim, cur, out, st(i), partials.d(), s);
                        launch_finalize_beta(st(i), partials.d(), nparts, be(i), k, tol, shifts, omega, n_omega, eta,
                                             s);
                    }
                }
            });
            if (Vbuf && (k - k0 + 1 == nb || k == n - 1)) {
                flush(k0, k - k0 + 1);
                k0 = k + 1;
            }
        }
        if (fuse) {
            // alpha and the second half of the last step
            if (fa_on) launch_finalize_alpha(st(i), pa, nparts_hv, al(i), n - 1, s);
            const double *cur = n == 1 ? start : W[(n - 2) % 2];
            launch_lanczos_b(dim, cur, W[(n - 1) % 2], st(i), partials.d(), s);
            launch_finalize_beta(st(i), partials.d(), nparts, be(i), n - 1, tol, shifts, omega, n_omega, eta, s);
        }
    }

    SeqState read_state(int i)
    {
        SeqState r;
        HIP_CHECK(hipMemcpyAsync(&r, st(i), sizeof(SeqState), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        return r;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
struct ftk_states {
    const ftk_hamiltonian *h = nullptr;
    int nv = 0, na = 0, L = 0, M = 0, n_steps = 0;
    std::vector<double> betas, E_b, eps;
    std::vector<double> log_norm;     // [nv][na]
    std::vector<double> n_m;          // [nv][na][L]
    std::vector<double> alpha, beta;  // [nv][na][n_steps]
    std::vector<int> steps;           // [nv][na]
    std::vector<DevBuf> phi;          // [nv][na], each L vectors
    std::vector<double> h1, h2;       // [nv][na][L] shell moments (when asked for)
};

struct ftk_spectrum {
    const ftk_states *st = nullptr;
    int nalpha = 0, nq = 0, nw = 0, n_steps = 0;
    int solver = FTK_SOLVER_LANCZOS;
    std::vector<double> ca, cb, cc;   // COCG: [seq][n] a_k, [seq][n] b_{k+1}, [seq][n+1] c_k (complex)
    std::vector<int> seed;            // COCG: final seed index per sequence
    std::vector<double> g;            // [nv][na][L][nalpha][nq][nw] complex
    std::vector<double> resid;        // [nv][na][L][nalpha][nq]
    std::vector<double> chi2;         // [nv][na][L][nalpha][nq] ||S^alpha_Q phi^m||^2
    std::vector<double> alpha, beta;  // [seq][n_steps]
    std::vector<int> steps;           // [seq]
};

struct ftk_pair_spectrum {
    const ftk_states *st = nullptr;
    int np = 0, nw = 0, n_steps = 0;
    int solver = FTK_SOLVER_LANCZOS;
    std::vector<double> ca, cb, cc;   // COCG: per (pair, run k = 0 G_AB, 1 G_BA) a_k, b_{k+1}, c_k (complex)
    std::vector<int> seed;            // COCG: final seed index per run
    std::vector<double> gab, gba;     // [nv][na][L][np][nw] complex
    std::vector<double> overlap;      // [nv][na][L][np] complex <A phi^m|B phi^m>
    std::vector<double> resid;        // [nv][na][L][np] largest of the four sequences
    std::vector<double> alpha, beta;  // [nv][na][L][np][4][n_steps]
    std::vector<int> steps;           // [nv][na][L][np][4]
};

extern "C" {

const char *ftk_last_error(void) { return g_error.c_str(); }

ftk_status ftk_ctx_create(int device, void *hip_stream, ftk_ctx **out)
{
    return guard([&] {
        need(out != nullptr, "out must not be NULL");
        int n = 0;
        HIP_CHECK(hipGetDeviceCount(&n));
        need(device >= 0 && device < n, "device index out of range");
        HIP_CHECK(hipSetDevice(device));
        hv_set_attributes();
        auto c = std::make_unique<ftk_ctx>();
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        if (!c->stream) {
            // a blocking stream of our own: it stays ordered with the null stream and,
            // unlike it, can be captured into a graph
            HIP_CHECK(hipStreamCreate(&c->stream));
            c->own_stream = true;
        }
        *out = c.release();
    });
}

ftk_status ftk_ctx_create_with_allocator(int device, void *hip_stream, ftk_alloc_fn alloc, ftk_free_fn release,
                                         void *user, ftk_ctx **out)
{
    ftk_status st = guard([&] {
        need(out != nullptr, "out must not be NULL");
        need((alloc == nullptr) == (release == nullptr), "give both allocator callbacks or neither");
    });
    if (st != FTK_OK) return st;
    ftk_ctx *c = nullptr;
    st = ftk_ctx_create(device, hip_stream, &c);
    if (st != FTK_OK) return st;
    c->alloc_fn = alloc;
    c->free_fn = release;
    c->alloc_user = user;
    *out = c;
    return FTK_OK;
}

ftk_status ftk_ctx_destroy(ftk_ctx *ctx)
{
    return guard([&] { delete ctx; });
}

ftk_status ftk_sync(ftk_ctx *ctx)
{
    return guard([&] {
        need(ctx != nullptr, "ctx must not be NULL");
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
    });
}

ftk_status ftk_ctx_memory(const ftk_ctx *ctx, size_t *bytes)
{
    return guard([&] {
        need(ctx && bytes, "NULL argument");
        *bytes = ctx->bytes;
    });
}

ftk_status ftk_ctx_peak_memory(ftk_ctx *ctx, size_t *peak, int reset)
{
    return guard([&] {
        need(ctx != nullptr, "ctx must not be NULL");
        if (peak) *peak = ctx->peak;
        if (reset) ctx->peak = ctx->bytes;
    });
}

ftk_status ftk_ctx_set_timing(ftk_ctx *ctx, int enable)
{
    return guard([&] {
        need(ctx != nullptr, "ctx must not be NULL");
        ctx->timing = enable != 0;
    });
}

ftk_status ftk_set_tuning(const char *key, int value)
{
    return guard([&] {
        need(key != nullptr, "key must not be NULL");
        if (std::string(key) == "hv_variant") {
            need(value >= -1 && value <= 3, "hv_variant must be -1, 0, 1, 2 or 3");
            set_hv_mode(value);
        } else if (std::string(key) == "pass_grid") {
            need(value >= 0 && value <= kMaxGrid, "pass_grid must be in [0, 4096]");
            set_pass_grid(value);
        } else if (std::string(key) == "stream_hints") {
            need(value >= -1 && value <= 1, "stream_hints must be -1, 0 or 1");
            set_hints(value);
        } else if (std::string(key) == "fuse_finalize") {
            need(value == 0 || value == 1, "fuse_finalize must be 0 or 1");
            set_fuse_finalize(value);
        } else if (std::string(key) == "full_grid") {
            need(value == 0 || value == 1, "full_grid must be 0 or 1");
            set_full_grid(value);
        } else if (std::string(key) == "graphs") {
            need(value == 0 || value == 1, "graphs must be 0 or 1");
            g_use_graphs = value != 0;
        } else if (std::string(key) == "plain_loop") {
            need(value == 0 || value == 1, "plain_loop must be 0 or 1");
            g_plain_loop = value != 0;
        } else if (std::string(key) == "stack_batch") {
            need(value >= -1 && value <= 1, "stack_batch must be -1, 0 or 1");
            g_stack_mode = value;
        } else {
            fail(FTK_EINVAL, std::string("unknown tuning key ") + key);
        }
    });
}

ftk_status ftk_ctx_kernel_time(ftk_ctx *ctx, const char *kernel, int *count, double *mean_ms)
{
    return guard([&] {
        need(ctx && kernel && count && mean_ms, "NULL argument");
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
        auto it = ctx->events.find(kernel);
        *count = 0;
        *mean_ms = 0.0;
        if (it == ctx->events.end()) return;
        double tot = 0.0;
        for (auto &e : it->second) {
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, e.first, e.second));
            tot += ms;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        *count = (int)it->second.size();
        *mean_ms = *count ? tot / *count : 0.0;
        ctx->events.erase(it);
    });
}

ftk_status ftk_honeycomb_cluster(int t11, int t12, int t21, int t22, int *n_sites, int *n_bonds,
                                 int32_t *bi, int32_t *bj, int8_t *gamma, double *site_xy)
{
    return guard([&] {
        HoneyCluster cl = honeycomb(t11, t12, t21, t22);
        if (n_sites) *n_sites = 2 * cl.n_cells;
        if (n_bonds) *n_bonds = (int)cl.bi.size();
        if (bi) std::copy(cl.bi.begin(), cl.bi.end(), bi);
        if (bj) std::copy(cl.bj.begin(), cl.bj.end(), bj);
        if (gamma) std::copy(cl.gamma.begin(), cl.gamma.end(), gamma);
        if (site_xy) std::copy(cl.xy.begin(), cl.xy.end(), site_xy);
    });
}

ftk_status ftk_honeycomb_momenta(int t11, int t12, int t21, int t22, int *n_q, double *q_xy)
{
    return guard([&] {
        need(n_q != nullptr, "n_q must not be NULL");
        std::vector<double> q = honeycomb_momenta(t11, t12, t21, t22);
        *n_q = (int)(q.size() / 2);
        if (q_xy) std::copy(q.begin(), q.end(), q_xy);
    });
}

ftk_status ftk_named_momentum(const char *name, double *q_xy)
{
    return guard([&] {
        need(name && q_xy, "NULL argument");
        need(named_momentum(name, q_xy), "unknown momentum name");
    });
}

ftk_status ftk_build_hamiltonian(ftk_ctx *ctx, const ftk_cluster *c, double K, double J,
                                 ftk_hamiltonian **out)
{
    return guard([&] {
        need(ctx && c && out, "NULL argument");
        auto h = std::make_unique<ftk_hamiltonian>();
        h->ctx = ctx;
        h->table = make_bond_table(*c, K, J);
        h->op.P = make_hv_params(h->table);
        h->op.plan = make_hv_plan(h->table);
        h->n_sites = c->n_sites;
        h->dim = 1u << c->n_sites;
        if (h->op.plan.n_passes > 0 && h->n_sites >= kPassMinSites) {
            h->scratch = DevBuf(ctx, sizeof(double) * 2 * (size_t)h->dim);
            h->op.scratch = h->scratch.d();
        }
        h->site_xy.assign(c->site_xy, c->site_xy + 2 * c->n_sites);
        *out = h.release();
    });
}

ftk_status ftk_hv_plan(const ftk_cluster *c, int *n_passes, int *core, int *segment_end)
{
    return guard([&] {
        need(c && n_passes, "NULL argument");
        const HvPlan plan = make_hv_plan(make_bond_table(*c, -1.0, 0.0));
        *n_passes = plan.n_passes;
        if (core) *core = plan.core;
        if (segment_end)
            for (int p = 0; p < plan.n_passes; ++p) segment_end[p] = plan.pass[p].b1;
    });
}

ftk_status ftk_plan_layout(const ftk_cluster *c, int *site_perm, int *bond_order, int *n_passes)
{
    return guard([&] {
        need(c && site_perm && bond_order && n_passes, "NULL argument");
        const BondTable t = make_bond_table(*c, -1.0, 0.0);
        std::vector<int32_t> perm(c->n_sites), order(c->n_bonds);
        const int P = plan_layout(t.n_sites, t.n_bonds, t.bi, t.bj, kPassBits, 6, perm.data(), order.data());
        if (P == 0) {
            for (int l = 0; l < c->n_sites; ++l) perm[l] = l;
            for (int b = 0; b < c->n_bonds; ++b) order[b] = b;
        }
        std::copy(perm.begin(), perm.end(), site_perm);
        std::copy(order.begin(), order.end(), bond_order);
        *n_passes = P;
    });
}

ftk_status ftk_hamiltonian_destroy(ftk_hamiltonian *h)
{
    return guard([&] { delete h; });
}

ftk_status ftk_hamiltonian_info(const ftk_hamiltonian *h, int *n_sites, double *norm_bound)
{
    return guard([&] {
        need(h != nullptr, "h must not be NULL");
        if (n_sites) *n_sites = h->n_sites;
        if (norm_bound) *norm_bound = h->table.norm_bound;
    });
}

ftk_status ftk_apply_h(const ftk_hamiltonian *h, const double *v, double *w, int n_rhs)
{
    return ftk_apply_h_strided(h, v, w, n_rhs, h ? (int64_t)h->dim : 0);
}

ftk_status ftk_apply_h_strided(const ftk_hamiltonian *h, const double *v, double *w, int n_rhs, int64_t ld)
{
    return guard([&] {
        need(h && v && w, "NULL argument");
        need(n_rhs >= 0, "n_rhs must be >= 0");
        need(ld >= (int64_t)h->dim, "ld must be >= 2^N");
        const size_t stride = 2 * (size_t)ld;
        const size_t span = n_rhs > 0 ? stride * (size_t)(n_rhs - 1) + 2 * (size_t)h->dim : 0;
        need(v + span <= w || w + span <= v, "v and w overlap");
        HIP_CHECK(hipSetDevice(h->ctx->device));
        for (int r = 0; r < n_rhs; ++r)
            h->ctx->timed("apply_h", true,
                          [&] { launch_apply_h(h->op, v + r * stride, w + r * stride, h->ctx->stream); });
        HIP_CHECK(hipGetLastError());
    });
}

}  // extern "C"

namespace {

// Partial sums of the multi-pass H v for ftk_apply_h_noalloc: one array per GPU,
// held until the process ends.  Host code must never pass the array's name to a
// kernel (it is a host-side stand-in there); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device with that device current.
constexpr size_t kNoAllocScratchEntries = size_t(1) << kNoAllocMaxSites;  // complex entries (64 MiB)
static __device__ __align__(256) double2 scratch[kNoAllocScratchEntries];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's array (the device must be current)
double *noalloc_scratch(int device)
{
    need(device >= 0 && device < kMaxDevices, "device index out of range for the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        need(p != nullptr, "static scratch array has no device address");
        g_scratch_ptr[device] = (double *)p;
    }
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

ftk_status ftk_apply_h_noalloc(const ftk_hamiltonian *h, const double *v, double *w, int n_rhs)
{
    return guard([&] {
        need(h && v && w, "NULL argument");
        need(n_rhs >= 0, "n_rhs must be >= 0");
        const size_t span = 2 * (size_t)h->dim * (size_t)n_rhs;
        need(v + span <= w || w + span <= v, "v and w overlap");
        HIP_CHECK(hipSetDevice(h->ctx->device));
        HvOp op = h->op;
        if (hv_mode(h->op) == 3) {
            // the multi-pass form keeps its partial sums in the static array instead of
            // the Hamiltonian's scratch vector; every pass overwrites each entry before it
            // is read, so nothing has to start at zero
            if (h->dim > kNoAllocScratchEntries)
                fail(FTK_EINVAL, "ftk_apply_h_noalloc: the multi-pass H v of " + std::to_string(h->n_sites) +
                                     " sites needs 2^" + std::to_string(h->n_sites) +
                                     " scratch entries, more than the static maximum 2^" +
                                     std::to_string(kNoAllocMaxSites));
            op.scratch = noalloc_scratch(h->ctx->device);
        }
        for (int r = 0; r < n_rhs; ++r)
            launch_apply_h(op, v + 2 * (size_t)h->dim * r, w + 2 * (size_t)h->dim * r, h->ctx->stream);
        HIP_CHECK(hipGetLastError());
    });
}

ftk_status ftk_device_checks(ftk_ctx *ctx, int *compiled, uint32_t *violations, uint32_t *first_site,
                             uint32_t *first_index, int clear)
{
    return guard([&] {
        need(ctx != nullptr, "NULL argument");
        if (compiled) *compiled = device_checks_compiled();
        unsigned int r[3] = {0u, 0u, 0u};
        if (device_checks_compiled()) {
            HIP_CHECK(hipSetDevice(ctx->device));
            HIP_CHECK(hipStreamSynchronize(ctx->stream));
            device_checks_read(r, clear != 0);
            if (r[0] == ~0u && r[1] == ~0u) fail(FTK_EDEVICE, "reading the device check counters failed");
        }
        if (violations) *violations = r[0];
        if (first_site) *first_site = r[1];
        if (first_index) *first_index = r[2];
    });
}

ftk_status ftk_device_checks_selftest(ftk_ctx *ctx, uint32_t *redirected)
{
    return guard([&] {
        need(ctx != nullptr, "NULL argument");
        need(device_checks_compiled() != 0, "device checks are compiled into libftkw_check.so only");
        HIP_CHECK(hipSetDevice(ctx->device));
        DevBuf out(ctx, sizeof(uint32_t));
        device_checks_selftest((uint32_t *)out.p, ctx->stream);
        HIP_CHECK(hipGetLastError());
        uint32_t r = ~0u;
        HIP_CHECK(hipMemcpyAsync(&r, out.p, sizeof r, hipMemcpyDeviceToHost, ctx->stream));
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
        if (redirected) *redirected = r;
    });
}

ftk_status ftk_random_vector(ftk_ctx *ctx, uint64_t seed, uint64_t sample, int n_sites, double *out)
{
    return guard([&] {
        need(ctx && out, "NULL argument");
        need(n_sites >= 1 && n_sites <= kMaxSites, "n_sites must be in [1, 30]");
        HIP_CHECK(hipSetDevice(ctx->device));
        launch_gaussian(1u << n_sites, seed, sample, out, ctx->stream);
        HIP_CHECK(hipGetLastError());
    });
}

ftk_status ftk_filter_coefficients(const double *alpha, const double *beta, int n, double norm, double E_b,
                                   double eps, int L, int M, double *out)
{
    return guard([&] {
        need(alpha && beta && out, "NULL argument");
        need(n >= 1 && L >= 1, "n and L must be >= 1");
        need(M >= 2 && M % 2 == 0, "M must be even and >= 2");
        need(std::isfinite(eps) && eps > 0 && std::isfinite(E_b) && std::isfinite(norm), "bad eps, E_b or norm");
        shell_coefficients(alpha, beta, n, norm, E_b, eps, L, M, out);
    });
}

ftk_status ftk_shell_window(const double *alpha, const double *beta, int n, int L, double margin, double *E_b,
                            double *eps)
{
    return guard([&] {
        need(alpha && beta && E_b && eps, "NULL argument");
        need(n >= 1 && L >= 1, "n and L must be >= 1");
        need(std::isfinite(margin) && margin >= 0, "margin must be finite and >= 0");
        for (int i = 0; i < n; ++i) need(std::isfinite(alpha[i]), "non-finite T_n");
        for (int i = 0; i + 1 < n; ++i) need(std::isfinite(beta[i]), "non-finite T_n");
        shell_window(alpha, beta, n, L, margin, E_b, eps);
    });
}

ftk_status ftk_truncation_steps(const double *alpha, const double *beta, int n, const double *z_re,
                                const double *z_im, int n_z, double tol, int *k)
{
    return guard([&] {
        need(alpha && beta && z_re && z_im && k, "NULL argument");
        need(n >= 1 && n_z >= 1, "n and n_z must be >= 1");
        need(std::isfinite(tol) && tol >= 0, "tol must be finite and >= 0");
        *k = truncation_steps(alpha, beta, n, z_re, z_im, n_z, tol);
    });
}

ftk_status ftk_residual_history(const double *alpha, const double *beta, int n, const double *z_re,
                                const double *z_im, int n_z, double *out)
{
    return guard([&] {
        need(alpha && beta && z_re && z_im && out, "NULL argument");
        need(n >= 1 && n_z >= 1, "n and n_z must be >= 1");
        residual_history(alpha, beta, n, z_re, z_im, n_z, out);
    });
}

ftk_status ftk_taylor_plan(int n_sites, double beta, double norm_bound, double lambda, int *Md, int *K, double *c,
                           double *ell)
{
    return guard([&] {
        need(n_sites >= 1 && std::isfinite(beta) && beta >= 0 && norm_bound > 0, "bad arguments");
        TaylorPlan p = taylor_plan(n_sites, beta, norm_bound, lambda > 0 ? lambda : 1e8);
        if (Md) *Md = p.Md;
        if (K) *K = p.K;
        if (c) *c = p.c;
        if (ell) *ell = p.ell;
    });
}

// ---------------------------------------------------------------------------
ftk_status ftk_typical_states(const ftk_hamiltonian *h, const ftk_ts_params *p, ftk_states **out)
{
    return guard([&] {
        need(h && p && out, "NULL argument");
        need(p->n_vectors >= 1 && p->n_anchors >= 1, "n_vectors and n_anchors must be >= 1");
        need(p->anchor_beta != nullptr, "anchor_beta must not be NULL");
        need((p->E_b == nullptr) == (p->eps == nullptr), "E_b and eps must both be given or both be NULL");
        const bool auto_window = p->E_b == nullptr;
        const double margin = p->window_margin > 0 ? p->window_margin : 0.1;
        need(std::isfinite(margin), "window_margin must be finite");
        need(std::isfinite(p->resid_tol) && p->resid_tol >= 0, "resid_tol must be finite and >= 0");
        need(p->M >= 2 && p->M % 2 == 0, "M must be even and >= 2");
        need(p->L >= 1, "L must be >= 1");
        need(p->n_steps >= 1, "n_steps must be >= 1");
        need(p->first_vector >= 0, "first_vector must be >= 0");
        for (int a = 0; a < p->n_anchors; ++a) {
            need(std::isfinite(p->anchor_beta[a]) && p->anchor_beta[a] >= 0, "anchor beta must be finite and >= 0");
            if (auto_window) continue;
            need(std::isfinite(p->eps[a]) && p->eps[a] > 0, "eps must be > 0");
            need(std::isfinite(p->E_b[a]), "E_b must be finite");
        }
        const double lambda = p->taylor_lambda > 0 ? p->taylor_lambda : 1e8;
        ftk_ctx *ctx = h->ctx;
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t s = ctx->stream;
        const uint32_t dim = h->dim;
        const size_t vbytes = sizeof(double) * 2 * (size_t)dim;
        const int n = p->n_steps;
        const int nb = std::max(1, std::min(n, p->block_steps > 0 ? p->block_steps : 64));

        auto st = std::make_unique<ftk_states>();
        st->h = h;
        st->nv = p->n_vectors;
        st->na = p->n_anchors;
        st->L = p->L;
        st->M = p->M;
        st->n_steps = n;
        st->betas.assign(p->anchor_beta, p->anchor_beta + p->n_anchors);
        if (auto_window) {
            st->E_b.assign(p->n_anchors, 0.0);
            st->eps.assign(p->n_anchors, 0.0);
        } else {
            st->E_b.assign(p->E_b, p->E_b + p->n_anchors);
            st->eps.assign(p->eps, p->eps + p->n_anchors);
        }
        st->log_norm.assign((size_t)st->nv * st->na, 0.0);
        st->n_m.assign((size_t)st->nv * st->na * st->L, 0.0);
        st->alpha.assign((size_t)st->nv * st->na * n, 0.0);
        st->beta.assign((size_t)st->nv * st->na * n, 0.0);
        st->steps.assign((size_t)st->nv * st->na, 0);
        if (p->shell_moments) {
            st->h1.assign((size_t)st->nv * st->na * st->L, 0.0);
            st->h2.assign((size_t)st->nv * st->na * st->L, 0.0);
        }

        Krylov kr(h, n, 1);
        bool any_beta = false;
        for (int a = 0; a < st->na; ++a) any_beta = any_beta || st->betas[a] > 0;
        // Taylor workspace only when some anchor has beta > 0
        const size_t tbytes = any_beta ? vbytes : 0;
        DevBuf phi0(ctx, vbytes), phib(ctx, vbytes), t(ctx, tbytes), tn(ctx, tbytes), acc(ctx, tbytes);
        DevBuf W0(ctx, vbytes), W1(ctx, vbytes), Vbuf(ctx, vbytes * nb);
        DevBuf coef(ctx, sizeof(double) * 2 * (size_t)st->L * n);
        std::vector<double> hcoef((size_t)2 * st->L * n);
        const double N = (double)h->n_sites;

        for (int sv = 0; sv < st->nv; ++sv) {
            // phi_0 = g / ||g||
            if (p->gaussian_dev)
                launch_copy(dim, p->gaussian_dev + (size_t)sv * 2 * dim, phi0.d(), s);
            else
                launch_gaussian(dim, p->seed, (uint64_t)p->first_vector + sv, phi0.d(), s);
            {
                const double nrm = std::sqrt(kr.dot(phi0.d(), phi0.d()));
                if (!(nrm > 0) || !std::isfinite(nrm)) fail(FTK_ENUMERIC, "start vector has zero or non-finite norm");
                launch_scale(dim, phi0.d(), 1.0 / nrm, s);
            }
            for (int a = 0; a < st->na; ++a) {
                const size_t sa = (size_t)sv * st->na + a;
                // phi_beta = e^{-beta H / 2} phi_0 (Appendix A)
                launch_copy(dim, phi0.d(), phib.d(), s);
                const TaylorPlan plan = taylor_plan(h->n_sites, st->betas[a], h->table.norm_bound, lambda);
                double log_norm = 0.0;
                for (int sp = 0; sp < plan.Md; ++sp) {
                    launch_copy(dim, phib.d(), t.d(), s);
                    launch_copy(dim, phib.d(), acc.d(), s);
                    double *tc = t.d(), *tnx = tn.d();
                    for (int k = 1; k <= plan.K; ++k) {
                        const double sk = plan.c / (double)k;
                        const double ca = sk * plan.ell;
                        const double cb = -(sk / N);
                        launch_taylor_term(h->op, tc, tnx, acc.d(), ca, cb, s);
                        std::swap(tc, tnx);
                    }
                    const double nrm = std::sqrt(kr.dot(acc.d(), acc.d()));
                    if (!(nrm > 0) || !std::isfinite(nrm)) fail(FTK_ENUMERIC, "imaginary-time state lost its norm");
                    launch_copy(dim, acc.d(), phib.d(), s);
                    launch_scale(dim, phib.d(), 1.0 / nrm, s);
                    log_norm += std::log(nrm);
                }
                log_norm -= N * st->betas[a] * plan.ell / 2.0;
                st->log_norm[sa] = log_norm;

                // pass 1: Lanczos coefficients of phi_beta
                auto noflush = [](int, int) {};
                kr.run(0, phib.d(), W0.d(), W1.d(), n, 0.0, nullptr, nullptr, 0, 0.0, nullptr, 0, noflush);
                SeqState q1 = kr.read_state(0);
                if (q1.numeric_error) fail(FTK_ENUMERIC, "NaN/Inf in filter Lanczos coefficients");
                int steps = q1.steps;
                std::vector<double> al(steps), be(steps);
                HIP_CHECK(hipMemcpyAsync(al.data(), kr.al(0), sizeof(double) * steps, hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipMemcpyAsync(be.data(), kr.be(0), sizeof(double) * steps, hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipStreamSynchronize(s));
                if (auto_window && sv == 0) {
                    shell_window(al.data(), be.data(), steps, st->L, margin, &st->E_b[a], &st->eps[a]);
                    if (!(std::isfinite(st->eps[a]) && st->eps[a] > 0))
                        fail(FTK_ENUMERIC, "automatic shell window is empty or not finite");
                }
                std::vector<int> k_m;  // per-shell steps under residual truncation
                if (p->resid_tol > 0) {
                    // each filter operator on its own (Sec. V): shell m takes T_{k_m} for the
                    // first k_m at which all of its M contour shifts have converged
                    std::vector<double> zr(st->M), zi(st->M);
                    k_m.resize(st->L);
                    int kmax = 1;
                    for (int m = 0; m < st->L; ++m) {
                        for (int j = 1; j <= st->M; ++j) {
                            const double th = 2.0 * M_PI * ((double)j - 0.5) / (double)st->M;
                            zr[j - 1] = shell_energy(st->E_b[a], st->eps[a], m) + st->eps[a] * std::cos(th);
                            zi[j - 1] = st->eps[a] * std::sin(th);
                        }
                        k_m[m] = truncation_steps(al.data(), be.data(), steps, zr.data(), zi.data(), st->M,
                                                  p->resid_tol);
                        kmax = std::max(kmax, k_m[m]);
                    }
                    steps = kmax;
                    al.resize(steps);
                    be.resize(steps);
                }
                std::copy(al.begin(), al.end(), st->alpha.begin() + sa * n);
                std::copy(be.begin(), be.end(), st->beta.begin() + sa * n);
                st->steps[sa] = steps;

                // shell coefficients c^m (host, Sec. III.B); the device accumulates the
                // unnormalised residuals w_{k-1} = v_k / inv_k, so fold inv_k into c^m_k
                shell_coefficients(al.data(), be.data(), steps, q1.norm, st->E_b[a], st->eps[a], st->L, st->M,
                                   hcoef.data(), k_m.empty() ? nullptr : k_m.data());
                {
                    std::vector<double> inv(steps);
                    inv[0] = 1.0 / q1.norm;
                    for (int k = 1; k < steps; ++k) inv[k] = 1.0 / be[k - 1];
                    for (int m = 0; m < st->L; ++m)
                        for (int k = 0; k < steps; ++k) {
                            double *c = &hcoef[2 * ((size_t)m * steps + k)];
                            c[0] = c[0] * inv[k];
                            c[1] = c[1] * inv[k];
                        }
                }
                HIP_CHECK(hipMemcpyAsync(coef.p, hcoef.data(), sizeof(double) * 2 * st->L * steps,
                                         hipMemcpyHostToDevice, s));

                // pass 2: regenerate v_k and accumulate phi^m = sum_k c^m_k v_k
                DevBuf shells(ctx, vbytes * st->L);
                HIP_CHECK(hipMemsetAsync(shells.p, 0, vbytes * st->L, s));
                auto flush = [&](int k0, int cnt) {
                    launch_accumulate(dim, Vbuf.d(), cnt, coef.d(), steps, k0, shells.d(), st->L, s);
                };
                kr.run(0, phib.d(), W0.d(), W1.d(), steps, 0.0, nullptr, nullptr, 0, 0.0, Vbuf.d(), nb, flush);
                std::vector<double> al2(steps);
                HIP_CHECK(hipMemcpyAsync(al2.data(), kr.al(0), sizeof(double) * steps, hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipStreamSynchronize(s));
                if (std::memcmp(al2.data(), al.data(), sizeof(double) * steps) != 0)
                    fail(FTK_EDEVICE, "regenerated Lanczos sequence differs from the first pass");
                for (int m = 0; m < st->L; ++m) {
                    const double *pm = shells.d() + (size_t)m * 2 * dim;
                    st->n_m[sa * st->L + m] = kr.dot(pm, pm);
                    if (p->shell_moments) {
                        // H phi^m into the (now free) first Lanczos buffer
                        launch_apply_h(h->op, pm, W0.d(), s);
                        st->h1[sa * st->L + m] = kr.dot(pm, W0.d());
                        st->h2[sa * st->L + m] = kr.dot(W0.d(), W0.d());
                    }
                }
                st->phi.push_back(std::move(shells));
            }
        }
        HIP_CHECK(hipGetLastError());
        *out = st.release();
    });
}

ftk_status ftk_states_scalars(const ftk_states *st, double *log_norm, double *shell_norm2, double *E_m,
                              double *eps)
{
    return guard([&] {
        need(st != nullptr, "st must not be NULL");
        if (log_norm) std::copy(st->log_norm.begin(), st->log_norm.end(), log_norm);
        if (shell_norm2) std::copy(st->n_m.begin(), st->n_m.end(), shell_norm2);
        if (E_m)
            for (int a = 0; a < st->na; ++a)
                for (int m = 0; m < st->L; ++m) E_m[(size_t)a * st->L + m] = shell_energy(st->E_b[a], st->eps[a], m);
        if (eps) std::copy(st->eps.begin(), st->eps.end(), eps);
    });
}

ftk_status ftk_states_moments(const ftk_states *st, double *h1, double *h2)
{
    return guard([&] {
        need(st != nullptr, "st must not be NULL");
        need(!st->h1.empty(), "states were built without shell_moments");
        if (h1) std::copy(st->h1.begin(), st->h1.end(), h1);
        if (h2) std::copy(st->h2.begin(), st->h2.end(), h2);
    });
}

ftk_status ftk_states_window(const ftk_states *st, double *E_b, double *eps)
{
    return guard([&] {
        need(st != nullptr, "st must not be NULL");
        if (E_b) std::copy(st->E_b.begin(), st->E_b.end(), E_b);
        if (eps) std::copy(st->eps.begin(), st->eps.end(), eps);
    });
}

ftk_status ftk_states_lanczos(const ftk_states *st, int s, int a, double *alpha, double *beta, int *n_steps)
{
    return guard([&] {
        need(st != nullptr, "st must not be NULL");
        need(s >= 0 && s < st->nv && a >= 0 && a < st->na, "index out of range");
        const size_t sa = (size_t)s * st->na + a;
        const int k = st->steps[sa];
        if (n_steps) *n_steps = k;
        if (alpha) std::copy(st->alpha.begin() + sa * st->n_steps, st->alpha.begin() + sa * st->n_steps + k, alpha);
        if (beta) std::copy(st->beta.begin() + sa * st->n_steps, st->beta.begin() + sa * st->n_steps + k, beta);
    });
}

ftk_status ftk_states_copy_shell(const ftk_states *st, int s, int a, int m, double *out_dev)
{
    return guard([&] {
        need(st && out_dev, "NULL argument");
        need(s >= 0 && s < st->nv && a >= 0 && a < st->na && m >= 0 && m < st->L, "index out of range");
        const size_t vbytes = sizeof(double) * 2 * (size_t)st->h->dim;
        const DevBuf &b = st->phi[(size_t)s * st->na + a];
        HIP_CHECK(hipMemcpyAsync(out_dev, (const char *)b.p + (size_t)m * vbytes, vbytes, hipMemcpyDeviceToDevice,
                                 st->h->ctx->stream));
    });
}

ftk_status ftk_states_destroy(ftk_states *st)
{
    return guard([&] { delete st; });
}

// ---------------------------------------------------------------------------
namespace {

// B Green's-function sequences run together.  Two layouts for B > 1: the block
// layout (entry (x, r) at x*B + r) of the batched kernels, or a stack of B
// separate vectors driven through the multi-pass kernels in one grid (when the
// Hamiltonian uses the multi-pass form).  The n-step loop is captured once into
// a graph and replayed for every batch.
struct BatchRunner {
    const ftk_hamiltonian *h;
    HvOp op;  // h's operator with this runner's pass grid
    ftk_ctx *ctx;
    hipStream_t s;
    uint32_t dim;
    int B, n, nw;
    double eta, tol, rtol;  // breakdown threshold; residual truncation (0: off)
    bool stacked;           // B > 1 as a stack of multi-pass sequences
    int nparts_a, nparts_b;
    bool fuse;  // multi-pass H v: halves of consecutive steps fused
    DevBuf chi, W0, W1, st, al, be, shifts, omega, partials, partials_b, part;  // partials_b: norms of fused steps
    Stack sk;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool capturing = false;

    static bool stack_for(const ftk_hamiltonian *H, int B_, int stack)
    {
        if (B_ <= 1 || !lanczos_stackable(H->op) || g_plain_loop) return false;
        return stack == 1 || (stack < 0 && g_stack_mode != 0);
    }

    static HvOp with_grid(const HvOp &o, int pass_grid, int hints)
    {
        HvOp r = o;
        if (pass_grid > 0) r.pass_grid = pass_grid;
        if (hints >= 0) r.hints = hints;
        return r;
    }

    BatchRunner(const ftk_hamiltonian *H, int B_, int n_, const double *omega_host, int nw_, double eta_,
                double rtol_ = 0.0, int stack = -1, int pass_grid = 0, int hints = -1)
        : h(H), op(with_grid(H->op, pass_grid, hints)), ctx(H->ctx), s(H->ctx->stream), dim(H->dim), B(B_), n(n_), nw(nw_),
          eta(eta_), tol(1e-12 * H->table.norm_bound), rtol(rtol_), stacked(stack_for(H, B_, stack)),
          nparts_a(B_ == 1 ? hv_grid(op) : (stacked ? hv_grid(op, B_) : hv_batch_grid(H->dim, B_))),
          nparts_b(B_ == 1 || stacked ? vec_grid(H->dim) : vec_batch_grid(H->dim, B_)),
          fuse(stacked || (B_ == 1 && lanczos_fusable(op) && !g_plain_loop)),
          chi(H->ctx, sizeof(double) * 2 * (size_t)H->dim * B_), W0(H->ctx, sizeof(double) * 2 * (size_t)H->dim * B_),
          W1(H->ctx, sizeof(double) * 2 * (size_t)H->dim * B_), st(H->ctx, sizeof(SeqState) * B_),
          al(H->ctx, sizeof(double) * (size_t)n_ * B_), be(H->ctx, sizeof(double) * (size_t)n_ * B_),
          shifts(H->ctx, sizeof(ShiftState) * (size_t)nw_ * B_), omega(H->ctx, sizeof(double) * nw_),
          partials(H->ctx, sizeof(double) * 2 * (size_t)kMaxGrid * B_),
          partials_b(H->ctx, fuse ? sizeof(double) * 2 * (size_t)kMaxGrid * B_ : sizeof(double)),
          part(H->ctx, stacked ? sizeof(double) * 2 * (size_t)H->dim * B_ : sizeof(double))
    {
        need(B <= 16 || stacked, "more than 16 sequences per launch need the stacked layout");
        if (stacked) {
            sk.B = B;
            sk.scratch = part.d();
            sk.vs = 2 * (size_t)dim;
        }
        HIP_CHECK(hipMemcpyAsync(omega.p, omega_host, sizeof(double) * nw, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
    ~BatchRunner()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
    SeqState *states() const { return (SeqState *)st.p; }

    // right-hand side r = S^alpha_Q phi in the runner's layout
    void load_rhs(const SqParams &P, const double *phi, int r)
    {
        if (stacked)
            launch_apply_sq(P, phi, chi.d() + (size_t)r * 2 * dim, s);
        else
            launch_apply_sq(P, phi, chi.d(), s, B, r);
    }

    // right-hand side r = one of the polarization vectors of (lam, rho)
    void load_polarized(int k, const double *lam, const double *rho, int r)
    {
        if (stacked)
            launch_polarize(dim, k, lam, rho, chi.d() + (size_t)r * 2 * dim, s);
        else
            launch_polarize(dim, k, lam, rho, chi.d(), s, B, r);
    }

    void start(const BatchShifts &sh)
    {
        if (B == 1) {
            launch_dot(dim, chi.d(), chi.d(), partials.d(), s);
            launch_start_sequence(states(), partials.d(), nparts_b, sh.re[0], s);
        } else if (stacked) {
            launch_start_stacked(B, dim, chi.d(), partials.d(), states(), sh, s);
        } else {
            launch_start_batch(B, dim, chi.d(), partials.d(), states(), sh, s);
        }
    }

    void step(int k)
    {
        double *W[2] = {W0.d(), W1.d()};
        const double *cur = k == 0 ? chi.d() : W[(k - 1) % 2];
        const double *prv = k == 1 ? chi.d() : W[k % 2];
        double *out = W[k % 2];
        SeqState *q = states();
        ShiftState *sh = (ShiftState *)shifts.p;
        // per-step events only outside graph capture (a captured graph is timed as a whole)
        ctx->timed("lanczos_step", !capturing && (k & 7) == 1, [&] {
            if (B > 1 && !stacked) {
                launch_lanczos_a_batch(B, op.P, cur, prv, out, q, partials.d(), k == 0, s);
                launch_finalize_alpha_batch(B, q, partials.d(), nparts_a, al.d(), n, k, s);
                launch_lanczos_b_batch(B, dim, cur, out, q, partials.d(), s);
                launch_finalize_beta_batch(B, q, partials.d(), nparts_b, be.d(), n, k, tol, sh, omega.d(), nw, eta,
                                           s, rtol);
            } else if (fuse && k > 0) {
                // second half of step k-1 inside the first pass of step k (which also
                // finalises alpha_{k-1}); its beta finalisation rides in the middle pass
                // when there is one.  alpha partials in pa, norm partials in pb.
                const bool fa_on = alpha_in_fused_pass();
                double *pa = partials.d(), *pb = fa_on ? partials_b.d() : partials.d();
                const FinAlpha fa{pa, nparts_a, al.d(), n, k - 1};
                launch_lanczos_fused_first(op, W[(k - 1) % 2], prv, q, pb, s, sk, fa_on ? &fa : nullptr);
                const FinBeta fb{q, pb, nparts_a, be.d(), k - 1, tol, sh, omega.d(), nw, eta, rtol, n};
                const bool mid = beta_in_middle_pass(op);
                if (!mid)
                    launch_finalize_beta(q, pb, nparts_a, be.d(), k - 1, tol, sh, omega.d(), nw, eta, s, rtol, B, n);
                launch_lanczos_a_rest(op, cur, prv, out, nullptr, q, pa, s, sk, mid ? &fb : nullptr);
                if (!fa_on) launch_finalize_alpha(q, pa, nparts_a, al.d(), k, s, B, n);
            } else {
                launch_lanczos_a(op, cur, prv, out, nullptr, q, partials.d(), k == 0, s, sk);
                if (!(fuse && alpha_in_fused_pass()))
                    launch_finalize_alpha(q, partials.d(), nparts_a, al.d(), k, s, B, n);
                if (!fuse) {
                    launch_lanczos_b(dim, cur, out, q, partials.d(), s);
                    launch_finalize_beta(q, partials.d(), nparts_b, be.d(), k, tol, sh, omega.d(), nw, eta, s, rtol);
                }
            }
        });
    }

    // the second half of the last step when the halves are fused across steps
    void finish()
    {
        if (!fuse) return;
        if (alpha_in_fused_pass()) launch_finalize_alpha(states(), partials.d(), nparts_a, al.d(), n - 1, s, B, n);
        double *W[2] = {W0.d(), W1.d()};
        const double *cur = n == 1 ? chi.d() : W[(n - 2) % 2];
        launch_lanczos_b(dim, cur, W[(n - 1) % 2], states(), partials.d(), s, B, sk.vs);
        launch_finalize_beta(states(), partials.d(), nparts_b, be.d(), n - 1, tol, (ShiftState *)shifts.p, omega.d(),
                             nw, eta, s, rtol, B, n);
    }

    void run()
    {
        if (g_plain_loop) {
            // the reference loop: every step's coefficients go to the host before the next step
            double ab[2];
            for (int k = 0; k < n; ++k) {
                step(k);
                HIP_CHECK(hipMemcpyAsync(&ab[0], al.d() + k, sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipMemcpyAsync(&ab[1], be.d() + k, sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_CHECK(hipStreamSynchronize(s));
            }
            return;
        }
        if (g_use_graphs) {
            if (!exec) {
                capturing = true;
                HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
                for (int k = 0; k < n; ++k) step(k);
                finish();
                HIP_CHECK(hipStreamEndCapture(s, &graph));
                capturing = false;
                HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            }
            // the whole n-step loop of the batch: B sequences x n steps
            ctx->timed("lanczos_block", true, [&] { HIP_CHECK(hipGraphLaunch(exec, s)); });
        } else {
            for (int k = 0; k < n; ++k) step(k);
            finish();
        }
    }
};

}  // namespace

}  // extern "C"

namespace {

bool valid_rhs_block(int b) { return b == 0 || b == 1 || b == 2 || b == 4 || b == 8 || b == 16 || b == 32; }

struct TuneResult {
    int rhs_block;
    double ips;
    int stacked;        // B > 1 run as a stack of multi-pass sequences
    int pass_grid = 0;  // workgroups of the reducing multi-pass launches (0: the default)
    int hints = -1;     // cache hints of the multi-pass kernels (1 streaming, 0 cached, -1 by working set)
};
// every candidate's measurement of the last tuning per key (process memory only)
std::map<std::string, std::vector<TuneResult>> g_tune_all;
std::mutex g_tune_mu;
std::map<std::string, TuneResult> g_tune;

std::string tune_key(int device, int n_sites, int n_omega)
{
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == '"' || c == ':') c = '_';
    std::ostringstream k;
    k << arch << "/N" << n_sites << "/w" << n_omega << (g_use_graphs ? "/graph" : "/stream")
      << (g_plain_loop ? "/plain" : "");
    return k.str();
}

// the cache file is a flat JSON object {"key": [rhs_block, iters_per_s, stacked, pass_grid, hints], ...}
void tune_load(const char *path)
{
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t i = 0;
    while ((i = t.find('"', i)) != std::string::npos) {
        size_t j = t.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = t.substr(i + 1, j - i - 1);
        size_t a = t.find('[', j), b = t.find(']', j);
        if (a == std::string::npos || b == std::string::npos) break;
        int rb = 0, stk = 0, pg = 0, hn = -1;
        double ips = 0;
        const int got = std::sscanf(t.c_str() + a + 1, "%d , %lf , %d , %d , %d", &rb, &ips, &stk, &pg, &hn);
        if (got >= 2 && (rb == 1 || rb == 2 || rb == 4 || rb == 8 || rb == 16 || rb == 32))
            g_tune[key] = {rb, ips, got >= 3 && stk == 1 ? 1 : 0, got >= 4 && pg > 0 && pg <= kMaxGrid ? pg : 0,
                           got == 5 && (hn == 0 || hn == 1) ? hn : -1};
        i = b + 1;
    }
}

void tune_save(const char *path)
{
    std::ofstream f(path);
    if (!f) return;
    f << "{\n";
    size_t n = 0;
    for (auto &kv : g_tune)
        f << "  \"" << kv.first << "\": [" << kv.second.rhs_block << ", " << kv.second.ips << ", " << kv.second.stacked
          << ", " << kv.second.pass_grid << ", " << kv.second.hints << "]"
          << (++n < g_tune.size() ? ",\n" : "\n");
    f << "}\n";
}

TuneResult autotune(const ftk_hamiltonian *h, int n_omega);

}  // namespace

void ftk::set_last_error(const std::string &msg) { g_error = msg; }

int ftk::tuned_rhs_block(int device, int n_sites, int n_omega)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const std::string key = tune_key(device, n_sites, n_omega);
    const char *path = std::getenv("FTK_TUNE_CACHE");
    if (path && g_tune.find(key) == g_tune.end()) tune_load(path);
    auto it = g_tune.find(key);
    return it == g_tune.end() ? 0 : it->second.rhs_block;
}

namespace {

// the tuned layout for B sequences (1 stacked, 0 block), -1 when not tuned for B
int tuned_layout(int device, int n_sites, int n_omega, int B)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(tune_key(device, n_sites, n_omega));
    return it != g_tune.end() && it->second.rhs_block == B ? it->second.stacked : -1;
}

// the tuned pass grid and hint set for B sequences in layout stack: {0, -1} (the
// defaults) when not tuned for them
std::pair<int, int> tuned_passes(int device, int n_sites, int n_omega, int B, int stack)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(tune_key(device, n_sites, n_omega));
    if (it == g_tune.end() || it->second.rhs_block != B || !(B == 1 || it->second.stacked == stack)) return {0, -1};
    return {it->second.pass_grid, it->second.hints};
}

TuneResult autotune(const ftk_hamiltonian *h, int n_omega)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const char *path = std::getenv("FTK_TUNE_CACHE");
    const std::string key = tune_key(h->ctx->device, h->n_sites, n_omega);
    if (path && g_tune.find(key) == g_tune.end()) tune_load(path);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
    hipStream_t s = h->ctx->stream;
    const int nt = 64;
    std::vector<double> omega(n_omega);
    for (int j = 0; j < n_omega; ++j) omega[j] = -4.0 + 8.0 * j / std::max(1, n_omega - 1);
    struct TimingOff {  // kernel timing would split the captured graph; restore it on any exit
        ftk_ctx *c;
        bool was;
        ~TimingOff() { c->timing = was; }
    } off{h->ctx, h->ctx->timing};
    h->ctx->timing = false;
    size_t free_b = 0, total_b = 0;
    HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    DevBuf g(h->ctx, sizeof(double) * 2 * (size_t)h->dim);
    SqParams P;
    std::memset(&P, 0, sizeof(P));
    P.n_sites = h->n_sites;
    P.alpha = 2;
    for (int l = 0; l < h->n_sites; ++l) P.h[2 * l] = 1.0;  // uniform S^z sum
    TuneResult best{1, 0.0, 0};
    std::vector<TuneResult> all;
    // (rhs_block, layout): block layout, and the stacked one where the multi-pass form allows it
    std::vector<std::pair<int, int>> cands{{1, 0}};
    for (int B : {4, 16, 32}) {
        if (g_stack_mode != 1 && B <= 16) cands.push_back({B, 0});
        if (g_stack_mode != 0 && BatchRunner::stack_for(h, B, 1)) cands.push_back({B, 1});
    }
    // Krylov iterations per second of B sequences in layout stk with pass grid pg and
    // hint set hn (-1: by working set)
    auto time_it = [&](int B, int stk, int pg, int hn) {
        BatchRunner run(h, B, nt, omega.data(), n_omega, 0.01, 0.0, stk, pg, hn);
        for (int r = 0; r < B; ++r) {
            launch_gaussian(h->dim, 7, r, g.d(), s);
            run.load_rhs(P, g.d(), r);
        }
        BatchShifts bs;
        for (int r = 0; r < kMaxBatch; ++r) bs.re[r] = 0.0;
        double secs = 1e30;
        for (int rep = 0; rep < 4; ++rep) {  // the first repetition includes graph capture
            run.start(bs);
            HIP_CHECK(hipStreamSynchronize(s));
            auto t0 = std::chrono::steady_clock::now();
            run.run();
            HIP_CHECK(hipStreamSynchronize(s));
            auto t1 = std::chrono::steady_clock::now();
            if (rep > 0) secs = std::min(secs, std::chrono::duration<double>(t1 - t0).count());
        }
        return (double)B * nt / secs;
    };
    for (auto [B, stk] : cands) {
        // three dim x B vectors per batch (four stacked); leave a quarter of the free memory untouched
        if (B > 1 && (3.0 + stk) * 16.0 * h->dim * B > 0.75 * (double)free_b) continue;
        // candidates come in increasing memory order: a larger one must win by 0.5 %
        const double ips = time_it(B, stk, 0, -1);
        all.push_back({B, ips, stk, 0, stream_hints(h->op, B) ? 1 : 0});
        if (ips > 1.005 * best.ips) best = {B, ips, stk, 0, -1};
    }
    // the winner's persistent workgroups per reducing multi-pass launch: half and twice
    // the default (results do not depend on it: the partial sums are exact)
    if (hv_mode(h->op) == 3 && (best.rhs_block == 1 || best.stacked)) {
        const int cap = pass_grid_cap(h->op);
        for (int pg : {cap / 2, 2 * cap}) {
            if (pg < 1 || pg > kMaxGrid) continue;
            const double ips = time_it(best.rhs_block, best.stacked, pg, -1);
            all.push_back({best.rhs_block, ips, best.stacked, pg, stream_hints(h->op, best.rhs_block) ? 1 : 0});
            if (ips > 1.005 * best.ips) best = {best.rhs_block, ips, best.stacked, pg, -1};
        }
        // and the other cache-hint set than the working-set rule's (results do not
        // depend on it either: hints and tile order only)
        if (forced_hints() < 0) {
            const int other = stream_hints(h->op, best.rhs_block) ? 0 : 1;
            const double ips = time_it(best.rhs_block, best.stacked, best.pass_grid, other);
            all.push_back({best.rhs_block, ips, best.stacked, best.pass_grid, other});
            if (ips > 1.005 * best.ips) best = {best.rhs_block, ips, best.stacked, best.pass_grid, other};
        }
    }
    g_tune[key] = best;
    g_tune_all[key] = all;
    if (path) tune_save(path);
    return best;
}

// One Green's sequence of a batched run: its output slot, the real shift of its
// resolvent (E_m), its shell vector and a tag for the right-hand-side loader.
struct GreenItem {
    int index;
    double Em;
    const double *phi;
    int tag;
};

struct GreenOut {
    std::vector<double> g;            // [nseq][nw] complex
    std::vector<double> alpha, beta;  // [nseq][n]
    std::vector<SeqState> states;     // [nseq]
};

// rhs_block and layout of a run: the autotuner's pick for rhs_block 0.  32
// sequences exist only as a stack.
void resolve_layout(const ftk_hamiltonian *h, int rhs_block, int n_omega, int &B, int &stack)
{
    B = rhs_block;
    stack = -1;
    if (B == 0) {
        const TuneResult t = autotune(h, n_omega);
        B = t.rhs_block;
        stack = t.stacked;
    } else {
        stack = tuned_layout(h->ctx->device, h->n_sites, n_omega, B);
    }
    if (B > 16)
        need(BatchRunner::stack_for(h, B, stack < 0 ? -1 : stack),
             "rhs_block 32 runs only as a stack of multi-pass sequences (N >= 16, stack_batch not 0, no plain loop)");
}

// Runs the items in batches of B through one graph-captured BatchRunner; load(run, r,
// item) writes the item's right-hand side into slot r.  Slots of sequences not listed
// stay zero.
template <class Load>
GreenOut run_green(const ftk_hamiltonian *h, int B, int stack, int n, const double *omega, int nw, double eta,
                   double rtol, int nseq, const std::vector<GreenItem> &work, Load &&load)
{
    ftk_ctx *ctx = h->ctx;
    hipStream_t s = ctx->stream;
    DevBuf gdev(ctx, sizeof(double) * 2 * (size_t)std::max(1, nseq) * nw);
    DevBuf adev(ctx, sizeof(double) * (size_t)std::max(1, nseq) * n), bdev(ctx, sizeof(double) * (size_t)std::max(1, nseq) * n);
    DevBuf sdev(ctx, sizeof(SeqState) * (size_t)std::max(1, nseq));
    HIP_CHECK(hipMemsetAsync(gdev.p, 0, gdev.n, s));
    HIP_CHECK(hipMemsetAsync(adev.p, 0, adev.n, s));
    HIP_CHECK(hipMemsetAsync(bdev.p, 0, bdev.n, s));
    HIP_CHECK(hipMemsetAsync(sdev.p, 0, sdev.n, s));
    if (!work.empty()) {
        const auto [pgrid, phints] = tuned_passes(h->ctx->device, h->n_sites, nw, B, stack);
        BatchRunner run(h, B, n, omega, nw, eta, rtol, stack, pgrid, phints);
        for (size_t w0 = 0; w0 < work.size(); w0 += B) {
            const int cnt = (int)std::min<size_t>(B, work.size() - w0);
            if (cnt < B) HIP_CHECK(hipMemsetAsync(run.chi.p, 0, run.chi.n, s));
            BatchShifts bs;
            for (int r = 0; r < kMaxBatch; ++r) bs.re[r] = 0.0;
            for (int r = 0; r < cnt; ++r) {
                load(run, r, work[w0 + r]);
                bs.re[r] = work[w0 + r].Em;
            }
            run.start(bs);
            run.run();
            for (int r = 0; r < cnt; ++r) {
                const GreenItem &q = work[w0 + r];
                launch_finish_green(run.states() + r, (ShiftState *)run.shifts.p + (size_t)r * nw, nw,
                                    gdev.d() + (size_t)q.index * 2 * nw, s);
                HIP_CHECK(hipMemcpyAsync(adev.d() + (size_t)q.index * n, run.al.d() + (size_t)r * n,
                                         sizeof(double) * n, hipMemcpyDeviceToDevice, s));
                HIP_CHECK(hipMemcpyAsync(bdev.d() + (size_t)q.index * n, run.be.d() + (size_t)r * n,
                                         sizeof(double) * n, hipMemcpyDeviceToDevice, s));
                HIP_CHECK(hipMemcpyAsync((SeqState *)sdev.p + q.index, run.states() + r, sizeof(SeqState),
                                         hipMemcpyDeviceToDevice, s));
            }
        }
    }
    HIP_CHECK(hipGetLastError());
    GreenOut out;
    out.g.resize((size_t)nseq * nw * 2);
    out.alpha.resize((size_t)nseq * n);
    out.beta.resize((size_t)nseq * n);
    out.states.resize(nseq);
    HIP_CHECK(hipMemcpyAsync(out.states.data(), sdev.p, sizeof(SeqState) * nseq, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(out.g.data(), gdev.p, sizeof(double) * out.g.size(), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(out.alpha.data(), adev.p, sizeof(double) * out.alpha.size(), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(out.beta.data(), bdev.p, sizeof(double) * out.beta.size(), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int i = 0; i < nseq; ++i)
        if (out.states[i].numeric_error) fail(FTK_ENUMERIC, "NaN/Inf in Green's-function Lanczos coefficients");
    return out;
}

// Shifted COCG sequences, one at a time: load(chi, lam, item) writes the right-hand
// side chi and, when it returns true, a projection vector lam (else lam = chi); the
// n-step complex-symmetric Lanczos loop with the per-shift recurrences, then
// g = <lam|x(z)>.
struct CocgOut {
    std::vector<double> g;         // [nseq][nw] complex
    std::vector<double> a, b, c;   // [nseq][n], [nseq][n], [nseq][n+1] complex
    std::vector<CocgState> states; // [nseq]
};

template <class Load>
CocgOut run_cocg(const ftk_hamiltonian *h, int n, const double *omega, int nw, double eta, double rtol,
                 double seed_tol, int nseq, const std::vector<GreenItem> &work, Load &&load)
{
    ftk_ctx *ctx = h->ctx;
    hipStream_t s = ctx->stream;
    const uint32_t dim = h->dim;
    const size_t vb = sizeof(double) * 2 * (size_t)dim;
    const double tol = 1e-12 * h->table.norm_bound;
    CocgOut out;
    out.g.assign((size_t)nseq * nw * 2, 0.0);
    out.a.assign((size_t)nseq * n * 2, 0.0);
    out.b.assign((size_t)nseq * n * 2, 0.0);
    out.c.assign((size_t)nseq * (n + 1) * 2, 0.0);
    out.states.assign(nseq, CocgState{});
    if (work.empty()) return out;
    DevBuf chi(ctx, vb), lamb(ctx, vb), W0(ctx, vb), W1(ctx, vb), Hw(ctx, vb), st(ctx, sizeof(CocgState)),
        sh(ctx, sizeof(CocgShift) * (size_t)nw), om(ctx, sizeof(double) * nw),
        partials(ctx, sizeof(double) * 10 * (size_t)kMaxGrid), ad(ctx, sizeof(double) * 2 * (size_t)n),
        bd(ctx, sizeof(double) * 2 * (size_t)n), cd(ctx, sizeof(double) * 2 * (size_t)(n + 1)),
        gd(ctx, sizeof(double) * 2 * (size_t)nw);
    HIP_CHECK(hipMemcpyAsync(om.p, omega, sizeof(double) * nw, hipMemcpyHostToDevice, s));
    double *W[2] = {W0.d(), W1.d()};
    for (const GreenItem &q : work) {
        const double *lam = load(chi.d(), lamb.d(), q) ? lamb.d() : chi.d();
        HIP_CHECK(hipMemsetAsync(ad.p, 0, ad.n, s));
        HIP_CHECK(hipMemsetAsync(bd.p, 0, bd.n, s));
        HIP_CHECK(hipMemsetAsync(cd.p, 0, cd.n, s));
        launch_cocg_start(dim, chi.d(), lam, partials.d(), (CocgState *)st.p, (CocgShift *)sh.p, nw, q.Em, cd.d(), s);
        for (int k = 0; k < n; ++k) {
            const double *cur = k == 0 ? chi.d() : W[(k - 1) % 2];
            const double *prv = k == 1 ? chi.d() : W[k % 2];
            launch_cocg_step(h->op, lam, cur, prv, W[k % 2], Hw.d(), partials.d(), (CocgState *)st.p,
                             (CocgShift *)sh.p, om.d(), nw, eta, k, tol, rtol, seed_tol, ad.d(), bd.d(), cd.d(), s);
        }
        launch_cocg_finish((const CocgState *)st.p, (const CocgShift *)sh.p, nw, gd.d(), s);
        const size_t i = (size_t)q.index;
        HIP_CHECK(hipMemcpyAsync(out.g.data() + i * nw * 2, gd.p, gd.n, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(out.a.data() + i * n * 2, ad.p, ad.n, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(out.b.data() + i * n * 2, bd.p, bd.n, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(out.c.data() + i * (n + 1) * 2, cd.p, cd.n, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(&out.states[i], st.p, sizeof(CocgState), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (out.states[i].numeric_error) fail(FTK_ENUMERIC, "NaN/Inf in shifted COCG coefficients");
    }
    HIP_CHECK(hipGetLastError());
    return out;
}

}  // namespace

extern "C" {

ftk_status ftk_autotune(const ftk_hamiltonian *h, int n_omega, int *rhs_block, double *iters_per_s)
{
    return guard([&] {
        need(h != nullptr, "h must not be NULL");
        need(n_omega >= 1, "n_omega must be >= 1");
        HIP_CHECK(hipSetDevice(h->ctx->device));
        TuneResult t = autotune(h, n_omega);
        if (rhs_block) *rhs_block = t.rhs_block;
        if (iters_per_s) *iters_per_s = t.ips;
    });
}

ftk_status ftk_autotune_candidates(const ftk_hamiltonian *h, int n_omega, int max_n, int *n, int *rhs_block,
                                   int *stacked, double *iters_per_s, int *pass_grid, int *hints)
{
    return guard([&] {
        need(h && n && rhs_block && stacked && iters_per_s && max_n >= 1, "bad arguments");
        HIP_CHECK(hipSetDevice(h->ctx->device));
        autotune(h, n_omega);
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune_all.find(tune_key(h->ctx->device, h->n_sites, n_omega));
        *n = 0;
        if (it == g_tune_all.end()) return;  // read from the cache file: no measurements in this process
        for (const TuneResult &t : it->second) {
            if (*n >= max_n) break;
            rhs_block[*n] = t.rhs_block;
            stacked[*n] = t.stacked;
            iters_per_s[*n] = t.ips;
            if (pass_grid) pass_grid[*n] = t.pass_grid;
            if (hints) hints[*n] = t.hints;
            ++*n;
        }
    });
}

ftk_status ftk_autotune_layout(const ftk_hamiltonian *h, int n_omega, int *stacked)
{
    return guard([&] {
        need(h != nullptr && stacked != nullptr, "NULL argument");
        need(n_omega >= 1, "n_omega must be >= 1");
        HIP_CHECK(hipSetDevice(h->ctx->device));
        *stacked = autotune(h, n_omega).stacked;
    });
}

ftk_status ftk_shifted_krylov_spectrum(const ftk_hamiltonian *h, const ftk_states *st,
                                       const ftk_spec_params *p, ftk_spectrum **out)
{
    return guard([&] {
        need(h && st && p && out, "NULL argument");
        need(st->h == h, "states were built with another Hamiltonian");
        need(p->n_q >= 1 && p->q_xy, "need at least one momentum");
        need((p->alpha_mask & 7) != 0 && (p->alpha_mask & ~7) == 0, "alpha_mask must be a non-empty subset of {x,y,z}");
        need(p->n_omega >= 1 && p->omega, "need at least one frequency");
        need(std::isfinite(p->eta) && p->eta > 0, "eta must be > 0");
        need(p->n_steps >= 1, "n_steps must be >= 1");
        need(valid_rhs_block(p->rhs_block), "rhs_block must be 0, 1, 2, 4, 8, 16 or 32");
        for (int i = 0; i < p->n_omega; ++i) need(std::isfinite(p->omega[i]), "omega must be finite");
        for (int i = 0; i < 2 * p->n_q; ++i) need(std::isfinite(p->q_xy[i]), "q must be finite");
        need(std::isfinite(p->resid_tol) && p->resid_tol >= 0, "resid_tol must be finite and >= 0");
        need(p->first_shell >= 0 && p->first_shell < st->L && p->n_shells >= 0 &&
                 p->n_shells <= st->L - p->first_shell,
             "shell range outside [0, L)");
        need(p->solver == FTK_SOLVER_LANCZOS || p->solver == FTK_SOLVER_COCG, "unknown solver");
        need(std::isfinite(p->seed_tol) && p->seed_tol >= 0, "seed_tol must be finite and >= 0");
        const bool cocg = p->solver == FTK_SOLVER_COCG;
        const int m_lo = p->first_shell, m_hi = p->n_shells ? p->first_shell + p->n_shells : st->L;
        ftk_ctx *ctx = h->ctx;
        HIP_CHECK(hipSetDevice(ctx->device));
        const uint32_t dim = h->dim;
        const int n = p->n_steps;
        int B = 1, stack = -1;
        if (!cocg) resolve_layout(h, p->rhs_block, p->n_omega, B, stack);
        int alphas[3], nal = 0;
        for (int a = 0; a < 3; ++a)
            if (p->alpha_mask & (1 << a)) alphas[nal++] = a;
        const int nq = p->n_q, nw = p->n_omega;
        const int nseq = st->nv * st->na * st->L * nal * nq;

        auto sp = std::make_unique<ftk_spectrum>();
        sp->st = st;
        sp->nalpha = nal;
        sp->nq = nq;
        sp->nw = nw;
        sp->n_steps = n;
        sp->resid.assign((size_t)nseq, 0.0);
        sp->chi2.assign((size_t)nseq, 0.0);
        sp->steps.assign((size_t)nseq, 0);

        std::vector<SqParams> sq((size_t)nal * nq);
        for (int ia = 0; ia < nal; ++ia)
            for (int iq = 0; iq < nq; ++iq) {
                SqParams &P = sq[(size_t)ia * nq + iq];
                std::memset(&P, 0, sizeof(P));
                P.n_sites = h->n_sites;
                P.alpha = alphas[ia];
                sq_coefficients(h->n_sites, h->site_xy.data(), p->q_xy[2 * iq], p->q_xy[2 * iq + 1], P.h);
            }
        // the sequences with a non-empty shell, in output order
        std::vector<GreenItem> work;
        int seq = 0;
        for (int sv = 0; sv < st->nv; ++sv)
            for (int a = 0; a < st->na; ++a) {
                const size_t sa = (size_t)sv * st->na + a;
                for (int m = 0; m < st->L; ++m) {
                    const double Em = shell_energy(st->E_b[a], st->eps[a], m);
                    const double *phim = st->phi[sa].d() + (size_t)m * 2 * dim;
                    const bool skip = !(st->n_m[sa * st->L + m] > 0.0) || m < m_lo || m >= m_hi;
                    for (int ia = 0; ia < nal; ++ia)
                        for (int iq = 0; iq < nq; ++iq, ++seq)
                            if (!skip) work.push_back({seq, Em, phim, ia * nq + iq});
                }
            }
        if (cocg) {
            sp->solver = FTK_SOLVER_COCG;
            CocgOut res = run_cocg(h, n, p->omega, nw, p->eta, p->resid_tol, p->seed_tol > 0 ? p->seed_tol : 1e-12,
                                   nseq, work, [&](double *chi, double *, const GreenItem &q) {
                                       launch_apply_sq(sq[q.tag], q.phi, chi, ctx->stream);
                                       return false;
                                   });
            sp->g = std::move(res.g);
            sp->ca = std::move(res.a);
            sp->cb = std::move(res.b);
            sp->cc = std::move(res.c);
            sp->seed.assign((size_t)nseq, 0);
            for (int i = 0; i < nseq; ++i) {
                sp->steps[i] = res.states[i].steps;
                sp->resid[i] = res.states[i].max_resid;
                sp->chi2[i] = res.states[i].norm2;
                sp->seed[i] = res.states[i].seed;
            }
            *out = sp.release();
            return;
        }
        GreenOut res = run_green(h, B, stack, n, p->omega, nw, p->eta, p->resid_tol, nseq, work,
                                 [&](BatchRunner &run, int r, const GreenItem &q) { run.load_rhs(sq[q.tag], q.phi, r); });
        sp->g = std::move(res.g);
        sp->alpha = std::move(res.alpha);
        sp->beta = std::move(res.beta);
        for (int i = 0; i < nseq; ++i) {
            sp->steps[i] = res.states[i].steps;
            sp->resid[i] = res.states[i].max_resid;
            sp->chi2[i] = res.states[i].norm2;
        }
        *out = sp.release();
    });
}

ftk_status ftk_spectrum_raw(const ftk_spectrum *sp, double *g, double *max_resid)
{
    return guard([&] {
        need(sp != nullptr, "sp must not be NULL");
        if (g) std::copy(sp->g.begin(), sp->g.end(), g);
        if (max_resid) std::copy(sp->resid.begin(), sp->resid.end(), max_resid);
    });
}

ftk_status ftk_spectrum_work(const ftk_spectrum *sp, int64_t *krylov_steps, int *sequences)
{
    return guard([&] {
        need(sp != nullptr, "sp must not be NULL");
        int64_t k = 0;
        int n = 0;
        for (int s : sp->steps)
            if (s > 0) {
                k += s;
                ++n;
            }
        if (krylov_steps) *krylov_steps = k;
        if (sequences) *sequences = n;
    });
}

ftk_status ftk_spectrum_norms(const ftk_spectrum *sp, double *chi2)
{
    return guard([&] {
        need(sp && chi2, "NULL argument");
        std::copy(sp->chi2.begin(), sp->chi2.end(), chi2);
    });
}

ftk_status ftk_spectrum_lanczos(const ftk_spectrum *sp, int s, int a, int m, int ia, int iq, double *alpha,
                                double *beta, int *n_steps)
{
    return guard([&] {
        need(sp != nullptr, "sp must not be NULL");
        need(sp->solver == FTK_SOLVER_LANCZOS, "a shifted COCG spectrum has no Hermitian Lanczos coefficients");
        const ftk_states *st = sp->st;
        need(s >= 0 && s < st->nv && a >= 0 && a < st->na && m >= 0 && m < st->L && ia >= 0 && ia < sp->nalpha &&
                 iq >= 0 && iq < sp->nq,
             "index out of range");
        const size_t seq = (((((size_t)s * st->na + a) * st->L + m) * sp->nalpha + ia) * sp->nq + iq);
        const int k = sp->steps[seq];
        if (n_steps) *n_steps = k;
        if (alpha) std::copy(sp->alpha.begin() + seq * sp->n_steps, sp->alpha.begin() + seq * sp->n_steps + k, alpha);
        if (beta) std::copy(sp->beta.begin() + seq * sp->n_steps, sp->beta.begin() + seq * sp->n_steps + k, beta);
    });
}

ftk_status ftk_spectrum_cocg(const ftk_spectrum *sp, int s, int a, int m, int ia, int iq, double *a_out,
                             double *b_out, double *c_out, int *n_steps, int *seed)
{
    return guard([&] {
        need(sp != nullptr, "sp must not be NULL");
        need(sp->solver == FTK_SOLVER_COCG, "not a shifted COCG spectrum");
        const ftk_states *st = sp->st;
        need(s >= 0 && s < st->nv && a >= 0 && a < st->na && m >= 0 && m < st->L && ia >= 0 && ia < sp->nalpha &&
                 iq >= 0 && iq < sp->nq,
             "index out of range");
        const size_t seq = (((((size_t)s * st->na + a) * st->L + m) * sp->nalpha + ia) * sp->nq + iq);
        const int k = sp->steps[seq], n = sp->n_steps;
        if (n_steps) *n_steps = k;
        if (seed) *seed = sp->seed[seq];
        if (a_out) std::copy(sp->ca.begin() + seq * n * 2, sp->ca.begin() + seq * n * 2 + 2 * k, a_out);
        if (b_out) std::copy(sp->cb.begin() + seq * n * 2, sp->cb.begin() + seq * n * 2 + 2 * k, b_out);
        if (c_out)
            std::copy(sp->cc.begin() + seq * (n + 1) * 2, sp->cc.begin() + seq * (n + 1) * 2 + 2 * (k + 1), c_out);
    });
}

ftk_status ftk_spectrum_destroy(ftk_spectrum *sp)
{
    return guard([&] { delete sp; });
}

ftk_status ftk_pair_green(const ftk_hamiltonian *h, const ftk_states *st, const ftk_pair_params *p,
                          ftk_pair_spectrum **out)
{
    return guard([&] {
        need(h && st && p && out, "NULL argument");
        need(st->h == h, "states were built with another Hamiltonian");
        need(p->n_pairs >= 1 && p->op_a && p->op_b, "need at least one operator pair");
        need(p->n_omega >= 1 && p->omega, "need at least one frequency");
        need(std::isfinite(p->eta) && p->eta > 0, "eta must be > 0");
        need(p->n_steps >= 1, "n_steps must be >= 1");
        need(valid_rhs_block(p->rhs_block), "rhs_block must be 0, 1, 2, 4, 8, 16 or 32");
        need(std::isfinite(p->resid_tol) && p->resid_tol >= 0, "resid_tol must be finite and >= 0");
        need(p->solver == FTK_SOLVER_LANCZOS || p->solver == FTK_SOLVER_COCG, "unknown solver");
        need(std::isfinite(p->seed_tol) && p->seed_tol >= 0, "seed_tol must be finite and >= 0");
        for (int i = 0; i < p->n_omega; ++i) need(std::isfinite(p->omega[i]), "omega must be finite");
        const int N = h->n_sites, np = p->n_pairs, nw = p->n_omega, n = p->n_steps;
        const size_t ncoef = (size_t)np * N * 3 * 2;
        for (size_t i = 0; i < ncoef; ++i)
            need(std::isfinite(p->op_a[i]) && std::isfinite(p->op_b[i]), "operator coefficients must be finite");
        ftk_ctx *ctx = h->ctx;
        HIP_CHECK(hipSetDevice(ctx->device));
        const uint32_t dim = h->dim;
        const bool cocg = p->solver == FTK_SOLVER_COCG;
        int B = 1, stack = -1;
        if (!cocg) resolve_layout(h, p->rhs_block, nw, B, stack);

        // S = sigma / 2: the per-site factors are half the coefficients
        std::vector<SpinOpParams> opa(np), opb(np);
        for (int q = 0; q < np; ++q)
            for (int which = 0; which < 2; ++which) {
                SpinOpParams &P = which == 0 ? opa[q] : opb[q];
                const double *c = (which == 0 ? p->op_a : p->op_b) + (size_t)q * N * 6;
                std::memset(&P, 0, sizeof(P));
                P.n_sites = N;
                for (int l = 0; l < N; ++l)
                    for (int a = 0; a < 3; ++a) {
                        P.h[a][2 * l] = 0.5 * c[(l * 3 + a) * 2];
                        P.h[a][2 * l + 1] = 0.5 * c[(l * 3 + a) * 2 + 1];
                    }
            }
        const int npair_total = st->nv * st->na * st->L * np;  // (vector, anchor, shell, pair)
        if (cocg) {
            // shifted BiCG with the shadow conj(rho) (COCG): G_AB = <lam|x(z)> from the run on
            // rho = B phi^m projected on lam = A phi^m, G_BA from the run on lam projected on rho
            std::vector<GreenItem> work;
            for (int sv = 0, i = 0; sv < st->nv; ++sv)
                for (int a = 0; a < st->na; ++a) {
                    const size_t sa = (size_t)sv * st->na + a;
                    for (int m = 0; m < st->L; ++m) {
                        const double Em = shell_energy(st->E_b[a], st->eps[a], m);
                        const double *phim = st->phi[sa].d() + (size_t)m * 2 * dim;
                        const bool empty = !(st->n_m[sa * st->L + m] > 0.0);
                        for (int q = 0; q < np; ++q, ++i)
                            for (int k = 0; k < 2; ++k)
                                if (!empty) work.push_back({2 * i + k, Em, phim, 2 * q + k});
                    }
                }
            CocgOut res = run_cocg(h, n, p->omega, nw, p->eta, p->resid_tol, p->seed_tol > 0 ? p->seed_tol : 1e-12,
                                   2 * npair_total, work, [&](double *chi, double *lam, const GreenItem &q) {
                                       const int pair = q.tag / 2;
                                       const bool ab = q.tag % 2 == 0;
                                       launch_apply_spin_op(ab ? opb[pair] : opa[pair], q.phi, chi, ctx->stream);
                                       launch_apply_spin_op(ab ? opa[pair] : opb[pair], q.phi, lam, ctx->stream);
                                       return true;
                                   });
            auto sp = std::make_unique<ftk_pair_spectrum>();
            sp->st = st;
            sp->np = np;
            sp->nw = nw;
            sp->n_steps = n;
            sp->solver = FTK_SOLVER_COCG;
            sp->gab.assign((size_t)npair_total * nw * 2, 0.0);
            sp->gba.assign((size_t)npair_total * nw * 2, 0.0);
            sp->overlap.assign((size_t)npair_total * 2, 0.0);
            sp->resid.assign((size_t)npair_total, 0.0);
            sp->steps.assign((size_t)2 * npair_total, 0);
            sp->seed.assign((size_t)2 * npair_total, 0);
            for (int i = 0; i < npair_total; ++i) {
                std::copy(res.g.begin() + (size_t)(2 * i) * nw * 2, res.g.begin() + (size_t)(2 * i + 1) * nw * 2,
                          sp->gab.begin() + (size_t)i * nw * 2);
                std::copy(res.g.begin() + (size_t)(2 * i + 1) * nw * 2, res.g.begin() + (size_t)(2 * i + 2) * nw * 2,
                          sp->gba.begin() + (size_t)i * nw * 2);
                // <lam|rho> = c_0 delta_0 of the run on rho (c_0 = <lam|q_0>, q_0 = rho/delta_0)
                const CocgState &q = res.states[2 * i];
                const double c0r = res.c[(size_t)(2 * i) * (n + 1) * 2], c0i = res.c[(size_t)(2 * i) * (n + 1) * 2 + 1];
                sp->overlap[2 * i] = c0r * q.d0r - c0i * q.d0i;
                sp->overlap[2 * i + 1] = c0r * q.d0i + c0i * q.d0r;
                sp->resid[i] = std::max(res.states[2 * i].max_resid, res.states[2 * i + 1].max_resid);
                for (int k = 0; k < 2; ++k) {
                    sp->steps[2 * i + k] = res.states[2 * i + k].steps;
                    sp->seed[2 * i + k] = res.states[2 * i + k].seed;
                }
            }
            sp->ca = std::move(res.a);
            sp->cb = std::move(res.b);
            sp->cc = std::move(res.c);
            *out = sp.release();
            return;
        }
        const int nseq = 4 * npair_total;
        std::vector<GreenItem> work;
        for (int sv = 0, i = 0; sv < st->nv; ++sv)
            for (int a = 0; a < st->na; ++a) {
                const size_t sa = (size_t)sv * st->na + a;
                for (int m = 0; m < st->L; ++m) {
                    const double Em = shell_energy(st->E_b[a], st->eps[a], m);
                    const double *phim = st->phi[sa].d() + (size_t)m * 2 * dim;
                    const bool empty = !(st->n_m[sa * st->L + m] > 0.0);
                    for (int q = 0; q < np; ++q, ++i)
                        for (int k = 0; k < 4; ++k)
                            if (!empty) work.push_back({4 * i + k, Em, phim, 4 * q + k});
                }
            }
        // lam = A phi^m and rho = B phi^m of the pair being loaded
        DevBuf lam(ctx, sizeof(double) * 2 * (size_t)dim), rho(ctx, sizeof(double) * 2 * (size_t)dim);
        const double *cur_phi = nullptr;
        int cur_pair = -1;
        GreenOut res = run_green(h, B, stack, n, p->omega, nw, p->eta, p->resid_tol, nseq, work,
                                 [&](BatchRunner &run, int r, const GreenItem &q) {
                                     const int pair = q.tag / 4;
                                     if (q.phi != cur_phi || pair != cur_pair) {
                                         launch_apply_spin_op(opa[pair], q.phi, lam.d(), ctx->stream);
                                         launch_apply_spin_op(opb[pair], q.phi, rho.d(), ctx->stream);
                                         cur_phi = q.phi;
                                         cur_pair = pair;
                                     }
                                     run.load_polarized(q.tag % 4, lam.d(), rho.d(), r);
                                 });

        auto sp = std::make_unique<ftk_pair_spectrum>();
        sp->st = st;
        sp->np = np;
        sp->nw = nw;
        sp->n_steps = n;
        sp->gab.assign((size_t)npair_total * nw * 2, 0.0);
        sp->gba.assign((size_t)npair_total * nw * 2, 0.0);
        sp->overlap.assign((size_t)npair_total * 2, 0.0);
        sp->resid.assign((size_t)npair_total, 0.0);
        sp->steps.assign((size_t)nseq, 0);
        for (int i = 0; i < npair_total; ++i) {
            // polarization identity: G_AB = (g0 - g1 - i g2 + i g3) / 4, G_BA with +i, -i
            const double *g0 = res.g.data() + (size_t)(4 * i) * nw * 2;
            const double *g1 = g0 + (size_t)nw * 2, *g2 = g1 + (size_t)nw * 2, *g3 = g2 + (size_t)nw * 2;
            double *ab = sp->gab.data() + (size_t)i * nw * 2, *ba = sp->gba.data() + (size_t)i * nw * 2;
            for (int j = 0; j < nw; ++j) {
                const double d_re = g0[2 * j] - g1[2 * j], d_im = g0[2 * j + 1] - g1[2 * j + 1];
                const double e_re = g2[2 * j + 1] - g3[2 * j + 1], e_im = g2[2 * j] - g3[2 * j];
                ab[2 * j] = 0.25 * (d_re + e_re);
                ab[2 * j + 1] = 0.25 * (d_im - e_im);
                ba[2 * j] = 0.25 * (d_re - e_re);
                ba[2 * j + 1] = 0.25 * (d_im + e_im);
            }
            const SeqState *q = res.states.data() + 4 * i;
            sp->overlap[2 * i] = 0.25 * (q[0].norm2 - q[1].norm2);
            sp->overlap[2 * i + 1] = 0.25 * (q[3].norm2 - q[2].norm2);
            double r = 0.0;
            for (int k = 0; k < 4; ++k) r = std::max(r, q[k].max_resid);
            sp->resid[i] = r;
        }
        for (int i = 0; i < nseq; ++i) sp->steps[i] = res.states[i].steps;
        sp->alpha = std::move(res.alpha);
        sp->beta = std::move(res.beta);
        *out = sp.release();
    });
}

ftk_status ftk_pair_raw(const ftk_pair_spectrum *sp, double *g_ab, double *g_ba, double *overlap, double *max_resid)
{
    return guard([&] {
        need(sp != nullptr, "sp must not be NULL");
        if (g_ab) std::copy(sp->gab.begin(), sp->gab.end(), g_ab);
        if (g_ba) std::copy(sp->gba.begin(), sp->gba.end(), g_ba);
        if (overlap) std::copy(sp->overlap.begin(), sp->overlap.end(), overlap);
        if (max_resid) std::copy(sp->resid.begin(), sp->resid.end(), max_resid);
    });
}

ftk_status ftk_pair_lanczos(const ftk_pair_spectrum *sp, int s, int a, int m, int p, int k, double *alpha,
                            double *beta, int *n_steps)
{
    return guard([&] {
        need(sp != nullptr, "sp must not be NULL");
        need(sp->solver == FTK_SOLVER_LANCZOS, "a shifted COCG pair spectrum has no polarization sequences");
        const ftk_states *st = sp->st;
        need(s >= 0 && s < st->nv && a >= 0 && a < st->na && m >= 0 && m < st->L && p >= 0 && p < sp->np && k >= 0 &&
                 k < 4,
             "index out of range");
        const size_t seq = ((((size_t)s * st->na + a) * st->L + m) * sp->np + p) * 4 + k;
        const int kk = sp->steps[seq];
        if (n_steps) *n_steps = kk;
        if (alpha) std::copy(sp->alpha.begin() + seq * sp->n_steps, sp->alpha.begin() + seq * sp->n_steps + kk, alpha);
        if (beta) std::copy(sp->beta.begin() + seq * sp->n_steps, sp->beta.begin() + seq * sp->n_steps + kk, beta);
    });
}

ftk_status ftk_pair_cocg(const ftk_pair_spectrum *sp, int s, int a, int m, int p, int k, double *a_out,
                         double *b_out, double *c_out, int *n_steps, int *seed)
{
    return guard([&] {
        need(sp != nullptr, "sp must not be NULL");
        need(sp->solver == FTK_SOLVER_COCG, "not a shifted COCG pair spectrum");
        const ftk_states *st = sp->st;
        need(s >= 0 && s < st->nv && a >= 0 && a < st->na && m >= 0 && m < st->L && p >= 0 && p < sp->np && k >= 0 &&
                 k < 2,
             "index out of range");
        const size_t seq = ((((size_t)s * st->na + a) * st->L + m) * sp->np + p) * 2 + k;
        const int kk = sp->steps[seq], n = sp->n_steps;
        if (n_steps) *n_steps = kk;
        if (seed) *seed = sp->seed[seq];
        if (a_out) std::copy(sp->ca.begin() + seq * n * 2, sp->ca.begin() + seq * n * 2 + 2 * kk, a_out);
        if (b_out) std::copy(sp->cb.begin() + seq * n * 2, sp->cb.begin() + seq * n * 2 + 2 * kk, b_out);
        if (c_out)
            std::copy(sp->cc.begin() + seq * (n + 1) * 2, sp->cc.begin() + seq * (n + 1) * 2 + 2 * (kk + 1), c_out);
    });
}

ftk_status ftk_pair_destroy(ftk_pair_spectrum *sp)
{
    return guard([&] { delete sp; });
}

ftk_status ftk_reweight_observable(int nv, int na, int L, int n_obs, const double *betas, const double *E_m,
                                  const double *log_norm, const double *n_m, const double *O, const double *T, int nT,
                                  int n_bins, double *out, double *err)
{
    return guard([&] {
        need(nv >= 1 && na >= 1 && L >= 1 && n_obs >= 1 && nT >= 1, "sizes must be >= 1");
        need(betas && E_m && log_norm && n_m && O && T && out, "NULL argument");
        for (int i = 0; i < nT; ++i) need(std::isfinite(T[i]) && T[i] > 0, "T must be finite and > 0");
        for (int a = 0; a < na; ++a) need(std::isfinite(betas[a]) && betas[a] >= 0, "anchor beta must be >= 0");
        reweight_observable(nv, na, L, n_obs, betas, E_m, log_norm, n_m, O, T, nT, n_bins, out, err);
    });
}

ftk_status ftk_thermodynamics(int nv, int na, int L, const double *betas, const double *E_m, const double *log_norm,
                              const double *n_m, const double *h1, const double *h2, int n_sites, const double *T,
                              int nT, int n_bins, double *out, double *err)
{
    return guard([&] {
        need(nv >= 1 && na >= 1 && L >= 1 && nT >= 1, "sizes must be >= 1");
        need(n_sites >= 1 && n_sites <= 1000, "n_sites out of range");
        need(betas && E_m && log_norm && n_m && T && out, "NULL argument");
        for (int i = 0; i < nT; ++i) need(std::isfinite(T[i]) && T[i] > 0, "T must be finite and > 0");
        for (int a = 0; a < na; ++a) need(std::isfinite(betas[a]) && betas[a] >= 0, "anchor beta must be >= 0");
        thermodynamics(nv, na, L, betas, E_m, log_norm, n_m, h1, h2, n_sites, T, nT, n_bins, out, err);
    });
}

ftk_status ftk_thermo_diagnostics(int nv, int na, int L, const double *betas, const double *E_m,
                                  const double *log_norm, const double *n_m, const double *h1, const double *h2,
                                  int n_sites, const double *inv_T, int nT, int n_bins, double *out, double *err)
{
    return guard([&] {
        need(nv >= 1 && na >= 1 && L >= 1 && nT >= 1, "sizes must be >= 1");
        need(n_sites >= 1 && n_sites <= 1000, "n_sites out of range");
        need(betas && E_m && log_norm && n_m && inv_T && out, "NULL argument");
        for (int i = 0; i < nT; ++i)
            need(std::isfinite(inv_T[i]) && inv_T[i] >= 0, "inverse temperatures must be finite and >= 0");
        for (int a = 0; a < na; ++a) need(std::isfinite(betas[a]) && betas[a] >= 0, "anchor beta must be >= 0");
        thermo_diagnostics(nv, na, L, betas, E_m, log_norm, n_m, h1, h2, n_sites, inv_T, nT, n_bins, out, err);
    });
}

ftk_status ftk_choose_anchors(int n, const double *beta_grid, const double *E, const double *var, double r_max,
                              int max_anchors, int *anchors, int *n_anchors)
{
    return guard([&] {
        need(n >= 1 && beta_grid && E && var && anchors && n_anchors, "bad arguments");
        need(max_anchors >= 1, "max_anchors must be >= 1");
        need(std::isfinite(r_max) && r_max > 0, "r_max must be > 0");
        for (int i = 0; i < n; ++i) {
            need(std::isfinite(beta_grid[i]) && beta_grid[i] >= 0, "grid must be finite inverse temperatures >= 0");
            need(i == 0 || beta_grid[i] > beta_grid[i - 1], "grid must be ascending in beta");
            need(std::isfinite(E[i]) && std::isfinite(var[i]) && var[i] >= 0, "E and var must be finite, var >= 0");
        }
        *n_anchors = choose_anchors(n, E, var, r_max, max_anchors, anchors);
    });
}

ftk_status ftk_fit_asymmetric_lorentzian(const double *omega, const double *s, int n, double lo, double hi,
                                         const double *init, int max_iter, double *params, double *cost,
                                         int *iters, double *width_ratio)
{
    return guard([&] {
        need(omega && s && params && n >= 0, "bad arguments");
        need(std::isfinite(lo) && std::isfinite(hi) && lo <= hi, "need a finite window lo <= hi");
        need(max_iter >= 0, "max_iter must be >= 0");
        std::vector<double> w, y;
        for (int i = 0; i < n; ++i)
            if (omega[i] >= lo && omega[i] <= hi) {
                need(std::isfinite(s[i]), "spectrum values in the window must be finite");
                need(w.empty() || omega[i] > w.back(), "omega must be ascending in the window");
                w.push_back(omega[i]);
                y.push_back(s[i]);
            }
        const int m = (int)w.size();
        need(m >= 5, "fewer than 5 points in the window");
        double p[5];
        if (init) {
            for (int j = 0; j < 5; ++j) need(std::isfinite(init[j]), "init must be finite");
            need(init[3] != 0, "init gamma must be nonzero");
            std::memcpy(p, init, sizeof p);
        } else {
            asym_lorentzian_start(w.data(), y.data(), m, p);
            need(p[3] > 0 && p[0] > 0, "no positive peak in the window");
        }
        double f = 0;
        const int it = fit_asym_lorentzian(w.data(), y.data(), m, max_iter ? max_iter : 1000, p, &f);
        for (int j = 0; j < 5; ++j)
            if (!std::isfinite(p[j])) fail(FTK_ENUMERIC, "the fit left finite numbers");
        std::memcpy(params, p, sizeof p);
        if (cost) *cost = f;
        if (iters) *iters = it;
        if (width_ratio) *width_ratio = p[4] != 0.0 ? p[3] / p[4] : HUGE_VAL;
    });
}

ftk_status ftk_reweight(int nv, int na, int L, int nq, int nw, const double *betas, const double *E_m,
                        const double *eps, const double *log_norm, const double *n_m, const double *g,
                        const double *T, int nT, int n_bins, double *S, double *S_err, double *P)
{
    return guard([&] {
        need(nv >= 1 && na >= 1 && L >= 1 && nq >= 1 && nw >= 1 && nT >= 1, "sizes must be >= 1");
        need(betas && E_m && eps && log_norm && n_m && g && T && S, "NULL argument");
        for (int i = 0; i < nT; ++i) need(std::isfinite(T[i]) && T[i] > 0, "T must be finite and > 0");
        for (int a = 0; a < na; ++a) need(betas[a] >= 0 && eps[a] > 0, "anchor beta >= 0 and eps > 0 required");
        reweight(nv, na, L, nq, nw, betas, E_m, eps, log_norm, n_m, g, T, nT, n_bins, S, S_err, P);
    });
}

ftk_status ftk_reweight_spectrum(const ftk_states *st, const ftk_spectrum *sp, const double *T, int nT, int n_bins,
                                 double *S, double *S_err, double *P)
{
    return guard([&] {
        need(st && sp && T && S, "NULL argument");
        need(sp->st == st, "the spectrum was computed from other states");
        need(nT >= 1, "n_T must be >= 1");
        for (int i = 0; i < nT; ++i) need(std::isfinite(T[i]) && T[i] > 0, "T must be finite and > 0");
        const int nv = st->nv, na = st->na, L = st->L, nq = sp->nq, nw = sp->nw, nal = sp->nalpha;
        // g summed over alpha in x, y, z order: [nv][na][L][nq][nw]
        std::vector<double> g((size_t)nv * na * L * nq * nw * 2, 0.0);
        for (size_t sal = 0; sal < (size_t)nv * na * L; ++sal)
            for (int ia = 0; ia < nal; ++ia)
                for (int iq = 0; iq < nq; ++iq)
                    for (int j = 0; j < nw; ++j)
                        for (int c = 0; c < 2; ++c) {
                            const size_t src = ((((sal * nal + ia) * nq + iq) * nw + j) * 2 + c);
                            const size_t dst = (((sal * nq + iq) * nw + j) * 2 + c);
                            g[dst] = g[dst] + sp->g[src];
                        }
        std::vector<double> Em((size_t)na * L);
        for (int a = 0; a < na; ++a)
            for (int m = 0; m < L; ++m) Em[(size_t)a * L + m] = shell_energy(st->E_b[a], st->eps[a], m);
        reweight(nv, na, L, nq, nw, st->betas.data(), Em.data(), st->eps.data(), st->log_norm.data(), st->n_m.data(),
                 g.data(), T, nT, n_bins, S, S_err, P);
    });
}

ftk_status ftk_reweight_pair(int nv, int na, int L, int np, int nw, const double *betas, const double *E_m,
                             const double *eps, const double *log_norm, const double *n_m, const double *g_ab,
                             const double *g_ba, const double *T, int nT, int n_bins, double *S, double *S_err)
{
    return guard([&] {
        need(nv >= 1 && na >= 1 && L >= 1 && np >= 1 && nw >= 1 && nT >= 1, "sizes must be >= 1");
        need(betas && E_m && eps && log_norm && n_m && g_ab && g_ba && T && S, "NULL argument");
        for (int i = 0; i < nT; ++i) need(std::isfinite(T[i]) && T[i] > 0, "T must be finite and > 0");
        for (int a = 0; a < na; ++a) need(betas[a] >= 0 && eps[a] > 0, "anchor beta >= 0 and eps > 0 required");
        // X = (G_AB - conj(G_BA)) / 2: Re S_AB is the reweighted -(1/pi) Im X, Im S_AB
        // minus that of i X
        const size_t ng = (size_t)nv * na * L * np * nw;
        std::vector<double> X(2 * ng), iX(2 * ng);
        for (size_t i = 0; i < ng; ++i) {
            const double xr = 0.5 * (g_ab[2 * i] - g_ba[2 * i]);
            const double xi = 0.5 * (g_ab[2 * i + 1] + g_ba[2 * i + 1]);
            X[2 * i] = xr;
            X[2 * i + 1] = xi;
            iX[2 * i] = -xi;
            iX[2 * i + 1] = xr;
        }
        const size_t nout = (size_t)np * nT * nw;
        std::vector<double> sr(nout), si(nout), er(nout), ei(nout);
        reweight(nv, na, L, np, nw, betas, E_m, eps, log_norm, n_m, X.data(), T, nT, n_bins, sr.data(), er.data(),
                 nullptr);
        reweight(nv, na, L, np, nw, betas, E_m, eps, log_norm, n_m, iX.data(), T, nT, n_bins, si.data(), ei.data(),
                 nullptr);
        for (size_t i = 0; i < nout; ++i) {
            S[2 * i] = sr[i];
            S[2 * i + 1] = -si[i];
            if (S_err) {
                S_err[2 * i] = er[i];
                S_err[2 * i + 1] = ei[i];
            }
        }
    });
}

ftk_status ftk_momentum_operator(int n_sites, const double *site_xy, int alpha, double qx, double qy, double *coef)
{
    return guard([&] {
        need(n_sites >= 1 && n_sites <= kMaxSites && site_xy && coef, "bad arguments");
        need(alpha >= 0 && alpha <= 2, "alpha must be 0, 1 or 2");
        need(std::isfinite(qx) && std::isfinite(qy), "q must be finite");
        std::vector<double> h(2 * (size_t)n_sites);
        sq_coefficients(n_sites, site_xy, qx, qy, h.data());  // e^{iQ.R_l} / (2 sqrt N)
        std::fill(coef, coef + 6 * (size_t)n_sites, 0.0);
        for (int l = 0; l < n_sites; ++l) {
            coef[(l * 3 + alpha) * 2] = 2.0 * h[2 * l];
            coef[(l * 3 + alpha) * 2 + 1] = 2.0 * h[2 * l + 1];
        }
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One Green's-function sequence that can stop after any step, go to host memory and
// resume, in this process or another: after k steps its state is (w_{k-1}, w_{k-2}
// (chi stands in for w_{-1}), the sequence scalars, alpha_0..alpha_{k-1},
// beta_1..beta_k, the per-shift LDL^T state).  Steps run in chunks; a chunk ends with
// both halves of its last step and the next chunk starts with an unfused step.
// Every reduction is an exact sum rounded once, so the split of the work does not
// change a bit: a resumed sequence equals the straight run.
struct ftk_green_seq {
    const ftk_hamiltonian *h = nullptr;
    int n_max = 0, nw = 0, k = 0;  // k: steps run so far (both halves)
    double eta = 0, shift_re = 0;
    DevBuf chi, W0, W1, st, al, be, shifts, omega, partials, partials_b, g;
    std::vector<double> omega_h;
};

namespace {

constexpr char kSeqMagic[8] = {'F', 'T', 'K', 'G', 'S', 'Q', '0', '1'};

struct SeqBlobHeader {
    char magic[8];
    uint64_t h_hash;   // of the Hamiltonian's bond table
    int32_t n_sites, n_max, nw, k;
    double eta, shift_re;
    uint64_t payload_bytes;
    uint64_t payload_hash;
};

// omega, scalars, shift states, alpha, beta, two vectors
size_t seq_payload_bytes(uint32_t dim, int nw, int n_max)
{
    return sizeof(double) * (size_t)nw + sizeof(SeqState) + sizeof(ShiftState) * (size_t)nw +
           2 * sizeof(double) * (size_t)n_max + 2 * sizeof(double) * 2 * (size_t)dim;
}

// FNV-1a over 64-bit words (a trailing partial word is zero-padded)
uint64_t fnv64(const void *p, size_t bytes, uint64_t h = 1469598103934665603ull)
{
    const unsigned char *c = (const unsigned char *)p;
    size_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
        uint64_t w;
        std::memcpy(&w, c + i, 8);
        h = (h ^ w) * 1099511628211ull;
    }
    if (i < bytes) {
        uint64_t w = 0;
        std::memcpy(&w, c + i, bytes - i);
        h = (h ^ w) * 1099511628211ull;
    }
    return h;
}

uint64_t table_hash(const ftk_hamiltonian *h)
{
    const BondTable &t = h->table;
    uint64_t x = fnv64(&t.n_sites, sizeof(int));
    x = fnv64(&t.n_bonds, sizeof(int), x);
    x = fnv64(t.bi, sizeof(int32_t) * t.n_bonds, x);
    x = fnv64(t.bj, sizeof(int32_t) * t.n_bonds, x);
    x = fnv64(t.ap, sizeof(double) * t.n_bonds, x);
    x = fnv64(t.aa, sizeof(double) * t.n_bonds, x);
    x = fnv64(&t.jq, sizeof(double), x);
    return fnv64(&t.kq, sizeof(double), x);
}

std::unique_ptr<ftk_green_seq> seq_alloc(const ftk_hamiltonian *h, const double *omega, int nw, double eta,
                                         double shift_re, int n_max)
{
    need(nw >= 1 && n_max >= 1, "n_omega and n_max must be >= 1");
    need(std::isfinite(eta) && eta > 0, "eta must be finite and > 0");
    need(std::isfinite(shift_re), "shift_re must be finite");
    for (int j = 0; j < nw; ++j) need(std::isfinite(omega[j]), "omega must be finite");
    HIP_CHECK(hipSetDevice(h->ctx->device));
    auto q = std::make_unique<ftk_green_seq>();
    ftk_ctx *c = h->ctx;
    const size_t vb = sizeof(double) * 2 * (size_t)h->dim;
    q->h = h;
    q->n_max = n_max;
    q->nw = nw;
    q->eta = eta;
    q->shift_re = shift_re;
    q->chi = DevBuf(c, vb);
    q->W0 = DevBuf(c, vb);
    q->W1 = DevBuf(c, vb);
    q->st = DevBuf(c, sizeof(SeqState));
    q->al = DevBuf(c, sizeof(double) * (size_t)n_max);
    q->be = DevBuf(c, sizeof(double) * (size_t)n_max);
    q->shifts = DevBuf(c, sizeof(ShiftState) * (size_t)nw);
    q->omega = DevBuf(c, sizeof(double) * (size_t)nw);
    q->partials = DevBuf(c, sizeof(double) * 2 * (size_t)kMaxGrid);
    q->partials_b = DevBuf(c, sizeof(double) * 2 * (size_t)kMaxGrid);
    q->g = DevBuf(c, sizeof(double) * 2 * (size_t)nw);
    q->omega_h.assign(omega, omega + nw);
    HIP_CHECK(hipMemcpyAsync(q->omega.p, omega, sizeof(double) * nw, hipMemcpyHostToDevice, c->stream));
    // states saved before their first step hold zeros, not stale memory
    HIP_CHECK(hipMemsetAsync(q->shifts.p, 0, q->shifts.n, c->stream));
    HIP_CHECK(hipMemsetAsync(q->al.p, 0, q->al.n, c->stream));
    HIP_CHECK(hipMemsetAsync(q->be.p, 0, q->be.n, c->stream));
    return q;
}

SeqState seq_state(const ftk_green_seq *q)
{
    SeqState r;
    HIP_CHECK(hipMemcpyAsync(&r, q->st.p, sizeof(SeqState), hipMemcpyDeviceToHost, q->h->ctx->stream));
    HIP_CHECK(hipStreamSynchronize(q->h->ctx->stream));
    return r;
}

// the vectors the next step reads: v_k from cur = w_{k-1}, v_{k-1} from prv = w_{k-2}
const double *seq_cur(const ftk_green_seq *q) { return q->k == 0 ? q->chi.d() : (q->k % 2 ? q->W0.d() : q->W1.d()); }
const double *seq_prv(const ftk_green_seq *q) { return q->k <= 1 ? q->chi.d() : (q->k % 2 ? q->W1.d() : q->W0.d()); }

// steps k .. k1-1 of the sequence, both halves of the last one included
void seq_chunk(ftk_green_seq *q, int k1)
{
    const ftk_hamiltonian *h = q->h;
    hipStream_t s = h->ctx->stream;
    const uint32_t dim = h->dim;
    const int nparts = vec_grid(dim), nparts_hv = hv_grid(h->op);
    const double tol = 1e-12 * h->table.norm_bound;
    double *W[2] = {q->W0.d(), q->W1.d()};
    SeqState *st = (SeqState *)q->st.p;
    ShiftState *sh = (ShiftState *)q->shifts.p;
    const bool fuse = lanczos_fusable(h->op) && !g_plain_loop;
    const bool fa_on = fuse && alpha_in_fused_pass();
    double *pa = q->partials.d(), *pb = fa_on ? q->partials_b.d() : q->partials.d();
    const int k0 = q->k;
    for (int k = k0; k < k1; ++k) {
        const double *cur = k == 0 ? q->chi.d() : W[(k - 1) % 2];
        const double *prv = k == 1 ? q->chi.d() : W[k % 2];
        double *out = W[k % 2];
        if (fuse && k > k0) {
            const FinAlpha fa{pa, nparts_hv, q->al.d(), 0, k - 1};
            launch_lanczos_fused_first(h->op, W[(k - 1) % 2], prv, st, pb, s, Stack(), fa_on ? &fa : nullptr);
            const FinBeta fb{st, pb, nparts_hv, q->be.d(), k - 1, tol, sh, q->omega.d(), q->nw, q->eta, 0.0, 0};
            const bool mid = beta_in_middle_pass(h->op);
            if (!mid)
                launch_finalize_beta(st, pb, nparts_hv, q->be.d(), k - 1, tol, sh, q->omega.d(), q->nw, q->eta, s);
            launch_lanczos_a_rest(h->op, cur, prv, out, nullptr, st, pa, s, Stack(), mid ? &fb : nullptr);
            if (!fa_on) launch_finalize_alpha(st, pa, nparts_hv, q->al.d(), k, s);
        } else {
            launch_lanczos_a(h->op, cur, prv, out, nullptr, st, q->partials.d(), k == 0, s);
            if (!fa_on) launch_finalize_alpha(st, q->partials.d(), nparts_hv, q->al.d(), k, s);
            if (!fuse) {
                launch_lanczos_b(dim, cur, out, st, q->partials.d(), s);
                launch_finalize_beta(st, q->partials.d(), nparts, q->be.d(), k, tol, sh, q->omega.d(), q->nw, q->eta,
                                     s);
            }
        }
    }
    if (fuse && k1 > k0) {
        if (fa_on) launch_finalize_alpha(st, pa, nparts_hv, q->al.d(), k1 - 1, s);
        const double *cur = k1 == 1 ? q->chi.d() : W[(k1 - 2) % 2];
        launch_lanczos_b(dim, cur, W[(k1 - 1) % 2], st, q->partials.d(), s);
        launch_finalize_beta(st, q->partials.d(), nparts, q->be.d(), k1 - 1, tol, sh, q->omega.d(), q->nw, q->eta, s);
    }
    HIP_CHECK(hipGetLastError());
    q->k = k1;
}

}  // namespace

extern "C" {

ftk_status ftk_green_seq_create(const ftk_hamiltonian *h, const double *chi, const double *omega, int n_omega,
                                double eta, double shift_re, int n_max, ftk_green_seq **out)
{
    return guard([&] {
        need(h && chi && omega && out, "NULL argument");
        *out = nullptr;
        auto q = seq_alloc(h, omega, n_omega, eta, shift_re, n_max);
        hipStream_t s = h->ctx->stream;
        HIP_CHECK(hipMemcpyAsync(q->chi.p, chi, q->chi.n, hipMemcpyDeviceToDevice, s));
        launch_dot(h->dim, q->chi.d(), q->chi.d(), q->partials.d(), s);
        launch_start_sequence((SeqState *)q->st.p, q->partials.d(), vec_grid(h->dim), shift_re, s);
        HIP_CHECK(hipGetLastError());
        const SeqState r = seq_state(q.get());
        if (!(r.norm2 > 0) || !std::isfinite(r.norm2)) fail(FTK_ENUMERIC, "start vector has zero or non-finite norm");
        *out = q.release();
    });
}

ftk_status ftk_green_seq_advance(ftk_green_seq *q, int n_steps, int *steps)
{
    return guard([&] {
        need(q != nullptr, "NULL argument");
        need(n_steps >= 0, "n_steps must be >= 0");
        HIP_CHECK(hipSetDevice(q->h->ctx->device));
        SeqState r = seq_state(q);
        const int k1 = std::min(q->n_max, q->k + n_steps);
        if (!r.done && !r.numeric_error && k1 > q->k) {
            seq_chunk(q, k1);
            r = seq_state(q);
        }
        if (steps) *steps = std::max(0, std::min(r.steps, q->n_max));
        if (r.numeric_error) fail(FTK_ENUMERIC, "NaN/Inf in Green's-function Lanczos coefficients");
    });
}

ftk_status ftk_green_seq_read(ftk_green_seq *q, double *g, double *alpha, double *beta, int *steps,
                              double *max_resid, int *done)
{
    return guard([&] {
        need(q != nullptr, "NULL argument");
        HIP_CHECK(hipSetDevice(q->h->ctx->device));
        hipStream_t s = q->h->ctx->stream;
        const SeqState r = seq_state(q);
        const int k = std::max(0, std::min(r.steps, q->n_max));  // a restored state is trusted no further
        if (g) {
            launch_finish_green((const SeqState *)q->st.p, (const ShiftState *)q->shifts.p, q->nw, q->g.d(), s);
            HIP_CHECK(hipMemcpyAsync(g, q->g.p, q->g.n, hipMemcpyDeviceToHost, s));
        }
        if (alpha && k > 0) HIP_CHECK(hipMemcpyAsync(alpha, q->al.p, sizeof(double) * k, hipMemcpyDeviceToHost, s));
        if (beta && k > 0) HIP_CHECK(hipMemcpyAsync(beta, q->be.p, sizeof(double) * k, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (steps) *steps = k;
        if (max_resid) *max_resid = r.max_resid;
        if (done) *done = r.done || r.numeric_error || k >= q->n_max;
    });
}

ftk_status ftk_green_seq_save(ftk_green_seq *q, void *buf, size_t cap, size_t *bytes)
{
    return guard([&] {
        need(q && bytes, "NULL argument");
        const ftk_hamiltonian *h = q->h;
        const size_t vb = sizeof(double) * 2 * (size_t)h->dim;
        const size_t payload = seq_payload_bytes(h->dim, q->nw, q->n_max);
        *bytes = sizeof(SeqBlobHeader) + payload;
        if (!buf) return;
        need(cap >= *bytes, "buffer too small for the sequence state");
        HIP_CHECK(hipSetDevice(h->ctx->device));
        hipStream_t s = h->ctx->stream;
        SeqBlobHeader hd{};
        std::memcpy(hd.magic, kSeqMagic, 8);
        hd.h_hash = table_hash(h);
        hd.n_sites = h->n_sites;
        hd.n_max = q->n_max;
        hd.nw = q->nw;
        hd.k = q->k;
        hd.eta = q->eta;
        hd.shift_re = q->shift_re;
        hd.payload_bytes = payload;
        char *p = (char *)buf + sizeof(SeqBlobHeader);
        char *p0 = p;
        std::memcpy(p, q->omega_h.data(), sizeof(double) * q->nw);
        p += sizeof(double) * q->nw;
        HIP_CHECK(hipMemcpyAsync(p, q->st.p, sizeof(SeqState), hipMemcpyDeviceToHost, s));
        p += sizeof(SeqState);
        HIP_CHECK(hipMemcpyAsync(p, q->shifts.p, sizeof(ShiftState) * q->nw, hipMemcpyDeviceToHost, s));
        p += sizeof(ShiftState) * q->nw;
        HIP_CHECK(hipMemcpyAsync(p, q->al.p, sizeof(double) * q->n_max, hipMemcpyDeviceToHost, s));
        p += sizeof(double) * q->n_max;
        HIP_CHECK(hipMemcpyAsync(p, q->be.p, sizeof(double) * q->n_max, hipMemcpyDeviceToHost, s));
        p += sizeof(double) * q->n_max;
        HIP_CHECK(hipMemcpyAsync(p, seq_cur(q), vb, hipMemcpyDeviceToHost, s));
        p += vb;
        HIP_CHECK(hipMemcpyAsync(p, seq_prv(q), vb, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        hd.payload_hash = fnv64(p0, payload);
        std::memcpy(buf, &hd, sizeof hd);
    });
}

ftk_status ftk_green_seq_restore(const ftk_hamiltonian *h, const void *buf, size_t bytes, ftk_green_seq **out)
{
    return guard([&] {
        need(h && buf && out, "NULL argument");
        *out = nullptr;
        need(bytes >= sizeof(SeqBlobHeader), "sequence state truncated");
        SeqBlobHeader hd;
        std::memcpy(&hd, buf, sizeof hd);
        need(std::memcmp(hd.magic, kSeqMagic, 8) == 0, "not a sequence state (bad magic)");
        need(hd.n_sites == h->n_sites && hd.h_hash == table_hash(h),
             "sequence state belongs to another Hamiltonian");
        need(hd.nw >= 1 && hd.n_max >= 1 && hd.k >= 0 && hd.k <= hd.n_max, "corrupt sequence state header");
        const size_t vb = sizeof(double) * 2 * (size_t)h->dim;
        const size_t payload = seq_payload_bytes(h->dim, hd.nw, hd.n_max);
        need(hd.payload_bytes == payload && bytes >= sizeof(SeqBlobHeader) + payload, "sequence state truncated");
        const char *p = (const char *)buf + sizeof(SeqBlobHeader);
        need(fnv64(p, payload) == hd.payload_hash, "sequence state corrupt (checksum)");
        const double *om = (const double *)p;
        auto q = seq_alloc(h, om, hd.nw, hd.eta, hd.shift_re, hd.n_max);
        q->k = hd.k;
        hipStream_t s = h->ctx->stream;
        p += sizeof(double) * hd.nw;
        HIP_CHECK(hipMemcpyAsync(q->st.p, p, sizeof(SeqState), hipMemcpyHostToDevice, s));
        p += sizeof(SeqState);
        HIP_CHECK(hipMemcpyAsync(q->shifts.p, p, sizeof(ShiftState) * hd.nw, hipMemcpyHostToDevice, s));
        p += sizeof(ShiftState) * hd.nw;
        HIP_CHECK(hipMemcpyAsync(q->al.p, p, sizeof(double) * hd.n_max, hipMemcpyHostToDevice, s));
        p += sizeof(double) * hd.n_max;
        HIP_CHECK(hipMemcpyAsync(q->be.p, p, sizeof(double) * hd.n_max, hipMemcpyHostToDevice, s));
        p += sizeof(double) * hd.n_max;
        HIP_CHECK(hipMemcpyAsync((void *)seq_cur(q.get()), p, vb, hipMemcpyHostToDevice, s));
        p += vb;
        if (q->k >= 1) HIP_CHECK(hipMemcpyAsync((void *)seq_prv(q.get()), p, vb, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
        *out = q.release();
    });
}

ftk_status ftk_green_seq_info(const ftk_green_seq *q, int *n_omega, int *n_max, size_t *state_bytes)
{
    return guard([&] {
        need(q != nullptr, "NULL argument");
        if (n_omega) *n_omega = q->nw;
        if (n_max) *n_max = q->n_max;
        if (state_bytes) *state_bytes = sizeof(SeqBlobHeader) + seq_payload_bytes(q->h->dim, q->nw, q->n_max);
    });
}

ftk_status ftk_green_seq_destroy(ftk_green_seq *q)
{
    return guard([&] { delete q; });
}

}  // extern "C"
