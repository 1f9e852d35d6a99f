// Spectrum server: independent S(Q, omega, T') requests on one GPU.
//
// Each request is the whole method for one Hamiltonian: typical states one
// vector at a time (the L shells of that vector stay resident while its
// Green's sequences run), the Green's functions of every shell, and the
// reweighting of the accumulated shell data to the requested temperatures.
// Requests run concurrently on worker threads, each with its own context and
// stream, as device memory allows (scheduler.h): a request starts as soon as a
// worker is free and its peak footprint fits, so small requests keep the GPU
// busy around large ones.  Every request's arithmetic is that of a standalone
// run: results do not depend on what else is running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ftkw_internal.h"
#include "kernels.h"
#include "scheduler.h"

using namespace ftk;

namespace {

using Clock = std::chrono::steady_clock;

// rhs_block a request runs with: its own, else the autotuner's recorded pick,
// else 16 sequences per launch up to 20 sites, a stack of 4 up to 24 and one
// sequence above (memory)
int resolve_block(int device, int n_sites, const ftk_spec_params *sp)
{
    if (sp->rhs_block != 0) return sp->rhs_block;
    const int t = tuned_rhs_block(device, n_sites, sp->n_omega);
    if (t) return t;
    return n_sites <= 20 ? 16 : 1;  // measured fastest without a tuning record
}

int resolve_block_steps(const ftk_ts_params *tp) { return tp->block_steps > 0 ? tp->block_steps : 16; }

size_t footprint(int n_sites, const ftk_ts_params *tp, const ftk_spec_params *sp, int B, int nb)
{
    const double V = 16.0 * std::ldexp(1.0, n_sites);
    const double na = tp->n_anchors, L = tp->L, nf = tp->n_steps, ng = sp->n_steps, nw = sp->n_omega;
    int nal = 0;
    for (int a = 0; a < 3; ++a) nal += (sp->alpha_mask >> a) & 1;
    bool any_beta = false;
    for (int a = 0; a < tp->n_anchors; ++a) any_beta = any_beta || tp->anchor_beta[a] > 0;
    const double nseq = na * L * nal * sp->n_q;
    const double nbk = std::min<double>(nb, nf);
    const double partials = 16.0 * kMaxGrid * 16;
    // typical states of one vector: start vector, phi_beta, Taylor term/next/sum,
    // two Lanczos buffers, the buffered Lanczos vectors, the shells of every anchor
    const double states = ((any_beta ? 7 : 4) + nbk + na * L) * V + 16.0 * L * nf + partials + 16.0 * nf + 4096;
    // Green's functions of that vector: the shells plus a batch of B sequences
    // (three vectors each, four when the batch is a stack of multi-pass sequences)
    const double per_seq = B > 1 && n_sites >= kPassMinSites ? 4.0 : 3.0;
    const double green = na * L * V + per_seq * B * V + 16.0 * nseq * nw + 16.0 * nseq * ng +
                         (double)sizeof(SeqState) * (nseq + B) + 16.0 * ng * B + 48.0 * nw * B + 8.0 * nw +
                         16.0 * kMaxGrid * B;
    // the Hamiltonian's scratch vector of the multi-pass H v
    const double scratch = n_sites >= kPassMinSites ? V : 0.0;
    const double peak = std::max(states, green) + scratch;
    // allocation granularity (2 MiB per buffer, 32 buffers at most) and a 2 % margin
    // for what the count above leaves out (largest measured peak: 0.993 of it)
    return (size_t)std::ceil(1.02 * peak + 64.0 * 1024 * 1024);
}

struct Request {
    uint64_t id = 0;
    // copies of the caller's arrays
    int n_sites = 0, n_bonds = 0;
    std::vector<int32_t> bi, bj;
    std::vector<int8_t> gamma;
    std::vector<double> site_xy;
    double K = 0, J = 0;
    ftk_ts_params tp{};
    std::vector<double> betas, E_b, eps;
    bool auto_window = false;
    ftk_spec_params sp{};
    std::vector<double> q_xy, omega, T;
    int B = 1, nb = 16;
    size_t bytes = 0;
    // state and results
    enum { QUEUED, RUNNING, DONE, FAILED } state = QUEUED;
    ftk_status status = FTK_OK;
    std::string error;
    std::vector<double> S, S_err;
    Clock::time_point t_submit, t_start, t_done;
    size_t peak_bytes = 0;
    std::atomic<bool> cancel{false};  // set by ftk_server_cancel while the request runs
    // per-request metrics: seconds per stage, Krylov steps of the Green's sequences,
    // largest Galerkin residual over them
    double t_hamiltonian = 0, t_states = 0, t_spectra = 0, t_reweight = 0;
    int64_t krylov_steps = 0;
    double max_resid = 0;
};

double since(Clock::time_point t) { return std::chrono::duration<double>(Clock::now() - t).count(); }

void check(ftk_status s)
{
    if (s != FTK_OK) fail(s, ftk_last_error());
}

struct Handles {
    ftk_hamiltonian *h = nullptr;
    ftk_states *st = nullptr;
    ftk_spectrum *sp = nullptr;
    ~Handles()
    {
        if (sp) ftk_spectrum_destroy(sp);
        if (st) ftk_states_destroy(st);
        if (h) ftk_hamiltonian_destroy(h);
    }
};

void stop_if_cancelled(const Request &r)
{
    if (r.cancel.load()) fail(FTK_ECANCELED, "request cancelled");
}

// the whole method for one request on one context; a cancellation takes effect at
// the stage boundaries below
void run_request(ftk_ctx *ctx, Request &r)
{
    Handles H;
    ftk_cluster c{r.n_sites, r.n_bonds, r.bi.data(), r.bj.data(), r.gamma.data(), r.site_xy.data()};
    Clock::time_point t = Clock::now();
    check(ftk_build_hamiltonian(ctx, &c, r.K, r.J, &H.h));
    r.t_hamiltonian = since(t);
    stop_if_cancelled(r);
    const int nv = r.tp.n_vectors, na = r.tp.n_anchors, L = r.tp.L, nq = r.sp.n_q, nw = r.sp.n_omega;
    int nal = 0;
    for (int a = 0; a < 3; ++a) nal += (r.sp.alpha_mask >> a) & 1;
    std::vector<double> E_b = r.E_b, eps = r.eps, E_m((size_t)na * L);
    std::vector<double> log_norm((size_t)nv * na), n_m((size_t)nv * na * L);
    std::vector<double> g((size_t)nv * na * L * nq * nw * 2, 0.0);
    std::vector<double> graw((size_t)na * L * nal * nq * nw * 2);
    std::vector<double> resid((size_t)na * L * nal * nq);
    bool have_window = !r.auto_window;
    for (int sv = 0; sv < nv; ++sv) {
        ftk_ts_params tp = r.tp;
        tp.first_vector = r.tp.first_vector + sv;
        tp.n_vectors = 1;
        tp.anchor_beta = r.betas.data();
        tp.E_b = have_window ? E_b.data() : nullptr;
        tp.eps = have_window ? eps.data() : nullptr;
        tp.block_steps = r.nb;
        tp.gaussian_dev = nullptr;
        t = Clock::now();
        check(ftk_typical_states(H.h, &tp, &H.st));
        if (!have_window) {
            // vector 0 fixed the window; the others use it unchanged
            E_b.assign(na, 0.0);
            eps.assign(na, 0.0);
            check(ftk_states_window(H.st, E_b.data(), eps.data()));
            have_window = true;
        }
        check(ftk_states_scalars(H.st, &log_norm[(size_t)sv * na], &n_m[(size_t)sv * na * L], E_m.data(), nullptr));
        r.t_states += since(t);
        stop_if_cancelled(r);
        t = Clock::now();
        ftk_spec_params sp = r.sp;
        sp.q_xy = r.q_xy.data();
        sp.omega = r.omega.data();
        sp.rhs_block = r.B;
        check(ftk_shifted_krylov_spectrum(H.h, H.st, &sp, &H.sp));
        check(ftk_spectrum_raw(H.sp, graw.data(), resid.data()));
        int64_t ks = 0;
        check(ftk_spectrum_work(H.sp, &ks, nullptr));
        r.krylov_steps += ks;
        for (double x : resid) r.max_resid = std::max(r.max_resid, x);
        // sum over alpha: graw [na][L][nal][nq][nw] -> g[sv] [na][L][nq][nw]
        double *gs = &g[(size_t)sv * na * L * nq * nw * 2];
        for (size_t am = 0; am < (size_t)na * L; ++am)
            for (int ia = 0; ia < nal; ++ia)
                for (size_t j = 0; j < (size_t)nq * nw * 2; ++j)
                    gs[am * nq * nw * 2 + j] += graw[(am * nal + ia) * nq * nw * 2 + j];
        check(ftk_spectrum_destroy(H.sp));
        H.sp = nullptr;
        check(ftk_states_destroy(H.st));
        H.st = nullptr;
        r.t_spectra += since(t);
        stop_if_cancelled(r);
    }
    t = Clock::now();
    const int nT = (int)r.T.size();
    r.S.assign((size_t)nq * nT * nw, 0.0);
    r.S_err.assign((size_t)nq * nT * nw, 0.0);
    check(ftk_reweight(nv, na, L, nq, nw, r.betas.data(), E_m.data(), eps.data(), log_norm.data(), n_m.data(),
                       g.data(), r.T.data(), nT, std::min(8, nv), r.S.data(), r.S_err.data(), nullptr));
    r.t_reweight = since(t);
}

// one JSON line of a finished request's metrics
std::string metrics_line(const Request &r, double t_origin_s, double submit_s)
{
    const double wait = std::chrono::duration<double>(r.t_start - r.t_submit).count();
    const double lat = std::chrono::duration<double>(r.t_done - r.t_submit).count();
    int nal = 0;
    for (int a = 0; a < 3; ++a) nal += (r.sp.alpha_mask >> a) & 1;
    const double alg = 48.0 * (double)(1ull << r.n_sites) * (double)r.krylov_steps;  // 48 B per element and step
    char buf[1024];
    std::snprintf(buf, sizeof buf,
                  "{\"ticket\": %llu, \"status\": %d, \"n_sites\": %d, \"n_vectors\": %d, \"n_anchors\": %d, "
                  "\"L\": %d, \"n_alpha\": %d, \"n_q\": %d, \"n_omega\": %d, \"n_steps\": %d, \"rhs_block\": %d, "
                  "\"submitted_s\": %.6f, \"queue_wait_s\": %.6f, \"latency_s\": %.6f, \"hamiltonian_s\": %.6f, "
                  "\"states_s\": %.6f, \"spectra_s\": %.6f, \"reweight_s\": %.6f, \"krylov_steps\": %lld, "
                  "\"krylov_iters_per_s\": %.3f, \"green_algorithmic_gbps\": %.3f, \"max_residual\": %.6e, "
                  "\"reserved_bytes\": %zu, \"peak_bytes\": %zu}",
                  (unsigned long long)r.id, (int)r.status, r.n_sites, r.tp.n_vectors, r.tp.n_anchors, r.tp.L, nal,
                  r.sp.n_q, r.sp.n_omega, r.sp.n_steps, r.B, submit_s - t_origin_s, wait, lat, r.t_hamiltonian,
                  r.t_states, r.t_spectra, r.t_reweight, (long long)r.krylov_steps,
                  r.t_spectra > 0 ? (double)r.krylov_steps / r.t_spectra : 0.0,
                  r.t_spectra > 0 ? alg / r.t_spectra / 1e9 : 0.0, r.max_resid, r.bytes, r.peak_bytes);
    return buf;
}

}  // namespace

struct ftk_server {
    int device = 0;
    std::unique_ptr<Admission> adm;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<ftk_ctx *> ctxs;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_id = 1;
    Clock::time_point t0;
    bool any_submit = false;
    Clock::time_point first_submit, last_done;
    std::vector<double> latencies;
    size_t completed = 0, failed = 0, cancelled = 0;
    double max_peak_ratio = 0.0;
    std::vector<std::pair<double, double>> occupancy;  // (seconds since create, reserved bytes)
    std::string log_path;  // FTK_SERVE_LOG at creation: one JSON line per finished request

    void record_occupancy() { occupancy.push_back({secs(Clock::now()), (double)adm->in_use()}); }
    double secs(Clock::time_point t) const { return std::chrono::duration<double>(t - t0).count(); }

    void worker(int w)
    {
        ftk_ctx *ctx = ctxs[w];
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lock(mu);
                uint64_t id = 0;
                size_t bytes = 0;
                cv_work.wait(lock, [&] { return stop || adm->pick(&id, &bytes); });
                if (stop && id == 0) return;
                r = reqs.at(id).get();
                r->state = Request::RUNNING;
                r->t_start = Clock::now();
                record_occupancy();
            }
            ftk_status st = FTK_OK;
            std::string err;
            size_t peak = 0;
            try {
                check(ftk_ctx_peak_memory(ctx, nullptr, 1));
                run_request(ctx, *r);
                check(ftk_ctx_peak_memory(ctx, &peak, 0));
            } catch (const Error &e) {
                st = e.status;
                err = e.what();
            } catch (const std::bad_alloc &) {
                st = FTK_ENOMEM;
                err = "host allocation failed";
            } catch (const std::exception &e) {
                st = FTK_EDEVICE;
                err = e.what();
            }
            {
                std::lock_guard<std::mutex> lock(mu);
                adm->release(r->bytes);
                r->t_done = Clock::now();
                r->peak_bytes = peak;
                r->status = st;
                r->error = err;
                r->state = st == FTK_OK ? Request::DONE : Request::FAILED;
                if (st == FTK_OK) {
                    ++completed;
                    latencies.push_back(std::chrono::duration<double>(r->t_done - r->t_submit).count());
                    max_peak_ratio = std::max(max_peak_ratio, (double)peak / (double)r->bytes);
                } else if (st == FTK_ECANCELED) {
                    ++cancelled;
                } else {
                    ++failed;
                }
                last_done = r->t_done;
                record_occupancy();
                if (!log_path.empty()) {
                    std::ofstream f(log_path, std::ios::app);
                    if (f) f << metrics_line(*r, 0.0, secs(r->t_submit)) << "\n";
                }
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

namespace {

template <class F>
ftk_status srv_guard(F &&f)
{
    try {
        f();
        return FTK_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return FTK_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return FTK_EDEVICE;
    }
}

void need(bool ok, const char *msg)
{
    if (!ok) fail(FTK_EINVAL, msg);
}

double quantile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

void validate(const ftk_cluster *c, const ftk_ts_params *tp, const ftk_spec_params *sp, const double *T, int n_T)
{
    need(c && tp && sp && T, "NULL argument");
    need(c->n_sites >= 4 && c->n_sites <= kMaxSites, "n_sites must be in [4, 30]");
    need(c->n_bonds >= 1 && c->bond_i && c->bond_j && c->bond_gamma && c->site_xy, "cluster arrays must not be NULL");
    need(tp->n_vectors >= 1 && tp->n_anchors >= 1 && tp->anchor_beta, "need vectors and anchors");
    need((tp->E_b == nullptr) == (tp->eps == nullptr), "E_b and eps must both be given or both be NULL");
    need(tp->L >= 1 && tp->M >= 2 && tp->M % 2 == 0 && tp->n_steps >= 1, "bad L, M or n_steps");
    need(tp->gaussian_dev == nullptr, "requests draw their own start vectors (gaussian_dev must be NULL)");
    need(sp->n_q >= 1 && sp->q_xy && sp->n_omega >= 1 && sp->omega, "need momenta and frequencies");
    need((sp->alpha_mask & 7) != 0 && (sp->alpha_mask & ~7) == 0, "alpha_mask must be a non-empty subset of {x,y,z}");
    need(sp->n_steps >= 1 && std::isfinite(sp->eta) && sp->eta > 0, "bad n_steps or eta");
    need(sp->rhs_block == 0 || sp->rhs_block == 1 || sp->rhs_block == 2 || sp->rhs_block == 4 || sp->rhs_block == 8 ||
             sp->rhs_block == 16 || sp->rhs_block == 32,
         "rhs_block must be 0, 1, 2, 4, 8, 16 or 32");
    need(n_T >= 1, "need at least one temperature");
    for (int i = 0; i < n_T; ++i) need(std::isfinite(T[i]) && T[i] > 0, "temperatures must be > 0");
}

}  // namespace

extern "C" {

ftk_status ftk_request_footprint(int n_sites, const ftk_ts_params *tp, const ftk_spec_params *sp, int device,
                                 size_t *bytes)
{
    return srv_guard([&] {
        need(tp && sp && bytes && tp->anchor_beta, "NULL argument");
        need(n_sites >= 4 && n_sites <= kMaxSites, "n_sites must be in [4, 30]");
        need(tp->n_anchors >= 1 && tp->L >= 1 && tp->n_steps >= 1 && sp->n_steps >= 1 && sp->n_omega >= 1 &&
                 sp->n_q >= 1,
             "bad sizes");
        *bytes = footprint(n_sites, tp, sp, resolve_block(device, n_sites, sp), resolve_block_steps(tp));
    });
}

ftk_status ftk_server_create(int device, size_t hbm_budget, int n_workers, ftk_server **out)
{
    return srv_guard([&] {
        need(out != nullptr, "out must not be NULL");
        need(n_workers >= 0 && n_workers <= 16, "n_workers must be in [0, 16]");
        if (n_workers == 0) n_workers = 4;
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess) fail(FTK_EDEVICE, "no HIP device");
        need(device >= 0 && device < n, "device index out of range");
        if (hipSetDevice(device) != hipSuccess) fail(FTK_EDEVICE, "hipSetDevice failed");
        if (hbm_budget == 0) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) fail(FTK_EDEVICE, "hipMemGetInfo failed");
            hbm_budget = (size_t)(0.9 * (double)fr);
        }
        auto srv = std::make_unique<ftk_server>();
        srv->device = device;
        srv->adm = std::make_unique<Admission>(hbm_budget, n_workers, 4);
        srv->t0 = Clock::now();
        for (int w = 0; w < n_workers; ++w) {
            ftk_ctx *c = nullptr;
            ftk_status s = ftk_ctx_create(device, nullptr, &c);
            if (s != FTK_OK) {
                for (ftk_ctx *x : srv->ctxs) ftk_ctx_destroy(x);
                fail(s, ftk_last_error());
            }
            srv->ctxs.push_back(c);
        }
        srv->record_occupancy();
        if (const char *lp = std::getenv("FTK_SERVE_LOG")) srv->log_path = lp;
        ftk_server *p = srv.get();
        for (int w = 0; w < n_workers; ++w) srv->workers.emplace_back([p, w] { p->worker(w); });
        *out = srv.release();
    });
}

ftk_status ftk_server_submit(ftk_server *srv, const ftk_cluster *c, double K, double J, const ftk_ts_params *tp,
                             const ftk_spec_params *sp, const double *T, int n_T, uint64_t *ticket)
{
    return srv_guard([&] {
        need(srv && ticket, "NULL argument");
        validate(c, tp, sp, T, n_T);
        need(std::isfinite(K) && std::isfinite(J), "K and J must be finite");
        auto r = std::make_unique<Request>();
        r->n_sites = c->n_sites;
        r->n_bonds = c->n_bonds;
        r->bi.assign(c->bond_i, c->bond_i + c->n_bonds);
        r->bj.assign(c->bond_j, c->bond_j + c->n_bonds);
        r->gamma.assign(c->bond_gamma, c->bond_gamma + c->n_bonds);
        r->site_xy.assign(c->site_xy, c->site_xy + 2 * c->n_sites);
        r->K = K;
        r->J = J;
        r->tp = *tp;
        r->betas.assign(tp->anchor_beta, tp->anchor_beta + tp->n_anchors);
        r->auto_window = tp->E_b == nullptr;
        if (!r->auto_window) {
            r->E_b.assign(tp->E_b, tp->E_b + tp->n_anchors);
            r->eps.assign(tp->eps, tp->eps + tp->n_anchors);
        }
        r->sp = *sp;
        r->q_xy.assign(sp->q_xy, sp->q_xy + 2 * sp->n_q);
        r->omega.assign(sp->omega, sp->omega + sp->n_omega);
        r->T.assign(T, T + n_T);
        r->B = resolve_block(srv->device, c->n_sites, sp);
        r->nb = resolve_block_steps(tp);
        r->bytes = footprint(c->n_sites, tp, sp, r->B, r->nb);
        std::lock_guard<std::mutex> lock(srv->mu);
        need(!srv->stop, "server is shutting down");
        const uint64_t id = srv->next_id++;
        r->id = id;
        r->t_submit = Clock::now();
        if (!srv->adm->submit(id, r->bytes))
            fail(FTK_ENOMEM, "request needs " + std::to_string(r->bytes) + " device bytes, more than the budget of " +
                                 std::to_string(srv->adm->budget()));
        if (!srv->any_submit) {
            srv->any_submit = true;
            srv->first_submit = r->t_submit;
        }
        srv->reqs[id] = std::move(r);
        *ticket = id;
        srv->cv_work.notify_one();
    });
}

ftk_status ftk_server_poll(ftk_server *srv, uint64_t ticket, double *S_out, double *S_stderr, double *latency_s)
{
    ftk_status result = FTK_OK;
    ftk_status g = srv_guard([&] {
        need(srv != nullptr, "NULL argument");
        std::lock_guard<std::mutex> lock(srv->mu);
        auto it = srv->reqs.find(ticket);
        need(it != srv->reqs.end(), "unknown ticket");
        Request &r = *it->second;
        if (r.state == Request::QUEUED || r.state == Request::RUNNING) {
            result = FTK_ENOTREADY;
            set_last_error("request not finished");
            return;
        }
        if (r.state == Request::FAILED) {
            result = r.status;
            set_last_error(r.error);
        } else {
            if (S_out) std::copy(r.S.begin(), r.S.end(), S_out);
            if (S_stderr) std::copy(r.S_err.begin(), r.S_err.end(), S_stderr);
            if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
        }
        srv->reqs.erase(it);
    });
    return g != FTK_OK ? g : result;
}

ftk_status ftk_server_wait(ftk_server *srv, uint64_t ticket, double timeout_s)
{
    ftk_status result = FTK_OK;
    ftk_status g = srv_guard([&] {
        need(srv != nullptr, "NULL argument");
        need(std::isfinite(timeout_s) && timeout_s >= 0, "timeout must be >= 0");
        std::unique_lock<std::mutex> lock(srv->mu);
        auto ready = [&] {
            auto it = srv->reqs.find(ticket);
            return it == srv->reqs.end() || it->second->state == Request::DONE ||
                   it->second->state == Request::FAILED;
        };
        need(srv->reqs.count(ticket) != 0, "unknown ticket");
        if (!srv->cv_done.wait_for(lock, std::chrono::duration<double>(timeout_s), ready)) {
            result = FTK_ENOTREADY;
            set_last_error("request not finished");
        }
    });
    return g != FTK_OK ? g : result;
}

ftk_status ftk_server_stats(ftk_server *srv, ftk_serving_stats *out)
{
    return srv_guard([&] {
        need(srv && out, "NULL argument");
        std::lock_guard<std::mutex> lock(srv->mu);
        out->completed = (int64_t)srv->completed;
        out->failed = (int64_t)srv->failed;
        out->waiting = (int64_t)srv->adm->waiting();
        out->running = srv->adm->running();
        out->p50_latency_s = quantile(srv->latencies, 0.50);
        out->p99_latency_s = quantile(srv->latencies, 0.99);
        const double span = srv->completed ? std::chrono::duration<double>(srv->last_done - srv->first_submit).count() : 0;
        out->requests_per_s = span > 0 ? (double)srv->completed / span : 0.0;
        out->hbm_budget = srv->adm->budget();
        out->hbm_reserved = srv->adm->in_use();
        out->hbm_reserved_peak = srv->adm->peak();
        out->max_peak_over_footprint = srv->max_peak_ratio;
        out->cancelled = (int64_t)srv->cancelled;
    });
}

ftk_status ftk_server_cancel(ftk_server *srv, uint64_t ticket)
{
    return srv_guard([&] {
        need(srv != nullptr, "NULL argument");
        {
            std::lock_guard<std::mutex> lock(srv->mu);
            auto it = srv->reqs.find(ticket);
            need(it != srv->reqs.end(), "unknown ticket");
            Request &r = *it->second;
            need(r.state == Request::QUEUED || r.state == Request::RUNNING, "request already finished");
            if (r.state == Request::RUNNING) {
                r.cancel.store(true);  // the worker stops at the next stage boundary
                return;
            }
            srv->adm->cancel(ticket);
            r.state = Request::FAILED;
            r.status = FTK_ECANCELED;
            r.error = "request cancelled before it started";
            r.t_done = Clock::now();
            ++srv->cancelled;
        }
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();  // a request waiting behind the cancelled one may start
    });
}

ftk_status ftk_server_occupancy(ftk_server *srv, double *t, double *bytes, int cap, int *n)
{
    return srv_guard([&] {
        need(srv && n, "NULL argument");
        std::lock_guard<std::mutex> lock(srv->mu);
        const int m = (int)srv->occupancy.size();
        *n = m;
        for (int i = 0; i < std::min(m, cap); ++i) {
            if (t) t[i] = srv->occupancy[i].first;
            if (bytes) bytes[i] = srv->occupancy[i].second;
        }
    });
}

ftk_status ftk_server_destroy(ftk_server *srv)
{
    return srv_guard([&] {
        if (!srv) return;
        {
            std::lock_guard<std::mutex> lock(srv->mu);
            srv->stop = true;
            for (auto &kv : srv->reqs)
                if (kv.second->state == Request::QUEUED) srv->adm->cancel(kv.first);
        }
        srv->cv_work.notify_all();
        for (auto &th : srv->workers) th.join();
        for (ftk_ctx *c : srv->ctxs) ftk_ctx_destroy(c);
        delete srv;
    });
}

}  // extern "C"
