"""Benchmark of the FTKw hot path on one MI355X: the 24-site workload (default;
--workload plain-N16 / plain-N8 run the smaller configurations the same way).

Workload (plain-N24): 24-site hexagonal cluster (dim 2^24, 268 MB per complex128
vector), K = -1, J = 0.1; 8 random vectors; anchors T = inf, 1, 0.5, 0.2 with the
24-site discretisation of Table I (E_b = -5, L = 128, M = 16); 500 Krylov steps
for filters and Green's functions; 2000 frequencies in [-4, 4], eta = 0.01;
Q in {Gamma, M, K}, alpha in {x, y, z}; 100 temperatures in [0.1, 10].

One bench step is one batch of 16 Green's-function sequences of the job (at 24
sites: 16 consecutive shells of one (vector, anchor, alpha, Q); 500 Lanczos steps
each with the 2000-shift update every step), run rhs_block sequences per launch
(the autotuner's pick; a step holds max(16, rhs_block) sequences).  The job is
8 vectors x 4 anchors x 72 steps = 2304 steps.  The states of a (vector, anchor)
pair -- random vector, imaginary-time state, the 128 filtered states (two
500-step Lanczos passes and the shell accumulation) -- are built by the first of
its 72 steps and reused by the others, as in the job.  The timed steps walk the
job in order from the first step of (vector 0, anchor T = 1), so the first timed
step also builds that pair's states (state building then weighs ~3.6x its share
of the job: one build per 20 steps instead of per 72); the warmup runs the same
anchor on the last vector.  The timed region ends with the reweighting of
everything accumulated so far to the 100 temperatures (the job reweights once,
at its end).  value = Krylov iterations per second (RHS-steps of the Green's
sequences: one Lanczos step of one sequence, including its multi-shift update)
over the timed steps.  The defaults (--steps 20 --warmup 2) finish in a few
minutes; each step takes ~4 s at 24 sites.

roofline: one Lanczos step (all its launches), priced at the method's minimum of
48 B per basis element and sequence (read v_k and v_{k-1}, write v_{k+1});
hv_roofline: the standalone H v at 32 B per element (read v, write w).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --serve [--serve-sizes 12,14,16,18,20] [--serve-vectors 2,4]
                       [--serve-requests 48] [--serve-workers 4] [--serve-steps n] [--serve-shells L]
                       [--serve-weights w1,w2,...]
       python bench.py --batching [--batching-sizes 20,24]

--batching times 16 Green's sequences (one random vector, 4 shells, 4 momenta)
three ways: the plain one-vector loop (alpha, beta read on the host every step),
the one-vector device loop, and blocks of 16 sequences replayed from a HIP
graph; the spectra must agree bit for bit.

--serve measures the spectrum server instead (one JSON line of its own): a
stream of independent requests (the serving workload: N from a size mix with
weights 0.4/0.3/0.2/0.07/0.03, J ~ U[0, 0.3], n_vectors ~ U{lo..hi}, L = 16 on
the automatic window, 300 steps, 1000 frequencies, Q = Gamma, 20 T'), first
submitted all at once to measure the service capacity, then as a Poisson stream
at 0.8 x that capacity; reports requests/s, p50/p99 latency and the reserved
device memory over time.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H*v HBM GB/s + Krylov iters/s at N=24; spectra/s and p99 latency served"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name="plain-N24"):
    from seeded_inputs import BASE_SEED, SUPERCELLS, WORKLOADS, eps_table1_24, omega_grid, temperature_grid
    w = dict(WORKLOADS[name])
    w["name"] = name
    w["T1"], w["T2"] = SUPERCELLS[w["N"]]
    w["seed"] = BASE_SEED
    anchors = w["temps_anchor"]
    w["betas"] = [0.0 if math.isinf(T) else 1.0 / T for T in anchors]
    w["eps_list"] = [eps_table1_24(T) if w["eps"] == "table1" else w["eps"] for T in anchors]
    w["omega_arr"] = omega_grid(*w["omega"])
    w["temps_arr"] = temperature_grid(*w["temps"])
    return w


def workload_text(w, nq):
    nsteps = w["n_vectors"] * len(w["betas"]) * steps_per_pair(w)
    return (f"{w['name']} ({w['N']}-site honeycomb, dim 2^{w['N']}, K={w['K']}, J={w['J']}, {w['n_green']} Krylov "
            f"steps, {len(w['omega_arr'])} shifts, eta={w['eta']}, L={w['L']}, M={w['M']}; one step = one batch of "
            f"{w['group']} Green's sequences (consecutive shells of one (vector, anchor, alpha, Q)) of the "
            f"{nsteps}-step job; sites relabelled by the library's layout planner)")


def steps_per_pair(w):
    """Steps of one (vector, anchor) pair: 3 spin components x n_q momenta x shell groups."""
    return 3 * w["n_q"] * ((w["L"] + w["group"] - 1) // w["group"])


def step_of(i, w):
    """(vector, anchor, alpha, q, shell group) of step i in job order."""
    nv, na, nq = w["n_vectors"], len(w["betas"]), w["n_q"]
    ng = (w["L"] + w["group"] - 1) // w["group"]
    u = i % (nv * na * 3 * nq * ng)
    s, rem = divmod(u, na * 3 * nq * ng)
    a, rem = divmod(rem, 3 * nq * ng)
    ia, rem = divmod(rem, nq * ng)
    iq, g = divmod(rem, ng)
    return s, a, ia, iq, g


def cpu_baseline(w, n_steps=None, min_seconds=12.0):
    """The oracle on the host cores: Green's sequences of the workload (n_steps Lanczos
    steps each plus the multi-shift resolvent, the oracle's own route through the Ritz
    decomposition), repeated until about min_seconds of CPU work have run."""
    from oracle import _native, cluster, green, hamiltonian
    from seeded_inputs import gaussian_vector
    N = w["N"]
    if n_steps is None:
        n_steps = min(w["n_green"], max(16, 16 << max(0, 24 - N)))
    cl = cluster.honeycomb(w["T1"], w["T2"])
    H = hamiltonian.Hamiltonian(cl, w["K"], w["J"])
    chi = gaussian_vector(w["seed"], 0, N)
    runs, dt = 0, 0.0
    while runs == 0 or dt < min_seconds:
        t0 = time.perf_counter()
        green.green_sequence(H, chi, n_steps, w["omega_arr"], w["eta"], 0.0)
        dt += time.perf_counter() - t0
        runs += 1
    cores = int(_native.lib().orc_num_threads())
    return {"value": runs * n_steps / dt, "unit": "Krylov iters/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{runs} x {n_steps} Lanczos steps of one N={N} Green's sequence (H v, exact-sum dots, "
                      f"vector updates) plus its {len(w['omega_arr'])}-shift resolvent, {dt:.1f} s",
            "cpu_model": cpu_model(), "stream_add_gbps": round(stream_add_gbps(cores), 1)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def stream_add_gbps(threads, n=1 << 25, reps=5):
    """STREAM's add kernel a = b + c on the host (float64, 3 x 256 MiB, one pass: 24 bytes
    per element), split over `threads` threads (NumPy releases the GIL inside the ufunc)."""
    from concurrent.futures import ThreadPoolExecutor
    a, b, c = np.empty(n), np.ones(n), np.full(n, 2.0)
    parts = [(i * n // threads, (i + 1) * n // threads) for i in range(threads)]

    def work(lo_hi):
        lo, hi = lo_hi
        np.add(b[lo:hi], c[lo:hi], out=a[lo:hi])

    best = 0.0
    with ThreadPoolExecutor(threads) as ex:
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(work, parts))
            best = max(best, 24.0 * n / (time.perf_counter() - t0) / 1e9)
    return best


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "exact_sum.h"):
        with open(os.path.join(ROOT, "paper_1802_02854_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, layout, units, algorithmic_bytes):
    """HBM bytes of `units` units of `kernel` (sequence-steps of the Lanczos step, launches of
    H v) from the committed counter summary, if it was taken on the current kernel source,
    for the same algorithmic bytes per unit (the same vector size) and a layout whose
    per-sequence traffic it covers (one sequence per launch and stacks move the same bytes
    per sequence); else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel)
    if not e or e.get("kernel_source") != kernel_source_hash() or layout not in e.get("layouts", []):
        return None
    if e.get("algorithmic_bytes") * units != algorithmic_bytes:
        return None
    return (e["fetch_bytes"] + e["write_bytes"]) * units


def serve_main(args):
    import paper_1802_02854_amd as ftk
    from seeded_inputs import BASE_SEED, SUPERCELLS, WORKLOADS, omega_grid, poisson_arrivals, serve_stream, \
        temperature_grid
    w = WORKLOADS["serve"]
    sizes = [int(x) for x in args.serve_sizes.split(",")]
    weights = [float(x) for x in args.serve_weights.split(",")] if args.serve_weights else list(w["weights"][: len(sizes)])
    if len(weights) != len(sizes):
        raise SystemExit("--serve-weights needs one weight per size")
    lo, hi = (int(x) for x in args.serve_vectors.split(","))
    n_req = args.serve_requests
    omega = omega_grid(*w["omega"])
    temps = temperature_grid(*w["temps"])
    clusters = {N: ftk.honeycomb_cluster(*SUPERCELLS[N]) for N in sizes}
    q = [ftk.named_momentum(n) for n in w["q"]]

    n_filter = args.serve_steps or w["n_filter"]
    n_green = args.serve_steps or w["n_green"]
    L = args.serve_shells or w["L"]

    def make(d):
        return ftk.Request(clusters[d["N"]], w["K"], d["J"], seed=d["seed"], n_vectors=d["n_vectors"],
                           betas=[0.0], L=L, M=w["M"], n_filter=n_filter, q_xy=q, omega=omega,
                           eta=w["eta"], n_green=n_green, temps=temps, window_margin=w["margin"])

    stream = [make(d) for d in serve_stream(BASE_SEED, n_req, sizes, weights, w["J"], (lo, hi))]
    # capacity is measured on the stream's own requests (the same sizes, all queued at once): with a
    # heavy-tailed size mix another sample could miss the large sizes and overstate it
    cal = [make(d) for d in serve_stream(BASE_SEED, n_req, sizes, weights, w["J"], (lo, hi))]
    Ns = [r.cluster.n_sites for r in stream]
    log(f"serve: sizes {sizes} weights {weights} vectors U{{{lo}..{hi}}}, {n_req} requests "
        f"({ {N: Ns.count(N) for N in sizes} }), {args.serve_workers} workers")

    # service capacity: every request of the stream queued at once
    srv = ftk.Server(0, n_workers=args.serve_workers)
    t0 = time.perf_counter()
    tickets = [srv.submit(r) for r in cal]
    for i, t in enumerate(tickets):
        srv.wait(t, timeout=900)
        log(f"calibration request {i + 1}/{len(cal)} done at {time.perf_counter() - t0:.1f} s")
    capacity = len(cal) / (time.perf_counter() - t0)
    srv.close()
    rate = 0.8 * capacity
    log(f"capacity {capacity:.3f} req/s -> Poisson arrivals at {rate:.3f} req/s")

    # open loop: Poisson arrivals at 0.8 x capacity
    arrivals = poisson_arrivals(BASE_SEED, rate, n_req)
    srv = ftk.Server(0, n_workers=args.serve_workers)
    pending, lat, done_at = {}, [], []
    t0 = time.perf_counter()
    i = 0
    last_log = t0
    while i < n_req or pending:
        now = time.perf_counter() - t0
        while i < n_req and arrivals[i] <= now:
            pending[srv.submit(stream[i])] = i
            i += 1
        for t in list(pending):
            r = srv.poll(t)
            if r is not None:
                lat.append(r[2])
                done_at.append(time.perf_counter() - t0)
                del pending[t]
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            log(f"t={now:.0f} s: {i} submitted, {len(lat)} done")
        time.sleep(0.002)
    span = time.perf_counter() - t0
    st = srv.stats()
    ot, ob = srv.occupancy()
    srv.close()
    lat = np.array(lat)
    occ_mean = float(np.sum(ob[:-1] * np.diff(ot)) / max(ot[-1] - ot[0], 1e-9)) if len(ot) > 1 else 0.0
    result = {
        "metric": "spectra/s served (requests/s) and p50/p99 latency",
        "value": n_req / span,
        "unit": "requests/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "capacity_requests_per_s": capacity,
        "arrival_rate_per_s": rate,
        "hbm_budget_gb": st["hbm_budget"] / 1e9,
        "hbm_reserved_peak_gb": st["hbm_reserved_peak"] / 1e9,
        "hbm_reserved_mean_gb": occ_mean / 1e9,
        "max_measured_peak_over_reservation": st["max_peak_over_footprint"],
        "failed": st["failed"],
        "config": {"workload": "serve (independent S(Q, omega, T') requests, Poisson arrivals at 0.8 x capacity)",
                   "sizes": sizes, "weights": weights, "n_vectors": [lo, hi], "requests": n_req,
                   "size_counts": {str(N): Ns.count(N) for N in sizes}, "workers": args.serve_workers,
                   "L": L, "n_steps": n_green, "n_omega": len(omega), "n_T": len(temps)},
        "occupancy": {"t_s": [round(float(x), 3) for x in ot[:: max(1, len(ot) // 64)]],
                      "reserved_gb": [round(float(x) / 1e9, 4) for x in ob[:: max(1, len(ob) // 64)]]},
    }
    print(json.dumps(result), flush=True)


def batching_main(args):
    """Batched Green's sequences against the one-vector loops, same spectra required."""
    import torch

    import paper_1802_02854_amd as ftk
    from seeded_inputs import BASE_SEED, SUPERCELLS, omega_grid
    ctx = ftk.Context(0)
    omega = omega_grid(-4.0, 4.0, 2000)
    n, L = 500, 4
    out = {"metric": "Krylov iters/s, batched vs one-vector loops (same spectra)", "unit": "Krylov iters/s",
           "n_gpus": 1, "dtype": "f64", "data": "synthetic", "higher_is_better": True, "vs_baseline": None,
           "config": {"workload": "batching: one random vector at T = inf, L = 4 shells on the automatic window, "
                                  "4 momenta, alpha = z: 16 Green's sequences of 500 steps, 2000 shifts, eta 0.01",
                      "n_steps": n, "n_omega": len(omega), "sequences": 16}, "results": {}}
    for N in [int(x) for x in args.batching_sizes.split(",")]:
        cl = ftk.plan_layout(ftk.honeycomb_cluster(*SUPERCELLS[N]))[0]
        h = ftk.Hamiltonian(ctx, cl, -1.0, 0.1)
        if N == 24:
            qs = [ftk.named_momentum(q) for q in ("Gamma", "M", "K", "M'")]
        else:
            qs = [tuple(q) for q in ftk.honeycomb_momenta(*SUPERCELLS[N])[:4]]
        st = ftk.TypicalStates(h, seed=BASE_SEED, n_vectors=1, betas=[0.0], E_b=None, eps=None, L=L, M=16,
                               n_steps=n, window_margin=0.1)
        nseq = int((st.scalars()[1] > 0).sum()) * len(qs)
        res, ref = {}, None
        runs = [("plain_loop_B1", 1, 1, -1), ("one_vector_B1", 1, 0, -1)] + [("block_B16", 16, 0, 0)] * 2
        if N >= 16:  # a multi-pass plan exists: batches can run as a stack
            runs += [("stacked_B4", 4, 0, 1)] * 2 + [("stacked_B16", 16, 0, 1)] * 2
        for name, B, plain, stack in runs:
            ftk.set_tuning("plain_loop", plain)
            ftk.set_tuning("stack_batch", stack)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sp = ftk.Spectrum(h, st, q_xy=qs, omega=omega, eta=0.01, n_steps=n, alpha_mask=4, rhs_block=B)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            finally:
                ftk.set_tuning("plain_loop", 0)
                ftk.set_tuning("stack_batch", -1)
            g, _ = sp.raw()
            if ref is None:
                ref = g
            same = bool(np.array_equal(g, ref))
            if not same:
                raise SystemExit(f"N={N} {name}: spectra differ from the plain loop")
            res[name] = nseq * n / dt  # a repeated run replaces the first (graph capture excluded)
            log(f"N={N} {name}: {nseq * n / dt:.0f} Krylov iters/s ({dt:.2f} s), identical spectra: {same}")
            sp.close()
        best = max((k for k in res if k != "plain_loop_B1"), key=lambda k: res[k])
        res["best"] = best
        res["speedup_best_vs_plain"] = res[best] / res["plain_loop_B1"]
        res["H_v_passes"] = ftk.hv_plan(cl)[0]
        out["results"][f"N{N}"] = res
        st.close()
        h.close()
    r0 = out["results"][f"N{args.batching_sizes.split(',')[0]}"]
    out["value"] = r0[r0["best"]]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (batches of Green's sequences)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--serve-sizes", default="12,14,16,18,20")
    ap.add_argument("--serve-vectors", default="2,4")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-weights", default="", help="comma list, one weight per size (default: the mix's own)")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-steps", type=int, default=0, help="Krylov steps per request (0: the workload's 300)")
    ap.add_argument("--serve-shells", type=int, default=0, help="shells per request (0: the workload's 16)")
    ap.add_argument("--batching", action="store_true")
    ap.add_argument("--batching-sizes", default="16,18,20,24")
    ap.add_argument("--workload", default="plain-N24",
                    choices=["plain-N24", "plain-N16", "plain-N16-J0", "plain-N8"])
    ap.add_argument("--rhs-block", type=int, default=0, choices=[0, 1, 4, 16, 32],
                    help="sequences per launch (0: the autotuner's pick)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel of the Green's loops instead of replaying captured graphs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the job runs on a single MI355X (independent Krylov sequences "
              "would shard over GPUs by random vector with one final all-reduce); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_main(args)
        return
    if args.batching:
        batching_main(args)
        return

    import torch

    import paper_1802_02854_amd as ftk
    if args.no_graphs:
        ftk.set_tuning("graphs", 0)
    w = workload(args.workload)
    N = w["N"]
    ctx = ftk.Context(0)
    # the cluster with its sites relabelled for the multi-pass H v (same system)
    cl = ftk.plan_layout(ftk.honeycomb_cluster(w["T1"], w["T2"]))[0]
    h = ftk.Hamiltonian(ctx, cl, w["K"], w["J"])
    if isinstance(w["q"], int):  # the first allowed momenta in canonical order
        qs = [tuple(q) for q in ftk.honeycomb_momenta(w["T1"], w["T2"])[: w["q"]]]
    else:
        qs = [ftk.named_momentum(n) for n in w["q"]]
    w["n_q"] = len(qs)
    na, L, nw, nT = len(w["betas"]), w["L"], len(w["omega_arr"]), len(w["temps_arr"])
    log(f"{w['name']}: N={N} dim={h.dim} bonds={cl.n_bonds} L={L} M={w['M']} n={w['n_green']} shifts={nw}")
    t_tune = time.perf_counter()
    if args.rhs_block:
        rhs_block = args.rhs_block
        log(f"rhs_block={rhs_block} (given)")
    else:
        rhs_block, tuned_ips = h.autotune(nw)
        log(f"autotuned rhs_block={rhs_block} ({tuned_ips:.0f} Krylov iters/s in the tuning runs, "
            f"{time.perf_counter() - t_tune:.1f} s)")
    layout = "single" if rhs_block == 1 else (h.autotune_layout(nw) if not args.rhs_block else "default")
    tuned = [] if args.rhs_block else h.autotune_candidates(nw)
    if tuned:
        log("autotuner candidates: " + ", ".join(f"B={b} {l} grid={g or 'default'} {hs} {x:.0f} it/s"
                                                  for b, l, x, g, hs in tuned))
    # one step = one batch of G Green's sequences: G consecutive shells of one (vector, anchor,
    # alpha, Q), run rhs_block at a time
    G = max(16, rhs_block)
    w["group"] = G

    # accumulated shell data of the job: [nv][na] scalars and [nv][na][L][nq] spectra
    log_norm = np.zeros((w["n_vectors"], na))
    n_m = np.zeros((w["n_vectors"], na, L))
    E_m = np.zeros((na, L))
    eps = np.array(w["eps_list"])
    Gacc = np.zeros((w["n_vectors"], na, L, len(qs), nw), dtype=np.complex128)
    have = np.zeros((w["n_vectors"], na), dtype=bool)
    cache = {}
    built = []  # seconds spent building the states of a (vector, anchor) pair, per build

    def run_step(i):
        s, a, ia, iq, g = step_of(i, w)
        key = (s, a)
        if key not in cache:
            t0 = time.perf_counter()
            cache.clear()
            cache[key] = ftk.TypicalStates(
                h, seed=w["seed"], first_vector=s, n_vectors=1, betas=[w["betas"][a]], E_b=w["E_b"],
                eps=w["eps_list"][a], L=L, M=w["M"], n_steps=w["n_filter"])
            ln, nm, em, _ = cache[key].scalars()
            log_norm[s, a], n_m[s, a], E_m[a] = ln[0, 0], nm[0, 0], em[0]
            have[s, a] = True
            built.append(time.perf_counter() - t0)
        m0 = g * G
        cnt = min(G, L - m0)
        sp = ftk.Spectrum(h, cache[key], q_xy=[qs[iq]], omega=w["omega_arr"], eta=w["eta"],
                          n_steps=w["n_green"], alpha_mask=1 << ia, rhs_block=rhs_block, shells=(m0, cnt))
        gr, _ = sp.raw()
        Gacc[s, a, m0:m0 + cnt, iq, :] += gr[0, 0, m0:m0 + cnt, 0, 0, :]
        sp.close()
        seqs = int((n_m[s, a, m0:m0 + cnt] > 0).sum())
        return seqs * w["n_green"]

    def reweight_all():
        """S(Q, w, T') of everything accumulated so far: the vectors with any data, over
        the anchors every one of them has."""
        vs = np.flatnonzero(have.any(axis=1))
        if not len(vs):
            return
        an = np.flatnonzero(have[vs].all(axis=0))
        if len(an):
            sel = np.ix_(vs, an)
            ftk.reweight([w["betas"][k] for k in an], E_m[an], eps[an], log_norm[sel], n_m[sel], Gacc[sel],
                         w["temps_arr"], n_bins=min(8, len(vs)))

    # timed steps in job order from the first step of (vector 0, anchor T = 1), so that
    # the first of them builds that pair's states (random vector, imaginary-time state,
    # both filter passes, shell accumulation); the warmup runs the same anchor on the
    # last vector
    per_pair = steps_per_pair(w)
    a_t = min(1, na - 1)
    first_timed = a_t * per_pair
    first_warm = ((w["n_vectors"] - 1) * na + a_t) * per_pair
    for i in range(args.warmup):
        log(f"warmup step {i} (vector, anchor, alpha, Q, shell group) = {step_of(first_warm + i, w)}")
        run_step(first_warm + i)
    reweight_all()
    torch.cuda.synchronize()
    built.clear()
    ctx.set_timing(True)
    iters = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        iters += run_step(first_timed + i)
        log(f"timed step {i} {step_of(first_timed + i, w)} done at {time.perf_counter() - t0:.1f} s")
    reweight_all()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_st, ms_st = ctx.kernel_time("lanczos_step")  # per-step events (loops without graphs)
    n_bl, ms_bl = ctx.kernel_time("lanczos_block")  # whole graph-replayed n-step loops
    if n_bl:  # a block advances rhs_block sequences by n_green steps
        n_st, ms_st = n_bl * w["n_green"], ms_bl / w["n_green"]
    ctx.set_timing(False)

    # standalone H v (the headline kernel), timed on the library's stream
    v = torch.randn(h.dim, dtype=torch.complex128, device="cuda")
    out = torch.empty_like(v)
    for _ in range(3):
        h.apply(v, out)
    ctx.set_timing(True)
    for _ in range(20):
        h.apply(v, out)
    n_ap, ms_ap = ctx.kernel_time("apply_h")
    ctx.set_timing(False)
    # plain copy of one vector: the practical bandwidth ceiling (STREAM-style copy, read +
    # write) measured in the same run
    c = torch.empty_like(v)
    for _ in range(3):
        c.copy_(v)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        c.copy_(v)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 32.0 * h.dim / (e0.elapsed_time(e1) * 1e-3) / 1e9
    dim = h.dim
    hv_bytes = 32.0 * dim  # read v + write w
    # one Lanczos step of one sequence: read v_k and v_{k-1}, write v_{k+1}; a timed
    # step advances rhs_block sequences
    st_bytes = 48.0 * dim * rhs_block
    hv_gbs = hv_bytes / (ms_ap * 1e-3) / 1e9
    st_gbs = st_bytes / (ms_st * 1e-3) / 1e9
    log(f"lanczos_step {n_st} x {ms_st:.3f} ms ({st_gbs:.0f} GB/s algorithmic at 48 B/element), "
        f"apply_h {n_ap} x {ms_ap:.3f} ms ({hv_gbs:.0f} GB/s), H v passes {ftk.hv_plan(cl)}")

    hv_traffic = measured_traffic("apply_h", "single", 1, hv_bytes)
    st_traffic = measured_traffic("lanczos_step", "single" if rhs_block == 1 else layout, rhs_block, st_bytes)
    result = {
        "metric": METRIC,
        "value": iters / dt,
        "unit": "Krylov iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload_text(w, len(qs)),
                   "N": N, "n_vectors": w["n_vectors"], "anchors_T": [str(T) for T in w["temps_anchor"]],
                   "n_steps": w["n_green"], "n_omega": nw, "n_q": len(qs), "n_T": nT, "L": L, "M": w["M"],
                   "sequences_per_step": G, "rhs_block": rhs_block, "batch_layout": layout,
                   "graphs": not args.no_graphs,
                   "autotune": [{"rhs_block": b, "layout": l, "pass_grid": g, "hints": hs, "iters_per_s": x}
                                for b, l, x, g, hs in tuned]},
        "roofline": {"bound": "hbm",
                     "kernel": f"lanczos_step (all launches of one Lanczos step of {rhs_block} sequence(s) incl. "
                               f"the {nw}-shift update)",
                     "achieved": st_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": st_gbs / HBM_PEAK_GBS,
                     "traffic": st_traffic,
                     "algorithmic_bytes_per_launch": st_bytes,
                     "algorithmic_bytes_per_element": 48,
                     "mean_launch_ms": ms_st, "timed_launches": n_st,
                     "traffic_over_algorithmic": (st_traffic / st_bytes if st_traffic else None),
                     # counter bytes over the same launch time: the HBM rate actually drawn
                     "traffic_gbps": (st_traffic / (ms_st * 1e6) if st_traffic else None),
                     "frac_two_sweep_96B": 2.0 * st_gbs / HBM_PEAK_GBS},
        "hv_roofline": {"bound": "hbm", "kernel": "apply_h (H v of one vector, all passes)",
                        "achieved": hv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hv_gbs / HBM_PEAK_GBS,
                        "algorithmic_bytes_per_launch": hv_bytes, "mean_launch_ms": ms_ap, "timed_launches": n_ap,
                        "traffic": hv_traffic,
                        "traffic_over_algorithmic": (hv_traffic / hv_bytes if hv_traffic else None),
                        "traffic_gbps": (hv_traffic / (ms_ap * 1e6) if hv_traffic else None)},
        "copy_gbps": copy_gbs,
        "frac_of_copy": st_gbs / copy_gbs,
        "state_build_s": built,
        "krylov_iters": iters,
        "kernel_source": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
