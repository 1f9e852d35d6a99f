"""The host half of the library (csrc/host_math.cpp: clusters, momenta, layout
planner, tridiagonal steps, shell coefficients, reweighting, thermodynamics,
anchors, peak fit) built with g++ under the address and undefined-behaviour
sanitizers and driven over sizes from the degenerate (one step, one sample, one
bin per sample, five fit points) to the 26-site cluster; any sanitizer report
fails the test.  The routines' values are checked against the oracle elsewhere.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1802_02854_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "ftkw_internal.h"
using namespace ftk;

static int failures = 0;
#define EXPECT(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++failures; } } while (0)

int main()
{
    std::mt19937_64 g(7);
    std::normal_distribution<double> N01;
    std::uniform_real_distribution<double> U(0, 1);
    const int shapes[][4] = {{1, 1, -1, 2}, {2, 0, 0, 2}, {2, 2, -2, 2}, {3, 0, 0, 3}, {2, 2, -2, 4}, {3, 1, -1, 4}};
    for (auto &s : shapes) {
        HoneyCluster c = honeycomb(s[0], s[1], s[2], s[3]);
        const int ns = (int)c.xy.size() / 2, nb = (int)c.bi.size();
        EXPECT(nb == 3 * ns / 2);
        auto q = honeycomb_momenta(s[0], s[1], s[2], s[3]);
        EXPECT((int)q.size() == ns);  // N/2 momenta, two numbers each
        std::vector<double> h(2 * ns);
        for (size_t k = 0; k + 1 < q.size(); k += 2) sq_coefficients(ns, c.xy.data(), q[k], q[k + 1], h.data());
        std::vector<int32_t> perm(ns), order(nb);
        const int P = plan_layout(ns, nb, c.bi.data(), c.bj.data(), 12, 8, perm.data(), order.data());
        EXPECT(P >= 0 && P <= 6);
    }
    double qq[2];
    EXPECT(named_momentum("M", qq) && !named_momentum("nonsense", qq));
    for (int n : {1, 2, 5, 64, 300}) {
        std::vector<double> a(n), b(n), zr(40), zi(40), hist(n), coef((size_t)16 * n * 2);
        for (int k = 0; k < n; ++k) a[k] = N01(g), b[k] = 0.5 + U(g);
        for (int k = 0; k < 40; ++k) zr[k] = -3 + 6 * U(g), zi[k] = 0.01 + 0.1 * U(g);
        double lo, hi, Eb, eps;
        ritz_extremes(a.data(), b.data(), n, &lo, &hi);
        EXPECT(lo <= hi);
        shell_window(a.data(), b.data(), n, 16, 0.1, &Eb, &eps);
        EXPECT(eps > 0);
        residual_history(a.data(), b.data(), n, zr.data(), zi.data(), 40, hist.data());
        const int k = truncation_steps(a.data(), b.data(), n, zr.data(), zi.data(), 40, 1e-6);
        EXPECT(k >= 1 && k <= n);
        std::vector<int> kn(16);
        for (int m = 0; m < 16; ++m) kn[m] = 1 + (int)(U(g) * n) % n;
        shell_coefficients(a.data(), b.data(), n, 1.3, Eb, eps, 16, 16, coef.data());
        shell_coefficients(a.data(), b.data(), n, 1.3, Eb, eps, 16, 16, coef.data(), kn.data());
    }
    for (int nv : {1, 3, 8, 17}) {
        const int na = 2, L = 7, nq = 2, nw = 9, nT = 5;
        const double betas[2] = {0.0, 1.0};
        std::vector<double> E_m(na * L), eps(na, 0.1), ln(nv * na), n_m(nv * na * L),
            gg((size_t)nv * na * L * nq * nw * 2);
        for (int a = 0; a < na; ++a)
            for (int m = 0; m < L; ++m) E_m[a * L + m] = -2 + 0.5 * m;
        for (auto &x : ln) x = N01(g);
        for (auto &x : n_m) x = U(g) < 0.1 ? 0.0 : U(g);
        for (auto &x : gg) x = N01(g);
        std::vector<double> T = {0.1, 0.5, 1.0, 3.0, 100.0}, S(nq * nT * nw), Se(S.size()), P(nT * L);
        for (int bins : {0, 2, 8, 40})
            reweight(nv, na, L, nq, nw, betas, E_m.data(), eps.data(), ln.data(), n_m.data(), gg.data(), T.data(),
                     nT, bins, S.data(), Se.data(), P.data());
        for (double x : S) EXPECT(std::isfinite(x));
        std::vector<double> O((size_t)nv * na * L * 3), out(3 * nT), err(3 * nT);
        for (auto &x : O) x = N01(g);
        reweight_observable(nv, na, L, 3, betas, E_m.data(), ln.data(), n_m.data(), O.data(), T.data(), nT, 8,
                            out.data(), err.data());
        std::vector<double> h1(n_m.size()), h2(n_m.size()), to(nT * 4), te(nT * 4), it(nT);
        for (size_t i = 0; i < h1.size(); ++i) h1[i] = n_m[i] * N01(g), h2[i] = n_m[i] * (1 + U(g));
        thermodynamics(nv, na, L, betas, E_m.data(), ln.data(), n_m.data(), h1.data(), h2.data(), 12, T.data(), nT,
                       8, to.data(), te.data());
        thermodynamics(nv, na, L, betas, E_m.data(), ln.data(), n_m.data(), nullptr, nullptr, 12, T.data(), nT, 8,
                       to.data(), nullptr);
        for (int i = 0; i < nT; ++i) it[i] = 1.0 / T[i];
        std::vector<double> dout(nT * 2), derr(nT * 2);
        thermo_diagnostics(nv, na, L, betas, E_m.data(), ln.data(), n_m.data(), h1.data(), h2.data(), 12, it.data(),
                           nT, 8, dout.data(), derr.data());
    }
    {
        std::vector<double> E(41), var(41);
        for (int i = 0; i < 41; ++i) {
            const double ch = std::cosh(0.125 * i);
            E[i] = -2 * std::tanh(0.125 * i), var[i] = 0.8 / (ch * ch) + 1e-3;
        }
        std::vector<int> an(41);
        for (int cap : {1, 3, 41}) {
            const int k = choose_anchors(41, E.data(), var.data(), 0.3, cap, an.data());
            EXPECT(k >= 1 && k <= cap && an[0] == 0);
        }
    }
    for (int n : {5, 6, 101, 601}) {
        std::vector<double> w(n), y(n);
        for (int i = 0; i < n; ++i) {
            w[i] = 1.0 + (double)i / (n - 1);
            const double x = w[i] - 1.35;
            y[i] = 0.22 / (0.22 * 0.22 + x * x) * (0.3 + 0.25 / (1 + std::exp(6 * x))) * (1 + 0.02 * N01(g));
        }
        double p[5], cost;
        asym_lorentzian_start(w.data(), y.data(), n, p);
        fit_asym_lorentzian(w.data(), y.data(), n, 1000, p, &cost);
        EXPECT(p[3] > 0 && std::fabs(p[4] - 1.35) < 0.1);
        double p2[5] = {1, 1, 300, 1e-3, 1.5};  // a far start with a steep step
        fit_asym_lorentzian(w.data(), y.data(), n, 50, p2, &cost);
        EXPECT(p2[3] > 0);
    }
    std::printf(failures ? "FAILED\n" : "OK\n");
    return failures ? 1 : 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_math_under_sanitizers(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-I", CSRC, str(src), os.path.join(CSRC, "host_math.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "Sanitizer" not in out.stderr, out.stderr
    assert out.stdout.strip().endswith("OK"), out.stdout
