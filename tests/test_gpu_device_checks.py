"""The debug library with device bounds checks (libftkw_check.so, FTK_LIBRARY=check).

A child process on the debug library runs a workload that reaches every
instrumented kernel form: the single-element (8 sites), blocked (12) and tiled (16)
H v, the two-pass (18, planner's labels) and three-pass (24) forms, the fused
Lanczos step, the block layout (B = 4) and a stack of multi-pass sequences, the
Taylor and filter kernels (8, 18 and 24 sites), S^alpha_Q, a linear spin operator
and shifted COCG.  It
must report zero violations, and its results must be bit for bit those of the
release library run here on the same inputs (the checks change no arithmetic).  The
counter itself is exercised by the self-test, a claimed access outside a 4-entry
buffer that touches no memory there.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from seeded_inputs import SUPERCELLS, gaussian_vector, real_vector

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def workload(ftk, torch, ctx):
    """Outputs of every instrumented kernel form, keyed by name."""
    out = {}

    def dev(v):
        return torch.from_numpy(np.ascontiguousarray(v).view(np.complex128)).to("cuda")

    def system(N, relabel):
        cl = ftk.honeycomb_cluster(*SUPERCELLS[N])
        if relabel:
            cl = ftk.plan_layout(cl)[0]
        return ftk.Hamiltonian(ctx, cl, -1.0, 0.1)

    for N, relabel in ((8, False), (12, False), (16, False), (18, True), (24, True)):
        h = system(N, relabel)
        out[f"hv{N}"] = h.apply(dev(real_vector(900 + N, 2 << N))).cpu().numpy()
        print(f"  hv N={N}", flush=True)
    omega = np.linspace(-3, 3, 41)
    for N, relabel, n in ((8, False, 24), (18, True, 12), (24, True, 8)):
        h = system(N, relabel)
        g0 = gaussian_vector(31, 0, N)
        st = ftk.TypicalStates(h, seed=31, n_vectors=1, betas=[0.0, 1.0], E_b=-0.6, eps=0.05, L=4, M=8,
                               n_steps=n, gaussians=dev(g0).reshape(1, -1))
        ln, nm, _, _ = st.scalars()
        out[f"nm{N}"] = nm
        out[f"ln{N}"] = ln
        q = [tuple(x) for x in ftk.honeycomb_momenta(*SUPERCELLS[N])[:2]]
        for B in (1, 4):
            sp = ftk.Spectrum(h, st, q_xy=q, omega=omega, eta=0.1, n_steps=n, alpha_mask=7, rhs_block=B)
            out[f"g{N}_B{B}"] = sp.raw()[0]
            sp.close()
        if N == 8:
            cl = ftk.honeycomb_cluster(*SUPERCELLS[N])
            op_a = np.stack([ftk.momentum_operator(cl, 0, q[1])])
            op_b = np.zeros_like(op_a)
            op_b[0, 1, 2] = 1.0
            ps = ftk.PairSpectrum(h, st, op_a=op_a, op_b=op_b, omega=omega, eta=0.1, n_steps=n)
            out["pair8"] = ps.raw()[0]
            ps.close()
            sp = ftk.Spectrum(h, st, q_xy=q, omega=omega, eta=0.1, n_steps=n, alpha_mask=3, solver="cocg")
            out["cocg8"] = sp.raw()[0]
            sp.close()
        print(f"  pipeline N={N}", flush=True)
    return out


def _child(path):
    import torch

    import paper_1802_02854_amd as ftk
    assert ftk.LIB_PATH.endswith("libftkw_check.so"), ftk.LIB_PATH
    ctx = ftk.Context(0)
    compiled, v, _, _ = ctx.device_checks(clear=True)
    assert compiled and v == 0
    assert ctx.device_checks_selftest() == 0
    compiled, v, site, idx = ctx.device_checks(clear=True)
    assert (v, site, idx) == (1, 99, 5), (v, site, idx)
    out = workload(ftk, torch, ctx)
    compiled, v, site, idx = ctx.device_checks()
    out["violations"] = np.array([v, site, idx])
    np.savez(path, **out)


@pytest.mark.gpu
def test_debug_build_finds_no_violation_and_changes_no_bit(tmp_path):
    import torch

    import paper_1802_02854_amd as ftk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    assert os.path.exists(os.path.join(ROOT, "paper_1802_02854_amd", "libftkw_check.so"))
    path = str(tmp_path / "checked.npz")
    print("device checks: child on the debug library", flush=True)
    env = dict(os.environ, FTK_LIBRARY="check", PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), path], env=env, cwd=ROOT, timeout=300)
    assert r.returncode == 0
    got = dict(np.load(path))
    assert list(got.pop("violations")) == [0, 0, 0]
    print("device checks: the same workload on the release library", flush=True)
    ctx = ftk.Context(0)
    assert ctx.device_checks() == (False, 0, 0, 0)
    ref = workload(ftk, torch, ctx)
    assert sorted(ref) == sorted(got)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k


if __name__ == "__main__":
    _child(sys.argv[1])
