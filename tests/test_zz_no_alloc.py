"""ftk_apply_h_noalloc: H v with the multi-pass partial sums in the library's static
device array instead of the Hamiltonian's scratch vector, called through the C-ABI,
against ftk_apply_h (bit for bit) on two calls in a row, the second on a smaller
input; sizes beyond the static maximum are refused; no device memory is allocated."""
import ctypes

import numpy as np
import pytest

from seeded_inputs import SUPERCELLS, real_vector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1802_02854_amd as ftk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ftk, torch, ftk.Context(0)


def _cabi(ftk, h, v, w, n_rhs):
    from paper_1802_02854_amd import _lib
    return _lib.lib().ftk_apply_h_noalloc(h.handle, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                          n_rhs)


def test_noalloc_matches_apply_h_twice(env):
    """Two calls in a row through the C-ABI -- 20 sites with three vectors (multi-pass
    form, partial sums in the static array), then 18 sites with one vector (a smaller
    input; same array, the first call's contents left behind) -- each bit for bit equal
    to ftk_apply_h; the context's device memory does not change during the calls."""
    ftk, torch, ctx = env
    runs = []
    for N, n_rhs in ((20, 3), (18, 1)):
        print(f"apply_h_noalloc N={N} n_rhs={n_rhs}", flush=True)
        cl = ftk.plan_layout(ftk.honeycomb_cluster(*SUPERCELLS[N]))[0]
        h = ftk.Hamiltonian(ctx, cl, -1.0, 0.1)
        v = torch.from_numpy(real_vector(900 + N, n_rhs * (2 << N)).view(np.complex128)).to("cuda")
        v = v.reshape(n_rhs, -1)
        ref = h.apply(v)
        out = torch.full_like(v, complex(np.nan, np.nan))
        torch.cuda.synchronize()
        before = ctx.memory_in_use()
        assert _cabi(ftk, h, v, out, n_rhs) == 0
        assert ctx.memory_in_use() == before
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref)), N
        runs.append((h, v, ref))
    # the first Hamiltonian once more after the smaller call
    h, v, ref = runs[0]
    out = torch.empty_like(v)
    assert _cabi(ftk, h, v, out, v.shape[0]) == 0
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref))
    # the binding's method is the same call
    out2 = h.apply_noalloc(v[0], torch.empty_like(v[0]))
    assert torch.equal(torch.view_as_real(out2), torch.view_as_real(ref[0]))


def test_noalloc_small_form_and_size_limit(env):
    """A 12-site cluster (a form without partial sums) runs at any size; the 24-site
    multi-pass form needs more than the static maximum and is refused with FTK_EINVAL
    before any device work."""
    ftk, torch, ctx = env
    h12 = ftk.Hamiltonian(ctx, ftk.honeycomb_cluster(*SUPERCELLS[12]), -1.0, 0.1)
    v = torch.from_numpy(real_vector(912, 2 << 12).view(np.complex128)).to("cuda")
    out = torch.empty_like(v)
    assert _cabi(ftk, h12, v, out, 1) == 0
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(out), torch.view_as_real(h12.apply(v)))
    cl = ftk.plan_layout(ftk.honeycomb_cluster(*SUPERCELLS[24]))[0]
    h24 = ftk.Hamiltonian(ctx, cl, -1.0, 0.1)
    x = torch.zeros(1 << 24, dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    from paper_1802_02854_amd import _lib
    assert _cabi(ftk, h24, x, y, 1) == -1
    assert b"static maximum" in _lib.lib().ftk_last_error()
    torch.cuda.synchronize()
    assert not torch.view_as_real(y).any()
