"""Failure paths of the C-ABI that need the device: non-finite numbers reach the
library as FTK_ENUMERIC (a numeric check on the host side of the call, no device
fault), and the context keeps working afterwards."""
import ctypes

import numpy as np
import pytest

from seeded_inputs import SUPERCELLS, gaussian_vector

pytestmark = pytest.mark.gpu

FTK_ENUMERIC = -4


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1802_02854_amd as ftk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = ftk.Context(0)
    h = ftk.Hamiltonian(ctx, ftk.honeycomb_cluster(*SUPERCELLS[12]), -1.0, 0.1)
    return ftk, torch, ctx, h


def _states(ftk, torch, h, g):
    G = torch.from_numpy(np.ascontiguousarray(g).view(np.complex128)).to("cuda").reshape(1, -1)
    return ftk.TypicalStates(h, seed=1, n_vectors=1, betas=[0.0, 1.0], E_b=-2.0, eps=0.1, L=8, M=8, n_steps=12,
                             gaussians=G)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_start_vector_is_enumeric(env, bad):
    """A start vector with one NaN or infinite entry: FTK_ENUMERIC through the C-ABI with a
    message; nothing else happens on the device."""
    ftk, torch, ctx, h = env
    print(f"non-finite start vector {bad}", flush=True)
    g = gaussian_vector(5, 0, 12)
    g[2 * 777 + 1] = bad
    with pytest.raises(ftk.FTKError) as e:
        _states(ftk, torch, h, g)
    assert e.value.status == FTK_ENUMERIC
    assert "norm" in str(e.value)


def test_overflowing_start_vector_is_enumeric(env):
    """Finite entries whose squared norm overflows: FTK_ENUMERIC, not a silent Inf."""
    ftk, torch, ctx, h = env
    g = gaussian_vector(6, 0, 12) * 1e300
    with pytest.raises(ftk.FTKError) as e:
        _states(ftk, torch, h, g)
    assert e.value.status == FTK_ENUMERIC


def test_context_usable_after_numeric_error(env):
    """After the failures above the same context and Hamiltonian give a normal result."""
    ftk, torch, ctx, h = env
    st = _states(ftk, torch, h, gaussian_vector(7, 0, 12))
    ln, nm, em, ep = st.scalars()
    assert np.isfinite(ln).all() and np.isfinite(nm).all() and (nm >= 0).all()
    sp = ftk.Spectrum(h, st, q_xy=[(0.0, 0.0)], omega=np.linspace(-2, 2, 9), eta=0.1, n_steps=12, alpha_mask=4)
    g, r = sp.raw()
    assert np.isfinite(g).all()


def test_direct_c_call_status(env):
    """The raw C entry point returns the status code itself (no Python exception layer)."""
    ftk, torch, ctx, h = env
    from paper_1802_02854_amd import _lib
    g = gaussian_vector(8, 0, 12)
    g[0] = np.nan
    G = torch.from_numpy(g.view(np.complex128)).to("cuda")
    betas = np.array([0.0])
    E_b = np.array([-2.0])
    eps = np.array([0.1])
    p = _lib.TsParamsC(1, 0, 1, betas.ctypes.data, 1, E_b.ctypes.data, eps.ctypes.data, 4, 8, 6, 0.0,
                       G.data_ptr(), 0, 0.0, 0.0, 0)
    out = ctypes.c_void_p()
    rc = _lib.lib().ftk_typical_states(h.handle, ctypes.byref(p), ctypes.byref(out))
    assert rc == FTK_ENUMERIC and not out.value
    assert b"norm" in _lib.lib().ftk_last_error()
