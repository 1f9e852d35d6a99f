"""Python binding of libftkw: argument marshalling only.

Every step of the method runs inside the library (HIP kernels on the GPU and its
host-side scalar code); torch supplies device memory (tensors) and the stream.
Names follow the C-ABI in include/ftkw.h.
"""
import ctypes
from dataclasses import dataclass

import numpy as np

from ._lib import (ALLOC_FN, FREE_FN, FTKError, ClusterC, PairParamsC, ServingStatsC, SpecParamsC, TsParamsC, call,
                   lib)

c_void_p = ctypes.c_void_p


def _ptr(a):
    """Address of a host numpy array (C-contiguous) or None."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return a.ctypes.data


def _dptr(t):
    """Address of a device torch tensor (contiguous) or None."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return t.data_ptr()


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ---------------------------------------------------------------------------
@dataclass
class Cluster:
    """Periodic honeycomb cluster: bonds (i, j, gamma) in accumulation order, site positions."""
    n_sites: int
    bond_i: np.ndarray
    bond_j: np.ndarray
    bond_gamma: np.ndarray
    site_xy: np.ndarray
    T1: tuple = None
    T2: tuple = None

    @property
    def n_bonds(self):
        return len(self.bond_i)

    @property
    def bonds(self):
        return [(int(i), int(j), int(g)) for i, j, g in zip(self.bond_i, self.bond_j, self.bond_gamma)]

    def relabeled(self, site_perm, bond_order):
        """The same system with site l renamed site_perm[l] and bonds listed in bond_order."""
        perm = np.asarray(site_perm, dtype=np.int64)
        order = np.asarray(bond_order, dtype=np.int64)
        xy = np.empty_like(np.asarray(self.site_xy, dtype=np.float64))
        xy[perm] = self.site_xy
        return Cluster(self.n_sites, perm[self.bond_i[order]].astype(np.int32),
                       perm[self.bond_j[order]].astype(np.int32), self.bond_gamma[order].astype(np.int8), xy,
                       self.T1, self.T2)

    def as_c(self):
        self._keep = (np.ascontiguousarray(self.bond_i, dtype=np.int32),
                      np.ascontiguousarray(self.bond_j, dtype=np.int32),
                      np.ascontiguousarray(self.bond_gamma, dtype=np.int8),
                      np.ascontiguousarray(self.site_xy, dtype=np.float64))
        bi, bj, bg, xy = self._keep
        return ClusterC(self.n_sites, len(bi), _ptr(bi), _ptr(bj), _ptr(bg), _ptr(xy))


def honeycomb_cluster(T1, T2):
    (t11, t12), (t21, t22) = T1, T2
    n_sites, n_bonds = ctypes.c_int(), ctypes.c_int()
    call("ftk_honeycomb_cluster", t11, t12, t21, t22, ctypes.byref(n_sites), ctypes.byref(n_bonds),
         None, None, None, None)
    bi = np.zeros(n_bonds.value, np.int32)
    bj = np.zeros(n_bonds.value, np.int32)
    bg = np.zeros(n_bonds.value, np.int8)
    xy = np.zeros((n_sites.value, 2))
    call("ftk_honeycomb_cluster", t11, t12, t21, t22, ctypes.byref(n_sites), ctypes.byref(n_bonds),
         _ptr(bi), _ptr(bj), _ptr(bg), _ptr(xy))
    return Cluster(n_sites.value, bi, bj, bg, xy, tuple(T1), tuple(T2))


def plan_layout(cluster):
    """(relabelled cluster, n_passes, site_perm, bond_order) for the multi-pass H v."""
    perm = np.zeros(cluster.n_sites, np.int32)
    order = np.zeros(cluster.n_bonds, np.int32)
    n = ctypes.c_int()
    c = cluster.as_c()
    call("ftk_plan_layout", ctypes.byref(c), _ptr(perm), _ptr(order), ctypes.byref(n))
    return cluster.relabeled(perm, order), n.value, perm, order


def hv_plan(cluster):
    """(n_passes, core, segment ends) of the multi-pass H v for this bond list."""
    n, core = ctypes.c_int(), ctypes.c_int()
    ends = np.zeros(8, np.int32)
    c = cluster.as_c()
    call("ftk_hv_plan", ctypes.byref(c), ctypes.byref(n), ctypes.byref(core), _ptr(ends))
    return n.value, core.value, [int(e) for e in ends[: n.value]]


def honeycomb_momenta(T1, T2):
    (t11, t12), (t21, t22) = T1, T2
    n = ctypes.c_int()
    call("ftk_honeycomb_momenta", t11, t12, t21, t22, ctypes.byref(n), None)
    q = np.zeros((n.value, 2))
    call("ftk_honeycomb_momenta", t11, t12, t21, t22, ctypes.byref(n), _ptr(q))
    return q


def named_momentum(name):
    q = np.zeros(2)
    call("ftk_named_momentum", name.encode(), _ptr(q))
    return q


def set_tuning(key, value):
    """Process-wide tuning knob (see ftk_set_tuning in include/ftkw.h)."""
    call("ftk_set_tuning", key.encode(), int(value))


def shell_window(alpha, beta, L, margin=0.1):
    """(E_b, eps) of L shells tiling the extreme Ritz values of T_n widened by margin."""
    a, b = _f64(alpha), _f64(beta)
    if len(b) < len(a):
        b = _f64(np.concatenate([b, np.zeros(len(a) - len(b))]))
    E_b, eps = ctypes.c_double(), ctypes.c_double()
    call("ftk_shell_window", _ptr(a), _ptr(b), len(a), int(L), float(margin), ctypes.byref(E_b), ctypes.byref(eps))
    return E_b.value, eps.value


def truncation_steps(alpha, beta, z, tol):
    """First k whose Galerkin residuals over the shifts z are all <= tol (per unit RHS)."""
    a, b = _f64(alpha), _f64(beta)
    z = np.asarray(z, dtype=np.complex128)
    zr, zi = _f64(z.real), _f64(z.imag)
    k = ctypes.c_int()
    call("ftk_truncation_steps", _ptr(a), _ptr(b), len(a), _ptr(zr), _ptr(zi), len(zr), float(tol), ctypes.byref(k))
    return k.value


def residual_history(alpha, beta, z):
    """Largest Galerkin residual over the shifts z after each step (per unit RHS), [n]."""
    a, b = _f64(alpha), _f64(beta)
    z = np.asarray(z, dtype=np.complex128)
    zr, zi = _f64(z.real), _f64(z.imag)
    out = np.zeros(len(a))
    call("ftk_residual_history", _ptr(a), _ptr(b), len(a), _ptr(zr), _ptr(zi), len(zr), _ptr(out))
    return out


def fit_asymmetric_lorentzian(omega, s, lo=1.0, hi=2.0, init=None, max_iter=0):
    """Asymmetric-Lorentzian fit of a spectrum on [lo, hi] (Sec. V.F, Eq. asymmetricLorentzian): dict with
    a, b, c, gamma, eps, width_ratio = gamma / eps, cost and iters."""
    w, y = _f64(omega), _f64(s)
    if w.shape != y.shape or w.ndim != 1:
        raise ValueError("omega and s must be 1-D arrays of one length")
    p0 = None if init is None else _f64(init)
    if p0 is not None and p0.shape != (5,):
        raise ValueError("init must hold (a, b, c, gamma, eps)")
    out = np.zeros(5)
    cost, iters, ratio = ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
    call("ftk_fit_asymmetric_lorentzian", _ptr(w), _ptr(y), len(w), float(lo), float(hi),
         None if p0 is None else _ptr(p0), int(max_iter), _ptr(out), ctypes.byref(cost), ctypes.byref(iters),
         ctypes.byref(ratio))
    a, b, c, g, e = (float(x) for x in out)
    return {"a": a, "b": b, "c": c, "gamma": g, "eps": e, "width_ratio": ratio.value, "cost": cost.value,
            "iters": iters.value}


def filter_coefficients(alpha, beta, norm, E_b, eps, L, M):
    """c^m_k [L, n] complex (the host-side step of typical_states, Sec. III.B)."""
    alpha, beta = _f64(alpha), _f64(beta)
    n = len(alpha)
    assert len(beta) == n
    out = np.zeros((L, n), dtype=np.complex128)
    call("ftk_filter_coefficients", _ptr(alpha), _ptr(beta), n, float(norm), float(E_b), float(eps), int(L),
         int(M), _ptr(out.view(np.float64)))
    return out


def taylor_plan(n_sites, beta, norm_bound, lam=0.0):
    """(M_d, K, c, l) of the Appendix-A imaginary-time series."""
    md, k, c, ell = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    call("ftk_taylor_plan", int(n_sites), float(beta), float(norm_bound), float(lam), ctypes.byref(md),
         ctypes.byref(k), ctypes.byref(c), ctypes.byref(ell))
    return md.value, k.value, c.value, ell.value


def random_vector(ctx, seed, sample, n_sites):
    """Un-normalised complex Gaussian draws (device tensor, complex128 [2^N])."""
    import torch
    out = torch.empty(1 << n_sites, dtype=torch.complex128, device=ctx.torch_device)
    call("ftk_random_vector", ctx.handle, int(seed) & 0xFFFFFFFFFFFFFFFF, int(sample), int(n_sites),
         c_void_p(_dptr(out)))
    return out


# ---------------------------------------------------------------------------
class Context:
    """One GPU and one HIP stream (torch's current stream unless given)."""

    def __init__(self, device=0, stream=None, allocator=None):
        """allocator="torch" takes the library's device memory from torch's caching
        allocator, in stream order on a torch stream that the context then uses
        (a new one unless given)."""
        import torch
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = (torch.cuda.Stream(self.torch_device) if allocator == "torch"
                      else torch.cuda.current_stream(self.torch_device))
        self.stream = stream
        h = c_void_p()
        if allocator is None:
            call("ftk_ctx_create", device, c_void_p(stream.cuda_stream), ctypes.byref(h))
        elif allocator == "torch":
            def _alloc(nbytes, _user):
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)

            def _free(ptr, _user):
                torch.cuda.caching_allocator_delete(ptr)

            # the callbacks must outlive the context
            self._alloc_cb, self._free_cb = ALLOC_FN(_alloc), FREE_FN(_free)
            call("ftk_ctx_create_with_allocator", device, c_void_p(stream.cuda_stream), self._alloc_cb, self._free_cb,
                 None, ctypes.byref(h))
        else:
            raise ValueError("allocator must be None or 'torch'")
        self.handle = h

    def sync(self):
        call("ftk_sync", self.handle)

    def peak_memory(self, reset=False):
        """Largest device byte count held since the last reset."""
        b = ctypes.c_size_t()
        call("ftk_ctx_peak_memory", self.handle, ctypes.byref(b), int(bool(reset)))
        return b.value

    def memory_in_use(self):
        b = ctypes.c_size_t()
        call("ftk_ctx_memory", self.handle, ctypes.byref(b))
        return b.value

    def set_timing(self, enable=True):
        call("ftk_ctx_set_timing", self.handle, int(bool(enable)))

    def device_checks(self, clear=False):
        """(compiled, violations, first site, first index) of the device bounds checks
        (nonzero only with the debug library, FTK_LIBRARY=check)."""
        c = ctypes.c_int()
        v, s, i = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        call("ftk_device_checks", self.handle, ctypes.byref(c), ctypes.byref(v), ctypes.byref(s), ctypes.byref(i),
             int(bool(clear)))
        return bool(c.value), v.value, s.value, i.value

    def device_checks_selftest(self):
        """Debug library only: one claimed out-of-range access, counted and redirected;
        returns the index used instead (0)."""
        r = ctypes.c_uint32()
        call("ftk_device_checks_selftest", self.handle, ctypes.byref(r))
        return r.value

    def kernel_time(self, kernel):
        """(number of timed launches, mean duration in ms) of a timed kernel; forgets them."""
        n, ms = ctypes.c_int(), ctypes.c_double()
        call("ftk_ctx_kernel_time", self.handle, kernel.encode(), ctypes.byref(n), ctypes.byref(ms))
        return n.value, ms.value

    def close(self):
        if getattr(self, "handle", None):
            lib().ftk_ctx_destroy(self.handle)
            self.handle = None

    __del__ = close


class Hamiltonian:
    """Kitaev-Heisenberg H on a cluster (Sec. V.A); matrix-free on the device."""

    def __init__(self, ctx, cluster, K, J):
        self.ctx, self.cluster, self.K, self.J = ctx, cluster, float(K), float(J)
        cc = cluster.as_c()
        h = c_void_p()
        call("ftk_build_hamiltonian", ctx.handle, ctypes.byref(cc), self.K, self.J, ctypes.byref(h))
        self.handle = h
        n, nb = ctypes.c_int(), ctypes.c_double()
        call("ftk_hamiltonian_info", h, ctypes.byref(n), ctypes.byref(nb))
        self.n_sites, self.norm_bound = n.value, nb.value
        self.dim = 1 << self.n_sites

    def apply(self, v, out=None):
        """w = H v for a complex128 device tensor of shape [2^N] or [n_rhs, 2^N] (rows may be
        ld >= 2^N entries apart; out gets the same row spacing)."""
        import torch
        assert v.dtype == torch.complex128 and v.shape[-1] == self.dim and v.stride(-1) == 1
        ld = self.dim if v.dim() == 1 else v.stride(0)
        if out is None:
            out = torch.empty_strided(v.shape, v.stride(), dtype=v.dtype, device=v.device)
        assert out.shape == v.shape and out.stride() == v.stride(), "out must have v's shape and strides"
        n_rhs = 1 if v.dim() == 1 else v.shape[0]
        for t in (v, out):
            assert t.is_cuda and t.stride(-1) == 1 and (t.dim() == 1 or t.stride(0) == ld)
        call("ftk_apply_h_strided", self.handle, c_void_p(v.data_ptr()), c_void_p(out.data_ptr()), n_rhs, int(ld))
        return out

    def apply_noalloc(self, v, out):
        """w = H v into the caller's out (contiguous [2^N] or [n_rhs, 2^N] complex128 device
        tensors) through ftk_apply_h_noalloc: no device allocation by the library."""
        import torch
        for t in (v, out):
            assert t.dtype == torch.complex128 and t.is_cuda and t.is_contiguous() and t.shape[-1] == self.dim
        assert out.shape == v.shape
        n_rhs = 1 if v.dim() == 1 else v.shape[0]
        call("ftk_apply_h_noalloc", self.handle, c_void_p(v.data_ptr()), c_void_p(out.data_ptr()), n_rhs)
        return out

    def autotune(self, n_omega):
        """(rhs_block, Krylov iters/s) picked by the library's autotuner for this H."""
        rb, ips = ctypes.c_int(), ctypes.c_double()
        call("ftk_autotune", self.handle, int(n_omega), ctypes.byref(rb), ctypes.byref(ips))
        return rb.value, ips.value

    def autotune_candidates(self, n_omega):
        """[(rhs_block, 'stacked'|'block', iters/s, pass grid, 'streaming'|'cached')] the
        autotuner measured in this process (pass grid 0: the default; the last entry is
        the cache-hint set of the multi-pass kernels)."""
        m = 16
        rb, stk, ips = np.zeros(m, dtype=np.int32), np.zeros(m, dtype=np.int32), np.zeros(m)
        pg, hn = np.zeros(m, dtype=np.int32), np.zeros(m, dtype=np.int32)
        n = ctypes.c_int()
        call("ftk_autotune_candidates", self.handle, int(n_omega), m, ctypes.byref(n), _ptr(rb), _ptr(stk), _ptr(ips),
             _ptr(pg), _ptr(hn))
        return [(int(rb[i]), "stacked" if stk[i] else "block", float(ips[i]), int(pg[i]),
                 "streaming" if hn[i] == 1 else "cached") for i in range(n.value)]

    def autotune_layout(self, n_omega):
        """'stacked' or 'block' (one sequence per launch counts as block) for the pick."""
        st = ctypes.c_int()
        call("ftk_autotune_layout", self.handle, int(n_omega), ctypes.byref(st))
        return "stacked" if st.value else "block"

    def close(self):
        if getattr(self, "handle", None):
            lib().ftk_hamiltonian_destroy(self.handle)
            self.handle = None

    __del__ = close


class TypicalStates:
    """Filtered typical pure states phi^m for every (vector, anchor) (Sec. III.B)."""

    def __init__(self, h, *, seed, n_vectors, betas, E_b, eps, L, M, n_steps, first_vector=0,
                 gaussians=None, taylor_lambda=0.0, block_steps=0, window_margin=0.0, resid_tol=0.0,
                 shell_moments=False):
        """E_b = eps = None takes each anchor's window from vector 0's Ritz extremes
        widened by window_margin (0 -> 0.1)."""
        self.h = h
        self.betas = _f64(betas)
        na = len(self.betas)
        if (E_b is None) != (eps is None):
            raise ValueError("give both E_b and eps, or neither")
        if E_b is None:
            self.E_b = self.eps = None
        else:
            self.E_b = _f64(np.broadcast_to(np.asarray(E_b, dtype=np.float64), (na,)))
            self.eps = _f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (na,)))
        self.nv, self.na, self.L, self.M, self.n_steps = int(n_vectors), na, int(L), int(M), int(n_steps)
        self._gauss = gaussians  # keep the device tensor alive during the call
        p = TsParamsC(int(seed) & 0xFFFFFFFFFFFFFFFF, int(first_vector), self.nv, _ptr(self.betas), na,
                      _ptr(self.E_b) if self.E_b is not None else None,
                      _ptr(self.eps) if self.eps is not None else None, self.L, self.M, self.n_steps,
                      float(taylor_lambda), _dptr(gaussians) if gaussians is not None else None,
                      int(block_steps), float(window_margin), float(resid_tol), int(bool(shell_moments)))
        hs = c_void_p()
        call("ftk_typical_states", h.handle, ctypes.byref(p), ctypes.byref(hs))
        self.handle = hs
        self._gauss = None

    def scalars(self):
        """(log_norm [nv, na], n_m [nv, na, L], E_m [na, L], eps [na])."""
        ln = np.zeros((self.nv, self.na))
        nm = np.zeros((self.nv, self.na, self.L))
        em = np.zeros((self.na, self.L))
        ep = np.zeros(self.na)
        call("ftk_states_scalars", self.handle, _ptr(ln), _ptr(nm), _ptr(em), _ptr(ep))
        return ln, nm, em, ep

    def moments(self):
        """(h1, h2) [nv, na, L]: <phi^m|H|phi^m> and ||H phi^m||^2 (built with shell_moments)."""
        h1 = np.zeros((self.nv, self.na, self.L))
        h2 = np.zeros((self.nv, self.na, self.L))
        call("ftk_states_moments", self.handle, _ptr(h1), _ptr(h2))
        return h1, h2

    def window(self):
        """(E_b [na], eps [na]) of the shell grid used."""
        E_b, eps = np.zeros(self.na), np.zeros(self.na)
        call("ftk_states_window", self.handle, _ptr(E_b), _ptr(eps))
        return E_b, eps

    def lanczos(self, s, a):
        al = np.zeros(self.n_steps)
        be = np.zeros(self.n_steps)
        k = ctypes.c_int()
        call("ftk_states_lanczos", self.handle, s, a, _ptr(al), _ptr(be), ctypes.byref(k))
        return al[: k.value], be[: k.value]

    def shell(self, s, a, m):
        import torch
        out = torch.empty(self.h.dim, dtype=torch.complex128, device=self.h.ctx.torch_device)
        call("ftk_states_copy_shell", self.handle, s, a, m, c_void_p(_dptr(out)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().ftk_states_destroy(self.handle)
            self.handle = None

    __del__ = close


class Spectrum:
    """Green's functions g_m^{alpha,Q}(omega) of every shell (Sec. III.C)."""

    def __init__(self, h, states, *, q_xy, omega, eta, n_steps, alpha_mask=7, rhs_block=0, resid_tol=0.0,
                 shells=None, solver="lanczos", seed_tol=0.0):
        """shells = (first, count) restricts the run to those shells of every (vector,
        anchor); the others stay zero in the outputs.  solver: "lanczos" (Lanczos-Galerkin)
        or "cocg" (shifted COCG with seed switching)."""
        self.h, self.states = h, states
        self.q = _f64(q_xy).reshape(-1, 2)
        self.omega = _f64(omega)
        self.alphas = [a for a in range(3) if alpha_mask & (1 << a)]
        self.n_steps = int(n_steps)
        first, count = shells if shells is not None else (0, 0)
        solvers = {"lanczos": 0, "cocg": 1}
        if solver not in solvers:
            raise ValueError(f"solver must be one of {sorted(solvers)}")
        self.solver = solver
        p = SpecParamsC(_ptr(self.q), len(self.q), int(alpha_mask), _ptr(self.omega), len(self.omega),
                        float(eta), self.n_steps, int(rhs_block), float(resid_tol), int(first), int(count),
                        solvers[solver], float(seed_tol))
        hs = c_void_p()
        call("ftk_shifted_krylov_spectrum", h.handle, states.handle, ctypes.byref(p), ctypes.byref(hs))
        self.handle = hs

    def raw(self):
        """(g [nv, na, L, n_alpha, n_q, n_omega] complex, max residual [nv, na, L, n_alpha, n_q])."""
        st = self.states
        shape = (st.nv, st.na, st.L, len(self.alphas), len(self.q))
        g = np.zeros(shape + (len(self.omega),), dtype=np.complex128)
        r = np.zeros(shape)
        call("ftk_spectrum_raw", self.handle, _ptr(g.view(np.float64)), _ptr(r))
        return g, r

    def norms(self):
        """||chi||^2 per sequence [nv, na, L, n_alpha, n_q] (static structure factor shell values)."""
        st = self.states
        out = np.zeros((st.nv, st.na, st.L, len(self.alphas), len(self.q)))
        call("ftk_spectrum_norms", self.handle, _ptr(out))
        return out

    def lanczos(self, s, a, m, ia, iq):
        al = np.zeros(self.n_steps)
        be = np.zeros(self.n_steps)
        k = ctypes.c_int()
        call("ftk_spectrum_lanczos", self.handle, s, a, m, ia, iq, _ptr(al), _ptr(be), ctypes.byref(k))
        return al[: k.value], be[: k.value]

    def cocg(self, s, a, m, ia, iq):
        """Shifted COCG runs: (a_k [n], b_{k+1} [n], c_k = <chi|q_k> [n+1], final seed index)."""
        av = np.zeros(self.n_steps, dtype=np.complex128)
        bv = np.zeros(self.n_steps, dtype=np.complex128)
        cv = np.zeros(self.n_steps + 1, dtype=np.complex128)
        k, seed = ctypes.c_int(), ctypes.c_int()
        call("ftk_spectrum_cocg", self.handle, s, a, m, ia, iq, _ptr(av.view(np.float64)), _ptr(bv.view(np.float64)),
             _ptr(cv.view(np.float64)), ctypes.byref(k), ctypes.byref(seed))
        return av[: k.value], bv[: k.value], cv[: k.value + 1], seed.value

    def work(self):
        """(Krylov steps summed over the sequences that ran, number of those sequences)."""
        k, n = ctypes.c_int64(), ctypes.c_int()
        call("ftk_spectrum_work", self.handle, ctypes.byref(k), ctypes.byref(n))
        return k.value, n.value

    def reweight(self, temps, n_bins=8):
        """Eqs. (FRW1)/(FRW2) on this spectrum and its states (alpha summed):
        S [n_q, n_T, n_omega], stderr, P [n_T, L]."""
        temps = _f64(temps)
        S = np.zeros((len(self.q), len(temps), len(self.omega)))
        err = np.zeros_like(S)
        P = np.zeros((len(temps), self.states.L))
        call("ftk_reweight_spectrum", self.states.handle, self.handle, _ptr(temps), len(temps), int(n_bins), _ptr(S),
             _ptr(err), _ptr(P))
        return S, err, P

    def close(self):
        if getattr(self, "handle", None):
            lib().ftk_spectrum_destroy(self.handle)
            self.handle = None

    __del__ = close


def momentum_operator(cluster, alpha, q):
    """Coefficients [N, 3] complex of S^alpha_{+Q} for PairSpectrum (e^{iQ.R_l}/sqrt(N) on
    component alpha)."""
    xy = _f64(cluster.site_xy)
    out = np.zeros((cluster.n_sites, 3), dtype=np.complex128)
    call("ftk_momentum_operator", cluster.n_sites, _ptr(xy), int(alpha), float(q[0]), float(q[1]),
         _ptr(out.view(np.float64)))
    return out


class GreenSequence:
    """One Green's-function sequence that can be stopped, saved and resumed
    (ftk_green_seq_*): chi a complex128 device tensor [2^N], shifts omega + shift_re +
    i eta, at most n_max steps."""

    def __init__(self, h, chi=None, omega=None, eta=None, shift_re=0.0, n_max=None, _handle=None):
        self.h = h
        if _handle is not None:
            self.handle = _handle
        else:
            import torch
            assert chi.dtype == torch.complex128 and chi.shape == (h.dim,)
            om = _f64(omega)
            out = c_void_p()
            call("ftk_green_seq_create", h.handle, c_void_p(_dptr(chi)), _ptr(om), len(om), float(eta),
                 float(shift_re), int(n_max), ctypes.byref(out))
            self.handle = out.value
        self._sizes()

    def _sizes(self):
        nw, nm, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        call("ftk_green_seq_info", self.handle, ctypes.byref(nw), ctypes.byref(nm), ctypes.byref(nb))
        self.n_omega, self.n_max, self.state_bytes = nw.value, nm.value, nb.value

    def advance(self, n_steps):
        """Runs up to n_steps more steps; returns the steps done in all."""
        k = ctypes.c_int()
        call("ftk_green_seq_advance", self.handle, int(n_steps), ctypes.byref(k))
        return k.value

    def read(self):
        """(g [n_omega] complex, alpha, beta, max_resid, done) after the steps done."""
        g = np.zeros(self.n_omega, dtype=np.complex128)
        al, be = np.zeros(self.n_max), np.zeros(self.n_max)
        k, r, d = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        call("ftk_green_seq_read", self.handle, _ptr(g.view(np.float64)), _ptr(al), _ptr(be), ctypes.byref(k),
             ctypes.byref(r), ctypes.byref(d))
        return g, al[: k.value], be[: k.value], r.value, bool(d.value)

    def save(self):
        """The sequence's state as bytes."""
        buf = ctypes.create_string_buffer(self.state_bytes)
        nb = ctypes.c_size_t()
        call("ftk_green_seq_save", self.handle, buf, self.state_bytes, ctypes.byref(nb))
        return buf.raw[: nb.value]

    @classmethod
    def restore(cls, h, state):
        """A new sequence on h resumed from save()'s bytes."""
        out = c_void_p()
        call("ftk_green_seq_restore", h.handle, state, len(state), ctypes.byref(out))
        return cls(h, _handle=out.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().ftk_green_seq_destroy(self.handle)
            self.handle = None

    __del__ = close


class PairSpectrum:
    """Green's functions of general operator pairs (Sec. III.B): G_AB and G_BA of every
    shell for linear spin operators A, B given by coefficients [n_pairs, N, 3] complex."""

    def __init__(self, h, states, *, op_a, op_b, omega, eta, n_steps, rhs_block=0, resid_tol=0.0,
                 solver="lanczos", seed_tol=0.0):
        """solver: "lanczos" (four polarization sequences per pair) or "cocg" (two shifted
        COCG runs per pair, one projected on each operator's vector)."""
        self.h, self.states = h, states
        self.op_a = np.ascontiguousarray(op_a, dtype=np.complex128).reshape(-1, h.n_sites, 3)
        self.op_b = np.ascontiguousarray(op_b, dtype=np.complex128).reshape(-1, h.n_sites, 3)
        if self.op_a.shape != self.op_b.shape:
            raise ValueError("op_a and op_b must have the same number of pairs")
        self.omega = _f64(omega)
        self.n_steps = int(n_steps)
        self.n_pairs = self.op_a.shape[0]
        solvers = {"lanczos": 0, "cocg": 1}
        if solver not in solvers:
            raise ValueError(f"solver must be one of {sorted(solvers)}")
        self.solver = solver
        p = PairParamsC(_ptr(self.op_a.view(np.float64)), _ptr(self.op_b.view(np.float64)), self.n_pairs,
                        _ptr(self.omega), len(self.omega), float(eta), self.n_steps, int(rhs_block),
                        float(resid_tol), solvers[solver], float(seed_tol))
        hs = c_void_p()
        call("ftk_pair_green", h.handle, states.handle, ctypes.byref(p), ctypes.byref(hs))
        self.handle = hs

    def raw(self):
        """(g_ab, g_ba [nv, na, L, n_pairs, n_omega] complex, overlap <A phi^m|B phi^m>
        [nv, na, L, n_pairs] complex, max residual [nv, na, L, n_pairs])."""
        st = self.states
        shape = (st.nv, st.na, st.L, self.n_pairs)
        gab = np.zeros(shape + (len(self.omega),), dtype=np.complex128)
        gba = np.zeros_like(gab)
        ov = np.zeros(shape, dtype=np.complex128)
        r = np.zeros(shape)
        call("ftk_pair_raw", self.handle, _ptr(gab.view(np.float64)), _ptr(gba.view(np.float64)),
             _ptr(ov.view(np.float64)), _ptr(r))
        return gab, gba, ov, r

    def cocg(self, s, a, m, p, k):
        """Shifted COCG pairs: run k (0 on rho = B phi, 1 on lam = A phi): (a_k, b_{k+1}, c_k, seed)."""
        av = np.zeros(self.n_steps, dtype=np.complex128)
        bv = np.zeros(self.n_steps, dtype=np.complex128)
        cv = np.zeros(self.n_steps + 1, dtype=np.complex128)
        n, seed = ctypes.c_int(), ctypes.c_int()
        call("ftk_pair_cocg", self.handle, s, a, m, p, k, _ptr(av.view(np.float64)), _ptr(bv.view(np.float64)),
             _ptr(cv.view(np.float64)), ctypes.byref(n), ctypes.byref(seed))
        return av[: n.value], bv[: n.value], cv[: n.value + 1], seed.value

    def lanczos(self, s, a, m, p, k):
        """(alpha, beta) of polarization sequence k (lam + rho, lam - rho, lam + i rho, lam - i rho)."""
        al = np.zeros(self.n_steps)
        be = np.zeros(self.n_steps)
        n = ctypes.c_int()
        call("ftk_pair_lanczos", self.handle, s, a, m, p, k, _ptr(al), _ptr(be), ctypes.byref(n))
        return al[: n.value], be[: n.value]

    def close(self):
        if getattr(self, "handle", None):
            lib().ftk_pair_destroy(self.handle)
            self.handle = None

    __del__ = close


def reweight_pair(betas, E_m, eps, log_norm, n_m, g_ab, g_ba, temps, n_bins=8):
    """Eq. FRW1 for operator pairs: complex S_AB [n_pairs, n_T, n_omega] and the binned
    errors of its real and imaginary parts (as one complex array)."""
    g_ab = np.ascontiguousarray(g_ab, dtype=np.complex128)
    g_ba = np.ascontiguousarray(g_ba, dtype=np.complex128)
    nv, na, L, npair, nw = g_ab.shape
    temps, betas, E_m, eps = _f64(temps), _f64(betas), _f64(E_m), _f64(eps)
    log_norm, n_m = _f64(log_norm), _f64(n_m)
    S = np.zeros((npair, len(temps), nw), dtype=np.complex128)
    err = np.zeros_like(S)
    call("ftk_reweight_pair", nv, na, L, npair, nw, _ptr(betas), _ptr(E_m), _ptr(eps), _ptr(log_norm), _ptr(n_m),
         _ptr(g_ab.view(np.float64)), _ptr(g_ba.view(np.float64)), _ptr(temps), len(temps), int(n_bins),
         _ptr(S.view(np.float64)), _ptr(err.view(np.float64)))
    return S, err


def reweight_observable(betas, E_m, log_norm, n_m, O, temps, n_bins=8):
    """Eq. FRW1 for real static observables O [nv, na, L, K]: (out [K, n_T], err [K, n_T])."""
    betas, E_m, log_norm, n_m, temps = _f64(betas), _f64(E_m), _f64(log_norm), _f64(n_m), _f64(temps)
    O = _f64(O)
    nv, na, L, K = O.shape
    out = np.zeros((K, len(temps)))
    err = np.zeros((K, len(temps)))
    call("ftk_reweight_observable", nv, na, L, K, _ptr(betas), _ptr(E_m), _ptr(log_norm), _ptr(n_m), _ptr(O),
         _ptr(temps), len(temps), int(n_bins), _ptr(out), _ptr(err))
    return out, err


def thermodynamics(betas, E_m, log_norm, n_m, h1, h2, n_sites, temps, n_bins=8):
    """(E, C, S, lnZ) [n_T] each and their binned errors (dict), from the shell data."""
    betas, E_m, log_norm, n_m, temps = _f64(betas), _f64(E_m), _f64(log_norm), _f64(n_m), _f64(temps)
    nv, na, L = n_m.shape
    h1 = None if h1 is None else _f64(h1)
    h2 = None if h2 is None else _f64(h2)
    out = np.zeros((len(temps), 4))
    err = np.zeros((len(temps), 4))
    call("ftk_thermodynamics", nv, na, L, _ptr(betas), _ptr(E_m), _ptr(log_norm), _ptr(n_m), _ptr(h1), _ptr(h2),
         int(n_sites), _ptr(temps), len(temps), int(n_bins), _ptr(out), _ptr(err))
    res = {k: out[:, j].copy() for j, k in enumerate(("E", "C", "S", "lnZ"))}
    res.update({k + "_err": err[:, j].copy() for j, k in enumerate(("E", "C", "S", "lnZ"))})
    return res


def thermo_diagnostics(betas, E_m, log_norm, n_m, h1, h2, n_sites, inv_temps, n_bins=8):
    """Energy variance and ln[Z(2b)/Z(b)^2] per inverse temperature b, with binned errors
    (dict var, log_typ, var_err, log_typ_err)."""
    betas, E_m, log_norm, n_m, bts = _f64(betas), _f64(E_m), _f64(log_norm), _f64(n_m), _f64(inv_temps)
    nv, na, L = n_m.shape
    h1 = None if h1 is None else _f64(h1)
    h2 = None if h2 is None else _f64(h2)
    out = np.zeros((len(bts), 2))
    err = np.zeros((len(bts), 2))
    call("ftk_thermo_diagnostics", nv, na, L, _ptr(betas), _ptr(E_m), _ptr(log_norm), _ptr(n_m), _ptr(h1),
         _ptr(h2), int(n_sites), _ptr(bts), len(bts), int(n_bins), _ptr(out), _ptr(err))
    return {"var": out[:, 0].copy(), "log_typ": out[:, 1].copy(), "var_err": err[:, 0].copy(),
            "log_typ_err": err[:, 1].copy()}


def choose_anchors(beta_grid, E, var, r_max=0.6, max_anchors=16):
    """Anchor ladder on an ascending inverse-temperature grid: indices of the anchors."""
    beta_grid, E, var = _f64(beta_grid), _f64(E), _f64(var)
    out = np.zeros(max(1, int(max_anchors)), dtype=np.int32)
    k = ctypes.c_int()
    call("ftk_choose_anchors", len(beta_grid), _ptr(beta_grid), _ptr(E), _ptr(var), float(r_max), int(max_anchors),
         _ptr(out), ctypes.byref(k))
    return [int(x) for x in out[: k.value]]


def reweight(betas, E_m, eps, log_norm, n_m, g, temps, n_bins=8):
    """Eqs. (FRW1)/(FRW2): S [n_q, n_T, n_omega], stderr (same shape), P [n_T, L].

    g: [nv, na, L, n_q, n_omega] complex, already summed over alpha."""
    g = np.ascontiguousarray(g, dtype=np.complex128)
    nv, na, L, nq, nw = g.shape
    temps, betas, E_m, eps = _f64(temps), _f64(betas), _f64(E_m), _f64(eps)
    log_norm, n_m = _f64(log_norm), _f64(n_m)
    assert betas.shape == (na,) and E_m.shape == (na, L) and eps.shape == (na,)
    assert log_norm.shape == (nv, na) and n_m.shape == (nv, na, L)
    S = np.zeros((nq, len(temps), nw))
    err = np.zeros_like(S)
    P = np.zeros((len(temps), L))
    call("ftk_reweight", nv, na, L, nq, nw, _ptr(betas), _ptr(E_m), _ptr(eps), _ptr(log_norm), _ptr(n_m),
         _ptr(g.view(np.float64)), _ptr(temps), len(temps), int(n_bins), _ptr(S), _ptr(err), _ptr(P))
    return S, err, P


# ---------------------------------------------------------------------------
class Request:
    """One S(Q, omega, T') request: the whole method for one Hamiltonian.

    E_b = eps = None takes the window from vector 0's Ritz extremes +- window_margin."""

    def __init__(self, cluster, K, J, *, seed, n_vectors, betas, L, M, n_filter, q_xy, omega, eta, n_green,
                 temps, E_b=None, eps=None, alpha_mask=7, rhs_block=0, first_vector=0, block_steps=0,
                 window_margin=0.0, taylor_lambda=0.0, filter_tol=0.0, green_tol=0.0):
        self.cluster, self.K, self.J = cluster, float(K), float(J)
        self.betas = _f64(betas)
        na = len(self.betas)
        if (E_b is None) != (eps is None):
            raise ValueError("give both E_b and eps, or neither")
        self.E_b = None if E_b is None else _f64(np.broadcast_to(np.asarray(E_b, dtype=np.float64), (na,)))
        self.eps = None if eps is None else _f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (na,)))
        self.q = _f64(q_xy).reshape(-1, 2)
        self.omega, self.temps = _f64(omega), _f64(temps)
        self.nv, self.L = int(n_vectors), int(L)
        self.ts = TsParamsC(int(seed) & 0xFFFFFFFFFFFFFFFF, int(first_vector), self.nv, _ptr(self.betas), na,
                            _ptr(self.E_b) if self.E_b is not None else None,
                            _ptr(self.eps) if self.eps is not None else None, self.L, int(M), int(n_filter),
                            float(taylor_lambda), None, int(block_steps), float(window_margin), float(filter_tol))
        self.sp = SpecParamsC(_ptr(self.q), len(self.q), int(alpha_mask), _ptr(self.omega), len(self.omega),
                              float(eta), int(n_green), int(rhs_block), float(green_tol))

    @property
    def shape(self):
        return (len(self.q), len(self.temps), len(self.omega))

    def footprint(self, device=0):
        """Device bytes the server reserves for this request."""
        b = ctypes.c_size_t()
        call("ftk_request_footprint", self.cluster.n_sites, ctypes.byref(self.ts), ctypes.byref(self.sp),
             int(device), ctypes.byref(b))
        return b.value


class Server:
    """Concurrent requests on one GPU with device-memory admission (ftk_server_*)."""

    def __init__(self, device=0, hbm_budget=0, n_workers=0):
        h = c_void_p()
        call("ftk_server_create", int(device), int(hbm_budget), int(n_workers), ctypes.byref(h))
        self.handle = h
        self._shapes = {}

    def submit(self, req):
        t = ctypes.c_uint64()
        c = req.cluster.as_c()
        call("ftk_server_submit", self.handle, ctypes.byref(c), req.K, req.J, ctypes.byref(req.ts),
             ctypes.byref(req.sp), _ptr(req.temps), len(req.temps), ctypes.byref(t))
        self._shapes[t.value] = req.shape
        return t.value

    def poll(self, ticket):
        """None while the request waits or runs; else (S, stderr, latency_s)."""
        shape = self._shapes[ticket]
        S, err, lat = np.zeros(shape), np.zeros(shape), ctypes.c_double()
        st = lib().ftk_server_poll(self.handle, ticket, _ptr(S), _ptr(err), ctypes.byref(lat))
        if st == -6:  # FTK_ENOTREADY
            return None
        del self._shapes[ticket]
        if st != 0:
            raise FTKError(st, lib().ftk_last_error().decode())
        return S, err, lat.value

    def wait(self, ticket, timeout=600.0):
        """Blocks until the request is done, then returns poll()'s result."""
        st = lib().ftk_server_wait(self.handle, ticket, float(timeout))
        if st not in (0, -6):
            raise FTKError(st, lib().ftk_last_error().decode())
        if st == -6:
            raise TimeoutError(f"request {ticket} not finished after {timeout} s")
        return self.poll(ticket)

    def cancel(self, ticket):
        """Cancels a waiting or running request; its poll/wait then raise FTK_ECANCELED."""
        call("ftk_server_cancel", self.handle, int(ticket))

    def stats(self):
        s = ServingStatsC()
        call("ftk_server_stats", self.handle, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in ServingStatsC._fields_}

    def occupancy(self):
        """(t [s], reserved bytes) at every request start and end."""
        n = ctypes.c_int()
        call("ftk_server_occupancy", self.handle, None, None, 0, ctypes.byref(n))
        t, b = np.zeros(n.value), np.zeros(n.value)
        call("ftk_server_occupancy", self.handle, _ptr(t), _ptr(b), n.value, ctypes.byref(n))
        return t, b

    def close(self):
        if getattr(self, "handle", None):
            lib().ftk_server_destroy(self.handle)
            self.handle = None

    __del__ = close
