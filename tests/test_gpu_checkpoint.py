"""Checkpoint and resume of one Green's-function sequence (ftk_green_seq_*).

The sequence is run straight, and again in chunks with its state saved to host bytes
and restored into a new sequence between them (at 0, 1, 2 and 21 steps, the boundaries
where the start vector still stands in for w_{-1} and where it no longer does): the
Lanczos coefficients and g must be bit for bit the straight run's, on the single-pass
form of H v (16 sites), the two-pass (18 sites) and the three-pass benchmark form
(24 sites) on the layout planner's labels.  At 16 and 18 sites the straight run also
matches the oracle (coefficients bit for bit, g within 1e-8).  Invalid states are
refused with FTK_EINVAL, a breakdown ends the sequence for good, and a NaN start
vector is FTK_ENUMERIC.
"""
import numpy as np
import pytest

from seeded_inputs import SUPERCELLS, omega_grid, real_vector

pytestmark = pytest.mark.gpu

N_MAX = 60
ETA, SHIFT = 0.05, 0.3


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1802_02854_amd as ftk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ftk, torch, ftk.Context(0)


def _system(ftk, ctx, N, relabel):
    from oracle import cluster, hamiltonian
    if relabel:
        rc, P, perm, order = ftk.plan_layout(ftk.honeycomb_cluster(*SUPERCELLS[N]))
        ocl = cluster.relabel(cluster.honeycomb(*SUPERCELLS[N]), perm, order)
    else:
        rc, ocl = ftk.honeycomb_cluster(*SUPERCELLS[N]), cluster.honeycomb(*SUPERCELLS[N])
    return ftk.Hamiltonian(ctx, rc, -1.0, 0.1), hamiltonian.Hamiltonian(ocl, -1.0, 0.1)


def _dev(torch, v):
    return torch.from_numpy(np.ascontiguousarray(v).view(np.complex128)).to("cuda")


@pytest.mark.parametrize("N,relabel", [(16, False), (18, True), (24, True)])
def test_resume_is_bitwise(env, N, relabel):
    ftk, torch, ctx = env
    print(f"checkpoint N={N}", flush=True)
    h, oh = _system(ftk, ctx, N, relabel)
    chi = real_vector(500 + N, 2 << N)
    omega = omega_grid(-3.0, 3.0, 200)
    straight = ftk.GreenSequence(h, _dev(torch, chi), omega, ETA, SHIFT, N_MAX)
    assert straight.advance(N_MAX) == N_MAX
    g0, al0, be0, r0, done0 = straight.read()
    assert len(al0) == N_MAX and done0
    straight.close()

    q = ftk.GreenSequence(h, _dev(torch, chi), omega, ETA, SHIFT, N_MAX)
    for stop in (0, 1, 2, 21):
        assert q.advance(stop - len(q.read()[1])) == stop
        state = q.save()
        assert len(state) == q.state_bytes
        q.close()
        q = ftk.GreenSequence.restore(h, state)
        g, al, be, _, done = q.read()
        assert len(al) == stop and not done
        assert np.array_equal(al, al0[:stop]) and np.array_equal(be, be0[:stop])
    assert q.advance(10 * N_MAX) == N_MAX  # capped at n_max
    g, al, be, r, done = q.read()
    q.close()
    assert done and np.array_equal(al, al0) and np.array_equal(be, be0)
    assert np.array_equal(g, g0) and r == r0

    if N <= 18:
        from oracle import green
        go, ro, alo, beo = green.green_sequence(oh, chi, N_MAX, omega, ETA, SHIFT)
        assert np.array_equal(al0, alo) and np.array_equal(be0, beo)
        assert np.abs(g0 - go).max() <= 1e-8 * np.abs(go).max()


def test_invalid_states_are_refused(env):
    ftk, torch, ctx = env
    from paper_1802_02854_amd import FTKError
    print("checkpoint invalid states", flush=True)
    N = 12
    h, _ = _system(ftk, ctx, N, False)
    other = ftk.Hamiltonian(ctx, ftk.honeycomb_cluster(*SUPERCELLS[N]), -1.0, 0.2)
    chi = real_vector(77, 2 << N)
    q = ftk.GreenSequence(h, _dev(torch, chi), omega_grid(-2, 2, 16), ETA, SHIFT, 20)
    q.advance(5)
    state = q.save()
    q.close()
    bad = {
        "another Hamiltonian": (other, state),
        "truncated": (h, state[:-8]),
        "bad magic": (h, b"X" + state[1:]),
        "payload byte flipped": (h, state[:200] + bytes([state[200] ^ 1]) + state[201:]),
    }
    for name, (hh, st) in bad.items():
        with pytest.raises(FTKError) as e:
            ftk.GreenSequence.restore(hh, st)
        assert e.value.status == -1, name
    r = ftk.GreenSequence.restore(h, state)  # the intact state still loads
    assert len(r.read()[1]) == 5
    r.close()
    nan = chi.copy()
    nan[3] = np.nan
    with pytest.raises(FTKError) as e:
        ftk.GreenSequence(h, _dev(torch, nan), omega_grid(-2, 2, 16), ETA, SHIFT, 20)
    assert e.value.status == -4


def test_breakdown_ends_the_sequence(env):
    """A fully polarised basis state is an eigenvector of the Heisenberg model (K = 0,
    J = 1, E = J/4 per bond): beta_1 = 0 ends the sequence after one step, before and
    after a restore, with g the one-pole resolvent 1/(z - E)."""
    ftk, torch, ctx = env
    print("checkpoint breakdown", flush=True)
    N = 8
    cl = ftk.honeycomb_cluster(*SUPERCELLS[N])
    h = ftk.Hamiltonian(ctx, cl, 0.0, 1.0)
    chi = np.zeros(2 << N)
    chi[0] = 1.0  # basis state 0: every S^z equal
    omega = omega_grid(-3.0, 3.0, 31)
    q = ftk.GreenSequence(h, _dev(torch, chi), omega, ETA, 0.0, 20)
    assert q.advance(20) == 1
    g, al, be, r, done = q.read()
    assert done and be[0] == 0.0
    E = 0.25 * cl.n_bonds
    assert al[0] == E
    z = omega + 1j * ETA
    assert np.abs(g - 1.0 / (z - E)).max() <= 1e-14 * np.abs(1.0 / (z - E)).max()
    r2 = ftk.GreenSequence.restore(h, q.save())
    assert r2.advance(5) == 1
    assert np.array_equal(r2.read()[0], g)
    q.close()
    r2.close()
