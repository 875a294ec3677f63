"""Pins of the DEIM oracle: interpolation property, exactness on the DEIM
space, the Chaturantabut-Sorensen error bound, and reduction to the
Galerkin gradient when every particle is an interpolation point."""
import numpy as np

from oracle import deim, rom
from workloads import make_ensemble, workload


def test_interpolation_property_and_exactness():
    rng = np.random.default_rng(0)
    N, d = 50, 6
    Psi, _ = np.linalg.qr(rng.normal(size=(N, d)))
    idx = deim.greedy_indices(Psi)
    assert len(set(idx.tolist())) == d
    P = np.eye(N)[:, idx]
    proj = Psi @ np.linalg.solve(P.T @ Psi, P.T)
    f = rng.normal(size=N)
    # the DEIM approximation interpolates f on the selected indices
    np.testing.assert_allclose((proj @ f)[idx], f[idx], atol=1e-12)
    # and is exact on span(Psi)
    c = rng.normal(size=d)
    np.testing.assert_allclose(proj @ (Psi @ c), Psi @ c, atol=1e-12)
    # error bound ||f - Df|| <= ||(P^T Psi)^{-1}|| ||(I - Psi Psi^T) f||
    bound = np.linalg.norm(np.linalg.inv(P.T @ Psi), 2) * np.linalg.norm(f - Psi @ (Psi.T @ f))
    assert np.linalg.norm(f - proj @ f) <= bound * (1 + 1e-12)


def test_greedy_first_index_and_ties():
    """The first index is the largest entry of psi_1; ties go to the
    smallest index."""
    Psi = np.array([[0.5, 0.1], [-0.5, 0.7], [0.5, 0.1], [0.5, -0.7]])
    Psi[:, 1] -= Psi[:, 0] * (Psi[:, 0] @ Psi[:, 1])
    idx = deim.greedy_indices(Psi)
    assert idx[0] == 0
    assert idx[1] != 0


def test_full_deim_reduces_to_galerkin():
    """d = N: P is a permutation, w = 1 and the DEIM gradient is the Galerkin
    gradient exactly (eq. grHDD against eq. grads)."""
    N = 40
    w = workload("twostream_deim", N=N, p=12, Nx=16)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=12, Nx=16, two_n=6, dt=0.05)
    st = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    gr = rom.gradient(st.U, st.Z, st.L, 16)
    rng = np.random.default_rng(1)
    Y = rng.normal(size=(N, 3 * N))
    op = deim.build_operator(Y, N)
    assert sorted(op.idx.tolist()) == list(range(N))
    np.testing.assert_allclose(op.w, np.ones(N), atol=1e-10)
    g = deim.deim_gradient(st.U, st.Z, gr, op, cfg)
    np.testing.assert_allclose(g, gr.g, atol=1e-10 * np.abs(gr.g).max())


def test_snapshot_is_potential_at_particles():
    """Lambda^0(X) Phi interpolates the nodal potential linearly."""
    from oracle import pic
    L = np.array([8.0])
    Phi = np.arange(8.0)[:, None] ** 2
    X = np.array([[0.0], [0.5], [3.25], [7.5], [8.5]])
    y = deim.snapshot(X, Phi, L)
    np.testing.assert_allclose(y[:, 0], [0.0, 0.5, 9 + 0.25 * 7, 49 + 0.5 * (0 - 49), 0.5])
    # against the brute-force dense Lambda^0
    Lam = pic.lambda0_dense(X[:, 0], 8.0, 8)
    np.testing.assert_allclose(y[:, 0], Lam @ Phi[:, 0], atol=1e-14)


def test_deim_rom_runs_and_switches_after_window():
    N = 600
    w = workload("twostream_deim", N=N, p=16, Nx=32)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=16, Nx=32, two_n=6, dt=0.05, projection="deim",
                        deim_window=3, fp_tol=1e-11)
    st = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    for s in range(6):
        assert rom.prk_step(st, cfg) == rom.OK
        if s < 3:
            assert st.deim_indices is None
        else:
            assert st.deim_indices is not None and len(st.deim_indices) == 6


def test_snapshot_parameter_subset():
    """p* (T+1) covers the largest DEIM dimension d = two_n_max; the subset is
    evenly spaced and starts at the first parameter."""
    for p, cap, T in ((64, 60, 3), (16, 10, 3), (4, 10, 3), (300, 8, 5)):
        sub = deim.snapshot_params(p, cap, T)
        assert sub[0] == 0 and len(set(sub.tolist())) == len(sub)
        assert len(sub) == min(p, max(8, -(-cap // (T + 1))))
        assert np.all(np.diff(sub) > 0) and sub[-1] < p
