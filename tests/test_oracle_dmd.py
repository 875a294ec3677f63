"""Pins of the oracle's parameter subsampling (Sec. 4.1, eq. pSampl), DMD of
the potential (Sec. 4.2.1, Alg. 1, eq. DMD_approx_potential_subset), radial
basis interpolation of the DMD coordinates, the DMD-DEIM gradient (eq. grHDD)
and the Alg. 2 step, each against something other than the oracle itself:
brute force, closed forms of exactly linear dynamics, a library routine, and
a finite difference of the hyper-reduced Hamiltonian."""

import numpy as np

from oracle import deim, dmd, pic, rom
from workloads import make_ensemble, workload


# --------------------------------------------------------------------------
# eq. pSampl
# --------------------------------------------------------------------------

def test_subset_greedy_brute_force():
    """Each pick maximises the distance to the nearest chosen column (over
    every candidate, written out), the first pick is the largest column."""
    rng = np.random.default_rng(3)
    Z = rng.normal(size=(4, 11))
    S = dmd.select_subset(Z, 6)
    assert S[0] == int(np.argmax([np.sqrt(sum(Z[r, i] ** 2 for r in range(4)))
                                  for i in range(11)]))
    for k in range(1, 6):
        best, arg = -1.0, None
        for i in range(11):
            if i in S[:k]:
                continue
            dmin = min(np.sqrt(sum((Z[r, i] - Z[r, j]) ** 2 for r in range(4))) for j in S[:k])
            if dmin > best:
                best, arg = dmin, i
        assert S[k] == arg
    assert len(set(S.tolist())) == 6


def test_subset_gauge_invariant():
    """Distances between reduced states do not depend on the orthonormal
    basis: any orthogonal change of the coefficients gives the same subset."""
    rng = np.random.default_rng(4)
    Z = rng.normal(size=(6, 20))
    Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    assert np.array_equal(dmd.select_subset(Z, 7), dmd.select_subset(Q @ Z, 7))


# --------------------------------------------------------------------------
# Alg. 1 and the prediction on exactly linear data
# --------------------------------------------------------------------------

def _linear_system(Nx=40, seed=5):
    """A = Q M Q^+ with M block-diagonal: a damped rotation (eigenvalues
    rho e^{+-i theta}) and three real positive eigenvalues."""
    rng = np.random.default_rng(seed)
    rho, th = 0.97, 0.3
    M = np.zeros((5, 5))
    M[:2, :2] = rho * np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    M[2, 2], M[3, 3], M[4, 4] = 1.02, 0.9, 0.5
    Q = rng.normal(size=(Nx, 5))
    Qp = np.linalg.pinv(Q)
    return Q, Qp, M, rho, th


def _M_power(M, rho, th, s):
    """M^s with the principal branch, written out block by block."""
    out = np.zeros_like(M)
    r = rho ** s
    out[:2, :2] = r * np.array([[np.cos(s * th), -np.sin(s * th)], [np.sin(s * th), np.cos(s * th)]])
    for k in (2, 3, 4):
        out[k, k] = M[k, k] ** s
    return out


def test_dmd_recovers_linear_dynamics():
    Q, Qp, M, rho, th = _linear_system()
    rng = np.random.default_rng(6)
    T, pst = 3, 3
    c0 = rng.normal(size=(5, pst))
    levels = [Q @ np.linalg.matrix_power(M, t) @ c0 for t in range(T + 1)]
    Y, Yp = dmd.window_matrices(levels)
    lam, Theta, r = dmd.dmd(Y, Yp, 1e-10)
    assert r == 5
    want = np.sort_complex(np.array([rho * np.exp(1j * th), rho * np.exp(-1j * th), 1.02, 0.9, 0.5]))
    assert np.allclose(np.sort_complex(lam), want, atol=1e-10)
    # the parameter-major layout: column t of parameter i is level t
    assert np.array_equal(Y[:, T * 1 + 2], levels[2][:, 1])
    assert np.array_equal(Yp[:, T * 2 + 0], levels[1][:, 2])
    eta = rng.uniform(size=(2, pst))
    op = dmd.build_operator(levels, np.arange(pst), eta, 0.05, 1e-10)
    last = levels[-1]
    for s in (0.0, 0.5, 1.0, 2.0):
        pred = dmd.predict(op, s * 0.05)
        ref = Q @ _M_power(M, rho, th, s) @ (Qp @ last)
        assert np.abs(pred - ref).max() < 1e-9 * np.abs(ref).max(), s


def test_dmd_truncation_is_relative():
    """Singular values below tol * sigma_1 are cut: data of rank 5 plus a
    1e-8 relative component keep 5 modes at tol 1e-5 and 6 at 1e-10."""
    Q, Qp, M, rho, th = _linear_system()
    rng = np.random.default_rng(7)
    c0 = rng.normal(size=(5, 3))
    levels = [Q @ np.linalg.matrix_power(M, t) @ c0 for t in range(4)]
    extra = rng.normal(size=(Q.shape[0], 1))
    levels = [L + 1e-8 * np.linalg.norm(L) * extra * (1 + t) for t, L in enumerate(levels)]
    Y, Yp = dmd.window_matrices(levels)
    assert dmd.dmd(Y, Yp, 1e-5)[2] == 5
    assert dmd.dmd(Y, Yp, 1e-12)[2] == 6


def test_untruncated_dmd_reproduces_the_last_potential():
    """With every mode kept, Theta spans the range of Y', which holds
    Phi_{tau-1}: the prediction at t_{tau-1} is the last level itself on the
    subset."""
    rng = np.random.default_rng(8)
    levels = [rng.normal(size=(32, 4)) for _ in range(4)]
    op = dmd.build_operator(levels, np.arange(4), rng.uniform(size=(3, 4)), 0.1, 1e-14)
    assert op.r == 12
    assert np.abs(dmd.predict(op, 0.0) - levels[-1]).max() < 1e-10


# --------------------------------------------------------------------------
# Gaussian radial basis interpolation
# --------------------------------------------------------------------------

def test_rbf_matches_scipy():
    from scipy.interpolate import RBFInterpolator
    rng = np.random.default_rng(9)
    xs = rng.uniform(size=(3, 10))
    vals = rng.normal(size=(4, 10))
    xq = rng.uniform(size=(3, 7))
    eps = dmd.rbf_width(xs)
    got = dmd.rbf_interpolate(xs, vals, xq, eps)
    ref = RBFInterpolator(xs.T, vals.T, kernel="gaussian", epsilon=1.0 / eps, degree=-1)(xq.T).T
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()
    assert np.abs(dmd.rbf_interpolate(xs, vals, xs, eps) - vals).max() < 1e-9


def test_rbf_width_and_scaling_by_hand():
    xs = np.array([[0.0, 1.0, 3.0]])
    assert dmd.rbf_width(xs) == 2.0          # pair distances 1, 3, 2
    eta = np.array([[1e-3, 1e-2, 5e-3], [2.0, 2.0, 2.0]])
    sc = dmd.scaled_parameters(eta)
    assert np.allclose(sc[0], [0.0, 1.0, 4.0 / 9.0]) and np.all(sc[1] == 0.0)


def test_interpolated_coordinates_at_subset_parameters():
    """Subset parameters keep Theta^+ Phi exactly; the others take the
    interpolant (complex coordinates: real and imaginary parts apart)."""
    rng = np.random.default_rng(10)
    p, S = 9, np.array([0, 4, 8, 2])
    levels = [rng.normal(size=(24, 4)) for _ in range(4)]
    eta = rng.uniform(size=(2, p))
    op = dmd.build_operator(levels, S, eta, 0.05, 1e-5)
    Pi_s = np.linalg.pinv(op.Theta) @ levels[-1]
    assert np.abs(op.Pi[:, S] - Pi_s).max() < 1e-12 * np.abs(Pi_s).max()
    xs_all = dmd.scaled_parameters(eta)
    eps = dmd.rbf_width(xs_all[:, S])
    from scipy.interpolate import RBFInterpolator
    rest = np.array([1, 3, 5, 6, 7])
    f = RBFInterpolator(xs_all[:, S].T, np.concatenate([Pi_s.real, Pi_s.imag]).T,
                        kernel="gaussian", epsilon=1.0 / eps, degree=-1)
    ref = f(xs_all[:, rest].T).T
    r = op.r
    assert np.abs(op.Pi[:, rest] - (ref[:r] + 1j * ref[r:])).max() < 1e-9 * np.abs(ref).max()


# --------------------------------------------------------------------------
# eq. grHDD: the gradient of the DMD-DEIM Hamiltonian
# --------------------------------------------------------------------------

def test_dmd_deim_gradient_is_the_hamiltonian_gradient():
    """g^DD_i = grad_{Z_i} of H_i = 1/2 |V_r|^2 + (q/m) w^T P^T Lambda^0(X_r) Phi
    for a fixed potential Phi (reading: the electric term without the 1/2 of
    eq. Hdd, whose gradient is the printed eq. grHDD), by central finite
    differences through the brute-force Lambda^0."""
    rng = np.random.default_rng(11)
    N, p, Nx, two_n, Lx = 60, 2, 16, 6, 4 * np.pi
    X0 = rng.uniform(0, Lx, size=(N, p))
    V0 = rng.normal(size=(N, p))
    U, Z = rom.init_csvd(X0, V0, two_n)
    Y = rng.normal(size=(N, 12))
    Psi, _ = deim.deim_basis(Y, 8)
    idx = deim.greedy_indices(Psi)
    op = deim.DeimOp(idx=idx, w=deim.weights(Psi, idx), Psi=Psi)
    xs = np.arange(Nx) * Lx / Nx
    Phi = np.stack([np.cos(2 * np.pi * xs / Lx) + 0.3 * np.sin(6 * np.pi * xs / Lx),
                    0.5 * np.sin(4 * np.pi * xs / Lx)], axis=1)
    L = np.full(p, Lx)
    e = pic.field(Phi, L)
    cfg = rom.RomConfig(N=N, p=p, Nx=Nx, two_n=two_n)
    g = rom.dmd_deim_gradient(U, Z, e, L, op, cfg)

    def H(z, i):
        x = U[:N] @ z
        v = U[N:] @ z
        lam = pic.lambda0_dense(x[idx], Lx, Nx)
        return 0.5 * v @ v + (cfg.q / cfg.m) * op.w @ (lam @ Phi[:, i])

    h = 1e-6
    for i in range(p):
        j, th = pic.cell_index((U[:N] @ Z[:, i])[idx][:, None], L[:1], Nx)
        assert np.min(np.minimum(th, 1 - th)) > 1e-3   # no node within the step
        fd = np.array([(H(Z[:, i] + h * ek, i) - H(Z[:, i] - h * ek, i)) / (2 * h)
                       for ek in np.eye(two_n)])
        assert np.abs(fd - g[:, i]).max() < 1e-6 * max(1.0, np.abs(g[:, i]).max())


# --------------------------------------------------------------------------
# Alg. 2
# --------------------------------------------------------------------------

def _twostream(N=3000, p=12, Nx=32):
    w = workload("twostream_deim", N=N, p=p, Nx=Nx)
    e = make_ensemble(w)
    return w, e


def test_alg2_first_T_steps_are_the_plain_reduced_model():
    w, e = _twostream()
    T = 3
    cfg_d = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=8, dt=w["dt"], fp_tol=1e-10,
                          projection="dmd_deim", deim_window=T, p_star=4, deim_rows=16)
    cfg_g = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=8, dt=w["dt"], fp_tol=1e-10)
    sd = rom.init_state(e["X0"], e["V0"], e["L"], cfg_d, eta=e["eta"])
    sg = rom.init_state(e["X0"], e["V0"], e["L"], cfg_g)
    for _ in range(T):
        assert rom.prk_step(sd, cfg_d) == rom.OK
        assert rom.prk_step(sg, cfg_g) == rom.OK
        assert sd.deim_indices is None
    assert np.array_equal(sd.U, sg.U) and np.array_equal(sd.Z, sg.Z)
    assert len(sd.phi_window) == T and len(sd.window) == T
    assert rom.prk_step(sd, cfg_d) == rom.OK
    assert sd.deim_indices is not None and sd.last_dmd_rank > 0
    assert len(sd.phi_window) == T + 1


def test_alg2_enoconv_restores_both_windows():
    w, e = _twostream()
    T = 2
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=8, dt=w["dt"], fp_tol=1e-10,
                        projection="dmd_deim", deim_window=T, p_star=4, deim_rows=12)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg, eta=e["eta"])
    for _ in range(T + 1):
        assert rom.prk_step(st, cfg) == rom.OK
    U, Z = st.U.copy(), st.Z.copy()
    win = [a.copy() for a in st.window]
    phw = [a.copy() for a in st.phi_window]
    idx, builds = st.deim_indices.copy(), st.deim_builds
    bad = rom.RomConfig(**cfg.__dict__)
    bad.fp_max_iters, bad.fp_stall_tol = 1, 0.0
    assert rom.prk_step(st, bad) == rom.ENOCONV
    assert np.array_equal(st.U, U) and np.array_equal(st.Z, Z)
    assert all(np.array_equal(a, b) for a, b in zip(st.window, win))
    assert all(np.array_equal(a, b) for a, b in zip(st.phi_window, phw))
    assert np.array_equal(st.deim_indices, idx) and st.deim_builds == builds
    assert rom.prk_step(st, cfg) == rom.OK


def test_alg2_stays_close_to_the_reduced_model():
    """Sanity of the hyper-reduction (accuracy against the paper is parity
    unpinned: no printed values): over a few DMD-DEIM steps the state stays
    within a few percent of the Galerkin reduced model's."""
    w, e = _twostream(N=6000, p=16, Nx=32)
    T = 3
    cfg_d = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=8, dt=w["dt"], fp_tol=1e-10,
                          projection="dmd_deim", deim_window=T, p_star=6, deim_rows=24)
    cfg_g = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=8, dt=w["dt"], fp_tol=1e-10)
    sd = rom.init_state(e["X0"], e["V0"], e["L"], cfg_d, eta=e["eta"])
    sg = rom.init_state(e["X0"], e["V0"], e["L"], cfg_g)
    for _ in range(T + 4):
        assert rom.prk_step(sd, cfg_d) == rom.OK
        assert rom.prk_step(sg, cfg_g) == rom.OK
    Xd, Vd = rom.reconstruct(sd)
    Xg, Vg = rom.reconstruct(sg)
    ex = np.linalg.norm(Xd - Xg) / np.linalg.norm(Xg)
    ev = np.linalg.norm(Vd - Vg) / np.linalg.norm(Vg)
    print(f"DMD-DEIM vs Galerkin after {T + 4} steps: X {ex:.2e}, V {ev:.2e}")
    assert ex < 1e-2 and ev < 5e-2
