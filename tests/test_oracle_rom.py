"""Pins of the reduced-model oracle: identities, special cases that reduce to
the full model, closed forms and invariants (none of them re-types the
oracle's own formula)."""
import math

import numpy as np
import pytest

from oracle import pic, rom
from workloads import make_ensemble, workload


def _rand_basis(rng, N, n):
    Q, _ = np.linalg.qr(rng.normal(size=(N, n)) + 1j * rng.normal(size=(N, n)))
    return rom.from_complex_basis(Q)


def _J(N):
    return np.block([[np.zeros((N, N)), np.eye(N)], [-np.eye(N), np.zeros((N, N))]])


def _orth_err(U):
    N = U.shape[0] // 2
    r = U.shape[1]
    return max(np.abs(U.T @ U - np.eye(r)).max(),
               np.abs(U.T @ _J(N) @ U - rom.J_small(r)).max())


def test_complex_structure_is_orthosymplectic():
    """U = [[A,-B],[B,A]] with A + iB unitary columns satisfies U^T U = I and
    U^T J U = J (Sec. 3.2, definition of the orthosymplectic manifold)."""
    rng = np.random.default_rng(0)
    U = _rand_basis(rng, 15, 3)
    assert _orth_err(U) < 1e-14
    # and J U = U J holds for every such U
    assert np.abs(_J(15) @ U - U @ rom.J_small(6)).max() < 1e-15


def test_S_commutes_with_J_and_is_real_form_of_ZZstar():
    rng = np.random.default_rng(1)
    Z = rng.normal(size=(6, 9))
    S = rom.S_of(Z)
    J = rom.J_small(6)
    assert np.abs(S @ J - J @ S).max() < 1e-13
    Zt = rom.to_complex_coeff(Z)
    H = Zt @ Zt.conj().T
    ref = np.block([[H.real, -H.imag], [H.imag, H.real]])
    np.testing.assert_allclose(S, ref, atol=1e-13)


def test_basis_velocity_complex_form_and_tangency():
    """Real form (eq. UZred_basis) equals the complex form
    -i (I - U~U~*) G~ Z~* (Z~Z~*)^{-1}; U^T X = 0 (horizontal)."""
    rng = np.random.default_rng(2)
    N, n, p = 20, 3, 8
    U = _rand_basis(rng, N, n)
    Z = rng.normal(size=(2 * n, p))
    G = rng.normal(size=(2 * N, p))
    X = rom.basis_velocity(U, Z, G)
    Ut = rom.to_complex_basis(U)
    Gt = G[:N] + 1j * G[N:]
    Zt = rom.to_complex_coeff(Z)
    Xc = -1j * (Gt - Ut @ (Ut.conj().T @ Gt)) @ Zt.conj().T @ np.linalg.inv(Zt @ Zt.conj().T)
    np.testing.assert_allclose(X, rom.from_complex_basis(Xc), atol=1e-13)
    assert np.abs(U.T @ X).max() < 1e-13


def test_pseudo_inverse_when_p_less_than_n():
    """With p < n the full-rank condition fails; the Moore-Penrose inverse
    then matches numpy's pinv of S."""
    rng = np.random.default_rng(3)
    Z = rng.normal(size=(10, 4))
    S = rom.S_of(Z)
    np.testing.assert_allclose(rom.pinv_sym(S, 1e-12), np.linalg.pinv(S, rcond=1e-12, hermitian=True),
                               atol=1e-10)


def test_cayley_woodbury_equals_dense_and_stays_orthosymplectic():
    rng = np.random.default_rng(4)
    N, n = 14, 3
    U0 = _rand_basis(rng, N, n)
    xi = rom.from_complex_basis(0.3 * (rng.normal(size=(N, n)) + 1j * rng.normal(size=(N, n))))
    np.testing.assert_allclose(rom.cayley(U0, xi), rom.cayley_dense(U0, xi), atol=1e-14)
    assert _orth_err(rom.cayley(U0, xi)) < 1e-13
    # R_{U0}(0) = U0
    assert np.abs(rom.cayley(U0, 0 * xi) - U0).max() == 0.0


def test_tangent_velocity_identities():
    """Y(0, Z) = X(U0, Z), and d/de R_{U0}(xi + e Y) at e = 0 equals
    X(R_{U0}(xi), Z): Y is the pull-back of the basis velocity through the
    retraction (pins the transcription of the printed formula and the 1/2
    scaling of the Cayley transform)."""
    rng = np.random.default_rng(5)
    N, n, p = 16, 2, 6
    U0 = _rand_basis(rng, N, n)
    Z = rng.normal(size=(2 * n, p))
    G = rng.normal(size=(2 * N, p))
    xi = rom.from_complex_basis(0.2 * (rng.normal(size=(N, n)) + 1j * rng.normal(size=(N, n))))
    np.testing.assert_allclose(rom.tangent_velocity(U0, 0 * xi, Z, G), rom.basis_velocity(U0, Z, G),
                               atol=1e-14)
    Y = rom.tangent_velocity(U0, xi, Z, G)
    eps = 1e-6
    fd = (rom.cayley(U0, xi + eps * Y) - rom.cayley(U0, xi - eps * Y)) / (2 * eps)
    target = rom.basis_velocity(rom.cayley(U0, xi), Z, G)
    assert np.abs(fd - target).max() < 1e-8 * max(1.0, np.abs(target).max())
    # an unscaled Cayley transform would miss by O(1): the identity is sharp
    def cay1(U0, xi):
        W = xi - 0.5 * U0 @ (U0.T @ xi)
        Om = W @ U0.T - U0 @ W.T
        I = np.eye(Om.shape[0])
        return np.linalg.solve(I - Om, (I + Om) @ U0)
    fd1 = (cay1(U0, xi + eps * Y) - cay1(U0, xi - eps * Y)) / (2 * eps)
    assert np.abs(fd1 - rom.basis_velocity(cay1(U0, xi), Z, G)).max() > 1e-3


def test_init_csvd_eckart_young():
    """||R0 - U0 Z0||_F^2 = sum of the squared tail singular values of X0 + iV0."""
    w = workload("landau_tiny", N=3000, p=6)
    ens = make_ensemble(w)
    X0, V0 = ens["X0"], ens["V0"]
    s = np.linalg.svd(X0 + 1j * V0, compute_uv=False)
    for two_n in (2, 4, 8):
        U, Z = rom.init_csvd(X0, V0, two_n)
        R = U @ Z
        err2 = np.linalg.norm(R[:3000] - X0) ** 2 + np.linalg.norm(R[3000:] - V0) ** 2
        np.testing.assert_allclose(err2, np.sum(s[two_n // 2:] ** 2), rtol=1e-10,
                                   atol=1e-20 + 1e-24 * np.sum(s ** 2))
        assert _orth_err(U) < 1e-13


def test_init_completion_when_n_exceeds_p():
    w = workload("landau_tiny", N=500)          # p = 4 < n = 5
    ens = make_ensemble(w)
    U, Z = rom.init_csvd(ens["X0"], ens["V0"], 10)
    assert U.shape == (1000, 10)
    assert _orth_err(U) < 1e-13
    R = U @ Z
    assert np.abs(R[:500] - ens["X0"]).max() < 1e-11
    assert np.abs(R[500:] - ens["V0"]).max() < 1e-11


def _cold_case(N=600, p=2, Nx=16, seed=11):
    """Particles inside cells away from nodes, nearly at rest (no node
    crossing over the horizons used, so the dynamics is smooth)."""
    rng = np.random.default_rng(seed)
    L = np.array([4 * np.pi, 3 * np.pi])[:p]
    h = L / Nx
    c = rng.integers(0, Nx, size=(N, p))
    X = h[None, :] * (c + 0.3 + 0.4 * rng.random((N, p)))
    V = 0.01 * rng.normal(size=(N, p))
    return X, V, L, Nx


def test_full_rank_reduced_model_is_implicit_midpoint_on_full_model():
    """2n = 2N and U0 = I: (I - U U^T) = 0 so the basis never moves and the
    partitioned scheme is the implicit midpoint rule on the full model."""
    rng = np.random.default_rng(6)
    N, p, Nx = 30, 2, 8
    L = np.array([6.0, 7.5])
    X = rng.uniform(0, 1, size=(N, p)) * L[None, :]
    V = rng.normal(size=(N, p))
    cfg = rom.RomConfig(N=N, p=p, Nx=Nx, two_n=2 * N, dt=0.05, fp_tol=1e-14, fp_max_iters=400)
    st = rom.RomState(U=np.eye(2 * N), Z=np.concatenate([X, V], axis=0), L=L)
    for _ in range(3):
        assert rom.prk_step(st, cfg) == rom.OK
        X, V = pic.fom_implicit_midpoint_step(X, V, L, Nx, 0.05, tol=1e-14, max_iters=400)
    R = st.U @ st.Z
    np.testing.assert_allclose(R[:N], X, atol=1e-12)
    np.testing.assert_allclose(R[N:], V, atol=1e-12)
    assert np.abs(st.U - np.eye(2 * N)).max() < 1e-14


def test_low_rank_exact_manifold_converges_at_order_two():
    """p <= n: the reduced manifold contains the full solution (Z~ has full
    column rank, so the tangent space is all of C^{N x p}); the reduced
    scheme then converges to the full trajectory at order 2 in dt."""
    X, V, L, Nx = _cold_case()
    N = X.shape[0]
    T = 0.4
    j0, _ = pic.cell_index(X, L, Nx)
    Xr, Vr = pic.fom_run(X, V, L, Nx, T / 128, 128)
    assert np.array_equal(pic.cell_index(Xr, L, Nx)[0], j0)
    errs = []
    for nsteps in (4, 8):
        cfg = rom.RomConfig(N=N, p=2, Nx=Nx, two_n=6, dt=T / nsteps, fp_tol=1e-13)
        st = rom.init_state(X, V, L, cfg)
        for _ in range(nsteps):
            assert rom.prk_step(st, cfg) == rom.OK
        R = st.U @ st.Z
        errs.append(np.linalg.norm(R[:N] - Xr) + np.linalg.norm(R[N:] - Vr))
    order = math.log2(errs[0] / errs[1])
    assert 1.8 <= order <= 2.2, (order, errs)


def _tiny_landau(steps=0, two_n=10, N=2000):
    w = workload("landau_tiny", N=N)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=w["p"], Nx=w["Nx"], two_n=two_n, dt=w["dt"], fp_tol=1e-12)
    st = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    for _ in range(steps):
        assert rom.prk_step(st, cfg) == rom.OK
    return st, cfg, ens


def test_orthosymplectic_after_steps():
    st, cfg, _ = _tiny_landau()
    for _ in range(5):
        assert rom.prk_step(st, cfg) == rom.OK
        assert _orth_err(st.U) < 1e-12


def test_gauge_covariance():
    """(U Q, Q^T Z) with Q orthosymplectic gives the same R trajectory."""
    rng = np.random.default_rng(8)
    N = 800
    w = workload("twostream_deim", N=N, p=8, Nx=32)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=8, Nx=32, two_n=6, dt=0.05, fp_tol=1e-13)
    st1 = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    Qc, _ = np.linalg.qr(rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
    Q = rom.from_complex_basis(Qc)
    st2 = rom.RomState(U=st1.U @ Q, Z=Q.T @ st1.Z, L=ens["L"])
    for _ in range(3):
        assert rom.prk_step(st1, cfg) == rom.OK
        assert rom.prk_step(st2, cfg) == rom.OK
    R1, R2 = st1.U @ st1.Z, st2.U @ st2.Z
    assert np.abs(R1 - R2).max() < 1e-10 * np.abs(R1).max()


def test_reorthonormalisation_keeps_R():
    rng = np.random.default_rng(9)
    N, n, p = 40, 3, 5
    U = _rand_basis(rng, N, n)
    U = U + 1e-6 * rom.from_complex_basis(rng.normal(size=(N, n)) + 1j * rng.normal(size=(N, n)))
    Z = rng.normal(size=(2 * n, p))
    U2, Z2 = rom.reorthonormalise(U, Z)
    assert _orth_err(U2) < 1e-14
    np.testing.assert_allclose(U2 @ Z2, U @ Z, atol=1e-13)


def test_rank_growth_keeps_R_bitwise_and_shrink_error():
    st, cfg, _ = _tiny_landau(steps=1, two_n=4, N=1500)
    cfg.two_n_max = 12
    R0 = st.U @ st.Z
    rom.adapt_rank(st, cfg, 8)
    assert st.U.shape[1] == 8 and _orth_err(st.U) < 1e-11
    R1 = st.U @ st.Z
    assert np.array_equal(R1, R0)
    # after a step the new coefficient rows are populated; shrinking removes
    # exactly the energy of the dropped singular values of Z~ (Eckart-Young)
    cfg.two_n = 8
    assert rom.prk_step(st, cfg) == rom.OK
    R1 = st.U @ st.Z
    s = np.linalg.svd(rom.to_complex_coeff(st.Z), compute_uv=False)
    assert s[3] > 1e-6 * s[0]
    dropped = rom.rank_shrink(st, 6)
    R2 = st.U @ st.Z
    np.testing.assert_allclose(np.linalg.norm(R2 - R1), math.sqrt(np.sum(s[3:] ** 2)),
                               rtol=1e-8)
    np.testing.assert_allclose(dropped, s[3:], rtol=1e-10)
    assert _orth_err(st.U) < 1e-12
    assert rom.adapt_rank(st, cfg, 14)[0] == rom.ERANKCAP
    # the automatic policy grows one pair when the indicator exceeds its threshold
    cfg.rank_tol_up = 0.0
    st2, cfg2, _ = _tiny_landau(two_n=4, N=800)
    cfg2.two_n_max, cfg2.rank_tol_up = 8, 0.0
    status, r2, eps = rom.adapt_rank(st2, cfg2, 0)
    assert status == rom.OK and r2 == 6 and eps > 0


def test_rank_indicator_identity():
    """||(I - U U^T) J G||_F^2 = ||G||^2 - ||g||^2 (uses U^T J = J U^T)."""
    st, cfg, _ = _tiny_landau(two_n=4, N=600)
    eps, gr = rom.rank_indicator(st, cfg)
    JG = rom.J_apply(gr.G)
    P = JG - st.U @ (st.U.T @ JG)
    np.testing.assert_allclose(eps, np.linalg.norm(P) / np.linalg.norm(gr.G), rtol=1e-10)


def test_galerkin_gradient_equals_paper_split_form():
    """g = U_X^T F + (U_V^T U_V) Z (eq. grHDD's linear part and the
    projected force), with F from the brute-force dense operators."""
    st, cfg, ens = _tiny_landau(two_n=6, N=60)
    cfg.Nx = 8
    gr = rom.gradient(st.U, st.Z, st.L, 8)
    N = 60
    UX, UV = st.U[:N], st.U[N:]
    Xr = UX @ st.Z
    F = np.zeros_like(Xr)
    for i in range(st.Z.shape[1]):
        L = st.L[i]
        h = L / 8
        Lam = pic.lambda0_dense(Xr[:, i], L, 8)
        dLam = pic.grad_lambda0_dense(Xr[:, i], L, 8)
        Mq = np.full(N, -L / N)
        Phi = np.linalg.pinv(pic.stiffness_dense(8, h)) @ (Lam.T @ Mq + h)
        F[:, i] = (Mq / (L / N)) * (dLam @ Phi)
    np.testing.assert_allclose(gr.g, UX.T @ F + (UV.T @ UV) @ st.Z, atol=1e-11)


def test_hamiltonian_error_bounded():
    """Relative Hamiltonian error of the reduced solution stays small and does
    not grow secularly over the run (Sec. 6.2, Hamiltonian error study)."""
    st, cfg, _ = _tiny_landau(two_n=10, N=2000)
    _, H0 = rom.diagnostics(st, cfg)
    errs = []
    for _ in range(40):
        assert rom.prk_step(st, cfg) == rom.OK
        errs.append(np.abs(rom.diagnostics(st, cfg)[1] - H0) / np.abs(H0))
    errs = np.array(errs)
    assert errs.max() < 1e-2
    assert errs[20:].max() < 3.0 * errs[:20].max() + 1e-12


def test_enoconv_leaves_state_unchanged():
    st, cfg, _ = _tiny_landau(two_n=6, N=500)
    U0, Z0 = st.U.copy(), st.Z.copy()
    cfg.fp_max_iters = 1
    cfg.fp_tol = 0.0
    assert rom.prk_step(st, cfg) == rom.ENOCONV
    assert np.array_equal(st.U, U0) and np.array_equal(st.Z, Z0)


def test_enoconv_with_deim_keeps_the_snapshot_window():
    """A failed DEIM step leaves the snapshot window as it was, so a retry
    gives the same step as a run that never failed."""
    N = 500
    w = workload("twostream_deim", N=N, p=12, Nx=32)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=12, Nx=32, two_n=6, dt=0.05, projection="deim",
                        deim_window=2, fp_tol=1e-11)
    st = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    ref = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    for _ in range(4):
        assert rom.prk_step(st, cfg) == rom.OK
        assert rom.prk_step(ref, cfg) == rom.OK
    win = [y.copy() for y in st.window]
    bad = rom.RomConfig(**{**cfg.__dict__, "fp_max_iters": 1, "fp_tol": 0.0})
    assert rom.prk_step(st, bad) == rom.ENOCONV
    assert len(st.window) == len(win) and all(np.array_equal(a, b) for a, b in zip(st.window, win))
    assert rom.prk_step(st, cfg) == rom.OK
    assert rom.prk_step(ref, cfg) == rom.OK
    assert np.array_equal(st.U, ref.U) and np.array_equal(st.Z, ref.Z)


def test_stagnation_accepted_only_below_its_floor(monkeypatch):
    """The stagnation rule (a reading: a column whose relative update stops
    decreasing is accepted) applies only once that update is below
    fp_stall_tol.  A gradient that 2-cycles with a large amplitude is a stall
    far above the floor: the step must fail with ENOCONV, and is accepted
    only if the floor is lifted."""
    st, cfg, _ = _tiny_landau(two_n=6, N=400)
    real = rom.reduced_gradient
    calls = {"n": 0}

    def cycling(sub, c, U, Z, op=None):
        g, gr = real(sub, c, U, Z, op)
        calls["n"] += 1
        return g * (1.0 + 0.1 * (calls["n"] % 2)), gr

    monkeypatch.setattr(rom, "reduced_gradient", cycling)
    cfg.fp_max_iters = 30
    s1 = rom.RomState(U=st.U.copy(), Z=st.Z.copy(), L=st.L)
    assert rom.prk_step(s1, cfg) == rom.ENOCONV
    cfg2 = rom.RomConfig(**{**cfg.__dict__, "fp_stall_tol": np.inf})
    s2 = rom.RomState(U=st.U.copy(), Z=st.Z.copy(), L=st.L)
    assert rom.prk_step(s2, cfg2) == rom.OK and s2.last_stalled > 0


def test_automatic_shrink_drops_negligible_pairs():
    """Reading R-4: with no growth (indicator below its threshold), the pairs
    whose singular value of Z~ is below rank_tol_down times the largest are
    dropped, and R changes by exactly the dropped singular values."""
    st, cfg, _ = _tiny_landau(two_n=8, N=900)
    Zt = rom.to_complex_coeff(st.Z)
    Q, s, Wh = np.linalg.svd(Zt, full_matrices=False)
    s_new = s.copy()
    s_new[-1] = 1e-11 * s[0]           # one pair far below the threshold 1e-8
    st.Z = rom.from_complex_coeff((Q * s_new) @ Wh)
    R1 = st.U @ st.Z
    cfg.two_n_max, cfg.rank_tol_up, cfg.rank_tol_down = 12, 2.0, 1e-8
    status, two_n, eps = rom.adapt_rank(st, cfg, 0)
    assert status == rom.OK and two_n == 6 and eps < 1.0
    np.testing.assert_allclose(np.linalg.norm(st.U @ st.Z - R1), s_new[-1], rtol=1e-3)
    assert _orth_err(st.U) < 1e-12
    # nothing below the threshold: the rank stays
    status, two_n, _ = rom.adapt_rank(st, cfg, 0)
    assert two_n == 6


def test_stagnation_accepts_a_cycle_with_a_contracted_phase(monkeypatch):
    """The cycle a node crossing makes (Sec. 2.1: the gathered force is
    piecewise constant in the particle position): the particle changes cell
    every second evaluation, so the updates alternate between a jump of
    about 1e-2 and a contraction step far below it.  The stagnation rule
    measures the cycle by its smaller update: the column is accepted (the
    accepted update, the jump, is reported), whereas a rule on the current
    update alone never fires and the step would fail."""
    st, cfg, _ = _tiny_landau(two_n=6, N=400)
    real = rom.reduced_gradient
    calls = {"n": 0}

    def flipping(sub, c, U, Z, op=None):
        g, gr = real(sub, c, U, Z, op)
        calls["n"] += 1
        jump = 1.0 + 1e-2 * ((calls["n"] // 2) % 2)   # cell A, A, B, B, A, A, ...
        return g * jump, gr

    monkeypatch.setattr(rom, "reduced_gradient", flipping)
    cfg.fp_max_iters = 40
    s1 = rom.RomState(U=st.U.copy(), Z=st.Z.copy(), L=st.L)
    assert rom.prk_step(s1, cfg) == rom.OK
    assert s1.last_stalled > 0 and 1e-3 < s1.last_stall_rel < 5e-2
    # the floor still matters: with it at 1e-12 no contracted phase is small
    # enough and the step fails
    calls["n"] = 0
    cfg2 = rom.RomConfig(**{**cfg.__dict__, "fp_stall_tol": 1e-12})
    s2 = rom.RomState(U=st.U.copy(), Z=st.Z.copy(), L=st.L)
    assert rom.prk_step(s2, cfg2) == rom.ENOCONV


def test_local_singular_values_and_numerical_rank():
    """eq. local_snapshots and the numerical rank of Sec. 6.1: a snapshot
    matrix built from random orthogonal factors and prescribed singular values
    gives those values back, in decreasing order, and the rank counts the
    values strictly above tol times the largest (hand-counted)."""
    rng = np.random.default_rng(7)
    N, p = 200, 12
    sig = np.array([3.0, 1.0, 0.5, 2e-3, 1e-3, 5e-4, 1e-5, 5e-6, 1e-8, 0, 0, 0])
    Uq, _ = np.linalg.qr(rng.normal(size=(N, p)))
    Vq, _ = np.linalg.qr(rng.normal(size=(p, p)))
    order = rng.permutation(p)             # columns of the factor in another order
    S = (Uq * sig[order]) @ Vq.T
    s = rom.local_singular_values(S)
    np.testing.assert_allclose(s, sig, rtol=0, atol=1e-14 * sig[0])
    assert rom.numerical_rank(s, 1e-3) == 3   # above 3e-3: 3, 1, 0.5
    assert rom.numerical_rank(s, 1e-4) == 6   # above 3e-4: and 2e-3, 1e-3, 5e-4
    assert rom.numerical_rank(s, 1e-5) == 6   # 1e-5 is below 3e-5
    assert rom.numerical_rank(s, 1e-6) == 8   # above 3e-6: and 1e-5, 5e-6
    assert rom.numerical_rank(s, 1.0) == 0    # strictly above the largest: none
    assert rom.numerical_rank([], 1e-3) == 0


def test_hamiltonian_split_complete_basis_and_end_rows():
    """eq. error_ham_tot: with a complete basis (2n = 2N) the basis cannot
    move, so U_{tau-1/2} = U_{tau-1} = U_tau: the two basis terms vanish and
    the whole change of the Hamiltonian is the coefficient term.  On a
    low-rank step the first and last rows are the Hamiltonians of the
    states before and after the step, and the basis terms are not zero."""
    rng = np.random.default_rng(11)
    N, p, Nx = 30, 2, 8
    L = np.array([6.0, 7.5])
    X = rng.uniform(0, 1, size=(N, p)) * L[None, :]
    V = rng.normal(size=(N, p))
    cfg = rom.RomConfig(N=N, p=p, Nx=Nx, two_n=2 * N, dt=0.05, fp_tol=1e-14, fp_max_iters=400)
    st = rom.RomState(U=np.eye(2 * N), Z=np.concatenate([X, V], axis=0), L=L)
    U0, Z0 = st.U.copy(), st.Z.copy()
    assert rom.prk_step(st, cfg) == rom.OK
    H = rom.hamiltonian_split(U0, Z0, st.last_U_half, st.last_Z_new, st.U, st.Z, L, Nx)
    scale = np.abs(H).max()
    assert np.abs(H[1] - H[0]).max() < 1e-13 * scale
    assert np.abs(H[3] - H[2]).max() < 1e-13 * scale
    assert np.abs(H[2] - H[1]).max() > 1e-8 * scale      # the coefficients did move
    # a reduced step of the small Landau case
    st, cfg, _ = _tiny_landau(two_n=6, N=400)
    U0, Z0 = st.U.copy(), st.Z.copy()
    _, H0 = rom.diagnostics(st, cfg)
    assert rom.prk_step(st, cfg) == rom.OK
    _, H1 = rom.diagnostics(st, cfg)
    H = rom.hamiltonian_split(U0, Z0, st.last_U_half, st.last_Z_new, st.U, st.Z, st.L, cfg.Nx)
    np.testing.assert_allclose(H[0], H0, rtol=1e-13)
    np.testing.assert_allclose(H[3], H1, rtol=1e-12)
    assert np.linalg.norm(H[1] - H[0]) > 0 and np.linalg.norm(H[3] - H[2]) > 0
