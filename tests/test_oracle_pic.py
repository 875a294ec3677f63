"""Pins of the full-order PIC oracle against closed forms, invariants and
brute force (none of them re-types the oracle's own formula)."""
import math

import numpy as np
import pytest
from scipy.special import wofz

from oracle import pic
from workloads import hammersley_uniforms, load_particles


def _tiny(seed=0, N=24, p=3, Nx=8):
    rng = np.random.default_rng(seed)
    L = rng.uniform(8.0, 14.0, size=p)
    X = rng.uniform(-2.0, 3.0, size=(N, p)) * L[None, :]   # unwrapped positions
    V = rng.normal(size=(N, p))
    return X, V, L, Nx


def test_cell_index_brute_force_and_node_ties():
    X, _, L, Nx = _tiny()
    j, th = pic.cell_index(X, L, Nx)
    for i in range(X.shape[1]):
        h = L[i] / Nx
        for l in range(X.shape[0]):
            x = X[l, i] % L[i]
            # brute force: the node j with j h <= x < (j+1) h
            jj = int(math.floor(x / h + 1e-300)) % Nx
            assert abs(jj - j[l, i]) in (0, Nx) or abs(x / h - round(x / h)) < 1e-9
            assert 0.0 <= th[l, i] < 1.0
    # particles exactly on nodes belong to the cell on their right (theta = 0)
    L1 = np.array([8.0])
    Xn = np.array([[0.0], [1.0], [7.0], [-1.0], [8.0], [16.0]])
    j, th = pic.cell_index(Xn, L1, 8)
    assert list(j[:, 0]) == [0, 1, 7, 7, 0, 0]
    assert np.all(th == 0.0)


def test_deposit_total_charge_and_partition_of_unity():
    """Sum of particle charges is q w N = -L; with the background, sum rho = 0."""
    X, _, L, Nx = _tiny(N=5000, p=4, Nx=32)
    rho = pic.deposit(X, L, Nx)
    particle = rho - (L / Nx)[None, :]
    np.testing.assert_allclose(particle.sum(axis=0), -L, rtol=1e-13)
    assert np.all(np.abs(rho.sum(axis=0)) < 1e-12 * L)


def test_deposit_equals_dense_lambda0():
    """rho = Lambda^0(X)^T M_q + h 1 with the brute-force dense Lambda^0."""
    X, _, L, Nx = _tiny()
    rho = pic.deposit(X, L, Nx)
    N = X.shape[0]
    for i in range(X.shape[1]):
        Lam = pic.lambda0_dense(X[:, i], L[i], Nx)
        ref = Lam.T @ np.full(N, -L[i] / N) + L[i] / Nx
        np.testing.assert_allclose(rho[:, i], ref, rtol=0, atol=1e-13)


def test_poisson_single_mode_closed_form():
    """A cosine mode m is an eigenvector of the periodic P1 stiffness with
    eigenvalue mu_m = (4/h) sin^2(pi m / N_x)."""
    Nx = 16
    L = np.array([10.0, 3.0])
    j = np.arange(Nx)
    for m in (1, 3, 7):
        rho = np.cos(2 * np.pi * m * j / Nx)[:, None] * np.ones((1, 2))
        Phi = pic.poisson(rho, L)
        h = L / Nx
        mu = 4.0 / h * np.sin(np.pi * m / Nx) ** 2
        np.testing.assert_allclose(Phi, rho / mu[None, :], rtol=0, atol=1e-13)


def test_poisson_residual_and_gauge():
    X, _, L, Nx = _tiny(N=400)
    rho = pic.deposit(X, L, Nx)
    Phi = pic.poisson(rho, L)
    for i in range(len(L)):
        K = pic.stiffness_dense(Nx, L[i] / Nx)
        np.testing.assert_allclose(K @ Phi[:, i], rho[:, i] - rho[:, i].mean(), atol=1e-12)
        assert abs(Phi[:, i].mean()) < 1e-13


def test_energy_identity():
    """Phi^T rho / (2 m_p) equals Phi^T L Phi / (2 m_p) (eq. HamEEfull)."""
    X, _, L, Nx = _tiny(N=400)
    rho = pic.deposit(X, L, Nx)
    Phi = pic.poisson(rho, L)
    E = pic.electric_energy(Phi, rho, L, X.shape[0])
    for i in range(len(L)):
        K = pic.stiffness_dense(Nx, L[i] / Nx)
        mp = L[i] / X.shape[0]
        np.testing.assert_allclose(E[i], Phi[:, i] @ K @ Phi[:, i] / (2 * mp), rtol=1e-12)


def test_gradient_is_finite_difference_of_hamiltonian():
    """dH/dX_l by central differences matches (q/m) e_{j(X_l)}: the discrete
    energy is quadratic in X_l inside a cell, so the difference is exact up to
    rounding."""
    X, V, L, Nx = _tiny(seed=3, N=20, p=2)
    rho, Phi, e = pic.fields_of(X, L, Nx)
    F = pic.grad_x(X, e, L)
    eps = 1e-6
    for i in range(2):
        for l in range(X.shape[0]):
            Xp = X.copy(); Xp[l, i] += eps
            Xm = X.copy(); Xm[l, i] -= eps
            Hp = pic.hamiltonian(Xp, V, L, Nx)[i]
            Hm = pic.hamiltonian(Xm, V, L, Nx)[i]
            fd = (Hp - Hm) / (2 * eps)
            assert abs(fd - F[l, i]) < 1e-7 * max(1.0, abs(F[l, i]))


def test_gradient_equals_dense_formula():
    """m_p^-1 diag(M_q) nabla Lambda0 L^+ Lambda0^T M_q + background, brute force."""
    X, _, L, Nx = _tiny(seed=5)
    _, _, e = pic.fields_of(X, L, Nx)
    F = pic.grad_x(X, e, L)
    N = X.shape[0]
    for i in range(X.shape[1]):
        h = L[i] / Nx
        Lam = pic.lambda0_dense(X[:, i], L[i], Nx)
        dLam = pic.grad_lambda0_dense(X[:, i], L[i], Nx)
        Mq = np.full(N, -L[i] / N)
        rho = Lam.T @ Mq + h
        K = pic.stiffness_dense(Nx, h)
        Phi = np.linalg.pinv(K) @ rho
        mp = L[i] / N
        ref = (Mq / mp) * (dLam @ Phi)
        np.testing.assert_allclose(F[:, i], ref, atol=1e-11)


def _small_fom(N=2000, p=2, Nx=32):
    rng = np.random.default_rng(7)
    L = np.array([4 * np.pi, 4 * np.pi])[:p]
    ux, uv = hammersley_uniforms(N)
    params = dict(alpha=np.full(p, 0.3), k=2 * np.pi / L, v0=np.zeros(p),
                  sigma=np.array([1.0, 0.8])[:p])
    X, V = load_particles(params, ux, uv, "landau")
    return np.array(X), np.array(V), L, Nx


def _no_crossing_case(N=2000, p=2, Nx=32, seed=11):
    """Particles placed inside cells, away from the nodes, nearly at rest:
    over the short horizon used below no particle reaches a node, so the
    force is a smooth function of the state (the P1 field is discontinuous
    across nodes, which caps the observed order at 1 when particles cross)."""
    rng = np.random.default_rng(seed)
    L = np.array([4 * np.pi, 3 * np.pi])[:p]
    h = L / Nx
    c = rng.integers(0, Nx, size=(N, p))
    X = h[None, :] * (c + 0.3 + 0.4 * rng.random((N, p)))
    V = 0.01 * rng.normal(size=(N, p))
    return X, V, L, Nx


def test_stormer_verlet_order_two():
    X, V, L, Nx = _no_crossing_case()
    T = 0.2
    j0, _ = pic.cell_index(X, L, Nx)
    ref = pic.fom_run(X, V, L, Nx, T / 64, 64)
    assert np.array_equal(pic.cell_index(ref[0], L, Nx)[0], j0)
    errs = []
    for nsteps in (4, 8):
        Xs, Vs = pic.fom_run(X, V, L, Nx, T / nsteps, nsteps)
        assert np.array_equal(pic.cell_index(Xs, L, Nx)[0], j0)
        errs.append(np.linalg.norm(Xs - ref[0]) + np.linalg.norm(Vs - ref[1]))
    order = math.log2(errs[0] / errs[1])
    assert 1.9 <= order <= 2.1, order


def test_stormer_verlet_time_reversible():
    X, V, L, Nx = _small_fom()
    X1, V1 = pic.fom_run(X, V, L, Nx, 0.05, 10)
    X2, V2 = pic.fom_run(X1, V1, L, Nx, -0.05, 10)
    assert np.abs(X2 - X).max() < 1e-11
    assert np.abs(V2 - V).max() < 1e-11


def test_stormer_verlet_energy_bounded():
    X, V, L, Nx = _small_fom()
    H0 = pic.hamiltonian(X, V, L, Nx)
    dev = []
    a = None
    for _ in range(200):
        X, V, a = pic.fom_step(X, V, L, Nx, 0.05, a0=a)
        dev.append(np.abs(pic.hamiltonian(X, V, L, Nx) - H0) / np.abs(H0))
    dev = np.array(dev)
    # no secular drift: the second half is not worse than twice the first
    assert dev.max() < 1e-3
    assert dev[100:].max() < 2.0 * dev[:100].max() + 1e-12


def _landau_rate(k, sigma=1.0):
    """Least-damped root of the Maxwellian Langmuir dispersion relation
    1 + (1 + zeta Z(zeta)) / (k sigma)^2 = 0, Z(z) = i sqrt(pi) w(z)."""
    def D(om):
        z = om / (k * sigma * math.sqrt(2))
        Zf = 1j * math.sqrt(math.pi) * wofz(z)
        return 1 + (1 + z * Zf) / (k * sigma) ** 2
    om = complex(math.sqrt(1 + 3 * (k * sigma) ** 2), -0.1)
    for _ in range(100):
        d = (D(om + 1e-7) - D(om - 1e-7)) / 2e-7
        step = D(om) / d
        om -= step
        if abs(step) < 1e-14:
            break
    return om


def test_landau_dispersion_root_known_value():
    """Textbook value for k = 0.5: omega = 1.4157 - 0.1534 i."""
    om = _landau_rate(0.5)
    assert abs(om.real - 1.4157) < 1e-3 and abs(om.imag + 0.1534) < 1e-3


@pytest.mark.slow
def test_linear_landau_damping_rate():
    """Peaks of the electric energy decay as exp(2 gamma t) with gamma the
    imaginary part of the dispersion root (the paper's damping-rate study,
    Sec. 6.2, fits peaks of E(t))."""
    N, Nx, dt = 100_000, 64, 0.05
    k, alpha = 0.5, 0.05
    L = np.array([2 * np.pi / k])
    ux, uv = hammersley_uniforms(N)
    params = dict(alpha=np.array([alpha]), k=np.array([k]), v0=np.zeros(1), sigma=np.ones(1))
    X, V = load_particles(params, ux, uv, "landau")
    X, V = np.array(X), np.array(V)
    ts, Es = [], []
    a = None
    for s in range(1, int(15.0 / dt) + 1):
        X, V, a = pic.fom_step(X, V, L, Nx, dt, a0=a)
        rho, Phi, _ = pic.fields_of(X, L, Nx)
        ts.append(s * dt)
        Es.append(pic.electric_energy(Phi, rho, L, N)[0])
    ts, Es = np.array(ts), np.array(Es)
    peaks = [i for i in range(1, len(Es) - 1) if Es[i] > Es[i - 1] and Es[i] >= Es[i + 1]
             and ts[i] >= 2.0]
    slope = np.polyfit(ts[peaks], np.log(Es[peaks]), 1)[0]
    gamma2 = 2 * _landau_rate(k).imag
    assert abs(slope - gamma2) < 0.05 * abs(gamma2), (slope, gamma2)


def test_nonlinear_landau_growth_rate_golden():
    """Trapping-phase growth rate of the field amplitude for the nonlinear
    Landau case eta = (0.5, 1) against the value the paper prints (Sec. 6.3,
    fixture tests/golden/nld_rates.txt), within 10 %."""
    from rates import read_golden, trapping_growth_rate
    g = read_golden("nld_rates.txt")
    N, Nx, dt = 100_000, int(g["Nx"]), 0.05
    L = np.array([2 * np.pi / g["k"]])
    ux, uv = hammersley_uniforms(N)
    params = dict(alpha=np.array([g["alpha"]]), k=np.array([g["k"]]), v0=np.zeros(1),
                  sigma=np.array([g["sigma"]]))
    X, V = load_particles(params, ux, uv, "landau")
    X, V = np.array(X), np.array(V)
    ts, Es = [], []
    a = None
    for s in range(1, int(round(g["t_end"] / dt)) + 1):
        X, V, a = pic.fom_step(X, V, L, Nx, dt, a0=a)
        rho, Phi, _ = pic.fields_of(X, L, Nx)
        ts.append(s * dt)
        Es.append(pic.electric_energy(Phi, rho, L, N)[0])
    rate = trapping_growth_rate(ts, Es)
    assert abs(rate - g["growth_rate"]) < 0.1 * g["growth_rate"], rate
