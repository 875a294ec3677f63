"""Oracle: geometric particle-in-cell full-order model (paper Sec. 2.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (readings of the paper, each listed with its reason in the
design notes):
* q = -1, m = 1 (Sec. 6.1); per parameter i the domain is [0, L_i) with
  L_i = 2 pi / k_i, N_x cells of width h_i = L_i / N_x, nodes x_j = j h_i.
* particle weight w_i = L_i / N, so that the particle charge q w_i N = -L_i
  cancels the uniform neutralising background of density 1 (Sec. 2, the
  background charge remark), whose P1 load vector is h_i on every node.
* cell of a particle: s = x * (N_x / L_i) with the factor formed once in
  FP64; c = floor(s); theta = s - c; node index j = c mod N_x (Euclidean).
  A particle on a node belongs to the cell on its right.
* positions are unwrapped; wrapping happens only inside the cell lookup.
* the potential is the zero-mean solution of the singular periodic
  stiffness system (the gauge does not change the field or the energy).
All arrays of particle quantities have shape (N, p): column i is parameter i.
"""
import numpy as np


def mesh(L, Nx):
    """Cell width h_i = L_i / N_x for every parameter."""
    return np.asarray(L, dtype=np.float64) / Nx


def cell_index(X, L, Nx):
    """Node index j (int64) and fraction theta in [0,1) of every particle.

    P1 hat functions on the periodic mesh (Sec. 2.1): a particle in cell
    [x_j, x_{j+1}) has lambda_j = 1 - theta and lambda_{j+1} = theta.
    """
    X = np.asarray(X, dtype=np.float64)
    factor = Nx / np.asarray(L, dtype=np.float64)   # N_x / L_i, one rounding
    s = X * factor
    c = np.floor(s)
    theta = s - c
    j = np.mod(c.astype(np.int64), Nx)
    return j, theta


def lambda0_dense(x, L, Nx):
    """Dense Lambda^0(X) (N x N_x), entries lambda_j(X_l) (Sec. 2.1, def. of Lambda^0).

    Brute-force form, used only on tiny inputs.
    """
    h = L / Nx
    out = np.zeros((x.size, Nx))
    for l, xl in enumerate(x):
        xw = xl - np.floor(xl / L) * L
        for jj in range(Nx):
            for shift in (-L, 0.0, L):
                d = abs(xw - (jj * h + shift)) / h
                if d < 1.0:
                    out[l, jj] += 1.0 - d
    return out


def grad_lambda0_dense(x, L, Nx):
    """Dense nabla Lambda^0(X) (N x N_x): derivative of lambda_j at X_l.

    On the open cell [x_j, x_{j+1}) the derivatives are -1/h (node j) and
    +1/h (node j+1); a particle exactly on a node takes the right cell.
    """
    j, _ = cell_index(np.asarray(x)[:, None], np.array([L]), Nx)
    h = L / Nx
    out = np.zeros((x.size, Nx))
    for l in range(x.size):
        jl = j[l, 0]
        out[l, jl] -= 1.0 / h
        out[l, (jl + 1) % Nx] += 1.0 / h
    return out


def stiffness_dense(Nx, h):
    """Periodic P1 stiffness L_ij = (d lambda_j, d lambda_i) (Sec. 2.1): (1/h) circ(-1, 2, -1)."""
    K = 2.0 * np.eye(Nx) - np.roll(np.eye(Nx), 1, axis=0) - np.roll(np.eye(Nx), -1, axis=0)
    return K / h


def deposit(X, L, Nx, q=-1.0):
    """Charge vector rho_h = Lambda^0(X)^T M_q + background, one column per parameter.

    eq. (PoissonSystem): M_q = q w; plus the P1 load vector h of the uniform
    unit background.  Shape (N_x, p).
    """
    N, p = X.shape
    L = np.asarray(L, dtype=np.float64)
    j, theta = cell_index(X, L, Nx)
    w = L / N
    rho = np.empty((Nx, p))
    for i in range(p):
        qw = q * w[i]
        left = np.bincount(j[:, i], weights=qw * (1.0 - theta[:, i]), minlength=Nx)
        right = np.bincount((j[:, i] + 1) % Nx, weights=qw * theta[:, i], minlength=Nx)
        rho[:, i] = left + right + L[i] / Nx
    return rho


def poisson(rho, L):
    """Zero-mean potential Phi solving L Phi = rho (eq. PoissonSystem).

    The periodic stiffness is singular (constants); the system is solved in
    bordered form [[L, 1], [1^T, 0]] [Phi; lam] = [rho; 0], whose solution is
    the pseudo-inverse solution (rho is projected on zero mean).
    """
    Nx, p = rho.shape
    L = np.asarray(L, dtype=np.float64)
    K1 = stiffness_dense(Nx, 1.0)       # stiffness for h = 1; L = K1 / h
    B = np.zeros((Nx + 1, Nx + 1))
    B[:Nx, :Nx] = K1
    B[:Nx, Nx] = 1.0
    B[Nx, :Nx] = 1.0
    h = mesh(L, Nx)
    rhs = np.zeros((Nx + 1, p))
    rhs[:Nx] = rho * h[None, :]         # K1 Phi = h rho
    sol = np.linalg.solve(B, rhs)
    return sol[:Nx]


def field(Phi, L):
    """Cell field e_j = (Phi_{j+1} - Phi_j) / h (derivative of phi_h on cell j)."""
    Nx = Phi.shape[0]
    h = mesh(L, Nx)
    return (np.roll(Phi, -1, axis=0) - Phi) / h[None, :]


def grad_x(X, e, L, q=-1.0, m=1.0):
    """Position part of the Hamiltonian gradient, eq. (VPHamEqn):
    m_p^{-1} diag(M_q) nabla Lambda^0 L^{-1} Lambda^0^T M_q = (q/m) e_{j(X)}.
    """
    Nx = e.shape[0]
    j, _ = cell_index(X, L, Nx)
    cols = np.arange(X.shape[1])[None, :]
    return (q / m) * e[j, cols]


def electric_energy(Phi, rho, L, N, m=1.0):
    """Electric energy eq. (HamEEfull): E = Phi^T L Phi / (2 m_p) = Phi^T rho / (2 m_p), m_p = m w."""
    mp = m * np.asarray(L, dtype=np.float64) / N
    return np.sum(Phi * rho, axis=0) / (2.0 * mp)


def fields_of(X, L, Nx, q=-1.0):
    """rho, Phi and e for positions X (all parameters)."""
    rho = deposit(X, L, Nx, q)
    Phi = poisson(rho, L)
    return rho, Phi, field(Phi, L)


def hamiltonian(X, V, L, Nx, q=-1.0, m=1.0):
    """Discrete Hamiltonian eq. (high_fidelity_Hamiltonian): 1/2 V^T V + E(X), per parameter."""
    rho, Phi, _ = fields_of(X, L, Nx, q)
    return 0.5 * np.sum(V * V, axis=0) + electric_energy(Phi, rho, L, X.shape[0], m)


def acceleration(X, L, Nx, q=-1.0, m=1.0):
    """dV/dt = -dH/dX = -(q/m) e_{j(X)} (eq. VPHamEqn with the Poisson tensor J_2N)."""
    _, _, e = fields_of(X, L, Nx, q)
    return -grad_x(X, e, L, q, m)


def fom_step(X, V, L, Nx, dt, q=-1.0, m=1.0, a0=None):
    """One Stormer-Verlet step, eq. (sv_full_order), for every parameter.

    X+ = X + dt (V + dt/2 a(X));  V+ = V + dt/2 (a(X) + a(X+)),
    with a = -dH/dX the acceleration (the printed E_h "up to constants").
    Returns (X+, V+, a(X+)) so that a caller can reuse the last field.
    """
    a = acceleration(X, L, Nx, q, m) if a0 is None else a0
    Xn = X + dt * (V + 0.5 * dt * a)
    an = acceleration(Xn, L, Nx, q, m)
    Vn = V + 0.5 * dt * (a + an)
    return Xn, Vn, an


def fom_run(X, V, L, Nx, dt, steps, q=-1.0, m=1.0):
    """``steps`` Stormer-Verlet steps; returns the final state."""
    a = None
    for _ in range(steps):
        X, V, a = fom_step(X, V, L, Nx, dt, q, m, a)
    return X, V


def fom_implicit_midpoint_step(X, V, L, Nx, dt, q=-1.0, m=1.0, tol=1e-13, max_iters=200):
    """Implicit midpoint on W' = J grad H(W), solved by fixed point (test-only variant).

    k = J grad H(W + dt/2 k), iterated from k = J grad H(W) until the relative
    update is below tol; W+ = W + dt k.  This is what the reduced model with
    2n = 2N and U = I must reproduce.
    """
    def rhs(Xe, Ve):
        _, _, e = fields_of(Xe, L, Nx, q)
        return Ve, -grad_x(Xe, e, L, q, m)

    kx, kv = rhs(X, V)
    for _ in range(max_iters):
        nx_, nv_ = rhs(X + 0.5 * dt * kx, V + 0.5 * dt * kv)
        num = np.sqrt(np.sum((nx_ - kx) ** 2) + np.sum((nv_ - kv) ** 2))
        den = np.sqrt(np.sum(nx_ ** 2) + np.sum(nv_ ** 2))
        kx, kv = nx_, nv_
        if num <= tol * den:
            break
    return X + dt * kx, V + dt * kv
