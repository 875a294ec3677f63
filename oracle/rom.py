"""Oracle: dynamical symplectic reduced model (paper Sec. 3.2 and Sec. 5).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Real formulation as printed: U in R^{2N x 2n} orthosymplectic (U^T U = I,
U^T J_2N U = J_2n), Z in R^{2n x p}, R = U Z.  U = [U_X; U_V] by rows.
The time step is the order-2 partitioned Runge-Kutta scheme of Sec. 5
(eq. discrete_dynROM): implicit midpoint for Z, explicit midpoint on the
tangent space for U through the Cayley retraction, with tableaux
  Z:  A = [[0, 0], [0, 1/2]], b = (0, 1), c = (0, 1/2)
  U:  A^ = [[0, 0], [1/2, 0]], b^ = (0, 1).
Readings where the paper is silent are listed in the design notes; the ones
that shape code here are marked "reading:" in the docstrings.
"""
from dataclasses import dataclass, field as dc_field
from typing import Optional

import numpy as np

from . import pic

OK, ENOCONV, ESINGULAR, ERANKCAP = 0, -4, -3, -7


# ----------------------------------------------------------------------------
# Poisson tensors and the complex representation
# ----------------------------------------------------------------------------

def J_small(r):
    """J_{2n} = [[0, I], [-I, 0]] (Sec. 2.1, definition of the Poisson tensor)."""
    n = r // 2
    J = np.zeros((r, r))
    J[:n, n:] = np.eye(n)
    J[n:, :n] = -np.eye(n)
    return J


def J_apply(M):
    """J_{2N} M for a matrix with 2N rows: [M_V; -M_X]."""
    N = M.shape[0] // 2
    return np.concatenate([M[N:], -M[:N]], axis=0)


def to_complex_basis(U):
    """U = [[A, -B], [B, A]] -> U~ = A + iB (N x n)."""
    N = U.shape[0] // 2
    n = U.shape[1] // 2
    return U[:N, :n] + 1j * U[N:, :n]


def from_complex_basis(Ut):
    """U~ = A + iB -> U = [[A, -B], [B, A]] (2N x 2n)."""
    A, B = Ut.real, Ut.imag
    return np.block([[A, -B], [B, A]])


def to_complex_coeff(Z):
    n = Z.shape[0] // 2
    return Z[:n] + 1j * Z[n:]


def from_complex_coeff(Zt):
    return np.concatenate([Zt.real, Zt.imag], axis=0)


def canonical_phase(Q):
    """Rotate each column so its largest-modulus entry is real positive
    (ties go to the smallest row index).  reading: fixes the SVD gauge."""
    Q = Q.copy()
    for k in range(Q.shape[1]):
        i = int(np.argmax(np.abs(Q[:, k])))
        a = Q[i, k]
        if abs(a) > 0:
            Q[:, k] *= np.conj(a) / abs(a)
    return Q


# ----------------------------------------------------------------------------
# Configuration and state
# ----------------------------------------------------------------------------

@dataclass
class RomConfig:
    N: int
    p: int
    Nx: int
    two_n: int
    two_n_max: int = 0
    dt: float = 0.05
    q: float = -1.0
    m: float = 1.0
    fp_tol: float = 1e-9          # relative update threshold (Sec. 6.1)
    fp_max_iters: int = 100
    fp_stall_tol: float = 1e-3    # stagnation accepted only below this update
    pinv_rtol: float = 1e-12
    projection: str = "galerkin"  # "deim" (exact potential) or "dmd_deim" (Alg. 2)
    deim_window: int = 3          # T: the window holds T + 1 snapshots
    deim_rows: int = 0            # d, DEIM sample rows; 0: d = 2n
    deim_update_every: int = 1    # k_DEIM: full greedy every k-th DEIM operator
    deim_update_rows: int = 0     # n_DEIM: positions chosen again in between
    p_star: int = 0               # dmd_deim: subset size p* (0: p), eq. pSampl
    dmd_tol: float = 1e-5         # dmd_deim: relative singular value cut (Sec. 6.1)
    reorth: bool = True
    rank_auto: bool = False
    rank_tol_up: float = 1e-2
    rank_tol_down: float = 1e-8

    def __post_init__(self):
        if self.two_n_max == 0:
            self.two_n_max = self.two_n


@dataclass
class RomState:
    U: np.ndarray                 # 2N x 2n
    Z: np.ndarray                 # 2n x p
    L: np.ndarray                 # p domain lengths
    step: int = 0
    window: list = dc_field(default_factory=list)   # DEIM snapshots (N x p each)
    last_iters: int = 0
    last_stalled: int = 0
    last_stall_rel: float = 0.0   # largest relative update accepted by the stagnation rule
    last_status: int = OK
    deim_indices: Optional[np.ndarray] = None
    deim_psi: Optional[np.ndarray] = None   # DEIM basis of the last operator
    deim_builds: int = 0                    # DEIM operators built so far
    eta: Optional[np.ndarray] = None        # dim x p parameters (dmd_deim)
    subset: Optional[np.ndarray] = None     # S_{p*}, fixed at t = 0 (dmd_deim)
    phi_window: list = dc_field(default_factory=list)   # subset potentials (N_x x p*)
    last_dmd_rank: int = 0
    last_dmd: object = None                 # DMD operator of the last DMD-DEIM step
    last_dmd_tables: object = None          # its field tables (e at t_{tau-1}, at + dt/2)
    last_U_half: Optional[np.ndarray] = None   # U_{tau-1/2} of the last step
    last_Z_new: Optional[np.ndarray] = None    # Z_tau of that step, before re-orthonormalisation


# ----------------------------------------------------------------------------
# Initialisation: truncated complex SVD of R_0 (eq. UZred, initial condition)
# ----------------------------------------------------------------------------

def init_csvd(X0, V0, two_n):
    """U^0, Z^0 from the truncated complex SVD of C_0 = X_0 + i V_0.

    The leading n left singular vectors form U~ (canonical phase); when n
    exceeds the number of available singular vectors the basis is completed
    by complex Gram-Schmidt of e_1, e_2, ... (reading: the paper needs
    2n < p; the tiny workload has p < n).  Z~ = U~^* C_0.
    """
    n = two_n // 2
    C = X0 + 1j * V0
    Q, s, _ = np.linalg.svd(C, full_matrices=False)
    k = min(n, Q.shape[1])
    Ut = canonical_phase(Q[:, :k])
    e = 0
    while Ut.shape[1] < n:
        v = np.zeros(C.shape[0], dtype=complex)
        v[e] = 1.0
        e += 1
        for _ in range(2):
            v = v - Ut @ (Ut.conj().T @ v)
        nv = np.linalg.norm(v)
        if nv > 1e-8:
            Ut = np.concatenate([Ut, (v / nv)[:, None]], axis=1)
    Zt = Ut.conj().T @ C
    return from_complex_basis(Ut), from_complex_coeff(Zt)


def local_singular_values(S):
    """Singular values, decreasing, of a local snapshot matrix S^tau = [X^1
    ... X^p] (or of the velocities) of eq. local_snapshots (Sec. 6.1)."""
    return np.linalg.svd(np.asarray(S), compute_uv=False)


def numerical_rank(sig, tol):
    """The numerical rank of Sec. 6.1: the number of singular values above
    tol times the largest."""
    sig = np.asarray(sig, dtype=np.float64)
    return int(np.sum(sig > tol * sig[0])) if sig.size else 0


def init_state(X0, V0, L, cfg, eta=None):
    U, Z = init_csvd(X0, V0, cfg.two_n)
    st = RomState(U=U, Z=Z, L=np.asarray(L, dtype=np.float64).copy())
    if cfg.projection == "dmd_deim":
        from . import dmd
        p = Z.shape[1]
        st.eta = None if eta is None else np.atleast_2d(np.asarray(eta, dtype=np.float64))
        st.subset = dmd.select_subset(Z, cfg.p_star if cfg.p_star > 0 else p)
    return st


# ----------------------------------------------------------------------------
# Hamiltonian gradient (eq. grads, eq. grH-full)
# ----------------------------------------------------------------------------

@dataclass
class Gradient:
    G: np.ndarray        # 2N x p : [F; V_r]
    g: np.ndarray        # 2n x p : U^T G
    rho: np.ndarray      # Nx x p
    Phi: np.ndarray      # Nx x p
    e: np.ndarray        # Nx x p
    Xr: np.ndarray       # N x p


def gradient(U, Z, L, Nx, q=-1.0, m=1.0):
    """G_i = grad_{U Z_i} H = [(q/m) e_{j(X_r^i)}; V_r^i] and g_i = U^T G_i."""
    N = U.shape[0] // 2
    Xr = U[:N] @ Z
    Vr = U[N:] @ Z
    rho, Phi, e = pic.fields_of(Xr, L, Nx, q)
    F = pic.grad_x(Xr, e, L, q, m)
    G = np.concatenate([F, Vr], axis=0)
    return Gradient(G=G, g=U.T @ G, rho=rho, Phi=Phi, e=e, Xr=Xr)


# ----------------------------------------------------------------------------
# Basis velocity (eq. UZred_basis) and S(Z)
# ----------------------------------------------------------------------------

def S_of(Z):
    """S(Z) = Z Z^T + J^T Z Z^T J (Sec. 3.2; reading of the sign, see notes)."""
    J = J_small(Z.shape[0])
    ZZ = Z @ Z.T
    return ZZ + J.T @ ZZ @ J


def pinv_sym(S, rtol):
    """Moore-Penrose inverse of a symmetric PSD matrix by eigendecomposition,
    dropping eigenvalues below rtol * lambda_max (reading: S may be singular
    when p < n)."""
    lam, Q = np.linalg.eigh(S)
    lmax = lam.max() if lam.size else 0.0
    keep = lam > rtol * lmax
    inv = np.zeros_like(lam)
    inv[keep] = 1.0 / lam[keep]
    return (Q * inv[None, :]) @ Q.T


def basis_velocity(U, Z, G, rtol=1e-12):
    """X(U, Z) = (I - U U^T)(J_2N G Z^T - G Z^T J_2n^T) S(Z)^+ (eq. UZred_basis)."""
    J = J_small(Z.shape[0])
    GZ = G @ Z.T
    M = J_apply(GZ) - GZ @ J.T
    M = M - U @ (U.T @ M)
    return M @ pinv_sym(S_of(Z), rtol)


# ----------------------------------------------------------------------------
# Cayley retraction and tangent velocity (Sec. 5)
# ----------------------------------------------------------------------------

def _W_of(U0, xi):
    """W with 2W = (2I - U0 U0^T) xi."""
    return xi - 0.5 * U0 @ (U0.T @ xi)


def cayley_dense(U0, xi):
    """R_{U0}(xi) = cay(W U0^T - U0 W^T) U0 with cay(O) = (I - O/2)^{-1}(I + O/2).

    Dense 2N x 2N form; tiny inputs only.  reading: the 1/2 scaling of the
    Cayley transform (the only one for which the printed tangent velocity is
    consistent with the retraction; checked numerically in the tests).
    """
    W = _W_of(U0, xi)
    Om = W @ U0.T - U0 @ W.T
    I = np.eye(Om.shape[0])
    return np.linalg.solve(I - 0.5 * Om, (I + 0.5 * Om) @ U0)


def cayley(U0, xi):
    """Same map as ``cayley_dense`` in O(N n^2): with Om = Lc Rc^T,
    Lc = [W, -U0], Rc = [U0, W], cay(Om) U0 = U0 + Lc (I - Rc^T Lc / 2)^{-1} Rc^T U0
    (Sherman-Morrison-Woodbury applied to (I - Om/2)^{-1})."""
    W = _W_of(U0, xi)
    Lc = np.concatenate([W, -U0], axis=1)
    Rc = np.concatenate([U0, W], axis=1)
    K = np.eye(Lc.shape[1]) - 0.5 * (Rc.T @ Lc)
    return U0 + Lc @ np.linalg.solve(K, Rc.T @ U0)


def tangent_velocity(U0, xi, Z, G, rtol=1e-12, Ux=None):
    """Y(xi, Z) of Sec. 5: the local velocity on the tangent space at U0.

    G is the gradient evaluated at (R_{U0}(xi), Z).
      Ups = (2 X - (W U0^T - U0 W^T) X) (U0^T Ux + I)^{-1}
      Y   = -U0 (Ux^T U0 + I)^{-1} (Ux + U0)^T Ups + Ups - U0 Ups^T U0
    with Ux = R_{U0}(xi) and X = X(Ux, Z); the 2N x 2N product is applied as
    W (U0^T X) - U0 (W^T X).
    """
    if Ux is None:
        Ux = cayley(U0, xi)
    W = _W_of(U0, xi)
    Xv = basis_velocity(Ux, Z, G, rtol)
    I = np.eye(U0.shape[1])
    Ups = (2.0 * Xv - (W @ (U0.T @ Xv) - U0 @ (W.T @ Xv))) @ np.linalg.inv(U0.T @ Ux + I)
    return (-U0 @ np.linalg.solve(Ux.T @ U0 + I, (Ux + U0).T @ Ups)
            + Ups - U0 @ (Ups.T @ U0))


# ----------------------------------------------------------------------------
# Re-orthonormalisation (not in the paper: exact invariants drift in FP)
# ----------------------------------------------------------------------------

def reorthonormalise(U, Z):
    """Complex QR U~ = Q R with real positive diag(R); U~ <- Q, Z~ <- R Z~.

    R = U Z is unchanged; the real form of Q is orthosymplectic.
    """
    Ut = to_complex_basis(U)
    Q, Rm = np.linalg.qr(Ut)
    d = np.diag(Rm)
    ph = d / np.abs(d)
    Q = Q * ph[None, :]
    Rm = np.conj(ph)[:, None] * Rm
    Zt = Rm @ to_complex_coeff(Z)
    return from_complex_basis(Q), from_complex_coeff(Zt)


# ----------------------------------------------------------------------------
# One partitioned Runge-Kutta step (eq. discrete_dynROM)
# ----------------------------------------------------------------------------

def _col_norms(A):
    return np.sqrt(np.sum(A * A, axis=0))


def reduced_gradient(st, cfg, U, Z, deim_op=None):
    """g(U, Z) for the coefficient equation: Galerkin U^T G, or the DEIM
    variant (eq. grHDD with the exact potential)."""
    gr = gradient(U, Z, st.L, cfg.Nx, cfg.q, cfg.m)
    if deim_op is None:
        return gr.g, gr
    from . import deim
    return deim.deim_gradient(U, Z, gr, deim_op, cfg), gr


def prk_step(st, cfg, fixed_iters=None):
    """Advance (U, Z) by one step of the partitioned RK scheme.

    1. k1 = J g(U0, Z0);  k^1 = X(U0, Z0).
    2. xi_half = dt/2 k^1;  U_half = R_{U0}(xi_half).
    3. k2 = J g(U_half, Z0 + dt/2 k2) by fixed point from k2 = k1, per column,
       stopping on relative update < fp_tol (Sec. 6.1); converged columns are
       frozen (reading).  ``fixed_iters`` forces an exact iteration count.
    4. Z1 = Z0 + dt k2.
    5. k^2 = Y(xi_half, Z_G), Z_G the point of the last gradient of each
       column (reading);  U1 = R_{U0}(dt k^2).
    6. re-orthonormalise (an addition to the paper's scheme).
    Returns the status (OK or ENOCONV); on ENOCONV the state (U, Z and the
    DEIM snapshot window) is unchanged.
    """
    from . import deim as deim_mod
    if cfg.projection == "dmd_deim":
        return _prk_step_dmd(st, cfg, fixed_iters)
    return _prk_step_core(st, cfg, fixed_iters)


def _prk_step_core(st, cfg, fixed_iters):
    from . import deim as deim_mod
    J = J_small(cfg.two_n)
    U0, Z0 = st.U, st.Z
    dt = cfg.dt
    p = Z0.shape[1]

    gr0 = gradient(U0, Z0, st.L, cfg.Nx, cfg.q, cfg.m)
    deim_op = None
    window0 = list(st.window)
    indices0, psi0, builds0 = st.deim_indices, st.deim_psi, st.deim_builds
    if cfg.projection == "deim":
        deim_op = deim_mod.update_window(st, cfg, U0, gr0)
    g1 = gr0.g if deim_op is None else deim_mod.deim_gradient(U0, Z0, gr0, deim_op, cfg)
    k1 = J @ g1
    kh1 = basis_velocity(U0, Z0, gr0.G, cfg.pinv_rtol)

    xi_half = 0.5 * dt * kh1
    U_half = cayley(U0, xi_half)

    def g_of(cols, Ze):
        sub = RomState(U=U_half, Z=Ze, L=st.L[cols])
        op = None if deim_op is None else deim_mod.restrict(deim_op, cols)
        return reduced_gradient(sub, cfg, U_half, Ze, op)[0]

    # reading (stagnation rule, in ``_fixed_point``): the gathered force is
    # piecewise constant in a particle's own position (the cell field of
    # Sec. 2.1), so a particle whose midpoint sits at a node can put the map
    # into a cycle: the iterates alternate between contraction steps with the
    # particle in one cell and jumps when it changes cell.  A column whose
    # relative update stops decreasing is accepted at its current iterate,
    # provided the smaller of its last two updates is below fp_stall_tol (the
    # cycle has a contracted phase); otherwise the column keeps iterating and
    # the step fails at fp_max_iters
    k, ZG, iters, stalled, stall_rel, ok = _fixed_point(Z0, k1, dt, cfg, fixed_iters, g_of)
    st.last_iters = iters
    st.last_stalled = stalled
    st.last_stall_rel = stall_rel
    if not ok:
        # the state, the DEIM snapshot window included, stays as it was
        st.window = window0
        st.deim_indices, st.deim_psi, st.deim_builds = indices0, psi0, builds0
        st.last_status = ENOCONV
        return ENOCONV

    Z1 = Z0 + dt * k
    grG = gradient(U_half, ZG, st.L, cfg.Nx, cfg.q, cfg.m)
    kh2 = tangent_velocity(U0, xi_half, ZG, grG.G, cfg.pinv_rtol, Ux=U_half)
    U1 = cayley(U0, dt * kh2)
    st.last_U_half, st.last_Z_new = U_half, Z1.copy()
    if cfg.reorth:
        U1, Z1 = reorthonormalise(U1, Z1)
    st.U, st.Z = U1, Z1
    st.step += 1
    st.last_status = OK
    return OK


def _fixed_point(Z0, k1, dt, cfg, fixed_iters, g_of):
    """k = J g(Z0 + dt/2 k) per column from k = k1 with the convergence and
    stagnation rules of ``prk_step``; g_of(cols, Ze) evaluates the gradient
    of the active columns.  Returns (k, ZG, iters, stalled, stall_rel, ok)."""
    J = J_small(Z0.shape[0])
    p = Z0.shape[1]
    k = k1.copy()
    ZG = Z0.copy()
    active = np.ones(p, dtype=bool)
    prev = np.full(p, np.inf)
    iters = stalled = 0
    stall_rel = 0.0
    limit = fixed_iters if fixed_iters is not None else cfg.fp_max_iters
    while active.any() and iters < limit:
        iters += 1
        cols = np.nonzero(active)[0]
        Ze = Z0[:, cols] + 0.5 * dt * k[:, cols]
        kn = J @ g_of(cols, Ze)
        ZG[:, cols] = Ze
        if fixed_iters is None:
            nk = _col_norms(kn)
            rel = _col_norms(kn - k[:, cols]) / np.where(nk > 0, nk, 1.0)
            conv = rel < cfg.fp_tol
            stall = ~conv & (rel >= prev[cols]) & (np.minimum(rel, prev[cols]) < cfg.fp_stall_tol)
            stalled += int(np.sum(stall))
            if stall.any():
                stall_rel = max(stall_rel, float(rel[stall].max()))
            done = conv | stall
            prev[cols] = rel
        else:
            done = np.zeros(cols.size, dtype=bool)
        k[:, cols] = kn
        active[cols[done]] = False
    ok = fixed_iters is not None or not active.any()
    return k, ZG, iters, stalled, stall_rel, ok


def dmd_deim_gradient(U, Z, e, L, op, cfg):
    """eq. grHDD: g^DD = U_V^T V_r + (q/m) U_X[I,:]^T (w * e_{j(X_r[I])}), with
    e the cell field of the DMD potential Phi_DMD(t) (the gradient of the
    Lambda^0(X_r) Phi_DMD term at the DEIM particles).  Only the d sampled
    rows of X_r are formed."""
    N = U.shape[0] // 2
    XI = U[:N][op.idx, :] @ Z
    j, _ = pic.cell_index(XI, L, cfg.Nx)
    FI = (cfg.q / cfg.m) * e[j, np.arange(Z.shape[1])[None, :]]
    return U[N:].T @ (U[N:] @ Z) + U[:N][op.idx, :].T @ (FI * op.w[:, None])


def _prk_step_dmd(st, cfg, fixed_iters):
    """One step of Alg. 2.  At the start of every step the exact potential of
    the subset parameters S (Sec. 4.1) is computed with the basis velocity of
    the subset; it enters the DMD window (eq. DMD_potential_Y_time) and the
    DEIM snapshots Lambda^0(X_r) Phi (eq. Ydeim).  While the windows hold
    fewer than T+1 levels the step is the plain reduced step (Alg. 2, first
    T steps).  Afterwards:
      k^1 = X(U0, Z0[S]) with the exact subset gradient G^{p*} (eq. UZredhyp);
      k1  = J g^DD(U0, Z0, t_{tau-1});  U_half = R_{U0}(dt/2 k^1);
      k2  = J g^DD(U_half, Z0 + dt/2 k2, t_{tau-1} + dt/2) by fixed point;
      Z1  = Z0 + dt k2;
      k^2 = Y(dt/2 k^1, Z_G[S]) with G^{p*} at (U_half, Z_G[S]);  U1 = R_{U0}(dt k^2).
    On ENOCONV the state and both windows are unchanged."""
    from . import deim as deim_mod
    from . import dmd
    S = st.subset
    T = cfg.deim_window
    U0, Z0, L = st.U, st.Z, st.L
    dt = cfg.dt
    saved = (list(st.window), list(st.phi_window), st.deim_indices, st.deim_psi,
             st.deim_builds)

    grS = gradient(U0, Z0[:, S], L[S], cfg.Nx, cfg.q, cfg.m)
    st.phi_window.append(grS.Phi.copy())
    st.window.append(deim_mod.snapshot(grS.Xr, grS.Phi, L[S]))
    if len(st.window) > T + 1:
        st.window.pop(0)
        st.phi_window.pop(0)
    if len(st.window) < T + 1:
        st.deim_indices = None
        status = _prk_step_core(st, replace_projection(cfg, "galerkin"), fixed_iters)
        if status != OK:
            st.window, st.phi_window = saved[0], saved[1]
        return status

    op = deim_mod.build_from_window(st, cfg)
    if st.eta is None:
        raise ValueError("dmd_deim needs the parameters eta for the interpolation")
    dop = dmd.build_operator(st.phi_window, S, st.eta, dt, cfg.dmd_tol)
    st.last_dmd_rank = dop.r
    from . import pic as pic_mod
    e0 = pic_mod.field(dmd.predict(dop, 0.0), L)
    eh = pic_mod.field(dmd.predict(dop, 0.5 * dt), L)
    st.last_dmd, st.last_dmd_tables = dop, (e0, eh)

    J = J_small(cfg.two_n)
    k1 = J @ dmd_deim_gradient(U0, Z0, e0, L, op, cfg)
    kh1 = basis_velocity(U0, Z0[:, S], grS.G, cfg.pinv_rtol)
    xi_half = 0.5 * dt * kh1
    U_half = cayley(U0, xi_half)

    def g_of(cols, Ze):
        return dmd_deim_gradient(U_half, Ze, eh[:, cols], L[cols], op, cfg)

    k, ZG, iters, stalled, stall_rel, ok = _fixed_point(Z0, k1, dt, cfg, fixed_iters, g_of)
    st.last_iters, st.last_stalled, st.last_stall_rel = iters, stalled, stall_rel
    if not ok:
        st.window, st.phi_window = saved[0], saved[1]
        st.deim_indices, st.deim_psi, st.deim_builds = saved[2], saved[3], saved[4]
        st.last_status = ENOCONV
        return ENOCONV

    Z1 = Z0 + dt * k
    grG = gradient(U_half, ZG[:, S], L[S], cfg.Nx, cfg.q, cfg.m)
    kh2 = tangent_velocity(U0, xi_half, ZG[:, S], grG.G, cfg.pinv_rtol, Ux=U_half)
    U1 = cayley(U0, dt * kh2)
    st.last_U_half, st.last_Z_new = U_half, Z1.copy()
    if cfg.reorth:
        U1, Z1 = reorthonormalise(U1, Z1)
    st.U, st.Z = U1, Z1
    st.step += 1
    st.last_status = OK
    return OK


def replace_projection(cfg, projection):
    c = RomConfig(**cfg.__dict__)
    c.projection = projection
    return c


def run(st, cfg, steps):
    for _ in range(steps):
        s = prk_step(st, cfg)
        if s != OK:
            return s
        if cfg.rank_auto:
            adapt_rank(st, cfg, 0)
    return OK


# ----------------------------------------------------------------------------
# Rank adaptation (a policy of its own here; the paper defers rank adaptation)
# ----------------------------------------------------------------------------

def rank_indicator(st, cfg, gr=None):
    """eps_perp = ||(I - U U^T) J G||_F / ||G||_F = sqrt(1 - ||g||^2 / ||G||^2)
    at the current state (uses U^T J = J U^T).  parity unpinned as a policy."""
    if gr is None:
        gr = gradient(st.U, st.Z, st.L, cfg.Nx, cfg.q, cfg.m)
    G2 = np.sum(gr.G ** 2)
    g2 = np.sum(gr.g ** 2)
    return float(np.sqrt(max(0.0, 1.0 - g2 / G2))) if G2 > 0 else 0.0, gr


def rank_grow(st, cfg, pairs, gr=None):
    """Append ``pairs`` symplectic pairs: the leading left singular vectors of
    (I - U~ U~^*)(-i G~) (canonical phase), with zero coefficient rows, so
    R = U Z is unchanged."""
    if gr is None:
        gr = gradient(st.U, st.Z, st.L, cfg.Nx, cfg.q, cfg.m)
    N = st.U.shape[0] // 2
    Ut = to_complex_basis(st.U)
    Gt = gr.G[:N] + 1j * gr.G[N:]
    H = -1j * Gt
    H = H - Ut @ (Ut.conj().T @ H)
    Y, s, _ = np.linalg.svd(H, full_matrices=False)
    Y = canonical_phase(Y[:, :pairs])
    Ut = np.concatenate([Ut, Y], axis=1)
    Zt = to_complex_coeff(st.Z)
    Zt = np.concatenate([Zt, np.zeros((pairs, Zt.shape[1]), dtype=complex)], axis=0)
    st.U, st.Z = from_complex_basis(Ut), from_complex_coeff(Zt)
    return s[:pairs]


def rank_shrink(st, new_two_n):
    """Rotate to the SVD of Z~ = Q S W^* (U~ <- U~ Q, Z~ <- Q^* Z~) and drop
    the trailing pairs; returns the dropped singular values."""
    Ut = to_complex_basis(st.U)
    Zt = to_complex_coeff(st.Z)
    Q, s, _ = np.linalg.svd(Zt, full_matrices=True)
    Q = canonical_phase(Q)
    Ut = Ut @ Q
    Zt = Q.conj().T @ Zt
    n = new_two_n // 2
    st.U, st.Z = from_complex_basis(Ut[:, :n]), from_complex_coeff(Zt[:n])
    return s[n:]


def shrink_target(st, cfg):
    """Rank kept by the shrink rule (reading R-4): the pairs whose singular
    value of Z~ is at least rank_tol_down times the largest (at least one)."""
    s = np.linalg.svd(to_complex_coeff(st.Z), compute_uv=False)
    if s.size == 0 or s[0] <= 0.0:
        return st.U.shape[1]
    keep = max(1, int(np.sum(s >= cfg.rank_tol_down * s[0])))
    return 2 * min(keep, st.U.shape[1] // 2)


def adapt_rank(st, cfg, target_two_n=0):
    """Force the rank to ``target_two_n`` (even), or apply the policy when
    target is 0 (reading R-4): grow one pair if eps_perp > rank_tol_up and the
    cap allows; otherwise drop the pairs whose singular value of Z~ falls
    below rank_tol_down times the largest.  Returns (status, new 2n, eps_perp
    or None)."""
    r = st.U.shape[1]
    if target_two_n:
        if target_two_n % 2 or target_two_n <= 0:
            raise ValueError("rank must be a positive even number")
        if target_two_n > cfg.two_n_max:
            return ERANKCAP, r, None
        if target_two_n > r:
            rank_grow(st, cfg, (target_two_n - r) // 2)
        elif target_two_n < r:
            rank_shrink(st, target_two_n)
        cfg.two_n = st.U.shape[1]
        return OK, cfg.two_n, None
    eps, gr = rank_indicator(st, cfg)
    if eps > cfg.rank_tol_up and r < cfg.two_n_max:
        rank_grow(st, cfg, 1, gr)
    else:
        keep = shrink_target(st, cfg)
        if keep < r:
            rank_shrink(st, keep)
    cfg.two_n = st.U.shape[1]
    return OK, cfg.two_n, eps


# ----------------------------------------------------------------------------
# Diagnostics (Sec. 6.1)
# ----------------------------------------------------------------------------

def reconstruct(st):
    N = st.U.shape[0] // 2
    R = st.U @ st.Z
    return R[:N], R[N:]


def diagnostics(st, cfg):
    """Electric energy E(X_r^i) and Hamiltonian H(U Z_i) per parameter."""
    Xr, Vr = reconstruct(st)
    rho, Phi, _ = pic.fields_of(Xr, st.L, cfg.Nx, cfg.q)
    E = pic.electric_energy(Phi, rho, st.L, Xr.shape[0], cfg.m)
    return E, 0.5 * np.sum(Vr * Vr, axis=0) + E


def hamiltonian_split(U_prev, Z_prev, U_half, Z_new, U_tau, Z_tau, L, Nx, q=-1.0, m=1.0):
    """The four Hamiltonians of the splitting eq. error_ham_tot of one step,
    per parameter: H(U_{tau-1} Z_{tau-1}), H(U_{tau-1/2} Z_{tau-1}),
    H(U_{tau-1/2} Z_tau), H(U_tau Z_tau) (rows of a 4 x p array).  With them
    Delta H = |H_3 - H_0| is bounded by |H_3 - H_2| + |H_1 - H_0| (the two
    basis terms) + |H_2 - H_1| (the coefficient term), each taken as the
    2-norm over the parameters.  Z_tau is the coefficient matrix of the
    step before the re-orthonormalisation, which rotates U_tau and Z_tau
    together and leaves U_tau Z_tau unchanged; (U_tau, Z_tau) is the state
    after the step."""
    N = U_prev.shape[0] // 2
    rows = []
    for U, Z in ((U_prev, Z_prev), (U_half, Z_prev), (U_half, Z_new), (U_tau, Z_tau)):
        R = U @ Z
        rows.append(pic.hamiltonian(R[:N], R[N:], L, Nx, q, m))
    return np.array(rows)


def relative_errors(X, V, Xr, Vr):
    """eq. (relative_errors): Frobenius errors of positions and velocities."""
    return (np.linalg.norm(X - Xr) / np.linalg.norm(X),
            np.linalg.norm(V - Vr) / np.linalg.norm(V))
