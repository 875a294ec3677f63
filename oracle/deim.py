"""Oracle: DEIM hyper-reduction of the particle-to-grid term (paper Sec. 4.2.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The nonlinear term N_i = Lambda^0(X_r^i) Phi^i (values of the potential at
the particles) is interpolated on d particle indices.  With the exact
potential (no DMD; a reading) the DEIM gradient of eq. (grHDD) is
  g_i = U_V^T V_r^i + U_X[I,:]^T ( (q/m) e_i[j(X_r^i[I])] * w ),
  w = (P^T Psi)^{-T} Psi^T 1,
since m_p^{-1} M_q = (q/m) 1 and nabla Lambda^0 Phi is the cell field e.
Snapshots: the last T+1 time levels of N_i for a parameter subset of size
p*, the matrix Y = [Y_1 ... Y_p*] of eq. (Ydeim) (N x p*(T+1)); Psi = its
first d left singular vectors; the indices follow the greedy DEIM selection
(Sec. 4.2.2: at step k, the index of the largest interpolation residual of
psi_k on the previous vectors; with the adaptive update of eq.
indices_adaptive_DEIM only the positions of the most rotated basis vectors
are chosen again between full selections).  reading: the subset is evenly
spaced in the
parameter index, i_k = floor(k p / p*), with p* = min(p, max(8,
ceil(two_n_max / (T+1)))) so that p*(T+1) >= d for every rank reached.
"""
from dataclasses import dataclass

import numpy as np

from . import pic


@dataclass
class DeimOp:
    idx: np.ndarray      # d int64 particle indices, in greedy order
    w: np.ndarray        # d weights (P^T Psi)^{-T} Psi^T 1
    Psi: np.ndarray      # N x d


def snapshot_params(p, two_n_max, T):
    """Indices of the DEIM snapshot parameters (see the module docstring)."""
    pstar = min(p, max(8, -(-two_n_max // (T + 1))))
    return np.array([(k * p) // pstar for k in range(pstar)], dtype=np.int64)


def snapshot(Xr, Phi, L):
    """N_i = Lambda^0(X_r^i) Phi^i: (1 - theta) Phi_j + theta Phi_{j+1} per particle."""
    Nx = Phi.shape[0]
    j, th = pic.cell_index(Xr, L, Nx)
    cols = np.arange(Xr.shape[1])[None, :]
    return (1.0 - th) * Phi[j, cols] + th * Phi[(j + 1) % Nx, cols]


def deim_basis(Y, d):
    """First d left singular vectors of Y, each signed so that its
    largest-modulus entry is positive (reading: fixes the SVD sign)."""
    Q, s, _ = np.linalg.svd(Y, full_matrices=False)
    Psi = Q[:, :d].copy()
    for k in range(d):
        i = int(np.argmax(np.abs(Psi[:, k])))
        if Psi[i, k] < 0:
            Psi[:, k] = -Psi[:, k]
    return Psi, s


def greedy_indices(Psi):
    """DEIM greedy selection: l_1 = argmax |psi_1|; for k >= 2 solve
    (P^T Psi_{k-1}) c = P^T psi_k, r = psi_k - Psi_{k-1} c, l_k = argmax |r|
    (ties to the smallest index)."""
    d = Psi.shape[1]
    idx = [int(np.argmax(np.abs(Psi[:, 0])))]
    for k in range(1, d):
        A = Psi[idx, :k]
        c = np.linalg.solve(A, Psi[idx, k])
        r = Psi[:, k] - Psi[:, :k] @ c
        idx.append(int(np.argmax(np.abs(r))))
    return np.array(idx, dtype=np.int64)


def greedy_with_kept(Psi, kept):
    """Greedy DEIM selection in which position k keeps the index kept[k] when
    that is given and not chosen already (the adaptive update of Sec. 4.2.2,
    eq. indices_adaptive_DEIM: the indices not in I* are inherited); every
    other position takes the index of the largest interpolation residual of
    psi_k on the indices chosen before it, ties to the smallest index."""
    d = Psi.shape[1]
    idx = []
    for k in range(d):
        if kept[k] is not None and int(kept[k]) not in idx:
            idx.append(int(kept[k]))
            continue
        if k == 0:
            r = Psi[:, 0]
        else:
            c = np.linalg.solve(Psi[idx, :k], Psi[idx, k])
            r = Psi[:, k] - Psi[:, :k] @ c
        idx.append(int(np.argmax(np.abs(r))))
    return np.array(idx, dtype=np.int64)


def update_positions(Psi_new, Psi_old, n_up):
    """The n_up positions I* of eq. indices_adaptive_DEIM whose basis vectors
    rotated most from the previous DEIM basis.  reading: the printed argmax of
    sum psi_k^new . psi_k^old would pick the least rotated vectors, while the
    text asks for the most rotated ones; the smallest |psi_k^new . psi_k^old|
    are taken (the modulus removes the sign freedom of singular vectors),
    ties to the smaller position."""
    rot = np.abs(np.sum(Psi_new * Psi_old, axis=0))
    order = np.argsort(rot, kind="stable")
    return set(int(k) for k in order[:n_up])


def weights(Psi, idx):
    """w = (P^T Psi)^{-T} Psi^T 1 (the M_q-dependent factor of eq. grHDD)."""
    PtPsi = Psi[idx, :]
    return np.linalg.solve(PtPsi.T, Psi.T @ np.ones(Psi.shape[0]))


def build_operator(Y, d):
    Psi, _ = deim_basis(Y, d)
    idx = greedy_indices(Psi)
    return DeimOp(idx=idx, w=weights(Psi, idx), Psi=Psi)


def update_window(st, cfg, U0, gr0):
    """Append the snapshot at the start of the step; once T+1 snapshots are
    held, return the DEIM operator for this step, else None (the first T
    steps use the Galerkin gradient, Alg. 2)."""
    sub = snapshot_params(st.Z.shape[1], cfg.two_n_max, cfg.deim_window)
    st.window.append(snapshot(gr0.Xr[:, sub], gr0.Phi[:, sub], st.L[sub]))
    T = cfg.deim_window
    if len(st.window) > T + 1:
        st.window.pop(0)
    if len(st.window) < T + 1:
        st.deim_indices = None
        return None
    return build_from_window(st, cfg)


def build_from_window(st, cfg):
    """The DEIM operator of the current snapshot window (T+1 levels)."""
    Y = np.concatenate(st.window, axis=1)
    d = cfg.deim_rows if cfg.deim_rows > 0 else cfg.two_n
    d = min(d, Y.shape[1])
    Psi, _ = deim_basis(Y, d)
    # every deim_update_every-th operator (and the first, and after a change
    # of d) by the full greedy; in between only deim_update_rows positions
    # are chosen again (eq. indices_adaptive_DEIM)
    k_full = max(1, cfg.deim_update_every)
    full = (k_full == 1 or st.deim_builds % k_full == 0 or st.deim_psi is None
            or st.deim_psi.shape[1] != d)
    if full:
        idx = greedy_indices(Psi)
    else:
        upd = update_positions(Psi, st.deim_psi, cfg.deim_update_rows)
        kept = [None if k in upd else st.deim_indices[k] for k in range(d)]
        idx = greedy_with_kept(Psi, kept)
    op = DeimOp(idx=idx, w=weights(Psi, idx), Psi=Psi)
    st.deim_indices = op.idx
    st.deim_psi = Psi
    st.deim_builds += 1
    return op


def restrict(op, cols):
    """The operator is shared by every parameter."""
    return op


def deim_gradient(U, Z, gr, op, cfg):
    """g = U_V^T V_r + U_X[I,:]^T ((q/m) e_{j(X_r[I])} * w)  (eq. grHDD)."""
    N = U.shape[0] // 2
    F_I = gr.G[:N][op.idx, :]
    return U[N:].T @ gr.G[N:] + U[:N][op.idx, :].T @ (F_I * op.w[:, None])
