"""Oracle: parameter subsampling and DMD of the electric potential
(paper Sec. 4.1 and Sec. 4.2.1, Alg. 1), the pieces of the DMD-DEIM reduced
model of Sec. 4.3 (eq. grHDD, eq. UZredhyp) and Alg. 2.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings (the paper leaves these open):
* eq. pSampl: the inner minimum runs over the parameters already selected
  (over all of Gamma_h it would be zero); the first pick is the column of
  Z^0 of largest norm; ties go to the smaller index.  The subset is fixed at
  t = 0 (as in Sec. 4.1).
* Alg. 1, step 1: singular values above tol * sigma_1 are kept (relative
  tolerance; tol = 1e-5 in Sec. 6.1).
* eq. DMD_approx_potential_subset: the time origin is t_{tau-1}, so
  Pi_i = Theta^+ Phi^i_{tau-1}; the prediction is the real part of
  Theta (Pi_i * exp(omega (t - t_{tau-1}))) with the principal logarithm.
* Gaussian radial basis interpolation of Pi_i over the parameters outside
  the subset: kernel exp(-(r / eps)^2) on parameters scaled to [0, 1] per
  coordinate by the ensemble's range, eps = the median distance between
  pairs of subset parameters, no polynomial term.
"""
from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------------------
# Parameter subsampling (Sec. 4.1, eq. pSampl)
# ----------------------------------------------------------------------------

def select_subset(Z0, pstar):
    """Greedy farthest-point choice of p* columns of Z^0 (eq. pSampl):
    first argmax ||Z_i||, then repeatedly the column whose distance to the
    nearest chosen column is largest.  Returns the indices in pick order."""
    p = Z0.shape[1]
    pstar = min(pstar, p)
    norms = np.linalg.norm(Z0, axis=0)
    chosen = [int(np.argmax(norms))]
    dmin = np.linalg.norm(Z0 - Z0[:, [chosen[0]]], axis=0)
    while len(chosen) < pstar:
        cand = dmin.copy()
        cand[chosen] = -1.0
        i = int(np.argmax(cand))
        chosen.append(i)
        dmin = np.minimum(dmin, np.linalg.norm(Z0 - Z0[:, [i]], axis=0))
    return np.array(chosen, dtype=np.int64)


# ----------------------------------------------------------------------------
# DMD (Alg. 1) on the sliding parametric window (eq. DMD_potential_Y_time,
# eq. DMD_potential_Y_time_parameter)
# ----------------------------------------------------------------------------

def window_matrices(levels):
    """levels: the T+1 potentials Phi_{tau-T-1}, ..., Phi_{tau-1}, each N_x x p*
    (columns: the subset parameters).  Returns Y, Y' (N_x x p*T): for each
    parameter the first T levels, resp. the last T, parameter-major."""
    T = len(levels) - 1
    pst = levels[0].shape[1]
    Y = np.concatenate([np.stack([levels[t][:, i] for t in range(T)], axis=1)
                        for i in range(pst)], axis=1)
    Yp = np.concatenate([np.stack([levels[t + 1][:, i] for t in range(T)], axis=1)
                         for i in range(pst)], axis=1)
    return Y, Yp


def dmd(Y, Yp, tol):
    """Alg. 1: truncated SVD Y = U S V^T (s_j > tol s_1), A_tol = U^T Y' V S^-1,
    A_tol W = W Lambda, Theta = Y' V S^-1 W.  Returns (Lambda, Theta, r)."""
    Uy, s, Vt = np.linalg.svd(Y, full_matrices=False)
    r = int(np.sum(s > tol * s[0]))
    Ur, sr, Vr = Uy[:, :r], s[:r], Vt[:r].T
    B = Yp @ Vr / sr[None, :]
    A = Ur.T @ B
    lam, W = np.linalg.eig(A)
    return lam, B @ W, r


# ----------------------------------------------------------------------------
# Gaussian radial basis interpolation of the DMD coordinates
# ----------------------------------------------------------------------------

def scaled_parameters(eta):
    """eta: dim x p.  Each coordinate mapped to [0, 1] by the ensemble range
    (a coordinate with zero range is left at 0)."""
    eta = np.asarray(eta, dtype=np.float64)
    lo = eta.min(axis=1, keepdims=True)
    span = eta.max(axis=1, keepdims=True) - lo
    span[span == 0] = 1.0
    return (eta - lo) / span


def rbf_width(xs):
    """Median distance over the pairs of nodes (columns of xs)."""
    k = xs.shape[1]
    d = [np.linalg.norm(xs[:, a] - xs[:, b]) for a in range(k) for b in range(a + 1, k)]
    return float(np.median(d)) if d else 1.0


def rbf_interpolate(xs, values, xq, eps):
    """Gaussian RBF interpolant through (xs[:, k], values[:, k]) evaluated at
    the columns of xq: K a = values^T with K_kl = exp(-(|x_k - x_l| / eps)^2)."""
    def kern(a, b):
        d = np.linalg.norm(a[:, :, None] - b[:, None, :], axis=0)
        return np.exp(-(d / eps) ** 2)
    coef = np.linalg.solve(kern(xs, xs), values.T)
    return (kern(xq, xs) @ coef).T


# ----------------------------------------------------------------------------
# The DMD operator of one step and the predicted potential
# ----------------------------------------------------------------------------

@dataclass
class DmdOp:
    lam: np.ndarray      # r DMD eigenvalues
    Theta: np.ndarray    # N_x x r DMD modes
    Pi: np.ndarray       # r x p coordinates of every parameter
    dt: float
    r: int


def build_operator(levels, subset, eta, dt, tol):
    """DMD of the last T+1 subset potentials; Pi_i = Theta^+ Phi^i_{tau-1} on
    the subset, radial basis interpolation elsewhere (Sec. 4.2.1)."""
    Y, Yp = window_matrices(levels)
    lam, Theta, r = dmd(Y, Yp, tol)
    Pi_s = np.linalg.pinv(Theta) @ levels[-1]
    p = eta.shape[1]
    xs_all = scaled_parameters(eta)
    xs = xs_all[:, subset]
    Pi = np.empty((r, p), dtype=np.complex128)
    rest = np.setdiff1d(np.arange(p), subset)
    Pi[:, subset] = Pi_s
    if rest.size:
        eps = rbf_width(xs)
        Pi[:, rest] = (rbf_interpolate(xs, Pi_s.real, xs_all[:, rest], eps)
                       + 1j * rbf_interpolate(xs, Pi_s.imag, xs_all[:, rest], eps))
    return DmdOp(lam=lam, Theta=Theta, Pi=Pi, dt=dt, r=r)


def predict(op, t_off):
    """Phi_DMD at t = t_{tau-1} + t_off for every parameter (N_x x p):
    Re(Theta (Pi * exp(omega t_off))), omega = log(Lambda) / dt."""
    if t_off == 0.0:
        growth = np.ones(op.r, dtype=np.complex128)
    else:
        growth = np.exp(np.log(op.lam.astype(np.complex128)) / op.dt * t_off)
    return np.real(op.Theta @ (op.Pi * growth[:, None]))
