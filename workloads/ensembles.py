"""Seeded ensembles of initial particle states.

Recipe (quiet-start loading of the paper's numerical experiments, Sec. 6.1,
with the initial distribution f0 = f_v(v) (1 + alpha cos kx)):

* one stream of uniforms per coordinate, ``u_x`` and ``u_v`` of length N,
  SHARED by every parameter of the ensemble (common random numbers, so the
  initial ensemble is smooth in the parameter and hence of low rank);
  either Philox4x32-10 keyed by a seed, or the Hammersley points the paper
  uses ((l + 1/2)/N and the base-2 radical inverse of l);
* position x = F_x^{-1}(u_x) on [0, 2 pi / k) with
  F_x(x) = (x + (alpha/k) sin kx) / L, solved by safeguarded Newton;
* velocity v = F_v^{-1}(u_v) on the truncated interval [-10, 10]: a Gaussian
  of standard deviation sigma (Landau family) or the two-beam mixture
  1/2 [N(+v0, sigma) + N(-v0, sigma)] (two-stream family).

Particle order in memory is generator order (random in x for Philox).
Arrays are returned with shape (N, p), column i belonging to parameter i.
"""
import math

import numpy as np
from scipy.special import ndtr, ndtri

VMAX = 10.0


def philox_uniforms(seed, n, streams=2):
    """``streams`` arrays of n uniforms in the open interval (0, 1)."""
    gen = np.random.Generator(np.random.Philox(key=int(seed)))
    out = []
    for _ in range(streams):
        u = gen.random(n)
        out.append(u + 2.0 ** -54)
    return out


def _radical_inverse_base2(idx):
    idx = idx.astype(np.uint64)
    r = np.zeros(idx.shape, dtype=np.float64)
    f = 0.5
    while np.any(idx):
        r += f * (idx & np.uint64(1)).astype(np.float64)
        idx >>= np.uint64(1)
        f *= 0.5
    return r


def hammersley_uniforms(n):
    """The 2-D Hammersley point set of size n, both coordinates in (0, 1)."""
    idx = np.arange(n)
    ux = (idx + 0.5) / n
    uv = _radical_inverse_base2(idx) + 0.5 / n
    return ux, uv


def draw_parameters(w, seed=None):
    """Draw the ensemble parameters of workload ``w`` uniformly in their ranges.

    Returns a dict of length-p arrays: alpha, k, v0, sigma, and L = 2 pi / k.
    """
    p = w["p"]
    if seed is None:
        seed = 1000 * w["number"] + 1
    gen = np.random.Generator(np.random.Philox(key=int(seed)))
    rng = w["ranges"]

    def uni(name, default):
        if name in rng:
            lo, hi = rng[name]
            return lo + (hi - lo) * gen.random(p)
        return np.full(p, float(default))

    alpha = uni("alpha", 0.0)
    k = uni("k", w.get("k", 0.5))
    v0 = uni("v0", w.get("v0", 0.0))
    sigma = uni("sigma", w.get("sigma", 1.0))
    return dict(alpha=alpha, k=k, v0=v0, sigma=sigma, L=2.0 * math.pi / k)


def parameter_matrix(params):
    """eta as a 4 x p matrix (rows alpha, k, v0, sigma): the parameter
    coordinates of every ensemble member, constant rows included."""
    return np.stack([params["alpha"], params["k"], params["v0"], params["sigma"]]).astype(np.float64)


def _invert_position(u, alpha, k):
    """x in [0, L) with (x + (alpha/k) sin kx)/L = u; all arrays broadcast."""
    L = 2.0 * np.pi / k
    target = u * L
    x = target.copy()
    for _ in range(100):
        g = x + (alpha / k) * np.sin(k * x) - target
        dg = 1.0 + alpha * np.cos(k * x)
        step = g / dg
        x = np.clip(x - step, 0.0, L)
        if np.max(np.abs(step)) <= 1e-15 * np.max(L):
            break
    return x


def _mixture_cdf(v, v0, sigma):
    return 0.5 * (ndtr((v - v0) / sigma) + ndtr((v + v0) / sigma))


def _mixture_pdf(v, v0, sigma):
    a = (v - v0) / sigma
    b = (v + v0) / sigma
    return 0.5 * (np.exp(-0.5 * a * a) + np.exp(-0.5 * b * b)) / (
        sigma * math.sqrt(2.0 * math.pi))


def _invert_velocity(u, v0, sigma):
    """v in [-VMAX, VMAX] inverting the truncated (mixture) Gaussian CDF."""
    lo_mass = _mixture_cdf(-VMAX, v0, sigma)
    hi_mass = _mixture_cdf(VMAX, v0, sigma)
    target = lo_mass + u * (hi_mass - lo_mass)
    if np.all(v0 == 0.0):
        return np.clip(sigma * ndtri(target), -VMAX, VMAX)
    # initial guess from the nearer beam, then Newton inside a shrinking bracket
    left = target < 0.5
    guess_left = -v0 + sigma * ndtri(np.clip(2.0 * target, 1e-300, 1.0))
    guess_right = v0 + sigma * ndtri(np.clip(2.0 * target - 1.0, 1e-300, 1.0 - 1e-16))
    v = np.where(left, guess_left, guess_right)
    v = np.clip(np.nan_to_num(v, nan=0.0), -VMAX, VMAX)
    lo = np.full(v.shape, -VMAX)
    hi = np.full(v.shape, VMAX)
    v0 = np.broadcast_to(v0, v.shape)
    sigma = np.broadcast_to(sigma, v.shape)
    # Newton inside a shrinking bracket, iterating only on unconverged entries
    flat_v = v.reshape(-1).copy()
    act = np.arange(flat_v.size)
    t, a, b = target.reshape(-1), v0.reshape(-1), sigma.reshape(-1)
    lo, hi = lo.reshape(-1), hi.reshape(-1)
    for _ in range(200):
        if act.size == 0:
            break
        vv, ta, aa, bb = flat_v[act], t[act], a[act], b[act]
        f = _mixture_cdf(vv, aa, bb) - ta
        lo[act] = np.where(f < 0, vv, lo[act])
        hi[act] = np.where(f >= 0, vv, hi[act])
        d = _mixture_pdf(vv, aa, bb)
        # a zero or tiny density gives a non-finite step, replaced by bisection
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            vn = vv - f / d
        bad = ~np.isfinite(vn) | (vn <= lo[act]) | (vn >= hi[act])
        vn = np.where(bad, 0.5 * (lo[act] + hi[act]), vn)
        hit = np.abs(f) <= 1e-16
        vn = np.where(hit, vv, vn)
        flat_v[act] = vn
        done = hit | (np.abs(vn - vv) <= 1e-12 * (1.0 + np.abs(vn))) | (hi[act] - lo[act] <= 1e-14)
        act = act[~done]
    return flat_v.reshape(v.shape)


def load_particles(params, ux, uv, family):
    """Initial positions and velocities, arrays of shape (N, p)."""
    alpha = params["alpha"][None, :]
    k = params["k"][None, :]
    X = _invert_position(ux[:, None] * np.ones_like(alpha), alpha, k)
    if family == "landau":
        v0 = np.zeros_like(params["sigma"])[None, :]
    else:
        v0 = params["v0"][None, :]
    sigma = params["sigma"][None, :]
    V = _invert_velocity(uv[:, None] * np.ones_like(sigma), v0 * np.ones_like(sigma),
                         sigma * np.ones_like(v0))
    return np.asfortranarray(X), np.asfortranarray(V)


def particle_uniforms(w, seed=None):
    """The N shared uniforms of workload w: the Hammersley point set (quiet
    start, Sec. 6.1) in a seeded random particle order when the workload asks
    for it, else Philox streams."""
    if seed is None:
        seed = 1000 * w["number"] + 2
    if w.get("loading") == "hammersley":
        ux, uv = hammersley_uniforms(w["N"])
        perm = np.random.Generator(np.random.Philox(key=int(seed))).permutation(w["N"])
        return ux[perm], uv[perm]
    return philox_uniforms(seed, w["N"])


def make_ensemble(w, loading="philox", param_seed=None, particle_seed=None):
    """Parameters and initial particle states for workload ``w``.

    Returns dict(params=..., L=(p,), X0=(N, p), V0=(N, p), eta=(4, p)).
    """
    params = draw_parameters(w, param_seed)
    if loading == "hammersley":
        ux, uv = hammersley_uniforms(w["N"])
    else:
        if particle_seed is None:
            particle_seed = 1000 * w["number"] + 2
        ux, uv = philox_uniforms(particle_seed, w["N"])
    X0, V0 = load_particles(params, ux, uv, w["family"])
    return dict(params=params, L=params["L"].copy(), X0=X0, V0=V0, eta=parameter_matrix(params))
