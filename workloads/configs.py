"""Named synthetic workloads.

Each entry fixes the ensemble family, the particle / parameter / grid sizes,
the time step and the reduced rank.  The parameter ranges follow the
perturbed-Maxwellian initial conditions of the paper's numerical experiments
(weak Landau damping, Sec. 6.2; two-stream instability, Sec. 6.4), widened to
the ranges used here.  Seeds: parameter draws use ``1000*c + 1`` and the
shared particle uniforms ``1000*c + 2`` where ``c`` is the workload number.
"""

WORKLOADS = {
    # tiny plain-FP64 Landau ensemble: every parameter has its own domain
    "landau_tiny": dict(
        number=1, family="landau", N=10_000, p=4, Nx=64, steps=100, dt=0.1,
        two_n=10, two_n_max=10, projection="galerkin",
        ranges=dict(alpha=(0.01, 0.1), k=(0.3, 0.6)), sigma=1.0,
    ),
    # two-stream ensemble, FP64, DEIM with d = 2n, adaptive rank 10 -> 60
    "twostream_deim": dict(
        number=2, family="twostream", N=100_000, p=64, Nx=128, steps=500,
        dt=0.05, two_n=10, two_n_max=60, projection="deim", deim_window=3,
        ranges=dict(alpha=(1e-3, 1e-2), v0=(2.0, 3.0), sigma=(0.1, 0.5)),
        k=0.2,
    ),
    # large two-stream ensemble (mixed-precision target sizes)
    "twostream_mixed": dict(
        number=3, family="twostream", N=1_000_000, p=256, Nx=256, steps=1000,
        dt=0.05, two_n=16, two_n_max=64, projection="galerkin",
        ranges=dict(alpha=(1e-3, 1e-2), v0=(2.0, 3.0), sigma=(0.1, 0.5)),
        k=0.2,
    ),
    # very large two-stream ensemble, Galerkin projection (the library's
    # rank cap is 2n = 60)
    "twostream_large": dict(
        number=5, family="twostream", N=4_000_000, p=1024, Nx=512, steps=2000,
        dt=0.05, two_n=16, two_n_max=60, projection="galerkin", deim_window=3,
        ranges=dict(alpha=(1e-3, 1e-2), v0=(2.0, 3.0), sigma=(0.1, 0.5)),
        k=0.2,
    ),
    # the weak Landau damping experiment of Sec. 6.2 with DMD-DEIM (Alg. 2):
    # eta = (alpha, sigma), k fixed (one domain for every parameter), quiet
    # start, rank 2n = 4, d = 32 DEIM rows with 12 updated per step and a
    # full greedy every 3 steps, window T = 3, p* = 16 subset parameters
    "landau_ld": dict(
        number=6, family="landau", N=50_000, p=300, Nx=32, steps=8000, dt=0.0025,
        two_n=4, two_n_max=4, projection="dmd_deim", deim_window=3, p_star=16,
        deim_rows=32, deim_update_every=3, deim_update_rows=12, loading="hammersley",
        ranges=dict(alpha=(0.03, 0.06), sigma=(0.8, 1.0)), k=0.5,
    ),
    # the two-stream instability experiment of Sec. 6.4: eta = (alpha, sigma),
    # v0 = 3 and k = 0.2 fixed, N = 1.5e5, N_x = 64, dt = 0.0025; the
    # reduced model restarted at t = 30 from the full-order state with
    # larger ranks (DMD-DEIM with T = 3, p* = 8, d = 64, a full greedy every
    # 3rd step)
    "twostream_tsi": dict(
        number=7, family="twostream", N=150_000, p=300, Nx=64, steps=8000, dt=0.0025,
        two_n=8, two_n_max=24, projection="dmd_deim", deim_window=3, p_star=8,
        deim_rows=64, deim_update_every=3, deim_update_rows=24, v0=3.0,
        ranges=dict(alpha=(0.009, 0.011), sigma=(0.98, 1.02)), k=0.2,
        restart_t=30.0,
    ),
}


def workload(name, **overrides):
    """Return a copy of a named workload with some fields replaced."""
    w = dict(WORKLOADS[name])
    w["name"] = name
    w.update(overrides)
    return w
