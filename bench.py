"""Benchmark: particle-parameter steps per second of the reduced model (ROM)
and of the full-order PIC model (FOM) on one MI355X, on a synthetic
two-stream ensemble (default: the large ensemble N = 4,000,000 particles,
p = 1024 parameters, Nx = 512 cells, dt = 0.05, reduced rank 2n from 16 with
cap 60, DEIM with d = 2n; `--workload twostream_deim` runs N = 100,000,
p = 64, Nx = 128, 2n from 10).  The initial ensemble is formed on the device
from its parameters and shared uniforms.

Prints ONE JSON line.  `value` is the ROM throughput N * p * steps / time of
the timed steps (inputs resident in HBM); by default two warm-up steps and 25
timed steps (steps 3 to 27, the averaging window of the paper's timings).

Beside it: the same metric for the FOM on the same ensemble and their ratio
at matched error (relative position / velocity errors of eq. relative_errors
and the largest relative electric-energy error of the ROM against the FOM,
over the same steps from t = 0, with the complex-SVD target error of
eq. relative_errors_complex_SVD); per-step latency percentiles; `roofline`
for the dominant kernel on the caller's stream from the algorithmic work of
its operation (HIP events on the library's stream); `critical_path` for the
DEIM chain on the second stream; `cpu_baseline` times the FP64 oracle on a
bounded sample of the same workload, on one host core and on all of them.
`dmd_deim` runs the paper's full method (Alg. 2: DMD of the potential, DEIM,
parameter subset) on its weak Landau damping ensemble (Sec. 6.2) with the
same fields, and `serve` a Poisson-arrival mix of requests.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12        # B/s, MI355X HBM3E
PEAK_FP64 = 78.6e12      # flop/s, MI355X FP64 vector (= FP64 matrix) peak

# timing families that hold one kernel each on the caller's stream
SINGLE_KERNEL = {
    "deposit": "deposit_rom_mfma_kernel (reconstruct on FP64 MFMA + cell + LDS histogram)",
    "gather": "gather_project_mfma_kernel (reconstruct + field gather + g = U^* F on FP64 MFMA)",
    "gather_xi": "gather_xi_mfma_kernel (reconstruct + field gather + xi = -i h F Q + U M + conj(U) N on FP64 MFMA)",
}

# HBM bytes per launch of the dominant kernel, measured with two counter
# passes (FETCH_SIZE, WRITE_SIZE) calibrated on a plain device copy; valid
# only for the kernel sources it was taken on (their SHA-256 in the profile)
_CSRC = os.path.join(ROOT, "paper_2201_05555_amd", "csrc")
TRAFFIC_PROFILE = {
    ("gather", "twostream_large"): (
        os.path.join(ROOT, "profiles", "gather_project_mfma_kernel_twostream_large_N4e6_p1024_hbm_traffic.md"),
        [os.path.join(_CSRC, "rom_kernels.hip"), os.path.join(_CSRC, "common.h")]),
    ("deposit", "twostream_deim"): (
        os.path.join(ROOT, "profiles", "deposit_rom_mfma_kernel_twostream_deim_N1e5_p64_hbm_traffic.md"),
        [os.path.join(_CSRC, "pic_kernels.hip"), os.path.join(_CSRC, "common.h")]),
}


def _progress(msg):
    """One line on stderr as each part of the run ends (the JSON line stays
    the only output on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _leg(name, fn):
    """Run an optional part of the benchmark; a failure of the library in it
    (for example a fixed point that does not converge) is reported in its
    place instead of ending the run, so the headline line is still printed."""
    try:
        out = fn()
        _progress(f"{name} done")
        return out
    except Exception as e:  # reported, not hidden: the leg's entry says what failed
        _progress(f"{name} failed: {type(e).__name__}: {e}")
        return {"failed": f"{type(e).__name__}: {e}"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="twostream_large")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-matched", action="store_true", help="skip the matched-error pass")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving mix")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-step-scale", type=float, default=0.25)
    ap.add_argument("--serve-gap", type=float, default=1.0, help="mean inter-arrival (s)")
    ap.add_argument("--no-dmd", action="store_true", help="skip the DMD-DEIM leg")
    ap.add_argument("--no-restart", action="store_true",
                    help="skip the paper-workload legs: the two-stream restart at t = 30 "
                         "(Sec. 6.4), the local-rank study (Sec. 6.1) and the Hamiltonian "
                         "splitting (Sec. 6.2)")
    ap.add_argument("--restart-only", action="store_true",
                    help="run only the paper-workload legs and print their results")
    ap.add_argument("--dmd-only", action="store_true",
                    help="run only the DMD-DEIM leg (at p = 1024, no sweep) and print its line")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    return ap.parse_args()


def roofline_of(ms, flops, nbytes, launches):
    """Binding roofline of a kernel family from the algorithmic work of its
    operation and its measured time: the resource with the larger lower
    bound on time (FP64 ALU against 78.6 TFLOP/s, or HBM against 8 TB/s)."""
    t = ms * 1e-3
    if t <= 0:
        return None
    t_alu = flops / PEAK_FP64
    t_hbm = nbytes / PEAK_HBM
    base = {"avg_launch_us": 1e3 * ms / max(launches, 1), "launches": launches,
            "algorithmic_flops_per_launch": flops / max(launches, 1),
            "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
            "frac_hbm": (nbytes / t) / PEAK_HBM, "frac_alu": (flops / t) / PEAK_FP64}
    if t_hbm >= t_alu:
        ach = nbytes / t / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": ach / (PEAK_HBM / 1e9), "traffic": None, **base}
    ach = flops / t / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": ach / (PEAK_FP64 / 1e12), "traffic": None, **base}


def measured_traffic(family, workload):
    """Counter-measured HBM bytes per launch of a kernel family, or None when
    the profile is missing or a kernel source has changed since it was taken."""
    import hashlib
    try:
        path, sources = TRAFFIC_PROFILE[(family, workload)]
        text = open(path).read()
        shas = {os.path.relpath(f, ROOT): hashlib.sha256(open(f, "rb").read()).hexdigest()
                for f in sources}
    except (OSError, KeyError):
        return None
    val = None
    seen = {}
    for line in text.splitlines():
        if line.startswith("traffic-bytes-per-launch:"):
            val = float(line.split(":")[1])
        elif line.startswith("source-sha256 ("):
            name = line[len("source-sha256 ("):line.index(")")]
            seen[name] = line.split(":")[-1].strip()
    return val if (val is not None and seen == shas) else None


def _oracle_rate(w, ens, seconds, threads):
    """The oracle's reduced step (+ rank policy) on its first p_sub
    parameters and first N_sub particles, same rank and time step, with
    `threads` BLAS threads."""
    import numpy as np
    from oracle import rom
    from threadpoolctl import threadpool_limits
    p_sub = min(8, w["p"], ens["X0"].shape[1])
    N_sub = min(w["N"], ens["X0"].shape[0])
    X0 = np.asfortranarray(ens["X0"][:N_sub, :p_sub])
    V0 = np.asfortranarray(ens["V0"][:N_sub, :p_sub])
    cfg = rom.RomConfig(N=N_sub, p=p_sub, Nx=w["Nx"], two_n=w["two_n"], dt=w["dt"],
                        fp_tol=1e-9, two_n_max=w["two_n_max"],
                        projection=w.get("projection", "galerkin"),
                        deim_window=w.get("deim_window", 3),
                        rank_auto=w["two_n_max"] > w["two_n"], rank_tol_up=1e-2)
    with threadpool_limits(limits=threads):
        st = rom.init_state(X0, V0, ens["L"][:p_sub], cfg)
        steps = 0
        t0 = time.perf_counter()
        while True:
            rom.prk_step(st, cfg)
            if cfg.rank_auto:
                rom.adapt_rank(st, cfg, 0)
            steps += 1
            el = time.perf_counter() - t0
            if el > seconds or steps >= 50:
                break
    return N_sub * p_sub * steps / el, steps, el, p_sub, st.U.shape[1], N_sub


def cpu_baseline(w, ens, seconds):
    """The oracle (not tuned) on the host: one core, then every core."""
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    v1, s1, e1, p_sub, r1, N_sub = _oracle_rate(w, ens, seconds, 1)
    va, sa, ea, _, ra, _ = _oracle_rate(w, ens, seconds, ncpu)
    return {"value": va, "unit": "particle-param-steps/s", "cores": ncpu, "kind": "oracle",
            "single_core_value": v1,
            "sample": f"oracle prk_step (+ rank policy) on the first {p_sub} of {w['p']} "
                      f"parameters and the first {N_sub} of {w['N']} particles, "
                      f"2n={w['two_n']}->{ra}, "
                      f"{w.get('projection', 'galerkin')}: {sa} steps in {ea:.1f} s on {ncpu} "
                      f"threads, {s1} steps in {e1:.1f} s on 1 thread; the reduced step's "
                      f"work is about linear in N and in p, so the rate is per "
                      f"particle-parameter"}


def _frob_rel_err(torch, A, B):
    """||A - B||_F / ||A||_F for (p, N) device arrays, a parameter at a time
    (no N x p temporary)."""
    num = den = 0.0
    for i in range(A.shape[0]):
        num += float(torch.sum((A[i] - B[i]) ** 2))
        den += float(torch.sum(A[i] ** 2))
    return (num / den) ** 0.5


def matched_error(binding, torch, w, src, cfg, steps):
    """ROM and FOM over the same steps from t = 0 on the same ensemble:
    eq. relative_errors at the last step, the complex-SVD target error of
    eq. relative_errors_complex_SVD (the truncated complex SVD of the FOM
    state at that step, at the ROM's final rank), and the largest relative
    electric-energy error max_{t, i} |E_rom - E_fom| / max_t E_fom.  The
    models run one after the other (the FOM state of a large ensemble and
    the reduced model's workspace are each tens of GB)."""
    import numpy as np
    N, p, Nx = w["N"], w["p"], w["Nx"]
    fom_h = binding.Fom(N, p, Nx, w["dt"], None, None, None, **src)
    E_f = []
    for _ in range(steps):
        fom_h.step(1)
        E_f.append(fom_h.diagnostics()[0].cpu().numpy())
    Xf, Vf = fom_h.get_state()
    fom_h.close()
    del fom_h
    torch.cuda.empty_cache()
    rom_h = binding.Rom(cfg, None, None, None, **src)
    E_r = []
    for _ in range(steps):
        rom_h.step(1)
        E_r.append(rom_h.diagnostics()[0].cpu().numpy())
    E_r, E_f = np.array(E_r), np.array(E_f)
    e_rel_E = float(np.max(np.abs(E_r - E_f) / np.maximum(np.max(np.abs(E_f), axis=0), 1e-300)))
    Xr, Vr = rom_h.reconstruct()
    two_n = rom_h.two_n
    rom_h.close()
    del rom_h
    ex = _frob_rel_err(torch, Xf, Xr)
    ev = _frob_rel_err(torch, Vf, Vr)
    del Xr, Vr
    torch.cuda.empty_cache()
    # target: the truncated complex SVD of the FOM state (rom_init computes it)
    tcfg = binding.make_config(N, p, Nx, two_n, dt=w["dt"])
    t_h = binding.Rom(tcfg, src["params"]["L"], Xf, Vf)
    Xt, Vt = t_h.reconstruct()
    t_h.close()
    del t_h
    tx = _frob_rel_err(torch, Xf, Xt)
    tv = _frob_rel_err(torch, Vf, Vt)
    del Xt, Vt, Xf, Vf
    torch.cuda.empty_cache()
    return {"steps_from_t0": steps, "eps_rel_X": ex, "eps_rel_V": ev,
            "target_eps_rel_X": tx, "target_eps_rel_V": tv, "rank_2n": two_n,
            "max_rel_energy_error": e_rel_E,
            "definition": "eq. relative_errors (Frobenius over all particles and parameters) "
                          "at the last step; target = truncated complex SVD of the FOM state; "
                          "energy error max over steps and parameters of |E_rom - E_fom| / "
                          "max_t E_fom"}


# Stagnation floor of the fixed point in the DMD-DEIM leg: with DEIM the
# reduced gradient of a column jumps when one of its d sampled particles
# (each carrying a weight of order N/d) crosses a node, so a column can
# settle into a cycle at the size of that jump; with the default floor of
# 1e-3 one column of 1024 occasionally ended a step with ENOCONV.  The leg
# reports the floor it uses.
DMD_STALL_TOL = 1e-2
# The floor for the DMD-DEIM runs of the restart leg (ranks 8 to 24 of the
# two-stream ensemble at t = 30, d = 64 sampled rows): single columns cycle
# at a few per cent there (with a floor of 1e-2 the 2n = 12 run ended with
# ENOCONV after about 100 steps; with d = 32 cycles of 10-20 % ended every
# run from 2n = 12 on within 50-520 steps); the largest update accepted is
# reported.
RESTART_DMD_STALL_TOL = 1e-1


def dmd_deim_leg(binding, torch, steps, warmup, p=1024, p_sweep=(300, 1024, 2048)):
    """The DMD-DEIM reduced model (Alg. 2) on the weak Landau damping
    ensemble of Sec. 6.2 (eta = (alpha, sigma), k = 0.5, N = 5e4, N_x = 32,
    dt = 0.0025, quiet start; p* = 16 subset parameters, window T = 3, d = 32
    DEIM rows, 12 of them chosen again per step with a full greedy every 3rd)
    at p parameters and rank 2n = 6 (the quiet-start ensemble has complex
    rank 3 at t = 0, the density perturbation its smallest part; the paper's
    2n = 4 drops it): throughput of the reduced and full-order steps, their
    ratio, the matched error over the same steps from t = 0, and the step
    time over a range of p (the reduced step's cost per parameter does not
    depend on N)."""
    import numpy as np
    from workloads import workload, particle_uniforms
    from workloads.ensembles import draw_parameters

    def setup(pp):
        w = workload("landau_ld", p=pp)
        params = draw_parameters(w)
        ux, uv = particle_uniforms(w)
        src = dict(family=w["family"], params=params, ux=ux, uv=uv)
        cfg = binding.make_config(w["N"], pp, w["Nx"], 6, two_n_max=6, dt=w["dt"],
                                  projection="dmd_deim", deim_window=w["deim_window"],
                                  p_star=w["p_star"], deim_rows=w["deim_rows"],
                                  deim_update_every=w["deim_update_every"],
                                  deim_update_rows=w["deim_update_rows"], fp_tol=1e-9,
                                  fp_stall_tol=DMD_STALL_TOL)
        return w, src, cfg

    def rates(w, src, cfg, with_events=False):
        r = binding.Rom(cfg, None, None, None, **src)
        r.step(warmup + w["deim_window"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = r.step(steps)
        torch.cuda.synchronize()
        t_rom = time.perf_counter() - t0
        rank = r.dmd_state()[1]
        fams = None
        if with_events:
            binding.set_timing(True)
            for fam in binding.FAMILIES:
                binding.kernel_ms(fam)
            r.step(steps)
            torch.cuda.synchronize()
            fams = {f: binding.kernel_ms(f)[0] / steps for f in binding.FAMILIES}
            binding.set_timing(False)
        r.close()
        del r
        torch.cuda.empty_cache()
        f = binding.Fom(w["N"], cfg.p, w["Nx"], w["dt"], None, None, None, **src)
        f.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.step(steps)
        torch.cuda.synchronize()
        t_fom = time.perf_counter() - t0
        f.close()
        del f
        torch.cuda.empty_cache()
        return t_rom, t_fom, info, rank, fams

    w, src, cfg = setup(p)
    t_rom, t_fom, info, rank, fams = rates(w, src, cfg, with_events=True)
    pp = w["N"] * p
    out = {"workload": "landau_ld", "N": w["N"], "p": p, "Nx": w["Nx"], "dt": w["dt"],
           "two_n": 6, "p_star": w["p_star"], "deim_rows": w["deim_rows"],
           "deim_window": w["deim_window"], "deim_update_every": w["deim_update_every"],
           "deim_update_rows": w["deim_update_rows"], "loading": "hammersley (quiet start)",
           "fp_stall_tol": DMD_STALL_TOL,
           "value": pp * steps / t_rom, "unit": "particle-param-steps/s",
           "ms_per_step": 1e3 * t_rom / steps, "mean_fp_iters": info["iters_total"] / steps,
           "stalled_columns": info["stalled_total"], "dmd_rank": rank,
           "fom": {"value": pp * steps / t_fom, "ms_per_step": 1e3 * t_fom / steps},
           "rom_over_fom": t_fom / t_rom,
           "kernel_families_ms_per_step": fams}
    out["matched_error"] = matched_error(binding, torch, w, src, cfg,
                                         warmup + w["deim_window"] + steps)
    sweep = []
    for pv in p_sweep:
        if pv == p:
            sweep.append({"p": pv, "rom_ms": out["ms_per_step"],
                          "fom_ms": out["fom"]["ms_per_step"], "rom_over_fom": out["rom_over_fom"]})
            continue
        def point(pv=pv):
            w2, src2, cfg2 = setup(pv)
            tr, tf, _, _, _ = rates(w2, src2, cfg2)
            return {"p": pv, "rom_ms": 1e3 * tr / steps, "fom_ms": 1e3 * tf / steps,
                    "rom_over_fom": tf / tr}
        res = _leg(f"DMD-DEIM sweep p = {pv}", point)
        sweep.append(res if "failed" not in res else dict(res, p=pv))
    out["p_sweep"] = sweep
    return out


def serve_bench(binding, torch, n_req, step_scale, slots, pool_gb, mean_gap_s, seed=4001):
    """A serving mix after the request recipe of the serving configuration:
    Poisson arrivals; each request a Landau or two-stream ensemble (1/2 each,
    eta drawn in that family's box), p uniform on 1..128, N in {1e5, 1e6},
    initial rank 2n in {8, 16, 32, 60} (60: the library's cap, in place of
    64), the step count uniform on 200..1000 times step_scale, Galerkin,
    rank adaptation on (cap 60).  Reported: latency (results ready minus
    arrival) p50 / p99, throughput over the makespan, peak pool occupancy."""
    import numpy as np
    from workloads import workload
    from workloads.ensembles import draw_parameters, philox_uniforms
    rng = np.random.default_rng(seed)
    reqs = []
    for j in range(n_req):
        fam = "landau_tiny" if rng.random() < 0.5 else "twostream_deim"
        p = int(rng.integers(1, 129))
        N = int(rng.choice([100_000, 1_000_000]))
        Nx = 128 if N == 100_000 else 256
        two_n = int(rng.choice([8, 16, 32, 60]))
        steps = max(1, int(round(int(rng.integers(200, 1001)) * step_scale)))
        w = workload(fam, p=p, N=N, Nx=Nx)
        params = draw_parameters(w, seed=seed + 10 * j)
        ux, uv = philox_uniforms(seed + 10 * j + 1, N)
        cfg = binding.make_config(N, p, Nx, two_n, two_n_max=60, dt=0.05, fp_tol=1e-9,
                                  rank_auto=True, rank_tol_up=1e-2)
        reqs.append((cfg, w["family"], params, ux, uv, steps))
    gaps = rng.exponential(mean_gap_s, size=n_req)
    srv = binding.Server(slots, int(pool_gb * (1 << 30)))
    ids = []
    t0 = time.perf_counter()
    t_next = 0.0
    for (cfg, fam, params, ux, uv, steps), g in zip(reqs, gaps):
        t_next += g
        dt = t_next - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(srv.submit(cfg, fam, params, ux, uv, steps))
    peak = srv.drain()
    infos = [srv.info(i) for i in ids]
    srv.close()
    bad = [i for i in infos if i["status"] != 0]
    lat = np.array([i["t_finish"] - i["t_arrival"] for i in infos])
    span = max(i["t_finish"] for i in infos) - min(i["t_arrival"] for i in infos)
    pp = sum(i["pp_steps"] for i in infos if i["status"] == 0)
    return {"requests": n_req, "failed": len(bad),
            "failed_status": [i["status"] for i in bad], "slots": slots, "pool_gb": pool_gb,
            "mean_interarrival_s": mean_gap_s, "step_scale": step_scale,
            "latency_s": {"p50": float(np.percentile(lat, 50)),
                          "p99": float(np.percentile(lat, 99)), "max": float(lat.max())},
            "throughput_pp_steps_per_s": pp / span, "makespan_s": span,
            "peak_pool_gb": peak / (1 << 30),
            "mix": "Landau / two-stream 1:1, p ~ U{1..128}, N in {1e5, 1e6}, 2n in "
                   "{8, 16, 32, 60}, steps ~ U{200..1000} x step_scale, Galerkin, "
                   "rank adaptation to 60, Poisson arrivals"}


def restart_leg(binding, torch, ranks=(8, 12, 18, 24), steps=2000, every=500):
    """The restart of Sec. 6.4: the two-stream instability ensemble (eta =
    (alpha, sigma), N = 1.5e5, p = 300, N_x = 64, dt = 0.0025) is run with the
    full-order model to t = 30, where a rank 2n <= 8 no longer follows the
    dynamics; the reduced model is started again there from the truncated
    complex SVD of the full-order state at each rank 2n in ``ranks``, with
    the Galerkin projection and with DMD-DEIM (T = 3, p* = 8, d = 64 rows, a
    full greedy every 3rd step), and run ``steps`` further steps beside the
    full-order
    model.  Reported every ``every`` steps: eq. relative_errors of each run
    and the complex-SVD target error of eq. relative_errors_complex_SVD at
    that rank; a run that fails reports its status."""
    from workloads import workload, particle_uniforms
    from workloads.ensembles import draw_parameters, parameter_matrix
    w = workload("twostream_tsi")
    N, p, Nx, dt = w["N"], w["p"], w["Nx"], w["dt"]
    params = draw_parameters(w)
    ux, uv = particle_uniforms(w)
    n0 = int(round(w["restart_t"] / dt))
    f = binding.Fom(N, p, Nx, dt, None, None, None, family=w["family"], params=params, ux=ux,
                    uv=uv)
    f.step(n0)
    X0, V0 = f.get_state()
    cps = []
    for _ in range(steps // every):
        f.step(every)
        cps.append(f.get_state())
    f.close()
    del f
    L = params["L"]
    eta = parameter_matrix(params)
    times = [w["restart_t"] + every * dt * (c + 1) for c in range(len(cps))]
    out = {"workload": "twostream_tsi", "N": N, "p": p, "Nx": Nx, "dt": dt,
           "t_restart": w["restart_t"], "times": times, "ranks": list(ranks),
           "p_star": w["p_star"], "deim_window": w["deim_window"], "deim_rows": w["deim_rows"],
           "deim_update_every": w["deim_update_every"],
           "deim_update_rows": w["deim_update_rows"]}

    def target(tn):
        ex, ev = [], []
        for Xc, Vc in [(X0, V0)] + cps:
            t_h = binding.Rom(binding.make_config(N, p, Nx, tn, dt=dt), L, Xc, Vc)
            Xt, Vt = t_h.reconstruct()
            t_h.close()
            ex.append(_frob_rel_err(torch, Xc, Xt))
            ev.append(_frob_rel_err(torch, Vc, Vt))
            del Xt, Vt
        return {"eps_rel_X": ex, "eps_rel_V": ev, "note": "first entry at t_restart"}

    def run(proj, tn):
        cfg = binding.make_config(N, p, Nx, tn, two_n_max=tn, dt=dt, projection=proj,
                                  deim_window=w["deim_window"], p_star=w["p_star"],
                                  deim_rows=w["deim_rows"],
                                  deim_update_every=w["deim_update_every"],
                                  deim_update_rows=w["deim_update_rows"], fp_tol=1e-9,
                                  fp_stall_tol=RESTART_DMD_STALL_TOL if proj == "dmd_deim"
                                  else 1e-3)
        r = binding.Rom(cfg, L, X0, V0)
        if proj == "dmd_deim":
            r.set_parameters(eta)
        ex, ev, t_steps, iters, stalled, srel, fail = [], [], 0.0, 0, 0, 0.0, None
        try:
            for Xc, Vc in cps:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = r.step_status(every)
                torch.cuda.synchronize()
                if st == 0:
                    t_steps += time.perf_counter() - t0
                    iters += info["iters_total"]
                stalled += info["stalled_total"]
                srel = max(srel, info["stall_rel"])
                if st != 0:
                    # the state is the one before the failing step
                    fail = {"status": binding.lib().symrom_status_string(st).decode(),
                            "after_steps": r.get_state()[2],
                            "worst_rel": info["worst_rel"], "unconverged": info["unconverged"]}
                    break
                Xm, Vm = r.reconstruct()
                ex.append(_frob_rel_err(torch, Xc, Xm))
                ev.append(_frob_rel_err(torch, Vc, Vm))
                del Xm, Vm
        finally:
            r.close()
        n = max(1, every * len(ex))
        out = {"eps_rel_X": ex, "eps_rel_V": ev, "ms_per_step": 1e3 * t_steps / n,
               "mean_fp_iters": iters / n, "stalled_columns": stalled,
               "max_stall_accepted_update": srel, "fp_stall_tol": cfg.fp_stall_tol}
        if fail:
            out["failed_step"] = fail
        return out

    out["target"] = {str(tn): _leg(f"restart target 2n = {tn}", lambda tn=tn: target(tn))
                     for tn in ranks}
    for proj in ("galerkin", "dmd_deim"):
        out[proj] = {str(tn): _leg(f"restart {proj} 2n = {tn}", lambda tn=tn: run(proj, tn))
                     for tn in ranks}
    del X0, V0, cps
    torch.cuda.empty_cache()
    return out


def local_rank_leg(binding, torch, p=64, every=400, tols=(1e-3, 1e-4, 1e-5)):
    """The local-rank study of Sec. 6.1 (eq. local_snapshots) on the
    full-order solutions of the weak Landau damping (Sec. 6.2) and the
    two-stream instability (Sec. 6.4) ensembles at p parameters, over the
    paper's interval (0, 20]: every ``every`` steps the singular values of
    S_X^tau = [X^1 ... X^p] and of S_V^tau, found by the library's
    initialisation (rom_init of C0 = X + 0 i, all p values for p <= 64), and
    the numerical ranks at each tolerance (values above tol * sigma_1).
    Positions are the unwrapped ones the reduced model represents."""
    import numpy as np
    from workloads import workload, particle_uniforms
    from workloads.ensembles import draw_parameters
    out = {"p": p, "every_steps": every, "tolerances": list(tols),
           "definition": "number of singular values of S_X^tau (S_V^tau) above tol * sigma_1"}
    for name in ("landau_ld", "twostream_tsi"):
        w = workload(name, p=p)
        N, Nx, dt = w["N"], w["Nx"], w["dt"]
        params = draw_parameters(w)
        ux, uv = particle_uniforms(w)
        f = binding.Fom(N, p, Nx, dt, None, None, None, family=w["family"], params=params, ux=ux,
                        uv=uv)
        nsteps = int(round(20.0 / dt))
        times, rx, rv = [], [], []
        for k in range(0, nsteps + 1, every):
            if k:
                f.step(every)
            X, V = f.get_state()
            ranks = []
            for S in (X, V):
                r = binding.Rom(binding.make_config(N, p, Nx, 2, dt=dt), params["L"], S,
                                torch.zeros_like(S))
                sg = r.init_singular_values()
                r.close()
                ranks.append([int(np.sum(sg > t * sg[0])) for t in tols])
            del X, V
            times.append(k * dt)
            rx.append(ranks[0])
            rv.append(ranks[1])
        f.close()
        del f
        torch.cuda.empty_cache()
        out[name] = {"N": N, "Nx": Nx, "dt": dt, "times": times, "rank_X": rx, "rank_V": rv}
    return out


def hamiltonian_split_leg(binding, torch, steps=200, p=300):
    """The splitting of the step-to-step Hamiltonian change of Sec. 6.2
    (eq. error_ham_tot) on the weak Landau damping ensemble (eta = (alpha,
    sigma), k = 0.5, N = 5e4, N_x = 32, dt = 0.0025, quiet start) at p
    parameters and 2n = 6, with the Galerkin projection, with DEIM of the
    exact potential (T = 3, d = 32) and with DMD-DEIM (Alg. 2, as in the
    DMD-DEIM leg): per step the 2-norms over the
    parameters of Delta H = |H(U_tau Z_tau) - H(U_{tau-1} Z_{tau-1})|, of the
    two basis terms and of the coefficient term, through
    rom_step_hamiltonian_split; reported: their mean and maximum over the
    steps, and the mean relative Hamiltonian change per step."""
    import numpy as np
    from workloads import workload, particle_uniforms
    from workloads.ensembles import draw_parameters
    w = workload("landau_ld", p=p)
    params = draw_parameters(w)
    ux, uv = particle_uniforms(w)
    src = dict(family=w["family"], params=params, ux=ux, uv=uv)
    out = {"workload": "landau_ld", "N": w["N"], "p": p, "Nx": w["Nx"], "dt": w["dt"],
           "two_n": 6, "steps": steps,
           "terms": "dH = |H_tau - H_{tau-1}|, basis_new = |H(U_tau Z_tau) - H(U_{tau-1/2} "
                    "Z_tau)|, basis_old = |H(U_{tau-1/2} Z_{tau-1}) - H(U_{tau-1} Z_{tau-1})|, "
                    "coeff = |H(U_{tau-1/2} Z_tau) - H(U_{tau-1/2} Z_{tau-1})|, 2-norms over "
                    "the parameters"}
    for proj in ("galerkin", "deim", "dmd_deim"):
        def run(proj=proj):
            dmd = proj == "dmd_deim"
            cfg = binding.make_config(w["N"], p, w["Nx"], 6, dt=w["dt"], projection=proj,
                                      deim_window=3, deim_rows=32, fp_tol=1e-9,
                                      fp_stall_tol=DMD_STALL_TOL, p_star=w["p_star"],
                                      deim_update_every=w["deim_update_every"] if dmd else 1,
                                      deim_update_rows=w["deim_update_rows"] if dmd else 0)
            r = binding.Rom(cfg, None, None, None, **src)
            T = []
            try:
                for _ in range(steps):
                    _, H4 = r.step_hamiltonian_split()
                    H = H4.cpu().numpy()
                    T.append([np.linalg.norm(H[3] - H[0]), np.linalg.norm(H[3] - H[2]),
                              np.linalg.norm(H[1] - H[0]), np.linalg.norm(H[2] - H[1]),
                              np.linalg.norm(H[3] - H[0]) / np.linalg.norm(H[0])])
            finally:
                r.close()
            T = np.array(T)
            names = ("dH", "basis_new", "basis_old", "coeff")
            res = {k: {"mean": float(T[:, i].mean()), "max": float(T[:, i].max())}
                   for i, k in enumerate(names)}
            res["mean_relative_dH_per_step"] = float(T[:, 4].mean())
            return res
        out[proj] = _leg(f"Hamiltonian split {proj}", run)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {a.gpus}); "
              "sharding over several GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2201_05555_amd import binding
    from workloads import workload
    from workloads.ensembles import draw_parameters, load_particles, philox_uniforms

    torch.cuda.set_device(0)
    if a.restart_only:
        print(json.dumps({"restart": _leg("restart leg", lambda: restart_leg(binding, torch)),
                          "local_rank": _leg("local rank leg",
                                             lambda: local_rank_leg(binding, torch)),
                          "hamiltonian_split": _leg("Hamiltonian split leg",
                                                    lambda: hamiltonian_split_leg(binding,
                                                                                  torch))}),
              flush=True)
        return
    if a.dmd_only:
        print(json.dumps({"dmd_deim": _leg("DMD-DEIM leg", lambda: dmd_deim_leg(
            binding, torch, a.steps, a.warmup, p_sweep=()))}), flush=True)
        return
    if a.calib_copy_mib:
        src = torch.empty(a.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = workload(a.workload)
    N, p, Nx = w["N"], w["p"], w["Nx"]
    # the ensemble: parameters and shared uniforms drawn on the host, the
    # N x p initial states formed on the device (rom_init_family,
    # fom_init_family)
    params = draw_parameters(w)
    ux, uv = philox_uniforms(1000 * w["number"] + 2, N)
    src = dict(family=w["family"], params=params, ux=ux, uv=uv)

    # ---------------- reduced model ----------------
    proj = w.get("projection", "galerkin")
    rank_auto = w["two_n_max"] > w["two_n"]
    cfg = binding.make_config(N, p, Nx, w["two_n"], two_n_max=w["two_n_max"], dt=w["dt"],
                              projection=proj, deim_window=w.get("deim_window", 3), fp_tol=1e-9,
                              rank_auto=rank_auto, rank_tol_up=1e-2, rank_tol_down=1e-8)
    t_init = time.perf_counter()
    rom_h = binding.Rom(cfg, None, None, None, **src)
    t_init = time.perf_counter() - t_init
    # launch shape of the fused gather-projection for these sizes (before the
    # warm-up, outside every timed region)
    tune = _leg("autotune", rom_h.autotune)
    for _ in range(a.warmup):
        rom_h.step(1)
    torch.cuda.synchronize()
    # timed region: one call for the K steps (as a caller stepping the
    # ensemble would), no per-kernel events in the stream
    two_n_start = rom_h.two_n
    t0 = time.perf_counter()
    info = rom_h.step(a.steps)
    torch.cuda.synchronize()
    t_rom = time.perf_counter() - t0
    two_n_end = rom_h.two_n
    # per-step latency: K further steps, each its own call (the call returns
    # with the step's status read back)
    lat, stall_rel, stalled = [], info["stall_rel"], 0
    for _ in range(a.steps):
        t1 = time.perf_counter()
        inf = rom_h.step(1)
        lat.append(time.perf_counter() - t1)
        stall_rel = max(stall_rel, inf["stall_rel"])
        stalled += inf["stalled"]
    # third pass of the same length: HIP events on the library's streams
    # around every kernel family, for the roofline figures
    binding.set_timing(True)
    for fam in binding.FAMILIES:
        binding.kernel_ms(fam)
        binding.kernel_work(fam)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        inf = rom_h.step(1)
        stall_rel = max(stall_rel, inf["stall_rel"])
        stalled += inf["stalled"]
    torch.cuda.synchronize()
    t_rom_ev = time.perf_counter() - t0
    fams = {}
    for fam in binding.FAMILIES:
        ms, n = binding.kernel_ms(fam)
        fl, by = binding.kernel_work(fam)
        fams[fam] = dict(ms=ms, launches=n, flops=fl, bytes=by)
    binding.set_timing(False)
    rom_h.close()
    del rom_h
    torch.cuda.empty_cache()
    _progress(f"reduced model: {1e3 * t_rom / a.steps:.2f} ms per step")

    # ---------------- full-order model ----------------
    fom_h = binding.Fom(N, p, Nx, w["dt"], None, None, None, **src)
    fom_h.step(a.warmup)
    torch.cuda.synchronize()
    binding.set_timing(True)
    binding.kernel_ms("fom_push")
    binding.kernel_work("fom_push")
    t0 = time.perf_counter()
    fom_h.step(a.steps)
    torch.cuda.synchronize()
    t_fom = time.perf_counter() - t0
    ms_push, n_push = binding.kernel_ms("fom_push")
    fl_push, by_push = binding.kernel_work("fom_push")
    binding.set_timing(False)
    fom_h.close()
    del fom_h
    torch.cuda.empty_cache()
    _progress(f"full-order model: {1e3 * t_fom / a.steps:.2f} ms per step")

    pp = N * p
    rom_rate = pp * a.steps / t_rom
    fom_rate = pp * a.steps / t_fom
    # dominant kernel of the ROM step on the caller's stream: the
    # single-kernel family with the largest device time over the
    # instrumented steps
    dom = max(SINGLE_KERNEL, key=lambda f: fams[f]["ms"])
    d = fams[dom]
    roof = roofline_of(d["ms"], d["flops"], d["bytes"], d["launches"])
    if roof is not None:
        roof["kernel"] = SINGLE_KERNEL[dom]
        roof["ms_per_step"] = d["ms"] / a.steps
        t = measured_traffic(dom, a.workload)
        if t is not None:
            roof["traffic"] = t
            roof["traffic_over_algorithmic"] = t / roof["algorithmic_bytes_per_launch"]
    fom_roof = roofline_of(ms_push, fl_push, by_push, n_push)
    # the DEIM chain on the second stream (snapshot, Gram block, top-d
    # eigenpairs, Psi, greedy, weights): device time per step
    crit = None
    if fams["deim_eig"]["launches"]:
        e = fams["deim_eig"]
        eig = roofline_of(e["ms"], e["flops"], e["bytes"], e["launches"])
        crit = {"stream": "second (beside the basis velocity and Cayley map of the step)",
                "deim_chain_ms_per_step": (e["ms"] + fams["deim_chain"]["ms"]) / a.steps,
                "eigensolver_ms_per_step": e["ms"] / a.steps,
                "eigensolver": dict(eig or {}, kernel="dense_topeig_kernel (top-d eigenpairs "
                                                      "of the P x P snapshot Gram, one workgroup)"),
                "rest_of_chain_ms_per_step": fams["deim_chain"]["ms"] / a.steps}
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": "particle-param steps/s, reduced model (ROM) on 1 GPU; FOM and ratio at "
                  "matched error beside",
        "value": rom_rate,
        "unit": "particle-param-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * t_rom / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded two-stream ensemble, inverse-CDF loading)",
        "config": {"workload": a.workload, "N": N, "p": p, "Nx": Nx, "dt": w["dt"],
                   "two_n_start": two_n_start, "two_n_end": two_n_end,
                   "two_n_max": w["two_n_max"], "projection": proj,
                   "rank_auto": bool(rank_auto), "rank_tol_up": 1e-2, "rank_tol_down": 1e-8,
                   "deim_steps": info["deim_steps"], "fp_tol": 1e-9,
                   "mean_fp_iters": info["iters_total"] / a.steps},
        "fixed_point": {"stalled_columns": info["stalled_total"] + stalled,
                        "max_stall_accepted_update": stall_rel,
                        "fp_stall_tol": 1e-3, "note": "over the timed, latency and event passes"},
        "step_latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                            "p99": float(np.percentile(lat_ms, 99)),
                            "max": float(lat_ms.max())},
        "fom": {"value": fom_rate, "unit": "particle-param-steps/s",
                "ms_per_step": 1e3 * t_fom / a.steps, "roofline": fom_roof},
        "rom_over_fom": rom_rate / fom_rate,
        "roofline": roof,
        "critical_path": crit,
        "kernel_families_ms_per_step": {f: fams[f]["ms"] / a.steps for f in fams},
        "ms_per_step_with_events": 1e3 * t_rom_ev / a.steps,
    }
    out["config"]["init_s"] = t_init
    out["config"]["autotune"] = tune
    if not a.no_matched:
        out["matched_error"] = _leg("matched error", lambda: matched_error(
            binding, torch, w, src, cfg, a.warmup + a.steps))
        if "failed" not in out["matched_error"]:
            out["matched_error"]["rom_over_fom_at_this_error"] = rom_rate / fom_rate
    if not a.no_dmd:
        out["dmd_deim"] = _leg("DMD-DEIM leg", lambda: dmd_deim_leg(binding, torch, a.steps,
                                                                     a.warmup))
    if not a.no_restart:
        out["restart"] = _leg("restart leg", lambda: restart_leg(binding, torch))
        out["local_rank"] = _leg("local rank leg", lambda: local_rank_leg(binding, torch))
        out["hamiltonian_split"] = _leg("Hamiltonian split leg",
                                        lambda: hamiltonian_split_leg(binding, torch))
    if not a.no_serve:
        out["serve"] = _leg("serving mix", lambda: serve_bench(
            binding, torch, a.serve_requests, a.serve_step_scale, 4, 96.0, a.serve_gap))
    if not a.no_cpu:
        # the oracle's sample: the first 8 parameters and 1e5 particles
        ns = min(N, 100_000)
        sub = {k: v[:8] for k, v in params.items()}
        Xs, Vs = load_particles(sub, ux[:ns], uv[:ns], w["family"])
        ens = dict(X0=Xs, V0=Vs, L=sub["L"])
        out["cpu_baseline"] = cpu_baseline(w, ens, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
