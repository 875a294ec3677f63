"""Benchmark: particle-parameter steps per second of the reduced model (ROM)
and of the full-order PIC model (FOM) on one MI355X, on the synthetic
two-stream ensemble N = 100,000 particles, p = 64 parameters, Nx = 128 cells,
dt = 0.05, reduced rank 2n starting at 10 (cap 60).

Prints ONE JSON line.  `value` is the ROM throughput N * p * steps / time of
the timed steps (inputs resident in HBM); by default two warm-up steps and 25
timed steps (steps 3 to 27, the averaging window of the paper's timings).  `roofline` describes the
dominant kernel family of the ROM step, timed with HIP events on the
library's stream over the timed region; `cpu_baseline` times the FP64
oracle on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12        # B/s, MI355X HBM3E

# timing families that hold one kernel each, and that kernel; the first
# three run on the caller's stream (the step's critical path), the last on
# the second stream beside the basis-velocity kernels
SINGLE_KERNEL = {
    "deposit": "deposit_rom_kernel (reconstruct + cell + LDS histogram)",
    "gather": "gather_project_kernel (reconstruct + field gather + g = U^* G)",
    "gather_xi": "gather_xi_kernel (reconstruct + field gather + xi = -i h G Q + U M)",
}
SIDE_KERNEL = {
    "deim_eig": "dense_topeig_kernel (top-d eigenpairs of the DEIM snapshot Gram)",
}
PEAK_FP64 = 78.6e12      # flop/s, MI355X FP64 vector (= FP64 matrix) peak

# HBM bytes per launch of the deposit kernel, measured with two counter
# passes (FETCH_SIZE, WRITE_SIZE) calibrated on a plain device copy; valid
# only for the kernel source it was taken on
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles",
                               "deposit_rom_kernel_twostream_deim_N1e5_p64_hbm_traffic.md")
TRAFFIC_SOURCE = os.path.join(ROOT, "paper_2201_05555_amd", "csrc", "pic_kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="twostream_deim")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    return ap.parse_args()


def roofline_of(ms, flops, nbytes, launches):
    """Binding roofline of a kernel family from its algorithmic work and its
    measured time: the resource with the larger lower bound on time."""
    t = ms * 1e-3
    if t <= 0:
        return None
    t_alu = flops / PEAK_FP64
    t_hbm = nbytes / PEAK_HBM
    if t_hbm >= t_alu:
        ach = nbytes / t / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": ach / (PEAK_HBM / 1e9), "traffic": None,
                "avg_launch_us": 1e3 * ms / max(launches, 1), "launches": launches}
    ach = flops / t / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": ach / (PEAK_FP64 / 1e12), "traffic": None,
            "avg_launch_us": 1e3 * ms / max(launches, 1), "launches": launches}


def measured_traffic():
    """Counter-measured HBM bytes per deposit launch, or None when the
    profile is missing or the kernel source has changed since it was taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        sha = hashlib.sha256(open(TRAFFIC_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    val = src = None
    for line in text.splitlines():
        if line.startswith("traffic-bytes-per-launch:"):
            val = float(line.split(":")[1])
        elif line.startswith("source-sha256"):
            src = line.split(":")[-1].strip()
    return val if (val is not None and src == sha) else None


def cpu_baseline(w, ens, seconds):
    """The oracle's reduced step on a sample of the workload: the first
    p_sub parameters, the same N, rank and time step."""
    import numpy as np
    from oracle import rom
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    p_sub = min(8, w["p"])
    X0 = np.asfortranarray(ens["X0"][:, :p_sub])
    V0 = np.asfortranarray(ens["V0"][:, :p_sub])
    cfg = rom.RomConfig(N=w["N"], p=p_sub, Nx=w["Nx"], two_n=w["two_n"], dt=w["dt"],
                        fp_tol=1e-9, two_n_max=w["two_n_max"],
                        projection=w.get("projection", "galerkin"),
                        deim_window=w.get("deim_window", 3),
                        rank_auto=w["two_n_max"] > w["two_n"], rank_tol_up=1e-2)
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
    val = w["N"] * p_sub * steps / el
    return {"value": val, "unit": "particle-param-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle prk_step (+ rank policy), first {p_sub} of {w['p']} parameters, "
                      f"N={w['N']}, 2n={w['two_n']}->{st.U.shape[1]}, {cfg.projection}, "
                      f"{steps} steps in {el:.1f} s"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {a.gpus}); the "
              "multi-GPU design is described but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2201_05555_amd import binding
    from workloads import make_ensemble, workload

    torch.cuda.set_device(0)
    if a.calib_copy_mib:
        src = torch.empty(a.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = workload(a.workload)
    N, p, Nx = w["N"], w["p"], w["Nx"]
    ens = make_ensemble(w)
    X0 = binding._dev(ens["X0"])
    V0 = binding._dev(ens["V0"])
    torch.cuda.synchronize()

    # ---------------- reduced model ----------------
    proj = w.get("projection", "galerkin")
    cfg = binding.make_config(N, p, Nx, w["two_n"], two_n_max=w["two_n_max"], dt=w["dt"],
                              projection=proj, deim_window=w.get("deim_window", 3), fp_tol=1e-9,
                              rank_auto=w["two_n_max"] > w["two_n"], rank_tol_up=1e-2)
    rom_h = binding.Rom(cfg, ens["L"], X0, V0)
    for _ in range(a.warmup):
        rom_h.step(1)
    torch.cuda.synchronize()
    # timed region: no per-kernel events (each event record leaves a gap in
    # the stream), so `value` is the plain throughput
    # (one call for the K steps, as a caller stepping the ensemble would)
    two_n_start = rom_h.two_n
    t0 = time.perf_counter()
    info = rom_h.step(a.steps)
    torch.cuda.synchronize()
    t_rom = time.perf_counter() - t0
    iters_timed = info["iters_total"]
    deim_steps = info["deim_steps"]
    two_n_end = rom_h.two_n
    # second timed region of the same length: HIP events on the library's
    # stream around every kernel family, for the roofline figures
    binding.set_timing(True)
    for fam in binding.FAMILIES:
        binding.kernel_ms(fam)
        binding.kernel_work(fam)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        rom_h.step(1)
    torch.cuda.synchronize()
    t_rom_ev = time.perf_counter() - t0
    fams = {}
    for fam in binding.FAMILIES:
        ms, n = binding.kernel_ms(fam)
        fl, by = binding.kernel_work(fam)
        fams[fam] = dict(ms=ms, launches=n, flops=fl, bytes=by)
    binding.set_timing(False)
    rom_h.close()

    # ---------------- full-order model ----------------
    fom_h = binding.Fom(N, p, Nx, w["dt"], ens["L"], X0, V0)
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

    pp = N * p
    rom_rate = pp * a.steps / t_rom
    fom_rate = pp * a.steps / t_fom
    # dominant kernel of the ROM step: the single-kernel family on the
    # caller's stream with the largest device time over the instrumented
    # steps (the "basis" and "dense" families are groups of different small
    # kernels; the DEIM eigensolver runs beside them on the second stream and
    # is reported separately)
    dom = max(SINGLE_KERNEL, key=lambda f: fams[f]["ms"])
    d = fams[dom]
    roof = roofline_of(d["ms"], d["flops"], d["bytes"], d["launches"])
    if roof is not None:
        roof["kernel"] = SINGLE_KERNEL[dom]
        if dom == "deposit":
            t = measured_traffic()
            if t is not None:
                roof["traffic"] = t
                roof["algorithmic_bytes_per_launch"] = d["bytes"] / max(d["launches"], 1)
        roof["ms_per_step"] = d["ms"] / a.steps
    fom_roof = roofline_of(ms_push, fl_push, by_push, n_push)
    side = {}
    for f, name in SIDE_KERNEL.items():
        r = roofline_of(fams[f]["ms"], fams[f]["flops"], fams[f]["bytes"], fams[f]["launches"])
        if r is not None:
            r["kernel"] = name
            r["ms_per_step"] = fams[f]["ms"] / a.steps
            r["stream"] = "second (beside the basis-velocity kernels)"
            side[f] = r

    out = {
        "metric": "particle-param steps/s, reduced model (ROM) on 1 GPU; FOM and ratio beside",
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
                   "rank_auto": bool(cfg.rank_auto), "rank_tol_up": 1e-2,
                   "deim_steps": deim_steps, "fp_tol": 1e-9,
                   "mean_fp_iters": iters_timed / a.steps},
        "fom": {"value": fom_rate, "unit": "particle-param-steps/s",
                "ms_per_step": 1e3 * t_fom / a.steps, "roofline": fom_roof},
        "rom_over_fom": rom_rate / fom_rate,
        "roofline": roof,
        "roofline_side_stream": side,
        "kernel_families_ms_per_step": {f: fams[f]["ms"] / a.steps for f in fams},
        "ms_per_step_with_events": 1e3 * t_rom_ev / a.steps,
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, ens, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
