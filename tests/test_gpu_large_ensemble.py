"""GPU parity for large ensembles (p above 64 parameters: the p x p Gram in
64-column blocks, its leading eigenvectors by subspace iteration, parameter
chunks in the fused basis-velocity kernel, wide row combinations in slices)
and for the device-side loading of the initial ensemble, against the FP64
oracle and the seeded input generator."""
import numpy as np
import pytest

from oracle import rom
from workloads import make_ensemble, workload
from workloads.ensembles import draw_parameters, philox_uniforms

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _say(*a):
    print("[case]", *a, flush=True)


def _b():
    import torch
    from paper_2201_05555_amd import binding
    assert torch.cuda.is_available()
    return binding, torch


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _set_from_oracle(r, st, torch):
    N = st.U.shape[0] // 2
    UX = torch.from_numpy(np.ascontiguousarray(st.U[:N].T)).cuda()
    Z = torch.from_numpy(np.ascontiguousarray(st.Z.T)).cuda()
    r.set_state(UX, Z, st.step)


def _sensitivity(st, cfg, iters, steps=1, pert=1e-15):
    rng = np.random.default_rng(0)
    outs = []
    for eps in (0.0, pert):
        s2 = rom.RomState(U=st.U.copy(), Z=st.Z * (1 + eps * rng.normal(size=st.Z.shape)),
                          L=st.L)
        for _ in range(steps):
            rom.prk_step(s2, cfg, fixed_iters=iters)
        outs.append(s2.U @ s2.Z)
    return _rel(outs[1], outs[0])


def _within(err, sens, what, floor=RTOL):
    bound = max(floor, 50.0 * sens)
    print(f"  {what}: err {err:.2e}  oracle sensitivity {sens:.2e}  bound {bound:.2e}",
          flush=True)
    assert err < bound, (what, err, sens, bound)


@pytest.mark.parametrize("name,N,p", [("landau_tiny", 4099, 37), ("twostream_deim", 5003, 70)])
def test_device_loading_matches_the_generator(name, N, p):
    """symrom_load_family against the seeded generator of the inputs
    (inverse-CDF loading of Sec. 6.1 with shared uniforms): positions and
    velocities agree to Newton's tolerance."""
    binding, torch = _b()
    w = workload(name, N=N, p=p)
    _say("load family", name, N, p)
    e = make_ensemble(w)
    ux, uv = philox_uniforms(1000 * w["number"] + 2, N)
    X, V = binding.load_family(w["family"], e["params"], ux, uv)
    ex = float(np.max(np.abs(_np(X).T - e["X0"]) / e["L"][None, :]))
    ev = float(np.max(np.abs(_np(V).T - e["V0"])))
    print(f"  max |dx| / L {ex:.2e}, max |dv| {ev:.2e}", flush=True)
    assert ex < 1e-13 and ev < 1e-11


def test_rom_init_family_equals_rom_init():
    binding, torch = _b()
    w = workload("twostream_deim", N=6000, p=24, Nx=64)
    _say("rom_init_family")
    e = make_ensemble(w)
    ux, uv = philox_uniforms(1000 * w["number"] + 2, w["N"])
    cfg = binding.make_config(w["N"], w["p"], w["Nx"], 10, dt=w["dt"])
    r1 = binding.Rom(cfg, e["L"], e["X0"], e["V0"])
    r2 = binding.Rom(cfg, None, None, None, family="twostream", params=e["params"], ux=ux, uv=uv)
    X1, V1 = r1.reconstruct()
    X2, V2 = r2.reconstruct()
    err = max(_rel(_np(X2), _np(X1)), _rel(_np(V2), _np(V1)))
    print(f"  R0 rel diff {err:.2e}", flush=True)
    assert err < 1e-10
    f1 = binding.Fom(w["N"], w["p"], w["Nx"], w["dt"], e["L"], e["X0"], e["V0"])
    f2 = binding.Fom(w["N"], w["p"], w["Nx"], w["dt"], None, None, None, family="twostream",
                     params=e["params"], ux=ux, uv=uv)
    f1.step(3)
    f2.step(3)
    Xa, Va = f1.get_state()
    Xb, Vb = f2.get_state()
    assert _rel(_np(Xb), _np(Xa)) < 1e-12 and _rel(_np(Vb), _np(Va)) < 1e-10


@pytest.mark.parametrize("N,p,two_n", [(6000, 130, 10), (3001, 256, 20)])
def test_large_p_init_parity(N, p, two_n):
    """Truncated complex SVD initialisation with p > 64 (Gram in blocks,
    subspace iteration for the leading eigenvectors): R_0 = U U^* C_0 as in
    the oracle's SVD, and an orthonormal basis."""
    binding, torch = _b()
    w = workload("twostream_deim", N=N, p=p, Nx=64)
    _say("large-p init", N, p, two_n)
    e = make_ensemble(w)
    r = binding.Rom(binding.make_config(N, p, w["Nx"], two_n, dt=w["dt"]), e["L"], e["X0"],
                    e["V0"])
    X, V = r.reconstruct()
    cfg = rom.RomConfig(N=N, p=p, Nx=w["Nx"], two_n=two_n, dt=w["dt"])
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    Xo, Vo = rom.reconstruct(st)
    ex, ev = _rel(_np(X).T, Xo), _rel(_np(V).T, Vo)
    print(f"  R0 rel err {ex:.2e} {ev:.2e}", flush=True)
    assert ex < 1e-9 and ev < 1e-9
    UX, Z, _ = r.get_state()
    UXn = _np(UX).T
    n = two_n // 2
    Ut = UXn[:, :n] - 1j * UXn[:, n:]
    assert np.abs(Ut.conj().T @ Ut - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("N,p,two_n,iters,proj", [
    (6000, 130, 10, 4, "galerkin"),
    (2000, 520, 36, 3, "galerkin"),   # n > 16 (stored G~): wide row combinations in slices
    (4000, 200, 12, 4, "deim"),
])
def test_large_p_steps_parity(N, p, two_n, iters, proj):
    """Steps with p > 64 (parameter chunks of the fused basis-velocity
    kernel, the per-column fixed-point update): U_X, Z and R = U Z against
    the oracle within the conditioning-aware bound."""
    binding, torch = _b()
    w = workload("twostream_deim", N=N, p=p, Nx=64)
    _say("large-p steps", N, p, two_n, iters, proj)
    e = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=p, Nx=w["Nx"], two_n=two_n, dt=w["dt"], projection=proj,
                        deim_window=3, fp_tol=1e-10)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    steps = 5 if proj == "deim" else 1
    if proj == "deim":
        st_s = rom.RomState(U=st.U.copy(), Z=st.Z.copy(), L=st.L)
        rng = np.random.default_rng(0)
        outs = []
        for pert in (0.0, 1e-15):
            s2 = rom.RomState(U=st.U.copy(), Z=st.Z * (1 + pert * rng.normal(size=st.Z.shape)),
                              L=st.L)
            c2 = rom.RomConfig(**cfg.__dict__)
            for _ in range(steps):
                assert rom.prk_step(s2, c2) == rom.OK
            outs.append(s2.U @ s2.Z)
        sR = _rel(outs[1], outs[0])
        gcfg = binding.make_config(N, p, w["Nx"], two_n, dt=w["dt"], projection="deim",
                                   deim_window=3, fp_tol=1e-10)
    else:
        sR = _sensitivity(st, cfg, iters)
        gcfg = binding.make_config(N, p, w["Nx"], two_n, dt=w["dt"], fp_fixed_iters=iters)
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    for s in range(steps):
        info = r.step(1)
        if proj == "deim":
            assert rom.prk_step(st, cfg) == rom.OK
            assert info["iters"] == st.last_iters, (s, info, st.last_iters)
        else:
            assert rom.prk_step(st, cfg, fixed_iters=iters) == rom.OK
    X, V = r.reconstruct()
    Xo, Vo = rom.reconstruct(st)
    floor = 1e-9 if proj == "deim" else RTOL
    _within(_rel(_np(X).T, Xo), sR, "X_r", floor)
    _within(_rel(_np(V).T, Vo), sR, "V_r", floor)


def test_large_p_rank_growth():
    """Growth by two pairs with p > 64 (the Gram of H = (I - U~U~^*)(-i G~)
    in blocks, its leading eigenvectors by subspace iteration): R bitwise
    unchanged, the new directions as the oracle's to the accuracy of the Gram
    route, and an orthonormal basis."""
    binding, torch = _b()
    N, p = 5000, 150
    w = workload("twostream_deim", N=N, p=p, Nx=64)
    _say("large-p growth", N, p)
    e = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=p, Nx=w["Nx"], two_n=8, two_n_max=12, dt=w["dt"])
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    r = binding.Rom(binding.make_config(N, p, w["Nx"], 8, two_n_max=12, dt=w["dt"]), e["L"],
                    e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    X0, V0 = r.reconstruct()
    gr = rom.gradient(st.U, st.Z, st.L, w["Nx"])
    Ut = rom.to_complex_basis(st.U)
    Gt = gr.G[:N] + 1j * gr.G[N:]
    H = Gt - Ut @ (Ut.conj().T @ Gt)
    sv = np.linalg.svd(H, compute_uv=False)
    assert r.adapt_rank(12) == 12
    rom.adapt_rank(st, cfg, 12)
    X1, V1 = r.reconstruct()
    assert torch.equal(X0, X1) and torch.equal(V0, V1)
    UXn = _np(r.get_state()[0]).T
    tol = max(1e-9, 1e-14 * (sv[0] / sv[2]) ** 2)
    err = _rel(UXn, st.U[:N])
    print(f"  U rel err {err:.2e} (bound {tol:.2e})", flush=True)
    assert err < tol
    Utg = UXn[:, :6] - 1j * UXn[:, 6:]
    assert np.abs(Utg.conj().T @ Utg - np.eye(6)).max() < 1e-12


def test_init_beyond_the_numerical_rank():
    """A rank far above the ensemble's numerical rank (Landau, p = 51, whose
    singular values fall below 1e-13 of the largest after about ten; 2n =
    60): the eigenpairs of C0^* C0 that the Gram resolves (above 1e-13 of
    the largest eigenvalue) are kept and Gram-Schmidt completes the basis.
    The basis is orthonormal and R_0 misses only the dropped tail (2e-8 of
    |C_0| here; the oracle's SVD keeps it)."""
    binding, torch = _b()
    w = workload("landau_tiny", p=51, N=20000, Nx=128)
    _say("init beyond the numerical rank")
    e = make_ensemble(w)
    r = binding.Rom(binding.make_config(w["N"], w["p"], w["Nx"], 60, dt=w["dt"]), e["L"],
                    e["X0"], e["V0"])
    X, V = r.reconstruct()
    C = e["X0"] + 1j * e["V0"]
    R = _np(X).T + 1j * _np(V).T
    err = float(np.linalg.norm(R - C) / np.linalg.norm(C))
    UX = _np(r.get_state()[0]).T
    Ut = UX[:, :30] - 1j * UX[:, 30:]
    orth = float(np.abs(Ut.conj().T @ Ut - np.eye(30)).max())
    print(f"  |R0 - C0| / |C0| = {err:.2e}, orthonormality {orth:.2e}", flush=True)
    assert err < 1e-7 and orth < 1e-12
