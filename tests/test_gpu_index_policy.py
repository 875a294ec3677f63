"""GPU parity of the index work and of the step's control policy, through the
C ABI, against the FP64 oracle on the same seeded inputs:

* DEIM greedy indices bit for bit and weights at 1e-10 on an identical basis
  (``deim_select``), and the indices of the DEIM operator the step builds;
* the particle-to-cell map of the fused kernels against the cells of an
  independent reconstruction (every mismatch must sit on a node);
* deterministic mode (integer theta sums): runs repeat bit for bit;
* ENOCONV restores the DEIM snapshot window (a retry equals a run that never
  failed), and the stagnation counters;
* the automatic shrink, and growth that keeps the basis orthonormal;
* row-subset reconstruction.
"""
import numpy as np
import pytest

from oracle import deim, pic, rom
from workloads import make_ensemble, workload

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


def _ens(name, **kw):
    w = workload(name, **kw)
    return w, make_ensemble(w)


def _set_from_oracle(r, st, torch):
    N = st.U.shape[0] // 2
    UX = torch.from_numpy(np.ascontiguousarray(st.U[:N].T)).cuda()
    Z = torch.from_numpy(np.ascontiguousarray(st.Z.T)).cuda()
    r.set_state(UX, Z, st.step)


def _greedy_margins(Psi):
    """Per greedy step, 1 - (runner-up |r|) / (winner |r|) of the oracle's
    residuals: how far each choice is from a tie."""
    idx = deim.greedy_indices(Psi)
    out = []
    for k in range(Psi.shape[1]):
        if k == 0:
            r = Psi[:, 0].copy()
        else:
            c = np.linalg.solve(Psi[idx[:k], :k], Psi[idx[:k], k])
            r = Psi[:, k] - Psi[:, :k] @ c
        a = np.sort(np.abs(r))[::-1]
        out.append(1.0 - a[1] / a[0])
    return np.array(out)


@pytest.mark.parametrize("N,d,seed", [(5000, 10, 1), (4099, 14, 2), (20000, 36, 3),
                                      (3001, 64, 4), (257, 7, 5)])
def test_deim_select_bit_exact_indices(N, d, seed):
    """Same orthonormal basis on both sides: identical greedy indices, and
    weights within 1e-10 relative (Sec. 4.2.2)."""
    binding, torch = _b()
    _say("deim_select", N, d, seed)
    rng = np.random.default_rng(seed)
    Psi, _ = np.linalg.qr(rng.normal(size=(N, d)))
    margins = _greedy_margins(Psi)
    print(f"  smallest greedy margin {margins.min():.2e}", flush=True)
    assert margins.min() > 1e-9          # no near ties in these seeded bases
    idx, w = binding.deim_select(Psi)
    ref = deim.greedy_indices(Psi)
    wref = deim.weights(Psi, ref)
    assert np.array_equal(_np(idx).astype(np.int64), ref), (_np(idx), ref)
    err = _rel(_np(w), wref)
    print(f"  weights rel err {err:.2e}", flush=True)
    assert err < RTOL


def test_deim_select_snapshot_basis():
    """The basis of a real snapshot window (left singular vectors of Y from
    the oracle), fed to the library's selection kernels."""
    binding, torch = _b()
    w, e = _ens("twostream_deim", N=20000, p=24, Nx=128)
    _say("deim_select snapshot basis")
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=12, dt=w["dt"], fp_tol=1e-10,
                        projection="deim", deim_window=3)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    for _ in range(4):
        assert rom.prk_step(st, cfg) == rom.OK
    Y = np.concatenate(st.window, axis=1)
    Psi, _ = deim.deim_basis(Y, 12)
    margins = _greedy_margins(Psi)
    print(f"  smallest greedy margin {margins.min():.2e}", flush=True)
    idx, wg = binding.deim_select(Psi)
    ref = deim.greedy_indices(Psi)
    assert np.array_equal(_np(idx).astype(np.int64), ref)
    err = _rel(_np(wg), deim.weights(Psi, ref))
    print(f"  weights rel err {err:.2e}", flush=True)
    assert err < RTOL


@pytest.mark.parametrize("kw,two_n,steps", [
    (dict(N=20000, p=24, Nx=128), 8, 6),
    (dict(N=30000, p=64, Nx=128), 10, 5),
])
def test_deim_operator_indices_in_the_step(kw, two_n, steps):
    """The DEIM indices the library builds inside its steps equal the
    oracle's (Psi from the eigenpairs of the snapshot Gram on the GPU, from
    an SVD in the oracle) wherever the oracle's greedy choice is not a near
    tie (margin above 1e-6); the weights are reported."""
    binding, torch = _b()
    w, e = _ens("twostream_deim", **kw)
    _say("deim operator in the step", kw, two_n, steps)
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=two_n, dt=w["dt"], fp_tol=1e-10,
                        projection="deim", deim_window=3)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    gcfg = binding.make_config(w["N"], w["p"], w["Nx"], two_n, dt=w["dt"], fp_tol=1e-10,
                               projection="deim", deim_window=3)
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    compared = 0
    for s in range(steps):
        info = r.step(1)
        assert rom.prk_step(st, cfg) == rom.OK
        assert info["iters"] == st.last_iters
        if st.deim_indices is None:
            continue
        Y = np.concatenate(st.window, axis=1)
        Psi, _ = deim.deim_basis(Y, min(two_n, Y.shape[1]))
        margins = _greedy_margins(Psi)
        idx, wg = r.deim_operator()
        gi = _np(idx).astype(np.int64)
        wo = deim.weights(Psi, st.deim_indices)
        print(f"  step {s}: margin {margins.min():.2e}, indices equal "
              f"{np.array_equal(gi, st.deim_indices)}, weights rel err "
              f"{_rel(_np(wg), wo):.2e}", flush=True)
        if margins.min() > 1e-6:
            assert np.array_equal(gi, st.deim_indices), (gi, st.deim_indices)
            compared += 1
    assert compared >= 1


@pytest.mark.parametrize("name,kw,two_n", [
    ("landau_tiny", dict(N=4099), 10),
    ("twostream_deim", dict(N=30000, p=64, Nx=128), 10),
    ("twostream_deim", dict(N=7777, p=20, Nx=64), 14),
    ("twostream_deim", dict(N=6000, p=24, Nx=64), 36),
])
def test_fused_kernel_cells(name, kw, two_n):
    """The cells of the fused reduced kernels (their own position arithmetic)
    against the cells of the oracle's X_r = U_X Z: every mismatch must be a
    particle within rounding of a node (|s - round(s)| < 1e-12 |s|)."""
    binding, torch = _b()
    w, e = _ens(name, **kw)
    _say("fused cells", name, kw, two_n)
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=two_n, dt=w["dt"])
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    for _ in range(2):
        assert rom.prk_step(st, cfg, fixed_iters=3) == rom.OK
    gcfg = binding.make_config(w["N"], w["p"], w["Nx"], two_n, dt=w["dt"])
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    cells, sv = r.cells()
    Xo, _ = rom.reconstruct(st)
    jo, _ = pic.cell_index(Xo, st.L, w["Nx"])
    cg = _np(cells).T
    s = _np(sv).T
    bad = cg != jo
    nbad = int(bad.sum())
    print(f"  {cg.size} cells, {nbad} mismatches", flush=True)
    if nbad:
        sb = s[bad]
        assert np.all(np.abs(sb - np.round(sb)) < 1e-12 * np.maximum(1.0, np.abs(sb)))


def test_deterministic_mode_repeats_bit_for_bit():
    """With deterministic = 1 (integer theta sums in the deposit), two runs
    of the same DEIM ensemble give identical bits after several steps, and
    the run stays within the parity bound of the oracle."""
    binding, torch = _b()
    w, e = _ens("twostream_deim", N=20000, p=24, Nx=128)
    _say("deterministic repeat")
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=10, dt=w["dt"], fp_tol=1e-10,
                        projection="deim", deim_window=3)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    outs = []
    for rep in range(2):
        gcfg = binding.make_config(w["N"], w["p"], w["Nx"], 10, dt=w["dt"], fp_tol=1e-10,
                                   projection="deim", deim_window=3, deterministic=True)
        r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
        _set_from_oracle(r, st, torch)
        r.step(6)
        outs.append(r.get_state()[:2])
        r.close()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    # the charge of the deterministic deposit against the oracle's
    gcfg = binding.make_config(w["N"], w["p"], w["Nx"], 10, dt=w["dt"], deterministic=True)
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    Zt = torch.from_numpy(np.ascontiguousarray(st.Z.T)).cuda()
    g, rho, Phi, ef = r.gradient(Zt)
    gr = rom.gradient(st.U, st.Z, st.L, w["Nx"])
    err = _rel(_np(rho).T, gr.rho)
    print(f"  deterministic rho rel err {err:.2e}", flush=True)
    assert err < 1e-12
    assert _rel(_np(g).T, gr.g) < RTOL


def test_enoconv_restores_the_deim_window():
    """A DEIM step that fails (ENOCONV) leaves U, Z and the snapshot window as
    they were: the retry gives the same bits as a run that never failed
    (deterministic mode, so that the comparison can be exact)."""
    binding, torch = _b()
    w, e = _ens("twostream_deim", N=20000, p=24, Nx=128)
    _say("enoconv deim window")
    kw = dict(dt=w["dt"], fp_tol=1e-10, projection="deim", deim_window=3, deterministic=True)
    ra = binding.Rom(binding.make_config(w["N"], w["p"], w["Nx"], 10, **kw), e["L"], e["X0"],
                     e["V0"])
    rb = binding.Rom(binding.make_config(w["N"], w["p"], w["Nx"], 10, **kw), e["L"], e["X0"],
                     e["V0"])
    ra.step(5)
    rb.step(5)
    UX0, Z0, step0 = rb.get_state()
    rb.set_fixed_point(0.0, 1, 0)
    status, info = rb.step_status(1)
    assert status == binding.ENOCONV
    UX1, Z1, step1 = rb.get_state()
    assert step1 == step0 and torch.equal(UX0, UX1) and torch.equal(Z0, Z1)
    rb.set_fixed_point(1e-10, 100, 0)
    ia = ra.step(2)
    ib = rb.step(2)
    assert ia["iters"] == ib["iters"] and ia["deim_active"] == ib["deim_active"] == 1
    UXa, Za, _ = ra.get_state()
    UXb, Zb, _ = rb.get_state()
    assert torch.equal(UXa, UXb) and torch.equal(Za, Zb)
    ia_op, ib_op = ra.deim_operator(), rb.deim_operator()
    assert torch.equal(ia_op[0], ib_op[0]) and torch.equal(ia_op[1], ib_op[1])


def test_stagnation_counters_match_the_oracle():
    """Steps with the stagnation rule active: the GPU reports the same number
    of stall-accepted columns as the oracle and the largest accepted update
    (both zero when no column stalls)."""
    binding, torch = _b()
    w, e = _ens("landau_tiny", N=2000)
    _say("stagnation counters")
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=10, dt=w["dt"], fp_tol=1e-14)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    gcfg = binding.make_config(w["N"], w["p"], w["Nx"], 10, dt=w["dt"], fp_tol=1e-14)
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    for s in range(3):
        info = r.step(1)
        assert rom.prk_step(st, cfg) == rom.OK
        print(f"  step {s}: iters {info['iters']}/{st.last_iters}, stalled "
              f"{info['stalled']}/{st.last_stalled}, stall_rel {info['stall_rel']:.2e}/"
              f"{st.last_stall_rel:.2e}", flush=True)
        assert info["iters"] == st.last_iters
        assert info["stalled"] == st.last_stalled
        assert (info["stall_rel"] == 0.0) == (st.last_stall_rel == 0.0)
        assert info["stall_rel"] < cfg.fp_stall_tol


def test_multi_step_call_reports_the_largest_stall_of_the_call():
    """A call of three steps reports the stall acceptances and iterations
    summed over its steps and the largest update accepted in any of them:
    the same as three one-step calls from the same state (deterministic
    mode, so that the two runs are identical).  With fp_tol = 0 no column
    converges by the tolerance, so every column ends by the stagnation rule
    once its updates reach the rounding floor."""
    binding, torch = _b()
    w, e = _ens("landau_tiny", N=2000)
    _say("stall report of a multi-step call")
    kw = dict(dt=w["dt"], fp_tol=0.0, deterministic=True)
    ra = binding.Rom(binding.make_config(w["N"], w["p"], w["Nx"], 10, **kw), e["L"], e["X0"],
                     e["V0"])
    rb = binding.Rom(binding.make_config(w["N"], w["p"], w["Nx"], 10, **kw), e["L"], e["X0"],
                     e["V0"])
    per = [ra.step(1) for _ in range(3)]
    ib = rb.step(3)
    rels = " ".join(f"{i['stall_rel']:.2e}" for i in per)
    print(f"  per step: stalled {[i['stalled'] for i in per]}, stall_rel {rels}; one call: "
          f"stalled_total {ib['stalled_total']}, stall_rel {ib['stall_rel']:.2e}", flush=True)
    assert sum(i["stalled"] for i in per) > 0
    assert ib["stalled_total"] == sum(i["stalled"] for i in per)
    assert ib["iters_total"] == sum(i["iters"] for i in per)
    assert ib["stall_rel"] == max(i["stall_rel"] for i in per)
    assert torch.equal(ra.get_state()[1], rb.get_state()[1])


def test_automatic_shrink_matches_the_oracle():
    """rom_adapt_rank(0) with growth ruled out: the pair whose singular value
    of Z~ is 1e-11 of the largest (below rank_tol_down = 1e-8) is dropped,
    R changes by exactly that singular value, and the result matches the
    oracle's shrink; a second call (certificate) keeps the rank."""
    binding, torch = _b()
    w, e = _ens("landau_tiny", N=900)
    _say("automatic shrink")
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=8, dt=w["dt"], fp_tol=1e-12)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    Zt = rom.to_complex_coeff(st.Z)
    Q, sv, Wh = np.linalg.svd(Zt, full_matrices=False)
    sv[-1] = 1e-11 * sv[0]
    st.Z = rom.from_complex_coeff((Q * sv) @ Wh)
    gcfg = binding.make_config(w["N"], w["p"], w["Nx"], 8, two_n_max=12, dt=w["dt"],
                               rank_tol_up=2.0, rank_tol_down=1e-8)
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    X0, V0 = r.reconstruct()
    cfg.two_n_max, cfg.rank_tol_up, cfg.rank_tol_down = 12, 2.0, 1e-8
    status, two_n_o, _ = rom.adapt_rank(st, cfg, 0)
    assert r.adapt_rank(0) == two_n_o == 6
    X1, V1 = r.reconstruct()
    dR = np.sqrt(np.sum(_np(X1 - X0) ** 2) + np.sum(_np(V1 - V0) ** 2))
    np.testing.assert_allclose(dR, sv[-1], rtol=1e-3)
    Xo, Vo = rom.reconstruct(st)
    assert _rel(_np(X1).T, Xo) < RTOL and _rel(_np(V1).T, Vo) < RTOL
    UX, Z, _ = r.get_state()
    Ut = _np(UX).T[:, :3] - 1j * _np(UX).T[:, 3:]
    assert np.abs(Ut.conj().T @ Ut - np.eye(3)).max() < 1e-12
    assert r.adapt_rank(0) == 6


def test_automatic_shrink_inside_the_step():
    """rank_auto with growth ruled out on the tiny Landau ensemble (p = 4 < n
    = 5: Z~ has rank 4): after the first step the fifth pair is dropped, as
    in the oracle's run (prk_step then adapt_rank(0))."""
    binding, torch = _b()
    w, e = _ens("landau_tiny", N=3001)
    _say("automatic shrink in the step")
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=10, dt=w["dt"], fp_tol=1e-10,
                        rank_auto=True, rank_tol_up=2.0, rank_tol_down=1e-8)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    gcfg = binding.make_config(w["N"], w["p"], w["Nx"], 10, dt=w["dt"], fp_tol=1e-10,
                               rank_auto=True, rank_tol_up=2.0, rank_tol_down=1e-8)
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    for s in range(3):
        info = r.step(1)
        assert rom.prk_step(st, cfg) == rom.OK
        _, two_n_o, eps = rom.adapt_rank(st, cfg, 0)
        print(f"  step {s}: 2n {info['two_n']}/{two_n_o}, shrunk {info['shrunk']}", flush=True)
        assert info["two_n"] == two_n_o
        assert info["shrunk"] == (1 if s == 0 else 0)
    X, V = r.reconstruct()
    Xo, Vo = rom.reconstruct(st)
    ex, ev = _rel(_np(X).T, Xo), _rel(_np(V).T, Vo)
    print(f"  R rel err {ex:.2e} {ev:.2e}", flush=True)
    assert ex < 1e-9 and ev < 1e-9


def test_reconstruct_rows():
    binding, torch = _b()
    w, e = _ens("twostream_deim", N=5000, p=16, Nx=64)
    _say("reconstruct rows")
    r = binding.Rom(binding.make_config(w["N"], w["p"], w["Nx"], 10, dt=w["dt"]), e["L"],
                    e["X0"], e["V0"])
    X, V = r.reconstruct()
    rows = np.array([0, 4999, 17, 17, 2500, 5000, -1], dtype=np.int32)
    Xs, Vs = r.reconstruct_rows(rows)
    ok = (rows >= 0) & (rows < 5000)
    assert torch.equal(Xs[:, ok], X[:, rows[ok]]) and torch.equal(Vs[:, ok], V[:, rows[ok]])
    assert torch.isnan(Xs[:, ~ok]).all() and torch.isnan(Vs[:, ~ok]).all()


@pytest.mark.parametrize("kw,two_n,k_full,n_up,steps", [
    # 9 steps: at the tenth, a 1e-15 perturbation of Z flips the cell of a
    # sampled particle in the oracle and its sensitivity jumps from 8e-8 to
    # 5e-6, which would make the bound meaningless
    (dict(N=20000, p=24, Nx=128), 10, 3, 4, 9),
    (dict(N=30000, p=64, Nx=128), 12, 2, 5, 8),
])
def test_adaptive_deim_parity(kw, two_n, k_full, n_up, steps):
    """Adaptive DEIM index updates (Sec. 4.2.2, eq. indices_adaptive_DEIM):
    every k_full-th operator by the full greedy, in between n_up positions of
    the most rotated basis vectors chosen again.  Same iteration counts and
    indices as the oracle (where its greedy margin allows), R within the DEIM
    bound."""
    binding, torch = _b()
    w, e = _ens("twostream_deim", **kw)
    _say("adaptive deim", kw, two_n, k_full, n_up, steps)
    cfg = rom.RomConfig(N=w["N"], p=w["p"], Nx=w["Nx"], two_n=two_n, dt=w["dt"], fp_tol=1e-10,
                        projection="deim", deim_window=3, deim_update_every=k_full,
                        deim_update_rows=n_up)
    st = rom.init_state(e["X0"], e["V0"], e["L"], cfg)
    gcfg = binding.make_config(w["N"], w["p"], w["Nx"], two_n, dt=w["dt"], fp_tol=1e-10,
                               projection="deim", deim_window=3, deim_update_every=k_full,
                               deim_update_rows=n_up)
    # the oracle's own sensitivity over the same steps, of X_r and of V_r
    # apart: Z perturbed by 1e-15
    rng = np.random.default_rng(0)
    outs = []
    for pert in (0.0, 1e-15):
        s2 = rom.RomState(U=st.U.copy(), Z=st.Z * (1 + pert * rng.normal(size=st.Z.shape)),
                          L=st.L)
        for _ in range(steps):
            assert rom.prk_step(s2, cfg) == rom.OK
        outs.append(rom.reconstruct(s2))
    sx, sv = _rel(outs[1][0], outs[0][0]), _rel(outs[1][1], outs[0][1])
    r = binding.Rom(gcfg, e["L"], e["X0"], e["V0"])
    _set_from_oracle(r, st, torch)
    same = 0
    for s in range(steps):
        info = r.step(1)
        assert rom.prk_step(st, cfg) == rom.OK
        assert info["iters"] == st.last_iters, (s, info, st.last_iters)
        if st.deim_indices is None:
            continue
        gi = _np(r.deim_operator()[0]).astype(np.int64)
        eq = np.array_equal(gi, st.deim_indices)
        print(f"  step {s}: operator {st.deim_builds - 1}, indices equal {eq}", flush=True)
        same += int(eq)
    assert same >= 3
    X, V = r.reconstruct()
    Xo, Vo = rom.reconstruct(st)
    ex, ev = _rel(_np(X).T, Xo), _rel(_np(V).T, Vo)
    bx, bv = max(1e-9, 50.0 * sx), max(1e-9, 50.0 * sv)
    print(f"  X_r rel err {ex:.2e} (sensitivity {sx:.2e}, bound {bx:.2e}); V_r rel err "
          f"{ev:.2e} (sensitivity {sv:.2e}, bound {bv:.2e})", flush=True)
    assert ex < bx and ev < bv
