"""Pins of the DEIM oracle: interpolation property, exactness on the DEIM
space, the Chaturantabut-Sorensen error bound, and reduction to the
Galerkin gradient when every particle is an interpolation point."""
import numpy as np

from oracle import deim, rom
from workloads import make_ensemble, workload


def test_interpolation_property_and_exactness():
    rng = np.random.default_rng(0)
    N, d = 50, 6
    Psi, _ = np.linalg.qr(rng.normal(size=(N, d)))
    idx = deim.greedy_indices(Psi)
    assert len(set(idx.tolist())) == d
    P = np.eye(N)[:, idx]
    proj = Psi @ np.linalg.solve(P.T @ Psi, P.T)
    f = rng.normal(size=N)
    # the DEIM approximation interpolates f on the selected indices
    np.testing.assert_allclose((proj @ f)[idx], f[idx], atol=1e-12)
    # and is exact on span(Psi)
    c = rng.normal(size=d)
    np.testing.assert_allclose(proj @ (Psi @ c), Psi @ c, atol=1e-12)
    # error bound ||f - Df|| <= ||(P^T Psi)^{-1}|| ||(I - Psi Psi^T) f||
    bound = np.linalg.norm(np.linalg.inv(P.T @ Psi), 2) * np.linalg.norm(f - Psi @ (Psi.T @ f))
    assert np.linalg.norm(f - proj @ f) <= bound * (1 + 1e-12)


def test_greedy_first_index_and_ties():
    """The first index is the largest entry of psi_1; ties go to the
    smallest index."""
    Psi = np.array([[0.5, 0.1], [-0.5, 0.7], [0.5, 0.1], [0.5, -0.7]])
    Psi[:, 1] -= Psi[:, 0] * (Psi[:, 0] @ Psi[:, 1])
    idx = deim.greedy_indices(Psi)
    assert idx[0] == 0
    assert idx[1] != 0


def test_full_deim_reduces_to_galerkin():
    """d = N: P is a permutation, w = 1 and the DEIM gradient is the Galerkin
    gradient exactly (eq. grHDD against eq. grads)."""
    N = 40
    w = workload("twostream_deim", N=N, p=12, Nx=16)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=12, Nx=16, two_n=6, dt=0.05)
    st = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    gr = rom.gradient(st.U, st.Z, st.L, 16)
    rng = np.random.default_rng(1)
    Y = rng.normal(size=(N, 3 * N))
    op = deim.build_operator(Y, N)
    assert sorted(op.idx.tolist()) == list(range(N))
    np.testing.assert_allclose(op.w, np.ones(N), atol=1e-10)
    g = deim.deim_gradient(st.U, st.Z, gr, op, cfg)
    np.testing.assert_allclose(g, gr.g, atol=1e-10 * np.abs(gr.g).max())


def test_snapshot_is_potential_at_particles():
    """Lambda^0(X) Phi interpolates the nodal potential linearly."""
    from oracle import pic
    L = np.array([8.0])
    Phi = np.arange(8.0)[:, None] ** 2
    X = np.array([[0.0], [0.5], [3.25], [7.5], [8.5]])
    y = deim.snapshot(X, Phi, L)
    np.testing.assert_allclose(y[:, 0], [0.0, 0.5, 9 + 0.25 * 7, 49 + 0.5 * (0 - 49), 0.5])
    # against the brute-force dense Lambda^0
    Lam = pic.lambda0_dense(X[:, 0], 8.0, 8)
    np.testing.assert_allclose(y[:, 0], Lam @ Phi[:, 0], atol=1e-14)


def test_deim_rom_runs_and_switches_after_window():
    N = 600
    w = workload("twostream_deim", N=N, p=16, Nx=32)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=16, Nx=32, two_n=6, dt=0.05, projection="deim",
                        deim_window=3, fp_tol=1e-11)
    st = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    for s in range(6):
        assert rom.prk_step(st, cfg) == rom.OK
        if s < 3:
            assert st.deim_indices is None
        else:
            assert st.deim_indices is not None and len(st.deim_indices) == 6


def test_snapshot_parameter_subset():
    """p* (T+1) covers the largest DEIM dimension d = two_n_max; the subset is
    evenly spaced and starts at the first parameter."""
    for p, cap, T in ((64, 60, 3), (16, 10, 3), (4, 10, 3), (300, 8, 5)):
        sub = deim.snapshot_params(p, cap, T)
        assert sub[0] == 0 and len(set(sub.tolist())) == len(sub)
        assert len(sub) == min(p, max(8, -(-cap // (T + 1))))
        assert np.all(np.diff(sub) > 0) and sub[-1] < p


def _greedy_by_determinants(Psi):
    """An independent characterisation of the greedy choice (Sec. 4.2.2):
    with the first k-1 indices fixed, the k-th maximises over j the volume
    |det Psi[I_{k-1} + (j), :k]|.  By the Schur complement that determinant is
    det(P^T Psi_{k-1}) times the interpolation residual r_k(j), so maximising
    one maximises the other; no solve of the greedy's linear system is used.
    Returns the indices and the ratio of the runner-up to the winner at each
    step (to keep away from near ties)."""
    N, d = Psi.shape
    idx, margins = [], []
    for k in range(d):
        vols = np.array([abs(np.linalg.det(Psi[idx + [j], :k + 1])) if j not in idx else -1.0
                         for j in range(N)])
        order = np.argsort(-vols, kind="stable")
        idx.append(int(order[0]))
        margins.append(vols[order[1]] / vols[order[0]])
    return np.array(idx), np.array(margins)


def test_greedy_matches_determinant_maximisation():
    """Brute force on tiny inputs for every k >= 1: the oracle's greedy
    indices equal the successive maximisers of the interpolation volume.  A
    greedy that took argmax |psi_k| instead of the residual's argmax (or
    skipped the solve) fails here: the seeds below include cases where the
    two rules disagree, which the test checks it has seen."""
    rng = np.random.default_rng(7)
    disagree = 0
    cases = 0
    while cases < 40:
        N = int(rng.integers(6, 13))
        d = int(rng.integers(2, 6))
        Psi, _ = np.linalg.qr(rng.normal(size=(N, d)))
        ref, margin = _greedy_by_determinants(Psi)
        if margin.max() > 1 - 1e-6:
            continue          # a near tie: any rule may pick either index
        cases += 1
        got = deim.greedy_indices(Psi)
        assert np.array_equal(got, ref), (got, ref)
        naive = [int(np.argmax(np.where(np.isin(np.arange(N), ref[:k]), -1.0,
                                        np.abs(Psi[:, k])))) for k in range(d)]
        disagree += int(naive != ref.tolist())
    assert disagree >= 10, disagree


def test_greedy_hand_worked_example():
    """A 4 x 3 basis worked by hand (Sec. 4.2.2 greedy):
      psi_1 = (1, 3, 2, 0):       l_1 = 1 (|3| largest).
      psi_2 = (1.5, 9, 7, 2.5):   c = psi_2[1] / psi_1[1] = 3,
                                  r_2 = psi_2 - 3 psi_1 = (-1.5, 0, 1, 2.5), l_2 = 3
                                  (not 2, the largest unselected entry of psi_2).
      psi_3 = (4, 3, 1, 5):       [[3, 9], [0, 2.5]] c = (3, 5) gives c = (-5, 2),
                                  r_3 = psi_3 + 5 psi_1 - 2 psi_2 = (6, 0, -3, 0), l_3 = 0.
    The weights w = (P^T Psi)^{-T} Psi^T 1 solve the transposed system for
    Psi^T 1 = (6, 20, 13)."""
    Psi = np.array([[1.0, 1.5, 4.0], [3.0, 9.0, 3.0], [2.0, 7.0, 1.0], [0.0, 2.5, 5.0]])
    assert deim.greedy_indices(Psi).tolist() == [1, 3, 0]
    # P^T Psi rows (1, 3, 0): [[3, 9, 3], [0, 2.5, 5], [1, 1.5, 4]]; by hand,
    # (P^T Psi)^T w = (6, 20, 13):  3 w1 + w3 = 6,  9 w1 + 2.5 w2 + 1.5 w3 = 20,
    # 3 w1 + 5 w2 + 4 w3 = 13  ->  18 w1 = 33, so w = (11/6, 1.1, 0.5)
    w = deim.weights(Psi, np.array([1, 3, 0]))
    np.testing.assert_allclose(w, [11.0 / 6.0, 1.1, 0.5], rtol=1e-14)
    A = Psi[[1, 3, 0], :]
    # the DEIM interpolant of the constant 1 reproduces 1 on the selected rows
    proj = Psi @ np.linalg.solve(A, np.ones(3))
    assert np.allclose(proj[[1, 3, 0]], 1.0, atol=1e-13)


def test_greedy_with_kept_reduces_to_the_greedy():
    """Nothing kept: the adaptive selection is the full greedy."""
    rng = np.random.default_rng(11)
    for _ in range(10):
        Psi, _ = np.linalg.qr(rng.normal(size=(40, 7)))
        assert np.array_equal(deim.greedy_with_kept(Psi, [None] * 7), deim.greedy_indices(Psi))


def test_greedy_with_kept_maximises_the_volume_at_free_positions():
    """Brute force (Sec. 4.2.2, eq. indices_adaptive_DEIM): kept positions keep
    their index; each free position takes the maximiser over j of
    |det Psi[I_{k-1} + (j), :k]| given the indices before it (the Schur
    complement identity of the greedy pin above), and a kept index already
    chosen is chosen again."""
    rng = np.random.default_rng(12)
    cases = 0
    while cases < 30:
        N = int(rng.integers(8, 14))
        d = int(rng.integers(3, 6))
        Psi, _ = np.linalg.qr(rng.normal(size=(N, d)))
        kept = [int(rng.integers(0, N)) if rng.random() < 0.5 else None for _ in range(d)]
        got = deim.greedy_with_kept(Psi, kept)
        ok = True
        for k in range(d):
            prev = got[:k].tolist()
            if kept[k] is not None and kept[k] not in prev:
                assert got[k] == kept[k]
                continue
            vols = np.array([abs(np.linalg.det(Psi[prev + [j], :k + 1])) if j not in prev else -1.0
                             for j in range(N)])
            order = np.argsort(-vols, kind="stable")
            if vols[order[1]] > (1 - 1e-6) * vols[order[0]]:
                ok = False      # a near tie: either index is right
                break
            assert got[k] == order[0], (k, got, order[:3])
        cases += int(ok)
    # a kept index equal to an earlier choice is chosen again
    Psi, _ = np.linalg.qr(rng.normal(size=(12, 3)))
    first = deim.greedy_indices(Psi)[0]
    got = deim.greedy_with_kept(Psi, [None, int(first), None])
    assert len(set(got.tolist())) == 3


def test_update_positions_hand_example():
    """Columns rotated by 10, 60, 30 and 80 degrees (and one sign flip): the
    two most rotated are positions 1 and 3; the flipped column counts as not
    rotated."""
    ang = np.radians([10.0, 60.0, 30.0, 80.0, 0.0])
    old = np.zeros((10, 5))
    new = np.zeros((10, 5))
    for k, a in enumerate(ang):
        old[2 * k, k] = 1.0
        new[2 * k, k] = np.cos(a)
        new[2 * k + 1, k] = np.sin(a)
    new[:, 4] *= -1.0
    assert deim.update_positions(new, old, 2) == {1, 3}
    assert deim.update_positions(new, old, 0) == set()


def test_adaptive_deim_schedule():
    """k_DEIM = 3, n_DEIM = 2: operators 0 and 3 by the full greedy; in
    between, every position outside the two most rotated inherits its index
    (unless that index was already taken)."""
    N = 600
    w = workload("twostream_deim", N=N, p=12, Nx=32)
    ens = make_ensemble(w)
    cfg = rom.RomConfig(N=N, p=12, Nx=32, two_n=6, dt=0.05, projection="deim",
                        deim_window=2, fp_tol=1e-10, deim_update_every=3, deim_update_rows=2)
    st = rom.init_state(ens["X0"], ens["V0"], ens["L"], cfg)
    prev_idx = prev_psi = None
    for s in range(7):
        assert rom.prk_step(st, cfg) == rom.OK
        if st.deim_indices is None:
            continue
        b = st.deim_builds - 1
        if b % 3 == 0:
            assert np.array_equal(st.deim_indices, deim.greedy_indices(st.deim_psi))
        else:
            upd = deim.update_positions(st.deim_psi, prev_psi, 2)
            for k in range(6):
                if k not in upd and prev_idx[k] not in st.deim_indices[:k].tolist():
                    assert st.deim_indices[k] == prev_idx[k]
        prev_idx, prev_psi = st.deim_indices.copy(), st.deim_psi.copy()
    assert st.deim_builds >= 4
