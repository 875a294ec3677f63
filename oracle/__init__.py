"""FP64 CPU oracle for the particle-in-cell full-order model and the dynamical
symplectic reduced model of Hesthaven, Pagliantini and Ripamonti,
"Adaptive symplectic model order reduction of parametric particle-based
Vlasov-Poisson equation" (arXiv:2201.05555).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
never does, and shares no code with it.

It follows the paper's real formulation (2N x 2n bases, explicit Poisson
tensors J), with numpy library primitives (matmul, eigh, QR, SVD, dense
solves, bincount) as steps.  Every function cites the passage it follows.

Parity status of each piece is listed in ``PINS`` below; a piece whose result
no closed form, invariant or brute-force check fixes says "parity unpinned".
"""
from . import pic, rom, deim, dmd  # noqa: F401

PINS = {
    "pic.cell_index": "brute force on tiny inputs; node ties",
    "pic.deposit": "total charge = q w N, partition of unity; dense Lambda0 brute force",
    "pic.poisson": "single cosine mode closed form; residual of the stiffness system",
    "pic.field / gradient": "central finite difference of the discrete Hamiltonian",
    "pic.energy": "Phi^T rho = Phi^T L Phi identity",
    "pic.fom_step": "observed order 2, time reversibility, bounded energy error, Landau rate",
    "rom.init_csvd": "Eckart-Young: truncation error = tail singular values",
    "rom.basis_velocity": "real form equals complex form; tangency U^T X = 0",
    "rom.cayley": "Woodbury form equals the dense Cayley transform; orthosymplecticity",
    "rom.tangent_velocity": "Y(0,Z) = X(U0,Z); central FD of the retraction",
    "rom.prk_step": "2n = 2N reduces to implicit midpoint on the full model; order 2; "
                    "gauge covariance; orthosymplecticity after each step",
    "rom.reorthonormalise": "R = UZ unchanged; U^T U = I",
    "rom.rank_grow": "R bitwise unchanged (zero coefficient rows)",
    "rom.rank_shrink": "removed energy equals dropped singular values",
    "rom.rank_indicator": "identity ||(I - U U^T) J G||^2 = ||G||^2 - ||g||^2",
    "rom.local_singular_values / numerical_rank": "a matrix built with prescribed singular "
                                                  "values (random orthogonal factors); rank "
                                                  "counts by hand",
    "rom.hamiltonian_split": "complete basis (2n = 2N): the basis does not move, both basis "
                             "terms vanish; the end rows equal the Hamiltonians of the states "
                             "before and after the step",
    "rom.rank_policy": "parity unpinned (grow/shrink thresholds are a reading; the paper defers "
                       "rank adaptation)",
    "rom.fixed_point_stagnation": "parity unpinned (a reading); the floor is pinned by a planted "
                                  "2-cycle that must end in ENOCONV",
    "deim.greedy": "brute force on tiny inputs for every k: each index maximises the "
                   "interpolation volume |det Psi[I, :k]|; a hand-worked 4 x 3 example",
    "deim.weights": "hand-worked 4 x 3 example; interpolation of the constant 1",
    "deim.greedy_with_kept": "brute force on tiny inputs: kept positions keep their index, free "
                             "ones maximise the interpolation volume; nothing kept = the greedy",
    "deim.update_positions": "hand-worked rotations (10, 60, 30, 80 degrees and a sign flip)",
    "deim.gradient": "d = N reduces exactly to the Galerkin gradient",
    "deim.accuracy_with_exact_potential": "parity unpinned (no printed values)",
    "dmd.select_subset": "brute force of every greedy pick (eq. pSampl); gauge invariance",
    "dmd.dmd / dmd.predict": "exactly linear data: eigenvalues (a damped rotation and real "
                             "ones) and the prediction at 0, dt/2, dt, 2 dt against the closed-form "
                             "principal powers; relative truncation; untruncated DMD reproduces "
                             "the last potential",
    "dmd.rbf_interpolate": "scipy RBFInterpolator (gaussian, no polynomial); interpolation at "
                           "the nodes; width and scaling by hand",
    "dmd.build_operator": "subset coordinates = Theta^+ Phi; others = the scipy interpolant",
    "rom.dmd_deim_gradient": "central finite difference of the DMD-DEIM Hamiltonian through the "
                             "brute-force Lambda^0",
    "rom.prk_step (dmd_deim)": "the first T steps equal the plain reduced model bit for bit; "
                               "ENOCONV restores both windows",
    "dmd.accuracy": "parity unpinned (the paper prints no values for it)",
}
