"""ctypes binding of the symrom C ABI (include/symrom.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch CUDA tensors; the library's column-major N x p arrays
are tensors of shape (p, N), U_X (N x 2n) is (2n, N), Z (2n x p) is (p, 2n)
and the grids (Nx x p) are (p, Nx).  The library is loaded from
``lib/libsymrom.so`` next to this file; if it is missing, every entry point
raises (there is no CPU fallback).
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libsymrom.so")

OK, EINVAL, ENOMEM, ESINGULAR, ENOCONV, EDEVICE, ESTATE, ERANKCAP = 0, -1, -2, -3, -4, -5, -6, -7
GALERKIN, DEIM, DMD_DEIM = 0, 1, 2
PROJECTIONS = {"galerkin": GALERKIN, "deim": DEIM, "dmd_deim": DMD_DEIM}
FAMILIES = {"deposit": 0, "gather": 1, "poisson": 2, "fom_push": 3, "basis": 4, "dense": 5,
            "deim_eig": 6, "gather_xi": 7, "deim_chain": 8, "dmd_chain": 9, "dmd_fixed_point": 10}


class SymromError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"symrom status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("p", ctypes.c_int32), ("Nx", ctypes.c_int32),
        ("two_n", ctypes.c_int32), ("two_n_max", ctypes.c_int32),
        ("dt", ctypes.c_double), ("q", ctypes.c_double), ("m", ctypes.c_double),
        ("projection", ctypes.c_int32), ("deim_window", ctypes.c_int32),
        ("fp_tol", ctypes.c_double), ("fp_max_iters", ctypes.c_int32),
        ("fp_fixed_iters", ctypes.c_int32), ("pinv_rtol", ctypes.c_double),
        ("reorth", ctypes.c_int32), ("rank_auto", ctypes.c_int32),
        ("rank_tol_up", ctypes.c_double), ("fp_stall_tol", ctypes.c_double),
        ("rank_tol_down", ctypes.c_double), ("deim_rows", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("deterministic", ctypes.c_int32),
        ("deim_update_every", ctypes.c_int32), ("deim_update_rows", ctypes.c_int32),
        ("p_star", ctypes.c_int32), ("reserved", ctypes.c_int32), ("dmd_tol", ctypes.c_double),
    ]


class StepInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("stalled", ctypes.c_int32), ("two_n", ctypes.c_int32),
        ("deim_active", ctypes.c_int32), ("rank_indicator", ctypes.c_double),
        ("iters_total", ctypes.c_int32), ("deim_steps", ctypes.c_int32),
        ("stall_rel", ctypes.c_double), ("stalled_total", ctypes.c_int32),
        ("shrunk", ctypes.c_int32), ("worst_rel", ctypes.c_double),
        ("unconverged", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class RequestInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("two_n", ctypes.c_int32), ("steps_done", ctypes.c_int64),
        ("t_arrival", ctypes.c_double), ("t_start", ctypes.c_double),
        ("t_finish", ctypes.c_double), ("pp_steps", ctypes.c_double),
    ]


_VP = ctypes.c_void_p
_SIGS = {
    "rom_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
    "rom_init": (ctypes.c_int32, [ctypes.POINTER(Config), _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP,
                                  ctypes.POINTER(_VP)]),
    "rom_init_family": (ctypes.c_int32, [ctypes.POINTER(Config), ctypes.c_int32, _VP, _VP, _VP,
                                         _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "fom_init_family": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int32, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP,
                                         ctypes.POINTER(_VP)]),
    "symrom_load_family": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                            _VP, _VP, _VP, _VP, _VP]),
    "rom_step": (ctypes.c_int32, [_VP, ctypes.c_int32, ctypes.POINTER(StepInfo)]),
    "rom_adapt_rank": (ctypes.c_int32, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "rom_set_fixed_point": (ctypes.c_int32, [_VP, ctypes.c_double, ctypes.c_int32,
                                             ctypes.c_int32]),
    "rom_get_state": (ctypes.c_int32, [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "rom_set_state": (ctypes.c_int32, [_VP, ctypes.c_int32, _VP, _VP, ctypes.c_int64]),
    "rom_reconstruct": (ctypes.c_int32, [_VP, _VP, _VP]),
    "rom_reconstruct_rows": (ctypes.c_int32, [_VP, _VP, ctypes.c_int32, _VP, _VP]),
    "rom_cells": (ctypes.c_int32, [_VP, _VP, _VP, _VP]),
    "rom_deim_operator": (ctypes.c_int32, [_VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32)]),
    "rom_set_parameters": (ctypes.c_int32, [_VP, _VP, ctypes.c_int32]),
    "rom_dmd_state": (ctypes.c_int32, [_VP, _VP, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), _VP, _VP, _VP]),
    "deim_select_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "deim_select": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP, _VP,
                                     ctypes.c_size_t, _VP]),
    "rom_diagnostics": (ctypes.c_int32, [_VP, _VP, _VP]),
    "rom_init_singular_values": (ctypes.c_int32, [_VP, _VP, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_int32)]),
    "rom_autotune": (ctypes.c_int32, [_VP] + [ctypes.POINTER(ctypes.c_int32)] * 3
                     + [ctypes.POINTER(ctypes.c_double)] * 2),
    "rom_hamiltonian_split_bytes": (ctypes.c_size_t, [_VP]),
    "rom_step_hamiltonian_split": (ctypes.c_int32, [_VP, _VP, ctypes.c_size_t, _VP,
                                                    ctypes.POINTER(StepInfo)]),
    "rom_gradient": (ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "rom_destroy": (None, [_VP]),
    "fom_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32] * 3),
    "fom_init": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, _VP, _VP, _VP, _VP,
                                  ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "fom_step": (ctypes.c_int32, [_VP, ctypes.c_int32]),
    "fom_get_state": (ctypes.c_int32, [_VP, _VP, _VP]),
    "fom_diagnostics": (ctypes.c_int32, [_VP, _VP, _VP]),
    "fom_destroy": (None, [_VP]),
    "pic_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32] * 3),
    "pic_fields": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                    ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t,
                                    _VP]),
    "pic_fields_noalloc": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                            ctypes.c_double, _VP, _VP, _VP, _VP, _VP, _VP]),
    "srv_request_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config), ctypes.c_int32]),
    "srv_create": (ctypes.c_int32, [ctypes.c_int32, _VP, ctypes.c_size_t, ctypes.POINTER(_VP)]),
    "srv_submit": (ctypes.c_int32, [_VP, ctypes.POINTER(Config), ctypes.c_int32, _VP, _VP, _VP,
                                    ctypes.c_int32, ctypes.c_int32, _VP,
                                    ctypes.POINTER(ctypes.c_int64)]),
    "srv_info": (ctypes.c_int32, [_VP, ctypes.c_int64, ctypes.POINTER(RequestInfo)]),
    "srv_wait": (ctypes.c_int32, [_VP, ctypes.c_int64]),
    "srv_drain": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_double)]),
    "srv_result": (ctypes.c_int32, [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP]),
    "srv_destroy": (None, [_VP]),
    "symrom_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "symrom_last_error": (ctypes.c_char_p, []),
    "symrom_set_timing": (None, [ctypes.c_int32]),
    "symrom_kernel_ms": (ctypes.c_double, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "symrom_kernel_work": (None, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status):
    if status != OK:
        msg = lib().symrom_last_error().decode()
        raise SymromError(status, msg)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host_doubles(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def set_timing(on):
    lib().symrom_set_timing(1 if on else 0)


def kernel_ms(family):
    """(total ms, launches) of a kernel family since the last query."""
    n = ctypes.c_int64(0)
    ms = lib().symrom_kernel_ms(FAMILIES[family], ctypes.byref(n))
    return ms, n.value


def kernel_work(family):
    """(algorithmic flops, algorithmic HBM bytes) of the timed launches."""
    f = ctypes.c_double(0.0)
    b = ctypes.c_double(0.0)
    lib().symrom_kernel_work(FAMILIES[family], ctypes.byref(f), ctypes.byref(b))
    return f.value, b.value


def make_config(N, p, Nx, two_n, two_n_max=None, dt=0.05, q=-1.0, m=1.0, projection="galerkin",
                deim_window=3, fp_tol=1e-9, fp_max_iters=100, fp_fixed_iters=0, pinv_rtol=1e-12,
                reorth=True, rank_auto=False, rank_tol_up=1e-2, fp_stall_tol=1e-3,
                rank_tol_down=1e-8, deim_rows=0, deterministic=False, deim_update_every=1,
                deim_update_rows=0, p_star=0, dmd_tol=1e-5):
    return Config(N=N, p=p, Nx=Nx, two_n=two_n, two_n_max=two_n_max or two_n, dt=dt, q=q, m=m,
                  projection=PROJECTIONS[projection],
                  deim_window=deim_window, fp_tol=fp_tol, fp_max_iters=fp_max_iters,
                  fp_fixed_iters=fp_fixed_iters, pinv_rtol=pinv_rtol, reorth=int(reorth),
                  rank_auto=int(rank_auto), rank_tol_up=rank_tol_up, fp_stall_tol=fp_stall_tol,
                  rank_tol_down=rank_tol_down, deim_rows=deim_rows, precision=0,
                  deterministic=int(deterministic), deim_update_every=deim_update_every,
                  deim_update_rows=deim_update_rows, p_star=p_star, reserved=0,
                  dmd_tol=dmd_tol)


def _info_dict(info):
    return dict(iters=info.iters, stalled=info.stalled, two_n=info.two_n,
                deim_active=info.deim_active, rank_indicator=info.rank_indicator,
                iters_total=info.iters_total, deim_steps=info.deim_steps,
                stall_rel=info.stall_rel, stalled_total=info.stalled_total, shrunk=info.shrunk,
                worst_rel=info.worst_rel, unconverged=info.unconverged)


def _dev1(x):
    """1-D host or device array -> contiguous FP64 device tensor."""
    if isinstance(x, torch.Tensor):
        return x.to(dtype=torch.float64, device="cuda").contiguous()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64))).cuda()


def load_family(family, params, ux, uv, stream=None):
    """Initial states X, V (p, N) device tensors of an ensemble, loaded on the
    device (symrom_load_family)."""
    eta = torch.from_numpy(eta_array(params)).cuda()
    uxd, uvd = _dev1(ux), _dev1(uv)
    N, p = uxd.numel(), eta.shape[0]
    X = torch.empty((p, N), dtype=torch.float64, device="cuda")
    V = torch.empty_like(X)
    _check(lib().symrom_load_family(FAMILY[family], N, p, _ptr(eta), _ptr(uxd), _ptr(uvd),
                                    _ptr(X), _ptr(V), _stream(stream)))
    return X, V


def _dev(x, device="cuda"):
    """(N, p) numpy -> (p, N) contiguous device tensor (column-major N x p)."""
    if isinstance(x, torch.Tensor):
        return x.contiguous()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64).T)).to(device)


FAMILY = {"landau": 0, "twostream": 1}


def eta_array(params):
    """p x 4 host array (alpha, k, v0, sigma) from a parameter dict."""
    return np.ascontiguousarray(np.stack([params["alpha"], params["k"], params["v0"],
                                          params["sigma"]], axis=1), dtype=np.float64)


class Rom:
    """Reduced-model handle (rom_* entry points).  With X0 = None the initial
    ensemble is loaded on the device (rom_init_family): pass family, params
    (dict of alpha, k, v0, sigma arrays) and the shared uniforms ux, uv."""

    def __init__(self, cfg, L, X0, V0, stream=None, family=None, params=None, ux=None, uv=None):
        self.cfg = cfg
        self.stream = stream
        nbytes = lib().rom_workspace_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            raise SymromError(EINVAL, "invalid configuration")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        if X0 is None:
            eta = eta_array(params)
            self.L = 2.0 * np.pi / np.asarray(params["k"], dtype=np.float64)
            uxd, uvd = _dev1(ux), _dev1(uv)
            _check(lib().rom_init_family(ctypes.byref(cfg), FAMILY[family],
                                         eta.ctypes.data_as(ctypes.c_void_p), _ptr(uxd),
                                         _ptr(uvd), _ptr(self.ws), nbytes, _stream(stream),
                                         ctypes.byref(h)))
        else:
            self.L = np.asarray(L, dtype=np.float64).copy()
            X0, V0 = _dev(X0), _dev(V0)
            Lh, Lp = _host_doubles(self.L)
            _check(lib().rom_init(ctypes.byref(cfg), Lp, _ptr(X0), _ptr(V0), _ptr(self.ws),
                                  nbytes, _stream(stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().rom_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def two_n(self):
        t = ctypes.c_int32()
        _check(lib().rom_get_state(self.h, None, None, ctypes.byref(t), None))
        return t.value

    def step(self, nsteps=1):
        info = StepInfo()
        _check(lib().rom_step(self.h, nsteps, ctypes.byref(info)))
        return _info_dict(info)

    def step_status(self, nsteps=1):
        info = StepInfo()
        st = lib().rom_step(self.h, nsteps, ctypes.byref(info))
        return st, _info_dict(info)

    def set_fixed_point(self, fp_tol, fp_max_iters=100, fp_fixed_iters=0):
        _check(lib().rom_set_fixed_point(self.h, fp_tol, fp_max_iters, fp_fixed_iters))

    def adapt_rank(self, target=0):
        out = ctypes.c_int32()
        _check(lib().rom_adapt_rank(self.h, target, ctypes.byref(out)))
        return out.value

    def get_state(self):
        r = self.two_n
        UX = torch.empty((r, self.cfg.N), dtype=torch.float64, device="cuda")
        Z = torch.empty((self.cfg.p, r), dtype=torch.float64, device="cuda")
        step = ctypes.c_int64()
        _check(lib().rom_get_state(self.h, _ptr(UX), _ptr(Z), None, ctypes.byref(step)))
        return UX, Z, step.value

    def set_state(self, UX, Z, step=0):
        UX = UX.contiguous()
        Z = Z.contiguous()
        _check(lib().rom_set_state(self.h, UX.shape[0], _ptr(UX), _ptr(Z), step))

    def reconstruct(self):
        X = torch.empty((self.cfg.p, self.cfg.N), dtype=torch.float64, device="cuda")
        V = torch.empty_like(X)
        _check(lib().rom_reconstruct(self.h, _ptr(X), _ptr(V)))
        return X, V

    def reconstruct_rows(self, rows):
        """X_r, V_r of the listed particle rows: tensors (p, len(rows))."""
        rows = torch.as_tensor(np.asarray(rows, dtype=np.int32)).cuda()
        nr = rows.numel()
        X = torch.empty((self.cfg.p, nr), dtype=torch.float64, device="cuda")
        V = torch.empty_like(X)
        _check(lib().rom_reconstruct_rows(self.h, _ptr(rows), nr, _ptr(X), _ptr(V)))
        return X, V

    def cells(self, Z=None):
        """Cells (p, N) int32 and scaled positions s (p, N) of the fused kernels."""
        cells = torch.empty((self.cfg.p, self.cfg.N), dtype=torch.int32, device="cuda")
        sv = torch.empty((self.cfg.p, self.cfg.N), dtype=torch.float64, device="cuda")
        Zp = _ptr(Z.contiguous()) if Z is not None else None
        _check(lib().rom_cells(self.h, Zp, _ptr(cells), _ptr(sv)))
        return cells, sv

    def deim_operator(self):
        """(indices int32 (d,), weights (d,)) of the last DEIM step."""
        idx = torch.empty(64, dtype=torch.int32, device="cuda")
        w = torch.empty(64, dtype=torch.float64, device="cuda")
        d = ctypes.c_int32()
        _check(lib().rom_deim_operator(self.h, _ptr(idx), _ptr(w), ctypes.byref(d)))
        return idx[: d.value], w[: d.value]

    def autotune(self):
        """Time the launch shapes of the fused gather-projection for this
        handle's sizes and keep the fastest (process-wide): dict of the shape
        kept and the times per launch (ms) of it and of the built-in rule."""
        c, e, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        tb, tr = ctypes.c_double(), ctypes.c_double()
        _check(lib().rom_autotune(self.h, ctypes.byref(c), ctypes.byref(e), ctypes.byref(nb),
                                  ctypes.byref(tb), ctypes.byref(tr)))
        return dict(params_per_tile=16 * c.value, table_in_lds=bool(e.value),
                    row_blocks_max=nb.value, ms=tb.value, rule_ms=tr.value)

    def step_hamiltonian_split(self):
        """One step with the four Hamiltonians of eq. error_ham_tot: (info,
        H4 (4, p) device tensor: H(U_{tau-1} Z_{tau-1}), H(U_{tau-1/2}
        Z_{tau-1}), H(U_{tau-1/2} Z_tau), H(U_tau Z_tau))."""
        nb = lib().rom_hamiltonian_split_bytes(self.h)
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        off = (-scratch.data_ptr()) % 256
        H4 = torch.empty((4, self.cfg.p), dtype=torch.float64, device="cuda")
        info = StepInfo()
        _check(lib().rom_step_hamiltonian_split(self.h, ctypes.c_void_p(scratch.data_ptr() + off),
                                                nb, _ptr(H4), ctypes.byref(info)))
        return _info_dict(info), H4

    def init_singular_values(self):
        """Singular values (numpy, decreasing) of the initial state the
        handle decomposed: all p for p <= 64, the n leading ones beyond."""
        m = ctypes.c_int32()
        _check(lib().rom_init_singular_values(self.h, None, 0, ctypes.byref(m)))
        sig = np.zeros(max(1, m.value), dtype=np.float64)
        _check(lib().rom_init_singular_values(self.h, sig.ctypes.data_as(ctypes.c_void_p),
                                              m.value, ctypes.byref(m)))
        return sig[: m.value]

    def set_parameters(self, eta):
        """Parameters of the ensemble (dim x p host array, e.g. rows alpha, k,
        v0, sigma) for the radial basis interpolation of DMD-DEIM."""
        eta = np.ascontiguousarray(np.asarray(eta, dtype=np.float64).T)
        _check(lib().rom_set_parameters(self.h, eta.ctypes.data_as(ctypes.c_void_p),
                                        eta.shape[1]))

    def dmd_state(self):
        """(subset S (numpy int), DMD rank r, eigenvalues (numpy complex, r),
        field tables e0, eh (p, Nx) device tensors) of the last DMD-DEIM step."""
        S = np.zeros(64, dtype=np.int32)
        ps = ctypes.c_int32()
        rk = ctypes.c_int32()
        lam = np.zeros(2 * 64, dtype=np.float64)
        e0 = torch.empty((self.cfg.p, self.cfg.Nx), dtype=torch.float64, device="cuda")
        eh = torch.empty_like(e0)
        _check(lib().rom_dmd_state(self.h, S.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ps),
                                   ctypes.byref(rk), lam.ctypes.data_as(ctypes.c_void_p),
                                   _ptr(e0), _ptr(eh)))
        r = rk.value
        return (S[: ps.value].astype(np.int64), r, lam[0:2 * r:2] + 1j * lam[1:2 * r:2], e0, eh)

    def diagnostics(self):
        E = torch.empty(self.cfg.p, dtype=torch.float64, device="cuda")
        H = torch.empty_like(E)
        _check(lib().rom_diagnostics(self.h, _ptr(E), _ptr(H)))
        return E, H

    def gradient(self, Z):
        Z = Z.contiguous()
        g = torch.empty_like(Z)
        grid = (self.cfg.p, self.cfg.Nx)
        rho = torch.empty(grid, dtype=torch.float64, device="cuda")
        Phi = torch.empty_like(rho)
        e = torch.empty_like(rho)
        _check(lib().rom_gradient(self.h, _ptr(Z), _ptr(g), _ptr(rho), _ptr(Phi), _ptr(e)))
        return g, rho, Phi, e


class Fom:
    """Full-order PIC handle (fom_* entry points)."""

    def __init__(self, N, p, Nx, dt, L, X0, V0, q=-1.0, m=1.0, stream=None, family=None,
                 params=None, ux=None, uv=None):
        self.N, self.p, self.Nx = N, p, Nx
        nbytes = lib().fom_workspace_bytes(N, p, Nx)
        if nbytes == 0:
            raise SymromError(EINVAL, "invalid sizes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        if X0 is None:
            eta = eta_array(params)
            uxd, uvd = _dev1(ux), _dev1(uv)
            _check(lib().fom_init_family(N, p, Nx, dt, q, m, FAMILY[family],
                                         eta.ctypes.data_as(ctypes.c_void_p), _ptr(uxd),
                                         _ptr(uvd), _ptr(self.ws), nbytes, _stream(stream),
                                         ctypes.byref(h)))
        else:
            X0, V0 = _dev(X0), _dev(V0)
            Lh, Lp = _host_doubles(L)
            _check(lib().fom_init(N, p, Nx, dt, q, m, Lp, _ptr(X0), _ptr(V0), _ptr(self.ws),
                                  nbytes, _stream(stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().fom_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        _check(lib().fom_step(self.h, nsteps))

    def get_state(self):
        X = torch.empty((self.p, self.N), dtype=torch.float64, device="cuda")
        V = torch.empty_like(X)
        _check(lib().fom_get_state(self.h, _ptr(X), _ptr(V)))
        return X, V

    def diagnostics(self):
        E = torch.empty(self.p, dtype=torch.float64, device="cuda")
        H = torch.empty_like(E)
        _check(lib().fom_diagnostics(self.h, _ptr(E), _ptr(H)))
        return E, H


def pic_fields(X, L, Nx, q=-1.0, stream=None):
    """cells (p, N) int32 and rho, Phi, e (p, Nx) for positions X (p, N)."""
    X = _dev(X)
    p, N = X.shape
    nbytes = lib().pic_workspace_bytes(N, p, Nx)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    cells = torch.empty((p, N), dtype=torch.int32, device="cuda")
    rho = torch.empty((p, Nx), dtype=torch.float64, device="cuda")
    Phi = torch.empty_like(rho)
    e = torch.empty_like(rho)
    Lh, Lp = _host_doubles(L)
    _check(lib().pic_fields(N, p, Nx, Lp, q, _ptr(X), _ptr(cells), _ptr(rho), _ptr(Phi), _ptr(e),
                            _ptr(ws), nbytes, _stream(stream)))
    return cells, rho, Phi, e


def deim_select(Psi, stream=None):
    """Greedy DEIM indices and weights of a basis Psi (numpy N x d, or a
    device tensor (d, N)): (idx int32 (d,), w (d,)) device tensors."""
    P = _dev(Psi)
    d, N = P.shape
    nbytes = lib().deim_select_workspace_bytes(N, d)
    if nbytes == 0:
        raise SymromError(EINVAL, "invalid sizes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    idx = torch.empty(d, dtype=torch.int32, device="cuda")
    w = torch.empty(d, dtype=torch.float64, device="cuda")
    _check(lib().deim_select(N, d, _ptr(P), _ptr(idx), _ptr(w), _ptr(ws), nbytes,
                             _stream(stream)))
    return idx, w


def pic_fields_noalloc(X, L, Nx, q=-1.0, stream=None):
    """pic_fields through the allocation-free entry point (L on the device):
    cells (p, N) int32 and rho, Phi, e (p, Nx)."""
    X = _dev(X)
    p, N = X.shape
    Ld = torch.as_tensor(np.asarray(L, dtype=np.float64)).cuda()
    cells = torch.empty((p, N), dtype=torch.int32, device="cuda")
    rho = torch.empty((p, Nx), dtype=torch.float64, device="cuda")
    Phi = torch.empty_like(rho)
    e = torch.empty_like(rho)
    _check(lib().pic_fields_noalloc(N, p, Nx, _ptr(Ld), q, _ptr(X), _ptr(cells), _ptr(rho),
                                    _ptr(Phi), _ptr(e), _stream(stream)))
    return cells, rho, Phi, e


class Server:
    """The serving loop (srv_* entry points) over a device pool of pool_bytes."""

    def __init__(self, slots, pool_bytes):
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(lib().srv_create(slots, _ptr(self.pool), int(pool_bytes), ctypes.byref(h)))
        self.h = h
        self.meta = {}

    def submit(self, cfg, family, params, ux, uv, nsteps, rows=()):
        eta = eta_array(params)
        ux = np.ascontiguousarray(ux, dtype=np.float64)
        uv = np.ascontiguousarray(uv, dtype=np.float64)
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32))
        if ux.size != cfg.N or uv.size != cfg.N or eta.shape[0] != cfg.p:
            raise ValueError("uniforms must hold N values and eta p rows")
        rid = ctypes.c_int64()
        _check(lib().srv_submit(self.h, ctypes.byref(cfg), FAMILY[family],
                                eta.ctypes.data_as(_VP), ux.ctypes.data_as(_VP),
                                uv.ctypes.data_as(_VP), nsteps, rows.size,
                                rows.ctypes.data_as(_VP) if rows.size else None,
                                ctypes.byref(rid)))
        self.meta[rid.value] = (cfg.p, rows.size)
        return rid.value

    def info(self, rid):
        inf = RequestInfo()
        _check(lib().srv_info(self.h, rid, ctypes.byref(inf)))
        return dict(status=inf.status, two_n=inf.two_n, steps_done=inf.steps_done,
                    t_arrival=inf.t_arrival, t_start=inf.t_start, t_finish=inf.t_finish,
                    pp_steps=inf.pp_steps)

    def wait(self, rid):
        _check(lib().srv_wait(self.h, rid))

    def drain(self):
        peak = ctypes.c_double()
        _check(lib().srv_drain(self.h, ctypes.byref(peak)))
        return peak.value

    def result(self, rid):
        p, nr = self.meta[rid]
        E = np.empty(p)
        H = np.empty(p)
        X = np.empty((p, nr))
        V = np.empty((p, nr))
        _check(lib().srv_result(self.h, rid, E.ctypes.data_as(_VP), H.ctypes.data_as(_VP),
                                X.ctypes.data_as(_VP), V.ctypes.data_as(_VP)))
        return E, H, X, V

    def close(self):
        if self.h:
            lib().srv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
