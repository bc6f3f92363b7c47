"""Python binding of libthcsox (ctypes).  Argument marshalling only: every
step of the SOX path runs in the library's HIP kernels.  PyTorch is used for
device memory and streams only.

The module-level functions mirror the C interface one to one (same names,
same argument order, device pointers as integers).  ``Plan`` is a small
convenience wrapper over torch tensors.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libthcsox.so")


THCSOX_FP64, THCSOX_FP32, THCSOX_BF16X3, THCSOX_FP16X2 = 0, 1, 2, 3
PRECISIONS = {"fp64": THCSOX_FP64, "fp32": THCSOX_FP32, "bf16x3": THCSOX_BF16X3,
              "fp16x2": THCSOX_FP16X2}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE", -5: "ENOTDEV"}

# every symbol declared in include/thcsox.h
EXPORTS = ("thcsox_plan", "thcsox_sigma_sox", "thcsox_energy", "thcsox_destroy",
           "thcsox_last_error", "thcsox_plan_info", "thcsox_profile", "thcsox_stage_times",
           "thcsox_backproject", "thcsox_dyson_plan", "thcsox_dyson_step",
           "thcsox_dyson_onebody", "thcsox_dyson_destroy", "thcsox_mlp_create",
           "thcsox_mlp_forward", "thcsox_mlp_forward_bf16", "thcsox_mlp_gradients",
           "thcsox_mlp_train_step",
           "thcsox_mlp_params", "thcsox_mlp_destroy", "thcsox_pair_scale",
           "thcsox_pair_gather", "thcsox_pair_scatter", "thcsox_set_symmetry",
           "thcsox_symmetric_flags", "thcsox_dyson_step_mu", "thcsox_mix",
           "thcsox_diis_create", "thcsox_diis_step", "thcsox_diis_destroy",
           "thcsox_sigma_direct", "thcsox_energy_basis", "thcsox_dyson_plan_sampled",
           "thcsox_ir_create", "thcsox_ir_sizes", "thcsox_ir_get", "thcsox_ir_destroy",
           "thcsox_energy_noalloc", "thcsox_static_screening", "thcsox_sigma_screened",
           "thcsox_dyson_commutator", "thcsox_diis_create_res", "thcsox_diis_step_res")
SYMMETRY = {"auto": 0, "off": 1}
STAGES = ("project", "a_stage", "fused", "back")


class ThcsoxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("naux", ctypes.c_int), ("ntau", ctypes.c_int),
                ("precision", ctypes.c_int), ("tau_batch", ctypes.c_int),
                ("bytes", ctypes.c_size_t), ("mac_per_tau", ctypes.c_double),
                ("fused_mac_per_tau", ctypes.c_double),
                ("fused_bytes_per_tau", ctypes.c_double),
                ("vsplit", ctypes.c_int), ("vrange", ctypes.c_int),
                ("partial_f32", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load the compiled library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libthcsox is not built ({LIB_PATH} missing); run "
                               "__graft_entry__.build() or paper_2404_17744_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.thcsox_plan.argtypes = [ctypes.POINTER(vp), i, i, i, d, vp, vp, vp, vp, i, sz, vp]
        L.thcsox_plan.restype = i
        L.thcsox_sigma_sox.argtypes = [vp, vp, vp, vp, i, i]
        L.thcsox_sigma_sox.restype = i
        L.thcsox_energy.argtypes = [vp, vp, vp, ctypes.POINTER(d)]
        L.thcsox_energy.restype = i
        L.thcsox_energy_noalloc.argtypes = [vp, vp, vp, i, i, vp, vp]
        L.thcsox_energy_noalloc.restype = i
        L.thcsox_static_screening.argtypes = [vp, vp, vp]
        L.thcsox_static_screening.restype = i
        L.thcsox_sigma_screened.argtypes = [vp, vp, vp, i, vp, i, i]
        L.thcsox_sigma_screened.restype = i
        L.thcsox_destroy.argtypes = [vp]
        L.thcsox_destroy.restype = i
        L.thcsox_last_error.argtypes = []
        L.thcsox_last_error.restype = ctypes.c_char_p
        L.thcsox_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.thcsox_plan_info.restype = i
        L.thcsox_profile.argtypes = [vp, i]
        L.thcsox_profile.restype = i
        L.thcsox_stage_times.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i)]
        L.thcsox_stage_times.restype = i
        L.thcsox_backproject.argtypes = [vp, vp, vp, i, i]
        L.thcsox_backproject.restype = i
        L.thcsox_set_symmetry.argtypes = [vp, i]
        L.thcsox_set_symmetry.restype = i
        L.thcsox_symmetric_flags.argtypes = [vp, vp]
        L.thcsox_symmetric_flags.restype = i
        L.thcsox_dyson_plan.argtypes = [ctypes.POINTER(vp), i, i, i, d, d, vp, vp, vp]
        L.thcsox_dyson_plan.restype = i
        L.thcsox_dyson_step.argtypes = [vp, vp, vp, vp]
        L.thcsox_dyson_step.restype = i
        L.thcsox_dyson_onebody.argtypes = [vp, vp, ctypes.POINTER(d)]
        L.thcsox_dyson_onebody.restype = i
        L.thcsox_dyson_destroy.argtypes = [vp]
        L.thcsox_dyson_destroy.restype = i
        L.thcsox_dyson_step_mu.argtypes = [vp, vp, d, d, ctypes.POINTER(d), vp, vp,
                                           ctypes.POINTER(i)]
        L.thcsox_dyson_step_mu.restype = i
        L.thcsox_sigma_direct.argtypes = [vp, vp, vp, i, i, i]
        L.thcsox_sigma_direct.restype = i
        L.thcsox_energy_basis.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(d)]
        L.thcsox_energy_basis.restype = i
        L.thcsox_dyson_plan_sampled.argtypes = [ctypes.POINTER(vp), i, i, i, d, d, vp, vp, vp,
                                                vp, vp]
        L.thcsox_dyson_plan_sampled.restype = i
        L.thcsox_ir_create.argtypes = [ctypes.POINTER(vp), d, d, d]
        L.thcsox_ir_create.restype = i
        L.thcsox_ir_sizes.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.thcsox_ir_sizes.restype = i
        L.thcsox_ir_get.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.thcsox_ir_get.restype = i
        L.thcsox_ir_destroy.argtypes = [vp]
        L.thcsox_ir_destroy.restype = i
        L.thcsox_mix.argtypes = [ctypes.c_int64, d, vp, vp, vp]
        L.thcsox_mix.restype = i
        L.thcsox_diis_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int64, i, vp]
        L.thcsox_diis_create.restype = i
        L.thcsox_diis_step.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i)]
        L.thcsox_diis_step.restype = i
        L.thcsox_diis_destroy.argtypes = [vp]
        L.thcsox_diis_destroy.restype = i
        L.thcsox_diis_create_res.argtypes = [ctypes.POINTER(vp), ctypes.c_int64, ctypes.c_int64,
                                             i, vp]
        L.thcsox_diis_create_res.restype = i
        L.thcsox_diis_step_res.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i)]
        L.thcsox_diis_step_res.restype = i
        L.thcsox_dyson_commutator.argtypes = [vp, vp, vp, vp]
        L.thcsox_dyson_commutator.restype = i
        fp = ctypes.c_float
        L.thcsox_mlp_create.argtypes = [ctypes.POINTER(vp), i, i, i, vp, vp]
        L.thcsox_mlp_create.restype = i
        L.thcsox_mlp_forward.argtypes = [vp, vp, vp, i]
        L.thcsox_mlp_forward.restype = i
        L.thcsox_mlp_forward_bf16.argtypes = [vp, vp, vp, ctypes.c_int64]
        L.thcsox_mlp_forward_bf16.restype = i
        L.thcsox_mlp_gradients.argtypes = [vp, vp, vp, i, vp, ctypes.POINTER(d)]
        L.thcsox_mlp_gradients.restype = i
        L.thcsox_mlp_train_step.argtypes = [vp, vp, vp, i, fp, ctypes.POINTER(d)]
        L.thcsox_mlp_train_step.restype = i
        L.thcsox_mlp_params.argtypes = [vp, vp]
        L.thcsox_mlp_params.restype = i
        L.thcsox_mlp_destroy.argtypes = [vp]
        L.thcsox_mlp_destroy.restype = i
        ll = ctypes.c_longlong
        L.thcsox_pair_scale.argtypes = [i, i, vp, vp, vp]
        L.thcsox_pair_scale.restype = i
        L.thcsox_pair_gather.argtypes = [i, i, vp, vp, vp, ll, vp, vp]
        L.thcsox_pair_gather.restype = i
        L.thcsox_pair_scatter.argtypes = [i, i, vp, vp, vp, vp]
        L.thcsox_pair_scatter.restype = i
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise ThcsoxError(rc, thcsox_last_error())


def thcsox_last_error() -> str:
    return lib().thcsox_last_error().decode()


def thcsox_plan(n: int, naux: int, ntau: int, beta: float, tau_host: np.ndarray,
                wq_host: np.ndarray, X_dev: int, V_dev: int, precision: int,
                workspace_limit: int = 0, hip_stream: int = 0) -> ctypes.c_void_p:
    tau = np.ascontiguousarray(tau_host, dtype=np.float64)
    wq = np.ascontiguousarray(wq_host, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib().thcsox_plan(ctypes.byref(h), n, naux, ntau, beta,
                             tau.ctypes.data_as(ctypes.c_void_p),
                             wq.ctypes.data_as(ctypes.c_void_p), X_dev, V_dev,
                             precision, workspace_limit, hip_stream))
    return h


def thcsox_sigma_sox(plan, G_dev: int, Sigma_dev: int, Sigma_thc_dev: int | None,
                     k_begin: int, k_end: int) -> None:
    _check(lib().thcsox_sigma_sox(plan, G_dev, Sigma_dev, Sigma_thc_dev, k_begin, k_end))


def thcsox_energy(plan, G_dev: int, Sigma_dev: int) -> float:
    e = ctypes.c_double()
    _check(lib().thcsox_energy(plan, G_dev, Sigma_dev, ctypes.byref(e)))
    return e.value


def thcsox_energy_noalloc(G_dev: int, Sigma_dev: int, w_dev: int, n: int, ntau: int,
                          E_dev: int, hip_stream: int = 0) -> None:
    _check(lib().thcsox_energy_noalloc(G_dev, Sigma_dev, w_dev, n, ntau, E_dev, hip_stream))


SCREENED = {"sosex": 0, "g3w2": 1}


def thcsox_static_screening(plan, G_dev: int, W_dev: int) -> None:
    _check(lib().thcsox_static_screening(plan, G_dev, W_dev))


def thcsox_sigma_screened(plan, G_dev: int, W_dev: int, kind: int, Sigma_dev: int,
                          k_begin: int, k_end: int) -> None:
    _check(lib().thcsox_sigma_screened(plan, G_dev, W_dev, kind, Sigma_dev, k_begin, k_end))


def thcsox_destroy(plan) -> None:
    _check(lib().thcsox_destroy(plan))


def thcsox_plan_info(plan) -> dict:
    info = PlanInfo()
    _check(lib().thcsox_plan_info(plan, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in PlanInfo._fields_}


def thcsox_profile(plan, enable: bool) -> None:
    _check(lib().thcsox_profile(plan, 1 if enable else 0))


def thcsox_stage_times(plan) -> dict:
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_int * len(STAGES))()
    _check(lib().thcsox_stage_times(plan, ms, cnt))
    return {st: (ms[i], cnt[i]) for i, st in enumerate(STAGES)}


def thcsox_backproject(plan, Sigma_thc_dev: int, Sigma_dev: int, k_begin: int, k_end: int):
    _check(lib().thcsox_backproject(plan, Sigma_thc_dev, Sigma_dev, k_begin, k_end))


def thcsox_set_symmetry(plan, mode: int) -> None:
    _check(lib().thcsox_set_symmetry(plan, mode))


def thcsox_symmetric_flags(plan, ntau: int) -> np.ndarray:
    flags = np.zeros(ntau, dtype=np.int32)
    _check(lib().thcsox_symmetric_flags(plan, flags.ctypes.data_as(ctypes.c_void_p)))
    return flags


def thcsox_dyson_plan(n: int, ntau: int, n_matsubara: int, beta: float, mu: float,
                      tau_host: np.ndarray, F_dev: int, hip_stream: int = 0):
    tau = np.ascontiguousarray(tau_host, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib().thcsox_dyson_plan(ctypes.byref(h), n, ntau, n_matsubara, beta, mu,
                                   tau.ctypes.data_as(ctypes.c_void_p), F_dev, hip_stream))
    return h


def thcsox_dyson_plan_sampled(n: int, ntau: int, nfreq: int, beta: float, mu: float,
                              freq_n: np.ndarray, Wf: np.ndarray, Wb: np.ndarray, F_dev: int,
                              hip_stream: int = 0):
    fn = np.ascontiguousarray(freq_n, dtype=np.int32)
    wf = np.ascontiguousarray(Wf, dtype=np.float64)
    wb = np.ascontiguousarray(Wb, dtype=np.float64)
    if fn.shape != (nfreq,) or wf.shape != (2 * nfreq, ntau) or wb.shape != (ntau + 1, 2 * nfreq):
        raise ValueError("freq_n [nfreq], Wf [2 nfreq, ntau], Wb [ntau + 1, 2 nfreq] expected")
    h = ctypes.c_void_p()
    vpp = ctypes.c_void_p
    _check(lib().thcsox_dyson_plan_sampled(ctypes.byref(h), n, ntau, nfreq, beta, mu,
                                           fn.ctypes.data_as(vpp), wf.ctypes.data_as(vpp),
                                           wb.ctypes.data_as(vpp), F_dev, hip_stream))
    return h


def thcsox_energy_basis(plan, G_dev: int, Sigma_dev: int, coef: np.ndarray,
                        sign: np.ndarray) -> float:
    c = np.ascontiguousarray(coef, dtype=np.float64)
    sg = np.ascontiguousarray(sign, dtype=np.float64)
    E = ctypes.c_double()
    _check(lib().thcsox_energy_basis(plan, G_dev, Sigma_dev, c.ctypes.data_as(ctypes.c_void_p),
                                     sg.ctypes.data_as(ctypes.c_void_p), ctypes.byref(E)))
    return E.value


def thcsox_ir_grid(beta: float, wmax: float, eps: float = 1e-10) -> dict:
    """The IR basis sampling grids and tables (host only)."""
    h = ctypes.c_void_p()
    _check(lib().thcsox_ir_create(ctypes.byref(h), float(beta), float(wmax), float(eps)))
    try:
        m, nf = ctypes.c_int(), ctypes.c_int()
        _check(lib().thcsox_ir_sizes(h, ctypes.byref(m), ctypes.byref(nf)))
        m, nf = m.value, nf.value
        out = {"tau": np.empty(m), "freq_n": np.empty(nf, dtype=np.int32),
               "Wf": np.empty((2 * nf, m)), "Wb": np.empty((m + 1, 2 * nf)),
               "coef": np.empty((m, m)), "sign": np.empty(m), "sv": np.empty(m)}
        ptr = {k: v.ctypes.data_as(ctypes.c_void_p) for k, v in out.items()}
        _check(lib().thcsox_ir_get(h, ptr["tau"], ptr["freq_n"], ptr["Wf"], ptr["Wb"],
                                   ptr["coef"], ptr["sign"], ptr["sv"]))
    finally:
        lib().thcsox_ir_destroy(h)
    out.update(beta=float(beta), wmax=float(wmax), eps=float(eps))
    return out


def thcsox_dyson_step(d, Sigma_dev: int, G_dev: int, gamma_dev: int | None) -> None:
    _check(lib().thcsox_dyson_step(d, Sigma_dev, G_dev, gamma_dev))


def thcsox_dyson_onebody(d, gamma_dev: int) -> float:
    e = ctypes.c_double()
    _check(lib().thcsox_dyson_onebody(d, gamma_dev, ctypes.byref(e)))
    return e.value


def thcsox_dyson_destroy(d) -> None:
    _check(lib().thcsox_dyson_destroy(d))


def thcsox_dyson_step_mu(d, Sigma_dev: int, nelec: float, tol: float, mu: float, G_dev: int,
                         gamma_dev: int | None):
    """Returns (mu, number of Dyson solves)."""
    m = ctypes.c_double(mu)
    ev = ctypes.c_int(0)
    _check(lib().thcsox_dyson_step_mu(d, Sigma_dev, nelec, tol, ctypes.byref(m), G_dev,
                                      gamma_dev, ctypes.byref(ev)))
    return m.value, ev.value


def thcsox_mix(length: int, alpha: float, sigma_out: int, sigma_io: int, stream: int) -> None:
    _check(lib().thcsox_mix(length, alpha, sigma_out, sigma_io, stream))


def thcsox_diis_create(length: int, depth: int, stream: int):
    h = ctypes.c_void_p()
    _check(lib().thcsox_diis_create(ctypes.byref(h), length, depth, stream))
    return h


def thcsox_diis_step(h, sigma_in: int, sigma_out: int, sigma_next: int) -> int:
    used = ctypes.c_int(0)
    _check(lib().thcsox_diis_step(h, sigma_in, sigma_out, sigma_next, ctypes.byref(used)))
    return used.value


def thcsox_diis_destroy(h) -> None:
    _check(lib().thcsox_diis_destroy(h))


def thcsox_diis_create_res(length: int, length_res: int, depth: int, stream: int):
    h = ctypes.c_void_p()
    _check(lib().thcsox_diis_create_res(ctypes.byref(h), length, length_res, depth, stream))
    return h


def thcsox_diis_step_res(h, residual: int, sigma_out: int, sigma_next: int) -> int:
    used = ctypes.c_int(0)
    _check(lib().thcsox_diis_step_res(h, residual, sigma_out, sigma_next, ctypes.byref(used)))
    return used.value


def thcsox_dyson_commutator(d, Sigma_in_dev: int, Sigma_out_dev: int, e_dev: int) -> None:
    _check(lib().thcsox_dyson_commutator(d, Sigma_in_dev, Sigma_out_dev, e_dev))


class Dyson:
    """Owns one Dyson/transform plan; tensors are torch float64 device tensors."""

    def __init__(self, F, mu: float, tau, beta: float, n_matsubara: int = 256, stream=None,
                 grid: dict | None = None):
        """Chebyshev-root tau grid with n_matsubara frequencies, or (grid given)
        the sampling grids of thcsox_ir_grid, whose tau points `tau` must be."""
        import torch
        self.n = F.shape[0]
        self.ntau = len(tau)
        self.device = F.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(F.device)
        Fc = F.contiguous().to(torch.float64)
        self.nfreq = n_matsubara if grid is None else len(grid["freq_n"])
        if grid is None:
            self.handle = _ordered(self.stream, thcsox_dyson_plan, self.n, self.ntau, n_matsubara,
                                   float(beta), float(mu), np.asarray(tau), Fc.data_ptr(),
                                   self.stream.cuda_stream)
        else:
            if not np.array_equal(np.asarray(tau, dtype=np.float64), grid["tau"]):
                raise ValueError("tau must be the grid's sampling points")
            self.handle = _ordered(self.stream, thcsox_dyson_plan_sampled, self.n, self.ntau,
                                   len(grid["freq_n"]), float(beta), float(mu), grid["freq_n"],
                                   grid["Wf"], grid["Wb"], Fc.data_ptr(), self.stream.cuda_stream)

    def step(self, Sigma, G_out=None, gamma_out=None):
        import torch
        if G_out is None:
            G_out = torch.empty((self.ntau, self.n, self.n), dtype=torch.float64, device=self.device)
        if gamma_out is None:
            gamma_out = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        _dev64(Sigma, "Sigma", (self.n, self.n), self.ntau, exact=True)
        _dev64(G_out, "G_out", (self.n, self.n), self.ntau, exact=True)
        _dev64(gamma_out, "gamma_out", (self.n,), self.n, exact=True)
        _ordered(self.stream, thcsox_dyson_step, self.handle, Sigma.data_ptr(), G_out.data_ptr(),
                 gamma_out.data_ptr())
        return G_out, gamma_out

    def commutator(self, Sigma_in, Sigma_out, out=None):
        """[G(i w), Sigma_out(i w) - Sigma_in(i w)] on the plan's frequencies for the
        G of the last step (taken with Sigma_in): [2, nfreq, n, n] (Re, Im)."""
        import torch
        _dev64(Sigma_in, "Sigma_in", (self.n, self.n), self.ntau, exact=True)
        _dev64(Sigma_out, "Sigma_out", (self.n, self.n), self.ntau, exact=True)
        if out is None:
            out = torch.empty((2, self.nfreq, self.n, self.n), dtype=torch.float64,
                              device=self.device)
        _dev64(out, "out", (self.nfreq, self.n, self.n), 2, exact=True)
        _ordered(self.stream, thcsox_dyson_commutator, self.handle, Sigma_in.data_ptr(),
                 Sigma_out.data_ptr(), out.data_ptr())
        return out

    def step_mu(self, Sigma, nelec: float, mu: float, tol: float = 1e-8, G_out=None,
                gamma_out=None):
        """Dyson step with the chemical potential that conserves nelec electrons:
        returns (G, gamma, mu, number of Dyson solves)."""
        import torch
        if G_out is None:
            G_out = torch.empty((self.ntau, self.n, self.n), dtype=torch.float64, device=self.device)
        if gamma_out is None:
            gamma_out = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        _dev64(Sigma, "Sigma", (self.n, self.n), self.ntau, exact=True)
        _dev64(G_out, "G_out", (self.n, self.n), self.ntau, exact=True)
        _dev64(gamma_out, "gamma_out", (self.n,), self.n, exact=True)
        mu, ev = _ordered(self.stream, thcsox_dyson_step_mu, self.handle, Sigma.data_ptr(),
                          float(nelec), float(tol), float(mu), G_out.data_ptr(),
                          gamma_out.data_ptr())
        return G_out, gamma_out, mu, ev

    def onebody(self, gamma) -> float:
        return _ordered(self.stream, thcsox_dyson_onebody, self.handle, gamma.data_ptr())

    def close(self) -> None:
        if getattr(self, "handle", None):
            thcsox_dyson_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def thcsox_pair_scale(m, naux, S_dev, scale_dev, hip_stream=0):
    _check(lib().thcsox_pair_scale(m, naux, S_dev, scale_dev, hip_stream))


def thcsox_pair_gather(m, naux, S_dev, scale_dev, pairs_dev, npairs, x_dev, hip_stream=0):
    _check(lib().thcsox_pair_gather(m, naux, S_dev, scale_dev, pairs_dev, npairs, x_dev,
                                    hip_stream))


def thcsox_pair_scatter(m, naux, y_dev, scale_dev, S_dev, hip_stream=0):
    _check(lib().thcsox_pair_scatter(m, naux, y_dev, scale_dev, S_dev, hip_stream))


class MLP:
    """Residual warm-start MLP on the GPU (thcsox_mlp_*); params packed FP32."""

    ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, m: int, hidden: int, params: dict, max_batch: int = 65536, stream=None):
        import torch
        self.m, self.H, self.max_batch = m, hidden, max_batch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        flat = np.concatenate([np.asarray(params[k], dtype=np.float32).ravel()
                               for k in self.ORDER])
        h = ctypes.c_void_p()
        _check(lib().thcsox_mlp_create(ctypes.byref(h), m, hidden, max_batch,
                                       flat.ctypes.data_as(ctypes.c_void_p),
                                       self.stream.cuda_stream))
        self.handle = h
        self.nparam = flat.size

    def _unpack(self, flat: np.ndarray) -> dict:
        m, H = self.m, self.H
        shapes = {"W1": (H, m), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (m, H), "b3": (m,)}
        out, o = {}, 0
        for k in self.ORDER:
            size = int(np.prod(shapes[k]))
            out[k] = flat[o:o + size].reshape(shapes[k])
            o += size
        return out

    def forward(self, x, out=None):
        import torch
        _dev64(x, "x", (self.m,), x.shape[0], exact=True, f32=True)
        if out is None:
            out = torch.empty_like(x)
        _dev64(out, "out", (self.m,), x.shape[0], exact=True, f32=True)
        _check(_ordered(self.stream, lib().thcsox_mlp_forward, self.handle, x.data_ptr(),
                        out.data_ptr(), x.shape[0]))
        return out

    def forward_bf16(self, x, out=None):
        """Inference with the weights and layer inputs rounded to bf16 (FP32
        accumulation), one fused kernel per 64 rows; any batch size."""
        import torch
        _dev64(x, "x", (self.m,), x.shape[0], exact=True, f32=True)
        if out is None:
            out = torch.empty_like(x)
        _dev64(out, "out", (self.m,), x.shape[0], exact=True, f32=True)
        if out.data_ptr() == x.data_ptr() and x.numel() > 0:
            raise ValueError("out may not alias x")
        _check(_ordered(self.stream, lib().thcsox_mlp_forward_bf16, self.handle, x.data_ptr(),
                        out.data_ptr(), x.shape[0]))
        return out

    def gradients(self, x, t):
        _dev64(x, "x", (self.m,), x.shape[0], exact=True, f32=True)
        _dev64(t, "t", (self.m,), x.shape[0], exact=True, f32=True)
        g = np.empty(self.nparam, dtype=np.float32)
        loss = ctypes.c_double()
        _check(_ordered(self.stream, lib().thcsox_mlp_gradients, self.handle, x.data_ptr(),
                        t.data_ptr(), x.shape[0], g.ctypes.data_as(ctypes.c_void_p),
                        ctypes.byref(loss)))
        return loss.value, self._unpack(g)

    def train_step(self, x, t, lr: float, want_loss: bool = True):
        _dev64(x, "x", (self.m,), x.shape[0], exact=True, f32=True)
        _dev64(t, "t", (self.m,), x.shape[0], exact=True, f32=True)
        loss = ctypes.c_double()
        _check(_ordered(self.stream, lib().thcsox_mlp_train_step, self.handle, x.data_ptr(),
                        t.data_ptr(), x.shape[0], lr, ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def params(self) -> dict:
        p = np.empty(self.nparam, dtype=np.float32)
        _check(lib().thcsox_mlp_params(self.handle, p.ctypes.data_as(ctypes.c_void_p)))
        return self._unpack(p)

    def close(self) -> None:
        if getattr(self, "handle", None):
            _check(lib().thcsox_mlp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ordered(stream, fn, *args):
    """Run a library call that queues work on `stream` after the work already on
    torch's current stream (the call's inputs, outputs just allocated and zeroed
    there), and make the current stream's later work wait for it."""
    import torch
    cur = torch.cuda.current_stream(stream.device)
    if cur == stream:
        return fn(*args)
    stream.wait_stream(cur)
    try:
        return fn(*args)
    finally:
        cur.wait_stream(stream)


def _dev64(t, name: str, tail: tuple, lead: int, exact: bool = False, f32: bool = False):
    """Check that t is a contiguous float64 (float32 with f32) device tensor of
    shape [lead, *tail] (or [>= lead, *tail] unless exact): the library indexes
    its arrays by raw pointer, so a short buffer would be written past its end."""
    import torch
    dt = torch.float32 if f32 else torch.float64
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt \
            or not t.is_contiguous():
        raise ValueError(f"{name}: a contiguous {'float32' if f32 else 'float64'} device tensor "
                         "is required")
    shape = tuple(t.shape)
    if shape[1:] != tuple(tail) or (shape[0] != lead if exact else shape[0] < lead):
        want = f"[{lead}{'' if exact else '+'}, {', '.join(str(x) for x in tail)}]"
        raise ValueError(f"{name}: shape {shape}, expected {want}")
    return t


class Plan:
    """Owns one libthcsox plan; tensors are torch CUDA (HIP) float64 tensors."""

    def __init__(self, X, V, tau, w, beta: float, precision="fp64", stream=None,
                 workspace_limit: int = 0):
        import torch
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.n, self.naux = X.shape
        self.ntau = len(tau)
        self.device = X.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(X.device)
        Xc = X.contiguous().to(torch.float64)
        Vc = V.contiguous().to(torch.float64)
        self.handle = _ordered(self.stream, thcsox_plan, self.n, self.naux, self.ntau,
                               float(beta), np.asarray(tau), np.asarray(w), Xc.data_ptr(),
                               Vc.data_ptr(), precision, workspace_limit, self.stream.cuda_stream)
        self.precision = precision

    def sigma(self, G, k_begin: int = 0, k_end: int | None = None, thc: bool = False,
              out=None, out_thc=None):
        import torch
        k_end = self.ntau if k_end is None else k_end
        nn, aa = (self.n, self.n), (self.naux, self.naux)
        _dev64(G, "G", nn, self.ntau, exact=True)
        if out is None:
            out = torch.zeros((self.ntau, self.n, self.n), dtype=torch.float64, device=self.device)
        _dev64(out, "out", nn, k_end)
        if thc and out_thc is None:
            out_thc = torch.zeros((self.ntau, self.naux, self.naux), dtype=torch.float64,
                                  device=self.device)
        if thc:
            _dev64(out_thc, "out_thc", aa, k_end)
        _ordered(self.stream, thcsox_sigma_sox, self.handle, G.data_ptr(), out.data_ptr(),
                 out_thc.data_ptr() if thc else None, k_begin, k_end)
        return (out, out_thc) if thc else out

    def sigma_direct(self, G, k_begin: int = 0, k_end: int | None = None, out=None,
                     accumulate: bool = False):
        """Second-order direct (bubble) self-energy, FP64, for k in [k_begin, k_end);
        accumulate=True adds it to `out` (e.g. onto the SOX term)."""
        import torch
        k_end = self.ntau if k_end is None else k_end
        _dev64(G, "G", (self.n, self.n), self.ntau, exact=True)
        if out is None:
            out = torch.zeros((self.ntau, self.n, self.n), dtype=torch.float64, device=self.device)
        _dev64(out, "out", (self.n, self.n), k_end)
        _check(_ordered(self.stream, lib().thcsox_sigma_direct, self.handle, G.data_ptr(),
                        out.data_ptr(), k_begin, k_end, 1 if accumulate else 0))
        return out

    def static_screening(self, G, out=None):
        """Statically screened core W = (1 + V Pi0)^-1 V [naux][naux] (FP64)."""
        import torch
        _dev64(G, "G", (self.n, self.n), self.ntau, exact=True)
        if out is None:
            out = torch.empty((self.naux, self.naux), dtype=torch.float64, device=self.device)
        _dev64(out, "out", (self.naux,), self.naux, exact=True)
        _check(_ordered(self.stream, lib().thcsox_static_screening, self.handle, G.data_ptr(),
                        out.data_ptr()))
        return out

    def sigma_screened(self, G, W, kind: str = "sosex", k_begin: int = 0,
                       k_end: int | None = None, out=None):
        """Screened exchange self-energy ("sosex": one line screened, "g3w2": both)."""
        import torch
        k_end = self.ntau if k_end is None else k_end
        _dev64(G, "G", (self.n, self.n), self.ntau, exact=True)
        _dev64(W, "W", (self.naux,), self.naux, exact=True)
        if out is None:
            out = torch.zeros((self.ntau, self.n, self.n), dtype=torch.float64, device=self.device)
        _dev64(out, "out", (self.n, self.n), k_end)
        _check(_ordered(self.stream, lib().thcsox_sigma_screened, self.handle, G.data_ptr(),
                        W.data_ptr(), SCREENED[kind], out.data_ptr(), k_begin, k_end))
        return out

    def energy(self, G, Sigma) -> float:
        _dev64(G, "G", (self.n, self.n), self.ntau, exact=True)
        _dev64(Sigma, "Sigma", (self.n, self.n), self.ntau, exact=True)
        return _ordered(self.stream, thcsox_energy, self.handle, G.data_ptr(), Sigma.data_ptr())

    def energy_basis(self, G, Sigma, grid: dict) -> float:
        """The energy on an IR grid (thcsox_ir_grid): the basis-coefficient form."""
        _dev64(G, "G", (self.n, self.n), self.ntau, exact=True)
        _dev64(Sigma, "Sigma", (self.n, self.n), self.ntau, exact=True)
        if np.shape(grid["coef"]) != (self.ntau, self.ntau) or len(grid["sign"]) != self.ntau:
            raise ValueError("the grid's basis size differs from the plan's tau count")
        return _ordered(self.stream, thcsox_energy_basis, self.handle, G.data_ptr(),
                        Sigma.data_ptr(), grid["coef"], grid["sign"])

    def backproject(self, Sigma_thc, k_begin: int = 0, k_end: int | None = None, out=None):
        import torch
        k_end = self.ntau if k_end is None else k_end
        _dev64(Sigma_thc, "Sigma_thc", (self.naux, self.naux), k_end)
        if out is None:
            out = torch.zeros((self.ntau, self.n, self.n), dtype=torch.float64, device=self.device)
        _dev64(out, "out", (self.n, self.n), k_end)
        _ordered(self.stream, thcsox_backproject, self.handle, Sigma_thc.data_ptr(), out.data_ptr(),
                 k_begin, k_end)
        return out

    def info(self) -> dict:
        return thcsox_plan_info(self.handle)

    def set_symmetry(self, mode="auto") -> None:
        """'auto': use D's symmetry where G is symmetric; 'off': never."""
        thcsox_set_symmetry(self.handle, SYMMETRY[mode] if isinstance(mode, str) else mode)

    def symmetric_flags(self) -> np.ndarray:
        """Per tau point: 1 where the last sigma call took the symmetric path."""
        return thcsox_symmetric_flags(self.handle, self.ntau)

    def profile(self, enable: bool = True) -> None:
        thcsox_profile(self.handle, enable)

    def stage_times(self) -> dict:
        """{stage: (total ms, launches)} since the last read."""
        return thcsox_stage_times(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            thcsox_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mix(alpha: float, sigma_out, sigma_io, stream=None) -> None:
    """sigma_io = alpha sigma_io + (1 - alpha) sigma_out (float64 device tensors)."""
    import torch
    _dev64(sigma_io, "sigma_io", tuple(sigma_io.shape[1:]), sigma_io.shape[0], exact=True)
    _dev64(sigma_out, "sigma_out", tuple(sigma_io.shape[1:]), sigma_io.shape[0], exact=True)
    st = stream if stream is not None else torch.cuda.current_stream(sigma_io.device)
    _ordered(st, thcsox_mix, sigma_io.numel(), float(alpha), sigma_out.data_ptr(),
             sigma_io.data_ptr(), st.cuda_stream)


class Diis:
    """DIIS over a history held on the device: Pulay's (residual Sigma_out -
    Sigma_in, `step`) or with caller-given residuals such as the commutator of
    Dyson.commutator (`residual_like` given, `step_res`)."""

    def __init__(self, like, depth: int = 6, stream=None, residual_like=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream(like.device)
        self.shape = tuple(like.shape)
        if residual_like is None:
            self.res_shape = None
            self.handle = thcsox_diis_create(like.numel(), depth, self.stream.cuda_stream)
        else:
            self.res_shape = tuple(residual_like.shape)
            self.handle = thcsox_diis_create_res(like.numel(), residual_like.numel(), depth,
                                                 self.stream.cuda_stream)

    def step_res(self, residual, sigma_out, sigma_next) -> int:
        """Adds (residual, sigma_out); writes sum_i c_i Sigma_out_i into sigma_next."""
        _dev64(residual, "residual", self.res_shape[1:], self.res_shape[0], exact=True)
        for name, t in (("sigma_out", sigma_out), ("sigma_next", sigma_next)):
            _dev64(t, name, self.shape[1:], self.shape[0], exact=True)
        return _ordered(self.stream, thcsox_diis_step_res, self.handle, residual.data_ptr(),
                        sigma_out.data_ptr(), sigma_next.data_ptr())

    def step(self, sigma_in, sigma_out, sigma_next) -> int:
        """Writes the extrapolated input into sigma_next; returns the entries used."""
        for name, t in (("sigma_in", sigma_in), ("sigma_out", sigma_out),
                        ("sigma_next", sigma_next)):
            _dev64(t, name, self.shape[1:], self.shape[0], exact=True)
        return _ordered(self.stream, thcsox_diis_step, self.handle, sigma_in.data_ptr(),
                        sigma_out.data_ptr(), sigma_next.data_ptr())

    def close(self) -> None:
        if getattr(self, "handle", None):
            thcsox_diis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
