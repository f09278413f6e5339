"""Thin ctypes binding of libnuhalo.so (include/nuhalo.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory and streams.  The
binding imports torch before loading the library so that the process holds a
single HIP runtime.  If the library has not been built, loading fails loudly;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library shares)

from .request import Request

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnuhalo.so")

NH_OK, NH_EINVAL, NH_ENOMEM, NH_EDEVICE, NH_ESTEPS = 0, -1, -2, -3, -4
NH_ENONFINITE, NH_EBUSY, NH_ENOTREADY, NH_ENOTFOUND, NH_ECANCELED = -5, -6, -7, -8, -9
OPTIONS = {"queue_order": 1, "free_exit": 2, "fp64_below_h": 3, "table_nodes": 4, "block_threads": 5,
           "batch_slots": 6, "slice_us": 7, "serve_graph": 8, "workgroups": 9, "fp32c_rtol": 10,
           "trajectory_stats": 11}

_MASS = {"zero": 0, "paper": 1, "exponential": 2, "table": 3}
_CONC = {"constant": 0, "power": 1, "table": 2}
_KAPPA = {"none": 0, "log": 1, "paper": 2, "constant": 3, "table": 4}
_GEOM = {"paper": 0, "delta200": 1}
_F0 = {"fermi_dirac": 0, "freeze_in": 1, "table": 2}
_METHOD = {"rk4": 0, "dp5": 1}
_PREC = {"fp64": 0, "fp32c": 1}

_dp = ctypes.POINTER(ctypes.c_double)


class NhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nuhalo error {code}: {msg}")
        self.code = code


class nh_cosmology(ctypes.Structure):
    _fields_ = [("H0_km_s_Mpc", ctypes.c_double), ("Omega_m", ctypes.c_double),
                ("Omega_L", ctypes.c_double)]


class nh_history(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("z_max", ctypes.c_double), ("M_Msun", _dp), ("c", _dp),
                ("kappa", _dp)]


class nh_halo(ctypes.Structure):
    _fields_ = [("mass_kind", ctypes.c_int), ("M0_Msun", ctypes.c_double),
                ("mass_alpha", ctypes.c_double), ("z_form", ctypes.c_double),
                ("mass_beta", ctypes.c_double), ("conc_kind", ctypes.c_int),
                ("c0", ctypes.c_double), ("conc_gamma", ctypes.c_double),
                ("kappa_kind", ctypes.c_int), ("kappa_a", ctypes.c_double),
                ("kappa_b", ctypes.c_double), ("geometry", ctypes.c_int),
                ("compensated", ctypes.c_int), ("history", nh_history)]


class nh_f0(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("T_K", ctypes.c_double), ("n", ctypes.c_int),
                ("ln_y0", ctypes.c_double), ("d_ln_y", ctypes.c_double), ("ln_f", _dp)]


class nh_grid(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int), ("r_kpc", _dp), ("n_y", ctypes.c_int), ("y", _dp),
                ("n_mu", ctypes.c_int), ("mu", _dp), ("w_mu", _dp)]


class nh_integrator(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("n_steps", ctypes.c_int), ("rtol", ctypes.c_double),
                ("atol_x", ctypes.c_double), ("atol_v", ctypes.c_double), ("h0", ctypes.c_double),
                ("max_steps", ctypes.c_longlong), ("z_end", ctypes.c_double),
                ("precision", ctypes.c_int), ("z_obs", ctypes.c_double)]


class nh_request(ctypes.Structure):
    _fields_ = [("cosmo", nh_cosmology), ("halo", nh_halo), ("m_eV", ctypes.c_double),
                ("f0", nh_f0), ("grid", nh_grid), ("integ", nh_integrator)]


class nh_stats(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_longlong), ("accepted_steps", ctypes.c_longlong),
                ("rejected_steps", ctypes.c_longlong), ("max_steps_one_traj", ctypes.c_longlong),
                ("n_failed", ctypes.c_longlong), ("fp64_steps", ctypes.c_longlong),
                ("free_exits", ctypes.c_longlong), ("kernel_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


NH_FORM_PLAIN, NH_FORM_BATCH = 0, 1


class nh_tune_result(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("precision", ctypes.c_int), ("block_threads", ctypes.c_int),
                ("batch_slots", ctypes.c_int), ("n_tried", ctypes.c_int), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# Every symbol the header declares, with its ctypes signature.
_SIGNATURES = {
    "nh_context_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "nh_context_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nh_footprint_bytes": (ctypes.c_int, [ctypes.POINTER(nh_request), ctypes.POINTER(ctypes.c_size_t)]),
    "nh_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(nh_request), _dp, ctypes.POINTER(nh_stats)]),
    "nh_solve_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(nh_request), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "nh_last_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(nh_stats)]),
    "nh_last_trajectory_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "nh_solve_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(nh_request), ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "nh_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "nh_solve_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(nh_request),
                                      ctypes.c_void_p, ctypes.POINTER(nh_stats), ctypes.c_void_p]),
    "nh_serve_set_budget": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t]),
    "nh_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(nh_request),
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "nh_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, _dp, ctypes.POINTER(nh_stats)]),
    "nh_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "nh_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "nh_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "nh_version": (ctypes.c_char_p, []),
    "nh_fp64_fma_peak": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "nh_device_function": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(nh_request), ctypes.c_longlong,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "nh_solve_integrand": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(nh_request), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nh_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(nh_request),
                                   ctypes.POINTER(nh_tune_result)]),
    "nh_solve_masses": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(nh_request), ctypes.c_int, _dp,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nh_gauss_legendre": (ctypes.c_int, [ctypes.c_int, _dp, _dp]),
    "nh_set_option": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]),
    "nh_coefficients": (ctypes.c_int, [ctypes.POINTER(nh_request), ctypes.c_int, _dp, _dp]),
}

_lib = None


def lib():
    """Load libnuhalo.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return list(_SIGNATURES)


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _Marshalled:
    """nh_request plus the numpy arrays it points into (kept alive with it)."""

    def __init__(self, req: Request):
        self.r = _arr(req.r_kpc)
        self.y = _arr(req.y)
        self.mu = None if req.mu is None else _arr(req.mu)
        self.w_mu = None if req.w_mu is None else _arr(req.w_mu)
        self.hist = {k: (None if getattr(req, "hist_" + k) is None else _arr(getattr(req, "hist_" + k)))
                     for k in ("M", "c", "kappa")}
        self.ln_f = None if req.f0_ln_f is None else _arr(req.f0_ln_f)
        q = nh_request()
        q.cosmo.H0_km_s_Mpc = req.H0
        q.cosmo.Omega_m = req.Omega_m
        q.cosmo.Omega_L = req.Omega_L
        h = q.halo
        h.mass_kind = _MASS[req.mass_kind]
        h.M0_Msun = req.M0
        h.mass_alpha = req.mass_alpha
        h.z_form = req.z_form
        h.mass_beta = req.mass_beta
        h.conc_kind = _CONC[req.conc_kind]
        h.c0 = req.c0
        h.conc_gamma = req.conc_gamma
        h.kappa_kind = _KAPPA[req.kappa_kind]
        h.kappa_a = req.kappa_a
        h.kappa_b = req.kappa_b
        h.geometry = _GEOM[req.geometry]
        h.compensated = int(bool(req.compensated))
        sizes = {a.size for a in self.hist.values() if a is not None}
        if len(sizes) > 1:
            raise ValueError("hist_M, hist_c and hist_kappa must have the same length")
        h.history.n = sizes.pop() if sizes else 0
        h.history.z_max = req.hist_z_max
        h.history.M_Msun = None if self.hist["M"] is None else self.hist["M"].ctypes.data_as(_dp)
        h.history.c = None if self.hist["c"] is None else self.hist["c"].ctypes.data_as(_dp)
        h.history.kappa = None if self.hist["kappa"] is None else self.hist["kappa"].ctypes.data_as(_dp)
        q.m_eV = req.m_eV
        q.f0.kind = _F0[req.f0_kind]
        q.f0.T_K = req.T_K
        if self.ln_f is not None:
            q.f0.n = self.ln_f.size
            q.f0.ln_y0 = req.f0_ln_y0
            q.f0.d_ln_y = req.f0_d_ln_y
            q.f0.ln_f = self.ln_f.ctypes.data_as(_dp)
        g = q.grid
        g.n_r = self.r.size
        g.r_kpc = self.r.ctypes.data_as(_dp)
        g.n_y = self.y.size
        g.y = self.y.ctypes.data_as(_dp)
        if self.mu is not None:
            g.n_mu = self.mu.size
            g.mu = self.mu.ctypes.data_as(_dp)
            g.w_mu = self.w_mu.ctypes.data_as(_dp)
        else:
            g.n_mu = int(req.n_mu)
            g.mu = None
            g.w_mu = None
        it = q.integ
        it.method = _METHOD[req.method]
        it.n_steps = int(req.n_steps)
        it.rtol = req.rtol
        it.atol_x = 0.0 if req.atol_x is None else req.atol_x
        it.atol_v = 0.0 if req.atol_v is None else req.atol_v
        it.h0 = req.h0
        it.max_steps = int(req.max_steps)
        it.z_end = req.z_end
        it.precision = _PREC[req.precision]
        it.z_obs = req.z_obs
        self.q = q


def marshal(req: Request) -> _Marshalled:
    return _Marshalled(req)


def footprint_bytes(req: Request) -> int:
    """Device bytes the request needs (validates it; needs no GPU)."""
    m = marshal(req)
    out = ctypes.c_size_t()
    rc = lib().nh_footprint_bytes(ctypes.byref(m.q), ctypes.byref(out))
    if rc != NH_OK:
        raise NhError(rc, lib().nh_last_error(None).decode())
    return out.value


def gauss_legendre(n: int):
    """The library's Gauss-Legendre nodes and weights (host computation)."""
    x = np.empty(n)
    w = np.empty(n)
    rc = lib().nh_gauss_legendre(n, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp))
    if rc != NH_OK:
        raise NhError(rc, lib().nh_last_error(None).decode())
    return x, w


def coefficients(req: Request, u) -> np.ndarray:
    """(n, 6) EOM coefficients (A, K, Kc, 1/s, c, R) as the library tabulates them."""
    m = marshal(req)
    u = _arr(u).ravel()
    out = np.empty((u.size, 6))
    rc = lib().nh_coefficients(ctypes.byref(m.q), u.size, u.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    if rc != NH_OK:
        raise NhError(rc, lib().nh_last_error(None).decode())
    return out


def strerror(code: int) -> str:
    return lib().nh_strerror(code).decode()


class Context:
    """One nh_context on a HIP device."""

    def __init__(self, device: int = 0):
        self._lib = lib()
        h = ctypes.c_void_p()
        rc = self._lib.nh_context_create(device, ctypes.byref(h))
        if rc != NH_OK:
            raise NhError(rc, self._lib.nh_last_error(None).decode())
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self._lib.nh_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int, allow=(NH_OK,)):
        if rc not in allow:
            raise NhError(rc, self._lib.nh_last_error(self.h).decode())
        return rc

    def set_option(self, name: str, value: float):
        self._check(self._lib.nh_set_option(self.h, OPTIONS[name], float(value)))

    def last_error(self) -> str:
        return self._lib.nh_last_error(self.h).decode()

    def solve(self, req: Request, allow_failed: bool = False):
        """Synchronous solve: returns (n_over_nbar numpy array, stats dict, status code)."""
        m = marshal(req)
        out = np.empty(m.r.size)
        st = nh_stats()
        rc = self._lib.nh_solve(self.h, ctypes.byref(m.q), out.ctypes.data_as(_dp), ctypes.byref(st))
        self._check(rc, (NH_OK, NH_ESTEPS, NH_ENONFINITE) if allow_failed else (NH_OK,))
        return out, st.as_dict(), rc

    def solve_async(self, req: Request, out: "torch.Tensor", ratio: Optional["torch.Tensor"] = None,
                    stream: Optional["torch.cuda.Stream"] = None):
        """Enqueue on `stream` (default: torch's current stream); out/ratio are float64 device tensors."""
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        if ratio is not None:
            assert ratio.dtype == torch.float64 and ratio.is_cuda and ratio.is_contiguous()
        m = marshal(req)
        if out.numel() < m.r.size:
            raise ValueError("out is too small")
        if ratio is not None and ratio.numel() < req.n_traj:
            raise ValueError("ratio is too small")
        s = stream if stream is not None else torch.cuda.current_stream(out.device)
        rc = self._lib.nh_solve_async(self.h, ctypes.byref(m.q), ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(ratio.data_ptr()) if ratio is not None else None,
                                      ctypes.c_void_p(s.cuda_stream))
        self._check(rc)
        return m

    def last_stats(self, allow_failed: bool = False):
        st = nh_stats()
        rc = self._lib.nh_last_stats(self.h, ctypes.byref(st))
        self._check(rc, (NH_OK, NH_ESTEPS, NH_ENONFINITE) if allow_failed else (NH_OK,))
        return st.as_dict(), rc

    def trajectory_stats(self, n_traj: int):
        """(accepted, rejected, status) per trajectory of the last completed solve
        (one that stored per-trajectory results); n_traj: its trajectory count."""
        acc = np.empty(n_traj, dtype=np.int32)
        rej = np.empty(n_traj, dtype=np.int32)
        st = np.empty(n_traj, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        self._check(self._lib.nh_last_trajectory_stats(self.h, n_traj, acc.ctypes.data_as(ip),
                                                       rej.ctypes.data_as(ip), st.ctypes.data_as(ip)))
        return acc, rej, st

    def solve_noalloc(self, req: Request, out: "torch.Tensor", stream: Optional["torch.cuda.Stream"] = None):
        """nh_solve_noalloc: the plain solve into out (float64 device tensor of n_r),
        allocating nothing; statistics through last_stats()."""
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        m = marshal(req)
        if out.numel() < m.r.size:
            raise ValueError("out is too small")
        s = stream if stream is not None else torch.cuda.current_stream(out.device)
        self._check(self._lib.nh_solve_noalloc(self.h, ctypes.byref(m.q), ctypes.c_void_p(out.data_ptr()),
                                               ctypes.c_void_p(s.cuda_stream)))

    def solve_masses(self, req: Request, masses, out: "torch.Tensor", ratio=None, stream=None):
        """Profiles for several relic masses from one integration (velocities fixed by
        req.y at req.m_eV); out: float64 device tensor of len(masses) * n_r, mass-major."""
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        m = marshal(req)
        ms = np.ascontiguousarray(np.asarray(masses, dtype=np.float64))
        if out.numel() < ms.size * m.r.size:
            raise ValueError("out is too small")
        s = stream if stream is not None else torch.cuda.current_stream(out.device)
        rc = self._lib.nh_solve_masses(self.h, ctypes.byref(m.q), int(ms.size), ms.ctypes.data_as(_dp),
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(ratio.data_ptr()) if ratio is not None else None,
                                       ctypes.c_void_p(s.cuda_stream))
        self._check(rc)

    def solve_integrand(self, req: Request, out: "torch.Tensor", integrand: "torch.Tensor",
                        ratio: Optional["torch.Tensor"] = None, stream=None):
        """Profile plus the direction-integrated distribution per (radius, momentum node):
        integrand[k * n_y + j] = sum_l w_mu,l f0(y_j P_i/P0) (float64 device tensors)."""
        for t in (out, integrand) + ((ratio,) if ratio is not None else ()):
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
        m = marshal(req)
        if out.numel() < m.r.size or integrand.numel() < req.n_r * req.n_y:
            raise ValueError("out or integrand is too small")
        if ratio is not None and ratio.numel() < req.n_traj:
            raise ValueError("ratio is too small")
        s = stream if stream is not None else torch.cuda.current_stream(out.device)
        rc = self._lib.nh_solve_integrand(self.h, ctypes.byref(m.q), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(integrand.data_ptr()),
                                          ctypes.c_void_p(ratio.data_ptr()) if ratio is not None else None,
                                          ctypes.c_void_p(s.cuda_stream))
        self._check(rc)
        return m

    def fp64_fma_peak(self) -> float:
        """Measured FP64 vector FMA throughput of the device, TFLOP/s."""
        t = ctypes.c_double()
        self._check(self._lib.nh_fp64_fma_peak(self.h, ctypes.byref(t)))
        return t.value

    def device_function(self, fn: str, x, req: Optional[Request] = None) -> np.ndarray:
        """The device's own values of an elementary function of the right-hand side
        (nh_device_function): fn "nfw_I" (x = q) or "pow_factor" (x = u, for req)."""
        code = {"nfw_I": 1, "pow_factor": 2}[fn]
        xs = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        ys = np.empty_like(xs)
        m = marshal(req) if req is not None else None
        rc = self._lib.nh_device_function(self.h, code, ctypes.byref(m.q) if m is not None else None, int(xs.size),
                                          xs.ctypes.data_as(_dp), ys.ctypes.data_as(_dp))
        self._check(rc)
        return ys

    def autotune(self, reqs, form: str = "plain") -> dict:
        """Time the launch configurations of one form on a sample of requests and
        make the fastest the context's default (nh_autotune); returns the choice."""
        ms = [marshal(r) for r in reqs]
        arr = (nh_request * len(ms))(*[m.q for m in ms])
        res = nh_tune_result()
        f = {"plain": NH_FORM_PLAIN, "batch": NH_FORM_BATCH}[form]
        self._check(self._lib.nh_autotune(self.h, f, len(ms), arr, ctypes.byref(res)))
        return res.as_dict()

    def solve_batch(self, reqs, out: "torch.Tensor", stream=None):
        """Solve several requests in one persistent launch; out (float64 device tensor)
        receives the concatenated profiles in request order.  Waits for completion."""
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        ms = [marshal(r) for r in reqs]
        if out.numel() < sum(m.r.size for m in ms):
            raise ValueError("out is too small")
        arr = (nh_request * len(ms))(*[m.q for m in ms])
        stats = (nh_stats * len(ms))()
        s = stream if stream is not None else torch.cuda.current_stream(out.device)
        rc = self._lib.nh_solve_batch(self.h, len(ms), arr, ctypes.c_void_p(out.data_ptr()), stats,
                                      ctypes.c_void_p(s.cuda_stream))
        self._check(rc, (NH_OK, NH_ESTEPS, NH_ENONFINITE))
        return [st.as_dict() for st in stats], rc

    # ---- serving ----
    def set_budget(self, nbytes: int):
        self._check(self._lib.nh_serve_set_budget(self.h, ctypes.c_size_t(int(nbytes))))

    def submit(self, req: Request):
        """Returns a ticket, or None when the request does not fit the free budget now."""
        m = marshal(req)
        t = ctypes.c_uint64()
        rc = self._lib.nh_submit(self.h, ctypes.byref(m.q), ctypes.byref(t))
        if rc == NH_EBUSY:
            return None
        self._check(rc)
        return t.value

    def poll(self, ticket: int, n_r: int):
        """Returns (profile, stats, rc) when done, None while running."""
        out = np.empty(n_r)
        st = nh_stats()
        rc = self._lib.nh_poll(self.h, ctypes.c_uint64(ticket), out.ctypes.data_as(_dp), ctypes.byref(st))
        if rc == NH_ENOTREADY:
            return None
        self._check(rc, (NH_OK, NH_ESTEPS, NH_ENONFINITE))
        return out, st.as_dict(), rc

    def cancel(self, ticket: int) -> int:
        return self._lib.nh_cancel(self.h, ctypes.c_uint64(ticket))
