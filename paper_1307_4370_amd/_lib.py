"""ctypes binding of libriop.so (argument marshalling only).

Every computation happens in the HIP library; this module converts torch
tensors to device pointers, allocates outputs and turns status codes into
exceptions.  There is no fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libriop.so")

RIOP_F32 = 1
RIOP_F64 = 2
FULL_MASK = (1 << 9) - 1

STATUS = {0: "RIOP_OK", -1: "RIOP_EINVAL", -2: "RIOP_ESHAPE", -3: "RIOP_ENOMEM",
          -4: "RIOP_EDEVICE", -5: "RIOP_ENOTSUP", -6: "RIOP_ENONFINITE"}

# Entry points declared in include/riop.h (checked by the ABI test).
EXPORTS = ("riop_plan_create", "riop_plan_destroy", "riop_plan_info", "riop_plan_layout",
           "riop_plan_sync", "riop_device_bytes", "riop_noise_bound", "riop_gram_build", "riop_gram_release",
           "riop_phi", "riop_phi_adj", "riop_phi_sorted", "riop_phi_adj_sorted",
           "riop_apply_q", "riop_psi_adj", "riop_psi", "riop_cg", "riop_cg_noalloc", "riop_gamma",
           "riop_sdmm", "riop_sdmm_reweighted", "riop_sdmm_blocks", "riop_sdmm_tv", "riop_batch_create", "riop_batch_sdmm", "riop_batch_plan", "riop_batch_tile",
           "riop_batch_destroy", "riop_autotune_tile", "riop_sdmm_init", "riop_sdmm_step", "riop_sdmm_finish", "riop_timing_enable", "riop_timing_read", "riop_timing_kinds",
           "riop_timing_name", "riop_last_error", "riop_version")


class RiopError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("oversample", ctypes.c_int32), ("M", ctypes.c_int64),
                ("J", ctypes.c_int32), ("levels", ctypes.c_int32), ("dict_mask", ctypes.c_uint32),
                ("prec", ctypes.c_int32), ("tile", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("K", ctypes.c_int32), ("J", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("q", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("M", ctypes.c_int64), ("tile", ctypes.c_int32), ("ntiles", ctypes.c_int32),
                ("nunits", ctypes.c_int32), ("kernel_degree", ctypes.c_int32),
                ("kb_beta", ctypes.c_double), ("kernel_fit_err", ctypes.c_double),
                ("device_bytes", ctypes.c_int64)]


class SdmmParams(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("n_cg", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("beta", ctypes.c_double), ("xi", ctypes.c_double), ("tau", ctypes.c_double),
                ("early_stop", ctypes.c_int32), ("resume", ctypes.c_int32),
                ("f1_prev", ctypes.c_double), ("weights", ctypes.c_void_p),
                ("z1", ctypes.c_void_p), ("z2", ctypes.c_void_p), ("z3", ctypes.c_void_p),
                ("rhs", ctypes.c_void_p), ("history", ctypes.POINTER(ctypes.c_double)),
                ("cg_tol", ctypes.c_double)]

HIST = 5  # doubles per iteration in the SDMM history: f1, zeta, nu, CG <r, r>, CG iterations


class ReweightParams(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32), ("delta0", ctypes.c_double), ("rho", ctypes.c_double),
                ("delta_min", ctypes.c_double), ("tol", ctypes.c_double)]


class SdmmStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("gamma", ctypes.c_double), ("f1", ctypes.c_double),
                ("zeta", ctypes.c_double), ("nu", ctypes.c_double), ("status_iter", ctypes.c_int32),
                ("cg_iters", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libriop.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with paper_1307_4370_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.riop_plan_create.argtypes = [ctypes.POINTER(Desc), vp, vp, ctypes.POINTER(vp)]
        L.riop_plan_destroy.argtypes = [vp]
        L.riop_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.riop_plan_layout.argtypes = [vp, vp, vp, vp, vp]
        for name in ("riop_phi", "riop_phi_adj", "riop_phi_sorted", "riop_phi_adj_sorted",
                     "riop_apply_q", "riop_psi_adj", "riop_psi"):
            getattr(L, name).argtypes = [vp, vp, vp, vp]
        L.riop_cg.argtypes = [vp, vp, vp, i32, dbl, ctypes.POINTER(dbl), ctypes.POINTER(i32), vp]
        L.riop_cg_noalloc.argtypes = [vp, vp, vp, i32, dbl, ctypes.POINTER(dbl), ctypes.POINTER(i32), vp]
        L.riop_plan_sync.argtypes = [vp, vp]
        L.riop_gram_build.argtypes = [vp, vp]
        L.riop_gram_release.argtypes = [vp]
        L.riop_device_bytes.argtypes = []
        L.riop_noise_bound.argtypes = [i64, dbl]
        L.riop_gamma.argtypes = [vp, vp, dbl, ctypes.POINTER(dbl), vp]
        L.riop_sdmm.argtypes = [vp, vp, dbl, ctypes.POINTER(SdmmParams), vp,
                                ctypes.POINTER(SdmmStats), vp]
        L.riop_sdmm_init.argtypes = [vp, vp, dbl, ctypes.POINTER(SdmmParams), vp, vp]
        L.riop_sdmm_tv.argtypes = [vp, vp, dbl, ctypes.POINTER(SdmmParams), i32, ctypes.POINTER(ReweightParams), vp,
                                   vp, ctypes.POINTER(SdmmStats), ctypes.POINTER(i32), vp]
        L.riop_sdmm_blocks.argtypes = [vp, vp, i32, vp, ctypes.POINTER(dbl), ctypes.POINTER(SdmmParams), vp,
                                       ctypes.POINTER(SdmmStats), ctypes.POINTER(dbl), vp]
        L.riop_sdmm_reweighted.argtypes = [vp, vp, dbl, ctypes.POINTER(SdmmParams), ctypes.POINTER(ReweightParams),
                                           vp, vp, ctypes.POINTER(SdmmStats), ctypes.POINTER(i32), vp]
        L.riop_sdmm_step.argtypes = [vp, i32, vp]
        L.riop_sdmm_finish.argtypes = [vp, ctypes.POINTER(SdmmParams), vp, ctypes.POINTER(SdmmStats), vp]
        L.riop_batch_create.argtypes = [ctypes.POINTER(Desc), i32, ctypes.POINTER(vp), i32, vp,
                                        ctypes.POINTER(vp)]
        L.riop_batch_sdmm.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(dbl), ctypes.POINTER(SdmmParams),
                                      i32, ctypes.POINTER(vp), ctypes.POINTER(SdmmStats), vp]
        L.riop_batch_plan.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.riop_batch_tile.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
        L.riop_batch_destroy.argtypes = [vp]
        L.riop_autotune_tile.argtypes = [ctypes.POINTER(Desc), vp, i32, vp, ctypes.POINTER(i32),
                                         ctypes.POINTER(dbl)]
        L.riop_timing_enable.argtypes = [vp, i32]
        L.riop_timing_read.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.riop_timing_kinds.argtypes = []
        L.riop_timing_name.argtypes = [i32]
        for name in EXPORTS:
            if name not in ("riop_last_error", "riop_version", "riop_timing_name", "riop_device_bytes",
                            "riop_noise_bound"):
                getattr(L, name).restype = ctypes.c_int
        L.riop_device_bytes.restype = i64
        L.riop_noise_bound.restype = dbl
        L.riop_timing_name.restype = ctypes.c_char_p
        L.riop_last_error.restype = ctypes.c_char_p
        L.riop_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise RiopError(status, lib().riop_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


class Plan:
    """One coverage: Phi, Phi^dagger, Psi, Psi^dagger, CG and SDMM on the GPU.

    uv: (M, 2) real tensor on the GPU (float32 for prec='f32', float64 for 'f64'),
    continuous (u, v) in radians per pixel in [-pi, pi].
    """

    def __init__(self, n: int, uv: torch.Tensor, J: int = 8, levels: int = 4,
                 dict_mask: int = FULL_MASK, prec: str = "f32", tile: int = 0, stream=None):
        self.prec = prec
        self.rdtype = torch.float32 if prec == "f32" else torch.float64
        self.cdtype = torch.complex64 if prec == "f32" else torch.complex128
        if uv.dtype != self.rdtype or not uv.is_cuda or uv.dim() != 2 or uv.shape[1] != 2:
            raise ValueError(f"uv must be a (M, 2) {self.rdtype} CUDA tensor")
        uv = uv.contiguous()
        self.device = uv.device
        self.n, self.M, self.J, self.levels = n, uv.shape[0], J, levels
        self.q = bin(dict_mask).count("1")
        d = Desc(n=n, oversample=2, M=self.M, J=J, levels=levels, dict_mask=dict_mask,
                 prec=RIOP_F32 if prec == "f32" else RIOP_F64, tile=tile)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().riop_plan_create(ctypes.byref(d), uv.data_ptr(), _stream(stream), ctypes.byref(h)))
        self._h = h
        self._uv = uv

    # -- helpers -----------------------------------------------------------------
    def _c(self, t: torch.Tensor, shape, name: str) -> torch.Tensor:
        if t.dtype != self.cdtype or t.device != self.device or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must be a {self.cdtype} tensor of shape {tuple(shape)} on {self.device}")
        return t.contiguous()

    def _new(self, shape):
        return torch.empty(shape, dtype=self.cdtype, device=self.device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().riop_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = Info()
        _check(lib().riop_plan_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    def timing(self, on: bool = True):
        """Enable (and reset) or disable per-kernel event timing."""
        _check(lib().riop_timing_enable(self._h, int(on)))

    def timing_read(self) -> dict:
        """{kernel kind: (total ms, launches)} since timing was enabled."""
        out = {}
        for k in range(lib().riop_timing_kinds()):
            ms, cnt = ctypes.c_double(), ctypes.c_int64()
            _check(lib().riop_timing_read(self._h, k, ctypes.byref(ms), ctypes.byref(cnt)))
            out[lib().riop_timing_name(k).decode()] = (ms.value, cnt.value)
        return out

    def layout(self, stream=None):
        inf = self.info()
        perm = torch.empty(self.M, dtype=torch.int32, device=self.device)
        cell = torch.empty(self.M, dtype=torch.int32, device=self.device)
        ts = torch.empty(inf["ntiles"] + 1, dtype=torch.int32, device=self.device)
        _check(lib().riop_plan_layout(self._h, perm.data_ptr(), cell.data_ptr(), ts.data_ptr(), _stream(stream)))
        return perm, cell, ts

    # -- operators ---------------------------------------------------------------
    def phi(self, x, y=None, sorted: bool = False, stream=None):
        x = self._c(x, (self.n, self.n), "x")
        y = self._new(self.M) if y is None else y
        fn = lib().riop_phi_sorted if sorted else lib().riop_phi
        _check(fn(self._h, x.data_ptr(), y.data_ptr(), _stream(stream)))
        return y

    def phi_adj(self, y, x=None, sorted: bool = False, stream=None):
        y = self._c(y, (self.M,), "y")
        x = self._new((self.n, self.n)) if x is None else x
        fn = lib().riop_phi_adj_sorted if sorted else lib().riop_phi_adj
        _check(fn(self._h, y.data_ptr(), x.data_ptr(), _stream(stream)))
        return x

    def apply_q(self, x, out=None, stream=None):
        x = self._c(x, (self.n, self.n), "x")
        out = self._new((self.n, self.n)) if out is None else out
        _check(lib().riop_apply_q(self._h, x.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def psi_adj(self, x, alpha=None, stream=None):
        x = self._c(x, (self.n, self.n), "x")
        alpha = self._new((self.q, self.n, self.n)) if alpha is None else alpha
        _check(lib().riop_psi_adj(self._h, x.data_ptr(), alpha.data_ptr(), _stream(stream)))
        return alpha

    def psi(self, alpha, x=None, stream=None):
        alpha = self._c(alpha, (self.q, self.n, self.n), "alpha")
        x = self._new((self.n, self.n)) if x is None else x
        _check(lib().riop_psi(self._h, alpha.data_ptr(), x.data_ptr(), _stream(stream)))
        return x

    def cg(self, b, x0=None, n_iter: int = 16, tol: float = 0.0, stream=None, with_iters: bool = False):
        """Solve Q x = b with at most n_iter CG iterations (stopping once
        ||r|| <= tol ||r_0|| when tol > 0); returns (x, final <r, r>) or, with
        with_iters, (x, final <r, r>, iterations that changed x)."""
        b = self._c(b, (self.n, self.n), "b")
        x = torch.zeros_like(b) if x0 is None else self._c(x0, (self.n, self.n), "x0").clone()
        rr = ctypes.c_double()
        it = ctypes.c_int32()
        _check(lib().riop_cg(self._h, b.data_ptr(), x.data_ptr(), n_iter, float(tol), ctypes.byref(rr),
                             ctypes.byref(it), _stream(stream)))
        return (x, rr.value, it.value) if with_iters else (x, rr.value)

    def gram_build(self, stream=None):
        """Precompute G^T G; CG and Q then apply it instead of degridding and gridding."""
        _check(lib().riop_gram_build(self._h, _stream(stream)))

    def gram_release(self):
        _check(lib().riop_gram_release(self._h))

    def sync(self, stream=None):
        """Synchronise; raises RiopError(RIOP_ENONFINITE) if an earlier call's input held NaN or Inf."""
        _check(lib().riop_plan_sync(self._h, _stream(stream)))

    def gamma(self, y, beta: float = 1e-3, stream=None) -> float:
        y = self._c(y, (self.M,), "y")
        g = ctypes.c_double()
        _check(lib().riop_gamma(self._h, y.data_ptr(), beta, ctypes.byref(g), _stream(stream)))
        return g.value

    def sdmm(self, y, eps: float, T: int, n_cg: int = 16, gamma: float = 0.0, beta: float = 1e-3,
             x0=None, weights=None, state: dict | None = None, early_stop: bool = False,
             xi: float = 1e-3, tau: float = 0.1, cg_tol: float = 0.0, stream=None, stats_out: dict | None = None):
        """Run Algorithm 1.  Returns (x, stats, history, state).

        ``state`` (optional) is a dict with z1, z2, z3, rhs tensors and f1_prev;
        passing one returned by an earlier call resumes that run.
        """
        y = self._c(y, (self.M,), "y")
        n, q = self.n, self.q
        resume = state is not None
        if state is None:
            state = {"z1": self._new((q, n, n)), "z2": self._new(self.M), "z3": self._new((n, n)),
                     "rhs": self._new((n, n)), "f1_prev": 0.0}
        if x0 is not None:
            x = self._c(x0, (n, n), "x0").clone()
        elif resume:
            raise ValueError("resuming needs x0 (the previous iterate)")
        else:
            x = None
        w = None
        if weights is not None:
            if weights.dtype != self.rdtype or tuple(weights.shape) != (q, n, n):
                raise ValueError("weights must be a real tensor of shape (q, n, n)")
            w = weights.contiguous()
        hist = (ctypes.c_double * (HIST * max(1, T)))()
        prm = SdmmParams(T=T, n_cg=n_cg, gamma=gamma, beta=beta, xi=xi, tau=tau,
                         early_stop=int(early_stop), resume=int(resume), f1_prev=state["f1_prev"],
                         weights=_ptr(w), z1=state["z1"].data_ptr(), z2=state["z2"].data_ptr(),
                         z3=state["z3"].data_ptr(), rhs=state["rhs"].data_ptr(), history=hist,
                         cg_tol=float(cg_tol))
        st = SdmmStats()
        if x is None:
            x = torch.zeros((n, n), dtype=self.cdtype, device=self.device)
        status = lib().riop_sdmm(self._h, y.data_ptr(), float(eps), ctypes.byref(prm), x.data_ptr(),
                                 ctypes.byref(st), _stream(stream))
        if stats_out is not None:
            stats_out.update({k: getattr(st, k) for k, _ in SdmmStats._fields_})
        _check(status)
        history = [tuple(hist[HIST * t:HIST * t + HIST]) for t in range(min(st.iters, T))]
        state["f1_prev"] = st.f1 if st.iters else state["f1_prev"]
        stats = {k: getattr(st, k) for k, _ in SdmmStats._fields_}
        return x, stats, history, state


    def sdmm_enqueue(self, y, eps: float, T: int, n_cg: int = 16, gamma: float = 0.0, beta: float = 1e-3,
                     cg_tol: float = 0.0, stream=None):
        """Algorithm 1's set-up and T iterations enqueued without waiting
        (riop_sdmm_init, riop_sdmm_step); sdmm_collect returns the result."""
        y = self._c(y, (self.M,), "y")
        prm = SdmmParams(T=T, n_cg=n_cg, gamma=gamma, beta=beta, xi=1e-3, tau=0.1, cg_tol=float(cg_tol))
        _check(lib().riop_sdmm_init(self._h, y.data_ptr(), float(eps), ctypes.byref(prm), None, _stream(stream)))
        _check(lib().riop_sdmm_step(self._h, int(T), _stream(stream)))

    def sdmm_collect(self, stream=None):
        """(x, stats) of the run enqueued by sdmm_enqueue (riop_sdmm_finish; synchronises)."""
        x = self._new((self.n, self.n))
        st = SdmmStats()
        _check(lib().riop_sdmm_finish(self._h, None, x.data_ptr(), ctypes.byref(st), _stream(stream)))
        return x, {k: getattr(st, k) for k, _ in SdmmStats._fields_}

    def sdmm_tv(self, y, eps: float, T: int, n_cg: int = 16, n_inner: int = 20, weights=None, gamma: float = 0.0,
                beta: float = 1e-3, x0=None, reweight: dict | None = None, cg_tol: float = 0.0,
                early_stop: bool = False, xi: float = 1e-3, tau: float = 0.1, stream=None):
        """Weighted TV with positivity (TV, or RWTV with ``reweight`` = dict of
        outer, delta0, rho, delta_min, tol).  weights: (n, n) real tensor, one
        per pixel's gradient magnitude.  Returns (x, stats, history, passes,
        weights of the last pass or None)."""
        y = self._c(y, (self.M,), "y")
        n = self.n
        x = (torch.zeros((n, n), dtype=self.cdtype, device=self.device) if x0 is None
             else self._c(x0, (n, n), "x0").clone())
        w = None
        if weights is not None:
            if weights.dtype != self.rdtype or tuple(weights.shape) != (n, n):
                raise ValueError("TV weights must be a real tensor of shape (n, n)")
            w = weights.contiguous()
        rw, wout, hist = None, None, None
        if reweight is not None:
            rw = ReweightParams(outer=reweight.get("outer", 3), delta0=reweight.get("delta0", 0.0),
                                rho=reweight.get("rho", 0.1), delta_min=reweight.get("delta_min", 0.0),
                                tol=reweight.get("tol", 0.0))
            wout = torch.empty((n, n), dtype=self.rdtype, device=self.device)
        else:
            hist = (ctypes.c_double * (HIST * max(1, T)))()
        prm = SdmmParams(T=T, n_cg=n_cg, gamma=gamma, beta=beta, xi=xi, tau=tau, early_stop=int(early_stop),
                         weights=_ptr(w), history=hist, cg_tol=float(cg_tol))
        st = SdmmStats()
        passes = ctypes.c_int32()
        _check(lib().riop_sdmm_tv(self._h, y.data_ptr(), float(eps), ctypes.byref(prm), n_inner,
                                  ctypes.byref(rw) if rw is not None else None, x.data_ptr(), _ptr(wout),
                                  ctypes.byref(st), ctypes.byref(passes), _stream(stream)))
        history = ([tuple(hist[HIST * t:HIST * t + HIST]) for t in range(min(st.iters, T))]
                   if hist is not None else None)
        return x, {k: getattr(st, k) for k, _ in SdmmStats._fields_}, history, passes.value, wout

    def sdmm_blocks(self, y, eps, block_of, T: int, n_cg: int = 16, gamma: float = 0.0, beta: float = 1e-3,
                    x0=None, weights=None, cg_tol: float = 0.0, early_stop: bool = False, xi: float = 1e-3,
                    tau: float = 0.1, stream=None):
        """Block SDMM: one l2 ball per data block.  block_of: int32 tensor (M,)
        of block indices in caller order; eps: one bound per block.  Returns
        (x, stats, history, per-block nu at the last iteration)."""
        y = self._c(y, (self.M,), "y")
        R = len(eps)
        if block_of.dtype != torch.int32 or tuple(block_of.shape) != (self.M,) or block_of.device != self.device:
            raise ValueError(f"block_of must be an int32 tensor of shape ({self.M},) on {self.device}")
        block_of = block_of.contiguous()
        n = self.n
        x = (torch.zeros((n, n), dtype=self.cdtype, device=self.device) if x0 is None
             else self._c(x0, (n, n), "x0").clone())
        w = None
        if weights is not None:
            if weights.dtype != self.rdtype or tuple(weights.shape) != (self.q, n, n):
                raise ValueError("weights must be a real tensor of shape (q, n, n)")
            w = weights.contiguous()
        hist = (ctypes.c_double * (HIST * max(1, T)))()
        prm = SdmmParams(T=T, n_cg=n_cg, gamma=gamma, beta=beta, xi=xi, tau=tau, early_stop=int(early_stop),
                         weights=_ptr(w), history=hist, cg_tol=float(cg_tol))
        st = SdmmStats()
        ep = (ctypes.c_double * R)(*[float(e) for e in eps])
        nu = (ctypes.c_double * R)()
        _check(lib().riop_sdmm_blocks(self._h, y.data_ptr(), R, block_of.data_ptr(), ep, ctypes.byref(prm),
                                      x.data_ptr(), ctypes.byref(st), nu, _stream(stream)))
        history = [tuple(hist[HIST * t:HIST * t + HIST]) for t in range(min(st.iters, T))]
        return x, {k: getattr(st, k) for k, _ in SdmmStats._fields_}, history, list(nu)

    def sdmm_reweighted(self, y, eps: float, T: int, n_cg: int = 16, outer: int = 3, delta0: float = 0.0,
                        rho: float = 0.1, delta_min: float = 0.0, tol: float = 0.0, gamma: float = 0.0,
                        beta: float = 1e-3, x0=None, cg_tol: float = 0.0, early_stop: bool = False,
                        xi: float = 1e-3, tau: float = 0.1, stream=None):
        """Reweighted l1 (SARA): pass 0 with W = I, then up to `outer` passes
        with w = delta / (delta + |Psi^dagger x|).  Returns (x, stats of the
        last pass, passes run, weights of the last pass)."""
        y = self._c(y, (self.M,), "y")
        n = self.n
        x = (torch.zeros((n, n), dtype=self.cdtype, device=self.device) if x0 is None
             else self._c(x0, (n, n), "x0").clone())
        w = torch.empty((self.q, n, n), dtype=self.rdtype, device=self.device)
        prm = SdmmParams(T=T, n_cg=n_cg, gamma=gamma, beta=beta, xi=xi, tau=tau, early_stop=int(early_stop),
                         cg_tol=float(cg_tol))
        rw = ReweightParams(outer=outer, delta0=delta0, rho=rho, delta_min=delta_min, tol=tol)
        st = SdmmStats()
        passes = ctypes.c_int32()
        _check(lib().riop_sdmm_reweighted(self._h, y.data_ptr(), float(eps), ctypes.byref(prm), ctypes.byref(rw),
                                          x.data_ptr(), w.data_ptr(), ctypes.byref(st), ctypes.byref(passes),
                                          _stream(stream)))
        return x, {k: getattr(st, k) for k, _ in SdmmStats._fields_}, passes.value, w


class _BorrowedPlan(Plan):
    """A channel plan owned by a Batch (not destroyed by Python)."""

    def __init__(self, handle, n, M, J, levels, q, prec, device):
        self._h = handle
        self.prec = prec
        self.rdtype = torch.float32 if prec == "f32" else torch.float64
        self.cdtype = torch.complex64 if prec == "f32" else torch.complex128
        self.device = device
        self.n, self.M, self.J, self.levels, self.q = n, M, J, levels, q

    def close(self):
        self._h = ctypes.c_void_p()


class Batch:
    """Many channels of uneven sizes solved by SDMM in one replayed HIP graph.

    channels: list of (n, uv tensor) with uv a (M_c, 2) real CUDA tensor.
    """

    def __init__(self, channels, J: int = 8, levels: int = 4, dict_mask: int = FULL_MASK,
                 prec: str = "f32", autotune: bool = True, stream=None):
        self.prec = prec
        rd = torch.float32 if prec == "f32" else torch.float64
        self.cdtype = torch.complex64 if prec == "f32" else torch.complex128
        self.uv = [uv.contiguous() for _, uv in channels]
        for uv in self.uv:
            if uv.dtype != rd or not uv.is_cuda or uv.dim() != 2 or uv.shape[1] != 2:
                raise ValueError(f"uv must be (M, 2) {rd} CUDA tensors")
        self.device = self.uv[0].device
        self.sizes = [(n, uv.shape[0]) for (n, _), uv in zip(channels, self.uv)]
        nc = len(channels)
        descs = (Desc * nc)(*[Desc(n=n, oversample=2, M=M, J=J, levels=levels, dict_mask=dict_mask,
                                   prec=RIOP_F32 if prec == "f32" else RIOP_F64) for n, M in self.sizes])
        uvp = (ctypes.c_void_p * nc)(*[uv.data_ptr() for uv in self.uv])
        h = ctypes.c_void_p()
        _check(lib().riop_batch_create(descs, nc, uvp, int(autotune), _stream(stream), ctypes.byref(h)))
        self._h = h
        q = bin(dict_mask).count("1")
        self.plans = []
        for c, (n, M) in enumerate(self.sizes):
            ph = ctypes.c_void_p()
            _check(lib().riop_batch_plan(self._h, c, ctypes.byref(ph)))
            self.plans.append(_BorrowedPlan(ph, n, M, J, levels, q, prec, self.device))

    def tiles(self):
        out = []
        for c in range(len(self.sizes)):
            t = ctypes.c_int32()
            ms = (ctypes.c_double * 4)()
            _check(lib().riop_batch_tile(self._h, c, ctypes.byref(t), ms))
            out.append((t.value, list(ms)))
        return out

    def sdmm(self, ys, eps, T: int, n_cg: int = 16, gamma: float = 0.0, beta: float = 1e-3,
             iters_per_graph: int = 10, stream=None):
        nc = len(self.sizes)
        ys = [y.contiguous() for y in ys]
        xs = [torch.empty((n, n), dtype=self.cdtype, device=self.device) for n, _ in self.sizes]
        yp = (ctypes.c_void_p * nc)(*[y.data_ptr() for y in ys])
        xp = (ctypes.c_void_p * nc)(*[x.data_ptr() for x in xs])
        ep = (ctypes.c_double * nc)(*[float(e) for e in eps])
        st = (SdmmStats * nc)()
        prm = SdmmParams(T=T, n_cg=n_cg, gamma=gamma, beta=beta, xi=1e-3, tau=0.1)
        _check(lib().riop_batch_sdmm(self._h, yp, ep, ctypes.byref(prm), iters_per_graph, xp, st, _stream(stream)))
        stats = [{k: getattr(s, k) for k, _ in SdmmStats._fields_} for s in st]
        return xs, stats

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            for p in self.plans:
                p.close()
            _check(lib().riop_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_tile(n: int, uv: torch.Tensor, J: int = 8, prec: str = "f32", reps: int = 3, stream=None):
    """(best tile, ms per Phi/Phi^dagger pair for tiles 8, 16, 32, 64)."""
    d = Desc(n=n, oversample=2, M=uv.shape[0], J=J, levels=1, dict_mask=1,
             prec=RIOP_F32 if prec == "f32" else RIOP_F64)
    t = ctypes.c_int32()
    ms = (ctypes.c_double * 4)()
    _check(lib().riop_autotune_tile(ctypes.byref(d), uv.contiguous().data_ptr(), reps, _stream(stream),
                                    ctypes.byref(t), ms))
    return t.value, list(ms)


def noise_bound(M: int, sigma: float) -> float:
    """The l2 bound eps on the noise of M visibilities (riop_noise_bound)."""
    return float(lib().riop_noise_bound(int(M), float(sigma)))


def device_bytes() -> int:
    """Device bytes held by the library's allocations in this process."""
    return int(lib().riop_device_bytes())


def version() -> str:
    return lib().riop_version().decode()
