"""MI355X (gfx950) guided-filter non-blind deconvolution.

Thin Python binding over ``libgfdeconv.so`` (declared in ``include/gfdeconv.h``).  Every step
of the method runs in the library's HIP kernels; this module only checks tensor arguments,
passes device pointers and the current HIP stream, and turns status codes into exceptions.
PyTorch supplies device memory and streams.

Method: Yang, Zhu, Zhang, Huang, "Guided Filter based Edge-preserving Image Non-blind
Deconvolution" -- Sec. 3.1 (Steps 0-3, Eqs.(8)-(9)), Sec. 3.2 (Eqs.(10)-(12)), Sec. 2
(Eqs.(3)-(5)).
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["GFDError", "GFDeconv", "GFDeconvBatch", "GfdImage", "GFDeconvFn", "deconvolve_autograd", "deconvolve",
           "deconvolve_static", "guided_filter", "guided_filter_clipped", "guided_filter_color", "spectral_solve", "discrepancy_lambda",
           "library_path", "load_library", "EXPORTS", "FLAG_INF_BRANCH", "FLAG_NO_ROOT", "FLAG_NONFINITE",
           "FLAG_UNCONVERGED", "STRIP_MAX_WINDOW"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libgfdeconv.so"
_lib = None

FLAG_INF_BRANCH, FLAG_NO_ROOT, FLAG_NONFINITE, FLAG_UNCONVERGED = 1, 2, 4, 8
STRIP_MAX_WINDOW = 17  # widest window of the single-pass filter kernels; wider ones run as separable passes
BOUNDARY_PERIODIC, BOUNDARY_CLIP, BOUNDARY_PAD = 0, 1, 2
_ERRNAMES = {-1: "GFD_ERR_ARG", -2: "GFD_ERR_SIZE", -3: "GFD_ERR_HIP", -4: "GFD_ERR_NOMEM", -5: "GFD_ERR_STATE",
             -6: "GFD_ERR_UNIMPLEMENTED"}

_vp, _i, _f, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
# name -> (restype, argtypes)
EXPORTS = {
    "deconv_init": (_i, [ctypes.POINTER(_vp), _vp, _i, _i, _vp, _i, _i, _d, _i, _f, _d, _vp]),
    "deconv_init_batch": (_i, [ctypes.POINTER(_vp), _vp, _i, _vp]),
    "deconv_image_info": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "deconv_image_domain": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "deconv_iterate": (_i, [_vp, _i, _vp, _vp, _vp]),
    "guided_filter": (_i, [_vp, _vp, _vp, _i, _i, _i, _f, _vp]),
    "guided_filter_color": (_i, [_vp, _vp, _vp, _i, _i, _i, _f, _vp]),
    "guided_filter_clipped": (_i, [_vp, _vp, _vp, _i, _i, _i, _f, _vp]),
    "spectral_solve": (_i, [_vp, _vp, _f, _vp, _vp, _vp]),
    "discrepancy_lambda": (_i, [_vp, _vp, _vp, _vp]),
    "deconv_set_scales": (_i, [_vp, _vp, _i, _vp]),
    "deconv_set_estimate": (_i, [_vp, _vp, _vp]),
    "deconv_reset": (_i, [_vp, _vp]),
    "deconv_info": (_i, [_vp, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_i)]),
    "deconv_get_status": (_i, [_vp, ctypes.POINTER(ctypes.c_uint)]),
    "deconv_set_graph": (_i, [_vp, _i]),
    "deconv_profile": (_i, [_vp, _i, ctypes.POINTER(_f), _i, _vp]),
    "deconv_backward": (_i, [_vp, _vp, _vp, _vp, _i, _vp]),
    "deconv_autotune": (_i, [_vp, _i, ctypes.POINTER(_i), _vp]),
    "deconv_set_tuning": (_i, [_vp, ctypes.POINTER(_i)]),
    "deconvolve_static": (_i, [_vp, _i, _i, _vp, _i, _i, _d, _i, _f, _d, _i, _vp, _vp, _vp]),
    "deconv_destroy": (None, [_vp]),
    "gfd_last_error": (ctypes.c_char_p, []),
}


class GfdImage(ctypes.Structure):
    """``gfd_image`` of the C ABI: one image of a batch."""
    _fields_ = [("y", _vp), ("M", _i), ("N", _i), ("h", _vp), ("kh", _i), ("kw", _i), ("sigma2", _d), ("w", _i),
                ("eps", _f), ("rho", _d), ("boundary", _i)]


class GFDError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {message}")
        self.code = code


def library_path() -> str:
    return os.path.join(_HERE, _LIBNAME)


def load_library():
    """Load the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_1609_01839_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        raise GFDError(rc, load_library().gfd_last_error().decode())


def _dev(t: torch.Tensor, name: str, shape=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor on the GPU")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class GFDeconv:
    """One deconvolution problem bound to the current GPU (a library context).

    ``y`` (M x N) and ``h`` (kh x kw, odd sides) are float32 GPU tensors; ``sigma2`` the noise
    variance; ``w``, ``eps`` the guided-filter window and regulariser; ``rho=None`` takes
    Eq.(12), otherwise 0 < rho <= 1.  ``clip`` clips the guided filter's windows to the image;
    ``pad`` treats y as a non-circular blur and solves on a padded domain (``domain``), returning
    estimates of y's size (GFD_BOUNDARY_* of the C ABI).
    """

    def __init__(self, y: torch.Tensor, h: torch.Tensor, sigma2: float, w: int, eps: float, rho=None,
                 clip: bool = False, pad: bool = False):
        lib = load_library()
        if y.dim() != 2 or h.dim() != 2:
            raise ValueError("y and h must be 2-D")
        self.M, self.N = (int(s) for s in y.shape)
        self.device = y.device
        self._y, self._h = y, h
        ctx = _vp()
        boundary = (BOUNDARY_CLIP if clip else 0) | (BOUNDARY_PAD if pad else 0)
        if boundary == 0:
            rc = lib.deconv_init(ctypes.byref(ctx), _dev(y, "y"), self.M, self.N, _dev(h, "h"), int(h.shape[0]),
                                 int(h.shape[1]), float(sigma2), int(w), float(eps),
                                 -1.0 if rho is None else float(rho), _stream(self.device))
        else:
            img = GfdImage(_dev(y, "y"), self.M, self.N, _dev(h, "h"), int(h.shape[0]), int(h.shape[1]),
                           float(sigma2), int(w), float(eps), -1.0 if rho is None else float(rho), boundary)
            rc = lib.deconv_init_batch(ctypes.byref(ctx), ctypes.byref(img), 1, _stream(self.device))
        _check(rc)
        self._ctx = ctx
        self.domain = self._domain(0)

    def _domain(self, b: int):
        M, N, fl = _i(), _i(), _i()
        _check(load_library().deconv_image_domain(self.handle, int(b), ctypes.byref(M), ctypes.byref(N),
                                                  ctypes.byref(fl)))
        return M.value, N.value

    # -- lifetime
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            load_library().deconv_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        if self._ctx is None:
            raise GFDError(-5, "context closed")
        return self._ctx

    # -- iteration
    def iterate(self, n: int, out: torch.Tensor | None = None, lambdas: torch.Tensor | None = None):
        """Run n iterations; returns (u, lambdas) as GPU tensors (allocated if not given)."""
        out = torch.empty((self.M, self.N), device=self.device, dtype=torch.float32) if out is None else out
        lambdas = torch.empty((max(n, 0),), device=self.device, dtype=torch.float32) if lambdas is None else lambdas
        _check(load_library().deconv_iterate(self.handle, int(n), _dev(out, "out", (self.M, self.N)),
                                             _dev(lambdas, "lambdas", (n,)) if n > 0 else None,
                                             _stream(self.device)))
        return out, lambdas

    def set_scales(self, scales):
        s = torch.as_tensor(scales, dtype=torch.float32, device=self.device).contiguous()
        _check(load_library().deconv_set_scales(self.handle, _dev(s, "scales") if s.numel() else None, s.numel(),
                                                _stream(self.device)))
        self._keep_scales = s  # the copy is stream-ordered: keep the source alive

    def set_estimate(self, uE: torch.Tensor):
        _check(load_library().deconv_set_estimate(self.handle, _dev(uE, "uE", (self.M, self.N)), _stream(self.device)))
        self._k_start = self.info()["iterations"]

    def reset(self):
        _check(load_library().deconv_reset(self.handle, _stream(self.device)))
        self._k_start = 0

    TUNING_KEYS = ("gf_strip_rows", "row_pairs_fwd", "rows_inv", "rows_lds", "radix")

    def autotune(self, iters: int = 4) -> dict:
        """Time candidate launch shapes and keep the fastest (needs no iterations run yet;
        single-image contexts only: a batch raises GFDError, give it shapes with set_tuning)."""
        ch = (_i * 5)()
        _check(load_library().deconv_autotune(self.handle, int(iters), ch, _stream(self.device)))
        return dict(zip(self.TUNING_KEYS, list(ch)))

    def set_tuning(self, gf_strip_rows: int = 0, row_pairs_fwd: int = 0, rows_inv: int = 0, rows_lds: int = 0,
                   radix: int = 0):
        """Set the launch shapes autotune would choose, without timing (0 keeps a default)."""
        ch = (_i * 5)(int(gf_strip_rows), int(row_pairs_fwd), int(rows_inv), int(rows_lds), int(radix))
        _check(load_library().deconv_set_tuning(self.handle, ch))

    def set_graph(self, use_graph: bool):
        _check(load_library().deconv_set_graph(self.handle, 1 if use_graph else 0))

    def info(self):
        rho, T, it = _d(), _d(), _i()
        _check(load_library().deconv_info(self.handle, ctypes.byref(rho), ctypes.byref(T), ctypes.byref(it)))
        return {"rho": rho.value, "target": T.value, "iterations": it.value}

    def status(self) -> int:
        f = ctypes.c_uint()
        _check(load_library().deconv_get_status(self.handle, ctypes.byref(f)))
        return f.value

    STAGES = ("row_fwd", "col_fwd_resid", "lambda_sweeps", "col_inv_solve", "row_inv", "guided_filter")

    def profile(self, n: int) -> dict:
        """Run n iterations launching pass by pass; summed device milliseconds per pass."""
        ms = (ctypes.c_float * 6)()
        _check(load_library().deconv_profile(self.handle, int(n), ms, 6, _stream(self.device)))
        return dict(zip(self.STAGES, list(ms)))

    def backward(self, grad_u: torch.Tensor, checkpoint_every: int = 5):
        """Gradient of a loss with respect to eps and to the lambda scales of the iterations run
        since the estimate was last set, given ``grad_u`` = dLoss/du for the current estimate.
        Returns (g_eps, g_scales) as GPU tensors of shapes (count,) and (count, K)."""
        info = self.info()
        K = info["iterations"] - getattr(self, "_k_start", 0)
        count = getattr(self, "count", 1)
        total = getattr(self, "total", self.M * self.N)
        g = grad_u.reshape(-1).contiguous()
        if g.numel() != total:
            raise ValueError(f"grad_u must hold {total} values")
        g_eps = torch.empty((count,), device=self.device, dtype=torch.float32)
        g_s = torch.empty((count, max(K, 0)), device=self.device, dtype=torch.float32)
        _check(load_library().deconv_backward(self.handle, _dev(g, "grad_u"), g_eps.data_ptr(),
                                              g_s.data_ptr() if K > 0 else None, int(checkpoint_every),
                                              _stream(self.device)))
        return g_eps, g_s

    def spectral_solve(self, uE: torch.Tensor, lam: float):
        return spectral_solve(self, uE, lam)

    def discrepancy_lambda(self, uE: torch.Tensor):
        return discrepancy_lambda(self, uE)


class GFDeconvBatch(GFDeconv):
    """Independent problems in one context: every pass of an iteration is one launch for all.

    ``problems`` is a sequence of dicts with keys y, h, sigma2, w, eps and optionally rho, clip
    and pad (the arguments of :class:`GFDeconv`).  Estimates are returned as a list of M_b x N_b views of
    one flat tensor, lambdas as a (count, n) tensor.
    """

    def __init__(self, problems):
        lib = load_library()
        problems = list(problems)
        if not problems:
            raise ValueError("need at least one problem")
        arr = (GfdImage * len(problems))()
        self._keep = []
        self.shapes = []
        for b, pr in enumerate(problems):
            y, h = pr["y"], pr["h"]
            if y.dim() != 2 or h.dim() != 2:
                raise ValueError("y and h must be 2-D")
            M, N = (int(v) for v in y.shape)
            rho = pr.get("rho")
            boundary = (BOUNDARY_CLIP if pr.get("clip") else 0) | (BOUNDARY_PAD if pr.get("pad") else 0)
            arr[b] = GfdImage(_dev(y, f"y[{b}]"), M, N, _dev(h, f"h[{b}]"), int(h.shape[0]), int(h.shape[1]),
                              float(pr["sigma2"]), int(pr["w"]), float(pr["eps"]), -1.0 if rho is None else float(rho),
                              boundary)
            self._keep += [y, h]
            self.shapes.append((M, N))
        self.count = len(problems)
        self.device = problems[0]["y"].device
        self.M, self.N = self.shapes[0]
        self.total = sum(M * N for M, N in self.shapes)
        ctx = _vp()
        _check(lib.deconv_init_batch(ctypes.byref(ctx), ctypes.cast(arr, _vp), self.count, _stream(self.device)))
        self._ctx = ctx
        self.domain = self._domain(0)

    def split(self, flat: torch.Tensor):
        out, off = [], 0
        for M, N in self.shapes:
            out.append(flat[off:off + M * N].view(M, N))
            off += M * N
        return out

    def iterate(self, n: int, out: torch.Tensor | None = None, lambdas: torch.Tensor | None = None):
        """Run n iterations of every problem; returns (list of estimates, (count, n) lambdas)."""
        out = torch.empty((self.total,), device=self.device, dtype=torch.float32) if out is None else out
        lambdas = (torch.empty((self.count, max(n, 0)), device=self.device, dtype=torch.float32)
                   if lambdas is None else lambdas)
        _check(load_library().deconv_iterate(self.handle, int(n), _dev(out, "out", (self.total,)),
                                             _dev(lambdas, "lambdas", (self.count, n)) if n > 0 else None,
                                             _stream(self.device)))
        return self.split(out), lambdas

    def set_estimate(self, estimates):
        flat = torch.cat([u.reshape(-1) for u in estimates]).contiguous()
        _check(load_library().deconv_set_estimate(self.handle, _dev(flat, "estimates", (self.total,)),
                                                  _stream(self.device)))
        torch.cuda.current_stream(self.device).synchronize()
        self._k_start = self.info()["iterations"]

    def image_info(self, b: int):
        M, N, rho, T = _i(), _i(), _d(), _d()
        _check(load_library().deconv_image_info(self.handle, int(b), ctypes.byref(M), ctypes.byref(N),
                                                ctypes.byref(rho), ctypes.byref(T)))
        return {"M": M.value, "N": N.value, "rho": rho.value, "target": T.value}

    def spectral_solve(self, uE, lam):
        raise GFDError(-5, "spectral_solve needs a single-image context")

    def discrepancy_lambda(self, uE):
        raise GFDError(-5, "discrepancy_lambda needs a single-image context")


class GFDeconvFn(torch.autograd.Function):
    """u^K of ``iters`` iterations from u_E = 0, differentiable with respect to eps (a 0-d
    tensor) and the per-iteration lambda scales (a tensor of ``iters`` values) through the
    library's hand-written adjoint (deconv_backward); y, h and the other arguments are
    constants."""

    @staticmethod
    def forward(ctx, eps, scales, y, h, sigma2, w, iters, rho, checkpoint_every):
        g = GFDeconv(y, h, sigma2, w, float(eps), rho)
        try:
            g.set_scales(scales.detach().float())
            u, _ = g.iterate(int(iters))
        except Exception:
            g.close()
            raise
        ctx.g = g
        ctx.checkpoint_every = int(checkpoint_every)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        g = ctx.g
        try:
            g_eps, g_s = g.backward(grad_u.float(), ctx.checkpoint_every)
        finally:
            g.close()
            ctx.g = None
        return g_eps[0], g_s[0], None, None, None, None, None, None, None


def deconvolve_autograd(y, h, sigma2, w, eps, iters, scales=None, rho=None, checkpoint_every=5):
    """Differentiable deconvolution: returns u^K; gradients flow to ``eps`` and ``scales`` when
    they are tensors that require them."""
    dev = y.device
    eps_t = eps if isinstance(eps, torch.Tensor) else torch.tensor(float(eps), device=dev)
    s = scales if scales is not None else torch.ones(int(iters), device=dev)
    return GFDeconvFn.apply(eps_t, s, y, h, float(sigma2), int(w), int(iters), rho, int(checkpoint_every))


def deconvolve(y, h, sigma2, w, eps, iters, rho=None, scales=None):
    """Run ``iters`` iterations from u_E = 0; returns (u, lambdas) as GPU tensors."""
    with GFDeconv(y, h, sigma2, w, eps, rho) as g:
        if scales is not None:
            g.set_scales(scales)
        return g.iterate(iters)


def deconvolve_static(y, h, sigma2, w, eps, iters, rho=None, out=None, lambdas=None):
    """``deconvolve`` without device allocation inside the library (``deconvolve_static`` of the
    C ABI: every buffer in the library's fixed per-device array).  Returns (u, lambdas); pass
    ``out`` and ``lambdas`` to avoid torch allocations as well."""
    M, N = (int(s) for s in y.shape)
    out = torch.empty((M, N), device=y.device, dtype=torch.float32) if out is None else out
    lambdas = torch.empty((max(int(iters), 0),), device=y.device, dtype=torch.float32) if lambdas is None else lambdas
    _check(load_library().deconvolve_static(_dev(y, "y"), M, N, _dev(h, "h"), int(h.shape[0]), int(h.shape[1]),
                                            float(sigma2), int(w), float(eps), -1.0 if rho is None else float(rho),
                                            int(iters), _dev(out, "out", (M, N)),
                                            _dev(lambdas, "lambdas", (int(iters),)) if iters > 0 else None,
                                            _stream(y.device)))
    return out, lambdas


def guided_filter(uI: torch.Tensor, up: torch.Tensor, w: int, eps: float, out: torch.Tensor | None = None,
                  clip: bool = False):
    """u = guidfilter(u_I, u_p, w, eps) (Sec. 2, Eqs.(3)-(5)): periodic windows, or windows
    clipped to the image with count-normalised means when ``clip``."""
    M, N = (int(s) for s in uI.shape)
    out = torch.empty_like(uI) if out is None else out
    fn = load_library().guided_filter_clipped if clip else load_library().guided_filter
    _check(fn(_dev(uI, "uI"), _dev(up, "up", (M, N)), _dev(out, "out", (M, N)), M, N, int(w), float(eps),
              _stream(uI.device)))
    return out


def guided_filter_color(I3: torch.Tensor, up: torch.Tensor, w: int, eps: float, out: torch.Tensor | None = None):
    """Guided filter with a (3, M, N) colour guide: per window (Sigma + eps U)^-1 in place of 1 / (var + eps)."""
    if I3.dim() != 3 or int(I3.shape[0]) != 3:
        raise GFDError(f"I3 must have shape (3, M, N), got {tuple(I3.shape)}")
    M, N = (int(s) for s in I3.shape[1:])
    out = torch.empty_like(up) if out is None else out
    _check(load_library().guided_filter_color(_dev(I3, "I3", (3, M, N)), _dev(up, "up", (M, N)),
                                              _dev(out, "out", (M, N)), M, N, int(w), float(eps), _stream(up.device)))
    return out


def spectral_solve(g: GFDeconv, uE: torch.Tensor, lam: float):
    """(u_I, u_p) from Eqs.(8)-(9) for pre-estimate uE and a given lambda (+inf allowed)."""
    uI = torch.empty(g.domain, device=g.device, dtype=torch.float32)
    up = torch.empty_like(uI)
    _check(load_library().spectral_solve(g.handle, _dev(uE, "uE", g.domain), float(lam), uI.data_ptr(),
                                         up.data_ptr(), _stream(g.device)))
    return uI, up


def discrepancy_lambda(g: GFDeconv, uE: torch.Tensor):
    """lambda_star for pre-estimate uE by the discrepancy principle (Sec. 3.2); 1-element GPU tensor."""
    lam = torch.empty((1,), device=g.device, dtype=torch.float32)
    _check(load_library().discrepancy_lambda(g.handle, _dev(uE, "uE", g.domain), lam.data_ptr(),
                                             _stream(g.device)))
    return lam
