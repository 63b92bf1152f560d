"""ctypes binding of the LOVE C ABI (include/love.h).

Argument marshalling only: tensors must already live on the GPU; their data
pointers and the current HIP stream are handed to the native library.
"""
from __future__ import annotations

import ctypes as C
import math
import sys
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16split": 2}
KERNELS = {"rbf": 0, "matern52": 1}
TOEPLITZ_MODES = {"auto": 0, "direct": 1, "fft": 2}
FLAG_ASYNC, FLAG_NO_MEAN, FLAG_PLAIN_CG, FLAG_EIG_QL, FLAG_MEAN_KRYLOV = 1, 2, 4, 8, 16
FLAG_ADDITIVE = 32   # additive composition: grid vectors stack the axes, m = sum of m_i
FLAG_HYPER = 64      # keep B = W^T Q L^{-T} for the hyper-parameter gradient

STATUS = {0: "ok", -1: "EINVAL", -2: "EDOMAIN", -3: "ENOTPD", -4: "ENOMEM", -5: "EHIP",
          -6: "ENONFINITE", -7: "EUNSUPPORTED", -8: "ELIMIT"}


class LoveError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)} ({code})")
        self.code = code


class love_config(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("m", C.c_int32 * 4), ("lo", C.c_double * 4), ("hi", C.c_double * 4),
        ("kernel", C.c_int32), ("lengthscale", C.c_double * 4), ("outputscale", C.c_double),
        ("noise", C.c_double), ("k", C.c_int32), ("k_sample", C.c_int32),
        ("precision", C.c_int32), ("toeplitz", C.c_int32), ("cg_tol", C.c_double),
        ("cg_maxit", C.c_int32), ("flags", C.c_uint32), ("restart_tol", C.c_double),
        ("restart_k", C.c_int32), ("restart_max", C.c_int32), ("restart_groups", C.c_int32),
    ]


class love_cache_info_t(C.Structure):
    _fields_ = [
        ("k_eff", C.c_int32), ("k_eff_sample", C.c_int32), ("cg_iters", C.c_int32),
        ("d", C.c_int32), ("n", C.c_int64), ("m", C.c_int64), ("beta_last", C.c_double),
        ("ortho_loss", C.c_double), ("status_flags", C.c_uint32), ("toeplitz_mode", C.c_uint32 * 4),
        ("fft_len", C.c_uint32 * 4), ("bytes", C.c_size_t), ("restarts", C.c_int32),
        ("solve_residual", C.c_double),
    ]


class love_export(C.Structure):
    _fields_ = [("alpha", C.c_void_p), ("beta", C.c_void_p), ("rt", C.c_void_p),
                ("rt64", C.c_void_p), ("a", C.c_void_p), ("s", C.c_void_p)]


class love_import(C.Structure):
    _fields_ = [("k_eff", C.c_int32), ("k_eff_sample", C.c_int32), ("alpha", C.c_void_p),
                ("beta", C.c_void_p), ("rt", C.c_void_p), ("rt64", C.c_void_p),
                ("a", C.c_void_p), ("s", C.c_void_p)]


# love_allocator: device memory callbacks (alloc(bytes, stream, ctx), free(ptr, stream, ctx), ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class love_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class TorchAllocator:
    """A love_allocator over torch's caching allocator: blocks come from
    torch.cuda.caching_allocator_alloc on the stream the library names and go
    back through caching_allocator_delete (stream-ordered reuse on that stream,
    which is what the library's release order assumes).  Counts the calls."""

    def __init__(self):
        self.allocs = 0
        self.frees = 0
        self.live = 0

        def _alloc(nbytes, stream, ctx):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            except Exception:
                return None
            self.allocs += 1
            self.live += 1
            return p

        def _free(ptr, stream, ctx):
            self.frees += 1
            self.live -= 1
            torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = love_allocator(self._alloc, self._free, None)

    def ref(self):
        return C.byref(self.struct)


_TORCH_ALLOC: Optional[TorchAllocator] = None


def torch_allocator() -> TorchAllocator:
    """The process-wide TorchAllocator (kept alive as long as any cache may use it)."""
    global _TORCH_ALLOC
    if _TORCH_ALLOC is None:
        _TORCH_ALLOC = TorchAllocator()
    return _TORCH_ALLOC


def _alloc_arg(allocator):
    """allocator argument of the entry points: "torch" (the process-wide
    TorchAllocator), None (the library's own stream-ordered pool) or a
    TorchAllocator instance."""
    if allocator is None:
        return None, None
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError("allocator must be 'torch', None or a TorchAllocator")
        allocator = torch_allocator()
    return allocator.ref(), allocator


SYMBOLS = [
    "love_abi_version", "love_status_string", "love_build_cache", "love_build_cache_batched",
    "love_predict_mean_var", "love_predict_mean_var_batched", "love_predict_covar_pairs",
    "love_predict_covar_block",
    "love_sample_posterior", "love_sample_posterior_noalloc", "love_predict_backward",
    "love_predict_var_hyper_grad", "love_apply_khat", "love_apply_kuu",
    "love_cache_info", "love_cache_keff", "love_cache_export", "love_cache_import", "love_cache_free",
    "love_profile_enable",
    "love_profile_read", "love_profile_select",
]

_lib = None


def lib_path() -> str:
    return os.path.join(_HERE, "_lib", "liblove.so")


def load_library():
    """Load liblove.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = lib_path()
    if not os.path.exists(p):
        raise RuntimeError(f"native LOVE library not built: {p} (run python -m paper_1803_06058_amd.build)")
    L = C.CDLL(p)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.love_abi_version.restype = i32
    L.love_status_string.restype = C.c_char_p
    L.love_status_string.argtypes = [i32]
    L.love_build_cache.restype = i32
    AP = C.POINTER(love_allocator)
    L.love_build_cache.argtypes = [C.POINTER(love_config), vp, vp, i64, AP, vp, C.POINTER(vp)]
    L.love_build_cache_batched.restype = i32
    L.love_build_cache_batched.argtypes = [i32, C.POINTER(love_config), C.POINTER(vp),
                                           C.POINTER(vp), C.POINTER(i64), AP, vp, C.POINTER(vp)]
    L.love_predict_mean_var.restype = i32
    L.love_predict_mean_var.argtypes = [vp, vp, i64, vp, vp, vp]
    L.love_predict_mean_var_batched.restype = i32
    L.love_predict_mean_var_batched.argtypes = [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(i64),
                                                C.POINTER(vp), C.POINTER(vp), vp]
    L.love_predict_covar_pairs.restype = i32
    L.love_predict_covar_pairs.argtypes = [vp, vp, vp, i64, vp, vp]
    L.love_predict_covar_block.restype = i32
    L.love_predict_covar_block.argtypes = [vp, vp, i64, vp, i64, vp, AP, vp]
    L.love_sample_posterior.restype = i32
    L.love_sample_posterior.argtypes = [vp, vp, i64, vp, i64, vp, vp]
    L.love_sample_posterior_noalloc.restype = i32
    L.love_sample_posterior_noalloc.argtypes = [vp, vp, i64, vp, i64, vp, vp]
    L.love_predict_backward.restype = i32
    L.love_predict_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    L.love_predict_var_hyper_grad.restype = i32
    L.love_predict_var_hyper_grad.argtypes = [vp, vp, i64, vp, vp, vp]
    L.love_apply_khat.restype = i32
    L.love_apply_khat.argtypes = [vp, vp, vp, vp]
    L.love_apply_kuu.restype = i32
    L.love_apply_kuu.argtypes = [vp, vp, vp, vp]
    L.love_cache_info.restype = i32
    L.love_cache_info.argtypes = [vp, C.POINTER(love_cache_info_t)]
    L.love_cache_keff.restype = i32
    L.love_cache_keff.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.love_cache_export.restype = i32
    L.love_cache_export.argtypes = [vp, C.POINTER(love_export), vp]
    L.love_cache_import.restype = i32
    L.love_cache_import.argtypes = [C.POINTER(love_config), C.POINTER(love_import), AP, vp,
                                    C.POINTER(vp)]
    L.love_cache_free.restype = None
    L.love_cache_free.argtypes = [vp]
    L.love_profile_enable.restype = i32
    L.love_profile_enable.argtypes = [i32]
    L.love_profile_select.restype = i32
    L.love_profile_select.argtypes = [C.c_char_p]
    L.love_profile_read.restype = i32
    L.love_profile_read.argtypes = [C.c_char_p, C.POINTER(i64), C.POINTER(C.c_double)]
    _lib = L
    return L


def _check(code: int, what: str):
    if code != 0:
        raise LoveError(code, what)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def config_struct(d: int, m: Sequence[int], lo: Sequence[float], hi: Sequence[float],
                  kernel: str = "rbf", lengthscale: Sequence[float] = (0.1,),
                  outputscale: float = 1.0, noise: float = 0.01, k: int = 50,
                  k_sample: int = 0, precision: str = "fp32", toeplitz: str = "auto",
                  cg_tol: float = 0.0, cg_maxit: int = 0, flags: int = 0,
                  restart_tol: float = 0.0, restart_k: int = 0, restart_max: int = 0,
                  restart_groups: int = 0) -> love_config:
    c = love_config()
    c.d = d
    for e in range(d):
        c.m[e] = int(m[e])
        c.lo[e] = float(lo[e])
        c.hi[e] = float(hi[e])
        c.lengthscale[e] = float(lengthscale[e] if len(lengthscale) > e else lengthscale[0])
    c.kernel = KERNELS[kernel]
    c.outputscale = outputscale
    c.noise = noise
    c.k = k
    c.k_sample = k_sample
    c.precision = PRECISIONS[precision]
    c.toeplitz = TOEPLITZ_MODES[toeplitz]
    c.cg_tol = cg_tol
    c.cg_maxit = cg_maxit
    c.flags = flags
    c.restart_tol = restart_tol
    c.restart_k = restart_k
    c.restart_max = restart_max
    c.restart_groups = restart_groups
    return c


def _dtype(precision: int):
    return torch.float64 if precision == 0 else torch.float32


def _need(t: torch.Tensor, dtype, shape, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class LoveCache:
    """A built LOVE cache (owned by the native library)."""

    def __init__(self, handle: int, cfg: love_config, allocator=None):
        self._h = C.c_void_p(handle)
        self._allocator = allocator   # keeps the callbacks alive while the cache lives
        self.cfg = cfg
        self.d = cfg.d
        self.dtype = _dtype(cfg.precision)
        sizes = [int(cfg.m[e]) for e in range(cfg.d)]
        self.m = sum(sizes) if cfg.flags & FLAG_ADDITIVE else math.prod(sizes)

    # -- lifetime --------------------------------------------------------
    def free(self):
        if self._h is not None and self._h.value:
            load_library().love_cache_free(self._h)
        self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():   # torch may be gone: leave the memory to process exit
            return
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- queries ---------------------------------------------------------
    def _xs(self, xs: torch.Tensor, name="xs") -> int:
        if xs.dim() == 1 and self.d == 1:
            xs = xs.view(-1, 1)
        _need(xs, self.dtype, None, name)
        if xs.dim() != 2 or xs.shape[1] != self.d:
            raise ValueError(f"{name} must be t x {self.d}")
        return xs.shape[0]

    def predict_mean_var(self, xs: torch.Tensor, mean: bool = True, out=None):
        t = self._xs(xs)
        if out is None:
            mu = torch.empty(t, device=xs.device, dtype=self.dtype) if mean else None
            var = torch.empty(t, device=xs.device, dtype=self.dtype)
        else:
            mu, var = out
        _check(load_library().love_predict_mean_var(self._h, _ptr(xs), t, _ptr(mu), _ptr(var),
                                                    C.c_void_p(_stream())), "predict_mean_var")
        return mu, var

    def predict_covar_pairs(self, xa: torch.Tensor, xb: torch.Tensor):
        t = self._xs(xa, "xa")
        if self._xs(xb, "xb") != t:
            raise ValueError("xa and xb must have the same number of points")
        cov = torch.empty(t, device=xa.device, dtype=self.dtype)
        _check(load_library().love_predict_covar_pairs(self._h, _ptr(xa), _ptr(xb), t, _ptr(cov),
                                                       C.c_void_p(_stream())), "predict_covar_pairs")
        return cov

    def predict_covar_block(self, xa: torch.Tensor, xb: torch.Tensor, allocator="cache"):
        """cov[i, j] = k(xa_i, xb_j) for every pair (ta x tb).  allocator: "cache"
        (the cache's own memory source), "torch", None (library pool) or a
        TorchAllocator."""
        ta = self._xs(xa, "xa")
        tb = self._xs(xb, "xb")
        cov = torch.empty(ta, tb, device=xa.device, dtype=self.dtype)
        aref, _ = (None, None) if allocator == "cache" else _alloc_arg(allocator)
        _check(load_library().love_predict_covar_block(self._h, _ptr(xa), ta, _ptr(xb), tb,
                                                       _ptr(cov), aref, C.c_void_p(_stream())),
               "predict_covar_block")
        return cov

    def keff(self):
        """(k_eff, k_eff_sample); no device synchronisation after a synchronous build."""
        k = C.c_int32()
        ks = C.c_int32()
        _check(load_library().love_cache_keff(self._h, C.byref(k), C.byref(ks)), "cache_keff")
        return k.value, ks.value

    def sample_posterior(self, xs: torch.Tensor, z: torch.Tensor, out=None):
        t = self._xs(xs)
        _need(z, torch.float32, None, "z")
        if z.dim() != 2:
            raise ValueError("z must be k_sample x s")
        if z.shape[0] < self.keff()[1]:
            raise ValueError("z needs at least k_eff_sample rows")
        s = z.shape[1]
        if out is None:
            out = torch.empty(t, s, device=xs.device, dtype=self.dtype)
        _check(load_library().love_sample_posterior(self._h, _ptr(xs), t, _ptr(z), s, _ptr(out),
                                                    C.c_void_p(_stream())), "sample_posterior")
        return out

    def sample_posterior_noalloc(self, xs: torch.Tensor, z: torch.Tensor, out: torch.Tensor):
        """love_sample_posterior_noalloc: the library allocates nothing; the
        caller passes the t x s output."""
        t = self._xs(xs)
        _need(z, torch.float32, None, "z")
        if z.dim() != 2:
            raise ValueError("z must be k_sample x s")
        if z.shape[0] < self.keff()[1]:
            raise ValueError("z needs at least k_eff_sample rows")
        s = z.shape[1]
        _need(out, self.dtype, (t, s), "out")
        _check(load_library().love_sample_posterior_noalloc(
            self._h, _ptr(xs), t, _ptr(z), s, _ptr(out), C.c_void_p(_stream())),
            "sample_posterior_noalloc")
        return out

    def predict_backward(self, xs: torch.Tensor, g_mean: Optional[torch.Tensor],
                         g_var: Optional[torch.Tensor], want_grt: bool = False):
        t = self._xs(xs)
        for g, nm in ((g_mean, "g_mean"), (g_var, "g_var")):
            if g is not None:
                _need(g, self.dtype, (t,), nm)
        gx = torch.empty(t, self.d, device=xs.device, dtype=self.dtype)
        grt = None
        if want_grt:
            grt = torch.zeros(self.m, self.keff()[0], device=xs.device, dtype=torch.float32)
        _check(load_library().love_predict_backward(self._h, _ptr(xs), t, _ptr(g_mean), _ptr(g_var),
                                                    _ptr(gx), _ptr(grt), C.c_void_p(_stream())),
               "predict_backward")
        return gx, grt

    def predict_var_hyper_grad(self, xs: torch.Tensor, g_var: torch.Tensor) -> torch.Tensor:
        """d(sum g_var * var)/d theta, theta = (lengthscales, outputscale, noise):
        a (d + 2,) float64 tensor (the cache needs FLAG_HYPER)."""
        t = self._xs(xs)
        _need(g_var, self.dtype, (t,), "g_var")
        out = torch.empty(self.d + 2, device=xs.device, dtype=torch.float64)
        _check(load_library().love_predict_var_hyper_grad(self._h, _ptr(xs), t, _ptr(g_var),
                                                          _ptr(out), C.c_void_p(_stream())),
               "predict_var_hyper_grad")
        return out

    def apply_khat(self, v: torch.Tensor):
        out = torch.empty_like(v)
        _need(v, self.dtype, None, "v")
        _check(load_library().love_apply_khat(self._h, _ptr(v), _ptr(out), C.c_void_p(_stream())),
               "apply_khat")
        return out

    def apply_kuu(self, g: torch.Tensor):
        _need(g, self.dtype, None, "g")
        out = torch.empty_like(g)
        _check(load_library().love_apply_kuu(self._h, _ptr(g), _ptr(out), C.c_void_p(_stream())),
               "apply_kuu")
        return out

    def info(self) -> love_cache_info_t:
        inf = love_cache_info_t()
        _check(load_library().love_cache_info(self._h, C.byref(inf)), "cache_info")
        return inf

    def export(self) -> Dict[str, torch.Tensor]:
        inf = self.info()
        dev = torch.device("cuda", torch.cuda.current_device())
        k, m = inf.k_eff, inf.m
        out = {
            "alpha": torch.empty(k, device=dev, dtype=torch.float64),
            "beta": torch.empty(k, device=dev, dtype=torch.float64),
            "rt": torch.empty(m, k, device=dev, dtype=torch.float32),
            "a": torch.empty(m, device=dev, dtype=self.dtype),
        }
        if self.cfg.precision == 0:
            out["rt64"] = torch.empty(m, k, device=dev, dtype=torch.float64)
        if inf.k_eff_sample > 0:
            out["s"] = torch.empty(m, inf.k_eff_sample, device=dev, dtype=torch.float32)
        e = love_export(_ptr(out["alpha"]), _ptr(out["beta"]), _ptr(out["rt"]),
                        _ptr(out.get("rt64")), _ptr(out["a"]), _ptr(out.get("s")))
        _check(load_library().love_cache_export(self._h, C.byref(e), C.c_void_p(_stream())), "export")
        torch.cuda.current_stream().synchronize()
        return out


def build_cache(cfg: love_config, x: torch.Tensor, y: torch.Tensor,
                allocator="torch") -> LoveCache:
    """love_build_cache on device tensors x (n x d) and y (n).  allocator:
    "torch" (torch's caching allocator backs the cache and its workspace),
    None (the library's stream-ordered pool) or a TorchAllocator."""
    L = load_library()
    aref, aobj = _alloc_arg(allocator)
    dt = _dtype(cfg.precision)
    n = x.shape[0]
    if x.dim() == 1 and cfg.d == 1:
        x = x.view(-1, 1)
    _need(x, dt, (n, cfg.d), "x")
    _need(y, dt, (n,), "y")
    h = C.c_void_p()
    _check(L.love_build_cache(C.byref(cfg), _ptr(x), _ptr(y), n, aref, C.c_void_p(_stream()),
                              C.byref(h)), "build_cache")
    return LoveCache(h.value, cfg, aobj)


def import_cache(cfg: love_config, parts: Dict[str, torch.Tensor], allocator="torch") -> LoveCache:
    """love_cache_import from the dict LoveCache.export() returns (device
    tensors: rt (m x k_eff float) or rt64, a, optional alpha, beta, s)."""
    L = load_library()
    rt = parts.get("rt64") if cfg.precision == 0 else parts.get("rt")
    if rt is None or rt.dim() != 2:
        raise ValueError("parts needs rt (rt64 for FP64) as an m x k_eff tensor")
    s = parts.get("s")
    im = love_import(int(rt.shape[1]), int(s.shape[1]) if s is not None else 0,
                     _ptr(parts.get("alpha")), _ptr(parts.get("beta")),
                     _ptr(parts.get("rt")) if cfg.precision != 0 else None,
                     _ptr(parts.get("rt64")) if cfg.precision == 0 else None,
                     _ptr(parts.get("a")), _ptr(s))
    h = C.c_void_p()
    aref, aobj = _alloc_arg(allocator)
    _check(L.love_cache_import(C.byref(cfg), C.byref(im), aref, C.c_void_p(_stream()), C.byref(h)),
           "cache_import")
    return LoveCache(h.value, cfg, aobj)


def build_cache_batched(cfgs: List[love_config], xs: List[torch.Tensor],
                        ys: List[torch.Tensor], allocator="torch") -> List[LoveCache]:
    L = load_library()
    aref, aobj = _alloc_arg(allocator)
    G = len(cfgs)
    arr = (love_config * G)(*cfgs)
    xp = (C.c_void_p * G)(*[x.data_ptr() for x in xs])
    yp = (C.c_void_p * G)(*[y.data_ptr() for y in ys])
    ns = (C.c_int64 * G)(*[x.shape[0] for x in xs])
    for g in range(G):
        dt = _dtype(cfgs[g].precision)
        _need(xs[g], dt, (xs[g].shape[0], cfgs[g].d), f"xs[{g}]")
        _need(ys[g], dt, (xs[g].shape[0],), f"ys[{g}]")
    out = (C.c_void_p * G)()
    _check(L.love_build_cache_batched(G, arr, xp, yp, ns, aref, C.c_void_p(_stream()), out),
           "build_cache_batched")
    return [LoveCache(out[g], cfgs[g], aobj) for g in range(G)]


def predict_mean_var_batched(caches: List[LoveCache], xs: List[torch.Tensor], outs=None):
    """Mean and variance for G caches in one launch; outs: optional list of
    (mean, var) tensors to write into."""
    L = load_library()
    G = len(caches)
    hs = (C.c_void_p * G)(*[c.handle.value for c in caches])
    for c, x in zip(caches, xs):
        _need(x, c.dtype, (x.shape[0], c.cfg.d), "xs")
    xp = (C.c_void_p * G)(*[x.data_ptr() for x in xs])
    ts = (C.c_int64 * G)(*[x.shape[0] for x in xs])
    if outs is None:
        means = [torch.empty(x.shape[0], device=x.device, dtype=c.dtype) for c, x in zip(caches, xs)]
        vars_ = [torch.empty(x.shape[0], device=x.device, dtype=c.dtype) for c, x in zip(caches, xs)]
    else:
        means = [o[0] for o in outs]
        vars_ = [o[1] for o in outs]
        for c, x, m, v in zip(caches, xs, means, vars_):
            _need(m, c.dtype, (x.shape[0],), "mean")
            _need(v, c.dtype, (x.shape[0],), "var")
    mp = (C.c_void_p * G)(*[m.data_ptr() for m in means])
    vp = (C.c_void_p * G)(*[v.data_ptr() for v in vars_])
    _check(L.love_predict_mean_var_batched(G, hs, xp, ts, mp, vp, C.c_void_p(_stream())),
           "predict_mean_var_batched")
    return means, vars_


def profile_enable(on: bool):
    _check(load_library().love_profile_enable(1 if on else 0), "profile_enable")


def profile_select(names: Optional[Sequence[str]]):
    arg = None if not names else ",".join(names).encode()
    _check(load_library().love_profile_select(arg), "profile_select")


def profile_read(names: Sequence[str]) -> Dict[str, Tuple[int, float]]:
    n = len(names)
    calls = (C.c_int64 * n)()
    ms = (C.c_double * n)()
    _check(load_library().love_profile_read(",".join(names).encode(), calls, ms), "profile_read")
    return {names[i]: (int(calls[i]), float(ms[i])) for i in range(n)}


class LovePredict(torch.autograd.Function):
    """Differentiable predictive mean and variance with respect to x*.

    forward(xs, cache) -> (mean, var); backward runs love_predict_backward."""

    @staticmethod
    def forward(ctx, xs: torch.Tensor, cache: LoveCache):
        mu, var = cache.predict_mean_var(xs.detach().contiguous())
        ctx.cache = cache
        ctx.save_for_backward(xs)
        return mu, var

    @staticmethod
    def backward(ctx, g_mean, g_var):
        (xs,) = ctx.saved_tensors
        cache = ctx.cache
        gm = None if g_mean is None else g_mean.contiguous()
        gv = None if g_var is None else g_var.contiguous()
        gx, _ = cache.predict_backward(xs.detach().contiguous(), gm, gv)
        return gx.view_as(xs), None
