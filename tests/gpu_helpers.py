"""Shared helpers of the GPU parity tests: move a seeded workload to the
device, build through the C ABI, and compute the oracle's answer on the
same (rounded) inputs."""
import numpy as np
import torch

from oracle import love_fp64 as O
from paper_1803_06058_amd import binding as B


def dev():
    return torch.device("cuda", 0)


def tdev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def cfg_of(P, **over):
    kw = dict(kernel=P.kernel, lengthscale=list(P.lengthscale), outputscale=P.outputscale,
              noise=P.noise, k=P.k, k_sample=P.k_sample, precision=P.precision)
    kw.update(over)
    if P.additive:
        kw["flags"] = kw.get("flags", 0) | B.FLAG_ADDITIVE
    return B.config_struct(P.d, list(P.m), list(P.lo), list(P.hi), **kw)


def torch_dtype(P):
    return torch.float64 if P.precision == "fp64" else torch.float32


def build(P, **over):
    dt = torch_dtype(P)
    x = tdev(P.x, dt)
    y = tdev(P.y, dt)
    cache = B.build_cache(cfg_of(P, **over), x, y)
    return cache


def spec_of(P):
    return O.Spec(P.m, P.lo, P.hi, P.kernel, P.lengthscale, P.outputscale, P.noise, P.additive)


def oracle_cache(P, k=None, cg_tol=1e-10):
    return O.love_build(P.x.astype(np.float64), P.y.astype(np.float64), spec_of(P),
                        P.k if k is None else k, cg_tol=cg_tol, cg_maxit=5000)


def errors(var_gpu, var_ref, prior, mean_gpu=None, mean_ref=None, y=None):
    dv = np.abs(np.asarray(var_gpu, np.float64) - var_ref)
    out = {
        "e_p_max": float(np.max(dv / prior)),
        "e_v_max": float(np.max(dv / np.abs(var_ref))),
        "e_v_median": float(np.median(dv / np.abs(var_ref))),
    }
    if mean_gpu is not None:
        rms = float(np.sqrt(np.mean(np.asarray(y, np.float64) ** 2)))
        out["mean_err_rel_rms_y"] = float(np.max(np.abs(np.asarray(mean_gpu, np.float64) - mean_ref)) / rms)
    return out
