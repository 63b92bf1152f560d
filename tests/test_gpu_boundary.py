"""The C ABI's memory and backend contracts on the GPU: builds, imports and
covariance blocks through a caller-supplied love_allocator (torch's caching
allocator) equal the library-pool results bit for bit and return every block
they took; an explicit FFT request the LDS-resident FFT cannot meet is
refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1803_06058_amd import binding as B
from paper_1803_06058_amd import workloads as WL

from gpu_helpers import cfg_of, tdev, torch_dtype

pytestmark = pytest.mark.gpu


def _build(P, allocator, **over):
    dt = torch_dtype(P)
    return B.build_cache(cfg_of(P, **over), tdev(P.x, dt), tdev(P.y, dt), allocator=allocator)


def _contents(cache, xs):
    ex = cache.export()
    _, var = cache.predict_mean_var(xs)
    torch.cuda.synchronize()
    return {k: v.cpu() for k, v in ex.items()} | {"var": var.cpu()}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_build_through_torch_allocator(precision):
    P = WL.config(2, scale=0.05, s=16, dtype="f64" if precision == "fp64" else "f32",
                  precision=precision)
    print(P.name, P.n, P.m, precision, flush=True)
    dt = torch_dtype(P)
    xs = tdev(P.xs[:4000], dt)
    ref_cache = _build(P, None)
    ref = _contents(ref_cache, xs)
    ref_cache.free()
    torch.cuda.synchronize()
    ta = B.TorchAllocator()
    base = torch.cuda.memory_allocated()
    c = _build(P, ta)
    held = torch.cuda.memory_allocated() - base
    got = _contents(c, xs)
    print("allocator calls", ta.allocs, ta.frees, ta.live, "held", held, flush=True)
    assert ta.allocs > 0 and ta.live >= 1 and held > 0
    for k in ref:
        assert torch.equal(ref[k], got[k]), k
    # the query-side calls on this cache take their scratch from it too
    c.sample_posterior(tdev(P.xs_sample[:100], dt), tdev(P.z, torch.float32))
    c.predict_covar_block(xs[:50], xs[50:90])
    torch.cuda.synchronize()
    c.free()
    torch.cuda.synchronize()
    assert ta.live == 0 and ta.allocs == ta.frees
    assert torch.cuda.memory_allocated() == base


def test_batched_import_and_covar_block_through_allocator():
    Ps = WL.batched_config(G=3, scale=0.05, t_per_gp=2000)
    cfgs = [cfg_of(P) for P in Ps]
    xs = [tdev(P.x, torch.float32) for P in Ps]
    ys = [tdev(P.y, torch.float32) for P in Ps]
    ta = B.TorchAllocator()
    base = torch.cuda.memory_allocated()
    a = B.build_cache_batched(cfgs, xs, ys, allocator=None)
    b = B.build_cache_batched(cfgs, xs, ys, allocator=ta)
    for ca, cb, P in zip(a, b, Ps):
        q = tdev(P.xs[:1000], torch.float32)
        assert torch.equal(ca.predict_mean_var(q)[1], cb.predict_mean_var(q)[1])
        # import through the allocator; the covariance block with an explicit allocator
        imp = B.import_cache(cfg_of(P), cb.export(), allocator=ta)
        blk_ref = ca.predict_covar_block(q[:40], q[40:70], allocator=None)
        blk = imp.predict_covar_block(q[:40], q[40:70], allocator=ta)
        assert torch.equal(blk_ref, blk)
        imp.free()
    # the loop's last query and output tensors are torch's, not the library's
    del q, blk_ref, blk
    for c in a + b:
        c.free()
    torch.cuda.synchronize()
    print("allocator calls", ta.allocs, ta.frees, ta.live, flush=True)
    assert ta.live == 0 and ta.allocs == ta.frees > 0
    assert torch.cuda.memory_allocated() == base


def test_failing_allocator_reports_enomem():
    """An allocator that refuses every request makes the build return
    LOVE_ENOMEM (no cache, nothing left behind)."""
    P = WL.config(2, scale=0.02, k_sample=0)
    refuse = B.love_allocator(B.ALLOC_FN(lambda n, s, ctx: None),
                              B.FREE_FN(lambda p, s, ctx: None), None)

    class Refuse:
        def ref(self):
            import ctypes
            return ctypes.byref(refuse)

    with pytest.raises(B.LoveError) as ei:
        _build(P, Refuse())
    assert ei.value.code == -4


def test_explicit_fft_beyond_lds_refused():
    """m = 5000 needs a circulant of 16384 points, beyond the LDS-resident
    FFT: an explicit FFT request is refused (LOVE_EUNSUPPORTED), the automatic
    choice takes the direct product."""
    P = WL.config(2, scale=0.5, k_sample=0)          # m = 5000
    assert P.m[0] == 5000
    with pytest.raises(B.LoveError) as ei:
        _build(P, None, toeplitz="fft", k=4, flags=B.FLAG_NO_MEAN)
    assert ei.value.code == -7
    c = _build(P, None, toeplitz="auto", k=4, flags=B.FLAG_NO_MEAN)
    assert c.info().toeplitz_mode[0] == 1
    c.free()


class _RefuseNth:
    """A love_allocator over torch's caching allocator that refuses its n-th
    request (n = 0: none) and counts the blocks it has handed out and not had
    back."""

    def __init__(self, n):
        self.n, self.calls, self.live = n, 0, 0

        def _alloc(nbytes, stream, ctx):
            self.calls += 1
            if self.calls == self.n:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            self.live += 1
            return p

        def _free(ptr, stream, ctx):
            self.live -= 1
            torch.cuda.caching_allocator_delete(int(ptr))

        self._a, self._f = B.ALLOC_FN(_alloc), B.FREE_FN(_free)
        self.struct = B.love_allocator(self._a, self._f, None)

    def ref(self):
        return C.byref(self.struct)


@pytest.mark.parametrize("batched", [False, True])
def test_refused_allocation_returns_enomem_and_releases_every_block(batched):
    """Each device allocation of a build refused in turn (a single build, and a
    batch of two GPs whose samplers run on the side stream): the build returns
    ENOMEM, every block handed out comes back once the stream is done, and a
    build afterwards gives the same variances as before."""
    P = WL.config(2, scale=0.05, s=16)
    dt = torch_dtype(P)
    x, y = tdev(P.x, dt), tdev(P.y, dt)
    xs = tdev(P.xs[:2000], dt)

    def run(alloc):
        if batched:
            return B.build_cache_batched([cfg_of(P)] * 2, [x, x], [y, y], allocator=alloc)
        return [B.build_cache(cfg_of(P), x, y, allocator=alloc)]

    def variances(cs):
        out = [c.predict_mean_var(xs)[1].cpu() for c in cs]
        for c in cs:
            c.free()
        torch.cuda.synchronize()
        return out

    ref = variances(run(None))
    count = _RefuseNth(0)
    variances(run(count))
    n = count.calls
    print("allocations per build", n, flush=True)
    assert n >= 2 and count.live == 0
    for k in range(1, n + 1):
        a = _RefuseNth(k)
        with pytest.raises(B.LoveError) as ei:
            run(a)
        torch.cuda.synchronize()
        assert ei.value.code == -4, (k, ei.value.code)
        assert a.live == 0, (k, a.live)
    for u, v in zip(variances(run(_RefuseNth(0))), ref):
        assert torch.equal(u, v)


def test_refused_query_workspace_returns_enomem_and_keeps_the_cache():
    """The query calls that take workspace from the cache's allocator (samples,
    covariance block, backward with d var / d Rt, hyper-parameter gradient),
    each with its first workspace request refused: ENOMEM, every block handed
    out for the call comes back, and the same call afterwards gives the
    answer of an unrefused call."""
    P = WL.config(2, scale=0.05, s=16)
    dt = torch_dtype(P)
    a = _RefuseNth(0)
    c = B.build_cache(cfg_of(P, flags=B.FLAG_HYPER), tdev(P.x, dt), tdev(P.y, dt), allocator=a)
    xs = tdev(P.xs[:500], dt)
    g = torch.ones(500, device=xs.device, dtype=dt)
    calls = {
        "sample": lambda: c.sample_posterior(tdev(P.xs_sample[:100], dt), tdev(P.z, torch.float32)),
        "covar_block": lambda: c.predict_covar_block(xs[:40], xs[40:70]),
        "backward_grt": lambda: c.predict_backward(xs, g, g, want_grt=True)[1],
        "hyper_grad": lambda: c.predict_var_hyper_grad(xs, g),
    }
    for name, f in calls.items():
        ref = f().clone()
        torch.cuda.synchronize()
        held = a.live
        a.n = a.calls + 1
        with pytest.raises(B.LoveError) as ei:
            f()
        torch.cuda.synchronize()
        print(name, "code", ei.value.code, "live", a.live, "held", held, flush=True)
        assert ei.value.code == -4, name
        assert a.live == held, name
        assert torch.equal(f(), ref), name
    c.free()
    torch.cuda.synchronize()
    assert a.live == 0
