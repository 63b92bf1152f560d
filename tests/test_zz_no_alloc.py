"""love_sample_posterior_noalloc: posterior samples (eq. sample) through the
entry point that allocates nothing.  Its intermediate W_{X*} S and means live
in the library's fixed device scratch array, so its output must equal
love_sample_posterior's bit for bit (same kernels, same order), on two calls
in a row (the second smaller, over the first call's leftovers), at the
largest point count the array holds, while the cache's allocator sees no
request; one point more is refused with LOVE_ELIMIT before any device work."""
import numpy as np
import pytest
import torch

from paper_1803_06058_amd import binding as B
from paper_1803_06058_amd import workloads as WL

from gpu_helpers import cfg_of, tdev, torch_dtype

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 8 << 20     # LOVE_NOALLOC_SCRATCH_BYTES


def max_points(kspad):
    return SCRATCH_BYTES // (4 * (kspad + 1))


@pytest.mark.parametrize("precision,k_sample", [("fp32", 100), ("fp64", 40)])
def test_noalloc_sample_equals_allocating_call(precision, k_sample):
    P = WL.config(2, scale=0.2, k_sample=k_sample, s=8,
                  dtype="f64" if precision == "fp64" else "f32", precision=precision)
    dt = torch_dtype(P)
    kspad = 64 if min(k_sample, P.m[0]) <= 64 else 128
    t1 = max_points(kspad)
    print(P.name, precision, "k_sample", k_sample, "kspad", kspad, "t1", t1, flush=True)
    ta = B.TorchAllocator()
    cache = B.build_cache(cfg_of(P), tdev(P.x, dt), tdev(P.y, dt), allocator=ta)
    _, ks = cache.keff()
    assert 0 < ks <= k_sample
    rng = np.random.default_rng(7)
    xs1 = tdev(rng.uniform(0.0, 1.0, size=(t1, 1)), dt)
    xs2 = tdev(rng.uniform(0.0, 1.0, size=(3001, 1)), dt)
    z1 = tdev(rng.standard_normal((k_sample, 300)), torch.float32)
    z2 = tdev(rng.standard_normal((k_sample, 257)), torch.float32)

    ref1 = cache.sample_posterior(xs1, z1)
    ref2 = cache.sample_posterior(xs2, z2)
    torch.cuda.synchronize()
    allocs_before = ta.allocs
    out1 = torch.full((t1, 300), float("nan"), device=xs1.device, dtype=dt)
    out2 = torch.full((3001, 257), float("nan"), device=xs1.device, dtype=dt)
    cache.sample_posterior_noalloc(xs1, z1, out1)      # fills the array
    cache.sample_posterior_noalloc(xs2, z2, out2)      # smaller, over the leftovers
    torch.cuda.synchronize()
    assert ta.allocs == allocs_before, "the no-allocation call asked the cache's allocator"
    assert torch.isfinite(out1).all() and torch.isfinite(out2).all()
    assert torch.equal(out1, ref1)
    assert torch.equal(out2, ref2)

    # one point beyond the array: refused on the host, output untouched
    xs3 = tdev(rng.uniform(0.0, 1.0, size=(t1 + 1, 1)), dt)
    out3 = torch.zeros((t1 + 1, 4), device=xs1.device, dtype=dt)
    with pytest.raises(B.LoveError) as ei:
        cache.sample_posterior_noalloc(xs3, z1[:, :4].contiguous(), out3)
    assert ei.value.code == -8
    torch.cuda.synchronize()
    assert not out3.any()
    cache.free()
    torch.cuda.synchronize()
    assert ta.live == 0
