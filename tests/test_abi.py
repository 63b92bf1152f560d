"""The C-ABI library builds, loads, exports every declared symbol, its struct
layouts match the binding, and host-side argument validation rejects bad
calls before any device work (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "love.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1803_06058_amd import binding
    if not os.path.exists(binding.lib_path()):
        from paper_1803_06058_amd import build
        build.build()
    return binding.load_library()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(love_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(lib, nm), nm
    from paper_1803_06058_amd import binding
    assert sorted(binding.SYMBOLS) == names


def test_abi_version_and_status_strings(lib):
    assert lib.love_abi_version() == 4
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert lib.love_status_string(code)
    assert lib.love_status_string(12345) == b"unknown status"


def test_struct_layout_matches_c(lib):
    from paper_1803_06058_amd import binding as B
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "love.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(love_config),
         offsetof(love_config, flags), offsetof(love_config, cg_tol), sizeof(love_cache_info_t),
         offsetof(love_cache_info_t, bytes), sizeof(love_export), sizeof(love_import),
         offsetof(love_import, s), sizeof(love_allocator), offsetof(love_allocator, free),
         offsetof(love_allocator, ctx));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "t.c")
        open(cpath, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), cpath, "-o", exe],
                       check=True)
        got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                              check=True).stdout.split()]
    want = [C.sizeof(B.love_config), B.love_config.flags.offset, B.love_config.cg_tol.offset,
            C.sizeof(B.love_cache_info_t), B.love_cache_info_t.bytes.offset, C.sizeof(B.love_export),
            C.sizeof(B.love_import), B.love_import.s.offset, C.sizeof(B.love_allocator),
            B.love_allocator.free.offset, B.love_allocator.ctx.offset]
    assert got == want


def test_import_validation_rejects_bad_arguments(lib):
    from paper_1803_06058_amd import binding as B
    out = C.c_void_p()
    cfg = B.config_struct(1, [100], [0.0], [1.0], lengthscale=[0.1], k=10)
    im = B.love_import(10, 0, None, None, C.c_void_p(256), None, None, None)
    assert lib.love_cache_import(None, C.byref(im), None, None, C.byref(out)) == -1
    assert lib.love_cache_import(C.byref(cfg), None, None, None, C.byref(out)) == -1
    for keff, ks in ((0, 0), (129, 0), (10, -1), (10, 129)):
        bad = B.love_import(keff, ks, None, None, C.c_void_p(256), None, None, None)
        assert lib.love_cache_import(C.byref(cfg), C.byref(bad), None, None, C.byref(out)) == -1
    no_rt = B.love_import(10, 0, None, None, None, None, None, None)
    assert lib.love_cache_import(C.byref(cfg), C.byref(no_rt), None, None, C.byref(out)) == -1
    s_missing = B.love_import(10, 5, None, None, C.c_void_p(256), None, None, None)
    assert lib.love_cache_import(C.byref(cfg), C.byref(s_missing), None, None, C.byref(out)) == -1


def test_host_validation_rejects_bad_arguments(lib):
    from paper_1803_06058_amd import binding as B
    out = C.c_void_p()
    # null config / null pointers / bad sizes: rejected before touching the device
    assert lib.love_build_cache(None, C.c_void_p(8), C.c_void_p(8), 10, None, None, C.byref(out)) == -1
    cfg = B.config_struct(1, [100], [0.0], [1.0], lengthscale=[0.1], k=10)
    assert lib.love_build_cache(C.byref(cfg), None, C.c_void_p(8), 10, None, None, C.byref(out)) == -1
    assert lib.love_build_cache(C.byref(cfg), C.c_void_p(8), C.c_void_p(8), 0, None, None, C.byref(out)) == -1
    for field, bad in (("d", 0), ("d", 5), ("k", 0), ("k", 129), ("noise", 0.0), ("noise", -1.0),
                       ("outputscale", 0.0), ("precision", 7), ("toeplitz", 9), ("kernel", 3),
                       ("k_sample", -1), ("cg_tol", -1.0)):
        c2 = B.config_struct(1, [100], [0.0], [1.0], lengthscale=[0.1], k=10)
        setattr(c2, field, bad)
        assert lib.love_build_cache(C.byref(c2), C.c_void_p(8), C.c_void_p(8), 10, None, None,
                                    C.byref(out)) == -1, field
    c3 = B.config_struct(1, [3], [0.0], [1.0], lengthscale=[0.1], k=10)        # m < 4
    assert lib.love_build_cache(C.byref(c3), C.c_void_p(8), C.c_void_p(8), 10, None, None, C.byref(out)) == -1
    c4 = B.config_struct(1, [100], [1.0], [0.0], lengthscale=[0.1], k=10)      # lo >= hi
    assert lib.love_build_cache(C.byref(c4), C.c_void_p(8), C.c_void_p(8), 10, None, None, C.byref(out)) == -1
    c5 = B.config_struct(1, [100], [0.0], [1.0], lengthscale=[-0.1], k=10)     # lengthscale <= 0
    assert lib.love_build_cache(C.byref(c5), C.c_void_p(8), C.c_void_p(8), 10, None, None, C.byref(out)) == -1
    assert lib.love_predict_mean_var(None, C.c_void_p(8), 1, None, C.c_void_p(8), None) == -1
    assert lib.love_sample_posterior(None, C.c_void_p(8), 1, C.c_void_p(8), 1, C.c_void_p(8), None) == -1
    assert lib.love_predict_backward(None, C.c_void_p(8), 1, None, None, C.c_void_p(8), None, None) == -1
    assert lib.love_cache_info(None, None) == -1
    k1, k2 = C.c_int32(), C.c_int32()
    assert lib.love_cache_keff(None, C.byref(k1), C.byref(k2)) == -1
    assert lib.love_apply_khat(None, None, None, None) == -1
    assert lib.love_build_cache_batched(0, None, None, None, None, None, None, None) == -1
    lib.love_cache_free(None)   # no-op


def test_additive_validation(lib):
    """Additive compositions: the stacked grid's sizes are checked as sums,
    and a batch must agree on the composition (both before any device call)."""
    from paper_1803_06058_amd import binding as B
    out = C.c_void_p()
    big = B.config_struct(2, [1 << 25, 100], [0.0, 0.0], [1.0, 1.0], lengthscale=[0.1], k=10,
                          flags=B.FLAG_ADDITIVE)
    assert lib.love_build_cache(C.byref(big), C.c_void_p(8), C.c_void_p(8), 10, None, None, C.byref(out)) == -1
    small = B.config_struct(2, [3, 100], [0.0, 0.0], [1.0, 1.0], lengthscale=[0.1], k=10,
                            flags=B.FLAG_ADDITIVE)                        # m < 4 on an axis
    assert lib.love_build_cache(C.byref(small), C.c_void_p(8), C.c_void_p(8), 10, None, None, C.byref(out)) == -1
    a = B.config_struct(2, [50, 60], [0.0, 0.0], [1.0, 1.0], lengthscale=[0.1], k=10,
                        flags=B.FLAG_ADDITIVE)
    p = B.config_struct(2, [50, 60], [0.0, 0.0], [1.0, 1.0], lengthscale=[0.1], k=10)
    cfgs = (B.love_config * 2)(a, p)
    ptrs = (C.c_void_p * 2)(8, 8)
    ns = (C.c_int64 * 2)(10, 10)
    outs = (C.c_void_p * 2)()
    assert lib.love_build_cache_batched(2, cfgs, ptrs, ptrs, ns, None, None, outs) == -1


def test_python_binding_refuses_cpu_tensors(lib):
    import torch
    from paper_1803_06058_amd import binding as B
    cfg = B.config_struct(1, [100], [0.0], [1.0], lengthscale=[0.1], k=10)
    with pytest.raises(ValueError):
        B.build_cache(cfg, torch.zeros(10, 1), torch.zeros(10))


def test_allocator_without_callbacks_rejected(lib):
    """A love_allocator must carry both callbacks: a missing one is an
    argument error, reported before any device memory is touched."""
    from paper_1803_06058_amd import binding as B
    out = C.c_void_p()
    cfg = B.config_struct(1, [100], [0.0], [1.0], lengthscale=[0.1], k=10)
    half = B.love_allocator()
    half.alloc = B.ALLOC_FN(lambda n, s, ctx: None)      # free missing
    assert lib.love_build_cache(C.byref(cfg), C.c_void_p(8), C.c_void_p(8), 10, C.byref(half),
                                None, C.byref(out)) == -1
    im = B.love_import(10, 0, None, None, C.c_void_p(256), None, None, None)
    assert lib.love_cache_import(C.byref(cfg), C.byref(im), C.byref(half), None, C.byref(out)) == -1
    cfgs = (B.love_config * 1)(cfg)
    ptrs = (C.c_void_p * 1)(8)
    ns = (C.c_int64 * 1)(10)
    outs = (C.c_void_p * 1)()
    assert lib.love_build_cache_batched(1, cfgs, ptrs, ptrs, ns, C.byref(half), None, outs) == -1
    assert lib.love_predict_covar_block(None, None, 0, None, 0, None, C.byref(half), None) == -1
    assert not out.value
