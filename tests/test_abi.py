"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, the ctypes structures match the C layout, and
argument validation happens before any device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpchol.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mpchol_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2408_04440_amd.mpchol as M

    L = M.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n


def test_struct_layouts_match_header(tmp_path):
    import paper_2408_04440_amd.mpchol as M

    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mpchol.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(mpchol_opts), sizeof(mpchol_stats),'
                    ' offsetof(mpchol_opts, verify_eps), offsetof(mpchol_stats, t_gemm_ms), offsetof(mpchol_stats, fallbacks),'
                    ' offsetof(mpchol_stats, verify_first), offsetof(mpchol_opts, lo8));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(M.Opts), C.sizeof(M.Stats), M.Opts.verify_eps.offset, M.Stats.t_gemm_ms.offset,
            M.Stats.fallbacks.offset, M.Stats.verify_first.offset, M.Opts.lo8.offset]
    assert got == want


def test_strerror_and_codes():
    import paper_2408_04440_amd.mpchol as M

    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        s = M.strerror(code)
        assert s and s != "unknown status"
    assert M.strerror(12345) == "unknown status"


def test_argument_validation_without_gpu():
    import paper_2408_04440_amd.mpchol as M

    L = M.lib()
    h = C.c_void_p()
    assert L.mpchol_create(None, 1024, 128, None) == -1
    assert L.mpchol_create(C.byref(h), 0, 128, None) == -1
    assert L.mpchol_create(C.byref(h), 1024, 100, None) == -1   # tile not a multiple of 128
    assert L.mpchol_create(C.byref(h), 1024, 4096, None) == -1
    for field, bad in (("lo8", 2), ("lo8", -1), ("lo64", 2), ("lo32", 7)):
        o = M.mpchol_default_opts()
        setattr(o, field, bad)
        assert L.mpchol_create(C.byref(h), 1024, 128, C.byref(o)) == -1, field
    assert h.value is None
    assert L.mpchol_destroy(None) == 0
    assert L.mpchol_factor(None, None) == -1
    assert L.mpchol_logdet(None, None) == -1
    m = C.c_void_p()
    assert L.mpchol_mlp_create(None, 0, None) == -1
    assert L.mpchol_set_verify(None, 1, C.c_double(1e-9)) == -1
    assert L.mpchol_set_samples(None, None, 0, 0, C.c_double(1.0), C.c_double(0.0), 0) == -1


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_2408_04440_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", txt, re.M), f
                assert "liboracle" not in txt, f
                assert "orc_" not in txt, f


def test_default_opts():
    import paper_2408_04440_amd.mpchol as M

    o = M.mpchol_default_opts()
    assert o.band == 1 and o.allowed == 0xF and o.lo16 == M.LO16_F16 and o.verify_eps == 1e-9
    assert o.lo32 == M.LO32_BF16X3 and o.lo64 == M.LO64_FP64 and o.lo8 == M.LO8_TILE


def test_sht_argument_checks_before_any_device_call():
    import paper_2408_04440_amd.mpchol as M

    L = M.lib()
    s = C.c_void_p()
    bad = [(0, 2, 1, 1), (10, 10, 20, 4), (10, 11, 18, 4), (10, 11, 19, 4), (7, 8, 14, 4), (8, 9, 15, 0),
           (1025, 1026, 2050, 1), (300, 301, 4200, 1)]
    for Lb, nth, nph, tmax in bad:
        assert L.mpchol_sht_create(C.byref(s), Lb, nth, nph, tmax, 0, None) == M.EINVAL, (Lb, nth, nph, tmax)
        assert not s.value
    assert b"2, 3 and 5" in L.mpchol_sht_last_error()  # the last case: 4200 > 4096 and 4200 = 2^3 3 5^2 7
    assert L.mpchol_sht_create(None, 8, 9, 15, 1, 0, None) == M.EINVAL
    assert L.mpchol_sht_forward(None, None, 1, None) == M.EINVAL
    assert L.mpchol_sht_inverse(None, None, 1, None) == M.EINVAL
    assert L.mpchol_sht_info(None, None, None, None) == M.EINVAL
    assert L.mpchol_sht_destroy(None) == 0


def test_sht_binding_checks_shapes():
    import torch

    import paper_2408_04440_amd.mpchol as M

    with pytest.raises(ValueError):
        M.mpchol_sht_forward(C.c_void_p(1), torch.zeros((2, 9, 15), dtype=torch.float64),
                             torch.zeros((2, 63), dtype=torch.float64), 8)
    with pytest.raises(ValueError):
        M.mpchol_sht_inverse(C.c_void_p(1), torch.zeros((2, 64), dtype=torch.float64),
                             torch.zeros((3, 9, 15), dtype=torch.float64), 8)


class _FakeDev:
    """Stands in for a CUDA tensor (no GPU here): only what the binding's
    checks read."""

    def __init__(self, shape, dtype, cuda=True):
        self.shape, self.is_cuda = tuple(shape), cuda
        self.dtype = dtype

    def dim(self):
        return len(self.shape)

    def numel(self):
        n = 1
        for s in self.shape:
            n *= s
        return n

    def stride(self):
        return (1, self.shape[0]) if len(self.shape) == 2 else (1,)

    def data_ptr(self):
        raise AssertionError("the library must not be reached")


def test_binding_rejects_wrong_device_buffers():
    """Wrong dtype, host memory or too few rows/columns are refused by the
    binding before any library call, so a short buffer never reaches a kernel."""
    import torch

    import paper_2408_04440_amd.mpchol as M

    n = 1024
    good32 = _FakeDev((n, 8), torch.float32)
    cases = [
        lambda: M.mpchol_sample(None, 8, 1, _FakeDev((n, 8), torch.float64), n),      # wrong dtype
        lambda: M.mpchol_sample(None, 9, 1, good32, n),                                # too few columns
        lambda: M.mpchol_sample(None, 8, 1, _FakeDev((n - 1, 8), torch.float32), n),  # too few rows
        lambda: M.mpchol_sample(None, 8, 1, torch.zeros((8, n), dtype=torch.float32).T, n),  # host tensor
        lambda: M.mpchol_sample_noalloc(None, 8, 1, _FakeDev((n, 4), torch.float32), n),
        lambda: M.mpchol_sample_z(None, good32, _FakeDev((n, 7), torch.float32), n),
        lambda: M.mpchol_sample_z(None, _FakeDev((n, 8), torch.float16), good32, n),
        lambda: M.mpchol_solve(None, _FakeDev((n, 2), torch.float32), n),             # solve needs float64
        lambda: M.mpchol_solve(None, _FakeDev((n - 5,), torch.float64), n),
        lambda: M.mpchol_get_factor(None, _FakeDev((n, n - 1), torch.float64), n),
        lambda: M.mpchol_normal_draws(None, 100, 1, _FakeDev((99,), torch.float32)),
        lambda: M.mpchol_normal_draws(None, 100, 1, None, _FakeDev((100,), torch.float32)),
        lambda: M.mpchol_set_generator(None, np.ones(n - 1), np.ones(n), 5.0, 1e-8, n=n),
    ]
    for i, f in enumerate(cases):
        with pytest.raises(ValueError):
            f()
