"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (host only; the kernels are built as usual): the driver
tests/host_sanitize_driver.cpp takes every call of the C ABI through small
problems on the GPU -- every rule and arithmetic option, solve, sampling,
residuals, the selector with verification and fallback, labels, the
covariance producer, the trainer state, the SHT object -- and the error
paths.  Built on the host by paper_2408_04440_amd/build_sanitize.py."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2408_04440_amd",
                   "mpchol_host_sanitize")


def test_host_code_under_sanitizers():
    if not os.path.exists(EXE):
        pytest.skip("the host-sanitized driver is not built (python -m paper_2408_04440_amd.build_sanitize)")
    # leak detection off: the HIP runtime keeps allocations of its own until exit;
    # the link-order check off: the environment may preload a library ahead of the runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.strip().endswith("ok") and "Sanitizer" not in r.stderr, r.stderr[-4000:]
