"""Build the host-sanitized test driver: every source of the library and
tests/host_sanitize_driver.cpp with AddressSanitizer and UndefinedBehavior-
Sanitizer on the host code only (each -fsanitize directly after -Xarch_host;
the device code is compiled as usual), linked into one executable,
paper_2408_04440_amd/mpchol_host_sanitize.  tests/test_gpu_host_sanitize.py
runs it."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2408_04440_amd import build as B  # noqa: E402

OUT = os.path.join(HERE, "mpchol_host_sanitize")
SAN_BUILD = os.path.join(B.BUILD, "host_sanitize")
# UndefinedBehaviorSanitizer without its function-type check: with that check
# the update kernels launched through host function pointers (k_factor.hip)
# silently computed wrong factors (device code unchanged, no report), while
# AddressSanitizer and the other UBSan checks leave every result intact.
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize=function "
            "-Xarch_host -fno-omit-frame-pointer").split()
DRIVER = os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")


def _compile(src: str) -> str:
    obj = os.path.join(SAN_BUILD, os.path.basename(src) + ".o")
    cmd = [B.HIPCC, *B.FLAGS, "-g", *HOST_SAN, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_host_sanitize(verbose: bool = False) -> str:
    os.makedirs(SAN_BUILD, exist_ok=True)
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [DRIVER]
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [B.HIPCC, f"--offload-arch={B.ARCH}", *HOST_SAN, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build_host_sanitize(verbose=True)
