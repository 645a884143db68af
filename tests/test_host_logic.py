"""Host-side logic that needs no GPU: the benchmark's one-GPU guard, the
selector driver's initialization, class weights and weight files, and the
seeded input module's layout."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_he_uniform_init_bounds():
    from paper_2408_04440_amd import selector as S

    p = S.he_uniform_init(3)
    assert p.shape == (4996,) and p.dtype == np.float32
    w1 = p[:512]
    assert np.max(np.abs(w1)) <= np.sqrt(6 / 8) + 1e-6
    assert np.all(p[512:576] == 0)  # b1
    w2 = p[576:576 + 4096]
    assert np.max(np.abs(w2)) <= np.sqrt(6 / 64) + 1e-6
    assert np.array_equal(p, S.he_uniform_init(3))


def test_class_weights_and_roundtrip(tmp_path):
    from paper_2408_04440_amd import selector as S

    y = np.array([0] * 10 + [1] * 30 + [3] * 60, dtype=np.int32)
    w = S.class_weights(y)
    assert w[2] == 0.0 and w[0] > w[1] > w[3] > 0
    p = S.he_uniform_init(5)
    f = tmp_path / "w.json"
    S.save(p, str(f), meta={"k": 1})
    assert np.array_equal(S.load(str(f)), p)
    assert json.load(open(f))["meta"] == {"k": 1}


def test_checkpoint_roundtrip(tmp_path):
    """A checkpoint holds the weights, Adam's two moments and the step count,
    and reads back exactly (float32 values through JSON); a weights-only file
    is refused as a checkpoint."""
    from paper_2408_04440_amd import selector as S

    p = S.he_uniform_init(7)
    m1 = (np.arange(p.size, dtype=np.float32) - 2000.0) * np.float32(1.0e-7)
    m2 = np.abs(m1) * np.float32(3.3e-3) + np.float32(1e-30)
    f = tmp_path / "ck.json"
    S.save(p, str(f), meta={"k": 2}, state=(p, m1, m2, 123))
    q, n1, n2, st = S.load_checkpoint(str(f))
    assert st == 123 and q.dtype == np.float32
    assert np.array_equal(q, p) and np.array_equal(n1, m1) and np.array_equal(n2, m2)
    assert np.array_equal(S.load(str(f)), p)
    g = tmp_path / "w.json"
    S.save(p, str(g))
    with pytest.raises(ValueError):
        S.load_checkpoint(str(g))


def test_synth_layout():
    L = 7
    l, m = synth.sh_degrees(L), synth.sh_orders(L)
    assert len(l) == L * L
    i = l * l + l + m
    assert np.array_equal(i, np.arange(L * L))
    x = synth.sh_coords(L)
    assert np.all(np.diff(x) > 0)
    s = synth.sh_sigma(L)
    assert np.all(s > 0) and np.all(s * (1 + l) < 2.0)
    u = synth.uniform01(0, 100000)
    assert u.min() > 0 and u.max() <= 1 and abs(u.mean() - 0.5) < 0.01
    assert np.array_equal(synth.splitmix64(5, 4), synth.splitmix64(5, 4))


def test_bench_solve_backward_error():
    """The bench's solve check: ~1e-16 for a numpy solve of the same Sigma,
    exactly 1 for X = 0, and independent of the row blocking."""
    import bench
    import synth

    sigma, x = synth.workload(48)  # n = 2304, two row blocks
    n = len(sigma)
    S = sigma[:, None] * sigma[None, :] * np.exp(-np.abs(x[:, None] - x[None, :]) / 5.0) + 1e-8 * np.eye(n)
    B = synth.rhs(n, 3)
    X = np.linalg.solve(S, B)
    fro = np.linalg.norm(S)
    be = bench.solve_backward_error(sigma, x, 5.0, 1e-8, X, B, fro)
    assert be < 1e-14
    assert bench.solve_backward_error(sigma, x, 5.0, 1e-8, np.zeros_like(B), B, fro) == 1.0
    R = B - S @ (X * (1 + 1e-6))
    want = np.linalg.norm(R) / (fro * np.linalg.norm(X * (1 + 1e-6)) + np.linalg.norm(B))
    got = bench.solve_backward_error(sigma, x, 5.0, 1e-8, X * (1 + 1e-6), B, fro)
    assert abs(got - want) <= 1e-6 * want


# ---------------------------------------------------------------- the oracle under host sanitizers
def test_oracle_under_address_and_undefined_behavior_sanitizers():
    """oracle.c built with AddressSanitizer (leak detection on) and
    UndefinedBehaviorSanitizer, every entry point driven on small cases with a
    ragged last tile (tests/oracle_sanitize_check.c): no invalid access, leak
    or undefined operation, and the driver's checks hold."""
    import shutil
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    out = os.path.join(root, "_build", "oracle_sanitize_check")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
                           os.path.join(root, "oracle", "oracle.c"), os.path.join(root, "tests", "oracle_sanitize_check.c"),
                           "-lm", "-o", out])
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([out], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok" and "Sanitizer" not in r.stderr


# ---------------------------------------------------------------- residue arithmetic of the INT8-emulated FP64 products
def _ozaki_host_check():
    """Build (hipcc, host code) the CPU driver of the library's residue helpers."""
    import shutil
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = os.path.join(root, "_build", "ozaki_host_check")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                           "-Xclang", "-packed-fp32-ops", os.path.join(root, "tests", "ozaki_host_check.cpp"),
                           os.path.join(root, "paper_2408_04440_amd", "csrc", "k_ozaki.hip"), "-o", out],
                          stderr=subprocess.DEVNULL)
    return out


def test_crt_reconstruction_rounds_like_python():
    """The exact integer product recovered from its 15 residues (both exact
    forms of the residue sum) and rounded once to FP64 equals Python's
    correctly rounded float(P), bit for bit, for
    random |P| < 2^116 (the bound of 1024 products of 54-bit integers),
    halfway cases of every size, powers of two, +-1, 0 and the extremes."""
    import random
    import struct
    import subprocess

    exe = _ozaki_host_check()
    rng = random.Random(2024)
    Ps = [0, 1, -1, 2 ** 116, -(2 ** 116), 2 ** 53, 2 ** 53 + 1, -(2 ** 53 + 1), 2 ** 64 - 1, 2 ** 64, 2 ** 64 + 1]
    for e in range(54, 117):
        ulp = 2 ** (e - 52)
        base = rng.randrange(2 ** 52, 2 ** 53) * ulp
        Ps += [base + ulp // 2, -(base + ulp // 2), base + ulp // 2 + 1, base + ulp // 2 - 1, base, 2 ** e,
               base + ulp + ulp // 2]
    for _ in range(4000):
        bits = rng.randrange(1, 117)
        Ps.append(rng.randrange(-(2 ** bits), 2 ** bits))
    lines = [f"P {1 if P < 0 else 0} {abs(P) >> 64:x} {abs(P) & (2 ** 64 - 1):x}" for P in Ps]
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True).stdout.split()
    assert len(out) == 2 * len(Ps)
    for i, P in enumerate(Ps):
        for h in out[2 * i:2 * i + 2]:  # four-limb sums, and the three FP64 parts the update kernel keeps
            got = struct.unpack("<d", struct.pack("<Q", int(h, 16)))[0]
            assert got == float(P) and (got != 0 or P == 0), (P, got, float(P))


def test_residue_conversions():
    """Signed residues of integer-valued doubles |a| <= 2^53 (the operands'
    integers) and residues of INT8 product sums |x| <= 2^24, against Python."""
    import random
    import subprocess

    exe = _ozaki_host_check()
    rng = random.Random(7)
    ps = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197]
    cases, want = [], []
    for _ in range(3000):
        p = rng.choice(ps)
        a = rng.choice([rng.randrange(-(2 ** 53), 2 ** 53 + 1), rng.randrange(-300, 300), 2 ** 53, -(2 ** 53)])
        cases.append(f"sym {float(a)!r} {p}")
        r = a % p
        want.append(r - p if r >= (p + 1) // 2 else r)
        x = rng.randrange(-(2 ** 24), 2 ** 24 + 1)
        cases.append(f"small {x} {p}")
        want.append(x % p)
    out = subprocess.run([exe], input="\n".join(cases) + "\n", capture_output=True, text=True, check=True).stdout.split()
    assert [int(v) for v in out] == want
    for w, c in zip(want[::2], cases[::2]):
        p = int(c.split()[-1])
        assert -(p // 2) <= w <= (p - 1) // 2
