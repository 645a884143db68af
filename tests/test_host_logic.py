"""Host-side logic that needs no GPU: the benchmark's one-GPU guard, the
selector driver's initialization, class weights and weight files, and the
seeded input module's layout."""
import json
import os
import subprocess
import sys

import numpy as np

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
