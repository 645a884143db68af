"""Benchmark of the mixed-precision tile Cholesky on one MI355X.

A step is one pass of the hot path over the synthetic covariance of the
band-limit-L spherical-harmonic workload: device generation, tile norms and
the precision map (norm rule), the factorization, the log-determinant and the
emulation draws L z.  The reported value is the Cholesky rate
(N^3/3) / t_factor in TFLOP/s, t_factor being the wall time of the
mpchol_factor call of each timed step (median; the call synchronizes and
includes any verification and fallback); the event-timed kernel span is
reported beside it.  The plain FP64 path (same library, every tile
FP64) is timed after the mixed steps for the speedup.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c4]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONFIGS = {
    # name: L, tile, rho, eps, lo16, allowed mask, draws, rhs
    "c1": dict(L=32, tile=128, rho=5.0, eps=1e-9, lo16=0, allowed=0b0001, draws=0, rhs=1, label="FP64"),
    "c2": dict(L=128, tile=512, rho=5.0, eps=1e-9, lo16=0, allowed=0b0001, draws=0, rhs=16, label="FP64"),
    "c3": dict(L=256, tile=1024, rho=5.0, eps=1e-9, lo16=1, allowed=0b0111, draws=0, rhs=0, label="FP64/FP32/BF16"),
    "c4": dict(L=360, tile=1024, rho=5.0, eps=1e-9, lo16=0, allowed=0b1111, draws=1000, rhs=0,
               label="FP64/FP32/FP16/FP8-e4m3"),
    "c5": dict(L=400, tile=1024, rho=5.0, eps=1e-9, lo16=0, allowed=0b1111, draws=0, rhs=0,
               label="FP64/FP32/FP16/FP8-e4m3"),
}
PEAK = [78.6, 157.3, 2500.0, 5000.0]  # dense MFMA TFLOP/s: FP64, FP32, FP16, FP8
CLASS = ["fp64", "fp32", "fp16", "fp8"]
METRIC = "Cholesky TFLOP/s (N³/3) mixed vs FP64 at backward err ≤1e-9, N=129,600"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


UPDATE_SOURCES = ["paper_2408_04440_amd/csrc/gemm_core.h", "paper_2408_04440_amd/csrc/k_factor.hip",
                  "paper_2408_04440_amd/build.py"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_update_c4.json")


def update_kernel_hash():
    """Hash of the update kernels' sources and build flags: counter-based
    traffic numbers are only reported while the kernels are the ones they were
    measured on."""
    import hashlib

    h = hashlib.sha256()
    for f in UPDATE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def solve_backward_error(sigma, x, rho, nugget, X, B0, fro):
    """Normwise backward error ||B - Sigma X||_F / (||Sigma||_F ||X||_F + ||B||_F)
    of the solve, with Sigma regenerated on the host in row blocks."""
    n = len(sigma)
    R = np.array(B0, dtype=np.float64, copy=True)
    for i0 in range(0, n, 2048):
        i1 = min(n, i0 + 2048)
        S = sigma[i0:i1, None] * sigma[None, :] * np.exp(-np.abs(x[i0:i1, None] - x[None, :]) / rho)
        S[np.arange(i1 - i0), np.arange(i0, i1)] += nugget
        R[i0:i1] -= S @ X
    return float(np.linalg.norm(R) / (fro * np.linalg.norm(X) + np.linalg.norm(B0)))


def verify_value(v):
    """The first verified map's backward error for the JSON line: None when no
    map was verified, "breakdown" when its factorization failed."""
    if v < 0:
        return None
    return v if math.isfinite(v) else "breakdown"


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None when absent or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != update_kernel_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(sigma, x, rho, nugget, target_s=15.0):
    """The oracle's plain FP64 Cholesky timed on the host on a bounded sample
    (the leading n_s x n_s block of the same covariance), plus the O(N)
    closed-form log-determinant of the full workload used for the accuracy
    report."""
    import oracle

    oracle.lib()
    ns = 1024
    t = 0.0
    while True:
        A = oracle.cov_dense(sigma[:ns], x[:ns], rho, nugget)
        t0 = time.perf_counter()
        _, info = oracle.potrf(A)
        t = time.perf_counter() - t0
        if t * 6.0 > target_s or ns >= 8192:
            break
        ns *= 2
    ld_ref = oracle.markov_logdet(sigma, x, rho, nugget)
    n = len(sigma)
    rate = ns ** 3 / 3.0 / t
    return {"value": rate / 1e12, "unit": "TFLOP/s", "cores": oracle.threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"plain FP64 right-looking Cholesky of the leading {ns}x{ns} block of the same covariance "
                      f"({t:.2f} s, info={info})",
            # the full workload at the sample's N^3 rate (not run: the oracle's dense FP64 matrix
            # alone would take 8 N^2 bytes of host memory)
            "extrapolated_full_s": round(n ** 3 / 3.0 / rate, 1),
            "extrapolated_full_note": f"N={n} at the measured rate of the {ns}x{ns} sample; extrapolated, not run"}, ld_ref


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_sht(M, torch, L, T, reps, cpu):
    """Forward and inverse SHT of T band-limited fields (inverse of N(0,1)/(1+l)
    coefficients, generated on the device) on the L+1 x 2L grid, timed with
    events on the transform's stream; per-field rates and the whole-call
    rooflines (algorithmic HBM bytes: the field and its coefficients once;
    FP64 GEMM flops of the folded tables)."""
    import synth

    nth, nph = L + 1, 2 * L
    st = torch.cuda.current_stream()
    s = M.mpchol_sht_create(L, nth, nph, T, stream=st)
    try:
        info = M.mpchol_sht_info(s)
        g = torch.Generator(device="cuda")
        g.manual_seed(synth.SEED_SHT_COEFFS)
        f = torch.randn((T, L * L), dtype=torch.float64, device="cuda", generator=g)
        f *= torch.tensor(1.0 / (1.0 + synth.sh_degrees(L)), device="cuda")
        Z = torch.empty((T, nth, nph), dtype=torch.float64, device="cuda")
        f2 = torch.empty_like(f)
        M.mpchol_sht_inverse(s, f, Z, L)
        M.mpchol_sht_forward(s, Z, f2, L)
        torch.cuda.synchronize()
        rt = ((f2 - f).abs().max() / f.abs().max()).item()
        times = {}
        for name, fn in (("forward", lambda: M.mpchol_sht_forward(s, Z, f2, L)),
                         ("inverse", lambda: M.mpchol_sht_inverse(s, f, Z, L))):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(st)
            for _ in range(reps):
                fn()
            ev[1].record(st)
            ev[1].synchronize()
            times[name] = ev[0].elapsed_time(ev[1]) / reps
    finally:
        M.mpchol_sht_destroy(s)
    field_b, coef_b = nth * nph * 8, L * L * 8
    out = {"L": L, "grid": [nth, nph], "batch": T, "round_trip_rel_err": rt,
           "table_bytes": info["table_bytes"], "work_bytes": info["work_bytes"]}
    for name in ("forward", "inverse"):
        ms = times[name]
        out[name] = {"ms_per_call": round(ms, 3), "us_per_field": round(ms * 1e3 / T, 3),
                     "fields_per_s": round(T / ms * 1e3, 1),
                     "hbm_gbs_algorithmic": round((field_b + coef_b) * T / ms / 1e6, 1),
                     "gemm_tflops": round(info["gemm_flops_per_step"] * T / ms / 1e9, 2)}
    if cpu:
        import oracle.sht as osht  # CPU leg only

        from threadpoolctl import threadpool_limits

        D = osht.wigner_table(L)
        Zs = synth.sht_fields(2, nth, nph)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            for t in range(2):
                osht.sht_forward_real(Zs[t], L, D)
            tc = (time.perf_counter() - t0) / 2
        out["cpu_baseline"] = {"value": round(1.0 / tc, 4), "unit": "fields/s", "cores": 1, "kind": "oracle",
                               "sample": f"oracle forward SHT (numpy FFT + Wigner-d sums) of 2 white-noise fields "
                                         f"at L={L} ({tc:.2f} s per field, Wigner table excluded)"}
    return out


def bench_band(M, torch, n, tile, cfg, sigma, x, rho, nugget, flops, fp64, lo32, lo64):
    """The band precision variants of Sec. IV.B on the same workload, one
    untimed run then one timed run each: DP/SP (one FP64 band, the rest
    FP32), DP/SP/HP (then the narrowest band holding >= 5% of the
    strict-lower tiles in FP32, the rest 16-bit), DP/HP (the rest 16-bit).
    Backward error by the randomized estimate (64 probes; relative standard
    deviation about 0.09); these maps ignore the accuracy budget."""
    names = {1: "DP/SP", 2: "DP/SP/HP", 3: "DP/HP"}
    out = {}
    for v in (1, 2, 3):
        hb = M.mpchol_create(n, tile, stream=torch.cuda.current_stream(), lo16=cfg["lo16"], allowed=cfg["allowed"],
                             band_variant=v, lo32=lo32, lo64=lo64)
        try:
            ts = []
            for r in range(2):
                M.mpchol_set_generator(hb, sigma, x, rho, nugget)
                cm = M.mpchol_precision_map(hb, M.RULE_BAND)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = M.mpchol_factor(hb)
                ts.append((time.perf_counter() - t0) * 1e3)
            st = M.mpchol_get_stats(hb)
            be = M.mpchol_backward_error_estimate(hb, 1, 5) if info == 0 else None
        finally:
            M.mpchol_destroy(hb)
        nt = st["nt"]
        out[names[v]] = {"t_factor_ms": round(ts[-1], 1), "tflops": round(flops / ts[-1] / 1e9, 3),
                         "speedup_vs_fp64": None if fp64 is None else round(flops / ts[-1] / 1e9 / fp64, 3),
                         "backward_error_estimate": be, "info": info,
                         "tiles_per_class": np.bincount(cm[np.tril_indices(nt, -1)], minlength=4).tolist()}
        log(f"  band {names[v]}: {out[names[v]]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4", choices=sorted(CONFIGS))
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed runs of the plain FP64 path (median reported; one untimed warm-up run first)")
    ap.add_argument("--no-band", action="store_true",
                    help="skip the band variants (DP/SP, DP/SP/HP, DP/HP) timed after the steps")
    ap.add_argument("--no-berr", action="store_true", help="skip the FP64 residual check")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--rho", type=float, default=None, help="override the workload's rho")
    ap.add_argument("--eps", type=float, default=None, help="override the workload's accuracy threshold")
    ap.add_argument("--lo32", default="bf16x3", choices=["fp32", "bf16x3"],
                    help="FP32-class update arithmetic: FP32 MFMA or three-way BF16 split products")
    ap.add_argument("--lo64", default="fp64", choices=["fp64", "int8"],
                    help="FP64-class update products beyond the FP64 band: FP64 MFMA, or exact integer products "
                         "from INT8 residues (the plain FP64 comparison path always uses the FP64 MFMA)")
    ap.add_argument("--lo8", default="tile", choices=["tile", "mx"],
                    help="FP8-class copies: one power-of-two scale per tile, or an E8M0 scale per 32 K elements of "
                         "a row applied inside the block-scaled FP8 MFMA")
    ap.add_argument("--band-variant", type=int, default=None, choices=[1, 2, 3],
                    help="band rule variant: 1 DP/SP, 2 DP/SP/HP, 3 DP/HP")
    ap.add_argument("--rule", default=None, choices=["norm", "learned", "fp64", "band", "learned_unverified"],
                    help="precision map of the timed steps (default: learned for the four-class workloads c4/c5, "
                         "norm for c3, fp64 for FP64-only workloads)")
    ap.add_argument("--compare", default=None, help="comma list of extra rules timed once after the steps, "
                    "each with its backward error (e.g. norm,learned)")
    ap.add_argument("--producer", type=int, default=0, metavar="M",
                    help="also time the covariance producer (Sigma = Xi Xi^T / M + nugget I) for M samples")
    ap.add_argument("--sht", type=int, default=None, metavar="L",
                    help="also time the spherical harmonic transform and its inverse at band limit L "
                         "(grid L+1 x 2L) on a batch of --sht-batch fields (default 360 with --config c4, 0 = off)")
    ap.add_argument("--sht-batch", type=int, default=0, metavar="T",
                    help="fields per SHT call (default 512 at L <= 400, else 128)")
    ap.add_argument("--sht-only", action="store_true", help="skip the factorization; time only the SHT")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="run one plain device copy of MB megabytes first (counter calibration)")
    args = ap.parse_args()
    # the path's precision choice on the four-class workloads is the learned selector
    # (MLP map, randomized backward-error check, norm-rule fallback); the norm rule
    # alone is timed beside it
    if args.rule is None and args.config in ("c4", "c5"):
        args.rule = "learned"
    if args.compare is None:
        args.compare = {"learned": "norm", "norm": "learned"}.get(args.rule, "") if args.config in ("c4", "c5") else ""
    if args.sht is None:  # the transform of the same band limit beside the default workload
        args.sht = 360 if args.config == "c4" and not args.sht_only else 0
    if args.gpus != 1:
        print(f"bench.py: the factorization runs on one GPU (asked for --gpus {args.gpus}); "
              "its decomposition over several GPUs is designed, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2408_04440_amd.mpchol as M

    sht_T = args.sht_batch or (512 if args.sht <= 400 else 128)
    if args.sht_only:
        Ls = args.sht or 360
        sht = bench_sht(M, torch, Ls, sht_T, max(args.steps, 1), not args.no_cpu)
        log(f"  sht: {sht}")
        print(json.dumps({"metric": f"SHT fields/s (forward), L={Ls}", "value": sht["forward"]["fields_per_s"],
                          "unit": "fields/s", "n_gpus": 1, "steps": args.steps, "higher_is_better": True,
                          "dtype": "f64", "data": "synthetic", "sht": sht}), flush=True)
        return

    cfg = CONFIGS[args.config]
    L, tile, rho, eps = cfg["L"], cfg["tile"], cfg["rho"], cfg["eps"]
    if args.rho is not None:
        rho = args.rho
    if args.eps is not None:
        eps = args.eps
    n = L * L
    nugget = 1e-8
    flops = n ** 3 / 3.0
    sigma, x = synth.workload(L)
    log(f"bench: config={args.config} N={n} tile={tile} rho={rho} eps={eps} classes={cfg['label']}")

    if args.copy_calibration > 0:
        nb = args.copy_calibration * (1 << 20)
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"  copy calibration: {nb} bytes read, {nb} bytes written by one copy kernel")
        del src, dst

    RULES = {"norm": M.RULE_NORM, "learned": M.RULE_LEARNED, "fp64": M.RULE_FP64, "band": M.RULE_BAND,
             "learned_unverified": M.RULE_LEARNED}
    stream = torch.cuda.current_stream()
    need_w = (args.rule or "").startswith("learned") or "learned" in args.compare
    extra = {} if args.band_variant is None else {"band_variant": args.band_variant}
    extra["lo32"] = M.LO32_BF16X3 if args.lo32 == "bf16x3" else M.LO32_FP32
    extra["lo64"] = M.LO64_INT8 if args.lo64 == "int8" else M.LO64_FP64
    extra["lo8"] = M.LO8_MX if args.lo8 == "mx" else M.LO8_TILE
    h = M.mpchol_create(n, tile, stream=stream, lo16=cfg["lo16"], allowed=cfg["allowed"], profile=1,
                        verify=2 if need_w else 0, verify_eps=eps, **extra)
    M.mpchol_set_generator(h, sigma, x, rho, nugget)
    if need_w:
        from paper_2408_04440_amd import selector as S

        M.mpchol_selector_set(h, S.load())
    rule = RULES[args.rule] if args.rule else (M.RULE_NORM if cfg["allowed"] != 1 else M.RULE_FP64)
    Y = torch.empty((cfg["draws"], n), dtype=torch.float32, device="cuda") if cfg["draws"] else None
    B = torch.empty((cfg["rhs"], n), dtype=torch.float64, device="cuda") if cfg["rhs"] else None
    Brhs = torch.tensor(np.ascontiguousarray(synth.rhs(n, cfg["rhs"]).T), device="cuda") if cfg["rhs"] else None

    def step():
        M.mpchol_set_generator(h, sigma, x, rho, nugget)
        cmap = M.mpchol_precision_map(h, rule, eps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = M.mpchol_factor(h)  # synchronizes; includes verification and fallbacks
        t_call = (time.perf_counter() - t0) * 1e3
        if info:
            raise RuntimeError(f"factorization failed at column {info}")
        ld = M.mpchol_logdet(h)
        if Y is not None:
            M.mpchol_sample(h, cfg["draws"], synth.SEED_DRAWS, Y.T, n)
        if B is not None:
            B.copy_(Brhs)
            M.mpchol_solve(h, B.T, n)
        st = M.mpchol_get_stats(h)
        st["t_call_ms"] = t_call
        return cmap, ld, st

    for w in range(args.warmup):
        _, _, st = step()
        log(f"  warmup {w}: t_factor={st['t_factor_ms']:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tf, sts = [], []
    for s in range(args.steps):
        cmap, ld, st = step()
        tf.append(st["t_call_ms"])
        sts.append(st)
        log(f"  step {s}: factor call={st['t_call_ms']:.1f} ms (kernels {st['t_factor_ms']:.1f} ms, "
            f"fallbacks {st['fallbacks']})  map={st['t_map_ms']:.1f} ms  {flops / st['t_call_ms'] / 1e9:.2f} TFLOP/s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_med = statistics.median(tf)
    st = sts[tf.index(t_med)] if t_med in tf else sts[-1]
    value = flops / t_med / 1e9
    nt = st["nt"]
    hist = np.bincount(cmap[np.tril_indices(nt, -1)], minlength=4)

    # accuracy of the mixed factor of the last step
    solve_be = None
    if B is not None:
        X = B.cpu().numpy().T  # n x rhs, the last step's solution
        solve_be = solve_backward_error(sigma, x, rho, nugget, X, synth.rhs(n, cfg["rhs"]), st["total_fro"])
        log(f"  solve backward error {solve_be:.3e}")
    berr = None
    if not args.no_berr:
        berr = M.mpchol_backward_error(h)
        log(f"  backward error {berr:.3e} ({M.mpchol_get_stats(h)['t_residual_ms']:.0f} ms)")

    # dominant update kernel: the class with the most GEMM time
    q = int(np.argmax(st["t_gemm_ms"]))
    ach = st["gemm_flops"][q] / st["t_gemm_ms"][q] / 1e9 if st["t_gemm_ms"][q] > 0 else 0.0
    t_roof = sum(st["flops_per_class"][c] / (PEAK[c] * 1e12) for c in range(4))
    roofline = {"bound": "mfma", "kernel": f"update_{CLASS[q]}", "achieved": round(ach, 3), "peak": PEAK[q],
                "unit": "TFLOP/s", "frac": round(ach / PEAK[q], 4),
                "traffic": measured_traffic(f"update_{CLASS[q]}") if args.config == "c4" else None,
                "algorithmic_flops_per_launch": st["gemm_flops"][q] / max(st["gemm_launches"][q], 1),
                "launches": st["gemm_launches"][q],
                "mixed_roofline_frac": round(t_roof / (t_med / 1e3), 4)}

    # plain FP64 path, same library
    fp64, t64 = None, []
    if rule != M.RULE_FP64 and args.fp64_steps > 0:
        for r in range(args.fp64_steps + 1):  # the first run is an untimed warm-up
            M.mpchol_set_generator(h, sigma, x, rho, nugget)
            M.mpchol_precision_map(h, M.RULE_FP64)
            torch.cuda.synchronize()
            t640 = time.perf_counter()
            if M.mpchol_factor(h):
                raise RuntimeError("FP64 factorization failed")
            tr = (time.perf_counter() - t640) * 1e3
            log(f"  fp64 {'warmup' if r == 0 else 'run ' + str(r)}: t_factor={tr:.1f} ms  {flops / tr / 1e9:.2f} TFLOP/s")
            if r > 0:
                t64.append(tr)
        fp64 = flops / statistics.median(t64) / 1e9
        # the plain FP64 path as a fraction of the FP64 MFMA peak
        roofline["fp64_path_frac"] = round(fp64 / PEAK[0], 4)
    compare = {}
    for name in [c for c in args.compare.split(",") if c]:
        M.mpchol_set_verify(h, 0 if name == "learned_unverified" else 2, eps)
        M.mpchol_set_generator(h, sigma, x, rho, nugget)
        cm = M.mpchol_precision_map(h, RULES[name], eps)
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        info = M.mpchol_factor(h)
        t_call = (time.perf_counter() - tc0) * 1e3
        stc = M.mpchol_get_stats(h)
        bec = M.mpchol_backward_error(h) if info == 0 else None
        compare[name] = {"t_factor_ms": round(t_call, 1), "t_factor_kernels_ms": round(stc["t_factor_ms"], 1),
                         "tflops": round(flops / t_call / 1e9, 3), "backward_error": bec,
                         "fallbacks": stc["fallbacks"], "rule_used": stc["rule_used"],
                         "verify_first": verify_value(stc["verify_first"]),
                         "tiles_per_class": [int(v) for v in stc["tiles_per_class"]]}
        log(f"  compare {name}: {compare[name]}")
    producer = None
    if args.producer > 0:
        # residual-like samples on the device: N(0,1) scaled by (1+l)^-1, seed 4
        m_s = args.producer
        g = torch.Generator(device="cuda")
        g.manual_seed(synth.SEED_SAMPLES)
        Xs = torch.randn((m_s, n), dtype=torch.float64, device="cuda", generator=g)
        Xs *= torch.tensor(1.0 / (1.0 + synth.sh_degrees(L)[:n]), device="cuda")
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        M.mpchol_set_samples(h, Xs.T, 1.0 / m_s, nugget)
        t_wall = (time.perf_counter() - tp0) * 1e3
        stp = M.mpchol_get_stats(h)
        fl = float(n) * (n + 1) * m_s
        producer = {"m": m_s, "t_ms": round(stp["t_samples_ms"], 2), "t_call_ms": round(t_wall, 2),
                    "tflops": round(fl / stp["t_samples_ms"] / 1e9, 3), "fp64_peak_frac": round(fl / stp["t_samples_ms"] / 1e9 / PEAK[0], 4),
                    "algorithmic_flops": fl}
        log(f"  producer: {producer}")
        del Xs
    M.mpchol_destroy(h)
    band = None
    if not args.no_band and args.config in ("c3", "c4"):
        band = bench_band(M, torch, n, tile, cfg, sigma, x, rho, nugget, flops, fp64, extra["lo32"], extra["lo64"])
    sht = None
    if args.sht > 0:
        sht = bench_sht(M, torch, args.sht, sht_T, max(args.steps, 1), False)
        log(f"  sht: {sht}")

    cpu, ld_ref = (None, None)
    if not args.no_cpu:
        cpu, ld_ref = cpu_baseline(sigma, x, rho, nugget)
        log(f"  cpu baseline {cpu}")

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if rule == M.RULE_FP64 else ("f64+int8crt" if args.lo64 == "int8" else "f64") + "/" +
                 ("bf16x3-f32acc" if args.lo32 == "bf16x3" else "f32") + "/" +
                 ("bf16" if cfg["lo16"] else "f16") +
                 (("/fp8-e4m3" + ("-mx32" if args.lo8 == "mx" else "")) if cfg["allowed"] & 8 else ""),
        "data": "synthetic",
        "config": {"workload": f"SH covariance L={L} (N={n}), tile {tile}, rho={rho}, nugget 1e-8, "
                               f"{[k for k, v in RULES.items() if v == rule][0]} rule eps={eps}, classes {cfg['label']}",
                   "N": n, "tile": tile, "nt": nt, "rho": rho, "eps": eps, "fp32_class": args.lo32,
                   "fp64_class": args.lo64, "fp8_scales": "per 32 K elements (E8M0)" if args.lo8 == "mx" else "per tile",
                   "step": "generate+norms+map+factor+logdet" + ("+1000 draws" if cfg["draws"] else "")
                           + (f"+solve({cfg['rhs']} rhs)" if cfg["rhs"] else "")},
        "t_factor_ms": round(t_med, 2),
        "t_factor_kernels_ms": round(st["t_factor_ms"], 2),
        "fp64_tflops": None if fp64 is None else round(fp64, 3),
        "speedup_vs_fp64": None if fp64 is None else round(value / fp64, 3),
        "rule": [k for k, v in RULES.items() if v == rule][0],
        "fallbacks": st["fallbacks"],
        "verify_first": verify_value(st["verify_first"]),
        "compare": compare or None,
        "fp64_ms": None if not t64 else [round(v, 1) for v in t64],
        "band_variants": band,
        "producer": producer,
        "sht": sht,
        "backward_error": berr,
        "logdet_rel_err": None if ld_ref is None else abs(ld - ld_ref) / abs(ld_ref),
        "solve_backward_error": solve_be,
        "tiles_per_class": {CLASS[c]: int(hist[c]) for c in range(4)},
        "flop_share": {CLASS[c]: round(st["flops_per_class"][c] / sum(st["flops_per_class"]), 4) for c in range(4)},
        "gemm_tflops": {CLASS[c]: round(st["gemm_flops"][c] / st["t_gemm_ms"][c] / 1e9, 2)
                        for c in range(4) if st["t_gemm_ms"][c] > 0},
        "gemm_ms": {CLASS[c]: round(st["t_gemm_ms"][c], 1) for c in range(4)},
        "gemm_fp64_int8": None if not st["gemm_int8_launches"] else
        {"ms": round(st["t_gemm_int8_ms"], 1), "launches": st["gemm_int8_launches"],
         "tflops_fp64_equivalent": round(st["gemm_int8_flops"] / st["t_gemm_int8_ms"] / 1e9, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "context": "paper: 0.976 EFlop/s DP/HP on 9,025 Frontier nodes (36,100 MI250X), multi-node; not comparable",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
