"""The learned selector at L = 400 (N = 160,000, tile 1024, 157 tiles per side
with a 256-row last tile), rho in {5, 20}: the learned map (randomized
verification, norm-rule refactorization on a violation) against the norm
rule and the plain FP64 path on the same handle.  Acceptance as for the mixed
path: exact backward error <= 1e-9 after any fallback, logdet within 1e-8 of
the closed form; fallbacks are counted and reported."""
import numpy as np
import pytest

import synth
from _gpu import M, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rho", [5.0, 20.0])
def test_c5_learned_norm_fp64(orc, rho):
    import paper_2408_04440_amd.selector as S

    L, tile, eps = 400, 1024, 1e-9
    n = L * L
    nt = (n + tile - 1) // tile
    sigma, x = synth.workload(L)
    ref = orc.markov_logdet(sigma, x, rho, 1e-8)
    mod = M()
    res = {}
    h = mod.mpchol_create(n, tile, verify=2, verify_eps=eps)
    try:
        mod.mpchol_selector_set(h, S.load())
        for name, rule in (("learned", mod.RULE_LEARNED), ("norm", mod.RULE_NORM), ("fp64", mod.RULE_FP64)):
            log(f"C5 rho={rho} rule={name}")
            mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
            mp = mod.mpchol_precision_map(h, rule, eps)
            assert mod.mpchol_factor(h) == 0
            st = mod.mpchol_get_stats(h)
            ld = mod.mpchol_logdet(h)
            # exact FP64 residual for the mixed maps; the plain FP64 path by the estimator
            be = mod.mpchol_backward_error(h) if rule != mod.RULE_FP64 else mod.mpchol_backward_error_estimate(h, 1, 3)
            hist = np.bincount(mp[np.tril_indices(nt, -1)], minlength=4)
            res[name] = dict(t=st["t_factor_ms"], be=be, ld=abs(ld - ref) / abs(ref), fb=st["fallbacks"],
                             used=st["rule_used"], first=st["verify_first"], hist=hist.tolist())
            log(f"  {name}: t_factor={st['t_factor_ms']:.0f} ms ({n ** 3 / 3 / st['t_factor_ms'] / 1e9:.1f} TF/s) "
                f"be={be:.3e} logdet rel={res[name]['ld']:.2e} fallbacks={st['fallbacks']} "
                f"rule used={st['rule_used']} verify={st['verify_first']:.3e} hist={hist.tolist()}")
    finally:
        mod.mpchol_destroy(h)
    for name in ("learned", "norm"):
        assert res[name]["be"] <= eps
        assert res[name]["ld"] <= 1e-8
    assert res["fp64"]["be"] <= 1e-13 and res["fp64"]["ld"] <= 1e-11
    # a learned map that failed verification was replaced (and counted); the
    # map kept is then the norm rule's or the FP64 one
    if res["learned"]["fb"] > 0:
        assert res["learned"]["used"] in (mod.RULE_NORM, mod.RULE_FP64)
    else:
        assert res["learned"]["used"] == mod.RULE_LEARNED
        assert 0 < res["learned"]["first"] * (1 + 3 / np.sqrt(128)) <= eps
    log(f"  C5 rho={rho}: learned {res['learned']['t']:.0f} ms, norm {res['norm']['t']:.0f} ms, "
        f"fp64 {res['fp64']['t']:.0f} ms; speedup over FP64 learned {res['fp64']['t'] / res['learned']['t']:.2f}x, "
        f"norm {res['fp64']['t'] / res['norm']['t']:.2f}x")
    # the mixed maps are faster than the plain FP64 path
    assert res["norm"]["t"] < res["fp64"]["t"] and res["learned"]["t"] < res["fp64"]["t"]
