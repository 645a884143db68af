"""Learned precision selector: MLP kernels against the FP64 oracle MLP, the
feature kernel against the feature definition, the inference map, the
fallback to the norm rule, and the label/training pipeline."""
import numpy as np
import pytest

import synth
from _gpu import M, log, torch_cuda

pytestmark = pytest.mark.gpu


def _rand_params(seed, scale=0.3):
    return (synth.normal(seed, 4996) * scale).astype(np.float32)


def test_mlp_grad_matches_oracle(orc):
    torch = torch_cuda()
    mod = M()
    P = _rand_params(3)
    X, y = synth.features_toy(333, 5)
    cw = np.array([1.0, 1.5, 2.0, 0.5])
    m = mod.mpchol_mlp_create()
    try:
        mod.mpchol_mlp_set_params(m, P)
        g = torch.zeros(mod.MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss = mod.mpchol_mlp_grad(m, torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda"), cw, 0.7, g)
        gg = g.cpu().numpy().astype(np.float64)
    finally:
        mod.mpchol_mlp_destroy(m)
    lo, go = orc.mlp_loss_grad(P.astype(np.float64), X.astype(np.float64), y, cw, 0.7)
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    log(f"  grad rel {rel:.2e} loss {loss} vs {lo}")
    assert rel <= 1e-4
    assert abs(loss - lo) <= 1e-5 * abs(lo)


def test_mlp_forward_and_classes(orc):
    torch = torch_cuda()
    mod = M()
    P = _rand_params(8)
    X, _ = synth.features_toy(1000, 9)
    m = mod.mpchol_mlp_create()
    try:
        mod.mpchol_mlp_set_params(m, P)
        logits = torch.zeros((1000, 4), dtype=torch.float32, device="cuda")
        cls = torch.zeros(1000, dtype=torch.int32, device="cuda")
        mod.mpchol_mlp_predict(m, torch.tensor(X, device="cuda"), logits=logits, cls=cls)
        torch.cuda.synchronize()
    finally:
        mod.mpchol_mlp_destroy(m)
    zo = orc.mlp_forward(P.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(logits.cpu().numpy() - zo)) <= 1e-5 * max(1.0, np.max(np.abs(zo)))
    srt = np.sort(zo, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-4
    assert np.array_equal(cls.cpu().numpy()[clear], np.argmax(zo, axis=1)[clear])


def test_adam_steps_match_oracle(orc):
    torch = torch_cuda()
    mod = M()
    P = _rand_params(11, 0.2)
    X, y = synth.features_toy(256, 12)
    cw = np.ones(4)
    m = mod.mpchol_mlp_create()
    try:
        mod.mpchol_mlp_set_params(m, P)
        Xt, yt = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
        for _ in range(3):
            mod.mpchol_mlp_train_step(m, Xt, yt, cw, 0.0, 1e-3, want_loss=False)
        Pg = mod.mpchol_mlp_get_params(m).astype(np.float64)
    finally:
        mod.mpchol_mlp_destroy(m)
    Po = P.astype(np.float64).copy()
    mo, vo = np.zeros_like(Po), np.zeros_like(Po)
    for s in range(1, 4):
        _, g = orc.mlp_loss_grad(Po, X.astype(np.float64), y, cw, 0.0)
        orc.adam_step(Po, g, mo, vo, s, lr=1e-3)
    d_go = np.linalg.norm(Pg - Po) / np.linalg.norm(Po - P)
    log(f"  adam 3 steps: |GPU-oracle| / |step| = {d_go:.2e}")
    assert d_go <= 2e-2


def test_training_reduces_loss():
    import paper_2408_04440_amd.selector as S

    X, y = synth.features_toy(512, 21)
    params, losses = S.train(X, y, steps=300, lr=3e-3, alpha=0.0, log_every=50)
    log(f"  losses {losses}")
    assert losses[-1][1] < 0.3 * losses[0][1]
    acc = np.mean(S.predict(params, X) == y)
    assert acc > 0.9


def test_training_resumes_from_checkpoint_bit_for_bit(tmp_path):
    """20 Adam steps in one run equal 10 steps, a checkpoint through a file
    (weights, both moments, step) and 10 more steps on a fresh trainer, bit
    for bit; the state setter refuses bad moments and sizes."""
    import paper_2408_04440_amd.selector as S

    X, y = synth.features_toy(384, 33)
    p_all, _, st_all = S.train(X, y, steps=20, lr=3e-3, alpha=2.0, return_state=True)
    _, _, st10 = S.train(X, y, steps=10, lr=3e-3, alpha=2.0, return_state=True)
    f = tmp_path / "ck.json"
    S.save(st10[0], str(f), state=st10)
    p_res, _, st_res = S.train(X, y, steps=10, lr=3e-3, alpha=2.0, state=S.load_checkpoint(str(f)),
                               return_state=True)
    assert st10[3] == 10 and st_res[3] == 20 == st_all[3]
    assert np.array_equal(p_res, p_all)
    assert np.array_equal(st_res[1], st_all[1]) and np.array_equal(st_res[2], st_all[2])
    mod = M()
    m = mod.mpchol_mlp_create()
    try:
        bad = st10[2].copy()
        bad[5] = -1.0
        with pytest.raises(mod.MpcholError):
            mod.mpchol_mlp_set_state(m, st10[0], st10[1], bad, 10)
        with pytest.raises(mod.MpcholError):
            mod.mpchol_mlp_set_state(m, st10[0], st10[1], st10[2], -1)
        with pytest.raises(ValueError):
            mod.mpchol_mlp_set_state(m, st10[0][:10], st10[1], st10[2], 10)
    finally:
        mod.mpchol_mlp_destroy(m)


def _features_ref(fro2, amax, tot, eps, n, b):
    nt = fro2.shape[0]
    Lw = int(np.floor(np.sqrt(n - 1))) + 1
    deg = lambda i: int(np.floor(np.sqrt(i)))
    lg = lambda v: max(np.log10(v), -40.0) if v > 0 else -40.0
    F = np.zeros((nt * nt, 8))
    for J in range(nt):
        for I in range(J + 1, nt):
            vj = min(b, n - J * b)
            F[I + J * nt] = [lg(np.sqrt(fro2[I, J]) * nt / (eps * tot)), lg(amax[I, J] * b * nt / (eps * tot)),
                             (I - J) / nt, deg(I * b) / Lw, deg(min((I + 1) * b, n) - 1) / Lw, deg(J * b + vj // 2) / Lw,
                             lg(np.sqrt(fro2[I, I]) / tot), lg(np.sqrt(fro2[J, J]) / tot)]
    return F


def _mlp_map(orc, P, F, nt, band):
    z = orc.mlp_forward(P.astype(np.float64), F)
    cls = np.argmax(z, axis=1)
    srt = np.sort(z, axis=1)
    margin = srt[:, -1] - srt[:, -2]
    m = np.zeros((nt, nt), np.uint8)
    clear = np.ones((nt, nt), bool)
    for J in range(nt):
        for I in range(J + 1, nt):
            t = I + J * nt
            m[I, J] = 0 if I - J <= band else cls[t]
            clear[I, J] = margin[t] > 1e-3
    return m, clear


@pytest.mark.parametrize("L,tile", [(32, 128), (30, 128)])
def test_features_and_learned_map(orc, L, tile):
    n = L * L
    nt = (n + tile - 1) // tile
    eps = 1e-7
    sigma, x = synth.workload(L)
    A = orc.cov_dense(sigma, x, 5.0, 1e-8)
    fro2, amax, tot = orc.tile_norms(A, tile)
    Fr = _features_ref(fro2, amax, tot, eps, n, tile)
    P = _rand_params(40, 0.5)
    mod = M()
    h = mod.mpchol_create(n, tile)
    try:
        mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
        mod.mpchol_precision_map(h, mod.RULE_FP64)
        Fg = mod.mpchol_selector_features(h, eps, nt).astype(np.float64)
        mod.mpchol_selector_set(h, P)
        mg = mod.mpchol_precision_map(h, mod.RULE_LEARNED, eps)
    finally:
        mod.mpchol_destroy(h)
    assert np.max(np.abs(Fg - Fr)) <= 1e-5 * max(1.0, np.max(np.abs(Fr)))
    mo, clear = _mlp_map(orc, P, Fr, nt, 1)
    assert np.array_equal(mg[clear], mo[clear])
    assert np.all(np.diag(mg) == 0) and all(mg[I, I - 1] == 0 for I in range(1, nt))


def test_learned_rule_falls_back_to_norm_rule(orc):
    """Weights that send every tile to FP8 violate the budget; with verify on,
    the factorization is redone under the norm rule and the fallback counted.
    With verify switched off (mpchol_set_verify) the same map is kept, and the
    first verification's backward error is the one the exact residual gives."""
    L, tile = 32, 128
    n = L * L
    sigma, x = synth.workload(L)
    P = np.zeros(4996, np.float32)
    P[-1] = 100.0  # b3 = (0, 0, 0, 100): always class FP8
    mod = M()
    h = mod.mpchol_create(n, tile, verify=1, verify_eps=1e-9)
    try:
        mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
        mod.mpchol_selector_set(h, P)
        mp = mod.mpchol_precision_map(h, mod.RULE_LEARNED, 1e-9)
        assert np.all(mp[np.tril_indices(n // tile, -2)] == 3)
        info = mod.mpchol_factor(h)
        st = mod.mpchol_get_stats(h)
        be = mod.mpchol_backward_error(h)
        # verify off: the all-FP8 map is kept and its error is reported as is
        mod.mpchol_set_verify(h, 0, 1e-9)
        mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
        mod.mpchol_precision_map(h, mod.RULE_LEARNED, 1e-9)
        info0 = mod.mpchol_factor(h)
        st0 = mod.mpchol_get_stats(h)
        be0 = mod.mpchol_backward_error(h) if info0 == 0 else None
        with pytest.raises(Exception):
            mod.mpchol_set_verify(h, 3, 1e-9)
    finally:
        mod.mpchol_destroy(h)
    log(f"  fallback: info={info} fallbacks={st['fallbacks']} rule={st['rule_used']} be={be:.2e} "
        f"first={st['verify_first']:.2e}; verify off: info={info0} be={be0}")
    assert info == 0
    assert st["fallbacks"] >= 1 and st["rule_used"] in (1, 0)
    assert be <= 1e-9
    assert st["verify_first"] > 1e-9          # the learned map's own error, which failed the check
    assert st0["fallbacks"] == 0 and st0["rule_used"] == mod.RULE_LEARNED and st0["verify_first"] == -1.0
    if info0 == 0:
        assert be0 > 1e-9
        assert abs(be0 - st["verify_first"]) <= 1e-6 * be0  # exact residual of the same map, same kernels


def test_labels_train_apply_small(orc):
    """Labels from greedy lowering on small matrices, training on the GPU
    kernels, and the learned map applied to a larger matrix of the same
    family: the result keeps the backward-error budget (after fallback if
    needed) and the gain over the norm rule is reported."""
    import paper_2408_04440_amd.selector as S

    eps = 1e-8
    Xs, ys = [], []
    for (L, tile, rho, seed) in [(24, 128, 5.0, 100), (32, 128, 2.0, 101), (32, 128, 20.0, 102)]:
        X, y, be = S.label_matrix(L, tile, rho, seed, eps)
        log(f"  labels L={L} rho={rho}: hist={np.bincount(y, minlength=4)} verified be={be:.2e}")
        assert be <= eps
        Xs.append(X)
        ys.append(y)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    params, losses = S.train(X, y, steps=400, lr=3e-3, alpha=2.0, log_every=100)
    log(f"  training losses {losses}")
    assert losses[-1][1] < losses[0][1]
    L, tile = 48, 128
    n = L * L
    sigma, x = synth.workload(L, 7)
    mod = M()
    res = {}
    for rule in (mod.RULE_NORM, mod.RULE_LEARNED):
        h = mod.mpchol_create(n, tile, verify=1, verify_eps=eps)
        try:
            mod.mpchol_set_generator(h, sigma, x, 5.0, 1e-8)
            mod.mpchol_selector_set(h, params)
            mp = mod.mpchol_precision_map(h, rule, eps)
            assert mod.mpchol_factor(h) == 0
            st = mod.mpchol_get_stats(h)
            be = mod.mpchol_backward_error(h)
        finally:
            mod.mpchol_destroy(h)
        peaks = np.array([78.6, 157.3, 2500.0, 5000.0])
        model_t = float(np.sum(np.array(st["flops_per_class"]) / peaks))
        res[rule] = (be, model_t, st["fallbacks"], np.bincount(mp[np.tril_indices(n // tile + 1 if n % tile else n // tile, -1)], minlength=4))
        log(f"  rule={rule}: be={be:.2e} modelled time={model_t:.3e} fallbacks={st['fallbacks']} hist={res[rule][3]}")
        assert be <= eps
    gain = res[mod.RULE_NORM][1] / res[mod.RULE_LEARNED][1]
    log(f"  learned vs norm rule modelled speedup: {gain:.3f}")


@pytest.mark.gpu
def test_shipped_weights_gain_on_held_out_matrix(orc):
    """The committed selector weights on a matrix outside their training set
    (band limit 192, seed 11): the learned map passes the estimator check
    without a fallback, keeps the budget under the exact residual, and needs
    less peak-weighted time than the norm rule's map."""
    import paper_2408_04440_amd.selector as S

    eps = 1e-9
    L, tile, rho = 192, 512, 5.0
    n = L * L
    nt = (n + tile - 1) // tile
    sigma, x = synth.workload(L, 11)
    mod = M()
    params = S.load()
    peaks = np.array([78.6, 157.3, 2500.0, 5000.0])
    res = {}
    for rule in (mod.RULE_NORM, mod.RULE_LEARNED):
        h = mod.mpchol_create(n, tile, verify=2, verify_eps=eps)
        try:
            mod.mpchol_set_generator(h, sigma, x, rho, 1e-8)
            mod.mpchol_selector_set(h, params)
            mp = mod.mpchol_precision_map(h, rule, eps)
            assert mod.mpchol_factor(h) == 0
            st = mod.mpchol_get_stats(h)
            be = mod.mpchol_backward_error(h)
        finally:
            mod.mpchol_destroy(h)
        model_t = float(np.sum(np.array(st["flops_per_class"]) / peaks))
        hist = np.bincount(mp[np.tril_indices(nt, -1)], minlength=4)
        res[rule] = (be, model_t, st["fallbacks"], st["t_factor_ms"])
        log(f"  rule={rule}: be={be:.2e} modelled={model_t:.3e} s factor={st['t_factor_ms']:.1f} ms "
            f"fallbacks={st['fallbacks']} verify={st['verify_first']:.2e} hist={hist}")
        assert be <= eps
    assert res[mod.RULE_LEARNED][2] == 0
    gain = res[mod.RULE_NORM][1] / res[mod.RULE_LEARNED][1]
    log(f"  learned vs norm: modelled gain {gain:.3f}, measured factor "
        f"{res[mod.RULE_NORM][3]:.1f} -> {res[mod.RULE_LEARNED][3]:.1f} ms")
    assert gain > 1.0
