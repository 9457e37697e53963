"""GPU parity of the learned screen (forward, MSE gradient, Adam) against the
FP64 oracle, and the gain of a trained screen inside the full local energy."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import dev, eloc_complex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_16705_amd as nn
    return nn


def _print_case(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


def _connection_inputs(K, n, seed):
    """``n`` random (x', excitation) pairs from the oracle's enumeration of a
    few samples of an N=2K system, with random regression targets."""
    d = synth.config_inputs(2, K=K, n_up=K // 4, n_dn=K // 4, n_unique=16)
    rng = np.random.default_rng(seed)
    keys, excs = [], []
    for k in rng.choice(len(d["keys"]), size=4, replace=False):
        xp, _, exc, _ = oracle.connections(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], 0.0, d["keys"][k])
        c = rng.choice(len(xp), size=(n + 3) // 4, replace=len(xp) < (n + 3) // 4)
        keys.append(xp[c])
        excs.append(exc[c])
    keys = np.concatenate(keys)[:n]
    excs = np.concatenate(excs)[:n]
    return keys, excs, rng.normal(-6.0, 3.0, size=n)


def _weights(N, H, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 0.15, size=oracle.screen_size(N, H))


@pytest.mark.parametrize("K,H,n", [(24, 256, 300), (24, 40, 37), (12, 16, 1), (60, 256, 129)])
def test_forward_and_gradient_fp64_match_oracle(nn, K, H, n):
    N = 2 * K
    _print_case("screen_fp64", N=N, H=H, n=n)
    keys, exc, target = _connection_inputs(K, n, seed=K + H)
    w = _weights(N, H, seed=n)
    S = nn.Screen(N, H, w)
    pred = S.forward(dev(keys), dev(exc), nn.NNQS_FP64).cpu().numpy()
    ref = oracle.screen_forward(N, H, w, keys, exc)
    assert np.max(np.abs(pred - ref) / np.maximum(1.0, np.abs(ref))) < 1e-12
    g, loss = S.gradient(dev(keys), dev(exc), dev(target), nn.NNQS_FP64)
    oloss, og = oracle.screen_loss_grad(N, H, w, keys, exc, target)
    assert abs(loss.item() - oloss) <= 1e-12 * max(1.0, abs(oloss))
    g = g.cpu().numpy()
    assert np.max(np.abs(g - og)) <= 1e-11 * np.abs(og).max()


@pytest.mark.parametrize("K,H,n", [(24, 256, 300), (24, 40, 37)])
def test_fp32_error_vs_oracle(nn, K, H, n):
    """FP32 training precision: forward within 1e-4 (1 + |y|) and gradient
    within 1e-4 of its largest component, against the FP64 oracle."""
    N = 2 * K
    _print_case("screen_fp32", N=N, H=H, n=n)
    keys, exc, target = _connection_inputs(K, n, seed=3 * K + H)
    w = _weights(N, H, seed=7)
    S = nn.Screen(N, H, w)
    pred = S.forward(dev(keys), dev(exc), nn.NNQS_FP32).cpu().numpy()
    ref = oracle.screen_forward(N, H, w, keys, exc)
    assert np.all(np.abs(pred - ref) <= 1e-4 * (1.0 + np.abs(ref)))
    g, loss = S.gradient(dev(keys), dev(exc), dev(target), nn.NNQS_FP32)
    oloss, og = oracle.screen_loss_grad(N, H, w, keys, exc, target)
    rel = np.max(np.abs(g.cpu().numpy() - og)) / np.abs(og).max()
    print(f"FP32 screen: max fwd err {np.max(np.abs(pred - ref)):.3e}, grad rel {rel:.3e}, "
          f"loss {loss.item():.6g} vs {oloss:.6g}")
    assert rel < 1e-4
    assert abs(loss.item() - oloss) <= 1e-4 * max(1.0, abs(oloss))


def test_adam_steps_match_oracle(nn):
    """Three FP64 gradient + Adam steps on the device against the same three
    steps of the oracle (each side computes its own gradients)."""
    K, H, n = 24, 64, 200
    N = 2 * K
    _print_case("screen_adam", N=N, H=H, n=n)
    keys, exc, target = _connection_inputs(K, n, seed=11)
    w = _weights(N, H, seed=12)
    S = nn.Screen(N, H, w)
    dk, de, dt = dev(keys), dev(exc), dev(target)
    ow, om, ov = w.copy(), np.zeros_like(w), np.zeros_like(w)
    for t in range(1, 4):
        g, _ = S.gradient(dk, de, dt, nn.NNQS_FP64)
        S.adam_step(g, lr=1e-2)
        _, og = oracle.screen_loss_grad(N, H, ow, keys, exc, target)
        oracle.adam_step(ow, og, om, ov, 1e-2, 0.9, 0.999, 1e-8, t)
    gw = S.weights()
    assert np.max(np.abs(gw - ow)) <= 1e-10 * max(1.0, np.abs(ow).max())


@pytest.mark.parametrize("n", [1, 64, 1000])
def test_bf16_inference_error_vs_oracle(nn, n):
    """BF16 inference (FP32 sparse first layer, BF16 MFMA second layer): the
    error against the FP64 oracle is within 0.05 + 0.01 |y| nats, far inside
    the 12-nat skip margin it serves."""
    K, H = 60, 256
    N = 2 * K
    _print_case("screen_bf16", N=N, H=H, n=n)
    keys, exc, _ = _connection_inputs(K, n, seed=n)
    w = _weights(N, H, seed=n + 1)
    S = nn.Screen(N, H, w)
    pred = S.forward(dev(keys), dev(exc), nn.NNQS_BF16).cpu().numpy()
    ref = oracle.screen_forward(N, H, w, keys, exc)
    err = np.abs(pred - ref)
    print(f"BF16 screen n={n}: max err {err.max():.3e} over y range [{ref.min():.3f}, {ref.max():.3f}]")
    assert np.all(err <= 0.05 + 0.01 * np.abs(ref))


@pytest.mark.parametrize("K,nu,nd,cfg", [(24, 6, 6, 2), (60, 20, 20, 3)])
def test_bf16_inference_on_contiguous_runs(nn, K, nu, nd, cfg):
    """Connections in runs of one sample (the layout of the full local
    energy), with run boundaries off the 16-row groups and a sample that
    comes back after another: the first layer is then assembled from the
    sample's sum plus signed flip rows.  The result stays within the BF16
    bound against the FP64 oracle and agrees with the same rows in shuffled
    order (every row assembled from its own bits) to FP32 rounding.  At
    N = 120 the samples' keys fill both 64-bit words (the run's sample is
    compared word by word across the wave)."""
    H = 256
    N = 2 * K
    _print_case("screen_bf16_runs", N=N, H=H)
    d = (synth.config_inputs(2, K=K, n_up=nu, n_dn=nd, n_unique=8) if cfg == 2
         else synth.config_inputs(3, n_unique=8))
    runs = []
    for k, (a, b) in ((0, (5, 700)), (1, (0, 333)), (2, (17, 420)), (1, (333, 900))):
        xp, _, exc, _ = oracle.connections(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], 0.0, d["keys"][k])
        runs.append((xp[a:b], exc[a:b]))
    keys = np.concatenate([r[0] for r in runs])
    exc = np.concatenate([r[1] for r in runs])
    w = _weights(N, H, seed=7)
    S = nn.Screen(N, H, w)
    pred = S.forward(dev(keys), dev(exc), nn.NNQS_BF16).cpu().numpy()
    ref = oracle.screen_forward(N, H, w, keys, exc)
    err = np.abs(pred - ref)
    print(f"BF16 screen runs n={len(keys)}: max err {err.max():.3e} over y range [{ref.min():.3f}, {ref.max():.3f}]")
    assert np.all(err <= 0.05 + 0.01 * np.abs(ref))
    perm = np.random.default_rng(3).permutation(len(keys))
    pred_s = S.forward(dev(keys[perm]), dev(exc[perm]), nn.NNQS_BF16).cpu().numpy()
    assert np.max(np.abs(pred_s - pred[perm])) <= 1e-2


def test_screen_shape_errors(nn):
    w = _weights(24, 40, 0)
    S = nn.Screen(24, 40, w)
    keys, exc, _ = _connection_inputs(12, 8, 0)
    with pytest.raises(nn.NNQSError):  # BF16 inference is built for hidden = 256
        S.forward(dev(keys), dev(exc), nn.NNQS_BF16)
    with pytest.raises(nn.NNQSError):
        S.gradient(dev(keys), dev(exc), dev(np.zeros(8)), nn.NNQS_BF16)
    with pytest.raises(ValueError):
        nn.Screen(24, 40, w[:-1])


def test_trained_screen_cuts_evaluations_within_1e4_ha(nn):
    """N=120 (20 up + 20 down) with the transformer: a screen trained on
    connections of training samples (labels: the network's own BF16
    log|psi(x')|) sends at most half of the connections of held-out samples
    to the network.  With the amplitude-ratio rule at 12 nats the energy
    shift against the unscreened BF16 evaluation is stated; with the
    contribution rule (each skipped term predicted below exp(-18) Ha) it is
    at most 1e-4 Ha."""
    from paper_2306_16705_amd import screen_train
    d = synth.config_inputs(3, n_unique=24)
    _print_case("screen_gain", K=d["K"])
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys = dev(d["keys"])
    cnt = dev(d["counts"], torch.int32)
    xk, ex, lab = screen_train.connection_dataset(S, M, keys[:16], per_sample=8192, seed=1)
    (xk, ex, lab), held = screen_train.split(xk, ex, lab, held_out=0.05, seed=4)
    scr = nn.Screen(d["N"], 256, screen_train.init_weights(d["N"], 256, seed=2))
    losses = screen_train.train(scr, xk, ex, lab, steps=1500, batch=4096, lr=2e-3, seed=3)
    print(f"screen training loss {losses[0]:.4g} -> {np.mean(losses[-20:]):.4g} on {xk.shape[0]} pairs")
    assert np.mean(losses[-20:]) < 0.01 * losses[0]
    tk, tc = keys[16:20].contiguous(), cnt[16:20].contiguous()
    e0, en0, st0 = nn.eloc_model(S, M, tk, tc, nn.NNQS_BF16, with_stats=True)
    torch.cuda.synchronize()
    assert st0["evaluated"] == st0["connections"]
    res = {}
    for rule, thr in [(nn.NNQS_SKIP_RATIO, 12.0), (nn.NNQS_SKIP_CONTRIBUTION, 14.0),
                      (nn.NNQS_SKIP_CONTRIBUTION, 16.0), (nn.NNQS_SKIP_CONTRIBUTION, 18.0),
                      (nn.NNQS_SKIP_CONTRIBUTION, 20.0)]:
        e1, en1, st1 = nn.eloc_model(S, M, tk, tc, nn.NNQS_BF16, with_stats=True, screen=scr, skip_nats=thr,
                                     skip_rule=rule)
        torch.cuda.synchronize()
        de = abs(en1[0].item() - en0[0].item())
        frac = st1["evaluated"] / st1["connections"]
        # required rows: at least one per evaluated x', at most its class
        # blocks (rows from 16 b); each row attends to 1 .. K keys
        K = d["K"]
        blocks = sum(st1["evaluated_class"][b] * (K - 16 * b) for b in range(4))
        assert st1["evaluated"] <= st1["evaluated_rows"] <= blocks
        assert st1["evaluated_rows"] <= st1["evaluated_keys"] <= K * st1["evaluated_rows"]
        per = np.max(np.abs(eloc_complex(e1) - eloc_complex(e0)))
        res[(rule, thr)] = (frac, de)
        print(f"rule {'ratio' if rule == nn.NNQS_SKIP_RATIO else 'contribution'} {thr}: evaluated "
              f"{st1['evaluated']} of {st1['connections']} ({frac:.3f}), |dE| {de:.3e} Ha, "
              f"max per-sample |dE_loc| {per:.3e}")
    # held-out pairs kept out of training: the trained screen passes the
    # 1-nat rule, an untrained one falls back to the plain evaluation
    used, rmse = screen_train.screen_or_plain(scr, *held)
    print(f"held-out RMSE {rmse:.3f} nats")
    assert used is scr
    raw = nn.Screen(d["N"], 256, screen_train.init_weights(d["N"], 256, seed=5))
    assert screen_train.screen_or_plain(raw, *held)[0] is None
    frac, de = res[(nn.NNQS_SKIP_RATIO, 12.0)]
    assert frac < 0.5 and de < 0.05
    frac, de = res[(nn.NNQS_SKIP_CONTRIBUTION, 18.0)]
    assert frac < 0.5
    assert de <= 1e-4


def test_fallback_judge_matches_the_forward(nn):
    """nnqs_screen_judge: RMSE of the screen's own BF16 and FP64 predictions
    against targets, and the usable flag on both sides of the threshold."""
    d = synth.config_inputs(2, n_unique=8)
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    con = nn.connections(S, dev(d["keys"][:2]))
    xk = con["xprime"].reshape(-1, 2)[:3001].contiguous()
    ex = con["exc"].reshape(-1, 4)[:3001].contiguous()
    from paper_2306_16705_amd import screen_train
    scr = nn.Screen(d["N"], 256, screen_train.init_weights(d["N"], 256, seed=5))
    rng = np.random.default_rng(3)
    target = torch.from_numpy(rng.normal(0.0, 2.0, size=3001)).cuda()
    for prec in (nn.NNQS_BF16, nn.NNQS_FP64):
        pred = scr.forward(xk, ex, prec).cpu().numpy()
        want = float(np.sqrt(np.mean((pred - target.cpu().numpy()) ** 2)))
        rmse, ok = scr.judge(xk, ex, target, prec, max_rmse=want * 1.001)
        assert abs(rmse - want) <= 1e-12 * want and ok
        rmse2, ok2 = scr.judge(xk, ex, target, prec, max_rmse=want * 0.999)
        assert rmse2 == rmse and not ok2


def test_kernel_timing_records_launches(nn):
    d = synth.config_inputs(2, K=12, n_up=3, n_dn=3, n_unique=40, model=True)
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys = dev(d["keys"])
    nn.timing_enable(True)
    nn.model_logpsi(M, keys, nn.NNQS_BF16)
    nn.model_logpsi(M, keys, nn.NNQS_BF16)
    ms, cnt = nn.timing_read("k_transformer_bf16")
    nn.timing_enable(False)
    assert cnt == 2 and ms > 0.0
    assert nn.timing_read("k_transformer_bf16") == (0.0, 0)


@pytest.mark.parametrize("n", [64, 1000])
def test_fp8_inference_error_vs_oracle(nn, n):
    """FP8 rung of the screen: the hidden layer on v_mfma_f32_16x16x32_fp8_fp8
    (OCP E4M3 activations, W2 with a power-of-two scale), the rest as BF16.
    The error against the FP64 oracle is stated and bounded by
    0.25 + 0.03 |y| nats (E4M3 keeps 3 mantissa bits)."""
    K, H = 60, 256
    N = 2 * K
    _print_case("screen_fp8", N=N, H=H, n=n)
    keys, exc, _ = _connection_inputs(K, n, seed=n)
    w = _weights(N, H, seed=n + 1)
    S = nn.Screen(N, H, w)
    pred = S.forward(dev(keys), dev(exc), nn.NNQS_FP8).cpu().numpy()
    p16 = S.forward(dev(keys), dev(exc), nn.NNQS_BF16).cpu().numpy()
    ref = oracle.screen_forward(N, H, w, keys, exc)
    err, e16 = np.abs(pred - ref), np.abs(p16 - ref)
    print(f"FP8 screen n={n}: max err {err.max():.3e} (BF16 {e16.max():.3e}), RMS {np.sqrt(np.mean(err ** 2)):.3e} "
          f"over y range [{ref.min():.3f}, {ref.max():.3f}]")
    assert np.all(err <= 0.25 + 0.03 * np.abs(ref))


def test_screen_save_load_round_trip(nn, tmp_path):
    """Screen weights persist through a safetensors file bit for bit."""
    N, H = 48, 32
    rng = np.random.default_rng(12)
    w = rng.normal(0.0, 0.1, size=int(oracle.screen_size(N, H)))
    s1 = nn.Screen(N, H, w)
    path = str(tmp_path / "screen.safetensors")
    s1.save(path)
    s2 = nn.Screen.load(path)
    assert (s2.n_spin_orb, s2.hidden) == (N, H)
    assert np.array_equal(s2.weights(), s1.weights())


def test_screen_training_resumes_from_a_checkpoint(nn, tmp_path):
    """Weights and Adam state (both moments, the step count) saved after some
    steps and loaded into a new screen: the next steps of the two screens
    agree bit for bit, and a screen loaded without the state (fresh moments)
    does not."""
    N, H = 48, 32
    rng = np.random.default_rng(13)
    cnt = int(oracle.screen_size(N, H))
    s1 = nn.Screen(N, H, rng.normal(0.0, 0.1, size=cnt))
    grads = [torch.tensor(rng.normal(0.0, 1.0, size=cnt), device="cuda") for _ in range(6)]
    for g in grads[:3]:
        s1.adam_step(g, lr=1e-3)
    m, v, t = s1.state()
    assert t == 3 and np.all(v > 0.0)
    path = str(tmp_path / "screen_ckpt.safetensors")
    s1.save(path)
    s2 = nn.Screen.load(path)
    m2, v2, t2 = s2.state()
    assert t2 == 3 and np.array_equal(m2, m) and np.array_equal(v2, v)
    s3 = nn.Screen(N, H, s1.weights())  # weights only: moments restart at zero
    for g in grads[3:]:
        s1.adam_step(g, lr=1e-3)
        s2.adam_step(g, lr=1e-3)
        s3.adam_step(g, lr=1e-3)
    assert np.array_equal(s2.weights(), s1.weights())
    assert not np.array_equal(s3.weights(), s1.weights())
    with pytest.raises(nn.NNQSError):
        s2.set_state(m, v, -1)


def test_screened_bf16_path_replays_from_a_hip_graph(nn):
    """Without FP64 refinement, validation or statistics the screened BF16
    full path makes no host synchronisation once its scratch is grown, so it
    can be captured into a graph: every replay, with eager work between the
    replays, reproduces the eager local energies and energy bit for bit."""
    from paper_2306_16705_amd import screen_train
    d = synth.config_inputs(2, K=16, n_up=4, n_dn=4, n_unique=24, model=True)
    _print_case("screened_graph", K=d["K"])
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    scr = nn.Screen(d["N"], 256, screen_train.init_weights(d["N"], 256, seed=2))
    keys, cnt = dev(d["keys"]), dev(d["counts"], torch.int32)
    n = keys.shape[0]
    eloc = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    energy = torch.empty(4, dtype=torch.float64, device="cuda")
    kw = dict(eloc=eloc, energy=energy, screen=scr, skip_nats=14.0, skip_rule=nn.NNQS_SKIP_CONTRIBUTION)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(2):  # grows every scratch buffer before the capture
            nn.eloc_model(S, M, keys, cnt, nn.NNQS_BF16, stream=s, **kw)
    s.synchronize()
    ref, ref_en = eloc.clone(), energy.clone()
    assert torch.isfinite(ref).all()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        nn.eloc_model(S, M, keys, cnt, nn.NNQS_BF16, stream=s, **kw)
    for rep in range(3):
        eloc.fill_(float("nan"))  # eager work between replays
        energy.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(eloc, ref), rep
        assert torch.equal(energy, ref_en), rep
