"""Warm-start network on the GPU against the FP64 reference (oracle.mlp)."""

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _bf16_tensor(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).cuda()


def test_features_match_reference(gpu, synth_lib):
    from paper_2411_10258_amd import surrogate
    b = synth_lib.batch_m16(W=64)
    print("[surrogate] features", flush=True)
    x = surrogate.features(b.offsets, b.t, b.dim, b.T, 16).float().cpu().numpy()
    ref = mlp.features(b.offsets, b.t, b.dim, b.T, 16)
    # FP32 log1p on the GPU vs FP64 here: at most one BF16 step apart.
    assert np.all(np.abs(x - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-30)
    assert np.mean(x == ref) > 0.99


def _net(gpu, seed=3, max_batch=256, M=16):
    from paper_2411_10258_amd import surrogate
    return surrogate.Surrogate(M, hidden=512, max_batch=max_batch, seed=seed)


@pytest.mark.parametrize("M", [16, 64])
def test_forward_matches_reference(gpu, M):
    import torch
    net = _net(gpu, M=M)
    rng = np.random.default_rng(0)
    B = 200 if M == 16 else 72  # ragged against the 64-row tiles
    x = mlp.bf16(np.abs(rng.standard_normal((B, net.in_dim))))
    print("[surrogate] forward", flush=True)
    y = net.forward(_bf16_tensor(x)).cpu().numpy()
    w = net.get_weights().cpu().numpy()
    params = mlp.unpack(w, net.in_dim, net.hidden, net.out_dim)
    h1r, h2r, yr = mlp.forward(x, params)
    h1, h2 = (h.float().cpu().numpy() for h in net.get_hidden(B))
    # Hidden activations: the same BF16 value except where FP32 vs FP64
    # accumulation straddles a rounding boundary (one BF16 step).
    assert np.mean(h1 == h1r) > 0.97 and np.all(np.abs(h1 - h1r) <= 2 ** -7 * np.abs(h1r) + 1e-6)
    assert np.mean(h2 == h2r) > 0.97
    scale = np.abs(h2r) @ np.abs(mlp.bf16(params[4])).T + np.abs(params[5])
    assert np.all(np.abs(y - yr) <= 1e-2 * scale + 1e-6)
    net.close()


def test_backward_matches_reference(gpu):
    import torch
    net = _net(gpu, seed=5)
    rng = np.random.default_rng(1)
    B = 128
    x = mlp.bf16(np.abs(rng.standard_normal((B, net.in_dim))))
    t = rng.standard_normal((B, net.out_dim)).astype(np.float32)
    print("[surrogate] backward", flush=True)
    loss = net.backward(_bf16_tensor(x), torch.from_numpy(t).cuda())
    g = net.get_gradients().cpu().numpy().astype(np.float64)
    w = net.get_weights().cpu().numpy()
    params = mlp.unpack(w, net.in_dim, net.hidden, net.out_dim)
    loss_r, g_r = mlp.backward(x, t.astype(np.float64), params)
    assert float(loss.item()) == pytest.approx(loss_r, rel=1e-3)
    gs = mlp.unpack(g, net.in_dim, net.hidden, net.out_dim)
    grs = mlp.unpack(g_r, net.in_dim, net.hidden, net.out_dim)
    for a, r in zip(gs, grs):
        assert np.linalg.norm(a - r) <= 2e-2 * np.linalg.norm(r) + 1e-12
    net.close()


def test_training_reduces_loss(gpu):
    import torch
    net = _net(gpu, seed=7, max_batch=256)
    rng = np.random.default_rng(2)
    N = 4096
    x = np.abs(rng.standard_normal((N, net.in_dim))).astype(np.float32)
    proj = rng.standard_normal((net.in_dim, net.out_dim)) / np.sqrt(net.in_dim)
    y = np.tanh(x @ proj).astype(np.float32)
    print("[surrogate] training", flush=True)
    losses = net.train(_bf16_tensor(x), torch.from_numpy(y).cuda(), epochs=6, lr=1e-3)
    assert losses[-1] < 0.5 * losses[0]
    w = net.get_weights()
    net.set_weights(w * 0.0)
    assert float(net.forward(_bf16_tensor(x[:8])).abs().max()) == 0.0
    net.close()


def test_warm_start_falls_back_to_cold(gpu, oracle_lib, synth_lib):
    import torch
    from paper_2411_10258_amd import surrogate
    b = synth_lib.batch_m16(W=32)
    M = 16
    net = _net(gpu, seed=9, max_batch=64)
    x = surrogate.features(b.offsets, b.t, b.dim, b.T, M)
    # Targets at the truth for even windows; nonsense (huge alpha) for odd ones.
    y = surrogate.log_targets(M, b.mu, b.alpha, b.beta,
                              surrogate.dim_counts(b.offsets, b.dim, M), b.T)
    stats = surrogate.TargetStats.fit(y)
    pred_true = torch.from_numpy(stats.normalize(y)).cuda()
    plan = gpu.Plan(b.offsets, b.t, b.dim, b.T, M, 0)
    mu_c = np.full((b.W, M), 0.2, np.float32)
    al_c = np.full((b.W, M, M), 0.01, np.float32)
    be_c = np.ones(b.W, np.float32)
    # Feed the prediction directly by setting the net to zero and the stats
    # so that exp(0 * std + mean) reproduces chosen values is awkward; call
    # the C entry with a handmade prediction instead.
    import ctypes
    from paper_2411_10258_amd import _lib
    from paper_2411_10258_amd.api import _ptr
    pred = pred_true.clone()
    bad = np.arange(b.W) % 2 == 1
    pred[torch.from_numpy(bad).cuda(), M:M + M * M] = 50.0  # 50 std + mean: explosive alpha
    mean = torch.from_numpy(stats.mean).cuda()
    std = torch.from_numpy(stats.std).cuda()
    mu = torch.empty(b.W, M, device="cuda")
    alpha = torch.empty(b.W, M, M, device="cuda")
    beta = torch.empty(b.W, device="cuda")
    used = torch.empty(b.W, dtype=torch.int32, device="cuda")
    opts = gpu.FitOptions().to_c()
    tmc, tac, tbc = (torch.from_numpy(v).cuda() for v in (mu_c, al_c, be_c))
    print("[surrogate] warm start", flush=True)
    _lib.check(_lib.load().mdhp_warm_start(ctypes.c_void_p(plan.handle), _ptr(pred), _ptr(mean),
                                           _ptr(std), ctypes.byref(opts), _ptr(tmc), _ptr(tac),
                                           _ptr(tbc), _ptr(mu), _ptr(alpha), _ptr(beta),
                                           _ptr(used), None))
    torch.cuda.synchronize()
    used = used.cpu().numpy()
    assert np.all(used[bad] == 0)
    assert np.all(used[~bad] == 1)
    assert np.allclose(alpha.cpu().numpy()[bad], al_c[bad])
    # The warm windows start at the truth.
    assert np.allclose(alpha.cpu().numpy()[~bad], b.alpha[~bad], rtol=1e-4, atol=1e-6)
    assert np.allclose(mu.cpu().numpy()[~bad], b.mu[~bad], rtol=1e-4)
    assert np.allclose(beta.cpu().numpy()[~bad], b.beta[~bad], rtol=1e-4)
    plan.close()
    net.close()


def test_checkpoint_round_trip(gpu, tmp_path):
    """save/load restores weights, both Adam moments and the step: the next
    training step of the restored network gives bitwise the original's
    weights."""
    import torch
    from paper_2411_10258_amd import _lib, surrogate
    rng = np.random.default_rng(4)
    a = _net(gpu, seed=5, max_batch=64)
    x = _bf16_tensor(np.abs(rng.standard_normal((64, a.in_dim))))
    t = torch.from_numpy(rng.standard_normal((64, a.out_dim)).astype(np.float32)).cuda()
    print("[surrogate] checkpoint", flush=True)
    for _ in range(3):
        a.train_step(x, t, 1e-3)
    a.stats = surrogate.TargetStats(rng.standard_normal(a.out_dim).astype(np.float32),
                                    rng.uniform(0.5, 2, a.out_dim).astype(np.float32))
    path = str(tmp_path / "net.ckpt")
    a.save(path)
    b = _net(gpu, seed=99, max_batch=64)
    assert not torch.equal(a.get_weights(), b.get_weights())
    b.load(path)
    assert torch.equal(a.get_weights(), b.get_weights())
    assert np.array_equal(a.stats.mean, b.stats.mean) and np.array_equal(a.stats.std, b.stats.std)
    la = a.train_step(x, t, 1e-3).item()
    lb = b.train_step(x, t, 1e-3).item()
    torch.cuda.synchronize()
    # the step's weights are bitwise equal; the reported loss is an FP64
    # atomic sum over the batch, equal up to its summation order
    assert torch.equal(a.get_weights(), b.get_weights())
    assert abs(la - lb) <= 1e-12 * abs(la)
    assert torch.equal(a.get_weights(), b.get_weights())
    # Another shape, a foreign file, a truncated file, a missing file.
    c = surrogate.Surrogate(16, hidden=256, max_batch=8, seed=1)
    with pytest.raises(gpu.MdhpError) as e:
        c.load(path)
    assert e.value.status == -1
    bad = tmp_path / "foreign.bin"
    bad.write_bytes(b"not a checkpoint" * 8)
    with pytest.raises(gpu.MdhpError) as e:
        b.load(str(bad))
    assert e.value.status == -7
    cut = tmp_path / "cut.ckpt"
    cut.write_bytes(open(path, "rb").read()[:1000])
    with pytest.raises(gpu.MdhpError) as e:
        b.load(str(cut))
    assert e.value.status == -7
    with pytest.raises(gpu.MdhpError) as e:
        b.load(str(tmp_path / "missing.ckpt"))
    assert e.value.status == -7
    for n in (a, b, c):
        n.close()
