"""Pins of the FP64 screen oracle: forward, loss gradient and Adam step against
central finite differences and PyTorch FP64 library routines (autograd,
torch.optim.Adam)."""
import numpy as np
import torch
import torch.nn.functional as F

import oracle
import synth


def _data(N=12, n=24, seed=0):
    d = synth.config_inputs(1, K=N // 2, n_up=2, n_dn=2)
    rng = np.random.default_rng(seed)
    keys, excs = [], []
    for k in rng.choice(len(d["keys"]), size=n):
        xp, _, exc, _ = oracle.connections(d["K"], 2, 2, d["h"], d["g"], 0.0, d["keys"][k])
        c = rng.integers(len(xp))
        keys.append(xp[c])
        excs.append(exc[c])
    return np.array(keys, np.uint64), np.array(excs, np.uint8), rng.normal(size=n)


def _weights(N, H, seed=1):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 0.3, size=oracle.screen_size(N, H))


def _torch_forward(N, H, w, keys, exc):
    w = torch.tensor(w, requires_grad=True)
    o = 0
    W1 = w[o:o + 5 * N * H].view(5 * N, H); o += 5 * N * H
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].view(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    w3 = w[o:o + H]; o += H
    b3 = w[o]
    occ = synth.unpack_keys(keys, N // 2)
    u = np.zeros((len(keys), 5 * N))
    u[:, 0:N:2] = occ[:, 0]
    u[:, 1:N:2] = occ[:, 1]
    for t in range(4):
        for r, e in enumerate(exc[:, t]):
            if e != 255:
                u[r, (t + 1) * N + e] = 1.0
    u = torch.tensor(u)
    y = F.gelu(F.gelu(u @ W1 + b1) @ W2 + b2) @ w3 + b3
    return w, y


def test_forward_and_gradient_match_autograd():
    N, H = 12, 16
    keys, exc, target = _data(N)
    w = _weights(N, H)
    pred = oracle.screen_forward(N, H, w, keys, exc)
    wt, y = _torch_forward(N, H, w, keys, exc)
    assert np.max(np.abs(pred - y.detach().numpy())) < 1e-12
    loss, g = oracle.screen_loss_grad(N, H, w, keys, exc, target)
    tl = torch.mean((y - torch.tensor(target)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-12
    assert np.max(np.abs(g - wt.grad.numpy())) < 1e-12 * max(1.0, np.abs(g).max())


def test_gradient_matches_central_differences():
    N, H = 12, 8
    keys, exc, target = _data(N, n=10, seed=3)
    w = _weights(N, H, seed=4)
    _, g = oracle.screen_loss_grad(N, H, w, keys, exc, target)
    rng = np.random.default_rng(5)
    idx = rng.choice(w.size, size=60, replace=False)
    eps = 1e-5
    for q in idx:
        wp, wm = w.copy(), w.copy()
        wp[q] += eps
        wm[q] -= eps
        fd = (oracle.screen_loss_grad(N, H, wp, keys, exc, target)[0] -
              oracle.screen_loss_grad(N, H, wm, keys, exc, target)[0]) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1e-3, abs(g[q])) + 1e-9, (q, fd, g[q])


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(7)
    w = rng.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    wt = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        oracle.adam_step(w, g, m, v, 1e-2, 0.9, 0.999, 1e-8, t)
        wt.grad = torch.tensor(g)
        opt.step()
    assert np.max(np.abs(w - wt.detach().numpy())) < 1e-12
