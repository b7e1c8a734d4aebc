"""Retraining parity: hand-written NLL backward (GPU) vs FP64 finite differences of the
oracle loss, vs PyTorch FP64 autograd of a from-scratch loss, and Adam vs torch.optim.Adam."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stack():
    return synth.mri_stack(2000, 16)


def _weights(seed=3, width=64):
    w = synth.xavier_mlp((12, width, width, 15), seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3"):
        w[k] = rng.normal(0, 0.1, w[k].shape).astype(np.float32)
    return w


def _torch_loss(w, stack, idx):
    """Mean mixture NLL in bits written with PyTorch FP64 ops (library reference)."""
    T = {k: torch.from_numpy(np.asarray(v, np.float64)).requires_grad_(True) for k, v in w.items()}
    feats = torch.from_numpy(oracle.sample_features(stack, idx))
    tgt = torch.from_numpy(stack[idx[:, 0], idx[:, 1], idx[:, 2]].astype(np.int64))
    h = torch.relu(feats @ T["W1"].T + T["b1"])
    h = torch.relu(h @ T["W2"].T + T["b2"])
    o = h @ T["W3"].T + T["b3"]
    logit, mu, ls = o[:, 0:5], o[:, 5:10], torch.clamp(o[:, 10:15], min=-7.0)
    inv_s = torch.exp(-ls)
    v = tgt[:, None].double()
    hi = (2 * v + 1) / 255 - 1
    lo = (2 * v - 1) / 255 - 1
    A = (hi - mu) * inv_s
    B = (lo - mu) * inv_s
    sp = torch.nn.functional.softplus
    interior = -sp(-A) - sp(B) + torch.log(-torch.expm1(B - A))
    lp = torch.where(v == 0, -sp(-A), torch.where(v == 255, -sp(B), interior))
    LP = torch.logsumexp(torch.log_softmax(logit, dim=1) + lp, dim=1)
    loss = -LP.mean() / math.log(2)
    loss.backward()
    return loss.item(), {k: T[k].grad.numpy() for k in dl.PARAM_NAMES}


def _split(flat, h):
    out, off = {}, 0
    for k, shp in dl.param_shapes(h, h).items():
        n = int(np.prod(shp))
        out[k] = flat[off:off + n].reshape(shp)
        off += n
    return out


def _run(dev, w, stack, idx, dtype):
    m = dl.TrainModel(w, dev, dtype)
    loss, grad = dl.nll(m, to_dev(stack, dev), to_dev(idx, dev))
    torch.cuda.synchronize()
    return float(loss.item()), _split(grad.cpu().numpy().astype(np.float64), w["W1"].shape[0])


def test_fp64_gradient_matches_central_differences(dev, stack):
    """Every bias and 512 seeded weights (spread over the three matrices by size) against
    FP64 central differences (h = 1e-6): per tensor normwise below 1e-5, and elementwise
    within 1e-5 relative plus the quotient's own rounding error, 8 eps |L| / h (the two
    loss values carry a few ulps of |L| each), wherever the quotient is at least 1e-3 of
    the tensor's largest."""
    w = _weights()
    idx = synth.train_indices(0, 512, len(stack), 256, 256)
    say("nll fp64 vs finite differences")
    loss, g = _run(dev, w, stack, idx, torch.float64)
    assert abs(loss - oracle.nll_bits(w, stack, idx)) < 1e-12 * max(1, loss)
    rng = np.random.default_rng(0)
    picks = [(k, i) for k in ("b1", "b2", "b3") for i in range(w[k].size)]
    sizes = {k: w[k].size for k in ("W1", "W2", "W3")}
    total = sum(sizes.values())
    counts = {k: max(16, int(round(512 * n / total))) for k, n in sizes.items()}
    counts["W2"] += 512 - sum(counts.values())
    for k, c in counts.items():
        picks += [(k, int(i)) for i in rng.choice(sizes[k], c, replace=False)]
    assert len(picks) == 143 + 512
    _, fd = oracle.nll_and_grad_fd(w, stack, idx, picks, h=1e-6)
    gpu = np.array([g[k].reshape(-1)[i] for k, i in picks])
    for name in dl.PARAM_NAMES:
        sel = np.array([k == name for k, _ in picks])
        err = np.linalg.norm(gpu[sel] - fd[sel]) / max(np.linalg.norm(fd[sel]), 1e-30)
        assert err < 1e-5, (name, err)
        big = np.abs(fd[sel]) >= 1e-3 * np.abs(fd[sel]).max()
        a, b = gpu[sel][big], fd[sel][big]
        fd_round = 8 * np.finfo(np.float64).eps * max(abs(loss), 1.0) / 1e-6
        excess = np.abs(a - b) - (1e-5 * np.abs(b) + fd_round)
        worst = int(np.argmax(excess))
        assert big.any() and excess.max() <= 0, (name, a[worst], b[worst], fd_round)


def test_fp32_gradient_matches_torch_fp64_autograd(dev, stack):
    w = _weights()
    # the training workload's batch: 2^20 windows
    idx = synth.train_indices(1, 1 << 20, len(stack), 256, 256)
    say("nll fp32 vs torch fp64 autograd")
    loss, g = _run(dev, w, stack, idx, torch.float32)
    ref_loss, ref = _torch_loss(w, stack, idx)
    assert abs(loss - ref_loss) < 1e-5 * ref_loss
    for k in dl.PARAM_NAMES:
        err = np.linalg.norm(g[k] - ref[k]) / np.linalg.norm(ref[k])
        assert err < 1e-5, (k, err)
    # softmax gauge: logit gradients of every sample sum to zero
    assert abs(g["b3"][0:5].sum()) < 1e-6 * np.abs(g["b3"]).sum() + 1e-9
    assert np.abs(g["W3"][0:5].sum(axis=0)).max() < 1e-6 * np.abs(g["W3"]).max() + 1e-9


def test_autograd_function_and_adam(dev, stack):
    w = _weights()
    idx = to_dev(synth.train_indices(2, 4096, len(stack), 256, 256), dev)
    sl = to_dev(stack, dev)
    P = {k: torch.from_numpy(w[k]).to(dev).requires_grad_(True) for k in dl.PARAM_NAMES}
    loss = dl.DLICNLL().apply(*[P[k] for k in dl.PARAM_NAMES], sl, idx)
    (2.0 * loss).backward()
    m = dl.TrainModel(w, dev)
    _, grad = dl.nll(m, sl, idx)
    g = _split(grad.cpu().numpy(), 64)
    for k in dl.PARAM_NAMES:
        assert np.allclose(P[k].grad.cpu().numpy(), 2.0 * g[k], rtol=1e-6, atol=0)
    # Adam on the flat buffer vs the oracle's FP64 Adam (pinned against torch.optim.Adam)
    p64 = m.flat.detach().cpu().numpy().astype(np.float64)
    m64 = np.zeros_like(p64)
    v64 = np.zeros_like(p64)
    mm = torch.zeros_like(m.flat)
    vv = torch.zeros_like(m.flat)
    for step in range(1, 4):
        _, grad = dl.nll(m, sl, idx)
        p64, m64, v64 = oracle.adam_update(p64, grad.cpu().numpy().astype(np.float64), m64, v64,
                                           step)
        dl.dlic_adam_step(m.flat.numel(), m.flat, grad, mm, vv, step)
        torch.cuda.synchronize()
        got = m.flat.detach().cpu().numpy().astype(np.float64)
        assert np.allclose(got, p64, rtol=1e-6, atol=1e-9), step
        # the FP32 kernel keeps the parameters at FP32 rounding of the FP64 update
        p64 = got
