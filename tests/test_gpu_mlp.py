"""GPU parity of the surrogate network kernels (bfloat16 MFMA, FP32 accumulate)
against the FP64 reference with bfloat16-rounded operands."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
pah = pytest.importorskip("paper_1201_3588_amd.pah")


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("shape,n", [((200, 256, 217), 2048), ((200, 256, 217), 77), ((37, 70, 29), 130)])
def test_forward_backward_match_reference(shape, n):
    ni, nh, no = shape
    rng = np.random.default_rng(3)
    p = omlp.init_params(ni, nh, no, seed=5)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, size=p[k].shape)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    X = rng.normal(size=(n, ni)).astype(np.float32)
    T = rng.normal(size=(n, no)).astype(np.float32)
    net = pah.PahMLP(ni, nh, no, batch=max(n, 64))
    net.load(p)
    Yg = net.forward(torch.as_tensor(X).cuda()).cpu().numpy()
    Yr, cache = omlp.forward(p, X.astype(np.float64), bf16=True)
    assert rel_fro(Yg, Yr) < 1e-4
    net.train_step(torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda(), 0.0, 1)
    torch.cuda.synchronize()
    g = net.grads()
    _, dY = omlp.mse(Yr, T.astype(np.float64))
    gr = omlp.backward(cache, dY, bf16=True)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert rel_fro(g[k], gr[k]) < 2e-4, k
    loss_ref = float(((Yr - T) ** 2).mean())
    assert abs(net.loss() / loss_ref - 1) < 1e-4


def test_adam_step_matches_reference():
    rng = np.random.default_rng(7)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in omlp.init_params(200, 256, 217, seed=1).items()}
    X = rng.normal(size=(512, 200)).astype(np.float32)
    T = rng.normal(size=(512, 217)).astype(np.float32)
    net = pah.PahMLP(batch=512)
    net.load(p)
    net.train_step(torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda(), 1e-3, 1)
    torch.cuda.synchronize()
    g = net.grads()
    new = net.params()
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    ref = {k: val.copy() for k, val in p.items()}
    omlp.adam_step(ref, g, m, v, 1, 1e-3)
    for k in p:
        assert np.max(np.abs(new[k] - ref[k])) <= 1e-6 * max(1.0, np.max(np.abs(ref[k]))), k


def test_training_reduces_loss():
    rng = np.random.default_rng(11)
    ni, nh, no = 32, 64, 16
    Wt = rng.normal(size=(no, ni)) / np.sqrt(ni)
    X = rng.normal(size=(4096, ni)).astype(np.float32)
    T = np.tanh(X @ Wt.T).astype(np.float32)
    net = pah.PahMLP(ni, nh, no, batch=512)
    net.load(omlp.init_params(ni, nh, no, seed=2))
    Xt, Tt = torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda()
    losses = []
    step = 0
    for ep in range(30):
        for b in range(0, 4096, 512):
            step += 1
            net.train_step(Xt[b:b + 512], Tt[b:b + 512], 3e-3, step)
        losses.append(net.loss())
    assert losses[-1] < 0.1 * losses[0]


@pytest.mark.parametrize("nh", [256, 320])
def test_inference_matches_reference(nh):
    # nh = 256 takes the fused on-chip path, nh = 320 the layer-by-layer one
    import oracle
    import synth
    lam = synth.lambda_grid(200)
    pm = synth.pah_model(30, lam)
    solver = pah.PahSolver.from_model(pm)
    ni, no = lam.size + 1, 17 + lam.size
    rng = np.random.default_rng(21)
    p = omlp.init_params(ni, nh, no, seed=8)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, size=p[k].shape)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    net = pah.PahMLP(ni, nh, no, batch=512)
    net.load(p)
    J = synth.pah_fields(1000, lam, seed=23)[0]
    J[::7] *= rng.poisson(3.0, size=J[::7].shape)          # sparse Monte Carlo-like rows
    J[5] = 0.0                                            # a dark cell
    J = J.astype(np.float32)
    # features as the network defines them, from the float32 field
    nu, dnu = oracle.lambda_bins(lam)
    cjd = pm.cabs * J.astype(np.float64) * dnu
    tot = cjd.sum(1)
    pabs_r = 4 * np.pi * tot
    feat = np.hstack([(cjd / np.where(tot > 0, tot, 1.0)[:, None]).astype(np.float32),
                      np.log10(np.maximum(pabs_r, 1e-300)).astype(np.float32)[:, None]])
    x_mu, x_sd = feat.mean(0).astype(np.float32), (feat.std(0) + 1e-3).astype(np.float32)
    Xs = (feat - x_mu) / x_sd
    x_lo, x_hi = np.quantile(Xs, 0.02, axis=0), np.quantile(Xs, 0.98, axis=0)
    y_mu, y_sd = rng.normal(-3.0, 0.5, size=no), rng.uniform(0.05, 0.2, size=no)
    net.set_norm(x_mu, x_sd, x_lo, x_hi, y_mu, y_sd)
    out, ood, pabs = (a.cpu().numpy() for a in net.infer(solver, torch.as_tensor(J).cuda(), 0.5, 0.02))
    assert np.allclose(pabs, pabs_r, rtol=1e-12, atol=0)
    Yr, _ = omlp.forward(p, Xs.astype(np.float64), bf16=True)
    with np.errstate(divide="ignore"):
        Yg = (np.log10(out / np.where(pabs > 0, pabs, 1.0)[:, None]) - y_mu.astype(np.float32)) / y_sd.astype(np.float32)
    lit = pabs > 0
    assert rel_fro(Yg[lit], Yr[lit]) < 1e-4
    assert np.all(out[~lit] == 0.0)
    # range flag: away from the margin it is exactly the reference's
    dist = np.minimum(Xs - (x_lo - 0.5), (x_hi + 0.5) - Xs).min(1)
    clear = (np.abs(dist) > 1e-4) & lit
    assert np.array_equal((ood[clear] & 1) == 1, dist[clear] < 0)
    assert 0.05 < (ood & 1).mean() < 0.95
    # balance flag from the network's own outputs
    ratio = out.sum(1) / np.where(lit, pabs, 1.0)
    far = lit & (np.abs(np.abs(ratio - 1) - 0.02) > 1e-9)
    assert np.array_equal((ood[far] & 2) == 2, np.abs(ratio[far] - 1) > 0.02)
    assert np.all(ood[~lit] == 0)            # a dark cell's answer, zero, is exact


def test_checkpoint_resumes_training_exactly():
    # every training kernel is deterministic, so a network restored from a
    # checkpoint and fed the same batches ends bit-identical to one never stopped
    rng = np.random.default_rng(31)
    ni, nh, no, B = 201, 256, 217, 512
    p = omlp.init_params(ni, nh, no, seed=9)
    batches = [(torch.as_tensor(rng.normal(size=(B, ni)).astype(np.float32)).cuda(),
                torch.as_tensor(rng.normal(size=(B, no)).astype(np.float32)).cuda()) for _ in range(6)]
    a = pah.PahMLP(ni, nh, no, batch=B)
    a.load(p)
    ck = None
    for s, (X, T) in enumerate(batches, start=1):
        a.train_step(X, T, 1e-3, s)
        if s == 3:
            ck = a.checkpoint()
    b = pah.PahMLP(ni, nh, no, batch=B)
    b.restore(ck)
    for s, (X, T) in list(enumerate(batches, start=1))[3:]:
        b.train_step(X, T, 1e-3, s)
    torch.cuda.synchronize()
    n = a.off["X16"]
    assert torch.equal(a.state[:n], b.state[:n])
    Y = batches[0][0][:64]
    assert torch.equal(a.forward(Y), b.forward(Y))
    with pytest.raises(ValueError):
        pah.PahMLP(37, 70, 29, batch=64).restore(ck)
