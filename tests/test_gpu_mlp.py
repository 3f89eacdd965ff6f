"""The proposal network's GPU kernels (BF16 MFMA, FP32 accumulation) against
the FP64 oracle network, the sampler against the oracle's mixture and
inverse-CDF draws, and the configuration features against an independent
numpy computation.

Tolerances: BF16 operands carry 8 significant bits, so forward outputs and
gradients are compared normwise (relative <= 2e-2, cosine >= 0.999); the
FP32 instantiation of the same kernels to FP32 rounding (relative <= 1e-5);
the
sampler's q is FP64 (relative 1e-12) and its indices are exact except where a
uniform falls within 1e-12 of a CDF boundary."""
import math

import numpy as np
import pytest

import oracle
from oracle import estimators as est
from oracle import mlp as omlp
from workload import synth

pytestmark = pytest.mark.gpu

N_IN, WIDTH = 18, 256


def _net(max_batch=1024):
    import paper_1708_07045_amd as fd
    return fd.Network(N_IN, WIDTH, max_batch)


def _data(B, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, N_IN))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 3] ** 2
    w = rng.uniform(0.5, 2.0, B)
    return X, t, w


def _params(seed=1):
    return omlp.init_params(N_IN, WIDTH, np.random.default_rng(seed))


def test_forward_matches_oracle():
    net = _net()
    p = _params()
    net.set_params(p)
    X, _, _ = _data(700)
    y = net.forward(X).cpu().numpy().astype(np.float64)
    yr = omlp.forward(p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64), N_IN, WIDTH)
    rel = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    assert rel < 2e-2, rel
    assert np.corrcoef(y, yr)[0, 1] > 0.999


def test_params_roundtrip():
    net = _net()
    p = _params(3).astype(np.float32)
    net.set_params(p)
    np.testing.assert_array_equal(net.get_params(), p)
    assert net.n_params == omlp.n_params(N_IN, WIDTH)


@pytest.mark.parametrize("B", [64, 333, 1000])
def test_gradient_matches_oracle(B):
    net = _net()
    p = _params(5)
    net.set_params(p)
    X, t, w = _data(B, seed=B)
    loss, g = net.grad(X, t, w)
    g = g.cpu().numpy().astype(np.float64)
    p64 = p.astype(np.float32).astype(np.float64)
    Lr, gr = omlp.grad(p64, X.astype(np.float32).astype(np.float64), t.astype(np.float32),
                       w.astype(np.float32), N_IN, WIDTH)
    assert loss == pytest.approx(Lr, rel=2e-2)
    cos = g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr))
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    assert cos > 0.999 and rel < 2e-2, (cos, rel)
    # every block of the flat layout, not only the largest
    lay = omlp.unpack(np.arange(p.size, dtype=np.float64), N_IN, WIDTH)
    for W, b in lay:
        for blk in (W.ravel().astype(int), b.astype(int)):
            a, r = g[blk], gr[blk]
            assert np.linalg.norm(a - r) <= 3e-2 * np.linalg.norm(r) + 1e-7


@pytest.mark.parametrize("B", [64, 333])
def test_fp32_instantiation_matches_oracle_to_fp32_rounding(B):
    """The same network with FP32 operands and activations
    (fftdg_mlp_create_ex): forward, loss and gradients against the FP64
    oracle on the same FP32-rounded inputs, normwise relative <= 1e-5 (FP32
    rounding of 256-term products and B-row sums, ~1e-6), every block of the
    layout within 1e-4 of its own norm."""
    import paper_1708_07045_amd as fd
    net = fd.Network(N_IN, WIDTH, 1024, fp32=True)
    p = _params(5)
    net.set_params(p)
    X, t, w = _data(B, seed=B)
    p64 = p.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    y = net.forward(X).cpu().numpy().astype(np.float64)
    yr = omlp.forward(p64, X32, N_IN, WIDTH)
    assert np.linalg.norm(y - yr) <= 1e-5 * np.linalg.norm(yr)
    loss, g = net.grad(X, t, w)
    g = g.cpu().numpy().astype(np.float64)
    Lr, gr = omlp.grad(p64, X32, t.astype(np.float32), w.astype(np.float32), N_IN, WIDTH)
    assert loss == pytest.approx(Lr, rel=1e-5)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    assert rel <= 1e-5, rel
    lay = omlp.unpack(np.arange(p.size, dtype=np.float64), N_IN, WIDTH)
    for W, b in lay:
        for blk in (W.ravel().astype(int), b.astype(int)):
            a, r = g[blk], gr[blk]
            assert np.linalg.norm(a - r) <= 1e-4 * np.linalg.norm(r) + 1e-9 * np.linalg.norm(gr)


def test_skip_connection_matches_oracle():
    """Output net(x) + s x[col]: forward (the skip term exact in FP32, the
    network part to the BF16 tolerance) and gradients over an index subset
    against the FP64 oracle with the same skip; removing the skip restores
    the plain network."""
    net = _net()
    p = _params(9)
    net.set_params(p)
    X, t, w = _data(500, seed=11)
    X[:, 4] *= 40.0  # a skip input far larger than the network's output
    net.set_skip(4, 0.25)
    y = net.forward(X).cpu().numpy().astype(np.float64)
    p64 = p.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    yr = omlp.forward(p64, X32, N_IN, WIDTH, skip=(4, 0.25))
    y0 = omlp.forward(p64, X32, N_IN, WIDTH)
    # the skip part is added in FP32: residual to the oracle is the network's own error
    assert np.linalg.norm((y - yr)) <= 2e-2 * np.linalg.norm(y0)
    idx = np.random.default_rng(12).choice(500, 200, replace=False).astype(np.int32)
    _, g = net.grad(X, t, w, idx)
    _, gr = omlp.grad(p64, X32[idx], t[idx].astype(np.float32), w[idx].astype(np.float32), N_IN, WIDTH,
                      skip=(4, 0.25))
    g = g.cpu().numpy()
    assert np.linalg.norm(g - gr) / np.linalg.norm(gr) < 2e-2
    net.set_skip(-1)
    y1 = net.forward(X).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(y1 - y0) / np.linalg.norm(y0) < 2e-2
    import paper_1708_07045_amd as fd
    with pytest.raises(fd.FFTDGError):
        net.set_skip(N_IN, 1.0)


def test_gradient_with_index_subset():
    net = _net()
    p = _params(6)
    net.set_params(p)
    X, t, w = _data(900, seed=7)
    idx = np.random.default_rng(8).choice(900, 256, replace=False).astype(np.int32)
    _, g = net.grad(X, t, w, idx)
    _, gr = omlp.grad(p.astype(np.float32).astype(np.float64), X[idx].astype(np.float32).astype(np.float64),
                      t[idx].astype(np.float32), w[idx].astype(np.float32), N_IN, WIDTH)
    g = g.cpu().numpy()
    assert np.linalg.norm(g - gr) / np.linalg.norm(gr) < 2e-2


def test_training_reduces_loss():
    import torch
    net = _net(512)
    p = _params(9)
    net.set_params(p)
    X, t, w = _data(4096, seed=11)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), device="cuda").to(dt)
    x_d, t_d, w_d = dev(X, torch.float32), dev(t, torch.float32), dev(np.ones_like(w), torch.float32)
    rng = np.random.default_rng(12)
    L0 = omlp.loss(p.astype(np.float64), X, t, np.ones_like(w), N_IN, WIDTH)
    for epoch in range(15):
        perm = rng.permutation(4096).astype(np.int32)
        for s in range(0, 4096, 512):
            net.train_step(x_d, t_d, w_d, dev(perm[s:s + 512], torch.int32), 1e-3)
    L1 = omlp.loss(net.get_params().astype(np.float64), X, t, np.ones_like(w), N_IN, WIDTH)
    assert L1 < 0.1 * L0, (L0, L1)


@pytest.mark.parametrize("alpha,tau", [(0.1, 1.0), (0.0, 0.5), (1.0, 2.0)])
def test_proposal_sampler_matches_oracle(alpha, tau):
    net = _net()
    rng = np.random.default_rng(13)
    P = 1777
    yhat = (rng.normal(size=P) * 3).astype(np.float32)
    u = synth.uniforms(5, 5000)
    q, idx = net.sample(yhat, alpha, tau, u)
    q = q.cpu().numpy()
    idx = idx.cpu().numpy()
    qr = est.proposal(yhat.astype(np.float64), alpha, tau)
    np.testing.assert_allclose(q, qr, rtol=1e-12, atol=0)
    ir = est.inverse_cdf_sample(qr, u)
    cdf = np.cumsum(qr)
    bad = idx != ir
    if np.any(bad):
        # only where u * total lies within rounding of a CDF boundary
        x = u[bad] * cdf[-1]
        assert np.all(np.min(np.abs(cdf[None, :] - x[:, None]), axis=1) < 1e-12)
    assert np.all((idx >= 0) & (idx < P))


def test_features_match_numpy():
    import paper_1708_07045_amd as fd
    w = synth.config3(n_ligands=3, n_snap=1, cfg_scale=0.01)
    ctx = fd.FFTDG.from_workload(w)
    b = fd.Batch(w.ligands)
    F = ctx.features(b)
    c = 0
    for L in w.ligands:
        for k in range(L.n_cfg):
            q = L.cfg_quat[k] / np.linalg.norm(L.cfg_quat[k])
            q = -q if q[0] < 0 else q
            np.testing.assert_allclose(F[c, :4], q, rtol=1e-6, atol=1e-7)
            oh = np.zeros(8)
            oh[L.cfg_conf[k] % 8] = 1
            np.testing.assert_array_equal(F[c, 4:12], oh)
            assert F[c, 12] == pytest.approx(L.n_atoms / 40, rel=1e-6)
            assert F[c, 13] == pytest.approx(math.log(L.n_atoms) / math.log(40), rel=1e-6)
            u, _ = oracle.place(L.conformers[L.cfg_conf[k]], L.cfg_quat[k], w.h)
            np.testing.assert_allclose(F[c, 14:17], (u.max(axis=0) - 2.0) * w.h / 10.0, rtol=1e-6, atol=1e-6)
            X = L.conformers[L.cfg_conf[k]]
            rg = np.sqrt(np.mean(np.sum((X - X.mean(axis=0)) ** 2, axis=1)))
            assert F[c, 17] == pytest.approx(rg / 5.0, rel=1e-6)
            c += 1
