"""GPU checks of the learned strategy selector.

* The network kernels (forward, masked-MSE backward, Adam) in float32 match
  the float64 oracle within 1e-4 relative (floor 1e-6).
* The feature kernel recovers known properties of synthetic jobs.
* Training with the library's kernels lowers the loss.
* Without weights, LEARNED falls back to the paper-style rule; with the
  committed weights it chooses a feasible container and the output is exact.
"""
import ctypes as C
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def job(torch):
    from paper_1309_0215_amd import Job
    return Job(device=0)


def _close(a, b, rel=1e-4, floor=1e-6):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    assert np.all(np.abs(a - b) <= rel * np.maximum(np.abs(b), floor) + floor), np.max(np.abs(a - b))


def _params(rng):
    return (rng.standard_normal(oracle.MLP_NPARAM) * 0.3).astype(np.float32)


def test_forward_matches_oracle(torch, job):
    rng = np.random.default_rng(0)
    P = _params(rng)
    X = rng.standard_normal((37, 12)).astype(np.float32)
    Pd, Xd = torch.from_numpy(P).cuda(), torch.from_numpy(X).cuda()
    H1, H2, Y = (torch.empty(37, n, device="cuda:0") for n in (64, 64, 4))
    assert job.lib.mr_mlp_forward(job.h, Pd.data_ptr(), Xd.data_ptr(), 37, H1.data_ptr(), H2.data_ptr(), Y.data_ptr()) == 0
    y, (_, z1, h1, z2, h2) = oracle.mlp_forward(P.astype(np.float64), X.astype(np.float64))
    _close(Y.cpu().numpy(), y, rel=1e-4, floor=1e-5)
    _close(H2.cpu().numpy(), h2, rel=1e-4, floor=1e-5)


@pytest.mark.parametrize("B", [1, 64, 200])
def test_backward_matches_oracle(torch, job, B):
    rng = np.random.default_rng(B)
    P = _params(rng)
    X = rng.standard_normal((B, 12)).astype(np.float32)
    T = rng.standard_normal((B, 4)).astype(np.float32)
    M = (rng.random((B, 4)) < 0.7).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    Pd, Xd, Td, Md = d(P), d(X), d(T), d(M)
    H1, H2, Y = (torch.empty(B, n, device="cuda:0") for n in (64, 64, 4))
    G = torch.empty(oracle.MLP_NPARAM, device="cuda:0")
    loss = torch.empty(1, device="cuda:0")
    lib = job.lib
    assert lib.mr_mlp_forward(job.h, Pd.data_ptr(), Xd.data_ptr(), B, H1.data_ptr(), H2.data_ptr(), Y.data_ptr()) == 0
    assert lib.mr_mlp_loss_backward(job.h, Pd.data_ptr(), Xd.data_ptr(), H1.data_ptr(), H2.data_ptr(), Y.data_ptr(),
                                    Td.data_ptr(), Md.data_ptr(), B, loss.data_ptr(), G.data_ptr()) == 0
    l64, g64 = oracle.mlp_grad(P.astype(np.float64), X.astype(np.float64), T.astype(np.float64), M.astype(np.float64))
    _close(loss.item(), l64)
    g = G.cpu().numpy()
    # float32 sums over the batch: relative 1e-4 against the float64 gradient, floor 1e-6 x its scale
    scale = max(1.0, float(np.abs(g64).max()))
    assert np.all(np.abs(g - g64) <= 1e-4 * np.abs(g64) + 1e-6 * scale * np.sqrt(B)), np.max(np.abs(g - g64))


def test_adam_matches_oracle(torch, job):
    rng = np.random.default_rng(3)
    P = _params(rng)
    g = rng.standard_normal(oracle.MLP_NPARAM).astype(np.float32)
    Pd = torch.from_numpy(P.copy()).cuda()
    Gd = torch.from_numpy(g).cuda()
    m = torch.zeros_like(Pd)
    v = torch.zeros_like(Pd)
    th, mm, vv = P.astype(np.float64), np.zeros(oracle.MLP_NPARAM), np.zeros(oracle.MLP_NPARAM)
    for t in (1, 2, 3, 4, 5):
        assert job.lib.mr_mlp_adam(job.h, Pd.data_ptr(), Gd.data_ptr(), m.data_ptr(), v.data_ptr(), t, 1e-3, 0.9, 0.999,
                                   1e-8) == 0
        th, mm, vv = oracle.adam_step(th, g.astype(np.float64), mm, vv, t)
    _close(Pd.cpu().numpy(), th, rel=1e-5, floor=1e-6)


def _features(torch, job, buf, kind, op=0, R=0):
    f = np.zeros(12, np.float32)
    d = torch.from_numpy(buf).cuda()
    assert job.lib.mr_job_features(job.h, kind, op, d.data_ptr(), d.numel(), R, f.ctypes.data_as(C.c_void_p)) == 0
    return f


def test_features_of_known_jobs(torch, job):
    # 100 distinct keys, Zipf(1): top-1 share is 1 / H_100 ~ 0.193
    keys, _ = gen.u32_keys(1, 1 << 20, 100, 1.0)
    f = _features(torch, job, keys.view(np.uint8), 1, 0, 100)
    assert f[0] == pytest.approx(22.0) and f[1] == 0 and f[2] == 1 and f[3] == 0
    assert abs(f[4] - np.log2(100)) < 0.4
    assert abs(f[6] - 1 / np.sum(1.0 / np.arange(1, 101))) < 0.03
    assert f[5] == pytest.approx(1.0, abs=0.25)
    assert f[10] == pytest.approx(np.log2(100))
    # 1M possible keys, uniform: the estimate grows towards the key count
    keys2, _ = gen.u32_keys(2, 1 << 22, 1 << 20, 0.0)
    f2 = _features(torch, job, keys2.view(np.uint8), 1)
    assert 17.5 < f2[4] <= 22.01 and f2[6] < 0.001
    # words: mean length of the generated vocabulary (3..12 letters)
    txt = gen.text(3, 1 << 20, V=5000)
    f3 = _features(torch, job, txt, 0)
    assert f3[1] == 1 and 5.0 < f3[8] < 10.0 and f3[9] > 1.0
    assert abs(f3[4] - np.log2(len(oracle.words(txt)))) < 1.0


def test_training_lowers_loss(torch):
    from paper_1309_0215_amd import selector as S
    rng = np.random.default_rng(7)
    X = rng.standard_normal((300, 12)).astype(np.float32)
    w = rng.standard_normal((12, 4))
    T = np.exp(0.5 * np.tanh(X @ w) + 1.0)
    feas = rng.random((300, 4)) < 0.8
    feas[:, 2] = True
    model, hist = S.train(torch, X, T, feas, epochs=60, batch=64)
    assert hist[-1] < 0.5 * hist[0]


def test_learned_falls_back_to_rule_without_weights(torch):
    from paper_1309_0215_amd import Job
    keys, _ = gen.u32_keys(4, 200_000, 3000, 1.0)
    kt = torch.from_numpy(keys.view(np.int32)).cuda()
    r = Job(device=0, strategy=1).u32(kt, key_range=3000)
    assert r.stats["selector_used"] == 0 and r.stats["strategy_used"] == 2  # the rule: LDS array


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(__file__), "..", "paper_1309_0215_amd",
                                                    "selector_weights.json")), reason="no trained weights committed")
def test_learned_with_weights_is_exact(torch):
    from paper_1309_0215_amd import Job, selector as S
    j = Job(device=0, strategy=1)
    S.load_model(j)
    for seed, (C_, s, R) in enumerate([(5000, 1.2, 0), (1 << 20, 0.3, 1 << 20), (300, 1.0, 300)]):
        keys, vals = gen.u32_keys(30 + seed, 1 << 21, C_, s, with_values=True)
        r = j.u32(torch.from_numpy(keys.view(np.int32)).cuda(), torch.from_numpy(vals.view(np.int32)).cuda(), op=1,
                  key_range=R)
        ek, ev = oracle.u32(keys, vals, "sum")
        assert np.array_equal(r.keys.cpu().numpy().view(np.uint32), ek)
        assert np.array_equal(r.values.cpu().numpy().view(np.uint64), ev)
        assert r.stats["strategy_used"] in (2, 3, 4, 5)
