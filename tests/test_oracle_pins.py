"""Pins for the CPU oracle: it is checked against things other than itself.

* hand-worked cases (tests/golden/words_hand.json),
* library routines that compute the same plain definition by other means
  (bytes.split + collections.Counter, numpy.unique / bincount / add.at,
  scipy's cdist), on seeded random inputs,
* invariants (counts sum to the number of word starts, histogram totals),
* closed forms (k = 1 means column sums; a first Adam step moves each
  parameter by -lr * sign(g); zero weights make the MLP output its bias),
* central finite differences for the MLP gradient.

Each pin is chosen so that a plausible mistake in the oracle (a missing
separator byte, a dropped last word, signed byte order, records not cutting
words, an off-by-one in a reduce op, a wrong sign or transposed weight in the
MLP backward pass) fails at least one test.
"""
import collections
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WS = b" \t\n\x0b\x0c\r"


def _counter_words(buf: bytes, offsets=None):
    """Independent word count: bytes.split() splits on exactly the six ASCII whitespace bytes."""
    if offsets is None:
        recs = [buf]
    else:
        recs = [buf[offsets[i]:offsets[i + 1]] for i in range(len(offsets) - 1)]
    c = collections.Counter()
    for r in recs:
        c.update(r.split())
    return sorted(c.items())


def _word_starts(buf: bytes, offsets=None) -> int:
    """Number of positions where a word begins: a non-separator after a separator or a record start."""
    if offsets is None:
        offsets = [0, len(buf)]
    n = 0
    for r in range(len(offsets) - 1):
        prev_sep = True
        for i in range(offsets[r], offsets[r + 1]):
            s = buf[i] in WS
            if not s and prev_sep:
                n += 1
            prev_sep = s
    return n


def test_bytes_split_uses_the_six_separators():
    # The brute-force pin relies on bytes.split() splitting exactly on these six bytes.
    for b in range(256):
        assert (len(bytes([65, b, 66]).split()) == 2) == (b in WS), b


def test_words_golden_hand_cases():
    with open(os.path.join(GOLDEN, "words_hand.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        buf = np.frombuffer(c["input"].encode("latin-1"), np.uint8)
        offs = None if c["offsets"] is None else np.array(c["offsets"], np.uint64)
        got = oracle.words(buf, offs).items()
        exp = [(k.encode("latin-1"), v) for k, v in c["expect"]]
        assert got == exp, (c["input"], got, exp)


def _random_text(rng, n, alphabet):
    return bytes(rng.choice(alphabet, size=n).astype(np.uint8))


@pytest.mark.parametrize("seed", range(12))
def test_words_brute_force(seed):
    rng = np.random.default_rng(seed)
    # small alphabets give many repeats; include every separator, NUL and high bytes
    alphabet = np.array(list(b"ab") + list(WS) + [0, 0x80, 0xFF, ord("A")])
    n = int(rng.integers(0, 3000))
    buf = _random_text(rng, n, alphabet)
    got = oracle.words(np.frombuffer(buf, np.uint8)).items()
    assert got == _counter_words(buf)
    assert sum(v for _, v in got) == _word_starts(buf)


@pytest.mark.parametrize("seed", range(8))
def test_words_records_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    alphabet = np.array(list(b"abc") + [ord(" "), ord("\n")])
    n = int(rng.integers(1, 2000))
    buf = _random_text(rng, n, alphabet)
    cuts = np.sort(rng.integers(0, n + 1, size=int(rng.integers(1, 40))))
    offs = [int(x) for x in cuts]
    got = oracle.words(np.frombuffer(buf, np.uint8), np.array(offs, np.uint64)).items()
    assert got == _counter_words(buf, offs)
    assert sum(v for _, v in got) == _word_starts(buf, offs)


def test_words_generated_text_matches_counter():
    import gen
    buf = gen.text(11, 1 << 18, V=2000, s=1.0)
    got = oracle.words(buf).items()
    assert got == _counter_words(buf.tobytes())


def test_words_rejects_bad_offsets():
    buf = np.frombuffer(b"abc def", np.uint8)
    with pytest.raises(ValueError):
        oracle.words(buf, np.array([0, 5, 3], np.uint64))
    with pytest.raises(ValueError):
        oracle.words(buf, np.array([0, 8], np.uint64))


@pytest.mark.parametrize("op", ["count", "sum", "min", "max"])
def test_u32_against_numpy(op):
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 300, size=20000).astype(np.uint32)
    keys[:5] = [0, 2**32 - 1, 2**32 - 1, 17, 0]
    vals = rng.integers(0, 2**32, size=20000, dtype=np.uint64).astype(np.uint32)
    k, v = oracle.u32(keys, None if op == "count" else vals, op)
    uk, inv, cnt = np.unique(keys, return_inverse=True, return_counts=True)
    assert np.array_equal(k, uk)
    if op == "count":
        exp = cnt.astype(np.uint64)
        assert int(v.sum()) == len(keys)
    elif op == "sum":
        exp = np.zeros(len(uk), np.uint64)
        np.add.at(exp, inv, vals.astype(np.uint64))
    elif op == "min":
        exp = np.full(len(uk), 2**32, np.uint64)
        np.minimum.at(exp, inv, vals.astype(np.uint64))
    else:
        exp = np.zeros(len(uk), np.uint64)
        np.maximum.at(exp, inv, vals.astype(np.uint64))
    assert np.array_equal(v, exp)


def test_u32_empty():
    k, v = oracle.u32(np.zeros(0, np.uint32))
    assert len(k) == 0 and len(v) == 0


def test_rgb_against_bincount():
    import gen
    buf = gen.rgb(2, 3 * 50001)
    bins = oracle.rgb(buf)
    px = buf.reshape(-1, 3)
    for c in range(3):
        assert np.array_equal(bins[c], np.bincount(px[:, c], minlength=256).astype(np.uint64))
        assert int(bins[c].sum()) == len(px)


def test_rgb_channel_order():
    buf = np.array([1, 2, 3, 1, 1, 1], np.uint8)
    bins = oracle.rgb(buf)
    assert bins[0, 1] == 2 and bins[1, 2] == 1 and bins[1, 1] == 1 and bins[2, 3] == 1 and bins[2, 1] == 1
    assert int(bins.sum()) == 6


def test_kmeans_k1_is_column_sum():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((500, 7)).astype(np.float32)
    a, S, n, newC = oracle.kmeans_step(X, X[:1])
    assert np.all(a == 0) and n[0] == 500
    assert np.allclose(S[0], X.astype(np.float64).sum(0), rtol=0, atol=1e-9)
    assert np.allclose(newC[0], X.astype(np.float64).mean(0), rtol=0, atol=1e-12)


def test_kmeans_identity_assignment():
    rng = np.random.default_rng(4)
    Cn = rng.uniform(-10, 10, (16, 5)).astype(np.float32)
    a, S, n, newC = oracle.kmeans_step(Cn, Cn)
    assert np.array_equal(a, np.arange(16))
    assert np.array_equal(n, np.ones(16))
    assert np.array_equal(newC, Cn.astype(np.float64))


def test_kmeans_ties_take_lowest_index_and_empty_keeps_centroid():
    X = np.array([[0.0, 0.0], [2.0, 0.0]], np.float32)
    Cn = np.array([[1.0, 0.0], [1.0, 0.0], [9.0, 9.0]], np.float32)  # centroids 0 and 1 tie exactly
    a, S, n, newC = oracle.kmeans_step(X, Cn)
    assert list(a) == [0, 0]
    assert list(n) == [2, 0, 0]
    assert np.array_equal(newC[1], Cn[1].astype(np.float64)) and np.array_equal(newC[2], Cn[2].astype(np.float64))


def test_kmeans_against_cdist():
    from scipy.spatial.distance import cdist
    import gen
    X, Cn = gen.kmeans(3, n=2048, d=32, k=64)
    D = cdist(X.astype(np.float64), Cn.astype(np.float64), "sqeuclidean")
    ours = oracle.kmeans_distances(X, Cn)
    assert np.allclose(ours, D, rtol=1e-12, atol=1e-9)
    a = oracle.kmeans_assign(X, Cn)
    assert np.array_equal(a, np.argmin(D, axis=1))
    S, n, newC = oracle.kmeans_update(X, a, Cn)
    onehot = np.zeros((len(X), len(Cn)))
    onehot[np.arange(len(X)), a] = 1
    assert np.allclose(S, onehot.T @ X.astype(np.float64), rtol=1e-12, atol=1e-9)
    assert int(n.sum()) == len(X)


def test_mlp_param_count():
    assert oracle.MLP_NPARAM == 5252


def test_mlp_zero_weights_output_bias():
    theta = np.zeros(oracle.MLP_NPARAM)
    theta[-4:] = [1.5, -2.0, 0.25, 3.0]
    y, _ = oracle.mlp_forward(theta, np.random.default_rng(0).standard_normal((5, 12)))
    assert np.array_equal(y, np.tile([1.5, -2.0, 0.25, 3.0], (5, 1)))


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(oracle.MLP_NPARAM) * 0.3
    X = rng.standard_normal((9, 12))
    T = rng.standard_normal((9, 4))
    M = (rng.random((9, 4)) < 0.7).astype(np.float64)
    loss, g = oracle.mlp_grad(theta, X, T, M)
    assert abs(loss - oracle.mlp_loss(theta, X, T, M)) < 1e-15
    h = 1e-6
    idx = np.concatenate([rng.choice(oracle.MLP_NPARAM, 200, replace=False), np.arange(oracle.MLP_NPARAM - 8, oracle.MLP_NPARAM)])
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (oracle.mlp_loss(tp, X, T, M) - oracle.mlp_loss(tm, X, T, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    # At t = 1 the bias-corrected moments are g and g^2, so the step is -lr * g / (|g| + eps).
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = oracle.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_regret_arithmetic():
    t = np.array([[1.0, 2.0, 4.0, 8.0], [3.0, 1.0, 2.0, 5.0]])
    feas = np.array([[True, True, True, True], [True, False, True, True]])
    r = oracle.regret(t, feas, np.array([1, 2]))
    assert np.allclose(r, [1.0, 0.0])


# ----------------------------------------------------------------------------
# selector network pinned to an independent implementation (torch, float64)
# ----------------------------------------------------------------------------

def _torch_mlp(theta):
    """The same 12-64-64-4 ReLU network built from torch.nn layers, float64."""
    import torch
    p = oracle.mlp_unpack(theta)
    net = torch.nn.Sequential(torch.nn.Linear(12, 64), torch.nn.ReLU(), torch.nn.Linear(64, 64), torch.nn.ReLU(),
                              torch.nn.Linear(64, 4)).double()
    with torch.no_grad():
        for layer, (w, b) in zip((net[0], net[2], net[4]), (("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
            layer.weight.copy_(torch.from_numpy(p[w]))
            layer.bias.copy_(torch.from_numpy(p[b]))
    return net


def test_mlp_forward_matches_torch_layers():
    # Biases are shifted so that about half the hidden pre-activations are
    # negative: a missing, extra or misplaced ReLU changes the output.
    import torch
    rng = np.random.default_rng(11)
    theta = rng.standard_normal(oracle.MLP_NPARAM) * 0.4
    X = rng.standard_normal((33, 12))
    y, (_, z1, _, z2, _) = oracle.mlp_forward(theta, X)
    assert 0.2 < (z1 < 0).mean() < 0.8 and 0.2 < (z2 < 0).mean() < 0.8
    ref = _torch_mlp(theta)(torch.from_numpy(X)).detach().numpy()
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_mlp_forward_hand_worked():
    # One input, weights chosen so that ReLU zeroes a hidden unit in each layer:
    # z1 = [1*2 - 1, -3*2 + 1] = [1, -5] -> h1 = [1, 0]
    # z2 = [2*1 + 0.5, -1*1 - 0.25] = [2.5, -1.25] -> h2 = [2.5, 0]
    # y0 = 4 * 2.5 + 0.1 = 10.1, y3 = -1 * 2.5 + 7 = 4.5
    p = {n: np.zeros(s) for n, s in oracle.MLP_SHAPES}
    p["W1"][0, 0], p["b1"][0] = 1.0, -1.0
    p["W1"][1, 0], p["b1"][1] = -3.0, 1.0
    p["W2"][0, 0], p["b2"][0] = 2.0, 0.5
    p["W2"][1, 0], p["b2"][1] = -1.0, -0.25
    p["W3"][0, 0], p["b3"][0] = 4.0, 0.1
    p["W3"][3, 0], p["b3"][3] = -1.0, 7.0
    p["W3"][1, 1] = 100.0  # reads h2[1], which ReLU zeroes
    p["W2"][0, 1] = 100.0  # reads h1[1], which ReLU zeroes
    theta = np.concatenate([p[n].ravel() for n, _ in oracle.MLP_SHAPES])
    x = np.zeros((1, 12))
    x[0, 0] = 2.0
    y, _ = oracle.mlp_forward(theta, x)
    assert np.allclose(y[0], [10.1, 0.0, 0.0, 4.5], rtol=0, atol=1e-12)


def test_mlp_loss_hand_worked_masked_mean():
    # y = b3 = [1, 2, 3, 4] for both rows (zero weights).
    # Row 0 targets [0, 2, 5, 4], mask [1, 1, 1, 0]: errors 1, 0, 4 (the masked 100 is ignored).
    # Row 1 targets [1, 0, 3, 4], mask [0, 1, 0, 0]: error 4.
    # Loss = (1 + 0 + 4 + 4) / 4 = 2.25.
    theta = np.zeros(oracle.MLP_NPARAM)
    theta[-4:] = [1.0, 2.0, 3.0, 4.0]
    X = np.ones((2, 12))
    T = np.array([[0.0, 2.0, 5.0, 104.0], [1.0, 0.0, 3.0, 4.0]])
    M = np.array([[1.0, 1.0, 1.0, 0.0], [0.0, 1.0, 0.0, 0.0]])
    assert oracle.mlp_loss(theta, X, T, M) == 2.25
    loss, g = oracle.mlp_grad(theta, X, T, M)
    assert loss == 2.25
    # dL/db3 = sum_b 2 m (y - t) / sum m = [2*1/4, 2*(0 + 2)/4, 2*(-2)/4, 0] = [0.5, 1.0, -1.0, 0]
    assert np.allclose(g[-4:], [0.5, 1.0, -1.0, 0.0], rtol=0, atol=1e-15)


def test_mlp_gradient_matches_torch_autograd():
    import torch
    rng = np.random.default_rng(12)
    theta = rng.standard_normal(oracle.MLP_NPARAM) * 0.4
    X = rng.standard_normal((17, 12))
    T = rng.standard_normal((17, 4))
    M = (rng.random((17, 4)) < 0.6).astype(np.float64)
    loss, g = oracle.mlp_grad(theta, X, T, M)
    net = _torch_mlp(theta)
    y = net(torch.from_numpy(X))
    Mt = torch.from_numpy(M)
    tl = (Mt * (y - torch.from_numpy(T)) ** 2).sum() / Mt.sum()
    tl.backward()
    tg = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(), net[2].weight.grad.numpy().ravel(),
                         net[2].bias.grad.numpy(), net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])
    assert abs(loss - float(tl.detach())) < 1e-12
    assert np.allclose(g, tg, rtol=1e-10, atol=1e-12)


def test_adam_matches_torch_optim_over_ten_steps():
    # torch.optim.Adam (bias-corrected, eps added to the corrected root) over
    # steps t = 1..10 with changing gradients: a wrong bias-correction exponent
    # or moment update diverges after the first step.
    import torch
    rng = np.random.default_rng(13)
    th = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.nn.Parameter(torch.from_numpy(th.copy()))
    opt = torch.optim.Adam([p], lr=3e-2, betas=(0.8, 0.95), eps=1e-6)
    for t in range(1, 11):
        g = rng.standard_normal(50) * (1 + t)
        th, m, v = oracle.adam_step(th, g, m, v, t, lr=3e-2, b1=0.8, b2=0.95, eps=1e-6)
        opt.zero_grad()
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        assert np.allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14), t


def test_kmeans_abs_sums_hand_worked():
    # Points (1, -2), (-3, 4), (5, 0.5) in clusters 1, 1, 0 of three:
    # cluster 0: |5| + ... = (5, 0.5); cluster 1: (1 + 3, 2 + 4) = (4, 6); cluster 2: empty.
    X = np.array([[1.0, -2.0], [-3.0, 4.0], [5.0, 0.5]], np.float32)
    A = oracle.kmeans_abs_sums(X, np.array([1, 1, 0]), 3)
    assert np.array_equal(A, np.array([[5.0, 0.5], [4.0, 6.0], [0.0, 0.0]]))
    # and it bounds |S| with equality when all signs agree within a cluster
    S, _, _ = oracle.kmeans_update(X, np.array([1, 1, 0]), np.zeros((3, 2), np.float32))
    assert np.all(np.abs(S) <= A) and S[0, 0] == A[0, 0]
