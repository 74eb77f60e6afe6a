"""GPU parity of one k-means step (MR_MAP_KMEANS) against the float64 oracle.

Tolerances (float32 arithmetic on the GPU, float64 in the oracle):
* assignment a_i is accepted iff d64(a_i) <= d64_min * (1 + 1e-6) + 1e-12
  (ties within 1e-6 relative may go either way);
* counts are exact given the GPU's assignments;
* sums: |s32 - s64| <= 1e-5 * max(|s64|, sum_i |x_id|) per (cluster, dim),
  s64 recomputed in float64 with the GPU's assignments;
* centroids: new centroid = s / n in float64 rounded to float32, same bound
  divided by n.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _run(torch, X, Cn, offset=0):
    from paper_1309_0215_amd import Job
    job = Job(device=0, km_centroids=torch.from_numpy(Cn).to("cuda:0"))
    Xd = torch.from_numpy(X).to("cuda:0")
    if offset:
        big = torch.zeros(X.size + offset, dtype=torch.float32, device="cuda:0")
        big[offset:] = Xd.reshape(-1)
        Xd = big[offset:].view(X.shape)
    a, s, c, cent, st = job.kmeans(Xd)
    return (a.cpu().numpy(), s.cpu().numpy(), c.cpu().numpy().view(np.uint32), cent.cpu().numpy(), st)


def _check_assign(X, Cn, a, idx=None):
    if idx is None:
        idx = np.arange(len(X))
    D = oracle.kmeans_distances(X[idx], Cn)
    dmin = D.min(axis=1)
    dg = D[np.arange(len(idx)), a[idx]]
    ok = dg <= dmin * (1 + 1e-6) + 1e-12
    assert ok.all(), (np.flatnonzero(~ok)[:10], dg[~ok][:5], dmin[~ok][:5])
    return int((a[idx] != D.argmin(axis=1)).sum())


def _check_assign_all(X, Cn, a, chunk=1 << 20):
    """_check_assign over every point, for sizes where the direct form of
    every distance takes minutes. Each point is screened with the expanded
    float64 form |x|^2 - 2 x.c + |c|^2 (float32 inputs: the products are
    exact, the 32-term sums round by less than 32 * 2^-53 of |x|^2 + 2|x||c|
    + |c|^2), taken here with the margin m = 1e-12 (|x|^2 + max |c|^2), over
    a hundred times that bound. A point whose distance to its assigned
    centroid lies more than 3m inside the acceptance limit passes, more than
    3m outside it fails; the others are decided by the oracle's direct form.
    Returns the number of points so decided."""
    C64 = np.asarray(Cn, np.float64)
    cn = (C64 * C64).sum(axis=1)
    near = []
    for lo in range(0, len(X), chunk):
        x = np.asarray(X[lo:lo + chunk], np.float64)
        xn = (x * x).sum(axis=1)
        De = xn[:, None] - 2.0 * (x @ C64.T) + cn[None, :]
        lim = De.min(axis=1) * (1 + 1e-6) + 1e-12
        dg = De[np.arange(len(x)), a[lo:lo + chunk]]
        m = 1e-12 * (xn + cn.max())
        assert not (dg > lim + 3 * m).any(), lo + np.flatnonzero(dg > lim + 3 * m)[:10]
        near.append(lo + np.flatnonzero(np.abs(dg - lim) <= 3 * m))
    idx = np.concatenate(near)
    if len(idx):
        _check_assign(X, Cn, a, idx)
    return len(idx)


def _check_update(X, Cn, a, s, c, cent):
    k = len(Cn)
    S64, n64, newC = oracle.kmeans_update(X, a, Cn)
    assert np.array_equal(c.astype(np.int64), n64)
    A = oracle.kmeans_abs_sums(X, a, k)
    tol = 1e-5 * np.maximum(np.abs(S64), A)
    assert (np.abs(s.astype(np.float64) - S64) <= tol).all()
    ctol = tol / np.maximum(n64, 1)[:, None] + 1e-7 * np.abs(newC)
    assert (np.abs(cent.astype(np.float64) - newC) <= ctol).all()


@pytest.mark.parametrize("n", [1, 31, 32, 33, 4097, 50_000])
def test_mfma_path(torch, n):
    X, Cn = gen.kmeans(3, n=max(n, 64), d=32, k=64)
    X = X[:n].copy()
    a, s, c, cent, st = _run(torch, X, Cn)
    assert st["strategy_used"] == 1  # matrix-core path
    _check_assign(X, Cn, a)
    _check_update(X, Cn, a, s, c, cent)


@pytest.mark.parametrize("scale", [1e-3, 1e3])
def test_mfma_path_scales(torch, scale):
    # the near-tie bound scales with |x| and max |c|: small and large coordinates
    X, Cn = gen.kmeans(7, n=50_000, d=32, k=64)
    X = (X * scale).astype(np.float32)
    Cn = (Cn * scale).astype(np.float32)
    a, s, c, cent, st = _run(torch, X, Cn)
    assert st["strategy_used"] == 1
    _check_assign(X, Cn, a)
    _check_update(X, Cn, a, s, c, cent)


def test_tiny_coordinates_redo_the_step_generically(torch):
    # a nonzero coordinate below 2^-100 (in a point or a centroid) is outside
    # the exact bfloat16 split of the matrix-core path: the generic kernel
    # redoes the step
    X, Cn = gen.kmeans(8, n=4096, d=32, k=64)
    X = X.copy()
    X[100:200] *= np.float32(1e-33)
    a, s, c, cent, st = _run(torch, X, Cn)
    assert st["strategy_used"] == 0
    _check_assign(X, Cn, a)
    _check_update(X, Cn, a, s, c, cent)
    X, Cn = gen.kmeans(9, n=4096, d=32, k=64)
    Cn = Cn.copy()
    Cn[5, 3] = np.float32(1e-35)
    a, s, c, cent, st = _run(torch, X, Cn)
    assert st["strategy_used"] == 0
    _check_assign(X, Cn, a)
    _check_update(X, Cn, a, s, c, cent)


def test_generic_path_any_shape(torch):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3001, 5)).astype(np.float32)
    Cn = X[:7].copy()
    a, s, c, cent, st = _run(torch, X, Cn)
    assert st["strategy_used"] == 0
    _check_assign(X, Cn, a)
    _check_update(X, Cn, a, s, c, cent)


def test_unaligned_points_use_generic_path(torch):
    X, Cn = gen.kmeans(4, n=2000, d=32, k=64)
    a, s, c, cent, st = _run(torch, X, Cn, offset=1)
    assert st["strategy_used"] == 0
    _check_assign(X, Cn, a)
    _check_update(X, Cn, a, s, c, cent)


def test_exact_ties_take_lowest_index_and_empty_clusters_keep_centroid(torch):
    X, Cn = gen.kmeans(5, n=8192, d=32, k=64)
    Cn = Cn.copy()
    Cn[10] = Cn[3]          # identical centroids: every point of cluster 3 ties with 10
    Cn[20] = 1000.0         # far away: an empty cluster
    a, s, c, cent, st = _run(torch, X, Cn)
    assert not (a == 10).any() and not (a == 20).any()
    assert c[20] == 0 and np.array_equal(cent[20], Cn[20])
    _check_assign(X, Cn, a)
    _check_update(X, Cn, a, s, c, cent)


def test_points_equal_to_centroids(torch):
    X, Cn = gen.kmeans(6, n=64, d=32, k=64)
    a, s, c, cent, st = _run(torch, Cn.copy(), Cn)
    assert np.array_equal(a, np.arange(64))


@pytest.mark.parametrize("d,k", [(32, 64), (5, 7)])
def test_no_points(torch, d, k):
    """An input of no points: every cluster is empty, so the counts and sums
    are zero and every centroid stays where it was (the oracle's update of an
    empty input gives the same)."""
    rng = np.random.default_rng(8)
    Cn = rng.standard_normal((k, d)).astype(np.float32)
    X = np.zeros((0, d), np.float32)
    a, s, c, cent, st = _run(torch, X, Cn)
    assert len(a) == 0 and (c == 0).all() and (s == 0).all()
    assert np.array_equal(cent, Cn)
    _check_update(X, Cn, a, s, c, cent)


def test_full_config_16m(torch):
    """The full 16,777,216-point step. The assignments of all points are
    checked (the first and the last 2^19, which hold the grid's ragged tail,
    against the oracle's direct form; every point through _check_assign_all),
    the counts and sums over all points."""
    X, Cn = gen.kmeans(3)  # 16,777,216 x 32, k = 64, first 64 points
    a, s, c, cent, st = _run(torch, X, Cn)
    assert int(c.astype(np.int64).sum()) == len(X)
    half = 1 << 19
    idx = np.concatenate([np.arange(half), np.arange(len(X) - half, len(X))])
    _check_assign(X, Cn, a, idx)
    print(f"points decided by the direct form: {_check_assign_all(X, Cn, a)}")
    # sums over all points in float64 with the GPU's assignments (bincount per dim)
    k, d = Cn.shape
    n64 = np.bincount(a, minlength=k)
    assert np.array_equal(c.astype(np.int64), n64)
    worst_rel = 0.0
    for t in range(d):
        col = X[:, t].astype(np.float64)
        S = np.bincount(a, weights=col, minlength=k)
        A = np.bincount(a, weights=np.abs(col), minlength=k)
        err = np.abs(s[:, t].astype(np.float64) - S)
        assert (err <= 1e-5 * np.maximum(np.abs(S), A)).all()
        # the plain relative bound wherever the sum is not a cancellation
        big = np.abs(S) > 1e-3 * A
        assert (err[big] <= 1e-5 * np.abs(S[big])).all()
        worst_rel = max(worst_rel, float((err[big] / np.abs(S[big])).max(initial=0.0)))
    print(f"largest plain relative sum error {worst_rel:.3e}")
    assert st["km_rechecked"] < len(X) // 100
