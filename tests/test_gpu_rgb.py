"""GPU parity of the RGB histogram (MR_MAP_RGB_HIST) against the CPU oracle, bit-exact."""
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


@pytest.mark.parametrize("n_px", [0, 1, 5, 17, 1000, 65_537, 1_000_003])
def test_sizes(torch, job, n_px):
    buf = gen.rgb(2, 3 * n_px)
    d = torch.from_numpy(buf).to("cuda:0") if n_px else torch.empty(0, dtype=torch.uint8, device="cuda:0")
    h, _ = job.rgb_hist(d)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(buf))


@pytest.mark.parametrize("shift", [1, 2, 5, 13])
def test_unaligned(torch, job, shift):
    buf = gen.rgb(3, 3 * 333_333)
    big = torch.zeros(len(buf) + 32, dtype=torch.uint8, device="cuda:0")
    big[shift:shift + len(buf)] = torch.from_numpy(buf).to("cuda:0")
    h, _ = job.rgb_hist(big[shift:shift + len(buf)])
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(buf))


def test_length_not_multiple_of_three(torch, job):
    from paper_1309_0215_amd import MRError
    d = torch.zeros(10, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(MRError) as e:
        job.rgb_hist(d)
    assert e.value.status == -1


def test_full_config_1gib(torch, job):
    buf = gen.rgb(2)  # floor(2^30 / 3) pixels
    d = torch.from_numpy(buf).to("cuda:0")
    h, st = job.rgb_hist(d)
    exp = oracle.rgb(buf)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), exp)
    assert int(exp.sum()) == len(buf)


@pytest.mark.parametrize("mib", [17, 35, 52])
def test_whole_rounds_per_workgroup(torch, job, mib):
    # 1,024 workgroups of 512 lanes load 2 x 16 bytes per lane per round: at
    # these sizes each workgroup runs 1, 2 or 3 whole rounds, then a ragged tail
    n = (mib << 20) // 3 * 3 + 3 * 7
    buf = gen.rgb(40 + mib, n)
    d = torch.from_numpy(buf).to("cuda:0")
    h, _ = job.rgb_hist(d)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(buf))


def test_repeated_calls_replay_a_graph(torch):
    # the second identical call captures a graph and later ones replay it:
    # new input contents in place, another job kind growing the workspace in
    # between, a timed job and a fresh output all give the oracle's bins
    from paper_1309_0215_amd import Job
    job = Job(device=0, timing=1)
    out = torch.empty(768, dtype=torch.int64, device="cuda:0")
    bufs = [gen.rgb(50 + i, 3 * 400_007) for i in range(3)]
    d = torch.from_numpy(bufs[0]).to("cuda:0")
    for i in range(4):
        h, st = job.rgb_hist(d, out=out)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(bufs[0])), i
        assert st["map_ms"] > 0 and st["gpu_ms"] >= st["map_ms"]
    d.copy_(torch.from_numpy(bufs[1]).to("cuda:0"))
    h, _ = job.rgb_hist(d, out=out)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(bufs[1]))
    text = torch.from_numpy(gen.text(3, 40 << 20, V=20_000)).to("cuda:0")
    job.words(text)  # grows the shared workspace
    for _ in range(3):
        h, _ = job.rgb_hist(d, out=out)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(bufs[1]))
    d2 = torch.from_numpy(bufs[2]).to("cuda:0")
    for _ in range(3):
        h, _ = job.rgb_hist(d2)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(bufs[2]))
    with pytest.raises(ValueError):
        job.rgb_hist(d, out=torch.empty(767, dtype=torch.int64, device="cuda:0"))
