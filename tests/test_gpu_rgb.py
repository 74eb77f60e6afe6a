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
