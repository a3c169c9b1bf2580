"""The streaming-read probe that measures the L2 and HBM read bandwidths the
ray kernels are rated against: it must read every float4 it claims to read."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_vec,blocks,reps", [(2048, 1, 1), (4096, 7, 3), (1 << 15, 64, 2)])
def test_shared_footprint_sums(n_vec, blocks, reps):
    import paper_2508_13304_amd as dp
    buf = torch.ones(4 * n_vec, dtype=torch.float32, device="cuda:0")
    out = dp.read_probe(buf, reps, True, blocks)
    torch.cuda.synchronize()
    # every thread reads reps * n_vec / 256 float4 of ones
    assert torch.all(out == reps * n_vec * 4 / 256)


def _partition_owner(n_vec, blocks):
    """Output slot (256 b + j) that reads each float4 in partitioned mode: block
    b's slab of `per` float4 (thread j: slab offset mod 256), then the tail
    shared grid-stride."""
    import numpy as np
    per = n_vec // (blocks * 2048) * 2048
    i = np.arange(n_vec)
    owner = np.empty(n_vec, np.int64)
    main = i < blocks * per
    if per:
        owner[main] = (i[main] // per) * 256 + (i[main] % per) % 256
    owner[~main] = (i[~main] - blocks * per) % (blocks * 256)
    return owner


@pytest.mark.parametrize("n_vec,blocks,reps", [(1, 1, 1), (1000, 1, 2), (10007, 3, 1),
                                               (12288, 3, 1), (1 << 20, 40, 2)])
def test_partitioned_reads_every_element_once_per_pass(n_vec, blocks, reps):
    import numpy as np
    import paper_2508_13304_amd as dp
    # element i of the float4 view holds (i mod 251) + 1 in its x lane and zeros
    # elsewhere, so a skipped, repeated or misassigned element changes a sum
    val = (np.arange(n_vec) % 251 + 1).astype(np.float64)
    host = np.zeros((n_vec, 4), np.float32)
    host[:, 0] = val
    buf = torch.from_numpy(host.reshape(-1)).to("cuda:0")
    out = dp.read_probe(buf, reps, False, blocks)
    torch.cuda.synchronize()
    want = reps * np.bincount(_partition_owner(n_vec, blocks), weights=val, minlength=256 * blocks)
    # integer sums far below 2^24 per thread: exact in FP32
    assert np.array_equal(out.cpu().numpy().astype(np.float64), want)
