"""CPU checks of the test-side helpers that recompute results on the device
(run here on CPU tensors): the torch statement of the digest equals the
oracle's per-triangle digest, and the device sort equals numpy's lexsort."""
import numpy as np
import torch

import oracle
from gpu_util import digest_sum_torch, sort_rows, sorted_rows_device


def test_digest_helper_matches_oracle():
    rs = np.random.default_rng(5)
    tri = np.sort(rs.integers(0, 2**32, (500, 3), dtype=np.uint64), axis=1).astype(np.uint32)
    tri[:5] = [[0, 1, 2], [0, 0xFFFFFFFE, 0xFFFFFFFF], [7, 8, 9], [1 << 31, (1 << 31) + 1, 0xFFFFFFFF], [3, 4, 5]]
    want = oracle.hash_of(tri)
    got = digest_sum_torch(torch.from_numpy(tri.view(np.int32)))
    assert got == want
    assert digest_sum_torch(torch.zeros((0, 3), dtype=torch.int32)) == 0


def test_device_sort_helper_matches_lexsort():
    rs = np.random.default_rng(6)
    for bits in (10, 21, 26, 32):
        tri = rs.integers(0, 2**bits, (2000, 3), dtype=np.uint64).astype(np.uint32)
        tri[:100] = tri[100:200]  # repeated rows
        got = sorted_rows_device(torch.from_numpy(tri.view(np.int32)), bits).numpy().view(np.uint32)
        assert np.array_equal(got, sort_rows(tri)), bits
