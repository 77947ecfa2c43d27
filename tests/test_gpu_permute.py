"""ltn_permute (LDS-staged bit permutation) against numpy.transpose:
pure data movement, so the result must be bit-identical."""
import time

import numpy as np
import pytest

from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def _reference(x, perm):
    """numpy: axis a of a [2]*rank array is bit rank-1-a."""
    rank = len(perm)
    inv = np.argsort(perm)
    b = x.shape[0]
    arr = x.reshape([b] + [2] * rank)
    axes = [0] + [1 + (rank - 1 - inv[rank - 1 - a]) for a in range(rank)]
    return np.ascontiguousarray(arr.transpose(axes)).reshape(b, -1)


@pytest.mark.parametrize("rank,batch,seed", [(0, 1, 0), (1, 3, 1), (3, 2, 2), (6, 1, 3), (9, 3, 4),
                                             (12, 2, 5), (15, 1, 6), (20, 2, 7)])
def test_permute_matches_transpose(rank, batch, seed):
    import torch
    import paper_2205_00393_amd as P
    rng = np.random.default_rng(seed)
    perm = [int(v) for v in rng.permutation(rank)]
    x = (rng.standard_normal((batch, 1 << rank)) + 1j * rng.standard_normal((batch, 1 << rank))).astype(np.complex64)
    banner(f"permute rank {rank} batch {batch} perm {perm}")
    xd = torch.from_numpy(x).cuda()
    y = P.permute(xd, perm)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), _reference(x, perm))


def test_permute_special_cases_and_bandwidth():
    import torch
    import paper_2205_00393_amd as P
    rank = 26
    rng = np.random.default_rng(11)
    x = torch.randn(2, 1 << rank, dtype=torch.complex64, device="cuda")
    # identity, a full reversal, and the permutation that swaps the low and
    # high halves (a plain matrix transpose)
    ident = list(range(rank))
    rev = list(reversed(range(rank)))
    half = [(j + rank // 2) % rank for j in range(rank)]
    xs = x[:, : 1 << 14].contiguous()
    for perm in ([j for j in range(14)], [13 - j for j in range(14)], [(j + 7) % 14 for j in range(14)]):
        y = P.permute(xs, perm)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), _reference(xs.cpu().numpy(), perm))
    out = torch.empty_like(x)
    for perm in (ident, rev, half, [int(v) for v in rng.permutation(rank)]):
        P.permute(x, perm, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            P.permute(x, perm, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        gbs = 2 * x.numel() * 8 / dt / 1e9
        banner(f"permute rank {rank} x2: {dt * 1e3:.3f} ms, {gbs:.0f} GB/s (HBM peak 8000)")
    back = P.permute(P.permute(x, half), [(j + rank - rank // 2) % rank for j in range(rank)])
    torch.cuda.synchronize()
    assert torch.equal(back, x)
