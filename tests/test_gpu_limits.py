"""Counter-width limits: a block's per-class totals are 32-bit, and the launch code
raises the grid so that no block takes 2^31 bytes or more.  With an explicit grid
of one block, an all-ones input of about 5 GiB would give one block more than 2^32
set bits per class; the counts must still be exact (closed forms: every position
of an all-ones word is set n times, and every id of a constant stream is that id)."""
import pytest
import torch

from paper_1911_02696_amd import api

from gpu_util import counts_np, say

pytestmark = pytest.mark.gpu

NBYTES = (1 << 32) + (1 << 30) + 40  # 5 GiB + 40 bytes: more than 2^32 set bits per class


@pytest.fixture(scope="module")
def ones():
    buf = torch.full((NBYTES + 16,), 0xFF, dtype=torch.uint8, device="cuda")
    yield buf
    del buf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [8, 16, 32, 64])
def test_one_block_grid_is_raised_and_exact(ones, k):
    n = (NBYTES - 3) // (k // 8)
    say(f"limits k={k} n={n} grid=1")
    got = counts_np(api.pospopcnt(ones, k, n=n, byte_offset=3, grid=1))
    assert (got == n).all(), got


def test_planes_one_block_per_plane(ones):
    n = (NBYTES // 2) // 2 - 8  # two planes side by side in the same buffer
    planes = [ones[:2 * n], ones[2 * n:4 * n]]
    say(f"limits planes n={n} grid=1")
    got = counts_np(api.pospopcnt_planes(planes, n=n, grid=1))
    assert (got == n).all(), got


def test_histogram_one_block(ones):
    n = NBYTES - 1
    say(f"limits histogram n={n} grid=1")
    got = counts_np(api.histogram(ones, 8, id_bytes=1, n=n, byte_offset=1, grid=1))
    assert got[:8].tolist() == [0] * 8 and got[8] == n  # id 255 has no category of 8
    zeros = torch.zeros(NBYTES, dtype=torch.uint8, device="cuda")
    got = counts_np(api.histogram(zeros, 32, id_bytes=1, grid=1))
    assert got[0] == NBYTES and (got[1:] == 0).all()
