"""Host logic of the planner's chunk policy (no GPU): asynchronous calls on
batches that stream over 1 GB of matrices contract their int16 operands over
rows in longer chunks, which shows in the workspace they need (fewer chunk
sums); small calls, blocking calls and calls with an explicit lane_macs keep
the short chunks."""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2508_21393_amd import binding
    if not os.path.exists(os.path.join(ROOT, "paper_2508_21393_amd", "libverilora.so")):
        pytest.skip("library not built")
    binding.lib()
    return binding


def test_long_row_chunks_only_for_large_async_calls(B):
    # four groups of 2048 x 16384 . 16384 x 8192 (int16 A and B, int64 C):
    # 1.9 GB of matrices; one 2048 x 4096 . 4096 x 4096 group: 0.2 GB
    big = [B.GroupArgs.shapes_only(k, [(2048, 16384, 8192)]) for k in range(4)]
    small = [B.GroupArgs.shapes_only(0, [(2048, 4096, 4096)])]
    short = B.tuning(lane_macs=8192)
    big_async = B.workspace_size(big, 1, async_=True)
    assert big_async < B.workspace_size(big, 1, async_=True, tuning_=short)
    assert big_async < B.workspace_size(big, 1)
    assert B.workspace_size(small, 1, async_=True) == B.workspace_size(small, 1, async_=True, tuning_=short)
