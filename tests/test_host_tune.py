"""Host logic of the launch-shape planner (no GPU): shape signatures and the
candidates it times."""
from paper_2508_21393_amd import binding as B
from paper_2508_21393_amd import tune


def test_candidates_equal_to_the_defaults_are_not_timed_twice():
    assert tune._resolved((0, 0, 0, 0), B.VL_MODE_BATCHED) == tune.LIBRARY_DEFAULTS
    # blocking batched calls default to two segments
    assert tune._resolved((8192, 2, 1, 0), B.VL_MODE_BATCHED) == tune._defaults(B.VL_MODE_BATCHED)
    assert tune._resolved((8192, 1, 1, 0), B.VL_MODE_BATCHED) != tune._defaults(B.VL_MODE_BATCHED)
    # persistent calls default to four segments
    assert tune._resolved((8192, 1, 1, 0), B.VL_MODE_PERSISTENT) != tune._defaults(B.VL_MODE_PERSISTENT)
    assert tune._resolved((0, 0, 0, 0), B.VL_MODE_PERSISTENT) == tune._defaults(B.VL_MODE_PERSISTENT)
    grid = tune.DEFAULT_GRID
    assert len(grid) == 24 and len(set(grid)) == 24
    assert sum(tune._resolved(c, B.VL_MODE_BATCHED) == tune.LIBRARY_DEFAULTS for c in grid) == 1
