"""Pin of the oracle's corner turn: the definition written out with loops."""
import numpy as np

import oracle


def test_corner_turn_loops():
    g = np.random.default_rng(5)
    x = g.integers(0, 256, size=(7, 5), dtype=np.uint8)
    for flip in (False, True):
        y = oracle.corner_turn(x, flip)
        assert y.shape == (5, 7) and y.flags["C_CONTIGUOUS"]
        for c in range(5):
            for t in range(7):
                assert y[c, t] == x[t, 4 - c if flip else c]
