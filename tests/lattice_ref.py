"""Velocity sets rebuilt from the documented population ordering, for tests only
(independent of both the oracle's and the GPU library's tables)."""
import numpy as np


def velocities(Q):
    if Q == 9:
        return np.array([[i % 3 - 1, i // 3 - 1] for i in range(9)], dtype=np.float64)
    return np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)],
                    dtype=np.float64)
