"""A seeded sweep of small cases against the oracle: random graphs, power-law
graphs with uniform and per-edge probabilities, stars and paths, with R on
both sides of the tile and mask-word boundaries, probabilities from 0 to 1
and K up to n.  Every case compares labels, sizes, initial gains, seeds,
marginal counts, the cover count and sigma counts exactly."""

import numpy as np
import pytest

from tests.test_gpu_parity import _full_check
from workloads import chung_lu, normal_p, path_graph, random_small_graph, star_graph, trivalency_p, uniform_p

pytestmark = pytest.mark.gpu

PS = [0.0, 2.0 ** -32, 0.003, 0.02, 0.1, 0.5, 1.0]
RS = [1, 17, 64, 255, 256, 257, 700, 1024, 1300]


def _case(i):
    rng = np.random.default_rng(9000 + i)
    kind = i % 4
    seed = 700 + i
    p = float(rng.choice(PS))
    if kind == 0:
        n = int(rng.integers(2, 40))
        g = random_small_graph(n, int(rng.integers(0, n * (n - 1) // 2 + 1)), seed)
    elif kind == 1:
        n = int(rng.integers(50, 1500))
        g = chung_lu(n, int(rng.integers(n, 6 * n)), float(rng.choice([2.1, 2.5, 3.0])), seed)
    elif kind == 2:
        n = int(rng.integers(2, 600))
        g = star_graph(n) if i % 8 == 2 else path_graph(n)
    else:
        n = int(rng.integers(50, 1200))
        g = chung_lu(n, int(rng.integers(n, 5 * n)), 2.3, seed)
        g.p_slot = (uniform_p, trivalency_p, normal_p)[(i // 4) % 3](g, seed)
        p = 0.0
    R = int(rng.choice(RS))
    K = int(rng.integers(1, min(g.n, 30) + 1))
    sets = [[int(rng.integers(0, g.n))], [int(x) for x in rng.integers(0, g.n, int(rng.integers(1, 20)))]]
    return g, p, R, seed, K, sets


@pytest.mark.parametrize("i", range(48))
def test_sweep_case(gpu_ctx, i):
    g, p, R, seed, K, sets = _case(i)
    _full_check(gpu_ctx, g, p, R, seed, K, sigma_sets=sets, name=f"sweep {i}")
