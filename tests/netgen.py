"""Small random networks for planner tests (structure only; seeded)."""
import numpy as np


def random_network(seed, L, E, n_open):
    """L tensors joined by E closed indices (a random spanning tree plus
    extra edges) and n_open open indices; returns (leaf index lists, n_indices,
    open ids)."""
    rng = np.random.default_rng(seed)
    idx = [[] for _ in range(L)]
    x = 0
    for i in range(1, L):
        j = int(rng.integers(i))
        idx[i].append(x)
        idx[j].append(x)
        x += 1
    while x < E:
        i, j = rng.choice(L, 2, replace=False)
        idx[int(i)].append(x)
        idx[int(j)].append(x)
        x += 1
    opens = []
    for _ in range(n_open):
        idx[int(rng.integers(L))].append(x)
        opens.append(x)
        x += 1
    return idx, x, opens
