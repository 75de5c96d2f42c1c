"""The distance colouring of exact probing (Sec. 6: the last term by probing)
checked by brute force on the CPU: two distinct sites at taxicab distance
<= D on the periodic lattice never share a colour.  The colouring is computed
by the library's host code (no device work)."""
import itertools

import numpy as np
import pytest

from paper_2402_00016_amd import mpmc


def colours(dims, k, m, W):
    L = np.array(dims)
    V = int(np.prod(L))
    s = np.arange(V)
    x = np.empty((V, 4), dtype=np.int64)
    q = s.copy()
    for mu in range(4):
        x[:, mu] = q % L[mu]
        q //= L[mu]
    col = np.zeros(V, dtype=np.int64)
    mul = 1
    for i in range(k):
        col += ((x @ np.array(W[i])) % m[i]) * mul
        mul *= m[i]
    return x, col


def torus_dist(x, y, L):
    d = np.abs(x - y) % L
    return np.sum(np.minimum(d, L - d), axis=-1)


@pytest.mark.parametrize("dims,D", [((4, 4, 4, 4), 1), ((4, 4, 4, 4), 3), ((6, 6, 6, 6), 2), ((6, 6, 6, 6), 4),
                                    ((8, 8, 8, 8), 4), ((4, 4, 2, 2), 2), ((3, 5, 2, 7), 3), ((4, 4, 4, 4), 9)])
def test_distance_property_brute_force(dims, D):
    k, m, W, nc = mpmc.mpmc_probe_colouring(dims, D)
    assert nc == int(np.prod(m))
    L = np.array(dims)
    x, col = colours(dims, k, m, W)
    V = len(col)
    assert col.min() >= 0 and col.max() < nc
    for s in range(V):
        same = np.flatnonzero(col == col[s])
        same = same[same != s]
        if len(same):
            assert torus_dist(x[same], x[s], L).min() > D, (dims, D, s)
    # colour count: at least the sites of a ball of radius D // 2 (pairwise within D)
    r = D // 2
    ball = sum(1 for d in itertools.product(range(-r, r + 1), repeat=4) if sum(map(abs, d)) <= r)
    if all(2 * r < Lm for Lm in dims):
        assert nc >= ball


def test_large_lattice_colouring_is_compact():
    """24^4 with D = 8 (the degree-8 last polynomial of the 24^4 workload):
    far fewer colours than sites; the translation-invariant check over every
    displacement of the ball stands in for the all-pairs one."""
    dims, D = (24, 24, 24, 24), 8
    k, m, W, nc = mpmc.mpmc_probe_colouring(dims, D)
    assert nc <= 1024 and k <= 3
    W = np.array(W)
    for d in itertools.product(range(-D, D + 1), repeat=4):
        if 0 < sum(map(abs, d)) <= D:
            assert np.any((W @ np.array(d)) % np.array(m) != 0), d
    with pytest.raises(mpmc.MpmcError):
        mpmc.mpmc_probe_colouring(dims, -1)


@pytest.mark.parametrize("dims,D", [((16, 16, 16, 16), 255), ((16, 16, 16, 16), 32), ((24, 24, 24, 24), 129)])
def test_distance_beyond_the_torus_is_every_site(dims, D):
    """A distance at or beyond the torus diameter (sum of L_mu / 2; 255 is the
    degree of the 16x16 double polynomial) puts every pair of sites within
    reach, so every site is its own colour; found without enumerating the
    ball of radius D (about 10^9 displacements at D = 255)."""
    k, m, W, nc = mpmc.mpmc_probe_colouring(dims, D)
    assert nc == int(np.prod(dims)) and k == 4
    assert sorted(m) == sorted(dims)
