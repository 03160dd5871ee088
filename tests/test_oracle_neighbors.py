"""Pins for the oracle's neighbour search (CPU).

* Brute force agrees with SciPy's k-d tree pair query (an independent library
  routine) for uniform smoothing lengths.
* The cell-list search agrees with brute force for variable h.
* Unjittered lattices give the lattice-point counts inside the support:
  20 neighbours in 2D at h = 1.3 spacing (support 2.6 spacings: |i|^2+|j|^2 <= 5)
  and 56 in 3D at h = 1.2 spacing (|i|^2+|j|^2+|k|^2 <= 5), self excluded.
* The relation is symmetric.
"""
import itertools

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import kernels, neighbors


def _kdtree_csr(pos, radius):
    n = pos.shape[1]
    pr = cKDTree(pos.T).query_pairs(radius, output_type="ndarray")
    I = np.concatenate([pr[:, 0], pr[:, 1]])
    J = np.concatenate([pr[:, 1], pr[:, 0]])
    o = np.lexsort((J, I))
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(I, minlength=n), out=ptr[1:])
    return ptr, J[o].astype(np.int32)


@pytest.mark.parametrize("dim", [2, 3])
def test_bruteforce_matches_kdtree(dim):
    rng = np.random.default_rng(7)
    n = 14 if dim == 2 else 9
    pos, nin = synth.jittered_lattice(dim, n, 0.3, 2, rng)
    h = np.full(pos.shape[1], 1.25 / n)
    ptr, idx = neighbors.brute_force(pos, h, 2.0)
    kptr, kidx = _kdtree_csr(pos, 2.0 * 1.25 / n)
    assert np.array_equal(ptr, kptr)
    assert np.array_equal(idx, kidx)


def test_random_points_match_kdtree():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 1, (3, 1500))
    h = np.full(1500, 0.06)
    ptr, idx = neighbors.brute_force(pos, h, 2.0)
    kptr, kidx = _kdtree_csr(pos, 0.12)
    assert np.array_equal(ptr, kptr) and np.array_equal(idx, kidx)


def test_cell_list_matches_bruteforce_variable_h():
    p = synth.config3(n=12)
    a = neighbors.brute_force(p.pos, p.h, 2.0)
    b = neighbors.cell_list(p.pos, p.h, 2.0, chunk=997)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_cell_list_matches_bruteforce_dart_points():
    p = synth.config4(n=14)
    a = neighbors.brute_force(p.pos, p.h, 2.0)
    b = neighbors.cell_list(p.pos, p.h, 2.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("dim,eta,count", [(2, 1.3, 20), (3, 1.2, 56)])
def test_unjittered_lattice_counts(dim, eta, count):
    n = 12
    pos, nin = synth.jittered_lattice(dim, n, 0.0, 0, np.random.default_rng(0))
    h = np.full(pos.shape[1], eta / n)
    ptr, idx = neighbors.cell_list(pos, h, 2.0)
    deg = np.diff(ptr)
    lat = np.rint(pos * n - 0.5).astype(int)
    interior = np.all((lat >= 3) & (lat < n - 3), axis=0)
    assert np.all(deg[interior] == count)


def test_symmetric_relation():
    p = synth.config1(n=16)
    ptr, idx = neighbors.build(p.pos, p.h, 2.0)
    I, J = neighbors.pairs(ptr, idx)
    fwd = set(zip(I.tolist(), J.tolist()))
    assert all((j, i) in fwd for i, j in fwd)
    assert not np.any(I == J)


@pytest.mark.parametrize("dim,n", [(2, 12), (3, 10)])
def test_periodic_neighbours_equal_explicit_images(dim, n):
    """Nearest-image pairs on a periodic box equal the pairs found by testing
    every particle against every shifted copy of the others (3^dim images,
    plain distances): with a box wider than twice the support, at most one
    image of a particle is in range.  (The two round differently only for a
    pair within rounding of the support edge; the jittered lattice has none.)"""
    prob = synth.periodic_wendland(dim, n)
    pos, h, L = prob.pos, prob.h, prob.period
    kappa = kernels.KAPPA[prob.kernel]
    assert np.all(2.0 * kappa * h.max() < L)
    ptr, idx = neighbors.brute_force(pos, h, kappa, period=L)
    N = h.shape[0]
    pairs = set()
    for shift in itertools.product((-1.0, 0.0, 1.0), repeat=dim):
        img = pos + (np.array(shift) * L)[:, None]
        both = np.concatenate([pos, img], axis=1)
        hh = np.concatenate([h, h])
        for i in range(N):
            J = np.arange(N)
            d2 = np.zeros(N)
            for ax in range(dim):
                d = both[ax][i] - both[ax][N + J]
                d2 = d2 + d * d
            t = kappa * np.maximum(hh[i], hh[N + J])
            for j in J[(d2 < t * t) & (J != i)]:
                pairs.add((i, int(j)))
    got = {(i, int(j)) for i in range(N) for j in idx[ptr[i]:ptr[i + 1]]}
    assert got == pairs
    assert all((j, i) in got for i, j in got)   # the relation stays symmetric
