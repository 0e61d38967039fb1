"""Pins of the oracle's local energies and low-energy clusters (CPU only).

  - local energies against a brute-force neighbour-table sum, and their total
    against the brute-force energy;
  - clusters against scipy's connected components of the marked sites on
    the nearest-neighbour graph (labels = smallest site index, sizes, count),
    with the threshold on an exact local-energy value so that ties at the
    threshold count;
  - limits: every site marked gives one cluster of N sites, none marked none.
"""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import brute

BCC, FCC = 0, 1


def sym_V(S, K, scale, seed):
    V = np.random.default_rng(seed).normal(0, scale, (S, K, K))
    return 0.5 * (V + V.transpose(0, 2, 1))


CASES = [(BCC, (6, 5, 7), 4, 4, 1), (FCC, (4, 5, 3), 5, 3, 2), (BCC, (2, 3, 2), 3, 2, 3), (FCC, (5, 5, 5), 2, 1, 4)]


@pytest.mark.parametrize("lattice,dims,K,S,seed", CASES)
def test_local_energy_brute_force(oracle, lattice, dims, K, S, seed):
    m = 2 if lattice == BCC else 4
    N = m * int(np.prod(dims))
    occ = np.random.default_rng(seed).integers(0, K, N).astype(np.uint8)
    V = sym_V(S, K, 0.05, seed + 10)
    e = oracle.local_energy(lattice, dims, K, S, occ, V)
    nbr = brute.neighbour_table(lattice, dims, S)
    ref = np.array([brute.local_energy(nbr, occ, V, i) for i in range(N)])
    assert np.allclose(e, ref, rtol=1e-12, atol=1e-15)
    E = brute.energy_from_table(nbr, occ, V)
    assert abs(math.fsum(e.tolist()) - E) <= 1e-12 * max(1.0, abs(E))
    idx = np.random.default_rng(seed).integers(0, N, 25)
    assert np.array_equal(oracle.local_energy_at(lattice, dims, K, S, occ, V, idx), e[idx])


def reference_clusters(lattice, dims, e, thr):
    """Connected components of {i: e_i <= thr} on the shell-1 graph (scipy)."""
    nbr = brute.neighbour_table(lattice, dims, 1)[0]
    N = len(e)
    mark = e <= thr
    i = np.repeat(np.arange(N), nbr.shape[1])
    j = nbr.ravel()
    keep = mark[i] & mark[j]
    g = coo_matrix((np.ones(keep.sum()), (i[keep], j[keep])), shape=(N, N))
    _, comp = connected_components(g, directed=False)
    label = np.full(N, -1, np.int32)
    size = np.zeros(N, np.int32)
    roots = {}
    for s in np.nonzero(mark)[0]:  # ascending: the first site of a component is its smallest
        roots.setdefault(comp[s], s)
        label[s] = roots[comp[s]]
    for r in roots.values():
        size[r] = int((label == r).sum())
    return label, size, len(roots)


@pytest.mark.parametrize("lattice,dims,K,S,seed", CASES)
@pytest.mark.parametrize("q", [0.15, 0.4, 0.7])
def test_clusters_against_connected_components(oracle, lattice, dims, K, S, seed, q):
    m = 2 if lattice == BCC else 4
    N = m * int(np.prod(dims))
    occ = np.random.default_rng(seed).integers(0, K, N).astype(np.uint8)
    V = sym_V(S, K, 0.05, seed + 10)
    e = oracle.local_energy(lattice, dims, K, S, occ, V)
    thr = float(np.sort(e)[int(q * (N - 1))])  # an exact local energy: ties sit on the threshold
    label, size, n = oracle.clusters(lattice, dims, e, thr)
    rl, rs, rn = reference_clusters(lattice, dims, e, thr)
    assert np.array_equal(label, rl)
    assert np.array_equal(size, rs)
    assert n == rn
    assert size.sum() == (e <= thr).sum()


def test_cluster_limits(oracle):
    dims = (5, 4, 6)
    N = 2 * 120
    e = np.random.default_rng(3).normal(size=N)
    label, size, n = oracle.clusters(BCC, dims, e, math.inf)
    assert n == 1 and (label == 0).all() and size[0] == N
    label, size, n = oracle.clusters(BCC, dims, e, -math.inf)
    assert n == 0 and (label == -1).all() and (size == 0).all()


def test_planted_cluster(oracle):
    """A 2 x 2 x 2 block of low local energies in a high-energy matrix is
    one cluster of exactly its 16 sites, labelled by its first site."""
    dims = (8, 8, 8)
    e = np.ones(2 * 512)
    for z in range(3, 5):
        for y in range(2, 4):
            for x in range(5, 7):
                for b in range(2):
                    e[b + 2 * (x + 8 * (y + 8 * z))] = -1.0
    label, size, n = oracle.clusters(BCC, dims, e, 0.0)
    first = 0 + 2 * (5 + 8 * (2 + 8 * 3))
    assert n == 1 and size[first] == 16 and (label[e < 0] == first).all()
