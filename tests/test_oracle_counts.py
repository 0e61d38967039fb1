"""Pins of the oracle's pair counts, energy and Warren-Cowley SRO (CPU only).

Brute force on tiny lattices (position lookup with duplicates, and all-pairs
minimum-image distances), exact invariants of directed counts, linearity of E
in V, and closed-form SRO of an ordered B2 arrangement.
"""
import numpy as np
import pytest

import brute

BCC, FCC = 0, 1


def rand_occ(N, K, seed):
    return np.random.default_rng(seed).integers(0, K, N).astype(np.uint8)


@pytest.mark.parametrize("lattice,dims,K,S", [(BCC, (4, 4, 4), 4, 4), (FCC, (4, 5, 4), 5, 4),
                                              (BCC, (5, 4, 6), 3, 2), (FCC, (4, 4, 4), 2, 3)])
def test_counts_vs_min_image_pairs(oracle, lattice, dims, K, S):
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ = rand_occ(N, K, 1)
    C = oracle.pair_counts(lattice, dims, K, S, occ)
    ref = brute.counts_min_image(lattice, dims, S, occ, K)
    assert np.array_equal(C, ref)


@pytest.mark.parametrize("nthreads", [2, 3, 7])
def test_threaded_counts_vs_min_image_pairs(oracle, nthreads):
    """The threaded counts (sites split over threads, tables added) against
    brute force, with site ranges that do not divide evenly."""
    for lattice, dims, K, S in [(BCC, (5, 4, 6), 4, 4), (FCC, (4, 5, 4), 5, 3)]:
        N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
        occ = rand_occ(N, K, 3)
        C = oracle.pair_counts(lattice, dims, K, S, occ, nthreads=nthreads)
        assert np.array_equal(C, brute.counts_min_image(lattice, dims, S, occ, K))


@pytest.mark.parametrize("lattice,dims,K,S", [(BCC, (2, 2, 2), 2, 2), (BCC, (2, 3, 2), 3, 4),
                                              (FCC, (2, 2, 3), 3, 4), (BCC, (3, 3, 3), 4, 4)])
def test_counts_small_cells_with_duplicate_images(oracle, lattice, dims, K, S):
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ = rand_occ(N, K, 2)
    C = oracle.pair_counts(lattice, dims, K, S, occ)
    ref = brute.counts_from_table(brute.neighbour_table(lattice, dims, S), occ, K)
    assert np.array_equal(C, ref)


@pytest.mark.parametrize("lattice,dims,K,S", [(BCC, (2, 2, 2), 2, 2), (BCC, (2, 3, 2), 3, 4),
                                              (FCC, (2, 2, 3), 3, 4), (BCC, (5, 4, 6), 4, 4), (FCC, (4, 5, 4), 5, 4)])
def test_half_shell_counts_give_the_directed_counts(oracle, lattice, dims, K, S):
    """Counting, at every site, one direction d of each +-d pair of a shell
    (the lexicographically smaller half) gives H with C[k][l] = H[k][l] +
    H[l][k]: the pairs along -d from species k to l are the pairs along +d
    from l to k.  This holds also on cells where +d and -d reach the same
    site (duplicate images)."""
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ = rand_occ(N, K, 3)
    dims_a = np.asarray(dims, dtype=np.int64)
    pos = brute.positions(lattice, dims_a)
    lookup = {tuple(p): i for i, p in enumerate(pos)}
    _, vecs = brute.shell_vectors(lattice, S)
    H = np.zeros((S, K, K), np.int64)
    for s, vs in enumerate(vecs):
        vs = sorted(tuple(int(c) for c in v) for v in vs)
        half, rest = vs[:len(vs) // 2], set(vs[len(vs) // 2:])
        assert all(tuple(-c for c in v) in rest for v in half)
        for v in half:
            q = np.mod(pos + np.asarray(v), 2 * dims_a)
            j = np.array([lookup[tuple(t)] for t in q])
            np.add.at(H[s], (occ, occ[j]), 1)
    C = oracle.pair_counts(lattice, dims, K, S, occ)
    assert np.array_equal(H + H.transpose(0, 2, 1), C)


@pytest.mark.parametrize("lattice,dims,K,S", [(BCC, (6, 5, 4), 4, 4), (FCC, (3, 4, 5), 5, 4)])
def test_count_invariants(oracle, lattice, dims, K, S):
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ = rand_occ(N, K, 3)
    Z, _ = oracle.shells(lattice, S)
    C = oracle.pair_counts(lattice, dims, K, S, occ)
    Nk = np.bincount(occ, minlength=K)
    for s in range(S):
        assert np.array_equal(C[s], C[s].T)
        assert np.array_equal(C[s].sum(axis=1), Z[s] * Nk)
        assert C[s].sum() == N * Z[s]


def test_energy_vs_brute_force(oracle):
    lattice, dims, K, S = BCC, (4, 5, 4), 4, 4
    N = int(np.prod(dims)) * 2
    occ = rand_occ(N, K, 4)
    V = np.random.default_rng(9).normal(0, 0.05, (S, K, K))
    V = V + V.transpose(0, 2, 1)
    E = oracle.energy(oracle.pair_counts(lattice, dims, K, S, occ), V)
    ref = brute.energy_from_table(brute.neighbour_table(lattice, dims, S), occ, V)
    assert abs(E - ref) <= 1e-12 * max(1.0, abs(ref))


def test_energy_is_half_counts_dot_V(oracle):
    """E is linear in V with gradient C/2: central differences are exact up to
    rounding (pins the factor 1/2 and the index order)."""
    lattice, dims, K, S = FCC, (3, 3, 4), 3, 2
    N = int(np.prod(dims)) * 4
    occ = rand_occ(N, K, 5)
    C = oracle.pair_counts(lattice, dims, K, S, occ)
    V = np.random.default_rng(3).normal(0, 0.1, (S, K, K))
    h = 1e-3
    for s in range(S):
        for k in range(K):
            for l in range(K):
                Vp, Vm = V.copy(), V.copy()
                Vp[s, k, l] += h
                Vm[s, k, l] -= h
                g = (oracle.energy(C, Vp) - oracle.energy(C, Vm)) / (2 * h)
                assert abs(g - 0.5 * C[s, k, l]) <= 1e-9 * max(1.0, abs(C[s, k, l]))


def b2_occupancy(dims):
    """Two species on the two BCC sublattices: every nearest-neighbour bond
    joins unlike species."""
    N = int(np.prod(dims)) * 2
    return (np.arange(N) % 2).astype(np.uint8)


def test_sro_of_b2_order(oracle):
    dims, K, S = (4, 4, 4), 2, 2
    occ = b2_occupancy(dims)
    Z, _ = oracle.shells(BCC, S)
    C = oracle.pair_counts(BCC, dims, K, S, occ)
    a = oracle.sro(C, Z)
    # shell 1: all unlike -> alpha_AB = 1 - N*Z*N/2 / (Z*N/2*N/2) = -1; alpha_AA = 1
    assert a[0, 0, 1] == -1.0 and a[0, 1, 0] == -1.0
    assert a[0, 0, 0] == 1.0 and a[0, 1, 1] == 1.0
    # shell 2 joins the same sublattice: all like -> alpha_AB = 1, alpha_AA = -1
    assert a[1, 0, 1] == 1.0 and a[1, 0, 0] == -1.0


def test_sro_rejects_absent_species(oracle):
    dims, K, S = (4, 4, 4), 3, 1
    occ = b2_occupancy(dims)  # species 2 absent
    Z, _ = oracle.shells(BCC, S)
    C = oracle.pair_counts(BCC, dims, K, S, occ)
    with pytest.raises(ValueError):
        oracle.sro(C, Z)
