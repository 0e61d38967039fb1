"""Brute-force numpy computations that pin the oracle (test-only).

Written independently of ``oracle/``: sites are handled as explicit Cartesian
positions, shells come from sorting distances of a block of sites, and pair
counts come either from a position lookup (any lattice size, duplicate images
counted) or from all-pairs minimum-image distances (edges >= 4).
"""
from __future__ import annotations

import itertools

import numpy as np

BASIS = {
    0: np.array([(0, 0, 0), (1, 1, 1)], dtype=np.int64),                        # BCC
    1: np.array([(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)], dtype=np.int64),  # FCC
}


def positions(lattice: int, dims) -> np.ndarray:
    """Half-unit positions, site index i = b + m*(x + Lx*(y + Ly*z))."""
    Lx, Ly, Lz = (int(v) for v in dims)
    B = BASIS[lattice]
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    cells = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    pos = 2 * cells[:, None, :] + B[None, :, :]
    return pos.reshape(-1, 3)


def shell_vectors(lattice: int, S: int):
    """Distinct squared lengths (ascending) and the vectors of each shell,
    found by measuring every site of a 9^3 block from a central site."""
    pos = positions(lattice, (9, 9, 9))
    centre = np.array([8, 8, 8])
    d = pos - centre
    r2 = (d * d).sum(axis=1)
    radii = np.unique(r2[r2 > 0])[:S]
    vecs = [d[r2 == r] for r in radii]
    return radii, vecs


def neighbour_table(lattice: int, dims, S: int):
    """nbr[s] : int array [N, Z_s] of neighbour indices (periodic, duplicates
    kept), via a dictionary from wrapped position to site index."""
    dims = np.asarray(dims, dtype=np.int64)
    pos = positions(lattice, dims)
    period = 2 * dims
    lookup = {tuple(p): i for i, p in enumerate(pos)}
    _, vecs = shell_vectors(lattice, S)
    out = []
    for vs in vecs:
        tab = np.empty((len(pos), len(vs)), dtype=np.int64)
        for n, v in enumerate(vs):
            q = np.mod(pos + v, period)
            tab[:, n] = [lookup[tuple(t)] for t in q]
        out.append(tab)
    return out


def counts_from_table(nbr, occ: np.ndarray, K: int) -> np.ndarray:
    S = len(nbr)
    C = np.zeros((S, K, K), np.int64)
    for s in range(S):
        k = np.repeat(occ, nbr[s].shape[1])
        l = occ[nbr[s]].ravel()
        np.add.at(C[s], (k, l), 1)
    return C


def counts_min_image(lattice: int, dims, S: int, occ: np.ndarray, K: int) -> np.ndarray:
    """All-pairs counting by minimum-image distance (requires every edge >= 4,
    so that each neighbour pair is a single image)."""
    dims = np.asarray(dims, dtype=np.int64)
    assert (dims >= 4).all()
    pos = positions(lattice, dims)
    period = 2 * dims
    d = pos[:, None, :] - pos[None, :, :]
    d = (d + period // 2) % period - period // 2
    r2 = (d * d).sum(axis=2)
    radii, _ = shell_vectors(lattice, S)
    C = np.zeros((S, K, K), np.int64)
    for s, r in enumerate(radii):
        i, j = np.nonzero(r2 == r)
        np.add.at(C[s], (occ[i], occ[j]), 1)
    return C


def energy_from_table(nbr, occ: np.ndarray, V: np.ndarray) -> float:
    """E = 1/2 sum_i sum_s sum_n V_s[sigma_i][sigma_nbr]  (math.fsum)."""
    import math
    terms = []
    for s in range(len(nbr)):
        terms.append(V[s][occ[:, None], occ[nbr[s]]].ravel())
    return 0.5 * math.fsum(np.concatenate(terms).tolist())


def local_energy(nbr, occ: np.ndarray, V: np.ndarray, i: int) -> float:
    e = 0.0
    for s in range(len(nbr)):
        e += V[s][occ[i], occ[nbr[s][i]]].sum()
    return 0.5 * e


def all_configs(N: int, n_ones: int) -> np.ndarray:
    """Every 2-species configuration with n_ones sites of species 1."""
    combos = list(itertools.combinations(range(N), n_ones))
    occ = np.zeros((len(combos), N), np.uint8)
    for r, c in enumerate(combos):
        occ[r, list(c)] = 1
    return occ


def energies_batch(nbr, occs: np.ndarray, V: np.ndarray) -> np.ndarray:
    E = np.zeros(len(occs))
    for s in range(len(nbr)):
        E += V[s][occs[:, :, None], occs[:, nbr[s]]].sum(axis=(1, 2))
    return 0.5 * E
