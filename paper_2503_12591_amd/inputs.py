"""Seeded synthetic inputs: lattices, compositions, EPI tensors, schedules.

This module holds no Monte Carlo arithmetic: it only draws and shapes inputs
(numpy ``Generator(PCG64(seed))``), so that the CPU oracle and the HIP path can
be fed identical data.  It imports nothing else from this package.

Workloads stand in for the paper's two alloys (its trained EPI values and
DFT data are not available): a BCC 4-component equiatomic alloy shaped like
MoNbTaW and an FCC 5-component alloy shaped like Fe29Co29Ni28Al7Ti7
(Results, nanostructure sections; Methods, Tab. 4 for the lattice sizes).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

BCC, FCC = 0, 1
BASIS_SITES = {BCC: 2, FCC: 4}
K_B_EV = 8.617333262e-5  # Boltzmann constant in eV/K (CODATA 2018)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def composition(fractions, n_sites: int) -> np.ndarray:
    """Largest-remainder rounding of species fractions to integer counts.

    floor(f_k N) each, then +1 to the largest fractional parts, ties to the
    lower species index.  Fractions are read exactly from their decimal form.
    """
    fr = [Fraction(str(f)) for f in fractions]
    if sum(fr) != 1:
        raise ValueError("fractions must sum to 1")
    exact = [f * n_sites for f in fr]
    base = [int(e) for e in exact]  # floor (all non-negative)
    left = n_sites - sum(base)
    order = sorted(range(len(fr)), key=lambda k: (-(exact[k] - base[k]), k))
    for k in order[:left]:
        base[k] += 1
    return np.array(base, dtype=np.int64)


def equiatomic(K: int, n_sites: int) -> np.ndarray:
    return composition([Fraction(1, K)] * K, n_sites)


def occupancy(counts, seed: int) -> np.ndarray:
    """Species laid out in order with the given counts, then permuted."""
    counts = np.asarray(counts, dtype=np.int64)
    occ = np.repeat(np.arange(len(counts), dtype=np.uint8), counts)
    rng(seed).shuffle(occ)
    return occ


def occupancy_device(counts, seed: int, device: str = "cuda"):
    """Large-lattice variant of :func:`occupancy` (the host shuffle of 1e9
    sites takes about a minute): a seeded ``torch.randperm`` on the device,
    site i gets the species whose cumulative-count range holds perm[i].
    Species counts are exact; the arrangement is a uniform random one.
    Returns a uint8 torch tensor on ``device``."""
    import torch
    counts = np.asarray(counts, dtype=np.int64)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    N = int(counts.sum())
    perm = torch.randperm(N, generator=g, device=device)
    bounds = torch.tensor(np.cumsum(counts), device=device)
    occ = torch.searchsorted(bounds, perm, right=True).to(torch.uint8)
    del perm
    return occ


def epi(K: int, S: int, sigma, seed: int) -> np.ndarray:
    """Symmetric V[S][K][K]: the upper triangle (k <= l, row-major) of each
    shell drawn iid N(0, sigma_s^2), then mirrored."""
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (S,))
    g = rng(seed)
    V = np.zeros((S, K, K), np.float64)
    iu = np.triu_indices(K)
    for s in range(S):
        vals = g.normal(0.0, sig[s], size=len(iu[0]))
        V[s][iu] = vals
        V[s][(iu[1], iu[0])] = vals
    return V


def beta_of_T(T) -> np.ndarray:
    """Inverse temperature in 1/eV, computed once in binary64."""
    T = np.asarray(T, dtype=np.float64)
    return 1.0 / (K_B_EV * T)


def linear_anneal(T0: float, T1: float, n: int) -> np.ndarray:
    """T_t = T0 + (T1 - T0) * t / (n - 1), t = 0 .. n-1."""
    t = np.arange(n, dtype=np.float64)
    return T0 + (T1 - T0) * t / (n - 1)


def stepwise_temperatures(T0: float = 2000.0, T1: float = 300.0, dT: float = 50.0) -> np.ndarray:
    """Annealing temperatures T0, T0 - dT, ... down to T1 (inclusive when it
    falls on the grid): the paper starts at 2000 K and lowers T by 50 K."""
    n = int(np.floor((T0 - T1) / dT + 1e-9)) + 1
    return T0 - dT * np.arange(n, dtype=np.float64)


def n_sites(lattice: int, dims) -> int:
    return int(BASIS_SITES[lattice] * int(np.prod(np.asarray(dims, dtype=np.int64))))


@dataclass
class Workload:
    """A concrete single-lattice workload."""
    name: str
    lattice: int
    dims: tuple
    K: int
    S: int
    counts: np.ndarray
    V: np.ndarray
    betas: np.ndarray  # one per sweep
    occ_seed: int
    mc_seed: int = 0
    measure_every: int = 0  # energy / SRO period in sweeps (0 = none)
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return n_sites(self.lattice, self.dims)

    def occ(self) -> np.ndarray:
        return occupancy(self.counts, self.occ_seed)


def c1_small_bcc() -> Workload:
    """BCC 8^3 (1024 sites), 4 species equiatomic, 2 shells, 1000 K, 100 sweeps."""
    dims = (8, 8, 8)
    N = n_sites(BCC, dims)
    return Workload("bcc8_k4_s2_T1000", BCC, dims, 4, 2, equiatomic(4, N),
                    epi(4, 2, 0.02, seed=1), np.full(100, beta_of_T(1000.0)), occ_seed=0)


def c2_anneal_bcc() -> Workload:
    """BCC 64^3, 4 species, 4 shells (shell-1 scale 2x), linear 3000->300 K over
    2000 sweeps; 64 snapshots for the backward pass."""
    dims = (64, 64, 64)
    N = n_sites(BCC, dims)
    n = 2000
    snaps = [((j + 1) * n) // 64 for j in range(64)]
    return Workload("bcc64_k4_s4_anneal3000to300", BCC, dims, 4, 4, equiatomic(4, N),
                    epi(4, 4, [0.04, 0.02, 0.02, 0.02], seed=2),
                    beta_of_T(linear_anneal(3000.0, 300.0, n)), occ_seed=0,
                    extra={"snapshots_after": snaps})


def c3_fcc() -> Workload:
    """FCC 128^3, 5 species 0.28/0.28/0.28/0.08/0.08, 4 shells, 800 K, 500
    sweeps, energy and SRO every 10 sweeps."""
    dims = (128, 128, 128)
    N = n_sites(FCC, dims)
    return Workload("fcc128_k5_s4_T800", FCC, dims, 5, 4,
                    composition(["0.28", "0.28", "0.28", "0.08", "0.08"], N),
                    epi(5, 4, 0.03, seed=3), np.full(500, beta_of_T(800.0)), occ_seed=0,
                    measure_every=10)


def c5_large_bcc(n_sweeps: int = 50) -> Workload:
    """BCC 800^3 (1.024e9 sites, uint8), 4 species, 4 shells, 1200 K, 50
    sweeps, SRO every 10 sweeps."""
    dims = (800, 800, 800)
    N = n_sites(BCC, dims)
    return Workload("bcc800_k4_s4_T1200", BCC, dims, 4, 4, equiatomic(4, N),
                    epi(4, 4, 0.02, seed=5), np.full(n_sweeps, beta_of_T(1200.0)), occ_seed=0,
                    measure_every=10)


def paper_large_bcc(S: int, n_sweeps: int = 5) -> Workload:
    """The paper's large BCC lattice shape (Tab. 4, MoNbTaW_1B_EPI: 795^3
    conventional cells, 1.005e9 sites) with synthetic inputs: 4 species
    equiatomic, S shells of V ~ N(0, 0.02 eV), 1200 K."""
    dims = (795, 795, 795)
    N = n_sites(BCC, dims)
    return Workload(f"bcc795_k4_s{S}_T1200", BCC, dims, 4, S, equiatomic(4, N),
                    epi(4, S, 0.02, seed=5), np.full(n_sweeps, beta_of_T(1200.0)), occ_seed=3)


@dataclass
class Ladder:
    """Batched temperature ladder: R cubic BCC replicas of uneven edge."""
    edges: np.ndarray  # [R]
    K: int
    S: int
    V: np.ndarray
    betas: np.ndarray  # [R]
    n_sweeps: int

    @property
    def R(self) -> int:
        return len(self.edges)

    def dims(self) -> np.ndarray:
        return np.stack([self.edges] * 3, axis=1).astype(np.int32)

    def occ(self, r: int) -> np.ndarray:
        N = n_sites(BCC, (self.edges[r],) * 3)
        return occupancy(equiatomic(self.K, N), 1000 + r)


def c4a_ladder(R: int = 256, n_sweeps: int = 1000, lo: int = 16, hi: int = 48) -> Ladder:
    """R cubic BCC replicas, edges iid uniform in [lo, hi], T_r = 300 * 10^(r/(R-1)) K."""
    edges = rng(8).integers(lo, hi + 1, size=R)
    r = np.arange(R, dtype=np.float64)
    T = 300.0 * 10.0 ** (r / max(R - 1, 1))
    return Ladder(edges.astype(np.int32), 4, 4, epi(4, 4, 0.02, seed=4), beta_of_T(T), n_sweeps)


def qsro_fcc(edge: int = 64):
    """FCC edge^3 (1,048,576 sites at 64), 5 species 0.28/0.28/0.28/0.08/0.08,
    2 shells, 1000 K: shaped like the paper's one-million-atom FeCoNiAlTi
    runs with its qSRO model.  Returns (dims, counts, V [2][5][5],
    W [2][5], beta)."""
    dims = (edge, edge, edge)
    N = n_sites(FCC, dims)
    counts = composition([0.28, 0.28, 0.28, 0.08, 0.08], N)
    V = epi(5, 2, 0.03, seed=3)
    W = rng(9).normal(0.0, 0.05, (2, 5))
    return dims, counts, V, W, float(beta_of_T(1000.0))


def tempering_ladder(R: int = 256, edge: int = 32, n_sweeps: int = 1000) -> Ladder:
    """R cubic BCC replicas of one edge for replica exchange (the ladder's
    temperatures and EPI; the edge is the mean of its 16..48 range)."""
    r = np.arange(R, dtype=np.float64)
    T = 300.0 * 10.0 ** (r / max(R - 1, 1))
    return Ladder(np.full(R, edge, np.int32), 4, 4, epi(4, 4, 0.02, seed=4), beta_of_T(T), n_sweeps)


def c4b_fit_set(B: int = 4096, edge: int = 16):
    """Random equiatomic BCC configurations and a seeded teacher V*."""
    dims = (edge, edge, edge)
    N = n_sites(BCC, dims)
    g = rng(7)
    counts = equiatomic(4, N)
    base = np.repeat(np.arange(4, dtype=np.uint8), counts)
    occs = np.empty((B, N), np.uint8)
    for b in range(B):
        occs[b] = g.permutation(base)
    V_teacher = epi(4, 4, 0.02, seed=6)
    return dims, occs, V_teacher
