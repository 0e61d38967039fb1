"""Pins of the oracle's geometry and schedule (CPU only).

Coordination shells against textbook coordination numbers and brute-force
distance sorting; the link-cell rule against the link cells printed in the
paper (Methods, Tab. 4 and the 300^3 worked example); schedule coverage and
mini-step independence by brute force over read and write sets.
"""
import os

import numpy as np
import pytest

import brute

HERE = os.path.dirname(os.path.abspath(__file__))
BCC, FCC = 0, 1


def read_lattices():
    rows = []
    with open(os.path.join(HERE, "golden", "paper_lattices.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            rows.append(dict(name=p[0], lattice=BCC if p[1] == "BCC" else FCC,
                             dims=(int(p[2]), int(p[3]), int(p[4])), m=int(p[5]), model=p[6],
                             shells=int(p[7]), link=int(p[8]), N=int(p[9]), nA=int(p[10]),
                             nC=None if p[11] == "-" else int(p[11])))
    return rows


def test_textbook_coordination(oracle):
    Zb, _ = oracle.shells(BCC, 4)
    Zf, _ = oracle.shells(FCC, 4)
    assert list(Zb) == [8, 6, 12, 24]
    assert list(Zf) == [12, 6, 24, 12]


@pytest.mark.parametrize("lattice", [BCC, FCC])
def test_shells_match_distance_sort(oracle, lattice):
    Z, vecs = oracle.shells(lattice, 4)
    radii, bvecs = brute.shell_vectors(lattice, 4)
    exp_r2 = {BCC: [3, 4, 8, 11], FCC: [2, 4, 6, 8]}[lattice]
    assert list(radii) == exp_r2
    for s in range(4):
        got = [tuple(v) for v in vecs[s]]
        assert got == sorted(got), "shell vectors must be in lexicographic order"
        assert set(got) == set(map(tuple, bvecs[s]))
        assert all(v[0] ** 2 + v[1] ** 2 + v[2] ** 2 == exp_r2[s] for v in got)


def test_site_counts_of_paper_cells():
    for row in read_lattices():
        nx, ny, nz = row["dims"]
        assert nx * ny * nz * row["m"] == row["N"], row["name"]


def test_link_cell_rule_reproduces_paper(oracle):
    for row in read_lattices():
        ell = oracle.lmin(row["lattice"], row["shells"], liz=row["model"] == "liz")
        assert ell == row["link"], row["name"]
        assert ell ** 3 * row["m"] == row["nA"], row["name"]


def test_worked_example_partition(oracle):
    row = [r for r in read_lattices() if r["name"] == "worked_example_300"][0]
    cells = oracle.default_cells(row["dims"], row["link"])
    nC = int(np.prod([len(c) for c in cells]))
    nA = int(np.prod([max(c) for c in cells])) * row["m"]
    assert nC == row["nC"] and nA == row["nA"]


@pytest.mark.parametrize("L,ell", [(8, 4), (17, 4), (11, 4), (7, 4), (800, 3), (800, 4), (19, 3)])
def test_default_partition_rule(oracle, L, ell):
    sizes = oracle.partition(L, ell)
    assert sizes.sum() == L
    n = max(1, L // ell)
    assert len(sizes) == n
    assert sizes.max() - sizes.min() <= 1
    if n > 1:
        assert sizes.min() >= ell


def _mini_step_of_site(lattice, dims, cells):
    """Independent recomputation of each site's mini-step from the partition."""
    m = 2 if lattice == BCC else 4
    pos = brute.positions(lattice, dims)
    b = np.arange(len(pos)) % m
    conv = (pos - brute.BASIS[lattice][b]) // 2
    M = [max(c) for c in cells]
    off = []
    for a in range(3):
        origin = np.concatenate([[0], np.cumsum(cells[a])[:-1]])
        cell_of = np.searchsorted(np.cumsum(cells[a]), conv[:, a], side="right")
        off.append(conv[:, a] - origin[cell_of])
    return b + m * (off[0] + M[0] * (off[1] + M[1] * off[2]))


def _trace_sweep(oracle, lattice, dims, K, S, cells, seed=3):
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    g = np.random.default_rng(seed)
    occ = g.integers(0, K, N).astype(np.uint8)
    V = np.zeros((S, K, K))
    res = oracle.run(lattice, dims, K, S, cells, occ, V, seed=11, betas=[1.0], trace=True)
    return res.trace


@pytest.mark.parametrize("lattice,dims,ell", [(BCC, (8, 8, 8), 4), (FCC, (6, 7, 9), 3),
                                              (BCC, (9, 10, 7), 3), (FCC, (5, 4, 4), 4)])
def test_schedule_covers_each_site_once_in_order(oracle, lattice, dims, ell):
    S, K = 2, 3
    cells = oracle.default_cells(dims, ell)
    tr = _trace_sweep(oracle, lattice, dims, K, S, cells)
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    assert len(tr) == N
    assert np.array_equal(np.sort(tr["a"]), np.arange(N))  # one trial per site (a sweep)
    tau = _mini_step_of_site(lattice, dims, cells)[tr["a"]]
    assert (np.diff(tau) >= 0).all(), "mini-steps must run in ascending order"


def _read_write_sets(lattice, dims, S):
    """Per site: the set of sites a trial there may read (its neighbours, every
    possible partner, the partners' neighbours) and may write (itself and
    every possible partner)."""
    nbr = brute.neighbour_table(lattice, dims, S)
    allnb = np.concatenate(nbr, axis=1)
    reads, writes = [], []
    for a in range(allnb.shape[0]):
        partners = nbr[0][a]
        r = set(allnb[a]) | set(partners) | {a}
        for b in partners:
            r |= set(allnb[b])
        reads.append(r)
        writes.append({a} | set(partners))
    return reads, writes


def _conflicts(lattice, dims, S, cells):
    reads, writes = _read_write_sets(lattice, dims, S)
    tau = _mini_step_of_site(lattice, dims, cells)
    bad = 0
    for t in np.unique(tau):
        act = np.nonzero(tau == t)[0]
        for i in act:
            for j in act:
                if i != j and (writes[j] & reads[i]):
                    bad += 1
    return bad


@pytest.mark.parametrize("lattice,dims,S", [(BCC, (9, 10, 6), 4), (FCC, (6, 7, 6), 4),
                                            (BCC, (7, 6, 6), 2), (FCC, (7, 6, 6), 2)])
def test_link_cell_rule_is_sufficient(oracle, lattice, dims, S):
    """Every pair of trials of one mini-step is independent (uneven partitions
    included), with cells at the minimum edge."""
    ell = oracle.lmin(lattice, S)
    cells = oracle.default_cells(dims, ell)
    assert _conflicts(lattice, dims, S, cells) == 0


@pytest.mark.parametrize("lattice,S", [(BCC, 4), (FCC, 4), (BCC, 2), (FCC, 2)])
def test_link_cell_rule_is_tight(oracle, lattice, S):
    """One conventional cell less than the rule gives conflicting trials."""
    ell = oracle.lmin(lattice, S) - 1
    dims = (3 * ell, 2 * ell, 2 * ell)
    cells = [np.full(3, ell, np.int32), np.full(2, ell, np.int32), np.full(2, ell, np.int32)]
    assert _conflicts(lattice, dims, S, cells) > 0


@pytest.mark.parametrize("lattice,dims,ell", [(BCC, (8, 9, 8), 4), (FCC, (7, 6, 6), 3)])
def test_ministep_ranges_compose_to_a_sweep(oracle, lattice, dims, ell):
    K, S = 4, 4
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ0 = np.random.default_rng(2).integers(0, K, N).astype(np.uint8)
    V = np.random.default_rng(3).normal(0, 0.05, (S, K, K))
    V = V + V.transpose(0, 2, 1)
    cells = oracle.default_cells(dims, ell)
    nA = int(np.prod([max(c) for c in cells])) * (2 if lattice == BCC else 4)
    full = occ0.copy()
    r_full = oracle.run(lattice, dims, K, S, cells, full, V, seed=4, betas=[6.0], first_sweep=2)
    part = occ0.copy()
    att = acc = 0
    for lo, hi in [(0, 5), (5, 6), (6, nA)]:
        r = oracle.run_ministeps(lattice, dims, K, S, cells, part, V, seed=4, beta=6.0, sweep=2,
                                 tau_begin=lo, tau_end=hi, nthreads=1 + lo % 3)
        att += r.stats[0]
        acc += r.stats[1]
    assert np.array_equal(full, part)
    assert att == r_full.stats[0] and acc == r_full.stats[1]
