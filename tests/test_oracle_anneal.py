"""Pins of the oracle's heat capacity and stepwise-anneal driver (CPU only).

c = beta^2 Var(E) / N per site, in units of k_B (canonical fluctuation
formula).  Pinned by closed forms (constant and two-level series), by the
exact heat capacity of the 16-site BCC cell from enumeration against a long
chain, and by the driver's sweep numbering against the loop written out.
"""
import math

import numpy as np

import brute
from paper_2503_12591_amd import inputs as I

BCC = 0
KB = 8.617333262e-5


def test_heat_capacity_closed_forms(oracle):
    assert oracle.heat_capacity(np.full(7, -3.25), 5.0, 16) == 0.0
    # E alternates m - a, m + a: Var = a^2 exactly
    E = np.array([2.5, 3.5] * 4)
    assert oracle.heat_capacity(E, 4.0, 8) == 16.0 * 0.25 / 8
    # one value in n away from the rest: Var = (n - 1) d^2 / n^2
    E = np.array([0.0, 0.0, 0.0, 4.0])
    assert oracle.heat_capacity(E, 1.0, 1) == 3.0


def sixteen_site_cell():
    dims, K, S = (2, 2, 2), 2, 2
    V = np.zeros((S, K, K))
    V[0, 0, 1] = V[0, 1, 0] = 0.05
    V[1, 0, 1] = V[1, 1, 0] = -0.03
    V[0, 1, 1] = 0.01
    return dims, K, S, V


def test_heat_capacity_exact_sixteen_site_cell(oracle):
    """Exact c(T) from the C(16,8) levels against one anneal step (warm-up,
    then 24000 recorded sweeps) at 1500 K; tolerance from 24 batch values."""
    dims, K, S, V = sixteen_site_cell()
    nbr = brute.neighbour_table(BCC, dims, S)
    levels = brute.energies_batch(nbr, brute.all_configs(16, 8), V)
    T = 1500.0
    beta = 1.0 / (KB * T)
    w = np.exp(-beta * (levels - levels.min()))
    w /= w.sum()
    mean = float((levels * w).sum())
    exact = beta * beta * float((((levels - mean) ** 2) * w).sum()) / 16
    occ = np.array([0, 1] * 8, np.uint8)
    cells = oracle.default_cells(dims, 3)
    out = oracle.anneal(BCC, dims, K, S, cells, occ, V, seed=17, beta_steps=[beta], warmup=300,
                        record=24000)
    c = out["cv"][0]
    batches = np.array([oracle.heat_capacity(b, beta, 16) for b in np.array_split(out["E"][0], 24)])
    err = batches.std(ddof=1) / math.sqrt(len(batches))
    assert abs(c - exact) < 4 * err, (c, exact, err)
    assert exact > 0.05  # the case is not trivially flat


def test_anneal_driver_matches_loop(oracle):
    dims, K, S, V = sixteen_site_cell()
    cells = oracle.default_cells(dims, 3)
    betas = 1.0 / (KB * np.array([2000.0, 1950.0, 1900.0]))
    a = np.array([0, 1] * 8, np.uint8)
    b = a.copy()
    out = oracle.anneal(BCC, dims, K, S, cells, a, V, seed=4, beta_steps=betas, warmup=3, record=5,
                        first_sweep=10)
    t = 10
    for s, beta in enumerate(betas):
        oracle.run(BCC, dims, K, S, cells, b, V, 4, np.full(3, beta), first_sweep=t)
        t += 3
        E = []
        for j in range(5):
            oracle.run(BCC, dims, K, S, cells, b, V, 4, [beta], first_sweep=t)
            t += 1
            E.append(oracle.energy(oracle.pair_counts(BCC, dims, K, S, b), V))
        assert np.array_equal(out["E"][s], np.array(E))
        assert out["cv"][s] == oracle.heat_capacity(np.array(E), beta, 16)
    assert np.array_equal(a, b)


def test_stepwise_temperatures_follow_the_paper():
    T = I.stepwise_temperatures(2000.0, 1000.0, 50.0)
    assert len(T) == 21 and T[0] == 2000.0 and T[-1] == 1000.0
    assert np.all(np.diff(T) == -50.0)
    assert I.stepwise_temperatures(2000.0, 300.0)[-1] == 300.0
