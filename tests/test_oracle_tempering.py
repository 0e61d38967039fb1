"""Pins of the oracle's replica exchange (parallel tempering), CPU only.

The exchange rule is the textbook one (Swendsen and Wang 1986; Hukushima and
Nemoto 1996): slots i and i + 1 trade replicas with probability
min(1, exp((beta_i - beta_{i+1}) (E_i - E_{i+1}))).  Pinned by
  - special cases: x >= 0 always trades, round parity picks the pairs, the
    slot -> replica map stays a permutation, stats count every attempt;
  - the acceptance frequency of a trade at frozen energies equals exp(x);
  - tempering on the 16-site BCC cell leaves every slot's energy distributed
    canonically at that slot's temperature (exact enumeration).
"""
import math

import numpy as np
import pytest

import brute

BCC = 0
KB = 8.617333262e-5


def test_exchange_special_cases(oracle):
    beta = np.array([1.0, 2.0, 3.0, 4.0])
    rep_at = np.arange(4, dtype=np.int32)
    stats = np.zeros((3, 2), np.int64)
    # round 0 pairs (0,1) and (2,3): x = (1-2)(1-3) = 2 and (3-4)(0.5-2) = 1.5,
    # both >= 0, so both trade
    E = np.array([1.0, 3.0, 0.5, 2.0])
    ties, nt = oracle.exchange(E, beta, rep_at, seed=5, round_=0, stats=stats)
    assert nt == 0
    assert rep_at.tolist() == [1, 0, 3, 2]
    assert stats.tolist() == [[1, 1], [0, 0], [1, 1]]
    # round 1: only pair (1, 2), which now holds replicas 0 and 3
    # x = (2-3)(E[0] - E[3]) = -(1 - 2) = 1 >= 0 -> trade
    oracle.exchange(E, beta, rep_at, seed=5, round_=1, stats=stats)
    assert rep_at.tolist() == [1, 3, 0, 2]
    assert stats.tolist() == [[1, 1], [1, 1], [1, 1]]
    assert sorted(rep_at.tolist()) == [0, 1, 2, 3]
    # equal temperatures: x = 0, every pair trades whatever the energies
    r2 = np.arange(5, dtype=np.int32)
    oracle.exchange(np.array([5.0, -1.0, 2.0, 9.0, 0.0]), np.full(5, 7.0), r2, seed=1, round_=0)
    assert r2.tolist() == [1, 0, 3, 2, 4]
    # one replica: nothing to trade
    r1 = np.zeros(1, np.int32)
    oracle.exchange(np.array([1.0]), np.array([1.0]), r1, seed=1, round_=0)
    assert r1.tolist() == [0]
    with pytest.raises(ValueError):
        oracle.exchange(E, beta, np.array([0, 1, 2, 7], np.int32), seed=1, round_=0)


def test_exchange_acceptance_frequency(oracle):
    """At frozen energies a trade with x < 0 happens with probability exp(x)."""
    beta = np.array([2.0, 1.0])
    E = np.array([1.0, 1.5])  # x = (2 - 1)(1 - 1.5) = -0.5
    p = math.exp(-0.5)
    n = 6000
    acc = 0
    for j in range(n):
        rep_at = np.arange(2, dtype=np.int32)
        oracle.exchange(E, beta, rep_at, seed=11, round_=2 * j)  # even rounds pair (0, 1)
        acc += int(rep_at[0] == 1)
    assert abs(acc / n - p) < 5 * math.sqrt(p * (1 - p) / n), (acc / n, p)


def sixteen_site_cell():
    dims, K, S = (2, 2, 2), 2, 2
    V = np.zeros((S, K, K))
    V[0, 0, 1] = V[0, 1, 0] = 0.05
    V[1, 0, 1] = V[1, 1, 0] = -0.03
    V[0, 1, 1] = 0.01
    return dims, K, S, V


def test_tempering_slots_sample_their_temperature(oracle):
    """Three slots at 700, 1500, 3000 K over three replicas of the 16-site
    cell: after every exchange round the replica held by slot i is a sample of
    the canonical distribution at T_i, so each slot's mean energy matches the
    exact <E>(T_i), and trades happen on both pairs."""
    dims, K, S, V = sixteen_site_cell()
    nbr = brute.neighbour_table(BCC, dims, S)
    occs_all = brute.all_configs(16, 8)
    levels = brute.energies_batch(nbr, occs_all, V)
    Ts = np.array([700.0, 1500.0, 3000.0])
    beta = 1.0 / (KB * Ts)
    exact = []
    for b in beta:
        w = np.exp(-b * (levels - levels.min()))
        exact.append(float((levels * w).sum() / w.sum()))
    cells = oracle.default_cells(dims, 3)
    occs = [np.array([0, 1] * 8, np.uint8) for _ in range(3)]
    rep_at = np.arange(3, dtype=np.int32)
    xst = np.zeros((2, 2), np.int64)
    slot_E = []
    n_rounds = 4000
    for j in range(n_rounds):
        slot_of = np.empty(3, np.int64)
        slot_of[rep_at] = np.arange(3)
        for r in range(3):
            oracle.run(BCC, dims, K, S, cells, occs[r], V, seed=3, betas=[beta[slot_of[r]]],
                       first_sweep=j, replica=r)
        E = np.array([oracle.energy(oracle.pair_counts(BCC, dims, K, S, o), V) for o in occs])
        oracle.exchange(E, beta, rep_at, seed=3, round_=j, stats=xst)
        slot_E.append(E[rep_at])
    slot_E = np.array(slot_E)[200:]
    for i in range(3):
        b = np.array_split(slot_E[:, i], 20)
        means = np.array([x.mean() for x in b])
        m, err = means.mean(), means.std(ddof=1) / math.sqrt(len(b))
        assert abs(m - exact[i]) < 4 * err + 1e-12, (i, m, exact[i], err)
    assert (xst[:, 1] > 0).all() and (xst[:, 1] < xst[:, 0]).all()
    assert xst[0, 0] == n_rounds // 2 and xst[1, 0] == n_rounds // 2
    for o in occs:
        assert np.bincount(o, minlength=2).tolist() == [8, 8]


def test_tempering_driver_matches_manual_rounds(oracle):
    """oracle.tempering runs the same rounds as the loop written out."""
    dims, K, S, V = sixteen_site_cell()
    cells = oracle.default_cells(dims, 3)
    beta = 1.0 / (KB * np.array([800.0, 1600.0]))
    occs_a = [np.array([0, 1] * 8, np.uint8), np.array([1, 0] * 8, np.uint8)]
    occs_b = [o.copy() for o in occs_a]
    out = oracle.tempering(BCC, dims, K, S, cells, occs_a, V, seed=9, beta_slot=beta, n_rounds=7,
                           sweeps_per_round=3)
    rep_at = np.arange(2, dtype=np.int32)
    for j in range(7):
        slot_of = np.empty(2, np.int64)
        slot_of[rep_at] = np.arange(2)
        for r in range(2):
            oracle.run(BCC, dims, K, S, cells, occs_b[r], V, seed=9,
                       betas=np.full(3, beta[slot_of[r]]), first_sweep=3 * j, replica=r)
        E = np.array([oracle.energy(oracle.pair_counts(BCC, dims, K, S, o), V) for o in occs_b])
        assert np.array_equal(E, out["energies"][j])
        oracle.exchange(E, beta, rep_at, seed=9, round_=j)
    assert np.array_equal(rep_at, out["rep_at"])
    for a, b in zip(occs_a, occs_b):
        assert np.array_equal(a, b)
