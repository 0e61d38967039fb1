"""Pins of the oracle's near-tie protocol on forced ties.

A trial (or an exchange) whose uniform u lies within 1e-12 of its acceptance
probability is a near-tie: it is logged as {replica, sweep, site,
decision}, and a replayed decision for exactly those keys replaces the
oracle's own (Supplementary, "Monte Carlo Simulation Algorithms", the
acceptance rule; the window and the replay are this library's convention
for comparing trajectories whose exp differs in the last place).  Random
inputs never produce one, so each test builds one (tests/ties.py): a trial
of mini-step 0 and the beta that puts exp(-beta dE) on its u.

These pin the replay branch: flipping the replayed decision at a real tie
flips exactly that swap, an entry under any other key changes nothing, and
the log holds the decision that was taken.
"""
import math

import numpy as np
import pytest

from ties import forced_exchange_tie, forced_trial_tie
from oracle import oracle as O
from paper_2503_12591_amd import inputs as I

BCC, FCC = 0, 1


def tie_entry(replica, sweep, site, decision):
    e = np.zeros(1, O.TIE_DTYPE)
    e[0]["replica"], e[0]["sweep"], e[0]["site"], e[0]["decision"] = replica, sweep, site, decision
    return e


def small_case(edge=8):
    """The BCC 8^3 parity workload (4 species, 2 shells), or the same model on
    a larger cube (more link cells, so more candidate trials)."""
    w = I.c1_small_bcc()
    if edge != 8:
        w.dims = (edge, edge, edge)
        w.counts = I.equiatomic(w.K, I.n_sites(w.lattice, w.dims))
    cells = O.default_cells(w.dims, 4)
    return w, cells, w.occ()


def test_forced_trial_tie_is_logged():
    w, cells, occ0 = small_case()
    t = forced_trial_tie(w.lattice, w.dims, w.K, w.S, cells, occ0, w.V, seed=11, replica=0, sweep=3)
    occ = occ0.copy()
    res = O.run(w.lattice, w.dims, w.K, w.S, cells, occ, w.V, 11, [t["beta"]], first_sweep=3)
    assert res.n_ties == 1 and res.stats[2] == 1
    e = res.ties[0]
    own = int(t["u"] < t["P"])  # the oracle's exp is the C library's, as math.exp
    assert (int(e["replica"]), int(e["sweep"]), int(e["site"]), int(e["decision"])) == (0, 3, t["site"], own)


def ministep0(w, cells, occ0, t, replay=None, sweep=3, replica=0):
    occ = occ0.copy()
    res = O.run_ministeps(w.lattice, w.dims, w.K, w.S, cells, occ, w.V, 11, t["beta"], sweep, 0, 1,
                          replica=replica, replay=replay)
    return occ, res


def test_replay_flips_exactly_the_tied_swap():
    w, cells, occ0 = small_case()
    t = forced_trial_tie(w.lattice, w.dims, w.K, w.S, cells, occ0, w.V, seed=11, replica=0, sweep=3)
    own_occ, own = ministep0(w, cells, occ0, t)
    d0 = int(own.ties[0]["decision"])
    same_occ, same = ministep0(w, cells, occ0, t, replay=tie_entry(0, 3, t["site"], d0))
    assert np.array_equal(same_occ, own_occ) and same.stats.tolist() == own.stats.tolist()
    flip_occ, flip = ministep0(w, cells, occ0, t, replay=tie_entry(0, 3, t["site"], 1 - d0))
    diff = np.flatnonzero(flip_occ != own_occ)
    assert sorted(diff.tolist()) == sorted([t["site"], t["partner"]])
    assert flip.stats[1] - own.stats[1] == (1 if d0 == 0 else -1)
    assert int(flip.ties[0]["decision"]) == 1 - d0  # the log holds the decision taken
    # the swap of the flipped run is the tied pair's exchange of species
    swapped = own_occ if d0 == 1 else flip_occ
    assert swapped[t["site"]] == occ0[t["partner"]] and swapped[t["partner"]] == occ0[t["site"]]


def test_replay_under_other_keys_is_ignored():
    w, cells, occ0 = small_case()
    t = forced_trial_tie(w.lattice, w.dims, w.K, w.S, cells, occ0, w.V, seed=11, replica=0, sweep=3)
    own_occ, own = ministep0(w, cells, occ0, t)
    d1 = 1 - int(own.ties[0]["decision"])
    for key in [(1, 3, t["site"]), (0, 4, t["site"]), (0, 2, t["site"]), (0, 3, t["site"] + 2),
                (0, 3, t["partner"])]:
        occ, res = ministep0(w, cells, occ0, t, replay=tie_entry(*key, d1))
        assert np.array_equal(occ, own_occ), key
        assert res.stats.tolist() == own.stats.tolist(), key


def test_replay_keyed_by_replica_and_sweep():
    """The same site tied in another replica and sweep: only the entry with
    that replica and sweep applies."""
    w, cells, occ0 = small_case(16)
    t = forced_trial_tie(w.lattice, w.dims, w.K, w.S, cells, occ0, w.V, seed=11, replica=5, sweep=9)
    own_occ, own = ministep0(w, cells, occ0, t, sweep=9, replica=5)
    assert own.n_ties == 1
    d1 = 1 - int(own.ties[0]["decision"])
    flip_occ, _ = ministep0(w, cells, occ0, t, sweep=9, replica=5, replay=tie_entry(5, 9, t["site"], d1))
    assert sorted(np.flatnonzero(flip_occ != own_occ).tolist()) == sorted([t["site"], t["partner"]])
    for key in [(0, 9, t["site"]), (5, 0, t["site"])]:
        occ, _ = ministep0(w, cells, occ0, t, sweep=9, replica=5, replay=tie_entry(*key, d1))
        assert np.array_equal(occ, own_occ), key


def test_forced_tie_in_a_full_sweep_fcc():
    """FCC, 5 species, 4 shells: the tie is logged once in a full sweep, and a
    flipped replay gives another trajectory whose log holds the flipped
    decision."""
    dims, K, S = (6, 5, 7), 5, 4
    occ0 = I.occupancy(I.equiatomic(K, 4 * 210), 3)
    V = I.epi(K, S, 0.03, 3)
    cells = O.default_cells(dims, 3)
    t = forced_trial_tie(FCC, dims, K, S, cells, occ0, V, seed=2, replica=0, sweep=1)
    a = occ0.copy()
    ra = O.run(FCC, dims, K, S, cells, a, V, 2, [t["beta"]], first_sweep=1)
    assert ra.n_ties == 1 and int(ra.ties[0]["site"]) == t["site"]
    d1 = 1 - int(ra.ties[0]["decision"])
    b = occ0.copy()
    rb = O.run(FCC, dims, K, S, cells, b, V, 2, [t["beta"]], first_sweep=1, replay=tie_entry(0, 1, t["site"], d1))
    assert not np.array_equal(a, b)
    assert int(rb.ties[0]["decision"]) == d1
    assert np.array_equal(np.bincount(a, minlength=K), np.bincount(b, minlength=K))


def test_forced_qsro_tie():
    dims, K, S = (8, 8, 8), 4, 2
    occ0 = I.occupancy(I.equiatomic(K, 2 * 512), 4)
    V = I.epi(K, S, 0.05, 21)
    W = np.random.default_rng(22).normal(0, 0.2, (S, K))
    cells = O.default_cells(dims, 4)
    t = forced_trial_tie(BCC, dims, K, S, cells, occ0, V, seed=5, replica=0, sweep=2, W=W)
    a = occ0.copy()
    ra = O.run_qsro(BCC, dims, K, S, cells, a, V, W, 5, [t["beta"]], first_sweep=2)
    assert ra.n_ties == 1
    e = ra.ties[0]
    assert (int(e["replica"]), int(e["sweep"]), int(e["site"])) == (0, 2, t["site"])
    assert int(e["decision"]) == int(t["u"] < t["P"])
    b = occ0.copy()
    rb = O.run_qsro(BCC, dims, K, S, cells, b, V, W, 5, [t["beta"]], first_sweep=2,
                    replay=tie_entry(0, 2, t["site"], 1 - int(e["decision"])))
    assert not np.array_equal(a, b)
    assert int(rb.ties[0]["decision"]) == 1 - int(e["decision"])


@pytest.fixture
def exchange_case():
    R = 6
    E = np.random.default_rng(3).normal(-50.0, 2.0, R)
    beta = 1.0 / (I.K_B_EV * np.geomspace(600.0, 1500.0, R))
    rep_at = np.array([3, 0, 5, 1, 4, 2], np.int32)  # a slot need not hold its own replica
    bs, u, x = forced_exchange_tie(E, beta, rep_at, seed=9, round_=0, pair=2)
    return E, bs, rep_at, u, x


def test_forced_exchange_tie_is_logged(exchange_case):
    E, bs, rep_at, u, x = exchange_case
    ra = rep_at.copy()
    ties, nt = O.exchange(E, bs, ra, seed=9, round_=0)
    assert nt == 1
    e = ties[0]
    own = int(u < math.exp(x))
    assert (int(e["replica"]), int(e["sweep"]), int(e["site"]), int(e["decision"])) == (-1, 0, 2, own)


def test_exchange_replay_flips_the_tied_pair(exchange_case):
    E, bs, rep_at, u, x = exchange_case
    own = rep_at.copy()
    ties, _ = O.exchange(E, bs, own, seed=9, round_=0)
    d1 = 1 - int(ties[0]["decision"])
    flip = rep_at.copy()
    st = np.zeros((5, 2), np.int64)
    fties, _ = O.exchange(E, bs, flip, seed=9, round_=0, replay=tie_entry(-1, 0, 2, d1), stats=st)
    assert sorted(np.flatnonzero(flip != own).tolist()) == [2, 3]
    assert int(fties[0]["decision"]) == d1
    assert st[2, 0] == 1 and st[2, 1] == d1
    # entries under other keys: another round, a replica's index instead of
    # the slot's, a trial's replica field
    for key in [(-1, 1, 2), (-1, 0, int(rep_at[2])), (0, 0, 2), (-1, 0, 3)]:
        ra = rep_at.copy()
        O.exchange(E, bs, ra, seed=9, round_=0, replay=tie_entry(*key, d1))
        assert np.array_equal(ra, own), key
