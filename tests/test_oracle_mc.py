"""Pins of the oracle's Metropolis swap chain (CPU only).

(i)   every traced trial: dE equals the brute-force energy difference, and the
      pair-model rule dE = 2 (de_a + de_b) on local energies holds;
(ii)  exact canonical <E> on the 16-site BCC cell by enumeration;
(iii) composition is conserved;
(iv)  detailed balance: the joint (x, y) table of one single-site trial from
      exact samples of pi is symmetric, and the long-chain energy histogram
      matches g(E) exp(-beta E) / Z;
(v)   beta = 0: mean Warren-Cowley SRO equals its exact finite-N expectation.
Plus the closed-form B2 ground state of an unlike-attracting binary.
"""
import math

import numpy as np
import pytest
from scipy import stats

import brute

BCC, FCC = 0, 1
KB = 8.617333262e-5


def sym_V(S, K, scale, seed):
    V = np.random.default_rng(seed).normal(0, scale, (S, K, K))
    return 0.5 * (V + V.transpose(0, 2, 1))


@pytest.mark.parametrize("lattice,dims,K,S,ell,beta", [
    (BCC, (8, 8, 8), 4, 2, 4, 11.6),     # shaped like the small BCC parity case
    (FCC, (4, 4, 5), 5, 4, 3, 14.5),
    (BCC, (3, 4, 3), 3, 4, 3, 5.0),
])
def test_delta_e_matches_recomputation(oracle, lattice, dims, K, S, ell, beta):
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ0 = np.random.default_rng(1).integers(0, K, N).astype(np.uint8)
    V = sym_V(S, K, 0.05, 2)
    cells = oracle.default_cells(dims, ell)
    occ = occ0.copy()
    res = oracle.run(lattice, dims, K, S, cells, occ, V, seed=5, betas=[beta] * 2, trace=True)
    nbr = brute.neighbour_table(lattice, dims, S)
    cur = occ0.copy()
    E = brute.energy_from_table(nbr, cur, V)
    n_checked = 0
    for tr in res.trace:
        a, b = int(tr["a"]), int(tr["b"])
        p, q = cur[a], cur[b]
        if p == q:
            assert tr["dE"] == 0.0 and tr["accepted"] == 0
            continue
        new = cur.copy()
        new[a], new[b] = q, p
        E_new = brute.energy_from_table(nbr, new, V)
        assert abs(tr["dE"] - (E_new - E)) <= 1e-12 * max(1.0, abs(E)), (a, b)
        de_loc = (brute.local_energy(nbr, new, V, a) - brute.local_energy(nbr, cur, V, a) +
                  brute.local_energy(nbr, new, V, b) - brute.local_energy(nbr, cur, V, b))
        assert abs(tr["dE"] - 2.0 * de_loc) <= 1e-12 * max(1.0, abs(E))
        n_checked += 1
        if tr["accepted"]:
            cur, E = new, E_new
    assert np.array_equal(cur, occ)
    assert n_checked > len(res.trace) // 3


def test_acceptance_rule_on_trace(oracle):
    """dE <= 0 always accepted; dE > 0 accepted with the Metropolis frequency."""
    lattice, dims, K, S = BCC, (8, 8, 8), 4, 2
    N = 1024
    occ = np.random.default_rng(4).integers(0, K, N).astype(np.uint8)
    V = sym_V(S, K, 0.05, 7)
    beta = 8.0
    res = oracle.run(lattice, dims, K, S, oracle.default_cells(dims, 4), occ, V, seed=1,
                     betas=[beta] * 20, trace=True)
    tr = res.trace
    moved = tr["dE"] != 0.0
    down = tr[moved & (tr["dE"] <= 0)]
    assert (down["accepted"] == 1).all()
    up = tr[tr["dE"] > 0]
    p = np.exp(-beta * up["dE"])
    # sum of Bernoulli(p): accepted count within 5 sigma of its mean
    assert abs(up["accepted"].sum() - p.sum()) < 5 * math.sqrt((p * (1 - p)).sum())
    assert res.stats[0] == 20 * N


def sixteen_site_cell():
    """BCC 2x2x2 conventional cells, 2 species 8/8, shells 1-2 (shell 2 sees
    each neighbour twice through the periodic images)."""
    dims, K, S = (2, 2, 2), 2, 2
    V = np.zeros((S, K, K))
    V[0, 0, 1] = V[0, 1, 0] = 0.05
    V[1, 0, 1] = V[1, 1, 0] = -0.03
    V[0, 1, 1] = 0.01
    return dims, K, S, V


def exact_levels(dims, K, S, V):
    nbr = brute.neighbour_table(BCC, dims, S)
    occs = brute.all_configs(16, 8)
    E = brute.energies_batch(nbr, occs, V)
    return occs, E


def test_enumeration_size_and_ground_state():
    """C(16,8) states; with only an unlike nearest-neighbour attraction v < 0
    the minimum is the B2 arrangement, E_min = N Z1 v / 2."""
    dims, S = (2, 2, 2), 1
    V = np.zeros((S, 2, 2))
    v = -0.1
    V[0, 0, 1] = V[0, 1, 0] = v
    occs, E = exact_levels(dims, 2, S, V)
    assert len(occs) == 12870
    assert np.isclose(E.min(), 0.5 * 16 * 8 * v)
    gs = occs[np.argmin(E)]
    assert len(set(gs[0::2])) == 1 and len(set(gs[1::2])) == 1  # sublattice order


def batch_mean_err(x, n_batches=20):
    b = np.array_split(np.asarray(x), n_batches)
    means = np.array([bb.mean() for bb in b])
    return means.mean(), means.std(ddof=1) / math.sqrt(n_batches)


def chain_energies(oracle, dims, K, S, V, beta, n_sweeps, seed, thin=1):
    occ = np.array([0, 1] * 8, np.uint8)
    cells = oracle.default_cells(dims, 3)
    out = []
    for t in range(n_sweeps):
        oracle.run(BCC, dims, K, S, cells, occ, V, seed=seed, betas=[beta], first_sweep=t)
        if t % thin == 0:
            out.append(oracle.energy(oracle.pair_counts(BCC, dims, K, S, occ), V))
    return np.array(out), occ


@pytest.mark.parametrize("T", [700.0, 1000.0, 3000.0])
def test_exact_canonical_mean_energy(oracle, T):
    dims, K, S, V = sixteen_site_cell()
    _, E = exact_levels(dims, K, S, V)
    beta = 1.0 / (KB * T)
    w = np.exp(-beta * (E - E.min()))
    exact = float((E * w).sum() / w.sum())
    Es, occ = chain_energies(oracle, dims, K, S, V, beta, 6000, seed=T.__hash__() % 1000)
    m, err = batch_mean_err(Es[500:])
    assert abs(m - exact) < 4 * err + 1e-12, (m, exact, err)
    assert np.bincount(occ, minlength=2).tolist() == [8, 8]


def test_energy_histogram_matches_boltzmann(oracle):
    dims, K, S, V = sixteen_site_cell()
    _, E = exact_levels(dims, K, S, V)
    beta = 1.0 / (KB * 1500.0)
    levels, g = np.unique(np.round(E, 9), return_counts=True)
    pw = g * np.exp(-beta * (levels - levels.min()))
    pw /= pw.sum()
    Es, _ = chain_energies(oracle, dims, K, S, V, beta, 24000, seed=77, thin=4)
    Es = np.round(Es[100:], 9)
    idx = np.searchsorted(levels, Es)
    assert np.allclose(levels[idx], Es)
    obs = np.bincount(idx, minlength=len(levels))
    exp = pw * len(Es)
    keep = exp >= 5
    obs_k = np.append(obs[keep], obs[~keep].sum())
    exp_k = np.append(exp[keep], exp[~keep].sum())
    if exp_k[-1] == 0:
        obs_k, exp_k = obs_k[:-1], exp_k[:-1]
    assert stats.chisquare(obs_k, exp_k).pvalue > 1e-4


def test_single_site_kernel_detailed_balance(oracle):
    """x ~ pi exactly, one trial at site 0, tally (x, y).  Detailed balance
    pi(x) P(x->y) = pi(y) P(y->x) makes the flow between any two energy levels
    symmetric: N(e1->e2) ~ N(e2->e1), binomial(1/2) per level pair."""
    dims, K, S, V = sixteen_site_cell()
    occs, E = exact_levels(dims, K, S, V)
    beta = 1.0 / (KB * 1500.0)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    levels = np.unique(np.round(E, 9))
    lev = np.searchsorted(levels, np.round(E, 9))
    code = {int(np.packbits(o).view(">u2")[0]): i for i, o in enumerate(occs)}
    g = np.random.default_rng(123)
    n = 120000
    xs = np.minimum(np.searchsorted(np.cumsum(pi), g.random(n)), len(pi) - 1)
    flow = np.zeros((len(levels), len(levels)), np.int64)
    moved = 0
    for j, x in enumerate(xs):
        occ = occs[x].copy()
        oracle.single_trial(BCC, dims, K, S, occ, V, seed=1000 + j, replica=0, sweep=0, a=0,
                            beta=beta)
        y = code[int(np.packbits(occ).view(">u2")[0])]
        if y != x:
            moved += 1
            flow[lev[x], lev[y]] += 1
    chi2, dof = 0.0, 0
    for i in range(len(levels)):
        for j in range(i + 1, len(levels)):
            t = flow[i, j] + flow[j, i]
            if t >= 10:
                chi2 += (flow[i, j] - flow[j, i]) ** 2 / t
                dof += 1
    assert moved > n // 10 and dof >= 15, (moved, dof)
    assert stats.chi2.sf(chi2, dof) > 1e-4, (chi2, dof)


def test_sro_vanishes_at_infinite_temperature(oracle):
    """beta = 0: every unlike swap is accepted and the chain samples uniform
    arrangements; E[alpha_s^kl] = 1 - N (N_l - delta_kl) / (N_l (N - 1))."""
    dims, K, S = (4, 4, 4), 4, 2
    N = 128
    Z, _ = oracle.shells(BCC, S)
    occ = np.repeat(np.arange(K, dtype=np.uint8), N // K)
    V = sym_V(S, K, 0.05, 1)
    cells = oracle.default_cells(dims, 3)
    alphas = []
    for t in range(3000):
        res = oracle.run(BCC, dims, K, S, cells, occ, V, seed=9, betas=[0.0], first_sweep=t)
        if t >= 20:
            alphas.append(oracle.sro(oracle.pair_counts(BCC, dims, K, S, occ), Z))
    # every distinct-species proposal accepted at beta = 0
    alphas = np.array(alphas)
    Nk = N // K
    for s in range(S):
        for k in range(K):
            for l in range(K):
                exp = 1.0 - N * (Nk - (k == l)) / (Nk * (N - 1))
                m, err = batch_mean_err(alphas[:, s, k, l])
                assert abs(m - exp) < 4 * err + 1e-12, (s, k, l, m, exp, err)
    assert np.bincount(occ, minlength=K).tolist() == [N // K] * K


def test_beta_zero_accepts_every_unlike_swap(oracle):
    dims, K, S = (4, 4, 4), 4, 2
    occ = np.random.default_rng(0).permutation(np.repeat(np.arange(K, dtype=np.uint8), 32))
    V = sym_V(S, K, 0.05, 1)
    res = oracle.run(BCC, dims, K, S, oracle.default_cells(dims, 3), occ, V, seed=3,
                     betas=[0.0] * 3, trace=True)
    tr = res.trace
    assert (tr["accepted"][tr["dE"] != 0.0] == 1).all()


def test_composition_conserved_and_stats(oracle):
    lattice, dims, K, S = FCC, (5, 6, 4), 5, 4
    N = 480
    occ = np.random.default_rng(2).integers(0, K, N).astype(np.uint8)
    before = np.bincount(occ, minlength=K)
    V = sym_V(S, K, 0.03, 3)
    res = oracle.run(lattice, dims, K, S, oracle.default_cells(dims, 3), occ, V, seed=1,
                     betas=[14.5] * 5)
    assert np.array_equal(np.bincount(occ, minlength=K), before)
    assert res.stats[0] == 5 * N and 0 < res.stats[1] < res.stats[0]


def test_low_temperature_anneal_reaches_b2(oracle):
    """Smoke check: annealing an unlike-attracting binary on BCC 4^3 lowers the
    energy to (near) the B2 ground state N Z1 v / 2."""
    dims, K, S = (4, 4, 4), 2, 1
    N = 128
    V = np.zeros((S, K, K))
    v = -0.05
    V[0, 0, 1] = V[0, 1, 0] = v
    occ = np.random.default_rng(1).permutation(np.repeat(np.arange(2, dtype=np.uint8), 64))
    Ts = np.linspace(3000, 50, 400)
    oracle.run(BCC, dims, K, S, oracle.default_cells(dims, 3), occ, V, seed=2,
               betas=1.0 / (KB * Ts))
    E = oracle.energy(oracle.pair_counts(BCC, dims, K, S, occ), V)
    assert E <= 0.9 * (0.5 * N * 8 * v)


def test_replay_overrides_near_tie(oracle):
    """A replayed decision replaces the oracle's own at a near-tie; entries
    for trials that are not near-ties are ignored."""
    dims, K, S = (4, 4, 4), 3, 2
    occ0 = np.random.default_rng(0).integers(0, K, 128).astype(np.uint8)
    V = sym_V(S, K, 0.05, 4)
    cells = oracle.default_cells(dims, 3)
    base = occ0.copy()
    r0 = oracle.run(BCC, dims, K, S, cells, base, V, seed=8, betas=[5.0], trace=True)
    up = r0.trace[(r0.trace["dE"] > 0)]
    rep = np.zeros(1, oracle.TIE_DTYPE)
    rep[0]["site"] = int(up[0]["a"])
    rep[0]["decision"] = 1 - int(up[0]["accepted"])
    other = occ0.copy()
    oracle.run(BCC, dims, K, S, cells, other, V, seed=8, betas=[5.0], replay=rep)
    assert np.array_equal(base, other)  # not a near-tie: replay entry ignored
