"""Pins of the oracle's qSRO model (CPU only).

E_i = sum_m sum_t V_m[p][t] (n_i[m][t] / Z_m) + sum_m W_m[p] (n_i[m][p] / Z_m)^2
(p = sigma_i, centre-neighbour pair fractions).  Pinned by
  - closed forms on ordered structures: a pure element (every fraction 0 or
    1) and the B2 arrangement on BCC;
  - the pair-model limit: with W = 0 the total equals the EPI energy with
    V' = 2 V / Z, and every swap's energy change matches the EPI one;
  - the swap energy change from the affected set equals the difference of
    the total energies before and after the swap (all sites recomputed), for
    every partner direction at many sites, on BCC and FCC, 1 to 4 shells.
"""
import numpy as np
import pytest

BCC, FCC = 0, 1


def sym_V(S, K, scale, seed):
    V = np.random.default_rng(seed).normal(0, scale, (S, K, K))
    return 0.5 * (V + V.transpose(0, 2, 1))


def test_closed_form_pure_element(oracle):
    S, K = 3, 3
    V = sym_V(S, K, 0.1, 1)
    W = np.random.default_rng(2).normal(0, 0.1, (S, K))
    occ = np.full(2 * 6 ** 3, 2, np.uint8)
    e = oracle.qsro_local_energy(BCC, (6, 6, 6), K, S, occ, V, W)
    expect = 0.0
    for s in range(S):
        expect = expect + V[s, 2, 2] * 1.0
    for s in range(S):
        expect = expect + W[s, 2] * 1.0
    assert np.all(e == expect)


def test_closed_form_b2(oracle):
    """B2 order (species 0 on the cube corners, 1 on the centres): every
    nearest neighbour unlike, every second neighbour alike."""
    S, K = 2, 2
    V = sym_V(S, K, 0.1, 3)
    W = np.random.default_rng(4).normal(0, 0.1, (S, K))
    occ = np.tile(np.array([0, 1], np.uint8), 6 ** 3)
    e = oracle.qsro_local_energy(BCC, (6, 6, 6), K, S, occ, V, W)
    for p, q in ((0, 1), (1, 0)):
        expect = ((V[0, p, q] * 1.0 + V[1, p, p] * 1.0) + W[0, p] * 0.0) + W[1, p] * 1.0
        assert np.all(e[p::2] == expect)


@pytest.mark.parametrize("lattice,dims,K,S", [(BCC, (6, 5, 7), 4, 4), (FCC, (5, 6, 5), 3, 3), (BCC, (5, 5, 5), 2, 1)])
def test_pair_limit(oracle, lattice, dims, K, S):
    V = sym_V(S, K, 0.05, 5)
    W = np.zeros((S, K))
    m = 2 if lattice == BCC else 4
    N = m * int(np.prod(dims))
    occ = np.random.default_rng(6).integers(0, K, N).astype(np.uint8)
    Z, _ = oracle.shells(lattice, S)
    Vp = 2.0 * V / np.asarray(Z, np.float64)[:, None, None]
    e = oracle.qsro_local_energy(lattice, dims, K, S, occ, V, W)
    E_pair = oracle.energy(oracle.pair_counts(lattice, dims, K, S, occ), Vp)
    assert abs(e.sum() - E_pair) <= 1e-12 * max(1.0, abs(E_pair))
    rng = np.random.default_rng(7)
    for _ in range(20):
        a, k = int(rng.integers(N)), int(rng.integers(Z[0]))
        dq, b = oracle.qsro_delta_e(lattice, dims, K, S, occ, V, W, a, k)
        dp, b2 = oracle.delta_e(lattice, dims, K, S, occ, Vp, a, k)
        assert b == b2
        assert abs(dq - dp) <= 1e-12 * max(1.0, abs(dp))


@pytest.mark.parametrize("lattice,dims,K,S", [
    (BCC, (6, 5, 7), 4, 4), (BCC, (5, 6, 5), 3, 2), (FCC, (5, 5, 6), 5, 4), (FCC, (4, 5, 4), 3, 1),
])
def test_delta_e_is_the_total_energy_difference(oracle, lattice, dims, K, S):
    V = sym_V(S, K, 0.05, 8)
    W = np.random.default_rng(9).normal(0, 0.2, (S, K))
    m = 2 if lattice == BCC else 4
    N = m * int(np.prod(dims))
    occ = np.random.default_rng(10).integers(0, K, N).astype(np.uint8)
    Z, _ = oracle.shells(lattice, S)
    E0 = oracle.qsro_local_energy(lattice, dims, K, S, occ, V, W).sum()
    rng = np.random.default_rng(11)
    n_diff = 0
    for a in rng.integers(0, N, 12):
        for k in range(Z[0]):
            dE, b = oracle.qsro_delta_e(lattice, dims, K, S, occ, V, W, int(a), k)
            o2 = occ.copy()
            o2[a], o2[b] = o2[b], o2[a]
            E1 = oracle.qsro_local_energy(lattice, dims, K, S, o2, V, W).sum()
            assert abs(dE - (E1 - E0)) <= 1e-11 * max(1.0, abs(E0)), (a, k)
            n_diff += occ[a] != occ[b]
    assert n_diff > 0


def test_small_edges_rejected(oracle):
    V = sym_V(4, 2, 0.05, 1)
    W = np.zeros((4, 2))
    occ = np.zeros(2 * 4 ** 3, np.uint8)
    with pytest.raises(ValueError):  # BCC 4 shells reach 3 half-units: edges must exceed 4
        oracle.qsro_delta_e(BCC, (4, 4, 4), 2, 4, occ, V, W, 0, 0)


def test_closed_form_one_impurity(oracle):
    """Pure species 0 with one site of species 1: each of the impurity's 8
    nearest neighbours has pair fractions 7/8 (like) and 1/8 (unlike) in
    shell 1, so E = V[0][0] 7/8 + V[0][1] 1/8 + W[0] (7/8)^2; dyadic
    parameters make it exact: 0.4375 + 0.03125 + 1.53125 = 2.  The impurity
    has E = V[1][0] = 0.25, every other site V[0][0] + W[0] = 2.5."""
    V = np.array([[[0.5, 0.25], [0.25, 0.0]]])
    W = np.array([[2.0, 0.0]])
    occ = np.zeros(2 * 216, np.uint8)
    j = 1 + 2 * (2 + 6 * (3 + 6 * 2))  # a body-centre site
    occ[j] = 1
    e = oracle.qsro_local_energy(BCC, (6, 6, 6), 2, 1, occ, V, W)
    assert int((e == 2.0).sum()) == 8
    assert e[j] == 0.25
    assert int((e == 2.5).sum()) == len(e) - 9
