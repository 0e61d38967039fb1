"""Forced near-ties on the GPU, through the C ABI, against the oracle.

Each case puts one trial (or one exchange) exactly on its threshold
(tests/ties.py: beta = -log(u) / dE from the oracle's Philox block and energy
change), runs the HIP path, and checks the near-tie protocol end to end:

- the GPU logs exactly that {replica, sweep, site} once, and counts it in
  the replica's statistics;
- the oracle, replaying the GPU's decision, reproduces the GPU's occupancy,
  counters and log;
- the oracle replaying the opposite decision does not: the tie decided the
  trajectory, so the replay branch was really taken.

Covered: row windows (runtime geometry, BCC and FCC), tile windows,
persistent and plain modes, a replayed stream graph, several replicas of
different sizes, the qSRO model and one replica-exchange round.
"""
import ctypes as C

import numpy as np
import pytest

from gpu_cases import say
from oracle import oracle as O
from paper_2503_12591_amd import inputs as I
from ties import forced_exchange_tie, forced_trial_tie

pytestmark = pytest.mark.gpu
BCC, FCC = 0, 1
SEED = 11


@pytest.fixture(scope="module")
def smcx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_12591_amd import smcx as S
    S.lib()
    return S


def flipped(log):
    f = log.copy()
    f["decision"] = 1 - f["decision"]
    return f


def check_tie_run(lattice, dims, K, S, cells, occ0, V, gpu_occ, stats, log, nt, t, replica, sweep, betas,
                  W=None):
    """The GPU's run of sweep `sweep` against the oracle's, with and without
    its decision at the forced tie."""
    assert nt == 1 and len(log) == 1, f"GPU logged {nt} near-ties"
    e = log[0]
    assert (int(e["replica"]), int(e["sweep"]), int(e["site"])) == (replica, sweep, t["site"])
    assert stats[2] == 1
    say(f"tie site={t['site']} u={t['u']!r} beta={t['beta']!r} gpu decision={int(e['decision'])} "
        f"oracle exp decision={int(t['u'] < t['P'])}")

    def oracle(replay):
        ref = occ0.copy()
        if W is None:
            res = O.run(lattice, dims, K, S, cells, ref, V, SEED, betas, first_sweep=sweep, replica=replica,
                        replay=replay, nthreads=4)
        else:
            res = O.run_qsro(lattice, dims, K, S, cells, ref, V, W, SEED, betas, first_sweep=sweep,
                             replica=replica, replay=replay, nthreads=4)
        return ref, res

    ref, res = oracle(log)
    assert np.array_equal(gpu_occ, ref), f"{int((gpu_occ != ref).sum())} sites differ"
    assert stats[0] == res.stats[0] and stats[1] == res.stats[1] and res.stats[2] == 1
    assert res.n_ties == 1 and res.ties[0].tolist() == e.tolist()
    other, _ = oracle(flipped(log))
    assert not np.array_equal(gpu_occ, other), "the tied decision did not matter"


@pytest.mark.parametrize("lattice,dims,K,S,ell,mode,rows", [
    (BCC, (8, 8, 8), 4, 2, 4, "stream", True),      # row windows, runtime geometry
    (BCC, (8, 8, 8), 4, 2, 4, "stream", False),     # tile windows
    (BCC, (8, 8, 8), 4, 2, 4, "persistent", True),
    (BCC, (8, 8, 8), 4, 2, 4, "plain", True),
    (BCC, (12, 12, 12), 4, 4, 4, "stream", True),   # row windows, 4 species and 4 shells at compile time
    (FCC, (8, 8, 8), 5, 4, 4, "stream", True),      # FCC row windows, 6-bit counters
    (FCC, (6, 5, 7), 8, 3, 3, "stream", False),     # 64-bit counters
])
def test_forced_tie_sweep(smcx, lattice, dims, K, S, ell, mode, rows):
    say(f"forced tie lattice={lattice} dims={dims} K={K} S={S} ell={ell} mode={mode} rows={rows}")
    m = 2 if lattice == BCC else 4
    occ0 = I.occupancy(I.equiatomic(K, m * int(np.prod(dims))), 7)
    V = I.epi(K, S, 0.03, 5)
    lat = smcx.Lattice(lattice, dims, K, S, occ0, ell=ell, rows=rows)
    lat.set_epi(V)
    cells, _ = lat.schedule(0)
    sweep = 3
    t = forced_trial_tie(lattice, dims, K, S, cells, occ0, V, seed=SEED, replica=0, sweep=sweep)
    betas = [t["beta"]]
    stats, ties, tc = lat.sweep(1, SEED, betas, first_sweep=sweep, mode=mode)
    gpu = lat.occupancy()
    log, nt = lat.ties_to_numpy(ties, tc)
    st = stats.cpu().numpy()
    lat.close()
    check_tie_run(lattice, dims, K, S, cells, occ0, V, gpu, st, log, nt, t, 0, sweep, betas)


def test_forced_tie_stream_graph(smcx):
    """A captured stream sweep replayed twice: the tie sits in the second
    replay's sweep (the sweep index comes from the graph's device counter)."""
    dims, K, S = (8, 8, 8), 4, 2
    occ0 = I.occupancy(I.equiatomic(K, 2 * 512), 8)
    V = I.epi(K, S, 0.03, 6)
    lat = smcx.Lattice(BCC, dims, K, S, occ0, ell=4)
    lat.set_epi(V)
    cells, _ = lat.schedule(0)
    # the first replay (sweep 4) runs at beta_hot from occ0; the tie is built on
    # the configuration the oracle reaches after it
    beta_hot = float(I.beta_of_T(1500.0))
    mid = occ0.copy()
    O.run(BCC, dims, K, S, cells, mid, V, SEED, [beta_hot], first_sweep=4, nthreads=4)
    t = forced_trial_tie(BCC, dims, K, S, cells, mid, V, seed=SEED, replica=0, sweep=5)
    say(f"stream graph tie beta={t['beta']!r}")
    import torch
    g = smcx.LadderGraph(lat, 1, SEED, [beta_hot], first_sweep=4, mode="stream")
    g.launch()
    log0, n0 = lat.ties_to_numpy(g.ties, g.tie_count)
    assert n0 == 0
    g.beta.fill_(t["beta"])
    g.launch()
    torch.cuda.synchronize()
    gpu = lat.occupancy()
    log, nt = lat.ties_to_numpy(g.ties, g.tie_count)
    st = g.stats.cpu().numpy()
    g.close()
    lat.close()
    st_second = st.copy()
    st_second[0] -= 2 * 512  # the first replay's attempts
    first = O.run(BCC, dims, K, S, cells, occ0.copy(), V, SEED, [beta_hot], first_sweep=4)
    st_second[1] -= first.stats[1]
    check_tie_run(BCC, dims, K, S, cells, mid, V, gpu, st_second, log, nt, t, 0, 5, [t["beta"]])


def test_forced_tie_in_one_of_several_replicas(smcx):
    """Three replicas of different sizes in one stream launch; only replica 1
    runs at the tie's beta, in sweep 2."""
    dims = np.array([[8, 8, 8], [12, 8, 8], [8, 12, 12]], np.int32)
    K, S = 4, 4
    occs = [I.occupancy(I.equiatomic(K, 2 * int(np.prod(d))), 40 + r) for r, d in enumerate(dims)]
    V = I.epi(K, S, 0.03, 7)
    lat = smcx.Lattice(BCC, dims, K, S, np.concatenate(occs), ell=4)
    lat.set_epi(V)
    cells1, _ = lat.schedule(1)
    t = forced_trial_tie(BCC, dims[1], K, S, cells1, occs[1], V, seed=SEED, replica=1, sweep=2)
    betas = np.array([[20.0, t["beta"], 15.0]])
    stats, ties, tc = lat.sweep(1, SEED, betas, first_sweep=2, mode="stream")
    gpu = lat.occupancy()
    log, nt = lat.ties_to_numpy(ties, tc)
    st = stats.cpu().numpy().reshape(3, 3)
    scheds = [lat.schedule(r)[0] for r in range(3)]
    lat.close()
    off = np.concatenate([[0], np.cumsum([len(o) for o in occs])])
    for r in (0, 2):
        ref = occs[r].copy()
        res = O.run(BCC, dims[r], K, S, scheds[r], ref, V, SEED, betas[:, r], first_sweep=2, replica=r)
        assert np.array_equal(gpu[off[r]:off[r + 1]], ref) and res.n_ties == 0
        assert st[r].tolist() == res.stats.tolist()
    check_tie_run(BCC, dims[1], K, S, cells1, occs[1], V, gpu[off[1]:off[2]], st[1], log, nt, t, 1, 2,
                  betas[:, 1])


def test_forced_tie_qsro(smcx):
    dims, K, S = (8, 8, 8), 4, 2
    occ0 = I.occupancy(I.equiatomic(K, 2 * 512), 4)
    V = I.epi(K, S, 0.05, 21)
    W = np.random.default_rng(22).normal(0, 0.2, (S, K))
    lat = smcx.Lattice(BCC, dims, K, S, occ0, ell=4)
    lat.set_qsro(V, W)
    cells, _ = lat.schedule(0)
    t = forced_trial_tie(BCC, dims, K, S, cells, occ0, V, seed=SEED, replica=0, sweep=2, W=W)
    say(f"qsro tie beta={t['beta']!r}")
    stats, ties, tc = lat.sweep_qsro(1, SEED, [t["beta"]], first_sweep=2)
    gpu = lat.occupancy()
    log, nt = lat.ties_to_numpy(ties, tc)
    st = stats.cpu().numpy()
    lat.close()
    check_tie_run(BCC, dims, K, S, cells, occ0, V, gpu, st, log, nt, t, 0, 2, [t["beta"]], W=W)


def test_forced_exchange_tie(smcx):
    """One exchange round with slot pair 2 on its threshold (replicas held
    out of order): the GPU logs {-1, round, 2, decision}; the oracle's
    exchange replaying it gives the same slot map and trade counts, and the
    opposite decision does not."""
    import torch
    R, dims, K, S = 6, (8, 8, 8), 4, 4
    occs = [I.occupancy(I.equiatomic(K, 1024), 60 + r) for r in range(R)]
    V = I.epi(K, S, 0.03, 8)
    E = np.array([O.energy(O.pair_counts(BCC, dims, K, S, o), V) for o in occs])
    beta = 1.0 / (I.K_B_EV * np.geomspace(600.0, 1500.0, R))
    rep_at = np.array([3, 0, 5, 1, 4, 2], np.int32)
    bs, u, x = forced_exchange_tie(E, beta, rep_at, seed=SEED, round_=0, pair=2)
    say(f"exchange tie u={u!r} x={x!r}")
    lat = smcx.Lattice(BCC, [dims] * R, K, S, np.concatenate(occs))
    lat.set_epi(V)
    L = smcx.lib()
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    bs_d, rep_d = dev(bs, np.float64), dev(rep_at, np.int32)
    beta_rows = torch.zeros((1, R), dtype=torch.float64, device="cuda")
    Ed = torch.zeros(R, dtype=torch.float64, device="cuda")
    xst = torch.zeros(2 * (R - 1), dtype=torch.int64, device="cuda")
    ties = torch.zeros(16 * O.TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    tc = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = lambda t_: C.c_void_p(t_.data_ptr())
    rc = L.smcx_exchange(lat.h, 0, C.c_uint64(SEED), p(bs_d), p(rep_d), p(beta_rows), 1, p(lat.counts), p(Ed),
                         p(xst), p(ties), 16, p(tc), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, smcx.lib().smcx_last_error()
    log, nt = lat.ties_to_numpy(ties, tc)
    gpu_rep = rep_d.cpu().numpy()
    gpu_xst = xst.cpu().numpy().reshape(R - 1, 2)
    gpu_rows = beta_rows.cpu().numpy()[0]
    assert np.array_equal(Ed.cpu().numpy(), E)
    lat.close()
    assert nt == 1 and (int(log[0]["replica"]), int(log[0]["sweep"]), int(log[0]["site"])) == (-1, 0, 2)
    say(f"exchange gpu decision={int(log[0]['decision'])} oracle exp decision={int(u < np.exp(x))}")
    ref = rep_at.copy()
    st = np.zeros((R - 1, 2), np.int64)
    oties, ont = O.exchange(E, bs, ref, seed=SEED, round_=0, replay=log, stats=st)
    assert np.array_equal(gpu_rep, ref) and np.array_equal(gpu_xst, st)
    assert ont == 1 and oties[0].tolist() == log[0].tolist()
    # every replica's new beta is that of the slot now holding it
    assert np.array_equal(gpu_rows[ref], bs)
    other = rep_at.copy()
    O.exchange(E, bs, other, seed=SEED, round_=0, replay=flipped(log))
    assert not np.array_equal(gpu_rep, other)
