"""Parallel tempering on the GPU (smcx_energy_dev, smcx_exchange) against the
oracle's tempering driver: after every run the occupancies, the slot ->
replica map, the per-pair attempt / trade counts, the sweep counters and the
energies of the last exchange are identical.  Sweep and exchange near-ties
from the GPU's log are replayed by the oracle."""
import numpy as np
import pytest

from gpu_cases import NTHREADS, rand_occ, say, sym_V
from oracle import oracle as O

pytestmark = pytest.mark.gpu
BCC, FCC = 0, 1
KB = 8.617333262e-5


@pytest.fixture(scope="module")
def smcx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_12591_amd import smcx as S
    S.lib()
    return S


def tempering_inputs(lattice, dims, K, S, R, T0, T1, seed):
    V = sym_V(S, K, 0.02, seed)
    m = 2 if lattice == BCC else 4
    N = m * int(np.prod(dims))
    occs = [rand_occ(N, K, 100 * seed + r) for r in range(R)]
    beta = 1.0 / (KB * np.geomspace(T0, T1, R))
    return V, occs, beta


@pytest.mark.parametrize("lattice,dims,K,S,R,T0,T1,mode,rounds,n", [
    (BCC, (8, 8, 8), 4, 4, 6, 1600.0, 2400.0, "stream", 6, 2),
    (BCC, (8, 8, 8), 4, 4, 6, 1600.0, 2400.0, "persistent", 6, 2),
    (BCC, (8, 8, 8), 4, 4, 6, 1600.0, 2400.0, "plain", 3, 1),
    (FCC, (6, 6, 6), 5, 4, 4, 1800.0, 2600.0, "stream", 6, 2),
    (BCC, (12, 12, 12), 4, 2, 9, 900.0, 1400.0, "stream", 5, 3),
])
def test_tempering_matches_oracle(smcx, lattice, dims, K, S, R, T0, T1, mode, rounds, n):
    say(f"tempering lattice={lattice} dims={dims} K={K} S={S} R={R} mode={mode} rounds={rounds} n={n}")
    V, occs, beta = tempering_inputs(lattice, dims, K, S, R, T0, T1, seed=21)
    lat = smcx.Lattice(lattice, [dims] * R, K, S, np.concatenate(occs))
    lat.set_epi(V)
    pt = smcx.Tempering(lat, beta, seed=7, sweeps_per_round=n, mode=mode)
    pt.run(rounds)
    gpu = lat.occupancy()
    tnp, nt = pt.ties_numpy()
    rep_at = pt.rep_at.cpu().numpy()
    xst = pt.xstats.cpu().numpy().reshape(-1, 2)
    st = pt.stats.cpu().numpy().reshape(R, 3)
    E = pt.E.cpu().numpy()
    cells, _ = lat.schedule(0)
    lat.close()
    ref = [o.copy() for o in occs]
    out = O.tempering(lattice, dims, K, S, cells, ref, V, 7, beta, n_rounds=rounds,
                      sweeps_per_round=n, replay=tnp, nthreads=NTHREADS)
    N = len(ref[0])
    for r in range(R):
        assert np.array_equal(gpu[r * N:(r + 1) * N], ref[r]), f"replica {r}"
    assert rep_at.tolist() == out["rep_at"].tolist()
    assert np.array_equal(xst, out["xstats"])
    assert np.array_equal(st[:, :2], out["stats"][:, :2])
    assert np.array_equal(E, out["energies"][-1])
    assert nt == len(out["ties"])
    # the case exercises both outcomes of the exchange
    assert 0 < xst[:, 1].sum() < xst[:, 0].sum(), xst


def test_energy_dev_equals_host_energy(smcx):
    V, occs, _ = tempering_inputs(BCC, (8, 8, 8), 4, 4, 3, 1000.0, 2000.0, seed=3)
    lat = smcx.Lattice(BCC, [(8, 8, 8)] * 3, 4, 4, np.concatenate(occs))
    lat.set_epi(V)
    lat.sweep(2, 1, np.full((2, 3), 10.0))
    E_dev = lat.energy_dev().cpu().numpy()
    E_host = lat.energy()
    lat.close()
    assert np.array_equal(E_dev, E_host)


def test_exchange_needs_one_size(smcx):
    import torch
    V, _, _ = tempering_inputs(BCC, (8, 8, 8), 4, 2, 2, 1000.0, 2000.0, seed=4)
    dims = [(8, 8, 8), (8, 8, 12)]
    occ = np.concatenate([rand_occ(2 * 512, 4, 1), rand_occ(2 * 768, 4, 2)])
    lat = smcx.Lattice(BCC, dims, 4, 2, occ)
    lat.set_epi(V)
    pt = smcx.Tempering(lat, [10.0, 9.0], seed=1, sweeps_per_round=1)
    with pytest.raises(smcx.SmcxError):
        pt.run(1)
    torch.cuda.synchronize()
    lat.close()
