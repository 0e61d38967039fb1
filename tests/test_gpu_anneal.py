"""Stepwise anneal with energy recording and heat capacity (smcx_anneal)
against the oracle's anneal driver: occupancies, every recorded energy, the
heat capacity of every step and the sweep counters are identical."""
import numpy as np
import pytest

from gpu_cases import NTHREADS, rand_occ, say, sym_V
from oracle import oracle as O
from paper_2503_12591_amd import inputs as I

pytestmark = pytest.mark.gpu
BCC, FCC = 0, 1


@pytest.fixture(scope="module")
def smcx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_12591_amd import smcx as S
    S.lib()
    return S


@pytest.mark.parametrize("lattice,dims,K,S,mode,warmup,record", [
    (BCC, [(8, 8, 8), (8, 12, 8)], 4, 4, "stream", 2, 4),
    (BCC, [(8, 8, 8), (8, 12, 8)], 4, 4, "persistent", 1, 3),
    (FCC, [(6, 6, 6)], 5, 4, "stream", 2, 3),
    (BCC, [(12, 12, 12)], 4, 2, "plain", 0, 2),
])
def test_anneal_matches_oracle(smcx, lattice, dims, K, S, mode, warmup, record):
    say(f"anneal lattice={lattice} dims={dims} K={K} S={S} mode={mode} warmup={warmup} record={record}")
    V = sym_V(S, K, 0.02, 31)
    m = 2 if lattice == BCC else 4
    occs = [rand_occ(m * int(np.prod(d)), K, 40 + r) for r, d in enumerate(dims)]
    T = I.stepwise_temperatures(2000.0, 1800.0, 50.0)
    beta = I.beta_of_T(T)
    lat = smcx.Lattice(lattice, dims, K, S, np.concatenate(occs))
    lat.set_epi(V)
    out = lat.anneal(beta, warmup, record, seed=13, first_sweep=5, mode=mode)
    gpu = lat.occupancy()
    E = out["E"].cpu().numpy()
    cv = out["cv"].cpu().numpy()
    st = out["stats"].cpu().numpy().reshape(-1, 3)
    tnp, nt = lat.ties_to_numpy(out["ties"], out["tie_count"])
    scheds = [lat.schedule(r)[0] for r in range(len(dims))]
    lat.close()
    off = 0
    for r, d in enumerate(dims):
        ref = occs[r].copy()
        res = O.anneal(lattice, d, K, S, scheds[r], ref, V, 13, beta, warmup, record, first_sweep=5,
                       replica=r, replay=tnp[tnp["replica"] == r], nthreads=NTHREADS)
        assert np.array_equal(gpu[off:off + len(ref)], ref), f"replica {r}"
        assert np.array_equal(E[:, :, r], res["E"]), f"energies of replica {r}"
        assert np.array_equal(cv[:, r], res["cv"]), f"heat capacity of replica {r}"
        assert st[r, 0] == res["stats"][0] and st[r, 1] == res["stats"][1]
        off += len(ref)
    assert (cv > 0).all()
