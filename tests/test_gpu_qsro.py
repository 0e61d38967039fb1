"""qSRO model on the GPU (smcx_set_qsro, smcx_sweep_qsro) against the
oracle's qSRO sweeps: identical occupancy, attempted and accepted counts,
with the GPU's near-ties replayed."""
import numpy as np
import pytest

from gpu_cases import NTHREADS, rand_occ, say, sym_V
from oracle import oracle as O

pytestmark = pytest.mark.gpu
BCC, FCC = 0, 1


@pytest.fixture(scope="module")
def smcx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_12591_amd import smcx as S
    S.lib()
    return S


@pytest.mark.parametrize("lattice,dims,K,S,ell,R,n", [
    (BCC, (10, 10, 10), 4, 2, 4, 1, 3),
    (BCC, (12, 12, 10), 4, 4, 5, 1, 2),
    (FCC, (8, 8, 9), 5, 2, 4, 1, 2),
    (BCC, (8, 8, 8), 3, 2, 4, 2, 2),
    (BCC, (6, 6, 6), 2, 2, 6, 1, 3),
])
def test_qsro_sweeps_match_oracle(smcx, lattice, dims, K, S, ell, R, n):
    say(f"qsro lattice={lattice} dims={dims} K={K} S={S} ell={ell} R={R} n={n}")
    V = sym_V(S, K, 0.05, 21)
    W = np.random.default_rng(22).normal(0, 0.2, (S, K))
    m = 2 if lattice == BCC else 4
    N = m * int(np.prod(dims))
    occs = [rand_occ(N, K, 30 + r) for r in range(R)]
    betas = np.tile(np.array([20.0, 12.0, 30.0][:n])[:, None], (1, R))
    lat = smcx.Lattice(lattice, [dims] * R, K, S, np.concatenate(occs), ell=ell)
    lat.set_qsro(V, W)
    stats, ties, tc = lat.sweep_qsro(n, 5, betas, first_sweep=2)
    gpu = lat.occupancy()
    tnp, nt = lat.ties_to_numpy(ties, tc)
    st = stats.cpu().numpy().reshape(R, 3)
    scheds = [lat.schedule(r)[0] for r in range(R)]
    lat.close()
    for r in range(R):
        ref = occs[r].copy()
        res = O.run_qsro(lattice, dims, K, S, scheds[r], ref, V, W, 5, betas[:, r], first_sweep=2, replica=r,
                         replay=tnp[tnp["replica"] == r], nthreads=NTHREADS)
        assert np.array_equal(gpu[r * N:(r + 1) * N], ref), f"replica {r}: {int((gpu[r * N:(r + 1) * N] != ref).sum())} sites"
        assert st[r, 0] == res.stats[0] == n * N
        assert st[r, 1] == res.stats[1]
        assert 0 < st[r, 1] < st[r, 0]


def test_qsro_needs_the_interaction_zone_rule(smcx):
    V = sym_V(4, 4, 0.05, 1)
    W = np.zeros((4, 4))
    lat = smcx.Lattice(BCC, (12, 12, 12), 4, 4, rand_occ(2 * 12 ** 3, 4, 1), ell=4)
    lat.set_qsro(V, W)
    with pytest.raises(smcx.SmcxError):
        lat.sweep_qsro(1, 0, [10.0])  # link cells of 4 < 5 for 4 BCC shells
    lat.close()
