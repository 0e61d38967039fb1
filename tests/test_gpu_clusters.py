"""Local energies and low-energy clusters on the GPU (smcx_local_energy,
smcx_clusters) against the oracle: local energies bit-identical, cluster
labels (smallest site index), sizes and counts identical, with thresholds on
exact local-energy values (ties count) and at the limits."""
import math

import numpy as np
import pytest

from gpu_cases import rand_occ, say, sym_V
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


@pytest.mark.parametrize("lattice,dims,K,S,sweeps", [
    (BCC, (6, 5, 7), 4, 4, 0),
    (FCC, (4, 5, 3), 5, 3, 0),
    (BCC, (2, 3, 2), 3, 2, 0),
    (BCC, (16, 16, 16), 4, 4, 3),
    (FCC, (12, 10, 14), 5, 4, 2),
    (BCC, (64, 64, 64), 4, 4, 2),
])
def test_local_energy_and_clusters_match_oracle(smcx, lattice, dims, K, S, sweeps):
    say(f"clusters lattice={lattice} dims={dims} K={K} S={S} sweeps={sweeps}")
    V = sym_V(S, K, 0.05, 7)
    m = 2 if lattice == BCC else 4
    N = m * int(np.prod(dims))
    occ = rand_occ(N, K, 5)
    lat = smcx.Lattice(lattice, dims, K, S, occ)
    lat.set_epi(V)
    if sweeps:
        lat.sweep(sweeps, 3, np.full(sweeps, 12.0))
    cur = lat.occupancy()
    e_gpu = lat.local_energy()
    e = O.local_energy(lattice, dims, K, S, cur, V)
    assert np.array_equal(e_gpu.cpu().numpy(), e)
    srt = np.sort(e)
    for q in (0.1, 0.3, 0.6):
        thr = float(srt[int(q * (N - 1))])
        label, size, nc = lat.clusters(thr, e=e_gpu)
        rl, rs, rn = O.clusters(lattice, dims, e, thr)
        assert np.array_equal(label.cpu().numpy(), rl), f"labels at q={q}"
        assert np.array_equal(size.cpu().numpy(), rs), f"sizes at q={q}"
        assert int(nc.item()) == rn
    for thr, n_expect in ((math.inf, 1), (-math.inf, 0)):
        label, size, nc = lat.clusters(thr, e=e_gpu)
        assert int(nc.item()) == n_expect
        lab = label.cpu().numpy()
        assert (lab == (0 if n_expect else -1)).all()
    lat.close()


def test_clusters_per_replica(smcx):
    """Replica r's local energies and clusters come from its own sites."""
    V = sym_V(4, 4, 0.05, 9)
    dims = [(8, 8, 8), (6, 10, 8)]
    occs = [rand_occ(2 * 512, 4, 1), rand_occ(2 * 480, 4, 2)]
    lat = smcx.Lattice(BCC, dims, 4, 4, np.concatenate(occs))
    lat.set_epi(V)
    for r in range(2):
        e = O.local_energy(BCC, dims[r], 4, 4, occs[r], V)
        eg = lat.local_energy(r)
        assert np.array_equal(eg.cpu().numpy(), e)
        thr = float(np.sort(e)[len(e) // 4])
        label, size, nc = lat.clusters(thr, r=r, e=eg)
        rl, rs, rn = O.clusters(BCC, dims[r], e, thr)
        assert np.array_equal(label.cpu().numpy(), rl) and np.array_equal(size.cpu().numpy(), rs)
        assert int(nc.item()) == rn
    lat.close()
