"""The allocation-free entry point smcx_lattice_init_static against
smcx_lattice_init with a caller workspace, through the C ABI (GPU).

Two calls in a row, the second with a smaller lattice: each handle made on
the library's static workspace must give the trajectory, counters, pair
counts and energies of a handle on a workspace the caller allocated, in
stream (row windows), tile-window and persistent modes.  Also: a
description too large for the static workspace is refused, and a handle
whose static workspace a later call took over is refused.
"""
import numpy as np
import pytest

from gpu_cases import rand_occ, say, sym_V
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


def run(smcx, lattice, dims, K, S, occ, V, betas, mode, static, rows=True):
    lat = smcx.Lattice(lattice, dims, K, S, occ.copy(), ell=4, rows=rows, static_workspace=static)
    lat.set_epi(V)
    stats, ties, tc = lat.sweep(len(betas), 7, betas, first_sweep=2, mode=mode)
    out = dict(occ=lat.occupancy(), stats=stats.cpu().numpy(), nt=int(tc.item()),
               counts=lat.pair_counts().cpu().numpy(), E=lat.energy())
    lat.close()
    return out


@pytest.mark.parametrize("lattice,dims,K,S", [
    (BCC, [(24, 20, 16), (16, 16, 16)], 4, 4),   # first call: two replicas
    (FCC, [(8, 8, 8)], 5, 4),                     # second call: a smaller lattice
])
def test_static_workspace_matches_caller_workspace(smcx, lattice, dims, K, S):
    m = 2 if lattice == BCC else 4
    occ = np.concatenate([rand_occ(m * int(np.prod(d)), K, 40 + r) for r, d in enumerate(dims)])
    V = sym_V(S, K, 0.04, 3)
    R = len(dims)
    betas = np.tile(I.beta_of_T(np.array([1500.0, 1100.0, 800.0]))[:, None], (1, R))
    for mode, rows in (("stream", True), ("stream", False), ("persistent", True)):
        say(f"static workspace lattice={lattice} dims={dims} mode={mode} rows={rows}")
        a = run(smcx, lattice, dims, K, S, occ, V, betas, mode, static=True, rows=rows)
        b = run(smcx, lattice, dims, K, S, occ, V, betas, mode, static=False, rows=rows)
        assert np.array_equal(a["occ"], b["occ"])
        assert np.array_equal(a["stats"], b["stats"]) and a["nt"] == b["nt"]
        assert np.array_equal(a["counts"], b["counts"])
        assert np.array_equal(a["E"], b["E"])
        assert not np.array_equal(a["occ"], occ)  # the sweeps did something


def test_static_workspace_limits(smcx):
    import torch
    occ = rand_occ(2 * 512, 4, 1)
    V = sym_V(2, 4, 0.04, 1)
    # too large for the static workspace: refused before any device work
    big = torch.zeros(2 * 320 ** 3, dtype=torch.uint8, device="cuda")
    with pytest.raises(smcx.SmcxError, match="static workspace"):
        smcx.Lattice(BCC, (320, 320, 320), 4, 4, big, ell=4, static_workspace=True)
    del big
    # a later handle on the same device takes the workspace over
    first = smcx.Lattice(BCC, (8, 8, 8), 4, 2, occ.copy(), static_workspace=True)
    first.set_epi(V)
    second = smcx.Lattice(BCC, (8, 8, 8), 4, 2, occ.copy(), static_workspace=True)
    second.set_epi(V)
    with pytest.raises(smcx.SmcxError, match="taken over"):
        first.sweep(1, 0, [10.0], mode="stream")
    second.sweep(1, 0, [10.0], mode="stream")
    torch.cuda.synchronize()
    first.close()
    second.close()
