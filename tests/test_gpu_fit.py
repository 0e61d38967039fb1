"""EPI fit through the HIP backward (energy_backward behind EnergyFn).

4096 random equiatomic BCC 16^3 configurations, per-site energies from a
seeded teacher V* (labels from the oracle's pair counts).  Adam through
EnergyFn must reproduce the gauge-invariant W_s[k][l] = V_kl - (V_kk + V_ll)/2
(k < l) of the closed-form least-squares fit and of the teacher within 1e-6 eV.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_cases import NTHREADS, say
from oracle import oracle as O
from paper_2503_12591_amd import inputs as I

pytestmark = pytest.mark.gpu


def gauge_w(V):
    K = V.shape[-1]
    ku, lu = np.triu_indices(K, 1)
    d = np.diagonal(V, axis1=-2, axis2=-1)
    return V[..., ku, lu] - 0.5 * (d[..., ku] + d[..., lu])


def test_epi_fit_matches_lstsq_and_teacher():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_12591_amd import smcx
    dims, occs, Vt = I.c4b_fit_set()
    B, N = occs.shape
    say(f"fit: oracle counts of {B} configurations")
    with ThreadPoolExecutor(max(1, NTHREADS)) as ex:
        C = np.stack(list(ex.map(lambda o: O.pair_counts(I.BCC, dims, 4, 4, o), occs)))
    y = np.array([O.energy(C[b], Vt) for b in range(B)]) / N
    # closed-form reference: least squares on the k < l count features (+ a constant)
    ku, lu = np.triu_indices(4, 1)
    F = np.concatenate([C[:, :, ku, lu].reshape(B, -1) / N, np.ones((B, 1))], axis=1)
    w_ls = np.linalg.lstsq(F, y, rcond=None)[0][:-1].reshape(4, -1)
    say("fit: Adam through EnergyFn")
    V, loss = smcx.fit_epi(I.BCC, dims, 4, 4, torch.from_numpy(occs).cuda(), y)
    w_fit = gauge_w(V.cpu().numpy())
    w_teacher = gauge_w(Vt)
    assert np.abs(w_ls - w_teacher).max() < 1e-9
    assert np.abs(w_fit - w_ls).max() < 1e-6, np.abs(w_fit - w_ls).max()
    assert np.abs(w_fit - w_teacher).max() < 1e-6
    assert loss < 1e-12
