"""Shared helpers of the GPU parity tests: run the HIP path and the CPU oracle
on the same seeded inputs and compare."""
import os
import sys

import numpy as np

from oracle import oracle as O
from paper_2503_12591_amd import inputs as I

NTHREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def sym_V(S, K, scale, seed):
    V = np.random.default_rng(seed).normal(0, scale, (S, K, K))
    return 0.5 * (V + V.transpose(0, 2, 1))


def rand_occ(N, K, seed, equi=True):
    if equi:
        return I.occupancy(I.equiatomic(K, N), seed)
    return np.random.default_rng(seed).integers(0, K, N).astype(np.uint8)


def gpu_vs_oracle(lattice, dims, K, S, occ0, V, betas, seed=0, mode="auto", ell=None, cells=None,
                  tile=(0, 0, 0), first_sweep=0, check_every_sweep=False, rows=True):
    """Run len(betas) sweeps on the GPU and in the oracle; assert equality of
    the occupancy, attempted/accepted counts and near-tie counts."""
    from paper_2503_12591_amd import smcx
    say(f"sweep lattice={lattice} dims={tuple(dims)} K={K} S={S} n={len(betas)} mode={mode} "
        f"ell={ell} tile={tile} seed={seed} rows={rows}")
    lat = smcx.Lattice(lattice, dims, K, S, occ0, ell=ell,
                       cells=None if cells is None else [cells], tile=tile, rows=rows)
    lat.set_epi(V)
    sched, nA = lat.schedule(0)
    if cells is not None:
        for a in range(3):
            assert list(sched[a]) == list(cells[a])
    ref = occ0.copy()
    if check_every_sweep:
        for j, b in enumerate(betas):
            stats, ties, tc = lat.sweep(1, seed, [b], first_sweep=first_sweep + j, mode=mode)
            tnp, nt = lat.ties_to_numpy(ties, tc)
            res = O.run(lattice, dims, K, S, sched, ref, V, seed, [b], first_sweep=first_sweep + j,
                        replay=tnp)
            gpu = lat.occupancy()
            assert np.array_equal(gpu, ref), f"trajectory differs after sweep {first_sweep + j}"
            s = stats.cpu().numpy()
            assert s[0] == res.stats[0] and s[1] == res.stats[1] and s[2] == res.stats[2] == nt
        lat.close()
        return ref
    stats, ties, tc = lat.sweep(len(betas), seed, betas, first_sweep=first_sweep, mode=mode)
    gpu = lat.occupancy()
    tnp, nt = lat.ties_to_numpy(ties, tc)
    res = O.run(lattice, dims, K, S, sched, ref, V, seed, betas, first_sweep=first_sweep, replay=tnp,
                nthreads=NTHREADS)
    s = stats.cpu().numpy()
    lat.close()
    assert np.array_equal(gpu, ref), f"{int((gpu != ref).sum())} sites differ"
    assert s[0] == res.stats[0], (s, res.stats)
    assert s[1] == res.stats[1], (s, res.stats)
    assert s[2] == res.stats[2] == nt
    return ref
