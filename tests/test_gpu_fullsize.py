"""Full-size parity on the GPU (the sizes the benchmark and the workloads use).

- BCC 800^3 (1.024e9 sites), in the benchmark's launch configuration: single
  mini-steps run from the generated initial configuration and compared site
  by site with the oracle's run of the same mini-step; then full sweeps
  checked through exact invariants (composition, pair-count symmetry and row
  sums, attempted count).
- FCC 128^3, 5 species: two full sweeps identical to the (threaded) oracle,
  energies and SRO equal.
- BCC 64^3 anneal: the first sweeps identical to the oracle; batched backward
  counts of snapshots identical to the oracle's counts.
- 256-replica ladder with edges 16..48: every replica identical to the oracle.
- Backward on 4096 configurations of BCC 16^3: sampled configurations equal to
  the oracle, invariants on all.
"""
import numpy as np
import pytest

from gpu_cases import NTHREADS, say
from oracle import oracle as O
from paper_2503_12591_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smcx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_12591_amd import smcx as S
    S.lib()
    return S


def test_large_bcc_ministeps_and_invariants(smcx):
    import torch
    w = I.c5_large_bcc()
    say("bcc800: generate")
    occ0_dev = I.occupancy_device(w.counts, seed=0)
    occ0 = occ0_dev.cpu().numpy()
    work = occ0_dev.clone()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, work, ell=4)
    lat.set_epi(w.V)
    cells, nA = lat.schedule(0)
    assert nA == 128
    beta = float(w.betas[0])
    for tau in (0, 1, 77, 127):
        say(f"bcc800 mini-step {tau}")
        work.copy_(occ0_dev)
        stats, ties, tc = lat.sweep_partial(0, tau, tau + 1, 0, [beta], mode="stream")
        gpu = work.cpu().numpy()
        tnp, nt = lat.ties_to_numpy(ties, tc)
        ref = occ0.copy()
        res = O.run_ministeps(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, 0, beta, 0, tau, tau + 1,
                              replay=tnp, nthreads=NTHREADS)
        s = stats.cpu().numpy()
        assert s[0] == res.stats[0] == 8_000_000
        assert s[1] == res.stats[1]
        assert np.array_equal(gpu, ref), f"mini-step {tau}: {int((gpu != ref).sum())} sites differ"
        assert int((gpu != occ0).sum()) <= 2 * s[1]
    say("bcc800: two sweeps + invariants")
    work.copy_(occ0_dev)
    betas = np.full(2, beta)
    stats, ties, tc = lat.sweep(2, 0, betas, mode="stream")
    s = stats.cpu().numpy()
    assert s[0] == 2 * w.N
    after = torch.bincount(work.long(), minlength=w.K).cpu().numpy()
    assert after.tolist() == w.counts.tolist()
    C = lat.pair_counts().cpu().numpy()[0]
    Z, _ = O.shells(w.lattice, w.S)
    for sh in range(w.S):
        assert np.array_equal(C[sh], C[sh].T)
        assert np.array_equal(C[sh].sum(axis=1), Z[sh] * w.counts)
    alpha = lat.sro()[0]
    assert np.all(np.abs(alpha) < 1.0)
    say("bcc800: local energies (sampled against the oracle) and clusters (invariants)")
    e = lat.local_energy()
    E = float(lat.energy()[0])
    assert abs(float(e.sum().item()) - E) <= 1e-9 * abs(E)
    cur = work.cpu().numpy()
    idx = np.random.default_rng(5).integers(0, w.N, 2000)
    assert np.array_equal(e[torch.from_numpy(idx).cuda()].cpu().numpy(),
                          O.local_energy_at(w.lattice, w.dims, w.K, w.S, cur, w.V, idx))
    thr = float(torch.quantile(e[::4096].float(), 0.15).item())
    label, size, nc = lat.clusters(thr, e=e)
    marked = e <= thr
    n_marked = int(marked.sum().item())
    assert int(size.sum(dtype=torch.int64).item()) == n_marked
    assert int((label >= 0).sum().item()) == n_marked
    ar = torch.arange(w.N, device="cuda", dtype=torch.int32)
    roots = label == ar
    assert int(roots.sum().item()) == int(nc.item()) == int((size > 0).sum().item())
    assert bool((label <= ar).all().item())
    lab = label.cpu().numpy()
    # sampled marked sites: their label is a root, and every marked nearest
    # neighbour carries the same label
    nbr_tab = O.shells(w.lattice, 1)
    for i in idx[:300]:
        if lab[i] < 0:
            continue
        assert lab[lab[i]] == lab[i]
        b = int(i % 2)
        c = int(i // 2)
        x, y, z = c % 800, (c // 800) % 800, c // 640000
        for v in (np.array(nbr_tab[1]).reshape(-1, 3)[:8]):
            hx, hy, hz = 2 * x + b + v[0], 2 * y + b + v[1], 2 * z + b + v[2]
            hx, hy, hz = hx % 1600, hy % 1600, hz % 1600
            bt = hx & 1
            j = bt + 2 * ((hx - bt) // 2 + 800 * ((hy - bt) // 2 + 800 * ((hz - bt) // 2)))
            if lab[j] >= 0:
                assert lab[j] == lab[i], (i, j)
    lat.close()


def test_fcc128_two_sweeps_energy_sro(smcx):
    w = I.c3_fcc()
    say("fcc128: two sweeps")
    occ0 = w.occ()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, occ0, ell=4)
    lat.set_epi(w.V)
    cells, nA = lat.schedule(0)
    assert nA == 256
    E0 = lat.energy()[0]
    C0 = O.pair_counts(w.lattice, w.dims, w.K, w.S, occ0)
    assert E0 == O.energy(C0, w.V)
    stats, ties, tc = lat.sweep(2, w.mc_seed, w.betas[:2], mode="stream")
    gpu = lat.occupancy()
    tnp, nt = lat.ties_to_numpy(ties, tc)
    ref = occ0.copy()
    res = O.run(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, w.mc_seed, w.betas[:2], replay=tnp,
                nthreads=NTHREADS)
    assert np.array_equal(gpu, ref)
    s = stats.cpu().numpy()
    assert s[0] == res.stats[0] and s[1] == res.stats[1]
    C1 = O.pair_counts(w.lattice, w.dims, w.K, w.S, ref)
    E1 = lat.energy()[0]
    assert abs(E1 - O.energy(C1, w.V)) <= 1e-12 * abs(E1)
    Z, _ = O.shells(w.lattice, w.S)
    assert np.allclose(lat.sro()[0], O.sro(C1, Z), rtol=1e-12, atol=1e-14)
    lat.close()


def test_bcc64_anneal_and_snapshot_counts(smcx):
    import torch
    w = I.c2_anneal_bcc()
    n = 8
    say("bcc64 anneal: first sweeps one by one, snapshots")
    occ0 = w.occ()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, occ0, ell=4)
    lat.set_epi(w.V)
    cells, _ = lat.schedule(0)
    ref = occ0.copy()
    snaps_gpu, snaps_ref = [], []
    for t in range(n):
        stats, ties, tc = lat.sweep(1, w.mc_seed, w.betas[t:t + 1], first_sweep=t, mode="stream")
        tnp, _ = lat.ties_to_numpy(ties, tc)
        O.run(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, w.mc_seed, w.betas[t:t + 1],
              first_sweep=t, replay=tnp, nthreads=NTHREADS)
        snaps_gpu.append(lat.occ.clone())
        snaps_ref.append(ref.copy())
        assert np.array_equal(lat.occupancy(), ref), f"sweep {t}"
    batch = torch.stack(snaps_gpu)
    C = smcx.energy_backward_counts(w.lattice, w.dims, w.K, w.S, batch).cpu().numpy()
    for j in range(n):
        assert np.array_equal(C[j], O.pair_counts(w.lattice, w.dims, w.K, w.S, snaps_ref[j]))
    lat.close()


def test_ladder_256_replicas(smcx):
    lad = I.c4a_ladder()
    n = 2
    say("ladder 256 replicas persistent")
    occs = [lad.occ(r) for r in range(lad.R)]
    dims = lad.dims()
    lat = smcx.Lattice(I.BCC, dims, lad.K, lad.S, np.concatenate(occs), ell=4)
    lat.set_epi(lad.V)
    bt = np.tile(lad.betas, (n, 1))
    stats, ties, tc = lat.sweep(n, 0, bt, mode="persistent")
    gpu = lat.occupancy()
    tnp, _ = lat.ties_to_numpy(ties, tc)
    s = stats.cpu().numpy().reshape(-1, 3)
    off = 0
    for r in range(lad.R):
        cells, _ = lat.schedule(r)
        ref = occs[r].copy()
        res = O.run(I.BCC, dims[r], lad.K, lad.S, cells, ref, lad.V, 0, bt[:, r], replica=r,
                    replay=tnp[tnp["replica"] == r], nthreads=4)
        assert np.array_equal(gpu[off:off + len(ref)], ref), f"replica {r} (edge {dims[r][0]})"
        assert s[r, 0] == res.stats[0] and s[r, 1] == res.stats[1]
        off += len(ref)
    lat.close()


def test_backward_4096_configs(smcx):
    import torch
    dims, occs, _ = I.c4b_fit_set()
    say("backward 4096 x bcc16")
    C = smcx.energy_backward_counts(I.BCC, dims, 4, 4, torch.from_numpy(occs).cuda()).cpu().numpy()
    Z, _ = O.shells(I.BCC, 4)
    Nk = np.bincount(occs[0], minlength=4)
    assert (C == C.transpose(0, 1, 3, 2)).all()
    assert (C.sum(axis=3) == (Z[None, :, None] * Nk[None, None, :])).all()
    for b in np.random.default_rng(0).choice(len(occs), 64, replace=False):
        assert np.array_equal(C[b], O.pair_counts(I.BCC, dims, 4, 4, occs[b]))
