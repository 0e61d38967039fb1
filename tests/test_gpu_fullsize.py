"""Full-size parity on the GPU: the workloads' own sizes, in the launch
configurations the benchmark times, compared site by site with the oracle.

- BCC 800^3 (1.024e9 sites), 4 species, 4 shells, 1200 K, link cells of 4:
  one full sweep in the benchmark's launch (stream mode, row windows, 16
  launches of the row kernel each running the 8 mini-steps of one (o_y, o_z)
  group) against the threaded oracle's sweep; pair counts, energy and
  Warren-Cowley SRO of the result against the oracle's; local energies
  sampled and clusters by their invariants.  Then single row-kernel launches
  (one 8-mini-step group each), one of them with a forced near-tie.
- The paper's large lattice shape, BCC 795^3: single row-kernel launches with
  4 shells (uneven link cells of 4 and 5) and with 2 shells (link cells of 3).
- FCC 128^3, 5 species: 50 sweeps with energy and SRO every 10 sweeps.
- BCC 64^3: the whole 2000-sweep linear anneal 3000 -> 300 K, final
  occupancy and the pair counts of all 64 snapshots (batched backward).
- 256-replica ladder with edges 16..48: every replica identical to the oracle
  in stream mode (row windows over replicas of different decompositions), as
  a replayed stream graph, and in persistent mode.
- Backward on 4096 configurations of BCC 16^3: sampled configurations equal to
  the oracle, invariants on all.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from gpu_cases import NTHREADS, say
from oracle import oracle as O
from paper_2503_12591_amd import inputs as I
from ties import forced_trial_tie

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smcx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_12591_amd import smcx as S
    S.lib()
    return S


@pytest.fixture(scope="module")
def bcc800(smcx):
    """The benchmark lattice: occupancy drawn on the device (seeded), a host
    copy of it for the oracle, and a Lattice built as the benchmark builds it."""
    w = I.c5_large_bcc()
    say("bcc800: generate")
    occ0_dev = I.occupancy_device(w.counts, seed=0)
    occ0 = occ0_dev.cpu().numpy()
    work = occ0_dev.clone()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, work, ell=4)
    lat.set_epi(w.V)
    cells, nA = lat.schedule(0)
    assert nA == 128 and [list(c) for c in cells] == [[4] * 200] * 3
    yield w, occ0_dev, occ0, work, lat, cells
    lat.close()


def test_large_bcc_full_sweep_benchmark_launch(smcx, bcc800):
    import torch
    w, occ0_dev, occ0, work, lat, cells = bcc800
    beta = float(w.betas[0])
    work.copy_(occ0_dev)
    say("bcc800: one sweep, benchmark launch")
    lat.timing(True)
    lat.timing_read()
    stats, ties, tc = lat.sweep(1, w.mc_seed, [beta], mode="stream")
    _, launches = lat.timing_read()
    lat.timing(False)
    assert launches == 16, launches  # one row-kernel launch per (o_y, o_z) group
    gpu = work.cpu().numpy()
    tnp, nt = lat.ties_to_numpy(ties, tc)
    s = stats.cpu().numpy()
    say(f"bcc800: oracle sweep on {NTHREADS} threads")
    ref = occ0.copy()
    res = O.run(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, w.mc_seed, [beta], replay=tnp, nthreads=NTHREADS)
    assert s[0] == res.stats[0] == w.N
    assert s[1] == res.stats[1] and s[2] == res.stats[2] == nt
    assert np.array_equal(gpu, ref), f"{int((gpu != ref).sum())} sites differ"
    del gpu
    say("bcc800: pair counts, energy, SRO against the oracle")
    C = lat.pair_counts().cpu().numpy()[0]
    Cref = O.pair_counts(w.lattice, w.dims, w.K, w.S, ref, nthreads=NTHREADS)
    assert np.array_equal(C, Cref)
    E = float(lat.energy()[0])
    Eref = O.energy(Cref, w.V)
    assert abs(E - Eref) <= 1e-12 * abs(Eref)
    Z, _ = O.shells(w.lattice, w.S)
    assert np.allclose(lat.sro()[0], O.sro(Cref, Z), rtol=1e-12, atol=1e-14)

    say("bcc800: local energies (sampled against the oracle) and clusters (invariants)")
    e = lat.local_energy()
    assert abs(float(e.sum().item()) - E) <= 1e-9 * abs(E)
    idx = np.random.default_rng(5).integers(0, w.N, 2000)
    assert np.array_equal(e[torch.from_numpy(idx).cuda()].cpu().numpy(),
                          O.local_energy_at(w.lattice, w.dims, w.K, w.S, ref, w.V, idx))
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
    nbr = np.array(O.shells(w.lattice, 1)[1][0]).reshape(-1, 3)
    for i in idx[:300]:
        if lab[i] < 0:
            continue
        assert lab[lab[i]] == lab[i]
        b = int(i % 2)
        c = int(i // 2)
        x, y, z = c % 800, (c // 800) % 800, c // 640000
        for v in nbr:
            hx, hy, hz = (2 * x + b + v[0]) % 1600, (2 * y + b + v[1]) % 1600, (2 * z + b + v[2]) % 1600
            bt = hx & 1
            j = bt + 2 * ((hx - bt) // 2 + 800 * ((hy - bt) // 2 + 800 * ((hz - bt) // 2)))
            if lab[j] >= 0:
                assert lab[j] == lab[i], (i, j)


@pytest.mark.parametrize("tau0,tie", [(0, True), (56, False), (120, False)])
def test_large_bcc_one_row_launch(smcx, bcc800, tau0, tie):
    """One row-kernel launch (the 8 mini-steps of one (o_y, o_z) group) from
    the initial configuration; with `tie`, at the inverse temperature that
    puts one trial of mini-step 0 on its threshold."""
    w, occ0_dev, occ0, work, lat, cells = bcc800
    beta, t = float(w.betas[0]), None
    if tie:
        t = forced_trial_tie(w.lattice, w.dims, w.K, w.S, cells, occ0, w.V, seed=w.mc_seed, replica=0, sweep=0)
        beta = t["beta"]
    say(f"bcc800: row launch tau {tau0}..{tau0 + 8} beta={beta!r} tie={tie}")
    work.copy_(occ0_dev)
    lat.timing(True)
    lat.timing_read()
    stats, ties, tc = lat.sweep_partial(0, tau0, tau0 + 8, w.mc_seed, [beta], mode="stream")
    _, launches = lat.timing_read()
    lat.timing(False)
    assert launches == 1
    gpu = work.cpu().numpy()
    tnp, nt = lat.ties_to_numpy(ties, tc)
    s = stats.cpu().numpy()
    ref = occ0.copy()
    res = O.run_ministeps(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, w.mc_seed, beta, 0, tau0, tau0 + 8,
                          replay=tnp, nthreads=NTHREADS)
    assert s[0] == res.stats[0] == 8 * 8_000_000
    assert s[1] == res.stats[1] and s[2] == res.stats[2] == nt
    assert np.array_equal(gpu, ref), f"{int((gpu != ref).sum())} sites differ"
    if tie:
        assert nt == 1 and (int(tnp[0]["replica"]), int(tnp[0]["sweep"]), int(tnp[0]["site"])) == (0, 0, t["site"])
        say(f"bcc800 tie: gpu decision {int(tnp[0]['decision'])}, oracle exp decision {int(t['u'] < t['P'])}")
        flip = tnp.copy()
        flip["decision"] = 1 - flip["decision"]
        other = occ0.copy()
        O.run_ministeps(w.lattice, w.dims, w.K, w.S, cells, other, w.V, w.mc_seed, beta, 0, tau0, tau0 + 8,
                        replay=flip, nthreads=NTHREADS)
        assert not np.array_equal(gpu, other)


@pytest.fixture(scope="module")
def bcc795(smcx):
    """The paper's large lattice shape (795^3 cells): one seeded occupancy on
    the device and its host copy, shared by both shell counts."""
    w = I.paper_large_bcc(4)
    say("bcc795: generate")
    occ0_dev = I.occupancy_device(w.counts, seed=w.occ_seed)
    yield occ0_dev, occ0_dev.cpu().numpy()


# (shells, link cell, first mini-step): with 4 shells the cells are 4 and 5
# (195 + 3 per axis, 250 mini-steps, groups of 10); with 2 shells all are 3
# (54 mini-steps, groups of 6).  Groups: the first, one past the shorter
# cells (o_y = 4: only the rows of the cells of 5 are active), the last.
@pytest.mark.parametrize("S,ell,tau0", [(4, 4, 0), (4, 4, 40), (4, 4, 240), (2, 3, 0), (2, 3, 24), (2, 3, 48)])
def test_paper_lattice_one_row_launch(smcx, bcc795, S, ell, tau0):
    """One row-kernel launch (every mini-step of one (o_y, o_z) group) on the
    paper's 795^3 lattice shape, site by site against the oracle."""
    occ0_dev, occ0 = bcc795
    w = I.paper_large_bcc(S)
    work = occ0_dev.clone()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, work, ell=ell)
    try:
        lat.set_epi(w.V)
        cells, nA = lat.schedule(0)
        if S == 4:
            assert nA == 250 and sorted(set(cells[0])) == [4, 5] and list(cells[0]).count(5) == 3
        else:
            assert nA == 54 and [list(c) for c in cells] == [[3] * 265] * 3
        g = 2 * max(cells[0])  # mini-steps of one (o_y, o_z) group
        beta = float(w.betas[0])
        say(f"bcc795 S={S} ell={ell}: row launch tau {tau0}..{tau0 + g}")
        lat.timing(True)
        lat.timing_read()
        stats, ties, tc = lat.sweep_partial(0, tau0, tau0 + g, w.mc_seed, [beta], mode="stream")
        _, launches = lat.timing_read()
        lat.timing(False)
        assert launches == 1
        gpu = work.cpu().numpy()
        tnp, nt = lat.ties_to_numpy(ties, tc)
        s = stats.cpu().numpy()
    finally:
        lat.close()
    del work
    ref = occ0.copy()
    res = O.run_ministeps(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, w.mc_seed, beta, 0, tau0, tau0 + g,
                          replay=tnp, nthreads=NTHREADS)
    assert s[0] == res.stats[0] > 0
    assert s[1] == res.stats[1] and s[2] == res.stats[2] == nt
    assert np.array_equal(gpu, ref), f"{int((gpu != ref).sum())} sites differ"


def test_fcc128_50_sweeps_energy_sro_every_10(smcx):
    w = I.c3_fcc()
    n = 50
    say(f"fcc128: {n} sweeps, energy and SRO every 10")
    occ0 = w.occ()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, occ0, ell=4)
    lat.set_epi(w.V)
    cells, nA = lat.schedule(0)
    assert nA == 256
    Z, _ = O.shells(w.lattice, w.S)
    ref = occ0.copy()
    for t0 in range(0, n + 1, w.measure_every):
        if t0 > 0:
            stats, ties, tc = lat.sweep(w.measure_every, w.mc_seed, w.betas[t0 - 10:t0], first_sweep=t0 - 10,
                                        mode="stream")
            tnp, nt = lat.ties_to_numpy(ties, tc)
            res = O.run(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, w.mc_seed, w.betas[t0 - 10:t0],
                        first_sweep=t0 - 10, replay=tnp, nthreads=NTHREADS)
            s = stats.cpu().numpy()
            assert s[0] == res.stats[0] and s[1] == res.stats[1] and s[2] == res.stats[2] == nt
            assert np.array_equal(lat.occupancy(), ref), f"after sweep {t0}"
        C = lat.pair_counts().cpu().numpy()[0]
        Cref = O.pair_counts(w.lattice, w.dims, w.K, w.S, ref, nthreads=NTHREADS)
        assert np.array_equal(C, Cref), f"counts at sweep {t0}"
        E = lat.energy()[0]
        assert abs(E - O.energy(Cref, w.V)) <= 1e-12 * abs(E)
        assert np.allclose(lat.sro()[0], O.sro(Cref, Z), rtol=1e-12, atol=1e-14)
        say(f"fcc128: sweep {t0} E = {E!r}")
    lat.close()


def test_bcc64_full_anneal_and_snapshot_counts(smcx):
    """The whole 2000-sweep anneal, 64 snapshots, their counts by the batched
    backward kernel."""
    import torch
    w = I.c2_anneal_bcc()
    snaps = w.extra["snapshots_after"]
    assert len(snaps) == 64 and snaps[-1] == 2000
    say("bcc64 anneal: 2000 sweeps in 64 chunks")
    occ0 = w.occ()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, occ0, ell=4)
    lat.set_epi(w.V)
    cells, _ = lat.schedule(0)
    stats = torch.zeros(3, dtype=torch.int64, device="cuda")
    ties = torch.zeros(4096 * O.TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    tc = torch.zeros(1, dtype=torch.int32, device="cuda")
    batch = torch.empty((64, w.N), dtype=torch.uint8, device="cuda")
    t = 0
    for j, t1 in enumerate(snaps):
        lat.sweep(t1 - t, w.mc_seed, w.betas[t:t1], first_sweep=t, mode="stream", stats=stats, ties=ties,
                  tie_count=tc)
        batch[j].copy_(lat.occ)
        t = t1
    C = smcx.energy_backward_counts(w.lattice, w.dims, w.K, w.S, batch).cpu().numpy()
    tnp, nt = lat.ties_to_numpy(ties, tc)
    s = stats.cpu().numpy()
    gpu_final = lat.occupancy()
    lat.close()
    say(f"bcc64 anneal: oracle on {NTHREADS} threads ({nt} near-ties)")
    ref = occ0.copy()
    ost = np.zeros(3, np.int64)
    t = 0
    for j, t1 in enumerate(snaps):
        res = O.run(w.lattice, w.dims, w.K, w.S, cells, ref, w.V, w.mc_seed, w.betas[t:t1], first_sweep=t,
                    replay=tnp, nthreads=NTHREADS)
        ost += res.stats
        assert np.array_equal(C[j], O.pair_counts(w.lattice, w.dims, w.K, w.S, ref, nthreads=NTHREADS)), \
            f"snapshot {j} (after sweep {t1})"
        t = t1
    assert np.array_equal(gpu_final, ref)
    assert s.tolist() == ost.tolist()


def oracle_replicas(lad, dims, occs, scheds, bt, tnp, first_sweep=0):
    """Every replica's run on the oracle, replicas spread over threads."""
    def one(r):
        ref = occs[r].copy()
        res = O.run(I.BCC, dims[r], lad.K, lad.S, scheds[r], ref, lad.V, 0, bt[:, r], first_sweep=first_sweep,
                    replica=r, replay=tnp[tnp["replica"] == r])
        return ref, res.stats
    with ThreadPoolExecutor(NTHREADS) as ex:
        return list(ex.map(one, range(lad.R)))


@pytest.mark.parametrize("mode", ["stream", "stream_graph", "persistent"])
def test_ladder_256_replicas(smcx, mode):
    import torch
    lad = I.c4a_ladder()
    n = 2
    say(f"ladder 256 replicas, {mode}")
    occs = [lad.occ(r) for r in range(lad.R)]
    dims = lad.dims()
    lat = smcx.Lattice(I.BCC, dims, lad.K, lad.S, np.concatenate(occs), ell=4)
    lat.set_epi(lad.V)
    bt = np.tile(lad.betas, (n, 1))
    if mode == "stream_graph":
        g = smcx.LadderGraph(lat, n, 0, lad.betas, first_sweep=0, mode="stream")
        g.launch()
        torch.cuda.synchronize()
        stats, ties, tc = g.stats, g.ties, g.tie_count
    else:
        stats, ties, tc = lat.sweep(n, 0, bt, mode=mode)
    gpu = lat.occupancy()
    tnp, _ = lat.ties_to_numpy(ties, tc)
    s = stats.cpu().numpy().reshape(-1, 3)
    scheds = [lat.schedule(r)[0] for r in range(lad.R)]
    if mode == "stream_graph":
        g.close()
    lat.close()
    out = oracle_replicas(lad, dims, occs, scheds, bt, tnp)
    off = 0
    for r in range(lad.R):
        ref, st = out[r]
        assert np.array_equal(gpu[off:off + len(ref)], ref), f"replica {r} (edge {dims[r][0]})"
        assert s[r].tolist() == st.tolist(), r
        off += len(ref)


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
