"""Parity of the HIP path with the CPU oracle, through the C ABI (GPU).

Bar: pair counts, trajectories (occupancy after the run and after every
sweep), attempted / accepted counts and near-tie counts identical; energies
and Warren-Cowley SRO within 1e-12 relative (in practice identical, since
they are formed from identical integer counts in the same order).
"""
import numpy as np
import pytest

from gpu_cases import NTHREADS, gpu_vs_oracle, rand_occ, say, sym_V
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


@pytest.mark.parametrize("lattice,dims,K,S", [
    (BCC, (8, 8, 8), 4, 2), (BCC, (5, 6, 7), 4, 4), (FCC, (6, 5, 7), 5, 4), (BCC, (2, 2, 2), 2, 4),
    (FCC, (2, 3, 2), 3, 4), (BCC, (9, 4, 3), 8, 3), (FCC, (4, 4, 4), 8, 1), (BCC, (33, 17, 9), 2, 4),
    # rows of 48 cells and more: whole-row slabs, rows and planes wrapping inside one slab
    (BCC, (50, 9, 7), 4, 4), (FCC, (48, 5, 6), 3, 4), (BCC, (96, 2, 3), 2, 4), (BCC, (64, 13, 21), 4, 3),
    # five species: 6-bit fields in the slabs
    (FCC, (48, 5, 6), 5, 4), (BCC, (50, 9, 7), 5, 4), (FCC, (56, 3, 11), 5, 2),
])
def test_pair_counts_energy_sro(smcx, lattice, dims, K, S):
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ = rand_occ(N, K, 7, equi=True)
    V = sym_V(S, K, 0.05, 3)
    say(f"pair_counts lattice={lattice} dims={dims} K={K} S={S}")
    lat = smcx.Lattice(lattice, dims, K, S, occ)
    lat.set_epi(V)
    C = lat.pair_counts().cpu().numpy()[0]
    ref = O.pair_counts(lattice, dims, K, S, occ)
    assert np.array_equal(C, ref)
    E = lat.energy()[0]
    Eref = O.energy(ref, V)
    assert abs(E - Eref) <= 1e-12 * max(1.0, abs(Eref))
    Z, _ = O.shells(lattice, S)
    if (np.bincount(occ, minlength=K) > 0).all():
        a = lat.sro()[0]
        aref = O.sro(ref, Z)
        assert np.allclose(a, aref, rtol=1e-12, atol=1e-12)
    lat.close()


def test_pair_counts_multi_replica(smcx):
    dims = np.array([[5, 5, 5], [8, 6, 7], [4, 4, 9]], np.int32)
    K, S = 4, 4
    occs = [rand_occ(int(2 * np.prod(d)), K, 11 + r) for r, d in enumerate(dims)]
    say("pair_counts multi-replica")
    lat = smcx.Lattice(BCC, dims, K, S, np.concatenate(occs))
    lat.set_epi(sym_V(S, K, 0.05, 1))
    C = lat.pair_counts().cpu().numpy()
    for r in range(3):
        assert np.array_equal(C[r], O.pair_counts(BCC, dims[r], K, S, occs[r]))
    lat.close()


@pytest.mark.parametrize("lattice,dims,K,S,B", [(BCC, (52, 6, 5), 4, 4, 3), (FCC, (48, 4, 4), 4, 4, 2),
                                               (FCC, (48, 3, 5), 5, 4, 3)])
def test_energy_backward_batch_wide_rows(smcx, lattice, dims, K, S, B):
    import torch
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occs = np.stack([rand_occ(N, K, 300 + b, equi=False) for b in range(B)])
    say(f"energy_backward wide rows lattice={lattice} dims={dims} B={B}")
    C = smcx.energy_backward_counts(lattice, dims, K, S, torch.from_numpy(occs).cuda()).cpu().numpy()
    for b in range(B):
        assert np.array_equal(C[b], O.pair_counts(lattice, dims, K, S, occs[b]))


def test_energy_backward_batch_and_autograd(smcx):
    import torch
    dims, K, S, B = (5, 4, 6), 4, 4, 7
    N = 2 * 5 * 4 * 6
    occs = np.stack([rand_occ(N, K, 100 + b) for b in range(B)])
    say("energy_backward batch")
    t = torch.from_numpy(occs).cuda()
    C = smcx.energy_backward_counts(BCC, dims, K, S, t).cpu().numpy()
    for b in range(B):
        assert np.array_equal(C[b], O.pair_counts(BCC, dims, K, S, occs[b]))
    V = torch.tensor(sym_V(S, K, 0.05, 2), dtype=torch.float64, device="cuda", requires_grad=True)
    E = smcx.EnergyFn().apply(V, t, BCC, dims)
    g = torch.arange(1, B + 1, dtype=torch.float64, device="cuda")
    (E * g).sum().backward()
    expect = 0.5 * (np.arange(1, B + 1)[:, None, None, None] * C).sum(axis=0)
    assert np.allclose(V.grad.cpu().numpy(), expect, rtol=0, atol=1e-9)
    Eref = [O.energy(C[b], V.detach().cpu().numpy()) for b in range(B)]
    # the same binary64 sum as the oracle's (s, k, l ascending)
    assert np.array_equal(E.detach().cpu().numpy(), np.array(Eref))


def test_energy_autograd_gradcheck_and_central_differences(smcx):
    """The HIP autograd path of E(sigma; V) against finite differences of its
    own forward: torch.autograd.gradcheck in binary64 on a small batch, and
    central differences of the summed energy along every entry of V (E is
    linear in V, so the differences are exact up to rounding)."""
    import torch
    dims, K, S, B = (4, 4, 4), 3, 4, 5
    occs = np.stack([rand_occ(128, K, 200 + b, equi=False) for b in range(B)])
    t = torch.from_numpy(occs).cuda()
    fn = smcx.EnergyFn()
    V = torch.tensor(sym_V(S, K, 0.05, 9), dtype=torch.float64, device="cuda", requires_grad=True)
    say("gradcheck EnergyFn")
    assert torch.autograd.gradcheck(lambda v: fn.apply(v, t, BCC, dims), (V,), eps=1e-6, atol=1e-8, rtol=1e-7)
    g = torch.tensor(np.random.default_rng(3).normal(size=B), dtype=torch.float64, device="cuda")
    (fn.apply(V, t, BCC, dims) * g).sum().backward()
    grad = V.grad.cpu().numpy()
    h = 1e-3
    Vn = V.detach()
    fd = np.zeros_like(grad)
    for idx in np.ndindex(S, K, K):
        e = torch.zeros_like(Vn)
        e[idx] = h
        plus = float((fn.apply(Vn + e, t, BCC, dims) * g).sum())
        minus = float((fn.apply(Vn - e, t, BCC, dims) * g).sum())
        fd[idx] = (plus - minus) / (2 * h)
    assert np.allclose(grad, fd, rtol=1e-9, atol=1e-9), np.abs(grad - fd).max()
    # and against brute-force counts: d/dV of sum_b g_b E_b is 1/2 sum_b g_b C_b
    Cref = np.stack([O.pair_counts(BCC, dims, K, S, occs[b]) for b in range(B)])
    expect = 0.5 * np.einsum("b,bskl->skl", g.cpu().numpy(), Cref)
    assert np.allclose(grad, expect, rtol=1e-13, atol=1e-12)


def test_energy_backward_rejects_bad_species(smcx):
    import torch
    occ = rand_occ(2 * 64, 4, 5)
    occ[77] = 4  # species 4 with K = 4
    t = torch.from_numpy(np.stack([rand_occ(128, 4, 6), occ])).cuda()
    with pytest.raises(smcx.SmcxError):
        smcx.energy_backward_counts(BCC, (4, 4, 4), 4, 2, t)
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["persistent", "stream", "plain"])
def test_small_bcc_case_every_sweep(smcx, mode):
    """BCC 8^3, 4 species, 2 shells, 1000 K: identical after every sweep."""
    w = I.c1_small_bcc()
    n = 100 if mode == "persistent" else 12
    gpu_vs_oracle(w.lattice, w.dims, w.K, w.S, w.occ(), w.V, w.betas[:n], seed=w.mc_seed,
                  mode=mode, check_every_sweep=True)


def test_small_bcc_case_full_run(smcx):
    w = I.c1_small_bcc()
    gpu_vs_oracle(w.lattice, w.dims, w.K, w.S, w.occ(), w.V, w.betas, seed=w.mc_seed,
                  mode="persistent")


@pytest.mark.parametrize("lattice,dims,K,S,ell,tile,mode", [
    (FCC, (6, 5, 7), 5, 4, 3, (0, 0, 0), "persistent"),
    (FCC, (6, 5, 7), 5, 4, 3, (2, 2, 2), "stream"),
    (FCC, (9, 8, 7), 4, 2, 4, (3, 1, 2), "stream"),
    (BCC, (11, 9, 13), 4, 4, 3, (4, 2, 3), "stream"),       # uneven cells 3/4 and 4/5
    (BCC, (17, 10, 9), 4, 4, 4, (16, 4, 4), "stream"),
    (BCC, (19, 7, 6), 3, 3, 5, (1, 1, 1), "persistent"),
    (BCC, (10, 10, 10), 8, 4, 3, (8, 4, 2), "stream"),       # 64-bit counters
    (FCC, (5, 5, 6), 7, 3, 3, (0, 0, 0), "persistent"),
    (BCC, (2, 2, 2), 2, 4, 4, (0, 0, 0), "persistent"),      # partner images in shell 4
    (BCC, (2, 3, 2), 3, 4, 4, (0, 0, 0), "stream"),
    (FCC, (2, 2, 3), 3, 4, 4, (0, 0, 0), "persistent"),
    (BCC, (3, 3, 3), 4, 4, 3, (1, 1, 1), "persistent"),
])
def test_trajectories_varied_geometry(smcx, lattice, dims, K, S, ell, tile, mode):
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ = rand_occ(N, K, sum(dims), equi=False)
    V = sym_V(S, K, 0.04, K + S)
    betas = I.beta_of_T(np.linspace(2500, 600, 6))
    gpu_vs_oracle(lattice, dims, K, S, occ, V, betas, seed=12345, mode=mode, ell=ell, tile=tile,
                  first_sweep=3)


@pytest.mark.parametrize("rows", [True, False])
@pytest.mark.parametrize("lattice,dims,K,S,ell", [
    (BCC, (16, 12, 20), 4, 4, 4),
    (BCC, (17, 13, 9), 4, 4, 4),      # uneven cells 4/5
    (BCC, (40, 8, 8), 4, 4, 4),       # ten cells along x, x-images in the window
    (FCC, (9, 8, 10), 5, 4, 3),       # 6-bit counters
    (BCC, (12, 9, 10), 4, 2, 3),      # two shells
    (FCC, (10, 9, 11), 5, 2, 3),      # five species, two shells (compile-time counts)
    (FCC, (12, 12, 12), 3, 3, 4),
    (BCC, (332, 8, 8), 4, 4, 4),      # long padded rows: a wave per window row when staging
    (BCC, (327, 9, 8), 4, 4, 4),      # long rows, uneven cells
    (FCC, (170, 6, 6), 5, 4, 4),      # long FCC rows, 6-bit counters
    (BCC, (16, 12, 8), 5, 4, 4),      # BCC with 6-bit counters (species codes 6 s)
    (BCC, (12, 8, 10), 7, 3, 4),      # BCC with 64-bit counters (up to 8 species)
])
def test_stream_rows_and_tiles(smcx, lattice, dims, K, S, ell, rows):
    """Stream mode with whole-row windows (all offsets o_x of a group in one
    launch) and with per-mini-step tile windows: both equal the oracle."""
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    occ = rand_occ(N, K, 7 * sum(dims))
    V = sym_V(S, K, 0.04, 3 * K + S)
    betas = I.beta_of_T(np.linspace(2000, 500, 5))
    gpu_vs_oracle(lattice, dims, K, S, occ, V, betas, seed=4242, mode="stream", ell=ell,
                  first_sweep=11, rows=rows)


@pytest.mark.parametrize("lattice,dims,K,S,ell,rows,per_sweep", [
    (BCC, (16, 12, 20), 4, 4, 4, True, 16),    # one launch per (o_y, o_z)
    (BCC, (16, 12, 20), 4, 4, 4, False, 64),   # one per offset, basis sites sharing it
    (BCC, (12, 12, 12), 4, 4, 3, True, 54),    # 2*3 <= 3 + 3: one mini-step per launch
    (BCC, (8, 8, 8), 4, 2, 4, True, 16),
])
def test_stream_launch_structure(smcx, lattice, dims, K, S, ell, rows, per_sweep):
    """The launches a sweep takes show which window scheme ran."""
    N = int(np.prod(dims)) * (2 if lattice == BCC else 4)
    lat = smcx.Lattice(lattice, dims, K, S, rand_occ(N, K, 3), ell=ell, rows=rows)
    lat.set_epi(sym_V(S, K, 0.03, 2))
    lat.timing(True)
    lat.timing_read()
    lat.sweep(2, 0, I.beta_of_T([900.0, 900.0]), mode="stream")
    _, launches = lat.timing_read()
    lat.close()
    assert launches == 2 * per_sweep


def test_stream_rows_partial_ranges(smcx):
    """Mini-step ranges that cut row groups (inside an o_x run and between
    basis sites) compose to the full sweep."""
    from paper_2503_12591_amd import smcx as S
    dims, K, Sh = (16, 12, 12), 4, 4
    occ0 = rand_occ(2 * 16 * 12 * 12, K, 31)
    V = sym_V(Sh, K, 0.04, 8)
    b = I.beta_of_T([1100.0])
    say("row partial ranges")
    full = S.Lattice(BCC, dims, K, Sh, occ0, ell=4)
    full.set_epi(V)
    full.sweep(1, 5, b, first_sweep=2, mode="stream")
    parts = S.Lattice(BCC, dims, K, Sh, occ0, ell=4)
    parts.set_epi(V)
    _, nA = parts.schedule(0)
    for lo, hi in [(0, 3), (3, 8), (8, 13), (13, 40), (40, 41), (41, nA)]:
        parts.sweep_partial(2, lo, hi, 5, b, mode="stream")
    assert np.array_equal(full.occupancy(), parts.occupancy())
    cells, _ = full.schedule(0)
    ref = occ0.copy()
    O.run(BCC, dims, K, Sh, cells, ref, V, 5, b, first_sweep=2)
    assert np.array_equal(full.occupancy(), ref)
    full.close()
    parts.close()


@pytest.mark.parametrize("dims", [
    [[16, 16, 16], [20, 16, 12], [12, 24, 16]],   # one decomposition: launches per (o_y, o_z) group
    [[16, 17, 16], [21, 18, 19], [13, 22, 20]],   # cells of 4 and 5: launches per group index
], ids=["same", "mixed"])
def test_stream_rows_multi_replica(smcx, dims):
    """Replicas of different shapes in one row launch per group (of the same
    mini-steps, or of each replica's q-th (o_y, o_z) group)."""
    from paper_2503_12591_amd import smcx as S
    dims = np.array(dims, np.int32)
    K, Sh = 4, 4
    occs = [rand_occ(int(2 * np.prod(d)), K, 50 + r) for r, d in enumerate(dims)]
    V = sym_V(Sh, K, 0.03, 21)
    betas = I.beta_of_T(np.array([500.0, 1200.0, 3000.0]))
    n = 3
    say("rows multi-replica")
    lat = S.Lattice(BCC, dims, K, Sh, np.concatenate(occs), ell=4)
    lat.set_epi(V)
    bt = np.tile(betas, (n, 1))
    stats, ties, tc = lat.sweep(n, 9, bt, mode="stream")
    gpu = lat.occupancy()
    tnp, _ = lat.ties_to_numpy(ties, tc)
    s = stats.cpu().numpy().reshape(-1, 3)
    off = 0
    for r in range(len(dims)):
        cells, _ = lat.schedule(r)
        ref = occs[r].copy()
        res = O.run(BCC, dims[r], K, Sh, cells, ref, V, 9, bt[:, r], replica=r,
                    replay=tnp[tnp["replica"] == r])
        assert np.array_equal(gpu[off:off + len(ref)], ref), f"replica {r}"
        assert s[r, 0] == res.stats[0] and s[r, 1] == res.stats[1]
        off += len(ref)
    lat.close()


def test_explicit_partition(smcx):
    dims = (12, 10, 9)
    cells = [np.array([3, 5, 4]), np.array([4, 3, 3]), np.array([9])]
    occ = rand_occ(2 * 12 * 10 * 9, 4, 5)
    V = sym_V(4, 4, 0.04, 9)
    gpu_vs_oracle(BCC, dims, 4, 4, occ, V, I.beta_of_T([900.0] * 4), seed=77, mode="stream",
                  cells=cells, tile=(2, 2, 1))


def test_seed_sweep_and_replica_keys_change_the_stream(smcx):
    """Different seeds / first sweep give different trajectories (the key and
    counter are really used), each still matching the oracle."""
    w = I.c1_small_bcc()
    a = gpu_vs_oracle(w.lattice, w.dims, w.K, w.S, w.occ(), w.V, w.betas[:3], seed=1)
    b = gpu_vs_oracle(w.lattice, w.dims, w.K, w.S, w.occ(), w.V, w.betas[:3], seed=2)
    c = gpu_vs_oracle(w.lattice, w.dims, w.K, w.S, w.occ(), w.V, w.betas[:3], seed=1, first_sweep=9)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_partial_sweeps_compose(smcx):
    w = I.c1_small_bcc()
    from paper_2503_12591_amd import smcx as S
    say("partial sweeps")
    occ0 = w.occ()
    full = S.Lattice(w.lattice, w.dims, w.K, w.S, occ0)
    full.set_epi(w.V)
    full.sweep(1, 0, w.betas[:1], first_sweep=4, mode="stream")
    parts = S.Lattice(w.lattice, w.dims, w.K, w.S, occ0)
    parts.set_epi(w.V)
    _, nA = parts.schedule(0)
    for lo, hi in [(0, 37), (37, 38), (38, nA)]:
        parts.sweep_partial(4, lo, hi, 0, w.betas[:1], mode="persistent")
    assert np.array_equal(full.occupancy(), parts.occupancy())
    full.close()
    parts.close()


def ladder_inputs(R, lo, hi, seed=3):
    g = np.random.default_rng(seed)
    edges = g.integers(lo, hi + 1, size=R)
    dims = np.stack([edges, np.roll(edges, 1), np.roll(edges, 2)], axis=1).astype(np.int32)
    K, S = 4, 4
    occs = [rand_occ(int(2 * np.prod(d)), K, 1000 + r) for r, d in enumerate(dims)]
    V = sym_V(S, K, 0.02, 4)
    betas = I.beta_of_T(300.0 * 10.0 ** (np.arange(R) / max(R - 1, 1)))
    return dims, K, S, occs, V, betas


@pytest.mark.parametrize("mode", ["persistent", "stream", "plain"])
def test_ladder_replicas_match_oracle(smcx, mode):
    dims, K, S, occs, V, betas = ladder_inputs(6, 4, 11)
    n = 3
    say(f"ladder R=6 mode={mode}")
    lat = smcx.Lattice(BCC, dims, K, S, np.concatenate(occs))
    lat.set_epi(V)
    bt = np.tile(betas, (n, 1))
    stats, ties, tc = lat.sweep(n, 99, bt, first_sweep=0, mode=mode)
    gpu = lat.occupancy()
    tnp, _ = lat.ties_to_numpy(ties, tc)
    s = stats.cpu().numpy().reshape(-1, 3)
    off = 0
    for r in range(len(dims)):
        cells, _ = lat.schedule(r)
        ref = occs[r].copy()
        res = O.run(BCC, dims[r], K, S, cells, ref, V, 99, bt[:, r], replica=r,
                    replay=tnp[tnp["replica"] == r])
        N = len(ref)
        assert np.array_equal(gpu[off:off + N], ref), f"replica {r}"
        assert s[r, 0] == res.stats[0] and s[r, 1] == res.stats[1]
        off += N
    lat.close()


@pytest.mark.parametrize("mode", ["persistent", "stream", "plain"])
def test_ladder_graph_replays_continue_the_chain(smcx, mode):
    import torch
    dims, K, S, occs, V, betas = ladder_inputs(5, 5, 9, seed=8)
    say(f"ladder graph {mode}")
    lat = smcx.Lattice(BCC, dims, K, S, np.concatenate(occs))
    lat.set_epi(V)
    g = smcx.LadderGraph(lat, 2, 31, betas, first_sweep=0, mode=mode)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        _ = lat.pair_counts().cpu()  # eager work between replays
    assert int(g.counter.item()) == 6
    gpu = lat.occupancy()
    off = 0
    for r in range(len(dims)):
        cells, _ = lat.schedule(r)
        ref = occs[r].copy()
        O.run(BCC, dims[r], K, S, cells, ref, V, 31, [betas[r]] * 6, replica=r)
        assert np.array_equal(gpu[off:off + len(ref)], ref), f"replica {r}"
        off += len(ref)
    g.close()
    lat.close()


def test_row_kernel_graph_replays(smcx):
    """Captured stream sweeps with whole-row windows continue the chain."""
    import torch
    dims, K, S = (16, 12, 20), 4, 4
    occ = rand_occ(2 * 16 * 12 * 20, K, 77)
    V = sym_V(S, K, 0.03, 5)
    b = float(I.beta_of_T(900.0))
    say("row kernel graph")
    lat = smcx.Lattice(BCC, dims, K, S, occ, ell=4)
    lat.set_epi(V)
    g = smcx.LadderGraph(lat, 3, 19, [b], first_sweep=0, mode="stream")
    for _ in range(2):
        g.launch()
        torch.cuda.synchronize()
    gpu = lat.occupancy()
    cells, _ = lat.schedule(0)
    ref = occ.copy()
    O.run(BCC, dims, K, S, cells, ref, V, 19, [b] * 6)
    assert np.array_equal(gpu, ref)
    assert int(g.stats.cpu().numpy()[0]) == 6 * len(occ)
    g.close()
    lat.close()


def test_invalid_occupancy_rejected(smcx):
    occ = np.zeros(2 * 4 * 4 * 4, np.uint8)
    occ[17] = 4
    with pytest.raises(smcx.SmcxError):
        smcx.Lattice(BCC, (4, 4, 4), 4, 2, occ)


def test_asymmetric_epi_rejected(smcx):
    occ = rand_occ(128, 4, 0)
    lat = smcx.Lattice(BCC, (4, 4, 4), 4, 2, occ)
    V = sym_V(2, 4, 0.05, 0)
    V[1, 0, 2] += 1e-9
    with pytest.raises(smcx.SmcxError):
        lat.set_epi(V)
    with pytest.raises(smcx.SmcxError):
        lat.sweep(1, 0, [1.0])  # EPI not set
    lat.close()
