"""ctypes wrapper of the CPU oracle (``smcx_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never imports it.  It
imports nothing from the HIP package either.

Every function takes and returns numpy arrays.  The C source documents which
passage of the paper each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smcx_oracle.c")
# SMCX_ORACLE_LIB points the tests at another build of this source (the
# mutation tests use it to run the pins against planted mistakes)
LIB = os.environ.get("SMCX_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

BCC, FCC = 0, 1
MAXZ = 24

TIE_DTYPE = np.dtype([("replica", "<i4"), ("sweep", "<u4"), ("site", "<i8"),
                      ("decision", "<i4"), ("pad", "<i4")])
TRACE_DTYPE = np.dtype([("a", "<i8"), ("b", "<i8"), ("dE", "<f8"), ("k", "<i4"),
                        ("accepted", "<i4")])


def compile_source(src: str, out: str) -> str:
    """gcc, binary64, no contraction, OpenMP."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle (no-op for an external build named by SMCX_ORACLE_LIB)."""
    if os.environ.get("SMCX_ORACLE_LIB"):
        return LIB
    if force or not os.path.exists(LIB):
        compile_source(SRC, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        p = C.c_void_p
        i32, i64, u32, u64, dbl = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.or_shells.argtypes = [C.c_int, C.c_int, p, p]
        L.or_lmin.argtypes = [C.c_int, C.c_int, C.c_int]
        L.or_partition.argtypes = [C.c_int, C.c_int, p]
        L.or_philox4x32_10.argtypes = [p, p, p]
        L.or_philox4x32_10.restype = None
        L.or_pair_counts.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p]
        L.or_pair_counts_threads.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, i32]
        L.or_energy.argtypes = [C.c_int, C.c_int, p, p]
        L.or_energy.restype = dbl
        L.or_sro.argtypes = [C.c_int, C.c_int, p, p, p]
        L.or_delta_e.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, i64, i32, p, p]
        L.or_single_trial.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, u64, u32, u32, i64, dbl]
        L.or_run.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, p, p, u64, u32, u32, i32, p, p,
                             i32, p, p, i32, p, p, i64, i32]
        L.or_run_ministeps.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, p, p, u64, u32, u32,
                                       i32, i32, dbl, p, i32, p, p, i32, p, i32]
        L.or_max_threads.argtypes = []
        L.or_exchange.argtypes = [C.c_int, p, p, p, u64, u32, p, i32, p, p, i32, p]
        L.or_heat_capacity.argtypes = [C.c_int, p, dbl, i64]
        L.or_heat_capacity.restype = dbl
        L.or_local_energy.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, p]
        L.or_clusters.argtypes = [C.c_int, p, p, dbl, p, p, p, p]
        L.or_local_energy_at.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, p, i64, p]
        L.or_run_qsro.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, p, p, p, u64, u32, u32, i32, p, p, i32,
                                  p, p, i32, p, i32]
        L.or_qsro_local_energy.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, p, p]
        L.or_qsro_delta_e.argtypes = [C.c_int, p, C.c_int, C.c_int, p, p, p, i64, i32, p, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dims(L) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32).reshape(3))


def shells(lattice: int, S: int):
    """Return (Z[S], list of S arrays of shape (Z_s, 3)) for the first S shells."""
    Z = np.zeros(4, np.int32)
    d = np.zeros((4, MAXZ, 3), np.int32)
    rc = lib().or_shells(lattice, S, _ptr(Z), _ptr(d))
    if rc != 0:
        raise ValueError("or_shells failed")
    return Z[:S].copy(), [d[s, :Z[s]].copy() for s in range(S)]


def lmin(lattice: int, S: int, liz: bool = False) -> int:
    return int(lib().or_lmin(lattice, S, 1 if liz else 0))


def partition(L: int, ell: int) -> np.ndarray:
    sizes = np.zeros(max(L, 1), np.int32)
    n = lib().or_partition(L, ell, _ptr(sizes))
    if n < 0:
        raise ValueError("bad partition request")
    return sizes[:n].copy()


def default_cells(dims, ell: int):
    """Per-axis cell edges by the default rule, as a list of three arrays."""
    return [partition(int(L), ell) for L in dims]


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def pair_counts(lattice: int, dims, K: int, S: int, occ: np.ndarray, nthreads: int = 1) -> np.ndarray:
    """Directed pair counts C[S][K][K]; nthreads > 1 splits the sites over
    OpenMP threads (same integer result)."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    Cn = np.zeros((S, K, K), np.int64)
    if nthreads > 1:
        rc = lib().or_pair_counts_threads(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(Cn), nthreads)
    else:
        rc = lib().or_pair_counts(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(Cn))
    if rc != 0:
        raise ValueError("or_pair_counts failed")
    return Cn


def energy(Cn: np.ndarray, V: np.ndarray) -> float:
    S, K, _ = Cn.shape
    Cn = np.ascontiguousarray(Cn, dtype=np.int64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    return float(lib().or_energy(K, S, _ptr(Cn), _ptr(V)))


def sro(Cn: np.ndarray, Z) -> np.ndarray:
    S, K, _ = Cn.shape
    Cn = np.ascontiguousarray(Cn, dtype=np.int64)
    Zs = np.ascontiguousarray(np.asarray(Z, dtype=np.int32))
    alpha = np.zeros((S, K, K), np.float64)
    rc = lib().or_sro(K, S, _ptr(Zs), _ptr(Cn), _ptr(alpha))
    if rc != 0:
        raise ValueError("or_sro failed (absent species?)")
    return alpha


def delta_e(lattice, dims, K, S, occ, V, a: int, k: int):
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    V = np.ascontiguousarray(V, dtype=np.float64)
    dE = np.zeros(1, np.float64)
    b = np.zeros(1, np.int64)
    rc = lib().or_delta_e(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(V), a, k, _ptr(dE),
                          _ptr(b))
    if rc != 0:
        raise ValueError("or_delta_e failed")
    return float(dE[0]), int(b[0])


def single_trial(lattice, dims, K, S, occ: np.ndarray, V, seed: int, replica: int, sweep: int,
                 a: int, beta: float) -> int:
    """One trial in place on ``occ`` (uint8, C-contiguous).  Returns flags."""
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous
    V = np.ascontiguousarray(V, dtype=np.float64)
    f = lib().or_single_trial(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(V), seed, replica,
                              sweep, a, beta)
    if f < 0:
        raise ValueError("or_single_trial failed")
    return int(f)


class RunResult:
    def __init__(self, stats, ties, n_ties, trace):
        self.stats = stats
        self.ties = ties
        self.n_ties = n_ties
        self.trace = trace


def run(lattice, dims, K, S, cells, occ: np.ndarray, V, seed: int, betas, first_sweep: int = 0,
        replica: int = 0, replay=None, tie_cap: int = 1024, trace: bool = False,
        nthreads: int = 1) -> RunResult:
    """Run len(betas) sweeps in place on ``occ``.

    cells: list of three int arrays of link-cell edges (one per axis).
    replay: structured array of TIE_DTYPE whose decisions override near-ties.
    """
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous
    V = np.ascontiguousarray(V, dtype=np.float64)
    betas = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).reshape(-1))
    ncell = np.array([len(c) for c in cells], np.int32)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in cells]))
    if replay is None:
        replay = np.zeros(0, TIE_DTYPE)
    replay = np.ascontiguousarray(replay, dtype=TIE_DTYPE)
    stats = np.zeros(3, np.int64)
    ties = np.zeros(max(tie_cap, 1), TIE_DTYPE)
    n_ties = np.zeros(1, np.int32)
    n_trials = int(np.prod(dims)) * (2 if lattice == BCC else 4) * len(betas)
    tr = np.zeros(n_trials if trace else 0, TRACE_DTYPE)
    rc = lib().or_run(lattice, _ptr(_dims(dims)), K, S, _ptr(ncell), _ptr(flat), _ptr(occ),
                      _ptr(V), seed, replica, first_sweep, len(betas), _ptr(betas),
                      _ptr(replay), len(replay), _ptr(stats), _ptr(ties), tie_cap,
                      _ptr(n_ties), _ptr(tr) if trace else None, len(tr), nthreads)
    if rc != 0:
        raise ValueError("or_run failed (bad arguments)")
    nt = int(n_ties[0])
    return RunResult(stats, ties[:min(nt, tie_cap)].copy(), nt, tr if trace else None)


def run_ministeps(lattice, dims, K, S, cells, occ: np.ndarray, V, seed: int, beta: float,
                  sweep: int, tau_begin: int, tau_end: int, replica: int = 0, replay=None,
                  tie_cap: int = 1024, nthreads: int = 1) -> RunResult:
    """Mini-steps [tau_begin, tau_end) of one sweep, in place on ``occ``."""
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous
    V = np.ascontiguousarray(V, dtype=np.float64)
    ncell = np.array([len(c) for c in cells], np.int32)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in cells]))
    if replay is None:
        replay = np.zeros(0, TIE_DTYPE)
    replay = np.ascontiguousarray(replay, dtype=TIE_DTYPE)
    stats = np.zeros(3, np.int64)
    ties = np.zeros(max(tie_cap, 1), TIE_DTYPE)
    n_ties = np.zeros(1, np.int32)
    rc = lib().or_run_ministeps(lattice, _ptr(_dims(dims)), K, S, _ptr(ncell), _ptr(flat),
                                _ptr(occ), _ptr(V), seed, replica, sweep, tau_begin, tau_end, beta,
                                _ptr(replay), len(replay), _ptr(stats), _ptr(ties), tie_cap,
                                _ptr(n_ties), nthreads)
    if rc != 0:
        raise ValueError("or_run_ministeps failed (bad arguments)")
    nt = int(n_ties[0])
    return RunResult(stats, ties[:min(nt, tie_cap)].copy(), nt, None)


def max_threads() -> int:
    return int(lib().or_max_threads())


def exchange(E, beta_slot, rep_at, seed: int, round_: int, replay=None, stats=None,
             tie_cap: int = 64):
    """One replica-exchange round (``or_exchange``).  rep_at (int32, slot ->
    replica) and stats ([R-1][2] int64: attempts, acceptances per slot pair)
    are updated in place.  Returns (ties, n_ties)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    beta_slot = np.ascontiguousarray(beta_slot, dtype=np.float64)
    assert rep_at.dtype == np.int32 and rep_at.flags.c_contiguous
    R = len(rep_at)
    if stats is None:
        stats = np.zeros((max(R - 1, 1), 2), np.int64)
    assert stats.dtype == np.int64 and stats.flags.c_contiguous
    if replay is None:
        replay = np.zeros(0, TIE_DTYPE)
    replay = np.ascontiguousarray(replay, dtype=TIE_DTYPE)
    ties = np.zeros(max(tie_cap, 1), TIE_DTYPE)
    n_ties = np.zeros(1, np.int32)
    rc = lib().or_exchange(R, _ptr(E), _ptr(beta_slot), _ptr(rep_at), seed, round_, _ptr(replay),
                           len(replay), _ptr(stats), _ptr(ties), tie_cap, _ptr(n_ties))
    if rc != 0:
        raise ValueError("or_exchange failed (rep_at is not a slot -> replica map)")
    nt = int(n_ties[0])
    return ties[:min(nt, tie_cap)].copy(), nt


def tempering(lattice, dims, K, S, cells, occs, V, seed: int, beta_slot, n_rounds: int,
              sweeps_per_round: int, first_round: int = 0, rep_at=None, replay=None,
              nthreads: int = 1):
    """Parallel tempering of R replicas of one lattice (``occs``: list of R
    uint8 arrays, updated in place).  Round j: every replica r runs sweeps
    j n .. j n + n - 1 (n = sweeps_per_round) at the beta of its slot, then
    the energies from fresh pair counts decide one exchange round j.

    Returns dict(rep_at, stats [R][3], xstats [R-1][2], ties (sweep and
    exchange near-ties), energies [n_rounds][R])."""
    R = len(occs)
    rep_at = np.arange(R, dtype=np.int32) if rep_at is None else np.array(rep_at, np.int32)
    beta_slot = np.asarray(beta_slot, np.float64)
    stats = np.zeros((R, 3), np.int64)
    xstats = np.zeros((max(R - 1, 1), 2), np.int64)
    ties, energies = [], []
    n = sweeps_per_round
    for j in range(first_round, first_round + n_rounds):
        slot_of = np.empty(R, np.int64)
        slot_of[rep_at] = np.arange(R)
        for r in range(R):
            res = run(lattice, dims, K, S, cells, occs[r], V, seed,
                      np.full(n, beta_slot[slot_of[r]]), first_sweep=j * n, replica=r,
                      replay=replay, nthreads=nthreads)
            stats[r] += res.stats
            ties.append(res.ties)
        E = np.array([energy(pair_counts(lattice, dims, K, S, occs[r]), V) for r in range(R)])
        energies.append(E)
        t, _ = exchange(E, beta_slot, rep_at, seed, j, replay=replay, stats=xstats)
        ties.append(t)
    return dict(rep_at=rep_at, stats=stats, xstats=xstats,
                ties=np.concatenate(ties) if ties else np.zeros(0, TIE_DTYPE),
                energies=np.array(energies))


def heat_capacity(E, beta: float, N: int) -> float:
    """Heat capacity per site in units of k_B from recorded energies
    (``or_heat_capacity``: beta^2 Var(E) / N, two-pass, population variance)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    return float(lib().or_heat_capacity(len(E), _ptr(E), float(beta), int(N)))


def anneal(lattice, dims, K, S, cells, occ: np.ndarray, V, seed: int, beta_steps, warmup: int,
           record: int, first_sweep: int = 0, replica: int = 0, replay=None, nthreads: int = 1):
    """Stepwise anneal of one replica (``occ`` updated in place): step s runs
    ``warmup`` sweeps at beta_steps[s], then ``record`` sweeps each followed by
    the energy; the step's heat capacity comes from its recorded energies.
    Sweep indices continue from first_sweep.  Returns dict(E [n_steps][record],
    cv [n_steps], stats [3], ties)."""
    beta_steps = np.asarray(beta_steps, np.float64)
    n_steps = len(beta_steps)
    N = len(occ)
    E = np.zeros((n_steps, record), np.float64)
    cv = np.zeros(n_steps, np.float64)
    stats = np.zeros(3, np.int64)
    ties = []
    for s, b in enumerate(beta_steps):
        t0 = first_sweep + s * (warmup + record)
        if warmup:
            res = run(lattice, dims, K, S, cells, occ, V, seed, np.full(warmup, b), first_sweep=t0,
                      replica=replica, replay=replay, nthreads=nthreads)
            stats += res.stats
            ties.append(res.ties)
        for j in range(record):
            res = run(lattice, dims, K, S, cells, occ, V, seed, [b], first_sweep=t0 + warmup + j,
                      replica=replica, replay=replay, nthreads=nthreads)
            stats += res.stats
            ties.append(res.ties)
            E[s, j] = energy(pair_counts(lattice, dims, K, S, occ), V)
        if record:
            cv[s] = heat_capacity(E[s], b, N)
    return dict(E=E, cv=cv, stats=stats,
                ties=np.concatenate(ties) if ties else np.zeros(0, TIE_DTYPE))


def local_energy(lattice, dims, K, S, occ, V) -> np.ndarray:
    """Per-site local energies (``or_local_energy``)."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    V = np.ascontiguousarray(V, dtype=np.float64)
    e = np.zeros(len(occ), np.float64)
    if lib().or_local_energy(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(V), _ptr(e)) != 0:
        raise ValueError("or_local_energy failed")
    return e


def local_energy_at(lattice, dims, K, S, occ, V, idx) -> np.ndarray:
    """Local energies of the listed sites only (``or_local_energy_at``)."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    V = np.ascontiguousarray(V, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    e = np.zeros(len(idx), np.float64)
    if lib().or_local_energy_at(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(V), _ptr(idx), len(idx),
                                _ptr(e)) != 0:
        raise ValueError("or_local_energy_at failed")
    return e


def clusters(lattice, dims, e, threshold: float):
    """Clusters of sites with e <= threshold (``or_clusters``): returns
    (label int32 [N], size int32 [N], n_clusters)."""
    e = np.ascontiguousarray(e, dtype=np.float64)
    N = len(e)
    label = np.zeros(N, np.int32)
    size = np.zeros(N, np.int32)
    nc = np.zeros(1, np.int64)
    stack = np.zeros(max(N, 1), np.int64)
    if lib().or_clusters(lattice, _ptr(_dims(dims)), _ptr(e), float(threshold), _ptr(label), _ptr(size),
                         _ptr(nc), _ptr(stack)) != 0:
        raise ValueError("or_clusters failed")
    return label, size, int(nc[0])


def run_qsro(lattice, dims, K, S, cells, occ: np.ndarray, V, W, seed: int, betas, first_sweep: int = 0,
             replica: int = 0, replay=None, tie_cap: int = 1024, nthreads: int = 1) -> RunResult:
    """Sweeps under the qSRO model (``or_run_qsro``), in place on ``occ``."""
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous
    V = np.ascontiguousarray(V, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    betas = np.ascontiguousarray(np.asarray(betas, dtype=np.float64).reshape(-1))
    ncell = np.array([len(c) for c in cells], np.int32)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in cells]))
    if replay is None:
        replay = np.zeros(0, TIE_DTYPE)
    replay = np.ascontiguousarray(replay, dtype=TIE_DTYPE)
    stats = np.zeros(3, np.int64)
    ties = np.zeros(max(tie_cap, 1), TIE_DTYPE)
    n_ties = np.zeros(1, np.int32)
    rc = lib().or_run_qsro(lattice, _ptr(_dims(dims)), K, S, _ptr(ncell), _ptr(flat), _ptr(occ), _ptr(V),
                           _ptr(W), seed, replica, first_sweep, len(betas), _ptr(betas), _ptr(replay),
                           len(replay), _ptr(stats), _ptr(ties), tie_cap, _ptr(n_ties), nthreads)
    if rc != 0:
        raise ValueError("or_run_qsro failed (bad arguments or an edge <= c_max + 1)")
    nt = int(n_ties[0])
    return RunResult(stats, ties[:min(nt, tie_cap)].copy(), nt, None)


def qsro_local_energy(lattice, dims, K, S, occ, V, W) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    V = np.ascontiguousarray(V, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    e = np.zeros(len(occ), np.float64)
    if lib().or_qsro_local_energy(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(V), _ptr(W), _ptr(e)) != 0:
        raise ValueError("or_qsro_local_energy failed")
    return e


def qsro_delta_e(lattice, dims, K, S, occ, V, W, a: int, k: int):
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    V = np.ascontiguousarray(V, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    dE = np.zeros(1, np.float64)
    b = np.zeros(1, np.int64)
    if lib().or_qsro_delta_e(lattice, _ptr(_dims(dims)), K, S, _ptr(occ), _ptr(V), _ptr(W), a, k, _ptr(dE),
                             _ptr(b)) != 0:
        raise ValueError("or_qsro_delta_e failed")
    return float(dE[0]), int(b[0])
