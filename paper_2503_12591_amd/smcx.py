"""ctypes binding of libsmcx (C ABI in include/smcx.h).

Argument marshalling only: torch supplies device memory and the stream, every
step of the Monte Carlo path runs in the library's HIP kernels.  The module
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmcx.so")

BCC, FCC = 0, 1
MODE_AUTO, MODE_STREAM, MODE_PERSISTENT, MODE_PLAIN = 0, 1, 2, 3
FLAG_DOUBLE_BUFFER = 1
FLAG_TILES = 2
MODES = {"auto": MODE_AUTO, "stream": MODE_STREAM, "persistent": MODE_PERSISTENT, "plain": MODE_PLAIN}
TIE_DTYPE = np.dtype([("replica", "<i4"), ("sweep", "<u4"), ("site", "<i8"), ("decision", "<i4"),
                      ("pad", "<i4")])

EXPORTS = [
    "smcx_version", "smcx_last_error", "smcx_min_cell_edge", "smcx_workspace_size",
    "smcx_lattice_init", "smcx_lattice_destroy", "smcx_get_schedule", "smcx_set_epi", "smcx_sweep",
    "smcx_sweep_partial",
    "smcx_pair_counts", "smcx_energy", "smcx_sro", "smcx_energy_backward", "smcx_ladder_capture",
    "smcx_sweep_capture",
    "smcx_graph_launch", "smcx_graph_destroy", "smcx_timing_enable", "smcx_timing_read",
    "smcx_energy_dev", "smcx_exchange", "smcx_anneal", "smcx_local_energy", "smcx_clusters",
    "smcx_set_qsro", "smcx_sweep_qsro", "smcx_energy_of_counts", "smcx_energy_grad",
    "smcx_lattice_init_static",
]


class SmcxError(RuntimeError):
    pass


class Desc(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("n_species", C.c_int32), ("n_shells", C.c_int32),
                ("n_replicas", C.c_int32), ("dims", C.c_void_p), ("ell", C.c_void_p),
                ("ncell", C.c_void_p), ("cells", C.c_void_p), ("tile", C.c_int32 * 3),
                ("flags", C.c_uint32)]


_lib = None


def lib():
    """Load libsmcx.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SmcxError(f"{LIB_PATH} is not built; run `python -m paper_2503_12591_amd.build`")
    L = C.CDLL(LIB_PATH)
    p, i32, u32, u64, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_size_t
    L.smcx_version.argtypes = []
    L.smcx_last_error.argtypes = []
    L.smcx_last_error.restype = C.c_char_p
    L.smcx_min_cell_edge.argtypes = [i32, i32]
    L.smcx_workspace_size.argtypes = [C.POINTER(Desc), C.POINTER(sz)]
    L.smcx_lattice_init.argtypes = [C.POINTER(p), C.POINTER(Desc), p, p, sz, p]
    L.smcx_lattice_init_static.argtypes = [C.POINTER(p), C.POINTER(Desc), p, p]
    L.smcx_lattice_destroy.argtypes = [p]
    L.smcx_get_schedule.argtypes = [p, i32, p, p, p]
    L.smcx_set_epi.argtypes = [p, p, p]
    L.smcx_sweep.argtypes = [p, i32, u64, u32, p, p, p, i32, p, i32, p]
    L.smcx_sweep_partial.argtypes = [p, u32, i32, i32, u64, p, p, p, i32, p, i32, p]
    L.smcx_pair_counts.argtypes = [p, p, p]
    L.smcx_energy.argtypes = [p, p, p, p]
    L.smcx_sro.argtypes = [p, p, p, p]
    L.smcx_energy_backward.argtypes = [i32, p, i32, i32, p, i32, p, p]
    L.smcx_energy_of_counts.argtypes = [p, p, i32, i32, p, p]
    L.smcx_energy_grad.argtypes = [p, p, i32, i32, p, p]
    L.smcx_ladder_capture.argtypes = [p, i32, u64, p, p, p, p, i32, p, p, C.POINTER(p)]
    L.smcx_sweep_capture.argtypes = [p, i32, u64, p, p, p, p, i32, p, i32, p, C.POINTER(p)]
    L.smcx_graph_launch.argtypes = [p, p]
    L.smcx_graph_destroy.argtypes = [p]
    L.smcx_timing_enable.argtypes = [p, i32]
    L.smcx_timing_read.argtypes = [p, p, p]
    L.smcx_energy_dev.argtypes = [p, p, p, p]
    L.smcx_exchange.argtypes = [p, i32, u64, p, p, p, i32, p, p, p, p, i32, p, p]
    L.smcx_anneal.argtypes = [p, i32, i32, i32, u64, u32, p, p, p, p, p, p, i32, p, i32, p]
    L.smcx_local_energy.argtypes = [p, i32, p, p]
    L.smcx_clusters.argtypes = [p, i32, p, C.c_double, p, p, p, p]
    L.smcx_set_qsro.argtypes = [p, p, p, p]
    L.smcx_sweep_qsro.argtypes = [p, i32, u64, u32, p, p, p, i32, p, p]
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        msg = lib().smcx_last_error().decode(errors="replace")
        raise SmcxError(f"libsmcx error {rc}: {msg}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise SmcxError("no GPU visible: libsmcx runs on gfx950 devices only")
    return torch


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return a, a.ctypes.data_as(C.c_void_p)


def min_cell_edge(lattice: int, n_shells: int) -> int:
    v = lib().smcx_min_cell_edge(lattice, n_shells)
    if v < 0:
        _check(v)
    return v


class Lattice:
    """R replicas of one lattice kind and energy model, resident on the GPU.

    occ: host uint8 array of all replicas back to back (or a torch uint8 CUDA
    tensor, used in place).
    """

    def __init__(self, lattice: int, dims, K: int, S: int, occ, ell=None, cells=None,
                 tile=(0, 0, 0), double_buffer: bool = False, rows: bool = True,
                 static_workspace: bool = False):
        torch = _torch()
        self.torch = torch
        dims = np.asarray(dims, dtype=np.int32).reshape(-1, 3)
        self.R = dims.shape[0]
        self.lattice, self.K, self.S = lattice, K, S
        self.dims = dims
        self.m = 2 if lattice == BCC else 4
        self.N = (self.m * dims.prod(axis=1)).astype(np.int64)
        if isinstance(occ, torch.Tensor):
            assert occ.dtype == torch.uint8 and occ.is_cuda and occ.is_contiguous()
            self.occ = occ
        else:
            self.occ = torch.from_numpy(np.ascontiguousarray(occ, dtype=np.uint8)).cuda()
        if self.occ.numel() != int(self.N.sum()):
            raise SmcxError("occupancy size does not match dims")
        self._keep = []
        self._dims_arr, dptr = _host(dims, np.int32)
        d = Desc()
        d.lattice, d.n_species, d.n_shells, d.n_replicas = lattice, K, S, self.R
        d.dims = dptr
        if ell is not None:
            arr, ptr = _host(np.broadcast_to(np.asarray(ell, np.int32), (self.R,)), np.int32)
            self._keep.append(arr)
            d.ell = ptr
        if cells is not None:
            # cells: per replica a list of three arrays of edges
            nc = np.array([[len(c[a]) for a in range(3)] for c in cells], np.int32)
            flat = np.concatenate([np.asarray(c[a], np.int32) for c in cells for a in range(3)])
            a1, p1 = _host(nc, np.int32)
            a2, p2 = _host(flat, np.int32)
            self._keep += [a1, a2]
            d.ncell, d.cells = p1, p2
        for a in range(3):
            d.tile[a] = int(tile[a])
        d.flags = (FLAG_DOUBLE_BUFFER if double_buffer else 0) | (0 if rows else FLAG_TILES)
        self._desc = d
        nbytes = C.c_size_t(0)
        _check(lib().smcx_workspace_size(C.byref(d), C.byref(nbytes)))
        h = C.c_void_p()
        if static_workspace:
            # the library's own per-device workspace (smcx_lattice_init_static)
            self.ws = None
            _check(lib().smcx_lattice_init_static(C.byref(h), C.byref(d), _ptr(self.occ), _stream(torch)))
        else:
            self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device="cuda")
            base = self.ws.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            _check(lib().smcx_lattice_init(C.byref(h), C.byref(d), _ptr(self.occ), C.c_void_p(self._ws_ptr),
                                           nbytes.value, _stream(torch)))
        self.h = h
        self.ws_bytes = int(nbytes.value)
        self.counts = torch.zeros(self.R * S * K * K, dtype=torch.int64, device="cuda")
        self.V = None

    def close(self):
        if getattr(self, "h", None):
            lib().smcx_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration ----------------------------------------------------
    def schedule(self, r: int = 0):
        """(cells as three arrays of edges, n_ministeps) used by replica r."""
        nc = np.zeros(3, np.int32)
        cells = np.zeros(int(self.dims[r].sum()), np.int32)
        nA = np.zeros(1, np.int32)
        _check(lib().smcx_get_schedule(self.h, r, nc.ctypes.data_as(C.c_void_p),
                                       cells.ctypes.data_as(C.c_void_p), nA.ctypes.data_as(C.c_void_p)))
        out, pos = [], 0
        for a in range(3):
            out.append(cells[pos:pos + nc[a]].copy())
            pos += nc[a]
        return out, int(nA[0])

    def set_epi(self, V):
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(self.S, self.K, self.K))
        _check(lib().smcx_set_epi(self.h, V.ctypes.data_as(C.c_void_p), _stream(self.torch)))
        self.V = V.copy()

    # -- Monte Carlo ------------------------------------------------------
    def sweep(self, n_sweeps: int, seed: int, betas, first_sweep: int = 0, mode="auto",
              tie_cap: int = 4096, stats=None, ties=None, tie_count=None):
        """Run n_sweeps sweeps.  betas: [n_sweeps][R] (or [n_sweeps] for R = 1,
        or a CUDA float64 tensor of that shape).  Returns (stats, ties,
        tie_count) device tensors unless given."""
        torch = self.torch
        if isinstance(betas, torch.Tensor):
            b = betas.to(device="cuda", dtype=torch.float64).contiguous()
        else:
            b = torch.from_numpy(np.array(
                np.broadcast_to(np.asarray(betas, np.float64).reshape(n_sweeps, -1),
                                (n_sweeps, self.R)))).cuda()
        if stats is None:
            stats = torch.zeros(self.R * 3, dtype=torch.int64, device="cuda")
        if ties is None:
            ties = torch.zeros(max(tie_cap, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        if tie_count is None:
            tie_count = torch.zeros(1, dtype=torch.int32, device="cuda")
        mode = MODES[mode] if isinstance(mode, str) else int(mode)
        _check(lib().smcx_sweep(self.h, n_sweeps, C.c_uint64(seed), C.c_uint32(first_sweep), _ptr(b),
                                _ptr(stats), _ptr(ties), tie_cap, _ptr(tie_count), mode,
                                _stream(torch)))
        self._last_beta = b  # keep alive until the stream has consumed it
        return stats, ties, tie_count

    def set_qsro(self, V, W):
        """qSRO model parameters: V [S][K][K] (symmetric), W [S][K]."""
        V = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(self.S, self.K, self.K))
        W = np.ascontiguousarray(np.asarray(W, dtype=np.float64).reshape(self.S, self.K))
        _check(lib().smcx_set_qsro(self.h, V.ctypes.data_as(C.c_void_p), W.ctypes.data_as(C.c_void_p),
                                   _stream(self.torch)))

    def sweep_qsro(self, n_sweeps: int, seed: int, betas, first_sweep: int = 0, tie_cap: int = 4096,
                   stats=None, ties=None, tie_count=None):
        """n_sweeps sweeps under the qSRO model; betas [n_sweeps][R] (host)."""
        torch = self.torch
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(betas, np.float64).reshape(n_sweeps, -1),
                                                 (n_sweeps, self.R)))
        if stats is None:
            stats = torch.zeros(self.R * 3, dtype=torch.int64, device="cuda")
        if ties is None:
            ties = torch.zeros(max(tie_cap, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        if tie_count is None:
            tie_count = torch.zeros(1, dtype=torch.int32, device="cuda")
        _check(lib().smcx_sweep_qsro(self.h, n_sweeps, C.c_uint64(seed), C.c_uint32(first_sweep),
                                     b.ctypes.data_as(C.c_void_p), _ptr(stats), _ptr(ties), tie_cap,
                                     _ptr(tie_count), _stream(torch)))
        return stats, ties, tie_count

    def sweep_partial(self, sweep: int, tau_begin: int, tau_end: int, seed: int, betas, mode="auto",
                      tie_cap: int = 4096, stats=None, ties=None, tie_count=None):
        """Mini-steps [tau_begin, tau_end) of global sweep `sweep`; betas: [R]."""
        torch = self.torch
        b = torch.from_numpy(np.array(
            np.broadcast_to(np.asarray(betas, np.float64).reshape(-1), (self.R,)))).cuda()
        if stats is None:
            stats = torch.zeros(self.R * 3, dtype=torch.int64, device="cuda")
        if ties is None:
            ties = torch.zeros(max(tie_cap, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        if tie_count is None:
            tie_count = torch.zeros(1, dtype=torch.int32, device="cuda")
        mode = MODES[mode] if isinstance(mode, str) else int(mode)
        _check(lib().smcx_sweep_partial(self.h, C.c_uint32(sweep), tau_begin, tau_end, C.c_uint64(seed),
                                        _ptr(b), _ptr(stats), _ptr(ties), tie_cap, _ptr(tie_count), mode,
                                        _stream(torch)))
        self._last_beta = b
        return stats, ties, tie_count

    @staticmethod
    def ties_to_numpy(ties, tie_count):
        n = int(tie_count.item())
        raw = ties.cpu().numpy().view(TIE_DTYPE)
        return raw[:min(n, len(raw))].copy(), n

    # -- observables ------------------------------------------------------
    def pair_counts(self):
        _check(lib().smcx_pair_counts(self.h, _ptr(self.counts), _stream(self.torch)))
        return self.counts.view(self.R, self.S, self.K, self.K)

    def energy(self) -> np.ndarray:
        E = np.zeros(self.R, np.float64)
        _check(lib().smcx_energy(self.h, _ptr(self.counts), E.ctypes.data_as(C.c_void_p),
                                 _stream(self.torch)))
        return E

    def energy_dev(self, E=None):
        """Energies of every replica into a CUDA float64 tensor [R], no host
        synchronisation (smcx_energy_dev)."""
        if E is None:
            E = self.torch.zeros(self.R, dtype=self.torch.float64, device="cuda")
        _check(lib().smcx_energy_dev(self.h, _ptr(self.counts), _ptr(E), _stream(self.torch)))
        return E

    def anneal(self, beta_steps, warmup: int, record: int, seed: int, first_sweep: int = 0, mode="auto",
               tie_cap: int = 4096, stats=None, ties=None, tie_count=None):
        """Stepwise anneal (smcx_anneal): beta_steps [n_steps] or [n_steps][R].
        Returns dict of CUDA tensors E [n_steps][record][R], cv [n_steps][R]
        (heat capacity per site in units of k_B), stats, ties, tie_count."""
        torch = self.torch
        b = np.asarray(beta_steps, np.float64)
        n_steps = b.shape[0]
        b = torch.from_numpy(np.array(np.broadcast_to(b.reshape(n_steps, -1), (n_steps, self.R)))).cuda()
        E = torch.zeros((n_steps, max(record, 1), self.R), dtype=torch.float64, device="cuda")
        cv = torch.zeros((n_steps, self.R), dtype=torch.float64, device="cuda")
        if stats is None:
            stats = torch.zeros(self.R * 3, dtype=torch.int64, device="cuda")
        if ties is None:
            ties = torch.zeros(max(tie_cap, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        if tie_count is None:
            tie_count = torch.zeros(1, dtype=torch.int32, device="cuda")
        mode = MODES[mode] if isinstance(mode, str) else int(mode)
        _check(lib().smcx_anneal(self.h, n_steps, warmup, record, C.c_uint64(seed), C.c_uint32(first_sweep),
                                 _ptr(b), _ptr(self.counts), _ptr(E), _ptr(cv), _ptr(stats), _ptr(ties), tie_cap,
                                 _ptr(tie_count), mode, _stream(torch)))
        self._last_beta = b
        return dict(E=E[:, :record], cv=cv, stats=stats, ties=ties, tie_count=tie_count)

    def local_energy(self, r: int = 0, e=None):
        """Per-site local energies of replica r (CUDA float64 [N_r])."""
        if e is None:
            e = self.torch.empty(int(self.N[r]), dtype=self.torch.float64, device="cuda")
        _check(lib().smcx_local_energy(self.h, r, _ptr(e), _stream(self.torch)))
        return e

    def clusters(self, threshold: float, r: int = 0, e=None):
        """Clusters of sites with local energy <= threshold in replica r:
        (label int32 [N_r], size int32 [N_r], n_clusters int64 [1]) CUDA
        tensors; e (local energies) is computed when not given."""
        torch = self.torch
        if e is None:
            e = self.local_energy(r)
        n = int(self.N[r])
        label = torch.empty(n, dtype=torch.int32, device="cuda")
        size = torch.empty(n, dtype=torch.int32, device="cuda")
        nc = torch.zeros(1, dtype=torch.int64, device="cuda")
        _check(lib().smcx_clusters(self.h, r, _ptr(e), C.c_double(threshold), _ptr(label), _ptr(size), _ptr(nc),
                                   _stream(torch)))
        return label, size, nc

    def sro(self) -> np.ndarray:
        a = np.zeros((self.R, self.S, self.K, self.K), np.float64)
        _check(lib().smcx_sro(self.h, _ptr(self.counts), a.ctypes.data_as(C.c_void_p),
                              _stream(self.torch)))
        return a

    def occupancy(self) -> np.ndarray:
        return self.occ.cpu().numpy()

    # -- timing -----------------------------------------------------------
    def timing(self, enable: bool):
        _check(lib().smcx_timing_enable(self.h, 1 if enable else 0))

    def timing_read(self):
        ms = np.zeros(1, np.float64)
        n = np.zeros(1, np.int64)
        _check(lib().smcx_timing_read(self.h, ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)))
        return float(ms[0]), int(n[0])


class Tempering:
    """Parallel tempering over the R replicas (one size) of a Lattice.

    Round j: every replica runs sweeps j n .. j n + n - 1 (n =
    sweeps_per_round) at the inverse temperature of the slot holding it, then
    smcx_exchange trades neighbouring slots' replicas and writes the betas of
    the next round's sweeps.  Everything stays on the device; rep_at (slot ->
    replica), E (energies at the last exchange), xstats ([R-1][2] attempts,
    trades), stats ([R][3] sweep counters) and the shared tie log are CUDA
    tensors.
    """

    def __init__(self, lat: Lattice, beta_slot, seed: int, sweeps_per_round: int, mode="auto",
                 tie_cap: int = 4096):
        torch = lat.torch
        R = lat.R
        self.lat, self.seed, self.n, self.mode, self.tie_cap = lat, seed, sweeps_per_round, mode, tie_cap
        self.beta_slot = torch.tensor(np.asarray(beta_slot, np.float64).reshape(R), dtype=torch.float64,
                                      device="cuda")
        self.rep_at = torch.arange(R, dtype=torch.int32, device="cuda")
        self.beta_rows = self.beta_slot.repeat(sweeps_per_round, 1).contiguous()
        self.E = torch.zeros(R, dtype=torch.float64, device="cuda")
        self.xstats = torch.zeros(max(R - 1, 1) * 2, dtype=torch.int64, device="cuda")
        self.stats = torch.zeros(R * 3, dtype=torch.int64, device="cuda")
        self.ties = torch.zeros(max(tie_cap, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self.tie_count = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.round = 0

    def run(self, n_rounds: int):
        lat, torch = self.lat, self.lat.torch
        for _ in range(n_rounds):
            lat.sweep(self.n, self.seed, self.beta_rows, first_sweep=self.round * self.n, mode=self.mode,
                      tie_cap=self.tie_cap, stats=self.stats, ties=self.ties, tie_count=self.tie_count)
            _check(lib().smcx_exchange(lat.h, self.round, C.c_uint64(self.seed), _ptr(self.beta_slot),
                                       _ptr(self.rep_at), _ptr(self.beta_rows), self.n, _ptr(lat.counts),
                                       _ptr(self.E), _ptr(self.xstats), _ptr(self.ties), self.tie_cap,
                                       _ptr(self.tie_count), _stream(torch)))
            self.round += 1

    def ties_numpy(self):
        return Lattice.ties_to_numpy(self.ties, self.tie_count)


class LadderGraph:
    """n_sweeps sweeps of every replica captured in a replayable graph with
    fixed betas per replica; every replay continues the chain (the sweep index
    lives in a device counter).  mode "persistent" captures the one-launch
    ladder (smcx_ladder_capture); other modes capture smcx_sweep's launches
    (smcx_sweep_capture).  The default, "stream", replays one launch per
    mini-step group over all replicas, the faster of the two for ladders of
    many replicas."""

    def __init__(self, lat: Lattice, n_sweeps: int, seed: int, betas, first_sweep: int = 0,
                 tie_cap: int = 4096, mode: str = "stream"):
        torch = lat.torch
        self.lat = lat
        b = np.ascontiguousarray(np.asarray(betas, np.float64).reshape(-1))
        if mode != "persistent":
            b = np.ascontiguousarray(np.tile(b, (n_sweeps, 1)))
        self.beta = torch.from_numpy(b).cuda()
        self.counter = torch.tensor([first_sweep], dtype=torch.int32, device="cuda")
        self.stats = torch.zeros(lat.R * 3, dtype=torch.int64, device="cuda")
        self.ties = torch.zeros(max(tie_cap, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        self.tie_count = torch.zeros(1, dtype=torch.int32, device="cuda")
        g = C.c_void_p()
        # the legacy default stream cannot be captured: capture on a side stream
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            if mode == "persistent":
                _check(lib().smcx_ladder_capture(lat.h, n_sweeps, C.c_uint64(seed), _ptr(self.beta),
                                                 _ptr(self.counter), _ptr(self.stats), _ptr(self.ties),
                                                 tie_cap, _ptr(self.tie_count), _stream(torch),
                                                 C.byref(g)))
            else:
                _check(lib().smcx_sweep_capture(lat.h, n_sweeps, C.c_uint64(seed), _ptr(self.beta),
                                                _ptr(self.counter), _ptr(self.stats), _ptr(self.ties),
                                                tie_cap, _ptr(self.tie_count), MODES[mode], _stream(torch),
                                                C.byref(g)))
        torch.cuda.current_stream().wait_stream(side)
        self.g = g
        self.n_sweeps = n_sweeps

    def launch(self):
        _check(lib().smcx_graph_launch(self.g, _stream(self.lat.torch)))

    def close(self):
        if getattr(self, "g", None):
            lib().smcx_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def energy_backward_counts(lattice: int, dims, K: int, S: int, occ_batch):
    """Pair counts C[B][S][K][K] (int64 CUDA tensor) of a batch of
    configurations (uint8 CUDA tensor [B][N]); dE_b/dV = C_b / 2."""
    torch = _torch()
    assert occ_batch.dtype == torch.uint8 and occ_batch.is_cuda
    occ_batch = occ_batch.contiguous()
    B = occ_batch.shape[0]
    counts = torch.empty((B, S, K, K), dtype=torch.int64, device="cuda")
    d, dp = _host(np.asarray(dims, np.int32).reshape(3), np.int32)
    _check(lib().smcx_energy_backward(lattice, dp, K, S, _ptr(occ_batch), B, _ptr(counts),
                                      _stream(torch)))
    return counts


def energy_of_counts(counts, V):
    """E_b = 1/2 <C_b, V> (CUDA float64 [B]) from int64 counts [B][S][K][K]
    and a float64 V [S][K][K] (smcx_energy_of_counts)."""
    torch = _torch()
    counts = counts.contiguous()
    V = V.detach().to(dtype=torch.float64).contiguous()
    B = counts.shape[0]
    E = torch.empty(B, dtype=torch.float64, device="cuda")
    _check(lib().smcx_energy_of_counts(_ptr(counts), _ptr(V), B, V.numel(), _ptr(E), _stream(torch)))
    return E


def energy_grad(counts, g):
    """1/2 sum_b g_b C_b (CUDA float64 [S][K][K]) (smcx_energy_grad)."""
    torch = _torch()
    counts = counts.contiguous()
    g = g.detach().to(dtype=torch.float64).contiguous()
    B = counts.shape[0]
    grad = torch.empty(counts.shape[1:], dtype=torch.float64, device="cuda")
    _check(lib().smcx_energy_grad(_ptr(counts), _ptr(g), B, grad.numel(), _ptr(grad), _stream(torch)))
    return grad


def _make_energy_fn():
    import torch

    class EnergyFn(torch.autograd.Function):
        """E_b = 1/2 <C_b, V> for a batch of configurations; dE_b/dV = C_b / 2.

        The counts come from the HIP pair-count kernel (smcx_energy_backward),
        the energies and the gradient from smcx_energy_of_counts and
        smcx_energy_grad, all in binary64.  `counts` may pass the batch's
        counts when they are already known (they do not depend on V)."""

        @staticmethod
        def forward(ctx, V, occ_batch, lattice, dims, counts=None):
            S, K, _ = V.shape
            if counts is None:
                counts = energy_backward_counts(lattice, dims, K, S, occ_batch)
            ctx.save_for_backward(counts)
            ctx.v_dtype = V.dtype
            return energy_of_counts(counts, V).to(V.dtype)

        @staticmethod
        def backward(ctx, g):
            (counts,) = ctx.saved_tensors
            return energy_grad(counts, g).to(ctx.v_dtype), None, None, None, None

    return EnergyFn


_energy_fn = None


def EnergyFn():
    global _energy_fn
    if _energy_fn is None:
        _energy_fn = _make_energy_fn()
    return _energy_fn


def autotune(lattice: int, dims, K: int, S: int, occ, V, betas, seed: int = 0, tiles=None,
             modes=("persistent", "stream"), ells=(None,), rows=(True, False), sweeps: int = 2,
             cache: str | None = None):
    """Choose the launch configuration with the most attempted swaps/s.

    Every candidate (tile, mode, row windows or not, link-cell edge) runs
    `sweeps` sweeps (after
    one untimed sweep) on a fresh copy of `occ` (host uint8 array or CUDA
    tensor, all replicas back to back) with inverse temperatures `betas` ([R]
    or scalar).  Tile and mode leave the trajectory unchanged; a link-cell
    edge other than None is a different partition, which `Lattice.schedule`
    exports for replay.  With `cache` (a JSON file), a result for the same
    geometry and candidate set is reused.  Returns a dict with the best
    "tile", "mode", "ell", its "swaps_per_s" and the full "table".
    """
    import hashlib
    import json
    torch = _torch()
    dims = np.asarray(dims, np.int32).reshape(-1, 3)
    if tiles is None:
        tiles = [(16, 4, 2), (16, 4, 4), (8, 4, 4), (8, 8, 2), (4, 4, 4)]
    key_src = json.dumps([lattice, dims.tolist(), K, S, [list(t) for t in tiles], list(modes),
                          [e if e is None else int(e) for e in ells], [bool(x) for x in rows], sweeps])
    key = hashlib.sha256(key_src.encode()).hexdigest()[:16]
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
        if key in db:
            return db[key]
    if isinstance(occ, torch.Tensor):
        occ0 = occ.detach().to("cuda").contiguous()
    else:
        occ0 = torch.from_numpy(np.ascontiguousarray(occ, dtype=np.uint8)).cuda()
    R = dims.shape[0]
    N = int((dims.prod(axis=1) * (2 if lattice == BCC else 4)).sum())
    b1 = np.broadcast_to(np.asarray(betas, np.float64).reshape(-1), (R,))
    table = []
    cands = [(ell, tile, mode, rw) for ell in ells for tile in tiles for mode in modes for rw in rows
             if rw or mode == "stream"]  # row windows only change stream mode
    for ell, tile, mode, rw in cands:
        work = occ0.clone()
        try:
            lat = Lattice(lattice, dims, K, S, work, ell=ell, tile=tile, rows=rw)
        except SmcxError as e:
            table.append({"tile": list(tile), "mode": mode, "ell": ell, "rows": rw, "error": str(e)})
            continue
        lat.set_epi(V)
        bt = np.tile(b1, (sweeps, 1))
        lat.sweep(1, seed, b1.reshape(1, R), first_sweep=0, mode=mode)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lat.sweep(sweeps, seed, bt, first_sweep=1, mode=mode)
        e1.record()
        torch.cuda.synchronize()
        secs = e0.elapsed_time(e1) / 1e3
        table.append({"tile": list(tile), "mode": mode, "ell": ell, "rows": rw,
                      "swaps_per_s": sweeps * N / secs})
        lat.close()
        del work
    ok = [t for t in table if "swaps_per_s" in t]
    if not ok:
        raise SmcxError("no candidate configuration could be built")
    best = dict(max(ok, key=lambda t: t["swaps_per_s"]))
    best["table"] = table
    if cache:
        db = {}
        if os.path.exists(cache):
            with open(cache) as f:
                db = json.load(f)
        db[key] = best
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return best


def fit_epi(lattice: int, dims, K: int, S: int, occ_batch, e_per_site, steps: int = 1500,
            lr: float = 1e-2, gamma: float = 0.99):
    """Fit an EPI to per-site energies of B configurations by Adam, the
    gradient flowing back through `EnergyFn` (Methods, "The EPI and qSRO
    model": the EPI is trained with Adam and back-propagation).

    At fixed composition E = const + sum_s sum_{k<l} C_s[k][l] W_s[k][l] with
    the gauge-invariant W_s[k][l] = V_s[k][l] - (V_s[k][k] + V_s[l][l]) / 2, so
    only W is identifiable: V is returned in the gauge V_s[k][k] = 0 and the
    loss compares energies after removing their means.  W is parametrised
    through the inverse Cholesky factor of the centred feature covariance
    (features C_s[k][l] / N, k < l), which makes the quadratic loss well
    conditioned.

    occ_batch: uint8 CUDA tensor [B][N]; e_per_site: [B] float64 (host or
    CUDA).  Returns (V [S][K][K] float64 CUDA tensor, final relative loss).
    """
    torch = _torch()
    occ_batch = occ_batch.contiguous()
    B, N = occ_batch.shape
    y = torch.as_tensor(np.asarray(e_per_site, np.float64) if not isinstance(e_per_site, torch.Tensor)
                        else e_per_site, dtype=torch.float64).cuda().reshape(-1)
    ku, lu = np.triu_indices(K, 1)
    ku_t, lu_t = torch.tensor(ku).cuda(), torch.tensor(lu).cuda()
    # the counts do not depend on V: one batched count serves every Adam step
    counts_i = energy_backward_counts(lattice, dims, K, S, occ_batch)
    counts = counts_i.to(torch.float64)
    F = counts[:, :, ku_t, lu_t].reshape(B, -1) / N
    Fc = F - F.mean(dim=0)
    L = torch.linalg.cholesky(Fc.T @ Fc / B)
    A = torch.linalg.inv(L).T
    theta = torch.zeros(A.shape[1], dtype=torch.float64, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([theta], lr=lr)
    sched = torch.optim.lr_scheduler.ExponentialLR(opt, gamma=gamma)
    fn = EnergyFn()
    sidx = torch.arange(S, device="cuda")[:, None].expand(S, len(ku))

    def v_of(th):
        W = (A @ th).reshape(S, -1)
        V = torch.zeros((S, K, K), dtype=torch.float64, device="cuda")
        V = V.index_put((sidx, ku_t.expand(S, -1), lu_t.expand(S, -1)), W)
        return V.index_put((sidx, lu_t.expand(S, -1), ku_t.expand(S, -1)), W)

    yc = y - y.mean()
    scale = (yc * yc).mean()
    loss = None
    for _ in range(steps):
        opt.zero_grad()
        e = fn.apply(v_of(theta), occ_batch, lattice, dims, counts_i) / N
        r = (e - e.mean()) - yc
        loss = (r * r).mean() / scale
        loss.backward()
        opt.step()
        sched.step()
    return v_of(theta.detach()), float(loss.item())
