"""The C-ABI library on the CPU: it loads, exports every symbol that
include/smcx.h declares, and its host-side argument checks work without a GPU
(no compute call is made here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smcx.h")


@pytest.fixture(scope="module")
def smcx():
    from paper_2503_12591_amd import smcx as S
    if not os.path.exists(S.LIB_PATH):
        from paper_2503_12591_amd import build
        build.build()
    S.lib()
    return S


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smcx_\w+)\s*\(", text)))


def test_header_declares_the_binding_exports(smcx):
    assert declared_functions() == sorted(smcx.EXPORTS)


def test_library_exports_every_declared_symbol(smcx):
    L = smcx.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_version(smcx):
    assert smcx.lib().smcx_version() == 100


def test_min_cell_edge_matches_oracle(smcx, oracle):
    for lat in (0, 1):
        for S in (1, 2, 3, 4):
            assert smcx.min_cell_edge(lat, S) == oracle.lmin(lat, S)
    assert smcx.lib().smcx_min_cell_edge(5, 2) == -1


def make_desc(smcx, lattice=0, K=4, S=4, dims=((8, 8, 8),), ell=None, cells=None, tile=(0, 0, 0)):
    keep = []
    d = smcx.Desc()
    d.lattice, d.n_species, d.n_shells = lattice, K, S
    dims = np.ascontiguousarray(np.asarray(dims, np.int32))
    keep.append(dims)
    d.n_replicas = dims.shape[0]
    d.dims = dims.ctypes.data_as(C.c_void_p)
    if ell is not None:
        e = np.ascontiguousarray(np.asarray(ell, np.int32))
        keep.append(e)
        d.ell = e.ctypes.data_as(C.c_void_p)
    if cells is not None:
        nc = np.ascontiguousarray(np.array([[len(c[a]) for a in range(3)] for c in cells], np.int32))
        flat = np.ascontiguousarray(np.concatenate([np.asarray(c[a], np.int32) for c in cells
                                                    for a in range(3)]))
        keep += [nc, flat]
        d.ncell = nc.ctypes.data_as(C.c_void_p)
        d.cells = flat.ctypes.data_as(C.c_void_p)
    for a in range(3):
        d.tile[a] = tile[a]
    return d, keep


def ws_size(smcx, d):
    n = C.c_size_t(0)
    rc = smcx.lib().smcx_workspace_size(C.byref(d), C.byref(n))
    return rc, n.value


def test_workspace_size_accounts_for_padded_copy(smcx):
    d, keep = make_desc(smcx, dims=((800, 800, 800),))
    rc, n = ws_size(smcx, d)
    assert rc == 0
    # rows of the padded copy: interleaved (16-byte aligned m * (L + 4)) or
    # basis-planar (m columns of 16-byte aligned L + 4); the region fits either
    prow = max((2 * 804 + 15) // 16 * 16, 2 * ((804 + 15) // 16 * 16))
    assert n >= prow * 804 * 804
    assert n < prow * 804 * 804 + (1 << 22)


@pytest.mark.parametrize("kw,code", [
    (dict(K=9), -1), (dict(K=1), -1), (dict(S=0), -1), (dict(S=5), -1), (dict(lattice=2), -1),
    (dict(dims=((1, 8, 8),)), -1),
    (dict(cells=[[[2, 6], [8], [8]]]), -1),           # edge 2 below the minimum 3
    (dict(cells=[[[4, 3], [8], [8]]]), -1),           # does not sum to 8
    (dict(tile=(16, 16, 2)), -1),                      # more than 256 link cells
    (dict(dims=((4096, 8, 8),), tile=(256, 1, 1), ell=[8]), -2),  # window rows wider than the block
])
def test_workspace_size_rejects_bad_descriptions(smcx, kw, code):
    d, keep = make_desc(smcx, **kw)
    rc, _ = ws_size(smcx, d)
    assert rc == code, smcx.lib().smcx_last_error()
    assert len(smcx.lib().smcx_last_error()) > 0


def test_single_cell_axes_allowed_below_minimum(smcx):
    d, keep = make_desc(smcx, dims=((2, 2, 2),), K=2, S=2)
    assert ws_size(smcx, d)[0] == 0


def test_init_rejects_null_pointers(smcx):
    d, keep = make_desc(smcx)
    h = C.c_void_p()
    rc = smcx.lib().smcx_lattice_init(C.byref(h), C.byref(d), None, None, 0, None)
    assert rc == -1 and h.value is None


def test_stateless_backward_rejects_bad_args(smcx):
    dims = np.array([1, 4, 4], np.int32)
    rc = smcx.lib().smcx_energy_backward(0, dims.ctypes.data_as(C.c_void_p), 4, 4, None, 3, None, None)
    assert rc == -1
    dims = np.array([4, 4, 4], np.int32)
    rc = smcx.lib().smcx_energy_backward(0, dims.ctypes.data_as(C.c_void_p), 9, 4, None, 3, None, None)
    assert rc == -1
    # B == 0 is a no-op that touches no memory
    rc = smcx.lib().smcx_energy_backward(0, dims.ctypes.data_as(C.c_void_p), 4, 4, None, 0, None, None)
    assert rc == 0


def test_energy_of_counts_and_grad_reject_bad_args(smcx):
    L = smcx.lib()
    assert L.smcx_energy_of_counts(None, None, -1, 64, None, None) == -1
    assert L.smcx_energy_of_counts(None, None, 3, 0, None, None) == -1
    assert L.smcx_energy_of_counts(None, None, 3, 64, None, None) == -1
    assert L.smcx_energy_of_counts(None, None, 0, 64, None, None) == 0  # empty batch: no-op
    assert L.smcx_energy_grad(None, None, 2, 64, None, None) == -1
    assert L.smcx_energy_grad(None, None, -1, 64, None, None) == -1


def test_null_handle_calls_fail_cleanly(smcx):
    L = smcx.lib()
    assert L.smcx_set_epi(None, None, None) == -1
    assert L.smcx_sweep(None, 1, 0, 0, None, None, None, 0, None, 0, None) == -1
    assert L.smcx_pair_counts(None, None, None) == -1
    assert L.smcx_graph_launch(None, None) == -1
    assert L.smcx_lattice_destroy(None) == 0


def test_python_binding_fails_loudly_without_gpu(smcx):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(smcx.SmcxError):
        smcx.Lattice(0, (8, 8, 8), 4, 2, np.zeros(1024, np.uint8))
