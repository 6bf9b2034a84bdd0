"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and the host-side validation rejects bad configurations
without touching a GPU (ttn_workspace_bytes runs on the host only)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1905_01331_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "ttn.h")).read()
    return sorted(set(re.findall(r"\b(ttn_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1905_01331_amd import build
        build.build()
    return binding.load_library()


def test_header_and_binding_agree():
    assert header_symbols() == sorted(binding.EXPORTS)


def test_library_exports_every_symbol(lib):
    for name in header_symbols():
        assert hasattr(lib, name), name


def _bytes(model, L, chi, **kw):
    return binding.ttn_workspace_bytes([binding.ChainInput(model, L, chi, **kw)])


def test_workspace_sizes(lib):
    small = _bytes(inputs.tfim_chain(1.0), 16, 8)
    big = _bytes(inputs.tfim_chain(1.0), 1024, 64)
    assert 0 < small < big
    # the chi = 256 chain of 4096 sites keeps its tensors well inside one GPU
    assert _bytes(inputs.xxx_chain(), 4096, 256, precision="bf16x3") < 16 * 2 ** 30


@pytest.mark.parametrize("L", [3, 6, 2, 0])
def test_rejects_bad_length(lib, L):
    with pytest.raises(binding.TTNError) as e:
        _bytes(inputs.tfim_chain(1.0), L, 8)
    assert e.value.status == binding.TTN_EINVAL


def test_rejects_nonfinite_and_asymmetric(lib):
    m = inputs.tfim_chain(1.0)
    m.h1 = m.h1.copy()
    m.h1[0, 0] = math.nan
    with pytest.raises(binding.TTNError) as e:
        _bytes(m, 16, 8)
    assert e.value.status == binding.TTN_ENONFINITE
    m = inputs.tfim_chain(1.0)
    m.h1 = np.array([[0.0, 1.0], [0.5, 0.0]])
    with pytest.raises(binding.TTNError) as e:
        _bytes(m, 16, 8)
    assert e.value.status == binding.TTN_EINVAL


def test_rejects_mixed_parity_pair(lib):
    m = inputs.ChainModel("bad", np.zeros((2, 2)), [inputs.PAULI_X], [inputs.PAULI_IY])
    with pytest.raises(binding.TTNError) as e:
        _bytes(m, 16, 8)
    assert e.value.status == binding.TTN_EINVAL


def test_rejects_bad_precision_and_chi(lib):
    with pytest.raises(binding.TTNError):
        _bytes(inputs.tfim_chain(1.0), 16, 8, precision=7)
    with pytest.raises(binding.TTNError):
        _bytes(inputs.tfim_chain(1.0), 16, 0)
    with pytest.raises(binding.TTNError):
        _bytes(inputs.tfim_chain(1.0), 16, 1025)


def test_rejects_empty_batch_and_bad_solver_settings(lib):
    out = ctypes.c_size_t(0)
    arr = (binding.TTNConfig * 1)(binding.ChainInput(inputs.tfim_chain(1.0), 16, 8).cfg)
    assert lib.ttn_workspace_bytes(arr, 0, ctypes.byref(out)) == binding.TTN_EINVAL
    with pytest.raises(binding.TTNError) as e:
        _bytes(inputs.tfim_chain(1.0), 16, 8, krylov=64)
    assert e.value.status == binding.TTN_EINVAL
    with pytest.raises(binding.TTNError) as e:
        _bytes(inputs.tfim_chain(1.0), 16, 8, shift=math.inf)
    assert e.value.status in (binding.TTN_EINVAL, binding.TTN_ENONFINITE)


def test_zero_hamiltonian_and_unit_bond_dimension_are_accepted(lib):
    zero = inputs.ChainModel("zero", np.zeros((2, 2)), [], [])
    assert _bytes(zero, 32, 3, shift=1.0) > 0
    assert _bytes(inputs.tfim_chain(1.3), 8, 1) > 0
    assert _bytes(inputs.tfim_chain(1.0), 4, 2) > 0


def test_grouped_sweep_rejects_a_null_handle(lib):
    # argument checks run before any device call
    assert lib.ttn_sweep_grouped(None, 1, 2, 0) == binding.TTN_EINVAL
    assert lib.ttn_sweep_grouped(None, 1, 3, 1) == binding.TTN_EINVAL


def test_position_resolved_calls_reject_bad_arguments(lib):
    # every check happens before any device call
    import ctypes
    n = ctypes.c_size_t(0)
    site = (ctypes.c_double * 4)()
    bond = (ctypes.c_double * 4)()
    assert lib.ttn_positions_bytes(None, 0, ctypes.byref(n)) == binding.TTN_EINVAL
    assert lib.ttn_positions_offset(None, 0, 0, ctypes.byref(n)) == binding.TTN_EINVAL
    assert lib.ttn_local_energies(None, 0, None, 0, site, bond) == binding.TTN_EINVAL
    S = ctypes.c_double(0.0)
    assert lib.ttn_entanglement_node(None, 0, 0, 0, site, ctypes.byref(S)) == binding.TTN_EINVAL
    assert b"bad arguments" in lib.ttn_last_error()


def _pos_cfg(model, L, chi, w0, chunk=0):
    h1, A, B = model.packed()
    keep = [np.ascontiguousarray(x, dtype=np.float64) for x in (h1, A, B)]
    cfg = binding.TTNPosConfig()
    cfg.L, cfg.d, cfg.chi, cfg.D = L, model.d, chi, model.D
    cfg.h1 = binding._dptr(keep[0])
    cfg.A = binding._dptr(keep[1]) if model.D else None
    cfg.B = binding._dptr(keep[2]) if model.D else None
    cfg.shift, cfg.ly, cfg.chunk_nodes = math.nan, model.ly, chunk
    if w0 is not None:
        ws = [np.ascontiguousarray(w) for w in w0]
        keep.append(ws)
        arr = (ctypes.POINTER(ctypes.c_double) * len(ws))(*[binding._dptr(w) for w in ws])
        keep.append(arr)
        cfg.w0 = ctypes.cast(arr, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))
    return cfg, keep


def test_node_resolved_workspace_and_validation(lib):
    # host-only: sizes grow with the node count, missing isometries and a
    # negative chunk are rejected, null handles too
    model = inputs.xxx_chain()
    out = ctypes.c_size_t(0)
    sizes = []
    for L in (16, 64):
        w0 = inputs.random_node_isometries(L, model.d, 8, 0)
        cfg, keep = _pos_cfg(model, L, 8, w0)
        assert lib.ttn_pos_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_OK
        sizes.append(out.value)
    assert 0 < sizes[0] < sizes[1]
    cfg, keep = _pos_cfg(model, 16, 8, None)
    assert lib.ttn_pos_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_EINVAL
    cfg, keep = _pos_cfg(model, 16, 8, inputs.random_node_isometries(16, 2, 8, 0), chunk=-1)
    assert lib.ttn_pos_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_EINVAL
    cfg, keep = _pos_cfg(model, 12, 8, inputs.random_node_isometries(16, 2, 8, 0))
    assert lib.ttn_pos_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_EINVAL
    e = (ctypes.c_double * 2)()
    assert lib.ttn_pos_sweep(None, 1) == binding.TTN_EINVAL
    assert lib.ttn_pos_energy(None, e) == binding.TTN_EINVAL
    assert lib.ttn_pos_env(None, 1, 0, e) == binding.TTN_EINVAL
    assert lib.ttn_pos_get(None, binding.TTN_POS_W, 1, e) == binding.TTN_EINVAL
    assert lib.ttn_pos_free(None) == binding.TTN_OK


def _cplx_cfg(model, L, chi, ws):
    keep = []
    cfg = binding.TTNCplxConfig()
    h1, A, B = model.packed()
    h1, A, B = (np.ascontiguousarray(x, dtype=np.complex128) for x in (h1, A, B))
    keep += [h1, A, B]
    cfg.L, cfg.d, cfg.chi, cfg.D = L, model.d, chi, model.D
    cfg.h1, cfg.A, cfg.B = binding._cptr(h1), binding._cptr(A), binding._cptr(B)
    cfg.shift = math.nan
    cfg.ly = 1
    if ws is not None:
        ws = [np.ascontiguousarray(w, dtype=np.complex128) for w in ws]
        keep += ws
        arr = (ctypes.POINTER(ctypes.c_double) * len(ws))(*[binding._cptr(w) for w in ws])
        keep.append(arr)
        cfg.w0 = ctypes.cast(arr, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))
    return cfg, keep


def test_complex_workspace_and_validation(lib):
    # host-only: the workspace grows with chi; a non-Hermitian h1, a bond term
    # that is not Hermitian, missing isometries and a bad length are
    # rejected; null handles too
    model = inputs.dm_chain(1.0, 0.5, 1.0, 0.2)
    out = ctypes.c_size_t(0)
    sizes = []
    for chi in (8, 32):
        ws = inputs.random_complex_isometries(inputs.layer_shapes(64, 2, chi), 0)
        cfg, keep = _cplx_cfg(model, 64, chi, ws)
        assert lib.ttn_cplx_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_OK
        sizes.append(out.value)
    assert 0 < sizes[0] < sizes[1]
    ws = inputs.random_complex_isometries(inputs.layer_shapes(16, 2, 8), 0)
    bad = inputs.ChainModel("bad", np.array([[0, 1j], [1j, 0]]), model.A, model.B, dtype=np.complex128)
    cfg, keep = _cplx_cfg(bad, 16, 8, ws)
    assert lib.ttn_cplx_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_EINVAL
    assert b"Hermitian" in lib.ttn_last_error()
    # i Sx x Sy alone is anti-Hermitian: the bond term is not Hermitian
    sx, sy = model.A[0], model.A[1]
    bad = inputs.ChainModel("bad", np.zeros((2, 2)), [1j * sx], [sy], dtype=np.complex128)
    cfg, keep = _cplx_cfg(bad, 16, 8, ws)
    assert lib.ttn_cplx_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_EINVAL
    cfg, keep = _cplx_cfg(model, 16, 8, None)
    assert lib.ttn_cplx_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_EINVAL
    cfg, keep = _cplx_cfg(model, 12, 8, ws)
    assert lib.ttn_cplx_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == binding.TTN_EINVAL
    e = (ctypes.c_double * 2)()
    assert lib.ttn_cplx_sweep(None, 1) == binding.TTN_EINVAL
    assert lib.ttn_cplx_energy(None, e) == binding.TTN_EINVAL
    assert lib.ttn_cplx_env(None, 1, e) == binding.TTN_EINVAL
    assert lib.ttn_cplx_get(None, binding.TTN_CPLX_W, 1, e) == binding.TTN_EINVAL
    assert lib.ttn_cplx_free(None) == binding.TTN_OK
