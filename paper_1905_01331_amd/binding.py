"""ctypes binding of libttn.so (include/ttn.h): the same entry points, argument
marshalling only.  PyTorch provides the device workspace and the stream.

The library is loaded from this package directory; if it is missing the
import of any entry point raises (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttn.so")

TTN_OK, TTN_WRANK, TTN_WNOCONV, TTN_WPROF = 0, 1, 2, 3
TTN_EINVAL, TTN_ENOMEM, TTN_EHIP, TTN_ENONFINITE, TTN_ENOCONV, TTN_EORTHO, TTN_ESTATE = -1, -2, -3, -4, -5, -6, -7
TTN_FP64, TTN_FP32, TTN_SPLIT_BF16 = 0, 1, 2
TTN_DESCEND_RHO, TTN_DESCEND_DRESSED = 0, 1
TTN_ENT_AVERAGE, TTN_ENT_LEFTMOST = 0, 1
TTN_TOP = -1
TTN_OP_H, TTN_OP_A, TTN_OP_B, TTN_OP_RHO, TTN_OP_RBAR, TTN_OP_LBAR, TTN_OP_ENV = range(7)
PRECISIONS = {"fp64": TTN_FP64, "fp32": TTN_FP32, "bf16x3": TTN_SPLIT_BF16}

# Every symbol declared in include/ttn.h.
EXPORTS = [
    "ttn_workspace_bytes", "ttn_init", "ttn_ascend", "ttn_descend", "ttn_env", "ttn_update",
    "ttn_energy", "ttn_sweep", "ttn_sweep_grouped", "ttn_get_tensor", "ttn_set_tensor", "ttn_get_operator", "ttn_autotune",
    "ttn_stats", "ttn_entanglement", "ttn_bond_dim", "ttn_last_error", "ttn_free", "ttn_profile", "ttn_profile_read",
    "ttn_positions_bytes", "ttn_positions_offset", "ttn_local_energies", "ttn_entanglement_node",
    "ttn_autotune_save", "ttn_autotune_load", "ttn_local_energies_noalloc",
    "ttn_pos_workspace_bytes", "ttn_pos_init", "ttn_pos_sweep", "ttn_pos_energy", "ttn_pos_descend", "ttn_pos_env",
    "ttn_pos_get", "ttn_pos_set", "ttn_pos_free", "ttn_pos_stats", "ttn_pos_profile", "ttn_pos_profile_read",
    "ttn_cplx_workspace_bytes", "ttn_cplx_init", "ttn_cplx_sweep", "ttn_cplx_energy", "ttn_cplx_descend",
    "ttn_cplx_env", "ttn_cplx_get", "ttn_cplx_set", "ttn_cplx_stats", "ttn_cplx_profile", "ttn_cplx_profile_read",
    "ttn_cplx_free",
]
TTN_POS_W, TTN_POS_OPS, TTN_POS_DX, TTN_POS_TOP = range(4)
TTN_CPLX_W, TTN_CPLX_OPS, TTN_CPLX_RHO, TTN_CPLX_RBAR, TTN_CPLX_LBAR, TTN_CPLX_TOP = range(6)


class TTNConfig(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int), ("d", ctypes.c_int), ("chi", ctypes.c_int), ("D", ctypes.c_int),
        ("h1", ctypes.POINTER(ctypes.c_double)), ("A", ctypes.POINTER(ctypes.c_double)),
        ("B", ctypes.POINTER(ctypes.c_double)), ("shift", ctypes.c_double), ("ly", ctypes.c_int),
        ("precision", ctypes.c_int), ("seed", ctypes.c_ulonglong),
        ("w0", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
        ("v0", ctypes.POINTER(ctypes.c_double)), ("krylov", ctypes.c_int), ("restarts", ctypes.c_int),
        ("lanczos_tol", ctypes.c_double), ("keep_gauge", ctypes.c_int), ("evd_update", ctypes.c_int),
    ]


class TTNPosConfig(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int), ("d", ctypes.c_int), ("chi", ctypes.c_int), ("D", ctypes.c_int),
        ("h1", ctypes.POINTER(ctypes.c_double)), ("A", ctypes.POINTER(ctypes.c_double)),
        ("B", ctypes.POINTER(ctypes.c_double)), ("shift", ctypes.c_double), ("ly", ctypes.c_int),
        ("seed", ctypes.c_ulonglong), ("w0", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
        ("v0", ctypes.POINTER(ctypes.c_double)), ("krylov", ctypes.c_int), ("restarts", ctypes.c_int),
        ("lanczos_tol", ctypes.c_double), ("chunk_nodes", ctypes.c_int),
    ]


class TTNStats(ctypes.Structure):
    _fields_ = [
        ("energy", ctypes.c_double), ("lam", ctypes.c_double), ("lanczos_resid", ctypes.c_double),
        ("ortho_err_max", ctypes.c_double), ("sigma_ratio_min", ctypes.c_double), ("shift", ctypes.c_double),
        ("flops_bulk", ctypes.c_double), ("flops_fp64", ctypes.c_double), ("n_levels", ctypes.c_int),
        ("lanczos_iters", ctypes.c_int), ("jacobi_sweeps", ctypes.c_int * 4),
        ("e_prev", ctypes.c_double), ("bytes_hbm", ctypes.c_double),
    ]


class TTNPosStats(ctypes.Structure):
    _fields_ = [
        ("energy", ctypes.c_double), ("lam", ctypes.c_double), ("flops_sweep", ctypes.c_double),
        ("bytes_sweep", ctypes.c_double), ("lanczos_resid", ctypes.c_double), ("n_levels", ctypes.c_int),
        ("top_converged", ctypes.c_int),
    ]


class TTNCplxConfig(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int), ("d", ctypes.c_int), ("chi", ctypes.c_int), ("D", ctypes.c_int),
        ("h1", ctypes.POINTER(ctypes.c_double)), ("A", ctypes.POINTER(ctypes.c_double)),
        ("B", ctypes.POINTER(ctypes.c_double)), ("shift", ctypes.c_double), ("ly", ctypes.c_int),
        ("seed", ctypes.c_ulonglong), ("w0", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
        ("v0", ctypes.POINTER(ctypes.c_double)), ("krylov", ctypes.c_int), ("restarts", ctypes.c_int),
        ("lanczos_tol", ctypes.c_double),
    ]


class TTNCplxStats(ctypes.Structure):
    _fields_ = [
        ("energy", ctypes.c_double), ("lam", ctypes.c_double), ("flops_sweep", ctypes.c_double),
        ("bytes_sweep", ctypes.c_double), ("lanczos_resid", ctypes.c_double), ("ortho_err_max", ctypes.c_double),
        ("sigma_ratio_min", ctypes.c_double), ("n_levels", ctypes.c_int), ("top_converged", ctypes.c_int),
        ("repairs", ctypes.c_longlong),
    ]


class TTNProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libttn.so and declares the argument types of every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1905_01331_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ttn_workspace_bytes": ([ctypes.POINTER(TTNConfig), I, ctypes.POINTER(ctypes.c_size_t)], I),
        "ttn_init": ([ctypes.POINTER(TTNConfig), I, P, ctypes.c_size_t, P, ctypes.POINTER(P)], I),
        "ttn_ascend": ([P, I, I], I),
        "ttn_descend": ([P, I, I], I),
        "ttn_env": ([P, I], I),
        "ttn_update": ([P, I], I),
        "ttn_energy": ([P, DP], I),
        "ttn_sweep": ([P, I, I], I),
        "ttn_sweep_grouped": ([P, I, I, I], I),
        "ttn_autotune": ([I, ctypes.POINTER(ctypes.c_int)], I),
        "ttn_autotune_save": ([ctypes.c_char_p], I),
        "ttn_autotune_load": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)], I),
        "ttn_get_tensor": ([P, I, I, DP], I),
        "ttn_set_tensor": ([P, I, I, DP], I),
        "ttn_get_operator": ([P, I, I, I, I, DP], I),
        "ttn_stats": ([P, I, ctypes.POINTER(TTNStats)], I),
        "ttn_bond_dim": ([P, I, I], I),
        "ttn_last_error": ([], ctypes.c_char_p),
        "ttn_free": ([P], I),
        "ttn_profile": ([P, I], I),
        "ttn_entanglement": ([P, I, I, I, DP, DP], I),
        "ttn_entanglement_node": ([P, I, I, ctypes.c_longlong, DP, DP], I),
        "ttn_positions_bytes": ([P, I, ctypes.POINTER(ctypes.c_size_t)], I),
        "ttn_positions_offset": ([P, I, I, ctypes.POINTER(ctypes.c_size_t)], I),
        "ttn_local_energies": ([P, I, P, ctypes.c_size_t, DP, DP], I),
        "ttn_local_energies_noalloc": ([P, I, DP, DP], I),
        "ttn_profile_read": ([P, ctypes.POINTER(TTNProfileEntry), I, ctypes.POINTER(I)], I),
        "ttn_pos_workspace_bytes": ([ctypes.POINTER(TTNPosConfig), ctypes.POINTER(ctypes.c_size_t)], I),
        "ttn_pos_init": ([ctypes.POINTER(TTNPosConfig), P, ctypes.c_size_t, P, ctypes.POINTER(P)], I),
        "ttn_pos_sweep": ([P, I], I),
        "ttn_pos_energy": ([P, DP], I),
        "ttn_pos_descend": ([P], I),
        "ttn_pos_env": ([P, I, I, DP], I),
        "ttn_pos_get": ([P, I, I, DP], I),
        "ttn_pos_set": ([P, I, I, DP], I),
        "ttn_pos_free": ([P], I),
        "ttn_pos_stats": ([P, ctypes.POINTER(TTNPosStats)], I),
        "ttn_pos_profile": ([P, I], I),
        "ttn_pos_profile_read": ([P, ctypes.POINTER(TTNProfileEntry), I, ctypes.POINTER(I)], I),
        "ttn_cplx_workspace_bytes": ([ctypes.POINTER(TTNCplxConfig), ctypes.POINTER(ctypes.c_size_t)], I),
        "ttn_cplx_init": ([ctypes.POINTER(TTNCplxConfig), P, ctypes.c_size_t, P, ctypes.POINTER(P)], I),
        "ttn_cplx_sweep": ([P, I], I),
        "ttn_cplx_energy": ([P, DP], I),
        "ttn_cplx_descend": ([P], I),
        "ttn_cplx_env": ([P, I, DP], I),
        "ttn_cplx_get": ([P, I, I, DP], I),
        "ttn_cplx_set": ([P, I, I, DP], I),
        "ttn_cplx_stats": ([P, ctypes.POINTER(TTNCplxStats)], I),
        "ttn_cplx_profile": ([P, I], I),
        "ttn_cplx_profile_read": ([P, ctypes.POINTER(TTNProfileEntry), I, ctypes.POINTER(I)], I),
        "ttn_cplx_free": ([P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class TTNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _check(status, allow_warn=True):
    if status < 0 or (status > 0 and not allow_warn):
        raise TTNError(status, load_library().ttn_last_error().decode())
    return status


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class ChainInput:
    """Host-side arrays of one batch member, kept alive for the ctypes config."""

    def __init__(self, model, L, chi, precision="fp64", seed=0, w0=None, v0=None, shift=None,
                 krylov=0, restarts=0, lanczos_tol=0.0, keep_gauge=False, evd_update=False):
        h1, A, B = model.packed()
        self.h1 = np.ascontiguousarray(h1, dtype=np.float64)
        self.A = np.ascontiguousarray(A, dtype=np.float64)
        self.B = np.ascontiguousarray(B, dtype=np.float64)
        self.w0 = None if w0 is None else [np.ascontiguousarray(w, dtype=np.float64) for w in w0]
        self.v0 = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
        self._wptrs = None
        cfg = TTNConfig()
        cfg.L, cfg.d, cfg.chi, cfg.D = int(L), int(model.d), int(chi), int(model.D)
        cfg.h1 = _dptr(self.h1)
        cfg.A = _dptr(self.A) if model.D else None
        cfg.B = _dptr(self.B) if model.D else None
        cfg.shift = math.nan if shift is None else float(shift)
        cfg.ly = int(model.ly)
        cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        cfg.seed = int(seed)
        if self.w0 is not None:
            arr = (ctypes.POINTER(ctypes.c_double) * len(self.w0))(*[_dptr(w) for w in self.w0])
            self._wptrs = arr
            cfg.w0 = ctypes.cast(arr, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))
        else:
            cfg.w0 = None
        cfg.v0 = _dptr(self.v0) if self.v0 is not None else None
        cfg.krylov, cfg.restarts, cfg.lanczos_tol = int(krylov), int(restarts), float(lanczos_tol)
        cfg.keep_gauge = 1 if keep_gauge else 0
        cfg.evd_update = 1 if evd_update else 0
        self.cfg = cfg


def autotune(mode=-1):
    """Sets the process-wide autotuning mode (0 off, 1 tune new shapes, 2 use
    kept choices; -1 unchanged) and returns the number of kept choices."""
    lib = load_library()
    n = ctypes.c_int(0)
    _check(lib.ttn_autotune(int(mode), ctypes.byref(n)))
    return n.value


def autotune_save(path):
    """Writes the kept launch choices to a text file."""
    _check(load_library().ttn_autotune_save(str(path).encode()))


def autotune_load(path):
    """Merges the launch choices of a text file into the table; returns how
    many it held."""
    n = ctypes.c_int(0)
    _check(load_library().ttn_autotune_load(str(path).encode(), ctypes.byref(n)))
    return n.value


def ttn_workspace_bytes(inputs):
    lib = load_library()
    arr = (TTNConfig * len(inputs))(*[x.cfg for x in inputs])
    out = ctypes.c_size_t(0)
    _check(lib.ttn_workspace_bytes(arr, len(inputs), ctypes.byref(out)))
    return out.value


class TTN:
    """One handle over a batch of chains; the workspace is a torch uint8 tensor."""

    def __init__(self, inputs, device="cuda", stream=None):
        import torch
        lib = load_library()
        if not isinstance(inputs, (list, tuple)):
            inputs = [inputs]
        self.inputs = list(inputs)
        self.batch = len(self.inputs)
        nbytes = ttn_workspace_bytes(self.inputs)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(device=self.workspace.device)
        arr = (TTNConfig * self.batch)(*[x.cfg for x in self.inputs])
        h = ctypes.c_void_p(0)
        self.init_status = _check(lib.ttn_init(arr, self.batch, ctypes.c_void_p(aligned), nbytes,
                                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.lib = lib

    # stage calls -------------------------------------------------------------
    def ascend(self, tau_from, tau_to):
        return _check(self.lib.ttn_ascend(self.h, tau_from, tau_to))

    def descend(self, what, tau=0):
        return _check(self.lib.ttn_descend(self.h, tau, what))

    def env(self, tau):
        return _check(self.lib.ttn_env(self.h, tau))

    def update(self, tau):
        return _check(self.lib.ttn_update(self.h, tau))

    def energy(self):
        """Energies per site; the call's status (0 or a warning such as
        TTN_WNOCONV) is kept in self.energy_status."""
        out = np.zeros(self.batch)
        self.energy_status = _check(self.lib.ttn_energy(self.h, _dptr(out)))
        return out

    def sweep(self, nsweeps=1, graph=False):
        """graph: False eager, True (or 1) graph replay with one host read per
        sweep for the top solver's restarts, 2 graph replay with the whole
        restart budget in the graph and no host read."""
        return _check(self.lib.ttn_sweep(self.h, nsweeps, int(graph)))

    def sweep_grouped(self, nsweeps=1, groups=2, graph=False):
        return _check(self.lib.ttn_sweep_grouped(self.h, nsweeps, groups, int(graph)))

    # access -----------------------------------------------------------------
    def bond_dim(self, tau, b=0):
        return self.lib.ttn_bond_dim(self.h, b, tau)

    def n_levels(self, b=0):
        return self.stats(b).n_levels

    def get_tensor(self, tau, b=0):
        n = self.n_levels(b)
        if tau == TTN_TOP:
            x = self.bond_dim(n - 1, b)
            out = np.zeros((x, x))
        else:
            a, bb = self.bond_dim(tau, b), self.bond_dim(tau - 1, b)
            out = np.zeros((a, bb, bb))
        _check(self.lib.ttn_get_tensor(self.h, b, tau, _dptr(out)))
        return out

    def set_tensor(self, tau, arr, b=0):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        _check(self.lib.ttn_set_tensor(self.h, b, tau, _dptr(arr)))

    def get_operator(self, level, kind, k=0, b=0):
        x = self.bond_dim(level, b)
        if kind == TTN_OP_ENV:
            y = self.bond_dim(level - 1, b)
            out = np.zeros((x, y, y))
        else:
            out = np.zeros((x, x))
        _check(self.lib.ttn_get_operator(self.h, b, level, kind, k, _dptr(out)))
        return out

    def stats(self, b=0):
        st = TTNStats()
        _check(self.lib.ttn_stats(self.h, b, ctypes.byref(st)))
        return st

    def profile(self, enable=True):
        return _check(self.lib.ttn_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        arr = (TTNProfileEntry * 64)()
        n = ctypes.c_int(0)
        # an incomplete record (launches not timed) is an error here
        _check(self.lib.ttn_profile_read(self.h, arr, 64, ctypes.byref(n)), allow_warn=False)
        return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops,
                                           bytes=arr[i].bytes) for i in range(n.value)}

    def entanglement(self, tau, which=TTN_ENT_AVERAGE, b=0):
        """(p, S): the spectrum (descending) of the reduced density matrix on
        an upper bond index of layer tau, and the entropy in bits."""
        p = np.zeros(max(self.bond_dim(tau, b), 1))  # the library rejects a bad tau
        S = ctypes.c_double(0.0)
        _check(self.lib.ttn_entanglement(self.h, b, tau, which, _dptr(p), ctypes.byref(S)))
        return p, S.value

    def entanglement_node(self, tau, node, b=0):
        """(p, S) for the block of node `node` of level tau (sites
        node 2**tau .. (node + 1) 2**tau - 1)."""
        p = np.zeros(max(self.bond_dim(tau, b), 1))
        S = ctypes.c_double(0.0)
        _check(self.lib.ttn_entanglement_node(self.h, b, tau, node, _dptr(p), ctypes.byref(S)))
        return p, S.value

    def positions_bytes(self, b=0):
        need = ctypes.c_size_t(0)
        _check(self.lib.ttn_positions_bytes(self.h, b, ctypes.byref(need)))
        return need.value

    def local_energies(self, b=0, levels=(), work=None):
        """(site, bond, rhos): the expectation of every one-site term and of
        every bond (j, j+1) of member b, and the reduced density matrices of
        the nodes of the requested levels ({tau: array (L >> tau, chi, chi)}).
        work: a CUDA uint8 tensor to compute in (at least positions_bytes()
        + 256 bytes); by default one of that size is taken for the call."""
        import torch
        need = self.positions_bytes(b)
        if work is None:
            work = torch.empty(need + 256, dtype=torch.uint8, device=self.workspace.device)
        base = work.data_ptr()
        skip = ((base + 255) & ~255) - base
        nbytes = work.numel() - skip
        n = self.n_levels(b)
        L = 1 << n
        site, bond = np.zeros(L), np.zeros(L)
        _check(self.lib.ttn_local_energies(self.h, b, ctypes.c_void_p(base + skip), nbytes, _dptr(site), _dptr(bond)))
        rhos = {}
        for tau in levels:
            off = ctypes.c_size_t(0)
            _check(self.lib.ttn_positions_offset(self.h, b, tau, ctypes.byref(off)))
            c = self.bond_dim(tau, b)
            cnt = (L >> tau) * c * c
            raw = work[skip + off.value: skip + off.value + 8 * cnt].cpu().numpy()
            rhos[tau] = raw.view(np.float64).reshape(L >> tau, c, c).copy()
        return site, bond, rhos

    def local_energies_noalloc(self, b=0):
        """(site, bond) of member b from ttn_local_energies_noalloc: the
        library's static device scratch instead of a caller's work buffer."""
        n = self.n_levels(b)
        L = 1 << n
        site, bond = np.zeros(L), np.zeros(L)
        _check(self.lib.ttn_local_energies_noalloc(self.h, b, _dptr(site), _dptr(bond)))
        return site, bond

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.ttn_free(self.h)
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bond_dims(L, d, chi):
    """chi_tau = min(chi_{tau-1}^2, chi), chi_0 = d, for tau < n (L = 2^n)."""
    n = int(L).bit_length() - 1
    dims = [int(d)]
    for _ in range(1, n):
        dims.append(min(dims[-1] * dims[-1], int(chi)))
    return dims


class PosTTN:
    """Handle of a position-resolved network (include/ttn.h, ttn_pos_*).
    w0: one array per layer tau = 1..n-1 of shape (L >> tau, chi_tau,
    chi_{tau-1}, chi_{tau-1}); v0 optional."""

    def __init__(self, model, L, chi, w0, v0=None, shift=None, seed=0, krylov=0, restarts=0, lanczos_tol=0.0,
                 chunk_nodes=0, device="cuda", stream=None):
        import torch
        lib = load_library()
        h1, A, B = model.packed()
        self.h1 = np.ascontiguousarray(h1, dtype=np.float64)
        self.A = np.ascontiguousarray(A, dtype=np.float64)
        self.B = np.ascontiguousarray(B, dtype=np.float64)
        self.L, self.chi, self.d, self.D = int(L), int(chi), int(model.d), int(model.D)
        self.dims = bond_dims(L, model.d, chi)
        self.n = len(self.dims)
        self.w0 = [np.ascontiguousarray(w, dtype=np.float64) for w in w0]
        self.v0 = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
        cfg = TTNPosConfig()
        cfg.L, cfg.d, cfg.chi, cfg.D = self.L, self.d, self.chi, self.D
        cfg.h1 = _dptr(self.h1)
        cfg.A = _dptr(self.A) if self.D else None
        cfg.B = _dptr(self.B) if self.D else None
        cfg.shift = math.nan if shift is None else float(shift)
        cfg.ly = int(model.ly)
        cfg.seed = int(seed)
        self._wptrs = (ctypes.POINTER(ctypes.c_double) * max(1, len(self.w0)))(*[_dptr(w) for w in self.w0])
        cfg.w0 = ctypes.cast(self._wptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))
        cfg.v0 = _dptr(self.v0) if self.v0 is not None else None
        cfg.krylov, cfg.restarts, cfg.lanczos_tol = int(krylov), int(restarts), float(lanczos_tol)
        cfg.chunk_nodes = int(chunk_nodes)
        self.cfg = cfg
        need = ctypes.c_size_t(0)
        _check(lib.ttn_pos_workspace_bytes(ctypes.byref(cfg), ctypes.byref(need)))
        self.workspace = torch.empty(need.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(device=self.workspace.device)
        h = ctypes.c_void_p(0)
        self.init_status = _check(lib.ttn_pos_init(ctypes.byref(cfg), ctypes.c_void_p(aligned), need.value,
                                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.lib = lib

    def sweep(self, nsweeps=1):
        return _check(self.lib.ttn_pos_sweep(self.h, int(nsweeps)))

    def energy(self):
        """(lambda, energy per spin); the call's status in self.energy_status."""
        out = np.zeros(2)
        self.energy_status = _check(self.lib.ttn_pos_energy(self.h, _dptr(out)))
        return float(out[0]), float(out[1])

    def descend(self):
        return _check(self.lib.ttn_pos_descend(self.h))

    def env(self, tau, parity):
        a, b = self.dims[tau], self.dims[tau - 1]
        out = np.zeros(((self.L >> tau) // 2, a, b, b))
        _check(self.lib.ttn_pos_env(self.h, int(tau), int(parity), _dptr(out)))
        return out

    def isometries(self, tau):
        a, b = self.dims[tau], self.dims[tau - 1]
        out = np.zeros((self.L >> tau, a, b, b))
        _check(self.lib.ttn_pos_get(self.h, TTN_POS_W, int(tau), _dptr(out)))
        return out

    def operators(self, level):
        """(h, A, B): per node (node-major) h (x, x), A and B (D, x, x); level 0
        one node."""
        x = self.dims[level]
        nodes = 1 if level == 0 else self.L >> level
        out = np.zeros((nodes, 1 + 2 * self.D, x, x))
        _check(self.lib.ttn_pos_get(self.h, TTN_POS_OPS, int(level), _dptr(out)))
        return out[:, 0], out[:, 1:1 + self.D], out[:, 1 + self.D:]

    def node_matrices(self, level):
        """(rho, X, Y) of every node of a level as of the last descend()."""
        x = self.dims[level]
        out = np.zeros((self.L >> level, 1 + 2 * self.D, x, x))
        _check(self.lib.ttn_pos_get(self.h, TTN_POS_DX, int(level), _dptr(out)))
        return out[:, 0], out[:, 1:1 + self.D], out[:, 1 + self.D:]

    def top(self):
        x = self.dims[-1]
        out = np.zeros((x, x))
        _check(self.lib.ttn_pos_get(self.h, TTN_POS_TOP, 0, _dptr(out)))
        return out

    def set_top(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        _check(self.lib.ttn_pos_set(self.h, TTN_POS_TOP, 0, _dptr(v)))

    def set_isometries(self, tau, ws):
        """Layer tau's isometries (L >> tau, chi_tau, chi_{tau-1}, chi_{tau-1});
        the levels from tau up are ascended again."""
        ws = np.ascontiguousarray(ws, dtype=np.float64)
        a, b = self.dims[tau], self.dims[tau - 1]
        if ws.shape != (self.L >> tau, a, b, b):
            raise ValueError(f"layer {tau}: shape {ws.shape}")
        _check(self.lib.ttn_pos_set(self.h, TTN_POS_W, int(tau), _dptr(ws)))

    def stats(self):
        st = TTNPosStats()
        _check(self.lib.ttn_pos_stats(self.h, ctypes.byref(st)))
        return st

    def profile(self, enable=True):
        return _check(self.lib.ttn_pos_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        arr = (TTNProfileEntry * 64)()
        n = ctypes.c_int(0)
        _check(self.lib.ttn_pos_profile_read(self.h, arr, 64, ctypes.byref(n)), allow_warn=False)
        return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops,
                                           bytes=arr[i].bytes) for i in range(n.value)}

    def close(self):
        if getattr(self, "h", None):
            self.lib.ttn_pos_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cptr(a: np.ndarray):
    """Pointer to a contiguous complex128 array as interleaved doubles."""
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class CplxTTN:
    """Handle of a uniform network with complex tensors (include/ttn.h,
    ttn_cplx_*).  model: a ChainModel (complex or real matrices, passed as
    complex128); w0: one complex array per layer tau = 1..n-1 of shape
    (chi_tau, chi_{tau-1}, chi_{tau-1}); v0 optional."""

    def __init__(self, model, L, chi, w0, v0=None, shift=None, seed=0, krylov=0, restarts=0, lanczos_tol=0.0,
                 device="cuda", stream=None):
        import torch
        lib = load_library()
        h1, A, B = model.packed()
        self.h1 = np.ascontiguousarray(h1, dtype=np.complex128)
        self.A = np.ascontiguousarray(A, dtype=np.complex128)
        self.B = np.ascontiguousarray(B, dtype=np.complex128)
        self.L, self.chi, self.d, self.D = int(L), int(chi), int(model.d), int(model.D)
        self.dims = bond_dims(L, model.d, chi)
        self.n = len(self.dims)
        self.w0 = [np.ascontiguousarray(w, dtype=np.complex128) for w in w0]
        self.v0 = None if v0 is None else np.ascontiguousarray(v0, dtype=np.complex128)
        cfg = TTNCplxConfig()
        cfg.L, cfg.d, cfg.chi, cfg.D = self.L, self.d, self.chi, self.D
        cfg.h1 = _cptr(self.h1)
        cfg.A = _cptr(self.A) if self.D else None
        cfg.B = _cptr(self.B) if self.D else None
        cfg.shift = math.nan if shift is None else float(shift)
        cfg.ly = int(model.ly)
        cfg.seed = int(seed)
        self._wptrs = (ctypes.POINTER(ctypes.c_double) * max(1, len(self.w0)))(*[_cptr(w) for w in self.w0])
        cfg.w0 = ctypes.cast(self._wptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))
        cfg.v0 = _cptr(self.v0) if self.v0 is not None else None
        cfg.krylov, cfg.restarts, cfg.lanczos_tol = int(krylov), int(restarts), float(lanczos_tol)
        self.cfg = cfg
        need = ctypes.c_size_t(0)
        _check(lib.ttn_cplx_workspace_bytes(ctypes.byref(cfg), ctypes.byref(need)))
        self.workspace = torch.empty(need.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(device=self.workspace.device)
        h = ctypes.c_void_p(0)
        self.init_status = _check(lib.ttn_cplx_init(ctypes.byref(cfg), ctypes.c_void_p(aligned), need.value,
                                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.lib = lib

    def sweep(self, nsweeps=1):
        return _check(self.lib.ttn_cplx_sweep(self.h, int(nsweeps)))

    def energy(self):
        """(lambda, energy per spin); the call's status in self.energy_status."""
        out = np.zeros(2)
        self.energy_status = _check(self.lib.ttn_cplx_energy(self.h, _dptr(out)))
        return float(out[0]), float(out[1])

    def descend(self):
        return _check(self.lib.ttn_cplx_descend(self.h))

    def env(self, tau):
        a, b = self.dims[tau], self.dims[tau - 1]
        out = np.zeros((a, b, b), dtype=np.complex128)
        _check(self.lib.ttn_cplx_env(self.h, int(tau), _cptr(out)))
        return out

    def _get(self, what, level, shape):
        out = np.zeros(shape, dtype=np.complex128)
        _check(self.lib.ttn_cplx_get(self.h, what, int(level), _cptr(out)))
        return out

    def isometry(self, tau):
        a, b = self.dims[tau], self.dims[tau - 1]
        return self._get(TTN_CPLX_W, tau, (a, b, b))

    def operators(self, level):
        """(h, A, B) of a level: h (x, x), A and B (D, x, x)."""
        x = self.dims[level]
        out = self._get(TTN_CPLX_OPS, level, (1 + 2 * self.D, x, x))
        return out[0], out[1:1 + self.D], out[1 + self.D:]

    def rho(self, level):
        x = self.dims[level]
        return self._get(TTN_CPLX_RHO, level, (x, x))

    def dressed(self, tau):
        """(Rbar, Lbar) of the last env() call's level tau, (D, x, x) each."""
        x = self.dims[tau]
        return (self._get(TTN_CPLX_RBAR, 0, (self.D, x, x)), self._get(TTN_CPLX_LBAR, 0, (self.D, x, x)))

    def top(self):
        x = self.dims[-1]
        return self._get(TTN_CPLX_TOP, 0, (x, x))

    def set_top(self, v):
        v = np.ascontiguousarray(v, dtype=np.complex128)
        _check(self.lib.ttn_cplx_set(self.h, TTN_CPLX_TOP, 0, _cptr(v)))

    def set_isometry(self, tau, w):
        w = np.ascontiguousarray(w, dtype=np.complex128)
        a, b = self.dims[tau], self.dims[tau - 1]
        if w.shape != (a, b, b):
            raise ValueError(f"layer {tau}: shape {w.shape}")
        _check(self.lib.ttn_cplx_set(self.h, TTN_CPLX_W, int(tau), _cptr(w)))

    def stats(self):
        st = TTNCplxStats()
        _check(self.lib.ttn_cplx_stats(self.h, ctypes.byref(st)))
        return st

    def profile(self, enable=True):
        return _check(self.lib.ttn_cplx_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        arr = (TTNProfileEntry * 64)()
        n = ctypes.c_int(0)
        _check(self.lib.ttn_cplx_profile_read(self.h, arr, 64, ctypes.byref(n)), allow_warn=False)
        return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops,
                                           bytes=arr[i].bytes) for i in range(n.value)}

    def close(self):
        if getattr(self, "h", None):
            self.lib.ttn_cplx_free(self.h)
            self.h = None
