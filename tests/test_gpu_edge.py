"""Edge cases of the method on the GPU path (float64 unless stated).

* Full bond dimension: every isometry is square, the network spans the
  whole Hilbert space, and the energy right after initialisation (and after
  any sweep) is the exact ground energy (values from exact
  diagonalisation, tests/golden).
* The shortest chain (L = 4: one isometry layer and the top), bond
  dimension one (a product state), a bond dimension below the site
  dimension and deep trees (18 and 20 levels), against the reference, sweep
  by sweep from identical states.
* The zero Hamiltonian with an explicit shift: every site term is -c, the
  environment is -2 rho w, and with full-rank rho the polar update returns
  the isometry unchanged; the energy is exactly zero.
* A chain without product terms, whose environments become nearly rank one:
  their numerically null rows are completed from the current isometry, in
  eager and replayed sweeps alike.
* The largest bond dimension the library accepts (chi = 1024): the top
  layer's ascended operators against the reference, orthonormal isometries
  after a sweep, a lower energy, and the free-fermion bound.
"""
import json
import os

import numpy as np
import pytest

from oracle import physics_ref as P
from oracle import ttn_ref as T
from paper_1905_01331_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "ed_energies.json")) as f:
    GOLD = json.load(f)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1905_01331_amd import binding
    binding.load_library()
    return binding


def rel_err(x, y):
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.abs(x - y).max() / max(1.0, np.abs(y).max()))


FULL_CHI = [
    ("tfim8", I.tfim_chain(1.0), 8, 16, "tfim_chain_L8_h1", "fp64"),
    ("xxx8", I.xxx_chain(), 8, 16, "xxx_chain_L8", "fp64"),
    ("xxx16", I.xxx_chain(), 16, 256, "xxx_chain_L16", "fp64"),
    ("torus4x3", I.torus_tfim_column(3, 3.0), 4, 64, "torus_tfim_4x3_h3", "fp64"),
    ("torus4x4", I.torus_tfim_column(4, 3.0), 4, 256, "torus_tfim_4x4_h3", "fp64"),
    ("tfim16_fp32", I.tfim_chain(1.0), 16, 256, "tfim_chain_L16_h1", "fp32"),
]


@pytest.mark.parametrize("name,model,L,chi,key,prec", FULL_CHI, ids=[c[0] for c in FULL_CHI])
def test_full_bond_dimension_is_exact(B, name, model, L, chi, key, prec):
    print(f"[edge] full chi {name}", flush=True)
    t = B.TTN(B.ChainInput(model, L, chi, prec, seed=3, restarts=40))
    exact = GOLD[key] / (L * model.ly)
    scale = max(abs(exact), abs(t.stats().shift) / model.ly)
    tol = 1e-10 if prec == "fp64" else 2e-6
    e0 = t.energy()[0]
    t.sweep(1)
    e1 = t.energy()[0]
    print(f"  exact {exact:.12f} init {e0:.12f} after a sweep {e1:.12f}")
    assert abs(e0 - exact) <= tol * scale
    assert abs(e1 - exact) <= tol * scale
    t.close()


# (name, model, L, chi, sweeps)
SMALL = [
    ("tfim_L4_chi2", I.tfim_chain(0.7), 4, 2, 3),
    ("xxx_L4_chi3", I.xxx_chain(), 4, 3, 3),
    ("tfim_L8_chi1", I.tfim_chain(1.3), 8, 1, 3),
    ("torus8x3_chi4", I.torus_tfim_column(3, 3.0), 8, 4, 3),
    # deep trees: 18 and 20 levels (2^18 and 2^20 sites; the energy scale
    # grows with L, the bar is relative)
    ("tfim_L262144_chi6_deep", I.tfim_chain(1.0), 1 << 18, 6, 2),
    ("xxx_L1048576_chi4_deep", I.xxx_chain(), 1 << 20, 4, 2),
]


@pytest.mark.parametrize("name,model,L,chi,sweeps", SMALL, ids=[c[0] for c in SMALL])
def test_small_and_degenerate_shapes(B, name, model, L, chi, sweeps):
    # anchored sweeps, as in the float64 sweep parity: the bar follows the
    # conditioning of the reference's environments
    print(f"[edge] {name}", flush=True)
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 9)
    ref = T.TTNRef(L, chi, model.h1, model.A, model.B, ly=model.ly, ws=ws)
    ref.initialise()
    gpu = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, keep_gauge=True))
    assert abs(gpu.energy()[0] - ref.history[0]) <= 1e-12 * abs(ref.history[0]) + 1e-14
    eps = np.finfo(np.float64).eps
    for s in range(sweeps):
        for tau in range(1, ref.n):
            gpu.set_tensor(tau, ref.ws[tau - 1])
        gpu.set_tensor(B.TTN_TOP, ref.v)
        gpu.ascend(1, ref.n - 1)
        gpu.sweep(1)
        e_gpu = gpu.energy()[0]
        e_ref = ref.sweep()
        d = abs(e_gpu - e_ref) / max(abs(e_ref), 1e-300)
        r = float(np.min(ref.diag[-1]["sigma_ratio"]))
        tol = max(1e-10, eps / (10.0 * r))
        print(f"  sweep {s}: relative difference {d:.3e}, sigma_min/sigma_max {r:.2e}, bar {tol:.1e}")
        assert d <= tol
    gpu.close()


def test_zero_hamiltonian_fixed_point(B):
    d, c = 2, 1.0
    model = I.ChainModel("zero", np.zeros((d, d)), np.zeros((0, d, d)), np.zeros((0, d, d)))
    L, chi = 32, 3
    ws = I.random_isometries(T.layer_shapes(L, d, chi), 4)
    gpu = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, shift=c, keep_gauge=True))
    assert abs(gpu.energy()[0]) <= 1e-13
    n = gpu.n_levels()
    gpu.sweep(1)
    assert abs(gpu.energy()[0]) <= 1e-13
    rhos = T.descend_rho_all([gpu.get_tensor(tau) for tau in range(1, n)], gpu.get_tensor(B.TTN_TOP))
    for tau in range(1, n):
        w = gpu.get_tensor(tau)
        ev = np.linalg.eigvalsh(rhos[tau])
        assert ev.min() > 1e-8 * ev.max()  # full rank: the fixed point is unique
        assert np.abs(w - ws[tau - 1]).max() < 1e-11
    gpu.close()


def test_rank_deficient_environments_are_completed(B):
    """A chain without product terms (h1 = -X, D = 0): once the state is
    near its product ground state every one-site density matrix is nearly
    rank one, so are the environments, and the polar update completes their
    numerically null rows from the current isometry (a device flag turns the
    completion on).  Over six sweeps: the energy never rises and stays above
    the exact -1 per site, every isometry keeps orthonormal rows, and sweeps
    replayed from the captured graph (where the flag is read on the device)
    give the eager sweeps' energies and isometries bit for bit."""
    model = I.ChainModel("field", -I.PAULI_X, [], [])
    L, chi = 32, 4
    ws = I.random_isometries(T.layer_shapes(L, 2, chi), 8)
    eager = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws))
    graph = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws))
    hist = [eager.energy()[0]]
    for s in range(6):
        eager.sweep(1)
        graph.sweep(1, graph=True)
        e = eager.energy()[0]
        assert graph.energy()[0] == e, s
        hist.append(e)
    assert all(b <= a + 1e-13 for a, b in zip(hist, hist[1:])), hist
    assert hist[-1] >= -1.0 - 1e-12
    n = eager.n_levels()
    for tau in range(1, n):
        w = eager.get_tensor(tau)
        assert np.array_equal(w, graph.get_tensor(tau)), tau
        W = w.reshape(w.shape[0], -1)
        assert np.abs(W @ W.T - np.eye(W.shape[0])).max() <= 1e-13, tau
    rhos = T.descend_rho_all([eager.get_tensor(tau) for tau in range(1, n)], eager.get_tensor(B.TTN_TOP))
    ev = np.linalg.eigvalsh(rhos[1])
    print(f"  energies {np.array2string(np.array(hist), precision=10)}; level-1 rho spectrum {ev}")
    eager.close()
    graph.close()


def test_largest_bond_dimension(B):
    model, L, chi = I.tfim_chain(1.0), 32, 1024
    print("[edge] chi = 1024", flush=True)
    t = B.TTN(B.ChainInput(model, L, chi, "fp64", seed=5))
    n = t.n_levels()
    assert [t.bond_dim(tau) for tau in range(n)] == [2, 4, 16, 256, 1024]
    top = n - 1
    w = t.get_tensor(top)
    W = w.reshape(w.shape[0], -1)
    assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 2e-15 * 1024
    h = t.get_operator(top - 1, B.TTN_OP_H)
    A = [t.get_operator(top - 1, B.TTN_OP_A, 0)]
    Bm = [t.get_operator(top - 1, B.TTN_OP_B, 0)]
    h2, A2, B2 = T.ascend(w, h, A, Bm)
    assert rel_err(t.get_operator(top, B.TTN_OP_H), h2) < 1e-12
    assert rel_err(t.get_operator(top, B.TTN_OP_A, 0), A2[0]) < 1e-12
    assert rel_err(t.get_operator(top, B.TTN_OP_B, 0), B2[0]) < 1e-12
    del w, W
    e0 = t.energy()[0]
    t.sweep(1)
    e1 = t.energy()[0]
    print(f"  e {e0:.12f} -> {e1:.12f}")
    assert e1 <= e0 + 1e-12
    assert e1 >= P.tfim_free_fermion_energy(L, 1.0) / L - 1e-12
    # Frobenius norm over a x a entries, each within a few eps sqrt(a)
    assert t.stats().ortho_err_max < 64 * np.finfo(np.float64).eps * 1024 ** 1.5
    w = t.get_tensor(top)
    W = w.reshape(w.shape[0], -1)
    assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 2e-15 * 1024
    t.close()
