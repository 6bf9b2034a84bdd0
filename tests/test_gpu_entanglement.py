"""Entanglement spectrum and entropy of a block (Sec. V) on the GPU path
against the CPU reference, from identical states.

Every case loads the reference's isometries and a random top tensor into
the handle and compares, for every level tau and both the position-averaged
and the leftmost block, the spectrum element by element (absolute, the
spectrum sums to one) and the entropy.  The computation is float64 from the
master isometries whatever the bulk precision, so mixed-precision handles are
held to the same bar.  Levels whose bond exceeds 64 take the persistent
blocked Jacobi solver.
"""
import numpy as np
import pytest

from oracle import ttn_ref as T
from paper_1905_01331_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1905_01331_amd import binding
    binding.load_library()
    return binding


CASES = [
    ("tfim_L64_chi24", I.tfim_chain(1.0), 64, 24, "fp64"),
    ("xxx_L32_chi160", I.xxx_chain(), 32, 160, "fp64"),
    ("torus8x4_chi64_bf16x3", I.torus_tfim_column(4, 3.0), 8, 64, "bf16x3"),
    ("tfim_L16_chi7_fp32", I.tfim_chain(0.6), 16, 7, "fp32"),
]


@pytest.mark.parametrize("name,model,L,chi,prec", CASES, ids=[c[0] for c in CASES])
def test_entanglement_matches_reference(B, name, model, L, chi, prec):
    print(f"[entanglement] {name}", flush=True)
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 11)
    v = I.random_top(ws[-1].shape[0], 11)
    t = B.TTN(B.ChainInput(model, L, chi, prec, w0=ws))
    t.set_tensor(B.TTN_TOP, v)
    n = len(ws) + 1
    worst_p, worst_s = 0.0, 0.0
    for tau in range(n):
        for which, ref_rho in ((B.TTN_ENT_AVERAGE, T.rho_average), (B.TTN_ENT_LEFTMOST, T.rho_leftmost)):
            p, S = t.entanglement(tau, which)
            p_ref, _, S_ref = T.entanglement(ref_rho(ws, v, tau))
            assert p.shape == p_ref.shape
            assert np.all(np.diff(p) <= 0.0)
            worst_p = max(worst_p, float(np.abs(p - p_ref).max()))
            worst_s = max(worst_s, abs(S - S_ref))
    print(f"  worst spectrum difference {worst_p:.2e}, entropy {worst_s:.2e}")
    assert worst_p < 1e-12
    assert worst_s < 1e-10
    t.close()


def test_entanglement_after_sweeps_and_state_unchanged(B):
    # the entanglement call must not disturb the sweep: the same sweeps with
    # and without entanglement calls in between give identical energies
    model, L, chi = I.tfim_chain(1.0), 128, 32
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 12)
    a = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws))
    b = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws))
    n = a.n_levels()
    for _ in range(3):
        a.sweep(1)
        b.sweep(1)
        for tau in range(n):
            b.entanglement(tau, B.TTN_ENT_AVERAGE)
            b.entanglement(tau, B.TTN_ENT_LEFTMOST)
        assert a.energy()[0] == b.energy()[0]
    state = [b.get_tensor(tau) for tau in range(1, n)]
    v = b.get_tensor(B.TTN_TOP)
    for tau in range(n):
        p, S = b.entanglement(tau, B.TTN_ENT_AVERAGE)
        p_ref, _, S_ref = T.entanglement(T.rho_average(state, v, tau))
        assert np.abs(p - p_ref).max() < 1e-12 and abs(S - S_ref) < 1e-10
        assert abs(p.sum() - 1.0) < 1e-12
    # the two halves of the chain (leftmost block at the top level vs its
    # complement) share their spectrum
    pl, Sl = b.entanglement(n - 1, B.TTN_ENT_LEFTMOST)
    pr = T.entanglement(v.T @ v)[0]
    assert np.abs(pl - pr).max() < 1e-12
    a.close()
    b.close()


def test_entanglement_rejects_bad_arguments(B):
    t = B.TTN(B.ChainInput(I.tfim_chain(1.0), 16, 8, "fp64", seed=1))
    with pytest.raises(B.TTNError) as e:
        t.entanglement(t.n_levels(), B.TTN_ENT_AVERAGE)
    assert e.value.status == B.TTN_EINVAL
    with pytest.raises(B.TTNError) as e:
        t.entanglement(1, 7)
    assert e.value.status == B.TTN_EINVAL
    t.close()


@pytest.mark.parametrize("name,model,L,chi,prec", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_node_entanglement_matches_reference(B, name, model, L, chi, prec):
    # the block of any node: its matrix descended along its own path, against
    # the reference's matrix of that node (rho_positions); node 0 is the
    # leftmost block, and the two halves of v share their spectrum
    print(f"[entanglement] nodes {name}", flush=True)
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 12)
    v = I.random_top(ws[-1].shape[0], 12)
    t = B.TTN(B.ChainInput(model, L, chi, prec, w0=ws))
    t.set_tensor(B.TTN_TOP, v)
    n = len(ws) + 1
    rhos = T.rho_positions(ws, v)
    rng = np.random.default_rng(1)
    worst_p, worst_s = 0.0, 0.0
    for tau in range(n):
        cnt = L >> tau
        for node in sorted({0, 1, cnt - 1, int(rng.integers(cnt))}):
            p, S = t.entanglement_node(tau, node)
            p_ref, _, S_ref = T.entanglement(rhos[tau][node])
            worst_p = max(worst_p, float(np.abs(p - p_ref).max()))
            worst_s = max(worst_s, abs(S - S_ref))
        p0, S0 = t.entanglement_node(tau, 0)
        pl, Sl = t.entanglement(tau, B.TTN_ENT_LEFTMOST)
        assert np.array_equal(p0, pl) and S0 == Sl
    pa, Sa = t.entanglement_node(n - 1, 0)
    pb, Sb = t.entanglement_node(n - 1, 1)
    assert np.abs(pa - pb).max() < 1e-13 and abs(Sa - Sb) < 1e-12
    print(f"  worst spectrum difference {worst_p:.2e}, entropy {worst_s:.2e}")
    assert worst_p < 1e-12
    assert worst_s < 1e-10
    for tau, node in ((0, L), (1, -1), (n, 0)):
        with pytest.raises(B.TTNError) as e:
            t.entanglement_node(tau, node)
        assert e.value.status == B.TTN_EINVAL
    t.close()
