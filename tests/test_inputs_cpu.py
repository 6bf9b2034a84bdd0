"""The seeded input builders used by the bond-dimension ladder of the paper's
workload: a state embedded into larger bond dimensions is the same state."""
import numpy as np
import pytest

from oracle import ttn_ref as T
from paper_1905_01331_amd import inputs as I


def _energy(model, L, ws, v):
    """<v, H_top v> + c L of the network (ws, v), without re-solving the top."""
    h0 = model.h1 - T.shift_constant(model.h1, model.A, model.B) * np.eye(model.d)
    hs, As, Bs = T.ascend_all(ws, h0, list(model.A), list(model.B))
    top = len(ws)
    c = T.shift_constant(model.h1, model.A, model.B)
    return T.pair(v, T.top_matvec(v, hs[top], As[top], Bs[top])) + c * L


@pytest.mark.parametrize("name,model,L,chi0,chi1", [
    ("tfim", I.tfim_chain(0.9), 32, 6, 10),
    ("xxx", I.xxx_chain(), 32, 5, 12),
    ("torus", I.torus_tfim_column(3, 2.9), 8, 12, 20),
])
def test_embedding_keeps_the_state(name, model, L, chi0, chi1):
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi0), 3)
    v = I.random_top(ws[-1].shape[0], 4)
    shapes = T.layer_shapes(L, model.d, chi1)
    ws2 = I.embed_isometries(ws, shapes, 5)
    v2 = I.embed_top(v, shapes[-1][0])
    for w, (a, b) in zip(ws2, shapes):
        assert w.shape == (a, b, b)
        W = w.reshape(w.shape[0], -1)
        assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 1e-13
    e1 = _energy(model, L, ws, v)
    e2 = _energy(model, L, ws2, v2)
    assert e2 == pytest.approx(e1, rel=1e-12, abs=1e-12)
    # the added directions carry no weight: the one-site density matrices of
    # the larger network vanish outside the old corner
    rhos = T.descend_rho_all(ws2, v2)
    for tau, r in enumerate(rhos):
        k = ws[tau - 1].shape[0] if tau > 0 else model.d
        assert np.abs(r[k:, :]).max(initial=0.0) < 1e-14
        assert np.abs(r[:, k:]).max(initial=0.0) < 1e-14
