"""Plants plausible mistakes in the CPU reference (on the CPU only) and checks
that the pins of test_oracle_pins.py catch each one."""
import numpy as np
import pytest

from oracle import physics_ref as P
from oracle import ttn_ref as T
from paper_1905_01331_amd import inputs as I


def _setup(model, L=16, chi=6, seed=2):
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), seed)
    r = T.TTNRef(L, chi, model.h1, model.A, model.B, ly=model.ly, ws=ws)
    r.initialise()
    return r


def _pins_hold():
    """A compact run of the brute-force / invariant pins; False on any miss."""
    for model, phys in ((I.xxx_chain(), P.heisenberg_chain_hamiltonian(16)),
                        (I.tfim_chain(0.8), P.tfim_chain_hamiltonian(16, 0.8))):
        r = _setup(model)
        L = r.L
        v = I.random_top(r.dims[-1], 9)
        top = r.n - 1
        e_ttn = T.pair(v, T.top_matvec(v, r.hs[top], r.As[top], r.Bs[top])) + r.c * L
        psi = P.full_state(r.ws, v)
        if abs(e_ttn - float(psi @ (phys @ psi))) > 1e-10:
            return False
        rhos = T.descend_rho_all(r.ws, v)
        for tau in range(r.n):
            bf = P.one_site_rdm_average(P.level_state(r.ws, v, tau))
            if np.abs(rhos[tau] - bf).max() > 1e-12:
                return False
        for tau in range(1, r.n):
            R, Lb = T.dressed_chain(r.ws, v, rhos, tau, r.As[tau - 1], r.Bs[tau - 1])
            psi_t = P.level_state(r.ws, v, tau)
            for k in range(model.D):
                bf = P.bond_expectation_sum(psi_t, r.As[tau][k], r.Bs[tau][k])
                if abs((L >> tau) * T.pair(R[k], r.Bs[tau][k]) - bf) > 1e-10:
                    return False
                if abs((L >> tau) * T.pair(Lb[k], r.As[tau][k]) - bf) > 1e-10:
                    return False
            Rs, Ls = T.dressed_all(r.ws, v, rhos, r.As, r.Bs)
            for k in range(model.D):
                bf = P.bond_expectation_sum(psi_t, r.As[tau][k], r.Bs[tau][k])
                if abs((L >> tau) * T.pair(Rs[tau][k], r.Bs[tau][k]) - bf) > 1e-10:
                    return False
                if abs((L >> tau) * T.pair(Ls[tau][k], r.As[tau][k]) - bf) > 1e-10:
                    return False
            w = r.ws[tau - 1]
            env = T.environment(w, r.hs[tau - 1], r.As[tau - 1], r.Bs[tau - 1], rhos[tau], R, Lb)
            e_bond = (L >> tau) * sum(T.pair(x, y) for x, y in zip(R, r.Bs[tau]))
            e_shift = e_ttn - r.c * L
            if abs((L >> tau) * T.pair(w, env) - (e_shift + e_bond)) > 1e-10:
                return False
    # the update is the polar factor: -Env w^T symmetric positive definite
    env = np.random.default_rng(3).standard_normal((6, 4, 4))
    w, _ = T.polar_update(env)
    M = -env.reshape(6, -1) @ w.reshape(6, -1).T
    if np.abs(M - M.T).max() > 1e-12 or np.linalg.eigvalsh(0.5 * (M + M.T)).min() <= 0:
        return False
    # the sweep lowers the energy
    r = _setup(I.tfim_chain(1.0), 16, 8, 0)
    hist = r.run(4)
    if not all(b <= a + 1e-12 for a, b in zip(hist, hist[1:])):
        return False
    if max(max(info["ortho"]) for info in r.diag) > 1e-12:
        return False
    return True


def test_unmutated_reference_passes():
    assert _pins_hold()


MUTATIONS = {
    "apply_l transposed operator": ("apply_l", lambda O, w: np.einsum("yx,ayr->axr", O, w)),
    "apply_r on the wrong leg": ("apply_r", lambda O, w: np.einsum("xy,ayr->axr", O, w)),
    "descend without the 1/2": ("descend_rho", lambda w, rho: T.close_l(w, T.left_mul(rho, w)) + T.close_r(w, T.left_mul(rho, w))),
    "top dressing v <-> v^T": ("dressed_top", lambda v, A, B: ([0.5 * (v @ a @ v.T + v @ a @ v.T) for a in A], [0.5 * (v @ b @ v.T + v.T @ b @ v) for b in B])),
    "environment drops Lbar term": ("environment", lambda w, h, A, B, rho, R, Lb: T.left_mul(rho, T.s_apply(w, h, A, B)) + sum((T.left_mul(r, T.apply_l(b, w)) for b, r in zip(B, R)), np.zeros_like(w))),
    "update keeps the singular values": ("polar_update", lambda env: _svd_variant(env, keep_s=True)),
    "update drops the left factor": ("polar_update", lambda env: _svd_variant(env, drop_u=True)),
    "one-pass chain carries Lbar as Rbar": ("dressed_all", lambda ws, v, rhos, As, Bs: _dressed_all_swapped(ws, v, rhos, As, Bs)),
    "s_apply B on the left child": ("s_apply", lambda w, h, A, B: T.apply_l(h, w) + T.apply_r(h, w) + sum((T.apply_r(a, T.apply_l(b, w)) for a, b in zip(A, B)), np.zeros_like(w))),
}
_ORIG = {}


def _dressed_all_swapped(ws, v, rhos, As, Bs):
    n = len(ws) + 1
    Rs, Ls = [None] * n, [None] * n
    R, Lb = T.dressed_top(v, As[n - 1], Bs[n - 1])
    Rs[n - 1], Ls[n - 1] = R, Lb
    for sigma in range(n - 1, 1, -1):
        R, Lb = T.descend_dressed(ws[sigma - 1], rhos[sigma], Lb, R, As[sigma - 1], Bs[sigma - 1])
        Rs[sigma - 1], Ls[sigma - 1] = R, Lb
    return Rs, Ls


def _svd_variant(env, keep_s=False, drop_u=False):
    a = env.shape[0]
    U, s, Vt = np.linalg.svd(env.reshape(a, -1), full_matrices=False)
    if keep_s:
        W = -(U * (s / s.max())) @ Vt
    else:
        W = -Vt
    return W.reshape(env.shape), s


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    _ORIG[attr] = getattr(T, attr)
    monkeypatch.setattr(T, attr, fn)
    assert not _pins_hold(), f"pins missed: {name}"
