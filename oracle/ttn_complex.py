"""Plain complex128 CPU reference of the binary-TTN sweep for Hamiltonians
with complex matrix elements.

TEST INFRASTRUCTURE (see the package docstring): slow, obviously correct,
numpy only, no blocking or fusion beyond the definitions below.

The paper writes the method for real tensors (Secs. II.C, III).  Nothing in
it depends on that except the transposes, which become conjugate
transposes.  The readings taken here:

* State: |psi> = sum v[al, be] |al>|be> at the top; a level-tau basis state
  is |a> = sum_{l,r} w[a; l, r] |l>|r> with complex w whose rows are
  orthonormal in the Hermitian sense, sum_{l,r} w[a; l, r] conj(w[a'; l, r])
  = delta (Sec. II.C, the isometric constraint).  v has unit norm.
* Every network value is a bra copy and a ket copy of the same tensors; the
  bra copy is conjugated.  Operators ascend as O'[a, a'] = <a| O |a'> =
  sum conj(w[a; x]) (O w)[a'; x] (Fig. 3), so close() conjugates its first
  argument, and the matrices that descend pair with operators element by
  element: rho[a, a'] = <conj(c_a) c_a'>, the transpose of the usual
  density matrix, so that <O> = sum rho[a, a'] O[a, a'] (the same pairing as
  the real reference).
* Environment (Sec. III.A): the same expression as for real tensors, linear
  in the ket copy; for the energy E(w) of the level (every copy of the
  layer's w), dE along w + eps Delta is 2 L_tau Re sum conj(Delta) Env.
* Update (Sec. III.B, Fig. 10(a)): the isometry minimising the energy
  linearised in w, Re <w, Env>, is w = -U V^H for Env = U S V^H (a x b*b).
* Top tensor: the lowest eigenvector of the Hermitian top Hamiltonian, its
  phase fixed so that its entry of largest magnitude is real and positive.
* Sweep: bottom-up over the layers, then v (Sec. IV), as the real reference.

Pins (tests/test_oracle_complex.py): the complex chain's exact ground energy
against a real chain it maps to exactly (a gauge rotation on a ring whose
total twist is a multiple of 2 pi), full-chi equality with exact
diagonalisation, brute-force state-vector energies, density matrices and
bond energies, finite differences of the brute-force energy and the Euler
identity (environment), the polar characterisation, agreement with the real
reference on real inputs, sweeps that lower the energy above the exact one,
and a planted missing conjugation that a pin catches.
"""
from __future__ import annotations

import numpy as np

from oracle import ttn_ref as _real


num_levels = _real.num_levels
bond_dims = _real.bond_dims
layer_shapes = _real.layer_shapes


def bond_term(h1, A, B):
    """Two-site term 1/2 (h1 x I + I x h1) + sum_k A_k x B_k (complex)."""
    d = h1.shape[0]
    I = np.eye(d)
    b = 0.5 * (np.kron(h1, I) + np.kron(I, h1))
    for a_k, b_k in zip(A, B):
        b = b + np.kron(a_k, b_k)
    return b


def shift_constant(h1, A, B) -> float:
    """c = largest eigenvalue of the (Hermitian) bond term."""
    bt = bond_term(h1, A, B)
    return float(np.linalg.eigvalsh(0.5 * (bt + bt.conj().T))[-1])


# --------------------------------------------------------------------------
# building blocks: the real reference's, with the bra copy conjugated
# --------------------------------------------------------------------------
def apply_r(O, w):
    return np.einsum("xy,aly->alx", O, w)


def apply_l(O, w):
    return np.einsum("xy,ayr->axr", O, w)


def left_mul(X, P):
    return np.einsum("ab,blr->alr", X, P)


def close(P, Q):
    """sum_{l,r} conj(P[a; l, r]) Q[a'; l, r]."""
    return np.einsum("alr,blr->ab", P.conj(), Q)


def close_l(P, Q):
    return np.einsum("alr,amr->lm", P.conj(), Q)


def close_r(P, Q):
    return np.einsum("alr,als->rs", P.conj(), Q)


def pair(X, Y):
    """sum X[x, x'] Y[x, x'] (complex; energies are its real part)."""
    return complex(np.sum(X * Y))


def s_apply(w, h, A, B):
    out = apply_l(h, w) + apply_r(h, w)
    for a_k, b_k in zip(A, B):
        out = out + apply_l(a_k, apply_r(b_k, w))
    return out


def ascend(w, h, A, B):
    """h' = <w| S |w>, A'_k = <w| I x A_k |w>, B'_k = <w| B_k x I |w>."""
    h_new = close(w, s_apply(w, h, A, B))
    A_new = [close(w, apply_r(a_k, w)) for a_k in A]
    B_new = [close(w, apply_l(b_k, w)) for b_k in B]
    return h_new, A_new, B_new


def ascend_all(ws, h0, A0, B0):
    hs, As, Bs = [h0], [list(A0)], [list(B0)]
    for w in ws:
        h, A, B = ascend(w, hs[-1], As[-1], Bs[-1])
        hs.append(h)
        As.append(A)
        Bs.append(B)
    return hs, As, Bs


# --------------------------------------------------------------------------
# the top tensor
# --------------------------------------------------------------------------
def top_matvec(v, h, A, B):
    """H_top v = h v + v h^T + sum_k (A_k v B_k^T + B_k v A_k^T)."""
    out = h @ v + v @ h.T
    for a_k, b_k in zip(A, B):
        out = out + a_k @ v @ b_k.T + b_k @ v @ a_k.T
    return out


def top_matrix(h, A, B):
    x = h.shape[0]
    I = np.eye(x)
    H = np.kron(h, I) + np.kron(I, h)
    for a_k, b_k in zip(A, B):
        H = H + np.kron(a_k, b_k) + np.kron(b_k, a_k)
    return H


def fix_phase(vec):
    """Phase such that the entry of largest magnitude is real and positive."""
    flat = vec.reshape(-1)
    i = int(np.argmax(np.abs(flat)))
    return vec * (abs(flat[i]) / flat[i]) if flat[i] != 0 else vec


def top_eigen(h, A, B):
    """Lowest eigenpair of the Hermitian H_top (dense; small chi only)."""
    x = h.shape[0]
    H = top_matrix(h, A, B)
    evals, evecs = np.linalg.eigh(0.5 * (H + H.conj().T))
    v = evecs[:, 0].reshape(x, x)
    return float(evals[0]), fix_phase(v / np.linalg.norm(v))


# --------------------------------------------------------------------------
# descending matrices
# --------------------------------------------------------------------------
def rho_top(v):
    """1/2 (conj(v) v^T + v^H v): left and right site of the top pair."""
    return 0.5 * (v.conj() @ v.T + v.conj().T @ v)


def descend_rho(w, rho):
    P = left_mul(rho, w)
    return 0.5 * (close_l(w, P) + close_r(w, P))


def descend_rho_all(ws, v):
    n = len(ws) + 1
    rhos = [None] * n
    rhos[n - 1] = rho_top(v)
    for tau in range(n - 1, 0, -1):
        rhos[tau - 1] = descend_rho(ws[tau - 1], rhos[tau])
    return rhos


def dressed_top(v, A_top, B_top):
    """Rbar_k = 1/2 (v^H A_k v + conj(v) A_k v^T), Lbar_k = 1/2 (conj(v) B_k v^T
    + v^H B_k v): the two bonds of the top pair, seen from the B site and
    from the A site."""
    vb = v.conj()
    R = [0.5 * (vb.T @ a @ v + vb @ a @ v.T) for a in A_top]
    Lb = [0.5 * (vb @ b @ v.T + vb.T @ b @ v) for b in B_top]
    return R, Lb


def descend_dressed(w, rho, R, Lb, A_low, B_low):
    R_new, L_new = [], []
    for a_k, b_k, r_k, l_k in zip(A_low, B_low, R, Lb):
        inside_R = close_r(w, left_mul(rho, apply_l(a_k, w)))
        cross_R = close_l(w, left_mul(r_k, w))
        R_new.append(0.5 * (inside_R + cross_R))
        inside_L = close_l(w, left_mul(rho, apply_r(b_k, w)))
        cross_L = close_r(w, left_mul(l_k, w))
        L_new.append(0.5 * (inside_L + cross_L))
    return R_new, L_new


def dressed_chain(ws, v, rhos, tau, A_low, B_low):
    """Rbar^(tau), Lbar^(tau): A^(tau-1), B^(tau-1) carried up through the
    current layers tau..n-1, dressed at the top, descended back to tau."""
    n = len(ws) + 1
    At = {tau - 1: list(A_low)}
    Bt = {tau - 1: list(B_low)}
    for sigma in range(tau, n):
        w = ws[sigma - 1]
        At[sigma] = [close(w, apply_r(a, w)) for a in At[sigma - 1]]
        Bt[sigma] = [close(w, apply_l(b, w)) for b in Bt[sigma - 1]]
    R, Lb = dressed_top(v, At[n - 1], Bt[n - 1])
    for sigma in range(n - 1, tau, -1):
        R, Lb = descend_dressed(ws[sigma - 1], rhos[sigma], R, Lb, At[sigma - 1], Bt[sigma - 1])
    return R, Lb


# --------------------------------------------------------------------------
# environment, update, energy
# --------------------------------------------------------------------------
def environment(w, h, A, B, rho, R, Lb):
    E = left_mul(rho, s_apply(w, h, A, B))
    for a_k, b_k, r_k, l_k in zip(A, B, R, Lb):
        E = E + left_mul(r_k, apply_l(b_k, w)) + left_mul(l_k, apply_r(a_k, w))
    return E


def polar_update(env):
    """w = -U V^H from the thin SVD of Env (a x b*b)."""
    a = env.shape[0]
    U, s, Vh = np.linalg.svd(env.reshape(a, -1), full_matrices=False)
    return -(U @ Vh).reshape(env.shape), s


def level_energy(L, tau, h, B, rho, R, c):
    """Re(L_tau [<rho, h> + sum_k <Rbar_k, B_k>]) + c L."""
    e = pair(rho, h) + sum(pair(r, b) for r, b in zip(R, B))
    return (L >> tau) * e.real + c * L


def ortho_error(w):
    W = w.reshape(w.shape[0], -1)
    return float(np.linalg.norm(W @ W.conj().T - np.eye(W.shape[0])))


class ComplexTTNRef:
    """State of a uniform binary TTN with complex tensors and its sweep."""

    def __init__(self, L, chi, h1, A, B, ws, ly=1, shift=None, v=None):
        self.L = int(L)
        self.n = num_levels(L)
        self.h1 = np.asarray(h1, dtype=np.complex128)
        self.A0 = [np.asarray(a, dtype=np.complex128) for a in A]
        self.B0 = [np.asarray(b, dtype=np.complex128) for b in B]
        self.d = self.h1.shape[0]
        self.D = len(self.A0)
        self.ly = ly
        self.dims = bond_dims(L, self.d, chi)
        self.c = shift_constant(self.h1, self.A0, self.B0) if shift is None else float(shift)
        self.h0 = self.h1 - self.c * np.eye(self.d)
        self.ws = [np.array(w, dtype=np.complex128) for w in ws]
        for t, w in enumerate(self.ws, start=1):
            if w.shape != (self.dims[t], self.dims[t - 1], self.dims[t - 1]):
                raise ValueError(f"layer {t}: shape {w.shape}")
        self.v = None if v is None else np.array(v, dtype=np.complex128)
        self.lam = None
        self.history = []
        self.diag = []

    def energy_per_site(self):
        return (self.lam + self.c * self.L) / (self.L * self.ly)

    def initialise(self):
        self.hs, self.As, self.Bs = ascend_all(self.ws, self.h0, self.A0, self.B0)
        top = self.n - 1
        self.lam, self.v = top_eigen(self.hs[top], self.As[top], self.Bs[top])
        self.history.append(self.energy_per_site())
        return self.energy_per_site()

    def sweep(self):
        n = self.n
        rhos = descend_rho_all(self.ws, self.v)
        info = {"ortho": [], "sigma_ratio": []}
        for tau in range(1, n):
            w = self.ws[tau - 1]
            h, A, B = self.hs[tau - 1], self.As[tau - 1], self.Bs[tau - 1]
            R, Lb = dressed_chain(self.ws, self.v, rhos, tau, A, B)
            env = environment(w, h, A, B, rhos[tau], R, Lb)
            w_new, s = polar_update(env)
            self.ws[tau - 1] = w_new
            info["ortho"].append(ortho_error(w_new))
            info["sigma_ratio"].append(float(s[-1] / s[0]) if s[0] > 0 else 0.0)
            self.hs[tau], self.As[tau], self.Bs[tau] = ascend(w_new, h, A, B)
        top = n - 1
        self.lam, self.v = top_eigen(self.hs[top], self.As[top], self.Bs[top])
        self.history.append(self.energy_per_site())
        self.diag.append(info)
        return self.energy_per_site()

    def run(self, sweeps):
        if self.v is None:
            self.initialise()
        for _ in range(sweeps):
            self.sweep()
        return list(self.history)
