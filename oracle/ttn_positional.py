"""CPU reference of the position-resolved binary TTN: every node its own
isometry (test infrastructure; only tests/, the smoke check and the bench's
CPU leg use it).

The paper labels the isometries w^(tau, m) by layer and position (Sec. II.C)
and makes them equal along a layer only because its Hamiltonians are
translation invariant (Sec. III).  Here the L_tau isometries of layer tau are
independent.  Plain float64 numpy, written from the paper's construction:

* Network: node m of level tau (tau = 1..n-1, m = 0..L_tau - 1, L_tau =
  L / 2^tau) has the isometry w^(tau, m)[a; l, r] whose input legs are the
  upper indices of nodes 2m (left) and 2m+1 (right) of level tau-1; level 0
  are the sites.  The top tensor v[alpha, beta] joins nodes 0 and 1 of
  level n-1 (Eq. (normalization)).
* Ascending (Sec. III.A, Fig. 3): node m of level tau carries h^(tau, m), the
  sum of every term inside its block, and for each product term k the
  operators of its edges: A^(tau, m)_k from its last site (the A of a bond
  leaving the block to the right) and B^(tau, m)_k from its first site (the B
  of a bond arriving from the left).  Through w (left child L, right child
  R): h = w [h_L x I + I x h_R + sum_k A_{L,k} x B_{R,k}] w^T,
  A_k = w (I x A_{R,k}) w^T, B_k = w (B_{L,k} x I) w^T.  The one-site term at
  level 0 is h1 - c I with the shift c of the uniform reference.
* Top: H_top v = h_0 v + v h_1^T + sum_k (A_{0,k} v B_{1,k}^T + B_{0,k} v
  A_{1,k}^T), the second product for the periodic bond from the last site
  back to the first; E = lambda + c L.
* Descending: rho^(n-1, 0) = v v^T, rho^(n-1, 1) = v^T v; a left child takes
  C_L(w, rho o w) of its parent, a right child C_R(w, rho o w).  The two-site
  information of a node's edges: X^(tau, m)_k multiplies B^(tau, m)_k (its
  left edge; the partner A sits at the right edge of the block to the left)
  and Y^(tau, m)_k multiplies A^(tau, m)_k, so that each bond energy is one
  pairing.  At the top X^(n-1, 1) = v^T A_0 v, Y^(n-1, 0) = v B_1 v^T,
  X^(n-1, 0) = v A_1 v^T, Y^(n-1, 1) = v^T B_0 v.  Through a parent: the
  outer edges take the parent's (X_L = C_L(w, X o w), Y_R = C_R(w, Y o w));
  the inner edges meet inside the parent (X_R = C_R(w, rho o (A_L .l w)),
  Y_L = C_L(w, rho o (B_R .r w))).
* Environment of w^(tau, m) (Sec. III.A, Fig. 2(b)): Env = rho o (S w) +
  sum_k X_k o (B_{L,k} .l w) + sum_k Y_k o (A_{R,k} .r w), with S w =
  h_L .l w + h_R .r w + sum_k A_{L,k} .l (B_{R,k} .r w); the energy is
  quadratic in each single w and Env = 1/2 dE/dw.
* Update (Sec. III.B): w <- -U V^T from the SVD of Env (the same reading as
  the uniform reference).
* Sweep (Sec. IV): layers bottom-up; within a layer the even nodes and then
  the odd ones, each group from one state (nodes of one parity are never
  neighbours, so each group is an exact block step); then the top tensor is
  the lowest eigenvector of H_top.
"""
from __future__ import annotations

import numpy as np

from oracle import ttn_ref as T


# --------------------------------------------------------------------------
# the network
# --------------------------------------------------------------------------
def level_state(nws, v, level):
    """State on the sites of `level` (one index per node, left to right),
    contracted from the top through every node's own isometry."""
    n = len(nws) + 1
    psi = np.array(v)
    for tau in range(n - 1, level, -1):
        layer = nws[tau - 1]
        for pos in range(psi.ndim):
            axis = 2 * pos
            psi = np.tensordot(psi, layer[pos], axes=([axis], [0]))
            psi = np.moveaxis(psi, [-2, -1], [axis, axis + 1])
    return psi


# --------------------------------------------------------------------------
# ascending
# --------------------------------------------------------------------------
def ascend_node(w, hL, hR, AL, BL, AR, BR):
    """Operators of a node from those of its children (left L, right R)."""
    Sw = T.apply_l(hL, w) + T.apply_r(hR, w)
    for a_k, b_k in zip(AL, BR):
        Sw = Sw + T.apply_l(a_k, T.apply_r(b_k, w))
    h = T.close(w, Sw)
    A = [T.close(w, T.apply_r(a_k, w)) for a_k in AR]
    B = [T.close(w, T.apply_l(b_k, w)) for b_k in BL]
    return h, A, B


def ascend_all(nws, h0, A0, B0, L):
    """hs[tau][m], As[tau][m][k], Bs[tau][m][k] for every level and node."""
    hs = [[h0.copy() for _ in range(L)]]
    As = [[list(A0) for _ in range(L)]]
    Bs = [[list(B0) for _ in range(L)]]
    for tau, layer in enumerate(nws, start=1):
        h_t, A_t, B_t = [], [], []
        for m, w in enumerate(layer):
            l, r = 2 * m, 2 * m + 1
            h, A, B = ascend_node(w, hs[tau - 1][l], hs[tau - 1][r], As[tau - 1][l], Bs[tau - 1][l],
                                  As[tau - 1][r], Bs[tau - 1][r])
            h_t.append(h)
            A_t.append(A)
            B_t.append(B)
        hs.append(h_t)
        As.append(A_t)
        Bs.append(B_t)
    return hs, As, Bs


# --------------------------------------------------------------------------
# the top tensor
# --------------------------------------------------------------------------
def top_matvec(v, h0, h1, A0, B0, A1, B1):
    out = h0 @ v + v @ h1.T
    for a0, b0, a1, b1 in zip(A0, B0, A1, B1):
        out = out + a0 @ v @ b1.T + b0 @ v @ a1.T
    return out


def top_matrix(h0, h1, A0, B0, A1, B1):
    x = h0.shape[0]
    I = np.eye(x)
    H = np.kron(h0, I) + np.kron(I, h1)
    for a0, b0, a1, b1 in zip(A0, B0, A1, B1):
        H = H + np.kron(a0, b1) + np.kron(b0, a1)
    return H


def top_eigen(h0, h1, A0, B0, A1, B1):
    """Lowest eigenpair of H_top (dense; the tests keep chi small)."""
    H = top_matrix(h0, h1, A0, B0, A1, B1)
    H = 0.5 * (H + H.T)
    evals, evecs = np.linalg.eigh(H)
    x = h0.shape[0]
    v = evecs[:, 0].reshape(x, x)
    return float(evals[0]), T.fix_sign(v / np.linalg.norm(v))


# --------------------------------------------------------------------------
# descending
# --------------------------------------------------------------------------
def descend_all(nws, v, As, Bs):
    """rho[tau][m], X[tau][m][k], Y[tau][m][k] for every level tau >= 0 and
    node, from the current tensors (As, Bs ascended with them)."""
    n = len(nws) + 1
    rho = [None] * n
    X = [None] * n
    Y = [None] * n
    top = n - 1
    rho[top] = [v @ v.T, v.T @ v]
    X[top] = [[v @ a1 @ v.T for a1 in As[top][1]], [v.T @ a0 @ v for a0 in As[top][0]]]
    Y[top] = [[v @ b1 @ v.T for b1 in Bs[top][1]], [v.T @ b0 @ v for b0 in Bs[top][0]]]
    for tau in range(top, 0, -1):
        layer = nws[tau - 1]
        Lc = len(layer) * 2
        rho_lo, X_lo, Y_lo = [None] * Lc, [None] * Lc, [None] * Lc
        for m, w in enumerate(layer):
            l, r = 2 * m, 2 * m + 1
            P = T.left_mul(rho[tau][m], w)
            rho_lo[l] = T.close_l(w, P)
            rho_lo[r] = T.close_r(w, P)
            X_lo[l] = [T.close_l(w, T.left_mul(x, w)) for x in X[tau][m]]
            Y_lo[r] = [T.close_r(w, T.left_mul(y, w)) for y in Y[tau][m]]
            X_lo[r] = [T.close_r(w, T.left_mul(rho[tau][m], T.apply_l(a, w))) for a in As[tau - 1][l]]
            Y_lo[l] = [T.close_l(w, T.left_mul(rho[tau][m], T.apply_r(b, w))) for b in Bs[tau - 1][r]]
        rho[tau - 1], X[tau - 1], Y[tau - 1] = rho_lo, X_lo, Y_lo
    return rho, X, Y


def environment(w, hL, hR, AL, BL, AR, BR, rho, X, Y):
    """Env of one node's isometry (same index shape as w)."""
    Sw = T.apply_l(hL, w) + T.apply_r(hR, w)
    for a_k, b_k in zip(AL, BR):
        Sw = Sw + T.apply_l(a_k, T.apply_r(b_k, w))
    E = T.left_mul(rho, Sw)
    for x_k, b_k in zip(X, BL):
        E = E + T.left_mul(x_k, T.apply_l(b_k, w))
    for y_k, a_k in zip(Y, AR):
        E = E + T.left_mul(y_k, T.apply_r(a_k, w))
    return E


# --------------------------------------------------------------------------
# the reference
# --------------------------------------------------------------------------
class PositionalTTN:
    """Position-resolved TTN energy minimisation, float64.  nws[tau-1][m] is
    the isometry of node m of layer tau (an input: inputs.random_node_isometries
    draws seeded ones); v the top tensor (solved at initialisation when not
    given)."""

    def __init__(self, L, chi, h1, A, B, nws, ly=1, v=None, shift=None):
        self.L, self.chi, self.ly = L, chi, ly
        self.h1 = np.asarray(h1, dtype=np.float64)
        self.A = [np.asarray(a, dtype=np.float64) for a in A]
        self.B = [np.asarray(b, dtype=np.float64) for b in B]
        self.D = len(self.A)
        self.d = self.h1.shape[0]
        self.n = T.num_levels(L)
        self.dims = T.bond_dims(L, self.d, chi)
        self.c = T.shift_constant(self.h1, self.A, self.B) if shift is None else float(shift)
        self.h0 = self.h1 - self.c * np.eye(self.d)
        self.nws = [[np.array(w, dtype=np.float64) for w in layer] for layer in nws]
        self.v = v
        self.history = []
        self.diag = []

    def operators(self):
        return ascend_all(self.nws, self.h0, self.A, self.B, self.L)

    def solve_top(self, hs, As, Bs):
        top = self.n - 1
        lam, v = top_eigen(hs[top][0], hs[top][1], As[top][0], Bs[top][0], As[top][1], Bs[top][1])
        self.v = v
        return lam

    def energy(self, hs=None, As=None, Bs=None):
        """Energy per spin of the current tensors (v as it is)."""
        if hs is None:
            hs, As, Bs = self.operators()
        top = self.n - 1
        Hv = top_matvec(self.v, hs[top][0], hs[top][1], As[top][0], Bs[top][0], As[top][1], Bs[top][1])
        return (T.pair(self.v, Hv) / T.pair(self.v, self.v) + self.c * self.L) / (self.L * self.ly)

    def initialise(self):
        hs, As, Bs = self.operators()
        if self.v is None:
            self.solve_top(hs, As, Bs)
        e = self.energy(hs, As, Bs)
        self.history = [e]
        return e

    def node_env(self, tau, m, hs, As, Bs, rho, X, Y):
        l, r = 2 * m, 2 * m + 1
        lo = tau - 1
        return environment(self.nws[tau - 1][m], hs[lo][l], hs[lo][r], As[lo][l], Bs[lo][l], As[lo][r],
                           Bs[lo][r], rho[tau][m], X[tau][m], Y[tau][m])

    def sweep(self):
        """One sweep: layers bottom-up, even nodes then odd nodes of each
        layer, each group's environments from one state; then the top."""
        info = {"sigma_ratio": []}
        for tau in range(1, self.n):
            for parity in (0, 1):
                hs, As, Bs = self.operators()
                rho, X, Y = descend_all(self.nws, self.v, As, Bs)
                for m in range(parity, self.L >> tau, 2):
                    env = self.node_env(tau, m, hs, As, Bs, rho, X, Y)
                    w_new, s = T.polar_update(env)
                    info["sigma_ratio"].append(float(s[-1] / s[0]) if s[0] > 0 else 0.0)
                    self.nws[tau - 1][m] = w_new
        hs, As, Bs = self.operators()
        self.solve_top(hs, As, Bs)
        e = self.energy(hs, As, Bs)
        self.history.append(e)
        self.diag.append(info)
        return e

    def run(self, sweeps):
        if not self.history:
            self.initialise()
        for _ in range(sweeps):
            self.sweep()
        return list(self.history)
