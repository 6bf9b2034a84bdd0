"""Plain float64 CPU reference of the binary-TTN energy-minimisation sweep.

TEST INFRASTRUCTURE (see the package docstring): slow, obviously correct,
numpy/scipy only, no blocking or fusion beyond the definitions below.

What the paper fixes, and the readings taken where it is silent
---------------------------------------------------------------
* Ansatz (Sec. II.C, Eqs. (constraint), (normalization)): a binary tree over
  L = 2**n effective sites.  Layer tau = 1..n-1 holds one isometry w_tau that
  is shared by every position (translation invariance, Sec. III), shape
  (a, b, b) with a = chi_tau, b = chi_{tau-1}, and rows orthonormal:
  sum_{l,r} w[a;l,r] w[a';l,r] = delta.  The top tensor v (chi_{n-1} x
  chi_{n-1}) joins the two sites of level n-1 and has unit Frobenius norm.
  Reading: chi_0 = d, chi_tau = min(chi_{tau-1}**2, chi) (a bond cannot
  exceed the Hilbert-space dimension of the block below it).
* Hamiltonian (Eqs. (H1D), (1)-(5)): an effective chain
  H = sum_j [h1_j + sum_k A_{k,j} B_{k,j+1}], periodic; the product form of
  the bond term is the "bond index of dimension L_y" of Fig. 2(b).
* Environment (Sec. III.A, Figs. 2(b), 3): the sum over Hamiltonian terms of
  the network with one copy of w removed, w w^T pairs outside the causal cone
  removed by the isometric constraint, evaluated as a sequence of matrix
  products of cost at most O(chi**4) (Fig. 4(b)).  Reading: for a layer whose
  copies are all equal, Env = (1 / (2 L_tau)) dE/dw summed over all copies at
  the current tensors, with the one-site reduced density matrices averaged
  over positions.
* Update (Sec. III.B, Fig. 4(c-d), Fig. 10(a)): SVD of the flattened
  environment and w = V U^dagger.  Reading: with the Hamiltonian shifted so
  that every bond term is negative semidefinite (shift c = largest eigenvalue
  of the bond term), w = -U V^T for Env = U S V^T written with w's index
  shape (a x b*b); this is the same polar factor and it minimises the energy
  linearised in w.
* Top tensor: "updated similarly" (Sec. III.B).  Reading: v is the lowest
  eigenvector of the top Hamiltonian (the fixed point of repeating the update
  on v), sign fixed so that its entry of largest magnitude is positive.
* Sweep (Sec. IV, Sec. V): one update of every isometry; bottom-up
  (tau = 1..n-1), then v.  Convergence: the energy per site changes by less
  than 1e-10 over a sweep (Sec. IV).

Notation
--------
Operators are one-site matrices O[x, x'] (ket index first); the pairing is
<X, Y> = sum X[x, x'] Y[x, x'].  Building blocks, each one matrix product:
  apply_r(O, w)[a;l,r] = sum_r' O[r,r'] w[a;l,r']
  apply_l(O, w)[a;l,r] = sum_l' O[l,l'] w[a;l',r]
  left_mul(X, P)[a;l,r] = sum_a' X[a,a'] P[a';l,r]
  close(P, Q)[a,a']   = sum_{l,r} P[a;l,r] Q[a';l,r]
  close_l(P, Q)[l,l'] = sum_{a,r} P[a;l,r] Q[a;l',r]
  close_r(P, Q)[r,r'] = sum_{a,l} P[a;l,r] Q[a;l,r']

Pins (tests/test_oracle_*.py): full-chi equality with exact diagonalisation
(ascend + top + shift), brute-force state-vector energies and one-site RDMs
(ascend, descend), brute-force bond energies and level independence
(dressed chains), finite differences of a brute-force quartic energy and the
Euler identity (environment), the polar characterisation (update), residual
and dense eigensolver agreement (top), closed-form shifts, free-fermion and
Bethe energies (whole sweep).  The grouped sweep (a schedule of our own, see
TTNRef.sweep_grouped): brute-force bond energies of every level of the
one-pass chains, finite differences of every environment taken from them,
full-chi equality with exact diagonalisation, the fixed point of a converged
state and the variational bound.  Position-resolved matrices and local
energies (rho_positions, local_energies): brute-force one-site matrices,
one-site and bond expectations and block spectra of every node, the averaged
descent, the energy of the state, and a product state in closed form.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla


# --------------------------------------------------------------------------
# shapes and the shift
# --------------------------------------------------------------------------
def num_levels(L: int) -> int:
    """n with L = 2**n; the tree has levels 0..n-1 and isometry layers 1..n-1."""
    n = int(round(math.log2(L)))
    if 2 ** n != L or n < 2:
        raise ValueError("L must be a power of two >= 4")
    return n


def bond_dims(L: int, d: int, chi: int):
    """[chi_0, ..., chi_{n-1}] with chi_0 = d, chi_tau = min(chi_{tau-1}^2, chi)."""
    n = num_levels(L)
    dims = [d]
    for _ in range(1, n):
        dims.append(min(dims[-1] ** 2, chi))
    return dims


def layer_shapes(L: int, d: int, chi: int):
    """[(a, b)] for layers tau = 1..n-1 (a = chi_tau, b = chi_{tau-1})."""
    dims = bond_dims(L, d, chi)
    return [(dims[t], dims[t - 1]) for t in range(1, len(dims))]


def bond_term(h1, A, B):
    """Two-site term b = 1/2 (h1 x I + I x h1) + sum_k A_k x B_k (d^2 x d^2).

    The one-site term is split evenly between the two bonds that touch a
    site, as in Eqs. (2)-(5) of the paper (factor 1/2 against double
    counting in Eq. (H1D)).
    """
    d = h1.shape[0]
    I = np.eye(d)
    b = 0.5 * (np.kron(h1, I) + np.kron(I, h1))
    for a_k, b_k in zip(A, B):
        b = b + np.kron(a_k, b_k)
    return b


def shift_constant(h1, A, B) -> float:
    """c = largest eigenvalue of the bond term, so that every b - c <= 0."""
    return float(np.linalg.eigvalsh(bond_term(h1, A, B))[-1])


# --------------------------------------------------------------------------
# building blocks (Fig. 4(b): each is one matrix product after flattening)
# --------------------------------------------------------------------------
def apply_r(O, w):
    return np.einsum("xy,aly->alx", O, w, optimize=True)


def apply_l(O, w):
    return np.einsum("xy,ayr->axr", O, w, optimize=True)


def left_mul(X, P):
    return np.einsum("ab,blr->alr", X, P, optimize=True)


def close(P, Q):
    return np.einsum("alr,blr->ab", P, Q, optimize=True)


def close_l(P, Q):
    return np.einsum("alr,amr->lm", P, Q, optimize=True)


def close_r(P, Q):
    return np.einsum("alr,als->rs", P, Q, optimize=True)


def pair(X, Y) -> float:
    return float(np.sum(X * Y))


# --------------------------------------------------------------------------
# ascending the Hamiltonian (Fig. 3: w w^T pairs outside the cone drop out)
# --------------------------------------------------------------------------
def s_apply(w, h, A, B):
    """(h x I + I x h + sum_k A_k x B_k) applied to the two input legs of w.

    The left child carries A_k and the right child B_k of the internal bond
    (site j+1 of A_{k,j} B_{k,j+1} is the right one).
    """
    out = apply_l(h, w) + apply_r(h, w)
    for a_k, b_k in zip(A, B):
        out = out + apply_l(a_k, apply_r(b_k, w))
    return out


def ascend(w, h, A, B):
    """Level-tau operators from level tau-1 through the layer isometry w.

    One-site term: internal bond plus both one-site terms, h' = w S w^T.
    Product terms across the boundary between two parents: A acts on the
    right child of parent j, B on the left child of parent j+1, so
    A'_k = w (I x A_k) w^T and B'_k = w (B_k x I) w^T.
    """
    h_new = close(w, s_apply(w, h, A, B))
    A_new = [close(w, apply_r(a_k, w)) for a_k in A]
    B_new = [close(w, apply_l(b_k, w)) for b_k in B]
    return h_new, A_new, B_new


def ascend_all(ws, h0, A0, B0):
    """Operators at every level 0..n-1 (ws[tau-1] is the isometry of layer tau)."""
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
    """H_top v for the two sites of level n-1 with both periodic bonds.

    Sites: v[alpha, beta], alpha the left half.  H_top = h x I + I x h
    + sum_k (A_k x B_k + B_k x A_k).
    """
    out = h @ v + v @ h.T
    for a_k, b_k in zip(A, B):
        out = out + a_k @ v @ b_k.T + b_k @ v @ a_k.T
    return out


def top_matrix(h, A, B):
    """Dense H_top acting on v flattened row-major (only for small chi)."""
    x = h.shape[0]
    I = np.eye(x)
    H = np.kron(h, I) + np.kron(I, h)
    for a_k, b_k in zip(A, B):
        H = H + np.kron(a_k, b_k) + np.kron(b_k, a_k)
    return H


def fix_sign(vec):
    """Sign such that the entry of largest magnitude is positive (first on ties)."""
    flat = vec.reshape(-1)
    i = int(np.argmax(np.abs(flat)))
    return vec if flat[i] >= 0 else -vec


def top_eigen(h, A, B, v0=None, dense_limit=1024, tol=1e-14):
    """Lowest eigenpair (lambda, v) of H_top, v of unit norm and sign-fixed."""
    x = h.shape[0]
    dim = x * x
    if dim <= dense_limit:
        evals, evecs = np.linalg.eigh(top_matrix(h, A, B))
        lam = float(evals[0])
        v = evecs[:, 0].reshape(x, x)
    else:
        op = spla.LinearOperator(
            (dim, dim), dtype=np.float64,
            matvec=lambda y: top_matvec(y.reshape(x, x), h, A, B).reshape(-1))
        start = None if v0 is None else v0.reshape(-1)
        evals, evecs = spla.eigsh(op, k=1, which="SA", v0=start, tol=tol,
                                  ncv=min(dim, 64), maxiter=100000)
        lam = float(evals[0])
        v = evecs[:, 0].reshape(x, x)
    v = v / np.linalg.norm(v)
    return lam, fix_sign(v)


# --------------------------------------------------------------------------
# descending reduced density matrices
# --------------------------------------------------------------------------
def rho_top(v):
    """Position-averaged one-site RDM of level n-1: 1/2 (v v^T + v^T v)."""
    return 0.5 * (v @ v.T + v.T @ v)


def descend_rho(w, rho):
    """Position-averaged one-site RDM one level down through w.

    Each site of the lower level is either the left or the right child of
    exactly one parent, hence the average of the two partial traces.
    """
    P = left_mul(rho, w)
    return 0.5 * (close_l(w, P) + close_r(w, P))


def descend_rho_all(ws, v):
    """rhos[tau] for tau = 0..n-1 from the top down."""
    n = len(ws) + 1
    rhos = [None] * n
    rhos[n - 1] = rho_top(v)
    for tau in range(n - 1, 0, -1):
        rhos[tau - 1] = descend_rho(ws[tau - 1], rhos[tau])
    return rhos


def dressed_top(v, A_top, B_top):
    """Two-site information at level n-1 for every product term k.

    Rbar_k is the A_k-dressed RDM seen from the B site, so that the bond
    energy sum_j <A_{k,j} B_{k,j+1}> = L_tau <Rbar_k, B_k>; Lbar_k is the
    B_k-dressed RDM seen from the A site (<Lbar_k, A_k> gives the same sum).
    The two bonds of the top pair are (1,2) and (2,1).
    """
    R = [0.5 * (v.T @ a @ v + v @ a @ v.T) for a in A_top]
    Lb = [0.5 * (v @ b @ v.T + v.T @ b @ v) for b in B_top]
    return R, Lb


def descend_dressed(w, rho, R, Lb, A_low, B_low):
    """Rbar, Lbar one level down through w (level sigma -> sigma-1).

    Half of the bonds of the lower level lie inside a parent (A on the left
    child, B on the right child, weighted by rho of the parent level); the
    other half cross from the right child of one parent to the left child of
    the next (carried by Rbar/Lbar of the parent level).
    """
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
    """Rbar^(tau), Lbar^(tau) for the current tensors.

    A_low, B_low are the product terms at level tau-1 (ascended with the
    current layers below).  They are carried up through layers tau..n-1
    with the current isometries, the top dressing is formed from v and the
    result is descended back to level tau.
    """
    n = len(ws) + 1
    At = {tau - 1: list(A_low)}
    Bt = {tau - 1: list(B_low)}
    for sigma in range(tau, n):
        w = ws[sigma - 1]
        At[sigma] = [close(w, apply_r(a, w)) for a in At[sigma - 1]]
        Bt[sigma] = [close(w, apply_l(b, w)) for b in Bt[sigma - 1]]
    R, Lb = dressed_top(v, At[n - 1], Bt[n - 1])
    for sigma in range(n - 1, tau, -1):
        R, Lb = descend_dressed(ws[sigma - 1], rhos[sigma], R, Lb,
                                At[sigma - 1], Bt[sigma - 1])
    return R, Lb


def dressed_all(ws, v, rhos, As, Bs):
    """Rbar^(tau), Lbar^(tau) for every level tau = 1..n-1 in one pass.

    For a state whose operators As, Bs (levels 0..n-1) are all ascended with
    the current isometries.  The chain of dressed_chain for level tau carries
    A^(tau-1), B^(tau-1) up through the layers above; when no layer changes
    in between, the carried operators are the ascended ones, As[sigma] and
    Bs[sigma], so the descents for all levels are one recursion from the top
    and a single pass yields every level.  Returns two lists indexed by level
    (entry 0 unused).
    """
    n = len(ws) + 1
    Rs, Ls = [None] * n, [None] * n
    R, Lb = dressed_top(v, As[n - 1], Bs[n - 1])
    Rs[n - 1], Ls[n - 1] = R, Lb
    for sigma in range(n - 1, 1, -1):
        R, Lb = descend_dressed(ws[sigma - 1], rhos[sigma], R, Lb, As[sigma - 1], Bs[sigma - 1])
        Rs[sigma - 1], Ls[sigma - 1] = R, Lb
    return Rs, Ls


def layer_groups(n, groups):
    """Layers 1..n-1 in the groups of the grouped sweep: one group of every
    layer (groups = 1), or the odd layers and then the even ones (groups = 2,
    so that no two neighbouring layers take their environments from the same
    state)."""
    layers = list(range(1, n))
    if groups == 1:
        return [layers]
    if groups == 2:
        return [[t for t in layers if t % 2 == 1], [t for t in layers if t % 2 == 0]]
    raise ValueError("groups must be 1 or 2")


# --------------------------------------------------------------------------
# environment, update, energy
# --------------------------------------------------------------------------
def environment(w, h, A, B, rho, R, Lb):
    """Env of the layer isometry w (same index shape as w).

    Env = rho o (S w) + sum_k Rbar_k o (B_k .l w) + sum_k Lbar_k o (A_k .r w)
    with h, A, B at the level below w and rho, Rbar, Lbar at w's level.
    """
    E = left_mul(rho, s_apply(w, h, A, B))
    for a_k, b_k, r_k, l_k in zip(A, B, R, Lb):
        E = E + left_mul(r_k, apply_l(b_k, w)) + left_mul(l_k, apply_r(a_k, w))
    return E


def polar_update(env):
    """w = -U V^T from the thin SVD of Env (a x b*b), LAPACK gesdd."""
    a = env.shape[0]
    U, s, Vt = np.linalg.svd(env.reshape(a, -1), full_matrices=False)
    return -(U @ Vt).reshape(env.shape), s


def polar_update_evd(env):
    """The eigenvalue-decomposition variant of the update (appendix,
    Fig. 10(b)), in w's index shape: G = Env Env^T = U S^2 U^T (a x a,
    LAPACK syevd) and w = -U S^-1 U^T Env.  The same factor as polar_update
    in exact arithmetic; squaring Env costs half of the precision (relative
    errors of order eps (s_max / s_min)^2)."""
    a = env.shape[0]
    E = env.reshape(a, -1)
    s2, U = np.linalg.eigh(E @ E.T)
    s = np.sqrt(s2)
    w = -(U @ np.diag(1.0 / s) @ U.T @ E)
    return w.reshape(env.shape), s[::-1]


def level_energy(L, tau, h, B, rho, R, c):
    """E = L_tau [<rho, h> + sum_k <Rbar_k, B_k>] + c L at level tau."""
    L_tau = L >> tau
    e = pair(rho, h) + sum(pair(r, b) for r, b in zip(R, B))
    return L_tau * e + c * L


def ortho_error(w):
    W = w.reshape(w.shape[0], -1)
    return float(np.linalg.norm(W @ W.T - np.eye(W.shape[0])))


# --------------------------------------------------------------------------
# entanglement of a block of sites (Sec. V, "Ground state entanglement")
# --------------------------------------------------------------------------
def rho_leftmost(ws, v, tau):
    """Reduced density matrix on the upper bond index of the leftmost
    isometry of layer tau (the block of the first 2**tau sites; tau = 0: the
    first site).  At level n-1 the left site of v: v v^T; one level down the
    leftmost block is the left child of the leftmost block above, so the
    right child is traced out: C_L(w, rho o w)."""
    n = len(ws) + 1
    rho = v @ v.T
    for sigma in range(n - 1, tau, -1):
        w = ws[sigma - 1]
        rho = close_l(w, left_mul(rho, w))
    return rho


def rho_average(ws, v, tau):
    """Position average of the reduced density matrices on the upper bond
    indices of layer tau (the same as descend_rho_all)."""
    return descend_rho_all(ws, v)[tau]


def entanglement(rho):
    """Spectrum p (descending) of a reduced density matrix, the entanglement
    spectrum lambda = -log2 p and the entanglement entropy
    S = -sum p log2 p (Sec. V), terms with p <= 0 counted as zero (inf in
    lambda)."""
    p = np.sort(np.linalg.eigvalsh(0.5 * (rho + rho.T)))[::-1]
    pos = p > 0
    lam = np.full(p.shape, np.inf)
    lam[pos] = -np.log2(p[pos])
    S = float(-np.sum(p[pos] * np.log2(p[pos])))
    return p, lam, S


# --------------------------------------------------------------------------
# position-resolved reduced density matrices and local energies (the same
# state read node by node instead of averaged over positions)
# --------------------------------------------------------------------------
def rho_positions(ws, v):
    """Reduced density matrix on the upper bond of every node of every level.

    rhos[tau][m] belongs to node m of level tau: the block of sites
    m 2**tau .. (m+1) 2**tau - 1 (tau = 0: site m).  Level n-1 holds the two
    halves of v: v v^T (left) and v^T v (right).  One level down node 2m is
    the left child of node m (its right sibling traced out,
    C_L(w, rho o w)) and node 2m+1 the right child (C_R(w, rho o w)).  The
    position average of rhos[tau] is the averaged matrix of descend_rho_all.
    """
    n = len(ws) + 1
    rhos = [None] * n
    rhos[n - 1] = np.stack([v @ v.T, v.T @ v])
    for tau in range(n - 1, 0, -1):
        w = ws[tau - 1]
        b = w.shape[1]
        out = np.empty((2 * rhos[tau].shape[0], b, b))
        for m in range(rhos[tau].shape[0]):
            P = left_mul(rhos[tau][m], w)
            out[2 * m] = close_l(w, P)
            out[2 * m + 1] = close_r(w, P)
        rhos[tau - 1] = out
    return rhos


def bond_site(tau, m):
    """Left site j of the bond (j, j+1) whose two sites first meet under node m
    of level tau >= 1: the last site of its left child."""
    return m * (1 << tau) + (1 << (tau - 1)) - 1


def local_energies(ws, v, h1, A, B):
    """Expectation of every one-site term and of every bond of the chain.

    site[j] = <h1_j>, bond[j] = sum_k <A_{k,j} B_{k,j+1}> (site L is site 0),
    for the unshifted Hamiltonian.  Sites: <rho^(0,j), h1>.  A bond whose two
    sites meet under node m of level tau (bond_site): with A^(tau-1) and
    B^(tau-1) the operators that A on the last site and B on the first site of
    a level tau-1 block become (ascend_all), its expectation is
    <rho^(tau,m), w (A^(tau-1) x B^(tau-1)) w^T>.  The two bonds between the
    halves of v: the middle one <v, A v B^T> and the periodic one
    <v, B v A^T>, with the level n-1 operators.  sum(site) + sum(bond) is the
    energy of the state.
    """
    n = len(ws) + 1
    L = 1 << n
    h1 = np.asarray(h1, dtype=np.float64)
    _, As, Bs = ascend_all(ws, h1, list(A), list(B))
    rhos = rho_positions(ws, v)
    site = np.array([pair(r, h1) for r in rhos[0]])
    bond = np.full(L, np.nan)
    for tau in range(1, n):
        w = ws[tau - 1]
        op = sum((close(w, apply_l(a_k, apply_r(b_k, w))) for a_k, b_k in zip(As[tau - 1], Bs[tau - 1])),
                 np.zeros((w.shape[0], w.shape[0])))
        for m in range(L >> tau):
            bond[bond_site(tau, m)] = pair(rhos[tau][m], op)
    top = n - 1
    bond[L // 2 - 1] = sum((pair(v, a_k @ v @ b_k.T) for a_k, b_k in zip(As[top], Bs[top])), 0.0)
    bond[L - 1] = sum((pair(v, b_k @ v @ a_k.T) for a_k, b_k in zip(As[top], Bs[top])), 0.0)
    return site, bond, rhos


# --------------------------------------------------------------------------
# the sweep
# --------------------------------------------------------------------------
class TTNRef:
    """State of a uniform binary TTN and the bottom-up sweep of Sec. III."""

    def __init__(self, L, chi, h1, A, B, ly=1, ws=None, shift=None):
        self.L = int(L)
        self.n = num_levels(L)
        self.h1 = np.asarray(h1, dtype=np.float64)
        self.A0 = [np.asarray(a, dtype=np.float64) for a in A]
        self.B0 = [np.asarray(b, dtype=np.float64) for b in B]
        self.d = self.h1.shape[0]
        self.D = len(self.A0)
        self.ly = ly
        self.dims = bond_dims(L, self.d, chi)
        self.c = shift_constant(self.h1, self.A0, self.B0) if shift is None else float(shift)
        self.h0 = self.h1 - self.c * np.eye(self.d)
        if ws is None:
            raise ValueError("initial isometries are an input (see inputs.random_isometries)")
        self.ws = [np.array(w, dtype=np.float64) for w in ws]
        for t, w in enumerate(self.ws, start=1):
            if w.shape != (self.dims[t], self.dims[t - 1], self.dims[t - 1]):
                raise ValueError(f"layer {t}: shape {w.shape}")
        self.v = None
        self.lam = None
        self.history = []
        self.diag = []

    # energies -------------------------------------------------------------
    def energy_total(self):
        return self.lam + self.c * self.L

    def energy_per_site(self):
        return self.energy_total() / (self.L * self.ly)

    # initial state (ascend everything, solve the top) -----------------------
    def initialise(self):
        self.hs, self.As, self.Bs = ascend_all(self.ws, self.h0, self.A0, self.B0)
        top = self.n - 1
        self.lam, self.v = top_eigen(self.hs[top], self.As[top], self.Bs[top])
        self.history.append(self.energy_per_site())
        return self.energy_per_site()

    def sweep(self):
        """One bottom-up sweep; returns the energy per site after it."""
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
        self.lam, self.v = top_eigen(self.hs[top], self.As[top], self.Bs[top], v0=self.v)
        self.history.append(self.energy_per_site())
        self.diag.append(info)
        return self.energy_per_site()

    def sweep_grouped(self, groups):
        """One sweep in which every layer of a group takes its environment
        from the same state (a schedule of our own, not the paper's: the
        dressed chains of a group come from one pass, dressed_all, instead of
        one chain per layer).  Per group: descend rho, one pass of the dressed
        chains, the environment and the polar update of every layer of the
        group, then ascend every layer; after the last group the top tensor.
        Returns the energy per site after it."""
        n = self.n
        info = {"ortho": [], "sigma_ratio": []}
        for members in layer_groups(n, groups):
            if not members:
                continue
            rhos = descend_rho_all(self.ws, self.v)
            Rs, Ls = dressed_all(self.ws, self.v, rhos, self.As, self.Bs)
            new = list(self.ws)
            for tau in members:
                w = self.ws[tau - 1]
                env = environment(w, self.hs[tau - 1], self.As[tau - 1], self.Bs[tau - 1], rhos[tau],
                                  Rs[tau], Ls[tau])
                new[tau - 1], s = polar_update(env)
                info["ortho"].append(ortho_error(new[tau - 1]))
                info["sigma_ratio"].append(float(s[-1] / s[0]) if s[0] > 0 else 0.0)
            self.ws = new
            self.hs, self.As, self.Bs = ascend_all(self.ws, self.h0, self.A0, self.B0)
        top = n - 1
        self.lam, self.v = top_eigen(self.hs[top], self.As[top], self.Bs[top], v0=self.v)
        self.history.append(self.energy_per_site())
        self.diag.append(info)
        return self.energy_per_site()

    def run(self, sweeps, tol=None):
        """Sweep up to ``sweeps`` times; with ``tol`` stop when |de| < tol."""
        if self.v is None:
            self.initialise()
        for _ in range(sweeps):
            before = self.history[-1]
            after = self.sweep()
            if tol is not None and abs(after - before) < tol:
                break
        return list(self.history)
