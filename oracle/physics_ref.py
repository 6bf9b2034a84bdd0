"""Exact references used to pin ``ttn_ref`` (TEST INFRASTRUCTURE).

* Physical Hamiltonians built spin by spin from their textbook definitions
  (not from the effective-chain matrices the TTN consumes), as sparse
  matrices, and their ground energies by sparse Lanczos (scipy eigsh).
* Closed forms: the free-fermion ground energy of the periodic
  transverse-field Ising chain (Pfeuty 1970) and the Bethe-ansatz energy
  density of the Heisenberg chain (Hulthen 1938).
* Brute-force contraction of a TTN into its full state vector, and exact
  expectation values / reduced density matrices from it.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_X = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
_Z = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, -1.0]]))
_Y_IM = sp.csr_matrix(np.array([[0.0, -1.0], [1.0, 0.0]]))  # sigma^y / i
_Y = sp.csr_matrix(np.array([[0.0, -1.0j], [1.0j, 0.0]]))  # sigma^y (complex)


def _site_op(op, i, n_spins):
    """Operator on spin i of n_spins (spin 0 = most significant bit)."""
    left = sp.identity(2 ** i, format="csr")
    right = sp.identity(2 ** (n_spins - i - 1), format="csr")
    return sp.kron(sp.kron(left, op, format="csr"), right, format="csr")


def tfim_chain_hamiltonian(L, h, J=1.0):
    """H = -J sum_i Z_i Z_{i+1} - h sum_i X_i on a periodic chain (sparse)."""
    H = sp.csr_matrix((2 ** L, 2 ** L))
    for i in range(L):
        j = (i + 1) % L
        H = H - J * (_site_op(_Z, i, L) @ _site_op(_Z, j, L))
        H = H - h * _site_op(_X, i, L)
    return H.tocsr()


def heisenberg_chain_hamiltonian(L):
    """H = sum_i S_i . S_{i+1}, S = sigma / 2, periodic chain (sparse, real).

    S^y S^y = -(sigma^y/i)(sigma^y/i)/4 keeps everything real.
    """
    H = sp.csr_matrix((2 ** L, 2 ** L))
    for i in range(L):
        j = (i + 1) % L
        H = H + 0.25 * (_site_op(_X, i, L) @ _site_op(_X, j, L))
        H = H - 0.25 * (_site_op(_Y_IM, i, L) @ _site_op(_Y_IM, j, L))
        H = H + 0.25 * (_site_op(_Z, i, L) @ _site_op(_Z, j, L))
    return H.tocsr()


def xxz_chain_hamiltonian(L, J, Delta, hz=0.0):
    """H = sum_i [J (Sx Sx + Sy Sy) + Delta Sz Sz + hz Sz_i], S = sigma / 2,
    periodic chain (sparse, real: Sy Sy = -(sigma^y/i)(sigma^y/i)/4)."""
    H = sp.csr_matrix((2 ** L, 2 ** L))
    for i in range(L):
        j = (i + 1) % L
        H = H + 0.25 * J * (_site_op(_X, i, L) @ _site_op(_X, j, L))
        H = H - 0.25 * J * (_site_op(_Y_IM, i, L) @ _site_op(_Y_IM, j, L))
        H = H + 0.25 * Delta * (_site_op(_Z, i, L) @ _site_op(_Z, j, L))
        H = H + 0.5 * hz * _site_op(_Z, i, L)
    return H.tocsr()


def dm_xxz_chain_hamiltonian(L, J, Dm, Delta, hz=0.0):
    """H = sum_i [J (Sx Sx + Sy Sy) + Delta Sz Sz + Dm (Sx_i Sy_{i+1} -
    Sy_i Sx_{i+1}) + hz Sz_i], S = sigma / 2, periodic chain, built spin by
    spin with the complex sigma^y (sparse, complex Hermitian)."""
    H = sp.csr_matrix((2 ** L, 2 ** L), dtype=np.complex128)
    for i in range(L):
        j = (i + 1) % L
        xi, xj = _site_op(_X, i, L), _site_op(_X, j, L)
        yi, yj = _site_op(_Y, i, L), _site_op(_Y, j, L)
        H = H + 0.25 * J * (xi @ xj + yi @ yj)
        H = H + 0.25 * Delta * (_site_op(_Z, i, L) @ _site_op(_Z, j, L))
        H = H + 0.25 * Dm * (xi @ yj - yi @ xj)
        H = H + 0.5 * hz * _site_op(_Z, i, L)
    return H.tocsr()


def torus_tfim_hamiltonian(Lx, Ly, h):
    """Eq. (H2D): sum_{m,n} (-X_{m,n} X_{m+1,n} - X_{m,n} X_{m,n+1} + h Z_{m,n}).

    Periodic in both directions.  Spin (m, n) (0-based) is bit m*Ly + n of
    the basis index counted from the most significant bit, i.e. column m
    occupies one contiguous block of Ly bits with its n = 0 spin first.
    """
    N = Lx * Ly
    idx = lambda m, n: (m % Lx) * Ly + (n % Ly)
    H = sp.csr_matrix((2 ** N, 2 ** N))
    for m in range(Lx):
        for n in range(Ly):
            H = H - _site_op(_X, idx(m, n), N) @ _site_op(_X, idx(m + 1, n), N)
            H = H - _site_op(_X, idx(m, n), N) @ _site_op(_X, idx(m, n + 1), N)
            H = H + h * _site_op(_Z, idx(m, n), N)
    return H.tocsr()


def ground_energy(H):
    """Lowest eigenvalue of a sparse symmetric (or complex Hermitian) matrix
    (scipy Lanczos)."""
    if H.shape[0] <= 512:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    vals = spla.eigsh(H, k=1, which="SA", tol=1e-14, return_eigenvectors=False)
    return float(vals[0])


def tfim_free_fermion_energy(L, h, J=1.0):
    """Ground energy of the periodic TFIM chain, -J sum Z Z - h sum X.

    Jordan-Wigner fermions in the even-parity sector take antiperiodic
    momenta k = pi (2m+1) / L, each mode contributing
    -sqrt(J^2 + h^2 - 2 J h cos k); the sum over all L modes is the ground
    energy (Pfeuty, Ann. Phys. 57, 79 (1970)).
    """
    m = np.arange(L)
    k = np.pi * (2 * m + 1) / L
    return float(-np.sum(np.sqrt(J * J + h * h - 2 * J * h * np.cos(k))))


def tfim_critical_energy(L):
    """h = J = 1 special case of the free-fermion sum: -2 / sin(pi / (2L))."""
    return -2.0 / math.sin(math.pi / (2 * L))


def xx_chain_free_fermion_energy(L, J=1.0):
    """Ground energy of the periodic XX chain J sum (Sx Sx + Sy Sy), S = sigma/2.

    Jordan-Wigner: (J/2) sum_j (c_j^+ c_{j+1} + h.c.) with one-particle
    energies J cos k; with N particles the boundary bond is periodic for odd N
    (k = 2 pi m / L) and antiperiodic for even N (k = 2 pi (m + 1/2) / L).
    The ground energy is the least over N of the N lowest energies' sum
    (Lieb, Schultz and Mattis, Ann. Phys. 16, 407 (1961))."""
    m = np.arange(L)
    per = np.sort(J * np.cos(2 * np.pi * m / L))
    anti = np.sort(J * np.cos(2 * np.pi * (m + 0.5) / L))
    best = 0.0
    for N in range(1, L + 1):
        e = (per if N % 2 == 1 else anti)[:N].sum()
        best = min(best, float(e))
    return best


BETHE_XXX_ENERGY_DENSITY = 0.25 - math.log(2.0)  # Hulthen: 1/4 - ln 2


# --------------------------------------------------------------------------
# brute-force contraction of a uniform binary TTN
# --------------------------------------------------------------------------
def level_state(ws, v, level):
    """State on the L_level sites of a given level, as an array with one
    index per site (site order left to right), contracted from the top.

    ws[tau-1] is the isometry of layer tau; a site index x of level tau is
    expanded into its two children with w[x; l, r].
    """
    n = len(ws) + 1
    psi = np.array(v)  # level n-1: two sites
    for tau in range(n - 1, level, -1):
        w = ws[tau - 1]
        k = psi.ndim
        # replace every index by the two children (l, r)
        for pos in range(k):
            # index at position 2*pos after previous expansions
            axis = 2 * pos
            psi = np.tensordot(psi, w, axes=([axis], [0]))  # appends (l, r) at the end
            psi = np.moveaxis(psi, [-2, -1], [axis, axis + 1])
    return psi


def full_state(ws, v):
    """Flattened state on all L sites (only for tiny systems)."""
    return level_state(ws, v, 0).reshape(-1)


def one_site_rdm_average(psi_sites):
    """Position average of the one-site reduced density matrices of a state
    given with one index per site."""
    k = psi_sites.ndim
    acc = 0.0
    for j in range(k):
        other = [i for i in range(k) if i != j]
        acc = acc + np.tensordot(psi_sites, psi_sites, axes=(other, other))
    return acc / k


def bond_expectation_sum(psi_sites, A, B):
    """sum_j <A_j B_{j+1}> (periodic) for one product term, brute force."""
    k = psi_sites.ndim
    total = 0.0
    for j in range(k):
        jn = (j + 1) % k
        phi = np.moveaxis(np.tensordot(A, psi_sites, axes=([1], [j])), 0, j)
        phi = np.moveaxis(np.tensordot(B, phi, axes=([1], [jn])), 0, jn)
        total += float(np.sum(psi_sites * phi))
    return total


def chain_operator_expectation(psi_sites, h, A, B):
    """<psi| sum_j [h_j + sum_k A_{k,j} B_{k,j+1}] |psi> (periodic), brute force."""
    k = psi_sites.ndim
    total = 0.0
    for j in range(k):
        phi = np.moveaxis(np.tensordot(h, psi_sites, axes=([1], [j])), 0, j)
        total += float(np.sum(psi_sites * phi))
    for a_k, b_k in zip(A, B):
        total += bond_expectation_sum(psi_sites, a_k, b_k)
    return total


def site_expectations(psi_sites, h):
    """<h_j> for every site j, brute force."""
    out = []
    for j in range(psi_sites.ndim):
        phi = np.moveaxis(np.tensordot(h, psi_sites, axes=([1], [j])), 0, j)
        out.append(float(np.sum(psi_sites * phi)))
    return np.array(out)


def bond_expectations(psi_sites, A, B):
    """sum_k <A_{k,j} B_{k,j+1}> for every j (periodic), brute force."""
    k = psi_sites.ndim
    out = np.zeros(k)
    for a_k, b_k in zip(A, B):
        for j in range(k):
            jn = (j + 1) % k
            phi = np.moveaxis(np.tensordot(a_k, psi_sites, axes=([1], [j])), 0, j)
            phi = np.moveaxis(np.tensordot(b_k, phi, axes=([1], [jn])), 0, jn)
            out[j] += float(np.sum(psi_sites * phi))
    return out


def one_site_rdm(psi_sites, j):
    """Reduced density matrix of site j, brute force."""
    other = [i for i in range(psi_sites.ndim) if i != j]
    return np.tensordot(psi_sites, psi_sites, axes=(other, other))



# --------------------------------------------------------------------------
# complex states (one index per site): expectations with the bra conjugated
# --------------------------------------------------------------------------
def complex_chain_expectation(psi_sites, h, A, B):
    """<psi| sum_j [h_j + sum_k A_{k,j} B_{k,j+1}] |psi> (periodic), complex
    state, brute force; the real part (the operator is Hermitian)."""
    k = psi_sites.ndim
    total = 0.0 + 0.0j
    for j in range(k):
        phi = np.moveaxis(np.tensordot(h, psi_sites, axes=([1], [j])), 0, j)
        total += np.vdot(psi_sites, phi)
    for a_k, b_k in zip(A, B):
        for j in range(k):
            jn = (j + 1) % k
            phi = np.moveaxis(np.tensordot(a_k, psi_sites, axes=([1], [j])), 0, j)
            phi = np.moveaxis(np.tensordot(b_k, phi, axes=([1], [jn])), 0, jn)
            total += np.vdot(psi_sites, phi)
    return float(total.real)


def complex_bond_expectations(psi_sites, A, B):
    """sum_k <A_{k,j} B_{k,j+1}> for every j (periodic), complex state."""
    k = psi_sites.ndim
    out = np.zeros(k, dtype=np.complex128)
    for a_k, b_k in zip(A, B):
        for j in range(k):
            jn = (j + 1) % k
            phi = np.moveaxis(np.tensordot(a_k, psi_sites, axes=([1], [j])), 0, j)
            phi = np.moveaxis(np.tensordot(b_k, phi, axes=([1], [jn])), 0, jn)
            out[j] += np.vdot(psi_sites, phi)
    return out


def pairing_matrix_average(psi_sites):
    """Position average of M_j[x, x'] = sum conj(psi[.. x ..]) psi[.. x' ..]
    over the other sites: the transpose of site j's density matrix, which
    pairs with an operator element by element, <O_j> = sum M_j * O."""
    k = psi_sites.ndim
    acc = 0.0
    for j in range(k):
        other = [i for i in range(k) if i != j]
        acc = acc + np.tensordot(psi_sites.conj(), psi_sites, axes=(other, other))
    return acc / k
