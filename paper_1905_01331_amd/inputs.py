"""Seeded synthetic inputs shared by the GPU path and the CPU checker.

This module holds no arithmetic of the TTN sweep itself.  It only produces
the inputs a run starts from:

* the one-site term ``h1`` and the product terms ``(A_k, B_k)`` of an
  effective chain ``H = sum_j [ h1_j + sum_k A_{k,j} B_{k,j+1} ]`` for the
  three model families used by the workloads (transverse-field Ising chain,
  2D transverse-field Ising model on a thin torus with one column per
  effective site, spin-1/2 Heisenberg XXX chain);
* seeded random isometries (Gaussian draw, reduced QR, sign-fixed) for a list
  of layer shapes;
* the seeded draw of the batched workload (many independent chains);
* a chain with complex product terms (the chiral XXZ chain) and seeded
  complex isometries and top tensors for it.

All matrices are row-major, ket index first; real float64 except those of
the complex chain (complex128).
"""
from __future__ import annotations

import numpy as np

# Pauli matrices (paper Sec. II.A, below Eq. (H2D)).
PAULI_X = np.array([[0.0, 1.0], [1.0, 0.0]])
PAULI_Z = np.array([[1.0, 0.0], [0.0, -1.0]])
# i*sigma^y is real and antisymmetric: i * [[0, -i], [i, 0]] = [[0, 1], [-1, 0]].
PAULI_IY = np.array([[0.0, 1.0], [-1.0, 0.0]])
EYE2 = np.eye(2)


class ChainModel:
    """Effective chain ``H = sum_j [h1_j + sum_k A_{k,j} B_{k,j+1}]`` (periodic).

    ``d``: effective site dimension; ``ly``: physical spins per effective site
    (energy per physical spin divides by ``L * ly``).  Each pair (A_k, B_k) is
    either both symmetric or both antisymmetric so every bond term is a
    symmetric operator.
    """

    def __init__(self, name, h1, A, B, ly=1, dtype=np.float64):
        self.name = name
        self.dtype = np.dtype(dtype)
        self.h1 = np.ascontiguousarray(h1, dtype=self.dtype)
        self.A = [np.ascontiguousarray(a, dtype=self.dtype) for a in A]
        self.B = [np.ascontiguousarray(b, dtype=self.dtype) for b in B]
        self.d = self.h1.shape[0]
        self.D = len(self.A)
        self.ly = ly

    def packed(self):
        """(h1, A[D,d,d], B[D,d,d]) as contiguous arrays of the model's dtype."""
        d, D = self.d, self.D
        A = np.stack(self.A) if D else np.zeros((0, d, d), dtype=self.dtype)
        B = np.stack(self.B) if D else np.zeros((0, d, d), dtype=self.dtype)
        return self.h1, np.ascontiguousarray(A), np.ascontiguousarray(B)


def tfim_chain(h: float = 1.0, J: float = 1.0) -> ChainModel:
    """Transverse-field Ising chain ``H = -J sum Z_i Z_{i+1} - h sum X_i``.

    One spin per effective site (d = 2): h1 = -h X, one product term with
    A = Z, B = -J Z.
    """
    return ChainModel(f"tfim(h={h})", -h * PAULI_X, [PAULI_Z], [-J * PAULI_Z], ly=1)


def _spin_op(op, n, ly):
    """Operator ``op`` on spin n (0-based, n = 0 is the most significant bit)."""
    out = np.ones((1, 1))
    for m in range(ly):
        out = np.kron(out, op if m == n else EYE2)
    return out


def torus_tfim_column(ly: int, h: float) -> ChainModel:
    """2D transverse-field Ising model on an Lx x Ly torus, one column per site.

    Follows Eq. (H2D) of the paper (Sec. II.A): ``sum_{m,n} (-X_{m,n} X_{m+1,n}
    - X_{m,n} X_{m,n+1} + h Z_{m,n})`` with periodic n.  A column of ``ly``
    spins is one effective site of dimension 2**ly (Sec. II.B); spin n = 1 of
    the paper is the most significant bit.  The intra-column couplings and
    fields form h1; the horizontal couplings are the ly product terms
    A_k = X_k, B_k = -X_k (the bond index of dimension L_y, Fig. 2(b)).
    Only ly >= 3 is accepted: for ly <= 2 the periodic vertical sum of
    Eq. (H2D) counts a pair more than once.
    """
    if ly < 3:
        raise ValueError("torus column builder needs ly >= 3")
    d = 2 ** ly
    h1 = np.zeros((d, d))
    for n in range(ly):
        h1 -= _spin_op(PAULI_X, n, ly) @ _spin_op(PAULI_X, (n + 1) % ly, ly)
        h1 += h * _spin_op(PAULI_Z, n, ly)
    A = [_spin_op(PAULI_X, n, ly) for n in range(ly)]
    B = [-_spin_op(PAULI_X, n, ly) for n in range(ly)]
    return ChainModel(f"torus_tfim(ly={ly},h={h})", h1, A, B, ly=ly)


def xxx_chain() -> ChainModel:
    """Spin-1/2 Heisenberg chain ``H = sum_i S_i . S_{i+1}`` with S = sigma/2.

    Sy Sy is written with the real antisymmetric pair (iSy, -iSy), since
    (iSy) x (-iSy) = Sy x Sy.
    """
    sx = 0.5 * PAULI_X
    sz = 0.5 * PAULI_Z
    isy = 0.5 * PAULI_IY
    return ChainModel("xxx", np.zeros((2, 2)), [sx, isy, sz], [sx, -isy, sz], ly=1)


def dm_chain(J: float = 1.0, Dm: float = 1.0, Delta: float = 1.0, hz: float = 0.0,
             form: str = "hermitian") -> ChainModel:
    """Spin-1/2 XXZ chain with a Dzyaloshinskii-Moriya term along z (complex):
    ``H = sum_i [J (Sx_i Sx_{i+1} + Sy_i Sy_{i+1}) + Delta Sz_i Sz_{i+1}
    + Dm (Sx_i Sy_{i+1} - Sy_i Sx_{i+1}) + hz Sz_i]`` with S = sigma/2 and
    the complex Sy.  The DM term makes the Hamiltonian matrix complex (Sx Sy
    is imaginary).  Two ways of writing it with three product terms:
    form="hermitian": A = (Sx, Sy, Sz), B = (J Sx + Dm Sy, J Sy - Dm Sx,
    Delta Sz), every factor Hermitian; form="ladder": with S+- = Sx +- i Sy,
    A = ((J + i Dm)/2 S+, (J - i Dm)/2 S-, Sz), B = (S-, S+, Delta Sz), whose
    first two terms have factors that are neither Hermitian nor
    anti-Hermitian (their sum is Hermitian)."""
    sx = 0.5 * PAULI_X.astype(np.complex128)
    sy = 0.5 * np.array([[0.0, -1.0j], [1.0j, 0.0]])
    sz = 0.5 * PAULI_Z.astype(np.complex128)
    name = f"dm_xxz(J={J},Dm={Dm},Delta={Delta},hz={hz},{form})"
    if form == "hermitian":
        return ChainModel(name, hz * sz, [sx, sy, sz], [J * sx + Dm * sy, J * sy - Dm * sx, Delta * sz], ly=1,
                          dtype=np.complex128)
    if form == "ladder":
        sp, sm = sx + 1j * sy, sx - 1j * sy
        return ChainModel(name, hz * sz, [0.5 * (J + 1j * Dm) * sp, 0.5 * (J - 1j * Dm) * sm, sz],
                          [sm, sp, Delta * sz], ly=1, dtype=np.complex128)
    raise ValueError("form must be 'hermitian' or 'ladder'")


def random_complex_isometries(shapes, seed: int):
    """Seeded complex isometries for layer shapes [(a, b), ...]: for each layer
    in order a complex Gaussian (b*b x a) matrix G = X + iY (X drawn before Y
    from ``numpy.random.default_rng(seed)``), its reduced QR with the phases of
    diag(R) folded into Q, and w[a; l, r] = Q[(l, r), a]; the rows of w are
    orthonormal in the Hermitian sense, sum_{l,r} w[a; l, r] conj(w[a'; l, r])
    = delta."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in shapes:
        g = rng.standard_normal((b * b, a)) + 1j * rng.standard_normal((b * b, a))
        q, r = np.linalg.qr(g)
        dg = np.diag(r)
        ph = np.where(np.abs(dg) > 0, dg / np.maximum(np.abs(dg), 1e-300), 1.0)
        q = q * ph[None, :]
        out.append(np.ascontiguousarray(q.T.reshape(a, b, b)))
    return out


def random_complex_top(chi: int, seed: int):
    """Seeded random complex top tensor of unit norm (real part drawn first)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((chi, chi)) + 1j * rng.standard_normal((chi, chi))
    return v / np.linalg.norm(v)


def random_isometries(shapes, seed: int):
    """Seeded random isometries for layer shapes [(a, b), ...] (bottom to top).

    For each layer in order a Gaussian matrix G (b*b x a) is drawn from
    ``numpy.random.default_rng(seed)``; its reduced QR G = Q R is taken with
    the sign of diag(R) folded into Q, and w[a; l, r] = Q[(l, r), a].  Rows of
    the returned (a, b, b) arrays are orthonormal.
    """
    rng = np.random.default_rng(seed)
    out = []
    for a, b in shapes:
        g = rng.standard_normal((b * b, a))
        q, r = np.linalg.qr(g)
        s = np.sign(np.diag(r))
        s[s == 0] = 1.0
        q = q * s[None, :]
        out.append(np.ascontiguousarray(q.T.reshape(a, b, b)))
    return out


def random_node_isometries(L: int, d: int, chi: int, seed: int):
    """Seeded random isometries of a position-resolved network: for layer
    tau = 1..n-1 an array (L >> tau, a, b, b), node-major.  For each layer in
    order and each node in order, a Gaussian (b*b x a) matrix from
    ``numpy.random.default_rng(seed)``, its reduced QR with the signs of
    diag(R) folded into Q, w = Q^T (as random_isometries)."""
    rng = np.random.default_rng(seed)
    out = []
    for t, (a, b) in enumerate(layer_shapes(L, d, chi), start=1):
        layer = np.empty((L >> t, a, b, b))
        for m in range(L >> t):
            g = rng.standard_normal((b * b, a))
            q, r = np.linalg.qr(g)
            s = np.sign(np.diag(r))
            s[s == 0] = 1.0
            layer[m] = (q * s[None, :]).T.reshape(a, b, b)
        out.append(layer)
    return out


def uniform_node_isometries(ws, L: int):
    """Position-resolved copies of a uniform network (layer tau of ws repeated
    on its L >> tau nodes): the same state."""
    return [np.repeat(np.asarray(w)[None], L >> t, axis=0) for t, w in enumerate(ws, start=1)]


def layer_shapes(L: int, d: int, chi: int):
    """[(a, b), ...] of layers 1..n-1 (L = 2**n): bond dimensions chi_0 = d,
    chi_tau = min(chi_{tau-1}**2, chi)."""
    n = L.bit_length() - 1
    dims = [d]
    for _ in range(1, n):
        dims.append(min(dims[-1] ** 2, chi))
    return [(dims[t], dims[t - 1]) for t in range(1, n)]


def embed_isometries(ws, shapes, seed: int):
    """Isometries of larger bond dimensions that represent the same state:
    each old w (a, b, b) sits in the corner of the new (a', b', b') (zero
    weight on the added child directions), and the a' - a added rows are a
    seeded orthonormal complement of the old rows.  With the top tensor
    embedded the same way (embed_top) the network is the same state and the
    added directions start with zero weight."""
    rng = np.random.default_rng(seed)
    out = []
    for w, (a2, b2) in zip(ws, shapes):
        a, b = w.shape[0], w.shape[1]
        W = np.zeros((a2, b2, b2))
        W[:a, :b, :b] = w
        if a2 > a:
            M = W[:a].reshape(a, -1)
            g = rng.standard_normal((a2 - a, b2 * b2))
            g -= (g @ M.T) @ M
            g -= (g @ M.T) @ M
            q, r = np.linalg.qr(g.T)
            s = np.sign(np.diag(r))
            s[s == 0] = 1.0
            W[a:] = (q * s[None, :]).T.reshape(a2 - a, b2, b2)
        out.append(W)
    return out


def embed_top(v, x: int):
    """The top tensor in the corner of a larger (x, x) one (same state)."""
    V = np.zeros((x, x))
    V[:v.shape[0], :v.shape[1]] = v
    return V


def random_top(chi: int, seed: int):
    """Seeded random normalised top tensor (chi x chi)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((chi, chi))
    return v / np.linalg.norm(v)


def batched_tfim_draws(count: int = 128, seed: int = 2026):
    """Seeded draw of many independent transverse-field Ising chains.

    In this order: L uniform over {64, 128, 256, 512, 1024}, h uniform on
    [0.5, 1.5], chi uniform over {32, 48, 64, 96}; member i uses init seed
    1000 + i.  Returns a list of dicts (L, h, chi, seed).
    """
    rng = np.random.default_rng(seed)
    Ls = rng.choice(np.array([64, 128, 256, 512, 1024]), size=count)
    hs = rng.uniform(0.5, 1.5, size=count)
    chis = rng.choice(np.array([32, 48, 64, 96]), size=count)
    return [dict(L=int(Ls[i]), h=float(hs[i]), chi=int(chis[i]), seed=1000 + i)
            for i in range(count)]
