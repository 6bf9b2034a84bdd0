"""Pins of the position-resolved TTN reference (oracle/ttn_positional.py):
every node its own isometry.  Each pin is fixed by something other than the
reference itself: brute-force contraction of the network into a state
vector, exact diagonalisation at full bond dimension, finite differences,
and the uniform reference (pinned on its own) for networks whose layers are
copies of one isometry."""
import json
import os

import numpy as np
import pytest

from oracle import physics_ref as P
from oracle import ttn_positional as Q
from oracle import ttn_ref as T
from paper_1905_01331_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ed_energies.json")))

MODELS = [
    ("tfim", I.tfim_chain(0.8), 8, 4),
    ("xxx", I.xxx_chain(), 8, 3),
    ("torus_col3", I.torus_tfim_column(3, 2.0), 4, 6),
]


def make(model, L, chi, seed):
    nws = I.random_node_isometries(L, model.d, chi, seed)
    return Q.PositionalTTN(L, chi, model.h1, model.A, model.B, nws, ly=model.ly)


def brute_energy(r, psi_sites):
    """<psi| H - c L |psi> of a state given one index per site."""
    return P.chain_operator_expectation(psi_sites, r.h0, r.A, r.B)


def block_energy(r, psi_sites, tau, m):
    """<psi| H_blk |psi> for the terms that touch block m of level tau: its
    sites and every bond with at least one end in it.  The other terms meet
    w^(tau, m) only as w w^T = 1 on isometries and take no part in its
    environment."""
    L = r.L
    first, last = m << tau, ((m + 1) << tau) - 1
    site = P.site_expectations(psi_sites, r.h0)[first:last + 1].sum()
    bonds = P.bond_expectations(psi_sites, r.A, r.B)
    touch = {(j - 1) % L for j in range(first, last + 1)} | set(range(first, last + 1))
    return float(site + sum(bonds[j] for j in touch))


@pytest.mark.parametrize("name,model,L,chi", MODELS, ids=[m[0] for m in MODELS])
def test_energy_equals_brute_force_contraction(name, model, L, chi):
    r = make(model, L, chi, seed=3)
    e = r.initialise()
    psi = Q.level_state(r.nws, r.v, 0)
    assert np.linalg.norm(psi) == pytest.approx(1.0, abs=1e-12)
    e_bf = (brute_energy(r, psi) + r.c * L) / (L * model.ly)
    assert e == pytest.approx(e_bf, abs=1e-12)


def test_uniform_copies_reproduce_the_uniform_reference():
    model, L, chi = I.xxx_chain(), 16, 5
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 4)
    ref = T.TTNRef(L, chi, model.h1, model.A, model.B, ws=[w.copy() for w in ws])
    e_u = ref.initialise()
    r = Q.PositionalTTN(L, chi, model.h1, model.A, model.B, I.uniform_node_isometries(ws, L))
    assert r.initialise() == pytest.approx(e_u, abs=1e-12)
    # averaged over the nodes of a level, the node matrices are the uniform
    # reference's position-averaged descent
    hs, As, Bs = r.operators()
    rho, X, Y = Q.descend_all(r.nws, r.v, As, Bs)
    rho_u = T.descend_rho_all(ref.ws, ref.v)
    for tau in range(r.n):
        assert np.abs(np.mean(rho[tau], axis=0) - rho_u[tau]).max() < 1e-13


@pytest.mark.parametrize("name,model,L,chi", MODELS, ids=[m[0] for m in MODELS])
def test_node_matrices_equal_brute_force_block_rdms(name, model, L, chi):
    r = make(model, L, chi, seed=5)
    r.initialise()
    hs, As, Bs = r.operators()
    rho, X, Y = Q.descend_all(r.nws, r.v, As, Bs)
    for tau in range(r.n):
        psi = Q.level_state(r.nws, r.v, tau)
        for m in range(L >> tau):
            assert np.abs(rho[tau][m] - P.one_site_rdm(psi, m)).max() < 1e-13
            assert np.trace(rho[tau][m]) == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("name,model,L,chi", MODELS, ids=[m[0] for m in MODELS])
def test_edge_information_gives_every_bond_energy(name, model, L, chi):
    # <X^(tau,m), B^(tau,m)> is the bond that arrives at the first site of
    # block m, <Y^(tau,m), A^(tau,m)> the bond that leaves its last site
    r = make(model, L, chi, seed=7)
    r.initialise()
    hs, As, Bs = r.operators()
    rho, X, Y = Q.descend_all(r.nws, r.v, As, Bs)
    psi0 = Q.level_state(r.nws, r.v, 0)
    bonds = P.bond_expectations(psi0, r.A, r.B)
    for tau in range(r.n):
        for m in range(L >> tau):
            first, last = m << tau, ((m + 1) << tau) - 1
            left = sum(T.pair(x, b) for x, b in zip(X[tau][m], Bs[tau][m]))
            right = sum(T.pair(y, a) for y, a in zip(Y[tau][m], As[tau][m]))
            assert left == pytest.approx(bonds[(first - 1) % L], abs=1e-12), (tau, m)
            assert right == pytest.approx(bonds[last], abs=1e-12), (tau, m)


@pytest.mark.parametrize("name,model,L,chi", MODELS, ids=[m[0] for m in MODELS])
def test_environment_is_the_derivative_of_the_energy(name, model, L, chi):
    # moving one node's isometry alone: dE/deps = 2 <Env, Delta> for the
    # energy of the terms that touch its block (quadratic in it), from the
    # brute-force state
    r = make(model, L, chi, seed=11)
    r.initialise()
    hs, As, Bs = r.operators()
    rho, X, Y = Q.descend_all(r.nws, r.v, As, Bs)
    rng = np.random.default_rng(2)
    eps = 1e-4
    for tau in range(1, r.n):
        for m in range(L >> tau):
            env = r.node_env(tau, m, hs, As, Bs, rho, X, Y)
            w = r.nws[tau - 1][m]
            Dw = rng.standard_normal(w.shape)
            vals = []
            for sgn in (1, -1):
                r.nws[tau - 1][m] = w + sgn * eps * Dw
                vals.append(block_energy(r, Q.level_state(r.nws, r.v, 0), tau, m))
            r.nws[tau - 1][m] = w
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert 2 * T.pair(env, Dw) == pytest.approx(fd, rel=1e-7, abs=1e-9), (tau, m)
            # Euler: that energy is homogeneous of degree two in this w
            e_blk = block_energy(r, Q.level_state(r.nws, r.v, 0), tau, m)
            assert T.pair(w, env) == pytest.approx(e_blk, abs=1e-11)


@pytest.mark.parametrize("L,chi,key", [(8, 16, "tfim_chain_L8_h1")])
def test_full_bond_dimension_is_exact(L, chi, key):
    model = I.tfim_chain(1.0)
    r = make(model, L, chi, seed=1)
    assert r.initialise() == pytest.approx(GOLD[key] / L, abs=1e-12)


def test_sweeps_lower_the_energy_above_the_exact_ground_energy():
    model, L, chi = I.tfim_chain(1.0), 16, 4
    r = make(model, L, chi, seed=2)
    hist = np.array(r.run(4))
    assert np.all(np.diff(hist) <= 1e-12 * np.abs(hist[:-1]))
    assert hist[-1] >= GOLD["tfim_chain_L16_h1"] / L - 1e-12
    # every updated isometry has orthonormal rows
    for layer in r.nws:
        for w in layer:
            W = w.reshape(w.shape[0], -1)
            assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 1e-13


def test_a_converged_uniform_state_is_not_raised():
    # the uniform network is one point of the position-resolved family: its
    # sweeps start from the uniform state and cannot raise its energy
    model, L, chi = I.xxx_chain(), 16, 4
    ref = T.TTNRef(L, chi, model.h1, model.A, model.B,
                   ws=I.random_isometries(T.layer_shapes(L, model.d, chi), 6))
    ref.run(12)
    r = Q.PositionalTTN(L, chi, model.h1, model.A, model.B, I.uniform_node_isometries(ref.ws, L), v=ref.v.copy())
    e0 = r.initialise()
    assert e0 == pytest.approx(ref.history[-1], abs=1e-12)
    hist = r.run(2)
    assert hist[-1] <= e0 + 1e-12


def test_planted_mistake_in_the_inner_edges_is_caught():
    # the inner edges of a parent built from the wrong child (A of the right
    # child instead of the left one) must fail the bond-energy pin
    model, L, chi = I.tfim_chain(0.8), 8, 4
    r = make(model, L, chi, seed=7)
    r.initialise()
    hs, As, Bs = r.operators()

    def wrong_descend(nws, v, As, Bs):
        swapped = [[As[t][m ^ 1] if t < len(As) - 1 else As[t][m] for m in range(len(As[t]))]
                   for t in range(len(As))]
        return Q.descend_all(nws, v, swapped, Bs)

    rho, X, Y = wrong_descend(r.nws, r.v, As, Bs)
    psi0 = Q.level_state(r.nws, r.v, 0)
    bonds = P.bond_expectations(psi0, r.A, r.B)
    caught = False
    for tau in range(r.n):
        for m in range(L >> tau):
            first = m << tau
            left = sum(T.pair(x, b) for x, b in zip(X[tau][m], Bs[tau][m]))
            caught |= abs(left - bonds[(first - 1) % L]) > 1e-8
    assert caught
