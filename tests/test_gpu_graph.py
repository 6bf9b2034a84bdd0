"""Graph replay and batches of chains.

The layer part of a sweep is captured into a HIP graph on the first
ttn_sweep(.., use_graph=1) and replayed afterwards; every replay must give
the energies of the eager path exactly (same kernels, same order), with the
eager top update, synchronisations and energy reads between replays.  A
batch runs its members side by side on internal streams; each member must
follow the path it follows alone.
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


# (name, model, L, chi, precision): the one-work-group Jacobi (a <= 96), the
# persistent blocked Jacobi (a = 160), a mixed-precision bulk
GRAPH_CASES = [
    ("tfim_L64_chi24_fp64", I.tfim_chain(1.0), 64, 24, "fp64"),
    ("xxx_L32_chi160_fp64", I.xxx_chain(), 32, 160, "fp64"),
    ("torus8x4_chi64_bf16x3", I.torus_tfim_column(4, 3.0), 8, 64, "bf16x3"),
]


@pytest.mark.parametrize("name,model,L,chi,prec", GRAPH_CASES, ids=[c[0] for c in GRAPH_CASES])
def test_graph_replays_match_eager(B, name, model, L, chi, prec):
    print(f"[graph] {name}", flush=True)
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 7)
    eager = B.TTN(B.ChainInput(model, L, chi, prec, w0=ws))
    graph = B.TTN(B.ChainInput(model, L, chi, prec, w0=ws))
    for s in range(5):
        eager.sweep(1)
        graph.sweep(1, graph=True)
        e0, e1 = eager.energy()[0], graph.energy()[0]
        assert e0 == e1, f"sweep {s}: eager {e0!r} graph {e1!r}"
    # the graph reads the workspace at replay time: a state loaded between
    # sweeps is honoured
    n = eager.n_levels()
    state = [eager.get_tensor(tau) for tau in range(1, n)]
    v = eager.get_tensor(B.TTN_TOP)
    for h in (eager, graph):
        for tau in range(1, n):
            h.set_tensor(tau, state[tau - 1])
        h.set_tensor(B.TTN_TOP, v)
        h.ascend(1, n - 1)
    eager.sweep(1)
    graph.sweep(1, graph=True)
    assert eager.energy()[0] == graph.energy()[0]
    w_e = eager.get_tensor(1)
    w_g = graph.get_tensor(1)
    assert np.array_equal(w_e, w_g)
    eager.close()
    graph.close()


def test_top_update_from_graphs(B):
    # graph sweeps replay the top update from a graph too: mode 2 with every
    # restart of the budget (the ones after convergence return at once on a
    # device flag), mode 1 with the restarts needed so far and an eager
    # completion when a member needs more; the eager sweep stops launching at
    # convergence.  All end with the same vector, energy and Krylov count,
    # over sweeps whose restart needs vary (a small Krylov space).  With too
    # small a budget (4 Krylov vectors, one restart) the eager sweep returns
    # TTN_WNOCONV, so does a mode-1 sweep, and ttn_energy reports it after
    # either graph mode
    model, L, chi = I.tfim_chain(1.0), 64, 16
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 9)
    small = dict(krylov=6, restarts=8)
    eager = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, **small))
    g1 = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, **small))
    g2 = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, **small))
    iters = set()
    for s in range(4):
        st_e = eager.sweep(1)
        assert g1.sweep(1, graph=1) == st_e
        g2.sweep(1, graph=2)
        e = eager.energy()[0]
        assert g1.energy()[0] == e and g2.energy()[0] == e
        assert g1.energy_status == eager.energy_status == g2.energy_status
        it = eager.stats().lanczos_iters
        assert g1.stats().lanczos_iters == it == g2.stats().lanczos_iters > 0
        assert eager.stats().e_prev == g1.stats().e_prev == g2.stats().e_prev
        iters.add(it)
        v = eager.get_tensor(B.TTN_TOP)
        assert np.array_equal(g1.get_tensor(B.TTN_TOP), v) and np.array_equal(g2.get_tensor(B.TTN_TOP), v)
    print(f"  Krylov steps per top update: {sorted(iters)}")
    for h in (eager, g1, g2):
        h.close()
    tight = dict(krylov=4, restarts=1)
    eager = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, **tight))
    g1 = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, **tight))
    g2 = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, **tight))
    assert eager.sweep(1) == B.TTN_WNOCONV
    assert g1.sweep(1, graph=1) == B.TTN_WNOCONV
    g2.sweep(1, graph=2)
    e = eager.energy()[0]
    assert eager.energy_status == B.TTN_WNOCONV
    for g in (g1, g2):
        assert g.energy()[0] == e
        assert g.energy_status == B.TTN_WNOCONV
        assert g.stats().lanczos_iters == 4
    for h in (eager, g1, g2):
        h.close()


def test_batch_members_follow_their_solo_paths(B):
    # uneven L, chi and couplings; a <= 64 everywhere, so a member runs the
    # same kernels in the batch as alone
    draws = [(I.tfim_chain(0.7), 64, 32), (I.tfim_chain(1.3), 128, 48), (I.xxx_chain(), 32, 16),
             (I.tfim_chain(1.0), 256, 64)]
    inputs = [B.ChainInput(m, L, chi, "fp32", seed=100 + i) for i, (m, L, chi) in enumerate(draws)]
    batch = B.TTN(inputs)
    solo = [B.TTN(B.ChainInput(m, L, chi, "fp32", seed=100 + i)) for i, (m, L, chi) in enumerate(draws)]
    e_b0 = batch.energy()
    e_s0 = np.array([t.energy()[0] for t in solo])
    assert np.array_equal(e_b0, e_s0)
    for s in range(3):
        batch.sweep(1, graph=(s > 0))
        for t in solo:
            t.sweep(1)
        e_b = batch.energy()
        e_s = np.array([t.energy()[0] for t in solo])
        print(f"  sweep {s}: batch {e_b} solo {e_s}")
        assert np.array_equal(e_b, e_s)
    for t in solo:
        t.close()
    batch.close()


def test_batch_with_larger_bond_dimension(B):
    # a member with 96 < a <= 128 takes the blocked Jacobi solver in a batch
    # as it does alone, a member with a = 96 the one-work-group solver in both
    # (the solver is chosen by the order of the Gram matrix only), so every
    # member follows its solo run bit for bit
    draws = [(1.0, 64, 112), (1.1, 128, 32), (0.9, 64, 96)]
    ws = [I.random_isometries(T.layer_shapes(L, 2, chi), 20 + i) for i, (h, L, chi) in enumerate(draws)]
    batch = B.TTN([B.ChainInput(I.tfim_chain(h), L, chi, "fp64", w0=w) for (h, L, chi), w in zip(draws, ws)])
    solo = [B.TTN(B.ChainInput(I.tfim_chain(h), L, chi, "fp64", w0=w)) for (h, L, chi), w in zip(draws, ws)]
    for s in range(2):
        batch.sweep(1, graph=True)
        for t in solo:
            t.sweep(1)
        e = batch.energy()
        e_s = np.array([t.energy()[0] for t in solo])
        assert np.array_equal(e, e_s), (s, e, e_s)
    for tau in range(1, batch.n_levels(0)):
        assert np.array_equal(batch.get_tensor(tau, 0), solo[0].get_tensor(tau))
    for t in solo:
        t.close()
    batch.close()


def test_autotuner_choices_leave_results_unchanged(B):
    # mode 1 times the launch shapes of each new product when first met
    # eagerly; a choice changes only the tile size and the order in which
    # tiles are handed out, never the split of a contraction or an element's
    # instruction sequence, so the tuned run gives the same bits as the
    # default one, eagerly and from the captured graph, for every bulk
    # precision; the kept table written to a file and read back is the same
    import os
    import tempfile
    model, L, chi = I.tfim_chain(1.0), 128, 64
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 3)
    try:
        for prec in ("fp64", "fp32", "bf16x3"):
            B.autotune(0)
            ref = B.TTN(B.ChainInput(model, L, chi, prec, w0=ws))
            e_ref = [ref.energy()[0]]
            for _ in range(3):
                ref.sweep(1)
                e_ref.append(ref.energy()[0])
            ref.close()
            B.autotune(1)
            tuned = B.TTN(B.ChainInput(model, L, chi, prec, w0=ws))
            e_t = [tuned.energy()[0]]
            tuned.sweep(1)
            e_t.append(tuned.energy()[0])
            for _ in range(2):
                tuned.sweep(1, graph=True)
                e_t.append(tuned.energy()[0])
            tuned.close()
            print(f"  {prec}: default {e_ref} tuned {e_t}", flush=True)
            assert e_t == e_ref, prec
        kept = B.autotune(2)
        assert kept > 0
        path = os.path.join(tempfile.mkdtemp(), "launches.txt")
        B.autotune_save(path)
        assert B.autotune_load(path) == kept
        assert B.autotune(-1) == kept
    finally:
        B.autotune(0)


def test_benchmarked_batch_follows_solo_runs_with_tuner_and_graph(B):
    # the batch as the benchmark runs it: float32 bulk, launch tuner on,
    # sweeps replayed from the captured graph, members of uneven L, chi and
    # h, two launch groups, chi = 96 members (the one-work-group Jacobi with
    # G and its eigenvectors in LDS, one launch for their group); every member
    # equals its solo run (tuner on too, eager) bit for bit
    draws = [(0.9, 64, 96), (1.2, 128, 48), (0.7, 128, 48), (1.4, 256, 32), (1.1, 64, 96), (0.6, 512, 64)]
    mk = lambda i, d: B.ChainInput(I.tfim_chain(d[0]), d[1], d[2], "fp32", seed=1000 + i)
    try:
        B.autotune(1)
        batch = B.TTN([mk(i, d) for i, d in enumerate(draws)])
        batch.sweep(1)
        for _ in range(3):
            batch.sweep(1, graph=True)
        e_b = batch.energy()
        B.autotune(0)
        for i, d in enumerate(draws):
            t = B.TTN(mk(i, d))
            t.sweep(4)
            e_s = t.energy()[0]
            print(f"  member {i} (L={d[1]}, chi={d[2]}): batch {e_b[i]!r} solo {e_s!r}", flush=True)
            assert e_b[i] == e_s, i
            for tau in range(1, t.n_levels()):
                assert np.array_equal(batch.get_tensor(tau, i), t.get_tensor(tau)), (i, tau)
            t.close()
        batch.close()
    finally:
        B.autotune(0)


@pytest.mark.parametrize("prec,keep_gauge", [("fp32", False), ("fp64", True)])
def test_members_of_one_bond_dimension_and_different_lengths(B, prec, keep_gauge):
    # chains of one chi and five lengths (depths 6 to 10) form one coarse group:
    # the layer part of a sweep advances them level by level together, the
    # members at a level a prefix of the group, those whose top is there a
    # range of it (their top dressing, their gauge rotation into v); each
    # member's arithmetic is its own, so every member equals its solo run bit
    # for bit, eager and replayed, with the gauge fixed and kept (warm starts)
    draws = [(0.8, 256, 32), (1.2, 64, 32), (1.0, 128, 32), (0.6, 64, 32), (1.4, 1024, 32)]
    mk = lambda i, d: B.ChainInput(I.tfim_chain(d[0]), d[1], d[2], prec, seed=300 + i, keep_gauge=keep_gauge)
    batch = B.TTN([mk(i, d) for i, d in enumerate(draws)])
    solo = [B.TTN(mk(i, d)) for i, d in enumerate(draws)]
    for s in range(4):
        batch.sweep(1, graph=(s >= 2))
        for t in solo:
            t.sweep(1)
        e_b = batch.energy()
        e_s = np.array([t.energy()[0] for t in solo])
        assert np.array_equal(e_b, e_s), (s, e_b, e_s)
    for i, t in enumerate(solo):
        for tau in range(1, t.n_levels()):
            assert np.array_equal(batch.get_tensor(tau, i), t.get_tensor(tau)), (i, tau)
        t.close()
    batch.close()


def test_launch_groups_match_solo_runs(B):
    # members of equal configuration (L, chi, precision; only h differs) are
    # laid out side by side and run every kernel of a stage as one launch; a
    # group shares the restart loop of the top eigensolver, but a member that
    # has converged sets a device flag and its kernels skip every later
    # restart, so each member does the arithmetic it does alone
    draws = [(0.8, 128, 48), (1.2, 64, 32), (1.0, 128, 48), (0.6, 128, 48), (1.4, 64, 32)]
    ws = [I.random_isometries(T.layer_shapes(L, 2, chi), 40 + i) for i, (h, L, chi) in enumerate(draws)]
    batch = B.TTN([B.ChainInput(I.tfim_chain(h), L, chi, "fp64", w0=w) for (h, L, chi), w in zip(draws, ws)])
    solo = [B.TTN(B.ChainInput(I.tfim_chain(h), L, chi, "fp64", w0=w)) for (h, L, chi), w in zip(draws, ws)]
    e_b = batch.energy()
    e_s = np.array([t.energy()[0] for t in solo])
    assert np.array_equal(e_b, e_s)
    for s in range(3):
        batch.sweep(1, graph=(s > 0))
        for t in solo:
            t.sweep(1)
        e_b = batch.energy()
        e_s = np.array([t.energy()[0] for t in solo])
        print(f"  sweep {s}: batch {e_b} solo {e_s}")
        assert np.array_equal(e_b, e_s)
    for i in range(len(draws)):
        for tau in range(1, batch.n_levels(i)):
            w = batch.get_tensor(tau, i)
            W = w.reshape(w.shape[0], -1)
            assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 1e-13
    for t in solo:
        t.close()
    batch.close()
