"""Position-resolved density matrices and local energies (ttn_local_energies)
against the CPU reference's rho_positions / local_energies on the state the
handle holds (its isometries and top tensor read back).

Element by element at sizes the reference finishes in seconds (ragged bonds
across several tiles, the antisymmetric XXX pair, a d = 8 torus column, bonds
above 64, a split-bf16 handle whose float64 masters are read); at the full
L = 4096, chi = 256 workload on sampled nodes and bonds the reference computes
one by one, and the invariants that hold at any size.

The float64 bars.  A matrix entry is a sum of K = chi_tau chi_{tau-1}^2
products per level of descent, each level rounding in its own order on the
two sides: about sqrt(K) eps of the entry's scale per level, 1e-13 absolute
for K <= 80^3 and entries <= 1, 1e-12 at chi = 256 over ten levels.  A bond
energy pairs chi^2 entries with its operator: 1e-12 absolute for
chi <= 80, 1e-11 at chi = 256.
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


def _state(B, t, b=0):
    n = t.n_levels(b)
    return [t.get_tensor(tau, b) for tau in range(1, n)], t.get_tensor(B.TTN_TOP, b)


CASES = [
    ("tfim_L64_chi12", I.tfim_chain(0.9), 64, 12, "fp64"),
    ("xxx_L32_chi20", I.xxx_chain(), 32, 20, "fp64"),
    ("torus8x3_chi24", I.torus_tfim_column(3, 2.9), 8, 24, "fp64"),
    ("xxx_L32_chi80", I.xxx_chain(), 32, 80, "fp64"),
    ("xxx_L128_chi48_bf16x3", I.xxx_chain(), 128, 48, "bf16x3"),
    ("tfim_L4_chi2", I.tfim_chain(1.1), 4, 2, "fp64"),
    ("tfim_L16_chi1", I.tfim_chain(0.5), 16, 1, "fp64"),  # product states: 1 x 1 matrices above level 0
    # the paper's column sites: d = 32, five product terms
    ("torus8x5_chi40_fp32", I.torus_tfim_column(5, 2.9), 8, 40, "fp32"),
]


@pytest.mark.parametrize("name,model,L,chi,prec", CASES, ids=[c[0] for c in CASES])
def test_local_energies_parity(B, name, model, L, chi, prec):
    print(f"[positions] {name}", flush=True)
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 21)
    t = B.TTN(B.ChainInput(model, L, chi, prec, w0=ws))
    t.sweep(1)
    n = t.n_levels()
    site, bond, rhos = t.local_energies(levels=range(n))
    ws_h, v_h = _state(B, t)
    site_r, bond_r, rhos_r = T.local_energies(ws_h, v_h, model.h1, model.A, model.B)
    ds, db = np.abs(site - site_r).max(), np.abs(bond - bond_r).max()
    print(f"  site {ds:.2e}, bond {db:.2e}")
    assert ds <= 1e-12 and db <= 1e-12
    for tau in range(n):
        assert rhos[tau].shape == rhos_r[tau].shape
        dr = np.abs(rhos[tau] - rhos_r[tau]).max()
        assert dr <= 1e-13, f"level {tau}: {dr:.2e}"
    if prec == "fp64":  # the energy the handle reports for its state
        e = t.energy()[0] * L * model.ly
        assert abs(site.sum() + bond.sum() - e) <= 1e-11 * max(1.0, abs(e))
    t.close()


def test_energy_sum_after_sweeps_and_repeat_calls(B):
    # the handle's state is untouched: sweeping on after the call gives the same
    # energies as a handle that never made it; a second call in a larger work
    # buffer (more parents per launch, so the products may split their sums
    # differently) agrees to rounding
    model, L, chi = I.xxx_chain(), 256, 32
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 5)
    a = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws))
    b = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws))
    for s in range(3):
        a.sweep(1)
        b.sweep(1)
        site, bond, _ = a.local_energies()
        big = torch.empty(4 * a.positions_bytes() + 256, dtype=torch.uint8, device="cuda")
        site2, bond2, _ = a.local_energies(work=big)
        assert np.abs(site - site2).max() <= 1e-14 and np.abs(bond - bond2).max() <= 1e-14
        e = a.energy()[0]
        assert e == b.energy()[0]
        assert abs(site.sum() + bond.sum() - e * L) <= 1e-12 * L
        print(f"  sweep {s}: e {e:.12f}, bond energies {bond.min():.6f} .. {bond.max():.6f}")
    a.close()
    b.close()


def test_batch_members_match_solo_handles(B):
    # members of a batch (two of one configuration, one launch group, and one
    # of another) read one by one give what the same states give alone
    draws = [(0.8, 64, 12), (1.2, 64, 12), (1.0, 32, 20)]
    ws = [I.random_isometries(T.layer_shapes(L, 2, chi), 30 + i) for i, (_, L, chi) in enumerate(draws)]
    batch = B.TTN([B.ChainInput(I.tfim_chain(h), L, chi, "fp64", w0=w) for (h, L, chi), w in zip(draws, ws)])
    batch.sweep(1)
    for i, (h, L, chi) in enumerate(draws):
        site, bond, _ = batch.local_energies(b=i)
        ws_h = [batch.get_tensor(tau, i) for tau in range(1, batch.n_levels(i))]
        v_h = batch.get_tensor(B.TTN_TOP, i)
        model = I.tfim_chain(h)
        site_r, bond_r, _ = T.local_energies(ws_h, v_h, model.h1, model.A, model.B)
        assert site.shape == (L,)
        assert np.abs(site - site_r).max() <= 1e-12 and np.abs(bond - bond_r).max() <= 1e-12
        assert abs(site.sum() + bond.sum() - batch.energy()[i] * L) <= 1e-11 * L
    batch.close()


def test_zero_product_terms_and_rejections(B):
    model = I.ChainModel("field", -0.7 * I.PAULI_X, [], [])
    t = B.TTN(B.ChainInput(model, 16, 4, "fp64", seed=2, shift=0.0))
    site, bond, _ = t.local_energies()
    assert np.all(bond == 0.0)
    ws_h, v_h = _state(B, t)
    site_r, _, _ = T.local_energies(ws_h, v_h, model.h1, [], [])
    assert np.abs(site - site_r).max() <= 1e-13
    small = torch.empty(t.positions_bytes() // 2 + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.TTNError) as e:
        t.local_energies(work=small)
    assert e.value.status == B.TTN_ENOMEM
    with pytest.raises(B.TTNError) as e:
        t.local_energies(b=1)
    assert e.value.status == B.TTN_EINVAL
    t.close()


def _path_rhos(ws, v, j):
    """Reference matrices of the nodes above site j, {tau: (m, rho)}, descended
    along that path only."""
    n = len(ws) + 1
    m = j >> (n - 1)
    rho = v @ v.T if m == 0 else v.T @ v
    out = {n - 1: (m, rho)}
    for sigma in range(n - 1, 0, -1):
        w = ws[sigma - 1]
        m = j >> (sigma - 1)
        P = T.left_mul(rho, w)
        rho = T.close_r(w, P) if m & 1 else T.close_l(w, P)
        out[sigma - 1] = (m, rho)
    return out


def test_full_size_sampled(B):
    # the XXX chain at L = 4096, chi = 256 (split-bf16 handle, float64
    # masters): sampled nodes of every level and sampled bonds against the
    # reference computed node by node, and the invariants
    import time
    model, L, chi = I.xxx_chain(), 4096, 256
    print("[positions] full size", flush=True)
    t = B.TTN(B.ChainInput(model, L, chi, "bf16x3", seed=0))
    t.sweep_grouped(1, 2)
    n = t.n_levels()
    t.local_energies()  # first call: launch choices
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    site, bond, rhos = t.local_energies(levels=range(n))
    dt = time.perf_counter() - t0
    print(f"  local energies of L = {L}: {dt * 1e3:.1f} ms (including the copies to the host)")
    ws, v = _state(B, t)
    rng = np.random.default_rng(0)
    paths = [_path_rhos(ws, v, j) for j in (0, L - 1, int(rng.integers(L)))]
    for path in paths:
        for tau, (m, ref) in path.items():
            d = np.abs(rhos[tau][m] - ref).max()
            assert d <= 1e-12, f"node ({tau}, {m}): {d:.2e}"
    for tau in range(n):
        tr = np.trace(rhos[tau], axis1=1, axis2=2)
        assert np.abs(tr - 1.0).max() < 1e-12
        assert np.abs(rhos[tau] - np.transpose(rhos[tau], (0, 2, 1))).max() < 1e-13
    # bonds: the ascended product operators, then node by node
    As, Bs = [list(model.A)], [list(model.B)]
    for w in ws:
        As.append([T.close(w, T.apply_r(a, w)) for a in As[-1]])
        Bs.append([T.close(w, T.apply_l(b_, w)) for b_ in Bs[-1]])
    for tau in (1, 4, n - 1):
        w = ws[tau - 1]
        op = sum(T.close(w, T.apply_l(a, T.apply_r(b_, w))) for a, b_ in zip(As[tau - 1], Bs[tau - 1]))
        for path in paths:
            m, rho = path[tau]
            ref = T.pair(rho, op)
            j = T.bond_site(tau, m)
            assert abs(bond[j] - ref) <= 1e-11, (tau, m, bond[j], ref)
    mid = sum(T.pair(v, a @ v @ b_.T) for a, b_ in zip(As[n - 1], Bs[n - 1]))
    wrap = sum(T.pair(v, b_ @ v @ a.T) for a, b_ in zip(As[n - 1], Bs[n - 1]))
    assert abs(bond[L // 2 - 1] - mid) <= 1e-11 and abs(bond[L - 1] - wrap) <= 1e-11
    for j in rng.integers(L, size=4):
        assert abs(site[j] - T.pair(rhos[0][j], model.h1)) <= 1e-14
    # the sum against the float64 evaluation of the same state
    f = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, v0=v))
    e64 = f.energy()[0]
    f.close()
    t.close()
    total = site.sum() + bond.sum()
    print(f"  sum of local energies / L {total / L:.12f}, float64 energy {e64:.12f}")
    assert abs(total / L - e64) <= 1e-11
