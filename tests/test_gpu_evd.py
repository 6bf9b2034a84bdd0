"""The eigenvalue-decomposition variant of the isometry update (appendix,
Fig. 10(b)) on the GPU path.

With evd_update = 1 an update is one Gram matrix G = Env Env^T = U S^2 U^T,
its float64 Jacobi eigendecomposition and w = -U S^-1 U^T Env.  Checked, from
the reference's state layer by layer: the result equals the reference's
variant (LAPACK eigendecomposition of the same Gram matrix) to about
eps (s_max/s_min)^2, which is the precision the squaring leaves; where the
environments are well conditioned, whole sweeps agree with the default
update.
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


CASES = [
    ("xxx_L64_chi3", I.xxx_chain(), 64, 3),
    ("tfim_L32_chi6", I.tfim_chain(1.2), 32, 6),
    ("torus8x3_chi12", I.torus_tfim_column(3, 3.0), 8, 12),
]


@pytest.mark.parametrize("name,model,L,chi", CASES, ids=[c[0] for c in CASES])
def test_evd_update_matches_reference_variant(B, name, model, L, chi):
    print(f"[evd] {name}", flush=True)
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 13)
    ref = T.TTNRef(L, chi, model.h1, model.A, model.B, ly=model.ly, ws=ws)
    ref.initialise()
    gpu = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, keep_gauge=True, evd_update=True))
    gpu.set_tensor(B.TTN_TOP, ref.v)
    gpu.descend(B.TTN_DESCEND_RHO)
    rhos = T.descend_rho_all(ref.ws, ref.v)
    eps = np.finfo(np.float64).eps
    checked = 0
    for tau in range(1, ref.n):
        gpu.descend(B.TTN_DESCEND_DRESSED, tau)
        h, A, Bm = ref.hs[tau - 1], ref.As[tau - 1], ref.Bs[tau - 1]
        R, Lb = T.dressed_chain(ref.ws, ref.v, rhos, tau, A, Bm)
        gpu.env(tau)
        env = gpu.get_operator(tau, B.TTN_OP_ENV)
        gpu.update(tau)
        w_gpu = gpu.get_tensor(tau)
        sv = np.linalg.svd(env.reshape(env.shape[0], -1), compute_uv=False)
        cond = float(sv[0] / sv[-1])
        if cond < 1e5:
            w_ref, _ = T.polar_update_evd(env)
            d = float(np.abs(w_gpu - w_ref).max())
            print(f"  tau {tau}: condition {cond:.2e}, difference {d:.2e}")
            assert d <= 1e3 * eps * cond ** 2
            checked += 1
        else:
            # the squared environment has lost the weak directions: the
            # variant is not defined to working precision there; both sides
            # continue from the SVD factor
            print(f"  tau {tau}: condition {cond:.2e}, not compared")
            w_ref, _ = T.polar_update(env)
        # both sides continue from the reference's isometry
        ref.ws[tau - 1] = w_ref
        gpu.set_tensor(tau, w_ref)
        ref.hs[tau], ref.As[tau], ref.Bs[tau] = T.ascend(w_ref, h, A, Bm)
        gpu.ascend(tau, tau)
    assert checked > 0
    gpu.close()


def test_evd_sweeps_follow_the_default_update_to_the_squared_precision(B):
    # sweeps of the two updates from the same start: the variant's error is
    # of order eps / r^2 with r the smallest sigma_min / sigma_max of the
    # sweep's environments (reported by ttn_stats), and the trajectories
    # carry it on
    model, L, chi = I.xxx_chain(), 64, 3
    ws = I.random_isometries(T.layer_shapes(L, model.d, chi), 1)
    acc = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws))
    evd = B.TTN(B.ChainInput(model, L, chi, "fp64", w0=ws, evd_update=True))
    eps = np.finfo(np.float64).eps
    r_min = 1.0
    for s in range(4):
        acc.sweep(1)
        evd.sweep(1, graph=(s > 0))
        ea, ee = acc.energy()[0], evd.energy()[0]
        r_min = min(r_min, acc.stats().sigma_ratio_min)
        bar = max(1e-10, 1e3 * eps / r_min ** 2)
        print(f"  sweep {s}: default {ea:.15f} evd {ee:.15f}, r {r_min:.1e}, bar {bar:.1e}")
        assert abs(ea - ee) <= bar * abs(ea)
    acc.close()
    evd.close()
