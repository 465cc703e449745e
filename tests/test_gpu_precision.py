"""Precision form (OCSC_FLAG_CHOLESKY): the minibatch history on the BF16
matrix cores with a split-precision correction, C recomputed from an FP64
Cholesky per frequency (for K > 128 through two 128-blocks and a Schur
complement); FP32 code ADMM.  Against the FP64 oracle every quantity must be
within 1e-3 (norm-wise relative); the errors are printed.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np, unpack_cinv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def images(n, ph, K_true, seed):
    wl = synth.Workload(name="t", pad_h=ph, pad_w=ph, content_h=ph - 10, content_w=ph - 10, k_true=K_true,
                        density=0.01, sigma_z=10.0, noise=0.01, K=K_true, filt_h=11, filt_w=11, lam=1.0, rho=1.0,
                        iters_code=10, iters_dict=10, batch=1, n_images=n, passes=1, precision="f64", seed=seed)
    return synth.images(wl, range(n))


@pytest.mark.parametrize("K,B,batches,n,refine", [(16, 8, 2, 64, False), (100, 6, 2, 64, False),
                                                  (40, 70, 1, 64, False), (256, 4, 2, 32, False),
                                                  (200, 3, 1, 32, False), (129, 2, 1, 32, False),
                                                  (120, 3, 1, 32, False), (100, 6, 2, 64, True),
                                                  (256, 4, 2, 32, True)])
def test_cholesky_form_matches_oracle(K, B, batches, n, refine):
    """K > 128 takes the block (Schur complement) inverse and the streaming
    D-step; refine adds one refinement step after each D-step."""
    say(f"case precision form K={K} B={B} grid {n}{' with refinement' if refine else ''}")
    from paper_1706_06972_amd.ocsc import OCSC
    xs = images(B * batches, n, 16, 11)
    g = OCSC(K, 11, 11, n, n, 1.0, 1.0, precision="f32", max_batch=B, cholesky=True, refine=refine)
    o = O.OCSC(K, 11, 11, n, n, 1.0, 1.0, keep_history=True)
    D0 = synth.initial_dictionary(K, 11, 11, 0)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    errs = {}
    for bi in range(batches):
        x = xs[bi * B:(bi + 1) * B]
        U = to_np(g.code_update(x))
        Uo = o.code_update(x)
        errs["codes"] = max(errs.get("codes", 0), rel(U, Uo))
        g.history_accumulate()
        o.history_accumulate()
        H = unpack_cinv(to_np(g.state("H")), K, n, n)
        C = unpack_cinv(to_np(g.state("cinv")), K, n, n)
        errs["H"] = max(errs.get("H", 0), rel(H, o.H))
        errs["G"] = max(errs.get("G", 0), rel(spectra(to_np(g.state("G")), (K,), n, n), o.G))
        errs["C"] = max(errs.get("C", 0), rel(C, o.C))
        # solve residual of the recomputed inverse against the device's own H
        A = H + o.rho_d * np.eye(K)
        res = np.linalg.norm(A @ C - np.eye(K), axis=(-2, -1)) / np.sqrt(K)
        errs["solve_residual"] = max(errs.get("solve_residual", 0), float(res.max()))
        g.dict_update()
        o.dict_update()
        errs["dict"] = max(errs.get("dict", 0), rel(to_np(g.get_dictionary()), o.get_dictionary()))
        errs["V"] = max(errs.get("V", 0), rel(to_np(g.state("V")).reshape(K, 11, 11), o.V))
        f = g.objective(x, torch.as_tensor(U, device="cuda"))
        fo = o.objective(x, Uo)
        errs["objective"] = max(errs.get("objective", 0), float(np.max(np.abs(np.array(f) - fo) / np.abs(fo))))
    say("errors vs FP64 oracle", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < 1e-3, (k, v)
    assert g.count == B * batches
    g.close()


@pytest.mark.parametrize("K", [16, 200])
def test_cholesky_breakdown_is_reported(K):
    """An indefinite history, set from the host through the state interface
    (H = -2 rho_d I at every frequency), makes H + rho_d I negative definite:
    the FP64 factorisation meets a negative pivot at the next fold, and the next
    call that waits returns OCSC_E_NUMERIC (once).  K = 200 takes the block
    (Schur complement) path, whose first block then breaks down."""
    say(f"case Cholesky breakdown K={K}")
    from paper_1706_06972_amd.ocsc import OCSC, OcscError, OCSC_E_NUMERIC
    n = 32
    xs = images(2, n, 16, 3)
    g = OCSC(K, 11, 11, n, n, 1.0, 1.0, precision="f32", max_batch=2, cholesky=True)
    g.set_dictionary(synth.initial_dictionary(K, 11, 11, 0))
    Pf = n * (n // 2 + 1)
    rho_d = 1.0 * n * n
    H = np.zeros((Pf, K, K), np.float32)
    H[:, np.arange(K), np.arange(K)] = -2.0 * rho_d                # packed form: the diagonal is real
    g.set_state("H", torch.as_tensor(H.reshape(-1), device="cuda"))
    g.code_update(xs, want_codes=False)
    g.history_accumulate()
    with pytest.raises(OcscError) as e:
        g.sync()
    assert e.value.status == OCSC_E_NUMERIC
    assert "Cholesky breakdown" in str(e.value)
    g.sync()                                                        # reported once
    g.close()


@pytest.mark.parametrize("K", [100, 256])
def test_refinement_of_the_dstep_solve(K):
    """One DictOCSC iteration (J_d = 1, so d_p solves (H_p + rho_d I) d_p = G_p,
    eq. sub_d_sol from V = Theta = 0), without and with the refinement step,
    on the same minibatch.  Each d is compared with the FP64 solve of the
    library's own H and G; the errors and solve residuals are printed.  The
    refined solve must not be worse than the plain one beyond FP32 rounding."""
    say(f"case refinement of the D-step solve K={K}")
    from paper_1706_06972_amd.ocsc import OCSC
    n, B = 32, 4
    xs = images(2 * B, n, 16, 13)
    D0 = synth.initial_dictionary(K, 11, 11, 0)
    res = {}
    for refine in (False, True):
        g = OCSC(K, 11, 11, n, n, 1.0, 1.0, precision="f32", max_batch=B, cholesky=True, refine=refine,
                 iters_dict=1)
        g.set_dictionary(D0)
        for bi in range(2):
            g.code_update(xs[bi * B:(bi + 1) * B], want_codes=False)
            g.history_accumulate()
            if bi == 0:
                g.dict_update()
        H = unpack_cinv(to_np(g.state("H")), K, n, n).reshape(-1, K, K)
        G = spectra(to_np(g.state("G")), (K,), n, n).reshape(K, -1).T
        g.dict_update()
        d = spectra(to_np(g.state("dict_hat")), (K,), n, n).reshape(K, -1).T
        A = H + (n * n) * np.eye(K)
        dx = np.linalg.solve(A, G[:, :, None])[:, :, 0]
        r = (A @ d[:, :, None])[:, :, 0] - G
        res[refine] = (rel(d, dx), np.linalg.norm(r) / np.linalg.norm(G))
        g.close()
    say(f"  d vs FP64 solve of the library's H: plain {res[False][0]:.2e}, refined {res[True][0]:.2e}; "
        f"residual plain {res[False][1]:.2e}, refined {res[True][1]:.2e}")
    assert res[False][0] < 1e-3 and res[True][0] < 1e-3
    assert res[True][0] <= 1.5 * res[False][0] + 1e-7
