"""Parity of the two-pass plane path (grids with sides 256 and 512) with the
FP64 oracle through the C ABI: dictionary transforms, one full step (codes,
spectra, history, dictionary, objective) and coding against a fixed
dictionary on several grid sizes.

Tolerances: norm-wise relative 1e-10 (FP64 contexts), 1e-3 (FP32 contexts).
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np, unpack_cinv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-3}


def images(n, ph, pw, seed=0):
    wl = synth.Workload(name="t", pad_h=ph, pad_w=pw, content_h=ph // 2, content_w=pw // 2, k_true=8,
                        density=0.01, sigma_z=10.0, noise=0.01, K=8, filt_h=11, filt_w=11, lam=1.0, rho=1.0,
                        iters_code=10, iters_dict=10, batch=1, n_images=n, passes=1, precision="f64", seed=seed)
    return synth.images(wl, range(n))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ph,pw", [(256, 256), (512, 512), (256, 512), (512, 256)])
def test_big_dictionary_transforms(prec, ph, pw):
    say(f"case big dictionary transforms {prec} {ph}x{pw}")
    from paper_1706_06972_amd.ocsc import OCSC
    K, fh, fw = 3, 11, 9
    g = OCSC(K, fh, fw, ph, pw, 1.0, 1.0, precision=prec)
    o = O.OCSC(K, fh, fw, ph, pw, 1.0, 1.0)
    D0 = synth.initial_dictionary(K, fh, fw, 0)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    assert rel(spectra(to_np(g.state("dict_hat")), (K,), ph, pw), o.Dh) < TOL[prec] * 1e-2
    assert rel(to_np(g.get_dictionary()), D0) < TOL[prec] * 1e-2
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ph,pw,K", [(256, 256, 4), (512, 512, 3)])
def test_big_steps_match_oracle(prec, ph, pw, K):
    say(f"case big steps {prec} {ph}x{pw} K={K}")
    from paper_1706_06972_amd.ocsc import OCSC
    fh = fw = 11
    xs = images(2, ph, pw)
    g = OCSC(K, fh, fw, ph, pw, 0.5, 1.0, precision=prec)
    o = O.OCSC(K, fh, fw, ph, pw, 0.5, 1.0)
    D0 = synth.initial_dictionary(K, fh, fw, 0)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    tol = TOL[prec]
    for step, x in enumerate(xs):
        U = g.code_update(x)
        Uo = o.code_update(x[None])
        assert np.count_nonzero(Uo) > 0
        assert rel(to_np(U), Uo) < tol, f"codes step {step}"
        fg = g.objective(x, U)[0]
        fo = o.objective(x[None], Uo)[0]
        assert abs(fg - fo) / abs(fo) < tol
        g.history_accumulate()
        o.history_accumulate()
        assert rel(spectra(to_np(g.state("G")), (K,), ph, pw), o.G) < tol
        assert rel(unpack_cinv(to_np(g.state("cinv")), K, ph, pw), o.C) < tol
        g.dict_update()
        o.dict_update()
        assert rel(spectra(to_np(g.state("dict_hat")), (K,), ph, pw), o.Dh) < tol
        assert rel(to_np(g.state("V")).reshape(K, fh, fw), o.V) < tol
        assert rel(to_np(g.get_dictionary()), o.get_dictionary()) < tol
    g.close()


def test_coding_on_mixed_grids_fp32():
    """Coding only, one fixed dictionary, samples on 64, 128, 256 and 512 grids
    (one context per grid, a batch per grid)."""
    say("case mixed-grid coding f32")
    from paper_1706_06972_amd.ocsc import OCSC
    K, fh, fw = 6, 11, 11
    D0 = synth.initial_dictionary(K, fh, fw, 3)
    for n in (64, 128, 256, 512):
        xs = images(2, n, n, seed=n)
        g = OCSC(K, fh, fw, n, n, 0.5, 1.0, precision="f32", max_batch=2)
        o = O.OCSC(K, fh, fw, n, n, 0.5, 1.0)
        g.set_dictionary(D0)
        o.set_dictionary(D0)
        U = to_np(g.code_update(xs))
        Uo = o.code_update(xs)
        assert rel(U, Uo) < 1e-3, n
        g.close()
