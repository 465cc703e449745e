"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Tolerances: norm-wise relative error 1e-10 for FP64 contexts and 1e-3 for
FP32 contexts against the FP64 oracle, per quantity (codes, spectra, history,
dictionary, objective).  Inputs are the seeded synthetic workloads.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np, unpack_cinv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-3}


def make_pair(K, fh, fw, ph, pw, lam=1.0, rho=1.0, prec="f64", jz=10, jd=10, max_batch=1, seed=0):
    from paper_1706_06972_amd.ocsc import OCSC
    g = OCSC(K, fh, fw, ph, pw, lam, rho, iters_code=jz, iters_dict=jd, max_batch=max_batch, precision=prec)
    o = O.OCSC(K, fh, fw, ph, pw, lam, rho, iters_code=jz, iters_dict=jd)
    D0 = synth.initial_dictionary(K, fh, fw, seed)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    return g, o


def synth_images(n, ph, pw, K_true=16, density=0.01, sigma=10.0, seed=0):
    wl = synth.Workload(name="t", pad_h=ph, pad_w=pw, content_h=ph - 10, content_w=pw - 10, k_true=K_true,
                        density=density, sigma_z=sigma, noise=0.01, K=K_true, filt_h=11, filt_w=11, lam=1.0,
                        rho=1.0, iters_code=10, iters_dict=10, batch=1, n_images=n, passes=1, precision="f64",
                        seed=seed)
    return synth.images(wl, range(n))


GRIDS = [(32, 32), (32, 64), (32, 128), (64, 32), (64, 64), (64, 128), (128, 32), (128, 64), (128, 128)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ph,pw", GRIDS)
def test_dictionary_spectrum_and_export(prec, ph, pw):
    say(f"case dictionary transforms {prec} {ph}x{pw}")
    K, fh, fw = 5, 7, 9
    g, o = make_pair(K, fh, fw, ph, pw, prec=prec)
    Dh = spectra(to_np(g.state("dict_hat")), (K,), ph, pw)
    assert rel(Dh, o.Dh) < TOL[prec] * 1e-2
    D = to_np(g.get_dictionary())
    assert rel(D, synth.initial_dictionary(K, fh, fw, 0)) < TOL[prec] * 1e-2
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ph,pw,K,fh,fw", [(64, 64, 16, 11, 11), (32, 64, 7, 5, 3), (128, 32, 3, 11, 11)])
def test_one_step_matches_oracle(prec, ph, pw, K, fh, fw):
    say(f"case one step {prec} {ph}x{pw} K={K} filt={fh}x{fw}")
    xs = synth_images(2, ph, pw)
    g, o = make_pair(K, fh, fw, ph, pw, lam=0.5, prec=prec)
    tol = TOL[prec]
    for step, x in enumerate(xs):
        U = to_np(g.code_update(x))
        Uo = o.code_update(x[None])
        assert np.count_nonzero(Uo) > 0
        assert rel(U, Uo) < tol, f"codes step {step}"
        zh = spectra(to_np(g.state("zhat")), (1, K), ph, pw)[0]
        assert rel(zh, o._pending[0][0]) < tol
        xh = spectra(to_np(g.state("xhat")), (1,), ph, pw)[0]
        assert rel(xh, o._pending[0][1]) < tol
        fg = g.objective(x, torch.as_tensor(U))[0]
        fo = o.objective(x[None], Uo)[0]
        assert abs(fg - fo) / abs(fo) < tol
        g.history_accumulate()
        o.history_accumulate()
        G = spectra(to_np(g.state("G")), (K,), ph, pw)
        assert rel(G, o.G) < tol
        C = unpack_cinv(to_np(g.state("cinv")), K, ph, pw)
        assert rel(C, o.C) < tol
        g.dict_update()
        o.dict_update()
        assert rel(spectra(to_np(g.state("dict_hat")), (K,), ph, pw), o.Dh) < tol
        assert rel(to_np(g.state("V")).reshape(K, fh, fw), o.V) < tol
        assert rel(spectra(to_np(g.state("theta")), (K,), ph, pw), o.Th) < tol
        assert rel(to_np(g.get_dictionary()), o.get_dictionary()) < tol
    assert g.count == 2
    g.close()


def test_trajectory_64x64_k16_f64():
    """The 50-image, one-pass FP64 workload: every step within 1e-10."""
    wl = synth.WORKLOADS["ocsc_64x64_k16_f64"]
    say(f"case trajectory {wl.name}")
    xs = synth.images(wl, range(wl.n_images))
    g, o = make_pair(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, "f64",
                     wl.iters_code, wl.iters_dict, seed=wl.seed)
    worst = {"codes": 0.0, "objective": 0.0, "dict": 0.0}
    for i in synth.pass_order(wl.n_images, wl.seed, 0):
        U = g.code_update(xs[i])
        Uo = o.code_update(xs[i][None])
        fg = g.objective(xs[i], U)[0]
        fo = o.objective(xs[i][None], Uo)[0]
        worst["codes"] = max(worst["codes"], rel(to_np(U), Uo))
        worst["objective"] = max(worst["objective"], abs(fg - fo) / abs(fo))
        g.history_accumulate()
        o.history_accumulate()
        g.dict_update()
        o.dict_update()
        worst["dict"] = max(worst["dict"], rel(to_np(g.get_dictionary()), o.get_dictionary()))
    say("worst relative errors", worst)
    assert all(v < 1e-10 for v in worst.values()), worst
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_minibatch_and_ragged_batch(prec):
    """B samples share one dictionary and fold in index order; a smaller B follows."""
    say(f"case minibatch {prec}")
    ph = pw = 64
    K = 8
    xs = synth_images(5, ph, pw)
    g, o = make_pair(K, 7, 7, ph, pw, lam=0.5, prec=prec, max_batch=3)
    for sl in (slice(0, 3), slice(3, 5)):
        U = to_np(g.code_update(xs[sl]))
        Uo = o.code_update(xs[sl])
        assert rel(U, Uo) < TOL[prec]
        fg = g.objective(xs[sl], torch.as_tensor(U))
        fo = o.objective(xs[sl], Uo)
        assert np.max(np.abs(np.array(fg) - fo) / np.abs(fo)) < TOL[prec]
        g.history_accumulate()
        o.history_accumulate()
        g.dict_update()
        o.dict_update()
        assert rel(to_np(g.get_dictionary()), o.get_dictionary()) < TOL[prec]
    assert g.count == 5
    g.close()


def test_fp32_128x128_k100_first_steps():
    """The throughput workload in FP32 against the FP64 oracle, first 2 steps."""
    wl = synth.WORKLOADS["ocsc_128x128_k100_f32"]
    say(f"case first steps {wl.name}")
    order = synth.pass_order(wl.n_images, wl.seed, 0)[:2]
    xs = synth.images(wl, order)
    g, o = make_pair(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, "f32",
                     wl.iters_code, wl.iters_dict, seed=wl.seed)
    for x in xs:
        U = g.code_update(x)
        Uo = o.code_update(x[None])
        assert rel(to_np(U), Uo) < 1e-3
        fg, fo = g.objective(x, U)[0], o.objective(x[None], Uo)[0]
        assert abs(fg - fo) / fo < 1e-3
        g.history_accumulate()
        o.history_accumulate()
        g.dict_update()
        o.dict_update()
        assert rel(to_np(g.get_dictionary()), o.get_dictionary()) < 1e-3
    g.close()


def test_call_order_errors():
    from paper_1706_06972_amd.ocsc import OCSC, OcscError, OCSC_E_STATE, OCSC_E_INVALID_ARG
    say("case call order errors")
    g = OCSC(4, 5, 5, 32, 32, 1.0, 1.0)
    with pytest.raises(OcscError) as e:
        g.history_accumulate()
    assert e.value.status == OCSC_E_STATE
    with pytest.raises(OcscError) as e:
        g.dict_update()
    assert e.value.status == OCSC_E_STATE
    g.set_dictionary(synth.initial_dictionary(4, 5, 5))
    x = torch.zeros((2, 32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(OcscError) as e:
        g.code_update(x)
    assert e.value.status == OCSC_E_INVALID_ARG
    g.code_update(x[:1])
    g.history_accumulate()
    with pytest.raises(OcscError) as e:
        g.history_accumulate()
    assert e.value.status == OCSC_E_STATE
    g.dict_update()
    g.close()


def test_runs_are_bitwise_deterministic():
    say("case determinism")
    xs = synth_images(3, 64, 64)
    outs = []
    for _ in range(2):
        g, _o = make_pair(16, 11, 11, 64, 64, prec="f32")
        codes = [to_np(g.step(x)) for x in xs]
        outs.append((codes, to_np(g.get_dictionary()), to_np(g.state("cinv"))))
        g.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])
