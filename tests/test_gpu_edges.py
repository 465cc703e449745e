"""Edge and degenerate cases of the HIP library (through the C ABI), against the
FP64 oracle and, where one exists, a closed form:

* the largest K of the Sherman-Morrison form in each precision (C_p held in
  LDS: K = 92 in FP64, K = 128 in FP32);
* FP32 minibatches folded sixteen samples at a time on the matrix cores,
  with a ragged last block and K not a multiple of 16;
* filters as large as the grid (the crop of the V-step keeps every tap);
* lambda = 0 (no shrinkage: dense codes);
* an all-zero sample: zero codes, an unchanged history, and the zero
  dictionary that the cold-start DictOCSC then returns; coding against that
  dictionary gives zero codes and the objective (1/2)||x||^2;
* K = 1 with the unit impulse as the filter: the code problem is the lasso with
  the identity operator, whose minimiser is the soft threshold S_lambda(x); the
  scaled ADMM reaches it to rounding within 60 iterations.

Tolerances: norm-wise relative error 1e-10 (FP64) and 1e-3 (FP32) against the
oracle; the closed forms as stated per test.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np, unpack_cinv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-3}


def images(n, ph, pw, filt=5, seed=0):
    wl = synth.Workload(name="t", pad_h=ph, pad_w=pw, content_h=ph - filt + 1, content_w=pw - filt + 1, k_true=8,
                        density=0.02, sigma_z=10.0, noise=0.01, K=8, filt_h=filt, filt_w=filt, lam=1.0, rho=1.0,
                        iters_code=10, iters_dict=10, batch=1, n_images=n, passes=1, precision="f64", seed=seed)
    return synth.images(wl, range(n))


def learn_both(K, fh, fw, ph, pw, prec, xs, lam=0.5, rho=1.0, jz=10, jd=10, D0=None):
    """Feed the same samples to the library and the oracle; return the worst
    relative error per quantity and the last codes of both."""
    from paper_1706_06972_amd.ocsc import OCSC
    g = OCSC(K, fh, fw, ph, pw, lam, rho, iters_code=jz, iters_dict=jd, precision=prec)
    o = O.OCSC(K, fh, fw, ph, pw, lam, rho, iters_code=jz, iters_dict=jd)
    D0 = synth.initial_dictionary(K, fh, fw, 0) if D0 is None else D0
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    worst = {}

    def note(key, v):
        worst[key] = max(worst.get(key, 0.0), v)

    U = Uo = None
    for x in xs:
        U = to_np(g.code_update(x))
        Uo = o.code_update(x[None])
        note("codes", rel(U, Uo))
        g.history_accumulate()
        o.history_accumulate()
        note("G", rel(spectra(to_np(g.state("G")), (K,), ph, pw), o.G))
        g.dict_update()
        o.dict_update()
        note("dict_hat", rel(spectra(to_np(g.state("dict_hat")), (K,), ph, pw), o.Dh))
        note("D", rel(to_np(g.get_dictionary()), o.get_dictionary()))
    g.close()
    return worst, U, Uo


@pytest.mark.parametrize("prec,K", [("f64", 92), ("f32", 128)])
def test_largest_k_of_the_sherman_morrison_form(prec, K):
    say(f"case largest K {prec} K={K}")
    xs = images(2, 32, 32)
    worst, U, Uo = learn_both(K, 5, 5, 32, 32, prec, xs)
    say(f"  errors {worst}")
    assert np.count_nonzero(Uo) > 0
    assert all(v < TOL[prec] for v in worst.values()), worst


@pytest.mark.parametrize("prec,K", [("f64", 92), ("f32", 128), ("f32", 100), ("f64", 16)])
def test_minibatch_fold_at_the_largest_k(prec, K):
    """Four samples coded together and folded in one sweep (blocks of three,
    then one), at the largest K of each precision and at the compiled K."""
    say(f"case minibatch fold {prec} K={K}")
    from paper_1706_06972_amd.ocsc import OCSC
    B = 4
    xs = images(B, 32, 32, seed=9)
    g = OCSC(K, 5, 5, 32, 32, 0.5, 1.0, precision=prec, max_batch=B)
    o = O.OCSC(K, 5, 5, 32, 32, 0.5, 1.0)
    D0 = synth.initial_dictionary(K, 5, 5, 0)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    U = to_np(g.code_update(xs))
    Uo = o.code_update(xs)
    g.history_accumulate()
    o.history_accumulate()
    g.dict_update()
    o.dict_update()
    errs = {"codes": rel(U, Uo),
            "G": rel(spectra(to_np(g.state("G")), (K,), 32, 32), o.G),
            "C": rel(unpack_cinv(to_np(g.state("cinv")), K, 32, 32), o.C),
            "D": rel(to_np(g.get_dictionary()), o.get_dictionary())}
    say(f"  errors {errs}")
    assert all(v < TOL[prec] for v in errs.values()), errs
    g.close()


@pytest.mark.parametrize("K,B", [(37, 37), (100, 33), (16, 48)])
def test_minibatch_fold_in_blocks_of_sixteen(K, B):
    """FP32: a minibatch of B samples folds sixteen at a time on the matrix
    cores (whole blocks, then a ragged one; K not a multiple of 16 pads the
    blocks), against the oracle's sample-by-sample recursion; then a second
    minibatch on the updated dictionary."""
    say(f"case matrix-core fold f32 K={K} B={B}")
    from paper_1706_06972_amd.ocsc import OCSC
    xs = images(2 * B, 32, 32, seed=11)
    g = OCSC(K, 5, 5, 32, 32, 0.5, 1.0, precision="f32", max_batch=B)
    o = O.OCSC(K, 5, 5, 32, 32, 0.5, 1.0)
    D0 = synth.initial_dictionary(K, 5, 5, 1)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    for step in range(2):
        batch = xs[step * B:(step + 1) * B]
        U = to_np(g.code_update(batch))
        Uo = o.code_update(batch)
        g.history_accumulate()
        o.history_accumulate()
        g.dict_update()
        o.dict_update()
        errs = {"codes": rel(U, Uo),
                "G": rel(spectra(to_np(g.state("G")), (K,), 32, 32), o.G),
                "C": rel(unpack_cinv(to_np(g.state("cinv")), K, 32, 32), o.C),
                "D": rel(to_np(g.get_dictionary()), o.get_dictionary())}
        say(f"  minibatch {step}: errors {errs}")
        assert all(v < TOL["f32"] for v in errs.values()), errs
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ph,pw", [(32, 32), (64, 32)])
def test_filters_as_large_as_the_grid(prec, ph, pw):
    say(f"case full-size filters {prec} {ph}x{pw}")
    xs = images(2, ph, pw, seed=4)
    worst, U, Uo = learn_both(3, ph, pw, ph, pw, prec, xs, lam=0.2)
    say(f"  errors {worst}")
    assert np.count_nonzero(Uo) > 0
    assert all(v < TOL[prec] for v in worst.values()), worst


def test_lambda_zero_gives_dense_codes():
    say("case lambda = 0")
    xs = images(2, 64, 64, seed=5)
    worst, U, Uo = learn_both(4, 7, 7, 64, 64, "f64", xs, lam=0.0)
    say(f"  errors {worst}")
    assert np.count_nonzero(Uo) > 0.9 * Uo.size
    assert all(v < 1e-10 for v in worst.values()), worst


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zero_sample_and_the_zero_dictionary(prec):
    say(f"case zero sample {prec}")
    from paper_1706_06972_amd.ocsc import OCSC
    K, ph, pw = 4, 32, 32
    g = OCSC(K, 5, 5, ph, pw, 1.0, 1.0, precision=prec)
    g.set_dictionary(synth.initial_dictionary(K, 5, 5, 0))
    C0 = to_np(g.state("cinv"))
    U = to_np(g.code_update(np.zeros((1, ph, pw))))
    assert not np.any(U)
    g.history_accumulate()
    assert not np.any(to_np(g.state("G")))
    assert np.array_equal(to_np(g.state("cinv")), C0)
    g.dict_update()
    assert not np.any(to_np(g.get_dictionary()))
    assert not np.any(to_np(g.state("dict_hat")))
    # coding against the zero dictionary: zero codes, objective (1/2)||x||^2
    x = images(1, ph, pw, seed=6)
    U = g.code_update(x)
    assert not np.any(to_np(U))
    f = g.objective(x, U)[0]
    xr = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    ref = 0.5 * float(np.sum(xr ** 2))
    assert abs(f - ref) / ref < (1e-12 if prec == "f64" else 1e-6)
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unit_impulse_filter_gives_the_soft_threshold(prec):
    say(f"case unit impulse {prec}")
    from paper_1706_06972_amd.ocsc import OCSC
    lam, ph, pw = 0.7, 64, 32
    rng = np.random.default_rng(3)
    x = rng.normal(0.0, 2.0, (ph, pw))
    if prec == "f32":
        x = x.astype(np.float32).astype(np.float64)
    g = OCSC(1, 1, 1, ph, pw, lam, 1.0, iters_code=60, precision=prec)
    g.set_dictionary(np.ones((1, 1, 1)))
    U = to_np(g.code_update(x))[0, 0]
    S = np.sign(x) * np.maximum(np.abs(x) - lam, 0.0)
    assert rel(U, S) < (1e-12 if prec == "f64" else 1e-5)
    o = O.OCSC(1, 1, 1, ph, pw, lam, 1.0, iters_code=60)
    o.set_dictionary(np.ones((1, 1, 1)))
    assert rel(U, o.code_update(x[None])[0, 0]) < TOL[prec]
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_non_finite_input_is_reported(prec):
    """A sample with a NaN: the asynchronous calls enqueue as usual; the calls
    that bring results back to the host report OCSC_E_NUMERIC."""
    say(f"case non-finite input {prec}")
    from paper_1706_06972_amd import ocsc as L
    from paper_1706_06972_amd.ocsc import OCSC
    K, ph, pw = 4, 32, 32
    g = OCSC(K, 5, 5, ph, pw, 1.0, 1.0, precision=prec)
    g.set_dictionary(synth.initial_dictionary(K, 5, 5, 0))
    x = images(1, ph, pw, seed=8)
    x[0, 3, 4] = np.nan
    U = g.code_update(x)
    with pytest.raises(L.OcscError) as e:
        g.objective(x, U)
    assert e.value.status == L.OCSC_E_NUMERIC
    g.history_accumulate()
    g.dict_update()
    with pytest.raises(L.OcscError) as e:
        g.diagnostics()
    assert e.value.status == L.OCSC_E_NUMERIC
    g.close()
