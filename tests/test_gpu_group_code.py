"""One persistent launch coding batches on several grids (ocsc_code_update_group)
against separate per-grid code updates, through the C ABI.

The grouped launch runs the same device bodies as the per-grid kernels, so
codes, code spectra, sample spectra and everything learned from them must be
equal bit for bit; the per-grid path itself is checked against the FP64
oracle by the parity tests (and here once more on the group's codes).
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def images(n, ph, pw, seed):
    wl = synth.Workload(name="t", pad_h=ph, pad_w=pw, content_h=ph // 2, content_w=pw // 2, k_true=4,
                        density=0.02, sigma_z=10.0, noise=0.01, K=4, filt_h=5, filt_w=5, lam=1.0, rho=1.0,
                        iters_code=10, iters_dict=10, batch=1, n_images=n, passes=1, precision="f64", seed=seed)
    return synth.images(wl, range(n))


def pair(K, n, prec, B, **kw):
    from paper_1706_06972_amd.ocsc import OCSC
    D0 = synth.initial_dictionary(K, 5, 5, 4)
    a = OCSC(K, 5, 5, n[0], n[1], 0.5, 1.0, precision=prec, max_batch=B, **kw)
    b = OCSC(K, 5, 5, n[0], n[1], 0.5, 1.0, precision=prec, max_batch=B, **kw)
    a.set_dictionary(D0)
    b.set_dictionary(D0)
    return a, b


CASES = {
    "f32-mix": ("f32", 12, [((64, 64), 3), ((128, 128), 2), ((256, 256), 2), ((512, 512), 1)]),
    "f64-mix": ("f64", 8, [((32, 32), 2), ((64, 128), 1), ((256, 512), 2)]),
    "f32-one": ("f32", 20, [((128, 64), 3)]),
    "f32-big": ("f32", 3, [((512, 256), 2), ((256, 256), 1)]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_group_launch_equals_per_grid_launches(case):
    prec, K, grids = CASES[case]
    say(f"case grouped coding {case}")
    from paper_1706_06972_amd.ocsc import OCSC
    pairs = [pair(K, n, prec, B) for n, B in grids]
    xs = [images(B, n[0], n[1], 11 + i) for i, (n, B) in enumerate(grids)]
    for step in range(2):
        codes = OCSC.code_update_group([a for a, _ in pairs], xs)
        for (a, b), x, U in zip(pairs, xs, codes):
            Ub = b.code_update(x)
            assert np.count_nonzero(to_np(Ub)) > 0
            assert np.array_equal(to_np(U), to_np(Ub))
            for item in ("zhat", "xhat"):
                assert np.array_equal(to_np(a.state(item)), to_np(b.state(item))), item
            a.history_accumulate()
            b.history_accumulate()
            a.dict_update()
            b.dict_update()
            assert np.array_equal(to_np(a.state("dict_hat")), to_np(b.state("dict_hat")))
        xs = [x[::-1].copy() for x in xs]
    for a, b in pairs:
        a.close()
        b.close()


def test_group_codes_match_the_oracle():
    say("case grouped coding vs oracle")
    from paper_1706_06972_amd.ocsc import OCSC
    K = 6
    grids = [((64, 64), 2), ((256, 256), 1)]
    D0 = synth.initial_dictionary(K, 5, 5, 4)
    models, oracles, xs = [], [], []
    for i, (n, B) in enumerate(grids):
        m = OCSC(K, 5, 5, n[0], n[1], 0.5, 1.0, precision="f64", max_batch=B)
        o = O.OCSC(K, 5, 5, n[0], n[1], 0.5, 1.0)
        m.set_dictionary(D0)
        o.set_dictionary(D0)
        models.append(m)
        oracles.append(o)
        xs.append(images(B, n[0], n[1], 30 + i))
    codes = OCSC.code_update_group(models, xs)
    for U, o, x in zip(codes, oracles, xs):
        assert rel(to_np(U), o.code_update(x)) < 1e-10
    for m in models:
        m.close()


def test_group_with_kept_history_and_precision_form():
    """Members with the kept history and with the matrix-core history (the
    last iterate also goes out frequency-major) learn the same bits."""
    say("case grouped coding keep/cholesky")
    from paper_1706_06972_amd.ocsc import OCSC
    K = 12
    pa = pair(K, (64, 64), "f32", 4, cholesky=True)
    pb = pair(K, (128, 128), "f32", 2, keep_history=True)
    xa, xb = images(4, 64, 64, 5), images(2, 128, 128, 6)
    OCSC.code_update_group([pa[0], pb[0]], [xa, xb], want_codes=False)
    pa[1].code_update(xa, want_codes=False)
    pb[1].code_update(xb, want_codes=False)
    for a, b in (pa, pb):
        a.history_accumulate()
        b.history_accumulate()
        for item in ("H", "cinv", "G", "sums"):
            assert np.array_equal(to_np(a.state(item)), to_np(b.state(item))), item
        assert a.surrogate() == b.surrogate()
        a.close()
        b.close()


def test_group_call_errors():
    say("case grouped coding errors")
    from paper_1706_06972_amd import ocsc as L
    from paper_1706_06972_amd.ocsc import OCSC
    a, _ = pair(4, (32, 32), "f32", 2)
    b, _ = pair(4, (64, 64), "f64", 2)
    x32, x64 = images(2, 32, 32, 1), images(2, 64, 64, 1)
    for models, xs in (([a, a], [x32, x32]), ([a, b], [x32, x64]), ([a], [images(3, 32, 32, 1)])):
        with pytest.raises(L.OcscError) as e:
            OCSC.code_update_group(models, xs)
        assert e.value.status == L.OCSC_E_INVALID_ARG
    a.close()
    b.close()
