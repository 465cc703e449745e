"""Appended coding and the shared-dictionary update over several grids,
through the C ABI, against the FP64 oracle (norm-wise relative 1e-10 for FP64
contexts, 1e-3 for FP32), and the same-alone-and-in-the-mix property.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-3}
K, FH, FW = 3, 5, 5


def images(n, ph, pw, seed):
    wl = synth.Workload(name="t", pad_h=ph, pad_w=pw, content_h=ph // 2, content_w=pw // 2, k_true=4,
                        density=0.02, sigma_z=10.0, noise=0.01, K=4, filt_h=5, filt_w=5, lam=1.0, rho=1.0,
                        iters_code=10, iters_dict=10, batch=1, n_images=n, passes=1, precision="f64", seed=seed)
    return synth.images(wl, range(n))


def learner(n, prec, max_batch=4):
    from paper_1706_06972_amd.ocsc import OCSC
    g = OCSC(K, FH, FW, n, n, 0.3, 1.0, precision=prec, max_batch=max_batch)
    o = O.OCSC(K, FH, FW, n, n, 0.3, 1.0)
    D0 = synth.initial_dictionary(K, FH, FW, 5)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    return g, o


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_append_then_fold_equals_minibatch(prec):
    say(f"case code append {prec}")
    xs = images(4, 64, 64, 1)
    g, o = learner(64, prec)
    U1 = g.code_append(xs[0])
    U23 = g.code_append(xs[1:3])
    U4 = g.code_append(xs[3])
    Uo = o.code_update(xs)
    assert rel(to_np(torch.cat([U1, U23, U4])), Uo) < TOL[prec]
    g.history_accumulate()
    o.history_accumulate()
    g.dict_update()
    o.dict_update()
    assert rel(spectra(to_np(g.state("dict_hat")), (K,), 64, 64), o.Dh) < TOL[prec]
    assert g.count == 4
    # pending samples may not exceed max_batch
    from paper_1706_06972_amd import ocsc as L
    g.code_append(xs[:4])
    with pytest.raises(L.OcscError):
        g.code_append(xs[0])
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("grids", [(32, 64), (64, 256), (128,)])
def test_shared_dictionary_update_matches_oracle(prec, grids):
    say(f"case group update {prec} {grids}")
    from paper_1706_06972_amd.ocsc import OCSC
    pairs = [learner(n, prec) for n in grids]
    for step in range(2):
        for i, ((g, o), n) in enumerate(zip(pairs, grids)):
            xs = images(2, n, n, 10 * i + step)
            g.code_update(xs)
            o.code_update(xs)
            g.history_accumulate()
            o.history_accumulate()
        OCSC.dict_update_group([g for g, _ in pairs])
        O.OCSC.dict_update_group([o for _, o in pairs])
        for (g, o), n in zip(pairs, grids):
            assert rel(spectra(to_np(g.state("dict_hat")), (K,), n, n), o.Dh) < TOL[prec], (n, step)
            assert rel(to_np(g.state("V")).reshape(K, FH, FW), o.V) < TOL[prec]
            assert rel(spectra(to_np(g.state("theta")), (K,), n, n), o.Th) < TOL[prec]
    for g, _ in pairs:
        g.close()


def test_group_call_errors():
    say("case group errors")
    from paper_1706_06972_amd import ocsc as L
    from paper_1706_06972_amd.ocsc import OCSC
    a, _ = learner(32, "f64")
    b = OCSC(K + 1, FH, FW, 32, 32, 0.3, 1.0)
    with pytest.raises(L.OcscError) as e:
        OCSC.dict_update_group([a, a])
    assert e.value.status == L.OCSC_E_INVALID_ARG
    with pytest.raises(L.OcscError) as e:
        OCSC.dict_update_group([a])
    assert e.value.status == L.OCSC_E_STATE
    a.code_update(images(1, 32, 32, 0))
    a.history_accumulate()
    with pytest.raises(L.OcscError) as e:
        OCSC.dict_update_group([a, b])
    assert e.value.status == L.OCSC_E_INVALID_ARG
    a.close()
    b.close()
