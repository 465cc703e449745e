"""Parity of the library's evaluation calls (objective terms, online surrogate,
diagnostics), of the kept history, of warm-start DictOCSC and of checkpoint
restore, through the C ABI, against the FP64 oracle.

Tolerances as elsewhere: norm-wise relative 1e-10 (FP64 contexts) and 1e-3
(FP32 contexts); a restored learner must continue bit for bit.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np, unpack_cinv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-3}
K, FH, FW, PH, PW = 8, 7, 7, 64, 64


def images(n, seed=0):
    wl = synth.WORKLOADS["ocsc_64x64_k16_f64"]
    return synth.images(wl, synth.pass_order(wl.n_images, seed, 0)[:n])


def pair(prec="f64", keep=False, warm=False, jd=10, max_batch=1, lam=0.5):
    from paper_1706_06972_amd.ocsc import OCSC
    g = OCSC(K, FH, FW, PH, PW, lam, 1.0, iters_dict=jd, max_batch=max_batch, precision=prec,
             keep_history=keep, warm_start=warm)
    o = O.OCSC(K, FH, FW, PH, PW, lam, 1.0, iters_dict=jd, keep_history=keep, warm_start=warm)
    D0 = synth.initial_dictionary(K, FH, FW, 0)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    return g, o


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_objective_terms_and_psnr(prec):
    say(f"case objective terms {prec}")
    xs = images(3)
    g, o = pair(prec)
    for x in xs:
        U = g.code_update(x)
        Uo = o.code_update(x[None])
        (data, l1), = g.objective_terms(x, U)
        data_o, l1_o = o.objective_terms(x[None], Uo)[0]
        assert abs(data - data_o) / data_o < TOL[prec]
        assert abs(l1 - l1_o) / l1_o < TOL[prec]
        f = g.objective(x, U)[0]
        assert abs(f - (data + 0.5 * l1)) <= 1e-12 * abs(f)
        # PSNR of the paper's evaluation from the data term
        rec_err = 2.0 * data
        p_gpu = 10.0 * np.log10(255.0 ** 2 * PH * PW / rec_err)
        rec_o = O.idft2_real(np.sum(o.Dh * O.dft2(Uo[0]), axis=0), (PH, PW))
        assert abs(p_gpu - O.psnr(x, rec_o)) < (1e-9 if prec == "f64" else 1e-3)
        g.history_accumulate()
        o.history_accumulate()
        g.dict_update()
        o.dict_update()
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_kept_history_and_surrogate(prec):
    """H, the running sums and F_t at the dictionary and at given filters."""
    say(f"case surrogate {prec}")
    xs = images(5)
    g, o = pair(prec, keep=True, max_batch=2)
    for sl in (slice(0, 2), slice(2, 3), slice(3, 5)):
        g.code_update(xs[sl], want_codes=(sl.start != 2))   # one call keeps no codes
        o.code_update(xs[sl])
        g.history_accumulate()
        o.history_accumulate()
        Hg = unpack_cinv(to_np(g.state("H")), K, PH, PW)
        assert rel(Hg, o.H) < TOL[prec]
        sums = to_np(g.state("sums"))
        assert abs(sums[0] - o.sum_xh2 / (PH * PW)) / sums[0] < 1e-12 * (1 if prec == "f64" else 1e6)
        assert abs(sums[1] - o.l1_sum) / o.l1_sum < TOL[prec]
        # deferred fold is applied before the surrogate reads G
        fg = g.surrogate()
        fo = o.surrogate_at(o.Dh)
        assert abs(fg - fo) / abs(fo) < TOL[prec], (fg, fo)
        g.dict_update()
        o.dict_update()
        V = o.V
        fg = g.surrogate(V)
        fo = o.surrogate_at(O.dft2(O.zero_pad(V, (PH, PW))))
        assert abs(fg - fo) / abs(fo) < TOL[prec], (fg, fo)
    assert g.count == 5
    g.close()


def test_online_surrogate_is_monotone_on_gpu():
    """P16 on the device: with DictOCSC run to convergence, F_t(V_t) <= F_t(V_{t-1})."""
    say("case surrogate monotone f64 jd=600")
    from paper_1706_06972_amd.ocsc import OCSC
    xs = images(6)[:, :32, :32].copy()
    g = OCSC(4, 5, 5, 32, 32, 0.1, 1.0, iters_dict=600, keep_history=True)
    g.set_dictionary(synth.initial_dictionary(4, 5, 5))
    V_prev = None
    for x in xs:
        g.code_update(x, want_codes=False)
        g.history_accumulate()
        if V_prev is not None:
            before = g.surrogate(V_prev)
        g.dict_update()
        V = g.state("V").reshape(4, 5, 5).clone()
        if V_prev is not None:
            after = g.surrogate(V)
            assert after <= before + 1e-10 * abs(before), (before, after)
        V_prev = V
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_diagnostics(prec):
    say(f"case diagnostics {prec}")
    xs = images(3)
    g, o = pair(prec)
    dg = g.diagnostics()
    do = o.diagnostics()
    assert abs(dg["dict_norm"] - do["dict_norm"]) / do["dict_norm"] < TOL[prec]
    for x in xs:
        g.step(x)
        o.step(x[None])
        dg = g.diagnostics()
        do = o.diagnostics()
        assert abs(dg["primal_residual"] - do["primal_residual"]) / do["primal_residual"] < TOL[prec]
        assert abs(dg["dict_norm"] - do["dict_norm"]) / do["dict_norm"] < TOL[prec]
        assert rel(dg["V_norms"], do["V_norms"]) < TOL[prec]
        assert rel(dg["D_norms"], do["D_norms"]) < TOL[prec]
        assert max(dg["V_norms"]) <= 1.0 + (1e-12 if prec == "f64" else 1e-6)
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_warm_start_trajectory(prec):
    say(f"case warm start {prec}")
    xs = images(6)
    g, o = pair(prec, warm=True, max_batch=2)
    # samples one by one, a batch of two, and two accumulations before one update
    g.step(xs[0]); o.step(xs[0][None])
    g.step(xs[1:3]); o.step(xs[1:3])
    for x in xs[3:5]:
        g.code_update(x); o.code_update(x[None])
        g.history_accumulate(); o.history_accumulate()
    g.dict_update(); o.dict_update()
    g.dict_update(); o.dict_update()      # no new sample: continues the same run
    tol = TOL[prec]
    assert rel(spectra(to_np(g.state("dict_hat")), (K,), PH, PW), o.Dh) < tol
    assert rel(to_np(g.state("V")).reshape(K, FH, FW), o.V) < tol
    assert rel(spectra(to_np(g.state("theta")), (K,), PH, PW), o.Th) < tol
    rhs_o = o.G + o.rho_d * (O.dft2(O.zero_pad(o.V, (PH, PW))) - o.Th)
    assert rel(spectra(to_np(g.state("rhs")), (K,), PH, PW), rhs_o) < tol
    U = to_np(g.code_update(xs[5]))
    assert rel(U, o.code_update(xs[5][None])) < tol
    g.close()


@pytest.mark.parametrize("prec,keep,warm", [("f64", False, False), ("f32", False, False),
                                             ("f64", True, True), ("f32", True, True)])
def test_checkpoint_restore_is_bitwise(prec, keep, warm):
    """P18 on the device: 3 steps, copy the checkpoint state into a fresh
    learner, 3 more steps on both: codes, dictionary and surrogate agree bit for bit."""
    say(f"case checkpoint {prec} keep={keep} warm={warm}")
    from paper_1706_06972_amd.ocsc import OCSC
    xs = images(6)

    def learner():
        g = OCSC(K, FH, FW, PH, PW, 0.5, 1.0, precision=prec, keep_history=keep, warm_start=warm)
        g.set_dictionary(synth.initial_dictionary(K, FH, FW, 0))
        return g
    a = learner()
    for x in xs[:3]:
        a.step(x)
    b = learner()
    b.set_dictionary(np.zeros((K, FH, FW)))
    items = ["dict_hat", "G", "cinv"] + (["H", "sums"] if keep else []) + (["V", "theta", "rhs"] if warm else [])
    for it in items:
        b.set_state(it, a.state(it))
    b.count = a.count
    for x in xs[3:]:
        ua, ub = a.step(x), b.step(x)
        assert torch.equal(ua, ub)
    assert torch.equal(a.state("dict_hat"), b.state("dict_hat"))
    if keep:
        assert a.surrogate() == b.surrogate()
    assert a.count == b.count == 6
    a.close()
    b.close()


def test_flag_gated_calls():
    say("case flag-gated calls")
    from paper_1706_06972_amd import ocsc as L
    g, _ = pair("f64")
    with pytest.raises(L.OcscError) as e:
        g.surrogate()
    assert e.value.status == L.OCSC_E_STATE
    for item in ("H", "sums", "rhs"):
        with pytest.raises(L.OcscError) as e:
            g.state(item)
        assert e.value.status == L.OCSC_E_INVALID_ARG
    g.close()


def test_evaluation_layer_matches_oracle():
    """Test-set objective (codes re-solved), PSNR, the code-ADMM study and the
    relative-change stopping rule, FP64 against the oracle."""
    say("case evaluation layer f64")
    from paper_1706_06972_amd import evaluate as E
    from paper_1706_06972_amd.ocsc import OCSC
    xs = images(8)
    train, test = xs[:5], xs[5:]
    g, o = pair("f64", max_batch=2)
    for x in train:
        g.step(x)
        o.step(x[None])
    # test objective: mean over the test set with codes re-solved, nothing folded
    t_gpu = E.test_objective(g, test)
    t_or = float(np.mean([o.objective(x[None], o.code_update(x[None]))[0] for x in test]))
    assert abs(t_gpu - t_or) / t_or < 1e-10
    assert g.count == 5
    p_gpu = E.psnr(g, test)
    p_or = []
    for x in test:
        U = o.code_update(x[None])[0]
        rec = O.idft2_real(np.sum(o.Dh * O.dft2(U), axis=0), (PH, PW))
        p_or.append(O.psnr(x, rec))
    assert abs(p_gpu - float(np.mean(p_or))) < 1e-8
    # code-ADMM objective after J iterations
    D0 = synth.initial_dictionary(K, FH, FW, 0)
    study = E.code_admm_study(lambda J: OCSC(K, FH, FW, PH, PW, 0.5, 1.0, iters_code=J), D0, test, [1, 5, 20])
    for rec in study:
        m = O.OCSC(K, FH, FW, PH, PW, 0.5, 1.0, iters_code=rec["iters"])
        m.set_dictionary(D0)
        ref = float(np.mean([m.objective(x[None], m.code_update(x[None]))[0] for x in test]))
        assert abs(rec["objective"] - ref) / ref < 1e-10
    assert study[-1]["objective"] < study[0]["objective"]
    g.close()


def test_learn_stops_on_relative_change():
    say("case learn with stopping rule")
    from paper_1706_06972_amd import evaluate as E
    xs = images(3)[:, :32, :32].copy()
    from paper_1706_06972_amd.ocsc import OCSC
    g = OCSC(4, 5, 5, 32, 32, 0.1, 1.0)
    g.set_dictionary(synth.initial_dictionary(4, 5, 5))
    hist = E.learn(g, xs, passes=40, tol=1e-2, test_xs=xs[:1])
    assert hist[0]["rel_change_Z"] is None and hist[0]["rel_change_D"] > 0
    last = hist[-1]
    stopped = last["rel_change_Z"] is not None and last["rel_change_Z"] < 1e-2 and last["rel_change_D"] < 1e-2
    assert stopped or len(hist) == 40
    assert all(np.isfinite(h["test_objective"]) for h in hist)
    g.close()
