"""Launch shapes of the code update and their autotuner, through the C ABI.

Every shape with two_pass 0 or 1 must give the codes and code spectra of the
default shape bit for bit (same arithmetic, same order of every sum), on grids
with one-pass and two-pass transforms and on batches that do not fill the last
Z-step workgroup.  The split plane step (two_pass 2: each plane over two
workgroups by row parity, the last radix-2 step of the column DFTs in the
Z-step; on 256 and 512 grids F row residues, so that a residue fits in LDS)
rounds differently: its shapes must agree with each other bit for bit
and with the default to rounding (norm-wise 1e-5 in FP32, 1e-12 in FP64).  The
autotuner must pick a valid shape, keep the learner state and refuse to run
over pending codes.  The default and the split shapes are checked against the
FP64 oracle by the parity tests.
"""
import itertools

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


def shapes(ph, pw):
    """Every valid shape: Z-step tiles x (workgroup sizes, one-pass grids, or
    column block x row block, two-pass grids)."""
    z = list(itertools.product((16, 32, 64), (1, 2, 4)))
    two = [(256, cb, rb, 1) for cb in (128, 256, 512) for rb in (4, 8, 16) if ph * cb <= 131072]
    if max(ph, pw) <= 128:
        planes = [(nt, 128, 8, 0) for nt in (256, 512, 1024) if nt * 4 <= ph * pw]
        if (ph, pw) in ((64, 64), (128, 128)):
            planes += two
    else:
        planes = two
    planes += [(nt, 128, 8, 2) for nt in (256, 512, 1024) if nt * 4 <= ph * pw]
    # sample groups of 0 (whole batch), 1 and 2 in turn (the batch has 3 samples)
    return [dict(plane_threads=nt, zstep_freqs=zf, zstep_samples=sb, col_bytes=cb, row_block=rb,
                 chunk_samples=(0, 1, 2)[i % 3], two_pass=tp)
            for i, ((nt, cb, rb, tp), (zf, sb)) in enumerate(itertools.product(planes, z))]


@pytest.mark.parametrize("prec,ph,pw,K", [("f32", 128, 128, 20), ("f64", 64, 64, 16), ("f32", 32, 64, 40),
                                          ("f32", 64, 64, 5),
                                          ("f32", 256, 256, 6), ("f64", 128, 128, 3), ("f64", 256, 512, 3),
                                          ("f32", 512, 512, 2)])
def test_every_shape_gives_the_same_bits(prec, ph, pw, K):
    say(f"case shapes {prec} {ph}x{pw} K={K}")
    from paper_1706_06972_amd.ocsc import OCSC
    B = 3
    xs = images(B, ph, pw, 7)
    g = OCSC(K, 5, 5, ph, pw, 0.5, 1.0, precision=prec, max_batch=B)
    g.set_dictionary(synth.initial_dictionary(K, 5, 5, 1))
    default = g.tuning
    U0 = to_np(g.code_update(xs))
    Z0 = to_np(g.state("zhat"))
    assert np.count_nonzero(U0) > 0
    tol = 1e-5 if prec == "f32" else 1e-12
    split = None          # codes and spectra of the first split shape
    for sh in shapes(ph, pw):
        g.set_tuning(**sh)
        assert g.tuning == sh
        U = to_np(g.code_update(xs))
        Z = to_np(g.state("zhat"))
        if sh["two_pass"] != 2:
            assert np.array_equal(U, U0), sh
            assert np.array_equal(Z, Z0), sh
        elif split is None:
            split = (U, Z)
            say(f"  split planes against the default: codes {rel(U, U0):.2e}, spectra {rel(Z, Z0):.2e}")
            assert rel(U, U0) < tol and rel(Z, Z0) < tol, sh
        else:
            assert np.array_equal(U, split[0]), sh
            assert np.array_equal(Z, split[1]), sh
    assert split is not None
    g.set_tuning(**default)
    g.close()


def test_invalid_shapes_are_refused():
    say("case invalid shapes")
    from paper_1706_06972_amd import ocsc as L
    from paper_1706_06972_amd.ocsc import OCSC
    small = OCSC(4, 5, 5, 32, 32, 0.5, 1.0, precision="f32")
    big = OCSC(4, 5, 5, 256, 256, 0.5, 1.0, precision="f32")
    for g, bad in ((small, dict(plane_threads=512)), (small, dict(plane_threads=128)), (small, dict(zstep_freqs=8)),
                   (small, dict(zstep_samples=3)), (big, dict(plane_threads=1024)), (small, dict(col_bytes=64)),
                   (small, dict(row_block=2)), (big, dict(row_block=32)), (small, dict(chunk_samples=3)),
                   (small, dict(two_pass=1)), (big, dict(two_pass=0)), (big, dict(two_pass=3)),
                   (small, dict(two_pass=3))):
        before = g.tuning
        with pytest.raises(L.OcscError) as e:
            g.set_tuning(**bad)
        assert e.value.status == L.OCSC_E_INVALID_ARG
        assert g.tuning == before
    assert small.tuning == dict(plane_threads=256, zstep_freqs=16, zstep_samples=1, col_bytes=128, row_block=8,
                                chunk_samples=0, two_pass=0)
    assert big.tuning["two_pass"] == 1
    big512 = OCSC(2, 5, 5, 512, 512, 0.5, 1.0, precision="f32")
    with pytest.raises(L.OcscError):
        big512.set_tuning(col_bytes=512)   # 512 rows x 512 bytes exceed the column workgroup's LDS
    big512.set_tuning(col_bytes=256, row_block=16)
    big512.close()
    small.close()
    big.close()


@pytest.mark.parametrize("prec,n,K", [("f64", 64, 8), ("f32", 128, 12)])
def test_autotune_keeps_the_learner(prec, n, K):
    """Two learners fed the same samples, one autotuned between its history
    accumulation (deferred fold) and its dictionary update, the other given the
    shape it picked: every result is bitwise the same, and both match the
    oracle."""
    say(f"case autotune {prec} {n}")
    from paper_1706_06972_amd import ocsc as L
    from paper_1706_06972_amd.ocsc import OCSC
    B = 2
    xs = images(2 * B, n, n, 3)
    D0 = synth.initial_dictionary(K, 5, 5, 2)
    a = OCSC(K, 5, 5, n, n, 0.5, 1.0, precision=prec, max_batch=B)
    b = OCSC(K, 5, 5, n, n, 0.5, 1.0, precision=prec, max_batch=B)
    o = O.OCSC(K, 5, 5, n, n, 0.5, 1.0)
    for m in (a, b, o):
        m.set_dictionary(D0)
    for step in range(2):
        x = xs[step * B:(step + 1) * B]
        Ua = to_np(a.code_update(x))
        Ub = to_np(b.code_update(x))
        Uo = o.code_update(x)
        assert np.array_equal(Ua, Ub)
        assert rel(Ua, Uo) < (1e-10 if prec == "f64" else 1e-3)
        if step == 0:
            with pytest.raises(L.OcscError) as e:
                b.autotune(B)
            assert e.value.status == L.OCSC_E_STATE
        for m in (a, b, o):
            m.history_accumulate()
        shape, ms = b.autotune(B)
        assert ms > 0 and b.tuning == shape
        b.set_tuning(**shape)
        a.set_tuning(**shape)   # a split-plane pick rounds differently from the default
        for m in (a, b, o):
            m.dict_update()
        for item in ("dict_hat", "G", "cinv", "V", "theta"):
            assert np.array_equal(to_np(a.state(item)), to_np(b.state(item))), item
        assert a.count == b.count == (step + 1) * B
    with pytest.raises(L.OcscError) as e:
        b.autotune(B + 1)
    assert e.value.status == L.OCSC_E_INVALID_ARG
    a.close()
    b.close()
