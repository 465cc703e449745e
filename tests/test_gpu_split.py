"""The split plane step (launch shape two_pass = 2) against the FP64 oracle,
through the C ABI.

With two_pass = 2 each plane of the code update runs on F workgroups, one
per row residue (F = 2 on grids up to 128; 2 to 16 on 256 and 512 grids, so
that a residue's rows fit in LDS), and the last radix-F step of its column
DFTs runs in the Z-step (eq. fcsc_code: the U-step and the dual on the rows
of one residue; the spectrum of U - W formed from the F column DFTs).  Whole
learning steps (code update, history, DictOCSC) are compared with the oracle
per quantity at the suite's tolerances (norm-wise 1e-10 FP64, 1e-3 FP32):
grids of every height up to 512 (F = 2, 4, 8 and 16), single samples and
ragged minibatches, and
the 128x128, K = 100 FP32 workload at B = 1.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np, unpack_cinv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-3}


def images(n, ph, pw, seed):
    wl = synth.Workload(name="t", pad_h=ph, pad_w=pw, content_h=ph - 8, content_w=pw - 8, k_true=6,
                        density=0.02, sigma_z=10.0, noise=0.01, K=6, filt_h=7, filt_w=7, lam=1.0, rho=1.0,
                        iters_code=10, iters_dict=10, batch=1, n_images=n, passes=1, precision="f64", seed=seed)
    return synth.images(wl, range(n))


@pytest.mark.parametrize("prec,ph,pw,K,batches,nt", [
    ("f64", 32, 32, 4, (1, 1), 256),
    ("f64", 64, 128, 6, (1, 2), 512),
    ("f64", 128, 32, 5, (3, 2), 256),
    ("f64", 128, 128, 7, (1, 1), 1024),
    ("f32", 32, 64, 9, (2, 1), 256),
    ("f32", 128, 128, 12, (1, 3), 512),
    ("f32", 256, 256, 4, (1, 2), 512),
    ("f64", 256, 256, 3, (1, 1), 512),
    ("f32", 256, 512, 2, (2, 1), 1024),
    ("f64", 512, 256, 2, (1, 1), 512),
    ("f32", 512, 512, 3, (1, 1), 512),
    ("f64", 512, 512, 2, (1, 1), 1024),
])
def test_split_planes_match_oracle(prec, ph, pw, K, batches, nt):
    say(f"case split planes {prec} {ph}x{pw} K={K} batches={batches} threads={nt}")
    from paper_1706_06972_amd.ocsc import OCSC
    fh = fw = 5
    xs = images(sum(batches), ph, pw, 11)
    g = OCSC(K, fh, fw, ph, pw, 0.5, 1.0, precision=prec, max_batch=max(batches))
    o = O.OCSC(K, fh, fw, ph, pw, 0.5, 1.0)
    D0 = synth.initial_dictionary(K, fh, fw, 4)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    g.set_tuning(two_pass=2, plane_threads=nt)
    tol = TOL[prec]
    i0 = 0
    for B in batches:
        x = xs[i0:i0 + B]
        i0 += B
        U = to_np(g.code_update(x))
        Uo = o.code_update(x)
        assert np.count_nonzero(Uo) > 0
        e = {"codes": rel(U, Uo)}
        zh = spectra(to_np(g.state("zhat")), (max(batches), K), ph, pw)[:B]   # the workspace holds max_batch slots
        e["zhat"] = rel(zh, np.stack([p[0] for p in o._pending[-B:]]))
        g.history_accumulate()
        o.history_accumulate()
        e["G"] = rel(spectra(to_np(g.state("G")), (K,), ph, pw), o.G)
        e["C"] = rel(unpack_cinv(to_np(g.state("cinv")), K, ph, pw), o.C)
        g.dict_update()
        o.dict_update()
        e["dict_hat"] = rel(spectra(to_np(g.state("dict_hat")), (K,), ph, pw), o.Dh)
        e["dict"] = rel(to_np(g.get_dictionary()), o.get_dictionary())
        say("  B=%d: " % B + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
        for k, v in e.items():
            assert v < tol, (k, v)
    assert g.tuning["two_pass"] == 2
    g.close()


def test_split_planes_128x128_k100_f32():
    """The throughput workload's first two steps with split planes, B = 1."""
    wl = synth.WORKLOADS["ocsc_128x128_k100_f32"]
    say("case split planes 128x128 K=100 FP32, 2 steps")
    from paper_1706_06972_amd.ocsc import OCSC
    g = OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, iters_code=wl.iters_code,
             iters_dict=wl.iters_dict, precision="f32")
    o = O.OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, iters_code=wl.iters_code,
               iters_dict=wl.iters_dict)
    D0 = synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed)
    g.set_dictionary(D0)
    o.set_dictionary(D0)
    g.set_tuning(two_pass=2, plane_threads=512, zstep_freqs=32)
    for i in synth.pass_order(wl.n_images, wl.seed, 0)[:2]:
        x = synth.images(wl, [int(i)])
        U = to_np(g.code_update(x))
        Uo = o.code_update(x)
        e = {"codes": rel(U, Uo)}
        g.history_accumulate()
        o.history_accumulate()
        g.dict_update()
        o.dict_update()
        e["dict"] = rel(to_np(g.get_dictionary()), o.get_dictionary())
        say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
        assert all(v < TOL["f32"] for v in e.values()), e
    g.close()
