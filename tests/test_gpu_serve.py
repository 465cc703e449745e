"""Serving form: continuous batching over several grid sizes with a shared,
online-updated dictionary.

* Each request's codes are the same alone and in the mix, with the same launch
  shape (bitwise: a sample's arithmetic does not depend on the others in its
  batch).
* A served run with dictionary updates, replayed event by event on the FP64
  oracle (same batches, same fold points, same shared updates), agrees within
  the FP32 bound (norm-wise relative 1e-3 per quantity).
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests.gpu_util import rel, say, spectra, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_same_alone_and_in_the_mix():
    say("case serving: alone vs mix")
    from paper_1706_06972_amd.ocsc import OCSC
    from paper_1706_06972_amd.serve import Server, poisson_requests
    K, filt = 8, 11
    grids, shares = (64, 128, 256), (4, 2, 1)
    D0 = synth.initial_dictionary(K, filt, filt, 2)
    reqs = poisson_requests(60, 20000.0, grids, shares, seed=3)
    srv = Server(K, filt, D0, grids=grids, shares=shares, update_every=10 ** 9, keep_codes=True,
                 max_launch={64: 8, 128: 4, 256: 2}, slots={64: 64, 128: 32, 256: 16}, lam=0.5)
    m = srv.run(reqs)
    assert m["requests"] == 60 and m["dictionary_updates"] == 0
    assert any(len(ev[2]) > 1 for ev in srv.log if ev[0] == "code"), "no batching happened"
    alone = {n: OCSC(K, filt, filt, n, n, 0.5, 1.0, precision="f32") for n in grids}
    for n, g in alone.items():
        g.set_dictionary(D0)
        g.set_tuning(**srv.grids[n].model.tuning)   # the launch shape the server tuned (split planes round differently)
    for r in reqs:
        U = alone[r.grid].code_update(r.image)[0]
        assert torch.equal(U, r.codes), r.rid
    for g in alone.values():
        g.close()
    srv.close()


@pytest.mark.parametrize("cholesky", [False, True])
def test_served_run_matches_oracle_replay(cholesky):
    say(f"case serving: oracle replay with updates, precision form {cholesky}")
    from paper_1706_06972_amd.serve import Server, poisson_requests
    K, filt = 3, 5
    grids, shares = (32, 64), (2, 1)
    D0 = synth.initial_dictionary(K, filt, filt, 4)
    reqs = poisson_requests(30, 5000.0, grids, shares, seed=5)
    srv = Server(K, filt, D0, grids=grids, shares=shares, update_every=7, keep_codes=True,
                 max_launch={32: 4, 64: 2}, slots={32: 6, 64: 4}, lam=0.3, cholesky=cholesky)
    srv.run(reqs)
    assert srv.updates >= 3
    # replay on the oracle, one learner per grid
    orc = {n: O.OCSC(K, filt, filt, n, n, 0.3, 1.0) for n in grids}
    for o in orc.values():
        o.set_dictionary(D0)
    pend = {n: [] for n in grids}
    codes = {}
    by_id = {r.rid: r for r in reqs}

    def accumulate(n):
        if pend[n]:
            orc[n]._pending = pend[n]
            orc[n].history_accumulate()
            pend[n] = []
    for ev in srv.log:
        if ev[0] == "code":
            n, ids = ev[1], ev[2]
            U = orc[n].code_update(np.stack([by_id[i].image.astype(np.float64) for i in ids]))
            pend[n].extend(orc[n]._pending)
            for i, u in zip(ids, U):
                codes[i] = u
        elif ev[0] == "accumulate":
            accumulate(ev[1])
        else:
            for n in grids:
                accumulate(n)
            O.OCSC.dict_update_group([orc[n] for n in ev[1]])
    for n in grids:
        got = np.stack([to_np(r.codes) for r in reqs if r.grid == n])
        ref = np.stack([codes[r.rid] for r in reqs if r.grid == n])
        assert rel(got, ref) < 1e-3, n
        Dh = spectra(to_np(srv.grids[n].model.state("dict_hat")), (K,), n, n)
        assert rel(Dh, orc[n].Dh) < 1e-3, n
    srv.close()
