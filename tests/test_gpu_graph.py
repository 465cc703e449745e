"""The steady-state step captured as a HIP graph: every replay (two steps)
must equal, bit for bit, the same two steps run by eager calls on a twin
learner, with eager work and synchronisations between the replays."""
import pytest

import synth
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replays_match_eager_steps(prec):
    say(f"case graph replay {prec}")
    from paper_1706_06972_amd import ocsc as L
    from paper_1706_06972_amd.ocsc import OCSC
    K, n, filt = 8, 64, 7
    wl = synth.WORKLOADS["ocsc_64x64_k16_f64"]
    xs = synth.images(wl, range(6))
    D0 = synth.initial_dictionary(K, filt, filt, 1)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = OCSC(K, filt, filt, n, n, 0.5, 1.0, precision=prec)
    e = OCSC(K, filt, filt, n, n, 0.5, 1.0, precision=prec)
    g.set_dictionary(D0)
    e.set_dictionary(D0)
    dt = torch.float64 if prec == "f64" else torch.float32
    xbuf = torch.empty((2, 1, n, n), dtype=dt, device="cuda")
    cbuf = torch.empty((2, 1, K, n, n), dtype=dt, device="cuda")
    h = L.ocsc_graph_create(g.ctx, xbuf, 1, cbuf)
    assert g.count == 0                      # capturing runs nothing
    for r in range(3):
        with torch.cuda.stream(st):
            xbuf.copy_(torch.as_tensor(xs[2 * r:2 * r + 2], dtype=dt, device="cuda")[:, None])
        L.ocsc_graph_launch(g.ctx, h)
        U = []
        for s in range(2):
            U.append(e.code_update(xs[2 * r + s]))
            e.history_accumulate()
            e.dict_update()
        st.synchronize()
        torch.cuda.synchronize()
        for s in range(2):
            assert torch.equal(cbuf[s], U[s]), (r, s)
        assert torch.equal(g.state("dict_hat"), e.state("dict_hat")), r
        assert torch.equal(g.state("cinv"), e.state("cinv")), r
        # eager work on the graph's learner between replays
        with torch.cuda.stream(st):
            f = g.objective(xs[2 * r], cbuf[0])
        assert f[0] > 0
    assert g.count == e.count == 6
    L.ocsc_graph_destroy(h)
    g.close()
    e.close()


def test_graph_needs_a_stream_and_clean_state():
    say("case graph preconditions")
    from paper_1706_06972_amd import ocsc as L
    from paper_1706_06972_amd.ocsc import OCSC
    e = OCSC(4, 5, 5, 32, 32, 0.5, 1.0)      # default stream
    x = torch.zeros((2, 1, 32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(L.OcscError) as err:
        L.ocsc_graph_create(e.ctx, x, 1, None)
    assert err.value.status == L.OCSC_E_UNSUPPORTED
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = OCSC(4, 5, 5, 32, 32, 0.5, 1.0)
    g.set_dictionary(synth.initial_dictionary(4, 5, 5, 0))
    g.code_update(x[0])
    with pytest.raises(L.OcscError) as err:
        L.ocsc_graph_create(g.ctx, x, 1, None)
    assert err.value.status == L.OCSC_E_STATE
    e.close()
    g.close()
