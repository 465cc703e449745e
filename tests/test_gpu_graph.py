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


def test_coding_batch_over_grids_as_one_graph():
    """A mixed batch -- per-grid code updates (eq. fcsc_code) on 64, 128 and
    256 grids -- captured once as a HIP graph on the contexts' stream and
    replayed three times with new samples copied in between: every replay's
    codes and kept spectra equal those of eager code updates on twin
    contexts, bit for bit, with eager work on the captured contexts between
    the replays."""
    say("case coding batch over grids as one graph")
    from paper_1706_06972_amd.ocsc import OCSC
    K, filt = 6, 7
    grids = ((64, 3), (128, 2), (256, 1))
    st = torch.cuda.Stream()
    D0 = synth.initial_dictionary(K, filt, filt, 2)
    cap, twin, xb, cb, pools = [], [], [], [], []
    for n, B in grids:
        wl = synth.Workload(name=f"gg{n}", pad_h=n, pad_w=n, content_h=n // 2, content_w=n // 2, k_true=8,
                            density=0.01, sigma_z=10.0, noise=0.01, K=8, filt_h=filt, filt_w=filt, lam=0.5,
                            rho=1.0, iters_code=10, iters_dict=10, batch=B, n_images=3 * B, passes=1,
                            precision="f32", seed=n)
        pools.append(torch.as_tensor(synth.images(wl, range(3 * B)), dtype=torch.float32, device="cuda"))
        with torch.cuda.stream(st):
            g = OCSC(K, filt, filt, n, n, 0.5, 1.0, precision="f32", max_batch=B)
        e = OCSC(K, filt, filt, n, n, 0.5, 1.0, precision="f32", max_batch=B)
        g.set_dictionary(D0)
        e.set_dictionary(D0)
        cap.append(g)
        twin.append(e)
        xb.append(torch.zeros((B, n, n), dtype=torch.float32, device="cuda"))
        cb.append(torch.zeros((B, K, n, n), dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()

    def batch():
        for g, x, c in zip(cap, xb, cb):
            g.code_update(x, codes=c)

    batch()                                   # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        batch()
    torch.cuda.synchronize()
    for r in range(3):
        with torch.cuda.stream(st):
            for (n, B), x, pool in zip(grids, xb, pools):
                x.copy_(pool[r * B:(r + 1) * B])
        graph.replay()
        want = [e.code_update(pool[r * B:(r + 1) * B]) for e, (n, B), pool in zip(twin, grids, pools)]
        st.synchronize()
        torch.cuda.synchronize()
        for i, (g, e) in enumerate(zip(cap, twin)):
            assert torch.equal(cb[i], want[i]), (r, i)
            assert torch.equal(g.state("zhat"), e.state("zhat")), (r, i)
        # eager work on the captured contexts between the replays
        with torch.cuda.stream(st):
            f = cap[0].objective(xb[0], cb[0])
        assert min(f) > 0
    del graph
    for m in cap + twin:
        m.close()
