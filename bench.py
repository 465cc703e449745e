"""Throughput of online convolutional sparse coding on one MI355X.

One step = one body of Algorithm 3 for one sample: the code update (J_z = 10
code-ADMM iterations), the history fold and DictOCSC (J = 10 dictionary-ADMM
iterations), on 128 x 128 grids with K = 100 filters of 11 x 11, in FP32.
Samples are synthetic (Bernoulli-Gaussian codes on 100 x 100 content, the
paper's K, filter size and beta), generated on the host and resident in HBM
before the timed region.

Prints one JSON line.  The roofline object covers the dominant kernel, the
D-step sweep that streams the inverse history matrices C (K x K per
frequency), timed over the timed region by HIP events that each sweep launch
carries on the library's stream (they take the kernel's own start and end and
add no packets between kernels).  The cpu_baseline object times the FP64 oracle on a bounded sample of
the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "images/s coded+dict-updated (K=100, 128²) plain vs BF16/served; p99 latency"
WORKLOAD = "ocsc_128x128_k100_f32"
HBM_PEAK_GBS = 8000.0
# the D-step sweep's source: common helpers and the sweep itself
KERNEL_SRC = [os.path.join(ROOT, "paper_1706_06972_amd", "csrc", f) for f in ("fft_lds.hpp", "common.hpp", "dstep.hpp")]
HBM_SUMMARY = os.path.join(ROOT, "profiles", f"{WORKLOAD}_hbm_bytes.md")


def kernel_source_sha256() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per plain D-step launch from the committed counter summary.

    The summary records the SHA-256 of the kernel source it was measured on;
    if the source has changed since, the figure no longer describes this
    kernel and None is returned.
    """
    if not os.path.exists(HBM_SUMMARY):
        return None
    vals = {}
    with open(HBM_SUMMARY) as fh:
        for line in fh:
            if ":" in line and line.split(":", 1)[0].strip() in ("dstep_traffic_bytes_per_launch", "dstep_source_sha256"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("dstep_source_sha256") != kernel_source_sha256():
        return None
    try:
        return int(float(vals["dstep_traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def dstep_bytes_per_launch(K: int, Pf: int, real_bytes: int) -> int:
    """Algorithmic HBM bytes of one D-step sweep without a fold.

    Per frequency: read C_p (K*K reals, packed Hermitian), read the right-hand
    side (K complex), write d_p (K complex).
    """
    return Pf * (K * K * real_bytes + 2 * K * 2 * real_bytes)


def oracle_baseline(wl, n_steps: int):
    import numpy as np
    import oracle.ocsc_oracle as O
    import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    xs = synth.images(wl, synth.pass_order(wl.n_images, wl.seed, 0)[:n_steps + 1])
    m = O.OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho,
               iters_code=wl.iters_code, iters_dict=wl.iters_dict)
    m.set_dictionary(synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed))
    m.step(xs[0][None])                      # first step allocates; not timed
    t0 = time.perf_counter()
    for x in xs[1:]:
        m.step(x[None])
    dt = time.perf_counter() - t0
    return {"value": n_steps / dt, "unit": "images/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_steps} steps of the {wl.name} workload (FP64 NumPy oracle, after one untimed step)",
            "seconds": dt, "host_cpus": os.cpu_count(), "nproc": host_nproc(), "cpu_model": host_cpu_model()}


def host_nproc():
    """Processing units available to this process (``nproc``)."""
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count()


def host_cpu_model() -> str:
    """The host CPU model, as ``lscpu`` reports it (``/proc/cpuinfo`` if lscpu is missing)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batched_run(wl, B: int, xs, dev, steps: int = 10, warmup: int = 2, cholesky: bool = False, K=None) -> dict:
    """Minibatch form: B samples coded against one dictionary, folded in index
    order, one DictOCSC per minibatch (same kernels, same precision).  With
    cholesky: the precision form (history on the BF16 matrix cores, C from an
    FP64 Cholesky per frequency)."""
    import torch
    import synth
    from paper_1706_06972_amd import ocsc as L
    n_img = xs.shape[0]
    reps = (B + n_img - 1) // n_img
    pool = torch.cat([xs] * reps, 0)[:B].contiguous()
    K = K or wl.K
    g = L.OCSC(K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, iters_code=wl.iters_code,
               iters_dict=wl.iters_dict, max_batch=B, precision="f32", cholesky=cholesky, device=dev)
    g.set_dictionary(synth.initial_dictionary(K, wl.filt_h, wl.filt_w, wl.seed))
    shape, _ = g.autotune(B)

    def step():
        L.ocsc_code_update(g.ctx, pool, B, None)
        L.ocsc_history_accumulate(g.ctx)
        L.ocsc_dict_update(g.ctx)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # untimed breakdown: milliseconds per step of each kernel class
    classes = ("dstep", "history", "zstep", "codeplane", "vstep", "fft")
    L.ocsc_profile_enable(g.ctx, list(classes))
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    kern = {c: L.ocsc_profile_read(g.ctx, c)[0] / 2 for c in classes}
    L.ocsc_profile_enable(g.ctx, [])
    del g
    torch.cuda.synchronize()
    return {"batch": B, "K": K, "value": B * steps / dt, "unit": "images/s", "ms_per_step": 1000.0 * dt / steps,
            "steps": steps, "warmup": warmup, "launch_shape": shape,
            "form": ("precision form: BF16 matrix-core history + FP64 Cholesky inverse, FP32 code"
                     if cholesky else "minibatch Sherman-Morrison, FP32"),
            "kernel_ms_per_step": kern}


CODING_GRIDS = ((64, 64), (128, 32), (256, 8), (512, 2))   # (grid side, samples per launch)


def code_bytes_per_image(K: int, n: int, iters: int, real_bytes: int) -> int:
    """Algorithmic HBM bytes of coding one n x n sample of a batch: per
    iteration the Z and F(U - W) hand-offs written and read and the dual read
    and written (the dictionary spectrum read is shared by the batch); the
    codes written once."""
    Pf, P = n * (n // 2 + 1), n * n
    return iters * (4 * K * Pf * 2 * real_bytes + 2 * K * P * real_bytes) + K * P * real_bytes


def coding_run(dev, K: int = 100, iters: int = 10, reps: int = 5) -> dict:
    """Coding only (no history, no dictionary update) against one fixed
    dictionary on 64, 128, 256 and 512 grids, samples of content n/2 x n/2,
    one context per grid, a batch of samples per launch."""
    import torch
    import synth
    from paper_1706_06972_amd import ocsc as L
    D0 = synth.initial_dictionary(K, 11, 11, 0)
    out, inv_sum, bytes_sum = {}, 0.0, 0
    for n, B in CODING_GRIDS:
        wl = synth.Workload(name=f"code{n}", pad_h=n, pad_w=n, content_h=n // 2, content_w=n // 2, k_true=K,
                            density=0.005, sigma_z=10.0, noise=0.01, K=K, filt_h=11, filt_w=11, lam=1.0, rho=1.0,
                            iters_code=iters, iters_dict=10, batch=B, n_images=B, passes=1, precision="f32", seed=n)
        xs = torch.as_tensor(synth.images(wl, range(B)), dtype=torch.float32, device=dev).contiguous()
        g = L.OCSC(K, 11, 11, n, n, 1.0, 1.0, iters_code=iters, max_batch=B, precision="f32", device=dev)
        g.set_dictionary(D0)
        codes = torch.empty((B, K, n, n), dtype=torch.float32, device=dev)

        def timed():
            L.ocsc_code_update(g.ctx, xs, B, codes)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                L.ocsc_code_update(g.ctx, xs, B, codes)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        default = g.tuning
        shape, _ = g.autotune(B)   # before any code update: the workspace holds no pending codes
        g.set_tuning(**default)
        dt0 = timed()
        g.set_tuning(**shape)
        dt = timed()
        g.close()
        del g, codes
        torch.cuda.synchronize()
        rate = B / dt
        nb = code_bytes_per_image(K, n, iters, 4)
        out[str(n)] = {"batch": B, "images_per_s": rate, "ms_per_launch": 1000.0 * dt,
                       "bytes_per_image": nb, "achieved_GBs": nb * rate / 1e9, "tuned_shape": shape,
                       "default_shape": default, "default_images_per_s": B / dt0}
        inv_sum += 1.0 / rate
        bytes_sum += nb
    mix = len(CODING_GRIDS) / inv_sum
    return {"grids": out, "mix_images_per_s": mix,
            "mix_achieved_GBs": bytes_sum / len(CODING_GRIDS) * mix / 1e9,
            "note": "equal shares of the four grids; FP32; K=100, 11x11 filters, J_z=10; launch shapes "
                    "picked by ocsc_autotune per grid"}


def grouped_run(dev, K: int = 100, iters: int = 10, reps: int = 5) -> dict:
    """Uneven sizes: one batch per grid coded (a) by per-grid launches in
    turn, with autotuned shapes, (b) the same launches captured once in a HIP
    graph and replayed, and (c) by one persistent grouped launch
    (ocsc_code_update_group); full batches (the samples per launch of the
    coding run) and single samples per grid."""
    return {"full": _grouped(dev, CODING_GRIDS, K, iters, reps),
            "single": _grouped(dev, tuple((n, 1) for n, _ in CODING_GRIDS), K, iters, 4 * reps),
            "note": ("K=100, FP32, J_z=10; separate: per-grid launch sequences in turn on one stream; graph: "
                     "the same launches replayed from one HIP graph; grouped: every iteration of every grid in "
                     "one cooperative launch")}


def _grouped(dev, grids, K, iters, reps) -> dict:
    import torch
    import synth
    from paper_1706_06972_amd import ocsc as L
    D0 = synth.initial_dictionary(K, 11, 11, 0)
    models, xs = [], []
    # every context on one side stream, so that their launches can be captured in one HIP graph
    st = torch.cuda.Stream(device=dev)
    for n, B in grids:
        wl = synth.Workload(name=f"group{n}", pad_h=n, pad_w=n, content_h=n // 2, content_w=n // 2, k_true=K,
                            density=0.005, sigma_z=10.0, noise=0.01, K=K, filt_h=11, filt_w=11, lam=1.0, rho=1.0,
                            iters_code=iters, iters_dict=10, batch=B, n_images=B, passes=1, precision="f32", seed=n)
        xs.append(torch.as_tensor(synth.images(wl, range(B)), dtype=torch.float32, device=dev).contiguous())
        with torch.cuda.stream(st):
            g = L.OCSC(K, 11, 11, n, n, 1.0, 1.0, iters_code=iters, max_batch=B, precision="f32", device=dev)
        g.set_dictionary(D0)
        g.autotune(B)
        models.append(g)
    total = sum(B for _, B in grids)
    torch.cuda.synchronize()

    def separate():
        for g, x in zip(models, xs):
            L.ocsc_code_update(g.ctx, x, x.shape[0], None)

    def grouped():
        L.ocsc_code_update_group([g.ctx for g in models], xs, [x.shape[0] for x in xs], None)

    # the per-grid launch sequences of one mixed batch captured once as a HIP graph
    separate()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        separate()
    torch.cuda.synchronize()

    out = {}
    for name, fn in (("separate", separate), ("graph", graph.replay), ("grouped", grouped)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"images_per_s": total / dt, "ms_per_launch": 1000.0 * dt}
    del graph
    for g in models:
        g.close()
    out["batch"] = {str(n): B for n, B in grids}
    return out


def graph_run(wl, xs, steps: int, warmup: int = 4, shape=None) -> dict:
    """The same B=1 step replayed from HIP graphs (two steps per graph, one
    graph per pair of resident images), on a context with its own stream."""
    import torch
    import synth
    from paper_1706_06972_amd import ocsc as L
    n_img = xs.shape[0] // 2 * 2
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = L.OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, iters_code=wl.iters_code,
                   iters_dict=wl.iters_dict, max_batch=1, precision="f32")
    g.set_dictionary(synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed))
    if shape:
        g.set_tuning(**shape)
    codes = torch.empty((2, 1, wl.K, wl.pad_h, wl.pad_w), dtype=torch.float32, device=xs.device)
    graphs = [L.ocsc_graph_create(g.ctx, xs[i:i + 2].contiguous(), 1, codes) for i in range(0, n_img, 2)]
    for i in range(warmup):
        L.ocsc_graph_launch(g.ctx, graphs[i % len(graphs)])
    st.synchronize()
    launches = max(1, steps // 2)
    t0 = time.perf_counter()
    for i in range(launches):
        L.ocsc_graph_launch(g.ctx, graphs[i % len(graphs)])
    st.synchronize()
    dt = time.perf_counter() - t0
    for h in graphs:
        L.ocsc_graph_destroy(h)
    g.close()
    return {"value": 2 * launches / dt, "unit": "images/s", "ms_per_step": 1000.0 * dt / (2 * launches),
            "steps": 2 * launches, "form": "the B=1 step above, replayed from HIP graphs"}


def served_run(dev, K: int = 100, full: bool = False) -> dict:
    """Serving form (continuous batching, resident dictionary updated every
    256 requests, FP32): Poisson arrivals on a mix of 64/128/256/512 grids
    (shares 8:4:2:1, a 64 GB HBM budget) at a sustainable and at the
    configured 5,000/s offered rate, and a 128x128-only stream (the shape of
    the B=1 workload above).  The first tenth of each run is excluded.
    full: the configured serving workload only -- 100,000 requests per rate,
    the first 10,000 excluded, at 5,000/s and at 1,800/s (about the measured
    capacity of the mix)."""
    import synth
    from paper_1706_06972_amd.serve import Server, poisson_requests, summarize
    D0 = synth.initial_dictionary(K, 11, 11, 0)
    out = {}
    grids, shares = (64, 128, 256, 512), (8, 4, 2, 1)
    srv = Server(K, 11, D0, grids=grids, shares=shares, update_every=256, budget=64e9)
    runs = ((5000.0, 100000), (1800.0, 100000)) if full else ((1000.0, 2000), (5000.0, 3000))
    for rate, n in runs:
        reqs = poisson_requests(n, rate, grids, shares, seed=int(rate))
        m = srv.run(reqs)
        out[f"mix_{int(rate)}"] = summarize(reqs, m["wall_s"], m["dictionary_updates"], warmup=n // 10)
        print(f"served mix at {rate:.0f}/s: {out[f'mix_{int(rate)}']}", file=sys.stderr, flush=True)
    out["mix_slots"] = srv.slots
    srv.close()
    if full:
        out["note"] = ("configured serving workload: 100,000 Poisson requests per offered rate, the first 10,000 "
                       "excluded; latency = completion event - arrival (input copy from pinned host memory included)")
        return out
    for chol in (False, True):
        # the 128x128 stream with the Sherman-Morrison fold, then in the precision form
        srv = Server(K, 11, D0, grids=(128,), shares=(1,), update_every=256, budget=64e9,
                     max_launch={128: 64}, cholesky=chol)
        for rate, n in ((4000.0, 6000), (20000.0, 6000)):
            reqs = poisson_requests(n, rate, (128,), (1,), seed=7)
            m = srv.run(reqs)
            key = f"grid128{'_precision' if chol else ''}_{int(rate)}"
            out[key] = summarize(reqs, m["wall_s"], m["dictionary_updates"], warmup=n // 10)
        srv.close()
    out["note"] = ("latency = completion event - arrival; inputs copied from pinned host memory inside the "
                   "latency; dictionary updated every 256 requests (shared across grids); grid128_precision: "
                   "the history on the BF16 matrix cores and C from FP64 Cholesky factors")
    return out


def copy_ceiling(dev, nbytes: int = 346112000, reps: int = 20) -> dict:
    """Measured device-to-device copy rate of a buffer the size of one D-step
    sweep's algorithmic bytes (read + write counted), for context beside the
    8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    s = a.elapsed_time(b) / 1000.0 / reps
    del src, dst
    return {"GBs": 2 * nbytes / s / 1e9, "bytes_moved": 2 * nbytes, "kernel": "torch copy_"}


def copy_calibration(mib: int) -> None:
    """Device-to-device copies of a known size, to scale the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 5}), flush=True)


def quality_run(dev, n_train: int = 1000, n_test: int = 16, passes: int = 2, j_eval: int = 200):
    """Quality on the synthetic stand-in, as the paper's section 4 measures it:
    test objective and PSNR of held-out images coded against D_0, against the
    exported learned dictionary and against the generator's ground-truth
    filters, with the learner's J_z code iterations and with J_eval (codes
    close to converged); per pass the relative changes of the codes and of the
    dictionary (the quantities of the stopping rule) and the test objective;
    and the code-ADMM objective against the iteration count J (the code side
    of the synthetic study of Appendix B).  B = 1, FP32, the workload's K,
    lambda and rho."""
    import numpy as np
    import torch
    import synth
    from paper_1706_06972_amd import evaluate as E
    from paper_1706_06972_amd.ocsc import OCSC

    wl = synth.WORKLOADS[WORKLOAD]
    order = synth.pass_order(wl.n_images, wl.seed, 0)
    train = torch.as_tensor(synth.images(wl, order[:n_train]), dtype=torch.float32, device=dev).contiguous()
    test_np = synth.images(wl, order[-n_test:])   # never presented for learning
    test = torch.as_tensor(test_np, dtype=torch.float32, device=dev).contiguous()
    peak = float(np.abs(test_np).max())

    def make(J=wl.iters_code):
        return OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, iters_code=J,
                    iters_dict=wl.iters_dict, precision="f32", device=dev)

    def scores(D):
        out = {}
        for J in (wl.iters_code, j_eval):
            m = make(J)
            m.set_dictionary(D)
            out[f"J{J}"] = {"test_objective": E.test_objective(m, test), "psnr_db": E.psnr(m, test, peak)}
            m.close()
        return out

    D0 = synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed)
    g = make()
    g.set_dictionary(D0)
    t0 = time.perf_counter()
    hist = E.learn(g, train, passes, tol=1e-3, order_seed=wl.seed + 3, test_xs=test)
    torch.cuda.synchronize()
    learn_s = time.perf_counter() - t0
    D = g.get_dictionary()
    g.close()
    study = E.code_admm_study(make, D, test[:4], [1, 2, 5, 10, 20, 50, 100, 200])
    return {"train_images": n_train, "test_images": n_test, "passes": passes, "psnr_peak": peak,
            "initial": scores(D0), "learned": scores(D), "ground_truth_filters": scores(synth.truth_filters(wl)),
            "per_pass": hist, "learn_seconds": learn_s, "code_admm_objective_vs_iters": study}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--pool", type=int, default=64, help="distinct images resident on the device")
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle steps timed for cpu_baseline (0: skip)")
    ap.add_argument("--traffic", type=str, default="", help="JSON file with measured HBM bytes per D-step launch")
    ap.add_argument("--batch", type=int, default=64,
                    help="also time minibatch steps of this many samples (0: skip)")
    ap.add_argument("--coding", type=int, default=1, help="also time coding on 64..512 grids (0: skip)")
    ap.add_argument("--grouped", type=int, default=1,
                    help="also time the grouped persistent (cooperative) launch against per-grid launches (0: skip)")
    ap.add_argument("--served", type=int, default=1,
                    help="also run the serving form (0: skip; 2: only the configured 100,000-request mix runs)")
    ap.add_argument("--quality", type=int, default=1,
                    help="also measure test objective / PSNR before and after learning (0: skip)")
    ap.add_argument("--launch-shape", type=str, default="", metavar="JSON",
                    help="launch shape of the B=1 step, e.g. '{\"two_pass\": 2}', instead of the autotuner's "
                         "(reproducible hardware-counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run device copies of MIB MiB (hardware-counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import numpy as np
    import torch

    import synth
    from paper_1706_06972_amd import ocsc as L

    wl = synth.WORKLOADS[WORKLOAD]
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    n_img = max(1, min(args.pool, args.warmup + args.steps))
    order = synth.pass_order(wl.n_images, wl.seed, 0)[:n_img]
    xs = torch.as_tensor(synth.images(wl, order), dtype=torch.float32, device=dev).contiguous()
    codes = torch.empty((1, wl.K, wl.pad_h, wl.pad_w), dtype=torch.float32, device=dev)

    g = L.OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho, iters_code=wl.iters_code,
               iters_dict=wl.iters_dict, max_batch=1, precision="f32", device=dev)
    g.set_dictionary(synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed))
    # launch shapes of the code update for single samples (bitwise the same results for every shape)
    if args.launch_shape:
        g.set_tuning(**json.loads(args.launch_shape))
        tuned = dict(g.tuning)
    else:
        tuned, _ = g.autotune(1)

    def step(i):
        x = xs[i % n_img:i % n_img + 1]
        L.ocsc_code_update(g.ctx, x, 1, codes)
        L.ocsc_history_accumulate(g.ctx)
        L.ocsc_dict_update(g.ctx)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    # timed region: each D-step sweep (the dominant kernel) carries its own start/stop events
    L.ocsc_profile_enable(g.ctx, ["dstep"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n = L.ocsc_profile_read(g.ctx, "dstep")
    dstep_avg_us = 1000.0 * ms / n
    # untimed breakdown pass: every kernel class bracketed by events
    classes = ("dstep", "history", "zstep", "codeplane", "vstep", "fft")
    nb = min(args.steps, 50)
    L.ocsc_profile_enable(g.ctx, list(classes))
    for i in range(nb):
        step(args.warmup + args.steps + i)
    torch.cuda.synchronize()
    kern = {}
    for cls in classes:
        ms, n = L.ocsc_profile_read(g.ctx, cls)
        kern[cls] = {"avg_us": 1000.0 * ms / n if n else None, "launches": n, "ms_per_step": ms / nb}
    L.ocsc_profile_enable(g.ctx, [])

    Pf = wl.pad_h * (wl.pad_w // 2 + 1)
    per_launch = dstep_bytes_per_launch(wl.K, Pf, 4)
    avg_s = dstep_avg_us * 1e-6
    achieved = per_launch / avg_s / 1e9
    traffic = recorded_traffic()
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as fh:
            traffic = json.load(fh).get("dstep_bytes_per_launch")

    value = args.steps / dt
    out = {
        "metric": METRIC, "value": value, "unit": "images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (Bernoulli-Gaussian codes * unit-norm Gaussian 11x11 filters + noise)",
        "config": {"workload": WORKLOAD, "grid": f"{wl.pad_h}x{wl.pad_w}", "content": f"{wl.content_h}x{wl.content_w}",
                   "K": wl.K, "filter": f"{wl.filt_h}x{wl.filt_w}", "batch": 1, "iters_code": wl.iters_code,
                   "iters_dict": wl.iters_dict, "lambda": wl.lam, "rho": wl.rho, "form": "plain",
                   "distinct_images": n_img},
        "roofline": {"kernel": "k_dict_sweep (D-step, no fold)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": per_launch,
                     "avg_launch_us": dstep_avg_us},
        "kernels": kern,
        "launch_shape": tuned,
    }
    del g
    torch.cuda.synchronize()
    out["graph"] = graph_run(wl, xs, args.steps, shape=tuned)
    out["batched"] = batched_run(wl, args.batch, xs, dev) if args.batch > 1 else None
    out["precision"] = batched_run(wl, args.batch, xs, dev, cholesky=True) if args.batch > 1 else None
    # the precision form at K=256 (same grid and minibatch; C from block Cholesky inverses)
    out["precision_k256"] = (batched_run(wl, args.batch, xs, dev, steps=4, warmup=1, cholesky=True, K=256)
                             if args.batch > 1 else None)
    out["coding"] = coding_run(dev) if args.coding else None
    out["grouped"] = grouped_run(dev) if args.grouped else None
    out["copy_ceiling"] = copy_ceiling(dev)
    out["served"] = served_run(dev, full=args.served == 2) if args.served else None
    out["quality"] = quality_run(dev) if args.quality else None
    if args.cpu_steps > 0:
        out["cpu_baseline"] = oracle_baseline(wl, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
