"""The FP32 library along the 128x128, K = 100 workload's trajectory (Algorithm
3, one sample per step, J_z = J_d = 10), through the C ABI.

* Against FP64 oracle checkpoints of the first steps of the first pass
  (``tests/golden/ocsc_128x128_k100_first*.npz``, written from the oracle
  alone by ``tests/golden/make_c2_checkpoints.py``): every step's objective,
  ||U||_1 and number of non-zero codes; at the checkpoint steps the exported
  dictionary, and at 32 sampled frequencies the dictionary spectrum, G_p and
  C_p r for two probe vectors; the codes at a few steps.  Norm-wise relative
  error per quantity, 1e-3 as for every FP32 context; the errors are printed
  per checkpoint, with the worst single frequency.
* The whole run, 10,000 images in two passes (20,000 Sherman-Morrison
  updates of C in FP32, eq. C_update): the history H_p = sum_i conj(z_ip)
  z_ip^T is summed in FP64 from the library's own last Z-step spectra at 32
  sampled frequencies, and every 1,000 steps the inverse the library keeps
  must still solve (H_p + rho_d I) C_p = I.  The residual is printed per
  checkpoint: it is the drift of the recursion.
"""
import glob
import os
import time

import numpy as np
import pytest

import synth
from tests.gpu_util import rel, say, spectra, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["ocsc_128x128_k100_f32"]
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-3


def golden_file():
    files = sorted(glob.glob(os.path.join(HERE, "golden", "ocsc_128x128_k100_first*.npz")))
    assert files, "oracle checkpoints missing: run tests/golden/make_c2_checkpoints.py"
    return files[-1]


def packed_at(flat, K, idx):
    """[Pf][K][K] packed reals (Re on/above the diagonal, Im below) at frequencies idx
    -> complex (len(idx), K, K), on the device."""
    R = flat.view(-1, K, K)[torch.as_tensor(idx, device=flat.device)].double()
    up = torch.triu(R)
    re = up + torch.triu(R, 1).transpose(1, 2)
    lo = torch.tril(R, -1)
    im = lo.transpose(1, 2) - lo
    return torch.complex(re, im)


def learner():
    from paper_1706_06972_amd.ocsc import OCSC
    g = OCSC(WL.K, WL.filt_h, WL.filt_w, WL.pad_h, WL.pad_w, WL.lam, WL.rho, iters_code=WL.iters_code,
             iters_dict=WL.iters_dict, precision="f32")
    g.set_dictionary(synth.initial_dictionary(WL.K, WL.filt_h, WL.filt_w, WL.seed))
    shape, _ = g.autotune(1)             # the launch shapes bench.py times (every shape gives the same bits)
    g.set_tuning(**shape)
    return g


def test_c2_trajectory_against_oracle_checkpoints():
    gold = np.load(golden_file())
    n = int(gold["n_done"])
    say(f"case 128x128 K=100 FP32 trajectory, {n} steps against the FP64 oracle checkpoints")
    K, ph, pw = WL.K, WL.pad_h, WL.pad_w
    idx = gold["freq_idx"]
    probes = gold["probes"]
    rho_d = float(gold["rho_d"])
    cps = [int(c) for c in gold["checkpoints"] if c <= n]
    g = learner()
    worst = {}
    f_err = l1_err = 0.0
    nnz_err = 0.0

    def note(name, v):
        worst[name] = max(worst.get(name, 0.0), v)
        return v

    for t, i in enumerate(gold["order"][:n], start=1):
        x = synth.images(WL, [int(i)])
        U = g.code_update(x)
        f = g.objective(x, U)[0]
        f_err = max(f_err, abs(f - gold["objective"][t - 1]) / abs(gold["objective"][t - 1]))
        l1 = float(U.double().abs().sum())
        l1_err = max(l1_err, abs(l1 - gold["codes_l1"][t - 1]) / gold["codes_l1"][t - 1])
        nnz = int(torch.count_nonzero(U))
        nnz_err = max(nnz_err, abs(nnz - int(gold["codes_nnz"][t - 1])) / int(gold["codes_nnz"][t - 1]))
        if f"U_idx_{t}" in gold:
            Uo = np.zeros(U.numel())
            Uo[gold[f"U_idx_{t}"]] = gold[f"U_val_{t}"]
            note("codes", rel(to_np(U).reshape(-1), Uo))
        g.history_accumulate()
        g.dict_update()
        if t in cps:
            e = {"dict": note("dict", rel(to_np(g.get_dictionary()), gold[f"D_{t}"]))}
            Dh = spectra(to_np(g.state("dict_hat")), (K,), ph, pw).reshape(K, -1)[:, idx]
            G = spectra(to_np(g.state("G")), (K,), ph, pw).reshape(K, -1)[:, idx]
            C = packed_at(g.state("cinv"), K, idx).cpu().numpy()
            Cr = C @ probes
            Cr_o = gold[f"Cr_{t}"]
            eye_r = probes / rho_d                       # C_0 r: the part every C_p shares
            per_f = {
                "dict_hat": np.linalg.norm(Dh - gold[f"Dh_{t}"], axis=0) / np.linalg.norm(gold[f"Dh_{t}"], axis=0),
                "G": np.linalg.norm(G - gold[f"G_{t}"], axis=0) / np.linalg.norm(gold[f"G_{t}"], axis=0),
                "C r": np.linalg.norm(Cr - Cr_o, axis=(1, 2)) / np.linalg.norm(Cr_o, axis=(1, 2)),
                "(C - I/rho_d) r": (np.linalg.norm(Cr - Cr_o, axis=(1, 2))
                                    / np.linalg.norm(Cr_o - eye_r, axis=(1, 2))),
            }
            e["dict_hat"] = note("dict_hat", rel(Dh, gold[f"Dh_{t}"]))
            e["G"] = note("G", rel(G, gold[f"G_{t}"]))
            e["C r"] = note("C r", rel(Cr, Cr_o))
            e["(C - I/rho_d) r"] = note("(C - I/rho_d) r", rel(Cr - eye_r, Cr_o - eye_r))
            say(f"  step {t:4d}: " + "  ".join(f"{k} {v:.2e}" for k, v in e.items())
                + "  | worst frequency: " + "  ".join(f"{k} {v.max():.2e}" for k, v in per_f.items()))
            for k, v in per_f.items():
                note(f"{k}, worst frequency", float(v.max()))
    worst["objective"], worst["codes_l1"], worst["codes_nnz (relative count)"] = f_err, l1_err, nnz_err
    say("  worst over the run: " + "  ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    g.close()
    for k in ("objective", "codes_l1", "codes", "dict", "dict_hat", "G", "C r", "(C - I/rho_d) r"):
        assert worst[k] < TOL, (k, worst[k])


def _image_chunk(lo_hi):
    import synth as s
    lo, hi = lo_hi
    return s.images(s.WORKLOADS["ocsc_128x128_k100_f32"], range(lo, hi)).astype(np.float32)


def all_images(dev):
    """The workload's 10,000 images on the device (float32), generated by a pool
    of host processes (about 70 ms of host time per image)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n = WL.n_images
    step = 250
    chunks = [(lo, min(n, lo + step)) for lo in range(0, n, step)]
    out = torch.empty((n, WL.pad_h, WL.pad_w), dtype=torch.float32, device=dev)
    workers = min(16, os.cpu_count() or 1)
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for (lo, hi), arr in zip(chunks, ex.map(_image_chunk, chunks)):
            out[lo:hi] = torch.as_tensor(arr, device=dev)
    return out


@pytest.mark.timeout(900)
def test_c2_full_run_inverse_drift():
    K, ph, pw = WL.K, WL.pad_h, WL.pad_w
    dev = torch.device("cuda")
    say(f"case 128x128 K=100 FP32, full run: {WL.n_images} images x {WL.passes} passes; generating images")
    t0 = time.time()
    xs = all_images(dev)
    say(f"  images ready in {time.time() - t0:.0f} s")
    g = learner()
    rho_d = WL.rho * ph * pw
    Pf = ph * (pw // 2 + 1)
    idx = np.sort(np.random.default_rng(5).choice(Pf, 32, replace=False))
    tidx = torch.as_tensor(idx, device=dev)
    H = torch.zeros((32, K, K), dtype=torch.complex128, device=dev)
    eye = torch.eye(K, dtype=torch.complex128, device=dev)
    curve = []
    t = 0
    t0 = time.time()
    for q in range(WL.passes):
        for i in synth.pass_order(WL.n_images, WL.seed, q):
            g.code_update(xs[int(i)], want_codes=False)
            zh = g.state("zhat").view(K, Pf, 2)[:, tidx].double()        # the spectra about to be folded
            z = torch.complex(zh[..., 0], zh[..., 1]).T                     # (32, K)
            H += torch.conj(z)[:, :, None] * z[:, None, :]                  # H_p += conj(z_p) z_p^T
            g.history_accumulate()
            g.dict_update()
            t += 1
            if t % 1000 == 0:
                C = packed_at(g.state("cinv"), K, idx)
                A = H + rho_d * eye
                res = torch.linalg.matrix_norm(C @ A - eye) / np.sqrt(K)
                fwd = (torch.linalg.matrix_norm(C - torch.linalg.inv(A)) / torch.linalg.matrix_norm(torch.linalg.inv(A)))
                hn = float(torch.linalg.matrix_norm(H, ord=2).max())
                curve.append((t, float(res.max()), float(fwd.max()), hn))
                say(f"  step {t:6d}: max_p ||C_p (H_p + rho_d I) - I||_F / sqrt(K) = {res.max():.2e}; "
                    f"max_p ||C_p - (H_p + rho_d I)^-1|| / ||.|| = {fwd.max():.2e}; "
                    f"max_p ||H_p||_2 = {hn:.3e}  ({time.time() - t0:.0f} s)")
    assert t == WL.n_images * WL.passes
    D = g.get_dictionary()
    assert torch.isfinite(D).all()
    g.close()
    for step, res, fwd, _ in curve:
        assert res < TOL and fwd < TOL, (step, res, fwd)
