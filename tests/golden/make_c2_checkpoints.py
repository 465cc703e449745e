"""Write FP64 oracle checkpoints of the 128x128, K = 100 workload.

Runs the FP64 oracle (Algorithm 3, one sample per step, J_z = J_d = 10) over
the first N samples of the workload's first pass and stores, in
``ocsc_128x128_k100_first<N>.npz``:

* every step t: the objective of eq. csc of the sample's codes against the
  dictionary that coded them, ||U_t||_1 and the number of non-zero codes;
* at the checkpoint steps (after that step's dictionary update): the exported
  dictionary crop(F^-1 D~), and at 32 seeded frequencies the dictionary
  spectrum D~_p, the history G_p and C_p r for two seeded complex probe
  vectors r (a sketch of C_p = (H_p + rho_d I)^-1: for a probe with unit-variance
  entries, the mean of ||E r||^2 is ||E||_F^2);
* at a few of them also the codes of that step, as flat indices and values
  of the non-zeros.

Calls only the oracle and the synthetic-input generator, never the HIP
library.  The values are the oracle's own (the paper prints no trajectory);
they spare the GPU test an hour of CPU work.  About 16 s per step on 8 cores.

    python tests/golden/make_c2_checkpoints.py [N]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.ocsc_oracle as O  # noqa: E402
import synth  # noqa: E402

NAME = "ocsc_128x128_k100_f32"
CHECKPOINTS = (1, 2, 5, 10, 20, 50, 100, 150, 200, 300, 400)
CODE_CHECKPOINTS = (1, 100, 200)
N_FREQ = 32
N_PROBE = 2


def path_for(n_steps: int) -> str:
    return os.path.join(HERE, f"ocsc_128x128_k100_first{n_steps}.npz")


def run(n_steps: int) -> str:
    wl = synth.WORKLOADS[NAME]
    order = synth.pass_order(wl.n_images, wl.seed, 0)[:n_steps]
    m = O.OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho,
               iters_code=wl.iters_code, iters_dict=wl.iters_dict)
    m.set_dictionary(synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed))
    pf = wl.pad_h * (wl.pad_w // 2 + 1)
    rng = np.random.default_rng(20170620)
    idx = np.sort(rng.choice(pf, N_FREQ, replace=False))
    probes = (rng.standard_normal((N_FREQ, wl.K, N_PROBE))
              + 1j * rng.standard_normal((N_FREQ, wl.K, N_PROBE))) / np.sqrt(2.0)
    cps = [c for c in CHECKPOINTS if c <= n_steps]
    out = {
        "order": np.asarray(order, np.int64), "freq_idx": idx.astype(np.int64), "probes": probes,
        "checkpoints": np.asarray(cps, np.int64), "rho_d": np.float64(m.rho_d),
        "objective": np.zeros(n_steps), "codes_l1": np.zeros(n_steps),
        "codes_nnz": np.zeros(n_steps, np.int64),
    }
    t0 = time.time()
    for t, i in enumerate(order, start=1):
        x = synth.images(wl, [i])
        U = m.code_update(x)
        out["objective"][t - 1] = m.objective(x, U)[0]
        out["codes_l1"][t - 1] = np.abs(U).sum()
        out["codes_nnz"][t - 1] = np.count_nonzero(U)
        m.history_accumulate()
        m.dict_update()
        if t in cps:
            fl = lambda a: a.reshape(a.shape[0], -1)          # (K, Pf)
            C = m.C.reshape(pf, wl.K, wl.K)[idx]             # (32, K, K)
            out[f"D_{t}"] = m.get_dictionary()
            out[f"Dh_{t}"] = fl(m.Dh)[:, idx]
            out[f"G_{t}"] = fl(m.G)[:, idx]
            out[f"Cr_{t}"] = C @ probes
            if t in CODE_CHECKPOINTS:
                flat = U.reshape(-1)
                nz = np.flatnonzero(flat)
                out[f"U_idx_{t}"] = nz.astype(np.int32)
                out[f"U_val_{t}"] = flat[nz]
            np.savez_compressed(path_for(n_steps), n_done=np.int64(t), **out)
        print(f"step {t}/{n_steps}  f {out['objective'][t - 1]:.6e}  nnz {out['codes_nnz'][t - 1]}  "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(path_for(n_steps), n_done=np.int64(n_steps), **out)
    return path_for(n_steps)


if __name__ == "__main__":
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 200
    print("wrote", run(n))
