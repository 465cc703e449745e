"""Write the stored oracle trajectory summaries under tests/golden/.

Calls only the FP64 oracle and the synthetic-input generator.  The stored
values guard the oracle against unintended change: the paper prints no worked
example or trajectory, so these are the oracle's own values, not the paper's.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.ocsc_oracle as O  # noqa: E402
import synth  # noqa: E402


def trajectory_summary(name: str, n_steps: int) -> dict:
    wl = synth.WORKLOADS[name]
    order = synth.pass_order(wl.n_images, wl.seed, 0)[:n_steps]
    xs = synth.images(wl, order)
    m = O.OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho,
               iters_code=wl.iters_code, iters_dict=wl.iters_dict)
    m.set_dictionary(synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed))
    steps = []
    for x in xs:
        U = m.code_update(x[None])
        f = float(m.objective(x[None], U)[0])
        m.history_accumulate()
        m.dict_update()
        D = m.get_dictionary()
        steps.append({
            "objective": f,
            "codes_l1": float(np.abs(U).sum()),
            "codes_nnz": int(np.count_nonzero(U)),
            "dict_fro": float(np.linalg.norm(D)),
            "dict_sum": float(D.sum()),
        })
    return {"workload": name, "order": [int(i) for i in order], "steps": steps}


if __name__ == "__main__":
    out = trajectory_summary("ocsc_64x64_k16_f64", 5)
    with open(os.path.join(HERE, "ocsc_64x64_k16_f64_first5.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", len(out["steps"]), "steps")
