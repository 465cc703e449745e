"""Evaluation of a learner (section 4 and Appendix B of the paper), on top of
the C calls: every number comes from the library's kernels; this module only
sequences calls and averages the scalars they return.

* ``test_objective``: the paper's test-set objective, the mean over a test set
  of 1/2 ||x - sum_k D_k * Z_k||^2 + lambda ||Z||_1 with each sample's codes
  re-solved against the current dictionary (no history update).
* ``psnr``: the paper's reconstruction quality, the mean over a test set of
  10 log10(peak^2 P / ||x_rec - x||^2), from the data term of the objective.
* ``learn``: passes over a training set in a seeded order, stopped by the
  paper's rule: the relative changes of the codes and of the dictionary both
  below ``tol``.  The codes of sample i are compared with the codes sample i
  got in the previous pass (the online method codes each sample once per
  pass), the dictionary with the dictionary at the end of the previous pass.
* ``code_admm_study``: objective of the code ADMM after J iterations for a list
  of J, the code side of the synthetic convergence study of Appendix B.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Sequence


def relative_change(new, old) -> float:
    """||new - old|| / ||new|| (0 when both are zero)."""
    import torch
    n = float(torch.linalg.vector_norm(new.double()))
    dlt = float(torch.linalg.vector_norm((new - old).double()))
    if n == 0.0:
        return 0.0 if dlt == 0.0 else math.inf
    return dlt / n


def _codes(model, x):
    return model.code_update(x)


def test_objective(model, xs) -> float:
    """Mean test-set objective with codes re-solved against the current dictionary.

    The samples are coded in chunks of the learner's max_batch; nothing is
    folded into the history.
    """
    total, n = 0.0, 0
    for x in _chunks(model, xs):
        U = _codes(model, x)
        vals = model.objective(x, U)
        total += float(sum(vals))
        n += len(vals)
    return total / n


def psnr(model, xs, peak: float = 255.0) -> float:
    """Mean PSNR (dB) of the reconstructions sum_k D_k * Z_k of a test set."""
    P = model.shape[0] * model.shape[1]
    total, n = 0.0, 0
    for x in _chunks(model, xs):
        U = _codes(model, x)
        for data, _l1 in model.objective_terms(x, U):
            total += 10.0 * math.log10(peak * peak * P / (2.0 * data))
            n += 1
    return total / n


def learn(model, xs, passes: int, tol: float = 1e-3, order_seed: int = 0,
          test_xs=None) -> List[dict]:
    """Online learning over ``xs`` for at most ``passes`` passes (one sample per
    step, B = 1), stopped early by the relative-change rule.  Returns one
    record per pass: the relative changes, the mean training objective of the
    samples as they were coded, and the test objective if a test set is given.
    """
    import numpy as np
    N = xs.shape[0]
    prev_codes: dict = {}
    prev_D = model.get_dictionary().clone()
    history = []
    for ps in range(passes):
        order = np.random.default_rng(order_seed + ps).permutation(N)
        rel_z, train_obj = [], 0.0
        for i in order:
            x = xs[int(i)]
            U = model.code_update(x)
            train_obj += float(model.objective(x, U)[0])
            model.history_accumulate()
            model.dict_update()
            key = int(i)
            if key in prev_codes:
                rel_z.append(relative_change(U, prev_codes[key]))
            prev_codes[key] = U.clone()
        D = model.get_dictionary()
        rel_d = relative_change(D, prev_D)
        prev_D = D.clone()
        rec = {"pass": ps, "train_objective": train_obj / N, "rel_change_D": rel_d,
               "rel_change_Z": (sum(rel_z) / len(rel_z)) if rel_z else None}
        if test_xs is not None:
            rec["test_objective"] = test_objective(model, test_xs)
        history.append(rec)
        if rel_z and rec["rel_change_Z"] < tol and rel_d < tol:
            break
    return history


def code_admm_study(make_model, D, xs, iters: Sequence[int]) -> List[dict]:
    """Objective of the code ADMM after J iterations, for each J in ``iters``.

    ``make_model(J)`` returns a learner with J code iterations; every learner
    gets the same dictionary D and codes the same samples.  Returns
    [{"iters": J, "objective": mean objective}] in the order of ``iters``.
    """
    out = []
    for J in iters:
        m = make_model(int(J))
        m.set_dictionary(D)
        vals = []
        for x in _chunks(m, xs):
            U = m.code_update(x)
            vals.extend(m.objective(x, U))
        out.append({"iters": int(J), "objective": float(sum(vals)) / len(vals)})
        m.close()
    return out


def _chunks(model, xs) -> Iterable:
    import torch
    xs = torch.as_tensor(xs, dtype=model.dtype, device=model.device)
    if xs.dim() == 2:
        xs = xs[None]
    B = model.max_batch
    for s in range(0, xs.shape[0], B):
        yield xs[s:s + B].contiguous()
