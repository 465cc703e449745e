"""Planted mistakes in copies of oracle steps must fail the pins (CPU only).

Each mutant is a plausible slip -- a dropped conjugate, a flipped sign, a
transposed operand, a missing term -- applied to a local copy of an oracle
function; the corresponding pin check must then report a large error.
"""
import numpy as np

import oracle.ocsc_oracle as O
from tests import test_oracle_pins as pins


def zstep_no_conj(Dh, xh, Sh, rho):
    a = Dh
    b = a * xh[None] + rho * Sh
    atb = np.sum(a * b, axis=0)
    n2 = np.sum(np.abs(a) ** 2, axis=0)
    return (b - a * (atb / (rho + n2))[None]) / rho


def zstep_no_rho_in_denominator(Dh, xh, Sh, rho):
    a = Dh
    b = np.conj(a) * xh[None] + rho * Sh
    atb = np.sum(a * b, axis=0)
    n2 = np.sum(np.abs(a) ** 2, axis=0)
    return (b - np.conj(a) * (atb / n2)[None]) / rho


def fold_wrong_sign(G, C, Zh, xh, H=None):
    u = np.moveaxis(np.conj(Zh), 0, -1)[..., None]
    G += np.conj(Zh) * xh[None]
    Cu = C @ u
    s = np.real(np.swapaxes(np.conj(u), -1, -2) @ Cu)
    C -= (Cu @ np.swapaxes(np.conj(Cu), -1, -2)) / (1.0 - s)


def fold_unconjugated(G, C, Zh, xh, H=None):
    u = np.moveaxis(Zh, 0, -1)[..., None]
    G += Zh * xh[None]
    Cu = C @ u
    s = np.real(np.swapaxes(np.conj(u), -1, -2) @ Cu)
    C -= (Cu @ np.swapaxes(np.conj(Cu), -1, -2)) / (1.0 + s)


def dstep_transposed(C, G, Vh, Th, rho_d):
    w = np.moveaxis(G + rho_d * (Vh - Th), 0, -1)[..., None]
    return np.moveaxis((np.swapaxes(C, -1, -2) @ w)[..., 0], -1, 0)


def dstep_row_form(C, G, Vh, Th, rho_d):
    # the row form of eq. sub_d_sol read literally: (b^H + rho_d v^T - rho_d theta^T) C
    w = np.moveaxis(np.conj(G) + rho_d * (Vh - Th), 0, -1)[..., None, :]
    return np.moveaxis((w @ C)[..., 0, :], -1, 0)


def test_zstep_mutants_fail_p1():
    assert pins.zstep_error() < 1e-13
    assert pins.zstep_error(zstep_no_conj) > 1e-3
    assert pins.zstep_error(zstep_no_rho_in_denominator) > 1e-3


def test_fold_mutants_fail_p2():
    assert max(pins.sm_error()) < 1e-12
    assert max(pins.sm_error(fold_wrong_sign)) > 1e-3
    assert max(pins.sm_error(fold_unconjugated)) > 1e-3


def test_dstep_mutants_fail_p6():
    assert pins.dstep_error() < 1e-12
    assert pins.dstep_error(dstep_transposed) > 1e-3
    assert pins.dstep_error(dstep_row_form) > 1e-3


def test_vstep_without_real_part_or_ball_is_caught():
    rng = np.random.default_rng(0)
    shape, filt = (8, 8), (3, 3)
    d = O.dft2(rng.standard_normal((2,) + shape) * 2)
    V = O.dict_vstep(d, 0 * d, filt, shape)
    # forgetting the ball projection leaves norms above one
    alpha = O.crop(O.idft2_real(d, shape), *filt)
    assert np.max(np.sqrt(np.sum(alpha ** 2, axis=(1, 2)))) > 1.0
    assert np.max(np.sqrt(np.sum(V ** 2, axis=(1, 2)))) <= 1.0 + 1e-15


def test_group_closed_form_catches_equal_weights():
    """The shared-dictionary pin fails when the consensus V-step averages the
    grid sizes with equal weights instead of P_s."""
    import tests.test_oracle_pins_eval as T
    rng = np.random.default_rng(22)
    filt, groups, crops = (3, 3), [], []
    for shape, n in (((8, 8), 3), ((16, 16), 5)):
        xs = [rng.standard_normal(shape) * 0.05 for _ in range(n)]
        crops += [x[:3, :3] for x in xs]
        G, C = T._delta_history(xs, shape, float(shape[0] * shape[1]))
        groups.append((G, C, float(shape[0] * shape[1]), shape))
    mean = np.mean(crops, axis=0)
    expect = mean / max(np.linalg.norm(mean), 1.0)

    def equal_weights(members, iters, filt):
        V = np.zeros((1,) + filt)
        Ths = [np.zeros_like(G) for G, _, _, _ in members]
        ds = [None] * len(members)
        for _ in range(iters):
            acc = np.zeros_like(V)
            for i, (G, C, rho_d, shape) in enumerate(members):
                ds[i] = O.dict_dstep(C, G, O.dft2(O.zero_pad(V, shape)), Ths[i], rho_d)
                acc += O.crop(O.idft2_real(ds[i] + Ths[i], shape), *filt)
            alpha = acc / len(members)
            V = alpha / np.maximum(np.sqrt(np.sum(alpha * alpha, axis=(-2, -1))), 1.0)[:, None, None]
            for i, (G, C, rho_d, shape) in enumerate(members):
                Ths[i] = Ths[i] + ds[i] - O.dft2(O.zero_pad(V, shape))
        return V
    assert np.linalg.norm(O.dict_update_group(groups, 3000, filt)[1][0] - expect) < 1e-8
    assert np.linalg.norm(equal_weights(groups, 3000, filt)[0] - expect) > 1e-2
