"""Pins of the oracle's evaluation and diagnostic parts, and of the state a
checkpoint must hold (P18-P22), each against a route the oracle does not take.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests import refs


def small_model(warm=False, keep=False, iters_dict=10):
    m = O.OCSC(4, 5, 5, 32, 32, 0.1, 1.0, iters_code=10, iters_dict=iters_dict, keep_history=keep,
               warm_start=warm)
    m.set_dictionary(synth.initial_dictionary(4, 5, 5))
    return m


def small_images(n):
    wl = synth.WORKLOADS["ocsc_64x64_k16_f64"]
    return synth.images(wl, range(n))[:, :32, :32].copy()


# --------------------------------------------- P18: checkpoint = the listed state

@pytest.mark.parametrize("warm", [False, True])
def test_p18_listed_state_is_a_complete_checkpoint(warm):
    """Cold start: D~, G, C and t determine the future; warm start adds V and Theta.
    A fresh learner given only those continues bit for bit like the original."""
    xs = small_images(6)
    a = small_model(warm=warm)
    for x in xs[:3]:
        a.step(x[None])
    b = small_model(warm=warm)
    b.set_dictionary(np.zeros((4, 5, 5)))           # nothing else may leak through
    cp = lambda z: z.copy(order="K")                # same memory layout -> same BLAS rounding
    b.Dh, b.G, b.C, b.t = cp(a.Dh), cp(a.G), cp(a.C), a.t
    if warm:
        b.V, b.Th = cp(a.V), cp(a.Th)
    for x in xs[3:]:
        ua = a.step(x[None])
        ub = b.step(x[None])
        assert np.array_equal(ua, ub)
    assert np.array_equal(a.Dh, b.Dh)


def test_p18_cold_start_does_not_read_v_or_theta():
    xs = small_images(3)
    a = small_model()
    b = small_model()
    for x in xs[:2]:
        a.step(x[None])
        b.step(x[None])
    b.V = np.full_like(b.V, 7.0)
    b.Th = np.full_like(b.Th, 3.0 + 1j)
    a.step(xs[2][None])
    b.step(xs[2][None])
    assert np.array_equal(a.Dh, b.Dh)


# ------------------------------------------------ P19: warm-start DictOCSC

def test_p19_two_warm_updates_equal_one_cold_update_of_twice_the_length():
    """With no sample folded in between, warm start continues the same ADMM run."""
    xs = small_images(3)
    warm = small_model(warm=True, iters_dict=7)
    cold = small_model(iters_dict=14)
    for x in xs:
        for m in (warm, cold):
            m.code_update(x[None])
            m.history_accumulate()
    warm.dict_update()
    warm.dict_update()
    cold.dict_update()
    assert np.linalg.norm(warm.Dh - cold.Dh) / np.linalg.norm(cold.Dh) < 1e-13
    assert np.linalg.norm(warm.V - cold.V) / np.linalg.norm(cold.V) < 1e-13


def test_p19_warm_start_from_zero_is_cold_start():
    xs = small_images(1)
    warm, cold = small_model(warm=True), small_model()
    for m in (warm, cold):
        m.step(xs[0][None])
    assert np.array_equal(warm.Dh, cold.Dh)


# ---------------------------------------------------- P20: diagnostics

def test_p20_primal_residual_is_the_last_change_of_theta():
    xs = small_images(2)
    m = small_model()
    m.step(xs[0][None])
    m.code_update(xs[1][None])
    m.history_accumulate()
    trace = []
    m.dict_update(trace)
    dg = m.diagnostics()
    dTh = trace[-1][2] - trace[-2][2]
    r = O.idft2_real(dTh, (32, 32))
    assert abs(dg["primal_residual"] - np.sqrt(np.sum(r * r))) < 1e-12 * max(dg["primal_residual"], 1e-300)
    assert np.all(dg["V_norms"] <= 1.0 + 1e-12)
    assert dg["primal_residual"] > 0


def test_p20_norms_of_a_set_dictionary():
    rng = np.random.default_rng(3)
    D = rng.standard_normal((4, 5, 5))
    m = small_model()
    m.set_dictionary(D)
    dg = m.diagnostics()
    assert abs(dg["dict_norm"] - np.linalg.norm(D)) < 1e-12 * np.linalg.norm(D)
    assert np.allclose(dg["D_norms"], np.sqrt(np.sum(D * D, axis=(1, 2))), rtol=1e-12, atol=0)
    # V = 0 before any update: the primal residual is the whole dictionary
    assert abs(dg["primal_residual"] - np.linalg.norm(D)) < 1e-12 * np.linalg.norm(D)


# ------------------------------------------------ P21: the terms of eq. csc

def test_p21_objective_terms_match_direct_circular_convolution():
    rng = np.random.default_rng(4)
    shape, K, M = (6, 8), 3, (3, 2)
    D = rng.standard_normal((K,) + M)
    U = rng.standard_normal((K,) + shape) * (rng.random((K,) + shape) < 0.3)
    x = rng.standard_normal(shape)
    Dh = O.dft2(O.zero_pad(D, shape))
    data, l1 = O.objective_terms(x, U, Dh)
    rec = sum(refs.circ_conv2(D[k], U[k]) for k in range(K))
    assert abs(data - 0.5 * np.sum((x - rec) ** 2)) < 1e-12 * data
    assert abs(l1 - np.sum(np.abs(U))) < 1e-12 * l1
    assert abs(O.objective(x, U, Dh, 0.3) - (data + 0.3 * l1)) < 1e-12 * data


# ----------------------------------------------------------- P22: PSNR

def test_p22_psnr_of_a_constant_error():
    x = np.zeros((16, 16))
    for c in (1.0, 2.5, 255.0):
        assert abs(O.psnr(x, x + c) - 20.0 * np.log10(255.0 / c)) < 1e-12
    assert abs(O.psnr(x, x + 0.5, peak=1.0) - 20.0 * np.log10(2.0)) < 1e-12


# ------------------------------------- P23: DictOCSC shared across grid sizes

def _delta_history(xs, shape, rho_d):
    """History of delta codes (every code spectrum = 1) for K = 1 on one grid."""
    fshape = O.dft2(np.zeros(shape)).shape
    G = np.zeros((1,) + fshape, complex)
    C = np.broadcast_to(np.eye(1) / rho_d, fshape + (1, 1)).astype(complex)
    for x in xs:
        O.history_fold(G, C, np.ones((1,) + fshape, complex), O.dft2(x))
    return G, C


def test_p23_group_with_one_member_is_dict_update():
    rng = np.random.default_rng(21)
    shape, filt, K = (8, 8), (3, 3), 3
    fshape = (8, 5)
    G = np.zeros((K,) + fshape, complex)
    C = np.broadcast_to(np.eye(K) / 64.0, fshape + (K, K)).astype(complex)
    for _ in range(4):
        O.history_fold(G, C, O.dft2(rng.standard_normal((K,) + shape)), O.dft2(rng.standard_normal(shape)))
    d1, V1, T1 = O.dict_update(G, C, 64.0, 7, filt, shape)
    ds, V, Ts = O.dict_update_group([(G, C, 64.0, shape)], 7, filt)
    assert np.array_equal(d1, ds[0]) and np.array_equal(V1, V) and np.array_equal(T1, Ts[0])


@pytest.mark.parametrize("scale", [0.05, 3.0])
def test_p23_group_closed_form_delta_codes(scale):
    """K = 1, every code a delta, samples on an 8x8 and a 16x16 grid: the
    shared filter minimises the sum of all samples' spatial losses over the
    unit ball, i.e. it is the projection of the mean crop of all samples."""
    rng = np.random.default_rng(22)
    filt = (3, 3)
    groups = []
    crops = []
    for shape, n in (((8, 8), 3), ((16, 16), 5)):
        xs = [rng.standard_normal(shape) * scale for _ in range(n)]
        crops += [x[:3, :3] for x in xs]
        rho_d = 1.0 * shape[0] * shape[1]
        G, C = _delta_history(xs, shape, rho_d)
        groups.append((G, C, rho_d, shape))
    mean = np.mean(crops, axis=0)
    expect = mean / max(np.linalg.norm(mean), 1.0)
    ds, V, Ts = O.dict_update_group(groups, 3000, filt)
    assert np.linalg.norm(V[0] - expect) < 1e-8 * max(np.linalg.norm(expect), 1e-3)
