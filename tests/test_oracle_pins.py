"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each check computes the expected value by a route the oracle does not take
(dense solves, explicit DFT matrices, direct convolution loops, brute force,
projected gradient, the paper's own printed recursion) so that a dropped term,
a wrong sign, a missing conjugate or a transposed operand fails at least one.
"""
import numpy as np
import pytest

import oracle.ocsc_oracle as O
import synth
from tests import refs


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------- P1: Z-step

def zstep_error(zstep=O.code_zstep, seed=0):
    """Z-step (Sherman-Morrison form) vs a dense solve of its normal equations."""
    rng = np.random.default_rng(seed)
    K, F, rho = 6, 9, 0.7
    a, x, s = rand_c(rng, K, F), rand_c(rng, F), rand_c(rng, K, F)
    z = zstep(a, x, s, rho)
    err = 0.0
    for f in range(F):
        M = np.outer(np.conj(a[:, f]), a[:, f]) + rho * np.eye(K)
        b = np.conj(a[:, f]) * x[f] + rho * s[:, f]
        err = max(err, rel(z[:, f], np.linalg.solve(M, b)))
    return err


def test_p1_zstep_matches_dense_solve():
    assert zstep_error() < 1e-13


def test_p1_zstep_minimises_per_frequency_quadratic():
    # z minimises |x - a^T z|^2/2 + rho/2 ||z - s||^2: random perturbations never decrease it.
    rng = np.random.default_rng(1)
    K, rho = 5, 1.3
    a, x, s = rand_c(rng, K, 1), rand_c(rng, 1), rand_c(rng, K, 1)
    z = O.code_zstep(a, x, s, rho)[:, 0]

    def f(zz):
        return 0.5 * abs(x[0] - a[:, 0] @ zz) ** 2 + 0.5 * rho * np.linalg.norm(zz - s[:, 0]) ** 2
    f0 = f(z)
    for _ in range(200):
        assert f(z + 1e-3 * rand_c(rng, K)) >= f0 - 1e-14


# ------------------------------------------------------ P2: C recursion (R8)

def paper_printed_recursion(Zs, rho_P):
    """eq. C_update exactly as printed (row vectors Z_t(p,:), t/(t-1) factors)."""
    Cs = []
    C = None
    for t, z in enumerate(Zs, start=1):
        r = z[None, :]                       # 1 x K row
        rH = np.conj(r).T                    # K x 1 column
        if t == 1:
            C = np.eye(len(z)) / rho_P - (rH @ r) / rho_P / (rho_P + (r @ rH)[0, 0])
        else:
            C = t / (t - 1) * (C - (C @ rH @ r @ C) / ((t - 1) + (r @ C @ rH)[0, 0]))
        Cs.append(C.copy())
    return Cs


def sm_error(fold=O.history_fold, seed=2):
    rng = np.random.default_rng(seed)
    K, F, T, rho_d = 4, 3, 20, 3.7
    G = np.zeros((K, F), complex)
    C = np.broadcast_to(np.eye(K) / rho_d, (F, K, K)).astype(complex)
    H = np.zeros((F, K, K), complex)
    Zs = [rand_c(rng, K, F) for _ in range(T)]
    e_inv, e_paper = 0.0, 0.0
    printed = [paper_printed_recursion([Z[:, f] for Z in Zs], rho_d) for f in range(F)]
    for t, Z in enumerate(Zs, start=1):
        fold(G, C, Z, rand_c(rng, F))
        for f in range(F):
            Hf = sum(np.outer(np.conj(Zi[:, f]), Zi[:, f]) for Zi in Zs[:t])
            e_inv = max(e_inv, rel(C[f], np.linalg.inv(Hf + rho_d * np.eye(K))))
            e_paper = max(e_paper, rel(t * C[f], printed[f][t - 1]))
    return e_inv, e_paper


def test_p2_sherman_morrison_equals_inverse_and_paper_recursion():
    e_inv, e_paper = sm_error()
    assert e_inv < 1e-12
    assert e_paper < 1e-12


def test_p2_history_sums():
    rng = np.random.default_rng(3)
    K, F = 3, 5
    G = np.zeros((K, F), complex)
    C = np.broadcast_to(np.eye(K), (F, K, K)).astype(complex)
    H = np.zeros((F, K, K), complex)
    Zs, xs = [rand_c(rng, K, F) for _ in range(4)], [rand_c(rng, F) for _ in range(4)]
    for Z, x in zip(Zs, xs):
        O.history_fold(G, C, Z, x, H)
    for f in range(F):
        assert rel(G[:, f], sum(np.conj(Z[:, f]) * x[f] for Z, x in zip(Zs, xs))) < 1e-14
        assert rel(H[f], sum(np.outer(np.conj(Z[:, f]), Z[:, f]) for Z in Zs)) < 1e-14


# ----------------------------------------------------------- P3: soft threshold

def test_p3_soft_threshold_is_the_prox():
    rng = np.random.default_rng(4)
    v = rng.standard_normal(200) * 3
    kappa = 0.9
    u = O.soft_threshold(v, kappa)
    grid = np.linspace(-12, 12, 240001)
    for vi, ui in zip(v[:40], u[:40]):
        g = grid[np.argmin(kappa * np.abs(grid) + 0.5 * (grid - vi) ** 2)]
        assert abs(g - ui) <= 1e-4
    nz = u != 0
    assert np.allclose(v[nz] - u[nz], kappa * np.sign(u[nz]), atol=1e-15)
    assert np.all(np.abs(v[~nz]) <= kappa)
    assert O.soft_threshold(np.array([kappa, -kappa]), kappa).tolist() == [0.0, 0.0]


# ------------------------------------------------ P4: DFT, Parseval, convolution

@pytest.mark.parametrize("half", [True, False])
def test_p4_dft_against_definition_and_parseval(half):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((8, 16))
    X = O.dft2(x, half)
    full = refs.naive_dft2(x)
    assert rel(X, full[:, : X.shape[1]]) < 1e-13
    P = x.size
    assert abs(np.sum(O.parseval_weights(x.shape, half) * np.abs(X) ** 2) / P - np.sum(x * x)) < 1e-10
    assert rel(O.idft2_real(X, x.shape, half), x) < 1e-14


@pytest.mark.parametrize("half", [True, False])
def test_p4_convolution_theorem_is_circular(half):
    rng = np.random.default_rng(6)
    d, z = rng.standard_normal((3, 4)), rng.standard_normal((8, 8))
    via_f = O.idft2_real(O.dft2(O.zero_pad(d, z.shape), half) * O.dft2(z, half), z.shape, half)
    assert rel(via_f, refs.circ_conv2(d, z)) < 1e-13


def test_p4_paper_toeplitz_operator_wraps_around():
    # The printed T(D(:,k)) has D(2,k) in its top-right corner: circular convolution.
    d = np.array([1.0, 2.0, 3.0])
    T = refs.toeplitz_operator(d[:, None], (5, 1))
    assert T[0, -1] == 2.0 and T[1, -1] == 3.0 and T[0, 0] == 1.0 and T[-1, -1] == 1.0


# ------------------------------------------- P5: Proposition 1 with its constant

@pytest.mark.parametrize("half", [True, False])
def test_p5_proposition1_reorders_the_loss_by_frequency(half):
    rng = np.random.default_rng(7)
    shape, K, M, T = (6, 8), 2, (3, 2), 3
    D = rng.standard_normal((K,) + M)
    xs = [rng.standard_normal(shape) for _ in range(T)]
    Zs = [rng.standard_normal((K,) + shape) for _ in range(T)]
    lhs = sum(0.5 * np.sum((x - sum(refs.circ_conv2(D[k], Z[k]) for k in range(K))) ** 2)
              for x, Z in zip(xs, Zs))
    fshape = O.dft2(xs[0], half).shape
    G = np.zeros((K,) + fshape, complex)
    C = np.broadcast_to(np.eye(K), fshape + (K, K)).astype(complex)
    H = np.zeros(fshape + (K, K), complex)
    sx = 0.0
    w = O.parseval_weights(shape, half)
    for x, Z in zip(xs, Zs):
        xh = O.dft2(x, half)
        O.history_fold(G, C, O.dft2(Z, half), xh, H)
        sx += np.sum(w * np.abs(xh) ** 2)
    rhs = O.surrogate(O.dft2(O.zero_pad(D, shape), half), H, G, sx, 0.0, 0.0, shape, half)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


# --------------------------------------------------------- P6: D-step (R7)

def dstep_error(dstep=O.dict_dstep, seed=8):
    rng = np.random.default_rng(seed)
    K, F, T, rho_d = 3, 4, 5, 2.5
    Zs, xs = [rand_c(rng, K, F) for _ in range(T)], [rand_c(rng, F) for _ in range(T)]
    G = np.zeros((K, F), complex)
    C = np.broadcast_to(np.eye(K) / rho_d, (F, K, K)).astype(complex)
    for Z, x in zip(Zs, xs):
        O.history_fold(G, C, Z, x)
    Vh, Th = rand_c(rng, K, F), rand_c(rng, K, F)
    d = dstep(C, G, Vh, Th, rho_d)
    err = 0.0
    for f in range(F):
        A = np.vstack([np.stack([Z[:, f] for Z in Zs]), np.sqrt(rho_d) * np.eye(K)])
        y = np.concatenate([[x[f] for x in xs], np.sqrt(rho_d) * (Vh[:, f] - Th[:, f])])
        ls = np.linalg.lstsq(A, y, rcond=None)[0]
        err = max(err, rel(d[:, f], ls))
    return err


def test_p6_dstep_is_stacked_least_squares():
    assert dstep_error() < 1e-12


# ------------------------------------------------ P7: V-step (Proposition 2)

def test_p7_vstep_projection_properties():
    rng = np.random.default_rng(9)
    shape, filt, K = (8, 8), (3, 3), 4
    planes = rng.standard_normal((K,) + shape) * 0.4
    Th = O.dft2(rng.standard_normal((K,) + shape) * 0.2)
    d = O.dft2(planes)
    V = O.dict_vstep(d, Th, filt, shape)
    assert V.shape == (K,) + filt
    assert np.all(np.sqrt(np.sum(V ** 2, axis=(1, 2))) <= 1 + 1e-15)
    # alpha from the explicit inverse DFT matrix (not the oracle's FFT)
    full = np.concatenate([d + Th, np.conj((d + Th)[:, (-np.arange(8)) % 8, 1:4][:, :, ::-1])], axis=2)
    Fi = refs.dft_matrix(8, +1) / 8
    alpha = np.real(np.einsum("ij,kjl,ml->kim", Fi, full, Fi))[:, :3, :3]
    for k in range(K):
        for _ in range(50):
            Y = refs.project_ball(rng.standard_normal(filt) * rng.uniform(0.1, 2))
            assert np.sum((alpha[k] - V[k]) * (Y - V[k])) <= 1e-13
    # special cases: inside the ball it is the identity; zero maps to zero
    small = O.dict_vstep(d * 1e-3, Th * 1e-3, filt, shape)
    assert rel(small, alpha * 1e-3) < 1e-12
    assert np.all(O.dict_vstep(0 * d, 0 * Th, filt, shape) == 0)


def test_p7_vstep_solves_the_frequency_domain_subproblem():
    # min_V ||c - F(zp V)||^2, ||V|| <= 1, by a generic constrained solver.
    from scipy.optimize import minimize
    rng = np.random.default_rng(10)
    shape, filt = (4, 4), (2, 2)
    c = O.dft2(rng.standard_normal((1,) + shape) * 0.8, half=False)
    V = O.dict_vstep(c, 0 * c, filt, shape, half=False)[0]

    def f(v):
        return float(np.sum(np.abs(c[0] - refs.naive_dft2(O.zero_pad(v.reshape(filt), shape))) ** 2))
    res = minimize(f, np.zeros(4), constraints=[{"type": "ineq", "fun": lambda v: 1 - v @ v}],
                   method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
    assert np.linalg.norm(res.x - V.ravel()) < 1e-5
    assert f(V.ravel()) <= res.fun + 1e-9


# ---------------------------------------------------- P8: dual telescoping

def test_p8_theta_is_sum_of_primal_residuals():
    rng = np.random.default_rng(11)
    shape, filt, K, T = (8, 8), (3, 3), 3, 4
    fshape = (8, 5)
    G = np.zeros((K,) + fshape, complex)
    C = np.broadcast_to(np.eye(K) / 64.0, fshape + (K, K)).astype(complex)
    for _ in range(T):
        O.history_fold(G, C, O.dft2(rng.standard_normal((K,) + shape)), O.dft2(rng.standard_normal(shape)))
    trace = []
    O.dict_update(G, C, 64.0, 6, filt, shape, True, trace)
    acc = np.zeros_like(G)
    for d, V, Th in trace:
        acc = acc + d - O.dft2(O.zero_pad(V, shape))
        assert rel(Th, acc) < 1e-13


# ---------------------------------------- P9: DictOCSC closed form (K=1, codes = delta)

@pytest.mark.parametrize("scale", [0.05, 3.0])
def test_p9_dictocsc_closed_form_delta_codes(scale):
    rng = np.random.default_rng(12)
    shape, filt, T = (8, 8), (3, 3), 5
    xs = [rng.standard_normal(shape) * scale for _ in range(T)]
    fshape = (8, 5)
    G = np.zeros((1,) + fshape, complex)
    C = np.broadcast_to(np.eye(1) / 64.0, fshape + (1, 1)).astype(complex)
    delta = np.zeros((1,) + shape)
    delta[0, 0, 0] = 1.0
    for x in xs:
        O.history_fold(G, C, O.dft2(delta), O.dft2(x))
    d, V, Th = O.dict_update(G, C, 64.0, 2000, filt, shape)
    want = refs.project_ball(np.mean(xs, axis=0)[:3, :3])
    assert np.max(np.abs(V[0] - want)) < 1e-8


# --------------------------- P10: DictOCSC vs projected gradient on the spatial surrogate

def test_p10_dictocsc_matches_projected_gradient_on_toeplitz_form():
    rng = np.random.default_rng(13)
    shape, filt, K, T = (6, 6), (3, 3), 2, 4
    Zs = [rng.standard_normal((K,) + shape) for _ in range(T)]
    Dtrue = rng.standard_normal((K,) + filt) * 0.7
    xs = [sum(refs.circ_conv2(Dtrue[k], Z[k]) for k in range(K)) + 0.3 * rng.standard_normal(shape)
          for Z in Zs]
    As = [np.hstack([refs.code_shift_matrix(Z[k], filt) for k in range(K)]) for Z in Zs]
    want = refs.fista_ball(As, [x.ravel() for x in xs], K, 9, iters=20000).reshape((K,) + filt)
    fshape = (6, 4)
    G = np.zeros((K,) + fshape, complex)
    C = np.broadcast_to(np.eye(K) / 36.0, fshape + (K, K)).astype(complex)
    for Z, x in zip(Zs, xs):
        O.history_fold(G, C, O.dft2(Z), O.dft2(x))
    d, V, Th = O.dict_update(G, C, 36.0, 6000, filt, shape)
    assert np.max(np.abs(V - want)) < 1e-7


# ------------------------------------------------ P11: code ADMM vs brute-force lasso

def test_p11_code_admm_reaches_bruteforce_lasso():
    rng = np.random.default_rng(14)
    shape, lam = (3, 3), 0.3
    filt = rng.standard_normal((2, 2))
    x = rng.standard_normal(shape)
    A = refs.toeplitz_operator(filt, shape)
    u_bf, f_bf = refs.brute_force_lasso(A, x.ravel(), lam)
    Dh = O.dft2(O.zero_pad(filt[None], shape), half=False)
    U, Zh, xh = O.code_update(x, Dh, lam, 1.0, 5000, half=False)
    f_admm = refs.lasso_objective(A, x.ravel(), U[0].ravel(), lam)
    assert abs(f_admm - f_bf) / f_bf < 1e-9
    # A is invertible here, so the lasso is strictly convex and its minimiser unique
    assert np.linalg.matrix_rank(A) == 9
    assert np.max(np.abs(U[0].ravel() - u_bf)) < 1e-7


# ------------------------------------------------ P12: identity filter -> soft threshold

def test_p12_identity_filter_gives_soft_threshold():
    rng = np.random.default_rng(15)
    x = rng.standard_normal((8, 8)) * 2
    Dh = O.dft2(O.zero_pad(np.ones((1, 1, 1)), x.shape))
    U, _, _ = O.code_update(x, Dh, 0.7, 1.0, 400)
    assert np.max(np.abs(U[0] - O.soft_threshold(x, 0.7))) < 1e-10


# ------------------------------------------------ P13 / P14: equivariances

def test_p13_shift_equivariance():
    rng = np.random.default_rng(16)
    x = rng.standard_normal((16, 16))
    Dh = O.dft2(O.zero_pad(rng.standard_normal((3, 4, 4)), x.shape))
    U1, _, _ = O.code_update(x, Dh, 0.2, 1.0, 10)
    U2, _, _ = O.code_update(np.roll(x, (3, 5), axis=(0, 1)), Dh, 0.2, 1.0, 10)
    assert rel(U2, np.roll(U1, (3, 5), axis=(1, 2))) < 1e-12


def test_p14_scale_equivariance_at_every_iteration():
    rng = np.random.default_rng(17)
    x = rng.standard_normal((16, 16))
    Dh = O.dft2(O.zero_pad(rng.standard_normal((3, 4, 4)), x.shape))
    for it in (1, 2, 7):
        U1, _, _ = O.code_update(x, Dh, 0.2, 1.0, it)
        U2, _, _ = O.code_update(4.0 * x, Dh, 0.8, 1.0, it)
        assert rel(U2, 4.0 * U1) < 1e-12


# ------------------------------------------------ P15: half vs full spectrum

def test_p15_half_and_full_spectrum_trajectories_agree():
    wl = synth.WORKLOADS["ocsc_64x64_k16_f64"]
    xs = synth.images(wl, range(4))[:, :32, :32].copy()
    D0 = synth.initial_dictionary(6, 5, 5)
    runs = []
    for half in (True, False):
        m = O.OCSC(6, 5, 5, 32, 32, 0.1, 1.0, iters_code=6, iters_dict=6, half=half, keep_history=True)
        m.set_dictionary(D0)
        Us = [m.step(x[None]) for x in xs]
        runs.append((np.stack(Us), m.get_dictionary(), m))
    assert rel(runs[0][0], runs[1][0]) < 1e-12
    assert rel(runs[0][1], runs[1][1]) < 1e-12
    H = runs[1][2].H                                  # full spectrum: H(-p) = conj(H(p))
    neg = H[(-np.arange(32)) % 32][:, (-np.arange(32)) % 32]
    assert rel(neg, np.conj(H)) < 1e-13


# ------------------------------------------------ P16: monotone online surrogate

def test_p16_online_surrogate_is_monotone_at_converged_dictocsc():
    wl = synth.WORKLOADS["ocsc_64x64_k16_f64"]
    xs = synth.images(wl, range(6))[:, :32, :32].copy()
    m = O.OCSC(4, 5, 5, 32, 32, 0.1, 1.0, iters_code=10, iters_dict=600, keep_history=True)
    m.set_dictionary(synth.initial_dictionary(4, 5, 5))
    shape = (32, 32)
    V_prev = None
    for x in xs:
        m.code_update(x[None])
        m.history_accumulate()
        if V_prev is not None:
            before = m.surrogate_at(O.dft2(O.zero_pad(V_prev, shape)))
        m.dict_update()
        if V_prev is not None:
            after = m.surrogate_at(O.dft2(O.zero_pad(m.V, shape)))
            assert after <= before + 1e-10 * abs(before)
        V_prev = m.V.copy()


# ------------------------------------------------ P17: non-degenerate workload

def test_p17_parity_workload_is_not_degenerate():
    wl = synth.WORKLOADS["ocsc_64x64_k16_f64"]
    xs = synth.images(wl, range(wl.n_images))
    m = O.OCSC(wl.K, wl.filt_h, wl.filt_w, wl.pad_h, wl.pad_w, wl.lam, wl.rho,
               iters_code=wl.iters_code, iters_dict=wl.iters_dict)
    m.set_dictionary(synth.initial_dictionary(wl.K, wl.filt_h, wl.filt_w, wl.seed))
    rels = []
    for i in synth.pass_order(wl.n_images, wl.seed, 0):
        U = m.code_update(xs[i][None])
        f = m.objective(xs[i][None], U)[0]
        rels.append(f / (0.5 * np.sum(xs[i] ** 2)))
        if len(rels) == 1:
            assert np.count_nonzero(U) > 0
        m.history_accumulate()
        m.dict_update()
    assert np.mean(rels[:10]) < 0.9
    norms = np.sqrt(np.sum(m.get_dictionary() ** 2, axis=(1, 2)))
    assert np.median(norms) > 0.5
