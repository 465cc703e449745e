"""Plain FP64 CPU oracle of online convolutional sparse coding (OCSC).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path (the HIP library
and its Python binding) never does.  It shares no code with the GPU path.

Everything is float64 / complex128 and written for reading against the paper
(Wang, Yao, Kwok, Ni: "Scalable Online Convolutional Sparse Coding"), not for
speed: NumPy's FFT and stacked matrix products are the only library primitives.

Conventions (readings of the paper where it is silent or garbled):

* DFT: ``F`` is the unnormalised 2-D DFT and ``F^-1`` carries the 1/P factor,
  which is what makes the 1/(2P) factor of the frequency-domain objective come
  from Parseval's theorem (Section 2.3, eq. fcsc).
* Convolution is circular on the padded P_h x P_w grid (the frequency product of
  Section 2.3 and the wrap-around Toeplitz operator of Section 3.4 are both
  circular).  Filters and images sit at offset (0, 0) of the grid; the operator
  H of eq. fcsc is the crop to the top-left M_h x M_w block.
* ``half=True`` stores only the frequencies of ``numpy.fft.rfft2`` (columns
  0..P_w/2); ``half=False`` stores the full spectrum.  Both give the same
  trajectory up to rounding.
* Code update (eq. fcsc_code, "solved by ADMM", steps not printed): scaled ADMM
  (Section 2.2) with the split constraint ``U_k = F^-1 Z_k`` written in space and
  penalty rho/2; per frequency p the Z-step solves
  ``(conj(a_p) a_p^T + rho I) z_p = conj(a_p) x_p + rho s_p`` with ``a_p`` the
  dictionary spectrum at p and ``s = F(U - W)``; the U-step is the soft
  threshold at lambda/rho; the dual is ``W += Y - U``.  U = W = 0 at the start of
  every sample.  The spectrum that enters the history is the last Z-step iterate.
* History (eqs. A_update, B_update, C_update): unnormalised sums
  ``H_p = sum_i conj(z_ip) z_ip^T`` and ``G_p = sum_i conj(z_ip) x_ip``, and
  ``C_p = (H_p + rho_d I)^-1`` kept by the Sherman-Morrison formula from
  ``C_p = I / rho_d``.  The paper's printed recursion (with its t/(t-1)
  factors) equals ``t * C_p``; the constrained minimiser is the same.
* D-step (eq. sub_d_sol) in column form: ``d_p = C_p (G_p + rho_d (v_p - theta_p))``,
  the exact minimiser of the per-frequency quadratic plus the ADMM penalty;
  ``rho_d`` defaults to rho * P as in eq. sub_d_sol.
* DictOCSC (Algorithm 2) starts every call from V = 0, Theta = 0 and returns the
  last D-step iterate, which codes the next sample.  ``warm_start=True`` is a
  variant that carries V and Theta from one call to the next.
* V-step (Proposition 2): ``alpha_k = crop(Re F^-1(d_k + theta_k))``,
  ``V_k = alpha_k / max(||alpha_k||_2, 1)``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "dft2", "idft2_real", "parseval_weights", "zero_pad", "crop",
    "soft_threshold", "code_zstep", "code_update", "history_fold",
    "dict_dstep", "dict_vstep", "dict_update", "objective", "surrogate", "OCSC",
]


# --------------------------------------------------------------------------
# Transforms and the support operator (Section 2.3, eq. fcsc)
# --------------------------------------------------------------------------

def dft2(x: np.ndarray, half: bool = True) -> np.ndarray:
    """Unnormalised 2-D DFT over the last two axes of a real array."""
    x = np.asarray(x, dtype=np.float64)
    return np.fft.rfft2(x) if half else np.fft.fft2(x)


def idft2_real(X: np.ndarray, shape, half: bool = True) -> np.ndarray:
    """Real part of the inverse 2-D DFT (with its 1/P factor) over the last two axes."""
    if half:
        return np.fft.irfft2(X, s=tuple(shape))
    return np.real(np.fft.ifft2(X))


def parseval_weights(shape, half: bool = True) -> np.ndarray:
    """Multiplicity of each stored frequency in the full spectrum, shape (P_h, W_f).

    With the half spectrum, columns 1..P_w/2-1 stand for themselves and their
    conjugate mirror, so they count twice; columns 0 and P_w/2 count once.
    """
    ph, pw = shape
    if not half:
        return np.ones((ph, pw))
    wf = pw // 2 + 1
    w = np.full((ph, wf), 2.0)
    w[:, 0] = 1.0
    if pw % 2 == 0:
        w[:, -1] = 1.0
    return w


def zero_pad(D: np.ndarray, shape) -> np.ndarray:
    """Place (..., M_h, M_w) filters at offset (0, 0) of a zero (..., P_h, P_w) grid."""
    out = np.zeros(D.shape[:-2] + tuple(shape))
    out[..., : D.shape[-2], : D.shape[-1]] = D
    return out


def crop(Y: np.ndarray, mh: int, mw: int) -> np.ndarray:
    """The operator H of eq. fcsc: keep the top-left M_h x M_w block."""
    return Y[..., :mh, :mw].copy()


# --------------------------------------------------------------------------
# Code update (eq. fcsc_code by scaled ADMM, Section 2.2)
# --------------------------------------------------------------------------

def soft_threshold(v: np.ndarray, kappa: float) -> np.ndarray:
    """Proximal map of kappa*|.|: sign(v) * max(|v| - kappa, 0)."""
    return np.sign(v) * np.maximum(np.abs(v) - kappa, 0.0)


def code_zstep(Dh: np.ndarray, xh: np.ndarray, Sh: np.ndarray, rho: float) -> np.ndarray:
    """Z-step of the code ADMM at every frequency.

    Solves ``(conj(a) a^T + rho I) z = b`` with ``b = conj(a) x + rho s`` by the
    Sherman-Morrison formula, ``z = (b - conj(a) (a^T b) / (rho + ||a||^2)) / rho``.
    Shapes: Dh (K, ...), xh (...), Sh (K, ...); returns (K, ...).
    """
    a = Dh
    b = np.conj(a) * xh[None] + rho * Sh
    atb = np.sum(a * b, axis=0)
    n2 = np.sum(np.abs(a) ** 2, axis=0)
    return (b - np.conj(a) * (atb / (rho + n2))[None]) / rho


def code_update(x: np.ndarray, Dh: np.ndarray, lam: float, rho: float, iters: int,
                half: bool = True):
    """Sparse codes of one image against the dictionary spectrum ``Dh``.

    Returns (U, Zh, xh): the spatial codes U (K, P_h, P_w) after ``iters``
    iterations, the last Z-step iterate Zh and the image spectrum xh.
    """
    shape = x.shape
    K = Dh.shape[0]
    xh = dft2(x, half)
    U = np.zeros((K,) + shape)
    W = np.zeros((K,) + shape)
    Zh = None
    for _ in range(iters):
        Sh = dft2(U - W, half)
        Zh = code_zstep(Dh, xh, Sh, rho)
        Y = idft2_real(Zh, shape, half)
        U = soft_threshold(Y + W, lam / rho)
        W = W + Y - U
    return U, Zh, xh


# --------------------------------------------------------------------------
# History (eqs. A_update, B_update, C_update)
# --------------------------------------------------------------------------

def history_fold(G: np.ndarray, C: np.ndarray, Zh: np.ndarray, xh: np.ndarray,
                 H: np.ndarray | None = None) -> None:
    """Fold one sample's spectra into the history, in place.

    G (K, ...) += conj(z) x;  C (..., K, K) <- C - (C u)(C u)^H / (1 + u^H C u)
    with u = conj(z), i.e. C stays (H + rho_d I)^-1;  H (..., K, K) += u u^H.
    """
    u = np.moveaxis(np.conj(Zh), 0, -1)[..., None]          # (..., K, 1)
    G += np.conj(Zh) * xh[None]
    Cu = C @ u
    s = np.real(np.swapaxes(np.conj(u), -1, -2) @ Cu)        # (..., 1, 1)
    C -= (Cu @ np.swapaxes(np.conj(Cu), -1, -2)) / (1.0 + s)
    if H is not None:
        H += u @ np.swapaxes(np.conj(u), -1, -2)


# --------------------------------------------------------------------------
# Dictionary update (Algorithm 2 DictOCSC; eq. sub_d_sol; Proposition 2)
# --------------------------------------------------------------------------

def dict_dstep(C: np.ndarray, G: np.ndarray, Vh: np.ndarray, Th: np.ndarray,
               rho_d: float) -> np.ndarray:
    """D-step: ``d_p = C_p (G_p + rho_d (v_p - theta_p))`` at every frequency."""
    w = np.moveaxis(G + rho_d * (Vh - Th), 0, -1)[..., None]  # (..., K, 1)
    return np.moveaxis((C @ w)[..., 0], -1, 0)


def dict_vstep(d: np.ndarray, Th: np.ndarray, filt, shape, half: bool = True) -> np.ndarray:
    """V-step (Proposition 2): crop the real inverse DFT, then project on the unit ball."""
    alpha = crop(idft2_real(d + Th, shape, half), *filt)
    nrm = np.sqrt(np.sum(alpha * alpha, axis=(-2, -1)))
    return alpha / np.maximum(nrm, 1.0)[:, None, None]


def dict_update(G: np.ndarray, C: np.ndarray, rho_d: float, iters: int, filt, shape,
                half: bool = True, trace: list | None = None,
                V0: np.ndarray | None = None, Th0: np.ndarray | None = None):
    """DictOCSC: ``iters`` ADMM iterations from V = 0, Theta = 0.

    Returns (d, V, Th): the last D-step iterate (the new dictionary spectrum),
    the last feasible V and the last scaled dual.  If ``trace`` is a list, the
    per-iteration (d, V, Th) are appended to it.  Given V0 and Th0 the
    iterations start from them instead (warm start, a variant: Algorithm 2
    itself starts from zero).
    """
    K = G.shape[0]
    V = np.zeros((K,) + tuple(filt)) if V0 is None else np.array(V0, dtype=np.float64)
    Th = np.zeros_like(G) if Th0 is None else np.array(Th0, dtype=np.complex128)
    d = None
    for _ in range(iters):
        Vh = dft2(zero_pad(V, shape), half)
        d = dict_dstep(C, G, Vh, Th, rho_d)
        V = dict_vstep(d, Th, filt, shape, half)
        Th = Th + d - dft2(zero_pad(V, shape), half)
        if trace is not None:
            trace.append((d.copy(), V.copy(), Th.copy()))
    return d, V, Th


def dict_update_group(members: list, iters: int, filt, half: bool = True):
    """DictOCSC over several grid sizes that share one dictionary.

    ``members`` is a list of (G, C, rho_d, shape), one per grid size, each with
    its own history.  Every iteration runs each size's D-step, then one
    consensus V-step
        V = proj_ball( sum_s P_s alpha_s / sum_s P_s ),
        alpha_s = crop(Re F_s^-1(d_s + Theta_s)),
    and each size's dual step Theta_s += d_s - F_s(zero-pad V).  The P_s
    weights follow from rho_d = rho P per size: in the spatial domain each
    size's penalty is rho/2 ||zero-pad V - F_s^-1(d_s + Theta_s)||^2 times P_s.
    With one member this is ``dict_update``.  Returns ([d_s], V, [Theta_s]).
    """
    K = members[0][0].shape[0]
    V = np.zeros((K,) + tuple(filt))
    Ths = [np.zeros_like(G) for G, _, _, _ in members]
    ds = [None] * len(members)
    wsum = float(sum(sh[0] * sh[1] for _, _, _, sh in members))
    for _ in range(iters):
        acc = np.zeros_like(V)
        for i, (G, C, rho_d, shape) in enumerate(members):
            Vh = dft2(zero_pad(V, shape), half)
            ds[i] = dict_dstep(C, G, Vh, Ths[i], rho_d)
            acc += shape[0] * shape[1] * crop(idft2_real(ds[i] + Ths[i], shape, half), *filt)
        alpha = acc / wsum
        nrm = np.sqrt(np.sum(alpha * alpha, axis=(-2, -1)))
        V = alpha / np.maximum(nrm, 1.0)[:, None, None]
        for i, (G, C, rho_d, shape) in enumerate(members):
            Ths[i] = Ths[i] + ds[i] - dft2(zero_pad(V, shape), half)
    return ds, V, Ths


# --------------------------------------------------------------------------
# Objective (eq. csc) and online surrogate (Proposition 1)
# --------------------------------------------------------------------------

def objective(x: np.ndarray, U: np.ndarray, Dh: np.ndarray, lam: float,
              half: bool = True) -> float:
    """``1/2 ||x - sum_k F^-1(Dh_k * F U_k)||^2 + lam ||U||_1`` for one image."""
    shape = x.shape
    rec = idft2_real(np.sum(Dh * dft2(U, half), axis=0), shape, half)
    r = x - rec
    return 0.5 * float(np.sum(r * r)) + lam * float(np.sum(np.abs(U)))


def objective_terms(x: np.ndarray, U: np.ndarray, Dh: np.ndarray, half: bool = True):
    """The two terms of eq. csc separately: (1/2 ||x - reconstruction||^2, ||U||_1)."""
    shape = x.shape
    rec = idft2_real(np.sum(Dh * dft2(U, half), axis=0), shape, half)
    r = x - rec
    return 0.5 * float(np.sum(r * r)), float(np.sum(np.abs(U)))


def psnr(x: np.ndarray, rec: np.ndarray, peak: float = 255.0) -> float:
    """Peak signal-to-noise ratio of a reconstruction (section 4):
    ``10 log10(peak^2 P / ||rec - x||^2)``."""
    err = float(np.sum((rec - x) ** 2))
    return 10.0 * np.log10(peak * peak * x.size / err)


def dict_diagnostics(Dh: np.ndarray, V: np.ndarray, filt, shape, half: bool = True) -> dict:
    """Primal residual ``||F^-1(D~ - F zp V)||``, ``||F^-1 D~||`` over the padded
    grid, the norms of the V_k and of the exported filters crop(F^-1 D~_k)."""
    r = idft2_real(Dh - dft2(zero_pad(V, shape), half), shape, half)
    full = idft2_real(Dh, shape, half)
    D = crop(full, *filt)
    return {"primal_residual": float(np.sqrt(np.sum(r * r))),
            "dict_norm": float(np.sqrt(np.sum(full * full))),
            "V_norms": np.sqrt(np.sum(V * V, axis=(-2, -1))),
            "D_norms": np.sqrt(np.sum(D * D, axis=(-2, -1)))}


def surrogate(Dh: np.ndarray, H: np.ndarray, G: np.ndarray, sum_xh2: float,
              l1_sum: float, lam: float, shape, half: bool = True) -> float:
    """Online surrogate at dictionary spectrum Dh (Proposition 1, unnormalised).

    ``(1/2P) sum_p [d^H H_p d - 2 Re d^H G_p] + (1/2P) sum_i ||x_i||^2_F + lam sum_i ||U_i||_1``
    where ``sum_xh2`` is the Parseval-weighted sum of |x_i(p)|^2 over samples.
    """
    P = shape[0] * shape[1]
    wts = parseval_weights(shape, half)
    d = np.moveaxis(Dh, 0, -1)[..., None]                    # (..., K, 1)
    dH = np.swapaxes(np.conj(d), -1, -2)
    quad = np.real(dH @ H @ d)[..., 0, 0]
    lin = np.real(dH @ np.moveaxis(G, 0, -1)[..., None])[..., 0, 0]
    return float(np.sum(wts * (quad - 2.0 * lin))) / (2 * P) + sum_xh2 / (2 * P) + lam * l1_sum


# --------------------------------------------------------------------------
# Online convolutional sparse coding (Algorithm 3)
# --------------------------------------------------------------------------

class OCSC:
    """Online CSC learner, one minibatch at a time, following Algorithm 3.

    The calls mirror the C library: ``set_dictionary``, ``code_update``,
    ``history_accumulate``, ``dict_update``, ``get_dictionary``, ``objective``.
    A minibatch of B samples is coded against one dictionary, its B rank-one
    terms are folded into the history in index order, then one DictOCSC runs.
    """

    def __init__(self, K, filt_h, filt_w, pad_h, pad_w, lam, rho, rho_dict=None,
                 iters_code=10, iters_dict=10, half=True, keep_history=False, warm_start=False):
        if K < 1 or not (1 <= filt_h <= pad_h and 1 <= filt_w <= pad_w):
            raise ValueError("bad sizes")
        if lam < 0 or rho <= 0:
            raise ValueError("need lam >= 0 and rho > 0")
        self.K, self.filt = K, (filt_h, filt_w)
        self.shape = (pad_h, pad_w)
        self.P = pad_h * pad_w
        self.lam, self.rho = float(lam), float(rho)
        self.rho_d = float(rho_dict) if rho_dict and rho_dict > 0 else self.rho * self.P
        self.iters_code, self.iters_dict = iters_code, iters_dict
        self.half = half
        self.warm_start = warm_start
        wf = pad_w // 2 + 1 if half else pad_w
        fshape = (pad_h, wf)
        self.G = np.zeros((K,) + fshape, dtype=np.complex128)
        self.C = np.broadcast_to(np.eye(K) / self.rho_d, fshape + (K, K)).astype(np.complex128)
        self.H = np.zeros(fshape + (K, K), dtype=np.complex128) if keep_history else None
        self.Dh = np.zeros((K,) + fshape, dtype=np.complex128)
        self.V = np.zeros((K, filt_h, filt_w))
        self.Th = np.zeros_like(self.G)
        self.t = 0
        self.sum_xh2 = 0.0
        self.l1_sum = 0.0
        self._pending = None

    # dictionary in / out (Algorithm 3, initialisation and final loop)
    def set_dictionary(self, D: np.ndarray) -> None:
        self.Dh = dft2(zero_pad(np.asarray(D, np.float64), self.shape), self.half)

    def get_dictionary(self) -> np.ndarray:
        return crop(idft2_real(self.Dh, self.shape, self.half), *self.filt)

    def code_update(self, xs: np.ndarray) -> np.ndarray:
        """Code a minibatch (B, P_h, P_w) against the current dictionary."""
        xs = np.asarray(xs, np.float64)
        if xs.ndim == 2:
            xs = xs[None]
        Us, pend = [], []
        for x in xs:
            U, Zh, xh = code_update(x, self.Dh, self.lam, self.rho, self.iters_code, self.half)
            Us.append(U)
            pend.append((Zh, xh, float(np.sum(np.abs(U)))))
        self._pending = pend
        return np.stack(Us)

    def history_accumulate(self) -> None:
        if not self._pending:
            raise RuntimeError("history_accumulate needs the codes of a code_update")
        wts = parseval_weights(self.shape, self.half)
        for Zh, xh, l1 in self._pending:
            history_fold(self.G, self.C, Zh, xh, self.H)
            self.sum_xh2 += float(np.sum(wts * np.abs(xh) ** 2))
            self.l1_sum += l1
            self.t += 1
        self._pending = None

    def dict_update(self, trace: list | None = None) -> None:
        if self.t == 0:
            raise RuntimeError("dict_update needs at least one accumulated sample")
        warm = (self.V, self.Th) if self.warm_start else (None, None)
        d, V, Th = dict_update(self.G, self.C, self.rho_d, self.iters_dict, self.filt,
                               self.shape, self.half, trace, *warm)
        self.Dh, self.V, self.Th = d, V, Th

    def step(self, xs: np.ndarray) -> np.ndarray:
        """One body of Algorithm 3's loop for a minibatch; returns the codes."""
        U = self.code_update(xs)
        self.history_accumulate()
        self.dict_update()
        return U

    def objective(self, xs: np.ndarray, Us: np.ndarray) -> np.ndarray:
        xs = np.asarray(xs, np.float64)
        if xs.ndim == 2:
            xs, Us = xs[None], Us[None]
        return np.array([objective(x, U, self.Dh, self.lam, self.half) for x, U in zip(xs, Us)])

    @staticmethod
    def dict_update_group(models: list) -> None:
        """Consensus DictOCSC over learners on different grids (``dict_update_group``);
        each learner's dictionary becomes its last D-step iterate."""
        m0 = models[0]
        members = [(m.G, m.C, m.rho_d, m.shape) for m in models]
        ds, V, Ths = dict_update_group(members, m0.iters_dict, m0.filt, m0.half)
        for m, d, Th in zip(models, ds, Ths):
            m.Dh, m.V, m.Th = d, V.copy(), Th

    def objective_terms(self, xs: np.ndarray, Us: np.ndarray) -> list:
        xs = np.asarray(xs, np.float64)
        if xs.ndim == 2:
            xs, Us = xs[None], Us[None]
        return [objective_terms(x, U, self.Dh, self.half) for x, U in zip(xs, Us)]

    def diagnostics(self) -> dict:
        return dict_diagnostics(self.Dh, self.V, self.filt, self.shape, self.half)

    def surrogate_at(self, Dh: np.ndarray) -> float:
        if self.H is None:
            raise RuntimeError("surrogate needs keep_history=True")
        return surrogate(Dh, self.H, self.G, self.sum_xh2, self.l1_sum, self.lam,
                         self.shape, self.half)
