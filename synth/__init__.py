"""Seeded synthetic inputs for online convolutional sparse coding.

This module only draws inputs: ground-truth filters, sparse codes, images,
initial dictionaries and presentation orders.  It holds none of the coding or
dictionary-learning arithmetic, so both the FP64 oracle and the HIP library can
be fed from it without sharing any of the method's code.

Recipe (images are sums of filters convolved with Bernoulli-Gaussian codes plus
Gaussian noise, filters i.i.d. standard normal and normalised to the unit
ball, as in the paper's synthetic study, Appendix B.2):

* ground-truth filters: ``K_true`` x ``M_h`` x ``M_w`` i.i.d. N(0,1), each scaled
  to unit l2 norm;
* codes of one image: ``K_true`` x ``H_c`` x ``W_c``, Bernoulli(density) times
  N(0, sigma_z^2);
* image content: sum over k of the 'same'-cropped linear convolution of code k
  with filter k, plus N(0, noise^2) per pixel, placed at offset (0, 0) of a
  zero ``P_h`` x ``P_w`` grid;
* initial dictionary: ``K`` x ``M_h`` x ``M_w`` i.i.d. N(0,1), unit l2 norm per
  filter (the paper initialises with a Gaussian random matrix, Algorithm 3);
* pass q presents the images in a seeded random permutation.

Sub-seeds: base+0 ground-truth filters, base+1 codes and noise (one stream per
image index, so any image can be drawn on its own), base+2 initial dictionary,
base+3+q the order of pass q.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Iterable

import numpy as np
from scipy import signal as _signal

__all__ = [
    "Workload", "WORKLOADS", "truth_filters", "initial_dictionary", "image",
    "images", "pass_order", "code_sample",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and hyper-parameters of one synthetic OCSC workload."""
    name: str
    pad_h: int            # FFT grid rows (P_h)
    pad_w: int            # FFT grid columns (P_w)
    content_h: int        # image content rows (H_c), placed at (0, 0)
    content_w: int
    k_true: int           # ground-truth filters used to synthesise images
    density: float        # Bernoulli probability of a non-zero code
    sigma_z: float        # standard deviation of non-zero code amplitudes
    noise: float          # standard deviation of additive pixel noise
    K: int                # filters learned
    filt_h: int
    filt_w: int
    lam: float            # l1 weight (the paper's beta)
    rho: float            # code-ADMM penalty
    iters_code: int       # code-ADMM iterations per sample
    iters_dict: int       # dictionary-ADMM iterations per update
    batch: int            # samples coded against one dictionary
    n_images: int
    passes: int
    precision: str        # arithmetic of the GPU path: "f64" or "f32"
    seed: int = 0

    @property
    def P(self) -> int:
        return self.pad_h * self.pad_w


WORKLOADS: Dict[str, Workload] = {
    # 50 images of 54x54 on a 64x64 grid, 16 filters, FP64: the parity workload.
    "ocsc_64x64_k16_f64": Workload(
        name="ocsc_64x64_k16_f64", pad_h=64, pad_w=64, content_h=54, content_w=54,
        k_true=16, density=0.01, sigma_z=10.0, noise=0.01, K=16, filt_h=11,
        filt_w=11, lam=1.0, rho=1.0, iters_code=10, iters_dict=10, batch=1,
        n_images=50, passes=1, precision="f64"),
    # 10,000 images of 100x100 on a 128x128 grid, 100 filters, FP32 on the GPU:
    # the throughput workload (K=100 and 11x11 filters as in the paper's
    # experiments).
    "ocsc_128x128_k100_f32": Workload(
        name="ocsc_128x128_k100_f32", pad_h=128, pad_w=128, content_h=100,
        content_w=100, k_true=100, density=0.005, sigma_z=10.0, noise=0.01,
        K=100, filt_h=11, filt_w=11, lam=1.0, rho=1.0, iters_code=10,
        iters_dict=10, batch=1, n_images=10000, passes=2, precision="f32"),
}


def _rng(*words: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(words))))


def _unit_filters(rng: np.random.Generator, k: int, mh: int, mw: int) -> np.ndarray:
    f = rng.standard_normal((k, mh, mw))
    n = np.sqrt((f * f).sum(axis=(1, 2), keepdims=True))
    return f / n


def truth_filters(wl: Workload) -> np.ndarray:
    """Ground-truth filters, shape (K_true, M_h, M_w), unit l2 norm each."""
    return _unit_filters(_rng(wl.seed + 0), wl.k_true, wl.filt_h, wl.filt_w)


def initial_dictionary(K: int, filt_h: int, filt_w: int, seed: int = 0) -> np.ndarray:
    """Initial dictionary D_0, shape (K, M_h, M_w), unit l2 norm per filter."""
    return _unit_filters(_rng(seed + 2), K, filt_h, filt_w)


def code_sample(wl: Workload, index: int) -> np.ndarray:
    """Bernoulli-Gaussian codes of image ``index``, shape (K_true, H_c, W_c)."""
    rng = _rng(wl.seed + 1, index)
    shape = (wl.k_true, wl.content_h, wl.content_w)
    mask = rng.random(shape) < wl.density
    return np.where(mask, rng.standard_normal(shape) * wl.sigma_z, 0.0)


def image(wl: Workload, index: int, filters: np.ndarray | None = None) -> np.ndarray:
    """Image ``index`` on the zero-padded grid, shape (P_h, P_w), float64."""
    if filters is None:
        filters = truth_filters(wl)
    codes = code_sample(wl, index)
    rng = _rng(wl.seed + 1, index, 1)
    # 'same' linear convolution per ground-truth filter (library routine), summed.
    content = _signal.fftconvolve(codes, filters, mode="same", axes=(1, 2)).sum(axis=0)
    content = content + rng.standard_normal(content.shape) * wl.noise
    out = np.zeros((wl.pad_h, wl.pad_w))
    out[: wl.content_h, : wl.content_w] = content
    return out


def images(wl: Workload, indices: Iterable[int]) -> np.ndarray:
    """Stack of images, shape (len(indices), P_h, P_w), float64."""
    f = truth_filters(wl)
    idx = list(indices)
    out = np.empty((len(idx), wl.pad_h, wl.pad_w))
    for j, i in enumerate(idx):
        out[j] = image(wl, i, f)
    return out


def pass_order(n: int, seed: int, q: int) -> np.ndarray:
    """Presentation order of pass ``q`` over ``n`` images."""
    return _rng(seed + 3 + q).permutation(n)
