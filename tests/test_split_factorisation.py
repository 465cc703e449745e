"""The factorisation behind the split plane step, checked on the CPU against
NumPy's FFT (no GPU, no library code).

The split plane step (launch shape two_pass = 2) runs each plane of the code
update (eq. fcsc_code) on F workgroups, one per row residue e (rows F m + e),
and moves the outer radix-F step of the column DFTs into the Z-step.  Its
kernels implement two identities of the DFT of length PH (decimation in time),
with w = e^{-2 pi i/PH} and PHS = PH/F:

* inverse: rows F m + e of the unnormalised inverse column DFT of Y are the
  unnormalised inverse DFTs of length PHS of
  conj(w^{h e}) sum_j Y[h + j PHS] e^{+2 pi i j e/F}, h < PHS;
* forward: X[h] = sum_e w^{h e} E_e[h mod PHS], E_e the DFTs of length PHS
  of rows F m + e.

A dropped twiddle, a wrong sign of the residue rotation or a transposed
residue index fails these checks; the GPU tests compare the kernels built on
them with the FP64 oracle.
"""
import numpy as np
import pytest


def inverse_slices(Y, F):
    """The F length-PHS spectra whose inverse DFTs are the rows of each residue."""
    PH = Y.shape[0]
    PHS = PH // F
    h = np.arange(PHS)
    w = np.exp(-2j * np.pi * np.arange(PH) / PH)
    out = []
    for e in range(F):
        inner = sum(Y[j * PHS:(j + 1) * PHS] * np.exp(2j * np.pi * j * e / F) for j in range(F))
        out.append(inner * np.conj(w[(h * e) % PH])[:, None])
    return out


def forward_combine(E, PH):
    F = len(E)
    PHS = PH // F
    w = np.exp(-2j * np.pi * np.arange(PH) / PH)
    return np.stack([sum(w[(h * e) % PH] * E[e][h % PHS] for e in range(F)) for h in range(PH)])


@pytest.mark.parametrize("PH,PW,F", [(32, 32, 2), (128, 128, 2), (256, 256, 2), (256, 512, 4), (512, 256, 4),
                                     (512, 512, 8), (512, 512, 16), (64, 32, 2)])
def test_row_residue_split_of_the_2d_real_dft(PH, PW, F):
    rng = np.random.default_rng(PH + PW + F)
    x = rng.standard_normal((PH, PW))
    X = np.fft.rfft2(x)                                   # (PH, PW/2 + 1)
    # inverse: each residue's rows from its own length-PHS spectrum
    for e, A in enumerate(inverse_slices(X, F)):
        rows = np.fft.irfft(np.fft.ifft(A, axis=0) * (PH // F), n=PW, axis=1) / PH
        assert np.allclose(rows, x[e::F], atol=1e-12)
    # forward: the column DFTs of each residue's rows, combined
    R = np.fft.rfft(x, axis=1)
    E = [np.fft.fft(R[e::F], axis=0) for e in range(F)]
    assert np.allclose(forward_combine(E, PH), X, atol=1e-9)


def test_a_wrong_residue_rotation_is_caught():
    """The checks above fail for the plausible slip of rotating by e^{-2 pi i j e/F}."""
    PH, PW, F = 64, 32, 4
    x = np.random.default_rng(1).standard_normal((PH, PW))
    X = np.fft.rfft2(x)
    PHS = PH // F
    w = np.exp(-2j * np.pi * np.arange(PH) / PH)
    e = 1
    inner = sum(X[j * PHS:(j + 1) * PHS] * np.exp(-2j * np.pi * j * e / F) for j in range(F))
    A = inner * np.conj(w[(np.arange(PHS) * e) % PH])[:, None]
    rows = np.fft.irfft(np.fft.ifft(A, axis=0) * PHS, n=PW, axis=1) / PH
    assert not np.allclose(rows, x[e::F], atol=1e-6)
