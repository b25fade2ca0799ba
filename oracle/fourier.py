"""Azimuthal Fourier decomposition (Sec. 2.2) -- oracle side (test
infrastructure only).

Reading of Eq. fourier_decomposition (its index range 1..N_phi is taken as
0..N_phi-1): the forward transform is normalised,

    rho^m_ij = (1/N_phi) sum_k rho_ijk exp(-2 pi i m k / N_phi),

the inverse is the unnormalised sum with exp(+2 pi i m k / N_phi), and only
m = 0..N_phi/2 are kept (Eq. Hermitian_symmetry).  Arrays in real space are
(n_a, n_b, n_phi) with phi fastest; mode arrays are (n_phi/2 + 1, n_a, n_b).
"""
import numpy as np


def forward(rho):
    """Modes m = 0..N/2 of a real (n_a, n_b, N) array (numpy FFT)."""
    n = rho.shape[-1]
    return np.moveaxis(np.fft.rfft(rho, axis=-1) / n, -1, 0)


def inverse(modes, n_phi):
    """Real (n_a, n_b, N) array from modes m = 0..N/2, completing the upper
    half by Hermitian symmetry (the imaginary parts of m = 0 and m = N/2 do
    not contribute)."""
    return np.fft.irfft(np.moveaxis(modes, 0, -1), n=n_phi, axis=-1) * n_phi


def forward_plain(x):
    """O(N^2) transcription of the forward sum for one real line (pins the
    FFT-based version on small N)."""
    n = len(x)
    out = np.zeros(n // 2 + 1, dtype=np.complex128)
    for m in range(n // 2 + 1):
        acc = 0.0 + 0.0j
        for k in range(n):
            acc += x[k] * np.exp(-2j * np.pi * m * k / n)
        out[m] = acc / n
    return out


def inverse_plain(modes, n):
    """O(N^2) Hermitian-completed inverse sum for one line."""
    full = np.zeros(n, dtype=np.complex128)
    half = n // 2
    full[: half + 1] = modes
    full[half] = modes[half].real
    full[0] = modes[0].real
    for m in range(1, half):
        full[n - m] = np.conj(modes[m])
    out = np.zeros(n)
    for k in range(n):
        acc = 0.0 + 0.0j
        for m in range(n):
            acc += full[m] * np.exp(2j * np.pi * m * k / n)
        out[k] = acc.real
    return out
