"""HIP odd-length batched DFT (K1) and per-mode real circulants against
numpy / the oracle's explicit DFT matrices."""
import numpy as np
import pytest

import paper_1902_07455_amd as P
from oracle import brute

pytestmark = pytest.mark.gpu

LENGTHS = [1, 3, 5, 7, 9, 11, 13, 15, 25, 27, 45, 49, 81, 121, 125, 135, 243, 401, 405, 625, 675, 729]


# the largest lengths only with few lines, to keep the test short
FFT_CASES = [(N, o, i) for N in LENGTHS for (o, i) in [(1, 1), (3, 1), (2, 37), (5, 16), (1, 100), (2, 13)]
             if N < 401 or o * i <= 40]


@pytest.mark.parametrize("N,outer,inner", FFT_CASES)
def test_fft_lines_matches_numpy(dev, N, outer, inner):
    import torch
    rng = np.random.default_rng(N * 1000 + outer * 10 + inner)
    x = rng.standard_normal((outer, N, inner)) + 1j * rng.standard_normal((outer, N, inner))
    t = torch.from_numpy(x.copy()).to(dev)
    P.fft_lines(t, outer, N, inner, -1)
    torch.cuda.synchronize()
    ref = np.fft.fft(x, axis=1) / N
    got = t.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.log2(N)) * np.max(np.abs(ref)) * 10
    P.fft_lines(t, outer, N, inner, +1)
    torch.cuda.synchronize()
    back = t.cpu().numpy()
    assert np.max(np.abs(back - x)) <= 1e-13 * np.max(np.abs(x)) * max(1.0, np.log2(N))


@pytest.mark.parametrize("N", [3, 9, 15, 45, 135, 13, 243])
@pytest.mark.parametrize("outer,inner", [(1, 1), (4, 7), (20, 20)])
def test_mode_derivative_matches_dense_dft(dev, N, outer, inner):
    """Spectral derivative on nodal values (eq. grad_trig) against the
    oracle's explicit DFT-matrix derivative."""
    import torch
    rng = np.random.default_rng(7 + N)
    x = rng.standard_normal((outer, N, inner))
    t = torch.from_numpy(x.copy()).to(dev)
    P.mode_op(t, outer, N, inner, 0)
    torch.cuda.synchronize()
    D = brute.derivative_matrix_1d(N)
    ref = np.einsum("mn,anb->amb", D, x)
    assert np.max(np.abs(t.cpu().numpy() - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("N,tpar", [(15, 0.01), (135, 0.001), (243, 0.0005), (45, 1.3)])
def test_mode_heat_kernel(dev, N, tpar):
    import torch
    rng = np.random.default_rng(3)
    outer, inner = 6, 11
    x = rng.standard_normal((outer, N, inner))
    t = torch.from_numpy(x.copy()).to(dev)
    P.mode_op(t, outer, N, inner, 1, tpar)
    torch.cuda.synchronize()
    k = np.fft.fftfreq(N, 1.0 / N).round()
    ref = np.fft.ifft(np.exp(-tpar * k ** 2)[None, :, None] * np.fft.fft(x, axis=1), axis=1).real
    assert np.max(np.abs(t.cpu().numpy() - ref)) <= 1e-13 * max(1.0, np.max(np.abs(x)))


@pytest.mark.parametrize("N,K", [(29, 7), (45, 11), (17, 0), (89, 22), (243, 60)])
def test_mode_low_pass(dev, N, K):
    """op 2: the projection of each fibre onto the trigonometric polynomials
    of degree K (frequencies |k| <= K kept, the rest zeroed)."""
    import torch
    rng = np.random.default_rng(11 + N)
    outer, inner = 5, 7
    x = rng.standard_normal((outer, N, inner))
    t = torch.from_numpy(x.copy()).to(dev)
    P.mode_op(t, outer, N, inner, 2, K)
    torch.cuda.synchronize()
    X = np.fft.fft(x, axis=1)
    k = np.fft.fftfreq(N, d=1.0 / N)
    X[:, np.abs(k) > K, :] = 0.0
    ref = np.fft.ifft(X, axis=1).real
    assert np.max(np.abs(t.cpu().numpy() - ref)) <= 1e-13 * max(1.0, np.max(np.abs(x))) * np.log2(N + 1)
