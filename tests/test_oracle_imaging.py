"""Pins for the oracle's bilinear gridding and imaging (CPU only).

Pinned by the conservation of the gridded weight, the Hermitian symmetry of
the grid, a visibility at a cell centre, the direct Fourier sum the FFT form
must equal, and the image of a point source peaking at its pixel.
"""
import numpy as np
import pytest

import oracle

C = oracle.C_LIGHT


def _vis(rng, B, P, Na, W_max=10):
    nbl = Na * (Na + 1) // 2
    V = rng.standard_normal((B, P, nbl, 2, 2, 2)).astype(np.float32)
    W = rng.integers(0, W_max, size=(B, nbl)).astype(np.int32)
    return V, W


def test_weight_is_conserved_and_grid_hermitian():
    rng = np.random.default_rng(1)
    B, P, Na, N, du = 2, 3, 9, 64, 0.5
    V, W = _vis(rng, B, P, Na)
    pos = rng.uniform(-20, 20, size=(Na, 2))
    freq = 60e6 + 2e5 * rng.random((B, P))
    G, norm = oracle.grid_visibilities(V, W, pos, freq, N, du)
    # each gridded visibility deposits w I and w conj(I): sum = 2 w Re(I)
    a, c = np.tril_indices(Na)
    blx = np.flatnonzero(a != c)
    total = 0.0
    for b in range(B):
        for k in range(P):
            I = 0.5 * (V[b, k, blx, 0, 0, 0].astype(np.float64) + V[b, k, blx, 1, 1, 0])
            total += (2.0 * W[b, blx] * I).sum()
    np.testing.assert_allclose(G.sum().real, total, rtol=1e-10)
    assert abs(G.sum().imag) < 1e-9 * np.abs(G).sum()
    np.testing.assert_allclose(norm, 2.0 * P * sum(W[b, blx].sum() for b in range(B)))
    Gm = np.conj(G[::-1, ::-1])                      # G[N-1-q][N-1-p]
    np.testing.assert_allclose(G[1:, 1:], np.roll(np.roll(Gm, 1, 0), 1, 1)[1:, 1:], atol=1e-12)
    assert np.all(G[0, :] == 0) and np.all(G[:, 0] == 0)


def test_visibility_at_a_cell_centre():
    N, du, nu = 32, 0.5, 60e6
    pos = np.array([[0.0, 0.0], [7 * du * C / nu, -3 * du * C / nu]])
    V = np.zeros((1, 1, 3, 2, 2, 2), np.float32)
    V[0, 0, 1, 0, 0] = [2.0, 1.0]
    V[0, 0, 1, 1, 1] = [4.0, 3.0]
    G, norm = oracle.grid_visibilities(V, None, pos, np.array([[nu]]), N, du)
    # baseline (1, 0): u = x_1 - x_0 = 7 cells, v = -3 cells, I = 3 + 2i
    np.testing.assert_allclose(G[N // 2 - 3, N // 2 + 7], 3 + 2j, atol=1e-9)
    np.testing.assert_allclose(G[N // 2 + 3, N // 2 - 7], 3 - 2j, atol=1e-9)
    assert np.abs(G).sum() == pytest.approx(2 * np.sqrt(13), rel=1e-9)
    assert norm == 2.0


def test_image_equals_the_direct_fourier_sum():
    rng = np.random.default_rng(2)
    N = 16
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    img = oracle.image_from_grid(G, 3.0)
    k = np.arange(N) - N // 2
    E = np.exp(-2j * np.pi * np.outer(k, k) / N)          # [pixel][cell]
    direct = (E @ G @ E.T).real / 3.0                      # sum_q sum_p E[j,q] G[q,p] E[i,p]
    np.testing.assert_allclose(img, direct, atol=1e-10 * np.abs(direct).max())


def test_point_source_images_at_its_pixel():
    rng = np.random.default_rng(3)
    Na, N, du = 24, 64, 0.5
    pos = rng.uniform(-25, 25, size=(Na, 2))
    freq = np.array([[58e6, 60e6, 62e6]])
    i0, j0 = 40, 21
    l0, m0 = (i0 - N // 2) / (N * du), (j0 - N // 2) / (N * du)
    a, c = np.tril_indices(Na)
    nbl = a.size
    V = np.zeros((1, 3, nbl, 2, 2, 2), np.float32)
    for k in range(3):
        u = (pos[a, 0] - pos[c, 0]) * freq[0, k] / C
        v = (pos[a, 1] - pos[c, 1]) * freq[0, k] / C
        vis = np.exp(2j * np.pi * (u * l0 + v * m0))
        for pol in (0, 1):
            V[0, k, :, pol, pol, 0] = vis.real
            V[0, k, :, pol, pol, 1] = vis.imag
    G, norm = oracle.grid_visibilities(V, None, pos, freq, N, du)
    img = oracle.image_from_grid(G, norm)
    jj, ii = np.unravel_index(np.argmax(img), img.shape)
    assert (ii, jj) == (i0, j0)
    assert 0.5 < img[j0, i0] <= 1.0 + 1e-9
    # the grid is Hermitian, so the complex transform is real
    s = (-1.0) ** np.add.outer(np.arange(N), np.arange(N))
    F = np.fft.fft2(G * s)
    assert np.abs(F.imag).max() < 1e-9 * np.abs(F.real).max()
