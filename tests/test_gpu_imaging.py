"""GPU parity of gridding and imaging (afc_grid_visibilities,
afc_image_from_grid) against the CPU oracle.

Grid: float32 output of float64 sums (fixed-point accumulation, bitwise
reproducible) against the float64 oracle: <= 1e-6 of the largest cell; the
normalisation exactly.  Image: float32 FFT, <= 1e-5 of the image peak.  At
the AARTFAAC-12 size (576 antennas, 8 subbands, 2048^2 grid): sampled cells
summed one by one from all contributing visibilities, sampled pixels by the
direct Fourier sum of the grid, and point sources imaged at their pixels."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

C = oracle.C_LIGHT


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def _freqs(B):
    return np.array([[W.subband_frequency(b) + W.channel_offset(k, 64) * W.F_SUBBAND / 64 for k in range(64)]
                     for b in range(B)])


def _cg(grid):
    g = grid.cpu().numpy()
    return g[..., 0].astype(np.float64) + 1j * g[..., 1]


@pytest.mark.parametrize("Na,B,N,du,weighted", [(24, 2, 64, 0.5, True), (9, 1, 32, 0.25, False),
                                                (40, 3, 256, 1.0, True)])
def test_grid_and_image_match_oracle(afc, dev, Na, B, N, du, weighted):
    rng = np.random.default_rng(Na * 7 + B)
    nbl = Na * (Na + 1) // 2
    V = rng.standard_normal((B, 64, nbl, 2, 2, 2)).astype(np.float32)
    Wt = rng.integers(0, 5, size=(B, nbl)).astype(np.int32) if weighted else None
    pos = rng.uniform(-25, 25, size=(Na, 2))
    freq = _freqs(B)
    log(f"grid Na={Na} B={B} N={N} du={du}")
    im = afc.Imager(torch.from_numpy(pos).to(dev), B, N, du)
    vt = torch.from_numpy(V).to(dev)
    ft = torch.from_numpy(freq).to(dev)
    wt = None if Wt is None else torch.from_numpy(Wt).to(dev)
    grid = im.grid(vt, ft, wt)
    img = im.image(grid).cpu().numpy()
    G, norm = oracle.grid_visibilities(V, Wt, pos, freq, N, du)
    g = _cg(grid)
    assert im.norm.item() == norm
    err = np.abs(g - G).max() / np.abs(G).max()
    log(f"  grid max err {err:.2e} (relative to the largest cell), norm {norm}")
    assert err <= 1e-6
    ref = oracle.image_from_grid(G, norm)
    ierr = np.abs(img - ref).max() / np.abs(ref).max()
    log(f"  image max err {ierr:.2e}")
    assert ierr <= 1e-5
    # bitwise reproducible
    again = im.grid(vt, ft, wt)
    assert torch.equal(again, grid)


def _point_source_vis(pos_t, freq_t, srcs, dev):
    """V[b][k][bl][p][p] = sum_s flux exp(2 pi i nu/c (dx l + dy m)), a >= c."""
    Na = pos_t.shape[0]
    a, c = np.tril_indices(Na)
    dx = (pos_t[a, 0] - pos_t[c, 0])
    dy = (pos_t[a, 1] - pos_t[c, 1])
    B = freq_t.shape[0]
    V = torch.zeros((B, 64, a.size, 2, 2, 2), dtype=torch.float32, device=dev)
    for b in range(B):
        for k in range(64):
            nu = float(freq_t[b, k])
            re = torch.zeros(a.size, dtype=torch.float64, device=dev)
            im = torch.zeros_like(re)
            for flux, l0, m0 in srcs:
                ph = 2.0 * np.pi * nu / C * (dx * l0 + dy * m0)
                re += flux * torch.cos(ph)
                im += flux * torch.sin(ph)
            for p in range(2):
                V[b, k, :, p, p, 0] = re.float()
                V[b, k, :, p, p, 1] = im.float()
    return V


def test_point_sources_image_at_their_pixels(afc, dev):
    Na, B, N, du = 48, 2, 256, 0.5
    cfg = W.Config("img", Na, B, layout="disc", seed=3)
    pos = W.antenna_positions(cfg)
    post = torch.from_numpy(pos).to(dev)
    freq = _freqs(B)
    pix = [(150, 90, 5.0), (60, 200, 2.0)]
    srcs = [(f, (i - N // 2) / (N * du), (j - N // 2) / (N * du)) for i, j, f in pix]
    V = _point_source_vis(post, torch.from_numpy(freq).to(dev), srcs, dev)
    im = afc.Imager(post, B, N, du)
    img = im.image(im.grid(V, torch.from_numpy(freq).to(dev))).cpu().numpy()
    for i, j, f in pix:
        win = img[j - 2:j + 3, i - 2:i + 3]
        jj, ii = np.unravel_index(np.argmax(win), win.shape)
        log(f"  source at ({i}, {j}) flux {f}: peak {win.max():.3f} at offset ({ii - 2}, {jj - 2})")
        assert (ii, jj) == (2, 2)
        assert 0.5 * f < win.max() < 1.2 * f


def test_full_size_aartfaac12(afc, dev):
    """576 antennas (12 stations), 8 subbands x 64 channels, 2048^2 grid,
    three point sources."""
    Na, B, N, du = 576, 8, 2048, 0.5
    cfg = W.A12
    pos = W.antenna_positions(cfg)
    post = torch.from_numpy(pos).to(dev)
    freq = _freqs(B)
    ft = torch.from_numpy(freq).to(dev)
    pix = [(1300, 700, 10.0), (900, 1500, 4.0), (1024, 1100, 2.0)]
    srcs = [(f, (i - N // 2) / (N * du), (j - N // 2) / (N * du)) for i, j, f in pix]
    V = _point_source_vis(post, ft, srcs, dev)
    im = afc.Imager(post, B, N, du)
    grid = im.grid(V, ft)
    img = im.image(grid).cpu().numpy()
    g = _cg(grid)
    norm = im.norm.item()
    # sampled cells against the sum of every contribution, one by one
    Vh = V.cpu().numpy()
    occ = np.argwhere(np.abs(g) > 0)
    rng = np.random.default_rng(0)
    cells = [tuple(occ[i]) for i in rng.choice(len(occ), size=12, replace=False)]
    cells.append(tuple(np.unravel_index(np.argmax(np.abs(g)), g.shape)))
    a, c = np.tril_indices(Na)
    cross = np.flatnonzero(a != c)
    dx, dy = pos[a[cross], 0] - pos[c[cross], 0], pos[a[cross], 1] - pos[c[cross], 1]
    T = np.sort(np.array([q * N + p for (q, p) in cells]))
    acc = np.zeros(T.size, np.complex128)
    for b in range(B):
        for k in range(64):
            nu = freq[b, k]
            pu = dx * nu / C / du + N / 2
            pv = dy * nu / C / du + N / 2
            i0, j0 = np.floor(pu).astype(np.int64), np.floor(pv).astype(np.int64)
            fu, fv = pu - i0, pv - j0
            I = 0.5 * ((Vh[b, k, cross, 0, 0, 0].astype(np.float64) + Vh[b, k, cross, 1, 1, 0])
                       + 1j * (Vh[b, k, cross, 0, 0, 1].astype(np.float64) + Vh[b, k, cross, 1, 1, 1]))
            for dj in (0, 1):
                for di in (0, 1):
                    wgt = (fu if di else 1 - fu) * (fv if dj else 1 - fv)
                    for idx, val in (((j0 + dj) * N + i0 + di, wgt * I),
                                     ((N - j0 - dj) * N + N - i0 - di, wgt * np.conj(I))):
                        hit = np.isin(idx, T)
                        if hit.any():
                            np.add.at(acc, np.searchsorted(T, idx[hit]), val[hit])
    gmax = np.abs(g).max()
    for n, t in enumerate(T):
        cell = (t // N, t % N)
        assert abs(g[cell] - acc[n]) <= 1e-6 * gmax, (cell, g[cell], acc[n])
    assert norm == 2.0 * cross.size * B * 64
    # sampled pixels: the direct Fourier sum of the device's grid
    qs, ps = np.nonzero(np.abs(g) > 0)
    vals = g[qs, ps]
    for (i, j) in [(1300, 700), (5, 2040), (1024, 1024), (333, 1777)]:
        ph = np.exp(-2j * np.pi * ((ps - N // 2) * (i - N // 2) + (qs - N // 2) * (j - N // 2)) / N)
        direct = (vals * ph).sum().real / norm
        assert abs(img[j, i] - direct) <= 1e-5 * np.abs(img).max(), ((i, j), img[j, i], direct)
    for i, j, f in pix:
        win = img[j - 2:j + 3, i - 2:i + 3]
        jj, ii = np.unravel_index(np.argmax(win), win.shape)
        log(f"  source ({i}, {j}) flux {f}: peak {win.max():.3f} at offset ({ii - 2}, {jj - 2})")
        assert (ii, jj) == (2, 2)
    del V, grid
    torch.cuda.empty_cache()
