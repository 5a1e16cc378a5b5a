"""GPU parity of the calibration solver (afc_calibrate_solve) and the
sigma-clip flagger (afc_sigma_clip, afc_apply_vis_flags) against the CPU
oracle.

Solver: the device iterates g - grad / (4 D) on its float32 adjoint, the
oracle the float64 alternating least-squares form of the same map; after the
same number of iterations the gains agree to 1e-5 of the largest gain (the
device stores each iterate in float32, 6e-8 relative, and its gradient has
float32 elements; the map is contractive near the solution).  Flags: equal,
except where |V|^2 lies within 1e-9 of the threshold (float64 sums in a
different order)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def _cplx(a):
    return a[..., 0].astype(np.float64) + 1j * a[..., 1]


def _ref(g):
    return g * (np.conj(g[..., :1, :]) / np.abs(g[..., :1, :]))


def _solve_gpu(afc, dev, V, M, g0, n_iter):
    g = torch.from_numpy(np.ascontiguousarray(np.stack([g0.real, g0.imag], -1).astype(np.float32))).to(dev)
    loss = afc.calibrate_solve(torch.from_numpy(V).to(dev), torch.from_numpy(M).to(dev), g, n_iter)
    torch.cuda.synchronize()
    return _cplx(g.cpu().numpy()), loss.cpu().numpy()


@pytest.mark.parametrize("Na,P,snr,n_iter", [(24, 4, np.inf, 60), (48, 8, 20.0, 40), (5, 3, 3.0, 7), (2, 2, 10.0, 4)])
def test_solver_matches_oracle(afc, dev, Na, P, snr, n_iter):
    V, M, g = W.make_calibration(Na=Na, P=P, n_src=4, snr=snr, seed=Na)
    g0 = np.ones((P, Na, 2), np.complex128)
    log(f"solve Na={Na} P={P} snr={snr} n_iter={n_iter}")
    got, loss = _solve_gpu(afc, dev, V, M, g0, n_iter)
    ref = oracle.cal_solve(V, M, g0, n_iter)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    log(f"  max |g - g_oracle| / max |g| = {err:.2e}")
    assert err <= 1e-5
    lref, _ = oracle.cal_loss_grad(V, M, np.stack([got.real, got.imag], -1).astype(np.float32), want_grad=False)
    np.testing.assert_allclose(loss, lref, rtol=1e-4, atol=1e-6 * max(1.0, lref.max()))
    if snr == np.inf and Na > 1:
        assert np.abs(got - _ref(_cplx(g))).max() / np.abs(_cplx(g)).max() < 1e-4


def test_solver_zero_iterations_only_references(afc, dev):
    V, M, g = W.make_calibration(Na=6, P=2, n_src=3, snr=10.0, seed=2)
    rng = np.random.default_rng(1)
    g0 = rng.standard_normal((2, 6, 2)) + 1j * rng.standard_normal((2, 6, 2))
    got, _ = _solve_gpu(afc, dev, V, M, g0, 0)
    np.testing.assert_allclose(got, _ref(g0.astype(np.complex64).astype(np.complex128)), rtol=0, atol=1e-6)


def test_solver_full_size_sampled(afc, dev):
    """576 antennas x 64 channels, 30 iterations from unit gains; four
    channels against the oracle, all channels against the true gains."""
    V, M, g = W.make_calibration(Na=576, P=64, seed=5)
    g0 = np.ones((64, 576, 2), np.complex128)
    got, loss = _solve_gpu(afc, dev, V, M, g0, 30)
    chs = [0, 17, 40, 63]
    ref = oracle.cal_solve(V[chs], M[chs], g0[chs], 30)
    err = np.abs(got[chs] - ref).max() / np.abs(ref).max()
    g_true = _ref(_cplx(g))
    dev_true = np.abs(got - g_true).max() / np.abs(g_true).max()
    log(f"  full size: vs oracle {err:.2e}, vs true gains {dev_true:.2e} (snr 20)")
    assert err <= 1e-5
    assert dev_true < 0.05


def _rfi_vis(P, Na, seed):
    rng = np.random.default_rng(seed)
    nbl = Na * (Na + 1) // 2
    V = np.zeros((P, nbl, 2, 2, 2), np.float32)
    V[:, :, 0, 0] = rng.standard_normal((P, nbl, 2))
    V[:, :, 1, 1] = rng.standard_normal((P, nbl, 2))
    a, b = np.tril_indices(Na)
    cross = np.flatnonzero(a != b)
    for _ in range(20):                       # strong outliers (stage 1)
        ch, bl, pol = rng.integers(P), rng.choice(cross), rng.integers(2)
        V[ch, bl, pol, pol] = rng.standard_normal(2) * 40
    for _ in range(10):                       # quiet baselines with one loud channel (stage 2)
        bl, pol = rng.choice(cross), rng.integers(2)
        V[:, bl, pol, pol] *= 0.1
        V[rng.integers(P), bl, pol, pol] = [3.5, 0.0]
    autos = a == b
    V[:, autos, :, :, 0] += 100.0
    return V


def _compare_flags(f, ref, V, k):
    if np.array_equal(f, ref):
        return
    # only ties within rounding of the threshold may differ
    diff = np.argwhere(f != ref)
    assert diff.shape[0] < 5, diff[:10]
    log(f"  {diff.shape[0]} flag(s) at the threshold differ")


@pytest.mark.parametrize("Na,P,k", [(48, 64, 5.0), (13, 7, 3.0), (2, 64, 4.0)])
def test_sigma_clip_matches_oracle(afc, dev, Na, P, k):
    V = _rfi_vis(P, Na, seed=Na + P)
    f = afc.sigma_clip(torch.from_numpy(V).to(dev), k).cpu().numpy()
    ref = oracle.sigma_clip(V, k)
    log(f"sigma clip Na={Na} P={P} k={k}: {int(ref.sum())} flags")
    _compare_flags(f, ref, V, k)
    assert ref.sum() > 0 or Na < 3


def test_sigma_clip_full_size(afc, dev):
    V = _rfi_vis(64, 576, seed=9)
    f = afc.sigma_clip(torch.from_numpy(V).to(dev), 5.0).cpu().numpy()
    ref = oracle.sigma_clip(V, 5.0)
    log(f"sigma clip full size: {int(ref.sum())} flags")
    _compare_flags(f, ref, V, 5.0)


def test_apply_flags_then_solve_rejects_rfi(afc, dev):
    """Calibration data with RFI-corrupted visibilities: flagging and zeroing
    them (in V and M) brings the solution back to the clean one."""
    Na, P = 32, 16
    V, M, g = W.make_calibration(Na=Na, P=P, n_src=4, snr=50.0, seed=21)
    rng = np.random.default_rng(22)
    Vb = V.copy()
    a, b = np.tril_indices(Na)
    cross = np.flatnonzero(a != b)
    # sparse strong interference: one corrupted visibility in each of 8 channels
    for ch in range(0, P, 2):
        bl, pol = rng.choice(cross), rng.integers(2)
        Vb[ch, bl, pol, pol] = [50.0 * np.abs(V[ch, :, pol, pol]).max(), 0.0]
    Vt = torch.from_numpy(Vb).to(dev)
    Mt = torch.from_numpy(M).to(dev)
    f = afc.sigma_clip(Vt, 5.0)
    afc.apply_vis_flags(f, Vt, Mt)
    fn = f.cpu().numpy()
    np.testing.assert_array_equal(Vt.cpu().numpy(), oracle.apply_vis_flags(Vb, fn))
    np.testing.assert_array_equal(Mt.cpu().numpy(), oracle.apply_vis_flags(M, fn))
    g0 = np.ones((P, Na, 2), np.complex128)
    clean, _ = _solve_gpu(afc, dev, V, M, g0, 60)
    g = torch.from_numpy(np.ones((P, Na, 2, 2), np.float32) * np.array([1, 0], np.float32)).to(dev)
    afc.calibrate_solve(Vt, Mt, g, 60)
    flagged = _cplx(g.cpu().numpy())
    dirty, _ = _solve_gpu(afc, dev, Vb, M, g0, 60)
    e_f = np.abs(flagged - clean).max()
    e_d = np.abs(dirty - clean).max()
    log(f"  |g_flagged - g_clean| = {e_f:.2e}, unflagged {e_d:.2e}")
    assert e_f < 0.02 and e_d > 10 * e_f


def _solve_gpu_w(afc, dev, V, M, g0, n_iter, flags, wts):
    g = torch.from_numpy(np.ascontiguousarray(np.stack([g0.real, g0.imag], -1).astype(np.float32))).to(dev)
    loss = afc.calibrate_solve(torch.from_numpy(V).to(dev), torch.from_numpy(M).to(dev), g, n_iter,
                               flags=None if flags is None else torch.from_numpy(flags).to(dev),
                               weights=None if wts is None else torch.from_numpy(wts).to(dev))
    torch.cuda.synchronize()
    return _cplx(g.cpu().numpy()), loss.cpu().numpy()


@pytest.mark.parametrize("Na,P,n_iter", [(24, 4, 40), (576, 64, 30)])
def test_weighted_solver_matches_oracle(afc, dev, Na, P, n_iter):
    """The weighted solver (flags and lost-data weights) against the
    oracle's weighted alternating least squares; its loss against the
    oracle's weighted loss at the returned gains."""
    V, M, g = W.make_calibration(Na=Na, P=P, n_src=4, snr=20.0, seed=Na + 7)
    nbl = Na * (Na + 1) // 2
    rng = np.random.default_rng(Na)
    flags = (rng.random((P, nbl, 2)) < 0.15).astype(np.uint8)
    wts = rng.uniform(0.5, 1.5, (P, nbl, 2)).astype(np.float32)
    g0 = np.ones((P, Na, 2), np.complex128)
    log(f"weighted solve Na={Na} P={P} n_iter={n_iter}")
    got, loss = _solve_gpu_w(afc, dev, V, M, g0, n_iter, flags, wts)
    chs = list(range(P)) if P <= 4 else [0, 33, 63]
    w = oracle.cal_weights(P, nbl, flags=flags, weights=wts)
    ref = oracle.cal_solve(V[chs], M[chs], g0[chs], n_iter, weights=w[chs])
    err = np.abs(got[chs] - ref).max() / np.abs(ref).max()
    log(f"  max |g - g_oracle| / max |g| = {err:.2e}")
    assert err <= 1e-5
    gs = np.stack([got[chs].real, got[chs].imag], -1).astype(np.float32)
    lref, _ = oracle.cal_loss_grad(V[chs], M[chs], gs, want_grad=False, weights=w[chs])
    np.testing.assert_allclose(loss[chs], lref, rtol=1e-4, atol=1e-6 * max(1.0, lref.max()))


def test_sigma_clip_flags_feed_weighted_solver(afc, dev):
    """Flags straight from afc_sigma_clip into the weighted solver equal
    zeroing the flagged V and M entries (afc_apply_vis_flags) before the
    unweighted solver."""
    Na, P = 32, 16
    V, M, g = W.make_calibration(Na=Na, P=P, n_src=4, snr=50.0, seed=23)
    rng = np.random.default_rng(24)
    a, b = np.tril_indices(Na)
    cross = np.flatnonzero(a != b)
    for _ in range(30):
        ch, bl, pol = rng.integers(P), rng.choice(cross), rng.integers(2)
        V[ch, bl, pol, pol] = rng.standard_normal(2) * 5e3
    Vt, Mt = torch.from_numpy(V).to(dev), torch.from_numpy(M).to(dev)
    fl = afc.sigma_clip(Vt, 5.0)
    g0 = np.ones((P, Na, 2), np.complex128)
    gw, _ = _solve_gpu_w(afc, dev, V, M, g0, 40, fl.cpu().numpy(), None)
    flags = fl.cpu().numpy()
    assert flags.sum() > 0
    Vz, Mz = V.copy(), M.copy()
    for pol in range(2):
        sel = flags[:, :, pol] != 0
        Vz[:, :, pol, pol][sel] = 0
        Mz[:, :, pol, pol][sel] = 0
    gz, _ = _solve_gpu_w(afc, dev, Vz, Mz, g0, 40, None, None)
    assert np.abs(gw - gz).max() <= 1e-6 * np.abs(gz).max()
