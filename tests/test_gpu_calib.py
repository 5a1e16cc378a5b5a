"""GPU parity of the calibration loss and adjoint (afc_calibrate_grad, CalLoss)."""
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


def _check(afc, dev, V, M, g, chans=None, tol_g=1e-6, tol_l=1e-5):
    Vt, Mt, gt = (torch.from_numpy(a).to(dev) for a in (V, M, g))
    loss, grad = afc.calibrate_grad(Vt, Mt, gt)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    grad = _cplx(grad.cpu().numpy())
    chans = range(g.shape[0]) if chans is None else list(chans)
    sel = np.array(chans)
    lref, gref = oracle.cal_loss_grad(V[sel], M[sel], g[sel])
    worst_g = worst_l = 0.0
    for k, ch in enumerate(chans):
        for pol in range(2):
            rl = abs(loss[ch, pol] - lref[k, pol]) / abs(lref[k, pol])
            gn = np.linalg.norm(gref[k, :, pol])
            rg = np.linalg.norm(grad[ch, :, pol] - gref[k, :, pol]) / gn if gn > 0 else 0.0
            worst_g, worst_l = max(worst_g, rg), max(worst_l, rl)
    log(f"  loss rel err {worst_l:.2e}, grad rel err {worst_g:.2e}")
    assert worst_l <= tol_l
    assert worst_g <= tol_g


def test_small_random(afc, dev):
    rng = np.random.default_rng(1)
    Na, P = 70, 3                       # 70 antennas: ragged against the 64-antenna tiles
    nbl = Na * (Na + 1) // 2
    V = rng.standard_normal((P, nbl, 2, 2, 2)).astype(np.float32)
    M = rng.standard_normal((P, nbl, 2, 2, 2)).astype(np.float32)
    d = np.array([a * (a + 1) // 2 + a for a in range(Na)])
    for arr in (V, M):
        arr[:, d, 0, 0, 1] = 0
        arr[:, d, 1, 1, 1] = 0
    g = rng.standard_normal((P, Na, 2, 2)).astype(np.float32)
    _check(afc, dev, V, M, g)


@pytest.mark.parametrize("at", ["true", "unit"])
def test_grad_small(afc, dev, at):
    V, M, g = W.make_calibration(Na=48, P=4, seed=15)
    if at == "unit":
        g = np.zeros_like(g)
        g[..., 0] = 1.0
    _check(afc, dev, V, M, g)


@pytest.mark.parametrize("at", ["true", "unit"])
def test_grad_full_size(afc, dev, at):
    """576 antennas x 64 channels at SNR 20, at the true gains (residual ~ 5% of V) and at g = 1."""
    log(f"calibration full size at {at}")
    V, M, g = W.make_calibration(Na=576, P=64, seed=5)
    if at == "unit":
        g = np.zeros_like(g)
        g[..., 0] = 1.0
    _check(afc, dev, V, M, g, chans=[0, 17, 40, 63])


def test_autograd_matches_torch(afc, dev):
    """CalLoss backward equals torch autograd of the same loss in float64."""
    V, M, g = W.make_calibration(Na=24, P=2, seed=21)
    Vt, Mt = torch.from_numpy(V).to(dev), torch.from_numpy(M).to(dev)
    gc = torch.view_as_complex(torch.from_numpy(g).to(dev)).clone().requires_grad_(True)
    L = afc.cal_loss(Vt, Mt, gc)
    w = torch.tensor([[1.0, 0.5], [2.0, -1.0]], dtype=torch.float64, device=dev)
    (L * w).sum().backward()
    # reference: full Hermitian matrices in float64 on the CPU
    Na = 24
    a, b = np.tril_indices(Na)
    ref_grad = np.zeros((2, Na, 2), np.complex128)
    for k in range(2):
        for pol in range(2):
            Vf = np.zeros((Na, Na), np.complex128)
            Mf = np.zeros((Na, Na), np.complex128)
            Vf[a, b] = _cplx(V[k, :, pol, pol])
            Vf[b, a] = np.conj(Vf[a, b])
            Mf[a, b] = _cplx(M[k, :, pol, pol])
            Mf[b, a] = np.conj(Mf[a, b])
            gt = torch.tensor(_cplx(g[k, :, pol]), requires_grad=True)
            R = torch.tensor(Vf) - gt[:, None] * torch.tensor(Mf) * gt.conj()[None, :]
            ((R.abs() ** 2).sum() * float(w[k, pol])).backward()
            ref_grad[k, :, pol] = gt.grad.numpy()
    got = gc.grad.cpu().numpy()
    rel = np.linalg.norm(got - ref_grad) / np.linalg.norm(ref_grad)
    assert rel <= 1e-6


def test_grad_unaligned_records_match_aligned(afc, dev):
    """V and M at an 8-byte (not 16-byte) offset take the 8-byte-load path;
    it gives bit-identical loss and gradient to the 16-byte record path, and
    both pass the oracle check."""
    V, M, g = W.make_calibration(Na=70, P=3, seed=21)
    Vt, Mt, gt = (torch.from_numpy(a).to(dev) for a in (V, M, g))

    def shifted(t):
        buf = torch.empty(t.numel() + 2, dtype=t.dtype, device=dev)
        u = buf[2:].view(t.shape)
        u.copy_(t)
        assert u.data_ptr() % 16 == 8
        return u

    la, ga = afc.calibrate_grad(Vt, Mt, gt)
    lu, gu = afc.calibrate_grad(shifted(Vt), shifted(Mt), gt)
    torch.cuda.synchronize()
    assert Vt.data_ptr() % 16 == 0 and Mt.data_ptr() % 16 == 0
    assert torch.equal(la, lu) and torch.equal(ga, gu)
    _check(afc, dev, V, M, g)


def _weights_case(rng, P, nbl, frac=0.2):
    flags = (rng.random((P, nbl, 2)) < frac).astype(np.uint8)
    wts = rng.uniform(0.25, 2.0, (P, nbl, 2)).astype(np.float32)
    return flags, wts


@pytest.mark.parametrize("Na,P,chans", [(70, 3, None), (576, 64, [0, 21, 63])])
def test_weighted_grad_matches_oracle(afc, dev, Na, P, chans):
    """Flags (weight 0) and lost-data weights: the weighted loss and gradient
    against the oracle's weighted sums (same tolerances as unweighted)."""
    log(f"weighted calibration Na={Na} P={P}")
    V, M, g = W.make_calibration(Na=Na, P=P, seed=Na + 3)
    nbl = Na * (Na + 1) // 2
    flags, wts = _weights_case(np.random.default_rng(Na), P, nbl)
    Vt, Mt, gt = (torch.from_numpy(a).to(dev) for a in (V, M, g))
    loss, grad = afc.calibrate_grad(Vt, Mt, gt, flags=torch.from_numpy(flags).to(dev),
                                    weights=torch.from_numpy(wts).to(dev))
    torch.cuda.synchronize()
    loss, grad = loss.cpu().numpy(), _cplx(grad.cpu().numpy())
    chans = list(range(P)) if chans is None else chans
    w = oracle.cal_weights(P, nbl, flags=flags, weights=wts)
    lref, gref = oracle.cal_loss_grad(V[chans], M[chans], g[chans], weights=w[chans])
    worst_l = worst_g = 0.0
    for k, ch in enumerate(chans):
        for pol in range(2):
            worst_l = max(worst_l, abs(loss[ch, pol] - lref[k, pol]) / abs(lref[k, pol]))
            gn = np.linalg.norm(gref[k, :, pol])
            worst_g = max(worst_g, np.linalg.norm(grad[ch, :, pol] - gref[k, :, pol]) / gn)
    log(f"  loss rel err {worst_l:.2e}, grad rel err {worst_g:.2e}")
    assert worst_l <= 1e-5 and worst_g <= 1e-6


def test_weighted_unit_weights_bit_identical(afc, dev):
    """Weights of 1 and no flags give the unweighted call's bits."""
    V, M, g = W.make_calibration(Na=40, P=4, seed=8)
    Vt, Mt, gt = (torch.from_numpy(a).to(dev) for a in (V, M, g))
    nbl = 40 * 41 // 2
    l0, g0 = afc.calibrate_grad(Vt, Mt, gt)
    l1, g1 = afc.calibrate_grad(Vt, Mt, gt, weights=torch.ones((4, nbl, 2), dtype=torch.float32, device=dev))
    l2, g2 = afc.calibrate_grad(Vt, Mt, gt, flags=torch.zeros((4, nbl, 2), dtype=torch.uint8, device=dev))
    torch.cuda.synchronize()
    assert torch.equal(l0, l1) and torch.equal(g0, g1)
    assert torch.equal(l0, l2) and torch.equal(g0, g2)


def test_weighted_autograd_matches_torch(afc, dev):
    """cal_loss with flags and weights: backward equals torch autograd of
    sum w_ab |R_ab|^2 in float64 on the CPU."""
    Na, P = 20, 2
    V, M, g = W.make_calibration(Na=Na, P=P, seed=27)
    nbl = Na * (Na + 1) // 2
    flags, wts = _weights_case(np.random.default_rng(28), P, nbl)
    Vt, Mt = torch.from_numpy(V).to(dev), torch.from_numpy(M).to(dev)
    gc = torch.view_as_complex(torch.from_numpy(g).to(dev)).clone().requires_grad_(True)
    L = afc.cal_loss(Vt, Mt, gc, flags=torch.from_numpy(flags).to(dev), weights=torch.from_numpy(wts).to(dev))
    L.sum().backward()
    a, b = np.tril_indices(Na)
    wfull = oracle.cal_weights(P, nbl, flags=flags, weights=wts)
    ref_grad = np.zeros((P, Na, 2), np.complex128)
    ref_loss = np.zeros((P, 2))
    for k in range(P):
        for pol in range(2):
            Vf = np.zeros((Na, Na), np.complex128)
            Mf = np.zeros((Na, Na), np.complex128)
            Wf = np.zeros((Na, Na))
            Vf[a, b] = _cplx(V[k, :, pol, pol]); Vf[b, a] = np.conj(Vf[a, b])
            Mf[a, b] = _cplx(M[k, :, pol, pol]); Mf[b, a] = np.conj(Mf[a, b])
            Wf[a, b] = wfull[k, :, pol]; Wf[b, a] = wfull[k, :, pol]
            gt = torch.tensor(_cplx(g[k, :, pol]), requires_grad=True)
            R = torch.tensor(Vf) - gt[:, None] * torch.tensor(Mf) * gt.conj()[None, :]
            lk = (torch.tensor(Wf) * R.abs() ** 2).sum()
            lk.backward()
            ref_grad[k, :, pol] = gt.grad.numpy()
            ref_loss[k, pol] = float(lk.detach())
    np.testing.assert_allclose(L.detach().cpu().numpy(), ref_loss, rtol=1e-5)
    got = gc.grad.cpu().numpy()
    assert np.linalg.norm(got - ref_grad) / np.linalg.norm(ref_grad) <= 1e-6
