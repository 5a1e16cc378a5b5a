"""Checked (debug) mode: non-finite floating-point inputs are refused with
an error naming the input; finite inputs give the unchecked results; the
count itself is exact; with the mode off nothing is checked."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


@pytest.fixture
def checked(afc):
    afc.set_checked_mode(True)
    try:
        yield
    finally:
        afc.set_checked_mode(False)


def test_count_is_exact(afc, dev):
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    for dt in (torch.float32, torch.float16, torch.float64):
        t = torch.randn(1_000_003, generator=g, device=dev).to(dt)
        assert afc.count_nonfinite(t) == 0
        idx = torch.randperm(t.numel(), generator=g, device=dev)[:777]
        t[idx[:300]] = float("nan")
        t[idx[300:500]] = float("inf")
        t[idx[500:]] = float("-inf")
        assert afc.count_nonfinite(t) == 777
    big = torch.full((70000,), 65504.0, dtype=torch.float16, device=dev)      # largest finite fp16
    assert afc.count_nonfinite(big) == 0


def test_counts_from_two_threads(afc, dev):
    """Two host threads count different buffers on streams of their own at
    the same time (the count uses one device counter per GPU): every count is
    its own buffer's."""
    import threading
    a = torch.zeros(1 << 22, device=dev)
    a[::1000] = float("nan")
    b = torch.zeros(1 << 22, dtype=torch.float16, device=dev)
    b[::777] = float("inf")
    want = {0: -(-(1 << 22) // 1000), 1: -(-(1 << 22) // 777)}
    torch.cuda.synchronize()
    wrong = []

    def run(k, t):
        s = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(s):
            for _ in range(40):
                got = afc.count_nonfinite(t)
                if got != want[k]:
                    wrong.append((k, got))

    ths = [threading.Thread(target=run, args=(0, a)), threading.Thread(target=run, args=(1, b))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not wrong, wrong[:5]


def test_checked_calls_refuse_non_finite_inputs(afc, dev, checked):
    assert afc.checked_mode()
    taps = torch.from_numpy(W.prototype_taps()).to(dev)
    cfg = W.Config("chk", 8, 1, n_spectra=64, sigma_n=30.0, seed=2)
    x = W.make_voltages(cfg, device=dev)
    z = afc.channelise(x, taps, 64, "f16")                     # finite: runs
    vis, _ = afc.correlate(z, n_spectra=64)
    bad = taps.clone()
    bad[17] = float("nan")
    with pytest.raises(afc.AfcError, match="non-finite values in taps"):
        afc.channelise(x, bad, 64, "f32")
    z[0, 3, 1, 5, 2, 0] = float("inf")
    with pytest.raises(afc.AfcError, match="1 non-finite values in z"):
        afc.correlate(z, n_spectra=64)
    Vc, Mc, gc = (torch.from_numpy(a).to(dev) for a in W.make_calibration(Na=12, P=2, seed=4))
    loss, grad = afc.calibrate_grad(Vc, Mc, gc)
    Vb = Vc.clone()
    Vb[1, 7, 0, 0, 1] = float("-inf")
    with pytest.raises(afc.AfcError, match="non-finite values in V"):
        afc.calibrate_grad(Vb, Mc, gc)
    gb = gc.clone()
    gb[0, 3, 1, 0] = float("nan")
    with pytest.raises(afc.AfcError, match="non-finite values in g"):
        afc.calibrate_solve(Vc, Mc, gb, 3)
    afc.set_checked_mode(False)
    loss2, grad2 = afc.calibrate_grad(Vc, Mc, gc)
    assert torch.equal(loss, loss2) and torch.equal(grad, grad2)
    vis2, _ = afc.correlate(z, n_spectra=64)                   # unchecked: the Inf propagates
    torch.cuda.synchronize()
    assert not torch.isfinite(vis2).all()
    assert torch.isfinite(vis).all()
