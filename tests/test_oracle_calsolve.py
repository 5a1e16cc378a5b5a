"""Pins for the oracle's calibration solver and sigma-clip flagger (CPU only).

The solver is pinned by convergence to the true gains on noise-free data,
by the identity that ties its update to the gradient of the loss (the
oracle's own adjoint, written independently), by the fixed point and by the
phase gauge; the flagger by planted outliers with known outcomes.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _ref(g):
    """Remove the common phase: g_0 real and positive."""
    return g * (np.conj(g[..., :1, :]) / np.abs(g[..., :1, :]))


def _cplx(a):
    return a[..., 0].astype(np.float64) + 1j * a[..., 1]


def test_noise_free_converges_to_true_gains():
    V, M, g = W.make_calibration(Na=12, P=3, n_src=4, snr=np.inf, seed=2)
    g_true = _cplx(g)
    g0 = np.ones_like(g_true)
    sol = oracle.cal_solve(V, M, g0, 80)
    err = np.abs(sol - _ref(g_true)).max() / np.abs(g_true).max()
    assert err < 1e-5, err                       # V and M carry float32 rounding


def test_update_is_a_preconditioned_gradient_step():
    """grad_a = dL/dRe g_a + i dL/dIm g_a (the oracle's adjoint) equals
    -4 (sum_b V_ab conj(z_ab) - g_a sum_b |z_ab|^2), z_ab = M_ab conj(g_b),
    so the alternating update g_a <- num_a / den_a is g_a - grad_a / (4 den_a)."""
    rng = np.random.default_rng(3)
    V, M, _ = W.make_calibration(Na=9, P=2, n_src=3, snr=5.0, seed=4)
    g = (rng.standard_normal((2, 9, 2)) + 1j * rng.standard_normal((2, 9, 2))).astype(np.complex64)
    gf = np.stack([g.real, g.imag], -1).astype(np.float32)
    _, grad = oracle.cal_loss_grad(V, M, gf)
    for ch in range(2):
        for pol in range(2):
            Vf = oracle._full(V[ch], 9, pol)
            Mf = oracle._full(M[ch], 9, pol)
            gg = g[ch, :, pol].astype(np.complex128)
            z = Mf * np.conj(gg)[None, :]
            num = (Vf * np.conj(z)).sum(1)
            den = (np.abs(z) ** 2).sum(1)
            np.testing.assert_allclose(grad[ch, :, pol], -4.0 * (num - gg * den), rtol=1e-9,
                                       atol=1e-9 * np.abs(num).max())


def test_fixed_point_and_gauge():
    V, M, g = W.make_calibration(Na=10, P=2, n_src=4, snr=20.0, seed=6)
    g0 = np.ones((2, 10, 2), np.complex128)
    sol = oracle.cal_solve(V, M, g0, 200)
    again = oracle.cal_solve(V, M, sol, 2)
    np.testing.assert_allclose(again, sol, rtol=0, atol=1e-9)
    rot = oracle.cal_solve(V, M, g0 * np.exp(1j * 0.7), 200)
    np.testing.assert_allclose(rot, sol, rtol=0, atol=1e-9)
    assert np.all(np.abs(np.imag(sol[:, 0, :])) < 1e-12) and np.all(np.real(sol[:, 0, :]) > 0)


def _vis(P, Na, rng, scale=1.0):
    nbl = Na * (Na + 1) // 2
    V = np.zeros((P, nbl, 2, 2, 2), np.float32)
    V[:, :, 0, 0] = rng.standard_normal((P, nbl, 2)) * scale
    V[:, :, 1, 1] = rng.standard_normal((P, nbl, 2)) * scale
    return V


def test_sigma_clip_stage1_outliers():
    rng = np.random.default_rng(5)
    P, Na, k = 8, 20, 5.0
    V = _vis(P, Na, rng)
    bad = [(0, 30, 0), (3, 78, 1), (7, 100, 0)]          # none of them an autocorrelation
    for ch, bl, pol in bad:
        V[ch, bl, pol, pol] *= 60.0
    # autocorrelations are large and never flagged
    for a in range(Na):
        V[:, a * (a + 1) // 2 + a, :, :, 0] += 1e4
    f = oracle.sigma_clip(V, k)
    expect = np.zeros_like(f)
    for ch, bl, pol in bad:
        expect[ch, bl, pol] = 1
    np.testing.assert_array_equal(f, expect)


def test_sigma_clip_stage2_channel_spike():
    """A visibility that is quiet in most channels and 3 sigma of its channel
    in one passes stage 1 (k = 5) but is flagged across channels."""
    rng = np.random.default_rng(6)
    P, Na, k = 64, 12, 5.0
    V = _vis(P, Na, rng)
    bl = 40
    V[:, bl, 0, 0] *= 0.1
    V[17, bl, 0, 0] = [3.0, 0.0]
    f = oracle.sigma_clip(V, k)
    assert f[17, bl, 0] == 1
    assert f[:, bl, 0].sum() == 1
    assert f[:, :, 1].sum() == 0
    # without stage 2 (all channels quiet) nothing is flagged
    V[17, bl, 0, 0] = [0.1, 0.0]
    assert oracle.sigma_clip(V, k)[:, bl, 0].sum() == 0


def test_apply_vis_flags():
    rng = np.random.default_rng(7)
    V = _vis(2, 5, rng)
    f = np.zeros((2, 15, 2), np.uint8)
    f[1, 3, 1] = 1
    Z = oracle.apply_vis_flags(V, f)
    assert np.all(Z[1, 3, 1, 1] == 0) and np.all(Z[1, 3, 0, 0] == V[1, 3, 0, 0])
    Z[1, 3, 1, 1] = V[1, 3, 1, 1]
    np.testing.assert_array_equal(Z, V)


def _ls_step(V, M, g):
    """One simultaneous update: for every antenna a, the least-squares gain
    gamma minimising sum_b |V_ab - gamma M_ab conj(g_b)|^2 with the other
    gains held at g, found by numpy's least-squares solver."""
    Na = g.size
    out = np.empty(Na, np.complex128)
    for a in range(Na):
        A = (M[a, :] * np.conj(g))[:, None]
        out[a] = np.linalg.lstsq(A, V[a, :], rcond=None)[0][0]
    return out


def test_first_iterations_are_least_squares_steps():
    """Iteration 1 is the plain least-squares step, iteration 2 averages the
    step with the previous iterate, iteration 3 is a plain step again; the
    result is phase-referenced (the update commutes with a common phase)."""
    rng = np.random.default_rng(8)
    Na, P = 7, 2
    V, M, _ = W.make_calibration(Na=Na, P=P, n_src=3, snr=4.0, seed=9)
    g0 = rng.uniform(0.7, 1.3, (P, Na, 2)) * np.exp(1j * rng.uniform(0, 2 * np.pi, (P, Na, 2)))
    sols = [oracle.cal_solve(V, M, g0, n) for n in (1, 2, 3)]
    for ch in range(P):
        for pol in range(2):
            Vf = oracle._full(V[ch], Na, pol)
            Mf = oracle._full(M[ch], Na, pol)
            g1 = _ls_step(Vf, Mf, g0[ch, :, pol])
            g2 = 0.5 * (_ls_step(Vf, Mf, g1) + g1)
            g3 = _ls_step(Vf, Mf, g2)
            for n, ref in enumerate((g1, g2, g3)):
                ref = ref * np.conj(ref[0]) / abs(ref[0])
                np.testing.assert_allclose(sols[n][ch, :, pol], ref, rtol=1e-9, atol=1e-12)


def test_sigma_clip_stage2_rms_excludes_stage1_flags():
    """Stage 2 computes each visibility's RMS over the channels that stage 1
    left unflagged.  A quiet baseline with a huge spike in channel 5 (flagged
    by stage 1) and a moderate one in channel 9 (1.5, under 5 RMS of its
    channel): over the 63 remaining channels RMS^2 = (62 * 0.02 + 2.25) / 63
    ~ 0.055, so 1.5 > 5 RMS ~ 1.18 is flagged; had channel 5 been kept,
    RMS ~ 6.3 would hide it."""
    rng = np.random.default_rng(10)
    P, Na, k = 64, 12, 5.0
    V = _vis(P, Na, rng)
    bl = 40
    V[:, bl, 0, 0] = [0.1, 0.1]
    V[5, bl, 0, 0] = [50.0, 0.0]
    V[9, bl, 0, 0] = [1.5, 0.0]
    f = oracle.sigma_clip(V, k)
    assert f[5, bl, 0] == 1 and f[9, bl, 0] == 1
    assert f[:, bl, 0].sum() == 2


def test_weighted_solve_zero_weights_equal_zeroed_data_and_noise_free_recovery():
    """The weighted update with 0/1 weights equals the unweighted one on
    data zeroed at the zero-weight baselines (the sums see the same terms),
    and with any positive weights noise-free data give back the true gains."""
    V, M, g = W.make_calibration(Na=10, P=2, snr=6.0, seed=41)
    P, nbl = V.shape[0], V.shape[1]
    rng = np.random.default_rng(42)
    flags = (rng.random((P, nbl, 2)) < 0.25).astype(np.uint8)
    w = oracle.cal_weights(P, nbl, flags=flags)
    g0 = np.ones((P, 10, 2), np.complex128)
    sw = oracle.cal_solve(V, M, g0, 30, weights=w)
    Vz, Mz = V.copy(), M.copy()
    for pol in range(2):
        sel = flags[:, :, pol] != 0
        Vz[:, :, pol, pol][sel] = 0
        Mz[:, :, pol, pol][sel] = 0
    sz = oracle.cal_solve(Vz, Mz, g0, 30)
    np.testing.assert_allclose(sw, sz, rtol=1e-12, atol=1e-12)
    # noise-free, positive random weights: the true gains (phase-referenced)
    Vc, Mc, gc = W.make_calibration(Na=10, P=2, snr=1e12, seed=43)
    wp = rng.uniform(0.5, 2.0, (P, nbl, 2))
    sol = oracle.cal_solve(Vc, Mc, g0, 300, weights=wp)
    gt = gc[..., 0].astype(np.float64) + 1j * gc[..., 1]
    gt = gt * (np.conj(gt[:, :1, :]) / np.abs(gt[:, :1, :]))
    assert np.abs(sol - gt).max() <= 1e-5 * np.abs(gt).max()
