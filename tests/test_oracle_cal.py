"""Pins for the oracle's calibration loss and gradient (CPU only).

Independent references: a hand-worked two-antenna example (golden file),
numpy's Frobenius norm of the full matrices, torch autograd on complex128,
central finite differences, zero gradient at noise-free true gains, phase-
gauge invariance and the scaling identity.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cplx(a):
    return a[..., 0] + 1j * a[..., 1]


def _full(lower, Na):
    """Hermitian completion of a lower-triangle vector (numpy)."""
    F = np.zeros((Na, Na), np.complex128)
    a, b = np.tril_indices(Na)
    F[a, b] = lower
    F[b, a] = np.conj(lower)
    return F


def _rand_case(rng, Na, P):
    nbl = Na * (Na + 1) // 2
    V = rng.standard_normal((P, nbl, 2, 2, 2)).astype(np.float32)
    M = rng.standard_normal((P, nbl, 2, 2, 2)).astype(np.float32)
    # autos of a Hermitian matrix are real
    d = np.array([a * (a + 1) // 2 + a for a in range(Na)])
    V[:, d, 0, 0, 1] = 0
    V[:, d, 1, 1, 1] = 0
    M[:, d, 0, 0, 1] = 0
    M[:, d, 1, 1, 1] = 0
    g = rng.standard_normal((P, Na, 2, 2)).astype(np.float32)
    return V, M, g


def test_hand_worked_two_antennas():
    gd = json.load(open(os.path.join(GOLDEN, "cal_na2_hand.json")))
    Na = gd["Na"]
    V = np.zeros((1, 3, 2, 2, 2), np.float32)
    M = np.zeros_like(V)
    g = np.zeros((1, Na, 2, 2), np.float32)
    V[0, :, 0, 0] = gd["V_xx_lower"]
    M[0, :, 0, 0] = gd["M_xx_lower"]
    g[0, :, 0] = gd["g_x"]
    g[0, :, 1, 0] = 1.0
    loss, grad = oracle.cal_loss_grad(V, M, g)
    assert loss[0, 0] == gd["loss_xx"] and loss[0, 1] == gd["loss_yy"]
    np.testing.assert_array_equal(grad[0, :, 0], _cplx(np.array(gd["grad_x"], float)))
    np.testing.assert_array_equal(grad[0, :, 1], _cplx(np.array(gd["grad_y"], float)))


def test_loss_matches_numpy_norm():
    rng = np.random.default_rng(1)
    Na, P = 6, 3
    V, M, g = _rand_case(rng, Na, P)
    loss, _ = oracle.cal_loss_grad(V, M, g, want_grad=False)
    for k in range(P):
        for pol in range(2):
            Vf = _full(_cplx(V[k, :, pol, pol].astype(np.float64)), Na)
            Mf = _full(_cplx(M[k, :, pol, pol].astype(np.float64)), Na)
            G = np.diag(_cplx(g[k, :, pol].astype(np.float64)))
            ref = np.linalg.norm(Vf - G @ Mf @ G.conj().T) ** 2
            assert np.isclose(loss[k, pol], ref, rtol=1e-12)


def test_grad_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    Na, P = 5, 2
    V, M, g = _rand_case(rng, Na, P)
    _, grad = oracle.cal_loss_grad(V, M, g)
    for k in range(P):
        for pol in range(2):
            Vf = torch.tensor(_full(_cplx(V[k, :, pol, pol].astype(np.float64)), Na))
            Mf = torch.tensor(_full(_cplx(M[k, :, pol, pol].astype(np.float64)), Na))
            gt = torch.tensor(_cplx(g[k, :, pol].astype(np.float64)), requires_grad=True)
            R = Vf - gt[:, None] * Mf * gt.conj()[None, :]
            L = (R.abs() ** 2).sum()
            L.backward()
            np.testing.assert_allclose(grad[k, :, pol], gt.grad.numpy(), rtol=1e-10, atol=1e-10)


def test_grad_central_differences():
    rng = np.random.default_rng(3)
    Na, P = 7, 1
    V, M, g = _rand_case(rng, Na, P)
    # work in float64 gains for the finite differences: pass through float32 exactly
    g = np.round(g * 64) / 64
    loss, grad = oracle.cal_loss_grad(V, M, g)
    h = 1.0 / 1024          # a power of two near 1e-3 keeps g +- h exact in float32
    for a in [0, 3, 6]:
        for comp, unit in [(0, 1.0), (1, 1j)]:
            gp = g.copy(); gp[0, a, 0, comp] += h
            gm = g.copy(); gm[0, a, 0, comp] -= h
            lp, _ = oracle.cal_loss_grad(V, M, gp, want_grad=False)
            lm, _ = oracle.cal_loss_grad(V, M, gm, want_grad=False)
            fd = (lp[0, 0] - lm[0, 0]) / (2 * h)
            an = grad[0, a, 0].real if comp == 0 else grad[0, a, 0].imag
            # the loss is quartic in g: central-difference error is O(h^2) * |g|^2 |M|^2
            assert abs(fd - an) <= 1e-4 * max(1.0, abs(an))


def test_zero_residual_zero_grad_and_invariants():
    V, M, g = W.make_calibration(Na=12, P=2, snr=1e12, seed=11)
    # noise-free data at the true gains: V = G M G^H up to float32 storage
    loss, grad = oracle.cal_loss_grad(V, M, g)
    scale = np.abs(_cplx(V.astype(np.float64))).max()
    assert np.all(loss <= (1e-6 * scale) ** 2 * V.shape[1] * 4)
    # and the gradient vanishes there: each term of grad_a carries a residual
    # R_ab, bounded by the float32 storage of V and g (|R| <= 4 * 2^-24 max|V|),
    # so |grad_a| <= 4 Na max|R| max|g| max|M| (2.7 here against 33; 7e6 at
    # the generic point below)
    Na = g.shape[1]
    r_max = 4 * 2.0 ** -24 * np.abs(V.astype(np.float64)).max()
    assert np.abs(grad).max() <= 4 * Na * r_max * np.abs(g.astype(np.float64)).max() * np.abs(M.astype(np.float64)).max()
    # a generic point: noisy data, perturbed gains
    V2, M2, g2 = W.make_calibration(Na=12, P=2, snr=5.0, seed=12)
    g2 = (g2 * 1.1).astype(np.float32)
    loss2, grad2 = oracle.cal_loss_grad(V2, M2, g2)
    gg2 = _cplx(g2.astype(np.float64))
    for k in range(2):
        for pol in range(2):
            # phase gauge: L(g e^{i phi}) = L(g)  =>  sum Im(conj(g) grad) = 0
            gauge = np.sum(np.imag(np.conj(gg2[k, :, pol]) * grad2[k, :, pol]))
            mag = np.sum(np.abs(gg2[k, :, pol] * grad2[k, :, pol]))
            assert abs(gauge) <= 1e-10 * mag
            # scaling: d/dt L(t g) at t=1 = sum Re(conj(g) grad) = -4 Re tr(R^H G M G^H)
            Vf = _full(_cplx(V2[k, :, pol, pol].astype(np.float64)), 12)
            Mf = _full(_cplx(M2[k, :, pol, pol].astype(np.float64)), 12)
            G = np.diag(gg2[k, :, pol])
            S_ = G @ Mf @ G.conj().T
            R = Vf - S_
            lhs = np.sum(np.real(np.conj(gg2[k, :, pol]) * grad2[k, :, pol]))
            rhs = -4.0 * np.real(np.trace(R.conj().T @ S_))
            assert np.isclose(lhs, rhs, rtol=1e-9)


# ---- weighted loss (flags and lost-data weights)

def _weights(rng, P, Na, zero_frac=0.2):
    nbl = Na * (Na + 1) // 2
    w = rng.uniform(0.25, 2.0, (P, nbl, 2))
    w[rng.random((P, nbl, 2)) < zero_frac] = 0.0
    return w


def test_weighted_loss_is_weighted_frobenius_sum():
    """L = sum_{a,b} w_ab |R_ab|^2 over the full matrices (numpy), with the
    weights completed symmetrically."""
    rng = np.random.default_rng(31)
    Na, P = 9, 2
    V, M, g = _rand_case(rng, Na, P)
    w = _weights(rng, P, Na)
    loss, _ = oracle.cal_loss_grad(V, M, g, weights=w)
    a_, b_ = np.tril_indices(Na)
    for k in range(P):
        for pol in range(2):
            Vf = _full(_cplx(V[k, :, pol, pol].astype(np.float64)), Na)
            Mf = _full(_cplx(M[k, :, pol, pol].astype(np.float64)), Na)
            Wf = np.zeros((Na, Na))
            Wf[a_, b_] = w[k, :, pol]
            Wf[b_, a_] = w[k, :, pol]
            G = np.diag(_cplx(g[k, :, pol].astype(np.float64)))
            R = Vf - G @ Mf @ G.conj().T
            assert np.isclose(loss[k, pol], np.sum(Wf * np.abs(R) ** 2), rtol=1e-12)


def test_weighted_unit_weights_equal_unweighted_and_scaling():
    rng = np.random.default_rng(32)
    V, M, g = _rand_case(rng, 8, 2)
    l0, g0 = oracle.cal_loss_grad(V, M, g)
    l1, g1 = oracle.cal_loss_grad(V, M, g, weights=np.ones((2, 36, 2)))
    np.testing.assert_array_equal(l0, l1)
    np.testing.assert_array_equal(g0, g1)
    w = _weights(rng, 2, 8)
    lw, gw = oracle.cal_loss_grad(V, M, g, weights=w)
    l2, g2 = oracle.cal_loss_grad(V, M, g, weights=2 * w)      # exact: a power of two
    np.testing.assert_array_equal(l2, 2 * lw)
    np.testing.assert_array_equal(g2, 2 * gw)


def test_flagged_baselines_equal_zeroed_data():
    """A zero weight removes the baseline: the same loss and gradient as
    zeroing V and M there (R = 0).  Flags map to zero weights."""
    rng = np.random.default_rng(33)
    Na, P = 10, 2
    V, M, g = _rand_case(rng, Na, P)
    nbl = Na * (Na + 1) // 2
    flags = (rng.random((P, nbl, 2)) < 0.3).astype(np.uint8)
    w = oracle.cal_weights(P, nbl, flags=flags)
    assert np.all(w[flags != 0] == 0) and np.all(w[flags == 0] == 1)
    lw, gw = oracle.cal_loss_grad(V, M, g, weights=w)
    Vz, Mz = V.copy(), M.copy()
    for pol in range(2):
        sel = flags[:, :, pol] != 0
        Vz[:, :, pol, pol][sel] = 0
        Mz[:, :, pol, pol][sel] = 0
    lz, gz = oracle.cal_loss_grad(Vz, Mz, g)
    np.testing.assert_allclose(lw, lz, rtol=1e-13)
    np.testing.assert_allclose(gw, gz, rtol=1e-12, atol=1e-12 * np.abs(gz).max())
    # flags and weights together: flagged entries 0, others the weight
    w2 = oracle.cal_weights(P, nbl, flags=flags, weights=np.full((P, nbl, 2), 3.0))
    assert np.all(w2[flags != 0] == 0) and np.all(w2[flags == 0] == 3.0)


def test_weighted_gradient_finite_differences():
    rng = np.random.default_rng(34)
    Na, P = 7, 1
    V, M, g = _rand_case(rng, Na, P)
    g = np.round(g * 64) / 64
    w = _weights(rng, P, Na)
    _, grad = oracle.cal_loss_grad(V, M, g, weights=w)
    h = 1.0 / 1024
    for a in [0, 2, 6]:
        for pol in range(2):
            for comp in range(2):
                gp = g.copy(); gp[0, a, pol, comp] += h
                gm = g.copy(); gm[0, a, pol, comp] -= h
                lp, _ = oracle.cal_loss_grad(V, M, gp, want_grad=False, weights=w)
                lm, _ = oracle.cal_loss_grad(V, M, gm, want_grad=False, weights=w)
                fd = (lp[0, pol] - lm[0, pol]) / (2 * h)
                an = grad[0, a, pol].real if comp == 0 else grad[0, a, pol].imag
                assert abs(fd - an) <= 1e-4 * max(1.0, abs(an))
