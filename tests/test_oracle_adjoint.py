"""Pins of the oracle's discrete adjoint and gradient (CPU).

The adjoint is pinned by the dot-product identity <F q, d'> = <q, F^T d'>
and the gradient by a Taylor test: |J(m + h dm) - J(m) - h <g, dm>| must
fall as h^2. A wrong sign, a dropped term (for example the m-dependence of
the dt^2/m injection) or an off-by-one in the time index breaks one of them.
"""
import numpy as np
import pytest

from paper_2010_10248_amd import workloads as W


def _shot(nt=45, nbl=4, n=(22, 24, 26), so=8, seed=11):
    return W.acoustic_scaled(seed, n, so, nt, nbl, nsrc=2, nrec=5, layered=True)


@pytest.mark.parametrize("so", [4, 8])
def test_dot_product_adjoint(orc, so):
    s = _shot(so=so)
    rng = np.random.Generator(np.random.PCG64(5))
    q = rng.standard_normal(s.src_wav.shape)
    dp = rng.standard_normal((s.nt, s.rec_xyz.shape[0]))
    Fq = orc.acoustic_forward(s, src_wav=q)["traces"]
    FTd = orc.acoustic_adjoint(s, dp)["qhat"]
    lhs = float(np.sum(Fq * dp))
    rhs = float(np.sum(q * FTd))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))
    # the last adjoint sample is identically zero (nu^{nt} = 0)
    assert np.all(FTd[-1] == 0.0)


def test_dot_product_fails_for_wrong_time_shift(orc):
    """Control: shifting the adjoint output by one sample breaks the identity,
    so the dot test is sensitive to the time index."""
    s = _shot()
    rng = np.random.Generator(np.random.PCG64(6))
    q = rng.standard_normal(s.src_wav.shape)
    dp = rng.standard_normal((s.nt, s.rec_xyz.shape[0]))
    Fq = orc.acoustic_forward(s, src_wav=q)["traces"]
    FTd = orc.acoustic_adjoint(s, dp)["qhat"]
    lhs = float(np.sum(Fq * dp))
    rhs = float(np.sum(q[1:] * FTd[:-1]))
    assert abs(lhs - rhs) > 1e-3 * abs(lhs)


def test_gradient_taylor(orc):
    s = _shot(nt=60)
    vmax = 4500.0
    m0 = 1.0 / s.vp ** 2
    # observed data from a smooth perturbation of the model
    n = s.shape
    ii = [np.arange(k, dtype=float) for k in n]
    X, Y, Z = np.meshgrid(*ii, indexing="ij")
    blob = np.exp(-((X - n[0] / 2) ** 2 + (Y - n[1] / 2) ** 2 + (Z - n[2] / 2) ** 2) / 18.0)
    vp_true = s.vp * (1.0 + 0.05 * blob)
    dobs = orc.acoustic_forward(s, vp=vp_true, vmax_damp=vmax)["traces"]
    J0, g, _ = orc.acoustic_gradient(s, dobs, vmax_damp=vmax)
    rng = np.random.Generator(np.random.PCG64(9))
    from scipy.ndimage import gaussian_filter
    dm = gaussian_filter(rng.standard_normal(n), 2.0)
    dm *= 0.02 * np.abs(m0).max() / np.abs(dm).max()
    gd = float(np.sum(g * dm))
    errs = []
    for k in range(5):
        hstep = 2.0 ** (-k)
        vp_h = 1.0 / np.sqrt(m0 + hstep * dm)
        Jh = orc.misfit(orc.acoustic_forward(s, vp=vp_h, vmax_damp=vmax)["traces"], dobs)
        errs.append(abs(Jh - J0 - hstep * gd))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    # second-order decay: each halving divides the remainder by ~4
    assert all(3.5 < r < 4.6 for r in ratios), ratios
    # and the first-order term is the dominant part of the change
    assert abs(gd) > 4 * errs[0]
