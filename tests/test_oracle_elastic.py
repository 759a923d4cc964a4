"""Pins of the FP64 elastic oracle (Section III-C): the zero-source invariant,
the fluid limit (mu = 0), exact conservation of the scheme's discrete energy
without damping, and the P-wave speed."""
import math

import numpy as np
import pytest

from paper_2010_10248_amd import workloads as W


def _shot(seed, n, so, nt, nbl, vp, vs, rho, h=10.0, nrec=6):
    s = W.elastic_smooth(seed=seed, n=n, so=so, nt=nt, nbl=nbl, h=h, nrec=nrec, sigma=3.0)
    if vp is not None:
        s.vp = np.broadcast_to(vp, s.shape).astype(np.float64).copy()
        s.vs = np.broadcast_to(vs, s.shape).astype(np.float64).copy()
        s.rho = np.broadcast_to(rho, s.shape).astype(np.float64).copy()
    return s


def test_zero_source_is_exactly_zero(orc):
    s = _shot(1, (20, 22, 24), 8, 20, 3, None, None, None)
    o = orc.elastic_forward(s, src_wav=np.zeros_like(s.src_wav))
    for k in o:
        assert np.all(o[k] == 0.0), k


@pytest.mark.parametrize("so", [4, 8])
def test_fluid_limit(orc, so):
    """mu = 0 and an explosive source: the three normal stresses obey the
    same update from the same data, so they stay equal, and no shear stress
    appears."""
    s = _shot(2, (22, 24, 26), so, 40, 4, None, None, None)
    s.vs = np.zeros(s.shape)
    o = orc.elastic_forward(s)
    assert np.abs(o["txx"]).max() > 0
    assert np.array_equal(o["txx"], o["tyy"]) and np.array_equal(o["txx"], o["tzz"])
    for k in ("txy", "txz", "tyz"):
        assert np.all(o[k] == 0.0), k
    assert np.array_equal(o["p"][0], np.zeros_like(o["p"][0]))  # d^0 = 0


@pytest.mark.parametrize("so", [4, 8])
def test_discrete_energy_conserved(orc, so):
    """Without damping, once the source is off, 1/2 <v^{n+1/2}, v^{n+1/2}>_{1/b}
    + 1/2 <t^{n+1}, C^{-1} t^n> is constant (the staggered differences are
    negative transposes of each other); the damped run is the control."""
    s = _shot(3, (24, 22, 26), so, 60, 0, None, None, None)
    k_off = 20
    s.src_wav[k_off:] = 0.0
    e = orc.elastic_forward(s, want_energy=True)["energy"]
    tail = e[k_off:]
    assert tail[0] > 0
    assert np.abs(tail - tail[0]).max() <= 1e-12 * tail[0]
    s.nbl = 6
    e2 = orc.elastic_forward(s, want_energy=True, vmax_damp=float(s.vp.max()))["energy"][k_off:]
    assert e2[-1] < 0.99 * e2[0]


def test_p_wave_speed(orc):
    """The explosive source radiates P waves only; their moveout between two
    receiver distances along x and along z is (R2 - R1) / vp (the positive
    lobe of the far-field pressure pulse, whose shape does not change with
    distance beyond the near field)."""
    n = (60, 36, 60)
    h = 10.0
    vp, vs, rho = 3000.0, 3000.0 / 1.8, 2000.0
    dt = W.cfl_dt(vp, h)
    f0 = 20.0
    R1, R2 = 16 * h, 32 * h
    nt = int((1.0 / f0 + R2 / vp + 0.04) / dt)
    s = _shot(4, n, 8, nt, 8, vp, vs, rho)
    s.dt = dt
    src = np.array([10.2, 18.0, 10.4]) * h
    s.src_xyz = src[None, :]
    s.src_wav = W.ricker(f0, nt, dt)[:, None]
    s.rec_xyz = np.array([src + [R1, 0, 0], src + [R2, 0, 0], src + [0, 0, R1], src + [0, 0, R2]])
    p = orc.elastic_forward(s)["p"]

    def tpk(k):
        i = int(np.argmax(p[:, k]))
        y0, y1, y2 = p[i - 1:i + 2, k]
        return (i + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * dt

    want = (R2 - R1) / vp
    for a, b in ((0, 1), (2, 3)):
        got = tpk(b) - tpk(a)
        assert abs(got - want) <= 0.02 * want, (a, b, got, want)


# --------------------------------------------------------------------------
# Adjoint of the elastic map q -> (vz, P) (or_elastic_adjoint): the FP64
# dot-product identity against the oracle forward, SO4 and SO8, damping on;
# a one-sample time shift breaks it, and so does a model whose shear modulus
# differs (the adjoint must carry the same C).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("so", [4, 8])
def test_elastic_adjoint_dot_product(orc, so):
    s = W.elastic_smooth(seed=51, n=(18, 20, 22), so=so, nt=36, nbl=4, nrec=6, sigma=3.0)
    rng = np.random.Generator(np.random.PCG64(13))
    q = rng.standard_normal(s.src_wav.shape)
    dp = rng.standard_normal((2, s.nt, s.rec_xyz.shape[0]))
    fw = orc.elastic_forward(s, src_wav=q)
    lhs = float(np.sum(fw["vz"] * dp[0]) + np.sum(fw["p"] * dp[1]))
    FTd = orc.elastic_adjoint(s, dp)
    rhs = float(np.sum(q * FTd))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs)), (lhs, rhs)
    assert np.all(FTd[-1] == 0.0)
    assert abs(lhs - float(np.sum(q[1:] * FTd[:-1]))) > 1e-3 * abs(lhs)
    import copy

    s2 = copy.copy(s)
    s2.vs = s.vs * 0.9
    assert abs(lhs - float(np.sum(q * orc.elastic_adjoint(s2, dp)))) > 1e-4 * abs(lhs)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_elastic_gradient_taylor(orc, which):
    """Gradient of the elastic misfit w.r.t. lambda, mu and b = 1/rho at the
    nodes (or_elastic_adjoint with the forward history): perturbing one of
    them along a smooth direction, the first-order Taylor remainder falls as
    h^2 over halvings. The model passes through (vp, vs, rho), so the test
    also checks the chain through the two- and four-node means."""
    s = W.elastic_smooth(seed=53, n=(16, 18, 20), so=8, nt=40, nbl=4, nrec=6, sigma=3.0)
    vmax = 4000.0
    rho0 = s.rho
    lam0 = rho0 * (s.vp ** 2 - 2 * s.vs ** 2)
    mu0 = rho0 * s.vs ** 2
    b0 = 1.0 / rho0
    n = s.shape
    X, Y, Z = np.meshgrid(*[np.arange(k, dtype=float) for k in n], indexing="ij")
    blob = np.exp(-((X - n[0] / 2) ** 2 + (Y - n[1] / 2) ** 2 + (Z - n[2] / 2) ** 2) / 12.0)
    fw = orc.elastic_forward(s, vmax_damp=vmax, vs=s.vs * (1.0 + 0.04 * blob),
                             vp=s.vp * (1.0 + 0.03 * blob))
    dobs = np.stack([fw["vz"], fw["p"]])

    def model(lam, mu, b):
        rho = 1.0 / b
        return dict(vp=np.sqrt((lam + 2 * mu) * b), vs=np.sqrt(mu * b), rho=rho)

    J0, g = orc.elastic_gradient(s, dobs, vmax_damp=vmax)
    rng = np.random.Generator(np.random.PCG64(20 + which))
    from scipy.ndimage import gaussian_filter

    base = (lam0, mu0, b0)
    dp = gaussian_filter(rng.standard_normal(n), 2.0)
    dp *= 0.005 * np.abs(base[which]).max() / np.abs(dp).max()
    gd = float(np.sum(g[which] * dp))
    errs = []
    for k in range(5):
        hstep = 2.0 ** (-k)
        p = [x.copy() for x in base]
        p[which] = p[which] + hstep * dp
        f2 = orc.elastic_forward(s, vmax_damp=vmax, **model(*p))
        Jh = 0.5 * float(np.sum((np.stack([f2["vz"], f2["p"]]) - dobs) ** 2))
        errs.append(abs(Jh - J0 - hstep * gd))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.4 < r < 4.7 for r in ratios), ratios
    # The first-order term dominates the remainder at the smallest step (a
    # random smooth direction can be nearly orthogonal to the gradient, so
    # the largest step is not used for this).
    assert abs(2.0 ** (-4) * gd) > 4 * errs[-1]
