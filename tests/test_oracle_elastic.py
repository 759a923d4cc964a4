"""Pins of the FP64 elastic oracle (Section III-C): the zero-source invariant,
the fluid limit (mu = 0), exact conservation of the scheme's discrete energy
without damping, and the P-wave speed."""
import math
import os

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


# --------------------------------------------------------------------------
# The two passes on their own, against closed forms (Section III-C's
# first-order system: rho v_t = div tau, tau_t = lambda tr(e) I + 2 mu e with
# e the symmetric velocity gradient). Every field is a quadratic polynomial
# sampled at its component's staggered position, so the staggered
# derivatives of the space order are exact away from the edges and each pass
# must return the pointwise formula there. A half-cell error in a position,
# a swapped lambda/mu role, a missing factor 2 or a wrong mean fails these.
# --------------------------------------------------------------------------
_FIELDS = ("vx", "vy", "vz", "txx", "tyy", "tzz", "txy", "txz", "tyz")
_OFF = {"vx": (0.5, 0, 0), "vy": (0, 0.5, 0), "vz": (0, 0, 0.5), "txx": (0, 0, 0),
        "tyy": (0, 0, 0), "tzz": (0, 0, 0), "txy": (0.5, 0.5, 0), "txz": (0.5, 0, 0.5),
        "tyz": (0, 0.5, 0.5)}


def _coords(n, h, off):
    return np.meshgrid(*[(np.arange(m) + o) * hh for m, o, hh in zip(n, off, h)], indexing="ij")


def _quad(rng):
    return rng.standard_normal(), rng.standard_normal(3), rng.standard_normal((3, 3))


def _qval(c, X):
    c0, b, A = c
    return c0 + sum(b[i] * X[i] for i in range(3)) + sum(
        A[i, j] * X[i] * X[j] for i in range(3) for j in range(3))


def _qgrad(c, X, a):
    _, b, A = c
    return b[a] + sum((A[a, j] + A[j, a]) * X[j] for j in range(3))


def _materials(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    vp = W.smooth_field(rng, n, 2000.0, 4000.0, 3.0)
    vs = vp / W.smooth_field(rng, n, 1.6, 2.2, 3.0)
    rho = W.smooth_field(rng, n, 1800.0, 2600.0, 3.0)
    return vp, vs, rho


@pytest.mark.parametrize("so", [4, 8])
def test_velocity_pass_closed_form(orc, so):
    n, h, dt = (22, 20, 24), (10.0, 12.0, 9.0), 1e-3
    vp, vs, rho = _materials(n, 31 + so)
    rng = np.random.Generator(np.random.PCG64(so))
    polys = {f: _quad(rng) for f in _FIELDS}
    # (scaled so the stresses are O(1e6) Pa over the box)
    state = np.stack([_qval(polys[f], [x / 100.0 for x in _coords(n, h, _OFF[f])]) * 1e6
                      for f in _FIELDS])
    state[:3] = rng.standard_normal((3,) + n)  # v^{n-1/2} is carried over (alpha = beta = 1)
    out = orc.elastic_passes(state, h, so, dt, vp, vs, rho, which=1)
    b = 1.0 / rho
    r = so // 2
    inner = tuple(slice(r, m - r) for m in n)
    comps = {"vx": ("txx", "txy", "txz"), "vy": ("txy", "tyy", "tyz"), "vz": ("txz", "tyz", "tzz")}
    for a, f in enumerate(("vx", "vy", "vz")):
        X = [x / 100.0 for x in _coords(n, h, _OFF[f])]
        div = sum(_qgrad(polys[t], X, ax) * 1e6 / 100.0 for ax, t in enumerate(comps[f]))
        bn = np.roll(b, -1, axis=a)  # b at the next node along a (interior only)
        want = state[a] + dt * 0.5 * (b + bn) * div
        scale = np.abs(want[inner]).max()
        assert np.abs(out[a][inner] - want[inner]).max() <= 1e-10 * scale, f
        assert np.abs(out[a] - want).max() > 1e-4 * scale  # edges differ: not vacuous
    assert np.array_equal(out[3:], state[3:])


@pytest.mark.parametrize("so", [4, 8])
def test_stress_pass_closed_form(orc, so):
    n, h, dt = (22, 20, 24), (10.0, 12.0, 9.0), 1e-3
    vp, vs, rho = _materials(n, 41 + so)
    lam = rho * (vp ** 2 - 2 * vs ** 2)
    mu = rho * vs ** 2
    rng = np.random.Generator(np.random.PCG64(10 + so))
    polys = {f: _quad(rng) for f in _FIELDS}
    state = np.stack([_qval(polys[f], [x / 100.0 for x in _coords(n, h, _OFF[f])])
                      for f in _FIELDS])
    state[3:] = rng.standard_normal((6,) + n) * 1e3  # tau^n is carried over
    out = orc.elastic_passes(state, h, so, dt, vp, vs, rho, which=2)

    def grad(comp, at, ax):
        X = [x / 100.0 for x in _coords(n, h, _OFF[at])]
        return _qgrad(polys[comp], X, ax) / 100.0

    r = so // 2
    inner = tuple(slice(r, m - r) for m in n)
    e = [grad(f, "txx", a) for a, f in enumerate(("vx", "vy", "vz"))]
    tr = e[0] + e[1] + e[2]
    for a, f in enumerate(("txx", "tyy", "tzz")):
        want = state[3 + a] + dt * (lam * tr + 2.0 * mu * e[a])
        scale = np.abs(want[inner] - state[3 + a][inner]).max()
        assert np.abs(out[3 + a][inner] - want[inner]).max() <= 1e-9 * scale, f
    for k, (f, a1, a2) in enumerate((("txy", 0, 1), ("txz", 0, 2), ("tyz", 1, 2))):
        v1, v2 = ("vx", "vy", "vz")[a1], ("vx", "vy", "vz")[a2]
        g = grad(v1, f, a2) + grad(v2, f, a1)
        m1 = np.roll(mu, -1, axis=a1)
        mbar = 0.25 * (mu + m1 + np.roll(mu, -1, axis=a2) + np.roll(m1, -1, axis=a2))
        want = state[6 + k] + dt * mbar * g
        scale = np.abs(want[inner] - state[6 + k][inner]).max()
        assert np.abs(out[6 + k][inner] - want[inner]).max() <= 1e-9 * scale, f
        # the node value of mu instead of the 4-node mean is detectably wrong
        bad = state[6 + k] + dt * mu * g
        assert np.abs(out[6 + k][inner] - bad[inner]).max() > 1e-4 * scale, f
    assert np.array_equal(out[:3], state[:3])


def test_passes_with_damping(orc):
    """Damping multiplies the carried level by beta and divides by alpha,
    with d at the element's node index, in both passes."""
    n, h, dt, nbl, vmax = (20, 22, 18), (10.0, 10.0, 10.0), 1e-3, 5, 4000.0
    vp, vs, rho = _materials(n, 61)
    rng = np.random.Generator(np.random.PCG64(62))
    state = rng.standard_normal((9,) + n)
    d = orc.damping(n, h, nbl, vmax)
    al, be = 1.0 + d * dt / 2.0, 1.0 - d * dt / 2.0
    free = orc.elastic_passes(state, h, 8, dt, vp, vs, rho, which=1)
    damp = orc.elastic_passes(state, h, 8, dt, vp, vs, rho, which=1, nbl=nbl, vmax_damp=vmax)
    for a in range(3):
        # undamped increment dt b D t = free - state
        want = (be * state[a] + (free[a] - state[a])) / al
        assert np.abs(damp[a] - want).max() <= 1e-12 * np.abs(want).max()
    free = orc.elastic_passes(state, h, 8, dt, vp, vs, rho, which=2)
    damp = orc.elastic_passes(state, h, 8, dt, vp, vs, rho, which=2, nbl=nbl, vmax_damp=vmax)
    for f in range(3, 9):
        want = (be * state[f] + (free[f] - state[f])) / al
        assert np.abs(damp[f] - want).max() <= 1e-10 * np.abs(want).max()
    assert np.abs(d).max() > 0


# --------------------------------------------------------------------------
# Fluid limit against a separate brute-force velocity-pressure code. With
# mu = 0 and an explosive source the normal stresses stay equal (p), the
# shear stresses zero, and the system is the staggered acoustic
# velocity-pressure scheme
#   v_a <- (beta v_a + dt bbar_a D+_a p) / alpha,
#   p   <- (beta p + dt lambda sum_a D-_a v_a) / alpha + dt W q,
# written below from that statement alone (numpy slices on zero-padded
# arrays, the printed staggered weights, its own trilinear weights).
# --------------------------------------------------------------------------
def _stag_weights(so):
    from fractions import Fraction

    for line in open(os.path.join(os.path.dirname(__file__), "golden", "fd_weights.txt")):
        f = line.split()
        if f and f[0] == "d1s" and int(f[1]) == so:
            return [float(Fraction(x)) for x in f[2:]]
    raise KeyError(so)


def _tri(p, o, h):
    xi = [(p[a] - o[a]) / h[a] for a in range(3)]
    i0 = [int(math.floor(x)) for x in xi]
    fr = [x - i for x, i in zip(xi, i0)]
    out = []
    for bx in (0, 1):
        for by in (0, 1):
            for bz in (0, 1):
                w = 1.0
                for a, bb in enumerate((bx, by, bz)):
                    w *= fr[a] if bb else 1.0 - fr[a]
                if w != 0.0:
                    out.append(((i0[0] + bx, i0[1] + by, i0[2] + bz), w))
    return out


def _brute_velocity_pressure(s, d):
    n, h, dt, r = s.shape, s.spacing, s.dt, s.space_order // 2
    w = _stag_weights(s.space_order)
    lam = s.rho * s.vp ** 2
    b = 1.0 / s.rho
    al, be = 1.0 + d * dt / 2.0, 1.0 - d * dt / 2.0

    def pad(u):
        return np.pad(u, r + 1)

    def sl(u, a, k):  # u shifted by k along axis a, on the padded array
        idx = [slice(r + 1, r + 1 + m) for m in n]
        idx[a] = slice(r + 1 + k, r + 1 + k + n[a])
        return u[tuple(idx)]

    def dplus(u, a):  # field at nodes, result half a cell up
        up = pad(u)
        return sum(w[m] * (sl(up, a, m + 1) - sl(up, a, -m)) for m in range(r)) / h[a]

    def dminus(u, a):  # field half a cell up, result at nodes
        up = pad(u)
        return sum(w[m] * (sl(up, a, m) - sl(up, a, -m - 1)) for m in range(r)) / h[a]

    def bbar(a):
        bn = np.concatenate([np.take(b, range(1, n[a]), axis=a),
                             np.take(b, [n[a] - 1], axis=a)], axis=a)
        return 0.5 * (b + bn)

    v = [np.zeros(n) for _ in range(3)]
    p = np.zeros(n)
    nrec = s.rec_xyz.shape[0]
    tr_vz, tr_p = np.zeros((s.nt, nrec)), np.zeros((s.nt, nrec))
    ovz = (s.origin[0], s.origin[1], s.origin[2] + 0.5 * h[2])
    for t in range(s.nt):
        for k in range(nrec):
            tr_vz[t, k] = sum(wt * v[2][c] for c, wt in _tri(s.rec_xyz[k], ovz, h))
            tr_p[t, k] = sum(wt * p[c] for c, wt in _tri(s.rec_xyz[k], s.origin, h))
        v = [(be * v[a] + dt * bbar(a) * dplus(p, a)) / al for a in range(3)]
        p = (be * p + dt * lam * sum(dminus(v[a], a) for a in range(3))) / al
        for k in range(s.src_xyz.shape[0]):
            for c, wt in _tri(s.src_xyz[k], s.origin, h):
                p[c] += dt * wt * s.src_wav[t, k]
    return tr_vz, tr_p, v, p


@pytest.mark.parametrize("so", [4, 8])
def test_fluid_limit_equals_brute_force_velocity_pressure(orc, so):
    s = _shot(5, (20, 22, 24), so, 40, 4, None, None, None)
    s.vs = np.zeros(s.shape)
    vmax = float(s.vp.max())
    o = orc.elastic_forward(s, vmax_damp=vmax)
    tr_vz, tr_p, v, p = _brute_velocity_pressure(s, orc.damping(s.shape, s.spacing, s.nbl, vmax))
    assert np.abs(tr_p).max() > 0 and np.abs(tr_vz).max() > 0
    tol = 1e-12
    assert np.abs(o["p"] - tr_p).max() <= tol * np.abs(tr_p).max()
    assert np.abs(o["vz"] - tr_vz).max() <= tol * np.abs(tr_vz).max()
    for f, ref in (("vx", v[0]), ("vy", v[1]), ("vz_field", v[2]), ("txx", p)):
        assert np.abs(o[f] - ref).max() <= tol * np.abs(ref).max(), f
