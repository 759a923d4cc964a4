"""CPU model of the legality argument of Section II (Fig. 4): a temporally
blocked schedule with overlapped tiles computes every point of a tile's halo
redundantly, so an off-grid source whose support falls in a halo must be
injected into the redundant copy too. This is a small 1-D leapfrog in FP64,
independent of the GPU library: tiles of width W with halos of r(T-1) advance
T steps each from the state at the start of the time tile, and are compared
with the naive order (every point updated, then injected, per step).

* every computed copy injected  -> equal to the naive order (to rounding);
* only owned copies injected    -> different (the violation of Fig. 4b);
* spatial blocking (no halo)     -> both variants equal.
"""
import numpy as np
import pytest

W2 = {1: np.array([-2.0, 1.0]), 2: np.array([-5 / 2, 4 / 3, -1 / 12])}


def _lap(u, r):
    """Centred second difference of order 2r with zero outside."""
    w = W2[r]
    p = np.pad(u, r)
    n = u.size
    out = w[0] * u
    for j in range(1, r + 1):
        out = out + w[j] * (p[r + j:r + j + n] + p[r - j:r - j + n])
    return out


def _inject(n, src, t):
    """Increment of step t: sources as (position, weight-per-corner) pairs."""
    s = np.zeros(n)
    for x, amp in src:
        i = int(np.floor(x))
        f = x - i
        q = amp * np.sin(0.3 * t + x)
        if 1.0 - f != 0.0:
            s[i] += (1.0 - f) * q
        if f != 0.0:
            s[i + 1] += f * q
    return s


def naive(n, r, c, nt, src):
    um, u = np.zeros(n), np.zeros(n)
    for t in range(nt):
        un = c * _lap(u, r) + 2 * u - um + _inject(n, src, t)
        um, u = u, un
    return u, um


def tiled(n, r, c, nt, src, T, width, inject_halo):
    """Time tiles of T steps; each spatial tile of `width` owned points
    recomputes its halo of r(T-1) from the tile-start state."""
    um, u = np.zeros(n), np.zeros(n)
    t0 = 0
    while t0 < nt:
        Tt = min(T, nt - t0)
        H = r * (Tt - 1)
        nu, num = np.zeros(n), np.zeros(n)
        for a in range(0, n, width):
            b = min(n, a + width)
            lo, hi = max(0, a - H - r), min(n, b + H + r)
            lu, lum = u[lo:hi].copy(), um[lo:hi].copy()
            # Values beyond [lo, hi) are taken as zero, so the outer r points
            # go wrong each step; after Tt steps [a, b) (and its previous
            # level) is still exact because the region reaches H + r out.
            for s in range(Tt):
                full = np.zeros(n)
                full[lo:hi] = lu
                lap = _lap(full, r)[lo:hi]
                ln = c[lo:hi] * lap + 2 * lu - lum
                inc = _inject(n, src, t0 + s)[lo:hi]
                if inject_halo:
                    ln = ln + inc
                else:
                    own = np.zeros(hi - lo, bool)
                    own[a - lo:b - lo] = True
                    ln = ln + np.where(own, inc, 0.0)
                lum, lu = lu, ln
            nu[a:b] = lu[a - lo:b - lo]
            num[a:b] = lum[a - lo:b - lo]
        u, um = nu, num
        t0 += Tt
    return u, um


@pytest.mark.parametrize("r,T", [(1, 2), (2, 2), (2, 3), (1, 4)])
def test_halo_copies_must_be_injected(r, T):
    n, nt, width = 96, 30, 16
    c = np.full(n, 0.2)
    # A source straddling a tile seam: its support lies in the neighbour's halo.
    src = [(31.6, 1.0), (55.25, 0.7)]
    ref_u, ref_um = naive(n, r, c, nt, src)
    u, um = tiled(n, r, c, nt, src, T, width, inject_halo=True)
    assert np.abs(u - ref_u).max() <= 1e-12 * np.abs(ref_u).max()
    assert np.abs(um - ref_um).max() <= 1e-12 * np.abs(ref_um).max()
    bad, _ = tiled(n, r, c, nt, src, T, width, inject_halo=False)
    assert np.abs(bad - ref_u).max() > 1e-3 * np.abs(ref_u).max()


def test_owner_only_is_harmless_without_halo_sources():
    """Spatial blocking (T = 1) has no halo copies: both variants agree."""
    n, nt, width, r = 80, 25, 16, 2
    c = np.full(n, 0.2)
    src = [(31.6, 1.0)]
    ref_u, _ = naive(n, r, c, nt, src)
    for inject_halo in (True, False):
        u, _ = tiled(n, r, c, nt, src, 1, width, inject_halo)
        assert np.abs(u - ref_u).max() <= 1e-12 * np.abs(ref_u).max()
