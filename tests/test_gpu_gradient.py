"""GPU squared-slowness gradient (checkpointed forward, recompute, adjoint and
imaging in the HIP library) against the FP64 oracle's exact discrete adjoint
gradient, its independence of the checkpoint interval and the schedule, the
directional derivative against FP64 finite differences of the oracle's
misfit, and the torch.autograd wrappers."""
import sys

import numpy as np
import pytest

from paper_2010_10248_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP32 fields enter the imaging sum; the Laplacian of the imaging term and the
# accumulation are FP64, so the error is that of the FP32 wavefields (about
# 1e-6 relative; the forward parity bound is 1e-5). The residual r = d - d_obs
# carries the trace error delta_d unreduced, so relative to the residual it is
# scaled by kappa = |d| / |r|, and |delta_J| <= |r| |delta_d| (+ O(delta_d^2)).
# With d_obs = 0 (kappa = 1) the bound is the forward one, 1e-5.
TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _request(seed, n, nt, so):
    rng = np.random.Generator(np.random.PCG64(seed))
    shot, vp_true = W.serving_request(rng, sizes=(n,), nt_range=(nt, nt), so=so, nbl=6)
    return shot, vp_true


def _dobs(orc, shot, vp_true, vmax):
    return orc.acoustic_forward(shot, vp=vp_true, vmax_damp=vmax)["traces"]


@pytest.mark.parametrize("so,data", [(4, "zero"), (8, "zero"), (8, "blob"), (12, "zero")])
def test_gradient_matches_oracle_and_is_schedule_independent(torch_cuda, orc, so, data):
    """d_obs = 0 (J = 1/2 |d|^2, residual = traces) at the forward tolerance;
    d_obs from a model with a +5% velocity blob at the tolerance scaled by
    the residual's conditioning kappa."""
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    shot, vp_true = _request(40 + so, 44 if so == 4 else 40, 70, so)
    vmax = float(shot.vp.max())
    if data == "zero":
        dobs = np.zeros((shot.nt, shot.rec_xyz.shape[0]))
    else:
        dobs = _dobs(orc, shot, vp_true, vmax)
    J_ref, g_ref, fw = orc.acoustic_gradient(shot, dobs, vmax_damp=vmax)
    kappa = float(np.linalg.norm(fw["traces"]) / np.linalg.norm(fw["traces"] - dobs))
    _say(f"kappa {kappa:.2f}")
    prop = tb.Acoustic(shot, damp_vmax=vmax)
    d = torch.as_tensor(dobs.astype(np.float32), device="cuda")
    base = None
    cases = [(tb.schedule("sb"), 0), (tb.schedule("tb", 2, 32), 0),
             (tb.schedule("tb", 2, 32), 1), (tb.schedule("tb", 2, 16, 9), 7),
             (tb.schedule("tb", 2, 0, 0), 5), (tb.schedule("sb"), 70),
             (tb.schedule("tb", 2, 32, 2048), 3), (None, 7)]
    if so == 4:  # depth 3 (the default there) with spacings that are not multiples of it
        cases += [(tb.schedule("tb", 3, 32), 7), (tb.schedule("tb", 3, 32, 2048), 0),
                  (tb.schedule("tb", 4, 16), 5)]
    for sc, every in cases:
        _say(f"gradient so{so} {data} {sc} checkpoint_every={every}")
        J, g = prop.gradient(d, sc, every)
        g = g.cpu().numpy()
        e = _rel(g, g_ref)
        _say(f"  J {J:.9e} oracle {J_ref:.9e} rel {abs(J - J_ref) / J_ref:.2e}  grad relL2 {e:.3e}")
        assert abs(J - J_ref) <= 2 * TOL * kappa * abs(J_ref)
        assert e <= TOL * kappa
        if base is None:
            base = g
        else:
            assert np.array_equal(g.view(np.uint32), base.view(np.uint32)), (sc, every)
    prop.close()


def test_gradient_directional_derivative_vs_oracle_fd(torch_cuda, orc):
    """<g, dm> against the FP64 central difference of the oracle's misfit
    (truncation O(eps^2), far below the tolerance)."""
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    shot, vp_true = _request(77, 40, 80, 8)
    vmax = float(shot.vp.max())
    dobs = 0.5 * _dobs(orc, shot, vp_true, vmax)
    d0 = orc.acoustic_forward(shot, vmax_damp=vmax)["traces"]
    kappa = float(np.linalg.norm(d0) / np.linalg.norm(d0 - dobs))
    prop = tb.Acoustic(shot, damp_vmax=vmax)
    _, g = prop.gradient(torch.as_tensor(dobs.astype(np.float32), device="cuda"))
    g = g.double().cpu().numpy()
    prop.close()
    m0 = 1.0 / shot.vp.astype(np.float32).astype(np.float64) ** 2
    # A smooth direction (as model updates are): 1% Gaussian bump of radius
    # 6 cells at the centre of the true model's anomaly.
    c = np.unravel_index(np.argmax(np.abs(vp_true - shot.vp)), shot.shape)
    ii = [np.arange(n, dtype=np.float64) - ci for n, ci in zip(shot.shape, c)]
    r2 = ii[0][:, None, None] ** 2 + ii[1][None, :, None] ** 2 + ii[2][None, None, :] ** 2
    dm = 0.01 * m0 * np.exp(-r2 / (2 * 6.0 ** 2))
    eps = 1e-2

    def J(m):
        fw = orc.acoustic_forward(shot, vp=1.0 / np.sqrt(m), vmax_damp=vmax)
        return orc.misfit(fw["traces"], dobs)

    fd = (J(m0 + eps * dm) - J(m0 - eps * dm)) / (2 * eps)
    lin = float(np.sum(g * dm))
    _say(f"<g, dm> {lin:.9e}  FD {fd:.9e}  rel {abs(lin - fd) / abs(fd):.2e}  kappa {kappa:.2f}")
    assert abs(lin - fd) <= 2 * TOL * kappa * abs(fd)


def test_autograd_misfit_and_modelling(torch_cuda, orc):
    torch = torch_cuda
    from paper_2010_10248_amd import autograd as AG
    from paper_2010_10248_amd import tb

    shot, vp_true = _request(91, 36, 60, 8)
    vmax = float(shot.vp.max())
    dobs = 0.5 * _dobs(orc, shot, vp_true, vmax)
    d = torch.as_tensor(dobs.astype(np.float32), device="cuda")
    m = torch.as_tensor((1.0 / shot.vp.astype(np.float32) ** 2).astype(np.float32),
                        device="cuda").requires_grad_(True)
    J = AG.misfit(m, shot, d, damp_vmax=vmax)
    J.backward()
    # The library takes m itself (c = dt^2/m): the same model built from
    # slowness2 gives the same J and gradient, and the default damping
    # velocity is the shot model's largest vp, whatever m is.
    prop = tb.Acoustic(shot, slowness2=m.detach(), damp_vmax=vmax)
    J2, g2 = prop.gradient(d)
    assert float(J) == J2
    assert torch.equal(m.grad, g2)
    m2 = (0.97 * m.detach()).requires_grad_(True)
    J3 = AG.misfit(m2, shot, d)
    J4 = AG.misfit(m2, shot, d, damp_vmax=vmax)
    assert float(J3) == float(J4)
    _, g_ref, _ = orc.acoustic_gradient(shot, dobs, vp=1.0 / np.sqrt(m.detach().double().cpu().numpy()),
                                        vmax_damp=vmax)
    assert _rel(m.grad.cpu().numpy(), g_ref) <= 2 * TOL

    # Linear modelling map q -> d: autograd's vector-Jacobian product is the
    # adjoint; dot-product test <F q, w> = <q, F^T w>.
    rng = np.random.Generator(np.random.PCG64(3))
    q = torch.as_tensor(rng.standard_normal(shot.src_wav.shape).astype(np.float32),
                        device="cuda").requires_grad_(True)
    w = torch.as_tensor(rng.standard_normal((shot.nt, shot.rec_xyz.shape[0])).astype(np.float32),
                        device="cuda")
    dq = AG.modelling(q, prop)
    (dq * w).sum().backward()
    lhs = float((dq.double() * w.double()).sum())
    rhs = float((q.detach().double() * q.grad.double()).sum())
    _say(f"modelling dot {lhs:.9e} {rhs:.9e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    prop.close()


def test_gradient_degenerate_lengths(torch_cuda, orc):
    """nt = 1 (no imaging level: zero gradient) and nt = 2 (only the source
    term of level 1)."""
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    for nt in (1, 2, 3):
        s = W.acoustic_scaled(60 + nt, (20, 22, 24), 8, nt, 2, nsrc=2, nrec=5)
        dobs = np.zeros((nt, 5))
        J_ref, g_ref, _ = orc.acoustic_gradient(s, dobs)
        prop = tb.Acoustic(s)
        J, g = prop.gradient(torch.zeros((nt, 5), device="cuda"), tb.schedule("tb", 2, 32))
        g = g.cpu().numpy()
        _say(f"nt={nt} J {J:.3e} {J_ref:.3e} |g| {np.abs(g).max():.3e} {np.abs(g_ref).max():.3e}")
        if np.abs(g_ref).max() == 0:
            assert np.all(g == 0)
        else:
            assert _rel(g, g_ref) <= TOL
        assert abs(J - J_ref) <= 2 * TOL * max(abs(J_ref), 1e-300)
        prop.close()


@pytest.mark.parametrize("n", [128, 192, 256, 384])
def test_served_sizes_gradient_sample(torch_cuda, orc, n):
    """One request of each served grid size at the smallest served length
    (nt = 500; SO8, sponge 20, two-layer model, one source near the top, a
    receiver line at its depth). Observed data: half the FP64 oracle's traces
    of the model with the +5% velocity blob. (The blob's own data would leave
    a residual below FP32 resolution wherever its reflection has not reached
    the line within 500 steps, kappa up to 1e16; halving them keeps kappa
    near 2, so the bound stays the forward tolerance.) At 128^3 and 192^3
    the whole gradient is compared with the oracle's (the oracle keeps every
    forward level); at 256^3 and 384^3, where that history would take 67 and
    227 GB of host memory, the directional derivative <g, dm> along a smooth
    bump 8 cells below the source is compared with the FP64 central
    difference of the oracle's misfit."""
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    rng = np.random.Generator(np.random.PCG64(10253 + n))
    shot, vp_true = W.serving_request(rng, sizes=(n,), nt_range=(500, 500))
    vmax = float(shot.vp.max())
    _say(f"served size {n}^3 nt={shot.nt}: oracle data")
    dobs = 0.5 * _dobs(orc, shot, vp_true, vmax)
    prop = tb.Acoustic(shot, damp_vmax=vmax)
    J, g = prop.gradient(torch.as_tensor(dobs.astype(np.float32), device="cuda"))
    g = g.double().cpu().numpy()
    prop.close()
    if n <= 192:
        J_ref, g_ref, fw = orc.acoustic_gradient(shot, dobs, vmax_damp=vmax)
        kappa = float(np.linalg.norm(fw["traces"]) / np.linalg.norm(fw["traces"] - dobs))
        e = _rel(g, g_ref)
        _say(f"  {n}^3: kappa {kappa:.2f}  J {J:.9e} oracle {J_ref:.9e}  grad relL2 {e:.3e}")
        assert kappa < 3.0
        assert abs(J - J_ref) <= 2 * TOL * kappa * abs(J_ref)
        assert e <= TOL * kappa
        return
    m0 = 1.0 / shot.vp.astype(np.float32).astype(np.float64) ** 2
    c = shot.src_xyz[0] / np.array(shot.spacing) + np.array([0.0, 0.0, 8.0])
    ii = [np.arange(k, dtype=np.float64) - ci for k, ci in zip(shot.shape, c)]
    r2 = ii[0][:, None, None] ** 2 + ii[1][None, :, None] ** 2 + ii[2][None, None, :] ** 2
    dm = 0.01 * m0 * np.exp(-r2 / (2 * 6.0 ** 2))
    eps = 1e-2
    Js = []
    for sgn in (1.0, -1.0, 0.0):
        _say(f"  {n}^3: oracle forward at m0 + {sgn * eps} dm")
        fw = orc.acoustic_forward(shot, vp=1.0 / np.sqrt(m0 + sgn * eps * dm), vmax_damp=vmax)
        Js.append(orc.misfit(fw["traces"], dobs))
    kappa = float(np.linalg.norm(fw["traces"]) / np.linalg.norm(fw["traces"] - dobs))
    fd = (Js[0] - Js[1]) / (2 * eps)
    lin = float(np.sum(g * dm))
    _say(f"  {n}^3: kappa {kappa:.2f}  J {J:.9e} oracle {Js[2]:.9e}  <g, dm> {lin:.9e} "
         f"FD {fd:.9e} rel {abs(lin - fd) / abs(fd):.2e}")
    assert kappa < 3.0
    assert abs(J - Js[2]) <= 2 * TOL * kappa * abs(Js[2])
    assert abs(lin - fd) <= 2 * TOL * kappa * abs(fd)
