"""GPU parity of the acoustic propagator: HIP path vs the FP64 oracle
(relative L2 <= 1e-5 on traces and the last two wavefields), bit-identity of
every temporally blocked schedule with the spatially blocked one, and the
C-ABI error paths that need a device."""
import sys

import numpy as np
import pytest

from paper_2010_10248_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(tb, prop, sched):
    out = prop.forward(sched)
    import torch

    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# Time tiles of 3 and 4 exist at space order 4 only (4 with 16-row tiles).
# chunk_x 2048 streams whole x per tile, with the tails of the tiles on the
# spare workgroups.
SCHEDS = [("sb", 1, 32, 0), ("sb", 1, 16, 24), ("tb", 2, 32, 0), ("tb", 2, 16, 0),
          ("tb", 3, 16, 0), ("tb", 4, 16, 40), ("tb", 2, 32, 24), ("tb", 3, 16, 17),
          ("tb", 2, 0, 0), ("tb", 2, 32, 2048), ("sb", 1, 32, 2048), ("tb", 3, 32, 2048),
          ("tb", 3, 32, 24)]


def _check_case(torch_cuda, orc, shot, scheds=SCHEDS, tol=TOL):
    from paper_2010_10248_amd import tb

    ref = orc.acoustic_forward(shot)
    prop = tb.Acoustic(shot)
    base = None
    for mode, T, by, ch in scheds:
        if shot.space_order == 8 and T >= 3:
            continue
        sc = tb.schedule(mode, T, by, ch)
        _say(f"case {shot.name} sched {sc}")
        out = _run(tb, prop, sc)
        e_tr = _rel(out["traces"], ref["traces"])
        e_u = _rel(out["u_last"], ref["u_last"])
        e_up = _rel(out["u_prev"], ref["u_prev"])
        _say(f"  relL2 traces {e_tr:.3e} u {e_u:.3e} u_prev {e_up:.3e}")
        assert e_tr <= tol and e_u <= tol and e_up <= tol, (sc, e_tr, e_u, e_up)
        if base is None:
            base = out
        else:
            for k in ("traces", "u_last", "u_prev"):
                assert np.array_equal(out[k].view(np.uint32), base[k].view(np.uint32)), (sc, k)
    prop.close()


def test_parity_small_constant_so4(torch_cuda, orc):
    """64^3, h=10 m, SO4, nbl 10, 100 steps, one off-grid Ricker, 32 receivers."""
    _check_case(torch_cuda, orc, W.acoustic_small())


def test_parity_two_layer_so8_ragged(torch_cuda, orc):
    """SO8 two-layer model on a ragged grid (nz not a multiple of 4, nx not a
    multiple of any chunk), several sources and a receiver line."""
    s = W.acoustic_scaled(21, (61, 75, 70), 8, 60, 8, nsrc=3, nrec=24, layered=True)
    _check_case(torch_cuda, orc, s)


def test_sources_on_tile_boundaries(torch_cuda, orc):
    """Sources and receivers placed on the y/z tile seams and x-chunk seams of
    the schedules, where a halo copy must receive the same injection (the
    violation of the paper's Fig. 4b)."""
    s = W.acoustic_scaled(5, (72, 96, 128), 8, 40, 6, nsrc=4, nrec=16, layered=True)
    h = s.spacing[0]
    # T=2, tile_y=32: owned rows per tile 24, halo 4; owned columns 56.
    s.src_xyz[0] = np.array([23.5, 23.5, 55.5]) * h
    s.src_xyz[1] = np.array([24.0, 47.7, 56.2]) * h
    s.src_xyz[2] = np.array([39.9, 19.6, 59.9]) * h   # inside a y halo
    s.src_xyz[3] = np.array([40.2, 72.1, 111.6]) * h
    s.rec_xyz[:4] = s.src_xyz[:4] + 0.25 * h
    _check_case(torch_cuda, orc, s, scheds=[("sb", 1, 32, 0), ("tb", 2, 32, 24), ("tb", 2, 32, 0),
                                            ("tb", 2, 0, 40), ("tb", 2, 16, 17)])


def test_parity_so12(torch_cuda, orc):
    """Space order 12 (radius 6, two float4 of z neighbours on each side): a
    ragged two-layer case with sources on the z seams of the 16-lane tiles;
    spatial blocking and T = 2 (whose 32-row tile fits LDS only without the
    staged lists, so the global-list kernel runs it)."""
    s = W.acoustic_scaled(31, (57, 62, 70), 12, 50, 6, nsrc=3, nrec=16, layered=True)
    h = s.spacing[0]
    s.src_xyz[0] = np.array([20.5, 30.25, 47.5]) * h   # T=2 z seam (owned 48 per tile)
    s.src_xyz[1] = np.array([36.7, 19.6, 8.2]) * h     # inside the z halo of a tile
    s.rec_xyz[:2] = s.src_xyz[:2] + 0.3 * h
    _check_case(torch_cuda, orc, s, scheds=[("sb", 1, 32, 0), ("sb", 1, 16, 24), ("tb", 2, 32, 0),
                                            ("tb", 2, 32, 24), ("tb", 2, 16, 0), ("tb", 2, 0, 17)])


def test_zero_source_is_exactly_zero(torch_cuda):
    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(8, (40, 44, 48), 8, 30, 5, nsrc=2, nrec=8)
    prop = tb.Acoustic(s, src_wav=np.zeros_like(s.src_wav))
    for sc in (tb.schedule("sb"), tb.schedule("tb", 2, 16)):
        out = _run(tb, prop, sc)
        for k in ("traces", "u_last", "u_prev"):
            assert np.all(out[k].view(np.uint32) == 0), (sc, k)
    prop.close()


def test_tiny_and_degenerate_grids(torch_cuda, orc):
    """Grids smaller than one tile, a single plane of sources at the grid
    edge (x = 0, z = nz-1) and nt = 1 / nt = T - 1."""
    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(9, (9, 13, 6), 4, 7, 0, nsrc=2, nrec=3, layered=False)
    s.src_xyz[0] = [0.0, 40.0, 50.0]
    s.src_xyz[1] = [80.0, 120.0, 50.0]
    _check_case(torch_cuda, orc, s, scheds=[("sb", 1, 16, 0), ("tb", 2, 16, 0), ("tb", 3, 16, 4),
                                            ("tb", 4, 16, 0)])
    for nt in (1, 2):
        s2 = W.acoustic_scaled(10, (20, 18, 24), 8, nt, 2, nsrc=1, nrec=2)
        _check_case(torch_cuda, orc, s2, scheds=[("sb", 1, 32, 0), ("tb", 2, 32, 0)])


def test_error_paths_on_device(torch_cuda):
    import torch

    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(12, (24, 24, 24), 8, 10, 2, nsrc=1, nrec=2)
    vp = torch.as_tensor(s.vp.astype(np.float32), device="cuda")
    with pytest.raises(tb.TbError) as e:
        tb.create_model(s.shape, s.spacing, s.origin, 8, 2, s.dt * 1.2, 10, vp)
    assert e.value.status == tb.EUNSTABLE
    m = tb.create_model(s.shape, s.spacing, s.origin, 8, 2, s.dt, 10, vp)
    with pytest.raises(tb.TbError) as e:
        tb.inspect_sparse(m, [[0.0, 0.0, 231.0]], s.src_wav, s.rec_xyz)
    assert e.value.status == tb.ERANGE
    sp = tb.inspect_sparse(m, s.src_xyz, s.src_wav, s.rec_xyz)
    need = tb.workspace_size(m, sp, None)
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    rec = torch.empty((10, 2), device="cuda")
    with pytest.raises(tb.TbError) as e:
        tb.forward(m, sp, None, ws, rec)
    assert e.value.status == tb.EWORKSPACE
    with pytest.raises(tb.TbError) as e:
        tb.forward(m, sp, tb.schedule("tb", 4, 16), torch.empty(need * 2, dtype=torch.uint8,
                                                               device="cuda"), rec)
    assert e.value.status == tb.EUNSUPPORTED
    tb.destroy_sparse(sp)
    tb.destroy_model(m)


@pytest.mark.parametrize("so", [4, 8])
def test_adjoint_dot_product_and_oracle(torch_cuda, orc, so):
    import torch

    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(31, (40, 46, 52), so, 50, 5, nsrc=3, nrec=12, layered=True)
    rng = np.random.Generator(np.random.PCG64(4))
    q = rng.standard_normal(s.src_wav.shape)
    dp = rng.standard_normal((s.nt, s.rec_xyz.shape[0]))
    prop = tb.Acoustic(s, src_wav=q)
    scheds = [tb.schedule("sb"), tb.schedule("tb", 2, 32), tb.schedule("tb", 2, 16, 20),
              tb.schedule("tb", 2, 32, 2048), None]
    if so == 4:  # three steps per pass (the space-order-4 default) and four
        scheds += [tb.schedule("tb", 3, 32), tb.schedule("tb", 4, 16, 20)]
    for sc in scheds:
        _say(f"adjoint so{so} {sc}")
        Fq = prop.forward(sc)["traces"].double().cpu().numpy()
        FTd = prop.adjoint(torch.as_tensor(dp.astype(np.float32), device="cuda"), sc)
        FTd = FTd.double().cpu().numpy()
        lhs = float(np.sum(Fq * dp))
        rhs = float(np.sum(q * FTd))
        _say(f"  dot {lhs:.9e} {rhs:.9e} rel {abs(lhs - rhs) / abs(lhs):.2e}")
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
        ref = orc.acoustic_adjoint(s, dp)["qhat"]
        assert _rel(FTd, ref) <= TOL
    prop.close()


def test_full_size_c2_first_steps_and_schedule_identity(torch_cuda, orc):
    """The 512^3 SO8 two-layer workload (8 sources, 512 receivers) in the
    launch configurations the benchmark times: the first 8 steps against the
    FP64 oracle on the full grid (every tile seam, chunk seam and source
    placement of the real shape), then the full 1000-step run bitwise
    identical between the temporally and spatially blocked schedules."""
    import torch

    from paper_2010_10248_amd import tb

    tb_s, sb_s = tb.schedule("tb", 2, 32, 2048), tb.schedule("sb", 1, 32, 0)
    tb_c = tb.schedule("tb", 2, 32, 64)
    s8 = W.acoustic_two_layer(n=512, nt=8)
    ref = orc.acoustic_forward(s8)
    prop = tb.Acoustic(s8)
    for sc in (tb_s, sb_s, tb_c):
        out = _run(tb, prop, sc)
        e = (_rel(out["u_last"], ref["u_last"]), _rel(out["u_prev"], ref["u_prev"]))
        _say(f"512^3 first 8 steps {sc}: relL2 u {e[0]:.3e} u_prev {e[1]:.3e}")
        assert max(e) <= TOL
    prop.close()
    del ref
    s = W.acoustic_two_layer(n=512, nt=1000)
    prop = tb.Acoustic(s)
    a = prop.forward(tb_s)
    b = prop.forward(sb_s)
    torch.cuda.synchronize()
    for k in ("traces", "u_last", "u_prev"):
        assert torch.equal(a[k].view(torch.int32), b[k].view(torch.int32)), k
    assert float(a["traces"].abs().max()) > 0
    del b
    c = prop.forward(tb_c)
    torch.cuda.synchronize()
    for k in ("traces", "u_last", "u_prev"):
        assert torch.equal(a[k].view(torch.int32), c[k].view(torch.int32)), k
    prop.close()


def test_c2_recipe_full_length_reduced_grid(torch_cuda, orc):
    """The two-layer SO8 recipe with all 1000 steps on a 192^3 grid (8
    sources, 512 receivers): traces and final fields against the oracle."""
    s = W.acoustic_two_layer(n=192, nt=1000)
    _check_case(torch_cuda, orc, s, scheds=[("tb", 2, 32, 64), ("sb", 1, 32, 0), ("tb", 2, 0, 0),
                                            ("tb", 2, 32, 2048)])


def test_long_segments_dense_receiver_line(torch_cuda, orc):
    """Whole-x segments on a long x axis with a dense receiver line (600
    receivers over 320 planes, four nodes per plane): a segment on the line
    holds more receiver entries than the smallest LDS list, fewer than the
    32-row two-step shape stages; parity with the oracle and bitwise identity
    with chunked and spatially blocked schedules."""
    s = W.acoustic_two_layer(seed=41, n=(320, 40, 48), nt=60, nbl=6, nrec=600)
    _check_case(torch_cuda, orc, s, scheds=[("sb", 1, 32, 0), ("tb", 2, 32, 2048),
                                            ("sb", 1, 32, 2048), ("tb", 2, 32, 64),
                                            ("tb", 2, 16, 2048)])


@pytest.mark.parametrize("layout", ["plane", "volume"])
def test_dense_sources(torch_cuda, orc, layout):
    """A thousand sources (Section IV-E), on one plane of the tiles and
    uniform in the volume: segments whose lists exceed the LDS capacities run
    the global-list kernel; parity with the oracle and bitwise identity of
    the schedules."""
    s = W.acoustic_source_density(1000, layout, n=(48, 56, 64), nt=40, nbl=6)
    _check_case(torch_cuda, orc, s, scheds=[("sb", 1, 32, 0), ("tb", 2, 32, 64), ("tb", 2, 32, 0),
                                            ("tb", 2, 16, 8)])


def test_dense_x_plane_runs_the_global_list_kernel(torch_cuda, orc):
    """2000 sources on one x-plane of a 40x40x64 grid: the corner planes
    hold ~2000 injection entries per tile, more than the 1024 a segment can
    stage in LDS even for a single plane, so those passes run the variant
    that walks the lists in global memory; parity with the oracle and
    bitwise identity with the other schedules."""
    s = W.acoustic_two_layer(seed=77, n=(40, 40, 64), nt=30, nbl=4, nsrc=1, nrec=16)
    rng = np.random.Generator(np.random.PCG64(78))
    k = 2000
    src = np.empty((k, 3))
    src[:, 0] = 20.3 * s.spacing[0]
    src[:, 1] = rng.uniform(5, 34, k) * s.spacing[1]
    src[:, 2] = rng.uniform(5, 58, k) * s.spacing[2]
    s.src_xyz = src
    s.src_wav = np.stack([W.ricker(10.0 + 0.001 * i, s.nt, s.dt) for i in range(k)], axis=1)
    _check_case(torch_cuda, orc, s, scheds=[("sb", 1, 32, 0), ("tb", 2, 32, 2048),
                                            ("tb", 2, 32, 64), ("sb", 1, 16, 2048)])


def test_full_size_c2_all_steps(torch_cuda, orc):
    """The 512^3 SO8 two-layer workload over all 1000 steps in the launch
    configurations the benchmark times: TB (whole x) bitwise equal to SB, and
    traces and final fields against the FP64 oracle."""
    from paper_2010_10248_amd import tb

    s = W.acoustic_two_layer(n=512, nt=1000)
    prop = tb.Acoustic(s)
    a = _run(tb, prop, tb.schedule("tb", 2, 32, 2048))
    b = _run(tb, prop, tb.schedule("sb", 1, 16, 2048))
    prop.close()
    for k in ("traces", "u_last", "u_prev"):
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k
    _say("512^3 1000 steps: TB == SB bitwise; running the oracle")
    ref = orc.acoustic_forward(s)
    e = {k: _rel(a[k], ref[k]) for k in ("traces", "u_last", "u_prev")}
    _say(f"512^3 1000 steps vs oracle: {e}")
    assert np.abs(ref["traces"]).max() > 0
    assert all(v <= TOL for v in e.values()), e


@pytest.mark.parametrize("so", [4, 8])
def test_default_schedule_is_bitwise_sb(torch_cuda, so):
    """A NULL schedule (three steps per pass at space order 4, two at 8, with
    whole x where the tiles fill the CUs) gives the spatially blocked bits."""
    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(31 + so, (96, 70, 130), so, 40, 6, nsrc=2, nrec=20, layered=True)
    prop = tb.Acoustic(s)
    a = _run(tb, prop, None)
    b = _run(tb, prop, tb.schedule("sb"))
    prop.close()
    for k in ("traces", "u_last", "u_prev"):
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k
    assert np.abs(a["u_last"]).max() > 0
