"""The x-streaming TTI and elastic kernels on grids smaller than their tiles
and stencils: fewer x planes than the stencil radius (every plane of the
grid lies in the window warm-up of its chunk), fewer rows than a tile's y
halo, fewer z than one lane row, and z padding. Parity of the one-step
schedule with the FP64 oracles (relative L2 <= 1e-5 on the last two levels,
and on the traces where they carry signal above FP32 noise of the field),
and the temporally blocked schedules bitwise equal to it."""
import sys

import numpy as np
import pytest

from paper_2010_10248_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5
SHAPES = [(7, 19, 9), (5, 3, 70), (3, 33, 6)]


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


def _check(torch, prop, errs, trace_pairs, field_peak, tag):
    for got, ref in trace_pairs:
        if np.abs(ref).max() > 1e-4 * field_peak:
            errs["traces"] = max(errs.get("traces", 0.0), _rel(got, ref))
    print(f"{tag}: {errs}", flush=True)
    sys.stdout.flush()
    assert all(v <= TOL for v in errs.values()), errs


def _tb_bitwise(torch, prop, base):
    from paper_2010_10248_amd import tb

    for T, w in ((2, 1), (2, 4), (3, 2)):
        out = prop.forward(tb.schedule("tb", T, 0, w))
        for k in ("traces", "u_last", "u_prev"):
            assert torch.equal(out[k].view(torch.int32), base[k].view(torch.int32)), (T, w, k)


@pytest.mark.parametrize("so", [8, 4])
@pytest.mark.parametrize("n", SHAPES)
def test_tti_small_grids(torch_cuda, orc, so, n):
    from paper_2010_10248_amd import tb

    s = W.tti_smooth(seed=11, n=n, so=so, nt=40, nbl=1, nsrc=1, nrec=6, sigma=2.0)
    ref = orc.tti_forward(s)
    prop = tb.Propagator(s)
    base = prop.forward(tb.schedule("sb"))
    got = {k: v.cpu().numpy() for k, v in base.items()}
    errs = dict(p_last=_rel(got["u_last"], ref["p_last"]), p_prev=_rel(got["u_prev"], ref["p_prev"]))
    _check(torch_cuda, prop, errs, [(got["traces"], ref["traces"])],
           float(np.abs(ref["p_last"]).max()), f"TTI SO{so} {n}")
    _tb_bitwise(torch_cuda, prop, base)
    prop.close()


@pytest.mark.parametrize("so", [8, 4])
@pytest.mark.parametrize("n", SHAPES)
def test_elastic_small_grids(torch_cuda, orc, so, n):
    from paper_2010_10248_amd import tb

    s = W.elastic_smooth(seed=11, n=n, so=so, nt=40, nbl=1, nrec=6, sigma=2.0)
    ref = orc.elastic_forward(s)
    prop = tb.Propagator(s)
    base = prop.forward(tb.schedule("sb"))
    got = {k: v.cpu().numpy() for k, v in base.items()}
    errs = dict(vz_field=_rel(got["u_last"], ref["vz_field"]), tzz=_rel(got["u_prev"], ref["tzz"]))
    tr = got["traces"]
    _check(torch_cuda, prop, errs, [(tr[0], ref["vz"]), (tr[1], ref["p"])],
           float(np.abs(ref["tzz"]).max()), f"elastic SO{so} {n}")
    _tb_bitwise(torch_cuda, prop, base)
    prop.close()
