"""The forward entry point that allocates nothing (tb_forward_noalloc: the
library's fixed device workspace in place of caller memory) against
tb_forward through the C ABI: bitwise equal outputs on two calls in a row,
the second on a smaller grid (the array keeps the first call's contents),
for acoustic schedules and a TTI model; its refusals (lists not built yet,
a run beyond the fixed size)."""
import sys

import numpy as np
import pytest

from paper_2010_10248_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _outs(torch, prop):
    nt, nrec = prop.shot.nt, prop.nrec
    return (torch.full((nt, nrec), float("nan"), device="cuda"),
            torch.full(prop.shot.shape, float("nan"), device="cuda"),
            torch.full(prop.shot.shape, float("nan"), device="cuda"))


def _same(a, b):
    return all(np.array_equal(x.cpu().numpy().view(np.uint32), y.cpu().numpy().view(np.uint32))
               for x, y in zip(a, b))


def test_noalloc_equals_forward_on_two_calls(torch_cuda):
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    big = W.acoustic_scaled(301, (64, 64, 64), 8, 60, 8, nsrc=3, nrec=24, layered=True)
    small = W.acoustic_scaled(302, (36, 40, 44), 4, 50, 5, nsrc=2, nrec=10, layered=True)
    for shot, sched in ((big, tb.schedule("tb", 2, 32, 0)), (small, tb.schedule("tb", 3, 32, 0)),
                        (small, tb.schedule("sb")), (big, None)):
        _say(f"noalloc {shot.shape} SO{shot.space_order} {sched}")
        prop = tb.Acoustic(shot)
        ref = prop.forward(sched)
        rec, u, up = _outs(torch, prop)
        tb.forward_noalloc(prop.model, prop.sparse, sched, rec, u, up)
        torch.cuda.synchronize()
        assert _same((rec, u, up), (ref["traces"], ref["u_last"], ref["u_prev"]))
        assert float(ref["u_last"].abs().max()) > 0
        prop.close()


def test_noalloc_tti(torch_cuda):
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    s = W.tti_smooth(seed=303, n=(30, 34, 38), so=8, nt=40, nbl=5, nsrc=2, nrec=8, sigma=3.0)
    prop = tb.Propagator(s)
    ref = prop.forward(None)
    rec, u, up = _outs(torch, prop)
    tb.forward_noalloc(prop.model, prop.sparse, None, rec, u, up)
    torch.cuda.synchronize()
    assert _same((rec, u, up), (ref["traces"], ref["u_last"], ref["u_prev"]))
    prop.close()


def test_noalloc_refusals(torch_cuda):
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(304, (40, 40, 40), 8, 20, 4, nsrc=1, nrec=4, layered=True)
    prop = tb.Acoustic(s)
    rec, u, up = _outs(torch, prop)
    # No tb_forward with this schedule yet: its tile lists are not built.
    with pytest.raises(tb.TbError) as e:
        tb.forward_noalloc(prop.model, prop.sparse, tb.schedule("tb", 2, 16, 0), rec, u, up)
    assert e.value.status == tb.EINVAL and "not built" in str(e.value)
    prop.close()
    # 160^3 needs five 15.6 MiB fields plus the receiver rows: above 64 MiB.
    s = W.acoustic_scaled(305, (160, 160, 160), 8, 4, 4, nsrc=1, nrec=4, layered=True)
    prop = tb.Acoustic(s)
    with pytest.raises(tb.TbError) as e:
        tb.forward_noalloc(prop.model, prop.sparse, None)
    assert e.value.status == tb.EWORKSPACE
    prop.close()
