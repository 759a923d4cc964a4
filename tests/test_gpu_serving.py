"""Serving runtime and autotuner on the GPU: every request's results are
bit-identical alone (tb_forward / tb_gradient) and in a continuously batched
mix of grid sizes, space orders and request kinds, with admission limited by
slots and by arena memory, with and without hipGraph replay; the autotuned
schedule gives the same bits as any other."""
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


def _requests():
    """Mixed kinds and sizes: forward shots and gradients, SO8 and SO4."""
    out = []
    for k, (n, nt, so, kind) in enumerate([(36, 40, 8, "fwd"), (40, 46, 8, "grad"),
                                           (44, 52, 4, "fwd"), (32, 37, 8, "grad"),
                                           (48, 30, 8, "fwd"), (40, 41, 4, "grad"),
                                           (28, 25, 8, "fwd")]):
        rng = np.random.Generator(np.random.PCG64(500 + k))
        shot, vp_true = W.serving_request(rng, sizes=(n,), nt_range=(nt, nt), so=so, nbl=5)
        out.append((kind, shot, vp_true))
    return out


def _alone(torch, tb, reqs, sched):
    res = []
    props = []
    for kind, shot, vp_true in reqs:
        prop = tb.Acoustic(shot)
        props.append(prop)
        if kind == "fwd":
            res.append(("fwd", prop.forward(sched, want_fields=False)["traces"].clone(), None))
        else:
            dobs = torch.as_tensor(
                np.random.Generator(np.random.PCG64(shot.nt)).standard_normal(
                    (shot.nt, shot.rec_xyz.shape[0])).astype(np.float32) * 1e-3, device="cuda")
            J, g = prop.gradient(dobs, sched, 5)
            res.append(("grad", g.clone(), (J, dobs)))
    torch.cuda.synchronize()
    return props, res


@pytest.mark.parametrize("graphs", [True, False])
def test_alone_vs_mix_bit_identical(torch_cuda, graphs):
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    reqs = _requests()
    sched = tb.schedule("tb", 2, 32)
    props, alone = _alone(torch, tb, reqs, sched)
    # Arena for about two of the largest requests: admission waits for memory.
    need = max(tb.gradient_workspace_size(p.model, p.sparse, sched, 5) for p in props)
    sv = tb.Server(arena_bytes=int(2.2 * need), max_active=3, graphs=graphs)
    outs = {}
    pending = {}

    def submit(i):
        kind, shot, _ = reqs[i]
        p = props[i]
        if kind == "fwd":
            o = torch.full((shot.nt, p.nrec), float("nan"), device="cuda")
            rid = sv.submit_forward(p, o, sched)
        else:
            o = torch.full(shot.shape, float("nan"), device="cuda")
            rid = sv.submit_gradient(p, alone[i][2][1], o, sched, 5)
        outs[i] = o
        pending[rid] = i

    # Staggered arrivals: requests join while others are on the device.
    for i in range(3):
        submit(i)
    done = {}
    nxt = 3
    it = 0
    while len(done) < len(reqs):
        act, q = sv.step()
        for rid, loss in sv.poll():
            done[pending[rid]] = loss
        if nxt < len(reqs) and it % 3 == 2:
            submit(nxt)
            nxt += 1
        it += 1
        assert it < 100000
    st = sv.stats()
    _say(f"graphs={graphs} stats {st}")
    sv.close()
    for i, (kind, ref, extra) in enumerate(alone):
        got = outs[i]
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), (i, kind)
        if kind == "grad":
            assert done[i] == extra[0], (i, done[i], extra[0])
    assert st["completed"] == len(reqs)
    assert st["passes_batched"] > st["launches"]  # several jobs per launch
    if graphs:
        assert st["graph_replays"] > st["graph_captures"] > 0
    for p in props:
        p.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_dense_source_request_in_mix(torch_cuda, graphs):
    """A request with a thousand sources in the volume needs the global-list
    kernel for some passes; those run as launches of their own beside the
    batched launches of the other requests, with the same bits as alone."""
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    dense = W.acoustic_source_density(1000, "volume", n=(48, 56, 64), nt=40, nbl=6)
    reqs = [("fwd", dense, None)] + [r for r in _requests() if r[0] == "fwd"][:2]
    sched = tb.schedule("tb", 2, 32, 64)
    props, alone = _alone(torch, tb, reqs, sched)
    sv = tb.Server(arena_bytes=8 << 30, max_active=3, graphs=graphs)
    outs, pending = {}, {}
    for i, (kind, shot, _) in enumerate(reqs):
        o = torch.full((shot.nt, props[i].nrec), float("nan"), device="cuda")
        pending[sv.submit_forward(props[i], o, sched)] = i
        outs[i] = o
    done = set()
    it = 0
    while len(done) < len(reqs):
        sv.step()
        for rid, _ in sv.poll():
            done.add(pending[rid])
        it += 1
        assert it < 100000
    st = sv.stats()
    _say(f"dense mix graphs={graphs} stats {st}")
    sv.close()
    for i, (_, ref, _) in enumerate(alone):
        assert torch.equal(outs[i].view(torch.int32), ref.view(torch.int32)), i
    assert st["completed"] == len(reqs)
    for p in props:
        p.close()


def test_so12_request_in_mix(torch_cuda):
    """A space-order-12 shot at T = 2 (a shape that only the global-list
    kernel runs, so it gets launches of its own) and a gradient at space
    order 12 served beside space-order-8 shots: bits as alone."""
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    reqs = []
    for k, (n, nt, so, kind) in enumerate([(40, 33, 12, "fwd"), (36, 40, 8, "fwd"),
                                           (34, 29, 12, "grad"), (44, 35, 8, "fwd")]):
        rng = np.random.Generator(np.random.PCG64(900 + k))
        shot, vp_true = W.serving_request(rng, sizes=(n,), nt_range=(nt, nt), so=so, nbl=5)
        reqs.append((kind, shot, vp_true))
    sched = tb.schedule("tb", 2, 32)
    props, alone = _alone(torch, tb, reqs, sched)
    sv = tb.Server(arena_bytes=4 << 30, max_active=4)
    outs, pending = {}, {}
    for i, (kind, shot, _) in enumerate(reqs):
        if kind == "fwd":
            o = torch.full((shot.nt, props[i].nrec), float("nan"), device="cuda")
            rid = sv.submit_forward(props[i], o, sched)
        else:
            o = torch.full(shot.shape, float("nan"), device="cuda")
            rid = sv.submit_gradient(props[i], alone[i][2][1], o, sched, 5)
        outs[i] = o
        pending[rid] = i
    done = {}
    it = 0
    while len(done) < len(reqs):
        sv.step()
        for rid, loss in sv.poll():
            done[pending[rid]] = loss
        it += 1
        assert it < 100000
    st = sv.stats()
    _say(f"so12 mix stats {st}")
    sv.close()
    for i, (kind, ref, extra) in enumerate(alone):
        assert torch.equal(outs[i].view(torch.int32), ref.view(torch.int32)), (i, kind)
        if kind == "grad":
            assert done[i] == extra[0]
    for p in props:
        p.close()


def test_server_rejects_oversized_request(torch_cuda):
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(3, (64, 64, 64), 8, 10, 2, nsrc=1, nrec=4)
    p = tb.Acoustic(s)
    assert tb.workspace_size(p.model, p.sparse, None) > 1 << 20  # 4 fields of 1 MiB
    sv = tb.Server(arena_bytes=1 << 20, max_active=2)
    with pytest.raises(tb.TbError) as e:
        sv.submit_forward(p, torch.empty((10, 4), device="cuda"))
    assert e.value.status == tb.EWORKSPACE
    sv.close()
    p.close()


def test_autotune_choice_is_bit_identical(torch_cuda):
    torch = torch_cuda
    from paper_2010_10248_amd import tb

    s = W.acoustic_scaled(4, (64, 72, 80), 8, 24, 6, nsrc=2, nrec=12, layered=True)
    p = tb.Acoustic(s)
    ref = p.forward(tb.schedule("sb"))
    best, ms = tb.autotune(p.model, p.sparse, steps=6)
    _say(f"tuned {best} {ms:.4f} ms/step")
    assert best.time_tile >= 1 and ms > 0
    got = p.forward(None)  # resolves to the tuned choice
    for k in ("traces", "u_last", "u_prev"):
        assert torch.equal(got[k].view(torch.int32), ref[k].view(torch.int32)), k
    tb.autotune_clear()
    p.close()
