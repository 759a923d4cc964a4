"""Work decomposition of the acoustic schedules (Section II-B's loop nest as
the kernel runs it), checked on the host through tb_schedule_segments_host:
every tile's x range is covered exactly once, chunks respect their length,
the whole-x schedule puts one head per tile on its own workgroup and the
tails on the spare ones with the split point balancing the two, and the
error paths."""
import numpy as np
import pytest

from paper_2010_10248_amd import tb


def _tiles(shape, tile):
    rows, zw, oy, oz = tile
    return -(-shape[1] // oy), -(-shape[2] // oz)


def _check_partition(shape, tile, segs):
    ty, tz = _tiles(shape, tile)
    cover = {}
    for w, a, b, xs, xe in segs:
        assert 0 <= a < ty and 0 <= b < tz and 0 <= xs < xe <= shape[0], (w, a, b, xs, xe)
        cover.setdefault((a, b), []).append((xs, xe))
    assert len(cover) == ty * tz
    for key, iv in cover.items():
        iv.sort()
        assert iv[0][0] == 0 and iv[-1][1] == shape[0], key
        for (_, e0), (s1, _) in zip(iv, iv[1:]):
            assert e0 == s1, (key, iv)


CASES = [((96, 70, 130), 8, ("tb", 2, 32, 64), 256),
         ((96, 70, 130), 8, ("tb", 2, 32, 2048), 256),
         ((96, 70, 130), 8, ("tb", 2, 32, 0), 512),
         ((300, 41, 77), 4, ("tb", 4, 16, 40), 256),
         ((300, 41, 77), 4, ("sb", 1, 16, 2048), 256),
         ((512, 512, 512), 8, ("tb", 2, 32, 2048), 256),
         ((512, 512, 512), 8, ("tb", 2, 32, 64), 256),
         ((512, 512, 512), 12, ("tb", 2, 32, 2048), 256),
         ((33, 5, 9), 12, ("sb", 1, 32, 7), 16),
         ((1, 1, 1), 8, ("tb", 2, 0, 2048), 256)]


@pytest.mark.parametrize("shape,so,sched,wgs", CASES)
def test_segments_cover_every_tile_once(shape, so, sched, wgs):
    tile, segs = tb.schedule_segments(shape, so, tb.schedule(*sched), wgs)
    _check_partition(shape, tile, segs)
    rows, zw, oy, oz = tile
    R, T = so // 2, sched[1]
    assert zw == 64 and oy == rows - 2 * R * (T - 1) and oz == 64 - 2 * (-(-R * (T - 1) // 4) * 4)
    chunk = sched[3]
    if 0 < chunk < shape[0]:
        assert np.all(segs[:, 4] - segs[:, 3] <= min(chunk, 1024))
    # Workgroups in launch order, none idle.
    w = segs[:, 0]
    assert np.all(np.diff(w) >= 0) and set(w.tolist()) == set(range(int(w.max()) + 1))


@pytest.mark.parametrize("shape,so", [((512, 512, 512), 8), ((200, 96, 120), 8),
                                      ((130, 50, 70), 4)])
def test_whole_x_heads_and_tails(shape, so):
    wgs = 256
    tile, segs = tb.schedule_segments(shape, so, tb.schedule("tb", 2, 32, 2048), wgs)
    ty, tz = _tiles(shape, tile)
    nt = ty * tz
    assert nt < wgs
    heads = segs[:nt]
    # Tile t's head [0, s) on workgroup t, all with the same split point.
    assert np.array_equal(heads[:, 0], np.arange(nt))
    assert np.array_equal(heads[:, 1] * tz + heads[:, 2], np.arange(nt))
    assert np.all(heads[:, 3] == 0)
    s = int(heads[0, 4])
    assert np.all(heads[:, 4] == s) and 0 < s < shape[0]
    tails = segs[nt:]
    assert len(tails) == nt and np.all(tails[:, 3] == s) and np.all(tails[:, 4] == shape[0])
    ns = min(wgs - nt, nt)
    assert set(tails[:, 0].tolist()) == set(range(nt, nt + ns))
    # Balance: a head streams s + RT planes, a spare k tails of nx - s + 2RT.
    H = (so // 2) * 2
    head = s + H
    spare = max(np.sum(tails[:, 0] == w) for w in range(nt, nt + ns)) * (shape[0] - s + 2 * H)
    assert abs(spare - head) <= shape[0] - s + 2 * H, (head, spare)
    # Neighbouring tails run together: spare j takes tiles j, j + ns, ...
    for j in range(ns):
        t = tails[tails[:, 0] == nt + j]
        assert np.array_equal(t[:, 1] * tz + t[:, 2], np.arange(j, nt, wgs - nt))


def test_whole_x_with_more_tiles_than_workgroups_is_one_segment_per_tile():
    shape = (64, 400, 400)
    tile, segs = tb.schedule_segments(shape, 8, tb.schedule("tb", 2, 32, 2048), 16)
    _check_partition(shape, tile, segs)
    assert np.all(segs[:, 3] == 0) and np.all(segs[:, 4] == shape[0])


def test_segment_query_errors():
    sc = tb.schedule("tb", 2, 32, 64)
    with pytest.raises(tb.TbError) as e:
        tb.schedule_segments((64, 64, 64), 8, sc, 0)
    assert e.value.status == tb.EINVAL
    with pytest.raises(tb.TbError) as e:
        tb.schedule_segments((64, 0, 64), 8, sc, 16)
    assert e.value.status == tb.EINVAL
    with pytest.raises(tb.TbError) as e:
        tb.schedule_segments((64, 64, 64), 6, sc, 16)
    assert e.value.status == tb.EUNSUPPORTED
    with pytest.raises(tb.TbError) as e:  # three steps at space order 8: no LDS fit
        tb.schedule_segments((64, 64, 64), 8, tb.schedule("tb", 3, 32, 64), 16)
    assert e.value.status == tb.EUNSUPPORTED
