"""Benchmark: GPts/s of the temporally blocked acoustic propagator against the
spatially blocked one on the 512^3 SO8 two-layer workload (one MI355X).

One step = one full forward shot: nt updates of the whole grid with fused
off-grid injection of 8 sources and interpolation at 512 receivers, from
resident inputs. Prints one JSON line (see the keys below).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --copy-calibration   # plain 1 GiB device copies, for
                                         # scaling HBM counters

roofline.traffic comes from the committed FETCH_SIZE / WRITE_SIZE counter
summary of the wave-front kernel; it is reported only while the kernel source
and the schedule match the ones the counters were taken on (else null).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GPts/s temporal- vs spatial-blocked (1 GPU, rel L2≤1e-5); shots/s + p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT_STEP = 16  # read u^n, u^{n-1}, c; write u^{n+1}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "acoustic_wavefront_512_so8_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2010_10248_amd", "csrc", "acoustic_kernel.h")


def kernel_sha():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(sched_repr):
    """HBM bytes per launch of the TB kernel from the committed counter
    summary (lines 'key: value'), or None when it was taken on another
    kernel source or schedule."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^- (\w+): `?([^`\n]+)`?$", text, re.M))
    if kv.get("kernel_sha") != kernel_sha() or kv.get("schedule") != sched_repr:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


PHYS_COUNTERS = os.path.join(ROOT, "profiles", "tti_elastic_256_so8_counters.md")


def host_cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def code_text(path):
    """A C++ source without its comments, trailing blanks and empty lines, so
    that editing a comment does not detach a measurement from the code."""
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def physics_sha(which):
    """sha256 prefix of the code (comments dropped) the TTI or elastic forward
    kernels are compiled from: the physics file and the streaming building
    blocks."""
    h = hashlib.sha256()
    for name in ("tti.hip" if which == "tti" else "elastic.hip", "stream_kernel.h"):
        h.update(code_text(os.path.join(ROOT, "paper_2010_10248_amd", "csrc", name)).encode())
    return h.hexdigest()[:16]


def physics_traffic(which):
    """HBM bytes per step of the TTI or elastic kernels from the committed
    counter summary, or None when it was taken on other kernel sources."""
    try:
        text = open(PHYS_COUNTERS).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^- (\w+): `?([^`\n]+)`?$", text, re.M))
    sha = physics_sha(which)
    if kv.get(f"{which}_sha") != sha:
        return None
    try:
        return float(kv[f"{which}_hbm_bytes_per_step"])
    except (KeyError, ValueError):
        return None


def copy_calibration(torch):
    """Five device-to-device copies of 1 GiB: the counters of this plain copy
    kernel scale FETCH_SIZE / WRITE_SIZE to bytes."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}),
          flush=True)
    return 0


def serve_bench(tb, W, torch, nreq, loads, max_active, arena_gb, mix="tuned"):
    """C5 serving: gradient requests (forward, residual vs observed traces,
    adjoint, checkpointed squared-slowness gradient) on mixed 128-384^3 SO8
    grids with 500-1500 steps. Phase 1 submits every request at once
    (saturated shots/s); then the same requests are replayed with Poisson
    arrivals at each of `loads` x that rate, reporting completion - arrival
    latency per load. Models, sparse sets, observed data (forward runs of the
    true model with a +5% velocity anomaly) and one autotuner sweep per
    served grid size (requests then run the tuned schedule) are made before
    the clock starts. mix = "shared": sizes whose tuned kernel shape (steps
    per pass, tile rows) differs from the most common one among the served
    sizes run that shape instead, so that their passes batch with the
    others'."""
    import numpy as np

    rng = np.random.Generator(np.random.PCG64(10253))
    reqs = []
    t0 = time.perf_counter()
    tuned = {}
    best_of = {}
    for _ in range(nreq):
        shot, vp_true = W.serving_request(rng)
        vmax = float(shot.vp.max())
        prop = tb.Acoustic(shot, damp_vmax=vmax)
        n = shot.shape[0]
        if n not in tuned:
            best, ms = tb.autotune(prop.model, prop.sparse, steps=16)
            torch.cuda.synchronize()
            tuned[n] = dict(schedule=repr(best), ms_per_step=round(ms, 4))
            best_of[n] = best
            log(f"serving: tuned {n}^3: {best} {ms:.3f} ms/step")
        true = tb.Acoustic(shot, vp=vp_true, damp_vmax=vmax)
        d_obs = true.forward(None, want_fields=False)["traces"]
        true.close()
        reqs.append((shot, prop, d_obs))
    torch.cuda.synchronize()
    log(f"serving: {nreq} requests prepared in {time.perf_counter() - t0:.1f} s "
        f"(sizes {sorted(r[0].shape[0] for r in reqs)}, nt {sorted(r[0].nt for r in reqs)})")
    work = sum(int(np.prod(r[0].shape)) * r[0].nt for r in reqs)

    def shape(sc):  # what the server batches on: steps per pass, tile rows
        return (1 if sc.mode == tb.SCHED_SB else sc.time_tile, sc.tile_y or 32)

    sched_of = {n: None for n in best_of}  # None: the tuned choice
    if mix == "shared":
        shapes = [shape(best_of[r[0].shape[0]]) for r in reqs]
        major = max(set(shapes), key=lambda v: (shapes.count(v), v))
        for n, sc in best_of.items():
            if shape(sc) != major:
                sched_of[n] = tb.schedule("sb" if major[0] == 1 else "tb", major[0], major[1], 0)
                tuned[n]["served_schedule"] = repr(sched_of[n])
                log(f"serving: {n}^3 runs the shared shape {sched_of[n]}")

    def run(arrivals):
        sv = tb.Server(arena_bytes=int(arena_gb * 2**30), max_active=max_active, graphs=True)
        grads = [torch.empty(r[0].shape, dtype=torch.float32, device="cuda") for r in reqs]
        rid_of = {}
        lat = [None] * nreq
        losses = [None] * nreq
        nxt = 0
        start = time.perf_counter()
        while any(v is None for v in lat):
            now = time.perf_counter() - start
            while nxt < nreq and arrivals[nxt] <= now:
                shot, prop, d_obs = reqs[nxt]
                rid_of[sv.submit_gradient(prop, d_obs, grads[nxt],
                                          sched_of[shot.shape[0]])] = nxt
                nxt += 1
            act, queued = sv.step()
            for rid, J in sv.poll():
                i = rid_of[rid]
                lat[i] = time.perf_counter() - start - arrivals[i]
                losses[i] = J
            if act == 0 and queued == 0 and nxt < nreq:
                time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - start)))
        span = time.perf_counter() - start
        st = sv.stats()
        sv.close()
        return span, lat, losses, st

    span, lat_sat, losses, st = run([0.0] * nreq)
    rate = nreq / span
    log(f"serving saturated: {nreq} requests in {span:.2f} s = {rate:.3f} shots/s; stats {st}")
    per_load = []
    for k, load in enumerate(loads):
        gen = np.random.Generator(np.random.PCG64(7 + k))
        arr = np.cumsum(gen.exponential(1.0 / (load * rate), nreq))
        arr = arr - arr[0]
        span2, lat, losses2, st2 = run(list(arr))
        assert losses2 == losses, "a request's misfit changed between runs"
        lat_ms = np.array(lat) * 1e3
        per_load.append(dict(
            load=load, offered_shots_per_s=round(load * rate, 4),
            shots_per_s=round(nreq / span2, 4),
            p50_ms=round(float(np.percentile(lat_ms, 50)), 1),
            p99_ms=round(float(np.percentile(lat_ms, 99)), 1),
            batched_passes_per_launch=round(st2["passes_batched"] / max(st2["launches"], 1), 2),
            graph_replays=st2["graph_replays"], graph_captures=st2["graph_captures"]))
        log(f"serving Poisson at {load}x: {per_load[-1]}")
    out = dict(shots_per_s=round(rate, 4), requests=nreq,
               point_updates_per_request_mean=round(work / nreq / 1e9, 3),
               gradient_gpts_per_s_equiv=round(work / span / 1e9, 2),
               saturated_p50_ms=round(float(np.percentile(np.array(lat_sat) * 1e3, 50)), 1),
               saturated_p99_ms=round(float(np.percentile(np.array(lat_sat) * 1e3, 99)), 1),
               poisson=per_load, tuned_schedules=tuned, served_schedules=mix,
               saturated_batched_passes_per_launch=round(
                   st["passes_batched"] / max(st["launches"], 1), 2),
               max_active=max_active, arena_gib=arena_gb,
               request="gradient (forward + residual + adjoint + imaging, checkpoints every "
                       "ceil(sqrt(nt)))",
               mix="SO8 two-layer, N in {128,192,256,384}, nt 500-1500, Poisson arrivals")
    for _, prop, _ in reqs:
        prop.close()
    return out


def physics_bench(tb, W, torch, which, steps, nt=0, sb_only=False):
    """GPts/s of the TTI (256^3 SO8, 800 steps, 44 B per point-step) or
    elastic (256^3 SO8, 600 steps, 84 B per point-step) propagator on one
    shot, inputs resident, for the spatially blocked schedule and the
    autotuner's choice among the temporally blocked ones (passes of T steps
    over x-slabs); effective bandwidth at those algorithmic bytes, and the
    bitwise identity of the two."""
    import numpy as np

    if which == "tti":
        shot = W.tti_smooth(nt=nt) if nt else W.tti_smooth()
        bpp = 44
    else:
        shot = W.elastic_smooth(nt=nt) if nt else W.elastic_smooth()
        bpp = 84
    prop = tb.Propagator(shot)
    nt = shot.nt
    N3 = int(np.prod(shot.shape))
    shape = (2, nt, prop.nrec) if which == "elastic" else (nt, prop.nrec)

    def timed(sched):
        ws = prop.workspace(sched)
        rec = torch.empty(shape, dtype=torch.float32, device="cuda")
        u = torch.empty(shot.shape, dtype=torch.float32, device="cuda")
        tb.forward(prop.model, prop.sparse, sched, ws, rec, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            tb.forward(prop.model, prop.sparse, sched, ws, rec, u)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, rec, u

    dt_sb, rec_sb, u_sb = timed(tb.schedule("sb"))
    g_sb = N3 * nt / dt_sb / 1e9
    # Roofline of the spatially blocked step at the metric's algorithmic bytes
    # (shot time, so injection, gathers and launch gaps count against it).
    traffic = physics_traffic(which)
    roof = dict(bound="hbm", achieved=round(g_sb * bpp, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(g_sb * bpp / HBM_PEAK_GBS, 4),
                traffic=round(traffic) if traffic is not None else None,
                traffic_unit="HBM bytes per step (calibrated FETCH_SIZE + WRITE_SIZE)",
                algorithmic_bytes_per_step=bpp * N3)
    if sb_only:
        prop.close()
        log(f"{which}: {shot.name}: SB {dt_sb * 1e3:.1f} ms/shot {g_sb:.1f} GPts/s")
        return dict(workload=shot.name, ms_per_shot=round(dt_sb * 1e3, 2),
                    gpts_per_s=round(g_sb, 2), bytes_per_point_step=bpp,
                    effective_hbm_frac=round(g_sb * bpp / HBM_PEAK_GBS, 4), schedule="SB")
    best, _ = tb.autotune(prop.model, prop.sparse, steps=16)
    tbs = tb.schedule("tb", 2, 0, 32) if best.time_tile == 1 else best
    dt_tb, rec_tb, u_tb = timed(tbs)
    g_tb = N3 * nt / dt_tb / 1e9
    same = bool(torch.equal(rec_sb.view(torch.int32), rec_tb.view(torch.int32))
                and torch.equal(u_sb.view(torch.int32), u_tb.view(torch.int32)))
    prop.close()
    log(f"{which}: {shot.name}: SB {dt_sb * 1e3:.1f} ms/shot {g_sb:.1f} GPts/s; {tbs} "
        f"{dt_tb * 1e3:.1f} ms/shot {g_tb:.1f} GPts/s; tuned {best}; bitwise {same}")
    return dict(workload=shot.name, ms_per_shot=round(dt_sb * 1e3, 2), gpts_per_s=round(g_sb, 2),
                bytes_per_point_step=bpp,
                effective_hbm_frac=round(g_sb * bpp / HBM_PEAK_GBS, 4), schedule="SB",
                roofline=roof,
                temporal_blocked=dict(schedule=repr(tbs), ms_per_shot=round(dt_tb * 1e3, 2),
                                      gpts_per_s=round(g_tb, 2),
                                      effective_hbm_frac=round(g_tb * bpp / HBM_PEAK_GBS, 4),
                                      bitwise_equal_to_sb=same),
                tuned_schedule=repr(best))


def space_order_bench(tb, W, torch, nt):
    """Table 1's space-order axis on the 512^3 two-layer grid: GPts/s of the
    fastest spatially blocked schedule and the fastest temporally blocked
    one built for each order (nt steps per shot; one warm-up, one timed
    shot each)."""
    import numpy as np

    cands = {4: [("tb", 3, 32, 2048), ("tb", 3, 32, 64), ("tb", 2, 32, 2048), ("tb", 4, 16, 64)],
             8: [("tb", 2, 32, 2048), ("tb", 2, 32, 64)],
             12: [("tb", 2, 32, 64), ("tb", 2, 32, 2048), ("tb", 2, 16, 64)]}
    sb_cands = [("sb", 1, 16, 2048), ("sb", 1, 32, 128), ("sb", 1, 16, 128)]
    out = []
    for so in (4, 8, 12):
        shot = W.acoustic_two_layer(so=so, nt=nt)
        prop = tb.Acoustic(shot)
        N = int(np.prod(shot.shape)) * nt
        row = dict(space_order=so, nt=nt)
        sb_best = None
        for c in sb_cands:
            sc = tb.schedule(*c)
            dt, _, _, _, _, _ = time_forward(tb, prop, sc, 1, 1, torch)
            if sb_best is None or N / dt > sb_best[0]:
                sb_best = (N / dt, repr(sc))
        row["sb_gpts"], row["sb_schedule"] = round(sb_best[0] / 1e9, 1), sb_best[1]
        best = None
        for c in cands[so]:
            sc = tb.schedule(*c)
            dt, _, _, _, _, _ = time_forward(tb, prop, sc, 1, 1, torch)
            g = N / dt / 1e9
            if best is None or g > best[0]:
                best = (g, repr(sc))
        row["tb_gpts"], row["tb_schedule"] = round(best[0], 1), best[1]
        row["tb_over_sb"] = round(best[0] / row["sb_gpts"], 3)
        # The autotuner's sweep of every schedule (SB included) on this
        # model; the NULL schedule then runs its choice.
        tsc, _ = tb.autotune(prop.model, prop.sparse, steps=16)
        dt, _, _, _, _, _ = time_forward(tb, prop, None, 1, 1, torch)
        row["tuned_schedule"], row["tuned_gpts"] = repr(tsc), round(N / dt / 1e9, 1)
        prop.close()
        log(f"space order {row}")
        out.append(row)
    return out


def density_bench(tb, W, torch, counts, tb_sched, sb_sched, nt):
    """Section IV-E's source-density experiment on the 512^3 SO8 two-layer
    grid: TB and SB GPts/s with 1..many sources, uniform in the volume or on
    one horizontal plane (nt steps per shot; one warm-up and one timed shot
    per schedule)."""
    import numpy as np

    out = []
    for layout in ("volume", "plane"):
        for k in counts:
            shot = W.acoustic_source_density(k, layout, nt=nt)
            prop = tb.Acoustic(shot)
            insp = inspector_seconds(tb, prop, shot, torch)
            npts, _ = tb.sparse_counts(prop.sparse)
            g = {}
            for name, sc in (("tb", tb_sched), ("sb", sb_sched)):
                dt, _, _, _, _, _ = time_forward(tb, prop, sc, 1, 1, torch)
                g[name] = int(np.prod(shot.shape)) * nt / dt / 1e9
            prop.close()
            row = dict(layout=layout, sources=k, points=npts, inspector_s=round(insp, 4),
                       tb_gpts=round(g["tb"], 1), sb_gpts=round(g["sb"], 1),
                       tb_over_sb=round(g["tb"] / g["sb"], 3))
            log(f"density {row}")
            out.append(row)
    return out


def inspector_seconds(tb, prop, shot, torch):
    """Wall time of the inspector alone (support, SM/SID, decomposition and
    upload, Section II-A) for the shot's sparse set on an existing model: a
    second inspection, discarded. The per-schedule tile lists are built at
    the first forward of a schedule (inside the warm-up shot)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sp = tb.inspect_sparse(prop.model, shot.src_xyz, shot.src_wav, shot.rec_xyz)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tb.destroy_sparse(sp)
    return dt


def first_arrival_steps(shot, margin=1.15):
    """Steps until the direct wave's Ricker peak reaches the nearest receiver
    at the fastest velocity, with a margin: the parity leg's traces then
    carry the wavelet."""
    import numpy as np

    d = np.linalg.norm(shot.src_xyz[:, None, :] - shot.rec_xyz[None, :, :], axis=2).min()
    t = d / float(shot.vp.max()) + 1.0 / 8.0  # Ricker peak delay 1/f, f >= 8 Hz
    return int(np.ceil(margin * t / shot.dt))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rel_l2(a, b):
    import numpy as np

    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def time_forward(tb, prop, sched, steps, warmup, torch):
    """Run warmup + timed forward shots; return (seconds, kernel stats, outputs)."""
    ws = prop.workspace(sched)
    nt = prop.shot.nt
    rec = torch.empty((nt, prop.nrec), dtype=torch.float32, device="cuda")
    u = torch.empty(prop.shot.shape, dtype=torch.float32, device="cuda")
    up = torch.empty(prop.shot.shape, dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        tb.forward(prop.model, prop.sparse, sched, ws, rec, u, up)
    torch.cuda.synchronize()
    tb.kernel_timing(True)
    t0 = time.perf_counter()
    for k in range(steps):
        tb.forward(prop.model, prop.sparse, sched, ws, rec, u, up)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms = tb.kernel_timing_read()
    tb.kernel_timing(False)
    return dt, launches, kms, rec, u, up


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nt", type=int, default=1000)
    ap.add_argument("--T", type=int, default=2)
    ap.add_argument("--tile-y", type=int, default=32)
    # chunk 2048 (>= nx): each tile streams whole x, the spare workgroups take
    # the tails (the fastest TB and SB schedules at 512^3 SO8).
    ap.add_argument("--chunk", type=int, default=2048)
    ap.add_argument("--sb-tile-y", type=int, default=16)
    ap.add_argument("--sb-chunk", type=int, default=2048)
    ap.add_argument("--no-sb", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-orders", action="store_true",
                    help="skip the space-order sweep (SO 4, 8, 12)")
    ap.add_argument("--no-density", action="store_true",
                    help="skip the source-density sweep")
    ap.add_argument("--no-physics", action="store_true",
                    help="skip the TTI and elastic measurements")
    ap.add_argument("--physics-nt", type=int, default=0,
                    help="steps of the TTI and elastic shots (0: their workloads' 800 and 600)")
    ap.add_argument("--physics-sb-only", action="store_true",
                    help="time only the spatially blocked TTI and elastic schedules")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-mix", choices=("tuned", "shared"), default="shared",
                    help="served schedules: each size's tuned choice, or the most common tuned "
                         "kernel shape for every size (so that all passes can batch)")
    ap.add_argument("--serve-loads", type=str, default="0.5,0.8,1.0",
                    help="Poisson loads as fractions of the saturated rate")
    ap.add_argument("--serve-active", type=int, default=4)
    ap.add_argument("--serve-arena-gb", type=float, default=128.0)
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="steps of the full grid the FP64 oracle runs for the parity leg and "
                         "the CPU sample (0: until the direct wave reaches the receivers)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(shots shard across GPUs without communication; see the design notes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2010_10248_amd import tb
    from paper_2010_10248_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        return copy_calibration(torch)

    shot = W.acoustic_two_layer(n=args.n, nt=args.nt)
    N3 = int(np.prod(shot.shape))
    log(f"workload: {shot.name}, {shot.src_xyz.shape[0]} sources, {shot.rec_xyz.shape[0]} receivers")
    t0 = time.perf_counter()
    prop = tb.Acoustic(shot)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    npts, nrid = tb.sparse_counts(prop.sparse)
    insp_s = inspector_seconds(tb, prop, shot, torch)
    log(f"model + inspector: {setup_s:.3f} s, of which the inspector {insp_s:.4f} s "
        f"(npts {npts}, receiver points {nrid})")

    tb_sched = tb.schedule("tb", args.T, args.tile_y, args.chunk)
    sb_sched = tb.schedule("sb", 1, args.sb_tile_y, args.sb_chunk)

    dt_tb, nl_tb, kms_tb, rec_tb, u_tb, up_tb = time_forward(tb, prop, tb_sched, args.steps,
                                                            args.warmup, torch)
    gpts_tb = N3 * shot.nt * args.steps / dt_tb / 1e9
    log(f"TB {tb_sched}: {dt_tb / args.steps * 1e3:.2f} ms/shot, {gpts_tb:.1f} GPts/s, "
        f"{nl_tb} kernel launches, {kms_tb / max(nl_tb, 1):.3f} ms each")

    sb = None
    if not args.no_sb:
        dt_sb, nl_sb, kms_sb, rec_sb, u_sb, up_sb = time_forward(tb, prop, sb_sched, args.steps,
                                                                args.warmup, torch)
        gpts_sb = N3 * shot.nt * args.steps / dt_sb / 1e9
        same = (torch.equal(rec_tb.view(torch.int32), rec_sb.view(torch.int32))
                and torch.equal(u_tb.view(torch.int32), u_sb.view(torch.int32))
                and torch.equal(up_tb.view(torch.int32), up_sb.view(torch.int32)))
        sb = dict(value=round(gpts_sb, 2), ms_per_step=round(dt_sb / args.steps * 1e3, 3),
                  kernel_ms_avg=round(kms_sb / max(nl_sb, 1), 4), schedule=repr(sb_sched),
                  bitwise_equal_to_tb=bool(same))
        log(f"SB {sb_sched}: {dt_sb / args.steps * 1e3:.2f} ms/shot, {gpts_sb:.1f} GPts/s; "
            f"TB == SB bitwise: {same}")

    # Dominant kernel: the wave-front propagation kernel. Algorithmic bytes
    # per launch = 16 B x N^3 points x T steps.
    steps_per_launch = shot.nt * args.steps / max(nl_tb, 1)
    achieved = BYTES_PER_POINT_STEP * N3 * shot.nt * args.steps / (kms_tb * 1e-3) / 1e9
    traffic = measured_traffic(repr(tb_sched))
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=round(traffic) if traffic is not None else None,
                    traffic_unit="bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                    algorithmic_bytes_per_launch=BYTES_PER_POINT_STEP * N3 * round(steps_per_launch),
                    kernel_sha=kernel_sha(),
                    kernel=f"acoustic_wavefront<R=4,T={args.T},BYE={args.tile_y}>",
                    kernel_ms_avg=round(kms_tb / max(nl_tb, 1), 4),
                    steps_per_launch=round(steps_per_launch, 3),
                    bytes_per_point_step=BYTES_PER_POINT_STEP)

    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle

        steps = args.cpu_steps or first_arrival_steps(shot)
        sample = W.acoustic_two_layer(n=args.n, nt=min(steps, shot.nt))
        t0 = time.perf_counter()
        ref = oracle.acoustic_forward(sample)
        cpu_s = time.perf_counter() - t0
        cores = oracle.num_threads()
        cpu = dict(value=round(N3 * sample.nt / cpu_s / 1e9, 4), unit="GPts/s", cores=cores,
                   kind="oracle", cpu_model=host_cpu_model(), seconds=round(cpu_s, 2),
                   sample=f"FP64 oracle, full {args.n}^3 grid, first {sample.nt} of {shot.nt} "
                          f"steps (same sources/receivers; the run the parity leg compares)")
        log(f"oracle: {cpu_s:.1f} s for {sample.nt} steps on {cores} threads")
        sp = tb.Acoustic(sample)
        errs = {}
        tr_peak = float(np.abs(ref["traces"]).max())
        for name, sc in (("tb", tb_sched), ("sb", sb_sched)):
            o = sp.forward(sc)
            torch.cuda.synchronize()
            tr = o["traces"].cpu().numpy()
            errs[name] = dict(traces=rel_l2(tr, ref["traces"]),
                              u_last=rel_l2(o["u_last"].cpu().numpy(), ref["u_last"]),
                              u_prev=rel_l2(o["u_prev"].cpu().numpy(), ref["u_prev"]))

        sp.close()
        parity = dict(steps=sample.nt, oracle_trace_peak=float(f"{tr_peak:.3e}"),
                      **{k: {kk: float(f"{vv:.3e}") for kk, vv in v.items()}
                         for k, v in errs.items()})
        log(f"parity vs FP64 oracle at {sample.nt} steps: {parity}")

    orders = None
    if not args.no_orders:
        orders = space_order_bench(tb, W, torch, 200)
    density = None
    if not args.no_density:
        density = density_bench(tb, W, torch, (1, 64, 1024, 8192), tb_sched, sb_sched, 200)

    physics = None
    if not args.no_physics:
        physics = {k: physics_bench(tb, W, torch, k, 2, args.physics_nt, args.physics_sb_only)
                   for k in ("tti", "elastic")}

    serving = None
    if not args.no_serve:
        serving = serve_bench(tb, W, torch, args.serve_requests,
                              [float(x) for x in args.serve_loads.split(",")],
                              args.serve_active, args.serve_arena_gb, args.serve_mix)

    line = {
        "metric": METRIC,
        "value": round(gpts_tb, 2),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt_tb / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"isotropic acoustic {args.n}^3, h=10 m, SO8, {shot.nt} steps, "
                        f"two-layer vp 1500/4500, 8 off-grid Ricker sources, "
                        f"{shot.rec_xyz.shape[0]} receivers, sponge 40",
            "schedule": repr(tb_sched),
            "effective_hbm_frac": round(gpts_tb * BYTES_PER_POINT_STEP / HBM_PEAK_GBS, 4),
            "spatial_blocked": sb,
            "tb_over_sb": round(gpts_tb / sb["value"], 3) if sb else None,
            "parity_rel_l2": parity,
            "inspector_s": round(insp_s, 4),
            "model_setup_s": round(setup_s - insp_s, 3),
            "serving": serving,
            "other_physics": physics,
            "source_density": density,
            "space_orders": orders,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    prop.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
