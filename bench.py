"""Benchmark of the hot path on one MI355X.

One step = one B-mode frame of the triangle-mesh anatomy phantom (200,192
triangles in four nested closed meshes, 21 plane waves x 798,912 rays, 12
interactions, 192 elements x 8192 samples, 512 x 1024 pixels): transport and
RF synthesis, beamforming, envelope and log compression, all through the C-ABI
with inputs and buffers resident in HBM. The same protocol is repeated for
forward + backward (gradient of every parameter), then for the layered phantom
(11 plane waves x 2^20 rays, 8 interactions, 128 x 4096 samples, 256 x 512
pixels), followed by iterations of the inverse loop, the acquisition gradients
and the serving stream. Prints one JSON line with the throughput in
ray-segments/s (a segment is one closest-hit query, primary or secondary),
frames/s, per-kernel timings from HIP events recorded on the launch stream
inside the timed region, the roofline of the dominant kernel and the FP64
oracle timed on the host cores as a reported baseline.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
CALIBRATION_BYTES = 512 << 20
FP64_PEAK_TFLOPS = 78.6    # MI355X vector fp64


def kernel_bytes(name, wl, counts, n_px):
    """Algorithmic HBM bytes of one frame for each kernel (what it must read
    and write at least once), from the frame's event counts."""
    p = wl.probe
    rays = wl.n_tx * wl.rays_per_tx
    seg_p, seg_s, dep, inter, sec = counts
    row_samples = wl.n_tx * p.n_elem * p.n_t
    state = 8 * 8 + 2 * 4          # ray state in the queue [B]
    has_meshes = len(getattr(wl.scene, "meshes", ()) or ()) > 0
    sec_rec = 5 * 8 + 3 * 4        # secondary-ray record [B]
    return {
        # every primary segment after the first reads a queued state, every
        # surviving ray writes one, every diffuse hit writes a secondary record
        "bounce": 2 * state * (seg_p - rays) + sec_rec * sec,
        # each secondary record is read once; each deposit writes a 12-byte
        # record for the binned splat (scenes with meshes: two fp32 bins, and
        # the record is found through a 4-byte permutation entry)
        "secondary": (sec_rec + (4 if has_meshes else 0)) * sec + (8 if has_meshes else 12) * dep,
        # scenes with meshes: the receiver segments' counting sort reads each
        # record's key and rank and writes its 4-byte permutation entry
        "secondary_sort": (8 + 4) * sec if has_meshes else None,
        # binned splat (scenes without meshes): the counting pass reads each
        # record's 4-byte key, the scatter reads the 12-byte record and writes
        # it as 16 bytes; the accumulation reads the 16 bytes and updates every
        # RF bin once. `dep` also counts the few array hits that the bounce
        # kernel adds directly, so these are upper bounds on the records.
        "splat_bin": None if has_meshes else (4 + 12 + 16) * dep,
        "splat_accumulate": None if has_meshes else 16 * dep + 8 * row_samples,
        # the last chunk's deposits (16-byte records), the fixed-point row of
        # direct deposits read, the RF written
        "splat_pulse": None if has_meshes else 16 * dep + (8 + 4) * row_samples,
        # the fixed-point histogram read, the RF written
        "pulse": 12 * row_samples,
        "pulse_adjoint": 8 * row_samples,
        "analytic_adjoint": 12 * row_samples,
        # the analytic-signal gradient read, dL/dh written (dL/drf stays in LDS)
        "analytic_pulse_adjoint": 12 * row_samples,
        "das_adjoint": 8 * row_samples + 8 * n_px,
        "bmode_vjp": 28 * n_px,
        "image_loss": 12 * n_px,
        # replay: the forward phase moves the live rays through the queues as
        # the bounce kernel does, writes one 80-byte step record per primary
        # segment and a 4-byte queue entry per diffuse interaction; the
        # secondary phase reads the entry, the step record and dL/dh at its
        # deposit and writes 80 bytes of adjoints; the reverse phase reads the
        # step records, those adjoints and dL/dh at the array hits
        "replay_forward": 2 * state * (seg_p - rays) + 80 * seg_p + 4 * sec,
        "replay_secondary": (4 + 80 + 8 + 80) * sec,
        # a recorded forward: the replay's forward phase (array hits deposited
        # in place), then per queued interaction its entry and step record read
        # and the deposit made
        "recorded_forward": 2 * state * (seg_p - rays) + 80 * seg_p + 4 * sec,
        "recorded_deposit": (4 + 80) * sec + 8 * dep,
        "replay_reverse": 80 * seg_p + 80 * sec + 8 * (dep - sec),
        "analytic": 12 * row_samples,
        "das": 8 * row_samples + 8 * n_px,
        "bmode": 20 * n_px,
    }.get(name)


def measured_traffic(kernel, summary):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary profiles/`summary` (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or
    None when the summary is missing or the kernel sources changed since it
    was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    try:
        text = open(path).read()
    except OSError:
        return None
    vals, srcs, sha = {}, [], None
    for line in text.splitlines():
        t = line.split()
        if len(t) == 3 and t[0] == "traffic_bytes_per_launch":
            vals[t[1]] = float(t[2])
        elif len(t) == 2 and t[0] == "sources_sha256":
            sha = t[1]
        elif t and t[0] == "sources":
            srcs = t[1:]
    h = hashlib.sha256()
    try:
        for f in srcs:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    if sha is None or h.hexdigest() != sha:
        return None
    return vals.get(kernel)


def cpu_baseline(wl, ray_count=None):
    """The FP64 oracle on the host cores, segments/s of its transport (no
    image chain). With ray_count, a labelled sample: that many consecutive rays
    of every transmit, centred on the middle of the array (the oracle builds
    its own hierarchy first, which is timed too); else the whole frame."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    total = wl.probe.n_elem * wl.rays_per_elem
    if ray_count is None or ray_count >= total:
        begin, count = 0, total
    else:
        begin, count = total // 2 - ray_count // 2, ray_count
    t0 = time.perf_counter()
    tr = oracle.trace(wl.scene, wl.probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                      wl.max_bounces, ray_begin=begin, ray_count=count, n_threads=cores)
    dt = time.perf_counter() - t0
    what = ("one whole frame" if count == total else
            f"rays [{begin}, {begin + count}) of each transmit ({wl.n_tx} x {count} = {wl.n_tx * count} rays "
            f"of the frame's {wl.n_tx * total}; elements {begin // wl.rays_per_elem}-"
            f"{(begin + count - 1) // wl.rays_per_elem} of {wl.probe.n_elem})")
    return {"value": tr.segments / dt, "unit": "ray-segments/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}: FP64 transport, {wl.max_bounces} interactions, {tr.segments} segments in "
                      f"{dt:.2f} s"}


def inverse_leg(ctx, steps, warmup):
    """Algorithm opt on the layered phantom: the 34 perturbed parameters free
    within +-10 % (material and geometry learning-rate groups), the others
    fixed, three micro-batches of transmits (4, 4, 3 plane waves), MSE against
    the image of the seeded +-5 % target; iterations per second."""
    import numpy as np
    import torch
    from paper_2604_15017_amd import workloads as W
    from paper_2604_15017_amd.inverse import InverseLoop, MicroBatch, unconstrained_start
    wl = W.layered_phantom()
    sc = wl.scene
    theta0 = sc.theta()
    idx = W.perturbed_indices(sc)
    lo, hi = theta0.copy(), theta0.copy()
    lo[idx] = theta0[idx] - 0.1 * np.abs(theta0[idx])
    hi[idx] = theta0[idx] + 0.1 * np.abs(theta0[idx])
    lr = np.zeros_like(theta0)
    n_mat = 3 * (sc.n_regions - 1)
    lr[idx[:n_mat]], lr[idx[n_mat:]] = 0.02, 0.03
    batches = [MicroBatch(list(range(i, min(i + 4, wl.n_tx)))) for i in range(0, wl.n_tx, 4)]
    loop = InverseLoop(ctx, wl, lo, hi, lr, unconstrained_start(theta0, lo, hi), batches,
                       target=W.layered_phantom_target(wl), max_norm=1e3)
    losses = [float(loop.iterate().item()) for _ in range(warmup)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(loop.stream)
    out = [loop.iterate() for _ in range(steps)]
    end.record(loop.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    losses += [float(x.item()) for x in out]
    u_plain = loop.u.clone()
    del loop
    # the same iterations with each micro-batch's paths recorded by its forward
    rec = InverseLoop(ctx, wl, lo, hi, lr, unconstrained_start(theta0, lo, hi), batches,
                      target=W.layered_phantom_target(wl), max_norm=1e3, recorded=True)
    for _ in range(warmup):
        rec.iterate()
    torch.cuda.synchronize()
    start.record(rec.stream)
    for _ in range(steps):
        rec.iterate()
    end.record(rec.stream)
    torch.cuda.synchronize()
    ms_rec = start.elapsed_time(end) / steps
    return {"workload": f"layered_phantom, {len(idx)} free parameters, {len(batches)} transmit "
                        f"micro-batches, MSE vs the +-5 % target, Adam (lr 0.02 material / 0.03 geometry)",
            "ms_per_iteration": round(ms, 4), "iterations_per_s": round(1e3 / ms, 2),
            "loss_first": losses[0], "loss_last": losses[-1], "iterations": len(losses),
            "recorded": {"ms_per_iteration": round(ms_rec, 4), "speedup_vs_plain": round(ms / ms_rec, 4),
                         "iterates_bitwise_equal_to_plain": bool(torch.equal(u_plain, rec.u))}}


def acquisition_leg(ctx, steps, warmup):
    """Gradients of the image with respect to the acquisition parameters (the
    11 steering angles, c_ref, pitch) on the layered frame's RF and grid, from
    seeded channels and a seeded image gradient: ms per call, and the DAS
    kernel's rate in taps (pixel x element x transmit) per second. Then the
    transport VJP of the whole layered frame from a seeded dL/drf, timed
    without and with the acquisition adjoints (angles, c_ref, pitch, f0)."""
    import ctypes
    import numpy as np
    import torch
    from paper_2604_15017_amd import _lib as L
    from paper_2604_15017_amd import workloads as W
    wl = W.layered_phantom()
    p, g = wl.probe, wl.grid
    gen = torch.Generator(device="cuda").manual_seed(7)
    rf = torch.randn((wl.n_tx, p.n_elem, p.n_t), dtype=torch.float32, device="cuda", generator=gen)
    g_iq = torch.randn((g.n_x, g.n_z, 2), dtype=torch.float32, device="cuda", generator=gen)
    probe = L.Probe(ctx, p)
    out = torch.empty(wl.n_tx + 2, dtype=torch.float64, device="cuda")
    gd = L._grid(g)
    ws = L._workspace(L.load().us_beamform_acq_vjp_workspace_size(probe.handle, ctypes.byref(gd), wl.n_tx),
                      ctx.torch_device)
    f = lambda: L.us_beamform_acq_vjp(ctx, probe, g, wl.angles, wl.tx_ids, rf, g_iq, out=out, workspace=ws)
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    L.us_profile_enable(ctx, True)
    L.us_profile_read(ctx)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        f()
    end.record()
    torch.cuda.synchronize()
    prof = L.us_profile_read(ctx)
    L.us_profile_enable(ctx, False)
    ms = start.elapsed_time(end) / steps
    taps = g.n_px * p.n_elem * wl.n_tx
    das_ms = prof["das_acq"][0] / steps if "das_acq" in prof else float("nan")
    # through the transport: the replay VJP of the whole frame with and without
    # the acquisition adjoints (angles, c_ref, pitch, f0), seeded dL/drf
    scene = L.Scene(ctx, wl.scene)
    g_rf = torch.randn((wl.n_tx, p.n_elem, p.n_t), dtype=torch.float32, device="cuda", generator=gen)
    ws_r = L._workspace(L.us_simulate_rf_vjp_workspace_size(scene, probe, wl.n_tx, wl.rays_per_tx,
                                                            wl.max_bounces), ctx.torch_device)
    g_theta = torch.zeros(scene.n_params, dtype=torch.float64, device="cuda")
    g_acq = torch.zeros(wl.n_tx + 3, dtype=torch.float64, device="cuda")

    def vjp(acq):
        L.us_simulate_rf_vjp(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                             wl.max_bounces, g_rf, g_theta=g_theta, workspace=ws_r,
                             g_acq=g_acq if acq else None)
    replay_ms = {}
    for acq in (False, True):
        vjp(acq)
        torch.cuda.synchronize()
        start.record()
        for _ in range(max(1, steps // 4)):
            vjp(acq)
        end.record()
        torch.cuda.synchronize()
        replay_ms[acq] = start.elapsed_time(end) / max(1, steps // 4)
    acq_finite = bool(np.isfinite(g_acq.cpu().numpy()).all())
    del ws_r
    torch.cuda.empty_cache()
    return {"workload": f"layered_phantom grid {g.n_x} x {g.n_z}, {wl.n_tx} transmits x {p.n_elem} elements, "
                        f"d/d (steering angles, c_ref, pitch) of Re<g, I>; transport VJP of the frame "
                        f"({wl.n_tx} x {wl.rays_per_tx} rays) with d/d (angles, c_ref, pitch, f0)",
            "ms_per_call": round(ms, 4), "das_acq_ms": round(das_ms, 4),
            "taps_per_s": taps / (das_ms * 1e-3) if das_ms == das_ms else None,
            "transport_vjp_ms": round(replay_ms[False], 3),
            "transport_vjp_with_acquisition_ms": round(replay_ms[True], 3),
            "finite": bool(np.isfinite(out.cpu().numpy()).all()) and acq_finite}


def serving(ctx, n_requests):
    """Serving stream: Poisson arrivals at 80 % of the measured one-at-a-time
    throughput, scenes 40/40/20 from the two-layer, layered-phantom and mesh
    anatomy generators, 2^14..2^24 rays, grids 128x256..512x1024, 30 % gradient requests,
    200 GB admission cap; one slot (plain) against eight slots (continuous
    batching) on the same arrivals."""
    import torch
    from paper_2604_15017_amd import serve as S
    from paper_2604_15017_amd import workloads as W
    specs = W.serving_requests(n_requests, seed=4)
    ex1 = S.GpuExecutor(ctx, n_slots=1)
    reqs = S.build_requests(ex1, specs)

    def fresh():
        return [S.Request(r.rid, r.workload, r.want_grad, r.b_ref) for r in reqs]

    # warm-up: every distinct scene and shape once
    srv = S.Server(ex1, n_slots=1)
    for r in fresh()[:16]:
        srv.submit(r)
    srv.run(16)
    torch.cuda.synchronize()
    # plain throughput: all requests queued at once, one at a time
    srv = S.Server(ex1, n_slots=1)
    batch = fresh()
    for r in batch:
        srv.submit(r)
    t0 = time.perf_counter()
    srv.run(len(batch))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    plain_segs = sum(r.segments for r in srv.results.values() if r.ok)
    print(f"serving: plain closed loop {plain_s:.2f} s", file=sys.stderr, flush=True)
    # the same closed loop with eight overlapping slots
    ex8 = S.GpuExecutor(ctx, n_slots=8)
    srv = S.Server(ex8, n_slots=8)
    for r in fresh():
        srv.submit(r)
    t0 = time.perf_counter()
    srv.run(len(batch))
    torch.cuda.synchronize()
    batched_s = time.perf_counter() - t0
    batched_segs = sum(r.segments for r in srv.results.values() if r.ok)
    print(f"serving: batched closed loop {batched_s:.2f} s", file=sys.stderr, flush=True)
    rate = 0.8 * len(batch) / plain_s
    offsets = S.poisson_arrivals(len(batch), rate, seed=4)
    out = {"requests": len(batch), "grad_requests": int(sum(r.want_grad for r in batch)),
           "arrival_rate_hz": round(rate, 2),
           "plain_closed_loop_s": round(plain_s, 3),
           "batched_closed_loop_s": round(batched_s, 3),
           "closed_loop_speedup": round(plain_s / batched_s, 3),
           # capacity: every request queued at once, segments of all requests / wall time
           "plain_capacity_segments_per_s": plain_segs / plain_s,
           "batched_capacity_segments_per_s": batched_segs / batched_s}
    for name, slots in (("plain_one_at_a_time", 1), ("continuous_batching", 8)):
        ex = ex1 if slots == 1 else ex8
        srv = S.Server(ex, n_slots=slots, mem_cap_bytes=200 * 10**9)
        res = S.replay_stream(srv, fresh(), offsets)
        torch.cuda.synchronize()
        st = S.latency_stats(res)
        st.update({"slots": slots, "max_concurrent": srv.max_concurrent,
                   "peak_reserved_GB": round(srv.max_reserved / 1e9, 2)})
        out[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
        print(f"serving: {name} p50 {st.get('p50_ms')} ms p99 {st.get('p99_ms')} ms", file=sys.stderr,
              flush=True)
    return out


def frame_legs(ctx, wl, target, steps, warmup, backward=True):
    """Forward (one B-mode frame) and forward + backward (B-mode MSE against
    the image of `target`, gradient of every parameter) of one workload, each
    timed over `steps` frames after `warmup` untimed ones with HIP events on the
    launch stream; per-kernel times from the library's own event log."""
    import torch
    from paper_2604_15017_amd import _lib as L
    p, g = wl.probe, wl.grid
    scene, probe = L.Scene(ctx, wl.scene), L.Probe(ctx, wl.probe)
    dev = ctx.torch_device
    rf = torch.empty((wl.n_tx, p.n_elem, p.n_t), dtype=torch.float32, device=dev)
    iq = torch.empty((g.n_x, g.n_z, 2), dtype=torch.float32, device=dev)
    bm = torch.empty((g.n_x, g.n_z), dtype=torch.float32, device=dev)
    ws_t = L._workspace(L.us_simulate_rf_workspace_size(scene, probe, wl.n_tx, wl.rays_per_tx,
                                                        wl.max_bounces), dev)
    ws_b = L._workspace(L.load().us_beamform_workspace_size(probe.handle, wl.n_tx), dev)
    ws_m = L._workspace(L.load().us_bmode_workspace_size(g.n_px), dev)
    counters = torch.zeros(5, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step(sc=scene, cnt=None):
        L.us_simulate_rf(ctx, sc, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                         wl.max_bounces, rf=rf, counters=cnt, workspace=ws_t, stream=stream)
        L.us_beamform(ctx, probe, g, wl.angles, wl.tx_ids, rf, iq=iq, workspace=ws_b, stream=stream)
        L.us_bmode(ctx, iq, wl.dr_db, out=bm, workspace=ws_m, stream=stream)

    scene_t = L.Scene(ctx, target)
    step(scene_t)
    b_ref = bm.clone()
    del scene_t
    ws_r = L._workspace(L.us_simulate_rf_vjp_workspace_size(scene, probe, wl.n_tx, wl.rays_per_tx,
                                                            wl.max_bounces), dev)
    ws_bv = L._workspace(L.load().us_beamform_vjp_workspace_size(probe.handle, wl.n_tx), dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    ws_l = L._workspace(L.load().us_image_loss_workspace_size(g.n_px), dev)
    g_b = torch.empty_like(bm)
    g_iq = torch.empty_like(iq)
    g_rf = torch.empty_like(rf)
    g_theta = torch.zeros(scene.n_params, dtype=torch.float64, device=dev)

    def step_fb():
        step()
        L.us_image_loss(ctx, bm, b_ref, 0.0, 1.0, loss=loss, g_bmode=g_b, workspace=ws_l, stream=stream)
        L.us_bmode_vjp(ctx, iq, g_b, wl.dr_db, g_iq=g_iq, workspace=ws_m, stream=stream)
        L.us_beamform_vjp(ctx, probe, g, wl.angles, wl.tx_ids, g_iq, g_rf=g_rf, workspace=ws_bv,
                          stream=stream)
        g_theta.zero_()
        L.us_simulate_rf_vjp(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                             wl.max_bounces, g_rf, g_theta=g_theta, workspace=ws_r, stream=stream)

    # the same backward as one us_frame_vjp call (fused analytic + pulse adjoints)
    ws_f = L._workspace(L.us_frame_vjp_workspace_size(scene, probe, g, wl.n_tx, wl.rays_per_tx,
                                                      wl.max_bounces), dev) if backward else None
    g_theta_f = torch.zeros_like(g_theta)

    def step_fb_fused():
        step()
        L.us_image_loss(ctx, bm, b_ref, 0.0, 1.0, loss=loss, g_bmode=g_b, workspace=ws_l, stream=stream)
        g_theta_f.zero_()
        L.us_frame_vjp(ctx, scene, probe, g, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem, wl.max_bounces,
                       iq, g_b, wl.dr_db, g_theta=g_theta_f, workspace=ws_f, stream=stream)

    # a recorded frame: the forward keeps the path records, and the one-call
    # backward reads them instead of tracing the paths again
    rec_bytes = L.us_recorded_workspace_size(scene, probe, wl.n_tx, wl.rays_per_tx, wl.max_bounces) \
        if backward else 0
    ws_rec = L._workspace(rec_bytes, dev) if rec_bytes else None
    ws_fr = L._workspace(L.us_frame_vjp_recorded_workspace_size(probe, g, wl.n_tx), dev) if rec_bytes else None
    g_theta_r = torch.zeros_like(g_theta)
    rf_r = torch.empty_like(rf)

    def step_fb_recorded():
        _, rec = L.us_simulate_rf_recorded(ctx, scene, probe, wl.angles, wl.tx_ids, wl.seed, wl.rays_per_elem,
                                           wl.max_bounces, rf=rf_r, workspace=ws_rec, stream=stream)
        L.us_beamform(ctx, probe, g, wl.angles, wl.tx_ids, rf_r, iq=iq, workspace=ws_b, stream=stream)
        L.us_bmode(ctx, iq, wl.dr_db, out=bm, workspace=ws_m, stream=stream)
        L.us_image_loss(ctx, bm, b_ref, 0.0, 1.0, loss=loss, g_bmode=g_b, workspace=ws_l, stream=stream)
        g_theta_r.zero_()
        L.us_frame_vjp_recorded(ctx, rec, g, iq, g_b, wl.dr_db, g_theta=g_theta_r, workspace=ws_fr, stream=stream)

    step(cnt=counters)                  # event counts of one frame (deterministic)
    torch.cuda.synchronize()
    counts = [int(v) for v in counters.cpu().numpy()]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        L.us_profile_enable(ctx, True)
        L.us_profile_read(ctx)          # clear
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            fn()
        end.record(stream)
        torch.cuda.synchronize()
        prof = L.us_profile_read(ctx)
        L.us_profile_enable(ctx, False)
        return start.elapsed_time(end) / steps, prof

    def kernel_table(prof):
        out = {}
        for name, (ms, launches) in prof.items():
            per_step_ms = ms / steps
            nbytes = kernel_bytes(name, wl, counts, g.n_px)
            out[name] = {"ms_per_step": round(per_step_ms, 4), "launches_per_step": launches // steps,
                         "avg_launch_us": round(1e3 * ms / max(1, launches), 2),
                         "algorithmic_GBps": round(nbytes / (per_step_ms * 1e-3) / 1e9, 1) if nbytes else None}
        return out

    fwd_ms, prof = timed(step)
    fb_ms, prof_fb = timed(step_fb) if backward else (float("nan"), {})
    fused = None
    if backward:
        fused_ms, prof_fused = timed(step_fb_fused)
        step_fb()                       # the plain chain's gradient of the same frame
        torch.cuda.synchronize()
        fused = {"ms_per_step": round(fused_ms, 4), "frames_per_s": round(1e3 / fused_ms, 2),
                 "plain_ms_per_step": round(fb_ms, 4), "speedup_vs_plain": round(fb_ms / fused_ms, 4),
                 "gradient_bitwise_equal_to_plain": bool(torch.equal(g_theta, g_theta_f)),
                 "kernels": kernel_table(prof_fused)}
    recorded = None
    if rec_bytes:
        rec_ms, prof_rec = timed(step_fb_recorded)
        step_fb()
        torch.cuda.synchronize()
        rf_plain = rf.clone()
        step_fb_recorded()
        torch.cuda.synchronize()
        recorded = {"ms_per_step": round(rec_ms, 4), "frames_per_s": round(1e3 / rec_ms, 2),
                    "plain_ms_per_step": round(fb_ms, 4), "speedup_vs_plain": round(fb_ms / rec_ms, 4),
                    "record_GB": round(rec_bytes / 1e9, 2),
                    "rf_bitwise_equal_to_plain": bool(torch.equal(rf_plain, rf_r)),
                    "gradient_bitwise_equal_to_plain": bool(torch.equal(g_theta, g_theta_r)),
                    "kernels": kernel_table(prof_rec)}
    segments = counts[0] + counts[1]
    return {"counts": counts, "segments": segments, "n_params": scene.n_params,
            "fwd_ms": fwd_ms, "prof": prof, "kernels": kernel_table(prof),
            "fb_ms": fb_ms, "fb_kernels": kernel_table(prof_fb), "fused": fused, "recorded": recorded,
            "loss": float(loss.item()) if backward else None}


SEGMENT_BYTES = 120   # per transport segment: queued ray state in and out plus the hit record


def transport_roofline(name, prof, counts, steps, traffic_file):
    """Roofline of transport kernel `name` ("bounce" or "secondary"): its
    segments per launch (primary closest-hit queries for the bounce, receiver
    legs for the secondary rays) times SEGMENT_BYTES, divided by the launch's
    average duration from the HIP events recorded on the launch stream."""
    ms, launches = prof[name]
    per_step = launches // steps
    segs = counts[0] if name == "bounce" else counts[1]
    bytes_per_launch = SEGMENT_BYTES * segs / max(1, per_step)
    avg_s = ms * 1e-3 / max(1, launches)
    achieved = bytes_per_launch / avg_s / 1e9
    traffic = measured_traffic(name, traffic_file)
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": int(traffic) if traffic is not None else None,
            "bytes_per_launch": int(bytes_per_launch), "segments_per_launch": int(segs / max(1, per_step)),
            "avg_launch_us": round(avg_s * 1e6, 2)}


def frame_summary(r, wl, steps):
    counts = r["counts"]
    return {"ms_per_step": round(r["fwd_ms"], 4), "frames_per_s": round(1e3 / r["fwd_ms"], 2),
            "ray_segments_per_s": r["segments"] / (r["fwd_ms"] * 1e-3),
            "segments_per_frame": r["segments"],
            "frame_counts": {"primary_segments": counts[0], "secondary_segments": counts[1],
                             "deposits": counts[2], "interactions": counts[3], "secondary_rays": counts[4]},
            "kernels": r["kernels"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-layered", action="store_true", help="skip the layered-phantom legs")
    ap.add_argument("--no-inverse", action="store_true", help="skip the inverse-loop leg")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--no-backward", action="store_true",
                    help="forward legs only (for short profiler runs)")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="first copy 512 MiB device to device, the reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    from paper_2604_15017_amd import _lib as L
    from paper_2604_15017_amd import workloads as W

    ctx = L.Context(0)
    if args.pmc_calibration:
        import torch
        src = torch.ones(CALIBRATION_BYTES // 4, dtype=torch.float32, device=ctx.torch_device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # headline: the triangle-mesh anatomy phantom (the largest single-GPU workload)
    wa = W.anatomy_phantom()
    a = frame_legs(ctx, wa, W.anatomy_phantom_target(wa), args.steps, args.warmup,
                   backward=not args.no_backward)
    print(f"anatomy phantom: forward {a['fwd_ms']:.3f} ms/frame, forward+backward "
          f"{a['fb_ms']:.3f} ms/frame" + (f" ({a['fused']['ms_per_step']:.3f} fused)" if a["fused"] else "")
          + (f" ({a['recorded']['ms_per_step']:.3f} recorded)" if a["recorded"] else ""),
          file=sys.stderr, flush=True)
    prof, counts = a["prof"], a["counts"]
    transport = [k for k in ("bounce", "secondary") if k in prof]
    dom = max(transport, key=lambda k: prof[k][0])
    other = "secondary" if dom == "bounce" else "bounce"
    roofline = transport_roofline(dom, prof, counts, args.steps, "transport_anatomy_phantom_hbm_traffic.md")
    p, g = wa.probe, wa.grid
    fs = frame_summary(a, wa, args.steps)
    n_tri = sum(len(m.triangles) for m in wa.scene.meshes)
    out = {
        "metric": "ray-segments/s and B-mode frames/s (fwd, fwd+bwd)",
        "value": fs["ray_segments_per_s"],
        "unit": "ray-segments/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": fs["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 transport + f32 image chain",
        "data": "synthetic",
        "config": {"workload": "anatomy_phantom", "triangles": n_tri, "meshes": len(wa.scene.meshes),
                   "n_tx": wa.n_tx, "rays_per_tx": wa.rays_per_tx, "max_bounces": wa.max_bounces,
                   "n_elem": p.n_elem, "n_t": p.n_t, "grid": [g.n_x, g.n_z], "pass": "forward"},
        "frames_per_s": fs["frames_per_s"],
        "segments_per_frame": fs["segments_per_frame"],
        "frame_counts": fs["frame_counts"],
        "kernels": fs["kernels"],
        "roofline": roofline,
        # the other transport kernel of the frame, the same way
        "roofline_" + other: transport_roofline(other, prof, counts, args.steps,
                                                "transport_anatomy_phantom_hbm_traffic.md"),
        "fwd_bwd": None if args.no_backward else {
            "workload": f"anatomy_phantom forward + backward, B-mode MSE vs the perturbed target, "
                        f"gradient of all {a['n_params']} parameters",
            "ms_per_step": round(a["fb_ms"], 4), "frames_per_s": round(1e3 / a["fb_ms"], 2),
            "ray_segments_per_s": a["segments"] / (a["fb_ms"] * 1e-3),
            "loss": a["loss"], "kernels": a["fb_kernels"]},
        "fwd_bwd_fused": a["fused"],
        "fwd_bwd_recorded": a["recorded"],
    }
    if not args.no_layered:
        wl = W.layered_phantom()
        r = frame_legs(ctx, wl, W.layered_phantom_target(wl), args.steps, args.warmup,
                       backward=not args.no_backward)
        print(f"layered phantom: forward {r['fwd_ms']:.3f} ms/frame, forward+backward "
              f"{r['fb_ms']:.3f} ms/frame" + (f" ({r['fused']['ms_per_step']:.3f} fused)" if r["fused"] else "")
              + (f" ({r['recorded']['ms_per_step']:.3f} recorded)" if r["recorded"] else ""),
              file=sys.stderr, flush=True)
        lay = frame_summary(r, wl, args.steps)
        lay["workload"] = (f"layered_phantom: {wl.n_tx} x {wl.rays_per_tx} rays, {wl.max_bounces} interactions, "
                           f"{wl.probe.n_elem} x {wl.probe.n_t} samples, {wl.grid.n_x} x {wl.grid.n_z} pixels")
        lay["roofline"] = transport_roofline("bounce", r["prof"], r["counts"], args.steps,
                                             "transport_layered_phantom_hbm_traffic.md")
        if not args.no_backward:
            lay["fwd_bwd"] = {"ms_per_step": round(r["fb_ms"], 4), "frames_per_s": round(1e3 / r["fb_ms"], 2),
                              "ray_segments_per_s": r["segments"] / (r["fb_ms"] * 1e-3),
                              "gradient_parameters": r["n_params"], "loss": r["loss"],
                              "kernels": r["fb_kernels"]}
            lay["fwd_bwd_fused"] = r["fused"]
            lay["fwd_bwd_recorded"] = r["recorded"]
        out["layered_phantom"] = lay
    if not args.no_backward and not args.no_inverse:
        out["inverse"] = inverse_leg(ctx, args.steps, args.warmup)
        print(f"inverse loop: {out['inverse']['ms_per_iteration']:.3f} ms/iteration "
              f"({out['inverse']['recorded']['ms_per_iteration']:.3f} recorded)", file=sys.stderr, flush=True)
    if not args.no_backward and not args.no_layered:
        out["acquisition_gradients"] = acquisition_leg(ctx, args.steps, args.warmup)
    if not args.no_serving:
        out["serving"] = serving(ctx, args.serve_requests)
    if not args.no_cpu_baseline:
        # 655,360 rays of each of the 21 transmits: 13,762,560 of the frame's
        # 16,777,152 (about 11 s on 16 host cores)
        out["cpu_baseline"] = cpu_baseline(wa, ray_count=5 << 17)
        if "layered_phantom" in out:
            out["layered_phantom"]["cpu_baseline"] = cpu_baseline(W.layered_phantom())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
