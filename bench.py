"""Benchmark of the primary-vertex finding path on one MI355X.

A step is one pv_find call over the whole batch (every stage of the path:
projection, histogram, peak search, association, fit, selection) with the
inputs already resident in HBM.  The default workload is 10,000 synthetic
events at mu = 5 (pp_mu5_10kev).  One JSON line is printed with events/s,
the HBM roofline of the main fused kernel (timed with HIP events on its own
stream), the plain one-launch-per-event rate on the same GPU, and the CPU
oracle timed on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload pp_mu5_10kev]
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "events/s at mu=5 (batched vs per-event launch); p50/p99 latency in served mode"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2412_14966_amd", "csrc", f)
                  for f in ("pvfind_kernels.hip", "pvfind_device.h", "pvfind_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pv_find_hbm_traffic.json")
SQ_FILE = os.path.join(ROOT, "profiles", "pv_find_sq_counters.json")
# VALU issue peak without packed FP32: 256 CUs x 4 SIMDs, each starting one
# wave64 instruction every 4 cycles (16 lanes), at 2.4 GHz
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4.0   # G wave-instructions/s
STAGES = ("clear", "project_fill", "peak_search", "association", "gather", "fit", "selection", "final_outputs")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n_tracks, n_events, n_vertices):
    """Bytes a launch must move at minimum: track SoA read once (8 x 4 B),
    offsets (4 B per event), per-track vertex id + weight (8 B), 64 B per
    vertex record and 8 B per event (count + status)."""
    return 32 * n_tracks + 4 * n_events + 8 * n_tracks + 64 * n_vertices + 8 * n_events


def latency_summary(comp, warm_frac=0.01):
    k = int(len(comp) * warm_frac)
    order = np.argsort(comp["t_arrival_ns"])
    c = comp[order][k:]
    lat = (c["t_done_ns"] - c["t_arrival_ns"]) / 1e3
    span = (comp["t_done_ns"].max() - comp["t_arrival_ns"].min()) / 1e9
    return {"p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
            "achieved_events_per_s": round(len(comp) / span, 1)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pv, batch, params, seconds):
    """The oracle on the host cores: OpenMP over events on every thread it
    may use, and on one thread, each on a bounded sample of the workload."""
    import oracle
    op = oracle.params_from_fields(pv.params_dict(params))
    threads = oracle.max_threads()
    done, passes, t1 = 0, 0, time.perf_counter()
    while True:
        oracle.find(batch, op, n_threads=threads)
        done += batch.n_events
        passes += 1
        if time.perf_counter() - t1 >= seconds:
            break
    dt = time.perf_counter() - t1
    # one thread: the first events of the workload, as many as ~seconds/4 take
    n1 = min(batch.n_events, 500)
    t2 = time.perf_counter()
    oracle.find(batch.select(range(n1)), op, n_threads=1)
    d1 = time.perf_counter() - t2
    n_one = int(min(batch.n_events, max(n1, n1 * (seconds / 4.0) / max(d1, 1e-6))))
    if n_one > n1:
        t2 = time.perf_counter()
        oracle.find(batch.select(range(n_one)), op, n_threads=1)
        d1 = time.perf_counter() - t2
    else:
        n_one = n1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    cpu = {"value": round(done / dt, 1), "unit": "events/s", "cores": threads, "kind": "oracle",
           "sample": f"{passes} pass(es) over the same {batch.n_events}-event workload, {dt:.1f} s wall, "
                     f"OpenMP over events on {threads} threads",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "cpus_usable": affinity,
           "one_core": {"value": round(n_one / d1, 1), "unit": "events/s", "cores": 1,
                        "sample": f"the first {n_one} events of the workload, {d1:.1f} s wall"}}
    log(f"cpu oracle: {cpu['value']} events/s on {threads} threads, {cpu['one_core']['value']} on one "
        f"({cpu['cpu_model']})")
    return cpu


def end_to_end_leg(pv, batch, params, steps):
    """The batched path with its PCIe transfers, as the paper's throughput
    includes them: per step, the eight track columns and the offsets go from
    pinned host memory to the device, pv_find runs, the written vertex
    records are gathered into a dense array (pv_compact_vertices), and the
    vertex counts, statuses, per-event record offsets and per-track outputs
    come back, then the dense records (their total read from the first copy);
    one stream, synchronised per step."""
    import torch
    ne, nt, mv = batch.n_events, batch.n_tracks, params.max_vertices_per_event
    host_cols = [torch.from_numpy(np.ascontiguousarray(c)).pin_memory() for c in batch.fields()]
    host_offs = torch.from_numpy(np.ascontiguousarray(batch.offsets, dtype=np.int32)).pin_memory()
    db = pv.to_device(batch)
    out = pv.alloc_outputs(db, mv)
    dense = torch.empty(ne * mv * 64, dtype=torch.uint8, device=out.vertices.device)
    first = torch.empty(ne + 1, dtype=torch.int32, device=out.vertices.device)
    h_nv = torch.empty(ne, dtype=torch.int32).pin_memory()
    h_st = torch.empty(ne, dtype=torch.int32).pin_memory()
    h_first = torch.empty(ne + 1, dtype=torch.int32).pin_memory()
    h_tv = torch.empty(nt, dtype=torch.int32).pin_memory()
    h_tw = torch.empty(nt, dtype=torch.float32).pin_memory()
    h_v = torch.empty(ne * mv * 64, dtype=torch.uint8).pin_memory()
    stream = torch.cuda.current_stream()
    moved = [0, 0]

    def step():
        for d, h in zip(db.cols, host_cols):
            d.copy_(h, non_blocking=True)
        db.offsets.copy_(host_offs, non_blocking=True)
        pv.pv_find(db, out, params)
        pv.pv_compact_vertices(out, ne, dense, first)
        h_nv.copy_(out.n_vertices, non_blocking=True)
        h_st.copy_(out.status, non_blocking=True)
        h_first.copy_(first, non_blocking=True)
        h_tv.copy_(out.track_vertex, non_blocking=True)
        h_tw.copy_(out.track_weight, non_blocking=True)
        stream.synchronize()
        nbytes = 64 * int(h_first[ne])
        h_v[:nbytes].copy_(dense[:nbytes], non_blocking=True)
        stream.synchronize()
        moved[0] = 32 * nt + 4 * (ne + 1)
        moved[1] = 8 * ne + 4 * (ne + 1) + 8 * nt + nbytes

    for _ in range(3):
        step()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    dt = (time.perf_counter() - t0) / steps
    res = {"events_per_s": round(ne / dt, 1), "ms_per_step": round(dt * 1e3, 4), "h2d_bytes": moved[0],
           "d2h_bytes": moved[1], "pcie_gbs": round((moved[0] + moved[1]) / dt / 1e9, 2),
           "vertex_records": int(h_first[ne])}
    log(f"end to end with H2D/D2H: {res['events_per_s']:.4g} events/s ({res['ms_per_step']:.3f} ms per step, "
        f"{res['pcie_gbs']} GB/s over PCIe)")
    del db, out, dense
    return res


def end_to_end_streams_leg(pv, batch, params, steps, chunks=2, n_streams=2):
    """The same transfers with the batch cut into `chunks` contiguous event
    ranges issued round robin on `n_streams` streams (the paper overlaps
    transfers and kernels on several streams, Sec. 6): per range, its tracks
    and offsets go in, pv_find and the compaction run on the range, and its
    counts, statuses, record offsets, records and per-track outputs come
    back, so one range's copies overlap another's kernels and copies in the
    other direction.  The records' copy is sized before their number is
    known (2 per event plus 1 per 16 tracks of the range); a range with more
    gets a second copy after the step (counted).  Two ranges on two streams
    measured best: with more, the per-copy overheads of the 8 column copies
    per range outweigh the overlap."""
    import torch
    L = pv.lib()
    ne, nt, mv = batch.n_events, batch.n_tracks, params.max_vertices_per_event
    offs = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    host_cols = [torch.from_numpy(np.ascontiguousarray(c)).pin_memory() for c in batch.fields()]
    host_offs = torch.from_numpy(np.ascontiguousarray(batch.offsets, dtype=np.int32)).pin_memory()
    db = pv.to_device(batch)
    out = pv.alloc_outputs(db, mv)
    dev = out.vertices.device
    dense = torch.empty(ne * mv * 64, dtype=torch.uint8, device=dev)      # range c's records from 64 * mv * e0
    first = torch.empty(ne + chunks, dtype=torch.int32, device=dev)       # range c's offsets from e0 + c
    h_nv = torch.empty(ne, dtype=torch.int32).pin_memory()
    h_st = torch.empty(ne, dtype=torch.int32).pin_memory()
    h_first = torch.empty(ne + chunks, dtype=torch.int32).pin_memory()
    h_tv = torch.empty(nt, dtype=torch.int32).pin_memory()
    h_tw = torch.empty(nt, dtype=torch.float32).pin_memory()
    h_v = torch.empty(ne * mv * 64, dtype=torch.uint8).pin_memory()
    streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
    bounds = [int(round(ne * c / chunks)) for c in range(chunks + 1)]
    tr, bl, _, _ = pv._args(db, out, params)
    ot = pv.pv_track_out(out.track_vertex.data_ptr(), out.track_weight.data_ptr())
    stats = {"second_copies": 0, "d2h": 0}

    def step():
        budget = []
        for c in range(chunks):
            e0, e1 = bounds[c], bounds[c + 1]
            t0, t1 = int(offs[e0]), int(offs[e1])
            n = e1 - e0
            s = streams[c % n_streams]
            st = ctypes.c_void_p(s.cuda_stream)
            with torch.cuda.stream(s):
                for d, h in zip(db.cols, host_cols):
                    d[t0:t1].copy_(h[t0:t1], non_blocking=True)
                db.offsets[e0:e1 + 1].copy_(host_offs[e0:e1 + 1], non_blocking=True)
            vo = out.vertices.data_ptr() + 64 * mv * e0
            ov = pv.pv_vertices_out(vo, out.n_vertices.data_ptr() + 4 * e0, out.status.data_ptr() + 4 * e0)
            rc = L.pv_find(ctypes.byref(tr), ctypes.c_void_p(db.offsets.data_ptr() + 4 * e0), n, ctypes.byref(bl),
                           ctypes.byref(params), ctypes.byref(ov), ctypes.byref(ot), st)
            if rc == 0:
                rc = L.pv_compact_vertices(ctypes.c_void_p(vo), ctypes.c_void_p(out.n_vertices.data_ptr() + 4 * e0), n,
                                           mv, ctypes.c_void_p(dense.data_ptr() + 64 * mv * e0),
                                           ctypes.c_void_p(first.data_ptr() + 4 * (e0 + c)), st)
            if rc != 0:
                raise RuntimeError(pv.pv_last_error())
            nrec = min(mv * n, 2 * n + (t1 - t0) // 16)
            budget.append(nrec)
            with torch.cuda.stream(s):
                h_nv[e0:e1].copy_(out.n_vertices[e0:e1], non_blocking=True)
                h_st[e0:e1].copy_(out.status[e0:e1], non_blocking=True)
                h_first[e0 + c:e1 + c + 1].copy_(first[e0 + c:e1 + c + 1], non_blocking=True)
                b0 = 64 * mv * e0
                h_v[b0:b0 + 64 * nrec].copy_(dense[b0:b0 + 64 * nrec], non_blocking=True)
                h_tv[t0:t1].copy_(out.track_vertex[t0:t1], non_blocking=True)
                h_tw[t0:t1].copy_(out.track_weight[t0:t1], non_blocking=True)
        for s in streams:
            s.synchronize()
        d2h = 0
        for c in range(chunks):
            e0, e1 = bounds[c], bounds[c + 1]
            total = int(h_first[e1 + c])
            d2h += 8 * (e1 - e0) + 4 * (e1 - e0 + 1) + 64 * max(total, budget[c])
            if total > budget[c]:   # the rest of this range's records
                b0 = 64 * mv * e0
                h_v[b0 + 64 * budget[c]:b0 + 64 * total].copy_(dense[b0 + 64 * budget[c]:b0 + 64 * total])
                stats["second_copies"] += 1
        stats["d2h"] = d2h + 8 * nt

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    stats["second_copies"] = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    dt = (time.perf_counter() - t0) / steps
    h2d = 32 * nt + 4 * (ne + chunks)
    res = {"events_per_s": round(ne / dt, 1), "ms_per_step": round(dt * 1e3, 4), "chunks": chunks,
           "streams": n_streams, "h2d_bytes": h2d, "d2h_bytes": stats["d2h"],
           "pcie_gbs": round((h2d + stats["d2h"]) / dt / 1e9, 2),
           "second_copies_per_step": stats["second_copies"] / steps}
    log(f"end to end, {chunks} ranges on {n_streams} streams: {res['events_per_s']:.4g} events/s "
        f"({res['ms_per_step']:.3f} ms per step, {res['pcie_gbs']} GB/s over PCIe)")
    # the outputs equal those of one pv_find over the whole batch (device-resident)
    ref = pv.alloc_outputs(db, mv)
    pv.pv_find(db, ref, params)
    torch.cuda.synchronize()
    res["same_as_one_launch"] = bool(torch.equal(ref.track_vertex, out.track_vertex) and
                                     torch.equal(ref.track_weight.view(torch.int32), out.track_weight.view(torch.int32))
                                     and torch.equal(ref.n_vertices, out.n_vertices)
                                     and torch.equal(ref.status, out.status))
    del db, out, dense, ref
    return res


def served_leg(pv, synth, n_events):
    """Continuous-batching server vs the plain one-launch-per-event server on
    the served mix (mu log-uniform in [1, 40]), host buffers in and out, so
    every figure includes the PCIe transfers."""
    t0 = time.time()
    batch = synth.generate_parallel("served_mulog_200kev", n_events=n_events, workers=8)
    log(f"served mix: generated {batch.n_events} events / {batch.n_tracks} tracks in {time.time() - t0:.1f} s")
    params = pv.make_params({"max_vertices_per_event": 96})
    host = pv.HostEvents(batch, params.max_vertices_per_event)
    rng = np.random.default_rng(7)
    unit = rng.exponential(1.0, n_events)

    def offsets(rate):
        return np.cumsum(unit * (1e9 / rate)).astype(np.int64)

    cfg = pv.pv_server_config_default(max_events_per_batch=1024, max_tracks_per_batch=1024 * 600, n_slots=6,
                                      n_streams=3, max_wait_us=100, use_graphs=1)
    plain_cfg = pv.pv_server_config_default(max_events_per_batch=1, max_tracks_per_batch=4096, n_slots=8,
                                            n_streams=4, max_wait_us=0, use_graphs=1)
    out = {"workload": "served_mulog_200kev", "events": n_events, "tracks": batch.n_tracks,
           "config": {"max_events_per_batch": 1024, "slots": 6, "streams": 3, "max_wait_us": 100, "graphs": 1}}
    warm = batch.select(range(min(n_events, 2048)))
    hw = pv.HostEvents(warm, params.max_vertices_per_event)
    with pv.Server(params, batch.beamline, cfg) as srv:
        srv.replay(hw, np.zeros(warm.n_events, dtype=np.int64))   # warm-up
        # capacity: all events at once, the median of three replays (a single
        # replay of ~30 ms varies by tens of percent)
        caps = [latency_summary(srv.replay(host, np.zeros(n_events, dtype=np.int64)))["achieved_events_per_s"]
                for _ in range(3)]
        burst = float(np.median(caps))
        log(f"served capacity (all {n_events} events at once): {burst:.4g} events/s")
        # Poisson arrivals at that rate form smaller batches (sealed after
        # max_wait_us while the device is busy), which a slow host may not
        # sustain: the load points below are fractions of the throughput
        # achieved when arrivals come at the burst rate, never above it
        sus = latency_summary(srv.replay(host, offsets(burst)))["achieved_events_per_s"]
        cap = float(min(burst, sus))
        log(f"served capacity with Poisson arrivals at that rate: {sus:.4g} events/s")
        out["burst_capacity_events_per_s"] = burst
        out["capacity_events_per_s"] = cap
        # one untimed pass over the rates first: in the first ~0.2 s of a
        # server's life one replay showed a single stall of ~8 ms, once
        for f in (0.5, 0.8, 0.95):
            srv.replay(host, offsets(f * cap))
        rates = []
        for f in (0.5, 0.8, 0.95):
            comp = srv.replay(host, offsets(f * cap))
            rates.append(dict(offered_events_per_s=round(f * cap, 1), **latency_summary(comp)))
            log(f"served at {f:.2f} x capacity: {rates[-1]}")
        out["rates"] = rates
        out["stats"] = srv.stats()
    log(f"served capacity {cap:.4g} events/s; " + ", ".join(f"{r['offered_events_per_s']:.3g}/s: p50 {r['p50_us']} us "
                                                          f"p99 {r['p99_us']} us" for r in rates))
    n_plain = min(n_events, 4000)
    sub = batch.select(range(n_plain))
    hp = pv.HostEvents(sub, params.max_vertices_per_event)
    log(f"plain per-event server on {n_plain} events")
    with pv.Server(params, batch.beamline, plain_cfg) as srv:
        comp = srv.replay(hp, np.zeros(n_plain, dtype=np.int64))
        pcap = latency_summary(comp)["achieved_events_per_s"]
        rate = 0.5 * pcap
        comp = srv.replay(hp, np.cumsum(unit[:n_plain] * (1e9 / rate)).astype(np.int64))
        plain = dict(capacity_events_per_s=pcap, offered_events_per_s=round(rate, 1), **latency_summary(comp))
    with pv.Server(params, batch.beamline, cfg) as srv:
        comp = srv.replay(hp, np.cumsum(unit[:n_plain] * (1e9 / rate)).astype(np.int64))
        plain["batched_server_at_same_rate"] = latency_summary(comp)
    out["plain_per_event"] = plain
    log(f"plain per-event server capacity {pcap:.4g} events/s; at {rate:.3g}/s p50 {plain['p50_us']} us "
        f"p99 {plain['p99_us']} us (batched server: p99 {plain['batched_server_at_same_rate']['p99_us']} us)")
    return out


def batched_leg(pv, synth, workload: str, steps: int, warmup: int) -> dict:
    """Events/s of one further batched workload (beam-gas, high pile-up) under
    the schedule pv_autotune picks for it: steps bracketed by HIP events on the
    current stream, inputs resident in device memory."""
    import torch
    batch = synth.generate(workload, keep_truth=False)
    params = pv.pv_params_default()
    db = pv.to_device(batch)
    out = pv.alloc_outputs(db, params.max_vertices_per_event)
    best, _ = pv.pv_autotune(db, out, params, reps=3)
    sched = pv.pv_schedule(best["waves_per_team"], best["track_capacity"], best["persistent"], best["teams_per_cu"])
    for _ in range(warmup):
        pv.pv_find_sched(db, out, params, sched)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        pv.pv_find_sched(db, out, params, sched)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    res = {"events": batch.n_events, "tracks": batch.n_tracks, "events_per_s": round(batch.n_events / (ms / 1e3), 1),
           "ms_per_step": round(ms, 5), "n_vertices": int(out.n_vertices.sum().item()), "schedule": best}
    log(f"{workload}: {res['events_per_s']:.4g} events/s under {best}")
    # the multi-vertex variant (Eq. 18) on the same batch and schedule
    mvp = pv.make_params({"assoc_mode": 1})
    for _ in range(warmup):
        pv.pv_find_sched(db, out, mvp, sched)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        pv.pv_find_sched(db, out, mvp, sched)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    res["multivertex"] = {"events_per_s": round(batch.n_events / (ms / 1e3), 1), "ms_per_step": round(ms, 5),
                          "n_vertices": int(out.n_vertices.sum().item())}
    log(f"{workload} multi-vertex: {res['multivertex']['events_per_s']:.4g} events/s")
    del db, out
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pp_mu5_10kev")
    ap.add_argument("--per-event-sample", type=int, default=2000,
                    help="events timed with one launch each (plain form)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", default="",
                    help="waves,capacity,persistent,teams_per_cu (default: chosen by pv_autotune on the batch)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (HBM counter calibration)")
    ap.add_argument("--served-events", type=int, default=200000,
                    help="events of the served mix replayed per offered rate (0 skips the served leg)")
    ap.add_argument("--e2e-steps", type=int, default=10,
                    help="steps of the PCIe-inclusive end-to-end leg (0 skips it)")
    ap.add_argument("--batched-configs", default="pp_mu5_gas_50kev,pp_mu40_20kev",
                    help="further batched workloads timed last, each under its own autotuned schedule "
                         "(empty skips them)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): events are independent, so the "
              f"path shards by event range across GPUs without any exchange; bench.py measures one GPU.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_14966_amd import pvfind as pv
    from paper_2412_14966_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.time()
    batch = synth.generate(args.workload, keep_truth=False)
    log(f"generated {batch.n_events} events / {batch.n_tracks} tracks in {time.time() - t0:.1f} s")
    params = pv.pv_params_default()
    if args.schedule:
        w, c, m, t = (int(v) for v in args.schedule.split(","))
        pv.pv_set_schedule(w, c, m, t)

    if args.calibrate_copy_mib > 0:
        # a plain copy kernel reading and writing a known number of bytes
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy_mib} MiB read + written")
        del src, dst

    db = pv.to_device(batch, dev)
    out = pv.alloc_outputs(db, params.max_vertices_per_event, dev)
    tuned_us = None
    if not args.schedule:
        best, tuned_us = pv.pv_autotune(db, out, params, reps=5)
        log(f"autotuned schedule {best}: {tuned_us:.1f} us per launch")
    s = pv.pv_get_schedule()
    schedule = dict(waves_per_team=s.waves_per_team, track_capacity=s.track_capacity, persistent=s.persistent,
                    teams_per_cu=s.teams_per_cu, autotuned=not args.schedule)
    stream = torch.cuda.current_stream()
    L = pv.lib()
    tr, bl, ov, ot = pv._args(db, out, params)
    offs = ctypes.c_void_p(db.offsets.data_ptr())
    st = ctypes.c_void_p(stream.cuda_stream)
    args_ref = (ctypes.byref(tr), offs, db.n_events, ctypes.byref(bl), ctypes.byref(params), ctypes.byref(ov),
                ctypes.byref(ot), st)

    def step():
        rc = L.pv_find(*args_ref)
        if rc != 0:
            raise RuntimeError(pv.pv_last_error())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps bracketed by synchronisations
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    value = batch.n_events / (ms_per_step / 1e3)
    log(f"batched: {ms_per_step * 1e3:.1f} us per step, {value:.4g} events/s")

    # per-kernel durations of the same steps, from events the library records
    pv.pv_timing_start()
    for _ in range(args.steps):
        step()
    main_ms, large_ms, ncalls = pv.pv_timing_stop()
    main_us = main_ms / ncalls * 1e3
    large_us = large_ms / ncalls * 1e3
    log(f"main fused kernel {main_us:.1f} us, large-event kernel {large_us:.1f} us per step")

    # spread of single steps: one event pair around each of K more steps
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    marks[0].record(stream)
    for k in range(args.steps):
        step()
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    per_step = np.array([marks[k].elapsed_time(marks[k + 1]) * 1e3 for k in range(args.steps)])
    step_us = {"median": round(float(np.median(per_step)), 2), "p10": round(float(np.percentile(per_step, 10)), 2),
               "p90": round(float(np.percentile(per_step, 90)), 2)}

    nv = int(out.n_vertices.sum().item())
    abytes = algorithmic_bytes(batch.n_tracks, batch.n_events, nv)
    achieved = abytes / (main_us * 1e-6) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tf = json.load(f)
        # modes 2 and 4 run the same kernel, so (waves, capacity) names it
        sched_key = [schedule["waves_per_team"], schedule["track_capacity"]]
        if (tf.get("kernel_sha") == kernel_hash() and tf.get("workload") == args.workload
                and (tf.get("schedule") or [])[:2] == sched_key):
            traffic = tf.get("hbm_bytes_per_launch")
    # the second bound: LDS bytes of the same launch (from the shader counters
    # of a profiled run of this kernel source) against the LDS read bandwidth
    # measured now by the library's microbenchmark
    lds_peak_bs, lds_wg = pv.pv_measure_lds_peak()
    lds = {"bound": "lds", "peak": round(lds_peak_bs / 1e9, 1), "unit": "GB/s",
           "peak_source": f"pv_measure_lds_peak: {lds_wg} workgroups of 256 threads, 16-byte conflict-free reads",
           "achieved": None, "frac": None, "lds_bytes_per_launch": None}
    # what does bound it: VALU issue, from the same profiled run's instruction count
    valu = {"bound": "valu_issue", "peak": VALU_PEAK_GINST, "unit": "G wave-instructions/s",
            "peak_source": "256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 VALU instruction (no packed FP32)",
            "achieved": None, "frac": None, "insts_per_launch": None, "lane_utilisation": None}
    if os.path.exists(SQ_FILE):
        with open(SQ_FILE) as f:
            lf = json.load(f)
        sched_key = [schedule["waves_per_team"], schedule["track_capacity"]]
        if (lf.get("kernel_sha") == kernel_hash() and lf.get("workload") == args.workload
                and (lf.get("schedule") or [])[:2] == sched_key):
            lb = lf.get("lds_bytes_per_launch")
            lds.update(lds_bytes_per_launch=lb, achieved=round(lb / (main_us * 1e-6) / 1e9, 1),
                       frac=round(lb / (main_us * 1e-6) / lds_peak_bs, 4),
                       bank_conflict_cycle_frac=lf.get("bank_conflict_cycle_frac"))
            vi = lf.get("valu_insts_per_launch")
            va = vi / (main_us * 1e-6) / 1e9
            valu.update(insts_per_launch=vi, achieved=round(va, 1), frac=round(va / VALU_PEAK_GINST, 4),
                        lane_utilisation=lf.get("valu_lane_utilisation"))
    log(f"LDS read peak {lds['peak']} GB/s; main kernel LDS {lds['achieved']} GB/s; VALU issue {valu['frac']}")
    kname = f"pv_find_single<{schedule['waves_per_team']}, {schedule['track_capacity']}> (main fused launch)"
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "algorithmic_bytes_per_launch": abytes,
                "kernel_us": round(main_us, 2), "large_event_kernel_us": round(large_us, 2), "lds": lds,
                "valu": valu}

    # where an event's time goes: the kernel's own clock stamps between its
    # steps (the debug form of the same kernel, only the stamps written;
    # shader-clock cycles per event, mean over the batch)
    cyc = torch.zeros(db.n_events * 8, dtype=torch.int32, device=dev)
    dbg = pv.pv_debug_out(None, None, None, None, None, None, cyc.data_ptr())
    rc = L.pv_find_debug(ctypes.byref(tr), offs, db.n_events, ctypes.byref(bl), ctypes.byref(params),
                         ctypes.byref(ov), ctypes.byref(ot), ctypes.byref(dbg), None, st)
    if rc != 0:
        raise RuntimeError(pv.pv_last_error())
    c = cyc.cpu().numpy().view(np.uint32).reshape(db.n_events, 8).astype(np.float64)
    stage_cycles = {n: round(float(c[:, k].mean()), 1) for k, n in enumerate(STAGES)}
    stage_cycles["total"] = round(float(c.sum(axis=1).mean()), 1)
    log(f"cycles per event by step: {stage_cycles}")

    # the GPU variant of the association and fit (Eq. 18 weights over every
    # candidate), same batch and schedule, same timing
    mvp = pv.make_params({"assoc_mode": 1})
    mv_args = (ctypes.byref(tr), offs, db.n_events, ctypes.byref(bl), ctypes.byref(mvp), ctypes.byref(ov),
               ctypes.byref(ot), st)
    for _ in range(args.warmup):
        if L.pv_find(*mv_args) != 0:
            raise RuntimeError(pv.pv_last_error())
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        L.pv_find(*mv_args)
    ev1.record(stream)
    torch.cuda.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / args.steps
    pv.pv_timing_start()
    for _ in range(args.steps):
        L.pv_find(*mv_args)
    mv_main_ms, mv_large_ms, mv_n = pv.pv_timing_stop()
    multivertex = {"events_per_s": round(batch.n_events / (mv_ms / 1e3), 1), "ms_per_step": round(mv_ms, 5),
                   "kernel_us": round(mv_main_ms / mv_n * 1e3, 2),
                   "large_event_kernel_us": round(mv_large_ms / mv_n * 1e3, 2),
                   "n_vertices": int(out.n_vertices.sum().item())}
    log(f"multi-vertex variant: {mv_ms * 1e3:.1f} us per step, {multivertex['events_per_s']:.4g} events/s")

    # plain form: one pv_find launch per event on the same stream
    n_pe = min(args.per_event_sample, batch.n_events)
    mv = params.max_vertices_per_event
    base_v, base_n, base_s = out.vertices.data_ptr(), out.n_vertices.data_ptr(), out.status.data_ptr()
    obase = db.offsets.data_ptr()
    per_event_args = []
    for e in range(n_pe):
        ove = pv.pv_vertices_out(base_v + e * mv * 64, base_n + 4 * e, base_s + 4 * e)
        per_event_args.append((ove, ctypes.c_void_p(obase + 4 * e)))
    for e in range(min(50, n_pe)):
        L.pv_find(ctypes.byref(tr), per_event_args[e][1], 1, ctypes.byref(bl), ctypes.byref(params),
                  ctypes.byref(per_event_args[e][0]), ctypes.byref(ot), st)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    ev0.record(stream)
    for e in range(n_pe):
        rc = L.pv_find(ctypes.byref(tr), per_event_args[e][1], 1, ctypes.byref(bl), ctypes.byref(params),
                       ctypes.byref(per_event_args[e][0]), ctypes.byref(ot), st)
        if rc != 0:
            raise RuntimeError(pv.pv_last_error())
    ev1.record(stream)
    torch.cuda.synchronize()
    host_s = time.perf_counter() - t_host
    pe_ms = ev0.elapsed_time(ev1)
    per_event = {"events_per_s": round(n_pe / (pe_ms / 1e3), 1), "events_timed": n_pe,
                 "us_per_event": round(pe_ms * 1e3 / n_pe, 2), "host_wall_s": round(host_s, 3),
                 # main + large-event launches (a single event needs no ordering launch)
                 "launches_per_event": 2,
                 "batched_speedup": round(value / (n_pe / (pe_ms / 1e3)), 1)}
    log(f"per-event launches: {per_event['us_per_event']} us/event")

    # CPU oracle on a bounded sample (test infrastructure, timed as a baseline)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pv, batch, params, args.cpu_seconds)

    # the served leg before the multi-stream ones: streams torch hands out stay
    # mapped to the process's few hardware queues and would share them with
    # the server's
    served = None
    if args.served_events > 0:
        served = served_leg(pv, synth, args.served_events)

    e2e = end_to_end_leg(pv, batch, params, args.e2e_steps) if args.e2e_steps > 0 else None
    if e2e is not None:
        e2e["streams"] = end_to_end_streams_leg(pv, batch, params, args.e2e_steps)

    # last, because each autotune run changes the library's default schedule
    batched_configs = {}
    for wl in (w for w in args.batched_configs.split(",") if w):
        batched_configs[wl] = batched_leg(pv, synth, wl, args.steps, args.warmup)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n_events": batch.n_events, "n_tracks": batch.n_tracks,
                   "n_vertices": nv, "schedule": schedule},
        "step_us": step_us, "roofline": roofline, "stage_cycles": stage_cycles, "cpu_baseline": cpu,
        "per_event_launch": per_event,
        "multivertex": multivertex, "end_to_end_pcie": e2e, "served": served, "batched_configs": batched_configs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
