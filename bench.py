#!/usr/bin/env python3
"""Benchmark of the TimePix3 VMI hot path on one MI355X.

One step = tpx_process_stream over the whole synthetic c2 workload (100,000
laser shots at 1 kHz, Poisson(30) hits per shot, spot sigma U(0.6, 1.5) px,
10 % close pairs, TPX3 packets with spidr/ToA rollover and trigger words)
with flush: decode, unwrap, shot assignment with the ToF cut, clustering and
centroids of every hit.  The packets are resident in HBM before timing; each
step starts from a fresh stream state.

Prints one JSON line: pixel events/s (kept events that were clustered and
centroided), the roofline of the dominant kernel (algorithmic bytes over its
measured duration, HIP events on the stream it runs on), the oracle's
throughput on a bounded sample on the host CPU, and p50/p99 chunk latency of a
chunked c5 replay.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HIT_BYTES = 48
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_c2_full.md")
STAGE_KERNEL = {"tile_summary": "k_tile_summary", "assign": "k_assign", "cluster": "k_cluster",
                "centroid": "k_seg_centroid"}
FUSED_KERNEL = "k_cluster_fused"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_bytes(n_packets, n_events, n_hits, fused):
    """Bytes each stage's kernels must move at least (inputs read once,
    outputs written once): packets 8 B, packed events 8 B, component ranks
    4 B, hits 48 B.  The fused clustering kernel reads the packed events and
    writes the hits; the staged ones pass ranks between two launches."""
    if fused:
        cl, ce = 8 * n_events + HIT_BYTES * n_hits, 0
    else:
        cl, ce = 8 * n_events + 4 * n_events, 12 * n_events + HIT_BYTES * n_hits
    return {"tile_summary": 8 * n_packets, "tile_prefix": 0,
            "assign": 8 * n_packets + 8 * n_events, "group": 0, "cluster": cl, "centroid": ce,
            "carry": 0}


KERNEL_SOURCES = ("tpx_decode.hip", "tpx_cluster.hip", "tpx_util.hip", "tpx_internal.h",
                  "tpx_kernels.h", "tpx_decode_dev.h", "tpx_util_dev.h")


def source_digest():
    """sha256 over the code (comments and blank lines removed) of the sources
    that define and launch the stream path's kernels: HBM traffic counters are
    only reported while the code they were taken on is unchanged."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_04942_amd", "csrc")
    files = [os.path.join(csrc, f) for f in KERNEL_SOURCES]
    for f in files + [os.path.join(ROOT, "include", "tpx.h")]:
        with open(f) as fh:
            code = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = "\n".join(ln.rstrip() for ln in re.sub(r"//[^\n]*", "", code).splitlines()
                         if ln.strip())
        h.update(os.path.basename(f).encode() + b"\0" + code.encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch of `kernel` from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when absent or taken
    on other sources."""
    try:
        with open(PMC_SUMMARY) as f:
            text = f.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != source_digest():
        return None
    k = blob.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes"]


def run_gpu(args, wl):
    import torch

    import paper_2603_04942_amd as tpx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pk = torch.from_numpy(wl.packets.view(np.int64)).to(dev)
    n = pk.numel()
    kw = dict(pix_epoch0=wl.pix_epoch0, tdc_epoch0=wl.tdc_epoch0)
    s = tpx.Stream(n, **kw)
    cap = n // 4 + 1024
    hits = torch.empty((cap, 48), dtype=torch.uint8, device=dev)
    # clustering kernel and segment stride: the library's autotuner on the
    # workload itself (every kernel at each candidate stride, best of 2)
    # (or the pair given by --kernel / --stride: counter runs, whose timings
    # the counters distort)
    if args.kernel is not None or args.stride is not None:
        if args.kernel is not None:
            s.set_kernel(args.kernel)
        if args.stride is not None:
            s.set_segment(args.stride)
        best_q, best_k, sweep = s.segment(), s.kernel(), {}
    else:
        kernels = list(range(-1, tpx.kernel_count()))
        best_q, best_k, sweep = s.autotune(pk, True, args.c2_strides, hits, cap, reps=2,
                                           kernels=kernels)
    tune = dict(stride=best_q, kernel=best_k, kernel_name=tpx.kernel_name(best_k),
                pinned=not sweep,
                sweep_ms={f"{tpx.kernel_name(k)} @ {q}": round(v, 4)
                          for (k, q), v in sweep.items()})
    log(f"c2 autotune: {tune}")
    fresh = s.get_state()
    s.set_timing(True)

    def step():
        s.set_state(fresh)
        rc, nh, st = s.process_raw(pk, True, hits, cap)
        if rc != 0:
            raise tpx.TpxError(rc, "tpx_process_stream", s.lib.tpx_last_error().decode())
        return nh, st

    if args.copy_calib_mb:
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the HBM traffic counters of the kernels above
        nb = args.copy_calib_mb << 20
        src = torch.ones(nb // 8, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        nh, st = step()
    torch.cuda.synchronize()
    stages = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nh, st = step()
        for k, v in s.stage_times_ms().items():
            stages[k] = stages.get(k, 0.0) + v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    stages = {k: v / args.steps for k, v in stages.items()}
    stats = st.as_dict()
    stats["n_hits"] = nh
    s.close()
    return ms, stages, stats, tune


def run_latency(args):
    """Chunked replay of the c5 stream (1 kHz, Poisson(100) hits per shot, a
    pixel-counter wrap inside).  For each chunk size: back-to-back chunks
    (saturated: latency = processing time of one chunk), and paced replays in
    which chunk k is released when its last word would have been acquired at
    speedup x; latency = completion - release."""
    import torch

    import paper_2603_04942_amd as tpx
    import synth

    w = synth.make_config("c5", n_shots=args.latency_shots, with_truth=False,
                          workers=args.workers)
    pk = torch.from_numpy(w.packets.view(np.int64)).cuda()
    n_pk = pk.numel()
    acq_s = args.latency_shots * 1e-3          # 1 kHz
    pk_rate = n_pk / acq_s                     # packets per second of acquisition
    out = dict(workload=f"c5: 1 kHz, Poisson(100) hits/shot, sigma 0.8 px, {args.latency_shots} "
                        f"shots, {n_pk} packets, a pixel-counter wrap inside",
               sizes=[])
    for chunk in args.latency_chunks:
        s = tpx.Stream(chunk, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
        hits = torch.empty((chunk, 48), dtype=torch.uint8, device="cuda")
        starts = list(range(0, n_pk, chunk))

        def replay(limit, speed):
            s.set_state(fresh)
            lat, n_ev = [], 0
            t0 = time.perf_counter()
            for i, a in enumerate(starts[:limit]):
                last = i == len(starts) - 1 or i == limit - 1
                rel = t0 + (min(a + chunk, n_pk) / pk_rate / speed if speed else 0.0)
                if speed:
                    while time.perf_counter() < rel:
                        pass
                else:
                    rel = time.perf_counter()
                rc, nh, st = s.process_raw(pk[a:a + chunk], last, hits, chunk)
                lat.append((time.perf_counter() - rel) * 1e3)
                if rc != 0:
                    raise tpx.TpxError(rc, "tpx_process_stream", s.lib.tpx_last_error().decode())
                n_ev += st.n_events
            return np.array(lat), n_ev, time.perf_counter() - t0

        # segment stride for this chunk size: the one with the lowest p99 of
        # a back-to-back replay of (up to 1,500 of) the chunks
        fresh = s.get_state()
        q_sweep = {}
        for q in (256, 512, 1024):
            s.set_segment(q)
            replay(min(len(starts), 8), 0)
            lat_q, _, _ = replay(min(len(starts), 1500), 0)
            q_sweep[q] = (float(np.percentile(lat_q, 50)), float(np.percentile(lat_q, 99)))
        q_best = min(q_sweep, key=lambda q: q_sweep[q][1])
        s.set_segment(q_best)
        replay(min(len(starts), 8), 0)           # warm-up
        lat, n_ev, span = replay(len(starts), 0)
        row = dict(chunk_packets=chunk, chunk_kib=chunk * 8 // 1024, chunks=len(starts),
                   stride=q_best,
                   stride_sweep_p50_p99_ms={q: (round(a, 4), round(b, 4))
                                            for q, (a, b) in q_sweep.items()},
                   p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                   events_per_s=n_ev / span, replay_capacity=acq_s / span, paced={})
        for speed in args.latency_speeds:
            # bound each paced run to about 2 s of wall time
            lim = max(1, min(len(starts), int(2.0 * pk_rate * speed / chunk)))
            lat_p, _, _ = replay(lim, speed)
            row["paced"][f"{speed:g}x"] = dict(chunks=lim, p50_ms=float(np.percentile(lat_p, 50)),
                                               p99_ms=float(np.percentile(lat_p, 99)))
        s.set_patches(True)   # the refinement needs the hit of every event
        row["refined"] = refined_replay(args, tpx, s, fresh, pk, chunk, hits, starts)
        s.set_patches(False)
        s.close()
        del hits
        row["paced_batched"] = batched_replays(args, tpx, w, pk, chunk, pk_rate, q_best)
        row["paced_batched_threaded"] = threaded_replays(args, tpx, w, pk, chunk, pk_rate, q_best)
        out["sizes"].append(row)
    return out


def refined_replay(args, tpx, s, fresh, pk, chunk, hits, starts):
    """The whole streaming loop per chunk, back-to-back: decode -> cluster ->
    centroid (tpx_process_stream), then the learned refinement of the chunk's
    hits (tpx_stream_patches, forward, refine).  Latency does not depend on
    the weights; an untrained network of the same shape is used."""
    import torch

    import synth

    mlp = tpx.Mlp(synth.init_mlp_params(4001, zero_last=True), batch=16)
    n_pk = pk.numel()

    def one(a, last):
        rc, nh, st = s.process_raw(pk[a:a + chunk], last, hits, chunk)
        if rc != 0:
            raise tpx.TpxError(rc, "tpx_process_stream", s.lib.tpx_last_error().decode())
        if nh:
            tpx.refine(hits[:nh], mlp.forward(s.patches(hits, nh)))
        torch.cuda.synchronize()
        return nh

    s.set_state(fresh)
    for i, a in enumerate(starts[:8]):
        one(a, i == 7)
    s.set_state(fresh)
    lat, n_h = [], 0
    t0 = time.perf_counter()
    for i, a in enumerate(starts):
        t = time.perf_counter()
        n_h += one(a, i == len(starts) - 1)
        lat.append((time.perf_counter() - t) * 1e3)
    span = time.perf_counter() - t0
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                hits_per_s=n_h / span, replay_capacity=args.latency_shots * 1e-3 / span)


def batched_replays(args, tpx, w, pk, chunk, pk_rate, q):
    """Paced replays through tpx_service from one thread: every chunk released
    so far is admitted, then one run takes all of them (up to the batch
    limit); when chunks arrive faster than one call per chunk can finish,
    several go into one call.  Latency of a chunk = completion of its run -
    its release."""
    import ctypes

    import torch

    n_pk = pk.numel()
    starts = list(range(0, n_pk, chunk))
    max_batch = max(1 << 19, 4 * chunk)
    cap = 2 * max_batch
    hits = torch.empty((cap, 48), dtype=torch.uint8, device="cuda")
    res = {"max_batch_packets": max_batch}
    for speed in args.latency_speeds:
        lim = max(1, min(len(starts), int(2.0 * pk_rate * speed / chunk)))
        sv = tpx.Service(max_batch, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
        sv.set_segment(q)
        ptrs = [ctypes.c_void_p(pk[a:a + chunk].data_ptr()) for a in starts[:lim]]
        sizes = [min(chunk, n_pk - a) for a in starts[:lim]]
        hstream = tpx._stream(torch)
        submit = sv.lib.tpx_service_submit
        t0 = time.perf_counter()
        rel = [t0 + min(a + chunk, n_pk) / pk_rate / speed for a in starts[:lim]]
        nxt = done = runs = 0
        pending, lat = [], []
        while done < lim:
            if nxt < lim and not pending:
                while time.perf_counter() < rel[nxt]:
                    pass
            while nxt < lim and time.perf_counter() >= rel[nxt]:
                rc = submit(sv.h, ptrs[nxt], sizes[nxt], 1, None, hstream)
                if rc == tpx.ECAPACITY:
                    break
                if rc != 0:
                    raise tpx.TpxError(rc, "tpx_service_submit", sv.lib.tpx_last_error().decode())
                pending.append(rel[nxt])
                nxt += 1
            rc, nh, nd, st = sv.run_raw(nxt == lim, hits, cap)
            t = time.perf_counter()
            if rc != 0:
                raise tpx.TpxError(rc, "tpx_service_run", sv.lib.tpx_last_error().decode())
            k = nd - done
            lat += [(t - r) * 1e3 for r in pending[:k]]
            pending = pending[k:]
            done = nd
            runs += 1
        sv.close()
        res[f"{speed:g}x"] = dict(chunks=lim, runs=runs, p50_ms=float(np.percentile(lat, 50)),
                                  p99_ms=float(np.percentile(lat, 99)))
    del hits
    return res


def threaded_replays(args, tpx, w, pk, chunk, pk_rate, q):
    """Paced replays through tpx_service driven by the library's native
    producer (tpx_service_replay): a producer thread inside the library admits
    chunk k at its release (its copy goes on the service's own stream and
    overlaps the batch in flight); the calling thread runs the service in a
    loop, each run taking every chunk admitted so far (up to the batch limit).
    Latency of a chunk = completion of the run that took it - its release.
    No Python runs between a release and its processing."""
    n_pk = pk.numel()
    max_batch = max(1 << 19, 4 * chunk)
    res = {"max_batch_packets": max_batch, "producer": "native thread in the library"}
    for speed in args.latency_speeds:
        n_chunks = -(-n_pk // chunk)
        lim = max(1, min(n_chunks, int(2.0 * pk_rate * speed / chunk)))
        sv = tpx.Service(max_batch, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
        sv.set_segment(q)
        lat, runs = sv.replay(pk[:min(n_pk, lim * chunk)], chunk, pk_rate * speed,
                              hit_cap=2 * max_batch)
        sv.close()
        res[f"{speed:g}x"] = dict(chunks=int(lat.size), runs=runs,
                                 p50_ms=float(np.percentile(lat, 50)),
                                 p99_ms=float(np.percentile(lat, 99)))
    return res


def _cluster_block(job):
    import synth
    seed, b, n = job
    return synth.make_clusters(seed, n, block=n, first_block=b)


def run_learned(args, pool, plain_hits_per_s):
    """The learned centroider / multiplicity splitter: trained from scratch
    on generated clusters (30 % overlapping pairs, sigma 0.5-2.5, the same
    time-walk model), streamed from the worker pool in blocks; scored on
    held-out clusters against the weighted centroid; inference (patches,
    forward, refine) timed with HIP events on the calls' stream."""
    import torch

    import paper_2603_04942_amd as tpx
    import paper_2603_04942_amd.learned as LR
    import synth

    blk = args.learned_block
    n_tr = args.learned_train
    jobs = [(4003, b, min(blk, n_tr - b * blk)) for b in range((n_tr + blk - 1) // blk)]
    ejobs = [(4002, b, min(blk, args.learned_eval - b * blk))
             for b in range((args.learned_eval + blk - 1) // blk)]
    mlp = tpx.Mlp(synth.init_mlp_params(4001, zero_last=True), batch=args.learned_batch)
    lr0, lr1 = 2e-3, 1e-4
    t0 = time.perf_counter()
    train_s, seen, loss = 0.0, 0, None
    for k, cl in enumerate(pool.imap(_cluster_block, jobs)):
        d = LR.prepare(cl)
        torch.cuda.synchronize()
        t = time.perf_counter()
        f0, f1 = k / len(jobs), (k + 1) / len(jobs)
        loss = LR.fit(mlp, d, 1, lr=lr0 * (lr1 / lr0) ** f0, lr_final=lr0 * (lr1 / lr0) ** f1)
        torch.cuda.synchronize()
        train_s += time.perf_counter() - t
        seen += cl["n"]
        if k % 20 == 0:
            log(f"learned: block {k}/{len(jobs)}, loss {loss}")
    wall = time.perf_counter() - t0
    test = [cl for cl in pool.imap(_cluster_block, ejobs)]
    ev_parts = [LR.prepare(cl) for cl in test]
    feat = torch.cat([p[0] for p in ev_parts])
    hits = torch.cat([p[1] for p in ev_parts])
    truth = np.concatenate([cl["truth"] for cl in test])
    mult = np.concatenate([cl["mult"] for cl in test])
    n_ev = feat.shape[0]
    refined = LR.predict(mlp, feat, hits)
    hn = tpx.hits_to_numpy(hits, n_ev)
    s = LR.score(hn, refined.cpu().numpy(), truth, mult)
    # the network's own position for single hits, before the centroid is kept
    raw = mlp.forward(feat).cpu().numpy().astype(np.float64)
    one = mult == 1
    d = (hn["x"] + raw[:, 0] - truth[:, 0, 0]) ** 2 + (hn["y"] + raw[:, 1] - truth[:, 0, 1]) ** 2
    s["single_pos_rmse_px"]["network_raw"] = float(np.sqrt(np.mean(d[one])))
    # inference timing: patches + forward + refine over the held-out clusters
    cl0 = test[0]
    ev0 = tpx.to_device_events(cl0["events"])
    lab0 = torch.from_numpy(np.asarray(cl0["labels"], np.uint32).view(np.int32)).cuda()
    h0 = ev_parts[0][1]
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    for _ in range(2):
        tpx.patches(ev0, lab0, h0)
        LR.predict(mlp, feat, hits)
    torch.cuda.synchronize()
    reps = 5
    e0.record()
    for _ in range(reps):
        tpx.patches(ev0, lab0, h0)
    e1.record()
    for _ in range(reps):
        LR.predict(mlp, feat, hits)
    e2.record()
    torch.cuda.synchronize()
    patch_ms = e0.elapsed_time(e1) / reps * (n_ev / cl0["n"])
    fwd_ms = e1.elapsed_time(e2) / reps
    flop = 2 * (98 * 256 + 256 * 256 + 256 * 8) * n_ev
    return dict(
        workload="clusters with truth: 30% overlapping pairs (separation 0.5-3 px, dt 0-50 ns), "
                 "sigma U(0.5, 2.5) px, ToT = rint(400 amp), walk 20 ns (1 - amp), jitter 1.5 ns; "
                 "7x7 ToT/ToA patch, MLP 98-256-256-8, bf16 on MFMA with fp32 accumulation",
        train_clusters=seen, eval_clusters=int(n_ev), batch=args.learned_batch,
        final_loss=loss, train_s=train_s, train_wall_s=wall,
        train_clusters_per_s=seen / max(train_s, 1e-9),
        inference_clusters_per_s=n_ev / ((patch_ms + fwd_ms) * 1e-3),
        patch_ms_per_eval_set=patch_ms, forward_refine_ms=fwd_ms,
        forward_tflops=flop / (fwd_ms * 1e-3) / 1e12, mfma_peak_tflops_bf16=2500.0,
        plain_path_hits_per_s=plain_hits_per_s, score=s)


def run_uneven(args, w):
    """The uneven-shot workload (c3: mixture of Poisson(5), Poisson(40) and
    Poisson(200) hits per shot, electron- and ion-like spots): the segment
    stride is chosen by tpx_stream_autotune on the whole stream, then the
    stream step is timed at that stride like the c2 step."""
    import torch

    import paper_2603_04942_amd as tpx

    pk = torch.from_numpy(w.packets.view(np.int64)).cuda()
    n = pk.numel()
    s = tpx.Stream(n, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    cap = n // 4 + 1024
    hits = torch.empty((cap, 48), dtype=torch.uint8, device="cuda")
    best, best_k, sweep = s.autotune(pk, True, args.strides, hits, cap, reps=2,
                                     kernels=list(range(-1, tpx.kernel_count())))
    sweep = {f"{tpx.kernel_name(k)} @ {q}": round(v, 4) for (k, q), v in sweep.items()}
    fresh = s.get_state()
    s.set_timing(True)
    stages = {}
    reps = max(1, args.steps // 2)
    for _ in range(2):
        s.set_state(fresh)
        rc, nh, st = s.process_raw(pk, True, hits, cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.set_state(fresh)
        rc, nh, st = s.process_raw(pk, True, hits, cap)
        if rc != 0:
            raise tpx.TpxError(rc, "tpx_process_stream", s.lib.tpx_last_error().decode())
        for k, v in s.stage_times_ms().items():
            stages[k] = stages.get(k, 0.0) + v / reps
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    s.close()
    return dict(workload="c3: 200,000 shots, hits/shot 0.7 Poisson(5) + 0.25 Poisson(40) + "
                         "0.05 Poisson(200); 60% sigma 0.5 px, 40% sigma U(1.5, 2.5) px with ToT "
                         "scale up to 1023",
                packets=int(n), events=int(st.n_events), hits=int(nh),
                sweep_ms=sweep, stride=best, kernel=best_k, kernel_name=tpx.kernel_name(best_k),
                ms_per_step=ms, stages_ms=stages,
                events_per_s=st.n_events / (ms * 1e-3))


def run_out_of_order(args, wl):
    """The c2 step with three kept pixels each reported after a pixel of a
    later shot: the chunk is no longer in shot order, so the stream takes the
    general path (every event's shot materialised, a stable 4-bit radix sort
    by shot, clustering through the permutation).  Timed like the c2 step,
    host clock over whole calls."""
    import torch

    import paper_2603_04942_amd as tpx

    pk_h = wl.packets.copy()
    rng = np.random.default_rng(5)
    n = pk_h.size
    pix = np.nonzero((pk_h[n // 10: 9 * n // 10] >> np.uint64(60)) == np.uint64(0xB))[0] + n // 10
    moves = sorted(((int(a), int(a) + int(d)) for a, d in
                    zip(rng.choice(pix, 3, replace=False), rng.integers(2000, 5000, 3))),
                   reverse=True)
    for i, j in moves:          # word i moved behind word j (later moves first)
        pk_h = np.concatenate([pk_h[:i], pk_h[i + 1:j + 1], pk_h[i:i + 1], pk_h[j + 1:]])
    pk = torch.from_numpy(pk_h.view(np.int64)).cuda()
    del pk_h
    s = tpx.Stream(n, pix_epoch0=wl.pix_epoch0, tdc_epoch0=wl.tdc_epoch0)
    cap = n // 4 + 1024
    hits = torch.empty((cap, 48), dtype=torch.uint8, device="cuda")
    fresh = s.get_state()
    reps = max(1, args.steps // 4)
    for _ in range(2):
        s.set_state(fresh)
        rc, nh, st = s.process_raw(pk, True, hits, cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.set_state(fresh)
        rc, nh, st = s.process_raw(pk, True, hits, cap)
        if rc != 0:
            raise tpx.TpxError(rc, "tpx_process_stream", s.lib.tpx_last_error().decode())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    general = s.fallback_count
    s.close()
    return dict(workload="c2 with three kept pixels moved behind later shots' pixels (general "
                         "path: shot of every event, stable 4-bit radix sort by shot, "
                         "clustering through the permutation)",
                packets=int(n), events=int(st.n_events), hits=int(nh),
                general_path_calls=int(general), ms_per_step=ms,
                events_per_s=st.n_events / (ms * 1e-3))


def run_paper_mode(args, wl, name="c2"):
    """The paper's local-maximum hits (tpx_local_maxima) on the decoded
    events of a workload: events resident in HBM, HIP-event timing on the
    call's stream."""
    import torch

    import paper_2603_04942_amd as tpx

    pk = torch.from_numpy(wl.packets.view(np.int64)).cuda()
    ev, trig, _, _ = tpx.decode(pk, params=tpx.make_params(pix_epoch0=wl.pix_epoch0,
                                                           tdc_epoch0=wl.tdc_epoch0))
    del pk
    n = ev["x"].numel()
    cap = n // 2 + 1024
    hits = torch.empty((cap, 48), dtype=torch.uint8, device="cuda")
    ws = tpx.workspace(0, n)
    for _ in range(2):
        rc, nh = tpx.local_maxima_raw(ev, trig, hits, cap, ws)
        if rc != 0:
            raise tpx.TpxError(rc, "tpx_local_maxima", tpx.load().tpx_last_error().decode())
    reps = max(1, args.steps // 2)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        rc, nh = tpx.local_maxima_raw(ev, trig, hits, cap, ws)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    alg = 18 * n + HIT_BYTES * nh
    return dict(workload=f"{name} decoded events (SoA in HBM): local maxima of ToT over the "
                         "8-neighbourhood within 200 ns, Eq. 9 over each maximum's row",
                events=int(n), hits=int(nh), ms_per_call=ms, value=n / (ms * 1e-3), unit="events/s",
                algorithmic_bytes=int(alg), achieved_gbs=alg / (ms * 1e-3) / 1e9,
                frac=alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)


def run_cpu_baseline(wl, frac):
    import oracle

    n = int(wl.n_packets * frac)
    sample = np.ascontiguousarray(wl.packets[:n])
    o = oracle.get()
    t = time.perf_counter()
    hits, st = o.run(sample, pix_epoch0=wl.pix_epoch0, tdc_epoch0=wl.tdc_epoch0)
    dt = time.perf_counter() - t
    return dict(value=st["n_events"] / dt, unit="events/s", cores=1, kind="oracle",
                sample=f"first {n} packets ({frac:.0%}) of the c2 stream, {st['n_events']} "
                       f"events, single-threaded C oracle, {dt:.1f} s")


def _oracle_job(job):
    import oracle
    pk, kw = job
    t = time.perf_counter()
    _, st = oracle.get().run(pk, **kw)
    return st["n_events"], time.perf_counter() - t


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_info():
    """CPU model and counts from /proc/cpuinfo and the scheduler."""
    info = {"model": "unknown", "nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and info["model"] == "unknown":
                    info["model"] = v
                elif k in ("cpu family", "model", "stepping", "cpu MHz"):
                    info.setdefault(k if k != "model" else "model_number", v)
    except OSError:
        pass
    return info


# pixel times near a split lie within about 1 ms of its trigger: a split
# trigger at least this far from a pixel-counter wrap gives every pixel of
# the range the trigger's pixel epoch
_WRAP_MARGIN_TICKS = 2 * 640_000


def shot_ranges(wl, procs):
    """`procs` contiguous ranges of whole shots of the stream: packet
    [start, stop) and the counter epochs in force at the start (from the
    trigger that opens the range)."""
    S = wl.trig_ticks.size
    cuts = [0]
    for i in range(1, procs):
        k = max(cuts[-1] + 1, S * i // procs)
        while k < S and (int(wl.trig_ticks[k]) % (1 << 34) < _WRAP_MARGIN_TICKS or
                         (1 << 34) - int(wl.trig_ticks[k]) % (1 << 34) < _WRAP_MARGIN_TICKS):
            k += 1
        if k < S:
            cuts.append(k)
    out = []
    for i, k in enumerate(cuts):
        start = 0 if i == 0 else int(wl.trig_pos[k])
        stop = int(wl.trig_pos[cuts[i + 1]]) if i + 1 < len(cuts) else wl.n_packets
        kw = (dict(pix_epoch0=wl.pix_epoch0, tdc_epoch0=wl.tdc_epoch0) if i == 0 else
              dict(pix_epoch0=int(wl.trig_ticks[k]) >> 34, tdc_epoch0=int(wl.trig_ticks[k]) >> 36))
        out.append((start, stop, kw))
    return out


def run_cpu_multicore(pool, wl, procs):
    """The oracle in `procs` concurrent processes (the worker pool forked
    before the GPU was touched), each on its own contiguous range of whole
    shots of the c2 stream, together covering all of it: events of all
    processes over the slowest one's time."""
    jobs = [(np.ascontiguousarray(wl.packets[a:b]), kw) for a, b, kw in shot_ranges(wl, procs)]
    res = pool.map(_oracle_job, jobs, chunksize=1)
    ev = sum(r[0] for r in res)
    t_max = max(r[1] for r in res)
    info = _cpu_info()
    return dict(value=ev / t_max, unit="events/s", processes=len(jobs), cpu_model=info["model"],
                cpu=info, events=int(ev),
                sample=f"the whole c2 stream in {len(jobs)} contiguous ranges of whole shots, one "
                       f"per process, slowest {t_max:.1f} s")


def run_c1(args):
    """The small workload (c1: 1,000 shots, Poisson(10) hits): one flushed
    tpx_process_stream call over the whole stream, HIP-event timed on the
    call's stream; microseconds per call and events/s (the whole input fits
    the 256 MB last-level cache, so no HBM fraction is claimed)."""
    import torch

    import paper_2603_04942_amd as tpx
    import synth

    w = synth.make_config("c1", with_truth=False)
    pk = torch.from_numpy(w.packets.view(np.int64)).cuda()
    n = pk.numel()
    s = tpx.Stream(n, pix_epoch0=w.pix_epoch0, tdc_epoch0=w.tdc_epoch0)
    cap = n // 2 + 1024
    hits = torch.empty((cap, 48), dtype=torch.uint8, device="cuda")
    fresh = s.get_state()
    for _ in range(5):
        s.set_state(fresh)
        rc, nh, st = s.process_raw(pk, True, hits, cap)
    reps = 50
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = 0.0
    for _ in range(reps):
        s.set_state(fresh)
        t0.record()
        rc, nh, st = s.process_raw(pk, True, hits, cap)
        t1.record()
        t1.synchronize()
        if rc != 0:
            raise tpx.TpxError(rc, "tpx_process_stream", s.lib.tpx_last_error().decode())
        ms += t0.elapsed_time(t1)
    s.close()
    us = ms * 1e3 / reps
    return dict(workload="c1: 1,000 shots at 1 kHz, Poisson(10) hits/shot, sigma 0.8 px, 1% dark "
                         "counts", packets=int(n), events=int(st.n_events), hits=int(nh),
                us_per_call=us, events_per_s=st.n_events / (us * 1e-6))


def run_copy(args):
    """A plain 1 GiB device-to-device copy, HIP-event timed: the HBM rate
    this GPU reaches on a streaming kernel (read + write bytes over time)."""
    import torch

    nb = 1 << 30
    src = torch.ones(nb // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del src, dst
    return dict(bytes_moved=2 * nb, ms=ms, gbs=2 * nb / (ms * 1e-3) / 1e9,
                frac_of_peak=2 * nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shots", type=int, default=100_000, help="c2 shots (default: full size)")
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="workload of the timed step (c3 only to profile the uneven-shot "
                         "workload; the headline figure is c2)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cpu-frac", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-paper-mode", action="store_true")
    ap.add_argument("--latency-shots", type=int, default=36000)
    ap.add_argument("--latency-chunks", type=int, nargs="+", default=[8192, 131072, 2097152],
                    help="packets per chunk (64 KiB, 1 MiB, 16 MiB)")
    ap.add_argument("--latency-speeds", type=float, nargs="+", default=[1.0, 10.0, 200.0],
                    help="paced replay speedups over acquisition")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-out-of-order", action="store_true")
    ap.add_argument("--strides", type=int, nargs="+",
                    default=[128, 256, 512, 1024, 2048, 4096],
                    help="segment strides the autotuner tries on the uneven-shot workload")
    ap.add_argument("--kernel", type=int, default=None,
                    help="pin the clustering kernel of the main step (no autotune)")
    ap.add_argument("--stride", type=int, default=None,
                    help="pin the segment stride of the main step (no autotune)")
    ap.add_argument("--c2-strides", type=int, nargs="+", default=[512, 1024, 2048],
                    help="segment strides the autotuner tries on the c2 workload")
    ap.add_argument("--learned-train", type=int, default=10_000_000,
                    help="training clusters (learned centroider)")
    ap.add_argument("--learned-eval", type=int, default=1_000_000, help="held-out clusters")
    ap.add_argument("--learned-block", type=int, default=50_000)
    ap.add_argument("--learned-batch", type=int, default=4096)
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing "
                         "(calibration of HBM traffic counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(each GPU would process its own range of shots; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import synth

    # cluster generators for the learned leg, forked before the GPU is touched
    pool = None
    if not args.no_learned:
        import multiprocessing
        pool = multiprocessing.get_context("fork").Pool(args.workers)
    t = time.perf_counter()
    if args.workload == "c3":
        # profiling the uneven-shot workload: its stream step is the timed step
        args.no_uneven = True
        args.shots = 200_000 if args.shots == 100_000 else args.shots
    wl = synth.make_config(args.workload, n_shots=args.shots, with_truth=False,
                           workers=args.workers)
    log(f"generated c2: {wl.n_packets} packets in {time.perf_counter() - t:.1f} s")
    wl3 = None
    if not args.no_uneven:
        t = time.perf_counter()
        wl3 = synth.make_config("c3", with_truth=False, workers=args.workers)
        log(f"generated c3: {wl3.n_packets} packets in {time.perf_counter() - t:.1f} s")
    ms, stages, stats, tune = run_gpu(args, wl)
    log(f"gpu: {ms:.3f} ms/step, stages {json.dumps({k: round(v, 4) for k, v in stages.items()})}")
    n_ev, n_hits, n_pk = stats["n_events"], stats["n_hits"], wl.n_packets
    value = n_ev / (ms * 1e-3)
    fused = tune["kernel"] >= 0
    sb = stage_bytes(n_pk, n_ev, n_hits, fused)
    dom = max(stages, key=stages.get)
    # (the fused kernel by its variant: the traffic summary holds one variant)
    kname = (f"{FUSED_KERNEL}[{tune['kernel']}]" if (fused and dom == "cluster")
             else STAGE_KERNEL.get(dom, dom))
    # algorithmic bytes of the method per launch (8 B per packet in, 48 B per
    # hit out: every launch of the dominant kernel serves one whole step)
    path_bytes = 8 * n_pk + HIT_BYTES * n_hits
    achieved = path_bytes / (stages[dom] * 1e-3) / 1e9
    traffic = measured_traffic(kname)
    out = {
        "metric": "pixel events/s decoded+clustered+centroided at 1 GPU; % HBM peak; p99 chunk ms",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": ("c2: 100,000 shots at 1 kHz, Poisson(30) hits/shot, sigma U(0.6,1.5) px, "
                         "10% close pairs, 1% dark counts, TPX3 packets with spidr/ToA rollover "
                         "and trigger words; 8-connected, |dToA| <= 200 ns")
            if args.workload == "c2" else
            ("c3: 200,000 shots, hits/shot 0.7 Poisson(5) + 0.25 Poisson(40) + 0.05 "
             "Poisson(200); 60% sigma 0.5 px, 40% sigma U(1.5, 2.5) px with ToT scale up to "
             "1023; 8-connected, |dToA| <= 200 ns"),
            "shots": args.shots,
            "packets": int(n_pk),
            "events": int(n_ev),
            "hits": int(n_hits),
            "pixels_per_hit": n_ev / max(n_hits, 1),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes": int(path_bytes),
            "launch_ms": stages[dom],
            # the kernel's own inputs and outputs (at least) over its time
            "kernel_io_bytes": int(sb[dom]),
            "kernel_io_gbs": sb[dom] / (stages[dom] * 1e-3) / 1e9,
            # measured HBM bytes per launch over the same launch time
            "traffic_gbs": None if traffic is None else traffic / (stages[dom] * 1e-3) / 1e9,
            "traffic_frac": None if traffic is None else
            traffic / (stages[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "path_roofline": {
            "algorithmic_bytes_per_step": int(path_bytes),
            "achieved": path_bytes / (ms * 1e-3) / 1e9,
            "frac": path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "unit": "GB/s",
        },
        "stages_ms": stages,
        "c2_tuning": tune,
        "hits_per_s": n_hits / (ms * 1e-3),
        "acquisition_multiple": value / (n_ev / (args.shots * 1e-3)),
        # context, not a target: the paper's own figure on its hardware and data
        # (about 10 particles per shot at 1 kHz, batched on a desktop GPU)
        "paper_acquisition_multiple": 25,
    }
    out["copy_bandwidth"] = run_copy(args)
    log(f"copy: {out['copy_bandwidth']}")
    out["c1"] = run_c1(args)
    log(f"c1: {out['c1']}")
    if not args.no_latency:
        out["stream_latency"] = run_latency(args)
        log(f"latency: {out['stream_latency']}")
    if not args.no_uneven:
        out["uneven"] = run_uneven(args, wl3)
        log(f"uneven: {out['uneven']}")
    if not args.no_out_of_order:
        out["out_of_order"] = run_out_of_order(args, wl)
        log(f"out of order: {out['out_of_order']}")
    if not args.no_paper_mode:
        out["paper_mode"] = run_paper_mode(args, wl)
        log(f"paper mode: {out['paper_mode']}")
        if wl3 is not None:
            out["paper_mode_uneven"] = run_paper_mode(args, wl3, "c3")
            log(f"paper mode c3: {out['paper_mode_uneven']}")
    del wl3
    if pool is not None:
        out["learned"] = run_learned(args, pool, out["hits_per_s"])
        log(f"learned: {out['learned']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = run_cpu_baseline(wl, args.cpu_frac)
        out["cpu_baseline"]["acquisition_multiple"] = (out["cpu_baseline"]["value"]
                                                       / (n_ev / (args.shots * 1e-3)))
        log(f"cpu baseline: {out['cpu_baseline']}")
        if pool is not None:
            mc = run_cpu_multicore(pool, wl, min(os.cpu_count() or 1, args.workers))
            mc["acquisition_multiple"] = mc["value"] / (n_ev / (args.shots * 1e-3))
            out["cpu_baseline"]["multicore"] = mc
            log(f"cpu multicore: {mc}")
    if pool is not None:
        pool.terminate()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
