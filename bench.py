"""Throughput benchmark of the GPU SIFT path on one MI355X.

Default workload: a batch of 64 synthetic 1024x768 float32 images (1000 blobs
each, seeded), SIFT with the upsampled octave -1 (5 octaves), extracted by one
batched launch sequence per step.  A step is one pass of the whole path --
pyramid, detection, refinement, orientation, descriptors -- over the batch,
with inputs already resident in HBM.  The plain per-image path (one
sift_extract per image) is timed beside it on the same images, and its
outputs are compared bit for bit with the batched ones.

Prints one JSON line.  ``--gpus`` above 1 is refused: this benchmark runs on
one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2605_17869_amd import synth  # noqa: E402
from paper_2605_17869_amd.build import kernel_source_hash  # noqa: E402

HBM_PEAK_GBS = 8000.0
# HBM traffic of the blur kernel measured with rocprofv3 counters (summary text)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_blur_hbm_traffic_w2.txt")
def measured_traffic():
    """HBM bytes per blur launch from the committed counter summary, or None
    when it is missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            fields = dict(l.split(":", 1) for l in f.read().splitlines() if ":" in l)
    except OSError:
        return None
    if fields.get("kernel_source_sha256", "").strip() != kernel_source_hash():
        return None
    try:
        return int(fields["hbm_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def copy_calibration(mib: int, reps: int):
    """A plain elementwise pass of known size (read mib MiB, write mib MiB),
    the yardstick for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "neg", "bytes_read_per_dispatch": 4 * n,
                      "bytes_written_per_dispatch": 4 * n, "dispatches": reps}), flush=True)


def _gen(args):
    wl_no, k, n = args
    return synth.workload(wl_no, n).image(k)


def _warp(args):
    wl_no, k, img = args
    return synth.warped_copy(img, synth.workload_seed(wl_no, k, True))[0]


def make_images(wl_no: int, n: int):
    """The workload's images (with its affine-warped copies after the
    originals where the workload pairs them)."""
    wl = synth.workload(wl_no, n)
    jobs = [(wl_no, k, n) for k in range(len(wl.sizes))]
    workers = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    with ProcessPoolExecutor(max_workers=workers) as pool:
        imgs = list(pool.map(_gen, jobs))
        if wl.warped_pairs:
            imgs += list(pool.map(_warp, [(wl_no, k, im) for k, im in enumerate(imgs)]))
    return wl, imgs


def digest(kp, desc) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(kp).tobytes())
    h.update(np.ascontiguousarray(desc).tobytes())
    return h.hexdigest()


def serve_bench(args):
    """Serving: requests arrive as a Poisson process at fractions of the
    batched saturation rate; the continuous-batching server and the plain
    one-at-a-time path (max_batch 1, one in flight) serve the same arrivals.
    Latency is submit to observed completion, measured by the server."""
    import torch
    import paper_2605_17869_amd as sm
    wl = synth.workload(4, args.unique_images)
    t0 = time.time()
    _, imgs = make_images(4, args.unique_images)
    print(f"[serve] generated {len(imgs)} images in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_imgs = [torch.from_numpy(im).to(dev) for im in imgs]
    n_req = args.requests + args.warmup_requests
    order = [k % len(d_imgs) for k in range(n_req)]
    settings = dict(wl.settings)
    cap = settings["max_keypoints"]
    ex = sm.Extractor(settings)
    feats = [ex.alloc_features(cap) for _ in range(n_req)]
    torch.cuda.synchronize()
    arena = 24 << 30

    def run(arrivals, max_batch, max_inflight):
        srv = sm.Server(settings, arena_bytes=arena, max_batch=max_batch,
                        max_inflight=max_inflight)
        tickets = []
        start = time.perf_counter()
        for i in range(n_req):
            if arrivals is not None:
                while time.perf_counter() - start < arrivals[i]:
                    pass
            tickets.append(srv.submit(d_imgs[order[i]], out=feats[i]))
        lat = [srv.wait(t)[0] for t in tickets]
        wall = time.perf_counter() - start
        stats = srv.stats()
        srv.close()
        meas = np.array(lat[args.warmup_requests:])
        return dict(p50_ms=round(float(np.percentile(meas, 50)), 3),
                    p99_ms=round(float(np.percentile(meas, 99)), 3),
                    images_per_s=round(n_req / wall, 2),
                    batches=stats["batches"], mean_batch=round(n_req / stats["batches"], 2))

    run(None, 64, 2)   # warm-up
    sat = run(None, 64, 2)
    sat_rate = sat["images_per_s"]
    print(f"[serve] saturation {sat_rate} images/s {sat}", file=sys.stderr, flush=True)
    one = run(None, 1, 1)
    print(f"[serve] one-at-a-time saturation {one}", file=sys.stderr, flush=True)
    points = []
    for k, f in enumerate(float(x) for x in args.qps_fractions.split(",")):
        qps = f * sat_rate
        arr = synth.poisson_arrivals(synth.workload_seed(4, 500_000 + k), n_req, qps)
        batched = run(arr, 64, 2)
        plain = run(arr, 1, 1)
        points.append(dict(qps=round(qps, 1), fraction=f, batched=batched, one_at_a_time=plain))
        print(f"[serve] qps {qps:.1f}: batched {batched} one-at-a-time {plain}", file=sys.stderr,
              flush=True)
    mpix = float(np.mean([h * w for h, w in wl.sizes])) / 1e6
    line = {
        "metric": "served images/s and p50/p99 latency (continuous batching, Poisson arrivals)",
        "value": sat_rate, "unit": "images/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "requests": args.requests,
                   "warmup_requests": args.warmup_requests,
                   "unique_images": len(imgs), "mean_mpix": round(mpix, 3),
                   "max_batch": 64, "max_inflight": 2, "arena_gib": arena >> 30},
        "saturation": sat, "one_at_a_time_saturation": one, "points": points,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--images", type=int, default=None, help="images per batch (default: workload)")
    ap.add_argument("--per-image-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="blur chunk height (0: autotuned on the batch unless --no-autotune)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--n-streams", type=int, default=0,
                    help="sub-batches of a batched call (0: library choice, 1: one launch sequence)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise pass over MIB MiB (counter yardstick)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: Poisson arrivals, W, H ~ U[320, 2048]")
    ap.add_argument("--requests", type=int, default=700, help="serving: requests per QPS point")
    ap.add_argument("--warmup-requests", type=int, default=100)
    ap.add_argument("--unique-images", type=int, default=160,
                    help="serving: distinct images, cycled over the requests")
    ap.add_argument("--qps-fractions", default="0.25,0.5,0.75,0.9")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(images shard across GPUs with no exchange; run one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(1, args.steps))
        return
    if args.serve:
        serve_bench(args)
        return

    import torch
    import paper_2605_17869_amd as sm

    t0 = time.time()
    wl, imgs = make_images(args.workload, args.images)
    print(f"[bench] generated {len(imgs)} images in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    n = len(imgs)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_imgs = [torch.from_numpy(im).to(dev) for im in imgs]
    sizes = [tuple(im.shape) for im in imgs]
    stream = torch.cuda.current_stream()
    tune = None
    tile_rows = args.tile_rows
    if tile_rows == 0 and not args.no_autotune:
        probe = sm.Extractor(wl.settings)
        ws0 = torch.empty(probe.batch_workspace_size(sizes), dtype=torch.uint8, device=dev)
        tile_rows, tune_ms = probe.autotune(d_imgs, warmup=1, reps=3, workspace=ws0,
                                            stream=stream)
        tune = {str(k): round(v, 4) for k, v in tune_ms.items()}
        del probe, ws0
        print(f"[bench] autotune: tile_rows {tile_rows} ({tune})", file=sys.stderr, flush=True)
    settings = dict(wl.settings, tile_rows=tile_rows, n_streams=args.n_streams)
    ex = sm.Extractor(settings)
    ws = torch.empty(ex.batch_workspace_size(sizes), dtype=torch.uint8, device=dev)
    outs = [ex.alloc_features() for _ in range(n)]

    def batch_step():
        ex.extract_batch(d_imgs, outs=outs, workspace=ws, stream=stream)

    def timed(step, warmup, steps):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, (time.perf_counter() - wall0) / steps

    ms_eager, wall = timed(batch_step, args.warmup, args.steps)
    print(f"[bench] batched: {ms_eager:.3f} ms/step (wall {1e3 * wall:.3f})",
          file=sys.stderr, flush=True)
    batch_host = [f.host() for f in outs]
    ms, mode = ms_eager, "launch sequence"

    # the same batch recorded once as a graph and replayed per step
    ms_graph, graph_identical = None, None
    if not args.no_graph:
        outs_g = [ex.alloc_features() for _ in range(n)]
        ws_g = torch.empty_like(ws)
        g = ex.graph(d_imgs, outs=outs_g, workspace=ws_g)
        ms_graph, wall_g = timed(lambda: g.launch(stream), args.warmup, args.steps)
        graph_identical = all(digest(a[0], a[1]) == digest(b[0], b[1]) and a[2:] == b[2:]
                              for a, b in zip(batch_host, [f.host() for f in outs_g]))
        g.close()
        del ws_g, outs_g
        print(f"[bench] graph replay: {ms_graph:.3f} ms/step, identical={graph_identical}",
              file=sys.stderr, flush=True)
        if graph_identical and ms_graph < ms:
            ms, mode = ms_graph, "graph replay"

    # plain per-image path on the same images
    ms1, identical = None, None
    if args.per_image_steps > 0:
        ws1 = torch.empty(max(ex.workspace_size(*s) for s in sizes), dtype=torch.uint8, device=dev)
        outs1 = [ex.alloc_features() for _ in range(n)]

        def per_image_step():
            for k in range(n):
                ex.extract(d_imgs[k], out=outs1[k], workspace=ws1, stream=stream)

        per_image_step()
        ms1, _ = timed(per_image_step, 0, args.per_image_steps)
        single_host = [f.host() for f in outs1]
        identical = all(digest(a[0], a[1]) == digest(b[0], b[1]) and a[2:] == b[2:]
                        for a, b in zip(batch_host, single_host))
        print(f"[bench] per-image: {ms1:.3f} ms/step, identical={identical}", file=sys.stderr,
              flush=True)

    # stage breakdown with HIP events on the extraction stream
    stages = {}
    roofline = None
    if not args.no_profile:
        sm.profile_start()
        for _ in range(2):
            batch_step()
        torch.cuda.synchronize()
        stats = sm.profile_stop()
        for name, (launches, sms, sbytes) in stats.items():
            stages[name] = dict(launches=launches // 2, ms=round(sms / 2, 4),
                                gbs=round(sbytes / (sms * 1e6), 1) if sbytes and sms else None)
        blur = stats.get("blur")
        if blur:
            launches, bms, bbytes = blur
            achieved = (bbytes / launches) / (bms / launches * 1e-3) / 1e9
            roofline = {"kernel": "k_blur (separable Gaussian level, all radii)", "bound": "hbm",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                        "avg_launch_us": round(1e3 * bms / launches, 2),
                        "bytes_per_launch": round(bbytes / launches),
                        "kernel_source_sha256": kernel_source_hash()}
        print(f"[bench] stages: {json.dumps(stages)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle as it stands, single-threaded, on the first images of the
        # batch until about 10 s of work (at least one image)
        import oracle
        from oracle import sift_oracle as so
        p = so.Params.from_settings(wl.settings)
        done, dt = 0, 0.0
        while done < n and (done == 0 or dt < 10.0):
            t = time.perf_counter()
            oracle.sift(imgs[done], p)
            dt += time.perf_counter() - t
            done += 1
        cpu = {"value": round(done / dt, 5), "unit": "images/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {done} of the {n} images, full pipeline, {dt:.1f} s "
                         f"single-threaded FP64 NumPy"}

    mpix = sum(h * w for h, w in sizes) / 1e6
    n_kp = int(sum(len(b[0]) for b in batch_host))
    line = {
        "metric": "images/s (batched SIFT extraction, inputs resident in HBM)",
        "value": round(n / (ms * 1e-3), 2),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "images": n, "image_size": (f"{sizes[0][1]}x{sizes[0][0]}" if len(set(sizes)) == 1
                                  else f"mixed, mean {mpix / n:.3f} Mpix"),
                   "tile_rows": tile_rows, "upsample": wl.settings["upsample"], "octaves": wl.settings["n_octaves"] +
                   wl.settings["upsample"], "parallelism": "none (one GPU)"},
        "mpix_per_s": round(mpix / (ms * 1e-3), 2),
        "per_image_path": ({"images_per_s": round(n / (ms1 * 1e-3), 2),
                            "ms_per_step": round(ms1, 4)} if ms1 else None),
        "batched_vs_per_image": round(ms1 / ms, 3) if ms1 else None,
        "execution": mode,
        "ms_per_step_launch_sequence": round(ms_eager, 4),
        "ms_per_step_graph_replay": round(ms_graph, 4) if ms_graph else None,
        "bitwise_identical_graph_vs_launch_sequence": graph_identical,
        "autotune_ms_per_tile_rows": tune,
        "bitwise_identical_batched_vs_per_image": identical,
        "keypoints_per_image": round(n_kp / n, 1),
        "stages": stages,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
