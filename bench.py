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
# HBM traffic of the pyramid kernels measured with rocprofv3 counters (summary text)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pyramid_hbm_traffic_w2.txt")
def measured_traffic():
    """HBM bytes per pyramid launch from the committed counter summary, or None
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


FMA_PEAK_T = 256 * 64 * 2.4e9 / 1e12   # non-packed fp32 FMA issue: CUs x lanes x clock (T FMA/s)
FP16_MFMA_PEAK_TFLOPS = 2500.0         # dense fp16 matrix peak, TFLOP/s


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_worker_init():
    # one BLAS/OpenMP thread per worker process
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _oracle_one(args):
    wl_no, n, k = args
    import oracle
    from oracle import sift_oracle as so
    wl = synth.workload(wl_no, n)
    img = wl.image(k)
    p = so.Params.from_settings(wl.settings)
    t = time.perf_counter()
    oracle.sift(img, p)
    return time.perf_counter() - t


def pixel_octaves(sizes, upsample: int, n_oct: int) -> int:
    """Pixels summed over every octave of every image (octave sizes halve,
    rounding up; the first octave is 2H x 2W when upsampling)."""
    tot = 0
    for h, w in sizes:
        hh, ww = (2 * h, 2 * w) if upsample else (h, w)
        for _ in range(n_oct):
            tot += hh * ww
            hh, ww = (hh + 1) // 2, (ww + 1) // 2
    return tot


def digest(kp, desc) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(kp).tobytes())
    h.update(np.ascontiguousarray(desc).tobytes())
    return h.hexdigest()


def match_bench(n_pairs: int, n_a: int, n_b: int, reps: int = 20):
    """Symmetric ratio-test matching of n_pairs seeded descriptor-set pairs
    (n_a x n_b rows each) in one sift_match_batch call: pairs/s, and the
    similarity work against the dense fp16 matrix peak."""
    import torch
    import paper_2605_17869_amd as sm
    sets = [synth.descriptor_sets(900_000 + k, n_a, n_b, (3 * min(n_a, n_b)) // 4, 0.1)
            for k in range(n_pairs)]
    dev = torch.device("cuda:0")
    pairs = [(torch.from_numpy(a).to(dev), None, torch.from_numpy(b).to(dev), None)
             for a, b, _ in sets]
    stream = torch.cuda.current_stream()
    outs = sm.match_batch(pairs, stream=stream)
    ws = outs[0]._ws
    first = [m.host() for m in outs]
    for _ in range(3):
        sm.match_batch(pairs, workspace=ws, stream=stream, outs=outs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sm.match_batch(pairs, workspace=ws, stream=stream, outs=outs)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    again = [m.host() for m in outs]
    same = all(a[0].tobytes() == b[0].tobytes() for a, b in zip(first, again))
    flops = 2.0 * 128 * n_a * n_b * n_pairs
    kept = float(np.mean([len(m[0]) for m in again]))
    return {"pairs": n_pairs, "rows_per_set": [n_a, n_b], "ms_per_call": round(ms, 4),
            "pairs_per_s": round(n_pairs / (ms * 1e-3), 1),
            "similarity_tflops": round(flops / (ms * 1e-3) / 1e12, 2),
            "frac_fp16_mfma_peak": round(flops / (ms * 1e-3) / 1e12 / FP16_MFMA_PEAK_TFLOPS, 4),
            "mean_matches_per_pair": round(kept, 1), "bitwise_identical_reruns": same,
            "data": "seeded descriptor sets: 3/4 of the rows noisy copies, the rest fresh"}


def verify_bench(n_pairs: int = 32, n_corr: int = 1300, n_hyp: int = 1500, reps: int = 20):
    """Verification of n_pairs seeded correspondence sets (n_corr each, 40 %
    outliers, 0.7 px noise) with n_hyp hypotheses per pair, in one
    sift_verify_batch call."""
    import torch
    import paper_2605_17869_amd as sm
    dev = torch.device("cuda:0")
    pairs = []
    for k in range(n_pairs):
        a, b, _, _ = synth.homography_pairs(800_000 + k, n_corr, 0.4, 0.7)
        ka = np.zeros((n_corr, 12), np.int32)
        kb = np.zeros((n_corr, 12), np.int32)
        ka.view(np.float32)[:, 0:2] = a
        kb.view(np.float32)[:, 0:2] = b
        m = np.zeros((n_corr, 4), np.int32)
        m[:, 0] = m[:, 1] = np.arange(n_corr)
        pairs.append((torch.from_numpy(ka).to(dev), torch.from_numpy(kb).to(dev),
                      torch.from_numpy(m).to(dev), None))
    u = torch.from_numpy(synth.sample_numbers(810_000, n_hyp)).to(dev)
    stream = torch.cuda.current_stream()
    outs = sm.verify_batch(pairs, u, stream=stream)
    ws = outs[0]._ws
    first = [o.host() for o in outs]
    for _ in range(3):
        sm.verify_batch(pairs, u, workspace=ws, stream=stream, outs=outs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sm.verify_batch(pairs, u, workspace=ws, stream=stream, outs=outs)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    again = [o.host() for o in outs]
    same = all(x[0].tobytes() == y[0].tobytes() for x, y in zip(first, again))
    return {"pairs": n_pairs, "correspondences_per_pair": n_corr, "hypotheses_per_pair": n_hyp,
            "ms_per_call": round(ms, 4), "pairs_per_s": round(n_pairs / (ms * 1e-3), 1),
            "residuals_per_s": round(n_pairs * n_hyp * n_corr / (ms * 1e-3), 1),
            "mean_inliers": round(float(np.mean([x[2] for x in again])), 1),
            "bitwise_identical_reruns": same,
            "data": "seeded correspondences under random homographies, 40 % outliers"}


def serve_points(unique_images: int, requests: int, warmup_requests: int, fractions,
                 one_at_a_time: bool):
    """Serving: requests arrive as a Poisson process at fractions of the
    batched saturation rate; the continuous-batching server (and, if asked,
    the plain one-at-a-time path: max_batch 1, one in flight) serve the same
    arrivals.  Latency is from entry into submit to observed completion,
    measured by the server.  Returns (workload, images, saturation,
    one-at-a-time saturation, points)."""
    import torch
    import paper_2605_17869_amd as sm
    wl = synth.workload(4, unique_images)
    t0 = time.time()
    _, imgs = make_images(4, unique_images)
    print(f"[serve] generated {len(imgs)} images in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_imgs = [torch.from_numpy(im).to(dev) for im in imgs]
    n_req = requests + warmup_requests
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
        tickets, late = [], []
        start = time.perf_counter()
        for i in range(n_req):
            if arrivals is not None:
                while time.perf_counter() - start < arrivals[i]:
                    pass
                # a request submitted after its scheduled arrival (the client
                # was held up) is charged the delay as well
                late.append(max(0.0, time.perf_counter() - start - arrivals[i]) * 1e3)
            else:
                late.append(0.0)
            tickets.append(srv.submit(d_imgs[order[i]], out=feats[i]))
        lat = [srv.wait(t)[0] + d for t, d in zip(tickets, late)]
        wall = time.perf_counter() - start
        stats = srv.stats()
        srv.close()
        meas = np.array(lat[warmup_requests:])
        return dict(p50_ms=round(float(np.percentile(meas, 50)), 3),
                    p99_ms=round(float(np.percentile(meas, 99)), 3),
                    images_per_s=round(n_req / wall, 2),
                    batches=stats["batches"], mean_batch=round(n_req / stats["batches"], 2),
                    largest_batch=stats["largest_batch"],
                    overlapped_batches=stats["overlapped_batches"])

    # one batch of the random-size images: launch sequence against size
    # buckets recorded for the largest possible size and for the batch's own
    # largest image (the same bits either way)
    def bucket_cmp():
        batch = d_imgs[:64]
        bo = [ex.alloc_features(cap) for _ in batch]
        wsb = torch.empty(ex.batch_workspace_size([tuple(b.shape) for b in batch]),
                          dtype=torch.uint8, device=dev)

        def tm(fn, reps=10):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return round(a.elapsed_time(b) / reps, 4)

        res = {"images": len(batch),
               "launch_sequence_ms": tm(lambda: ex.extract_batch(batch, outs=bo, workspace=wsb))}
        ref = [digest(*f.host()[:2]) for f in bo]
        for name, (mh, mw) in (("bucket_2048x2048_ms", (2048, 2048)),
                               ("bucket_batch_max_ms", (max(b.shape[0] for b in batch),
                                                        max(b.shape[1] for b in batch)))):
            bk = ex.bucket(len(batch), mh, mw)
            res[name] = tm(lambda: bk.launch(batch, outs=bo))
            res[name.replace("_ms", "_identical")] = ref == [digest(*f.host()[:2]) for f in bo]
            bk.close()
        del wsb, bo
        return res

    buckets = bucket_cmp()
    print(f"[serve] buckets {buckets}", file=sys.stderr, flush=True)

    run(None, 64, 2)   # warm-up
    sat = run(None, 64, 2)
    sat_rate = sat["images_per_s"]
    print(f"[serve] saturation {sat_rate} images/s {sat}", file=sys.stderr, flush=True)
    one = run(None, 1, 1) if one_at_a_time else None
    if one:
        print(f"[serve] one-at-a-time saturation {one}", file=sys.stderr, flush=True)
    points = []
    for k, f in enumerate(fractions):
        qps = f * sat_rate
        arr = synth.poisson_arrivals(synth.workload_seed(4, 500_000 + k), n_req, qps)
        batched = run(arr, 64, 2)
        plain = run(arr, 1, 1) if one_at_a_time else None
        points.append(dict(qps=round(qps, 1), fraction=f, batched=batched, one_at_a_time=plain))
        print(f"[serve] qps {qps:.1f}: batched {batched} one-at-a-time {plain}", file=sys.stderr,
              flush=True)
    return wl, imgs, sat, one, points, buckets


def serve_bench(args):
    """Full serving sweep as its own JSON line (``--serve``)."""
    fr = [float(x) for x in args.qps_fractions.split(",")]
    wl, imgs, sat, one, points, buckets = serve_points(args.unique_images, args.requests,
                                                       args.warmup_requests, fr, True)
    sat_rate = sat["images_per_s"]
    arena = 24 << 30
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
        "buckets": buckets,
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
    ap.add_argument("--blur-chain", type=int, default=0,
                    help="pyramid levels per launch (0: autotuned unless --no-autotune, else 2)")
    ap.add_argument("--detect-waves", type=int, default=0,
                    help="waves per detection work-group, 4 or 8 (0: autotuned unless "
                         "--no-autotune, else 4)")
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
    ap.add_argument("--no-serve-point", action="store_true",
                    help="skip the serving point (saturation and p50/p99 at half of it)")
    ap.add_argument("--no-match", action="store_true", help="skip the matcher measurement")
    ap.add_argument("--no-fp16", action="store_true", help="skip the fp16-storage measurement")
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
    # host-to-device copy of the batch from pinned buffers, timed on its own
    # (the extraction timings below start from device-resident images)
    pinned = [torch.from_numpy(im).pin_memory() for im in imgs]
    d_imgs = [torch.empty(im.shape, dtype=torch.float32, device=dev) for im in imgs]
    h2d_passes = []
    for _ in range(3):       # the first pass also pays the copy engines' set-up
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        for d, h in zip(d_imgs, pinned):
            d.copy_(h, non_blocking=True)
        torch.cuda.synchronize()
        h2d_passes.append(time.perf_counter() - h0)
    h2d_s = min(h2d_passes[1:])
    h2d_bytes = sum(im.nbytes for im in imgs)
    del pinned
    sizes = [tuple(im.shape) for im in imgs]
    stream = torch.cuda.current_stream()
    tune = None
    tile_rows, n_streams, blur_chain = args.tile_rows, args.n_streams, args.blur_chain
    detect_waves = args.detect_waves
    if tile_rows == 0 and not args.no_autotune:
        # the launch knobs (chunk-height cap x sub-batch count, then pyramid
        # levels per launch, then waves per detection work-group), timed afresh
        # in the form the line reports (graph replay, unless --no-graph)
        probe = sm.Extractor(dict(wl.settings, blur_chain=blur_chain, detect_waves=detect_waves))
        tune = probe.tune(d_imgs, warmup=1, reps=5, as_graph=not args.no_graph, stream=stream)
        tile_rows = tune["tile_rows"]
        if n_streams == 0:
            n_streams = tune["n_streams"]
        if blur_chain == 0:
            blur_chain = tune["blur_chain"]
        if detect_waves == 0:
            detect_waves = tune["detect_waves"]
        del probe
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    settings = dict(wl.settings, tile_rows=tile_rows, n_streams=n_streams, blur_chain=blur_chain,
                    detect_waves=detect_waves)
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

    # the same batch through a size bucket recorded for its largest image
    ms_bucket, bucket_identical = None, None
    if not args.no_graph:
        maxh, maxw = max(h for h, _ in sizes), max(w for _, w in sizes)
        outs_b = [ex.alloc_features() for _ in range(n)]
        bk = ex.bucket(n, maxh, maxw)
        ms_bucket, _ = timed(lambda: bk.launch(d_imgs, outs=outs_b, stream=stream), args.warmup,
                             args.steps)
        bucket_identical = all(digest(a[0], a[1]) == digest(b[0], b[1]) and a[2:] == b[2:]
                               for a, b in zip(batch_host, [f.host() for f in outs_b]))
        bk.close()
        del outs_b
        print(f"[bench] bucket replay: {ms_bucket:.3f} ms/step, identical={bucket_identical}",
              file=sys.stderr, flush=True)

    # the same batch with fp16 storage of the octaves after the first
    fp16 = None
    if not args.no_fp16:
        ex16 = sm.Extractor(dict(settings, pyramid_fp16=1))
        ws16 = torch.empty(ex16.batch_workspace_size(sizes), dtype=torch.uint8, device=dev)
        outs16 = [ex16.alloc_features() for _ in range(n)]
        ms16, _ = timed(lambda: ex16.extract_batch(d_imgs, outs=outs16, workspace=ws16,
                                                   stream=stream), args.warmup, args.steps)
        n16 = int(sum(int(f.counters[0].item()) for f in outs16))
        fp16 = {"ms_per_step_launch_sequence": round(ms16, 4),
                "images_per_s": round(n / (ms16 * 1e-3), 2),
                "vs_fp32_launch_sequence": round(ms_eager / ms16, 3),
                "workspace_bytes": int(ws16.numel()), "workspace_bytes_fp32": int(ws.numel()),
                "keypoints_per_image": round(n16 / n, 1),
                "note": "levels of the octaves after the first stored as fp16 (pyramid_fp16 = 1); "
                        "parity against the oracle's fp16 mode under restated tolerances"}
        del ex16, ws16, outs16
        print(f"[bench] fp16 storage: {fp16}", file=sys.stderr, flush=True)

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
        launches_rec = sm.profile_launches()
        stats = sm.profile_stop()
        for name, (launches, sms, sbytes) in stats.items():
            stages[name] = dict(launches=launches // 2, ms=round(sms / 2, 4),
                                gbs=round(sbytes / (sms * 1e6), 1) if sbytes and sms else None)
        blur = stats.get("blur")
        if blur:
            launches, bms, bbytes = blur
            achieved = (bbytes / launches) / (bms / launches * 1e-3) / 1e9
            roofline = {"kernel": "Gaussian pyramid: k_chain (runs of levels, radius <= 8) and "
                                  "k_blur (single levels)", "bound": "hbm",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                        "avg_launch_us": round(1e3 * bms / launches, 2),
                        "bytes_per_launch": round(bbytes / launches),
                        "kernel_source_sha256": kernel_source_hash()}
            # every blur launch of the second profiled step: HBM and FMA-issue fractions
            blur_recs = [r for r in launches_rec if r[0] == "blur"]
            per = []
            for _, label, lms, lbytes, lfmas in blur_recs[len(blur_recs) // 2:]:
                sec = lms * 1e-3
                per.append({"launch": label, "us": round(lms * 1e3, 1),
                            "gb": round(lbytes / 1e9, 4), "gfma": round(lfmas / 1e9, 3),
                            "frac_hbm": round(lbytes / sec / 1e9 / HBM_PEAK_GBS, 3),
                            "frac_fma_nonpacked": round(lfmas / sec / (FMA_PEAK_T * 1e12), 3)})
            roofline["per_launch"] = per
            roofline["fma_peak_nonpacked_tfma_s"] = round(FMA_PEAK_T, 2)
            # pyramid + DoG + extrema judged on time under a stored-pyramid model of
            # 88 bytes per pixel-octave (5 levels read and written, 5 DoG planes
            # written and read back, the base read and written)
            det = stats.get("detect")
            if det:
                n_oct = wl.settings["n_octaves"] + wl.settings["upsample"]
                model = 88.0 * pixel_octaves(sizes, wl.settings["upsample"], n_oct)
                t_ms = (bms + det[1]) / 2
                roofline["pyramid_time_equivalent"] = {
                    "model_bytes_per_step": round(model), "blur_plus_detect_ms": round(t_ms, 4),
                    "gbs": round(model / (t_ms * 1e-3) / 1e9, 1),
                    "frac": round(model / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        print(f"[bench] stages: {json.dumps(stages)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle as it stands.  (i) one process, one BLAS thread, on the
        # first images of the batch until about 8 s of work; (ii) a pool of one
        # process per usable core (at most 16, the host share of one GPU),
        # one image each, wall time of the whole pool
        _oracle_worker_init()
        done, dt = 0, 0.0
        while done < n and (done == 0 or dt < 8.0):
            dt += _oracle_one((args.workload, args.images, done))
            done += 1
        single = round(done / dt, 5)
        workers = max(1, min(16, usable_cores(), n))
        t = time.perf_counter()
        with ProcessPoolExecutor(max_workers=workers, initializer=_oracle_worker_init) as pool:
            per_img = list(pool.map(_oracle_one, [(args.workload, args.images, k)
                                                  for k in range(workers)]))
        wall_pool = time.perf_counter() - t
        cpu = {"value": round(workers / wall_pool, 5), "unit": "images/s", "cores": workers,
               "kind": "oracle",
               "sample": f"pool of {workers} single-threaded FP64 NumPy processes, one of the "
                         f"first {workers} images each, full pipeline, {wall_pool:.1f} s wall",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(), "usable_cores": usable_cores(),
               "single_process": {"images_per_s": single, "threads": 1,
                                  "sample": f"the first {done} images, {dt:.1f} s"},
               "pool_mean_s_per_image": round(float(np.mean(per_img)), 2)}
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)

    serving = None
    if not args.no_serve_point:
        del ws
        torch.cuda.empty_cache()
        swl, simgs, sat, _, pts, buckets = serve_points(64, 2000, 200, [0.5], False)
        serving = {"workload": swl.name, "unique_images": len(simgs), "requests": 2000,
                   "warmup_requests": 200, "max_batch": 64, "max_inflight": 2,
                   "saturation_images_per_s": sat["images_per_s"],
                   "at_half_saturation": pts[0]["batched"], "qps": pts[0]["qps"],
                   "latency": "entry into submit (or the scheduled arrival, if later) to "
                              "observed completion",
                   "one_batch_of_64_launch_vs_buckets": buckets}

    matching = None
    if not args.no_match:
        matching = match_bench(32, 2000, 2000)
        matching["verification"] = verify_bench()

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
                   "tile_rows": tile_rows, "n_streams": n_streams, "blur_chain": blur_chain,
                   "detect_waves": detect_waves,
                   "upsample": wl.settings["upsample"], "octaves": wl.settings["n_octaves"] +
                   wl.settings["upsample"], "parallelism": "none (one GPU)"},
        "mpix_per_s": round(mpix / (ms * 1e-3), 2),
        "per_image_path": ({"images_per_s": round(n / (ms1 * 1e-3), 2),
                            "ms_per_step": round(ms1, 4)} if ms1 else None),
        "batched_vs_per_image": round(ms1 / ms, 3) if ms1 else None,
        "execution": mode,
        "ms_per_step_launch_sequence": round(ms_eager, 4),
        "ms_per_step_graph_replay": round(ms_graph, 4) if ms_graph else None,
        "bitwise_identical_graph_vs_launch_sequence": graph_identical,
        "ms_per_step_bucket_replay": round(ms_bucket, 4) if ms_bucket else None,
        "bitwise_identical_bucket_vs_launch_sequence": bucket_identical,
        "autotune": tune,
        "bitwise_identical_batched_vs_per_image": identical,
        "keypoints_per_image": round(n_kp / n, 1),
        "stages": stages,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "h2d": {"ms": round(h2d_s * 1e3, 2), "bytes": h2d_bytes,
                "gbs": round(h2d_bytes / h2d_s / 1e9, 2),
                "images_per_s_with_h2d": round(n / (ms * 1e-3 + h2d_s), 2),
                "first_pass_ms": round(h2d_passes[0] * 1e3, 2),
                "note": "pinned host buffers, one copy per image, before timing; best of two "
                        "passes after a first; not in value"},
        "fp16_storage": fp16,
        "serving": serving,
        "matching": matching,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
