/*
 * sift.h -- C ABI of the GPU-resident SIFT extraction library (gfx950).
 *
 * The library computes, for float32 grayscale images already resident in
 * device memory, the SIFT pipeline the paper lays out in Eq. (1) and its
 * method section (3.2): Gaussian scale space with 4-sigma truncated separable
 * kernels, DoG, 26-neighbour extrema with a contrast pre-gate, sub-pixel
 * refinement by a 3-D Taylor expansion solved with Cramer's rule (at most 5
 * steps) plus Hessian edge rejection, a 36-bin orientation histogram with
 * [1/4, 1/2, 1/4] smoothing and parabolic peak refinement, and the 4x4x8
 * gradient-histogram descriptor with optional domain-size pooling (DSP, the
 * "DSP Multi-Scale Descriptor Pooling" paragraph) and RootSIFT (the "RootSIFT
 * Normalization" paragraph).  Everything on the path is deterministic: the
 * same inputs give bit-identical outputs run after run, and an image gives
 * the same bits alone or inside any batch.
 *
 * Conventions
 *  - Every call returns sift_status; nothing throws across the ABI.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory read during the call only.
 *  - Extraction calls only enqueue work on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream) and return; outputs are valid once the
 *    stream has reached that point.  They never allocate device memory, copy
 *    to or from the host, or synchronise, so they may be captured in a HIP
 *    graph.
 *  - Argument errors are reported synchronously before anything is enqueued.
 *  - A handle is immutable after sift_create and may be shared by threads.
 *    A workspace must not be used by two extractions in flight at once.
 *  - Image pixel (r, c) sits at x = c, y = r; y grows downwards.  Angles are
 *    degrees in [0, 360), measured from +x towards +y.
 */
#ifndef SIFT_MI355X_H
#define SIFT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SIFT_OK = 0,
  SIFT_ERR_INVALID_ARG = 1,         /* null pointer, bad parameter, h/w <= 0, pitch < w */
  SIFT_ERR_IMAGE_TOO_SMALL = 2,     /* last octave would have min(h, w) < 2*border + 3 */
  SIFT_ERR_WORKSPACE_TOO_SMALL = 3, /* workspace_bytes below what *_workspace_size gives */
  SIFT_ERR_TOO_LARGE = 4,           /* image or batch beyond the library's index limits (side
                                       above 32768, a pyramid level of 2 GiB or more, batch
                                       above 4096) */
  SIFT_ERR_HIP = 5,                 /* HIP runtime error; sift_last_error() has the text */
  SIFT_ERR_NOT_SUPPORTED = 6        /* a parameter value the kernels do not implement */
} sift_status;

#define SIFT_MAX_DSP 16
#define SIFT_DESC_DIM 128

/* Extraction settings.  sift_params_default() fills the values noted. */
typedef struct {
  int32_t n_octaves;          /* 4: octaves 0..n_octaves-1 (plus -1 when upsample) */
  int32_t n_scales;           /* 3: s, DoG layers searched per octave, 1..6, provided
                                 every incremental blur has radius ceil(4 sigma) <= 24
                                 (with sigma0 1.6 that is s = 2..6; s = 1 would need 45
                                 and gives SIFT_ERR_NOT_SUPPORTED) */
  int32_t upsample;           /* 0: 1 adds octave -1 from a 2x bilinear upsample */
  float sigma0;               /* 1.6: blur of level 0 of each octave, octave pixels */
  float sigma_in;             /* 0.5: blur assumed present in the input */
  float contrast_threshold;   /* 0.04/3: |D(x^)| threshold, image values in [0,1] */
  float prefilter_ratio;      /* 0.5: candidate pre-gate |D| > ratio * threshold */
  float edge_ratio;           /* 10: Hessian principal-curvature ratio bound */
  int32_t border;             /* 5: frame of each octave not searched, >= 1 */
  int32_t refine_iters;       /* 5: Newton steps before a candidate is dropped */
  int32_t ori_bins;           /* 36: orientation histogram bins (fixed) */
  float ori_sigma_factor;     /* 1.5: orientation window sigma / keypoint sigma */
  float ori_radius_factor;    /* 3.0: window radius = round(factor * window sigma) */
  float ori_peak_ratio;       /* 0.8: secondary peaks kept down to ratio * max */
  int32_t upright;            /* 0: 1 assigns the single angle 0 */
  int32_t desc_width;         /* 4: spatial cells per side (fixed) */
  int32_t desc_ori_bins;      /* 8: orientation bins per cell (fixed) */
  float desc_magnif;          /* 3.0: cell width / keypoint sigma */
  float desc_clamp;           /* 0.2: clamp after the first L2 normalisation */
  int32_t n_dsp;              /* 1: number of domain sizes pooled (1..SIFT_MAX_DSP) */
  float dsp_scales[SIFT_MAX_DSP]; /* {1}: domain sizes relative to the keypoint scale, in
                                 (0, 64); the largest descriptor window that desc_magnif,
                                 the largest size and the largest keypoint scale
                                 (sigma0 * 2^((s + 1/2) / s)) can give must stay below
                                 2048 samples a side, else SIFT_ERR_NOT_SUPPORTED (with
                                 the defaults: sizes up to about 26) */
  int32_t rootsift;           /* 0: 1 applies L1 normalisation then sqrt */
  int32_t max_keypoints;      /* 65536: keypoints kept per image (canonical order) */
  int32_t max_candidates;     /* 65536: detections refined per image (canonical order) */
  int32_t tile_rows;          /* 0: library choice; else 32, 64, 128, 256 or 512: the most
                                 rows per blur work-group (octaves too small to give enough
                                 work-groups at that height use shorter chunks).  Any value
                                 gives bit-identical results (tuning only) */
  int32_t n_streams;          /* 0: library choice (a batch of 8 or more images runs as 4
                                 sub-batches on the handle's own streams, concurrently);
                                 1..8: that many sub-batches.  Any value gives bit-identical
                                 results (tuning only) */
  int32_t upsample_max_pixels; /* 0: no limit.  With upsample = 1, an image of more than
                                 this many pixels (height * width) is extracted without the
                                 upsampled octave -1, exactly as with upsample = 0: the
                                 paper's VRAM-adaptive suppression of the 2x base, which it
                                 applies above 4 MP (4000000) on a 4 GB GPU.  A batch may
                                 mix both kinds of image */
  int32_t pyramid_fp16;       /* 0: every level fp32.  1: the levels of every octave after
                                 the first are stored as fp16 (of L - 0.5, nearest even),
                                 all arithmetic stays fp32 and the first octave stays fp32
                                 (section 3.2, "GPU Pipeline Stages"): about half the pyramid
                                 bytes of those octaves, at fp16 accuracy for their keypoints */
  int32_t blur_chain;         /* 0: library choice (2); 1: one launch per Gaussian level; 2..4: up
                                 to that many consecutive levels of an octave blurred in one
                                 launch (runs of radius <= 8 that the library has a kernel
                                 for), so the levels between are not read back from memory.
                                 Any value gives bit-identical results (tuning only) */
  int32_t detect_waves;       /* 0: library choice (4); 4 or 8: waves per work-group of the
                                 extrema search, which share a band's column segments.
                                 Either gives bit-identical results (tuning only) */
} sift_params;

/* One keypoint, 48 bytes.  Keypoints of an image come in canonical order:
 * by the detection they were refined from -- (octave, src_layer, src_iy,
 * src_ix) ascending -- then by ascending orientation bin. */
typedef struct {
  float x, y;          /* input-image pixel coordinates of the refined extremum */
  float sigma;         /* scale in input-image pixels */
  float angle;         /* degrees, [0, 360) */
  float response;      /* |D(x^)|, the interpolated DoG magnitude */
  int32_t octave;      /* -1 .. n_octaves-1 */
  int32_t layer;       /* DoG layer 1..n_scales after refinement */
  int32_t ix, iy;      /* integer pixel after refinement, octave coordinates */
  int32_t src_layer;   /* the detection this keypoint was refined from: */
  int32_t src_iy;      /*   layer, row and column in octave coordinates */
  int32_t src_ix;
} sift_keypoint;

/* Where one image's results go; every pointer is device memory owned by the
 * caller.  keypoints[capacity], descriptors[capacity][128] row-major
 * (index (row_cell*4 + col_cell)*8 + orientation_bin).  On completion:
 * *count = min(*n_found, capacity, max_keypoints); *n_found = keypoints
 * produced from the refined detections; *n_candidates = detections found
 * (may exceed max_candidates, in which case only the first max_candidates in
 * canonical order were refined).  Any of n_found / n_candidates may be NULL. */
typedef struct {
  sift_keypoint* keypoints;
  float* descriptors;
  int32_t* count;
  int32_t* n_found;
  int32_t* n_candidates;
  int32_t capacity;
} sift_output;

typedef struct sift_handle sift_handle;

/* Fill *p with the defaults listed above (the settings section 3.2 states: 36
 * orientation bins, 4x4x8 descriptor, at most 5 refinement steps, 4-sigma
 * truncation; the rest as in Lowe's SIFT, which the paper follows).  Errors:
 * INVALID_ARG if p is NULL. */
sift_status sift_params_default(sift_params* p);

/* Validate *p and create an immutable handle (host memory only; no device
 * allocation).  It derives the level blurs of section 3.2 "GPU Pipeline
 * Stages" (sigma0 * 2^(i/s) per level, each level blurred incrementally from
 * the previous one with a separable kernel truncated at 4 sigma).  Errors: INVALID_ARG / NOT_SUPPORTED for bad or unimplemented
 * settings.  The caller releases the handle with sift_destroy. */
sift_status sift_create(const sift_params* p, sift_handle** out);
void sift_destroy(sift_handle* h);

/* Copy the handle's settings into *p. */
sift_status sift_get_params(const sift_handle* h, sift_params* p);

/* Device workspace bytes sift_extract needs for a height x width image: the
 * pyramid of section 3.2 (s + 3 levels per octave) plus detection and
 * keypoint state.  Errors: INVALID_ARG, IMAGE_TOO_SMALL, TOO_LARGE. */
sift_status sift_workspace_size(const sift_handle* h, int32_t height, int32_t width,
                                size_t* bytes);

/* Extract one image, the whole extraction of Eq. (1) as section 3.2 "GPU
 * Pipeline Stages" lays it out (scale space, DoG, extrema with the contrast
 * pre-gate, refinement and edge rejection, orientation, descriptor with the
 * "DSP Multi-Scale Descriptor Pooling" and "RootSIFT Normalization"
 * paragraphs), on the GPU from input to descriptors (the device-resident
 * pipeline of section 3.1, "Architecture Overview").  d_image is a device float32 array
 * of height rows of `pitch` elements (pitch >= width), values nominally in
 * [0, 1].
 * d_workspace (device, >= sift_workspace_size bytes, 256-byte aligned) holds
 * the pyramid and all intermediate state; its contents on entry do not
 * matter.  Results land in *out (see sift_output). */
sift_status sift_extract(sift_handle* h, const float* d_image, int32_t height, int32_t width,
                         int64_t pitch, void* d_workspace, size_t workspace_bytes,
                         const sift_output* out, void* stream);

/*
 * Extraction without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and results as sift_extract (bit-identical
 * outputs), but the workspace is a static device array inside the library,
 * SIFT_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, held from module load until the
 * process ends: enough for a 1600x1066 image with the default settings, or a
 * 640x480 image with the upsampled octave.  The call allocates nothing (no
 * hipMalloc/hipFree, no allocating library routine); its first call on a
 * device looks up that device's array address.  The image, outputs and stream
 * belong to the current device.  Errors: as sift_extract, plus
 * WORKSPACE_TOO_SMALL when sift_workspace_size for the image exceeds the
 * array (sift_last_error() gives both sizes).  Every call on one GPU uses that
 * GPU's single array and leaves the last call's state in it (nothing in it
 * needs clearing: each extraction writes every word it reads before reading
 * it).  Calls whose work overlaps on one GPU (enqueued on different streams,
 * or from different threads) race on the array; calls enqueued on one stream
 * run one after another and are safe.
 */
#define SIFT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sift_status sift_extract_noalloc(sift_handle* h, const float* d_image, int32_t height,
                                 int32_t width, int64_t pitch, const sift_output* out,
                                 void* stream);
/* SIFT_NOALLOC_SCRATCH_BYTES as built into the library. */
size_t sift_noalloc_scratch_bytes(void);

/* Workspace bytes for a batch of n images with the given sizes (host arrays). */
sift_status sift_batch_workspace_size(const sift_handle* h, int32_t n, const int32_t* heights,
                                      const int32_t* widths, size_t* bytes);

/* Extract n images of possibly different sizes in one launch sequence:
 * every stage runs once for the whole batch over (image, octave, tile) work
 * items.  The paper runs its ~20 kernels once per image and names that launch
 * count as its throughput ceiling (section 5, "Throughput Ceiling vs. Learned
 * Detectors"); the per-image computation is that of sift_extract.  d_images, heights, widths, pitches and outs are host arrays of n
 * entries (d_images[k] is a device pointer).  Each image's results are
 * bit-identical to sift_extract on that image alone. */
sift_status sift_extract_batch(sift_handle* h, int32_t n, const float* const* d_images,
                               const int32_t* heights, const int32_t* widths,
                               const int64_t* pitches, void* d_workspace,
                               size_t workspace_bytes, const sift_output* outs, void* stream);

/* Inspection of a workspace after sift_extract (tests and tooling): device
 * address of Gaussian level `level` (0..n_scales+2) of octave `octave`
 * (-1 or 0 .. n_octaves-1) for an image of height x width placed at
 * d_workspace, with its size and row pitch in elements.  Levels are stored
 * relative to mid-grey: the value held is L - 0.5. */
sift_status sift_workspace_level(const sift_handle* h, int32_t height, int32_t width,
                                 const void* d_workspace, int32_t octave, int32_t level,
                                 const float** d_level, int32_t* level_height,
                                 int32_t* level_width, int32_t* level_pitch);
/* Bytes per stored element of the levels of that octave: 4 (fp32), or 2 (fp16,
 * the octaves after the first with pyramid_fp16); *d_level then points at
 * fp16 values. */
sift_status sift_workspace_level_bytes(const sift_handle* h, int32_t height, int32_t width,
                                       int32_t octave, int32_t* elem_bytes);

/* Stage profiling (benchmarks and tests; not for production paths).
 * sift_profile_start begins recording, for every extraction this process then
 * enqueues, a HIP event before and after each stage on the extraction's
 * stream, together with the stage's algorithmic HBM bytes (what the stage must
 * read and write at least: each pyramid level read once and written once,
 * detection reading the s+3 levels once, ...).  sift_profile_stop waits for
 * the recorded events, writes per-stage totals into stats[0..max_stats-1],
 * sets *n_stats and ends recording.  Recording is process-wide; call
 * start/stop from one thread.  Errors: HIP if event creation or timing fails,
 * INVALID_ARG for null arguments or stop without start. */
typedef struct {
  char name[32];        /* stage: "blur", "detect", "describe", ... */
  int32_t launches;     /* kernel launches recorded */
  double ms;            /* summed event time over the launches */
  double bytes;         /* summed algorithmic bytes over the launches */
} sift_stage_stat;

sift_status sift_profile_start(void);
sift_status sift_profile_stop(sift_stage_stat* stats, int32_t max_stats, int32_t* n_stats);

/* The launches recorded so far, one entry each in enqueue order (at most
 * max_out; waits for their events; recording continues): stage name, a
 * detail label (blur: "o<octave> l<level> R<radius>"), event time, algorithmic
 * bytes and the fused multiply-adds the launch must issue (blur: two passes
 * of 2R + 1 taps per output pixel; 0 where not counted).  Call between
 * sift_profile_start and sift_profile_stop. */
typedef struct {
  char stage[32];
  char label[32];
  double ms;
  double bytes;
  double fmas;
} sift_launch_stat;

sift_status sift_profile_launches(sift_launch_stat* out, int32_t max_out, int32_t* n_out);

/* Bounds checks (tests and debugging; not for production paths).  The same
 * sources built with -DSIFT_DEBUG_BOUNDS (libsift_mi355x_bounds.so beside
 * the library) make the kernels count every access that falls outside the
 * memory it belongs to: an image's workspace region, its input image, its
 * output arrays, an LDS histogram; a pair's descriptors, summaries, matches,
 * correspondences, hypotheses and models.  The access still
 * happens (nothing traps); outputs are those of the normal library.
 * sift_bounds_violations waits for the device (hipDeviceSynchronize), sets
 * *count to the accesses counted since the last reset, process-wide, and
 * zeroes the counters when reset is non-zero.  Errors: INVALID_ARG for a null
 * count; NOT_SUPPORTED from a library built without the checks (*count = 0);
 * HIP if the device cannot be read. */
sift_status sift_bounds_violations(int32_t reset, uint64_t* count);

/* Static text for a status code. */
/*
 * Replayable batches (HIP graphs).  For a batch whose shapes and buffers
 * repeat (one graph per size bucket), sift_graph_create records the whole
 * launch sequence of sift_extract_batch with these exact arguments into a HIP
 * graph, on a private stream (nothing runs at create time), and
 * sift_graph_launch replays it on `stream` with one call.  A replay reads the
 * images at the recorded addresses as they are when it runs, so the caller
 * rewrites them in place between replays; the workspace and outputs are the
 * recorded ones and must not be in use by anything else while a replay is in
 * flight.  Results are bit-identical to sift_extract_batch.  Stage profiling
 * does not see replays.
 */
typedef struct sift_graph sift_graph;

sift_status sift_graph_create(sift_handle* h, int32_t n, const float* const* d_images,
                              const int32_t* heights, const int32_t* widths,
                              const int64_t* pitches, void* d_workspace, size_t workspace_bytes,
                              const sift_output* outs, sift_graph** out);
sift_status sift_graph_launch(sift_graph* g, void* stream);
sift_status sift_graph_destroy(sift_graph* g);

/*
 * Size buckets (replay for images that vary in size).  A bucket is a graph of
 * the launch sequence for up to n_slots images of at most max_height x
 * max_width each, recorded once with grids that cover every slot at the
 * largest size.  sift_bucket_launch writes the image table for the n images
 * given (their own sizes, host arrays as sift_extract_batch takes them) with a
 * few setup launches on `stream` and replays the graph there; the kernels read
 * each image's size from the table and surplus work-groups exit at once, so
 * each image's results are bit-identical to sift_extract on it.  Slots past n
 * stay empty.  Every image of a launch must take the same octave structure as
 * the bucket's largest size (with upsample_max_pixels, both sides of the
 * limit need their own buckets).  The workspace (sift_bucket_workspace_size,
 * 256-byte aligned) belongs to the bucket; a bucket serves one launch at a
 * time, and the handle must outlive it.  Errors: INVALID_ARG for sizes beyond
 * the bucket, too many images, or a different octave structure;
 * WORKSPACE_TOO_SMALL; HIP.
 */
typedef struct sift_bucket sift_bucket;

sift_status sift_bucket_workspace_size(const sift_handle* h, int32_t n_slots, int32_t max_height,
                                       int32_t max_width, size_t* bytes);
sift_status sift_bucket_create(sift_handle* h, int32_t n_slots, int32_t max_height,
                               int32_t max_width, void* d_workspace, size_t workspace_bytes,
                               sift_bucket** out);
sift_status sift_bucket_launch(sift_bucket* b, int32_t n, const float* const* d_images,
                               const int32_t* heights, const int32_t* widths,
                               const int64_t* pitches, const sift_output* outs, void* stream);
sift_status sift_bucket_destroy(sift_bucket* b);

/*
 * Tuning.  sift_autotune_batch times sift_extract_batch on the given batch
 * for every cap on the blur chunk height (64, 128, 256, 512 rows; all give
 * bit-identical results) and returns the fastest in *best_tile_rows and the mean time of
 * each candidate, in that order, in ms[4] (host, may be NULL).  It runs
 * `warmup` untimed and `reps` timed extractions per candidate on `stream` and
 * waits for them (it synchronises; it is not for a capture or a hot loop).
 * Set the result as sift_params.tile_rows of the handle used afterwards.
 */
sift_status sift_autotune_batch(const sift_params* p, int32_t n, const float* const* d_images,
                                const int32_t* heights, const int32_t* widths,
                                const int64_t* pitches, void* d_workspace,
                                size_t workspace_bytes, const sift_output* outs, void* stream,
                                int32_t warmup, int32_t reps, int32_t* best_tile_rows,
                                float* ms);

/*
 * Tuning over the launch knobs, with a persisted cache.  sift_autotune
 * times sift_extract_batch on the given batch for every blur chunk-height cap
 * (64, 128, 256, 512) and every sub-batch count (1, 2, 4, 8, at most n) at
 * the settings' blur_chain and detect_waves, then the other pyramid run
 * lengths (1, 2, 3 levels per launch) at the best of those, then the other
 * waves per detection work-group (4 or 8) at the best so far -- all of them
 * give bit-identical results -- and returns the fastest in *out.  With
 * cache_path non-NULL it first looks the batch up in that text file (one line
 * per entry: key, tile_rows, n_streams, blur_chain, detect_waves, ms; the last
 * entry of a key wins) and, on a hit, returns the entry without timing
 * (from_cache = 1); after timing it appends the winner.  The key names the
 * device (name, architecture, compute units), the settings other than the four
 * tuned fields, the image count,
 * the total input pixels to two significant figures and the execution form:
 * as_graph = 0 times the launch sequence (sift_extract_batch), 1 times
 * replays of it recorded as a graph (sift_graph_*), whose best split can
 * differ.  It synchronises on `stream` when it times; not for a capture or a
 * hot loop.
 */
typedef struct {
  int32_t tile_rows;    /* chosen chunk-height cap */
  int32_t n_streams;    /* chosen sub-batch count */
  float ms;             /* its mean time per batch, ms */
  int32_t from_cache;   /* 1: read from the cache file, nothing timed */
  int32_t n_tried;      /* candidates timed */
  int32_t blur_chain;   /* chosen pyramid levels per launch (1..3) */
  int32_t detect_waves; /* chosen waves per detection work-group (4 or 8) */
} sift_tuning;

/* Workspace that every candidate of sift_autotune fits in (a split into more
 * sub-batches needs a few headers more); candidates that do not fit the
 * workspace given to sift_autotune are skipped. */
sift_status sift_autotune_workspace_size(const sift_params* p, int32_t n, const int32_t* heights,
                                         const int32_t* widths, size_t* bytes);
sift_status sift_autotune(const sift_params* p, int32_t n, const float* const* d_images,
                          const int32_t* heights, const int32_t* widths, const int64_t* pitches,
                          void* d_workspace, size_t workspace_bytes, const sift_output* outs,
                          void* stream, int32_t warmup, int32_t reps, int32_t as_graph,
                          const char* cache_path, sift_tuning* out);

/*
 * Serving (a request stream of images of any sizes).
 *
 * The paper extracts one image per call; this is a continuous-batching
 * front end over sift_extract_batch.  sift_server_create copies the params,
 * takes a caller-owned device arena (256-byte aligned; the server carves
 * per-batch workspaces out of it and never allocates) and starts one host
 * worker thread bound to the device current at create time.  The worker
 * repeatedly (1) retires batches whose completion event has fired, freeing
 * their arena ranges, and (2) while fewer than max_inflight batches are in
 * flight, admits pending requests in arrival order into one batch as long as
 * the batch has at most max_batch images and its workspace fits in a free
 * arena range (admission by footprint), and launches it on one of
 * max_inflight streams of its own (default priority), so consecutive batches
 * overlap.  A batch is formed under the server's lock and its launch sequence
 * enqueued with the lock released; every stream has its own handle, so the
 * sub-batch streams of a large batch are never shared between batches in
 * flight.  Each request's outputs are bit-identical to sift_extract on the
 * same image.
 *
 * sift_server_submit enqueues a request and returns at once with a ticket;
 * the image and the output buffers (device) must stay valid and untouched
 * until the ticket is done.  A request whose workspace alone exceeds the arena
 * gives SIFT_ERR_TOO_LARGE; size errors are reported as by sift_extract.
 * sift_server_poll reports whether a ticket is done and, once it is, its
 * latency (from entry into sift_server_submit to observed completion,
 * milliseconds) and forgets it; sift_server_wait blocks until the ticket is
 * done, then behaves as poll.  Unknown (or already reported) tickets give
 * SIFT_ERR_INVALID_ARG.  sift_server_destroy finishes every pending and
 * in-flight request, stops the worker and releases the streams; the arena
 * stays the caller's.  All server calls are thread-safe.  max_batch 1 and
 * max_inflight 1 serve requests one at a time in arrival order (the plain
 * per-image path).
 *
 * sift_server_batch_bytes (host arithmetic only) gives the arena bytes the
 * server reserves for one batch of n images of the given sizes (host arrays):
 * an arena of at least that many bytes can take them as one batch.  It is at
 * least sift_batch_workspace_size for the same images, whatever n_streams.
 */
typedef struct sift_server sift_server;

typedef struct {
  int64_t submitted;      /* requests accepted */
  int64_t completed;      /* requests whose batch has finished */
  int64_t batches;        /* batches launched */
  int64_t peak_arena;     /* largest arena bytes in use at once */
  int64_t peak_inflight;  /* largest number of batches in flight at once */
  int64_t largest_batch;  /* most images in one batch */
  int64_t overlapped_batches;  /* batches launched while another was still in flight */
} sift_server_stats;

sift_status sift_server_batch_bytes(const sift_params* p, int32_t n, const int32_t* heights,
                                    const int32_t* widths, size_t* bytes);

sift_status sift_server_create(const sift_params* p, void* d_arena, size_t arena_bytes,
                               int32_t max_batch, int32_t max_inflight, sift_server** out);
sift_status sift_server_submit(sift_server* s, const float* d_image, int32_t height,
                               int32_t width, int64_t pitch, const sift_output* out,
                               uint64_t* ticket);
/* n requests at once (host arrays of n entries, as sift_extract_batch takes
 * them): all are checked before any is queued (an error queues none), then
 * they join the queue together, so a worker that is idle sees the whole group
 * when it next forms a batch.  tickets[n] receives their tickets. */
sift_status sift_server_submit_n(sift_server* s, int32_t n, const float* const* d_images,
                                 const int32_t* heights, const int32_t* widths,
                                 const int64_t* pitches, const sift_output* outs,
                                 uint64_t* tickets);
sift_status sift_server_poll(sift_server* s, uint64_t ticket, int32_t* done, double* latency_ms);
sift_status sift_server_wait(sift_server* s, uint64_t ticket, double* latency_ms);
sift_status sift_server_get_stats(sift_server* s, sift_server_stats* stats);
sift_status sift_server_destroy(sift_server* s);

/*
 * Descriptor matching: the symmetric ratio test of the paper's matching step
 * (Section 3.4, "Descriptor Matching", backend (1): a similarity matrix from
 * fp16 descriptors on the matrix cores, a nearest-neighbour ratio test and
 * mutual-consistency filtering), for many pairs of descriptor sets in one
 * launch sequence.
 *
 * For a pair (a, b): s_ij = <fp16(a_i), fp16(b_j)>, the descriptors rounded
 * to fp16 (nearest even) and the products accumulated in fp32 by the matrix
 * cores in an order fixed by the code (run-to-run bit-identical).  With
 * D = max(2 - 2 s, 0) (squared distance of unit vectors) a_i's nearest
 * neighbour j is the largest s_ij (smallest j among equals), D1 its distance,
 * D2 the second-nearest's (4 if b has one row); likewise b_j's nearest in a.
 * The pair (i, j) is kept when i and j are each other's nearest neighbours
 * and D1 < fp32(ratio^2) * D2 holds both ways (taken in fp32).  Matches come
 * in ascending query index.
 *
 * Each sift_match_pair names device memory the caller owns: desc_a
 * [cap_a][128] and desc_b [cap_b][128] fp32 row-major (sift_output's
 * descriptor layout); count_a / count_b point at the number of rows in use
 * (clamped to the cap; e.g. sift_output.count, so extraction and matching
 * chain on the device without the host reading counts), or are NULL for
 * cap_a / cap_b rows; matches [capacity]; *n_matches receives the number
 * written (min(kept, capacity)), *n_found (may be NULL) the number kept.
 * Caps are host values that size the launch; 0 <= cap <= 65536.
 * sift_match_workspace_size gives the workspace for the pairs (host array);
 * sift_match_batch enqueues the matching on `stream` (no allocation, copy
 * or synchronisation).  Errors: INVALID_ARG for null pointers, caps out of
 * range, ratio not in (0, 1], WORKSPACE_TOO_SMALL; HIP for launch failures.
 */
typedef struct {
  int32_t query;        /* row of desc_a */
  int32_t train;        /* row of desc_b */
  float similarity;     /* s_ij as accumulated */
  float distance;       /* sqrt(max(2 - 2 s_ij, 0)) */
} sift_match;

typedef struct {
  const float* desc_a;
  const int32_t* count_a;
  int32_t cap_a;
  const float* desc_b;
  const int32_t* count_b;
  int32_t cap_b;
  sift_match* matches;
  int32_t* n_matches;
  int32_t* n_found;
  int32_t capacity;
} sift_match_pair;

#define SIFT_MATCH_MAX_ROWS 65536
#define SIFT_MATCH_MAX_PAIRS 4096

sift_status sift_match_workspace_size(int32_t n, const sift_match_pair* pairs, size_t* bytes);
sift_status sift_match_batch(int32_t n, const sift_match_pair* pairs, float ratio,
                             void* d_workspace, size_t workspace_bytes, void* stream);

/*
 * Geometric verification of matched pairs: the estimator after matching
 * (Section 3.6, "GPU MAGSAC++": many minimal-sample hypotheses solved in one
 * batch, scored by soft marginalisation), as a planar homography, for many
 * pairs in one launch sequence.  All arithmetic is fp64.
 *
 * For a pair, the correspondences are the first *n_matches records of
 * `matches` (sift_match_batch output: query indexes kp_a, train kp_b), their
 * keypoint positions in pixels.  Each point set is normalised (mean to 0, mean
 * distance to sqrt 2).  Hypothesis k (k < n_hyp) takes correspondences
 * floor(u[k][j] * N), j = 0..3, from the caller's numbers d_samples
 * [n_hyp][4] in [0, 1) (device; the same numbers serve every pair), and
 * solves the 4-point DLT system (h33 = 1) by Gaussian elimination with partial
 * pivoting; repeated indices or a pivot below 1e-12 of the largest entry give
 * no hypothesis.  A correspondence with transfer residual r (pixels in image
 * b) counts w(r) = sqrt(pi/2) / sigma_max * (erf(tau / sqrt 2) - erf(r /
 * (sqrt 2 sigma_max))) for r < tau * sigma_max, tau = sqrt(2 ln 100), else 0:
 * the likelihood of a Rayleigh residual truncated at its 0.99 quantile,
 * marginalised over a noise scale uniform on (0, sigma_max].  The hypothesis
 * of largest summed w (first among equals) is refined by at most refine_iters
 * steps of reweighted least squares on the normalised DLT rows, each kept only
 * if it raises the score.  Outputs (device): H[9] row-major with h33 = 1 (NaN
 * when there is no hypothesis, e.g. fewer than 4 correspondences), *score,
 * *n_inliers (w > 0), *best (hypothesis index or -1; may be NULL), weights[cap]
 * (final w per correspondence, 0 past N; may be NULL).  Bit-identical run to
 * run.  sift_verify_workspace_size sizes the workspace; sift_verify_batch only
 * enqueues.  Errors: INVALID_ARG (null pointers, cap beyond 65536, n_hyp
 * beyond 65536, sigma_max <= 0), WORKSPACE_TOO_SMALL, HIP.
 */
typedef struct {
  const sift_keypoint* kp_a;
  const sift_keypoint* kp_b;
  const sift_match* matches;
  const int32_t* n_matches;
  int32_t cap;
  double* H;
  double* score;
  int32_t* n_inliers;
  int32_t* best;
  float* weights;
} sift_verify_pair;

#define SIFT_VERIFY_MAX_PAIRS 4096
#define SIFT_VERIFY_MAX_HYPOTHESES 65536

sift_status sift_verify_workspace_size(int32_t n, const sift_verify_pair* pairs, int32_t n_hyp,
                                       size_t* bytes);
sift_status sift_verify_batch(int32_t n, const sift_verify_pair* pairs, const float* d_samples,
                              int32_t n_hyp, float sigma_max, int32_t refine_iters,
                              void* d_workspace, size_t workspace_bytes, void* stream);

const char* sift_status_string(sift_status st);
/* Detail of the last error on the calling thread ("" if none). */
const char* sift_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIFT_MI355X_H */
