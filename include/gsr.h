/*
 * gsr.h -- C ABI of libgsr, a batched 3D Gaussian Splatting renderer for
 * thousands of rigid-body simulation environments per step on AMD Instinct
 * MI355X (gfx950).
 *
 * What it renders: the batch renderer of GS-Playground (arXiv 2604.25459),
 * Sec. "Batch Renderer Optimization" and Sec. "System Overview" (data flow:
 * the physics engine's rigid-body poses drive Gaussian clusters through
 * Rigid-Link Gaussian Kinematics, RLGK; the renderer returns RGB images and
 * depth maps per environment).  The image model is standard 3D Gaussian
 * Splatting (Kerbl et al. 2023, the representation the paper renders with;
 * the renderer is built on gsplat): EWA projection, spherical-harmonic colour,
 * tile binning by a (image, tile, depth) key sort, front-to-back alpha
 * compositing with alpha = min(0.99, o exp(-q/2)), Gaussians below alpha 1/255
 * skipped, pixels stopped once transmittance would fall below 1e-4.
 *
 * Conventions (fixed by this library where the paper is silent):
 *   - world right-handed; cameras OpenCV style (x right, y down, z forward);
 *     a viewmat is the 3x4 world->camera matrix [R | t], row-major floats;
 *   - quaternions are (w, x, y, z), normalised on use;
 *   - scales are linear (> 0), opacities are activated values in [0, 1];
 *   - body poses are world-from-body (qw, qx, qy, qz, tx, ty, tz);
 *   - Gaussian index g = storage order: static background first, then the
 *     Gaussians of body 0, body 1, ... (ranges given by body_offsets);
 *   - pixel (x, y) has its centre at (x + 0.5, y + 0.5);
 *   - images are ordered camera-slot-major: image i = c * n_envs + e.
 *
 * Threading: a context may be used from several host threads; render calls
 * on different streams run concurrently, each with its own working memory.
 *
 * Errors: every call returns GSR_OK (0) or a negative GSR_E_* code.  Arguments
 * are validated before any device work is enqueued; on failure nothing is
 * enqueued and gsr_last_error() (per host thread) describes the problem.  An
 * asynchronous device fault is sticky: the context reports GSR_E_DEVICE from
 * then on.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_OK 0
#define GSR_E_INVALID (-1)   /* bad argument (null pointer, size, degree, ...) */
#define GSR_E_OOM (-2)       /* device or host allocation failed */
#define GSR_E_DEVICE (-3)    /* no gfx950 device, or a HIP call failed */
#define GSR_E_NOT_FOUND (-4) /* unknown scene id or ticket */
#define GSR_E_BUSY (-5)      /* scene still referenced by in-flight work */
#define GSR_E_REJECTED (-6)  /* request can never fit the server's memory budget (one image too large) */
#define GSR_E_OVERFLOW (-7)  /* internal capacity exceeded (only surfaced if a retry fails) */
#define GSR_E_TIMEOUT (-8)   /* gsr_wait timed out */

#define GSR_STORAGE_F32 0    /* attributes and SH stored as float32 */
#define GSR_STORAGE_F16 1    /* scales, rotations, opacity and SH as IEEE half; means stay float32 */
#define GSR_STORAGE_BF16 2   /* same with bfloat16 */

#define GSR_OBS_U8 1         /* observation bytes: round(255 x), [..][H][W][3] uint8 */
#define GSR_OBS_F16 2        /* observation halves: x rounded to nearest even, [..][H][W][3] */

#define GSR_MEM_HOST 0       /* scene arrays are host pointers */
#define GSR_MEM_DEVICE 1     /* scene arrays are device pointers on the context's device */

typedef struct gsr_ctx gsr_ctx;
typedef struct gsr_server gsr_server;

/* Context options; zero-initialise for defaults. */
typedef struct {
    int tile_size;          /* 8, 16 or 32 pixels; 0 = 16 */
    int images_per_thread;  /* images one projection thread handles (1..16); 0 = 16 */
    int64_t chunk_bytes;    /* device working-memory budget per render chunk; 0 = 48 GiB, and never above 40 % of
                               the device memory free when a render is planned (with `overlap` on, a render of
                               several chunks holds two such working sets); chunks of a render are of equal size */
    float cutoff;           /* splat radius in standard deviations; 0 = 3.33 (conservative for alpha >= 1/255) */
    int profile;            /* 1 = record HIP events around every pipeline stage (see gsr_stage_times) */
    int graphs;             /* 0 = capture the per-chunk stages of gsr_render into hipGraphs and replay them
                               (default); -1 = launch every kernel eagerly */
    int overlap;            /* 0 = when a render has several memory chunks, run alternate chunks on two streams
                               (the caller's and an internal one, joined back before the call's work ends) with
                               a second working set, so one chunk's binning overlaps another's rasterisation
                               (default; a render whose second working set does not fit in device memory
                               runs on one stream); -1 = one stream, one working set */
    int sync_lists;         /* 0 = the first gsr_render of a job shape (scene, image sizes, launch parameters) on a
                               working set waits at every chunk for its list totals and sizes the tile-list buffers;
                               later renders of that shape enqueue every chunk and return without waiting, the device
                               checking each chunk's totals against the buffers (default); -1 = always wait */
    int list_cap;           /* tests of the overflow path: > 0 caps the list capacity (entries) that asynchronous
                               chunks may use, so that their lists overflow; 0 = off */
    int reserved[3];
} gsr_options;

/* A scene: static background plus Gaussian clusters bound to rigid bodies
 * (RLGK, Sec. "Batch Renderer Optimization").  All arrays are float32,
 * row-major, of the given shapes. */
typedef struct {
    int64_t n;                    /* Gaussians, >= 0 */
    int sh_degree;                /* 0..3; K = (sh_degree + 1)^2 coefficients per channel */
    int storage;                  /* GSR_STORAGE_* */
    int mem_kind;                 /* GSR_MEM_HOST or GSR_MEM_DEVICE for the arrays below */
    int n_bodies;                 /* B >= 0 */
    const float* means;           /* [n][3]; body Gaussians in their body frame */
    const float* scales;          /* [n][3] */
    const float* quats;           /* [n][4] (w, x, y, z) */
    const float* opacities;       /* [n] */
    const float* sh;              /* [n][K][3] (coefficient-major, channel-minor) */
    const int64_t* body_offsets;  /* host, [B + 1]: [0, off[0]) static, body b owns [off[b], off[b+1]), off[B] = n */
} gsr_scene_desc;

/* One camera slot.  Every environment has one camera per slot; slots may
 * differ in resolution and intrinsics.
 *
 * Body-attached cameras (a wrist camera riding on a robot link): with
 * attach_body = b >= 0 the slot's viewmats are body-b -> camera transforms
 * [R_o | t_o] (one per env, so a per-env offset also carries camera-pose
 * randomisation), and the world -> camera transform is composed on the
 * device from the env's pose (q_b, t_b) of body b:
 *     R_c = R_o R(q_b)^T,  t_c = t_o - R_c t_b
 * in binary32, each product and sum rounded separately, sums left to right
 * (so tile lists stay bit-exact).  attach_body = -1: viewmats are
 * world -> camera as given. */
typedef struct {
    int width, height;            /* pixels, 1..8192 */
    float fx, fy, cx, cy;         /* pinhole intrinsics in pixels */
    float near_plane;             /* Gaussians with camera depth <= near_plane are culled; > 0 */
    int attach_body;              /* -1, or the body (0..B-1) the camera rides on */
} gsr_camera;

/* Fused observation epilogue (image-level appearance randomisation and a
 * compact pixel format for a policy network, applied as each tile's pixels
 * are written; the domain randomisation of brightness, contrast and exposure
 * of the paper's sim-to-real manipulation experiment, Sec. "Vision-Centric
 * Manipulation Learning").  Per image
 * (camera slot c, env e), with the parameter arrays indexed [c][e] and each
 * optional (NULL = identity), on every channel of the composited colour rgb,
 * each step rounded to binary32:
 *     x = rgb * gain;  x = x - 0.5;  x = x * contrast;  x = x + 0.5;
 *     x = x + brightness;  x = min(max(x, 0), 1)
 * then GSR_OBS_U8 stores floor(x * 255 + 0.5) as a byte and GSR_OBS_F16 the
 * half nearest to x (ties to even).  `gain` is a linear exposure factor
 * (2^EV).  `out` has the layout of out_rgb with 1 (U8) or 2 (F16) bytes per
 * channel and is caller-owned device memory.  out_rgb may be NULL when an
 * observation is requested (only the observation and depth are written). */
typedef struct {
    int format;                   /* GSR_OBS_U8 or GSR_OBS_F16 */
    int reserved0;
    const float* gain;            /* device [C][E] or NULL (1) */
    const float* contrast;        /* device [C][E] or NULL (1) */
    const float* brightness;      /* device [C][E] or NULL (0) */
    void* out;                    /* device; u8 or half, [..][H_c][W_c][3] like out_rgb; 2-byte aligned for F16 */
} gsr_observation;

/* One render call: n_envs environments x n_cams camera slots. */
typedef struct {
    uint64_t scene_id;
    int n_envs;                   /* E >= 1 */
    int n_cams;                   /* C, 1..8 */
    const gsr_camera* cams;       /* host, [C] */
    const float* viewmats;        /* device, [C][E][3][4] world->camera */
    const float* body_poses;      /* device, [E][B][7] world-from-body; may be NULL when B = 0 */
    float bg[3];                  /* background colour */
    float* out_rgb;               /* device; slot c is a contiguous [E][H_c][W_c][3] block, slots in order */
    float* out_depth;             /* device; slot c is [E][H_c][W_c]; normalised expected depth, 0 where empty */
    float* out_alpha;             /* device, optional (NULL): 1 - final transmittance, same layout as depth */
    uint32_t* out_work;           /* device, optional (NULL): per pixel two counts, [..][H_c][W_c][2]: list entries
                                     visited up to and including the one that stopped the pixel (else the tile's
                                     list length), and Gaussians blended -- the algorithmic work of compositing */
    const gsr_observation* obs;   /* host, optional (NULL): fused observation epilogue */
} gsr_render_desc;

/* Materialised binning of one image (for parity checks). */
typedef struct {
    int64_t capacity;             /* in: entries available in keys / values */
    uint64_t* keys;               /* host, [capacity]: (global tile << 32) | float32 bits of depth */
    uint32_t* values;             /* host, [capacity]: Gaussian index g */
    uint32_t* ranges;             /* host, [tiles][2]: [start, end) of each tile of the image in keys/values; may be NULL */
    int64_t ranges_capacity;      /* in: tiles available in ranges */
    int64_t n_pairs;              /* out */
    int64_t n_visible;            /* out */
    int32_t tiles_x, tiles_y;     /* out */
    int64_t tile_base;            /* out: global tile id of the image's first tile */
    int32_t tile_size;            /* out: tile side the lists were built with (the tuned one) */
    int32_t reserved0;
} gsr_bins_out;

/* Per-Gaussian projection of one image (for parity checks).  Host arrays of
 * the scene's n entries. */
typedef struct {
    int64_t n;                    /* in: must equal the scene's Gaussian count */
    uint32_t* zkey;               /* [n] float32 bits of camera depth; 0xFFFFFFFF where culled */
    int32_t* rect;                /* [n][4] tile rectangle x0, x1, y0, y1 (half-open); unspecified where culled */
    float* rec;                   /* [n][12] u, v, a1, b1, c1, log2(o), z, r, R, G, B, 0 where
                                     log2(alpha) = log2(o) - (a1 dx + b1 dy)^2 - (c1 dy)^2; unspecified where culled */
} gsr_proj_out;

/* ---- context ---------------------------------------------------------
 * gsr_create: opens `device` (HIP ordinal), which must be a gfx950 GPU
 * (GSR_E_DEVICE otherwise).  `opt` may be NULL.  The library owns the context,
 * its scenes and working memory.  gsr_destroy waits for in-flight work and
 * frees everything the context owns; NULL is accepted. */
int gsr_create(int device, const gsr_options* opt, gsr_ctx** out);
int gsr_destroy(gsr_ctx* ctx);

/* gsr_trim: releases the device and pinned host memory of the context's
 * working sets that no call is using (buffers sized by earlier renders,
 * captured graphs, second-stream working sets), after their last work has
 * finished; scenes and tuning stay.  The next render allocates what it needs
 * again.  `freed_bytes` (may be NULL) receives the change of the device's
 * free memory over the call. */
int gsr_trim(gsr_ctx* ctx, int64_t* freed_bytes);

/* ---- scenes ----------------------------------------------------------
 * gsr_scene_create copies the caller's arrays into device memory in the
 * requested storage format and returns an id; the caller may free its arrays
 * when the call returns (it synchronises with the copy).  Validation: n >= 0,
 * sh_degree in 0..3, storage and mem_kind known, non-NULL arrays when n > 0,
 * body_offsets non-decreasing with off[B] = n.
 * gsr_scene_destroy frees a scene; GSR_E_BUSY if a render using it is still
 * in flight, GSR_E_NOT_FOUND for an unknown id. */
int gsr_scene_create(gsr_ctx* ctx, const gsr_scene_desc* desc, uint64_t* scene_id);
int gsr_scene_destroy(gsr_ctx* ctx, uint64_t scene_id);
/* Gaussians and bodies of a resident scene, and its resident size in bytes. */
int gsr_scene_info(gsr_ctx* ctx, uint64_t scene_id, int64_t* n, int* n_bodies, int64_t* bytes);

/* ---- rendering -------------------------------------------------------
 * gsr_render: renders every (camera slot, env) image of `desc` on `stream`
 * (a hipStream_t; NULL = default stream).  Images of all slots go through one
 * batched pipeline: RLGK posing + EWA projection + SH colour, a segmented
 * depth radix sort, stable tile binning, and one rasterisation launch per
 * memory chunk.  Inputs and outputs are caller-owned device memory and must
 * stay valid until the stream passes this call.  The first render of a job
 * shape on a working set blocks the host thread once per chunk until that
 * chunk's pair count is known, to size the tile-list buffers (with margin);
 * later renders of the same shape enqueue everything and return without
 * waiting for the device (see gsr_options.sync_lists).  A chunk whose lists
 * then outgrow the buffers is detected on the device: it writes no lists and
 * a fallback rasteriser composites it from the depth-ordered Gaussians (the
 * same images, slower), and the next render of the shape on the working set
 * that sees the overflow (once the earlier render has finished) plans the
 * buffers again.  With several
 * chunks, odd chunks run on an internal stream of the context (see
 * gsr_options.overlap) that waits for the caller's stream at the call's start
 * and is joined back into it before the call returns, so work the caller
 * queues on `stream` afterwards sees every image finished.
 * gsr_render_plain: same contract and results, one image at a time (one
 * launch chain per image, per-image sort): the reference per-environment path. */
int gsr_render(gsr_ctx* ctx, const gsr_render_desc* desc, void* stream);
int gsr_render_plain(gsr_ctx* ctx, const gsr_render_desc* desc, void* stream);

/* ---- rendering without device allocation ----------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 * gsr_render_noalloc renders like gsr_render (same kernels; every image
 * bit-identical to gsr_render's with the context's default launch parameters)
 * but calls no hipMalloc / hipFree and no allocating library routine: all of
 * its device working memory lies in one fixed scratch array of
 * GSR_NOALLOC_SCRATCH_BYTES per device, which the library holds on every
 * device it runs on until the process ends (its address is resolved by
 * gsr_create).  Images go through it in chunks that fit; the call blocks the
 * host once per chunk (as gsr_render does) and returns with the last chunk's
 * rasterisation in flight on `stream`.
 * Limits and errors: at most GSR_NOALLOC_MAX_IMAGES images per call, and one
 * image's working memory (about 84 bytes per Gaussian of the scene plus its
 * tile lists) must fit the scratch -- GSR_E_INVALID before any device work
 * when a call exceeds them, GSR_E_OVERFLOW when one image's tile lists turn
 * out larger than the scratch left for them (outputs of earlier images of the
 * call are then written, later ones are not).
 * Every call on a device shares that device's scratch, which keeps the last
 * call's contents (nothing in it is assumed zero).  Calls are serialised: a
 * call's work on `stream` waits for the previous call's work on any stream,
 * and host threads take turns. */
#define GSR_NOALLOC_SCRATCH_BYTES (256ll << 20)
#define GSR_NOALLOC_MAX_IMAGES 4096
int gsr_render_noalloc(gsr_ctx* ctx, const gsr_render_desc* desc, void* stream);

/* ---- batch LiDAR -----------------------------------------------------
 * Ray casting of the same resident Gaussians, posed with the same rigid-body
 * kinematics, for rotating and solid-state LiDARs (the paper's batch LiDAR
 * module, Sec. "User Interface and Ecosystem Design", and its LiDAR feature
 * table; dynamic objects and self-occlusion come from the posed scene).
 *
 * Sensor frame: x forward, y left, z up.  A LiDAR slot is a grid of rays,
 * H beams (rows) x W columns: ray (r, c) has azimuth az0 + (c + 0.5) az_step
 * and elevation elevations[r] (radians), direction
 * (cos el cos az, cos el sin az, sin el).  A rotating LiDAR spans a full
 * turn (W az_step = 2 pi); a solid-state one a sector.
 *
 * Non-repetitive scan patterns (pattern GSR_LIDAR_RAYS; the paper's
 * non-repetitive scan LiDAR, Table "tab:lidar"): the H x W rays of one scan
 * are listed one by one, ray k with azimuth ray_az[k] and elevation
 * ray_el[k] (any arrangement, e.g. the points of a rosette pattern at one
 * instant); results come back in the same order (out index k).  The library
 * sorts the rays into H elevation bands of W rays (azimuth order within a
 * band) and bins each Gaussian to the bands its cone crosses and, within
 * them, to the ray tiles whose azimuth span meets its azimuth window (the
 * hull over the tile rows), so the result is again that of casting every
 * ray against every Gaussian.
 *
 * Per ray and Gaussian (posed mean m, rotation R, scales S, opacity o in the
 * sensor frame), the Gaussian's response along the ray x(t) = t d peaks at
 * t* = argmin_t q(t), q(t) = |S^-1 R^T (t d - m)|^2; it contributes
 * alpha = min(0.99, o exp(-q(t*)/2)) at range t* if t* > near_range.
 * Contributions are composited front to back in the order of the Gaussians'
 * centre distances |m| (binary32 bits, ties by index) with the image model's
 * rules (skip alpha < 1/255, stop before adding when T(1 - alpha) < 1e-4):
 *     range = sum t* alpha T / (1 - T)  (0 where nothing was added),
 *     hit   = 1 - T  (the return probability).
 * Rays are binned into TS x TS tiles of the grid by conservative angular
 * bounds of each Gaussian's alpha >= 1/255 ellipsoid, so the result equals
 * casting every ray against every Gaussian.
 *
 * Heightmap scanner (pattern GSR_LIDAR_GRID; the paper's heightmap sensing
 * for locomotion, Table "tab:lidar"): an H x W grid of parallel rays cast
 * along -z of the sensor frame from its z = 0 plane, ray (r, c) starting at
 * (x0 + (c + 0.5) dx, y0 + (r + 0.5) dy, 0); t* and alpha as above with the
 * ray x(t) = origin + t (0, 0, -1), composited in the order of the
 * Gaussians' depths below the plane (max(0, -z) of the centre in binary32,
 * ties by index), so range = the expected depth of the surface below the
 * sensor plane (its height there is -range) and hit = 1 - T.  Rays are
 * binned by the sensor-plane footprint of each Gaussian's alpha >= 1/255
 * ellipsoid (a disc, widened by a relative 1e-4 against rounding). */
#define GSR_LIDAR_ANGULAR 0   /* rays from the sensor origin: beam elevations x azimuth columns */
#define GSR_LIDAR_GRID 1      /* heightmap: parallel rays along -z from a grid on the sensor's z = 0 plane */
#define GSR_LIDAR_RAYS 2      /* rays from the sensor origin, listed one by one (non-repetitive patterns) */
typedef struct {
    int width, height;            /* W columns, H beams (grid: W along x, H along y); 1..8192 each */
    float az0, az_step;           /* ANGULAR: radians; az_step > 0, W az_step <= 2 pi */
    const float* elevations;      /* ANGULAR: host [H], radians, strictly ascending, within (-pi/2, pi/2) */
    float near_range;             /* returns at t* <= near_range are ignored; > 0 */
    int attach_body;              /* -1: viewmats are world -> sensor; b: body-b -> sensor (as for cameras) */
    int pattern;                  /* GSR_LIDAR_ANGULAR (0), GSR_LIDAR_GRID (1) or GSR_LIDAR_RAYS (2) */
    float x0, y0, dx, dy;         /* GRID: metres in the sensor frame; dx, dy > 0 */
    const float* ray_az;          /* RAYS: host [H * W] azimuths, radians in [-pi, pi] */
    const float* ray_el;          /* RAYS: host [H * W] elevations, radians in (-pi/2, pi/2) */
} gsr_lidar;

typedef struct {
    uint64_t scene_id;
    int n_envs;                   /* E >= 1 */
    int n_lidars;                 /* L, 1..8 */
    const gsr_lidar* lidars;      /* host, [L] */
    const float* viewmats;        /* device, [L][E][3][4] world -> sensor (or body -> sensor when attached) */
    const float* body_poses;      /* device, [E][B][7]; may be NULL when B = 0 */
    float* out_range;             /* device; slot l is a contiguous [E][H_l][W_l] block, slots in order */
    float* out_hit;               /* device, optional (NULL): 1 - T, same layout */
} gsr_lidar_desc;

/* Asynchronous on `stream` like gsr_render (one host wait per memory chunk).
 * Inputs and outputs are caller-owned and must stay valid until the stream
 * passes this call.  GSR_E_INVALID on bad sizes, angles or null pointers,
 * before any device work. */
int gsr_render_lidar(gsr_ctx* ctx, const gsr_lidar_desc* desc, void* stream);

/* gsr_debug_bins: the sorted (tile, depth) keys, Gaussian ids and tile ranges
 * of image `image` (camera-slot-major index) of `desc`, as gsr_render builds
 * them: the same launch parameters (tuned for this scene and batch shape),
 * memory chunks, captured graphs and two streams, every chunk up to the one
 * holding the image stopping after its tile lists; the image's lists are read
 * from that chunk's buffers.  gsr_debug_project: the projection of image
 * `image` alone (one-image chunk, context defaults).  Both synchronous; output
 * pointers of `desc` are not used.  GSR_E_INVALID if out->capacity is smaller
 * than the number of pairs (n_pairs is still reported). */
int gsr_debug_bins(gsr_ctx* ctx, const gsr_render_desc* desc, int image, gsr_bins_out* out);
int gsr_debug_project(gsr_ctx* ctx, const gsr_render_desc* desc, int image, gsr_proj_out* out);

/* ---- serving ---------------------------------------------------------
 * A server renders requests from several producers (e.g. RL workers) as they
 * arrive, with continuous batching: worker threads, each with its own device
 * stream (default priority) and working memory, take the oldest pending
 * request and merge later pending requests of the same scene into one batched
 * launch (any resolutions, up to 8 image sizes and max_batch_images images);
 * requests that arrive while batches run join the next batch a worker forms,
 * and batches on different streams overlap on the device.  A batch is
 * rendered in memory chunks of at most min(memory_budget, the context's
 * chunk_bytes) of estimated working memory (at least one image each), so a
 * request occupies min(all its images, one chunk) while it runs.  A request is
 * admitted when that fits in memory_budget next to the requests in flight; it
 * waits in the queue otherwise.  Results are
 * identical to rendering the request alone: no per-image computation depends
 * on the batch. */
typedef struct {
    int n_streams;          /* concurrent batches (worker threads and streams), 1..8; 0 = 2 */
    int max_batch_images;   /* most images merged into one batch; 0 = 4096 */
    int64_t memory_budget;  /* bytes of working memory for admitted requests in flight; 0 = 32 GiB */
    int reserved[8];
} gsr_server_cfg;

typedef struct {
    int status;             /* GSR_OK or the error code of the request's batch */
    int n_images;           /* images of the request */
    int64_t batch_id;       /* batch the request was rendered in */
    int batch_requests;     /* requests merged into that batch */
    int batch_images;       /* images of that batch */
    int64_t t_submit_us;    /* steady-clock microseconds: submission, */
    int64_t t_admit_us;     /* admission into a batch, */
    int64_t t_start_us;     /* start of the batch's launches, */
    int64_t t_complete_us;  /* completion of the batch on the device */
} gsr_req_info;

typedef struct {
    int64_t submitted, completed, rejected, pending, batches, images;
    int64_t in_flight_bytes, in_flight_bytes_max;
    double latency_p50_us, latency_p99_us, latency_mean_us, latency_max_us;   /* completed requests */
    double mean_batch_requests;
} gsr_stats;

/* Starts the worker threads.  `cfg` may be NULL.  The context must outlive the
 * server. */
int gsr_server_create(gsr_ctx* ctx, const gsr_server_cfg* cfg, gsr_server** out);
/* Queues a render request; thread-safe, non-blocking.  The descriptor is
 * validated (as gsr_render) and copied, including its camera array; its device
 * buffers (viewmats, body_poses, outputs) must stay valid and untouched until
 * gsr_wait reports the request complete.  GSR_E_REJECTED if one image of the
 * request alone exceeds memory_budget (or the request has more images than
 * max_batch_images). */
int gsr_submit(gsr_server* srv, const gsr_render_desc* desc, uint64_t* ticket);
/* Waits for a request: timeout_us < 0 waits forever, 0 polls.  Returns the
 * request's status (GSR_E_TIMEOUT if it is not complete yet); once a completed
 * request has been reported its ticket is released (GSR_E_NOT_FOUND after). */
int gsr_wait(gsr_server* srv, uint64_t ticket, int64_t timeout_us, gsr_req_info* info);
/* Counters and latency percentiles (submission to completion) so far. */
int gsr_server_stats(gsr_server* srv, gsr_stats* stats);
/* Finishes every queued and running request, stops the workers, frees the
 * server.  NULL is accepted. */
int gsr_server_destroy(gsr_server* srv);

/* ---- autotuning --------------------------------------------------------
 * Launch parameters that change no pixel: tile side (8/16/32: pixels are
 * bit-identical across tile sizes because every tile's list is a filter of
 * one depth order and the radius is conservative), Gaussians staged in LDS
 * per raster round, images per projection thread, persistent raster
 * workgroups, images per memory chunk.  They are kept per shape class (scene,
 * env count, camera sizes); gsr_render of a tuned class uses them.  Sort keys
 * and tile lists reported by gsr_debug_bins use the tuned tile size (reported in
 * gsr_bins_out.tile_size). */
typedef struct {
    int tile_size;          /* 8, 16, 32 */
    int lds_batch;          /* 64/128/256 for 8x8 tiles, 64/128/256/512 otherwise */
    int images_per_thread;  /* 1..16 */
    int persistent;         /* 0 or 1 */
    int chunk_images;       /* 0 = from chunk_bytes, else images per memory chunk */
    float ms;               /* out: time of one render with these parameters (gsr_autotune) */
    int bin_schedule;       /* tile-row and tile lists: 0 by stable expansion (ranks from LDS lane masks),
                               1 by transposed ranks (one lane per bucket); identical lists */
    int reserved[3];
} gsr_tuning;

/* Times candidate parameters on `desc` (coordinate descent, each candidate one
 * warm-up and two timed renders into desc's outputs on `stream`), stores the
 * fastest for desc's shape class and returns it in `best`.  Synchronous. */
int gsr_autotune(gsr_ctx* ctx, const gsr_render_desc* desc, void* stream, gsr_tuning* best);
/* Parameters a render of desc's shape class uses now; sets them (validated). */
int gsr_tuning_get(gsr_ctx* ctx, const gsr_render_desc* desc, gsr_tuning* out);
int gsr_tuning_set(gsr_ctx* ctx, const gsr_render_desc* desc, const gsr_tuning* t);
/* Tuning cache as JSON lines (one shape class per line); load merges. */
int gsr_tuning_save(gsr_ctx* ctx, const char* path);
int gsr_tuning_load(gsr_ctx* ctx, const char* path);

/* Stage timers of a context created with profile = 1: device milliseconds
 * accumulated over the renders since the last reset, measured with HIP events
 * recorded on the stream each chunk runs on (with two-stream overlap the
 * stages of neighbouring chunks share the GPU, so a stage's time includes the
 * slowdown from the other stream and the stages can sum to more than the
 * wall time).  ms[0] compose + project, ms[1] depth sort,
 * ms[2] tile count, ms[3] tile scatter, ms[4] raster, ms[5] launches of the
 * raster kernel, ms[6] renders timed; if n >= 10 also the totals over the
 * timed renders of ms[7] visible Gaussians, ms[8] (tile, Gaussian) pairs,
 * ms[9] tile-row list entries.  `n` is the capacity of `ms` (>= 7).  Waits
 * for the timed work to finish.  reset = 1 clears the accumulators. */
int gsr_stage_times(gsr_ctx* ctx, double* ms, int n, int reset);

/* Description of the last error on this host thread ("" if none). */
const char* gsr_last_error(void);
/* Library version string. */
const char* gsr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
