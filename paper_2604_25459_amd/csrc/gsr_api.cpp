// C ABI and host runtime of libgsr: contexts, resident scenes, working-memory
// pools, chunk planning and the launch sequence of the batched renderer.
//
// Launch sequence per chunk of images (one stream, no host work between
// launches except one pair-count read-back):
//   compose (RLGK transforms) -> project (pose + EWA + SH + rect) ->
//   depth sort (4 x hist/scan/scatter) -> tile hist/scan + image scan ->
//   [host reads the chunk's pair total, grows the pair buffer if needed] ->
//   tile scatter -> raster (all images and camera slots of the chunk).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gsr.h"
#include "gsr_internal.h"

#define GSR_EXPORT extern "C" __attribute__((visibility("default")))

using gsr::ImageInfo;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? GSR_E_OOM : GSR_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_fail(_e, #expr); \
    } while (0)

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need)
    {
        if (need <= bytes && p) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
        }
        p = nullptr;
        bytes = 0;
        const size_t alloc = std::max<size_t>(need, 256);
        hipError_t e = hipMalloc(&p, alloc);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = alloc;
        return hipSuccess;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const
    {
        return static_cast<T*>(p);
    }
};

struct SceneRes {
    gsr::SceneDev dev{};
    DevBuf pos, rot, scale, sh, body_off;
    int64_t bytes = 0;
    hipEvent_t last_use = nullptr;
    bool used = false;
    ~SceneRes()
    {
        pos.release();
        rot.release();
        scale.release();
        sh.release();
        body_off.release();
        if (last_use) (void)hipEventDestroy(last_use);
    }
};

struct Workspace {
    DevBuf img, xform, keyz, rect, srect, rec, sk0, sk1, sv0, sv1, sort_hist, vis_count, tile_hist, tile_range,
        pair_count, pair_base, pairs, row_hist, row_range, row_count, row_base, rows, debug;
    uint64_t* h_total = nullptr;   // pinned: [0] pairs, [1] row entries of the current chunk
    ImageInfo* h_img = nullptr;    // pinned staging for image descriptions
    size_t h_img_cap = 0;
    hipEvent_t ev_total = nullptr, ev_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool used = false;
    ~Workspace()
    {
        for (DevBuf* b : {&img, &xform, &keyz, &rect, &srect, &rec, &sk0, &sk1, &sv0, &sv1, &sort_hist, &vis_count,
                          &tile_hist, &tile_range, &pair_count, &pair_base, &pairs, &row_hist, &row_range,
                          &row_count, &row_base, &rows, &debug})
            b->release();
        if (h_total) (void)hipHostFree(h_total);
        if (h_img) (void)hipHostFree(h_img);
        if (ev_total) (void)hipEventDestroy(ev_total);
        if (ev_done) (void)hipEventDestroy(ev_done);
    }
};

}  // namespace

// HIP events bracketing the pipeline stages of one chunk (profile option).
struct StageEvents {
    hipEvent_t e[6] = {};
};

struct gsr_ctx {
    int device = 0;
    gsr_options opt{};
    std::mutex mu;
    std::vector<StageEvents> pending;   // recorded, not yet read
    double stage_ms[5] = {0, 0, 0, 0, 0};
    double raster_launches = 0, renders = 0;
    std::map<uint64_t, std::unique_ptr<SceneRes>> scenes;
    uint64_t next_id = 1;
    std::vector<std::unique_ptr<Workspace>> pool;
    bool poisoned = false;
};

namespace {

constexpr int kMaxCams = 8;

int validate_options(const gsr_options& o)
{
    if (o.tile_size != 8 && o.tile_size != 16 && o.tile_size != 32)
        return fail(GSR_E_INVALID, "tile_size must be 8, 16 or 32");
    if (o.images_per_thread < 1 || o.images_per_thread > 16)
        return fail(GSR_E_INVALID, "images_per_thread must be in 1..16");
    if (o.chunk_bytes < (int64_t)(64 << 20)) return fail(GSR_E_INVALID, "chunk_bytes must be >= 64 MiB");
    if (!(o.cutoff >= 1.0f && o.cutoff <= 8.0f)) return fail(GSR_E_INVALID, "cutoff must be in [1, 8]");
    return GSR_OK;
}

gsr_options fill_defaults(const gsr_options* in)
{
    gsr_options o{};
    if (in) o = *in;
    if (o.tile_size == 0) o.tile_size = 16;
    if (o.images_per_thread == 0) o.images_per_thread = 4;
    if (o.chunk_bytes == 0) o.chunk_bytes = (int64_t)24 << 30;
    if (o.cutoff == 0.0f) o.cutoff = 3.33f;
    return o;
}

int validate_render(gsr_ctx* ctx, const gsr_render_desc* d, bool need_outputs, SceneRes** out_scene)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d) return fail(GSR_E_INVALID, "render desc is NULL");
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    auto it = ctx->scenes.find(d->scene_id);
    if (it == ctx->scenes.end()) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    SceneRes* sc = it->second.get();
    if (d->n_envs < 1) return fail(GSR_E_INVALID, "n_envs must be >= 1");
    if (d->n_cams < 1 || d->n_cams > kMaxCams) return fail(GSR_E_INVALID, "n_cams must be in 1..8");
    if (!d->cams) return fail(GSR_E_INVALID, "cams is NULL");
    if (!d->viewmats) return fail(GSR_E_INVALID, "viewmats is NULL");
    if (sc->dev.n_bodies > 0 && !d->body_poses) return fail(GSR_E_INVALID, "body_poses is NULL but the scene has bodies");
    if (((uintptr_t)d->viewmats & 3) || ((uintptr_t)d->body_poses & 3))
        return fail(GSR_E_INVALID, "viewmats / body_poses must be 4-byte aligned");
    const int ts = ctx->opt.tile_size;
    for (int c = 0; c < d->n_cams; ++c) {
        const gsr_camera& cam = d->cams[c];
        if (cam.width < 1 || cam.height < 1 || cam.width > 8192 || cam.height > 8192)
            return fail(GSR_E_INVALID, "camera size must be in 1..8192");
        if (!(cam.fx > 0.0f) || !(cam.fy > 0.0f)) return fail(GSR_E_INVALID, "focal lengths must be > 0");
        if (!(cam.near_plane > 0.0f)) return fail(GSR_E_INVALID, "near_plane must be > 0");
        const int64_t tiles = (int64_t)((cam.width + ts - 1) / ts) * ((cam.height + ts - 1) / ts);
        if (tiles > 15000) return fail(GSR_E_INVALID, "more than 15000 tiles per image for this tile size");
    }
    if (need_outputs) {
        if (!d->out_rgb || !d->out_depth) return fail(GSR_E_INVALID, "out_rgb / out_depth is NULL");
        if (((uintptr_t)d->out_rgb & 3) || ((uintptr_t)d->out_depth & 3) || ((uintptr_t)d->out_alpha & 3))
            return fail(GSR_E_INVALID, "outputs must be 4-byte aligned");
    }
    *out_scene = sc;
    return GSR_OK;
}

// Image descriptions of the whole batch, camera-slot-major.
std::vector<ImageInfo> plan_images(const gsr_render_desc* d, int ts)
{
    const int E = d->n_envs;
    std::vector<ImageInfo> v((size_t)E * d->n_cams);
    uint64_t tile_base = 0, pixel_base = 0;
    for (int c = 0; c < d->n_cams; ++c) {
        const gsr_camera& cam = d->cams[c];
        const int tx = (cam.width + ts - 1) / ts, ty = (cam.height + ts - 1) / ts;
        for (int e = 0; e < E; ++e) {
            ImageInfo& im = v[(size_t)c * E + e];
            std::memset(&im, 0, sizeof im);
            im.width = cam.width;
            im.height = cam.height;
            im.tiles_x = tx;
            im.tiles_y = ty;
            im.fx = cam.fx;
            im.fy = cam.fy;
            im.cx = cam.cx;
            im.cy = cam.cy;
            im.near_plane = cam.near_plane;
            im.cam = c;
            im.env = e;
            im.key_tile_base = (uint32_t)tile_base;
            im.out_pixel = pixel_base;
            tile_base += (uint64_t)tx * ty;
            pixel_base += (uint64_t)cam.width * cam.height;
        }
    }
    return v;
}

struct ChunkPlan {
    int chunk;          // images per chunk
    int t_max;          // max tiles of any image
    int tx_max, ty_max; // max tile columns / rows of any image
    int sort_blocks, tile_blocks;
};

size_t per_image_bytes(const SceneRes* sc, int t_max, int sort_blocks, int tile_blocks)
{
    const size_t n = (size_t)sc->dev.n;
    size_t b = n * (4 + 16 + 48 + 16);                                 // keyz, rect + sorted rect, records, sort buffers
    b += (size_t)(sc->dev.n_bodies + 1) * 64;                          // transforms
    b += (size_t)sort_blocks * 256 * 4 + (size_t)tile_blocks * t_max * 4 + (size_t)t_max * 8 + 32;
    b += n * 8 * 4 + n * 3 * 8;                                        // pair / row-entry estimates
    return b;
}

ChunkPlan plan_chunks(const gsr_ctx* ctx, const SceneRes* sc, const std::vector<ImageInfo>& imgs, bool plain)
{
    ChunkPlan p{};
    p.t_max = 1;
    p.tx_max = 1;
    p.ty_max = 1;
    for (const ImageInfo& im : imgs) {
        p.t_max = std::max(p.t_max, im.tiles_x * im.tiles_y);
        p.tx_max = std::max(p.tx_max, im.tiles_x);
        p.ty_max = std::max(p.ty_max, im.tiles_y);
    }
    const int64_t n = sc->dev.n;
    p.sort_blocks = (int)std::max<int64_t>(1, (n + gsr::kSortItems - 1) / gsr::kSortItems);
    p.tile_blocks = (int)std::max<int64_t>(1, (n + gsr::kTileGauss - 1) / gsr::kTileGauss);
    if (plain) {
        p.chunk = 1;
    } else {
        const size_t per = per_image_bytes(sc, p.t_max, p.sort_blocks, p.tile_blocks);
        const size_t c = std::max<size_t>(1, (size_t)ctx->opt.chunk_bytes / std::max<size_t>(per, 1));
        p.chunk = (int)std::min<size_t>(c, imgs.size());
    }
    return p;
}

hipError_t ensure_workspace(Workspace& ws, const SceneRes* sc, const ChunkPlan& p, size_t n_images_total)
{
    const size_t n = (size_t)std::max<int64_t>(sc->dev.n, 1);
    const size_t I = (size_t)p.chunk;
    hipError_t e;
#define ENS(buf, bytes) \
    if ((e = ws.buf.ensure(bytes)) != hipSuccess) return e
    ENS(img, n_images_total * sizeof(ImageInfo));
    ENS(xform, I * (sc->dev.n_bodies + 1) * 64);
    ENS(keyz, I * n * 4);
    ENS(rect, I * n * 8);
    ENS(srect, I * n * 8);
    ENS(rec, I * n * 48);
    ENS(sk0, I * n * 4);
    ENS(sk1, I * n * 4);
    ENS(sv0, I * n * 4);
    ENS(sv1, I * n * 4);
    ENS(sort_hist, I * p.sort_blocks * 256 * 4);
    ENS(vis_count, I * 4);
    ENS(tile_hist, I * p.tile_blocks * (size_t)p.t_max * 4);
    ENS(tile_range, I * (size_t)p.t_max * 8);
    ENS(pair_count, I * 4);
    ENS(pair_base, (I + 1) * 8);
    ENS(row_hist, I * p.tile_blocks * (size_t)p.ty_max * 4);
    ENS(row_range, I * (size_t)p.ty_max * 8);
    ENS(row_count, I * 4);
    ENS(row_base, (I + 1) * 8);
#undef ENS
    if (!ws.h_total) {
        if ((e = hipHostMalloc((void**)&ws.h_total, 64, hipHostMallocDefault)) != hipSuccess) return e;
    }
    if (ws.h_img_cap < n_images_total) {
        if (ws.h_img) (void)hipHostFree(ws.h_img);
        ws.h_img = nullptr;
        ws.h_img_cap = 0;
        if ((e = hipHostMalloc((void**)&ws.h_img, n_images_total * sizeof(ImageInfo), hipHostMallocDefault)) !=
            hipSuccess)
            return e;
        ws.h_img_cap = n_images_total;
    }
    if (!ws.ev_total) {
        if ((e = hipEventCreateWithFlags(&ws.ev_total, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&ws.ev_done, hipEventDisableTiming)) != hipSuccess) return e;
    }
    return hipSuccess;
}

Workspace* acquire_workspace(gsr_ctx* ctx, hipStream_t stream)
{
    for (auto& w : ctx->pool) {
        if (!w->used || w->last_stream == stream) return w.get();
    }
    for (auto& w : ctx->pool) {
        if (hipEventQuery(w->ev_done) == hipSuccess) return w.get();
    }
    ctx->pool.emplace_back(new Workspace());
    return ctx->pool.back().get();
}

gsr::ChunkDev chunk_view(Workspace& ws, const SceneRes* sc, const ChunkPlan& p, int i0, int n_img,
                         const std::vector<ImageInfo>& imgs)
{
    gsr::ChunkDev c{};
    c.n = (uint64_t)sc->dev.n;
    c.n_img = n_img;
    int t_max = 1, tx_max = 1, ty_max = 1;
    for (int k = 0; k < n_img; ++k) {
        t_max = std::max(t_max, imgs[i0 + k].tiles_x * imgs[i0 + k].tiles_y);
        tx_max = std::max(tx_max, imgs[i0 + k].tiles_x);
        ty_max = std::max(ty_max, imgs[i0 + k].tiles_y);
    }
    c.t_max = t_max;
    c.tx_max = tx_max;
    c.ty_max = ty_max;
    c.sort_blocks = p.sort_blocks;
    c.tile_blocks = p.tile_blocks;
    c.img = ws.img.as<ImageInfo>() + i0;
    c.xform = ws.xform.as<float>();
    c.keyz = ws.keyz.as<uint32_t>();
    c.rect = ws.rect.as<uint2>();
    c.srect = ws.srect.as<uint2>();
    c.rec = ws.rec.as<float4>();
    c.sk[0] = ws.sk0.as<uint32_t>();
    c.sk[1] = ws.sk1.as<uint32_t>();
    c.sv[0] = ws.sv0.as<uint32_t>();
    c.sv[1] = ws.sv1.as<uint32_t>();
    c.sort_hist = ws.sort_hist.as<uint32_t>();
    c.vis_count = ws.vis_count.as<uint32_t>();
    c.tile_hist = ws.tile_hist.as<uint32_t>();
    c.tile_range = ws.tile_range.as<uint32_t>();
    c.pair_count = ws.pair_count.as<uint32_t>();
    c.pair_base = ws.pair_base.as<uint64_t>();
    c.pairs = ws.pairs.as<uint32_t>();
    c.row_hist = ws.row_hist.as<uint32_t>();
    c.row_range = ws.row_range.as<uint32_t>();
    c.row_count = ws.row_count.as<uint32_t>();
    c.row_base = ws.row_base.as<uint64_t>();
    c.rows = ws.rows.as<uint2>();
    return c;
}

enum class Mode { kRender, kBins, kProject };

// Enqueue the pipeline of images [i0, i0 + n_img).  Returns GSR_OK or an error
// code; `pairs_total` receives the chunk's pair count (modes kRender, kBins).
int run_chunk(gsr_ctx* ctx, Workspace& ws, SceneRes* sc, const gsr_render_desc* d, const ChunkPlan& plan,
              const std::vector<ImageInfo>& imgs, int i0, int n_img, int ipt, hipStream_t st, Mode mode,
              uint64_t* pairs_total)
{
    gsr::ChunkDev c = chunk_view(ws, sc, plan, i0, n_img, imgs);
    const gsr::SceneDev& s = sc->dev;
    const bool prof = ctx->opt.profile && mode == Mode::kRender;
    StageEvents ev;
    if (prof) {
        for (hipEvent_t& e : ev.e) HIP_TRY(hipEventCreate(&e));
        HIP_TRY(hipEventRecord(ev.e[0], st));
    }
    HIP_TRY(gsr::launch_compose(s, c, d->viewmats, d->body_poses, d->n_envs, st));
    HIP_TRY(gsr::launch_project(s, c, ctx->opt.tile_size, ctx->opt.cutoff, ipt, st));
    if (mode == Mode::kProject) return GSR_OK;
    if (prof) HIP_TRY(hipEventRecord(ev.e[1], st));
    HIP_TRY(gsr::launch_depth_sort(s, c, st));
    if (prof) HIP_TRY(hipEventRecord(ev.e[2], st));
    HIP_TRY(gsr::launch_tile_count(s, c, st));
    if (prof) HIP_TRY(hipEventRecord(ev.e[3], st));
    HIP_TRY(hipMemcpyAsync(ws.h_total, c.pair_base + n_img, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(ws.h_total + 1, c.row_base + n_img, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(ws.ev_total, st));
    HIP_TRY(hipEventSynchronize(ws.ev_total));
    const uint64_t total = ws.h_total[0];
    const uint64_t row_total = ws.h_total[1];
    *pairs_total = total;
    // everything enqueued before ev_total has completed, including earlier chunks: growing is safe
    if (ws.pairs.bytes < total * 4) {
        const size_t want = std::max<size_t>(total * 4, (size_t)((double)ws.pairs.bytes * 1.5));
        HIP_TRY(ws.pairs.ensure(std::max<size_t>(want + (total * 4) / 8, 1 << 20)));
        c.pairs = ws.pairs.as<uint32_t>();
    }
    if (ws.rows.bytes < row_total * 8) {
        const size_t want = std::max<size_t>(row_total * 8, (size_t)((double)ws.rows.bytes * 1.5));
        HIP_TRY(ws.rows.ensure(std::max<size_t>(want + (row_total * 8) / 8, 1 << 20)));
        c.rows = ws.rows.as<uint2>();
    }
    HIP_TRY(gsr::launch_tile_scatter(s, c, st));
    if (mode == Mode::kBins) return GSR_OK;
    if (prof) HIP_TRY(hipEventRecord(ev.e[4], st));

    gsr::RasterParams rp{};
    rp.ts = ctx->opt.tile_size;
    rp.bg[0] = d->bg[0];
    rp.bg[1] = d->bg[1];
    rp.bg[2] = d->bg[2];
    rp.out_rgb = d->out_rgb;
    rp.out_depth = d->out_depth;
    rp.out_alpha = d->out_alpha;
    uint32_t blocks = 0;
    for (int k = 0; k < n_img;) {
        const int cam = imgs[i0 + k].cam;
        int m = k;
        while (m < n_img && imgs[i0 + m].cam == cam) ++m;
        if (rp.n_segs >= gsr::kMaxSegs) return fail(GSR_E_INVALID, "too many camera slots in one chunk");
        gsr::RasterSeg& sg = rp.segs[rp.n_segs++];
        sg.first_tile = blocks;
        sg.first_image = (uint32_t)k;
        sg.n_images = (uint32_t)(m - k);
        sg.tiles_per_image = (uint32_t)(imgs[i0 + k].tiles_x * imgs[i0 + k].tiles_y);
        blocks += sg.n_images * sg.tiles_per_image;
        k = m;
    }
    rp.n_blocks = blocks;
    HIP_TRY(gsr::launch_raster(s, c, rp, st));
    if (prof) {
        HIP_TRY(hipEventRecord(ev.e[5], st));
        ctx->pending.push_back(ev);
    }
    return GSR_OK;
}

int render_impl(gsr_ctx* ctx, const gsr_render_desc* d, void* stream, bool plain)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SceneRes* sc = nullptr;
    int rc = validate_render(ctx, d, true, &sc);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const std::vector<ImageInfo> imgs = plan_images(d, ctx->opt.tile_size);
    const ChunkPlan plan = plan_chunks(ctx, sc, imgs, plain);
    Workspace* ws = acquire_workspace(ctx, st);
    if (ws->used && ws->last_stream != st) HIP_TRY(hipEventSynchronize(ws->ev_done));
    HIP_TRY(ensure_workspace(*ws, sc, plan, imgs.size()));
    // the previous use of this workspace on this stream must have consumed its staging
    if (ws->used) HIP_TRY(hipEventSynchronize(ws->ev_done));
    std::memcpy(ws->h_img, imgs.data(), imgs.size() * sizeof(ImageInfo));
    HIP_TRY(hipMemcpyAsync(ws->img.p, ws->h_img, imgs.size() * sizeof(ImageInfo), hipMemcpyHostToDevice, st));
    const int ipt = plain ? 1 : ctx->opt.images_per_thread;
    for (int i0 = 0; i0 < (int)imgs.size(); i0 += plan.chunk) {
        const int n_img = std::min<int>(plan.chunk, (int)imgs.size() - i0);
        uint64_t total = 0;
        rc = run_chunk(ctx, *ws, sc, d, plan, imgs, i0, n_img, ipt, st, Mode::kRender, &total);
        if (rc) {
            if (rc == GSR_E_DEVICE) ctx->poisoned = true;
            return rc;
        }
    }
    HIP_TRY(hipEventRecord(ws->ev_done, st));
    ws->used = true;
    ws->last_stream = st;
    if (!sc->last_use) HIP_TRY(hipEventCreateWithFlags(&sc->last_use, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(sc->last_use, st));
    sc->used = true;
    ctx->renders += 1;
    return GSR_OK;
}

}  // namespace

// ============================================================== exported API

GSR_EXPORT const char* gsr_last_error(void) { return g_err.c_str(); }

GSR_EXPORT const char* gsr_version(void) { return "gsr 0.1 (gfx950)"; }

GSR_EXPORT int gsr_create(int device, const gsr_options* opt, gsr_ctx** out)
{
    if (!out) return fail(GSR_E_INVALID, "out is NULL");
    *out = nullptr;
    gsr_options o = fill_defaults(opt);
    int rc = validate_options(o);
    if (rc) return rc;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(GSR_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(GSR_E_DEVICE, "device ordinal out of range");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GSR_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", libgsr is built for gfx950");
    HIP_TRY(hipSetDevice(device));
    gsr_ctx* ctx = new (std::nothrow) gsr_ctx();
    if (!ctx) return fail(GSR_E_OOM, "context allocation failed");
    ctx->device = device;
    ctx->opt = o;
    *out = ctx;
    return GSR_OK;
}

GSR_EXPORT int gsr_destroy(gsr_ctx* ctx)
{
    if (!ctx) return GSR_OK;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        for (StageEvents& ev : ctx->pending)
            for (hipEvent_t e : ev.e) (void)hipEventDestroy(e);
        ctx->pending.clear();
        ctx->pool.clear();
        ctx->scenes.clear();
    }
    delete ctx;
    return GSR_OK;
}

GSR_EXPORT int gsr_scene_create(gsr_ctx* ctx, const gsr_scene_desc* d, uint64_t* scene_id)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d || !scene_id) return fail(GSR_E_INVALID, "desc / scene_id is NULL");
    if (d->n < 0 || d->n > ((int64_t)1 << 31) - 64) return fail(GSR_E_INVALID, "n must be in [0, 2^31 - 64)");
    if (d->sh_degree < 0 || d->sh_degree > gsr::kMaxShDegree) return fail(GSR_E_INVALID, "sh_degree must be 0..3");
    if (d->storage < GSR_STORAGE_F32 || d->storage > GSR_STORAGE_BF16) return fail(GSR_E_INVALID, "unknown storage");
    if (d->mem_kind != GSR_MEM_HOST && d->mem_kind != GSR_MEM_DEVICE) return fail(GSR_E_INVALID, "unknown mem_kind");
    if (d->n_bodies < 0 || d->n_bodies > 4096) return fail(GSR_E_INVALID, "n_bodies must be in 0..4096");
    if (d->n > 0 && (!d->means || !d->scales || !d->quats || !d->opacities || !d->sh))
        return fail(GSR_E_INVALID, "attribute array is NULL");
    if (!d->body_offsets) return fail(GSR_E_INVALID, "body_offsets is NULL");
    for (int b = 0; b <= d->n_bodies; ++b) {
        if (d->body_offsets[b] < 0 || d->body_offsets[b] > d->n) return fail(GSR_E_INVALID, "body_offsets out of range");
        if (b > 0 && d->body_offsets[b] < d->body_offsets[b - 1])
            return fail(GSR_E_INVALID, "body_offsets must be non-decreasing");
    }
    if (d->body_offsets[d->n_bodies] != d->n) return fail(GSR_E_INVALID, "body_offsets[n_bodies] must equal n");

    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<SceneRes> sc(new SceneRes());
    const int64_t n = d->n;
    const int64_t n_pad = std::max<int64_t>(64, (n + 63) / 64 * 64);
    const int K = (d->sh_degree + 1) * (d->sh_degree + 1);
    const bool half = d->storage != GSR_STORAGE_F32;
    const int chunks = half ? (3 * K + 7) / 8 : (3 * K + 3) / 4;
    HIP_TRY(sc->pos.ensure((size_t)n_pad * 16));
    HIP_TRY(sc->rot.ensure((size_t)n_pad * 16));
    if (!half) HIP_TRY(sc->scale.ensure((size_t)n_pad * 16));
    HIP_TRY(sc->sh.ensure((size_t)chunks * n_pad * 16));
    std::vector<int> off(d->n_bodies + 1);
    for (int b = 0; b <= d->n_bodies; ++b) off[b] = (int)d->body_offsets[b];
    HIP_TRY(sc->body_off.ensure(off.size() * sizeof(int)));
    HIP_TRY(hipMemcpy(sc->body_off.p, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    if (n > 0) {
        const float *m = d->means, *s = d->scales, *q = d->quats, *o = d->opacities, *f = d->sh;
        DevBuf tmp;
        if (d->mem_kind == GSR_MEM_HOST) {
            const size_t b_m = n * 12, b_s = n * 12, b_q = n * 16, b_o = n * 4, b_f = (size_t)n * K * 12;
            HIP_TRY(tmp.ensure(b_m + b_s + b_q + b_o + b_f));
            char* base = tmp.as<char>();
            HIP_TRY(hipMemcpy(base, d->means, b_m, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(base + b_m, d->scales, b_s, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(base + b_m + b_s, d->quats, b_q, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(base + b_m + b_s + b_q, d->opacities, b_o, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(base + b_m + b_s + b_q + b_o, d->sh, b_f, hipMemcpyHostToDevice));
            m = (const float*)base;
            s = (const float*)(base + b_m);
            q = (const float*)(base + b_m + b_s);
            o = (const float*)(base + b_m + b_s + b_q);
            f = (const float*)(base + b_m + b_s + b_q + b_o);
        }
        HIP_TRY(gsr::launch_scene_convert(d->storage, n, n_pad, d->sh_degree, m, s, q, o, f, sc->pos.as<float4>(),
                                          sc->rot.p, sc->scale.as<float4>(), sc->sh.p, nullptr));
        HIP_TRY(hipDeviceSynchronize());
        tmp.release();
    }
    gsr::SceneDev& dv = sc->dev;
    dv.n = n;
    dv.n_pad = n_pad;
    dv.degree = d->sh_degree;
    dv.storage = d->storage;
    dv.n_bodies = d->n_bodies;
    dv.sh_chunks = chunks;
    dv.pos = sc->pos.as<float4>();
    dv.rot = sc->rot.p;
    dv.scale = sc->scale.as<float4>();
    dv.sh = sc->sh.p;
    dv.body_off = sc->body_off.as<int>();
    sc->bytes = (int64_t)(sc->pos.bytes + sc->rot.bytes + sc->scale.bytes + sc->sh.bytes + sc->body_off.bytes);
    const uint64_t id = ctx->next_id++;
    ctx->scenes[id] = std::move(sc);
    *scene_id = id;
    return GSR_OK;
}

GSR_EXPORT int gsr_scene_destroy(gsr_ctx* ctx, uint64_t scene_id)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    SceneRes* sc = it->second.get();
    if (sc->used && sc->last_use && hipEventQuery(sc->last_use) == hipErrorNotReady)
        return fail(GSR_E_BUSY, "scene is used by in-flight work");
    ctx->scenes.erase(it);
    return GSR_OK;
}

GSR_EXPORT int gsr_scene_info(gsr_ctx* ctx, uint64_t scene_id, int64_t* n, int* n_bodies, int64_t* bytes)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->scenes.find(scene_id);
    if (it == ctx->scenes.end()) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    if (n) *n = it->second->dev.n;
    if (n_bodies) *n_bodies = it->second->dev.n_bodies;
    if (bytes) *bytes = it->second->bytes;
    return GSR_OK;
}

GSR_EXPORT int gsr_stage_times(gsr_ctx* ctx, double* ms, int n, int reset)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!ms || n < 7) return fail(GSR_E_INVALID, "ms must hold at least 7 values");
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    for (StageEvents& ev : ctx->pending) {
        HIP_TRY(hipEventSynchronize(ev.e[5]));
        for (int k = 0; k < 5; ++k) {
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, ev.e[k], ev.e[k + 1]));
            ctx->stage_ms[k] += t;
        }
        ctx->raster_launches += 1;
        for (hipEvent_t e : ev.e) (void)hipEventDestroy(e);
    }
    ctx->pending.clear();
    for (int k = 0; k < 5; ++k) ms[k] = ctx->stage_ms[k];
    ms[5] = ctx->raster_launches;
    ms[6] = ctx->renders;
    if (reset) {
        for (double& v : ctx->stage_ms) v = 0.0;
        ctx->raster_launches = 0;
        ctx->renders = 0;
    }
    return GSR_OK;
}

GSR_EXPORT int gsr_render(gsr_ctx* ctx, const gsr_render_desc* desc, void* stream)
{
    return render_impl(ctx, desc, stream, false);
}

GSR_EXPORT int gsr_render_plain(gsr_ctx* ctx, const gsr_render_desc* desc, void* stream)
{
    return render_impl(ctx, desc, stream, true);
}

namespace {

int debug_prepare(gsr_ctx* ctx, const gsr_render_desc* d, int image, SceneRes** sc, Workspace** ws,
                  std::vector<ImageInfo>* imgs, ChunkPlan* plan)
{
    int rc = validate_render(ctx, d, false, sc);
    if (rc) return rc;
    if (image < 0 || image >= d->n_envs * d->n_cams) return fail(GSR_E_INVALID, "image index out of range");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    *imgs = plan_images(d, ctx->opt.tile_size);
    *plan = plan_chunks(ctx, *sc, *imgs, true);
    *ws = acquire_workspace(ctx, nullptr);
    HIP_TRY(ensure_workspace(**ws, *sc, *plan, imgs->size()));
    std::memcpy((*ws)->h_img, imgs->data(), imgs->size() * sizeof(ImageInfo));
    HIP_TRY(hipMemcpy((*ws)->img.p, (*ws)->h_img, imgs->size() * sizeof(ImageInfo), hipMemcpyHostToDevice));
    return GSR_OK;
}

}  // namespace

GSR_EXPORT int gsr_debug_bins(gsr_ctx* ctx, const gsr_render_desc* d, int image, gsr_bins_out* out)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!out) return fail(GSR_E_INVALID, "out is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SceneRes* sc;
    Workspace* ws;
    std::vector<ImageInfo> imgs;
    ChunkPlan plan;
    int rc = debug_prepare(ctx, d, image, &sc, &ws, &imgs, &plan);
    if (rc) return rc;
    uint64_t total = 0;
    rc = run_chunk(ctx, *ws, sc, d, plan, imgs, image, 1, 1, nullptr, Mode::kBins, &total);
    if (rc) return rc;
    const ImageInfo& im = imgs[image];
    const int T = im.tiles_x * im.tiles_y;
    uint32_t vis = 0;
    if (sc->dev.n > 0) HIP_TRY(hipMemcpy(&vis, ws->vis_count.p, 4, hipMemcpyDeviceToHost));
    out->n_pairs = (int64_t)total;
    out->n_visible = vis;
    out->tiles_x = im.tiles_x;
    out->tiles_y = im.tiles_y;
    out->tile_base = im.key_tile_base;
    if (out->ranges) {
        if (out->ranges_capacity < T) return fail(GSR_E_INVALID, "ranges_capacity smaller than the tile count");
        HIP_TRY(hipMemcpy(out->ranges, ws->tile_range.p, (size_t)T * 8, hipMemcpyDeviceToHost));
    }
    if ((int64_t)total > out->capacity) return fail(GSR_E_INVALID, "capacity smaller than the number of pairs");
    if (total > 0) {
        gsr::ChunkDev c = chunk_view(*ws, sc, plan, image, 1, imgs);
        HIP_TRY(ws->debug.ensure(total * 8));
        HIP_TRY(gsr::launch_debug_keys(c, 0, (uint64_t)sc->dev.n, c.pairs, total, ws->debug.as<uint64_t>(), nullptr));
        HIP_TRY(hipDeviceSynchronize());
        if (out->keys) HIP_TRY(hipMemcpy(out->keys, ws->debug.p, total * 8, hipMemcpyDeviceToHost));
        if (out->values) HIP_TRY(hipMemcpy(out->values, ws->pairs.p, total * 4, hipMemcpyDeviceToHost));
    }
    ws->used = false;
    return GSR_OK;
}

GSR_EXPORT int gsr_debug_project(gsr_ctx* ctx, const gsr_render_desc* d, int image, gsr_proj_out* out)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!out) return fail(GSR_E_INVALID, "out is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    SceneRes* sc;
    Workspace* ws;
    std::vector<ImageInfo> imgs;
    ChunkPlan plan;
    int rc = debug_prepare(ctx, d, image, &sc, &ws, &imgs, &plan);
    if (rc) return rc;
    const int64_t n = sc->dev.n;
    if (out->n != n) return fail(GSR_E_INVALID, "out->n must equal the scene's Gaussian count");
    if (n == 0) return GSR_OK;
    uint64_t total = 0;
    rc = run_chunk(ctx, *ws, sc, d, plan, imgs, image, 1, 1, nullptr, Mode::kProject, &total);
    if (rc) return rc;
    HIP_TRY(hipDeviceSynchronize());
    if (out->zkey) HIP_TRY(hipMemcpy(out->zkey, ws->keyz.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (out->rect) {
        std::vector<uint32_t> r((size_t)n * 2);
        HIP_TRY(hipMemcpy(r.data(), ws->rect.p, (size_t)n * 8, hipMemcpyDeviceToHost));
        for (int64_t g = 0; g < n; ++g) {
            out->rect[4 * g + 0] = (int32_t)(r[2 * g] & 0xFFFF);
            out->rect[4 * g + 1] = (int32_t)(r[2 * g] >> 16);
            out->rect[4 * g + 2] = (int32_t)(r[2 * g + 1] & 0xFFFF);
            out->rect[4 * g + 3] = (int32_t)(r[2 * g + 1] >> 16);
        }
    }
    if (out->rec) HIP_TRY(hipMemcpy(out->rec, ws->rec.p, (size_t)n * 48, hipMemcpyDeviceToHost));
    ws->used = false;
    return GSR_OK;
}
