// C ABI and host runtime of libgsr: contexts, resident scenes, working-memory
// pools, chunk planning and the launch sequence of the batched renderer.
//
// Launch sequence per chunk of images (one stream, no host work between
// launches except one read-back of the chunk's totals):
//   compose (RLGK transforms) -> project (pose + EWA + SH + rect) ->
//   depth sort (4 x hist/scan/scatter) -> tile/row counts + image scan ->
//   [host reads the chunk's pair and row-entry totals, grows buffers] ->
//   two-level tile scatter -> raster (all images of the chunk, any sizes).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <sstream>

#include "gsr_runtime.h"

#define GSR_EXPORT extern "C" __attribute__((visibility("default")))

namespace gsr {

namespace {
thread_local std::string g_err;
constexpr int kMaxCams = 8;
}  // namespace

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? GSR_E_OOM : GSR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

hipError_t DevBuf::ensure(size_t need)
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

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

SceneRes::~SceneRes()
{
    pos.release();
    rot.release();
    scale.release();
    sh.release();
    body_off.release();
    if (last_use) (void)hipEventDestroy(last_use);
}

void Workspace::drop_graphs_of(uint64_t uid)
{
    for (auto it = graphs.begin(); it != graphs.end();) {
        if (it->second.scene_uid == uid) {
            if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
            it = graphs.erase(it);
        } else {
            ++it;
        }
    }
    if (twin) twin->drop_graphs_of(uid);
}

Workspace::~Workspace()
{
    // a fixed workspace's buffers point into memory it does not own
    if (!fixed)
        for (DevBuf* b : {&img, &xform, &keyz, &rect, &srect, &rec, &sk0, &sk1, &sv0, &sv1, &sort_hist, &kmm, &vis_count,
                      &tile_hist, &tile_range, &pair_count, &pair_base, &pairs, &row_hist, &row_range, &row_count,
                          &row_base, &rows, &debug, &stage_vm, &stage_pose, &stage_elev, &seg_off, &counter,
                          &ovf, &counter2})
            b->release();
    if (h_total) (void)hipHostFree(h_total);
    if (h_img) (void)hipHostFree(h_img);
    if (h_elev) (void)hipHostFree(h_elev);
    if (ev_total) (void)hipEventDestroy(ev_total);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (ev_staged) (void)hipEventDestroy(ev_staged);
    for (auto& kv : graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    twin.reset();
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
}

// ------------------------------------------------------------------ planning

int validate_desc(const gsr_ctx* ctx, const gsr_render_desc* d, const SceneRes* sc, bool need_outputs)
{
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
    if ((int64_t)d->n_envs * d->n_cams > (1 << 24)) return fail(GSR_E_INVALID, "more than 2^24 images in one call");
    if ((int64_t)d->n_envs * std::max(sc->dev.n_bodies, 1) * 7 > 0xFFFFFFFFLL ||
        (int64_t)d->n_envs * d->n_cams * 12 > 0xFFFFFFFFLL)
        return fail(GSR_E_INVALID, "pose / viewmat arrays too large");
    for (int c = 0; c < d->n_cams; ++c) {
        const int ab = d->cams[c].attach_body;
        if (ab < -1 || ab >= sc->dev.n_bodies)
            return fail(GSR_E_INVALID, "attach_body must be -1 or a body of the scene (0..B-1)");
    }
    if (need_outputs) {
        if (!d->out_depth) return fail(GSR_E_INVALID, "out_depth is NULL");
        if (!d->out_rgb && !d->obs) return fail(GSR_E_INVALID, "out_rgb is NULL and no observation is requested");
        if (((uintptr_t)d->out_rgb & 3) || ((uintptr_t)d->out_depth & 3) || ((uintptr_t)d->out_alpha & 3) ||
            ((uintptr_t)d->out_work & 3))
            return fail(GSR_E_INVALID, "outputs must be 4-byte aligned");
        if (d->obs) {
            const gsr_observation* o = d->obs;
            if (o->format != GSR_OBS_U8 && o->format != GSR_OBS_F16)
                return fail(GSR_E_INVALID, "observation format must be GSR_OBS_U8 or GSR_OBS_F16");
            if (!o->out) return fail(GSR_E_INVALID, "observation output is NULL");
            if (o->format == GSR_OBS_F16 && ((uintptr_t)o->out & 1))
                return fail(GSR_E_INVALID, "half observation output must be 2-byte aligned");
            if (((uintptr_t)o->gain & 3) || ((uintptr_t)o->contrast & 3) || ((uintptr_t)o->brightness & 3))
                return fail(GSR_E_INVALID, "observation parameters must be 4-byte aligned");
        }
    }
    return GSR_OK;
}

std::vector<ImageInfo> images_of(const gsr_render_desc* d, int ts, int n_bodies)
{
    std::vector<ImageInfo> v((size_t)d->n_envs * d->n_cams);
    fill_images(d, ts, n_bodies, v.data());
    return v;
}

void fill_images(const gsr_render_desc* d, int ts, int n_bodies, ImageInfo* v)
{
    const int E = d->n_envs;
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
            // binary32, one rounding per operation (this file is built without contraction)
            im.guard_x = 1.3f * ((0.5f * (float)cam.width) / cam.fx);
            im.guard_y = 1.3f * ((0.5f * (float)cam.height) / cam.fy);
            im.key_tile_base = (uint32_t)tile_base;
            im.vm_off = (uint32_t)(((size_t)c * E + e) * 12);
            im.pose_off = (uint32_t)((size_t)e * n_bodies * 7);
            im.bg[0] = d->bg[0];
            im.bg[1] = d->bg[1];
            im.bg[2] = d->bg[2];
            im.attach_body = cam.attach_body;
            if (d->out_depth) {
                im.out_rgb = d->out_rgb ? d->out_rgb + 3 * pixel_base : nullptr;
                im.out_depth = d->out_depth + pixel_base;
                im.out_alpha = d->out_alpha ? d->out_alpha + pixel_base : nullptr;
                im.out_work = d->out_work ? d->out_work + 2 * pixel_base : nullptr;
                if (d->obs) {
                    const gsr_observation* o = d->obs;
                    const size_t bpc = o->format == GSR_OBS_F16 ? 2 : 1;
                    im.out_obs = (char*)o->out + 3 * pixel_base * bpc;
                    im.obs_gain = o->gain;
                    im.obs_contrast = o->contrast;
                    im.obs_bright = o->brightness;
                    im.obs_fmt = o->format;
                    im.obs_idx = (uint32_t)((size_t)c * E + e);
                }
            }
            tile_base += (uint64_t)tx * ty;
            pixel_base += (uint64_t)cam.width * cam.height;
        }
    }
}

namespace {

size_t per_image_bytes(const SceneRes* sc, int t_max, int ty_max, int sort_blocks, int tile_blocks,
                       size_t rec_bytes = 48)
{
    const size_t n = (size_t)sc->dev.n;
    size_t b = n * (4 + 16 + rec_bytes + 16);                          // key, rect + sorted rect, record, sort buffers
    b += (size_t)(sc->dev.n_bodies + 1) * 64;                          // transforms
    b += (size_t)sort_blocks * (512 + 2) * 4 + (size_t)tile_blocks * ty_max * 4 + (size_t)(t_max + ty_max) * 8 + kKmmStride * 4;
    b += (size_t)(t_max + 2 * ty_max + 1) * 4;                         // tile difference array (bound)
    b += n * 8 * 4 + n * 3 * 8 + sizeof(ImageInfo) + 64;               // pair / row-entry estimates
    return b;
}

}  // namespace

size_t image_bytes_estimate(const SceneRes* sc, int width, int height, int ts)
{
    const int tx = (width + ts - 1) / ts, ty = (height + ts - 1) / ts;
    const int64_t n = sc->dev.n;
    const int sb = (int)std::max<int64_t>(1, (n + kSortItems - 1) / kSortItems);
    const int tb = (int)std::max<int64_t>(1, (n + kTileGauss - 1) / kTileGauss);
    return per_image_bytes(sc, tx * ty, ty, sb, tb);
}

ChunkPlan plan_chunks(const gsr_ctx* ctx, const SceneRes* sc, const std::vector<ImageInfo>& imgs, bool plain,
                      int chunk_images, size_t rec_bytes, int64_t chunk_bytes)
{
    const size_t budget = (size_t)(chunk_bytes > 0 ? chunk_bytes : ctx->opt.chunk_bytes);
    ChunkPlan p{};
    p.t_max = p.tx_max = p.ty_max = 1;
    for (const ImageInfo& im : imgs) {
        p.t_max = std::max(p.t_max, im.tiles_x * im.tiles_y);
        p.tx_max = std::max(p.tx_max, im.tiles_x);
        p.ty_max = std::max(p.ty_max, im.tiles_y);
    }
    const int64_t n = sc->dev.n;
    p.sort_blocks = (int)std::max<int64_t>(1, (n + kSortItems - 1) / kSortItems);
    p.tile_blocks = (int)std::max<int64_t>(1, (n + kTileGauss - 1) / kTileGauss);
    if (plain) {
        p.chunk = 1;
    } else {
        const size_t per = per_image_bytes(sc, p.t_max, p.ty_max, p.sort_blocks, p.tile_blocks, rec_bytes);
        size_t cap = budget;
        if (per * imgs.size() > cap) {
            // a job larger than one chunk: keep a chunk's working set (two with the
            // second stream) within 40 % of the device memory free now
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
                cap = std::min<size_t>(cap, std::max<size_t>(free_b / 5 * 2, (size_t)1 << 30));
        }
        size_t c = std::max<size_t>(1, cap / std::max<size_t>(per, 1));
        if (chunk_images > 0) c = std::min<size_t>(c, (size_t)chunk_images);
        // as many chunks as the budget needs, of equal size (no short last chunk)
        const size_t n_chunks = (imgs.size() + c - 1) / c;
        c = (imgs.size() + n_chunks - 1) / n_chunks;
        p.chunk = (int)std::min<size_t>(c, imgs.size());
    }
    return p;
}

WorkspaceSizes workspace_sizes(const SceneRes* sc, const ChunkPlan& p, size_t n_images_total, size_t rec_bytes)
{
    const size_t n = (size_t)std::max<int64_t>(sc->dev.n, 1);
    const size_t I = (size_t)p.chunk;
    WorkspaceSizes z{};
    int k = 0;
    auto add = [&](DevBuf Workspace::*b, size_t bytes) { z.b[k++] = {b, bytes}; };
    add(&Workspace::img, n_images_total * sizeof(ImageInfo));
    add(&Workspace::xform, I * (sc->dev.n_bodies + 1) * 64);
    add(&Workspace::keyz, I * n * 4);
    add(&Workspace::rect, I * n * 8);
    add(&Workspace::srect, I * n * 8);
    add(&Workspace::rec, I * n * rec_bytes);
    add(&Workspace::sk0, I * n * 4);
    add(&Workspace::sk1, I * n * 4);
    add(&Workspace::sv0, I * n * 4);
    add(&Workspace::sv1, I * n * 4);
    add(&Workspace::sort_hist, I * p.sort_blocks * (512 + 2) * 4);     // digit counts, then per-block key ranges
    add(&Workspace::kmm, I * kKmmStride * 4);
    add(&Workspace::vis_count, I * 4);
    add(&Workspace::tile_hist, I * (size_t)(p.tx_max + 1) * (p.ty_max + 1) * 4);
    add(&Workspace::tile_range, I * (size_t)p.t_max * 8);
    add(&Workspace::pair_count, I * 4);
    add(&Workspace::pair_base, (I + 2) * 8);
    add(&Workspace::row_hist, I * p.tile_blocks * (size_t)p.ty_max * 4);
    add(&Workspace::row_range, I * (size_t)p.ty_max * 8);
    add(&Workspace::row_count, I * 4);
    add(&Workspace::row_base, (I + 1) * 8);
    z.count = k;
    return z;
}

hipError_t ensure_workspace(Workspace& ws, const SceneRes* sc, const ChunkPlan& p, size_t n_images_total,
                            size_t rec_bytes)
{
    hipError_t e;
    const WorkspaceSizes z = workspace_sizes(sc, p, n_images_total, rec_bytes);
    for (int k = 0; k < z.count; ++k)
        if ((e = (ws.*(z.b[k].buf)).ensure(z.b[k].bytes)) != hipSuccess) return e;
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
        if ((e = hipEventCreateWithFlags(&ws.ev_staged, hipEventDisableTiming)) != hipSuccess) return e;
    }
    if ((e = ws.ovf.ensure(256)) != hipSuccess) return e;
    if ((e = ws.counter2.ensure(256)) != hipSuccess) return e;
    return hipSuccess;
}

std::string shape_key(const SceneRes* sc, const gsr_render_desc* d)
{
    std::string k = "n" + std::to_string(sc->dev.n) + "_b" + std::to_string(sc->dev.n_bodies) + "_d" +
                    std::to_string(sc->dev.degree) + "_s" + std::to_string(sc->dev.storage) + "_e" +
                    std::to_string(d->n_envs) + "_c";
    for (int c = 0; c < d->n_cams; ++c)
        k += (c ? "," : "") + std::to_string(d->cams[c].width) + "x" + std::to_string(d->cams[c].height);
    return k;
}

Tuning tuning_for(gsr_ctx* ctx, const SceneRes* sc, const gsr_render_desc* d)
{
    Tuning t;
    t.ts = ctx->opt.tile_size;
    t.ipt = ctx->opt.images_per_thread;
    t.batch = 64;                       // 64-record LDS batches: 8 workgroups per CU
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tuned.find(shape_key(sc, d));
    if (it != ctx->tuned.end()) t = it->second;
    return t;
}

namespace {

// Tile rectangles are packed into 4 bytes when every image of the chunk has at
// most kRect4MaxTiles tiles per axis (half the traffic of the rectangle
// gather in the last sort pass and of its readers).
int rect4_format(int tx_max, int ty_max) { return tx_max <= kRect4MaxTiles && ty_max <= kRect4MaxTiles ? 1 : 0; }

ChunkDev chunk_view(Workspace& ws, const SceneRes* sc, const ChunkPlan& p, int i0, int n_img,
                    const std::vector<ImageInfo>& imgs)
{
    ChunkDev c{};
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
    c.rect4 = rect4_format(tx_max, ty_max);
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
    c.kmm = ws.kmm.as<uint32_t>();
    c.kblk = c.sort_hist + (size_t)p.chunk * p.sort_blocks * 512;
    c.vis_count = ws.vis_count.as<uint32_t>();
    c.tile_hist = ws.tile_hist.as<int32_t>();
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

// One pipeline stage, launched eagerly or as a captured graph.  Graphs are
// captured on the workspace's private stream (capture executes nothing) and
// launched on the chunk's stream; a graph is re-captured when anything its
// launches depend on (buffers, sizes, parameters) changed.
int run_stage(Workspace& ws, bool graph, int chunk_idx, int stage, uint64_t scene_uid, const std::vector<uint64_t>& key,
              hipStream_t st, const std::function<hipError_t(hipStream_t)>& fn)
{
    if (!graph) {
        GSR_HIP_TRY(fn(st));
        return GSR_OK;
    }
    StageGraph& g = ws.graphs[{chunk_idx, stage}];
    if (!g.exec || g.key != key) {
        if (g.exec) {
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        if (!ws.capture_stream) GSR_HIP_TRY(hipStreamCreateWithFlags(&ws.capture_stream, hipStreamNonBlocking));
        GSR_HIP_TRY(hipStreamBeginCapture(ws.capture_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t e = fn(ws.capture_stream);
        hipGraph_t graph_ = nullptr;
        const hipError_t e2 = hipStreamEndCapture(ws.capture_stream, &graph_);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph_) (void)hipGraphDestroy(graph_);
            return hip_fail(e != hipSuccess ? e : e2, "stage capture");
        }
        const hipError_t e3 = hipGraphInstantiate(&g.exec, graph_, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph_);
        if (e3 != hipSuccess) {
            g.exec = nullptr;
            return hip_fail(e3, "hipGraphInstantiate");
        }
        g.key = key;
        g.scene_uid = scene_uid;
    }
    GSR_HIP_TRY(hipGraphLaunch(g.exec, st));
    return GSR_OK;
}

}  // namespace

// Enqueue the pipeline of images [i0, i0 + n_img) of `job` (image descriptions
// already on the device).  `pairs_total` receives the chunk's pair count.
int run_chunk(gsr_ctx* ctx, Workspace& ws, SceneRes* sc, const RenderJob& job, const ChunkPlan& plan, int i0,
              int n_img, int chunk_idx, hipStream_t st, Mode mode, bool graph, uint64_t* pairs_total,
              bool async_lists)
{
    ChunkDev c = chunk_view(ws, sc, plan, i0, n_img, job.imgs);
    c.err = ctx->d_err;
    c.ovf_count = ctx->d_err + 1;
    c.acc = reinterpret_cast<unsigned long long*>(ctx->d_err + 16);
    c.ovf = ws.ovf.as<uint32_t>();
    // synchronous lists: the host sizes the buffers from the totals, nothing overflows
    c.cap_pairs = async_lists ? ws.pairs.bytes / 4 : ~0ull;
    c.cap_rows = async_lists ? ws.rows.bytes / 8 : ~0ull;
    if (async_lists && ctx->list_cap) {            // a smaller capacity set for tests of the overflow path
        c.cap_pairs = std::min<uint64_t>(c.cap_pairs, ctx->list_cap);
        c.cap_rows = std::min<uint64_t>(c.cap_rows, ctx->list_cap);
    }
    if (async_lists && (int)ws.nseg_hint.size() <= chunk_idx)
        return fail(GSR_E_INVALID, "asynchronous lists without a planned chunk");
    const SceneDev& s = sc->dev;
    const Tuning& tu = job.tune;
    const bool prof = ctx->opt.profile && mode == Mode::kRender && !ws.fixed;
    StageEvents ev;
    // events of a chunk that fails before they are queued for reading go back to the spares
    struct Lease {
        gsr_ctx* ctx;
        StageEvents& ev;
        bool queued = false;
        ~Lease()
        {
            if (queued || !ev.e[0]) return;
            std::lock_guard<std::mutex> lk(ctx->mu);
            for (hipEvent_t e : ev.e)
                if (e) ctx->spare_events.push_back(e);
        }
    } lease{ctx, ev};
    if (prof) {
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            for (hipEvent_t& e : ev.e) {
                if (ctx->spare_events.empty()) break;
                e = ctx->spare_events.back();
                ctx->spare_events.pop_back();
            }
        }
        for (hipEvent_t& e : ev.e)
            if (!e) GSR_HIP_TRY(hipEventCreate(&e));
        GSR_HIP_TRY(hipEventRecord(ev.e[0], st));
    }
    // everything the captured launches depend on: the scene by its never-reused
    // uid and by what selects and feeds its kernels (storage format and SH
    // degree pick the projection's instantiation), the chunk's buffers, sizes
    // and launch parameters
    std::vector<uint64_t> key;
    if (graph)
        key = {sc->uid, (uint64_t)s.n, (uint64_t)s.storage, (uint64_t)s.degree,
                                 (uint64_t)s.n_bodies, (uint64_t)s.sh_chunks, (uint64_t)(uintptr_t)s.pos,
                                 (uint64_t)(uintptr_t)s.rot, (uint64_t)(uintptr_t)s.scale, (uint64_t)(uintptr_t)s.sh,
                                 (uint64_t)(uintptr_t)s.body_off, (uint64_t)job.lidar,
                                 (uint64_t)(uintptr_t)c.img, (uint64_t)n_img,
                                 (uint64_t)c.t_max, (uint64_t)c.tx_max, (uint64_t)c.ty_max, (uint64_t)c.sort_blocks,
                                 (uint64_t)c.tile_blocks, (uint64_t)tu.ts, (uint64_t)tu.batch, (uint64_t)tu.ipt,
                                 (uint64_t)tu.persistent, (uint64_t)(uintptr_t)job.viewmats,
                                 (uint64_t)(uintptr_t)job.poses, (uint64_t)(uintptr_t)ws.h_total,
                                 (uint64_t)(ctx->opt.cutoff * 1.0e6f), (uint64_t)tu.bin, (uint64_t)async_lists,
                                 c.cap_pairs, c.cap_rows};
    if (graph) {
        for (void* ptr : {(void*)c.xform, (void*)c.keyz, (void*)c.rect, (void*)c.srect, (void*)c.rec, (void*)c.sk[0],
                          (void*)c.sk[1], (void*)c.sv[0], (void*)c.sv[1], (void*)c.sort_hist, (void*)c.kmm,
                          (void*)c.vis_count,
                          (void*)c.tile_hist, (void*)c.tile_range, (void*)c.pair_count, (void*)c.pair_base,
                          (void*)c.row_hist, (void*)c.row_range, (void*)c.row_count, (void*)c.row_base})
            key.push_back((uint64_t)(uintptr_t)ptr);
        for (int k = 0; k < n_img; ++k)
            key.push_back(((uint64_t)job.imgs[i0 + k].width << 32) | (uint64_t)job.imgs[i0 + k].height);
    }

    int rc = run_stage(ws, graph, chunk_idx, 0, sc->uid, key, st, [&](hipStream_t q) {
        hipError_t e = launch_compose(s, c, job.viewmats, job.poses, q);
        if (e == hipSuccess)
            e = job.lidar ? launch_project_lidar(s, c, tu.ts, tu.ipt, q)
                          : launch_project(s, c, tu.ts, ctx->opt.cutoff, tu.ipt, q);
        return e;
    });
    if (rc) return rc;
    if (mode == Mode::kProject) return GSR_OK;
    if (prof) GSR_HIP_TRY(hipEventRecord(ev.e[1], st));
    rc = run_stage(ws, graph, chunk_idx, 1, sc->uid, key, st, [&](hipStream_t q) { return launch_depth_sort(s, c, q); });
    if (rc) return rc;
    if (prof) GSR_HIP_TRY(hipEventRecord(ev.e[2], st));
    rc = run_stage(ws, graph, chunk_idx, 2, sc->uid, key, st, [&](hipStream_t q) {
        hipError_t e = launch_tile_count(s, c, q);
        if (async_lists) return e;       // totals stay on the device
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws.h_total, c.pair_base + n_img, sizeof(uint64_t), hipMemcpyDeviceToHost, q);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws.h_total + 1, c.row_base + n_img, sizeof(uint64_t), hipMemcpyDeviceToHost, q);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws.h_total + 2, c.pair_base + n_img + 1, sizeof(uint64_t), hipMemcpyDeviceToHost, q);
        if (e == hipSuccess) e = hipMemcpyAsync(ws.h_total + 3, c.err, sizeof(uint32_t), hipMemcpyDeviceToHost, q);
        return e;
    });
    if (rc) return rc;
    if (prof) GSR_HIP_TRY(hipEventRecord(ev.e[3], st));
    uint64_t total = 0, row_total = 0;
    int n_seg = 1;
    const uint64_t n_rows = (uint64_t)n_img * (uint64_t)c.ty_max;
    if (async_lists) {
        // the buffers hold what the planning render needed (with margin); the
        // device checks this chunk's totals against them
        n_seg = ws.nseg_hint[chunk_idx];
        *pairs_total = 0;
    } else {
        GSR_HIP_TRY(hipEventRecord(ws.ev_total, st));
        GSR_HIP_TRY(hipEventSynchronize(ws.ev_total));
        // kernels of this or an earlier chunk met an entry their inputs cannot hold
        const uint32_t err = reinterpret_cast<const uint32_t*>(ws.h_total + 3)[0];
        if (err) {
            ctx->poisoned = true;
            char msg[160];
            std::snprintf(msg, sizeof msg, "device consistency check failed (error bits 0x%x: %s)", err,
                          err & kErrListEntry ? "tile list entry out of range"
                          : err & kErrSortSlot ? "depth-sort offset out of range" : "tile-row entry out of range");
            return fail(GSR_E_DEVICE, msg);
        }
        total = ws.h_total[0];
        row_total = ws.h_total[1];
        *pairs_total = total;
        // segments per tile-row list: enough level-2 waves for the launch, none shorter than kRowSegEntries
        const uint64_t per_row = n_rows ? row_total / n_rows : 0;
        const uint64_t by_len = std::max<uint64_t>(1, per_row / kRowSegEntries);
        const uint64_t by_waves = n_rows ? ((uint64_t)kLevel2Waves + n_rows - 1) / n_rows : 1;
        n_seg = (int)std::min<uint64_t>(32, std::min(by_len, by_waves));
        if ((int)ws.nseg_hint.size() <= chunk_idx) ws.nseg_hint.resize((size_t)chunk_idx + 1, 1);
        ws.nseg_hint[chunk_idx] = n_seg;
    }
    // everything enqueued before ev_total has completed, including earlier chunks: growing is safe
    auto grow = [&](DevBuf& b, uint64_t entries, size_t entry_bytes, const char* what) -> int {
        const size_t need = (size_t)entries * entry_bytes;
        if (b.bytes >= need) return GSR_OK;
        const size_t want = std::max<size_t>(std::max<size_t>(need, (size_t)((double)b.bytes * 1.5)) + need / 8, 1 << 20);
        const hipError_t e = b.ensure(want);
        if (e == hipSuccess) return GSR_OK;
        char msg[256];
        std::snprintf(msg, sizeof msg, "%s list of a %d-image chunk: %llu entries, %zu bytes requested (%s)", what,
                      n_img, (unsigned long long)entries, want, hipGetErrorString(e));
        return fail(e == hipErrorOutOfMemory ? GSR_E_OOM : GSR_E_DEVICE, msg);
    };
    const size_t seg_bytes = n_seg > 1 ? (size_t)(n_rows * (uint64_t)n_seg * (uint64_t)c.tx_max * 4) : 0;
    if (ws.fixed) {
        // lists carved from the fixed list region; the caller re-plans on GSR_E_OVERFLOW
        const size_t bp = ((size_t)total * 4 + 255) & ~(size_t)255, br = ((size_t)row_total * 8 + 255) & ~(size_t)255;
        if (bp + br + seg_bytes > ws.list_bytes) {
            char msg[256];
            std::snprintf(msg, sizeof msg,
                          "%d-image chunk needs %zu bytes of tile lists (%llu pairs, %llu row entries); %zu available",
                          n_img, bp + br + seg_bytes, (unsigned long long)total, (unsigned long long)row_total,
                          ws.list_bytes);
            return fail(GSR_E_OVERFLOW, msg);
        }
        ws.pairs = {ws.list_base, bp};
        ws.rows = {ws.list_base + bp, br};
        ws.seg_off = {ws.list_base + bp + br, seg_bytes};
    } else if (!async_lists) {
        if ((rc = grow(ws.pairs, total, 4, "tile")) != GSR_OK) return rc;
        if ((rc = grow(ws.rows, row_total, 8, "tile-row")) != GSR_OK) return rc;
        if (n_seg > 1) GSR_HIP_TRY(ws.seg_off.ensure(seg_bytes));
    } else if (n_seg > 1 && ws.seg_off.bytes < seg_bytes) {
        return fail(GSR_E_INVALID, "asynchronous lists: segment offsets not planned");
    }
    c.pairs = ws.pairs.as<uint32_t>();
    c.rows = ws.rows.as<uint2>();
    uint32_t* seg_off = n_seg > 1 ? ws.seg_off.as<uint32_t>() : nullptr;
    if (graph) {
        key.push_back((uint64_t)(uintptr_t)c.pairs);
        key.push_back((uint64_t)(uintptr_t)c.rows);
        key.push_back((uint64_t)n_seg);
        key.push_back((uint64_t)(uintptr_t)seg_off);
    }
    rc = run_stage(ws, graph, chunk_idx, 3, sc->uid, key, st,
                   [&](hipStream_t q) { return launch_tile_scatter(s, c, tu.bin, n_seg, seg_off, q); });
    if (rc) return rc;
    if (mode == Mode::kBins) return GSR_OK;
    if (prof) GSR_HIP_TRY(hipEventRecord(ev.e[4], st));

    RasterParams rp{};
    rp.ts = tu.ts;
    rp.batch = tu.batch;
    rp.persistent = tu.persistent;
    rp.count_work = 0;
    for (int k = 0; k < n_img; ++k) rp.count_work |= job.imgs[i0 + k].out_work != nullptr;
    rp.persistent_blocks = ctx->cu_count * (tu.ts == 8 ? 16 : 4);
    if (tu.persistent) {
        if (!ws.fixed) GSR_HIP_TRY(ws.counter.ensure(256));
        rp.counter = ws.counter.as<uint32_t>();
    }
    uint32_t blocks = 0;
    const std::vector<ImageInfo>& imgs = job.imgs;
    for (int k = 0; k < n_img;) {
        const ImageInfo& a = imgs[i0 + k];
        int m = k;
        while (m < n_img && imgs[i0 + m].width == a.width && imgs[i0 + m].height == a.height) ++m;
        if (rp.n_segs >= kMaxSegs) return fail(GSR_E_INVALID, "more than 8 image sizes in one chunk");
        RasterSeg& sg = rp.segs[rp.n_segs++];
        sg.first_tile = blocks;
        sg.first_image = (uint32_t)k;
        sg.n_images = (uint32_t)(m - k);
        sg.tiles_per_image = (uint32_t)(a.tiles_x * a.tiles_y);
        blocks += sg.n_images * sg.tiles_per_image;
        k = m;
    }
    rp.n_blocks = blocks;
    if (graph) {
        key.push_back((uint64_t)(uintptr_t)rp.counter);
        key.push_back((uint64_t)rp.count_work);
    }
    if (job.lidar) {
        rc = run_stage(ws, graph, chunk_idx, 4, sc->uid, key, st,
                       [&](hipStream_t q) { return launch_raster_lidar(s, c, rp, q); });
    } else {
        rc = run_stage(ws, graph, chunk_idx, 4, sc->uid, key, st, [&](hipStream_t q) {
            hipError_t e = launch_raster(s, c, rp, q);
            // asynchronous lists: the fallback composites the chunk if its lists overflowed (else it exits at once)
            if (e == hipSuccess && async_lists) e = launch_raster_fallback(s, c, rp, ws.counter2.as<uint32_t>(), q);
            return e;
        });
    }
    if (rc) return rc;
    if (prof) {
        GSR_HIP_TRY(hipEventRecord(ev.e[5], st));
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->pending.push_back(ev);
        lease.queued = true;
    }
    return GSR_OK;
}

Workspace* acquire_workspace_locked(gsr_ctx* ctx, hipStream_t stream)
{
    Workspace* got = nullptr;
    for (auto& w : ctx->pool)
        if (!got && !w->in_call && (!w->used || w->last_stream == stream)) got = w.get();
    for (auto& w : ctx->pool)
        if (!got && !w->in_call && hipEventQuery(w->ev_done) == hipSuccess) got = w.get();
    if (!got) {
        ctx->pool.emplace_back(new Workspace());
        got = ctx->pool.back().get();
    }
    // graphs of scenes destroyed while the workspace was in a call
    for (uint64_t uid : got->dead_scenes) got->drop_graphs_of(uid);
    got->dead_scenes.clear();
    return got;
}

int render_job(gsr_ctx* ctx, Workspace& ws, SceneRes* sc, const RenderJob& job_in, hipStream_t st, bool plain,
               bool graphs, bool two_streams)
{
    if (job_in.imgs.empty()) return GSR_OK;
    RenderJob job = job_in;
    const size_t rec_bytes = job.lidar ? 80 : 48;
    const ChunkPlan plan = plan_chunks(ctx, sc, job.imgs, plain, job.tune.chunk_images, rec_bytes, job.chunk_bytes);
    const int n_chunks = (int)((job.imgs.size() + plan.chunk - 1) / plan.chunk);
    bool two = two_streams && !plain && ctx->opt.overlap >= 0 && n_chunks > 1;
    // Asynchronous lists need a planning render of the same job shape on this
    // workspace (and its twin), whose list buffers and segment counts they
    // reuse, and no overflow seen since: the counter's copy made at the end of
    // this workspace's last render is read once that render has finished.
    std::vector<uint64_t> shape = {sc->uid, (uint64_t)plan.chunk, (uint64_t)job.imgs.size(), (uint64_t)job.tune.ts,
                                   (uint64_t)job.tune.batch, (uint64_t)job.tune.ipt, (uint64_t)job.tune.bin,
                                   (uint64_t)job.tune.persistent, (uint64_t)two, (uint64_t)ctx->list_cap};
    {
        uint64_t h = 1469598103934665603ull;          // FNV-1a over the image sizes
        for (const ImageInfo& im : job.imgs) {
            h = (h ^ (uint64_t)im.width) * 1099511628211ull;
            h = (h ^ (uint64_t)im.height) * 1099511628211ull;
        }
        shape.push_back(h);
    }
    bool async = !plain && !job.lidar && job.mode == Mode::kRender && !job.stop && !ws.fixed &&
                 ctx->opt.sync_lists >= 0 && ws.used && ws.plan_key == shape &&
                 (!two || (ws.twin && ws.twin->plan_key == shape));
    if (async && hipEventQuery(ws.ev_done) == hipSuccess) {
        const uint32_t seen = reinterpret_cast<const uint32_t*>(ws.h_total + 5)[0];
        if (seen != ctx->ovf_seen) {
            ctx->ovf_seen = seen;
            async = false;                              // a chunk overflowed: plan again (the buffers grow)
        }
    }
    // synchronous renders may reallocate buffers: earlier work on this workspace must be finished
    if (ws.used && !async) GSR_HIP_TRY(hipEventSynchronize(ws.ev_done));
    GSR_HIP_TRY(ensure_workspace(ws, sc, plan, job.imgs.size(), rec_bytes));
    // the staging buffer of the image descriptions is free once its last copy has run
    if (ws.used) GSR_HIP_TRY(hipEventSynchronize(ws.ev_staged));
    // per-step inputs staged at fixed addresses, so captured graphs replay across steps
    if (job.viewmats != ws.stage_vm.as<float>()) {
        GSR_HIP_TRY(ws.stage_vm.ensure(std::max<size_t>(job.viewmat_floats, 1) * 4));
        GSR_HIP_TRY(hipMemcpyAsync(ws.stage_vm.p, job.viewmats, job.viewmat_floats * 4, hipMemcpyDeviceToDevice, st));
        job.viewmats = ws.stage_vm.as<float>();
    }
    if (job.pose_floats && job.poses != ws.stage_pose.as<float>()) {
        GSR_HIP_TRY(ws.stage_pose.ensure(job.pose_floats * 4));
        GSR_HIP_TRY(hipMemcpyAsync(ws.stage_pose.p, job.poses, job.pose_floats * 4, hipMemcpyDeviceToDevice, st));
        job.poses = ws.stage_pose.as<float>();
    }
    std::memcpy(ws.h_img, job.imgs.data(), job.imgs.size() * sizeof(ImageInfo));
    GSR_HIP_TRY(hipMemcpyAsync(ws.img.p, ws.h_img, job.imgs.size() * sizeof(ImageInfo), hipMemcpyHostToDevice, st));
    if (plain) job.tune.ipt = 1;
    const bool use_graphs = graphs && !plain && ctx->opt.graphs >= 0;
    // Two streams: even chunks on the caller's stream in `ws`, odd chunks on
    // ws.side in ws.twin.  The host's wait for chunk k+1's pair total then
    // ends while chunk k still rasterises, and chunk k+1's lists and raster
    // follow on the other stream, so binning and raster of neighbouring
    // chunks share the GPU.  Each workspace is used by one stream only.
    Workspace* wk[2] = {&ws, &ws};
    hipStream_t sq[2] = {st, st};
    if (two) {
        if (!ws.twin) ws.twin.reset(new (std::nothrow) Workspace());
        if (!ws.twin) return fail(GSR_E_OOM, "workspace allocation failed");
        if (!ws.side) GSR_HIP_TRY(hipStreamCreateWithFlags(&ws.side, hipStreamNonBlocking));
        if (!ws.ev_fork) GSR_HIP_TRY(hipEventCreateWithFlags(&ws.ev_fork, hipEventDisableTiming));
        if (!ws.ev_join) GSR_HIP_TRY(hipEventCreateWithFlags(&ws.ev_join, hipEventDisableTiming));
        // the twin's earlier work was joined into `st` before ws.ev_done
        const hipError_t e = ensure_workspace(*ws.twin, sc, plan, job.imgs.size(), rec_bytes);
        if (e == hipErrorOutOfMemory) {
            // no room for a second working set: free it and render on one stream
            (void)hipGetLastError();
            ws.twin.reset();
            two = false;
        } else if (e != hipSuccess) {
            return hip_fail(e, "ensure_workspace (second working set)");
        }
    }
    if (two) {
        Workspace& t = *ws.twin;
        if (t.ev_staged) GSR_HIP_TRY(hipEventSynchronize(t.ev_staged));
        std::memcpy(t.h_img, job.imgs.data(), job.imgs.size() * sizeof(ImageInfo));
        GSR_HIP_TRY(hipMemcpyAsync(t.img.p, t.h_img, job.imgs.size() * sizeof(ImageInfo), hipMemcpyHostToDevice, st));
        GSR_HIP_TRY(hipEventRecord(t.ev_staged, st));
        GSR_HIP_TRY(hipEventRecord(ws.ev_fork, st));
        GSR_HIP_TRY(hipStreamWaitEvent(ws.side, ws.ev_fork, 0));
        wk[1] = &t;
        sq[1] = ws.side;
    }
    GSR_HIP_TRY(hipEventRecord(ws.ev_staged, st));
    int chunk_idx = 0;
    int rc = GSR_OK;
    for (int i0 = 0; i0 < (int)job.imgs.size() && !rc; i0 += plan.chunk, ++chunk_idx) {
        const int n_img = std::min<int>(plan.chunk, (int)job.imgs.size() - i0);
        const int h = chunk_idx & 1;
        uint64_t total = 0;
        rc = run_chunk(ctx, *wk[h], sc, job, plan, i0, n_img, chunk_idx, sq[h], job.mode, use_graphs, &total, async);
        if (!rc && job.stop && job.stop->image >= i0 && job.stop->image < i0 + n_img) {
            job.stop->ws = wk[h];
            job.stop->i0 = i0;
            job.stop->n_img = n_img;
            job.stop->plan = plan;
            job.stop->pairs = total;
            break;
        }
    }
    if (two) {
        // join the side stream even after a failure, so ws.ev_done covers it
        const hipError_t e1 = hipEventRecord(ws.ev_join, ws.side);
        const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(st, ws.ev_join, 0) : e1;
        if (e2 != hipSuccess && !rc) rc = hip_fail(e2, "joining the side stream");
    }
    if (rc) {
        if (rc == GSR_E_DEVICE) ctx->poisoned = true;
        ws.plan_key.clear();
        if (ws.twin) ws.twin->plan_key.clear();
        return rc;
    }
    // the overflow counter as of this render's end, read by a later render
    GSR_HIP_TRY(hipMemcpyAsync(ws.h_total + 5, ctx->d_err + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GSR_HIP_TRY(hipEventRecord(ws.ev_done, st));
    ws.used = true;
    ws.last_stream = st;
    if (!async && !plain && !job.lidar && job.mode == Mode::kRender && !job.stop) {
        // this render sized the list buffers of its shape: later ones may go asynchronously
        ws.plan_key = shape;
        if (two) ws.twin->plan_key = shape;
    }
    return GSR_OK;
}

SceneRes* acquire_scene(gsr_ctx* ctx, uint64_t id)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->scenes.find(id);
    if (it == ctx->scenes.end()) return nullptr;
    it->second->in_calls.fetch_add(1);
    return it->second.get();
}

void release_scene(SceneRes* sc) { sc->in_calls.fetch_sub(1); }

int mark_scene_use(gsr_ctx* ctx, SceneRes* sc, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!sc->last_use) GSR_HIP_TRY(hipEventCreateWithFlags(&sc->last_use, hipEventDisableTiming));
    GSR_HIP_TRY(hipEventRecord(sc->last_use, st));
    sc->used = true;
    return GSR_OK;
}

}  // namespace gsr

using namespace gsr;

namespace {

int render_impl(gsr_ctx* ctx, const gsr_render_desc* d, void* stream, bool plain, const Tuning* force = nullptr)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d) return fail(GSR_E_INVALID, "render desc is NULL");
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_desc(ctx, d, sc, true);
    if (rc) {
        release_scene(sc);
        return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    Workspace* ws;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws = acquire_workspace_locked(ctx, st);
        ws->in_call = true;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) rc = hip_fail(e, "hipSetDevice");
    if (!rc) {
        RenderJob job;
        job.tune = force ? *force : tuning_for(ctx, sc, d);
        job.imgs = images_of(d, job.tune.ts, sc->dev.n_bodies);
        job.viewmats = d->viewmats;
        job.poses = d->body_poses;
        job.viewmat_floats = (size_t)d->n_cams * d->n_envs * 12;
        job.pose_floats = (size_t)d->n_envs * sc->dev.n_bodies * 7;
        rc = render_job(ctx, *ws, sc, job, st, plain, true, true);
    }
    if (!rc) rc = mark_scene_use(ctx, sc, st);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws->in_call = false;
        if (!rc) ctx->renders += 1;
    }
    release_scene(sc);
    return rc;
}

int debug_run(gsr_ctx* ctx, const gsr_render_desc* d, int image, Mode mode, SceneRes** sc_out, Workspace** ws_out,
              RenderJob* job, ChunkPlan* plan, uint64_t* total)
{
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    *sc_out = sc;
    int rc = validate_desc(ctx, d, sc, false);
    if (rc) return rc;
    if (image < 0 || image >= d->n_envs * d->n_cams) return fail(GSR_E_INVALID, "image index out of range");
    GSR_HIP_TRY(hipSetDevice(ctx->device));
    GSR_HIP_TRY(hipDeviceSynchronize());
    Workspace* ws;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws = acquire_workspace_locked(ctx, nullptr);
        ws->in_call = true;
    }
    *ws_out = ws;
    job->tune.ts = ctx->opt.tile_size;
    job->tune.batch = 64;
    job->tune.ipt = 1;
    job->tune.bin = tuning_for(ctx, sc, d).bin;     // the tile lists as the tuned renderer builds them
    job->imgs = images_of(d, ctx->opt.tile_size, sc->dev.n_bodies);
    job->viewmats = d->viewmats;
    job->poses = d->body_poses;
    *plan = plan_chunks(ctx, sc, job->imgs, true);
    GSR_HIP_TRY(ensure_workspace(*ws, sc, *plan, job->imgs.size()));
    std::memcpy(ws->h_img, job->imgs.data(), job->imgs.size() * sizeof(ImageInfo));
    GSR_HIP_TRY(hipMemcpy(ws->img.p, ws->h_img, job->imgs.size() * sizeof(ImageInfo), hipMemcpyHostToDevice));
    rc = run_chunk(ctx, *ws, sc, *job, *plan, image, 1, 0, nullptr, mode, false, total);
    if (rc) return rc;
    GSR_HIP_TRY(hipDeviceSynchronize());
    return GSR_OK;
}

void debug_finish(gsr_ctx* ctx, SceneRes* sc, Workspace* ws)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ws) ws->in_call = false;
    if (sc) sc->in_calls.fetch_sub(1);
}

}  // namespace

// ============================================================== exported API

GSR_EXPORT const char* gsr_last_error(void) { return g_err.c_str(); }

GSR_EXPORT const char* gsr_version(void) { return "gsr 0.2 (gfx950)"; }

GSR_EXPORT int gsr_create(int device, const gsr_options* opt, gsr_ctx** out)
{
    if (!out) return fail(GSR_E_INVALID, "out is NULL");
    *out = nullptr;
    gsr_options o{};
    if (opt) o = *opt;
    if (o.tile_size == 0) o.tile_size = 16;
    if (o.images_per_thread == 0) o.images_per_thread = 16;
    if (o.chunk_bytes == 0) o.chunk_bytes = (int64_t)48 << 30;
    if (o.cutoff == 0.0f) o.cutoff = 3.33f;
    if (o.tile_size != 8 && o.tile_size != 16 && o.tile_size != 32)
        return fail(GSR_E_INVALID, "tile_size must be 8, 16 or 32");
    if (o.images_per_thread < 1 || o.images_per_thread > 16)
        return fail(GSR_E_INVALID, "images_per_thread must be in 1..16");
    if (o.chunk_bytes < (int64_t)(64 << 20)) return fail(GSR_E_INVALID, "chunk_bytes must be >= 64 MiB");
    if (!(o.cutoff >= 1.0f && o.cutoff <= 8.0f)) return fail(GSR_E_INVALID, "cutoff must be in [1, 8]");
    if (o.list_cap < 0) return fail(GSR_E_INVALID, "list_cap must be >= 0");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(GSR_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(GSR_E_DEVICE, "device ordinal out of range");
    hipDeviceProp_t prop;
    GSR_HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GSR_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", libgsr is built for gfx950");
    GSR_HIP_TRY(hipSetDevice(device));
    gsr_ctx* ctx = new (std::nothrow) gsr_ctx();
    if (!ctx) return fail(GSR_E_OOM, "context allocation failed");
    ctx->device = device;
    ctx->opt = o;
    ctx->list_cap = (uint64_t)o.list_cap;
    ctx->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    int rc = noalloc_setup(device);
    if (!rc) {
        // consistency bits the kernels raise (zero until something impossible happens)
        hipError_t e = hipMalloc((void**)&ctx->d_err, 256);
        if (e == hipSuccess) e = hipMemset(ctx->d_err, 0, 256);
        if (e != hipSuccess) rc = hip_fail(e, "context error word");
    }
    if (rc) {
        if (ctx->d_err) (void)hipFree(ctx->d_err);
        delete ctx;
        return rc;
    }
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
        for (hipEvent_t e : ctx->spare_events) (void)hipEventDestroy(e);
        ctx->spare_events.clear();
        ctx->pool.clear();
        ctx->scenes.clear();
        if (ctx->d_err) (void)hipFree(ctx->d_err);
    }
    delete ctx;
    return GSR_OK;
}

GSR_EXPORT int gsr_trim(gsr_ctx* ctx, int64_t* freed_bytes)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    GSR_HIP_TRY(hipSetDevice(ctx->device));
    size_t before = 0, after = 0, total = 0;
    GSR_HIP_TRY(hipMemGetInfo(&before, &total));
    for (auto it = ctx->pool.begin(); it != ctx->pool.end();) {
        Workspace* w = it->get();
        if (w->in_call) {
            ++it;
            continue;
        }
        // its last render (and its twin's, joined into the same stream) must have finished
        if (w->used) GSR_HIP_TRY(hipEventSynchronize(w->ev_done));
        it = ctx->pool.erase(it);
    }
    GSR_HIP_TRY(hipMemGetInfo(&after, &total));
    if (freed_bytes) *freed_bytes = (int64_t)after - (int64_t)before;
    return GSR_OK;
}

GSR_EXPORT int gsr_scene_create(gsr_ctx* ctx, const gsr_scene_desc* d, uint64_t* scene_id)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d || !scene_id) return fail(GSR_E_INVALID, "desc / scene_id is NULL");
    if (d->n < 0 || d->n > ((int64_t)1 << 31) - 64) return fail(GSR_E_INVALID, "n must be in [0, 2^31 - 64)");
    if (d->sh_degree < 0 || d->sh_degree > kMaxShDegree) return fail(GSR_E_INVALID, "sh_degree must be 0..3");
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
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    GSR_HIP_TRY(hipSetDevice(ctx->device));
    std::unique_ptr<SceneRes> sc(new SceneRes());
    const int64_t n = d->n;
    const int64_t n_pad = std::max<int64_t>(64, (n + 63) / 64 * 64);
    const int K = (d->sh_degree + 1) * (d->sh_degree + 1);
    const bool half = d->storage != GSR_STORAGE_F32;
    const int chunks = half ? (3 * K + 7) / 8 : (3 * K + 3) / 4;
    GSR_HIP_TRY(sc->pos.ensure((size_t)n_pad * 16));
    GSR_HIP_TRY(sc->rot.ensure((size_t)n_pad * 16));
    if (!half) GSR_HIP_TRY(sc->scale.ensure((size_t)n_pad * 16));
    GSR_HIP_TRY(sc->sh.ensure((size_t)chunks * n_pad * 16));
    std::vector<int> off(d->n_bodies + 1);
    for (int b = 0; b <= d->n_bodies; ++b) off[b] = (int)d->body_offsets[b];
    GSR_HIP_TRY(sc->body_off.ensure(off.size() * sizeof(int)));
    GSR_HIP_TRY(hipMemcpy(sc->body_off.p, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    if (n > 0) {
        const float *m = d->means, *s = d->scales, *q = d->quats, *o = d->opacities, *f = d->sh;
        DevBuf tmp;
        if (d->mem_kind == GSR_MEM_HOST) {
            const size_t b_m = n * 12, b_s = n * 12, b_q = n * 16, b_o = n * 4, b_f = (size_t)n * K * 12;
            GSR_HIP_TRY(tmp.ensure(b_m + b_s + b_q + b_o + b_f));
            char* base = tmp.as<char>();
            GSR_HIP_TRY(hipMemcpy(base, d->means, b_m, hipMemcpyHostToDevice));
            GSR_HIP_TRY(hipMemcpy(base + b_m, d->scales, b_s, hipMemcpyHostToDevice));
            GSR_HIP_TRY(hipMemcpy(base + b_m + b_s, d->quats, b_q, hipMemcpyHostToDevice));
            GSR_HIP_TRY(hipMemcpy(base + b_m + b_s + b_q, d->opacities, b_o, hipMemcpyHostToDevice));
            GSR_HIP_TRY(hipMemcpy(base + b_m + b_s + b_q + b_o, d->sh, b_f, hipMemcpyHostToDevice));
            m = (const float*)base;
            s = (const float*)(base + b_m);
            q = (const float*)(base + b_m + b_s);
            o = (const float*)(base + b_m + b_s + b_q);
            f = (const float*)(base + b_m + b_s + b_q + b_o);
        }
        GSR_HIP_TRY(launch_scene_convert(d->storage, n, n_pad, d->sh_degree, m, s, q, o, f, sc->pos.as<float4>(),
                                         sc->rot.p, sc->scale.as<float4>(), sc->sh.p, nullptr));
        GSR_HIP_TRY(hipDeviceSynchronize());
        tmp.release();
    }
    SceneDev& dv = sc->dev;
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
    // created here so that marking the scene's use allocates nothing
    GSR_HIP_TRY(hipEventCreateWithFlags(&sc->last_use, hipEventDisableTiming));
    static std::atomic<uint64_t> next_uid{1};
    sc->uid = next_uid.fetch_add(1);
    std::lock_guard<std::mutex> lk(ctx->mu);
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
    if (sc->in_calls.load() > 0) return fail(GSR_E_BUSY, "scene is used by a render call in progress");
    if (sc->used && sc->last_use && hipEventQuery(sc->last_use) == hipErrorNotReady)
        return fail(GSR_E_BUSY, "scene is used by in-flight work");
    // captured graphs hold the scene's device pointers: drop them now where no
    // call owns the workspace, else when the workspace is next handed out
    for (auto& w : ctx->pool) {
        if (w->in_call) w->dead_scenes.push_back(sc->uid);
        else w->drop_graphs_of(sc->uid);
    }
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
    GSR_HIP_TRY(hipSetDevice(ctx->device));
    for (StageEvents& ev : ctx->pending) {
        GSR_HIP_TRY(hipEventSynchronize(ev.e[5]));
        for (int k = 0; k < 5; ++k) {
            float t = 0.0f;
            GSR_HIP_TRY(hipEventElapsedTime(&t, ev.e[k], ev.e[k + 1]));
            ctx->stage_ms[k] += t;
        }
        ctx->raster_launches += 1;
        for (hipEvent_t e : ev.e) ctx->spare_events.push_back(e);
    }
    ctx->pending.clear();
    for (int k = 0; k < 5; ++k) ms[k] = ctx->stage_ms[k];
    ms[5] = ctx->raster_launches;
    ms[6] = ctx->renders;
    if (n >= 10) {
        // device accumulators of every chunk's totals (since the last reset)
        GSR_HIP_TRY(hipDeviceSynchronize());
        unsigned long long acc[3];
        GSR_HIP_TRY(hipMemcpy(acc, ctx->d_err + 16, sizeof acc, hipMemcpyDeviceToHost));
        ms[7] = (double)(acc[0] - ctx->acc_base[0]);
        ms[8] = (double)(acc[1] - ctx->acc_base[1]);
        ms[9] = (double)(acc[2] - ctx->acc_base[2]);
    }
    if (reset) {
        for (double& v : ctx->stage_ms) v = 0.0;
        ctx->raster_launches = 0;
        ctx->renders = 0;
        GSR_HIP_TRY(hipDeviceSynchronize());
        GSR_HIP_TRY(hipMemcpy(ctx->acc_base, ctx->d_err + 16, sizeof ctx->acc_base, hipMemcpyDeviceToHost));
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

// ------------------------------------------------------------------ LiDAR

namespace {

// A listed-ray slot's device tables, written to `out` (floats; the caller
// indices as their bit patterns): rays ordered by (elevation, index) and cut
// into H bands of W; within a band by (azimuth, index).  out = [H] smallest
// and [H] largest elevation of each band, then [H][W] azimuths, [H][W]
// elevations and [H][W] caller indices, then per ts x ts tile of rays the
// smallest and the largest azimuth ([TY][TX] each; along a tile row both
// ascend, since each band's azimuths do).
size_t ray_list_floats(const gsr_lidar& L, int ts)
{
    const size_t H = (size_t)L.height, W = (size_t)L.width;
    const size_t TX = (W + ts - 1) / ts, TY = (H + ts - 1) / ts;
    return 2 * H + 3 * H * W + 2 * TX * TY;
}

void stage_ray_list(const gsr_lidar& L, int ts, float* out)
{
    const size_t H = (size_t)L.height, W = (size_t)L.width, n = H * W;
    std::vector<uint32_t> idx(n);
    for (size_t k = 0; k < n; ++k) idx[k] = (uint32_t)k;
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return L.ray_el[a] < L.ray_el[b]; });
    float* lo = out;
    float* hi = out + H;
    float* az = out + 2 * H;
    float* el = az + n;
    float* perm = el + n;
    for (size_t r = 0; r < H; ++r) {
        uint32_t* band = idx.data() + r * W;
        lo[r] = L.ray_el[band[0]];
        hi[r] = L.ray_el[band[W - 1]];
        std::stable_sort(band, band + W, [&](uint32_t a, uint32_t b) { return L.ray_az[a] < L.ray_az[b]; });
        for (size_t c = 0; c < W; ++c) {
            const uint32_t k = band[c];
            az[r * W + c] = L.ray_az[k];
            el[r * W + c] = L.ray_el[k];
            std::memcpy(perm + r * W + c, &k, sizeof k);
        }
    }
    const size_t TX = (W + ts - 1) / ts, TY = (H + ts - 1) / ts;
    float* tmin = perm + n;
    float* tmax = tmin + TX * TY;
    for (size_t ty = 0; ty < TY; ++ty)
        for (size_t tx = 0; tx < TX; ++tx) {
            float a = az[ty * ts * W + tx * ts], b = a;
            const size_t c_end = std::min(W, (tx + 1) * ts) - 1;
            for (size_t r = ty * ts; r < std::min(H, (ty + 1) * ts); ++r) {
                a = std::min(a, az[r * W + tx * ts]);
                b = std::max(b, az[r * W + c_end]);
            }
            tmin[ty * TX + tx] = a;
            tmax[ty * TX + tx] = b;
        }
}

int validate_lidar(const gsr_ctx* ctx, const gsr_lidar_desc* d, const SceneRes* sc)
{
    if (d->n_envs < 1) return fail(GSR_E_INVALID, "n_envs must be >= 1");
    if (d->n_lidars < 1 || d->n_lidars > kMaxCams) return fail(GSR_E_INVALID, "n_lidars must be in 1..8");
    if (!d->lidars) return fail(GSR_E_INVALID, "lidars is NULL");
    if (!d->viewmats) return fail(GSR_E_INVALID, "viewmats is NULL");
    if (sc->dev.n_bodies > 0 && !d->body_poses) return fail(GSR_E_INVALID, "body_poses is NULL but the scene has bodies");
    if (!d->out_range) return fail(GSR_E_INVALID, "out_range is NULL");
    if (((uintptr_t)d->viewmats & 3) || ((uintptr_t)d->body_poses & 3) || ((uintptr_t)d->out_range & 3) ||
        ((uintptr_t)d->out_hit & 3))
        return fail(GSR_E_INVALID, "arrays must be 4-byte aligned");
    const int ts = ctx->opt.tile_size;
    if (ts > 16) return fail(GSR_E_INVALID, "LiDAR ray tiles need a context tile size of 8 or 16");
    const double two_pi = 6.283185307179586;
    for (int l = 0; l < d->n_lidars; ++l) {
        const gsr_lidar& L = d->lidars[l];
        if (L.width < 1 || L.height < 1 || L.width > 8192 || L.height > 8192)
            return fail(GSR_E_INVALID, "LiDAR grid size must be in 1..8192");
        if (L.pattern == GSR_LIDAR_GRID) {
            if (!(L.dx > 0.0f) || !(L.dy > 0.0f) || !std::isfinite(L.dx) || !std::isfinite(L.dy) ||
                !std::isfinite(L.x0) || !std::isfinite(L.y0))
                return fail(GSR_E_INVALID, "heightmap grid: x0, y0 finite and dx, dy > 0");
        } else if (L.pattern == GSR_LIDAR_ANGULAR) {
            if (!(L.az_step > 0.0f) || !std::isfinite(L.az0) || (double)L.width * L.az_step > two_pi * (1.0 + 1e-6))
                return fail(GSR_E_INVALID, "az_step must be > 0 with width * az_step <= 2 pi");
            if (!L.elevations) return fail(GSR_E_INVALID, "elevations is NULL");
            for (int r = 0; r < L.height; ++r) {
                const float e = L.elevations[r];
                if (!(e > -1.5707963f && e < 1.5707963f))
                    return fail(GSR_E_INVALID, "elevations must lie in (-pi/2, pi/2)");
                if (r > 0 && !(e > L.elevations[r - 1])) return fail(GSR_E_INVALID, "elevations must ascend strictly");
            }
        } else if (L.pattern == GSR_LIDAR_RAYS) {
            if (!L.ray_az || !L.ray_el) return fail(GSR_E_INVALID, "ray_az / ray_el is NULL");
            const int64_t n = (int64_t)L.width * L.height;
            if (n > (1 << 22)) return fail(GSR_E_INVALID, "more than 2^22 listed rays in one LiDAR slot");
            for (int64_t k = 0; k < n; ++k) {
                const float a = L.ray_az[k], e = L.ray_el[k];
                if (!(a >= -3.14159265f && a <= 3.14159265f))
                    return fail(GSR_E_INVALID, "ray azimuths must lie in [-pi, pi]");
                if (!(e > -1.5707963f && e < 1.5707963f))
                    return fail(GSR_E_INVALID, "ray elevations must lie in (-pi/2, pi/2)");
            }
        } else {
            return fail(GSR_E_INVALID, "LiDAR pattern must be GSR_LIDAR_ANGULAR, GSR_LIDAR_GRID or GSR_LIDAR_RAYS");
        }
        if (!(L.near_range > 0.0f)) return fail(GSR_E_INVALID, "near_range must be > 0");
        if (L.attach_body < -1 || L.attach_body >= sc->dev.n_bodies)
            return fail(GSR_E_INVALID, "attach_body must be -1 or a body of the scene (0..B-1)");
        const int64_t tiles = (int64_t)((L.width + ts - 1) / ts) * ((L.height + ts - 1) / ts);
        if (tiles > 15000) return fail(GSR_E_INVALID, "more than 15000 tiles per LiDAR grid for this tile size");
    }
    if ((int64_t)d->n_envs * d->n_lidars > (1 << 24)) return fail(GSR_E_INVALID, "more than 2^24 scans in one call");
    return GSR_OK;
}

}  // namespace

GSR_EXPORT int gsr_render_lidar(gsr_ctx* ctx, const gsr_lidar_desc* d, void* stream)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d) return fail(GSR_E_INVALID, "LiDAR desc is NULL");
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_lidar(ctx, d, sc);
    if (rc) {
        release_scene(sc);
        return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    Workspace* ws;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws = acquire_workspace_locked(ctx, st);
        ws->in_call = true;
    }
    auto body = [&]() -> int {
        GSR_HIP_TRY(hipSetDevice(ctx->device));
        // beam elevations of every slot, staged in pinned memory and copied to
        // the device (earlier work on this workspace must be done with them)
        if (ws->used) GSR_HIP_TRY(hipEventSynchronize(ws->ev_done));
        // per slot: angular, its H beam elevations; listed rays, the band
        // tables [2][H], azimuths, elevations and caller indices [H][W] each
        // and the tiles' azimuth spans [2][TY][TX]
        auto staged = [&](const gsr_lidar& L) -> size_t {
            if (L.pattern == GSR_LIDAR_ANGULAR) return (size_t)L.height;
            if (L.pattern == GSR_LIDAR_RAYS) return ray_list_floats(L, ctx->opt.tile_size);
            return 0;
        };
        size_t n_elev = 0;
        for (int l = 0; l < d->n_lidars; ++l) n_elev += staged(d->lidars[l]);
        n_elev = std::max<size_t>(n_elev, 1);
        if (ws->h_elev_cap < n_elev) {
            if (ws->h_elev) (void)hipHostFree(ws->h_elev);
            ws->h_elev = nullptr;
            ws->h_elev_cap = 0;
            GSR_HIP_TRY(hipHostMalloc((void**)&ws->h_elev, n_elev * sizeof(float), hipHostMallocDefault));
            ws->h_elev_cap = n_elev;
        }
        GSR_HIP_TRY(ws->stage_elev.ensure(n_elev * sizeof(float)));
        RenderJob job;
        job.lidar = true;
        job.tune.ts = ctx->opt.tile_size;
        job.tune.batch = 256;
        job.tune.ipt = ctx->opt.images_per_thread;
        // scan grids have few tile rows: the expansion schedule places their
        // row entries without a transpose per group (16 vs 28 ms per
        // 2048-scan step of the 32 x 1024 scanner)
        job.tune.bin = 0;
        const int E = d->n_envs, B = sc->dev.n_bodies, ts = job.tune.ts;
        job.imgs.resize((size_t)E * d->n_lidars);
        uint64_t tile_base = 0, ray_base = 0;
        size_t eo = 0;
        for (int l = 0; l < d->n_lidars; ++l) {
            const gsr_lidar& L = d->lidars[l];
            const bool grid = L.pattern == GSR_LIDAR_GRID, rays = L.pattern == GSR_LIDAR_RAYS;
            const size_t H = (size_t)L.height, W = (size_t)L.width;
            if (L.pattern == GSR_LIDAR_ANGULAR) std::memcpy(ws->h_elev + eo, L.elevations, H * sizeof(float));
            if (rays) stage_ray_list(L, ts, ws->h_elev + eo);
            const int tx = (L.width + ts - 1) / ts, ty = (L.height + ts - 1) / ts;
            for (int e = 0; e < E; ++e) {
                ImageInfo& im = job.imgs[(size_t)l * E + e];
                std::memset(&im, 0, sizeof im);
                im.kind = grid ? 2 : 1;
                im.width = L.width;
                im.height = L.height;
                im.tiles_x = tx;
                im.tiles_y = ty;
                im.near_plane = L.near_range;
                if (grid) {
                    im.gx0 = L.x0;
                    im.gy0 = L.y0;
                    im.gdx = L.dx;
                    im.gdy = L.dy;
                } else if (rays) {
                    im.kind = 3;
                    const float* base = ws->stage_elev.as<float>() + eo;
                    im.elev = base;
                    im.ray_az = base + 2 * H;
                    im.ray_el = base + 2 * H + H * W;
                    im.ray_perm = reinterpret_cast<const uint32_t*>(base + 2 * H + 2 * H * W);
                    im.ray_tile_az = base + 2 * H + 3 * H * W;
                } else {
                    im.az0 = L.az0;
                    im.az_step = L.az_step;
                    im.elev = ws->stage_elev.as<float>() + eo;
                }
                im.attach_body = L.attach_body;
                im.key_tile_base = (uint32_t)tile_base;
                im.vm_off = (uint32_t)(((size_t)l * E + e) * 12);
                im.pose_off = (uint32_t)((size_t)e * B * 7);
                im.out_depth = d->out_range + ray_base;
                im.out_alpha = d->out_hit ? d->out_hit + ray_base : nullptr;
                tile_base += (uint64_t)tx * ty;
                ray_base += (uint64_t)L.width * L.height;
            }
            eo += staged(L);
        }
        GSR_HIP_TRY(hipMemcpyAsync(ws->stage_elev.p, ws->h_elev, n_elev * sizeof(float), hipMemcpyHostToDevice, st));
        // grids of equal size contiguous (one raster segment each)
        std::stable_sort(job.imgs.begin(), job.imgs.end(), [](const ImageInfo& a, const ImageInfo& b) {
            return a.width != b.width ? a.width < b.width : a.height < b.height;
        });
        job.viewmats = d->viewmats;
        job.poses = d->body_poses;
        job.viewmat_floats = (size_t)d->n_lidars * E * 12;
        job.pose_floats = (size_t)E * B * 7;
        return render_job(ctx, *ws, sc, job, st, false, false, true);
    };
    rc = body();
    if (!rc) rc = mark_scene_use(ctx, sc, st);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws->in_call = false;
    }
    release_scene(sc);
    return rc;
}

GSR_EXPORT int gsr_debug_bins(gsr_ctx* ctx, const gsr_render_desc* d, int image, gsr_bins_out* out)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d || !out) return fail(GSR_E_INVALID, "desc / out is NULL");
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_desc(ctx, d, sc, false);
    if (!rc && (image < 0 || image >= d->n_envs * d->n_cams)) rc = fail(GSR_E_INVALID, "image index out of range");
    if (rc) {
        release_scene(sc);
        return rc;
    }
    Workspace* ws;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws = acquire_workspace_locked(ctx, nullptr);
        ws->in_call = true;
    }
    // The render sequence of gsr_render (its tuning, memory chunks, captured
    // graphs and two streams), every chunk up to the one holding `image`
    // stopping after its tile lists; the image's lists are then read from
    // that chunk's buffers.
    auto body = [&]() -> int {
        GSR_HIP_TRY(hipSetDevice(ctx->device));
        RenderJob job;
        job.tune = tuning_for(ctx, sc, d);
        job.imgs = images_of(d, job.tune.ts, sc->dev.n_bodies);
        job.viewmats = d->viewmats;
        job.poses = d->body_poses;
        job.viewmat_floats = (size_t)d->n_cams * d->n_envs * 12;
        job.pose_floats = (size_t)d->n_envs * sc->dev.n_bodies * 7;
        job.mode = Mode::kBins;
        DebugStop stop;
        stop.image = image;
        job.stop = &stop;
        int r = render_job(ctx, *ws, sc, job, nullptr, false, true, true);
        if (r) return r;
        GSR_HIP_TRY(hipDeviceSynchronize());
        if (!stop.ws) return fail(GSR_E_DEVICE, "debug stop not reached");
        Workspace& cw = *stop.ws;
        const int k = image - stop.i0;
        const ImageInfo& im = job.imgs[image];
        const int T = im.tiles_x * im.tiles_y;
        ChunkDev c = chunk_view(cw, sc, stop.plan, stop.i0, stop.n_img, job.imgs);
        uint32_t vis = 0, npairs = 0;
        uint64_t pbase = 0;
        if (sc->dev.n > 0) GSR_HIP_TRY(hipMemcpy(&vis, c.vis_count + k, 4, hipMemcpyDeviceToHost));
        GSR_HIP_TRY(hipMemcpy(&npairs, c.pair_count + k, 4, hipMemcpyDeviceToHost));
        GSR_HIP_TRY(hipMemcpy(&pbase, c.pair_base + k, 8, hipMemcpyDeviceToHost));
        out->n_pairs = npairs;
        out->n_visible = vis;
        out->tiles_x = im.tiles_x;
        out->tiles_y = im.tiles_y;
        out->tile_base = im.key_tile_base;
        out->tile_size = job.tune.ts;
        if (out->ranges) {
            if (out->ranges_capacity < T) return fail(GSR_E_INVALID, "ranges_capacity smaller than the tile count");
            GSR_HIP_TRY(hipMemcpy(out->ranges, c.tile_range + (size_t)k * c.t_max * 2, (size_t)T * 8,
                                  hipMemcpyDeviceToHost));
        }
        if ((int64_t)npairs > out->capacity) return fail(GSR_E_INVALID, "capacity smaller than the number of pairs");
        if (npairs == 0) return GSR_OK;
        GSR_HIP_TRY(cw.debug.ensure((size_t)npairs * 8));
        GSR_HIP_TRY(launch_debug_keys(c, k, (uint64_t)sc->dev.n, c.pairs + pbase, npairs, cw.debug.as<uint64_t>(),
                                      nullptr));
        GSR_HIP_TRY(hipDeviceSynchronize());
        if (out->keys) GSR_HIP_TRY(hipMemcpy(out->keys, cw.debug.p, (size_t)npairs * 8, hipMemcpyDeviceToHost));
        if (out->values)
            GSR_HIP_TRY(hipMemcpy(out->values, c.pairs + pbase, (size_t)npairs * 4, hipMemcpyDeviceToHost));
        return GSR_OK;
    };
    rc = body();
    if (rc == GSR_E_DEVICE) ctx->poisoned = true;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws->in_call = false;
    }
    release_scene(sc);
    return rc;
}

GSR_EXPORT int gsr_debug_project(gsr_ctx* ctx, const gsr_render_desc* d, int image, gsr_proj_out* out)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d || !out) return fail(GSR_E_INVALID, "desc / out is NULL");
    {
        SceneRes* probe = acquire_scene(ctx, d->scene_id);
        if (!probe) return fail(GSR_E_NOT_FOUND, "unknown scene id");
        const int64_t n = probe->dev.n;
        release_scene(probe);
        if (out->n != n) return fail(GSR_E_INVALID, "out->n must equal the scene's Gaussian count");
        if (n == 0) return GSR_OK;
    }
    SceneRes* sc = nullptr;
    Workspace* ws = nullptr;
    RenderJob job;
    ChunkPlan plan{};
    uint64_t total = 0;
    int rc = debug_run(ctx, d, image, Mode::kProject, &sc, &ws, &job, &plan, &total);
    const int64_t n = out->n;
    if (!rc && out->zkey && hipMemcpy(out->zkey, ws->keyz.p, (size_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(GSR_E_DEVICE, "copy of keys failed");
    if (!rc && out->rect) {
        std::vector<uint32_t> r((size_t)n * 2);
        if (hipMemcpy(r.data(), ws->rect.p, (size_t)n * 8, hipMemcpyDeviceToHost) != hipSuccess) {
            rc = fail(GSR_E_DEVICE, "copy of rectangles failed");
        } else {
            const ImageInfo& im = job.imgs[image];
            const bool packed = rect4_format(im.tiles_x, im.tiles_y) != 0;   // the debug chunk is this one image
            for (int64_t g = 0; g < n; ++g) {
                if (packed) {
                    const uint32_t v = r[g];
                    out->rect[4 * g + 0] = (int32_t)(v & 0xFF);
                    out->rect[4 * g + 1] = (int32_t)((v >> 8) & 0xFF);
                    out->rect[4 * g + 2] = (int32_t)((v >> 16) & 0xFF);
                    out->rect[4 * g + 3] = (int32_t)(v >> 24);
                } else {
                    out->rect[4 * g + 0] = (int32_t)(r[2 * g] & 0xFFFF);
                    out->rect[4 * g + 1] = (int32_t)(r[2 * g] >> 16);
                    out->rect[4 * g + 2] = (int32_t)(r[2 * g + 1] & 0xFFFF);
                    out->rect[4 * g + 3] = (int32_t)(r[2 * g + 1] >> 16);
                }
            }
        }
    }
    if (!rc && out->rec && hipMemcpy(out->rec, ws->rec.p, (size_t)n * 48, hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(GSR_E_DEVICE, "copy of records failed");
    debug_finish(ctx, sc, ws);
    return rc;
}

// ============================================================== autotuning

namespace {

bool tuning_valid(const gsr_ctx* ctx, const gsr_render_desc* d, const Tuning& t, std::string* why)
{
    if (t.ts != 8 && t.ts != 16 && t.ts != 32) return *why = "tile_size must be 8, 16 or 32", false;
    if (t.batch != 64 && t.batch != 128 && t.batch != 256 && (t.ts == 8 || t.batch != 512))
        return *why = "lds_batch must be 64/128/256 for 8-pixel tiles, 64/128/256/512 otherwise", false;
    if (t.ipt < 1 || t.ipt > 16) return *why = "images_per_thread must be in 1..16", false;
    if (t.persistent != 0 && t.persistent != 1) return *why = "persistent must be 0 or 1", false;
    if (t.chunk_images < 0) return *why = "chunk_images must be >= 0", false;
    if (t.bin != 0 && t.bin != 1) return *why = "bin_schedule must be 0 or 1", false;
    for (int c = 0; c < d->n_cams; ++c) {
        const int64_t tiles = (int64_t)((d->cams[c].width + t.ts - 1) / t.ts) * ((d->cams[c].height + t.ts - 1) / t.ts);
        if (tiles > 15000) return *why = "more than 15000 tiles per image for this tile size", false;
    }
    (void)ctx;
    return true;
}

Tuning from_public(const gsr_tuning* t)
{
    Tuning r;
    r.ts = t->tile_size;
    r.batch = t->lds_batch;
    r.ipt = t->images_per_thread;
    r.persistent = t->persistent;
    r.chunk_images = t->chunk_images;
    r.bin = t->bin_schedule;
    r.ms = t->ms;
    return r;
}

void to_public(const Tuning& t, gsr_tuning* o)
{
    std::memset(o, 0, sizeof *o);
    o->tile_size = t.ts;
    o->lds_batch = t.batch;
    o->images_per_thread = t.ipt;
    o->persistent = t.persistent;
    o->chunk_images = t.chunk_images;
    o->bin_schedule = t.bin;
    o->ms = t.ms;
}

}  // namespace

GSR_EXPORT int gsr_tuning_get(gsr_ctx* ctx, const gsr_render_desc* d, gsr_tuning* out)
{
    if (!ctx || !d || !out) return fail(GSR_E_INVALID, "ctx / desc / out is NULL");
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_desc(ctx, d, sc, false);
    if (!rc) to_public(tuning_for(ctx, sc, d), out);
    release_scene(sc);
    return rc;
}

GSR_EXPORT int gsr_tuning_set(gsr_ctx* ctx, const gsr_render_desc* d, const gsr_tuning* t)
{
    if (!ctx || !d || !t) return fail(GSR_E_INVALID, "ctx / desc / tuning is NULL");
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_desc(ctx, d, sc, false);
    std::string why;
    const Tuning tu = from_public(t);
    if (!rc && !tuning_valid(ctx, d, tu, &why)) rc = fail(GSR_E_INVALID, why);
    if (!rc) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tuned[shape_key(sc, d)] = tu;
    }
    release_scene(sc);
    return rc;
}

GSR_EXPORT int gsr_autotune(gsr_ctx* ctx, const gsr_render_desc* d, void* stream, gsr_tuning* best)
{
    if (!ctx || !d) return fail(GSR_E_INVALID, "ctx / desc is NULL");
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_desc(ctx, d, sc, true);
    const std::string key = rc ? std::string() : shape_key(sc, d);
    Tuning cur = rc ? Tuning() : tuning_for(ctx, sc, d);
    release_scene(sc);
    if (rc) return rc;
    GSR_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    GSR_HIP_TRY(hipEventCreate(&e0));
    GSR_HIP_TRY(hipEventCreate(&e1));
    auto time_of = [&](const Tuning& t, double* ms) -> int {
        int r = render_impl(ctx, d, stream, false, &t);     // warm-up (captures graphs, grows buffers)
        if (r) return r;
        if (hipEventRecord(e0, st) != hipSuccess) return fail(GSR_E_DEVICE, "event record");
        // four renders: candidates differ by a few per cent, about the spread of single renders
        for (int k = 0; k < 4 && !r; ++k) r = render_impl(ctx, d, stream, false, &t);
        if (r) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return fail(GSR_E_DEVICE, "event sync");
        float f = 0.0f;
        if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return fail(GSR_E_DEVICE, "event time");
        *ms = f / 4.0;
        return GSR_OK;
    };
    double best_ms = 0.0;
    rc = time_of(cur, &best_ms);
    std::string why;
    auto consider = [&](Tuning t) {
        if (rc || !tuning_valid(ctx, d, t, &why)) return;
        double ms = 0.0;
        const int r = time_of(t, &ms);
        if (r == GSR_E_OOM || r == GSR_E_INVALID) return;   // candidate does not fit: skip it
        if (r) {
            rc = r;
            return;
        }
        if (ms < best_ms) {
            // confirm against the incumbent timed again, back to back: the
            // incumbent's first timing may date from before the clocks settled,
            // and a stale, slow baseline lets any later candidate win
            double inc = 0.0, again = 0.0;
            int r2 = time_of(cur, &inc);
            if (!r2) r2 = time_of(t, &again);
            if (r2) {
                rc = r2;
                return;
            }
            if (again < inc) {
                best_ms = again;
                cur = t;
            } else {
                best_ms = inc;
            }
        }
    };
    for (int ts : {8, 16, 32}) {
        if (ts == cur.ts) continue;
        Tuning t = cur;
        t.ts = ts;
        t.batch = 64;
        consider(t);
    }
    for (int b : {64, 128, 256, 512}) {
        if (b == cur.batch) continue;
        Tuning t = cur;
        t.batch = b;
        consider(t);
    }
    for (int ipt : {1, 2, 4, 8, 16}) {
        if (ipt == cur.ipt) continue;
        Tuning t = cur;
        t.ipt = ipt;
        consider(t);
    }
    {
        Tuning t = cur;
        t.persistent = 1 - cur.persistent;
        consider(t);
    }
    {
        Tuning t = cur;
        t.bin = 1 - cur.bin;
        consider(t);
    }
    for (int ch : {0, 64, 256}) {
        if (ch == cur.chunk_images) continue;
        Tuning t = cur;
        t.chunk_images = ch;
        consider(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    cur.ms = (float)best_ms;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tuned[key] = cur;
    }
    if (best) to_public(cur, best);
    return GSR_OK;
}

GSR_EXPORT int gsr_tuning_save(gsr_ctx* ctx, const char* path)
{
    if (!ctx || !path) return fail(GSR_E_INVALID, "ctx / path is NULL");
    std::ofstream f(path);
    if (!f) return fail(GSR_E_INVALID, std::string("cannot write ") + path);
    f.precision(9);
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const auto& kv : ctx->tuned) {
        const Tuning& t = kv.second;
        f << "{\"key\": \"" << kv.first << "\", \"tile_size\": " << t.ts << ", \"lds_batch\": " << t.batch
          << ", \"images_per_thread\": " << t.ipt << ", \"persistent\": " << t.persistent
          << ", \"chunk_images\": " << t.chunk_images << ", \"bin_schedule\": " << t.bin << ", \"ms\": " << t.ms
          << "}\n";
    }
    return f ? GSR_OK : fail(GSR_E_INVALID, "write failed");
}

GSR_EXPORT int gsr_tuning_load(gsr_ctx* ctx, const char* path)
{
    if (!ctx || !path) return fail(GSR_E_INVALID, "ctx / path is NULL");
    std::ifstream f(path);
    if (!f) return fail(GSR_E_NOT_FOUND, std::string("cannot read ") + path);
    std::string line;
    std::map<std::string, Tuning> got;
    auto num = [](const std::string& l, const char* name, double* v) {
        const std::string pat = std::string("\"") + name + "\":";
        const size_t p = l.find(pat);
        if (p == std::string::npos) return false;
        *v = std::strtod(l.c_str() + p + pat.size(), nullptr);
        return true;
    };
    while (std::getline(f, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        const std::string kp = "\"key\": \"";
        const size_t a = line.find(kp);
        const size_t b = a == std::string::npos ? a : line.find('"', a + kp.size());
        double ts, ba, ipt, pe, ch, ms, bs = 1;
        if (a == std::string::npos || b == std::string::npos || !num(line, "tile_size", &ts) ||
            !num(line, "lds_batch", &ba) || !num(line, "images_per_thread", &ipt) || !num(line, "persistent", &pe) ||
            !num(line, "chunk_images", &ch) || !num(line, "ms", &ms))
            return fail(GSR_E_INVALID, "malformed tuning line: " + line);
        Tuning t;
        t.ts = (int)ts;
        t.batch = (int)ba;
        t.ipt = (int)ipt;
        t.persistent = (int)pe;
        t.chunk_images = (int)ch;
        (void)num(line, "bin_schedule", &bs);     // optional: older caches predate it
        t.bin = (int)bs;
        t.ms = (float)ms;
        if ((t.ts != 8 && t.ts != 16 && t.ts != 32) || t.ipt < 1 || t.ipt > 16 || (t.persistent != 0 && t.persistent != 1) ||
            t.chunk_images < 0 || (t.bin != 0 && t.bin != 1) ||
            (t.batch != 64 && t.batch != 128 && t.batch != 256 && (t.ts == 8 || t.batch != 512)))
            return fail(GSR_E_INVALID, "invalid tuning values: " + line);
        got[line.substr(a + kp.size(), b - a - kp.size())] = t;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const auto& kv : got) ctx->tuned[kv.first] = kv.second;
    return GSR_OK;
}
