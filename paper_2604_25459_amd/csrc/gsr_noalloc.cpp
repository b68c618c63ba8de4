// Allocation-free rendering: gsr_render_noalloc runs the batched pipeline of
// gsr_render (same kernels, same per-image results) with every byte of its
// device working memory inside one fixed scratch array per device, for
// callers that cannot allocate device memory.
//
// The scratch array is a file-scope __device__ array.  In host code its name
// is only a stand-in: the device address is resolved once per device at
// set-up (gsr_create, with that device current) and every host use -- kernel
// arguments, copies -- goes through that address.
//
// Layout of the scratch for one call: image descriptions of the whole call,
// then the per-chunk buffers of a chunk of I images, then the chunk's tile
// lists in the rest.  I starts from an estimate of the lists' size; a chunk
// whose lists turn out not to fit is planned again with fewer images (its
// binning runs again; nothing has been written to the outputs yet), and a
// single image whose lists do not fit fails with GSR_E_OVERFLOW.
#include <algorithm>
#include <cstring>
#include <memory>

#include "gsr_runtime.h"

#define GSR_EXPORT extern "C" __attribute__((visibility("default")))

namespace gsr {
namespace {

constexpr size_t kScratchBytes = (size_t)GSR_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxImages = GSR_NOALLOC_MAX_IMAGES;
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Allocation-free path of one device: created at set-up, kept until the
// process ends.
struct NoallocDev {
    std::mutex mu;                    // one call at a time on the host
    char* ptr = nullptr;              // device address of `scratch` on this device
    Workspace ws;                     // fixed workspace over ptr (pinned staging h_total / h_img, ev_total)
    RenderJob job;                    // image list with capacity for kMaxImages (never grows)
    hipEvent_t ev_staged = nullptr;   // the last call's image descriptions have left ws.h_img
    hipEvent_t ev_done = nullptr;     // the last call's work has finished
    bool used = false;
};

std::mutex g_setup_mu;
NoallocDev* g_dev[kMaxDevices] = {};

size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// Bytes of the per-chunk buffers of a chunk of plan.chunk images (image
// descriptions excluded), each 256-byte aligned, plus the raster counters and
// the overflow word.
size_t chunk_fixed_bytes(const SceneRes* sc, const ChunkPlan& plan)
{
    const WorkspaceSizes z = workspace_sizes(sc, plan, 0);
    size_t b = 3 * kAlign;            // persistent-raster counters and the chunk's overflow word
    for (int k = 0; k < z.count; ++k)
        if (z.b[k].buf != &Workspace::img) b += align_up(z.b[k].bytes);
    return b;
}

// Points the workspace's per-chunk buffers into the scratch from `base` on;
// the tile lists get what is left up to `end`.
void carve(Workspace& ws, const SceneRes* sc, const ChunkPlan& plan, char* base, char* end)
{
    const WorkspaceSizes z = workspace_sizes(sc, plan, 0);
    char* p = base;
    ws.counter = {p, kAlign};
    p += kAlign;
    ws.counter2 = {p, kAlign};
    p += kAlign;
    ws.ovf = {p, kAlign};
    p += kAlign;
    for (int k = 0; k < z.count; ++k) {
        if (z.b[k].buf == &Workspace::img) continue;
        ws.*(z.b[k].buf) = {p, z.b[k].bytes};
        p += align_up(z.b[k].bytes);
    }
    ws.list_base = p;
    ws.list_bytes = (size_t)(end - p);
}

}  // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(GSR_E_DEVICE, "device ordinal beyond the supported 64");
    std::lock_guard<std::mutex> lk(g_setup_mu);
    if (g_dev[device]) return GSR_OK;
    std::unique_ptr<NoallocDev> d(new (std::nothrow) NoallocDev());
    if (!d) return fail(GSR_E_OOM, "allocation-free path: host allocation failed");
    void* p = nullptr;
    GSR_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GSR_E_DEVICE, "allocation-free path: scratch array has no device address");
    d->ptr = static_cast<char*>(p);
    d->ws.fixed = true;
    GSR_HIP_TRY(hipHostMalloc((void**)&d->ws.h_total, 64, hipHostMallocDefault));
    GSR_HIP_TRY(hipHostMalloc((void**)&d->ws.h_img, (size_t)kMaxImages * sizeof(ImageInfo), hipHostMallocDefault));
    d->ws.h_img_cap = kMaxImages;
    GSR_HIP_TRY(hipEventCreateWithFlags(&d->ws.ev_total, hipEventDisableTiming));
    GSR_HIP_TRY(hipEventCreateWithFlags(&d->ev_staged, hipEventDisableTiming));
    GSR_HIP_TRY(hipEventCreateWithFlags(&d->ev_done, hipEventDisableTiming));
    d->job.imgs.reserve(kMaxImages);
    g_dev[device] = d.release();
    return GSR_OK;
}

namespace {

int render_noalloc(gsr_ctx* ctx, NoallocDev& nd, SceneRes* sc, const gsr_render_desc* d, hipStream_t st)
{
    const int n_img = d->n_envs * d->n_cams;
    RenderJob& job = nd.job;
    job.tune = Tuning();
    job.tune.ts = ctx->opt.tile_size;
    job.tune.ipt = ctx->opt.images_per_thread;
    job.imgs.resize((size_t)n_img);           // within the reserved capacity: no allocation
    fill_images(d, job.tune.ts, sc->dev.n_bodies, job.imgs.data());
    job.viewmats = d->viewmats;
    job.poses = d->body_poses;
    job.viewmat_floats = (size_t)d->n_cams * d->n_envs * 12;
    job.pose_floats = (size_t)d->n_envs * sc->dev.n_bodies * 7;

    // sizes first, so that a call that can never fit enqueues nothing
    const size_t img_bytes = align_up((size_t)n_img * sizeof(ImageInfo));
    const size_t budget = kScratchBytes - img_bytes;
    // images per chunk from the per-image estimate (tile lists included)
    ChunkPlan plan = plan_chunks(ctx, sc, job.imgs, false, 0, 48, (int64_t)budget);
    int chunk = std::max(1, std::min(plan.chunk, n_img));
    plan.chunk = 1;
    const size_t one = chunk_fixed_bytes(sc, plan);
    if (one + kAlign > budget) {
        char msg[256];
        std::snprintf(msg, sizeof msg,
                      "allocation-free render: one image of this scene (%lld Gaussians) needs %zu bytes of working "
                      "memory before its tile lists; the scratch holds %zu",
                      (long long)sc->dev.n, one, kScratchBytes);
        return fail(GSR_E_INVALID, msg);
    }
    // fewer if the fixed part alone would leave no room for lists
    while (chunk > 1) {
        plan.chunk = chunk;
        if (chunk_fixed_bytes(sc, plan) + (size_t)chunk * kAlign * 4 <= budget) break;
        chunk = (chunk + 1) / 2;
    }

    // work of the previous call (on any stream) has finished with the scratch
    // before this call's first write to it
    if (nd.used) {
        GSR_HIP_TRY(hipStreamWaitEvent(st, nd.ev_done, 0));
        GSR_HIP_TRY(hipEventSynchronize(nd.ev_staged));     // its descriptions have left the staging buffer
    }
    std::memcpy(nd.ws.h_img, job.imgs.data(), (size_t)n_img * sizeof(ImageInfo));
    GSR_HIP_TRY(hipMemcpyAsync(nd.ptr, nd.ws.h_img, (size_t)n_img * sizeof(ImageInfo), hipMemcpyHostToDevice, st));
    GSR_HIP_TRY(hipEventRecord(nd.ev_staged, st));
    nd.used = true;
    nd.ws.img = {nd.ptr, img_bytes};

    int rc = GSR_OK;
    int chunk_idx = 0;
    for (int i0 = 0; i0 < n_img;) {
        const int m = std::min(chunk, n_img - i0);
        plan.chunk = m;
        carve(nd.ws, sc, plan, nd.ptr + img_bytes, nd.ptr + kScratchBytes);
        uint64_t total = 0;
        rc = run_chunk(ctx, nd.ws, sc, job, plan, i0, m, chunk_idx, st, Mode::kRender, false, &total);
        if (rc == GSR_E_OVERFLOW && m > 1) {
            chunk = m / 2;             // the same images again in smaller chunks
            rc = GSR_OK;
            continue;
        }
        if (rc) break;
        i0 += m;
        ++chunk_idx;
    }
    const hipError_t e = hipEventRecord(nd.ev_done, st);
    if (!rc && e != hipSuccess) rc = hip_fail(e, "hipEventRecord");
    if (rc == GSR_E_DEVICE) ctx->poisoned = true;
    return rc;
}

}  // namespace
}  // namespace gsr

using namespace gsr;

GSR_EXPORT int gsr_render_noalloc(gsr_ctx* ctx, const gsr_render_desc* d, void* stream)
{
    if (!ctx) return fail(GSR_E_INVALID, "ctx is NULL");
    if (!d) return fail(GSR_E_INVALID, "render desc is NULL");
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_dev[ctx->device])
        return fail(GSR_E_DEVICE, "allocation-free path not set up on this device");
    NoallocDev& nd = *g_dev[ctx->device];
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_desc(ctx, d, sc, true);
    if (!rc && (int64_t)d->n_envs * d->n_cams > kMaxImages)
        rc = fail(GSR_E_INVALID, "allocation-free render: more than GSR_NOALLOC_MAX_IMAGES images in one call");
    if (!rc) {
        std::lock_guard<std::mutex> lk(nd.mu);
        const hipError_t e = hipSetDevice(ctx->device);
        rc = e != hipSuccess ? hip_fail(e, "hipSetDevice") : render_noalloc(ctx, nd, sc, d, (hipStream_t)stream);
    }
    if (!rc) rc = mark_scene_use(ctx, sc, (hipStream_t)stream);
    if (!rc) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->renders += 1;
    }
    release_scene(sc);
    return rc;
}
