// Serving loop with continuous batching (render requests from many producers).
//
// Worker threads, each owning a device stream (default priority) and its own
// working memory, repeatedly: take the oldest pending request once its memory
// estimate fits the budget next to the requests in flight, merge later pending
// requests of the same scene (FIFO, up to max_batch_images images and 8 image
// sizes), stage the batch's viewmats and poses contiguously, render the batch
// through the same pipeline as gsr_render, wait for the stream, and complete
// the batch's tickets.  Requests arriving while batches run are picked up by
// the next worker that becomes free, so batches overlap on the device and new
// work never waits for a whole queue to drain.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "gsr_runtime.h"

#define GSR_EXPORT extern "C" __attribute__((visibility("default")))

using namespace gsr;

namespace {

int64_t now_us()
{
    return std::chrono::duration_cast<std::chrono::microseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket = 0;
    gsr_render_desc desc{};
    std::vector<gsr_camera> cams;
    gsr_observation obs{};
    SceneRes* scene = nullptr;
    int n_images = 0;
    int64_t bytes = 0;          // working memory while rendering: min(all images, one memory chunk)
    int64_t image_bytes = 0;    // largest single-image estimate
    gsr_req_info info{};
    bool done = false;
};

}  // namespace

struct gsr_server {
    gsr_ctx* ctx = nullptr;
    gsr_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_work;   // pending work or freed memory
    std::condition_variable cv_done;   // a request completed
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    int64_t next_batch = 1;
    int64_t in_flight_bytes = 0, in_flight_bytes_max = 0;
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, images = 0, batch_requests_sum = 0;
    std::vector<double> latencies;
    bool stopping = false;
    std::vector<std::thread> workers;
};

namespace {

// Working-memory budget of one chunk of a served batch: the context's chunk
// size, never more than the server's whole memory budget.
int64_t server_chunk_bytes(const gsr_server* srv)
{
    return std::min<int64_t>(srv->ctx->opt.chunk_bytes, srv->cfg.memory_budget);
}

// Render one batch on the worker's stream; returns the batch status.
int render_batch(gsr_server* srv, Workspace& ws, hipStream_t st, const std::vector<Request*>& batch)
{
    gsr_ctx* ctx = srv->ctx;
    SceneRes* sc = batch.front()->scene;
    const int B = sc->dev.n_bodies;
    RenderJob job;
    size_t vm_floats = 0, pose_floats = 0;
    for (Request* r : batch) {
        vm_floats += (size_t)r->desc.n_cams * r->desc.n_envs * 12;
        pose_floats += (size_t)r->desc.n_envs * B * 7;
    }
    const bool single = batch.size() == 1;
    if (!single) {
        GSR_HIP_TRY(ws.stage_vm.ensure(std::max<size_t>(vm_floats, 1) * 4));
        GSR_HIP_TRY(ws.stage_pose.ensure(std::max<size_t>(pose_floats, 1) * 4));
    }
    size_t vm_at = 0, pose_at = 0;
    for (Request* r : batch) {
        std::vector<ImageInfo> imgs = images_of(&r->desc, ctx->opt.tile_size, B);
        const size_t nvm = (size_t)r->desc.n_cams * r->desc.n_envs * 12;
        const size_t npose = (size_t)r->desc.n_envs * B * 7;
        if (!single) {
            GSR_HIP_TRY(hipMemcpyAsync(ws.stage_vm.as<float>() + vm_at, r->desc.viewmats, nvm * 4,
                                       hipMemcpyDeviceToDevice, st));
            if (npose)
                GSR_HIP_TRY(hipMemcpyAsync(ws.stage_pose.as<float>() + pose_at, r->desc.body_poses, npose * 4,
                                           hipMemcpyDeviceToDevice, st));
            for (ImageInfo& im : imgs) {
                im.vm_off += (uint32_t)vm_at;
                im.pose_off += (uint32_t)pose_at;
            }
        }
        vm_at += nvm;
        pose_at += npose;
        job.imgs.insert(job.imgs.end(), imgs.begin(), imgs.end());
    }
    if (vm_at > 0xFFFFFFFFull || pose_at > 0xFFFFFFFFull) return fail(GSR_E_INVALID, "batch inputs too large");
    if (single) {
        job.viewmats = batch.front()->desc.viewmats;
        job.poses = batch.front()->desc.body_poses;
    } else {
        job.viewmats = ws.stage_vm.as<float>();
        job.poses = ws.stage_pose.as<float>();
    }
    job.viewmat_floats = vm_at;
    job.pose_floats = pose_at;
    job.tune.ts = ctx->opt.tile_size;
    job.tune.batch = ctx->opt.tile_size == 8 ? 64 : 256;
    job.tune.ipt = ctx->opt.images_per_thread;
    job.chunk_bytes = server_chunk_bytes(srv);
    // images of equal size contiguous (one raster segment each)
    std::stable_sort(job.imgs.begin(), job.imgs.end(), [](const ImageInfo& a, const ImageInfo& b) {
        return a.width != b.width ? a.width < b.width : a.height < b.height;
    });
    // batches change composition from one to the next: launched eagerly, not
    // captured; one working set per batch, as the memory admission assumes
    // (the server's own streams already overlap batches)
    int rc = render_job(ctx, ws, sc, job, st, false, false, false);
    if (!rc) rc = mark_scene_use(ctx, sc, st);
    if (!rc) GSR_HIP_TRY(hipStreamSynchronize(st));
    return rc;
}

int distinct_sizes(const std::vector<Request*>& batch, const Request* extra)
{
    std::vector<std::pair<int, int>> s;
    auto add = [&](const Request* r) {
        for (const gsr_camera& c : r->cams) s.emplace_back(c.width, c.height);
    };
    for (const Request* r : batch) add(r);
    if (extra) add(extra);
    std::sort(s.begin(), s.end());
    return (int)(std::unique(s.begin(), s.end()) - s.begin());
}

void worker_main(gsr_server* srv)
{
    (void)hipSetDevice(srv->ctx->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    std::unique_ptr<Workspace> ws(new Workspace());
    for (;;) {
        std::vector<Request*> batch;
        int64_t batch_bytes = 0, batch_id = 0;
        int batch_images = 0;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv_work.wait(lk, [&] {
                if (srv->pending.empty()) return srv->stopping;
                const Request* h = srv->pending.front();
                return srv->in_flight_bytes == 0 || srv->in_flight_bytes + h->bytes <= srv->cfg.memory_budget;
            });
            if (srv->pending.empty()) break;   // stopping and drained
            Request* head = srv->pending.front();
            srv->pending.pop_front();
            batch.push_back(head);
            batch_bytes = head->bytes;
            batch_images = head->n_images;
            const int64_t chunk = server_chunk_bytes(srv);
            int64_t sum_bytes = head->bytes, img_max = head->image_bytes;
            for (auto it = srv->pending.begin(); it != srv->pending.end();) {
                Request* r = *it;
                const int64_t merged = std::min(sum_bytes + r->bytes, std::max(std::max(img_max, r->image_bytes), chunk));
                if (r->scene == head->scene && batch_images + r->n_images <= srv->cfg.max_batch_images &&
                    srv->in_flight_bytes + merged <= srv->cfg.memory_budget && distinct_sizes(batch, r) <= kMaxSegs) {
                    batch.push_back(r);
                    sum_bytes += r->bytes;
                    img_max = std::max(img_max, r->image_bytes);
                    batch_bytes = merged;
                    batch_images += r->n_images;
                    it = srv->pending.erase(it);
                } else {
                    ++it;
                }
            }
            srv->in_flight_bytes += batch_bytes;
            srv->in_flight_bytes_max = std::max(srv->in_flight_bytes_max, srv->in_flight_bytes);
            batch_id = srv->next_batch++;
            const int64_t t = now_us();
            for (Request* r : batch) r->info.t_admit_us = t;
        }
        const int64_t t_start = now_us();
        int rc = st ? render_batch(srv, *ws, st, batch) : fail(GSR_E_DEVICE, "stream creation failed");
        const int64_t t_done = now_us();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->in_flight_bytes -= batch_bytes;
            srv->batches += 1;
            srv->images += batch_images;
            srv->batch_requests_sum += (int64_t)batch.size();
            for (Request* r : batch) {
                r->info.status = rc;
                r->info.batch_id = batch_id;
                r->info.batch_requests = (int)batch.size();
                r->info.batch_images = batch_images;
                r->info.t_start_us = t_start;
                r->info.t_complete_us = t_done;
                r->done = true;
                release_scene(r->scene);
                srv->completed += 1;
                srv->latencies.push_back((double)(t_done - r->info.t_submit_us));
            }
        }
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();
    }
    ws.reset();
    if (st) (void)hipStreamDestroy(st);
}

}  // namespace

GSR_EXPORT int gsr_server_create(gsr_ctx* ctx, const gsr_server_cfg* cfg, gsr_server** out)
{
    if (!ctx || !out) return fail(GSR_E_INVALID, "ctx / out is NULL");
    *out = nullptr;
    gsr_server_cfg c{};
    if (cfg) c = *cfg;
    if (c.n_streams == 0) c.n_streams = 2;
    if (c.max_batch_images == 0) c.max_batch_images = 4096;
    if (c.memory_budget == 0) c.memory_budget = (int64_t)32 << 30;
    if (c.n_streams < 1 || c.n_streams > 8) return fail(GSR_E_INVALID, "n_streams must be in 1..8");
    if (c.max_batch_images < 1) return fail(GSR_E_INVALID, "max_batch_images must be >= 1");
    if (c.memory_budget < ((int64_t)64 << 20)) return fail(GSR_E_INVALID, "memory_budget must be >= 64 MiB");
    gsr_server* srv = new (std::nothrow) gsr_server();
    if (!srv) return fail(GSR_E_OOM, "server allocation failed");
    srv->ctx = ctx;
    srv->cfg = c;
    for (int k = 0; k < c.n_streams; ++k) srv->workers.emplace_back(worker_main, srv);
    *out = srv;
    return GSR_OK;
}

GSR_EXPORT int gsr_submit(gsr_server* srv, const gsr_render_desc* d, uint64_t* ticket)
{
    if (!srv || !d || !ticket) return fail(GSR_E_INVALID, "server / desc / ticket is NULL");
    gsr_ctx* ctx = srv->ctx;
    if (ctx->poisoned) return fail(GSR_E_DEVICE, "context poisoned by an earlier device fault");
    SceneRes* sc = acquire_scene(ctx, d->scene_id);
    if (!sc) return fail(GSR_E_NOT_FOUND, "unknown scene id");
    int rc = validate_desc(ctx, d, sc, true);
    if (rc) {
        release_scene(sc);
        return rc;
    }
    std::unique_ptr<Request> r(new Request());
    r->desc = *d;
    r->cams.assign(d->cams, d->cams + d->n_cams);
    r->desc.cams = r->cams.data();
    if (d->obs) {
        r->obs = *d->obs;
        r->desc.obs = &r->obs;
    }
    r->scene = sc;
    r->n_images = d->n_envs * d->n_cams;
    int64_t all = 0;
    for (const gsr_camera& c : r->cams) {
        const int64_t one = (int64_t)image_bytes_estimate(sc, c.width, c.height, ctx->opt.tile_size);
        all += one * d->n_envs;
        r->image_bytes = std::max(r->image_bytes, one);
    }
    // a render holds one memory chunk of images at a time (at least one
    // image): that is what the request occupies while it runs
    r->bytes = std::min(all, std::max(r->image_bytes, server_chunk_bytes(srv)));
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) {
        release_scene(sc);
        return fail(GSR_E_INVALID, "server is shutting down");
    }
    if (r->image_bytes > srv->cfg.memory_budget || r->n_images > srv->cfg.max_batch_images) {
        srv->rejected += 1;
        release_scene(sc);
        return fail(GSR_E_REJECTED, "request can never fit the server's memory budget or batch size");
    }
    r->ticket = srv->next_ticket++;
    r->info.t_submit_us = now_us();
    r->info.n_images = r->n_images;
    *ticket = r->ticket;
    srv->pending.push_back(r.get());
    srv->reqs[r->ticket] = std::move(r);
    srv->submitted += 1;
    srv->cv_work.notify_one();
    return GSR_OK;
}

GSR_EXPORT int gsr_wait(gsr_server* srv, uint64_t ticket, int64_t timeout_us, gsr_req_info* info)
{
    if (!srv) return fail(GSR_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(GSR_E_NOT_FOUND, "unknown ticket");
    Request* r = it->second.get();
    auto ready = [&] { return r->done; };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fail(GSR_E_TIMEOUT, "request not complete");
    }
    if (info) *info = r->info;
    const int status = r->info.status;
    srv->reqs.erase(it);
    if (status != GSR_OK) return fail(status, "request failed");
    return GSR_OK;
}

GSR_EXPORT int gsr_server_stats(gsr_server* srv, gsr_stats* out)
{
    if (!srv || !out) return fail(GSR_E_INVALID, "server / stats is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->pending = (int64_t)srv->pending.size();
    out->batches = srv->batches;
    out->images = srv->images;
    out->in_flight_bytes = srv->in_flight_bytes;
    out->in_flight_bytes_max = srv->in_flight_bytes_max;
    out->mean_batch_requests = srv->batches ? (double)srv->batch_requests_sum / (double)srv->batches : 0.0;
    if (!srv->latencies.empty()) {
        std::vector<double> v = srv->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const double pos = q * (double)(v.size() - 1);
            const size_t lo = (size_t)pos;
            const size_t hi = std::min(lo + 1, v.size() - 1);
            return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
        };
        double sum = 0.0;
        for (double x : v) sum += x;
        out->latency_p50_us = pct(0.50);
        out->latency_p99_us = pct(0.99);
        out->latency_mean_us = sum / (double)v.size();
        out->latency_max_us = v.back();
    }
    return GSR_OK;
}

GSR_EXPORT int gsr_server_destroy(gsr_server* srv)
{
    if (!srv) return GSR_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (std::thread& t : srv->workers) t.join();
    delete srv;
    return GSR_OK;
}
