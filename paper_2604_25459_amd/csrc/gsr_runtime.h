// Host runtime internals shared by the C ABI (gsr_api.cpp) and the serving
// loop (gsr_server.cpp): contexts, resident scenes, working-memory pools and
// the launch sequence of the batched renderer.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gsr.h"
#include "gsr_internal.h"

namespace gsr {

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define GSR_HIP_TRY(expr)                                       \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return ::gsr::hip_fail(_e, #expr); \
    } while (0)

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need);
    void release();
    template <class T>
    T* as() const
    {
        return static_cast<T*>(p);
    }
};

struct SceneRes {
    SceneDev dev{};
    uint64_t uid = 0;                 // process-wide, never reused: identifies the scene in captured graphs
    DevBuf pos, rot, scale, sh, body_off;
    int64_t bytes = 0;
    hipEvent_t last_use = nullptr;   // recorded after the last render that used the scene
    bool used = false;
    std::atomic<int> in_calls{0};     // render calls currently enqueuing work on this scene
    ~SceneRes();
};

// HIP events bracketing the pipeline stages of one chunk (profile option).
struct StageEvents {
    hipEvent_t e[6] = {};
};

// Launch parameters of one shape class (none of them changes a pixel).
struct Tuning {
    int ts = 16;            // tile side
    int batch = 64;         // raster LDS batch
    int ipt = 4;            // images per projection thread
    int persistent = 0;     // persistent raster workgroups
    int chunk_images = 0;   // images per memory chunk (0 = from the memory budget)
    int bin = 1;            // tile-list schedule: 0 stable expansion, 1 transposed ranks
    float ms = 0.0f;        // measured step time when tuned
};

// Captured launch sequence of one pipeline stage of one chunk.
struct StageGraph {
    std::vector<uint64_t> key;
    uint64_t scene_uid = 0;          // scene whose buffers the captured launches read
    hipGraphExec_t exec = nullptr;
};

// Working memory of one render call at a time.
struct Workspace {
    DevBuf img, xform, keyz, rect, srect, rec, sk0, sk1, sv0, sv1, sort_hist, kmm, vis_count, tile_hist, tile_range,
        pair_count, pair_base, pairs, row_hist, row_range, row_count, row_base, rows, debug, stage_vm, stage_pose,
        stage_elev, seg_off;
    uint64_t* h_total = nullptr;   // pinned: [0] pairs, [1] row entries, [2] visible Gaussians of the current chunk,
                                   // [3] low word: the context's device consistency bits
    ImageInfo* h_img = nullptr;    // pinned staging for image descriptions
    size_t h_img_cap = 0;
    float* h_elev = nullptr;       // pinned staging for LiDAR beam elevations
    size_t h_elev_cap = 0;
    hipEvent_t ev_total = nullptr, ev_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool used = false;      // ev_done has been recorded at least once
    bool in_call = false;   // owned by a render call right now
    DevBuf counter;         // persistent raster tile counter
    hipStream_t capture_stream = nullptr;          // graphs are captured here, launched on the chunk's stream
    std::map<std::pair<int, int>, StageGraph> graphs;   // (chunk index, stage) -> executable graph
    std::vector<uint64_t> dead_scenes;   // uids of scenes destroyed while this workspace was in a call
    // Drops every captured graph (here and in the twin) that reads scene `uid`.
    void drop_graphs_of(uint64_t uid);
    // Second half of a two-stream render: odd chunks run on `side` in `twin`'s
    // buffers, so one chunk's binning overlaps the previous chunk's raster.
    std::unique_ptr<Workspace> twin;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // Fixed workspace: every buffer points into memory the workspace does not
    // own (never grown or freed); the tile lists of a chunk are carved from
    // [list_base, list_base + list_bytes), and a chunk whose lists do not fit
    // fails with GSR_E_OVERFLOW before its lists are written.
    bool fixed = false;
    char* list_base = nullptr;
    size_t list_bytes = 0;
    // Asynchronous lists: after a synchronous render has sized the list buffers
    // for a job shape (plan_key), renders of the same shape enqueue every
    // chunk without reading its totals; the device flags a chunk whose lists
    // would not fit (ovf) and composites it by the fallback rasteriser.
    DevBuf ovf, counter2;                 // overflow word of the running chunk; fallback raster counters
    std::vector<uint64_t> plan_key;       // job shape the list buffers were last sized for (empty: none)
    std::vector<int> nseg_hint;           // level-2 segments per tile-row list, per chunk index, of that render
    hipEvent_t ev_staged = nullptr;       // the image descriptions staged in h_img have been copied
    ~Workspace();
};

// Per-chunk buffers of a workspace and their sizes for a plan.
struct WorkspaceSizes {
    struct Item {
        DevBuf Workspace::*buf;
        size_t bytes;
    } b[24];
    int count;
};

enum class Mode { kRender, kBins, kProject };

struct ChunkPlan {
    int chunk;          // images per chunk
    int t_max;          // max tiles of any image
    int tx_max, ty_max; // max tile columns / rows of any image
    int sort_blocks, tile_blocks;
};

// Debug stop of a render sequence: the job ends after the chunk that holds
// image `image`, and reports where that chunk's buffers are.
struct DebugStop {
    int image = -1;
    Workspace* ws = nullptr;   // working set of that chunk (the context's or its twin)
    int i0 = 0, n_img = 0;     // the chunk's first image and image count
    ChunkPlan plan{};
    uint64_t pairs = 0;        // the chunk's pair total
};

// Images of one launch sequence (possibly from several requests), grouped so
// that images of equal size are contiguous.
struct RenderJob {
    std::vector<ImageInfo> imgs;
    const float* viewmats = nullptr;   // base of ImageInfo::vm_off
    const float* poses = nullptr;      // base of ImageInfo::pose_off
    size_t viewmat_floats = 0;         // extent of the arrays above (staged into the workspace)
    size_t pose_floats = 0;
    Tuning tune;
    bool lidar = false;                // LiDAR ray grids instead of camera images
    int64_t chunk_bytes = 0;           // working-memory budget of one chunk (0: the context's option)
    Mode mode = Mode::kRender;         // kBins: every chunk stops after its tile lists (no raster)
    DebugStop* stop = nullptr;         // optional debug stop (see DebugStop)
};

// Validated per-request image list of a render descriptor (camera-slot-major).
std::vector<ImageInfo> images_of(const gsr_render_desc* d, int ts, int n_bodies);
// The same list written into out[E * C].
void fill_images(const gsr_render_desc* d, int ts, int n_bodies, ImageInfo* out);
int validate_desc(const gsr_ctx* ctx, const gsr_render_desc* d, const SceneRes* sc, bool need_outputs);
size_t image_bytes_estimate(const SceneRes* sc, int width, int height, int ts);
ChunkPlan plan_chunks(const gsr_ctx* ctx, const SceneRes* sc, const std::vector<ImageInfo>& imgs, bool plain,
                      int chunk_images = 0, size_t rec_bytes = 48, int64_t chunk_bytes = 0);
// Shape-class key of a render descriptor (scene, envs, camera sizes).
std::string shape_key(const SceneRes* sc, const gsr_render_desc* d);
// Tuning a render of `d` uses: the tuned entry of its shape class or the context defaults.
Tuning tuning_for(gsr_ctx* ctx, const SceneRes* sc, const gsr_render_desc* d);
hipError_t ensure_workspace(Workspace& ws, const SceneRes* sc, const ChunkPlan& p, size_t n_images_total,
                            size_t rec_bytes = 48);
WorkspaceSizes workspace_sizes(const SceneRes* sc, const ChunkPlan& p, size_t n_images_total, size_t rec_bytes = 48);

// Enqueue the pipeline of images [i0, i0 + n_img) of `job` on `st` (image
// descriptions already on the device); blocks until the chunk's list totals
// are known.  `pairs_total` receives the chunk's pair count.
int run_chunk(gsr_ctx* ctx, Workspace& ws, SceneRes* sc, const RenderJob& job, const ChunkPlan& plan, int i0,
              int n_img, int chunk_idx, hipStream_t st, Mode mode, bool graph, uint64_t* pairs_total,
              bool async_lists = false);

// Set-up of the allocation-free render path on `device` (the current device):
// resolves the device address of its scratch array and allocates its pinned
// staging, once per device.  Called by gsr_create.
int noalloc_setup(int device);

// Enqueue the whole job on `st` (blocks once per chunk for its pair count);
// `graphs` allows replaying captured stage graphs (batched path only);
// `two_streams` allows running alternate chunks on ws.side in ws.twin (when
// the context's overlap option is on), joined back into `st`.
int render_job(gsr_ctx* ctx, Workspace& ws, SceneRes* sc, const RenderJob& job, hipStream_t st, bool plain,
               bool graphs, bool two_streams);

// Scene lookup that pins the scene against destruction; release_scene unpins.
SceneRes* acquire_scene(gsr_ctx* ctx, uint64_t id);
void release_scene(SceneRes* sc);
// Records that the scene is used by work enqueued on `st` (GSR_E_BUSY on destroy until it completes).
int mark_scene_use(gsr_ctx* ctx, SceneRes* sc, hipStream_t st);
// A workspace no other call owns (caller holds ctx->mu).
Workspace* acquire_workspace_locked(gsr_ctx* ctx, hipStream_t stream);

}  // namespace gsr

struct gsr_ctx {
    int device = 0;
    gsr_options opt{};
    std::mutex mu;                                   // scenes, pool, timers
    std::map<uint64_t, std::unique_ptr<gsr::SceneRes>> scenes;
    uint64_t next_id = 1;
    std::vector<std::unique_ptr<gsr::Workspace>> pool;
    std::vector<gsr::StageEvents> pending;            // recorded, not yet read
    std::vector<hipEvent_t> spare_events;             // read stage events, reused by later renders
    double stage_ms[5] = {0, 0, 0, 0, 0};
    double raster_launches = 0, renders = 0;
    std::atomic<bool> poisoned{false};
    uint32_t* d_err = nullptr;                        // device words: [0] consistency bits (ChunkDev::err), read
                                                      // at every synchronous chunk; [1] overflowed chunks
                                                      // (ChunkDev::ovf_count); from byte 64, three u64
                                                      // accumulators (ChunkDev::acc)
    uint32_t ovf_seen = 0;                            // overflow count the host has acted on
    uint64_t list_cap = 0;                            // tests: list capacity (entries) of asynchronous chunks
    unsigned long long acc_base[3] = {0, 0, 0};       // accumulator values at the last stage-timer reset
    std::map<std::string, gsr::Tuning> tuned;         // shape class -> launch parameters
    int cu_count = 256;
};
