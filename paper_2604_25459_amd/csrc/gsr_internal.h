// Internal declarations shared by the HIP kernels and the host runtime of
// libgsr (batched 3D Gaussian Splatting for rigid-body environments).
//
// Every file of the library is compiled with -ffp-contract=off: the binning
// arithmetic (projection, culls, radius, tile rectangle, depth key) is
// specified operation by operation in IEEE binary32 so that sort keys and tile
// lists are reproducible bit for bit.  Kernels that want fused multiply-adds
// (the rasteriser) call fmaf() explicitly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsr.h"

namespace gsr {

constexpr uint32_t kInvalidKey = 0xFFFFFFFFu;  // depth-key slot of a culled Gaussian
constexpr int kMaxShDegree = 3;

// Attribute storage formats of a resident scene.
enum Storage : int { kF32 = 0, kF16 = 1, kBF16 = 2 };

// Per-image description inside one launch (device resident).  Images of one
// launch may come from several render requests: every image carries its own
// input offsets and output pointers.
struct ImageInfo {
    int width, height;
    int tiles_x, tiles_y;
    float fx, fy, cx, cy, near_plane;
    float guard_x, guard_y;   // Jacobian clamp of x/z, y/z: 1.3 * ((0.5 W) / fx), same in y (binary32)
    uint32_t key_tile_base;   // first global tile id of the image in its request (sort keys)
    uint32_t vm_off;          // float offset of the image's world->camera [R | t] in the viewmat array
    uint32_t pose_off;        // float offset of the image's env body poses [B][7] in the pose array
    float bg[3];              // background colour of the image's request
    int attach_body;          // -1: viewmat is world->camera; b: viewmat is body-b->camera
    float* out_rgb;           // first pixel of the image: [H][W][3] or null
    float* out_depth;         // [H][W]
    float* out_alpha;         // [H][W] or null
    uint32_t* out_work;       // [H][W][2] (visited entries, blended Gaussians) or null
    void* out_obs;            // observation epilogue output [H][W][3] (u8 or half) or null
    const float* obs_gain;    // per-image parameters (indexed by obs_idx) or null
    const float* obs_contrast;
    const float* obs_bright;
    int obs_fmt;              // GSR_OBS_U8 / GSR_OBS_F16
    uint32_t obs_idx;         // c * E + e within the image's request
    // LiDAR images (kind 1 angular, 2 heightmap grid, 3 listed rays): width x height rays, range ->
    // out_depth, hit -> out_alpha
    int kind;                 // 0 camera, 1 angular LiDAR, 2 heightmap grid, 3 listed rays
    float az0, az_step;       // kind 1: ray azimuths az0 + (c + 0.5) az_step
    const float* elev;        // kind 1: device [height] beam elevations, ascending; kind 3: [2][height]
                              // smallest, then largest elevation of each band (both ascending)
    float gx0, gy0, gdx, gdy; // kind 2: ray (r, c) starts at (gx0 + (c + 0.5) gdx, gy0 + (r + 0.5) gdy, 0), along -z
    const float* ray_az;      // kind 3: device [height][width] azimuths, ascending within each band
    const float* ray_el;      // kind 3: device [height][width] elevations
    const uint32_t* ray_perm; // kind 3: device [height][width] caller's index of each ray (output position)
    const float* ray_tile_az; // kind 3: device [2][tiles_y][tiles_x] smallest, then largest azimuth of each
                              // ray tile (both ascending along a tile row)
};

// Resident scene, device pointers.
struct SceneDev {
    int64_t n;            // Gaussians
    int64_t n_pad;        // plane stride (n rounded up to 64)
    int degree;           // SH degree 0..3
    int storage;          // Storage
    int n_bodies;
    int sh_chunks;        // 16-byte chunks of SH per Gaussian
    const float4* pos;    // [n] (x, y, z, opacity); means are always float32
    const void* rot;      // F32: float4 quaternion [n]; F16/BF16: uint4 = 8 halves (qw qx qy qz sx sy sz 0) [n]
    const float4* scale;  // F32 only: (sx, sy, sz, 0) [n]
    const void* sh;       // planes [sh_chunks][n_pad] of 16 bytes
    const int* body_off;  // [n_bodies + 1] (int32): [0, off[0]) static, body b = [off[b], off[b+1])
};

// Segment of the chunk that shares one camera slot (uniform resolution).
struct RasterSeg {
    uint32_t first_tile;   // first block id of the segment
    uint32_t first_image;  // first chunk-local image
    uint32_t n_images;
    uint32_t tiles_per_image;
};
constexpr int kMaxSegs = 8;
constexpr int kRect4MaxTiles = 255;

// Streaming store of 16 bytes: non-temporal, for whole cache lines of a
// stream that is read back only after it has left L2 and the Infinity Cache
// (the projection's records, written 1 KB per wave instruction).  Scattered
// or partial-line streams keep ordinary stores, which L2 combines.
__device__ __forceinline__ void store_stream(float4* p, float4 v)
{
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    const f32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(p));
}

// Tile rectangle [x0, x1) x [y0, y1) of entry k in either format.
__device__ __forceinline__ void put_rect(void* a, int rect4, size_t k, uint32_t x0, uint32_t x1, uint32_t y0,
                                         uint32_t y1)
{
    if (rect4) static_cast<uint32_t*>(a)[k] = x0 | (x1 << 8) | (y0 << 16) | (y1 << 24);
    else static_cast<uint2*>(a)[k] = make_uint2(x0 | (x1 << 16), y0 | (y1 << 16));
}
// Raw entry k (the u32 in .x for the packed format), decoded by decode_rect.
__device__ __forceinline__ uint2 raw_rect(const void* a, int rect4, size_t k)
{
    return rect4 ? make_uint2(static_cast<const uint32_t*>(a)[k], 0u) : static_cast<const uint2*>(a)[k];
}
__device__ __forceinline__ void decode_rect(uint2 r, int rect4, uint32_t* x0, uint32_t* x1, uint32_t* y0,
                                            uint32_t* y1)
{
    if (rect4) {
        *x0 = r.x & 0xFFu;
        *x1 = (r.x >> 8) & 0xFFu;
        *y0 = (r.x >> 16) & 0xFFu;
        *y1 = r.x >> 24;
    } else {
        *x0 = r.x & 0xFFFFu;
        *x1 = r.x >> 16;
        *y0 = r.y & 0xFFFFu;
        *y1 = r.y >> 16;
    }
}

// Per-chunk device buffers and sizes handed to the kernels.
struct ChunkDev {
    uint64_t n;                // Gaussians of the scene (dense row length)
    int n_img;
    int t_max;                 // largest tile count of an image in the chunk
    int sort_blocks;           // depth-sort blocks per image (pass 0: ceil(n / kSortItems))
    int tile_blocks;           // tile-pass blocks per image (ceil(n / kTileGauss))
    const ImageInfo* img;      // [n_img]
    float* xform;              // [n_img][n_bodies + 1][16]
    uint32_t* keyz;            // [n_img][n] depth bits or kInvalidKey
    uint2* rect;               // [n_img][n] tile rectangle (format: rect4 below)
    float4* rec;               // [n_img][n][3] raster records ([..][5] for LiDAR)
    uint32_t* sk[2];           // depth-sort keys, ping-pong [n_img][n]
    uint32_t* sv[2];           // depth-sort values (Gaussian ids); sorted result in sv[0]
    uint2* srect;              // [n_img][n] tile rectangle of the j-th depth-ordered Gaussian
    uint32_t* sort_hist;       // [n_img][sort_blocks][512]
    uint32_t* kmm;             // [n_img][kKmmStride]: smallest visible key rounded down to 512, largest
    uint32_t* kblk;            // [n_img][sort_blocks][2] smallest, largest visible key of each pass-0 block
    uint32_t* vis_count;       // [n_img] visible Gaussians V_i
    int32_t* tile_hist;       // [n_img][(tx_max + 1) (ty_max + 1)] 2D difference array of tile counts
    uint32_t* tile_range;      // [n_img][t_max][2] local [start, end)
    uint32_t* pair_count;      // [n_img] P_i
    uint64_t* pair_base;       // [n_img + 2] exclusive prefix of P_i, total pairs, total visible
    uint32_t* pairs;           // [total pairs] Gaussian id per (tile, depth)-sorted entry
    int ty_max;                // largest tile-row count of an image in the chunk
    int tx_max;                // largest tile-column count
    // Rectangle format of rect / srect: 1 = one u32 per entry, bytes (x0, x1, y0,
    // y1), used when every image has at most kRect4MaxTiles tiles per axis; 0 =
    // one uint2 per entry (x0 | x1 << 16, y0 | y1 << 16).
    int rect4;
    uint32_t* row_hist;        // [n_img][tile_blocks][ty_max] per-block row counts, then offsets
    uint32_t* row_range;       // [n_img][ty_max][2] local [start, end) of each tile-row list
    uint32_t* row_count;       // [n_img] R_i (entries of all row lists)
    uint64_t* row_base;        // [n_img + 1] exclusive prefix of R_i
    uint2* rows;               // [total row entries] (Gaussian id, x0 | x1 << 16) per (row, depth)-sorted entry
    uint32_t* err;             // device word of the context: kErr* bits set by a kernel that meets an entry its
                               // inputs cannot contain (checked by the host at every chunk; poisons the context)
    // List capacity of the chunk (entries of `pairs` and `rows`).  k_image_scan
    // compares the chunk's totals with them and sets *ovf; an overflowed chunk
    // writes no lists and is composited by the fallback rasteriser, which
    // filters each tile's list from the depth-ordered Gaussians instead.
    uint64_t cap_pairs, cap_rows;
    uint32_t* ovf;             // device word of the workspace: 1 = this chunk's lists do not fit
    uint32_t* ovf_count;       // device counter of the context: overflowed chunks so far
    unsigned long long* acc;   // device accumulators of the context: visible Gaussians, pairs, row entries
};

// Bits of ChunkDev::err.
constexpr uint32_t kErrListEntry = 1u;    // a tile list held a Gaussian id >= n
constexpr uint32_t kErrSortSlot = 2u;     // a depth-sort rank or offset fell outside its segment
constexpr uint32_t kErrRowEntry = 4u;     // a depth-ordered id >= n reached the tile-row expansion

// Depth sort geometry.
// Words per image of ChunkDev::kmm (smallest and largest visible key).
constexpr int kKmmStride = 2;
constexpr int kSortBlock = 256;
constexpr int kSortIpt = 16;
constexpr int kSortItems = kSortBlock * kSortIpt;   // 4096 items per block
// Tile pass geometry: one wave per block, kTileGauss depth-ordered Gaussians per block.
constexpr int kTileGauss = 4096;
// Level 2 runs one wave per (image, tile row, segment).  Tile-row lists are
// cut into segments only as far as the launch needs to have about
// kLevel2Waves waves, and never into segments shorter than kRowSegEntries:
// every extra segment costs a per-segment count pass over its entries, and
// many short waves crowd out a rasteriser running beside them.
constexpr int kRowSegEntries = 1024;
constexpr int kLevel2Waves = 16384;

// ------------------------------------------------------------ launchers
// All launchers enqueue on `stream` and return hipGetLastError().
hipError_t launch_compose(const SceneDev& s, const ChunkDev& c, const float* viewmats, const float* poses,
                          hipStream_t stream);
hipError_t launch_project(const SceneDev& s, const ChunkDev& c, int ts, float cutoff, int img_per_thread,
                          hipStream_t stream);
hipError_t launch_depth_sort(const SceneDev& s, const ChunkDev& c, hipStream_t stream);
// Tile and tile-row histograms, ranges, image bases (before the host reads the totals).
hipError_t launch_tile_count(const SceneDev& s, const ChunkDev& c, hipStream_t stream);
// LiDAR: projection into the ray grid (keys = centre distance, conservative
// angular tile rectangles, 80-byte whitening and cone records) and per-ray compositing.
hipError_t launch_project_lidar(const SceneDev& s, const ChunkDev& c, int ts, int ipt, hipStream_t stream);

// Stable two-level scatter: depth-ordered Gaussians -> tile-row lists -> tile lists.
// schedule 0: both levels as stable expansions (two slots per lane, ranks
// from per-bucket lane masks); 1: by transposed ranks (a 64 x 64 bit transpose
// gives each bucket lane its items, each item places itself in its buckets).
// Both give identical lists.
// n_seg: segments per tile-row list (seg_off: n_img * ty_max * n_seg * tx_max
// words of scratch when n_seg > 1).
hipError_t launch_tile_scatter(const SceneDev& s, const ChunkDev& c, int schedule, int n_seg, uint32_t* seg_off,
                               hipStream_t stream);
struct RasterParams {
    int ts;                  // tile side: 8, 16 or 32
    int batch;               // records staged in LDS per round
    int persistent;          // 1: persistent workgroups pulling tiles from `counter`
    int count_work;          // 1: images carry out_work (counting instantiation)
    int persistent_blocks;   // workgroups of the persistent launch
    uint32_t* counter;       // device tile counters, one per XCD (persistent launch)
    int n_segs;
    RasterSeg segs[kMaxSegs];
    uint32_t n_blocks;
};
hipError_t launch_raster_lidar(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream);
hipError_t launch_raster(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream);
// Fallback compositing of a chunk whose lists overflowed (a persistent grid
// that exits at once when the chunk's lists fit); counter: kXcds words.
hipError_t launch_raster_fallback(const SceneDev& s, const ChunkDev& c, const RasterParams& p, uint32_t* counter,
                                  hipStream_t stream);

// Scene upload: convert caller float32 attributes to resident storage.
hipError_t launch_scene_convert(int storage, int64_t n, int64_t n_pad, int degree, const float* means,
                                const float* scales, const float* quats, const float* opac, const float* sh,
                                float4* pos, void* rot, float4* scale, void* sh_planes, hipStream_t stream);

// Debug: 64-bit keys of one image from its sorted pairs.
hipError_t launch_debug_keys(const ChunkDev& c, int image, uint64_t n, const uint32_t* pairs, uint64_t n_pairs,
                             uint64_t* keys_out, hipStream_t stream);

// Workgroups of a launch are handed to the chip's 8 XCDs round-robin by
// linear id, and each XCD has its own L2.  xcd_remap renumbers linear id b of
// a G-workgroup launch so that each XCD runs one contiguous range of logical
// ids: neighbouring work (the tiles or blocks of one image) then shares one
// L2 instead of being fetched into all eight.  A bijection of [0, G).
constexpr int kXcds = 8;

__host__ __device__ inline uint32_t xcd_remap(uint32_t b, uint32_t G)
{
    const uint32_t q = G / kXcds, r = G % kXcds, x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace gsr
