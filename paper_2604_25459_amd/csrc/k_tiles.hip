// Tile binning: the last (most significant) digit of the LSD sort of the
// 64-bit (tile, depth) keys.
//
// After the depth sort, every image's visible Gaussians are in ascending
// (depth bits, index) order.  Expanding each Gaussian into its touched tiles
// (row-major inside its rectangle) in that order yields the (tile, depth)
// pairs already sorted on the low 32 key bits; a stable counting sort by tile
// then gives exactly the order of the full 64-bit key sort with ties kept in
// index order.  The expansion is never written out: each kernel re-expands its
// Gaussians in LDS ("load-balanced" over one wave), so memory traffic per pair
// is one 4-byte id write.
//
// Kernels (one wave per block, kTileGauss Gaussians per block):
//   k_tile_hist    per-block tile histogram (LDS atomics)
//   k_tile_scan    per image: tile totals, tile ranges, per-block offsets
//   k_image_scan   pair base of every image in the chunk
//   k_tile_scatter stable scatter of Gaussian ids into tile lists; ranks of
//                  equal tiles inside a 64-pair window come from a ballot match
#include "gsr_internal.h"

namespace gsr {
namespace {

__device__ __forceinline__ uint64_t lanemask_lt64()
{
    const int lane = __lane_id();
    return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// LDS staging of one 64-Gaussian group of a block.
struct Group {
    uint32_t excl[64];   // exclusive prefix of pair counts
    uint32_t x0[64], nx[64], y0[64];
    uint32_t g[64];
};

// Loads Gaussians [jb, jb + 64) n [.., j1) of image i into `grp`; returns the
// number of pairs of the group.
__device__ __forceinline__ uint32_t load_group(const ChunkDev& c, uint64_t n, int i, uint32_t jb, uint32_t j1,
                                               Group& grp)
{
    const int lane = __lane_id();
    const uint32_t j = jb + lane;
    const bool ok = j < j1;
    uint32_t g = 0, cnt = 0, x0 = 0, nx = 1, y0 = 0;
    if (ok) g = c.sv[1][(size_t)i * n + j];
    if (ok && g < n) {      // guard: sorted ids are valid indices by construction
        const uint2 r = c.rect[(size_t)i * n + g];
        x0 = r.x & 0xFFFFu;
        nx = (r.x >> 16) - x0;
        y0 = r.y & 0xFFFFu;
        cnt = nx * ((r.y >> 16) - y0);
    }
    const uint32_t inc = wave_incl_scan(cnt);
    grp.excl[lane] = inc - cnt;
    grp.x0[lane] = x0;
    grp.nx[lane] = nx;
    grp.y0[lane] = y0;
    grp.g[lane] = g;
    return __shfl(inc, 63, 64);
}

// Owner (group slot) and tile of pair p of the current group.
__device__ __forceinline__ uint32_t pair_tile(const Group& grp, uint32_t p, int tiles_x, uint32_t* owner)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (grp.excl[lo + step] <= p) lo += step;     // largest k with excl[k] <= p (counts are >= 1)
    const uint32_t s = p - grp.excl[lo];
    const uint32_t nx = grp.nx[lo];
    uint32_t row = (uint32_t)((float)s * __builtin_amdgcn_rcpf((float)nx));
    if (row * nx > s) --row;
    else if ((row + 1) * nx <= s) ++row;
    const uint32_t col = s - row * nx;
    *owner = (uint32_t)lo;
    return (grp.y0[lo] + row) * (uint32_t)tiles_x + grp.x0[lo] + col;
}

__global__ __launch_bounds__(64) void k_tile_hist(ChunkDev c, uint64_t n)
{
    extern __shared__ uint32_t lds[];
    Group& grp = *reinterpret_cast<Group*>(lds);
    uint32_t* hist = lds + sizeof(Group) / 4;
    const int i = blockIdx.y, b = blockIdx.x, lane = __lane_id();
    const uint32_t V = c.n ? c.vis_count[i] : 0u;
    const uint32_t j0 = (uint32_t)b * kTileGauss;
    if (j0 >= V) return;
    const uint32_t j1 = min(j0 + (uint32_t)kTileGauss, V);
    const ImageInfo im = c.img[i];
    const int T = im.tiles_x * im.tiles_y;
    for (int t = lane; t < T; t += 64) hist[t] = 0;
    __syncthreads();
    for (uint32_t jb = j0; jb < j1; jb += 64) {
        const uint32_t total = load_group(c, n, i, jb, j1, grp);
        __syncthreads();
        for (uint32_t p0 = 0; p0 < total; p0 += 64) {
            const uint32_t p = p0 + lane;
            if (p < total) {
                uint32_t k;
                const uint32_t t = pair_tile(grp, p, im.tiles_x, &k);
                if (t < (uint32_t)T) atomicAdd(&hist[t], 1u);
            }
        }
        __syncthreads();
    }
    uint32_t* out = c.tile_hist + ((size_t)i * c.tile_blocks + b) * c.t_max;
    for (int t = lane; t < T; t += 64) out[t] = hist[t];
}

__device__ __forceinline__ uint32_t block_excl_scan256_t(uint32_t v, uint32_t* total, uint32_t* lds8)
{
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    const uint32_t x = wave_incl_scan(v);
    if (lane == 63) lds8[w] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t s = lds8[k];
        if (k < w) pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// One block of 256 threads per image.
__global__ __launch_bounds__(256) void k_tile_scan(ChunkDev c)
{
    __shared__ uint32_t lds8[8];
    const int i = blockIdx.x, tid = threadIdx.x;
    const uint32_t V = c.n ? c.vis_count[i] : 0u;
    const int nb = (int)((V + kTileGauss - 1) / kTileGauss);
    const ImageInfo im = c.img[i];
    const int T = im.tiles_x * im.tiles_y;
    uint32_t* H = c.tile_hist + (size_t)i * c.tile_blocks * c.t_max;
    uint32_t* R = c.tile_range + (size_t)i * c.t_max * 2;
    uint32_t run = 0;
    for (int t0 = 0; t0 < T; t0 += 256) {
        const int t = t0 + tid;
        uint32_t tot = 0;
        if (t < T)
            for (int b = 0; b < nb; ++b) tot += H[(size_t)b * c.t_max + t];
        uint32_t chunk_total;
        const uint32_t start = run + block_excl_scan256_t(tot, &chunk_total, lds8);
        if (t < T) {
            R[2 * t] = start;
            R[2 * t + 1] = start + tot;
            uint32_t o = start;
            for (int b = 0; b < nb; ++b) {
                const uint32_t v = H[(size_t)b * c.t_max + t];
                H[(size_t)b * c.t_max + t] = o;
                o += v;
            }
        }
        run += chunk_total;
    }
    if (tid == 0) c.pair_count[i] = run;
}

// Single block: pair_base[i] = sum of P over images before i; pair_base[n_img] = total.
__global__ __launch_bounds__(256) void k_image_scan(ChunkDev c)
{
    __shared__ uint64_t part[256];
    const int tid = threadIdx.x;
    const int per = (c.n_img + 255) / 256;
    uint64_t s = 0;
    for (int k = 0; k < per; ++k) {
        const int i = tid * per + k;
        if (i < c.n_img) s += c.pair_count[i];
    }
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        uint64_t run = 0;
        for (int k = 0; k < 256; ++k) {
            const uint64_t v = part[k];
            part[k] = run;
            run += v;
        }
        c.pair_base[c.n_img] = run;
    }
    __syncthreads();
    uint64_t run = part[tid];
    for (int k = 0; k < per; ++k) {
        const int i = tid * per + k;
        if (i < c.n_img) {
            c.pair_base[i] = run;
            run += c.pair_count[i];
        }
    }
}

__global__ __launch_bounds__(64) void k_tile_scatter(ChunkDev c, uint64_t n, int tile_bits)
{
    extern __shared__ uint32_t lds[];
    Group& grp = *reinterpret_cast<Group*>(lds);
    uint32_t* cursor = lds + sizeof(Group) / 4;
    const int i = blockIdx.y, b = blockIdx.x, lane = __lane_id();
    const uint32_t V = c.n ? c.vis_count[i] : 0u;
    const uint32_t j0 = (uint32_t)b * kTileGauss;
    if (j0 >= V) return;
    const uint32_t j1 = min(j0 + (uint32_t)kTileGauss, V);
    const ImageInfo im = c.img[i];
    const int T = im.tiles_x * im.tiles_y;
    const uint32_t* off = c.tile_hist + ((size_t)i * c.tile_blocks + b) * c.t_max;
    for (int t = lane; t < T; t += 64) cursor[t] = off[t];
    uint32_t* out = c.pairs + c.pair_base[i];
    const uint32_t P = c.pair_count[i];
    const uint64_t lt = lanemask_lt64();
    __syncthreads();
    for (uint32_t jb = j0; jb < j1; jb += 64) {
        const uint32_t total = load_group(c, n, i, jb, j1, grp);
        __syncthreads();
        for (uint32_t p0 = 0; p0 < total; p0 += 64) {
            const uint32_t p = p0 + lane;
            bool ok = p < total;
            uint32_t k = 0, t = 0;
            if (ok) t = pair_tile(grp, p, im.tiles_x, &k);
            ok = ok && t < (uint32_t)T;
            uint64_t peers = __ballot(ok);
            for (int bit = 0; bit < tile_bits; ++bit) {
                const bool v = (t >> bit) & 1u;
                const uint64_t m = __ballot(v);
                peers &= v ? m : ~m;
            }
            if (ok) {
                const uint32_t basev = cursor[t];
                const uint32_t pos = basev + (uint32_t)__popcll(peers & lt);
                if (lane == __ffsll((unsigned long long)peers) - 1) cursor[t] = basev + (uint32_t)__popcll(peers);
                if (pos < P) out[pos] = grp.g[k];
            }
        }
        __syncthreads();
    }
}

// Keys of one image: key = (global tile << 32) | depth bits of the Gaussian.
__global__ __launch_bounds__(256) void k_debug_keys(ChunkDev c, int image, uint64_t n, const uint32_t* pairs,
                                                    uint64_t* keys)
{
    const ImageInfo im = c.img[image];
    const int T = im.tiles_x * im.tiles_y;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= T) return;
    const uint32_t* R = c.tile_range + (size_t)image * c.t_max * 2;
    for (uint32_t k = R[2 * t]; k < R[2 * t + 1]; ++k) {
        const uint32_t g = pairs[k];
        keys[k] = ((uint64_t)(im.key_tile_base + (uint32_t)t) << 32) | c.keyz[(size_t)image * n + g];
    }
}

}  // namespace

static size_t tile_lds_bytes(const ChunkDev& c) { return sizeof(Group) + (size_t)c.t_max * 4; }

hipError_t launch_tile_count(const SceneDev& s, const ChunkDev& c, hipStream_t stream)
{
    if (c.n_img == 0) return hipSuccess;
    const uint64_t n = (uint64_t)s.n;
    if (n > 0) {
        hipLaunchKernelGGL(k_tile_hist, dim3((unsigned)c.tile_blocks, (unsigned)c.n_img), dim3(64),
                           tile_lds_bytes(c), stream, c, n);
    }
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)c.n_img), dim3(256), 0, stream, c);
    hipLaunchKernelGGL(k_image_scan, dim3(1), dim3(256), 0, stream, c);
    return hipGetLastError();
}

hipError_t launch_tile_scatter(const SceneDev& s, const ChunkDev& c, hipStream_t stream)
{
    if (c.n_img == 0 || s.n == 0) return hipSuccess;
    int bits = 1;
    while ((1 << bits) < c.t_max) ++bits;
    hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)c.tile_blocks, (unsigned)c.n_img), dim3(64),
                       tile_lds_bytes(c), stream, c, (uint64_t)s.n, bits);
    return hipGetLastError();
}

hipError_t launch_debug_keys(const ChunkDev& c, int image, uint64_t n, const uint32_t* pairs, uint64_t n_pairs,
                             uint64_t* keys_out, hipStream_t stream)
{
    (void)n_pairs;
    hipLaunchKernelGGL(k_debug_keys, dim3((unsigned)((c.t_max + 255) / 256)), dim3(256), 0, stream, c, image, n,
                       pairs, keys_out);
    return hipGetLastError();
}

}  // namespace gsr
