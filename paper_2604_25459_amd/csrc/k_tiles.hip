// Tile binning: the last (most significant) digit of the LSD sort of the
// 64-bit (tile, depth) keys.
//
// After the depth sort, every image's visible Gaussians are in ascending
// (depth bits, index) order.  Expanding each Gaussian into its touched tiles
// in that order yields the (tile, depth) pairs already sorted on the low 32
// key bits; a stable counting sort by tile then gives exactly the order of the
// full 64-bit key sort, ties kept in index order.
//
// The counting sort runs in two stable levels so that every block writes to
// few output streams (a block of depth-consecutive Gaussians touches every
// tile of the image; scattering straight into ~10^3 tile lists leaves as many
// partially written cache lines open per block):
//   level 1  depth-ordered Gaussians -> one list per tile row (a Gaussian
//            appears in each row its rectangle spans), blocks of kTileGauss
//            Gaussians, one output stream per tile row;
//   level 2  one wave per segment of an (image, tile row) list walks it in
//            order and expands each entry into the tiles of that row, one
//            output stream per tile of the row.
// The last depth-sort pass leaves every rectangle in depth order and row-list
// entries carry their x-range, so no stage gathers rectangles by id.
// Expansions are never written out: each kernel re-expands a group of 64
// items at a time, balanced over one wave (two expansion slots per lane).  A
// slot's item is found by marking each item's first slot and taking a prefix
// maximum across the lanes; ranks of equal buckets among the slots come from
// per-bucket lane masks in LDS, and a per-bucket cursor in LDS carries the
// rank across iterations.  Item loads run several groups ahead, so a wave
// waits for its own scattered stores only once per batch of groups.
//
// Kernels:
//   k_tile_hist       tile and tile-row counts as difference arrays (LDS atomics)
//   k_tile_scan       per image: tile ranges, row ranges, per-block row offsets
//   k_image_scan      pair and row-entry bases of every image of the chunk
//   k_row_scatter     level 1
//   k_rowseg_count    level 2, per-segment tile counts of long rows
//   k_rowseg_scan     level 2, first output position of each segment per tile
//   k_rowtile_scatter level 2
#include "gsr_internal.h"
#include "gsr_wave.h"

#include <algorithm>

namespace gsr {
namespace {

// Expansion of one group of 64 items (lane = item, in list order): item k
// covers the buckets first_k .. first_k + cnt_k - 1 and goes, with its two
// payload words, to each of those buckets' lists at the bucket's cursor, items
// in list order (stable).  `store(pos, v0, v1)` writes one placement.  All 64
// lanes must take part.  Slots are expanded 128 at a time, two per lane
// (p0 + lane and p0 + 64 + lane); `occ` holds two 64-bit lane masks per bucket
// (zero between calls), one per half, which collect the bucket's slots: a
// slot's rank is the number of its bucket's slots in lower lanes of its own
// half, plus all of them in the first half when it lies in the second.
struct ExpandLds {
    uint4 item[64];      // (first - excl, v0, v1, 0): slot p of the item holds bucket item.x + p
    uint32_t mark[128];  // first slot of an item in the current 128 slots -> item + 1 (0 elsewhere)
};

template <typename Store>
__device__ __forceinline__ void expand_group(ExpandLds& ex, uint64_t* occ, uint32_t* cursor, uint32_t cnt,
                                             uint32_t first, uint32_t v0, uint32_t v1, uint32_t n_buckets, Store store)
{
    const int lane = __lane_id();
    const uint32_t inc = wave_incl_sum(cnt);
    const uint32_t excl = inc - cnt;
    const uint32_t total = wave_last(inc);
    ex.item[lane] = make_uint4(first - excl, v0, v1, 0u);
    const uint64_t bit = 1ull << lane;
    uint32_t carry = 0;          // owner + 1 of the last slot of the previous iteration
    for (uint32_t p0 = 0; p0 < total; p0 += 128) {
        if (cnt != 0 && excl >= p0 && excl < p0 + 128u) ex.mark[excl - p0] = (uint32_t)lane + 1u;
        wave_lds_sync();
        const uint32_t mka = ex.mark[lane], mkb = ex.mark[64 + lane];
        ex.mark[lane] = 0u;
        ex.mark[64 + lane] = 0u;
        const uint32_t owna = max(wave_incl_max(mka), carry);
        const uint32_t ownb = max(wave_incl_max(mkb), wave_last(owna));
        carry = wave_last(ownb);
        const uint32_t pa = p0 + (uint32_t)lane, pb = pa + 64u;
        bool oka = pa < total && owna != 0u, okb = pb < total && ownb != 0u;
        uint4 ita = make_uint4(0u, 0u, 0u, 0u), itb = ita;
        uint32_t ba = 0, bb = 0;
        if (oka) {
            ita = ex.item[(owna - 1u) & 63u];
            ba = ita.x + pa;
            oka = ba < n_buckets;
        }
        if (okb) {
            itb = ex.item[(ownb - 1u) & 63u];
            bb = itb.x + pb;
            okb = bb < n_buckets;
        }
        if (oka) atomicOr(reinterpret_cast<unsigned long long*>(&occ[2 * ba]), bit);
        if (okb) atomicOr(reinterpret_cast<unsigned long long*>(&occ[2 * bb + 1]), bit);
        wave_lds_sync();
        // every read precedes the cursor and mask updates below (LDS requests
        // of one wave are served in order)
        uint64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
        uint32_t basea = 0, baseb = 0;
        if (oka) {
            a0 = occ[2 * ba];
            a1 = occ[2 * ba + 1];
            basea = cursor[ba];
        }
        if (okb) {
            b0 = occ[2 * bb];
            b1 = occ[2 * bb + 1];
            baseb = cursor[bb];
        }
        if (oka) {
            const uint32_t below = lanes_below(a0);
            if (below == 0u) {          // the bucket's first slot advances its cursor and clears its masks
                cursor[ba] = basea + (uint32_t)(__popcll(a0) + __popcll(a1));
                occ[2 * ba] = 0ull;
                occ[2 * ba + 1] = 0ull;
            }
            store(basea + below, ita.y, ita.z);
        }
        if (okb) {
            const uint32_t below = lanes_below(b1);
            if (b0 == 0ull && below == 0u) {
                cursor[bb] = baseb + (uint32_t)__popcll(b1);
                occ[2 * bb + 1] = 0ull;
            }
            store(baseb + (uint32_t)__popcll(b0) + below, itb.y, itb.z);
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ counts
// A Gaussian adds one to every tile of its rectangle [x0, x1) x [y0, y1) and
// one to every tile row [y0, y1).  Both are written as difference arrays --
// +1 at (x0, y0) and (x1, y1), -1 at (x1, y0) and (x0, y1); +1 at y0, -1 at
// y1 -- and summed up by prefix sums in k_tile_scan: four atomics per
// Gaussian instead of one per (tile, Gaussian) pair.  Tile counts are only
// needed per image (the tile lists are written by rows), so the block's 2D
// differences are added into the image's array; row counts are needed per
// block (level-1 offsets), so each block writes its own.
__global__ __launch_bounds__(256) void k_zero_diff(int32_t* __restrict__ d, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) d[i] = 0;
}

__global__ __launch_bounds__(256) void k_tile_hist(ChunkDev c, uint64_t n)
{
    extern __shared__ int32_t lds_i[];
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), b = (int)(L - (uint32_t)i * gridDim.x), tid = threadIdx.x;
    const uint32_t V = c.n ? c.vis_count[i] : 0u;
    const uint32_t j0 = (uint32_t)b * kTileGauss;
    if (j0 >= V) return;                // block-uniform
    const uint32_t j1 = min(j0 + (uint32_t)kTileGauss, V);
    const ImageInfo im = c.img[i];
    const int P1 = im.tiles_x + 1, Q1 = im.tiles_y + 1;
    const int D = P1 * Q1;
    int32_t* diff = lds_i;              // [Q1][P1]
    int32_t* rdiff = lds_i + D;         // [Q1]
    for (int t = tid; t < D; t += 256) diff[t] = 0;
    for (int y = tid; y < Q1; y += 256) rdiff[y] = 0;
    __syncthreads();
    // all of the thread's rectangle loads first, then the LDS atomics
    constexpr int kPer = kTileGauss / 256;
    uint2 rr[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t j = j0 + (uint32_t)tid + 256u * (uint32_t)q;
        rr[q] = j < j1 ? raw_rect(c.srect, c.rect4, (size_t)i * n + j) : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        uint32_t x0, x1, y0, y1;
        decode_rect(rr[q], c.rect4, &x0, &x1, &y0, &y1);     // an empty rectangle past j1
        if (x1 > x0 && y1 > y0 && x1 <= (uint32_t)im.tiles_x && y1 <= (uint32_t)im.tiles_y) {
            atomicAdd(&diff[y0 * P1 + x0], 1);
            atomicAdd(&diff[y0 * P1 + x1], -1);
            atomicAdd(&diff[y1 * P1 + x0], -1);
            atomicAdd(&diff[y1 * P1 + x1], 1);
            atomicAdd(&rdiff[y0], 1);
            atomicAdd(&rdiff[y1], -1);
        }
    }
    __syncthreads();
    int32_t* gd = c.tile_hist + (size_t)i * (size_t)(c.tx_max + 1) * (c.ty_max + 1);
    for (int t = tid; t < D; t += 256) {
        const int32_t v = diff[t];
        if (v) atomicAdd(&gd[t], v);
    }
    if (tid == 0) {                     // per-block row counts: prefix of the row differences
        uint32_t* rout = c.row_hist + ((size_t)i * c.tile_blocks + b) * c.ty_max;
        int32_t run = 0;
        for (int y = 0; y < im.tiles_y; ++y) {
            run += rdiff[y];
            rout[y] = (uint32_t)run;
        }
    }
}

__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* total, uint32_t* lds8)
{
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    const uint32_t x = wave_incl_sum(v);
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

// Per image (256 threads): bins summed over the image's blocks, exclusive scan
// over bins -> [start, end) per bin; optionally per-block offsets in place.
__device__ uint32_t scan_bins(uint32_t* H, int nb, int stride, int nbins, uint32_t* range, bool block_offsets,
                              uint32_t* lds8)
{
    const int tid = threadIdx.x;
    uint32_t run = 0;
    for (int t0 = 0; t0 < nbins; t0 += 256) {
        const int t = t0 + tid;
        uint32_t tot = 0;
        if (t < nbins)
            for (int b = 0; b < nb; ++b) tot += H[(size_t)b * stride + t];
        uint32_t chunk_total;
        const uint32_t start = run + block_excl_scan256(tot, &chunk_total, lds8);
        if (t < nbins) {
            range[2 * t] = start;
            range[2 * t + 1] = start + tot;
            if (block_offsets) {
                // 16 blocks at a time: a group's loads all complete (one
                // wait) before its stores
                uint32_t o = start;
                for (int b0 = 0; b0 < nb; b0 += 16) {
                    uint32_t v[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q) v[q] = b0 + q < nb ? H[(size_t)(b0 + q) * stride + t] : 0u;
                    __builtin_amdgcn_s_waitcnt(0x0F70);     // vmcnt(0)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        if (b0 + q < nb) H[(size_t)(b0 + q) * stride + t] = o;
                        o += v[q];
                    }
                }
            }
        }
        run += chunk_total;
    }
    return run;
}

__global__ __launch_bounds__(256) void k_tile_scan(ChunkDev c)
{
    __shared__ uint32_t lds8[8];
    const int i = blockIdx.x;
    const uint32_t V = c.n ? c.vis_count[i] : 0u;
    const int nb = (int)((V + kTileGauss - 1) / kTileGauss);
    const ImageInfo im = c.img[i];
    const int TX = im.tiles_x, TY = im.tiles_y, P1 = TX + 1;
    // 2D prefix of the image's difference array (rows, then columns) gives
    // the tile counts, in place; then the tile ranges by a scan in tile order
    int32_t* gd = c.tile_hist + (size_t)i * (size_t)(c.tx_max + 1) * (c.ty_max + 1);
    for (int y = threadIdx.x; y < TY; y += 256) {
        int32_t run = 0;
        for (int x = 0; x < TX; ++x) {
            run += gd[y * P1 + x];
            gd[y * P1 + x] = run;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < TX; x += 256) {
        int32_t run = 0;
        for (int y = 0; y < TY; ++y) {
            run += gd[y * P1 + x];
            gd[y * P1 + x] = run;
        }
    }
    __syncthreads();
    uint32_t* range = c.tile_range + (size_t)i * c.t_max * 2;
    uint32_t P = 0;
    for (int t0 = 0; t0 < TX * TY; t0 += 256) {
        const int t = t0 + threadIdx.x;
        const uint32_t cnt = t < TX * TY ? (uint32_t)gd[(t / TX) * P1 + (t % TX)] : 0u;
        uint32_t chunk_total;
        const uint32_t start = P + block_excl_scan256(cnt, &chunk_total, lds8);
        if (t < TX * TY) {
            range[2 * t] = start;
            range[2 * t + 1] = start + cnt;
        }
        P += chunk_total;
    }
    const uint32_t Rn = scan_bins(c.row_hist + (size_t)i * c.tile_blocks * c.ty_max, nb, c.ty_max, im.tiles_y,
                                  c.row_range + (size_t)i * c.ty_max * 2, true, lds8);
    if (threadIdx.x == 0) {
        c.pair_count[i] = P;
        c.row_count[i] = Rn;
    }
}

// Single block: exclusive prefixes of P_i and R_i over the chunk's images;
// pair_base[n_img] = total pairs, row_base[n_img] = total row entries,
// pair_base[n_img + 1] = total visible Gaussians of the chunk.
__global__ __launch_bounds__(256) void k_image_scan(ChunkDev c)
{
    __shared__ uint64_t part[3][256];
    const int tid = threadIdx.x;
    const int per = (c.n_img + 255) / 256;
    uint64_t sp = 0, sr = 0, sv = 0;
    for (int k = 0; k < per; ++k) {
        const int i = tid * per + k;
        if (i < c.n_img) {
            sp += c.pair_count[i];
            sr += c.row_count[i];
            sv += c.n ? c.vis_count[i] : 0u;
        }
    }
    part[0][tid] = sp;
    part[1][tid] = sr;
    part[2][tid] = sv;
    __syncthreads();
    __shared__ uint64_t tot[3];
    if (tid < 3) {
        uint64_t run = 0;
        for (int k = 0; k < 256; ++k) {
            const uint64_t v = part[tid][k];
            part[tid][k] = run;
            run += v;
        }
        tot[tid] = run;
        if (tid == 0) c.pair_base[c.n_img] = run;
        else if (tid == 1) c.row_base[c.n_img] = run;
        else c.pair_base[c.n_img + 1] = run;
        atomicAdd(&c.acc[tid == 2 ? 0 : tid + 1], (unsigned long long)run);   // visible, pairs, row entries
    }
    __syncthreads();
    if (tid == 0) {
        const uint32_t over = tot[0] > c.cap_pairs || tot[1] > c.cap_rows ? 1u : 0u;
        *c.ovf = over;
        if (over) atomicAdd(c.ovf_count, 1u);
    }
    uint64_t rp = part[0][tid], rr = part[1][tid];
    for (int k = 0; k < per; ++k) {
        const int i = tid * per + k;
        if (i < c.n_img) {
            c.pair_base[i] = rp;
            c.row_base[i] = rr;
            rp += c.pair_count[i];
            rr += c.row_count[i];
        }
    }
}

// ------------------------------------------------------------------ level 1
// Items are loaded this many groups of 64 ahead (see the header).  Two
// rather than eight: the registers saved raise the transposed-rank kernels'
// occupancy (level 2 from three to six waves per SIMD, with one line buffer
// per bucket), which hides more latency than the deeper prefetch did.
constexpr int kAhead = 2;
// Independent waves per workgroup in the expansion kernels (each wave has its
// own item range and LDS; more waves per CU than one-wave workgroups allow).
constexpr int kWavesPerBlock = 4;

// LDS words of one wave: its ExpandLds, two 64-bit slot masks and a cursor per
// bucket, rounded up to 16 bytes so that every wave's items stay 16-byte
// aligned.
__host__ __device__ constexpr size_t expand_lds_words(int buckets)
{
    return (sizeof(ExpandLds) / 4 + 5 * (size_t)buckets + 3) & ~(size_t)3;
}

__global__ __launch_bounds__(64 * kWavesPerBlock) void k_row_scatter(ChunkDev c, uint64_t n)
{
    if (*c.ovf) return;                 // the chunk's lists do not fit: no lists (fallback raster)
    extern __shared__ uint32_t lds[];
    const int wv = (int)(threadIdx.x >> 6), lane = __lane_id();
    uint32_t* mine = lds + (size_t)wv * expand_lds_words(c.ty_max);
    ExpandLds& ex = *reinterpret_cast<ExpandLds*>(mine);
    uint64_t* occ = reinterpret_cast<uint64_t*>(mine + sizeof(ExpandLds) / 4);
    uint32_t* cursor = mine + sizeof(ExpandLds) / 4 + 4 * (size_t)c.ty_max;
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), b = (int)(L - (uint32_t)i * gridDim.x) * kWavesPerBlock + wv;
    const uint32_t V = c.n ? c.vis_count[i] : 0u;
    const uint32_t j0 = (uint32_t)b * kTileGauss;
    if (b >= c.tile_blocks || j0 >= V) return;     // wave-uniform; the waves of a block never wait on each other
    const uint32_t j1 = min(j0 + (uint32_t)kTileGauss, V);
    const ImageInfo im = c.img[i];
    const uint32_t TY = (uint32_t)im.tiles_y;
    const uint32_t* off = c.row_hist + ((size_t)i * c.tile_blocks + b) * c.ty_max;
    for (uint32_t y = lane; y < TY; y += 64) {
        cursor[y] = off[y];
        occ[2 * y] = 0ull;
        occ[2 * y + 1] = 0ull;
    }
    ex.mark[lane] = 0u;
    ex.mark[64 + lane] = 0u;
    uint2* out = c.rows + c.row_base[i];
    const uint32_t Rn = c.row_count[i];
    const size_t seg = (size_t)i * n;
    uint32_t gn[kAhead];
    uint2 rn[kAhead];
    auto load = [&](uint32_t jb) {
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            const uint32_t j = jb + 64u * w + (uint32_t)lane;
            gn[w] = j < j1 ? c.sv[0][seg + j] : 0u;
            rn[w] = j < j1 ? raw_rect(c.srect, c.rect4, seg + j) : make_uint2(0u, 0u);
        }
    };
    load(j0);
    wave_lds_sync();
    for (uint32_t jb = j0; jb < j1; jb += 64u * kAhead) {
        uint32_t gc[kAhead];
        uint2 rc[kAhead];
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            gc[w] = gn[w];
            rc[w] = rn[w];
        }
        if (jb + 64u * kAhead < j1) load(jb + 64u * kAhead);
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            const uint32_t jw = jb + 64u * w;
            if (jw >= j1) break;
            const uint32_t g = gc[w];
            const uint2 r = rc[w];
            uint32_t x0, x1, y0, y1;
            decode_rect(r, c.rect4, &x0, &x1, &y0, &y1);
            const bool inside = jw + (uint32_t)lane < j1;
            if (inside && g >= n) atomicOr(c.err, kErrRowEntry);   // impossible by construction: report it
            const bool okg = inside && g < n && x1 > x0 && y1 > y0;
            expand_group(ex, occ, cursor, okg ? y1 - y0 : 0u, y0, g, x0 | (x1 << 16), TY,
                         [&](uint32_t pos, uint32_t v0, uint32_t v1) {
                             if (pos < Rn) out[pos] = make_uint2(v0, v1);
                         });
        }
    }
}

// ------------------------------------------------------------------ level 2
// A long tile-row list is cut into n_seg consecutive segments, one wave
// each.  k_rowseg_count counts each segment's pairs per tile column (a
// difference array over the columns: +1 at x0, -1 at x1 per entry);
// k_rowseg_scan turns the counts, per tile, into each segment's first output
// position (the tile's range start plus the pairs of the earlier segments),
// so that the segments scatter independently and together keep every tile
// list in row-list order.  With one segment the tile range starts are used
// directly.
__device__ __forceinline__ void segment_of(uint32_t r0, uint32_t r1, int sg, int n_seg, uint32_t* s0, uint32_t* s1)
{
    const uint64_t len = r1 - r0;
    *s0 = r0 + (uint32_t)(len * (uint64_t)sg / (uint64_t)n_seg);
    *s1 = r0 + (uint32_t)(len * (uint64_t)(sg + 1) / (uint64_t)n_seg);
}

__global__ __launch_bounds__(64) void k_rowseg_count(ChunkDev c, int n_seg, uint32_t* __restrict__ seg_off)
{
    if (*c.ovf) return;                 // the chunk's lists do not fit: no lists (fallback raster)
    extern __shared__ int32_t diff[];       // [TX + 1]
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), bx = (int)(L - (uint32_t)i * gridDim.x), lane = __lane_id();
    const int y = bx / n_seg, sg = bx - y * n_seg;
    const ImageInfo im = c.img[i];
    if (y >= im.tiles_y) return;
    const int TX = im.tiles_x;
    for (int x = lane; x <= TX; x += 64) diff[x] = 0;
    __syncthreads();
    const uint32_t* rr = c.row_range + ((size_t)i * c.ty_max + y) * 2;
    uint32_t s0, s1;
    segment_of(rr[0], rr[1], sg, n_seg, &s0, &s1);
    const uint2* list = c.rows + c.row_base[i];
    // eight loads per lane in flight, then their LDS atomics
    for (uint32_t e0 = s0; e0 < s1; e0 += 64u * 8u) {
        uint32_t xr[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t e = e0 + 64u * (uint32_t)q + (uint32_t)lane;
            xr[q] = e < s1 ? list[e].y : 0u;            // past s1: an empty range
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t x0 = min(xr[q] & 0xFFFFu, (uint32_t)TX), x1 = min(xr[q] >> 16, (uint32_t)TX);
            if (x1 > x0) {
                atomicAdd(&diff[x0], 1);
                atomicAdd(&diff[x1], -1);
            }
        }
    }
    __syncthreads();
    uint32_t* out = seg_off + (((size_t)i * c.ty_max + y) * n_seg + sg) * c.tx_max;
    int32_t carry = 0;
    for (int x0 = 0; x0 < TX; x0 += 64) {
        const int x = x0 + lane;
        const int32_t v = x < TX ? diff[x] : 0;
        const int32_t inc = (int32_t)wave_incl_sum((uint32_t)v) + carry;
        if (x < TX) out[x] = (uint32_t)inc;
        carry = (int32_t)wave_last((uint32_t)inc);
    }
}

__global__ __launch_bounds__(64) void k_rowseg_scan(ChunkDev c, int n_seg, uint32_t* __restrict__ seg_off)
{
    if (*c.ovf) return;                 // the chunk's lists do not fit: no lists (fallback raster)
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), y = (int)(L - (uint32_t)i * gridDim.x), lane = __lane_id();
    const ImageInfo im = c.img[i];
    if (y >= im.tiles_y) return;
    const int TX = im.tiles_x;
    const uint32_t* tr = c.tile_range + ((size_t)i * c.t_max + (size_t)y * TX) * 2;
    uint32_t* base = seg_off + ((size_t)i * c.ty_max + y) * n_seg * c.tx_max;
    for (int x = lane; x < TX; x += 64) {
        uint32_t run = tr[2 * x];
        for (int sg = 0; sg < n_seg; ++sg) {
            uint32_t* q = base + (size_t)sg * c.tx_max + x;
            const uint32_t v = *q;
            *q = run;
            run += v;
        }
    }
}

// Block (y * n_seg + sg, i): segment sg of tile row y of image i.
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_rowtile_scatter(ChunkDev c, int n_seg,
                                                                         const uint32_t* __restrict__ seg_off)
{
    if (*c.ovf) return;                 // the chunk's lists do not fit: no lists (fallback raster)
    extern __shared__ uint32_t lds[];
    const int wv = (int)(threadIdx.x >> 6), lane = __lane_id();
    uint32_t* mine = lds + (size_t)wv * expand_lds_words(c.tx_max);
    ExpandLds& ex = *reinterpret_cast<ExpandLds*>(mine);
    uint64_t* occ = reinterpret_cast<uint64_t*>(mine + sizeof(ExpandLds) / 4);
    uint32_t* cursor = mine + sizeof(ExpandLds) / 4 + 4 * (size_t)c.tx_max;
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), bx = (int)(L - (uint32_t)i * gridDim.x) * kWavesPerBlock + wv;
    const int y = bx / n_seg, sg = bx - y * n_seg;
    const ImageInfo im = c.img[i];
    if (y >= im.tiles_y) return;        // wave-uniform; the waves of a block never wait on each other
    const uint32_t TX = (uint32_t)im.tiles_x;
    const uint32_t* rr = c.row_range + ((size_t)i * c.ty_max + y) * 2;
    uint32_t r0, r1;
    segment_of(rr[0], rr[1], sg, n_seg, &r0, &r1);
    if (r0 >= r1) return;
    const uint2* list = c.rows + c.row_base[i];
    if (n_seg == 1) {
        const uint32_t* tr = c.tile_range + ((size_t)i * c.t_max + (size_t)y * TX) * 2;
        for (uint32_t x = lane; x < TX; x += 64) cursor[x] = tr[2 * x];
    } else {
        const uint32_t* so = seg_off + (((size_t)i * c.ty_max + y) * n_seg + sg) * c.tx_max;
        for (uint32_t x = lane; x < TX; x += 64) cursor[x] = so[x];
    }
    for (uint32_t x = lane; x < TX; x += 64) {
        occ[2 * x] = 0ull;
        occ[2 * x + 1] = 0ull;
    }
    ex.mark[lane] = 0u;
    ex.mark[64 + lane] = 0u;
    uint32_t* out = c.pairs + c.pair_base[i];
    const uint32_t P = c.pair_count[i];
    uint2 nx[kAhead];
    auto load = [&](uint32_t eb) {
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            const uint32_t e = eb + 64u * w + (uint32_t)lane;
            nx[w] = e < r1 ? list[e] : make_uint2(0u, 0u);
        }
    };
    load(r0);
    wave_lds_sync();
    for (uint32_t eb = r0; eb < r1; eb += 64u * kAhead) {
        uint2 cur[kAhead];
#pragma unroll
        for (int w = 0; w < kAhead; ++w) cur[w] = nx[w];
        if (eb + 64u * kAhead < r1) load(eb + 64u * kAhead);
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            const uint32_t ew = eb + 64u * w;
            if (ew >= r1) break;
            const uint2 ent = cur[w];
            uint32_t x0 = 0, cnt = 0;
            if (ew + (uint32_t)lane < r1) {
                x0 = ent.y & 0xFFFFu;
                const uint32_t x1 = min(ent.y >> 16, TX);
                cnt = x1 > x0 ? x1 - x0 : 0u;
            }
            expand_group(ex, occ, cursor, cnt, x0, ent.x, 0u, TX,
                         [&](uint32_t pos, uint32_t v0, uint32_t) {
                             if (pos < P) out[pos] = v0;
                         });
        }
    }
}

// ---------------------------------------- levels 1 and 2 by transposed ranks
// Schedule 1 places a group of 64 items (lane = item, in list order) into a
// window of up to 64 buckets (tile rows at level 1, tile columns at level 2)
// without expansion slots or LDS atomics.  Each lane turns its item's bucket
// range into a 64-bit mask over the window; a 64 x 64 bit transpose across the
// lanes (six butterfly stages) leaves in lane b the set of group items in
// bucket b, in list order.  Lane b owns bucket b's cursor.  An item's place in
// bucket b is the cursor plus the number of lower items in b's set (one
// mbcnt), so every bucket list keeps the (depth, index) order of the input:
// the same lists as schedule 0.
//
// The lists leave in whole 128-byte lines.  A group adds a few entries to each
// of tens of lists, so storing entries where they land writes every line in
// many small pieces, spread over the whole pass; each bucket therefore keeps
// the line that holds its cursor in LDS and writes it out once it is full.
// Only lines that a single group fills from end to end go to memory
// directly, and each list's first and last line are written in two parts
// (the neighbouring list owns the rest of such a line).  One line buffer per
// bucket (6 KB per wave for 40 buckets) keeps the LDS below what the
// registers allow (five waves per SIMD): the occupancy these kernels need to
// hide their LDS and cross-lane latencies.

// Value of lane (lane ^ S): DPP within quads (S = 1, 2) and rows (S = 8,
// row_ror:8), LDS-crossbar swizzles within 32 lanes (S = 4, 16), a backward
// permute across the halves (S = 32).
template <int S>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v)
{
    if constexpr (S == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xf, 0xf, false);  // [1,0,3,2]
    if constexpr (S == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xf, 0xf, false);  // [2,3,0,1]
    if constexpr (S == 4) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (4 << 10) | 0x1F);
    if constexpr (S == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xf, 0xf, false);  // row_ror:8
    if constexpr (S == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (16 << 10) | 0x1F);
    return __shfl_xor(v, 32, 64);
}

// One butterfly stage of the transpose for S < 32 (blocks of S bits inside
// each 32-bit word; m32 marks the low block of each pair): the lower lane of
// a pair keeps its low blocks and takes the partner's low blocks moved up,
// the upper lane keeps its high blocks and takes the partner's high blocks
// moved down.  A rotation by S (upper) or 32 - S (lower) moves the partner's
// blocks into place; the wrapped-around bits fall outside the taken mask.
template <int S>
__device__ __forceinline__ void transpose_stage(uint32_t& lo, uint32_t& hi, uint32_t m32, bool upper)
{
    const uint32_t vlo = xor_lane<S>(lo), vhi = xor_lane<S>(hi);
    const uint32_t keep = upper ? ~m32 : m32;
    const uint32_t r = upper ? (uint32_t)S : 32u - (uint32_t)S;
    lo = (lo & keep) | (__builtin_amdgcn_alignbit(vlo, vlo, r) & ~keep);
    hi = (hi & keep) | (__builtin_amdgcn_alignbit(vhi, vhi, r) & ~keep);
}

// Lane x of the result has bit k set iff lane k of the input has bit x set.
__device__ __forceinline__ uint64_t transpose_bits64(uint64_t w)
{
    const int lane = __lane_id();
    uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    {
        // S = 32: the lower lane's high word and the upper lane's low word trade places
        const bool upper = lane & 32;
        const uint32_t got = xor_lane<32>(upper ? lo : hi);
        lo = upper ? got : lo;
        hi = upper ? hi : got;
    }
    transpose_stage<16>(lo, hi, 0x0000FFFFu, lane & 16);
    transpose_stage<8>(lo, hi, 0x00FF00FFu, lane & 8);
    transpose_stage<4>(lo, hi, 0x0F0F0F0Fu, lane & 4);
    transpose_stage<2>(lo, hi, 0x33333333u, lane & 2);
    transpose_stage<1>(lo, hi, 0x55555555u, lane & 1);
    return ((uint64_t)hi << 32) | lo;
}

// Line-buffered lists of one wave's window: `out` the list array (absolute
// positions, none at or past `limit`), `buf` one 128-byte line per bucket in
// LDS (the line that holds the bucket's cursor), `info` a 64-entry LDS table.
template <typename T>
struct LineLists {
    static constexpr uint32_t kLine = 128 / sizeof(T);     // entries per line
    T* out;
    uint32_t limit;
    T* buf;
    uint4* info;
};

// Writes, for each bucket b in `mask` (lane b holds its cursor, first
// position and end), the line holding the cursor: positions in
// [max(line start, first), min(line end, end)).  Eight lanes write a line,
// 16 bytes each, so a round covers eight buckets.
template <typename T>
__device__ __forceinline__ void flush_lines(const LineLists<T>& L, uint64_t mask, uint32_t cur, uint32_t first,
                                            uint32_t end)
{
    constexpr uint32_t LINE = LineLists<T>::kLine, EPL = 16u / sizeof(T);
    const uint32_t lane = (uint32_t)__lane_id(), k = lane / 8u, j = lane % 8u;
    while (mask) {                      // wave-uniform
        uint32_t b = 64u;
#pragma unroll
        for (uint32_t q = 0; q < 8u; ++q) {
            const uint32_t bq = mask ? (uint32_t)__builtin_ctzll(mask) : 64u;
            if (q == k) b = bq;
            mask &= mask - 1ull;
        }
        const int src = b < 64u ? (int)b : (int)lane;
        const uint32_t cb = (uint32_t)__shfl((int)cur, src), fb = (uint32_t)__shfl((int)first, src),
                       eb = (uint32_t)__shfl((int)end, src);
        if (b < 64u) {
            const uint32_t line = cb / LINE;
            const uint32_t p0 = line * LINE + j * EPL;
            const uint4 w = *reinterpret_cast<const uint4*>(L.buf + b * LINE + j * EPL);
            if (p0 >= fb && p0 + EPL <= eb && p0 + EPL <= L.limit) {
                *reinterpret_cast<uint4*>(L.out + p0) = w;          // 16-byte aligned: lines are
            } else {
                const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
                for (uint32_t q = 0; q < EPL; ++q)
                    if (p0 + q >= fb && p0 + q < eb && p0 + q < L.limit) L.out[p0 + q] = e[q];
            }
        }
    }
}

// One group: this lane's item covers buckets [lo, hi) of the window (empty
// when hi <= lo) and is stored as `v`; `cur` and `first` are the cursor and
// first position of bucket `lane`.  An entry goes to its bucket's buffered
// line if it lies there, to memory if it lies in a line the group fills from
// end to end, and otherwise (a new, partial last line) to the line buffer
// once the full buffered lines have left.
template <typename T>
__device__ __forceinline__ void line_group(const LineLists<T>& L, uint32_t& cur, uint32_t first, uint32_t lo,
                                           uint32_t hi, T v)
{
    constexpr uint32_t LINE = LineLists<T>::kLine;
    const int lane = __lane_id();
    const uint64_t below_hi = hi >= 64u ? ~0ull : ((1ull << hi) - 1ull);
    const uint64_t below_lo = lo >= 64u ? ~0ull : ((1ull << lo) - 1ull);
    const uint64_t set = transpose_bits64(below_hi & ~below_lo);
    const uint32_t next = cur + (uint32_t)__popcll(set);
    L.info[lane] = make_uint4((uint32_t)set, (uint32_t)(set >> 32), cur, next);
    const uint64_t done = __ballot(next / LINE > cur / LINE);            // buckets whose buffered line fills
    wave_lds_sync();
    // four buckets' table entries are read before their stores, so the wave
    // waits for the LDS once per four buckets; bit q of `later`: bucket lo + q
    // has an entry in a new partial line
    uint64_t later = 0;
    for (uint32_t b = lo; b < hi; b += 4u) {
        uint4 in[4];
#pragma unroll
        for (uint32_t q = 0; q < 4u; ++q) in[q] = b + q < hi ? L.info[b + q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (uint32_t q = 0; q < 4u; ++q) {
            if (b + q >= hi) break;
            const uint32_t pos =
                in[q].z + __builtin_amdgcn_mbcnt_hi(in[q].y, __builtin_amdgcn_mbcnt_lo(in[q].x, 0u));
            const uint32_t l = pos / LINE;
            if (l == in[q].z / LINE) L.buf[(b + q) * LINE + pos % LINE] = v;
            else if (l < in[q].w / LINE) { if (pos < L.limit) L.out[pos] = v; }
            else later |= 1ull << (b + q - lo);
        }
    }
    if (done != 0ull) {                 // wave-uniform
        wave_lds_sync();
        flush_lines(L, done, cur, first, 0xFFFFFFFFu);
        if (__ballot(later != 0ull) != 0ull) {
            // a wave's LDS requests are served in order: the flush's reads
            // of a line precede the writes that reuse its buffer
            while (later != 0ull) {
                const uint32_t b = lo + (uint32_t)__builtin_ctzll(later);
                later &= later - 1ull;
                const uint4 in = L.info[b];
                const uint32_t pos = in.z + __builtin_amdgcn_mbcnt_hi(in.y, __builtin_amdgcn_mbcnt_lo(in.x, 0u));
                L.buf[b * LINE + pos % LINE] = v;
            }
        }
    }
    // the next group's table write and barrier order these LDS reads and
    // writes before its own (a wave's LDS requests are served in order)
    cur = next;
}

// The last, partial line of every bucket of the window.
template <typename T>
__device__ __forceinline__ void line_finish(const LineLists<T>& L, uint32_t cur, uint32_t first)
{
    constexpr uint32_t LINE = LineLists<T>::kLine;
    wave_lds_sync();
    flush_lines(L, __ballot(cur % LINE != 0u && cur > first), cur, first, cur);
}

// LDS bytes of one wave of the schedule-1 kernels: the info table and one
// 128-byte line for each of up to 64 buckets.
__host__ __device__ constexpr size_t line_lds_bytes(int buckets) { return 1024 + 128 * (size_t)buckets; }

// Level 1, schedule 1.  Block (gx, i), wave wv: task gx * kWavesPerBlock + wv
// over (kTileGauss block b of image i's depth-ordered Gaussians, window of 64
// tile rows); the block's rows start at its per-block row offsets.
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_row_rank(ChunkDev c, uint64_t n, int n_rw, int nb)
{
    if (*c.ovf) return;                 // the chunk's lists do not fit: no lists (fallback raster)
    extern __shared__ uint4 lds4[];
    const int wv = (int)(threadIdx.x >> 6), lane = __lane_id();
    uint4* mine = lds4 + (size_t)wv * (line_lds_bytes(nb) / 16);
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), task = (int)(L - (uint32_t)i * gridDim.x) * kWavesPerBlock + wv;
    const int b = task / n_rw, rw = task - b * n_rw;
    const uint32_t V = c.n ? c.vis_count[i] : 0u;
    const uint32_t j0 = (uint32_t)b * kTileGauss;
    if (b >= c.tile_blocks || j0 >= V) return;     // wave-uniform; the waves of a block never wait on each other
    const uint32_t j1 = min(j0 + (uint32_t)kTileGauss, V);
    const ImageInfo im = c.img[i];
    const uint32_t TY = (uint32_t)im.tiles_y, TX = (uint32_t)im.tiles_x;
    const uint32_t rbase = (uint32_t)rw * 64u;
    if (rbase >= TY) return;
    const uint32_t row = rbase + (uint32_t)lane;
    // positions are shifted by the image's offset within a line, so that
    // list lines are the array's 128-byte lines
    const uint32_t sh = (uint32_t)(c.row_base[i] % LineLists<uint2>::kLine);
    uint32_t cur = sh + (row < TY ? c.row_hist[((size_t)i * c.tile_blocks + b) * c.ty_max + row] : 0u);
    const uint32_t first = cur;
    const LineLists<uint2> lists{c.rows + (c.row_base[i] - sh), c.row_count[i] + sh, reinterpret_cast<uint2*>(mine + 64),
                                 mine};
    const size_t seg = (size_t)i * n;
    uint32_t gn[kAhead];
    uint2 rn[kAhead];
    auto load = [&](uint32_t jb) {
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            const uint32_t j = jb + 64u * w + (uint32_t)lane;
            gn[w] = j < j1 ? c.sv[0][seg + j] : 0u;
            rn[w] = j < j1 ? raw_rect(c.srect, c.rect4, seg + j) : make_uint2(0u, 0u);
        }
    };
    load(j0);
    for (uint32_t jb = j0; jb < j1; jb += 64u * kAhead) {
        uint32_t gc[kAhead];
        uint2 rc[kAhead];
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            gc[w] = gn[w];
            rc[w] = rn[w];
        }
        if (jb + 64u * kAhead < j1) load(jb + 64u * kAhead);
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            const uint32_t jw = jb + 64u * w;
            if (jw >= j1) break;
            const uint32_t g = gc[w];
            uint32_t x0, x1, y0, y1;
            decode_rect(rc[w], c.rect4, &x0, &x1, &y0, &y1);
            const bool inside = jw + (uint32_t)lane < j1;
            if (inside && g >= n) atomicOr(c.err, kErrRowEntry);   // impossible by construction: report it
            // the rows k_tile_hist counts: a non-empty rectangle inside the image
            const bool okg = inside && g < n && x1 > x0 && y1 > y0 && x1 <= TX && y1 <= TY;
            const uint32_t lo = okg ? min(max(y0, rbase) - rbase, 64u) : 0u;
            const uint32_t hi = okg ? min(max(y1, rbase) - rbase, 64u) : 0u;
            line_group(lists, cur, first, lo, hi, make_uint2(g, x0 | (x1 << 16)));
        }
    }
    line_finish(lists, cur, first);
}

// Level 2, schedule 1.  Block (gx, i), wave wv: task gx * kWavesPerBlock + wv
// over ((tile row * n_seg + segment) * n_cc + window of 64 tile columns).
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_rowtile_rank(ChunkDev c, int n_seg, int n_cc,
                                                                      const uint32_t* __restrict__ seg_off, int nb)
{
    if (*c.ovf) return;                 // the chunk's lists do not fit: no lists (fallback raster)
    extern __shared__ uint4 lds4[];
    const int wv = (int)(threadIdx.x >> 6), lane = __lane_id();
    uint4* mine = lds4 + (size_t)wv * (line_lds_bytes(nb) / 16);
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), task = (int)(L - (uint32_t)i * gridDim.x) * kWavesPerBlock + wv;
    const int cc = task % n_cc, ys = task / n_cc;
    const int y = ys / n_seg, sg = ys - y * n_seg;
    const ImageInfo im = c.img[i];
    const uint32_t TX = (uint32_t)im.tiles_x;
    const uint32_t base = (uint32_t)cc * 64u;
    if (y >= im.tiles_y || base >= TX) return;     // wave-uniform; the waves of a block never wait on each other
    const uint32_t* rr = c.row_range + ((size_t)i * c.ty_max + y) * 2;
    uint32_t r0, r1;
    segment_of(rr[0], rr[1], sg, n_seg, &r0, &r1);
    if (r0 >= r1) return;
    const uint2* list = c.rows + c.row_base[i];
    const uint32_t tx = base + (uint32_t)lane;
    // positions shifted as in level 1: list lines are the array's lines
    const uint32_t sh = (uint32_t)(c.pair_base[i] % LineLists<uint32_t>::kLine);
    uint32_t cur = sh;
    if (tx < TX) {
        const uint32_t* tr = c.tile_range + ((size_t)i * c.t_max + (size_t)y * TX + tx) * 2;
        cur += n_seg == 1 ? tr[0] : seg_off[(((size_t)i * c.ty_max + y) * n_seg + sg) * c.tx_max + tx];
    }
    const uint32_t first = cur;
    const LineLists<uint32_t> lists{c.pairs + (c.pair_base[i] - sh), c.pair_count[i] + sh,
                                    reinterpret_cast<uint32_t*>(mine + 64), mine};
    uint2 nx[kAhead];
    auto load = [&](uint32_t eb) {
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            const uint32_t e = eb + 64u * w + (uint32_t)lane;
            nx[w] = e < r1 ? list[e] : make_uint2(0u, 0u);     // past r1: an empty range
        }
    };
    load(r0);
    for (uint32_t eb = r0; eb < r1; eb += 64u * kAhead) {
        uint2 en[kAhead];
#pragma unroll
        for (int w = 0; w < kAhead; ++w) en[w] = nx[w];
        if (eb + 64u * kAhead < r1) load(eb + 64u * kAhead);
#pragma unroll
        for (int w = 0; w < kAhead; ++w) {
            if (eb + 64u * w >= r1) break;
            const uint32_t x0 = en[w].y & 0xFFFFu, x1 = min(en[w].y >> 16, TX);
            const uint32_t lo = min(max(x0, base) - base, 64u), hi = min(max(x1, base) - base, 64u);
            line_group(lists, cur, first, lo, hi, en[w].x);
        }
    }
    line_finish(lists, cur, first);
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

hipError_t launch_tile_count(const SceneDev& s, const ChunkDev& c, hipStream_t stream)
{
    if (c.n_img == 0) return hipSuccess;
    const uint64_t n = (uint64_t)s.n;
    const uint64_t nd = (uint64_t)c.n_img * (uint64_t)(c.tx_max + 1) * (uint64_t)(c.ty_max + 1);
    hipLaunchKernelGGL(k_zero_diff, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, stream, c.tile_hist, nd);
    if (n > 0) {
        const size_t lds = (size_t)((c.tx_max + 1) * (c.ty_max + 1) + c.ty_max + 1) * 4;
        hipLaunchKernelGGL(k_tile_hist, dim3((unsigned)c.tile_blocks, (unsigned)c.n_img), dim3(256), lds, stream, c,
                           n);
    }
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)c.n_img), dim3(256), 0, stream, c);
    hipLaunchKernelGGL(k_image_scan, dim3(1), dim3(256), 0, stream, c);
    return hipGetLastError();
}

hipError_t launch_tile_scatter(const SceneDev& s, const ChunkDev& c, int schedule, int n_seg, uint32_t* seg_off,
                               hipStream_t stream)
{
    if (c.n_img == 0 || s.n == 0) return hipSuccess;
    const uint64_t n = (uint64_t)s.n;
    if (schedule == 1) {
        const int n_rw = (c.ty_max + 63) / 64, nb = std::min(c.ty_max, 64);
        const unsigned rb = (unsigned)((c.tile_blocks * n_rw + kWavesPerBlock - 1) / kWavesPerBlock);
        hipLaunchKernelGGL(k_row_rank, dim3(rb, (unsigned)c.n_img), dim3(64 * kWavesPerBlock),
                           kWavesPerBlock * line_lds_bytes(nb), stream, c, n, n_rw, nb);
    } else {
        const unsigned rb = (unsigned)((c.tile_blocks + kWavesPerBlock - 1) / kWavesPerBlock);
        hipLaunchKernelGGL(k_row_scatter, dim3(rb, (unsigned)c.n_img), dim3(64 * kWavesPerBlock),
                           kWavesPerBlock * expand_lds_words(c.ty_max) * 4, stream, c, n);
    }
    if (n_seg < 1 || !seg_off) n_seg = 1;
    const dim3 grid((unsigned)(c.ty_max * n_seg), (unsigned)c.n_img);
    if (n_seg > 1) {
        hipLaunchKernelGGL(k_rowseg_count, grid, dim3(64), (size_t)(c.tx_max + 1) * 4, stream, c, n_seg, seg_off);
        hipLaunchKernelGGL(k_rowseg_scan, dim3((unsigned)c.ty_max, (unsigned)c.n_img), dim3(64), 0, stream, c, n_seg,
                           seg_off);
    }
    if (schedule == 1) {
        const int n_cc = (c.tx_max + 63) / 64;
        const unsigned tb = (unsigned)((c.ty_max * n_seg * n_cc + kWavesPerBlock - 1) / kWavesPerBlock);
        const int nb = std::min(c.tx_max, 64);
        hipLaunchKernelGGL(k_rowtile_rank, dim3(tb, (unsigned)c.n_img), dim3(64 * kWavesPerBlock),
                           kWavesPerBlock * line_lds_bytes(nb), stream, c, n_seg, n_cc, (const uint32_t*)seg_off, nb);
    } else {
        const unsigned tb = (unsigned)((c.ty_max * n_seg + kWavesPerBlock - 1) / kWavesPerBlock);
        hipLaunchKernelGGL(k_rowtile_scatter, dim3(tb, (unsigned)c.n_img), dim3(64 * kWavesPerBlock),
                           kWavesPerBlock * expand_lds_words(c.tx_max) * 4, stream, c, n_seg,
                           (const uint32_t*)seg_off);
    }
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
