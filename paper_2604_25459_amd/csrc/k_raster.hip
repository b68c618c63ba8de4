// Per-tile front-to-back alpha compositing (3D Gaussian Splatting volume
// rendering, the image model of the paper's batch renderer).
//
// One workgroup per (image, tile) of the whole chunk, images of all camera
// slots in one launch.  The tile's depth-sorted Gaussian list is staged into
// LDS in batches of records (double-buffered: the next batch is fetched into
// registers while the current one is composited).  Per pixel and Gaussian,
// with the conic in whitened form (a1, b1, c1) so that
//     p = log2(o) - (a1 dx + b1 dy)^2 - (c1 dy)^2 = log2(alpha before the clamp)
//     p < log2(1/255)          -> skip
//     alpha = min(0.99, 2^p); T' = T (1 - alpha)
//     T' < 1e-4                -> stop before adding
//     C += rgb alpha T, D += z alpha T, T = T'
//
// Wave-level culling ("ballot" step): for each group of 64 candidates every
// lane takes one Gaussian and bounds p over the wave's pixel-centre rectangle
// from above (p is concave: the maximum is at the mean if it lies inside,
// else on an edge, where the 1D maximiser is clamped).  Gaussians whose bound
// stays below log2(1/255) - kCullMargin cannot reach alpha >= 1/255 at any
// pixel of the block (narrowed to the bounding box of its still-live pixels).
// The same lane writes its Gaussian, re-centred on the 32x32 pixel block that
// holds the wave, into the wave's own LDS slots, packed by its rank among the
// survivors (10 floats each), and the wave walks the survivors two at a time
// (a pair is five 16-byte LDS reads: on this GPU an LDS read costs about the
// same per instruction whatever its width or active lanes, so fewer, wider
// reads are what count).  Each survivor costs five FMAs per pixel:
//     t1 = a1 x + b1 y - s1,  t2 = c1 y - s2,  p = log2(o) - t1^2 - t2^2
// with (x, y) the pixel centre relative to the block centre and (s1, s2) the
// whitened mean.  The block (not the tile or the wave) is the origin so that
// every tile size evaluates the same expression for a pixel and results do
// not depend on the tiling.  kCullMargin absorbs binary32 rounding of the
// per-pixel evaluation, so culling never removes a Gaussian a pixel would
// have accepted.  Blending runs under the mask of the pixels that take the
// Gaussian and takes a short path when none of them stops at it.
//
// Output: rgb = C + T bg, depth = D / (1 - T) (0 where nothing was added),
// optional alpha = 1 - T, optional work counts, and optionally the fused
// observation epilogue (gain, contrast about 0.5, brightness, clamp to
// [0, 1], then bytes or halves) on the colour before it leaves registers.
#include "gsr_internal.h"
#include "gsr_wave.h"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace gsr {
namespace {

constexpr float kLogAlphaMin = -7.99435343685886f;   // log2(1/255)
constexpr float kCullMargin = 0.05f;                  // in log2(alpha) units
// x coordinate given to a pixel once it has stopped (or lies outside the
// image): t1 overflows to infinity there for every Gaussian (a1 > 0), so p is
// -inf and the pixel never takes another Gaussian; no separate liveness flag
// is needed in the per-Gaussian loop.
constexpr float kDead = 1.0e30f;
// log2(0.99) less a little: a Gaussian whose log2(opacity) is at most this
// never reaches alpha = 0.99, so its blends skip the clamp.
constexpr float kLog2ClampFree = -0.0145f;
constexpr float kDeadTest = 1.0e29f;

// Pixel layout: TS <= 16: one pixel per thread, waves own 8x8 blocks.
// TS == 32: 256 threads x 4 pixels, wave w owns rows [8w, 8w + 8) (32 x 8).
template <int TS>
struct Layout {
    static constexpr int kThreads = TS <= 16 ? TS * TS : 256;
    static constexpr int kWaves = kThreads / 64;
    static constexpr int kPpt = TS <= 16 ? 1 : 4;
    static constexpr int kWaveW = TS <= 16 ? 8 : 32;
    static constexpr int kWaveH = 8;
    __device__ static void wave_origin(int w, int* ox, int* oy)
    {
        if (TS == 8) { *ox = 0; *oy = 0; }
        else if (TS == 16) { *ox = (w & 1) * 8; *oy = (w >> 1) * 8; }
        else { *ox = 0; *oy = w * 8; }
    }
    __device__ static void pixel(int lane, int k, int* x, int* y)
    {
        if (TS <= 16) { *x = lane & 7; *y = lane >> 3; }
        else { *x = lane & 31; *y = (lane >> 5) + 2 * k; }
    }
};

// Upper bound of p = lo - (a1 x + b1 y)^2 - (c1 y)^2 over [X0, X1] x [Y0, Y1]
// (coordinates relative to the mean; a1, c1 > 0).
__device__ __forceinline__ float max_logalpha_rect(float a1, float b1, float c1, float lo, float X0, float X1, float Y0,
                                                   float Y1)
{
    if (X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f) return lo;
    // The quadratic is convex with its minimum at the mean, which lies outside
    // the rectangle, so its minimum over the rectangle lies on an edge that
    // faces the mean: x = X0 if X0 > 0, x = X1 if X1 < 0, and likewise in y.
    // One x edge and one y edge are evaluated; where the mean lies between
    // X0 and X1 (or Y0 and Y1) the edge taken in that axis is just more of
    // the rectangle, which cannot lower the minimum.
    const float Xe = X0 > 0.0f ? X0 : X1;
    const float Ye = Y0 > 0.0f ? Y0 : Y1;
    // On an edge x = X the quadratic is smallest at y = ky X, on y = Y at
    // x = kx Y.  An approximate reciprocal moves the evaluated point along the
    // edge by a relative 1e-7, which lowers the bound by a second-order amount
    // only: the point stays on the edge, so the value is still attained there.
    const float ky = -(a1 * b1) * __builtin_amdgcn_rcpf(fmaf(b1, b1, c1 * c1));
    const float kx = -b1 * __builtin_amdgcn_rcpf(a1);
    float q;
    {
        const float y = fminf(fmaxf(ky * Xe, Y0), Y1);
        const float t = fmaf(a1, Xe, b1 * y), w = c1 * y;
        q = fmaf(t, t, w * w);
    }
    {
        const float x = fminf(fmaxf(kx * Ye, X0), X1);
        const float t = fmaf(a1, x, b1 * Ye), w = c1 * Ye;
        q = fminf(q, fmaf(t, t, w * w));
    }
    return lo - q;
}

// Fallback lists (a chunk whose tile lists do not fit their buffers): each
// tile's list is the subsequence of its image's depth-ordered visible
// Gaussians whose tile rectangle covers the tile -- the same sequence as the
// tile list.  The workgroup filters kRowScan entries at a time into a ring of
// kQueue ids, ahead of the batch being staged.
constexpr int kQueue = 1024;
constexpr int kRowScan = 512;

template <int TS, int kBatch>
struct RasterLds {
    float4 a[2][kBatch], b[2][kBatch], c[2][kBatch];    // staged records: (u, v, a1, b1), (c1, lo, z, r), rgb
    // per wave, the survivors of the current 64 candidates re-centred on the
    // wave's block, packed in candidate order, 10 floats each:
    // a1, b1, c1, lo, -s1, -s2, R, G, B, z (a pair of survivors = five
    // 16-byte words; survivor k starts at float 10 k)
    float4 w[Layout<TS>::kWaves][160];
    uint32_t bright[Layout<TS>::kWaves][64];   // survivor may reach alpha = 0.99
    uint32_t origin[Layout<TS>::kWaves][64];   // candidate index of the survivor (work counts)
    // per wave, whether it still has live pixels after a batch (by batch parity)
    uint32_t live[2][Layout<TS>::kWaves];
};

// Ring of the fallback lists: filtered ids and per-wave counts of one round.
template <int TS>
struct FilterLds {
    uint32_t id[kQueue];
    uint32_t wcount[kRowScan / Layout<TS>::kThreads][Layout<TS>::kWaves];
};

// Composites tile `bid` of the chunk (block id in segment order).  FILTER:
// the tile's list is filtered on the fly from the image's depth-ordered
// Gaussians (Q holds the ring); else it is read from the tile lists.
template <int TS, int kBatch, bool COUNT, bool FILTER>
__device__ __forceinline__ void raster_tile(const SceneDev& s, const ChunkDev& c, const RasterParams& p, uint32_t bid,
                                            RasterLds<TS, kBatch>& L_, FilterLds<TS>* Q)
{
    using L = Layout<TS>;
    constexpr int NT = L::kThreads;
    constexpr int PPT = L::kPpt;
    constexpr int PER_THREAD = (kBatch + NT - 1) / NT;     // records each thread stages per batch
    static_assert(kBatch % 64 == 0, "batch must be a multiple of 64");
    auto& sA = L_.a;
    auto& sB = L_.b;
    auto& sC = L_.c;

    int sgi = 0;
#pragma unroll
    for (int k = 1; k < kMaxSegs; ++k)
        if (k < p.n_segs && bid >= p.segs[k].first_tile) sgi = k;
    const RasterSeg seg = p.segs[sgi];
    const uint32_t rel = bid - seg.first_tile;
    const uint32_t io = rel / seg.tiles_per_image;
    const uint32_t t = rel - io * seg.tiles_per_image;
    const int i = (int)(seg.first_image + io);
    const ImageInfo im = c.img[i];
    const int tx = (int)(t % (uint32_t)im.tiles_x);
    const int ty = (int)(t / (uint32_t)im.tiles_x);

    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = __lane_id();
    int ox, oy;
    L::wave_origin(w, &ox, &oy);
    float* const Wf = reinterpret_cast<float*>(L_.w[w]);
    // pixel-centre rectangle of the wave's block
    const float wx0 = (float)(tx * TS + ox) + 0.5f;
    const float wx1 = wx0 + (float)(L::kWaveW - 1);
    const float wy0 = (float)(ty * TS + oy) + 0.5f;
    const float wy1 = wy0 + (float)(L::kWaveH - 1);
    // centre of the 32x32 pixel block holding the wave: origin of the pixel coordinates
    const float cxo = (float)((tx * TS + ox) & ~31) + 16.0f;
    const float cyo = (float)((ty * TS + oy) & ~31) + 16.0f;

    float xl[PPT], yl[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
    uint32_t stop_at[PPT], blended[PPT];     // work counters (COUNT only)
    int pxi[PPT], pyi[PPT];
    bool any_live = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        int lx, ly;
        L::pixel(lane, k, &lx, &ly);
        pxi[k] = tx * TS + ox + lx;
        pyi[k] = ty * TS + oy + ly;
        const bool inside = pxi[k] < im.width && pyi[k] < im.height;
        xl[k] = inside ? ((float)pxi[k] + 0.5f) - cxo : kDead;
        yl[k] = ((float)pyi[k] + 0.5f) - cyo;
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = D[k] = 0.0f;
        stop_at[k] = 0xFFFFFFFFu;
        blended[k] = 0u;
        any_live = any_live || inside;
    }

    // tile list [start, end) of the pairs, or (FILTER) positions [0, qt) of the
    // filtered list, qt growing as the depth-ordered list is filtered
    uint32_t start = 0, end = 0;
    const uint32_t* list = nullptr;
    constexpr int F = kRowScan / NT;                   // entries per thread per filtering round
    constexpr uint32_t QMASK = (uint32_t)kQueue - 1u;
    static_assert(kBatch + kRowScan <= kQueue, "the ring must hold a batch and a filtering round");
    const uint32_t* sv = nullptr;
    uint32_t vend = 0, scan = 0, qt = 0;
    uint32_t pre_g[F];
    uint2 pre_r[F];
    const size_t iseg = (size_t)i * (size_t)s.n;
    auto load_round = [&]() {
#pragma unroll
        for (int k = 0; k < F; ++k) {
            const uint32_t e = scan + (uint32_t)(k * NT + tid);
            pre_g[k] = e < vend ? sv[iseg + e] : 0u;
            pre_r[k] = e < vend ? raw_rect(c.srect, c.rect4, iseg + e) : make_uint2(0u, 0u);
        }
    };
    if (FILTER) {
        sv = c.sv[0];
        vend = c.vis_count[i];
        load_round();
    } else {
        const uint32_t* R = c.tile_range + ((size_t)i * c.t_max + t) * 2;
        start = R[0];
        end = R[1];
        list = c.pairs + c.pair_base[i];
    }
    // Appends the depth-ordered Gaussians whose rectangle covers this tile to
    // the ring, in order, until qt reaches `target` or the list ends; every
    // round filters the entries loaded the round before and loads the next
    // ones.  Block-uniform trip count (qt and scan are the same in every thread).
    auto refill = [&](uint32_t target) {
        while (qt < target && scan < vend) {
            bool pk[F];
            uint64_t bal[F];
#pragma unroll
            for (int k = 0; k < F; ++k) {
                const uint32_t e = scan + (uint32_t)(k * NT + tid);
                uint32_t x0, x1, y0, y1;
                decode_rect(pre_r[k], c.rect4, &x0, &x1, &y0, &y1);
                pk[k] = e < vend && x0 <= (uint32_t)tx && (uint32_t)tx < x1 && y0 <= (uint32_t)ty && (uint32_t)ty < y1;
                bal[k] = __ballot(pk[k]);
                if (lane == 0) Q->wcount[k][w] = (uint32_t)__popcll(bal[k]);
            }
            __syncthreads();
            // entries in (round k, thread) order, which is the list order
            uint32_t base = qt;
#pragma unroll
            for (int k = 0; k < F; ++k) {
                uint32_t below = 0, tot = 0;
#pragma unroll
                for (int ww = 0; ww < L::kWaves; ++ww) {
                    const uint32_t v = Q->wcount[k][ww];
                    below += ww < w ? v : 0u;
                    tot += v;
                }
                if (pk[k]) Q->id[(base + below + lanes_below(bal[k])) & QMASK] = pre_g[k];
                base += tot;
            }
            qt = base;
            scan += (uint32_t)kRowScan;
            load_round();
            __syncthreads();
        }
    };
    const float4* rec = c.rec + (size_t)i * (size_t)s.n * 3;
    const uint32_t n = (uint32_t)s.n;

    // register staging of the next batch
    float4 ra[PER_THREAD], rb[PER_THREAD], rc[PER_THREAD];
    bool bad_entry = false;
    auto fetch = [&](uint32_t b0) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            const uint32_t slot = (uint32_t)(q * NT + tid);
            const uint32_t e = b0 + slot;
            if (slot < (uint32_t)kBatch && e < (FILTER ? qt : end)) {
                uint32_t g = FILTER ? Q->id[e & QMASK] : list[e];
                if (g >= n) {           // impossible by construction: reported at the end, a valid record read
                    bad_entry = true;
                    g = 0;
                }
                ra[q] = rec[3 * (size_t)g];
                rb[q] = rec[3 * (size_t)g + 1];
                rc[q] = rec[3 * (size_t)g + 2];
            }
        }
    };
    if (FILTER) refill((uint32_t)kBatch);
    if (start < (FILTER ? qt : end)) fetch(start);
    int buf = 0;
    bool wave_live = __ballot(any_live) != 0ull;
    // pixel-centre rectangle still to be shaded (the live pixels' bounding
    // box), recomputed only when the set of live pixels has changed
    float lx0 = wx0, lx1 = wx1, ly0 = wy0, ly1 = wy1;
    uint64_t live_seen = 0;

    for (uint32_t b0 = start; b0 < (FILTER ? qt : end); b0 += kBatch) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            const int slot = q * NT + tid;
            if (slot < kBatch) {
                sA[buf][slot] = ra[q];
                sB[buf][slot] = rb[q];
                sC[buf][slot] = rc[q];
            }
        }
        __syncthreads();
        // every wave's flag from the previous batch is visible after the
        // barrier, so all waves take the same decision
        if (b0 != start) {
            uint32_t any = 0;
#pragma unroll
            for (int ww = 0; ww < L::kWaves; ++ww) any |= L_.live[buf ^ 1][ww];
            if (!any) break;
        }
        // the batch at b0 is staged: its ring slots may be reused
        if (FILTER) refill(b0 + 2u * (uint32_t)kBatch);
        const uint32_t lim = FILTER ? qt : end;
        if (b0 + kBatch < lim) fetch(b0 + kBatch);
        const int cnt = (int)min((uint32_t)kBatch, lim - b0);
        for (int sub = 0; sub < cnt && wave_live; sub += 64) {
            if (PPT == 1) {
                const uint64_t M = __ballot(xl[0] < kDeadTest);  // lane = 8 * row + column
                if (M != live_seen) {
                    live_seen = M;
                    uint64_t cm = M | (M >> 32);
                    cm |= cm >> 16;
                    cm |= cm >> 8;
                    cm &= 0xFFull;
                    lx0 = wx0 + (float)__builtin_ctzll(cm);
                    lx1 = wx0 + (float)(63 - __builtin_clzll(cm));
                    ly0 = wy0 + (float)(__builtin_ctzll(M) >> 3);
                    ly1 = wy0 + (float)((63 - __builtin_clzll(M)) >> 3);
                }
            }
            // ballot: which of these 64 Gaussians can touch the live pixels;
            // survivors are re-centred and packed into the wave's slots
            const int jl = sub + lane;
            // lanes past the batch's end test its last candidate and keep nothing
            const int jc = jl < cnt ? jl : cnt - 1;
            const float4 a = sA[buf][jc], bq = sB[buf][jc];
            const float m = max_logalpha_rect(a.z, a.w, bq.x, bq.y, lx0 - a.x, lx1 - a.x, ly0 - a.y, ly1 - a.y);
            const bool keep = jl < cnt && m >= kLogAlphaMin - kCullMargin;
            const bool bright = keep && bq.y > kLog2ClampFree;
            const uint64_t mask = __ballot(keep);
            const uint64_t bright_lanes = __ballot(bright);
            const uint32_t n_surv = (uint32_t)__popcll(mask);
            const uint32_t r = lanes_below(mask);
            if (keep) {
                const float du = a.x - cxo, dv = a.y - cyo;
                const float s1 = fmaf(a.z, du, a.w * dv), s2 = bq.x * dv;
                const float4 col = sC[buf][jl];
                float2* d = reinterpret_cast<float2*>(Wf + 10u * r);     // 8-byte aligned
                d[0] = make_float2(a.z, a.w);
                d[1] = make_float2(bq.x, bq.y);
                d[2] = make_float2(-s1, -s2);
                d[3] = make_float2(col.x, col.y);
                d[4] = make_float2(col.z, bq.z);
                if (COUNT) L_.origin[w][r] = (uint32_t)jl;
            }
            // bit k: survivor k may reach alpha = 0.99 (only those pay for the
            // clamp); bright survivors are rare, so the packed mask is built
            // only when the batch has one
            uint64_t clampmask = 0;
            if (bright_lanes != 0ull) {
                if (keep) L_.bright[w][r] = bright ? 1u : 0u;
                wave_lds_sync();
                clampmask = __ballot((uint32_t)lane < n_surv && L_.bright[w][lane] != 0u);
            }
            wave_lds_sync();
            // one survivor: a1, b1, c1, -s1 in q0; -s2, lo, z; colour
            auto shade = [&](const float4 q0, float ms2, float lo, float z, float cr, float cg, float cb,
                             uint32_t k_surv) {
                float pw[PPT];
                bool anyt = false;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const float t1 = fmaf(q0.x, xl[k], fmaf(q0.y, yl[k], q0.w));
                    const float t2 = fmaf(q0.z, yl[k], ms2);
                    pw[k] = fmaf(-t1, t1, fmaf(-t2, t2, lo));
                    anyt = anyt || pw[k] >= kLogAlphaMin;
                }
                if (__ballot(anyt) == 0ull) return;        // no live pixel of the wave reaches 1/255
                const bool clamp = (clampmask >> k_surv) & 1ull;     // wave-uniform
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (pw[k] >= kLogAlphaMin) {
                        // only the pixels that take the Gaussian run this
                        // (exec mask; the others keep T and the sums as they
                        // are, which adding 0 would have left them)
                        asm volatile("");
                        float e = __builtin_amdgcn_exp2f(pw[k]);
                        if (clamp) {
                            // only survivors whose opacity can reach 0.99 pay for the clamp
                            asm volatile("");
                            e = fminf(0.99f, e);
                        }
                        float wgt = e * T[k];
                        T[k] = T[k] - wgt;
                        if (__ballot(T[k] < 1e-4f) != 0ull) {
                            // rare: a pixel that stops here adds nothing and
                            // keeps its transmittance (T' + alpha T restores it
                            // to within one rounding)
                            asm volatile("");
                            const bool stop = T[k] < 1e-4f;
                            if (COUNT && stop) stop_at[k] = b0 - start + L_.origin[w][k_surv] + 1u;
                            T[k] = stop ? T[k] + wgt : T[k];
                            wgt = stop ? 0.0f : wgt;
                            xl[k] = stop ? kDead : xl[k];
                        }
                        C0[k] = fmaf(cr, wgt, C0[k]);
                        C1[k] = fmaf(cg, wgt, C1[k]);
                        C2[k] = fmaf(cb, wgt, C2[k]);
                        D[k] = fmaf(z, wgt, D[k]);
                        if (COUNT) blended[k] += wgt > 0.0f ? 1u : 0u;
                    }
                }
            };
            // survivors two at a time: five 16-byte reads per pair (the second
            // survivor's last two words are read only when it exists)
            for (uint32_t k = 0; k < n_surv; k += 2) {
                const float4* P = reinterpret_cast<const float4*>(Wf + 10u * k);     // 16-byte aligned (k even)
                const float4 r0 = P[0], r1 = P[1], r2 = P[2];
                shade(make_float4(r0.x, r0.y, r0.z, r1.x), r1.y, r0.w, r2.y, r1.z, r1.w, r2.x, k);
                if (k + 1 < n_surv) {
                    const float4 r3 = P[3], r4 = P[4];
                    shade(make_float4(r2.z, r2.w, r3.x, r3.z), r3.w, r3.y, r4.w, r4.x, r4.y, r4.z, k + 1);
                }
            }
            // the wave stops once none of its pixels is live (checked per 64 candidates)
            bool lv = false;
#pragma unroll
            for (int k = 0; k < PPT; ++k) lv = lv || xl[k] < kDeadTest;
            if (__ballot(lv) == 0ull) wave_live = false;
        }
        if (lane == 0) L_.live[buf][w] = wave_live ? 1u : 0u;
        buf ^= 1;
    }

    if (bad_entry) atomicOr(c.err, kErrListEntry);

    // observation epilogue parameters of this image (identity when absent)
    float gain = 1.0f, contrast = 1.0f, bright = 0.0f;
    if (im.out_obs) {
        if (im.obs_gain) gain = im.obs_gain[im.obs_idx];
        if (im.obs_contrast) contrast = im.obs_contrast[im.obs_idx];
        if (im.obs_bright) bright = im.obs_bright[im.obs_idx];
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (pxi[k] >= im.width || pyi[k] >= im.height) continue;
        const size_t pix = (size_t)pyi[k] * im.width + pxi[k];
        const float rgb[3] = {fmaf(T[k], im.bg[0], C0[k]), fmaf(T[k], im.bg[1], C1[k]), fmaf(T[k], im.bg[2], C2[k])};
        if (im.out_rgb) {
            im.out_rgb[3 * pix + 0] = rgb[0];
            im.out_rgb[3 * pix + 1] = rgb[1];
            im.out_rgb[3 * pix + 2] = rgb[2];
        }
        if (im.out_obs) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                // each step rounded on its own (no contraction in this file)
                float x = rgb[ch] * gain;
                x = x - 0.5f;
                x = x * contrast;
                x = x + 0.5f;
                x = x + bright;
                x = fminf(fmaxf(x, 0.0f), 1.0f);
                if (im.obs_fmt == GSR_OBS_U8) {
                    const float q = floorf(x * 255.0f + 0.5f);
                    static_cast<uint8_t*>(im.out_obs)[3 * pix + ch] = (uint8_t)q;
                } else {
                    static_cast<__half*>(im.out_obs)[3 * pix + ch] = __float2half_rn(x);
                }
            }
        }
        im.out_depth[pix] = T[k] < 1.0f ? D[k] / (1.0f - T[k]) : 0.0f;
        if (im.out_alpha) im.out_alpha[pix] = 1.0f - T[k];
        if (COUNT && im.out_work) {
            im.out_work[2 * pix] = stop_at[k] != 0xFFFFFFFFu ? stop_at[k] : (FILTER ? qt : end - start);
            im.out_work[2 * pix + 1] = blended[k];
        }
    }
}

// One workgroup per tile.
template <int TS, int kBatch, bool COUNT>
__global__ __launch_bounds__(Layout<TS>::kThreads) void k_raster(SceneDev s, ChunkDev c, RasterParams p)
{
    __shared__ RasterLds<TS, kBatch> lds;
    if (*c.ovf) return;                 // no tile lists: the fallback composites this chunk
    raster_tile<TS, kBatch, COUNT, false>(s, c, p, xcd_remap(blockIdx.x, gridDim.x), lds, nullptr);
}

// Persistent workgroups.  The tiles are split into one contiguous range per
// XCD that has workgroups (min(8, grid) of them); the workgroups of an XCD take
// that range's tiles in image order from the XCD's own counter (zeroed by
// k_zero_counter before the launch), so concurrently shaded tiles share their
// images' records in that XCD's L2.  Every workgroup exits once its counter
// passes its range.
template <int TS, int kBatch, bool COUNT>
__global__ __launch_bounds__(Layout<TS>::kThreads) void k_raster_persistent(SceneDev s, ChunkDev c, RasterParams p,
                                                                            uint32_t* counter)
{
    __shared__ RasterLds<TS, kBatch> lds;
    __shared__ uint32_t next;
    if (*c.ovf) return;                 // no tile lists: the fallback composites this chunk
    const uint32_t parts = gridDim.x < (uint32_t)kXcds ? gridDim.x : (uint32_t)kXcds;
    const uint32_t x = blockIdx.x % (uint32_t)kXcds;       // < parts
    const uint32_t q = p.n_blocks / parts, r = p.n_blocks % parts;
    const uint32_t first = x * q + (x < r ? x : r), count = q + (x < r ? 1u : 0u);
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(&counter[x], 1u);
        __syncthreads();
        const uint32_t k = next;
        __syncthreads();
        if (k >= count) break;
        raster_tile<TS, kBatch, COUNT, false>(s, c, p, first + k, lds, nullptr);
        __syncthreads();
    }
}

// Fallback compositing of an overflowed chunk: persistent workgroups take the
// chunk's tiles from per-XCD counters (as k_raster_persistent) and filter
// each tile's list from the depth-ordered Gaussians.  Exits at once when the
// chunk's lists fit.
template <int TS, bool COUNT>
__global__ __launch_bounds__(Layout<TS>::kThreads) void k_raster_fallback(SceneDev s, ChunkDev c, RasterParams p,
                                                                          uint32_t* counter)
{
    constexpr int kB = 64;
    __shared__ RasterLds<TS, kB> lds;
    __shared__ FilterLds<TS> ring;
    __shared__ uint32_t next;
    if (!*c.ovf) return;
    const uint32_t parts = gridDim.x < (uint32_t)kXcds ? gridDim.x : (uint32_t)kXcds;
    const uint32_t x = blockIdx.x % (uint32_t)kXcds;       // < parts
    const uint32_t q = p.n_blocks / parts, r = p.n_blocks % parts;
    const uint32_t first = x * q + (x < r ? x : r), count = q + (x < r ? 1u : 0u);
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(&counter[x], 1u);
        __syncthreads();
        const uint32_t k = next;
        __syncthreads();
        if (k >= count) break;
        raster_tile<TS, kB, COUNT, true>(s, c, p, first + k, lds, &ring);
        __syncthreads();
    }
}

// Clears the per-XCD tile counters (a kernel, so that it can sit in a graph).
__global__ void k_zero_counter(uint32_t* counter)
{
    if (threadIdx.x < (uint32_t)kXcds) counter[threadIdx.x] = 0u;
}

template <int TS, int kBatch, bool COUNT>
hipError_t launch_tsc(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream)
{
    constexpr int NT = Layout<TS>::kThreads;
    if (p.persistent && p.counter) {
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, p.counter);
        const uint32_t grid = std::min<uint32_t>(p.n_blocks, (uint32_t)p.persistent_blocks);
        hipLaunchKernelGGL((k_raster_persistent<TS, kBatch, COUNT>), dim3(grid), dim3(NT), 0, stream, s, c, p,
                           p.counter);
    } else {
        hipLaunchKernelGGL((k_raster<TS, kBatch, COUNT>), dim3(p.n_blocks), dim3(NT), 0, stream, s, c, p);
    }
    return hipGetLastError();
}

template <int TS, int kBatch>
hipError_t launch_ts(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream)
{
    return p.count_work ? launch_tsc<TS, kBatch, true>(s, c, p, stream) : launch_tsc<TS, kBatch, false>(s, c, p, stream);
}

// LDS batch sizes: 64 / 128 / 256 records for 8x8 tiles (one wave), 64 to 512
// for the 256-thread layouts (smaller batches leave room for more workgroups
// per CU; batches below the block size are staged by the first threads).
template <int TS>
hipError_t launch_batch(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream)
{
    if (p.batch == 64) return launch_ts<TS, 64>(s, c, p, stream);
    if (p.batch == 128) return launch_ts<TS, 128>(s, c, p, stream);
    if constexpr (TS != 8)
        if (p.batch == 512) return launch_ts<TS, 512>(s, c, p, stream);
    return launch_ts<TS, 256>(s, c, p, stream);
}

}  // namespace

hipError_t launch_raster_fallback(const SceneDev& s, const ChunkDev& c, const RasterParams& p, uint32_t* counter,
                                  hipStream_t stream)
{
    if (p.n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, counter);
    const uint32_t grid = std::min<uint32_t>(p.n_blocks, (uint32_t)p.persistent_blocks);
    switch (p.ts) {
    case 8:
        if (p.count_work) hipLaunchKernelGGL((k_raster_fallback<8, true>), dim3(grid), dim3(64), 0, stream, s, c, p, counter);
        else hipLaunchKernelGGL((k_raster_fallback<8, false>), dim3(grid), dim3(64), 0, stream, s, c, p, counter);
        break;
    case 32:
        if (p.count_work) hipLaunchKernelGGL((k_raster_fallback<32, true>), dim3(grid), dim3(256), 0, stream, s, c, p, counter);
        else hipLaunchKernelGGL((k_raster_fallback<32, false>), dim3(grid), dim3(256), 0, stream, s, c, p, counter);
        break;
    default:
        if (p.count_work) hipLaunchKernelGGL((k_raster_fallback<16, true>), dim3(grid), dim3(256), 0, stream, s, c, p, counter);
        else hipLaunchKernelGGL((k_raster_fallback<16, false>), dim3(grid), dim3(256), 0, stream, s, c, p, counter);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_raster(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream)
{
    if (p.n_blocks == 0) return hipSuccess;
    switch (p.ts) {
    case 8: return launch_batch<8>(s, c, p, stream);
    case 32: return launch_batch<32>(s, c, p, stream);
    default: return launch_batch<16>(s, c, p, stream);
    }
}

}  // namespace gsr
