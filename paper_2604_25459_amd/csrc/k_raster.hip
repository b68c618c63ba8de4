// Per-tile front-to-back alpha compositing (3D Gaussian Splatting volume
// rendering, the image model of the paper's batch renderer).
//
// One workgroup per (image, tile) of the whole chunk, images of all camera
// slots in one launch.  The tile's depth-sorted Gaussian list is staged into
// LDS in batches of 256 records (each thread fetches one record); every
// thread then composites its pixels against the batch, reading records by LDS
// broadcast.  Per pixel and Gaussian:
//     log2(alpha) = A dx^2 + B dx dy + C dy^2 + log2(o)   (conic pre-scaled)
//     alpha < 1/255            -> skip
//     alpha = min(0.99, alpha); T' = T (1 - alpha)
//     T' < 1e-4                -> stop before adding
//     C += rgb alpha T, D += z alpha T, T = T'
// A wave skips a Gaussian outright when its conservative square (mean +- r,
// r = ceil(3.33 sqrt(lambda_max))) misses the wave's pixel block; no pixel
// there can reach alpha >= 1/255.  The workgroup stops when every pixel has
// terminated (block-wide count at each batch boundary).
#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kBatch = 256;

// Pixel layout: TS <= 16: one pixel per thread, waves own 8x8 blocks.
// TS == 32: 256 threads x 4 pixels, wave w owns rows [8w, 8w + 8) (32 x 8).
template <int TS>
struct Layout {
    static constexpr int kThreads = TS <= 16 ? TS * TS : 256;
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

template <int TS>
__global__ __launch_bounds__(Layout<TS>::kThreads) void k_raster(SceneDev s, ChunkDev c, RasterParams p)
{
    using L = Layout<TS>;
    constexpr int NT = L::kThreads;
    constexpr int PPT = L::kPpt;
    __shared__ float4 sA[kBatch], sB[kBatch], sC[kBatch];

    const uint32_t bid = blockIdx.x;
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
    // pixel-centre extent of the wave's block (for the conservative skip)
    const float wx0 = (float)(tx * TS + ox) + 0.5f;
    const float wx1 = wx0 + (float)(L::kWaveW - 1);
    const float wy0 = (float)(ty * TS + oy) + 0.5f;
    const float wy1 = wy0 + (float)(L::kWaveH - 1);

    float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
    bool live[PPT];
    int pxi[PPT], pyi[PPT];
    int n_live = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        int lx, ly;
        L::pixel(lane, k, &lx, &ly);
        pxi[k] = tx * TS + ox + lx;
        pyi[k] = ty * TS + oy + ly;
        live[k] = pxi[k] < im.width && pyi[k] < im.height;
        px[k] = (float)pxi[k] + 0.5f;
        py[k] = (float)pyi[k] + 0.5f;
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = D[k] = 0.0f;
        n_live += live[k] ? 1 : 0;
    }

    const uint32_t* R = c.tile_range + ((size_t)i * c.t_max + t) * 2;
    const uint32_t start = R[0], end = R[1];
    const uint32_t* list = c.pairs + c.pair_base[i];
    const float4* rec = c.rec + (size_t)i * (size_t)s.n * 3;
    const float kLogAlphaMin = -7.99435343685886f;   // log2(1/255)

    for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
        for (int k = tid; k < kBatch; k += NT) {
            const uint32_t e = b0 + (uint32_t)k;
            if (e < end) {
                uint32_t g = list[e];
                if (g >= (uint32_t)s.n) g = 0;      // guard: list entries are valid indices by construction
                sA[k] = rec[3 * (size_t)g];
                sB[k] = rec[3 * (size_t)g + 1];
                sC[k] = rec[3 * (size_t)g + 2];
            }
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)kBatch, end - b0);
        if (n_live > 0) {
            for (int j = 0; j < cnt; ++j) {
                const float4 a = sA[j];
                const float4 bq = sB[j];
                const float r = bq.w;
                if (a.x + r < wx0 || a.x - r > wx1 || a.y + r < wy0 || a.y - r > wy1) continue;
                bool any = false;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (!live[k]) continue;
                    const float dx = px[k] - a.x;
                    const float dy = py[k] - a.y;
                    const float pw = fmaf(dx, fmaf(a.z, dx, a.w * dy), fmaf(bq.x * dy, dy, bq.y));
                    if (pw < kLogAlphaMin) continue;
                    const float alpha = fminf(0.99f, __builtin_amdgcn_exp2f(pw));
                    const float Tn = T[k] * (1.0f - alpha);
                    if (Tn < 1e-4f) {
                        live[k] = false;
                        --n_live;
                        continue;
                    }
                    any = true;
                    const float4 col = sC[j];
                    const float wgt = alpha * T[k];
                    C0[k] = fmaf(col.x, wgt, C0[k]);
                    C1[k] = fmaf(col.y, wgt, C1[k]);
                    C2[k] = fmaf(col.z, wgt, C2[k]);
                    D[k] = fmaf(bq.z, wgt, D[k]);
                    T[k] = Tn;
                }
                (void)any;
                if (n_live == 0) break;
            }
        }
        if (__syncthreads_count(n_live > 0 ? 1 : 0) == 0) break;
    }

#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (pxi[k] >= im.width || pyi[k] >= im.height) continue;
        const size_t pix = im.out_pixel + (size_t)pyi[k] * im.width + pxi[k];
        p.out_rgb[3 * pix + 0] = fmaf(T[k], p.bg[0], C0[k]);
        p.out_rgb[3 * pix + 1] = fmaf(T[k], p.bg[1], C1[k]);
        p.out_rgb[3 * pix + 2] = fmaf(T[k], p.bg[2], C2[k]);
        p.out_depth[pix] = T[k] < 1.0f ? D[k] / (1.0f - T[k]) : 0.0f;
        if (p.out_alpha) p.out_alpha[pix] = 1.0f - T[k];
    }
}

}  // namespace

hipError_t launch_raster(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream)
{
    if (p.n_blocks == 0) return hipSuccess;
    switch (p.ts) {
    case 8: hipLaunchKernelGGL(k_raster<8>, dim3(p.n_blocks), dim3(Layout<8>::kThreads), 0, stream, s, c, p); break;
    case 32: hipLaunchKernelGGL(k_raster<32>, dim3(p.n_blocks), dim3(Layout<32>::kThreads), 0, stream, s, c, p); break;
    default: hipLaunchKernelGGL(k_raster<16>, dim3(p.n_blocks), dim3(Layout<16>::kThreads), 0, stream, s, c, p); break;
    }
    return hipGetLastError();
}

}  // namespace gsr
