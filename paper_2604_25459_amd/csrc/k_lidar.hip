// Batch LiDAR: ray casting of the resident, rigidly posed Gaussians for grids
// of rays (rotating or solid-state sensors) and for listed rays
// (non-repetitive scan patterns, sorted on the host into elevation bands of
// azimuth-ordered rays), through the same sort and tile binning as the
// cameras.
//
// Projection (one thread per Gaussian, a group of scans per thread):
//   * pose into the sensor frame with the binary32 specification of the
//     camera path (t = A mu + a);
//   * key = bits of the centre distance |t| (binary32, sqrt correctly
//     rounded), so the compositing order is (distance, index);
//   * tile rectangle: rows and columns of rays whose direction lies in the
//     cone of the sphere of radius sqrt(Qmax) * max scale around t (Qmax the
//     opacity bucket bound of the camera path), widened by a relative 1e-4 and
//     an absolute 2e-6 rad against the rounding of the trigonometric
//     functions; a cone across the seam of a full turn takes the hull of its
//     two column ranges, a sensor inside the sphere takes the whole grid;
//   * record: whitening W = S^-1 R^T (R, S the Gaussian's rotation in the
//     sensor frame and its scales), the centre t, log2 o and W t, and the
//     cone (centre direction, cosine of the half-angle) for wave culling.
// Raster (one workgroup per tile of rays, one ray per thread): for each
// listed Gaussian, d' = W d, t* = (d' . W t) / |d'|^2 (the peak of the
// Gaussian along the ray), q = |W (t - t* d)|^2 (the offset taken in metres
// first, so that no large whitened terms cancel), log2 alpha = log2 o - q/2
// log2 e; then the compositing rules of the camera path with the range t* in
// place of the depth.
#include "gsr_device.h"
#include "gsr_wave.h"

#include <algorithm>

namespace gsr {
namespace {

constexpr float kLidarLogAlphaMin = -7.99435343685886f;   // log2(1/255)
constexpr float kHalfPi = 1.5707963267948966f;
constexpr float kTwoPi = 6.283185307179586f;
constexpr int kLdsBeams = 256;      // angular scans with at most this many beams search their elevations in LDS
constexpr int kLdsTileAz = 1024;     // listed rays: tile azimuth tables up to this many floats are read from LDS
constexpr int kLidarRec = 5;        // float4s per record: whitening rows + centre, log2 o + W t, cone

// First index r in [0, H) with v[r] >= x (strict = false) or v[r] > x
// (strict = true), v ascending; H if none.
__device__ __forceinline__ int first_at_least(const float* v, int H, float x, bool strict)
{
    int lo = 0, hi = H;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool below = strict ? v[mid] <= x : v[mid] < x;
        if (below) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Columns c in [0, W) whose ray azimuth az0 + (c + 0.5) step lies in
// [a0, a1] (radians, a1 - a0 < 2 pi); returns an empty range when none.
__device__ __forceinline__ void column_range(float a0, float a1, float az0, float step, int W, int* c0, int* c1)
{
    const float lo = (a0 - az0) / step - 0.5f;
    const float hi = (a1 - az0) / step - 0.5f;
    int x0 = (int)ceilf(fmaxf(lo, -1.0f));
    int x1 = (int)floorf(fminf(hi, (float)W)) + 1;
    x0 = max(x0, 0);
    x1 = min(x1, W);
    *c0 = x0;
    *c1 = x1;
}

// Grid rays with index k in [0, n) whose origin c0 + (k + 0.5) step lies in
// [a0, a1]; an empty range when none.
__device__ __forceinline__ void column_range_grid(float a0, float a1, float c0, float step, int n, int* k0, int* k1)
{
    const float lo = (a0 - c0) / step - 0.5f;
    const float hi = (a1 - c0) / step - 0.5f;
    int x0 = (int)ceilf(fmaxf(lo, -1.0f));
    int x1 = (int)floorf(fminf(hi, (float)n)) + 1;
    *k0 = max(x0, 0);
    *k1 = min(x1, n);
}

// Records leave through LDS as in the camera projection: a wave's 64 records
// (80 bytes each) are written to LDS and stored back lane-contiguously, so
// each store instruction writes 1 KB of consecutive records.  The image
// descriptions come in as a restrict argument (uniform reads become scalar
// loads).
template <int ST>
__global__ __launch_bounds__(256) void k_project_lidar(SceneDev s, ChunkDev c, const ImageInfo* __restrict__ imgs,
                                                       int ts, int ipt)
{
    __shared__ float4 stage[4][kLidarRec * 64];
    // the elevation table of the current angular image (up to kLdsBeams beams;
    // the row search reads it ten times per Gaussian), or a listed-ray image's
    // band tables, and its tiles' azimuth spans
    __shared__ float elev_s[kLdsBeams];
    __shared__ float taz_s[kLdsTileAz];
    float4* const st = stage[threadIdx.x >> 6];
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const uint32_t bx = L / gridDim.y, by = L - bx * gridDim.y;
    const int64_t g_lane = (int64_t)bx * 256 + threadIdx.x;
    // lanes past the last Gaussian stay (invisible) so that every record store slot of the wave has a lane
    const bool valid = g_lane < s.n;
    const int64_t g = valid ? g_lane : s.n - 1;
    const int lane = __lane_id();
    const int i_begin = (int)by * ipt;
    const int slot = body_slot(s, g);
    const float4 pm = s.pos[g];
    float q[4], sc[3];
    load_rot_scale<ST>(s, g, q, sc);
    float Rg[9];
    quat_rot(q[0], q[1], q[2], q[3], Rg);
    const float mu[3] = {pm.x, pm.y, pm.z};
    const float op = pm.w;
    const float log2o = log2f(op);
    const float rho = sqrtf(opacity_qmax(op)) * fmaxf(sc[0], fmaxf(sc[1], sc[2]));
    const float isc[3] = {1.0f / sc[0], 1.0f / sc[1], 1.0f / sc[2]};

    for (int ii = 0; ii < ipt; ++ii) {
        const int i = __builtin_amdgcn_readfirstlane(i_begin + ii);     // the same in every lane
        if (i >= c.n_img) break;
        const ImageInfo im = imgs[i];
        // block-uniform: every thread of the block projects into image i
        const int n_ev = im.kind == 3 ? 2 * im.height : im.height;
        const int n_taz = im.kind == 3 ? 2 * im.tiles_x * im.tiles_y : 0;
        const bool lds_elev = (im.kind == 1 || im.kind == 3) && n_ev <= kLdsBeams;
        const bool lds_taz = im.kind == 3 && n_taz <= kLdsTileAz;
        if (lds_elev || lds_taz) {
            __syncthreads();                    // the previous image's tables are no longer read
            if (lds_elev && (int)threadIdx.x < n_ev) elev_s[threadIdx.x] = im.elev[threadIdx.x];
            if (lds_taz)
                for (int k = (int)threadIdx.x; k < n_taz; k += 256) taz_s[k] = im.ray_tile_az[k];
            __syncthreads();
        }
        const float* ev = lds_elev ? elev_s : im.elev;
        const float* taz = lds_taz ? taz_s : im.ray_tile_az;
        const float* X = c.xform + ((size_t)i * (s.n_bodies + 1) + slot) * 16;
        float A[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) A[k] = X[k];
        const float tx = ((A[0] * mu[0] + A[1] * mu[1]) + A[2] * mu[2]) + X[9];
        const float ty = ((A[3] * mu[0] + A[4] * mu[1]) + A[5] * mu[2]) + X[10];
        const float tz = ((A[6] * mu[0] + A[7] * mu[1]) + A[8] * mu[2]) + X[11];
        const bool grid = im.kind == 2;
        // key: centre distance (angular), depth of the centre below the sensor plane (grid)
        const float D = grid ? (-tz > 0.0f ? -tz : 0.0f) : sqrtf((tx * tx + ty * ty) + tz * tz);
        const size_t o = (size_t)i * (size_t)s.n + (size_t)g;
        bool ok = valid && isfinite(tx) && isfinite(ty) && isfinite(tz) && op >= 1.0f / 255.0f && isfinite(D) &&
                  sc[0] > 0.0f && sc[1] > 0.0f && sc[2] > 0.0f;
        int r0 = 0, r1 = 0, c0 = 0, c1 = 0;
        float cone_c = -2.0f;                           // cosine of the cone half-angle; -2 = every direction
        float disc = 0.0f;                              // grid: footprint radius on the sensor plane
        if (grid) {
            // the alpha >= 1/255 ellipsoid lies in the sphere of radius rho: rays (which look
            // down from z = 0) can reach it only if it dips below the plane, and only inside
            // its footprint disc (widened against the rounding of the ray origins)
            ok = ok && tz < rho;
            disc = rho * 1.0001f + 1e-6f * ((((1.0f + fabsf(tx)) + fabsf(ty)) + fabsf(im.gx0)) + fabsf(im.gy0));
            if (ok) {
                column_range_grid(tx - disc, tx + disc, im.gx0, im.gdx, im.width, &c0, &c1);
                column_range_grid(ty - disc, ty + disc, im.gy0, im.gdy, im.height, &r0, &r1);
            }
        } else if ((ok = ok && D > 0.0f)) {
            if (D <= rho * 1.001f + 1e-6f) {            // the sensor may sit inside: every ray
                r0 = 0;
                r1 = im.height;
                c0 = 0;
                c1 = im.width;
            } else {
                const float ang = asinf(rho / D) * 1.0001f + 2e-6f;
                cone_c = cosf(ang);
                const float el = asinf(fminf(1.0f, fmaxf(-1.0f, tz / D)));
                if (im.kind == 3) {
                    // bands whose elevation span [lo, hi] meets [el - ang, el + ang]
                    r0 = first_at_least(ev + im.height, im.height, el - ang, false);   // hi >= el - ang
                    r1 = first_at_least(ev, im.height, el + ang, true);                // lo <= el + ang
                } else {
                    r0 = first_at_least(ev, im.height, el - ang, false);   // rows with el - ang <= elev
                    r1 = first_at_least(ev, im.height, el + ang, true);    // ... <= el + ang
                }
                if (fabsf(el) + ang >= kHalfPi - 1e-4f) {
                    c0 = 0;
                    c1 = im.width;
                } else {
                    const float daz = asinf(fminf(1.0f, sinf(ang) / cosf(fabsf(el) + ang))) * 1.0001f + 2e-6f;
                    const float th = atan2f(ty, tx);
                    if (2.0f * daz >= kTwoPi - 1e-4f) {
                        c0 = 0;
                        c1 = im.width;
                    } else if (im.kind == 3) {
                        // per tile row of the bands, the ray tiles whose azimuth span
                        // [smallest, largest] meets the window, at each 2 pi shift that
                        // meets [-pi, pi]; the hull over the tile rows, in rays
                        const int TX = im.tiles_x, y0 = r0 / ts, y1 = (r1 + ts - 1) / ts;
                        const float* tmin = taz;
                        const float* tmax = taz + (size_t)TX * im.tiles_y;
                        int lo = TX, hi = 0;
                        for (int y = y0; y < y1; ++y) {
#pragma unroll
                            for (int k = -1; k <= 1; ++k) {
                                const float a0 = th - daz + (float)k * kTwoPi, a1 = th + daz + (float)k * kTwoPi;
                                if (a1 < -3.1416f || a0 > 3.1416f) continue;
                                const int a = first_at_least(tmax + (size_t)y * TX, TX, a0, false);   // largest >= a0
                                const int b = first_at_least(tmin + (size_t)y * TX, TX, a1, true);    // smallest <= a1
                                if (a < b) {
                                    lo = min(lo, a);
                                    hi = max(hi, b);
                                }
                            }
                        }
                        c0 = lo * ts;
                        c1 = min(im.width, hi * ts);
                    } else {
                        // the azimuth window, tested at its three 2 pi shifts; the hull of the hits
                        int lo = im.width, hi = 0;
#pragma unroll
                        for (int k = -1; k <= 1; ++k) {
                            int a, b;
                            column_range(th - daz + (float)k * kTwoPi, th + daz + (float)k * kTwoPi, im.az0,
                                         im.az_step, im.width, &a, &b);
                            if (a < b) {
                                lo = min(lo, a);
                                hi = max(hi, b);
                            }
                        }
                        c0 = lo;
                        c1 = hi;
                    }
                }
            }
        }
        const bool vis = ok && r1 > r0 && c1 > c0;
        if (valid) c.keyz[o] = vis ? __float_as_uint(D) : kInvalidKey;
        const uint64_t vmask = __ballot(vis);
        if (vmask == 0ull) continue;            // wave-uniform
        if (vis) {
            const int x0 = c0 / ts, x1 = (c1 + ts - 1) / ts, y0 = r0 / ts, y1 = (r1 + ts - 1) / ts;
            put_rect(c.rect, c.rect4, o, (uint32_t)x0, (uint32_t)x1, (uint32_t)y0, (uint32_t)y1);
            // whitening W = S^-1 (A Rg)^T: row k = (A Rg)[:, k] / s_k
            float Rs[9];
            mat3_mul(A, Rg, Rs);
            float W[9];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j) W[3 * k + j] = Rs[3 * j + k] * isc[k];
            const float w0 = (W[0] * tx + W[1] * ty) + W[2] * tz;
            const float w1 = (W[3] * tx + W[4] * ty) + W[5] * tz;
            const float w2 = (W[6] * tx + W[7] * ty) + W[8] * tz;
            float4* r = st + kLidarRec * lane;
            r[0] = make_float4(W[0], W[1], W[2], tx);
            r[1] = make_float4(W[3], W[4], W[5], ty);
            r[2] = make_float4(W[6], W[7], W[8], tz);
            r[3] = make_float4(log2o, w0, w1, w2);
            if (grid) {
                r[4] = make_float4(tx, ty, disc, 0.0f);
            } else {
                const float iD = 1.0f / D;
                r[4] = make_float4(tx * iD, ty * iD, tz * iD, cone_c);
            }
        }
        wave_lds_sync();
        // float4 q of the wave's records belongs to lane q / kLidarRec
        float4* rec = c.rec + kLidarRec * ((size_t)i * (size_t)s.n + (size_t)(g_lane - lane));
#pragma unroll
        for (int k = 0; k < kLidarRec; ++k) {
            const int q = lane + 64 * k;
            if ((vmask >> (q / kLidarRec)) & 1ull) store_stream(rec + q, st[q]);
        }
        wave_lds_sync();
    }
}

// One workgroup per TS x TS tile of rays; batches of kLBatch records in LDS.
// Wave-level culling.  Angular rays: each wave bounds its rays by a cone
// (axis = their normalised mean direction, half-angle beta = the widest ray),
// and a Gaussian survives when its own cone (half-angle alpha around its
// centre direction, as used for the tile rectangle) comes within alpha + beta
// of that axis.  Grid rays: the wave's ray origins span a rectangle of the
// sensor plane, and a Gaussian survives when its footprint disc reaches it.
// Only survivors are evaluated, bit by bit of the wave's ballot.
template <int TS>
struct LidarLds {
    float4 sr[kLidarRec][TS * TS];
    uint32_t live_w[2][TS * TS / 64];     // per wave: live rays left after a batch (by batch parity)
};

template <int TS, bool GRID>
__device__ __forceinline__ void lidar_tile(const SceneDev& s, const ChunkDev& c, int i, const ImageInfo& im, int tx,
                                           int ty, uint32_t t, LidarLds<TS>& L_)
{
    constexpr int NT = TS * TS;
    constexpr int kLBatch = NT;
    auto& sr = L_.sr;
    auto& live_w = L_.live_w;
    const int tid = threadIdx.x, lane = __lane_id();
    const int col = tx * TS + (tid % TS), row = ty * TS + (tid / TS);
    const bool inside = col < im.width && row < im.height;
    // ray: origin o (grid; the sensor origin otherwise) and direction d
    float d[3] = {0.0f, 0.0f, GRID ? -1.0f : 0.0f};
    float ox = 0.0f, oy = 0.0f;
    if (GRID) {
        ox = im.gx0 + ((float)col + 0.5f) * im.gdx;
        oy = im.gy0 + ((float)row + 0.5f) * im.gdy;
    } else if (inside) {
        float az, el;
        if (im.kind == 3) {
            az = im.ray_az[(size_t)row * im.width + col];
            el = im.ray_el[(size_t)row * im.width + col];
        } else {
            az = im.az0 + ((float)col + 0.5f) * im.az_step;
            el = im.elev[row];
        }
        float sa, ca, se, ce;
        sincosf(az, &sa, &ca);
        sincosf(el, &se, &ce);
        d[0] = ce * ca;
        d[1] = ce * sa;
        d[2] = se;
    }
    // the wave's bound: a cone (angular; culling off when wider than 90 degrees) or the
    // rectangle of its ray origins (grid)
    float w[3] = {d[0], d[1], d[2]};
    bool cull = true;
    float cb = 1.0f, sb = 0.0f;
    float bx0 = inside ? ox : 3.0e38f, bx1 = inside ? ox : -3.0e38f;
    float by0 = inside ? oy : 3.0e38f, by1 = inside ? oy : -3.0e38f;
    if (GRID) {
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            bx0 = fminf(bx0, __shfl_xor(bx0, m, 64));
            bx1 = fmaxf(bx1, __shfl_xor(bx1, m, 64));
            by0 = fminf(by0, __shfl_xor(by0, m, 64));
            by1 = fmaxf(by1, __shfl_xor(by1, m, 64));
        }
    } else {
#pragma unroll
        for (int m = 1; m < 64; m <<= 1)
#pragma unroll
            for (int k = 0; k < 3; ++k) w[k] += __shfl_xor(w[k], m, 64);
        const float wn = sqrtf(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        cull = wn > 0.0f;
        if (cull)
#pragma unroll
            for (int k = 0; k < 3; ++k) w[k] /= wn;
        cb = inside ? d[0] * w[0] + d[1] * w[1] + d[2] * w[2] : 1.0f;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) cb = fminf(cb, __shfl_xor(cb, m, 64));
        cb = cb - 1e-5f;                              // rounding of the directions and of the axis
        cull = cull && cb > 0.0f;
        sb = sqrtf(fmaxf(0.0f, 1.0f - cb * cb));
    }

    bool live = inside;
    float T = 1.0f, Rg = 0.0f;
    const float near = im.near_plane;
    const uint32_t* R = c.tile_range + ((size_t)i * c.t_max + t) * 2;
    const uint32_t start = R[0], end = R[1];
    const uint32_t* list = c.pairs + c.pair_base[i];
    const float4* rec = c.rec + (size_t)i * (size_t)s.n * kLidarRec;
    const uint32_t n = (uint32_t)s.n;
    bool wave_live = __ballot(live) != 0ull;
    bool bad_entry = false;
    int par = 0;
    for (uint32_t b0 = start; b0 < end; b0 += kLBatch, par ^= 1) {
        __syncthreads();
        // every wave's flag from the previous batch is visible after the
        // barrier, so all waves take the same decision
        if (b0 != start) {
            uint32_t any = 0;
#pragma unroll
            for (int ww = 0; ww < NT / 64; ++ww) any |= live_w[par ^ 1][ww];
            if (!any) break;
        }
        const uint32_t e = b0 + (uint32_t)tid;
        if (e < end) {
            uint32_t g = list[e];
            if (g >= n) {               // impossible by construction: reported at the end, a valid record read
                bad_entry = true;
                g = 0;
            }
#pragma unroll
            for (int k = 0; k < kLidarRec; ++k) sr[k][tid] = rec[kLidarRec * (size_t)g + k];
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)kLBatch, end - b0);
        for (int sub = 0; sub < cnt && wave_live; sub += 64) {
            const int jl = sub + lane;
            bool keep = false;
            if (jl < cnt) {
                const float4 cn = sr[4][jl];
                if (GRID) {
                    // distance from the footprint centre to the origin rectangle, against the disc radius
                    const float ex = fmaxf(0.0f, fmaxf(bx0 - cn.x, cn.x - bx1));
                    const float ey = fmaxf(0.0f, fmaxf(by0 - cn.y, cn.y - by1));
                    keep = ex * ex + ey * ey <= cn.z * cn.z * 1.0001f;
                } else if (!cull || cn.w < -1.5f) {
                    keep = true;
                } else {
                    const float sa = sqrtf(fmaxf(0.0f, 1.0f - cn.w * cn.w));
                    keep = cn.x * w[0] + cn.y * w[1] + cn.z * w[2] >= cn.w * cb - sa * sb - 1e-6f;
                }
            }
            // survivors two at a time: both are evaluated (independent
            // dependency chains the wave interleaves), then composited in list order
            auto eval = [&](int j, float* ts_out, float* la_out) {
                const float4 m0 = sr[0][j], m1 = sr[1][j], m2 = sr[2][j], m3 = sr[3][j];
                // d' = W d
                const float dx = fmaf(m0.z, d[2], fmaf(m0.y, d[1], m0.x * d[0]));
                const float dy = fmaf(m1.z, d[2], fmaf(m1.y, d[1], m1.x * d[0]));
                const float dz = fmaf(m2.z, d[2], fmaf(m2.y, d[1], m2.x * d[0]));
                const float aa = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                // centre relative to the ray origin, and W times it
                float cx = m0.w, cy = m1.w, wcx = m3.y, wcy = m3.z, wcz = m3.w;
                if (GRID) {
                    cx = m0.w - ox;
                    cy = m1.w - oy;
                    wcx = m3.y - fmaf(m0.y, oy, m0.x * ox);
                    wcy = m3.z - fmaf(m1.y, oy, m1.x * ox);
                    wcz = m3.w - fmaf(m2.y, oy, m2.x * ox);
                }
                const float bb = fmaf(dz, wcz, fmaf(dy, wcy, dx * wcx));
                const float tstar = bb * __builtin_amdgcn_rcpf(aa);
                // offset of the centre from the ray's closest point, in metres, then whitened
                const float px = fmaf(-tstar, d[0], cx);
                const float py = fmaf(-tstar, d[1], cy);
                const float pz = fmaf(-tstar, d[2], m2.w);
                const float wx = fmaf(m0.z, pz, fmaf(m0.y, py, m0.x * px));
                const float wy = fmaf(m1.z, pz, fmaf(m1.y, py, m1.x * px));
                const float wz = fmaf(m2.z, pz, fmaf(m2.y, py, m2.x * px));
                const float qq = fmaf(wz, wz, fmaf(wy, wy, wx * wx));
                *ts_out = tstar;
                *la_out = fmaf(-0.72134752044448170f, qq, m3.x);      // log2 o - q/2 log2 e
            };
            auto take = [&](float tstar, float la) {
                if (live && tstar > near && la >= kLidarLogAlphaMin) {
                    // only the rays that take the Gaussian run this (exec mask);
                    // the empty asm keeps it a branch rather than selects
                    asm volatile("");
                    const float alpha = fminf(0.99f, __builtin_amdgcn_exp2f(la));
                    const float Tn = fmaf(-T, alpha, T);
                    if (Tn < 1e-4f) {
                        live = false;                   // stops here, adds nothing
                    } else {
                        Rg = fmaf(tstar, alpha * T, Rg);
                        T = Tn;
                    }
                }
            };
            uint64_t mask = __ballot(keep);
            while (mask) {
                const int j0 = sub + (int)__builtin_ctzll(mask);
                mask &= mask - 1ull;
                const bool two = mask != 0ull;                  // wave-uniform
                const int j1 = two ? sub + (int)__builtin_ctzll(mask) : j0;
                if (two) mask &= mask - 1ull;
                if (!live) continue;
                float t0, l0, t1, l1;
                eval(j0, &t0, &l0);
                eval(j1, &t1, &l1);
                take(t0, l0);
                if (two) take(t1, l1);
            }
            if (__ballot(live) == 0ull) wave_live = false;
        }
        if (lane == 0) live_w[par][tid >> 6] = wave_live ? 1u : 0u;
    }
    if (bad_entry) atomicOr(c.err, kErrListEntry);
    if (inside) {
        // listed rays leave in the caller's order
        const size_t pix = im.kind == 3 ? (size_t)im.ray_perm[(size_t)row * im.width + col]
                                        : (size_t)row * im.width + col;
        im.out_depth[pix] = T < 1.0f ? Rg / (1.0f - T) : 0.0f;
        if (im.out_alpha) im.out_alpha[pix] = 1.0f - T;
    }
}

template <int TS>
__global__ __launch_bounds__(TS * TS) void k_raster_lidar(SceneDev s, ChunkDev c, RasterParams p)
{
    __shared__ LidarLds<TS> lds;
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
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
    if (im.kind == 2) lidar_tile<TS, true>(s, c, i, im, tx, ty, t, lds);     // workgroup-uniform
    else lidar_tile<TS, false>(s, c, i, im, tx, ty, t, lds);
}

template <int ST>
hipError_t project_lidar_st(const SceneDev& s, const ChunkDev& c, int ts, int ipt, hipStream_t st)
{
    const dim3 grid((unsigned)((s.n + 255) / 256), (unsigned)((c.n_img + ipt - 1) / ipt));
    hipLaunchKernelGGL((k_project_lidar<ST>), grid, dim3(256), 0, st, s, c, c.img, ts, ipt);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project_lidar(const SceneDev& s, const ChunkDev& c, int ts, int ipt, hipStream_t stream)
{
    if (s.n == 0 || c.n_img == 0) return hipSuccess;
    ipt = std::max(1, std::min(ipt, c.n_img / 32));     // small chunks: more threads, fewer images each
    if (s.storage == kF16) return project_lidar_st<kF16>(s, c, ts, ipt, stream);
    if (s.storage == kBF16) return project_lidar_st<kBF16>(s, c, ts, ipt, stream);
    return project_lidar_st<kF32>(s, c, ts, ipt, stream);
}

hipError_t launch_raster_lidar(const SceneDev& s, const ChunkDev& c, const RasterParams& p, hipStream_t stream)
{
    if (p.n_blocks == 0) return hipSuccess;
    if (p.ts == 8) hipLaunchKernelGGL((k_raster_lidar<8>), dim3(p.n_blocks), dim3(64), 0, stream, s, c, p);
    else if (p.ts == 16) hipLaunchKernelGGL((k_raster_lidar<16>), dim3(p.n_blocks), dim3(256), 0, stream, s, c, p);
    else return hipErrorInvalidValue;           // 32 x 32 ray tiles exceed the workgroup size
    return hipGetLastError();
}

}  // namespace gsr
