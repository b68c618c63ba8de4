// Rigid-link posing, EWA projection, culling, tile rectangle and spherical-
// harmonic colour of every (image, Gaussian) pair.
//
// Posing follows the paper's Rigid-Link Gaussian Kinematics (Sec. "Batch
// Renderer Optimization"): a Gaussian cluster bound to a rigid body moves with
// that body, so its camera-from-local transform is A = R_c R(q_b),
// a = R_c t_b + t_c (static background: A = R_c, a = t_c).  Projection is the
// standard 3D Gaussian Splatting / EWA model the paper renders with.
//
// The binning quantities are computed in the library's binary32
// specification: one rounding per operation (this file is compiled with
// -ffp-contract=off), sums left to right, correctly rounded division and
// square root, constants as float literals.  The tile rectangle is the tighter
// of the conservative radius square and the axis-aligned box of the ellipse
// on which alpha falls to 1/255 for the Gaussian's opacity (per opacity
// bucket, with a 1 % margin), so no pixel that could take the Gaussian is
// left out of its tiles.
#include "gsr_device.h"
#include "gsr_wave.h"

namespace gsr {
namespace {

// ---------------------------------------------------------------- compose
// One thread per (image, body slot).  xform row: A (9, row-major), a (3),
// camera centre expressed in the slot's local frame (3), unused (1).
__global__ __launch_bounds__(256) void k_compose(SceneDev s, ChunkDev c, const float* __restrict__ viewmats,
                                                 const float* __restrict__ poses)
{
    const int slots = s.n_bodies + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= c.n_img * slots) return;
    const int i = idx / slots;
    const int slot = idx - i * slots;
    const ImageInfo im = c.img[i];
    const float* vm = viewmats + im.vm_off;
    float Rc[9] = {vm[0], vm[1], vm[2], vm[4], vm[5], vm[6], vm[8], vm[9], vm[10]};
    float tc[3] = {vm[3], vm[7], vm[11]};
    if (im.attach_body >= 0) {
        // camera rides on a body: the viewmat is body->camera [R_o | t_o];
        // world->camera = R_o R_k^T, t_o - (R_o R_k^T) t_k (k = attach_body)
        const float* pk = poses + im.pose_off + (size_t)im.attach_body * 7;
        float Rk[9], RkT[9], Ro[9];
        quat_rot(pk[0], pk[1], pk[2], pk[3], Rk);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) RkT[3 * r + q] = Rk[3 * q + r];
#pragma unroll
        for (int k = 0; k < 9; ++k) Ro[k] = Rc[k];
        mat3_mul(Ro, RkT, Rc);
#pragma unroll
        for (int r = 0; r < 3; ++r)
            tc[r] = tc[r] - ((Rc[3 * r + 0] * pk[4] + Rc[3 * r + 1] * pk[5]) + Rc[3 * r + 2] * pk[6]);
    }
    // camera centre in world: C = -R_c^T t_c (continuous quantity, colour only)
    const float Cw[3] = {-(Rc[0] * tc[0] + Rc[3] * tc[1] + Rc[6] * tc[2]),
                         -(Rc[1] * tc[0] + Rc[4] * tc[1] + Rc[7] * tc[2]),
                         -(Rc[2] * tc[0] + Rc[5] * tc[1] + Rc[8] * tc[2])};
    float* out = c.xform + (size_t)idx * 16;
    if (slot == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = Rc[k];
        out[9] = tc[0];
        out[10] = tc[1];
        out[11] = tc[2];
        out[12] = Cw[0];
        out[13] = Cw[1];
        out[14] = Cw[2];
        out[15] = 0.0f;
        return;
    }
    const float* p = poses + im.pose_off + (size_t)(slot - 1) * 7;
    float Rb[9], A[9];
    quat_rot(p[0], p[1], p[2], p[3], Rb);
    mat3_mul(Rc, Rb, A);
    const float tb[3] = {p[4], p[5], p[6]};
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k] = A[k];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        out[9 + r] = ((Rc[3 * r + 0] * tb[0] + Rc[3 * r + 1] * tb[1]) + Rc[3 * r + 2] * tb[2]) + tc[r];
    // camera centre in the body frame: R_b^T (C - t_b)
    const float d[3] = {Cw[0] - tb[0], Cw[1] - tb[1], Cw[2] - tb[2]};
    out[12] = Rb[0] * d[0] + Rb[3] * d[1] + Rb[6] * d[2];
    out[13] = Rb[1] * d[0] + Rb[4] * d[1] + Rb[7] * d[2];
    out[14] = Rb[2] * d[0] + Rb[5] * d[1] + Rb[8] * d[2];
    out[15] = 0.0f;
}

// ---------------------------------------------------------------- SH colour
// Real SH up to degree 3 in the coefficient order used by 3DGS (real
// harmonics with the Condon-Shortley phase, m = -l..l within each band).
template <int DEG>
__device__ __forceinline__ void sh_rgb(const float* f, float x, float y, float z, float rgb[3])
{
    constexpr float kC0 = 0.28209479177387814f;     // 1/(2 sqrt(pi))
    constexpr float kC1 = 0.48860251190291992f;     // sqrt(3)/(2 sqrt(pi))
    float Y[16];
    Y[0] = kC0;
    if (DEG >= 1) {
        Y[1] = -kC1 * y;
        Y[2] = kC1 * z;
        Y[3] = -kC1 * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484305920792f * x * y;                     // sqrt(15)/(2 sqrt(pi))
        Y[5] = -1.0925484305920792f * y * z;
        Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);    // sqrt(5)/(4 sqrt(pi))
        Y[7] = -1.0925484305920792f * x * z;
        Y[8] = 0.54627421529603959f * (xx - yy);                // sqrt(15)/(4 sqrt(pi))
        if (DEG >= 3) {
            Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);        // sqrt(35/2)/(4 sqrt(pi))
            Y[10] = 2.8906114426405538f * x * y * z;                    // sqrt(105)/(2 sqrt(pi))
            Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);  // sqrt(21/2)/(4 sqrt(pi))
            Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);   // sqrt(7)/(4 sqrt(pi))
            Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
            Y[14] = 1.4453057213202769f * z * (xx - yy);                // sqrt(105)/(4 sqrt(pi))
            Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
        }
    }
    constexpr int K = (DEG + 1) * (DEG + 1);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.5f;
#pragma unroll
        for (int k = 0; k < K; ++k) acc = fmaf(Y[k], f[3 * k + ch], acc);
        rgb[ch] = fmaxf(acc, 0.0f);
    }
}

// ---------------------------------------------------------------- project
// Grid: x = Gaussian blocks of 256, y = groups of `ipt` images.  A thread loads
// its Gaussian once and projects it into each image of its group.  Blocks are
// renumbered so that one XCD runs every image group of a run of Gaussian
// blocks back to back: the scene is fetched into each L2 about once.
// The image descriptions and transform rows come in as restrict arguments:
// nothing the kernel writes aliases them, so uniform reads of them can be
// scalar loads.  Records leave through LDS: a wave's 64 records (48 bytes
// each, one per lane) are written to LDS and stored back lane-contiguously,
// 1 KB per store instruction, instead of each lane storing its own 48 bytes
// (three times the cache lines per instruction).  Lanes past the last
// Gaussian stay in the loop (as invisible) so that every store slot of the
// wave has a lane.
template <int ST, int DEG>
__global__ __launch_bounds__(256) void k_project(SceneDev s, ChunkDev c, const ImageInfo* __restrict__ imgs,
                                                 const float* __restrict__ xform, int ts, float cutoff, int ipt)
{
    __shared__ float4 stage[4][3 * 64];
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const uint32_t bx = L / gridDim.y, by = L - bx * gridDim.y;
    const int64_t g_lane = (int64_t)bx * 256 + threadIdx.x;
    const bool valid = g_lane < s.n;
    const int64_t g = valid ? g_lane : s.n - 1;       // loads of lanes past the end read the last Gaussian
    const int i_begin = (int)by * ipt;
    const int lane = __lane_id();
    float4* const st = stage[threadIdx.x >> 6];

    int slot = 0;
    if (s.n_bodies > 0 && g >= s.body_off[0]) {
        int lo = 0, hi = s.n_bodies - 1;        // largest b with off[b] <= g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s.body_off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        slot = lo + 1;
    }

    const float4 pm = s.pos[g];
    float q[4], sc[3];
    constexpr int K = (DEG + 1) * (DEG + 1);
    float f[3 * K];
    if (ST == kF32) {
        const float4 qq = ((const float4*)s.rot)[g];
        const float4 ss = s.scale[g];
        q[0] = qq.x; q[1] = qq.y; q[2] = qq.z; q[3] = qq.w;
        sc[0] = ss.x; sc[1] = ss.y; sc[2] = ss.z;
        const float4* planes = (const float4*)s.sh;
        constexpr int NCH = (3 * K + 3) / 4;
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const float4 v = planes[(size_t)j * s.n_pad + g];
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (4 * j + k < 3 * K) f[4 * j + k] = vv[k];
        }
    } else {
        const uint4 hq = ((const uint4*)s.rot)[g];
        q[0] = decode<ST>(hq.x & 0xFFFF); q[1] = decode<ST>(hq.x >> 16);
        q[2] = decode<ST>(hq.y & 0xFFFF); q[3] = decode<ST>(hq.y >> 16);
        sc[0] = decode<ST>(hq.z & 0xFFFF); sc[1] = decode<ST>(hq.z >> 16);
        sc[2] = decode<ST>(hq.w & 0xFFFF);
        const uint4* planes = (const uint4*)s.sh;
        constexpr int NCH = (3 * K + 7) / 8;
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const uint4 v = planes[(size_t)j * s.n_pad + g];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (8 * j + k < 3 * K) f[8 * j + k] = decode<ST>((uint16_t)(w[k >> 1] >> (16 * (k & 1))));
        }
    }
    float Rg[9];
    quat_rot(q[0], q[1], q[2], q[3], Rg);
    const float mu[3] = {pm.x, pm.y, pm.z};
    const float op = pm.w;
    const float alpha_min = 1.0f / 255.0f;
    const float inv_ts = 1.0f / (float)ts;      // tile sides are powers of two: the scaling is exact
    const float log2o = log2f(op);
    // Opacity-aware extent: alpha >= 1/255 needs q <= 2 ln(255 o), bounded per
    // opacity bucket with 1 % to spare for the rounding of the extents.
    const float qmax = opacity_qmax(op);

    // one image: X is the image's transform row for the Gaussian's body slot
    auto project_into = [&](int i_any, int sl) {
        const int i = __builtin_amdgcn_readfirstlane(i_any);      // the same in every lane
        const ImageInfo im = imgs[i];
        const float* X = xform + ((size_t)i * (s.n_bodies + 1) + sl) * 16;
        float A[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) A[k] = X[k];
        const float tx = ((A[0] * mu[0] + A[1] * mu[1]) + A[2] * mu[2]) + X[9];
        const float ty = ((A[3] * mu[0] + A[4] * mu[1]) + A[5] * mu[2]) + X[10];
        const float tz = ((A[6] * mu[0] + A[7] * mu[1]) + A[8] * mu[2]) + X[11];

        float M[9];
        mat3_mul(A, Rg, M);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) M[3 * r + k] = M[3 * r + k] * sc[k];

        const float fx = im.fx, fy = im.fy;
        const float lx = im.guard_x, ly = im.guard_y;
        const float itz = 1.0f / tz;            // the one division by depth; products below
        const float itz2 = itz * itz;
        const float xcl = fminf(lx, fmaxf(-lx, tx * itz)) * tz;
        const float ycl = fminf(ly, fmaxf(-ly, ty * itz)) * tz;
        const float j00 = fx * itz;
        const float j02 = -((fx * xcl) * itz2);
        const float j11 = fy * itz;
        const float j12 = -((fy * ycl) * itz2);
        float v1[3], v2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v1[k] = j00 * M[k] + j02 * M[6 + k];
            v2[k] = j11 * M[3 + k] + j12 * M[6 + k];
        }
        const float n1 = (v1[0] * v1[0] + v1[1] * v1[1]) + v1[2] * v1[2];
        const float n2 = (v2[0] * v2[0] + v2[1] * v2[1]) + v2[2] * v2[2];
        const float ca = n1 + 0.3f;
        const float cc = n2 + 0.3f;
        const float cb = (v1[0] * v2[0] + v1[1] * v2[1]) + v1[2] * v2[2];
        const float w0 = v1[1] * v2[2] - v1[2] * v2[1];
        const float w1 = v1[2] * v2[0] - v1[0] * v2[2];
        const float w2 = v1[0] * v2[1] - v1[1] * v2[0];
        const float det = (((w0 * w0 + w1 * w1) + w2 * w2) + 0.3f * (n1 + n2)) + 0.09f;
        const float m = 0.5f * (ca + cc);
        const float h = 0.5f * (ca - cc);
        const float lam = m + sqrtf(fmaxf(0.1f, h * h + cb * cb));
        const float r = ceilf(cutoff * sqrtf(lam));
        const float u = (fx * tx) * itz + im.cx;
        const float v = (fy * ty) * itz + im.cy;
        // tighter of the radius square and the box of the ellipse q <= qmax
        const float rx = fminf(r, sqrtf(qmax * ca));
        const float ry = fminf(r, sqrtf(qmax * cc));
        const float x0 = fminf(fmaxf(floorf((u - rx) * inv_ts), 0.0f), (float)im.tiles_x);
        const float x1 = fminf(fmaxf(floorf((u + rx) * inv_ts) + 1.0f, 0.0f), (float)im.tiles_x);
        const float y0 = fminf(fmaxf(floorf((v - ry) * inv_ts), 0.0f), (float)im.tiles_y);
        const float y1 = fminf(fmaxf(floorf((v + ry) * inv_ts) + 1.0f, 0.0f), (float)im.tiles_y);

        bool vis = valid && isfinite(tx) && isfinite(ty) && isfinite(tz) && tz > im.near_plane && op >= alpha_min &&
                   isfinite(det) && det > 0.0f && isfinite(r) && isfinite(u) && isfinite(v);
        const int ix0 = vis ? (int)x0 : 0, ix1 = vis ? (int)x1 : 0;
        const int iy0 = vis ? (int)y0 : 0, iy1 = vis ? (int)y1 : 0;
        vis = vis && ix1 > ix0 && iy1 > iy0;

        const size_t o = (size_t)i * (size_t)s.n + (size_t)g_lane;
        if (valid) c.keyz[o] = vis ? __float_as_uint(tz) : kInvalidKey;
        const uint64_t vmask = __ballot(vis);
        if (vmask == 0ull) return;              // wave-uniform
        if (vis) {
            put_rect(c.rect, c.rect4, o, (uint32_t)ix0, (uint32_t)ix1, (uint32_t)iy0, (uint32_t)iy1);

            // Raster record: the quadratic form of the conic in whitened form,
            //     log2(alpha) = log2(o) - (a1 dx + b1 dy)^2 - (c1 dy)^2,
            // i.e. 0.5 log2(e) [dx dy] Sigma^-1 [dx dy]^T factored as W^T W with
            // W = [[a1, b1], [0, c1]] (Sigma = [[ca, cb], [cb, cc]], det = ca cc - cb^2):
            //     a1 = sqrt(k cc / det), b1 = -k cb / (det a1), c1 = sqrt(k / cc),
            // k = 0.5 log2(e).  A sum of squares stays accurate where the expanded
            // quadratic cancels (long, thin splats far from their centre).
            // Continuous quantities only (no binning decision depends on them):
            // hardware reciprocals and square roots.
            constexpr float kHalfLog2e = 0.72134752044448170f;
            constexpr float kSqrtHalfLog2e = 0.84932180028801907f;
            const float idet = __builtin_amdgcn_rcpf(det);
            const float wa = __builtin_amdgcn_sqrtf(kHalfLog2e * cc * idet);
            const float wb = -(kHalfLog2e * cb * idet) * __builtin_amdgcn_rcpf(wa);
            const float wc = kSqrtHalfLog2e * __builtin_amdgcn_rsqf(cc);
            float rgb[3];
            {
                float dx = mu[0] - X[12], dy = mu[1] - X[13], dz = mu[2] - X[14];
                const float inv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
                sh_rgb<DEG>(f, dx * inv, dy * inv, dz * inv, rgb);
            }
            st[3 * lane] = make_float4(u, v, wa, wb);
            st[3 * lane + 1] = make_float4(wc, log2o, tz, r);
            st[3 * lane + 2] = make_float4(rgb[0], rgb[1], rgb[2], 0.0f);
        }
        wave_lds_sync();
        // float4 q of the wave's records belongs to lane q / 3
        float4* rec = c.rec + 3 * (o - (size_t)lane);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int q = lane + 64 * k;
            if ((vmask >> (q / 3)) & 1ull) store_stream(rec + q, st[q]);
        }
        wave_lds_sync();
    };
    const int i_end = min(i_begin + ipt, c.n_img);
    // Waves whose Gaussians all ride on one body (nearly all: bodies are
    // contiguous runs of storage order) read the transform rows through a
    // wave-uniform address, i.e. scalar loads into scalar registers.
    const int slot0 = __builtin_amdgcn_readfirstlane(slot);
    if (__ballot(slot != slot0) == 0ull) {
        for (int i = i_begin; i < i_end; ++i) project_into(i, slot0);
    } else {
        for (int i = i_begin; i < i_end; ++i) project_into(i, slot);
    }
}

// ---------------------------------------------------------------- scene upload
template <int ST>
__global__ __launch_bounds__(256) void k_scene_convert(int64_t n, int64_t n_pad, int degree, const float* means,
                                                       const float* scales, const float* quats, const float* opac,
                                                       const float* sh, float4* pos, void* rot, float4* scale,
                                                       void* sh_planes)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n) return;
    const int K = (degree + 1) * (degree + 1);
    const float* f = sh + (size_t)g * 3 * K;
    if (ST == kF32) {
        pos[g] = make_float4(means[3 * g], means[3 * g + 1], means[3 * g + 2], opac[g]);
        ((float4*)rot)[g] = make_float4(quats[4 * g], quats[4 * g + 1], quats[4 * g + 2], quats[4 * g + 3]);
        scale[g] = make_float4(scales[3 * g], scales[3 * g + 1], scales[3 * g + 2], 0.0f);
        const int nch = (3 * K + 3) / 4;
        for (int j = 0; j < nch; ++j) {
            float v[4];
            for (int k = 0; k < 4; ++k) v[k] = (4 * j + k < 3 * K) ? f[4 * j + k] : 0.0f;
            ((float4*)sh_planes)[(size_t)j * n_pad + g] = make_float4(v[0], v[1], v[2], v[3]);
        }
    } else {
        const uint16_t hop = encode<ST>(opac[g]);
        pos[g] = make_float4(means[3 * g], means[3 * g + 1], means[3 * g + 2], decode<ST>(hop));
        uint16_t h[8];
        for (int k = 0; k < 4; ++k) h[k] = encode<ST>(quats[4 * g + k]);
        for (int k = 0; k < 3; ++k) h[4 + k] = encode<ST>(scales[3 * g + k]);
        h[7] = 0;
        ((uint4*)rot)[g] = make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                                      h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
        const int nch = (3 * K + 7) / 8;
        for (int j = 0; j < nch; ++j) {
            uint32_t w[4];
            for (int k = 0; k < 4; ++k) {
                const int a = 8 * j + 2 * k, b = a + 1;
                const uint16_t lo = a < 3 * K ? encode<ST>(f[a]) : 0;
                const uint16_t hi = b < 3 * K ? encode<ST>(f[b]) : 0;
                w[k] = lo | ((uint32_t)hi << 16);
            }
            ((uint4*)sh_planes)[(size_t)j * n_pad + g] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

}  // namespace

hipError_t launch_compose(const SceneDev& s, const ChunkDev& c, const float* viewmats, const float* poses,
                          hipStream_t stream)
{
    const int total = c.n_img * (s.n_bodies + 1);
    hipLaunchKernelGGL(k_compose, dim3((total + 255) / 256), dim3(256), 0, stream, s, c, viewmats, poses);
    return hipGetLastError();
}

template <int ST>
static hipError_t project_st(const SceneDev& s, const ChunkDev& c, int ts, float cutoff, int ipt, hipStream_t st)
{
    const dim3 grid((unsigned)((s.n + 255) / 256), (unsigned)((c.n_img + ipt - 1) / ipt));
    switch (s.degree) {
    case 0: hipLaunchKernelGGL((k_project<ST, 0>), grid, dim3(256), 0, st, s, c, c.img, c.xform, ts, cutoff, ipt); break;
    case 1: hipLaunchKernelGGL((k_project<ST, 1>), grid, dim3(256), 0, st, s, c, c.img, c.xform, ts, cutoff, ipt); break;
    case 2: hipLaunchKernelGGL((k_project<ST, 2>), grid, dim3(256), 0, st, s, c, c.img, c.xform, ts, cutoff, ipt); break;
    default: hipLaunchKernelGGL((k_project<ST, 3>), grid, dim3(256), 0, st, s, c, c.img, c.xform, ts, cutoff, ipt); break;
    }
    return hipGetLastError();
}

hipError_t launch_project(const SceneDev& s, const ChunkDev& c, int ts, float cutoff, int ipt, hipStream_t stream)
{
    if (s.n == 0 || c.n_img == 0) return hipSuccess;
    // small chunks (serving requests of a few dozen images) spread their
    // images over more threads: a thread's images run one after another
    ipt = std::max(1, std::min(ipt, c.n_img / 32));
    if (s.storage == kF16) return project_st<kF16>(s, c, ts, cutoff, ipt, stream);
    if (s.storage == kBF16) return project_st<kBF16>(s, c, ts, cutoff, ipt, stream);
    return project_st<kF32>(s, c, ts, cutoff, ipt, stream);
}

hipError_t launch_scene_convert(int storage, int64_t n, int64_t n_pad, int degree, const float* means,
                                const float* scales, const float* quats, const float* opac, const float* sh,
                                float4* pos, void* rot, float4* scale, void* sh_planes, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (storage == kF16)
        hipLaunchKernelGGL(k_scene_convert<kF16>, grid, dim3(256), 0, stream, n, n_pad, degree, means, scales,
                           quats, opac, sh, pos, rot, scale, sh_planes);
    else if (storage == kBF16)
        hipLaunchKernelGGL(k_scene_convert<kBF16>, grid, dim3(256), 0, stream, n, n_pad, degree, means, scales,
                           quats, opac, sh, pos, rot, scale, sh_planes);
    else
        hipLaunchKernelGGL(k_scene_convert<kF32>, grid, dim3(256), 0, stream, n, n_pad, degree, means, scales,
                           quats, opac, sh, pos, rot, scale, sh_planes);
    return hipGetLastError();
}

}  // namespace gsr
