// Device helpers shared by the projection kernels (camera and LiDAR): half
// storage decoding and the binary32 rotation arithmetic of the binning
// specification (one rounding per operation; callers are compiled without
// contraction).
#pragma once

#include <hip/hip_fp16.h>

#include "gsr_internal.h"

namespace gsr {
namespace {

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return __half2float(__ushort_as_half(h)); }

// Round-to-nearest-even float32 -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ uint16_t f32_to_f16(float f) { return __half_as_ushort(__float2half_rn(f)); }

template <int ST>
__device__ __forceinline__ float decode(uint16_t h)
{
    return ST == kBF16 ? bf16_to_f32(h) : f16_to_f32(h);
}
template <int ST>
__device__ __forceinline__ uint16_t encode(float f)
{
    return ST == kBF16 ? f32_to_bf16(f) : f32_to_f16(f);
}

// Rotation matrix of a (w, x, y, z) quaternion, normalised first (spec).
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float R[9])
{
    const float n = sqrtf(((w * w + x * x) + y * y) + z * z);
    w = w / n;
    x = x / n;
    y = y / n;
    z = z / n;
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, xz = x * z, yz = y * z;
    const float wx = w * x, wy = w * y, wz = w * z;
    R[0] = 1.0f - 2.0f * (yy + zz);
    R[1] = 2.0f * (xy - wz);
    R[2] = 2.0f * (xz + wy);
    R[3] = 2.0f * (xy + wz);
    R[4] = 1.0f - 2.0f * (xx + zz);
    R[5] = 2.0f * (yz - wx);
    R[6] = 2.0f * (xz - wy);
    R[7] = 2.0f * (yz + wx);
    R[8] = 1.0f - 2.0f * (xx + yy);
}

// C = A B for row-major 3x3, each entry ((a0 b0 + a1 b1) + a2 b2).
__device__ __forceinline__ void mat3_mul(const float A[9], const float B[9], float C[9])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = (A[3 * i + 0] * B[0 + j] + A[3 * i + 1] * B[3 + j]) + A[3 * i + 2] * B[6 + j];
}

// Scene attributes of Gaussian g: posed-independent quaternion (w, x, y, z)
// and scales, decoded from the storage type.
template <int ST>
__device__ __forceinline__ void load_rot_scale(const SceneDev& s, int64_t g, float q[4], float sc[3])
{
    if (ST == kF32) {
        const float4 qq = ((const float4*)s.rot)[g];
        const float4 ss = s.scale[g];
        q[0] = qq.x; q[1] = qq.y; q[2] = qq.z; q[3] = qq.w;
        sc[0] = ss.x; sc[1] = ss.y; sc[2] = ss.z;
    } else {
        const uint4 hq = ((const uint4*)s.rot)[g];
        q[0] = decode<ST>(hq.x & 0xFFFF); q[1] = decode<ST>(hq.x >> 16);
        q[2] = decode<ST>(hq.y & 0xFFFF); q[3] = decode<ST>(hq.y >> 16);
        sc[0] = decode<ST>(hq.z & 0xFFFF); sc[1] = decode<ST>(hq.z >> 16);
        sc[2] = decode<ST>(hq.w & 0xFFFF);
    }
}

// Body slot of Gaussian g: 0 = static background, b + 1 = body b.
__device__ __forceinline__ int body_slot(const SceneDev& s, int64_t g)
{
    int slot = 0;
    if (s.n_bodies > 0 && g >= s.body_off[0]) {
        int lo = 0, hi = s.n_bodies - 1;        // largest b with off[b] <= g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s.body_off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        slot = lo + 1;
    }
    return slot;
}

// Opacity bucket bound of the alpha >= 1/255 region: for o in
// (2^-(k+1), 2^-k] the bound 1.01 * 2 ln(255 * 2^-k), rounded up to binary32.
__device__ __forceinline__ float opacity_qmax(float op)
{
    int kq = 0;
#pragma unroll
    for (int j = 1; j < 8; ++j) kq += op <= __uint_as_float((uint32_t)(127 - j) << 23) ? 1 : 0;
    constexpr float kQmax[8] = {0x1.662ff2p+3f, 0x1.3961dcp+3f, 0x1.0c93c4p+3f, 0x1.bf8b5cp+2f,
                                0x1.65ef2ep+2f, 0x1.0c5300p+2f, 0x1.656da6p+1f, 0x1.646a94p+0f};
    float qmax = kQmax[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) qmax = kq == j ? kQmax[j] : qmax;
    return qmax;
}

}  // namespace
}  // namespace gsr
