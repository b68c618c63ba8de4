// Segmented, stable LSD radix sort of each image's visible Gaussians by the
// 32-bit pattern of their camera-space depth (the low word of the 64-bit
// (tile, depth) key; depth > near > 0, so the float bits order like the
// values).  Values are Gaussian indices.  Pass 0 reads the dense per-image
// key array in index order and drops culled entries, so equal depths keep
// ascending index -- the tie rule of the key sort.
//
// Per pass (8-bit digit): a histogram kernel, a per-image scan kernel and a
// scatter kernel.  No block waits on another block.  Local ranks inside a
// block are stable: each wave owns a contiguous quarter of the block's items,
// walks it in order 64 items at a time, and ranks equal digits with a ballot
// match (peers = lanes with the same digit) and a per-wave running counter in
// LDS.  The scatter first places the block's items in LDS in their stable
// digit order, then writes them out in that order, so each digit's run of
// the block leaves as consecutive addresses.
#include "gsr_internal.h"
#include "gsr_wave.h"

namespace gsr {
namespace {

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = __lane_id();
    return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// Lanes whose `key` equals this lane's, among lanes with `active` set.
template <int BITS>
__device__ __forceinline__ uint64_t match_bits(uint32_t key, bool active)
{
    uint64_t peers = __ballot(active);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (key >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// Exclusive scan over the 256 threads of a block; returns the block total.
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

template <bool FIRST>
__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ counts,
                                                   uint64_t n, int shift, uint32_t* __restrict__ hist, int blocks)
{
    __shared__ uint32_t h[256];
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), b = (int)(L - (uint32_t)i * gridDim.x), tid = threadIdx.x;
    const uint64_t cnt = FIRST ? n : counts[i];
    const uint64_t base = (uint64_t)b * kSortItems;
    if (base >= cnt) return;            // block-uniform: no barrier skipped by part of the block
    h[tid] = 0;
    __syncthreads();
    const uint32_t* kin = keys + (size_t)i * n;
    // all loads first, then the LDS atomics: each thread's loads overlap
    uint32_t key[kSortIpt];
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint64_t idx = base + (uint64_t)k * 256 + tid;
        key[k] = idx < cnt ? kin[idx] : kInvalidKey;
    }
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint64_t idx = base + (uint64_t)k * 256 + tid;
        if (idx < cnt && (!FIRST || key[k] != kInvalidKey)) atomicAdd(&h[(key[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[((size_t)i * blocks + b) * 256 + tid] = h[tid];
}

// Per image: digit-major, block-minor exclusive offsets (in place).  Pass 0
// also records the number of visible Gaussians.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t* __restrict__ hist, int blocks, uint32_t* __restrict__ counts,
                                                   uint64_t n)
{
    __shared__ uint32_t lds8[8];
    const int i = blockIdx.x, d = threadIdx.x;
    const uint64_t cnt = FIRST ? n : counts[i];
    const int nb = (int)((cnt + kSortItems - 1) / kSortItems);
    uint32_t* H = hist + (size_t)i * blocks * 256;
    uint32_t tot = 0;
    for (int b = 0; b < nb; ++b) tot += H[(size_t)b * 256 + d];
    uint32_t total;
    uint32_t run = block_excl_scan256(tot, &total, lds8);
    if (FIRST && d == 0) counts[i] = total;
    // offsets in place, 16 blocks at a time: the loads of a group are all
    // complete (one wait) before its stores
    for (int b0 = 0; b0 < nb; b0 += 16) {
        uint32_t v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = b0 + q < nb ? H[(size_t)(b0 + q) * 256 + d] : 0u;
        __builtin_amdgcn_s_waitcnt(0x0F70);     // vmcnt(0)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (b0 + q < nb) H[(size_t)(b0 + q) * 256 + d] = run;
            run += v[q];
        }
    }
}

// Write-out of the last pass: the values, and each Gaussian's tile rectangle
// gathered by its id into depth order.  Every gather of a thread is issued
// before its first store, so the loads (random ids, mostly L2 hits) overlap
// instead of each waiting out its own latency.  The final keys are not read
// again and are not written.
template <typename R>
__device__ __forceinline__ void write_last(const uint32_t* skey, const uint32_t* sval, const uint32_t* lstart,
                                           const uint32_t* gbase, uint32_t n_items, int shift, uint64_t n, size_t seg,
                                           uint32_t* __restrict__ vout, const R* __restrict__ rect,
                                           R* __restrict__ srect, uint32_t* __restrict__ err)
{
    constexpr int kPer = kSortItems / 256;
    const uint32_t tid = threadIdx.x;
    uint32_t pos[kPer], val[kPer];
    R r[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t t = tid + 256u * (uint32_t)q;
        pos[q] = 0xFFFFFFFFu;
        val[q] = 0u;
        r[q] = R{};
        if (t < n_items) {
            const uint32_t k = skey[t], v = sval[t];
            const uint32_t dg = (k >> shift) & 255u;
            const uint32_t p = gbase[dg] + (t - lstart[dg]);
            if (p >= n) atomicOr(err, kErrSortSlot);     // offsets are consistent by construction
            if (p < n) {
                pos[q] = p;
                val[q] = v;
                if (v < n) r[q] = rect[seg + v];
            }
        }
    }
    // one wait for all of them (vmcnt(0); the compiler would otherwise wait
    // before each store, as loads and stores share the counter)
    __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (pos[q] == 0xFFFFFFFFu) continue;
        vout[seg + pos[q]] = val[q];
        if (val[q] < n) srect[seg + pos[q]] = r[q];
    }
}

// LAST: also gathers each Gaussian's tile rectangle into depth order (once,
// so later stages read rectangles contiguously), and writes only the values:
// later stages read the depth order, not the keys.
template <bool FIRST, bool LAST>
__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                      uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                      const uint32_t* __restrict__ counts, uint64_t n, int shift,
                                                      const uint32_t* __restrict__ hist, int blocks,
                                                      const uint2* __restrict__ rect, uint2* __restrict__ srect,
                                                      int rect4, uint32_t* __restrict__ err)
{
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t lstart[256], gbase[256], lds8[8];
    __shared__ uint32_t skey[kSortItems], sval[kSortItems];
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), b = (int)(L - (uint32_t)i * gridDim.x), tid = threadIdx.x;
    const int w = tid >> 6, lane = __lane_id();
    const uint64_t count = FIRST ? n : counts[i];
    const uint64_t base = (uint64_t)b * kSortItems;
    if (base >= count) return;          // block-uniform
    const size_t seg = (size_t)i * n;

    uint32_t key[kSortIpt], val[kSortIpt];
    bool ok[kSortIpt];
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint64_t idx = base + (uint64_t)w * (kSortIpt * 64) + (uint64_t)k * 64 + lane;
        ok[k] = idx < count;
        key[k] = ok[k] ? kin[seg + idx] : kInvalidKey;
        if (FIRST) {
            ok[k] = ok[k] && key[k] != kInvalidKey;
            val[k] = (uint32_t)idx;
        } else {
            val[k] = ok[k] ? vin[seg + idx] : 0u;
        }
    }
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) cnt[ww][tid] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k)
        if (ok[k]) atomicAdd(&cnt[w][(key[k] >> shift) & 255u], 1u);
    __syncthreads();
    // block-local layout: digit-major, and within a digit wave-major, each
    // wave's items in order -- the stable order of the block's items
    uint32_t n_items;
    {
        const uint32_t c0 = cnt[0][tid], c1 = cnt[1][tid], c2 = cnt[2][tid], c3 = cnt[3][tid];
        const uint32_t start = block_excl_scan256(c0 + c1 + c2 + c3, &n_items, lds8);
        lstart[tid] = start;
        gbase[tid] = hist[((size_t)i * blocks + b) * 256 + tid];
        cnt[0][tid] = start;
        cnt[1][tid] = start + c0;
        cnt[2][tid] = start + c0 + c1;
        cnt[3][tid] = start + c0 + c1 + c2;
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint32_t dg = (key[k] >> shift) & 255u;
        const uint64_t peers = match_bits<8>(dg, ok[k]);
        if (ok[k]) {
            const uint32_t basev = cnt[w][dg];
            const uint32_t lpos = basev + (uint32_t)__popcll(peers & lt);
            if (lane == __ffsll((unsigned long long)peers) - 1) cnt[w][dg] = basev + (uint32_t)__popcll(peers);
            if (lpos < (uint32_t)kSortItems) {     // lpos < n_items <= kSortItems by construction
                skey[lpos] = key[k];
                sval[lpos] = val[k];
            } else {
                atomicOr(err, kErrSortSlot);
            }
        }
    }
    __syncthreads();
    // write out in block-local order: consecutive threads write consecutive
    // addresses inside each digit's run
    if (LAST) {
        if (rect4) write_last(skey, sval, lstart, gbase, n_items, shift, n, seg, vout,
                              reinterpret_cast<const uint32_t*>(rect), reinterpret_cast<uint32_t*>(srect), err);
        else write_last(skey, sval, lstart, gbase, n_items, shift, n, seg, vout, rect, srect, err);
        return;
    }
    for (uint32_t t = (uint32_t)tid; t < n_items; t += 256u) {
        const uint32_t k = skey[t], v = sval[t];
        const uint32_t dg = (k >> shift) & 255u;
        const uint32_t pos = gbase[dg] + (t - lstart[dg]);
        if (pos >= n) atomicOr(err, kErrSortSlot);     // offsets are consistent by construction
        if (pos < n) {
            kout[seg + pos] = k;
            vout[seg + pos] = v;
        }
    }
}

}  // namespace

hipError_t launch_depth_sort(const SceneDev& s, const ChunkDev& c, hipStream_t stream)
{
    if (s.n == 0 || c.n_img == 0) return hipSuccess;
    const uint64_t n = (uint64_t)s.n;
    const dim3 grid((unsigned)c.sort_blocks, (unsigned)c.n_img);
    // pass 0: dense keys (index order) -> compacted, digit 0
    hipLaunchKernelGGL(k_sort_hist<true>, grid, dim3(256), 0, stream, c.keyz, c.vis_count, n, 0, c.sort_hist,
                       c.sort_blocks);
    hipLaunchKernelGGL(k_sort_scan<true>, dim3(c.n_img), dim3(256), 0, stream, c.sort_hist, c.sort_blocks,
                       c.vis_count, n);
    hipLaunchKernelGGL((k_sort_scatter<true, false>), grid, dim3(256), 0, stream, c.keyz, (const uint32_t*)nullptr,
                       c.sk[0], c.sv[0], c.vis_count, n, 0, c.sort_hist, c.sort_blocks, c.rect, c.srect, c.rect4,
                       c.err);
    int src = 0;
    for (int pass = 1; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist<false>, grid, dim3(256), 0, stream, c.sk[src], c.vis_count, n, shift,
                           c.sort_hist, c.sort_blocks);
        hipLaunchKernelGGL(k_sort_scan<false>, dim3(c.n_img), dim3(256), 0, stream, c.sort_hist, c.sort_blocks,
                           c.vis_count, n);
        if (pass == 3)
            hipLaunchKernelGGL((k_sort_scatter<false, true>), grid, dim3(256), 0, stream, c.sk[src], c.sv[src],
                               c.sk[src ^ 1], c.sv[src ^ 1], c.vis_count, n, shift, c.sort_hist, c.sort_blocks, c.rect,
                               c.srect, c.rect4, c.err);
        else
            hipLaunchKernelGGL((k_sort_scatter<false, false>), grid, dim3(256), 0, stream, c.sk[src], c.sv[src],
                               c.sk[src ^ 1], c.sv[src ^ 1], c.vis_count, n, shift, c.sort_hist, c.sort_blocks,
                               c.rect, c.srect, c.rect4, c.err);
        src ^= 1;
    }
    // pass 0 wrote buffer 0; passes 1..3 alternate, so the sorted values are in sv[1] (the last
    // pass writes no keys)
    return hipGetLastError();
}

}  // namespace gsr
