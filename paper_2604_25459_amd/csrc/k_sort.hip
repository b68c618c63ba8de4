// Segmented, stable LSD radix sort of each image's visible Gaussians by the
// 32-bit pattern of their camera-space depth (the low word of the 64-bit
// (tile, depth) key; depth > near > 0, so the float bits order like the
// values).  Values are Gaussian indices.  Pass 0 reads the dense per-image
// key array in index order and drops culled entries, so equal depths keep
// ascending index -- the tie rule of the key sort.
//
// The sort runs on the key less the image's smallest visible key (rounded
// down to a multiple of 512; the first pass's histogram blocks record their
// key ranges and its scan combines them), in 9-bit digits: three passes
// order an image whose keys lie within 2^27 of that offset (depths within a
// factor of about 2^16), a fourth pass (the top five bits) runs only for
// images that need it.  The two ping-pong buffers are
// used in opposite order by three- and four-pass images, so every image's
// sorted values end in sv[0].
//
// Per pass: a histogram kernel, a per-image scan kernel and a scatter
// kernel.  No block waits on another block.  Local ranks inside a block are
// stable: each wave owns a contiguous quarter of the block's items, walks it
// in order 64 items at a time, and ranks equal digits with a ballot match
// (peers = lanes with the same digit) and a per-wave running counter in LDS.
// The scatter first places the block's items in LDS in their stable digit
// order, then writes them out in that order, so each digit's run of the
// block leaves as consecutive addresses.
#include "gsr_internal.h"
#include "gsr_wave.h"

namespace gsr {
namespace {

constexpr int kBits = 9;
constexpr int kRadix = 1 << kBits;               // 512 digits
constexpr int kDpt = kRadix / 256;               // digits per thread
constexpr uint32_t kDigitMask = kRadix - 1;
constexpr uint32_t kNarrowSpan = 1u << (3 * kBits);  // key span that three passes cover

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = __lane_id();
    return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// Lanes whose `key` equals this lane's in its low BITS bits, among lanes
// with `active` set: one ballot per bit; a lane differs from this one where
// the ballot differs from this lane's bit (the bit spread to a whole word),
// and the differences of all bits are ORed (three VALU per bit and half).
template <int BITS>
__device__ __forceinline__ uint64_t match_bits(uint32_t key, bool active)
{
    uint32_t dlo = 0u, dhi = 0u;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int)key, b, 1);   // 0 or all ones
        const uint64_t m = __builtin_amdgcn_uicmp(s, 0u, 33);                // ballot of s != 0
        dlo |= (uint32_t)m ^ s;
        dhi |= (uint32_t)(m >> 32) ^ s;
    }
    return __ballot(active) & ~(((uint64_t)dhi << 32) | dlo);
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

// Image i's keys span more than three passes cover (kmm: smallest, largest
// visible key per image; an image with no visible Gaussian has smallest >
// largest and needs no pass at all).
__device__ __forceinline__ bool wide_image(const uint32_t* kmm, int i)
{
    const uint32_t lo = kmm[kKmmStride * i], hi = kmm[kKmmStride * i + 1];
    return hi >= lo && hi - lo >= kNarrowSpan;
}
// Buffer written by pass p of an image (three-pass images: 0, 1, 0; four-pass
// images: 1, 0, 1, 0 -- the sorted values land in sv[0] either way).
__device__ __forceinline__ int out_buf(int pass, bool wide) { return (pass + (wide ? 1 : 0)) & 1; }

// Per-block digit counts of pass `pass`.  FIRST: the dense keys, culled
// entries dropped; the image's smallest key is not known yet, but it is
// taken rounded down to a multiple of 512, so the lowest digit of a key less
// it is the key's own lowest digit; the block also records its smallest and
// largest visible key (kblk) for the scan to combine.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t* __restrict__ k0, const uint32_t* __restrict__ k1,
                                                   const uint32_t* __restrict__ counts,
                                                   const uint32_t* __restrict__ kmm, uint64_t n, int pass,
                                                   uint32_t* __restrict__ hist, int blocks, uint32_t* __restrict__ kblk)
{
    __shared__ uint32_t h[kRadix];
    __shared__ uint32_t red[8];
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), b = (int)(L - (uint32_t)i * gridDim.x), tid = threadIdx.x;
    const bool wide = !FIRST && wide_image(kmm, i);
    if (pass == 3 && !wide) return;     // block-uniform: three passes order this image
    const uint64_t cnt = FIRST ? n : counts[i];
    const uint64_t base = (uint64_t)b * kSortItems;
    if (base >= cnt) return;            // block-uniform: no barrier skipped by part of the block
#pragma unroll
    for (int q = 0; q < kDpt; ++q) h[tid + 256 * q] = 0;
    __syncthreads();
    const uint32_t* kin = (FIRST || out_buf(pass - 1, wide) == 0 ? k0 : k1) + (size_t)i * n;
    const int shift = kBits * pass;
    // all loads first, then the LDS atomics: each thread's loads overlap
    uint32_t key[kSortIpt];
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint64_t idx = base + (uint64_t)k * 256 + tid;
        key[k] = idx < cnt ? kin[idx] : kInvalidKey;
    }
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint64_t idx = base + (uint64_t)k * 256 + tid;
        if (idx < cnt && (!FIRST || key[k] != kInvalidKey)) {
            atomicAdd(&h[(key[k] >> shift) & kDigitMask], 1u);
            kmin = min(kmin, key[k]);
            kmax = max(kmax, key[k]);
        }
    }
    if (FIRST) {
        // the wave's smallest and largest visible key (prefix maxima of the key and its complement)
        const uint32_t hi = wave_last(wave_incl_max(kmax)), lo = ~wave_last(wave_incl_max(~kmin));
        if (__lane_id() == 0) {
            red[2 * (tid >> 6)] = lo;
            red[2 * (tid >> 6) + 1] = hi;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kDpt; ++q) hist[((size_t)i * blocks + b) * kRadix + tid + 256 * q] = h[tid + 256 * q];
    if (FIRST && tid == 0) {
        kblk[((size_t)i * blocks + b) * 2] = min(min(red[0], red[2]), min(red[4], red[6]));
        kblk[((size_t)i * blocks + b) * 2 + 1] = max(max(red[1], red[3]), max(red[5], red[7]));
    }
}

// Per image: digit-major, block-minor exclusive offsets (in place).  Pass 0
// also records the number of visible Gaussians.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t* __restrict__ hist, int blocks, uint32_t* __restrict__ counts,
                                                   uint32_t* __restrict__ kmm, uint64_t n, int pass,
                                                   const uint32_t* __restrict__ kblk)
{
    __shared__ uint32_t lds8[8], red[8];
    const int i = blockIdx.x, d = threadIdx.x;
    if (pass == 3 && !wide_image(kmm, i)) return;
    const uint64_t cnt = FIRST ? n : counts[i];
    const int nb = (int)((cnt + kSortItems - 1) / kSortItems);
    if (FIRST) {
        // the image's key range from its blocks' ranges; the smallest key is
        // kept rounded down to a multiple of 512 (see k_sort_hist)
        uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
        for (int b = d; b < nb; b += 256) {
            kmin = min(kmin, kblk[((size_t)i * blocks + b) * 2]);
            kmax = max(kmax, kblk[((size_t)i * blocks + b) * 2 + 1]);
        }
        const uint32_t hi = wave_last(wave_incl_max(kmax)), lo = ~wave_last(wave_incl_max(~kmin));
        if (__lane_id() == 0) {
            red[2 * (d >> 6)] = lo;
            red[2 * (d >> 6) + 1] = hi;
        }
        __syncthreads();
        if (d == 0) {
            const uint32_t l = min(min(red[0], red[2]), min(red[4], red[6]));
            kmm[kKmmStride * i] = l <= max(max(red[1], red[3]), max(red[5], red[7])) ? (l & ~kDigitMask) : l;
            kmm[kKmmStride * i + 1] = max(max(red[1], red[3]), max(red[5], red[7]));
        }
    }
    uint32_t* H = hist + (size_t)i * blocks * kRadix;
    // thread d owns digits d and d + 256: the scan runs over the first half,
    // then over the second half after the first half's total
    uint32_t tot[kDpt] = {};
    for (int b = 0; b < nb; ++b)
#pragma unroll
        for (int q = 0; q < kDpt; ++q) tot[q] += H[(size_t)b * kRadix + d + 256 * q];
    uint32_t run[kDpt], all = 0;
#pragma unroll
    for (int q = 0; q < kDpt; ++q) {
        uint32_t total;
        run[q] = all + block_excl_scan256(tot[q], &total, lds8);
        all += total;
    }
    if (FIRST && d == 0) counts[i] = all;
    // offsets in place, 16 blocks at a time: the loads of a group are all
    // complete (one wait) before its stores
    for (int b0 = 0; b0 < nb; b0 += 16) {
        uint32_t v[16][kDpt];
#pragma unroll
        for (int q = 0; q < 16; ++q)
#pragma unroll
            for (int r = 0; r < kDpt; ++r) v[q][r] = b0 + q < nb ? H[(size_t)(b0 + q) * kRadix + d + 256 * r] : 0u;
        __builtin_amdgcn_s_waitcnt(0x0F70);     // vmcnt(0)
#pragma unroll
        for (int q = 0; q < 16; ++q)
#pragma unroll
            for (int r = 0; r < kDpt; ++r) {
                if (b0 + q < nb) H[(size_t)(b0 + q) * kRadix + d + 256 * r] = run[r];
                run[r] += v[q][r];
            }
    }
}

template <typename R>
__device__ __forceinline__ void write_last(const uint32_t* skey, const uint32_t* sval, const uint32_t* delta,
                                           uint32_t n_items, int shift, uint64_t n, size_t seg,
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
            const uint32_t dg = (k >> shift) & kDigitMask;
            const uint32_t p = delta[dg] + t;
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

// Scatter of pass `pass`.  The last pass of an image (pass 2, or 3 for a
// four-pass image) also gathers each Gaussian's tile rectangle into depth
// order (once, so later stages read rectangles contiguously) and writes only
// the values: later stages read the depth order, not the keys.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t* __restrict__ keyz, uint32_t* sk0, uint32_t* sk1,
                                                      uint32_t* sv0, uint32_t* sv1, const uint32_t* __restrict__ counts,
                                                      const uint32_t* __restrict__ kmm, uint64_t n, int pass,
                                                      const uint32_t* __restrict__ hist, int blocks,
                                                      const uint2* __restrict__ rect, uint2* __restrict__ srect,
                                                      int rect4, uint32_t* __restrict__ err)
{
    // per-wave digit counts, then per-wave running positions, as 16-bit
    // halves (a wave counts at most 1024 items, a block places 4096): with
    // one offset per digit the block's LDS fits four blocks per CU
    __shared__ uint32_t cnt32[4][kRadix / 2];
    __shared__ uint32_t delta[kRadix], lds8[8];          // global position - block-local position, per digit
    __shared__ uint32_t skey[kSortItems], sval[kSortItems];
    uint16_t (*cnt)[kRadix] = reinterpret_cast<uint16_t (*)[kRadix]>(cnt32);
    const uint32_t L = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int i = (int)(L / gridDim.x), b = (int)(L - (uint32_t)i * gridDim.x), tid = threadIdx.x;
    const int w = tid >> 6, lane = __lane_id();
    const bool wide = wide_image(kmm, i);
    if (pass == 3 && !wide) return;     // block-uniform
    const bool last = pass == (wide ? 3 : 2);
    const uint64_t count = FIRST ? n : counts[i];
    const uint64_t base = (uint64_t)b * kSortItems;
    if (base >= count) return;          // block-uniform
    const size_t seg = (size_t)i * n;
    // this image's input and output buffers of the pass (never the same)
    const int ib = FIRST ? 0 : out_buf(pass - 1, wide), ob = out_buf(pass, wide);
    const uint32_t* kin = FIRST ? keyz : (ib ? sk1 : sk0);
    const uint32_t* vin = ib ? sv1 : sv0;
    uint32_t* kout = ob ? sk1 : sk0;
    uint32_t* vout = ob ? sv1 : sv0;
    const uint32_t lo = FIRST ? kmm[kKmmStride * i] : 0u;
    const int shift = kBits * pass;

    uint32_t key[kSortIpt], val[kSortIpt];
    bool ok[kSortIpt];
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint64_t idx = base + (uint64_t)w * (kSortIpt * 64) + (uint64_t)k * 64 + lane;
        ok[k] = idx < count;
        key[k] = ok[k] ? kin[seg + idx] : kInvalidKey;
        if (FIRST) {
            ok[k] = ok[k] && key[k] != kInvalidKey;
            key[k] = key[k] - lo;               // sorted from here on relative to the smallest key
            val[k] = (uint32_t)idx;
        } else {
            val[k] = ok[k] ? vin[seg + idx] : 0u;
        }
    }
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) cnt32[ww][tid] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k)
        if (ok[k]) {
            const uint32_t dg = (key[k] >> shift) & kDigitMask;
            atomicAdd(&cnt32[w][dg >> 1], 1u << (16 * (dg & 1u)));
        }
    __syncthreads();
    // block-local layout: digit-major, and within a digit wave-major, each
    // wave's items in order -- the stable order of the block's items.  Thread
    // tid owns digits tid and tid + 256 (scanned half after half).
    uint32_t n_items = 0;
#pragma unroll
    for (int q = 0; q < kDpt; ++q) {
        const int dg = tid + 256 * q;
        const uint32_t c0 = cnt[0][dg], c1 = cnt[1][dg], c2 = cnt[2][dg], c3 = cnt[3][dg];
        uint32_t total;
        const uint32_t start = n_items + block_excl_scan256(c0 + c1 + c2 + c3, &total, lds8);
        n_items += total;
        delta[dg] = hist[((size_t)i * blocks + b) * kRadix + dg] - start;
        cnt[0][dg] = (uint16_t)start;
        cnt[1][dg] = (uint16_t)(start + c0);
        cnt[2][dg] = (uint16_t)(start + c0 + c1);
        cnt[3][dg] = (uint16_t)(start + c0 + c1 + c2);
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < kSortIpt; ++k) {
        const uint32_t dg = (key[k] >> shift) & kDigitMask;
        const uint64_t peers = match_bits<kBits>(dg, ok[k]);
        if (ok[k]) {
            const uint32_t basev = cnt[w][dg];
            const uint32_t lpos = basev + (uint32_t)__popcll(peers & lt);
            if (lane == __ffsll((unsigned long long)peers) - 1) cnt[w][dg] = (uint16_t)(basev + (uint32_t)__popcll(peers));
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
    if (last) {
        if (rect4) write_last(skey, sval, delta, n_items, shift, n, seg, vout,
                              reinterpret_cast<const uint32_t*>(rect), reinterpret_cast<uint32_t*>(srect), err);
        else write_last(skey, sval, delta, n_items, shift, n, seg, vout, rect, srect, err);
        return;
    }
    for (uint32_t t = (uint32_t)tid; t < n_items; t += 256u) {
        const uint32_t k = skey[t], v = sval[t];
        const uint32_t dg = (k >> shift) & kDigitMask;
        const uint32_t pos = delta[dg] + t;
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
    // pass 0: dense keys (index order) -> compacted keys relative to the image's smallest, digit 0
    hipLaunchKernelGGL(k_sort_hist<true>, grid, dim3(256), 0, stream, c.keyz, (const uint32_t*)nullptr, c.vis_count,
                       c.kmm, n, 0, c.sort_hist, c.sort_blocks, c.kblk);
    hipLaunchKernelGGL(k_sort_scan<true>, dim3(c.n_img), dim3(256), 0, stream, c.sort_hist, c.sort_blocks,
                       c.vis_count, c.kmm, n, 0, (const uint32_t*)c.kblk);
    hipLaunchKernelGGL(k_sort_scatter<true>, grid, dim3(256), 0, stream, c.keyz, c.sk[0], c.sk[1], c.sv[0], c.sv[1],
                       c.vis_count, c.kmm, n, 0, c.sort_hist, c.sort_blocks, c.rect, c.srect, c.rect4, c.err);
    // passes 1, 2 and (for images whose keys span 2^27 or more) 3; the blocks of
    // images that need no fourth pass leave at once
    for (int pass = 1; pass < 4; ++pass) {
        hipLaunchKernelGGL(k_sort_hist<false>, grid, dim3(256), 0, stream, c.sk[0], c.sk[1], c.vis_count, c.kmm, n,
                           pass, c.sort_hist, c.sort_blocks, c.kblk);
        hipLaunchKernelGGL(k_sort_scan<false>, dim3(c.n_img), dim3(256), 0, stream, c.sort_hist, c.sort_blocks,
                           c.vis_count, c.kmm, n, pass, (const uint32_t*)c.kblk);
        hipLaunchKernelGGL(k_sort_scatter<false>, grid, dim3(256), 0, stream, (const uint32_t*)nullptr, c.sk[0],
                           c.sk[1], c.sv[0], c.sv[1], c.vis_count, c.kmm, n, pass, c.sort_hist, c.sort_blocks, c.rect,
                           c.srect, c.rect4, c.err);
    }
    // every image's sorted values are in sv[0]
    return hipGetLastError();
}

}  // namespace gsr
