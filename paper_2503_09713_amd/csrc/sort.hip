// Stable LSD radix sort of (64-bit Morton key, 32-bit index) pairs.
//
// The paper sorts with a bitonic network (App. E.1) and names onesweep-style
// radix sorting as the faster alternative; this is a radix sort built for
// wave64: 8-bit digits, 4096-key tiles per 256-thread workgroup, per-wave
// digit counters in LDS, and stable in-wave ranking from 8 ballots per key
// (lanes with equal digits are found with 64-bit ballots, ranked with
// popcount).  Each pass: tile histograms -> scan of the digit-major histogram
// -> stable scatter staged through LDS so that each digit run is written to
// HBM contiguously.  Ties keep the input order (stable), so equal keys end
// up ordered by original index.
#include "common.hpp"
#include "kernels.hpp"

namespace shsph {

constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / WAVE;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;      // 4096 keys
constexpr int RS_WTILE = RS_TILE / RS_WAVES;      // 1024 keys per wave

// digit of an element: MODE 0 = bits of the key, MODE 1 = byte of the
// instance id of the element's original index (segmented batches).
template <int MODE>
__device__ inline u32 rs_digit(u64 key, u32 val, int shift, const i64* seg_off, int nseg)
{
    if (MODE == 0) return (u32)(key >> shift) & (RS_BINS - 1);
    u32 s = (u32)find_seg(seg_off, nseg, (i64)val);
    return (s >> shift) & (RS_BINS - 1);
}

template <int MODE>
__global__ void __launch_bounds__(RS_BLOCK)
k_rs_upsweep(const u64* __restrict__ keys, const u32* __restrict__ vals, i64 n, int shift,
             const i64* __restrict__ seg_off, int nseg, u32* __restrict__ hist, int nblocks)
{
    __shared__ u32 h[RS_WAVES][RS_BINS];
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
    for (int d = threadIdx.x; d < RS_WAVES * RS_BINS; d += RS_BLOCK) (&h[0][0])[d] = 0;
    __syncthreads();
    const i64 base = (i64)blockIdx.x * RS_TILE + (i64)wid * RS_WTILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        const i64 i = base + (i64)it * WAVE + lane;
        const bool valid = i < n;
        u32 d = 0;
        if (valid) d = rs_digit<MODE>(keys[i], MODE ? vals[i] : 0u, shift, seg_off, nseg);
        const u64 active = __ballot(valid);
        if (!active) break;
        const u64 m = match_digit<RS_BITS>(d, active);
        const int leader = __ffsll((unsigned long long)m) - 1;
        if (valid && lane == leader) h[wid][d] += (u32)__popcll(m);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RS_BINS; d += RS_BLOCK) {
        u32 s = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) s += h[w][d];
        hist[(i64)d * nblocks + blockIdx.x] = s;
    }
}

template <int MODE>
__global__ void __launch_bounds__(RS_BLOCK)
k_rs_downsweep(const u64* __restrict__ kin, const u32* __restrict__ vin, u64* __restrict__ kout,
               u32* __restrict__ vout, i64 n, int shift, const i64* __restrict__ seg_off, int nseg,
               const u32* __restrict__ gofs, int nblocks)
{
    __shared__ u64 sk[RS_TILE];
    __shared__ u32 sv[RS_TILE];
    __shared__ u32 wh[RS_WAVES][RS_BINS];
    __shared__ u32 bstart[RS_BINS];
    __shared__ u32 gbase[RS_BINS];
    __shared__ u32 scr[RS_BLOCK / WAVE];
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
    for (int d = threadIdx.x; d < RS_WAVES * RS_BINS; d += RS_BLOCK) (&wh[0][0])[d] = 0;
    __syncthreads();

    const i64 tile0 = (i64)blockIdx.x * RS_TILE;
    const i64 base = tile0 + (i64)wid * RS_WTILE;
    u64 key[RS_ITEMS];
    u32 val[RS_ITEMS];
    u32 pos[RS_ITEMS];
    u32 dig[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const i64 i = base + (i64)it * WAVE + lane;
        const bool valid = i < n;
        key[it] = valid ? kin[i] : 0;
        val[it] = valid ? vin[i] : 0;
        dig[it] = valid ? rs_digit<MODE>(key[it], val[it], shift, seg_off, nseg) : 0;
        const u64 active = __ballot(valid);
        const u64 m = match_digit<RS_BITS>(dig[it], active);
        const int leader = __ffsll((unsigned long long)m) - 1;
        const u32 prev = wh[wid][dig[it]];
        pos[it] = prev + (u32)__popcll(m & lanemask_lt());
        if (valid && lane == leader) wh[wid][dig[it]] = prev + (u32)__popcll(m);
    }
    __syncthreads();
    // digit totals over the waves -> per-wave prefix and block digit start
    {
        const int d = threadIdx.x;          // RS_BLOCK == RS_BINS
        u32 run = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) { u32 c = wh[w][d]; wh[w][d] = run; run += c; }
        u32 tot;
        u32 st = block_excl_scan<RS_BLOCK>(run, scr, tot);
        bstart[d] = st;
        gbase[d] = gofs[(i64)d * nblocks + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const i64 i = base + (i64)it * WAVE + lane;
        if (i < n) {
            const u32 p = bstart[dig[it]] + wh[wid][dig[it]] + pos[it];
            sk[p] = key[it];
            sv[p] = val[it];
        }
    }
    __syncthreads();
    const i64 cnt = (n - tile0) < RS_TILE ? (n - tile0) : RS_TILE;
    for (int j = threadIdx.x; j < cnt; j += RS_BLOCK) {
        const u64 k = sk[j];
        const u32 v = sv[j];
        const u32 d = rs_digit<MODE>(k, v, shift, seg_off, nseg);
        const i64 o = (i64)gbase[d] + (j - (i64)bstart[d]);
        kout[o] = k;
        vout[o] = v;
    }
}

size_t radix_hist_count(i64 n)
{
    i64 nb = (n + RS_TILE - 1) / RS_TILE;
    if (nb == 0) nb = 1;
    return (size_t)nb * RS_BINS;
}

// Sorts (keys, vals) over key bits [0, key_bits) and then, when nseg > 1,
// stably by the instance id of the original index.  Buffers ping-pong between
// (k0,v0) and (k1,v1); the return value says which pair holds the result
// (0 -> k0/v0, 1 -> k1/v1).
int radix_sort_pairs(u64* k0, u32* v0, u64* k1, u32* v1, i64 n, int key_bits,
                     const i64* seg_off, int nseg, u32* hist, u32* hist_scan, void* scan_tmp,
                     hipStream_t st)
{
    if (n <= 1) return 0;
    const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    const i64 nh = (i64)nblocks * RS_BINS;
    int cur = 0;
    u64* kb[2] = { k0, k1 };
    u32* vb[2] = { v0, v1 };
    auto pass = [&](int mode, int shift) {
        if (mode == 0) {
            hipLaunchKernelGGL((k_rs_upsweep<0>), dim3(nblocks), dim3(RS_BLOCK), 0, st,
                               kb[cur], vb[cur], n, shift, seg_off, nseg, hist, nblocks);
        } else {
            hipLaunchKernelGGL((k_rs_upsweep<1>), dim3(nblocks), dim3(RS_BLOCK), 0, st,
                               kb[cur], vb[cur], n, shift, seg_off, nseg, hist, nblocks);
        }
        scan_u32_u32(hist, hist_scan, nh, scan_tmp, st);
        if (mode == 0) {
            hipLaunchKernelGGL((k_rs_downsweep<0>), dim3(nblocks), dim3(RS_BLOCK), 0, st,
                               kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, shift, seg_off, nseg,
                               hist_scan, nblocks);
        } else {
            hipLaunchKernelGGL((k_rs_downsweep<1>), dim3(nblocks), dim3(RS_BLOCK), 0, st,
                               kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, shift, seg_off, nseg,
                               hist_scan, nblocks);
        }
        cur ^= 1;
    };
    for (int shift = 0; shift < key_bits; shift += RS_BITS) pass(0, shift);
    if (nseg > 1) {
        for (int shift = 0; (1 << shift) < nseg; shift += RS_BITS) pass(1, shift);
    }
    return cur;
}

}  // namespace shsph
