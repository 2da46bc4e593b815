// Stable LSD radix sort of (64-bit Morton key, 32-bit index) pairs.
//
// The paper sorts with a bitonic network (App. E.1) and names onesweep-style
// radix sorting as the faster alternative; this is such a sort built for
// wave64, 8-bit digits:
//   1. one read of all keys computes the digit histograms of every pass
//      (per-block LDS counts added into one global histogram, then scanned);
//   2. one kernel per pass: each 4096-key tile (256 threads x 16) ranks its
//      keys by digit (stable in-wave ranking from 8 ballots per key, per-wave
//      digit counters in LDS), publishes its digit counts, and finds the
//      counts of all earlier tiles by decoupled look-back over their
//      published words; the keys are then staged in LDS in digit order so
//      that each digit run is written to HBM contiguously.
// Tiles are numbered by an atomic ticket taken when a workgroup starts, so a
// tile only ever waits for tiles whose workgroups are already running; the
// wait is bounded all the same (error flag, never an endless loop).
// Ties keep the input order, so equal keys end up ordered by original index.
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
constexpr int RS_HBLOCKS = 1024;                  // histogram workgroups (at most)
constexpr int RS_MAXP = 10;                       // 8 key passes + 2 instance-id passes

// Look-back status word: bits 31..30 kind, 29..0 count (n < 2^30).
constexpr u32 ST_AGG = 1u << 30, ST_PREFIX = 2u << 30, ST_VAL = (1u << 30) - 1u;
constexpr u32 ST_SPIN_LIMIT = 1u << 22;

// digit of an element: MODE 0 = bits of the key, MODE 1 = byte of the
// instance id of the element's original index (segmented batches).
template <int MODE>
__device__ inline u32 rs_digit(u64 key, u32 val, int shift, const i64* seg_off, int nseg)
{
    if (MODE == 0) return (u32)(key >> shift) & (RS_BINS - 1);
    u32 s = (u32)find_seg(seg_off, nseg, (i64)val);
    return (s >> shift) & (RS_BINS - 1);
}

// Adds one element per active lane to bin d of an LDS histogram.  The first
// few distinct digits of the wave are counted with ballots and added once
// each (keys in near-Morton order share their high digits, which would make
// per-lane atomics collide); the lanes left over add one each.
__device__ inline void hist_add(u32* h, u32 d, bool valid)
{
    u64 rem = __ballot(valid);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        if (!rem) return;
        const int l = __ffsll((unsigned long long)rem) - 1;
        const u32 dv = __builtin_amdgcn_readlane(d, l);
        const u64 m = __ballot(d == dv) & rem;
        if (__lane_id() == l) atomicAdd(&h[dv], (u32)__popcll(m));
        rem &= ~m;
    }
    if ((rem >> __lane_id()) & 1ull) atomicAdd(&h[d], 1u);
}

// Digit histograms of all passes: pk key passes (bits 8p .. 8p+7) and ps
// instance-id passes, added into hist[p][bin] (zeroed beforehand).
__global__ void __launch_bounds__(RS_BLOCK)
k_rs_hist(const u64* __restrict__ keys, const u32* __restrict__ vals, i64 n, int pk, int ps,
          const i64* __restrict__ seg_off, int nseg, u32* __restrict__ hist)
{
    __shared__ u32 h[RS_MAXP][RS_BINS];
    const int np = pk + ps;
    for (int d = threadIdx.x; d < np * RS_BINS; d += RS_BLOCK) (&h[0][0])[d] = 0;
    __syncthreads();
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
    const i64 ntiles = (n + RS_TILE - 1) / RS_TILE;
    for (i64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const i64 base = t * RS_TILE + (i64)wid * RS_WTILE;
        u64 key[RS_ITEMS];
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            const i64 i = base + (i64)it * WAVE + lane;
            key[it] = i < n ? keys[i] : 0ull;
        }
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) {
            const i64 i = base + (i64)it * WAVE + lane;
            const bool valid = i < n;
            for (int p = 0; p < pk; ++p) hist_add(h[p], (u32)(key[it] >> (RS_BITS * p)) & (RS_BINS - 1), valid);
            if (ps) {
                const u32 s = valid ? (u32)find_seg(seg_off, nseg, (i64)vals[i]) : 0u;
                for (int p = 0; p < ps; ++p) hist_add(h[pk + p], (s >> (RS_BITS * p)) & (RS_BINS - 1), valid);
            }
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < np * RS_BINS; d += RS_BLOCK) {
        const u32 v = (&h[0][0])[d];
        if (v) atomicAdd(&hist[d], v);
    }
}

// One workgroup per pass: exclusive scan of the pass's digit counts.
__global__ void __launch_bounds__(RS_BLOCK)
k_rs_scan(const u32* __restrict__ hist, u32* __restrict__ base)
{
    __shared__ u32 scr[RS_WAVES];
    const int p = blockIdx.x, d = threadIdx.x;     // RS_BLOCK == RS_BINS
    u32 tot;
    base[p * RS_BINS + d] = block_excl_scan<RS_BLOCK>(hist[p * RS_BINS + d], scr, tot);
}

template <int MODE>
__global__ void __launch_bounds__(RS_BLOCK)
k_rs_pass(const u64* __restrict__ kin, const u32* __restrict__ vin, u64* __restrict__ kout,
          u32* __restrict__ vout, i64 n, int shift, const i64* __restrict__ seg_off, int nseg,
          const u32* __restrict__ dbase, u32* __restrict__ status, u32* __restrict__ ticket,
          u32* __restrict__ err)
{
    __shared__ u64 stage[RS_TILE];                 // keys, then values, in digit order
    __shared__ u32 wh[RS_WAVES][RS_BINS];
    __shared__ u32 bstart[RS_BINS];
    __shared__ u32 goff[RS_BINS];
    __shared__ u32 scr[RS_WAVES];
    __shared__ u32 s_tile;
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
    for (int d = threadIdx.x; d < RS_WAVES * RS_BINS; d += RS_BLOCK) (&wh[0][0])[d] = 0;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const i64 tile = s_tile;
    const i64 tile0 = tile * RS_TILE;
    const i64 base = tile0 + (i64)wid * RS_WTILE;
    u64 key[RS_ITEMS];
    u32 val[RS_ITEMS];
    u32 pos[RS_ITEMS];
    u32 dig[RS_ITEMS];
    // the array the digits come from is read first; the other one only after
    // the ranking (fewer live registers)
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const i64 i = base + (i64)it * WAVE + lane;
        const bool valid = i < n;
        if (MODE == 0) key[it] = valid ? kin[i] : 0;
        else val[it] = valid ? vin[i] : 0;
    }
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const i64 i = base + (i64)it * WAVE + lane;
        const bool valid = i < n;
        dig[it] = valid ? rs_digit<MODE>(MODE == 0 ? key[it] : 0ull, MODE == 0 ? 0u : val[it], shift,
                                         seg_off, nseg)
                        : 0;
        const u64 active = __ballot(valid);
        const u64 m = match_digit<RS_BITS>(dig[it], active);
        const int leader = __ffsll((unsigned long long)m) - 1;
        const u32 prev = wh[wid][dig[it]];
        pos[it] = prev + (u32)__popcll(m & lanemask_lt());
        if (valid && lane == leader) wh[wid][dig[it]] = prev + (u32)__popcll(m);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const i64 i = base + (i64)it * WAVE + lane;
        const bool valid = i < n;
        if (MODE == 0) val[it] = valid ? vin[i] : 0;
        else key[it] = valid ? kin[i] : 0;
    }
    // digit totals over the waves -> per-wave prefix, tile digit start, and
    // the tile's place among all tiles (look-back)
    {
        const int d = threadIdx.x;          // RS_BLOCK == RS_BINS
        u32 run = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) { u32 c = wh[w][d]; wh[w][d] = run; run += c; }
        u32 tot;
        bstart[d] = block_excl_scan<RS_BLOCK>(run, scr, tot);
        u32* mine = status + tile * RS_BINS + d;
        u32 excl = 0;
        if (tile == 0) {
            __hip_atomic_store(mine, ST_PREFIX | run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(mine, ST_AGG | run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            i64 t2 = tile - 1;
            u32 spins = 0;
            for (;;) {
                const u32 s = __hip_atomic_load(status + t2 * RS_BINS + d, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
                if ((s & ~ST_VAL) == 0u) {
                    if (++spins > ST_SPIN_LIMIT) { atomicOr(err, 1u); break; }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += s & ST_VAL;
                if ((s & ~ST_VAL) == ST_PREFIX || t2 == 0) break;
                --t2;
            }
            __hip_atomic_store(mine, ST_PREFIX | ((excl + run) & ST_VAL), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        goff[d] = dbase[d] + excl;
    }
    __syncthreads();
    // stable scatter through LDS: digit runs leave the tile contiguously.
    // The first array written out supplies each staged slot's digit (the
    // key for key digits, the value for instance-id digits); the second
    // reuses it.
    const i64 cnt = (n - tile0) < RS_TILE ? (n - tile0) : RS_TILE;
    u32 slot[RS_ITEMS], dj[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) slot[it] = bstart[dig[it]] + wh[wid][dig[it]] + pos[it];
    // (pos and dig are dead from here on)
    u32* sv = (u32*)stage;
    if (MODE == 0) {
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it)
            if (base + (i64)it * WAVE + lane < n) stage[slot[it]] = key[it];
    } else {
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it)
            if (base + (i64)it * WAVE + lane < n) sv[slot[it]] = val[it];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RS_ITEMS; ++q) {
        const int j = threadIdx.x + q * RS_BLOCK;
        if (j < cnt) {
            if (MODE == 0) {
                const u64 k = stage[j];
                dj[q] = (u32)(k >> shift) & (RS_BINS - 1);
                kout[(i64)goff[dj[q]] + (j - (i64)bstart[dj[q]])] = k;
            } else {
                const u32 v = sv[j];
                dj[q] = rs_digit<1>(0ull, v, shift, seg_off, nseg);
                vout[(i64)goff[dj[q]] + (j - (i64)bstart[dj[q]])] = v;
            }
        }
    }
    __syncthreads();
    if (MODE == 0) {
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it)
            if (base + (i64)it * WAVE + lane < n) sv[slot[it]] = val[it];
    } else {
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it)
            if (base + (i64)it * WAVE + lane < n) stage[slot[it]] = key[it];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RS_ITEMS; ++q) {
        const int j = threadIdx.x + q * RS_BLOCK;
        if (j < cnt) {
            const i64 o = (i64)goff[dj[q]] + (j - (i64)bstart[dj[q]]);
            if (MODE == 0) vout[o] = sv[j];
            else kout[o] = stage[j];
        }
    }
}

size_t radix_state_words(i64 n, int nseg)
{
    (void)nseg;
    const i64 ntiles = std::max<i64>(1, (n + RS_TILE - 1) / RS_TILE);
    return (size_t)(2 * RS_MAXP * RS_BINS + RS_MAXP + (i64)RS_MAXP * ntiles * RS_BINS);
}

// Sorts (keys, vals) over key bits [0, key_bits) and then, when nseg > 1,
// stably by the instance id of the original index.  Buffers ping-pong between
// (k0,v0) and (k1,v1); the return value says which pair holds the result
// (0 -> k0/v0, 1 -> k1/v1), or -1 for n >= 2^30 (not supported).  `state`
// holds radix_state_words(n) words; `err` (device) gets bit 0 set if a
// look-back wait ran past its bound.
int radix_sort_pairs(u64* k0, u32* v0, u64* k1, u32* v1, i64 n, int key_bits,
                     const i64* seg_off, int nseg, u32* state, u32* err, hipStream_t st)
{
    if (n <= 1) return 0;
    if (n >= (i64)ST_VAL) return -1;
    const i64 ntiles = (n + RS_TILE - 1) / RS_TILE;
    const int pk = (key_bits + RS_BITS - 1) / RS_BITS;
    int ps = 0;
    if (nseg > 1)
        for (int b = 0; (1ll << b) < nseg; b += RS_BITS) ++ps;
    const int np = pk + ps;
    if (np > RS_MAXP) return -1;
    u32* dbase = state;                                   // [np][256] digit starts
    u32* hist = dbase + RS_MAXP * RS_BINS;                // [np][256] digit counts
    u32* ticket = hist + RS_MAXP * RS_BINS;               // [np]
    u32* status = ticket + RS_MAXP;                       // [np][ntiles][256]
    // hist, tickets and look-back words start at zero (one contiguous range)
    launch_fill_u32(hist, RS_MAXP * RS_BINS + RS_MAXP + (i64)np * ntiles * RS_BINS, 0u, st);
    const int hb = (int)std::min<i64>(RS_HBLOCKS, ntiles);
    hipLaunchKernelGGL(k_rs_hist, dim3(hb), dim3(RS_BLOCK), 0, st, k0, v0, n, pk, ps, seg_off,
                       nseg, hist);
    hipLaunchKernelGGL(k_rs_scan, dim3(np), dim3(RS_BLOCK), 0, st, hist, dbase);
    int cur = 0;
    u64* kb[2] = { k0, k1 };
    u32* vb[2] = { v0, v1 };
    for (int p = 0; p < np; ++p) {
        u32* stp = status + (i64)p * ntiles * RS_BINS;
        if (p < pk)
            hipLaunchKernelGGL((k_rs_pass<0>), dim3((unsigned)ntiles), dim3(RS_BLOCK), 0, st,
                               kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, RS_BITS * p, seg_off,
                               nseg, dbase + p * RS_BINS, stp, ticket + p, err);
        else
            hipLaunchKernelGGL((k_rs_pass<1>), dim3((unsigned)ntiles), dim3(RS_BLOCK), 0, st,
                               kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, RS_BITS * (p - pk),
                               seg_off, nseg, dbase + p * RS_BINS, stp, ticket + p, err);
        cur ^= 1;
    }
    return cur;
}

}  // namespace shsph
