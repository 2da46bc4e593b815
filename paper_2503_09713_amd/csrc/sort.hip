// Stable LSD radix sort of (64-bit Morton key, 32-bit index) pairs.
//
// The paper sorts with a bitonic network (App. D.1) and names onesweep-style
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

// ---------------------------------------------------------------------------
// Nearly sorted input.  Between steps the particles keep their previous key
// order and few of them change place.  An isolated spike (a key out of order
// with its neighbours while the neighbours are in order with each other: one
// particle that jumped) is set aside first; of the other elements, one is
// "in place" when no earlier non-spike key is larger and no later one
// smaller.  The in-place elements (R) form a sorted sequence in index order,
// and a single far jump costs one out-of-place element, not the run it
// jumped over.  The others (O) are sorted by the
// radix passes and merged into R, both by (key, value).  With values that
// increase with the index (the iota of the key kernel) ties keep the index
// order on both sides, so the result is the stable sort.  Used when O holds
// at most n/8 elements; otherwise the full radix sort runs.
// ---------------------------------------------------------------------------
constexpr int AD_TILE = RS_TILE;                  // 4096 keys, RS_BLOCK threads x RS_ITEMS
constexpr int AD_SCAN = 1024;                     // threads of the one-block scans

__device__ inline u64 shfl_up_u64(u64 x, int d)
{
    const u32 lo = __shfl_up((u32)x, d, WAVE), hi = __shfl_up((u32)(x >> 32), d, WAVE);
    return ((u64)hi << 32) | lo;
}
__device__ inline u64 shfl_down_u64(u64 x, int d)
{
    const u32 lo = __shfl_down((u32)x, d, WAVE), hi = __shfl_down((u32)(x >> 32), d, WAVE);
    return ((u64)hi << 32) | lo;
}

// Exclusive prefix max and exclusive suffix min over the block's threads.
template <int BLOCK>
__device__ inline void block_pmax_smin(u64 vmax, u64 vmin, u64* lmax, u64* lmin, u64& pm, u64& sm)
{
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
    u64 a = vmax, b = vmin;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {          // inclusive scans within the wave
        const u64 ua = shfl_up_u64(a, d), db = shfl_down_u64(b, d);
        if (lane >= d) a = ua > a ? ua : a;
        if (lane + d < WAVE) b = db < b ? db : b;
    }
    if (lane == WAVE - 1) lmax[wid] = a;
    if (lane == 0) lmin[wid] = b;
    __syncthreads();
    u64 pw = 0, sw = ~0ull;
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        if (w < wid) pw = lmax[w] > pw ? lmax[w] : pw;
        if (w > wid) sw = lmin[w] < sw ? lmin[w] : sw;
    }
    __syncthreads();
    const u64 ea = shfl_up_u64(a, 1), eb = shfl_down_u64(b, 1);
    pm = lane > 0 ? (ea > pw ? ea : pw) : pw;
    sm = lane < WAVE - 1 ? (eb < sw ? eb : sw) : sw;
}

__device__ inline int ad_sw(int j) { return j + (j >> 4); }

// Isolated spike: key k between neighbours a <= b but out of order with them.
__device__ inline bool ad_spike(u64 a, u64 k, u64 b) { return a <= b && (k < a || k > b); }

// Per tile: the smallest and the largest key among the non-spikes.
__global__ void __launch_bounds__(RS_BLOCK)
k_ad_minmax(const u64* __restrict__ keys, i64 n, u64* __restrict__ tmin, u64* __restrict__ tmax)
{
    __shared__ u64 lmax[RS_WAVES], lmin[RS_WAVES];
    __shared__ u64 s_k[AD_TILE + 2];              // the tile and a key on each side
    constexpr int R = AD_TILE / RS_BLOCK;
    const i64 t0 = (i64)blockIdx.x * AD_TILE;
    {
        // every load of the thread in flight at once, then to LDS
        u64 ld[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const i64 i = t0 + r * RS_BLOCK + threadIdx.x;
            ld[r] = i < n ? keys[i] : 0ull;
        }
        u64 side = 0;
        if (threadIdx.x == 0) side = t0 > 0 ? keys[t0 - 1] : 0ull;
        if (threadIdx.x == 1) side = t0 + AD_TILE < n ? keys[t0 + AD_TILE] : ~0ull;
#pragma unroll
        for (int r = 0; r < R; ++r) s_k[1 + r * RS_BLOCK + threadIdx.x] = ld[r];
        if (threadIdx.x == 0) s_k[0] = side;
        if (threadIdx.x == 1) s_k[AD_TILE + 1] = side;
    }
    __syncthreads();
    u64 mx = 0, mn = ~0ull;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = r * RS_BLOCK + threadIdx.x;
        const i64 i = t0 + j;
        if (i < n) {
            const u64 k = s_k[j + 1];
            const u64 a = s_k[j], b = i + 1 < n ? s_k[j + 2] : ~0ull;
            if (!ad_spike(a, k, b)) {
                mx = k > mx ? k : mx;
                mn = k < mn ? k : mn;
            }
        }
    }
    u64 pm, sm;
    block_pmax_smin<RS_BLOCK>(mx, mn, lmax, lmin, pm, sm);
    // the last thread's exclusive prefix max plus its own is the tile max
    if (threadIdx.x == RS_BLOCK - 1) tmax[blockIdx.x] = mx > pm ? mx : pm;
    if (threadIdx.x == 0) tmin[blockIdx.x] = mn < sm ? mn : sm;
}

// One block: pmax[t] = max of the tile maxima before t (0 for t = 0),
// smin[t] = min of the tile minima after t (all ones for the last tile).
__global__ void __launch_bounds__(AD_SCAN)
k_ad_tilescan(const u64* __restrict__ tmin, const u64* __restrict__ tmax, i64 ntiles,
              u64* __restrict__ pmax, u64* __restrict__ smin)
{
    __shared__ u64 lmax[AD_SCAN / WAVE], lmin[AD_SCAN / WAVE];
    const i64 per = (ntiles + AD_SCAN - 1) / AD_SCAN;
    const i64 a0 = (i64)threadIdx.x * per, a1 = (a0 + per) < ntiles ? (a0 + per) : ntiles;
    u64 mx = 0, mn = ~0ull;
    for (i64 t = a0; t < a1; ++t) {
        mx = tmax[t] > mx ? tmax[t] : mx;
        mn = tmin[t] < mn ? tmin[t] : mn;
    }
    u64 pm, sm;
    block_pmax_smin<AD_SCAN>(mx, mn, lmax, lmin, pm, sm);
    for (i64 t = a0; t < a1; ++t) {
        pmax[t] = pm;
        pm = tmax[t] > pm ? tmax[t] : pm;
    }
    for (i64 t = a1 - 1; t >= a0; --t) {
        smin[t] = sm;
        sm = tmin[t] < sm ? tmin[t] : sm;
    }
}

// Classifies a tile's elements (out of place: a larger key before or a
// smaller one after).  COMPACT = false: writes the tile's count of out-of-
// place elements.  COMPACT = true: writes the in-place ones to R (at their
// index minus the out-of-place ones before them) and the others to O (at the
// tile's offset toff plus their rank), both in index order.
template <bool COMPACT>
__global__ void __launch_bounds__(RS_BLOCK)
k_ad_classify(const u64* __restrict__ keys, const u32* __restrict__ vals, i64 n,
              const u64* __restrict__ pmax, const u64* __restrict__ smin, u32* __restrict__ tcnt,
              const u32* __restrict__ toff, u64* __restrict__ rk, u32* __restrict__ rv,
              u64* __restrict__ ok, u32* __restrict__ ov)
{
    // element j at j + j/16: the blocked reads (16 consecutive elements per
    // thread) then fall on different banks
    __shared__ u64 s_k[AD_TILE + AD_TILE / 16];
    __shared__ u16 s_rank[AD_TILE + AD_TILE / 16];  // out-of-place elements before j; bit 15: j is one
    __shared__ u64 lmax[RS_WAVES], lmin[RS_WAVES];
    __shared__ u32 s_cnt[RS_WAVES];
    const i64 tile = blockIdx.x, t0 = tile * AD_TILE;
    const i64 cnt = (n - t0) < AD_TILE ? (n - t0) : AD_TILE;
    constexpr int R = AD_TILE / RS_BLOCK;
    u32 vl[R];                                    // values of the copy (COMPACT), loaded early
    {
        u64 ld[R];                                // all loads in flight, then to LDS
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = r * RS_BLOCK + threadIdx.x;
            ld[r] = j < cnt ? keys[t0 + j] : ~0ull;
            vl[r] = COMPACT && j < cnt ? vals[t0 + j] : 0u;
        }
#pragma unroll
        for (int r = 0; r < AD_TILE / RS_BLOCK; ++r) s_k[ad_sw(r * RS_BLOCK + threadIdx.x)] = ld[r];
    }
    const u64 kprev = t0 > 0 ? keys[t0 - 1] : 0ull;            // neighbours across the tile
    const u64 knext = t0 + cnt < n ? keys[t0 + cnt] : ~0ull;
    __syncthreads();
    // blocked: thread t holds elements RS_ITEMS t .. RS_ITEMS t + RS_ITEMS - 1
    const int b0 = threadIdx.x * RS_ITEMS;
    u32 spikes = 0;
#pragma unroll
    for (int q = 0; q < RS_ITEMS; ++q) {
        const int j = b0 + q;
        const u64 a = j > 0 ? s_k[ad_sw(j - 1)] : kprev;
        const u64 b = j + 1 < AD_TILE ? (j + 1 < cnt ? s_k[ad_sw(j + 1)] : knext) : knext;
        spikes |= (j < cnt && ad_spike(a, s_k[ad_sw(j)], b) ? 1u : 0u) << q;
    }
    u64 mx = 0, mn = ~0ull;
#pragma unroll
    for (int q = 0; q < RS_ITEMS; ++q) {
        if ((spikes >> q) & 1u) continue;
        const u64 k = s_k[ad_sw(b0 + q)];
        mx = k > mx ? k : mx;
        mn = k < mn ? k : mn;
    }
    u64 pm, sm;
    block_pmax_smin<RS_BLOCK>(mx, mn, lmax, lmin, pm, sm);
    const u64 tp = pmax[tile], ts = smin[tile];
    pm = tp > pm ? tp : pm;
    sm = ts < sm ? ts : sm;
    // suffix minima of the thread's own items, then a forward pass
    u64 suf[RS_ITEMS];
    {
        u64 r = sm;
#pragma unroll
        for (int q = RS_ITEMS - 1; q >= 0; --q) {
            suf[q] = r;
            const u64 k = s_k[ad_sw(b0 + q)];
            if (!((spikes >> q) & 1u)) r = k < r ? k : r;
        }
    }
    u32 flags = 0, nown = 0;
    {
        u64 r = pm;
#pragma unroll
        for (int q = 0; q < RS_ITEMS; ++q) {
            const u64 k = s_k[ad_sw(b0 + q)];
            const bool sp = (spikes >> q) & 1u;
            const bool out = (b0 + q < cnt) && (sp || k < r || k > suf[q]);
            flags |= (out ? 1u : 0u) << q;
            if (!sp) r = k > r ? k : r;
        }
        nown = (u32)__popc(flags);
    }
    // rank of each out-of-place element within the tile
    u32 total;
    {
        const int lane = __lane_id(), wid = threadIdx.x / WAVE;
        const u32 incl = wave_incl_scan(nown);
        if (lane == WAVE - 1) s_cnt[wid] = incl;
        __syncthreads();
        u32 before = 0;
        total = 0;
        for (int w = 0; w < RS_WAVES; ++w) {
            before += w < wid ? s_cnt[w] : 0u;
            total += s_cnt[w];
        }
        u32 r = before + incl - nown;
#pragma unroll
        for (int q = 0; q < RS_ITEMS; ++q) {
            const bool out = (flags >> q) & 1u;
            s_rank[ad_sw(b0 + q)] = (u16)(r | (out ? 0x8000u : 0u));
            r += out ? 1u : 0u;
        }
    }
    if (!COMPACT) {
        if (threadIdx.x == 0) tcnt[tile] = total;
        return;
    }
    __syncthreads();
    const u32 base = toff[tile];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int j = q * RS_BLOCK + threadIdx.x;
        if (j >= cnt) continue;
        const u32 r = s_rank[ad_sw(j)];
        const i64 i = t0 + j;
        const u64 k = s_k[ad_sw(j)];
        const u32 v = vl[q];
        if (r & 0x8000u) {
            const u32 o = base + (r & 0x7fffu);
            ok[o] = k;
            ov[o] = v;
        } else {
            const i64 ri = i - (i64)(base + r);
            rk[ri] = k;
            rv[ri] = v;
        }
    }
}

// One block: exclusive scan of the tile counts, total in toff[ntiles].
__global__ void __launch_bounds__(AD_SCAN)
k_ad_cntscan(const u32* __restrict__ tcnt, i64 ntiles, u32* __restrict__ toff)
{
    __shared__ u32 scr[AD_SCAN / WAVE];
    const i64 per = (ntiles + AD_SCAN - 1) / AD_SCAN;
    const i64 a0 = (i64)threadIdx.x * per, a1 = (a0 + per) < ntiles ? (a0 + per) : ntiles;
    u32 s = 0;
    for (i64 t = a0; t < a1; ++t) s += tcnt[t];
    u32 tot;
    u32 r = block_excl_scan<AD_SCAN>(s, scr, tot);
    for (i64 t = a0; t < a1; ++t) {
        toff[t] = r;
        r += tcnt[t];
    }
    if (threadIdx.x == 0) toff[ntiles] = tot;
}

// Number of O elements ordered before (key, val) (lower bound by (key, val)).
__device__ inline i64 o_before(const u64* ok, const u32* ov, i64 no, u64 k, u32 v)
{
    i64 lo = 0, hi = no;
    while (lo < hi) {
        const i64 mid = (lo + hi) >> 1;
        const u64 km = ok[mid];
        if (km < k || (km == k && ov[mid] < v)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merge, R side, one tile of R per workgroup: R element j goes to j + c_j,
// c_j = the O elements before it.  c is monotone, so the tile's first and
// last elements bound the O range its elements search (usually empty).
// Per R tile: c of its first and of its last element (one thread each).
__global__ void k_ad_bounds(const u64* __restrict__ rk, const u32* __restrict__ rv, i64 nr,
                            const u64* __restrict__ ok, const u32* __restrict__ ov, i64 no,
                            u32* __restrict__ cfirst, u32* __restrict__ clast)
{
    const i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 t = u >> 1;
    const i64 j0 = t * AD_TILE;
    if (j0 >= nr) return;
    const i64 j = (u & 1) ? ((j0 + AD_TILE) < nr ? (j0 + AD_TILE) : nr) - 1 : j0;
    const u32 c = (u32)o_before(ok, ov, no, rk[j], rv[j]);
    if (u & 1) clast[t] = c;
    else cfirst[t] = c;
}

__global__ void __launch_bounds__(RS_BLOCK)
k_ad_merge(const u64* __restrict__ rk, const u32* __restrict__ rv, i64 nr,
           const u64* __restrict__ ok, const u32* __restrict__ ov, i64 no,
           const u32* __restrict__ cfirst, const u32* __restrict__ clast, u64* __restrict__ outk,
           u32* __restrict__ outv)
{
    constexpr int OL = 1024;                     // O range staged in LDS up to this size
    __shared__ u64 s_ok[OL];
    __shared__ u32 s_ov[OL];
    const i64 j0 = (i64)blockIdx.x * AD_TILE;
    const i64 cnt = (nr - j0) < AD_TILE ? (nr - j0) : AD_TILE;
    const i64 lo = cfirst[blockIdx.x], hi = clast[blockIdx.x];
    // the tile's R elements, all loads issued first
    u64 kk[RS_ITEMS];
    u32 vv[RS_ITEMS];
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int j = threadIdx.x + it * RS_BLOCK;
        kk[it] = j < cnt ? rk[j0 + j] : 0ull;
        vv[it] = j < cnt ? rv[j0 + j] : 0u;
    }
    u32 cc[RS_ITEMS];
    if (lo == hi) {                              // no O element falls inside this tile
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it) cc[it] = (u32)lo;
    } else {
        const bool staged = hi - lo <= OL;
        if (staged) {
            for (i64 q = threadIdx.x; q < hi - lo; q += RS_BLOCK) {
                s_ok[q] = ok[lo + q];
                s_ov[q] = ov[lo + q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < RS_ITEMS; ++it)
            cc[it] = (u32)(lo + (staged ? o_before(s_ok, s_ov, hi - lo, kk[it], vv[it])
                                        : o_before(ok + lo, ov + lo, hi - lo, kk[it], vv[it])));
    }
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int j = threadIdx.x + it * RS_BLOCK;
        if (j < cnt) {
            outk[j0 + j + cc[it]] = kk[it];
            outv[j0 + j + cc[it]] = vv[it];
        }
    }
}

// O element q goes to q + (R elements before it): a binary search over R by
// (key, value), one thread per O element.
__global__ void k_ad_place_o(const u64* __restrict__ rk, const u32* __restrict__ rv, i64 nr,
                             const u64* __restrict__ ok, const u32* __restrict__ ov, i64 no,
                             u64* __restrict__ outk, u32* __restrict__ outv)
{
    const i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= no) return;
    const u64 k = ok[q];
    const u32 v = ov[q];
    i64 lo = 0, hi = nr;
    while (lo < hi) {
        const i64 mid = (lo + hi) >> 1;
        const u64 km = rk[mid];
        if (km < k || (km == k && rv[mid] < v)) lo = mid + 1;
        else hi = mid;
    }
    outk[q + lo] = k;
    outv[q + lo] = v;
}

__global__ void k_ad_copy(const u64* __restrict__ ok, const u32* __restrict__ ov, i64 no,
                          u64* __restrict__ outk, u32* __restrict__ outv)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < no) {
        outk[i] = ok[i];
        outv[i] = ov[i];
    }
}

static i64 radix_base_words(i64 n)
{
    const i64 ntiles = std::max<i64>(1, (n + RS_TILE - 1) / RS_TILE);
    return 2 * RS_MAXP * RS_BINS + RS_MAXP + (i64)RS_MAXP * ntiles * RS_BINS;
}

// Adaptive part of the state (single-instance sorts): tile min/max and their
// scans (4 x ntiles u64), tile counts and offsets, O keys and values twice
// (ping-pong of the radix passes), n/8 each.
static i64 adaptive_words(i64 n)
{
    const i64 ntiles = std::max<i64>(1, (n + AD_TILE - 1) / AD_TILE);
    const i64 omax = n / 8 + 1;
    return 8 * ntiles + 2 * ntiles + 2 + 4 * omax + 2 * omax + 8;
}

size_t radix_state_words(i64 n, int nseg)
{
    i64 w = radix_base_words(n);
    if (nseg <= 1) w += (w & 1) + adaptive_words(n);
    return (size_t)w;
}

// The radix passes (full sort) into the ping-pong pair; returns the side.
static int radix_passes(u64* k0, u32* v0, u64* k1, u32* v1, i64 n, int key_bits,
                        const i64* seg_off, int nseg, u32* state, u32* err, hipStream_t st)
{
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

// Sorts (keys, vals) over key bits [0, key_bits) and then, when nseg > 1,
// stably by the instance id of the original index.  Buffers ping-pong between
// (k0,v0) and (k1,v1); the return value says which pair holds the result
// (0 -> k0/v0, 1 -> k1/v1), or -1 for n >= 2^30 (not supported).  `state`
// holds radix_state_words(n, nseg) words; `err` (device) gets bit 0 set if a
// look-back wait ran past its bound.  With nseg <= 1 and `host_word`
// (pinned host memory) given, nearly sorted input takes the adaptive path
// (one host synchronisation to read the out-of-place count); it needs the
// values to increase with the index (the key kernel's iota).
int radix_sort_pairs(u64* k0, u32* v0, u64* k1, u32* v1, i64 n, int key_bits,
                     const i64* seg_off, int nseg, u32* state, u32* err, u32* host_word,
                     hipStream_t st)
{
    if (n <= 1) return 0;
    if (n >= (i64)ST_VAL) return -1;
    if (nseg <= 1 && host_word && n >= 2 * AD_TILE) {
        const i64 ntiles = (n + AD_TILE - 1) / AD_TILE;
        const i64 omax = n / 8;
        i64 off = radix_base_words(n);
        off += off & 1;                                   // u64 alignment
        u64* tmin = (u64*)(state + off);
        u64* tmax = tmin + ntiles;
        u64* pmax = tmax + ntiles;
        u64* smin = pmax + ntiles;
        u32* tcnt = (u32*)(smin + ntiles);
        u32* toff = tcnt + ntiles;                        // ntiles + 1
        u64* oka = (u64*)(toff + ntiles + 2);            // 2 ntiles + 2 words past tcnt: aligned
        u64* okb = oka + omax + 1;
        u32* ova = (u32*)(okb + omax + 1);
        u32* ovb = ova + omax + 1;
        hipLaunchKernelGGL(k_ad_minmax, dim3((unsigned)ntiles), dim3(RS_BLOCK), 0, st, k0, n, tmin,
                           tmax);
        hipLaunchKernelGGL(k_ad_tilescan, dim3(1), dim3(AD_SCAN), 0, st, tmin, tmax, ntiles, pmax,
                           smin);
        hipLaunchKernelGGL((k_ad_classify<false>), dim3((unsigned)ntiles), dim3(RS_BLOCK), 0, st,
                           k0, v0, n, pmax, smin, tcnt, nullptr, nullptr, nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(k_ad_cntscan, dim3(1), dim3(AD_SCAN), 0, st, tcnt, ntiles, toff);
        if (hipMemcpyAsync(host_word, toff + ntiles, sizeof(u32), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return -2;
        const i64 no = *host_word;
        if (no == 0) return 0;                            // already in order
        if (no <= omax) {
            const i64 nr = n - no;
            hipLaunchKernelGGL((k_ad_classify<true>), dim3((unsigned)ntiles), dim3(RS_BLOCK), 0,
                               st, k0, v0, n, pmax, smin, nullptr, toff, k1, v1, oka, ova);
            int so = 0;
            if (no > 1) so = radix_passes(oka, ova, okb, ovb, no, key_bits, nullptr, 1, state, err, st);
            if (so < 0) return so;
            const u64* osk = so ? okb : oka;
            const u32* osv = so ? ovb : ova;
            if (nr > 0) {
                const i64 rt = (nr + AD_TILE - 1) / AD_TILE;
                u32* cfirst = tcnt;                       // the tile counts are no longer needed
                u32* clast = (u32*)pmax;                  // nor the prefix maxima
                hipLaunchKernelGGL(k_ad_bounds, dim3((unsigned)((2 * rt + 255) / 256)), dim3(256), 0,
                                   st, k1, v1, nr, osk, osv, no, cfirst, clast);
                hipLaunchKernelGGL(k_ad_merge, dim3((unsigned)rt), dim3(RS_BLOCK), 0, st, k1, v1,
                                   nr, osk, osv, no, cfirst, clast, k0, v0);
                hipLaunchKernelGGL(k_ad_place_o, dim3((unsigned)((no + 255) / 256)), dim3(256), 0,
                                   st, k1, v1, nr, osk, osv, no, k0, v0);
            }
            else
                hipLaunchKernelGGL(k_ad_copy, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, st,
                                   osk, osv, no, k0, v0);
            return 0;
        }
    }
    return radix_passes(k0, v0, k1, v1, n, key_bits, seg_off, nseg, state, err, st);
}

}  // namespace shsph
