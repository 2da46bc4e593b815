// Tree build kernels: leapfrog predict + Morton keys, gather into key order,
// keep mask and leaf reduction, compaction, Karras radix tree and the
// bottom-up cell boxes.  All kernels work on a table of independent
// instances (segments of the particle arrays); a plain run is one instance.
#include "common.hpp"
#include "kernels.hpp"

namespace shsph {

static inline dim3 grid_for(i64 n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

// ---------------------------------------------------------------------------
// Leapfrog predictor (App. G.1): v^{n+1/2} = v + dt/2 a, r^{n+1} = r + dt v^{n+1/2},
// v* = v^{n+1/2} + dt/2 a, and the same for u; periodic positions are wrapped
// into [lo, hi).  Written with explicit roundings so that every kernel that
// evaluates it obtains bit-identical positions.
// ---------------------------------------------------------------------------
template <class T> struct Pred {
    T x[3], vh[3], vs[3], uh, us;
};

template <class T>
__device__ inline void predict(const T* const* xp, const T* const* vp, const T* const* ap,
                               const T* u, const T* du, i64 j, T dt, const Box<T>& bx,
                               Pred<T>& o)
{
#pragma clang fp contract(off)
    const T hdt = T(0.5) * dt;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T a = ap ? ap[d][j] : T(0);
        const T v = vp ? vp[d][j] : T(0);
        const T ka = hdt * a;
        const T vh = v + ka;
        const T dx = dt * vh;
        T x = xp[d][j] + dx;
        if (bx.periodic) {
            if (x >= bx.hi[d]) x = x - bx.L[d];
            if (x < bx.lo[d]) x = x + bx.L[d];
            if (x >= bx.hi[d]) x = bx.lo[d];
        }
        o.x[d] = x;
        o.vh[d] = vh;
        o.vs[d] = vh + ka;
    }
    const T uu = u ? u[j] : T(0);
    const T dd = du ? du[j] : T(0);
    const T kd = hdt * dd;
    o.uh = uu + kd;
    o.us = o.uh + kd;
}

// Morton key (App. B.1): X = min(2^21-1, max(0, floor((x - lo) * 2^21/(hi - lo))))
// in FP64, interleaved X0 Y0 Z0 X1 Y1 Z1 ... (bit 63 unused).
__device__ inline u64 spread3(u32 v)
{
    u64 x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline u32 quantize(double v, double lo, double scale, u32 qmax)
{
#pragma clang fp contract(off)
    const double d = v - lo;
    const double t = d * scale;
    const double f = floor(t);
    if (!(f >= 0.0)) return 0u;
    if (f > (double)qmax) return qmax;
    return (u32)f;
}

// `bits` per axis: 21 (63-bit codes) or 10 (30-bit codes, Sect. 5.2.1); the
// code sits in the low 3 bits bits of the key.
__device__ inline u64 morton_key(double x, double y, double z, const InstDev& in, int bits)
{
    const double g = (double)(1u << bits);
    const u32 qmax = (1u << bits) - 1u;
    const u32 X = quantize(x, in.lo[0], g / (in.hi[0] - in.lo[0]), qmax);
    const u32 Y = quantize(y, in.lo[1], g / (in.hi[1] - in.lo[1]), qmax);
    const u32 Z = quantize(z, in.lo[2], g / (in.hi[2] - in.lo[2]), qmax);
    return (spread3(X) << 2) | (spread3(Y) << 1) | spread3(Z);
}

template <class T>
__global__ void k_predict_morton(FieldPtrs<T> f, i64 n, const InstDev* __restrict__ inst,
                                 const i64* __restrict__ p_off, int ninst,
                                 const double* __restrict__ dt_inst, u64* __restrict__ keys,
                                 u32* __restrict__ vals, int bits)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = find_seg(p_off, ninst, i);
    const InstDev in = inst[k];
    const i64 ic = i + in.shift;
    double x, y, z;
    if (dt_inst) {
        const Box<T> bx = make_box<T>(in);
        const T* xp[3] = { f.x, f.y, f.z };
        const T* vp[3] = { f.vx, f.vy, f.vz };
        const T* ap[3] = { f.ax, f.ay, f.az };
        Pred<T> o;
        predict<T>(xp, vp, f.ax ? ap : nullptr, f.u, f.du, ic, (T)dt_inst[k], bx, o);
        x = o.x[0]; y = o.x[1]; z = o.x[2];
    } else {
        x = f.x[ic]; y = f.y[ic]; z = f.z[ic];
    }
    keys[i] = morton_key(x, y, z, in, bits);
    vals[i] = (u32)i;
}

// Gather the fields into key order: sorted slot i takes original index eps[i].
template <class T>
__global__ void k_gather(FieldPtrs<T> f, i64 n, const InstDev* __restrict__ inst,
                         const i64* __restrict__ p_off, int ninst, const double* __restrict__ dt_inst,
                         const u32* __restrict__ eps, SortedPtrs<T> s)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const i64 j0 = eps[i];
    const int k = find_seg(p_off, ninst, i);     // the sort keeps instances apart
    const i64 j = j0 + inst[k].shift;
    const T h = f.h[j];
    if (dt_inst) {
        const Box<T> bx = make_box<T>(inst[k]);
        const T* xp[3] = { f.x, f.y, f.z };
        const T* vp[3] = { f.vx, f.vy, f.vz };
        const T* ap[3] = { f.ax, f.ay, f.az };
        Pred<T> o;
        predict<T>(xp, vp, f.ax ? ap : nullptr, f.u, f.du, j, (T)dt_inst[k], bx, o);
        s.posh[i] = mk4<T>(o.x[0], o.x[1], o.x[2], h);
        s.velu[i] = mk4<T>(o.vs[0], o.vs[1], o.vs[2], o.us);
        if (s.vhalf) s.vhalf[i] = mk4<T>(o.vh[0], o.vh[1], o.vh[2], o.uh);
    } else {
        s.posh[i] = mk4<T>(f.x[j], f.y[j], f.z[j], h);
        if (s.velu && f.vx)
            s.velu[i] = mk4<T>(f.vx[j], f.vy[j], f.vz[j], f.u ? f.u[j] : T(0));
    }
    s.hn[i] = h;
    s.hcache[i] = h;
    if (s.pid) s.pid[i] = f.pid ? f.pid[j] : (u32)j0;
}

// ---------------------------------------------------------------------------
// Keep mask and reduction (App. C, Alg. 1).  Duplicates are dropped, then
// each pass removes code i when delta(i-2,i-1) < delta(i-1,i) > delta(i,i+1)
// over the currently kept codes, i.e. when i is the second leaf of a pair of
// sibling leaves.  Passes read the old mask and write a new one; neighbours
// outside the instance count as prefix length -1.
// ---------------------------------------------------------------------------
__device__ inline int delta_k(u64 a, u64 b) { return __clzll(a ^ b); }

__global__ void k_mask_init(const u64* __restrict__ mu, i64 n, const i64* __restrict__ p_off,
                            int ninst, u8* __restrict__ xi)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = find_seg(p_off, ninst, i);
    xi[i] = (i == p_off[k]) ? 1 : (mu[i] != mu[i - 1]);
}

__global__ void k_reduce_pass(const u64* __restrict__ mu, i64 n, const i64* __restrict__ p_off,
                              int ninst, const u8* __restrict__ xold, u8* __restrict__ xnew)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!xold[i]) { xnew[i] = 0; return; }
    const int k = find_seg(p_off, ninst, i);
    const i64 f = p_off[k], l = p_off[k + 1];
    i64 im1 = i - 1;
    while (im1 >= f && !xold[im1]) --im1;
    i64 im2 = im1 - 1;
    while (im2 >= f && !xold[im2]) --im2;
    i64 ip1 = i + 1;
    while (ip1 < l && !xold[ip1]) ++ip1;
    const u64 m = mu[i];
    const int d0 = (ip1 < l) ? delta_k(m, mu[ip1]) : -1;
    const int dm1 = (im1 >= f) ? delta_k(mu[im1], m) : -1;
    const int dm2 = (im1 >= f && im2 >= f) ? delta_k(mu[im2], mu[im1]) : -1;
    xnew[i] = ((d0 < dm1) && (dm2 < dm1)) ? 0 : 1;
}

// Compaction: id[k] = index of the k-th kept code, mu_leaf[k] its code,
// id[n_leaf] = n (App. D.1, Fig. mortonlistbuild).
__global__ void k_compact(const u64* __restrict__ mu, const u8* __restrict__ xi,
                          const u32* __restrict__ xscan, i64 n, u32* __restrict__ id,
                          u64* __restrict__ mu_leaf)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (xi[i]) {
        const u32 k = xscan[i];
        id[k] = (u32)i;
        mu_leaf[k] = mu[i];
    }
    if (i == 0) id[xscan[n]] = (u32)n;
}

// The keep mask, the reduction passes, the scan and the compaction in one
// kernel, with the results of k_mask_init + n_red k_reduce_pass + scan +
// k_compact.  Each workgroup takes a tile of LV_TILE sorted codes (tiles
// numbered by an atomic ticket) and a window reaching LV_HALO codes beyond
// it on both sides, and runs the mask and the Jacobi passes on the window in
// LDS.  The window is held in rows of LV_BLOCK codes, code r * LV_BLOCK + t
// with thread t, so that a wave's LDS accesses and global stores touch
// consecutive codes.  In each pass the nearest kept code before and after
// every code come from the wave's ballot of its row and a table of the
// last / first nonzero code of every (row, wave) (the one before that from
// the first table's results, kept in LDS).  Codes outside the window are
// unknown (state 2): a nearest code that would lie outside the window while
// still inside the instance, or that is unknown itself, makes the result
// unknown, so every code whose state is 0 or 1 has exactly the value the
// global passes give it.  A tile with an unknown code of its own (a run of
// dropped codes longer than the halo, e.g. many coincident particles) sets
// flag[0], and the caller runs the separate passes instead; the others
// publish their kept count and find the exclusive prefix by decoupled
// look-back over the earlier tiles (bounded waits: flag[1] on overrun).
// Writes xi, xscan[0..n], id[0..n_leaf] and mu_leaf.
constexpr int LV_BLOCK = 256, LV_ITEMS = 16, LV_TILE = LV_BLOCK * LV_ITEMS, LV_HALO = LV_BLOCK;
constexpr int LV_WIN = LV_TILE + 2 * LV_HALO, LV_PER = LV_WIN / LV_BLOCK, LV_NW = LV_BLOCK / WAVE;
constexpr u32 LV_AGG = 1u << 30, LV_PREFIX = 2u << 30, LV_VAL = (1u << 30) - 1u;
constexpr u32 LV_SPIN_LIMIT = 1u << 22;
constexpr u16 LV_NONE = 0xffffu;
constexpr int LV_FAR = 1 << 30;          // "no nonzero code after" in the window
static_assert(LV_WIN % LV_BLOCK == 0 && LV_WIN < 0xffff, "window split into rows");
static_assert(LV_HALO % LV_BLOCK == 0, "the tile starts on a row");
static_assert(LV_ITEMS * LV_NW == WAVE, "one (row, wave) kept count per lane of a wave");

// Nearest kept code found by a scan (`a`: -1 / >= W when none in the window)
// for a code of the instance [f, l) (window coordinates): the slot, -1 for
// none inside the instance, -2 for unknown.  `m` holds the current mask in
// bits sh, sh + 1 of each byte.
__device__ inline int lv_resolve_prev(const u8* m, int sh, int a, int f)
{
    if (a >= 0 && a >= f) return ((m[a] >> sh) & 3) == 2 ? -2 : a;
    return f >= 0 ? -1 : -2;
}
__device__ inline int lv_resolve_next(const u8* m, int sh, int c, int l, int W)
{
    if (c < W && c < l) return ((m[c] >> sh) & 3) == 2 ? -2 : c;
    return l <= W ? -1 : -2;
}

template <bool MULTI>
__global__ void __launch_bounds__(LV_BLOCK)
k_leaves_fused(const u64* __restrict__ mu, i64 n, const i64* __restrict__ p_off, int ninst,
               int nred, u32* __restrict__ ticket, u32* __restrict__ status, u8* __restrict__ xi,
               u32* __restrict__ xscan, u32* __restrict__ id, u64* __restrict__ mu_leaf,
               u32* __restrict__ flag)
{
    __shared__ u64 s_mu[LV_WIN];
    // mask of the current pass in bits 2 cur .. 2 cur + 1, the next pass's
    // in the other two: a thread rewrites only its own codes' bytes and
    // leaves the current field as it was, so readers of that field race
    // with nothing
    __shared__ u8 s_m[LV_WIN];
    __shared__ u16 s_prev[LV_WIN];
    __shared__ int s_last[LV_PER][LV_NW], s_first[LV_PER][LV_NW];
    __shared__ u32 s_cnt[WAVE];
    __shared__ u32 s_tile, s_excl, s_tot;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
    const u64 below = (1ull << lane) - 1ull;                      // lanes before this one
    const u64 above = lane == WAVE - 1 ? 0ull : ~0ull << (lane + 1);
    const i64 tile = s_tile;
    const i64 ntiles = (n + LV_TILE - 1) / LV_TILE;
    const i64 t0 = tile * LV_TILE, t1 = (t0 + LV_TILE) < n ? (t0 + LV_TILE) : n;
    const i64 w0 = t0 > LV_HALO ? t0 - LV_HALO : 0;
    const i64 w1 = (t1 + LV_HALO) < n ? (t1 + LV_HALO) : n;
    const int W = (int)(w1 - w0);
    {
        // all the window's loads in flight at once, then to LDS
        u64 ld[LV_PER];
#pragma unroll
        for (int r = 0; r < LV_PER; ++r) {
            const int j = r * LV_BLOCK + threadIdx.x;
            ld[r] = j < W ? mu[w0 + j] : 0ull;
        }
#pragma unroll
        for (int r = 0; r < LV_PER; ++r) {
            const int j = r * LV_BLOCK + threadIdx.x;
            if (j < W) s_mu[j] = ld[r];
        }
    }
    // the instance range [f, l) of this thread's code in every row (window
    // coordinates, clamped into int range)
    int fr[LV_PER], lr[LV_PER];
    {
        i64 f = 0, l = n;
        int k = 0;
        if (MULTI) {
            k = find_seg(p_off, ninst, w0 + ((int)threadIdx.x < W ? (int)threadIdx.x : 0));
            f = p_off[k];
            l = p_off[k + 1];
        }
#pragma unroll
        for (int r = 0; r < LV_PER; ++r) {
            if (MULTI) {
                const i64 i = w0 + r * LV_BLOCK + threadIdx.x;
                while (k + 1 < ninst && i >= l) { ++k; f = l; l = p_off[k + 1]; }
            }
            fr[r] = (int)((f - w0) > -(1 << 30) ? (f - w0) : -(1 << 30));
            lr[r] = (int)((l - w0) < (1 << 30) ? (l - w0) : (1 << 30));
        }
    }
    __syncthreads();
    // keep mask: the first code of an instance, else a code unlike the one before
#pragma unroll
    for (int r = 0; r < LV_PER; ++r) {
        const int j = r * LV_BLOCK + threadIdx.x;
        if (j >= W) continue;
        u8 v;
        if (j == fr[r]) v = 1;
        else if (j == 0) v = 2;
        else v = s_mu[j] != s_mu[j - 1] ? 1 : 0;
        s_m[j] = v;
    }
    __syncthreads();
    int cur = 0;
    for (int p = 0; p < nred; ++p) {
        const int sh = 2 * cur, nsh = 2 - sh;
        // last and first nonzero (kept or unknown) code of every (row, wave)
#pragma unroll
        for (int r = 0; r < LV_PER; ++r) {
            const int j = r * LV_BLOCK + threadIdx.x;
            const u64 nz = __ballot(j < W && ((s_m[j] >> sh) & 3) != 0);
            if (lane == 0) {
                const int base = r * LV_BLOCK + wid * WAVE;
                s_last[r][wid] = nz ? base + 63 - __clzll(nz) : -1;
                s_first[r][wid] = nz ? base + __ffsll((unsigned long long)nz) - 1 : LV_FAR;
            }
        }
        __syncthreads();
        // nearest nonzero code before each code, to LDS (the resolution also
        // needs it at the code found)
        int run = -1;                         // last nonzero code of the rows before r
#pragma unroll
        for (int r = 0; r < LV_PER; ++r) {
            const int j = r * LV_BLOCK + threadIdx.x;
            const u64 nz = __ballot(j < W && ((s_m[j] >> sh) & 3) != 0);
            int bw = run, rowmax = run;
#pragma unroll
            for (int w = 0; w < LV_NW; ++w) {
                const int x = s_last[r][w];
                if (w < wid) bw = bw > x ? bw : x;
                rowmax = rowmax > x ? rowmax : x;
            }
            const u64 lo = nz & below;
            const int pv = lo ? r * LV_BLOCK + wid * WAVE + 63 - __clzll(lo) : bw;
            if (j < W) s_prev[j] = pv < 0 ? LV_NONE : (u16)pv;
            run = rowmax;
        }
        __syncthreads();                      // s_prev complete
        // resolve the kept codes, last row first; the nearest nonzero code
        // after each comes from the same ballot and the rows already passed
        run = LV_FAR;                         // first nonzero code of the rows after r
#pragma unroll
        for (int r = LV_PER - 1; r >= 0; --r) {
            const int j = r * LV_BLOCK + threadIdx.x;
            const u8 byte = j < W ? s_m[j] : (u8)0;
            const u8 v = (byte >> sh) & 3;
            const u64 nz = __ballot(v != 0);
            int aw = run, rowmin = run;
#pragma unroll
            for (int w = 0; w < LV_NW; ++w) {
                const int x = s_first[r][w];
                if (w > wid) aw = aw < x ? aw : x;
                rowmin = rowmin < x ? rowmin : x;
            }
            run = rowmin;
            if (j >= W) continue;
            const u64 hi = nz & above;
            const int nx = hi ? r * LV_BLOCK + wid * WAVE + __ffsll((unsigned long long)hi) - 1 : aw;
            u8 out = v;
            if (v == 1) {
                const int pa = s_prev[j] == LV_NONE ? -1 : (int)s_prev[j];
                const int a = lv_resolve_prev(s_m, sh, pa, fr[r]);
                const int c = lv_resolve_next(s_m, sh, nx, lr[r], W);
                if (a == -2 || c == -2) {
                    out = 2;
                } else {
                    const u64 m0 = s_mu[j];
                    const int d0 = c >= 0 ? delta_k(m0, s_mu[c]) : -1;
                    const int dm1 = a >= 0 ? delta_k(s_mu[a], m0) : -1;
                    if (d0 < dm1) {                   // else kept whatever lies beyond a
                        const int pb = s_prev[a] == LV_NONE ? -1 : (int)s_prev[a];   // a >= 0 here
                        const int b = lv_resolve_prev(s_m, sh, pb, fr[r]);
                        if (b == -2) out = 2;
                        else {
                            const int dm2 = b >= 0 ? delta_k(s_mu[b], s_mu[a]) : -1;
                            out = (dm2 < dm1) ? 0 : 1;
                        }
                    }
                }
            }
            s_m[j] = (u8)((byte & (3u << sh)) | (out << nsh));
        }
        __syncthreads();
        cur ^= 1;
    }
    const int fsh = 2 * cur;
    // the tile's rows: kept counts per (row, wave), scanned by the first wave
    const int r0 = (int)(t0 - w0) / LV_BLOCK;
    const int te = (int)(t1 - w0);
    bool unknown = false;
#pragma unroll
    for (int q = 0; q < LV_ITEMS; ++q) {
        const int j = (r0 + q) * LV_BLOCK + threadIdx.x;
        const u8 v = j < te ? (s_m[j] >> fsh) & 3 : 0;
        unknown |= v == 2;
        const u64 km = __ballot(v == 1);
        if (lane == 0) s_cnt[q * LV_NW + wid] = (u32)__popcll(km);
    }
    const bool bad = __syncthreads_or(unknown) != 0;
    __syncthreads();                          // s_cnt complete
    if (threadIdx.x < WAVE) {
        const u32 x = bad ? 0u : s_cnt[lane];    // keep the look-back of later tiles going
        u32 incl = x;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const u32 y = __shfl_up(incl, d, WAVE);
            if (lane >= d) incl += y;
        }
        s_cnt[lane] = incl - x;
        if (lane == WAVE - 1) s_tot = incl;
        if (bad && lane == 0) atomicOr(&flag[0], 1u);
    }
    __syncthreads();
    const u32 tot = s_tot;
    // decoupled look-back by the first wave, 64 earlier tiles per round: each
    // lane reads one status word; the nearest inclusive prefix ends the walk
    if (threadIdx.x < WAVE) {
        u32* mine = status + tile;
        u32 excl = 0;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(mine, LV_PREFIX | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(mine, LV_AGG | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            i64 base = tile - 1;            // the round reads tiles base, base-1, ..., base-63
            u32 spins = 0;
            for (;;) {
                const i64 t2 = base - lane;
                const u32 sw = t2 >= 0 ? __hip_atomic_load(status + t2, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)
                                       : LV_PREFIX;        // before tile 0: prefix 0
                const u64 pre = __ballot((sw & ~LV_VAL) == LV_PREFIX);
                const u64 none = __ballot((sw & ~LV_VAL) == 0u);
                // lanes up to the nearest prefix (all 64 when there is none)
                const int last = pre ? __ffsll((unsigned long long)pre) - 1 : WAVE - 1;
                const u64 need = last == WAVE - 1 ? ~0ull : ((1ull << (last + 1)) - 1ull);
                if (none & need) {
                    if (++spins > LV_SPIN_LIMIT) {
                        if (lane == 0) atomicOr(&flag[1], 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                u32 v = lane <= last ? (sw & LV_VAL) : 0u;
#pragma unroll
                for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
                excl += v;
                if (pre) break;
                base -= WAVE;
            }
            if (lane == 0)
                __hip_atomic_store(mine, LV_PREFIX | ((excl + tot) & LV_VAL), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_excl = excl;
            if (tile == ntiles - 1) {
                xscan[n] = excl + tot;
                id[excl + tot] = (u32)n;
            }
        }
    }
    __syncthreads();
    const u32 ex = s_excl;
#pragma unroll
    for (int q = 0; q < LV_ITEMS; ++q) {
        const int j = (r0 + q) * LV_BLOCK + threadIdx.x;
        const u8 v = j < te ? (s_m[j] >> fsh) & 3 : 0;
        const u64 km = __ballot(v == 1);
        if (j < te) {
            const i64 i = w0 + j;
            const u32 k = ex + s_cnt[q * LV_NW + wid] + (u32)__popcll(km & below);
            xi[i] = v;
            xscan[i] = k;
            if (v == 1 && !bad) {
                id[k] = (u32)i;
                mu_leaf[k] = s_mu[j];
            }
        }
    }
}

// Per-instance leaf ranges: leaf_off[k] = number of kept codes before the
// instance's first particle (leaf_off[ninst] = all leaves); root node of each
// instance.
// Node numbering: internal nodes 0 .. ni-1 (ni = leaves - instances), leaf j
// at node lbase + j, where lbase >= ni is fixed by the caller (the largest ni
// the particle count allows), so that no launch needs the leaf count.
__global__ void k_inst_leaves(const i64* __restrict__ p_off, int ninst, const u32* __restrict__ xscan,
                              i64 n, i64* __restrict__ leaf_off, i64* __restrict__ ioff,
                              u32* __restrict__ root, u32* __restrict__ parent, i64 lbase)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > ninst) return;
    const i64 lo = xscan[p_off[k]];
    leaf_off[k] = lo;
    ioff[k] = lo - k;
    if (k < ninst) {
        const i64 hi = xscan[p_off[k + 1]];
        const u32 r = (hi - lo > 1) ? (u32)(lo - k) : (u32)(lbase + lo);
        root[k] = r;
        parent[r] = 0xffffffffu;
    }
}

// ---------------------------------------------------------------------------
// Karras radix tree (App. B.7): one thread per internal node, no ordering
// between nodes.  Direction from the larger of the neighbouring prefix
// lengths, range end by exponential + binary search, split by binary search
// for the last code sharing more than delta_node bits with node i.
// ---------------------------------------------------------------------------
__device__ inline int dlt(const u64* m, i64 nl, i64 i, i64 j)
{
    if (j < 0 || j >= nl) return -1;
    return __clzll(m[i] ^ m[j]);
}

__global__ void k_karras(const u64* __restrict__ mu_leaf, const i64* __restrict__ leaf_off,
                         const i64* __restrict__ ioff, int ninst, i64 lbase, TreePtrs t)
{
    const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= leaf_off[ninst] - ninst) return;     // internal nodes: leaves - instances
    const int k = find_seg(ioff, ninst, g);
    const i64 L0 = leaf_off[k];
    const i64 nl = leaf_off[k + 1] - L0;
    const i64 i = g - ioff[k];
    const u64* m = mu_leaf + L0;
    const int d = (dlt(m, nl, i, i + 1) - dlt(m, nl, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = dlt(m, nl, i, i - d);
    i64 lmax = 2;
    while (dlt(m, nl, i, i + lmax * d) > dmin) lmax <<= 1;
    i64 l = 0;
    for (i64 s = lmax >> 1; s >= 1; s >>= 1)
        if (dlt(m, nl, i, i + (l + s) * d) > dmin) l += s;
    const i64 j = i + l * d;
    const int dnode = dlt(m, nl, i, j);
    i64 s = 0, step = l;
    do {
        step = (step + 1) >> 1;
        if (dlt(m, nl, i, i + (s + step) * d) > dnode) s += step;
    } while (step > 1);
    const i64 gam = i + s * d + (d < 0 ? -1 : 0);
    const i64 lo = i < j ? i : j, hi = i < j ? j : i;
    const bool lleaf = (lo == gam), rleaf = (hi == gam + 1);
    t.lchild[g] = (u32)gam;
    t.rchild[g] = (u32)(gam + 1);
    t.lflag[g] = lleaf;
    t.rflag[g] = rleaf;
    t.endrange[g] = (u32)j;
    const u32 cl = lleaf ? (u32)(lbase + L0 + gam) : (u32)(ioff[k] + gam);
    const u32 cr = rleaf ? (u32)(lbase + L0 + gam + 1) : (u32)(ioff[k] + gam + 1);
    t.child[2 * g] = cl;
    t.child[2 * g + 1] = cr;
    t.parent[cl] = (u32)g;
    t.parent[cr] = (u32)g;
}

// ---------------------------------------------------------------------------
// Cell boxes, bottom-up (tight AABB + h_max of every node).  Pass 1: each
// workgroup owns BOX_BLK consecutive leaves; a thread computes its leaf's box
// from the leaf's particles (h = posh.w, the h the cache is built with), then
// climbs: at a parent whose whole leaf range lies in the block, the second of
// the two arriving threads (LDS counters) merges the children's boxes (held
// in LDS) and continues.  A climb that reaches a parent straddling two blocks
// records its node and stops.  Pass 2 (one workgroup) finishes the nodes
// above those records with workgroup-scope arrival counters in memory.  No
// device-wide fence is needed anywhere.
// Node layout: lo = (xmin, ymin, zmin, hmax), hi = (xmax, ymax, zmax, 0).
// ---------------------------------------------------------------------------
constexpr int BOX_BLK = 1024;
constexpr int BOX_OUT = 128;     // records per block: at most 2 * depth <= 126
constexpr int TOP_BLOCK = 1024;

// Leaf range [f, l] (global leaf indices) of internal node p and its
// Karras index in global leaf numbering.
__device__ inline void node_span(u32 p, const i64* ioff, const i64* leaf_off, int ninst,
                                 const u32* endrange, i64& f, i64& l, i64& kidx)
{
    const int k = find_seg(ioff, ninst, (i64)p);
    const i64 L0 = leaf_off[k];
    const i64 i = (i64)p - ioff[k], j = endrange[p];
    f = L0 + (i < j ? i : j);
    l = L0 + (i < j ? j : i);
    kidx = L0 + i;
}

template <class T>
__global__ void __launch_bounds__(BOX_BLK)
k_boxes_local(const vec4<T>* __restrict__ posh, const u32* __restrict__ id, i64 lbase,
              const u32* __restrict__ child, const u32* __restrict__ parent,
              const u32* __restrict__ endrange, const i64* __restrict__ ioff,
              const i64* __restrict__ leaf_off, int ninst, vec4<T>* __restrict__ blo,
              vec4<T>* __restrict__ bhi, u32* __restrict__ rec, u32* __restrict__ nrec,
              u32* __restrict__ flags, const u32* __restrict__ skip)
{
    __shared__ vec4<T> s_llo[BOX_BLK], s_lhi[BOX_BLK];   // leaves of the block
    if (skip && *skip) return;
    __shared__ vec4<T> s_nlo[BOX_BLK], s_nhi[BOX_BLK];   // internal nodes, by Karras index
    __shared__ u32 s_arr[BOX_BLK];
    __shared__ u32 s_rec[BOX_OUT];
    __shared__ u32 s_nrec;
    const i64 n_leaf = leaf_off[ninst];
    const i64 B0 = (i64)blockIdx.x * BOX_BLK;
    const i64 B1 = (B0 + BOX_BLK) < n_leaf ? (B0 + BOX_BLK) : n_leaf;
    const int t = threadIdx.x;
    s_arr[t] = 0;
    if (t == 0) s_nrec = 0;
    const i64 g = B0 + t;
    const bool live = g < B1;
    T lo0 = 0, lo1 = 0, lo2 = 0, hi0 = 0, hi1 = 0, hi2 = 0, hm = 0;
    if (live) {
        const u32 b0 = id[g], b1 = id[g + 1];
        vec4<T> p = posh[b0];
        lo0 = hi0 = p.x; lo1 = hi1 = p.y; lo2 = hi2 = p.z; hm = p.w;
        // four independent loads in flight per round (a slot past the leaf
        // repeats its first particle, which changes no min or max)
        for (u32 b = b0 + 1; b < b1; b += 4) {
            vec4<T> q[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = posh[b + k < b1 ? b + k : b0];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                lo0 = fmin(lo0, q[k].x); lo1 = fmin(lo1, q[k].y); lo2 = fmin(lo2, q[k].z);
                hi0 = fmax(hi0, q[k].x); hi1 = fmax(hi1, q[k].y); hi2 = fmax(hi2, q[k].z);
                hm = fmax(hm, q[k].w);
            }
        }
        const vec4<T> l = mk4<T>(lo0, lo1, lo2, hm), h = mk4<T>(hi0, hi1, hi2, T(0));
        s_llo[t] = l;
        s_lhi[t] = h;
        blo[lbase + g] = l;
        bhi[lbase + g] = h;
    }
    __syncthreads();
    if (live) {
        u32 node = (u32)(lbase + g);
        u32 par = parent[node];
        while (par != 0xffffffffu) {
            // the read-only topology of this level (span, children, the next
            // parent, the sibling's Karras index) before the counter
            i64 f, l, kidx;
            node_span(par, ioff, leaf_off, ninst, endrange, f, l, kidx);
            const u32 c0 = child[2 * par], c1 = child[2 * par + 1];
            const u32 gp = parent[par];
            if (f < B0 || l >= B1) {               // parent straddles blocks
                const u32 q = atomicAdd(&s_nrec, 1u);
                if (q < BOX_OUT) s_rec[q] = node;
                break;
            }
            const int ps = (int)(kidx - B0);
            const u32 other = (c0 == node) ? c1 : c0;
            i64 k2 = 0;
            if (other < lbase) {
                i64 f2, l2;
                node_span(other, ioff, leaf_off, ninst, endrange, f2, l2, k2);
            }
            __threadfence_block();
            if (atomicAdd(&s_arr[ps], 1u) == 0) break;   // the sibling's thread continues
            __threadfence_block();
            vec4<T> ol, oh;
            if (other >= lbase) {
                ol = s_llo[other - lbase - B0];
                oh = s_lhi[other - lbase - B0];
            } else {
                ol = s_nlo[k2 - B0];
                oh = s_nhi[k2 - B0];
            }
            lo0 = fmin(lo0, ol.x); lo1 = fmin(lo1, ol.y); lo2 = fmin(lo2, ol.z); hm = fmax(hm, ol.w);
            hi0 = fmax(hi0, oh.x); hi1 = fmax(hi1, oh.y); hi2 = fmax(hi2, oh.z);
            const vec4<T> nl = mk4<T>(lo0, lo1, lo2, hm), nh = mk4<T>(hi0, hi1, hi2, T(0));
            s_nlo[ps] = nl;
            s_nhi[ps] = nh;
            blo[par] = nl;
            bhi[par] = nh;
            node = par;
            par = gp;
        }
    }
    __syncthreads();
    const u32 nr = s_nrec < BOX_OUT ? s_nrec : BOX_OUT;
    for (u32 q = t; q < nr; q += BOX_BLK) rec[(i64)blockIdx.x * BOX_OUT + q] = s_rec[q];
    if (t == 0) {
        nrec[blockIdx.x] = nr;
        if (s_nrec > BOX_OUT) atomicOr(flags, 16u);
    }
}

// Middle level: workgroup c takes the climbs recorded by local blocks
// c*BOX_MID .. c*BOX_MID + BOX_MID - 1 (one thread per block) and finishes
// every parent whose leaf range lies inside those blocks' leaves, with
// workgroup-scope arrival counters (both children of such a parent are
// climbed by threads of this workgroup); climbs whose parent leaves that
// range are recorded again for the top pass.
constexpr int BOX_MID = 64;

template <class T>
__global__ void __launch_bounds__(BOX_MID)
k_boxes_mid(const u32* __restrict__ rec, const u32* __restrict__ nrec, i64 nblocks,
            const u32* __restrict__ child, const u32* __restrict__ parent,
            const u32* __restrict__ endrange, const i64* __restrict__ ioff,
            const i64* __restrict__ leaf_off, int ninst, u32* __restrict__ arrive, vec4<T>* blo,
            vec4<T>* bhi, u32* __restrict__ rec2, u32* __restrict__ nrec2, u32* __restrict__ flags,
            const u32* __restrict__ skip)
{
    __shared__ u32 s_rec[BOX_OUT];
    __shared__ u32 s_nrec;
    if (skip && *skip) return;
    if (threadIdx.x == 0) s_nrec = 0;
    __syncthreads();
    const i64 n_leaf = leaf_off[ninst];
    const i64 b = (i64)blockIdx.x * BOX_MID + threadIdx.x;
    const i64 C0 = (i64)blockIdx.x * BOX_MID * BOX_BLK;
    const i64 C1 = (C0 + (i64)BOX_MID * BOX_BLK) < n_leaf ? (C0 + (i64)BOX_MID * BOX_BLK) : n_leaf;
    if (b < nblocks) {
        const u32 nr = nrec[b];
        for (u32 q = 0; q < nr; ++q) {
            u32 node = rec[b * BOX_OUT + q];
            vec4<T> ml = blo[node], mh = bhi[node];
            u32 par = parent[node];
            while (par != 0xffffffffu) {
                // the read-only topology of this level (span, children, the
                // next parent) in one round of loads
                i64 f, l, kidx;
                node_span(par, ioff, leaf_off, ninst, endrange, f, l, kidx);
                const u32 c0 = child[2 * par], c1 = child[2 * par + 1];
                const u32 gp = parent[par];
                if (f < C0 || l >= C1) {               // parent straddles this range
                    const u32 r = atomicAdd(&s_nrec, 1u);
                    if (r < BOX_OUT) s_rec[r] = node;
                    break;
                }
                // release fence + counter + acquire fence: the second arrival
                // sees the first one's box
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                const u32 prev = __hip_atomic_fetch_add(&arrive[par], 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                if (prev == 0) break;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const u32 other = (c0 == node) ? c1 : c0;
                const vec4<T> ol = blo[other], oh = bhi[other];
                ml = mk4<T>(fmin(ml.x, ol.x), fmin(ml.y, ol.y), fmin(ml.z, ol.z), fmax(ml.w, ol.w));
                mh = mk4<T>(fmax(mh.x, oh.x), fmax(mh.y, oh.y), fmax(mh.z, oh.z), T(0));
                blo[par] = ml;
                bhi[par] = mh;
                node = par;
                par = gp;
            }
        }
    }
    __syncthreads();
    const u32 nr = s_nrec < BOX_OUT ? s_nrec : BOX_OUT;
    for (u32 q = threadIdx.x; q < nr; q += BOX_MID) rec2[(i64)blockIdx.x * BOX_OUT + q] = s_rec[q];
    if (threadIdx.x == 0) {
        nrec2[blockIdx.x] = nr;
        if (s_nrec > BOX_OUT) atomicOr(flags, 16u);
    }
}

template <class T>
__global__ void __launch_bounds__(TOP_BLOCK)
k_boxes_top(const u32* __restrict__ rec, const u32* __restrict__ nrec, i64 nblocks,
            const u32* __restrict__ child, const u32* __restrict__ parent,
            u32* __restrict__ arrive, vec4<T>* blo, vec4<T>* bhi, const u32* __restrict__ skip)
{
    if (skip && *skip) return;
    // thread t finishes the climbs recorded by blocks t, t + TOP_BLOCK, ...
    for (i64 b = threadIdx.x; b < nblocks; b += TOP_BLOCK) {
        const u32 nr = nrec[b];
        for (u32 q = 0; q < nr; ++q) {
            u32 node = rec[b * BOX_OUT + q];
            vec4<T> ml = blo[node], mh = bhi[node];
            u32 par = parent[node];
            while (par != 0xffffffffu) {
                // release fence + counter + acquire fence: the second arrival
                // sees the first one's box; the read-only topology of the
                // level (children, next parent) loads while the counter does
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                const u32 prev = __hip_atomic_fetch_add(&arrive[par], 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                const u32 c0 = child[2 * par], c1 = child[2 * par + 1];
                const u32 gp = parent[par];
                if (prev == 0) break;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const u32 other = (c0 == node) ? c1 : c0;
                const vec4<T> ol = blo[other], oh = bhi[other];
                ml = mk4<T>(fmin(ml.x, ol.x), fmin(ml.y, ol.y), fmin(ml.z, ol.z), fmax(ml.w, ol.w));
                mh = mk4<T>(fmax(mh.x, oh.x), fmax(mh.y, oh.y), fmax(mh.z, oh.z), T(0));
                blo[par] = ml;
                bhi[par] = mh;
                node = par;
                par = gp;
            }
        }
    }
}

// Integer prefix boxes (App. B.6, Eqs. lowboundbox/highboundbox): internal
// nodes use delta(first, last) bits of their codes, leaves their parent's
// length + 1; corners p0 = code & mask, p1 = p0 | ~mask, de-interleaved.
__device__ inline u32 compact3(u64 x)
{
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x100f00f00f00f00full;
    x = (x | (x >> 8)) & 0x001f0000ff0000ffull;
    x = (x | (x >> 16)) & 0x001f00000000ffffull;
    x = (x | (x >> 32)) & 0x00000000001fffffull;
    return (u32)x;
}

// Output rows in compact numbering: internal nodes, then leaf j at row
// n_internal + j (its parent read at node lbase + j).
__global__ void k_prefix_boxes(const u64* __restrict__ mu_leaf, const i64* __restrict__ leaf_off,
                               const i64* __restrict__ ioff, int ninst, i64 n_internal, i64 n_leaf,
                               i64 lbase, const u32* __restrict__ endrange,
                               const u32* __restrict__ parent, u32* __restrict__ pbox,
                               i32* __restrict__ plen, int shift)
{
    // shorter codes (30 bits in the low bits) are read in the 63-bit layout:
    // the code moved up by `shift` and its prefix lengths shortened by as much
    const i64 v = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_internal + n_leaf) return;
    auto range_len = [&](i64 g) {
        const int k = find_seg(ioff, ninst, g);
        const i64 L0 = leaf_off[k];
        const i64 i = g - ioff[k], j = endrange[g];
        return __clzll(mu_leaf[L0 + i] ^ mu_leaf[L0 + j]);
    };
    int len;
    u64 code;
    if (v < n_internal) {
        const int k = find_seg(ioff, ninst, v);
        const i64 i = v - ioff[k], j = endrange[v];
        code = mu_leaf[leaf_off[k] + (i < j ? i : j)];
        len = range_len(v);
    } else {
        code = mu_leaf[v - n_internal];
        const u32 p = parent[lbase + (v - n_internal)];
        len = (p == 0xffffffffu) ? 0 : range_len(p) + 1;
    }
    if (len > 0) len -= shift;
    code <<= shift;
    const u64 mask = (len >= 64) ? ~0ull : ~((~0ull) >> len);
    const u64 p0 = code & mask;
    const u64 p1 = p0 | (~mask & 0x7fffffffffffffffull);
    u32* o = pbox + 6 * v;
    o[0] = compact3(p0 >> 2); o[1] = compact3(p0 >> 1); o[2] = compact3(p0);
    o[3] = compact3(p1 >> 2); o[4] = compact3(p1 >> 1); o[5] = compact3(p1);
    plen[v] = len;
}

// ---------------------------------------------------------------------------
// Isolated instances: the box is the extent of the (predicted) positions.
// Reduced as order-preserving 64-bit integers of the FP64 values.
// ---------------------------------------------------------------------------
__device__ inline u64 ord64(double d)
{
    const u64 b = (u64)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double unord64(u64 k)
{
    const u64 b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}

__global__ void k_bbox_init(u64* bb, int ninst)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ninst) return;
    for (int d = 0; d < 3; ++d) { bb[6 * k + d] = ~0ull; bb[6 * k + 3 + d] = 0ull; }
}

constexpr int BB_ITEMS = 16;

template <class T>
__global__ void k_bbox_reduce(FieldPtrs<T> f, i64 n, const InstDev* __restrict__ inst,
                              const i64* __restrict__ p_off, int ninst,
                              const double* __restrict__ dt_inst, u64* __restrict__ bb)
{
    const i64 i0 = ((i64)blockIdx.x * blockDim.x + threadIdx.x) * BB_ITEMS;
    const bool live = i0 < n;
    int k = find_seg(p_off, ninst, live ? i0 : n - 1);
    u64 mn[3] = { ~0ull, ~0ull, ~0ull }, mx[3] = { 0ull, 0ull, 0ull };
    bool any = false;
    auto flush_lane = [&](int kk) {
        if (any && !inst[kk].periodic)
            for (int d = 0; d < 3; ++d) { atomicMin(&bb[6 * kk + d], mn[d]); atomicMax(&bb[6 * kk + 3 + d], mx[d]); }
        for (int d = 0; d < 3; ++d) { mn[d] = ~0ull; mx[d] = 0ull; }
        any = false;
    };
    if (live) {
        for (int t = 0; t < BB_ITEMS; ++t) {
            const i64 i = i0 + t;
            if (i >= n) break;
            if (i >= p_off[k + 1]) { flush_lane(k); k = find_seg(p_off, ninst, i); }
            const InstDev in = inst[k];
            if (in.periodic) continue;
            double p[3];
            if (dt_inst) {
                const Box<T> bx = make_box<T>(in);
                const T* xp[3] = { f.x, f.y, f.z };
                const T* vp[3] = { f.vx, f.vy, f.vz };
                const T* ap[3] = { f.ax, f.ay, f.az };
                Pred<T> o;
                predict<T>(xp, vp, f.ax ? ap : nullptr, f.u, f.du, i + in.shift, (T)dt_inst[k], bx, o);
                p[0] = o.x[0]; p[1] = o.x[1]; p[2] = o.x[2];
            } else {
                const i64 ic = i + in.shift;
                p[0] = f.x[ic]; p[1] = f.y[ic]; p[2] = f.z[ic];
            }
            for (int d = 0; d < 3; ++d) {
                const u64 o = ord64(p[d]);
                mn[d] = o < mn[d] ? o : mn[d];
                mx[d] = o > mx[d] ? o : mx[d];
            }
            any = true;
        }
    }
    // the wave's lanes usually share one instance: reduce, one atomic per wave
    const int k0 = __shfl(k, 0, WAVE);
    const bool uni = __ballot(live && k != k0) == 0;
    if (uni) {
        const bool anyw = __ballot(any) != 0;
        for (int d = 0; d < 3; ++d) {
            u64 a = mn[d], b = mx[d];
            for (int s = WAVE / 2; s > 0; s >>= 1) {
                const u64 oa = __shfl_xor(a, s, WAVE), ob = __shfl_xor(b, s, WAVE);
                a = oa < a ? oa : a;
                b = ob > b ? ob : b;
            }
            mn[d] = a; mx[d] = b;
        }
        if (__lane_id() == 0 && anyw && !inst[k0].periodic)
            for (int d = 0; d < 3; ++d) { atomicMin(&bb[6 * k0 + d], mn[d]); atomicMax(&bb[6 * k0 + 3 + d], mx[d]); }
    } else if (live) {
        flush_lane(k);
    }
}

__global__ void k_bbox_finish(InstDev* inst, const u64* bb, int ninst)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ninst || inst[k].periodic) return;
    for (int d = 0; d < 3; ++d) {
        inst[k].lo[d] = unord64(bb[6 * k + d]);
        inst[k].hi[d] = unord64(bb[6 * k + 3 + d]);
    }
}

template <class T>
void launch_bbox(const FieldPtrs<T>& f, i64 n, InstDev* inst, const i64* p_off, int ninst,
                 const double* dt_inst, u64* bb, hipStream_t st)
{
    hipLaunchKernelGGL(k_bbox_init, grid_for(ninst, 64), dim3(64), 0, st, bb, ninst);
    const i64 nt = (n + BB_ITEMS - 1) / BB_ITEMS;
    if (nt > 0)
        hipLaunchKernelGGL((k_bbox_reduce<T>), grid_for(nt, 256), dim3(256), 0, st, f, n, inst, p_off,
                           ninst, dt_inst, bb);
    hipLaunchKernelGGL(k_bbox_finish, grid_for(ninst, 64), dim3(64), 0, st, inst, bb, ninst);
}

// ------------------------------------------------------------ launchers ----
template <class T>
void launch_predict_morton(const FieldPtrs<T>& f, i64 n, const InstDev* inst, const i64* p_off,
                           int ninst, const double* dt_inst, u64* keys, u32* vals, int bits,
                           hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL((k_predict_morton<T>), grid_for(n, 256), dim3(256), 0, st, f, n, inst, p_off,
                       ninst, dt_inst, keys, vals, bits);
}

template <class T>
void launch_gather(const FieldPtrs<T>& f, i64 n, const InstDev* inst, const i64* p_off, int ninst,
                   const double* dt_inst, const u32* eps, const SortedPtrs<T>& s, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL((k_gather<T>), grid_for(n, 256), dim3(256), 0, st, f, n, inst, p_off, ninst,
                       dt_inst, eps, s);
}

void launch_mask_init(const u64* mu, i64 n, const i64* p_off, int ninst, u8* xi, hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_init, grid_for(n, 256), dim3(256), 0, st, mu, n, p_off, ninst, xi);
}

void launch_reduce_pass(const u64* mu, i64 n, const i64* p_off, int ninst, const u8* xold, u8* xnew,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_pass, grid_for(n, 256), dim3(256), 0, st, mu, n, p_off, ninst, xold,
                       xnew);
}

void launch_compact(const u64* mu, const u8* xi, const u32* xscan, i64 n, u32* id, u64* mu_leaf,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_compact, grid_for(n, 256), dim3(256), 0, st, mu, xi, xscan, n, id, mu_leaf);
}

size_t leaves_fused_state_words(i64 n) { return 1 + (size_t)((n + LV_TILE - 1) / LV_TILE); }

void launch_leaves_fused(const u64* mu, i64 n, const i64* p_off, int ninst, int nred, u32* state,
                         u8* xi, u32* xscan, u32* id, u64* mu_leaf, u32* flag, hipStream_t st)
{
    const i64 ntiles = (n + LV_TILE - 1) / LV_TILE;
    launch_fill_u32(state, (i64)leaves_fused_state_words(n), 0u, st);
    if (ninst > 1)
        hipLaunchKernelGGL(k_leaves_fused<true>, dim3((unsigned)ntiles), dim3(LV_BLOCK), 0, st, mu, n,
                           p_off, ninst, nred, state, state + 1, xi, xscan, id, mu_leaf, flag);
    else
        hipLaunchKernelGGL(k_leaves_fused<false>, dim3((unsigned)ntiles), dim3(LV_BLOCK), 0, st, mu, n,
                           p_off, ninst, nred, state, state + 1, xi, xscan, id, mu_leaf, flag);
}

void launch_inst_leaves(const i64* p_off, int ninst, const u32* xscan, i64 n, i64* leaf_off,
                        i64* ioff, u32* root, u32* parent, i64 lbase, hipStream_t st)
{
    hipLaunchKernelGGL(k_inst_leaves, grid_for(ninst + 1, 64), dim3(64), 0, st, p_off, ninst, xscan,
                       n, leaf_off, ioff, root, parent, lbase);
}

void launch_karras(const u64* mu_leaf, const i64* leaf_off, const i64* ioff, int ninst,
                   i64 lbase, i64 grid_internal, const TreePtrs& t, hipStream_t st)
{
    if (grid_internal <= 0) return;
    hipLaunchKernelGGL(k_karras, grid_for(grid_internal, 256), dim3(256), 0, st, mu_leaf, leaf_off,
                       ioff, ninst, lbase, t);
}

template <class T>
void launch_boxes_up(const vec4<T>* posh, const u32* id, i64 grid_leaves, i64 lbase,
                     const u32* child, const u32* parent, const u32* endrange, const i64* ioff,
                     const i64* leaf_off, int ninst, u32* arrive, u32* rec, u32* nrec,
                     u32* rscan, void* scan_tmp, vec4<T>* blo, vec4<T>* bhi, u32* flags,
                     hipStream_t st, const u32* skip)
{
    if (grid_leaves <= 0) return;
    const i64 nb = (grid_leaves + BOX_BLK - 1) / BOX_BLK;
    hipLaunchKernelGGL((k_boxes_local<T>), dim3((unsigned)nb), dim3(BOX_BLK), 0, st, posh, id,
                       lbase, child, parent, endrange, ioff, leaf_off, ninst, blo, bhi, rec,
                       nrec, flags, skip);
    if (nb > 1) {
        // middle level (ranges of BOX_MID local blocks), then one workgroup
        // for the climbs that cross those ranges
        const i64 nb2 = (nb + BOX_MID - 1) / BOX_MID;
        u32* rec2 = rec + nb * BOX_OUT;
        u32* nrec2 = nrec + nb;
        hipLaunchKernelGGL((k_boxes_mid<T>), dim3((unsigned)nb2), dim3(BOX_MID), 0, st, rec, nrec,
                           nb, child, parent, endrange, ioff, leaf_off, ninst, arrive, blo,
                           bhi, rec2, nrec2, flags, skip);
        if (nb2 > 1)
            hipLaunchKernelGGL((k_boxes_top<T>), dim3(1), dim3(TOP_BLOCK), 0, st, rec2, nrec2, nb2,
                               child, parent, arrive, blo, bhi, skip);
    }
}

// Record space: BOX_OUT per local block, then BOX_OUT per middle range.
size_t boxes_rec_count(i64 n_leaf)
{
    const i64 nb = (n_leaf + BOX_BLK - 1) / BOX_BLK;
    return (size_t)(nb + (nb + BOX_MID - 1) / BOX_MID) * BOX_OUT;
}

void launch_prefix_boxes(const u64* mu_leaf, const i64* leaf_off, const i64* ioff, int ninst,
                         i64 n_internal, i64 n_leaf, i64 lbase, const u32* endrange,
                         const u32* parent, u32* pbox, i32* plen, int shift, hipStream_t st)
{
    const i64 nn = n_internal + n_leaf;
    if (nn <= 0) return;
    hipLaunchKernelGGL(k_prefix_boxes, grid_for(nn, 256), dim3(256), 0, st, mu_leaf, leaf_off, ioff,
                       ninst, n_internal, n_leaf, lbase, endrange, parent, pbox, plen, shift);
}

#define INST(T)                                                                                   \
    template void launch_predict_morton<T>(const FieldPtrs<T>&, i64, const InstDev*, const i64*,  \
                                           int, const double*, u64*, u32*, int, hipStream_t);     \
    template void launch_gather<T>(const FieldPtrs<T>&, i64, const InstDev*, const i64*, int,     \
                                   const double*, const u32*, const SortedPtrs<T>&, hipStream_t); \
    template void launch_bbox<T>(const FieldPtrs<T>&, i64, InstDev*, const i64*, int,            \
                                 const double*, u64*, hipStream_t);                               \
    template void launch_boxes_up<T>(const vec4<T>*, const u32*, i64, i64, const u32*,            \
                                     const u32*, const u32*, const i64*, const i64*, int, u32*,   \
                                     u32*, u32*, u32*, void*, vec4<T>*, vec4<T>*, u32*,           \
                                     hipStream_t, const u32*);
INST(float)
INST(double)
#undef INST

}  // namespace shsph
