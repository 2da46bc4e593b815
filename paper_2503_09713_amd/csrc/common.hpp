// Device-side building blocks shared by the shsph kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shsph {

typedef uint8_t u8;
typedef uint16_t u16;
typedef uint32_t u32;
typedef uint64_t u64;
typedef int32_t i32;
typedef int64_t i64;

constexpr int WAVE = 64;
constexpr int MORTON_BITS = 21;             // per axis, 63-bit keys (App. B.1)
constexpr u32 MORTON_MAX = (1u << MORTON_BITS) - 1u;

// ---------------------------------------------------------------- vectors --
template <class T> struct V4;
template <> struct V4<float> { typedef float4 type; };
template <> struct V4<double> { typedef double4 type; };
template <class T> using vec4 = typename V4<T>::type;

template <class T> __host__ __device__ inline vec4<T> mk4(T a, T b, T c, T d)
{
    vec4<T> v; v.x = a; v.y = b; v.z = c; v.w = d; return v;
}

// ------------------------------------------------------- instance table ----
// One row per independent SPH instance; the plain API is a table of one.
struct InstDev {
    i64 p_off, p_cnt;        // particle range in the (batched) arrays
    i64 shift;               // caller-array index = batch index + shift (0 for
                             // caller arrays; pool offset - p_off for pooled
                             // instances, which live anywhere in the pool)
    double lo[3], hi[3];     // box; isolated instances get the data extent
    double mass;
    i32 periodic;
    i32 pad;
};

// Per-instance reductions written by the step kernels.  Sums are spread
// over STAT_SLOTS partial slots (slot = block index mod STAT_SLOTS) so that
// no single address takes an atomic from every workgroup.
constexpr int STAT_SLOTS = 16;
struct InstStat {
    u32 dt_bits;             // CFL dt as the bit pattern of a positive float
    u32 dvmax_bits;          // max |dv| (positive float bits)
    u32 n_exceed, n_noconv;  // h iteration outcome counters
    u32 max_iter_seen;
    u32 pad[3];
    double dv2_part[STAT_SLOTS];   // sum |dv|^2
    double v2_part[STAT_SLOTS];    // sum |v|^2
};



// Largest k with off[k] <= i, for a sorted table off[0..n] (binary search).
__device__ inline int find_seg(const i64* off, int n, i64 i)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Particles are processed in groups of GROUP consecutive key-order slots,
// one workgroup per group; groups never straddle two instances.
constexpr int GROUP = 256;
struct GroupMap {
    const i64* goff;    // ninst+1: first group of each instance
    const i64* p_off;   // ninst+1: first particle of each instance
    int ninst;
    __device__ int inst_of(i64 g) const { return find_seg(goff, ninst, g); }
    __device__ i64 ngroups_total() const { return goff[ninst]; }
    __device__ void range(i64 g, i64& beg, i64& end, int& k) const
    {
        k = inst_of(g);
        beg = p_off[k] + (g - goff[k]) * GROUP;
        end = beg + GROUP < p_off[k + 1] ? beg + GROUP : p_off[k + 1];
    }
};

// ------------------------------------------------------ wave primitives ----
__device__ inline u64 lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

template <class T> __device__ inline T wave_incl_scan(T x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    return x;
}

// The same inclusive sum for 32-bit integers with DPP lane moves (no LDS
// round trips): shifts by 1, 2, 4, 8 within each row of 16 lanes, then the
// total of row 0 added into row 1 and of row 2 into row 3 (row_bcast:15),
// then the total of rows 0-1 into rows 2-3 (row_bcast:31).  Lanes a move
// does not write, or whose source lies outside the row, receive 0.
__device__ inline u32 wave_incl_scan_dpp(u32 x)
{
    int v = (int)x;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);    // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);    // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);    // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);    // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return (u32)v;
}

template <class T> __device__ inline T wave_sum(T x)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

template <class T> __device__ inline T wave_max(T x)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) { T y = __shfl_xor(x, d, WAVE); x = y > x ? y : x; }
    return x;
}

template <class T> __device__ inline T wave_min(T x)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) { T y = __shfl_xor(x, d, WAVE); x = y < x ? y : x; }
    return x;
}

// Exclusive scan over a block of BLOCK threads; `lds` holds BLOCK/64 slots.
template <int BLOCK, class T> __device__ inline T block_excl_scan(T v, T* lds, T& total)
{
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
    T x = wave_incl_scan(v);
    if (lane == WAVE - 1) lds[wid] = x;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        T s = lds[w];
        off += (w < wid) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

// Lanes of the wave whose `bits`-bit digit equals this lane's, among `active`.
template <int BITS> __device__ inline u64 match_digit(u32 d, u64 active)
{
    u64 m = active;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool s = (d >> b) & 1u;
        const u64 bal = __ballot(s);
        m &= s ? bal : ~bal;
    }
    return m;
}

// ---------------------------------------------- exact float arithmetic ----
// The neighbour decision and the predicted positions must be bit-identical
// to their CPU definitions (and between kernels), so the code that computes
// them sits in scopes with FMA contraction disabled.

// Periodic box constants in the storage type: L = (T)(hi-lo),
// halfL = (T)(0.5*(hi-lo)).
template <class T> struct Box {
    T L[3], halfL[3];
    T lo[3], hi[3];
    int periodic;
};

template <class T> __device__ inline Box<T> make_box(const InstDev& in)
{
    Box<T> b;
    for (int d = 0; d < 3; ++d) {
        b.L[d] = (T)(in.hi[d] - in.lo[d]);
        b.halfL[d] = (T)(0.5 * (in.hi[d] - in.lo[d]));
        b.lo[d] = (T)in.lo[d];
        b.hi[d] = (T)in.hi[d];
    }
    b.periodic = in.periodic;
    return b;
}

// Minimum image applied once: d -> d - L if d > L/2, d + L if d < -L/2
// (written with selects: no divergent branches).
template <class T> __device__ inline T min_image(T d, T L, T halfL, int periodic)
{
#pragma clang fp contract(off)
    const T dm = d - L, dp = d + L;
    const T w = d > halfL ? dm : (d < -halfL ? dp : d);
    return periodic ? w : d;
}

// A group is interior when its box grown by the largest cache radius
// (rk * h_max of the whole tree, inflated) stays inside the periodic box: then
// every cached pair is closer than half a period and the minimum image is the
// identity, so it can be skipped exactly.
template <class T>
__device__ inline bool group_interior(const vec4<T>& gl, const vec4<T>& gh, T hmax_all, T rk,
                                      const Box<T>& bx)
{
    if (!bx.periodic) return true;
    const T r = rk * hmax_all * T(1.001) + T(1e-5) * (bx.L[0] + bx.L[1] + bx.L[2]);
    return gl.x - r > bx.lo[0] && gl.y - r > bx.lo[1] && gl.z - r > bx.lo[2] &&
           gh.x + r < bx.hi[0] && gh.y + r < bx.hi[1] && gh.z + r < bx.hi[2];
}

// The group cache stores four 16-bit union slots per 64-bit word, ELL
// layout word[(gbase[g] + j / 4) * GROUP + lane], slot j at bits 16 (j % 4);
// unused slots of the last word hold SLOT_NONE.  A group whose union holds
// more than 65535 particles (slots_wide) stores 32-bit slots instead, two per
// word: slot j at bits 32 (j % 2) of word j / 2, padding SLOT32_NONE.
constexpr u32 SLOT_NONE = 0xffffu;
constexpr u32 SLOT32_NONE = 0xffffffffu;
__device__ inline u32 slot_of(u64 w, u32 r) { return (u32)(w >> (16u * r)) & 0xffffu; }
__device__ inline u32 slot32_of(u64 w, u32 r) { return (u32)(w >> (32u * r)); }
__host__ __device__ inline bool slots_wide(u32 union_size) { return union_size > 0xffffu; }

// ------------------------------------------------------------- M4 spline --
// f(q) = 1 - 3/2 q^2 + 3/4 q^3 (q<1), (2-q)^3/4 (1<=q<2), 0 beyond;
// C_norm = 1/pi in 3D; the support radius is 2h (Sect. 2.1).
// Both pieces are evaluated and selected (no divergent branches); the outer
// piece uses t = max(2 - q, 0), so it is zero from q = 2 on by itself and a
// single select remains.

template <class T> __device__ inline void m4(T q, T& f, T& df)
{
    const T t = fmax(T(2) - q, T(0));
    const T t2 = t * t;
    const T fi = T(1) + q * q * (T(0.75) * q - T(1.5));
    const T dfi = q * (T(2.25) * q - T(3));
    const T fo = T(0.25) * t2 * t;
    const T dfo = T(-0.75) * t2;
    const bool in1 = q < T(1);
    f = in1 ? fi : fo;
    df = in1 ? dfi : dfo;
}

template <class T> __device__ inline T m4_df(T q)
{
    const T t = fmax(T(2) - q, T(0));
    const T dfi = q * (T(2.25) * q - T(3));
    const T dfo = T(-0.75) * t * t;
    return q < T(1) ? dfi : dfo;
}

template <class T> __device__ inline T inv_pi() { return T(0.318309886183790671537767526745); }

// ------------------------------------------------- kernel family (Sect. 2.1.1) --
// f(q) and f'(q) of the B-splines M4, M5, M6 and the Wendland functions C2,
// C4, C6, with support radius R (in units of h) and 3-D normalisation C:
//   M4  R 2    C 1/pi       (the spline above)
//   M5  R 5/2  C 1/(20 pi)  f = t1^4 - 5 t2^4 + 10 t3^4, t_i = max(5/2, 3/2, 1/2 - q, 0)
//   M6  R 3    C 1/(120 pi) f = t1^5 - 6 t2^5 + 15 t3^5, t_i = max(3, 2, 1 - q, 0)
//   C2  R 2    C 21/(16 pi)   f = t^4 (1 + 2q),                 t = max(1 - q/2, 0)
//   C4  R 2    C 495/(256 pi) f = t^6 (1 + 3q + 35/12 q^2)
//   C6  R 2    C 1365/(512 pi) f = t^8 (1 + 4q + 25/4 q^2 + 4q^3)
// Every piece is clamped at its own breakpoint, so no branch remains.  The
// Wendland derivatives are the simplified products
//   C2: -5 q t^3,  C4: -14/3 q (1 + 5/2 q) t^5,  C6: -11/2 q (1 + 7/2 q + 4 q^2) t^7.
enum KernelId { KM4 = 0, KM5 = 1, KM6 = 2, KC2 = 3, KC4 = 4, KC6 = 5, KERNEL_COUNT = 6 };

inline double kernel_support(int k) { return k == KM5 ? 2.5 : (k == KM6 ? 3.0 : 2.0); }

template <int K> struct Kern;

template <> struct Kern<KM4> {
    template <class T> __device__ static T R() { return T(2); }
    template <class T> __device__ static T C() { return inv_pi<T>(); }
    template <class T> __device__ static void fdf(T q, T& f, T& df) { m4<T>(q, f, df); }
    template <class T> __device__ static T df(T q) { return m4_df<T>(q); }
};

template <> struct Kern<KM5> {
    template <class T> __device__ static T R() { return T(2.5); }
    template <class T> __device__ static T C() { return T(0.05) * inv_pi<T>(); }
    template <class T> __device__ static void fdf(T q, T& f, T& d)
    {
        const T a = fmax(T(2.5) - q, T(0)), b = fmax(T(1.5) - q, T(0)), c = fmax(T(0.5) - q, T(0));
        const T a3 = a * a * a, b3 = b * b * b, c3 = c * c * c;
        f = a3 * a - T(5) * b3 * b + T(10) * c3 * c;
        d = T(-4) * a3 + T(20) * b3 - T(40) * c3;
    }
    template <class T> __device__ static T df(T q)
    {
        const T a = fmax(T(2.5) - q, T(0)), b = fmax(T(1.5) - q, T(0)), c = fmax(T(0.5) - q, T(0));
        return T(-4) * a * a * a + T(20) * b * b * b - T(40) * c * c * c;
    }
};

template <> struct Kern<KM6> {
    template <class T> __device__ static T R() { return T(3); }
    template <class T> __device__ static T C() { return inv_pi<T>() / T(120); }
    template <class T> __device__ static void fdf(T q, T& f, T& d)
    {
        const T a = fmax(T(3) - q, T(0)), b = fmax(T(2) - q, T(0)), c = fmax(T(1) - q, T(0));
        const T a4 = (a * a) * (a * a), b4 = (b * b) * (b * b), c4 = (c * c) * (c * c);
        f = a4 * a - T(6) * b4 * b + T(15) * c4 * c;
        d = T(-5) * a4 + T(30) * b4 - T(75) * c4;
    }
    template <class T> __device__ static T df(T q)
    {
        const T a = fmax(T(3) - q, T(0)), b = fmax(T(2) - q, T(0)), c = fmax(T(1) - q, T(0));
        return T(-5) * (a * a) * (a * a) + T(30) * (b * b) * (b * b) - T(75) * (c * c) * (c * c);
    }
};

template <> struct Kern<KC2> {
    template <class T> __device__ static T R() { return T(2); }
    template <class T> __device__ static T C() { return T(21.0 / 16.0) * inv_pi<T>(); }
    template <class T> __device__ static void fdf(T q, T& f, T& d)
    {
        const T t = fmax(T(1) - T(0.5) * q, T(0)), t3 = t * t * t;
        f = t3 * t * (T(1) + T(2) * q);
        d = T(-5) * q * t3;
    }
    template <class T> __device__ static T df(T q)
    {
        const T t = fmax(T(1) - T(0.5) * q, T(0));
        return T(-5) * q * t * t * t;
    }
};

template <> struct Kern<KC4> {
    template <class T> __device__ static T R() { return T(2); }
    template <class T> __device__ static T C() { return T(495.0 / 256.0) * inv_pi<T>(); }
    template <class T> __device__ static void fdf(T q, T& f, T& d)
    {
        const T t = fmax(T(1) - T(0.5) * q, T(0)), t2 = t * t, t5 = t2 * t2 * t;
        f = t5 * t * (T(1) + q * (T(3) + T(35.0 / 12.0) * q));
        d = T(-14.0 / 3.0) * q * (T(1) + T(2.5) * q) * t5;
    }
    template <class T> __device__ static T df(T q)
    {
        const T t = fmax(T(1) - T(0.5) * q, T(0)), t2 = t * t;
        return T(-14.0 / 3.0) * q * (T(1) + T(2.5) * q) * (t2 * t2 * t);
    }
};

template <> struct Kern<KC6> {
    template <class T> __device__ static T R() { return T(2); }
    template <class T> __device__ static T C() { return T(1365.0 / 512.0) * inv_pi<T>(); }
    template <class T> __device__ static void fdf(T q, T& f, T& d)
    {
        const T t = fmax(T(1) - T(0.5) * q, T(0)), t2 = t * t, t4 = t2 * t2, t7 = t4 * t2 * t;
        f = t7 * t * (T(1) + q * (T(4) + q * (T(6.25) + T(4) * q)));
        d = T(-5.5) * q * (T(1) + q * (T(3.5) + T(4) * q)) * t7;
    }
    template <class T> __device__ static T df(T q)
    {
        const T t = fmax(T(1) - T(0.5) * q, T(0)), t2 = t * t, t4 = t2 * t2;
        return T(-5.5) * q * (T(1) + q * (T(3.5) + T(4) * q)) * (t4 * t2 * t);
    }
};

// Reciprocal, reciprocal square root and square root for the derivative
// sums: the hardware instructions (about 1 ulp) in FP32, IEEE operations in
// FP64.  The neighbour decision never uses them.
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double fast_rcp(double x) { return 1.0 / x; }
__device__ inline double fast_rsq(double x) { return 1.0 / sqrt(x); }
__device__ inline double fast_sqrt(double x) { return sqrt(x); }

// Positive-float atomic min/max through the integer order of the bit pattern.
__device__ inline void atomic_min_posf(u32* addr, float v) { atomicMin(addr, __float_as_uint(v)); }
__device__ inline void atomic_max_posf(u32* addr, float v) { atomicMax(addr, __float_as_uint(v)); }

// Block-wide reductions (BLOCK threads); results valid in every thread.
template <int BLOCK, class T, class Op> __device__ inline T block_reduce(T v, T* lds, Op op)
{
    const int lane = __lane_id(), wid = threadIdx.x / WAVE;
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v = op(v, __shfl_xor(v, d, WAVE));
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    T r = lds[0];
#pragma unroll
    for (int w = 1; w < BLOCK / WAVE; ++w) r = op(r, lds[w]);
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Staging of a group's candidate union into LDS: slots [c0, c1) of the union
// (its leaves' particles in ascending key order) are copied from the
// key-order arrays.  BATCH = 0: one thread per union leaf copies the leaf's
// particles, one load after another.  BATCH > 0: one thread per union leaf
// writes, into the first word of each of its slots, the offset from slot to
// key-order index; then one thread per slot copies, with BATCH slots' loads
// in flight per thread (shorter latency, BATCH * NF more live registers).
// Slots past the last staged leaf (a union larger than the cache capacity)
// stay unwritten.  Every thread of the block must call it (BATCH > 0 holds a
// barrier).
// ---------------------------------------------------------------------------
template <class T, int NF, int NT = GROUP, int BATCH = 0>
__device__ inline void stage_union(const vec4<T>* const* src, vec4<T>* const* dst, const u32* id,
                                   const u32* ul, const u32* us, u32 nu, u32 c0, u32 c1)
{
    if (BATCH == 0) {
        for (u32 j = threadIdx.x; j < nu; j += NT) {
            const u32 s0 = us[j];
            const u32 leaf = ul[j];
            const u32 b0 = id[leaf], sz = id[leaf + 1] - b0;
            const u32 lo = s0 > c0 ? s0 : c0;
            const u32 hi = (s0 + sz) < c1 ? (s0 + sz) : c1;
            for (u32 s = lo; s < hi; ++s) {
#pragma unroll
                for (int f = 0; f < NF; ++f) dst[f][s - c0] = src[f][b0 + (s - s0)];
            }
        }
        return;
    }
    constexpr int B = BATCH > 0 ? BATCH : 1;
    u32 se = 0;                                  // end of the staged leaves' slots
    if (nu > 0) {
        const u32 lz = ul[nu - 1];
        se = us[nu - 1] + (id[lz + 1] - id[lz]);
    }
    for (u32 j = threadIdx.x; j < nu; j += NT) {
        const u32 s0 = us[j];
        const u32 leaf = ul[j];
        const u32 b0 = id[leaf], sz = id[leaf + 1] - b0;
        const u32 lo = s0 > c0 ? s0 : c0;
        const u32 hi = (s0 + sz) < c1 ? (s0 + sz) : c1;
        for (u32 s = lo; s < hi; ++s) *reinterpret_cast<int*>(&dst[0][s - c0]) = (int)(b0 - s0);
    }
    __syncthreads();
    const u32 ce = se < c1 ? se : c1;
    const u32 cnt = ce > c0 ? ce - c0 : 0u;
    for (u32 s0 = threadIdx.x; s0 < cnt; s0 += B * NT) {
        vec4<T> v[B][NF];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const u32 s = s0 + b * NT;
            if (s < cnt) {
                const i64 i = (i64)c0 + s + *reinterpret_cast<const int*>(&dst[0][s]);
#pragma unroll
                for (int f = 0; f < NF; ++f) v[b][f] = src[f][i];
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const u32 s = s0 + b * NT;
            if (s < cnt) {
#pragma unroll
                for (int f = 0; f < NF; ++f) dst[f][s] = v[b][f];
            }
        }
    }
}

}  // namespace shsph
