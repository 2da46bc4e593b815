// Two-stage neighbour cache (App. D.3-E.4, Alg. 4-6), laid out for gfx950.
//
// Particles are taken in groups of GROUP = 256 consecutive key-order slots
// (one workgroup).  Stage 1 runs once per group (Alg. 4 walked for all the
// group's leaves at once): one wave walks the tree level by level and keeps
// the leaves that pass the group-group criterion of App. E,
//     box_A  n  [box_C (+) R chi max(hmax_A, hmax_C)]  !=  0,
// for some target leaf A of the group, with periodic images and a slight
// outward inflation so that the prune is a superset of the exact particle
// test.  The kept leaves, in ascending order, form the group's candidate
// "union"; their particles are numbered by 16-bit slots (32-bit slots for a
// union of more than 65535 particles).
// Stage 2 runs one workgroup per group: each particle prefilters the union's
// leaves by box and tests their particles with the exact object-object
// criterion in the storage type, writing the accepted slots (ascending)
// into an ELL layout [group][entry][lane] so that reads and writes of the
// cache are coalesced across a wave.  The derivative kernels stage the union's
// particle data in LDS and resolve slots there.
#include "common.hpp"
#include "kernels.hpp"

namespace shsph {

constexpr int STACK = 64;   // tree depth is bounded by the 63 key bits
constexpr int TRAV_BLOCK = 64;
constexpr int LCHUNK = 256;  // union leaves staged in LDS at a time (stage 2)
constexpr int UCH = 1280;    // union particles staged in LDS (larger unions read HBM/L2)

template <class T> struct Inflate;
template <> struct Inflate<float> {
    static constexpr float rel = 2e-5f, abs = 1e-6f;
};
template <> struct Inflate<double> {
    static constexpr double rel = 1e-12, abs = 1e-14;
};

template <class T>
__device__ inline T gap1(T a0, T a1, T b0, T b1, T L, int periodic)
{
    T g = fmax(T(0), fmax(b0 - a1, a0 - b1));
    if (periodic) {
        const T g1 = fmax(T(0), fmax(b0 + L - a1, a0 - b1 - L));
        const T g2 = fmax(T(0), fmax(b0 - L - a1, a0 - b1 + L));
        g = fmin(g, fmin(g1, g2));
    }
    return g;
}

template <class T> __device__ inline T abs_inflation(const Box<T>& bx)
{
    T s = fmax(fmax(fabs(bx.lo[0]), fabs(bx.hi[0])), fmax(fabs(bx.lo[1]), fabs(bx.hi[1])));
    s = fmax(s, fmax(fabs(bx.lo[2]), fabs(bx.hi[2])));
    s = fmax(s, fmax(bx.L[0], fmax(bx.L[1], bx.L[2])));
    return Inflate<T>::abs * s;
}

// Box-box prune with the inflated radius; explicit roundings keep it
// identical wherever it is evaluated.  WRAP = false drops the periodic images
// (exact for boxes far enough from the faces, see prune_interior).
template <class T, bool WRAP = true>
__device__ inline bool box_hit(const vec4<T>& al, const vec4<T>& ah, const vec4<T>& bl,
                               const vec4<T>& bh, T rk, T eps_abs, const Box<T>& bx)
{
    const T r = rk * fmax(al.w, bl.w) * (T(1) + Inflate<T>::rel) + eps_abs;
    const int per = WRAP ? bx.periodic : 0;
    // all three axes evaluated (no short circuit): one branch-free test
    return (gap1<T>(al.x, ah.x, bl.x, bh.x, bx.L[0], per) <= r) &
           (gap1<T>(al.y, ah.y, bl.y, bh.y, bx.L[1], per) <= r) &
           (gap1<T>(al.z, ah.z, bl.z, bh.z, bx.L[2], per) <= r);
}

// A box at least r_all = rk h_max(all) 1.001 + 2 eps_abs + 1e-5 (Lx+Ly+Lz)
// inside every face: any periodic image of any box of the domain lies at a
// gap of at least r_all from it along the shifted axis, more than the prune
// radius of any pair, so per axis the image gaps never decide box_hit and it
// equals its version without images.
template <class T>
__device__ inline bool prune_interior(const vec4<T>& l, const vec4<T>& h, T hmax_all, T rk,
                                      T eps_abs, const Box<T>& bx)
{
    if (!bx.periodic) return true;
    const T r = rk * hmax_all * T(1.001) + T(2) * eps_abs + T(1e-5) * (bx.L[0] + bx.L[1] + bx.L[2]);
    return l.x - r > bx.lo[0] && l.y - r > bx.lo[1] && l.z - r > bx.lo[2] &&
           h.x + r < bx.hi[0] && h.y + r < bx.hi[1] && h.z + r < bx.hi[2];
}

// Tight box and h_max of each group: one wave per group (GB_WAVES groups
// per workgroup), each lane taking every 64th particle; min / max are exact,
// so the order of the reduction does not matter.
constexpr int GB_WAVES = 4;

template <class T>
__global__ void __launch_bounds__(GB_WAVES * WAVE)
k_group_boxes(const vec4<T>* __restrict__ posh, const GroupMap gm, i64 ngroups,
              vec4<T>* __restrict__ glo, vec4<T>* __restrict__ ghi, const u32* __restrict__ skip)
{
    if (skip && *skip) return;
    const i64 g = (i64)blockIdx.x * GB_WAVES + threadIdx.x / WAVE;
    if (g >= ngroups) return;                  // per wave; no workgroup barrier below
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    const int lane = __lane_id();
    T v[7];                                    // min of x, y, z, -x, -y, -z, -h
    {
        const vec4<T> p = posh[beg];
        v[0] = p.x; v[1] = p.y; v[2] = p.z; v[3] = -p.x; v[4] = -p.y; v[5] = -p.z; v[6] = -p.w;
    }
#pragma unroll
    for (int j = 0; j < GROUP / WAVE; ++j) {
        const i64 a = beg + lane + j * WAVE;
        if (a < end) {
            const vec4<T> p = posh[a];
            v[0] = fmin(v[0], p.x); v[1] = fmin(v[1], p.y); v[2] = fmin(v[2], p.z);
            v[3] = fmin(v[3], -p.x); v[4] = fmin(v[4], -p.y); v[5] = fmin(v[5], -p.z);
            v[6] = fmin(v[6], -p.w);
        }
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        T x = v[c];
        for (int d = WAVE / 2; d > 0; d >>= 1) x = fmin(x, __shfl_xor(x, d, WAVE));
        v[c] = x;
    }
    if (lane == 0) {
        glo[g] = mk4<T>(v[0], v[1], v[2], -v[6]);
        ghi[g] = mk4<T>(-v[3], -v[4], -v[5], T(0));
    }
}

// Stage 1: neighbour leaves of each group, ascending, with the slot where
// each leaf's particles start in the group's union.  Writes at most `cap`
// leaves per group; reports the largest count and union size.
// The union is first gathered with the group's box (one box test per node).
// A group whose union passes `spread` particles (256 consecutive Morton
// codes can straddle a jump of the curve and span a wide, sparse region)
// is traversed again keeping only nodes within reach of one of its target
// leaves -- the same leaf-pair prune stage 2 applies -- so its union holds
// exactly the leaves some particle of the group can reach.
constexpr u32 S1_SERIAL = 0xffffffffu;   // ucnt marker: group left to the serial walk

template <class T>
__global__ void __launch_bounds__(TRAV_BLOCK)
k_group_leaves_serial(bool only_marked, const vec4<T>* __restrict__ blo, const vec4<T>* __restrict__ bhi,
               const u32* __restrict__ child, const u32* __restrict__ id,
               const u32* __restrict__ xscan, i64 n_internal,
               const vec4<T>* __restrict__ glo, const vec4<T>* __restrict__ ghi, i64 ngroups,
               const GroupMap gm, const u32* __restrict__ root, const InstDev* __restrict__ inst,
               T rk, i64 cap, u32 spread, u32* __restrict__ uleaf, u32* __restrict__ uslot,
               u32* __restrict__ ucnt, u32* __restrict__ ustot, u32* __restrict__ flags,
               const u8* __restrict__ redo)
{
    __shared__ u32 stack[STACK][TRAV_BLOCK];
    const int lane = threadIdx.x;
    const i64 g0 = (i64)blockIdx.x * TRAV_BLOCK + lane;
    const i64 g = g0 < ngroups ? g0 : ngroups - 1;
    bool live0 = g0 < ngroups && (!only_marked || ucnt[g] == S1_SERIAL);
    if (only_marked && __ballot(live0) == 0) return;
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    if (redo && !redo[k]) live0 = false;      // this instance keeps its caches
    const bool live = live0;
    const Box<T> bx = make_box<T>(inst[k]);
    const T eps_abs = abs_inflation(bx);
    const vec4<T> ql = glo[g], qh = ghi[g];
    const u32 t0 = xscan[beg + 1] - 1u;          // target leaves t0 .. t0 + nt - 1
    const u32 nt = xscan[end] - t0;
    u32* ul = uleaf + g * cap;
    u32* us = uslot + g * cap;
    u32 count = 0, slots = 0;
    bool stack_over = false;
    for (int pass = 0; pass < 2; ++pass) {
        count = 0;
        slots = 0;
        bool wide = false;
        int sp = 0;
        if (live) stack[sp++][lane] = root[k];
        while (sp > 0) {
            const u32 node = stack[--sp][lane];
            const vec4<T> nl = blo[node], nh = bhi[node];
            if (!box_hit<T>(ql, qh, nl, nh, rk, eps_abs, bx)) continue;
            if (pass == 1) {
                bool near = false;
                for (u32 t = 0; t < nt && !near; ++t)
                    near = box_hit<T>(blo[n_internal + t0 + t], bhi[n_internal + t0 + t], nl, nh,
                                      rk, eps_abs, bx);
                if (!near) continue;
            }
            if (node >= n_internal) {
                const u32 leaf = (u32)(node - n_internal);
                if (count < cap) { ul[count] = leaf; us[count] = slots; }
                ++count;
                slots += id[leaf + 1] - id[leaf];
                if (pass == 0 && slots > spread) { wide = true; break; }
            } else {
                if (sp + 2 > STACK) { stack_over = true; break; }
                stack[sp++][lane] = child[2 * node + 1];
                stack[sp++][lane] = child[2 * node];
            }
        }
        if (!wide || stack_over) break;
    }
    if (live) {
        ucnt[g] = count;
        ustot[g] = slots;
    }
    u32 f = stack_over ? 1u : 0u;
    if (count > cap) f |= 2u;
    if (f) atomicOr(&flags[0], f);
    // largest leaf count (for the capacity of the next build)
    const u32 wmax = wave_max(count);
    if (__lane_id() == 0 && wmax > __hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&flags[1], wmax);
}

// Stage 1, one wave per group.  A stack in LDS holds the pending nodes in
// left-to-right order (the top is the leftmost) and each iteration the 64
// lanes take the 64 leftmost.  A node is kept when it passes the group's box
// and, more tightly, the box of at least one of the group's target leaves;
// each entry carries the set of targets that reached its parent, so a node
// is tested only against those (as a mask over S1_TS runs of consecutive
// targets: a run's bit stays set while any of its targets reaches the node;
// every target is still tested on its own, so the prune is exact).  A kept leaf is written out at once when no
// kept internal node lies to its left in the batch, otherwise it goes back on
// the stack marked final; kept internal nodes go back as their two children.
// Everything pushed back keeps the order, so the union comes out ascending
// with its slot starts (a running wave scan of the leaf sizes).  The union is
// the set of leaves within reach of some target leaf: the same leaf-pair
// prune stage 2 applies.  A compact group (box at most four cache radii of
// its smallest target wide, h within 1.5x, the common case) uses the
// group's box alone, which is then nearly as tight.
// A group whose stack outgrows the LDS buffer is marked and left to the
// serial walk.
// The walk is compiled twice: FULL = false keeps only the node stack in LDS
// (4 KB per wave, so many more waves hide the tree's load latency) and takes
// the compact groups, marking the others; FULL = true, with the per-entry
// target masks and the target boxes, then takes the marked groups.  1024
// stack entries: at 1536 the LDS allowed the compact walk six waves per
// SIMD instead of eight, and the Sedov and batched workloads ran slower (a
// group that outgrows the stack takes the serial walk).
constexpr int S1_WAVES = 1;             // waves per workgroup, full walk
constexpr int S1_CWAVES = 4;            // waves per workgroup, compact walk
constexpr int S1_SMAX = 1024;
constexpr u32 S1_WIDE = 0xfffffffeu;    // ucnt marker: group left to the full walk
constexpr int S1_TS = 32;               // target runs (mask bits)
constexpr u32 S1_FINAL = 0x80000000u;      // stack entry: an accepted leaf

// Orders one wave's LDS accesses across its lanes.  A wave's LDS
// instructions are performed in issue order, so only the compiler must keep
// them in place: a wavefront-scope fence (no wait on the wave's outstanding
// global stores) and a wave barrier.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <class T, bool FULL>
__global__ void __launch_bounds__((FULL ? S1_WAVES : S1_CWAVES) * WAVE)
k_group_leaves_wave(const vec4<T>* __restrict__ blo, const vec4<T>* __restrict__ bhi,
                    const u32* __restrict__ child, const u32* __restrict__ id,
                    const u32* __restrict__ xscan, i64 n_internal,
                    const vec4<T>* __restrict__ glo, const vec4<T>* __restrict__ ghi, i64 ngroups,
                    const GroupMap gm, const u32* __restrict__ root,
                    const InstDev* __restrict__ inst, T rk, i64 cap, u32* __restrict__ uleaf,
                    u32* __restrict__ uslot, u32* __restrict__ ucnt, u32* __restrict__ ustot,
                    u32* __restrict__ flags, const u8* __restrict__ redo)
{
    constexpr int NW = FULL ? S1_WAVES : S1_CWAVES;
    __shared__ u32 s_sn[NW][S1_SMAX];
    __shared__ u32 s_sm[FULL ? NW : 1][FULL ? S1_SMAX : 1];
    __shared__ vec4<T> s_tl[FULL ? NW : 1][FULL ? GROUP : 1];   // target leaf boxes
    __shared__ vec4<T> s_th[FULL ? NW : 1][FULL ? GROUP : 1];   // (at most one per particle)
    const int w = threadIdx.x / WAVE;
    const u32 lane = (u32)__lane_id();
    const i64 g = (i64)blockIdx.x * NW + w;
    if (g >= ngroups) return;                 // per wave; no workgroup barrier below
    if (FULL && ucnt[g] != S1_WIDE) return;   // the compact walk took this group
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    if (redo && !redo[k]) return;             // this instance keeps its caches
    const Box<T> bx = make_box<T>(inst[k]);
    const T eps_abs = abs_inflation(bx);
    const vec4<T> ql = glo[g], qh = ghi[g];
    const u32 t0 = xscan[beg + 1] - 1u;       // target leaves t0 .. t0 + nt - 1
    const u32 nt = xscan[end] - t0;
    const u32 ns = nt < (u32)S1_TS ? nt : (u32)S1_TS;     // runs; run r = targets
    const u32 rl = (nt + ns - 1u) / ns;                     // [r rl, min(nt, r rl + rl))
    T hmin = ql.w;                            // smallest target h_max
    for (u32 a = lane; a < nt; a += WAVE) {
        const vec4<T> tl = blo[n_internal + t0 + a];
        if (FULL) {
            s_tl[w][a] = tl;
            s_th[w][a] = bhi[n_internal + t0 + a];
        }
        hmin = fmin(hmin, tl.w);
    }
    hmin = wave_min(hmin);
    // a compact group (box no wider than a few cache radii of its smallest
    // target, h nearly uniform) keeps the plain group-box test: per-target
    // tests would prune little and cost up to nt box tests per node
    const T reach = rk * hmin;
    const bool compact = ql.w <= T(1.5) * hmin && (qh.x - ql.x) <= T(4) * reach &&
                         (qh.y - ql.y) <= T(4) * reach && (qh.z - ql.z) <= T(4) * reach;
    if (!FULL && !compact) {
        if (lane == 0) ucnt[g] = S1_WIDE;
        return;
    }
    if (lane == 0) {
        s_sn[w][0] = root[k];
        if (FULL) s_sm[w][0] = ns == 32u ? 0xffffffffu : ((1u << ns) - 1u);
    }
    wave_lds_sync();
    u32* ul = uleaf + g * cap;
    u32* us = uslot + g * cap;
    u32 sp = 1, count = 0, slots = 0;
    bool over = false;
    while (sp > 0) {
        const u32 take_n = sp < (u32)WAVE ? sp : (u32)WAVE;
        const u32 base = sp - take_n;
        u32 e = 0, m = 0;
        if (lane < take_n) {                  // lane 0 takes the top (leftmost)
            e = s_sn[w][sp - 1u - lane];
            m = FULL ? s_sm[w][sp - 1u - lane] : 1u;
        }
        wave_lds_sync();                       // popped before anything is pushed over them
        const u32 v = e & ~S1_FINAL;
        // one round of loads per iteration: the node's box and its pair of
        // pointers (children of an internal node, particle range of a leaf)
        const bool act = lane < take_n, fin = (e & S1_FINAL) != 0u;
        const bool is_leaf = v >= (u32)n_internal;
        u32 p0 = 0, p1 = 0;
        vec4<T> nl{}, nh{};
        if (act) {
            const u32* pp = is_leaf ? id + (v - (u32)n_internal) : child + 2 * (u64)v;
            p0 = pp[0];
            p1 = pp[1];
            if (!fin) {
                nl = blo[v];
                nh = bhi[v];
            }
        }
        bool keep = false, leaf = false;
        u32 cm = 0;
        if (act) {
            if (fin) {
                keep = true;
                leaf = true;
            } else {
                if (box_hit<T>(ql, qh, nl, nh, rk, eps_abs, bx)) {
                    if (!FULL || compact) cm = m;
                    else while (m) {
                        const u32 r = (u32)(__ffs(m) - 1);
                        m &= m - 1u;
                        const u32 a1 = min(nt, r * rl + rl);
                        for (u32 a = r * rl; a < a1; ++a)
                            if (box_hit<T>(s_tl[w][a], s_th[w][a], nl, nh, rk, eps_abs, bx)) {
                                cm |= 1u << r;
                                break;
                            }
                    }
                    keep = cm != 0u;
                    leaf = is_leaf;
                }
            }
        }
        // leaves left of the first kept internal node are final in order
        const u64 bint = __ballot(keep && !leaf);
        const u32 first_int = bint ? (u32)(__ffsll((unsigned long long)bint) - 1) : (u32)WAVE;
        const bool emit = keep && leaf && lane < first_int;
        const bool defer = keep && leaf && lane > first_int;
        const u32 nres = (keep && !leaf) ? 2u : (defer ? 1u : 0u);
        // nres is 0, 1 or 2: its prefix sum is two masked population counts
        const u64 b1 = __ballot(nres >= 1u), b2 = __ballot(nres == 2u);
        const u32 rincl = (u32)__popcll(b1 & lanemask_lt()) + (u32)__popcll(b2 & lanemask_lt()) + nres;
        const u32 rtot = (u32)__popcll(b1) + (u32)__popcll(b2);
        if (base + rtot > (u32)S1_SMAX) { over = true; break; }
        // emitted leaves: ascending, with their slot starts
        const u64 bem = __ballot(emit);
        const u32 sz = emit ? p1 - p0 : 0u;
        const u32 sincl = wave_incl_scan_dpp(sz);
        if (emit) {
            const u32 q = count + (u32)__popcll(bem & lanemask_lt());
            if ((i64)q < cap) {
                ul[q] = v - (u32)n_internal;
                us[q] = slots + sincl - sz;
            }
        }
        count += (u32)__popcll(bem);
        slots += (u32)__builtin_amdgcn_readlane((int)sincl, WAVE - 1);
        // push back: result r (0 = leftmost) goes to base + rtot - 1 - r
        const u32 r0 = rincl - nres;
        if (keep && !leaf) {
            s_sn[w][base + rtot - 1u - r0] = p0;
            s_sn[w][base + rtot - 2u - r0] = p1;
            if (FULL) {
                s_sm[w][base + rtot - 1u - r0] = cm;
                s_sm[w][base + rtot - 2u - r0] = cm;
            }
        } else if (defer) {
            s_sn[w][base + rtot - 1u - r0] = v | S1_FINAL;
            if (FULL) s_sm[w][base + rtot - 1u - r0] = 0u;
        }
        sp = base + rtot;
        wave_lds_sync();
    }
    if (over) {
        if (lane == 0) {
            ucnt[g] = S1_SERIAL;
            ustot[g] = 0;
        }
        return;
    }
    if (lane == 0) {
        ucnt[g] = count;
        ustot[g] = slots;
        u32 f = 0;
        if ((i64)count > cap) f |= 2u;
        if (f) atomicOr(&flags[0], f);
        if (count > __hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&flags[1], count);
    }
}

// Stage 2: per particle, its neighbours among the group's union (Alg. 5 with
// the object-object criterion), as ascending 16-bit slots, four per 64-bit
// word in ELL layout (see slot_of); ncnt[a] = number of neighbours.
// The workgroup first marks, for every leaf holding particles of the group
// ("target leaf"), the union leaves that pass the group-group prune against
// it (bitmasks in LDS, built cooperatively); each lane then walks only the
// particles of its own leaf's marked union leaves, positions read from LDS.
constexpr int TMAX = GROUP;      // target leaves of a group: at most one per particle
constexpr int MW = LCHUNK / 64;  // mask words per target leaf
static_assert(MW == 4, "the per-lane walk selects among four mask words");

// Stage-2 candidate test in the storage type:
//   dx = x_b - x_a (minimum image), r2 = fma(dz, dz, fma(dy, dy, dx*dx)),
//   accept iff r2 < max(qa, qb), q = (rkc h)^2 rounded as (rkc h)(rkc h);
//   rounding is monotone, so max(qa, qb) equals (rkc max(h_a, h_b))^2 exactly.
// Squared radii staged in LDS (and qa) have a NaN replaced by +0: that
// changes no decision (max(q, +0) = max(q, NaN) = q for q >= 0, and both
// reject everything when the other operand is NaN too), and lets the FP32
// test compare bit patterns: for r2 >= +0 or NaN and q in [+0, inf] the
// unsigned order of the bits is the float order, a NaN r2 is rejected.
template <class T> __device__ inline T q_clean(T q) { return q == q ? q : T(0); }

template <class T, bool LDS>
__device__ inline T cand_q(const vec4<T>& pb, T rkc)
{
#pragma clang fp contract(off)
    if (LDS) return pb.w;                         // staged as (rkc h_b)^2
    const T r = rkc * pb.w;
    return r * r;
}

template <class T, bool LDS, bool WRAP>
__device__ inline bool cache_acc(const vec4<T>& pa, T qa, const Box<T>& bx, const vec4<T>& pb,
                                 T rkc)
{
#pragma clang fp contract(off)
    const int per = WRAP ? bx.periodic : 0;
    const T dx = min_image(pb.x - pa.x, bx.L[0], bx.halfL[0], per);
    const T dy = min_image(pb.y - pa.y, bx.L[1], bx.halfL[1], per);
    const T dz = min_image(pb.z - pa.z, bx.L[2], bx.halfL[2], per);
    const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if constexpr (LDS && sizeof(T) == 4) {
        const u32 qa_b = __float_as_uint(qa), qb_b = __float_as_uint(pb.w);
        return __float_as_uint(r2) < (qa_b > qb_b ? qa_b : qb_b);
    } else {
        return r2 < fmax(qa, cand_q<T, LDS>(pb, rkc));
    }
}

// Accepted slots are queued per lane in LDS: each lane owns QLEN 16-bit
// entries; every tested slot is written at the queue's fill position and the
// position advances by the accept flag, so the packing costs no branch and no
// variable shift per candidate.  After every group of up to four candidates
// a completed ELL word (the first four entries) is copied to the cache and
// the rest moves to the front; groups of eight candidates complete up to two
// words.  At most 3 entries are pending before a group and 11 after it.
// A lane's queue starts 28 bytes after the previous lane's: an odd number of
// 4-byte LDS banks, so the lanes' writes at equal fill positions fall in
// distinct banks.  The queues are then only 4-byte aligned, and their words
// are moved as two 32-bit halves.
constexpr u32 QLEN = 12;
constexpr u32 QSTRIDE = 14;   // u16 per lane (28 B)

__device__ inline u64 q_ld(const u16* p)
{
    const u32* q = (const u32*)p;
    return (u64)q[0] | ((u64)q[1] << 32);
}
__device__ inline void q_st(u16* p, u64 v)
{
    u32* q = (u32*)p;
    q[0] = (u32)v;
    q[1] = (u32)(v >> 32);
}

struct LaneQueue {
    u16* e;       // this lane's entries in LDS
    u32 pos;      // pending entries
    u32 q;        // ELL words completed so far
    u64* out;     // where word q goes
};

__device__ inline void queue_put(LaneQueue& lq, u32 s, bool acc)
{
    lq.e[lq.pos] = (u16)s;
    lq.pos += acc ? 1u : 0u;
}

__device__ inline void queue_flush(LaneQueue& lq, u32 capq)
{
    if (lq.pos >= 4u) {
        const u64 w = q_ld(lq.e);
        if (lq.q < capq) *lq.out = w;
        lq.out += GROUP;
        ++lq.q;
        q_st(lq.e, q_ld(lq.e + 4));
        lq.pos -= 4u;
    }
}

// After a group of eight candidates: up to two completed words.
__device__ inline void queue_flush2(LaneQueue& lq, u32 capq)
{
    if (lq.pos >= 4u) {
        if (lq.q < capq) *lq.out = q_ld(lq.e);
        lq.out += GROUP;
        ++lq.q;
        q_st(lq.e, q_ld(lq.e + 4));
        q_st(lq.e + 4, q_ld(lq.e + 8));
        lq.pos -= 4u;
        queue_flush(lq, capq);
    }
}

// The queue of a group with 32-bit slots (a union of more than 65535
// particles, rare: a few groups that span a sparse region next to a dense
// one): two entries per word, the pending one held in a register.
struct WideQueue {
    u32 pend;     // an accepted slot waiting for the second half of its word
    u32 n;        // 1 if pend holds one
    u32 q;        // ELL words completed so far
    u32 capq;
    u64* out;     // where word q goes
};

__device__ inline void queue_append(WideQueue& wq, u32 s, u32 capq)
{
    if (wq.n) {
        if (wq.q < capq) *wq.out = (u64)wq.pend | ((u64)s << 32);
        wq.out += GROUP;
        ++wq.q;
        wq.n = 0u;
    } else {
        wq.pend = s;
        wq.n = 1u;
    }
}
__device__ inline void queue_put(WideQueue& wq, u32 s, bool acc)
{
    if (acc) queue_append(wq, s, wq.capq);
}
__device__ inline void queue_flush(WideQueue&, u32) {}
__device__ inline void queue_flush2(WideQueue&, u32) {}

// Per-particle leaf test (groups that need no minimum image): the gaps from
// the particle to the leaf's tight box, g = max(lo - x_a, x_a - hi, 0) per
// axis, give d2 = fma(gz, gz, fma(gy, gy, gx gx)).  For any particle b of the
// leaf, |x_b - x_a| >= g and the roundings are monotone, so its r2 >= d2;
// and its staged q_b <= q_leaf = (rkc h_max)^2 rounded the same way.  So
// d2 >= max(q_a, q_leaf) rejects every particle of the leaf exactly, and
// only leaves that pass are walked.  q_leaf is staged in the box's .w.
template <class T>
__device__ inline bool leaf_reach(const vec4<T>& pa, T qa, const vec4<T>& bl, const vec4<T>& bh)
{
#pragma clang fp contract(off)
    const T gx = fmax(fmax(bl.x - pa.x, pa.x - bh.x), T(0));
    const T gy = fmax(fmax(bl.y - pa.y, pa.y - bh.y), T(0));
    const T gz = fmax(fmax(bl.z - pa.z, pa.z - bh.z), T(0));
    const T d2 = fma(gz, gz, fma(gy, gy, gx * gx));
    if constexpr (sizeof(T) == 4) {
        const u32 qa_b = __float_as_uint(qa), ql_b = __float_as_uint(bh.w);
        return __float_as_uint(d2) < (qa_b > ql_b ? qa_b : ql_b);
    } else {
        return d2 < fmax(qa, bh.w);
    }
}

// Tests the particles [b0, b1) of one union leaf (union slots from sl) and
// queues the accepted ones (the per-lane walk).
template <class T, bool LDS, bool WRAP, class Q>
__device__ inline void cache_leaf(const vec4<T>& pa, T qa, const Box<T>& bx, T rkc,
                                  u32 b0, u32 b1, u32 sl, const vec4<T>* s_upos,
                                  const vec4<T>* posh, Q& lq, u32 capq)
{
    u32 b = b0;
    for (; b + 8 <= b1; b += 8) {         // eight candidate loads in flight
        const u32 s = sl + (b - b0);
        vec4<T> p[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k] = LDS ? s_upos[s + k] : posh[b + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) queue_put(lq, s + k, cache_acc<T, LDS, WRAP>(pa, qa, bx, p[k], rkc));
        queue_flush2(lq, capq);
    }
    for (; b + 4 <= b1; b += 4) {
        const u32 s = sl + (b - b0);
        const vec4<T> p0 = LDS ? s_upos[s] : posh[b];
        const vec4<T> p1 = LDS ? s_upos[s + 1] : posh[b + 1];
        const vec4<T> p2 = LDS ? s_upos[s + 2] : posh[b + 2];
        const vec4<T> p3 = LDS ? s_upos[s + 3] : posh[b + 3];
        queue_put(lq, s, cache_acc<T, LDS, WRAP>(pa, qa, bx, p0, rkc));
        queue_put(lq, s + 1, cache_acc<T, LDS, WRAP>(pa, qa, bx, p1, rkc));
        queue_put(lq, s + 2, cache_acc<T, LDS, WRAP>(pa, qa, bx, p2, rkc));
        queue_put(lq, s + 3, cache_acc<T, LDS, WRAP>(pa, qa, bx, p3, rkc));
        queue_flush(lq, capq);
    }
    for (; b < b1; ++b) {
        const u32 s = sl + (b - b0);
        const vec4<T> p = LDS ? s_upos[s] : posh[b];
        queue_put(lq, s, cache_acc<T, LDS, WRAP>(pa, qa, bx, p, rkc));
        queue_flush(lq, capq);
    }
}

// Stage-2 walk, per lane: each lane takes the union leaves of its target
// leaf's mask, one leaf per iteration across all the mask's words, so lanes
// whose marked leaves fall in different words still visit in step.  For
// groups that need no minimum image, when some lane of the wave has many
// candidates (marked leaves x the union's mean leaf size >= 300: then the
// rejected leaves save more tests than the pass costs), a first pass clears
// the leaves that fail the particle's own leaf test (leaf_reach) from the
// lane's copy of the mask, so the walk's iterations follow the leaves the
// lane really visits (a skip inside the walk would cost the wave the test
// and the visit).
template <class T, bool LDS, bool WRAP, class Q>
__device__ inline void cache_walk_lane(const vec4<T>& pa, T qa, bool live, u32 S, u32 nu,
                                       const Box<T>& bx,
                                       T rkc, const u64* mrow, const u32* s_b0, const u32* s_b1,
                                       const u32* s_slot, const u32* ulc, const vec4<T>* lblo,
                                       const vec4<T>* lbhi, const vec4<T>* s_upos,
                                       const vec4<T>* posh, Q& lq, u32 capq, u32& tested)
{
    bool refine = false;
    if (!WRAP) {
        u32 marked = 0;
        if (live)
#pragma unroll
            for (int w = 0; w < MW; ++w) marked += (u32)__popcll(mrow[w]);
        refine = __ballot((u64)marked * S >= 300ull * nu) != 0ull;
    }
    if (!live) return;
    u64 mk[MW];
#pragma unroll
    for (int w = 0; w < MW; ++w) {
        u64 m = mrow[w];
        if (!WRAP && refine) {
            u64 cur = m;
            while (cur) {
                const u32 b = (u32)(__ffsll((unsigned long long)cur) - 1);
                cur &= cur - 1;
                const u32 j = (u32)(w * 64) + b;
                const u32 leaf = ulc[j];
                const vec4<T> bl = lblo[leaf];
                vec4<T> bh = lbhi[leaf];
                {
#pragma clang fp contract(off)
                    const T r = rkc * bl.w;
                    bh.w = q_clean(r * r);
                }
                if (!leaf_reach<T>(pa, qa, bl, bh)) m &= ~(1ull << b);
            }
        }
        mk[w] = m;
    }
    u32 wb = 0;                 // 64 x (current word)
    u64 cur = mk[0];
    for (;;) {
        while (cur == 0ull && wb < (u32)(MW - 1) * 64u) {
            wb += 64u;
            cur = wb == 64u ? mk[1] : (wb == 128u ? mk[2] : mk[3]);
        }
        if (cur == 0ull) break;
        const u32 j = wb + (u32)(__ffsll((unsigned long long)cur) - 1);
        cur &= cur - 1;
        const u32 b0 = s_b0[j], b1 = s_b1[j];
        tested += b1 - b0;
        cache_leaf<T, LDS, WRAP, Q>(pa, qa, bx, rkc, b0, b1, s_slot[j], s_upos, posh, lq, capq);
    }
}

// Appends one accepted slot (the per-wave walk's accept path, taken only for
// accepted candidates): at most 3 entries are pending between calls.
__device__ inline void queue_append(LaneQueue& lq, u32 s, u32 capq)
{
    lq.e[lq.pos] = (u16)s;
    if (++lq.pos == 4u) {
        const u64 w = q_ld(lq.e);
        if (lq.q < capq) *lq.out = w;
        lq.out += GROUP;
        ++lq.q;
        lq.pos = 0u;
    }
}

// Stage-2 walk, per wave: the wave takes the union leaves marked for any of
// its lanes (the OR of their masks), in ascending order, and every lane tests
// every particle of them: the criterion is exact, so a lane never accepts a
// particle its own mask would have skipped, and its slots stay ascending.
// Uniform control and broadcast LDS reads; worth it when the lanes' candidate
// sets overlap (the wave's union is not much larger than one lane's).  Most
// of a lane's tests here are rejections, so a leaf's tests set bits of a
// 32-candidate mask first and only the accepted slots are queued.
template <class T, bool LDS, bool WRAP>
__device__ inline void cache_walk_wave(const vec4<T>& pa, T qa, bool live, const Box<T>& bx, T rkc,
                                       const u64* wmask, const u32* s_b0, const u32* s_b1,
                                       const u32* s_slot, const vec4<T>* s_upos,
                                       const vec4<T>* posh, LaneQueue& lq, u32 capq, u32& tested)
{
#pragma unroll
    for (int w = 0; w < MW; ++w) {
        u64 cur = wmask[w];
        while (cur) {
            const u32 j = (u32)(w * 64) + (u32)(__ffsll((unsigned long long)cur) - 1);
            cur &= cur - 1;
            const u32 b0 = __builtin_amdgcn_readfirstlane(s_b0[j]);
            const u32 b1 = __builtin_amdgcn_readfirstlane(s_b1[j]);
            const u32 sl = __builtin_amdgcn_readfirstlane(s_slot[j]);
            if (live) tested += b1 - b0;
            for (u32 bc = b0; bc < b1; bc += 32u) {
                const u32 e = min(b1, bc + 32u);
                const u32 s0 = sl + (bc - b0);
                u32 bits = 0, k = 0;
                u32 b = bc;
                for (; b + 4 <= e; b += 4, k += 4) {
                    const u32 s = s0 + k;
                    const vec4<T> p0 = LDS ? s_upos[s] : posh[b];
                    const vec4<T> p1 = LDS ? s_upos[s + 1] : posh[b + 1];
                    const vec4<T> p2 = LDS ? s_upos[s + 2] : posh[b + 2];
                    const vec4<T> p3 = LDS ? s_upos[s + 3] : posh[b + 3];
                    bits |= (cache_acc<T, LDS, WRAP>(pa, qa, bx, p0, rkc) ? 1u : 0u) << k;
                    bits |= (cache_acc<T, LDS, WRAP>(pa, qa, bx, p1, rkc) ? 2u : 0u) << k;
                    bits |= (cache_acc<T, LDS, WRAP>(pa, qa, bx, p2, rkc) ? 4u : 0u) << k;
                    bits |= (cache_acc<T, LDS, WRAP>(pa, qa, bx, p3, rkc) ? 8u : 0u) << k;
                }
                for (; b < e; ++b, ++k) {
                    const vec4<T> p = LDS ? s_upos[s0 + k] : posh[b];
                    bits |= (cache_acc<T, LDS, WRAP>(pa, qa, bx, p, rkc) ? 1u : 0u) << k;
                }
                if (!live) bits = 0;
                while (bits) {
                    const u32 t = (u32)(__ffs(bits) - 1);
                    bits &= bits - 1u;
                    queue_append(lq, s0 + t, capq);
                }
            }
        }
    }
}

__device__ inline u64 wave_or64(u64 x)
{
    u32 lo = (u32)x, hi = (u32)(x >> 32);
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        lo |= __shfl_xor(lo, d, WAVE);
        hi |= __shfl_xor(hi, d, WAVE);
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    return ((u64)hi << 32) | lo;
}

template <class T, int MODE>
__global__ void __launch_bounds__(GROUP)
k_group_cache(const vec4<T>* __restrict__ posh, const vec4<T>* __restrict__ blo,
              const vec4<T>* __restrict__ bhi, const u32* __restrict__ id,
              const u32* __restrict__ xscan, i64 n_internal, const GroupMap gm,
              const InstDev* __restrict__ inst, T rk, T rkc, i64 cap,
              const u32* __restrict__ uleaf, const u32* __restrict__ uslot,
              const u32* __restrict__ ucnt, const u32* __restrict__ ustot,
              const u64* __restrict__ gbase, const u32* __restrict__ gcap, u64 words_alloc,
              u32* __restrict__ gneed, const u8* __restrict__ gredo,
              u64* __restrict__ nlist, u32* __restrict__ ncnt, u32* __restrict__ flags,
              const vec4<T>* __restrict__ glo, const vec4<T>* __restrict__ ghi,
              const u32* __restrict__ root, u64* __restrict__ work, const u8* __restrict__ redo)
{
    constexpr int mode = MODE;
    __shared__ u64 s_w[GROUP / WAVE];
    __shared__ u32 s_b0[LCHUNK];
    __shared__ u32 s_b1[LCHUNK];
    __shared__ u32 s_slot[LCHUNK];
    // union-leaf boxes of the chunk (.w of the high corner: q of the leaf's
    // h_max), for the prune and the per-particle leaf test
    // target-leaf boxes (prune only, loaded per chunk); the walk reuses the
    // space for the lanes' queues (pending entries carried over chunks in a
    // register)
    __shared__ vec4<T> s_tbox[2 * TMAX];
    vec4<T>* const s_tlo = s_tbox;
    vec4<T>* const s_thi = s_tbox + TMAX;
    static_assert(GROUP * QSTRIDE * sizeof(u16) <= sizeof(s_tbox), "queues do not fit");
    __shared__ u64 s_mask[TMAX][MW];
    __shared__ vec4<T> s_upos[UCH];
    const i64 g = blockIdx.x;
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    if (redo && !redo[k]) return;             // this instance keeps its caches (block-uniform)
    if (gredo && !gredo[g]) return;           // this group's cache fitted (regrow retry)
    if (gbase[gm.ngroups_total()] > words_alloc) {   // the planned layout does not fit
        if (threadIdx.x == 0) atomicOr(&flags[0], 32u);
        return;
    }
    const u32 capq = gcap[g];
    const Box<T> bx = make_box<T>(inst[k]);
    const T eps_abs = abs_inflation(bx);
    const i64 a = beg + threadIdx.x;
    const bool live = a < end;
    const i64 ai = live ? a : beg;
    const vec4<T> pa = posh[ai];
    const u32 nu = min((u32)cap, ucnt[g]);
    const u32 S = ustot[g];
    const bool in_lds = S <= (u32)UCH;
    const bool interior = group_interior<T>(glo[g], ghi[g], blo[root[k]].w, rk, bx);
    static_assert(LCHUNK == GROUP && MW == GROUP / WAVE, "prune: one mask word per wave");
    // target leaves: the leaves holding slots beg .. end-1
    const u32 t0 = xscan[beg + 1] - 1u;
    const u32 nt = xscan[end] - t0;              // <= GROUP
    const u32 ta = xscan[ai + 1] - 1u - t0;
    const T hmax_all = blo[root[k]].w;
    bool t_in = true;
    for (u32 t = threadIdx.x; t < nt; t += GROUP)
        t_in = t_in && prune_interior<T>(blo[n_internal + t0 + t], bhi[n_internal + t0 + t], hmax_all,
                                         rk, eps_abs, bx);
    const bool prune_wrap = __syncthreads_or(!t_in);
    if (in_lds) {
        const vec4<T>* src[1] = { posh };
        vec4<T>* dst[1] = { s_upos };
        stage_union<T, 1>(src, dst, id, uleaf + g * cap, uslot + g * cap, nu, 0u, S);
        __syncthreads();
        for (u32 t = threadIdx.x; t < S; t += GROUP) {   // h -> (rkc h)^2
#pragma clang fp contract(off)
            const T r = rkc * s_upos[t].w;
            s_upos[t].w = q_clean(r * r);
        }
    }
    T qa;
    {
#pragma clang fp contract(off)
        const T r = rkc * pa.w;
        qa = q_clean(r * r);
    }
    u64* out = nlist + gbase[g] * GROUP + threadIdx.x;
    u32 tested = 0;
    u64 wbuf = 0, boxtests = 0;   // wbuf: the queue's pending entries between chunks
    LaneQueue lq{(u16*)s_tbox + threadIdx.x * QSTRIDE, 0u, 0u, out};
    const bool w32 = slots_wide(S);    // block-uniform; then in_lds is false
    WideQueue wq{0u, 0u, 0u, capq, out};
    for (u32 c0 = 0; c0 < nu; c0 += LCHUNK) {
        const u32 c1 = min(nu, c0 + LCHUNK);
        const u32 nl = c1 - c0;
        boxtests += (u64)nt * nl;
        __syncthreads();
        vec4<T> ul{}, uh{};      // this thread's union leaf of the chunk (prune)
        for (u32 j = c0 + threadIdx.x; j < c1; j += GROUP) {
            const u32 leaf = uleaf[g * cap + j];
            s_b0[j - c0] = id[leaf];
            s_b1[j - c0] = id[leaf + 1];
            s_slot[j - c0] = uslot[g * cap + j];
            ul = blo[n_internal + leaf];
            uh = bhi[n_internal + leaf];
        }
        for (u32 t = threadIdx.x; t < nt; t += GROUP) {
            s_tlo[t] = blo[n_internal + t0 + t];
            s_thi[t] = bhi[n_internal + t0 + t];
        }
        __syncthreads();
        // target leaf x union leaf prune, shared by the lanes of each target
        // leaf: wave w owns mask word w (union leaves 64w .. 64w+63 of the
        // chunk, one per lane) and sweeps the target leaves
        {
            const u32 wv = threadIdx.x / WAVE, j = threadIdx.x;
            if (wv * WAVE >= nl) {
                for (u32 t = __lane_id(); t < nt; t += WAVE) s_mask[t][wv] = 0ull;
            } else {
                const bool jv = j < nl;
                const vec4<T> bl = ul, bh = uh;
                for (u32 t = 0; t < nt; ++t) {
                    const bool hit = jv && (prune_wrap ? box_hit<T, true>(s_tlo[t], s_thi[t], bl, bh, rk, eps_abs, bx)
                                                       : box_hit<T, false>(s_tlo[t], s_thi[t], bl, bh, rk, eps_abs, bx));
                    const u64 word = __ballot(hit);
                    if (__lane_id() == 0) s_mask[t][wv] = word;
                }
            }
        }
        __syncthreads();
        u64 mk[MW], wm[MW];
#pragma unroll
        for (int w = 0; w < MW; ++w) {
            mk[w] = live && mode != 1 ? s_mask[ta][w] : 0ull;
            wm[w] = mode != 1 ? wave_or64(mk[w]) : 0ull;
        }
        // walk per wave or per lane: the wave issues about (leaves of the
        // wave's mask) uniform leaf visits or (leaves of the busiest lane's
        // mask) divergent ones; weighted 1 : 1.4 this picks the faster walk
        // on lattices (per lane) and on clustered instances (per wave)
        bool uniform = mode == 2;
        if constexpr (mode == 0) {
            u32 mine = 0, all = 0;
#pragma unroll
            for (int w = 0; w < MW; ++w) {
                mine += (u32)__popcll(mk[w]);
                all += (u32)__popcll(wm[w]);
            }
            uniform = 10u * all < 14u * wave_max(mine);
        }
        if (lq.pos) q_st(lq.e, wbuf);   // pending entries
        if (w32) {
            // exact for interior groups too: no image is closer there
            cache_walk_lane<T, false, true>(pa, qa, live, S, nu, bx, rkc, s_mask[ta], s_b0, s_b1,
                                            s_slot, uleaf + g * cap + c0, blo + n_internal, bhi + n_internal, s_upos, posh, wq, capq, tested);
        } else if (mode != 1 && uniform) {
            if (in_lds && interior)
                cache_walk_wave<T, true, false>(pa, qa, live, bx, rkc, wm, s_b0, s_b1, s_slot,
                                                s_upos, posh, lq, capq, tested);
            else if (in_lds)
                cache_walk_wave<T, true, true>(pa, qa, live, bx, rkc, wm, s_b0, s_b1, s_slot,
                                               s_upos, posh, lq, capq, tested);
            else
                cache_walk_wave<T, false, true>(pa, qa, live, bx, rkc, wm, s_b0, s_b1, s_slot,
                                                s_upos, posh, lq, capq, tested);
        } else if (mode != 2) {
            if (in_lds && interior)
                cache_walk_lane<T, true, false>(pa, qa, live, S, nu, bx, rkc, s_mask[ta], s_b0, s_b1,
                                                s_slot, uleaf + g * cap + c0, blo + n_internal, bhi + n_internal, s_upos, posh, lq, capq, tested);
            else if (in_lds)
                cache_walk_lane<T, true, true>(pa, qa, live, S, nu, bx, rkc, s_mask[ta], s_b0, s_b1,
                                               s_slot, uleaf + g * cap + c0, blo + n_internal, bhi + n_internal, s_upos, posh, lq, capq, tested);
            else if (interior)
                cache_walk_lane<T, false, false>(pa, qa, live, S, nu, bx, rkc, s_mask[ta], s_b0, s_b1,
                                                 s_slot, uleaf + g * cap + c0, blo + n_internal, bhi + n_internal, s_upos, posh, lq, capq,
                                                 tested);
            else
                cache_walk_lane<T, false, true>(pa, qa, live, S, nu, bx, rkc, s_mask[ta], s_b0, s_b1,
                                                s_slot, uleaf + g * cap + c0, blo + n_internal, bhi + n_internal, s_upos, posh, lq, capq, tested);
        }
        wbuf = lq.pos ? q_ld(lq.e) : 0ull;
    }
    const u32 c = w32 ? 2u * wq.q + wq.n : 4u * lq.q + lq.pos;
    if (live) {
        if (w32) {
            if (wq.n && wq.q < capq) *wq.out = (u64)wq.pend | ((u64)SLOT32_NONE << 32);
        } else if (c & 3u) {
            for (u32 r = c & 3u; r < 4u; ++r) wbuf |= (u64)SLOT_NONE << (16u * r);
            const u32 q = c >> 2;
            if (q < capq) out[(u64)q * GROUP] = wbuf;
        }
        ncnt[a] = c;
    }
    if (work) {   // work counters (profiling): candidate tests, prune tests
        const u64 t = block_reduce<GROUP>((u64)tested, s_w, [](u64 x, u64 y) { return x + y; });
        if (threadIdx.x == 0) {
            atomicAdd((unsigned long long*)&work[2 * (g & 63)], (unsigned long long)t);
            atomicAdd((unsigned long long*)&work[2 * (g & 63) + 1], (unsigned long long)boxtests);
        }
    }
    // the group's need in words (for the next build's plan and a regrow)
    const u32 esh = w32 ? 1u : 2u;     // log2 of the entries per word
    const u32 wmax = block_reduce<GROUP>(live ? (c + (1u << esh) - 1u) >> esh : 0u, (u32*)s_w,
                                         [](u32 x, u32 y) { return x > y ? x : y; });
    if (threadIdx.x == 0) {
        gneed[g] = wmax;
        if (wmax > capq) atomicOr(&flags[0], 4u);
        const u32 ecap = wmax << esh;
        if (ecap > __hip_atomic_load(&flags[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&flags[2], ecap);
    }
}

// Capacity plan of a build (see kernels.hpp): one thread per group.
__global__ void k_cache_plan(const u32* __restrict__ ustot, const u32* __restrict__ gneed,
                             i64 ngroups, u32 dflt, u32* __restrict__ gcap,
                             const u32* __restrict__ skip)
{
    const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups || (skip && *skip)) return;
    const u32 need = gneed ? gneed[g] : 0u;
    u32 w = need ? need + need / 4u + 2u : dflt;
    const u32 S = ustot[g];                        // a lane holds at most the union
    const u32 top = slots_wide(S) ? (S + 1u) / 2u + 1u : (S + 3u) / 4u + 1u;
    gcap[g] = w < top ? w : top;
}

// Regrow after an overflow: one thread per group; ranges appended in any
// order (the layout is free, the contents are not affected).
__global__ void k_cache_regrow(const u32* __restrict__ gneed, i64 ngroups, u32* __restrict__ gcap,
                               u64* __restrict__ gbase, u8* __restrict__ gredo)
{
    const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    const u32 need = gneed[g];
    if (need > gcap[g]) {
        const u32 w = need + need / 4u + 2u;
        gcap[g] = w;
        gbase[g] = atomicAdd((unsigned long long*)&gbase[ngroups], (unsigned long long)w);
        gredo[g] = 1;
    } else {
        gredo[g] = 0;
    }
}

// Convert the cache to global key-order indices (export / tests only):
// list[off[a] + j] = key slot of the j-th neighbour of a.
__global__ void __launch_bounds__(GROUP)
k_cache_to_global(const u32* __restrict__ id, const GroupMap gm, i64 cap,
                  const u32* __restrict__ uleaf, const u32* __restrict__ uslot,
                  const u32* __restrict__ ucnt, const u32* __restrict__ ustot,
                  const u64* __restrict__ gbase, const u64* __restrict__ nlist,
                  const u32* __restrict__ ncnt, const u64* __restrict__ off, u32* __restrict__ list)
{
    const i64 g = blockIdx.x;
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    const i64 a = beg + threadIdx.x;
    if (a >= end) return;
    const u32 nu = min((u32)cap, ucnt[g]);
    const u32* sl = uslot + g * cap;
    const u32* ul = uleaf + g * cap;
    const u32 c = ncnt[a];
    const bool w32 = slots_wide(ustot[g]);
    for (u32 j = 0; j < c; ++j) {
        const u64 w = nlist[(gbase[g] + (w32 ? j >> 1 : j >> 2)) * GROUP + threadIdx.x];
        const u32 s = w32 ? slot32_of(w, j & 1u) : slot_of(w, j & 3u);
        u32 lo = 0, hi = nu - 1;       // last leaf whose start slot <= s
        while (lo < hi) {
            const u32 mid = (lo + hi + 1) >> 1;
            if (sl[mid] <= s) lo = mid; else hi = mid - 1;
        }
        list[off[a] + j] = id[ul[lo]] + (s - sl[lo]);
    }
}

template <class T>
void launch_group_boxes(const vec4<T>* posh, const GroupMap& gm, i64 ngroups, vec4<T>* glo,
                        vec4<T>* ghi, hipStream_t st, const u32* skip)
{
    if (ngroups <= 0) return;
    hipLaunchKernelGGL((k_group_boxes<T>), dim3((unsigned)((ngroups + GB_WAVES - 1) / GB_WAVES)),
                       dim3(GB_WAVES * WAVE), 0, st, posh, gm, ngroups, glo, ghi, skip);
}

template <class T>
void launch_group_leaves(const vec4<T>* blo, const vec4<T>* bhi, const u32* child, const u32* id,
                         const u32* xscan, i64 n_internal, const vec4<T>* glo, const vec4<T>* ghi,
                         i64 ngroups, const GroupMap& gm, const u32* root, const InstDev* inst,
                         double rk, i64 cap, u32 spread, bool serial, u32* uleaf, u32* uslot,
                         u32* ucnt, u32* ustot, u32* flags, const u8* redo, hipStream_t st)
{
    if (ngroups <= 0) return;
    if (!serial) {
        const dim3 gc((unsigned)((ngroups + S1_CWAVES - 1) / S1_CWAVES));
        hipLaunchKernelGGL((k_group_leaves_wave<T, false>), gc, dim3(S1_CWAVES * WAVE), 0, st, blo,
                           bhi, child, id, xscan, n_internal, glo, ghi, ngroups, gm, root, inst,
                           (T)rk, cap, uleaf, uslot, ucnt, ustot, flags, redo);
        const dim3 gw((unsigned)((ngroups + S1_WAVES - 1) / S1_WAVES));
        hipLaunchKernelGGL((k_group_leaves_wave<T, true>), gw, dim3(S1_WAVES * WAVE), 0, st, blo,
                           bhi, child, id, xscan, n_internal, glo, ghi, ngroups, gm, root, inst,
                           (T)rk, cap, uleaf, uslot, ucnt, ustot, flags, redo);
    }
    // the serial walk takes every group (serial) or the marked ones
    const dim3 grid((unsigned)((ngroups + TRAV_BLOCK - 1) / TRAV_BLOCK));
    hipLaunchKernelGGL((k_group_leaves_serial<T>), grid, dim3(TRAV_BLOCK), 0, st, !serial, blo,
                       bhi, child, id, xscan, n_internal, glo, ghi, ngroups, gm, root, inst, (T)rk,
                       cap, spread, uleaf, uslot, ucnt, ustot, flags, redo);
}

template <class T>
void launch_group_cache(const vec4<T>* posh, const vec4<T>* blo, const vec4<T>* bhi, const u32* id,
                        const u32* xscan, i64 n_internal, const GroupMap& gm, i64 ngroups, const InstDev* inst,
                        double rk, double rkc, i64 cap, const u32* uleaf, const u32* uslot,
                        const u32* ucnt, const u32* ustot, const u64* gbase, const u32* gcap,
                        u64 words_alloc, u32* gneed, const u8* gredo, u64* nlist, u32* ncnt,
                        u32* flags, const vec4<T>* glo, const vec4<T>* ghi, const u32* root,
                        u64* work, int mode, const u8* redo, hipStream_t st)
{
    if (ngroups <= 0) return;
    auto kern = mode == 2 ? k_group_cache<T, 2> : mode == 0 ? k_group_cache<T, 0> : k_group_cache<T, 1>;
    hipLaunchKernelGGL(kern, dim3((unsigned)ngroups), dim3(GROUP), 0, st, posh, blo,
                       bhi, id, xscan, n_internal, gm, inst, (T)rk, (T)rkc, cap, uleaf, uslot, ucnt, ustot,
                       gbase, gcap, words_alloc, gneed, gredo, nlist, ncnt, flags, glo, ghi, root, work,
                       redo);
}

void launch_cache_plan(const u32* ustot, const u32* gneed, i64 ngroups, u32 dflt, u32* gcap,
                       u64* gbase, void* scan_tmp, hipStream_t st, const u32* skip)
{
    if (ngroups <= 0) return;
    // (with skip set the scan recomputes the same layout from the same gcap)
    hipLaunchKernelGGL(k_cache_plan, dim3((unsigned)((ngroups + 255) / 256)), dim3(256), 0, st, ustot, gneed, ngroups,
                       dflt, gcap, skip);
    scan_u32_u64(gcap, gbase, ngroups, scan_tmp, st);
}

void launch_cache_regrow(const u32* gneed, i64 ngroups, u32* gcap, u64* gbase, u8* gredo,
                         hipStream_t st)
{
    if (ngroups <= 0) return;
    hipLaunchKernelGGL(k_cache_regrow, dim3((unsigned)((ngroups + 255) / 256)), dim3(256), 0, st, gneed, ngroups,
                       gcap, gbase, gredo);
}

void launch_cache_to_global(const u32* id, const GroupMap& gm, i64 ngroups, i64 cap,
                            const u32* uleaf, const u32* uslot, const u32* ucnt, const u32* ustot,
                            const u64* gbase, const u64* nlist, const u32* ncnt, const u64* off,
                            u32* list, hipStream_t st)
{
    if (ngroups <= 0) return;
    hipLaunchKernelGGL(k_cache_to_global, dim3((unsigned)ngroups), dim3(GROUP), 0, st, id, gm, cap,
                       uleaf, uslot, ucnt, ustot, gbase, nlist, ncnt, off, list);
}

#define INST(T)                                                                                   \
    template void launch_group_boxes<T>(const vec4<T>*, const GroupMap&, i64, vec4<T>*, vec4<T>*, \
                                        hipStream_t, const u32*);                                 \
    template void launch_group_leaves<T>(const vec4<T>*, const vec4<T>*, const u32*, const u32*, const u32*,  \
                                         i64, const vec4<T>*, const vec4<T>*, i64,                \
                                         const GroupMap&, const u32*, const InstDev*, double,     \
                                         i64, u32, bool, u32*, u32*, u32*, u32*, u32*,            \
                                         const u8*, hipStream_t);                                 \
    template void launch_group_cache<T>(const vec4<T>*, const vec4<T>*, const vec4<T>*,           \
                                        const u32*, const u32*, i64, const GroupMap&, i64, const InstDev*,    \
                                        double, double, i64, const u32*, const u32*, const u32*,  \
                                        const u32*, const u64*, const u32*, u64, u32*, const u8*,  \
                                        u64*, u32*, u32*, const vec4<T>*,                          \
                                        const vec4<T>*, const u32*, u64*, int, const u8*,         \
                                        hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace shsph
