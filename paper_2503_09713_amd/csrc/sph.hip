// SPH loops over the neighbour cache: the smoothing-length / density
// iteration with Omega (App. F, Alg. 7; Sect. 2.1 Eq. sphomega), the force and
// energy equations with artificial viscosity and conductivity (Sect. 2.1
// Eqs. sphvel, sphuint), the leapfrog corrector and the timestep reductions
// (App. G).  One thread per particle in key order; arithmetic and
// accumulation in the storage type.
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>

#include <hip/hip_cooperative_groups.h>

namespace shsph {

static inline dim3 grid_for(i64 n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

__global__ void k_fill_u32(u32* p, i64 n, u32 v)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_iota_u32(u32* p, i64 n)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (u32)i;
}

// Reset per-instance reductions: what & 1 the h-iteration counters (only for
// instances with redo[k] != 0 when redo is given), what & 2 the timestep and
// corrector reductions.
__global__ void k_stat_reset(InstStat* s, int ninst, int what, const u8* redo, const u32* skip)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ninst || (skip && *skip)) return;
    InstStat& z = s[k];
    if ((what & 1) && (!redo || redo[k])) {
        z.n_exceed = 0u;
        z.n_noconv = 0u;
        z.max_iter_seen = 0u;
    }
    if (what & 2) {
        z.dt_bits = 0x7f800000u;   // +inf
        z.dvmax_bits = 0u;
        for (int i = 0; i < STAT_SLOTS; ++i) { z.dv2_part[i] = 0.0; z.v2_part[i] = 0.0; }
    }
    z.pad[0] = z.pad[1] = z.pad[2] = 0u;
}

// h_max of each instance's root cell (for the periodic radius check).
template <class T>
__global__ void k_root_hmax(const vec4<T>* __restrict__ blo, const u32* __restrict__ root,
                            int ninst, double* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < ninst) out[k] = (double)blo[root[k]].w;
}

// ---------------------------------------------------------------------------
// Gates of a captured pass (one workgroup each).  gs[0] is the pass's abort
// word: set when the build met a condition that the launch-by-launch pass
// handles on the host between launches (a capacity to grow and a stage to
// redo, the leaf-pass fallback, a look-back overrun, a periodic box below
// twice the cache radius) or when some h left chi h_cache (a cache rebuild).
// Every later stage then does nothing, the caller's arrays keep their state
// and the host runs the pass again launch by launch.  gate[k] = 1 - gs[0]
// for every instance (the density's per-instance switch).  The word tells
// why: bit 0 the build's capacity / stack / box-record flags (flag word in
// bits 8-15), bit 1 a sort look-back overrun, bit 2 the leaf pass's fallback
// or overrun, bit 3 a periodic box below twice the cache radius, bit 4 a
// rebuild round's flags (in bits 16-23), bit 5 an h still past chi h_cache
// after the rebuild rounds.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_gate_build(const u32* __restrict__ flags, u32 mask0, int w_sort, int w_leaves,
             const double* __restrict__ rhmax, const InstDev* __restrict__ inst, int ninst,
             double rk, u32* __restrict__ gs, u8* __restrict__ gate, u32* __restrict__ reruns)
{
    __shared__ int s_bad;
    if (threadIdx.x == 0) {
        const u32 f0 = flags[0] & mask0;
        s_bad = (int)((f0 ? 1u | (f0 << 8) : 0u) | (flags[w_sort] ? 2u : 0u) |
                      ((flags[w_leaves] | flags[w_leaves + 1]) ? 4u : 0u));
    }
    __syncthreads();
    for (int k = threadIdx.x; k < ninst; k += blockDim.x) {
        reruns[k] = 0u;
        const InstDev in = inst[k];
        if (!in.periodic) continue;
        for (int d = 0; d < 3; ++d)
            if (rk * rhmax[k] >= 0.5 * (in.hi[d] - in.lo[d])) atomicOr(&s_bad, 8);
    }
    __syncthreads();
    const bool bad = s_bad != 0;
    if (threadIdx.x == 0) gs[0] = (u32)s_bad;
    for (int k = threadIdx.x; k < ninst; k += blockDim.x) gate[k] = bad ? 0 : 1;
}

__global__ void __launch_bounds__(256)
k_gate_density(const InstStat* __restrict__ stat, int ninst, u32* __restrict__ gs,
               u8* __restrict__ gate)
{
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = gs[0] != 0u;
    __syncthreads();
    for (int k = threadIdx.x; k < ninst; k += blockDim.x)
        if (stat[k].n_exceed) atomicOr(&s_bad, 1);
    __syncthreads();
    if (!s_bad) return;
    if (threadIdx.x == 0) gs[0] |= 32u;
    for (int k = threadIdx.x; k < ninst; k += blockDim.x) gate[k] = 0;
}

// Cache-rebuild round of a captured pass: the instances with a particle past
// chi h_cache (rx[k] = 1) get new caches and run the h iteration again, as
// the launch-by-launch pass does; *skw = 1 when there are none (or the pass
// was switched off), which switches the round's launches off.
__global__ void __launch_bounds__(256)
k_gate_exceed(const InstStat* __restrict__ stat, int ninst, const u32* __restrict__ gs,
              u32* __restrict__ skw, u8* __restrict__ rx)
{
    __shared__ int s_any;
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    const bool off = gs[0] != 0u;
    for (int k = threadIdx.x; k < ninst; k += blockDim.x) {
        const bool x = !off && stat[k].n_exceed != 0u;
        rx[k] = x ? 1 : 0;
        if (x) atomicOr(&s_any, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *skw = s_any ? 0u : 1u;
}

// After a rebuild round's caches: the build's conditions (as k_gate_build)
// switch the pass off, and the round's h iteration with it.
__global__ void __launch_bounds__(256)
k_gate_round(const u32* __restrict__ flags, u32 mask0, const double* __restrict__ rhmax,
             const InstDev* __restrict__ inst, int ninst, double rk, const u32* __restrict__ skw,
             u32* __restrict__ gs, u8* __restrict__ rx)
{
    __shared__ int s_bad;
    if (*skw) return;
    if (threadIdx.x == 0) {
        const u32 f0 = flags[0] & mask0;
        s_bad = (int)(f0 ? 16u | (f0 << 16) : 0u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < ninst; k += blockDim.x) {
        const InstDev in = inst[k];
        if (!in.periodic) continue;
        for (int d = 0; d < 3; ++d)
            if (rk * rhmax[k] >= 0.5 * (in.hi[d] - in.lo[d])) atomicOr(&s_bad, 8);
    }
    __syncthreads();
    if (!s_bad) return;
    if (threadIdx.x == 0) gs[0] |= (u32)s_bad;
    for (int k = threadIdx.x; k < ninst; k += blockDim.x) rx[k] = 0;
}

// Corrector re-run round r of a captured pass (App. G.1, the reversibility
// check): instance k runs again when max|dv| > eps_v sqrt(sum|v|^2 / N_k)
// and it has re-run fewer than max_reruns times, from the reductions of the
// last corrector that ran (gs[r]: the pass's own for r = 0, else round r-1's;
// when that one was switched off, so is this round).  gs[1 + r] = 1 when no
// instance runs again.
__global__ void __launch_bounds__(256)
k_rerun_decide(const InstStat* __restrict__ stat, const i64* __restrict__ p_off, int ninst,
               double eps_v, int max_reruns, int r, u32* __restrict__ gs, u8* __restrict__ redo,
               u32* __restrict__ reruns)
{
    __shared__ int s_any;
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    const bool off = gs[r] != 0u;
    for (int k = threadIdx.x; k < ninst; k += blockDim.x) {
        bool want = false;
        if (!off) {
            const float dv = __uint_as_float(stat[k].dvmax_bits);
            double v2 = 0.0;
            for (int i = 0; i < STAT_SLOTS; ++i) v2 += stat[k].v2_part[i];
            const i64 cnt = p_off[k + 1] - p_off[k];
            want = (double)dv > eps_v * sqrt(v2 / (double)(cnt > 1 ? cnt : 1)) &&
                   reruns[k] < (u32)max_reruns;
        }
        redo[k] = want ? 1 : 0;
        if (want) {
            ++reruns[k];
            atomicOr(&s_any, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) gs[1 + r] = s_any ? 0u : 1u;
}

// dt for the coming step: the caller's value when positive, else the CFL dt
// left by the previous force evaluation.
// dt of each instance: dt_host > 0 is a fixed dt; otherwise the CFL dt of
// the last force evaluation, times -dt_host when dt_host < 0 (the CFL
// multiplier of App. G; 0 means a multiplier of 1).
__global__ void k_dt_select(double* dt_inst, const InstStat* s, const double* dt_host, int ninst)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ninst) return;
    const double h = dt_host[k];
    const double lam = h < 0.0 ? -h : 1.0;
    dt_inst[k] = (h > 0.0) ? h : lam * (double)__uint_as_float(s[k].dt_bits);
}

template <class T> __global__ void k_copy_h(const vec4<T>* __restrict__ posh, T* __restrict__ hc, i64 n,
                                            const u32* __restrict__ skip)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(skip && *skip)) hc[i] = posh[i].w;
}


// Visit the cache entries of one particle (ELL words `my`, cnt entries).
// One LDS tile: all entries, four per word, padding skipped.  Several
// tiles: entries with slots in [c0, c1), resuming at entry j.
// f(slot) for each stored slot (single visits; for heavy per-pair bodies).
// The next word is loaded while the current one is used; the load is
// unconditional (the last word is read again at the end) so that no branch
// around it makes the compiler wait for it before the current word.
template <class F> __device__ inline void entries_each(const u64* my, u32 cnt, F&& f)
{
    const u32 nq = (cnt + 3u) >> 2;
    u64 w = nq ? my[0] : 0;
    for (u32 q = 0; q < nq; ++q) {
        const u64 wn = my[(u64)(q + 1 < nq ? q + 1 : q) * GROUP];   // prefetch
#pragma unroll
        for (u32 r = 0; r < 4u; ++r) {
            const u32 sl = slot_of(w, r);
            if (sl != SLOT_NONE) f(sl);
        }
        w = wn;
    }
}

// Entries [4 q0, min(cnt, 4 q1)) only (words q0 .. q1-1), single visits.
template <class F> __device__ inline void entries_words(const u64* my, u32 cnt, u32 q0, u32 q1, F&& f)
{
    const u32 nq = min((cnt + 3u) >> 2, q1);
    u64 w = q0 < nq ? my[(u64)q0 * GROUP] : 0;
    for (u32 q = q0; q < nq; ++q) {
        const u64 wn = my[(u64)(q + 1 < nq ? q + 1 : q) * GROUP];   // prefetch (see entries_each)
#pragma unroll
        for (u32 r = 0; r < 4u; ++r) {
            const u32 sl = slot_of(w, r);
            if (sl != SLOT_NONE) f(sl);
        }
        w = wn;
    }
}

// Entries of one particle with slots in [c0, c1), from entry j on (the
// tiled path: the union staged chunk by chunk, the entries ascending), f(slot
// - c0) each; j is left at the first entry of a later chunk.  Each word is
// read once per chunk, the next one loaded while the current one is used.
// (w32: the group stores 32-bit slots, two per word.)
template <class F>
__device__ inline void entries_tile(const u64* my, u32 cnt, u32& j, u32 c0, u32 c1, bool w32,
                                    F&& f)
{
    if (j >= cnt) return;
    const u32 sh = w32 ? 1u : 2u, per = 1u << sh;
    const u32 nq = (cnt + per - 1u) >> sh;
    u32 q = j >> sh;
    u64 w = my[(u64)q * GROUP];
    for (;;) {
        const u64 wn = my[(u64)(q + 1 < nq ? q + 1 : q) * GROUP];   // prefetch
        const u32 rend = min(per, cnt - (q << sh));
        for (u32 r = j & (per - 1u); r < rend; ++r) {
            const u32 sl = w32 ? slot32_of(w, r) : slot_of(w, r);
            if (sl >= c1) {
                j = (q << sh) + r;
                return;
            }
            f(sl - c0);
        }
        if (++q >= nq) {
            j = cnt;
            return;
        }
        j = q << sh;
        w = wn;
    }
}

// Block-wide reduction helpers for per-instance statistics: the block's
// lanes usually share one instance, then a single atomic per block is done
// (and min/max atomics only when they can change the stored value).
__device__ inline bool block_uniform(int k, int* s_k)
{
    if (threadIdx.x == 0) *s_k = k;
    __syncthreads();
    const int k0 = *s_k;
    return __syncthreads_and(k == k0) != 0;
}

template <class T> __device__ inline T block_max(T v, T* lds)
{
    return block_reduce<GROUP>(v, lds, [](T a, T b) { return a > b ? a : b; });
}
template <class T> __device__ inline T block_min(T v, T* lds)
{
    return block_reduce<GROUP>(v, lds, [](T a, T b) { return a < b ? a : b; });
}
template <class T> __device__ inline T block_sum(T v, T* lds)
{
    return block_reduce<GROUP>(v, lds, [](T a, T b) { return a + b; });
}

__device__ inline void atomic_max_if(u32* p, u32 v)
{
    if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}
__device__ inline void atomic_min_if(u32* p, u32 v)
{
    if (v < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(p, v);
}

// ---------------------------------------------------------------------------
// h iteration (App. F, Alg. 7), per particle, over the cached neighbours:
//   rho_sum = sum_b m W(r_ab, h),   W = f(r/h)/(pi h^3)
//   drho = rho_sum - m (hfact/h)^3,  d(drho)/dh = sum_b m dW/dh + 3 rho_sum/h
//   (the derivative term as Alg. 7 prints it, with the SPH sum: it equals the
//   exact derivative at the root, and since every M4 term has
//   dW/dh >= -3 W / h it never goes negative, so the step always points
//   towards smaller |drho|; only the particle itself within 2h gives 0,
//   and then the step is the clamp in the direction that lowers |drho|);
//   Newton step, clamped to [h/lambda, h lambda]; eps = |h' - h| / h^n.
// The particle stops when eps < eps_h.  If h' exceeds chi times the h the
// cache was built with, h' is clamped there and the particle is flagged: the
// caller rebuilds the cache with the new h and iterates again (the
// single-device form of the ghost re-exchange).
// Final values: rho = m (hfact/h)^3 (App. F uses rho(h), not the sum) and
// Omega = 1 + h/(3 rho) sum_b m dW/dh (Eq. sphomega with dh/drho = -h/(3 rho)),
// both taken at the last h where the sums were evaluated.
// One workgroup per group: the union's positions are staged in LDS once and
// every Newton pass reads neighbours from there.
// ---------------------------------------------------------------------------
// Union staging of the density and the force: FP32 with two slots' loads in
// flight per thread; FP64 one leaf per thread (the batch's registers would
// cost the FP64 force a wave per SIMD).
template <class T> constexpr int STAGE_B = sizeof(T) == 4 ? 2 : 0;

template <class T, int CH> struct DensShared {
    vec4<T> pos[CH];
    u32 red[GROUP / WAVE];
    u64 w[GROUP / WAVE];
    int k;
};

// Arguments of the density pass (one group at a time).
template <class T> struct DensArgs {
    vec4<T>* posh;
    const T *hn, *hc;
    const vec4<T>* velu;
    const u32* id;
    GroupMap gm;
    const InstDev* inst;
    SphParams P;
    CacheView cv;
    T* omega;
    vec4<T>* thermo;
    u8* status;
    InstStat* stat;
    const u8* redo;
};

template <class T, int CH, int K>
__device__ __attribute__((always_inline)) inline void
density_group(const i64 g, vec4<T>* __restrict__ posh, const T* __restrict__ hn,
              const T* __restrict__ hc, const vec4<T>* __restrict__ velu,
              const u32* __restrict__ id, const GroupMap gm, const InstDev* __restrict__ inst,
              const SphParams P, const CacheView cv, T* __restrict__ omega,
              vec4<T>* __restrict__ thermo, u8* __restrict__ status, InstStat* __restrict__ stat,
              const u8* __restrict__ redo, DensShared<T, CH>& sh)
{
    vec4<T>* const s_pos = sh.pos;
    u32* const s_red = sh.red;
    u64* const s_w = sh.w;
    int* const s_k = &sh.k;
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    if (redo && !redo[k]) return;     // this instance's h is final (uniform per group)
    const InstDev in = inst[k];
    const Box<T> bx = make_box<T>(in);
    const i64 a = beg + threadIdx.x;
    const bool live = a < end;
    const i64 ai = live ? a : beg;
    const vec4<T> pa = posh[ai];
    const T m = (T)in.mass, hfact = (T)P.hfact, lam = (T)P.lambda, chi = (T)P.chi;
    const T h_n = hn[ai], h_c = hc[ai];
    const u32 cnt = live ? cv.ncnt[a] : 0u;
    const u32 nu = min((u32)cv.cap, cv.ucnt[g]);
    const u32 S = cv.ustot[g];
    const u32 nch = (S + CH - 1) / CH;
    const u32* ul = cv.uleaf + g * cv.cap;
    const u32* us = cv.uslot + g * cv.cap;
    const u64* my = cv.nlist + cv.gbase[g] * GROUP + threadIdx.x;
    const vec4<T>* src[1] = { posh };
    vec4<T>* dst[1] = { s_pos };
    T h = pa.w, h_eval = pa.w, dsum = T(0);
    int st = 1;   // 0 converged, 1 not converged, 2 chi exceeded
    int iters = 0;
    bool active = live;
    u64 evals = 0;                       // entries evaluated (profiling)
    u32 inrange = 0;                     // of them within 2h (profiling)
    const bool wrap = !group_interior<T>(((const vec4<T>*)cv.glo)[g], ((const vec4<T>*)cv.ghi)[g],
                                         ((const vec4<T>*)cv.blo)[cv.root[k]].w, (T)cv.rk, bx);
    const T RK = Kern<K>::template R<T>(), CK = Kern<K>::template C<T>();
    if (nch == 1) {                      // the whole union, staged once for every pass
        stage_union<T, 1, GROUP, STAGE_B<T>>(src, dst, id, ul, us, nu, 0u, S);
        __syncthreads();
    }
    for (int it = 0; it < P.max_iter; ++it) {
        const T hinv = T(1) / h;
        const T hR2 = RK * RK * h * h;
        T s = T(0), dq = T(0);          // sum f, sum -q f' (>= 0: f is non-increasing)
        if (active) evals += cnt;
        auto add_r2 = [&](T r2) {
            if (r2 < hR2) {
                ++inrange;
                const T q = fast_sqrt(r2) * hinv;
                T f, df;
                Kern<K>::template fdf<T>(q, f, df);
                s += f;
                dq -= q * df;
            }
        };
        auto add = [&](u32 sl) {          // any group: minimum image
            const vec4<T> pb = s_pos[sl];
            const T dx = min_image(pa.x - pb.x, bx.L[0], bx.halfL[0], bx.periodic);
            const T dy = min_image(pa.y - pb.y, bx.L[1], bx.halfL[1], bx.periodic);
            const T dz = min_image(pa.z - pb.z, bx.L[2], bx.halfL[2], bx.periodic);
            add_r2(dx * dx + dy * dy + dz * dz);
        };
        auto add_in = [&](u32 sl) {       // interior group: no image can be closer
            const vec4<T> pb = s_pos[sl];
            const T dx = pa.x - pb.x, dy = pa.y - pb.y, dz = pa.z - pb.z;
            add_r2(dx * dx + dy * dy + dz * dz);
        };
        if (nch == 1) {
            if (active) {
                if (wrap) entries_each(my, cnt, add);
                else entries_each(my, cnt, add_in);
            }
        } else {
            u32 j = 0;
            for (u32 ch = 0; ch < nch; ++ch) {
                const u32 c0 = ch * CH, c1 = min(S, c0 + CH);
                __syncthreads();
                stage_union<T, 1, GROUP, STAGE_B<T>>(src, dst, id, ul, us, nu, c0, c1);
                __syncthreads();
                if (active) entries_tile(my, cnt, j, c0, c1, slots_wide(S), add);
            }
        }
        if (active) {
            const T hinv3 = hinv * hinv * hinv;
            const T rho_sum = m * s * hinv3 * CK;
            const T mh4 = m * hinv3 * hinv * CK;
            const T dsum_h = mh4 * (dq - T(3) * s);      // sum_b m dW/dh
            const T hf = hfact * hinv;
            const T rho_h = m * hf * hf * hf;
            const T ddrho = mh4 * dq;                     // = dsum_h + 3 rho_sum / h
            const T drho = rho_sum - rho_h;
            T hnew = ddrho > T(0) ? h - drho / ddrho : (drho < T(0) ? h * lam : h / lam);
            if (hnew > h * lam) hnew = h * lam;
            else if (hnew < h / lam) hnew = h / lam;
            const T eps = fabs(hnew - h) / h_n;
            h_eval = h;
            dsum = dsum_h;
            iters = it + 1;
            if (hnew > h_c * chi) { h = h_c * chi; st = 2; active = false; }
            else {
                h = hnew;
                if (eps < (T)P.eps_h) { st = 0; active = false; }
            }
        }
        if (!__syncthreads_or(active)) break;
    }
    // per-instance outcome counters (rare events: per-lane atomics)
    if (live && st == 2) atomicAdd(&stat[k].n_exceed, 1u);
    if (live && st == 1) atomicAdd(&stat[k].n_noconv, 1u);
    if (block_uniform(k, s_k)) {
        const u32 mx = block_max<u32>(live ? (u32)iters : 0u, s_red);
        if (threadIdx.x == 0) atomic_max_if(&stat[k].max_iter_seen, mx);
    } else if (live) {
        atomic_max_if(&stat[k].max_iter_seen, (u32)iters);
    }
    if (cv.work) {   // work counters (profiling): pair evaluations, those within 2h
        const u64 t1 = block_reduce<GROUP>(evals, s_w, [](u64 x, u64 y) { return x + y; });
        const u64 t2 = block_reduce<GROUP>((u64)inrange, s_w, [](u64 x, u64 y) { return x + y; });
        if (threadIdx.x == 0) {
            atomicAdd((unsigned long long*)&cv.work[2 * (g & 63)], (unsigned long long)t1);
            atomicAdd((unsigned long long*)&cv.work[2 * (g & 63) + 1], (unsigned long long)t2);
        }
    }
    if (!live) return;
    const T hf = hfact / h_eval;
    const T rho_e = m * hf * hf * hf;
    const T om = T(1) + h_eval / (T(3) * rho_e) * dsum;
    const T hfo = hfact / h;
    const T rho = m * hfo * hfo * hfo;
    posh[a].w = h;
    omega[a] = om;
    status[a] = (u8)st;
    if (thermo) {
        const T u = velu ? velu[a].w : T(0);
        const T gm1 = (T)P.gamma - T(1);
        const T Pr = gm1 * rho * u;
        const T cs = sqrt((T)P.gamma * gm1 * u);
        const T B = T(1) / (rho * om);
        thermo[a] = mk4<T>(Pr * B / rho, T(0.5) * B, (T)P.alpha * cs, Pr);
    }
}

template <class T, int CH, int K>
__device__ __attribute__((always_inline)) inline void density_group(const i64 g, const DensArgs<T>& A,
                                                                    DensShared<T, CH>& sh)
{
    density_group<T, CH, K>(g, A.posh, A.hn, A.hc, A.velu, A.id, A.gm, A.inst, A.P, A.cv, A.omega,
                            A.thermo, A.status, A.stat, A.redo, sh);
}

// FP32: at most 64 VGPRs, so that registers allow the eight waves per SIMD
// that its LDS chunk allows.
template <class T, int CH, int K>
__global__ void __launch_bounds__(GROUP, sizeof(T) == 4 ? 8 : 1)
k_density(vec4<T>* __restrict__ posh, const T* __restrict__ hn, const T* __restrict__ hc,
          const vec4<T>* __restrict__ velu, const u32* __restrict__ id, const GroupMap gm,
          const InstDev* __restrict__ inst, SphParams P, CacheView cv, T* __restrict__ omega,
          vec4<T>* __restrict__ thermo, u8* __restrict__ status, InstStat* __restrict__ stat,
          const u8* __restrict__ redo)
{
    __shared__ DensShared<T, CH> sh;
    density_group<T, CH, K>(blockIdx.x, posh, hn, hc, velu, id, gm, inst, P, cv, omega, thermo,
                            status, stat, redo, sh);
}

// ---------------------------------------------------------------------------
// Force and energy (Sect. 2.1):
//   dv_a/dt = -sum_b m [(P_a+q^a)/(rho_a^2 Om_a) F_a + (P_b+q^b)/(rho_b^2 Om_b) F_b] rhat_ab
//   du_a/dt =  sum_b m (P_a+q^a)/(rho_a^2 Om_a) (v_ab . rhat_ab) F_a + Lambda_cond
// F_x = f'(r/h_x)/(pi h_x^4) (= rhat . grad W), q^x = -rho_x vsig_x w / 2 for
// w = v_ab . rhat_ab < 0, vsig_x = alpha_x c_x + beta |w| (alpha_x c_x staged
// per particle: the constant alpha, or the shock detector's alpha_x).  With
// A = P/(rho^2 Om) and the staged half B' = 1/(2 rho Om):
// (P+q)/(rho^2 Om) = A - vsig w B'.
// Conductivity: m beta_u vsig_u (u_a-u_b) (F_a B'_a + F_b B'_b) with
// vsig_u = sqrt(|P_a - P_b| / rhobar), rhobar = (rho_a+rho_b)/2, formed as
// d rsq(d rhobar) for d = |P_a - P_b| > 0 (one reciprocal square root).
// The timestep signal speed is the largest vsig_a over the pairs (floor c_a);
// dt_a = min(C_cour h/vsig, C_force sqrt(h/|a|)) is min-reduced per instance.
// One workgroup per group: the union's position, velocity and pressure terms
// are staged in LDS.
// ---------------------------------------------------------------------------
// SPLIT threads per particle (1 or 2: workgroups of 256 or 512 threads),
// each taking its share of the particle's list; the shares are combined in a
// fixed order.
template <class T, int CH, int SPLIT> struct ForceShared {
    vec4<T> pos[CH], vel[CH], thm[CH];
    T half[6][SPLIT > 1 ? GROUP : 1];   // second-half sums, added by the first half
    float red[SPLIT * GROUP / WAVE];
    u64 w[SPLIT * GROUP / WAVE];
    int k;
};

// Arguments of the force pass (one group at a time).
template <class T> struct ForceArgs {
    const vec4<T> *posh, *velu, *thermo;
    const u32* id;
    GroupMap gm;
    const InstDev* inst;
    SphParams P;
    CacheView cv;
    vec4<T>* acc;
    T* vsig_out;
    InstStat* stat;
};

template <class T, int CH, int K, int SPLIT>
__device__ __attribute__((always_inline)) inline void
force_group(const i64 g, const vec4<T>* __restrict__ posh, const vec4<T>* __restrict__ velu,
            const vec4<T>* __restrict__ thermo, const u32* __restrict__ id, const GroupMap gm,
            const InstDev* __restrict__ inst, const SphParams P, const CacheView cv,
            vec4<T>* __restrict__ acc, T* __restrict__ vsig_out, InstStat* __restrict__ stat,
            ForceShared<T, CH, SPLIT>& sh)
{
    constexpr int FT = SPLIT * GROUP;
    vec4<T>* const s_pos = sh.pos;
    vec4<T>* const s_vel = sh.vel;
    vec4<T>* const s_thm = sh.thm;
    auto& s_half = sh.half;
    float* const s_red = sh.red;
    u64* const s_w = sh.w;
    int* const s_k = &sh.k;
    if (cv.skip && *cv.skip) return;      // switched off on the device (uniform)
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    const InstDev in = inst[k];
    const Box<T> bx = make_box<T>(in);
    const u32 lt = threadIdx.x & (GROUP - 1), half = threadIdx.x / GROUP;
    const i64 a = beg + lt;
    const bool live = a < end;
    const i64 ai = live ? a : beg;
    const T m = (T)in.mass, hfact = (T)P.hfact;
    const T beta = (T)P.beta, beta_u = (T)P.beta_u;
    const vec4<T> pa = posh[ai], va = velu[ai], ta = thermo[ai];
    const T ha = pa.w, hia = T(1) / ha;
    const T RK = Kern<K>::template R<T>(), CK = Kern<K>::template C<T>();
    const T hia4 = hia * hia * hia * hia * CK;
    const T hfa = hfact * hia;
    const T rhoa = m * hfa * hfa * hfa;
    const T mhf3 = m * hfact * hfact * hfact;    // rho_b = mhf3 / h_b^3
    const T Aa = ta.x, Ba = ta.y, aca = ta.z, Pa = ta.w;     // Ba = B'_a, aca = alpha_a c_a
    const T mbu = m * beta_u;
    const T ca = sqrt((T)P.gamma * ((T)P.gamma - T(1)) * va.w);   // c_a: floor of the signal speed
    const u32 cnt = live ? cv.ncnt[a] : 0u;
    const u32 nu = min((u32)cv.cap, cv.ucnt[g]);
    const u32 S = cv.ustot[g];
    const u32 nch = (S + CH - 1) / CH;
    const u32* ul = cv.uleaf + g * cv.cap;
    const u32* us = cv.uslot + g * cv.cap;
    const u64* my = cv.nlist + cv.gbase[g] * GROUP + lt;
    const vec4<T>* src[3] = { posh, velu, thermo };
    vec4<T>* dst[3] = { s_pos, s_vel, s_thm };
    // this thread's share of the list: words [q0, q1) (with two threads the
    // first takes the first ceil(nq/2) words), entries [e0, e1) for the
    // tiled path
    const bool w32 = slots_wide(S);
    const u32 esh = w32 ? 1u : 2u;      // log2 of the entries per word
    const u32 nq = (cnt + (1u << esh) - 1u) >> esh, qh = SPLIT > 1 ? (nq + 1u) >> 1 : nq;
    const u32 q0 = half ? qh : 0u, q1 = half ? nq : qh;
    const u32 e0 = min(cnt, q0 << esh), e1 = min(cnt, q1 << esh);
    T ax = T(0), ay = T(0), az = T(0), du = T(0), lam = T(0), vmax = ca;
    u32 inter = 0;                      // interacting pairs (profiling)
    const bool wrap = !group_interior<T>(((const vec4<T>*)cv.glo)[g], ((const vec4<T>*)cv.ghi)[g],
                                         ((const vec4<T>*)cv.blo)[cv.root[k]].w, (T)cv.rk, bx);
    // s_pos[].w holds 1/h of the staged particles (one reciprocal per
    // staged particle instead of one per pair); r < 2 max(h_a, h_b) is
    // tested as r^2 min(1/h_a, 1/h_b)^2 < 4 (the kernel gradient vanishes
    // at q = 2, so the rounding of that boundary changes no sum)
    auto sep = [&](u32 sl, bool img, T& dx, T& dy, T& dz) -> vec4<T> {
        const vec4<T> pb = s_pos[sl];
        if (img) {
            dx = min_image(pa.x - pb.x, bx.L[0], bx.halfL[0], bx.periodic);
            dy = min_image(pa.y - pb.y, bx.L[1], bx.halfL[1], bx.periodic);
            dz = min_image(pa.z - pb.z, bx.L[2], bx.halfL[2], bx.periodic);
        } else {
            dx = pa.x - pb.x; dy = pa.y - pb.y; dz = pa.z - pb.z;
        }
        return pb;
    };
    auto interacts = [&](T r2, T hib) -> bool {
        const T hmi = hia < hib ? hia : hib;
        return (r2 > T(0)) & (r2 * hmi * hmi < RK * RK);
    };
    auto eval_d = [&](u32 sl, T dx, T dy, T dz, const vec4<T>& pb) {   // an interacting pair
        const T r2 = dx * dx + dy * dy + dz * dz;
        const T hib = pb.w;
        ++inter;
        const vec4<T> vb = s_vel[sl], tb = s_thm[sl];
        const T rinv = fast_rsq(r2), r = r2 * rinv;
        const T ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
        const T w = (va.x - vb.x) * ex + (va.y - vb.y) * ey + (va.z - vb.z) * ez;
        const T Fa = Kern<K>::template df<T>(r * hia) * hia4;
        const T hib3 = hib * hib * hib;           // shared by F_b and rho_b
        const T Fb = Kern<K>::template df<T>(r * hib) * (hib3 * hib * CK);
        const T aw = fabs(w);
        const T vsa = aca + beta * aw;
        const T vsb = tb.z + beta * aw;
        const T wn = w < T(0) ? w : T(0);
        const T ka = (Aa - vsa * wn * Ba) * Fa;
        const T kb = (tb.x - vsb * wn * tb.y) * Fb;
        const T fab = m * (ka + kb);
        ax -= fab * ex;
        ay -= fab * ey;
        az -= fab * ez;
        du += m * ka * w;
        const T rhob = mhf3 * hib3;
        const T dP = fabs(Pa - tb.w);
        const T vsu = dP > T(0) ? dP * fast_rsq(dP * (T(0.5) * (rhoa + rhob))) : T(0);
        lam += mbu * vsu * (va.w - vb.w) * (Fa * Ba + Fb * tb.y);
        vmax = vsa > vmax ? vsa : vmax;
    };
    auto pair = [&](u32 sl) {             // any group: minimum image
        T dx, dy, dz;
        const vec4<T> pb = sep(sl, true, dx, dy, dz);
        if (interacts(dx * dx + dy * dy + dz * dz, pb.w)) eval_d(sl, dx, dy, dz, pb);
    };
    auto pair_in = [&](u32 sl) {          // interior group: no image can be closer
        T dx, dy, dz;
        const vec4<T> pb = sep(sl, false, dx, dy, dz);
        if (interacts(dx * dx + dy * dy + dz * dz, pb.w)) eval_d(sl, dx, dy, dz, pb);
    };
    auto invert_h = [&](u32 n_st) {
        for (u32 t = threadIdx.x; t < n_st; t += FT) s_pos[t].w = fast_rcp(s_pos[t].w);
    };
    if (nch == 1) {
        stage_union<T, 3, FT, STAGE_B<T>>(src, dst, id, ul, us, nu, 0u, S);
        __syncthreads();
        invert_h(S);
        __syncthreads();
        if (wrap) entries_words(my, cnt, q0, q1, pair);
        else entries_words(my, cnt, q0, q1, pair_in);
    } else {
        u32 j = e0;
        for (u32 ch = 0; ch < nch; ++ch) {
            const u32 c0 = ch * CH, c1 = min(S, c0 + CH);
            __syncthreads();
            stage_union<T, 3, FT, STAGE_B<T>>(src, dst, id, ul, us, nu, c0, c1);
            __syncthreads();
            invert_h(c1 - c0);
            __syncthreads();
            entries_tile(my, e1, j, c0, c1, w32, pair);
        }
    }
    // first half + second half, in that order
    if constexpr (SPLIT > 1) {
        if (half) {
            s_half[0][lt] = ax; s_half[1][lt] = ay; s_half[2][lt] = az;
            s_half[3][lt] = du; s_half[4][lt] = lam; s_half[5][lt] = vmax;
        }
        __syncthreads();
        if (!half) {
            ax += s_half[0][lt]; ay += s_half[1][lt]; az += s_half[2][lt];
            du += s_half[3][lt]; lam += s_half[4][lt];
            vmax = vmax > s_half[5][lt] ? vmax : s_half[5][lt];
        }
    }
    if (cv.work) {   // work counters (profiling): visited entries, interacting pairs
        const u64 t1 = block_reduce<FT>((u64)(e1 - e0), s_w, [](u64 x, u64 y) { return x + y; });
        const u64 t2 = block_reduce<FT>((u64)inter, s_w, [](u64 x, u64 y) { return x + y; });
        if (threadIdx.x == 0) {
            atomicAdd((unsigned long long*)&cv.work[2 * (g & 63)], (unsigned long long)t1);
            atomicAdd((unsigned long long*)&cv.work[2 * (g & 63) + 1], (unsigned long long)t2);
        }
    }
    float dta = __int_as_float(0x7f800000);
    if (live && !half) {
        acc[a] = mk4<T>(ax, ay, az, du + lam);
        if (vsig_out) vsig_out[a] = vmax;
        const T am = sqrt(ax * ax + ay * ay + az * az);
        const T t1 = vmax > T(0) ? (T)P.c_cour * ha / vmax : T(INFINITY);
        const T t2 = am > T(0) ? (T)P.c_force * sqrt(ha / am) : T(INFINITY);
        dta = (float)(t1 < t2 ? t1 : t2);
    }
    if (block_uniform(k, s_k)) {
        const float bmin = block_reduce<FT>(dta, s_red, [](float x, float y) { return x < y ? x : y; });
        if (threadIdx.x == 0) atomic_min_if(&stat[k].dt_bits, __float_as_uint(bmin));
    } else if (live && !half) {
        atomic_min_if(&stat[k].dt_bits, __float_as_uint(dta));
    }
}

template <class T, int CH, int K, int SPLIT>
__device__ __attribute__((always_inline)) inline void force_group(const i64 g, const ForceArgs<T>& A,
                                                                  ForceShared<T, CH, SPLIT>& sh)
{
    force_group<T, CH, K, SPLIT>(g, A.posh, A.velu, A.thermo, A.id, A.gm, A.inst, A.P, A.cv, A.acc,
                                 A.vsig_out, A.stat, sh);
}

template <class T, int CH, int K, int SPLIT>
__global__ void __launch_bounds__(SPLIT * GROUP)
k_force(const vec4<T>* __restrict__ posh, const vec4<T>* __restrict__ velu,
        const vec4<T>* __restrict__ thermo, const u32* __restrict__ id, const GroupMap gm,
        const InstDev* __restrict__ inst, SphParams P, CacheView cv, vec4<T>* __restrict__ acc,
        T* __restrict__ vsig_out, InstStat* __restrict__ stat)
{
    __shared__ ForceShared<T, CH, SPLIT> sh;
    force_group<T, CH, K, SPLIT>(blockIdx.x, posh, velu, thermo, id, gm, inst, P, cv, acc, vsig_out,
                                 stat, sh);
}

// ---------------------------------------------------------------------------
// Shock detector and viscosity switch (App. G, Shock detection), after the
// density pass of a step, before the force:
//   grad v* and grad a^n by the SPH estimate
//     (d_j f_i)_a = -m/(rho_a Omega_a) sum_b (f_a - f_b)_i rhat_j F_ab(h_a),
//   div v, curl v, d(div v)/dt = div a - sum_ij (d_j v_i)(d_i v_j),
//   xi = (div v)^2 / ((div v)^2 + |curl v|^2), A = xi max(-d(div v)/dt, 0),
//   alpha_loc = max(alpha_min, alpha_max 10 h^2 A / (10 h^2 A + c^2)),
//   tau = h / (sigma_decay c), and the implicit update
//   alpha^{n+1} = max((alpha^n + alpha_loc dt/tau) / (1 + dt/tau), alpha_loc).
// alpha (key order) is updated in place and alpha c staged in thermo.z for
// the force.  One workgroup per group, the union's positions, v* and a^n
// staged in LDS.
// ---------------------------------------------------------------------------
template <class T, int CH, int K>
__global__ void __launch_bounds__(GROUP)
k_alpha(const vec4<T>* __restrict__ posh, const vec4<T>* __restrict__ velu,
        const vec4<T>* __restrict__ acc_n, const T* __restrict__ omega,
        const u32* __restrict__ id, const GroupMap gm, const InstDev* __restrict__ inst,
        SphParams P, CacheView cv, const double* __restrict__ dt_inst, T* __restrict__ alpha,
        vec4<T>* __restrict__ thermo)
{
    __shared__ vec4<T> s_pos[CH];
    __shared__ vec4<T> s_vel[CH];
    __shared__ vec4<T> s_acc[CH];
    const i64 g = blockIdx.x;
    i64 beg, end;
    int k;
    gm.range(g, beg, end, k);
    const InstDev in = inst[k];
    const Box<T> bx = make_box<T>(in);
    const i64 a = beg + threadIdx.x;
    const bool live = a < end;
    const i64 ai = live ? a : beg;
    const vec4<T> pa = posh[ai], va = velu[ai], aa = acc_n[ai];
    const T RK = Kern<K>::template R<T>(), CK = Kern<K>::template C<T>();
    const T ha = pa.w, hia = T(1) / ha;
    const T hia4 = hia * hia * hia * hia * CK;
    const u32 cnt = live ? cv.ncnt[a] : 0u;
    const u32 nu = min((u32)cv.cap, cv.ucnt[g]);
    const u32 S = cv.ustot[g];
    const u32 nch = (S + CH - 1) / CH;
    const u32* ul = cv.uleaf + g * cv.cap;
    const u32* us = cv.uslot + g * cv.cap;
    const u64* my = cv.nlist + cv.gbase[g] * GROUP + threadIdx.x;
    const vec4<T>* src[3] = { posh, velu, acc_n };
    vec4<T>* dst[3] = { s_pos, s_vel, s_acc };
    T gv[9], ga[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) { gv[t] = T(0); ga[t] = T(0); }
    const bool wrap = !group_interior<T>(((const vec4<T>*)cv.glo)[g], ((const vec4<T>*)cv.ghi)[g],
                                         ((const vec4<T>*)cv.blo)[cv.root[k]].w, (T)cv.rk, bx);
    auto pair_d = [&](u32 sl, T dx, T dy, T dz) {
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 > T(0)) || !(r2 * hia * hia < RK * RK)) return;
        const T rinv = fast_rsq(r2);
        const T Fr = Kern<K>::template df<T>(r2 * rinv * hia) * hia4 * rinv;   // F / r
        const T ex = dx * Fr, ey = dy * Fr, ez = dz * Fr;                    // rhat F
        const vec4<T> vb = s_vel[sl], ab = s_acc[sl];
        const T d[3] = { va.x - vb.x, va.y - vb.y, va.z - vb.z };
        const T e[3] = { aa.x - ab.x, aa.y - ab.y, aa.z - ab.z };
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            gv[3 * i + 0] += d[i] * ex; gv[3 * i + 1] += d[i] * ey; gv[3 * i + 2] += d[i] * ez;
            ga[3 * i + 0] += e[i] * ex; ga[3 * i + 1] += e[i] * ey; ga[3 * i + 2] += e[i] * ez;
        }
    };
    auto pair = [&](u32 sl) {
        const vec4<T> pb = s_pos[sl];
        pair_d(sl, min_image(pa.x - pb.x, bx.L[0], bx.halfL[0], bx.periodic),
               min_image(pa.y - pb.y, bx.L[1], bx.halfL[1], bx.periodic),
               min_image(pa.z - pb.z, bx.L[2], bx.halfL[2], bx.periodic));
    };
    auto pair_in = [&](u32 sl) {
        const vec4<T> pb = s_pos[sl];
        pair_d(sl, pa.x - pb.x, pa.y - pb.y, pa.z - pb.z);
    };
    if (nch == 1) {
        stage_union<T, 3>(src, dst, id, ul, us, nu, 0u, S);
        __syncthreads();
        if (live) {
            if (wrap) entries_each(my, cnt, pair);
            else entries_each(my, cnt, pair_in);
        }
    } else {
        u32 j = 0;
        for (u32 ch = 0; ch < nch; ++ch) {
            const u32 c0 = ch * CH, c1 = min(S, c0 + CH);
            __syncthreads();
            stage_union<T, 3>(src, dst, id, ul, us, nu, c0, c1);
            __syncthreads();
            if (live) entries_tile(my, cnt, j, c0, c1, slots_wide(S), pair);
        }
    }
    if (!live) return;
    const T m = (T)in.mass;
    const T hf = (T)P.hfact * hia;
    const T rho = m * hf * hf * hf;
    const T sc = -m / (rho * omega[a]);
#pragma unroll
    for (int t = 0; t < 9; ++t) { gv[t] *= sc; ga[t] *= sc; }
    const T divv = gv[0] + gv[4] + gv[8];
    const T diva = ga[0] + ga[4] + ga[8];
    const T cx = gv[7] - gv[5], cy = gv[2] - gv[6], cz = gv[3] - gv[1];
    T vv = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) vv += gv[3 * i + j] * gv[3 * j + i];
    const T ddiv = diva - vv;
    const T d2 = divv * divv, c2 = cx * cx + cy * cy + cz * cz;
    const T xi = (d2 + c2 > T(0)) ? d2 / (d2 + c2) : T(0);
    const T Ash = xi * (ddiv < T(0) ? -ddiv : T(0));
    const T gam = (T)P.gamma;
    const T cs = sqrt(gam * (gam - T(1)) * va.w);
    const T hh = T(10) * ha * ha * Ash;
    T aloc = (hh + cs * cs > T(0)) ? (T)P.alpha_max * hh / (hh + cs * cs) : T(0);
    aloc = aloc < (T)P.alpha_min ? (T)P.alpha_min : aloc;
    const T an = alpha[a];
    T al;
    if (cs > T(0)) {
        const T x = (T)dt_inst[k] * (T)P.sigma_decay * cs * hia;     // dt / tau
        al = (an + aloc * x) / (T(1) + x);
        al = al < aloc ? aloc : al;
    } else {
        al = an > aloc ? an : aloc;
    }
    alpha[a] = al;
    thermo[a].z = al * cs;
}

// ---------------------------------------------------------------------------
// Leapfrog corrector (App. G.1): v^{n+1} = v^{n+1/2} + dt/2 a^{n+1}
// (= v* + dt/2 (a^{n+1} - a^n)), same for u.  Writes the new state into the
// caller's arrays at the particle's key-order position and reduces
// max|dv|, sum|dv|^2 and sum|v|^2 per instance for the reversibility check.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(GROUP)
k_correct(const vec4<T>* __restrict__ posh, const vec4<T>* __restrict__ velu,
          const vec4<T>* __restrict__ vhalf, const vec4<T>* __restrict__ acc,
          const T* __restrict__ omega, const u32* __restrict__ pid, i64 n,
          const i64* __restrict__ p_off, int ninst, const InstDev* __restrict__ inst,
          const double* __restrict__ dt_inst, double hfact, OutPtrs<T> o,
          InstStat* __restrict__ stat, BlockPart* __restrict__ part, const u32* __restrict__ skip)
{
    __shared__ double s_red[GROUP / WAVE];
    __shared__ float s_redf[GROUP / WAVE];
    __shared__ int s_k;
    if (skip && *skip) return;
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    const i64 ii = live ? i : n - 1;
    const int k = find_seg(p_off, ninst, ii);
    const T hdt = (T)(0.5 * dt_inst[k]);
    const vec4<T> p = posh[ii], vs = velu[ii], vh = vhalf[ii], a = acc[ii];
    const T vx = vh.x + hdt * a.x, vy = vh.y + hdt * a.y, vz = vh.z + hdt * a.z;
    const T u = vh.w + hdt * a.w;
    const T dvx = vx - vs.x, dvy = vy - vs.y, dvz = vz - vs.z;
    float dv = 0.f;
    double dv2 = 0.0, v2 = 0.0;
    if (live) {
        const i64 c = i + inst[k].shift;
        o.x[c] = p.x; o.y[c] = p.y; o.z[c] = p.z; o.h[c] = p.w;
        o.vx[c] = vx; o.vy[c] = vy; o.vz[c] = vz; o.u[c] = u;
        o.ax[c] = a.x; o.ay[c] = a.y; o.az[c] = a.z; o.du[c] = a.w;
        if (o.pid) o.pid[c] = pid[i];
        if (o.omega) o.omega[c] = omega[i];
        if (o.rho) {
            const double hf = hfact / (double)p.w;
            o.rho[c] = (T)(inst[k].mass * hf * hf * hf);
        }
        dv2 = (double)dvx * dvx + (double)dvy * dvy + (double)dvz * dvz;
        dv = (float)sqrt(dv2);
        v2 = (double)vx * vx + (double)vy * vy + (double)vz * vz;
    }
    // one partial per block (no atomics); blocks spanning two instances add
    // their lanes directly (rare: only at instance boundaries)
    const int slot = blockIdx.x % STAT_SLOTS;
    if (block_uniform(k, &s_k)) {
        const float mx = block_max<float>(dv, s_redf);
        const double s1 = block_sum<double>(dv2, s_red);
        const double s2 = block_sum<double>(v2, s_red);
        if (threadIdx.x == 0) {
            atomic_max_if(&stat[k].dvmax_bits, __float_as_uint(mx));
            BlockPart bp;
            bp.inst = k;
            bp.dv2 = s1;
            bp.v2 = s2;
            part[blockIdx.x] = bp;
        }
    } else {
        if (live) {
            atomic_max_if(&stat[k].dvmax_bits, __float_as_uint(dv));
            atomicAdd(&stat[k].dv2_part[slot], dv2);
            atomicAdd(&stat[k].v2_part[slot], v2);
        }
        if (threadIdx.x == 0) {
            BlockPart bp;
            bp.inst = -1;
            bp.dv2 = 0.0;
            bp.v2 = 0.0;
            part[blockIdx.x] = bp;
        }
    }
}

// Fold the per-block partials of the corrector into the instance stats
// (one workgroup per instance).
__global__ void __launch_bounds__(GROUP)
k_fold_parts(const BlockPart* __restrict__ part, i64 nblocks, InstStat* __restrict__ stat,
             const u32* __restrict__ skip)
{
    __shared__ double s_red[GROUP / WAVE];
    if (skip && *skip) return;
    const int k = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (i64 i = threadIdx.x; i < nblocks; i += GROUP) {
        const BlockPart p = part[i];
        if (p.inst == k) { a += p.dv2; b += p.v2; }
    }
    a = block_sum<double>(a, s_red);
    b = block_sum<double>(b, s_red);
    if (threadIdx.x == 0) {
        stat[k].dv2_part[0] += a;
        stat[k].v2_part[0] += b;
    }
}

// Pressure terms for the force from h, Omega and u* (key order):
// thermo = (P/(rho^2 Om), 1/(2 rho Om), alpha c_s, P), P = (gamma-1) rho u,
// c_s = sqrt(gamma (gamma-1) u), rho = m (hfact/h)^3.
template <class T>
__global__ void k_thermo(const vec4<T>* __restrict__ posh, const vec4<T>* __restrict__ velu,
                         const T* __restrict__ omega, i64 n, const i64* __restrict__ p_off,
                         int ninst, const InstDev* __restrict__ inst, double hfact, double gamma,
                         double alpha, const T* __restrict__ alpha_s, vec4<T>* __restrict__ thermo,
                         const u32* __restrict__ skip)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (skip && *skip)) return;
    const int k = find_seg(p_off, ninst, i);
    const T hf = (T)hfact / posh[i].w;
    const T rho = (T)inst[k].mass * hf * hf * hf;
    const T om = omega[i], u = velu[i].w, g = (T)gamma;
    const T Pr = (g - T(1)) * rho * u;
    const T B = T(1) / (rho * om);
    const T al = alpha_s ? alpha_s[i] : (T)alpha;
    thermo[i] = mk4<T>(Pr * B / rho, T(0.5) * B, al * sqrt(g * (g - T(1)) * u), Pr);
}

// Corrector re-run (App. G.1): v* <- v^{n+1}, u* <- u^{n+1} for the particles
// of the instances flagged in `redo`, read back from the step's outputs
// (key order, at i + shift).
template <class T>
__global__ void k_velu_from_out(OutPtrs<T> o, i64 n, const i64* __restrict__ p_off, int ninst,
                                const InstDev* __restrict__ inst, const u8* __restrict__ redo,
                                vec4<T>* __restrict__ velu)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = find_seg(p_off, ninst, i);
    if (!redo[k]) return;
    const i64 c = i + inst[k].shift;
    velu[i] = mk4<T>(o.vx[c], o.vy[c], o.vz[c], o.u[c]);
}

// Gather v, u into key order for a derivative evaluation outside a step.
template <class T>
__global__ void k_gather_velu(const u32* __restrict__ eps, i64 n, const T* vx, const T* vy,
                              const T* vz, const T* u, vec4<T>* __restrict__ velu)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 j = eps[i];
    velu[i] = mk4<T>(vx[j], vy[j], vz[j], u ? u[j] : T(0));
}

// Scatter a key-order quantity back to caller order: dst[eps[i]] = src[i].
template <class T>
__global__ void k_scatter(const u32* __restrict__ eps, i64 n, const vec4<T>* __restrict__ src4,
                          int comp, const T* __restrict__ src1, T* __restrict__ dst)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T v;
    if (src4) {
        const vec4<T> s = src4[i];
        v = comp == 0 ? s.x : comp == 1 ? s.y : comp == 2 ? s.z : s.w;
    } else {
        v = src1[i];
    }
    dst[eps[i]] = v;
}

template <class T>
__global__ void k_scatter_rho(const u32* __restrict__ eps, i64 n, const vec4<T>* __restrict__ posh,
                              const i64* __restrict__ p_off, int ninst,
                              const InstDev* __restrict__ inst, double hfact, T* __restrict__ dst)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = find_seg(p_off, ninst, i);
    const T hf = (T)hfact / posh[i].w;
    dst[eps[i]] = (T)inst[k].mass * hf * hf * hf;
}

// ------------------------------------------------------------ launchers ----
void launch_fill_u32(u32* p, i64 n, u32 v, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, grid_for(n, 256), dim3(256), 0, st, p, n, v);
}

void launch_iota_u32(u32* p, i64 n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_iota_u32, grid_for(n, 256), dim3(256), 0, st, p, n);
}

void launch_stat_reset(InstStat* s, int ninst, int what, const u8* redo, hipStream_t st,
                       const u32* skip)
{
    hipLaunchKernelGGL(k_stat_reset, grid_for(ninst, 64), dim3(64), 0, st, s, ninst, what, redo,
                       skip);
}

template <class T>
void launch_root_hmax(const vec4<T>* blo, const u32* root, int ninst, double* out, hipStream_t st)
{
    hipLaunchKernelGGL((k_root_hmax<T>), grid_for(ninst, 64), dim3(64), 0, st, blo, root, ninst, out);
}

void launch_gate_build(const u32* flags, u32 mask0, int w_sort, int w_leaves, const double* rhmax,
                       const InstDev* inst, int ninst, double rk, u32* gs, u8* gate, u32* reruns,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_gate_build, dim3(1), dim3(256), 0, st, flags, mask0, w_sort, w_leaves, rhmax,
                       inst, ninst, rk, gs, gate, reruns);
}

void launch_gate_density(const InstStat* stat, int ninst, u32* gs, u8* gate, hipStream_t st)
{
    hipLaunchKernelGGL(k_gate_density, dim3(1), dim3(256), 0, st, stat, ninst, gs, gate);
}

__global__ void k_flag_and(u32* f, u32 mask) { f[0] &= mask; }

void launch_flag_and(u32* f, u32 mask, hipStream_t st)
{
    hipLaunchKernelGGL(k_flag_and, dim3(1), dim3(1), 0, st, f, mask);
}

void launch_gate_exceed(const InstStat* stat, int ninst, const u32* gs, u32* skw, u8* rx,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_gate_exceed, dim3(1), dim3(256), 0, st, stat, ninst, gs, skw, rx);
}

void launch_gate_round(const u32* flags, u32 mask0, const double* rhmax, const InstDev* inst,
                       int ninst, double rk, const u32* skw, u32* gs, u8* rx, hipStream_t st)
{
    hipLaunchKernelGGL(k_gate_round, dim3(1), dim3(256), 0, st, flags, mask0, rhmax, inst, ninst, rk,
                       skw, gs, rx);
}

void launch_rerun_decide(const InstStat* stat, const i64* p_off, int ninst, double eps_v,
                         int max_reruns, int r, u32* gs, u8* redo, u32* reruns, hipStream_t st)
{
    hipLaunchKernelGGL(k_rerun_decide, dim3(1), dim3(256), 0, st, stat, p_off, ninst, eps_v,
                       max_reruns, r, gs, redo, reruns);
}

void launch_dt_select(double* dt_inst, const InstStat* s, const double* dt_host, int ninst,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_dt_select, grid_for(ninst, 64), dim3(64), 0, st, dt_inst, s, dt_host, ninst);
}

template <class T> void launch_copy_h(const vec4<T>* posh, T* hc, i64 n, hipStream_t st, const u32* skip)
{
    if (n > 0) hipLaunchKernelGGL((k_copy_h<T>), grid_for(n, 256), dim3(256), 0, st, posh, hc, n, skip);
}

// Union slots staged per LDS chunk.  FP32 density: 1256 slots keep a
// workgroup's LDS within an eighth of the CU's 160 KiB, so the LDS and its
// registers (held to 64 VGPRs) both allow eight waves per SIMD (larger
// unions take several chunks, restaged on every Newton pass: the occupancy
// pays for that on the Sedov and lattice workloads).  FP64 density is
// FP64-ALU bound: a chunk small enough for a fifth workgroup per CU was no
// faster.  FP32 force needs its union in one chunk (multi-chunk force is
// twice as slow), which caps it at two workgroups per CU.
constexpr int DENS_CH_F = 1256, DENS_CH_D = 1024;
static_assert(sizeof(DensShared<float, DENS_CH_F>) <= 160 * 1024 / 8,
              "FP32 density LDS must allow eight workgroups per CU");
constexpr int FORCE_CH_F = 1536, FORCE_CH_D = 640;

template <class T, int K>
void launch_density_k(const SortedPtrs<T>& s, const u32* id, const GroupMap& gm, i64 ngroups,
                      const InstDev* inst, const SphParams& P, const CacheView& cv, T* omega,
                      vec4<T>* thermo, u8* status, InstStat* stat, const u8* redo, hipStream_t st)
{
    if (sizeof(T) == 4)
        hipLaunchKernelGGL((k_density<T, DENS_CH_F, K>), dim3((unsigned)ngroups), dim3(GROUP), 0, st,
                           s.posh, s.hn, s.hcache, s.velu, id, gm, inst, P, cv, omega, thermo,
                           status, stat, redo);
    else
        hipLaunchKernelGGL((k_density<T, DENS_CH_D, K>), dim3((unsigned)ngroups), dim3(GROUP), 0, st,
                           s.posh, s.hn, s.hcache, s.velu, id, gm, inst, P, cv, omega, thermo,
                           status, stat, redo);
}

template <class T>
void launch_density(const SortedPtrs<T>& s, const u32* id, const GroupMap& gm, i64 ngroups,
                    const InstDev* inst, const SphParams& P, const CacheView& cv, T* omega,
                    vec4<T>* thermo, u8* status, InstStat* stat, const u8* redo, hipStream_t st)
{
    if (ngroups <= 0) return;
    switch (P.kernel) {
    case KM5: launch_density_k<T, KM5>(s, id, gm, ngroups, inst, P, cv, omega, thermo, status, stat, redo, st); break;
    case KM6: launch_density_k<T, KM6>(s, id, gm, ngroups, inst, P, cv, omega, thermo, status, stat, redo, st); break;
    case KC2: launch_density_k<T, KC2>(s, id, gm, ngroups, inst, P, cv, omega, thermo, status, stat, redo, st); break;
    case KC4: launch_density_k<T, KC4>(s, id, gm, ngroups, inst, P, cv, omega, thermo, status, stat, redo, st); break;
    case KC6: launch_density_k<T, KC6>(s, id, gm, ngroups, inst, P, cv, omega, thermo, status, stat, redo, st); break;
    default:  launch_density_k<T, KM4>(s, id, gm, ngroups, inst, P, cv, omega, thermo, status, stat, redo, st); break;
    }
}

template <class T, int K, int SPLIT>
void launch_force_s(const SortedPtrs<T>& s, const vec4<T>* thermo, const u32* id, const GroupMap& gm,
                    i64 ngroups, const InstDev* inst, const SphParams& P, const CacheView& cv,
                    vec4<T>* acc, T* vsig, InstStat* stat, hipStream_t st)
{
    if (sizeof(T) == 4)
        hipLaunchKernelGGL((k_force<T, FORCE_CH_F, K, SPLIT>), dim3((unsigned)ngroups),
                           dim3(SPLIT * GROUP), 0, st, s.posh, s.velu, thermo, id, gm, inst, P, cv,
                           acc, vsig, stat);
    else
        hipLaunchKernelGGL((k_force<T, FORCE_CH_D, K, SPLIT>), dim3((unsigned)ngroups),
                           dim3(SPLIT * GROUP), 0, st, s.posh, s.velu, thermo, id, gm, inst, P, cv,
                           acc, vsig, stat);
}

template <class T, int K>
void launch_force_k(const SortedPtrs<T>& s, const vec4<T>* thermo, const u32* id, const GroupMap& gm,
                    i64 ngroups, const InstDev* inst, const SphParams& P, const CacheView& cv,
                    vec4<T>* acc, T* vsig, InstStat* stat, hipStream_t st)
{
    if (P.force_split == 1)
        launch_force_s<T, K, 1>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st);
    else
        launch_force_s<T, K, 2>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st);
}

// Density and force in one persistent launch: the workgroups (as many as
// the device holds at once, launched cooperatively) take the groups
// g = blockIdx.x, + gridDim.x, ... through the h iteration; the grid then
// synchronises (every h, rho, Omega and pressure term written and visible to
// all workgroups), and unless some particle left chi h_cache (its instance's
// cache must be rebuilt first: the caller then runs the separate passes) the
// same workgroups take the groups through the force, one thread per
// particle.  The LDS of the two passes is shared.
template <class T, int DCH, int FCH, int K>
__global__ void __launch_bounds__(GROUP)
k_density_force(const DensArgs<T> D, const ForceArgs<T> F, i64 ngroups, int ninst)
{
    constexpr size_t DB = sizeof(DensShared<T, DCH>), FB = sizeof(ForceShared<T, FCH, 1>);
    __shared__ __align__(16) unsigned char buf[DB > FB ? DB : FB];
    auto& ds = *reinterpret_cast<DensShared<T, DCH>*>(buf);
    auto& fs = *reinterpret_cast<ForceShared<T, FCH, 1>*>(buf);
    for (i64 g = blockIdx.x; g < ngroups; g += gridDim.x) {
        __syncthreads();
        density_group<T, DCH, K>(g, D, ds);
    }
    cooperative_groups::this_grid().sync();
    bool exceed = false;
    for (int k = threadIdx.x; k < ninst; k += GROUP) exceed |= D.stat[k].n_exceed != 0u;
    if (__syncthreads_or(exceed)) return;
    for (i64 g = blockIdx.x; g < ngroups; g += gridDim.x) {
        __syncthreads();
        force_group<T, FCH, K, 1>(g, F, fs);
    }
}

template <class T, int K>
int launch_density_force_k(const DensArgs<T>& D, const ForceArgs<T>& F, i64 ngroups, int ninst,
                           hipStream_t st)
{
    const void* kern = sizeof(T) == 4
        ? (const void*)&k_density_force<T, DENS_CH_F, FORCE_CH_F, K>
        : (const void*)&k_density_force<T, DENS_CH_D, FORCE_CH_D, K>;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, GROUP, 0) != hipSuccess || per < 1)
        return -1;
    const i64 nb = std::min<i64>(ngroups, (i64)per * cus);
    DensArgs<T> d = D;
    ForceArgs<T> f = F;
    void* args[] = { &d, &f, &ngroups, &ninst };
    return hipLaunchCooperativeKernel(kern, dim3((unsigned)nb), dim3(GROUP), args, 0, st) == hipSuccess ? 0 : -1;
}

template <class T>
int launch_density_force(const SortedPtrs<T>& s, const vec4<T>* thermo, const u32* id,
                         const GroupMap& gm, i64 ngroups, int ninst, const InstDev* inst,
                         const SphParams& P, const CacheView& cvd, const CacheView& cvf, T* omega,
                         u8* status, InstStat* stat, vec4<T>* acc, T* vsig, hipStream_t st)
{
    if (ngroups <= 0) return 0;
    const DensArgs<T> D{s.posh, s.hn, s.hcache, s.velu, id, gm, inst, P, cvd, omega,
                        const_cast<vec4<T>*>(thermo), status, stat, nullptr};
    const ForceArgs<T> F{s.posh, s.velu, thermo, id, gm, inst, P, cvf, acc, vsig, stat};
    switch (P.kernel) {
    case KM5: return launch_density_force_k<T, KM5>(D, F, ngroups, ninst, st);
    case KM6: return launch_density_force_k<T, KM6>(D, F, ngroups, ninst, st);
    case KC2: return launch_density_force_k<T, KC2>(D, F, ngroups, ninst, st);
    case KC4: return launch_density_force_k<T, KC4>(D, F, ngroups, ninst, st);
    case KC6: return launch_density_force_k<T, KC6>(D, F, ngroups, ninst, st);
    default:  return launch_density_force_k<T, KM4>(D, F, ngroups, ninst, st);
    }
}

template <class T>
void launch_force(const SortedPtrs<T>& s, const vec4<T>* thermo, const u32* id, const GroupMap& gm,
                  i64 ngroups, const InstDev* inst, const SphParams& P, const CacheView& cv,
                  vec4<T>* acc, T* vsig, InstStat* stat, hipStream_t st)
{
    if (ngroups <= 0) return;
    switch (P.kernel) {
    case KM5: launch_force_k<T, KM5>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st); break;
    case KM6: launch_force_k<T, KM6>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st); break;
    case KC2: launch_force_k<T, KC2>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st); break;
    case KC4: launch_force_k<T, KC4>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st); break;
    case KC6: launch_force_k<T, KC6>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st); break;
    default:  launch_force_k<T, KM4>(s, thermo, id, gm, ngroups, inst, P, cv, acc, vsig, stat, st); break;
    }
}

constexpr int ALPHA_CH_F = 1280, ALPHA_CH_D = 640;

template <class T, int K>
void launch_alpha_k(const SortedPtrs<T>& s, const vec4<T>* acc_n, const T* omega, const u32* id,
                    const GroupMap& gm, i64 ngroups, const InstDev* inst, const SphParams& P,
                    const CacheView& cv, const double* dt_inst, T* alpha, vec4<T>* thermo,
                    hipStream_t st)
{
    if (sizeof(T) == 4)
        hipLaunchKernelGGL((k_alpha<T, ALPHA_CH_F, K>), dim3((unsigned)ngroups), dim3(GROUP), 0, st,
                           s.posh, s.velu, acc_n, omega, id, gm, inst, P, cv, dt_inst, alpha, thermo);
    else
        hipLaunchKernelGGL((k_alpha<T, ALPHA_CH_D, K>), dim3((unsigned)ngroups), dim3(GROUP), 0, st,
                           s.posh, s.velu, acc_n, omega, id, gm, inst, P, cv, dt_inst, alpha, thermo);
}

template <class T>
void launch_alpha(const SortedPtrs<T>& s, const vec4<T>* acc_n, const T* omega, const u32* id,
                  const GroupMap& gm, i64 ngroups, const InstDev* inst, const SphParams& P,
                  const CacheView& cv, const double* dt_inst, T* alpha, vec4<T>* thermo,
                  hipStream_t st)
{
    if (ngroups <= 0) return;
    switch (P.kernel) {
    case KM5: launch_alpha_k<T, KM5>(s, acc_n, omega, id, gm, ngroups, inst, P, cv, dt_inst, alpha, thermo, st); break;
    case KM6: launch_alpha_k<T, KM6>(s, acc_n, omega, id, gm, ngroups, inst, P, cv, dt_inst, alpha, thermo, st); break;
    case KC2: launch_alpha_k<T, KC2>(s, acc_n, omega, id, gm, ngroups, inst, P, cv, dt_inst, alpha, thermo, st); break;
    case KC4: launch_alpha_k<T, KC4>(s, acc_n, omega, id, gm, ngroups, inst, P, cv, dt_inst, alpha, thermo, st); break;
    case KC6: launch_alpha_k<T, KC6>(s, acc_n, omega, id, gm, ngroups, inst, P, cv, dt_inst, alpha, thermo, st); break;
    default:  launch_alpha_k<T, KM4>(s, acc_n, omega, id, gm, ngroups, inst, P, cv, dt_inst, alpha, thermo, st); break;
    }
}

// Gather a key-order copy of one caller array: dst[i] = src[eps[i]].
template <class T>
__global__ void k_gather1(const u32* __restrict__ eps, i64 n, const T* __restrict__ src,
                          T* __restrict__ dst)
{
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[eps[i]];
}

template <class T> void launch_gather1(const u32* eps, i64 n, const T* src, T* dst, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL((k_gather1<T>), grid_for(n, 256), dim3(256), 0, st, eps, n, src, dst);
}

template <class T>
void launch_correct(const SortedPtrs<T>& s, const vec4<T>* acc, const T* omega, i64 n,
                    const i64* p_off, int ninst, const InstDev* inst, const double* dt_inst,
                    double hfact, const OutPtrs<T>& o, InstStat* stat, BlockPart* part,
                    hipStream_t st, const u32* skip)
{
    if (n <= 0) return;
    const i64 nb = (n + GROUP - 1) / GROUP;
    hipLaunchKernelGGL((k_correct<T>), dim3((unsigned)nb), dim3(GROUP), 0, st, s.posh, s.velu,
                       s.vhalf, acc, omega, s.pid, n, p_off, ninst, inst, dt_inst, hfact, o, stat,
                       part, skip);
}

void launch_fold_parts(const BlockPart* part, i64 nblocks, int ninst, InstStat* stat, hipStream_t st,
                       const u32* skip)
{
    if (nblocks > 0)
        hipLaunchKernelGGL(k_fold_parts, dim3((unsigned)ninst), dim3(GROUP), 0, st, part, nblocks, stat,
                           skip);
}

template <class T>
void launch_gather_velu(const u32* eps, i64 n, const T* vx, const T* vy, const T* vz, const T* u,
                        vec4<T>* velu, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL((k_gather_velu<T>), grid_for(n, 256), dim3(256), 0, st, eps, n, vx, vy,
                           vz, u, velu);
}

template <class T>
void launch_velu_from_out(const OutPtrs<T>& o, i64 n, const i64* p_off, int ninst,
                          const InstDev* inst, const u8* redo, vec4<T>* velu, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL((k_velu_from_out<T>), grid_for(n, 256), dim3(256), 0, st, o, n, p_off,
                           ninst, inst, redo, velu);
}

template <class T>
void launch_thermo(const vec4<T>* posh, const vec4<T>* velu, const T* omega, i64 n,
                   const i64* p_off, int ninst, const InstDev* inst, double hfact, double gamma,
                   double alpha, const T* alpha_s, vec4<T>* thermo, hipStream_t st,
                   const u32* skip)
{
    if (n > 0)
        hipLaunchKernelGGL((k_thermo<T>), grid_for(n, 256), dim3(256), 0, st, posh, velu, omega, n,
                           p_off, ninst, inst, hfact, gamma, alpha, alpha_s, thermo, skip);
}

template <class T>
void launch_scatter(const u32* eps, i64 n, const vec4<T>* src4, int comp, const T* src1, T* dst,
                    hipStream_t st)
{
    if (n > 0 && dst)
        hipLaunchKernelGGL((k_scatter<T>), grid_for(n, 256), dim3(256), 0, st, eps, n, src4, comp,
                           src1, dst);
}

template <class T>
void launch_scatter_rho(const u32* eps, i64 n, const vec4<T>* posh, const i64* p_off, int ninst,
                        const InstDev* inst, double hfact, T* dst, hipStream_t st)
{
    if (n > 0 && dst)
        hipLaunchKernelGGL((k_scatter_rho<T>), grid_for(n, 256), dim3(256), 0, st, eps, n, posh,
                           p_off, ninst, inst, hfact, dst);
}

#define INST(T)                                                                                   \
    template void launch_copy_h<T>(const vec4<T>*, T*, i64, hipStream_t, const u32*);             \
    template void launch_density<T>(const SortedPtrs<T>&, const u32*, const GroupMap&, i64,       \
                                    const InstDev*, const SphParams&, const CacheView&, T*,       \
                                    vec4<T>*, u8*, InstStat*, const u8*, hipStream_t);             \
    template void launch_root_hmax<T>(const vec4<T>*, const u32*, int, double*, hipStream_t);     \
    template int launch_density_force<T>(const SortedPtrs<T>&, const vec4<T>*, const u32*,        \
                                         const GroupMap&, i64, int, const InstDev*,              \
                                         const SphParams&, const CacheView&, const CacheView&,    \
                                         T*, u8*, InstStat*, vec4<T>*, T*, hipStream_t);          \
    template void launch_force<T>(const SortedPtrs<T>&, const vec4<T>*, const u32*,               \
                                  const GroupMap&, i64, const InstDev*, const SphParams&,         \
                                  const CacheView&, vec4<T>*, T*, InstStat*, hipStream_t);         \
    template void launch_correct<T>(const SortedPtrs<T>&, const vec4<T>*, const T*, i64,          \
                                    const i64*, int, const InstDev*, const double*, double,       \
                                    const OutPtrs<T>&, InstStat*, BlockPart*, hipStream_t,         \
                                    const u32*);                                                   \
    template void launch_gather_velu<T>(const u32*, i64, const T*, const T*, const T*, const T*,  \
                                        vec4<T>*, hipStream_t);                                   \
    template void launch_alpha<T>(const SortedPtrs<T>&, const vec4<T>*, const T*, const u32*,     \
                                  const GroupMap&, i64, const InstDev*, const SphParams&,         \
                                  const CacheView&, const double*, T*, vec4<T>*, hipStream_t);    \
    template void launch_gather1<T>(const u32*, i64, const T*, T*, hipStream_t);                  \
    template void launch_velu_from_out<T>(const OutPtrs<T>&, i64, const i64*, int,                \
                                          const InstDev*, const u8*, vec4<T>*, hipStream_t);      \
    template void launch_thermo<T>(const vec4<T>*, const vec4<T>*, const T*, i64, const i64*,     \
                                   int, const InstDev*, double, double, double, const T*,         \
                                   vec4<T>*, hipStream_t, const u32*);                            \
    template void launch_scatter<T>(const u32*, i64, const vec4<T>*, int, const T*, T*,           \
                                    hipStream_t);                                                 \
    template void launch_scatter_rho<T>(const u32*, i64, const vec4<T>*, const i64*, int,         \
                                        const InstDev*, double, T*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace shsph
