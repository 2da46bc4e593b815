// Two-stage neighbour cache (App. E.3-E.4, Alg. 4-6).
//
// Stage 1: one thread per leaf walks its instance's tree with a 64-entry
// stack kept in LDS (one column per lane, conflict free) and keeps the
// leaves that pass the group-group criterion
//     AABB_L  n  [AABB_C (+) R chi max(hmax_L, hmax_C)]  !=  0
// (App. F), with periodic images and a small outward inflation so that the
// prune is a superset of the exact particle test.  Children are pushed right
// then left, so leaves come out in ascending order.
// Stage 2: one thread per particle tests the particles of its leaf's
// neighbour leaves with the exact object-object criterion in the storage
// type, writing neighbours in ascending key order.  Both stages run a count
// pass, an exclusive scan and a fill pass (Alg. 5).
#include "common.hpp"
#include "kernels.hpp"

namespace shsph {

constexpr int STACK = 64;   // tree depth is bounded by the 63 key bits
constexpr int TRAV_BLOCK = 64;

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

template <class T, bool FILL>
__global__ void __launch_bounds__(TRAV_BLOCK)
k_leaf_neigh(const vec4<T>* __restrict__ blo, const vec4<T>* __restrict__ bhi,
             const u32* __restrict__ child, i64 n_internal, i64 n_leaf,
             const i64* __restrict__ leaf_off, int ninst, const u32* __restrict__ root,
             const InstDev* __restrict__ inst, T rk, const u64* __restrict__ off,
             u32* __restrict__ cnt, u32* __restrict__ list, u32* __restrict__ overflow)
{
    __shared__ u32 stack[STACK][TRAV_BLOCK];
    const int lane = threadIdx.x;
    const i64 g = (i64)blockIdx.x * TRAV_BLOCK + lane;
    if (g >= n_leaf) return;
    const int k = find_seg(leaf_off, ninst, g);
    const InstDev in = inst[k];
    const Box<T> bx = make_box<T>(in);
    T scale = fmax(fmax(fabs(bx.lo[0]), fabs(bx.hi[0])), fmax(fabs(bx.lo[1]), fabs(bx.hi[1])));
    scale = fmax(scale, fmax(fabs(bx.lo[2]), fabs(bx.hi[2])));
    scale = fmax(scale, fmax(bx.L[0], fmax(bx.L[1], bx.L[2])));
    const T eps_abs = Inflate<T>::abs * scale;
    const vec4<T> ql = blo[n_internal + g], qh = bhi[n_internal + g];
    u64 out = FILL ? off[g] : 0;
    const u64 out_end = FILL ? off[g + 1] : 0;
    const T onep = T(1) + Inflate<T>::rel;
    u32 count = 0;
    int sp = 0;
    stack[sp++][lane] = root[k];
    while (sp > 0) {
        const u32 node = stack[--sp][lane];
        const vec4<T> l = blo[node], h = bhi[node];
        const T r = add_rn(mul_rn(mul_rn(rk, fmax(ql.w, l.w)), onep), eps_abs);
        const bool hit = gap1<T>(ql.x, qh.x, l.x, h.x, bx.L[0], bx.periodic) <= r &&
                         gap1<T>(ql.y, qh.y, l.y, h.y, bx.L[1], bx.periodic) <= r &&
                         gap1<T>(ql.z, qh.z, l.z, h.z, bx.L[2], bx.periodic) <= r;
        if (!hit) continue;
        if (node >= n_internal) {
            if (FILL) {
                if (out < out_end) list[out++] = (u32)(node - n_internal);
                else { atomicOr(overflow, 2u); break; }
            } else {
                ++count;
            }
        } else {
            if (sp + 2 > STACK) { atomicOr(overflow, 1u); break; }
            stack[sp++][lane] = child[2 * node + 1];
            stack[sp++][lane] = child[2 * node];
        }
    }
    if (!FILL) cnt[g] = count;
}

template <class T, bool FILL>
__global__ void __launch_bounds__(256)
k_part_neigh(const vec4<T>* __restrict__ posh, const u32* __restrict__ xscan,
             const u32* __restrict__ id, const u64* __restrict__ loff, const u32* __restrict__ llist,
             i64 n, const i64* __restrict__ p_off, int ninst, const InstDev* __restrict__ inst,
             T rkc, u32* __restrict__ cnt, const u64* __restrict__ noff, u32* __restrict__ nlist,
             u32* __restrict__ overflow)
{
    const i64 a = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int k = find_seg(p_off, ninst, a);
    const Box<T> bx = make_box<T>(inst[k]);
    const u32 L = xscan[a + 1] - 1u;
    const vec4<T> pa = posh[a];
    u64 out = FILL ? noff[a] : 0;
    const u64 out_end = FILL ? noff[a + 1] : 0;
    u32 c = 0;
    const u64 j1 = loff[L + 1];
    for (u64 j = loff[L]; j < j1; ++j) {
        const u32 M = llist[j];
        const u32 b1 = id[M + 1];
        for (u32 b = id[M]; b < b1; ++b) {
            const vec4<T> pb = posh[b];
            if (cache_crit<T>(pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w, bx, rkc)) {
                if (FILL) {
                    if (out < out_end) nlist[out++] = b;
                    else atomicOr(overflow, 4u);
                } else {
                    ++c;
                }
            }
        }
    }
    if (!FILL) cnt[a] = c;
}

template <class T>
void launch_leaf_neigh(bool fill, const vec4<T>* blo, const vec4<T>* bhi, const u32* child,
                       i64 n_internal, i64 n_leaf, const i64* leaf_off, int ninst, const u32* root,
                       const InstDev* inst, double rk, const u64* off, u32* cnt, u32* list,
                       u32* overflow, hipStream_t st)
{
    if (n_leaf <= 0) return;
    const dim3 grid((unsigned)((n_leaf + TRAV_BLOCK - 1) / TRAV_BLOCK));
    if (fill)
        hipLaunchKernelGGL((k_leaf_neigh<T, true>), grid, dim3(TRAV_BLOCK), 0, st, blo, bhi, child,
                           n_internal, n_leaf, leaf_off, ninst, root, inst, (T)rk, off, cnt, list,
                           overflow);
    else
        hipLaunchKernelGGL((k_leaf_neigh<T, false>), grid, dim3(TRAV_BLOCK), 0, st, blo, bhi, child,
                           n_internal, n_leaf, leaf_off, ninst, root, inst, (T)rk, off, cnt, list,
                           overflow);
}

template <class T>
void launch_part_neigh(bool fill, const vec4<T>* posh, const u32* xscan, const u32* id,
                       const u64* loff, const u32* llist, i64 n, const i64* p_off, int ninst,
                       const InstDev* inst, double rkc, u32* cnt, const u64* noff, u32* nlist,
                       u32* overflow, hipStream_t st)
{
    if (n <= 0) return;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (fill)
        hipLaunchKernelGGL((k_part_neigh<T, true>), grid, dim3(256), 0, st, posh, xscan, id, loff,
                           llist, n, p_off, ninst, inst, (T)rkc, cnt, noff, nlist, overflow);
    else
        hipLaunchKernelGGL((k_part_neigh<T, false>), grid, dim3(256), 0, st, posh, xscan, id, loff,
                           llist, n, p_off, ninst, inst, (T)rkc, cnt, noff, nlist, overflow);
}

#define INST(T)                                                                                 \
    template void launch_leaf_neigh<T>(bool, const vec4<T>*, const vec4<T>*, const u32*, i64,  \
                                       i64, const i64*, int, const u32*, const InstDev*, double, \
                                       const u64*, u32*, u32*, u32*, hipStream_t);              \
    template void launch_part_neigh<T>(bool, const vec4<T>*, const u32*, const u32*,            \
                                       const u64*, const u32*, i64, const i64*, int,            \
                                       const InstDev*, double, u32*, const u64*, u32*, u32*,    \
                                       hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace shsph
