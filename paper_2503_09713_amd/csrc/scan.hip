// Device-wide exclusive scan (reduce, scan of block sums, downsweep).
// Used for the stream compaction of the keep mask (App. D.1), the offsets of
// the leaf and particle neighbour caches (Alg. 5) and the radix-sort digit
// offsets.  out has n+1 entries; out[n] is the total.
#include "common.hpp"
#include "kernels.hpp"

namespace shsph {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr i64 SCAN_TILE = (i64)SCAN_BLOCK * SCAN_ITEMS;
constexpr int SCAN_PBLOCK = 1024;

template <class Tin, class Tacc>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const Tin* __restrict__ in, i64 n,
                                                            Tacc* __restrict__ part)
{
    __shared__ Tacc lds[SCAN_BLOCK / WAVE];
    const i64 base = (i64)blockIdx.x * SCAN_TILE;
    Tacc s = 0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        i64 i = base + (i64)it * SCAN_BLOCK + threadIdx.x;
        if (i < n) s += (Tacc)in[i];
    }
    s = block_reduce<SCAN_BLOCK>(s, lds, [](Tacc a, Tacc b) { return a + b; });
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <class Tacc>
__global__ void __launch_bounds__(SCAN_PBLOCK) k_scan_partials(Tacc* __restrict__ part, i64 nb)
{
    __shared__ Tacc lds[SCAN_PBLOCK / WAVE];
    const i64 per = (nb + SCAN_PBLOCK - 1) / SCAN_PBLOCK;
    const i64 b0 = (i64)threadIdx.x * per;
    Tacc s = 0;
    for (i64 k = 0; k < per; ++k) if (b0 + k < nb) s += part[b0 + k];
    Tacc tot;
    Tacc off = block_excl_scan<SCAN_PBLOCK>(s, lds, tot);
    for (i64 k = 0; k < per; ++k) {
        if (b0 + k < nb) { Tacc v = part[b0 + k]; part[b0 + k] = off; off += v; }
    }
    if (threadIdx.x == 0) part[nb] = tot;
}

template <class Tin, class Tacc, class Tout>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_down(const Tin* __restrict__ in, i64 n,
                                                          const Tacc* __restrict__ part, i64 nb,
                                                          Tout* __restrict__ out, int write_total)
{
    __shared__ Tacc lds[SCAN_BLOCK / WAVE];
    const i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_ITEMS;
    Tacc v[SCAN_ITEMS];
    Tacc s = 0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        i64 i = base + it;
        v[it] = (i < n) ? (Tacc)in[i] : Tacc(0);
        s += v[it];
    }
    Tacc tot;
    Tacc off = block_excl_scan<SCAN_BLOCK>(s, lds, tot) + part[blockIdx.x];
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        i64 i = base + it;
        if (i < n) out[i] = (Tout)off;
        off += v[it];
    }
    if (write_total && blockIdx.x == 0 && threadIdx.x == 0) out[n] = (Tout)part[nb];
}

size_t scan_tmp_bytes(i64 n)
{
    i64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(nb + 2) * sizeof(u64);
}

template <class Tin, class Tacc, class Tout>
static void scan_impl(const Tin* in, Tout* out, i64 n, void* tmp, hipStream_t st)
{
    i64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) nb = 1;
    Tacc* part = (Tacc*)tmp;
    hipLaunchKernelGGL((k_scan_reduce<Tin, Tacc>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, st,
                       in, n, part);
    hipLaunchKernelGGL((k_scan_partials<Tacc>), dim3(1), dim3(SCAN_PBLOCK), 0, st, part, nb);
    hipLaunchKernelGGL((k_scan_down<Tin, Tacc, Tout>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, st,
                       in, n, part, nb, out, 1);
}

void scan_u8_u32(const u8* in, u32* out, i64 n, void* tmp, hipStream_t st)
{
    scan_impl<u8, u32, u32>(in, out, n, tmp, st);
}

void scan_u32_u32(const u32* in, u32* out, i64 n, void* tmp, hipStream_t st)
{
    scan_impl<u32, u32, u32>(in, out, n, tmp, st);
}

void scan_u32_u64(const u32* in, u64* out, i64 n, void* tmp, hipStream_t st)
{
    scan_impl<u32, u64, u64>(in, out, n, tmp, st);
}

}  // namespace shsph
