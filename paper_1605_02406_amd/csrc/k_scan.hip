// Exclusive prefix sums per grid (in place), reduce-then-scan: tile sums, a one-block scan of
// the tile sums per grid, and a tile-local scan plus the tile's offset.  Used for the radix
// sort's digit-major histogram (u32) and for the new-born masses in 2^-40 fixed point (u64,
// exact and independent of the summation order).
#include "launch.h"

namespace dogm {

struct HistSel {
    using T = uint32_t;
    __device__ static T* data(const GridDev& G) { return G.hist; }
    __host__ __device__ static uint32_t len(const GridDev& G, uint32_t bits)
    {
        return (1u << bits) * G.n_sort_tiles;
    }
    __device__ static void total(const GridDev&, uint64_t) {}
};

struct BornSel {
    using T = uint64_t;
    __device__ static T* data(const GridDev& G) { return G.born_q; }
    __host__ __device__ static uint32_t len(const GridDev& G, uint32_t) { return G.C; }
    __device__ static void total(const GridDev& G, uint64_t t) { *G.S_fixed = t; }
};

template <typename Sel>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Batch b, uint32_t bits)
{
    using T = typename Sel::T;
    __shared__ T tmp[kScanThreads / kWave + 1];
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t tile = blockIdx.x - b.bstart[gi];
    const uint32_t len = Sel::len(G, bits);
    const T* a = Sel::data(G);
    T acc = 0;
    for (int it = 0; it < kScanItems; ++it) {
        const uint32_t i = tile * kScanTile + it * kScanThreads + threadIdx.x;
        if (i < len) acc += a[i];
    }
    T total;
    block_excl_scan<T>(acc, tmp, &total);
    if (threadIdx.x == 0) G.scan_part[tile] = (uint64_t)total;
}

template <typename Sel>
__global__ __launch_bounds__(kScanThreads) void k_scan_mid(Batch b, uint32_t bits)
{
    __shared__ uint64_t tmp[kScanThreads / kWave + 1];
    const GridDev& G = *b.g[blockIdx.x];
    const uint32_t ntiles = (Sel::len(G, bits) + kScanTile - 1) / kScanTile;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < ntiles; base += kScanThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t v = i < ntiles ? G.scan_part[i] : 0;
        uint64_t chunk;
        const uint64_t ex = block_excl_scan<uint64_t>(v, tmp, &chunk);
        if (i < ntiles) G.scan_part[i] = carry + ex;
        carry += chunk;
    }
    if (threadIdx.x == 0) Sel::total(G, carry);
}

template <typename Sel>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(Batch b, uint32_t bits)
{
    using T = typename Sel::T;
    __shared__ T tmp[kScanThreads / kWave + 1];
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t tile = blockIdx.x - b.bstart[gi];
    const uint32_t len = Sel::len(G, bits);
    T* a = Sel::data(G);
    const uint32_t base = tile * kScanTile + threadIdx.x * kScanItems;
    T v[kScanItems];
    T acc = 0;
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        const uint32_t i = base + it;
        v[it] = i < len ? a[i] : 0;
        acc += v[it];
    }
    T total;
    T run = block_excl_scan<T>(acc, tmp, &total) + (T)G.scan_part[tile];
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        const uint32_t i = base + it;
        if (i < len) a[i] = run;
        run += v[it];
    }
}

template <typename Sel>
static hipError_t scan_impl(const GridRef* g, int n, uint32_t bits, hipStream_t s)
{
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [bits](const GridDev& G) {
        return ceil_div(Sel::len(G, bits), kScanTile);
    });
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_reduce<Sel>, dim3(blocks), dim3(kScanThreads), 0, s, b, bits);
    hipLaunchKernelGGL(k_scan_mid<Sel>, dim3(n), dim3(kScanThreads), 0, s, b, bits);
    hipLaunchKernelGGL(k_scan_down<Sel>, dim3(blocks), dim3(kScanThreads), 0, s, b, bits);
    return hipGetLastError();
}

hipError_t launch_scan(const GridRef* g, int n, ScanArray which, uint32_t bits, hipStream_t s)
{
    return which == ScanArray::SortHist ? scan_impl<HistSel>(g, n, bits, s)
                                        : scan_impl<BornSel>(g, n, bits, s);
}

}  // namespace dogm
