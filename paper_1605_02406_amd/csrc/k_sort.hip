// Alg. 2, first line: stable sort of the particles by cell key.
//
// LSD radix sort of (key, particle index) pairs with digits of at most 8 bits, one
// reduce-then-scan round per digit: a per-tile digit histogram, an exclusive scan of the
// digit-major histogram matrix, and a scatter in which every tile ranks its keys stably and
// writes them through LDS so that each digit's run leaves the tile as one contiguous block.
//
// Stable ranking inside a tile: each wave owns a contiguous quarter of the tile (1024 keys) and
// walks it 64 keys at a time; lanes holding the same digit find each other with one ballot per
// digit bit, take their rank from the mask of lower peers, and the lowest peer advances the
// wave's running count of that digit.  Wave quarters are then stacked in wave order, so the
// rank of every key is its position among equal digits in input order.
#include "launch.h"

namespace dogm {

// Source / destination of a pass: 0 = (key, implicit index), 1 = (skey, perm), 2 = (tkey, tval).
__device__ __forceinline__ const uint32_t* src_keys(const GridDev& G, int sel)
{
    return sel == 0 ? G.key : (sel == 1 ? G.skey : G.tkey);
}
__device__ __forceinline__ const uint32_t* src_vals(const GridDev& G, int sel)
{
    return sel == 1 ? G.perm : G.tval;
}
__device__ __forceinline__ uint32_t* dst_keys(const GridDev& G, int sel)
{
    return sel == 1 ? G.skey : G.tkey;
}
__device__ __forceinline__ uint32_t* dst_vals(const GridDev& G, int sel)
{
    return sel == 1 ? G.perm : G.tval;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(Batch b, uint32_t shift,
                                                             uint32_t bits, int src)
{
    __shared__ uint32_t h[kSortThreads / kWave][1 << kMaxDigitBits];
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t tile = blockIdx.x - b.bstart[gi];
    const uint32_t nbins = 1u << bits, mask = nbins - 1;
    const int wave = threadIdx.x / kWave;
    for (uint32_t d = threadIdx.x; d < (kSortThreads / kWave) * nbins; d += kSortThreads)
        h[d / nbins][d % nbins] = 0;
    __syncthreads();
    const uint32_t* keys = src_keys(G, src);
    const uint32_t base = tile * kSortTile;
#pragma unroll 4
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t idx = base + it * kSortThreads + threadIdx.x;
        if (idx < G.nu) atomicAdd(&h[wave][(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nbins; d += kSortThreads) {
        uint32_t t = 0;
        for (int w = 0; w < kSortThreads / kWave; ++w) t += h[w][d];
        G.hist[d * G.n_sort_tiles + tile] = t;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(Batch b, uint32_t shift,
                                                                uint32_t bits, int src, int dst)
{
    constexpr int kWaves = kSortThreads / kWave;
    constexpr int kBins = 1 << kMaxDigitBits;
    __shared__ uint32_t cnt[kWaves][kBins];  // running count per wave, then wave offsets
    __shared__ uint32_t tstart[kBins];       // first local position of each digit
    __shared__ uint32_t goff[kBins];         // first global position of each digit
    __shared__ uint32_t scan_tmp[kWaves + 1];
    __shared__ uint32_t stage_k[kSortTile];
    __shared__ uint32_t stage_v[kSortTile];

    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t tile = blockIdx.x - b.bstart[gi];
    const uint32_t nbins = 1u << bits, mask = nbins - 1;
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;

    for (int d = threadIdx.x; d < kWaves * kBins; d += kSortThreads) cnt[d / kBins][d % kBins] = 0;
    __syncthreads();

    const uint32_t* keys = src_keys(G, src);
    const uint32_t* vals = src_vals(G, src);
    const uint32_t base = tile * kSortTile + wave * (kSortTile / kWaves);
    uint32_t k[kSortItems], v[kSortItems], rank[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t idx = base + it * kWave + lane;
        const bool valid = idx < G.nu;
        const uint32_t kk = valid ? keys[idx] : 0u;
        const uint32_t vv = valid ? (src == 0 ? idx : vals[idx]) : 0u;
        const uint32_t d = (kk >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (uint32_t bit = 0; bit < bits; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t bb = __ballot(set);
            peers &= set ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        uint32_t before = 0;
        if (valid) before = cnt[wave][d];
        if (valid && below == 0) cnt[wave][d] = before + (uint32_t)__popcll(peers);
        k[it] = kk;
        v[it] = vv;
        rank[it] = valid ? before + below : 0xFFFFFFFFu;
    }
    __syncthreads();

    // digit totals of the tile, wave offsets inside each digit, local digit starts
    uint32_t total = 0;
    if (threadIdx.x < nbins) {
        uint32_t acc = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = cnt[w][threadIdx.x];
            cnt[w][threadIdx.x] = acc;
            acc += c;
        }
        total = acc;
        goff[threadIdx.x] = G.hist[threadIdx.x * G.n_sort_tiles + tile];
    }
    uint32_t tile_total;
    const uint32_t start = block_excl_scan<uint32_t>(total, scan_tmp, &tile_total);
    if (threadIdx.x < nbins) tstart[threadIdx.x] = start;
    __syncthreads();

#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        if (rank[it] != 0xFFFFFFFFu) {
            const uint32_t d = (k[it] >> shift) & mask;
            const uint32_t lpos = tstart[d] + cnt[wave][d] + rank[it];
            if (lpos < (uint32_t)kSortTile) {
                stage_k[lpos] = k[it];
                stage_v[lpos] = v[it];
            } else {
                atomicOr(G.status, kStInternal);
            }
        }
    }
    __syncthreads();

    uint32_t* ok = dst_keys(G, dst);
    uint32_t* ov = dst_vals(G, dst);
    const uint32_t nvalid = min((uint32_t)kSortTile, G.nu - tile * kSortTile);
    for (uint32_t j = threadIdx.x; j < nvalid; j += kSortThreads) {
        const uint32_t kk = stage_k[j];
        const uint32_t d = (kk >> shift) & mask;
        const uint32_t g = goff[d] + (j - tstart[d]);
        if (g < G.nu) {
            ok[g] = kk;
            ov[g] = stage_v[j];
        } else {
            atomicOr(G.status, kStInternal);
        }
    }
}

hipError_t launch_sort(const GridRef* g, int n, hipStream_t s)
{
    // one digit plan for the whole launch, from the largest key (C) of the batch
    int kb = 1;
    for (int i = 0; i < n; ++i) kb = key_bits(g[i].hd->C) > kb ? key_bits(g[i].hd->C) : kb;
    const int passes = (kb + kMaxDigitBits - 1) / kMaxDigitBits;
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [](const GridDev& G) { return G.n_sort_tiles; });
    if (blocks == 0) return hipSuccess;
    uint32_t shift = 0;
    int src = 0;
    for (int p = 0; p < passes; ++p) {
        const uint32_t bits = (uint32_t)((kb - (int)shift + (passes - p) - 1) / (passes - p));
        // the last pass lands in (skey, perm)
        const int dst = ((passes - 1 - p) % 2 == 0) ? 1 : 2;
        hipLaunchKernelGGL(k_sort_hist, dim3(blocks), dim3(kSortThreads), 0, s, b, shift, bits,
                           src);
        hipError_t e = launch_scan(g, n, ScanArray::SortHist, bits, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sort_scatter, dim3(blocks), dim3(kSortThreads), 0, s, b, shift, bits,
                           src, dst);
        shift += bits;
        src = dst;
    }
    return hipGetLastError();
}

}  // namespace dogm
