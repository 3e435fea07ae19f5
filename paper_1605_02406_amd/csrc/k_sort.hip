// Alg. 2, first line: stable sort of the particles by cell key.
//
// LSD radix sort over digits of at most kSortBits bits (two passes for grids up to 2^20 cells);
// each pass moves the key, the source index and the particle state (FP32, or FP64 in the all-FP64
// precision mode).  A pass is three kernels that communicate only through memory: the digit
// histogram of every tile (for the first pass it comes from the prediction kernel), a scan of
// each digit's row of tile counts, and the scatter.  No block waits for another.  The per-cell
// pass that follows marks where each cell's run of sorted particles starts and ends.
//
// The whole record travels with every pass, in runs of equal digits, so every read and write of
// the state is coalesced.  (Moving only (key, index) pairs through the passes and the state
// once, gathered in final order, measured no faster: position noise of half a cell spreads each
// cell's particles over about nine cells, so the gather's reads touch two dozen cache lines per
// wave and re-read three times the state through L2.)
//
// Stable ranking inside a tile: each of the block's 16 waves owns a contiguous sixteenth of the
// tile (256 keys) and walks it 64 keys at a time; lanes holding the same digit find each other
// with one ballot per digit bit, take their rank from the mask of lower peers, and the lowest
// peer advances the wave's running count of that digit (16-bit counters in LDS).  Sixteenths are
// stacked in wave order, so every key's rank is its position among equal digits in input order.
// The tile is then rearranged in LDS so each digit's run leaves as one contiguous block.
#include <mutex>
#include <vector>

#include "launch.h"

namespace dogm {

constexpr int kSortWaves = kSortThreads / kWave;

// The arrays one pass reads and writes, as raw pointers (P = HostPtr) or global-space views.
template <template <typename> class P>
struct SortArrays {
    P<uint32_t> ik;
    P<uint32_t> iv;  // null: the source index is the element index
    P<float> ix, iy, ivx, ivy, iw;
    P<uint32_t> ok, ov;
    P<float> ox, oy, ovx, ovy, ow;
};

// Pass p of P reads the predicted state (p == 0) or the previous pass's output and writes the
// sorted arrays on the last pass; the passes alternate between the sorted and the temporary
// arrays so that the last one lands in the sorted arrays.
template <template <typename> class P>
__device__ __forceinline__ SortArrays<P> sort_arrays(const GridT<P>& G, uint32_t pass)
{
    const bool dst_sorted = ((G.passes - 1 - pass) & 1u) == 0;
    SortArrays<P> a;
    if (pass == 0) {
        a.ik = G.key; a.iv = P<uint32_t>{};
        a.ix = G.x; a.iy = G.y; a.ivx = G.vx; a.ivy = G.vy; a.iw = G.w;
    } else if (dst_sorted) {
        a.ik = G.tkey; a.iv = G.tval;
        a.ix = G.tx; a.iy = G.ty; a.ivx = G.tvx; a.ivy = G.tvy; a.iw = G.tw;
    } else {
        a.ik = G.skey; a.iv = G.perm;
        a.ix = G.sx; a.iy = G.sy; a.ivx = G.svx; a.ivy = G.svy; a.iw = G.sw;
    }
    if (dst_sorted) {
        a.ok = G.skey; a.ov = G.perm;
        a.ox = G.sx; a.oy = G.sy; a.ovx = G.svx; a.ovy = G.svy; a.ow = G.sw;
    } else {
        a.ok = G.tkey; a.ov = G.tval;
        a.ox = G.tx; a.oy = G.ty; a.ovx = G.tvx; a.ovy = G.tvy; a.ow = G.tw;
    }
    return a;
}

// Digit histogram of every tile of the keys a pass (>= 1) reads.
constexpr int kHistItems = kHistTile / kHistThreads;  // 4

__global__ __launch_bounds__(kHistThreads) void k_sort_hist(Batch b, uint32_t pass)
{
    __shared__ uint32_t cnt[kSortBins];
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    // neighbouring tiles write neighbouring words of every digit row: keep them on one XCD so
    // the partial lines meet in its L2
    const uint32_t tile = xcd_tile(b, gi);
    if (tile >= G.n_hist_tiles) return;
    const uint32_t shift = pass_shift(b.g[gi], pass), bits = pass_bits(b.g[gi], pass);
    const uint32_t nbins = 1u << bits;
    for (uint32_t d = threadIdx.x; d < nbins; d += kHistThreads) cnt[d] = 0;
    __syncthreads();
    const auto keys = sort_arrays(G, pass).ik;
    uint32_t k[kHistItems];
#pragma unroll
    for (int it = 0; it < kHistItems; ++it) {
        const uint32_t i = tile * kHistTile + it * kHistThreads + threadIdx.x;
        k[it] = i < G.nu ? keys[i] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kHistItems; ++it) {
        const uint32_t i = tile * kHistTile + it * kHistThreads + threadIdx.x;
        digit_count(i < G.nu, (k[it] >> shift) & (nbins - 1u), cnt);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nbins; d += kHistThreads)
        G.hist[d * G.n_hist_tiles + tile] = cnt[d];
}

// Each block turns one digit's row of tile counts into exclusive prefixes (each thread scans
// kRowItems consecutive entries, then one block-wide scan) and stores the row's total.
constexpr int kRowItems = 8;

__global__ __launch_bounds__(kScanRowThreads) void k_scan_rows(Batch b, uint32_t pass)
{
    __shared__ uint32_t tmp[kScanRowThreads / kWave + 1];
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const uint32_t d = blockIdx.x - b.bstart[gi];
    const GArr<uint32_t> row{G.hist.p + (size_t)d * G.n_hist_tiles};
    uint32_t carry = 0;
    for (uint32_t base = 0; base < G.n_hist_tiles; base += kScanRowThreads * kRowItems) {
        const uint32_t t0 = base + threadIdx.x * kRowItems;
        uint32_t v[kRowItems], acc = 0;
#pragma unroll
        for (int j = 0; j < kRowItems; ++j) {
            v[j] = (t0 + j < G.n_hist_tiles) ? row[t0 + j] : 0u;
            acc += v[j];
        }
        uint32_t total;
        uint32_t run = carry + block_excl_scan(acc, tmp, &total);
#pragma unroll
        for (int j = 0; j < kRowItems; ++j) {
            if (t0 + j < G.n_hist_tiles) row[t0 + j] = run;
            run += v[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) G.rowtot[d] = carry;
}

// Reads one state array for a wave's items (coalesced, zeros past the end); the array holds
// the grid's real type R (its descriptor entry is typed FP32).
template <typename R>
__device__ __forceinline__ void load_items(const float* in, uint32_t base, uint32_t n,
                                           R (&out)[kSortItems])
{
    const R* a = reinterpret_cast<const R*>(in);
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t idx = base + it * kWave + lane_id();
        out[it] = idx < n ? a[idx] : (R)0;
    }
}

// Writes one payload array in destination order: every element goes to its local sorted slot in
// LDS, then each thread moves the slots it owns to their global positions.
template <typename T>
__device__ __forceinline__ void move_out(const T (&vals)[kSortItems], T* out, uint32_t* stage,
                                         const uint32_t (&lpos)[kSortItems],
                                         const uint32_t (&gpos)[kSortItems])
{
    T* row = reinterpret_cast<T*>(stage);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it)
        if (lpos[it] < (uint32_t)kSortTile) row[lpos[it]] = vals[it];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kSortItems; ++m)
        if (gpos[m] != 0xFFFFFFFFu) out[gpos[m]] = row[m * kSortThreads + threadIdx.x];
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(Batch b, uint32_t pass)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t scan_tmp[kSortWaves + 1];

    const int gi = batch_grid(b);
    // the descriptor is read in place: a private copy of both ping-pong pointer sets costs this
    // kernel more than the loads it saves
    const GridDev& G = *b.g[gi];
    const uint32_t tile = xcd_tile(b, gi);
    if (tile >= G.n_sort_tiles) return;
    const uint32_t shift = G.dshift[pass], bits = G.dbits[pass];
    const uint32_t nbins = 1u << bits, mask = nbins - 1u;
    // each thread owns a contiguous run of digits; their totals over all tiles and their counts
    // in the tiles before this one do not depend on the tile's keys and are read first
    constexpr int kMaxDpt = kSortBins / kSortThreads;
    const uint32_t dpt = nbins >= (uint32_t)kSortThreads ? nbins / kSortThreads : 1u;
    const uint32_t d0 = threadIdx.x * dpt;
    const bool owner = d0 < nbins;
    uint32_t gl[kMaxDpt], before[kMaxDpt];
    if (owner) {
#pragma unroll
        for (int j = 0; j < kMaxDpt; ++j) {
            if ((uint32_t)j >= dpt) break;
            const uint32_t d = d0 + j;
            gl[j] = G.rowtot[d];
            before[j] = G.hist[d * G.n_hist_tiles + tile * (kSortTile / kHistTile)];
        }
    }
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;

    // LDS: per-wave digit counts (16-bit: at most kSortTile per digit), local digit starts
    // (16-bit), global digit offsets; the staging row (kSortTile values of the widest array
    // moved) reuses the counters' space once every element's local position is known, which
    // keeps 11-bit digits within half the LDS of a CU (two blocks per CU)
    const uint32_t region_words = max((uint32_t)(kSortWaves * nbins) / 2u,
                                      (uint32_t)(kSortTile * sizeof(R)) / 4u);
    uint16_t* cnt = reinterpret_cast<uint16_t*>(lds);                      // [kSortWaves][nbins]
    uint16_t* tstart = reinterpret_cast<uint16_t*>(lds + region_words);    // [nbins]
    uint32_t* goff = lds + region_words + nbins / 2;                       // [nbins]
    uint32_t* stage = lds;                                                 // [kSortTile]

    for (uint32_t d = threadIdx.x; d < (kSortWaves * nbins) / 2; d += kSortThreads) lds[d] = 0;
    __syncthreads();

    const SortArrays<HostPtr> A = sort_arrays(G, pass);
    const uint32_t base = tile * kSortTile + wave * (kSortTile / kSortWaves);
    uint32_t k[kSortItems], v[kSortItems], rank[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t idx = base + it * kWave + lane;
        const bool valid = idx < G.nu;
        k[it] = valid ? A.ik[idx] : 0u;
        v[it] = valid ? (A.iv ? A.iv[idx] : idx) : 0u;
    }
    // the first state array is read while the tile is ranked
    R pa[kSortItems], pb[kSortItems];
    load_items(A.ix, base, G.nu, pa);
    // stable ranks inside the wave's quarter
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t idx = base + it * kWave + lane;
        const bool valid = idx < G.nu;
        const uint32_t d = (k[it] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (uint32_t bit = 0; bit < bits; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t bb = __ballot(set);
            peers &= set ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        uint32_t before = 0;
        if (valid) before = cnt[wave * nbins + d];
        // every lane has read its digit's count before the lowest peer advances it (the wave
        // runs in lockstep; the wave barrier states that order and costs no instruction)
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) cnt[wave * nbins + d] = (uint16_t)(before + (uint32_t)__popcll(peers));
        rank[it] = valid ? before + below : 0xFFFFFFFFu;
    }
    __syncthreads();

    // per owned digit: wave offsets inside the digit, the tile's digit totals (local starts)
    // and the digit's global start (all earlier digits, then this digit in all earlier tiles)
    uint32_t tot[kMaxDpt];
    uint32_t my_tot = 0, my_gl = 0;
    if (owner) {
#pragma unroll
        for (int j = 0; j < kMaxDpt; ++j) {
            if ((uint32_t)j >= dpt) break;
            const uint32_t d = d0 + j;
            uint32_t acc = 0;
            for (int w = 0; w < kSortWaves; ++w) {
                const uint32_t c = cnt[w * nbins + d];
                cnt[w * nbins + d] = (uint16_t)acc;
                acc += c;
            }
            tot[j] = acc;
            my_tot += acc;
            my_gl += gl[j];
        }
    }
    uint32_t tile_n, all_n;
    uint32_t lrun = block_excl_scan(my_tot, scan_tmp, &tile_n);
    uint32_t grun = block_excl_scan(my_gl, scan_tmp, &all_n);
    if (owner) {
#pragma unroll
        for (int j = 0; j < kMaxDpt; ++j) {
            if ((uint32_t)j >= dpt) break;
            const uint32_t d = d0 + j;
            tstart[d] = (uint16_t)lrun;
            goff[d] = grun + before[j];
            lrun += tot[j];
            grun += gl[j];
        }
    }
    __syncthreads();

    // keys into local sorted order, then out in runs; remember every element's destination
    uint32_t lpos[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        lpos[it] = 0xFFFFFFFFu;
        if (rank[it] != 0xFFFFFFFFu) {
            const uint32_t d = (k[it] >> shift) & mask;
            lpos[it] = (uint32_t)tstart[d] + cnt[wave * nbins + d] + rank[it];
            if (lpos[it] >= (uint32_t)kSortTile) status_or(G, kStInternal);
        }
    }
    __syncthreads();  // the counters are read: the staging row may overwrite them
#pragma unroll
    for (int it = 0; it < kSortItems; ++it)
        if (lpos[it] < (uint32_t)kSortTile) stage[lpos[it]] = k[it];
    __syncthreads();
    const uint32_t nvalid = min((uint32_t)kSortTile, G.nu - tile * kSortTile);
    uint32_t gpos[kSortItems];
#pragma unroll
    for (int m = 0; m < kSortItems; ++m) {
        const uint32_t j = m * kSortThreads + threadIdx.x;
        gpos[m] = 0xFFFFFFFFu;
        if (j < nvalid) {
            const uint32_t kk = stage[j];
            const uint32_t d = (kk >> shift) & mask;
            const uint32_t g = goff[d] + (j - tstart[d]);
            if (g < G.nu) {
                A.ok[g] = kk;
                gpos[m] = g;
            } else {
                status_or(G, kStInternal);
            }
        }
    }
    // the source index and the state, one array at a time through the same LDS row; the next
    // array's loads are in flight while the current one is staged
    move_out(v, A.ov, stage, lpos, gpos);
    load_items(A.iy, base, G.nu, pb);
    move_out(pa, reinterpret_cast<R*>(A.ox), stage, lpos, gpos);
    load_items(A.ivx, base, G.nu, pa);
    move_out(pb, reinterpret_cast<R*>(A.oy), stage, lpos, gpos);
    load_items(A.ivy, base, G.nu, pb);
    move_out(pa, reinterpret_cast<R*>(A.ovx), stage, lpos, gpos);
    load_items(A.iw, base, G.nu, pa);
    move_out(pb, reinterpret_cast<R*>(A.ovy), stage, lpos, gpos);
    move_out(pa, reinterpret_cast<R*>(A.ow), stage, lpos, gpos);
}

// The scatter's dynamic LDS (76 KiB with 11-bit digits) is above the default limit: raise it
// once on every device the library launches on (the attribute is per device).
constexpr int kScatterLdsMax = 80 * 1024;
hipError_t allow_scatter_lds()
{
    static std::mutex mu;
    static std::vector<bool> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev < done.size() && done[dev]) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sort_scatter<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kScatterLdsMax);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sort_scatter<double>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kScatterLdsMax);
    if (e != hipSuccess) return e;
    if ((size_t)dev >= done.size()) done.resize(dev + 1, false);
    done[dev] = true;
    return hipSuccess;
}

hipError_t launch_sort(const GridRef* g, int n, hipStream_t s)
{
    if (const hipError_t e = allow_scatter_lds(); e != hipSuccess) return e;
    uint32_t max_passes = 0;
    for (int i = 0; i < n; ++i)
        max_passes = g[i].hd->passes > max_passes ? g[i].hd->passes : max_passes;
    for (uint32_t pass = 0; pass < max_passes; ++pass) {
        // grids that still have this pass
        GridRef sub[kMaxBatch];
        int m = 0;
        uint32_t maxbits = 0;
        for (int i = 0; i < n; ++i)
            if (g[i].hd->passes > pass) {
                sub[m++] = g[i];
                maxbits = g[i].hd->dbits[pass] > maxbits ? g[i].hd->dbits[pass] : maxbits;
            }
        Batch b;
        if (pass > 0) {
            const uint32_t hb =
                make_batch(b, sub, m, [](const GridDev& G) { return xcd_blocks(G.n_hist_tiles); });
            if (hb) DOGM_LAUNCH(k_sort_hist, dim3(hb), dim3(kHistThreads), 0, s, b, pass);
        }
        const uint32_t rows =
            make_batch(b, sub, m, [pass](const GridDev& G) { return 1u << G.dbits[pass]; });
        if (rows) DOGM_LAUNCH(k_scan_rows, dim3(rows), dim3(kScanRowThreads), 0, s, b, pass);
        const uint32_t tiles =
            make_batch(b, sub, m, [](const GridDev& G) { return xcd_blocks(G.n_sort_tiles); });
        const uint32_t nbins = 1u << maxbits;
        const bool real64 = launch_real64(g, n);
        const size_t counters = sizeof(uint16_t) * (size_t)kSortWaves * nbins;
        const size_t row = (real64 ? sizeof(double) : sizeof(uint32_t)) * (size_t)kSortTile;
        const size_t lds = (counters > row ? counters : row) + sizeof(uint16_t) * nbins +
                           sizeof(uint32_t) * (size_t)nbins;
        if (tiles)
            DOGM_LAUNCH_REAL(real64, "k_sort_scatter", k_sort_scatter, dim3(tiles),
                             dim3(kSortThreads), lds, s, b, pass);
    }
    // the particle range of every occupied cell, with the per-cell sums of the update
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? launch_cell_sums(g, n, s) : e;
}

}  // namespace dogm
