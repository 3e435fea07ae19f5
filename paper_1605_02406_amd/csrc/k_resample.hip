// Alg. 7: systematic resampling of nu particles from the joint set [sorted persistent | new-born].
//
// The CDF is an exact integer prefix sum of the weights in 2^-40 fixed point, so it does not
// depend on the summation order; the per-tile totals were accumulated by the kernels that wrote
// the weights.  Draw j sits at u_j = (j + U) d with the spacing d = W / nu rounded once to FP64,
// and selects the first particle i with F_i > floor(u_j); for nu < 2^27 the last draw stays
// below W by more than the roundings of W, d and the product (1 - U >= 2^-24, so the margin is
// at least 2^-24 / nu of W against three half-ulps), so every draw finds a particle.
// Source i receives the draws J(F_{i-1}) <= j < J(F_i) with J(F) = min{ j : floor(u_j) >= F }.
// Each tile adds up the totals of the tiles before it (or, for grids with many tiles, reads
// their prefix from a scan kernel) and scans its own weights with wave prefix sums.  The draws of a tile's sources form one contiguous range
// of outputs; every source stores its first draw in LDS, and the block's threads then share
// the tile's outputs evenly, each finding the source of an output by binary search among
// those first draws.  A single source can receive a thousand draws or more (a new-born
// particle alone in a cell with high new-born mass), so the outputs are not left to the lanes
// that own the sources.  Consecutive outputs are written by consecutive lanes, and their sources ascend.
#include "launch.h"

namespace dogm {

constexpr int kResWaves = kResThreads / kWave;
// the automatic plan shares outputs evenly (k_resample) above this many persistent particles and
// lets the lanes that own the sources write their draws (k_resample_windowed) below it
constexpr uint32_t kBalancedFrom = 1u << 22;
constexpr int kResRounds = kResItems;  // consecutive sources per lane
static_assert(kResRounds % 4 == 0, "a lane reads its weights as 16-byte vectors");

__device__ __forceinline__ uint64_t draw_floor(uint32_t j, double U, double spacing)
{
    return (uint64_t)floor(__dmul_rn(__dadd_rn((double)j, U), spacing));
}

// min { j in [0, nu] : floor(u_j) >= F }, with u_nu taken as +infinity.
__device__ __forceinline__ uint32_t first_draw_at(uint64_t F, double U, double spacing,
                                                  double inv_spacing, uint32_t nu)
{
    double est = ceil((double)F * inv_spacing - U);
    est = est < 0.0 ? 0.0 : (est > (double)nu ? (double)nu : est);
    uint32_t j = (uint32_t)est;
    while (j > 0 && draw_floor(j - 1, U, spacing) >= F) --j;
    while (j < nu && draw_floor(j, U, spacing) < F) ++j;
    return j;
}

// This lane's kResRounds consecutive source weights (16-byte vectors where whole).
template <typename R>
__device__ __forceinline__ void load_weights(const GArr<R>& wsrc, uint32_t lbase, uint32_t n_src,
                                             R (&wl)[kResRounds])
{
    if (lbase + kResRounds <= n_src) {
        using V = typename RealVec16<R>::type;
        constexpr int kVec = 16 / (int)sizeof(R);
#pragma unroll
        for (int r = 0; r < kResRounds; r += kVec) {
            const V v = wsrc.template load_vec<V>(lbase + r);
#pragma unroll
            for (int e = 0; e < kVec; ++e) wl[r + e] = v[e];
        }
    } else {
#pragma unroll
        for (int r = 0; r < kResRounds; ++r) {
            const uint32_t i = lbase + r;
            wl[r] = i < n_src ? wsrc[i] : (R)0;
        }
    }
}

// Joint weight of the partial sums before `limit` (persistent tiles of kResTile particles, then
// new-born tiles of kBornTile slots) and in total: from their exclusive prefixes where a scan
// formed them, else added up by the block (tile 0 then stores the total).
__device__ __forceinline__ void tile_prefix(const GridView& G, uint32_t limit, int prefixed,
                                            uint32_t tile, uint64_t* before, uint64_t* W)
{
    if (prefixed) {
        *before = G.rpart[limit];
        *W = *G.W_fixed;
    } else {
        partials_before(G.rpart, G.n_res_ptiles + G.n_born_parts, limit, before, W);
        if (tile == 0 && threadIdx.x == 0) *G.W_fixed = *W;
    }
}

template <typename R>
__global__ __launch_bounds__(kResThreads) void k_resample(Batch b, int prefixed)
{
    __shared__ uint64_t wave_tot[kResWaves];  // each wave's weight total
    __shared__ uint32_t first[kResTile + 1];  // first draw of each source of the tile; the end
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const uint32_t ntiles = G.n_res_ptiles + G.n_res_btiles;
    const uint32_t tile = xcd_tile(b, gi);
    if (tile >= ntiles) return;
    const uint32_t cycle = *G.cycle_run;
    // the cycle ends here: every block stores the same next value of the counter that the
    // prediction reads (no block of this kernel reads it)
    if (threadIdx.x == 0) *G.cycle = cycle + 1u;
    const uint32_t nu = G.nu;
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;

    const bool born = tile >= G.n_res_ptiles;
    const uint32_t t_local = born ? tile - G.n_res_ptiles : tile;
    const uint32_t n_src = born ? G.nb : nu;
    const uint32_t tbase = t_local * kResTile;

    // each lane owns kResRounds consecutive sources
    const uint32_t lsrc = wave * (kResRounds * kWave) + lane * kResRounds;  // local index
    const uint32_t lbase = tbase + lsrc;
    R wl[kResRounds];
    load_weights<R>(real<R>(born ? G.bw : G.sw), lbase, n_src, wl);

    // joint weight before this tile and in total
    const uint32_t limit = born ? G.n_res_ptiles + t_local * (kResTile / kBornTile) : tile;
    uint64_t before, W;
    tile_prefix(G, limit, prefixed, tile, &before, &W);

    if (W == 0) {  // nothing carries weight: keep the sorted persistent set as it is
        if (!born) {
            for (int r = 0; r < kResRounds; ++r) {
                const uint32_t i = tbase + (uint32_t)(r * kResThreads) + threadIdx.x;
                if (i < nu) {
                    real<R>(G.x)[i] = real<R>(G.sx)[i];
                    real<R>(G.y)[i] = real<R>(G.sy)[i];
                    real<R>(G.vx)[i] = real<R>(G.svx)[i];
                    real<R>(G.vy)[i] = real<R>(G.svy)[i];
                    real<R>(G.w)[i] = real<R>(G.sw)[i];
                }
            }
        }
        return;
    }

    uint64_t q[kResRounds];
    uint64_t lsum = 0;
#pragma unroll
    for (int r = 0; r < kResRounds; ++r) {
        q[r] = fixed40(wl[r]);
        lsum += q[r];
    }
    const uint64_t lincl = wave_incl_scan(lsum);
    if (lane == kWave - 1) wave_tot[wave] = lincl;
    __syncthreads();
    uint64_t run = before;
    for (int w2 = 0; w2 < wave; ++w2) run += wave_tot[w2];
    uint64_t tile_end = before;
    for (int w2 = 0; w2 < kResWaves; ++w2) tile_end += wave_tot[w2];

    const double U = (double)unit_f32(draw(G, 0u, cycle, kPurposeResample).x);
    const double spacing = __ddiv_rn((double)W, (double)nu);
    const double inv_spacing = 1.0 / spacing;
    const R out_w = (R)((double)W * 0x1p-40 / (double)nu);

    // first draw of each of this lane's sources; the draws of local source s are
    // [first[s], first[s + 1]), and the tile's draws are [first[0], first[kResTile])
    uint64_t F = run + lincl - lsum;
#pragma unroll
    for (int r = 0; r < kResRounds; ++r) {
        first[lsrc + r] = first_draw_at(F, U, spacing, inv_spacing, nu);
        F += q[r];
    }
    if (threadIdx.x == 0) first[kResTile] = first_draw_at(tile_end, U, spacing, inv_spacing, nu);
    __syncthreads();
    const uint32_t j_begin = first[0], j_end = first[kResTile];

    const auto px = real<R>(born ? G.bx : G.sx);
    const auto py = real<R>(born ? G.by : G.sy);
    const auto pvx = real<R>(born ? G.bvx : G.svx);
    const auto pvy = real<R>(born ? G.bvy : G.svy);
    const auto X = real<R>(G.x), Y = real<R>(G.y), VX = real<R>(G.vx), VY = real<R>(G.vy);
    const auto Wt = real<R>(G.w);
    // four outputs per thread per step, their source reads issued together; the source of
    // output j is the last local source whose first draw is at or before j
    constexpr int kUnroll = 4;
    for (uint32_t j0 = j_begin + threadIdx.x; j0 < j_end; j0 += kUnroll * kResThreads) {
        uint32_t src[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t j = j0 + u * kResThreads;
            uint32_t lo = 0, hi = kResTile;  // first[lo] <= j < first[hi]
            if (j < j_end) {
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (first[mid] <= j) lo = mid;
                    else hi = mid;
                }
            }
            src[u] = tbase + lo;
        }
        R ox[kUnroll], oy[kUnroll], ovx[kUnroll], ovy[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            ox[u] = px[src[u]];
            oy[u] = py[src[u]];
            ovx[u] = pvx[src[u]];
            ovy[u] = pvy[src[u]];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t j = j0 + u * kResThreads;
            if (j < j_end) {
                X[j] = ox[u];
                Y[j] = oy[u];
                VX[j] = ovx[u];
                VY[j] = ovy[u];
                Wt[j] = out_w;
            }
        }
    }
}

// The same draws, each wave writing those of its own sources: it walks them in windows of
// kResWindow, marks in the window's LDS map where each source's draws begin, fills in the source
// of every draw with a running maximum over the map, then writes the window's outputs in order.
// Cheaper per output than the binary search when sources receive few draws each, and a source
// with many draws costs its wave no more map work than many sources with few.
constexpr int kResWindow = 1024;  // draws per LDS map window of a wave
constexpr int kMapPerLane = kResWindow / kWave;  // map entries a lane scans
static_assert(kMapPerLane == 16, "a lane scans its map entries as two 16-byte vectors");

template <typename R>
__global__ __launch_bounds__(kResThreads) void k_resample_windowed(Batch b, int prefixed)
{
    constexpr int kSrc = kResRounds * kWave;  // sources per wave
    static_assert(kSrc <= 65536, "local source indices are 16-bit");
    __shared__ uint64_t wave_tot[kResWaves];  // each wave's weight total
    __shared__ __attribute__((aligned(16))) uint16_t srcmap[kResWaves][kResWindow];
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const uint32_t ntiles = G.n_res_ptiles + G.n_res_btiles;
    const uint32_t tile = xcd_tile(b, gi);
    if (tile >= ntiles) return;
    const uint32_t cycle = *G.cycle_run;
    // the cycle ends here: every block stores the same next value of the counter that the
    // prediction reads (no block of this kernel reads it)
    if (threadIdx.x == 0) *G.cycle = cycle + 1u;
    const uint32_t nu = G.nu;
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;

    const bool born = tile >= G.n_res_ptiles;
    const uint32_t t_local = born ? tile - G.n_res_ptiles : tile;
    const uint32_t n_src = born ? G.nb : nu;
    const uint32_t wbase = t_local * kResTile + wave * kSrc;

    // each lane owns kResRounds consecutive sources
    const uint32_t lbase = wbase + lane * kResRounds;
    R wl[kResRounds];
    load_weights<R>(real<R>(born ? G.bw : G.sw), lbase, n_src, wl);

    // joint weight before this tile and in total
    const uint32_t limit = born ? G.n_res_ptiles + t_local * (kResTile / kBornTile) : tile;
    uint64_t before, W;
    tile_prefix(G, limit, prefixed, tile, &before, &W);

    if (W == 0) {  // nothing carries weight: keep the sorted persistent set as it is
        if (!born) {
            for (int r = 0; r < kResRounds; ++r) {
                const uint32_t i = wbase + r * kWave + lane;
                if (i < nu) {
                    real<R>(G.x)[i] = real<R>(G.sx)[i];
                    real<R>(G.y)[i] = real<R>(G.sy)[i];
                    real<R>(G.vx)[i] = real<R>(G.svx)[i];
                    real<R>(G.vy)[i] = real<R>(G.svy)[i];
                    real<R>(G.w)[i] = real<R>(G.sw)[i];
                }
            }
        }
        return;
    }

    uint64_t q[kResRounds];
    uint64_t lsum = 0;
#pragma unroll
    for (int r = 0; r < kResRounds; ++r) {
        q[r] = fixed40(wl[r]);
        lsum += q[r];
    }
    const uint64_t lincl = wave_incl_scan(lsum);
    if (lane == kWave - 1) wave_tot[wave] = lincl;
    __syncthreads();
    uint64_t run = before;
    for (int w2 = 0; w2 < wave; ++w2) run += wave_tot[w2];
    const uint64_t wave_end = run + wave_tot[wave];

    const double U = (double)unit_f32(draw(G, 0u, cycle, kPurposeResample).x);
    const double spacing = __ddiv_rn((double)W, (double)nu);
    const double inv_spacing = 1.0 / spacing;
    const R out_w = (R)((double)W * 0x1p-40 / (double)nu);

    // draws [j0, j1) of this lane's sources (local index lane * kResRounds + r); they tile the
    // wave's range [j_begin, j_end) in source order
    uint32_t j0[kResRounds], j1[kResRounds];
    uint64_t F = run + lincl - lsum;
#pragma unroll
    for (int r = 0; r < kResRounds; ++r) {
        j0[r] = first_draw_at(F, U, spacing, inv_spacing, nu);
        F += q[r];
    }
    const uint32_t j_end = first_draw_at(wave_end, U, spacing, inv_spacing, nu);
    const uint32_t next_lane = __shfl_down(j0[0], 1, kWave);
#pragma unroll
    for (int r = 0; r < kResRounds - 1; ++r) j1[r] = j0[r + 1];
    j1[kResRounds - 1] = lane < kWave - 1 ? next_lane : j_end;
    const uint32_t j_begin = __shfl(j0[0], 0, kWave);

    const auto px = real<R>(born ? G.bx : G.sx);
    const auto py = real<R>(born ? G.by : G.sy);
    const auto pvx = real<R>(born ? G.bvx : G.svx);
    const auto pvy = real<R>(born ? G.bvy : G.svy);
    const auto X = real<R>(G.x), Y = real<R>(G.y), VX = real<R>(G.vx), VY = real<R>(G.vy);
    const auto Wt = real<R>(G.w);
    uint16_t* map = srcmap[wave];
    u32x4* mine = reinterpret_cast<u32x4*>(map + lane * kMapPerLane);
    uint32_t carry = 0;  // 1 + local index of the source that holds the window's first draw
    for (uint32_t wb = j_begin; wb < j_end; wb += kResWindow) {
        const uint32_t we = min(wb + (uint32_t)kResWindow, j_end);
        // the map gets 1 + the local index of every source whose draws start in the window, at
        // its first draw, and 0 elsewhere; a running maximum over the window then gives every
        // draw its source (sources ascend with their draws), in the same few steps however the
        // draws are spread over the sources.  The map is written and read by this wave only.
        mine[0] = u32x4{0u, 0u, 0u, 0u};
        mine[1] = u32x4{0u, 0u, 0u, 0u};
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < kResRounds; ++r)
            if (j0[r] < j1[r] && j0[r] >= wb && j0[r] < we)
                map[j0[r] - wb] = (uint16_t)(lane * kResRounds + r + 1);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        {
            const u32x4 h0 = mine[0], h1 = mine[1];
            uint32_t e[kMapPerLane];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                e[2 * i] = h0[i] & 0xFFFFu;
                e[2 * i + 1] = h0[i] >> 16;
                e[8 + 2 * i] = h1[i] & 0xFFFFu;
                e[8 + 2 * i + 1] = h1[i] >> 16;
            }
#pragma unroll
            for (int i = 1; i < kMapPerLane; ++i) e[i] = e[i] > e[i - 1] ? e[i] : e[i - 1];
            uint32_t incl = e[kMapPerLane - 1];
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const uint32_t o = __shfl_up(incl, off, kWave);
                if (lane >= off) incl = o > incl ? o : incl;
            }
            uint32_t excl = __shfl_up(incl, 1, kWave);
            excl = lane == 0 ? carry : (excl > carry ? excl : carry);
            u32x4 o0, o1;
#pragma unroll
            for (int i = 0; i < kMapPerLane; ++i) e[i] = e[i] > excl ? e[i] : excl;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                o0[i] = e[2 * i] | (e[2 * i + 1] << 16);
                o1[i] = e[8 + 2 * i] | (e[8 + 2 * i + 1] << 16);
            }
            mine[0] = o0;
            mine[1] = o1;
            const uint32_t last = __shfl(incl, kWave - 1, kWave);
            carry = last > carry ? last : carry;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        // four outputs per lane per step, their source reads issued together
        constexpr int kUnroll = 4;
        for (uint32_t j0s = wb + lane; j0s < we; j0s += kUnroll * kWave) {
            uint32_t src[kUnroll];
            R ox[kUnroll], oy[kUnroll], ovx[kUnroll], ovy[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t j = j0s + u * kWave;
                src[u] = j < we ? wbase + map[j - wb] - 1u : wbase;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                ox[u] = px[src[u]];
                oy[u] = py[src[u]];
                ovx[u] = pvx[src[u]];
                ovy[u] = pvy[src[u]];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t j = j0s + u * kWave;
                if (j < we) {
                    X[j] = ox[u];
                    Y[j] = oy[u];
                    VX[j] = ovx[u];
                    VY[j] = ovy[u];
                    Wt[j] = out_w;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

hipError_t launch_resample(const GridRef* g, int n, hipStream_t s)
{
    bool prefixed = false;
    if (const hipError_t e = launch_scan_parts(g, n, 1, &prefixed, s); e != hipSuccess) return e;
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [](const GridDev& G) {
        return xcd_blocks(G.n_res_ptiles + G.n_res_btiles);
    });
    if (blocks) {
        // one kernel per launch (the results do not depend on it): the balanced one if any grid's
        // plan asks for it
        bool balanced = false;
        for (int i = 0; i < n; ++i) {
            const uint32_t mode = g[i].hd->resample;
            balanced |= mode == 1 || (mode == 0 && g[i].hd->nu > kBalancedFrom);
        }
        const bool r64 = launch_real64(g, n);
        if (balanced)
            DOGM_LAUNCH_REAL(r64, "k_resample", k_resample, dim3(blocks), dim3(kResThreads), 0, s, b,
                             prefixed ? 1 : 0);
        else
            DOGM_LAUNCH_REAL(r64, "k_resample", k_resample_windowed, dim3(blocks),
                             dim3(kResThreads), 0, s, b, prefixed ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace dogm
