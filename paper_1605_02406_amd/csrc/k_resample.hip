// Alg. 7: systematic resampling of nu particles from the joint set [sorted persistent | new-born].
//
// The CDF is an exact integer prefix sum of the weights in 2^-40 fixed point, so it does not
// depend on the summation order; the per-tile totals were accumulated by the kernels that wrote
// the weights.  Draw j sits at u_j = (j + U) d with the spacing d = W / nu rounded once to FP64,
// and selects the first particle i with F_i > floor(u_j); for nu < 2^27 the last draw stays
// below W by more than the roundings of W, d and the product (1 - U >= 2^-24, so the margin is
// at least 2^-24 / nu of W against three half-ulps), so every draw finds a particle.
// Source i receives the draws J(F_{i-1}) <= j < J(F_i) with J(F) = min{ j : floor(u_j) >= F }.
// One kernel: each tile adds up the totals of the tiles before it and scans its own weights
// with wave prefix sums.  The draws of a wave's sources form one contiguous range; the wave
// walks it in windows: every lane writes the local index of each of its sources into the
// window's LDS map at the source's draws, then the wave writes the window's outputs in order,
// so stores are coalesced and source reads ascend.
#include "launch.h"

namespace dogm {

constexpr int kResWaves = kResThreads / kWave;
constexpr int kResRounds = kResItems;  // each wave owns kResRounds * 64 consecutive items
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

constexpr int kResWindow = 1024;  // draws per LDS map window of a wave

__global__ __launch_bounds__(kResThreads) void k_resample(Batch b)
{
    constexpr int kSrc = kResRounds * kWave;  // sources per wave
    static_assert(kSrc <= 65536, "local source indices are 16-bit");
    __shared__ uint64_t tmp[kResWaves + 1];
    __shared__ uint64_t wave_tot[kResWaves];  // each wave's weight total
    __shared__ uint16_t srcmap[kResWaves][kResWindow];
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

    // each lane owns kResRounds consecutive sources; this wave's weights are read first so
    // their loads overlap the prefix below
    const uint32_t lbase = wbase + lane * kResRounds;
    const auto wsrc = born ? G.bw : G.sw;
    float wl[kResRounds];
    if (lbase + kResRounds <= n_src) {  // whole 16-byte vectors
#pragma unroll
        for (int r = 0; r < kResRounds; r += 4) {
            const f32x4 v = wsrc.load_vec<f32x4>(lbase + r);
#pragma unroll
            for (int e = 0; e < 4; ++e) wl[r + e] = v[e];
        }
    } else {
#pragma unroll
        for (int r = 0; r < kResRounds; ++r) {
            const uint32_t i = lbase + r;
            wl[r] = i < n_src ? wsrc[i] : 0.0f;
        }
    }

    // joint weight before this tile and in total, from the partial sums of the persistent tiles
    // (kResTile particles each) and of the new-born tiles (kBornTile slots each)
    const uint32_t nparts = G.n_res_ptiles + G.n_born_parts;
    const uint32_t limit = born ? G.n_res_ptiles + t_local * (kResTile / kBornTile) : tile;
    uint64_t before = 0, all = 0;
    for (uint32_t t0 = threadIdx.x; t0 < nparts; t0 += 4 * kResThreads) {
        uint64_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t t = t0 + u * kResThreads;
            v[u] = t < nparts ? G.rpart[t] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            all += v[u];
            if (t0 + u * kResThreads < limit) before += v[u];
        }
    }
    before = block_sum(before, tmp);
    const uint64_t W = block_sum(all, tmp);
    if (tile == 0 && threadIdx.x == 0) *G.W_fixed = W;

    if (W == 0) {  // nothing carries weight: keep the sorted persistent set as it is
        if (!born) {
            for (int r = 0; r < kResRounds; ++r) {
                const uint32_t i = wbase + r * kWave + lane;
                if (i < nu) {
                    G.x[i] = G.sx[i];
                    G.y[i] = G.sy[i];
                    G.vx[i] = G.svx[i];
                    G.vy[i] = G.svy[i];
                    G.w[i] = G.sw[i];
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
    const float out_w = (float)((double)W * 0x1p-40 / (double)nu);

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

    const auto px = born ? G.bx : G.sx;
    const auto py = born ? G.by : G.sy;
    const auto pvx = born ? G.bvx : G.svx;
    const auto pvy = born ? G.bvy : G.svy;
    uint16_t* map = srcmap[wave];
    for (uint32_t wb = j_begin; wb < j_end; wb += kResWindow) {
        const uint32_t we = min(wb + (uint32_t)kResWindow, j_end);
#pragma unroll
        for (int r = 0; r < kResRounds; ++r) {
            const uint32_t lo = j0[r] > wb ? j0[r] : wb;
            const uint32_t hi = j1[r] < we ? j1[r] : we;
            for (uint32_t j = lo; j < hi; ++j) map[j - wb] = (uint16_t)(lane * kResRounds + r);
        }
        // the map is written and read by this wave only
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        // four outputs per lane per step, their source reads issued together
        constexpr int kUnroll = 4;
        for (uint32_t j0s = wb + lane; j0s < we; j0s += kUnroll * kWave) {
            uint32_t src[kUnroll];
            float ox[kUnroll], oy[kUnroll], ovx[kUnroll], ovy[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t j = j0s + u * kWave;
                src[u] = j < we ? wbase + map[j - wb] : wbase;
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
                    G.x[j] = ox[u];
                    G.y[j] = oy[u];
                    G.vx[j] = ovx[u];
                    G.vy[j] = ovy[u];
                    G.w[j] = out_w;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

hipError_t launch_resample(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [](const GridDev& G) {
        return xcd_blocks(G.n_res_ptiles + G.n_res_btiles);
    });
    if (blocks) DOGM_LAUNCH(k_resample, dim3(blocks), dim3(kResThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace dogm
