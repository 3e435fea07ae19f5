// Alg. 7: systematic resampling of nu particles from the joint set [sorted persistent | new-born].
//
// The CDF is an exact integer prefix sum of the weights in 2^-40 fixed point, so it does not
// depend on the summation order.  Draw j sits at u_j = (j + U) W / nu (FP64, every operation
// rounded separately) and selects the first particle i with F_i > floor(u_j).  Instead of a
// search per draw, every source particle computes the range of draws that land in its CDF
// interval, J(F_{i-1}) <= j < J(F_i) with J(F) = min{ j : floor(u_j) >= F }, and writes its
// copies there: three passes (tile sums, a per-grid scan of them, the scatter), all reads
// coalesced, writes in increasing j across the lanes of a wave.
#include "launch.h"

namespace dogm {

constexpr int kResWaves = kResThreads / kWave;
constexpr int kResRounds = kResItems;  // each wave owns kResRounds * 64 consecutive items

__device__ __forceinline__ float joint_weight(const GridDev& G, uint32_t i)
{
    return i < G.nu ? G.sw[i] : G.bw[i - G.nu];
}

__device__ __forceinline__ uint64_t draw_floor(uint32_t j, double U, double Wd, double nu)
{
    const double u = __ddiv_rn(__dmul_rn(__dadd_rn((double)j, U), Wd), nu);
    return (uint64_t)floor(u);
}

// min { j in [0, nu] : floor(u_j) >= F }, with u_nu taken as +infinity.
__device__ __forceinline__ uint32_t first_draw_at(uint64_t F, double U, double Wd, uint32_t nu)
{
    const double dnu = (double)nu;
    double est = ceil((double)F * dnu / Wd - U);
    est = est < 0.0 ? 0.0 : (est > dnu ? dnu : est);
    uint32_t j = (uint32_t)est;
    while (j > 0 && draw_floor(j - 1, U, Wd, dnu) >= F) --j;
    while (j < nu && draw_floor(j, U, Wd, dnu) < F) ++j;
    return j;
}

__global__ __launch_bounds__(kResThreads) void k_res_tiles(Batch b)
{
    __shared__ uint64_t tmp[kResWaves + 1];
    __shared__ int32_t last;
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t tile = blockIdx.x - b.bstart[gi];
    const uint32_t N = G.nu + G.nb;
    if (threadIdx.x == 0) last = -1;
    __syncthreads();
    uint64_t acc = 0;
    int32_t my_last = -1;
    for (int it = 0; it < kResItems; ++it) {
        const uint32_t i = tile * kResTile + it * kResThreads + threadIdx.x;
        if (i < N) {
            const uint64_t q = fixed40(joint_weight(G, i));
            acc += q;
            if (q) my_last = (int32_t)i;
        }
    }
    if (my_last >= 0) atomicMax(&last, my_last);
    uint64_t total;
    block_excl_scan<uint64_t>(acc, tmp, &total);
    if (threadIdx.x == 0) {
        G.res_tile[tile] = total;
        G.res_last[tile] = last;
    }
}

__global__ __launch_bounds__(kResThreads) void k_res_mid(Batch b)
{
    __shared__ uint64_t tmp[kResWaves + 1];
    __shared__ int32_t last;
    const GridDev& G = *b.g[blockIdx.x];
    if (threadIdx.x == 0) last = -1;
    __syncthreads();
    uint64_t carry = 0;
    int32_t my_last = -1;
    for (uint32_t base = 0; base < G.n_res_tiles; base += kResThreads) {
        const uint32_t t = base + threadIdx.x;
        const uint64_t v = t < G.n_res_tiles ? G.res_tile[t] : 0;
        if (t < G.n_res_tiles && G.res_last[t] > my_last) my_last = G.res_last[t];
        uint64_t chunk;
        const uint64_t ex = block_excl_scan<uint64_t>(v, tmp, &chunk);
        if (t < G.n_res_tiles) G.res_tile[t] = carry + ex;
        carry += chunk;
    }
    if (my_last >= 0) atomicMax(&last, my_last);
    __syncthreads();
    if (threadIdx.x == 0) {
        *G.W_fixed = carry;
        *G.last_pos = last;
        *G.U = (double)unit_f32(draw(G, 0u, *G.cycle, kPurposeResample).x);
    }
}

__global__ __launch_bounds__(kResThreads) void k_res_scatter(Batch b)
{
    __shared__ uint64_t wave_tot[kResWaves + 1];
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t tile = blockIdx.x - b.bstart[gi];
    const uint32_t nu = G.nu, N = nu + G.nb;
    const uint64_t W = *G.W_fixed;
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    if (tile == 0 && threadIdx.x == 0) *G.cycle += 1u;

    if (W == 0) {  // nothing carries weight: keep the sorted persistent set as it is
        for (int it = 0; it < kResItems; ++it) {
            const uint32_t i = tile * kResTile + it * kResThreads + threadIdx.x;
            if (i < nu) {
                G.x[i] = G.sx[i];
                G.y[i] = G.sy[i];
                G.vx[i] = G.svx[i];
                G.vy[i] = G.svy[i];
                G.w[i] = G.sw[i];
            }
        }
        return;
    }

    const uint32_t wbase = tile * kResTile + wave * (kResRounds * kWave);
    uint64_t q[kResRounds];
    uint64_t wsum = 0;
#pragma unroll
    for (int r = 0; r < kResRounds; ++r) {
        const uint32_t i = wbase + r * kWave + lane;
        q[r] = i < N ? fixed40(joint_weight(G, i)) : 0;
        wsum += q[r];
    }
    // wave totals -> offsets of the waves inside the tile
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) wsum += __shfl_xor(wsum, off, kWave);
    if (lane == 0) wave_tot[wave] = wsum;
    __syncthreads();
    uint64_t run = G.res_tile[tile];
    for (int w2 = 0; w2 < wave; ++w2) run += wave_tot[w2];

    const double U = *G.U;
    const double Wd = (double)W;
    const int32_t last = *G.last_pos;
    const float out_w = (float)((double)W * 0x1p-40 / (double)nu);
#pragma unroll
    for (int r = 0; r < kResRounds; ++r) {
        const uint32_t i = wbase + r * kWave + lane;
        const uint64_t incl = wave_incl_scan_u64(q[r]);
        const uint64_t F_hi = run + incl;
        const uint64_t F_lo = F_hi - q[r];
        run += __shfl(incl, kWave - 1, kWave);
        if (i >= N || q[r] == 0) continue;
        const uint32_t j0 = first_draw_at(F_lo, U, Wd, nu);
        const uint32_t j1 = ((int32_t)i == last) ? nu : first_draw_at(F_hi, U, Wd, nu);
        if (j0 >= j1) continue;
        float px, py, pvx, pvy;
        if (i < nu) {
            px = G.sx[i];
            py = G.sy[i];
            pvx = G.svx[i];
            pvy = G.svy[i];
        } else {
            const uint32_t k = i - nu;
            px = G.bx[k];
            py = G.by[k];
            pvx = G.bvx[k];
            pvy = G.bvy[k];
        }
        for (uint32_t j = j0; j < j1; ++j) {
            G.x[j] = px;
            G.y[j] = py;
            G.vx[j] = pvx;
            G.vy[j] = pvy;
            G.w[j] = out_w;
        }
    }
}

hipError_t launch_resample(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [](const GridDev& G) { return G.n_res_tiles; });
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_res_tiles, dim3(blocks), dim3(kResThreads), 0, s, b);
    hipLaunchKernelGGL(k_res_mid, dim3(n), dim3(kResThreads), 0, s, b);
    hipLaunchKernelGGL(k_res_scatter, dim3(blocks), dim3(kResThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace dogm
