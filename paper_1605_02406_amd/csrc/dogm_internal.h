// Internal definitions shared by the gfx950 kernels and the host side of libdogm.
//
// Design: every array of a grid lives in one caller-owned device arena whose first bytes hold
// a GridDev descriptor (pointers + parameters).  Every kernel takes a Batch by value: the
// descriptors of up to kMaxBatch grids plus the first block of each grid in the launch, so one
// launch serves one grid or a batch of grids of different sizes alike.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dogm {

constexpr int kMaxBatch = 32;
constexpr int kWave = 64;

// Philox counter word 2: what a draw is for.
constexpr uint32_t kPurposeInit = 0, kPurposePredict = 1, kPurposeBirth = 2,
                   kPurposeResample = 3;

constexpr uint32_t kStConflict = 1u, kStNoCarrier = 2u, kStNonFinite = 4u, kStInternal = 8u;

// Radix sort of the cell keys: tiles of kSortTile keys, digits of at most 8 bits.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096
constexpr int kMaxDigitBits = 8;
constexpr int kMaxPasses = 4;

// Generic scans: tiles of kScanTile elements.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

// Segmented per-cell reductions: each wave owns kSegRange particles.
constexpr int kSegThreads = 256;
constexpr int kSegRange = 512;
constexpr int kSegBlockParticles = (kSegThreads / kWave) * kSegRange;  // 2048

// Resampling: tiles of the joint particle array.
constexpr int kResThreads = 256;
constexpr int kResItems = 8;
constexpr int kResTile = kResThreads * kResItems;  // 2048

constexpr int kElemThreads = 256;  // element-wise kernels

struct GridDev {
    // parameters
    int32_t nx, ny;
    uint32_t C, nu, nb;
    float r, dt, p_s, p_b, sig_pos, sig_vel, sig_birth, alpha;
    uint32_t seed_lo, seed_hi, grid_id;
    uint32_t n_sort_tiles, n_res_tiles;
    // persistent particles (start of a cycle / after resampling)
    float *x, *y, *vx, *vy, *w;
    uint32_t* key;
    // sorted particles
    float *sx, *sy, *svx, *svy, *sw;
    uint32_t *skey, *perm;
    // radix sort scratch
    uint32_t *tkey, *tval;  // ping-pong partner of (skey, perm)
    uint32_t* hist;         // digit-major counts, 2^kMaxDigitBits * n_sort_tiles
    // cells
    uint32_t *cstart, *cend;
    double *sum_w, *sum_wt;
    float *m_pO, *m_pF, *m_O, *m_F, *rho_b, *rho_p, *pign;
    double *mu_A, *mu_UA;
    uint64_t* born_q;  // fixed-point rho_b, then its exclusive prefix sum
    uint32_t* born_off;
    float *mean_x, *mean_y, *var_x, *var_y, *cov_xy;
    uint8_t* mflag;
    // new-born particles
    float *bx, *by, *bvx, *bvy, *bw;
    uint32_t* bkey;
    uint8_t* bassoc;
    // resampling scratch
    uint64_t* res_tile;  // per-tile weight sums, then their exclusive prefix
    int32_t* res_last;   // per-tile last positive-weight index
    // generic scan scratch (per-tile partial sums)
    uint64_t* scan_part;
    // device scalars
    uint32_t* cycle;
    uint32_t* status;
    uint64_t* W_fixed;
    uint64_t* S_fixed;
    int32_t* last_pos;
    double* U;
};

struct MeasDev {
    const float *m_occ, *m_free, *p_assoc, *mu_vx, *mu_vy, *var_v;
};

struct Batch {
    int n;
    uint32_t bstart[kMaxBatch + 1];  // first block of grid i; bstart[n] = blocks in the launch
    const GridDev* g[kMaxBatch];
    MeasDev m[kMaxBatch];
};

// Grid of this block and the block's index within the grid.
__device__ __forceinline__ int batch_grid(const Batch& b)
{
    int gi = 0;
    for (int i = 1; i < b.n; ++i) gi = (blockIdx.x >= b.bstart[i]) ? i : gi;
    return gi;
}

// --------------------------------------------------------------------------------------------
// Random numbers: Philox4x32-10 (Salmon et al., SC'11), uniform and Box-Muller in FP32.
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint32_t key_lo, uint32_t key_hi)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t a = ctr.x, b = ctr.y, c = ctr.z, d = ctr.w;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t ka = key_lo + W0 * (uint32_t)round;
        const uint32_t kb = key_hi + W1 * (uint32_t)round;
        const uint32_t hi_a = __umulhi(M0, a), lo_a = M0 * a;
        const uint32_t hi_c = __umulhi(M1, c), lo_c = M1 * c;
        a = hi_c ^ b ^ ka;
        b = lo_c;
        c = hi_a ^ d ^ kb;
        d = lo_a;
    }
    return make_uint4(a, b, c, d);
}

__device__ __forceinline__ uint4 draw(const GridDev& G, uint32_t index, uint32_t cycle,
                                      uint32_t purpose)
{
    return philox4x32_10(make_uint4(index, cycle, purpose, G.grid_id), G.seed_lo, G.seed_hi);
}

// (0,1): the 23 high bits plus one half, scaled by 2^-23; exact in FP32.
__device__ __forceinline__ float unit_f32(uint32_t bits)
{
    return ((float)(bits >> 9) + 0.5f) * 0x1p-23f;
}

__device__ __forceinline__ void box_muller_f32(float u1, float u2, float& n1, float& n2)
{
    const float radius = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    n1 = radius * c;
    n2 = radius * s;
}

// Cell of an FP32 position: one correctly rounded FP32 division per axis, C outside the grid.
__device__ __forceinline__ uint32_t cell_of(const GridDev& G, float x, float y)
{
    const float fx = x / G.r;
    const float fy = y / G.r;
    if (!(fx >= 0.0f && fx < (float)G.nx && fy >= 0.0f && fy < (float)G.ny)) return G.C;
    return (uint32_t)fy * (uint32_t)G.nx + (uint32_t)fx;
}

// Mass in fixed point: multiples of 2^-40, rounded to nearest (exact for FP32 input).
__device__ __forceinline__ uint64_t fixed40(float m)
{
    if (!(m > 0.0f)) return 0;
    return (uint64_t)floor((double)m * 0x1p40 + 0.5);
}

// --------------------------------------------------------------------------------------------
// Wave-level helpers (wave64).
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v)
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v)
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (blockDim.x = nthreads, multiple of 64).
// `lds` must hold nthreads/64 + 1 entries.  Returns the exclusive prefix; *total receives the
// block total.  Contains __syncthreads().
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T* total)
{
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    T incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const T o = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += o;
    }
    if (lane == kWave - 1) lds[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int i = 0; i < nwaves; ++i) {
            const T t = lds[i];
            lds[i] = acc;
            acc += t;
        }
        lds[nwaves] = acc;
    }
    __syncthreads();
    const T res = lds[wave] + incl - v;
    *total = lds[nwaves];
    __syncthreads();
    return res;
}

}  // namespace dogm
