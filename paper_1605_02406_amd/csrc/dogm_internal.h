// Internal definitions shared by the gfx950 kernels and the host side of libdogm.
//
// Design: every array of a grid lives in one caller-owned device arena whose first bytes hold
// a GridDev descriptor (pointers + parameters).  Every kernel takes a Batch by value: the
// descriptors of up to kMaxBatch grids plus the first block of each grid in the launch, so one
// launch serves one grid or a batch of grids of different sizes alike.
//
// Blocks never talk to each other inside a kernel (no atomics on shared counters, no spinning):
// every block stores its partial results (digit counts of a tile, fixed-point sums of a tile)
// and the next kernel combines them.  On a chip of eight dies, device-wide atomics and coherent
// polling cost far more than a kernel boundary.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dogm {

constexpr int kMaxBatch = 32;
constexpr int kWave = 64;
constexpr int kMaxBlockWaves = 1024 / kWave;  // waves of the largest block

// Philox counter word 2: what a draw is for.
constexpr uint32_t kModelPhdMib = 1;  // the particle PHD/MIB model of Sec. V (else Sec. VI)
constexpr uint32_t kPurposeInit = 0, kPurposePredict = 1, kPurposeBirth = 2,
                   kPurposeResample = 3;

constexpr uint32_t kStConflict = 1u, kStNoCarrier = 2u, kStNonFinite = 4u, kStInternal = 8u;

// Radix sort of the cell keys: tiles of kSortTile keys, digits of at most kSortBits bits.
constexpr int kSortThreads = 1024;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096
constexpr int kSortBits = 11;
constexpr int kSortBins = 1 << kSortBits;  // 2048
constexpr int kMaxPasses = 3;              // keys <= C < 2^24 (C is the outside key)
constexpr int kScanRowThreads = 256;       // one block scans a few digit rows of the histogram
constexpr int kHistTile = kSortTile;       // keys per digit-histogram tile
constexpr int kHistThreads = 1024;         // histogram blocks: kHistTile / kHistThreads keys each
constexpr uint32_t kNoCell = 0xFFFFFFFFu;

// Cells: one per thread, partial sums per block of kCellThreads cells.
constexpr int kCellThreads = 256;

// Fixed-point partial sums of the joint weights (persistent tiles, then new-born tiles) and of
// the new-born masses (cell tiles) are written per tile of 2048 elements.

// Segmented per-cell reductions: each wave owns 64 * kSegItems particles.
constexpr int kSegThreads = 256;
constexpr int kCellSums = 6;  // FP64 sums per cell without velocity evidence: one 48-byte record
constexpr int kSegItems = 8;
constexpr int kSegRange = kWave * kSegItems;                           // 512
static_assert(kSegItems % 4 == 0, "a lane reads its items as 16-byte vectors");
constexpr int kSegBlockParticles = (kSegThreads / kWave) * kSegRange;  // 2048

// New-born slots are initialised in tiles of kBornTile slots (one per thread); their fixed-point
// weight sums follow the persistent tiles' sums in the resampling's list of partial sums.
constexpr int kBornTile = 256;

// Resampling: tiles of persistent particles, then tiles of new-born slots; the joint weight of
// each tile is a fixed-point partial sum formed by the persistent weight update.
constexpr int kResThreads = 256;
constexpr int kResItems = 4;
constexpr int kResTile = kResThreads * kResItems;  // 1024
static_assert(kResTile % kBornTile == 0, "a resampling tile covers whole new-born tiles");
// The persistent weight update walks kPtSplit resampling tiles per block.
constexpr int kPtSplit = 2;
constexpr int kPtItems = kResItems * kPtSplit;
constexpr int kPtTile = kResTile * kPtSplit;  // 2048

constexpr int kElemThreads = 256;  // element-wise kernels

// The grid descriptor, over a pointer kind: the host builds and stores it with plain pointers
// (GridDev); kernels read a private copy whose pointers are in the global address space
// (GridView), so every array access uses the global memory instructions, which do not share
// the wait counter of LDS operations and cross-lane shuffles, and nothing is reloaded after a
// store.  Both kinds have the same layout.
template <typename T>
using HostPtr = T*;
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) T*;
template <typename T>
using ConstPtr = __attribute__((address_space(4))) const T*;  // read-only while a kernel runs

// A device array seen by a kernel: a global-address-space pointer whose element access forms
// the byte offset in 32 bits (every array holds fewer than 2^30 elements of at most 8 bytes),
// so the compiler addresses it with a scalar base and one 32-bit offset register instead of a
// 64-bit address pair per access.  Same size and bits as a plain pointer.
using u32x4 = uint32_t __attribute__((ext_vector_type(4)));
using f32x4 = float __attribute__((ext_vector_type(4)));
using f64x2 = double __attribute__((ext_vector_type(2)));
// A 16-byte vector of real values: four FP32 or two FP64 elements.
template <typename R>
struct RealVec16 {
    using type = f32x4;
};
template <>
struct RealVec16<double> {
    using type = f64x2;
};

template <typename T>
struct GArr {
    GlobalPtr<T> p;
    __device__ __forceinline__ __attribute__((address_space(1))) T& operator[](uint32_t i) const
    {
        using Byte = __attribute__((address_space(1))) unsigned char;
        return *(GlobalPtr<T>)((Byte*)(GlobalPtr<void>)p + i * (uint32_t)sizeof(T));
    }
    __device__ __forceinline__ __attribute__((address_space(1))) T& operator*() const { return *p; }
    __device__ __forceinline__ explicit operator bool() const { return p != nullptr; }
    // V = a vector of sizeof(V) / sizeof(T) elements from element i (aligned to sizeof(V))
    template <typename V>
    __device__ __forceinline__ V load_vec(uint32_t i) const
    {
        using Byte = __attribute__((address_space(1))) unsigned char;
        return *(__attribute__((address_space(1))) const V*)((Byte*)(GlobalPtr<void>)p +
                                                             i * (uint32_t)sizeof(T));
    }
    template <typename V>
    __device__ __forceinline__ void store_vec(uint32_t i, const V& v) const
    {
        using Byte = __attribute__((address_space(1))) unsigned char;
        *(__attribute__((address_space(1))) V*)((Byte*)(GlobalPtr<void>)p + i * (uint32_t)sizeof(T)) =
            v;
    }
};

template <template <typename> class P>
struct GridT {
    // parameters
    int32_t nx, ny;
    uint32_t C, nu, nb;
    float r, dt, p_s, p_b, sig_pos, sig_vel, sig_birth, alpha;
    uint32_t seed_lo, seed_hi, grid_id;
    uint32_t model;  // kModelPhdMib: Sec. V; otherwise the Dempster-Shafer model of Sec. VI
    uint32_t real64;  // 1: the real-valued arrays hold FP64 (all-FP64 precision mode), else FP32
    uint32_t scan_parts;  // prefix of the partial sums: 0 automatic, 1 always scanned, 2 never
    uint32_t resample;    // resampling kernel: 0 automatic, 1 outputs shared evenly, 2 by owner
    // sort plan (from the largest key, C) and tilings
    uint32_t passes;
    uint32_t dshift[kMaxPasses], dbits[kMaxPasses];
    uint32_t n_sort_tiles, n_hist_tiles, n_cell_parts, n_res_ptiles, n_res_btiles, n_born_parts;
    // persistent particles (start of a cycle / after resampling) and their cell keys
    P<float> x, y, vx, vy, w;
    P<uint32_t> key;
    // particles sorted by cell
    P<float> sx, sy, svx, svy, sw;
    P<uint32_t> skey, perm;
    // ping-pong partner of the sorted arrays during the sort
    P<float> tx, ty, tvx, tvy, tw;
    P<uint32_t> tkey, tval;
    // cells
    P<uint32_t> cstart, cend;
    P<double> sum_w, sum_wt;
    P<double> msum;  // [C][kCellSums]: per cell the sums of w, w vx, w vy, w vx^2, w vy^2, w vx vy
    P<float> m_pO, m_pF, m_O, m_F, rho_b, rho_p, pign;
    P<double> mu_A, mu_UA;
    P<uint32_t> born_off;
    P<float> mean_x, mean_y, var_x, var_y, cov_xy;
    P<uint8_t> mflag;
    // new-born particles
    P<float> bx, by, bvx, bvy, bw;
    P<uint32_t> bkey;
    P<uint8_t> bassoc;
    // per-cycle scratch: digit histograms of every sort tile (digit-major,
    // [kSortBins][n_hist_tiles]) with their row totals, fixed-point partial sums of new-born
    // masses (per 256 cells) and of joint weights (per persistent resampling tile, then per
    // new-born tile), each array turned into exclusive prefixes in place with the total in one
    // extra entry, the first slot of every cell with births (its cell id, kNoCell
    // elsewhere) and the cell of the first slot of every new-born tile
    P<uint32_t> hist, rowtot;
    P<uint64_t> bpart, rpart;
    P<uint32_t> born_mark, tile_first;
    // device scalars: the cycle to run next (advanced by the resampling) and the cycle being
    // run (set by the prediction); every writer of either stores one and the same value
    P<uint32_t> cycle;
    P<uint32_t> cycle_run;
    P<uint32_t> status;
    P<uint32_t> nc_flag;  // kStNoCarrier once any cell lacked a slot (plain stores, sticky)
    P<uint64_t> W_fixed;
    P<uint64_t> S_fixed;
};
using GridDev = GridT<HostPtr>;
using GridView = GridT<GArr>;
static_assert(sizeof(GridDev) == sizeof(GridView), "one layout for both pointer kinds");

template <template <typename> class P>
struct MeasT {
    P<const float> m_occ, m_free, p_assoc, mu_vx, mu_vy, var_v;
    P<const float> p_tp, p_fp, det;  // the particle PHD/MIB model's observation (Sec. V.C)
};
using MeasDev = MeasT<HostPtr>;
using MeasView = MeasT<GArr>;
static_assert(sizeof(MeasDev) == sizeof(MeasView), "one layout for both pointer kinds");

struct Batch {
    int n;
    uint32_t bstart[kMaxBatch + 1];  // first block of grid i; bstart[n] = blocks in the launch
    const GridDev* g[kMaxBatch];
    MeasDev m[kMaxBatch];
};
static_assert(sizeof(Batch) <= 4096, "a batch descriptor is one kernel argument");

// Real-valued arrays (particle state; per-cell masses, normalised weights and moments) hold FP32
// elements, or FP64 in the all-FP64 precision mode; their descriptor entries are typed as FP32
// and kernels templated on the real type R see them through real<R>().
template <typename R>
__device__ __forceinline__ GArr<R> real(const GArr<float>& a)
{
    return GArr<R>{(GlobalPtr<R>)(GlobalPtr<void>)a.p};
}

// Private copies of a grid's descriptor and measurement with global-address-space pointers.
// The descriptor is read through the constant address space (it is never written while a
// kernel runs), so its fields arrive by scalar loads into scalar registers.
static_assert(sizeof(GridView) % 8 == 0, "the descriptor is copied in 8-byte words");
__device__ __forceinline__ GridView grid_view(const GridDev* p)
{
    const auto src = (ConstPtr<uint64_t>)(const void*)p;
    GridView v;
#pragma unroll
    for (size_t i = 0; i < sizeof(GridView) / 8; ++i) {
        const uint64_t word = src[i];
        __builtin_memcpy(reinterpret_cast<char*>(&v) + 8 * i, &word, 8);
    }
    return v;
}

// Digit position and width of sort pass `pass` (read from the descriptor in memory: indexing
// the private copy with a run-time pass number would place it in scratch).
__device__ __forceinline__ uint32_t pass_shift(const GridDev* p, uint32_t pass)
{
    return ((ConstPtr<GridDev>)(const void*)p)->dshift[pass];
}
__device__ __forceinline__ uint32_t pass_bits(const GridDev* p, uint32_t pass)
{
    return ((ConstPtr<GridDev>)(const void*)p)->dbits[pass];
}
__device__ __forceinline__ MeasView meas_view(const MeasDev& m)
{
    MeasView v;
    __builtin_memcpy(&v, (const void*)&m, sizeof(v));
    return v;
}

// Sets status bits of a grid (a device-wide atomic OR; rare events only).
__device__ __forceinline__ void status_or(const GridView& G, uint32_t bits)
{
    atomicOr((uint32_t*)G.status.p, bits);
}
__device__ __forceinline__ void status_or(const GridDev& G, uint32_t bits)
{
    atomicOr(G.status, bits);
}

// Grid of this block and the block's index within the grid.
__device__ __forceinline__ int batch_grid(const Batch& b)
{
    int gi = 0;
    for (int i = 1; i < b.n; ++i) gi = (blockIdx.x >= b.bstart[i]) ? i : gi;
    return gi;
}

__device__ __forceinline__ uint32_t ceil_div_u32(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Workgroups are dealt to the eight XCDs (each with its own L2) in turn.  For kernels whose
// neighbouring tiles share data (adjacent output runs, overlapping inputs), each grid's blocks
// are padded to a multiple of 8 and block i of XCD slot i % 8 takes tile (i % 8) * per + i / 8:
// every XCD walks one contiguous run of tiles.  Returns a tile >= the grid's tile count for
// padding blocks, which exit.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(const Batch& b, int gi)
{
    const uint32_t lb = blockIdx.x - b.bstart[gi];
    const uint32_t per = (b.bstart[gi + 1] - b.bstart[gi]) / kXcds;
    return (lb % kXcds) * per + lb / kXcds;
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
        // each product as one 32 x 32 -> 64-bit multiply (both halves from one instruction)
        const uint64_t pa = (uint64_t)M0 * a, pc = (uint64_t)M1 * c;
        const uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        const uint32_t hi_c = (uint32_t)(pc >> 32), lo_c = (uint32_t)pc;
        a = hi_c ^ b ^ ka;
        b = lo_c;
        c = hi_a ^ d ^ kb;
        d = lo_a;
    }
    return make_uint4(a, b, c, d);
}

__device__ __forceinline__ uint4 draw(const GridView& G, uint32_t index, uint32_t cycle,
                                      uint32_t purpose)
{
    return philox4x32_10(make_uint4(index, cycle, purpose, G.grid_id), G.seed_lo, G.seed_hi);
}

// (0,1): the 23 high bits plus one half, scaled by 2^-23; exact in FP32.
__device__ __forceinline__ float unit_f32(uint32_t bits)
{
    return ((float)(bits >> 9) + 0.5f) * 0x1p-23f;
}

// Box-Muller on the transcendental units: v_log_f32 is log2, v_sqrt_f32 the square root and
// v_sin_f32 / v_cos_f32 take their argument in revolutions, so sin(2 pi u2) is one instruction.
// Each is accurate to a few units in the last place, far inside the position and velocity
// tolerances; the cell key is decided afterwards from the stored FP32 position.
__device__ __forceinline__ void box_muller_f32(float u1, float u2, float& n1, float& n2)
{
    const float ln_u1 = __builtin_amdgcn_logf(u1) * 0.693147180559945309f;  // ln 2
    const float radius = __builtin_amdgcn_sqrtf(-2.0f * ln_u1);
    n1 = radius * __builtin_amdgcn_cosf(u2);
    n2 = radius * __builtin_amdgcn_sinf(u2);
}

// Box-Muller in FP64 (the all-FP64 precision mode), on the device's double-precision log,
// square root, cosine and sine.
__device__ __forceinline__ void box_muller_f64(double u1, double u2, double& n1, double& n2)
{
    const double radius = sqrt(-2.0 * log(u1));
    const double a = 6.283185307179586476925286766559 * u2;
    n1 = radius * cos(a);
    n2 = radius * sin(a);
}

template <typename R>
__device__ __forceinline__ void box_muller(R u1, R u2, R& n1, R& n2)
{
    if constexpr (sizeof(R) == 8) box_muller_f64(u1, u2, n1, n2);
    else box_muller_f32(u1, u2, n1, n2);
}

// Cell of a position: one correctly rounded division per axis in the position's precision, C
// outside the grid.
template <typename R>
__device__ __forceinline__ uint32_t cell_of(const GridView& G, R x, R y)
{
    const R fx = x / (R)G.r;
    const R fy = y / (R)G.r;
    if (!(fx >= (R)0 && fx < (R)G.nx && fy >= (R)0 && fy < (R)G.ny)) return G.C;
    return (uint32_t)fy * (uint32_t)G.nx + (uint32_t)fx;
}

// Mass in fixed point: multiples of 2^-40, rounded to nearest (halves up).
__device__ __forceinline__ uint64_t fixed40(double m)
{
    if (!(m > 0.0)) return 0;
    return (uint64_t)floor(m * 0x1p40 + 0.5);
}
__device__ __forceinline__ uint64_t fixed40(float m) { return fixed40((double)m); }

// --------------------------------------------------------------------------------------------
// Wave- and block-level helpers (wave64).
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// a * b + c rounded twice, as written: where an integer decision depends on the value and the
// other side of a comparison computes it the same way, it must not become a fused multiply-add
// (device code contracts a * b + c by default).
__device__ __forceinline__ double mul_add_twice_rounded(double a, double b, double c)
{
#pragma clang fp contract(off)
    return a * b + c;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const T o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int32_t wave_max(int32_t v)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Adds one key's digit to the block's LDS histogram (counts need no order, so a plain LDS
// atomic; lanes that hit the same bin are serialised by the LDS, not by instructions).
__device__ __forceinline__ void digit_count(bool valid, uint32_t d, uint32_t* cnt)
{
    if (valid) atomicAdd(&cnt[d], 1u);
}

// Block-wide exclusive scan of one value per thread (blockDim.x a multiple of 64).  `lds` must
// hold blockDim.x/64 + 1 entries.  Returns the exclusive prefix; *total gets the block total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T* total)
{
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    const T incl = wave_incl_scan(v);
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

// Block-wide sum (result valid in every thread).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* lds)
{
    T total;
    block_excl_scan(v, lds, &total);
    return total;
}

// Sum of the partials part[0..limit) and of all n of them (one value per thread, block-wide).
// A thread issues up to sixteen loads before it adds, and both sums leave the block in one
// exchange through LDS.
__device__ __forceinline__ void partials_before(const GArr<uint64_t>& part, uint32_t n,
                                                uint32_t limit, uint64_t* before, uint64_t* all)
{
    constexpr int kLoads = 16;
    __shared__ uint64_t red[2][kMaxBlockWaves];
    uint64_t bsum = 0, asum = 0;
    for (uint32_t t0 = threadIdx.x; t0 < n; t0 += kLoads * blockDim.x) {
        uint64_t v[kLoads];
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            const uint32_t t = t0 + u * blockDim.x;
            v[u] = t < n ? part[t] : 0;
        }
#pragma unroll
        for (int u = 0; u < kLoads; ++u) {
            asum += v[u];
            if (t0 + u * blockDim.x < limit) bsum += v[u];
        }
    }
    bsum = wave_sum(bsum);
    asum = wave_sum(asum);
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) {
        red[0][wave] = bsum;
        red[1][wave] = asum;
    }
    __syncthreads();
    uint64_t b = 0, a = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
        b += red[0][w];
        a += red[1][w];
    }
    *before = b;
    *all = a;
    __syncthreads();  // the exchange row may be written again
}

}  // namespace dogm
