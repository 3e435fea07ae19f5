// The synthetic sensor ahead of the recursion: the filter of Sec. VII takes a measurement grid
// per cycle as its input; these kernels generate one on the device, so a closed loop of scene,
// sensor and filter needs no host work per cycle.
//
//  - truth: a cell is occupied when its centre lies in one of the given axis-aligned rectangles
//    (boxes and walls, bounds included) or in the static occupancy mask (clutter);
//  - rays: one Amanatides-Woo traversal per perimeter cell, from the sensor at the grid centre
//    towards that cell's centre, marking every cell it passes up to and including the first
//    occupied one (or the perimeter cell); all arithmetic in FP64, in the order of the
//    traversal's definition, so the cells marked do not depend on the device;
//  - detect: in every observed cell one Bernoulli draw from Philox4x32-10 (counter: cell, cycle,
//    purpose 4, 0): probability p_D where occupied, the clutter probability p_cl where free; the
//    evidence masses are (m_O, 0) for a detection and (0, m_F) for an observed cell without one.
#include <mutex>
#include <vector>

#include "launch.h"

namespace dogm {

constexpr uint32_t kPurposeSensor = 4;
constexpr int kSensorThreads = 256;
// the occupancy is held as a bit mask in LDS while the mask (rows padded to an odd number of
// 32-bit words) takes at most this many bytes, else read from memory
constexpr uint32_t kRayLdsMax = 160u * 1024u;

__global__ __launch_bounds__(kSensorThreads) void k_sensor_truth(const double* rects, int n_rects,
                                                                 const uint8_t* static_occ,
                                                                 int nx, int ny, double cell,
                                                                 uint8_t* occ, uint8_t* seen)
{
    const uint32_t C = (uint32_t)nx * (uint32_t)ny;
    const uint32_t c = blockIdx.x * kSensorThreads + threadIdx.x;
    if (c >= C) return;
    const uint32_t ix = c % (uint32_t)nx, iy = c / (uint32_t)nx;
    const double xc = ((double)ix + 0.5) * cell, yc = ((double)iy + 0.5) * cell;
    bool o = static_occ ? static_occ[c] != 0 : false;
    for (int r = 0; r < n_rects && !o; ++r) {
        const double x0 = rects[4 * r], y0 = rects[4 * r + 1];
        const double x1 = rects[4 * r + 2], y1 = rects[4 * r + 3];
        o = xc >= x0 && xc <= x1 && yc >= y0 && yc <= y1;
    }
    occ[c] = o ? 1 : 0;
    if (seen) seen[c] = 0;
}

__global__ __launch_bounds__(kSensorThreads) void k_sensor_clear(uint8_t* seen, uint32_t C)
{
    const uint32_t c = blockIdx.x * kSensorThreads + threadIdx.x;
    if (c < C) seen[c] = 0;
}

// Perimeter cell of ray k: the bottom row, the top row, then the left and right columns
// without their corners.
__device__ __forceinline__ void ray_target(uint32_t k, int nx, int ny, int& px, int& py)
{
    const uint32_t unx = (uint32_t)nx;
    if (k < unx) { px = (int)k; py = 0; return; }
    k -= unx;
    if (k < unx) { px = (int)k; py = ny - 1; return; }
    k -= unx;
    const uint32_t side = (uint32_t)(ny - 2);
    if (k < side) { px = 0; py = (int)k + 1; return; }
    px = nx - 1;
    py = (int)(k - side) + 1;
}

template <bool kLds>
__global__ __launch_bounds__(kSensorThreads) void k_sensor_rays(const uint8_t* occ, int nx,
                                                                int ny, uint32_t n_rays,
                                                                uint8_t* seen)
{
    extern __shared__ uint32_t bits[];
    const uint32_t C = (uint32_t)nx * (uint32_t)ny;
    // LDS mask: row iy of the grid is words [iy * stride, iy * stride + ceil(nx / 32)), bit b of
    // word w holding cell (32 w + b, iy); the row stride in words is odd, so the rays of a wave,
    // which fan out across rows, read words in different LDS banks
    const uint32_t row_words = ((uint32_t)nx + 31u) / 32u;
    const uint32_t stride = row_words | 1u;
    if (kLds) {
        // every block packs the whole occupancy grid, each word from 32 bytes of one row (two
        // 16-byte vectors where the row is whole and aligned); each thread issues the loads of
        // kPackBatch words before packing them, so their latencies overlap
        constexpr int kPackBatch = 8;
        const bool vec = (reinterpret_cast<uintptr_t>(occ) & 15u) == 0 && nx % 16 == 0;
        const uint32_t nwords = row_words * (uint32_t)ny;
        for (uint32_t w0 = threadIdx.x; w0 < nwords; w0 += kPackBatch * kSensorThreads) {
            uint4 va[kPackBatch], vb[kPackBatch];
#pragma unroll
            for (int q = 0; q < kPackBatch; ++q) {
                const uint32_t wd = w0 + q * kSensorThreads;
                const uint32_t row = wd / row_words, x0 = (wd - row * row_words) * 32u;
                const uint32_t c0 = row * (uint32_t)nx + x0;
                if (vec && wd < nwords && x0 + 32 <= (uint32_t)nx) {
                    va[q] = reinterpret_cast<const uint4*>(occ + c0)[0];
                    vb[q] = reinterpret_cast<const uint4*>(occ + c0)[1];
                } else {
                    va[q] = vb[q] = make_uint4(0u, 0u, 0u, 0u);
                }
            }
#pragma unroll
            for (int q = 0; q < kPackBatch; ++q) {
                const uint32_t wd = w0 + q * kSensorThreads;
                if (wd >= nwords) break;
                const uint32_t row = wd / row_words, x0 = (wd - row * row_words) * 32u;
                const uint32_t c0 = row * (uint32_t)nx + x0;
                uint32_t m = 0;
                if (vec && x0 + 32 <= (uint32_t)nx) {
                    const uint32_t w8[8] = {va[q].x, va[q].y, va[q].z, va[q].w,
                                            vb[q].x, vb[q].y, vb[q].z, vb[q].w};
#pragma unroll
                    for (int k = 0; k < 8; ++k)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if ((w8[k] >> (8 * e)) & 0xFFu) m |= 1u << (4 * k + e);
                } else {
                    for (uint32_t b = 0; b < 32 && x0 + b < (uint32_t)nx; ++b)
                        if (occ[c0 + b]) m |= 1u << b;
                }
                bits[row * stride + (wd - row * row_words)] = m;
            }
        }
        __syncthreads();
    }
    const uint32_t k = blockIdx.x * kSensorThreads + threadIdx.x;
    if (k >= n_rays) return;
    int px, py;
    ray_target(k, nx, ny, px, py);
    const double sx = (double)nx / 2.0, sy = (double)ny / 2.0;
    const double dx = ((double)px + 0.5) - sx, dy = ((double)py + 0.5) - sy;
    int ix = (int)floor(sx), iy = (int)floor(sy);
    const int stepx = dx > 0.0 ? 1 : -1, stepy = dy > 0.0 ? 1 : -1;
    const double inf = __builtin_huge_val();
    const double tdx = dx != 0.0 ? fabs(1.0 / dx) : inf;
    const double tdy = dy != 0.0 ? fabs(1.0 / dy) : inf;
    // ray parameter of the first x and y cell boundaries, and their spacing
    double tmx = dx > 0.0 ? ((double)(ix + 1) - sx) / dx
                          : (dx < 0.0 ? ((double)ix - sx) / dx : inf);
    double tmy = dy > 0.0 ? ((double)(iy + 1) - sy) / dy
                          : (dy < 0.0 ? ((double)iy - sy) / dy : inf);
    // one step per iteration with selects instead of branches: a wave runs one ray per lane, so
    // the loop is bound by its instruction count, not by memory
    for (int step = 0; step < 2 * (nx + ny); ++step) {
        const uint32_t c = (uint32_t)iy * (uint32_t)nx + (uint32_t)ix;
        seen[c] = 1;
        const bool hit = kLds ? ((bits[(uint32_t)iy * stride + ((uint32_t)ix >> 5)] >> (ix & 31)) & 1u) != 0
                              : occ[c] != 0;
        const bool xs = tmx < tmy;
        const double tmx_n = tmx + tdx, tmy_n = tmy + tdy;
        const int ixn = xs ? ix + stepx : ix, iyn = xs ? iy : iy + stepy;
        tmx = xs ? tmx_n : tmx;
        tmy = xs ? tmy : tmy_n;
        // bitwise, not short-circuit: every term is one compare, none needs a branch
        const bool stop = hit | ((ix == px) & (iy == py)) | (ixn < 0) | (ixn >= nx) | (iyn < 0) |
                          (iyn >= ny);
        if (stop) break;
        ix = ixn;
        iy = iyn;
    }
}

__global__ __launch_bounds__(kSensorThreads) void k_sensor_detect(
    const uint8_t* occ, const uint8_t* seen, uint32_t C, double p_d, double p_cl, float m_o,
    float m_f, uint32_t seed_lo, uint32_t seed_hi, uint32_t cycle, float* m_occ, float* m_free)
{
    const uint32_t c = blockIdx.x * kSensorThreads + threadIdx.x;
    if (c >= C) return;
    float mo = 0.0f, mf = 0.0f;
    if (seen[c]) {
        const uint4 r = philox4x32_10(make_uint4(c, cycle, kPurposeSensor, 0u), seed_lo, seed_hi);
        const double u = (double)unit_f32(r.x);
        const bool det = u < (occ[c] ? p_d : p_cl);
        mo = det ? m_o : 0.0f;
        mf = det ? 0.0f : m_f;
    }
    m_occ[c] = mo;
    m_free[c] = mf;
}

// The rays' bit mask (up to 128 KiB) is above the default dynamic LDS limit: raise it once on
// every device the library launches on (the attribute is per device).
hipError_t allow_ray_lds()
{
    static std::mutex mu;
    static std::vector<bool> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((size_t)dev < done.size() && done[dev]) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sensor_rays<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kRayLdsMax);
    if (e != hipSuccess) return e;
    if ((size_t)dev >= done.size()) done.resize(dev + 1, false);
    done[dev] = true;
    return hipSuccess;
}

hipError_t launch_sensor_truth(const double* rects, int n_rects, const uint8_t* static_occ,
                               int nx, int ny, double cell, uint8_t* occ, uint8_t* seen,
                               hipStream_t s)
{
    const uint32_t C = (uint32_t)nx * (uint32_t)ny;
    DOGM_LAUNCH(k_sensor_truth, dim3(ceil_div(C, kSensorThreads)), dim3(kSensorThreads), 0, s,
                rects, n_rects, static_occ, nx, ny, cell, occ, seen);
    return hipGetLastError();
}

hipError_t launch_sensor_scan(const uint8_t* occ, int nx, int ny, bool clear, double p_d,
                              double p_cl, float m_o, float m_f, uint64_t seed, uint32_t cycle,
                              uint8_t* seen, float* m_occ, float* m_free, hipStream_t s)
{
    const uint32_t C = (uint32_t)nx * (uint32_t)ny;
    const uint32_t cblocks = ceil_div(C, kSensorThreads);
    if (clear) DOGM_LAUNCH(k_sensor_clear, dim3(cblocks), dim3(kSensorThreads), 0, s, seen, C);
    const uint32_t n_rays = 2u * (uint32_t)nx + (ny >= 2 ? 2u * (uint32_t)(ny - 2) : 0u);
    const uint32_t rblocks = ceil_div(n_rays, kSensorThreads);
    const size_t lds = 4ull * ((((uint32_t)nx + 31u) / 32u) | 1u) * (uint32_t)ny;
    if (lds <= kRayLdsMax) {
        if (const hipError_t e = allow_ray_lds(); e != hipSuccess) return e;
        DOGM_LAUNCH(k_sensor_rays<true>, dim3(rblocks), dim3(kSensorThreads), lds, s, occ, nx, ny,
                    n_rays, seen);
    } else {
        DOGM_LAUNCH(k_sensor_rays<false>, dim3(rblocks), dim3(kSensorThreads), 0, s, occ, nx, ny,
                    n_rays, seen);
    }
    if (m_occ && m_free)
        DOGM_LAUNCH(k_sensor_detect, dim3(cblocks), dim3(kSensorThreads), 0, s, occ, seen, C, p_d,
                    p_cl, m_o, m_f, (uint32_t)seed, (uint32_t)(seed >> 32), cycle, m_occ, m_free);
    return hipGetLastError();
}

}  // namespace dogm
