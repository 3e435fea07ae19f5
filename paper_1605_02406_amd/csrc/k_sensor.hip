// The synthetic sensor ahead of the recursion: the filter of Sec. VII takes a measurement grid
// per cycle as its input; these kernels generate one on the device, so a closed loop of scene,
// sensor and filter needs no host work per cycle.
//
//  - truth: a cell is occupied when its centre lies in one of the given axis-aligned rectangles
//    (boxes and walls, bounds included) or in the static occupancy mask (clutter): the mask is
//    copied, then one block per rectangle marks its cells;
//  - rays: one Amanatides-Woo traversal per perimeter cell, from the sensor at the grid centre
//    towards that cell's centre, marking every cell it passes up to and including the first
//    occupied one (or the perimeter cell); the i-th boundary crossing along an axis is at
//    t_i = t_0 + i d (FP64, one rounded product and one rounded sum), so any step of the walk
//    can be formed on its own and a wave walks one ray 64 cells at a time;
//  - detect: in every observed cell one Bernoulli draw from Philox4x32-10 (counter: cell, cycle,
//    purpose 4, 0): probability p_D where occupied, the clutter probability p_cl where free; the
//    evidence masses are (m_O, 0) for a detection and (0, m_F) for an observed cell without one.
#include "launch.h"

namespace dogm {

constexpr uint32_t kPurposeSensor = 4;
constexpr int kSensorThreads = 256;
constexpr int kRaysPerBlock = kSensorThreads / kWave;  // one ray per wave

// Truth, first launch: every cell takes its static occupancy (none without a mask).
__global__ __launch_bounds__(kSensorThreads) void k_sensor_truth_static(const uint8_t* static_occ,
                                                                        uint32_t C, uint8_t* occ,
                                                                        uint8_t* seen)
{
    const uint32_t c = blockIdx.x * kSensorThreads + threadIdx.x;
    if (c >= C) return;
    occ[c] = (static_occ && static_occ[c] != 0) ? 1 : 0;
    if (seen) seen[c] = 0;
}

// First candidate index of a cell-centre range: centres (i + 1/2) cell for i >= v / cell - 1/2,
// one cell of margin for the rounding of that estimate, clamped to [0, n].
__device__ __forceinline__ int centre_index(double v, double cell, int n, int margin)
{
    const double e = floor(v / cell - 0.5) + (double)margin;
    return e < 0.0 ? 0 : (e > (double)n ? n : (int)e);
}

// Truth, second launch: one block per rectangle marks the cells whose centre lies in it (bounds
// included), testing every candidate cell with the same FP64 expressions as a test per cell.
__global__ __launch_bounds__(kSensorThreads) void k_sensor_truth_rects(const double* rects, int nx,
                                                                       int ny, double cell,
                                                                       uint8_t* occ)
{
    const double x0 = rects[4 * blockIdx.x], y0 = rects[4 * blockIdx.x + 1];
    const double x1 = rects[4 * blockIdx.x + 2], y1 = rects[4 * blockIdx.x + 3];
    if (!(x0 <= x1 && y0 <= y1)) return;  // empty, or a coordinate is not a number
    const int ixa = centre_index(x0, cell, nx, -1), ixb = centre_index(x1, cell, nx, 2);
    const int iya = centre_index(y0, cell, ny, -1), iyb = centre_index(y1, cell, ny, 2);
    if (ixa >= ixb || iya >= iyb) return;
    const uint32_t w = (uint32_t)(ixb - ixa), n = w * (uint32_t)(iyb - iya);
    for (uint32_t t = threadIdx.x; t < n; t += kSensorThreads) {
        const int ix = ixa + (int)(t % w), iy = iya + (int)(t / w);
        const double xc = ((double)ix + 0.5) * cell, yc = ((double)iy + 0.5) * cell;
        if (xc >= x0 && xc <= x1 && yc >= y0 && yc <= y1)
            occ[(uint32_t)iy * (uint32_t)nx + (uint32_t)ix] = 1;
    }
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

// Ray parameter of the i-th cell boundary crossed along one axis: t_0 is the first crossing,
// t_i = t_0 + i d after it (d = 1 / |direction|; infinite for an axis the ray does not move
// along, where every crossing is infinite).
__device__ __forceinline__ double crossing(double t0, double d, uint32_t i)
{
    return i == 0 ? t0 : mul_add_twice_rounded((double)i, d, t0);
}

// Steps along x among the first n steps of a ray.  Each step crosses the nearer boundary, an x
// boundary only when its crossing is strictly smaller, so the steps merge the two increasing
// sequences of crossings (ties to y), and after n steps the number of x steps is the largest i
// in [0, n] with i = 0 or X(i - 1) < Y(n - i): the predicate holds up to it and fails after it.
__device__ __forceinline__ uint32_t x_steps(uint32_t n, double tmx, double tdx, double tmy,
                                            double tdy)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (crossing(tmx, tdx, mid - 1) < crossing(tmy, tdy, n - mid)) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One ray per wave: each lane forms one cell of the walk (step base + lane), and one ballot
// finds the first lane whose cell ends the ray (occupied, the target cell, outside the grid, or
// past the step limit of 2 (nx + ny)); the lanes up to it mark their cells.
__global__ __launch_bounds__(kSensorThreads) void k_sensor_rays(const uint8_t* occ, int nx,
                                                                int ny, uint32_t n_rays,
                                                                uint8_t* seen)
{
    const uint32_t k = blockIdx.x * kRaysPerBlock + threadIdx.x / kWave;
    if (k >= n_rays) return;  // the whole wave
    const uint32_t lane = (uint32_t)lane_id();
    int px, py;
    ray_target(k, nx, ny, px, py);
    const double sx = (double)nx / 2.0, sy = (double)ny / 2.0;
    const double dx = ((double)px + 0.5) - sx, dy = ((double)py + 0.5) - sy;
    const int ix0 = (int)floor(sx), iy0 = (int)floor(sy);
    const int stepx = dx > 0.0 ? 1 : -1, stepy = dy > 0.0 ? 1 : -1;
    const double inf = __builtin_huge_val();
    const double tdx = dx != 0.0 ? fabs(1.0 / dx) : inf;
    const double tdy = dy != 0.0 ? fabs(1.0 / dy) : inf;
    // ray parameter of the first x and y cell boundaries
    const double tmx = dx > 0.0 ? ((double)(ix0 + 1) - sx) / dx
                                : (dx < 0.0 ? ((double)ix0 - sx) / dx : inf);
    const double tmy = dy > 0.0 ? ((double)(iy0 + 1) - sy) / dy
                                : (dy < 0.0 ? ((double)iy0 - sy) / dy : inf);
    const uint32_t limit = 2u * (uint32_t)(nx + ny);
    for (uint32_t base = 0; base < limit; base += kWave) {
        const uint32_t n = base + lane;
        const uint32_t i = x_steps(n, tmx, tdx, tmy, tdy);
        const int ix = ix0 + stepx * (int)i, iy = iy0 + stepy * (int)(n - i);
        const bool in = n < limit && ix >= 0 && ix < nx && iy >= 0 && iy < ny;
        const uint32_t c = in ? (uint32_t)iy * (uint32_t)nx + (uint32_t)ix : 0u;
        const bool ends = !in || occ[c] != 0 || (ix == px && iy == py);
        const uint64_t enders = __ballot(ends);
        const uint32_t first = enders ? (uint32_t)(__ffsll((unsigned long long)enders) - 1)
                                      : (uint32_t)kWave;
        if (in && lane <= first) seen[c] = 1;
        if (enders) return;
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

hipError_t launch_sensor_truth(const double* rects, int n_rects, const uint8_t* static_occ,
                               int nx, int ny, double cell, uint8_t* occ, uint8_t* seen,
                               hipStream_t s)
{
    const uint32_t C = (uint32_t)nx * (uint32_t)ny;
    DOGM_LAUNCH(k_sensor_truth_static, dim3(ceil_div(C, kSensorThreads)), dim3(kSensorThreads),
                0, s, static_occ, C, occ, seen);
    if (n_rects > 0)
        DOGM_LAUNCH(k_sensor_truth_rects, dim3((uint32_t)n_rects), dim3(kSensorThreads), 0, s,
                    rects, nx, ny, cell, occ);
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
    const uint32_t rblocks = ceil_div(n_rays, kRaysPerBlock);
    DOGM_LAUNCH(k_sensor_rays, dim3(rblocks), dim3(kSensorThreads), 0, s, occ, nx, ny, n_rays,
                seen);
    if (m_occ && m_free)
        DOGM_LAUNCH(k_sensor_detect, dim3(cblocks), dim3(kSensorThreads), 0, s, occ, seen, C, p_d,
                    p_cl, m_o, m_f, (uint32_t)seed, (uint32_t)(seed >> 32), cycle, m_occ, m_free);
    return hipGetLastError();
}

}  // namespace dogm
