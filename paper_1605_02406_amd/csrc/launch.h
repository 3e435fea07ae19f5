// Host-side launchers of the gfx950 kernels.  Each takes the grids of one launch (one grid or a
// batch) and enqueues its kernels on `s`; the return value is the first HIP error, if any.
#pragma once

#include "dogm_internal.h"

namespace dogm {

// Optional per-kernel timing.  While a trace is active on the calling thread, every launch of
// the traced kernel (all kernels if no name is given) is bracketed by two caller-created HIP
// events recorded on the launch's stream.
struct Trace {
    hipEvent_t* ev;      // 2 * cap events: before / after launch i
    const char** names;  // cap entries, or null
    const char* only;    // kernel name to trace, or null for every kernel
    int cap, n;
    hipError_t err;      // first failed event record
};
extern thread_local Trace* g_trace;

bool trace_wants(const char* name);
inline void trace_before(const char* name, hipStream_t s)
{
    if (!trace_wants(name)) return;
    const hipError_t e = hipEventRecord(g_trace->ev[2 * g_trace->n], s);
    if (g_trace->err == hipSuccess) g_trace->err = e;
}
inline void trace_after(const char* name, hipStream_t s)
{
    if (!trace_wants(name)) return;
    const hipError_t e = hipEventRecord(g_trace->ev[2 * g_trace->n + 1], s);
    if (g_trace->err == hipSuccess) g_trace->err = e;
    if (g_trace->names) g_trace->names[g_trace->n] = name;
    g_trace->n++;
}

// Every kernel launch of the library goes through these macros; a kernel instantiated for the
// precision mode is traced under its plain name.
#define DOGM_LAUNCH_AS(name, kernel, grid, block, lds, stream, ...)          \
    do {                                                                     \
        trace_before(name, stream);                                          \
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);  \
        trace_after(name, stream);                                           \
    } while (0)
#define DOGM_LAUNCH(kernel, grid, block, lds, stream, ...) \
    DOGM_LAUNCH_AS(#kernel, kernel, grid, block, lds, stream, __VA_ARGS__)
// The same kernel for the precision of the launch's grids (FP32 or FP64 real arrays).
#define DOGM_LAUNCH_REAL(real64, name, kernel, grid, block, lds, stream, ...)                    \
    do {                                                                                        \
        if (real64)                                                                             \
            DOGM_LAUNCH_AS(name, (kernel<double>), grid, block, lds, stream,      \
                           __VA_ARGS__);                                                        \
        else                                                                                    \
            DOGM_LAUNCH_AS(name, (kernel<float>), grid, block, lds, stream,       \
                           __VA_ARGS__);                                                        \
    } while (0)

struct GridRef {
    const GridDev* hd;  // host copy of the descriptor (sizes)
    const GridDev* dd;  // the descriptor in device memory
    MeasDev m;          // measurement of this cycle (update only)
};

// Precision of a launch: every grid of one launch has the same (the batched cycle groups them).
inline bool launch_real64(const GridRef* g, int n) { return n > 0 && g[0].hd->real64 != 0; }

// Fills b for grids g[0..n) with blocks_of(hd) blocks each; returns the total block count.
template <typename F>
inline uint32_t make_batch(Batch& b, const GridRef* g, int n, F blocks_of)
{
    b.n = n;
    uint32_t total = 0;
    for (int i = 0; i < n; ++i) {
        b.bstart[i] = total;
        b.g[i] = g[i].dd;
        b.m[i] = g[i].m;
        total += blocks_of(*g[i].hd);
    }
    b.bstart[n] = total;
    return total;
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Block count of an XCD-mapped launch over `tiles` tiles (see xcd_tile).
inline uint32_t xcd_blocks(uint32_t tiles) { return tiles == 0 ? 0 : ceil_div(tiles, kXcds) * kXcds; }

// Key bits of the largest key (C) of a grid.
inline int key_bits(uint32_t C)
{
    int bits = 1;
    while ((C >> bits) != 0) ++bits;
    return bits;
}

hipError_t launch_write_desc(const GridDev& hd, GridDev* dd, hipStream_t s);
hipError_t launch_init(const GridRef* g, int n, hipStream_t s);
hipError_t launch_set_cycle(const GridRef* g, int n, uint32_t cycle, hipStream_t s);
hipError_t launch_predict(const GridRef* g, int n, hipStream_t s);        // Alg. 1
hipError_t launch_sort(const GridRef* g, int n, hipStream_t s);           // Alg. 2 (sort)
hipError_t launch_cell_sums(const GridRef* g, int n, hipStream_t s);      // Alg. 2 ranges + sums
hipError_t launch_update(const GridRef* g, int n, hipStream_t s);         // Alg. 3, 4, 5
hipError_t launch_born_offsets(const GridRef* g, int n, hipStream_t s);   // Alg. 5 (slots)
// Turns a launch's partial sums into exclusive prefixes when one of its grids asks for it (its
// plan says always, or automatic and it has more than kScanPartsFrom of them; which = 0:
// new-born masses, 1: joint weights); returns whether it did in *prefixed.  Otherwise the
// consumers add up the partials before their own themselves.
constexpr uint32_t kScanPartsFrom = 4096;
hipError_t launch_scan_parts(const GridRef* g, int n, int which, bool* prefixed, hipStream_t s);
hipError_t launch_particle_tiles(const GridRef* g, int n, hipStream_t s); // Alg. 4 + 5
hipError_t launch_moments(const GridRef* g, int n, hipStream_t s);        // Alg. 6
hipError_t launch_resample(const GridRef* g, int n, hipStream_t s);       // Alg. 7
// the synthetic sensor ahead of the recursion
hipError_t launch_sensor_truth(const double* rects, int n_rects, const uint8_t* static_occ,
                               int nx, int ny, double cell, uint8_t* occ, uint8_t* seen,
                               hipStream_t s);
hipError_t launch_sensor_scan(const uint8_t* occ, int nx, int ny, bool clear, double p_d,
                              double p_cl, float m_o, float m_f, uint64_t seed, uint32_t cycle,
                              uint8_t* seen, float* m_occ, float* m_free, hipStream_t s);

}  // namespace dogm
