// Host-side launchers of the gfx950 kernels.  Each takes the grids of one launch (one grid or a
// batch) and enqueues its kernels on `s`; the return value is the first HIP error, if any.
#pragma once

#include "dogm_internal.h"

namespace dogm {

struct GridRef {
    const GridDev* hd;  // host copy of the descriptor (sizes)
    const GridDev* dd;  // the descriptor in device memory
    MeasDev m;          // measurement of this cycle (update only)
};

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
hipError_t launch_predict(const GridRef* g, int n, hipStream_t s);
hipError_t launch_sort(const GridRef* g, int n, hipStream_t s);
hipError_t launch_gather(const GridRef* g, int n, hipStream_t s);
hipError_t launch_cell_update(const GridRef* g, int n, hipStream_t s);
hipError_t launch_weight_update(const GridRef* g, int n, hipStream_t s);
hipError_t launch_births(const GridRef* g, int n, hipStream_t s);
hipError_t launch_moments(const GridRef* g, int n, hipStream_t s);
hipError_t launch_resample(const GridRef* g, int n, hipStream_t s);

// Generic per-grid exclusive scans (in place) used by the sort and the births.
enum class ScanArray { SortHist, BornMass };
hipError_t launch_scan(const GridRef* g, int n, ScanArray which, uint32_t digit_bits,
                       hipStream_t s);

}  // namespace dogm
