// Test infrastructure: poisons every byte of a grid's arena that belongs to no array, from the
// descriptor at the arena's start, so AddressSanitizer reports any access past an array's end
// (the emulation build leaves a gap after every array).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "dogm_internal.h"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#define EMU_POISON(p, n) ASAN_POISON_MEMORY_REGION(p, n)
#define EMU_UNPOISON(p, n) ASAN_UNPOISON_MEMORY_REGION(p, n)
#endif
#endif
#ifndef EMU_POISON
#define EMU_POISON(p, n) ((void)(p), (void)(n))
#define EMU_UNPOISON(p, n) ((void)(p), (void)(n))
#endif

// Returns the number of arrays found, or -1 if two of them overlap or one leaves the arena.
extern "C" int emu_guard_arena(void* arena, size_t bytes)
{
    using namespace dogm;
    char* base = static_cast<char*>(arena);
    EMU_UNPOISON(base, bytes);
    const GridDev& d = *reinterpret_cast<const GridDev*>(arena);
    const size_t rb = d.real64 ? 8 : 4, nu = d.nu, nb = d.nb, C = d.C;
    struct Range {
        const char* p;
        size_t n;
    };
    std::vector<Range> r;
    auto add = [&](const void* p, size_t n) { r.push_back({static_cast<const char*>(p), n}); };
    add(base, sizeof(GridDev));
    for (const float* p : {d.x, d.y, d.vx, d.vy, d.w, d.sx, d.sy, d.svx, d.svy, d.sw, d.tx, d.ty,
                           d.tvx, d.tvy, d.tw})
        add(p, rb * nu);
    for (const uint32_t* p : {d.key, d.skey, d.perm, d.tkey, d.tval}) add(p, 4 * nu);
    add(d.cstart, 4 * C);
    add(d.cend, 4 * C);
    for (const double* p : {d.sum_w, d.sum_wt, d.mu_A, d.mu_UA}) add(p, 8 * C);
    add(d.msum, kCellSums * 8 * C);
    for (const float* p : {d.m_pO, d.m_pF, d.m_O, d.m_F, d.rho_b, d.rho_p, d.pign, d.mean_x,
                           d.mean_y, d.var_x, d.var_y, d.cov_xy})
        add(p, rb * C);
    add(d.born_off, 4 * (C + 1));
    add(d.mflag, C);
    for (const float* p : {d.bx, d.by, d.bvx, d.bvy, d.bw}) add(p, rb * nb);
    add(d.bkey, 4 * nb);
    add(d.bassoc, nb);
    add(d.hist, 4ull * kSortBins * d.n_hist_tiles);
    add(d.rowtot, 4ull * kSortBins);
    add(d.bpart, 8ull * (d.n_cell_parts + 1));
    add(d.born_mark, 4 * nb);
    add(d.rpart, 8ull * (d.n_res_ptiles + d.n_born_parts + 1));
    add(d.tile_first, 4ull * d.n_born_parts);
    for (const uint32_t* p : {d.cycle, d.cycle_run, d.status, d.nc_flag}) add(p, 4);
    add(d.W_fixed, 8);
    add(d.S_fixed, 8);
    std::sort(r.begin(), r.end(), [](const Range& a, const Range& b) { return a.p < b.p; });
    const char* end = base + bytes;
    const char* at = base;
    for (const Range& x : r) {
        if (x.p < at || x.p + x.n > end) return -1;
        if (x.p > at) EMU_POISON(at, (size_t)(x.p - at));
        at = x.p + x.n;
    }
    if (at < end) EMU_POISON(at, (size_t)(end - at));
    return (int)r.size();
}
