// Host side of the C ABI declared in include/dogm.h: validation, arena layout, call order and
// the batched cycle.  All device work is in the k_*.hip kernels; nothing here computes filter
// values and nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dogm.h"
#include "launch.h"

using namespace dogm;

namespace dogm {
thread_local Trace* g_trace = nullptr;

bool trace_wants(const char* name)
{
    if (!g_trace || g_trace->n >= g_trace->cap) return false;
    return !g_trace->only || std::strcmp(g_trace->only, name) == 0;
}
}  // namespace dogm

namespace {

enum Phase { kReady = 0, kPredicted = 1, kAssigned = 2, kUpdated = 3, kMoments = 4 };

thread_local std::string g_last_error;
thread_local Trace g_trace_storage;

int hip_fail(hipError_t e, const char* where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return DOGM_EHIP;
}

bool finite_in(float v, float lo, float hi) { return std::isfinite(v) && v >= lo && v <= hi; }

bool valid_params(const dogm_params* p)
{
    if (!p) return false;
    if (p->nx < 1 || p->ny < 1) return false;
    // fixed-point sums of masses (2^-40 units, at most 1 per cell plus half a unit per
    // particle) stay below 2^64 for fewer than 2^24 cells
    if ((int64_t)p->nx * (int64_t)p->ny >= (int64_t(1) << 24)) return false;
    if (!(std::isfinite(p->cell_size) && p->cell_size > 0.0f)) return false;
    if (!finite_in(p->dt, 0.0f, 1e6f)) return false;
    if (!finite_in(p->p_s, 0.0f, 1.0f) || !finite_in(p->p_b, 0.0f, 1.0f)) return false;
    if (!finite_in(p->sigma_pos, 0.0f, 1e6f) || !finite_in(p->sigma_vel, 0.0f, 1e6f) ||
        !finite_in(p->sigma_birth_vel, 0.0f, 1e6f))
        return false;
    if (!finite_in(p->alpha_free, 0.0f, 1.0f)) return false;
    // below 2^27 the last systematic draw stays below the joint weight W after the three
    // FP64 roundings of W, W / nu and (j + U) W / nu, also where W exceeds 2^53
    if (p->n_pers < 1 || p->n_pers >= (int64_t(1) << 27)) return false;
    if (p->n_born < 0 || p->n_born >= (int64_t(1) << 30)) return false;
    if (p->model != DOGM_MODEL_DS && p->model != DOGM_MODEL_PHD_MIB) return false;
    if (p->precision != DOGM_PRECISION_FP32 && p->precision != DOGM_PRECISION_FP64) return false;
    // the plan: enough passes for the key bits with at most kSortBits per digit, at most 3
    const int kb = key_bits((uint32_t)p->nx * (uint32_t)p->ny);
    const uint32_t fewest = (uint32_t)((kb + kSortBits - 1) / kSortBits);
    if (p->sort_passes != 0 && (p->sort_passes < fewest || p->sort_passes > kMaxPasses))
        return false;
    if (p->scan_parts > 2 || p->resample > 2) return false;
    return true;
}

// Bytes left free after every array of the arena: none in the library; the CPU emulation of
// the kernels (a test build) leaves a gap that it poisons, so an access past any array's end
// is reported.
#ifndef DOGM_ARENA_GAP
#define DOGM_ARENA_GAP 0
#endif

// Offsets of every array inside the arena (the descriptor sits at offset 0).
struct Layout {
    size_t total = 0;
    size_t take(size_t bytes)
    {
        const size_t o = (total + 255) & ~size_t(255);
        total = o + (bytes ? bytes : 1) + DOGM_ARENA_GAP;
        return o;
    }
};

template <typename T>
T* at(char* base, size_t off)
{
    return reinterpret_cast<T*>(base + off);
}

// The per-cycle scratch of a grid: digit histograms of every sort tile (digit-major) with their
// row totals, fixed-point partial sums of new-born masses and of joint weights (turned into
// exclusive prefixes in place, the total in one extra entry), first-slot marks and the first
// cell of every new-born tile.  Every array is rewritten within each cycle before
// it is read, so none needs clearing.  Places the arrays at `base` (sizes and tilings of d must
// be set; base may be null to only measure) and returns the bytes they take.
size_t place_scratch(GridDev& d, char* base)
{
    Layout L;
    const size_t o_hist = L.take(4ull * kSortBins * d.n_hist_tiles);
    const size_t o_rowtot = L.take(4ull * kSortBins);
    const size_t o_bpart = L.take(8ull * (d.n_cell_parts + 1));
    const size_t o_mark = L.take(4ull * d.nb);
    const size_t o_rpart = L.take(8ull * (d.n_res_ptiles + d.n_born_parts + 1));
    const size_t o_tfirst = L.take(4ull * d.n_born_parts);
    if (base) {
        d.hist = at<uint32_t>(base, o_hist);
        d.rowtot = at<uint32_t>(base, o_rowtot);
        d.bpart = at<uint64_t>(base, o_bpart);
        d.rpart = at<uint64_t>(base, o_rpart);
        d.born_mark = at<uint32_t>(base, o_mark);
        d.tile_first = at<uint32_t>(base, o_tfirst);
    }
    return L.total;
}

// Builds the descriptor for `arena` (base may be null to only measure the size).
GridDev describe(const dogm_params* p, char* base, size_t* bytes)
{
    GridDev d;
    std::memset(&d, 0, sizeof(d));
    const uint32_t nu = (uint32_t)p->n_pers, nb = (uint32_t)p->n_born;
    const uint32_t C = (uint32_t)p->nx * (uint32_t)p->ny;
    d.nx = p->nx;
    d.ny = p->ny;
    d.C = C;
    d.nu = nu;
    d.nb = nb;
    d.r = p->cell_size;
    d.dt = p->dt;
    d.p_s = p->p_s;
    d.p_b = p->p_b;
    d.sig_pos = p->sigma_pos;
    d.sig_vel = p->sigma_vel;
    d.sig_birth = p->sigma_birth_vel;
    d.alpha = p->alpha_free;
    d.seed_lo = (uint32_t)p->seed;
    d.seed_hi = (uint32_t)(p->seed >> 32);
    d.grid_id = p->grid_id;
    d.model = p->model;
    d.real64 = p->precision == DOGM_PRECISION_FP64 ? 1u : 0u;
    // radix digits: as few passes of at most kSortBits bits as cover the largest key (C)
    const int kb = key_bits(C);
    d.passes = (uint32_t)((kb + kSortBits - 1) / kSortBits);
    if (p->sort_passes > d.passes) d.passes = p->sort_passes;
    d.scan_parts = p->scan_parts;
    d.resample = p->resample;
    uint32_t shift = 0;
    for (uint32_t q = 0; q < d.passes; ++q) {
        const uint32_t left = (uint32_t)kb - shift, passes_left = d.passes - q;
        d.dbits[q] = (left + passes_left - 1) / passes_left;
        d.dshift[q] = shift;
        shift += d.dbits[q];
    }
    d.n_sort_tiles = ceil_div(nu, kSortTile);
    d.n_hist_tiles = ceil_div(nu, kHistTile);
    d.n_cell_parts = ceil_div(C, kCellThreads);
    d.n_res_ptiles = ceil_div(nu, kResTile);
    d.n_res_btiles = ceil_div(nb, kResTile);
    d.n_born_parts = ceil_div(nb, kBornTile);

    Layout L;
    L.take(sizeof(GridDev));
    const size_t f_nu = 4ull * nu, f_c = 4ull * C, d_c = 8ull * C;
    // real-valued arrays: FP32, or FP64 in the all-FP64 precision mode
    const size_t rb = d.real64 ? 8 : 4;
    const size_t r_nu = rb * nu, r_nb = rb * nb, r_c = rb * C;
    float** pf_nu[] = {&d.x, &d.y, &d.vx, &d.vy, &d.w, &d.sx, &d.sy, &d.svx, &d.svy, &d.sw,
                       &d.tx, &d.ty, &d.tvx, &d.tvy, &d.tw};
    size_t o_pf_nu[15];
    for (int i = 0; i < 15; ++i) o_pf_nu[i] = L.take(r_nu);
    uint32_t** pu_nu[] = {&d.key, &d.skey, &d.perm, &d.tkey, &d.tval};
    size_t o_pu_nu[5];
    for (int i = 0; i < 5; ++i) o_pu_nu[i] = L.take(f_nu);
    uint32_t** pu_c[] = {&d.cstart, &d.cend};
    size_t o_pu_c[2];
    for (int i = 0; i < 2; ++i) o_pu_c[i] = L.take(f_c);
    double** pd_c[] = {&d.sum_w, &d.sum_wt, &d.mu_A, &d.mu_UA};
    size_t o_pd_c[4];
    for (int i = 0; i < 4; ++i) o_pd_c[i] = L.take(d_c);
    const size_t o_msum = L.take(kCellSums * d_c);
    float** pf_c[] = {&d.m_pO, &d.m_pF, &d.m_O, &d.m_F, &d.rho_b, &d.rho_p, &d.pign,
                      &d.mean_x, &d.mean_y, &d.var_x, &d.var_y, &d.cov_xy};
    size_t o_pf_c[12];
    for (int i = 0; i < 12; ++i) o_pf_c[i] = L.take(r_c);
    const size_t o_boff = L.take(4ull * (C + 1)), o_mfl = L.take(C);
    float** pf_nb[] = {&d.bx, &d.by, &d.bvx, &d.bvy, &d.bw};
    size_t o_pf_nb[5];
    for (int i = 0; i < 5; ++i) o_pf_nb[i] = L.take(r_nb);
    const size_t o_bkey = L.take(4ull * nb), o_bas = L.take(nb);
    const size_t o_scratch = L.take(place_scratch(d, nullptr));
    const size_t o_cyc = L.take(4), o_cycr = L.take(4), o_st = L.take(4), o_nc = L.take(4),
                 o_W = L.take(8), o_S = L.take(8);
    *bytes = L.total;
    if (!base) return d;

    for (int i = 0; i < 15; ++i) *pf_nu[i] = at<float>(base, o_pf_nu[i]);
    for (int i = 0; i < 5; ++i) *pu_nu[i] = at<uint32_t>(base, o_pu_nu[i]);
    for (int i = 0; i < 2; ++i) *pu_c[i] = at<uint32_t>(base, o_pu_c[i]);
    for (int i = 0; i < 4; ++i) *pd_c[i] = at<double>(base, o_pd_c[i]);
    d.msum = at<double>(base, o_msum);
    for (int i = 0; i < 12; ++i) *pf_c[i] = at<float>(base, o_pf_c[i]);
    d.born_off = at<uint32_t>(base, o_boff);
    d.mflag = at<uint8_t>(base, o_mfl);
    for (int i = 0; i < 5; ++i) *pf_nb[i] = at<float>(base, o_pf_nb[i]);
    d.bkey = at<uint32_t>(base, o_bkey);
    d.bassoc = at<uint8_t>(base, o_bas);
    place_scratch(d, base + o_scratch);
    d.cycle = at<uint32_t>(base, o_cyc);
    d.cycle_run = at<uint32_t>(base, o_cycr);
    d.status = at<uint32_t>(base, o_st);
    d.nc_flag = at<uint32_t>(base, o_nc);
    d.W_fixed = at<uint64_t>(base, o_W);
    d.S_fixed = at<uint64_t>(base, o_S);
    return d;
}

// The scratch of dogm_step_noalloc: one array per device, held until the process ends, with a
// private copy of the stepped grid's descriptor at its start and that grid's per-cycle scratch
// after it.  Host code uses only the device address hipGetSymbolAddress returns for it (the
// array's name is a host-side stand-in), looked up once per device with that device current.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
constexpr size_t kStaticDescBytes = (sizeof(GridDev) + 255) & ~size_t(255);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device id; null until looked up

hipError_t static_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev < g_scratch_ptr.size() && g_scratch_ptr[dev]) {
        *out = g_scratch_ptr[dev];
        return hipSuccess;
    }
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return hipSuccess;
}

// Velocity evidence (p_A > 0) is switched off: its kernels stay in the library but no entry
// point launches them until a device fault seen with them is explained.  The CPU emulation of
// the kernels (a test build) compiles it in with DOGM_EVIDENCE=1.
#ifndef DOGM_EVIDENCE
#define DOGM_EVIDENCE 0
#endif
bool evidence_enabled() { return DOGM_EVIDENCE != 0; }

int evidence_refused(const char* where)
{
    g_last_error = std::string(where) + ": velocity evidence (p_assoc) is disabled in this version of the library";
    return DOGM_ENOTIMPL;
}

static_assert(kModelPhdMib == DOGM_MODEL_PHD_MIB, "one model numbering");

bool valid_meas(const dogm_meas* m, uint32_t model)
{
    if (!m) return false;
    if (model == DOGM_MODEL_PHD_MIB) return m->p_tp && m->p_fp && m->det && !m->p_assoc;
    if (!m->m_occ || !m->m_free) return false;
    if (m->p_assoc && (!m->mu_vx || !m->mu_vy || !m->var_v)) return false;
    return true;
}

MeasDev to_dev(const dogm_meas* m)
{
    MeasDev d{};
    if (m) {
        d.m_occ = m->m_occ;
        d.m_free = m->m_free;
        d.p_assoc = m->p_assoc;
        d.mu_vx = m->mu_vx;
        d.mu_vy = m->mu_vy;
        d.var_v = m->var_v;
        d.p_tp = m->p_tp;
        d.p_fp = m->p_fp;
        d.det = m->det;
    }
    return d;
}

}  // namespace

struct dogm_grid {
    dogm_params p;
    GridDev hd;
    GridDev* dd;
    void* arena;
    size_t arena_bytes;
    hipStream_t stream;
    uint32_t cycle;
    int phase;
    bool assoc;           // the last update had velocity evidence
    // its measurement: dogm_moments passes it on only to mark the grid as one with evidence
    // (the moments kernel reads no measurement array)
    dogm_meas last_meas;

    GridRef ref(const dogm_meas* m = nullptr) const { return GridRef{&hd, dd, to_dev(m)}; }
};

extern "C" {

int dogm_arena_bytes(const dogm_params* params, size_t* bytes)
{
    if (!valid_params(params) || !bytes) return DOGM_EINVAL;
    describe(params, nullptr, bytes);
    return DOGM_OK;
}

int dogm_init_grid(const dogm_params* params, void* arena, size_t arena_bytes,
                   dogm_stream_t stream, dogm_grid** out)
{
    if (!valid_params(params) || !arena || !out) return DOGM_EINVAL;
    if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0) return DOGM_EINVAL;
    size_t need = 0;
    describe(params, nullptr, &need);
    if (arena_bytes < need) {
        g_last_error = "dogm_init_grid: arena of " + std::to_string(arena_bytes) + " bytes, " +
                       std::to_string(need) + " needed";
        return DOGM_ESIZE;
    }
    dogm_grid* g = new (std::nothrow) dogm_grid;
    if (!g) return DOGM_EINVAL;
    g->p = *params;
    g->hd = describe(params, static_cast<char*>(arena), &need);
    g->dd = static_cast<GridDev*>(arena);
    g->arena = arena;
    g->arena_bytes = arena_bytes;
    g->stream = static_cast<hipStream_t>(stream);
    g->cycle = 1;
    g->phase = kReady;
    g->assoc = false;
    std::memset(&g->last_meas, 0, sizeof(g->last_meas));
    // set-up of dogm_step_noalloc: the static scratch's address on the current device
    void* scr = nullptr;
    hipError_t e = static_scratch(&scr);
    if (e == hipSuccess) e = launch_write_desc(g->hd, g->dd, g->stream);
    if (e == hipSuccess) {
        const GridRef r = g->ref();
        e = launch_init(&r, 1, g->stream);
    }
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "dogm_init_grid");
    }
    *out = g;
    return DOGM_OK;
}

int dogm_destroy(dogm_grid* grid)
{
    if (!grid) return DOGM_EINVAL;
    delete grid;
    return DOGM_OK;
}

int dogm_set_stream(dogm_grid* grid, dogm_stream_t stream)
{
    if (!grid) return DOGM_EINVAL;
    grid->stream = static_cast<hipStream_t>(stream);
    return DOGM_OK;
}

int dogm_set_cycle(dogm_grid* grid, uint32_t cycle)
{
    if (!grid) return DOGM_EINVAL;
    const GridRef r = grid->ref();
    hipError_t e = launch_set_cycle(&r, 1, cycle, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_set_cycle");
    grid->cycle = cycle;
    grid->phase = kReady;
    return DOGM_OK;
}

int dogm_get_cycle(const dogm_grid* grid, uint32_t* cycle)
{
    if (!grid || !cycle) return DOGM_EINVAL;
    *cycle = grid->cycle;
    return DOGM_OK;
}

int dogm_view(const dogm_grid* grid, dogm_views* v)
{
    if (!grid || !v) return DOGM_EINVAL;
    const GridDev& d = grid->hd;
    v->x = d.x;
    v->y = d.y;
    v->vx = d.vx;
    v->vy = d.vy;
    v->w = d.w;
    v->key = d.key;
    v->sx = d.sx;
    v->sy = d.sy;
    v->svx = d.svx;
    v->svy = d.svy;
    v->sw = d.sw;
    v->skey = d.skey;
    v->perm = d.perm;
    v->cell_start = d.cstart;
    v->cell_end = d.cend;
    v->sum_w = d.sum_w;
    v->m_pO = d.m_pO;
    v->m_pF = d.m_pF;
    v->m_O = d.m_O;
    v->m_F = d.m_F;
    v->rho_b = d.rho_b;
    v->rho_p = d.rho_p;
    v->pign = d.pign;
    v->mu_A = d.mu_A;
    v->mu_UA = d.mu_UA;
    v->born_off = d.born_off;
    v->mean_x = d.mean_x;
    v->mean_y = d.mean_y;
    v->var_x = d.var_x;
    v->var_y = d.var_y;
    v->cov_xy = d.cov_xy;
    v->mom_flag = d.mflag;
    v->bx = d.bx;
    v->by = d.by;
    v->bvx = d.bvx;
    v->bvy = d.bvy;
    v->bw = d.bw;
    v->bkey = d.bkey;
    v->bassoc = d.bassoc;
    v->status = d.status;
    v->cycle = d.cycle;
    v->W_fixed = d.W_fixed;
    v->S_fixed = d.S_fixed;
    v->n_pers = d.nu;
    v->n_born = d.nb;
    v->n_cells = d.C;
    return DOGM_OK;
}

int dogm_predict(dogm_grid* grid)
{
    if (!grid) return DOGM_EINVAL;
    if (grid->phase != kReady) return DOGM_ESTATE;
    const GridRef r = grid->ref();
    hipError_t e = launch_predict(&r, 1, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_predict");
    grid->phase = kPredicted;
    return DOGM_OK;
}

int dogm_assign(dogm_grid* grid)
{
    if (!grid) return DOGM_EINVAL;
    if (grid->phase != kPredicted) return DOGM_ESTATE;
    const GridRef r = grid->ref();
    hipError_t e = launch_sort(&r, 1, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_assign");
    grid->phase = kAssigned;
    return DOGM_OK;
}

int dogm_update(dogm_grid* grid, const dogm_meas* meas)
{
    if (!grid || !valid_meas(meas, grid->p.model)) return DOGM_EINVAL;
    if (meas->p_assoc && !evidence_enabled()) return evidence_refused("dogm_update");
    if (grid->phase != kAssigned) return DOGM_ESTATE;
    const GridRef r = grid->ref(meas);
    hipError_t e = launch_update(&r, 1, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_update");
    grid->phase = kUpdated;
    grid->assoc = meas->p_assoc != nullptr;
    grid->last_meas = *meas;
    return DOGM_OK;
}

int dogm_moments(dogm_grid* grid)
{
    if (!grid) return DOGM_EINVAL;
    if (grid->phase != kUpdated && grid->phase != kMoments) return DOGM_ESTATE;
    const GridRef r = grid->ref(grid->assoc ? &grid->last_meas : nullptr);
    hipError_t e = launch_moments(&r, 1, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_moments");
    grid->phase = kMoments;
    return DOGM_OK;
}

int dogm_resample(dogm_grid* grid)
{
    if (!grid) return DOGM_EINVAL;
    if (grid->phase != kUpdated && grid->phase != kMoments) return DOGM_ESTATE;
    const GridRef r = grid->ref();
    hipError_t e = launch_resample(&r, 1, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_resample");
    grid->phase = kReady;
    grid->cycle += 1;
    return DOGM_OK;
}

int dogm_step(dogm_grid* grid, const dogm_meas* meas)
{
    if (!grid || !valid_meas(meas, grid->p.model)) return DOGM_EINVAL;
    if (meas->p_assoc && !evidence_enabled()) return evidence_refused("dogm_step");
    if (grid->phase != kReady) return DOGM_ESTATE;
    int rc = dogm_predict(grid);
    if (rc == DOGM_OK) rc = dogm_assign(grid);
    if (rc == DOGM_OK) rc = dogm_update(grid, meas);
    if (rc == DOGM_OK) rc = dogm_moments(grid);
    if (rc == DOGM_OK) rc = dogm_resample(grid);
    return rc;
}

int dogm_step_noalloc(dogm_grid* grid, const dogm_meas* meas)
{
    if (!grid || !valid_meas(meas, grid->p.model)) return DOGM_EINVAL;
    if (meas->p_assoc && !evidence_enabled()) return evidence_refused("dogm_step_noalloc");
    if (grid->phase != kReady) return DOGM_ESTATE;
    GridDev hs = grid->hd;
    const size_t need = kStaticDescBytes + place_scratch(hs, nullptr);
    if (need > kStaticScratchBytes) {
        g_last_error = "dogm_step_noalloc: the grid's per-cycle scratch needs " +
                       std::to_string(need) + " bytes, the static array holds " +
                       std::to_string(kStaticScratchBytes);
        return DOGM_ESIZE;
    }
    void* base = nullptr;
    hipError_t e = static_scratch(&base);
    if (e != hipSuccess) return hip_fail(e, "dogm_step_noalloc");
    place_scratch(hs, static_cast<char*>(base) + kStaticDescBytes);
    GridDev* dd = static_cast<GridDev*>(base);
    const GridRef r{&hs, dd, to_dev(meas)};
    const hipStream_t s = grid->stream;
    e = launch_write_desc(hs, dd, s);
    if (e == hipSuccess) e = launch_predict(&r, 1, s);
    if (e == hipSuccess) e = launch_sort(&r, 1, s);
    if (e == hipSuccess) e = launch_update(&r, 1, s);
    if (e == hipSuccess) e = launch_moments(&r, 1, s);
    if (e == hipSuccess) e = launch_resample(&r, 1, s);
    if (e != hipSuccess) return hip_fail(e, "dogm_step_noalloc");
    grid->assoc = false;
    grid->cycle += 1;
    return DOGM_OK;
}

int dogm_step_batch(dogm_grid* const* grids, const dogm_meas* meas, int n, dogm_stream_t stream)
{
    if (n < 0 || (n > 0 && (!grids || !meas))) return DOGM_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!grids[i] || !valid_meas(&meas[i], grids[i]->p.model)) return DOGM_EINVAL;
        if (meas[i].p_assoc && !evidence_enabled()) return evidence_refused("dogm_step_batch");
        if (grids[i]->phase != kReady) return DOGM_ESTATE;
        for (int j = 0; j < i; ++j)
            if (grids[j] == grids[i]) return DOGM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // one launch per kernel for up to kMaxBatch grids; grids with and without velocity
    // evidence, and grids of the two precision modes, go to separate launches
    for (int kind = 0; kind < 4; ++kind) {
        const bool assoc = (kind & 1) != 0, real64 = (kind & 2) != 0;
        std::vector<GridRef> refs;
        for (int i = 0; i < n; ++i)
            if ((meas[i].p_assoc != nullptr) == assoc && (grids[i]->hd.real64 != 0) == real64)
                refs.push_back(grids[i]->ref(&meas[i]));
        for (size_t c0 = 0; c0 < refs.size(); c0 += kMaxBatch) {
            const int m = (int)std::min(refs.size() - c0, (size_t)kMaxBatch);
            const GridRef* r = refs.data() + c0;
            hipError_t e = launch_predict(r, m, s);
            if (e == hipSuccess) e = launch_sort(r, m, s);
            if (e == hipSuccess) e = launch_update(r, m, s);
            if (e == hipSuccess) e = launch_moments(r, m, s);
            if (e == hipSuccess) e = launch_resample(r, m, s);
            if (e != hipSuccess) return hip_fail(e, "dogm_step_batch");
        }
    }
    for (int i = 0; i < n; ++i) grids[i]->cycle += 1;
    return DOGM_OK;
}

int dogm_sensor_truth(const double* rects, int32_t n_rects, const uint8_t* static_occ,
                      int32_t nx, int32_t ny, double cell_size, uint8_t* occ,
                      dogm_stream_t stream)
{
    if (nx < 1 || ny < 1 || (int64_t)nx * (int64_t)ny >= (int64_t(1) << 24) || !occ)
        return DOGM_EINVAL;
    if (n_rects < 0 || (n_rects > 0 && !rects)) return DOGM_EINVAL;
    if (!(std::isfinite(cell_size) && cell_size > 0.0)) return DOGM_EINVAL;
    const hipError_t e = launch_sensor_truth(rects, n_rects, static_occ, nx, ny, cell_size, occ,
                                             nullptr, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? DOGM_OK : hip_fail(e, "dogm_sensor_truth");
}

int dogm_sensor_scan(const uint8_t* occ, int32_t nx, int32_t ny, double p_d, double p_cl,
                     uint64_t seed, uint32_t cycle, uint8_t* seen, float* m_occ, float* m_free,
                     dogm_stream_t stream)
{
    if (nx < 1 || ny < 1 || (int64_t)nx * (int64_t)ny >= (int64_t(1) << 24)) return DOGM_EINVAL;
    if (!occ || !seen || (!m_occ) != (!m_free)) return DOGM_EINVAL;
    if (!(p_d >= 0.0 && p_d <= 1.0 && p_cl >= 0.0 && p_cl <= 1.0)) return DOGM_EINVAL;
    // evidence masses whose pignistic transform is the Bayesian occupancy with prior 1/2
    const double hit = p_d / (p_d + p_cl);
    const double miss = (1.0 - p_d) / ((1.0 - p_d) + (1.0 - p_cl));
    const double mo = 2.0 * hit - 1.0, mf = 1.0 - 2.0 * miss;
    if (!(mo >= 0.0 && mo <= 1.0 && mf >= 0.0 && mf <= 1.0)) return DOGM_EINVAL;
    const hipError_t e = launch_sensor_scan(occ, nx, ny, true, p_d, p_cl, (float)mo, (float)mf,
                                            seed, cycle, seen, m_occ, m_free,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? DOGM_OK : hip_fail(e, "dogm_sensor_scan");
}

const char* dogm_status_string(int code)
{
    switch (code) {
        case DOGM_OK: return "ok";
        case DOGM_EINVAL: return "invalid argument";
        case DOGM_ESIZE: return g_last_error.empty() ? "buffer too small" : g_last_error.c_str();
        case DOGM_EHIP: return g_last_error.empty() ? "HIP error" : g_last_error.c_str();
        case DOGM_ESTATE: return "call out of order";
        case DOGM_ENOTIMPL: return g_last_error.empty() ? "not implemented" : g_last_error.c_str();
        default: return "unknown status";
    }
}

const char* dogm_last_error(void) { return g_last_error.c_str(); }

int dogm_trace_begin(void* const* events, const char** names, int capacity, const char* kernel)
{
    if (capacity < 0 || (capacity > 0 && !events)) return DOGM_EINVAL;
    g_trace_storage = Trace{reinterpret_cast<hipEvent_t*>(const_cast<void**>(events)), names,
                            kernel, capacity, 0, hipSuccess};
    g_trace = &g_trace_storage;
    return DOGM_OK;
}

int dogm_trace_end(int* count)
{
    if (!g_trace) return DOGM_ESTATE;
    if (count) *count = g_trace->n;
    const hipError_t e = g_trace->err;
    g_trace = nullptr;
    return e == hipSuccess ? DOGM_OK : hip_fail(e, "dogm_trace_end");
}

}  // extern "C"
