// Host side of the C ABI declared in include/dogm.h: validation, arena layout, call order and
// the batched cycle.  All device work is in the k_*.hip kernels; nothing here computes filter
// values and nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dogm.h"
#include "launch.h"

using namespace dogm;

namespace {

enum Phase { kReady = 0, kPredicted = 1, kAssigned = 2, kUpdated = 3, kMoments = 4 };

thread_local std::string g_last_error;

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
    if ((int64_t)p->nx * (int64_t)p->ny >= (int64_t(1) << 26)) return false;
    if (!(std::isfinite(p->cell_size) && p->cell_size > 0.0f)) return false;
    if (!finite_in(p->dt, 0.0f, 1e6f)) return false;
    if (!finite_in(p->p_s, 0.0f, 1.0f) || !finite_in(p->p_b, 0.0f, 1.0f)) return false;
    if (!finite_in(p->sigma_pos, 0.0f, 1e6f) || !finite_in(p->sigma_vel, 0.0f, 1e6f) ||
        !finite_in(p->sigma_birth_vel, 0.0f, 1e6f))
        return false;
    if (!finite_in(p->alpha_free, 0.0f, 1.0f)) return false;
    if (p->n_pers < 1 || p->n_pers >= (int64_t(1) << 30)) return false;
    if (p->n_born < 0 || p->n_born >= (int64_t(1) << 30)) return false;
    if (p->reserved != 0) return false;
    return true;
}

// Offsets of every array inside the arena (the descriptor sits at offset 0).
struct Layout {
    size_t total = 0;
    size_t take(size_t bytes)
    {
        const size_t o = (total + 255) & ~size_t(255);
        total = o + (bytes ? bytes : 1);
        return o;
    }
};

template <typename T>
T* at(char* base, size_t off)
{
    return reinterpret_cast<T*>(base + off);
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
    d.n_sort_tiles = ceil_div(nu, kSortTile);
    d.n_res_tiles = ceil_div((uint64_t)nu + nb, kResTile);

    Layout L;
    L.take(sizeof(GridDev));
    const size_t f_nu = 4ull * nu, f_nb = 4ull * nb, f_c = 4ull * C, d_c = 8ull * C;
    size_t o_x = L.take(f_nu), o_y = L.take(f_nu), o_vx = L.take(f_nu), o_vy = L.take(f_nu),
           o_w = L.take(f_nu), o_key = L.take(f_nu);
    size_t o_sx = L.take(f_nu), o_sy = L.take(f_nu), o_svx = L.take(f_nu), o_svy = L.take(f_nu),
           o_sw = L.take(f_nu), o_skey = L.take(f_nu), o_perm = L.take(f_nu);
    size_t o_tkey = L.take(f_nu), o_tval = L.take(f_nu);
    size_t o_hist = L.take(4ull * (1u << kMaxDigitBits) * d.n_sort_tiles);
    size_t o_cs = L.take(f_c), o_ce = L.take(f_c), o_sumw = L.take(d_c), o_sumwt = L.take(d_c);
    size_t o_mpo = L.take(f_c), o_mpf = L.take(f_c), o_mo = L.take(f_c), o_mf = L.take(f_c),
           o_rb = L.take(f_c), o_rp = L.take(f_c), o_pign = L.take(f_c);
    size_t o_mua = L.take(d_c), o_muua = L.take(d_c), o_bq = L.take(d_c),
           o_boff = L.take(4ull * (C + 1));
    size_t o_mx = L.take(f_c), o_my = L.take(f_c), o_vx2 = L.take(f_c), o_vy2 = L.take(f_c),
           o_cxy = L.take(f_c), o_mfl = L.take(C);
    size_t o_bx = L.take(f_nb), o_by = L.take(f_nb), o_bvx = L.take(f_nb), o_bvy = L.take(f_nb),
           o_bw = L.take(f_nb), o_bkey = L.take(f_nb), o_bas = L.take(nb);
    size_t o_rt = L.take(8ull * d.n_res_tiles), o_rl = L.take(4ull * d.n_res_tiles);
    const uint32_t scan_tiles_c = ceil_div(C, kScanTile);
    const uint32_t scan_tiles_h = ceil_div((uint64_t)(1u << kMaxDigitBits) * d.n_sort_tiles, kScanTile);
    size_t o_sp = L.take(8ull * ((scan_tiles_c > scan_tiles_h ? scan_tiles_c : scan_tiles_h) + 1));
    size_t o_cyc = L.take(4), o_st = L.take(4), o_W = L.take(8), o_S = L.take(8),
           o_last = L.take(4), o_U = L.take(8);
    *bytes = L.total;
    if (!base) return d;

    d.x = at<float>(base, o_x);
    d.y = at<float>(base, o_y);
    d.vx = at<float>(base, o_vx);
    d.vy = at<float>(base, o_vy);
    d.w = at<float>(base, o_w);
    d.key = at<uint32_t>(base, o_key);
    d.sx = at<float>(base, o_sx);
    d.sy = at<float>(base, o_sy);
    d.svx = at<float>(base, o_svx);
    d.svy = at<float>(base, o_svy);
    d.sw = at<float>(base, o_sw);
    d.skey = at<uint32_t>(base, o_skey);
    d.perm = at<uint32_t>(base, o_perm);
    d.tkey = at<uint32_t>(base, o_tkey);
    d.tval = at<uint32_t>(base, o_tval);
    d.hist = at<uint32_t>(base, o_hist);
    d.cstart = at<uint32_t>(base, o_cs);
    d.cend = at<uint32_t>(base, o_ce);
    d.sum_w = at<double>(base, o_sumw);
    d.sum_wt = at<double>(base, o_sumwt);
    d.m_pO = at<float>(base, o_mpo);
    d.m_pF = at<float>(base, o_mpf);
    d.m_O = at<float>(base, o_mo);
    d.m_F = at<float>(base, o_mf);
    d.rho_b = at<float>(base, o_rb);
    d.rho_p = at<float>(base, o_rp);
    d.pign = at<float>(base, o_pign);
    d.mu_A = at<double>(base, o_mua);
    d.mu_UA = at<double>(base, o_muua);
    d.born_q = at<uint64_t>(base, o_bq);
    d.born_off = at<uint32_t>(base, o_boff);
    d.mean_x = at<float>(base, o_mx);
    d.mean_y = at<float>(base, o_my);
    d.var_x = at<float>(base, o_vx2);
    d.var_y = at<float>(base, o_vy2);
    d.cov_xy = at<float>(base, o_cxy);
    d.mflag = at<uint8_t>(base, o_mfl);
    d.bx = at<float>(base, o_bx);
    d.by = at<float>(base, o_by);
    d.bvx = at<float>(base, o_bvx);
    d.bvy = at<float>(base, o_bvy);
    d.bw = at<float>(base, o_bw);
    d.bkey = at<uint32_t>(base, o_bkey);
    d.bassoc = at<uint8_t>(base, o_bas);
    d.res_tile = at<uint64_t>(base, o_rt);
    d.res_last = at<int32_t>(base, o_rl);
    d.scan_part = at<uint64_t>(base, o_sp);
    d.cycle = at<uint32_t>(base, o_cyc);
    d.status = at<uint32_t>(base, o_st);
    d.W_fixed = at<uint64_t>(base, o_W);
    d.S_fixed = at<uint64_t>(base, o_S);
    d.last_pos = at<int32_t>(base, o_last);
    d.U = at<double>(base, o_U);
    return d;
}

bool valid_meas(const dogm_meas* m)
{
    if (!m || !m->m_occ || !m->m_free) return false;
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
    if (arena_bytes < need) return DOGM_ESIZE;
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
    hipError_t e = launch_write_desc(g->hd, g->dd, g->stream);
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
    if (e == hipSuccess) e = launch_gather(&r, 1, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_assign");
    grid->phase = kAssigned;
    return DOGM_OK;
}

int dogm_update(dogm_grid* grid, const dogm_meas* meas)
{
    if (!grid || !valid_meas(meas)) return DOGM_EINVAL;
    if (grid->phase != kAssigned) return DOGM_ESTATE;
    const GridRef r = grid->ref(meas);
    hipError_t e = launch_cell_update(&r, 1, grid->stream);
    if (e == hipSuccess) e = launch_weight_update(&r, 1, grid->stream);
    if (e == hipSuccess) e = launch_births(&r, 1, grid->stream);
    if (e != hipSuccess) return hip_fail(e, "dogm_update");
    grid->phase = kUpdated;
    return DOGM_OK;
}

int dogm_moments(dogm_grid* grid)
{
    if (!grid) return DOGM_EINVAL;
    if (grid->phase != kUpdated && grid->phase != kMoments) return DOGM_ESTATE;
    const GridRef r = grid->ref();
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
    if (!grid || !valid_meas(meas)) return DOGM_EINVAL;
    if (grid->phase != kReady) return DOGM_ESTATE;
    int rc = dogm_predict(grid);
    if (rc == DOGM_OK) rc = dogm_assign(grid);
    if (rc == DOGM_OK) rc = dogm_update(grid, meas);
    if (rc == DOGM_OK) rc = dogm_moments(grid);
    if (rc == DOGM_OK) rc = dogm_resample(grid);
    return rc;
}

int dogm_step_batch(dogm_grid* const* grids, const dogm_meas* meas, int n, dogm_stream_t stream)
{
    if (n < 0 || (n > 0 && (!grids || !meas))) return DOGM_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!grids[i] || !valid_meas(&meas[i])) return DOGM_EINVAL;
        if (grids[i]->phase != kReady) return DOGM_ESTATE;
        for (int j = 0; j < i; ++j)
            if (grids[j] == grids[i]) return DOGM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // one launch per kernel for up to kMaxBatch grids; grids with and without velocity
    // evidence go to separate launches of the update
    for (int kind = 0; kind < 2; ++kind) {
        std::vector<GridRef> refs;
        for (int i = 0; i < n; ++i)
            if ((meas[i].p_assoc != nullptr) == (kind == 1)) refs.push_back(grids[i]->ref(&meas[i]));
        for (size_t c0 = 0; c0 < refs.size(); c0 += kMaxBatch) {
            const int m = (int)std::min(refs.size() - c0, (size_t)kMaxBatch);
            const GridRef* r = refs.data() + c0;
            hipError_t e = launch_predict(r, m, s);
            if (e == hipSuccess) e = launch_sort(r, m, s);
            if (e == hipSuccess) e = launch_gather(r, m, s);
            if (e == hipSuccess) e = launch_cell_update(r, m, s);
            if (e == hipSuccess) e = launch_weight_update(r, m, s);
            if (e == hipSuccess) e = launch_births(r, m, s);
            if (e == hipSuccess) e = launch_moments(r, m, s);
            if (e == hipSuccess) e = launch_resample(r, m, s);
            if (e != hipSuccess) return hip_fail(e, "dogm_step_batch");
        }
    }
    for (int i = 0; i < n; ++i) grids[i]->cycle += 1;
    return DOGM_OK;
}

const char* dogm_status_string(int code)
{
    switch (code) {
        case DOGM_OK: return "ok";
        case DOGM_EINVAL: return "invalid argument";
        case DOGM_ESIZE: return "arena too small";
        case DOGM_EHIP: return g_last_error.empty() ? "HIP error" : g_last_error.c_str();
        case DOGM_ESTATE: return "call out of order";
        case DOGM_ENOTIMPL: return "not implemented";
        default: return "unknown status";
    }
}

const char* dogm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
