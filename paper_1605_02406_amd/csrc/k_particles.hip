// Element-wise particle kernels: descriptor upload, initial state, prediction (Alg. 1), the
// gather into cell order with per-cell ranges (Alg. 2), the persistent weight update (Alg. 4)
// and the new-born particles (Alg. 5).
#include "launch.h"

namespace dogm {

__global__ void k_write_desc(GridDev hd, GridDev* dd) { *dd = hd; }

hipError_t launch_write_desc(const GridDev& hd, GridDev* dd, hipStream_t s)
{
    hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(1), 0, s, hd, dd);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Initial state: particles uniform over the grid, velocity N(0, sigma_B^2), weight 0; m_F = 0.
// ----------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kElemThreads) void k_init(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t i = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (i < G.nu) {
        const uint4 r = draw(G, i, 0u, kPurposeInit);
        float n0, n1;
        box_muller_f32(unit_f32(r.z), unit_f32(r.w), n0, n1);
        G.x[i] = unit_f32(r.x) * ((float)G.nx * G.r);
        G.y[i] = unit_f32(r.y) * ((float)G.ny * G.r);
        G.vx[i] = G.sig_birth * n0;
        G.vy[i] = G.sig_birth * n1;
        G.w[i] = 0.0f;
    }
    if (i < G.C) G.m_F[i] = 0.0f;
    if (i == 0) {
        *G.cycle = 1u;
        *G.status = 0u;
        *G.W_fixed = 0;
        *G.S_fixed = 0;
    }
}

hipError_t launch_init(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [](const GridDev& G) {
        return ceil_div(G.nu > G.C ? G.nu : G.C, kElemThreads);
    });
    if (blocks) hipLaunchKernelGGL(k_init, dim3(blocks), dim3(kElemThreads), 0, s, b);
    return hipGetLastError();
}

__global__ void k_set_cycle(Batch b, uint32_t cycle)
{
    if (threadIdx.x == 0) *b.g[blockIdx.x]->cycle = cycle;
}

hipError_t launch_set_cycle(const GridRef* g, int n, uint32_t cycle, hipStream_t s)
{
    Batch b;
    make_batch(b, g, n, [](const GridDev&) { return 1u; });
    hipLaunchKernelGGL(k_set_cycle, dim3(n), dim3(64), 0, s, b, cycle);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Alg. 1: constant-velocity prediction with Philox noise, persistence, cell key.
// ----------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kElemThreads) void k_predict(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t i = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (i >= G.nu) return;
    const uint32_t cycle = *G.cycle;
    const uint4 r = draw(G, i, cycle, kPurposePredict);
    float n0, n1, n2, n3;
    box_muller_f32(unit_f32(r.x), unit_f32(r.y), n0, n1);
    box_muller_f32(unit_f32(r.z), unit_f32(r.w), n2, n3);
    const float x = G.x[i], y = G.y[i], vx = G.vx[i], vy = G.vy[i], w = G.w[i];
    const float xn = x + G.dt * vx + G.sig_pos * n0;
    const float yn = y + G.dt * vy + G.sig_pos * n1;
    const float vxn = vx + G.sig_vel * n2;
    const float vyn = vy + G.sig_vel * n3;
    const uint32_t k = cell_of(G, xn, yn);
    G.x[i] = xn;
    G.y[i] = yn;
    G.vx[i] = vxn;
    G.vy[i] = vyn;
    G.w[i] = (k == G.C) ? 0.0f : G.p_s * w;
    G.key[i] = k;
}

hipError_t launch_predict(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.nu, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_predict, dim3(blocks), dim3(kElemThreads), 0, s, b);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Alg. 2 (after the sort): particles into cell order; first/last particle of a cell group
// writes the cell's range.  Cells are cleared first so empty cells read start == end.
// ----------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kElemThreads) void k_clear_cells(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t c = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (c < G.C) {
        G.cstart[c] = 0;
        G.cend[c] = 0;
    }
}

__global__ __launch_bounds__(kElemThreads) void k_gather(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t s = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (s >= G.nu) return;
    uint32_t src = G.perm[s];
    if (src >= G.nu) {  // cannot happen for a correct sort; reported, never dereferenced
        atomicOr(G.status, kStInternal);
        src = s;
    }
    G.sx[s] = G.x[src];
    G.sy[s] = G.y[src];
    G.svx[s] = G.vx[src];
    G.svy[s] = G.vy[src];
    G.sw[s] = G.w[src];
    const uint32_t k = G.skey[s];
    if (k < G.C) {
        if (s == 0 || G.skey[s - 1] != k) G.cstart[k] = s;
        if (s + 1 == G.nu || G.skey[s + 1] != k) G.cend[k] = s + 1;
    }
}

hipError_t launch_gather(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.C, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_clear_cells, dim3(blocks), dim3(kElemThreads), 0, s, b);
    blocks = make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.nu, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(kElemThreads), 0, s, b);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Alg. 4 (last loop): w <- p_A mu_A g w + (1 - p_A) mu_UA w on the sorted particles.
// ----------------------------------------------------------------------------------------------

__device__ __forceinline__ double velocity_likelihood(double vx, double vy, double mx,
                                                      double my, double var)
{
    const double dx = vx - mx, dy = vy - my;
    return exp(-(dx * dx + dy * dy) / (2.0 * var));
}

__global__ __launch_bounds__(kElemThreads) void k_weight_update(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const MeasDev& M = b.m[gi];
    const uint32_t s = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (s >= G.nu) return;
    const uint32_t k = G.skey[s];
    if (k >= G.C) return;
    const double w = (double)G.sw[s];
    const double mu_ua = G.mu_UA[k];
    double wn;
    if (M.p_assoc != nullptr && G.sum_wt[k] > 0.0) {
        const double pa = (double)M.p_assoc[k];
        const double g = velocity_likelihood((double)G.svx[s], (double)G.svy[s],
                                             (double)M.mu_vx[k], (double)M.mu_vy[k],
                                             (double)M.var_v[k]);
        wn = pa * G.mu_A[k] * (g * w) + (1.0 - pa) * mu_ua * w;
    } else {
        wn = mu_ua * w;
    }
    G.sw[s] = (float)wn;
}

hipError_t launch_weight_update(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.nu, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_weight_update, dim3(blocks), dim3(kElemThreads), 0, s, b);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Alg. 5: slot allocation from the exclusive prefix E_c of the fixed-point new-born masses
// (born_q after the scan), then one thread per slot initialises its particle.
// ----------------------------------------------------------------------------------------------

// o_c = floor(nu_b E_c / S) in FP64 with every operation rounded separately (no contraction);
// the caller handles c == C (o_C = nu_b).
__device__ __forceinline__ uint32_t slot_offset(uint64_t E, uint64_t S, uint32_t nb)
{
    const double t = __ddiv_rn(__dmul_rn((double)E, (double)nb), (double)S);
    const double o = floor(t);
    return o > (double)nb ? nb : (uint32_t)o;
}

__global__ __launch_bounds__(kElemThreads) void k_born_offsets(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t c = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (c > G.C) return;
    const uint64_t S = *G.S_fixed;
    if (S == 0) {
        G.born_off[c] = 0;
        return;
    }
    const uint32_t o = (c == G.C) ? G.nb : slot_offset(G.born_q[c], S, G.nb);
    G.born_off[c] = o;
    if (c < G.C && G.nb > 0 && G.rho_b[c] > 0.0f) {
        const uint32_t o1 = (c + 1 == G.C) ? G.nb : slot_offset(G.born_q[c + 1], S, G.nb);
        if (o1 == o) atomicOr(G.status, kStNoCarrier);
    }
}

__global__ __launch_bounds__(kElemThreads) void k_born_init(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const MeasDev& M = b.m[gi];
    const uint32_t s = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (s >= G.nb) return;
    if (*G.S_fixed == 0) {  // no new-born mass anywhere: empty slots
        G.bx[s] = G.by[s] = G.bvx[s] = G.bvy[s] = G.bw[s] = 0.0f;
        G.bkey[s] = G.C;
        G.bassoc[s] = 0;
        return;
    }
    // cell of the slot: the last c with born_off[c] <= s (born_off[0] = 0, born_off[C] = nb)
    uint32_t lo = 0, hi = G.C;  // invariant: born_off[lo] <= s < born_off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (G.born_off[mid] <= s) lo = mid; else hi = mid;
    }
    const uint32_t c = lo;
    const uint32_t o0 = G.born_off[c], o1 = G.born_off[c + 1];
    const uint32_t n_c = o1 - o0;
    const double pa = M.p_assoc ? (double)M.p_assoc[c] : 0.0;
    const uint32_t na = (uint32_t)floor(__dadd_rn(__dmul_rn(pa, (double)n_c), 0.5));
    const uint32_t nua = n_c - na;
    const bool assoc = (s - o0) < na;
    const double rb = (double)G.rho_b[c];
    double w;
    if (assoc) w = (nua == 0) ? rb / (double)na : pa * rb / (double)na;
    else w = (na == 0) ? rb / (double)nua : (1.0 - pa) * rb / (double)nua;
    const uint4 r = draw(G, s, *G.cycle, kPurposeBirth);
    float n0, n1;
    box_muller_f32(unit_f32(r.z), unit_f32(r.w), n0, n1);
    const uint32_t ix = c % (uint32_t)G.nx, iy = c / (uint32_t)G.nx;
    G.bx[s] = ((float)ix + unit_f32(r.x)) * G.r;
    G.by[s] = ((float)iy + unit_f32(r.y)) * G.r;
    if (assoc) {
        const float sd = sqrtf(M.var_v[c]);
        G.bvx[s] = M.mu_vx[c] + sd * n0;
        G.bvy[s] = M.mu_vy[c] + sd * n1;
    } else {
        G.bvx[s] = G.sig_birth * n0;
        G.bvy[s] = G.sig_birth * n1;
    }
    G.bw[s] = (float)w;
    G.bkey[s] = c;
    G.bassoc[s] = assoc ? 1 : 0;
}

hipError_t launch_births(const GridRef* g, int n, hipStream_t s)
{
    hipError_t e = launch_scan(g, n, ScanArray::BornMass, 0, s);
    if (e != hipSuccess) return e;
    Batch b;
    uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.C + 1, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_born_offsets, dim3(blocks), dim3(kElemThreads), 0, s, b);
    blocks = make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.nb, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_born_init, dim3(blocks), dim3(kElemThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace dogm
