// Per-cell work: sums over each cell's particles (Alg. 3 and 4), the Dempster-Shafer cell
// update with the new-born split (Alg. 3) and the velocity moments (Alg. 6).
//
// Per-cell sums are segmented reductions over the sorted particles instead of the paper's
// prefix-sum differences (a global FP32 prefix loses the digits of late cells).  Each wave owns
// a range of kSegRange particles and sums every cell whose first particle lies in that range,
// reading past the range end to finish its last cell; 64 particles at a time it runs a
// segmented inclusive scan across lanes (keys are sorted, so lanes with equal keys are
// contiguous) and carries the running sum of the last cell into the next chunk.  Accumulators
// are FP64 and the summation order depends only on the data, never on the launch.
#include "launch.h"

namespace dogm {

// One wave's share of a segmented reduction with NV FP64 sums per particle.
//   load(i, k, v): fill v[0..NV) for sorted particle i of cell k
//   emit(k, v)   : the complete sums of cell k
template <int NV, typename Load, typename Emit>
__device__ __forceinline__ void seg_reduce_wave(const GridDev& G, uint32_t wave_index, Load load,
                                                Emit emit)
{
    const int lane = lane_id();
    const uint32_t n = G.nu, C = G.C;
    const uint32_t a = wave_index * kSegRange;
    if (a >= n) return;
    const uint32_t b = min(a + (uint32_t)kSegRange, n);
    const uint32_t ka = G.skey[a];
    if (ka >= C) return;  // only particles outside the grid from here on
    uint32_t p0 = a;
    if (a > 0 && G.skey[a - 1] == ka) p0 = G.cend[ka];  // that cell belongs to an earlier wave
    if (p0 >= b) return;
    const uint32_t kl = G.skey[b - 1];
    const uint32_t pend = (kl < C) ? max(b, G.cend[kl]) : b;

    double carry[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) carry[j] = 0.0;
    uint32_t carry_key = 0xFFFFFFFFu;

    for (uint32_t base = p0; base < pend; base += kWave) {
        const uint32_t i = base + lane;
        uint32_t k = (i < pend) ? G.skey[i] : 0xFFFFFFFFu;
        if (k >= C) k = 0xFFFFFFFFu;
        const bool valid = k != 0xFFFFFFFFu;
        double v[NV];
        if (valid) {
            load(i, k, v);
        } else {
#pragma unroll
            for (int j = 0; j < NV; ++j) v[j] = 0.0;
        }
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t ko = __shfl_up(k, off, kWave);
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const double o = __shfl_up(v[j], off, kWave);
                if (lane >= off && ko == k) v[j] += o;
            }
        }
        if (valid && k == carry_key) {
#pragma unroll
            for (int j = 0; j < NV; ++j) v[j] += carry[j];
        }
        // key of the next particle: the next lane, or for the last lane the next chunk
        uint32_t knext = __shfl_down(k, 1, kWave);
        if (lane == kWave - 1) {
            knext = (i + 1 < pend) ? G.skey[i + 1] : 0xFFFFFFFFu;
            if (knext >= C) knext = 0xFFFFFFFFu;
        }
        if (valid && knext != k) emit(k, v);
        // the cell still open at the end of the chunk continues in the next one
        const uint32_t klast = __shfl(k, kWave - 1, kWave);
        const uint32_t knl = __shfl(knext, kWave - 1, kWave);
        carry_key = (klast != 0xFFFFFFFFu && knl == klast) ? klast : 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < NV; ++j) carry[j] = __shfl(v[j], kWave - 1, kWave);
    }
}

// ----------------------------------------------------------------------------------------------
// Alg. 3 (sums) and Alg. 4 (sums of w~ = g w): per-cell FP64 sums of the predicted weights.
// ----------------------------------------------------------------------------------------------

__device__ __forceinline__ double likelihood(double vx, double vy, double mx, double my,
                                             double var)
{
    const double dx = vx - mx, dy = vy - my;
    return exp(-(dx * dx + dy * dy) / (2.0 * var));
}

template <bool kAssoc>
__global__ __launch_bounds__(kSegThreads) void k_seg_weights(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const MeasDev& M = b.m[gi];
    const uint32_t wave = (blockIdx.x - b.bstart[gi]) * (kSegThreads / kWave) + threadIdx.x / kWave;
    if (kAssoc) {
        seg_reduce_wave<2>(
            G, wave,
            [&](uint32_t i, uint32_t k, double* v) {
                const double w = (double)G.sw[i];
                v[0] = w;
                v[1] = likelihood((double)G.svx[i], (double)G.svy[i], (double)M.mu_vx[k],
                                  (double)M.mu_vy[k], (double)M.var_v[k]) * w;
            },
            [&](uint32_t k, const double* v) {
                G.sum_w[k] = v[0];
                G.sum_wt[k] = v[1];
            });
    } else {
        seg_reduce_wave<1>(
            G, wave, [&](uint32_t i, uint32_t, double* v) { v[0] = (double)G.sw[i]; },
            [&](uint32_t k, const double* v) { G.sum_w[k] = v[0]; });
    }
}

// Per cell, FP64: predicted BBA (eqs. (DS_particle_sum_pred), (DS_freespace_pred)), Dempster
// combination with the measurement (eq. (DS_comb)), new-born split (eqs.
// (DS_resulting_masses1/2), new-born mass only where m_z(O) > 0), normalisation components
// (eqs. (DSnormalizationfactor), (DSnormalizationfactor2)) and the fixed-point new-born mass.
__global__ __launch_bounds__(kElemThreads) void k_cell_update(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const MeasDev& M = b.m[gi];
    const uint32_t c = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (c >= G.C) return;
    const bool nonempty = G.cend[c] > G.cstart[c];
    const double s = nonempty ? G.sum_w[c] : 0.0;
    if (!nonempty) G.sum_w[c] = 0.0;
    const double st = (nonempty && M.p_assoc != nullptr) ? G.sum_wt[c] : 0.0;
    const double po = s < 1.0 ? s : 1.0;
    const double pf_cand = (double)G.alpha * (double)G.m_F[c];
    const double pf = pf_cand < 1.0 - po ? pf_cand : 1.0 - po;
    const double zo = (double)M.m_occ[c], zf = (double)M.m_free[c];
    // Dempster's rule on {O, F}: conflict K = o1 f2 + f1 o2
    const double u1 = 1.0 - po - pf, u2 = 1.0 - zo - zf;
    const double K = po * zf + pf * zo;
    const double norm = 1.0 - K;
    double o, f;
    uint32_t st_bits = 0;
    if (norm >= 1e-12) {
        o = (po * zo + po * u2 + u1 * zo) / norm;
        f = (pf * zf + pf * u2 + u1 * zf) / norm;
    } else {
        o = po;
        f = pf;
        st_bits |= kStConflict;
    }
    double rb = 0.0;
    if (zo > 0.0) {
        const double a = (double)G.p_b * (1.0 - po);
        const double den = po + a;
        rb = den > 0.0 ? o * a / den : 0.0;
    }
    const double rp = o - rb;
    const double mu_ua = s > 0.0 ? rp / s : 0.0;
    const double mu_a = st > 0.0 ? rp / st : 0.0;
    if (!isfinite(o) || !isfinite(f) || !isfinite(s)) st_bits |= kStNonFinite;
    const float rbf = (float)rb;
    G.m_pO[c] = (float)po;
    G.m_pF[c] = (float)pf;
    G.m_O[c] = (float)o;
    G.m_F[c] = (float)f;
    G.rho_b[c] = rbf;
    G.rho_p[c] = (float)rp;
    G.pign[c] = (float)(o + 0.5 * (1.0 - o - f));
    G.mu_UA[c] = mu_ua;
    G.mu_A[c] = mu_a;
    G.born_q[c] = fixed40(rbf);
    if (st_bits) atomicOr(G.status, st_bits);
}

hipError_t launch_cell_update(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.nu, kSegBlockParticles); });
    bool any_assoc = false, all_assoc = true;
    for (int i = 0; i < n; ++i) {
        any_assoc |= g[i].m.p_assoc != nullptr;
        all_assoc &= g[i].m.p_assoc != nullptr;
    }
    if (any_assoc && !all_assoc) return hipErrorInvalidValue;  // one kind per launch
    if (blocks) {
        if (any_assoc)
            hipLaunchKernelGGL(k_seg_weights<true>, dim3(blocks), dim3(kSegThreads), 0, s, b);
        else
            hipLaunchKernelGGL(k_seg_weights<false>, dim3(blocks), dim3(kSegThreads), 0, s, b);
    }
    blocks = make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.C, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_cell_update, dim3(blocks), dim3(kElemThreads), 0, s, b);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Alg. 6: velocity moments.  Sums are shifted by the velocity (a, b) of the cell's first
// particle:  S0 = sum w, S1 = sum w (vx - a), S2 = sum w (vy - b), S3 = sum w (vx - a)^2,
// S4 = sum w (vy - b)^2, S5 = sum w (vx - a)(vy - b).  With s = S0 / rho_p and
// d_x = S1 / rho_p + a (s - 1) these give exactly the printed moments
//   mean_x = a + d_x,   var_x = S3 / rho_p - d_x^2 - a^2 (s - 1),
//   cov_xy = S5 / rho_p - d_x d_y - a b (s - 1),
// without the cancellation of E[v^2] - mean^2.
// ----------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kSegThreads) void k_seg_moments(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t wave = (blockIdx.x - b.bstart[gi]) * (kSegThreads / kWave) + threadIdx.x / kWave;
    seg_reduce_wave<6>(
        G, wave,
        [&](uint32_t i, uint32_t k, double* v) {
            const uint32_t h = G.cstart[k];
            const double w = (double)G.sw[i];
            const double dx = (double)G.svx[i] - (double)G.svx[h];
            const double dy = (double)G.svy[i] - (double)G.svy[h];
            v[0] = w;
            v[1] = w * dx;
            v[2] = w * dy;
            v[3] = w * dx * dx;
            v[4] = w * dy * dy;
            v[5] = w * dx * dy;
        },
        [&](uint32_t k, const double* v) {
            const double rp = (double)G.rho_p[k];
            if (!(rp > 0.0)) {
                G.mean_x[k] = G.mean_y[k] = G.var_x[k] = G.var_y[k] = G.cov_xy[k] = 0.0f;
                G.mflag[k] = 0;
                return;
            }
            const uint32_t h = G.cstart[k];
            const double a = (double)G.svx[h], bb = (double)G.svy[h];
            const double sm1 = (v[0] - rp) / rp;  // s - 1
            const double dx = v[1] / rp + a * sm1;
            const double dy = v[2] / rp + bb * sm1;
            G.mean_x[k] = (float)(a + dx);
            G.mean_y[k] = (float)(bb + dy);
            G.var_x[k] = (float)(v[3] / rp - dx * dx - a * a * sm1);
            G.var_y[k] = (float)(v[4] / rp - dy * dy - bb * bb * sm1);
            G.cov_xy[k] = (float)(v[5] / rp - dx * dy - a * bb * sm1);
            G.mflag[k] = 1;
        });
}

__global__ __launch_bounds__(kElemThreads) void k_moments_empty(Batch b)
{
    const int gi = batch_grid(b);
    const GridDev& G = *b.g[gi];
    const uint32_t c = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (c >= G.C || G.cend[c] > G.cstart[c]) return;
    G.mean_x[c] = G.mean_y[c] = G.var_x[c] = G.var_y[c] = G.cov_xy[c] = 0.0f;
    G.mflag[c] = 0;
}

hipError_t launch_moments(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.nu, kSegBlockParticles); });
    if (blocks) hipLaunchKernelGGL(k_seg_moments, dim3(blocks), dim3(kSegThreads), 0, s, b);
    blocks = make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.C, kElemThreads); });
    if (blocks) hipLaunchKernelGGL(k_moments_empty, dim3(blocks), dim3(kElemThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace dogm
