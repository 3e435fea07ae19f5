// Per-cell work over the sorted particles: the particle range of every cell (Alg. 2), the
// Dempster-Shafer cell update with the new-born split (Alg. 3), the normalisation components of
// the persistent update (Alg. 4) and the velocity moments (Alg. 6).
//
// Two passes.  The first is particle-parallel: per-cell sums are segmented reductions over the
// sorted particles instead of the paper's prefix-sum differences (a global FP32 prefix loses the
// digits of late cells).  Each wave owns 64 * kSegItems particles and every cell whose first
// particle lies there, reading on past its range to finish its last cell.  Within a chunk each
// lane adds up kSegItems consecutive particles, closing the cells that end inside it, and one
// segmented scan across the lanes joins the cells that span lanes; the running sum of a cell
// still open at the end of the chunk is carried into the next one.  Accumulators are FP64 and
// the summation order depends only on the data, never on the launch or the batch.  A closed
// cell only stores its sums; the particles where a cell's run opens and closes store its range.
// The second pass is cell-parallel: one thread per cell
// (empty or not) runs the update with every lane of the wave busy.
//
// Without velocity evidence (p_A = 0) the updated persistent weights are w' = mu_UA w, so the
// velocity moments of the updated particles, normalised by rho_p = mu_UA sum w, equal the plain
// weighted moments of the predicted ones: the first pass also sums w v, w v^2 and w vx vy, and
// the second writes masses and moments together.  With velocity evidence the moments need the
// updated weights and take a pass of their own.
#include "launch.h"

namespace dogm {

constexpr uint32_t kNone = 0xFFFFFFFFu;

// One wave's share of a segmented reduction with NV FP64 sums per particle.
//   val(k, w, vx, vy, v): v[0..NV) of a particle of cell k with weight w and velocity (vx, vy)
//   emit(k, v)          : the complete sums of cell k (called once per cell, by one lane)
// The wave finds its first cell from the keys (the first particle whose cell differs from the
// one before the wave's share) and finishes the cell of its last particle past its share.
// kRanges: also store the range of every cell it handles.
template <int NV, bool kRanges, typename R, typename Val, typename Emit>
__device__ __forceinline__ void seg_reduce(const GridView& G, uint32_t wave_index, Val val,
                                           Emit emit)
{
    const auto SW = real<R>(G.sw), SVX = real<R>(G.svx), SVY = real<R>(G.svy);
    const int lane = lane_id();
    const uint32_t n = G.nu, C = G.C;
    const uint32_t a = wave_index * kSegRange;
    if (a >= n) return;
    const uint32_t b = min(a + (uint32_t)kSegRange, n);

    // chunks of kSegRange particles at fixed offsets from a; the first chunk is read while the
    // wave's first cell is looked up (particles before p0 are masked out below)
    uint32_t key[kSegItems];
    R pw[kSegItems], pvx[kSegItems], pvy[kSegItems];
    auto load_keys = [&](uint32_t base, uint32_t bound) {
        const uint32_t i0 = base + lane * kSegItems;
        if (i0 + kSegItems <= bound) {  // a lane's items are whole 16-byte vectors
#pragma unroll
            for (int q = 0; q < kSegItems; q += 4) {
                const u32x4 k4 = G.skey.load_vec<u32x4>(i0 + q);
#pragma unroll
                for (int e = 0; e < 4; ++e) key[q + e] = k4[e];
            }
        } else {
#pragma unroll
            for (int it = 0; it < kSegItems; ++it)
                key[it] = (i0 + it < bound) ? G.skey[i0 + it] : kNone;
        }
    };
    auto load_state = [&](uint32_t base, uint32_t bound) {
        const uint32_t i0 = base + lane * kSegItems;
        if (i0 + kSegItems <= bound) {
            // 16-byte vectors: four FP32 or two FP64 elements
            using V = typename RealVec16<R>::type;
            constexpr int kVec = 16 / (int)sizeof(R);
#pragma unroll
            for (int q = 0; q < kSegItems; q += kVec) {
                const V w4 = SW.template load_vec<V>(i0 + q);
                const V x4 = SVX.template load_vec<V>(i0 + q);
                const V y4 = SVY.template load_vec<V>(i0 + q);
#pragma unroll
                for (int e = 0; e < kVec; ++e) {
                    pw[q + e] = w4[e];
                    pvx[q + e] = x4[e];
                    pvy[q + e] = y4[e];
                }
            }
        } else {
#pragma unroll
            for (int it = 0; it < kSegItems; ++it) {
                const uint32_t i = i0 + it;
                pw[it] = (i < bound) ? SW[i] : (R)0;
                pvx[it] = (i < bound) ? SVX[i] : (R)0;
                pvy[it] = (i < bound) ? SVY[i] : (R)0;
            }
        }
    };
    load_keys(a, b);
    load_state(a, b);
    const uint32_t kprev = a > 0 ? G.skey[a - 1] : kNone;
    // p0: the first particle in [a, b) whose cell differs from that of the particle before a
    // (keys past b read as kNone, so a wave whose range holds no cell start finds p0 >= b)
    uint32_t lfirst = kSegItems, kfirst = kNone;
#pragma unroll
    for (int it = kSegItems - 1; it >= 0; --it)
        if (key[it] != kprev) {
            lfirst = it;
            kfirst = key[it];
        }
    const uint64_t has = __ballot(lfirst < (uint32_t)kSegItems);
    if (has == 0) return;
    const int l0 = __ffsll((unsigned long long)has) - 1;
    const uint32_t p0 = a + l0 * kSegItems + __shfl(lfirst, l0, kWave);
    if (p0 >= b || __shfl(kfirst, l0, kWave) >= C) return;  // no cell starts here
    // the cell of the range's last particle, which this wave finishes past b
    const uint32_t ib = (b - 1 - a) % kSegItems;
    uint32_t kb = kNone;
#pragma unroll
    for (int it = 0; it < kSegItems; ++it)
        if ((uint32_t)it == ib) kb = key[it];
    const uint32_t kl = __shfl(kb, (int)((b - 1 - a) / kSegItems), kWave);

    double carry[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) carry[j] = 0.0;
    uint32_t carry_key = kNone;
    uint32_t before_chunk = kNone;  // masked key of the particle before the chunk

    for (uint32_t base = a;; base += kSegRange) {
        if (base != a) {
            // past the wave's share only the run of kl continues: its state is read up to the
            // first particle of another cell
            load_keys(base, n);
            uint32_t lend = kSegItems;
#pragma unroll
            for (int it = kSegItems - 1; it >= 0; --it)
                if (key[it] != kl) lend = it;
            const uint64_t other = __ballot(lend < (uint32_t)kSegItems);
            const int lo = other ? __ffsll((unsigned long long)other) - 1 : kWave;
            const uint32_t run_end =
                lo < kWave ? base + lo * kSegItems + __shfl(lend, lo, kWave) : base + kSegRange;
            load_state(base, min(run_end, n));
        }
        const uint32_t i0 = base + lane * kSegItems;
        // particles outside [p0, end of kl's run) and outside the grid take no part
#pragma unroll
        for (int it = 0; it < kSegItems; ++it) {
            const uint32_t i = i0 + it;
            if (i < p0 || key[it] >= C || (i >= b && key[it] != kl)) key[it] = kNone;
        }
        const uint32_t first = key[0];
        uint32_t cur = key[0];
        bool multi = false;
        double head[NV], acc[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) head[j] = acc[j] = 0.0;
#pragma unroll
        for (int it = 0; it < kSegItems; ++it) {
            const uint32_t k = key[it];
            if (it > 0 && k != cur) {  // the cell `cur` ends inside this lane
                if (!multi) {
#pragma unroll
                    for (int j = 0; j < NV; ++j) head[j] = acc[j];
                    multi = true;
                } else if (cur != kNone) {
                    emit(cur, acc);  // began and ended inside this lane
                }
#pragma unroll
                for (int j = 0; j < NV; ++j) acc[j] = 0.0;
                cur = k;
            }
            if (k != kNone) {
                double v[NV];
                val(k, (double)pw[it], (double)pvx[it], (double)pvy[it], v);
#pragma unroll
                for (int j = 0; j < NV; ++j) acc[j] += v[j];
            }
        }
        const uint32_t prev_tail = __shfl_up(cur, 1, kWave);
        // the cell carried in from the previous chunk continues in lane 0
        if (lane == 0 && first != kNone && first == carry_key) {
            if (multi) {
#pragma unroll
                for (int j = 0; j < NV; ++j) head[j] += carry[j];
            } else {
#pragma unroll
                for (int j = 0; j < NV; ++j) acc[j] += carry[j];
            }
        }
        // join the tail cells across lanes: a lane's tail continues the previous lane's tail
        // when the lane holds a single cell equal to it
        bool start = lane == 0 || multi || prev_tail != cur || cur == kNone;
        double run[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) run[j] = acc[j];
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const bool so = __shfl_up(start ? 1 : 0, off, kWave) != 0;
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const double o = __shfl_up(run[j], off, kWave);
                if (lane >= off && !start) run[j] += o;
            }
            if (lane >= off && !start) start = so;
        }
        // a multi-cell lane closes its head cell, joined with the previous lane's tail
        double prev_run[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) prev_run[j] = __shfl_up(run[j], 1, kWave);
        if (multi && first != kNone) {
            if (lane > 0 && prev_tail == first) {
#pragma unroll
                for (int j = 0; j < NV; ++j) head[j] += prev_run[j];
            }
            emit(first, head);
        }
        // a tail cell ends here unless the next lane (or the next chunk) continues it
        uint32_t next_first = __shfl_down(first, 1, kWave);
        if (lane == kWave - 1) {
            const uint32_t inext = base + kSegRange;  // >= b: only kl's run continues
            next_first = (inext < n) ? G.skey[inext] : kNone;
            if (next_first >= C || next_first != kl) next_first = kNone;
        }
        if (cur != kNone && next_first != cur) emit(cur, run);
        if (kRanges) {
            // Alg. 2: a particle whose neighbour before (after) it belongs to another cell
            // opens (closes) its cell's run
            const uint32_t up = __shfl_up(key[kSegItems - 1], 1, kWave);  // every lane takes part
            const uint32_t left = lane == 0 ? before_chunk : up;
#pragma unroll
            for (int it = 0; it < kSegItems; ++it) {
                const uint32_t k = key[it];
                if (k == kNone) continue;
                const uint32_t kp = it == 0 ? left : key[it - 1];
                const uint32_t kn = it == kSegItems - 1 ? next_first : key[it + 1];
                if (kp != k) G.cstart[k] = i0 + it;
                if (kn != k) G.cend[k] = i0 + it + 1;
            }
        }
        before_chunk = __shfl(key[kSegItems - 1], kWave - 1, kWave);
        const uint32_t t63 = __shfl(cur, kWave - 1, kWave);
        const uint32_t n63 = __shfl(next_first, kWave - 1, kWave);
        carry_key = (t63 != kNone && n63 == t63) ? t63 : kNone;
        if (carry_key == kNone) break;
#pragma unroll
        for (int j = 0; j < NV; ++j) carry[j] = __shfl(run[j], kWave - 1, kWave);
    }
}

__device__ __forceinline__ double likelihood(double vx, double vy, double mx, double my,
                                             double var)
{
    const double dx = vx - mx, dy = vy - my;
    return exp(-(dx * dx + dy * dy) / (2.0 * var));
}

// Per cell, FP64: predicted BBA (eqs. (DS_particle_sum_pred), (DS_freespace_pred)), Dempster
// combination with the measurement (eq. (DS_comb)), new-born split (eqs.
// (DS_resulting_masses1/2), new-born mass only where m_z(O) > 0) and the normalisation
// components (eqs. (DSnormalizationfactor), (DSnormalizationfactor2)).  s = sum of predicted
// weights, st = sum of g w.  Returns rho_p; *rb_out gets the stored rho_b.
// The particle PHD/MIB model (Sec. V, p_A = 0), FP64: predicted existence r = r_p + r_b with
// r_p = min(s, 1) (eq. (predExistenceProbParticles), truncated) and r_b = p_B (1 - r_p) (eq.
// (pred_birth_prob)); every weight of the cell is scaled by the factor of eqs.
// (updateParticleWeightsUnnormalized), (applyNormalization), (normalizationCalculation) after a
// measurement, of eq. (updateParticleWeightsEmpty) without one.  Same outputs as cell_update.
template <typename R>
__device__ __forceinline__ double cell_update_phd(const GridView& G, const MeasView& M,
                                                  uint32_t c, double s, R* rb_out)
{
    const double rp = s < 1.0 ? s : 1.0;
    const double rb_pred = (double)G.p_b * (1.0 - rp);
    const double r = rp + rb_pred;
    const double tp = (double)M.p_tp[c], fp = (double)M.p_fp[c];
    const double f = M.det[c] != 0.0f ? tp / (fp * (1.0 - r) + tp * r)
                                      : (1.0 - tp) / ((1.0 - tp) * r + (1.0 - fp) * (1.0 - r));
    const double o = f * r, rho_p = f * rp, rb = f * rb_pred;
    if (!isfinite(f) || !isfinite(s)) status_or(G, kStNonFinite);
    real<R>(G.m_pO)[c] = (R)rp;
    real<R>(G.m_pF)[c] = (R)(1.0 - r);
    real<R>(G.m_O)[c] = (R)o;
    real<R>(G.m_F)[c] = (R)(1.0 - o);
    real<R>(G.rho_b)[c] = (R)rb;
    real<R>(G.rho_p)[c] = (R)rho_p;
    real<R>(G.pign)[c] = (R)o;
    G.mu_UA[c] = s > 0.0 ? rho_p / s : 0.0;
    G.mu_A[c] = G.mu_UA[c];
    *rb_out = (R)rb;
    return rho_p;
}

template <typename R>
__device__ __forceinline__ double cell_update(const GridView& G, const MeasView& M, uint32_t c,
                                              double s, double st, R* rb_out)
{
    if (G.model == kModelPhdMib) return cell_update_phd<R>(G, M, c, s, rb_out);
    const double po = s < 1.0 ? s : 1.0;
    const double pf_cand = (double)G.alpha * (double)real<R>(G.m_F)[c];
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
    if (!isfinite(o) || !isfinite(f) || !isfinite(s)) st_bits |= kStNonFinite;
    real<R>(G.m_pO)[c] = (R)po;
    real<R>(G.m_pF)[c] = (R)pf;
    real<R>(G.m_O)[c] = (R)o;
    real<R>(G.m_F)[c] = (R)f;
    real<R>(G.rho_b)[c] = (R)rb;
    real<R>(G.rho_p)[c] = (R)rp;
    real<R>(G.pign)[c] = (R)(o + 0.5 * (1.0 - o - f));
    G.mu_UA[c] = s > 0.0 ? rp / s : 0.0;
    G.mu_A[c] = st > 0.0 ? rp / st : 0.0;
    if (st_bits) status_or(G, st_bits);
    *rb_out = (R)rb;
    return rp;
}

// Moments are defined where the stored rho_p is positive and the cell holds particles (the
// caller decides); sums over weights that are all zero give zero moments.
template <typename R>
__device__ __forceinline__ void write_moments(const GridView& G, uint32_t c, bool defined,
                                              double norm, double sx, double sy, double sxx,
                                              double syy, double sxy)
{
    if (!defined || !(norm > 0.0)) {
        real<R>(G.mean_x)[c] = real<R>(G.mean_y)[c] = (R)0;
        real<R>(G.var_x)[c] = real<R>(G.var_y)[c] = real<R>(G.cov_xy)[c] = (R)0;
        G.mflag[c] = defined ? 1 : 0;
        return;
    }
    const double inv = 1.0 / norm;
    const double mx = sx * inv, my = sy * inv;
    real<R>(G.mean_x)[c] = (R)mx;
    real<R>(G.mean_y)[c] = (R)my;
    real<R>(G.var_x)[c] = (R)(sxx * inv - mx * mx);
    real<R>(G.var_y)[c] = (R)(syy * inv - my * my);
    real<R>(G.cov_xy)[c] = (R)(sxy * inv - mx * my);
    G.mflag[c] = 1;
}

// ----------------------------------------------------------------------------------------------
// Pass 1: per-cell sums of the cells that hold particles.  Without evidence (launched by the
// assignment, since nothing in it depends on the measurement): the particle range of every
// occupied cell (Alg. 2), the sum of weights (Alg. 3) and the weighted velocity sums (Alg. 6).
// With evidence (launched by the update): the sums of w and of g w (Alg. 3, Alg. 4).
// ----------------------------------------------------------------------------------------------

template <bool kAssoc, typename R>
__global__ __launch_bounds__(kSegThreads) void k_seg_sums(Batch b)
{
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const MeasView M = meas_view(b.m[gi]);
    const uint32_t tile = xcd_tile(b, gi);
    const uint32_t wave = tile * (kSegThreads / kWave) + threadIdx.x / kWave;
    if (kAssoc) {
        seg_reduce<2, false, R>(
            G, wave,
            [&](uint32_t k, double w, double vx, double vy, double* v) {
                v[0] = (double)w;
                v[1] = likelihood((double)vx, (double)vy, (double)M.mu_vx[k],
                                  (double)M.mu_vy[k], (double)M.var_v[k]) * (double)w;
            },
            [&](uint32_t k, const double* v) {
                G.sum_w[k] = v[0];
                G.sum_wt[k] = v[1];
            });
    } else {
        seg_reduce<6, true, R>(
            G, wave,
            [&](uint32_t, double w, double vx, double vy, double* v) {
                const double wd = w, x = vx, y = vy;
                v[0] = wd;
                v[1] = wd * x;
                v[2] = wd * y;
                v[3] = wd * x * x;
                v[4] = wd * y * y;
                v[5] = wd * x * y;
            },
            [&](uint32_t k, const double* v) {
                // the cell's six sums leave as one contiguous record
                const uint32_t r = k * kCellSums;
                G.msum.store_vec<f64x2>(r, f64x2{v[0], v[1]});
                G.msum.store_vec<f64x2>(r + 2, f64x2{v[2], v[3]});
                G.msum.store_vec<f64x2>(r + 4, f64x2{v[4], v[5]});
            });
    }
}

// ----------------------------------------------------------------------------------------------
// Pass 2: every cell, one per thread: Alg. 3 + the normalisers of Alg. 4 (+ Alg. 6 without
// velocity evidence); each block also stores the fixed-point new-born mass of its cells.
// ----------------------------------------------------------------------------------------------

template <bool kAssoc, typename R>
__global__ __launch_bounds__(kCellThreads) void k_cells(Batch b)
{
    __shared__ uint64_t tmp[kCellThreads / kWave + 1];
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const MeasView M = meas_view(b.m[gi]);
    const uint32_t part = blockIdx.x - b.bstart[gi];
    const uint32_t c = part * kCellThreads + threadIdx.x;
    uint64_t q = 0;
    if (c < G.C) {
        const bool has = G.cend[c] != G.cstart[c];
        double s = 0.0, st = 0.0, m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (kAssoc) {
            if (has) {
                s = G.sum_w[c];
                st = G.sum_wt[c];
            } else {
                G.sum_w[c] = 0.0;
                G.sum_wt[c] = 0.0;
            }
        } else {
            // the record of the per-cell sums (written for cells with particles only)
            if (has) {
                const uint32_t r = c * kCellSums;
                const f64x2 a = G.msum.load_vec<f64x2>(r), b = G.msum.load_vec<f64x2>(r + 2),
                            d = G.msum.load_vec<f64x2>(r + 4);
                s = a[0];
                m[0] = a[1];
                m[1] = b[0];
                m[2] = b[1];
                m[3] = d[0];
                m[4] = d[1];
            }
            G.sum_w[c] = s;
        }
        R rb;
        const double rp = cell_update<R>(G, M, c, s, st, &rb);
        // moments of the updated weights mu_UA w, normalised by rho_p = mu_UA sum w; with
        // velocity evidence those of cells with particles come from their own pass
        if (!kAssoc)
            write_moments<R>(G, c, has && (R)rp > (R)0, s, m[0], m[1], m[2], m[3], m[4]);
        else if (!has)
            write_moments<R>(G, c, false, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0);
        q = fixed40(rb);
    }
    const uint64_t qsum = block_sum(q, tmp);
    if (threadIdx.x == 0) G.bpart[part] = qsum;
}

hipError_t launch_cell_sums(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [](const GridDev& G) {
        return xcd_blocks(ceil_div(G.nu, kSegBlockParticles));
    });
    if (blocks) {
        if (launch_real64(g, n))
            DOGM_LAUNCH_AS("k_seg_sums<false>", (k_seg_sums<false, double>),
                           dim3(blocks), dim3(kSegThreads), 0, s, b);
        else
            DOGM_LAUNCH_AS("k_seg_sums<false>", (k_seg_sums<false, float>),
                           dim3(blocks), dim3(kSegThreads), 0, s, b);
    }
    return hipGetLastError();
}

hipError_t launch_update(const GridRef* g, int n, hipStream_t s)
{
    bool any_assoc = false, all_assoc = true;
    for (int i = 0; i < n; ++i) {
        any_assoc |= g[i].m.p_assoc != nullptr;
        all_assoc &= g[i].m.p_assoc != nullptr;
    }
    if (any_assoc && !all_assoc) return hipErrorInvalidValue;  // one kind per launch
    const bool real64 = launch_real64(g, n);
    Batch b;
    uint32_t blocks = 0;
    if (any_assoc) {  // without evidence the assignment already formed the sums
        blocks = make_batch(b, g, n, [](const GridDev& G) {
            return xcd_blocks(ceil_div(G.nu, kSegBlockParticles));
        });
        if (blocks) {
            if (real64)
                DOGM_LAUNCH_AS("k_seg_sums<true>", (k_seg_sums<true, double>),
                               dim3(blocks), dim3(kSegThreads), 0, s, b);
            else
                DOGM_LAUNCH_AS("k_seg_sums<true>", (k_seg_sums<true, float>),
                               dim3(blocks), dim3(kSegThreads), 0, s, b);
        }
    }
    blocks = make_batch(b, g, n, [](const GridDev& G) { return G.n_cell_parts; });
    if (blocks) {
        const dim3 grid(blocks), block(kCellThreads);
        if (any_assoc && real64)
            DOGM_LAUNCH_AS("k_cells<true>", (k_cells<true, double>), grid, block,
                           0, s, b);
        else if (any_assoc)
            DOGM_LAUNCH_AS("k_cells<true>", (k_cells<true, float>), grid, block,
                           0, s, b);
        else if (real64)
            DOGM_LAUNCH_AS("k_cells<false>", (k_cells<false, double>), grid, block,
                           0, s, b);
        else
            DOGM_LAUNCH_AS("k_cells<false>", (k_cells<false, float>), grid, block,
                           0, s, b);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_born_offsets(g, n, s);
    if (e == hipSuccess) e = launch_particle_tiles(g, n, s);
    return e;
}

// ----------------------------------------------------------------------------------------------
// Alg. 6 with velocity evidence: moments of the updated weights, normalised by rho_p.
// ----------------------------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(kSegThreads) void k_seg_moments(Batch b)
{
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const uint32_t tile = xcd_tile(b, gi);
    const uint32_t wave = tile * (kSegThreads / kWave) + threadIdx.x / kWave;
    seg_reduce<5, false, R>(
        G, wave,
        [&](uint32_t, double w, double vx, double vy, double* v) {
            const double wd = w, x = vx, y = vy;
            v[0] = wd * x;
            v[1] = wd * y;
            v[2] = wd * x * x;
            v[3] = wd * y * y;
            v[4] = wd * x * y;
        },
        [&](uint32_t k, const double* v) {
            const double rp = (double)real<R>(G.rho_p)[k];
            write_moments<R>(G, k, rp > 0.0, rp, v[0], v[1], v[2], v[3], v[4]);
        });
}

hipError_t launch_moments(const GridRef* g, int n, hipStream_t s)
{
    // without velocity evidence the update already wrote the moments
    GridRef sub[kMaxBatch];
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (g[i].m.p_assoc != nullptr) sub[m++] = g[i];
    if (m == 0) return hipSuccess;
    Batch b;
    const uint32_t blocks = make_batch(b, sub, m, [](const GridDev& G) {
        return xcd_blocks(ceil_div(G.nu, kSegBlockParticles));
    });
    if (blocks)
        DOGM_LAUNCH_REAL(launch_real64(sub, m), "k_seg_moments", k_seg_moments, dim3(blocks),
                         dim3(kSegThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace dogm
