// Element-wise kernels: descriptor upload, initial state, prediction (Alg. 1) with the digit
// histogram of the sort's first pass, the new-born slot allocation and initialisation of
// Alg. 5 and the last loop of Alg. 4 (weight normalisation).
#include "launch.h"

namespace dogm {

__global__ void k_write_desc(GridDev hd, GridDev* dd) { *dd = hd; }

hipError_t launch_write_desc(const GridDev& hd, GridDev* dd, hipStream_t s)
{
    DOGM_LAUNCH(k_write_desc, dim3(1), dim3(1), 0, s, hd, dd);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Initial state: particles uniform over the grid, velocity N(0, sigma_B^2), weight 0; m_F = 0.
// ----------------------------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(kElemThreads) void k_init(Batch b)
{
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const uint32_t i = (blockIdx.x - b.bstart[gi]) * kElemThreads + threadIdx.x;
    if (i < G.nu) {
        const uint4 r = draw(G, i, 0u, kPurposeInit);
        R n0, n1;
        box_muller<R>((R)unit_f32(r.z), (R)unit_f32(r.w), n0, n1);
        real<R>(G.x)[i] = (R)unit_f32(r.x) * (R)G.nx * (R)G.r;
        real<R>(G.y)[i] = (R)unit_f32(r.y) * (R)G.ny * (R)G.r;
        real<R>(G.vx)[i] = (R)G.sig_birth * n0;
        real<R>(G.vy)[i] = (R)G.sig_birth * n1;
        real<R>(G.w)[i] = (R)0;
    }
    if (i < G.C) real<R>(G.m_F)[i] = (R)0;
    if (i == 0) {
        *G.cycle = 1u;
        *G.cycle_run = 1u;
        *G.status = 0u;
        *G.nc_flag = 0u;
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
    if (blocks)
        DOGM_LAUNCH_REAL(launch_real64(g, n), "k_init", k_init, dim3(blocks), dim3(kElemThreads),
                         0, s, b);
    return hipGetLastError();
}

__global__ void k_set_cycle(Batch b, uint32_t cycle)
{
    if (threadIdx.x == 0) {
        *b.g[blockIdx.x]->cycle = cycle;
        *b.g[blockIdx.x]->cycle_run = cycle;
    }
}

hipError_t launch_set_cycle(const GridRef* g, int n, uint32_t cycle, hipStream_t s)
{
    Batch b;
    make_batch(b, g, n, [](const GridDev&) { return 1u; });
    DOGM_LAUNCH(k_set_cycle, dim3(n), dim3(64), 0, s, b, cycle);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Alg. 1: constant-velocity prediction with Philox noise, persistence, cell key.  One block per
// sort tile (kHistTile particles): it also stores the tile's digit histogram for the sort's first
// pass.  The blocks
// also clear what later kernels fill in sparsely (cell ranges, first-slot marks) and record the
// cycle being run.
// ----------------------------------------------------------------------------------------------

constexpr int kPredItems = kHistTile / kHistThreads;  // 4

template <typename R>
__global__ __launch_bounds__(kHistThreads) void k_predict(Batch b)
{
    __shared__ uint32_t cnt[kSortBins];
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const uint32_t tile = xcd_tile(b, gi);
    if (tile >= G.n_hist_tiles) return;
    const uint32_t cycle = *G.cycle;
    const uint32_t shift = G.dshift[0], bits = G.dbits[0], nbins = 1u << bits;
    const auto X = real<R>(G.x), Y = real<R>(G.y), VX = real<R>(G.vx), VY = real<R>(G.vy);
    const auto Wt = real<R>(G.w);

    const uint32_t nthreads = G.n_hist_tiles * kHistThreads;
    const uint32_t tid = tile * kHistThreads + threadIdx.x;
    for (uint32_t c = tid; c < G.C; c += nthreads) {
        G.cstart[c] = 0;
        G.cend[c] = 0;
    }
    for (uint32_t s = tid; s < G.nb; s += nthreads) G.born_mark[s] = kNoCell;
    if (tid == 0) *G.cycle_run = cycle;

    for (uint32_t d = threadIdx.x; d < nbins; d += kHistThreads) cnt[d] = 0;
    __syncthreads();

    R x[kPredItems], y[kPredItems], vx[kPredItems], vy[kPredItems], w[kPredItems];
#pragma unroll
    for (int it = 0; it < kPredItems; ++it) {
        const uint32_t i = tile * kHistTile + it * kHistThreads + threadIdx.x;
        const bool valid = i < G.nu;
        x[it] = valid ? X[i] : (R)0;
        y[it] = valid ? Y[i] : (R)0;
        vx[it] = valid ? VX[i] : (R)0;
        vy[it] = valid ? VY[i] : (R)0;
        w[it] = valid ? Wt[i] : (R)0;
    }
#pragma unroll
    for (int it = 0; it < kPredItems; ++it) {
        const uint32_t i = tile * kHistTile + it * kHistThreads + threadIdx.x;
        const bool valid = i < G.nu;
        uint32_t k = 0;
        if (valid) {
            const uint4 r = draw(G, i, cycle, kPurposePredict);
            R n0, n1, n2, n3;
            box_muller<R>((R)unit_f32(r.x), (R)unit_f32(r.y), n0, n1);
            box_muller<R>((R)unit_f32(r.z), (R)unit_f32(r.w), n2, n3);
            const R xn = x[it] + (R)G.dt * vx[it] + (R)G.sig_pos * n0;
            const R yn = y[it] + (R)G.dt * vy[it] + (R)G.sig_pos * n1;
            const R vxn = vx[it] + (R)G.sig_vel * n2;
            const R vyn = vy[it] + (R)G.sig_vel * n3;
            k = cell_of<R>(G, xn, yn);
            X[i] = xn;
            Y[i] = yn;
            VX[i] = vxn;
            VY[i] = vyn;
            Wt[i] = (k == G.C) ? (R)0 : (R)G.p_s * w[it];
            G.key[i] = k;
        }
        digit_count(valid, (k >> shift) & (nbins - 1u), cnt);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nbins; d += kHistThreads)
        G.hist[d * G.n_hist_tiles + tile] = cnt[d];
}

hipError_t launch_predict(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return xcd_blocks(G.n_hist_tiles); });
    if (blocks)
        DOGM_LAUNCH_REAL(launch_real64(g, n), "k_predict", k_predict, dim3(blocks),
                         dim3(kHistThreads), 0, s, b);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// Alg. 5: slot allocation from the exact prefix E_c of the fixed-point new-born masses; each cell
// that receives slots marks its first slot with its id and names itself as the first cell of
// every new-born tile that starts inside its slot range.
// ----------------------------------------------------------------------------------------------

__device__ __forceinline__ uint32_t ceil_div_dev(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// o_c = floor(nu_b E_c / S) in FP64 with every operation rounded separately (no contraction).
// Where all the new-born mass lies before the cell (E_c = S) the share is exactly nu_b: the
// rounded product fl(S nu_b) / S may fall just below it, which would leave the last slot
// without a cell that holds mass.
__device__ __forceinline__ uint32_t slot_offset(uint64_t E, uint64_t S, uint32_t nb)
{
    if (E >= S) return nb;
    const double t = __ddiv_rn(__dmul_rn((double)E, (double)nb), (double)S);
    const double o = floor(t);
    return o > (double)nb ? nb : (uint32_t)o;
}

// Exclusive prefix sums, in place, of a grid's fixed-point partial sums: the new-born masses
// per block of cells (which = 0; total S) or the joint weights per resampling tile (which = 1;
// total W), the total also in the extra last entry and in the grid's device scalar.  One block
// per grid, so every block that consumes the partials reads one word instead of adding up all
// the partials before its own (launched for grids with many partials only).
constexpr int kScanPartThreads = 1024;
constexpr int kScanPartItems = 4;

__global__ __launch_bounds__(kScanPartThreads) void k_scan_parts(Batch b, int which)
{
    __shared__ uint64_t tmp[kScanPartThreads / kWave + 1];
    const GridView G = grid_view(b.g[blockIdx.x]);
    const GArr<uint64_t> a = which == 0 ? G.bpart : G.rpart;
    const uint32_t n = which == 0 ? G.n_cell_parts : G.n_res_ptiles + G.n_born_parts;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < n; base += kScanPartThreads * kScanPartItems) {
        const uint32_t t0 = base + threadIdx.x * kScanPartItems;
        uint64_t v[kScanPartItems], acc = 0;
#pragma unroll
        for (int j = 0; j < kScanPartItems; ++j) {
            v[j] = t0 + j < n ? a[t0 + j] : 0;
            acc += v[j];
        }
        uint64_t total;
        uint64_t run = carry + block_excl_scan(acc, tmp, &total);
#pragma unroll
        for (int j = 0; j < kScanPartItems; ++j) {
            if (t0 + j < n) a[t0 + j] = run;
            run += v[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        a[n] = carry;
        if (which == 0) *G.S_fixed = carry;
        else *G.W_fixed = carry;
    }
}

hipError_t launch_scan_parts(const GridRef* g, int n, int which, bool* prefixed, hipStream_t s)
{
    bool scan = false;
    for (int i = 0; i < n; ++i) {
        const GridDev& G = *g[i].hd;
        const uint32_t parts = which == 0 ? G.n_cell_parts : G.n_res_ptiles + G.n_born_parts;
        scan |= G.scan_parts == 1 || (G.scan_parts == 0 && parts > kScanPartsFrom);
    }
    *prefixed = scan;
    if (!*prefixed) return hipSuccess;
    Batch b;
    const uint32_t blocks = make_batch(b, g, n, [](const GridDev&) { return 1u; });
    if (blocks) DOGM_LAUNCH(k_scan_parts, dim3(blocks), dim3(kScanPartThreads), 0, s, b, which);
    return hipGetLastError();
}

template <typename R>
__global__ __launch_bounds__(kCellThreads) void k_born_offsets(Batch b, int prefixed)
{
    __shared__ uint64_t tmp[kCellThreads / kWave + 1];
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const uint32_t part = blockIdx.x - b.bstart[gi];
    const uint32_t c = part * kCellThreads + threadIdx.x;
    const R rb = (c < G.C) ? real<R>(G.rho_b)[c] : (R)0;
    // new-born mass of the cell blocks before this one, and in total
    uint64_t before, Stot;
    if (prefixed) {
        before = G.bpart[part];
        Stot = *G.S_fixed;
    } else {
        partials_before(G.bpart, G.n_cell_parts, part, &before, &Stot);
        if (part == 0 && threadIdx.x == 0) *G.S_fixed = Stot;
    }
    const uint64_t q = fixed40(rb);
    uint64_t total;
    const uint64_t E = before + block_excl_scan(q, tmp, &total);
    // lanes past the last offset stay in the wave: the wave-wide tile fill below needs them
    const bool valid = c <= G.C;
    uint32_t o = 0;
    if (Stot != 0) o = (c == G.C) ? G.nb : slot_offset(E, Stot, G.nb);
    if (valid) G.born_off[c] = o;
    bool no_carrier = false;
    // new-born tiles [t_lo, t_hi) start inside this cell's slots [o, o1)
    uint32_t t_lo = 0, t_hi = 0;
    if (c < G.C && Stot != 0 && G.nb > 0 && q != 0) {
        const uint32_t o1 = (c + 1 == G.C) ? G.nb : slot_offset(E + q, Stot, G.nb);
        if (o1 > o) {
            G.born_mark[o] = c;
            t_lo = ceil_div_dev(o, kBornTile);
            t_hi = ceil_div_dev(o1, kBornTile);
        } else {
            no_carrier = true;
        }
    }
    // A cell may hold all nb slots (nb / kBornTile tiles): a lane fills a short run of tiles
    // itself and hands a long one to the whole wave.
    constexpr uint32_t kLaneTiles = 4;
    const bool wide = t_hi - t_lo > kLaneTiles;
    if (!wide)
        for (uint32_t t = t_lo; t < t_hi; ++t) G.tile_first[t] = c;
    for (uint64_t wl = __ballot(wide); wl != 0; wl &= wl - 1) {
        const int l = __ffsll((unsigned long long)wl) - 1;
        const uint32_t lo = __shfl(t_lo, l, kWave), hi = __shfl(t_hi, l, kWave);
        const uint32_t cl = __shfl(c, l, kWave);
        for (uint32_t t = lo + (uint32_t)lane_id(); t < hi; t += kWave) G.tile_first[t] = cl;
    }
    // With births in every cell most waves may hold a cell without a slot.  Device-scope atomics
    // on one word serialise across the whole chip (about 12 ns each), so such waves store the
    // same constant into a flag word instead; the next launch folds it into the status.
    const uint64_t nc = __ballot(no_carrier);
    if (nc != 0 && lane_id() == __ffsll((unsigned long long)nc) - 1) *G.nc_flag = kStNoCarrier;
}

hipError_t launch_born_offsets(const GridRef* g, int n, hipStream_t s)
{
    bool prefixed = false;
    if (const hipError_t e = launch_scan_parts(g, n, 0, &prefixed, s); e != hipSuccess) return e;
    Batch b;
    const uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) { return ceil_div(G.C + 1, kCellThreads); });
    if (blocks)
        DOGM_LAUNCH_REAL(launch_real64(g, n), "k_born_offsets", k_born_offsets, dim3(blocks),
                         dim3(kCellThreads), 0, s, b, prefixed ? 1 : 0);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------------------
// One launch, two kinds of blocks: persistent blocks of kPtSplit resampling tiles normalise the
// sorted weights (Alg. 4, last loop: w <- p_A mu_A g w + (1 - p_A) mu_UA w), new-born tiles of
// kBornTile slots initialise their slots (Alg. 5); both store the fixed-point weight sum of each
// resampling tile.
// ----------------------------------------------------------------------------------------------

__device__ __forceinline__ double likelihood(double vx, double vy, double mx, double my,
                                             double var)
{
    const double dx = vx - mx, dy = vy - my;
    return exp(-(dx * dx + dy * dy) / (2.0 * var));
}

// Initialises new-born slot s of cell c (born_off[c] <= s < born_off[c+1]); returns its weight.
template <typename R>
__device__ __forceinline__ R init_born(const GridView& G, const MeasView& M, uint32_t s,
                                      uint32_t c, uint32_t cycle)
{
    const uint32_t o0 = G.born_off[c], o1 = G.born_off[c + 1];
    const uint32_t n_c = o1 - o0;
    const double pa = M.p_assoc ? (double)M.p_assoc[c] : 0.0;
    const uint32_t na = (uint32_t)floor(mul_add_twice_rounded(pa, (double)n_c, 0.5));
    const uint32_t nua = n_c - na;
    const bool assoc = (s - o0) < na;
    const double rb = (double)real<R>(G.rho_b)[c];
    double w;
    if (assoc) w = (nua == 0) ? rb / (double)na : pa * rb / (double)na;
    else w = (na == 0) ? rb / (double)nua : (1.0 - pa) * rb / (double)nua;
    const uint4 r = draw(G, s, cycle, kPurposeBirth);
    R n0, n1;
    box_muller<R>((R)unit_f32(r.z), (R)unit_f32(r.w), n0, n1);
    const uint32_t ix = c % (uint32_t)G.nx, iy = c / (uint32_t)G.nx;
    real<R>(G.bx)[s] = ((R)ix + (R)unit_f32(r.x)) * (R)G.r;
    real<R>(G.by)[s] = ((R)iy + (R)unit_f32(r.y)) * (R)G.r;
    if (assoc) {
        const R sd = sqrt((R)M.var_v[c]);
        real<R>(G.bvx)[s] = (R)M.mu_vx[c] + sd * n0;
        real<R>(G.bvy)[s] = (R)M.mu_vy[c] + sd * n1;
    } else {
        real<R>(G.bvx)[s] = (R)G.sig_birth * n0;
        real<R>(G.bvy)[s] = (R)G.sig_birth * n1;
    }
    const R wr = (R)w;
    real<R>(G.bw)[s] = wr;
    G.bkey[s] = c;
    G.bassoc[s] = assoc ? 1 : 0;
    return wr;
}

template <typename R>
__global__ __launch_bounds__(kResThreads) void k_particle_tiles(Batch b)
{
    __shared__ uint64_t tmp[kResThreads / kWave + 1];
    __shared__ uint32_t wave_last[kResThreads / kWave];
    const int gi = batch_grid(b);
    const GridView G = grid_view(b.g[gi]);
    const MeasView M = meas_view(b.m[gi]);
    const uint32_t tile = blockIdx.x - b.bstart[gi];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t pblocks = ceil_div_u32(G.n_res_ptiles, kPtSplit);
    if (tile == 0 && threadIdx.x == 0 && *G.nc_flag != 0u) status_or(G, kStNoCarrier);
    uint64_t q = 0;
    if (tile < pblocks) {
        // kPtSplit resampling tiles; items [h * kResItems, (h + 1) * kResItems) lie in tile h
        const auto SW = real<R>(G.sw);
        uint64_t qh[kPtSplit] = {};
        uint32_t k[kPtItems];
        R w[kPtItems];
#pragma unroll
        for (int it = 0; it < kPtItems; ++it) {
            const uint32_t i = tile * kPtTile + it * kResThreads + threadIdx.x;
            k[it] = i < G.nu ? G.skey[i] : kNoCell;
            w[it] = i < G.nu ? SW[i] : (R)0;
        }
        const bool assoc = static_cast<bool>(M.p_assoc);
#pragma unroll
        for (int it = 0; it < kPtItems; ++it) {
            const uint32_t i = tile * kPtTile + it * kResThreads + threadIdx.x;
            if (k[it] >= G.C) continue;  // idle lane, or outside the grid (weight 0 already)
            const double wd = (double)w[it];
            double wn;
            if (assoc && G.sum_wt[k[it]] > 0.0) {
                const uint32_t c = k[it];
                const double pa = (double)M.p_assoc[c];
                const double g = likelihood((double)real<R>(G.svx)[i], (double)real<R>(G.svy)[i],
                                            (double)M.mu_vx[c], (double)M.mu_vy[c],
                                            (double)M.var_v[c]);
                wn = pa * G.mu_A[c] * (g * wd) + (1.0 - pa) * G.mu_UA[c] * wd;
            } else {
                wn = G.mu_UA[k[it]] * wd;
            }
            const R wr = (R)wn;
            SW[i] = wr;
            qh[it / kResItems] += fixed40(wr);
        }
#pragma unroll
        for (int h = 0; h < kPtSplit; ++h) {
            const uint64_t qsum = block_sum(qh[h], tmp);
            const uint32_t t = tile * kPtSplit + h;
            if (threadIdx.x == 0 && t < G.n_res_ptiles) G.rpart[t] = qsum;
        }
    } else {
        // new-born slots, one per thread: the cell of a slot is the last mark at or before it,
        // or the tile's first cell if there is none (cells are numbered in slot order)
        const uint32_t bt = tile - pblocks;
        const uint32_t s = bt * kBornTile + threadIdx.x;
        const uint64_t Stot = *G.S_fixed;
        const uint32_t cycle = *G.cycle_run;
        const uint32_t first = G.tile_first[bt];
        const uint32_t mk = (s < G.nb) ? G.born_mark[s] : kNoCell;
        uint32_t m = (mk == kNoCell) ? 0u : mk + 1u;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = __shfl_up(m, off, kWave);
            if (lane >= off) m = o > m ? o : m;
        }
        if (lane == kWave - 1) wave_last[wave] = m;
        __syncthreads();
        for (int w2 = 0; w2 < wave; ++w2) m = wave_last[w2] > m ? wave_last[w2] : m;
        if (s < G.nb) {
            if (Stot == 0) {  // no new-born mass anywhere: empty slots
                real<R>(G.bx)[s] = real<R>(G.by)[s] = (R)0;
                real<R>(G.bvx)[s] = real<R>(G.bvy)[s] = real<R>(G.bw)[s] = (R)0;
                G.bkey[s] = G.C;
                G.bassoc[s] = 0;
            } else {
                const uint32_t c = (m != 0u && m - 1u > first) ? m - 1u : first;
                q = fixed40(init_born<R>(G, M, s, c, cycle));
            }
        }
        const uint64_t qsum = block_sum(q, tmp);
        if (threadIdx.x == 0) G.rpart[G.n_res_ptiles + bt] = qsum;
    }
}

hipError_t launch_particle_tiles(const GridRef* g, int n, hipStream_t s)
{
    Batch b;
    const uint32_t blocks =
        make_batch(b, g, n, [](const GridDev& G) {
            return ceil_div(G.n_res_ptiles, kPtSplit) + G.n_born_parts;
        });
    if (blocks)
        DOGM_LAUNCH_REAL(launch_real64(g, n), "k_particle_tiles", k_particle_tiles,
                         dim3(blocks), dim3(kResThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace dogm
