/*
 * Plain CPU oracle of the DS-PHD/MIB particle recursion (Nuss et al., "A Random Finite Set
 * Approach for Dynamic Occupancy Grid Maps with Real-Time Application", arXiv 1605.02406).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file:
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Everything is FP64 and single-threaded, with direct loops that follow the paper's
 * equations in the paper's order: per-cell sums are direct loops (never prefix
 * differences), the sort is a textbook stable counting sort, the resampling CDF is a
 * sequential sum and the draws are merged against it linearly.
 *
 * Readings of points the paper leaves open (each one is also listed in the design notes):
 *  - cell index  : origin at the grid corner, cell = iy*nx + ix with floor; particles
 *                  outside [0,nx*r) x [0,ny*r) get key C (past the last cell) and weight 0.
 *  - noise       : independent zero-mean Gaussians, sigma_pos on px,py and sigma_vel on
 *                  vx,vy per step (the process noise xi of eq. (process) is not specified).
 *  - random draws: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed, counter
 *                  (index, cycle, purpose, grid_id); uniform u = ((b>>9)+1/2)*2^-23 and the
 *                  Box-Muller transform for normals.
 *  - truncation  : m_p(O) = min(sum w, 1); weights are not rescaled; the unassociated
 *                  normaliser uses the raw sum (first form of eq. (DSnormalizationfactor2)).
 *  - Dempster    : normalised rule on Omega = {O,F}; a total conflict (1-K < 1e-12) keeps
 *                  the prediction and sets a status bit.
 *  - birth split : eq. (DS_resulting_masses1) with the predicted m_p(O); new-born mass only
 *                  where m_z(O) > 0, elsewhere rho_b = 0 and rho_p = m(O).
 *  - born slots  : allocation proportional to rho_b over an exact fixed-point prefix sum
 *                  (masses rounded to multiples of 2^-40), o_c = floor(nu_b*E_c/S) in FP64.
 *  - resampling  : systematic draws u_j = (j+U)*W/nu over an exact fixed-point CDF of the
 *                  joint [persistent | new-born] weights (rounded to multiples of 2^-40),
 *                  chosen index = first i with F_i > floor(u_j).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status bits (shared meaning with the library's status word, defined independently). */
#define OR_ST_CONFLICT 1u  /* Dempster total conflict in some cell                   */
#define OR_ST_NOCARRIER 2u /* a cell with rho_b > 0 received no new-born slot        */
#define OR_ST_NONFINITE 4u /* a non-finite value was met                              */

/* Philox purposes: the third counter word. */
#define OR_PURPOSE_INIT 0u
#define OR_PURPOSE_PREDICT 1u
#define OR_PURPOSE_BIRTH 2u
#define OR_PURPOSE_RESAMPLE 3u

typedef struct {
    int32_t nx, ny;
    double cell_size;       /* r                                   Table I          */
    double dt;              /* T                                   eq. (process)    */
    double p_s;             /* persistence probability             eq. (particle_persistence) */
    double p_b;             /* birth probability                   eq. (predicted_ex_born) */
    double sigma_pos;       /* process noise on position, per step                   */
    double sigma_vel;       /* process noise on velocity, per step                   */
    double sigma_birth_vel; /* SD of new-born velocity, Table I                      */
    double alpha_free;      /* free-mass discount alpha(T), eq. (DS_freespace_pred)  */
    int64_t n_pers;         /* nu                                                    */
    int64_t n_born;         /* nu_b                                                  */
    uint64_t seed;
    uint32_t grid_id;
} or_params;

/* ------------------------------------------------------------------------------------ */
/* Random numbers                                                                       */
/* ------------------------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds, from its published definition (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11): each round multiplies words 0
 * and 2 by the two Philox multipliers, swaps the high halves crosswise with words 1 and 3
 * xor the round key, and the key is bumped by the two Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Four 32-bit words for (index, cycle, purpose) of one grid. */
static void draw4(const or_params* p, uint32_t index, uint32_t cycle, uint32_t purpose,
                  uint32_t out[4])
{
    uint32_t ctr[4] = {index, cycle, purpose, p->grid_id};
    or_philox4x32_10(ctr, p->seed, out);
}

/* Uniform in (0,1): 23 high bits of the word plus one half, times 2^-23 (exact in FP32). */
double or_uniform(uint32_t b) { return ((double)(b >> 9) + 0.5) * 0x1p-23; }

/* Box-Muller transform (Box & Muller 1958): two uniforms -> two independent N(0,1). */
void or_box_muller(double u1, double u2, double* n1, double* n2)
{
    const double two_pi = 6.283185307179586476925286766559;
    double radius = sqrt(-2.0 * log(u1));
    *n1 = radius * cos(two_pi * u2);
    *n2 = radius * sin(two_pi * u2);
}

/* Standard normals used by the prediction of particle `index` in `cycle`: (n_px, n_py,
 * n_vx, n_vy).  Exposed so tests can inject or inspect the noise. */
void or_predict_noise(const or_params* p, uint32_t cycle, int64_t n, double* noise)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t b[4];
        draw4(p, (uint32_t)i, cycle, OR_PURPOSE_PREDICT, b);
        or_box_muller(or_uniform(b[0]), or_uniform(b[1]), &noise[4 * i + 0], &noise[4 * i + 1]);
        or_box_muller(or_uniform(b[2]), or_uniform(b[3]), &noise[4 * i + 2], &noise[4 * i + 3]);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Cell index (reading: grid-corner origin, row-major, out-of-grid -> C)                */
/* ------------------------------------------------------------------------------------ */

uint32_t or_cell_key_f64(const or_params* p, double x, double y)
{
    const uint32_t C = (uint32_t)p->nx * (uint32_t)p->ny;
    double fx = x / p->cell_size;
    double fy = y / p->cell_size;
    if (!(fx >= 0.0 && fx < (double)p->nx && fy >= 0.0 && fy < (double)p->ny)) return C;
    return (uint32_t)floor(fy) * (uint32_t)p->nx + (uint32_t)floor(fx);
}

/* The same decision taken in single precision on single-precision coordinates: the
 * predicted state is stored in FP32, so the cell it lies in is decided on those values
 * with one correctly rounded FP32 division per axis. */
uint32_t or_cell_key_f32(int32_t nx, int32_t ny, float cell_size, float x, float y)
{
    const uint32_t C = (uint32_t)nx * (uint32_t)ny;
    volatile float fx = x / cell_size;
    volatile float fy = y / cell_size;
    if (!(fx >= 0.0f && fx < (float)nx && fy >= 0.0f && fy < (float)ny)) return C;
    return (uint32_t)fy * (uint32_t)nx + (uint32_t)fx;
}

void or_cell_keys_f32(int32_t nx, int32_t ny, float cell_size, int64_t n, const float* x,
                      const float* y, uint32_t* key)
{
    for (int64_t i = 0; i < n; ++i) key[i] = or_cell_key_f32(nx, ny, cell_size, x[i], y[i]);
}

/* ------------------------------------------------------------------------------------ */
/* a1: particle prediction (eq. (process), eq. (particle_persistence), Alg. 1)          */
/* ------------------------------------------------------------------------------------ */

/* In place on (x, y, vx, vy, w).  `noise` holds 4 standard normals per particle; pass NULL
 * to draw them from Philox for (index, cycle, PREDICT).  Writes the cell key. */
void or_predict(const or_params* p, uint32_t cycle, int64_t n, double* x, double* y, double* vx,
                double* vy, double* w, const double* noise, uint32_t* key)
{
    const uint32_t C = (uint32_t)p->nx * (uint32_t)p->ny;
    for (int64_t i = 0; i < n; ++i) {
        double nz[4];
        if (noise) {
            nz[0] = noise[4 * i + 0];
            nz[1] = noise[4 * i + 1];
            nz[2] = noise[4 * i + 2];
            nz[3] = noise[4 * i + 3];
        } else {
            uint32_t b[4];
            draw4(p, (uint32_t)i, cycle, OR_PURPOSE_PREDICT, b);
            or_box_muller(or_uniform(b[0]), or_uniform(b[1]), &nz[0], &nz[1]);
            or_box_muller(or_uniform(b[2]), or_uniform(b[3]), &nz[2], &nz[3]);
        }
        /* constant-velocity transition: position advances with the old velocity */
        double xn = x[i] + p->dt * vx[i] + p->sigma_pos * nz[0];
        double yn = y[i] + p->dt * vy[i] + p->sigma_pos * nz[1];
        double vxn = vx[i] + p->sigma_vel * nz[2];
        double vyn = vy[i] + p->sigma_vel * nz[3];
        x[i] = xn;
        y[i] = yn;
        vx[i] = vxn;
        vy[i] = vyn;
        w[i] = p->p_s * w[i];
        key[i] = or_cell_key_f64(p, xn, yn);
        if (key[i] == C) w[i] = 0.0; /* outside the grid: the filter's support ends there */
    }
}

/* ------------------------------------------------------------------------------------ */
/* a2: assignment of particles to cells (Alg. 2)                                         */
/* ------------------------------------------------------------------------------------ */

/* Stable counting sort by key (keys in [0, C]; C = outside).  perm[s] = source index of
 * sorted position s.  cell_start/cell_end (exclusive) for every cell c < C; empty cells
 * get start == end.  Returns 0, or -1 if a key exceeds C. */
int or_assign(int64_t n, int64_t C, const uint32_t* key, int64_t* perm, uint32_t* cell_start,
              uint32_t* cell_end)
{
    int64_t* count = (int64_t*)calloc((size_t)(C + 2), sizeof(int64_t));
    if (!count) return -2;
    for (int64_t i = 0; i < n; ++i) {
        if ((int64_t)key[i] > C) {
            free(count);
            return -1;
        }
        count[key[i] + 1] += 1;
    }
    for (int64_t k = 1; k <= C + 1; ++k) count[k] += count[k - 1]; /* count[k] = first slot of key k */
    for (int64_t c = 0; c < C; ++c) {
        cell_start[c] = (uint32_t)count[c];
        cell_end[c] = (uint32_t)count[c + 1];
    }
    for (int64_t i = 0; i < n; ++i) perm[count[key[i]]++] = i; /* input order kept: stable */
    free(count);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* a3: cell occupancy prediction and update (eqs. (DS_particle_sum_pred),                */
/*     (DS_freespace_pred), (DS_comb), (DS_resulting_masses1/2), Alg. 3)                 */
/* ------------------------------------------------------------------------------------ */

/* Dempster's rule of combination on the frame {O, F}: focal sets O, F and Omega with
 * masses (o, f, 1-o-f).  Conflict K = o1*f2 + f1*o2.  Returns 1 on total conflict. */
int or_dempster(double o1, double f1, double o2, double f2, double* o, double* f)
{
    double u1 = 1.0 - o1 - f1;
    double u2 = 1.0 - o2 - f2;
    double K = o1 * f2 + f1 * o2;
    double norm = 1.0 - K;
    if (!(norm >= 1e-12)) {
        *o = o1;
        *f = f1;
        return 1;
    }
    *o = (o1 * o2 + o1 * u2 + u1 * o2) / norm;
    *f = (f1 * f2 + f1 * u2 + u1 * f2) / norm;
    return 0;
}

/* Per cell c (direct loops over the sorted particles of c):
 *   sum_w  = sum of predicted persistent weights
 *   m_pO   = min(sum_w, 1)                                     eq. (DS_particle_sum_pred)
 *   m_pF   = min(alpha * m_F_prev, 1 - m_pO)                   eq. (DS_freespace_pred)
 *   (m_O, m_F) = m_p (+) m_z                                   eq. (DS_comb)
 *   rho_b  = m_O p_B (1-m_pO) / (m_pO + p_B (1-m_pO)) if m_zO > 0, else 0
 *   rho_p  = m_O - rho_b                                       eq. (DS_resulting_masses1/2)
 *   pign   = m_O + (m_U)/2, the pignistic occupancy probability
 * Returns the status bits. */
uint32_t or_cell_update(const or_params* p, int64_t C, const double* w_sorted,
                        const uint32_t* cell_start, const uint32_t* cell_end,
                        const double* m_free_prev, const double* z_occ, const double* z_free,
                        double* sum_w, double* m_pO, double* m_pF, double* m_O, double* m_F,
                        double* rho_b, double* rho_p, double* pign)
{
    uint32_t status = 0;
    for (int64_t c = 0; c < C; ++c) {
        double s = 0.0;
        for (uint32_t k = cell_start[c]; k < cell_end[c]; ++k) s += w_sorted[k];
        double po = s < 1.0 ? s : 1.0;
        double pf_cand = p->alpha_free * m_free_prev[c];
        double pf = pf_cand < 1.0 - po ? pf_cand : 1.0 - po;
        double o, f;
        if (or_dempster(po, pf, z_occ[c], z_free[c], &o, &f)) status |= OR_ST_CONFLICT;
        double rb = 0.0;
        if (z_occ[c] > 0.0) {
            double a = p->p_b * (1.0 - po);
            double den = po + a;
            rb = den > 0.0 ? o * a / den : 0.0;
        }
        sum_w[c] = s;
        m_pO[c] = po;
        m_pF[c] = pf;
        m_O[c] = o;
        m_F[c] = f;
        rho_b[c] = rb;
        rho_p[c] = o - rb;
        pign[c] = o + 0.5 * (1.0 - o - f);
        if (!isfinite(o) || !isfinite(f) || !isfinite(s)) status |= OR_ST_NONFINITE;
    }
    return status;
}

/* The per-cell step of the particle PHD/MIB filter itself (Sec. V), without the Dempster-Shafer
 * approximation, for p_A = 0: a true positive then has the clutter density as its likelihood,
 * so every weight in the cell (persistent and new-born) is scaled by the same factor f.
 *   r_p   = min(sum w, 1)                      eq. (predExistenceProbParticles), truncated
 *   r_b   = p_B (1 - r_p)                      eq. (pred_birth_prob), in every cell
 *   r     = r_p + r_b                          predicted existence of the cell
 *   measurement (det = 1):  f = p_TP / (p_FP (1 - r) + p_TP r)
 *       eqs. (updateParticleWeightsUnnormalized), (applyNormalization), (normalizationCalculation)
 *   no measurement:         f = (1 - p_TP) / ((1 - p_TP) r + (1 - p_FP) (1 - r))
 *       eq. (updateParticleWeightsEmpty)
 *   rho_p = f r_p, rho_b = f r_b; the posterior occupancy f r, eq. (occupancyProbParticles)
 * Outputs share the Dempster-Shafer layout: m_pO = r_p, m_pF = 1 - r, m_O = pign = f r,
 * m_F = 1 - f r.  Returns the status bits. */
uint32_t or_cell_update_bayes(const or_params* p, int64_t C, const double* w_sorted,
                              const uint32_t* cell_start, const uint32_t* cell_end,
                              const double* p_tp, const double* p_fp, const double* det,
                              double* sum_w, double* m_pO, double* m_pF, double* m_O, double* m_F,
                              double* rho_b, double* rho_p, double* pign)
{
    uint32_t status = 0;
    for (int64_t c = 0; c < C; ++c) {
        double s = 0.0;
        for (uint32_t k = cell_start[c]; k < cell_end[c]; ++k) s += w_sorted[k];
        const double rp = s < 1.0 ? s : 1.0;
        const double rb = p->p_b * (1.0 - rp);
        const double r = rp + rb;
        double f;
        if (det[c] != 0.0)
            f = p_tp[c] / (p_fp[c] * (1.0 - r) + p_tp[c] * r);
        else
            f = (1.0 - p_tp[c]) / ((1.0 - p_tp[c]) * r + (1.0 - p_fp[c]) * (1.0 - r));
        sum_w[c] = s;
        m_pO[c] = rp;
        m_pF[c] = 1.0 - r;
        m_O[c] = f * r;
        m_F[c] = 1.0 - f * r;
        rho_b[c] = f * rb;
        rho_p[c] = f * rp;
        pign[c] = f * r;
        if (!isfinite(f) || !isfinite(s)) status |= OR_ST_NONFINITE;
    }
    return status;
}

/* ------------------------------------------------------------------------------------ */
/* a4: update of persistent particles (eqs. (DSupdateParticleWeightsUnnormalized) to     */
/*     (DSnormalizationfactor2), Alg. 4)                                                 */
/* ------------------------------------------------------------------------------------ */

/* Spatial likelihood of a particle velocity under the cell's measured velocity: an
 * isotropic Gaussian N(v; mu_z, var_z I) without its constant factor (the factor cancels
 * in mu_A * w~). */
double or_velocity_likelihood(double vx, double vy, double mux, double muy, double var)
{
    double dx = vx - mux, dy = vy - muy;
    return exp(-(dx * dx + dy * dy) / (2.0 * var));
}

/* In place on w_sorted; the particles of cell c are [cell_start[c], cell_end[c]) (particles
 * outside the grid belong to no cell and keep their weight 0).  With p_assoc == NULL the association probability is
 * 0 everywhere and g is never evaluated.  Outputs mu_A and mu_UA per cell.
 *   w~   = g * w                                                eq. (DSupdate...Unnormalized)
 *   mu_A = rho_p / sum w~ ,  mu_UA = rho_p / sum w               eqs. (DSnormalizationfactor(2))
 *   w'   = p_A mu_A w~ + (1-p_A) mu_UA w                         eq. (DSnormalization)
 * If sum w~ underflows to 0 the likelihood carries no information and w' = mu_UA w. */
void or_persistent_update(int64_t C, double* w_sorted, const double* vx, const double* vy, const uint32_t* cell_start,
                          const uint32_t* cell_end, const double* rho_p, const double* p_assoc,
                          const double* mu_vx, const double* mu_vy, const double* var_v,
                          double* mu_A, double* mu_UA)
{
    for (int64_t c = 0; c < C; ++c) {
        double s = 0.0, st = 0.0;
        for (uint32_t k = cell_start[c]; k < cell_end[c]; ++k) {
            s += w_sorted[k];
            if (p_assoc)
                st += or_velocity_likelihood(vx[k], vy[k], mu_vx[c], mu_vy[c], var_v[c]) *
                      w_sorted[k];
        }
        double mua = s > 0.0 ? rho_p[c] / s : 0.0;
        double ma = st > 0.0 ? rho_p[c] / st : 0.0;
        mu_UA[c] = mua;
        mu_A[c] = ma;
        double pa = p_assoc ? p_assoc[c] : 0.0;
        for (uint32_t k = cell_start[c]; k < cell_end[c]; ++k) {
            double w = w_sorted[k];
            if (p_assoc && st > 0.0) {
                double g = or_velocity_likelihood(vx[k], vy[k], mu_vx[c], mu_vy[c], var_v[c]);
                w_sorted[k] = pa * ma * (g * w) + (1.0 - pa) * mua * w;
            } else {
                w_sorted[k] = mua * w;
            }
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* a5: initialisation of new particles (eqs. (weights_associated), (weights_unassociated), */
/*     (assoc_relation), (assoc_sum), Alg. 5)                                            */
/* ------------------------------------------------------------------------------------ */

/* Mass in fixed point: multiples of 2^-40, rounded to nearest. */
uint64_t or_fixed40(double m) { return (uint64_t)floor(m * 0x1p40 + 0.5); }

/* Slot allocation proportional to rho_b: exact prefix E_c of the fixed-point masses,
 * o_c = floor(nu_b * E_c / S) evaluated in FP64, o_C = nu_b.  Where E_c = S (every cell
 * with new-born mass lies before c) the share is nu_b exactly, as the definition gives it;
 * the FP64 evaluation alone can land one below.  S == 0 gives no births (all offsets 0).
 * Returns S. */
uint64_t or_born_alloc(int64_t C, int64_t nb, const double* rho_b, uint32_t* off)
{
    uint64_t S = 0;
    for (int64_t c = 0; c < C; ++c) S += or_fixed40(rho_b[c]);
    if (S == 0) {
        for (int64_t c = 0; c <= C; ++c) off[c] = 0;
        return 0;
    }
    uint64_t E = 0;
    for (int64_t c = 0; c < C; ++c) {
        double o = floor((double)E * (double)nb / (double)S);
        if (o > (double)nb || E >= S) o = (double)nb;
        off[c] = (uint32_t)o;
        E += or_fixed40(rho_b[c]);
    }
    off[C] = (uint32_t)nb;
    return S;
}

/* Number of associated new-born particles of a cell: the nearest integer to p_A * n_c,
 * halves rounded up, so that nu_A : nu_UA follows p_A : (1 - p_A) and nu_A + nu_UA = n_c. */
int64_t or_num_assoc(double p_a, int64_t n_c) { return (int64_t)floor(p_a * (double)n_c + 0.5); }

/* Births for `cycle`.  Slot s lies in cell c with off[c] <= s < off[c+1]; the first nu_A
 * slots of a cell are associated (velocity from p(x|z) = N(mu_z, var_z I)), the rest are
 * unassociated (velocity from the birth pdf N(0, sigma_B^2 I)); position is uniform in
 * the cell.  Weights follow the two weight equations; an empty set passes its share to the
 * other.  `noise` (4 per slot: u_x, u_y, n_vx, n_vy) may be NULL (drawn from Philox for
 * (slot, cycle, BIRTH)).  Unused slots (S == 0) get weight 0 and key C.
 * Returns the status bits (no-carrier). */
uint32_t or_born_init(const or_params* p, uint32_t cycle, int64_t C, int64_t nb,
                      const uint32_t* off, const double* rho_b, const double* p_assoc,
                      const double* mu_vx, const double* mu_vy, const double* var_v,
                      const double* noise, double* bx, double* by, double* bvx, double* bvy,
                      double* bw, uint32_t* bkey, uint8_t* bassoc)
{
    uint32_t status = 0;
    for (int64_t c = 0; c < C; ++c)
        if (rho_b[c] > 0.0 && off[c + 1] == off[c] && off[C] > 0) status |= OR_ST_NOCARRIER;
    int64_t c = 0;
    for (int64_t s = 0; s < nb; ++s) {
        if (off[C] == 0) {
            bx[s] = by[s] = bvx[s] = bvy[s] = bw[s] = 0.0;
            bkey[s] = (uint32_t)C;
            bassoc[s] = 0;
            continue;
        }
        while (!(off[c] <= (uint32_t)s && (uint32_t)s < off[c + 1])) ++c;
        int64_t n_c = (int64_t)off[c + 1] - (int64_t)off[c];
        int64_t k = s - (int64_t)off[c];
        double pa = p_assoc ? p_assoc[c] : 0.0;
        int64_t na = or_num_assoc(pa, n_c);
        int64_t nua = n_c - na;
        int assoc = k < na;
        double w;
        if (assoc)
            w = (nua == 0) ? rho_b[c] / (double)na : pa * rho_b[c] / (double)na;
        else
            w = (na == 0) ? rho_b[c] / (double)nua : (1.0 - pa) * rho_b[c] / (double)nua;
        double u0, u1, n0, n1;
        if (noise) {
            u0 = noise[4 * s + 0];
            u1 = noise[4 * s + 1];
            n0 = noise[4 * s + 2];
            n1 = noise[4 * s + 3];
        } else {
            uint32_t b[4];
            draw4(p, (uint32_t)s, cycle, OR_PURPOSE_BIRTH, b);
            u0 = or_uniform(b[0]);
            u1 = or_uniform(b[1]);
            or_box_muller(or_uniform(b[2]), or_uniform(b[3]), &n0, &n1);
        }
        int64_t ix = c % p->nx, iy = c / p->nx;
        bx[s] = ((double)ix + u0) * p->cell_size;
        by[s] = ((double)iy + u1) * p->cell_size;
        if (assoc) {
            double sd = sqrt(var_v[c]);
            bvx[s] = mu_vx[c] + sd * n0;
            bvy[s] = mu_vy[c] + sd * n1;
        } else {
            bvx[s] = p->sigma_birth_vel * n0;
            bvy[s] = p->sigma_birth_vel * n1;
        }
        bw[s] = w;
        bkey[s] = (uint32_t)c;
        bassoc[s] = (uint8_t)assoc;
    }
    return status;
}

/* ------------------------------------------------------------------------------------ */
/* a6: statistical moments of grid cells (eqs. (mean_x), (var_x), (covar_xy), Alg. 6)   */
/* ------------------------------------------------------------------------------------ */

/* Per cell over its updated persistent particles, normalised by rho_p as printed:
 *   mean = (1/rho_p) sum w v ;  var = (1/rho_p) sum w v^2 - mean^2 ;
 *   cov  = (1/rho_p) sum w vx vy - mean_x mean_y.
 * Cells with rho_p <= 0 or no particles get zeros and flag 0 (no estimate), else flag 1. */
void or_moments(int64_t C, const double* w, const double* vx, const double* vy,
                const uint32_t* cell_start, const uint32_t* cell_end, const double* rho_p,
                double* mean_x, double* mean_y, double* var_x, double* var_y, double* cov_xy,
                uint8_t* flag)
{
    for (int64_t c = 0; c < C; ++c) {
        double sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
        for (uint32_t k = cell_start[c]; k < cell_end[c]; ++k) {
            sx += w[k] * vx[k];
            sy += w[k] * vy[k];
            sxx += w[k] * vx[k] * vx[k];
            syy += w[k] * vy[k] * vy[k];
            sxy += w[k] * vx[k] * vy[k];
        }
        if (!(rho_p[c] > 0.0) || cell_end[c] == cell_start[c]) {
            mean_x[c] = mean_y[c] = var_x[c] = var_y[c] = cov_xy[c] = 0.0;
            flag[c] = 0;
            continue;
        }
        double r = rho_p[c];
        double mx = sx / r, my = sy / r;
        mean_x[c] = mx;
        mean_y[c] = my;
        var_x[c] = sxx / r - mx * mx;
        var_y[c] = syy / r - my * my;
        cov_xy[c] = sxy / r - mx * my;
        flag[c] = 1;
    }
}

/* ------------------------------------------------------------------------------------ */
/* a7: resampling (eq. (resampledParticleWeights), Alg. 7)                               */
/* ------------------------------------------------------------------------------------ */

/* The uniform offset U of the systematic draws of `cycle`. */
double or_resample_offset(const or_params* p, uint32_t cycle)
{
    uint32_t b[4];
    draw4(p, 0u, cycle, OR_PURPOSE_RESAMPLE, b);
    return or_uniform(b[0]);
}

/* Joint set J = [persistent (nu, sorted order) | new-born (nb, slot order)].  Writes the
 * nu chosen source indices into idx (index into J) and returns the fixed-point total W
 * (multiples of 2^-40) through *W_fixed.  Every resampled particle gets weight W/nu.
 * With W == 0 the persistent set is kept as it is: idx[j] = j.
 *   F_i = sum_{i' <= i} q_i'      q_i = round(w_i 2^40)
 *   d   = W / nu                  (the draw spacing, rounded once to FP64)
 *   t_j = floor((j + U) d)        (FP64)
 *   idx_j = min { i : F_i > t_j } (last positive-weight index if none) */
void or_resample_indices(int64_t nu, int64_t nb, const double* w_pers, const double* w_born,
                         double U, int64_t* idx, uint64_t* W_fixed)
{
    int64_t N = nu + nb;
    uint64_t* F = (uint64_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(uint64_t));
    uint64_t acc = 0;
    int64_t last_pos = -1;
    for (int64_t i = 0; i < N; ++i) {
        double wi = i < nu ? w_pers[i] : w_born[i - nu];
        uint64_t q = or_fixed40(wi > 0.0 ? wi : 0.0);
        acc += q;
        F[i] = acc;
        if (q > 0) last_pos = i;
    }
    *W_fixed = acc;
    if (acc == 0) {
        for (int64_t j = 0; j < nu; ++j) idx[j] = j;
        free(F);
        return;
    }
    double spacing = (double)acc / (double)nu;
    int64_t i = 0;
    for (int64_t j = 0; j < nu; ++j) {
        double u = ((double)j + U) * spacing;
        uint64_t t = (uint64_t)floor(u);
        while (i < N && F[i] <= t) ++i;
        idx[j] = i < N ? i : last_pos;
    }
    free(F);
}

/* Weight of every resampled particle: W / nu, evaluated in FP64. */
double or_resample_weight(uint64_t W_fixed, int64_t nu)
{
    return (double)W_fixed * 0x1p-40 / (double)nu;
}

/* ------------------------------------------------------------------------------------ */
/* Initial state (reading: the paper is silent)                                          */
/* ------------------------------------------------------------------------------------ */

/* nu particles uniform over the grid with velocity N(0, sigma_B^2 I) and weight 0. */
void or_init_state(const or_params* p, int64_t n, double* x, double* y, double* vx, double* vy,
                   double* w)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t b[4];
        draw4(p, (uint32_t)i, 0u, OR_PURPOSE_INIT, b);
        double n0, n1;
        or_box_muller(or_uniform(b[2]), or_uniform(b[3]), &n0, &n1);
        x[i] = or_uniform(b[0]) * (double)p->nx * p->cell_size;
        y[i] = or_uniform(b[1]) * (double)p->ny * p->cell_size;
        vx[i] = p->sigma_birth_vel * n0;
        vy[i] = p->sigma_birth_vel * n1;
        w[i] = 0.0;
    }
}
