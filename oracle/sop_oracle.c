/*
 * FP64 CPU oracle for overdamped Langevin dynamics of the Self Organized
 * Polymer (SOP) model -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg call
 * this code.  It shares nothing with the HIP library: no headers, no helpers,
 * no tables.  Everything is single-threaded except the residue-parallel
 * forms at the end (OpenMP over residues, the same arithmetic summed in
 * another order), which exist so that systems of 10^5 residues can be
 * followed for 10^4 steps.  It is written to be read against the paper (Zhmurov, Dima,
 * Kholodov, Barsegov, "Langevin dynamics simulations of biomolecules on
 * graphics processors", arXiv:1003.1148), not to be fast.
 *
 * What it computes, in the paper's order:
 *   - potential: Eq. 1 (FENE backbone bonds, native 12-6 contacts, soft
 *     repulsion (sigma/r)^6 for every other pair, including i,i+2);
 *   - pairwise forces: the CPU pair loop of Algorithm 1 (each pair once,
 *     +df on i and -df on j);
 *   - Verlet list: Algorithm 3's filter "r < cutoff" applied to every
 *     candidate pair of the same trajectory that is neither bonded nor
 *     native;
 *   - random force: Section III.C, Box-Muller on uniforms from a
 *     counter-based Philox4x32-10 stream (Salmon, Moraes, Dror, Shaw,
 *     SC'11) instead of the paper's Hybrid Taus;
 *   - update: the first-order Ermak-McCammon scheme of Eq. 2 / Algorithm 7,
 *     r <- r + f h/xi + g sqrt(2 kB T h/xi), every force taken at r(t_n).
 *
 * Readings of the paper that this code takes, each with its reason:
 *   - Eq. 2 prints f*xi*h; Algorithm 7 prints f*h/xi.  h/xi is taken (it is
 *     the dimensionally consistent form).
 *   - The third sum of Eq. 1 is garbled; it is read as the i,i+2 repulsion
 *     with sigma = 3.8 A, i.e. those pairs are ordinary repulsive pairs.
 *   - Every non-bonded, non-native pair of a trajectory is repulsive
 *     (Table I's counts: non-native pairs = N(N-1)/2 - bonds - natives).
 *   - The list predicate is taken in single precision, the precision of the
 *     paper's GPU code: with xf = (float)x, d2 = fl(fl(fl(dx*dx) + fl(dy*dy))
 *     + fl(dz*dz)), dx = fl(xf_i - xf_j), in the list iff d2 < (float)rc^2.
 *   - No per-step cutoff: every listed pair contributes until the next
 *     rebuild (Algorithm 2 has no distance test).
 *   - Uniforms: u = ((w >> 9) + 0.5) * 2^-23 for each 32-bit Philox word w,
 *     exact in FP32 and FP64; g_x, g_y = sqrt(-2 ln u0) (cos, sin)(2 pi u1),
 *     g_z = sqrt(-2 ln u2) cos(2 pi u3) (four uniforms, three Gaussians, as
 *     the paper's 4N numbers for 3N Gaussians).
 *   - Philox key = (seed low word, seed high word), counter = (residue index
 *     inside its trajectory, trajectory stream id, step low word, step high
 *     word).
 *   - FENE stretch |r - r0| >= R0 is an error, not clamped.
 *   - External terms (not in Eq. 1; they carry the pulling and indentation
 *     protocols of Section IV.B): a harmonic cantilever
 *     (kappa/2)|A(t) - r_c|^2 with A(t) = A0 + v t, and a spherical tip of
 *     radius R_t whose surface repels every residue with eps_t (sigma_t/s)^6,
 *     s = |r - T(t)| - R_t, T(t) = T0 + v_t t, t = n h.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_FENE (-5)
#define ORC_E_OVERFLOW (-6)
#define ORC_E_NONFINITE (-7)
#define ORC_E_TIP (-8)

#define ORC_NTERMS 5 /* FENE, native, repulsive, external, virial */

typedef struct {
    double k_fene, R0, eps_h, eps_l, sigma, r_list, kBT, zeta, h;
    int32_t list_every;
    int32_t pad;
    uint64_t seed;
} orc_params;

typedef struct {
    int64_t n_res, n_traj;
    const int64_t *res_offsets; /* n_traj+1 */
    const uint32_t *stream_ids; /* n_traj */
    int64_t n_bonds;
    const int32_t *bonds; /* 2*n_bonds */
    const double *bond_r0;
    int64_t n_native;
    const int32_t *natives; /* 2*n_native */
    const double *native_r0;
    const uint8_t *fixed; /* n_res or NULL */
    int32_t n_pull;
    int32_t has_tip;
    const int32_t *pull_traj; /* n_pull */
    const int32_t *pull_res;
    const double *pull_kappa;
    const double *pull_anchor0; /* 3*n_pull */
    const double *pull_v;       /* 3*n_pull */
    double tip_radius, tip_eps, tip_sigma;
    double tip_c0[3], tip_v[3];
} orc_system;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit    */
/* multiplications and xors; the key is bumped by the Weyl constants         */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
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

/* A uniform in (0,1) from the top 23 bits of a word: exact in FP32. */
double orc_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Section III.C: three standard Gaussians for one residue at one step. */
void orc_gauss3(uint64_t seed, uint32_t local, uint32_t stream, int64_t step, double g[3])
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint64_t n = (uint64_t)step;
    uint32_t ctr[4] = {local, stream, (uint32_t)n, (uint32_t)(n >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u0 = orc_uniform(w[0]), u1 = orc_uniform(w[1]);
    double u2 = orc_uniform(w[2]), u3 = orc_uniform(w[3]);
    double a = sqrt(-2.0 * log(u0));
    double b = sqrt(-2.0 * log(u2));
    g[0] = a * cos(two_pi * u1);
    g[1] = a * sin(two_pi * u1);
    g[2] = b * cos(two_pi * u3);
}

/* ------------------------------------------------------------------------ */
/* Eq. 1 pair terms.  Each returns the energy and stores dE/dr.              */
/* ------------------------------------------------------------------------ */

/* FENE: -(k R0^2 / 2) ln(1 - (r - r0)^2 / R0^2).  Sets *broken when
 * |r - r0| >= R0, where the logarithm has no real value. */
double orc_fene(double r, double r0, double k, double R0, double *dEdr, int *broken)
{
    double d = r - r0;
    double x = 1.0 - (d * d) / (R0 * R0);
    if (!(x > 0.0)) {
        *broken = 1;
        *dEdr = 0.0;
        return 0.0;
    }
    *dEdr = k * d / x;
    return -0.5 * k * R0 * R0 * log(x);
}

/* Native contact: eps [ (r0/r)^12 - 2 (r0/r)^6 ]. */
double orc_native(double r, double r0, double eps, double *dEdr)
{
    double q = pow(r0 / r, 6.0);
    *dEdr = 12.0 * eps * (q - q * q) / r;
    return eps * (q * q - 2.0 * q);
}

/* Soft repulsion: eps (sigma/r)^6. */
double orc_repulsive(double r, double sigma, double eps, double *dEdr)
{
    double q = pow(sigma / r, 6.0);
    *dEdr = -6.0 * eps * q / r;
    return eps * q;
}

/* Second derivatives d^2E/dr^2 of the three pair terms (the derivatives of
 * the dE/dr above): they set how much a pair's force moves when its distance
 * is perturbed, which is what rounding the distance does. */
double orc_fene_d2(double r, double r0, double k, double R0)
{
    double d = r - r0, u = (d * d) / (R0 * R0), x = 1.0 - u;
    return x > 0.0 ? k * (1.0 + u) / (x * x) : 0.0;
}

double orc_native_d2(double r, double r0, double eps)
{
    double q = pow(r0 / r, 6.0);
    return 12.0 * eps * (13.0 * q * q - 7.0 * q) / (r * r);
}

double orc_repulsive_d2(double r, double sigma, double eps)
{
    double q = pow(sigma / r, 6.0);
    return 42.0 * eps * q / (r * r);
}

/* ------------------------------------------------------------------------ */
/* helpers: trajectory of a residue and the sorted bonded/native partners    */
/* ------------------------------------------------------------------------ */

static int64_t traj_of(const orc_system *s, int64_t i)
{
    int64_t lo = 0, hi = s->n_traj; /* res_offsets[lo] <= i < res_offsets[hi] */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (s->res_offsets[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

typedef struct {
    int64_t *ptr;
    int32_t *col;
} excl_t;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int excl_build(const orc_system *s, excl_t *e)
{
    int64_t n = s->n_res;
    e->ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t m = 2 * (s->n_bonds + s->n_native);
    e->col = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!e->ptr || !e->col)
        return ORC_E_ARG;
    for (int64_t b = 0; b < s->n_bonds; ++b) {
        e->ptr[s->bonds[2 * b] + 1]++;
        e->ptr[s->bonds[2 * b + 1] + 1]++;
    }
    for (int64_t b = 0; b < s->n_native; ++b) {
        e->ptr[s->natives[2 * b] + 1]++;
        e->ptr[s->natives[2 * b + 1] + 1]++;
    }
    for (int64_t i = 0; i < n; ++i)
        e->ptr[i + 1] += e->ptr[i];
    int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!fill)
        return ORC_E_ARG;
    for (int64_t b = 0; b < s->n_bonds; ++b) {
        int32_t i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
        e->col[e->ptr[i] + fill[i]++] = j;
        e->col[e->ptr[j] + fill[j]++] = i;
    }
    for (int64_t b = 0; b < s->n_native; ++b) {
        int32_t i = s->natives[2 * b], j = s->natives[2 * b + 1];
        e->col[e->ptr[i] + fill[i]++] = j;
        e->col[e->ptr[j] + fill[j]++] = i;
    }
    free(fill);
    for (int64_t i = 0; i < n; ++i)
        qsort(e->col + e->ptr[i], (size_t)(e->ptr[i + 1] - e->ptr[i]), sizeof(int32_t), cmp_i32);
    return ORC_OK;
}

static void excl_free(excl_t *e)
{
    free(e->ptr);
    free(e->col);
}

static int excluded(const excl_t *e, int32_t i, int32_t j)
{
    const int32_t *c = e->col + e->ptr[i];
    return bsearch(&j, c, (size_t)(e->ptr[i + 1] - e->ptr[i]), sizeof(int32_t), cmp_i32) != NULL;
}

/* The single-precision list predicate (see the header comment). */
static int within_list_cutoff(const double *x, int64_t i, int64_t j, float rc2)
{
    float dx = (float)x[3 * i] - (float)x[3 * j];
    float dy = (float)x[3 * i + 1] - (float)x[3 * j + 1];
    float dz = (float)x[3 * i + 2] - (float)x[3 * j + 2];
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    s = s + zz;
    return s < rc2;
}

static float list_rc2(const orc_params *p)
{
    return (float)(p->r_list * p->r_list);
}

/* ------------------------------------------------------------------------ */
/* Verlet list (Algorithm 3's filter over all candidate pairs).              */
/* ------------------------------------------------------------------------ */

typedef struct {
    float xf;
    int32_t idx;
} sweep_t;

static int cmp_sweep(const void *a, const void *b)
{
    const sweep_t *x = (const sweep_t *)a, *y = (const sweep_t *)b;
    if (x->xf < y->xf)
        return -1;
    if (x->xf > y->xf)
        return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static int cmp_pair(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    if (x[0] != y[0])
        return (x[0] > y[0]) - (x[0] < y[0]);
    return (x[1] > y[1]) - (x[1] < y[1]);
}

/*
 * All pairs (i<j) of one trajectory that are neither bonded nor native and
 * pass the list predicate, sorted by (i, j).  Every candidate pair is tested;
 * a pair is skipped untested only when fl(xf_j - xf_i) >= rc along the
 * sorted x axis, which makes fl(dx*dx) >= rc^2 and the predicate false.
 * Returns the number of pairs (written only up to cap).
 */
int64_t orc_pairlist(const orc_system *s, const orc_params *p, const double *x, int32_t *ij,
                     int64_t cap)
{
    excl_t e;
    if (excl_build(s, &e) != ORC_OK)
        return ORC_E_ARG;
    float rc2 = list_rc2(p);
    float rcf = (float)p->r_list;
    int64_t count = 0, store = 0;
    int32_t *buf = NULL;
    for (int64_t t = 0; t < s->n_traj; ++t) {
        int64_t a = s->res_offsets[t], b = s->res_offsets[t + 1];
        int64_t n = b - a;
        if (n < 2)
            continue;
        sweep_t *sw = (sweep_t *)malloc((size_t)n * sizeof(sweep_t));
        for (int64_t k = 0; k < n; ++k) {
            sw[k].idx = (int32_t)(a + k);
            sw[k].xf = (float)x[3 * (a + k)];
        }
        qsort(sw, (size_t)n, sizeof(sweep_t), cmp_sweep);
        int64_t tstart = count;
        for (int64_t u = 0; u < n; ++u) {
            for (int64_t v = u + 1; v < n; ++v) {
                float gap = sw[v].xf - sw[u].xf;
                if (gap >= rcf)
                    break;
                int32_t i = sw[u].idx, j = sw[v].idx;
                if (i > j) {
                    int32_t tmp = i;
                    i = j;
                    j = tmp;
                }
                if (!within_list_cutoff(x, i, j, rc2) || excluded(&e, i, j))
                    continue;
                if ((count - tstart) % 4096 == 0) {
                    int32_t *nb = (int32_t *)realloc(buf, (size_t)(count - tstart + 4096) * 2 * sizeof(int32_t));
                    if (!nb) {
                        free(sw);
                        free(buf);
                        excl_free(&e);
                        return ORC_E_ARG;
                    }
                    buf = nb;
                }
                buf[2 * (count - tstart)] = i;
                buf[2 * (count - tstart) + 1] = j;
                ++count;
            }
        }
        free(sw);
        int64_t m = count - tstart;
        if (m > 0)
            qsort(buf, (size_t)m, 2 * sizeof(int32_t), cmp_pair);
        for (int64_t k = 0; k < m; ++k) {
            if (store < cap) {
                ij[2 * store] = buf[2 * k];
                ij[2 * store + 1] = buf[2 * k + 1];
            }
            ++store;
        }
    }
    free(buf);
    excl_free(&e);
    return count;
}

/* Plain O(N^2) double loop over (i<j), no pruning; for small systems. */
int64_t orc_pairlist_bruteforce(const orc_system *s, const orc_params *p, const double *x,
                                int32_t *ij, int64_t cap)
{
    excl_t e;
    if (excl_build(s, &e) != ORC_OK)
        return ORC_E_ARG;
    float rc2 = list_rc2(p);
    int64_t count = 0;
    for (int64_t t = 0; t < s->n_traj; ++t)
        for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i)
            for (int64_t j = i + 1; j < s->res_offsets[t + 1]; ++j)
                if (within_list_cutoff(x, i, j, rc2) && !excluded(&e, (int32_t)i, (int32_t)j)) {
                    if (count < cap) {
                        ij[2 * count] = (int32_t)i;
                        ij[2 * count + 1] = (int32_t)j;
                    }
                    ++count;
                }
    excl_free(&e);
    return count;
}

/* ------------------------------------------------------------------------ */
/* Forces (Algorithm 1) and energies                                        */
/* ------------------------------------------------------------------------ */

/* Add the pair force of dE/dr = g between i and j: f_i -= g d/r, f_j += g d/r. */
static void apply_pair(const double *x, int64_t i, int64_t j, double r, double g, double *F)
{
    for (int a = 0; a < 3; ++a) {
        double d = x[3 * i + a] - x[3 * j + a];
        double df = -g * d / r;
        F[3 * i + a] += df;
        F[3 * j + a] -= df;
    }
}

static double dist(const double *x, int64_t i, int64_t j)
{
    double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1], dz = x[3 * i + 2] - x[3 * j + 2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/*
 * External terms acting on residue i of trajectory t at time t_n = step*h:
 * every cantilever attached to i and the tip.  Adds the force to f, the
 * energy to *E_ext and the reported external force to *f_report.
 */
static int external_on_residue(const orc_system *s, const orc_params *p, const double *x,
                               int64_t step, int64_t t, int64_t i, double f[3], double *E_ext,
                               double *f_report)
{
    double tn = (double)step * p->h;
    for (int32_t k = 0; k < s->n_pull; ++k) {
        if (s->pull_traj[k] != t || s->pull_res[k] != i)
            continue;
        double kap = s->pull_kappa[k];
        double vv = 0.0, proj = 0.0, d2 = 0.0;
        for (int a = 0; a < 3; ++a)
            vv += s->pull_v[3 * k + a] * s->pull_v[3 * k + a];
        for (int a = 0; a < 3; ++a) {
            double A = s->pull_anchor0[3 * k + a] + s->pull_v[3 * k + a] * tn;
            double d = A - x[3 * i + a];
            d2 += d * d;
            f[a] += kap * d;
            if (vv > 0.0)
                proj += kap * d * s->pull_v[3 * k + a] / sqrt(vv);
        }
        *E_ext += 0.5 * kap * d2;
        *f_report += (vv > 0.0) ? proj : kap * sqrt(d2);
    }
    if (s->has_tip) {
        double vv = 0.0, d[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            vv += s->tip_v[a] * s->tip_v[a];
            d[a] = x[3 * i + a] - (s->tip_c0[a] + s->tip_v[a] * tn);
            r2 += d[a] * d[a];
        }
        double r = sqrt(r2);
        double gap = r - s->tip_radius;
        if (!(gap > 0.0))
            return ORC_E_TIP;
        double q = pow(s->tip_sigma / gap, 6.0);
        *E_ext += s->tip_eps * q;
        double mag = 6.0 * s->tip_eps * q / gap; /* -dE/ds, along (r_i - T)/|r_i - T| */
        for (int a = 0; a < 3; ++a) {
            f[a] += mag * d[a] / r;
            if (vv > 0.0)
                *f_report += mag * d[a] / r * s->tip_v[a] / sqrt(vv);
        }
    }
    return ORC_OK;
}

/*
 * Forces F (3*n_res) and per-trajectory energies E (n_traj*5: FENE, native,
 * repulsive, external, virial = -sum over internal pairs of r dE/dr) at the
 * configuration x for the given repulsive list.  f_ext (n_traj or NULL)
 * receives the cantilever force along its velocity plus the tip force along
 * the tip velocity.
 */
int orc_forces(const orc_system *s, const orc_params *p, const double *x, int64_t step,
               const int32_t *list_ij, int64_t n_list, double *F, double *E, double *f_ext)
{
    int broken = 0;
    memset(F, 0, (size_t)s->n_res * 3 * sizeof(double));
    if (E)
        memset(E, 0, (size_t)s->n_traj * ORC_NTERMS * sizeof(double));
    double *Et = (double *)calloc((size_t)s->n_traj * ORC_NTERMS, sizeof(double));
    if (!Et)
        return ORC_E_ARG;
    for (int64_t b = 0; b < s->n_bonds; ++b) {
        int64_t i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
        double r = dist(x, i, j), g;
        double en = orc_fene(r, s->bond_r0[b], p->k_fene, p->R0, &g, &broken);
        apply_pair(x, i, j, r, g, F);
        int64_t t = traj_of(s, i);
        Et[t * ORC_NTERMS + 0] += en;
        Et[t * ORC_NTERMS + 4] -= r * g;
    }
    for (int64_t b = 0; b < s->n_native; ++b) {
        int64_t i = s->natives[2 * b], j = s->natives[2 * b + 1];
        double r = dist(x, i, j), g;
        double en = orc_native(r, s->native_r0[b], p->eps_h, &g);
        apply_pair(x, i, j, r, g, F);
        int64_t t = traj_of(s, i);
        Et[t * ORC_NTERMS + 1] += en;
        Et[t * ORC_NTERMS + 4] -= r * g;
    }
    for (int64_t b = 0; b < n_list; ++b) {
        int64_t i = list_ij[2 * b], j = list_ij[2 * b + 1];
        double r = dist(x, i, j), g;
        double en = orc_repulsive(r, p->sigma, p->eps_l, &g);
        apply_pair(x, i, j, r, g, F);
        int64_t t = traj_of(s, i);
        Et[t * ORC_NTERMS + 2] += en;
        Et[t * ORC_NTERMS + 4] -= r * g;
    }
    int status = ORC_OK;
    for (int64_t t = 0; t < s->n_traj; ++t) {
        double fr = 0.0;
        for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i) {
            int st = external_on_residue(s, p, x, step, t, i, F + 3 * i, &Et[t * ORC_NTERMS + 3], &fr);
            if (st != ORC_OK && status == ORC_OK)
                status = st;
        }
        if (f_ext)
            f_ext[t] = fr;
    }
    if (E)
        memcpy(E, Et, (size_t)s->n_traj * ORC_NTERMS * sizeof(double));
    free(Et);
    if (broken)
        return ORC_E_FENE;
    if (status != ORC_OK)
        return status;
    for (int64_t k = 0; k < 3 * s->n_res; ++k)
        if (!isfinite(F[k]))
            return ORC_E_NONFINITE;
    return ORC_OK;
}

/*
 * Force on each listed residue computed on its own, straight from the
 * definition: every bonded and native partner, every other residue of its
 * trajectory that passes the list predicate at the configuration x_list
 * (the configuration of the last rebuild), and the external terms.  For
 * sampled checks of large systems.  F is 3*n_rows.
 */
int orc_forces_rows(const orc_system *s, const orc_params *p, const double *x,
                    const double *x_list, int64_t step, const int64_t *rows, int64_t n_rows,
                    double *F)
{
    excl_t e;
    if (excl_build(s, &e) != ORC_OK)
        return ORC_E_ARG;
    float rc2 = list_rc2(p);
    int status = ORC_OK;
    for (int64_t k = 0; k < n_rows; ++k) {
        int64_t i = rows[k];
        int64_t t = traj_of(s, i);
        double f[3] = {0.0, 0.0, 0.0};
        int broken = 0;
        for (int64_t b = 0; b < s->n_bonds; ++b) {
            int64_t u = s->bonds[2 * b], v = s->bonds[2 * b + 1];
            if (u != i && v != i)
                continue;
            int64_t j = (u == i) ? v : u;
            double r = dist(x, i, j), g;
            orc_fene(r, s->bond_r0[b], p->k_fene, p->R0, &g, &broken);
            for (int a = 0; a < 3; ++a)
                f[a] += -g * (x[3 * i + a] - x[3 * j + a]) / r;
        }
        for (int64_t b = 0; b < s->n_native; ++b) {
            int64_t u = s->natives[2 * b], v = s->natives[2 * b + 1];
            if (u != i && v != i)
                continue;
            int64_t j = (u == i) ? v : u;
            double r = dist(x, i, j), g;
            orc_native(r, s->native_r0[b], p->eps_h, &g);
            for (int a = 0; a < 3; ++a)
                f[a] += -g * (x[3 * i + a] - x[3 * j + a]) / r;
        }
        for (int64_t j = s->res_offsets[t]; j < s->res_offsets[t + 1]; ++j) {
            if (j == i || !within_list_cutoff(x_list, i, j, rc2) || excluded(&e, (int32_t)i, (int32_t)j))
                continue;
            double r = dist(x, i, j), g;
            orc_repulsive(r, p->sigma, p->eps_l, &g);
            for (int a = 0; a < 3; ++a)
                f[a] += -g * (x[3 * i + a] - x[3 * j + a]) / r;
        }
        if (broken)
            status = ORC_E_FENE;
        double dummyE = 0.0, dummyf = 0.0;
        int st = external_on_residue(s, p, x, step, t, i, f, &dummyE, &dummyf);
        if (st != ORC_OK && status == ORC_OK)
            status = st;
        for (int a = 0; a < 3; ++a)
            F[3 * k + a] = f[a];
    }
    excl_free(&e);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Integration (Eq. 2 / Algorithm 7)                                         */
/* ------------------------------------------------------------------------ */

/*
 * Advance x (3*n_res, in place) from step `step0` by n_steps steps.  The list
 * is rebuilt before the forces of step n when n % list_every == 0 and at the
 * first step of the call.  When energy_every > 0, the energies of x(t_n)
 * (before its update) are stored for every n with n % energy_every == 0 into
 * E_out (records of n_traj*5) and the external-force report into f_out
 * (records of n_traj); at most max_records records are written and the
 * number of records is returned through *n_records.
 */
int orc_run(const orc_system *s, const orc_params *p, double *x, int64_t step0, int64_t n_steps,
            int64_t energy_every, double *E_out, double *f_out, int64_t max_records,
            int64_t *n_records)
{
    int64_t n = s->n_res;
    double *F = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *E = (double *)malloc((size_t)s->n_traj * ORC_NTERMS * sizeof(double));
    double *fe = (double *)malloc((size_t)s->n_traj * sizeof(double));
    int32_t *list = NULL;
    int64_t n_list = 0, rec = 0;
    int status = ORC_OK;
    double drift = p->h / p->zeta;
    double noise = sqrt(2.0 * p->kBT * p->h / p->zeta);
    for (int64_t q = 0; q < n_steps && status == ORC_OK; ++q) {
        int64_t step = step0 + q;
        if (q == 0 || step % p->list_every == 0) {
            int64_t m = orc_pairlist(s, p, x, NULL, 0);
            free(list);
            list = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * 2 * sizeof(int32_t));
            n_list = orc_pairlist(s, p, x, list, m);
        }
        status = orc_forces(s, p, x, step, list, n_list, F, E, fe);
        if (status != ORC_OK)
            break;
        if (energy_every > 0 && step % energy_every == 0 && rec < max_records) {
            if (E_out)
                memcpy(E_out + rec * s->n_traj * ORC_NTERMS, E,
                       (size_t)s->n_traj * ORC_NTERMS * sizeof(double));
            if (f_out)
                memcpy(f_out + rec * s->n_traj, fe, (size_t)s->n_traj * sizeof(double));
            ++rec;
        }
        for (int64_t t = 0; t < s->n_traj; ++t) {
            for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i) {
                if (s->fixed && s->fixed[i])
                    continue;
                double g[3];
                orc_gauss3(p->seed, (uint32_t)(i - s->res_offsets[t]), s->stream_ids[t], step, g);
                for (int a = 0; a < 3; ++a)
                    x[3 * i + a] += drift * F[3 * i + a] + noise * g[a];
            }
        }
    }
    if (n_records)
        *n_records = rec;
    free(F);
    free(E);
    free(fe);
    free(list);
    return status;
}

/*
 * Underdamped Langevin dynamics, m dv = F dt - zeta v dt + sqrt(2 zeta kB T) dW
 * and dx = v dt, with the SOP forces of Eq. 1 and the list rules of orc_run
 * (the paper's conclusion names this limit as an extension of its
 * first-order integration kernel and gives no scheme).  Each step is the
 * BAOAB splitting of Leimkuhler and Matthews (Appl. Math. Res. Express,
 * 2013): with gamma = zeta/m, c1 = exp(-gamma h), c2 = sqrt((1 - c1^2) kB T/m)
 * and the residue's Gaussians g of step n (orc_gauss3, the same counters as
 * the overdamped noise),
 *   B: v += (h/2m) F(x_n);   A: x += (h/2) v;   O: v = c1 v + c2 g;
 *   A: x += (h/2) v;          B: v += (h/2m) F(x_{n+1}),
 * F(x_{n+1}) being the force of step n+1 (its list rebuilt when
 * (n+1) % list_every == 0).  Fixed residues neither move nor carry a
 * velocity.  x and v (3*n_res each) are the positions and velocities at
 * t_step0 on entry and at t_(step0+n_steps) on return.
 */
int orc_run_underdamped(const orc_system *s, const orc_params *p, double mass, double *x, double *v,
                        int64_t step0, int64_t n_steps)
{
    int64_t n = s->n_res;
    if (!(mass > 0.0))
        return ORC_E_ARG;
    double *F = (double *)malloc((size_t)n * 3 * sizeof(double));
    int32_t *list = NULL;
    int64_t n_list = 0;
    int status = ORC_OK;
    double h = p->h, kick = 0.5 * h / mass;
    double c1 = exp(-p->zeta / mass * h);
    double c2 = sqrt((1.0 - c1 * c1) * p->kBT / mass);
    for (int64_t q = 0; q <= n_steps && status == ORC_OK; ++q) {
        int64_t step = step0 + q;
        if (q == 0 || step % p->list_every == 0) {
            int64_t m = orc_pairlist(s, p, x, NULL, 0);
            free(list);
            list = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * 2 * sizeof(int32_t));
            n_list = orc_pairlist(s, p, x, list, m);
        }
        status = orc_forces(s, p, x, step, list, n_list, F, NULL, NULL);
        if (status != ORC_OK)
            break;
        for (int64_t t = 0; t < s->n_traj; ++t) {
            for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i) {
                if (s->fixed && s->fixed[i]) {
                    v[3 * i] = v[3 * i + 1] = v[3 * i + 2] = 0.0;
                    continue;
                }
                if (q > 0)  /* the last B of the previous step */
                    for (int a = 0; a < 3; ++a)
                        v[3 * i + a] += kick * F[3 * i + a];
                if (q == n_steps)
                    continue;
                double g[3];
                orc_gauss3(p->seed, (uint32_t)(i - s->res_offsets[t]), s->stream_ids[t], step, g);
                for (int a = 0; a < 3; ++a) {
                    double w = v[3 * i + a] + kick * F[3 * i + a];  /* B */
                    x[3 * i + a] += 0.5 * h * w;                    /* A */
                    w = c1 * w + c2 * g[a];                         /* O */
                    x[3 * i + a] += 0.5 * h * w;                    /* A */
                    v[3 * i + a] = w;
                }
            }
        }
    }
    free(F);
    free(list);
    return status;
}

/*
 * Replica exchange (parallel tempering) over an ensemble of independent
 * trajectories, the use of the many-runs-per-GPU approach the paper's
 * conclusion proposes.  The n_traj trajectories form groups of n_rep
 * consecutive ones (n_traj a multiple of n_rep); each group's members carry
 * the temperatures kbt[0 .. n_rep-1] as a permutation: tidx[t] is the
 * temperature index of trajectory t.  Each step is orc_run's first-order
 * step with the residue's noise amplitude sqrt(2 kbt[tidx[t]] h / zeta).
 * At every step n with n % exchange_every == 0, before its update, round
 * r = n / exchange_every attempts, in every group, the swaps of the
 * trajectories at temperatures k and k+1 for k = r mod 2, r mod 2 + 2, ...:
 * with E the potential energy of x(t_n) (FENE + native + repulsive +
 * external) and d = (1/kbt[k] - 1/kbt[k+1]) (E_k - E_(k+1)), the swap is
 * accepted when d >= 0 or u < exp(d) (Metropolis), u = orc_uniform of the
 * first Philox4x32-10 word for counter (group, k, r low, r high) and key
 * (seed low ^ 0x52455843, seed high) (a key of its own, so that these draws
 * never repeat a noise draw).  Accepted swaps exchange the two temperature
 * indices.  accepted[k] and attempted[k] (n_rep - 1 each, may be NULL) are
 * incremented.
 */
int orc_run_tempered(const orc_system *s, const orc_params *p, double *x, int64_t step0,
                     int64_t n_steps, int32_t n_rep, const double *kbt, int64_t exchange_every,
                     int32_t *tidx, int64_t *accepted, int64_t *attempted)
{
    int64_t n = s->n_res;
    if (n_rep < 1 || s->n_traj % n_rep != 0 || exchange_every < 0)
        return ORC_E_ARG;
    double *F = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *E = (double *)malloc((size_t)s->n_traj * ORC_NTERMS * sizeof(double));
    int32_t *at = (int32_t *)malloc((size_t)s->n_traj * sizeof(int32_t));
    int32_t *list = NULL;
    int64_t n_list = 0;
    int status = ORC_OK;
    double drift = p->h / p->zeta;
    int64_t n_groups = s->n_traj / n_rep;
    for (int64_t q = 0; q < n_steps && status == ORC_OK; ++q) {
        int64_t step = step0 + q;
        if (q == 0 || step % p->list_every == 0) {
            int64_t m = orc_pairlist(s, p, x, NULL, 0);
            free(list);
            list = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * 2 * sizeof(int32_t));
            n_list = orc_pairlist(s, p, x, list, m);
        }
        status = orc_forces(s, p, x, step, list, n_list, F, E, NULL);
        if (status != ORC_OK)
            break;
        if (exchange_every > 0 && step % exchange_every == 0 && n_rep > 1) {
            int64_t r = step / exchange_every;
            uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu) ^ 0x52455843u, (uint32_t)(p->seed >> 32)};
            for (int64_t g = 0; g < n_groups; ++g) {
                for (int32_t k = 0; k < n_rep; ++k)  /* the trajectory at each temperature */
                    at[g * n_rep + tidx[g * n_rep + k]] = (int32_t)(g * n_rep + k);
                for (int32_t k = (int32_t)(r % 2); k + 1 < n_rep; k += 2) {
                    int32_t a = at[g * n_rep + k], b = at[g * n_rep + k + 1];
                    double Ea = 0.0, Eb = 0.0;
                    for (int term = 0; term < 4; ++term) {
                        Ea += E[a * ORC_NTERMS + term];
                        Eb += E[b * ORC_NTERMS + term];
                    }
                    double d = (1.0 / kbt[k] - 1.0 / kbt[k + 1]) * (Ea - Eb);
                    uint32_t ctr[4] = {(uint32_t)g, (uint32_t)k, (uint32_t)r, (uint32_t)((uint64_t)r >> 32)};
                    uint32_t w[4];
                    orc_philox4x32_10(ctr, key, w);
                    if (attempted)
                        ++attempted[k];
                    if (d >= 0.0 || orc_uniform(w[0]) < exp(d)) {
                        tidx[a] = k + 1;
                        tidx[b] = k;
                        if (accepted)
                            ++accepted[k];
                    }
                }
            }
        }
        for (int64_t t = 0; t < s->n_traj; ++t) {
            double noise = sqrt(2.0 * kbt[tidx[t]] * p->h / p->zeta);
            for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i) {
                if (s->fixed && s->fixed[i])
                    continue;
                double g[3];
                orc_gauss3(p->seed, (uint32_t)(i - s->res_offsets[t]), s->stream_ids[t], step, g);
                for (int a = 0; a < 3; ++a)
                    x[3 * i + a] += drift * F[3 * i + a] + noise * g[a];
            }
        }
    }
    free(F);
    free(E);
    free(at);
    free(list);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Rounding scale of each residue's force and each energy term              */
/* ------------------------------------------------------------------------ */

/*
 * Magnitudes of the external forces on residue i of trajectory t at
 * t_n = step*h, term by term (each cantilever attached to i, then the tip);
 * their energies are added to *E_mag.  Returns the sum of the magnitudes.
 */
static double external_magnitude(const orc_system *s, const orc_params *p, const double *x,
                                 int64_t step, int64_t t, int64_t i, double *E_mag)
{
    double tn = (double)step * p->h, sum = 0.0;
    for (int32_t k = 0; k < s->n_pull; ++k) {
        if (s->pull_traj[k] != t || s->pull_res[k] != i)
            continue;
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double d = s->pull_anchor0[3 * k + a] + s->pull_v[3 * k + a] * tn - x[3 * i + a];
            d2 += d * d;
        }
        sum += s->pull_kappa[k] * sqrt(d2);
        *E_mag += 0.5 * s->pull_kappa[k] * d2;
    }
    if (s->has_tip) {
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double d = x[3 * i + a] - (s->tip_c0[a] + s->tip_v[a] * tn);
            r2 += d * d;
        }
        double gap = sqrt(r2) - s->tip_radius;
        if (gap > 0.0) {
            double q = pow(s->tip_sigma / gap, 6.0);
            sum += 6.0 * s->tip_eps * q / gap;
            *E_mag += s->tip_eps * q;
        }
    }
    return sum;
}

/*
 * The scale against which an approximate evaluation of the forces and
 * energies of Eq. 1 is compared with this oracle, term by term:
 *   S[i]       = sum over the bonded, native and listed pairs containing i
 *                of |dE/dr|, plus the magnitude of every external force
 *                on i (n_res values);
 *   Em[5t + k] = for k = 0, 1, 2: the sum of |E| over the FENE, native and
 *                repulsive pairs of trajectory t; k = 3: the sum of the
 *                external energies; k = 4: the sum of |r dE/dr| over the
 *                pairs (the terms of the virial).
 * By the triangle inequality |F_i| <= S[i], with equality when every term
 * acting on i points the same way (a residue with a single partner).
 */
int orc_force_scale(const orc_system *s, const orc_params *p, const double *x, int64_t step,
                    const int32_t *list_ij, int64_t n_list, double *S, double *Em)
{
    int broken = 0;
    memset(S, 0, (size_t)s->n_res * sizeof(double));
    if (Em)
        memset(Em, 0, (size_t)s->n_traj * ORC_NTERMS * sizeof(double));
    for (int64_t b = 0; b < s->n_bonds; ++b) {
        int64_t i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
        double r = dist(x, i, j), g;
        double en = orc_fene(r, s->bond_r0[b], p->k_fene, p->R0, &g, &broken);
        S[i] += fabs(g);
        S[j] += fabs(g);
        if (Em) {
            int64_t t = traj_of(s, i);
            Em[t * ORC_NTERMS + 0] += fabs(en);
            Em[t * ORC_NTERMS + 4] += fabs(r * g);
        }
    }
    for (int64_t b = 0; b < s->n_native; ++b) {
        int64_t i = s->natives[2 * b], j = s->natives[2 * b + 1];
        double r = dist(x, i, j), g;
        double en = orc_native(r, s->native_r0[b], p->eps_h, &g);
        S[i] += fabs(g);
        S[j] += fabs(g);
        if (Em) {
            int64_t t = traj_of(s, i);
            Em[t * ORC_NTERMS + 1] += fabs(en);
            Em[t * ORC_NTERMS + 4] += fabs(r * g);
        }
    }
    for (int64_t b = 0; b < n_list; ++b) {
        int64_t i = list_ij[2 * b], j = list_ij[2 * b + 1];
        double r = dist(x, i, j), g;
        double en = orc_repulsive(r, p->sigma, p->eps_l, &g);
        S[i] += fabs(g);
        S[j] += fabs(g);
        if (Em) {
            int64_t t = traj_of(s, i);
            Em[t * ORC_NTERMS + 2] += fabs(en);
            Em[t * ORC_NTERMS + 4] += fabs(r * g);
        }
    }
    for (int64_t t = 0; t < s->n_traj; ++t)
        for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i) {
            double e = 0.0;
            S[i] += external_magnitude(s, p, x, step, t, i, &e);
            if (Em)
                Em[t * ORC_NTERMS + 3] += e;
        }
    return broken ? ORC_E_FENE : ORC_OK;
}

/*
 * The stiffness scale: K[i] = the sum over the bonded, native and listed
 * pairs containing i of r |d^2E/dr^2|, plus, for every external term on i,
 * its force's change per relative change of its own distance (the
 * cantilever: kappa |A - x_i|, the magnitude of its force; the tip:
 * |d^2E/ds^2| |x_i - T| for the gap s = |x_i - T| - R).  A relative error
 * eta in every distance moves F_i by at most about eta K[i], which S[i]
 * cannot bound where the pair forces vanish (at r = r0 both the FENE and the
 * native terms of Eq. 1 are at their minima: dE/dr = 0 but d^2E/dr^2 > 0).
 */
int orc_force_stiffness(const orc_system *s, const orc_params *p, const double *x, int64_t step,
                        const int32_t *list_ij, int64_t n_list, double *K)
{
    memset(K, 0, (size_t)s->n_res * sizeof(double));
    for (int64_t b = 0; b < s->n_bonds; ++b) {
        int64_t i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
        double r = dist(x, i, j);
        double v = r * fabs(orc_fene_d2(r, s->bond_r0[b], p->k_fene, p->R0));
        K[i] += v;
        K[j] += v;
    }
    for (int64_t b = 0; b < s->n_native; ++b) {
        int64_t i = s->natives[2 * b], j = s->natives[2 * b + 1];
        double r = dist(x, i, j);
        double v = r * fabs(orc_native_d2(r, s->native_r0[b], p->eps_h));
        K[i] += v;
        K[j] += v;
    }
    for (int64_t b = 0; b < n_list; ++b) {
        int64_t i = list_ij[2 * b], j = list_ij[2 * b + 1];
        double r = dist(x, i, j);
        double v = r * fabs(orc_repulsive_d2(r, p->sigma, p->eps_l));
        K[i] += v;
        K[j] += v;
    }
    double tn = (double)step * p->h;
    for (int64_t t = 0; t < s->n_traj; ++t)
        for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i) {
            for (int32_t k = 0; k < s->n_pull; ++k) {
                if (s->pull_traj[k] != t || s->pull_res[k] != i)
                    continue;
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double d = s->pull_anchor0[3 * k + a] + s->pull_v[3 * k + a] * tn - x[3 * i + a];
                    d2 += d * d;
                }
                K[i] += s->pull_kappa[k] * sqrt(d2);
            }
            if (s->has_tip) {
                double r2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double d = x[3 * i + a] - (s->tip_c0[a] + s->tip_v[a] * tn);
                    r2 += d * d;
                }
                double rr = sqrt(r2), gap = rr - s->tip_radius;
                if (gap > 0.0)
                    K[i] += rr * orc_repulsive_d2(gap, s->tip_sigma, s->tip_eps);
            }
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The same dynamics, residue-parallel (OpenMP): each residue's force is    */
/* gathered from its own partners (the particle-based form of Algorithm 2)  */
/* instead of scattered pair by pair (Algorithm 1).  Only the order of the  */
/* floating-point sums differs from orc_forces / orc_run.                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t *ptr;  /* n_res + 1 */
    int32_t *col;  /* partners, ascending within a row */
} rows_t;

typedef struct {
    int64_t *ptr;  /* n_res + 1 */
    int32_t *col;  /* bonded partners first, then native partners */
    double *r0;
    int32_t *nb;   /* bonded partners per residue */
} topo_rows_t;

static int topo_rows_build(const orc_system *s, topo_rows_t *tr)
{
    int64_t n = s->n_res, m = 2 * (s->n_bonds + s->n_native);
    tr->ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    tr->col = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    tr->r0 = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    tr->nb = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!tr->ptr || !tr->col || !tr->r0 || !tr->nb || !fill) {
        free(fill);
        return ORC_E_ARG;
    }
    for (int64_t b = 0; b < s->n_bonds; ++b) {
        tr->ptr[s->bonds[2 * b] + 1]++;
        tr->ptr[s->bonds[2 * b + 1] + 1]++;
        tr->nb[s->bonds[2 * b]]++;
        tr->nb[s->bonds[2 * b + 1]]++;
    }
    for (int64_t b = 0; b < s->n_native; ++b) {
        tr->ptr[s->natives[2 * b] + 1]++;
        tr->ptr[s->natives[2 * b + 1] + 1]++;
    }
    for (int64_t i = 0; i < n; ++i)
        tr->ptr[i + 1] += tr->ptr[i];
    for (int64_t b = 0; b < s->n_bonds; ++b)
        for (int e = 0; e < 2; ++e) {
            int32_t i = s->bonds[2 * b + e], j = s->bonds[2 * b + 1 - e];
            tr->col[tr->ptr[i] + fill[i]] = j;
            tr->r0[tr->ptr[i] + fill[i]++] = s->bond_r0[b];
        }
    for (int64_t b = 0; b < s->n_native; ++b)
        for (int e = 0; e < 2; ++e) {
            int32_t i = s->natives[2 * b + e], j = s->natives[2 * b + 1 - e];
            tr->col[tr->ptr[i] + fill[i]] = j;
            tr->r0[tr->ptr[i] + fill[i]++] = s->native_r0[b];
        }
    free(fill);
    return ORC_OK;
}

static void topo_rows_free(topo_rows_t *tr)
{
    free(tr->ptr);
    free(tr->col);
    free(tr->r0);
    free(tr->nb);
}

static int cmp_sweep_idx(const void *a, const void *b) { return cmp_sweep(a, b); }

/*
 * Verlet-list rows: for every residue i, the residues j != i of its
 * trajectory that are neither bonded nor native to it and pass the
 * single-precision list predicate at x (Algorithm 3, row by row), in
 * ascending order.  A candidate is skipped untested only where the sorted x
 * coordinates are rc or more apart (the predicate is then false, as in
 * orc_pairlist).
 */
static int rows_build(const orc_system *s, const orc_params *p, const excl_t *e, const double *x,
                      rows_t *r, int nthreads)
{
    int64_t n = s->n_res;
    float rc2 = list_rc2(p);
    float rcf = (float)p->r_list;
    sweep_t *sw = (sweep_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(sweep_t));
    int64_t *pos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    r->ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!sw || !pos || !r->ptr) {
        free(sw);
        free(pos);
        return ORC_E_ARG;
    }
    for (int64_t t = 0; t < s->n_traj; ++t) {
        int64_t a = s->res_offsets[t], b = s->res_offsets[t + 1];
        for (int64_t k = a; k < b; ++k) {
            sw[k].idx = (int32_t)k;
            sw[k].xf = (float)x[3 * k];
        }
        qsort(sw + a, (size_t)(b - a), sizeof(sweep_t), cmp_sweep_idx);
        for (int64_t k = a; k < b; ++k)
            pos[sw[k].idx] = k;
    }
    /* two passes over the same candidates: count, then fill */
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < n; ++i)
                r->ptr[i + 1] += r->ptr[i];
            r->col = (int32_t *)malloc((size_t)(r->ptr[n] > 0 ? r->ptr[n] : 1) * sizeof(int32_t));
            if (!r->col) {
                free(sw);
                free(pos);
                return ORC_E_ARG;
            }
        }
#pragma omp parallel for schedule(dynamic, 512) num_threads(nthreads)
        for (int64_t i = 0; i < n; ++i) {
            int64_t t = traj_of(s, i);
            int64_t a = s->res_offsets[t], b = s->res_offsets[t + 1];
            int64_t u = pos[i], cnt = 0;
            int32_t *out = pass ? r->col + r->ptr[i] : NULL;
            for (int dir = -1; dir <= 1; dir += 2)
                for (int64_t v = u + dir; v >= a && v < b; v += dir) {
                    float gap = dir > 0 ? sw[v].xf - sw[u].xf : sw[u].xf - sw[v].xf;
                    if (gap >= rcf)
                        break;
                    int32_t j = sw[v].idx;
                    if (!within_list_cutoff(x, i, j, rc2) || excluded(e, (int32_t)i, j))
                        continue;
                    if (pass)
                        out[cnt] = j;
                    ++cnt;
                }
            if (pass)
                qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);
            else
                r->ptr[i + 1] = cnt;
        }
    }
    free(sw);
    free(pos);
    return ORC_OK;
}

/* Force on residue i from its bonded, native and listed partners and the
 * external terms; half of each pair energy and virial term goes to i. */
static int residue_force(const orc_system *s, const orc_params *p, const topo_rows_t *tr,
                         const rows_t *r, const double *x, int64_t step, int64_t i, double f[3],
                         double eh[ORC_NTERMS], double *f_report)
{
    int broken = 0;
    f[0] = f[1] = f[2] = 0.0;
    for (int k = 0; k < ORC_NTERMS; ++k)
        eh[k] = 0.0;
    for (int64_t e = tr->ptr[i]; e < tr->ptr[i + 1]; ++e) {
        int64_t j = tr->col[e];
        double rr = dist(x, i, j), g, en;
        if (e - tr->ptr[i] < tr->nb[i]) {
            en = orc_fene(rr, tr->r0[e], p->k_fene, p->R0, &g, &broken);
            eh[0] += 0.5 * en;
        } else {
            en = orc_native(rr, tr->r0[e], p->eps_h, &g);
            eh[1] += 0.5 * en;
        }
        eh[4] -= 0.5 * rr * g;
        for (int a = 0; a < 3; ++a)
            f[a] += -g * (x[3 * i + a] - x[3 * j + a]) / rr;
    }
    for (int64_t e = r->ptr[i]; e < r->ptr[i + 1]; ++e) {
        int64_t j = r->col[e];
        double rr = dist(x, i, j), g;
        double en = orc_repulsive(rr, p->sigma, p->eps_l, &g);
        eh[2] += 0.5 * en;
        eh[4] -= 0.5 * rr * g;
        for (int a = 0; a < 3; ++a)
            f[a] += -g * (x[3 * i + a] - x[3 * j + a]) / rr;
    }
    int st = external_on_residue(s, p, x, step, traj_of(s, i), i, f, &eh[3], f_report);
    if (broken)
        return ORC_E_FENE;
    return st;
}

/* Forces and energies of every residue at x (list rows built at x_list),
 * then the per-trajectory sums in residue order. */
static int forces_rowwise(const orc_system *s, const orc_params *p, const topo_rows_t *tr,
                          const rows_t *r, const double *x, int64_t step, double *F, double *E,
                          double *f_ext, double *eres, double *fres, int nthreads)
{
    int status = ORC_OK;
    int64_t n = s->n_res;
#pragma omp parallel for schedule(dynamic, 512) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
        double rep = 0.0;
        int st = residue_force(s, p, tr, r, x, step, i, F + 3 * i, eres + (size_t)i * ORC_NTERMS, &rep);
        fres[i] = rep;
        if (st != ORC_OK) {
#pragma omp critical
            if (status == ORC_OK)
                status = st;
        }
    }
    for (int64_t t = 0; t < s->n_traj; ++t) {
        double acc[ORC_NTERMS] = {0, 0, 0, 0, 0}, fr = 0.0;
        for (int64_t i = s->res_offsets[t]; i < s->res_offsets[t + 1]; ++i) {
            for (int k = 0; k < ORC_NTERMS; ++k)
                acc[k] += eres[(size_t)i * ORC_NTERMS + k];
            fr += fres[i];
        }
        if (E)
            memcpy(E + t * ORC_NTERMS, acc, sizeof acc);
        if (f_ext)
            f_ext[t] = fr;
    }
    if (status != ORC_OK)
        return status;
    for (int64_t k = 0; k < 3 * n; ++k)
        if (!isfinite(F[k]))
            return ORC_E_NONFINITE;
    return ORC_OK;
}

/* Residue-parallel form of orc_forces, with the list rebuilt at x. */
int orc_forces_par(const orc_system *s, const orc_params *p, const double *x, int64_t step,
                   double *F, double *E, double *f_ext, int nthreads)
{
    excl_t e;
    topo_rows_t tr;
    rows_t r = {NULL, NULL};
    if (nthreads <= 0)
        nthreads = 1;
    if (excl_build(s, &e) != ORC_OK || topo_rows_build(s, &tr) != ORC_OK)
        return ORC_E_ARG;
    int st = rows_build(s, p, &e, x, &r, nthreads);
    double *eres = (double *)malloc((size_t)(s->n_res > 0 ? s->n_res : 1) * ORC_NTERMS * sizeof(double));
    double *fres = (double *)malloc((size_t)(s->n_res > 0 ? s->n_res : 1) * sizeof(double));
    if (st == ORC_OK && eres && fres)
        st = forces_rowwise(s, p, &tr, &r, x, step, F, E, f_ext, eres, fres, nthreads);
    else if (st == ORC_OK)
        st = ORC_E_ARG;
    free(eres);
    free(fres);
    free(r.ptr);
    free(r.col);
    topo_rows_free(&tr);
    excl_free(&e);
    return st;
}

/* Residue-parallel form of orc_run: the same steps, list rebuilds, noise
 * and energy records. */
int orc_run_par(const orc_system *s, const orc_params *p, double *x, int64_t step0, int64_t n_steps,
                int64_t energy_every, double *E_out, double *f_out, int64_t max_records,
                int64_t *n_records, int nthreads)
{
    int64_t n = s->n_res, rec = 0;
    excl_t e;
    topo_rows_t tr;
    rows_t r = {NULL, NULL};
    if (nthreads <= 0)
        nthreads = 1;
    if (excl_build(s, &e) != ORC_OK || topo_rows_build(s, &tr) != ORC_OK)
        return ORC_E_ARG;
    double *F = (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    double *E = (double *)malloc((size_t)s->n_traj * ORC_NTERMS * sizeof(double));
    double *fe = (double *)malloc((size_t)s->n_traj * sizeof(double));
    double *eres = (double *)malloc((size_t)(n > 0 ? n : 1) * ORC_NTERMS * sizeof(double));
    double *fres = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int status = (F && E && fe && eres && fres) ? ORC_OK : ORC_E_ARG;
    double drift = p->h / p->zeta;
    double noise = sqrt(2.0 * p->kBT * p->h / p->zeta);
    for (int64_t q = 0; q < n_steps && status == ORC_OK; ++q) {
        int64_t step = step0 + q;
        if (q == 0 || step % p->list_every == 0) {
            free(r.ptr);
            free(r.col);
            r.ptr = NULL;
            r.col = NULL;
            status = rows_build(s, p, &e, x, &r, nthreads);
            if (status != ORC_OK)
                break;
        }
        status = forces_rowwise(s, p, &tr, &r, x, step, F, E, fe, eres, fres, nthreads);
        if (status != ORC_OK)
            break;
        if (energy_every > 0 && step % energy_every == 0 && rec < max_records) {
            if (E_out)
                memcpy(E_out + rec * s->n_traj * ORC_NTERMS, E,
                       (size_t)s->n_traj * ORC_NTERMS * sizeof(double));
            if (f_out)
                memcpy(f_out + rec * s->n_traj, fe, (size_t)s->n_traj * sizeof(double));
            ++rec;
        }
#pragma omp parallel for schedule(static) num_threads(nthreads)
        for (int64_t i = 0; i < n; ++i) {
            if (s->fixed && s->fixed[i])
                continue;
            int64_t t = traj_of(s, i);
            double g[3];
            orc_gauss3(p->seed, (uint32_t)(i - s->res_offsets[t]), s->stream_ids[t], step, g);
            for (int a = 0; a < 3; ++a)
                x[3 * i + a] += drift * F[3 * i + a] + noise * g[a];
        }
    }
    if (n_records)
        *n_records = rec;
    free(F);
    free(E);
    free(fe);
    free(eres);
    free(fres);
    free(r.ptr);
    free(r.col);
    topo_rows_free(&tr);
    excl_free(&e);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Section IV.C: an exactly solvable model for the accuracy of the           */
/* integrators.  A Brownian particle X in the harmonic well K_sp X^2/2 (well */
/* at the origin; X(0) = X0) under the force ramp f_ext = r_f t, friction    */
/* xi, tau = xi/K_sp.                                                         */
/* ------------------------------------------------------------------------ */

/* Eq. 3: <X(t)> = X0 exp(-t/tau) + (r_f tau/xi) (t - tau (1 - exp(-t/tau))). */
double orc_ramp_mean_exact(double X0, double rf, double xi, double Ksp, double t)
{
    double tau = xi / Ksp;
    return X0 * exp(-t / tau) + rf * tau / xi * (t - tau * (1.0 - exp(-t / tau)));
}

/*
 * The mean recursions from X_0 = X0 over n steps of h, t_k = k h:
 *   order 1 (Eq. 4): X_{k+1} = X_k + (r_f t_k/xi - X_k/tau) h;
 *   order 2 (Eq. 5): the same plus (X_k/(2 tau^2) - r_f t_k/(2 tau xi)) h^2.
 * Returns X_n.
 */
double orc_ramp_mean_recursion(int order, double X0, double rf, double xi, double Ksp, double h,
                               int64_t n)
{
    double tau = xi / Ksp, X = X0;
    for (int64_t k = 0; k < n; ++k) {
        double tk = (double)k * h;
        double next = X + (rf * tk / xi - X / tau) * h;
        if (order == 2)
            next += (X / (2.0 * tau * tau) - rf * tk / (2.0 * tau * xi)) * h * h;
        X = next;
    }
    return X;
}

/*
 * M independent particles of the same model, advanced in place from step
 * `step0` by n steps of the scheme of the given order with the random
 * displacement sqrt(2 kB T h/xi) g (the Eq. 2 noise):
 *   order 1: X += (r_f t_k - K_sp X) h/xi + noise;
 *   order 2: the deterministic part of the order-2 recursion (Eq. 5) + noise.
 * g is the first Gaussian of orc_gauss3 for counter (particle index,
 * stream, step).  The forces are those of the per-particle Eq. 4 / Eq. 5
 * steps, so the ensemble mean follows those recursions.
 */
void orc_ramp_run(int order, int64_t M, double *X, int64_t step0, int64_t n, double rf, double xi,
                  double Ksp, double kBT, double h, uint64_t seed, uint32_t stream)
{
    double tau = xi / Ksp;
    double noise = sqrt(2.0 * kBT * h / xi);
    for (int64_t m = 0; m < M; ++m) {
        double x = X[m];
        for (int64_t k = step0; k < step0 + n; ++k) {
            double tk = (double)k * h;
            double g[3];
            orc_gauss3(seed, (uint32_t)m, stream, k, g);
            double next = x + (rf * tk / xi - x / tau) * h;
            if (order == 2)
                next += (x / (2.0 * tau * tau) - rf * tk / (2.0 * tau * xi)) * h * h;
            x = next + noise * g[0];
        }
        X[m] = x;
    }
}

/* Residue-parallel form of orc_force_scale's S (list rebuilt at x). */
int orc_force_scale_par(const orc_system *s, const orc_params *p, const double *x, int64_t step,
                        double *S, int nthreads)
{
    excl_t e;
    topo_rows_t tr;
    rows_t r = {NULL, NULL};
    if (nthreads <= 0)
        nthreads = 1;
    if (excl_build(s, &e) != ORC_OK || topo_rows_build(s, &tr) != ORC_OK)
        return ORC_E_ARG;
    int st = rows_build(s, p, &e, x, &r, nthreads);
    int broken = 0;
    if (st == ORC_OK) {
#pragma omp parallel for schedule(dynamic, 512) num_threads(nthreads) reduction(| : broken)
        for (int64_t i = 0; i < s->n_res; ++i) {
            double sum = 0.0, g, dummy = 0.0;
            for (int64_t k = tr.ptr[i]; k < tr.ptr[i + 1]; ++k) {
                double rr = dist(x, i, tr.col[k]);
                if (k - tr.ptr[i] < tr.nb[i])
                    orc_fene(rr, tr.r0[k], p->k_fene, p->R0, &g, &broken);
                else
                    orc_native(rr, tr.r0[k], p->eps_h, &g);
                sum += fabs(g);
            }
            for (int64_t k = r.ptr[i]; k < r.ptr[i + 1]; ++k) {
                orc_repulsive(dist(x, i, r.col[k]), p->sigma, p->eps_l, &g);
                sum += fabs(g);
            }
            S[i] = sum + external_magnitude(s, p, x, step, traj_of(s, i), i, &dummy);
        }
        if (broken)
            st = ORC_E_FENE;
    }
    free(r.ptr);
    free(r.col);
    topo_rows_free(&tr);
    excl_free(&e);
    return st;
}

/* Residue-parallel form of orc_force_stiffness (list rebuilt at x). */
int orc_force_stiffness_par(const orc_system *s, const orc_params *p, const double *x, int64_t step,
                            double *K, int nthreads)
{
    excl_t e;
    topo_rows_t tr;
    rows_t r = {NULL, NULL};
    if (nthreads <= 0)
        nthreads = 1;
    if (excl_build(s, &e) != ORC_OK || topo_rows_build(s, &tr) != ORC_OK)
        return ORC_E_ARG;
    int st = rows_build(s, p, &e, x, &r, nthreads);
    if (st == ORC_OK) {
        double tn = (double)step * p->h;
#pragma omp parallel for schedule(dynamic, 512) num_threads(nthreads)
        for (int64_t i = 0; i < s->n_res; ++i) {
            double sum = 0.0;
            for (int64_t k = tr.ptr[i]; k < tr.ptr[i + 1]; ++k) {
                double rr = dist(x, i, tr.col[k]);
                double d2 = k - tr.ptr[i] < tr.nb[i] ? orc_fene_d2(rr, tr.r0[k], p->k_fene, p->R0)
                                                      : orc_native_d2(rr, tr.r0[k], p->eps_h);
                sum += rr * fabs(d2);
            }
            for (int64_t k = r.ptr[i]; k < r.ptr[i + 1]; ++k) {
                double rr = dist(x, i, r.col[k]);
                sum += rr * fabs(orc_repulsive_d2(rr, p->sigma, p->eps_l));
            }
            int64_t t = traj_of(s, i);
            for (int32_t q = 0; q < s->n_pull; ++q) {
                if (s->pull_traj[q] != t || s->pull_res[q] != i)
                    continue;
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double d = s->pull_anchor0[3 * q + a] + s->pull_v[3 * q + a] * tn - x[3 * i + a];
                    d2 += d * d;
                }
                sum += s->pull_kappa[q] * sqrt(d2);
            }
            if (s->has_tip) {
                double r2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double d = x[3 * i + a] - (s->tip_c0[a] + s->tip_v[a] * tn);
                    r2 += d * d;
                }
                double rr = sqrt(r2), gap = rr - s->tip_radius;
                if (gap > 0.0)
                    sum += rr * orc_repulsive_d2(gap, s->tip_sigma, s->tip_eps);
            }
            K[i] = sum;
        }
    }
    free(r.ptr);
    free(r.col);
    topo_rows_free(&tr);
    excl_free(&e);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Force-spectroscopy observables (the pulling protocol of Section IV.B)    */
/* ------------------------------------------------------------------------ */

/* Running average: out[k] = (y[k] + ... + y[k + w - 1]) / w, k = 0 .. n - w,
 * each window summed on its own. */
int orc_running_average(const double *y, int64_t n, int32_t w, double *out)
{
    if (w < 1 || n < w)
        return ORC_E_ARG;
    for (int64_t k = 0; k + w <= n; ++k) {
        double s = 0.0;
        for (int32_t j = 0; j < w; ++j)
            s += y[k + j];
        out[k] = s / (double)w;
    }
    return ORC_OK;
}

/* Peak force: the largest w-point running average and its first window. */
int orc_peak_force(const double *f, int64_t n, int32_t w, double *peak, int64_t *index)
{
    if (w < 1 || n < w)
        return ORC_E_ARG;
    double *a = (double *)malloc((size_t)(n - w + 1) * sizeof(double));
    if (!a)
        return ORC_E_ARG;
    orc_running_average(f, n, w, a);
    int64_t best = 0;
    for (int64_t k = 1; k <= n - w; ++k)
        if (a[k] > a[best])
            best = k;
    *peak = a[best];
    *index = best;
    free(a);
    return ORC_OK;
}

/* End-to-end distance |x_last - x_first| of every trajectory (0 for fewer
 * than two residues). */
void orc_end_to_end(const orc_system *s, const double *x, double *R)
{
    for (int64_t t = 0; t < s->n_traj; ++t) {
        int64_t a = s->res_offsets[t], b = s->res_offsets[t + 1];
        R[t] = (b - a < 2) ? 0.0 : dist(x, b - 1, a);
    }
}
