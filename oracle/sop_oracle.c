/*
 * FP64 CPU oracle for overdamped Langevin dynamics of the Self Organized
 * Polymer (SOP) model -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg call
 * this code.  It shares nothing with the HIP library: no headers, no helpers,
 * no tables.  It is written to be read against the paper (Zhmurov, Dima,
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
 * Readings of the paper that this code takes (each is listed with its reason
 * in the design notes of the repository):
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
