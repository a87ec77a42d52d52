// HIP kernels for gfx950: Verlet-list rebuild on a wrapped cell grid, the
// fused per-step kernel (SOP forces of Eq. 1 over bonds, natives and the
// list; Philox4x32-10 Box-Muller noise; first-order overdamped update of
// Eq. 2 / Algorithm 7 with compensated single-precision positions), and the
// double-precision energy reduction.
#include <algorithm>

#include "sop_internal.hpp"

namespace sop {

namespace {

constexpr int WG = 256;       // threads per workgroup (4 wave64)
constexpr int CHUNK = 1024;   // candidates staged in LDS per pass of the fill

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Gaussian mapping
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, unsigned k0, unsigned k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const unsigned hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const unsigned hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform in (0,1) from the top 23 bits: exact in single precision.
__device__ __forceinline__ float unit23(unsigned w)
{
    return (static_cast<float>(w >> 9) + 0.5f) * 0x1p-23f;
}

// Box-Muller: axis 0/1 = radius(u0) * (cos, sin)(2 pi u1), axis 2 =
// radius(u2) * cos(2 pi u3).
__device__ __forceinline__ float gaussian_axis(const uint4 &w, int axis)
{
    const float ur = unit23(axis < 2 ? w.x : w.z);
    const float ua = unit23(axis < 2 ? w.y : w.w);
    const float rad = sqrtf(-2.0f * logf(ur));
    float s, c;
    sincospif(2.0f * ua, &s, &c);
    return rad * (axis == 1 ? s : c);
}

__device__ __forceinline__ float comp(const float4 &v, int a)
{
    return a == 0 ? v.x : (a == 1 ? v.y : v.z);
}

// Cell index along one axis: floor(x / edge) shifted by the trajectory's
// offset and wrapped into [0, n), so every position has a valid cell.
__device__ __forceinline__ int wrap_cell(float x, float inv_cell, int off, int n)
{
    float v = floorf(x * inv_cell);
    if (!(v == v))
        v = 0.0f;  // NaN positions are flagged elsewhere; keep the index in range
    v = fminf(fmaxf(v, -1.0e9f), 1.0e9f);
    int c = (static_cast<int>(v) + off) % n;
    return c < 0 ? c + n : c;
}

// The list predicate in single precision without contraction:
// fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)) < rc2, dx = fl(xi - xj).
__device__ __forceinline__ bool within_cutoff(float4 a, float4 b, float rc2)
{
#pragma clang fp contract(off)
    const float dx = a.x - b.x;
    const float dy = a.y - b.y;
    const float dz = a.z - b.z;
    const float xx = dx * dx;
    const float yy = dy * dy;
    const float zz = dz * dz;
    const float s = xx + yy;
    const float d2 = s + zz;
    return d2 < rc2;
}

// Pair difference from compensated positions: (hi_i - hi_j) + (lo_i - lo_j).
__device__ __forceinline__ float3 pair_delta(const float4 &hi, const float4 &lo, const float4 &hj,
                                             const float4 &lj)
{
    return make_float3((hi.x - hj.x) + (lo.x - lj.x), (hi.y - hj.y) + (lo.y - lj.y),
                       (hi.z - hj.z) + (lo.z - lj.z));
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Verlet-list rebuild: clear cell counts -> bin into fixed-capacity cells ->
// one workgroup per cell fills the rows of its residues
// ---------------------------------------------------------------------------
__global__ void k_clear(int *__restrict__ a, int n, int *__restrict__ n_occupied)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        a[i] = 0;
    if (i == 0)
        *n_occupied = 0;
}

// Also advances the step counter of graph replays (once per rebuild) when
// step_base is given.
__global__ void k_bin(const float4 *__restrict__ pos, int n, GridDev g, const int4 *__restrict__ traj_cell,
                      int *__restrict__ count, float4 *__restrict__ cells, int *__restrict__ occupied,
                      int *__restrict__ n_occupied, unsigned *__restrict__ err,
                      long long *step_base, long long *step_next, int period)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && step_base) {
        const long long nb = *step_next;
        *step_base = nb;
        *step_next = nb + period;
    }
    if (i >= n)
        return;
    const float4 p = pos[2 * i];
    if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z))
        atomicOr(err, ERR_NONFINITE);
    const int4 off = traj_cell[__float_as_int(pos[2 * i + 1].w)];
    const int cx = wrap_cell(p.x, g.inv_cell, off.x, g.gx);
    const int cy = wrap_cell(p.y, g.inv_cell, off.y, g.gy);
    const int cz = wrap_cell(p.z, g.inv_cell, off.z, g.gz);
    const int c = cx + g.gx * (cy + g.gy * cz);
    const int slot = atomicAdd(&count[c], 1);
    if (slot == 0)
        occupied[atomicAdd(n_occupied, 1)] = c;  // order varies; each cell is filled on its own
    if (slot < CELL_CAP)
        cells[(size_t)c * CELL_CAP + slot] = make_float4(p.x, p.y, p.z, __int_as_float(i));
    else
        atomicOr(err, ERR_CELL);
}

struct FillArgs {
    const int *occupied;
    const int *n_occupied;
    const int *count;
    const float4 *cells;
    const int *traj_lo;
    const int *traj_hi;
    const int2 *trow;
    const float2 *tent;
    int *list;
    int *list_cnt;
    unsigned *err;
    GridDev g;
    float rc2;
    int cap;
};

// Rows of every residue of one cell.  Candidates are the residues of the 27
// surrounding cells, visited in a fixed cell order with each cell's residues
// ranked by id in LDS; a wave appends the passing candidates of one residue
// in that order (ballot + prefix count), so rows are deterministic.
template <int LANES>
__global__ __launch_bounds__(WG) void k_fill(FillArgs a)
{
    constexpr int G = 64 / LANES;
    __shared__ float4 own[CELL_CAP];
    __shared__ int own_cnt[CELL_CAP];
    __shared__ float4 raw[CHUNK];
    __shared__ float4 cand[CHUNK];
    __shared__ int seg_cell[27];
    __shared__ int seg_n[27];
    __shared__ int seg_off[28];

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const GridDev g = a.g;
    const int n_occ = *a.n_occupied;
    for (int oc = blockIdx.x; oc < n_occ; oc += gridDim.x) {
    const int c = a.occupied[oc];
    const int m = min(a.count[c], CELL_CAP);
    if (t < 27) {
        const int cx = c % g.gx, cy = (c / g.gx) % g.gy, cz = c / (g.gx * g.gy);
        const int xx = (cx + (t % 3) - 1 + g.gx) % g.gx;
        const int yy = (cy + (t / 3) % 3 - 1 + g.gy) % g.gy;
        const int zz = (cz + t / 9 - 1 + g.gz) % g.gz;
        const int nc = xx + g.gx * (yy + g.gy * zz);
        seg_cell[t] = nc;
        seg_n[t] = min(a.count[nc], CELL_CAP);
    }
    if (t < m)
        raw[t] = a.cells[(size_t)c * CELL_CAP + t];
    __syncthreads();
    if (t < m) {
        const int id = __float_as_int(raw[t].w);
        int rank = 0;
        for (int k = 0; k < m; ++k)
            rank += __float_as_int(raw[k].w) < id;
        own[rank] = raw[t];
        own_cnt[rank] = 0;
    }
    if (t == 0) {
        int o = 0;
        for (int k = 0; k < 27; ++k) {
            seg_off[k] = o;
            o += seg_n[k];
        }
        seg_off[27] = o;
    }
    __syncthreads();

    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int s0 = 0;
    while (s0 < 27) {
        int s1 = s0 + 1;
        while (s1 < 27 && seg_off[s1 + 1] - seg_off[s0] <= CHUNK)
            ++s1;
        const int base = seg_off[s0];
        const int tot = seg_off[s1] - base;
        for (int q = t; q < tot; q += WG) {
            int sg = s0;
            while (seg_off[sg + 1] - base <= q)
                ++sg;
            raw[q] = a.cells[(size_t)seg_cell[sg] * CELL_CAP + (q - (seg_off[sg] - base))];
        }
        __syncthreads();
        for (int q = t; q < tot; q += WG) {
            int sg = s0;
            while (seg_off[sg + 1] - base <= q)
                ++sg;
            const int so = seg_off[sg] - base, sn = seg_n[sg];
            const int id = __float_as_int(raw[q].w);
            int rank = 0;
            for (int k = 0; k < sn; ++k)
                rank += __float_as_int(raw[so + k].w) < id;
            cand[so + rank] = raw[q];
        }
        __syncthreads();
        for (int mi = wave; mi < m; mi += WG / 64) {
            const float4 p = own[mi];
            const int i = __builtin_amdgcn_readfirstlane(__float_as_int(p.w));
            const int tlo = a.traj_lo[i], thi = a.traj_hi[i];
            const int2 row = a.trow[i];
            const int nex = (row.y & 4095) + (row.y >> 12);
            // bonded and native partners of i, one per lane (the first 64)
            const int pv = lane < nex ? __float_as_int(a.tent[row.x + lane].x) : -1;
            int *rowp = a.list + (size_t)(i / G) * a.cap * G + (i % G) * LANES;
            int cnt = own_cnt[mi];
            for (int q0 = 0; q0 < tot; q0 += 64) {
                const int q = q0 + lane;
                bool ok = false;
                int j = -1;
                if (q < tot) {
                    const float4 cq = cand[q];
                    j = __float_as_int(cq.w);
                    ok = j != i && j >= tlo && j < thi && within_cutoff(p, cq, a.rc2);
                }
                if (__ballot(ok)) {
                    const int ne = min(nex, 64);
                    for (int e = 0; e < ne; ++e)
                        ok = ok && (j != __builtin_amdgcn_readlane(pv, e));
                    for (int e = 64; e < nex; ++e)
                        ok = ok && (__float_as_int(a.tent[row.x + e].x) != j);
                }
                const unsigned long long mask = __ballot(ok);
                if (ok) {
                    const int at = cnt + __popcll(mask & below);
                    if (at < a.cap)
                        rowp[(at / LANES) * 64 + (at % LANES)] = j;
                }
                cnt += __popcll(mask);
            }
            if (lane == 0)
                own_cnt[mi] = cnt;
        }
        __syncthreads();
        s0 = s1;
    }
    for (int mi = t; mi < m; mi += WG) {
        const int i = __float_as_int(own[mi].w);
        a.list_cnt[i] = own_cnt[mi];
        if (own_cnt[mi] > a.cap)
            atomicOr(a.err, ERR_OVERFLOW);
    }
    __syncthreads();  // LDS is reused by the next cell
    }
}

// ---------------------------------------------------------------------------
// Fused step: forces -> (noise -> compensated update) | force output
// ---------------------------------------------------------------------------
struct StepArgs {
    const float4 *pin;
    float4 *pout;
    const int2 *trow;
    const float2 *tent;
    const int *list;
    const int *list_cnt;
    const unsigned *stream_ids;
    const int *pull_slot;
    const PullDev *pulls;
    double *res_energy;
    float4 *fout;
    unsigned *err;
    const long long *step_base;
    long long step_off;
    int n, cap, has_pull, n_waves;
    StepConsts c;
    TipDev tip;
};

// Per-residue force and, on energy steps, double energy/virial sums.
struct Acc {
    float fx = 0.f, fy = 0.f, fz = 0.f;
    double e_b = 0.0, e_n = 0.0, e_r = 0.0, vir = 0.0;
};

// eps_l (sigma/r)^6 between residue (hi, lo) and a listed partner.
__device__ __forceinline__ void add_repulsive(Acc &A, const float4 &hi, const float4 &lo,
                                              const float4 &hj, const float4 &lj, float sg2,
                                              float el, float el6, bool ENERGY)
{
    const float3 d = pair_delta(hi, lo, hj, lj);
    const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    const float ir2 = fast_rcp(r2);
    const float s = sg2 * ir2;
    const float q = s * s * s;
    const float coef = el6 * q * ir2;
    A.fx += coef * d.x;
    A.fy += coef * d.y;
    A.fz += coef * d.z;
    if (ENERGY) {
        A.e_r += (double)(el * q);
        A.vir += (double)(el6 * q);
    }
}

template <int LANES, bool ENERGY, int MODE>
__global__ __launch_bounds__(WG) void k_step(StepArgs a)
{
    constexpr int G = 64 / LANES;
    const int lane = threadIdx.x & 63;
    // XCD-aware order: consecutive residue blocks stay on one XCD's L2.
    const int per = gridDim.x >> 3;
    const int blk = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int wave = blk * (WG / 64) + (threadIdx.x >> 6);
    if (wave >= a.n_waves)
        return;
    const int g = lane / LANES, l = lane % LANES;
    const int r = wave * G + g;
    if (r >= a.n)
        return;

    const float4 hi = a.pin[2 * r];
    const float4 lo = a.pin[2 * r + 1];
    Acc A;
    bool broken = false;

    const int2 row = a.trow[r];
    const int nb = row.y & 4095, nn = row.y >> 12;
    const float kf = a.c.k_fene, inv_R0sq = a.c.inv_R0sq;
    // FENE bonds
    for (int p = l; p < nb; p += LANES) {
        const float2 t = a.tent[row.x + p];
        const int j = __float_as_int(t.x);
        const float3 d = pair_delta(hi, lo, a.pin[2 * j], a.pin[2 * j + 1]);
        const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
        const float rr = __builtin_amdgcn_sqrtf(r2);
        const float dl = rr - t.y;
        float x = 1.0f - dl * dl * inv_R0sq;
        if (!(x > 0.0f)) {
            broken = true;
            x = 1.0f;
        }
        const float coef = -kf * dl * fast_rcp(x * rr);
        A.fx += coef * d.x;
        A.fy += coef * d.y;
        A.fz += coef * d.z;
        if (ENERGY) {
            const double dd = (double)dl;
            const double R0sq = (double)a.c.R0sq;
            A.e_b += -0.5 * (double)kf * R0sq * log1p(-dd * dd / R0sq);
            A.vir += -(double)rr * (double)kf * dd / (1.0 - dd * dd / R0sq);
        }
    }
    // native contacts
    const float eh = a.c.eps_h, eh12 = 12.0f * eh;
    for (int p = nb + l; p < nb + nn; p += LANES) {
        const float2 t = a.tent[row.x + p];
        const int j = __float_as_int(t.x);
        const float3 d = pair_delta(hi, lo, a.pin[2 * j], a.pin[2 * j + 1]);
        const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
        const float ir2 = fast_rcp(r2);
        const float s = t.y * t.y * ir2;
        const float q = s * s * s;
        const float coef = eh12 * (q * q - q) * ir2;
        A.fx += coef * d.x;
        A.fy += coef * d.y;
        A.fz += coef * d.z;
        if (ENERGY) {
            A.e_n += (double)(eh * (q * q - 2.0f * q));
            A.vir += (double)(eh12 * (q * q - q));
        }
    }
    // repulsive list, four partners per iteration to keep gathers in flight
    const float el = a.c.eps_l, el6 = 6.0f * el, sg2 = a.c.sigma2;
    const int cnt = min(a.list_cnt[r], a.cap);
    const int nk = cnt > l ? (cnt - l + LANES - 1) / LANES : 0;
    const int *lp = a.list + (size_t)wave * a.cap * G + g * LANES + l;
    int k = 0;
    for (; k + 4 <= nk; k += 4) {
        const int j0 = lp[(k + 0) * 64], j1 = lp[(k + 1) * 64];
        const int j2 = lp[(k + 2) * 64], j3 = lp[(k + 3) * 64];
        const float4 h0 = a.pin[2 * j0], l0 = a.pin[2 * j0 + 1];
        const float4 h1 = a.pin[2 * j1], l1 = a.pin[2 * j1 + 1];
        const float4 h2 = a.pin[2 * j2], l2 = a.pin[2 * j2 + 1];
        const float4 h3 = a.pin[2 * j3], l3 = a.pin[2 * j3 + 1];
        add_repulsive(A, hi, lo, h0, l0, sg2, el, el6, ENERGY);
        add_repulsive(A, hi, lo, h1, l1, sg2, el, el6, ENERGY);
        add_repulsive(A, hi, lo, h2, l2, sg2, el, el6, ENERGY);
        add_repulsive(A, hi, lo, h3, l3, sg2, el, el6, ENERGY);
    }
    for (; k < nk; ++k) {
        const int j = lp[k * 64];
        add_repulsive(A, hi, lo, a.pin[2 * j], a.pin[2 * j + 1], sg2, el, el6, ENERGY);
    }

    // external terms (one lane per residue), positions in double
    double e_x = 0.0, f_rep = 0.0;
    if (l == 0 && (a.has_pull || a.tip.on)) {
        const long long step = (a.step_base ? *a.step_base : 0) + a.step_off;
        const double tn = (double)step * a.c.h;
        const double px = (double)hi.x + (double)lo.x;
        const double py = (double)hi.y + (double)lo.y;
        const double pz = (double)hi.z + (double)lo.z;
        if (a.has_pull) {
            const int sl = a.pull_slot[r];
            if (sl >= 0) {
                const PullDev pd = a.pulls[sl];
                const double dx = pd.anchor0[0] + pd.v[0] * tn - px;
                const double dy = pd.anchor0[1] + pd.v[1] * tn - py;
                const double dz = pd.anchor0[2] + pd.v[2] * tn - pz;
                A.fx += (float)(pd.kappa * dx);
                A.fy += (float)(pd.kappa * dy);
                A.fz += (float)(pd.kappa * dz);
                if (ENERGY) {
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    e_x += 0.5 * pd.kappa * d2;
                    f_rep += pd.has_dir ? pd.kappa * (dx * pd.vhat[0] + dy * pd.vhat[1] + dz * pd.vhat[2])
                                        : pd.kappa * sqrt(d2);
                }
            }
        }
        if (a.tip.on) {
            const TipDev &tp = a.tip;
            const float dx = (float)(px - (tp.c0[0] + tp.v[0] * tn));
            const float dy = (float)(py - (tp.c0[1] + tp.v[1] * tn));
            const float dz = (float)(pz - (tp.c0[2] + tp.v[2] * tn));
            const float rr = sqrtf(dx * dx + dy * dy + dz * dz);
            const float gap = rr - (float)tp.radius;
            if (!(gap > 0.0f)) {
                atomicOr(a.err, ERR_TIP);
            } else {
                const float sg = (float)tp.sigma / gap;
                const float s3 = sg * sg * sg;
                const float q = s3 * s3;
                const float mag = 6.0f * (float)tp.eps * q / gap;
                const float cx = mag * dx / rr, cy = mag * dy / rr, cz = mag * dz / rr;
                A.fx += cx;
                A.fy += cy;
                A.fz += cz;
                if (ENERGY) {
                    e_x += tp.eps * (double)q;
                    if (tp.has_dir)
                        f_rep += (double)cx * tp.vhat[0] + (double)cy * tp.vhat[1] +
                                 (double)cz * tp.vhat[2];
                }
            }
        }
    }
    if (broken)
        atomicOr(a.err, ERR_FENE);

    // combine the LANES partial sums of one residue (butterfly)
    float fx = A.fx, fy = A.fy, fz = A.fz;
#pragma unroll
    for (int m = LANES / 2; m >= 1; m >>= 1) {
        fx += __shfl_xor(fx, m, 64);
        fy += __shfl_xor(fy, m, 64);
        fz += __shfl_xor(fz, m, 64);
        if (ENERGY) {
            A.e_b += __shfl_xor(A.e_b, m, 64);
            A.e_n += __shfl_xor(A.e_n, m, 64);
            A.e_r += __shfl_xor(A.e_r, m, 64);
            A.vir += __shfl_xor(A.vir, m, 64);
        }
    }
    if (ENERGY && l == 0) {
        double *er = a.res_energy + (size_t)r * RES_E;
        // each internal pair appears in both partners' rows
        er[0] = 0.5 * A.e_b;
        er[1] = 0.5 * A.e_n;
        er[2] = 0.5 * A.e_r;
        er[3] = e_x;
        er[4] = 0.5 * A.vir;
        er[5] = f_rep;
    }
    if (MODE == 1) {
        if (l == 0)
            a.fout[r] = make_float4(fx, fy, fz, 0.0f);
        return;
    }

    // noise and compensated update; lane l handles axes l, l+LANES, ...
    const long long step = (a.step_base ? *a.step_base : 0) + a.step_off;
    const unsigned tag = __float_as_uint(hi.w);
    const bool fixed = (tag >> 31) != 0;
    const unsigned local = tag & 0x7fffffffu;
    const unsigned stream = a.stream_ids[__float_as_int(lo.w)];
    const uint4 w = philox10(make_uint4(local, stream, (unsigned)step, (unsigned)((unsigned long long)step >> 32)),
                             a.c.key0, a.c.key1);
    float *ho = reinterpret_cast<float *>(a.pout + 2 * r);
    float *lw = reinterpret_cast<float *>(a.pout + 2 * r + 1);
    for (int ax = l; ax < 3; ax += LANES) {
        const float f = ax == 0 ? fx : (ax == 1 ? fy : fz);
        const float h0 = comp(hi, ax), l0 = comp(lo, ax);
        float nh = h0, nl = l0;
        if (!fixed) {
            const float delta = a.c.c_drift * f + a.c.c_noise * gaussian_axis(w, ax);
            // TwoSum(h0, delta + l0): exact error term kept in the low word
            const float y = delta + l0;
            const float t = h0 + y;
            const float bp = t - h0;
            const float ap = t - bp;
            nl = (h0 - ap) + (y - bp);
            nh = t;
        }
        if (!isfinite(nh) || !isfinite(nl))
            atomicOr(a.err, ERR_NONFINITE);
        ho[ax] = nh;
        lw[ax] = nl;
    }
}

// ---------------------------------------------------------------------------
// Batched ensemble: one workgroup per pack of whole trajectories, positions
// resident in LDS for n_steps steps; the list of each residue is rebuilt in
// LDS from all residues of its trajectory every list_every steps.
// ---------------------------------------------------------------------------
struct BatchArgs {
    const float4 *pin;
    float4 *pout;
    const int2 *trow;
    const float2 *tent;
    const int *pack_res;      // first residue of each pack (n_packs + 1)
    const int *traj_lo;
    const int *traj_hi;
    const unsigned *stream_ids;
    const int *pull_slot;
    const PullDev *pulls;
    unsigned short *list;     // pack p: entry k of residue base+t at base*cap + k*n + t
    int *list_cnt;
    double *energy;
    double *f_ext;
    float4 *fout;
    unsigned *err;
    const long long *step_base;
    long long step_off;
    long long energy_every;
    int n_steps, list_every, stale, cap, has_pull;
    StepConsts c;
    TipDev tip;
    float rc2;
};

// Deterministic per-trajectory sum of one value per residue held in `red`;
// the first residue of each trajectory adds its trajectory's values in order.
__device__ __forceinline__ double traj_sum(double *red, int t, bool act, double v, int tlo, int thi)
{
    red[t] = act ? v : 0.0;
    __syncthreads();
    double s = 0.0;
    if (act && t == tlo)
        for (int u = tlo; u < thi; ++u)
            s += red[u];
    __syncthreads();
    return s;
}

template <int WGS, int MODE>
__global__ __launch_bounds__(WGS) void k_batch(BatchArgs a)
{
    __shared__ float4 sh[2 * WGS];
    __shared__ double red[WGS];
    const int p = blockIdx.x;
    const int base = a.pack_res[p];
    const int n = a.pack_res[p + 1] - base;
    const int t = threadIdx.x;
    const bool act = t < n;
    const int i = base + t;

    float4 hi = make_float4(0.f, 0.f, 0.f, 0.f), lo = hi;
    int tlo = 0, thi = 0;
    int2 row = make_int2(0, 0);
    int cnt = 0;
    if (act) {
        hi = a.pin[2 * i];
        lo = a.pin[2 * i + 1];
        tlo = a.traj_lo[i] - base;
        thi = a.traj_hi[i] - base;
        row = a.trow[i];
        cnt = a.list_cnt[i];
        sh[2 * t] = hi;
        sh[2 * t + 1] = lo;
    }
    __syncthreads();
    const int nb = row.y & 4095, nn = row.y >> 12;
    unsigned short *lrow = a.list + (size_t)base * a.cap + t;
    const long long s0 = (a.step_base ? *a.step_base : 0) + a.step_off;
    const float kf = a.c.k_fene, inv_R0sq = a.c.inv_R0sq;
    const float eh = a.c.eps_h, eh12 = 12.0f * eh;
    const float el = a.c.eps_l, el6 = 6.0f * el, sg2 = a.c.sigma2;
    const unsigned tag = __float_as_uint(hi.w);
    const bool fixed = (tag >> 31) != 0;
    const unsigned local = tag & 0x7fffffffu;
    const int traj = __float_as_int(lo.w);
    const unsigned stream = act ? a.stream_ids[traj] : 0u;

    for (int q = 0; q < a.n_steps; ++q) {
        const long long step = s0 + q;
        if ((q == 0 && a.stale) || step % a.list_every == 0) {
            if (act) {
                cnt = 0;
                for (int j = tlo; j < thi; ++j) {
                    if (j == t || !within_cutoff(hi, sh[2 * j], a.rc2))
                        continue;
                    bool ex = false;
                    for (int e = 0; e < nb + nn; ++e)
                        ex |= (__float_as_int(a.tent[row.x + e].x) - base) == j;
                    if (ex)
                        continue;
                    if (cnt < a.cap)
                        lrow[(size_t)cnt * n] = (unsigned short)j;
                    ++cnt;
                }
                if (cnt > a.cap)
                    atomicOr(a.err, ERR_OVERFLOW);
                a.list_cnt[i] = cnt;
            }
        }
        Acc A;  // energy sums are only accumulated on record steps
        const bool rec = MODE == 1 || (a.energy_every > 0 && step % a.energy_every == 0);
        bool broken = false;
        double e_x = 0.0, f_rep = 0.0;
        if (act) {
            for (int e = 0; e < nb; ++e) {
                const float2 tt = a.tent[row.x + e];
                const int j = __float_as_int(tt.x) - base;
                const float3 d = pair_delta(hi, lo, sh[2 * j], sh[2 * j + 1]);
                const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
                const float rr = __builtin_amdgcn_sqrtf(r2);
                const float dl = rr - tt.y;
                float x = 1.0f - dl * dl * inv_R0sq;
                if (!(x > 0.0f)) {
                    broken = true;
                    x = 1.0f;
                }
                const float coef = -kf * dl * fast_rcp(x * rr);
                A.fx += coef * d.x;
                A.fy += coef * d.y;
                A.fz += coef * d.z;
                if (rec) {
                    const double dd = (double)dl;
                    const double R0sq = (double)a.c.R0sq;
                    A.e_b += -0.5 * (double)kf * R0sq * log1p(-dd * dd / R0sq);
                    A.vir += -(double)rr * (double)kf * dd / (1.0 - dd * dd / R0sq);
                }
            }
            for (int e = nb; e < nb + nn; ++e) {
                const float2 tt = a.tent[row.x + e];
                const int j = __float_as_int(tt.x) - base;
                const float3 d = pair_delta(hi, lo, sh[2 * j], sh[2 * j + 1]);
                const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
                const float ir2 = fast_rcp(r2);
                const float s = tt.y * tt.y * ir2;
                const float qq = s * s * s;
                const float coef = eh12 * (qq * qq - qq) * ir2;
                A.fx += coef * d.x;
                A.fy += coef * d.y;
                A.fz += coef * d.z;
                if (rec) {
                    A.e_n += (double)(eh * (qq * qq - 2.0f * qq));
                    A.vir += (double)(eh12 * (qq * qq - qq));
                }
            }
            const int m = min(cnt, a.cap);
            int k = 0;
            for (; k + 4 <= m; k += 4) {
                const int j0 = lrow[(size_t)(k + 0) * n], j1 = lrow[(size_t)(k + 1) * n];
                const int j2 = lrow[(size_t)(k + 2) * n], j3 = lrow[(size_t)(k + 3) * n];
                add_repulsive(A, hi, lo, sh[2 * j0], sh[2 * j0 + 1], sg2, el, el6, rec);
                add_repulsive(A, hi, lo, sh[2 * j1], sh[2 * j1 + 1], sg2, el, el6, rec);
                add_repulsive(A, hi, lo, sh[2 * j2], sh[2 * j2 + 1], sg2, el, el6, rec);
                add_repulsive(A, hi, lo, sh[2 * j3], sh[2 * j3 + 1], sg2, el, el6, rec);
            }
            for (; k < m; ++k) {
                const int j = lrow[(size_t)k * n];
                add_repulsive(A, hi, lo, sh[2 * j], sh[2 * j + 1], sg2, el, el6, rec);
            }
            if (a.has_pull || a.tip.on) {
                const double tn = (double)step * a.c.h;
                const double px = (double)hi.x + (double)lo.x;
                const double py = (double)hi.y + (double)lo.y;
                const double pz = (double)hi.z + (double)lo.z;
                if (a.has_pull) {
                    const int sl = a.pull_slot[i];
                    if (sl >= 0) {
                        const PullDev pd = a.pulls[sl];
                        const double dx = pd.anchor0[0] + pd.v[0] * tn - px;
                        const double dy = pd.anchor0[1] + pd.v[1] * tn - py;
                        const double dz = pd.anchor0[2] + pd.v[2] * tn - pz;
                        A.fx += (float)(pd.kappa * dx);
                        A.fy += (float)(pd.kappa * dy);
                        A.fz += (float)(pd.kappa * dz);
                        if (rec) {
                            const double d2 = dx * dx + dy * dy + dz * dz;
                            e_x += 0.5 * pd.kappa * d2;
                            f_rep += pd.has_dir ? pd.kappa * (dx * pd.vhat[0] + dy * pd.vhat[1] + dz * pd.vhat[2])
                                                : pd.kappa * sqrt(d2);
                        }
                    }
                }
                if (a.tip.on) {
                    const TipDev &tp = a.tip;
                    const float dx = (float)(px - (tp.c0[0] + tp.v[0] * tn));
                    const float dy = (float)(py - (tp.c0[1] + tp.v[1] * tn));
                    const float dz = (float)(pz - (tp.c0[2] + tp.v[2] * tn));
                    const float rr = sqrtf(dx * dx + dy * dy + dz * dz);
                    const float gap = rr - (float)tp.radius;
                    if (!(gap > 0.0f)) {
                        atomicOr(a.err, ERR_TIP);
                    } else {
                        const float sg = (float)tp.sigma / gap;
                        const float s3 = sg * sg * sg;
                        const float qq = s3 * s3;
                        const float mag = 6.0f * (float)tp.eps * qq / gap;
                        const float cx = mag * dx / rr, cy = mag * dy / rr, cz = mag * dz / rr;
                        A.fx += cx;
                        A.fy += cy;
                        A.fz += cz;
                        if (rec) {
                            e_x += tp.eps * (double)qq;
                            if (tp.has_dir)
                                f_rep += (double)cx * tp.vhat[0] + (double)cy * tp.vhat[1] +
                                         (double)cz * tp.vhat[2];
                        }
                    }
                }
            }
            if (broken)
                atomicOr(a.err, ERR_FENE);
        }
        if (rec) {
            // each internal pair appears in both partners' rows
            const double vals[RES_E] = {0.5 * A.e_b, 0.5 * A.e_n, 0.5 * A.e_r, e_x, 0.5 * A.vir, f_rep};
#pragma unroll
            for (int kk = 0; kk < RES_E; ++kk) {
                const double sum = traj_sum(red, t, act, vals[kk], tlo, thi);
                if (act && t == tlo) {
                    if (kk < SOP_NTERMS)
                        a.energy[(size_t)traj * SOP_NTERMS + kk] = sum;
                    else
                        a.f_ext[traj] = sum;
                }
            }
        }
        if (MODE == 1) {
            if (act)
                a.fout[i] = make_float4(A.fx, A.fy, A.fz, 0.0f);
            return;
        }
        float4 nh4 = hi, nl4 = lo;
        if (act) {
            const uint4 w = philox10(make_uint4(local, stream, (unsigned)step,
                                                (unsigned)((unsigned long long)step >> 32)),
                                     a.c.key0, a.c.key1);
            float nh[3], nl[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float f = ax == 0 ? A.fx : (ax == 1 ? A.fy : A.fz);
                const float h0 = comp(hi, ax), l0 = comp(lo, ax);
                nh[ax] = h0;
                nl[ax] = l0;
                if (!fixed) {
                    const float delta = a.c.c_drift * f + a.c.c_noise * gaussian_axis(w, ax);
                    const float y = delta + l0;
                    const float tt = h0 + y;
                    const float bp = tt - h0;
                    const float ap = tt - bp;
                    nl[ax] = (h0 - ap) + (y - bp);
                    nh[ax] = tt;
                }
                if (!isfinite(nh[ax]) || !isfinite(nl[ax]))
                    atomicOr(a.err, ERR_NONFINITE);
            }
            nh4 = make_float4(nh[0], nh[1], nh[2], hi.w);
            nl4 = make_float4(nl[0], nl[1], nl[2], lo.w);
        }
        __syncthreads();
        if (act) {
            sh[2 * t] = nh4;
            sh[2 * t + 1] = nl4;
        }
        hi = nh4;
        lo = nl4;
        __syncthreads();
    }
    if (MODE == 0 && act) {
        a.pout[2 * i] = hi;
        a.pout[2 * i + 1] = lo;
    }
}

__global__ void k_add_step(long long *base, long long k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *base += k;
}

// One workgroup per trajectory: double sums of the per-residue records.
__global__ __launch_bounds__(WG) void k_reduce_energy(const double *__restrict__ res_energy,
                                                      const long long *__restrict__ offs,
                                                      double *__restrict__ energy,
                                                      double *__restrict__ f_ext)
{
    __shared__ double part[WG / 64][RES_E];
    const int t = blockIdx.x;
    const long long a = offs[t], b = offs[t + 1];
    double s[RES_E] = {0, 0, 0, 0, 0, 0};
    for (long long i = a + threadIdx.x; i < b; i += WG)
#pragma unroll
        for (int k = 0; k < RES_E; ++k)
            s[k] += res_energy[i * RES_E + k];
#pragma unroll
    for (int k = 0; k < RES_E; ++k)
        for (int m = 32; m >= 1; m >>= 1)
            s[k] += __shfl_xor(s[k], m, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < RES_E; ++k)
            part[threadIdx.x >> 6][k] = s[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < RES_E; ++k) {
            double v = 0.0;
            for (int w = 0; w < WG / 64; ++w)
                v += part[w][k];
            if (k < SOP_NTERMS)
                energy[(size_t)t * SOP_NTERMS + k] = v;
            else
                f_ext[t] = v;
        }
    }
}

// Philox words and Gaussians of every residue at one step, computed with the
// same device functions as the step kernel.
__global__ void k_noise(const float4 *__restrict__ pos, int n, const unsigned *__restrict__ stream_ids,
                        unsigned k0, unsigned k1, long long step, uint4 *__restrict__ words,
                        float4 *__restrict__ g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const unsigned local = __float_as_uint(pos[2 * i].w) & 0x7fffffffu;
    const unsigned stream = stream_ids[__float_as_int(pos[2 * i + 1].w)];
    const uint4 w = philox10(make_uint4(local, stream, (unsigned)step,
                                        (unsigned)((unsigned long long)step >> 32)), k0, k1);
    words[i] = w;
    g[i] = make_float4(gaussian_axis(w, 0), gaussian_axis(w, 1), gaussian_axis(w, 2), 0.0f);
}

__global__ void k_set_step(long long *dst, long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dst = v;
}

inline int blocks_for(long long n, int per) { return (int)((n + per - 1) / per); }

template <int LANES>
void fill_lanes(const FillArgs &f, int n_cells, hipStream_t s)
{
    // occupied cells are spread over a bounded grid of workgroups
    hipLaunchKernelGGL(k_fill<LANES>, dim3(std::min(n_cells, 2048)), dim3(WG), 0, s, f);
}

template <int LANES, bool ENERGY, int MODE>
void step_lanes(const StepArgs &a, hipStream_t s)
{
    constexpr int G = 64 / LANES;
    StepArgs x = a;
    x.n_waves = blocks_for(a.n, G);
    int blocks = blocks_for(x.n_waves, WG / 64);
    blocks = ((blocks + 7) / 8) * 8;
    hipLaunchKernelGGL((k_step<LANES, ENERGY, MODE>), dim3(blocks), dim3(WG), 0, s, x);
}

template <bool ENERGY, int MODE>
void step_dispatch(int lanes, const StepArgs &a, hipStream_t s)
{
    switch (lanes) {
    case 1: step_lanes<1, ENERGY, MODE>(a, s); break;
    case 2: step_lanes<2, ENERGY, MODE>(a, s); break;
    case 4: step_lanes<4, ENERGY, MODE>(a, s); break;
    case 8: step_lanes<8, ENERGY, MODE>(a, s); break;
    default: step_lanes<16, ENERGY, MODE>(a, s); break;
    }
}

}  // namespace

void launch_rebuild(const DevBufs &b, int cur, int n, int cap, int lanes, const GridDev &g, float rc2,
                    hipStream_t s, bool advance_step_base, int list_every)
{
    hipLaunchKernelGGL(k_clear, dim3(blocks_for(g.n_cells, WG)), dim3(WG), 0, s, b.cell_count, g.n_cells,
                       b.n_occupied);
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.pos[cur], n, g, b.traj_cell,
                       b.cell_count, b.cells, b.occupied, b.n_occupied, b.err, advance_step_base ? b.step_base : nullptr, b.step_next,
                       list_every);
    FillArgs f{};
    f.occupied = b.occupied;
    f.n_occupied = b.n_occupied;
    f.count = b.cell_count;
    f.cells = b.cells;
    f.traj_lo = b.traj_lo;
    f.traj_hi = b.traj_hi;
    f.trow = b.trow;
    f.tent = b.tent;
    f.list = b.list;
    f.list_cnt = b.list_cnt;
    f.err = b.err;
    f.g = g;
    f.rc2 = rc2;
    f.cap = cap;
    switch (lanes) {
    case 1: fill_lanes<1>(f, g.n_cells, s); break;
    case 2: fill_lanes<2>(f, g.n_cells, s); break;
    case 4: fill_lanes<4>(f, g.n_cells, s); break;
    case 8: fill_lanes<8>(f, g.n_cells, s); break;
    default: fill_lanes<16>(f, g.n_cells, s); break;
    }
}

void launch_step(const DevBufs &b, int cur, int n, int cap, int lanes, const StepConsts &c,
                 const TipDev &tip, int has_pull, bool energy, int mode, const long long *step_base,
                 long long step_off, hipStream_t s)
{
    StepArgs a{};
    a.pin = b.pos[cur];
    a.pout = b.pos[cur ^ 1];
    a.trow = b.trow;
    a.tent = b.tent;
    a.list = b.list;
    a.list_cnt = b.list_cnt;
    a.stream_ids = b.stream_ids;
    a.pull_slot = b.pull_slot;
    a.pulls = b.pulls;
    a.res_energy = b.res_energy;
    a.fout = b.fout;
    a.err = b.err;
    a.step_base = step_base;
    a.step_off = step_off;
    a.n = n;
    a.cap = cap;
    a.has_pull = has_pull;
    a.c = c;
    a.tip = tip;
    if (mode == 1) {
        if (energy)
            step_dispatch<true, 1>(lanes, a, s);
        else
            step_dispatch<false, 1>(lanes, a, s);
    } else {
        if (energy)
            step_dispatch<true, 0>(lanes, a, s);
        else
            step_dispatch<false, 0>(lanes, a, s);
    }
}

void launch_batch(const DevBufs &b, int cur, int n_packs, int wg, int cap, const StepConsts &c,
                  const TipDev &tip, int has_pull, float rc2, int list_every, long long energy_every,
                  int n_steps, int stale, int mode, const long long *step_base, long long step_off,
                  hipStream_t s)
{
    BatchArgs a{};
    a.pin = b.pos[cur];
    a.pout = b.pos[cur ^ 1];
    a.trow = b.trow;
    a.tent = b.tent;
    a.pack_res = b.pack_res;
    a.traj_lo = b.traj_lo;
    a.traj_hi = b.traj_hi;
    a.stream_ids = b.stream_ids;
    a.pull_slot = b.pull_slot;
    a.pulls = b.pulls;
    a.list = b.list16;
    a.list_cnt = b.list_cnt;
    a.energy = b.energy;
    a.f_ext = b.f_ext;
    a.fout = b.fout;
    a.err = b.err;
    a.step_base = step_base;
    a.step_off = step_off;
    a.energy_every = energy_every;
    a.n_steps = n_steps;
    a.list_every = list_every;
    a.stale = stale;
    a.cap = cap;
    a.has_pull = has_pull;
    a.c = c;
    a.tip = tip;
    a.rc2 = rc2;
    const dim3 grid(n_packs);
    if (mode == 1) {
        switch (wg) {
        case 256: hipLaunchKernelGGL((k_batch<256, 1>), grid, dim3(256), 0, s, a); break;
        case 512: hipLaunchKernelGGL((k_batch<512, 1>), grid, dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL((k_batch<1024, 1>), grid, dim3(1024), 0, s, a); break;
        }
    } else {
        switch (wg) {
        case 256: hipLaunchKernelGGL((k_batch<256, 0>), grid, dim3(256), 0, s, a); break;
        case 512: hipLaunchKernelGGL((k_batch<512, 0>), grid, dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL((k_batch<1024, 0>), grid, dim3(1024), 0, s, a); break;
        }
    }
}

void launch_add_step(long long *base, long long k, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_step, dim3(1), dim3(64), 0, s, base, k);
}

void launch_reduce_energy(const DevBufs &b, int n_traj, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_energy, dim3(n_traj), dim3(WG), 0, s, b.res_energy, b.res_offsets,
                       b.energy, b.f_ext);
}

void launch_noise(const DevBufs &b, int cur, int n, const StepConsts &c, long long step, uint4 *words,
                  float4 *g, hipStream_t s)
{
    hipLaunchKernelGGL(k_noise, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.pos[cur], n, b.stream_ids,
                       c.key0, c.key1, step, words, g);
}

void launch_set_step(long long *dst, long long value, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, dst, value);
}

}  // namespace sop
