// HIP kernels for gfx950: Verlet-list rebuild on a wrapped cell grid, the
// fused per-step kernel (SOP forces of Eq. 1 over bonds, natives and the
// list; Philox4x32-10 Box-Muller noise; first-order overdamped update of
// Eq. 2 / Algorithm 7 with compensated single-precision positions), and the
// double-precision energy reduction.
#include "sop_internal.hpp"

namespace sop {

namespace {

constexpr int WG = 256;  // threads per workgroup (4 wave64)

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

__device__ __forceinline__ int wrap_cell(float x, float inv_cell, int n)
{
    float v = floorf(x * inv_cell);
    if (!(v == v))
        v = 0.0f;  // NaN positions are flagged elsewhere; keep the index in range
    v = fminf(fmaxf(v, -1.0e9f), 1.0e9f);
    int c = static_cast<int>(v) % n;
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

// ---------------------------------------------------------------------------
// Verlet-list rebuild: bin -> scan -> scatter -> per-cell sort -> fill
// ---------------------------------------------------------------------------
__global__ void k_clear(int *__restrict__ a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        a[i] = 0;
}

__global__ void k_bin(const float4 *__restrict__ hi, int n, GridDev g, int *__restrict__ cell_of,
                      int *__restrict__ slot, int *__restrict__ count, unsigned *__restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float4 p = hi[i];
    if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z))
        atomicOr(err, ERR_NONFINITE);
    const int cx = wrap_cell(p.x, g.inv_cell, g.gx);
    const int cy = wrap_cell(p.y, g.inv_cell, g.gy);
    const int cz = wrap_cell(p.z, g.inv_cell, g.gz);
    const int c = cx + g.gx * (cy + g.gy * cz);
    cell_of[i] = c;
    slot[i] = atomicAdd(&count[c], 1);
}

// One workgroup: exclusive scan of the per-cell counts.  Thread 0 also moves
// the graph step counter to the next list period when asked.
__global__ __launch_bounds__(1024) void k_scan(const int *__restrict__ count,
                                               int *__restrict__ start, int n,
                                               long long *step_base, long long *step_next,
                                               int advance, int period)
{
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int a = min(n, t * chunk), b = min(n, a + chunk);
    int s = 0;
    for (int k = a; k < b; ++k)
        s += count[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int k = a; k < b; ++k) {
        start[k] = run;
        run += count[k];
    }
    if (t == 1023)
        start[n] = part[1023];
    if (t == 0 && advance) {
        const long long nb = *step_next;
        *step_base = nb;
        *step_next = nb + period;
    }
}

__global__ void k_scatter(const float4 *__restrict__ hi, int n, const int *__restrict__ cell_of,
                          const int *__restrict__ slot, const int *__restrict__ start,
                          float4 *__restrict__ cpos)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float4 p = hi[i];
    cpos[start[cell_of[i]] + slot[i]] = make_float4(p.x, p.y, p.z, __int_as_float(i));
}

// Order each cell's residues by id so that list rows are deterministic.
__global__ void k_sort_cells(const int *__restrict__ start, int n_cells, float4 *__restrict__ cpos)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells)
        return;
    const int a = start[c], b = start[c + 1];
    for (int k = a + 1; k < b; ++k) {
        const float4 v = cpos[k];
        const int key = __float_as_int(v.w);
        int m = k - 1;
        while (m >= a && __float_as_int(cpos[m].w) > key) {
            cpos[m + 1] = cpos[m];
            --m;
        }
        cpos[m + 1] = v;
    }
}

template <int LANES>
__global__ __launch_bounds__(WG) void k_fill(const float4 *__restrict__ hi, int n, GridDev g,
                                             float rc2, const int *__restrict__ start,
                                             const float4 *__restrict__ cpos,
                                             const int *__restrict__ traj_lo,
                                             const int *__restrict__ traj_hi,
                                             const int2 *__restrict__ trow,
                                             const float2 *__restrict__ tent,
                                             int *__restrict__ list, int *__restrict__ list_cnt,
                                             int cap, unsigned *__restrict__ err)
{
    constexpr int G = 64 / LANES;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float4 p = hi[i];
    const int tlo = traj_lo[i], thi = traj_hi[i];
    const int2 row = trow[i];
    const int nex = (row.y & 4095) + (row.y >> 12);
    const int cx = wrap_cell(p.x, g.inv_cell, g.gx);
    const int cy = wrap_cell(p.y, g.inv_cell, g.gy);
    const int cz = wrap_cell(p.z, g.inv_cell, g.gz);
    int *rowp = list + (size_t)(i / G) * cap * G + (i % G) * LANES;
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        const int zz = (cz + dz + g.gz) % g.gz;
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = (cy + dy + g.gy) % g.gy;
            for (int dx = -1; dx <= 1; ++dx) {
                const int xx = (cx + dx + g.gx) % g.gx;
                const int c = xx + g.gx * (yy + g.gy * zz);
                const int a = start[c], b = start[c + 1];
                for (int k = a; k < b; ++k) {
                    const float4 q = cpos[k];
                    const int j = __float_as_int(q.w);
                    if (j == i || j < tlo || j >= thi)
                        continue;
                    if (!within_cutoff(p, q, rc2))
                        continue;
                    bool ex = false;
                    for (int e = 0; e < nex; ++e)
                        ex |= (__float_as_int(tent[row.x + e].x) == j);
                    if (ex)
                        continue;
                    if (cnt < cap)
                        rowp[(cnt / LANES) * 64 + (cnt % LANES)] = j;
                    ++cnt;
                }
            }
        }
    }
    list_cnt[i] = cnt;
    if (cnt > cap)
        atomicOr(err, ERR_OVERFLOW);
}

// ---------------------------------------------------------------------------
// Fused step: forces -> (noise -> compensated update) | force output
// ---------------------------------------------------------------------------
struct StepArgs {
    const float4 *hi_in;
    const float4 *lo_in;
    float4 *hi_out;
    float4 *lo_out;
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

    const float4 hi = a.hi_in[r];
    const float4 lo = a.lo_in[r];
    float fx = 0.f, fy = 0.f, fz = 0.f;
    double e_b = 0.0, e_n = 0.0, e_r = 0.0, vir = 0.0;
    bool broken = false;

    const int2 row = a.trow[r];
    const int nb = row.y & 4095, nn = row.y >> 12;
    const float kf = a.c.k_fene, R0sq = a.c.R0sq;
    // FENE bonds
    for (int p = l; p < nb; p += LANES) {
        const float2 t = a.tent[row.x + p];
        const int j = __float_as_int(t.x);
        const float3 d = pair_delta(hi, lo, a.hi_in[j], a.lo_in[j]);
        const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
        const float rr = sqrtf(r2);
        const float dl = rr - t.y;
        float x = 1.0f - dl * dl / R0sq;
        if (!(x > 0.0f)) {
            broken = true;
            x = 1.0f;
        }
        const float coef = -kf * dl / (x * rr);
        fx += coef * d.x;
        fy += coef * d.y;
        fz += coef * d.z;
        if (ENERGY) {
            const double dd = (double)dl;
            e_b += -0.5 * (double)kf * (double)R0sq * log1p(-dd * dd / (double)R0sq);
            vir += -(double)rr * (double)kf * dd / (double)x;
        }
    }
    // native contacts
    const float eh = a.c.eps_h;
    for (int p = nb + l; p < nb + nn; p += LANES) {
        const float2 t = a.tent[row.x + p];
        const int j = __float_as_int(t.x);
        const float3 d = pair_delta(hi, lo, a.hi_in[j], a.lo_in[j]);
        const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
        const float ir2 = 1.0f / r2;
        const float s = t.y * t.y * ir2;
        const float q = s * s * s;
        const float coef = 12.0f * eh * (q * q - q) * ir2;
        fx += coef * d.x;
        fy += coef * d.y;
        fz += coef * d.z;
        if (ENERGY) {
            e_n += (double)(eh * (q * q - 2.0f * q));
            vir += (double)(12.0f * eh * (q * q - q));
        }
    }
    // repulsive list
    const float el = a.c.eps_l, sg2 = a.c.sigma2;
    const int cnt = min(a.list_cnt[r], a.cap);
    const int *lp = a.list + (size_t)wave * a.cap * G + g * LANES + l;
    for (int k = 0, p = l; p < cnt; ++k, p += LANES) {
        const int j = lp[k * 64];
        const float3 d = pair_delta(hi, lo, a.hi_in[j], a.lo_in[j]);
        const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
        const float ir2 = 1.0f / r2;
        const float s = sg2 * ir2;
        const float q = s * s * s;
        const float coef = 6.0f * el * q * ir2;
        fx += coef * d.x;
        fy += coef * d.y;
        fz += coef * d.z;
        if (ENERGY) {
            e_r += (double)(el * q);
            vir += (double)(6.0f * el * q);
        }
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
                fx += (float)(pd.kappa * dx);
                fy += (float)(pd.kappa * dy);
                fz += (float)(pd.kappa * dz);
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
                fx += cx;
                fy += cy;
                fz += cz;
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
#pragma unroll
    for (int m = LANES / 2; m >= 1; m >>= 1) {
        fx += __shfl_xor(fx, m, 64);
        fy += __shfl_xor(fy, m, 64);
        fz += __shfl_xor(fz, m, 64);
        if (ENERGY) {
            e_b += __shfl_xor(e_b, m, 64);
            e_n += __shfl_xor(e_n, m, 64);
            e_r += __shfl_xor(e_r, m, 64);
            vir += __shfl_xor(vir, m, 64);
        }
    }
    if (ENERGY && l == 0) {
        double *er = a.res_energy + (size_t)r * RES_E;
        // each internal pair appears in both partners' rows
        er[0] = 0.5 * e_b;
        er[1] = 0.5 * e_n;
        er[2] = 0.5 * e_r;
        er[3] = e_x;
        er[4] = 0.5 * vir;
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
    float *ho = reinterpret_cast<float *>(a.hi_out + r);
    float *lw = reinterpret_cast<float *>(a.lo_out + r);
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
__global__ void k_noise(const float4 *__restrict__ hi, const float4 *__restrict__ lo, int n,
                        const unsigned *__restrict__ stream_ids, unsigned k0, unsigned k1,
                        long long step, uint4 *__restrict__ words, float4 *__restrict__ g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const unsigned local = __float_as_uint(hi[i].w) & 0x7fffffffu;
    const unsigned stream = stream_ids[__float_as_int(lo[i].w)];
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
void fill_lanes(const DevBufs &b, int cur, int n, int cap, const GridDev &g, float rc2, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill<LANES>, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.hi[cur], n, g, rc2,
                       b.cell_start, b.cpos, b.traj_lo, b.traj_hi, b.trow, b.tent, b.list, b.list_cnt,
                       cap, b.err);
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
    hipLaunchKernelGGL(k_clear, dim3(blocks_for(g.n_cells, WG)), dim3(WG), 0, s, b.cell_count, g.n_cells);
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.hi[cur], n, g, b.cell_of,
                       b.cell_slot, b.cell_count, b.err);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, b.cell_count, b.cell_start, g.n_cells,
                       b.step_base, b.step_next, advance_step_base ? 1 : 0, list_every);
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.hi[cur], n, b.cell_of,
                       b.cell_slot, b.cell_start, b.cpos);
    hipLaunchKernelGGL(k_sort_cells, dim3(blocks_for(g.n_cells, WG)), dim3(WG), 0, s, b.cell_start,
                       g.n_cells, b.cpos);
    switch (lanes) {
    case 1: fill_lanes<1>(b, cur, n, cap, g, rc2, s); break;
    case 2: fill_lanes<2>(b, cur, n, cap, g, rc2, s); break;
    case 4: fill_lanes<4>(b, cur, n, cap, g, rc2, s); break;
    case 8: fill_lanes<8>(b, cur, n, cap, g, rc2, s); break;
    default: fill_lanes<16>(b, cur, n, cap, g, rc2, s); break;
    }
}

void launch_step(const DevBufs &b, int cur, int n, int cap, int lanes, const StepConsts &c,
                 const TipDev &tip, int has_pull, bool energy, int mode, const long long *step_base,
                 long long step_off, hipStream_t s)
{
    StepArgs a{};
    a.hi_in = b.hi[cur];
    a.lo_in = b.lo[cur];
    a.hi_out = b.hi[cur ^ 1];
    a.lo_out = b.lo[cur ^ 1];
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

void launch_reduce_energy(const DevBufs &b, int n_traj, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_energy, dim3(n_traj), dim3(WG), 0, s, b.res_energy, b.res_offsets,
                       b.energy, b.f_ext);
}

void launch_noise(const DevBufs &b, int cur, int n, const StepConsts &c, long long step, uint4 *words,
                  float4 *g, hipStream_t s)
{
    hipLaunchKernelGGL(k_noise, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.hi[cur], b.lo[cur], n,
                       b.stream_ids, c.key0, c.key1, step, words, g);
}

void launch_set_step(long long *dst, long long value, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, dst, value);
}

}  // namespace sop
