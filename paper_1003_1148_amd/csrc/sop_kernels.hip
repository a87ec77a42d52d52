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
__global__ void k_clear(int *__restrict__ a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        a[i] = 0;
}

// Cell index of one residue in the wrapped grid (the trajectory's offset
// keeps independent trajectories in separate cells).
__device__ __forceinline__ int cell_index(const float4 &p, const int4 &off, const GridDev &g)
{
    const int cx = wrap_cell(p.x, g.inv_cell, off.x, g.gx);
    const int cy = wrap_cell(p.y, g.inv_cell, off.y, g.gy);
    const int cz = wrap_cell(p.z, g.inv_cell, off.z, g.gz);
    return cx + g.gx * (cy + g.gy * cz);
}

// Also advances the step counter of graph replays (once per rebuild) when
// step_base is given.
__global__ void k_bin(const float4 *__restrict__ pos, int n, GridDev g, const int4 *__restrict__ traj_cell,
                      int *__restrict__ count, float4 *__restrict__ cells, int *__restrict__ cell_of,
                      unsigned *__restrict__ err, long long *step_base, long long *step_next, int period)
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
    const int c = cell_index(p, traj_cell[__float_as_int(pos[2 * i + 1].w)], g);
    cell_of[i] = c;
    const int slot = atomicAdd(&count[c], 1);
    if (slot < CELL_CAP)
        cells[(size_t)c * CELL_CAP + slot] = make_float4(p.x, p.y, p.z, __int_as_float(i));
    else
        atomicOr(err, ERR_CELL);
}

// ---------------------------------------------------------------------------
// Pair terms of Eq. 1, external terms and the compensated update, shared by
// the plain and the batched schedules.
// ---------------------------------------------------------------------------

// Per-residue force and, on energy steps, double energy/virial sums.
struct Acc {
    float fx = 0.f, fy = 0.f, fz = 0.f;
    double e_b = 0.0, e_n = 0.0, e_r = 0.0, vir = 0.0;
};

struct PairConsts {
    float kf, inv_R0sq, R0sq, eh, eh12, el, el6, sg2;
};

__device__ __forceinline__ PairConsts pair_consts(const StepConsts &c)
{
    PairConsts k;
    k.kf = c.k_fene;
    k.inv_R0sq = c.inv_R0sq;
    k.R0sq = c.R0sq;
    k.eh = c.eps_h;
    k.eh12 = 12.0f * c.eps_h;
    k.el = c.eps_l;
    k.el6 = 6.0f * c.eps_l;
    k.sg2 = c.sigma2;
    return k;
}

// FENE: -(k R0^2/2) ln(1 - (r - r0)^2/R0^2); |r - r0| >= R0 sets `broken`.
__device__ __forceinline__ void add_fene(Acc &A, const float4 &hi, const float4 &lo, const float4 &hj,
                                         const float4 &lj, float r0, const PairConsts &k, bool rec,
                                         bool &broken)
{
    const float3 d = pair_delta(hi, lo, hj, lj);
    const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    const float rr = __builtin_amdgcn_sqrtf(r2);
    const float dl = rr - r0;
    float x = 1.0f - dl * dl * k.inv_R0sq;
    if (!(x > 0.0f)) {
        broken = true;
        x = 1.0f;
    }
    const float coef = -k.kf * dl * fast_rcp(x * rr);
    A.fx += coef * d.x;
    A.fy += coef * d.y;
    A.fz += coef * d.z;
    if (rec) {
        const double dd = (double)dl;
        const double R0sq = (double)k.R0sq;
        A.e_b += -0.5 * (double)k.kf * R0sq * log1p(-dd * dd / R0sq);
        A.vir += -(double)rr * (double)k.kf * dd / (1.0 - dd * dd / R0sq);
    }
}

// Native contact: eps_h [(r0/r)^12 - 2 (r0/r)^6].
__device__ __forceinline__ void add_native(Acc &A, const float4 &hi, const float4 &lo, const float4 &hj,
                                           const float4 &lj, float r0, const PairConsts &k, bool rec)
{
    const float3 d = pair_delta(hi, lo, hj, lj);
    const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    const float ir2 = fast_rcp(r2);
    const float s = r0 * r0 * ir2;
    const float q = s * s * s;
    const float coef = k.eh12 * (q * q - q) * ir2;
    A.fx += coef * d.x;
    A.fy += coef * d.y;
    A.fz += coef * d.z;
    if (rec) {
        A.e_n += (double)(k.eh * (q * q - 2.0f * q));
        A.vir += (double)(k.eh12 * (q * q - q));
    }
}

// Soft repulsion: eps_l (sigma/r)^6.
__device__ __forceinline__ void add_repulsive(Acc &A, const float4 &hi, const float4 &lo,
                                              const float4 &hj, const float4 &lj, const PairConsts &k,
                                              bool rec)
{
    const float3 d = pair_delta(hi, lo, hj, lj);
    const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    const float ir2 = fast_rcp(r2);
    const float s = k.sg2 * ir2;
    const float q = s * s * s;
    const float coef = k.el6 * q * ir2;
    A.fx += coef * d.x;
    A.fy += coef * d.y;
    A.fz += coef * d.z;
    if (rec) {
        A.e_r += (double)(k.el * q);
        A.vir += (double)(k.el6 * q);
    }
}

// Cantilever `pull` (index or -1) and tip on one residue at t_n = step*h.
__device__ __forceinline__ void add_external(Acc &A, double &e_x, double &f_rep, const float4 &hi,
                                             const float4 &lo, long long step, double h, int pull,
                                             const PullDev *pulls, const TipDev &tip, bool rec,
                                             unsigned *err)
{
    if (pull < 0 && !tip.on)
        return;
    const double tn = (double)step * h;
    const double px = (double)hi.x + (double)lo.x;
    const double py = (double)hi.y + (double)lo.y;
    const double pz = (double)hi.z + (double)lo.z;
    if (pull >= 0) {
        const PullDev pd = pulls[pull];
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
    if (tip.on) {
        const float dx = (float)(px - (tip.c0[0] + tip.v[0] * tn));
        const float dy = (float)(py - (tip.c0[1] + tip.v[1] * tn));
        const float dz = (float)(pz - (tip.c0[2] + tip.v[2] * tn));
        const float rr = sqrtf(dx * dx + dy * dy + dz * dz);
        const float gap = rr - (float)tip.radius;
        if (!(gap > 0.0f)) {
            atomicOr(err, ERR_TIP);
            return;
        }
        const float sg = (float)tip.sigma / gap;
        const float s3 = sg * sg * sg;
        const float q = s3 * s3;
        const float mag = 6.0f * (float)tip.eps * q / gap;
        const float cx = mag * dx / rr, cy = mag * dy / rr, cz = mag * dz / rr;
        A.fx += cx;
        A.fy += cy;
        A.fz += cz;
        if (rec) {
            e_x += tip.eps * (double)q;
            if (tip.has_dir)
                f_rep += (double)cx * tip.vhat[0] + (double)cy * tip.vhat[1] + (double)cz * tip.vhat[2];
        }
    }
}

// Noise (Section III.C) and the first-order update (Eq. 2 / Algorithm 7)
// with compensated positions: (hi, lo) <- TwoSum(hi, delta + lo) per axis.
__device__ __forceinline__ void langevin_update(float4 &hi, float4 &lo, const Acc &A, long long step,
                                                unsigned stream, const StepConsts &c, unsigned *err)
{
    const unsigned tag = __float_as_uint(hi.w);
    if (tag >> 31)
        return;  // fixed residue
    const uint4 w = philox10(make_uint4(tag & 0x7fffffffu, stream, (unsigned)step,
                                        (unsigned)((unsigned long long)step >> 32)),
                             c.key0, c.key1);
    float nh[3], nl[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float f = ax == 0 ? A.fx : (ax == 1 ? A.fy : A.fz);
        const float h0 = comp(hi, ax), l0 = comp(lo, ax);
        const float delta = c.c_drift * f + c.c_noise * gaussian_axis(w, ax);
        const float y = delta + l0;
        const float t = h0 + y;
        const float bp = t - h0;
        const float ap = t - bp;
        nl[ax] = (h0 - ap) + (y - bp);
        nh[ax] = t;
    }
    if (!isfinite(nh[0]) || !isfinite(nh[1]) || !isfinite(nh[2]) || !isfinite(nl[0]) ||
        !isfinite(nl[1]) || !isfinite(nl[2]))
        atomicOr(err, ERR_NONFINITE);
    hi = make_float4(nh[0], nh[1], nh[2], hi.w);
    lo = make_float4(nl[0], nl[1], nl[2], lo.w);
}

// ---------------------------------------------------------------------------
// Plain schedule, tile staging: at each rebuild, the residues a tile of
// consecutive residues interacts with (list partners, bonded and native
// partners, itself) become a sorted set of at most stage_max slots, and
// rows are rewritten as 16-bit slots into that set.
// ---------------------------------------------------------------------------
template <int TILE>
constexpr int stage_max() { return TILE >= 256 ? 2048 : 1024; }

// Entry k of lane t of a tile: rows are stored in chunks of 8 slots per lane
// so that one 16-byte load brings the next 8 partners of a residue.
template <int TILE>
__device__ __forceinline__ size_t list16_index(int tile, int t, int k, int cap)
{
    return (size_t)tile * cap * TILE + (size_t)(k >> 3) * (8 * TILE) + (size_t)t * 8 + (k & 7);
}

constexpr int CAND_MAX = 2816;  // candidate residues a tile stages in LDS during a rebuild
constexpr int CELLS_MAX = 640;  // distinct cells around one tile
constexpr int CHASH_BITS = 10;
constexpr int CHASH = 1 << CHASH_BITS;  // open-addressing table of those cells
constexpr int EXTRA_MAX = 128;  // bonded/native partners outside the tile's cells

struct BuildArgs {
    const float4 *pos;
    const int *cell_of;
    const int *count;
    const float4 *cells;
    const int4 *traj_cell;
    const int *traj_lo;
    const int *traj_hi;
    const int2 *trow;
    const float2 *tent;
    int *list_cnt;
    unsigned short *list16;
    uint2 *topo2;
    int *stage;
    int *stage_cnt;
    unsigned *err;
    GridDev g;
    float rc2, edge, cull2;
    int n, cap;
};

// One workgroup per tile.  (1) The cells around the tile's residues (their
// 27-cell neighbourhoods) go into an LDS table; their residues are copied to
// LDS and ranked by id within each cell.  (2) Each lane builds its residue's
// row over its 27 cells in a fixed order (cells whose box lies beyond the
// cutoff are skipped), members in id order: the Algorithm 3 filter r < r_list
// without bonded or native partners.  (3) The candidates that some row or
// bond/native entry uses become the tile's staging slots, and rows are
// rewritten as slots.
template <int TILE>
__global__ __launch_bounds__(TILE) void k_tile_build(BuildArgs a)
{
    constexpr int SM = stage_max<TILE>();
    __shared__ float4 cand[CAND_MAX];            // arrival order within each cell
    __shared__ unsigned short order[CAND_MAX];   // rank in cell -> arrival index
    __shared__ unsigned short used[CAND_MAX];    // 0/1, then the slot number
    __shared__ int hkey[CHASH];
    __shared__ short hval[CHASH];
    __shared__ int ccell[CELLS_MAX];
    __shared__ int cbase[CELLS_MAX + 1];
    __shared__ int part[TILE];
    __shared__ int extra[EXTRA_MAX];
    __shared__ int n_cu, n_extra, bad;

    const int tile = blockIdx.x, t = threadIdx.x;
    const int i = tile * TILE + t;
    const bool act = i < a.n;
    const GridDev g = a.g;
    for (int h = t; h < CHASH; h += TILE)
        hkey[h] = -1;
    if (t == 0) {
        n_cu = 0;
        n_extra = 0;
        bad = 0;
    }
    __syncthreads();

    auto wrap = [](int v, int n) { const int r = v % n; return r < 0 ? r + n : r; };
    auto hslot = [](int key) { return (int)(((unsigned)key * 2654435761u) >> (32 - CHASH_BITS)) & (CHASH - 1); };
    auto lookup = [&](int key) -> int {
        int h = hslot(key);
        for (int probe = 0; probe < CHASH; ++probe) {
            const int k = hkey[h];
            if (k == key)
                return hval[h];
            if (k < 0)
                return -1;
            h = (h + 1) & (CHASH - 1);
        }
        return -1;
    };

    // own residue: position, unwrapped cell coordinates, neighbourhood
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    int ux = 0, uy = 0, uz = 0;
    if (act) {
        p = a.pos[2 * i];
        const int4 off = a.traj_cell[__float_as_int(a.pos[2 * i + 1].w)];
        auto ucell = [&](float x, int o) {
            float v = floorf(x * g.inv_cell);
            if (!(v == v))
                v = 0.0f;
            return (int)fminf(fmaxf(v, -1.0e9f), 1.0e9f) + o;
        };
        ux = ucell(p.x, off.x);
        uy = ucell(p.y, off.y);
        uz = ucell(p.z, off.z);
        for (int d = 0; d < 27; ++d) {
            const int cid = wrap(ux + d % 3 - 1, g.gx) +
                            g.gx * (wrap(uy + (d / 3) % 3 - 1, g.gy) + g.gy * wrap(uz + d / 9 - 1, g.gz));
            int h = hslot(cid);
            for (int probe = 0; probe < CHASH; ++probe) {
                const int prev = atomicCAS(&hkey[h], -1, cid);
                if (prev == -1) {
                    const int m = atomicAdd(&n_cu, 1);
                    if (m < CELLS_MAX) {
                        ccell[m] = cid;
                        hval[h] = (short)m;
                    } else {
                        bad = 1;
                    }
                    break;
                }
                if (prev == cid)
                    break;
                h = (h + 1) & (CHASH - 1);
                if (probe == CHASH - 1)
                    bad = 1;
            }
        }
    }
    __syncthreads();
    const int NC = n_cu;
    if (bad == 0 && NC <= CELLS_MAX) {
        for (int m = t; m < NC; m += TILE)
            cbase[m + 1] = min(a.count[ccell[m]], CELL_CAP);
        __syncthreads();
        if (t == 0) {
            cbase[0] = 0;
            for (int m = 0; m < NC; ++m)
                cbase[m + 1] += cbase[m];
            if (cbase[NC] > CAND_MAX)
                bad = 1;
        }
    }
    __syncthreads();
    const int2 row = act ? a.trow[i] : make_int2(0, 0);
    const int ntop = (row.y & 4095) + (row.y >> 12);
    if (bad || NC > CELLS_MAX) {
        // report, leave the tile's slots at the empty slot so steps stay in bounds
        if (t == 0) {
            atomicOr(a.err, ERR_STAGE);
            a.stage_cnt[tile] = 0;
        }
        if (act) {
            a.list_cnt[i] = 0;
            uint2 *trw = a.topo2 + (size_t)tile * TOPO_CAP * TILE + t;
            for (int e = 0; e < ntop; ++e)
                trw[(size_t)e * TILE] = make_uint2((unsigned)SM, __float_as_uint(1.0f));
        }
        return;  // uniform: bad and NC are read after a barrier
    }
    const int M = cbase[NC];
    auto segment_of = [&](int ci) {  // last m with cbase[m] <= ci
        int lo = 0, hi = NC;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cbase[mid] <= ci)
                lo = mid;
            else
                hi = mid;
        }
        return lo;
    };
    for (int ci = t; ci < M; ci += TILE) {
        const int m = segment_of(ci);
        cand[ci] = a.cells[(size_t)ccell[m] * CELL_CAP + (ci - cbase[m])];
        used[ci] = 0;
    }
    __syncthreads();
    for (int ci = t; ci < M; ci += TILE) {
        const int m = segment_of(ci);
        const int id = __float_as_int(cand[ci].w);
        int rank = 0;
        for (int k = cbase[m]; k < cbase[m + 1]; ++k)
            rank += __float_as_int(cand[k].w) < id;
        order[cbase[m] + rank] = (unsigned short)ci;
    }
    __syncthreads();

    // rows, one lane per residue, with arrival indices for now
    int cnt = 0;
    if (act) {
        const int tlo = a.traj_lo[i], thi = a.traj_hi[i];
        int ex[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            ex[u] = u < ntop ? __float_as_int(a.tent[row.x + u].x) : -2;
        const float lx = floorf(p.x * g.inv_cell) * a.edge;
        const float ly = floorf(p.y * g.inv_cell) * a.edge;
        const float lz = floorf(p.z * g.inv_cell) * a.edge;
        const float gx[3] = {p.x - lx, 0.0f, lx + a.edge - p.x};
        const float gy[3] = {p.y - ly, 0.0f, ly + a.edge - p.y};
        const float gz[3] = {p.z - lz, 0.0f, lz + a.edge - p.z};
        for (int d = 0; d < 27; ++d) {
            const int dx = d % 3, dy = (d / 3) % 3, dz = d / 9;
            // smallest distance from p to that cell's box
            if (gx[dx] * gx[dx] + gy[dy] * gy[dy] + gz[dz] * gz[dz] > a.cull2)
                continue;
            const int cid = wrap(ux + dx - 1, g.gx) + g.gx * (wrap(uy + dy - 1, g.gy) + g.gy * wrap(uz + dz - 1, g.gz));
            const int m = lookup(cid);
            for (int r = cbase[m]; r < cbase[m + 1]; ++r) {
                const int ci = order[r];
                const float4 q = cand[ci];
                const int j = __float_as_int(q.w);
                if (j == i || j < tlo || j >= thi || !within_cutoff(p, q, a.rc2))
                    continue;
                bool excl = false;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    excl |= ex[u] == j;
                for (int e = 16; e < ntop; ++e)
                    excl |= __float_as_int(a.tent[row.x + e].x) == j;
                if (excl)
                    continue;
                if (cnt < a.cap)
                    a.list16[list16_index<TILE>(tile, t, cnt, a.cap)] = (unsigned short)ci;
                used[ci] = 1;
                ++cnt;
            }
        }
        a.list_cnt[i] = cnt;
        if (cnt > a.cap)
            atomicOr(a.err, ERR_OVERFLOW);
        // bonded and native partners: their candidate, or an extra slot
        uint2 *trw = a.topo2 + (size_t)tile * TOPO_CAP * TILE + t;
        for (int e = 0; e < ntop; ++e) {
            const float2 te = a.tent[row.x + e];
            const int j = __float_as_int(te.x);
            const int m = lookup(a.cell_of[j]);
            int ci = -1;
            if (m >= 0) {
                int lo = cbase[m], hi = cbase[m + 1];  // binary search by id in the cell
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const int idm = __float_as_int(cand[order[mid]].w);
                    if (idm < j)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo < cbase[m + 1] && __float_as_int(cand[order[lo]].w) == j)
                    ci = order[lo];
            }
            unsigned code;
            if (ci >= 0) {
                used[ci] = 1;
                code = (unsigned)ci;
            } else {
                const int k = atomicAdd(&n_extra, 1);
                if (k < EXTRA_MAX)
                    extra[k] = j;
                code = 0x80000000u | (unsigned)k;
            }
            trw[(size_t)e * TILE] = make_uint2(code, __float_as_uint(te.y));
        }
    }
    __syncthreads();
    // used candidates -> slots (exclusive prefix over arrival order)
    const int per = (M + TILE - 1) / TILE;
    const int c0 = min(M, t * per), c1 = min(M, c0 + per);
    int u = 0;
    for (int ci = c0; ci < c1; ++ci)
        u += used[ci];
    part[t] = u;
    __syncthreads();
    for (int off = 1; off < TILE; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int n_used = part[TILE - 1];
    const int S = n_used + min(n_extra, EXTRA_MAX);
    if (S > SM || n_extra > EXTRA_MAX) {
        if (t == 0) {
            atomicOr(a.err, ERR_STAGE);
            a.stage_cnt[tile] = 0;
        }
        if (act) {
            a.list_cnt[i] = 0;
            uint2 *trw = a.topo2 + (size_t)tile * TOPO_CAP * TILE + t;
            for (int e = 0; e < ntop; ++e)
                trw[(size_t)e * TILE] = make_uint2((unsigned)SM, __float_as_uint(1.0f));
        }
        return;  // uniform
    }
    int sl = part[t] - u;
    int *st = a.stage + (size_t)tile * SM;
    for (int ci = c0; ci < c1; ++ci) {
        if (used[ci]) {
            st[sl] = __float_as_int(cand[ci].w);
            used[ci] = (unsigned short)sl;
            ++sl;
        }
    }
    for (int k = t; k < min(n_extra, EXTRA_MAX); k += TILE)
        st[n_used + k] = extra[k];
    if (t == 0)
        a.stage_cnt[tile] = S;
    __syncthreads();
    if (act) {
        // rows padded to a multiple of 8 with the empty slot SM (a position
        // far away, so its pair term is exactly zero)
        const int m = min(cnt, a.cap);
        for (int k = 0; k < ((m + 7) & ~7); ++k) {
            const size_t x = list16_index<TILE>(tile, t, k, a.cap);
            a.list16[x] = k < m ? used[a.list16[x]] : (unsigned short)SM;
        }
        uint2 *trw = a.topo2 + (size_t)tile * TOPO_CAP * TILE + t;
        for (int e = 0; e < ntop; ++e) {
            const uint2 v = trw[(size_t)e * TILE];
            const unsigned sl2 = (v.x & 0x80000000u) ? (unsigned)n_used + (v.x & 0x7fffffffu) : used[v.x];
            trw[(size_t)e * TILE] = make_uint2(sl2, v.y);
        }
    }
}

struct TileArgs {
    const float4 *pin;
    float4 *pout;
    const int2 *trow;
    const float2 *tent;
    const unsigned short *list16;
    const uint2 *topo2;
    const int *list_cnt;
    const int *stage;
    const int *stage_cnt;
    const unsigned *stream_ids;
    const int *pull_slot;
    const PullDev *pulls;
    double *res_energy;
    float4 *fout;
    unsigned *err;
    const long long *step_base;
    long long step_off;
    int n, cap, has_pull, n_tiles;
    StepConsts c;
    TipDev tip;
};

// One workgroup per tile, one lane per residue: stage the tile's slots in
// LDS, then every pair term reads LDS.
// Few waves per SIMD (about one residue per lane across the GPU), so the
// compiler may trade registers for loads in flight.
template <int TILE, bool ENERGY, int MODE>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_tile_step(TileArgs a)
{
    constexpr int SM = stage_max<TILE>();
    __shared__ float4 sh[2 * (SM + 1)];  // slot SM: the far-away empty slot
    // XCD-aware order: consecutive tiles stay on one XCD's L2.
    const int per = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= a.n_tiles)
        return;
    const int t = threadIdx.x;
    const int i = tile * TILE + t;
    const bool act = i < a.n;
    const int S = a.stage_cnt[tile];
    const int *st = a.stage + (size_t)tile * SM;
    // independent loads of this residue's data first
    float4 hi0 = make_float4(0.f, 0.f, 0.f, 0.f), lo0 = hi0;
    int2 row = make_int2(0, 0);
    int cnt = 0;
    const uint4 *lp4 = reinterpret_cast<const uint4 *>(a.list16) + (size_t)tile * (a.cap >> 3) * TILE + t;
    const uint2 *tp = a.topo2 + (size_t)tile * TOPO_CAP * TILE + t;
    uint4 cur = make_uint4(0u, 0u, 0u, 0u);
    if (act) {
        hi0 = a.pin[2 * i];
        lo0 = a.pin[2 * i + 1];
        row = a.trow[i];
        cnt = min(a.list_cnt[i], a.cap);
        cur = lp4[0];
    }
    {
        // all slot ids first, then all positions, so the loads overlap
        constexpr int PER = SM / TILE;
        int ids[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int s = t + u * TILE;
            ids[u] = s < S ? st[s] : -1;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (ids[u] >= 0) {
                const int s = t + u * TILE;
                sh[2 * s] = a.pin[2 * ids[u]];
                sh[2 * s + 1] = a.pin[2 * ids[u] + 1];
            }
        }
        if (t == 0) {
            sh[2 * SM] = make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.0f);
            sh[2 * SM + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
    __syncthreads();
    if (!act)
        return;
    const PairConsts k = pair_consts(a.c);
    const long long step = (a.step_base ? *a.step_base : 0) + a.step_off;
    Acc A;
    bool broken = false;
    const int nb = row.y & 4095, ntop = nb + (row.y >> 12);
    // bonds and natives, four entries per block
    for (int e0 = 0; e0 < ntop; e0 += 4) {
        uint2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            v[u] = e0 + u < ntop ? tp[(size_t)(e0 + u) * TILE] : make_uint2((unsigned)SM, __float_as_uint(1.0f));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u, sj = (int)v[u].x;
            const float r0 = __uint_as_float(v[u].y);
            if (e < nb)
                add_fene(A, hi0, lo0, sh[2 * sj], sh[2 * sj + 1], r0, k, ENERGY, broken);
            else if (e < ntop)
                add_native(A, hi0, lo0, sh[2 * sj], sh[2 * sj + 1], r0, k, ENERGY);
        }
    }
    // list partners: chunks of 8 slots with four chunks in flight
    const int nch = (cnt + 7) >> 3;
    auto chunk8 = [&](const uint4 &q) {
        const unsigned w[4] = {q.x, q.y, q.z, q.w};
        float4 ph[8], pl[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {  // all 16 LDS reads before any use
            const int sj = (int)((w[u >> 1] >> ((u & 1) * 16)) & 0xffffu);
            ph[u] = sh[2 * sj];
            pl[u] = sh[2 * sj + 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            add_repulsive(A, hi0, lo0, ph[u], pl[u], k, ENERGY);
    };
    // unconditional loads (a branch around them would force a full wait);
    // chunks past the row are clamped into the row's region and never used
    const int last_ch = (a.cap >> 3) - 1;
    auto fetch = [&](int ch) -> uint4 { return lp4[(size_t)min(ch, last_ch) * TILE]; };
    uint4 q0 = cur, q1 = fetch(1), q2 = fetch(2), q3 = fetch(3);
    int ch = 0;
    for (; ch + 4 <= nch; ch += 4) {  // whole groups: no branches between the loads
        chunk8(q0);
        q0 = fetch(ch + 4);
        chunk8(q1);
        q1 = fetch(ch + 5);
        chunk8(q2);
        q2 = fetch(ch + 6);
        chunk8(q3);
        q3 = fetch(ch + 7);
    }
    if (ch < nch)
        chunk8(q0);
    if (ch + 1 < nch)
        chunk8(q1);
    if (ch + 2 < nch)
        chunk8(q2);
    double e_x = 0.0, f_rep = 0.0;
    add_external(A, e_x, f_rep, hi0, lo0, step, a.c.h, a.has_pull ? a.pull_slot[i] : -1, a.pulls,
                 a.tip, ENERGY, a.err);
    if (broken)
        atomicOr(a.err, ERR_FENE);
    if (ENERGY) {
        double *er = a.res_energy + (size_t)i * RES_E;
        // each internal pair appears in both partners' rows
        er[0] = 0.5 * A.e_b;
        er[1] = 0.5 * A.e_n;
        er[2] = 0.5 * A.e_r;
        er[3] = e_x;
        er[4] = 0.5 * A.vir;
        er[5] = f_rep;
    }
    if (MODE == 1) {
        a.fout[i] = make_float4(A.fx, A.fy, A.fz, 0.0f);
        return;
    }
    float4 hi = hi0, lo = lo0;
    langevin_update(hi, lo, A, step, a.stream_ids[__float_as_int(lo0.w)], a.c, a.err);
    a.pout[2 * i] = hi;
    a.pout[2 * i + 1] = lo;
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
    const PairConsts kc = pair_consts(a.c);
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
                add_fene(A, hi, lo, sh[2 * j], sh[2 * j + 1], tt.y, kc, rec, broken);
            }
            for (int e = nb; e < nb + nn; ++e) {
                const float2 tt = a.tent[row.x + e];
                const int j = __float_as_int(tt.x) - base;
                add_native(A, hi, lo, sh[2 * j], sh[2 * j + 1], tt.y, kc, rec);
            }
            const int m = min(cnt, a.cap);
            int k = 0;
            for (; k + 4 <= m; k += 4) {
                const int j0 = lrow[(size_t)(k + 0) * n], j1 = lrow[(size_t)(k + 1) * n];
                const int j2 = lrow[(size_t)(k + 2) * n], j3 = lrow[(size_t)(k + 3) * n];
                add_repulsive(A, hi, lo, sh[2 * j0], sh[2 * j0 + 1], kc, rec);
                add_repulsive(A, hi, lo, sh[2 * j1], sh[2 * j1 + 1], kc, rec);
                add_repulsive(A, hi, lo, sh[2 * j2], sh[2 * j2 + 1], kc, rec);
                add_repulsive(A, hi, lo, sh[2 * j3], sh[2 * j3 + 1], kc, rec);
            }
            for (; k < m; ++k) {
                const int j = lrow[(size_t)k * n];
                add_repulsive(A, hi, lo, sh[2 * j], sh[2 * j + 1], kc, rec);
            }
            add_external(A, e_x, f_rep, hi, lo, step, a.c.h, a.has_pull ? a.pull_slot[i] : -1, a.pulls,
                         a.tip, rec, a.err);
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
        if (act)
            langevin_update(nh4, nl4, A, step, stream, a.c, a.err);
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

template <int TILE>
void rebuild_tile(const DevBufs &b, int cur, int n, int cap, const GridDev &g, float rc2, float edge,
                  float cull2, hipStream_t s)
{
    BuildArgs a{};
    a.pos = b.pos[cur];
    a.cell_of = b.cell_of;
    a.count = b.cell_count;
    a.cells = b.cells;
    a.traj_cell = b.traj_cell;
    a.traj_lo = b.traj_lo;
    a.traj_hi = b.traj_hi;
    a.trow = b.trow;
    a.tent = b.tent;
    a.list_cnt = b.list_cnt;
    a.list16 = b.list16;
    a.topo2 = b.topo2;
    a.stage = b.stage;
    a.stage_cnt = b.stage_cnt;
    a.err = b.err;
    a.g = g;
    a.rc2 = rc2;
    a.edge = edge;
    a.cull2 = cull2;
    a.n = n;
    a.cap = cap;
    hipLaunchKernelGGL(k_tile_build<TILE>, dim3(blocks_for(n, TILE)), dim3(TILE), 0, s, a);
}

template <int TILE, bool ENERGY, int MODE>
void tile_step(const TileArgs &a, hipStream_t s)
{
    TileArgs x = a;
    x.n_tiles = blocks_for(a.n, TILE);
    const int blocks = ((x.n_tiles + 7) / 8) * 8;
    hipLaunchKernelGGL((k_tile_step<TILE, ENERGY, MODE>), dim3(blocks), dim3(TILE), 0, s, x);
}

template <bool ENERGY, int MODE>
void tile_dispatch(int tile, const TileArgs &a, hipStream_t s)
{
    switch (tile) {
    case 64: tile_step<64, ENERGY, MODE>(a, s); break;
    case 128: tile_step<128, ENERGY, MODE>(a, s); break;
    default: tile_step<256, ENERGY, MODE>(a, s); break;
    }
}

}  // namespace

void launch_rebuild(const DevBufs &b, int cur, int n, int cap, int tile, const GridDev &g, float rc2,
                    float edge, hipStream_t s, bool advance_step_base, int list_every)
{
    hipLaunchKernelGGL(k_clear, dim3(blocks_for(g.n_cells, WG)), dim3(WG), 0, s, b.cell_count, g.n_cells);
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.pos[cur], n, g, b.traj_cell,
                       b.cell_count, b.cells, b.cell_of, b.err,
                       advance_step_base ? b.step_base : nullptr, b.step_next, list_every);
    // a cell whose box is farther than the cutoff plus a rounding margin
    // holds no partner
    const float rc = sqrtf(rc2) + 0.1f;
    const float cull2 = rc * rc;
    switch (tile) {
    case 64: rebuild_tile<64>(b, cur, n, cap, g, rc2, edge, cull2, s); break;
    case 128: rebuild_tile<128>(b, cur, n, cap, g, rc2, edge, cull2, s); break;
    default: rebuild_tile<256>(b, cur, n, cap, g, rc2, edge, cull2, s); break;
    }
}

void launch_step(const DevBufs &b, int cur, int n, int cap, int tile, const StepConsts &c,
                 const TipDev &tip, int has_pull, bool energy, int mode, const long long *step_base,
                 long long step_off, hipStream_t s)
{
    TileArgs a{};
    a.pin = b.pos[cur];
    a.pout = b.pos[cur ^ 1];
    a.trow = b.trow;
    a.tent = b.tent;
    a.list16 = b.list16;
    a.topo2 = b.topo2;
    a.list_cnt = b.list_cnt;
    a.stage = b.stage;
    a.stage_cnt = b.stage_cnt;
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
            tile_dispatch<true, 1>(tile, a, s);
        else
            tile_dispatch<false, 1>(tile, a, s);
    } else {
        if (energy)
            tile_dispatch<true, 0>(tile, a, s);
        else
            tile_dispatch<false, 0>(tile, a, s);
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
