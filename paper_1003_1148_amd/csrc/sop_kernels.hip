// HIP kernels for gfx950: Verlet-list rebuild on a wrapped cell grid, the
// fused per-step kernel (SOP forces of Eq. 1 over bonds, natives and the
// list; Philox4x32-10 Box-Muller noise; first-order overdamped update of
// Eq. 2 / Algorithm 7 with compensated single-precision positions), and the
// double-precision energy reduction.
#include <algorithm>
#include <type_traits>

#include "sop_internal.hpp"
#include "sop_rng.hpp"

namespace sop {

namespace {

constexpr int WG = 256;       // threads per workgroup (4 wave64)

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
// Cell index of one residue in the wrapped grid (the trajectory's offset
// keeps independent trajectories in separate cells).
__device__ __forceinline__ int cell_index(const float4 &p, const int4 &off, const GridDev &g)
{
    const int cx = wrap_cell(p.x, g.inv_cell, off.x, g.gx);
    const int cy = wrap_cell(p.y, g.inv_cell, off.y, g.gy);
    const int cz = wrap_cell(p.z, g.inv_cell, off.z, g.gz);
    return cx + g.gx * (cy + g.gy * cz);
}

// Bin one residue at high part p into the grid of the next skin search:
// its cell, a slot in that cell, and a copy of p there.
__device__ __forceinline__ void bin_one(const float4 &p, int i, int traj, const GridDev &g,
                                        const int4 *__restrict__ traj_cell, int *__restrict__ count,
                                        float4 *__restrict__ cells, int *__restrict__ cell_of,
                                        unsigned *__restrict__ err)
{
    const int c = cell_index(p, traj_cell[traj], g);
    cell_of[i] = c;
    const int slot = atomicAdd(&count[c], 1);
    if (slot < CELL_CAP)
        cells[(size_t)c * CELL_CAP + slot] = make_float4(p.x, p.y, p.z, __int_as_float(i));
    else
        atomicOr(err, ERR_CELL);
}

__global__ void k_clear(int *__restrict__ a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        a[i] = 0;
}

// Every residue binned at its current position.  The last step kernel of
// each list period bins the positions it writes; this kernel serves the
// rebuilds that do not follow such a step (after new coordinates, a new
// step count or a new tile size), after k_clear.
__global__ void k_bin_all(const float4 *__restrict__ pos, int n, GridDev g, const int4 *__restrict__ traj_cell,
                          int *__restrict__ count, float4 *__restrict__ cells, int *__restrict__ cell_of,
                          unsigned *__restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float4 p = pos[2 * i];
    if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z))
        atomicOr(err, ERR_NONFINITE);
    bin_one(p, i, __float_as_int(pos[2 * i + 1].w), g, traj_cell, count, cells, cell_of, err);
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
    float kf, inv_R0sq, R0sq, eh, eh12, el, el6, sg2, sg6, c6;
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
    k.sg6 = c.sigma2 * c.sigma2 * c.sigma2;
    k.c6 = k.el6 * k.sg6;  // force coefficient 6 eps_l sigma^6 / r^8
    return k;
}

// The force arithmetic of the pair and external terms states every fused
// multiply-add and lets the compiler fuse nothing else, so a term's force has
// the same bits in every kernel that evaluates it, whether or not that
// kernel also takes the term's energy (which shares its subexpressions).
__device__ __forceinline__ float len2(const float3 &d)
{
#pragma clang fp contract(off)
    return __builtin_fmaf(d.z, d.z, __builtin_fmaf(d.y, d.y, d.x * d.x));
}

__device__ __forceinline__ void acc_force(Acc &A, float c, const float3 &d)
{
    A.fx = __builtin_fmaf(c, d.x, A.fx);
    A.fy = __builtin_fmaf(c, d.y, A.fy);
    A.fz = __builtin_fmaf(c, d.z, A.fz);
}

// FENE: -(k R0^2/2) ln(1 - (r - r0)^2/R0^2); |r - r0| >= R0 sets `broken`.
__device__ __forceinline__ void add_fene_d(Acc &A, const float3 &d, float r0, const PairConsts &k, bool rec,
                                           bool &broken)
{
#pragma clang fp contract(off)
    const float rr = __builtin_amdgcn_sqrtf(len2(d));
    const float dl = rr - r0;
    float x = __builtin_fmaf(-(dl * dl), k.inv_R0sq, 1.0f);
    if (!(x > 0.0f)) {
        broken = true;
        x = 1.0f;
    }
    acc_force(A, -k.kf * dl * fast_rcp(x * rr), d);
    if (rec) {
        const double dd = (double)dl;
        const double R0sq = (double)k.R0sq;
        A.e_b += -0.5 * (double)k.kf * R0sq * log1p(-dd * dd / R0sq);
        A.vir += -(double)rr * (double)k.kf * dd / (1.0 - dd * dd / R0sq);
    }
}

// Native contact: eps_h [(r0/r)^12 - 2 (r0/r)^6].
__device__ __forceinline__ void add_native_d(Acc &A, const float3 &d, float r0, const PairConsts &k, bool rec)
{
#pragma clang fp contract(off)
    const float ir2 = fast_rcp(len2(d));
    const float s = r0 * r0 * ir2;
    const float q = s * s * s;
    const float w = __builtin_fmaf(q, q, -q);  // q^2 - q
    acc_force(A, k.eh12 * w * ir2, d);
    if (rec) {
        A.e_n += (double)(k.eh * __builtin_fmaf(q, q, -2.0f * q));
        A.vir += (double)(k.eh12 * w);
    }
}

// Soft repulsion: eps_l (sigma/r)^6.
__device__ __forceinline__ void add_repulsive_d(Acc &A, const float3 &d, const PairConsts &k, bool rec)
{
#pragma clang fp contract(off)
    const float ir2 = fast_rcp(len2(d));
    const float ir4 = ir2 * ir2;
    acc_force(A, k.c6 * ir4 * ir4, d);
    if (rec) {
        const float q = k.sg6 * ir4 * ir2;
        A.e_r += (double)(k.el * q);
        A.vir += (double)(k.el6 * q);
    }
}

// The list-pair form of the soft repulsion: accumulates d / r^8, so the
// caller multiplies the row's sum by 6 eps_l sigma^6 once instead of every
// pair; the energy and virial terms are the full ones.
__device__ __forceinline__ void add_repulsive_u(Acc &A, const float3 &d, const PairConsts &k, bool rec)
{
#pragma clang fp contract(off)
    const float ir2 = fast_rcp(len2(d));
    const float ir4 = ir2 * ir2;
    acc_force(A, ir4 * ir4, d);
    if (rec) {
        const float q = k.sg6 * ir4 * ir2;
        A.e_r += (double)(k.el * q);
        A.vir += (double)(k.el6 * q);
    }
}

// The same terms from compensated positions (hi, lo) of both residues.
__device__ __forceinline__ void add_fene(Acc &A, const float4 &hi, const float4 &lo, const float4 &hj,
                                         const float4 &lj, float r0, const PairConsts &k, bool rec,
                                         bool &broken)
{
    add_fene_d(A, pair_delta(hi, lo, hj, lj), r0, k, rec, broken);
}

__device__ __forceinline__ void add_native(Acc &A, const float4 &hi, const float4 &lo, const float4 &hj,
                                           const float4 &lj, float r0, const PairConsts &k, bool rec)
{
    add_native_d(A, pair_delta(hi, lo, hj, lj), r0, k, rec);
}

// Cantilever `pull` (index or -1) and tip on one residue at t_n = step*h.
__device__ __forceinline__ void add_external(Acc &A, double &e_x, double &f_rep, const float4 &hi,
                                             const float4 &lo, long long step, double h, int pull,
                                             const PullDev *pulls, const TipDev &tip, bool rec,
                                             unsigned *err)
{
#pragma clang fp contract(off)
    if (pull < 0 && !tip.on)
        return;
    const double tn = (double)step * h;
    const double px = (double)hi.x + (double)lo.x;
    const double py = (double)hi.y + (double)lo.y;
    const double pz = (double)hi.z + (double)lo.z;
    if (pull >= 0) {
        const PullDev pd = pulls[pull];
        const double dx = __builtin_fma(pd.v[0], tn, pd.anchor0[0]) - px;
        const double dy = __builtin_fma(pd.v[1], tn, pd.anchor0[1]) - py;
        const double dz = __builtin_fma(pd.v[2], tn, pd.anchor0[2]) - pz;
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
        const float dx = (float)(px - __builtin_fma(tip.v[0], tn, tip.c0[0]));
        const float dy = (float)(py - __builtin_fma(tip.v[1], tn, tip.c0[1]));
        const float dz = (float)(pz - __builtin_fma(tip.v[2], tn, tip.c0[2]));
        const float rr = sqrtf(len2(make_float3(dx, dy, dz)));
        const float gap = rr - (float)tip.radius;
        if (!(gap > 0.0f)) {
            atomicOr(err, ERR_TIP);
            return;
        }
        const float igap = fast_rcp(gap);
        const float sg = (float)tip.sigma * igap;
        const float s3 = sg * sg * sg;
        const float q = s3 * s3;
        const float mag_r = 6.0f * (float)tip.eps * q * igap * fast_rcp(rr);  // magnitude / r
        acc_force(A, mag_r, make_float3(dx, dy, dz));
        if (rec) {
            e_x += tip.eps * (double)q;
            if (tip.has_dir)
                f_rep += (double)(mag_r * dx) * tip.vhat[0] + (double)(mag_r * dy) * tip.vhat[1] +
                         (double)(mag_r * dz) * tip.vhat[2];
        }
    }
}

// Philox words of one residue and step: counter (index in the trajectory,
// stream id, step), key = seed.
__device__ __forceinline__ uint4 noise_words(unsigned tag, unsigned stream, long long step, const StepConsts &c)
{
    return philox10(make_uint4(tag & 0x7fffffffu, stream, (unsigned)step,
                               (unsigned)((unsigned long long)step >> 32)),
                    c.key0, c.key1);
}

// First-order update with the Gaussian components g:
// (hi, lo) <- TwoSum(hi, f h/zeta + g sqrt(2 kB T h/zeta) + lo) per axis.
__device__ __forceinline__ void update_with_noise(float4 &hi, float4 &lo, const Acc &A, const float g[3],
                                                  const StepConsts &c, unsigned *err)
{
#pragma clang fp contract(off)
    if (__float_as_uint(hi.w) >> 31)
        return;  // fixed residue
    float nh[3], nl[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float f = ax == 0 ? A.fx : (ax == 1 ? A.fy : A.fz);
        const float h0 = comp(hi, ax), l0 = comp(lo, ax);
        const float delta = __builtin_fmaf(c.c_drift, f, c.c_noise * g[ax]);
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

// Underdamped Langevin step (BAOAB): the velocity v stored between steps is
// the one before the last half kick of the previous step, so one kick of
// `kick` (h/m, or h/2m on the first step after velocities were set) with
// the force of this step covers that half kick and this step's first one;
// then x += (h/2) w, w = c1 w + c2 g, x += (h/2) w (compensated), v = w.
struct UdConsts {
    float kick, c1, c2, half_h;
};

__device__ __forceinline__ void underdamped_update(float4 &hi, float4 &lo, float4 &v, const Acc &A,
                                                   const float g[3], const UdConsts &u, unsigned *err)
{
#pragma clang fp contract(off)
    if (__float_as_uint(hi.w) >> 31) {
        v = make_float4(0.f, 0.f, 0.f, 0.f);  // fixed residue
        return;
    }
    float nh[3], nl[3], nv[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float f = ax == 0 ? A.fx : (ax == 1 ? A.fy : A.fz);
        const float w0 = __builtin_fmaf(u.kick, f, comp(v, ax));
        const float w1 = __builtin_fmaf(u.c1, w0, u.c2 * g[ax]);
        const float delta = __builtin_fmaf(u.half_h, w0, u.half_h * w1);
        const float h0 = comp(hi, ax), l0 = comp(lo, ax);
        const float y = delta + l0;
        const float t = h0 + y;
        const float bp = t - h0;
        const float ap = t - bp;
        nl[ax] = (h0 - ap) + (y - bp);
        nh[ax] = t;
        nv[ax] = w1;
    }
    if (!isfinite(nh[0]) || !isfinite(nh[1]) || !isfinite(nh[2]) || !isfinite(nv[0]) ||
        !isfinite(nv[1]) || !isfinite(nv[2]))
        atomicOr(err, ERR_NONFINITE);
    hi = make_float4(nh[0], nh[1], nh[2], hi.w);
    lo = make_float4(nl[0], nl[1], nl[2], lo.w);
    v = make_float4(nv[0], nv[1], nv[2], 0.0f);
}

// Noise (Section III.C) and the first-order update (Eq. 2 / Algorithm 7)
// with compensated positions.
__device__ __forceinline__ void langevin_update(float4 &hi, float4 &lo, const Acc &A, long long step,
                                                unsigned stream, const StepConsts &c, unsigned *err)
{
    const unsigned tag = __float_as_uint(hi.w);
    if (tag >> 31)
        return;  // fixed residue
    const uint4 w = noise_words(tag, stream, step, c);
    const float2 gxy = gaussian_pair(w);
    const float g[3] = {gxy.x, gxy.y, gaussian_axis(w, 2)};
    update_with_noise(hi, lo, A, g, c, err);
}

// ---------------------------------------------------------------------------
// Plain schedule, tile staging: at each rebuild, the residues a tile of
// consecutive residues interacts with (list partners, bonded and native
// partners, itself) become a sorted set of at most stage_max slots, and
// rows are rewritten as 16-bit slots into that set.
// ---------------------------------------------------------------------------
template <int TILE>
constexpr int stage_max() { return 4096; }
// Slots held in LDS at once by the kernels that read the staging set; a
// tile with more slots is taken in windows of this many.
template <int TILE>
constexpr int stage_win() { return TILE >= 256 ? 2048 : 1024; }
// Row padding (and the slot of a bonded/native entry of a failed tile).
constexpr unsigned short EMPTY_SLOT = 0xffffu;

// Candidate residues (the residues of the cells around a tile) held in LDS
// at once during a rebuild; more are taken in windows of whole cells.  Small
// tiles keep less so that five workgroups fit a CU.
template <int TILE>
constexpr int cand_win() { return TILE == 64 ? 896 : 1024; }
// Distinct cells around one tile, and the bits of its open-addressing table.
template <int TILE>
constexpr int cells_max() { return TILE >= 256 ? 512 : (TILE >= 128 ? 1024 : 640); }
template <int TILE>
constexpr int chash_bits() { return TILE == 128 ? 11 : 10; }
constexpr int EXTRA_MAX = 128;  // bonded/native partners outside the tile's cells
constexpr int TREG = 8;  // bonded/native entries per residue kept in registers during a search (more: global)

struct BuildArgs {
    const int *tile_first;  // first residue of each tile, then n
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
    const unsigned *skin_flag;
    float4 *hi_skin;
    unsigned long long *stats;
    long long *step_base;  // graph replays: advanced once per rebuild, or NULL
    long long *step_next;
    GridDev g;
    float rc2;
    int n, cap, period;
};

// Exclusive prefix sum over the NT lanes of a workgroup (all lanes call it).
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int *part, int &total)
{
    const int t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        const int x = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    total = part[NT - 1];
    const int r = part[t] - v;
    __syncthreads();
    return r;
}

// Along one axis of the wrapped grid (n >= 3 cells), cell c is u's own or an
// adjacent one.
__device__ __forceinline__ bool adjacent_cell(int c, int u, int n)
{
    const int d = c - u;
    return (unsigned)(d + 1) <= 2u || d == n - 1 || d == 1 - n;
}

// OR of a 32-bit value over the 64 lanes of a wave.
__device__ __forceinline__ unsigned wave_or(unsigned v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v |= (unsigned)__shfl_xor((int)v, off, 64);
    return v;
}

// Bonded/native entry codes while a tile is built.
constexpr unsigned CODE_NONE = 0xffffffffu;     // partner not found yet
constexpr unsigned CODE_WINDOW = 0x80000000u;   // | candidate index in the current window
constexpr unsigned CODE_EXTRA = 0x40000000u;    // | index among the extra slots

// One workgroup of 256 lanes per tile of TILE consecutive residues; lane t
// serves residue t % TILE and part q = t / TILE of its work (NLB = 256/TILE
// parts).
//  1. The cells around the tile's residues (each residue's own and adjacent
//     cells) go into an LDS hash table and are sorted by cell index; their
//     residues, sorted by (cell, residue index), are the tile's candidates.
//  2. Per window of whole cells (at most cand_win candidates, usually one
//     window): candidates go to LDS; each residue is tested against them 32
//     at a time with the single-precision predicate r < r_list of
//     Algorithm 3, one bit per candidate, part q taking a contiguous range
//     of the 32-candidate words (words outside every neighbourhood of a wave
//     are skipped).  Self, bonded and native partners are cleared; the
//     candidates some row or entry uses get the next staging slots in sorted
//     order; each part appends its words' partners to the row at the offset
//     the lower parts leave.
//  3. Bonded/native partners outside the cells take extra slots at the end.
// A row lists its partners in (cell, residue index) order whatever the tile
// size or the order in which residues were binned.
template <int TILE, bool MULTI>
__global__ __launch_bounds__(256, TILE == 64 ? 5 : 2) void k_tile_build(BuildArgs a)
{
    constexpr int NT = 256, NLB = NT / TILE;
    constexpr int SM = stage_max<TILE>();
    constexpr int CM = cand_win<TILE>();
    constexpr int NW = CM / 32;
    constexpr int CELLS_MAX = cells_max<TILE>();
    constexpr int CHASH_BITS = chash_bits<TILE>();
    constexpr int CHASH = 1 << CHASH_BITS;
    static_assert(NW * TILE >= CM, "arrival ids alias the row bits");
    // Step 1 (cell table) and step 2 (candidates, row bits) share one region.
    constexpr int P1 = (CHASH + CELLS_MAX) * 4, P2 = CM * 16 + NW * TILE * 4;
    __shared__ __align__(16) unsigned char shared_region[P1 > P2 ? P1 : P2];
    int *hkey = reinterpret_cast<int *>(shared_region);               // step 1: open addressing
    int *ccell = reinterpret_cast<int *>(shared_region + CHASH * 4);  // step 1: arrival order
    float4 *cand = reinterpret_cast<float4 *>(shared_region);         // step 2: window, sorted
    unsigned *bits = reinterpret_cast<unsigned *>(shared_region + CM * 16);  // row bits, word-major
    __shared__ unsigned sxyz[CELLS_MAX];  // sorted cells: packed coordinates
    __shared__ int cbase[CELLS_MAX + 1];
    __shared__ unsigned used[NW];
    __shared__ int wbase[NW];
    __shared__ short wlo[NW], whi[NW];    // sorted cells spanned by each word
    __shared__ short pcnt[NT];            // partners of (part, residue) in this window
    __shared__ int rowbase[TILE];         // partners of the residue in earlier windows
    __shared__ int extra[EXTRA_MAX];
    __shared__ int part[NT];
    __shared__ int n_cu, n_extra, bad_cells, n_used_w;

    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // every rebuild starts here (the kernels after it do not read these)
        ++a.stats[0];
        if (a.step_base) {
            // graph replays: this rebuild starts the next list period
            const long long nb = *a.step_next;
            *a.step_base = nb;
            *a.step_next = nb + a.period;
        }
    }
    if (*a.skin_flag == 0u)
        return;  // the skin rows are still valid (uniform over the grid)
    const int tile = blockIdx.x, t = threadIdx.x;
    const int rho = t % TILE, q = t / TILE;
    const int first = a.tile_first[tile], tcnt = a.tile_first[tile + 1] - first;
    const int i = first + rho;
    const bool act = rho < tcnt;
    const bool lead = act && q == 0;  // writes the residue's count and padding
    const GridDev g = a.g;
    if (tile == 0 && t == 0)
        ++a.stats[1];
    if (lead)
        a.hi_skin[i] = a.pos[2 * i];  // the displacement check's reference
    for (int h = t; h < CHASH; h += NT)
        hkey[h] = -1;
    if (t < TILE)
        rowbase[t] = 0;
    if (t == 0) {
        n_cu = 0;
        n_extra = 0;
        bad_cells = 0;
    }
    __syncthreads();

    auto hslot = [](int key) { return (int)(((unsigned)key * 2654435761u) >> (32 - CHASH_BITS)); };

    // ---- 1. cells around the tile ----
    // independent loads first; this part's bonded/native entries (u = q mod
    // NLB, the first TREG kept in registers) and their partners' cells are
    // needed only in step 2
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    int own = 0;
    int2 row = make_int2(0, 0);
    if (act) {
        p = a.pos[2 * i];
        own = a.cell_of[i];
        row = a.trow[i];
    }
    const int ntop = (row.y & 4095) + (row.y >> 12);
    // entry e = v * NLB + q of the first TREG is this part's v-th
    constexpr int TPP = TREG / NLB;
    int tj[TPP], tm[TPP];
    unsigned tr0[TPP], tcode[TPP];
#pragma unroll
    for (int v = 0; v < TPP; ++v) {
        const int e = v * NLB + q;
        const float2 te = e < ntop ? a.tent[row.x + e] : make_float2(0.0f, 0.0f);
        tj[v] = __float_as_int(te.x);
        tr0[v] = __float_as_uint(te.y);
        tcode[v] = CODE_NONE;
    }
#pragma unroll
    for (int v = 0; v < TPP; ++v)
        tm[v] = v * NLB + q < ntop ? a.cell_of[tj[v]] : -1;
    const int tlo = (MULTI && act) ? a.traj_lo[i] : 0, thi = (MULTI && act) ? a.traj_hi[i] : 0;
    // own wrapped cell coordinates
    const int ux = own % g.gx, uy = (own / g.gx) % g.gy, uz = own / (g.gx * g.gy);
    if (act) {
        for (int d = q; d < 27; d += NLB) {
            const int cx = ux + d % 3 - 1, cy = uy + (d / 3) % 3 - 1, cz = uz + d / 9 - 1;
            const int cid = (cx < 0 ? cx + g.gx : (cx >= g.gx ? cx - g.gx : cx)) +
                            g.gx * ((cy < 0 ? cy + g.gy : (cy >= g.gy ? cy - g.gy : cy)) +
                                    g.gy * (cz < 0 ? cz + g.gz : (cz >= g.gz ? cz - g.gz : cz)));
            int h = hslot(cid);
            for (int probe = 0; probe < CHASH; ++probe) {
                const int prev = atomicCAS(&hkey[h], -1, cid);
                if (prev == -1) {
                    const int m = atomicAdd(&n_cu, 1);
                    if (m < CELLS_MAX)
                        ccell[m] = cid;
                    else
                        bad_cells = 1;
                    break;
                }
                if (prev == cid)
                    break;
                h = (h + 1) & (CHASH - 1);
                if (probe == CHASH - 1)
                    bad_cells = 1;
            }
        }
    }
    __syncthreads();
    uint2 *trw = a.topo2 + (size_t)tile * TOPO_CAP * TILE + rho;
    auto fail_tile = [&]() {
        // report; leave the tile pointing at the empty slot so steps stay in bounds
        if (t == 0) {
            atomicOr(a.err, ERR_STAGE);
            a.stage_cnt[tile] = 0;
        }
        if (lead) {
            a.list_cnt[i] = 0;
            for (int e = 0; e < ntop; ++e)
                trw[(size_t)e * TILE] = make_uint2((unsigned)EMPTY_SLOT, __float_as_uint(1.0f));
        }
    };
    if (bad_cells) {
        fail_tile();
        return;  // uniform: read after a barrier, written only before it
    }
    const int NC = n_cu;
    // coordinates packed in bx + by + bz <= 32 bits (the grid has at most 2^21 cells)
    const int bx = 32 - __clz(g.gx), by = 32 - __clz(g.gy);
    const unsigned mx = (1u << bx) - 1u, my = (1u << by) - 1u;
    auto cell_id = [&](unsigned v) { return (int)(v & mx) + g.gx * ((int)((v >> bx) & my) + g.gy * (int)(v >> (bx + by))); };
    // sort the cells by index (rank by counting; indices are distinct)
    for (int m = t; m < NC; m += NT) {
        const int c = ccell[m];
        int r = 0;
        for (int m2 = 0; m2 < NC; ++m2)
            r += ccell[m2] < c;
        sxyz[r] = (unsigned)(c % g.gx) | ((unsigned)((c / g.gx) % g.gy) << bx) |
                  ((unsigned)(c / (g.gx * g.gy)) << (bx + by));
    }
    __syncthreads();
    auto lookup = [&](int key) -> int {  // sorted number of cell `key`, or -1
        int lo = 0, hi = NC;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cell_id(sxyz[mid]) < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        return (lo < NC && cell_id(sxyz[lo]) == key) ? lo : -1;
    };
    // candidate counts -> cbase (exclusive prefix in sorted cell order)
    {
        const int cper = (NC + NT - 1) / NT;
        const int m0 = min(NC, t * cper), m1 = min(NC, m0 + cper);
        int csum = 0;
        for (int m = m0; m < m1; ++m) {
            const int c = min(a.count[cell_id(sxyz[m])], CELL_CAP);
            cbase[m] = c;
            csum += c;
        }
        int M = 0;
        int cb = block_exclusive_scan<NT>(csum, part, M);
        for (int m = m0; m < m1; ++m) {
            const int c = cbase[m];
            cbase[m] = cb;
            cb += c;
        }
        if (t == 0)
            cbase[NC] = M;
    }
    // entries beyond TREG live in the topology output meanwhile; entry
    // e >= TREG belongs to part (e - TREG) mod NLB throughout
    if (act)
        for (int e = TREG + q; e < ntop; e += NLB)
            trw[(size_t)e * TILE] = make_uint2(CODE_NONE, __float_as_uint(a.tent[row.x + e].y));
    __syncthreads();
    // partners' cells -> sorted cell numbers (or -1 outside the tile's cells)
#pragma unroll
    for (int v = 0; v < TPP; ++v)
        tm[v] = tm[v] >= 0 ? lookup(tm[v]) : -1;
    const int own_m = lead ? lookup(own) : -1;
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

    // ---- 2. windows of whole cells ----
    int *st = a.stage + (size_t)tile * SM;
    unsigned short *lrow = a.list16 + (size_t)i * a.cap;  // rows are residue-major
    auto row_store = [&](int k, unsigned short sl) {  // entry k of the residue's row
        if (k < a.cap)
            lrow[k] = sl;
    };
    int slot_base = 0;
    int *aid = reinterpret_cast<int *>(bits);
    for (int mA = 0; mA < NC;) {
        int mB = mA + 1;  // a cell holds at most CELL_CAP <= CM residues
        {
            int hi = NC;
            while (mB < hi) {
                const int mid = (mB + hi + 1) >> 1;
                if (cbase[mid] - cbase[mA] <= CM)
                    mB = mid;
                else
                    hi = mid - 1;
            }
        }
        const int base = cbase[mA], Mw = cbase[mB] - base;
        constexpr int CPT = (CM + NT - 1) / NT;  // candidates per lane
        float4 cv[CPT];
        int cm[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int ci = t + u * NT;
            cm[u] = ci < Mw ? segment_of(base + ci) : 0;
            cv[u] = ci < Mw ? a.cells[(size_t)cell_id(sxyz[cm[u]]) * CELL_CAP + (base + ci - cbase[cm[u]])]
                            : make_float4(0.f, 0.f, 0.f, 0.f);
            if (ci < Mw)
                aid[ci] = __float_as_int(cv[u].w);
        }
        for (int w = t; w < NW; w += NT)
            used[w] = 0u;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int ci = t + u * NT;
            if (ci < Mw) {
                const int id = __float_as_int(cv[u].w);
                const int k0 = cbase[cm[u]] - base, k1 = cbase[cm[u] + 1] - base;
                int r = k0, k = k0;
                for (; k + 4 <= k1; k += 4) {
                    const int a0 = aid[k], a1 = aid[k + 1], a2 = aid[k + 2], a3 = aid[k + 3];
                    r += (a0 < id) + (a1 < id) + (a2 < id) + (a3 < id);
                }
                for (; k < k1; ++k)
                    r += aid[k] < id;
                cand[r] = cv[u];
            }
        }
        const int NWm = (Mw + 31) >> 5;
        for (int w = t; w < NWm; w += NT) {
            wlo[w] = (short)segment_of(base + 32 * w);
            whi[w] = (short)segment_of(base + min(32 * w + 31, Mw - 1));
        }
        __syncthreads();
        // row bits; part q takes words [w0, w1) (uniform over a wave)
        const int wpp = (NWm + NLB - 1) / NLB;
        const int w0 = min(NWm, q * wpp), w1 = min(NWm, w0 + wpp);
        for (int w = w0; w < w1; ++w) {
            bool reach = false;
            if (act)
                for (int m = wlo[w]; m <= whi[w]; ++m) {
                    const unsigned v = sxyz[m];
                    reach |= adjacent_cell((int)(v & mx), ux, g.gx) &&
                             adjacent_cell((int)((v >> bx) & my), uy, g.gy) &&
                             adjacent_cell((int)(v >> (bx + by)), uz, g.gz);
                }
            unsigned word = 0u;
            if (__any(reach)) {
                // branch-free: BB LDS reads in flight, then the tests; the
                // window's tail and inactive lanes are masked afterwards
                constexpr int BB = TILE == 64 ? 4 : 8;
#pragma unroll 1
                for (int k0 = 0; k0 < 32; k0 += BB) {
                    float4 c8[BB];
#pragma unroll
                    for (int u = 0; u < BB; ++u)
                        c8[u] = cand[32 * w + k0 + u];
#pragma unroll
                    for (int u = 0; u < BB; ++u) {
                        bool pass = within_cutoff(p, c8[u], a.rc2);
                        if (MULTI) {
                            const int j = __float_as_int(c8[u].w);
                            pass = pass & (j >= tlo) & (j < thi);
                        }
                        word |= (unsigned)pass << (k0 + u);
                    }
                }
                const int left = Mw - 32 * w;
                word &= act ? (left >= 32 ? 0xffffffffu : ((1u << left) - 1u)) : 0u;
                const unsigned u = wave_or(word);
                if ((t & 63) == 0 && u)
                    atomicOr(&used[w], u);
            }
            bits[w * TILE + rho] = word;
        }
        __syncthreads();
        // self, bonded and native partners in this window: clear their bits
        // (their candidates are marked used: a partner's slot is needed anyway)
        auto find = [&](int j, int m) -> int {  // window candidate of residue j in sorted cell m, or -1
            if (m < mA || m >= mB)
                return -1;
            int lo = cbase[m] - base, hi = cbase[m + 1] - base;
            const int end = hi;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (__float_as_int(cand[mid].w) < j)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            return (lo < end && __float_as_int(cand[lo].w) == j) ? lo : -1;
        };
        auto take = [&](int r) {
            atomicAnd(&bits[(r >> 5) * TILE + rho], ~(1u << (r & 31)));
            atomicOr(&used[r >> 5], 1u << (r & 31));
        };
        if (lead) {
            const int rs = find(i, own_m);
            if (rs >= 0)
                atomicAnd(&bits[(rs >> 5) * TILE + rho], ~(1u << (rs & 31)));
        }
        if (act) {
            for (int e = TREG + q; e < ntop; e += NLB) {
                if (trw[(size_t)e * TILE].x != CODE_NONE)
                    continue;
                const int j = __float_as_int(a.tent[row.x + e].x);
                const int r = find(j, lookup(a.cell_of[j]));
                if (r >= 0) {
                    take(r);
                    trw[(size_t)e * TILE].x = CODE_WINDOW | (unsigned)r;
                }
            }
        }
#pragma unroll
        for (int v = 0; v < TPP; ++v) {
            if (v * NLB + q < ntop && tcode[v] == CODE_NONE) {
                const int r = find(tj[v], tm[v]);
                if (r >= 0) {
                    take(r);
                    tcode[v] = CODE_WINDOW | (unsigned)r;
                }
            }
        }
        __syncthreads();
        // slots of the used candidates: prefix over the window's words (<= 32);
        // row counts of each part
        if (t < 64) {
            const int c = t < NWm ? __popc(used[t]) : 0;
            int v = c;
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(v, off, 64);
                if (t >= off)
                    v += y;
            }
            if (t < NWm)
                wbase[t] = slot_base + v - c;
            if (t == 63)
                n_used_w = v;
        }
        {
            int c = 0;
            for (int w = w0; w < w1; ++w)
                c += __popc(bits[w * TILE + rho]);
            pcnt[t] = (short)c;
        }
        __syncthreads();
        const int nu = n_used_w;
        if (slot_base + nu > SM) {
            fail_tile();
            return;  // uniform
        }
        // staging: each used candidate of the window takes the next slot in
        // sorted order (all lanes, one candidate each)
        for (int ci = t; ci < Mw; ci += NT) {
            const unsigned uw = used[ci >> 5];
            if ((uw >> (ci & 31)) & 1u)
                st[wbase[ci >> 5] + __popc(uw & ((1u << (ci & 31)) - 1u))] = __float_as_int(cand[ci].w);
        }
        if (act) {
            // this part's partners, after those of the lower parts
            int k = rowbase[rho];
            for (int pq = 0; pq < q; ++pq)
                k += pcnt[pq * TILE + rho];
            for (int w = w0; w < w1; ++w) {
                unsigned b = bits[w * TILE + rho];
                const unsigned uw = used[w];
                const int wb = wbase[w];
                while (b) {
                    const int kb = __ffs(b) - 1;
                    b &= b - 1u;
                    row_store(k++, (unsigned short)(wb + __popc(uw & ((1u << kb) - 1u))));
                }
            }
            auto slot_of = [&](unsigned v) {
                const int r = (int)(v & ~CODE_WINDOW), w = r >> 5;
                return (unsigned)(wbase[w] + __popc(used[w] & ((1u << (r & 31)) - 1u)));
            };
#pragma unroll
            for (int v = 0; v < TPP; ++v)
                if (tcode[v] != CODE_NONE && (tcode[v] & CODE_WINDOW))
                    tcode[v] = slot_of(tcode[v]);
            for (int e = TREG + q; e < ntop; e += NLB) {
                const unsigned v = trw[(size_t)e * TILE].x;
                if (v != CODE_NONE && (v & CODE_WINDOW))
                    trw[(size_t)e * TILE].x = slot_of(v);
            }
        }
        slot_base += nu;
        mA = mB;
        __syncthreads();  // the window's buffers are reused
        if (lead) {
            int c = rowbase[rho];
            for (int pq = 0; pq < NLB; ++pq)
                c += pcnt[pq * TILE + rho];
            rowbase[rho] = c;
        }
    }

    // ---- 3. partners outside the cells ----
    if (act) {
#pragma unroll
        for (int v = 0; v < TPP; ++v)
            if (v * NLB + q < ntop && tcode[v] == CODE_NONE) {
                const int k = atomicAdd(&n_extra, 1);
                if (k < EXTRA_MAX)
                    extra[k] = tj[v];
                tcode[v] = CODE_EXTRA | (unsigned)k;
            }
        for (int e = TREG + q; e < ntop; e += NLB)
            if (trw[(size_t)e * TILE].x == CODE_NONE) {
                const int k = atomicAdd(&n_extra, 1);
                if (k < EXTRA_MAX)
                    extra[k] = __float_as_int(a.tent[row.x + e].x);
                trw[(size_t)e * TILE].x = CODE_EXTRA | (unsigned)k;
            }
    }
    __syncthreads();
    const int n_ex = n_extra;
    const int S = slot_base + min(n_ex, EXTRA_MAX);
    if (S > SM || n_ex > EXTRA_MAX) {
        fail_tile();
        return;  // uniform
    }
    for (int k = t; k < n_ex; k += NT)
        st[slot_base + k] = extra[k];
    if (t == 0)
        a.stage_cnt[tile] = S;
    if (!act)
        return;
    auto final_slot = [&](unsigned v) {
        return ((v & CODE_WINDOW) == 0 && (v & CODE_EXTRA)) ? (unsigned)slot_base + (v & ~CODE_EXTRA) : v;
    };
#pragma unroll
    for (int v = 0; v < TPP; ++v)
        if (v * NLB + q < ntop)
            trw[(size_t)(v * NLB + q) * TILE] = make_uint2(final_slot(tcode[v]), tr0[v]);
    for (int e = TREG + q; e < ntop; e += NLB)
        trw[(size_t)e * TILE].x = final_slot(trw[(size_t)e * TILE].x);
    if (!lead)
        return;
    // count; the last chunk padded with the empty slot
    const int cnt = rowbase[rho];
    for (int k = cnt; k < ((cnt + 3) & ~3); ++k)
        row_store(k, EMPTY_SLOT);
    a.list_cnt[i] = cnt;
    if (cnt > a.cap)
        atomicOr(a.err, ERR_OVERFLOW);
}

// ---------------------------------------------------------------------------
// List from the skin rows: every list_every steps each residue's skin row
// (its partners within r_list + skin at the last skin build, in slot order)
// is filtered with the single-precision predicate r < r_list of Algorithm 3
// on the current positions.  The skin build runs again before the filter
// whenever some residue has moved more than skin/2 since the last one, so
// every pair within r_list is in the skin rows and the filtered rows equal a
// rebuild from all pairs, entry for entry in the same order.
// ---------------------------------------------------------------------------
struct FilterArgs {
    const int *tile_first;
    const float4 *pos;
    const int *stage;
    const int *stage_cnt;
    const unsigned short *skin16;
    const int *skin_cnt;
    unsigned short *list16;
    int *list_cnt;
    int *cell_count;
    unsigned *skin_flag;
    unsigned char *tile_ord;  // per tile: its residues by decreasing list length
    const unsigned short *skin_ord;  // per tile: 1 + its residues by decreasing skin row length
    float rc2;
    int cap, n_cells;
};

template <int TILE>
__global__ __launch_bounds__(256, TILE == 64 ? 5 : (TILE == 128 ? 3 : 2)) void k_filter(FilterArgs a)
{
    constexpr int NL = 256 / TILE;  // lanes per residue, adjacent in the wave
    constexpr int SM = stage_max<TILE>();
    constexpr int SW = stage_win<TILE>();
    // filtered entries of a residue gathered in LDS (a multiple of 8, so
    // rows start 16-byte aligned); sized so that 64-residue tiles fit five
    // workgroups per CU
    constexpr int OUTW = TILE == 64 ? 184 : (TILE == 128 ? 96 : 48);
    constexpr int PF = 6;      // row pieces per lane loaded up front
    constexpr int MAXP = 128;  // pieces of 8 entries in a row (cap <= 1024)
    // the staged positions (predicate) and the gathered rows (emit) share
    // one region
    constexpr int HS_B = SW * 16, OUT_B = TILE * OUTW * 2;
    __shared__ __align__(16) unsigned char region[HS_B > OUT_B ? HS_B : OUT_B];
    float4 *hs = reinterpret_cast<float4 *>(region);
    unsigned short *out_s = reinterpret_cast<unsigned short *>(region);
    __shared__ int lens[TILE];
    __shared__ unsigned char pbits[TILE * MAXP];  // passing entries of each piece
    const int tile = blockIdx.x, t = threadIdx.x;
    const int q = t % NL;
    // the cell counts are read only by the skin build, which is done: clear
    // them for the next one; the flag is read only by the skin build too
    for (int k = tile * 256 + t; k < a.n_cells; k += gridDim.x * 256)
        a.cell_count[k] = 0;
    if (tile == 0 && t == 0)
        *a.skin_flag = 0u;
    const int first = a.tile_first[tile], tcnt = a.tile_first[tile + 1] - first;
    const int S = min(a.stage_cnt[tile], SM);
    const int *st = a.stage + (size_t)tile * SM;
    // the residue of this lane group: rows longest first (the order of the
    // last skin search)
    const bool act = t / NL < tcnt;
    const int ord = act ? (int)a.skin_ord[(size_t)tile * TILE + t / NL] : 0;
    const int rho = act ? (ord > 0 ? ord - 1 : t / NL) : t / NL;
    const int i = first + (act ? rho : 0);
    const int len = act ? min(a.skin_cnt[i], a.cap) : 0;
    // the row in 16-byte pieces of 8 entries, piece m NL + q to lane q, so
    // a residue's lanes read 16 NL contiguous bytes per round; the first PF
    // pieces of this lane are loaded before the staging
    const uint4 *src = reinterpret_cast<const uint4 *>(a.skin16 + (size_t)i * a.cap);
    const int npc = (len + 7) >> 3;
    uint4 pre[PF];
#pragma unroll
    for (int m = 0; m < PF; ++m)
        pre[m] = m * NL + q < npc ? src[m * NL + q] : make_uint4(0u, 0u, 0u, 0u);
    const float4 pi = a.pos[2 * i];
    unsigned char *pb = pbits + rho * MAXP;
    // passing entries of this lane's first PF pieces, eight bits a piece, in
    // registers; later pieces (rows longer than 8 PF NL entries) in LDS
    unsigned pbr[(PF + 3) / 4] = {};
    // the predicate, window by window of the staging set (one window for
    // nearly every tile): each entry is tested in the window holding its slot
    const bool one_win = S <= SW;
    for (int w0 = 0; w0 < S || w0 == 0; w0 += SW) {
        const int wn = min(SW, S - w0);
        if (w0 > 0)
            __syncthreads();  // the previous window's readers are done
        for (int sl = t; sl < wn; sl += 256)
            hs[sl] = a.pos[2 * st[w0 + sl]];
        __syncthreads();
        // branch-free: the eight staged positions are read, then all eight
        // are tested and the results masked.  One window (nearly every
        // tile): every entry of the row is a staged slot, and entries past
        // the row's end (masked afterwards) are clamped into the window.
        // Several windows: an entry outside the current one reads slot 0
        // and is masked.
        auto test = [&](const uint4 &w, int pc) -> unsigned {
            const unsigned ws[4] = {w.x, w.y, w.z, w.w};
            const int valid = len - pc * 8;
            const unsigned tail = valid >= 8 ? 0xffu : (valid > 0 ? (1u << valid) - 1u : 0u);
            unsigned ok = 0u, bits = 0u;
#pragma unroll
            for (int h = 0; h < 8; h += 4) {  // four reads in flight, then their tests
                float4 pj[4];
#pragma unroll
                for (int u = h; u < h + 4; ++u) {
                    const unsigned sl = (ws[u >> 1] >> ((u & 1) * 16)) & 0xffffu;
                    const int e = (int)sl - w0;
                    const bool in = one_win || (unsigned)e < (unsigned)wn;
                    ok |= (unsigned)in << u;
                    pj[u - h] = hs[one_win ? min(sl, (unsigned)(SW - 1)) : (in ? (unsigned)e : 0u)];
                }
#pragma unroll
                for (int u = h; u < h + 4; ++u)
                    bits |= (unsigned)within_cutoff(pi, pj[u - h], a.rc2) << u;
            }
            return bits & ok & tail;
        };
#pragma unroll
        for (int m = 0; m < PF; ++m)
            if (m * NL + q < npc)
                pbr[m >> 2] |= test(pre[m], m * NL + q) << (8 * (m & 3));
        for (int pc = PF * NL + q; pc < npc; pc += NL) {
            const unsigned bits = test(src[pc], pc);
            pb[pc] = (unsigned char)(w0 == 0 ? bits : (bits | pb[pc]));
        }
    }
    // the row's passing entries, over the residue's lanes
    int tot = 0;
#pragma unroll
    for (int k = 0; k < (PF + 3) / 4; ++k)
        tot += __popc(pbr[k]);
    for (int pc = PF * NL + q; pc < npc; pc += NL)
        tot += __popc((unsigned)pb[pc]);
#pragma unroll
    for (int off = 1; off < NL; off <<= 1)
        tot += __shfl_xor(tot, off, NL);
    __syncthreads();  // the staged positions are dead: the region takes the rows
    unsigned short *dst = a.list16 + (size_t)i * a.cap;
    // rows that fit (padding included) are gathered in LDS and written out
    // in 16-byte pieces
    const bool in_lds = ((tot + 7) & ~7) <= OUTW;
    unsigned short *ob_l = out_s + rho * OUTW;  // LDS
    int rounds = (npc + NL - 1) / NL;
#pragma unroll
    for (int off = 1; off < NL; off <<= 1)
        rounds = max(rounds, __shfl_xor(rounds, off, NL));  // uniform over the residue's lanes
    int base = 0;
    auto emit = [&](const uint4 &w, unsigned bits) {
        const unsigned ws[4] = {w.x, w.y, w.z, w.w};
        const int c = __popc(bits);
        // passing entries before this lane's piece: scan over the residue's lanes
        int v = c;
#pragma unroll
        for (int off = 1; off < NL; off <<= 1) {
            const int y = __shfl_up(v, off, NL);
            if (q >= off)
                v += y;
        }
        const int o = base + v - c;
        // passing entry u goes to o + (passing entries before it): unrolled
        // stores, LDS for rows that fit, else straight to the list
        if (in_lds) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if ((bits >> u) & 1u)
                    ob_l[o + __popc(bits & ((1u << u) - 1u))] =
                        (unsigned short)((ws[u >> 1] >> ((u & 1) * 16)) & 0xffffu);
        } else {
            for (int k = o; bits; ++k) {
                const int u = __ffs(bits) - 1;
                bits &= bits - 1u;
                dst[k] = (unsigned short)((ws[u >> 1] >> ((u & 1) * 16)) & 0xffffu);
            }
        }
        base += __shfl(v, NL - 1, NL);
    };
#pragma unroll
    for (int m = 0; m < PF; ++m)
        if (m < rounds)
            emit(pre[m], (pbr[m >> 2] >> (8 * (m & 3))) & 0xffu);
    for (int m = PF; m < rounds; ++m) {
        const int pc = m * NL + q;
        emit(pc < npc ? src[pc] : make_uint4(0u, 0u, 0u, 0u), pc < npc ? (unsigned)pb[pc] : 0u);
    }
    if (act && q == NL - 1) {
        // pad the row to a multiple of 8 entries: with the LDS slot of the
        // far-away position when the tile fits one window, else the empty slot
        const unsigned short pad = S <= SW ? (unsigned short)SW : EMPTY_SLOT;
        for (int k = base; k < ((base + 7) & ~7); ++k) {
            if (in_lds)
                ob_l[k] = pad;
            else
                dst[k] = pad;
        }
        a.list_cnt[i] = base;
        lens[rho] = base;
    }
    __syncthreads();
    if (act && in_lds) {
        const uint4 *sp = reinterpret_cast<const uint4 *>(out_s + rho * OUTW);
        uint4 *dp = reinterpret_cast<uint4 *>(dst);
        for (int pc = q; pc < ((base + 7) >> 3); pc += NL)
            dp[pc] = sp[pc];
    }
    // the step kernel hands the rows to its waves longest first, so that the
    // rows a wave sums have about the same length (ties in index order):
    // the residue's rank, counted by its NL lanes over a share of the tile
    int r = 0;
    if (act)
        for (int u = q * (TILE / NL); u < min(tcnt, (q + 1) * (TILE / NL)); ++u)
            r += (lens[u] > base || (lens[u] == base && u < rho)) ? 1 : 0;
#pragma unroll
    for (int off = 1; off < NL; off <<= 1)
        r += __shfl_xor(r, off, NL);
    if (act && q == 0)
        a.tile_ord[(size_t)tile * TILE + r] = (unsigned char)rho;
}

// ---------------------------------------------------------------------------
// Canonical order after a skin search: a tile's slots are renumbered in the
// order of their residues' global ids, and every skin row is rewritten in
// ascending slot order, so each row lists its partners by ascending residue
// id whatever the cell grid.  The list rows the filter derives keep that
// order, so the order in which a residue's pair terms are summed depends on
// its list alone, not on when or with which skin the last search ran.
// ---------------------------------------------------------------------------
struct CanonArgs {
    const int *tile_first;
    const int2 *trow;
    int *stage;
    const int *stage_cnt;
    unsigned short *skin16;
    const int *skin_cnt;
    uint2 *topo2;
    const unsigned *skin_flag;
    unsigned short *skin_ord;
    int cap;
};

template <int TILE>
__global__ __launch_bounds__(256) void k_canon(CanonArgs a)
{
    constexpr int SM = stage_max<TILE>();
    constexpr int G = 32;           // residues per pass
    constexpr int NLG = 256 / G;    // lanes per residue in a pass
    constexpr int MW = SM / 32;     // mask words per residue
    constexpr int MWP = MW + 1;     // their stride: a residue's word w in another bank than its neighbour's
    constexpr int BW = 2048;        // bitmap words: ids spanning up to 65,536 values
    // the ranks (ids, bitmap, word prefixes) and the row masks use one
    // region in turn, so that three workgroups fit a CU
    constexpr int P1 = (SM + 2 * BW) * 4, P2 = G * MWP * 4;
    __shared__ __align__(16) unsigned char region[P1 > P2 ? P1 : P2];
    int *sid = reinterpret_cast<int *>(region);
    unsigned *bmp = reinterpret_cast<unsigned *>(region + SM * 4);
    int *wpre = reinterpret_cast<int *>(region + (SM + BW) * 4);
    unsigned *mask = reinterpret_cast<unsigned *>(region);
    __shared__ unsigned short nslot[SM];
    __shared__ int part[256];
    __shared__ int id_lo, id_hi;
    if (*a.skin_flag == 0u)
        return;  // no search ran (uniform over the grid)
    const int tile = blockIdx.x, t = threadIdx.x;
    const int first = a.tile_first[tile], tcnt = a.tile_first[tile + 1] - first;
    const int S = min(a.stage_cnt[tile], SM);
    int *st = a.stage + (size_t)tile * SM;
    if (t == 0) {
        id_lo = 0x7fffffff;
        id_hi = -1;
    }
    __syncthreads();
    {
        int mn = 0x7fffffff, mx = -1;
        for (int k = t; k < S; k += 256) {
            const int id = st[k];
            sid[k] = id;
            mn = min(mn, id);
            mx = max(mx, id);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {  // one atomic a wave
            mn = min(mn, __shfl_xor(mn, off));
            mx = max(mx, __shfl_xor(mx, off));
        }
        if ((t & 63) == 0) {
            atomicMin(&id_lo, mn);
            atomicMax(&id_hi, mx);
        }
    }
    __syncthreads();
    // new slot = rank of the residue id among the tile's slots (ids distinct):
    // from a bitmap of the ids when they span few enough values, else by
    // counting
    const int lo = id_lo, span = id_hi - id_lo + 1;
    if (S > 0 && span <= 32 * BW) {
        const int nw = (span + 31) >> 5;
        for (int w = t; w < nw; w += 256)
            bmp[w] = 0u;
        __syncthreads();
        for (int k = t; k < S; k += 256)
            atomicOr(&bmp[(sid[k] - lo) >> 5], 1u << ((sid[k] - lo) & 31));
        __syncthreads();
        constexpr int WPL = BW / 256;
        int c = 0;
        for (int w = t * WPL; w < min(nw, (t + 1) * WPL); ++w)
            c += __popc(bmp[w]);
        int total = 0;
        int o = block_exclusive_scan<256>(c, part, total);
        for (int w = t * WPL; w < min(nw, (t + 1) * WPL); ++w) {
            wpre[w] = o;
            o += __popc(bmp[w]);
        }
        __syncthreads();
        for (int k = t; k < S; k += 256) {
            const int v = sid[k] - lo;
            nslot[k] = (unsigned short)(wpre[v >> 5] + __popc(bmp[v >> 5] & ((1u << (v & 31)) - 1u)));
        }
    } else {
        for (int k = t; k < S; k += 256) {
            const int id = sid[k];
            int r = 0;
            for (int m = 0; m < S; ++m)
                r += sid[m] < id ? 1 : 0;
            nslot[k] = (unsigned short)r;
        }
    }
    __syncthreads();
    for (int k = t; k < S; k += 256)
        st[nslot[k]] = sid[k];
    __syncthreads();  // the ids are dead: the region takes the masks
    for (int g0 = 0; g0 < tcnt; g0 += G) {
        const int rho = g0 + t / NLG, q = t % NLG;
        const bool act = rho < tcnt && t / NLG < G;
        for (int w = t; w < G * MWP; w += 256)
            mask[w] = 0u;
        __syncthreads();
        int len = 0;
        unsigned short *row = nullptr;
        if (act) {
            const int i = first + rho;
            len = min(a.skin_cnt[i], a.cap);
            row = a.skin16 + (size_t)i * a.cap;
            // the row in 16-byte pieces (8 entries), pieces q, q + NLG, ...;
            // the first CPF of them loaded up front
            constexpr int CPF = 8;
            const uint4 *rp = reinterpret_cast<const uint4 *>(row);
            const int npc = (len + 7) >> 3;
            uint4 pre[CPF];
#pragma unroll
            for (int m = 0; m < CPF; ++m)
                pre[m] = m * NLG + q < npc ? rp[m * NLG + q] : make_uint4(0u, 0u, 0u, 0u);
            for (int m = 0; m * NLG + q < npc; ++m) {
                const int pc = m * NLG + q;
                uint4 w;
                if (m < CPF) {
#pragma unroll
                    for (int mm = 0; mm < CPF; ++mm)
                        if (mm == m)
                            w = pre[mm];
                } else {
                    w = rp[pc];
                }
                const unsigned ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (pc * 8 + u < len) {
                        const int ns = nslot[(ws[u >> 1] >> ((u & 1) * 16)) & 0xffffu];
                        atomicOr(&mask[(t / NLG) * MWP + (ns >> 5)], 1u << (ns & 31));
                    }
                }
            }
            // bonded and native entries: renumber in place
            const int2 rw = a.trow[i];
            const int ntop = (rw.y & 4095) + (rw.y >> 12);
            uint2 *tp = a.topo2 + (size_t)tile * TOPO_CAP * TILE + rho;
            for (int e = q; e < ntop; e += NLG) {
                const unsigned v = tp[(size_t)e * TILE].x;
                if (v < (unsigned)S)
                    tp[(size_t)e * TILE].x = nslot[v];
            }
        }
        __syncthreads();
        // emit: lane q scans words [q MW/NLG, (q+1) MW/NLG) of its residue's mask
        constexpr int WPL = MW / NLG;
        int c = 0;
        if (act)
            for (int w = q * WPL; w < (q + 1) * WPL; ++w)
                c += __popc(mask[(t / NLG) * MWP + w]);
        // entries before this lane's words: scan over the residue's lanes (adjacent)
        int v = c;
#pragma unroll
        for (int off = 1; off < NLG; off <<= 1) {
            const int y = __shfl_up(v, off, NLG);
            if (q >= off)
                v += y;
        }
        if (act) {
            int o = v - c;
            for (int w = q * WPL; w < (q + 1) * WPL; ++w) {
                unsigned b = mask[(t / NLG) * MWP + w];
                while (b) {
                    const int kb = __ffs(b) - 1;
                    b &= b - 1u;
                    row[o++] = (unsigned short)(32 * w + kb);
                }
            }
        }
        __syncthreads();  // the masks are reused by the next pass
    }
    // the filter hands the skin rows to its waves longest first, so that the
    // rows a wave tests have about the same length (ties in index order)
    int *slen = sid;  // the ids are written out
    for (int u = t; u < tcnt; u += 256)
        slen[u] = min(a.skin_cnt[first + u], a.cap);
    __syncthreads();
    for (int u = t; u < tcnt; u += 256) {
        const int L = slen[u];
        int r = 0;
        for (int v = 0; v < tcnt; ++v)
            r += (slen[v] > L || (slen[v] == L && v < u)) ? 1 : 0;
        a.skin_ord[(size_t)tile * TILE + r] = (unsigned short)(u + 1);
    }
}

struct TileArgs {
    const int *tile_first;  // first residue of each tile, then n
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
    const uint2 *noise_key;  // per residue {tag, stream id}
    const int *pull_slot;
    const PullDev *pulls;
    double *res_energy;
    float4 *fout;
    unsigned *err;
    const long long *step_base;
    const float4 *hi_skin;
    unsigned *skin_flag;
    const unsigned char *tile_ord;
    float4 *vel;          // underdamped: per-residue velocity (NULL: overdamped)
    // the last step of a list period bins its new positions for the next
    // skin search (do_bin)
    const int4 *traj_cell;
    int *cell_count;
    float4 *cells;
    int *cell_of;
    GridDev g;
    int do_bin;
    long long step_off;
    float check_thr2;
    int n, cap, has_pull, n_tiles;
    StepConsts c;
    UdConsts ud;
    TipDev tip;
    // the first step of a list period filters the skin rows itself (FIRST):
    // it writes the list rows, their counts and the longest-first order the
    // later steps read, clears the cell counts and the skin flag
    const unsigned short *skin16;
    const int *skin_cnt;
    const unsigned short *skin_ord;
    unsigned short *list16_out;
    int *list_cnt_out;
    unsigned char *tile_ord_out;
    float rc2;
    int n_cells;
};

// Position relative to the tile's origin O as an unevaluated sum rh + rl:
// (hi - O) + lo by two error-free TwoSum steps, so rh + rl carries the
// compensated position to about 2^-44 relative.
__device__ __forceinline__ void tile_frame(const float4 &hi, const float4 &lo, const float4 &O, float4 &rh,
                                           float4 &rl)
{
    float h[3], l[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float x = comp(hi, ax), o = comp(O, ax), xl = comp(lo, ax);
        const float s = x - o;  // TwoSum(x, -o)
        const float bb = s - x;
        const float e = (x - (s - bb)) + (-o - bb);
        const float t = e + xl;
        const float r = s + t;  // TwoSum(s, t)
        const float bp = r - s;
        h[ax] = r;
        l[ax] = (s - (r - bp)) + (t - bp);
    }
    rh = make_float4(h[0], h[1], h[2], 0.0f);
    rl = make_float4(l[0], l[1], l[2], 0.0f);
}

// The low part of a tile coordinate is at most half an ulp of the high part;
// a staged slot keeps it as a 10-bit multiple of ulp/1000 per axis in the
// high part's w word, so one 16-byte LDS read brings both.
__device__ __forceinline__ float ulp_of(float x)
{
    return __int_as_float(__float_as_int(x) & 0x7f800000) * 0x1p-23f;
}

__device__ __forceinline__ unsigned pack_low(const float4 &rh, const float4 &rl)
{
    unsigned bitsw = 0u;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        // 1/ulp is a power of two: biased exponent 277 - E for exponent field E
        const int E = (__float_as_int(comp(rh, ax)) >> 23) & 0xff;
        const float inv_u = (E >= 24 && E <= 253) ? __int_as_float((277 - E) << 23) : 0.0f;
        const float v = comp(rl, ax) * inv_u * 1000.0f;
        const int qv = (int)rintf(fminf(fmaxf(v, -511.0f), 511.0f));
        bitsw |= ((unsigned)qv & 0x3ffu) << (10 * ax);
    }
    return bitsw;
}

__device__ __forceinline__ float3 unpack_low(const float4 &s)
{
    const unsigned w = __float_as_uint(s.w);
    float l[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int qv = ((int)(w << (22 - 10 * ax))) >> 22;  // sign-extended 10-bit field
        l[ax] = (float)qv * (ulp_of(comp(s, ax)) * 1.0e-3f);
    }
    return make_float3(l[0], l[1], l[2]);
}

// Batched schedule: each residue packs its low part in units of one quantum,
// ulp/1000 of its largest high coordinate (no coarser than ulp/1000 of any
// other), so that a partner's three fields take one exponent to unpack.
__device__ __forceinline__ float res_quantum(const float4 &h)
{
    return ulp_of(fmaxf(fabsf(h.x), fmaxf(fabsf(h.y), fabsf(h.z)))) * 1.0e-3f;
}

__device__ __forceinline__ unsigned pack_low_res(const float4 &hi, const float4 &lo)
{
    const int E = (__float_as_int(fmaxf(fabsf(hi.x), fmaxf(fabsf(hi.y), fabsf(hi.z)))) >> 23) & 0xff;
    // 1/quantum: a power of two (biased exponent 277 - E) times 1000
    const float inv_q = (E >= 24 && E <= 253) ? __int_as_float((277 - E) << 23) * 1000.0f : 0.0f;
    unsigned bitsw = 0u;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int qv = (int)rintf(fminf(fmaxf(comp(lo, ax) * inv_q, -511.0f), 511.0f));
        bitsw |= ((unsigned)qv & 0x3ffu) << (10 * ax);
    }
    return bitsw;
}

// hi_i + lo_i - (hj + its packed low part), per axis
__device__ __forceinline__ float3 pair_delta_packed(const float4 &hi, const float4 &lo, const float4 &hj)
{
    const unsigned w = __float_as_uint(hj.w);
    const float qm = res_quantum(hj);
    float d[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int qv = ((int)(w << (22 - 10 * ax))) >> 22;  // sign-extended 10-bit field
        d[ax] = (comp(hi, ax) - comp(hj, ax)) + __builtin_fmaf(-(float)qv, qm, comp(lo, ax));
    }
    return make_float3(d[0], d[1], d[2]);
}

// A tile whose residues all lie within this distance of its origin has its
// list partners (within r_list = 20 A of one of them at the rebuild, a few
// tenths of an Angstrom more after ten steps) within about 64 A of it, so
// list pairs use the high parts alone (separation error about 8e-6 A at most); other
// tiles add the low parts.  The test reads the tile's own residues only, so
// the arithmetic does not depend on which other residues are staged.
constexpr float NARROW_TILE = 40.0f;

// The plain step: one workgroup of 256 lanes per tile of TILE consecutive
// residues, NL = 256/TILE adjacent lanes per residue, the tile's residues
// handed to the lanes longest list row first.
//  1. Every load that does not need the staging is issued first: the
//     residue's own position and row, its first PRE list chunks (4 slots
//     each: chunks q, q + NL, ... for lane q), its first bonded/native
//     entries and their partners' compensated positions, and the tile's
//     slot ids.
//  2. The last TILE lanes draw their residue's Gaussians (Philox and
//     Box-Muller, from the counter words that do not depend on the
//     position) and evaluate its cantilever and tip terms; every lane stages
//     slots (each position relative to the tile origin, its middle residue,
//     as the exactly rounded high part of a TwoSum split) and evaluates its
//     bonded and native entries from the compensated positions.
//  3. After the barrier the list chunks are summed from the staged
//     positions: high parts only when every residue of the tile lies within
//     NARROW_TILE of the origin, else high and low parts (the low parts, a
//     10-bit multiple of the high part's ulp per axis, are staged then).
//     The NL partial sums of a residue are added by butterfly shuffles,
//     which give every lane the same bits.
//  4. After a second barrier the last TILE lanes add the external terms and
//     the noise and take the compensated step (first-order, or BAOAB).
// FIRST (the first step after a rebuild, which then needs no filter kernel):
// the rows read are the skin rows, in the order of the last skin search
// (longest first); the staging also keeps each slot's global high part, and
// after the barrier each residue's lanes test their skin row pieces with the
// list predicate and write the passing entries, in order, as its list row,
// which the list sums then read back: the same rows, sums and bits as a
// filter kernel followed by a plain step.
template <int TILE, bool ENERGY, int MODE, bool FIRST>
__global__ __launch_bounds__(256, ENERGY ? 2 : (TILE >= 256 ? 3 : 5)) void k_tile_step(TileArgs a)
{
    constexpr int NL = 256 / TILE;
    constexpr int SM = stage_max<TILE>();
    constexpr int SW = stage_win<TILE>();
    constexpr int PER = SW / 256;    // staging slots per lane
    constexpr int EPI = 256 - TILE;  // first lane of the update lanes
    constexpr int PRE = 6;           // list chunks per lane loaded before the staging
    constexpr int TPRE = 2;          // bonded/native entries per lane loaded before the staging
    __shared__ float4 sl_s[SW + 1];  // {rh.xyz, packed rl}; slot SW: the far-away empty slot
    // SOA: the same high parts by axis, read by the list sums of compact
    // tiles: three 4-byte reads a partner spread over all banks, where
    // 16-byte elements start on one bank in four (not in the first step or
    // with 2,048-slot windows, short of LDS)
    constexpr bool SOA = !FIRST && SW <= 1024;
    __shared__ float sr_s[3][SOA ? SW + 1 : 1];
    __shared__ float hg_s[3][FIRST ? SW : 1];  // FIRST: each slot's global high part, by axis
    __shared__ int lens_s[FIRST ? TILE : 1];    // FIRST: list row lengths
    __shared__ float f_s[3][TILE];   // list + bonded/native force of each residue
    __shared__ double e_s[ENERGY ? 4 : 1][ENERGY ? TILE : 1];
    if (FIRST) {
        // the cell counts were read by the skin search, which is done:
        // cleared for the binning at the end of this period; the flag too
        for (int k = blockIdx.x * 256 + threadIdx.x; k < a.n_cells; k += gridDim.x * 256)
            a.cell_count[k] = 0;
        if (blockIdx.x == 0 && threadIdx.x == 0)
            *a.skin_flag = 0u;
    }
    // XCD-aware order: consecutive tiles stay on one XCD's L2.
    const int per = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= a.n_tiles)
        return;  // uniform over the workgroup
    const int t = threadIdx.x;
    const int first = a.tile_first[tile], tcnt = a.tile_first[tile + 1] - first;
    const int S = min(a.stage_cnt[tile], SM);
    const int *st = a.stage + (size_t)tile * SM;
    // rare: a staging set larger than one LDS window is taken window by window
    const bool windowed = S > SW;
    const int mid = first + tcnt / 2;
    const long long step = (a.step_base ? *a.step_base : 0) + a.step_off;
    const int q = t % NL;
    const bool act = t / NL < tcnt;
    int rho = 0;
    if (FIRST) {
        const int ord = act ? (int)a.skin_ord[(size_t)tile * TILE + t / NL] : 0;
        rho = act ? (ord > 0 ? ord - 1 : t / NL) : 0;
    } else {
        rho = act ? (int)a.tile_ord[(size_t)tile * TILE + t / NL] : 0;
    }
    const int i = first + rho;
    const int ue = t - EPI;
    const bool upd = ue >= 0 && ue < tcnt;
    const int iu = first + ue;
    // ---- 1. loads ----
    int ids[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u)
        ids[u] = (!windowed && t + u * 256 < S) ? st[t + u * 256] : -1;
    float4 hi0 = make_float4(0.f, 0.f, 0.f, 0.f), lo0 = hi0;
    int2 row = make_int2(0, 0);
    int cnt = 0;
    int slen = 0;  // FIRST: the skin row's length
    if (act) {
        hi0 = a.pin[2 * i];
        lo0 = a.pin[2 * i + 1];
        row = a.trow[i];
        if (FIRST)
            slen = min(a.skin_cnt[i], a.cap);
        else
            cnt = min(a.list_cnt[i], a.cap);
    }
    const float4 O = a.pin[2 * mid];
    int nch = (cnt + 3) >> 2;
    const uint2 *lp = reinterpret_cast<const uint2 *>(a.list16 + (size_t)i * a.cap);
    constexpr int NPRE = FIRST ? 3 : PRE;
    uint2 lw[NPRE];
    constexpr int SPF = 1;  // FIRST: skin row pieces (8 entries) loaded up front
    uint4 spre[SPF];
    const uint4 *sp = reinterpret_cast<const uint4 *>(FIRST ? a.skin16 + (size_t)i * a.cap : nullptr);
    const int npc = (slen + 7) >> 3;
    if (FIRST) {
#pragma unroll
        for (int m = 0; m < SPF; ++m)
            spre[m] = m * NL + q < npc ? sp[m * NL + q] : make_uint4(0u, 0u, 0u, 0u);
    } else {
#pragma unroll
        for (int k = 0; k < NPRE; ++k)
            lw[k] = q + k * NL < nch ? lp[q + k * NL] : make_uint2(0u, 0u);
    }
    const int nb = row.y & 4095, ntop = nb + (row.y >> 12);
    // bonded entries: lane q takes bonds q, q + NL, ... and natives nb + q,
    // nb + q + NL, ..., in loops of their own so that a wave runs each
    // term's code once a round; its first bond and first TPRE - 1 natives
    // are loaded here
    float2 te[TPRE];
#pragma unroll
    for (int k = 0; k < TPRE; ++k) {
        const int e = k == 0 ? q : nb + q + (k - 1) * NL;
        te[k] = (k == 0 ? e < nb : e < ntop) ? a.tent[row.x + e] : make_float2(0.f, 0.f);
    }
    float4 ph[TPRE], pl[TPRE];
#pragma unroll
    for (int k = 0; k < TPRE; ++k) {
        const int e = k == 0 ? q : nb + q + (k - 1) * NL;
        if (k == 0 ? e < nb : e < ntop) {
            const int j = __float_as_int(te[k].x);
            ph[k] = a.pin[2 * j];
            pl[k] = a.pin[2 * j + 1];
        }
    }
    // ---- 2. noise and external terms (update lanes), staging, bonded/native ----
    float4 hu = make_float4(0.f, 0.f, 0.f, 0.f), lu = hu;
    float g[3] = {0.0f, 0.0f, 0.0f};
    Acc X;
    double e_x = 0.0, f_rep = 0.0;
    // the last step of a list period bins the new positions for the next
    // skin search; the cell slot is taken in the cell of the position before
    // the update (nearly always the cell of the new one), so the atomic's
    // round trip overlaps the step
    if (upd) {
        hu = a.pin[2 * iu];
        lu = a.pin[2 * iu + 1];
        if (MODE == 0) {
            const uint2 key = a.noise_key[iu];
            if (!(key.x >> 31)) {
                const uint4 w = noise_words(key.x, key.y, step, a.c);
                const float2 gxy = gaussian_pair(w);
                g[0] = gxy.x;
                g[1] = gxy.y;
                g[2] = gaussian_axis(w, 2);
            }
        }
        add_external(X, e_x, f_rep, hu, lu, step, a.c.h, a.has_pull ? a.pull_slot[iu] : -1, a.pulls,
                     a.tip, ENERGY, a.err);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        if (ids[u] >= 0) {
            const float4 gh = a.pin[2 * ids[u]];
            float4 rh, rl;
            tile_frame(gh, a.pin[2 * ids[u] + 1], O, rh, rl);
            rh.w = 0.0f;
            sl_s[t + u * 256] = rh;
            if (SOA) {
                sr_s[0][t + u * 256] = rh.x;
                sr_s[1][t + u * 256] = rh.y;
                sr_s[2][t + u * 256] = rh.z;
            }
            if (FIRST) {
                hg_s[0][t + u * 256] = gh.x;
                hg_s[1][t + u * 256] = gh.y;
                hg_s[2][t + u * 256] = gh.z;
            }
        }
    }
    if (t == 0) {
        sl_s[SW] = make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.0f);
        if (SOA)
            sr_s[0][SW] = sr_s[1][SW] = sr_s[2][SW] = 1.0e18f;
    }

    const PairConsts k = pair_consts(a.c);
    Acc A;   // bonded and native terms
    bool broken = false;
    if (act) {
        if (q < nb)
            add_fene_d(A, pair_delta(hi0, lo0, ph[0], pl[0]), te[0].y, k, ENERGY, broken);
        for (int e = q + NL; e < nb; e += NL) {
            const float2 tv = a.tent[row.x + e];
            const int j = __float_as_int(tv.x);
            add_fene_d(A, pair_delta(hi0, lo0, a.pin[2 * j], a.pin[2 * j + 1]), tv.y, k, ENERGY, broken);
        }
#pragma unroll
        for (int kk = 1; kk < TPRE; ++kk)
            if (nb + q + (kk - 1) * NL < ntop)
                add_native_d(A, pair_delta(hi0, lo0, ph[kk], pl[kk]), te[kk].y, k, ENERGY);
        for (int e = nb + q + (TPRE - 1) * NL; e < ntop; e += NL) {
            const float2 tv = a.tent[row.x + e];
            const int j = __float_as_int(tv.x);
            add_native_d(A, pair_delta(hi0, lo0, a.pin[2 * j], a.pin[2 * j + 1]), tv.y, k, ENERGY);
        }
        if (broken)
            atomicOr(a.err, ERR_FENE);
    }
    float4 rh0, rl0;
    tile_frame(hi0, lo0, O, rh0, rl0);
    const bool far = windowed || (act && !(fmaxf(fabsf(rh0.x), fmaxf(fabsf(rh0.y), fabsf(rh0.z))) < NARROW_TILE));
    const bool wide = __syncthreads_or(far ? 1 : 0) != 0;
    if (wide && !windowed) {
        // rare: the low parts of the staged positions, packed beside them
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (ids[u] >= 0) {
                float4 rh, rl;
                tile_frame(a.pin[2 * ids[u]], a.pin[2 * ids[u] + 1], O, rh, rl);
                sl_s[t + u * 256].w = __uint_as_float(pack_low(rh, rl));
            }
        }
        rh0.w = __uint_as_float(pack_low(rh0, rl0));
        __syncthreads();
    }
    if (windowed)
        rh0.w = __uint_as_float(pack_low(rh0, rl0));
    // the binning's slot and the displacement check's reference, requested
    // now so that they arrive during the list sums
    float4 hsk = make_float4(0.f, 0.f, 0.f, 0.f);
    if (MODE == 0 && upd && a.check_thr2 > 0.0f)
        hsk = a.hi_skin[iu];
    // the lanes of a wave that bin into one cell take consecutive slots
    // from one atomic, issued by the group's first lane (uniform branch:
    // the whole wave takes part in the ballots)
    // the first step of a period never bins (it clears the cell counts the
    // binning at the period's end fills; a period's first step is not its last)
    const bool do_bin = MODE == 0 && !FIRST && a.do_bin;
    int bin_lead = 0, bin_rank = 0, bin_base = 0;
    int bin_c0 = -1;           // the cell of the position before the update
    int4 bin_off = {0, 0, 0, 0};  // the trajectory's cell offset, kept for after the update
    if (do_bin) {
        const bool binning = upd;
        if (binning)
            bin_off = a.traj_cell[__float_as_int(lu.w)];
        const int c0 = binning ? cell_index(hu, bin_off, a.g) : -1;
        bin_c0 = c0;
        const int lane = (int)__lane_id();
        const unsigned long long below = (1ull << lane) - 1ull;
        unsigned long long todo = __ballot(binning);
        unsigned long long mine = 0ull;
        while (todo) {
            const int lead = __ffsll((long long)todo) - 1;
            const int cl = __shfl(c0, lead);
            const unsigned long long same = __ballot(binning && c0 == cl) & todo;
            if ((same >> lane) & 1ull) {
                bin_lead = lead;
                bin_rank = __popcll(same & below);
            }
            if (lane == lead)
                mine = same;
            todo &= ~same;
        }
        if (binning && lane == bin_lead)
            bin_base = atomicAdd(&a.cell_count[c0], __popcll(mine));
    }
    if (FIRST) {
        // ---- the list rows, filtered from the skin rows (Algorithm 3's
        // predicate at r_list) and written in order ----
        // ONE (compile time): the set fits one LDS window, as for nearly
        // every tile; the round loop below is compiled once for each case
        auto test = [&](const uint4 &w, int pc, auto one) -> unsigned {
            constexpr bool ONE = decltype(one)::value;
            const unsigned ws[4] = {w.x, w.y, w.z, w.w};
            const int valid = slen - pc * 8;
            const unsigned tail = valid >= 8 ? 0xffu : (valid > 0 ? (1u << valid) - 1u : 0u);
            unsigned bits = 0u;
#pragma unroll
            for (int h = 0; h < 8; h += 4) {  // four reads in flight, then their tests
                float4 pj[4];
#pragma unroll
                for (int u = h; u < h + 4; ++u) {
                    const unsigned sl = (ws[u >> 1] >> ((u & 1) * 16)) & 0xffffu;
                    if constexpr (ONE) {
                        // entries past the row's end (masked) clamped into the set
                        const int e = (int)min(sl, (unsigned)(SW - 1));
                        pj[u - h] = make_float4(hg_s[0][e], hg_s[1][e], hg_s[2][e], 0.0f);
                    } else {
                        // rare: a set larger than one window reads the positions themselves
                        pj[u - h] = a.pin[2 * st[min(sl, (unsigned)(SM - 1))]];
                    }
                }
#pragma unroll
                for (int u = h; u < h + 4; ++u)
                    bits |= (unsigned)within_cutoff(hi0, pj[u - h], a.rc2) << u;
            }
            return bits & tail;
        };
        unsigned short *dst = a.list16_out + (size_t)i * a.cap;
        int rounds = (npc + NL - 1) / NL;
#pragma unroll
        for (int off = 1; off < NL; off <<= 1)
            rounds = max(rounds, __shfl_xor(rounds, off, NL));  // uniform over the residue's lanes
        int base = 0;
        // lane q's piece of this round: its passing entries go after those
        // of the residue's earlier pieces
        auto emit = [&](const uint4 &w, unsigned bits) {
            const unsigned ws[4] = {w.x, w.y, w.z, w.w};
            const int c = __popc(bits);
            int v = c;
#pragma unroll
            for (int off = 1; off < NL; off <<= 1) {
                const int y = __shfl_up(v, off, NL);
                if (q >= off)
                    v += y;
            }
            // entry u goes after the passing entries below it: eight masked
            // stores, not a loop as long as the wave's longest run
            unsigned short *d = dst + (base + v - c);
#pragma unroll 1
            for (int h = 0; h < 2; ++h) {  // the piece's two halves, four entries each
                const unsigned w0 = h ? ws[2] : ws[0], w1 = h ? ws[3] : ws[1];
                const unsigned hb = bits >> (4 * h);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if ((hb >> u) & 1u)
                        d[__popc(hb & ((1u << u) - 1u))] = (unsigned short)((u < 2 ? w0 : w1) >> ((u & 1) * 16));
                d += __popc(hb & 0xfu);
            }
            base += __shfl(v, NL - 1, NL);
        };
        auto filter_rows = [&](auto one) {
#pragma unroll
            for (int m = 0; m < SPF; ++m)
                if (m < rounds)
                    emit(spre[m], m * NL + q < npc ? test(spre[m], m * NL + q, one) : 0u);
            // later pieces: the next one requested before the current one is used
            uint4 wn = SPF * NL + q < npc ? sp[SPF * NL + q] : make_uint4(0u, 0u, 0u, 0u);
            for (int m = SPF; m < rounds; ++m) {
                const int pc = m * NL + q;
                const uint4 w = wn;
                wn = pc + NL < npc ? sp[pc + NL] : make_uint4(0u, 0u, 0u, 0u);
                emit(w, pc < npc ? test(w, pc, one) : 0u);
            }
        };
        if (S <= SW)
            filter_rows(std::true_type{});
        else
            filter_rows(std::false_type{});
        if (act && q == NL - 1) {
            // padded to a multiple of 8 entries: with the LDS slot of the
            // far-away position when the set fits one window, else the empty slot
            const unsigned short pad = S <= SW ? (unsigned short)SW : EMPTY_SLOT;
            for (int k = base; k < ((base + 7) & ~7); ++k)
                dst[k] = pad;
            a.list_cnt_out[i] = base;
            lens_s[rho] = base;
        }
        cnt = act ? base : 0;
        nch = (cnt + 3) >> 2;
        __syncthreads();  // the rows are written (read back below) and the lengths known
        // the row's first chunks requested together, as the other steps do
        // before their staging; they arrive while the rank is counted
#pragma unroll
        for (int k = 0; k < NPRE; ++k)
            lw[k] = q + k * NL < nch ? lp[q + k * NL] : make_uint2(0u, 0u);
        // the later steps hand the rows to their waves longest first (ties
        // in index order): the residue's rank, counted by its NL lanes
        int r = 0;
        if (act)
            for (int u = q * (TILE / NL); u < min(tcnt, (q + 1) * (TILE / NL)); ++u)
                r += (lens_s[u] > base || (lens_s[u] == base && u < rho)) ? 1 : 0;
#pragma unroll
        for (int off = 1; off < NL; off <<= 1)
            r += __shfl_xor(r, off, NL);
        if (act && q == 0)
            a.tile_ord_out[(size_t)tile * TILE + r] = (unsigned char)rho;
    }
    // ---- 3. list chunks of this lane ----
    Acc L;   // list: sum of d / r^8 (scaled by 6 eps_l sigma^6 below)
    const float3 pl0 = unpack_low(rh0);
    // slot -> LDS index of the current window (identity for one window)
    int w0 = 0, wn = S;
    // FORM: 0 high parts, 1 high and low parts, 2 high and low parts of one
    // window (compile-time copies of `wide` and `windowed`, so that each list
    // loop holds one form)
    auto pairs4 = [&](const uint2 &w, auto form) {
        constexpr int FORM = decltype(form)::value;
        constexpr bool WIDE = FORM > 0;
        float4 pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sl = (int)(((u < 2 ? w.x : w.y) >> ((u & 1) * 16)) & 0xffffu);
            if constexpr (FORM == 2) {
                const int e = sl - w0;
                pj[u] = sl_s[(unsigned)e < (unsigned)wn ? e : SW];
            } else {
                if constexpr (FORM == 0 && SOA)
                    pj[u] = make_float4(sr_s[0][sl], sr_s[1][sl], sr_s[2][sl], 0.0f);
                else
                    pj[u] = sl_s[sl];
            }
        }
        if constexpr (!WIDE) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                add_repulsive_u(L, make_float3(rh0.x - pj[u].x, rh0.y - pj[u].y, rh0.z - pj[u].z), k,
                                ENERGY);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float3 lj = unpack_low(pj[u]);
                add_repulsive_u(L,
                                make_float3((rh0.x - pj[u].x) + (pl0.x - lj.x), (rh0.y - pj[u].y) + (pl0.y - lj.y),
                                            (rh0.z - pj[u].z) + (pl0.z - lj.z)),
                                k, ENERGY);
            }
        }
    };
    auto list_pass = [&](auto form) {
        if (!act)
            return;
#pragma unroll
        for (int kk = 0; kk < NPRE; ++kk)
            if (q + kk * NL < nch)
                pairs4(lw[kk], form);
        for (int c = q + NPRE * NL; c < nch; c += NL)
            pairs4(lp[c], form);
    };
    if (!windowed) {
        if (wide)
            list_pass(std::integral_constant<int, 1>{});
        else
            list_pass(std::integral_constant<int, 0>{});
    } else {
        // every window's slots staged with their low parts; each entry
        // contributes in the window holding its slot (elsewhere it reads the
        // far-away slot, whose term is exactly zero)
        for (w0 = 0; w0 < S; w0 += SW) {
            wn = min(SW, S - w0);
            __syncthreads();  // the previous window's readers are done
            for (int sl = t; sl < wn; sl += 256) {
                const int id = st[w0 + sl];
                float4 rh, rl;
                tile_frame(a.pin[2 * id], a.pin[2 * id + 1], O, rh, rl);
                rh.w = __uint_as_float(pack_low(rh, rl));
                sl_s[sl] = rh;
            }
            __syncthreads();
            list_pass(std::integral_constant<int, 2>{});
        }
    }
    // the residue's total over its NL lanes (butterfly: every lane gets the same bits)
    float fx = k.c6 * L.fx + A.fx, fy = k.c6 * L.fy + A.fy, fz = k.c6 * L.fz + A.fz;
    double eb = A.e_b, en = A.e_n, er = L.e_r, vir = A.vir + L.vir;
#pragma unroll
    for (int off = 1; off < NL; off <<= 1) {
        fx += __shfl_xor(fx, off, NL);
        fy += __shfl_xor(fy, off, NL);
        fz += __shfl_xor(fz, off, NL);
        if (ENERGY) {
            eb += __shfl_xor(eb, off, NL);
            en += __shfl_xor(en, off, NL);
            er += __shfl_xor(er, off, NL);
            vir += __shfl_xor(vir, off, NL);
        }
    }
    if (act && q == 0) {
        f_s[0][rho] = fx;
        f_s[1][rho] = fy;
        f_s[2][rho] = fz;
        if constexpr (ENERGY) {
            e_s[0][rho] = eb;
            e_s[1][rho] = en;
            e_s[2][rho] = er;
            e_s[3][rho] = vir;
        }
    }
    // this residue's slot in its cell (the group's atomic has returned)
    int bin_s0 = 0;
    if (do_bin)
        bin_s0 = __shfl(bin_base, bin_lead) + bin_rank;
    __syncthreads();
    if (!upd)
        return;
    // ---- 4. external terms, noise and the compensated update ----
    Acc F;
    F.fx = f_s[0][ue] + X.fx;
    F.fy = f_s[1][ue] + X.fy;
    F.fz = f_s[2][ue] + X.fz;
    if constexpr (ENERGY) {
        double *er_out = a.res_energy + (size_t)iu * RES_E;
        // each internal pair appears in both partners' rows
        er_out[0] = 0.5 * e_s[0][ue];
        er_out[1] = 0.5 * e_s[1][ue];
        er_out[2] = 0.5 * e_s[2][ue];
        er_out[3] = e_x;
        er_out[4] = 0.5 * e_s[3][ue];
        er_out[5] = f_rep;
    }
    if (MODE == 1) {
        a.fout[iu] = make_float4(F.fx, F.fy, F.fz, 0.0f);
        return;
    }
    float4 hi = hu, lo = lu;
    if (a.vel) {
        float4 v = a.vel[iu];
        underdamped_update(hi, lo, v, F, g, a.ud, a.err);
        a.vel[iu] = v;
    } else {
        update_with_noise(hi, lo, F, g, a.c, a.err);
    }
    a.pout[2 * iu] = hi;
    a.pout[2 * iu + 1] = lo;
    if (a.check_thr2 > 0.0f) {
        // moved farther than skin/2 from the last skin build: the next
        // rebuild rebuilds the skin
        const float dx = hi.x - hsk.x, dy = hi.y - hsk.y, dz = hi.z - hsk.z;
        if (!(dx * dx + dy * dy + dz * dz <= a.check_thr2))
            atomicOr(a.skin_flag, 1u);
    }
    if (do_bin) {
        const int traj = __float_as_int(lo.w);
        const int c1 = cell_index(hi, bin_off, a.g);
        if (c1 == bin_c0) {
            a.cell_of[iu] = c1;
            if (bin_s0 < CELL_CAP)
                a.cells[(size_t)c1 * CELL_CAP + bin_s0] = make_float4(hi.x, hi.y, hi.z, __int_as_float(iu));
            else
                atomicOr(a.err, ERR_CELL);
        } else {
            // moved into another cell: the slot taken holds a far-away copy
            // (no predicate passes it; the id keeps the cell's ids distinct)
            // and the residue is binned again
            if (bin_s0 < CELL_CAP)
                a.cells[(size_t)bin_c0 * CELL_CAP + bin_s0] =
                    make_float4(1.0e18f, 1.0e18f, 1.0e18f, __int_as_float(iu));
            bin_one(hi, iu, traj, a.g, a.traj_cell, a.cell_count, a.cells, a.cell_of, a.err);
        }
    }
}

// ---------------------------------------------------------------------------
// Pair-based forces (Algorithm 4 with the atomic additions its text proposes
// for GPUs that have them, Algorithm 5's gathering folded into the update
// kernel): each unordered pair of the list and of the bonded and native
// entries is evaluated once, in the row of its lower residue, and +df / -df
// are added to both residues' force accumulators with hardware float
// atomics.  The order of those additions is not fixed, so forces and
// trajectories are reproducible only to rounding.
// ---------------------------------------------------------------------------
struct PairArgs {
    const int *tile_first;
    const float4 *pin;
    const int2 *trow;
    const float2 *tent;
    const unsigned short *list16;
    const int *list_cnt;
    const int *stage;
    const int *stage_cnt;
    float4 *facc;   // per residue: accumulated force
    double4 *eacc;  // per residue: accumulated {FENE, native, repulsive, virial} halves
    unsigned *err;
    int cap, n_tiles;
    StepConsts c;
};

// One workgroup per tile.  A list pair (i, j), i < j, is evaluated in
// residue i's row; +df goes to i's running sum in registers and -df to j's
// staging slot in LDS (a shared-memory float atomic); at the end each
// residue's sum and each slot's sum are added to the device-wide
// accumulators with one hardware float atomic per component.  Bonded and
// native partners, which need no slot, take device-wide atomics directly.
template <int TILE, bool ENERGY>
__global__ __launch_bounds__(256) void k_pair_forces(PairArgs a)
{
    constexpr int NL = 256 / TILE;
    constexpr int SM = stage_max<TILE>();
    constexpr int SW = stage_win<TILE>();
    __shared__ float acc_s[3][SW];  // slots beyond SW take device-wide atomics
    const int tile = blockIdx.x, t = threadIdx.x;
    const int rho = t / NL, q = t % NL;
    const int first = a.tile_first[tile], tcnt = a.tile_first[tile + 1] - first;
    const int S = min(a.stage_cnt[tile], SM);
    const int *st = a.stage + (size_t)tile * SM;
    for (int sl = t; sl < min(S, SW); sl += 256) {
        acc_s[0][sl] = 0.0f;
        acc_s[1][sl] = 0.0f;
        acc_s[2][sl] = 0.0f;
    }
    __syncthreads();
    const bool act = rho < tcnt;
    const int i = first + (act ? rho : 0);
    const PairConsts k = pair_consts(a.c);
    Acc own;  // residue i's share of its pairs
    if (act) {
        const float4 hi = a.pin[2 * i], lo = a.pin[2 * i + 1];
        const int cnt = min(a.list_cnt[i], a.cap);
        const unsigned short *row = a.list16 + (size_t)i * a.cap;
        for (int e = q; e < cnt; e += NL) {
            const int sl = row[e];
            const int j = st[sl];
            if (j <= i)
                continue;  // the pair belongs to the lower residue's row
            Acc d;
            add_repulsive_d(d, pair_delta(hi, lo, a.pin[2 * j], a.pin[2 * j + 1]), k, ENERGY);
            own.fx += d.fx;
            own.fy += d.fy;
            own.fz += d.fz;
            if (sl < SW) {
                atomicAdd(&acc_s[0][sl], -d.fx);
                atomicAdd(&acc_s[1][sl], -d.fy);
                atomicAdd(&acc_s[2][sl], -d.fz);
            } else {
                unsafeAtomicAdd(&a.facc[j].x, -d.fx);
                unsafeAtomicAdd(&a.facc[j].y, -d.fy);
                unsafeAtomicAdd(&a.facc[j].z, -d.fz);
            }
            if (ENERGY) {
                const double he = 0.5 * d.e_r, hv = 0.5 * d.vir;
                own.e_r += he;
                own.vir += hv;
                unsafeAtomicAdd(&a.eacc[j].z, he);
                unsafeAtomicAdd(&a.eacc[j].w, hv);
            }
        }
        const int2 rw = a.trow[i];
        const int nb = rw.y & 4095, ntop = nb + (rw.y >> 12);
        bool broken = false;
        for (int e = q; e < ntop; e += NL) {
            const float2 te = a.tent[rw.x + e];
            const int j = __float_as_int(te.x);
            if (j <= i)
                continue;
            Acc d;
            const float3 dd = pair_delta(hi, lo, a.pin[2 * j], a.pin[2 * j + 1]);
            if (e < nb)
                add_fene_d(d, dd, te.y, k, ENERGY, broken);
            else
                add_native_d(d, dd, te.y, k, ENERGY);
            own.fx += d.fx;
            own.fy += d.fy;
            own.fz += d.fz;
            unsafeAtomicAdd(&a.facc[j].x, -d.fx);
            unsafeAtomicAdd(&a.facc[j].y, -d.fy);
            unsafeAtomicAdd(&a.facc[j].z, -d.fz);
            if (ENERGY) {
                const double hb = 0.5 * d.e_b, hn = 0.5 * d.e_n, hv = 0.5 * d.vir;
                own.e_b += hb;
                own.e_n += hn;
                own.vir += hv;
                unsafeAtomicAdd(&a.eacc[j].x, hb);
                unsafeAtomicAdd(&a.eacc[j].y, hn);
                unsafeAtomicAdd(&a.eacc[j].w, hv);
            }
        }
        if (broken)
            atomicOr(a.err, ERR_FENE);
    }
    // residue i: its NL lanes' shares, then one atomic per component
#pragma unroll
    for (int off = 1; off < NL; off <<= 1) {
        own.fx += __shfl_xor(own.fx, off, NL);
        own.fy += __shfl_xor(own.fy, off, NL);
        own.fz += __shfl_xor(own.fz, off, NL);
        if (ENERGY) {
            own.e_b += __shfl_xor(own.e_b, off, NL);
            own.e_n += __shfl_xor(own.e_n, off, NL);
            own.e_r += __shfl_xor(own.e_r, off, NL);
            own.vir += __shfl_xor(own.vir, off, NL);
        }
    }
    if (act && q == 0) {
        unsafeAtomicAdd(&a.facc[i].x, own.fx);
        unsafeAtomicAdd(&a.facc[i].y, own.fy);
        unsafeAtomicAdd(&a.facc[i].z, own.fz);
        if (ENERGY) {
            unsafeAtomicAdd(&a.eacc[i].x, own.e_b);
            unsafeAtomicAdd(&a.eacc[i].y, own.e_n);
            unsafeAtomicAdd(&a.eacc[i].z, own.e_r);
            unsafeAtomicAdd(&a.eacc[i].w, own.vir);
        }
    }
    __syncthreads();
    // the slots' shares
    for (int sl = t; sl < min(S, SW); sl += 256) {
        const float fx = acc_s[0][sl], fy = acc_s[1][sl], fz = acc_s[2][sl];
        if (fx != 0.0f || fy != 0.0f || fz != 0.0f) {
            const int j = st[sl];
            unsafeAtomicAdd(&a.facc[j].x, fx);
            unsafeAtomicAdd(&a.facc[j].y, fy);
            unsafeAtomicAdd(&a.facc[j].z, fz);
        }
    }
}

struct PairUpdArgs {
    const float4 *pin;
    float4 *pout;
    float4 *facc;
    double4 *eacc;
    const uint2 *noise_key;
    const int *pull_slot;
    const PullDev *pulls;
    double *res_energy;
    float4 *fout;
    unsigned *err;
    const long long *step_base;
    const float4 *hi_skin;
    unsigned *skin_flag;
    float4 *vel;
    const int4 *traj_cell;
    int *cell_count;
    float4 *cells;
    int *cell_of;
    GridDev g;
    int do_bin;
    long long step_off;
    float check_thr2;
    int n, has_pull;
    StepConsts c;
    UdConsts ud;
    TipDev tip;
};

// Algorithm 5's gathering and the update: the accumulated force (cleared
// for the next step), the external terms, the noise and the compensated step.
template <bool ENERGY, int MODE>
__global__ __launch_bounds__(256) void k_pair_update(PairUpdArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n)
        return;
    const long long step = (a.step_base ? *a.step_base : 0) + a.step_off;
    const float4 hi0 = a.pin[2 * i], lo0 = a.pin[2 * i + 1];
    const float4 f = a.facc[i];
    a.facc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    Acc F;
    F.fx = f.x;
    F.fy = f.y;
    F.fz = f.z;
    double e_x = 0.0, f_rep = 0.0;
    add_external(F, e_x, f_rep, hi0, lo0, step, a.c.h, a.has_pull ? a.pull_slot[i] : -1, a.pulls, a.tip,
                 ENERGY, a.err);
    if (ENERGY) {
        const double4 e = a.eacc[i];
        a.eacc[i] = make_double4(0.0, 0.0, 0.0, 0.0);
        double *er = a.res_energy + (size_t)i * RES_E;
        er[0] = e.x;
        er[1] = e.y;
        er[2] = e.z;
        er[3] = e_x;
        er[4] = e.w;
        er[5] = f_rep;
    }
    if (MODE == 1) {
        a.fout[i] = make_float4(F.fx, F.fy, F.fz, 0.0f);
        return;
    }
    float g[3] = {0.0f, 0.0f, 0.0f};
    const uint2 key = a.noise_key[i];
    if (!(key.x >> 31)) {
        const uint4 w = noise_words(key.x, key.y, step, a.c);
        const float2 gxy = gaussian_pair(w);
        g[0] = gxy.x;
        g[1] = gxy.y;
        g[2] = gaussian_axis(w, 2);
    }
    float4 hi = hi0, lo = lo0;
    if (a.vel) {
        float4 v = a.vel[i];
        underdamped_update(hi, lo, v, F, g, a.ud, a.err);
        a.vel[i] = v;
    } else {
        update_with_noise(hi, lo, F, g, a.c, a.err);
    }
    a.pout[2 * i] = hi;
    a.pout[2 * i + 1] = lo;
    if (a.check_thr2 > 0.0f) {
        const float4 hs = a.hi_skin[i];
        const float dx = hi.x - hs.x, dy = hi.y - hs.y, dz = hi.z - hs.z;
        if (!(dx * dx + dy * dy + dz * dz <= a.check_thr2))
            atomicOr(a.skin_flag, 1u);
    }
    if (a.do_bin)
        bin_one(hi, i, __float_as_int(lo.w), a.g, a.traj_cell, a.cell_count, a.cells, a.cell_of, a.err);
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
    const int *pack_off;      // first slot of each pack (n_packs + 1)
    const int *slot_res;      // residue of each slot; a pack's trajectories are consecutive
    const int *traj_lo;
    const int *traj_hi;
    const unsigned *stream_ids;
    const int *pull_slot;
    const PullDev *pulls;
    unsigned short *list;     // entry k of residue i at i*cap + k
    int *list_cnt;
    double *energy;
    double *f_ext;
    float4 *fout;
    unsigned *err;
    const long long *step_base;
    const float *tscale;      // per trajectory: noise amplitude factor (replica exchange), or NULL
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

// Batched schedule: the list partners of a residue are summed by one lane,
// pair by pair in row order, so the sum does not depend on the lane or on
// the packing. Which lane sums which row is chosen at each list rebuild by a
// counting sort on the row length (longest first), so the lanes of a wave
// run loops of about the same length.
constexpr int NBUCKET = 64;

template <int WGS, int MODE>
__global__ __launch_bounds__(WGS, 4) void k_batch(BatchArgs a)
{
    constexpr int TCAP = 8 * WGS;  // bonded/native entries of a pack kept in LDS
    __shared__ float4 shh[WGS + 1];     // {hi.xyz, packed lo} per residue; slot WGS: the far-away empty slot
    __shared__ float4 shl[WGS + 1];     // lo per residue
    __shared__ double red[WGS];         // trajectory sums
    __shared__ unsigned short tpart[TCAP];  // bonded/native entries of the pack: local partner
    __shared__ float tr0[TCAP];             // ... and r0 (CSR in slot order)
    __shared__ unsigned short tex[TCAP];    // the same partners in ascending order (list exclusions)
    __shared__ int perm[WGS];           // row summed by each lane: residue | chunks << 16
    __shared__ float lsum[3][WGS];      // list force of each residue
    __shared__ int hist[NBUCKET];
    __shared__ int sres[WGS];           // residue of each local slot
    __shared__ float3 bblo[WGS / 32], bbhi[WGS / 32];  // list rebuild: boxes of 32-slot blocks
    const int p = blockIdx.x;
    const int off = a.pack_off[p];
    const int n = a.pack_off[p + 1] - off;
    const int t = threadIdx.x;
    const bool act = t < n;
    const int i = act ? a.slot_res[off + t] : 0;  // this lane's residue
    // local slot of a residue of the same trajectory: residue + shift
    const int shift = t - i;

    float4 hi = make_float4(0.f, 0.f, 0.f, 0.f), lo = hi;
    int tlo = 0, thi = 0;
    int2 row = make_int2(0, 0);
    int cnt = 0;
    if (act) {
        hi = a.pin[2 * i];
        lo = a.pin[2 * i + 1];
        tlo = a.traj_lo[i] + shift;
        thi = a.traj_hi[i] + shift;
        row = a.trow[i];
        cnt = a.list_cnt[i];
        shh[t] = make_float4(hi.x, hi.y, hi.z, __uint_as_float(pack_low_res(hi, lo)));
        shl[t] = lo;
    }
    sres[t] = i;
    if (t == 0) {
        shh[WGS] = make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.0f);
        shl[WGS] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    const int nb = row.y & 4095, ntop = nb + (row.y >> 12);
    // the pack's bonded/native entries in LDS (entries past TCAP stay in
    // global memory); perm is the scan's workspace until the first assignment
    int tot_top = 0;
    const int toff = block_exclusive_scan<WGS>(ntop, perm, tot_top);
    const bool top_lds = toff + ntop <= TCAP;  // all of this residue's entries are in LDS
    for (int e = 0; e < ntop && toff + e < TCAP; ++e) {
        const float2 te = a.tent[row.x + e];
        const unsigned short j = (unsigned short)(__float_as_int(te.x) + shift);
        tpart[toff + e] = j;
        tr0[toff + e] = te.y;
        if (top_lds) {  // insertion into the ascending copy
            int k = e;
            while (k > 0 && tex[toff + k - 1] > j) {
                tex[toff + k] = tex[toff + k - 1];
                --k;
            }
            tex[toff + k] = j;
        }
    }
    auto partner = [&](int e) {
        return toff + e < TCAP ? (int)tpart[toff + e] : __float_as_int(a.tent[row.x + e].x) + shift;
    };
    // rows are residue-major: entry k (a local slot) of residue i at i cap + k
    unsigned short *lrow16 = a.list + (size_t)i * a.cap;
    const long long s0 = (a.step_base ? *a.step_base : 0) + a.step_off;
    const PairConsts kc = pair_consts(a.c);
    const int traj = __float_as_int(lo.w);
    // this trajectory's temperature (fixed within a launch)
    StepConsts cn = a.c;
    if (a.tscale && act)
        cn.c_noise *= a.tscale[traj];
    const unsigned stream = act ? a.stream_ids[traj] : 0u;

    // lane -> row assignment: counting sort of the rows by chunk count,
    // longest first (ties in any order; the sums do not depend on it)
    int my = 0;   // local slot | chunks << 16 of the row this lane sums
    int myg = 0;  // its residue
    auto assign = [&]() {
        const int nch = act ? (min(cnt, a.cap) + 3) >> 2 : 0;
        const int key = NBUCKET - 1 - min(nch, NBUCKET - 1);
        if (t < NBUCKET)
            hist[t] = 0;
        __syncthreads();
        if (act)
            atomicAdd(&hist[key], 1);
        __syncthreads();
        if (t < 64) {  // one wave scans the buckets
            const int v = t < NBUCKET ? hist[t] : 0;
            int x = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (t >= o)
                    x += y;
            }
            if (t < NBUCKET)
                hist[t] = x - v;
        }
        __syncthreads();
        if (act)
            perm[atomicAdd(&hist[key], 1)] = t | (nch << 16);
        __syncthreads();
        my = t < n ? perm[t] : 0;
        myg = sres[my & 0xffff];
    };
    __syncthreads();
    if (!(a.stale || s0 % a.list_every == 0))
        assign();

    for (int q = 0; q < a.n_steps; ++q) {
        const long long step = s0 + q;
        if ((q == 0 && a.stale) || step % a.list_every == 0) {
            {
                // boxes of the 32-slot blocks (empty slots add nothing)
                float3 bl = act ? make_float3(hi.x, hi.y, hi.z) : make_float3(3.0e38f, 3.0e38f, 3.0e38f);
                float3 bh = act ? make_float3(hi.x, hi.y, hi.z) : make_float3(-3.0e38f, -3.0e38f, -3.0e38f);
#pragma unroll
                for (int o = 1; o < 32; o <<= 1) {
                    bl.x = fminf(bl.x, __shfl_xor(bl.x, o, 64));
                    bl.y = fminf(bl.y, __shfl_xor(bl.y, o, 64));
                    bl.z = fminf(bl.z, __shfl_xor(bl.z, o, 64));
                    bh.x = fmaxf(bh.x, __shfl_xor(bh.x, o, 64));
                    bh.y = fmaxf(bh.y, __shfl_xor(bh.y, o, 64));
                    bh.z = fmaxf(bh.z, __shfl_xor(bh.z, o, 64));
                }
                if ((t & 31) == 0) {
                    bblo[t >> 5] = bl;
                    bbhi[t >> 5] = bh;
                }
                __syncthreads();
            }
            if (act) {
                // Algorithm 3 over the trajectory: r < r_list, not bonded or
                // native. Candidates are tested a 32-slot block at a time into
                // a bit word (blocks whose box is out of reach of every lane of
                // the wave are skipped); the row is written four entries (one
                // 8-byte chunk) at a time.
                uint2 *rowp = reinterpret_cast<uint2 *>(lrow16);
                unsigned w_lo = 0u, w_hi = 0u;
                int ep = 0;  // next entry of the ascending exclusion list
                cnt = 0;
                for (int jb = tlo >> 5; jb <= (thi - 1) >> 5; ++jb) {
                    const int j0 = jb << 5;
                    {
                        // the box test errs on the side of testing: a skipped
                        // block is farther than r_list by a margin far above
                        // the rounding of either distance
                        const float3 bl = bblo[jb], bh = bbhi[jb];
                        const float gx = fmaxf(fmaxf(bl.x - hi.x, hi.x - bh.x), 0.0f);
                        const float gy = fmaxf(fmaxf(bl.y - hi.y, hi.y - bh.y), 0.0f);
                        const float gz = fmaxf(fmaxf(bl.z - hi.z, hi.z - bh.z), 0.0f);
                        if (!__any(gx * gx + gy * gy + gz * gz <= a.rc2 * 1.001f))
                            continue;
                    }
                    // candidate j0 + u at bit 31 - u; slots of other
                    // trajectories are masked
                    unsigned m = 0u;
#pragma unroll 1
                    for (int u0 = 0; u0 < 32; u0 += 8) {
                        float4 q[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            q[u] = shh[j0 + u0 + u];
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            m = m + m + (within_cutoff(hi, q[u], a.rc2) ? 1u : 0u);
                    }
                    m &= 0xffffffffu >> max(tlo - j0, 0);
                    if (thi - j0 < 32)
                        m &= ~(0xffffffffu >> (thi - j0));
                    unsigned x = 0u;  // the residue itself and its bonded/native partners
                    auto drop = [&](int j) {
                        const unsigned d = (unsigned)(j - j0);
                        x |= d < 32u ? (0x80000000u >> d) : 0u;
                    };
                    drop(t);
                    if (top_lds) {
                        for (; ep < ntop; ++ep) {  // entries below this block were passed by skipped blocks
                            const int j = tex[toff + ep];
                            if (j >= j0 + 32)
                                break;
                            drop(j);
                        }
                    } else {
                        for (int e = 0; e < ntop; ++e)
                            drop(partner(e));
                    }
                    m &= ~x;
                    while (m) {
                        const int u = __builtin_clz(m);
                        const unsigned v = (unsigned)(j0 + u);
                        m ^= 0x80000000u >> u;
                        const int sl = cnt & 3;
                        if (sl == 0)
                            w_lo = v;
                        else if (sl == 1)
                            w_lo |= v << 16;
                        else if (sl == 2)
                            w_hi = v;
                        else
                            w_hi |= v << 16;
                        ++cnt;
                        if ((cnt & 3) == 0 && cnt <= a.cap)
                            rowp[(cnt >> 2) - 1] = make_uint2(w_lo, w_hi);
                    }
                }
                // pad the last chunk with the empty slot (its term is exactly zero)
                const int sl = cnt & 3;
                if (sl != 0 && cnt < a.cap) {
                    const unsigned e2 = (unsigned)WGS | ((unsigned)WGS << 16);
                    if (sl == 1)
                        rowp[cnt >> 2] = make_uint2(w_lo | ((unsigned)WGS << 16), e2);
                    else if (sl == 2)
                        rowp[cnt >> 2] = make_uint2(w_lo, e2);
                    else
                        rowp[cnt >> 2] = make_uint2(w_lo, w_hi | ((unsigned)WGS << 16));
                }
                if (cnt > a.cap)
                    atomicOr(a.err, ERR_OVERFLOW);
                a.list_cnt[i] = cnt;
            }
            assign();  // its barriers also publish the rows written above
        }
        // mode 0 never records (no FP64 sums in its registers); mode 2
        // records at multiples of the energy interval, in a copy of the
        // forces and update compiled for record steps alone
        const bool rec_step = MODE == 1 || (MODE == 2 && a.energy_every > 0 && step % a.energy_every == 0);
        auto forces_and_update = [&](auto rec_tag) {
            constexpr bool rec = decltype(rec_tag)::value;
            {
                // ---- list partners (forces) of the row this lane was given ----
                const int r = my & 0xffff, nch = my >> 16;
                const float4 ph = shh[r], pl = shl[r];
                // rows are read two chunks (16 bytes) at a time, the next pair
                // requested before the current one is used
                const uint4 *rp = reinterpret_cast<const uint4 *>(a.list + (size_t)myg * a.cap);
                const int nc2 = (nch + 1) >> 1;
                Acc L;  // the row's sum, pair by pair in row order
                auto chunk = [&](unsigned wx, unsigned wy) {
                    const unsigned idx[4] = {wx & 0xffffu, wx >> 16, wy & 0xffffu, wy >> 16};
                    // one 16-byte read a partner: the high part and its packed
                    // low part (10-bit multiples of the partner's quantum)
                    float4 qh[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        qh[u] = shh[idx[u]];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        add_repulsive_u(L, pair_delta_packed(ph, pl, qh[u]), kc, false);
                };
                uint4 w = rp[0];
                for (int c2 = 0; c2 < nc2; ++c2) {
                    const uint4 wn = rp[min(c2 + 1, nc2 - 1)];
                    chunk(w.x, w.y);
                    if (2 * c2 + 1 < nch)  // the second chunk of an odd row's last pair is not written
                        chunk(w.z, w.w);
                    w = wn;
                }
                if (t < n) {
                    lsum[0][r] = kc.c6 * L.fx;
                    lsum[1][r] = kc.c6 * L.fy;
                    lsum[2][r] = kc.c6 * L.fz;
                }
            }
            Acc A;  // energy sums are only accumulated on record steps
            bool broken = false;
            double e_x = 0.0, f_rep = 0.0;
            if (act) {
                // bonded, then native partners: two loops, so a wave whose
                // residues have different bond counts (chain ends) runs each
                // term's code alone
                auto entry = [&](int e, int &j, float &r0) {
                    if (toff + e < TCAP) {
                        j = tpart[toff + e];
                        r0 = tr0[toff + e];
                    } else {
                        const float2 te = a.tent[row.x + e];
                        j = __float_as_int(te.x) + shift;
                        r0 = te.y;
                    }
                };
                for (int e = 0; e < nb; ++e) {
                    int j;
                    float r0;
                    entry(e, j, r0);
                    add_fene(A, hi, lo, shh[j], shl[j], r0, kc, rec, broken);
                }
                for (int e = nb; e < ntop; ++e) {
                    int j;
                    float r0;
                    entry(e, j, r0);
                    add_native(A, hi, lo, shh[j], shl[j], r0, kc, rec);
                }
                add_external(A, e_x, f_rep, hi, lo, step, a.c.h, a.has_pull ? a.pull_slot[i] : -1, a.pulls,
                             a.tip, rec, a.err);
                if (broken)
                    atomicOr(a.err, ERR_FENE);
                if (rec) {
                    // record steps: the repulsive energy and virial over the own row
                    Acc E;
                    for (int k = 0; k < min(cnt, a.cap); ++k)
                        add_repulsive_d(E, pair_delta(hi, lo, shh[lrow16[k]], shl[lrow16[k]]), kc, true);
                    A.e_r = E.e_r;
                    A.vir += E.vir;
                }
            }
            __syncthreads();
            if (act) {
                A.fx += lsum[0][t];
                A.fy += lsum[1][t];
                A.fz += lsum[2][t];
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
            if (act) {
                langevin_update(hi, lo, A, step, stream, cn, a.err);
                shh[t] = make_float4(hi.x, hi.y, hi.z, __uint_as_float(pack_low_res(hi, lo)));
                shl[t] = lo;
            }
            __syncthreads();
        };
        if constexpr (MODE == 1) {
            forces_and_update(std::true_type{});
            return;
        } else if constexpr (MODE == 0) {
            forces_and_update(std::false_type{});
        } else {
            if (rec_step)
                forces_and_update(std::true_type{});
            else
                forces_and_update(std::false_type{});
        }
    }
    if (MODE != 1 && act) {
        a.pout[2 * i] = hi;
        a.pout[2 * i + 1] = lo;
    }
}

// Replica exchange: one lane per attempted swap of round `round` (the
// temperatures k, k+1 with k = round mod 2, round mod 2 + 2, ... of every
// group of n_rep consecutive trajectories), Metropolis on the potential
// energies recorded at this step, with a Philox draw under a key of its
// own.  Swaps of one round touch disjoint trajectories.
__global__ void k_exchange(const double *__restrict__ energy, const double *__restrict__ kbt, int n_rep,
                           int n_groups, int *__restrict__ tidx, float *__restrict__ tscale, double kbt_ref,
                           long long round, unsigned key0, unsigned key1, unsigned long long *__restrict__ stats)
{
    const int par = (int)(round & 1);
    const int pairs = (n_rep - par) / 2;  // k = par, par + 2, ... with k + 1 < n_rep
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (pairs <= 0 || id >= n_groups * pairs)
        return;
    const int g = id / pairs, k = par + 2 * (id % pairs);
    const int base = g * n_rep;
    int ta = -1, tb = -1;
    for (int m = 0; m < n_rep; ++m) {
        const int v = tidx[base + m];
        ta = v == k ? base + m : ta;
        tb = v == k + 1 ? base + m : tb;
    }
    if (ta < 0 || tb < 0)
        return;  // not a permutation (rejected on the host)
    double Ea = 0.0, Eb = 0.0;
    for (int term = 0; term < 4; ++term) {
        Ea += energy[(size_t)ta * SOP_NTERMS + term];
        Eb += energy[(size_t)tb * SOP_NTERMS + term];
    }
    const double d = (1.0 / kbt[k] - 1.0 / kbt[k + 1]) * (Ea - Eb);
    const uint4 w = philox10(make_uint4((unsigned)g, (unsigned)k, (unsigned)round,
                                        (unsigned)((unsigned long long)round >> 32)),
                             key0 ^ 0x52455843u, key1);
    const double u = ((double)(w.x >> 9) + 0.5) * 0x1p-23;
    atomicAdd(&stats[2 * k + 1], 1ull);
    if (d >= 0.0 || u < exp(d)) {
        atomicAdd(&stats[2 * k], 1ull);
        tidx[ta] = k + 1;
        tidx[tb] = k;
        tscale[ta] = (float)sqrt(kbt[k + 1] / kbt_ref);
        tscale[tb] = (float)sqrt(kbt[k] / kbt_ref);
    }
}

__global__ void k_add_step(long long *base, long long k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *base += k;
}

// One workgroup per trajectory: double sums of the per-residue records.
// Per-trajectory FP64 energy and virial sums in two fixed-order levels:
// one workgroup per chunk of at most ECHUNK residues of one trajectory, then
// one lane per trajectory over its chunks in order.
__global__ __launch_bounds__(WG) void k_reduce_chunks(const double *__restrict__ res_energy,
                                                      const int *__restrict__ chunk_lo,
                                                      double *__restrict__ chunk_sum)
{
    __shared__ double part[WG / 64][RES_E];
    const int ch = blockIdx.x;
    const int a = chunk_lo[ch], b = chunk_lo[ch + 1];
    double s[RES_E] = {0, 0, 0, 0, 0, 0};
    for (int i = a + threadIdx.x; i < b; i += WG)
#pragma unroll
        for (int k = 0; k < RES_E; ++k)
            s[k] += res_energy[(size_t)i * RES_E + k];
#pragma unroll
    for (int k = 0; k < RES_E; ++k)
        for (int m = 32; m >= 1; m >>= 1)
            s[k] += __shfl_xor(s[k], m, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < RES_E; ++k)
            part[threadIdx.x >> 6][k] = s[k];
    __syncthreads();
    if (threadIdx.x < RES_E) {
        double v = 0.0;
        for (int w = 0; w < WG / 64; ++w)
            v += part[w][threadIdx.x];
        chunk_sum[(size_t)ch * RES_E + threadIdx.x] = v;
    }
}

// One wave per trajectory: lane l takes chunks l, l + 64, ... in order, then
// a fixed butterfly over the lanes.
__global__ __launch_bounds__(WG) void k_reduce_energy(const double *__restrict__ chunk_sum,
                                                      const int *__restrict__ chunk_first, int n_traj,
                                                      double *__restrict__ energy, double *__restrict__ f_ext)
{
    const int t = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
    if (t >= n_traj)
        return;  // uniform over the wave
    double v[RES_E] = {0, 0, 0, 0, 0, 0};
    for (int ch = chunk_first[t] + lane; ch < chunk_first[t + 1]; ch += 64)
#pragma unroll
        for (int k = 0; k < RES_E; ++k)
            v[k] += chunk_sum[(size_t)ch * RES_E + k];
#pragma unroll
    for (int k = 0; k < RES_E; ++k)
        for (int m = 32; m >= 1; m >>= 1)
            v[k] += __shfl_xor(v[k], m, 64);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < SOP_NTERMS; ++k)
            energy[(size_t)t * SOP_NTERMS + k] = v[k];
        f_ext[t] = v[SOP_NTERMS];
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

__global__ void k_set_flag(unsigned *dst, unsigned v)
{
    if (threadIdx.x == 0)
        *dst = v;
}

__global__ void k_set_step(long long *dst, long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dst = v;
}

inline int blocks_for(long long n, int per) { return (int)((n + per - 1) / per); }

template <int TILE>
void canon_tile(const DevBufs &b, int cap, hipStream_t s)
{
    CanonArgs a{};
    a.tile_first = b.tile_first[tile_index(TILE)];
    a.trow = b.trow;
    a.stage = b.stage;
    a.stage_cnt = b.stage_cnt;
    a.skin16 = b.list16;
    a.skin_cnt = b.list_cnt;
    a.topo2 = b.topo2;
    a.skin_flag = b.skin_flag;
    a.skin_ord = b.skin_ord;
    a.cap = cap;
    hipLaunchKernelGGL((k_canon<TILE>), dim3(b.n_tiles[tile_index(TILE)]), dim3(256), 0, s, a);
}

template <int TILE>
void filter_tile(const DevBufs &b, int cur, int cap, const GridDev &g, float rc2, hipStream_t s)
{
    FilterArgs a{};
    a.tile_first = b.tile_first[tile_index(TILE)];
    a.pos = b.pos[cur];
    a.stage = b.stage;
    a.stage_cnt = b.stage_cnt;
    a.skin16 = b.list16;
    a.skin_cnt = b.list_cnt;
    a.list16 = b.flist16;
    a.list_cnt = b.fcnt;
    a.cell_count = b.cell_count;
    a.skin_flag = b.skin_flag;
    a.tile_ord = b.tile_ord;
    a.skin_ord = b.skin_ord;
    a.rc2 = rc2;
    a.cap = cap;
    a.n_cells = g.n_cells;
    hipLaunchKernelGGL((k_filter<TILE>), dim3(b.n_tiles[tile_index(TILE)]), dim3(256), 0, s, a);
}

template <int TILE>
void rebuild_tile(const DevBufs &b, int cur, int n, int cap, const GridDev &g, float rc2, int multi,
                  hipStream_t s, bool advance, int period)
{
    BuildArgs a{};
    a.step_base = advance ? b.step_base : nullptr;
    a.step_next = b.step_next;
    a.period = period;
    a.tile_first = b.tile_first[tile_index(TILE)];
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
    a.skin_flag = b.skin_flag;
    a.hi_skin = b.hi_skin;
    a.stats = b.list_stats;
    a.g = g;
    a.rc2 = rc2;
    a.n = n;
    a.cap = cap;
    const int nt = b.n_tiles[tile_index(TILE)];
    if (multi)
        hipLaunchKernelGGL((k_tile_build<TILE, true>), dim3(nt), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_tile_build<TILE, false>), dim3(nt), dim3(256), 0, s, a);
}

template <int TILE, bool ENERGY, int MODE, bool FIRST>
void tile_step(const TileArgs &a, hipStream_t s)
{
    const int blocks = ((a.n_tiles + 7) / 8) * 8;
    const TileArgs &x = a;
    hipLaunchKernelGGL((k_tile_step<TILE, ENERGY, MODE, FIRST>), dim3(blocks), dim3(256), 0, s, x);
}

template <bool ENERGY, int MODE, bool FIRST = false>
void tile_dispatch(int tile, const TileArgs &a, hipStream_t s)
{
    switch (tile) {
    case 64: tile_step<64, ENERGY, MODE, FIRST>(a, s); break;
    case 128: tile_step<128, ENERGY, MODE, FIRST>(a, s); break;
    default: tile_step<256, ENERGY, MODE, FIRST>(a, s); break;
    }
}

}  // namespace

void launch_rebuild(const DevBufs &b, int cur, int n, int cap, int tile, const GridDev &g, float rc2,
                    float rs2, int multi, hipStream_t s, bool advance_step_base, int list_every, bool binned,
                    bool filter)
{
    if (!binned)
        launch_bin_all(b, cur, n, g, s);  // not binned by a period's last step kernel
    switch (tile) {
    case 64:
        rebuild_tile<64>(b, cur, n, cap, g, rs2, multi, s, advance_step_base, list_every);
        canon_tile<64>(b, cap, s);
        if (filter)
            filter_tile<64>(b, cur, cap, g, rc2, s);
        break;
    case 128:
        rebuild_tile<128>(b, cur, n, cap, g, rs2, multi, s, advance_step_base, list_every);
        canon_tile<128>(b, cap, s);
        if (filter)
            filter_tile<128>(b, cur, cap, g, rc2, s);
        break;
    default:
        rebuild_tile<256>(b, cur, n, cap, g, rs2, multi, s, advance_step_base, list_every);
        canon_tile<256>(b, cap, s);
        if (filter)
            filter_tile<256>(b, cur, cap, g, rc2, s);
        break;
    }
}

void launch_bin_all(const DevBufs &b, int cur, int n, const GridDev &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear, dim3(blocks_for(g.n_cells, WG)), dim3(WG), 0, s, b.cell_count, g.n_cells);
    hipLaunchKernelGGL(k_bin_all, dim3(blocks_for(n, WG)), dim3(WG), 0, s, b.pos[cur], n, g, b.traj_cell,
                       b.cell_count, b.cells, b.cell_of, b.err);
}

void launch_force_skin(const DevBufs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, s, b.skin_flag, 1u);
}

template <int TILE>
void pair_forces(const PairArgs &a, bool energy, hipStream_t s)
{
    if (energy)
        hipLaunchKernelGGL((k_pair_forces<TILE, true>), dim3(a.n_tiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_pair_forces<TILE, false>), dim3(a.n_tiles), dim3(256), 0, s, a);
}

void launch_pair_step(const DevBufs &b, int cur, int n, int cap, int tile, const StepConsts &c,
                      const TipDev &tip, int has_pull, bool energy, int mode, const long long *step_base,
                      long long step_off, float check_thr2, hipStream_t s, const float4 *vel,
                      const UdConsts &ud, const GridDev *bin_grid)
{
    PairArgs a{};
    a.tile_first = b.tile_first[tile_index(tile)];
    a.n_tiles = b.n_tiles[tile_index(tile)];
    a.pin = b.pos[cur];
    a.trow = b.trow;
    a.tent = b.tent;
    a.list16 = b.flist16;
    a.list_cnt = b.fcnt;
    a.stage = b.stage;
    a.stage_cnt = b.stage_cnt;
    a.facc = b.facc;
    a.eacc = b.eacc;
    a.err = b.err;
    a.cap = cap;
    a.c = c;
    switch (tile) {
    case 64: pair_forces<64>(a, energy, s); break;
    case 128: pair_forces<128>(a, energy, s); break;
    default: pair_forces<256>(a, energy, s); break;
    }
    PairUpdArgs u{};
    u.pin = b.pos[cur];
    u.pout = b.pos[cur ^ 1];
    u.facc = b.facc;
    u.eacc = b.eacc;
    u.noise_key = b.noise_key;
    u.pull_slot = b.pull_slot;
    u.pulls = b.pulls;
    u.res_energy = b.res_energy;
    u.fout = b.fout;
    u.err = b.err;
    u.step_base = step_base;
    u.hi_skin = b.hi_skin;
    u.skin_flag = b.skin_flag;
    u.step_off = step_off;
    u.check_thr2 = mode == 0 ? check_thr2 : 0.0f;
    u.vel = const_cast<float4 *>(vel);
    u.ud = ud;
    u.do_bin = (mode == 0 && bin_grid) ? 1 : 0;
    if (bin_grid)
        u.g = *bin_grid;
    u.traj_cell = b.traj_cell;
    u.cell_count = b.cell_count;
    u.cells = b.cells;
    u.cell_of = b.cell_of;
    u.n = n;
    u.has_pull = has_pull;
    u.c = c;
    u.tip = tip;
    const dim3 g(blocks_for(n, WG));
    if (mode == 1) {
        if (energy)
            hipLaunchKernelGGL((k_pair_update<true, 1>), g, dim3(WG), 0, s, u);
        else
            hipLaunchKernelGGL((k_pair_update<false, 1>), g, dim3(WG), 0, s, u);
    } else {
        if (energy)
            hipLaunchKernelGGL((k_pair_update<true, 0>), g, dim3(WG), 0, s, u);
        else
            hipLaunchKernelGGL((k_pair_update<false, 0>), g, dim3(WG), 0, s, u);
    }
}

void launch_step(const DevBufs &b, int cur, int n, int cap, int tile, const StepConsts &c,
                 const TipDev &tip, int has_pull, bool energy, int mode, const long long *step_base,
                 long long step_off, float check_thr2, hipStream_t s, int force_mode, float ud_kick,
                 const GridDev *bin_grid, float filter_rc2, int n_cells)
{
    // underdamped when ud_kick > 0 (velocities in b.vel)
    const float4 *vel = ud_kick > 0.0f ? b.vel : nullptr;
    UdConsts ud{ud_kick, c.ud_c1, c.ud_c2, (float)(0.5 * c.h)};
    if (force_mode == 1) {
        launch_pair_step(b, cur, n, cap, tile, c, tip, has_pull, energy, mode, step_base, step_off,
                         check_thr2, s, vel, ud, bin_grid);
        return;
    }
    TileArgs a{};
    a.vel = const_cast<float4 *>(vel);
    a.ud = ud;
    a.do_bin = (mode == 0 && bin_grid) ? 1 : 0;
    if (bin_grid)
        a.g = *bin_grid;
    a.traj_cell = b.traj_cell;
    a.cell_count = b.cell_count;
    a.cells = b.cells;
    a.cell_of = b.cell_of;
    a.tile_ord = b.tile_ord;
    a.hi_skin = b.hi_skin;
    a.skin_flag = b.skin_flag;
    a.check_thr2 = mode == 0 ? check_thr2 : 0.0f;
    a.tile_first = b.tile_first[tile_index(tile)];
    a.n_tiles = b.n_tiles[tile_index(tile)];
    a.pin = b.pos[cur];
    a.pout = b.pos[cur ^ 1];
    a.trow = b.trow;
    a.tent = b.tent;
    a.list16 = b.flist16;
    a.topo2 = b.topo2;
    a.list_cnt = b.fcnt;
    a.stage = b.stage;
    a.stage_cnt = b.stage_cnt;
    a.stream_ids = b.stream_ids;
    a.noise_key = b.noise_key;
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
    if (mode == 0 && filter_rc2 > 0.0f) {
        // the first step after a rebuild, which filters the skin rows itself
        // (never a binning step: the callers bin only at a period's end)
        a.skin16 = b.list16;
        a.skin_cnt = b.list_cnt;
        a.skin_ord = b.skin_ord;
        a.list16_out = b.flist16;
        a.list_cnt_out = b.fcnt;
        a.tile_ord_out = b.tile_ord;
        a.rc2 = filter_rc2;
        a.n_cells = n_cells;
        if (energy)
            tile_dispatch<true, 0, true>(tile, a, s);
        else
            tile_dispatch<false, 0, true>(tile, a, s);
        return;
    }
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
                  hipStream_t s, const float *tscale)
{
    BatchArgs a{};
    a.pin = b.pos[cur];
    a.pout = b.pos[cur ^ 1];
    a.trow = b.trow;
    a.tent = b.tent;
    a.pack_off = b.pack_off;
    a.slot_res = b.slot_res;
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
    a.tscale = tscale;
    const dim3 grid(n_packs);
    if (mode == 1) {
        switch (wg) {
        case 256: hipLaunchKernelGGL((k_batch<256, 1>), grid, dim3(256), 0, s, a); break;
        case 512: hipLaunchKernelGGL((k_batch<512, 1>), grid, dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL((k_batch<1024, 1>), grid, dim3(1024), 0, s, a); break;
        }
    } else if (mode == 2) {
        switch (wg) {
        case 256: hipLaunchKernelGGL((k_batch<256, 2>), grid, dim3(256), 0, s, a); break;
        case 512: hipLaunchKernelGGL((k_batch<512, 2>), grid, dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL((k_batch<1024, 2>), grid, dim3(1024), 0, s, a); break;
        }
    } else {
        switch (wg) {
        case 256: hipLaunchKernelGGL((k_batch<256, 0>), grid, dim3(256), 0, s, a); break;
        case 512: hipLaunchKernelGGL((k_batch<512, 0>), grid, dim3(512), 0, s, a); break;
        default: hipLaunchKernelGGL((k_batch<1024, 0>), grid, dim3(1024), 0, s, a); break;
        }
    }
}

void launch_exchange(const DevBufs &b, int n_rep, int n_groups, double kbt_ref, long long round,
                     unsigned key0, unsigned key1, hipStream_t s)
{
    const int pairs = std::max(n_rep / 2, 1);
    hipLaunchKernelGGL(k_exchange, dim3(blocks_for((long long)n_groups * pairs, WG)), dim3(WG), 0, s, b.energy,
                       b.re_kbt, n_rep, n_groups, b.re_tidx, b.re_tscale, kbt_ref, round, key0, key1, b.re_stats);
}

void launch_add_step(long long *base, long long k, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_step, dim3(1), dim3(64), 0, s, base, k);
}

void launch_reduce_energy(const DevBufs &b, int n_traj, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_chunks, dim3(b.n_chunks), dim3(WG), 0, s, b.res_energy, b.chunk_lo,
                       b.chunk_sum);
    hipLaunchKernelGGL(k_reduce_energy, dim3(blocks_for((long long)n_traj * 64, WG)), dim3(WG), 0, s,
                       b.chunk_sum, b.chunk_first, n_traj, b.energy, b.f_ext);
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
