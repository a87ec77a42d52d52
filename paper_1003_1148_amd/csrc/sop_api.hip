// Host side of the C ABI: topology -> per-residue CSR (Algorithm 2's P_p and
// PairsMap, bonds and natives in both directions), workspace layout, the
// step driver with HIP-graph replays of whole list periods, and the
// asynchronous device error word.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "sop_internal.hpp"

using namespace sop;

struct sop_ctx {
    sop_params p{};
    hipStream_t stream = nullptr;

    // topology (host copies)
    int n_traj = 0;
    long long n_res = 0;
    std::vector<long long> res_offsets;
    std::vector<unsigned> stream_ids;
    std::vector<int2> trow;
    std::vector<float2> tent;
    std::vector<int> traj_lo, traj_hi, traj_of, local;
    std::vector<unsigned char> fixed;
    std::vector<PullDev> pulls;
    std::vector<int> pull_slot;
    std::vector<int4> traj_cell;
    std::vector<int> tiles[3];  // plain: first residue of each tile (+ n) for tiles of 64, 128, 256
    std::vector<int> chunk_lo, chunk_first;  // energy reduction chunks
    TipDev tip{};

    // schedule: plain (kernel per step) or batched (persistent packs)
    int schedule = SOP_SCHEDULE_PLAIN;
    int tile_req = 0, tile = 128, cap = 256, cap_req = 0;
    // plain: the Verlet skin.  Rows of pairs within r_list + skin are built
    // on the cell grid only when some residue has moved more than skin/2
    // since the last such build; every rebuild filters them to r_list.
    double skin = 4.0;
    int force_mode = SOP_FORCES_PARTICLE;  // plain: particle- or pair-based force evaluation
    int integrator = SOP_INTEGRATOR_OVERDAMPED;
    double mass = 1.0;               // underdamped: mass of a residue
    // batched: replica exchange over groups of re_rep consecutive trajectories
    int re_rep = 0;
    std::vector<double> re_kbt;
    long long re_every = 0, re_last = -1;
    bool ud_half = true;             // underdamped: the stored velocities are at the current step
    long long skin_checked = -1;     // step at which the skin was last known valid
    long long binned_at = -1;        // step whose positions the cells hold (consumed by a rebuild)
    std::vector<double> xyz_set;     // the coordinates the grid was laid out for
    int graph_steps = 1;
    long long energy_every = 0;
    int batch_wg_req = 0, batch_wg = 1024, batch_steps = 100;
    long long max_len = 0;           // longest trajectory
    std::vector<int> pack_off;       // batched: first slot of each pack
    std::vector<int> slot_res;       // batched: residue of each slot
    hipGraphExec_t bgraphs[2][2] = {};  // batched launch graphs by layer parity, records

    // device state
    bool topo = false, bound = false, coords = false, list_valid = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    DevBufs b{};
    GridDev grid{};
    int n_cells_cap = 0;
    int cur = 0;
    long long step = 0;
    long long energy_step = -1;
    unsigned sticky = 0;
    std::string last_error;

    // graphs over whole list periods, keyed by [layer parity][energy at first step]
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graphs[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
};

namespace {

sop_status fail(sop_ctx *c, sop_status s, const std::string &msg)
{
    if (c)
        c->last_error = msg;
    return s;
}

sop_status hip_fail(sop_ctx *c, hipError_t e, const char *what)
{
    return fail(c, SOP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                 \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess)                              \
            return hip_fail((ctx), e_, #expr);             \
    } while (0)

// A list that overflowed leaves the forces undefined, so it is reported first.
sop_status status_from_bits(unsigned bits)
{
    if (bits & (ERR_OVERFLOW | ERR_CELL | ERR_STAGE))
        return SOP_E_LIST_OVERFLOW;
    if (bits & ERR_FENE)
        return SOP_E_FENE;
    if (bits & ERR_TIP)
        return SOP_E_TIP;
    if (bits & ERR_NONFINITE)
        return SOP_E_NONFINITE;
    return SOP_OK;
}

const char *bits_message(unsigned bits)
{
    if (bits & ERR_OVERFLOW)
        return "a residue has more list partners than the list capacity";
    if (bits & ERR_CELL)
        return "more than 256 residues fell into one cell of the list-rebuild grid";
    if (bits & ERR_STAGE)
        return "a tile of the plain schedule interacts with more residues than its LDS staging holds, or its cell neighbourhood exceeds the rebuild's LDS table";
    if (bits & ERR_FENE)
        return "a FENE bond reached |r - r0| >= R0";
    if (bits & ERR_TIP)
        return "a residue reached the tip surface";
    if (bits & ERR_NONFINITE)
        return "a force or position became non-finite";
    return "";
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Row capacity: the requested one, else 1024 entries for the plain schedule
// (its skin rows hold the partners within r_list + skin: at protein density,
// about 120 A^3 per residue, some 480 within 24 A) and 256 for the batched
// one; a multiple of 16.
int list_cap(const sop_ctx *c)
{
    const int cap = c->cap_req ? c->cap_req : (c->schedule == SOP_SCHEDULE_PLAIN ? 1024 : 256);
    return ((cap + 15) / 16) * 16;
}

// Workspace layout: returns total bytes; fills pointers when base != null.
size_t layout(const sop_ctx *c, char *base, DevBufs *b)
{
    const size_t n = (size_t)c->n_res;
    const size_t T = (size_t)c->n_traj;
    const bool plain = c->schedule == SOP_SCHEDULE_PLAIN;
    // padded for the largest tile so that any tile size fits
    const size_t n_pad = ((n + 255) / 256) * 256;
    const size_t list16_elems = plain ? n_pad * (size_t)c->cap : n * (size_t)c->cap;
    // per-tile blocks, for the largest need over the tile sizes
    size_t topo2_elems = 0, n_tiles_max = 0, stage_elems = 0, tf_elems[3] = {1, 1, 1};
    if (plain)
        for (int k = 0; k < 3; ++k) {
            const size_t T = (size_t)64 << k, nt = c->tiles[k].size() - 1;
            topo2_elems = std::max(topo2_elems, nt * T * TOPO_CAP);
            stage_elems = std::max(stage_elems, nt * (size_t)stage_max_host((int)T));
            n_tiles_max = std::max(n_tiles_max, nt);
            tf_elems[k] = nt + 1;
        }
    const size_t ncell = plain ? (size_t)c->n_cells_cap : 0;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align256(off + std::max<size_t>(bytes, 1));
        return p;
    };
    DevBufs d{};
    d.pos[0] = (float4 *)take(2 * n * sizeof(float4));
    d.pos[1] = (float4 *)take(2 * n * sizeof(float4));
    d.trow = (int2 *)take(n * sizeof(int2));
    d.tent = (float2 *)take(c->tent.size() * sizeof(float2));
    d.list_cnt = (int *)take(n * sizeof(int));
    d.list16 = (unsigned short *)take(list16_elems * sizeof(unsigned short));
    d.fcnt = (int *)take((plain ? n : 0) * sizeof(int));
    d.flist16 = (unsigned short *)take((plain ? list16_elems : 0) * sizeof(unsigned short));
    d.hi_skin = (float4 *)take((plain ? n : 0) * sizeof(float4));
    d.skin_flag = (unsigned *)take(sizeof(unsigned));
    d.list_stats = (unsigned long long *)take(2 * sizeof(unsigned long long));
    d.tile_ord = (unsigned char *)take(plain ? n_tiles_max * 256 : 0);
    d.skin_ord = (unsigned short *)take((plain ? n_tiles_max * 256 : 0) * sizeof(unsigned short));
    d.vel = (float4 *)take((plain ? n : 0) * sizeof(float4));
    d.facc = (float4 *)take((plain ? n : 0) * sizeof(float4));
    d.re_kbt = (double *)take((plain ? 0 : T) * sizeof(double));
    d.re_tidx = (int *)take((plain ? 0 : T) * sizeof(int));
    d.re_tscale = (float *)take((plain ? 0 : T) * sizeof(float));
    d.re_stats = (unsigned long long *)take((plain ? 0 : 2 * T) * sizeof(unsigned long long));
    d.eacc = (double4 *)take((plain ? n : 0) * sizeof(double4));
    d.topo2 = (uint2 *)take(topo2_elems * sizeof(uint2));
    d.stage = (int *)take(stage_elems * sizeof(int));
    d.stage_cnt = (int *)take(n_tiles_max * sizeof(int));
    d.pack_off = (int *)take((T + 1) * sizeof(int));
    d.slot_res = (int *)take(n * sizeof(int));
    d.pos_save = (float4 *)take(2 * n * sizeof(float4));
    d.cell_count = (int *)take(ncell * sizeof(int));
    d.cells = (float4 *)take(ncell * CELL_CAP * sizeof(float4));
    d.cell_of = (int *)take((plain ? n : 0) * sizeof(int));
    for (int k = 0; k < 3; ++k) {
        d.tile_first[k] = (int *)take(tf_elems[k] * sizeof(int));
        d.n_tiles[k] = plain ? (int)(tf_elems[k] - 1) : 0;
    }
    d.traj_cell = (int4 *)take(T * sizeof(int4));
    d.traj_lo = (int *)take(n * sizeof(int));
    d.traj_hi = (int *)take(n * sizeof(int));
    d.pull_slot = (int *)take(n * sizeof(int));
    d.pulls = (PullDev *)take(std::max<size_t>(c->pulls.size(), 1) * sizeof(PullDev));
    d.stream_ids = (unsigned *)take(T * sizeof(unsigned));
    d.noise_key = (uint2 *)take(n * sizeof(uint2));
    d.res_offsets = (long long *)take((T + 1) * sizeof(long long));
    d.res_energy = (double *)take(n * RES_E * sizeof(double));
    d.n_chunks = (int)c->chunk_lo.size() - 1;
    d.chunk_lo = (int *)take(c->chunk_lo.size() * sizeof(int));
    d.chunk_first = (int *)take(c->chunk_first.size() * sizeof(int));
    d.chunk_sum = (double *)take((size_t)std::max(d.n_chunks, 1) * RES_E * sizeof(double));
    d.energy = (double *)take(T * SOP_NTERMS * sizeof(double));
    d.f_ext = (double *)take(T * sizeof(double));
    d.fout = (float4 *)take(n * sizeof(float4));
    d.words = (uint4 *)take(n * sizeof(uint4));
    d.step_base = (long long *)take(sizeof(long long));
    d.step_next = (long long *)take(sizeof(long long));
    d.err = (unsigned *)take(sizeof(unsigned));
    if (b)
        *b = d;
    return off;
}

// Residues per workgroup of the plain schedule: enough tiles to cover the
// 256 compute units a few times over.
// 64-residue tiles: four lanes per residue in the step kernel, four waves
// sharing each tile's rebuild (sop_autotune measures the others).
int default_tile(long long) { return 64; }

void destroy_graphs(sop_ctx *c)
{
    for (auto &row : c->graphs)
        for (auto &g : row)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    for (auto &gp : c->bgraphs)
        for (auto &g : gp)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

// Packs of whole trajectories for the batched schedule: first-fit
// decreasing by length (ties by index) into workgroups of `wg` residues, so
// packs start with the longest trajectories and all but one are more than
// half full. Inside a pack the trajectories keep their index order, residues
// consecutive. The results do not depend on the packing.
void make_packs(sop_ctx *c)
{
    const int T = c->n_traj, wg = c->batch_wg;
    std::vector<int> order(T);
    for (int t = 0; t < T; ++t)
        order[t] = t;
    auto len = [&](int t) { return c->res_offsets[t + 1] - c->res_offsets[t]; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return len(x) > len(y); });
    // first fit: the leftmost pack with room, from a max-tree over the rooms
    // of T packs (the ones not opened yet are empty, so the leftmost fit is
    // an open pack or the next new one)
    int leaves = 1;
    while (leaves < std::max(T, 1))
        leaves <<= 1;
    std::vector<long long> tree(2 * (size_t)leaves, 0);
    for (int k = 0; k < T; ++k)
        tree[leaves + k] = wg;
    for (int v = leaves - 1; v >= 1; --v)
        tree[v] = std::max(tree[2 * v], tree[2 * v + 1]);
    std::vector<std::vector<int>> members;
    for (int t : order) {
        int v = 1;
        while (v < leaves)
            v = tree[2 * v] >= len(t) ? 2 * v : 2 * v + 1;
        const int k = v - leaves;  // exists: every trajectory fits an empty pack
        if (k >= (int)members.size())
            members.resize(k + 1);
        members[k].push_back(t);
        tree[v] -= len(t);
        for (v >>= 1; v >= 1; v >>= 1)
            tree[v] = std::max(tree[2 * v], tree[2 * v + 1]);
    }
    c->pack_off.assign(1, 0);
    c->slot_res.clear();
    c->slot_res.reserve((size_t)c->n_res);
    for (auto &m : members) {
        std::sort(m.begin(), m.end());
        for (int t : m)
            for (long long r = c->res_offsets[t]; r < c->res_offsets[t + 1]; ++r)
                c->slot_res.push_back((int)r);
        c->pack_off.push_back((int)c->slot_res.size());
    }
}

sop_status upload_packs(sop_ctx *c)
{
    HIP_TRY(c, hipMemcpyAsync(c->b.pack_off, c->pack_off.data(), c->pack_off.size() * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->b.slot_res, c->slot_res.data(), c->slot_res.size() * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
    return SOP_OK;
}

int pick_batch_wg(const sop_ctx *c)
{
    if (c->batch_wg_req)
        return c->batch_wg_req;
    return c->max_len <= 256 ? 256 : (c->max_len <= 512 ? 512 : 1024);
}

int n_packs(const sop_ctx *c) { return (int)c->pack_off.size() - 1; }

StepConsts step_consts(const sop_ctx *c)
{
    StepConsts k{};
    k.k_fene = (float)c->p.k_fene;
    k.R0sq = (float)(c->p.R0 * c->p.R0);
    k.inv_R0sq = (float)(1.0 / (c->p.R0 * c->p.R0));
    k.eps_h = (float)c->p.eps_h;
    k.eps_l = (float)c->p.eps_l;
    k.sigma2 = (float)(c->p.sigma * c->p.sigma);
    k.c_drift = (float)(c->p.h / c->p.zeta);
    k.c_noise = (float)std::sqrt(2.0 * c->p.kBT * c->p.h / c->p.zeta);
    const double c1 = std::exp(-c->p.zeta / c->mass * c->p.h);
    k.ud_c1 = (float)c1;
    k.ud_c2 = (float)std::sqrt((1.0 - c1 * c1) * c->p.kBT / c->mass);
    k.key0 = (unsigned)(c->p.seed & 0xffffffffu);
    k.key1 = (unsigned)(c->p.seed >> 32);
    k.h = c->p.h;
    return k;
}

// Underdamped integrator: the kick of the next step (h/2m right after the
// velocities were set, else h/m); 0 selects the overdamped update.
float ud_kick(const sop_ctx *c)
{
    if (c->integrator != SOP_INTEGRATOR_UNDERDAMPED)
        return 0.0f;
    return (float)((c->ud_half ? 0.5 : 1.0) * c->p.h / c->mass);
}

float list_rc2(const sop_ctx *c) { return (float)(c->p.r_list * c->p.r_list); }

// The plain schedule's skin build radius r_list + skin (the batched schedule
// builds its list directly).
double skin_radius(const sop_ctx *c)
{
    return c->p.r_list + (c->schedule == SOP_SCHEDULE_PLAIN ? c->skin : 0.0);
}
float skin_rs2(const sop_ctx *c) { return (float)(skin_radius(c) * skin_radius(c)); }

// Largest displacement since the skin build that keeps the skin valid
// (squared; 0 = rebuild the skin at every rebuild): skin/2 less a margin
// far above the rounding of the single-precision distances.
float skin_check_thr2(const sop_ctx *c)
{
    const double thr = 0.5 * c->skin - 0.01;
    return (c->schedule == SOP_SCHEDULE_PLAIN && thr > 0.0) ? (float)(thr * thr) : 0.0f;
}

// Cell edge slightly above the skin radius so that any pair passing the
// single-precision predicate lies in adjacent cells despite rounding of the
// cell index.
float cell_edge(const sop_ctx *c) { return (float)(skin_radius(c) * 1.002 + 0.05); }

// Grid for the list rebuild.  Each trajectory's cells are shifted to its own
// block of a lattice of trajectory boxes so that independent trajectories
// that overlap in space do not share cells; the grid wraps, so positions
// outside the initial boxes still map to valid (shared) cells.
void set_grid(sop_ctx *c, const double *xyz)
{
    const double e = cell_edge(c);
    const int T = c->n_traj;
    std::vector<long long> lo(3 * (size_t)T), ext(3 * (size_t)T);
    long long span[3] = {1, 1, 1};
    for (int t = 0; t < T; ++t) {
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
        for (long long i = c->res_offsets[t]; i < c->res_offsets[t + 1]; ++i)
            for (int a = 0; a < 3; ++a) {
                mn[a] = std::min(mn[a], xyz[3 * i + a]);
                mx[a] = std::max(mx[a], xyz[3 * i + a]);
            }
        for (int a = 0; a < 3; ++a) {
            if (c->res_offsets[t + 1] == c->res_offsets[t]) {
                mn[a] = mx[a] = 0.0;
            }
            lo[3 * t + a] = (long long)std::floor(mn[a] / e);
            ext[3 * t + a] = (long long)std::floor(mx[a] / e) - lo[3 * t + a] + 1;
            span[a] = std::max(span[a], ext[3 * t + a] + 1);  // one empty cell between boxes
        }
    }
    // lattice of trajectory boxes, about as many along each axis
    long long A = 1;
    while (A * A * A < T)
        ++A;
    c->traj_cell.assign(T, int4{0, 0, 0, 0});
    long long g[3] = {3, 3, 3};
    for (int t = 0; t < T; ++t) {
        const long long ix = t % A, iy = (t / A) % A, iz = t / (A * A);
        const long long org[3] = {ix * span[0], iy * span[1], iz * span[2]};
        long long off[3];
        for (int a = 0; a < 3; ++a) {
            off[a] = org[a] - lo[3 * t + a];
            g[a] = std::max(g[a], org[a] + ext[3 * t + a] + 1);
        }
        c->traj_cell[t] = int4{(int)off[0], (int)off[1], (int)off[2], 0};
    }
    while (g[0] * g[1] * g[2] > c->n_cells_cap) {
        int m = 0;
        for (int a = 1; a < 3; ++a)
            if (g[a] > g[m])
                m = a;
        g[m] = std::max<long long>(3, (g[m] * 3) / 4);
        if (g[0] == 3 && g[1] == 3 && g[2] == 3)
            break;
    }
    c->grid.inv_cell = 1.0f / (float)e;
    c->grid.gx = (int)g[0];
    c->grid.gy = (int)g[1];
    c->grid.gz = (int)g[2];
    c->grid.n_cells = (int)(g[0] * g[1] * g[2]);
}

sop_status check_device_errors(sop_ctx *c)
{
    if (!c->bound)
        return SOP_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned bits = 0;
    HIP_TRY(c, hipMemcpy(&bits, c->b.err, sizeof(unsigned), hipMemcpyDeviceToHost));
    c->sticky |= bits;
    if (c->sticky)
        return fail(c, status_from_bits(c->sticky), bits_message(c->sticky));
    return SOP_OK;
}

sop_status need_ready(sop_ctx *c)
{
    if (!c)
        return SOP_E_ARG;
    if (!c->topo)
        return fail(c, SOP_E_STATE, "no topology loaded");
    if (!c->bound)
        return fail(c, SOP_E_STATE, "no workspace bound");
    if (!c->coords)
        return fail(c, SOP_E_STATE, "no coordinates set");
    return SOP_OK;
}

// Plain-schedule list rebuild at step c->step.  The skin is rebuilt first
// when there is no skin, or unless the displacement check of the step before
// left it valid (graph replays capture rebuilds that rely on that check:
// `captured`).
// `filter` false: the step kernel that follows filters the skin rows.
void rebuild(sop_ctx *c, hipStream_t s, bool advance, bool captured = false, bool filter = true)
{
    // in cadence: the step before was a period's last step, which binned its
    // positions and checked their displacements (a rebuild consumes the bins)
    const bool checked = captured || c->skin_checked == c->step;
    const bool binned = captured || c->binned_at == c->step;
    if (skin_check_thr2(c) <= 0.0f || !checked)
        launch_force_skin(c->b, s);
    launch_rebuild(c->b, c->cur, (int)c->n_res, c->cap, c->tile, c->grid, list_rc2(c), skin_rs2(c),
                   c->n_traj > 1 ? 1 : 0, s, advance, c->p.list_every, binned, filter);
    if (!captured)
        c->binned_at = -1;
}

// Whether step `step` is the last of a list period: its kernel checks the
// displacements against the skin.
bool checks_skin(const sop_ctx *c, long long step) { return (step + 1) % c->p.list_every == 0; }

// Whether the first step after a rebuild filters the skin rows itself: the
// particle-based step kernel does, unless that step is also the period's
// last (it would clear the cell counts it bins into).
bool fuses_filter(const sop_ctx *c, bool check) { return c->force_mode == SOP_FORCES_PARTICLE && !check; }

// `check`: the last step of a list period, which bins its new positions for
// the next skin search and checks their displacements.
// `first`: the first step after a rebuild launched without its filter,
// which filters the skin rows itself.
void one_step(sop_ctx *c, hipStream_t s, const long long *base, long long off, bool energy, bool check,
              bool first = false)
{
    launch_step(c->b, c->cur, (int)c->n_res, c->cap, c->tile, step_consts(c), c->tip,
                c->pulls.empty() ? 0 : 1, energy, 0, base, off, check ? skin_check_thr2(c) : 0.0f, s,
                c->force_mode, ud_kick(c), check ? &c->grid : nullptr, first ? list_rc2(c) : 0.0f,
                c->grid.n_cells);
    if (energy)
        launch_reduce_energy(c->b, c->n_traj, s);
}

// mode 1: one force evaluation; otherwise n_steps steps, recording energies
// only when `records` (a launch whose steps hold a multiple of the energy
// interval).
void batch_launch(sop_ctx *c, hipStream_t s, int n_steps, int stale, int mode, const long long *base,
                  long long off, bool records = false)
{
    launch_batch(c->b, c->cur, n_packs(c), c->batch_wg, c->cap, step_consts(c), c->tip,
                 c->pulls.empty() ? 0 : 1, list_rc2(c), c->p.list_every, c->energy_every, n_steps,
                 stale, mode == 1 ? 1 : (records ? 2 : 0), base, off, s,
                 c->re_rep > 0 ? c->b.re_tscale : nullptr);
}

// Last step in [first, first + n) whose energies are recorded, or -1.
long long last_record(const sop_ctx *c, long long first, long long n)
{
    const long long E = c->energy_every;
    if (E <= 0 || n <= 0)
        return -1;
    const long long last = first + n - 1;
    const long long r = last - last % E;
    return r >= first ? r : -1;
}

// Batched schedule: a graph of one persistent launch of batch_steps steps plus
// the device step-counter advance, for layer parity `par`, with or without
// energy records.
sop_status capture_batch_graph(sop_ctx *c, int par, int records)
{
    if (!c->cap_stream)
        HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const int saved = c->cur;
    c->cur = par;
    hipGraph_t g = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    batch_launch(c, c->cap_stream, c->batch_steps, 0, 0, c->b.step_base, 0, records != 0);
    launch_add_step(c->b.step_base, c->batch_steps, c->cap_stream);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->cur = saved;
    if (e != hipSuccess)
        return hip_fail(c, e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return hip_fail(c, e, "hipGraphInstantiate");
    c->bgraphs[par][records] = ex;
    return SOP_OK;
}

// Capture `periods` list periods (rebuild + list_every steps each) starting at
// layer parity `par`; energies are recorded at the first step when `energy`.
sop_status capture_graph(sop_ctx *c, int par, int energy)
{
    if (!c->cap_stream)
        HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const int saved = c->cur;
    c->cur = par;
    hipGraph_t g = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    const bool half_saved = c->ud_half;
    c->ud_half = false;  // graphs start only after the first (half-kick) step
    for (int q = 0; q < c->graph_steps; ++q) {
        const bool fuse = fuses_filter(c, c->p.list_every == 1);
        rebuild(c, c->cap_stream, true, true, !fuse);
        for (int k = 0; k < c->p.list_every; ++k) {
            one_step(c, c->cap_stream, c->b.step_base, k, energy && q == 0 && k == 0,
                     k == c->p.list_every - 1, fuse && k == 0);
            c->cur ^= 1;
        }
    }
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->cur = saved;
    c->ud_half = half_saved;
    if (e != hipSuccess)
        return hip_fail(c, e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return hip_fail(c, e, "hipGraphInstantiate");
    c->graphs[par][energy] = ex;
    return SOP_OK;
}

bool valid_pair(const sop_ctx *c, long long i, long long j)
{
    if (i < 0 || j < 0 || i >= c->n_res || j >= c->n_res || i == j)
        return false;
    return c->traj_of[i] == c->traj_of[j];
}

}  // namespace

extern "C" {

const char *sop_status_string(sop_status s)
{
    switch (s) {
    case SOP_OK: return "ok";
    case SOP_E_ARG: return "invalid argument";
    case SOP_E_STATE: return "call out of order";
    case SOP_E_WORKSPACE: return "workspace missing or too small";
    case SOP_E_HIP: return "HIP runtime error";
    case SOP_E_FENE: return "FENE bond broken";
    case SOP_E_LIST_OVERFLOW: return "pair list overflow";
    case SOP_E_NONFINITE: return "non-finite force or position";
    case SOP_E_TIP: return "residue reached the tip surface";
    }
    return "unknown status";
}

const char *sop_last_error(const sop_ctx *c) { return c ? c->last_error.c_str() : "null context"; }

sop_status sop_create(const sop_params *params, void *hip_stream, sop_ctx **out)
{
    if (!params || !out)
        return SOP_E_ARG;
    const sop_params &p = *params;
    const bool ok = p.k_fene > 0 && p.R0 > 0 && p.eps_h >= 0 && p.eps_l >= 0 && p.sigma > 0 &&
                    p.r_list > 0 && p.kBT >= 0 && p.zeta > 0 && p.h > 0 && p.list_every > 0 &&
                    p.list_capacity >= 0 && p.list_capacity <= 1024 && std::isfinite(p.r_list) && std::isfinite(p.h);
    if (!ok)
        return SOP_E_ARG;
    sop_ctx *c = new (std::nothrow) sop_ctx();
    if (!c)
        return SOP_E_ARG;
    c->p = p;
    c->stream = (hipStream_t)hip_stream;
    c->cap_req = p.list_capacity;
    c->cap = list_cap(c);
    *out = c;
    return SOP_OK;
}

sop_status sop_destroy(sop_ctx *c)
{
    if (!c)
        return SOP_E_ARG;
    destroy_graphs(c);
    if (c->cap_stream)
        (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return SOP_OK;
}

sop_status sop_load_topology(sop_ctx *c, int32_t n_traj, const int64_t *res_offsets,
                             const uint32_t *stream_ids, int64_t n_bonds, const int32_t *bonds,
                             const double *bond_r0, int64_t n_native, const int32_t *natives,
                             const double *native_r0, const uint8_t *fixed)
{
    if (!c)
        return SOP_E_ARG;
    if (n_traj <= 0 || !res_offsets || n_bonds < 0 || n_native < 0 ||
        (n_bonds > 0 && (!bonds || !bond_r0)) || (n_native > 0 && (!natives || !native_r0)))
        return fail(c, SOP_E_ARG, "bad topology arguments");
    if (res_offsets[0] != 0)
        return fail(c, SOP_E_ARG, "res_offsets[0] must be 0");
    for (int t = 0; t < n_traj; ++t)
        if (res_offsets[t + 1] < res_offsets[t])
            return fail(c, SOP_E_ARG, "res_offsets must be non-decreasing");
    const long long n = res_offsets[n_traj];
    if (n <= 0 || n >= (1LL << 31) - 64)
        return fail(c, SOP_E_ARG, "residue count out of range");

    c->topo = false;
    c->bound = false;
    c->coords = false;
    destroy_graphs(c);
    c->n_traj = n_traj;
    c->n_res = n;
    c->res_offsets.assign(res_offsets, res_offsets + n_traj + 1);
    c->stream_ids.resize(n_traj);
    for (int t = 0; t < n_traj; ++t)
        c->stream_ids[t] = stream_ids ? stream_ids[t] : (unsigned)t;
    c->traj_of.assign(n, 0);
    c->traj_lo.assign(n, 0);
    c->traj_hi.assign(n, 0);
    c->local.assign(n, 0);
    for (int t = 0; t < n_traj; ++t)
        for (long long i = res_offsets[t]; i < res_offsets[t + 1]; ++i) {
            c->traj_of[i] = t;
            c->traj_lo[i] = (int)res_offsets[t];
            c->traj_hi[i] = (int)res_offsets[t + 1];
            c->local[i] = (int)(i - res_offsets[t]);
        }
    c->fixed.assign(n, 0);
    if (fixed)
        for (long long i = 0; i < n; ++i)
            c->fixed[i] = fixed[i] ? 1 : 0;

    // validate pairs: range, same trajectory, no self/duplicate, r0 > 0
    std::vector<std::pair<long long, int>> keys;  // (i*n + j, kind)
    keys.reserve((size_t)(n_bonds + n_native));
    for (int kind = 0; kind < 2; ++kind) {
        const long long m = kind ? n_native : n_bonds;
        const int32_t *pr = kind ? natives : bonds;
        const double *r0 = kind ? native_r0 : bond_r0;
        for (long long k = 0; k < m; ++k) {
            long long i = pr[2 * k], j = pr[2 * k + 1];
            if (!valid_pair(c, i, j))
                return fail(c, SOP_E_ARG, (kind ? "native " : "bond ") + std::to_string(k) +
                                              ": index out of range, self pair, or pair across trajectories");
            if (!(r0[k] > 0.0) || !std::isfinite(r0[k]))
                return fail(c, SOP_E_ARG, (kind ? "native " : "bond ") + std::to_string(k) + ": r0 <= 0");
            if (i > j)
                std::swap(i, j);
            keys.push_back({i * n + j, kind});
        }
    }
    std::sort(keys.begin(), keys.end());
    for (size_t k = 1; k < keys.size(); ++k)
        if (keys[k].first == keys[k - 1].first)
            return fail(c, SOP_E_ARG, keys[k].second != keys[k - 1].second
                                          ? "a pair is both bonded and native"
                                          : "duplicate pair");

    // per-residue rows: bonds then natives, partners ascending
    std::vector<std::vector<std::pair<int, float>>> rb(n), rn(n);
    for (long long k = 0; k < n_bonds; ++k) {
        int i = bonds[2 * k], j = bonds[2 * k + 1];
        rb[i].push_back({j, (float)bond_r0[k]});
        rb[j].push_back({i, (float)bond_r0[k]});
    }
    for (long long k = 0; k < n_native; ++k) {
        int i = natives[2 * k], j = natives[2 * k + 1];
        rn[i].push_back({j, (float)native_r0[k]});
        rn[j].push_back({i, (float)native_r0[k]});
    }
    c->trow.assign(n, int2{0, 0});
    c->tent.clear();
    c->tent.reserve((size_t)(2 * (n_bonds + n_native)));
    for (long long i = 0; i < n; ++i) {
        std::sort(rb[i].begin(), rb[i].end());
        std::sort(rn[i].begin(), rn[i].end());
        if (rb[i].size() + rn[i].size() > (size_t)TOPO_CAP)
            return fail(c, SOP_E_ARG, "more than " + std::to_string(TOPO_CAP) +
                                          " bonded and native partners on residue " + std::to_string(i));
        c->trow[i] = int2{(int)c->tent.size(), (int)(rb[i].size() | (rn[i].size() << 12))};
        for (auto &e : rb[i]) {
            int bits = e.first;
            float f;
            std::memcpy(&f, &bits, 4);
            c->tent.push_back(float2{f, e.second});
        }
        for (auto &e : rn[i]) {
            int bits = e.first;
            float f;
            std::memcpy(&f, &bits, 4);
            c->tent.push_back(float2{f, e.second});
        }
    }
    // plain-schedule tiles: consecutive residues, a new tile at a chain start
    // (first residue of a trajectory or not bonded to its predecessor) once
    // the current one is half full, so that tiles stay compact in space
    std::vector<char> chain_start(n, 0);
    for (long long i = 0; i < n; ++i) {
        bool bonded = false;
        for (auto &e : rb[i])
            bonded |= e.first == i - 1;
        chain_start[i] = (i == c->traj_lo[i] || !bonded) ? 1 : 0;
    }
    for (int k = 0; k < 3; ++k) {
        const int T = 64 << k;
        auto &tl = c->tiles[k];
        tl.clear();
        int cnt = 0;
        for (long long i = 0; i < n; ++i) {
            if (cnt == 0 || cnt == T || (chain_start[i] && 2 * cnt >= T)) {
                tl.push_back((int)i);
                cnt = 0;
            }
            ++cnt;
        }
        tl.push_back((int)n);
    }
    // energy-reduction chunks: ECHUNK residues, never across trajectories
    c->chunk_lo.clear();
    c->chunk_first.clear();
    for (int t = 0; t < n_traj; ++t) {
        c->chunk_first.push_back((int)c->chunk_lo.size());
        const long long a0 = res_offsets[t], b0 = res_offsets[t + 1];
        for (long long r = a0; r < b0 || r == a0; r += ECHUNK) {
            c->chunk_lo.push_back((int)r);
            if (b0 == a0)
                break;
        }
    }
    c->chunk_first.push_back((int)c->chunk_lo.size());
    c->chunk_lo.push_back((int)n);
    c->pulls.clear();
    c->pull_slot.assign(n, -1);
    c->tip = TipDev{};
    c->tile = c->tile_req ? c->tile_req : default_tile(n);
    c->max_len = 0;
    for (int t = 0; t < n_traj; ++t)
        c->max_len = std::max<long long>(c->max_len, res_offsets[t + 1] - res_offsets[t]);
    c->n_cells_cap = (int)std::min<long long>(std::max<long long>(n / 2, 4096), 1LL << 21);
    c->topo = true;
    return SOP_OK;
}

sop_status sop_set_pulling(sop_ctx *c, int32_t traj, int64_t residue, double kappa,
                           const double anchor0[3], const double v[3])
{
    if (!c)
        return SOP_E_ARG;
    if (!c->topo)
        return fail(c, SOP_E_STATE, "load a topology first");
    if (c->bound)
        return fail(c, SOP_E_STATE, "set protocols before binding the workspace");
    if (traj < 0 || traj >= c->n_traj || residue < c->res_offsets[traj] ||
        residue >= c->res_offsets[traj + 1] || !anchor0 || !v || !(kappa >= 0))
        return fail(c, SOP_E_ARG, "bad cantilever arguments");
    if (c->pull_slot[residue] >= 0)
        return fail(c, SOP_E_ARG, "residue already has a cantilever");
    PullDev pd{};
    double vv = 0;
    for (int a = 0; a < 3; ++a) {
        pd.anchor0[a] = anchor0[a];
        pd.v[a] = v[a];
        vv += v[a] * v[a];
    }
    pd.has_dir = vv > 0 ? 1 : 0;
    for (int a = 0; a < 3; ++a)
        pd.vhat[a] = vv > 0 ? v[a] / std::sqrt(vv) : 0.0;
    pd.kappa = kappa;
    pd.residue = (int)residue;
    c->pull_slot[residue] = (int)c->pulls.size();
    c->pulls.push_back(pd);
    return SOP_OK;
}

sop_status sop_set_tip(sop_ctx *c, double radius, double eps, double sigma, const double c0[3],
                       const double v[3])
{
    if (!c)
        return SOP_E_ARG;
    if (!c->topo)
        return fail(c, SOP_E_STATE, "load a topology first");
    if (c->bound)
        return fail(c, SOP_E_STATE, "set protocols before binding the workspace");
    if (radius < 0) {
        c->tip = TipDev{};
        return SOP_OK;
    }
    if (!c0 || !v || !(sigma > 0) || !(eps >= 0))
        return fail(c, SOP_E_ARG, "bad tip arguments");
    TipDev t{};
    double vv = 0;
    for (int a = 0; a < 3; ++a) {
        t.c0[a] = c0[a];
        t.v[a] = v[a];
        vv += v[a] * v[a];
    }
    t.has_dir = vv > 0 ? 1 : 0;
    for (int a = 0; a < 3; ++a)
        t.vhat[a] = vv > 0 ? v[a] / std::sqrt(vv) : 0.0;
    t.radius = radius;
    t.eps = eps;
    t.sigma = sigma;
    t.on = 1;
    c->tip = t;
    return SOP_OK;
}

sop_status sop_set_tile(sop_ctx *c, int32_t tile)
{
    if (!c)
        return SOP_E_ARG;
    if (!(tile == 0 || tile == 64 || tile == 128 || tile == 256))
        return fail(c, SOP_E_ARG, "tile must be 0, 64, 128 or 256 residues");
    c->tile_req = tile;
    if (c->topo) {
        const int nt = tile ? tile : default_tile(c->n_res);
        if (nt != c->tile) {
            c->tile = nt;
            c->list_valid = false;  // the list layout follows the tile size
            c->skin_checked = c->binned_at = -1;
            destroy_graphs(c);
        }
    }
    return SOP_OK;
}

sop_status sop_get_tile(const sop_ctx *c, int32_t *tile)
{
    if (!c || !tile)
        return SOP_E_ARG;
    if (!c->topo)
        return SOP_E_STATE;
    *tile = c->tile;
    return SOP_OK;
}

sop_status sop_set_schedule(sop_ctx *c, int32_t schedule)
{
    if (!c)
        return SOP_E_ARG;
    if (schedule != SOP_SCHEDULE_PLAIN && schedule != SOP_SCHEDULE_BATCHED)
        return fail(c, SOP_E_ARG, "unknown schedule");
    if (c->bound)
        return fail(c, SOP_E_STATE, "set the schedule before binding the workspace");
    c->schedule = schedule;
    c->cap = list_cap(c);
    return SOP_OK;
}

sop_status sop_set_batch(sop_ctx *c, int32_t wg, int32_t steps)
{
    if (!c)
        return SOP_E_ARG;
    if (!(wg == 0 || wg == 256 || wg == 512 || wg == 1024) || steps < 1)
        return fail(c, SOP_E_ARG, "workgroup residues must be 0, 256, 512 or 1024 and steps >= 1");
    if (c->topo && wg && wg < c->max_len)
        return fail(c, SOP_E_ARG, "workgroup smaller than the longest trajectory");
    c->batch_wg_req = wg;
    c->batch_steps = steps;
    for (auto &gp : c->bgraphs)
        for (auto &g : gp)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    if (c->bound && c->schedule == SOP_SCHEDULE_BATCHED) {
        c->batch_wg = pick_batch_wg(c);
        make_packs(c);
        const sop_status st = upload_packs(c);
        if (st != SOP_OK)
            return st;
        c->list_valid = false;  // the list layout follows the packs
    }
    return SOP_OK;
}

sop_status sop_get_batch(const sop_ctx *c, int32_t *wg, int32_t *steps, int32_t *np)
{
    if (!c)
        return SOP_E_ARG;
    if (wg)
        *wg = c->bound ? c->batch_wg : pick_batch_wg(c);
    if (steps)
        *steps = c->batch_steps;
    if (np)
        *np = c->bound ? n_packs(c) : 0;
    return SOP_OK;
}

sop_status sop_set_force_mode(sop_ctx *c, int32_t mode)
{
    if (!c || (mode != SOP_FORCES_PARTICLE && mode != SOP_FORCES_PAIR))
        return SOP_E_ARG;
    if (mode != c->force_mode) {
        c->force_mode = mode;
        destroy_graphs(c);  // the graphs hold the kernels of the old mode
    }
    return SOP_OK;
}

sop_status sop_get_force_mode(const sop_ctx *c, int32_t *mode)
{
    if (!c || !mode)
        return SOP_E_ARG;
    *mode = c->force_mode;
    return SOP_OK;
}

sop_status sop_set_integrator(sop_ctx *c, int32_t kind, double mass)
{
    if (!c || (kind != SOP_INTEGRATOR_OVERDAMPED && kind != SOP_INTEGRATOR_UNDERDAMPED))
        return SOP_E_ARG;
    if (kind == SOP_INTEGRATOR_UNDERDAMPED && !(mass > 0.0 && std::isfinite(mass)))
        return fail(c, SOP_E_ARG, "the mass must be positive and finite");
    if (kind == SOP_INTEGRATOR_UNDERDAMPED && c->schedule != SOP_SCHEDULE_PLAIN)
        return fail(c, SOP_E_STATE, "the underdamped integrator runs on the plain schedule");
    c->integrator = kind;
    if (kind == SOP_INTEGRATOR_UNDERDAMPED)
        c->mass = mass;
    c->ud_half = true;
    destroy_graphs(c);  // the integrator's constants are kernel arguments
    return SOP_OK;
}

sop_status sop_set_velocities(sop_ctx *c, const double *v)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (!v)
        return fail(c, SOP_E_ARG, "null velocities");
    if (c->schedule != SOP_SCHEDULE_PLAIN)
        return fail(c, SOP_E_STATE, "velocities belong to the plain schedule");
    const long long n = c->n_res;
    std::vector<float4> vv(n);
    for (long long i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(v[3 * i + a]))
                return fail(c, SOP_E_ARG, "non-finite velocity");
        vv[i] = c->fixed[i] ? float4{0.f, 0.f, 0.f, 0.f}
                            : float4{(float)v[3 * i], (float)v[3 * i + 1], (float)v[3 * i + 2], 0.f};
    }
    HIP_TRY(c, hipMemcpyAsync(c->b.vel, vv.data(), n * sizeof(float4), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->ud_half = true;
    return SOP_OK;
}

sop_status sop_get_velocities(sop_ctx *c, double *v)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (!v)
        return fail(c, SOP_E_ARG, "null output");
    if (c->schedule != SOP_SCHEDULE_PLAIN)
        return fail(c, SOP_E_STATE, "velocities belong to the plain schedule");
    const long long n = c->n_res;
    std::vector<float4> fo(n, float4{0.f, 0.f, 0.f, 0.f}), vv(n);
    const bool add_kick = c->integrator == SOP_INTEGRATOR_UNDERDAMPED && !c->ud_half;
    if (add_kick) {
        // the stored velocities lack the last half kick, whose force is this step's
        if (!c->list_valid || c->step % c->p.list_every == 0)
            rebuild(c, c->stream, false);
        c->list_valid = true;
        launch_step(c->b, c->cur, (int)c->n_res, c->cap, c->tile, step_consts(c), c->tip,
                    c->pulls.empty() ? 0 : 1, false, 1, nullptr, c->step, 0.0f, c->stream, c->force_mode);
        HIP_TRY(c, hipGetLastError());
        st = check_device_errors(c);
        if (st != SOP_OK)
            return st;
        HIP_TRY(c, hipMemcpy(fo.data(), c->b.fout, n * sizeof(float4), hipMemcpyDeviceToHost));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(vv.data(), c->b.vel, n * sizeof(float4), hipMemcpyDeviceToHost));
    const double hk = 0.5 * c->p.h / c->mass;
    for (long long i = 0; i < n; ++i) {
        const bool fx = c->fixed[i] != 0;
        v[3 * i] = fx ? 0.0 : (double)vv[i].x + (add_kick ? hk * (double)fo[i].x : 0.0);
        v[3 * i + 1] = fx ? 0.0 : (double)vv[i].y + (add_kick ? hk * (double)fo[i].y : 0.0);
        v[3 * i + 2] = fx ? 0.0 : (double)vv[i].z + (add_kick ? hk * (double)fo[i].z : 0.0);
    }
    return check_device_errors(c);
}

sop_status sop_set_tempering(sop_ctx *c, int32_t n_rep, const double *kbt, int64_t exchange_every,
                             const int32_t *tidx)
{
    if (!c)
        return SOP_E_ARG;
    if (c->schedule != SOP_SCHEDULE_BATCHED || !c->bound)
        return fail(c, SOP_E_STATE, "replica exchange runs on a bound batched schedule");
    if (n_rep < 1 || !kbt || exchange_every < 0 || c->n_traj % n_rep != 0)
        return fail(c, SOP_E_ARG, "n_rep must divide the trajectory count; exchange_every >= 0");
    for (int k = 0; k < n_rep; ++k)
        if (!(kbt[k] > 0.0) || !std::isfinite(kbt[k]))
            return fail(c, SOP_E_ARG, "temperatures must be positive");
    const int T = c->n_traj;
    std::vector<int> ti(T);
    std::vector<float> ts(T);
    for (int t = 0; t < T; ++t)
        ti[t] = tidx ? tidx[t] : t % n_rep;
    for (int g = 0; g < T / n_rep; ++g) {  // each group a permutation of 0..n_rep-1
        std::vector<char> seen(n_rep, 0);
        for (int m = 0; m < n_rep; ++m) {
            const int v = ti[g * n_rep + m];
            if (v < 0 || v >= n_rep || seen[v])
                return fail(c, SOP_E_ARG, "temperature indices are not a permutation in each group");
            seen[v] = 1;
        }
    }
    for (int t = 0; t < T; ++t)
        ts[t] = (float)std::sqrt(kbt[ti[t]] / c->p.kBT);
    c->re_rep = n_rep;
    c->re_kbt.assign(kbt, kbt + n_rep);
    c->re_every = exchange_every;
    c->re_last = -1;
    hipStream_t s = c->stream;
    HIP_TRY(c, hipMemcpyAsync(c->b.re_kbt, kbt, n_rep * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->b.re_tidx, ti.data(), T * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->b.re_tscale, ts.data(), T * sizeof(float), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemsetAsync(c->b.re_stats, 0, 2 * (size_t)T * sizeof(unsigned long long), s));
    HIP_TRY(c, hipStreamSynchronize(s));
    destroy_graphs(c);
    return SOP_OK;
}

sop_status sop_get_tempering(sop_ctx *c, int32_t *tidx, int64_t *accepted, int64_t *attempted)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (c->re_rep < 1)
        return fail(c, SOP_E_STATE, "no replica exchange set");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int T = c->n_traj, R = c->re_rep;
    if (tidx)
        HIP_TRY(c, hipMemcpy(tidx, c->b.re_tidx, T * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<unsigned long long> stv(2 * (size_t)T);
    HIP_TRY(c, hipMemcpy(stv.data(), c->b.re_stats, stv.size() * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost));
    for (int k = 0; k + 1 < R; ++k) {
        if (accepted)
            accepted[k] = (int64_t)stv[2 * k];
        if (attempted)
            attempted[k] = (int64_t)stv[2 * k + 1];
    }
    return check_device_errors(c);
}

sop_status sop_set_list_skin(sop_ctx *c, double skin)
{
    if (!c || !(skin >= 0.0) || !std::isfinite(skin) || skin > 4.0 * c->p.r_list)
        return SOP_E_ARG;
    if (skin == c->skin)
        return SOP_OK;
    c->skin = skin;
    c->list_valid = false;
    c->skin_checked = c->binned_at = -1;
    destroy_graphs(c);  // the radius, the cell grid and the check are kernel arguments
    if (c->coords)
        set_grid(c, c->xyz_set.data());  // the cell edge follows the skin radius
    if (c->bound && c->coords)
        HIP_TRY(c, hipMemcpyAsync(c->b.traj_cell, c->traj_cell.data(), c->n_traj * sizeof(int4),
                                  hipMemcpyHostToDevice, c->stream));
    return SOP_OK;
}

sop_status sop_get_list_skin(const sop_ctx *c, double *skin)
{
    if (!c || !skin)
        return SOP_E_ARG;
    *skin = c->skin;
    return SOP_OK;
}

sop_status sop_get_list_stats(sop_ctx *c, int64_t *rebuilds, int64_t *skin_builds)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    unsigned long long v[2] = {0, 0};
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(v, c->b.list_stats, sizeof(v), hipMemcpyDeviceToHost));
    if (rebuilds)
        *rebuilds = (int64_t)v[0];
    if (skin_builds)
        *skin_builds = (int64_t)v[1];
    return SOP_OK;
}

sop_status sop_set_graph_steps(sop_ctx *c, int32_t k)
{
    if (!c || k < 0)
        return SOP_E_ARG;
    if (k != c->graph_steps)
        destroy_graphs(c);  // captured graphs hold the old span
    c->graph_steps = k;
    return SOP_OK;
}

sop_status sop_set_energy_interval(sop_ctx *c, int64_t k)
{
    if (!c || k < 0)
        return SOP_E_ARG;
    if (k != c->energy_every)
        destroy_graphs(c);  // batched graphs hold the interval as a kernel argument
    c->energy_every = k;
    return SOP_OK;
}

sop_status sop_workspace_size(const sop_ctx *c, size_t *bytes)
{
    if (!c || !bytes)
        return SOP_E_ARG;
    if (!c->topo)
        return SOP_E_STATE;
    *bytes = layout(c, nullptr, nullptr);
    return SOP_OK;
}

sop_status sop_bind_workspace(sop_ctx *c, void *dev, size_t bytes)
{
    if (!c)
        return SOP_E_ARG;
    if (!c->topo)
        return fail(c, SOP_E_STATE, "load a topology first");
    const size_t need = layout(c, nullptr, nullptr);
    if (!dev || ((uintptr_t)dev & 255) || bytes < need)
        return fail(c, SOP_E_WORKSPACE, "workspace null, not 256-byte aligned, or smaller than " +
                                            std::to_string(need) + " bytes");
    if (c->schedule == SOP_SCHEDULE_BATCHED && c->max_len > 1024)
        return fail(c, SOP_E_ARG, "the batched schedule holds trajectories of at most 1024 residues");
    destroy_graphs(c);
    c->bound = false;
    c->coords = false;
    c->list_valid = false;
    c->ws = dev;
    c->ws_bytes = bytes;
    layout(c, (char *)dev, &c->b);
    if (c->schedule == SOP_SCHEDULE_BATCHED) {
        c->batch_wg = pick_batch_wg(c);
        if (c->batch_wg < c->max_len)
            return fail(c, SOP_E_ARG, "batch workgroup smaller than the longest trajectory");
        make_packs(c);
        const sop_status st = upload_packs(c);
        if (st != SOP_OK)
            return st;
    }
    const DevBufs &b = c->b;
    const size_t n = (size_t)c->n_res;
    hipStream_t s = c->stream;
    HIP_TRY(c, hipMemcpyAsync(b.trow, c->trow.data(), n * sizeof(int2), hipMemcpyHostToDevice, s));
    if (!c->tent.empty())
        HIP_TRY(c, hipMemcpyAsync(b.tent, c->tent.data(), c->tent.size() * sizeof(float2),
                                  hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(b.traj_lo, c->traj_lo.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(b.traj_hi, c->traj_hi.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(b.pull_slot, c->pull_slot.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    if (!c->pulls.empty())
        HIP_TRY(c, hipMemcpyAsync(b.pulls, c->pulls.data(), c->pulls.size() * sizeof(PullDev),
                                  hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(b.stream_ids, c->stream_ids.data(), c->n_traj * sizeof(unsigned),
                              hipMemcpyHostToDevice, s));
    {
        std::vector<uint2> key(n);
        for (size_t i = 0; i < n; ++i) {
            key[i].x = (unsigned)c->local[i] | (c->fixed[i] ? 0x80000000u : 0u);
            key[i].y = c->stream_ids[c->traj_of[i]];
        }
        HIP_TRY(c, hipMemcpy(b.noise_key, key.data(), n * sizeof(uint2), hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpyAsync(b.res_offsets, c->res_offsets.data(), (c->n_traj + 1) * sizeof(long long),
                              hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemsetAsync(b.list_cnt, 0, n * sizeof(int), s));
    if (c->schedule == SOP_SCHEDULE_PLAIN) {
        // slot arrays start as slot 0, which every tile's staging holds
        const size_t n_pad = ((n + 255) / 256) * 256;
        size_t topo2_elems = 0, n_tiles_max = 0;
        for (int k = 0; k < 3; ++k) {
            const size_t nt = c->tiles[k].size() - 1;
            topo2_elems = std::max(topo2_elems, nt * ((size_t)64 << k) * TOPO_CAP);
            n_tiles_max = std::max(n_tiles_max, nt);
            HIP_TRY(c, hipMemcpyAsync(b.tile_first[k], c->tiles[k].data(), c->tiles[k].size() * sizeof(int),
                                      hipMemcpyHostToDevice, s));
        }
        HIP_TRY(c, hipMemsetAsync(b.list16, 0, n_pad * c->cap * sizeof(unsigned short), s));
        HIP_TRY(c, hipMemsetAsync(b.flist16, 0, n_pad * c->cap * sizeof(unsigned short), s));
        HIP_TRY(c, hipMemsetAsync(b.fcnt, 0, n * sizeof(int), s));
        HIP_TRY(c, hipMemsetAsync(b.cell_count, 0, (size_t)c->n_cells_cap * sizeof(int), s));
        HIP_TRY(c, hipMemsetAsync(b.facc, 0, n * sizeof(float4), s));
        HIP_TRY(c, hipMemsetAsync(b.vel, 0, n * sizeof(float4), s));
        HIP_TRY(c, hipMemsetAsync(b.tile_ord, 0, n_tiles_max * 256, s));
        HIP_TRY(c, hipMemsetAsync(b.skin_ord, 0, n_tiles_max * 256 * sizeof(unsigned short), s));
        HIP_TRY(c, hipMemsetAsync(b.eacc, 0, n * sizeof(double4), s));
        HIP_TRY(c, hipMemsetAsync(b.topo2, 0, topo2_elems * sizeof(uint2), s));
        HIP_TRY(c, hipMemsetAsync(b.stage_cnt, 0, n_tiles_max * sizeof(int), s));
    }
    HIP_TRY(c, hipMemsetAsync(b.res_energy, 0, n * RES_E * sizeof(double), s));
    HIP_TRY(c, hipMemcpyAsync(b.chunk_lo, c->chunk_lo.data(), c->chunk_lo.size() * sizeof(int),
                              hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(b.chunk_first, c->chunk_first.data(), c->chunk_first.size() * sizeof(int),
                              hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemsetAsync(b.energy, 0, (size_t)c->n_traj * SOP_NTERMS * sizeof(double), s));
    HIP_TRY(c, hipMemsetAsync(b.f_ext, 0, (size_t)c->n_traj * sizeof(double), s));
    HIP_TRY(c, hipMemsetAsync(b.err, 0, sizeof(unsigned), s));
    HIP_TRY(c, hipMemsetAsync(b.skin_flag, 0, sizeof(unsigned), s));
    HIP_TRY(c, hipMemsetAsync(b.list_stats, 0, 2 * sizeof(unsigned long long), s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->skin_checked = c->binned_at = -1;
    c->bound = true;
    c->sticky = 0;
    c->energy_step = -1;
    return SOP_OK;
}

sop_status sop_set_coordinates(sop_ctx *c, const double *xyz)
{
    if (!c || !xyz)
        return SOP_E_ARG;
    if (!c->topo || !c->bound)
        return fail(c, SOP_E_STATE, "load a topology and bind a workspace first");
    const long long n = c->n_res;
    for (long long k = 0; k < 3 * n; ++k)
        if (!std::isfinite(xyz[k]))
            return fail(c, SOP_E_ARG, "non-finite coordinate");
    std::vector<float4> pv(2 * n);
    for (long long i = 0; i < n; ++i) {
        float h[3], l[3];
        for (int a = 0; a < 3; ++a) {
            h[a] = (float)xyz[3 * i + a];
            l[a] = (float)(xyz[3 * i + a] - (double)h[a]);
        }
        unsigned tag = (unsigned)c->local[i] | (c->fixed[i] ? 0x80000000u : 0u);
        float tw, lw;
        int tr = c->traj_of[i];
        std::memcpy(&tw, &tag, 4);
        std::memcpy(&lw, &tr, 4);
        pv[2 * i] = float4{h[0], h[1], h[2], tw};
        pv[2 * i + 1] = float4{l[0], l[1], l[2], lw};
    }
    c->xyz_set.assign(xyz, xyz + 3 * n);
    set_grid(c, xyz);
    destroy_graphs(c);  // the grid is a kernel argument of captured rebuilds
    hipStream_t s = c->stream;
    for (int k = 0; k < 2; ++k)
        HIP_TRY(c, hipMemcpyAsync(c->b.pos[k], pv.data(), 2 * n * sizeof(float4), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->b.traj_cell, c->traj_cell.data(), c->n_traj * sizeof(int4),
                              hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemsetAsync(c->b.err, 0, sizeof(unsigned), s));
    if (c->schedule == SOP_SCHEDULE_PLAIN)
        HIP_TRY(c, hipMemsetAsync(c->b.vel, 0, n * sizeof(float4), s));  // new coordinates, zero velocities
    HIP_TRY(c, hipStreamSynchronize(s));
    c->ud_half = true;
    c->cur = 0;
    c->sticky = 0;
    c->coords = true;
    c->list_valid = false;
    c->skin_checked = c->binned_at = -1;
    c->last_error.clear();
    return SOP_OK;
}

sop_status sop_get_coordinates(sop_ctx *c, double *xyz)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (!xyz)
        return fail(c, SOP_E_ARG, "null output");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const long long n = c->n_res;
    std::vector<float4> pv(2 * n);
    HIP_TRY(c, hipMemcpy(pv.data(), c->b.pos[c->cur], 2 * n * sizeof(float4), hipMemcpyDeviceToHost));
    for (long long i = 0; i < n; ++i) {
        xyz[3 * i + 0] = (double)pv[2 * i].x + (double)pv[2 * i + 1].x;
        xyz[3 * i + 1] = (double)pv[2 * i].y + (double)pv[2 * i + 1].y;
        xyz[3 * i + 2] = (double)pv[2 * i].z + (double)pv[2 * i + 1].z;
    }
    return check_device_errors(c);
}

sop_status sop_set_step(sop_ctx *c, int64_t step)
{
    if (!c || step < 0)
        return SOP_E_ARG;
    c->step = step;
    c->list_valid = false;
    c->skin_checked = c->binned_at = -1;
    return SOP_OK;
}

sop_status sop_get_step(const sop_ctx *c, int64_t *step)
{
    if (!c || !step)
        return SOP_E_ARG;
    *step = c->step;
    return SOP_OK;
}

sop_status sop_build_pairlist(sop_ctx *c)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (c->schedule == SOP_SCHEDULE_BATCHED)
        batch_launch(c, c->stream, 1, 1, 1, nullptr, c->step);  // rebuild + one force evaluation
    else
        rebuild(c, c->stream, false);
    HIP_TRY(c, hipGetLastError());
    c->list_valid = true;
    return SOP_OK;
}

sop_status sop_get_pairlist(sop_ctx *c, int64_t cap, int32_t *ij, int64_t *n_pairs)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (!n_pairs || cap < 0 || (cap > 0 && !ij))
        return fail(c, SOP_E_ARG, "bad pairlist arguments");
    if (!c->list_valid)
        return fail(c, SOP_E_STATE, "no list built since the coordinates were set");
    st = check_device_errors(c);
    if (st != SOP_OK)
        return st;
    const long long n = c->n_res;
    std::vector<int> cnt(n);
    HIP_TRY(c, hipMemcpy(cnt.data(), c->b.list_cnt, n * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<std::pair<int, int>> pairs;
    if (c->schedule == SOP_SCHEDULE_BATCHED) {
        std::vector<unsigned short> list((size_t)n * c->cap);
        HIP_TRY(c, hipMemcpy(list.data(), c->b.list16, list.size() * sizeof(unsigned short),
                             hipMemcpyDeviceToHost));
        // rows hold local slots of the residue's pack
        for (int pk = 0; pk < n_packs(c); ++pk) {
            const int off = c->pack_off[pk], m = c->pack_off[pk + 1] - off;
            for (int t = 0; t < m; ++t) {
                const int i = c->slot_res[off + t];
                for (int k = 0; k < std::min(cnt[i], c->cap); ++k) {
                    const int sl = list[(size_t)i * c->cap + k];
                    if (sl >= m)
                        return fail(c, SOP_E_LIST_OVERFLOW, "list entry outside its pack");
                    const int j = c->slot_res[off + sl];
                    if (i < j)
                        pairs.push_back({i, j});
                }
            }
        }
    } else {
        // rows hold slots of their tile; the tile's stage maps slots to ids
        const int T = c->tile, SM = stage_max_host(T);
        const auto &tl = c->tiles[tile_index(T)];
        const size_t n_tiles = tl.size() - 1;
        std::vector<unsigned short> list((size_t)n * c->cap);
        std::vector<int> stage(n_tiles * (size_t)SM), stage_cnt(n_tiles);
        HIP_TRY(c, hipMemcpy(list.data(), c->b.flist16, list.size() * sizeof(unsigned short),
                             hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(cnt.data(), c->b.fcnt, n * sizeof(int), hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(stage.data(), c->b.stage, stage.size() * sizeof(int), hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(stage_cnt.data(), c->b.stage_cnt, n_tiles * sizeof(int), hipMemcpyDeviceToHost));
        size_t tile = 0;
        for (long long i = 0; i < n; ++i) {
            while (i >= tl[tile + 1])
                ++tile;
            for (int k = 0; k < std::min(cnt[i], c->cap); ++k) {
                const int sl = list[list16_index_host(i, k, c->cap)];
                if (sl >= stage_cnt[tile])
                    return fail(c, SOP_E_LIST_OVERFLOW, "list entry outside its tile's staging set");
                const int j = stage[tile * SM + sl];
                if (i < j)
                    pairs.push_back({(int)i, j});
            }
        }
    }
    std::sort(pairs.begin(), pairs.end());
    *n_pairs = (int64_t)pairs.size();
    if ((int64_t)pairs.size() > cap)
        return fail(c, SOP_E_ARG, "output capacity too small");
    for (size_t k = 0; k < pairs.size(); ++k) {
        ij[2 * k] = pairs[k].first;
        ij[2 * k + 1] = pairs[k].second;
    }
    return SOP_OK;
}

sop_status sop_compute_forces(sop_ctx *c, double *f, double *energies, double *f_ext)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    const bool stale = !c->list_valid || c->step % c->p.list_every == 0;
    if (c->schedule == SOP_SCHEDULE_BATCHED) {
        batch_launch(c, c->stream, 1, stale ? 1 : 0, 1, nullptr, c->step);
    } else {
        if (stale)
            rebuild(c, c->stream, false);
        launch_step(c->b, c->cur, (int)c->n_res, c->cap, c->tile, step_consts(c), c->tip,
                    c->pulls.empty() ? 0 : 1, true, 1, nullptr, c->step, 0.0f, c->stream, c->force_mode);
        launch_reduce_energy(c->b, c->n_traj, c->stream);
    }
    c->list_valid = true;
    HIP_TRY(c, hipGetLastError());
    st = check_device_errors(c);
    if (st != SOP_OK)
        return st;
    c->energy_step = c->step;
    const long long n = c->n_res;
    if (f) {
        std::vector<float4> fo(n);
        HIP_TRY(c, hipMemcpy(fo.data(), c->b.fout, n * sizeof(float4), hipMemcpyDeviceToHost));
        for (long long i = 0; i < n; ++i) {
            f[3 * i] = fo[i].x;
            f[3 * i + 1] = fo[i].y;
            f[3 * i + 2] = fo[i].z;
        }
    }
    if (energies)
        HIP_TRY(c, hipMemcpy(energies, c->b.energy, (size_t)c->n_traj * SOP_NTERMS * sizeof(double),
                             hipMemcpyDeviceToHost));
    if (f_ext)
        HIP_TRY(c, hipMemcpy(f_ext, c->b.f_ext, (size_t)c->n_traj * sizeof(double), hipMemcpyDeviceToHost));
    return SOP_OK;
}

sop_status sop_step(sop_ctx *c, int64_t n_steps)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (n_steps < 0)
        return fail(c, SOP_E_ARG, "negative step count");
    if (c->sticky)
        return fail(c, status_from_bits(c->sticky), bits_message(c->sticky));
    if (c->schedule == SOP_SCHEDULE_BATCHED) {
        const long long K = c->batch_steps;
        const long long X = c->re_rep > 1 ? c->re_every : 0;
        bool base_set = false;
        long long q = 0;
        while (q < n_steps) {
            if (X > 0 && c->step % X == 0 && c->re_last != c->step) {
                // replica exchange before this step's update: energies of
                // the current positions, then one round of swaps
                batch_launch(c, c->stream, 1, c->list_valid ? 0 : 1, 1, nullptr, c->step);
                c->list_valid = true;
                c->energy_step = c->step;
                launch_exchange(c->b, c->re_rep, (int)(c->n_traj / c->re_rep), c->p.kBT, c->step / X,
                                (unsigned)(c->p.seed & 0xffffffffu), (unsigned)(c->p.seed >> 32), c->stream);
                c->re_last = c->step;
                base_set = false;
            }
            long long k = std::min<long long>(K, n_steps - q);
            if (X > 0)
                k = std::min<long long>(k, X - c->step % X);  // stop at the next exchange
            const long long rec = last_record(c, c->step, k);
            if (c->graph_steps > 0 && c->list_valid && k == K && X == 0) {
                const int rg = rec >= 0 ? 1 : 0;
                if (!c->bgraphs[c->cur][rg]) {
                    st = capture_batch_graph(c, c->cur, rg);
                    if (st != SOP_OK)
                        return st;
                }
                if (!base_set) {
                    launch_set_step(c->b.step_base, c->step, c->stream);
                    base_set = true;
                }
                HIP_TRY(c, hipGraphLaunch(c->bgraphs[c->cur][rg], c->stream));
            } else {
                batch_launch(c, c->stream, (int)k, c->list_valid ? 0 : 1, 0, nullptr, c->step, rec >= 0);
                base_set = false;
            }
            if (rec >= 0)
                c->energy_step = rec;
            c->list_valid = true;
            c->cur ^= 1;
            c->step += k;
            q += k;
        }
        HIP_TRY(c, hipGetLastError());
        return SOP_OK;
    }
    const int L = c->p.list_every;
    const long long E = c->energy_every;
    const long long span = (long long)L * std::max(c->graph_steps, 1);
    // graphs replay whole list periods and record energies only at their
    // first step: with an energy interval (a multiple of the span) a graph
    // starts only on a multiple of the span, so no record step falls inside
    const bool graphs_ok = c->graph_steps > 0 && (E == 0 || E % span == 0);
    const long long align = E > 0 ? span : L;
    bool base_set = false;
    long long q = 0;
    while (q < n_steps) {
        if (graphs_ok && c->step % align == 0 && n_steps - q >= span &&
            !(c->integrator == SOP_INTEGRATOR_UNDERDAMPED && c->ud_half)) {
            const int en = (E > 0 && c->step % E == 0) ? 1 : 0;
            if (!c->graphs[c->cur][en]) {
                st = capture_graph(c, c->cur, en);
                if (st != SOP_OK)
                    return st;
            }
            if (!base_set) {
                launch_set_step(c->b.step_next, c->step, c->stream);
                base_set = true;
            }
            // the graph's first rebuild relies on the cells holding the
            // current positions and on the displacement check
            if (c->binned_at != c->step)
                launch_bin_all(c->b, c->cur, (int)c->n_res, c->grid, c->stream);
            if (c->skin_checked != c->step)
                launch_force_skin(c->b, c->stream);
            HIP_TRY(c, hipGraphLaunch(c->graphs[c->cur][en], c->stream));
            if (en)
                c->energy_step = c->step;
            c->list_valid = true;
            c->step += span;
            c->skin_checked = c->binned_at = c->step;
            if (span & 1)
                c->cur ^= 1;
            q += span;
            continue;
        }
        const bool en = E > 0 && c->step % E == 0;
        const bool chk = checks_skin(c, c->step);
        bool fused = false;
        if (!c->list_valid || c->step % L == 0) {
            fused = fuses_filter(c, chk);
            rebuild(c, c->stream, false, false, !fused);
            c->list_valid = true;
        }
        one_step(c, c->stream, nullptr, c->step, en, chk, fused);
        c->ud_half = false;
        if (en)
            c->energy_step = c->step;
        c->cur ^= 1;
        ++c->step;
        if (chk)
            c->skin_checked = c->binned_at = c->step;
        ++q;
        base_set = false;
    }
    HIP_TRY(c, hipGetLastError());
    return SOP_OK;
}

sop_status sop_step_timed(sop_ctx *c, int64_t n_steps, double *ms_out)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (n_steps < 0 || !ms_out)
        return fail(c, SOP_E_ARG, "bad timing arguments");
    if (c->sticky)
        return fail(c, status_from_bits(c->sticky), bits_message(c->sticky));
    hipEvent_t ev[4];
    for (auto &e : ev)
        HIP_TRY(c, hipEventCreate(&e));
    if (c->schedule == SOP_SCHEDULE_BATCHED) {
        double sum = 0.0;
        long long cnt = 0, q = 0;
        sop_status out = SOP_OK;
        while (q < n_steps) {
            const long long k = std::min<long long>(c->batch_steps, n_steps - q);
            const long long rec = last_record(c, c->step, k);
            (void)hipEventRecord(ev[0], c->stream);
            batch_launch(c, c->stream, (int)k, c->list_valid ? 0 : 1, 0, nullptr, c->step, rec >= 0);
            (void)hipEventRecord(ev[1], c->stream);
            hipError_t e = hipEventSynchronize(ev[1]);
            if (e != hipSuccess) {
                out = hip_fail(c, e, "hipEventSynchronize");
                break;
            }
            float ms = 0.0f;
            if (k == c->batch_steps && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) {
                sum += ms;
                ++cnt;
            }
            if (rec >= 0)
                c->energy_step = rec;
            c->list_valid = true;
            c->cur ^= 1;
            c->step += k;
            q += k;
        }
        for (auto &e : ev)
            (void)hipEventDestroy(e);
        ms_out[0] = cnt ? sum / (double)cnt : 0.0;
        ms_out[1] = 0.0;
        ms_out[2] = (double)c->batch_steps;
        if (out == SOP_OK)
            HIP_TRY(c, hipGetLastError());
        return out;
    }
    // Plain schedule: each kernel group is captured n_steps times back to back
    // in one graph (the step kernel reuses the current list; the rebuild
    // re-bins the same positions), so the events around the graph launch see
    // kernel time plus the short gaps between graph nodes.  The positions and
    // the error word are saved first and restored afterwards: steps on a
    // stale list may trip the error checks, which must not outlive the timing.
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    const long long K = n_steps;
    ms_out[0] = ms_out[1] = ms_out[2] = 0.0;
    if (K == 0)
        return SOP_OK;
    const size_t bytes = 2 * (size_t)c->n_res * sizeof(float4);
    hipStream_t s = c->stream;
    unsigned err_saved = 0;
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(&err_saved, c->b.err, sizeof(unsigned), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpyAsync(c->b.pos_save, c->b.pos[c->cur], bytes, hipMemcpyDeviceToDevice, s));
    if (!c->list_valid) {
        rebuild(c, s, false);
        c->list_valid = true;
    }
    if (!c->cap_stream)
        HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    sop_status out = SOP_OK;
    // kind 0: step kernels; 1: rebuilds with the skin build; 2: rebuilds
    // that only filter the skin rows (the skin stays valid in between)
    const int kinds = c->schedule == SOP_SCHEDULE_PLAIN ? 3 : 2;
    for (int kind = 0; kind < kinds && out == SOP_OK; ++kind) {
        const int saved = c->cur;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            out = hip_fail(c, e, "hipStreamBeginCapture");
            break;
        }
        for (long long q = 0; q < K; ++q) {
            if (kind == 0) {
                launch_step(c->b, c->cur, (int)c->n_res, c->cap, c->tile, step_consts(c), c->tip,
                            c->pulls.empty() ? 0 : 1, false, 0, nullptr, c->step + q, 0.0f,
                            c->cap_stream, c->force_mode, 0.0f);
                c->cur ^= 1;
            } else {
                // kind 1: a search from freshly binned positions; kind 2:
                // the filter alone (the skin stays valid)
                c->skin_checked = c->binned_at = -1;
                rebuild(c, c->cap_stream, false, kind == 2);
            }
        }
        e = hipStreamEndCapture(c->cap_stream, &g);
        c->cur = saved;
        if (e != hipSuccess) {
            out = hip_fail(c, e, "hipStreamEndCapture");
            break;
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            out = hip_fail(c, e, "hipGraphInstantiate");
            break;
        }
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first replay warms up
            (void)hipEventRecord(e0, s);
            e = hipGraphLaunch(ex, s);
            (void)hipEventRecord(e1, s);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
        }
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipGraphExecDestroy(ex);
        if (e != hipSuccess) {
            out = hip_fail(c, e, "timed graph");
            break;
        }
        ms_out[kind] = (double)ms / (double)K;
        // back to the saved positions; the next list is built from them
        HIP_TRY(c, hipMemcpyAsync(c->b.pos[c->cur], c->b.pos_save, bytes, hipMemcpyDeviceToDevice, s));
        if (kind == 0) {
            c->skin_checked = c->binned_at = -1;
            rebuild(c, s, false);
        }
    }
    c->skin_checked = c->binned_at = -1;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->list_valid = false;
    if (out == SOP_OK) {
        HIP_TRY(c, hipStreamSynchronize(s));
        HIP_TRY(c, hipMemcpy(c->b.err, &err_saved, sizeof(unsigned), hipMemcpyHostToDevice));
    }
    return out;
}

sop_status sop_get_energies(sop_ctx *c, double *energies, int64_t *step)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    st = check_device_errors(c);
    if (st != SOP_OK)
        return st;
    if (energies)
        HIP_TRY(c, hipMemcpy(energies, c->b.energy, (size_t)c->n_traj * SOP_NTERMS * sizeof(double),
                             hipMemcpyDeviceToHost));
    if (step)
        *step = c->energy_step;
    return SOP_OK;
}

sop_status sop_get_external_force(sop_ctx *c, double *f_ext)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (!f_ext)
        return fail(c, SOP_E_ARG, "null output");
    st = check_device_errors(c);
    if (st != SOP_OK)
        return st;
    HIP_TRY(c, hipMemcpy(f_ext, c->b.f_ext, (size_t)c->n_traj * sizeof(double), hipMemcpyDeviceToHost));
    return SOP_OK;
}

sop_status sop_sample_noise(sop_ctx *c, int64_t step, uint32_t *words, double *g)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (step < 0)
        return fail(c, SOP_E_ARG, "negative step");
    // fout is scratch outside a force evaluation
    launch_noise(c->b, c->cur, (int)c->n_res, step_consts(c), step, c->b.words, c->b.fout, c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const long long n = c->n_res;
    if (words)
        HIP_TRY(c, hipMemcpy(words, c->b.words, n * sizeof(uint4), hipMemcpyDeviceToHost));
    if (g) {
        std::vector<float4> gv(n);
        HIP_TRY(c, hipMemcpy(gv.data(), c->b.fout, n * sizeof(float4), hipMemcpyDeviceToHost));
        for (long long i = 0; i < n; ++i) {
            g[3 * i] = gv[i].x;
            g[3 * i + 1] = gv[i].y;
            g[3 * i + 2] = gv[i].z;
        }
    }
    return SOP_OK;
}

}  // extern "C"

namespace {

// FNV-1a digest of what the schedule's speed depends on.
unsigned long long topology_digest(const sop_ctx *c)
{
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((unsigned long long)c->n_res);
    mix((unsigned long long)c->n_traj);
    for (long long v : c->res_offsets)
        mix((unsigned long long)v);
    for (const int2 &r : c->trow)
        mix((unsigned long long)(unsigned)r.y);
    mix((unsigned long long)c->cap);
    mix((unsigned long long)c->p.list_every);
    return h;
}

std::string cache_key(const sop_ctx *c)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s|%d|%016llx", arch.c_str(), c->schedule, topology_digest(c));
    return buf;
}

// Cache lines: <key> <a> <b>   (plain schedule: a = tile, b = force mode; batched: a = wg,
// b = steps)
bool cache_lookup(const char *path, const std::string &key, int *a, int *b)
{
    if (!path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char k[200];
    int x, y;
    bool found = false;
    while (std::fscanf(f, "%199s %d %d", k, &x, &y) == 3)
        if (key == k) {
            *a = x;
            *b = y;
            found = true;
        }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, int a, int b)
{
    if (!path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f, "%s %d %d\n", key.c_str(), a, b);
    std::fclose(f);
}

// Residue-steps per second of `steps` steps from the saved state.
// A candidate slower than a third of `best` (residue-steps/s; 0: none yet)
// is stopped after the first eighth of its steps.
sop_status trial(sop_ctx *c, long long steps, double *rate, double best = 0.0)
{
    const size_t bytes = 2 * (size_t)c->n_res * sizeof(float4);
    HIP_TRY(c, hipMemcpyAsync(c->b.pos[c->cur], c->b.pos_save, bytes, hipMemcpyDeviceToDevice, c->stream));
    const long long step0 = c->step;
    c->list_valid = false;
    c->skin_checked = c->binned_at = -1;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    sop_status st = sop_step(c, 2 * c->p.list_every);  // warm up: capture graphs, touch caches
    const long long L2 = 2 * c->p.list_every;
    const long long chunk = std::max<long long>(L2, (steps / 8 / L2) * L2);
    long long done = 0;
    float ms = 0.0f;
    if (st == SOP_OK)
        (void)hipEventRecord(e0, c->stream);
    while (st == SOP_OK && done < steps) {
        const long long k = std::min(chunk, steps - done);
        st = sop_step(c, k);
        done += k;
        (void)hipEventRecord(e1, c->stream);
        if (st != SOP_OK || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            ms = 0.0f;
            break;
        }
        const double r = ms > 0 ? (double)c->n_res * (double)done / (1e-3 * ms) : 0.0;
        if (best > 0.0 && r < best / 3.0)
            break;  // clearly slower: no need for the rest
    }
    *rate = ms > 0 ? (double)c->n_res * (double)done / (1e-3 * ms) : 0.0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // back to the saved state (the trial advanced the layer parity too)
    HIP_TRY(c, hipMemcpyAsync(c->b.pos[c->cur], c->b.pos_save, bytes, hipMemcpyDeviceToDevice, c->stream));
    c->step = step0;
    c->list_valid = false;
    c->skin_checked = c->binned_at = -1;
    return st;
}

}  // namespace

extern "C" {

sop_status sop_autotune(sop_ctx *c, double budget_ms, const char *cache_path)
{
    sop_status st = need_ready(c);
    if (st != SOP_OK)
        return st;
    if (c->sticky)
        return fail(c, status_from_bits(c->sticky), bits_message(c->sticky));
    const std::string key = cache_key(c);
    int a = 0, b = 0;
    if (cache_lookup(cache_path, key, &a, &b)) {
        if (c->schedule == SOP_SCHEDULE_BATCHED)
            return sop_set_batch(c, a, b);
        const sop_status s1 = sop_set_tile(c, a);
        return s1 != SOP_OK ? s1 : sop_set_force_mode(c, b);
    }
    const size_t bytes = 2 * (size_t)c->n_res * sizeof(float4);
    HIP_TRY(c, hipMemcpyAsync(c->b.pos_save, c->b.pos[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream));
    const long long saved_energy_step = c->energy_step;
    std::vector<std::pair<int, int>> cand;
    if (c->schedule == SOP_SCHEDULE_BATCHED) {
        for (int wg : {256, 512, 1024})
            if (wg >= c->max_len)
                for (int k : {20, 50, 100, 200})
                    cand.push_back({wg, k});
    } else {
        for (int mode : {SOP_FORCES_PARTICLE, SOP_FORCES_PAIR})
            for (int tl : {64, 128, 256})
                cand.push_back({tl, mode});
    }
    // steps per trial from the budget, using the current schedule's speed as a guide
    double rate0 = 0.0;
    st = trial(c, 4 * c->p.list_every, &rate0);
    if (st != SOP_OK)
        return st;
    const double per_trial_ms = std::max(1.0, budget_ms / (double)cand.size());
    long long steps = (long long)(rate0 * 1e-3 * per_trial_ms / (double)c->n_res);
    steps = std::max<long long>(2 * c->p.list_every, (steps / (2 * c->p.list_every)) * 2 * c->p.list_every);
    if (c->schedule == SOP_SCHEDULE_BATCHED)
        steps = std::max<long long>(steps, 400);
    double best = -1.0;
    std::pair<int, int> pick = cand.front();
    for (const auto &cd : cand) {
        if (c->schedule == SOP_SCHEDULE_BATCHED) {
            st = sop_set_batch(c, cd.first, cd.second);
        } else {
            st = sop_set_tile(c, cd.first);
            if (st == SOP_OK)
                st = sop_set_force_mode(c, cd.second);
        }
        if (st != SOP_OK)
            return st;
        double rate = 0.0;
        st = trial(c, steps, &rate, best);
        if (st != SOP_OK)
            return st;
        if (rate > best) {
            best = rate;
            pick = cd;
        }
    }
    if (c->schedule == SOP_SCHEDULE_BATCHED) {
        st = sop_set_batch(c, pick.first, pick.second);
    } else {
        st = sop_set_tile(c, pick.first);
        if (st == SOP_OK)
            st = sop_set_force_mode(c, pick.second);
    }
    if (st != SOP_OK)
        return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->energy_step = saved_energy_step;
    cache_store(cache_path, key, pick.first, pick.second);
    return check_device_errors(c);
}

sop_status sop_synchronize(sop_ctx *c)
{
    if (!c)
        return SOP_E_ARG;
    return check_device_errors(c);
}

}  // extern "C"
