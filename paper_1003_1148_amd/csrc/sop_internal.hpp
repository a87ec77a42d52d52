// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sop.h"

namespace sop {

// Device-side error bits (sticky until new coordinates are loaded).
enum : unsigned {
    ERR_FENE = 1u << 0,
    ERR_OVERFLOW = 1u << 1,
    ERR_NONFINITE = 1u << 2,
    ERR_TIP = 1u << 3,
    ERR_CELL = 1u << 4,  // a rebuild cell holds more than CELL_CAP residues
    ERR_STAGE = 1u << 5, // a tile interacts with more residues than its LDS staging holds
};

// Per-residue energy record written on energy steps:
// FENE, native, repulsive, external, virial, external-force report.
constexpr int RES_E = 6;

struct PullDev {
    double anchor0[3];
    double v[3];
    double vhat[3];
    double kappa;
    int32_t residue;
    int32_t has_dir;
};

struct TipDev {
    double c0[3];
    double v[3];
    double vhat[3];
    double radius;
    double eps;
    double sigma;
    int32_t on;
    int32_t has_dir;
};

// Cell grid used to rebuild the list: wrapped (periodic-index) grid of
// gx*gy*gz cells of edge `cell`, so any position maps to a valid cell.
struct GridDev {
    float inv_cell;
    int gx, gy, gz;
    int n_cells;
};

// Residues per cell of the list-rebuild grid (fixed capacity; more is the
// list-overflow error).  A cell's edge is the search radius, 24 A by
// default: at protein density (about 120 A^3 per residue) a cell holds some
// 115 residues on average.
constexpr int CELL_CAP = 256;
// Bonded plus native partners per residue (larger is rejected at load).
constexpr int TOPO_CAP = 64;
// Largest staging set of a tile of the plain schedule (slots are 16-bit;
// the kernels hold 1,024 or 2,048 of them in LDS at once).
constexpr int STAGE_MAX = 4096;

// Device buffers carved out of the caller's workspace.
struct DevBufs {
    // positions, two time layers; residue i is pos[l][2i] = {hi.xyz, tag},
    // pos[l][2i+1] = {lo.xyz, trajectory}; tag = index inside the
    // trajectory | fixed << 31.  x = hi + lo.
    float4 *pos[2];
    int2 *trow;       // per residue: {first entry, n_bond | n_native << 12}
    float2 *tent;     // {partner id bits, r0}: bonds first, then natives
    int *list_cnt;    // partners per residue (plain: of the skin rows)
    unsigned short *list16;  // rows by residue (cap entries): plain, skin rows (pairs within
                             // r_list + skin at the last skin build) as slots of its tile;
                             // batched, the list as local slots of its pack
    int *fcnt;               // plain: list partners per residue (the skin rows filtered at r_list)
    unsigned short *flist16; // plain: the list rows (cap entries), slots of the residue's tile
    float4 *hi_skin;         // plain: high parts of the positions at the last skin build
    unsigned *skin_flag;     // plain: nonzero when the next rebuild must rebuild the skin
    unsigned long long *list_stats;  // plain: {rebuilds, skin builds} since binding
    unsigned char *tile_ord; // plain: per tile (tile * T + rank), its residues by decreasing list length
    unsigned short *skin_ord;  // plain: per tile (tile * T + rank), 1 + its residues by decreasing
                               // skin row length (0 before the first skin search: identity)
    float4 *vel;             // plain, underdamped: per-residue velocity before its last half kick
    double *re_kbt;          // batched, replica exchange: the temperature ladder (kB T)
    int *re_tidx;            // batched, replica exchange: temperature index of each trajectory
    float *re_tscale;        // batched, replica exchange: sqrt(kB T / kB T of the parameters)
    unsigned long long *re_stats;  // batched, replica exchange: {accepted, attempted} per ladder pair
    float4 *facc;            // plain, pair-based forces: per-residue force accumulator
    double4 *eacc;           // plain, pair-based forces: per-residue energy accumulator
    uint2 *topo2;            // plain: {slot, r0 bits} of bonded/native partners, (i/T)*TOPO_CAP*T + e*T + i%T
    int *stage;       // plain: per tile, global ids of its slots (stage_max per tile)
    int *stage_cnt;   // plain: slots per tile
    int *pack_off;    // batched form: first slot of each pack (n_packs + 1)
    int *slot_res;    // batched form: residue of each slot (a permutation of the residues)
    float4 *pos_save; // one saved layer (autotuning restores the state it found)
    int *cell_count;  // residues per cell
    float4 *cells;    // CELL_CAP slots per cell: {hi.xyz, residue id bits}
    int *cell_of;     // per residue: its cell at the last rebuild
    int *tile_first[3];  // plain: first residue of each tile (+ n) for tiles of 64, 128, 256
    int n_tiles[3];
    int4 *traj_cell;  // per trajectory: cell-index offset that keeps trajectories apart
    int *traj_lo;     // per residue: first residue of its trajectory
    int *traj_hi;     // per residue: one past the last residue of its trajectory
    int *pull_slot;   // per residue: cantilever index or -1
    PullDev *pulls;
    unsigned *stream_ids;    // per trajectory
    uint2 *noise_key;        // per residue: {tag, stream id}, the static words of its Philox counter
    long long *res_offsets;  // n_traj + 1
    double *res_energy;      // n_res * RES_E
    int *chunk_lo;           // energy reduction: first residue of each chunk (+ n_res)
    int *chunk_first;        // energy reduction: first chunk of each trajectory (+ n_chunks)
    double *chunk_sum;       // energy reduction: RES_E partial sums per chunk
    int n_chunks;
    double *energy;          // n_traj * SOP_NTERMS, last record
    double *f_ext;           // n_traj, last record
    float4 *fout;            // forces (compute_forces), noise samples
    uint4 *words;            // Philox words (noise samples)
    long long *step_base;    // graph replays: step of the period's first step
    long long *step_next;
    unsigned *err;
};

struct StepConsts {
    float k_fene, R0sq, inv_R0sq, eps_h, eps_l, sigma2;
    float c_drift, c_noise;
    float ud_c1, ud_c2;  // underdamped: exp(-zeta h/m), sqrt((1 - c1^2) kB T/m)
    unsigned key0, key1;
    double h;
};

// ---- kernel launchers (sop_kernels.hip) ----------------------------------
// Plain schedule, tiles of `tile` residues (64, 128 or 256).
// The skin search (the per-tile rows within sqrt(rs2) from the cell grid,
// renumbered by residue id) runs only when the device skin flag is set; the
// filter to rc2 runs unless `filter` is false (then the next step kernel
// filters).  `binned`: the cells already hold the current
// positions (binned by the last step kernel of the period); otherwise they
// are cleared and filled first.
void launch_rebuild(const DevBufs &b, int cur, int n_res, int cap, int tile, const GridDev &g,
                    float rc2, float rs2, int multi, hipStream_t s, bool advance_step_base, int list_every,
                    bool binned, bool filter = true);
// Sets the skin flag so that the next rebuild rebuilds the skin.
void launch_force_skin(const DevBufs &b, hipStream_t s);
// Clears the cells and bins every residue at its current position.
void launch_bin_all(const DevBufs &b, int cur, int n_res, const GridDev &g, hipStream_t s);
// mode: 0 = step, 1 = forces only.  check_thr2 > 0: after the update, a
// residue that moved more than sqrt(check_thr2) from its position at the
// last skin build sets the skin flag.
// force_mode 0: particle-based (each residue sums its own rows); 1:
// pair-based (each pair once, atomic accumulation, then the update kernel).
// filter_rc2 > 0 (particle-based stepping only): the first step after a
// rebuild launched without its filter (launch_rebuild, filter = false),
// which filters the skin rows at filter_rc2 itself, then clears the
// n_cells cell counts and the skin flag.
void launch_step(const DevBufs &b, int cur, int n_res, int cap, int tile, const StepConsts &c,
                 const TipDev &tip, int has_pull, bool energy, int mode,
                 const long long *step_base, long long step_off, float check_thr2, hipStream_t s,
                 int force_mode = 0, float ud_kick = 0.0f, const GridDev *bin_grid = nullptr,
                 float filter_rc2 = 0.0f, int n_cells = 0);
// Residues per chunk of the energy reduction (chunks never span trajectories).
constexpr int ECHUNK = 1024;
void launch_reduce_energy(const DevBufs &b, int n_traj, hipStream_t s);
// Batched ensemble: n_steps steps of every pack in one launch.  mode 0:
// steps without energy records; 2: steps that record at multiples of
// energy_every; 1: one force evaluation with records, no update.
void launch_batch(const DevBufs &b, int cur, int n_packs, int wg, int cap, const StepConsts &c,
                  const TipDev &tip, int has_pull, float rc2, int list_every, long long energy_every,
                  int n_steps, int stale, int mode, const long long *step_base, long long step_off,
                  hipStream_t s, const float *tscale = nullptr);
// Replica exchange: the swaps of one round from the energies recorded in
// b.energy (see k_exchange).
void launch_exchange(const DevBufs &b, int n_rep, int n_groups, double kbt_ref, long long round,
                     unsigned key0, unsigned key1, hipStream_t s);
void launch_add_step(long long *base, long long k, hipStream_t s);
void launch_set_step(long long *dst, long long value, hipStream_t s);
void launch_noise(const DevBufs &b, int cur, int n, const StepConsts &c, long long step, uint4 *words,
                  float4 *g, hipStream_t s);

// Plain schedule: entry k of residue r's row (a slot of its tile), and the
// slots a tile of `tile` residues can stage.
inline size_t list16_index_host(long long r, int k, int cap) { return (size_t)r * cap + (size_t)k; }
inline int stage_max_host(int) { return 4096; }
inline int tile_index(int tile) { return tile == 64 ? 0 : (tile == 128 ? 1 : 2); }

}  // namespace sop
