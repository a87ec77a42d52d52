/*
 * libsop -- overdamped Langevin dynamics of the Self Organized Polymer (SOP)
 * model on AMD Instinct MI355X (gfx950).
 *
 * The library advances r_i(t+h) = r_i(t) + f_i h/xi + g_i sqrt(2 kB T h/xi)
 * (first-order Ermak-McCammon scheme: paper Eq. 2, Algorithm 7) for many
 * residues at once, where f_i = -grad_i V with V the SOP potential of Eq. 1:
 *   - FENE backbone bonds  -(k R0^2/2) ln(1 - (r - r0)^2 / R0^2),
 *   - native contacts      eps_h [(r0/r)^12 - 2 (r0/r)^6],
 *   - every other pair of a trajectory (i,i+2 included) eps_l (sigma/r)^6,
 *     evaluated over a Verlet list of pairs closer than r_list, rebuilt every
 *     list_every steps (Section III.A, Algorithm 3),
 * and g_i are standard Gaussians (Section III.C) drawn by Box-Muller from a
 * counter-based Philox4x32-10 stream.  Optional external terms carry the
 * pulling and indentation protocols (Section IV.B): a harmonic cantilever on
 * chosen residues and a spherical tip moving at constant velocity.
 *
 * Units are the caller's; the reference workloads use kcal/mol, Angstrom and
 * a reduced time tau.  Positions are held on the device in single precision
 * as a compensated pair (hi, lo) with x = hi + lo; forces are single
 * precision; energy and virial sums are double precision.
 *
 * Conventions for every call:
 *   - Pointers named *host* or documented as host arrays are host memory,
 *     borrowed for the duration of the call and copied.  The workspace is
 *     device memory owned by the caller.
 *   - Every call returns a sop_status; nothing throws across the ABI.  On
 *     failure, sop_last_error() describes the cause.
 *   - A context is not thread safe; use one context per host thread.  All
 *     device work of a context runs in order on the stream given to
 *     sop_create (0 means the default stream).
 *   - Device-side failures (broken bond, list overflow, non-finite values,
 *     tip penetration) are detected asynchronously.  They are reported by the
 *     next synchronizing call (sop_synchronize, sop_get_*) and stay reported
 *     ("sticky") until sop_set_coordinates loads new coordinates.
 */
#ifndef SOP_H
#define SOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sop_status {
    SOP_OK = 0,
    SOP_E_ARG = -1,           /* invalid argument */
    SOP_E_STATE = -2,         /* call made in the wrong order */
    SOP_E_WORKSPACE = -3,     /* workspace missing, misaligned or too small */
    SOP_E_HIP = -4,           /* HIP runtime error */
    SOP_E_FENE = -5,          /* a bond stretched to |r - r0| >= R0 */
    SOP_E_LIST_OVERFLOW = -6, /* a residue has more list partners than the capacity */
    SOP_E_NONFINITE = -7,     /* a force or position became NaN or infinite */
    SOP_E_TIP = -8            /* a residue reached the tip surface */
} sop_status;

/* Energy terms recorded per trajectory (double precision). */
enum {
    SOP_TERM_FENE = 0,
    SOP_TERM_NATIVE = 1,
    SOP_TERM_REPULSIVE = 2,
    SOP_TERM_EXTERNAL = 3,
    SOP_TERM_VIRIAL = 4, /* -sum over bonded, native and listed pairs of r dV/dr */
    SOP_NTERMS = 5
};

/* Force-field, thermostat and list parameters (Eq. 1, Eq. 2, Algorithm 3). */
typedef struct sop_params {
    double k_fene;         /* FENE spring constant k */
    double R0;             /* FENE tolerance R0 */
    double eps_h;          /* native contact depth */
    double eps_l;          /* repulsion strength (eps_r in Eq. 1) */
    double sigma;          /* repulsion range */
    double r_list;         /* Verlet-list cutoff: pairs with r < r_list at a rebuild */
    double kBT;            /* thermal energy */
    double zeta;           /* friction coefficient (xi) */
    double h;              /* time step */
    int32_t list_every;    /* rebuild period in steps (> 0) */
    int32_t list_capacity; /* list partners per residue, at most 1024 (else SOP_E_ARG);
                            0 selects 1024 (plain schedule) or 256 (batched) */
    uint64_t seed;         /* Philox key (low word, high word) */
} sop_params;

typedef struct sop_ctx sop_ctx;

/* ---- lifetime ----------------------------------------------------------- */

/* Create a context.  `hip_stream` is a hipStream_t borrowed for the context's
 * lifetime (0 = default stream).  Host only: touches no device. */
sop_status sop_create(const sop_params *params, void *hip_stream, sop_ctx **out);

/* Destroy a context.  Frees host memory and library-owned streams and
 * graphs; the caller's workspace is not freed. */
sop_status sop_destroy(sop_ctx *ctx);

/* ---- topology (Algorithm 2's P_p / PairsMap, built once on the host) ------ */

/*
 * Load n_traj independent trajectories ("systems") stored back to back:
 * trajectory t owns global residues [res_offsets[t], res_offsets[t+1]).
 *   res_offsets  int64[n_traj+1], res_offsets[0] = 0, non-decreasing
 *   stream_ids   uint32[n_traj] Philox stream of each trajectory, or NULL for
 *                0..n_traj-1
 *   bonds        int32[2*n_bonds], pairs of global residue ids (FENE terms)
 *   bond_r0      double[n_bonds], reference lengths r0 > 0
 *   natives      int32[2*n_native], pairs of global residue ids (12-6 terms)
 *   native_r0    double[n_native], reference distances r0 > 0
 *   fixed        uint8[n_res] (nonzero = residue never moves) or NULL
 * Returns SOP_E_ARG for an id out of range, a pair spanning two trajectories,
 * a self pair, a duplicate pair, a pair both bonded and native, r0 <= 0, or
 * more than 64 bonded plus native partners on one residue.  Host only.
 * Invalidates any bound workspace.
 */
sop_status sop_load_topology(sop_ctx *ctx, int32_t n_traj, const int64_t *res_offsets,
                             const uint32_t *stream_ids, int64_t n_bonds, const int32_t *bonds,
                             const double *bond_r0, int64_t n_native, const int32_t *natives,
                             const double *native_r0, const uint8_t *fixed);

/*
 * Harmonic cantilever on one residue of trajectory `traj`:
 * V = (kappa/2) |A(t) - r_c|^2, A(t) = anchor0 + v t, t = step * h.
 * The reported external force of the trajectory adds kappa (A - r_c).v/|v|
 * (or kappa |A - r_c| when v = 0).  At most one cantilever per residue.
 * Call after sop_load_topology and before sop_bind_workspace.  Host only.
 */
sop_status sop_set_pulling(sop_ctx *ctx, int32_t traj, int64_t residue, double kappa,
                           const double anchor0[3], const double v[3]);

/*
 * Spherical tip acting on every residue: with s = |r_i - T(t)| - radius and
 * T(t) = c0 + v t, V = eps (sigma/s)^6; s <= 0 is the SOP_E_TIP error.  The
 * reported external force adds sum_i f_i.v/|v| over the trajectory's
 * residues.  radius < 0 removes the tip.  Call before sop_bind_workspace.
 */
sop_status sop_set_tip(sop_ctx *ctx, double radius, double eps, double sigma, const double c0[3],
                       const double v[3]);

/* ---- schedule ------------------------------------------------------------ */

enum {
    SOP_SCHEDULE_PLAIN = 0,   /* one fused kernel per step over a cell-grid list */
    SOP_SCHEDULE_BATCHED = 1  /* one persistent launch per many steps; each workgroup
                                 keeps whole trajectories (<= 1024 residues each)
                                 resident in LDS */
};

/*
 * Execution schedule (call before sop_bind_workspace).  Both schedules compute
 * the same dynamics from the same noise stream; they differ in how work maps
 * to the GPU.  The batched schedule is for ensembles of many independent
 * trajectories (the paper's many-runs-per-GPU mode, Section IV.D); it returns
 * SOP_E_ARG when a trajectory has more than 1024 residues.
 */
sop_status sop_set_schedule(sop_ctx *ctx, int32_t schedule);

/*
 * Batched schedule: residues per workgroup (256, 512 or 1024; 0 = the
 * smallest that holds the longest trajectory) and steps per launch (>= 1).
 * Whole trajectories are packed into workgroups first-fit decreasing by
 * length (ties by index); n_packs reports how many workgroups that makes.
 * Results do not depend on these choices.  May be changed after binding;
 * the list is rebuilt at the next step.
 */
sop_status sop_set_batch(sop_ctx *ctx, int32_t wg_residues, int32_t steps_per_launch);
sop_status sop_get_batch(const sop_ctx *ctx, int32_t *wg_residues, int32_t *steps_per_launch,
                         int32_t *n_packs);

/*
 * Choose the schedule parameters by timing: tile size (plain) or
 * workgroup size and steps per launch (batched).  Each candidate runs from
 * the current state, which is restored afterwards, for about budget_ms in
 * total.  With a cache_path, a matching entry (device, schedule, topology
 * digest) is used without timing and new results are appended; the choice
 * is therefore deterministic given the cache.  Needs bound coordinates.
 */
sop_status sop_autotune(sop_ctx *ctx, double budget_ms, const char *cache_path);

/*
 * Plain schedule: residues per workgroup ("tile" of consecutive residues;
 * 64, 128 or 256; 0 selects the default, 64).  At each list rebuild a tile
 * gathers the residues it interacts with into at most 1024 (tiles of 64 or
 * 128) or 2048 (tiles of 256) LDS slots, and the cells around it must number
 * at most 640, 1024 or 512 respectively; a tile that needs more reports
 * SOP_E_LIST_OVERFLOW.  May be changed after binding; the list is rebuilt at
 * the next step.
 */
sop_status sop_set_tile(sop_ctx *ctx, int32_t tile);

/* Tile size in effect (after a topology is loaded). */
sop_status sop_get_tile(const sop_ctx *ctx, int32_t *tile);

/*
 * HIP graphs: 0 launches every kernel from the host; k > 0 captures k whole
 * list periods (k rebuilds and k*list_every steps) per graph and replays it
 * while that many steps remain from a period start.  Graphs are used only when
 * the energy interval is 0 or a multiple of k*list_every, and then start only
 * on multiples of k*list_every, so every record step is a graph's first step.
 * Changing k drops the graphs already captured.  Default: 1.
 */
sop_status sop_set_graph_steps(sop_ctx *ctx, int32_t k);

/* Record energies every k steps (k = 0: never).  Energies of step n are
 * those of the configuration the forces of step n use, before its update.
 * Changing k drops the graphs already captured. */
sop_status sop_set_energy_interval(sop_ctx *ctx, int64_t k);

/* ---- workspace ----------------------------------------------------------- */

/* Bytes of device memory the bound workspace must provide (256-byte aligned
 * start).  Depends on the topology, the schedule and the list capacity. */
sop_status sop_workspace_size(const sop_ctx *ctx, size_t *bytes);

/*
 * Bind caller-owned device memory (e.g. a torch uint8 CUDA tensor) that must
 * outlive the context or the next bind.  Uploads the topology into it.
 * Coordinates must be set again after a bind.
 */
sop_status sop_bind_workspace(sop_ctx *ctx, void *device_ptr, size_t bytes);

/* ---- coordinates and steps ------------------------------------------------ */

/* Load positions from host double[3*n_res] (x0,y0,z0,x1,...), split into the
 * device's compensated single-precision pair.  Clears sticky errors and
 * marks the Verlet list stale.  Synchronous with respect to the host. */
sop_status sop_set_coordinates(sop_ctx *ctx, const double *xyz_host);

/* Copy positions (hi + lo, double) into host double[3*n_res].  Synchronizes. */
sop_status sop_get_coordinates(sop_ctx *ctx, double *xyz_host);

/* Step counter n (time t_n = n h) that seeds the noise and moves the
 * external anchors.  Setting it marks the list stale. */
sop_status sop_set_step(sop_ctx *ctx, int64_t step);
sop_status sop_get_step(const sop_ctx *ctx, int64_t *step);

/*
 * Advance n_steps steps of the first-order overdamped scheme (Eq. 2 with the
 * h/xi coefficient of Algorithm 7): every residue that is not fixed moves by
 * f_i h/xi + g_i sqrt(2 kB T h/xi), all forces taken at the positions of
 * t_n.  Asynchronous on the context's stream.  Before the forces of step n
 * the Verlet list is rebuilt when n % list_every == 0 or when it is stale.
 * Device-side failures surface at the next synchronizing call.
 */
sop_status sop_step(sop_ctx *ctx, int64_t n_steps);

/* Integrators of the plain schedule. */
enum {
    SOP_INTEGRATOR_OVERDAMPED = 0, /* the first-order scheme of Eq. 2 / Algorithm 7 (default) */
    SOP_INTEGRATOR_UNDERDAMPED = 1 /* Langevin dynamics with inertia (see sop_set_integrator) */
};

/*
 * Choose the plain schedule's integrator.  The paper's conclusion names the
 * underdamped limit as an extension of its integration kernel without
 * giving a scheme; SOP_INTEGRATOR_UNDERDAMPED integrates
 * m dv = F dt - zeta v dt + sqrt(2 zeta kB T) dW, dx = v dt with every
 * residue of mass `mass` (zeta, kB T and h from sop_params) by the BAOAB
 * splitting of Leimkuhler and Matthews (2013): with c1 = exp(-zeta h/m) and
 * c2 = sqrt((1 - c1^2) kB T/m), each step is v += (h/2m) F(x_n),
 * x += (h/2) v, v = c1 v + c2 g, x += (h/2) v, v += (h/2m) F(x_(n+1)), with
 * the same per-residue Gaussians g as the overdamped noise.  Positions stay
 * compensated; velocities are single precision.  Fixed residues keep zero
 * velocity.  sop_set_coordinates zeroes the velocities.  `mass` is ignored
 * for the overdamped integrator.  SOP_E_ARG for an unknown kind or a
 * non-positive mass; SOP_E_STATE on the batched schedule.
 */
sop_status sop_set_integrator(sop_ctx *ctx, int32_t kind, double mass);

/* Velocities at the current step, double[3*n_res] (host), single precision
 * on the device.  SOP_E_STATE on the batched schedule. */
sop_status sop_set_velocities(sop_ctx *ctx, const double *v_host);
/* Evaluates this step's forces when the stored velocities still lack their
 * last half kick.  Synchronizes. */
sop_status sop_get_velocities(sop_ctx *ctx, double *v_host);

/*
 * Replica exchange (parallel tempering) over the batched ensemble, the use of
 * the many-runs-per-GPU approach the paper's conclusion proposes.  The
 * trajectories form groups of n_rep consecutive ones (n_rep must divide the
 * trajectory count), normally copies of one system; trajectory t runs at
 * kB T = kbt[tidx[t]] (its noise amplitude sqrt(2 kbt h / zeta)), tidx being a
 * permutation of 0 .. n_rep-1 within each group (NULL: t mod n_rep).  At
 * every step n with n % exchange_every == 0 (0: never), before that step's
 * update, round r = n / exchange_every attempts in every group the swaps of
 * the trajectories at temperatures k and k+1 for k = r mod 2, r mod 2 + 2,
 * ...: with E the potential energy (FENE + native + repulsive + external)
 * at step n and d = (1/kbt[k] - 1/kbt[k+1]) (E_k - E_(k+1)), a swap is
 * accepted when d >= 0 or u < exp(d), u being the first word of Philox4x32-10
 * with counter (group, k, r low, r high) and key (seed low ^ 0x52455843, seed
 * high) mapped to (0,1) as the noise's uniforms are; an accepted swap
 * exchanges the two temperatures.  The energies of the exchange steps are
 * recorded (sop_get_energies).  Host arrays are copied.  SOP_E_STATE unless
 * the schedule is batched and a workspace is bound; SOP_E_ARG for a bad
 * n_rep, a non-positive temperature, a negative interval or indices that are
 * not a permutation in every group.
 */
sop_status sop_set_tempering(sop_ctx *ctx, int32_t n_rep, const double *kbt_host, int64_t exchange_every,
                             const int32_t *tidx_host);

/* Current temperature index of every trajectory (int32[n_traj], may be NULL)
 * and, per ladder pair k (n_rep - 1 entries each, may be NULL), the swaps
 * accepted and attempted since sop_set_tempering.  Synchronizes. */
sop_status sop_get_tempering(sop_ctx *ctx, int32_t *tidx_host, int64_t *accepted, int64_t *attempted);

/* Force evaluation of the plain schedule. */
enum {
    SOP_FORCES_PARTICLE = 0, /* each residue sums its own rows (Algorithms 1-2): every pair is
                                evaluated in both rows, with no write conflicts; deterministic */
    SOP_FORCES_PAIR = 1      /* each pair once (Algorithm 4), +df / -df added to both residues
                                with hardware float atomics and gathered in the update kernel
                                (Algorithm 5); reproducible to rounding only */
};

/*
 * Choose the plain schedule's force evaluation (SOP_FORCES_*; default
 * particle-based).  Both evaluate the same list and the same terms.
 * sop_autotune tries both.  SOP_E_ARG for an unknown mode.
 */
sop_status sop_set_force_mode(sop_ctx *ctx, int32_t mode);
sop_status sop_get_force_mode(const sop_ctx *ctx, int32_t *mode);

/*
 * Verlet skin of the plain schedule (Section III.A keeps a list of the pairs
 * closer than r_list and rebuilds it every list_every steps).  The cell-grid
 * search runs at r_list + skin and is repeated only when some residue has
 * moved more than skin/2 (less 0.01) since the last search; every rebuild
 * filters those rows with the list predicate at r_list, which gives exactly
 * the list a search over all pairs would give.  skin = 0 searches at every
 * rebuild.  Default 4 (the caller's length unit).  SOP_E_ARG for a negative
 * or non-finite skin or one above 4 r_list.  Takes effect at the next
 * rebuild.
 */
sop_status sop_set_list_skin(sop_ctx *ctx, double skin);

/* The Verlet skin in use (host only). */
sop_status sop_get_list_skin(const sop_ctx *ctx, double *skin);

/* Rebuilds of the list and cell-grid searches of the skin since the
 * workspace was bound (plain schedule).  Synchronizes. */
sop_status sop_get_list_stats(sop_ctx *ctx, int64_t *rebuilds, int64_t *skin_builds);

/*
 * Kernel timing (measurement only).  Plain schedule: the fused step kernel
 * and, separately, the list rebuild (all its kernels) are each captured
 * n_steps times back to back in one HIP graph and timed with a pair of HIP
 * events on the context's stream around the graph launch; ms_out[0] = mean
 * step-kernel duration, ms_out[1] = mean rebuild duration with the skin's
 * cell-grid search, ms_out[2] = mean rebuild duration that only filters the
 * skin rows.
 * The step launches reuse the current list, so the coordinates and the list
 * are restored afterwards (the step counter does not move).  Batched schedule:
 * n_steps steps in persistent launches, each timed with events and waited
 * for; ms_out[0] = mean duration of one launch, ms_out[1] = 0, ms_out[2] =
 * steps per launch (these steps advance the state).
 */
sop_status sop_step_timed(sop_ctx *ctx, int64_t n_steps, double *ms_out);

/* ---- pair list ------------------------------------------------------------- */

/* Rebuild the Verlet list (Section III.A, Algorithm 3) from the current
 * positions now: every pair of one trajectory that is neither bonded nor
 * native and whose single-precision distance is below r_list.  Asynchronous;
 * a row longer than the list capacity is SOP_E_LIST_OVERFLOW at the next
 * synchronizing call. */
sop_status sop_build_pairlist(sop_ctx *ctx);

/*
 * Copy the current list (Algorithm 3) as the sorted set of pairs (i < j),
 * lexicographic, into host int32[2*cap].  *n_pairs receives the list size; if it exceeds
 * cap, nothing is copied and SOP_E_ARG is returned.  Synchronizes.
 */
sop_status sop_get_pairlist(sop_ctx *ctx, int64_t cap, int32_t *ij_host, int64_t *n_pairs);

/* ---- forces and energies ---------------------------------------------------- */

/*
 * The forces f_i = -grad_i V of Eq. 1 (FENE bonds, native 12-6 contacts and
 * the (sigma/r)^6 repulsion over the list, each pair once per partner as in
 * Algorithms 1-2, plus the external terms) and the per-term energies at the
 * current positions and step, without moving anything; the list is rebuilt first when a step would rebuild it (stale,
 * or step % list_every == 0).  f_host: double[3*n_res]
 * or NULL; energies_host: double[n_traj*SOP_NTERMS] or NULL; f_ext_host:
 * double[n_traj] or NULL (reported external force).  Synchronizes.
 */
sop_status sop_compute_forces(sop_ctx *ctx, double *f_host, double *energies_host,
                              double *f_ext_host);

/* Latest recorded energies, double[n_traj*SOP_NTERMS], and the step they
 * belong to (-1 if none yet).  Synchronizes. */
sop_status sop_get_energies(sop_ctx *ctx, double *energies_host, int64_t *step);

/* Latest recorded external-force reports, double[n_traj].  Synchronizes. */
sop_status sop_get_external_force(sop_ctx *ctx, double *f_ext_host);

/*
 * The random numbers of Section III.C as the step kernel draws them for step
 * `step`: per residue the four Philox4x32-10 words (key = seed, counter =
 * (index inside the trajectory, stream id, step low word, step high word))
 * into words_host uint32[4*n_res], and the three Box-Muller Gaussians
 * (single precision, widened) into g_host double[3*n_res]; either may be
 * NULL.  Does not advance anything.  Synchronizes.
 */
sop_status sop_sample_noise(sop_ctx *ctx, int64_t step, uint32_t *words_host, double *g_host);

/* ---- force-spectroscopy observables (host arrays; no device work) ----------- */

/*
 * Running average of a recorded force trace (the smoothing of the pulling
 * protocol, Section IV.B): out[k] = (y[k] + ... + y[k+w-1]) / w for
 * k = 0 .. n-w, out has n-w+1 entries.  The windows are differences of
 * double-double prefix sums, so each is accurate to the last bit of a double
 * whatever n.  SOP_E_ARG for null pointers, w < 1 or n < w.
 */
sop_status sop_running_average(const double *y, int64_t n, int32_t w, double *out);

/*
 * Peak (unfolding) force of a trace: the largest w-point running average and
 * the index of its first window (the first of equal maxima).  SOP_E_ARG as
 * above.
 */
sop_status sop_peak_force(const double *f, int64_t n, int32_t w, double *peak, int64_t *index);

/*
 * Temperature from the virial (the paper plots a temperature without
 * defining it; this is the equipartition estimate): for a free chain of
 * n_res residues (no external terms, no fixed residues) the internal virial
 * W = -sum over pairs of r dV/dr averages to -3 (n_res - 1) kB T, so
 * T = -mean(W) / (3 (n_res - 1) kB) over n_records recorded virials.
 * SOP_E_ARG for null pointers, n_records < 1, n_res < 2 or kB <= 0.
 */
sop_status sop_virial_temperature(const double *virial, int64_t n_records, int64_t n_res, double kB,
                                  double *T);

/* ---- accuracy of the integrators (Section IV.C) ------------------------------ */

/*
 * The exactly solvable model the paper uses to measure integrator accuracy:
 * independent Brownian particles X in a one-dimensional harmonic well
 * V = k_sp X^2 / 2, pulled by the force ramp f = rf t, with friction xi
 * (tau = xi / k_sp).  Step k (t_k = k h) moves each particle by
 *   order 1:  c (rf t_k - k_sp X),         c = h / xi,
 *   order 2:  c (rf t_k - k_sp X),         c = (h / xi)(1 - h / (2 tau)),
 * plus sqrt(2 kBT h / xi) g, so that the ensemble mean obeys Eq. 4 (order 1)
 * or Eq. 5 (order 2) exactly and approaches Eq. 3.  g is the first Box-Muller
 * Gaussian of Philox4x32-10 with key = seed and counter = (particle index,
 * stream, k low word, k high word), the same map as sop_sample_noise's axis 0.
 * kBT = 0 runs the noise-free recursions.  The ramp force is formed in double
 * precision, the rest in single precision.
 */
typedef struct sop_ramp_params {
    double rf;          /* ramp rate of the force (force / time) */
    double xi;          /* friction, > 0 */
    double k_sp;        /* spring constant of the well, >= 0 */
    double kBT;         /* thermal energy, >= 0 (0: no noise) */
    double h;           /* time step, > 0 */
    uint64_t seed;      /* Philox key */
    uint32_t stream;    /* second Philox counter word */
    int32_t order;      /* 1 or 2 */
    int32_t compensated;/* 1: X = hi + lo updated by TwoSum; 0: X = hi in plain single precision */
    int32_t pad;
} sop_ramp_params;

/* Device bytes sop_ramp_run needs for the moment reduction of n_particles. */
sop_status sop_ramp_workspace_size(int64_t n_particles, size_t *bytes);

/*
 * Advance n_particles particles from step step0 by n_steps steps, then (when
 * moments is not NULL) write the ensemble mean and population variance of
 * X = hi + lo, summed in double precision in a fixed order, to moments.
 *   x          device float[2*n_particles], {hi, lo} per particle, read and
 *              written in place (lo is ignored and left unchanged when
 *              compensated = 0);
 *   workspace  device scratch of at least sop_ramp_workspace_size bytes,
 *              8-byte aligned, owned by the caller (unused when moments is
 *              NULL);
 *   moments    device double[2] or NULL;
 *   hip_stream the stream to run on (NULL: the default stream).
 * Asynchronous.  SOP_E_ARG for a null rp or x, n_particles outside
 * [1, 2^31 - 1], negative step0 or n_steps, an order other than 1 or 2, or
 * xi <= 0, k_sp < 0, kBT < 0, h <= 0 or a non-finite rf; SOP_E_WORKSPACE for a
 * missing, misaligned or short workspace; SOP_E_HIP for a launch failure.
 */
sop_status sop_ramp_run(const sop_ramp_params *rp, int64_t n_particles, float *x, int64_t step0,
                        int64_t n_steps, void *workspace, size_t workspace_bytes, double *moments,
                        void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid it): sop_ramp_run without a
 * workspace.  The moment reduction's block sums live in a fixed library
 * array of 2 * 1024 doubles (16 KiB) per GPU, held until the process ends;
 * the reduction uses at most 1024 blocks, so every n_particles the call
 * accepts fits.  Same arguments, results and errors as sop_ramp_run (the
 * workspace errors aside); SOP_E_HIP if the array's device address cannot
 * be found.  Calls no allocating routine.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams or host
 * threads) race, so the caller serializes them.
 */
sop_status sop_ramp_run_static(const sop_ramp_params *rp, int64_t n_particles, float *x, int64_t step0,
                               int64_t n_steps, double *moments, void *hip_stream);

/* ---- synchronization and errors ----------------------------------------------- */

/* Wait for the context's stream and return any device-side error. */
sop_status sop_synchronize(sop_ctx *ctx);

const char *sop_status_string(sop_status status);

/* Description of the last failure of this context ("" if none). */
const char *sop_last_error(const sop_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SOP_H */
