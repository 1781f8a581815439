/*
 * genga.h - C ABI of the MI355X (gfx950) kick library.
 *
 * The library implements the data-parallel hot path of a GENGA-style hybrid symplectic
 * N-body step (Brasser, Grimm, Hatalova & Stadel 2023): the all-pairs long-range gravity
 * kick weighted by a changeover function, the close-encounter pair list it produces, the
 * FP64 Kepler drift with a minimal FP64 close-encounter step, and FP64 energy /
 * angular-momentum diagnostics.  One process, one GPU.
 *
 * Conventions that hold for every entry point:
 *  - Units: G = 1.  Positions are heliocentric, velocities barycentric (democratic
 *    heliocentric coordinates).
 *  - Every array argument named in genga_bodies and every output array is a DEVICE
 *    pointer owned by the caller; the library never frees or retains it beyond the call
 *    (calls are asynchronous: the caller keeps the memory alive until the stream has
 *    finished the work).  Host arrays are marked "host".
 *  - Body arrays are structure-of-arrays float64, length n_total, systems stored one after
 *    the other in the order given to genga_set_systems (CSR offsets).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and never
 *    synchronises the host, except genga_set_systems, genga_set_test_bodies,
 *    genga_set_large_groups, genga_set_levels, genga_poll_status, genga_autotune, the graph
 *    calls, and genga_drift / genga_step while large groups are enabled, as documented.  Every launch
 *    sequence is otherwise capturable into a HIP graph (no memset nodes, no host round
 *    trips), except genga_sort_bodies, which refuses capture.
 *  - Return value: GENGA_OK (0) or a negative genga_status.  Errors knowable on the host
 *    (null pointer, bad enum, no layout set) return at once and enqueue nothing.
 *    Conditions found on the device (pair-list overflow, non-finite acceleration,
 *    non-converged Kepler or Bulirsch-Stoer solve) raise flags in the context that
 *    genga_poll_status reports later.  genga_last_error() gives a message for the last
 *    failing call on the calling thread.
 *  - A context is not thread-safe; calls that use one context must not overlap in time
 *    from several host threads.  Calls that share a context must be issued on one stream
 *    (or be ordered by the caller), because they share its scratch buffers.
 */
#ifndef GENGA_H
#define GENGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct genga_ctx genga_ctx;

typedef enum {
    GENGA_OK = 0,
    GENGA_ERR_ARG = -1,         /* invalid argument (host check) */
    GENGA_ERR_HIP = -2,         /* a HIP runtime call failed */
    GENGA_ERR_CAPACITY = -3,    /* encounter list, group or workspace capacity exceeded */
    GENGA_ERR_NONFINITE = -4,   /* a non-finite acceleration was produced */
    GENGA_ERR_NOCONVERGE = -5,  /* Kepler or Bulirsch-Stoer solve did not converge */
    GENGA_ERR_STATE = -6        /* call not valid in the context's state (e.g. no layout) */
} genga_status;

/* Precision of the long-range pair arithmetic (the paper's "Do Kick in single precision"
 * switch, Sect. 4).  FP32: coordinate differences are formed in FP64 and rounded to FP32,
 * the pair term is FP32, partial sums over blocks of 64 sources are FP32 and are folded into
 * an FP64 accumulator.  FP64: everything FP64.  Pairs inside the changeover region are
 * always evaluated in FP64 (Sect. 1: encounter forces are always FP64). */
typedef enum { GENGA_KICK_FP64 = 0, GENGA_KICK_FP32 = 1 } genga_kick_prec;

/* Accumulator of the FP32 kick across blocks of 64 sources (the paper fixes none; the per-body
 * sum is exact enough either way, see the kick below).  FP64: each block's FP32 partial sum is
 * rounded into an FP64 accumulator.  KAHAN32: the partial sums are added into an FP32 sum with
 * Kahan compensation, whose two FP32 words are combined in FP64 at the end.  The FP64 kick
 * ignores the selector. */
typedef enum { GENGA_ACC_FP64 = 0, GENGA_ACC_KAHAN32 = 1 } genga_acc_mode;

/* State of all bodies (device SoA, float64, length n_total). */
typedef struct {
    double *x, *y, *z;      /* heliocentric positions [au] */
    double *vx, *vy, *vz;   /* barycentric velocities [au / (day/k)] */
    const double *m;        /* masses [M_sun] */
    const double *rcrit;    /* critical radius r_crit,i of eq. (1) [au]; constant over a run */
} genga_bodies;

/* Create a context on HIP device `device` (it becomes current on the calling thread for
 * every later call with this context).  *out is NULL on failure. */
int genga_create(genga_ctx **out, int device);

/* Release the context, its scratch memory and any captured graph.  NULL is accepted. */
int genga_destroy(genga_ctx *ctx);

/* Set the system layout: n_sys >= 1 systems, host CSR offsets sys_off_host[n_sys+1]
 * (sys_off_host[0] = 0, non-decreasing, every system non-empty or empty), host central
 * masses mstar_host[n_sys] > 0, and the capacity of the encounter pair list (pairs kept
 * per kick; <= 0 selects 16 * n_total + 1024).  Allocates device scratch sized for the
 * layout, builds the launch plan, and synchronises the device.  Must precede every call
 * below except genga_last_error; may be called again to change the layout. */
int genga_set_systems(genga_ctx *ctx, int32_t n_sys, const int32_t *sys_off_host,
                      const double *mstar_host, int32_t pair_capacity);

/* TP2 mode (Sect. 3.3): in system s the first n_massive_host[s] bodies are massive and the
 * rest are test bodies, which feel and exert forces on the massive bodies but do not
 * interact with each other (no mutual force, no encounter pair, no pair energy).  NULL makes
 * every body massive (the default after genga_set_systems).  Rebuilds the launch plan,
 * synchronises the device and drops any captured graph. */
int genga_set_test_bodies(genga_ctx *ctx, const int32_t *n_massive_host);

/* Encounter groups of more than 64 bodies (the encounter-dominated phase of Sect. 3.5, where
 * with the full eq. (1) the groups can span most of a disc).  enable = 0 (the default): such a
 * group raises GENGA_ERR_CAPACITY and its bodies are only Kepler-drifted.  enable = 1: they
 * are integrated by the same FP64 Bulirsch-Stoer method as the small groups, with the group's
 * state spread over the device; genga_drift and genga_step then synchronise the host with
 * `stream` once per step (to read the group sizes) and once per Bulirsch-Stoer attempt, so
 * graph capture is refused (GENGA_ERR_STATE) while enabled.  Capacity: every body of the
 * layout may be in an encounter group; one group holds at most 65536 bodies.  A larger group
 * makes genga_drift return GENGA_ERR_CAPACITY before it enqueues anything (genga_step: with
 * the bodies left after its last kick).
 * Allocates about 0.6 KB of device memory per body of the layout, resized by
 * genga_set_systems; the switch itself is kept across genga_set_systems.  Synchronises the
 * device. */
int genga_set_large_groups(genga_ctx *ctx, int32_t enable);

/* Hierarchical levels (Sect. 1: intermediate symplectic levels with reduced steps between the
 * level-0 step and the Bulirsch-Stoer step).  n_levels symplectic levels (1..4; 1 = the plain
 * two-level step, the default); level k >= 1 has its own critical radius, host-unowned device
 * array rcrit_levels[(k - 1) * n_total + i] (float64, copied; e.g. genga_rcrit with the
 * level's step dt / n_sub^k), positive and not larger than level k-1's (level 0 is the bodies'
 * rcrit).  The pair force splits as K_0 F + W_1 K_1 F + ... + W_n F with W_l = prod_{k<l}
 * (1 - K_k), K_k the changeover of level k's radius.  Level l integrates each group of level
 * l-1 over its parent's interval in n_sub (1..64) Strang sub-steps: a half kick with W_l K_l F
 * over the group's pairs, the Kepler drift of members in no pair closer than level l's radius
 * and, for each group of such pairs, level l+1 (Bulirsch-Stoer with W_n F after the last
 * level), a half kick.  Needs genga_set_large_groups on (else GENGA_ERR_STATE); genga_drift /
 * genga_step then synchronise the host several times per sub-step.  Reset to 1 by
 * genga_set_systems and by turning large groups off.  Synchronises the device; rcrit_levels
 * may be NULL when n_levels = 1. */
int genga_set_levels(genga_ctx *ctx, int32_t n_levels, int32_t n_sub, const double *rcrit_levels);

/* Self-tuning of the hierarchical levels (Sect. 1: before a run GENGA tries configurations of
 * levels and sub-steps and keeps the fastest).  Tries 1 level, and n_levels = 2..max_levels
 * (<= 4) with n_sub = 2..max_sub (<= 64): for each, level k's radii are eq. (1) with n1, n2
 * and the step dt / n_sub^k from the bodies' current state (b->rcrit stays level 0's), and
 * trial_steps (>= 1) steps of genga_step in precision prec are timed from that state, which is
 * restored afterwards (bit for bit).  A configuration that raises a device condition or a
 * capacity error is not a candidate; collisions (genga_set_collisions) are left out of the
 * trials.  The fastest is set as by genga_set_levels and written to
 * *levels_out / *sub_out (host).  Needs genga_set_large_groups on; allocates and frees about
 * 72 B per body of device memory; synchronises the device. */
int genga_tune_levels(genga_ctx *ctx, genga_bodies *b, double dt, double n1, double n2, int32_t max_levels,
                      int32_t max_sub, int32_t trial_steps, int prec, int32_t *levels_out, int32_t *sub_out,
                      void *stream);

/* Collisions and removal (Sect. 2: collisions are perfect mergers; bodies are removed when
 * they come closer to the star than r_min or farther than r_max).  mass is the device array
 * passed as the bodies' m (the library then writes it: const in genga_bodies notwithstanding);
 * radius (physical radii, au) and status (int32: 0 live, 1 merged into another body, 2 removed
 * by distance) are caller-owned device arrays of n_total entries, written by genga_drift /
 * genga_step.  At the start of each drift, an encounter pair of two live bodies collides when
 * its straight-line relative motion over dt comes within R_i + R_j; after the drift the
 * colliding pairs merge in ascending (i, j) order, a pair with an already merged body skipped:
 * body i keeps m_i + m_j, the mass-weighted position and velocity and radius
 * (R_i^3 + R_j^3)^(1/3); body j gets m = 0 and status 1.  Then live bodies outside
 * [r_min, r_max] get m = 0 and status 2.  Bodies with m = 0 stay in the arrays (they exert no
 * force) until genga_compact.  b->rcrit is the caller's and is left as it is: a merged body
 * keeps its critical radius until the caller recomputes it with genga_rcrit (eq. (1) makes its
 * Hill radius grow as m^(1/3)), e.g. after each step that reports a merger.  At most 4096 colliding pairs per drift (more raise
 * GENGA_ERR_CAPACITY).  mass = NULL turns collisions off.  0 <= r_min < r_max.  The launches
 * stay capturable; refused (GENGA_ERR_STATE) while a captured graph exists.  Synchronises. */
int genga_set_collisions(genga_ctx *ctx, double *mass, double *radius, int32_t *status, double r_min,
                         double r_max);

/* Remove the bodies with status != 0: the bodies' arrays (x..vz, m, rcrit; the library writes
 * them), radius (may be NULL) and status are compacted in place, keeping the order of the
 * survivors, and the context takes the new layout (as genga_set_systems with the same central
 * masses and pair capacity; large groups and collisions stay on, TP2 counts follow the removed
 * massive bodies, hierarchical levels start again at 1).  Writes the new n_total to
 * *n_total_out (host).  Synchronises the device. */
int genga_compact(genga_ctx *ctx, genga_bodies *b, double *radius, int32_t *status, int32_t *n_total_out);

/* Reorder the bodies in space, in place: within each system the massive bodies, then the test
 * bodies, each in order of ring (equal-width bands of distance to the star, as many as make 64
 * consecutive bodies a patch about as wide as long) and azimuth, ties in the present order.
 * The paper fixes no body order; every result is the same up to the rounding order of sums.
 * What the order changes is speed where r_crit spans many neighbours: the kick's candidate
 * pairs then come in dense runs instead of one lane in every wave, and the union-find of the
 * encounter groups converges in fewer rounds.  Keplerian shear spreads each patch along its
 * ring again (in a dense annulus at 0.7-1 au, by about a patch's width in some tens of 5-day
 * steps), so call it every few steps, between genga_step calls.
 * Permuted: the bodies' x..vz, m and rcrit (the library writes m and rcrit: const in
 * genga_bodies notwithstanding), the radius and status arrays of genga_set_collisions (and its
 * mass array when it is not b->m), and the context's copy of the genga_set_levels radii.
 * perm_out (device int32[n_total], may be NULL) receives the old index of the body now at
 * each place, for the caller's own per-body data.  The context's encounter list no longer
 * names these bodies: asking for the last kick's list (genga_encounter_list with b = NULL)
 * then returns GENGA_ERR_STATE, as after a drift.
 * Enqueued on `stream`, no host synchronisation, no allocation (the work buffers come with
 * genga_set_systems); calls that share the context must be ordered after it on that stream.
 * Not capturable: on a stream under graph capture it returns GENGA_ERR_STATE and enqueues
 * nothing (its radix sort clears work memory with memset nodes). */
int genga_sort_bodies(genga_ctx *ctx, genga_bodies *b, int32_t *perm_out, void *stream);

/* Critical radius of every body, eq. (1): r_crit,i = max(n1 R_H,i, n2 dt v_i) with
 * R_H,i = a_i (m_i / 3 Mstar)^(1/3), a_i the osculating semi-major axis of the body's
 * Kepler part (mu = Mstar, or |r_i| for an unbound body) and v_i = sqrt(Mstar/a_i).
 * Reads b->x..b->m (b->rcrit is ignored); writes rc_out[n_total] (device). */
int genga_rcrit(genga_ctx *ctx, const genga_bodies *b, double n1, double n2, double dt,
                double *rc_out, void *stream);

/* Long-range accelerations only (no velocity update), Sect. 1 (the level-0 force of the
 * hybrid step; FP32 pair arithmetic is the "Do Kick in single precision" switch of Sect. 4):
 *   a_i = sum_{j != i, same system} m_j K(r_ij) (r_j - r_i) / r_ij^3
 * with the changeover weight K of Chambers (1999), y = (r - 0.1 r_crit,ij)/(0.9 r_crit,ij),
 * r_crit,ij = max(r_crit,i, r_crit,j).  prec: genga_kick_prec; acc: genga_acc_mode (FP32 only).
 * Writes ax, ay, az [n_total] (device).  Also refreshes the context's encounter list for these
 * positions. */
int genga_accel(genga_ctx *ctx, const genga_bodies *b, double *ax, double *ay, double *az, int prec,
                int acc, void *stream);

/* Largest n that genga_accel_noalloc takes. */
#define GENGA_NOALLOC_MAX_BODIES 65536

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): genga_accel for one system of n bodies, all massive
 * (0 <= n <= GENGA_NOALLOC_MAX_BODIES), with no context and no allocation.  Its scratch (source
 * records, launch plan, split shares; about 8.4 MB) is one static device array per GPU, held
 * until the process ends; its address is looked up on the first call on a device (or by
 * genga_create).  Reads b->x, b->y, b->z, b->m, b->rcrit (device, n entries; b may be NULL when
 * n = 0).  Writes ax, ay, az [n] (device), the encounter pairs (i < j, unordered, as the kick
 * finds them) into pairs[pair_cap][2] (device int32; pairs may be NULL when pair_cap = 0), the
 * full pair count into *d_count and the device conditions into *d_status (device int32 words,
 * both cleared by the call): bit 1 the list did not fit in pair_cap, bit 2 a non-finite
 * acceleration.  The launch shape is the one a context picks by default for the same system,
 * so the results equal genga_accel's bit for bit.  Everything is enqueued on `stream` (no
 * memset, no host wait), so the call can be captured.  All calls on one GPU share the scratch:
 * calls that overlap in time on one GPU (several streams or host threads) race; the caller
 * orders them. */
int genga_accel_noalloc(const genga_bodies *b, int32_t n, double *ax, double *ay, double *az, int32_t *pairs,
                        int32_t pair_cap, int32_t *d_count, int32_t *d_status, int prec, int acc, void *stream);

/* The kick (Sect. 1, level 0): v_i += tau * a_i with a_i as in genga_accel, in the given
 * precision and accumulator.  The same launch records every pair (i < j) with
 * r_ij^2 < r_crit,ij^2 (decided in FP64) into the context's encounter list, which the next
 * genga_drift uses.  With collisions on, pairs with a body of status != 0 are not recorded. */
int genga_kick(genga_ctx *ctx, genga_bodies *b, double tau, int prec, int acc, void *stream);

/* The close-encounter pair list (Sect. 1: the pairs closer than r_crit,ij, whose motion the
 * encounter step integrates; GENGA keeps such a list per level):
 *  - b == NULL: the list of the last genga_kick / genga_accel / genga_step of this context,
 *    which must have run on the current positions (GENGA_ERR_STATE after a genga_drift,
 *    a layout change or before any kick);
 *  - b != NULL: the list for b's positions and r_crit, computed standalone (FP64 decision, no
 *    forces); it also becomes the context's list, which the next genga_drift uses.
 * Writes pairs[cap][2] (device int32, global body indices, i < j, one system), sorted
 * lexicographically, and the list's full length into *d_count (device int32; it may exceed
 * cap, or the context's capacity, in which case the list is incomplete and
 * GENGA_ERR_CAPACITY is also flagged). */
int genga_encounter_list(genga_ctx *ctx, const genga_bodies *b, int32_t *pairs, int32_t cap,
                         int32_t *d_count, void *stream);

/* The drift over dt (Sect. 1): Sun drift dt/2 (r_i += dt/2 * sum_j m_j v_j / Mstar), then the
 * FP64 Kepler drift about Mstar for bodies outside encounter groups and an FP64
 * Bulirsch-Stoer integration over dt of each group (connected component of the encounter
 * list) under the Sun's force plus the (1 - K) share of the members' mutual forces, then Sun
 * drift dt/2.  pairs == NULL: the context's list (that of the last kick or of
 * genga_encounter_list).  Otherwise the caller's list pairs[*d_count][2] (device int32, in any
 * order; d_count a device int32) replaces it: it is checked on the device, and a pair that is
 * not 0 <= i < j < n_total within one system drops the whole list (the drift then treats no
 * body as in an encounter) and makes genga_poll_status report GENGA_ERR_ARG; entries beyond
 * the context's pair capacity are ignored and flagged GENGA_ERR_CAPACITY.  Unless
 * genga_set_large_groups is on, groups larger than 64 bodies or more than 8192 bodies in
 * encounters raise GENGA_ERR_CAPACITY (those bodies are then only Kepler-drifted). */
int genga_drift(genga_ctx *ctx, genga_bodies *b, double dt, const int32_t *pairs, const int32_t *d_count,
                void *stream);

/* Energy and angular momentum per system (Sect. 3.1 diagnostics), FP64:
 *   E = sum m v^2/2 + |sum m v|^2 / (2 Mstar) - sum Mstar m / r - sum_{i<j} m_i m_j / r_ij
 *   L = sum m r x v
 * Writes d_out[n_sys][4] = (E, Lx, Ly, Lz) (device). */
int genga_energy(genga_ctx *ctx, const genga_bodies *b, double *d_out, void *stream);

/* nsteps full steps of the level-0 step of Sect. 1 in democratic heliocentric form,
 * Kick(dt/2) Drift(dt) Kick(dt/2) with the kick and drift above, adjacent half-kicks merged
 * (nsteps + 1 force evaluations).  Velocities are synchronised on entry and exit.  If
 * energy_cadence > 0 and d_energy != NULL, record k (k = 0, 1, ...) of
 * d_energy[nsteps / energy_cadence][n_sys][4] receives (E, Lx, Ly, Lz) of Sect. 3.1 after
 * (k + 1) * energy_cadence steps, for the synchronised velocities (the half-kicked
 * velocities minus dt/2 times the accelerations of the last kick). */
int genga_step(genga_ctx *ctx, genga_bodies *b, double dt, int nsteps, int prec, int acc,
               int energy_cadence, double *d_energy, void *stream);

/* Capture genga_step(ctx, b, dt, nsteps, prec, acc, energy_cadence, d_energy) into a HIP graph
 * held by the context (replacing any earlier one); every replay runs those nsteps steps and
 * rewrites the same d_energy records.  Synchronises `stream` before capture. */
int genga_graph_capture(genga_ctx *ctx, genga_bodies *b, double dt, int nsteps, int prec, int acc,
                        int energy_cadence, double *d_energy, void *stream);

/* Launch the captured graph `repeats` times on `stream`. */
int genga_graph_launch(genga_ctx *ctx, int repeats, void *stream);

/* Time the kick's launch shapes (waves per workgroup x source split) on the current layout
 * and keep the fastest for `prec` (synchronises `stream`; computes accelerations only, the
 * velocities are not changed).  cache_path (host string, may be NULL): a text file of earlier
 * results, one line per (device, precision, layout); a line matching the device's
 * architecture and compute-unit count, prec and the layout's system sizes and TP2 counts is
 * applied without timing, otherwise the shapes are timed and a line is appended (the file is
 * created if missing; a file that cannot be read or written returns GENGA_ERR_ARG, with the
 * timed shape still applied). */
int genga_autotune(genga_ctx *ctx, genga_bodies *b, int prec, const char *cache_path, void *stream);

/* Launch shape of the kick for `prec`: `waves` per workgroup (4, 8 or 16; 0 = default) and
 * `split`, the number of workgroups that share one block of 64 targets' sources (1..4;
 * 0 = chosen from the layout; > 1 adds a small finishing kernel that sums the shares in a
 * fixed order). */
int genga_set_kick_shape(genga_ctx *ctx, int prec, int waves, int split);
int genga_get_kick_shape(genga_ctx *ctx, int prec, int *waves, int *split);

/* Synchronise the stream of the context's last call, then return and clear the deferred
 * device status: GENGA_ERR_ARG (an invalid pair in a caller's list), GENGA_ERR_CAPACITY,
 * GENGA_ERR_NONFINITE, GENGA_ERR_NOCONVERGE or GENGA_OK. */
int genga_poll_status(genga_ctx *ctx);

/* Message for the last failing call on this thread ("" if none).  Owned by the library. */
const char *genga_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GENGA_H */
