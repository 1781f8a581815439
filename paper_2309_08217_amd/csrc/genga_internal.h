// Internal declarations shared by the HIP sources of the kick library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "genga.h"

namespace genga {

// One unit of kick / energy work: up to 64 consecutive bodies (one per lane) of one system,
// all massive or all test bodies.
struct WorkItem {
    int32_t sys;
    int32_t i0;   // first body (global index)
    int32_t ni;   // number of bodies, 1..64
    int32_t nsrc; // sources: the first nsrc bodies of the system (all, or the massive ones
                  // for test-body targets)
};

// Source ("j") records, rebuilt from the SoA state before each kick; 32 bytes so that one
// scalar load brings a whole record into SGPRs for the wave-uniform inner loop.
struct JRec32 {
    double x, y, z;
    float m;
    float pad;
};
struct JRec64 {
    double x, y, z, m;
};

enum DeviceFlag : int32_t {
    FLAG_CAPACITY = 1,
    FLAG_NONFINITE = 2,
    FLAG_NOCONVERGE = 4,   // Bulirsch-Stoer step
    FLAG_KEPLER = 8,       // Kepler solve
    FLAG_BADPAIR = 16,     // a caller's pair list held an invalid pair
};

// Maximum sizes of the close-encounter step (one workgroup builds the groups in LDS).
constexpr int CE_MAX_MEMBERS = 8192;
constexpr int COLLIDE_CAP = 4096;          // colliding pairs per drift
constexpr int CE_MAX_GROUP = 64;
constexpr int BS_KMAX = 8;

// A run of at most CHUNK consecutive bodies of one system: the unit of the O(N) kernels
// (source records, momentum sums, Sun drift), so block reductions never mix systems.
constexpr int CHUNK = 1024;
struct Chunk {
    int32_t sys, b, e, pad;
};

struct Layout {
    int32_t n_sys = 0;
    int32_t n_total = 0;
    int32_t n_chunks = 0;
    int32_t *sys_off = nullptr;     // device [n_sys + 1]
    int32_t *sys_of = nullptr;      // device [n_total], system of each body
    double *mstar = nullptr;        // device [n_sys]
    Chunk *chunks = nullptr;        // device [n_chunks], systems in order
    int32_t *chunk_first = nullptr; // device [n_sys + 1]
    int32_t *n_massive = nullptr;   // device [n_sys]: bodies [off, off + n_massive) are massive
};

struct KickArgs {
    const WorkItem *items;
    int32_t n_items;
    const int32_t *sys_off;
    const double *x, *y, *z;
    double *vx, *vy, *vz;         // updated when update_v != 0
    const double *m, *rc;
    const void *jrec;             // JRec32[] or JRec64[]
    const double *rc2_part;       // [n_chunks] max r_crit^2 per chunk
    const int32_t *chunk_first;   // [n_sys + 1]
    double *ax, *ay, *az;         // a_i out (FP64), always written
    double tau;
    int32_t update_v;
    int32_t *pairs;               // [pair_cap][2]
    int32_t *pair_count;
    int32_t pair_cap;
    int32_t *flags;
    int32_t split;                // workgroups sharing one item's sources (>= 1)
    int32_t n_total;
    double *part;                 // [split][3][n_total] shares when split > 1
    const int32_t *status;        // with collisions: bodies with status != 0 are in no pair
};

constexpr int KICK_MAX_SPLIT = 4;

// Error message for genga_last_error(); returns code.
int fail(int code, const char *fmt, ...);

// Source split that best fills the chip: the kick's workgroups run about one per CU at a
// time, so pick the split whose number of workgroups wastes the least of the last round.
inline int default_kick_split(int n_items, int n_cu)
{
    int best = 1;
    double best_eff = 0.0;
    for (int sp = 1; sp <= KICK_MAX_SPLIT; ++sp) {
        const double tasks = (double)n_items * sp;
        const double rounds = __builtin_ceil(tasks / n_cu);
        const double eff = tasks / (rounds * n_cu);
        if (eff > best_eff + 0.02) {
            best_eff = eff;
            best = sp;
        }
    }
    return best;
}

// Waves per workgroup of the kick before any tuning.
inline int default_kick_waves(int fp32) { return fp32 ? 16 : 8; }

// Address of the allocation-free entry point's scratch array on `device` (looked up once).
int noalloc_prepare(int device, unsigned char **ptr_out, int *n_cu_out);

constexpr int ENERGY_SPLIT = 4;   // workgroups sharing one item's sources in the energy sum

// Kernel launchers (each enqueues on `stream`; return hipError_t of the launch).
// Source records and r_crit^2 maxima for the kick.  With shift_tau != 0 the launch first
// finishes a Sun drift: x += shift_tau P / Mstar per system, P summed from mom_part (the
// per-chunk partials of a preceding launch_momentum).
hipError_t launch_prep(const Layout &L, double *x, double *y, double *z, const double *m,
                       const double *rc, void *jrec, int fp32, double *rc2_part, int32_t *pair_count,
                       const double *mom_part, double shift_tau, hipStream_t stream);
// kahan: the FP32 kick's blocks are summed with Kahan compensation in FP32 (else in FP64)
hipError_t launch_kick(const KickArgs &a, int fp32, int kahan, int waves, int grid, hipStream_t stream);
// The encounter pairs of the state only (FP64 source records from launch_prep; no forces,
// nothing written but a.pairs / a.pair_count), 8 waves per workgroup.
hipError_t launch_pair_list(const KickArgs &a, int grid, hipStream_t stream);
hipError_t launch_rcrit(const Layout &L, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *m,
                        double n1, double n2, double dt, double *rc, hipStream_t stream);
hipError_t launch_sun_drift(const Layout &L, double *x, double *y, double *z, const double *vx,
                            const double *vy, const double *vz, const double *m, double tau,
                            double *mom_part, hipStream_t stream);
// Per-chunk partials of sum m v (the first half of launch_sun_drift).
hipError_t launch_momentum(const Layout &L, const double *vx, const double *vy, const double *vz,
                           const double *m, double *mom_part, hipStream_t stream);

// Momentum of system s for a block of SYS_P_THREADS threads: the chunk partials summed with a
// stride, then a fixed tree, so every block of the system gets the same value.
constexpr int SYS_P_THREADS = 256;
__device__ inline void system_momentum(const int32_t *chunk_first, const double *mom_part, int s,
                                       double (*red)[SYS_P_THREADS / 64], double P[3])
{
    double Px = 0.0, Py = 0.0, Pz = 0.0;
    for (int k = chunk_first[s] + threadIdx.x; k < chunk_first[s + 1]; k += SYS_P_THREADS) {
        Px += mom_part[3 * (size_t)k];
        Py += mom_part[3 * (size_t)k + 1];
        Pz += mom_part[3 * (size_t)k + 2];
    }
    for (int o = 32; o > 0; o >>= 1) {
        Px += __shfl_xor(Px, o, 64);
        Py += __shfl_xor(Py, o, 64);
        Pz += __shfl_xor(Pz, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = Px;
        red[1][threadIdx.x >> 6] = Py;
        red[2][threadIdx.x >> 6] = Pz;
    }
    __syncthreads();
    P[0] = P[1] = P[2] = 0.0;
    for (int w = 0; w < SYS_P_THREADS / 64; ++w)
        for (int q = 0; q < 3; ++q) P[q] += red[q][w];
    __syncthreads();
}
hipError_t launch_ce_groups(const Layout &L, const int32_t *pairs, const int32_t *pair_count,
                            int32_t pair_cap, int32_t *lab, int32_t *mark, int32_t *members,
                            int32_t *group_start, int32_t *n_groups, int32_t *member_slot,
                            int32_t *flags, hipStream_t stream);
// Kepler drift of the bodies outside encounter groups and Bulirsch-Stoer of each group of up
// to CE_MAX_GROUP members (groups of 9 and more in a launch of their own, listed in wg_list:
// [0] their number, then the groups; room for bs_blocks + 1); clears member_slot for the next
// step.  Larger groups
// are flagged (GENGA_ERR_CAPACITY) and Kepler-drifted, or, with big_groups != 0, left alone
// for the grid-wide path below.
// A second stream for the launch of the groups of 9..64 members, forked from and joined back
// into the drift's stream by the two events (default priority; used only while the drift's
// stream is not being captured into a graph, where the two launches stay in sequence).
struct DriftSide {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
hipError_t launch_drift(const Layout &L, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, const double *m, const double *rc, double dt, const int32_t *members,
                        const int32_t *group_start, const int32_t *n_groups, int32_t *member_slot,
                        int32_t *flags, int big_groups, int bs_blocks, int32_t *wg_list, hipStream_t stream,
                        const double *rc_lv = nullptr, int nlev = 1, bool kepler = true,
                        const DriftSide *side = nullptr);
// Grid-wide union-find of the encounter pairs (large-group mode; the host reads lab back):
// init (lab = body for the bodies of a pair), hook rounds (changed |= 1 while a round hooks),
// compress (every member's lab = its root), slots (member_slot for members[0..n), lab = -1).
hipError_t launch_uf_init(const int32_t *pairs, const int32_t *pair_count, int32_t pair_cap, int32_t *lab,
                          hipStream_t stream);
// run_if (device word, may be null): the launch does nothing when *run_if == 0 (the previous
// round changed nothing), so a fixed number of rounds can be enqueued without host waits.
hipError_t launch_uf_hook(const int32_t *pairs, const int32_t *pair_count, int32_t pair_cap, int32_t *lab,
                          int32_t *changed, hipStream_t stream, const int32_t *run_if = nullptr);
hipError_t launch_uf_compress(const Layout &L, int32_t *lab, hipStream_t stream, const int32_t *run_if = nullptr);
hipError_t launch_uf_slots(int n_members_max, const int32_t *members, const int32_t *n_members,
                           int32_t *member_slot, int32_t *lab, hipStream_t stream);

// Grid-wide Bulirsch-Stoer for the groups of more than CE_MAX_GROUP members.  Members of the G
// large groups are numbered f = 0..M-1, group g holding [off[g], off[g+1]) (in an order the
// host chooses: body[f]); state arrays are SoA with stride M.  Capacities (cap_*) follow the
// layout: every body in one group at most; a group spans at most BIG_TILES_PER_GROUP tiles.
struct BigBs {
    int32_t G = 0, M = 0, n_tiles = 0; // host copies of dims[0..2]
    int32_t cap_M = 0, cap_G = 0, cap_T = 0; // allocated members, groups, tiles
    int32_t *dims = nullptr;       // device [4]: G, M, n_tiles (read by the attempt kernels)
    double *dtp = nullptr;         // device [1]: dt of the step
    int32_t *k0 = nullptr;         // [G] first entry of the group in members[]
    int32_t *off = nullptr;        // [G + 1]
    int4 *tiles = nullptr;         // [n_tiles] (group, first member, count, 0): 64 targets
    int32_t *tfirst = nullptr;     // [G + 1] first tile of each group
    double *bb = nullptr;          // [3][cap_T][8] tile boxes of Y, B1, B2
    int32_t *body = nullptr, *grp = nullptr, *test = nullptr; // [M]
    double *rc = nullptr, *mass = nullptr, *i09 = nullptr;    // [M]; i09 = 1 / (0.9 r_crit)
    double *Y = nullptr;           // [3][6][cap_M]: the state, then two sub-step buffers (stride M)
    double *tcol = nullptr;        // [BS_KMAX][6][M]: T(k, 0)
    double *mstar = nullptr, *t = nullptr, *H = nullptr, *rcmax2 = nullptr; // [G]
    int32_t *last = nullptr, *attempts = nullptr, *acc = nullptr, *done = nullptr; // [G]
    unsigned long long *sr = nullptr, *sv = nullptr; // [G] bit patterns of max |r|, max |v|
    unsigned long long *err = nullptr;               // [G][BS_KMAX] bit patterns of the estimates
    int32_t *n_active = nullptr;   // groups not yet at dt after the last attempt
    // hierarchical levels: with nlev > 1 the pair weight is prod_{k<nlev} (1 - K_k), level 0
    // from rc, level k >= 1 from rcl[(k - 1) * cap_M + f]; the candidate radius is the deepest
    // level's.  Fixed when the attempt graph is captured.
    int32_t nlev = 1;
    double *rcl = nullptr;         // [LEVELS_MAX - 1][cap_M]
    // neighbour lists (the list path), built at the start of every attempt (bigbs.hip): member
    // f's sources in BIG_LIST_SEGS segments, nl[f * BIG_LIST_CAP + s * BIG_LIST_SEG + e],
    // e < nlen[f * BIG_LIST_SEGS + s]
    int32_t *nl = nullptr;         // [cap_M][BIG_LIST_CAP]
    int32_t *nlen = nullptr;       // [cap_M][BIG_LIST_SEGS]
    int32_t *ltot = nullptr;       // [cap_M] the list's length
    uint16_t *ll = nullptr;        // [cap_M][BIG_LIST_CAP] the list as one run of slot positions
                                   //   (slot * 64 + position in the slot's source tile)
    int2 *slot = nullptr;          // [cap_T][BIG_LIST_SLOTS] per target tile: the source tiles holding
                                   //   an entry of its members' lists, in tile order, as (first
                                   //   member, members)
    int32_t *nslot = nullptr;      // [cap_T] their number
    double4 *pred = nullptr;       // [cap_M] the star's pull A at the attempt's start and the bound S
    double *skin = nullptr;        // [cap_M] skin factor of each body's bound (indexed by body): 2 at the
                                   //   step's start, times 4 after each crossing
    int32_t *crossed = nullptr;    // [cap_M] the member crossed its bound in the last attempt
    double *a0 = nullptr;          // [3][cap_M] the members' pair sums at the attempt's start state Y
                                   //   (list path: column 0's first sub-step; the later columns reuse them)
    double *amut = nullptr;        // [cap_M] |pair acceleration| at the last attempt's start (column 0's
                                   //   first sub-step, on either path)
    int32_t *stale = nullptr;      // [G] a sub-step crossed a bound: the group's attempt is void
    int32_t *keep = nullptr;       // [G] the group's last attempt was rejected (not void): same start, a
                                   //   shorter step, so its lists and bounds still hold
    double *sbb = nullptr;         // [cap_T][8] box swept over the attempt by a tile, and its largest S
    double *rec = nullptr;         // [3][cap_M][8] per state buffer (Y, B1, B2): a source's words in one
                                   //   64-byte record (x, y, z, mass, r_crit, 1 / (0.9 r_crit), -, -),
                                   //   the sign of 1 / (0.9 r_crit) set for TP2 bodies
    int32_t *ovf = nullptr;        // device word: a list exceeded BIG_LIST_CAP (the host falls back to tiles)
};
constexpr int BIG_TILES_PER_GROUP = 1024; // a workgroup of 1024 threads tests one source tile each
constexpr int BIG_LIST_SEGS = 8;          // segments of a member's list (built by separate waves)
constexpr int BIG_LIST_SEG = 128;         // sources per segment
constexpr int BIG_LIST_CAP = BIG_LIST_SEGS * BIG_LIST_SEG; // sources per member on the list path
constexpr int BIG_LIST_LANES = 8;         // lanes that share one member's list in a sub-step
constexpr int BIG_LIST_SLOTS = 16;        // source tiles a target tile's sub-step stages in LDS
constexpr int LEVELS_MAX = 4;             // symplectic levels of the hierarchical step

// rc_lv: with b.nlev > 1, the critical radii of levels 1..nlev-1 ([nlev - 1][n_total]).
hipError_t launch_big_setup(const Layout &L, const BigBs &b, const int32_t *members, const double *x,
                            const double *y, const double *z, const double *vx, const double *vy,
                            const double *vz, const double *m, const double *rc, const double *rc_lv,
                            double dt, hipStream_t stream);
// One attempt of every active group: a fixed sequence of launches that takes its sizes and dt
// from device memory, so it can be captured once and replayed.
// tile_grid: workgroups of the per-tile launches (they visit the tiles grid-stride); waves: 8
// or 16 per workgroup (the sources of a target tile split over them).
hipError_t launch_big_attempt(const BigBs &b, double tol, int32_t *flags, int tile_grid, int waves,
                              hipStream_t stream);
// The same attempt on the list path: lists built at its start (one wave per target tile), then
// each sub-step sums every member's list (BIG_LIST_LANES lanes per member).
hipError_t launch_big_attempt_list(const BigBs &b, double tol, int32_t *flags, int tile_grid, hipStream_t stream);
hipError_t launch_big_finish(const BigBs &b, double *x, double *y, double *z, double *vx, double *vy,
                             double *vz, hipStream_t stream);
// Members of the parent groups of a hierarchical level, laid out as the grid-wide
// Bulirsch-Stoer lays out its groups: group g holds members [off[g], off[g+1]) (body[f], in an
// order the host chooses), cut into tiles of 64 (group, first member, count, 0).
struct LevelTiles {
    int32_t G = 0, M = 0, n_tiles = 0, cap_M = 0; // sizes (host and kernel arguments)
    int32_t *off = nullptr, *tfirst = nullptr;   // [G + 1]
    int4 *tiles = nullptr;                       // [n_tiles]
    int32_t *body = nullptr, *test = nullptr;    // [M]
    double *X = nullptr, *Y = nullptr, *Z = nullptr, *mass = nullptr; // [M]
    double *rc = nullptr;                        // [LEVELS_MAX][cap_M]: radii of levels 0..
    double *bb = nullptr;                        // [n_tiles][8] tile boxes of X, Y, Z
    double *cut2 = nullptr;                      // [G] largest level-(l-1) radius^2 of the group
    int32_t *tl = nullptr;                       // [n_tiles] tile indices: the n_multi tiles of groups of
    int32_t n_multi = 0;                         //   more than one tile, then one tile per smaller group
};

// Kick of level `level` (1 <= level < nlev) over the members of the parent groups:
// v += tau * sum over the member's group of m_j W_l K_l (r_j - r_i) / r^3 (FP64), and with
// emit the pairs of a group closer than the level's radius (body i < body j) into pairs.
struct LevelKickArgs {
    double *vx = nullptr, *vy = nullptr, *vz = nullptr;
    int32_t level = 1, emit = 0;
    double tau = 0.0;
    int32_t *pairs = nullptr, *pair_count = nullptr, *flags = nullptr;
    int32_t pair_cap = 0;
};
// Constants of the members (mass, TP2 flag, radii of levels 0..level) and each group's cut-off.
hipError_t launch_level_tiles_setup(const Layout &L, const LevelTiles &t, const double *m, const double *rc0,
                                    const double *rcl, int level, hipStream_t stream);
// Gather the members' positions and tile boxes, then kick (waves: 8 or 16 per workgroup of a
// multi-tile group's target tile).  An emitting kick starts its pair count from zero.
hipError_t launch_level_kick(const LevelTiles &t, const LevelKickArgs &a, const double *x, const double *y,
                             const double *z, int waves, hipStream_t stream);
// Kepler drift over dt of the bodies list[0..n-1] (with skip: those with skip[body] < 0; every
// listed skip[body] is then reset to -1).
hipError_t launch_kepler_list(const Layout &L, const int32_t *list, int32_t n, double *x, double *y,
                              double *z, double *vx, double *vy, double *vz, double dt, int32_t *flags,
                              hipStream_t stream, int32_t *skip = nullptr);

// Encounter groups of a level's pair list laid out on the device (groups.hip).  The host reads
// only the header, once per grouping.
constexpr int UF_ROUNDS = 3; // union-find rounds enqueued at once; more only if the last still hooked
struct GroupHeader {
    int32_t G, M;            // groups, members
    int32_t n_tiles, n_multi; // tiles of 64; of them in groups of several tiles
    int32_t max_nb;          // largest group
    int32_t unconverged;     // the last union-find round still hooked: more rounds are needed
    int32_t pair_count;      // length of the pair list (may exceed its capacity)
    int32_t pad;
};
// Where the layout goes: body[M] the members group by group, each group in the parent order;
// off[G + 1]; with tiles != null also tfirst[G + 1], tiles[n_tiles] (group, first member, count,
// 0) in group order, and tl[n_tiles]: the tiles of groups of several tiles first, then the one
// tile of each smaller group.
struct GroupOut {
    int32_t *body = nullptr, *off = nullptr, *tfirst = nullptr, *tl = nullptr;
    int4 *tiles = nullptr;
};
struct GroupWork {
    uint64_t *keys = nullptr, *keys_sorted = nullptr; // [cap]
    int32_t *flag = nullptr, *gidx = nullptr;         // [cap]
    uint64_t *tv = nullptr, *tscan = nullptr;         // [cap / 2 + 2]
    int32_t *changed = nullptr;                       // [UF_ROUNDS]
    GroupHeader *hdr = nullptr;                       // device
    void *temp = nullptr;                             // sort / scan temporary storage
    size_t temp_bytes = 0;
    int cap = 0;                                      // largest parent layout
};
hipError_t group_work_alloc(GroupWork &w, int cap);
// The members of every group of a layout in ring / azimuth order about the star (the order the
// force tiles want: 64 consecutive members close together): per group, equal-width rings of
// distance to the star, as many as make a tile of 64 members about as wide as long, then the
// azimuth; a stable radix sort of the keys (group, quantised ring + azimuth / 4) with the body
// as value.  members[k0[gi] ..] are group gi's bodies, off[gi] its first slot in body_out.
struct OrderWork {
    uint64_t *keys = nullptr, *keys_sorted = nullptr; // [cap]
    int32_t *vals = nullptr;                          // [cap]
    uint64_t *bounds = nullptr;                       // [2 cap]: per group, smallest and largest distance
    void *temp = nullptr;
    size_t temp_bytes = 0;
    int cap = 0;
};
hipError_t order_work_alloc(OrderWork &w, int cap);
void order_work_free(OrderWork &w);
// Per group gi: its members members[k0[gi] ..] (members NULL: the bodies k0[gi], k0[gi] + 1, ..)
// in ring / azimuth order into body_out[off[gi] ..], groups one after the other.  M (the
// layout's size) and n_groups at most the work's capacity.
hipError_t launch_ring_order(const int32_t *members, const int32_t *k0, const int32_t *off, int n_groups, int M,
                             const double *x, const double *y, OrderWork &w, int32_t *body_out, hipStream_t stream);
void group_work_free(GroupWork &w);
// With union_find: union-find of pairs (lab all -1 on entry; afterwards every body of a pair
// holds its component's smallest body, the caller clears it); then the components' members in
// the order of the parent layout pbody[Mp] into `out`, and the header.  Without: the layout of
// the labels as they are (after further rounds by the caller).
hipError_t launch_group_layout(const Layout &L, GroupWork &w, const int32_t *pairs, const int32_t *pair_count,
                               int32_t pair_cap, int32_t *lab, const int32_t *pbody, int Mp, const GroupOut &out,
                               hipStream_t stream, bool union_find);

// Collisions (perfect mergers) and removal by distance: caller-owned mass (the bodies' m),
// radius and status arrays; a list of the colliding pairs of the current drift.
struct CollideArgs {
    double *mass = nullptr, *radius = nullptr;
    int32_t *status = nullptr;   // 0 live, 1 merged into another body, 2 removed by distance
    int32_t *list = nullptr, *count = nullptr, *flags = nullptr;
    int32_t cap = 0;
    double r_min = 0.0, r_max = 0.0;
};
// Colliding encounter pairs at the start of a drift over dt (appended to c.list).
hipError_t launch_collide_check(const CollideArgs &c, const int32_t *pairs, const int32_t *pair_count,
                                int32_t pair_cap, const double *x, const double *y, const double *z,
                                const double *vx, const double *vy, const double *vz, double dt,
                                hipStream_t stream);
// After the drift: merge the listed pairs in order (the count is cleared), then removal.
hipError_t launch_collide_resolve(const CollideArgs &c, int n_total, double *x, double *y, double *z, double *vx,
                                  double *vy, double *vz, hipStream_t stream);

// dst[k] = src[idx[k]], k < n.
hipError_t launch_gather(const int32_t *idx, int n, const double *src, double *dst, hipStream_t stream);
hipError_t launch_gather(const int32_t *idx, int n, const int32_t *src, int32_t *dst, hipStream_t stream);

hipError_t launch_energy(const Layout &L, const WorkItem *items, int32_t n_items, const double *x,
                         const double *y, const double *z, const double *vx, const double *vy,
                         const double *vz, const double *m, const double *ax, const double *ay,
                         const double *az, double vshift, double *partial,
                         const int32_t *item_first, double *out, hipStream_t stream);
// A caller's pair list src[min(*src_count, cap)][2] checked (0 <= i < j < n_total, one system)
// and copied to dst; *dst_count = *src_count, or 0 with FLAG_BADPAIR when a pair is invalid
// (bad: a device word, zero on entry and left zero).
hipError_t launch_import_pairs(const Layout &L, const int32_t *src, const int32_t *src_count, int32_t *dst,
                               int32_t *dst_count, int32_t cap, int32_t *bad, int32_t *flags, hipStream_t stream);
hipError_t launch_sort_pairs(const int32_t *src, const int32_t *src_count, int32_t src_cap,
                             int32_t *dst, int32_t dst_cap, int32_t *dst_count, uint64_t *keys,
                             int32_t *flags, hipStream_t stream);

} // namespace genga
