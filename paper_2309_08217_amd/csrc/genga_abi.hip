// C ABI of the kick library: argument checks, the context (layout, scratch, launch plan,
// deferred device status), the step sequence and HIP graph capture.  Host code.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "genga_internal.h"

using namespace genga;

namespace {
thread_local std::string g_last_error;
} // namespace

int genga::fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

namespace {

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(GENGA_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                  \
    } while (0)

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename T>
hipError_t dalloc(T *&p, size_t count)
{
    dfree(p);
    if (count == 0) count = 1;
    return hipMalloc((void **)&p, count * sizeof(T));
}

} // namespace

struct genga_ctx {
    int device = 0;
    int n_cu = 256;
    char arch[64] = "unknown";      // gcnArchName of the device (autotune cache key)
    Layout L;
    std::vector<int32_t> sys_off_h;
    std::vector<int32_t> n_massive_h; // per system; bodies beyond are TP2 test bodies
    size_t max_items = 0;
    // launch plan
    WorkItem *items = nullptr;  // kick items, largest systems first
    int32_t n_items = 0;
    WorkItem *eitems = nullptr; // energy items, in system order
    int32_t *item_first = nullptr;
    int waves[2] = {default_kick_waves(0), default_kick_waves(1)}; // [prec] waves per workgroup of the kick
    int grid[2] = {0, 0};       // 0: one workgroup per task
    int split[2] = {1, 1};      // [prec] workgroups sharing an item's sources
    double *kpart = nullptr;    // [KICK_MAX_SPLIT][3][n_total]
    // scratch
    uint8_t *jrec = nullptr;    // 32 B per body
    double *rc2_part = nullptr;   // [n_chunks]
    double *mom_part = nullptr;   // [n_chunks][3]
    double *acc = nullptr;      // a_i of the last kick: [3][n_total]
    int32_t *pairs = nullptr;
    int32_t *pair_count = nullptr;
    int32_t pair_cap = 0;
    uint64_t *sort_keys = nullptr;
    int32_t *flags = nullptr;
    int32_t *lab = nullptr, *mark = nullptr, *members = nullptr, *group_start = nullptr;
    int32_t *n_groups = nullptr, *member_slot = nullptr;
    int32_t *wg_list = nullptr; // groups of 9..64 members of a drift (their count first)
    double *epartial = nullptr;
    // grid-wide Bulirsch-Stoer for groups of more than CE_MAX_GROUP members (opt-in)
    int32_t large_groups = 0;
    BigBs big;
    int32_t *pin = nullptr;            // pinned host words for the per-attempt status reads
    hipStream_t big_stream = nullptr;  // private stream to capture one attempt
    DriftSide side;                    // the drift's second stream (groups of 9..64 members)
    // the captured attempt, replayed on the caller's stream: one per tile-launch grid (a power
    // of two that covers the layout's tiles)
    hipGraphExec_t big_exec[32] = {};
    hipGraphExec_t big_exec_list[32] = {}; // the same on the list path
    int32_t *big_changed = nullptr;    // device word of the union-find rounds
    int32_t ce_cap = 0;                // members / group_start capacity
    std::vector<int32_t> gs_h;         // group_start copied to the host
    // host scratch of the grouping and tile ordering, kept so that the per-call vectors of
    // n_total entries are not allocated (and faulted in) again on every call
    OrderWork ow;                      // the device ring / azimuth ordering of the large groups
    // genga_sort_bodies: its ordering work, the bounds of the sorted runs (the massive and the
    // test bodies of each system: 2 n_sys + 1 offsets) and the permutation
    OrderWork sw;
    int32_t *sort_seg = nullptr, *sort_perm = nullptr;
    // hierarchical levels (with the large-group mode): levels 1..n_levels-1 and their radii
    int32_t n_levels = 1, n_sub = 1;
    double *rc_lv = nullptr;           // [n_levels - 1][n_total]
    LevelTiles lt[LEVELS_MAX - 1];     // parent groups of levels 1..n_levels-1, in tiles
    int32_t lt_cap_G = 0, lt_cap_T = 0;
    int32_t *lv_mem = nullptr, *lv_gs = nullptr, *lv_ng = nullptr; // the deepest level's groups
    int32_t *lv_pairs = nullptr, *lv_count = nullptr; // a level's pairs
    GroupWork gw;                      // device layout of a level's groups
    GroupHeader *ghdr = nullptr;       // pinned host copy of its header
    int32_t *iota = nullptr;           // [n_total] 0, 1, ..: the body order, level 0's parent layout
    // collisions and removal (opt-in)
    CollideArgs col;
    int32_t pair_cap_req = 0;          // pair capacity asked for at genga_set_systems
    std::vector<double> mstar_h;       // central masses (host copy)
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // the context's encounter list belongs to the current positions (a kick or a standalone
    // list ran on them, no drift since)
    bool list_valid = false;
    int32_t *import_bad = nullptr;     // device word of the pair-list import
    hipStream_t last_stream = nullptr; // stream of the last enqueuing call (genga_poll_status)
    int32_t *hpin = nullptr;           // pinned host word for genga_poll_status

    void release_big()
    {
        order_work_free(ow);
        dfree(iota);
        dfree(big.k0);
        dfree(big.off);
        dfree(big.tiles);
        dfree(big.tfirst);
        dfree(big.bb);
        dfree(big.body);
        dfree(big.grp);
        dfree(big.test);
        dfree(big.rc);
        dfree(big.mass);
        dfree(big.i09);
        dfree(big.Y);
        dfree(big.tcol);
        dfree(big.mstar);
        dfree(big.t);
        dfree(big.H);
        dfree(big.rcmax2);
        dfree(big.last);
        dfree(big.attempts);
        dfree(big.acc);
        dfree(big.done);
        dfree(big.sr);
        dfree(big.sv);
        dfree(big.err);
        dfree(big.n_active);
        dfree(big.rcl);
        dfree(big.nl);
        dfree(big.nlen);
        dfree(big.ltot);
        dfree(big.a0);
        dfree(big.ll);
        dfree(big.slot);
        dfree(big.nslot);
        dfree(big.pred);
        dfree(big.skin);
        dfree(big.crossed);
        dfree(big.amut);
        dfree(big.stale);
        dfree(big.keep);
        dfree(big.sbb);
        dfree(big.rec);
        dfree(big.ovf);
        big.nlev = 1;
        dfree(rc_lv);
        for (auto &t : lt) {
            dfree(t.off);
            dfree(t.tfirst);
            dfree(t.tiles);
            dfree(t.body);
            dfree(t.test);
            dfree(t.X);
            dfree(t.Y);
            dfree(t.Z);
            dfree(t.mass);
            dfree(t.rc);
            dfree(t.bb);
            dfree(t.cut2);
            dfree(t.tl);
            t.G = t.M = t.n_tiles = t.cap_M = t.n_multi = 0;
        }
        dfree(lv_mem);
        dfree(lv_gs);
        dfree(lv_ng);
        group_work_free(gw);
        dfree(lv_pairs);
        dfree(lv_count);
        n_levels = n_sub = 1;
        if (pin) (void)hipHostFree(pin);
        for (auto &e : big_exec)
            if (e) (void)hipGraphExecDestroy(e);
        for (auto &e : big_exec_list)
            if (e) (void)hipGraphExecDestroy(e);
        if (big_stream) (void)hipStreamDestroy(big_stream);
        for (auto &e : big_exec) e = nullptr;
        for (auto &e : big_exec_list) e = nullptr;
        big_stream = nullptr;
        dfree(big.dims);
        dfree(big.dtp);
        dfree(big_changed);
        pin = nullptr;
        big.G = big.M = big.n_tiles = 0;
        large_groups = 0;
    }

    void release()
    {
        if (side.stream) (void)hipStreamDestroy(side.stream);
        if (side.fork) (void)hipEventDestroy(side.fork);
        if (side.join) (void)hipEventDestroy(side.join);
        side = DriftSide();
        dfree(L.sys_off);
        dfree(L.sys_of);
        dfree(L.mstar);
        dfree(items);
        dfree(eitems);
        dfree(item_first);
        dfree(jrec);
        dfree(rc2_part);
        dfree(mom_part);
        dfree(L.chunks);
        dfree(L.chunk_first);
        dfree(L.n_massive);
        dfree(acc);
        dfree(pairs);
        dfree(pair_count);
        dfree(sort_keys);
        dfree(flags);
        dfree(lab);
        dfree(mark);
        dfree(members);
        dfree(group_start);
        dfree(n_groups);
        dfree(member_slot);
        dfree(wg_list);
        dfree(epartial);
        dfree(kpart);
        dfree(import_bad);
        order_work_free(sw);
        dfree(sort_seg);
        dfree(sort_perm);
        list_valid = false;
        dfree(col.list);
        dfree(col.count);
        col = CollideArgs{};
        release_big();
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        L.n_sys = L.n_total = L.n_chunks = 0;
        n_items = 0;
    }
};

namespace {

int check_ctx(genga_ctx *ctx, bool need_layout = true)
{
    if (!ctx) return fail(GENGA_ERR_ARG, "null context");
    if (need_layout && ctx->L.n_sys <= 0) return fail(GENGA_ERR_STATE, "no layout: call genga_set_systems first");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(GENGA_ERR_HIP, "hipSetDevice(%d) failed", ctx->device);
    return GENGA_OK;
}

int check_bodies(const genga_ctx *ctx, const genga_bodies *b, bool need_v, bool need_rc)
{
    if (!b) return fail(GENGA_ERR_ARG, "null bodies");
    if (ctx->L.n_total == 0) return GENGA_OK;
    if (!b->x || !b->y || !b->z || !b->m) return fail(GENGA_ERR_ARG, "null position or mass array");
    if (need_v && (!b->vx || !b->vy || !b->vz)) return fail(GENGA_ERR_ARG, "null velocity array");
    if (need_rc && !b->rcrit) return fail(GENGA_ERR_ARG, "null rcrit array");
    return GENGA_OK;
}

int default_split(const genga_ctx *ctx)
{
    return default_kick_split(ctx->n_items, ctx->n_cu);
}

int check_prec(int prec)
{
    if (prec != GENGA_KICK_FP32 && prec != GENGA_KICK_FP64) return fail(GENGA_ERR_ARG, "bad precision %d", prec);
    return GENGA_OK;
}

int check_acc(int acc)
{
    if (acc != GENGA_ACC_FP64 && acc != GENGA_ACC_KAHAN32) return fail(GENGA_ERR_ARG, "bad accumulator %d", acc);
    return GENGA_OK;
}

// shift_tau != 0: the source-record pass first applies the pending second half of a Sun drift
// (see enqueue_drift with defer_shift)
int enqueue_kick(genga_ctx *ctx, const genga_bodies *b, double tau, int update_v, int prec, int acc, double *ax,
                 double *ay, double *az, hipStream_t s, double shift_tau = 0.0)
{
    const Layout &L = ctx->L;
    ctx->list_valid = true;
    if (L.n_total == 0) return GENGA_OK;
    const int fp32 = prec == GENGA_KICK_FP32;
    HIP_TRY(launch_prep(L, b->x, b->y, b->z, b->m, b->rcrit, ctx->jrec, fp32, ctx->rc2_part, ctx->pair_count,
                        ctx->mom_part, shift_tau, s));
    KickArgs a{};
    a.items = ctx->items;
    a.n_items = ctx->n_items;
    a.sys_off = L.sys_off;
    a.x = b->x;
    a.y = b->y;
    a.z = b->z;
    a.vx = b->vx;
    a.vy = b->vy;
    a.vz = b->vz;
    a.m = b->m;
    a.rc = b->rcrit;
    a.jrec = ctx->jrec;
    a.rc2_part = ctx->rc2_part;
    a.chunk_first = L.chunk_first;
    a.ax = ax;
    a.ay = ay;
    a.az = az;
    a.tau = tau;
    a.update_v = update_v;
    a.pairs = ctx->pairs;
    a.pair_count = ctx->pair_count;
    a.pair_cap = ctx->pair_cap;
    a.flags = ctx->flags;
    a.split = ctx->split[fp32];
    a.n_total = L.n_total;
    a.part = ctx->kpart;
    a.status = ctx->col.mass ? ctx->col.status : nullptr;
    HIP_TRY(launch_kick(a, fp32, acc == GENGA_ACC_KAHAN32, ctx->waves[fp32], ctx->grid[fp32], s));
    return GENGA_OK;
}

// The encounter list of b's positions alone (FP64 decision, no forces) into the context's list.
int enqueue_pair_list(genga_ctx *ctx, const genga_bodies *b, hipStream_t s)
{
    const Layout &L = ctx->L;
    ctx->list_valid = true;
    if (L.n_total == 0) {
        HIP_TRY(hipMemsetAsync(ctx->pair_count, 0, sizeof(int32_t), s));
        return GENGA_OK;
    }
    HIP_TRY(launch_prep(L, b->x, b->y, b->z, b->m, b->rcrit, ctx->jrec, 0, ctx->rc2_part, ctx->pair_count, nullptr,
                        0.0, s));
    KickArgs a{};
    a.items = ctx->items;
    a.n_items = ctx->n_items;
    a.sys_off = L.sys_off;
    a.x = b->x;
    a.y = b->y;
    a.z = b->z;
    a.m = b->m;
    a.rc = b->rcrit;
    a.jrec = ctx->jrec;
    a.rc2_part = ctx->rc2_part;
    a.chunk_first = L.chunk_first;
    a.pairs = ctx->pairs;
    a.pair_count = ctx->pair_count;
    a.pair_cap = ctx->pair_cap;
    a.flags = ctx->flags;
    a.split = 1;
    a.n_total = L.n_total;
    a.status = ctx->col.mass ? ctx->col.status : nullptr;
    HIP_TRY(launch_pair_list(a, 0, s));
    return GENGA_OK;
}

int run_big_groups(genga_ctx *ctx, genga_bodies *b, double dt, hipStream_t s, const std::vector<int32_t> &gs,
                   const std::vector<int32_t> &mem_h, const int32_t *members_dev, int min_nb,
                   const std::vector<int32_t> *prev = nullptr);
int build_groups_large(genga_ctx *ctx, hipStream_t s);
int run_levels(genga_ctx *ctx, genga_bodies *b, double dt, hipStream_t s);

// Sun drift (dt/2), Kepler / Bulirsch-Stoer (dt), Sun drift (dt/2).  With defer_shift the
// last position shift is left to the next kick's source-record pass (only the momentum
// partials are formed here); that kick must be given shift_tau = dt/2.

// The drift's second stream and its events, made on first use outside graph capture; nullptr
// while `s` is being captured or if making them fails (the drift's launches then stay on one
// stream, with the same results).
const DriftSide *drift_side(genga_ctx *ctx, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    DriftSide &d = ctx->side;
    if (!d.stream) {
        if (hipStreamCreateWithFlags(&d.stream, hipStreamNonBlocking) != hipSuccess) d.stream = nullptr;
        if (d.stream && (hipEventCreateWithFlags(&d.fork, hipEventDisableTiming) != hipSuccess ||
                         hipEventCreateWithFlags(&d.join, hipEventDisableTiming) != hipSuccess)) {
            if (d.fork) (void)hipEventDestroy(d.fork);
            (void)hipStreamDestroy(d.stream);
            d = DriftSide();
        }
    }
    return d.stream ? &d : nullptr;
}

int enqueue_drift(genga_ctx *ctx, genga_bodies *b, double dt, hipStream_t s, bool defer_shift = false)
{
    const Layout &L = ctx->L;
    ctx->list_valid = false;
    if (L.n_total == 0) return GENGA_OK;
    const bool collide = ctx->col.mass != nullptr;
    if (collide) {
        if (b->m != ctx->col.mass)
            return fail(GENGA_ERR_ARG, "with collisions on, the bodies' m must be the mass array given to "
                                       "genga_set_collisions");
        if (defer_shift) return fail(GENGA_ERR_STATE, "collisions need the whole Sun drift inside the drift");
        // colliding encounter pairs, from the state at the start of the drift
        HIP_TRY(launch_collide_check(ctx->col, ctx->pairs, ctx->pair_count, ctx->pair_cap, b->x, b->y, b->z, b->vx,
                                     b->vy, b->vz, dt, s));
    }
    int bs_blocks = 0; // default: the one-workgroup group builder's maximum
    if (ctx->large_groups) {
        // the groups depend on the pair list only; built first, so that a group too large
        // for the grid-wide path is refused before any part of the drift is enqueued
        const int rc = build_groups_large(ctx, s);
        if (rc) return rc;
        // with levels every group is integrated by the level steps: Kepler blocks only
        bs_blocks = ctx->n_levels > 1 ? -1 : std::max(1, (int)ctx->gs_h.size() - 1);
    }
    HIP_TRY(launch_sun_drift(L, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, 0.5 * dt, ctx->mom_part, s));
    if (!ctx->large_groups) {
        HIP_TRY(launch_ce_groups(L, ctx->pairs, ctx->pair_count, ctx->pair_cap, ctx->lab, ctx->mark, ctx->members,
                                 ctx->group_start, ctx->n_groups, ctx->member_slot, ctx->flags, s));
    }
    HIP_TRY(launch_drift(L, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, b->rcrit, dt, ctx->members,
                         ctx->group_start, ctx->n_groups, ctx->member_slot, ctx->flags, ctx->large_groups,
                         bs_blocks, ctx->wg_list, s, nullptr, 1, true, drift_side(ctx, s)));
    if (ctx->n_levels > 1) {
        const int rc = run_levels(ctx, b, dt, s);
        if (rc) return rc;
    } else if (ctx->large_groups) {
        const int rc = run_big_groups(ctx, b, dt, s, ctx->gs_h, {}, ctx->members, CE_MAX_GROUP + 1);
        if (rc) return rc;
    }
    if (defer_shift)
        HIP_TRY(launch_momentum(L, b->vx, b->vy, b->vz, b->m, ctx->mom_part, s));
    else
        HIP_TRY(launch_sun_drift(L, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, 0.5 * dt, ctx->mom_part, s));
    if (collide) HIP_TRY(launch_collide_resolve(ctx->col, L.n_total, b->x, b->y, b->z, b->vx, b->vy, b->vz, s));
    return GENGA_OK;
}

int alloc_big(genga_ctx *ctx)
{
    BigBs &b = ctx->big;
    // every body may be in one large group; groups above CE_MAX_GROUP members (with levels:
    // the deepest level's groups of any size, at least 2 members each)
    const bool lvl = ctx->n_levels > 1;
    b.cap_M = std::max(ctx->L.n_total, 2);
    b.cap_G = lvl ? b.cap_M / 2 + 1 : b.cap_M / (CE_MAX_GROUP + 1) + 1;
    b.cap_T = b.cap_M / 64 + b.cap_G + 1;
    b.nlev = ctx->n_levels;
    if (lvl) {
        const size_t nt = (size_t)std::max(ctx->L.n_total, 1);
        HIP_TRY(dalloc(b.rcl, (size_t)(LEVELS_MAX - 1) * b.cap_M));
        HIP_TRY(dalloc(ctx->rc_lv, (size_t)(LEVELS_MAX - 1) * nt));
        ctx->lt_cap_G = (int32_t)nt / 2 + 1;
        ctx->lt_cap_T = (int32_t)nt / 64 + ctx->lt_cap_G + 1;
        const size_t G = (size_t)ctx->lt_cap_G, T = (size_t)ctx->lt_cap_T;
        for (auto &t : ctx->lt) {
            t.cap_M = (int32_t)nt;
            HIP_TRY(dalloc(t.off, G + 1));
            HIP_TRY(dalloc(t.tfirst, G + 1));
            HIP_TRY(dalloc(t.tiles, T));
            HIP_TRY(dalloc(t.body, nt));
            HIP_TRY(dalloc(t.test, nt));
            HIP_TRY(dalloc(t.X, nt));
            HIP_TRY(dalloc(t.Y, nt));
            HIP_TRY(dalloc(t.Z, nt));
            HIP_TRY(dalloc(t.mass, nt));
            HIP_TRY(dalloc(t.rc, (size_t)LEVELS_MAX * nt));
            HIP_TRY(dalloc(t.bb, 8 * T));
            HIP_TRY(dalloc(t.cut2, G));
            HIP_TRY(dalloc(t.tl, T));
        }
        HIP_TRY(dalloc(ctx->lv_mem, nt));
        HIP_TRY(dalloc(ctx->lv_gs, nt + 1));
        HIP_TRY(dalloc(ctx->lv_ng, 1));
        HIP_TRY(dalloc(ctx->lv_pairs, 2 * (size_t)ctx->pair_cap));
        HIP_TRY(dalloc(ctx->lv_count, 1));
    }
    {
        // the groupings on the device (level 0's in body order, the levels' in their parent's)
        const size_t nt = (size_t)std::max(ctx->L.n_total, 1);
        HIP_TRY(group_work_alloc(ctx->gw, (int)nt));
        if (!ctx->ghdr) HIP_TRY(hipHostMalloc((void **)&ctx->ghdr, sizeof(GroupHeader), hipHostMallocDefault));
        std::vector<int32_t> id(nt);
        for (size_t i = 0; i < nt; ++i) id[i] = (int32_t)i;
        HIP_TRY(dalloc(ctx->iota, nt));
        HIP_TRY(hipMemcpy(ctx->iota, id.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    const size_t M = (size_t)b.cap_M, G = (size_t)b.cap_G;
    HIP_TRY(dalloc(b.k0, G));
    HIP_TRY(order_work_alloc(ctx->ow, (int)std::max(M, G)));
    HIP_TRY(dalloc(b.off, G + 1));
    HIP_TRY(dalloc(b.tiles, (size_t)b.cap_T));
    HIP_TRY(dalloc(b.tfirst, G + 1));
    HIP_TRY(dalloc(b.bb, 3 * 8 * (size_t)b.cap_T));
    HIP_TRY(dalloc(b.body, M));
    HIP_TRY(dalloc(b.grp, M));
    HIP_TRY(dalloc(b.test, M));
    HIP_TRY(dalloc(b.rc, M));
    HIP_TRY(dalloc(b.mass, M));
    HIP_TRY(dalloc(b.i09, M));
    HIP_TRY(dalloc(b.Y, 3 * 6 * M));
    HIP_TRY(dalloc(b.tcol, (size_t)BS_KMAX * 6 * M));
    HIP_TRY(dalloc(b.mstar, G));
    HIP_TRY(dalloc(b.t, G));
    HIP_TRY(dalloc(b.H, G));
    HIP_TRY(dalloc(b.rcmax2, G));
    HIP_TRY(dalloc(b.last, G));
    HIP_TRY(dalloc(b.attempts, G));
    HIP_TRY(dalloc(b.acc, G));
    HIP_TRY(dalloc(b.done, G));
    HIP_TRY(dalloc(b.sr, G));
    HIP_TRY(dalloc(b.sv, G));
    HIP_TRY(dalloc(b.err, G * BS_KMAX));
    HIP_TRY(dalloc(b.n_active, 1));
    HIP_TRY(dalloc(b.nl, M * BIG_LIST_CAP));
    HIP_TRY(dalloc(b.nlen, M * BIG_LIST_SEGS));
    HIP_TRY(dalloc(b.ltot, M));
    HIP_TRY(dalloc(b.a0, 3 * (size_t)M));
    HIP_TRY(dalloc(b.ll, M * BIG_LIST_CAP));
    HIP_TRY(dalloc(b.slot, (size_t)b.cap_T * BIG_LIST_SLOTS));
    HIP_TRY(dalloc(b.nslot, (size_t)b.cap_T));
    HIP_TRY(dalloc(b.pred, M));
    HIP_TRY(dalloc(b.skin, M));
    HIP_TRY(dalloc(b.crossed, M));
    HIP_TRY(dalloc(b.amut, M));
    HIP_TRY(hipMemset(b.skin, 0, M * sizeof(double)));
    HIP_TRY(hipMemset(b.crossed, 0, M * sizeof(int32_t)));
    HIP_TRY(dalloc(b.stale, G));
    HIP_TRY(dalloc(b.keep, G));
    HIP_TRY(hipMemset(b.keep, 0, G * sizeof(int32_t)));
    HIP_TRY(dalloc(b.sbb, 8 * (size_t)b.cap_T));
    HIP_TRY(dalloc(b.rec, 3 * 8 * (size_t)M));
    HIP_TRY(dalloc(b.ovf, 1));
    HIP_TRY(hipMemset(b.ovf, 0, sizeof(int32_t)));
    HIP_TRY(hipMemset(b.stale, 0, G * sizeof(int32_t)));
    HIP_TRY(dalloc(b.dims, 4));
    HIP_TRY(dalloc(b.dtp, 1));
    HIP_TRY(dalloc(ctx->big_changed, 1));
    if (!ctx->pin) HIP_TRY(hipHostMalloc((void **)&ctx->pin, 4 * sizeof(int32_t), hipHostMallocDefault));
    return GENGA_OK;
}

// The encounter groups of the context's pair list, for the large-group mode: members /
// group_start / n_groups on the device, member_slot set for the drift launch.
int build_groups_large(genga_ctx *ctx, hipStream_t s)
{
    // the components of the pair list laid out on the device in body order (groups by their
    // smallest member, members ascending), and the header and group offsets read in one wait
    const Layout &L = ctx->L;
    const int nt = L.n_total;
    GroupOut out;
    out.body = ctx->members;
    out.off = ctx->group_start;
    const size_t ngs = (size_t)nt / 2 + 2; // groups have at least two members
    std::vector<int32_t> &gs = ctx->gs_h;
    const auto layout = [&](bool union_find) -> int {
        HIP_TRY(launch_group_layout(L, ctx->gw, ctx->pairs, ctx->pair_count, ctx->pair_cap, ctx->lab, ctx->iota, nt,
                                    out, s, union_find));
        gs.resize(ngs);
        HIP_TRY(hipMemcpyAsync(ctx->ghdr, ctx->gw.hdr, sizeof(GroupHeader), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(gs.data(), ctx->group_start, ngs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return GENGA_OK;
    };
    int rc = layout(true);
    if (rc) return rc;
    // a union-find not settled within the enqueued rounds: checked rounds, then the layout again
    for (int round = 0; ctx->ghdr->unconverged; ++round) {
        if (round > 4096) return fail(GENGA_ERR_STATE, "union-find of the encounter pairs did not settle");
        ctx->pin[2] = 0;
        HIP_TRY(hipMemcpyAsync(ctx->big_changed, ctx->pin + 2, sizeof(int32_t), hipMemcpyHostToDevice, s));
        for (int rep = 0; rep < 2; ++rep) {
            HIP_TRY(launch_uf_hook(ctx->pairs, ctx->pair_count, ctx->pair_cap, ctx->lab, ctx->big_changed, s));
            HIP_TRY(launch_uf_compress(L, ctx->lab, s));
        }
        HIP_TRY(hipMemcpyAsync(ctx->pin + 2, ctx->big_changed, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (ctx->pin[2] == 0 && (rc = layout(false))) return rc;
    }
    const GroupHeader h = *ctx->ghdr;
    if (h.max_nb > 64 * BIG_TILES_PER_GROUP) {
        if (nt > 0) (void)hipMemsetAsync(ctx->lab, 0xff, (size_t)nt * sizeof(int32_t), s);
        gs.assign(1, 0);
        return fail(GENGA_ERR_CAPACITY, "an encounter group of %d bodies (at most %d)", h.max_nb,
                    64 * BIG_TILES_PER_GROUP);
    }
    gs.resize((size_t)h.G + 1);
    // the drift's group count and the members' slots (their labels back to -1)
    HIP_TRY(hipMemcpyAsync(ctx->n_groups, &ctx->gw.hdr->G, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_uf_slots(nt, ctx->members, &ctx->gw.hdr->M, ctx->member_slot, ctx->lab, s));
    return GENGA_OK;
}
// The groups of gs / mem with at least min_nb members, cut into tiles of 64, each group's
// members ordered so that 64 consecutive ones are close together and force tiles can skip
// distant tiles.  With prev (an order of bodies that contains every member, e.g. the parent
// level's): in that order, which keeps its locality, into o.body.  Without: o.body is left
// empty and the caller orders the members on the device (launch_ring_order: rings of distance
// to the star, then azimuth).
struct TileOrder {
    std::vector<int32_t> k0, off{0}, tfirst{0}, body;
    std::vector<int4> tiles;
};

int order_tiles(genga_ctx *ctx, const std::vector<int32_t> &gs, const std::vector<int32_t> &mem, int min_nb,
                TileOrder &o, const std::vector<int32_t> *prev = nullptr)
{
    const int ng = (int)gs.size() - 1;
    for (int g = 0; g < ng; ++g) {
        const int nb = gs[g + 1] - gs[g];
        if (nb < min_nb) continue;
        const int gi = (int)o.k0.size(), f0 = o.off.back();
        o.k0.push_back(gs[g]);
        o.off.push_back(f0 + nb);
        for (int f = 0; f < nb; f += 64) o.tiles.push_back(make_int4(gi, f0 + f, std::min(64, nb - f), 0));
        o.tfirst.push_back((int32_t)o.tiles.size());
    }
    for (size_t gi = 0; gi + 1 < o.tfirst.size(); ++gi)
        if (o.tfirst[gi + 1] - o.tfirst[gi] > BIG_TILES_PER_GROUP)
            return fail(GENGA_ERR_CAPACITY, "an encounter group of more than %d bodies", 64 * BIG_TILES_PER_GROUP);
    if (o.k0.empty() || !prev) return GENGA_OK;
    const size_t nt = (size_t)ctx->L.n_total;
    o.body.resize((size_t)o.off.back());
    {
        std::vector<int32_t> grp(nt, -1), fill(o.k0.size());
        for (size_t gi = 0; gi < o.k0.size(); ++gi) {
            for (int l = 0; l < o.off[gi + 1] - o.off[gi]; ++l) grp[mem[o.k0[gi] + l]] = (int32_t)gi;
            fill[gi] = o.off[gi];
        }
        for (int32_t bi : *prev)
            if (grp[bi] >= 0) o.body[fill[grp[bi]]++] = bi;
        for (size_t gi = 0; gi < o.k0.size(); ++gi)
            if (fill[gi] != o.off[gi + 1]) return fail(GENGA_ERR_STATE, "tile order misses group members");
    }
    return GENGA_OK;
}

// ------------------------------------------------------------------------------------------
// Hierarchical levels (Sect. 1): level l integrates each group of level l-1 over tau in n_sub
// Strang sub-steps of h = tau / n_sub: kick(h/2) with the level-l share of the pair forces
// (which also lists the level-l pairs), the groups of those pairs, Kepler drift(h) for the
// parent members outside them, level l+1 (Bulirsch-Stoer after the last level) for each,
// kick(h/2).  The host drives the recursion; it reads each level's pair count and labels.
// ------------------------------------------------------------------------------------------
int level_kick(genga_ctx *ctx, genga_bodies *b, int level, const LevelTiles &T, double tau, bool emit,
               hipStream_t s)
{
    LevelKickArgs a;
    a.vx = b->vx;
    a.vy = b->vy;
    a.vz = b->vz;
    a.level = level;
    a.emit = emit ? 1 : 0;
    a.tau = tau;
    a.pairs = ctx->lv_pairs;
    a.pair_count = ctx->lv_count;
    a.flags = ctx->flags;
    a.pair_cap = ctx->pair_cap;
    // 16 waves per target tile while the tiles fit one workgroup per CU, else 8 (several per CU)
    HIP_TRY(launch_level_kick(T, a, b->x, b->y, b->z, T.n_multi <= ctx->n_cu ? 16 : 8, s));
    return GENGA_OK;
}

// The groups of the level-`level` pairs (ctx->lv_pairs), laid out on the device in the order of
// the parent layout T (members of each group in T's order): into the child level's tiles, or,
// for the deepest level, into lv_mem / lv_gs.  One host wait, for the header.  A union-find
// that has not settled within the enqueued rounds is finished with checked rounds (one wait
// each) and laid out again.
int group_level(genga_ctx *ctx, int level, const LevelTiles &T, bool deepest, hipStream_t s)
{
    GroupOut out;
    if (deepest) {
        out.body = ctx->lv_mem;
        out.off = ctx->lv_gs;
    } else {
        LevelTiles &C = ctx->lt[level];
        out.body = C.body;
        out.off = C.off;
        out.tfirst = C.tfirst;
        out.tiles = C.tiles;
        out.tl = C.tl;
    }
    HIP_TRY(launch_group_layout(ctx->L, ctx->gw, ctx->lv_pairs, ctx->lv_count, ctx->pair_cap, ctx->lab, T.body, T.M,
                                out, s, true));
    HIP_TRY(hipMemcpyAsync(ctx->ghdr, ctx->gw.hdr, sizeof(GroupHeader), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int round = 0; ctx->ghdr->unconverged; ++round) {
        if (round > 4096) return fail(GENGA_ERR_STATE, "union-find of the level pairs did not settle");
        ctx->pin[2] = 0;
        HIP_TRY(hipMemcpyAsync(ctx->big_changed, ctx->pin + 2, sizeof(int32_t), hipMemcpyHostToDevice, s));
        for (int rep = 0; rep < 2; ++rep) {
            HIP_TRY(launch_uf_hook(ctx->lv_pairs, ctx->lv_count, ctx->pair_cap, ctx->lab, ctx->big_changed, s));
            HIP_TRY(launch_uf_compress(ctx->L, ctx->lab, s));
        }
        HIP_TRY(hipMemcpyAsync(ctx->pin + 2, ctx->big_changed, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (ctx->pin[2] == 0) {
            HIP_TRY(launch_group_layout(ctx->L, ctx->gw, ctx->lv_pairs, ctx->lv_count, ctx->pair_cap, ctx->lab,
                                        T.body, T.M, out, s, false));
            HIP_TRY(hipMemcpyAsync(ctx->ghdr, ctx->gw.hdr, sizeof(GroupHeader), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    const GroupHeader &h = *ctx->ghdr;
    const auto refuse = [&](int status, const char *fmt, int a, int b) {
        if (ctx->L.n_total > 0)
            (void)hipMemsetAsync(ctx->lab, 0xff, (size_t)ctx->L.n_total * sizeof(int32_t), s);
        return fail(status, fmt, a, b);
    };
    // a list cut at its capacity has been flagged by the kick that filled it: refused
    if (h.pair_count > ctx->pair_cap)
        return refuse(GENGA_ERR_CAPACITY, "%d encounter pairs exceed the capacity %d", h.pair_count, ctx->pair_cap);
    if (h.max_nb > 64 * BIG_TILES_PER_GROUP)
        return refuse(GENGA_ERR_CAPACITY, "an encounter group of %d bodies (at most %d)", h.max_nb,
                      64 * BIG_TILES_PER_GROUP);
    if (!deepest && (h.G > ctx->lt_cap_G || h.n_tiles > ctx->lt_cap_T || h.M > ctx->lt[level].cap_M))
        return refuse(GENGA_ERR_STATE, "level layout of %d groups exceeds its allocation (%d)", h.G, ctx->lt_cap_G);
    return GENGA_OK;
}

// Level `level` (>= 1) over tau for the parent groups laid out in ctx->lt[level - 1].
int run_level(genga_ctx *ctx, genga_bodies *b, int level, double tau, hipStream_t s)
{
    LevelTiles &T = ctx->lt[level - 1];
    if (T.G <= 0) return GENGA_OK;
    HIP_TRY(launch_level_tiles_setup(ctx->L, T, b->m, b->rcrit, ctx->rc_lv, level, s));
    const double h = tau / ctx->n_sub;
    const bool deepest = level + 1 == ctx->n_levels;
    int rc;
    for (int sub = 0; sub < ctx->n_sub; ++sub) {
        // the emitting kick clears the pair count of the level
        if ((rc = level_kick(ctx, b, level, T, 0.5 * h, true, s))) return rc;
        if ((rc = group_level(ctx, level, T, deepest, s))) return rc;
        const GroupHeader hd = *ctx->ghdr;
        // parent members in no pair of this level (device label -1): Kepler drift over h; the
        // same launch clears the labels (only parent members carry one)
        HIP_TRY(launch_kepler_list(ctx->L, T.body, T.M, b->x, b->y, b->z, b->vx, b->vy, b->vz, h, ctx->flags, s,
                                   ctx->lab));
        if (hd.G > 0) {
            if (deepest) {
                // Bulirsch-Stoer with the product weight: one wave per group of up to 64 members
                // (the group count read on the device), the grid-wide path for larger ones
                HIP_TRY(launch_drift(ctx->L, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, b->rcrit, h, ctx->lv_mem,
                                     ctx->lv_gs, &ctx->gw.hdr->G, ctx->member_slot, ctx->flags, 1, hd.G, ctx->wg_list, s,
                                     ctx->rc_lv, ctx->n_levels, false, drift_side(ctx, s)));
                if (hd.max_nb > CE_MAX_GROUP) {
                    // rare: the groups and the parent order go to the host for the grid-wide path
                    std::vector<int32_t> cgs(hd.G + 1), cmem(hd.M), prev(T.M);
                    HIP_TRY(hipMemcpyAsync(cgs.data(), ctx->lv_gs, cgs.size() * sizeof(int32_t),
                                           hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipMemcpyAsync(cmem.data(), ctx->lv_mem, cmem.size() * sizeof(int32_t),
                                           hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipMemcpyAsync(prev.data(), T.body, prev.size() * sizeof(int32_t),
                                           hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipStreamSynchronize(s));
                    if ((rc = run_big_groups(ctx, b, h, s, cgs, cmem, ctx->lv_mem, CE_MAX_GROUP + 1, &prev)))
                        return rc;
                }
            } else {
                LevelTiles &C = ctx->lt[level];
                C.G = hd.G;
                C.M = hd.M;
                C.n_tiles = hd.n_tiles;
                C.n_multi = hd.n_multi;
                if ((rc = run_level(ctx, b, level + 1, h, s))) return rc;
            }
        }
        if ((rc = level_kick(ctx, b, level, T, 0.5 * h, false, s))) return rc;
    }
    return GENGA_OK;
}

// Level 1 over dt for the groups of the context's encounter list (built by enqueue_drift): the
// groups are ordered by ring and azimuth on the host, once per step, and laid out in tiles; the
// deeper levels inherit that order through the device layout.
int run_levels(genga_ctx *ctx, genga_bodies *b, double dt, hipStream_t s)
{
    const std::vector<int32_t> &pgs = ctx->gs_h;
    LevelTiles &T = ctx->lt[0];
    T.G = T.M = T.n_tiles = T.n_multi = 0;
    if ((int)pgs.size() <= 1) return GENGA_OK;
    TileOrder o;
    int rc = order_tiles(ctx, pgs, {}, 2, o);
    if (rc) return rc;
    if ((int)o.k0.size() > ctx->lt_cap_G || o.off.back() > T.cap_M || (int)o.tiles.size() > ctx->lt_cap_T)
        return fail(GENGA_ERR_STATE, "level layout exceeds its allocation");
    T.G = (int32_t)o.k0.size();
    T.M = o.off.back();
    T.n_tiles = (int32_t)o.tiles.size();
    if (T.G == 0) return GENGA_OK;
    // tiles of the groups of more than one tile first (a workgroup each), then the one tile of
    // every smaller group (a wave each)
    std::vector<int32_t> tl;
    tl.reserve(o.tiles.size());
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t gi = 0; gi < o.k0.size(); ++gi) {
            const int t0 = o.tfirst[gi], t1 = o.tfirst[gi + 1];
            if ((t1 - t0 > 1) == (pass == 0))
                for (int k = t0; k < t1; ++k) tl.push_back(k);
        }
        if (pass == 0) T.n_multi = (int32_t)tl.size();
    }
    // the layout's uploads on the stream, one host wait after the last
    if (!tl.empty())
        HIP_TRY(hipMemcpyAsync(T.tl, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(T.off, o.off.data(), o.off.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(T.tfirst, o.tfirst.data(), o.tfirst.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!o.tiles.empty())
        HIP_TRY(hipMemcpyAsync(T.tiles, o.tiles.data(), o.tiles.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    // the members in ring / azimuth order, on the device (the group offsets in the large-group
    // layout's k0, free until run_big_groups lays out its own)
    HIP_TRY(hipMemcpyAsync(ctx->big.k0, o.k0.data(), o.k0.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_ring_order(ctx->members, ctx->big.k0, T.off, T.G, T.M, b->x, b->y, ctx->ow, T.body, s));
    HIP_TRY(hipStreamSynchronize(s));
    return run_level(ctx, b, 1, dt, s);
}

// Grid-wide Bulirsch-Stoer over dt for the groups gs / mem (host copies; members_dev the
// device copy of mem) of at least min_nb members.
int run_big_groups(genga_ctx *ctx, genga_bodies *b, double dt, hipStream_t s, const std::vector<int32_t> &gs,
                   const std::vector<int32_t> &mem_h, const int32_t *members_dev, int min_nb,
                   const std::vector<int32_t> *prev)
{
    BigBs &bg = ctx->big;
    bg.G = bg.M = bg.n_tiles = 0;
    TileOrder o;
    int rc = order_tiles(ctx, gs, mem_h, min_nb, o, prev);
    if (rc) return rc;
    if (o.k0.empty()) return GENGA_OK;
    if ((int)o.k0.size() > bg.cap_G || o.off.back() > bg.cap_M || (int)o.tiles.size() > bg.cap_T)
        return fail(GENGA_ERR_STATE, "large-group layout exceeds its allocation");
    bg.G = (int32_t)o.k0.size();
    bg.M = o.off.back();
    bg.n_tiles = (int32_t)o.tiles.size();
    // the layout's uploads on the stream, one host wait after the last
    HIP_TRY(hipMemcpyAsync(bg.k0, o.k0.data(), o.k0.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(bg.off, o.off.data(), o.off.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(bg.tiles, o.tiles.data(), o.tiles.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(bg.tfirst, o.tfirst.data(), o.tfirst.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    const int32_t dims[4] = {bg.G, bg.M, bg.n_tiles, 0};
    HIP_TRY(hipMemcpyAsync(bg.dims, dims, sizeof(dims), hipMemcpyHostToDevice, s));
    if (prev)
        HIP_TRY(hipMemcpyAsync(bg.body, o.body.data(), o.body.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    else
        HIP_TRY(launch_ring_order(members_dev, bg.k0, bg.off, bg.G, bg.M, b->x, b->y, ctx->ow, bg.body, s));
    HIP_TRY(hipStreamSynchronize(s));
    const Layout &L = ctx->L;
    HIP_TRY(launch_big_setup(L, bg, members_dev, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, b->rcrit, ctx->rc_lv,
                             dt, s));
    // every attempt ends with the count of groups still short of dt; the device gives up on a
    // group after 20000 attempts, so the loop ends
    int gl = 6;
    while ((1 << gl) < bg.n_tiles && (1 << gl) < bg.cap_T) ++gl;
    // one attempt's launch sequence, captured once per context, path and grid (sizes and dt live
    // in device memory, every buffer address is fixed)
    const auto attempt_graph = [&](bool lists, hipGraphExec_t &exec) -> int {
        if (exec) return GENGA_OK;
        if (!ctx->big_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->big_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(ctx->big_stream, hipStreamCaptureModeThreadLocal));
        // tile path: 16 waves per tile while the grid fits one workgroup per CU, else 8 (two
        // workgroups per CU: at N = 40322, 631 tiles, 20.5 steps/s against 18.0 with 16 and 19.4
        // with 4)
        const int tg = 1 << gl, waves = tg <= ctx->n_cu ? 16 : 8;
        const hipError_t le = lists ? launch_big_attempt_list(bg, 1e-12, ctx->flags, tg, ctx->big_stream)
                                    : launch_big_attempt(bg, 1e-12, ctx->flags, tg, waves, ctx->big_stream);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(ctx->big_stream, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(GENGA_ERR_HIP, "capturing the large-group attempt failed: %s",
                        hipGetErrorString(le != hipSuccess ? le : ce));
        }
        const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            exec = nullptr;
            return fail(GENGA_ERR_HIP, "hipGraphInstantiate (large-group attempt) failed: %s", hipGetErrorString(ie));
        }
        return GENGA_OK;
    };
    // the list path; a list above its capacity sends the rest of the step to the tile path
    if ((rc = attempt_graph(true, ctx->big_exec_list[gl]))) return rc;
    bool lists = true;
    for (int attempt = 0; attempt <= 20001; ++attempt) {
        HIP_TRY(hipGraphLaunch(lists ? ctx->big_exec_list[gl] : ctx->big_exec[gl], s));
        HIP_TRY(hipMemcpyAsync(ctx->pin + 1, bg.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (lists) HIP_TRY(hipMemcpyAsync(ctx->pin + 2, bg.ovf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (lists && ctx->pin[2]) {
            ctx->pin[2] = 0;
            HIP_TRY(hipMemcpyAsync(bg.ovf, ctx->pin + 2, sizeof(int32_t), hipMemcpyHostToDevice, s));
            if ((rc = attempt_graph(false, ctx->big_exec[gl]))) return rc;
            lists = false;
        }
        if (ctx->pin[1] == 0) break;
    }
    HIP_TRY(launch_big_finish(bg, b->x, b->y, b->z, b->vx, b->vy, b->vz, s));
    return GENGA_OK;
}

int enqueue_energy(genga_ctx *ctx, const genga_bodies *b, double vshift, double *out, hipStream_t s)
{
    const Layout &L = ctx->L;
    const size_t n = (size_t)L.n_total;
    HIP_TRY(launch_energy(L, ctx->eitems, ctx->n_items, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, ctx->acc,
                          ctx->acc + n, ctx->acc + 2 * n, vshift, ctx->epartial, ctx->item_first, out, s));
    return GENGA_OK;
}

int enqueue_step(genga_ctx *ctx, genga_bodies *b, double dt, int nsteps, int prec, int acc, int cadence,
                 double *d_energy, hipStream_t s)
{
    const size_t n = (size_t)ctx->L.n_total;
    double *ax = ctx->acc, *ay = ctx->acc + n, *az = ctx->acc + 2 * n;
    int rc = enqueue_kick(ctx, b, 0.5 * dt, 1, prec, acc, ax, ay, az, s);
    if (rc) return rc;
    int rec = 0;
    for (int k = 1; k <= nsteps; ++k) {
        // the second half Sun drift is left to the next kick's source pass, except with
        // collisions, which are resolved on the drifted state
        const bool defer = ctx->col.mass == nullptr;
        rc = enqueue_drift(ctx, b, dt, s, defer);
        if (rc) return rc;
        const bool last = k == nsteps;
        rc = enqueue_kick(ctx, b, last ? 0.5 * dt : dt, 1, prec, acc, ax, ay, az, s, defer ? 0.5 * dt : 0.0);
        if (rc) return rc;
        if (cadence > 0 && d_energy && k % cadence == 0) {
            rc = enqueue_energy(ctx, b, last ? 0.0 : 0.5 * dt, d_energy + (size_t)rec * 4 * ctx->L.n_sys, s);
            if (rc) return rc;
            ++rec;
        }
    }
    return GENGA_OK;
}

// Work items: 64 consecutive bodies of one system, never mixing massive and test bodies;
// massive targets visit every body of their system, test targets only the massive ones.
// Kick items are ordered by work (largest first), energy items by system.
int upload_plan(genga_ctx *ctx)
{
    const int n_sys = ctx->L.n_sys;
    std::vector<WorkItem> it;
    std::vector<int32_t> first(n_sys + 1, 0);
    for (int s = 0; s < n_sys; ++s) {
        first[s] = (int32_t)it.size();
        const int b = ctx->sys_off_h[s], e = ctx->sys_off_h[s + 1];
        const int nm = ctx->n_massive_h[s];
        for (int i0 = b; i0 < b + nm; i0 += 64) it.push_back(WorkItem{s, i0, std::min(64, b + nm - i0), e - b});
        for (int i0 = b + nm; i0 < e; i0 += 64) it.push_back(WorkItem{s, i0, std::min(64, e - i0), nm});
    }
    first[n_sys] = (int32_t)it.size();
    if (it.size() > ctx->max_items) return fail(GENGA_ERR_STATE, "work plan larger than its allocation");
    std::vector<WorkItem> kit = it;
    std::stable_sort(kit.begin(), kit.end(), [](const WorkItem &a, const WorkItem &b) { return a.nsrc > b.nsrc; });
    ctx->n_items = (int32_t)it.size();
    if (!it.empty()) {
        HIP_TRY(hipMemcpy(ctx->items, kit.data(), kit.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(ctx->eitems, it.data(), it.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(ctx->item_first, first.data(), (n_sys + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->L.n_massive, ctx->n_massive_h.data(), n_sys * sizeof(int32_t), hipMemcpyHostToDevice));
    std::vector<int32_t> seg(2 * (size_t)n_sys + 1);
    for (int s = 0; s < n_sys; ++s) {
        seg[2 * s] = ctx->sys_off_h[s];
        seg[2 * s + 1] = ctx->sys_off_h[s] + ctx->n_massive_h[s];
    }
    seg[2 * n_sys] = ctx->sys_off_h[n_sys];
    HIP_TRY(hipMemcpy(ctx->sort_seg, seg.data(), seg.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    return GENGA_OK;
}

} // namespace

extern "C" {

const char *genga_last_error(void) { return g_last_error.c_str(); }

int genga_create(genga_ctx **out, int device)
{
    if (!out) return fail(GENGA_ERR_ARG, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(GENGA_ERR_ARG, "device %d out of range (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    // the allocation-free entry point's scratch address on this device
    int rc = noalloc_prepare(device, nullptr, nullptr);
    if (rc) return rc;
    genga_ctx *c = new genga_ctx();
    c->device = device;
    if (hipHostMalloc((void **)&c->hpin, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(GENGA_ERR_HIP, "hipHostMalloc of the status word failed");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->n_cu = prop.multiProcessorCount;
        // the architecture name up to its first ':' (feature suffixes), spaces excluded
        int k = 0;
        for (; k < 63 && prop.gcnArchName[k] && prop.gcnArchName[k] != ':' && prop.gcnArchName[k] != ' '; ++k)
            c->arch[k] = prop.gcnArchName[k];
        if (k > 0) c->arch[k] = 0;
    }
    *out = c;
    return GENGA_OK;
}

int genga_destroy(genga_ctx *ctx)
{
    if (!ctx) return GENGA_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->release();
    if (ctx->hpin) (void)hipHostFree(ctx->hpin);
    if (ctx->ghdr) (void)hipHostFree(ctx->ghdr);
    delete ctx;
    return GENGA_OK;
}

int genga_set_systems(genga_ctx *ctx, int32_t n_sys, const int32_t *sys_off_host, const double *mstar_host,
                      int32_t pair_capacity)
{
    int rc = check_ctx(ctx, false);
    if (rc) return rc;
    if (n_sys < 1) return fail(GENGA_ERR_ARG, "n_sys must be >= 1 (got %d)", n_sys);
    if (!sys_off_host || !mstar_host) return fail(GENGA_ERR_ARG, "null sys_off or mstar");
    if (sys_off_host[0] != 0) return fail(GENGA_ERR_ARG, "sys_off[0] must be 0");
    for (int s = 0; s < n_sys; ++s) {
        if (sys_off_host[s + 1] < sys_off_host[s]) return fail(GENGA_ERR_ARG, "sys_off not non-decreasing at %d", s);
        if (!(mstar_host[s] > 0.0)) return fail(GENGA_ERR_ARG, "mstar[%d] must be > 0", s);
    }
    const int64_t n_total64 = sys_off_host[n_sys];
    if (n_total64 > (int64_t)1 << 30) return fail(GENGA_ERR_ARG, "too many bodies");
    const int32_t n_total = (int32_t)n_total64;
    HIP_TRY(hipDeviceSynchronize());
    const int32_t keep_large = ctx->large_groups;
    ctx->release();
    ctx->sys_off_h.assign(sys_off_host, sys_off_host + n_sys + 1);
    ctx->mstar_h.assign(mstar_host, mstar_host + n_sys);
    ctx->pair_cap_req = pair_capacity;

    // work items: 64 consecutive bodies of one system
    std::vector<Chunk> chunks;
    std::vector<int32_t> cfirst(n_sys + 1, 0);
    for (int s = 0; s < n_sys; ++s) {
        cfirst[s] = (int32_t)chunks.size();
        for (int b = sys_off_host[s]; b < sys_off_host[s + 1]; b += CHUNK)
            chunks.push_back(Chunk{s, b, std::min(b + CHUNK, sys_off_host[s + 1]), 0});
    }
    cfirst[n_sys] = (int32_t)chunks.size();

    std::vector<int32_t> sys_of(n_total);
    for (int s = 0; s < n_sys; ++s)
        for (int i = sys_off_host[s]; i < sys_off_host[s + 1]; ++i) sys_of[i] = s;

    int32_t cap = pair_capacity > 0 ? pair_capacity : (int32_t)std::min<int64_t>(16 * (int64_t)n_total + 1024, INT32_MAX / 4);
    ctx->pair_cap = cap;
    int64_t npow = 1;
    while (npow < cap) npow <<= 1;
    const size_t nt = (size_t)n_total;

    HIP_TRY(dalloc(ctx->L.sys_off, n_sys + 1));
    HIP_TRY(dalloc(ctx->L.sys_of, nt));
    HIP_TRY(dalloc(ctx->L.mstar, n_sys));
    // at most one more item per system when the massive / test boundary splits a block
    size_t max_items = 0;
    for (int s = 0; s < n_sys; ++s) max_items += (size_t)(sys_off_host[s + 1] - sys_off_host[s] + 63) / 64 + 1;
    ctx->max_items = max_items;
    HIP_TRY(dalloc(ctx->items, max_items));
    HIP_TRY(dalloc(ctx->eitems, max_items));
    HIP_TRY(dalloc(ctx->item_first, n_sys + 1));
    HIP_TRY(dalloc(ctx->L.n_massive, n_sys));
    HIP_TRY(dalloc(ctx->jrec, nt * 32));
    HIP_TRY(dalloc(ctx->L.chunks, chunks.size()));
    HIP_TRY(dalloc(ctx->L.chunk_first, n_sys + 1));
    HIP_TRY(dalloc(ctx->rc2_part, chunks.size()));
    HIP_TRY(dalloc(ctx->mom_part, 3 * chunks.size()));
    HIP_TRY(dalloc(ctx->acc, 3 * nt));
    HIP_TRY(dalloc(ctx->pairs, 2 * (size_t)cap));
    HIP_TRY(dalloc(ctx->pair_count, 1));
    HIP_TRY(dalloc(ctx->sort_keys, (size_t)npow));
    HIP_TRY(dalloc(ctx->flags, 1));
    HIP_TRY(dalloc(ctx->lab, nt));
    HIP_TRY(dalloc(ctx->mark, nt));
    ctx->ce_cap = std::max(CE_MAX_MEMBERS, n_total);
    HIP_TRY(dalloc(ctx->members, (size_t)ctx->ce_cap));
    HIP_TRY(dalloc(ctx->group_start, (size_t)ctx->ce_cap + 1));
    HIP_TRY(dalloc(ctx->n_groups, 1));
    HIP_TRY(dalloc(ctx->member_slot, nt));
    HIP_TRY(dalloc(ctx->wg_list, (size_t)std::max(ctx->ce_cap, n_total) / 2 + 2));
    HIP_TRY(dalloc(ctx->epartial, 9 * (size_t)ENERGY_SPLIT * max_items));
    HIP_TRY(dalloc(ctx->kpart, (size_t)KICK_MAX_SPLIT * 3 * nt));
    HIP_TRY(dalloc(ctx->import_bad, 1));
    HIP_TRY(hipMemset(ctx->import_bad, 0, sizeof(int32_t)));
    HIP_TRY(order_work_alloc(ctx->sw, std::max(n_total, 2 * n_sys)));
    HIP_TRY(dalloc(ctx->sort_seg, 2 * (size_t)n_sys + 1));
    HIP_TRY(dalloc(ctx->sort_perm, std::max<size_t>(nt, 1)));

    HIP_TRY(hipMemcpy(ctx->L.sys_off, sys_off_host, (n_sys + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    if (nt) HIP_TRY(hipMemcpy(ctx->L.sys_of, sys_of.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->L.mstar, mstar_host, n_sys * sizeof(double), hipMemcpyHostToDevice));

    if (!chunks.empty())
        HIP_TRY(hipMemcpy(ctx->L.chunks, chunks.data(), chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->L.chunk_first, cfirst.data(), (n_sys + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(ctx->pair_count, 0, sizeof(int32_t)));
    HIP_TRY(hipMemset(ctx->flags, 0, sizeof(int32_t)));
    HIP_TRY(hipMemset(ctx->n_groups, 0, sizeof(int32_t)));
    HIP_TRY(hipMemset(ctx->lab, 0xff, nt * sizeof(int32_t)));
    HIP_TRY(hipMemset(ctx->mark, 0, nt * sizeof(int32_t)));
    HIP_TRY(hipMemset(ctx->member_slot, 0xff, nt * sizeof(int32_t)));
    HIP_TRY(hipMemset(ctx->acc, 0, 3 * nt * sizeof(double)));
    HIP_TRY(hipDeviceSynchronize());
    ctx->L.n_sys = n_sys;
    ctx->L.n_total = n_total;
    ctx->L.n_chunks = (int32_t)chunks.size();
    ctx->n_massive_h.assign(sys_off_host, sys_off_host + n_sys);
    for (int s = 0; s < n_sys; ++s) ctx->n_massive_h[s] = sys_off_host[s + 1] - sys_off_host[s];
    rc = upload_plan(ctx);
    if (rc) return rc;
    ctx->split[0] = ctx->split[1] = default_split(ctx);
    if (keep_large) {
        if ((rc = alloc_big(ctx))) return rc;
        ctx->large_groups = 1;
    }
    return GENGA_OK;
}

int genga_set_levels(genga_ctx *ctx, int32_t n_levels, int32_t n_sub, const double *rcrit_levels)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (n_levels < 1 || n_levels > LEVELS_MAX) return fail(GENGA_ERR_ARG, "n_levels must be in 1..%d", LEVELS_MAX);
    if (n_levels > 1 && (n_sub < 1 || n_sub > 64)) return fail(GENGA_ERR_ARG, "n_sub must be in 1..64");
    if (n_levels > 1 && !rcrit_levels) return fail(GENGA_ERR_ARG, "null rcrit_levels");
    if (!ctx->large_groups) return fail(GENGA_ERR_STATE, "levels need the large-group mode (genga_set_large_groups)");
    const size_t nt = (size_t)ctx->L.n_total;
    std::vector<double> h;
    if (n_levels > 1) {
        // the radii must be finite, positive and not grow with the level
        h.resize((size_t)(n_levels - 1) * nt);
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(h.data(), rcrit_levels, h.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < h.size(); ++k) {
            if (!(h[k] > 0.0) || !std::isfinite(h[k]))
                return fail(GENGA_ERR_ARG, "rcrit_levels[%zu] is not a positive finite radius", k);
            if (k >= nt && h[k] > h[k - nt])
                return fail(GENGA_ERR_ARG, "rcrit_levels[%zu] exceeds the level above", k);
        }
    }
    HIP_TRY(hipDeviceSynchronize());
    ctx->release_big();
    ctx->n_levels = n_levels;
    ctx->n_sub = n_levels > 1 ? n_sub : 1;
    if ((rc = alloc_big(ctx))) {
        ctx->release_big();
        return rc;
    }
    ctx->large_groups = 1;
    if (n_levels > 1 && nt)
        HIP_TRY(hipMemcpy(ctx->rc_lv, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    return GENGA_OK;
}

int genga_tune_levels(genga_ctx *ctx, genga_bodies *b, double dt, double n1, double n2, int32_t max_levels,
                      int32_t max_sub, int32_t trial_steps, int prec, int32_t *levels_out, int32_t *sub_out,
                      void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_prec(prec)) || (rc = check_bodies(ctx, b, true, true))) return rc;
    if (max_levels < 1 || max_levels > LEVELS_MAX) return fail(GENGA_ERR_ARG, "max_levels must be in 1..%d", LEVELS_MAX);
    if (max_levels > 1 && (max_sub < 2 || max_sub > 64)) return fail(GENGA_ERR_ARG, "max_sub must be in 2..64");
    if (trial_steps < 1) return fail(GENGA_ERR_ARG, "trial_steps must be >= 1");
    if (!levels_out || !sub_out) return fail(GENGA_ERR_ARG, "null output");
    if (!(n1 >= 0.0) || !(n2 >= 0.0) || !(dt > 0.0)) return fail(GENGA_ERR_ARG, "n1, n2 >= 0 and dt > 0 required");
    if (!ctx->large_groups) return fail(GENGA_ERR_STATE, "levels need the large-group mode (genga_set_large_groups)");
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    const size_t n = (size_t)ctx->L.n_total;
    // device conditions raised before the tuning and not yet polled are kept for the caller
    int32_t pending = 0;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(&pending, ctx->flags, sizeof(int32_t), hipMemcpyDeviceToHost));
    double *save = nullptr, *rcl = nullptr;
    HIP_TRY(dalloc(save, 6 * std::max<size_t>(n, 1)));
    if (dalloc(rcl, (LEVELS_MAX - 1) * std::max<size_t>(n, 1)) != hipSuccess) {
        dfree(save);
        return fail(GENGA_ERR_HIP, "allocation of the tuning buffers failed");
    }
    double *st[6] = {b->x, b->y, b->z, b->vx, b->vy, b->vz};
    auto copy_state = [&](bool to_save) -> hipError_t {
        for (int q = 0; q < 6; ++q) {
            const hipError_t e = hipMemcpyAsync(to_save ? save + q * n : st[q], to_save ? st[q] : save + q * n,
                                                n * sizeof(double), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
        return hipStreamSynchronize(s);
    };
    // the level radii of a configuration: eq. (1) with the level's step dt / n_sub^k
    auto set_config = [&](int nl, int ns) -> int {
        for (int k = 1; k < nl; ++k) {
            const hipError_t e = launch_rcrit(ctx->L, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, n1, n2,
                                              dt / std::pow((double)ns, k), rcl + (size_t)(k - 1) * n, s);
            if (e != hipSuccess) return fail(GENGA_ERR_HIP, "r_crit of the levels: %s", hipGetErrorString(e));
        }
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(GENGA_ERR_HIP, "%s", hipGetErrorString(e));
        return genga_set_levels(ctx, nl, ns, nl > 1 ? rcl : nullptr);
    };
    int best_l = 1, best_s = 1;
    double best_t = INFINITY;
    // the trials run without collisions, which would change masses, radii and statuses
    const CollideArgs col = ctx->col;
    ctx->col.mass = nullptr;
    hipError_t he = copy_state(true);
    rc = he == hipSuccess ? GENGA_OK : fail(GENGA_ERR_HIP, "%s", hipGetErrorString(he));
    for (int nl = 1; nl <= max_levels && !rc; ++nl)
        for (int ns = nl == 1 ? 1 : 2; ns <= (nl == 1 ? 1 : max_sub) && !rc; ++ns) {
            // radii from the starting state; the trial runs from it too
            if ((he = copy_state(false)) != hipSuccess) {
                rc = fail(GENGA_ERR_HIP, "%s", hipGetErrorString(he));
                break;
            }
            if ((rc = set_config(nl, ns))) break;
            if ((he = hipMemsetAsync(ctx->flags, 0, sizeof(int32_t), s)) != hipSuccess) {
                rc = fail(GENGA_ERR_HIP, "%s", hipGetErrorString(he));
                break;
            }
            const auto t0 = std::chrono::steady_clock::now();
            const int r = enqueue_step(ctx, b, dt, trial_steps, prec, GENGA_ACC_FP64, 0, nullptr, s);
            if ((he = hipStreamSynchronize(s)) != hipSuccess) {
                rc = fail(GENGA_ERR_HIP, "%s", hipGetErrorString(he));
                break;
            }
            const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            int32_t flags = 0;
            if ((he = hipMemcpy(&flags, ctx->flags, sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess) {
                rc = fail(GENGA_ERR_HIP, "%s", hipGetErrorString(he));
                break;
            }
            if (r == GENGA_ERR_CAPACITY) continue; // this configuration does not fit: not a candidate
            if (r) {
                rc = r;
                break;
            }
            if (flags == 0 && t < best_t) {
                best_t = t;
                best_l = nl;
                best_s = ns;
            }
        }
    // back to the starting state, with the fastest configuration that ran clean
    if (!rc && (he = copy_state(false)) != hipSuccess) rc = fail(GENGA_ERR_HIP, "%s", hipGetErrorString(he));
    if (!rc) rc = set_config(best_l, best_s);
    if (!rc && ((he = hipMemsetAsync(ctx->flags, 0, sizeof(int32_t), s)) != hipSuccess ||
                (he = hipStreamSynchronize(s)) != hipSuccess))
        rc = fail(GENGA_ERR_HIP, "%s", hipGetErrorString(he));
    ctx->col = col;
    dfree(save);
    dfree(rcl);
    if (pending && hipMemcpy(ctx->flags, &pending, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess && !rc)
        rc = fail(GENGA_ERR_HIP, "restoring the pending device status failed");
    if (rc) return rc;
    if (!(best_t < INFINITY)) return fail(GENGA_ERR_NOCONVERGE, "no configuration ran without a device condition");
    *levels_out = best_l;
    *sub_out = best_s;
    return GENGA_OK;
}

int genga_set_collisions(genga_ctx *ctx, double *mass, double *radius, int32_t *status, double r_min, double r_max)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    // a captured graph holds the collision launches (or lacks them): refused either way
    if (ctx->graph_exec)
        return fail(GENGA_ERR_STATE, "a captured graph exists: collisions cannot be switched while it does");
    if (mass && (!radius || !status)) return fail(GENGA_ERR_ARG, "null radius or status");
    if (mass && (!(r_min >= 0.0) || !(r_max > r_min))) return fail(GENGA_ERR_ARG, "need 0 <= r_min < r_max");
    HIP_TRY(hipDeviceSynchronize());
    if (!mass) {
        dfree(ctx->col.list);
        dfree(ctx->col.count);
        ctx->col = CollideArgs{};
        return GENGA_OK;
    }
    if (!ctx->col.list) {
        HIP_TRY(dalloc(ctx->col.list, 2 * (size_t)COLLIDE_CAP));
        HIP_TRY(dalloc(ctx->col.count, 1));
        HIP_TRY(hipMemset(ctx->col.count, 0, sizeof(int32_t)));
    }
    ctx->col.mass = mass;
    ctx->col.radius = radius;
    ctx->col.status = status;
    ctx->col.flags = ctx->flags;
    ctx->col.cap = COLLIDE_CAP;
    ctx->col.r_min = r_min;
    ctx->col.r_max = r_max;
    HIP_TRY(hipDeviceSynchronize());
    return GENGA_OK;
}

int genga_compact(genga_ctx *ctx, genga_bodies *b, double *radius, int32_t *status, int32_t *n_total_out)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_bodies(ctx, b, true, true))) return rc;
    if (!status || !n_total_out) return fail(GENGA_ERR_ARG, "null status or n_total_out");
    const int n = ctx->L.n_total, n_sys = ctx->L.n_sys;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<int32_t> st(n), idx, off(n_sys + 1, 0), nm(n_sys, 0);
    if (n) HIP_TRY(hipMemcpy(st.data(), status, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    bool any_test = false;
    for (int sy = 0; sy < n_sys; ++sy) {
        const int b0 = ctx->sys_off_h[sy], b1 = ctx->sys_off_h[sy + 1], nmass = ctx->n_massive_h[sy];
        any_test |= nmass < b1 - b0;
        for (int i = b0; i < b1; ++i)
            if (st[i] == 0) {
                idx.push_back(i);
                if (i - b0 < nmass) ++nm[sy];
            }
        off[sy + 1] = (int32_t)idx.size();
    }
    const int nk = (int)idx.size();
    if (nk < n) {
        int32_t *d_idx = nullptr;
        double *tmp = nullptr;
        HIP_TRY(dalloc(d_idx, std::max(nk, 1)));
        if (dalloc(tmp, std::max(nk, 1)) != hipSuccess) {
            dfree(d_idx);
            return fail(GENGA_ERR_HIP, "allocation for the compaction failed");
        }
        hipError_t e = nk ? hipMemcpy(d_idx, idx.data(), nk * sizeof(int32_t), hipMemcpyHostToDevice) : hipSuccess;
        double *arr[9] = {b->x, b->y, b->z, b->vx, b->vy, b->vz, const_cast<double *>(b->m),
                          const_cast<double *>(b->rcrit), radius};
        for (int a = 0; a < 9 && e == hipSuccess; ++a) {
            if (!arr[a]) continue;
            e = launch_gather(d_idx, nk, arr[a], tmp, nullptr);
            if (e == hipSuccess && nk) e = hipMemcpy(arr[a], tmp, nk * sizeof(double), hipMemcpyDeviceToDevice);
        }
        if (e == hipSuccess && nk) e = hipMemset(status, 0, nk * sizeof(int32_t));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        dfree(d_idx);
        dfree(tmp);
        if (e != hipSuccess) return fail(GENGA_ERR_HIP, "compaction: %s", hipGetErrorString(e));
    }
    // the new layout, with the context's settings carried over (levels start again at 1)
    const CollideArgs col = ctx->col;
    const std::vector<double> mstar = ctx->mstar_h;
    if ((rc = genga_set_systems(ctx, n_sys, off.data(), mstar.data(), ctx->pair_cap_req))) return rc;
    if (any_test && (rc = genga_set_test_bodies(ctx, nm.data()))) return rc;
    if (col.mass && (rc = genga_set_collisions(ctx, col.mass, col.radius, col.status, col.r_min, col.r_max)))
        return rc;
    *n_total_out = nk;
    return GENGA_OK;
}

int genga_sort_bodies(genga_ctx *ctx, genga_bodies *b, int32_t *perm_out, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_bodies(ctx, b, true, true))) return rc;
    hipStream_t s = (hipStream_t)stream;
    // the radix sort is a library call that clears its work memory with memset nodes, which
    // captured graphs must not hold
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(GENGA_ERR_STATE, "genga_sort_bodies cannot be captured into a graph");
    ctx->last_stream = s;
    ctx->list_valid = false; // the encounter list names bodies by their old places
    const int n = ctx->L.n_total;
    if (n == 0) return GENGA_OK;
    // runs: the massive, then the test bodies of each system, each in ring / azimuth order
    HIP_TRY(launch_ring_order(nullptr, ctx->sort_seg, ctx->sort_seg, 2 * ctx->L.n_sys, n, b->x, b->y, ctx->sw,
                              ctx->sort_perm, s));
    // every per-body array the context knows, staged through the kick's share buffer (at least
    // 3 n_total doubles; no kick is in flight between calls on the context's stream)
    double *tmp = ctx->kpart;
    std::vector<double *> arr = {b->x, b->y, b->z, b->vx, b->vy, b->vz, const_cast<double *>(b->m),
                                 const_cast<double *>(b->rcrit)};
    if (ctx->col.mass && ctx->col.mass != b->m) arr.push_back(ctx->col.mass);
    if (ctx->col.radius) arr.push_back(ctx->col.radius);
    for (int k = 0; ctx->rc_lv && k + 1 < ctx->n_levels; ++k) arr.push_back(ctx->rc_lv + (size_t)k * n);
    for (double *p : arr) {
        HIP_TRY(launch_gather(ctx->sort_perm, n, p, tmp, s));
        HIP_TRY(hipMemcpyAsync(p, tmp, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if (ctx->col.status) {
        int32_t *ti = reinterpret_cast<int32_t *>(tmp);
        HIP_TRY(launch_gather(ctx->sort_perm, n, ctx->col.status, ti, s));
        HIP_TRY(hipMemcpyAsync(ctx->col.status, ti, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    if (perm_out)
        HIP_TRY(hipMemcpyAsync(perm_out, ctx->sort_perm, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    return GENGA_OK;
}

int genga_set_large_groups(genga_ctx *ctx, int32_t enable)
{
    int rc = check_ctx(ctx, false);
    if (rc) return rc;
    if (enable != 0 && enable != 1) return fail(GENGA_ERR_ARG, "enable must be 0 or 1");
    HIP_TRY(hipDeviceSynchronize());
    if (!enable) {
        ctx->release_big();
        return GENGA_OK;
    }
    if (ctx->graph_exec) return fail(GENGA_ERR_STATE, "a captured graph exists: large groups need host round trips");
    if (!ctx->large_groups && (rc = alloc_big(ctx))) {
        ctx->release_big();
        return rc;
    }
    ctx->large_groups = 1;
    return GENGA_OK;
}

int genga_set_test_bodies(genga_ctx *ctx, const int32_t *n_massive_host)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    const int n_sys = ctx->L.n_sys;
    for (int s = 0; s < n_sys; ++s) {
        const int ns = ctx->sys_off_h[s + 1] - ctx->sys_off_h[s];
        const int nm = n_massive_host ? n_massive_host[s] : ns;
        if (nm < 0 || nm > ns) return fail(GENGA_ERR_ARG, "n_massive[%d] = %d outside [0, %d]", s, nm, ns);
    }
    HIP_TRY(hipDeviceSynchronize());
    for (int s = 0; s < n_sys; ++s)
        ctx->n_massive_h[s] = n_massive_host ? n_massive_host[s] : ctx->sys_off_h[s + 1] - ctx->sys_off_h[s];
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    return upload_plan(ctx);
}

int genga_rcrit(genga_ctx *ctx, const genga_bodies *b, double n1, double n2, double dt, double *rc_out,
                void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_bodies(ctx, b, true, false))) return rc;
    if (!rc_out && ctx->L.n_total) return fail(GENGA_ERR_ARG, "null rc_out");
    if (!(n1 >= 0.0) || !(n2 >= 0.0)) return fail(GENGA_ERR_ARG, "n1, n2 must be >= 0");
    HIP_TRY(launch_rcrit(ctx->L, b->x, b->y, b->z, b->vx, b->vy, b->vz, b->m, n1, n2, dt, rc_out,
                         (hipStream_t)stream));
    return GENGA_OK;
}

int genga_accel(genga_ctx *ctx, const genga_bodies *b, double *ax, double *ay, double *az, int prec, int acc,
                void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_prec(prec)) || (rc = check_acc(acc)) || (rc = check_bodies(ctx, b, false, true))) return rc;
    if (ctx->L.n_total && (!ax || !ay || !az)) return fail(GENGA_ERR_ARG, "null acceleration output");
    ctx->last_stream = (hipStream_t)stream;
    return enqueue_kick(ctx, b, 0.0, 0, prec, acc, ax, ay, az, (hipStream_t)stream);
}

int genga_kick(genga_ctx *ctx, genga_bodies *b, double tau, int prec, int acc, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_prec(prec)) || (rc = check_acc(acc)) || (rc = check_bodies(ctx, b, true, true))) return rc;
    const size_t n = (size_t)ctx->L.n_total;
    ctx->last_stream = (hipStream_t)stream;
    return enqueue_kick(ctx, b, tau, 1, prec, acc, ctx->acc, ctx->acc + n, ctx->acc + 2 * n, (hipStream_t)stream);
}

int genga_encounter_list(genga_ctx *ctx, const genga_bodies *b, int32_t *pairs, int32_t cap, int32_t *d_count,
                         void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!d_count) return fail(GENGA_ERR_ARG, "null d_count");
    if (cap < 0 || (cap > 0 && !pairs)) return fail(GENGA_ERR_ARG, "bad pairs buffer");
    if (b && (rc = check_bodies(ctx, b, false, true))) return rc;
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    if (b) {
        if ((rc = enqueue_pair_list(ctx, b, s))) return rc;
    } else if (!ctx->list_valid) {
        return fail(GENGA_ERR_STATE, "no kick has run on the current positions: pass the bodies to list their "
                                     "encounter pairs");
    }
    HIP_TRY(launch_sort_pairs(ctx->pairs, ctx->pair_count, ctx->pair_cap, pairs, cap, d_count, ctx->sort_keys,
                              ctx->flags, s));
    return GENGA_OK;
}

int genga_drift(genga_ctx *ctx, genga_bodies *b, double dt, const int32_t *pairs, const int32_t *d_count,
                void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_bodies(ctx, b, true, true))) return rc;
    if (pairs && !d_count) return fail(GENGA_ERR_ARG, "a pair list needs its device count");
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    if (pairs)
        HIP_TRY(launch_import_pairs(ctx->L, pairs, d_count, ctx->pairs, ctx->pair_count, ctx->pair_cap,
                                    ctx->import_bad, ctx->flags, s));
    return enqueue_drift(ctx, b, dt, s);
}

int genga_energy(genga_ctx *ctx, const genga_bodies *b, double *d_out, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_bodies(ctx, b, true, false))) return rc;
    if (!d_out) return fail(GENGA_ERR_ARG, "null d_out");
    ctx->last_stream = (hipStream_t)stream;
    return enqueue_energy(ctx, b, 0.0, d_out, (hipStream_t)stream);
}

int genga_step(genga_ctx *ctx, genga_bodies *b, double dt, int nsteps, int prec, int acc, int energy_cadence,
               double *d_energy, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_prec(prec)) || (rc = check_acc(acc)) || (rc = check_bodies(ctx, b, true, true))) return rc;
    if (nsteps < 0) return fail(GENGA_ERR_ARG, "nsteps must be >= 0");
    if (nsteps == 0) return GENGA_OK;
    ctx->last_stream = (hipStream_t)stream;
    return enqueue_step(ctx, b, dt, nsteps, prec, acc, energy_cadence, d_energy, (hipStream_t)stream);
}

int genga_graph_capture(genga_ctx *ctx, genga_bodies *b, double dt, int nsteps, int prec, int acc,
                        int energy_cadence, double *d_energy, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_prec(prec)) || (rc = check_acc(acc)) || (rc = check_bodies(ctx, b, true, true))) return rc;
    if (nsteps < 1) return fail(GENGA_ERR_ARG, "nsteps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(GENGA_ERR_ARG, "graph capture needs a non-default stream");
    ctx->last_stream = s;
    if (ctx->large_groups)
        return fail(GENGA_ERR_STATE, "graph capture is not available while large groups are enabled (host round trips)");
    HIP_TRY(hipStreamSynchronize(s));
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = enqueue_step(ctx, b, dt, nsteps, prec, acc, energy_cadence, d_energy, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(GENGA_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    ctx->graph = g;
    HIP_TRY(hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
    return GENGA_OK;
}

int genga_graph_launch(genga_ctx *ctx, int repeats, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!ctx->graph_exec) return fail(GENGA_ERR_STATE, "no captured graph");
    if (repeats < 0) return fail(GENGA_ERR_ARG, "repeats must be >= 0");
    ctx->last_stream = (hipStream_t)stream;
    for (int r = 0; r < repeats; ++r) HIP_TRY(hipGraphLaunch(ctx->graph_exec, (hipStream_t)stream));
    return GENGA_OK;
}

int genga_set_kick_shape(genga_ctx *ctx, int prec, int waves, int split)
{
    if (!ctx) return fail(GENGA_ERR_ARG, "null context");
    int rc = check_prec(prec);
    if (rc) return rc;
    if (waves == 0) waves = prec == GENGA_KICK_FP32 ? 16 : 8;
    if (waves != 4 && waves != 8 && waves != 16) return fail(GENGA_ERR_ARG, "waves must be 4, 8 or 16");
    if (split == 0) split = default_split(ctx);
    if (split < 1 || split > KICK_MAX_SPLIT) return fail(GENGA_ERR_ARG, "split must be 1..%d", KICK_MAX_SPLIT);
    ctx->waves[prec == GENGA_KICK_FP32] = waves;
    ctx->split[prec == GENGA_KICK_FP32] = split;
    return GENGA_OK;
}

int genga_get_kick_shape(genga_ctx *ctx, int prec, int *waves, int *split)
{
    if (!ctx || !waves || !split) return fail(GENGA_ERR_ARG, "null argument");
    int rc = check_prec(prec);
    if (rc) return rc;
    *waves = ctx->waves[prec == GENGA_KICK_FP32];
    *split = ctx->split[prec == GENGA_KICK_FP32];
    return GENGA_OK;
}

int genga_autotune(genga_ctx *ctx, genga_bodies *b, int prec, const char *cache_path, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if ((rc = check_prec(prec)) || (rc = check_bodies(ctx, b, false, true))) return rc;
    if (ctx->L.n_total == 0) return GENGA_OK;
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    const int fp32 = prec == GENGA_KICK_FP32;
    const size_t n = (size_t)ctx->L.n_total;
    // the cache key: device architecture and compute units, precision, and the layout (system
    // sizes and TP2 counts, hashed with 64-bit FNV-1a)
    char key[256] = {0};
    if (cache_path) {
        uint64_t h = 1469598103934665603ull;
        const auto mix = [&h](int32_t v) {
            for (int k = 0; k < 4; ++k) {
                h ^= (uint8_t)(v >> (8 * k));
                h *= 1099511628211ull;
            }
        };
        for (int32_t v : ctx->sys_off_h) mix(v);
        for (int32_t v : ctx->n_massive_h) mix(v);
        snprintf(key, sizeof(key), "genga-autotune v1 %s %d %d %d %d %016llx", ctx->arch, ctx->n_cu, prec,
                 ctx->L.n_sys, ctx->L.n_total, (unsigned long long)h);
        if (FILE *f = fopen(cache_path, "r")) {
            char line[512];
            bool hit = false;
            int cw = 0, cs = 0;
            const size_t kl = strlen(key);
            while (fgets(line, sizeof(line), f)) {
                if (strncmp(line, key, kl) == 0 && line[kl] == ' ' && sscanf(line + kl, "%d %d", &cw, &cs) == 2 &&
                    (cw == 4 || cw == 8 || cw == 16) && cs >= 1 && cs <= KICK_MAX_SPLIT)
                    hit = true; // the last matching line wins
            }
            const bool read_err = ferror(f) != 0;
            fclose(f);
            if (read_err) return fail(GENGA_ERR_ARG, "cannot read the autotune cache %s", cache_path);
            if (hit) {
                ctx->waves[fp32] = cw;
                ctx->split[fp32] = cs;
                return GENGA_OK;
            }
        }
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    int best_w = ctx->waves[fp32], best_s = ctx->split[fp32];
    for (int w : {4, 8, 16}) {
        for (int sp = 1; sp <= KICK_MAX_SPLIT && !rc; ++sp) {
            ctx->waves[fp32] = w;
            ctx->split[fp32] = sp;
            // accelerations only (velocities untouched); one warm-up then three timed launches
            rc = enqueue_kick(ctx, b, 0.0, 0, prec, GENGA_ACC_FP64, ctx->acc, ctx->acc + n, ctx->acc + 2 * n, s);
            if (rc) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < 3 && !rc; ++r)
                rc = enqueue_kick(ctx, b, 0.0, 0, prec, GENGA_ACC_FP64, ctx->acc, ctx->acc + n, ctx->acc + 2 * n, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                best_w = w;
                best_s = sp;
            }
        }
    }
    ctx->waves[fp32] = best_w;
    ctx->split[fp32] = best_s;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc || !cache_path) return rc;
    FILE *f = fopen(cache_path, "a");
    if (!f) return fail(GENGA_ERR_ARG, "cannot write the autotune cache %s", cache_path);
    const bool ok = fprintf(f, "%s %d %d\n", key, best_w, best_s) > 0;
    if (fclose(f) != 0 || !ok) return fail(GENGA_ERR_ARG, "cannot write the autotune cache %s", cache_path);
    return GENGA_OK;
}

int genga_poll_status(genga_ctx *ctx)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    hipStream_t s = ctx->last_stream;
    HIP_TRY(hipMemcpyAsync(ctx->hpin, ctx->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemsetAsync(ctx->flags, 0, sizeof(int32_t), s));
    HIP_TRY(hipStreamSynchronize(s));
    const int32_t f = *ctx->hpin;
    if (f & FLAG_BADPAIR) return fail(GENGA_ERR_ARG, "a pair list given to genga_drift held an invalid pair");
    if (f & FLAG_NONFINITE) return fail(GENGA_ERR_NONFINITE, "non-finite acceleration");
    if (f & FLAG_NOCONVERGE) return fail(GENGA_ERR_NOCONVERGE, "Bulirsch-Stoer step did not converge");
    if (f & FLAG_KEPLER) return fail(GENGA_ERR_NOCONVERGE, "Kepler solve did not converge");
    if (f & FLAG_CAPACITY) return fail(GENGA_ERR_CAPACITY, "encounter capacity exceeded");
    return GENGA_OK;
}

} // extern "C"
