// Kicks of the intermediate levels of the hierarchical step (Brasser et al. 2023, Sect. 1:
// symplectic levels with reduced steps between the level-0 step and the Bulirsch-Stoer step).
// Level l integrates each group of level l-1 in Strang sub-steps; its kick carries the share
// W_l K_l of the Newtonian pair force, W_l = prod_{k<l} (1 - K_k), K_k the changeover of
// level k's critical radius, and the same pass lists the pairs of the group closer than the
// level's critical radius (the next level's groups).  FP64 throughout: these are
// close-encounter forces.
//
// Layout as in the grid-wide Bulirsch-Stoer: the members of the parent groups are ordered by
// ring and azimuth (by the host, once per level interval) and cut into tiles of 64.  In a
// group of several tiles a workgroup of 16 waves (8 when such tiles outnumber the CUs, so that
// several workgroups share a CU) takes one target tile, lists the source tiles
// of the group whose box lies within the group's largest level-(l-1) radius of the target
// tile's box (no pair beyond that radius carries weight at level l), and deals their quarters
// out to its waves; a group of one tile is one wave, its members the sources in order.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

constexpr int LT_TILE = 64;

using CD = const __attribute__((address_space(4))) double;
using CI = const __attribute__((address_space(4))) int32_t;

// Per member f: mass, TP2 flag, the radii of levels 0..level; per group: the largest
// level-(level-1) radius squared, as the maximum over its tiles (bit patterns of non-negative
// doubles order as the values, so an integer atomic max gives the exact maximum).  One wave
// per tile; cut2 cleared first.
__global__ __launch_bounds__(256) void level_cut_clear_kernel(double *cut2, int G)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g < G) cut2[g] = 0.0;
}

__global__ __launch_bounds__(64) void level_tiles_setup_kernel(LevelTiles t, const int32_t *sys_of,
                                                               const int32_t *sys_off, const int32_t *n_massive,
                                                               const double *m, const double *rc0,
                                                               const double *rcl, int n_total, int level)
{
    const int4 tile = t.tiles[blockIdx.x];
    double mx = 0.0;
    if ((int)threadIdx.x < tile.z) {
        const int f = tile.y + threadIdx.x, body = t.body[f], s = sys_of[body];
        t.mass[f] = m[body];
        t.test[f] = body - sys_off[s] >= n_massive[s];
        t.rc[f] = rc0[body];
        for (int k = 1; k <= level; ++k) t.rc[(size_t)k * t.cap_M + f] = rcl[(size_t)(k - 1) * n_total + body];
        mx = fmax(0.0, sq_rn(t.rc[(size_t)(level - 1) * t.cap_M + f]));
    }
    mx = wave_maxv(mx);
    if (threadIdx.x == 0)
        atomicMax((unsigned long long *)&t.cut2[tile.x], (unsigned long long)__double_as_longlong(mx));
}

// Positions of the members of each tile, and the tile's box.  One wave per tile.
__global__ __launch_bounds__(64) void level_tiles_pos_kernel(LevelTiles t, const double *x, const double *y,
                                                             const double *z, int32_t *clear)
{
    const int me = blockIdx.x;
    if (clear && me == 0 && threadIdx.x == 0) *clear = 0; // the kick after this launch appends pairs
    const int4 tile = t.tiles[me];
    const bool v = (int)threadIdx.x < tile.z;
    const int f = tile.y + (v ? (int)threadIdx.x : 0);
    const int body = t.body[f];
    const double px = x[body], py = y[body], pz = z[body];
    if (v) {
        t.X[f] = px;
        t.Y[f] = py;
        t.Z[f] = pz;
    }
    tile_box(v, px, py, pz, t.bb, me);
}

// W_l K_l = prod_{k<l} (1 - K_k) times K_l (loops over the fixed bound, so the radii stay in
// registers)
__device__ __forceinline__ double level_share(double r, int l, const double *rcab)
{
    double w = 1.0, kl = 0.0;
#pragma unroll
    for (int k = 0; k < LEVELS_MAX; ++k) {
        if (k > l) break;
        const double kk = changeover_k((r - 0.1 * rcab[k]) / (0.9 * rcab[k]));
        if (k < l)
            w *= 1.0 - kk;
        else
            kl = kk;
    }
    return w * kl;
}

// The level's pairs found by a wave collect in its own LDS buffer and reach the list in
// blocks, one counter update per block: the pairs of a level kick over a whole disc number
// ~10^5, and one update per wave and source had queued on the counter.  Every lane of the
// wave takes part in each call (the fill count is the same in every lane).
constexpr int LV_BUF = 128;

__device__ __forceinline__ void lv_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void lv_flush(const LevelKickArgs &a, int2 *buf, int &fill)
{
    if (fill == 0) return;
    lv_wave_sync();
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == 0) base = atomicAdd(a.pair_count, fill);
    base = __shfl(base, 0, 64);
    for (int k = lane; k < fill; k += 64) {
        const int idx = base + k;
        if (idx < a.pair_cap) {
            a.pairs[2 * idx] = buf[k].x;
            a.pairs[2 * idx + 1] = buf[k].y;
        } else {
            atomicOr(a.flags, FLAG_CAPACITY);
        }
    }
    lv_wave_sync();
    fill = 0;
}

__device__ __forceinline__ void lv_emit(const LevelKickArgs &a, int2 *buf, int &fill, bool em, int i, int j)
{
    const unsigned long long m = __ballot(em);
    if (!m) return;
    const int c = __popcll(m);
    if (fill + c > LV_BUF) lv_flush(a, buf, fill);
    if (em) buf[fill + __popcll(m & ((1ull << (threadIdx.x & 63)) - 1))] = make_int2(i, j);
    fill += c;
}

// One target member (a lane) of a level kick.
struct LvTarget {
    bool valid, test;
    int f, body;
    double x, y, z;
    double rc[LEVELS_MAX]; // radii of levels 0..level (0 above)
    double rc_up;          // the radius of level - 1
};

__device__ __forceinline__ LvTarget lv_target(const LevelTiles &t, int4 tile, int lv)
{
    LvTarget me;
    const int lane = threadIdx.x & 63;
    me.valid = lane < tile.z;
    me.f = tile.y + (me.valid ? lane : 0);
    me.body = t.body[me.f];
    me.x = t.X[me.f];
    me.y = t.Y[me.f];
    me.z = t.Z[me.f];
    me.test = t.test[me.f] != 0;
#pragma unroll
    for (int k = 0; k < LEVELS_MAX; ++k) me.rc[k] = k <= lv ? t.rc[(size_t)k * t.cap_M + me.f] : 0.0;
    me.rc_up = t.rc[(size_t)(lv - 1) * t.cap_M + me.f];
    return me;
}

// Source member j (wave-uniform) for the target: its term if inside level (l-1)'s radius, and
// the level's pair.  Every lane of the wave calls it.
__device__ __forceinline__ void lv_source(const LevelTiles &t, const LevelKickArgs &a, const LvTarget &me, int lv,
                                          int j, double dx, double dy, double dz, double rcj_up, double &ax,
                                          double &ay, double &az, int2 *buf, int &fill)
{
    CD *SM = (CD *)t.mass;
    CD *SR = (CD *)t.rc;
    CI *ST = (CI *)t.test;
    CI *SB = (CI *)t.body;
    const double q = sep2_rn(dx, dy, dz);
    const double rc_up = fmax(me.rc_up, rcj_up);
    bool em = false;
    if (me.valid && j != me.f && !(me.test && ST[j] != 0) && q < sq_rn(rc_up)) {
        double rcab[LEVELS_MAX];
#pragma unroll
        for (int k = 0; k < LEVELS_MAX; ++k) rcab[k] = k <= lv ? fmax(me.rc[k], SR[(size_t)k * t.cap_M + j]) : 1.0;
        const double r = sqrt(q);
        const double w = level_share(r, lv, rcab);
        if (w > 0.0) {
            const double s = SM[j] * w / (q * r);
            ax += s * dx;
            ay += s * dy;
            az += s * dz;
        }
        em = a.emit && me.body < SB[j] && q < sq_rn(fmax(t.rc[(size_t)lv * t.cap_M + me.f], SR[(size_t)lv * t.cap_M + j]));
    }
    lv_emit(a, buf, fill, em, me.body, SB[j]);
}

// Sources [jb, je) of the group for the target: whole quads take the four sources' words in
// one scalar load per array.
__device__ __forceinline__ void lv_sources(const LevelTiles &t, const LevelKickArgs &a, const LvTarget &me, int lv,
                                           int jb, int je, double &ax, double &ay, double &az, int2 *buf,
                                           int &fill)
{
    CD *SX = (CD *)t.X;
    CD *SY = (CD *)t.Y;
    CD *SZ = (CD *)t.Z;
    CD *SR = (CD *)t.rc;
    const size_t up = (size_t)(lv - 1) * t.cap_M;
    int j = jb;
    for (; j + 4 <= je; j += 4) {
        double dx[4], dy[4], dz[4], ru[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            dx[v] = SX[j + v] - me.x;
            dy[v] = SY[j + v] - me.y;
            dz[v] = SZ[j + v] - me.z;
            ru[v] = SR[up + j + v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) lv_source(t, a, me, lv, j + v, dx[v], dy[v], dz[v], ru[v], ax, ay, az, buf, fill);
    }
    for (; j < je; ++j)
        lv_source(t, a, me, lv, j, SX[j] - me.x, SY[j] - me.y, SZ[j] - me.z, SR[up + j], ax, ay, az, buf, fill);
}

// Groups of more than one tile: one workgroup of W waves per target tile (tiles listed first
// in t.tl).
template <int W>
__global__ __launch_bounds__(LT_TILE *W) void level_tiles_kick_kernel(LevelTiles t, LevelKickArgs a)
{
    __shared__ double red[3][W][LT_TILE];
    __shared__ int near_tile[BIG_TILES_PER_GROUP];
    __shared__ int wave_cnt[W];
    __shared__ int2 pair_buf[W][LV_BUF];
    const int me = t.tl[blockIdx.x];
    const int4 tile = t.tiles[me]; // (group, first member, count, -)
    const int g = tile.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int o = t.off[g], nb = t.off[g + 1] - o;
    const int tf = t.tfirst[g], nt = t.tfirst[g + 1] - tf;
    const int lv = a.level;
    const LvTarget tg = lv_target(t, tile, lv);
    const double cut = t.cut2[g] * (1.0 + 0x1p-30);
    const double *bt = t.bb + (size_t)me * 8;
    const double tlx = bt[0], tly = bt[1], tlz = bt[2], thx = bt[3], thy = bt[4], thz = bt[5];
    // source tiles of the group in reach: one test per thread (in passes of W * 64 tiles),
    // ordered compaction
    int n_near = 0;
    for (int t0 = 0; t0 < nt; t0 += W * LT_TILE) {
        bool near = false;
        const int tt = t0 + (int)threadIdx.x;
        if (tt < nt) {
            const double *bs = t.bb + (size_t)(tf + tt) * 8;
            const double gx = fmax(0.0, fmax(bs[0] - thx, tlx - bs[3]));
            const double gy = fmax(0.0, fmax(bs[1] - thy, tly - bs[4]));
            const double gz = fmax(0.0, fmax(bs[2] - thz, tlz - bs[5]));
            near = (gx * gx + gy * gy) + gz * gz <= cut;
        }
        const unsigned long long bal = __ballot(near);
        if (lane == 0) wave_cnt[wave] = __popcll(bal);
        __syncthreads();
        int base = n_near;
        for (int w = 0; w < W; ++w) {
            if (w < wave) base += wave_cnt[w];
            n_near += wave_cnt[w];
        }
        if (near) near_tile[base + __popcll(bal & ((1ull << lane) - 1))] = tt;
        __syncthreads();
    }
    int2 *buf = pair_buf[wave];
    int fill = 0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int u = wave; u < 4 * n_near; u += W) {
        const int st = near_tile[u >> 2];
        const int jb = o + LT_TILE * st + 16 * (u & 3), je = min(jb + 16, o + nb);
        lv_sources(t, a, tg, lv, jb, je, ax, ay, az, buf, fill);
    }
    lv_flush(a, buf, fill);
    red[0][wave][lane] = ax;
    red[1][wave][lane] = ay;
    red[2][wave][lane] = az;
    __syncthreads();
    if (wave != 0 || !tg.valid) return;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int w = 0; w < W; ++w) {
        sx += red[0][w][lane];
        sy += red[1][w][lane];
        sz += red[2][w][lane];
    }
    a.vx[tg.body] += a.tau * sx;
    a.vy[tg.body] += a.tau * sy;
    a.vz[tg.body] += a.tau * sz;
}

// Groups of one tile (up to 64 members): one wave per group, its members the sources in order.
__global__ __launch_bounds__(LT_TILE) void level_tile_one_kernel(LevelTiles t, LevelKickArgs a)
{
    __shared__ int2 buf[LV_BUF];
    const int4 tile = t.tiles[t.tl[t.n_multi + blockIdx.x]];
    const LvTarget tg = lv_target(t, tile, a.level);
    int fill = 0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    lv_sources(t, a, tg, a.level, tile.y, tile.y + tile.z, ax, ay, az, buf, fill);
    lv_flush(a, buf, fill);
    if (!tg.valid) return;
    a.vx[tg.body] += a.tau * ax;
    a.vy[tg.body] += a.tau * ay;
    a.vz[tg.body] += a.tau * az;
}

} // namespace

hipError_t launch_level_tiles_setup(const Layout &L, const LevelTiles &t, const double *m, const double *rc0,
                                    const double *rcl, int level, hipStream_t stream)
{
    if (t.G == 0 || t.n_tiles == 0) return hipSuccess;
    level_cut_clear_kernel<<<(t.G + 255) / 256, 256, 0, stream>>>(t.cut2, t.G);
    level_tiles_setup_kernel<<<t.n_tiles, 64, 0, stream>>>(t, L.sys_of, L.sys_off, L.n_massive, m, rc0, rcl,
                                                           L.n_total, level);
    return hipGetLastError();
}

hipError_t launch_level_kick(const LevelTiles &t, const LevelKickArgs &a, const double *x, const double *y,
                             const double *z, int waves, hipStream_t stream)
{
    if (t.n_tiles == 0) return a.emit ? hipMemsetAsync(a.pair_count, 0, sizeof(int32_t), stream) : hipSuccess;
    level_tiles_pos_kernel<<<t.n_tiles, 64, 0, stream>>>(t, x, y, z, a.emit ? a.pair_count : nullptr);
    if (t.n_multi > 0) {
        if (waves == 16)
            level_tiles_kick_kernel<16><<<t.n_multi, LT_TILE * 16, 0, stream>>>(t, a);
        else if (waves == 8)
            level_tiles_kick_kernel<8><<<t.n_multi, LT_TILE * 8, 0, stream>>>(t, a);
        else
            return hipErrorInvalidValue;
    }
    if (t.n_tiles > t.n_multi) level_tile_one_kernel<<<t.n_tiles - t.n_multi, LT_TILE, 0, stream>>>(t, a);
    return hipGetLastError();
}

} // namespace genga
