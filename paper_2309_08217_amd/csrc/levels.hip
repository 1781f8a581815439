// Kicks of the intermediate levels of the hierarchical step (Brasser et al. 2023, Sect. 1:
// symplectic levels with reduced steps between the level-0 step and the Bulirsch-Stoer step).
// Level l integrates each group of level l-1 in Strang sub-steps; its kick carries the share
// W_l K_l of the Newtonian pair force, W_l = prod_{k<l} (1 - K_k), K_k the changeover of
// level k's critical radius, and the same pass lists the pairs of the group closer than the
// level's critical radius (the next level's groups).  FP64 throughout: these are
// close-encounter forces.
//
// Layout as in the grid-wide Bulirsch-Stoer: the members of the parent groups are ordered by
// ring and azimuth (by the host, once per level interval) and cut into tiles of 64; a
// workgroup of 16 waves takes one target tile, lists the source tiles of the group whose box
// lies within the group's largest level-(l-1) radius of the target tile's box (no pair beyond
// that radius carries weight at level l), and deals their quarters out to its waves.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

constexpr int LT_TILE = 64;
constexpr int LT_WAVES = 16;

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
                                                             const double *z)
{
    const int me = blockIdx.x;
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

__device__ __forceinline__ double level_share(double r, int l, const double *rcab)
{
    double w = 1.0;
    for (int k = 0; k < l; ++k) w *= 1.0 - changeover_k((r - 0.1 * rcab[k]) / (0.9 * rcab[k]));
    return w * changeover_k((r - 0.1 * rcab[l]) / (0.9 * rcab[l]));
}

__global__ __launch_bounds__(LT_TILE *LT_WAVES) void level_tiles_kick_kernel(LevelTiles t, LevelKickArgs a)
{
    __shared__ double red[3][LT_WAVES][LT_TILE];
    __shared__ int near_tile[BIG_TILES_PER_GROUP];
    __shared__ int wave_cnt[LT_WAVES];
    const int me = blockIdx.x;
    const int4 tile = t.tiles[me]; // (group, first member, count, -)
    const int g = tile.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int o = t.off[g], nb = t.off[g + 1] - o;
    const int tf = t.tfirst[g], nt = t.tfirst[g + 1] - tf;
    const int lv = a.level;
    const bool valid = lane < tile.z;
    const int fa = tile.y + (valid ? lane : 0);
    const int body_a = t.body[fa];
    const double xa = t.X[fa], ya = t.Y[fa], za = t.Z[fa];
    const bool testa = t.test[fa] != 0;
    double rca[LEVELS_MAX];
    for (int k = 0; k <= lv; ++k) rca[k] = t.rc[(size_t)k * t.cap_M + fa];
    const double cut = t.cut2[g] * (1.0 + 0x1p-30);
    const double *bt = t.bb + (size_t)me * 8;
    const double tlx = bt[0], tly = bt[1], tlz = bt[2], thx = bt[3], thy = bt[4], thz = bt[5];
    // source tiles of the group in reach: one test per thread, ordered compaction
    bool near = false;
    const int tt = threadIdx.x;
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
    int base = 0, n_near = 0;
    for (int w = 0; w < LT_WAVES; ++w) {
        if (w < wave) base += wave_cnt[w];
        n_near += wave_cnt[w];
    }
    if (near) near_tile[base + __popcll(bal & ((1ull << lane) - 1))] = tt;
    static_assert(BIG_TILES_PER_GROUP <= LT_TILE * LT_WAVES, "one thread per source tile");
    __syncthreads();
    CD *SX = (CD *)t.X;
    CD *SY = (CD *)t.Y;
    CD *SZ = (CD *)t.Z;
    CD *SM = (CD *)t.mass;
    CD *SR = (CD *)t.rc;
    CI *ST = (CI *)t.test;
    CI *SB = (CI *)t.body;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int u = wave; u < 4 * n_near; u += LT_WAVES) {
        const int st = near_tile[u >> 2];
        const int jb = o + LT_TILE * st + 16 * (u & 3), je = min(jb + 16, o + nb);
        // one source: its term if inside level (l-1)'s radius, and the level's pair
        auto source = [&](int j, double dx, double dy, double dz, double rcj_up) {
            const double q = sep2_rn(dx, dy, dz);
            const double rc_up = fmax(rca[lv - 1], rcj_up);
            bool em = false;
            if (valid && j != fa && !(testa && ST[j] != 0) && q < sq_rn(rc_up)) {
                double rcab[LEVELS_MAX];
                for (int k = 0; k <= lv; ++k) rcab[k] = fmax(rca[k], SR[(size_t)k * t.cap_M + j]);
                const double r = sqrt(q);
                const double w = level_share(r, lv, rcab);
                if (w > 0.0) {
                    const double s = SM[j] * w / (q * r);
                    ax += s * dx;
                    ay += s * dy;
                    az += s * dz;
                }
                em = a.emit && body_a < SB[j] && q < sq_rn(rcab[lv]);
            }
            // the level's pairs: one counter update per wave and source
            const unsigned long long m = __ballot(em);
            if (m) {
                const int leader = __ffsll((long long)m) - 1;
                int pb = 0;
                if (lane == leader) pb = atomicAdd(a.pair_count, __popcll(m));
                pb = __shfl(pb, leader, 64);
                if (em) {
                    const int idx = pb + __popcll(m & ((1ull << lane) - 1));
                    if (idx < a.pair_cap) {
                        a.pairs[2 * idx] = body_a;
                        a.pairs[2 * idx + 1] = SB[j];
                    } else {
                        atomicOr(a.flags, FLAG_CAPACITY);
                    }
                }
            }
        };
        // whole quads: the four sources' words in one scalar load per array
        int j = jb;
        for (; j + 4 <= je; j += 4) {
            double dx[4], dy[4], dz[4], ru[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                dx[v] = SX[j + v] - xa;
                dy[v] = SY[j + v] - ya;
                dz[v] = SZ[j + v] - za;
                ru[v] = SR[(size_t)(lv - 1) * t.cap_M + j + v];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) source(j + v, dx[v], dy[v], dz[v], ru[v]);
        }
        for (; j < je; ++j)
            source(j, SX[j] - xa, SY[j] - ya, SZ[j] - za, SR[(size_t)(lv - 1) * t.cap_M + j]);
    }
    red[0][wave][lane] = ax;
    red[1][wave][lane] = ay;
    red[2][wave][lane] = az;
    __syncthreads();
    if (wave != 0 || !valid) return;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int w = 0; w < LT_WAVES; ++w) {
        sx += red[0][w][lane];
        sy += red[1][w][lane];
        sz += red[2][w][lane];
    }
    a.vx[body_a] += a.tau * sx;
    a.vy[body_a] += a.tau * sy;
    a.vz[body_a] += a.tau * sz;
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
                             const double *z, hipStream_t stream)
{
    if (t.n_tiles == 0) return hipSuccess;
    level_tiles_pos_kernel<<<t.n_tiles, 64, 0, stream>>>(t, x, y, z);
    level_tiles_kick_kernel<<<t.n_tiles, LT_TILE * LT_WAVES, 0, stream>>>(t, a);
    return hipGetLastError();
}

} // namespace genga
