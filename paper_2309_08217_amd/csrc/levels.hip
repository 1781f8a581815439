// Kicks of the intermediate levels of the hierarchical step (Brasser et al. 2023, Sect. 1:
// symplectic levels with reduced steps between the level-0 step and the Bulirsch-Stoer step).
// Level l integrates each group of level l-1 in Strang sub-steps; its kick carries the share
// W_l K_l of the Newtonian pair force, W_l = prod_{k<l} (1 - K_k), K_k the changeover of
// level k's critical radius, and the same pass lists the pairs of the group closer than the
// level's critical radius (the next level's groups).  FP64 throughout: these are
// close-encounter forces.
//
// One lane per member of the parent groups; it sums over the members of its own group in
// member order (the group's members are listed by ascending body index).  The groups are
// those of a level's encounter pairs, so a lane's loop is as long as its group; the launch
// covers every member of every parent group at once.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

// Level weight of a pair with separation r = q * rq: W_l K_l, or 0 when the pair lies beyond
// level l-1's radius (where W_l vanishes).  rc0 / rcj: the pair's radii of every level.
__device__ __forceinline__ double level_weight(double r, int l, const double *rcab)
{
    double w = 1.0;
    for (int k = 0; k < l; ++k) w *= 1.0 - changeover_k((r - 0.1 * rcab[k]) / (0.9 * rcab[k]));
    return w * changeover_k((r - 0.1 * rcab[l]) / (0.9 * rcab[l]));
}

__global__ __launch_bounds__(256) void level_kick_kernel(LevelKickArgs a)
{
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const bool act = k < a.n_mem;
    const int kk = act ? k : 0;
    const int i = a.mem[kk];
    const int g = a.mgrp[kk];
    const int gb = a.gs[g], ge = a.gs[g + 1];
    const int si = a.sys_of[i];
    const bool ti = i - a.sys_off[si] >= a.n_massive[si];
    const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
    double rci[LEVELS_MAX];
    rci[0] = a.rc0[i];
    for (int l = 1; l <= a.level; ++l) rci[l] = a.rcl[(size_t)(l - 1) * a.n_total + i];
    // pairs farther than level (l-1)'s radius carry no weight here; the radii do not grow with
    // the level, so that radius bounds the pairs to evaluate
    double sx = 0.0, sy = 0.0, sz = 0.0;
    const int n_it = act ? ge - gb : 0;
    // the wave runs as many iterations as its longest group
    int n_max = n_it;
    for (int o = 32; o > 0; o >>= 1) n_max = max(n_max, __shfl_xor(n_max, o, 64));
    for (int t = 0; t < n_max; ++t) {
        bool em = false;
        int j = i;
        if (t < n_it) {
            j = a.mem[gb + t];
            const int sj = a.sys_of[j];
            const bool tj = j - a.sys_off[sj] >= a.n_massive[sj];
            if (j != i && !(ti && tj)) {
                const double dx = a.x[j] - xi, dy = a.y[j] - yi, dz = a.z[j] - zi;
                const double q = sep2_rn(dx, dy, dz);
                double rcab[LEVELS_MAX];
                rcab[0] = fmax(rci[0], a.rc0[j]);
                for (int l = 1; l <= a.level; ++l)
                    rcab[l] = fmax(rci[l], a.rcl[(size_t)(l - 1) * a.n_total + j]);
                if (q < sq_rn(rcab[a.level - 1])) {
                    const double r = sqrt(q);
                    const double w = level_weight(r, a.level, rcab);
                    if (w > 0.0) {
                        const double s = a.m[j] * w / (q * r);
                        sx += s * dx;
                        sy += s * dy;
                        sz += s * dz;
                    }
                    em = a.emit && i < j && q < sq_rn(rcab[a.level]);
                }
            }
        }
        // the level's pairs: one counter update per wave and iteration
        const unsigned long long m = __ballot(em);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(a.pair_count, __popcll(m));
            base = __shfl(base, leader, 64);
            if (em) {
                const int idx = base + __popcll(m & ((1ull << lane) - 1));
                if (idx < a.pair_cap) {
                    a.pairs[2 * idx] = i;
                    a.pairs[2 * idx + 1] = j;
                } else {
                    atomicOr(a.flags, FLAG_CAPACITY);
                }
            }
        }
    }
    if (act) {
        a.vx[i] += a.tau * sx;
        a.vy[i] += a.tau * sy;
        a.vz[i] += a.tau * sz;
    }
}

} // namespace

hipError_t launch_level_kick(const LevelKickArgs &a, hipStream_t stream)
{
    if (a.n_mem <= 0) return hipSuccess;
    level_kick_kernel<<<(a.n_mem + 255) / 256, 256, 0, stream>>>(a);
    return hipGetLastError();
}

} // namespace genga
