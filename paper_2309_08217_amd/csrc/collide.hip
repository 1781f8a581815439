// Collisions as perfect mergers, and removal by distance to the star (Brasser et al. 2023,
// Sect. 2).  Detection: an encounter pair of two live bodies collides when its straight-line
// relative motion over the drift comes within R_i + R_j (closest approach t* clamped to
// [0, dt]); found at the start of the drift from the kick's encounter list.  After the drift
// the colliding pairs merge in ascending (i, j) order, a pair with an already merged body
// being skipped: the lower index keeps the summed mass, the mass-weighted position and velocity
// and the summed volume, the other gets m = 0 and status 1.  Then every live body closer to the
// star than r_min or farther than r_max gets m = 0 and status 2.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

__global__ __launch_bounds__(256) void collide_check_kernel(CollideArgs c, const int32_t *pairs,
                                                            const int32_t *pair_count, int32_t pair_cap,
                                                            const double *x, const double *y, const double *z,
                                                            const double *vx, const double *vy, const double *vz,
                                                            double dt)
{
    const int np = min(*pair_count, pair_cap);
    for (int p = blockIdx.x * 256 + threadIdx.x; p < np; p += gridDim.x * 256) {
        const int i = pairs[2 * p], j = pairs[2 * p + 1];
        if (c.status[i] || c.status[j]) continue;
        const double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        const double ux = vx[j] - vx[i], uy = vy[j] - vy[i], uz = vz[j] - vz[i];
        const double uu = sep2_rn(ux, uy, uz);
        double t = 0.0;
        if (uu > 0.0) {
#pragma clang fp contract(off)
            t = -((dx * ux + dy * uy) + dz * uz) / uu;
            t = fmin(fmax(t, 0.0), dt);
        }
        double ex, ey, ez;
        {
#pragma clang fp contract(off)
            ex = dx + t * ux;
            ey = dy + t * uy;
            ez = dz + t * uz;
        }
        const double rs = c.radius[i] + c.radius[j];
        if (sep2_rn(ex, ey, ez) < sq_rn(rs)) {
            const int k = atomicAdd(c.count, 1);
            if (k < c.cap) {
                c.list[2 * k] = i;
                c.list[2 * k + 1] = j;
            } else {
                atomicOr(c.flags, FLAG_CAPACITY);
            }
        }
    }
}

// Merge of the colliding pairs in ascending (i, j) order, one workgroup:
//  1. the pairs are sorted in LDS (bitonic);
//  2. one lane walks them in order and decides which merge: a pair is skipped when one of its
//     bodies was absorbed by an earlier merge (an LDS hash set of the absorbed bodies) or was
//     not live; the walk touches LDS only;
//  3. the merges run in parallel over the absorbing bodies.  An absorbing body i is never
//     absorbed itself (a pair (k, i) sorts before every (i, j), so it would have stopped them),
//     and all pairs (i, .) are adjacent in the sorted list: the lane holding the first of them
//     applies i's merges in order, so each body's arithmetic is the sequential one.
// The list's count is cleared for the next drift.
constexpr int MERGE_THREADS = 1024;
constexpr int DEAD_SLOTS = 2 * COLLIDE_CAP;         // open addressing, load factor <= 1/2
constexpr uint64_t KEY_APPLIED = 1ull << 63;
constexpr uint64_t KEY_BLOCKED = 1ull << 62;        // a body was not live before the merges
constexpr uint64_t KEY_PAIR = (1ull << 62) - 1;

__device__ __forceinline__ int dead_slot(int32_t b)
{
    return (int)(((uint32_t)b * 2654435761u) >> 19) & (DEAD_SLOTS - 1);
}

__device__ __forceinline__ bool dead_has(const int32_t *set, int32_t b)
{
    for (int h = dead_slot(b);; h = (h + 1) & (DEAD_SLOTS - 1)) {
        if (set[h] == b) return true;
        if (set[h] < 0) return false;
    }
}

__device__ __forceinline__ void dead_add(int32_t *set, int32_t b)
{
    int h = dead_slot(b);
    while (set[h] >= 0) h = (h + 1) & (DEAD_SLOTS - 1);
    set[h] = b;
}

__global__ __launch_bounds__(MERGE_THREADS) void collide_merge_kernel(CollideArgs c, double *x, double *y,
                                                                      double *z, double *vx, double *vy,
                                                                      double *vz)
{
    static_assert((COLLIDE_CAP & (COLLIDE_CAP - 1)) == 0 && DEAD_SLOTS == 8192, "power-of-two tables");
    __shared__ uint64_t key[COLLIDE_CAP];
    __shared__ int32_t dead[DEAD_SLOTS];
    const int tid = threadIdx.x;
    const int n = min(*c.count, c.cap);
    __syncthreads();
    if (n > 0) {
        int npow = 1;
        while (npow < n) npow <<= 1;
        for (int k = tid; k < npow; k += MERGE_THREADS) {
            uint64_t v = ~0ull;
            if (k < n) {
                const int i = c.list[2 * k], j = c.list[2 * k + 1];
                v = ((uint64_t)(uint32_t)i << 32) | (uint32_t)j;
                if (c.status[i] || c.status[j]) v |= KEY_BLOCKED;
            }
            key[k] = v;
        }
        for (int k = tid; k < DEAD_SLOTS; k += MERGE_THREADS) dead[k] = -1;
        __syncthreads();
        // sort by (i, j); the flag bits sit above both indices, and no pair is listed twice
        for (int len = 2; len <= npow; len <<= 1) {
            for (int half = len >> 1; half > 0; half >>= 1) {
                for (int t = tid; t < npow; t += MERGE_THREADS) {
                    const int p = t ^ half;
                    if (p > t) {
                        const uint64_t a = key[t], b = key[p];
                        const bool up = (t & len) == 0;
                        if (((a & KEY_PAIR) > (b & KEY_PAIR)) == up) {
                            key[t] = b;
                            key[p] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (tid == 0) {
            for (int a = 0; a < n; ++a) {
                const uint64_t v = key[a];
                const int32_t i = (int32_t)((v & KEY_PAIR) >> 32), j = (int32_t)(v & 0xffffffffu);
                if ((v & KEY_BLOCKED) || dead_has(dead, i) || dead_has(dead, j)) continue;
                dead_add(dead, j);
                key[a] = v | KEY_APPLIED;
            }
        }
        __syncthreads();
        for (int a = tid; a < n; a += MERGE_THREADS) {
            const int32_t i = (int32_t)((key[a] & KEY_PAIR) >> 32);
            if (a > 0 && (int32_t)((key[a - 1] & KEY_PAIR) >> 32) == i) continue;
            for (int b = a; b < n && (int32_t)((key[b] & KEY_PAIR) >> 32) == i; ++b) {
                if (!(key[b] & KEY_APPLIED)) continue;
                const int32_t j = (int32_t)(key[b] & 0xffffffffu);
                const double mi = c.mass[i], mj = c.mass[j], mt = mi + mj;
                if (mt > 0.0) {
#pragma clang fp contract(off)
                    x[i] = (mi * x[i] + mj * x[j]) / mt;
                    y[i] = (mi * y[i] + mj * y[j]) / mt;
                    z[i] = (mi * z[i] + mj * z[j]) / mt;
                    vx[i] = (mi * vx[i] + mj * vx[j]) / mt;
                    vy[i] = (mi * vy[i] + mj * vy[j]) / mt;
                    vz[i] = (mi * vz[i] + mj * vz[j]) / mt;
                }
                c.mass[i] = mt;
                {
#pragma clang fp contract(off)
                    const double ri = c.radius[i], rj = c.radius[j];
                    c.radius[i] = cbrt(ri * ri * ri + rj * rj * rj);
                }
                c.mass[j] = 0.0;
                c.status[j] = 1;
            }
        }
    }
    if (tid == 0) *c.count = 0;
}

__global__ __launch_bounds__(256) void collide_remove_kernel(CollideArgs c, int n, const double *x,
                                                             const double *y, const double *z)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n || c.status[i]) return;
    const double r2 = sep2_rn(x[i], y[i], z[i]);
    if (r2 < sq_rn(c.r_min) || r2 > sq_rn(c.r_max)) {
        c.mass[i] = 0.0;
        c.status[i] = 2;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const int32_t *idx, int n, const T *src, T *dst)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) dst[k] = src[idx[k]];
}

} // namespace

hipError_t launch_gather(const int32_t *idx, int n, const double *src, double *dst, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    gather_kernel<double><<<(n + 255) / 256, 256, 0, stream>>>(idx, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_gather(const int32_t *idx, int n, const int32_t *src, int32_t *dst, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    gather_kernel<int32_t><<<(n + 255) / 256, 256, 0, stream>>>(idx, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_collide_check(const CollideArgs &c, const int32_t *pairs, const int32_t *pair_count,
                                int32_t pair_cap, const double *x, const double *y, const double *z,
                                const double *vx, const double *vy, const double *vz, double dt,
                                hipStream_t stream)
{
    const int blocks = std::max(1, std::min(1024, (pair_cap + 255) / 256));
    collide_check_kernel<<<blocks, 256, 0, stream>>>(c, pairs, pair_count, pair_cap, x, y, z, vx, vy, vz, dt);
    return hipGetLastError();
}

hipError_t launch_collide_resolve(const CollideArgs &c, int n_total, double *x, double *y, double *z, double *vx,
                                  double *vy, double *vz, hipStream_t stream)
{
    collide_merge_kernel<<<1, MERGE_THREADS, 0, stream>>>(c, x, y, z, vx, vy, vz);
    if (n_total > 0) collide_remove_kernel<<<(n_total + 255) / 256, 256, 0, stream>>>(c, n_total, x, y, z);
    return hipGetLastError();
}

} // namespace genga
