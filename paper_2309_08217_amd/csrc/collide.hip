// Collisions as perfect mergers, and removal by distance to the star (Brasser et al. 2023,
// Sect. 2).  Detection: an encounter pair of two live bodies collides when its straight-line
// relative motion over the drift comes within R_i + R_j (closest approach t* clamped to
// [0, dt]); found at the start of the drift from the kick's encounter list.  After the drift
// the colliding pairs merge in ascending (i, j) order, a pair with an already merged body
// being skipped: the lower index keeps the summed mass, the mass-weighted position and velocity
// and the summed volume, the other gets m = 0 and status 1.  Then every live body closer to the
// star than r_min or farther than r_max gets m = 0 and status 2.  Collisions are rare, so the
// merging runs in one thread, in a fixed order.
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

// One thread: order the colliding pairs, merge them, clear the count for the next drift.
__global__ __launch_bounds__(64) void collide_merge_kernel(CollideArgs c, double *x, double *y, double *z,
                                                           double *vx, double *vy, double *vz)
{
    if (threadIdx.x != 0) return;
    const int n = min(*c.count, c.cap);
    int32_t *L = c.list;
    for (int a = 1; a < n; ++a) { // insertion sort by (i, j)
        const int i = L[2 * a], j = L[2 * a + 1];
        int b = a - 1;
        while (b >= 0 && (L[2 * b] > i || (L[2 * b] == i && L[2 * b + 1] > j))) {
            L[2 * b + 2] = L[2 * b];
            L[2 * b + 3] = L[2 * b + 1];
            --b;
        }
        L[2 * b + 2] = i;
        L[2 * b + 3] = j;
    }
    for (int a = 0; a < n; ++a) {
        const int i = L[2 * a], j = L[2 * a + 1];
        if (c.status[i] || c.status[j]) continue;
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
    *c.count = 0;
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

__global__ __launch_bounds__(256) void gather_kernel(const int32_t *idx, int n, const double *src, double *dst)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) dst[k] = src[idx[k]];
}

} // namespace

hipError_t launch_gather(const int32_t *idx, int n, const double *src, double *dst, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    gather_kernel<<<(n + 255) / 256, 256, 0, stream>>>(idx, n, src, dst);
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
    collide_merge_kernel<<<1, 64, 0, stream>>>(c, x, y, z, vx, vy, vz);
    if (n_total > 0) collide_remove_kernel<<<(n_total + 255) / 256, 256, 0, stream>>>(c, n_total, x, y, z);
    return hipGetLastError();
}

} // namespace genga
