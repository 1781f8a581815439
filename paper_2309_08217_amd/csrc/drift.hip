// Drift part of the hybrid symplectic step (Brasser et al. 2023, Sect. 1), all FP64:
//  * Sun drift: r_i += tau * (sum_j m_j v_j) / Mstar (democratic heliocentric split);
//  * Kepler drift of every body not in a close encounter, by universal variables
//    (Stumpff functions, safeguarded Newton on the universal Kepler equation);
//  * close-encounter step: the encounter pairs are joined into groups (connected components,
//    one workgroup, union-find in global memory, members sorted in LDS), and each group is
//    integrated over dt by Gragg-Bulirsch-Stoer under the Sun's force plus the (1 - K) share
//    of the members' mutual forces; the Kepler kernel then writes the group results back.
#include "genga_internal.h"

namespace genga {

namespace {

__device__ __forceinline__ double sep2_rn(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    return (a + b) + c;
}

__device__ __forceinline__ double sq_rn(double a)
{
#pragma clang fp contract(off)
    return a * a;
}

__device__ __forceinline__ double changeover_k(double y)
{
    if (y <= 0.0) return 0.0;
    if (y >= 1.0) return 1.0;
    double y2 = y * y;
    return y2 / (2.0 * y2 - 2.0 * y + 1.0);
}

// ------------------------------------------------------------------------------------------
// Sun drift in two launches over chunks of one system: partial momenta per chunk (fixed-order
// block reduction), then every chunk adds its system's partials in chunk order and shifts
// its positions.  Deterministic.
// ------------------------------------------------------------------------------------------
constexpr int SUN_THREADS = 256;

__global__ __launch_bounds__(SUN_THREADS) void momentum_kernel(const Chunk *chunks, const double *m,
                                                               const double *vx, const double *vy,
                                                               const double *vz, double *mom_part)
{
    __shared__ double red[3][SUN_THREADS / 64];
    const Chunk c = chunks[blockIdx.x];
    double px = 0.0, py = 0.0, pz = 0.0;
    for (int i = c.b + threadIdx.x; i < c.e; i += SUN_THREADS) {
        px += m[i] * vx[i];
        py += m[i] * vy[i];
        pz += m[i] * vz[i];
    }
    for (int o = 32; o > 0; o >>= 1) {
        px += __shfl_xor(px, o, 64);
        py += __shfl_xor(py, o, 64);
        pz += __shfl_xor(pz, o, 64);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[0][wave] = px;
        red[1][wave] = py;
        red[2][wave] = pz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double P[3] = {0.0, 0.0, 0.0};
        for (int w = 0; w < SUN_THREADS / 64; ++w)
            for (int q = 0; q < 3; ++q) P[q] += red[q][w];
        for (int q = 0; q < 3; ++q) mom_part[3 * (size_t)blockIdx.x + q] = P[q];
    }
}

__global__ __launch_bounds__(SUN_THREADS) void sun_shift_kernel(const Chunk *chunks,
                                                                const int32_t *chunk_first,
                                                                const double *mstar,
                                                                const double *mom_part, double tau,
                                                                double *x, double *y, double *z)
{
    __shared__ double red[3][SUN_THREADS / 64];
    const Chunk c = chunks[blockIdx.x];
    // the system's momentum: strided sums of the chunk partials, then a fixed tree
    double Px = 0.0, Py = 0.0, Pz = 0.0;
    for (int k = chunk_first[c.sys] + threadIdx.x; k < chunk_first[c.sys + 1]; k += SUN_THREADS) {
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
    Px = Py = Pz = 0.0;
    for (int w = 0; w < SUN_THREADS / 64; ++w) {
        Px += red[0][w];
        Py += red[1][w];
        Pz += red[2][w];
    }
    const double f = tau / mstar[c.sys];
    const double sx = f * Px, sy = f * Py, sz = f * Pz;
    for (int i = c.b + threadIdx.x; i < c.e; i += SUN_THREADS) {
        x[i] += sx;
        y[i] += sy;
        z[i] += sz;
    }
}

// ------------------------------------------------------------------------------------------
// Kepler drift by universal variables.
// ------------------------------------------------------------------------------------------

// Stumpff functions c2(z) = (1 - cos sqrt z)/z, c3(z) = (sqrt z - sin sqrt z)/z^(3/2)
// (hyperbolic forms for z < 0); series for |z| < 1.
__device__ void stumpff(double zz, double &c2, double &c3)
{
    if (fabs(zz) < 1.0) {
        // c2 = sum (-z)^k / (2k+2)!, c3 = sum (-z)^k / (2k+3)!
        double t2 = 0.5, t3 = 1.0 / 6.0;
        double s2 = t2, s3 = t3;
        for (int k = 1; k < 14; ++k) {
            t2 *= -zz / ((2.0 * k + 1.0) * (2.0 * k + 2.0));
            t3 *= -zz / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
            s2 += t2;
            s3 += t3;
        }
        c2 = s2;
        c3 = s3;
    } else if (zz > 0.0) {
        double sz = sqrt(zz);
        double h = sin(0.5 * sz);
        c2 = 2.0 * h * h / zz;
        c3 = (sz - sin(sz)) / (zz * sz);
    } else {
        double sz = sqrt(-zz);
        double h = sinh(0.5 * sz);
        c2 = 2.0 * h * h / (-zz);
        c3 = (sinh(sz) - sz) / (-zz * sz);
    }
}

// Advance (r, v) on the two-body orbit about mu by dt; returns false if not converged.
__device__ bool kepler_universal(double &x, double &y, double &z, double &vx, double &vy,
                                 double &vz, double mu, double dt)
{
    if (dt == 0.0) return true;
    const double r0 = sqrt(x * x + y * y + z * z);
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double sig = (x * vx + y * vy + z * vz) / sqrt(mu); // r0 . v0 / sqrt(mu)
    const double alpha = 2.0 / r0 - v2 / mu;                   // 1 / a
    const double smu = sqrt(mu);
    // universal Kepler equation F(chi) = sig chi^2 c2 + (1 - alpha r0) chi^3 c3 + r0 chi - sqrt(mu) dt
    // F'(chi) = r(chi) > 0.  Bracket the root, then safeguarded Newton.
    double chi = (alpha > 0.0) ? smu * dt * alpha : smu * dt / r0;
    double lo, hi;
    {
        // expand a bracket around the first guess
        double step = fabs(chi) + (alpha > 0.0 ? 1.0 / sqrt(alpha) : r0);
        lo = chi - step;
        hi = chi + step;
        for (int k = 0; k < 200; ++k) {
            double c2, c3, zz = alpha * lo * lo;
            stumpff(zz, c2, c3);
            double F = sig * lo * lo * c2 + (1.0 - alpha * r0) * lo * lo * lo * c3 + r0 * lo - smu * dt;
            if (F <= 0.0) break;
            lo -= step;
            step *= 2.0;
        }
        step = fabs(hi - chi) + 1e-300;
        for (int k = 0; k < 200; ++k) {
            double c2, c3, zz = alpha * hi * hi;
            stumpff(zz, c2, c3);
            double F = sig * hi * hi * c2 + (1.0 - alpha * r0) * hi * hi * hi * c3 + r0 * hi - smu * dt;
            if (F >= 0.0) break;
            hi += step;
            step *= 2.0;
        }
    }
    bool ok = false;
    double c2 = 0.5, c3 = 1.0 / 6.0, rr = r0;
    for (int it = 0; it < 100; ++it) {
        const double zz = alpha * chi * chi;
        stumpff(zz, c2, c3);
        const double chi2 = chi * chi;
        const double F = sig * chi2 * c2 + (1.0 - alpha * r0) * chi2 * chi * c3 + r0 * chi - smu * dt;
        rr = sig * chi * (1.0 - zz * c3) + (1.0 - alpha * r0) * chi2 * c2 + r0;
        if (F > 0.0) hi = chi; else lo = chi;
        const double step = F / rr;
        if (fabs(step) <= 1e-15 * fabs(chi) || hi - lo <= 4e-16 * fabs(chi)) {
            // converged: take the last Newton correction (it may sit on the bracket edge)
            chi -= step;
            ok = true;
            break;
        }
        double nx = chi - step;
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        chi = nx;
    }
    const double zz = alpha * chi * chi;
    stumpff(zz, c2, c3);
    const double chi2 = chi * chi;
    const double f = 1.0 - chi2 / r0 * c2;
    const double g = dt - chi2 * chi / smu * c3;
    const double nxp = f * x + g * vx, nyp = f * y + g * vy, nzp = f * z + g * vz;
    const double r = sqrt(nxp * nxp + nyp * nyp + nzp * nzp);
    const double fd = smu / (r * r0) * chi * (zz * c3 - 1.0);
    const double gd = 1.0 - chi2 / r * c2;
    const double nvx = fd * x + gd * vx, nvy = fd * y + gd * vy, nvz = fd * z + gd * vz;
    x = nxp;
    y = nyp;
    z = nzp;
    vx = nvx;
    vy = nvy;
    vz = nvz;
    return ok;
}

__global__ __launch_bounds__(64) void kepler_kernel(int n_total, const int32_t *sys_of,
                                                     const double *mstar, double *x, double *y,
                                                     double *z, double *vx, double *vy,
                                                     double *vz, double dt, int32_t *member_slot,
                                                     const double *bs_out, int32_t *flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const int slot = member_slot[i];
    if (slot >= 0) {
        // body integrated by the encounter step: take its result, clear the slot
        const double *o = bs_out + 6 * (size_t)slot;
        x[i] = o[0];
        y[i] = o[1];
        z[i] = o[2];
        vx[i] = o[3];
        vy[i] = o[4];
        vz[i] = o[5];
        member_slot[i] = -1;
        return;
    }
    double px = x[i], py = y[i], pz = z[i], ux = vx[i], uy = vy[i], uz = vz[i];
    const bool ok = kepler_universal(px, py, pz, ux, uy, uz, mstar[sys_of[i]], dt);
    if (!ok) atomicOr(flags, FLAG_KEPLER);
    x[i] = px;
    y[i] = py;
    z[i] = pz;
    vx[i] = ux;
    vy[i] = uy;
    vz[i] = uz;
}

// ------------------------------------------------------------------------------------------
// Encounter groups: one workgroup.  lab[] (init -1) and mark[] (init 0) are global arrays
// over all bodies that this kernel leaves clean again for the next step.
// Output: members[] sorted by (group root, body), group_start[g] (g < n_groups, plus an end
// sentinel), member_slot[body] = position in members[].
// ------------------------------------------------------------------------------------------
constexpr int CE_THREADS = 1024;

// lab[] is read with device-coherent atomic loads, so the hooks made by other waves through
// atomicMin (performed in L2) are seen without cache maintenance.
__device__ __forceinline__ int lab_load(int32_t *lab, int a)
{
    return __hip_atomic_load(&lab[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_root(int32_t *lab, int a)
{
    int r = lab_load(lab, a);
    while (r != a) {
        a = r;
        r = lab_load(lab, a);
    }
    return r;
}

__global__ __launch_bounds__(CE_THREADS) void ce_groups_kernel(
    const int32_t *pairs, const int32_t *pair_count, int32_t pair_cap, int32_t *lab, int32_t *mark,
    int32_t *members, int32_t *group_start, int32_t *n_groups, int32_t *member_slot, int32_t *flags)
{
    __shared__ uint64_t keys[CE_MAX_MEMBERS];
    __shared__ int32_t s_nmem;
    __shared__ int32_t s_changed;
    __shared__ int32_t s_ng;
    const int tid = threadIdx.x;
    const int np = min(*pair_count, pair_cap);
    if (tid == 0) {
        s_nmem = 0;
        s_ng = 0;
    }
    __syncthreads();
    if (np <= 0) {
        if (tid == 0) *n_groups = 0;
        return;
    }
    // collect distinct member bodies; each becomes its own root
    for (int p = tid; p < np; p += CE_THREADS) {
        for (int e = 0; e < 2; ++e) {
            const int b = pairs[2 * p + e];
            if (atomicCAS(&mark[b], 0, 1) == 0) {
                const int k = atomicAdd(&s_nmem, 1);
                if (k < CE_MAX_MEMBERS) keys[k] = (uint64_t)(uint32_t)b;
                __hip_atomic_store(&lab[b], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __syncthreads();
    const int nmem_all = s_nmem;
    const int nmem = min(nmem_all, CE_MAX_MEMBERS);
    if (nmem_all > CE_MAX_MEMBERS) {
        if (tid == 0) atomicOr(flags, FLAG_CAPACITY);
    }
    // union by hooking the larger root under the smaller until no pair spans two roots
    for (int round = 0; round < 4096; ++round) {
        if (tid == 0) s_changed = 0;
        __syncthreads();
        for (int p = tid; p < np; p += CE_THREADS) {
            int a = find_root(lab, pairs[2 * p]);
            int b = find_root(lab, pairs[2 * p + 1]);
            if (a != b) {
                const int lo = min(a, b), hi = max(a, b);
                atomicMin(&lab[hi], lo);
                s_changed = 1;
            }
        }
        __syncthreads();
        if (!s_changed) break;
        __syncthreads();
    }
    // sort members by (root, body) so each group is contiguous and in ascending order
    for (int k = tid; k < nmem; k += CE_THREADS) {
        const int b = (int)(keys[k] & 0xffffffffu);
        const int r = find_root(lab, b);
        keys[k] = ((uint64_t)(uint32_t)r << 32) | (uint32_t)b;
    }
    int npow = 1;
    while (npow < nmem) npow <<= 1;
    for (int k = nmem + tid; k < npow; k += CE_THREADS) keys[k] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int k = tid; k < npow; k += CE_THREADS) {
                const int partner = k ^ stride;
                if (partner > k) {
                    const bool up = (k & size) == 0;
                    const uint64_t a = keys[k], b = keys[partner];
                    if ((a > b) == up) {
                        keys[k] = b;
                        keys[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // write members and slots; number the groups with a chunked scan of the start flags
    __shared__ int32_t s_cnt[CE_THREADS / 64];
    const int per = (nmem + CE_THREADS - 1) / CE_THREADS;
    const int kb = min(tid * per, nmem), ke = min(kb + per, nmem);
    int nstart = 0;
    for (int k = kb; k < ke; ++k) {
        const int b = (int)(keys[k] & 0xffffffffu);
        members[k] = b;
        member_slot[b] = k;
        if (k == 0 || (keys[k - 1] >> 32) != (keys[k] >> 32)) ++nstart;
    }
    // exclusive scan of the per-thread start counts: in-wave shuffles, then the wave totals
    const int lane = tid & 63, wave = tid >> 6;
    int incl = nstart;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) s_cnt[wave] = incl;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < CE_THREADS / 64; ++w) {
            const int c = s_cnt[w];
            s_cnt[w] = acc;
            acc += c;
        }
        s_ng = acc;
    }
    __syncthreads();
    int g = s_cnt[wave] + incl - nstart;
    for (int k = kb; k < ke; ++k)
        if (k == 0 || (keys[k - 1] >> 32) != (keys[k] >> 32)) group_start[g++] = k;
    if (tid == 0) {
        group_start[s_ng] = nmem;
        *n_groups = s_ng;
    }
    // leave the marks clear for the next step (roots are re-initialised on marking)
    for (int p = tid; p < np; p += CE_THREADS) {
        mark[pairs[2 * p]] = 0;
        mark[pairs[2 * p + 1]] = 0;
    }
}

// ------------------------------------------------------------------------------------------
// Bulirsch-Stoer over dt: one wavefront per group, one member per lane.  Each lane keeps its
// member's state, midpoint sub-step values and extrapolation tableau in registers; the
// members' positions are exchanged through LDS for the pair forces; step decisions use
// wave-wide maxima, so the control flow is uniform.  Same method as the oracle: modified
// midpoint with n_k = 2k sub-steps (k = 1..8), polynomial extrapolation in h^2, accept when
// the last two diagonal entries agree to tol on the group's position / velocity scales,
// otherwise halve the step; after an accepted step the next one is twice as long.
// ------------------------------------------------------------------------------------------
constexpr int BS_LANES = 64;

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

struct LaneGroup {
    int a, nb;
    bool act;
    double m, rc, mstar;
    double (*sp)[BS_LANES]; // [3][64] positions of the members
    const double *sm, *src; // [64] masses and critical radii of the members
    bool test;              // this member is a test body (TP2)
    const int32_t *stest;   // [64] members that are test bodies
};

// dY/dt for this lane's member: Kepler term about the Sun plus the (1 - K) share of the
// Newtonian forces from the other members.  Every lane of the wave must call it.
__device__ void lane_deriv(const LaneGroup &g, const double y[6], double d[6])
{
    g.sp[0][g.a] = y[0];
    g.sp[1][g.a] = y[1];
    g.sp[2][g.a] = y[2];
    __syncthreads();
    const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    const double r = sqrt(r2);
    const double s = -g.mstar / (r2 * r);
    double ax = s * y[0], ay = s * y[1], az = s * y[2];
    for (int b = 0; b < g.nb; ++b) {
        if (b == g.a) continue;
        if (g.test && g.stest[b]) continue; // two test bodies do not interact
        const double dx = g.sp[0][b] - y[0], dy = g.sp[1][b] - y[1], dz = g.sp[2][b] - y[2];
        const double q = sep2_rn(dx, dy, dz);
        const double rcij = fmax(g.rc, g.src[b]);
        if (!(q < sq_rn(rcij))) continue;
        const double rr = sqrt(q);
        const double w = 1.0 - changeover_k((rr - 0.1 * rcij) / (0.9 * rcij));
        if (w == 0.0) continue;
        const double t = g.sm[b] * w / (q * rr);
        ax += t * dx;
        ay += t * dy;
        az += t * dz;
    }
    __syncthreads();
    if (g.act) {
        d[0] = y[3];
        d[1] = y[4];
        d[2] = y[5];
        d[3] = ax;
        d[4] = ay;
        d[5] = az;
    } else {
        for (int q = 0; q < 6; ++q) d[q] = 0.0;
    }
}

__device__ void lane_midpoint(const LaneGroup &g, const double y0[6], double H, int nsub, double out[6])
{
    const double h = H / nsub;
    double zm[6], zc[6], dd[6];
    lane_deriv(g, y0, dd);
    for (int q = 0; q < 6; ++q) {
        zm[q] = y0[q];
        zc[q] = y0[q] + h * dd[q];
    }
    for (int k = 1; k < nsub; ++k) {
        lane_deriv(g, zc, dd);
        for (int q = 0; q < 6; ++q) {
            const double t = zm[q] + 2.0 * h * dd[q];
            zm[q] = zc[q];
            zc[q] = t;
        }
    }
    lane_deriv(g, zc, dd);
    for (int q = 0; q < 6; ++q) out[q] = 0.5 * (zm[q] + zc[q] + h * dd[q]);
}

// Step reduction after a rejected step: 0.9 (tol/err)^(1/15) from the last column's error,
// kept within [1/50, 1/2].
__device__ __forceinline__ double shrink_factor(double err, double tol)
{
    const double f = 0.9 * pow(tol / err, 1.0 / (2 * BS_KMAX - 1));
    return fmax(0.02, fmin(0.5, f));
}

// Integrate this lane's member over dt (one lane per member, columns in sequence).  After a
// step accepted at column k the next step is doubled (k <= 4), kept (k = 5, 6) or halved
// (k = 7); a rejected step shrinks by shrink_factor.  Returns false (uniformly) if the step
// falls below dt * 2^-40 or more than 20000 steps are tried.
__device__ bool lane_bs(const LaneGroup &g, double Y[6], double dt, double tol)
{
    double t = 0.0, H = dt;
    int attempts = 0;
    while (t < dt) {
        const bool last = H >= (dt - t) * (1.0 - 0x1p-30); // ends the interval (exactly)
        if (last) H = dt - t;
        if (H < dt * 0x1p-40 || ++attempts > 20000) return false;
        const double sr = wave_max(g.act ? sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]) : 0.0);
        const double sv = wave_max(g.act ? sqrt(Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]) : 0.0);
        double T[BS_KMAX][6];
        int accepted = -1;
        double err_last = 0.0;
#pragma unroll
        for (int k = 0; k < BS_KMAX; ++k) {
            double est[6];
            lane_midpoint(g, Y, H, 2 * (k + 1), est);
            double err = 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                double prev = T[0][q]; // T(k-1, 0)
                double cur = est[q];   // T(k, 0)
                T[0][q] = cur;
                double last = cur;
#pragma unroll
                for (int l = 1; l <= k; ++l) {
                    const double ratio = (double)(k + 1) / (double)(k + 1 - l);
                    const double nxt = cur + (cur - prev) / (ratio * ratio - 1.0);
                    prev = T[l][q];
                    last = cur;
                    cur = nxt;
                    T[l][q] = cur;
                }
                if (k > 0) err = fmax(err, fabs(cur - last) / (q < 3 ? sr : sv));
            }
            if (k > 0) {
                err = wave_max(g.act ? err : 0.0);
                err_last = err;
                if (err <= tol) {
#pragma unroll
                    for (int q = 0; q < 6; ++q) Y[q] = T[k][q];
                    accepted = k;
                    break;
                }
            }
        }
        if (accepted >= 0) {
            t = last ? dt : t + H;
            if (accepted <= 4) H = 2.0 * H;
            else if (accepted == BS_KMAX - 1) H = 0.5 * H;
        } else {
            H = H * shrink_factor(err_last, tol);
        }
    }
    return true;
}

// ---- groups of up to 8 members: the 8 extrapolation columns run side by side -------------
// Lane = 8 k + a: column k (n_k = 2(k+1) midpoint sub-steps) of member a.  Members of one
// column exchange positions by shuffles within their 8 lanes; the tableau is built across
// columns by shuffles from the column below.  The accepted column is the first whose error
// estimate meets the tolerance, so the result equals the sequential scheme's.
constexpr int CP_MEM = 8;
static_assert(CP_MEM * BS_KMAX == BS_LANES, "one lane per (column, member)");

struct ColGroup {
    int k, a, base, nb;
    bool act;
    double mstar;
    // per partner b (constant over the step): r_crit,ab^2, 0.1 r_crit,ab, 1/(0.9 r_crit,ab), m_b
    double rc2[CP_MEM], r01[CP_MEM], inv09[CP_MEM], mb[CP_MEM];
    bool skip[CP_MEM]; // both this member and partner b are test bodies (TP2)
};

// 1/sqrt(q) in FP64: v_rsq_f64 (about 2^-24) and one third-order correction
__device__ __forceinline__ double inv_sqrt64(double q)
{
    const double y0 = __builtin_amdgcn_rsq(q);
    const double t = q * y0;
    const double e = fma(-t, y0, 1.0);
    const double p = fma(0.375, e, 0.5);
    return fma(y0 * e, p, y0);
}

__device__ void col_deriv(const ColGroup &g, const double y[6], double d[6])
{
    const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    const double ri = inv_sqrt64(r2);
    const double s = -g.mstar * (ri * ri) * ri;
    double ax = s * y[0], ay = s * y[1], az = s * y[2];
#pragma unroll
    for (int b = 0; b < CP_MEM; ++b) {
        if (b >= g.nb) break;
        const double xb = __shfl(y[0], g.base + b, 64);
        const double yb = __shfl(y[1], g.base + b, 64);
        const double zb = __shfl(y[2], g.base + b, 64);
        if (b == g.a || g.skip[b]) continue;
        const double dx = xb - y[0], dy = yb - y[1], dz = zb - y[2];
        const double q = sep2_rn(dx, dy, dz);
        if (!(q < g.rc2[b])) continue;
        const double rq = inv_sqrt64(q);
        const double w = 1.0 - changeover_k((q * rq - g.r01[b]) * g.inv09[b]);
        if (w == 0.0) continue;
        const double t = g.mb[b] * w * (rq * rq) * rq;
        ax += t * dx;
        ay += t * dy;
        az += t * dz;
    }
    if (g.act) {
        d[0] = y[3];
        d[1] = y[4];
        d[2] = y[5];
        d[3] = ax;
        d[4] = ay;
        d[5] = az;
    } else {
        for (int q = 0; q < 6; ++q) d[q] = 0.0;
    }
}

__device__ bool col_bs(const ColGroup &g, double Y[6], double dt, double tol)
{
    const int lane = g.base + g.a;
    const int nsub = 2 * (g.k + 1);
    double t = 0.0, H = dt;
    int attempts = 0;
    while (t < dt) {
        const bool last = H >= (dt - t) * (1.0 - 0x1p-30);
        if (last) H = dt - t;
        if (H < dt * 0x1p-40 || ++attempts > 20000) return false;
        const double sr = wave_max(g.act ? sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]) : 0.0);
        const double sv = wave_max(g.act ? sqrt(Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]) : 0.0);
        // this lane's column: modified midpoint with nsub sub-steps
        const double h = H / nsub;
        double zm[6], zc[6], dd[6], cur[6], sub[6];
        col_deriv(g, Y, dd);
        for (int q = 0; q < 6; ++q) {
            zm[q] = Y[q];
            zc[q] = Y[q] + h * dd[q];
        }
        for (int i = 1; i < nsub; ++i) {
            col_deriv(g, zc, dd);
            for (int q = 0; q < 6; ++q) {
                const double tq = zm[q] + 2.0 * h * dd[q];
                zm[q] = zc[q];
                zc[q] = tq;
            }
        }
        col_deriv(g, zc, dd);
        for (int q = 0; q < 6; ++q) {
            cur[q] = 0.5 * (zm[q] + zc[q] + h * dd[q]); // T(k, 0)
            sub[q] = cur[q];
        }
        // Neville across columns: round l turns T(k, l-1) into T(k, l) for k >= l
        const int below = g.k > 0 ? lane - CP_MEM : lane;
#pragma unroll
        for (int l = 1; l < BS_KMAX; ++l) {
            const double ratio = (double)(g.k + 1) / (double)(g.k + 1 - l);
            const double rden = 1.0 / (ratio * ratio - 1.0);
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const double tb = __shfl(cur[q], below, 64); // T(k-1, l-1)
                if (g.k >= l) {
                    const double nxt = cur[q] + (cur[q] - tb) * rden;
                    sub[q] = cur[q];
                    cur[q] = nxt;
                }
            }
        }
        // error of every column (over its members), then the first column that converged
        double err = 0.0;
        if (g.act && g.k > 0)
            for (int q = 0; q < 6; ++q) err = fmax(err, fabs(cur[q] - sub[q]) / (q < 3 ? sr : sv));
        for (int o = 1; o < CP_MEM; o <<= 1) err = fmax(err, __shfl_xor(err, o, 64));
        const bool conv = g.k > 0 && err <= tol && g.a == 0;
        const unsigned long long mask = __ballot(conv);
        if (mask) {
            const int kstar = (__ffsll((long long)mask) - 1) / CP_MEM;
            for (int q = 0; q < 6; ++q) Y[q] = __shfl(cur[q], kstar * CP_MEM + g.a, 64);
            t = last ? dt : t + H;
            if (kstar <= 4) H = 2.0 * H;
            else if (kstar == BS_KMAX - 1) H = 0.5 * H;
        } else {
            const double err_last = __shfl(err, (BS_KMAX - 1) * CP_MEM, 64);
            H = H * shrink_factor(err_last, tol);
        }
    }
    return true;
}

__global__ __launch_bounds__(BS_LANES) void ce_bs_kernel(const int32_t *sys_of, const int32_t *sys_off,
                                                         const int32_t *n_massive, const double *mstar,
                                                         const double *x, const double *y,
                                                         const double *z, const double *vx,
                                                         const double *vy, const double *vz,
                                                         const double *m, const double *rc, double dt,
                                                         const int32_t *members,
                                                         const int32_t *group_start,
                                                         const int32_t *n_groups, double *bs_out,
                                                         int32_t *flags)
{
    __shared__ double sp[3][BS_LANES];
    __shared__ double sm[BS_LANES], src[BS_LANES];
    __shared__ int32_t stest[BS_LANES];
    const int g = blockIdx.x;
    if (g >= *n_groups) return;
    const int k0 = group_start[g], nb = group_start[g + 1] - k0;
    const int a = threadIdx.x;
    const double ms = mstar[sys_of[members[k0]]];
    if (nb > BS_LANES) {
        // larger than one wave: Kepler-drift the members instead and flag it
        if (a == 0) atomicOr(flags, FLAG_CAPACITY);
        for (int k = a; k < nb; k += BS_LANES) {
            const int b = members[k0 + k];
            double px = x[b], py = y[b], pz = z[b], ux = vx[b], uy = vy[b], uz = vz[b];
            if (!kepler_universal(px, py, pz, ux, uy, uz, ms, dt)) atomicOr(flags, FLAG_KEPLER);
            double *o = bs_out + 6 * (size_t)(k0 + k);
            o[0] = px;
            o[1] = py;
            o[2] = pz;
            o[3] = ux;
            o[4] = uy;
            o[5] = uz;
        }
        return;
    }
    if (nb <= CP_MEM) {
        // column-parallel path
        const int k = a / CP_MEM, am = a % CP_MEM;
        const bool act = am < nb;
        const int b = members[k0 + (act ? am : 0)];
        const int sb = sys_of[b];
        const bool is_test = b - sys_off[sb] >= n_massive[sb];
        if (k == 0) {
            sm[am] = act ? m[b] : 0.0;
            src[am] = act ? rc[b] : 0.0;
            stest[am] = act && is_test;
        }
        __syncthreads();
        ColGroup cg;
        cg.k = k;
        cg.a = am;
        cg.base = k * CP_MEM;
        cg.nb = nb;
        cg.act = act;
        cg.mstar = ms;
        const double rca = rc[b];
#pragma unroll
        for (int p = 0; p < CP_MEM; ++p) {
            const double rcij = fmax(rca, src[p]);
            cg.rc2[p] = sq_rn(rcij);
            cg.r01[p] = 0.1 * rcij;
            cg.inv09[p] = 1.0 / (0.9 * rcij);
            cg.mb[p] = sm[p];
            cg.skip[p] = is_test && stest[p];
        }
        double Y[6] = {x[b], y[b], z[b], vx[b], vy[b], vz[b]};
        const bool ok = col_bs(cg, Y, dt, 1e-12);
        if (act && k == 0) {
            double *o = bs_out + 6 * (size_t)(k0 + am);
            for (int q = 0; q < 6; ++q) o[q] = Y[q];
        }
        if (!ok && a == 0) atomicOr(flags, FLAG_NOCONVERGE);
        return;
    }
    const bool act = a < nb;
    const int b = members[k0 + (act ? a : 0)];
    const int sb = sys_of[b];
    const bool is_test = b - sys_off[sb] >= n_massive[sb];
    sm[a] = act ? m[b] : 0.0;
    src[a] = act ? rc[b] : 0.0;
    stest[a] = act && is_test;
    __syncthreads();
    LaneGroup lg{a, nb, act, m[b], rc[b], ms, sp, sm, src, is_test, stest};
    double Y[6] = {x[b], y[b], z[b], vx[b], vy[b], vz[b]};
    const bool ok = lane_bs(lg, Y, dt, 1e-12);
    if (act) {
        double *o = bs_out + 6 * (size_t)(k0 + a);
        for (int q = 0; q < 6; ++q) o[q] = Y[q];
        if (!ok && a == 0) atomicOr(flags, FLAG_NOCONVERGE);
    }
}

} // namespace

hipError_t launch_sun_drift(const Layout &L, double *x, double *y, double *z, const double *vx,
                            const double *vy, const double *vz, const double *m, double tau,
                            double *mom_part, hipStream_t stream)
{
    if (L.n_chunks == 0) return hipSuccess;
    momentum_kernel<<<L.n_chunks, SUN_THREADS, 0, stream>>>(L.chunks, m, vx, vy, vz, mom_part);
    sun_shift_kernel<<<L.n_chunks, SUN_THREADS, 0, stream>>>(L.chunks, L.chunk_first, L.mstar, mom_part,
                                                             tau, x, y, z);
    return hipGetLastError();
}

hipError_t launch_ce_groups(const Layout &L, const int32_t *pairs, const int32_t *pair_count,
                            int32_t pair_cap, int32_t *lab, int32_t *mark, int32_t *members,
                            int32_t *group_start, int32_t *n_groups, int32_t *member_slot,
                            int32_t *flags, hipStream_t stream)
{
    (void)L;
    ce_groups_kernel<<<1, CE_THREADS, 0, stream>>>(pairs, pair_count, pair_cap, lab, mark, members,
                                                   group_start, n_groups, member_slot, flags);
    return hipGetLastError();
}

hipError_t launch_ce_bs(const Layout &L, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *m,
                        const double *rc, double dt, const int32_t *members,
                        const int32_t *group_start, const int32_t *n_groups, double *bs_out,
                        int32_t *flags, hipStream_t stream)
{
    // one wave per group; at most CE_MAX_MEMBERS / 2 groups (every group has >= 2 members)
    ce_bs_kernel<<<CE_MAX_MEMBERS / 2, BS_LANES, 0, stream>>>(L.sys_of, L.sys_off, L.n_massive, L.mstar,
                                                              x, y, z, vx, vy, vz, m, rc,
                                                              dt, members, group_start, n_groups, bs_out,
                                                              flags);
    return hipGetLastError();
}

hipError_t launch_kepler(const Layout &L, double *x, double *y, double *z, double *vx, double *vy,
                         double *vz, double dt, int32_t *member_slot, const double *bs_out,
                         int32_t *flags, hipStream_t stream)
{
    if (L.n_total == 0) return hipSuccess;
    // one wave per workgroup spreads the latency-bound solves over all CUs
    kepler_kernel<<<(L.n_total + 63) / 64, 64, 0, stream>>>(L.n_total, L.sys_of, L.mstar, x, y, z,
                                                               vx, vy, vz, dt, member_slot, bs_out,
                                                               flags);
    return hipGetLastError();
}

} // namespace genga
