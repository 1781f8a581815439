// Drift part of the hybrid symplectic step (Brasser et al. 2023, Sect. 1), all FP64:
//  * Sun drift: r_i += tau * (sum_j m_j v_j) / Mstar (democratic heliocentric split);
//  * Kepler drift of every body not in a close encounter, by universal variables
//    (Stumpff functions, safeguarded Newton on the universal Kepler equation);
//  * close-encounter step: the encounter pairs are joined into groups (connected components,
//    one workgroup, union-find in global memory, members sorted in LDS), and each group is
//    integrated over dt by Gragg-Bulirsch-Stoer under the Sun's force plus the (1 - K) share
//    of the members' mutual forces; the Kepler kernel then writes the group results back.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

// ------------------------------------------------------------------------------------------
// Sun drift in two launches over chunks of one system: partial momenta per chunk (fixed-order
// block reduction), then every chunk adds its system's partials in chunk order and shifts
// its positions.  Deterministic.
// ------------------------------------------------------------------------------------------
constexpr int SUN_THREADS = SYS_P_THREADS;

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
    __shared__ double red[3][SYS_P_THREADS / 64];
    const Chunk c = chunks[blockIdx.x];
    double P[3];
    system_momentum(chunk_first, mom_part, c.sys, red, P);
    const double f = tau / mstar[c.sys];
    const double sx = f * P[0], sy = f * P[1], sz = f * P[2];
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

__device__ __forceinline__ void store_state(double *x, double *y, double *z, double *vx, double *vy,
                                            double *vz, int b, const double *Y)
{
    x[b] = Y[0];
    y[b] = Y[1];
    z[b] = Y[2];
    vx[b] = Y[3];
    vy[b] = Y[4];
    vz[b] = Y[5];
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

// Root of a with path halving: every visited node is pointed at its grandparent.  Labels only
// ever move to a smaller index of the same tree (hooks link a root under a smaller root), so
// a halving step that races with a hook or another halving still leaves a valid ancestor.
__device__ __forceinline__ int find_root_halving(int32_t *lab, int a)
{
    int p = lab_load(lab, a);
    while (p != a) {
        const int gp = lab_load(lab, p);
        if (gp != p) __hip_atomic_store(&lab[a], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a = gp;
        p = lab_load(lab, a);
    }
    return a;
}

// Grid-wide union-find over the encounter pairs, for the large-group mode, where the host
// reads the labels back: every body of a pair becomes its own root, rounds of hooking (the
// larger root under the smaller) run until a round changes nothing, then every member's label
// is compressed to its root.  Non-members keep lab = -1.
__global__ __launch_bounds__(256) void uf_init_kernel(const int32_t *pairs, const int32_t *pair_count,
                                                      int32_t pair_cap, int32_t *lab)
{
    const int np = min(*pair_count, pair_cap);
    for (int p = blockIdx.x * 256 + threadIdx.x; p < np; p += gridDim.x * 256) {
        const int a = pairs[2 * p], b = pairs[2 * p + 1];
        __hip_atomic_store(&lab[a], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&lab[b], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(256) void uf_hook_kernel(const int32_t *pairs, const int32_t *pair_count,
                                                      int32_t pair_cap, int32_t *lab, int32_t *changed,
                                                      const int32_t *run_if)
{
    if (run_if && *run_if == 0) return;
    const int np = min(*pair_count, pair_cap);
    int ch = 0;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < np; p += gridDim.x * 256) {
        const int a = find_root_halving(lab, pairs[2 * p]);
        const int b = find_root_halving(lab, pairs[2 * p + 1]);
        if (a != b) {
            // a hook that would change nothing skips the atomic: pairs of two large trees
            // all hook the same root, and the atomics would queue on that one address
            const int lo = min(a, b), hi = max(a, b);
            if (lab_load(lab, hi) > lo) atomicMin(&lab[hi], lo);
            ch = 1;
        }
    }
    if (__ballot(ch) && (threadIdx.x & 63) == 0) atomicOr(changed, 1);
}

__global__ __launch_bounds__(256) void uf_compress_kernel(int n_total, int32_t *lab, const int32_t *run_if)
{
    if (run_if && *run_if == 0) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_total || lab_load(lab, i) < 0) return;
    __hip_atomic_store(&lab[i], find_root(lab, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// members[k] -> member_slot, and lab back to -1 (clean for the next step)
__global__ __launch_bounds__(256) void uf_slots_kernel(const int32_t *members, const int32_t *n_members,
                                                       int32_t *member_slot, int32_t *lab)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= *n_members) return;
    const int b = members[k];
    member_slot[b] = k;
    lab[b] = -1;
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
                if (lab_load(lab, hi) > lo) atomicMin(&lab[hi], lo);
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
// Bulirsch-Stoer over dt for the close-encounter groups (FP64): one wavefront per group.
// Same method as the oracle: modified midpoint with n_k = 2(k+1) sub-steps (k = 0..7),
// polynomial extrapolation in h^2 by Neville's scheme, and the step accepted at the first
// column k >= 1 whose last two entries agree to tol on the group's position and velocity
// scales.  After a step accepted at column k the next one is doubled (k <= 4), kept
// (k = 5, 6) or halved (k = 7); a rejected step shrinks by shrink_factor.  Step decisions use
// wave-wide values, so control flow stays uniform.
//
// Everything per lane lives in registers except what other lanes read: the positions
// published for the pair forces and the tableau rows, both in LDS.  Force evaluations are
// plain loops over the members, so the code stays small and nothing spills.
// ------------------------------------------------------------------------------------------
constexpr int BS_LANES = 64;
constexpr int CP_MEM = 8; // largest group whose extrapolation columns run side by side
static_assert(CP_MEM * BS_KMAX == BS_LANES, "one lane per (column, member)");

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Neville factor 1 / ((n_k / n_(k-l))^2 - 1) for n_k = 2(k+1), written as p^2 / (q^2 - p^2)
// with q = k + 1, p = k + 1 - l: exact small integers and one rounding.
__device__ __forceinline__ double neville_c(int k, int l)
{
    const double q = (double)(k + 1), p = (double)(k + 1 - l);
    return (p * p) / (q * q - p * p);
}

// Members' data shared by the lanes of the group's wave.
struct BsShared {
    double pos[BS_LANES][4];                   // positions published for the pair forces
    double m[BS_LANES];                        // member masses
    double rc[BS_LANES], r01[BS_LANES], i09[BS_LANES]; // r_crit, 0.1 r_crit, 1 / (0.9 r_crit)
    double rcl[LEVELS_MAX - 1][BS_LANES];      // hierarchical levels 1..nlev-1: r_crit of each
    int32_t test[BS_LANES];                    // member is a test body (TP2)
    int32_t nlev;                              // symplectic levels (1: the plain step)
};

// This lane's member: its constants and which lanes hold its partners' positions.
struct BsMember {
    int a, nb, base; // member index, group size, lane of member 0 in pos[]
    bool act, test;
    double mstar, rc, r01, i09;
};

// With LV (hierarchical levels), the pair weight (1 - K) of level 0 times prod over levels
// 1..nlev-1 of (1 - K_k) with the pair's level-k radius; the pair counts while closer than the
// deepest level's radius (the radii do not grow with the level).  The factor of the deeper
// levels, or 0 beyond the deepest radius; ra / rb give member a's / b's level radii.
template <bool LV>
__device__ __forceinline__ double deeper_levels(double r, double q, int nlev, const double *ra, const double *rb,
                                                int stride)
{
    if constexpr (!LV) return 1.0;
    double w = 1.0;
    for (int k = 1; k < nlev; ++k) {
        const double rck = fmax(ra[(k - 1) * stride], rb[(k - 1) * stride]);
        if (!(q < sq_rn(rck))) return 0.0;
        w *= 1.0 - changeover_k((r - 0.1 * rck) / (0.9 * rck));
    }
    return w;
}

// dY/dt: Kepler term about the Sun plus the (1 - K) share of the Newtonian forces from the
// other members (K of Chambers 1999 over [0.1, 1] r_crit,ab; two test bodies do not
// interact).  Every lane of the wave calls it.
template <bool LV>
__device__ void bs_forces(const BsMember &me, BsShared &S, int slot, const double z[6], double d[6])
{
    S.pos[slot][0] = z[0];
    S.pos[slot][1] = z[1];
    S.pos[slot][2] = z[2];
    __syncthreads();
    const double ri = inv_sqrt64(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    const double s = -me.mstar * (ri * ri) * ri;
    double ax = s * z[0], ay = s * z[1], az = s * z[2];
#pragma unroll 1
    for (int b = 0; b < me.nb; ++b) {
        if (b == me.a || (me.test && S.test[b])) continue;
        const double dx = S.pos[me.base + b][0] - z[0];
        const double dy = S.pos[me.base + b][1] - z[1];
        const double dz = S.pos[me.base + b][2] - z[2];
        const double q = sep2_rn(dx, dy, dz);
        // r_crit,ab = max(r_crit,a, r_crit,b), with that member's derived constants
        const bool own = me.rc >= S.rc[b];
        const double rcab = own ? me.rc : S.rc[b];
        if (!(q < sq_rn(rcab))) continue;
        const double rq = inv_sqrt64(q);
        double w = 1.0 - changeover_k((q * rq - (own ? me.r01 : S.r01[b])) * (own ? me.i09 : S.i09[b]));
        if constexpr (LV) w *= deeper_levels<LV>(q * rq, q, S.nlev, &S.rcl[0][me.a], &S.rcl[0][b], BS_LANES);
        const double t = S.m[b] * w * (rq * rq) * rq;
        ax = fma(t, dx, ax);
        ay = fma(t, dy, ay);
        az = fma(t, dz, az);
    }
    __syncthreads(); // the next call overwrites pos
    d[0] = me.act ? z[3] : 0.0;
    d[1] = me.act ? z[4] : 0.0;
    d[2] = me.act ? z[5] : 0.0;
    d[3] = me.act ? ax : 0.0;
    d[4] = me.act ? ay : 0.0;
    d[5] = me.act ? az : 0.0;
}

// Groups of up to CP_MEM members.  Lane 8k + a runs extrapolation column k for member a, so
// the columns advance side by side, one force evaluation per pass.  Column k's sub-steps end
// after n_k + 1 passes; its lanes then extend the tableau by row k (reading row k-1 from LDS)
// and the wave ends the attempt as soon as a column has converged.  The accepted column is
// the first converged one, as in the sequential scheme.
template <bool LV>
__device__ bool bs_columns(const BsMember &me, int k, BsShared &S, double (*row)[BS_KMAX][CP_MEM][6],
                           double Y[6], double dt, double tol)
{
    const int slot = me.base + me.a;
    const int nsub = 2 * (k + 1);
    double t = 0.0, H = dt;
    int attempts = 0;
    while (t < dt) {
        const bool last = H >= (dt - t) * (1.0 - 0x1p-30); // ends the interval (exactly)
        if (last) H = dt - t;
        if (H < dt * 0x1p-40 || ++attempts > 20000) return false;
        const double sr = wave_max(me.act ? sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]) : 0.0);
        const double sv = wave_max(me.act ? sqrt(Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]) : 0.0);
        const double h = H / nsub;
        double zm[6], zc[6], T[6];
        for (int q = 0; q < 6; ++q) zc[q] = zm[q] = T[q] = Y[q];
        int kstar = -1;
        double err_last = 0.0;
#pragma unroll 1
        for (int i = 0; i <= 2 * BS_KMAX; ++i) {
            double dd[6];
            bs_forces<LV>(me, S, slot, zc, dd);
            if (i == 0) {
                for (int q = 0; q < 6; ++q) zc[q] = zm[q] + h * dd[q];
            } else if (i < nsub) {
                for (int q = 0; q < 6; ++q) {
                    const double tq = zm[q] + 2.0 * h * dd[q];
                    zm[q] = zc[q];
                    zc[q] = tq;
                }
            } else if (i == nsub) {
                for (int q = 0; q < 6; ++q) T[q] = 0.5 * (zm[q] + zc[q] + h * dd[q]); // T(k, 0)
            }
            if (i < 2 || (i & 1)) continue;
            const int kk = i / 2 - 1; // the column whose sub-steps have just ended
            double err = 0.0;
            if (k == kk) {
                double(*mine)[CP_MEM][6] = row[kk & 1];
                const double(*below)[CP_MEM][6] = row[(kk + 1) & 1]; // row kk - 1
                for (int q = 0; q < 6; ++q) mine[0][me.a][q] = T[q];
                double dp = 0.0, dv = 0.0; // |T(kk, l) - T(kk, l-1)| of the last pass, l = kk
#pragma unroll 1
                for (int l = 1; l <= kk; ++l) {
                    const double c = neville_c(kk, l);
                    dp = dv = 0.0;
                    double bl[6];
                    for (int q = 0; q < 6; ++q) bl[q] = below[l - 1][me.a][q];
                    for (int q = 0; q < 6; ++q) {
                        const double nx = T[q] + (T[q] - bl[q]) * c;
                        if (q < 3) dp = fmax(dp, fabs(nx - T[q]));
                        else dv = fmax(dv, fabs(nx - T[q]));
                        T[q] = nx;
                    }
                    for (int q = 0; q < 6; ++q) mine[l][me.a][q] = T[q];
                }
                // max over elements of |diff| / scale (the scale is common, so divide once)
                err = me.act ? fmax(dp / sr, dv / sv) : 0.0;
            }
            if (kk == 0) continue;
            for (int o = 1; o < CP_MEM; o <<= 1) err = fmax(err, __shfl_xor(err, o, 64));
            if (__ballot(k == kk && me.a == 0 && err <= tol)) {
                kstar = kk;
                break;
            }
            if (kk == BS_KMAX - 1) err_last = __shfl(err, kk * CP_MEM, 64);
        }
        if (kstar >= 0) {
            __syncthreads(); // row kstar, written by its column's lanes, is read by all
            for (int q = 0; q < 6; ++q) Y[q] = row[kstar & 1][kstar][me.a][q];
            __syncthreads();
            t = last ? dt : t + H;
            if (kstar <= 4) H = 2.0 * H;
            else if (kstar == BS_KMAX - 1) H = 0.5 * H;
        } else {
            H = H * shrink_factor(err_last, tol);
        }
    }
    return true;
}

// Groups of CP_MEM + 1 .. BS_LANES members: one workgroup of BS_KMAX waves, wave k running
// extrapolation column k for every member, so the columns advance side by side, one force
// evaluation per pass, and an attempt takes at most 2 BS_KMAX + 1 passes.  A member has P
// lanes (4 for groups of up to 16, 2 up to 32, else 1) that share its sources, sum every
// P-th one and add the parts in a fixed tree.  Column k completes at pass 2(k + 1) and
// extends each member's Neville row in place in LDS: it reads row k - 1, which column k - 1
// wrote two passes before, and replaces it by row k, which column k + 1 reads two passes
// later.  The tableau arithmetic and the accepted column (the first converged one) are those
// of the sequential scheme.
constexpr int WG_THREADS = BS_KMAX * BS_LANES;

struct BsWgShared {
    double pos[BS_KMAX][BS_LANES][3];          // each column's positions, for its pair forces
    double m[BS_LANES], rc[BS_LANES], r01[BS_LANES], i09[BS_LANES];
    double rcl[LEVELS_MAX - 1][BS_LANES];      // hierarchical levels 1..nlev-1
    double tab[BS_KMAX][6][BS_LANES];          // Neville rows, extended in place
    double err_last;                           // column BS_KMAX - 1's estimate
    int32_t test[BS_LANES];
    int32_t nlev;
    int32_t kstar, kstar_att;                  // converged column and the attempt it ended
};

// One pass of column k for part `part` of member a's P lanes: the forces at z (when `on`),
// between two barriers that every thread of the workgroup reaches.
template <bool LV>
__device__ void wg_forces(bool on, int k, int a, int part, int P, int nb, bool act, bool test, double mstar,
                          double rc, double r01, double i09, BsWgShared &S, const double z[6], double d[6])
{
    if (part == 0) {
        S.pos[k][a][0] = z[0];
        S.pos[k][a][1] = z[1];
        S.pos[k][a][2] = z[2];
    }
    __syncthreads();
    if (on) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (part == 0) {
            const double ri = inv_sqrt64(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
            const double s = -mstar * (ri * ri) * ri;
            ax = s * z[0];
            ay = s * z[1];
            az = s * z[2];
        }
#pragma unroll 1
        for (int b = part; b < nb; b += P) {
            if (b == a || (test && S.test[b])) continue;
            const double dx = S.pos[k][b][0] - z[0];
            const double dy = S.pos[k][b][1] - z[1];
            const double dz = S.pos[k][b][2] - z[2];
            const double q = sep2_rn(dx, dy, dz);
            // r_crit,ab = max(r_crit,a, r_crit,b), with that member's derived constants
            const bool own = rc >= S.rc[b];
            const double rcab = own ? rc : S.rc[b];
            if (!(q < sq_rn(rcab))) continue;
            const double rq = inv_sqrt64(q);
            double w = 1.0 - changeover_k((q * rq - (own ? r01 : S.r01[b])) * (own ? i09 : S.i09[b]));
            if constexpr (LV) w *= deeper_levels<LV>(q * rq, q, S.nlev, &S.rcl[0][a], &S.rcl[0][b], BS_LANES);
            const double t = S.m[b] * w * (rq * rq) * rq;
            ax = fma(t, dx, ax);
            ay = fma(t, dy, ay);
            az = fma(t, dz, az);
        }
        for (int o = 1; o < P; o <<= 1) {
            ax += __shfl_xor(ax, o, 64);
            ay += __shfl_xor(ay, o, 64);
            az += __shfl_xor(az, o, 64);
        }
        d[0] = act ? z[3] : 0.0;
        d[1] = act ? z[4] : 0.0;
        d[2] = act ? z[5] : 0.0;
        d[3] = act ? ax : 0.0;
        d[4] = act ? ay : 0.0;
        d[5] = act ? az : 0.0;
    }
    __syncthreads(); // the next pass overwrites pos
}

template <bool LV>
__device__ bool bs_workgroup(int k, int a, int part, int P, int nb, bool act, bool test, double mstar, double rc,
                             double r01, double i09, BsWgShared &S, double Y[6], double dt, double tol)
{
    const int nsub = 2 * (k + 1);
    const int lane = threadIdx.x & (BS_LANES - 1);
    double t = 0.0, H = dt;
    int attempts = 0;
    while (t < dt) {
        const bool last = H >= (dt - t) * (1.0 - 0x1p-30); // ends the interval (exactly)
        if (last) H = dt - t;
        if (H < dt * 0x1p-40 || ++attempts > 20000) return false;
        const double sr = wave_max(act ? sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]) : 0.0);
        const double sv = wave_max(act ? sqrt(Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5]) : 0.0);
        const double h = H / nsub;
        double zm[6], zc[6], T[6];
        for (int q = 0; q < 6; ++q) zc[q] = zm[q] = T[q] = Y[q];
        int kstar = -1;
#pragma unroll 1
        for (int i = 0; i <= 2 * BS_KMAX; ++i) {
            double dd[6];
            wg_forces<LV>(i <= nsub, k, a, part, P, nb, act, test, mstar, rc, r01, i09, S, zc, dd);
            if (i == 0) {
                for (int q = 0; q < 6; ++q) zc[q] = zm[q] + h * dd[q];
            } else if (i < nsub) {
                for (int q = 0; q < 6; ++q) {
                    const double tq = zm[q] + 2.0 * h * dd[q];
                    zm[q] = zc[q];
                    zc[q] = tq;
                }
            } else if (i == nsub) {
                for (int q = 0; q < 6; ++q) T[q] = 0.5 * (zm[q] + zc[q] + h * dd[q]); // T(k, 0)
                // Neville: row k - 1 is replaced by row k in place (T(k, l-1) goes into slot
                // l-1 once T(k-1, l-1) has been read from it)
                double dp = 0.0, dv = 0.0;
#pragma unroll 1
                for (int l = 1; l <= k; ++l) {
                    const double c = neville_c(k, l);
                    double old[6];
                    for (int q = 0; q < 6; ++q) old[q] = S.tab[l - 1][q][a];
                    if (part == 0)
                        for (int q = 0; q < 6; ++q) S.tab[l - 1][q][a] = T[q];
                    for (int q = 0; q < 6; ++q) {
                        const double nx = T[q] + (T[q] - old[q]) * c;
                        if (l == k) {
                            if (q < 3) dp = fmax(dp, fabs(nx - T[q]));
                            else dv = fmax(dv, fabs(nx - T[q]));
                        }
                        T[q] = nx;
                    }
                }
                if (part == 0)
                    for (int q = 0; q < 6; ++q) S.tab[k][q][a] = T[q];
                if (k > 0) {
                    const double err = wave_max(act ? fmax(dp / sr, dv / sv) : 0.0);
                    if (lane == 0) {
                        if (err <= tol) {
                            S.kstar = k;
                            S.kstar_att = attempts;
                        }
                        if (k == BS_KMAX - 1) S.err_last = err;
                    }
                }
            }
            if (i < 2 || (i & 1)) continue; // columns complete at even passes
            __syncthreads();                // the completed column's verdict
            if (S.kstar_att == attempts) {
                kstar = S.kstar;
                break;
            }
        }
        if (kstar >= 0) {
            for (int q = 0; q < 6; ++q) Y[q] = S.tab[kstar][q][a];
            t = last ? dt : t + H;
            if (kstar <= 4) H = 2.0 * H;
            else if (kstar == BS_KMAX - 1) H = 0.5 * H;
        } else {
            H = H * shrink_factor(S.err_last, tol);
        }
        __syncthreads(); // tab[kstar] and err_last are read before the next attempt writes them
    }
    return true;
}

// Groups of 2 or 3 members (almost all groups when r_crit is a few Hill radii): lane k runs
// extrapolation column k for the whole group, so a force evaluation is lane-local (the pair
// force is formed once and applied to both members) and needs no exchange between lanes.
// When column k completes, T(k, 0) goes to LDS and the wave forms T(k, k) - T(k, k-1) with
// one lane per state element, from the Lagrange form of the extrapolation (LAGRANGE).
template <int NB>
struct SmallGroup {
    double mstar;
    double m[NB];
    double rc2[NB][NB], r01[NB][NB], i09[NB][NB]; // per pair a < b, from r_crit,ab
    bool skip[NB][NB];                            // both are test bodies (TP2)
    int nlev;                                     // hierarchical levels
    double rcl[LEVELS_MAX - 1][NB];               // levels 1..nlev-1: r_crit of each member
};

template <int NB, bool LV>
__device__ __forceinline__ void small_forces(const SmallGroup<NB> &g, const double (&z)[NB][6],
                                             double (&d)[NB][6])
{
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const double ri = inv_sqrt64(z[a][0] * z[a][0] + z[a][1] * z[a][1] + z[a][2] * z[a][2]);
        const double s = -g.mstar * (ri * ri) * ri;
        d[a][0] = z[a][3];
        d[a][1] = z[a][4];
        d[a][2] = z[a][5];
        d[a][3] = s * z[a][0];
        d[a][4] = s * z[a][1];
        d[a][5] = s * z[a][2];
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = a + 1; b < NB; ++b) {
            if (g.skip[a][b]) continue;
            const double dx = z[b][0] - z[a][0], dy = z[b][1] - z[a][1], dz = z[b][2] - z[a][2];
            const double q = sep2_rn(dx, dy, dz);
            if (!(q < g.rc2[a][b])) continue;
            const double rq = inv_sqrt64(q);
            double w = 1.0 - changeover_k((q * rq - g.r01[a][b]) * g.i09[a][b]);
            if constexpr (LV) w *= deeper_levels<LV>(q * rq, q, g.nlev, &g.rcl[0][a], &g.rcl[0][b], NB);
            const double u = w * (rq * rq) * rq;
            const double ua = g.m[b] * u, ub = g.m[a] * u;
            d[a][3] = fma(ua, dx, d[a][3]);
            d[a][4] = fma(ua, dy, d[a][4]);
            d[a][5] = fma(ua, dz, d[a][5]);
            d[b][3] = fma(-ub, dx, d[b][3]);
            d[b][4] = fma(-ub, dy, d[b][4]);
            d[b][5] = fma(-ub, dz, d[b][5]);
        }
}

// Sum over the completed columns 1..k of c[j] (T(j, 0) - T(0, 0)) for this lane's element,
// tcol[j * E + e] holding T(j, 0); every load is issued before the first use.
template <int E>
__device__ __forceinline__ double lagrange_sum(const double *tcol, const double *c, int k, int e)
{
    const double t0 = tcol[e];
    double v[BS_KMAX], cj[BS_KMAX];
#pragma unroll
    for (int j = 1; j < BS_KMAX; ++j) {
        v[j] = tcol[j * E + e];
        cj[j] = c[j];
    }
    double s = 0.0;
#pragma unroll
    for (int j = 1; j < BS_KMAX; ++j) {
        const double f = fma(cj[j], v[j] - t0, s);
        s = j <= k ? f : s; // rows above k are stale
    }
    return s;
}

// ybuf: the group state [NB][6] in LDS (read at entry, holds the result on return);
// tcol: LDS [BS_KMAX][NB * 6] for T(k, 0); lag: LAGRANGE copied to LDS (w, then d).
template <int NB, bool LV>
__device__ bool bs_small(const SmallGroup<NB> &g, int lane, double *ybuf, double *tcol, const double *lag,
                         double dt, double tol)
{
    constexpr int E = NB * 6;
    const double *lw = lag, *ld = lag + BS_KMAX * BS_KMAX;
    const int k = lane & (BS_KMAX - 1);
    const bool writer = lane < BS_KMAX;
    const int nsub = 2 * (k + 1);
    const int e = lane < E ? lane : 0; // state element of this lane in the extrapolation
    double t = 0.0, H = dt;
    int attempts = 0;
    while (t < dt) {
        const bool last = H >= (dt - t) * (1.0 - 0x1p-30); // ends the interval (exactly)
        if (last) H = dt - t;
        if (H < dt * 0x1p-40 || ++attempts > 20000) return false;
        const double h = H / nsub;
        double zm[NB][6], zc[NB][6];
        double sr = 0.0, sv = 0.0;
#pragma unroll
        for (int a = 0; a < NB; ++a) {
#pragma unroll
            for (int q = 0; q < 6; ++q) zc[a][q] = zm[a][q] = ybuf[6 * a + q];
            sr = fmax(sr, sqrt(zm[a][0] * zm[a][0] + zm[a][1] * zm[a][1] + zm[a][2] * zm[a][2]));
            sv = fmax(sv, sqrt(zm[a][3] * zm[a][3] + zm[a][4] * zm[a][4] + zm[a][5] * zm[a][5]));
        }
        const double scale = e % 6 < 3 ? sr : sv;
        int kstar = -1;
        double err_last = 0.0;
#pragma unroll 1
        for (int i = 0; i <= 2 * BS_KMAX; ++i) {
            double dd[NB][6];
            small_forces<NB, LV>(g, zc, dd);
            if (i == 0) {
#pragma unroll
                for (int a = 0; a < NB; ++a)
#pragma unroll
                    for (int q = 0; q < 6; ++q) zc[a][q] = zm[a][q] + h * dd[a][q];
            } else if (i < nsub) {
#pragma unroll
                for (int a = 0; a < NB; ++a)
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        const double tq = zm[a][q] + 2.0 * h * dd[a][q];
                        zm[a][q] = zc[a][q];
                        zc[a][q] = tq;
                    }
            } else if (i == nsub && writer) {
#pragma unroll
                for (int a = 0; a < NB; ++a)
#pragma unroll
                    for (int q = 0; q < 6; ++q) tcol[k * E + 6 * a + q] = 0.5 * (zm[a][q] + zc[a][q] + h * dd[a][q]);
            }
            if (i < 2 || (i & 1)) continue;
            const int kk = i / 2 - 1; // the column that has just completed
            __syncthreads();          // its T(kk, 0) is read by every lane
            if (kk == 0) continue;
            const double err = fabs(lagrange_sum<E>(tcol, ld + kk * BS_KMAX, kk, e)) / scale;
            if (!__ballot(lane < E && !(err <= tol))) {
                kstar = kk;
                break;
            }
            if (kk == BS_KMAX - 1) err_last = wave_max(lane < E ? err : 0.0);
        }
        if (kstar >= 0) {
            const double y = tcol[e] + lagrange_sum<E>(tcol, lw + kstar * BS_KMAX, kstar, e);
            __syncthreads(); // every lane has read ybuf and tcol
            if (lane < E) ybuf[e] = y;
            __syncthreads();
            t = last ? dt : t + H;
            if (kstar <= 4) H = 2.0 * H;
            else if (kstar == BS_KMAX - 1) H = 0.5 * H;
        } else {
            H = H * shrink_factor(err_last, tol);
        }
    }
    return true;
}

template <int NB, bool LV>
__device__ bool run_small(const BsShared &S, int lane, double ms, double *x, double *y, double *z,
                          double *vx, double *vy, double *vz, const int32_t *mem, double *ybuf,
                          double *tcol, double *lag, double dt)
{
    SmallGroup<NB> g;
    g.mstar = ms;
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        g.m[a] = S.m[a];
#pragma unroll
        for (int b = a + 1; b < NB; ++b) {
            const bool own = S.rc[a] >= S.rc[b];
            const double rcab = own ? S.rc[a] : S.rc[b];
            g.rc2[a][b] = sq_rn(rcab);
            g.r01[a][b] = own ? S.r01[a] : S.r01[b];
            g.i09[a][b] = own ? S.i09[a] : S.i09[b];
            g.skip[a][b] = S.test[a] && S.test[b];
        }
    }
    g.nlev = S.nlev;
    if constexpr (LV)
        for (int k = 1; k < S.nlev; ++k)
#pragma unroll
            for (int a = 0; a < NB; ++a) g.rcl[k - 1][a] = S.rcl[k - 1][a];
    if (lane < NB) {
        const int b = mem[lane];
        ybuf[6 * lane + 0] = x[b];
        ybuf[6 * lane + 1] = y[b];
        ybuf[6 * lane + 2] = z[b];
        ybuf[6 * lane + 3] = vx[b];
        ybuf[6 * lane + 4] = vy[b];
        ybuf[6 * lane + 5] = vz[b];
    }
    lag[lane] = (&LAGRANGE.w[0][0])[lane];
    lag[BS_LANES + lane] = (&LAGRANGE.d[0][0])[lane];
    __syncthreads();
    const bool ok = bs_small<NB, LV>(g, lane, ybuf, tcol, lag, dt, 1e-12);
    __syncthreads();
    if (lane < NB) store_state(x, y, z, vx, vy, vz, mem[lane], ybuf + 6 * lane);
    return ok;
}

// The drift over dt: blocks [0, bs_blocks) integrate one encounter group each with
// Bulirsch-Stoer, the blocks after them Kepler-drift 64 bodies each and skip the group
// members.  Each body is read and written by one block only.

template <bool LV>
__global__ __launch_bounds__(BS_LANES) void drift_kernel(const int32_t *sys_of, const int32_t *sys_off,
                                                         const int32_t *n_massive, const double *mstar,
                                                         int n_total, double *x, double *y, double *z,
                                                         double *vx, double *vy, double *vz,
                                                         const double *m, const double *rc, double dt,
                                                         const int32_t *members,
                                                         const int32_t *group_start,
                                                         const int32_t *n_groups, int32_t *member_slot,
                                                         int32_t *flags, int big_groups, int bs_blocks,
                                                         const double *rc_lv, int nlev)
{
    // the column path's two Neville rows; the small-group path's T(k, 0) table and Lagrange
    // weights fit in the same space.  The block's LDS sets how many share a CU.
    constexpr int TAB = 2 * BS_KMAX * CP_MEM * 6;
    static_assert(BS_KMAX * 3 * 6 + 2 * BS_LANES <= TAB, "small-group tables fit");
    __shared__ BsShared S;
    __shared__ double tab[TAB];
    const int lane = threadIdx.x;
    if ((int)blockIdx.x >= bs_blocks) {
        const int i = (blockIdx.x - bs_blocks) * BS_LANES + lane;
        if (i >= n_total) return;
        if (member_slot[i] >= 0) {
            member_slot[i] = -1; // integrated by its group's block; leave the slot clear
            return;
        }
        double Y[6] = {x[i], y[i], z[i], vx[i], vy[i], vz[i]};
        if (!kepler_universal(Y[0], Y[1], Y[2], Y[3], Y[4], Y[5], mstar[sys_of[i]], dt)) atomicOr(flags, FLAG_KEPLER);
        store_state(x, y, z, vx, vy, vz, i, Y);
        return;
    }
    const int g = blockIdx.x;
    if (g >= *n_groups) return;
    const int k0 = group_start[g], nb = group_start[g + 1] - k0;
    const double ms = mstar[sys_of[members[k0]]];
    if (nb > BS_LANES) {
        if (big_groups) return; // integrated by the grid-wide path
        // larger than one wave: Kepler-drift the members instead and flag it
        if (lane == 0) atomicOr(flags, FLAG_CAPACITY);
        for (int k = lane; k < nb; k += BS_LANES) {
            const int b = members[k0 + k];
            double Y[6] = {x[b], y[b], z[b], vx[b], vy[b], vz[b]};
            if (!kepler_universal(Y[0], Y[1], Y[2], Y[3], Y[4], Y[5], ms, dt)) atomicOr(flags, FLAG_KEPLER);
            store_state(x, y, z, vx, vy, vz, b, Y);
        }
        return;
    }
    if (lane < nb) {
        const int b = members[k0 + lane];
        const int sb = sys_of[b];
        S.m[lane] = m[b];
        S.rc[lane] = rc[b];
        S.r01[lane] = 0.1 * rc[b];
        S.i09[lane] = 1.0 / (0.9 * rc[b]);
        S.test[lane] = b - sys_off[sb] >= n_massive[sb];
        if constexpr (LV)
            for (int l = 1; l < nlev; ++l) S.rcl[l - 1][lane] = rc_lv[(size_t)(l - 1) * n_total + b];
    }
    if (lane == 0) S.nlev = nlev;
    __syncthreads();
    if (nb <= 3) {
        __shared__ double ybuf[3 * 6];
        double *lag = tab + BS_KMAX * 3 * 6;
        const bool ok = nb == 2 ? run_small<2, LV>(S, lane, ms, x, y, z, vx, vy, vz, members + k0, ybuf, tab, lag, dt)
                                : run_small<3, LV>(S, lane, ms, x, y, z, vx, vy, vz, members + k0, ybuf, tab, lag, dt);
        if (!ok && lane == 0) atomicOr(flags, FLAG_NOCONVERGE);
        return;
    }
    if (nb > CP_MEM) return; // a workgroup of drift_wg_kernel integrates it
    const int k = lane / CP_MEM;
    BsMember me;
    me.a = lane % CP_MEM;
    me.nb = nb;
    me.base = k * CP_MEM;
    me.act = me.a < nb;
    const int ai = me.act ? me.a : 0;
    me.test = S.test[ai] != 0;
    me.mstar = ms;
    me.rc = S.rc[ai];
    me.r01 = S.r01[ai];
    me.i09 = S.i09[ai];
    const int b = members[k0 + ai];
    double Y[6] = {x[b], y[b], z[b], vx[b], vy[b], vz[b]};
    const bool ok = bs_columns<LV>(me, k, S, (double(*)[BS_KMAX][CP_MEM][6])tab, Y, dt, 1e-12);
    // every lane has read its member's state before the first force evaluation's barrier
    if (me.act && k == 0) store_state(x, y, z, vx, vy, vz, b, Y);
    if (!ok && lane == 0) atomicOr(flags, FLAG_NOCONVERGE);
}

// The groups of CP_MEM + 1 .. BS_LANES members in group order, from one workgroup (a ballot
// and a scan per round of 1024 groups): list[0] their number, list[1 + i] the groups.
__global__ __launch_bounds__(1024) void wg_list_kernel(const int32_t *group_start, const int32_t *n_groups,
                                                       int bs_blocks, int32_t *list)
{
    __shared__ int wsum[1024 / 64];
    const int G = min(*n_groups, bs_blocks);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int base = 0;
    for (int c = 0; c < G; c += 1024) {
        const int g = c + (int)threadIdx.x;
        const int nb = g < G ? group_start[g + 1] - group_start[g] : 0;
        const bool med = nb > CP_MEM && nb <= BS_LANES;
        const unsigned long long bal = __ballot(med);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < 1024 / 64; ++w) {
            off += w < wave ? wsum[w] : 0;
            tot += wsum[w];
        }
        if (med) list[1 + base + off + __popcll(bal & ((1ull << lane) - 1))] = g;
        base += tot;
        __syncthreads(); // wsum is rewritten by the next round
    }
    if (threadIdx.x == 0) list[0] = base;
}

// The listed groups of CP_MEM + 1 .. BS_LANES members, one workgroup at a time each
// (bs_workgroup).
template <bool LV>
__global__ __launch_bounds__(WG_THREADS) void drift_wg_kernel(const int32_t *sys_of, const int32_t *sys_off,
                                                              const int32_t *n_massive, const double *mstar,
                                                              int n_total, double *x, double *y, double *z,
                                                              double *vx, double *vy, double *vz, const double *m,
                                                              const double *rc, double dt, const int32_t *members,
                                                              const int32_t *group_start, const int32_t *list,
                                                              int32_t *flags, const double *rc_lv, int nlev)
{
    __shared__ BsWgShared S;
    const int n_list = list[0];
    for (int li = blockIdx.x; li < n_list; li += gridDim.x) {
        const int g = list[1 + li];
        const int k0 = group_start[g], nb = group_start[g + 1] - k0;
        const int k = threadIdx.x / BS_LANES;
        const int P = nb <= 16 ? 4 : (nb <= 32 ? 2 : 1);
        const int a = (threadIdx.x % BS_LANES) / P, part = (threadIdx.x % BS_LANES) % P;
        const double ms = mstar[sys_of[members[k0]]];
        __syncthreads(); // the previous group's LDS is no longer read
        if (k == 0 && part == 0 && a < nb) {
            const int b = members[k0 + a];
            const int sb = sys_of[b];
            S.m[a] = m[b];
            S.rc[a] = rc[b];
            S.r01[a] = 0.1 * rc[b];
            S.i09[a] = 1.0 / (0.9 * rc[b]);
            S.test[a] = b - sys_off[sb] >= n_massive[sb];
            if constexpr (LV)
                for (int l = 1; l < nlev; ++l) S.rcl[l - 1][a] = rc_lv[(size_t)(l - 1) * n_total + b];
        }
        if (threadIdx.x == 0) {
            S.nlev = nlev;
            S.kstar_att = 0;
        }
        __syncthreads();
        const bool act = a < nb;
        const int ai = act ? a : 0;
        const int b = members[k0 + ai];
        double Y[6] = {x[b], y[b], z[b], vx[b], vy[b], vz[b]};
        const bool ok = bs_workgroup<LV>(k, a, part, P, nb, act, S.test[ai] != 0, ms, S.rc[ai], S.r01[ai], S.i09[ai],
                                         S, Y, dt, 1e-12);
        // every thread has read its member's state before the first force evaluation's barrier
        if (act && k == 0 && part == 0) store_state(x, y, z, vx, vy, vz, b, Y);
        if (!ok && threadIdx.x == 0) atomicOr(flags, FLAG_NOCONVERGE);
    }
}

// skip: labels read, then reset to -1 (the list holds every body whose label is set)
__global__ __launch_bounds__(256) void kepler_list_kernel(const int32_t *sys_of, const double *mstar,
                                                          const int32_t *list, int n, int32_t *skip,
                                                          double *x, double *y, double *z, double *vx,
                                                          double *vy, double *vz, double dt, int32_t *flags)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int i = list[k];
    if (skip) {
        const int s = skip[i];
        skip[i] = -1;
        if (s >= 0) return;
    }
    double Y[6] = {x[i], y[i], z[i], vx[i], vy[i], vz[i]};
    if (!kepler_universal(Y[0], Y[1], Y[2], Y[3], Y[4], Y[5], mstar[sys_of[i]], dt)) atomicOr(flags, FLAG_KEPLER);
    store_state(x, y, z, vx, vy, vz, i, Y);
}

} // namespace

hipError_t launch_kepler_list(const Layout &L, const int32_t *list, int32_t n, double *x, double *y,
                              double *z, double *vx, double *vy, double *vz, double dt, int32_t *flags,
                              hipStream_t stream, int32_t *skip)
{
    if (n <= 0) return hipSuccess;
    kepler_list_kernel<<<(n + 255) / 256, 256, 0, stream>>>(L.sys_of, L.mstar, list, n, skip, x, y, z, vx, vy, vz,
                                                            dt, flags);
    return hipGetLastError();
}

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

hipError_t launch_momentum(const Layout &L, const double *vx, const double *vy, const double *vz,
                           const double *m, double *mom_part, hipStream_t stream)
{
    if (L.n_chunks == 0) return hipSuccess;
    momentum_kernel<<<L.n_chunks, SUN_THREADS, 0, stream>>>(L.chunks, m, vx, vy, vz, mom_part);
    return hipGetLastError();
}

hipError_t launch_uf_init(const int32_t *pairs, const int32_t *pair_count, int32_t pair_cap, int32_t *lab,
                          hipStream_t stream)
{
    // 256 workgroups walk the pairs: a round that has nothing to do returns at once, and its
    // launch costs less the fewer workgroups it dispatches
    uf_init_kernel<<<256, 256, 0, stream>>>(pairs, pair_count, pair_cap, lab);
    return hipGetLastError();
}

hipError_t launch_uf_hook(const int32_t *pairs, const int32_t *pair_count, int32_t pair_cap, int32_t *lab,
                          int32_t *changed, hipStream_t stream, const int32_t *run_if)
{
    uf_hook_kernel<<<256, 256, 0, stream>>>(pairs, pair_count, pair_cap, lab, changed, run_if);
    return hipGetLastError();
}

hipError_t launch_uf_compress(const Layout &L, int32_t *lab, hipStream_t stream, const int32_t *run_if)
{
    if (L.n_total == 0) return hipSuccess;
    uf_compress_kernel<<<(L.n_total + 255) / 256, 256, 0, stream>>>(L.n_total, lab, run_if);
    return hipGetLastError();
}

hipError_t launch_uf_slots(int n_members_max, const int32_t *members, const int32_t *n_members,
                           int32_t *member_slot, int32_t *lab, hipStream_t stream)
{
    if (n_members_max <= 0) return hipSuccess;
    uf_slots_kernel<<<(n_members_max + 255) / 256, 256, 0, stream>>>(members, n_members, member_slot, lab);
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

hipError_t launch_drift(const Layout &L, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, const double *m, const double *rc, double dt, const int32_t *members,
                        const int32_t *group_start, const int32_t *n_groups, int32_t *member_slot,
                        int32_t *flags, int big_groups, int bs_blocks, int32_t *wg_list, hipStream_t stream,
                        const double *rc_lv, int nlev, bool kepler, const DriftSide *side)
{
    if (L.n_total == 0) return hipSuccess;
    // one block per possible group: every group has >= 2 members; bs_blocks < 0: no group
    // blocks (the groups are integrated elsewhere), only the Kepler drift of non-members
    if (bs_blocks == 0) bs_blocks = CE_MAX_MEMBERS / 2;
    if (bs_blocks < 0) bs_blocks = 0;
    const int grid = bs_blocks + (kepler ? (L.n_total + BS_LANES - 1) / BS_LANES : 0);
    if (grid == 0) return hipSuccess;
    auto kern = nlev > 1 ? drift_kernel<true> : drift_kernel<false>;
    auto wg = nlev > 1 ? drift_wg_kernel<true> : drift_wg_kernel<false>;
    // the groups of 9..64 members: listed, then one workgroup each (1024 workgroups, or the
    // largest number such groups can reach, walk the list); they run beside the launch of the
    // smaller groups on the side stream when there is one and nothing is being captured
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (side && side->stream && bs_blocks > 0) {
        const hipError_t e = hipStreamIsCapturing(stream, &cs);
        if (e != hipSuccess) return e;
    }
    const bool fork = side && side->stream && bs_blocks > 0 && cs == hipStreamCaptureStatusNone;
    const int wg_grid = std::max(1, std::min(1024, bs_blocks));
    hipError_t e = hipSuccess;
    if (bs_blocks > 0) wg_list_kernel<<<1, 1024, 0, stream>>>(group_start, n_groups, bs_blocks, wg_list);
    if (fork) {
        if ((e = hipEventRecord(side->fork, stream)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(side->stream, side->fork, 0)) != hipSuccess) return e;
        wg<<<wg_grid, WG_THREADS, 0, side->stream>>>(L.sys_of, L.sys_off, L.n_massive, L.mstar, L.n_total, x, y, z, vx,
                                                     vy, vz, m, rc, dt, members, group_start, wg_list, flags, rc_lv,
                                                     nlev);
        if ((e = hipEventRecord(side->join, side->stream)) != hipSuccess) return e;
    }
    kern<<<grid, BS_LANES, 0, stream>>>(L.sys_of, L.sys_off, L.n_massive, L.mstar, L.n_total, x, y, z, vx, vy, vz, m,
                                        rc, dt, members, group_start, n_groups, member_slot, flags, big_groups,
                                        bs_blocks, rc_lv, nlev);
    if (bs_blocks > 0 && !fork)
        wg<<<wg_grid, WG_THREADS, 0, stream>>>(L.sys_of, L.sys_off, L.n_massive, L.mstar, L.n_total, x, y, z, vx, vy, vz,
                                               m, rc, dt, members, group_start, wg_list, flags, rc_lv, nlev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (fork && (e = hipStreamWaitEvent(stream, side->join, 0)) != hipSuccess) return e;
    return hipGetLastError();
}

} // namespace genga
