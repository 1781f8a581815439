// Bulirsch-Stoer over dt for encounter groups larger than one wavefront.  In the
// encounter-dominated phase (Sect. 3.5: many planetesimals form almost one large close-encounter
// group and the run is bound by the Bulirsch-Stoer step) a group can hold most of a disc, so
// its state is spread over the whole GPU.  Method, tolerance and step control are those of
// the one-wave path and the oracle: modified midpoint with n_k = 2(k+1) sub-steps, polynomial
// extrapolation in h^2 (here in Lagrange form, relative to T(0,0)), acceptance at the first
// column k >= 1 whose estimate meets tol on the group's position / velocity scales, next step
// doubled / kept / halved, rejected steps shrunk by shrink_factor.
//
// One attempt is a fixed sequence of launches over all large groups at once: a force
// evaluation and midpoint update per sub-step (64 targets per workgroup, 8 or 16 waves that
// split the group's members as sources), then per column an error launch and a decision
// launch.  A group that has accepted a column, or reached dt, skips the rest.  The host
// repeats attempts until no group is active.
//
// The members of a group are ordered by ring and azimuth about the star (by the host, once per
// step), so a tile of 64 consecutive members is compact in space.  Each state buffer carries the
// bounding box of every tile, written by the launch that wrote the positions; a wave skips a
// source tile whose box is farther than the group's largest r_crit from the target tile's
// box, since no pair across the two can lie inside r_crit,ab.  The order only decides how
// much is skipped, never the result beyond rounding.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

using CD = const __attribute__((address_space(4))) double;
using CI = const __attribute__((address_space(4))) int32_t;

constexpr int GB_TILE = 64;
constexpr int GB_THREADS = 256;

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

// max into slot[g] for every lane with use = true: the lanes of the wave's first group
// combine first and one of them updates the slot; lanes of another group update their own.
// Every lane of the wave must call it.
__device__ __forceinline__ void wave_atomic_max(unsigned long long *slot, int g, bool use,
                                                unsigned long long v)
{
    const unsigned long long any = __ballot(use);
    if (!any) return;
    const int leader = __ffsll((long long)any) - 1;
    const int g0 = __shfl(g, leader, 64);
    const bool same = use && g == g0;
    unsigned long long m = same ? v : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(m, o, 64);
        m = w > m ? w : m;
    }
    if ((int)(threadIdx.x & 63) == leader) atomicMax(&slot[g0], m);
    if (use && !same) atomicMax(&slot[g], v);
}

// Per group: the step's start (t = 0, H = dt) and the star's mass; the largest squared
// candidate radius starts at 0 for big_setup_kernel's maxima.
__global__ __launch_bounds__(64) void big_setup_groups_kernel(BigBs b, const int32_t *sys_of, const double *mstar,
                                                              const int32_t *members, double dt)
{
    const int g = blockIdx.x * 64 + threadIdx.x;
    if (g >= b.dims[0]) return;
    if (g == 0) b.dtp[0] = dt;
    b.rcmax2[g] = 0.0;
    b.mstar[g] = mstar[sys_of[members[b.k0[g]]]];
    b.t[g] = 0.0;
    b.H[g] = dt;
    b.attempts[g] = 0;
    b.done[g] = 0;
    if (b.skin) {
        b.stale[g] = 0;
        b.keep[g] = 0;
    }
}

// Flat member f of large group g (one wave per tile): body index, constants, state
// Y[q * M + f], and the group's largest squared candidate radius (a maximum of bit patterns,
// which order non-negative doubles, so the result does not depend on the order of arrival).
__global__ __launch_bounds__(64) void big_setup_kernel(BigBs b, const int32_t *sys_of, const int32_t *sys_off,
                                                       const int32_t *n_massive, const double *x, const double *y,
                                                       const double *z, const double *vx, const double *vy,
                                                       const double *vz, const double *m, const double *rc,
                                                       const double *rc_lv, int n_total)
{
    const int4 tile = b.tiles[blockIdx.x];
    const int g = tile.x;
    const size_t M = (size_t)b.dims[1];
    double mx = 0.0;
    if ((int)threadIdx.x < tile.z) {
        const int f = tile.y + threadIdx.x, body = b.body[f], s = sys_of[body];
        b.grp[f] = g;
        b.rc[f] = rc[body];
        b.i09[f] = 1.0 / (0.9 * rc[body]);
        b.mass[f] = m[body];
        b.test[f] = body - sys_off[s] >= n_massive[s];
        b.Y[0 * M + f] = x[body];
        b.Y[1 * M + f] = y[body];
        b.Y[2 * M + f] = z[body];
        b.Y[3 * M + f] = vx[body];
        b.Y[4 * M + f] = vy[body];
        b.Y[5 * M + f] = vz[body];
        if (b.skin) {
            // every step starts from twice the bound's estimate, so a step's lists depend on its
            // starting state only (a run resumed from a saved state repeats them bit for bit)
            b.skin[body] = 2.0;
            b.crossed[f] = 0;
            b.amut[f] = 0.0;
        }
        // candidate radius: the deepest level's r_crit
        double rd = rc[body];
        for (int k = 1; k < b.nlev; ++k) {
            rd = rc_lv[(size_t)(k - 1) * n_total + body];
            b.rcl[(size_t)(k - 1) * b.cap_M + f] = rd;
        }
        mx = sq_rn(rd);
    }
    for (int s = 32; s > 0; s >>= 1) mx = fmax(mx, __shfl_xor(mx, s, 64));
    if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned long long *>(b.rcmax2) + g, dbits(mx));
}

// Start of an attempt, per group.
__global__ __launch_bounds__(64) void big_begin_kernel(BigBs b, int32_t *flags)
{
    const double dt = b.dtp[0];
    const int g = blockIdx.x * 64 + threadIdx.x;
    if (g >= b.dims[0] || b.done[g]) return;
    double H = b.H[g];
    const double t = b.t[g];
    const bool last = H >= (dt - t) * (1.0 - 0x1p-30); // ends the interval (exactly)
    if (last) H = dt - t;
    const int att = b.attempts[g] + 1;
    b.attempts[g] = att;
    if (b.skin) b.stale[g] = 0; // a void attempt is repeated with wider margins where they were crossed
    if (H < dt * 0x1p-40 || att > 20000) {
        atomicOr(flags, FLAG_NOCONVERGE);
        b.done[g] = 1;
        return;
    }
    b.H[g] = H;
    b.last[g] = last;
    b.acc[g] = -1;
    b.sr[g] = 0;
    b.sv[g] = 0;
    for (int k = 0; k < BS_KMAX; ++k) b.err[g * BS_KMAX + k] = 0;
}

// Position and velocity scales of each group: max |r|, max |v| over its members (max of
// non-negative doubles through their bit patterns, so the order of updates does not matter).
__global__ __launch_bounds__(GB_THREADS) void big_scale_kernel(BigBs b)
{
    const int f0 = blockIdx.x * GB_THREADS + threadIdx.x;
    const bool in = f0 < b.dims[1];
    const int f = in ? f0 : 0;
    const int g = b.grp[f];
    const bool use = in && !b.done[g];
    const size_t M = (size_t)b.dims[1];
    const double *Y = b.Y;
    const double rr = sqrt(sep2_rn(Y[f], Y[M + f], Y[2 * M + f]));
    const double vv = sqrt(sep2_rn(Y[3 * M + f], Y[4 * M + f], Y[5 * M + f]));
    wave_atomic_max(b.sr, g, use, dbits(rr));
    wave_atomic_max(b.sv, g, use, dbits(vv));
}

// Tile boxes of the attempt's starting state Y.
__global__ __launch_bounds__(64) void big_box_kernel(BigBs b)
{
    for (int me = blockIdx.x; me < b.dims[2]; me += gridDim.x) {
        const int4 tile = b.tiles[me];
        if (b.done[tile.x]) continue;
        const size_t M = (size_t)b.dims[1];
        const bool v = (int)threadIdx.x < tile.z;
        const int f = tile.y + (v ? (int)threadIdx.x : 0);
        tile_box(v, b.Y[f], b.Y[M + f], b.Y[2 * M + f], b.bb, me);
    }
}

// One sub-step of column k for the targets of a tile (one workgroup per tile): the (1 - K)
// share of the Newtonian forces from the group's other members at state Z, then
//   mode 0: OUT = Z + h f(Z)            (first sub-step, Z = Y)
//   mode 1: OUT = ZM + 2 h f(Z)         (OUT may be ZM's buffer: each lane rewrites its own)
//   mode 2: T(k, 0) = (ZM + Z + h f(Z)) / 2, into tcol[k]
// and, in modes 0 and 1, the tile's box in OUT's box array.  The workgroup first lists the
// source tiles in reach of the target tile (box gap within the largest r_crit); their
// quarters (16 members) are dealt out to the waves, so the few near tiles are spread over
// many waves.  Source positions and boxes come through scalar loads: neither is written by
// this launch.
template <bool LV, int W>
__device__ __forceinline__ void substep_tile(const BigBs &b, int me, int k, int mode, const double *Z,
                                             const double *ZM, double *OUT, const double *bbZ, double *bbOUT)
{
    __shared__ double red[3][W][GB_TILE];
    const int4 tile = b.tiles[me]; // (group, first member, count, -)
    const int g = tile.x;
    if (b.done[g] || b.acc[g] >= 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const size_t M = (size_t)b.dims[1];
    const int o = b.off[g], nb = b.off[g + 1] - o;
    const int tf = b.tfirst[g], nt = b.tfirst[g + 1] - tf;
    const bool valid = lane < tile.z;
    const int fa = tile.y + (valid ? lane : 0);
    const double xa = Z[fa], ya = Z[M + fa], za = Z[2 * M + fa];
    const double rca = b.rc[fa];
    const bool testa = b.test[fa] != 0;
    // candidate radius: the group's largest r_crit^2, with a margin for the contracted r^2;
    // a source tile is skipped when the gap between the boxes exceeds it
    const double T = b.rcmax2[g] * (1.0 + 0x1p-40);
    const double Tcull = b.rcmax2[g] * (1.0 + 0x1p-30);
    CD *ZX = (CD *)Z;
    CD *ZY = (CD *)(Z + M);
    CD *ZZ = (CD *)(Z + 2 * M);
    CD *RC = (CD *)b.rc;
    CD *MS = (CD *)b.mass;
    CI *TS = (CI *)b.test;
    CD *BB = (CD *)bbZ;
    const double tlx = BB[me * 8 + 0], tly = BB[me * 8 + 1], tlz = BB[me * 8 + 2];
    const double thx = BB[me * 8 + 3], thy = BB[me * 8 + 4], thz = BB[me * 8 + 5];
    double ax = 0.0, ay = 0.0, az = 0.0;
    const double i09a = b.i09[fa];
    CD *I9 = (CD *)b.i09;
    // levels 1..nlev-1: the target's radii, and the source radii through scalar loads
    double rcal[LEVELS_MAX - 1] = {};
    CD *RCL = (CD *)b.rcl;
    if constexpr (LV)
        for (int l = 1; l < b.nlev; ++l) rcal[l - 1] = b.rcl[(size_t)(l - 1) * b.cap_M + fa];
    // the (1 - K) Newtonian terms of sources j .. j + cnt - 1 (cnt <= 4), side by side and
    // without branches: a pair outside r_crit,ab, the target itself and a test-test pair get
    // weight zero; the terms are added in source order
    auto pairs4 = [&](int j, int cnt, const double (&dx)[4], const double (&dy)[4], const double (&dz)[4]) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int jj = min(j + u, j + cnt - 1);
            const double rcj = RC[jj], mj = MS[jj], i9j = I9[jj];
            const bool tj = TS[jj] != 0;
            const bool own = rca >= rcj;
            const double rcab = own ? rca : rcj;
            const double q = sep2_rn(dx[u], dy[u], dz[u]);
            const double rq = inv_sqrt64(q);
            const double yv = (q * rq - 0.1 * rcab) * (own ? i09a : i9j);
            const double y2 = yv * yv;
            const double kv = yv <= 0.0 ? 0.0 : (yv >= 1.0 ? 1.0 : y2 / (2.0 * y2 - 2.0 * yv + 1.0));
            double w = 1.0 - kv, rdeep = rcab;
            if constexpr (LV) {
                // prod over the deeper levels of (1 - K_l); inside the deepest radius every
                // level's radius holds the pair, as the radii do not grow with the level
                for (int l = 1; l < b.nlev; ++l) {
                    const double rcl_ab = fmax(rcal[l - 1], RCL[(size_t)(l - 1) * b.cap_M + jj]);
                    w *= 1.0 - changeover_k((q * rq - 0.1 * rcl_ab) / (0.9 * rcl_ab));
                    rdeep = rcl_ab;
                }
            }
            const bool in = u < cnt && j + u != fa && !(testa && tj) && q < sq_rn(rdeep);
            t[u] = in ? mj * w * (rq * rq) * rq : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ax = fma(t[u], dx[u], ax);
            ay = fma(t[u], dy[u], ay);
            az = fma(t[u], dz[u], az);
        }
    };
    // the source tiles in reach of this target tile, in tile order: one test per thread (in
    // passes of W * 64 tiles), then an ordered compaction (ballots within a wave, wave offsets
    // through LDS)
    __shared__ int near_tile[BIG_TILES_PER_GROUP];
    __shared__ int wave_cnt[W];
    int n_near = 0;
    for (int t0 = 0; t0 < nt; t0 += W * GB_TILE) {
        bool near = false;
        const int tt = t0 + (int)threadIdx.x;
        if (tt < nt) {
            const double *bs = bbZ + (size_t)(tf + tt) * 8;
            const double gx = fmax(0.0, fmax(bs[0] - thx, tlx - bs[3]));
            const double gy = fmax(0.0, fmax(bs[1] - thy, tly - bs[4]));
            const double gz = fmax(0.0, fmax(bs[2] - thz, tlz - bs[5]));
            near = (gx * gx + gy * gy) + gz * gz <= Tcull; // else no pair of the two tiles is close
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
    // units of 16 sources (quarters of the near tiles), dealt out to the waves; whole quads
    // index the sources directly, so the four sources' words come in one scalar load per array
    for (int u = wave; u < 4 * n_near; u += W) {
        const int st = near_tile[u >> 2];
        const int jb = o + GB_TILE * st + 16 * (u & 3), je = min(jb + 16, o + nb);
        int j = jb;
        for (; j + 4 <= je; j += 4) {
            double dx[4], dy[4], dz[4], q[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                dx[v] = ZX[j + v] - xa;
                dy[v] = ZY[j + v] - ya;
                dz[v] = ZZ[j + v] - za;
                q[v] = fma(dx[v], dx[v], fma(dy[v], dy[v], dz[v] * dz[v]));
            }
            if (fmin(fmin(q[0], q[1]), fmin(q[2], q[3])) < T) pairs4(j, 4, dx, dy, dz);
        }
        if (j < je) {
            const int cnt = je - j;
            double dx[4], dy[4], dz[4], q[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int jj = min(j + v, je - 1);
                dx[v] = ZX[jj] - xa;
                dy[v] = ZY[jj] - ya;
                dz[v] = ZZ[jj] - za;
                q[v] = v < cnt ? fma(dx[v], dx[v], fma(dy[v], dy[v], dz[v] * dz[v])) : INFINITY;
            }
            if (fmin(fmin(q[0], q[1]), fmin(q[2], q[3])) < T) pairs4(j, cnt, dx, dy, dz);
        }
    }
    red[0][wave][lane] = ax;
    red[1][wave][lane] = ay;
    red[2][wave][lane] = az;
    __syncthreads();
    if (wave != 0) return;
    const double ri = inv_sqrt64(sep2_rn(xa, ya, za));
    const double s = -b.mstar[g] * (ri * ri) * ri;
    double d[6] = {Z[3 * M + fa], Z[4 * M + fa], Z[5 * M + fa], s * xa, s * ya, s * za};
    for (int w = 0; w < W; ++w) {
        d[3] += red[0][w][lane];
        d[4] += red[1][w][lane];
        d[5] += red[2][w][lane];
    }
    if (mode == 0 && k == 0 && valid && b.amut) {
        // the pair acceleration at the attempt's start, for the list path's bounds
        double px = 0.0, py = 0.0, pz = 0.0;
        for (int w = 0; w < W; ++w) {
            px += red[0][w][lane];
            py += red[1][w][lane];
            pz += red[2][w][lane];
        }
        b.amut[fa] = sqrt(sep2_rn(px, py, pz));
    }
    const double h = b.H[g] / (2 * (k + 1));
    if (mode == 2) {
        double tk[6];
        for (int q = 0; q < 6; ++q) tk[q] = 0.5 * (ZM[q * M + fa] + Z[q * M + fa] + h * d[q]);
        if (valid) {
            double *T0 = b.tcol + (size_t)k * 6 * M;
            for (int q = 0; q < 6; ++q) T0[q * M + fa] = tk[q];
        }
        if (k == 0) return;
        // the column's error estimate for this member (Lagrange form of T(k, k) - T(k, k-1),
        // relative to T(0, 0)) into the group's maximum: per position / velocity element over
        // the group's scales; a non-finite estimate is kept as the all-ones pattern
        double dp = 0.0, dv = 0.0;
        bool bad = false;
        for (int q = 0; q < 6; ++q) {
            const double t0 = b.tcol[q * M + fa];
            double sum = 0.0;
            for (int jj = 1; jj <= k; ++jj) {
                const double v = jj == k ? tk[q] : b.tcol[((size_t)jj * 6 + q) * M + fa];
                sum = fma(LAGRANGE.d[k][jj], v - t0, sum);
            }
            if (q < 3) dp = fmax(dp, fabs(sum));
            else dv = fmax(dv, fabs(sum));
            bad |= !(sum == sum);
        }
        const double e = fmax(dp / bitsd(b.sr[g]), dv / bitsd(b.sv[g]));
        wave_atomic_max(b.err + k, g * BS_KMAX, valid, (bad || !(e == e)) ? ~0ull : dbits(e));
        return;
    }
    double nx[6];
    for (int q = 0; q < 6; ++q) nx[q] = (mode == 0 ? Z[q * M + fa] : ZM[q * M + fa]) + (mode == 0 ? h : 2.0 * h) * d[q];
    if (valid)
        for (int q = 0; q < 6; ++q) OUT[q * M + fa] = nx[q];
    tile_box(valid, nx[0], nx[1], nx[2], bbOUT, me);
}

// The tiles are visited grid-stride, so that a launch can be sized to the layout at hand
// (the captured attempt is kept per grid size) rather than to the largest one.
template <bool LV, int W>
__global__ __launch_bounds__(GB_TILE *W) void big_substep_kernel(BigBs b, int k, int mode, const double *Z,
                                                                const double *ZM, double *OUT, const double *bbZ,
                                                                double *bbOUT)
{
    for (int me = blockIdx.x; me < b.dims[2]; me += gridDim.x) {
        if (me != (int)blockIdx.x) __syncthreads(); // the previous tile's LDS is free again
        substep_tile<LV, W>(b, me, k, mode, Z, ZM, OUT, bbZ, bbOUT);
    }
}


// ---------------------------------------------------------------------------------------------
// The list path.  At an attempt's start each member lists the sources that can come within
// r_crit,ab during the attempt.  The sub-step states of the modified midpoint method with step h
// under a constant pull A lie at Y + V tau + A (tau^2 - h^2) / 2 for odd j (tau = j h) and at
// Y + V tau + A tau^2 / 2 for even j; with A the star's pull at Y that is each member's
// prediction P_j, and S bounds its departure from it (the change of the star's pull along the
// path, the jerk 3 Mstar |V| / |Y|^3 over H^3 / 6, and the members' mutual pull a_mut over
// H^2 / 2, a_mut as the last force evaluation at an attempt's start found it (0 before the
// step's first), times the body's skin factor, at least 2).  A source is listed when the
// straight lines Y + V t of the two members come within
// r_crit,ab + S_a + S_b + |A_a - A_b| H^2 / 2 over [0, H]: then no unlisted pair can be inside
// r_crit,ab at a state where every member is within S of its prediction.  Every sub-step state
// checks |Z - P_j| <= S for every member; a crossed bound marks the group stale: the attempt is
// neither accepted nor counted as rejected, and the next one lists again, with four times the
// skin of each member that crossed its bound (bodies in close encounters, whose mutual pull the
// prediction leaves out, get wider margins for the rest of the step; every step starts at 2).
// The lists are in a fixed order, so the sums are deterministic.
// ---------------------------------------------------------------------------------------------

// The member's prediction constants: the star's pull A at Y and the bound S for step H.
struct ListMember {
    double ax, ay, az, s;
};

__device__ __forceinline__ ListMember list_member(double skin, double ms, double H, double x, double y, double z,
                                                  double u, double v, double w, double amut)
{
    const double r2 = sep2_rn(x, y, z);
    const double ri = inv_sqrt64(r2);
    const double a = ms / r2;                 // |A|
    const double c = -a * ri;                 // A = -Mstar Y / |Y|^3
    const double vv = sqrt(sep2_rn(u, v, w));
    ListMember m;
    m.ax = c * x;
    m.ay = c * y;
    m.az = c * z;
    m.s = skin * 0.5 * (a * ri * vv * H + amut) * (H * H);
    return m;
}

// The source records of the list sub-steps: the constant words of every state buffer's records
// and the positions of Y (the sub-steps write those of B1 and B2).
__global__ __launch_bounds__(GB_THREADS) void big_src_kernel(BigBs b)
{
    const int f = blockIdx.x * GB_THREADS + threadIdx.x;
    if (f >= b.dims[1]) return;
    const size_t M = (size_t)b.dims[1], cm = (size_t)b.cap_M;
    const double2 c = make_double2(b.rc[f], b.test[f] ? -b.i09[f] : b.i09[f]);
    for (int i = 0; i < 3; ++i) reinterpret_cast<double2 *>(b.rec + (i * cm + f) * 8)[2] = c;
    reinterpret_cast<double4 *>(b.rec + (size_t)f * 8)[0] = make_double4(b.Y[f], b.Y[M + f], b.Y[2 * M + f], b.mass[f]);
}

// Per tile: the box swept by its members' straight lines over [0, H], and the largest
// S + |A| H^2 / 2 of its members.
__global__ __launch_bounds__(64) void big_sweep_kernel(BigBs b)
{
    for (int me = blockIdx.x; me < b.dims[2]; me += gridDim.x) {
        const int4 tile = b.tiles[me];
        const int g = tile.x;
        if (b.done[g] || b.keep[g]) continue;
        const size_t M = (size_t)b.dims[1];
        const bool v = (int)threadIdx.x < tile.z;
        const int f = tile.y + (v ? (int)threadIdx.x : 0);
        const double H = b.H[g];
        const double x = b.Y[f], y = b.Y[M + f], z = b.Y[2 * M + f];
        const double u = b.Y[3 * M + f], vy = b.Y[4 * M + f], w = b.Y[5 * M + f];
        const double x1 = fma(u, H, x), y1 = fma(vy, H, y), z1 = fma(w, H, z);
        double sk = 2.0;
        if (v) {
            const int body = b.body[f];
            sk = b.skin[body];
            if (b.crossed[f]) { // the member left its bound in the last attempt: four times wider
                sk *= 4.0;
                b.skin[body] = sk;
                b.crossed[f] = 0;
            }
        }
        const ListMember lm = list_member(sk, b.mstar[g], H, x, y, z, u, vy, w, v ? b.amut[f] : 0.0);
        if (v) b.pred[f] = make_double4(lm.ax, lm.ay, lm.az, lm.s);
        const double lo[3] = {wave_minv(v ? fmin(x, x1) : INFINITY), wave_minv(v ? fmin(y, y1) : INFINITY),
                              wave_minv(v ? fmin(z, z1) : INFINITY)};
        const double hi[3] = {wave_maxv(v ? fmax(x, x1) : -INFINITY), wave_maxv(v ? fmax(y, y1) : -INFINITY),
                              wave_maxv(v ? fmax(z, z1) : -INFINITY)};
        const double ext =
            wave_maxv(v ? lm.s + 0.5 * sqrt(sep2_rn(lm.ax, lm.ay, lm.az)) * H * H : 0.0);
        const int lane = threadIdx.x;
        if (lane < 3) {
            b.sbb[me * 8 + lane] = lo[lane];
            b.sbb[me * 8 + 3 + lane] = hi[lane];
        }
        if (lane == 0) b.sbb[me * 8 + 6] = ext;
    }
}

// One source j for the target lane's list segment (wave-uniform j): listed when the straight
// lines come within r = r_crit,ab + S_a + S_j + |A_a - A_j|_1 H^2 / 2 over [0, H] (the 1-norm
// bounds the length of the difference).  The minimum of |d + v t|^2 over [0, H] is taken
// without a division: at t = 0 when d.v >= 0, at t = H when -d.v >= |v|^2 H, else it is
// |d|^2 - (d.v)^2 / |v|^2, compared as (|d|^2 - r^2) |v|^2 < (d.v)^2.
__device__ __forceinline__ void list_source(const BigBs &b, bool valid, int fa, bool testa, double rfa,
                                            double xa, double ya, double za, double ua, double va, double wa,
                                            double4 pa, double H, int j, double xj, double yj, double zj, double uj,
                                            double vj, double wj, double rj, bool testj, double4 pj, int32_t *row,
                                            int &len, bool &over)
{
    const double dx = xj - xa, dy = yj - ya, dz = zj - za;
    const double du = uj - ua, dv = vj - va, dw = wj - wa;
    const double dd = sep2_rn(dx, dy, dz), vv = sep2_rn(du, dv, dw);
    const double dp = (dx * du + dy * dv) + dz * dw;
    const double r = fmax(rfa, rj) + pa.w + pj.w +
                     0.5 * (fabs(pj.x - pa.x) + fabs(pj.y - pa.y) + fabs(pj.z - pa.z)) * (H * H);
    // a margin of 2^-30 covers the rounding of the distance
    const double r2 = r * r * (1.0 + 0x1p-30);
    bool close;
    if (dp >= 0.0 || vv == 0.0) {
        close = dd < r2;
    } else if (-dp >= vv * H) {
        close = sep2_rn(fma(du, H, dx), fma(dv, H, dy), fma(dw, H, dz)) < r2;
    } else {
        close = (dd - r2) * vv < dp * dp;
    }
    if (valid && close && j != fa && !(testa && testj)) {
        if (len < BIG_LIST_SEG) row[len] = j;
        else over = true;
        ++len;
    }
}

// A segment of the lists of a target tile's members (one wave per tile and segment; segment s
// takes the group's source tiles tt = s, s + BIG_LIST_SEGS, ...): the source tiles whose swept
// boxes lie within the largest radius plus both tiles' largest extents, then their sources on
// the straight lines, in quads whose words come through scalar loads.
template <bool LV>
__global__ __launch_bounds__(64) void big_list_kernel(BigBs b)
{
    CD *YA = (CD *)b.Y;
    CD *SB = (CD *)b.sbb;
    CD *RC = (CD *)b.rc;
    CI *TS = (CI *)b.test;
    CD *RL = (CD *)b.rcl;
    CD *PR = (CD *)b.pred; // (A, S) of member j at PR[4 j .. 4 j + 3]
    for (int ms = blockIdx.x; ms < b.dims[2] * BIG_LIST_SEGS; ms += gridDim.x) {
        const int me = ms / BIG_LIST_SEGS, seg = ms % BIG_LIST_SEGS;
        const int4 tile = b.tiles[me];
        const int g = tile.x;
        if (b.done[g] || b.keep[g]) continue;
        const size_t M = (size_t)b.dims[1];
        const size_t lvo = LV ? (size_t)(b.nlev - 2) * b.cap_M : 0; // the deepest level's radii
        const int lane = threadIdx.x;
        const bool valid = lane < tile.z;
        const int fa = tile.y + (valid ? lane : 0);
        const int o = b.off[g], nb = b.off[g + 1] - o;
        const int tf = b.tfirst[g], nt = b.tfirst[g + 1] - tf;
        const double H = b.H[g];
        const double xa = b.Y[fa], ya = b.Y[M + fa], za = b.Y[2 * M + fa];
        const double ua = b.Y[3 * M + fa], va = b.Y[4 * M + fa], wa = b.Y[5 * M + fa];
        const double4 pa = b.pred[fa];
        const bool testa = b.test[fa] != 0;
        const double rfa = LV ? b.rcl[lvo + fa] : b.rc[fa];
        const double rmax = sqrt(b.rcmax2[g]);
        const double tlx = SB[me * 8 + 0], tly = SB[me * 8 + 1], tlz = SB[me * 8 + 2];
        const double thx = SB[me * 8 + 3], thy = SB[me * 8 + 4], thz = SB[me * 8 + 5], et = SB[me * 8 + 6];
        int32_t *row = b.nl + (size_t)fa * BIG_LIST_CAP + seg * BIG_LIST_SEG;
        int len = 0;
        bool over = false;
        for (int tt = seg; tt < nt; tt += BIG_LIST_SEGS) {
            const int st = tf + tt;
            const double gx = fmax(0.0, fmax(SB[st * 8 + 0] - thx, tlx - SB[st * 8 + 3]));
            const double gy = fmax(0.0, fmax(SB[st * 8 + 1] - thy, tly - SB[st * 8 + 4]));
            const double gz = fmax(0.0, fmax(SB[st * 8 + 2] - thz, tlz - SB[st * 8 + 5]));
            const double cut = rmax + et + SB[st * 8 + 6];
            if ((gx * gx + gy * gy) + gz * gz > cut * cut * (1.0 + 0x1p-30)) continue;
            const int jb = o + 64 * tt, je = min(jb + 64, o + nb);
            int j = jb;
            for (; j + 4 <= je; j += 4) {
                double X[4], Yv[4], Zv[4], U[4], V[4], W[4], R[4];
                double4 Pj[4];
                bool T[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    X[q] = YA[j + q];
                    Yv[q] = YA[M + j + q];
                    Zv[q] = YA[2 * M + j + q];
                    U[q] = YA[3 * M + j + q];
                    V[q] = YA[4 * M + j + q];
                    W[q] = YA[5 * M + j + q];
                    R[q] = LV ? RL[lvo + j + q] : RC[j + q];
                    T[q] = TS[j + q] != 0;
                    Pj[q] = make_double4(PR[4 * (j + q)], PR[4 * (j + q) + 1], PR[4 * (j + q) + 2],
                                         PR[4 * (j + q) + 3]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    list_source(b, valid, fa, testa, rfa, xa, ya, za, ua, va, wa, pa, H, j + q, X[q], Yv[q], Zv[q],
                                U[q], V[q], W[q], R[q], T[q], Pj[q], row, len, over);
            }
            for (; j < je; ++j)
                list_source(b, valid, fa, testa, rfa, xa, ya, za, ua, va, wa, pa, H, j, YA[j], YA[M + j],
                            YA[2 * M + j], YA[3 * M + j], YA[4 * M + j], YA[5 * M + j], LV ? RL[lvo + j] : RC[j],
                            TS[j] != 0, make_double4(PR[4 * j], PR[4 * j + 1], PR[4 * j + 2], PR[4 * j + 3]),
                            row, len, over);
        }
        if (valid) b.nlen[(size_t)fa * BIG_LIST_SEGS + seg] = min(len, BIG_LIST_SEG);
        if (__ballot(over) && lane == 0) {
            atomicOr(b.ovf, 1);
            b.stale[g] = 1;
        }
    }
}

// Per target tile (thread = member m, segment s): the source tiles holding an entry of one of
// its members' lists become the tile's slots, in tile order (more than BIG_LIST_SLOTS void the
// attempt and send the step to the tile path), and each member's segments are written as one
// run of slot positions, slot * 64 + the source's position in its tile.
constexpr int LOC_THREADS = 64 * BIG_LIST_SEGS; // one thread per (member, segment) of a tile

__global__ __launch_bounds__(LOC_THREADS) void big_localize_kernel(BigBs b)
{
    static_assert(BIG_LIST_SLOTS * 64 <= 65536, "16-bit slot positions");
    __shared__ int mark[BIG_TILES_PER_GROUP];
    __shared__ int wsum[LOC_THREADS / 64];
    for (int me = blockIdx.x; me < b.dims[2]; me += gridDim.x) {
        const int4 tile = b.tiles[me];
        const int g = tile.x;
        if (b.done[g] || b.keep[g]) continue; // the whole block
        const int o = b.off[g], nb = b.off[g + 1] - o, nt = b.tfirst[g + 1] - b.tfirst[g];
        for (int i = threadIdx.x; i < nt; i += LOC_THREADS) mark[i] = 0;
        __syncthreads();
        const int m = threadIdx.x / BIG_LIST_SEGS, s = threadIdx.x % BIG_LIST_SEGS;
        const bool valid = m < tile.z;
        const int f = tile.y + (valid ? m : 0);
        const int32_t *nlen = b.nlen + (size_t)f * BIG_LIST_SEGS;
        int start = 0, all = 0;
        for (int q = 0; q < BIG_LIST_SEGS; ++q) {
            const int l = nlen[q];
            start += q < s ? l : 0;
            all += l;
        }
        const int len = valid ? nlen[s] : 0;
        const int32_t *row = b.nl + (size_t)f * BIG_LIST_CAP + s * BIG_LIST_SEG;
        for (int e = 0; e < len; ++e) mark[(row[e] - o) >> 6] = 1;
        __syncthreads();
        // ordered compaction of the marks: thread t takes tiles [t per, (t + 1) per)
        const int per = (nt + LOC_THREADS - 1) / LOC_THREADS;
        const int t0 = (int)threadIdx.x * per, t1 = min(t0 + per, nt);
        int cnt = 0;
        for (int i = t0; i < t1; ++i) cnt += mark[i];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        int incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d, 64);
            if (lane >= d) incl += v;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int pos = incl - cnt, total = 0;
        for (int w = 0; w < LOC_THREADS / 64; ++w) {
            pos += w < wave ? wsum[w] : 0;
            total += wsum[w];
        }
        for (int i = t0; i < t1; ++i)
            if (mark[i]) {
                if (pos < BIG_LIST_SLOTS) b.slot[me * BIG_LIST_SLOTS + pos] = make_int2(o + 64 * i, min(64, nb - 64 * i));
                mark[i] = pos++;
            }
        __syncthreads();
        if (threadIdx.x == 0) {
            b.nslot[me] = min(total, BIG_LIST_SLOTS);
            if (total > BIG_LIST_SLOTS) {
                atomicOr(b.ovf, 1);
                b.stale[g] = 1;
            }
        }
        if (total <= BIG_LIST_SLOTS) {
            uint16_t *out = b.ll + (size_t)f * BIG_LIST_CAP + start;
            for (int e = 0; e < len; ++e) {
                const int r = row[e] - o;
                out[e] = (uint16_t)(mark[r >> 6] * 64 + (r & 63));
            }
        }
        // a tile beyond the slots lists nothing (its attempt is void)
        if (valid && s == 0) b.ltot[f] = total <= BIG_LIST_SLOTS ? all : 0;
        __syncthreads(); // the marks are cleared for the next tile
    }
}

// Group g's acceptance once column k (>= 1) has been decided: its column if it is the first
// whose estimate meets tol, unless the attempt is void (a sub-step left the lists' bound).  On
// the list path every launch that needs the verdict takes it itself, from the same words, and
// one thread per group stores it in acc for the launches after it.
__device__ __forceinline__ int decided(const BigBs &b, int g, int k, double tol)
{
    const int a = b.acc[g];
    if (a >= 0 || k < 1 || b.done[g] || (b.skin && b.stale[g])) return a;
    const unsigned long long e = b.err[g * BS_KMAX + k];
    return (e != ~0ull && bitsd(e) <= tol) ? k : -1;
}

// What follows a member's pair sum in a sub-step: the star's pull, then the midpoint update of
// OUT (modes 0 and 1, with the positions of OUT's source records) or, in mode 2, T(k, 0) and
// the group's error estimate of column k.  Every lane of the wave calls it; `lead` marks the
// member's first lane, `act` the members of an active group.
__device__ __forceinline__ void member_tail(const BigBs &b, int k, int mode, int g, int fa, bool act, bool lead,
                                            double xa, double ya, double za, double ax, double ay, double az,
                                            const double *Z, const double *ZM, double *OUT, double *ROUT)
{
    const size_t M = (size_t)b.dims[1];
    if (mode == 0 && k == 0 && lead) {
        b.amut[fa] = sqrt(sep2_rn(ax, ay, az));
        b.a0[fa] = ax;
        b.a0[M + fa] = ay;
        b.a0[2 * M + fa] = az;
    }
    const double ri = inv_sqrt64(sep2_rn(xa, ya, za));
    const double s = -b.mstar[g] * (ri * ri) * ri;
    double d[6] = {Z[3 * M + fa], Z[4 * M + fa], Z[5 * M + fa], s * xa + ax, s * ya + ay, s * za + az};
    const double h = b.H[g] / (2 * (k + 1));
    if (mode == 2) {
        double tk[6];
        for (int q = 0; q < 6; ++q) tk[q] = 0.5 * (ZM[q * M + fa] + Z[q * M + fa] + h * d[q]);
        if (lead) {
            double *T0 = b.tcol + (size_t)k * 6 * M;
            for (int q = 0; q < 6; ++q) T0[q * M + fa] = tk[q];
        }
        if (k == 0) return;
        double dp = 0.0, dvv = 0.0;
        bool bad = false;
        if (lead) {
            for (int q = 0; q < 6; ++q) {
                const double tz = b.tcol[q * M + fa];
                double sum = 0.0;
                for (int jj = 1; jj <= k; ++jj) {
                    const double v = jj == k ? tk[q] : b.tcol[((size_t)jj * 6 + q) * M + fa];
                    sum = fma(LAGRANGE.d[k][jj], v - tz, sum);
                }
                if (q < 3) dp = fmax(dp, fabs(sum));
                else dvv = fmax(dvv, fabs(sum));
                bad |= !(sum == sum);
            }
        }
        const double e = fmax(dp / bitsd(b.sr[g]), dvv / bitsd(b.sv[g]));
        wave_atomic_max(b.err + k, g * BS_KMAX, lead, (bad || !(e == e)) ? ~0ull : dbits(e));
        return;
    }
    if (lead) {
        double o[6];
        for (int q = 0; q < 6; ++q) {
            o[q] = (mode == 0 ? Z[q * M + fa] : ZM[q * M + fa]) + (mode == 0 ? h : 2.0 * h) * d[q];
            OUT[q * M + fa] = o[q];
        }
        reinterpret_cast<double4 *>(ROUT + (size_t)fa * 8)[0] = make_double4(o[0], o[1], o[2], b.mass[fa]);
    }
}

// One sub-step on the list path (modes and outputs as substep_tile; jstep: Z is the state at
// tau = jstep * H / (2 (k + 1))), one workgroup per target tile: the records of the tile's
// slots (the sources of RZ, Z's records) are staged in LDS, then BIG_LIST_LANES lanes share a
// member, each summing every BIG_LIST_LANES-th entry of its list in order, and the parts are
// added in a fixed tree.  48 bytes per staged source and at most 80 VGPRs: three workgroups
// fit a CU.
template <bool LV>
__global__ __launch_bounds__(64 * BIG_LIST_LANES) __attribute__((amdgpu_waves_per_eu(6))) void big_substep_list_kernel(BigBs b, int k, int mode, int jstep,
                                                                               const double *Z, const double *ZM,
                                                                               double *OUT, const double *RZ,
                                                                               double *ROUT)
{
    constexpr int P = BIG_LIST_LANES;
    constexpr int NS = BIG_LIST_SLOTS * 64;
    __shared__ double2 sxy[NS], szm[NS], sri[NS]; // (x, y), (z, mass), (r_crit, signed 1 / (0.9 r_crit))
    __shared__ int sgi[LV ? NS : 1];               // member index, for the levels' radii
    constexpr int PER = NS / (64 * P); // staged sources per thread
    static_assert(NS % (64 * P) == 0, "whole rounds of staging");
    const size_t M = (size_t)b.dims[1];
    // one target tile per workgroup (the grid covers the largest layout)
    const int me = blockIdx.x;
    if (me >= b.dims[2]) return;
    // first round of loads: the tile, its slots
    const int4 tile = b.tiles[me];
    const int ns = b.nslot[me];
    int2 si[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) si[u] = b.slot[me * BIG_LIST_SLOTS + ((int)threadIdx.x + u * 64 * P) / 64];
    const int g = tile.x;
    const int m = (int)threadIdx.x / P, part = (int)threadIdx.x % P;
    const bool act = m < tile.z;
    const int fa = tile.y + (act ? m : 0);
    // second round: the group's state, the sources to stage and the member's own words
    if (b.done[g] || b.acc[g] >= 0) return; // the whole workgroup
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = (int)threadIdx.x + u * 64 * P;
        if (i < ns * 64 && (i & 63) < si[u].y) {
            const size_t j = (size_t)(si[u].x + (i & 63));
            const double4 p = reinterpret_cast<const double4 *>(RZ + j * 8)[0];
            sxy[i] = make_double2(p.x, p.y);
            szm[i] = make_double2(p.z, p.w);
            sri[i] = reinterpret_cast<const double2 *>(RZ + j * 8)[2];
            if constexpr (LV) sgi[i] = (int)j;
        }
    }
    const double xa = Z[fa], ya = Z[M + fa], za = Z[2 * M + fa];
    const double2 ca = reinterpret_cast<const double2 *>(RZ + (size_t)fa * 8)[2];
    const int tot = b.ltot[fa];
    const uint16_t *L = b.ll + (size_t)fa * BIG_LIST_CAP;
    int l0 = L[part], l1 = L[part + P]; // the first two positions (used only below tot)
    __syncthreads();
    {
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (act) {
            // the bound of the lists: every member stays within S of its prediction
            if (part == 0 && jstep > 0) {
                const double H = b.H[g], hs = H / (2 * (k + 1)), tau = hs * jstep;
                const double4 pm = b.pred[fa];
                const double h2 = 0.5 * (tau * tau - ((jstep & 1) ? hs * hs : 0.0));
                const double px = fma(pm.x, h2, fma(b.Y[3 * M + fa], tau, b.Y[fa]));
                const double py = fma(pm.y, h2, fma(b.Y[4 * M + fa], tau, b.Y[M + fa]));
                const double pz = fma(pm.z, h2, fma(b.Y[5 * M + fa], tau, b.Y[2 * M + fa]));
                if (!(sep2_rn(xa - px, ya - py, za - pz) <= pm.w * pm.w * (1.0 - 0x1p-30))) {
                    b.stale[g] = 1;
                    b.crossed[fa] = 1;
                }
            }
            const double rca = ca.x, i09a = fabs(ca.y);
            const bool testa = signbit(ca.y);
            const auto term = [&](int l) {
                const double2 xy = sxy[l], zm = szm[l], cj = sri[l];
                const double dx = xy.x - xa, dy = xy.y - ya, dz = zm.x - za;
                const bool own = rca >= cj.x;
                const double rcab = own ? rca : cj.x;
                const double q = sep2_rn(dx, dy, dz);
                const double rq = inv_sqrt64(q);
                const double yv = (q * rq - 0.1 * rcab) * (own ? i09a : fabs(cj.y));
                const double y2 = yv * yv;
                const double kv = yv <= 0.0 ? 0.0 : (yv >= 1.0 ? 1.0 : y2 / (2.0 * y2 - 2.0 * yv + 1.0));
                double w = 1.0 - kv, rdeep = rcab;
                if constexpr (LV) {
                    const int j = sgi[l];
                    for (int lv = 1; lv < b.nlev; ++lv) {
                        const double rcl_ab = fmax(b.rcl[(size_t)(lv - 1) * b.cap_M + fa],
                                                   b.rcl[(size_t)(lv - 1) * b.cap_M + j]);
                        w *= 1.0 - changeover_k((q * rq - 0.1 * rcl_ab) / (0.9 * rcl_ab));
                        rdeep = rcl_ab;
                    }
                }
                // the lists hold no member itself
                const bool in = !(testa && signbit(cj.y)) && q < sq_rn(rdeep);
                const double s = in ? zm.y * w * (rq * rq) * rq : 0.0;
                ax = fma(s, dx, ax);
                ay = fma(s, dy, ay);
                az = fma(s, dz, az);
            };
            // lane `part` sums every P-th entry from `part` on, in order; the positions of the
            // next two are loaded ahead (past the end: entry 0, unused)
            const auto entry = [&](int e) { return (int)L[e < tot ? e : 0]; };
            for (int e = part; e < tot; e += P) {
                const int l = l0;
                l0 = l1;
                l1 = entry(e + 2 * P);
                term(l);
            }
        }
        // the parts of a member, in a fixed order
        for (int off = P / 2; off > 0; off >>= 1) {
            ax += __shfl_xor(ax, off, 64);
            ay += __shfl_xor(ay, off, 64);
            az += __shfl_xor(az, off, 64);
        }
        member_tail(b, k, mode, g, fa, act, act && part == 0, xa, ya, za, ax, ay, az, Z, ZM, OUT, ROUT);
    }
}

// The first sub-step of column k >= 1 on the list path: the pair sums at Y are column 0's
// (a0), so only the update runs, one thread per member; it also takes column k - 1's verdict.
__global__ __launch_bounds__(GB_THREADS) void big_substep_start_kernel(BigBs b, int k, double tol, double *OUT,
                                                                      double *ROUT)
{
    const int f = blockIdx.x * GB_THREADS + threadIdx.x;
    const bool valid = f < b.dims[1];
    const int fa = valid ? f : 0;
    const int g = b.grp[fa];
    const int ka = decided(b, g, k - 1, tol); // column k - 1's verdict
    if (valid && fa == b.off[g] && ka != b.acc[g]) b.acc[g] = ka;
    const bool act = valid && !b.done[g] && ka < 0;
    const size_t M = (size_t)b.dims[1];
    const double *Y = b.Y;
    member_tail(b, k, 0, g, fa, act, act, Y[fa], Y[M + fa], Y[2 * M + fa], act ? b.a0[fa] : 0.0,
                act ? b.a0[M + fa] : 0.0, act ? b.a0[2 * M + fa] : 0.0, Y, Y, OUT, ROUT);
}

__global__ __launch_bounds__(64) void big_decide_kernel(BigBs b, int k, double tol)
{
    const int g = blockIdx.x * 64 + threadIdx.x;
    if (g >= b.dims[0] || b.done[g] || b.acc[g] >= 0) return;
    if (b.skin && b.stale[g]) return; // a sub-step left the list's bound: no column counts
    const unsigned long long e = b.err[g * BS_KMAX + k];
    if (e != ~0ull && bitsd(e) <= tol) b.acc[g] = k;
}

// Accepted groups: Y = T(k*, k*) (the last column's verdict taken here).
__global__ __launch_bounds__(GB_THREADS) void big_accept_kernel(BigBs b, double tol)
{
    const int f = blockIdx.x * GB_THREADS + threadIdx.x;
    if (f >= b.dims[1]) return;
    const int g = b.grp[f];
    const int ks = decided(b, g, BS_KMAX - 1, tol);
    if (f == b.off[g] && ks != b.acc[g]) b.acc[g] = ks;
    if (b.done[g] || ks < 0) return;
    const size_t M = (size_t)b.dims[1];
    for (int q = 0; q < 6; ++q) {
        const double t0 = b.tcol[q * M + f];
        double s = 0.0;
        for (int jj = 1; jj <= ks; ++jj) s = fma(LAGRANGE.w[ks][jj], b.tcol[((size_t)jj * 6 + q) * M + f] - t0, s);
        b.Y[q * M + f] = t0 + s;
    }
}

// Step control per group, and the number of groups still short of dt.
__global__ __launch_bounds__(GB_THREADS) void big_control_kernel(BigBs b, double tol,
                                                                 int32_t *flags)
{
    __shared__ int cnt[GB_THREADS / 64];
    const double dt = b.dtp[0];
    int active = 0;
    for (int g = threadIdx.x; g < b.dims[0]; g += GB_THREADS) {
        if (b.done[g]) continue;
        if (b.skin && b.stale[g]) { // a void attempt: the same step again (with wider lists)
            b.keep[g] = 0;
            ++active;
            continue;
        }
        const int ks = decided(b, g, BS_KMAX - 1, tol);
        // a rejected attempt leaves Y and the skins as they were and only shortens the step: the
        // next attempt keeps its lists (the prediction and its bound hold over any shorter step)
        if (b.skin) b.keep[g] = ks < 0;
        if (ks >= 0) {
            const double t = b.last[g] ? dt : b.t[g] + b.H[g];
            b.t[g] = t;
            if (ks <= 4) b.H[g] = 2.0 * b.H[g];
            else if (ks == BS_KMAX - 1) b.H[g] = 0.5 * b.H[g];
            if (!(t < dt)) b.done[g] = 1;
        } else {
            const unsigned long long e = b.err[g * BS_KMAX + BS_KMAX - 1];
            if (e == ~0ull) { // non-finite estimate: give up on this group
                atomicOr(flags, FLAG_NOCONVERGE);
                b.done[g] = 1;
            } else {
                b.H[g] = b.H[g] * shrink_factor(bitsd(e), tol);
            }
        }
        active += !b.done[g];
    }
    for (int s = 32; s > 0; s >>= 1) active += __shfl_xor(active, s, 64);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = active;
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
        for (int w = 0; w < GB_THREADS / 64; ++w) total += cnt[w];
        *b.n_active = total;
    }
}

__global__ __launch_bounds__(GB_THREADS) void big_finish_kernel(BigBs b, double *x, double *y, double *z,
                                                                double *vx, double *vy, double *vz)
{
    const int f = blockIdx.x * GB_THREADS + threadIdx.x;
    if (f >= b.dims[1]) return;
    const size_t M = (size_t)b.dims[1];
    const int body = b.body[f];
    x[body] = b.Y[f];
    y[body] = b.Y[M + f];
    z[body] = b.Y[2 * M + f];
    vx[body] = b.Y[3 * M + f];
    vy[body] = b.Y[4 * M + f];
    vz[body] = b.Y[5 * M + f];
}

} // namespace

hipError_t launch_big_setup(const Layout &L, const BigBs &b, const int32_t *members, const double *x,
                            const double *y, const double *z, const double *vx, const double *vy,
                            const double *vz, const double *m, const double *rc, const double *rc_lv,
                            double dt, hipStream_t stream)
{
    if (b.G == 0) return hipSuccess;
    big_setup_groups_kernel<<<(b.G + 63) / 64, 64, 0, stream>>>(b, L.sys_of, L.mstar, members, dt);
    big_setup_kernel<<<b.n_tiles, 64, 0, stream>>>(b, L.sys_of, L.sys_off, L.n_massive, x, y, z, vx, vy, vz, m, rc,
                                                   rc_lv, L.n_total);
    return hipGetLastError();
}

hipError_t launch_big_attempt(const BigBs &b, double tol, int32_t *flags, int tile_grid, int waves,
                              hipStream_t stream)
{
    // grids for the largest layout: launches past the current one (sizes in b.dims) return at
    // once, so one captured sequence serves every step
    const int gg = (b.cap_G + 63) / 64, gm = (b.cap_M + GB_THREADS - 1) / GB_THREADS;
    const int nt = std::max(1, std::min(tile_grid, b.cap_T));
    const size_t M6 = 6 * (size_t)b.cap_M;
    double *buf[3] = {b.Y, b.Y + M6, b.Y + 2 * M6};           // Y, B1, B2
    double *box[3] = {b.bb, b.bb + 8 * (size_t)b.cap_T, b.bb + 16 * (size_t)b.cap_T};
    // waves per target tile: 16 while the tiles fit the chip in one round of workgroups, fewer
    // (more workgroups per CU, more sources per wave) for larger layouts
    if (waves != 8 && waves != 16) return hipErrorInvalidValue;
    const bool lv = b.nlev > 1;
    auto substep = waves == 16 ? (lv ? big_substep_kernel<true, 16> : big_substep_kernel<false, 16>)
                               : (lv ? big_substep_kernel<true, 8> : big_substep_kernel<false, 8>);
    big_begin_kernel<<<gg, 64, 0, stream>>>(b, flags);
    big_scale_kernel<<<gm, GB_THREADS, 0, stream>>>(b);
    big_box_kernel<<<nt, 64, 0, stream>>>(b);
    for (int k = 0; k < BS_KMAX; ++k) {
        const int nsub = 2 * (k + 1);
        // sub-step i reads zc_i and zm_i and writes zc_(i+1): zc_1 = B1 (zm_1 = Y), then the
        // new point goes into zm's buffer, B2 first
        substep<<<nt, GB_TILE * waves, 0, stream>>>(b, k, 0, buf[0], buf[0], buf[1], box[0], box[1]);
        int zc = 1, zm = 0;
        for (int i = 1; i < nsub; ++i) {
            const int out = zm == 0 ? 2 : zm;
            substep<<<nt, GB_TILE * waves, 0, stream>>>(b, k, 1, buf[zc], buf[zm], buf[out], box[zc],
                                                                       box[out]);
            zm = zc;
            zc = out;
        }
        substep<<<nt, GB_TILE * waves, 0, stream>>>(b, k, 2, buf[zc], buf[zm], nullptr, box[zc], nullptr);
        if (k > 0) big_decide_kernel<<<gg, 64, 0, stream>>>(b, k, tol); // the estimates came with T(k, 0)
    }
    big_accept_kernel<<<gm, GB_THREADS, 0, stream>>>(b, tol);
    big_control_kernel<<<1, GB_THREADS, 0, stream>>>(b, tol, flags);
    return hipGetLastError();
}

hipError_t launch_big_attempt_list(const BigBs &b, double tol, int32_t *flags, int tile_grid, hipStream_t stream)
{
    const int gg = (b.cap_G + 63) / 64, gm = (b.cap_M + GB_THREADS - 1) / GB_THREADS;
    const int nt = std::max(1, std::min(tile_grid, b.cap_T));
    const size_t M6 = 6 * (size_t)b.cap_M;
    double *buf[3] = {b.Y, b.Y + M6, b.Y + 2 * M6}; // Y, B1, B2
    double *rec[3] = {b.rec, b.rec + 8 * (size_t)b.cap_M, b.rec + 16 * (size_t)b.cap_M};
    const bool lv = b.nlev > 1;
    auto substep = lv ? big_substep_list_kernel<true> : big_substep_list_kernel<false>;
    big_begin_kernel<<<gg, 64, 0, stream>>>(b, flags);
    big_scale_kernel<<<gm, GB_THREADS, 0, stream>>>(b);
    big_src_kernel<<<gm, GB_THREADS, 0, stream>>>(b);
    big_sweep_kernel<<<nt, 64, 0, stream>>>(b);
    const int nl = std::min(nt * BIG_LIST_SEGS, 65536);
    if (lv)
        big_list_kernel<true><<<nl, 64, 0, stream>>>(b);
    else
        big_list_kernel<false><<<nl, 64, 0, stream>>>(b);
    big_localize_kernel<<<nt, LOC_THREADS, 0, stream>>>(b);
    for (int k = 0; k < BS_KMAX; ++k) {
        const int nsub = 2 * (k + 1);
        if (k == 0)
            substep<<<nt, 64 * BIG_LIST_LANES, 0, stream>>>(b, k, 0, 0, buf[0], buf[0], buf[1], rec[0], rec[1]);
        else
            big_substep_start_kernel<<<gm, GB_THREADS, 0, stream>>>(b, k, tol, buf[1], rec[1]);
        int zc = 1, zm = 0;
        for (int i = 1; i < nsub; ++i) {
            const int out = zm == 0 ? 2 : zm;
            substep<<<nt, 64 * BIG_LIST_LANES, 0, stream>>>(b, k, 1, i, buf[zc], buf[zm], buf[out], rec[zc], rec[out]);
            zm = zc;
            zc = out;
        }
        substep<<<nt, 64 * BIG_LIST_LANES, 0, stream>>>(b, k, 2, nsub, buf[zc], buf[zm], nullptr, rec[zc], nullptr);
    }
    big_accept_kernel<<<gm, GB_THREADS, 0, stream>>>(b, tol);
    big_control_kernel<<<1, GB_THREADS, 0, stream>>>(b, tol, flags);
    return hipGetLastError();
}

hipError_t launch_big_finish(const BigBs &b, double *x, double *y, double *z, double *vx, double *vy,
                             double *vz, hipStream_t stream)
{
    if (b.G == 0) return hipSuccess;
    big_finish_kernel<<<(b.M + GB_THREADS - 1) / GB_THREADS, GB_THREADS, 0, stream>>>(b, x, y, z, vx, vy, vz);
    return hipGetLastError();
}

} // namespace genga
