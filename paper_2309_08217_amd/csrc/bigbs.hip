// Bulirsch-Stoer over dt for encounter groups larger than one wavefront.  In the
// encounter-dominated phase (Sect. 4: many planetesimals form almost one large close-encounter
// group and the run is bound by the Bulirsch-Stoer step) a group can hold most of a disc, so
// its state is spread over the whole GPU.  Method, tolerance and step control are those of
// the one-wave path and the oracle: modified midpoint with n_k = 2(k+1) sub-steps, polynomial
// extrapolation in h^2 (here in Lagrange form, relative to T(0,0)), acceptance at the first
// column k >= 1 whose estimate meets tol on the group's position / velocity scales, next step
// doubled / kept / halved, rejected steps shrunk by shrink_factor.
//
// One attempt is a fixed sequence of launches over all large groups at once: a force
// evaluation and midpoint update per sub-step (64 targets per workgroup, GB_WAVES waves that
// split the group's members as sources), then per column an error launch and a decision
// launch.  A group that has accepted a column, or reached dt, skips the rest.  The host
// repeats attempts until no group is active.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

using CD = const __attribute__((address_space(4))) double;
using CI = const __attribute__((address_space(4))) int32_t;

constexpr int GB_TILE = 64;
constexpr int GB_WAVES = 8;
constexpr int GB_THREADS = 256;

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

// Flat member m of large group g: body index, constants, state Y[q * M + m].
__global__ __launch_bounds__(GB_THREADS) void big_setup_kernel(BigBs b, const int32_t *sys_of,
                                                               const int32_t *sys_off,
                                                               const int32_t *n_massive,
                                                               const double *mstar,
                                                               const int32_t *members,
                                                               const double *x, const double *y,
                                                               const double *z, const double *vx,
                                                               const double *vy, const double *vz,
                                                               const double *m, const double *rc,
                                                               double dt)
{
    __shared__ double red[GB_THREADS / 64];
    const int g = blockIdx.x;
    const int o = b.off[g], nb = b.off[g + 1] - o, k0 = b.k0[g];
    const size_t M = (size_t)b.M;
    double mx = 0.0;
    for (int l = threadIdx.x; l < nb; l += GB_THREADS) {
        const int body = members[k0 + l], f = o + l, s = sys_of[body];
        b.body[f] = body;
        b.grp[f] = g;
        b.rc[f] = rc[body];
        b.mass[f] = m[body];
        b.test[f] = body - sys_off[s] >= n_massive[s];
        b.Y[0 * M + f] = x[body];
        b.Y[1 * M + f] = y[body];
        b.Y[2 * M + f] = z[body];
        b.Y[3 * M + f] = vx[body];
        b.Y[4 * M + f] = vy[body];
        b.Y[5 * M + f] = vz[body];
        mx = fmax(mx, sq_rn(rc[body]));
    }
    for (int s = 32; s > 0; s >>= 1) mx = fmax(mx, __shfl_xor(mx, s, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < GB_THREADS / 64; ++w) mx = fmax(mx, red[w]);
        b.rcmax2[g] = mx;
        b.mstar[g] = mstar[sys_of[members[k0]]];
        b.t[g] = 0.0;
        b.H[g] = dt;
        b.attempts[g] = 0;
        b.done[g] = 0;
    }
}

// Start of an attempt, per group.
__global__ __launch_bounds__(64) void big_begin_kernel(BigBs b, double dt, int32_t *flags)
{
    const int g = blockIdx.x * 64 + threadIdx.x;
    if (g >= b.G || b.done[g]) return;
    double H = b.H[g];
    const double t = b.t[g];
    const bool last = H >= (dt - t) * (1.0 - 0x1p-30); // ends the interval (exactly)
    if (last) H = dt - t;
    const int att = b.attempts[g] + 1;
    b.attempts[g] = att;
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
    const int f = blockIdx.x * GB_THREADS + threadIdx.x;
    if (f >= b.M) return;
    const int g = b.grp[f];
    if (b.done[g]) return;
    const size_t M = (size_t)b.M;
    const double *Y = b.Y;
    const double rr = sqrt(sep2_rn(Y[f], Y[M + f], Y[2 * M + f]));
    const double vv = sqrt(sep2_rn(Y[3 * M + f], Y[4 * M + f], Y[5 * M + f]));
    atomicMax(&b.sr[g], dbits(rr));
    atomicMax(&b.sv[g], dbits(vv));
}

// One sub-step of column k for every target of a tile: f(Z) (Kepler term plus the (1 - K)
// share of the Newtonian forces from the group's other members), then
//   mode 0: OUT = Z + h f(Z)            (first sub-step, Z = Y)
//   mode 1: OUT = ZM + 2 h f(Z)         (OUT may be ZM's buffer: each lane rewrites its own)
//   mode 2: T(k, 0) = (ZM + Z + h f(Z)) / 2, into tcol[k]
// Source positions come through scalar loads: Z is not written by this launch.
__global__ __launch_bounds__(GB_TILE *GB_WAVES) void big_substep_kernel(BigBs b, int k, int mode,
                                                                       const double *Z,
                                                                       const double *ZM, double *OUT)
{
    __shared__ double red[3][GB_WAVES][GB_TILE];
    const int4 tile = b.tiles[blockIdx.x]; // (group, first member, count, -)
    const int g = tile.x;
    if (b.done[g] || b.acc[g] >= 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const size_t M = (size_t)b.M;
    const int o = b.off[g], nb = b.off[g + 1] - o;
    const bool valid = lane < tile.z;
    const int fa = tile.y + (valid ? lane : 0);
    const double xa = Z[fa], ya = Z[M + fa], za = Z[2 * M + fa];
    const double rca = b.rc[fa];
    const bool testa = b.test[fa] != 0;
    // candidate radius: the group's largest r_crit^2, with a margin for the contracted r^2
    const double T = b.rcmax2[g] * (1.0 + 0x1p-40);
    CD *ZX = (CD *)Z;
    CD *ZY = (CD *)(Z + M);
    CD *ZZ = (CD *)(Z + 2 * M);
    CD *RC = (CD *)b.rc;
    CD *MS = (CD *)b.mass;
    CI *TS = (CI *)b.test;
    const int chunk = (nb + GB_WAVES - 1) / GB_WAVES;
    const int jb = o + min(wave * chunk, nb), je = o + min(wave * chunk + chunk, nb);
    double ax = 0.0, ay = 0.0, az = 0.0;
    auto pair = [&](int j, double dx, double dy, double dz) {
        if (j == fa) return;
        if (testa && TS[j]) return;
        const double q = sep2_rn(dx, dy, dz);
        const double rcab = fmax(rca, RC[j]);
        if (!(q < sq_rn(rcab))) return;
        const double rq = inv_sqrt64(q);
        const double w = 1.0 - changeover_k((q * rq - 0.1 * rcab) / (0.9 * rcab));
        const double t = MS[j] * w * (rq * rq) * rq;
        ax = fma(t, dx, ax);
        ay = fma(t, dy, ay);
        az = fma(t, dz, az);
    };
    int j = jb;
    for (; j + 4 <= je; j += 4) {
        const double dx0 = ZX[j] - xa, dy0 = ZY[j] - ya, dz0 = ZZ[j] - za;
        const double dx1 = ZX[j + 1] - xa, dy1 = ZY[j + 1] - ya, dz1 = ZZ[j + 1] - za;
        const double dx2 = ZX[j + 2] - xa, dy2 = ZY[j + 2] - ya, dz2 = ZZ[j + 2] - za;
        const double dx3 = ZX[j + 3] - xa, dy3 = ZY[j + 3] - ya, dz3 = ZZ[j + 3] - za;
        const double q0 = fma(dx0, dx0, fma(dy0, dy0, dz0 * dz0));
        const double q1 = fma(dx1, dx1, fma(dy1, dy1, dz1 * dz1));
        const double q2 = fma(dx2, dx2, fma(dy2, dy2, dz2 * dz2));
        const double q3 = fma(dx3, dx3, fma(dy3, dy3, dz3 * dz3));
        if (__builtin_expect(fmin(fmin(q0, q1), fmin(q2, q3)) < T, 0)) {
            if (q0 < T) pair(j, dx0, dy0, dz0);
            if (q1 < T) pair(j + 1, dx1, dy1, dz1);
            if (q2 < T) pair(j + 2, dx2, dy2, dz2);
            if (q3 < T) pair(j + 3, dx3, dy3, dz3);
        }
    }
    for (; j < je; ++j) pair(j, ZX[j] - xa, ZY[j] - ya, ZZ[j] - za);
    red[0][wave][lane] = ax;
    red[1][wave][lane] = ay;
    red[2][wave][lane] = az;
    __syncthreads();
    if (wave != 0 || !valid) return;
    const double ri = inv_sqrt64(sep2_rn(xa, ya, za));
    const double s = -b.mstar[g] * (ri * ri) * ri;
    double d[6] = {Z[3 * M + fa], Z[4 * M + fa], Z[5 * M + fa], s * xa, s * ya, s * za};
    for (int w = 0; w < GB_WAVES; ++w) {
        d[3] += red[0][w][lane];
        d[4] += red[1][w][lane];
        d[5] += red[2][w][lane];
    }
    const double h = b.H[g] / (2 * (k + 1));
    if (mode == 0) {
        for (int q = 0; q < 6; ++q) OUT[q * M + fa] = Z[q * M + fa] + h * d[q];
    } else if (mode == 1) {
        for (int q = 0; q < 6; ++q) OUT[q * M + fa] = ZM[q * M + fa] + 2.0 * h * d[q];
    } else {
        double *T0 = b.tcol + (size_t)k * 6 * M;
        for (int q = 0; q < 6; ++q) T0[q * M + fa] = 0.5 * (ZM[q * M + fa] + Z[q * M + fa] + h * d[q]);
    }
}

// Error estimate of column k: per member max(|T(k,k) - T(k,k-1)| / scale) over its six
// elements, into the group's maximum.
__global__ __launch_bounds__(GB_THREADS) void big_err_kernel(BigBs b, int k)
{
    const int f = blockIdx.x * GB_THREADS + threadIdx.x;
    if (f >= b.M) return;
    const int g = b.grp[f];
    if (b.done[g] || b.acc[g] >= 0) return;
    const size_t M = (size_t)b.M;
    double dp = 0.0, dv = 0.0;
    bool bad = false;
    for (int q = 0; q < 6; ++q) {
        const double t0 = b.tcol[q * M + f];
        double s = 0.0;
        for (int jj = 1; jj <= k; ++jj) s = fma(LAGRANGE.d[k][jj], b.tcol[((size_t)jj * 6 + q) * M + f] - t0, s);
        if (q < 3) dp = fmax(dp, fabs(s));
        else dv = fmax(dv, fabs(s));
        bad |= !(s == s);
    }
    const double e = fmax(dp / bitsd(b.sr[g]), dv / bitsd(b.sv[g]));
    // a non-finite estimate is kept as the all-ones pattern, above every finite one
    atomicMax(&b.err[g * BS_KMAX + k], (bad || !(e == e)) ? ~0ull : dbits(e));
}

__global__ __launch_bounds__(64) void big_decide_kernel(BigBs b, int k, double tol)
{
    const int g = blockIdx.x * 64 + threadIdx.x;
    if (g >= b.G || b.done[g] || b.acc[g] >= 0) return;
    const unsigned long long e = b.err[g * BS_KMAX + k];
    if (e != ~0ull && bitsd(e) <= tol) b.acc[g] = k;
}

// Accepted groups: Y = T(k*, k*).
__global__ __launch_bounds__(GB_THREADS) void big_accept_kernel(BigBs b)
{
    const int f = blockIdx.x * GB_THREADS + threadIdx.x;
    if (f >= b.M) return;
    const int g = b.grp[f];
    const int ks = b.acc[g];
    if (b.done[g] || ks < 0) return;
    const size_t M = (size_t)b.M;
    for (int q = 0; q < 6; ++q) {
        const double t0 = b.tcol[q * M + f];
        double s = 0.0;
        for (int jj = 1; jj <= ks; ++jj) s = fma(LAGRANGE.w[ks][jj], b.tcol[((size_t)jj * 6 + q) * M + f] - t0, s);
        b.Y[q * M + f] = t0 + s;
    }
}

// Step control per group, and the number of groups still short of dt.
__global__ __launch_bounds__(GB_THREADS) void big_control_kernel(BigBs b, double dt, double tol,
                                                                 int32_t *flags)
{
    __shared__ int cnt[GB_THREADS / 64];
    int active = 0;
    for (int g = threadIdx.x; g < b.G; g += GB_THREADS) {
        if (b.done[g]) continue;
        const int ks = b.acc[g];
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
    if (f >= b.M) return;
    const size_t M = (size_t)b.M;
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
                            const double *vz, const double *m, const double *rc, double dt,
                            hipStream_t stream)
{
    if (b.G == 0) return hipSuccess;
    big_setup_kernel<<<b.G, GB_THREADS, 0, stream>>>(b, L.sys_of, L.sys_off, L.n_massive, L.mstar, members, x, y,
                                                     z, vx, vy, vz, m, rc, dt);
    return hipGetLastError();
}

hipError_t launch_big_attempt(const BigBs &b, double dt, double tol, int32_t *flags, hipStream_t stream)
{
    if (b.G == 0) return hipSuccess;
    const int gg = (b.G + 63) / 64, gm = (b.M + GB_THREADS - 1) / GB_THREADS;
    const size_t M6 = 6 * (size_t)b.M;
    double *Y = b.Y, *B1 = b.Y + M6, *B2 = b.Y + 2 * M6;
    big_begin_kernel<<<gg, 64, 0, stream>>>(b, dt, flags);
    big_scale_kernel<<<gm, GB_THREADS, 0, stream>>>(b);
    for (int k = 0; k < BS_KMAX; ++k) {
        const int nsub = 2 * (k + 1);
        // sub-step i reads zc_i and zm_i and writes zc_(i+1): zc_1 = B1 (zm_1 = Y), then the
        // new point goes into zm's buffer, B2 first
        big_substep_kernel<<<b.n_tiles, GB_TILE * GB_WAVES, 0, stream>>>(b, k, 0, Y, Y, B1);
        const double *zc = B1, *zm = Y;
        double *spare = B2;
        for (int i = 1; i < nsub; ++i) {
            double *out = zm == Y ? spare : const_cast<double *>(zm);
            big_substep_kernel<<<b.n_tiles, GB_TILE * GB_WAVES, 0, stream>>>(b, k, 1, zc, zm, out);
            zm = zc;
            zc = out;
        }
        big_substep_kernel<<<b.n_tiles, GB_TILE * GB_WAVES, 0, stream>>>(b, k, 2, zc, zm, nullptr);
        if (k > 0) {
            big_err_kernel<<<gm, GB_THREADS, 0, stream>>>(b, k);
            big_decide_kernel<<<gg, 64, 0, stream>>>(b, k, tol);
        }
    }
    big_accept_kernel<<<gm, GB_THREADS, 0, stream>>>(b);
    big_control_kernel<<<1, GB_THREADS, 0, stream>>>(b, dt, tol, flags);
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
