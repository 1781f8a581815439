// Long-range kick of the hybrid symplectic step (Brasser et al. 2023, Sect. 1): direct
// O(N^2) summation of Newtonian pair accelerations weighted by the changeover function,
// in FP32 pair arithmetic (coordinate differences formed in FP64) or in FP64, with the
// close-encounter pairs recorded by the same launch.  gfx950, wave64.
//
// Design (vector-ALU bound; no MFMA: a pair force is not a dense contraction):
//  * one workgroup = up to 64 target bodies i (one per lane, FP64 position in VGPRs) and
//    W waves; wave w visits a contiguous slice of the system's sources j, so a launch over
//    N/64 workgroups still fills the chip.  Partial sums of the W waves are added in LDS in
//    a fixed order, so results are deterministic.
//  * sources are read as 32-byte records through the scalar data path: the j index is
//    wave-uniform, so every lane's pair arithmetic takes x_j, y_j, z_j, m_j from SGPRs and
//    no LDS traffic or barrier is needed in the inner loop.
//  * four sources per step; the changeover test is a single compare against the system's
//    largest r_crit^2 per pair, and only a group of four that has a candidate takes the
//    slow path, which decides "inside r_crit,ij" in FP64 exactly as the definition states,
//    evaluates K and the pair term in FP64 and appends (i, j) to the encounter list.
//  * FP32 path: FP32 partial sums over blocks of 64 sources, folded into FP64 accumulators
//    or into Kahan-compensated FP32 sums.  FP64 path: r^-3 from v_rsq_f64 (about 2^-24) and a
//    second-order series correction of its cube.
//  * the same FP64 loop without the force terms lists the encounter pairs of a state on its
//    own (no kick has run on it).
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

using CJ32 = const __attribute__((address_space(4))) JRec32;
using CJ64 = const __attribute__((address_space(4))) JRec64;

// Source records are read through the constant address space: the index is wave-uniform, so
// the loads become scalar loads into SGPRs.
__device__ __forceinline__ JRec32 ldj(CJ32 *J, int j)
{
    JRec32 r;
    r.x = J[j].x;
    r.y = J[j].y;
    r.z = J[j].z;
    r.m = J[j].m;
    r.pad = 0.f;
    return r;
}

__device__ __forceinline__ JRec64 ldj(CJ64 *J, int j)
{
    JRec64 r;
    r.x = J[j].x;
    r.y = J[j].y;
    r.z = J[j].z;
    r.m = J[j].m;
    return r;
}

// Encounter pairs found by a wave collect in its own LDS buffer and reach the global list in
// blocks, one counter update per block, so that a dense list does not serialise on the
// counter.  The calls come from divergent code: only the wave's active lanes take part, and
// the fill count lives in LDS so that it stays one value for the whole wave.
constexpr int PAIR_BUF = 128;

struct PairBuf {
    int2 *buf;  // the wave's PAIR_BUF slots
    int *n;     // the wave's fill count
};

// orders the LDS accesses of the lanes of one wave
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void store_pair(const KickArgs &a, int idx, int2 p)
{
    if (idx < a.pair_cap) {
        a.pairs[2 * idx] = p.x;
        a.pairs[2 * idx + 1] = p.y;
    } else {
        atomicOr(a.flags, FLAG_CAPACITY);
    }
}

// Move the buffer's n pairs, followed by the pairs (i, j) of the active lanes with em set
// (m = their mask), to the global list; the active lanes share the copying.
__device__ __forceinline__ void spill_pairs(const KickArgs &a, PairBuf pb, int n,
                                            unsigned long long m, bool em, int i, int j)
{
    const unsigned long long act = __ballot(1);
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1;
    const int leader = __ffsll((long long)act) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(a.pair_count, n + __popcll(m));
    base = __shfl(base, leader, 64);
    const int rank = __popcll(act & below), n_act = __popcll(act);
    for (int k = rank; k < n; k += n_act) store_pair(a, base + k, pb.buf[k]);
    if (em) store_pair(a, base + n + __popcll(m & below), make_int2(i, j));
    wave_lds_sync();
    *pb.n = 0;
    wave_lds_sync();
}

// Record (i, j) for the active lanes with em set.
__device__ __forceinline__ void emit_pair(const KickArgs &a, PairBuf pb, bool em, int i, int j)
{
    const unsigned long long m = __ballot(em);
    if (!m) return;
    const int n = *pb.n, c = __popcll(m);
    if (n + c > PAIR_BUF) {
        spill_pairs(a, pb, n, m, em, i, j);
        return;
    }
    if (em) pb.buf[n + __popcll(m & ((1ull << (threadIdx.x & 63)) - 1))] = make_int2(i, j);
    wave_lds_sync();
    *pb.n = n + c;
    wave_lds_sync();
}

// Empty the buffer (every lane of the wave calls this).
__device__ __forceinline__ void flush_pairs(const KickArgs &a, PairBuf pb)
{
    wave_lds_sync();
    const int n = *pb.n;
    if (n > 0) spill_pairs(a, pb, n, 0ull, false, 0, 0);
}

// Pair inside the candidate radius: exact FP64 decision; inside r_crit,ij the weighted
// term is added in FP64 and the pair recorded; returns true when handled here.
__device__ __forceinline__ bool close_pair(const KickArgs &a, double xj, double yj, double zj,
                                           int j, int i, bool valid, double xi, double yi,
                                           double zi, double rci, double &sx, double &sy,
                                           double &sz, PairBuf pb)
{
    if (j == i) return true;
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    double r2 = sep2_rn(dx, dy, dz);
    double rcij = fmax(rci, a.rc[j]);
    if (!(r2 < sq_rn(rcij))) return false;
    double r = sqrt(r2);
    double k = changeover_k((r - 0.1 * rcij) / (0.9 * rcij));
    if (k > 0.0) {
        double s = a.m[j] * k / (r2 * r);
        sx += s * dx;
        sy += s * dy;
        sz += s * dz;
    }
    emit_pair(a, pb, valid && i < j && (!a.status || (a.status[i] == 0 && a.status[j] == 0)), i, j);
    return true;
}

// largest r_crit^2 of system s (wave-uniform loop over its chunks)
__device__ __forceinline__ double system_rc2max(const KickArgs &a, int s)
{
    double mx = 0.0;
    for (int k = a.chunk_first[s]; k < a.chunk_first[s + 1]; ++k) mx = fmax(mx, a.rc2_part[k]);
    return mx;
}

struct Acc32 {
    float fx, fy, fz;
};

// S + v with Kahan compensation: after the call S - C equals the exact sum of the values added
// so far up to the rounding of the last C
__device__ __forceinline__ void kahan_add(float &S, float &C, float v)
{
    const float y = v - C;
    const float t = S + y;
    C = (t - S) - y;
    S = t;
}

__device__ __forceinline__ void far32(float mj, float dx, float dy, float dz, float q, Acc32 &c)
{
    float ri = __builtin_amdgcn_rsqf(q);
    float s = mj * (ri * ri) * ri;
    c.fx = fmaf(s, dx, c.fx);
    c.fy = fmaf(s, dy, c.fy);
    c.fz = fmaf(s, dz, c.fz);
}

__device__ __forceinline__ void far64(double mj, double dx, double dy, double dz, double q,
                                      double &sx, double &sy, double &sz)
{
    const double y0 = __builtin_amdgcn_rsq(q);
    // r^-3 = q^(-3/2) = y0^3 (1 - e)^(-3/2) with e = 1 - q y0^2 (|e| about 2^-23): the
    // series 1 + 3/2 e + 15/8 e^2 leaves a relative error of about 2 e^3, below the rounding
    const double y2 = y0 * y0;
    const double e = fma(-q, y2, 1.0);
    const double w = fma(fma(1.875, e, 1.5), e, 1.0);
    const double s = (mj * w) * (y2 * y0);
    sx = fma(s, dx, sx);
    sy = fma(s, dy, sy);
    sz = fma(s, dz, sz);
}

// Sources visited by part `part` of an item when its source range (the first w.nsrc bodies
// of the system) is split over a.split workgroups.
__device__ __forceinline__ void source_range(const KickArgs &a, const WorkItem &w, int part, int &j0,
                                             int &j1)
{
    const int b = a.sys_off[w.sys], e = b + w.nsrc;
    const int per = (e - b + a.split - 1) / a.split;
    j0 = min(b + part * per, e);
    j1 = min(j0 + per, e);
}

// Sum the W waves' partial accelerations in a fixed order; then either finish the body
// (a_i out, v += tau a_i) or, when the sources are split over workgroups, store this
// workgroup's share for kick_finish_kernel.
template <int W>
__device__ __forceinline__ void finish(const KickArgs &a, double (*red)[W][64], int wave,
                                       int lane, bool valid, int i, int part, double sx,
                                       double sy, double sz)
{
    red[0][wave][lane] = sx;
    red[1][wave][lane] = sy;
    red[2][wave][lane] = sz;
    __syncthreads();
    if (wave == 0) {
        double tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            tx += red[0][w][lane];
            ty += red[1][w][lane];
            tz += red[2][w][lane];
        }
        if (valid) {
            if (a.split > 1) {
                const size_t n = (size_t)a.n_total;
                double *p = a.part + (size_t)part * 3 * n;
                p[i] = tx;
                p[n + i] = ty;
                p[2 * n + i] = tz;
            } else {
                a.ax[i] = tx;
                a.ay[i] = ty;
                a.az[i] = tz;
                if (!(isfinite(tx) && isfinite(ty) && isfinite(tz))) atomicOr(a.flags, FLAG_NONFINITE);
                if (a.update_v) {
                    a.vx[i] += a.tau * tx;
                    a.vy[i] += a.tau * ty;
                    a.vz[i] += a.tau * tz;
                }
            }
        }
    }
    __syncthreads();
}

// Adds the split shares of every body in part order, then as finish() above.
__global__ __launch_bounds__(256) void kick_finish_kernel(KickArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_total) return;
    const size_t n = (size_t)a.n_total;
    double tx = 0.0, ty = 0.0, tz = 0.0;
    for (int p = 0; p < a.split; ++p) {
        const double *q = a.part + (size_t)p * 3 * n;
        tx += q[i];
        ty += q[n + i];
        tz += q[2 * n + i];
    }
    a.ax[i] = tx;
    a.ay[i] = ty;
    a.az[i] = tz;
    if (!(isfinite(tx) && isfinite(ty) && isfinite(tz))) atomicOr(a.flags, FLAG_NONFINITE);
    if (a.update_v) {
        a.vx[i] += a.tau * tx;
        a.vy[i] += a.tau * ty;
        a.vz[i] += a.tau * tz;
    }
}

template <int W, bool KAHAN>
__global__ __launch_bounds__(64 * W) void kick32_kernel(KickArgs a)
{
    __shared__ double red[3][W][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ int2 pair_slots[W][PAIR_BUF];
    __shared__ int pair_fill[W];
    const PairBuf pb{pair_slots[wave], &pair_fill[wave]};
    pair_fill[wave] = 0;
    wave_lds_sync();
    CJ32 *J = (CJ32 *)a.jrec;
    const int n_tasks = a.n_items * a.split;
    for (int task = blockIdx.x; task < n_tasks; task += gridDim.x) {
        const int part = task % a.split;
        const WorkItem w = a.items[task / a.split];
        int j0, j1;
        source_range(a, w, part, j0, j1);
        const bool valid = lane < w.ni;
        const int i = w.i0 + (valid ? lane : 0);
        const double xi = a.x[i], yi = a.y[i], zi = a.z[i], rci = a.rc[i];
        // candidate threshold: the system's largest r_crit^2 with a margin that covers the
        // FP32 rounding of r^2; never zero, so the self pair always takes the exact path
        const float T = (float)(system_rc2max(a, w.sys) * 1.0001) + 1e-30f;
        const int chunk = (j1 - j0 + W - 1) / W;
        const int jb = min(j0 + wave * chunk, j1), je = min(jb + chunk, j1);
        double sx = 0.0, sy = 0.0, sz = 0.0;  // the pairs inside r_crit; with FP64 folding all
        Acc32 c{0.f, 0.f, 0.f};
        Acc32 S{0.f, 0.f, 0.f}, C{0.f, 0.f, 0.f}; // Kahan sums of the blocks (KAHAN only)
        int j = jb;
        while (j < je) {
            const int jend = min(j + 64, je);
            for (; j + 4 <= jend; j += 4) {
                const JRec32 r0 = ldj(J, j), r1 = ldj(J, j + 1), r2 = ldj(J, j + 2), r3 = ldj(J, j + 3);
                float dx0 = (float)(r0.x - xi), dy0 = (float)(r0.y - yi), dz0 = (float)(r0.z - zi);
                float dx1 = (float)(r1.x - xi), dy1 = (float)(r1.y - yi), dz1 = (float)(r1.z - zi);
                float dx2 = (float)(r2.x - xi), dy2 = (float)(r2.y - yi), dz2 = (float)(r2.z - zi);
                float dx3 = (float)(r3.x - xi), dy3 = (float)(r3.y - yi), dz3 = (float)(r3.z - zi);
                float q0 = fmaf(dx0, dx0, fmaf(dy0, dy0, dz0 * dz0));
                float q1 = fmaf(dx1, dx1, fmaf(dy1, dy1, dz1 * dz1));
                float q2 = fmaf(dx2, dx2, fmaf(dy2, dy2, dz2 * dz2));
                float q3 = fmaf(dx3, dx3, fmaf(dy3, dy3, dz3 * dz3));
                const bool near = fminf(fminf(q0, q1), fminf(q2, q3)) < T;
                if (__builtin_expect(near, 0)) {
                    if (!(q0 < T && close_pair(a, r0.x, r0.y, r0.z, j, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)))
                        far32(r0.m, dx0, dy0, dz0, q0, c);
                    if (!(q1 < T && close_pair(a, r1.x, r1.y, r1.z, j + 1, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)))
                        far32(r1.m, dx1, dy1, dz1, q1, c);
                    if (!(q2 < T && close_pair(a, r2.x, r2.y, r2.z, j + 2, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)))
                        far32(r2.m, dx2, dy2, dz2, q2, c);
                    if (!(q3 < T && close_pair(a, r3.x, r3.y, r3.z, j + 3, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)))
                        far32(r3.m, dx3, dy3, dz3, q3, c);
                } else {
                    far32(r0.m, dx0, dy0, dz0, q0, c);
                    far32(r1.m, dx1, dy1, dz1, q1, c);
                    far32(r2.m, dx2, dy2, dz2, q2, c);
                    far32(r3.m, dx3, dy3, dz3, q3, c);
                }
            }
            for (; j < jend; ++j) {
                const JRec32 r0 = ldj(J, j);
                float dx0 = (float)(r0.x - xi), dy0 = (float)(r0.y - yi), dz0 = (float)(r0.z - zi);
                float q0 = fmaf(dx0, dx0, fmaf(dy0, dy0, dz0 * dz0));
                if (!(q0 < T && close_pair(a, r0.x, r0.y, r0.z, j, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)))
                    far32(r0.m, dx0, dy0, dz0, q0, c);
            }
            // fold the block's FP32 partial sums into the accumulators
            if (KAHAN) {
                kahan_add(S.fx, C.fx, c.fx);
                kahan_add(S.fy, C.fy, c.fy);
                kahan_add(S.fz, C.fz, c.fz);
            } else {
                sx += (double)c.fx;
                sy += (double)c.fy;
                sz += (double)c.fz;
            }
            c.fx = c.fy = c.fz = 0.f;
        }
        if (KAHAN) {
            sx += (double)S.fx - (double)C.fx;
            sy += (double)S.fy - (double)C.fy;
            sz += (double)S.fz - (double)C.fz;
        }
        flush_pairs(a, pb);
        finish<W>(a, red, wave, lane, valid, i, part, sx, sy, sz);
    }
}

// LIST: the encounter pairs only (no far terms, nothing written but the list)
template <int W, bool LIST>
__global__ __launch_bounds__(64 * W) void kick64_kernel(KickArgs a)
{
    __shared__ double red[3][W][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ int2 pair_slots[W][PAIR_BUF];
    __shared__ int pair_fill[W];
    const PairBuf pb{pair_slots[wave], &pair_fill[wave]};
    pair_fill[wave] = 0;
    wave_lds_sync();
    CJ64 *J = (CJ64 *)a.jrec;
    const int n_tasks = a.n_items * a.split;
    for (int task = blockIdx.x; task < n_tasks; task += gridDim.x) {
        const int part = task % a.split;
        const WorkItem w = a.items[task / a.split];
        int j0, j1;
        source_range(a, w, part, j0, j1);
        const bool valid = lane < w.ni;
        const int i = w.i0 + (valid ? lane : 0);
        const double xi = a.x[i], yi = a.y[i], zi = a.z[i], rci = a.rc[i];
        // candidate threshold with a relative margin: q below is formed with fused
        // multiply-adds, the exact decision in close_pair without them
        const double T = system_rc2max(a, w.sys) * (1.0 + 1e-12) + 1e-300;
        const int chunk = (j1 - j0 + W - 1) / W;
        const int jb = min(j0 + wave * chunk, j1), je = min(jb + chunk, j1);
        double sx = 0.0, sy = 0.0, sz = 0.0;
        int j = jb;
        for (; j + 4 <= je; j += 4) {
            const JRec64 r0 = ldj(J, j), r1 = ldj(J, j + 1), r2 = ldj(J, j + 2), r3 = ldj(J, j + 3);
            double dx0 = r0.x - xi, dy0 = r0.y - yi, dz0 = r0.z - zi;
            double dx1 = r1.x - xi, dy1 = r1.y - yi, dz1 = r1.z - zi;
            double dx2 = r2.x - xi, dy2 = r2.y - yi, dz2 = r2.z - zi;
            double dx3 = r3.x - xi, dy3 = r3.y - yi, dz3 = r3.z - zi;
            double q0 = fma(dx0, dx0, fma(dy0, dy0, dz0 * dz0));
            double q1 = fma(dx1, dx1, fma(dy1, dy1, dz1 * dz1));
            double q2 = fma(dx2, dx2, fma(dy2, dy2, dz2 * dz2));
            double q3 = fma(dx3, dx3, fma(dy3, dy3, dz3 * dz3));
            const bool near = fmin(fmin(q0, q1), fmin(q2, q3)) < T;
            if (__builtin_expect(near, 0)) {
                if (!(q0 < T && close_pair(a, r0.x, r0.y, r0.z, j, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)) && !LIST)
                    far64(r0.m, dx0, dy0, dz0, q0, sx, sy, sz);
                if (!(q1 < T && close_pair(a, r1.x, r1.y, r1.z, j + 1, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)) && !LIST)
                    far64(r1.m, dx1, dy1, dz1, q1, sx, sy, sz);
                if (!(q2 < T && close_pair(a, r2.x, r2.y, r2.z, j + 2, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)) && !LIST)
                    far64(r2.m, dx2, dy2, dz2, q2, sx, sy, sz);
                if (!(q3 < T && close_pair(a, r3.x, r3.y, r3.z, j + 3, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)) && !LIST)
                    far64(r3.m, dx3, dy3, dz3, q3, sx, sy, sz);
            } else if (!LIST) {
                far64(r0.m, dx0, dy0, dz0, q0, sx, sy, sz);
                far64(r1.m, dx1, dy1, dz1, q1, sx, sy, sz);
                far64(r2.m, dx2, dy2, dz2, q2, sx, sy, sz);
                far64(r3.m, dx3, dy3, dz3, q3, sx, sy, sz);
            }
        }
        for (; j < je; ++j) {
            const JRec64 r0 = ldj(J, j);
            double dx0 = r0.x - xi, dy0 = r0.y - yi, dz0 = r0.z - zi;
            double q0 = fma(dx0, dx0, fma(dy0, dy0, dz0 * dz0));
            if (!(q0 < T && close_pair(a, r0.x, r0.y, r0.z, j, i, valid, xi, yi, zi, rci, sx, sy, sz, pb)) && !LIST)
                far64(r0.m, dx0, dy0, dz0, q0, sx, sy, sz);
        }
        flush_pairs(a, pb);
        if (!LIST) finish<W>(a, red, wave, lane, valid, i, part, sx, sy, sz);
    }
}

// Source records, the largest r_crit^2 of every chunk, and a cleared pair counter.
template <bool F32>
__global__ __launch_bounds__(SYS_P_THREADS) void prep_kernel(const Chunk *chunks, const int32_t *chunk_first,
                                                             const double *mstar, const double *mom_part,
                                                             double shift_tau, double *x, double *y,
                                                             double *z, const double *m,
                                                             const double *rc, void *jrec,
                                                             double *rc2_part, int32_t *pair_count)
{
    const Chunk c = chunks[blockIdx.x];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (shift_tau != 0.0) {
        // the pending half of a Sun drift: x += tau P / Mstar (same arithmetic as sun_shift)
        __shared__ double pred[3][SYS_P_THREADS / 64];
        double P[3];
        system_momentum(chunk_first, mom_part, c.sys, pred, P);
        const double f = shift_tau / mstar[c.sys];
        sx = f * P[0];
        sy = f * P[1];
        sz = f * P[2];
    }
    double mx = 0.0;
    for (int i = c.b + threadIdx.x; i < c.e; i += SYS_P_THREADS) {
        if (shift_tau != 0.0) {
            x[i] += sx;
            y[i] += sy;
            z[i] += sz;
        }
        if (F32) {
            JRec32 r;
            r.x = x[i];
            r.y = y[i];
            r.z = z[i];
            r.m = (float)m[i];
            r.pad = 0.f;
            ((JRec32 *)jrec)[i] = r;
        } else {
            JRec64 r;
            r.x = x[i];
            r.y = y[i];
            r.z = z[i];
            r.m = m[i];
            ((JRec64 *)jrec)[i] = r;
        }
        mx = fmax(mx, rc[i] * rc[i]);
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        rc2_part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        if (blockIdx.x == 0) *pair_count = 0;
    }
}

// eq. (1): r_crit,i = max(n1 R_H,i, n2 dt v_i)
__global__ __launch_bounds__(256) void rcrit_kernel(int n_total, const int32_t *sys_of,
                                                    const double *mstar, const double *x,
                                                    const double *y, const double *z,
                                                    const double *vx, const double *vy,
                                                    const double *vz, const double *m, double n1,
                                                    double n2, double dt, double *rc)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    double ms = mstar[sys_of[i]];
    double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
    double v2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
    double inv_a = 2.0 / r - v2 / ms;
    double a = inv_a > 0.0 ? 1.0 / inv_a : r;
    double rh = a * cbrt(m[i] / (3.0 * ms));
    double vk = sqrt(ms / a);
    rc[i] = fmax(n1 * rh, n2 * dt * vk);
}

} // namespace

hipError_t launch_prep(const Layout &L, double *x, double *y, double *z, const double *m,
                       const double *rc, void *jrec, int fp32, double *rc2_part, int32_t *pair_count,
                       const double *mom_part, double shift_tau, hipStream_t stream)
{
    if (L.n_chunks == 0) return hipSuccess;
    if (fp32)
        prep_kernel<true><<<L.n_chunks, SYS_P_THREADS, 0, stream>>>(L.chunks, L.chunk_first, L.mstar, mom_part,
                                                                    shift_tau, x, y, z, m, rc, jrec,
                                                                    rc2_part, pair_count);
    else
        prep_kernel<false><<<L.n_chunks, SYS_P_THREADS, 0, stream>>>(L.chunks, L.chunk_first, L.mstar, mom_part,
                                                                     shift_tau, x, y, z, m, rc, jrec,
                                                                     rc2_part, pair_count);
    return hipGetLastError();
}

hipError_t launch_kick(const KickArgs &a, int fp32, int kahan, int waves, int grid, hipStream_t stream)
{
    if (a.n_items == 0) return hipSuccess;
    const int n_tasks = a.n_items * a.split;
    if (grid <= 0 || grid > n_tasks) grid = n_tasks;
#define GENGA_KICK_CASE(Wv)                                                                   \
    case Wv:                                                                                  \
        if (fp32 && kahan)                                                                    \
            kick32_kernel<Wv, true><<<grid, 64 * Wv, 0, stream>>>(a);                        \
        else if (fp32)                                                                        \
            kick32_kernel<Wv, false><<<grid, 64 * Wv, 0, stream>>>(a);                       \
        else                                                                                  \
            kick64_kernel<Wv, false><<<grid, 64 * Wv, 0, stream>>>(a);                       \
        break;
    switch (waves) {
        GENGA_KICK_CASE(4)
        GENGA_KICK_CASE(8)
        GENGA_KICK_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GENGA_KICK_CASE
    if (a.split > 1) kick_finish_kernel<<<(a.n_total + 255) / 256, 256, 0, stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_pair_list(const KickArgs &a, int grid, hipStream_t stream)
{
    if (a.n_items == 0) return hipSuccess;
    const int n_tasks = a.n_items * a.split;
    if (grid <= 0 || grid > n_tasks) grid = n_tasks;
    kick64_kernel<8, true><<<grid, 64 * 8, 0, stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_rcrit(const Layout &L, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz, const double *m,
                        double n1, double n2, double dt, double *rc, hipStream_t stream)
{
    if (L.n_total == 0) return hipSuccess;
    rcrit_kernel<<<(L.n_total + 255) / 256, 256, 0, stream>>>(L.n_total, L.sys_of, L.mstar, x, y, z,
                                                              vx, vy, vz, m, n1, n2, dt, rc);
    return hipGetLastError();
}

} // namespace genga
