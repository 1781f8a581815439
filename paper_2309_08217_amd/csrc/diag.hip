// Diagnostics (Brasser et al. 2023, Sect. 3.1: Delta E/E and Delta L/L) and the canonical
// order of the encounter list.  FP64.
//
// Energy of the democratic heliocentric Hamiltonian per system:
//   E = sum m v^2/2 + |sum m v|^2/(2 Mstar) - sum Mstar m/r - sum_{i<j} m_i m_j / r_ij,
//   L = sum m r x v.
// The pair sum uses the kick's work items (64 targets per workgroup, W waves over the
// sources j > i); per-item partial sums are reduced in a fixed order, so the result is
// deterministic.  Velocities may be given half a kick ahead: v_sync = v - vshift * a.
#include "genga_internal.h"
#include "pair_math.h"

namespace genga {

namespace {

constexpr int EW = 8;      // waves per workgroup in the pair sum
constexpr int NPART = 9;   // pairpot, kin, sunpot, px, py, pz, lx, ly, lz

using CJ64 = const __attribute__((address_space(4))) double;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(64 * EW) void energy_kernel(
    const WorkItem *items, int n_items, const int32_t *sys_off, const double *mstar, const double *x,
    const double *y, const double *z, const double *vx, const double *vy, const double *vz,
    const double *m, const double *ax, const double *ay, const double *az, double vshift,
    double *partial, int split)
{
    __shared__ double red[EW][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    CJ64 *X = (CJ64 *)x;
    CJ64 *Y = (CJ64 *)y;
    CJ64 *Z = (CJ64 *)z;
    CJ64 *M = (CJ64 *)m;
    const int n_tasks = n_items * split;
    for (int it = blockIdx.x; it < n_tasks; it += gridDim.x) {
        const WorkItem w = items[it / split];
        const int part = it % split;
        const bool valid = lane < w.ni;
        const int i = w.i0 + (valid ? lane : 0);
        const double xi = x[i], yi = y[i], zi = z[i];
        // sources j in [i0, end of system), split into `split` parts over workgroups and each
        // part over the waves; only j > i counts
        // test-body items have nsrc <= i0 - off: no pair terms (test pairs do not count)
        const int jend = max(sys_off[w.sys] + w.nsrc, w.i0);
        const int per = (jend - w.i0 + split - 1) / split;
        const int p0 = min(w.i0 + part * per, jend);
        const int p1 = min(p0 + per, jend);
        const int chunk = (p1 - p0 + EW - 1) / EW;
        const int jb = min(p0 + wave * chunk, p1), je = min(jb + chunk, p1);
        double s = 0.0;
        const int jmask = min(je, w.i0 + 64);
        int j = jb;
        for (; j < jmask; ++j) {
            // sources inside the item's own range: only j > i counts (the self pair has q = 0,
            // so it is replaced by a harmless q = 1 with zero weight)
            const double dx = X[j] - xi, dy = Y[j] - yi, dz = Z[j] - zi;
            const bool take = j > i;
            const double q = take ? fma(dx, dx, fma(dy, dy, dz * dz)) : 1.0;
            const double mj = take ? M[j] : 0.0;
            s = fma(mj, inv_sqrt64(q), s);
        }
        for (; j + 2 <= je; j += 2) {
            const double dx0 = X[j] - xi, dy0 = Y[j] - yi, dz0 = Z[j] - zi;
            const double dx1 = X[j + 1] - xi, dy1 = Y[j + 1] - yi, dz1 = Z[j + 1] - zi;
            const double q0 = fma(dx0, dx0, fma(dy0, dy0, dz0 * dz0));
            const double q1 = fma(dx1, dx1, fma(dy1, dy1, dz1 * dz1));
            s = fma(M[j], inv_sqrt64(q0), s);
            s = fma(M[j + 1], inv_sqrt64(q1), s);
        }
        for (; j < je; ++j) {
            const double dx = X[j] - xi, dy = Y[j] - yi, dz = Z[j] - zi;
            const double q = fma(dx, dx, fma(dy, dy, dz * dz));
            s = fma(M[j], inv_sqrt64(q), s);
        }
        red[wave][lane] = s;
        __syncthreads();
        if (wave == 0) {
            double tot = 0.0;
#pragma unroll
            for (int k = 0; k < EW; ++k) tot += red[k][lane];
            double v[NPART];
            if (valid && part > 0) {
                v[0] = m[i] * tot;
                for (int k = 1; k < NPART; ++k) v[k] = 0.0;
            } else if (valid) {
                const double mi = m[i];
                const double ux = vx[i] - vshift * ax[i];
                const double uy = vy[i] - vshift * ay[i];
                const double uz = vz[i] - vshift * az[i];
                v[0] = mi * tot;
                v[1] = 0.5 * mi * (ux * ux + uy * uy + uz * uz);
                v[2] = -mstar[w.sys] * mi / sqrt(xi * xi + yi * yi + zi * zi);
                v[3] = mi * ux;
                v[4] = mi * uy;
                v[5] = mi * uz;
                v[6] = mi * (yi * uz - zi * uy);
                v[7] = mi * (zi * ux - xi * uz);
                v[8] = mi * (xi * uy - yi * ux);
            } else {
#pragma unroll
                for (int k = 0; k < NPART; ++k) v[k] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < NPART; ++k) {
                const double t = wave_sum(v[k]);
                if (lane == 0) partial[(size_t)it * NPART + k] = t;
            }
        }
        __syncthreads();
    }
}

// One workgroup per system: each thread sums a strided subset of the system's item partials
// in order, then a fixed tree in LDS combines the threads.
constexpr int EF_THREADS = 256;

__global__ __launch_bounds__(EF_THREADS) void energy_finish_kernel(const int32_t *item_first,
                                                                   const double *mstar,
                                                                   const double *partial, double *out,
                                                                   int split)
{
    __shared__ double red[NPART][EF_THREADS];
    const int s = blockIdx.x;
    double t[NPART];
    for (int k = 0; k < NPART; ++k) t[k] = 0.0;
    for (int it = item_first[s] * split + threadIdx.x; it < item_first[s + 1] * split; it += EF_THREADS)
        for (int k = 0; k < NPART; ++k) t[k] += partial[(size_t)it * NPART + k];
    for (int k = 0; k < NPART; ++k) red[k][threadIdx.x] = t[k];
    __syncthreads();
    for (int o = EF_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < NPART; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double p2 = red[3][0] * red[3][0] + red[4][0] * red[4][0] + red[5][0] * red[5][0];
        out[4 * s + 0] = red[1][0] + p2 / (2.0 * mstar[s]) + red[2][0] - red[0][0];
        out[4 * s + 1] = red[6][0];
        out[4 * s + 2] = red[7][0];
        out[4 * s + 3] = red[8][0];
    }
}

// ------------------------------------------------------------------------------------------
// Canonical (lexicographic) order of the encounter list: one workgroup, bitonic sort of
// 64-bit keys (i << 32 | j); in LDS up to 8192 pairs, otherwise in a global key buffer.
// ------------------------------------------------------------------------------------------
constexpr int SORT_THREADS = 1024;
constexpr int SORT_LDS = 8192;

template <typename KeyT>
__device__ void bitonic(KeyT *keys, int npow, bool global_mem)
{
    for (int size = 2; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int k = threadIdx.x; k < npow; k += SORT_THREADS) {
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
            if (global_mem) __threadfence();
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(SORT_THREADS) void sort_pairs_kernel(const int32_t *src,
                                                                  const int32_t *src_count,
                                                                  int32_t src_cap, int32_t *dst,
                                                                  int32_t dst_cap,
                                                                  int32_t *dst_count,
                                                                  uint64_t *gkeys, int32_t *flags)
{
    __shared__ uint64_t lkeys[SORT_LDS];
    const int count = *src_count;
    const int n = min(count, src_cap);
    if (threadIdx.x == 0) {
        *dst_count = count;
        if (count > src_cap) atomicOr(flags, FLAG_CAPACITY);
    }
    if (n <= 0) return;
    int npow = 1;
    while (npow < n) npow <<= 1;
    const bool in_lds = npow <= SORT_LDS;
    uint64_t *keys = in_lds ? lkeys : gkeys;
    for (int k = threadIdx.x; k < npow; k += SORT_THREADS)
        keys[k] = (k < n) ? (((uint64_t)(uint32_t)src[2 * k] << 32) | (uint32_t)src[2 * k + 1]) : ~0ull;
    if (!in_lds) __threadfence();
    __syncthreads();
    bitonic(keys, npow, !in_lds);
    const int nout = min(n, dst_cap);
    for (int k = threadIdx.x; k < nout; k += SORT_THREADS) {
        dst[2 * k] = (int32_t)(keys[k] >> 32);
        dst[2 * k + 1] = (int32_t)(keys[k] & 0xffffffffu);
    }
}

// ------------------------------------------------------------------------------------------
// A pair list handed in by the caller: every pair is checked before any launch indexes bodies
// with it; one invalid pair drops the list.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void import_pairs_kernel(const int32_t *sys_of, int n_total, const int32_t *src,
                                                           const int32_t *src_count, int32_t *dst, int32_t cap,
                                                           int32_t *bad)
{
    const int n = min(*src_count, cap);
    bool ok = true;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256) {
        const int i = src[2 * p], j = src[2 * p + 1];
        const bool good = i >= 0 && i < j && j < n_total && sys_of[i] == sys_of[j];
        ok = ok && good;
        dst[2 * p] = good ? i : 0;
        dst[2 * p + 1] = good ? j : 0;
    }
    if (!ok) atomicOr(bad, 1);
}

__global__ __launch_bounds__(64) void import_finish_kernel(const int32_t *src_count, int32_t *dst_count, int32_t cap,
                                                           int32_t *bad, int32_t *flags)
{
    if (threadIdx.x != 0) return;
    const int c = *src_count;
    if (*bad || c < 0) {
        *dst_count = 0;
        atomicOr(flags, FLAG_BADPAIR);
    } else {
        *dst_count = c;
        if (c > cap) atomicOr(flags, FLAG_CAPACITY);
    }
    *bad = 0;
}

} // namespace

hipError_t launch_import_pairs(const Layout &L, const int32_t *src, const int32_t *src_count, int32_t *dst,
                               int32_t *dst_count, int32_t cap, int32_t *bad, int32_t *flags, hipStream_t stream)
{
    const int blocks = std::max(1, std::min(1024, (cap + 255) / 256));
    import_pairs_kernel<<<blocks, 256, 0, stream>>>(L.sys_of, L.n_total, src, src_count, dst, cap, bad);
    import_finish_kernel<<<1, 64, 0, stream>>>(src_count, dst_count, cap, bad, flags);
    return hipGetLastError();
}

hipError_t launch_energy(const Layout &L, const WorkItem *items, int32_t n_items, const double *x,
                         const double *y, const double *z, const double *vx, const double *vy,
                         const double *vz, const double *m, const double *ax, const double *ay,
                         const double *az, double vshift, double *partial,
                         const int32_t *item_first, double *out, hipStream_t stream)
{
    if (n_items > 0)
        energy_kernel<<<n_items * ENERGY_SPLIT, 64 * EW, 0, stream>>>(items, n_items, L.sys_off, L.mstar, x, y,
                                                                      z, vx, vy, vz, m, ax, ay, az, vshift,
                                                                      partial, ENERGY_SPLIT);
    energy_finish_kernel<<<L.n_sys, EF_THREADS, 0, stream>>>(item_first, L.mstar, partial, out, ENERGY_SPLIT);
    return hipGetLastError();
}

hipError_t launch_sort_pairs(const int32_t *src, const int32_t *src_count, int32_t src_cap,
                             int32_t *dst, int32_t dst_cap, int32_t *dst_count, uint64_t *keys,
                             int32_t *flags, hipStream_t stream)
{
    sort_pairs_kernel<<<1, SORT_THREADS, 0, stream>>>(src, src_count, src_cap, dst, dst_cap, dst_count,
                                                      keys, flags);
    return hipGetLastError();
}

} // namespace genga
