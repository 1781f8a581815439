// Encounter groups of a level's pair list laid out on the device (hierarchical levels,
// Brasser et al. 2023, Sect. 1: the pairs closer than a level's critical radius form the groups
// that the next level integrates).  The groups are the connected components of the pairs, found
// by the grid-wide union-find (a fixed number of rounds, each skipped once the previous one
// changed nothing); their members are taken in the order of the parent level's layout, grouped
// by a stable radix sort of (root, parent position), and cut into tiles of 64 for the next
// level's kick.  Everything stays on the device; the host reads one small header per grouping
// (the sizes it needs to size the next launches).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "genga_internal.h"

namespace genga {

namespace {

constexpr int GL_THREADS = 256;

__device__ __forceinline__ int32_t lab_of(const int32_t *lab, int32_t b)
{
    return __hip_atomic_load(&lab[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Header cleared; with full, also the pair count of the list recorded and the round words cleared.
__global__ __launch_bounds__(64) void group_begin_kernel(GroupHeader *hdr, const int32_t *pair_count,
                                                         int32_t *changed, int full)
{
    if (threadIdx.x == 0) {
        hdr->G = 0;
        hdr->M = 0;
        hdr->n_tiles = 0;
        hdr->n_multi = 0;
        hdr->max_nb = 0;
        hdr->unconverged = 0;
        if (full) hdr->pair_count = *pair_count;
        hdr->pad = 0;
    }
    if (full && (int)threadIdx.x < UF_ROUNDS) changed[threadIdx.x] = 0;
}

// The round words: unconverged when the last round still hooked something.
__global__ __launch_bounds__(64) void group_rounds_kernel(GroupHeader *hdr, const int32_t *changed)
{
    if (threadIdx.x == 0) hdr->unconverged = changed[UF_ROUNDS - 1] != 0;
}

// Sort key of parent position p: (root of its body) * Mp + p, or the sentinel for a body in no
// pair.
__global__ __launch_bounds__(GL_THREADS) void group_keys_kernel(const int32_t *pbody, int Mp, const int32_t *lab,
                                                                uint64_t sentinel, uint64_t *keys)
{
    const int p = blockIdx.x * GL_THREADS + threadIdx.x;
    if (p >= Mp) return;
    const int32_t r = lab_of(lab, pbody[p]);
    keys[p] = r >= 0 ? (uint64_t)(uint32_t)r * (uint64_t)Mp + (uint64_t)p : sentinel;
}

// Members in sorted order and the first member of each group.
__global__ __launch_bounds__(GL_THREADS) void group_mark_kernel(const uint64_t *sorted, int Mp, uint64_t sentinel,
                                                                const int32_t *pbody, int32_t *body_out,
                                                                int32_t *flag)
{
    const int q = blockIdx.x * GL_THREADS + threadIdx.x;
    if (q >= Mp) return;
    const uint64_t k = sorted[q];
    const bool valid = k < sentinel;
    bool start = false;
    if (valid) {
        body_out[q] = pbody[(int)(k % (uint64_t)Mp)];
        start = q == 0 || sorted[q - 1] / (uint64_t)Mp != k / (uint64_t)Mp;
    }
    flag[q] = start ? 1 : 0;
}

// Group offsets; the last member writes the totals.
__global__ __launch_bounds__(GL_THREADS) void group_offsets_kernel(const uint64_t *sorted, int Mp, uint64_t sentinel,
                                                                   const int32_t *flag, const int32_t *gidx,
                                                                   int32_t *off, GroupHeader *hdr)
{
    const int q = blockIdx.x * GL_THREADS + threadIdx.x;
    if (q >= Mp) return;
    const bool valid = sorted[q] < sentinel;
    if (q == 0 && !valid) { // no member at all
        off[0] = 0;
        return;
    }
    if (!valid) return;
    if (flag[q]) off[gidx[q]] = q;
    if (q + 1 == Mp || sorted[q + 1] >= sentinel) {
        const int G = gidx[q] + flag[q];
        off[G] = q + 1;
        hdr->G = G;
        hdr->M = q + 1;
    }
}

// Per group: its size into the header's maximum and its tiles as (tiles of groups of several
// tiles) << 32 | (1 for a group of one tile), for the scan below.
__global__ __launch_bounds__(GL_THREADS) void group_sizes_kernel(const int32_t *off, GroupHeader *hdr, int Gcap,
                                                                 uint64_t *tv)
{
    const int g = blockIdx.x * GL_THREADS + threadIdx.x;
    if (g >= Gcap) return;
    const int G = hdr->G;
    uint64_t v = 0;
    if (g < G) {
        const int nb = off[g + 1] - off[g];
        const int nt = (nb + 63) / 64;
        v = nt > 1 ? (uint64_t)nt << 32 : 1ull;
        atomicMax(&hdr->max_nb, nb);
    }
    tv[g] = v;
}

// Tiles of 64 members, group by group: each group's first tile (tfirst) and the header's tile
// counts; group_tile_fill_kernel then writes the tiles and the launch list tl (the tiles of
// groups of several tiles first, a workgroup each, then the tile of every group of one tile, a
// wave each).
__global__ __launch_bounds__(GL_THREADS) void group_tiles_kernel(GroupHeader *hdr, int Gcap, const uint64_t *tv,
                                                                 const uint64_t *tscan, int32_t *tfirst)
{
    const int g = blockIdx.x * GL_THREADS + threadIdx.x;
    if (g >= Gcap) return;
    const int G = hdr->G;
    if (g >= G) return;
    const uint64_t tot = tscan[G - 1] + tv[G - 1];
    const int n_multi = (int)(tot >> 32), n_tiles = n_multi + (int)(tot & 0xffffffffu);
    const uint64_t e = tscan[g];
    const int mo = (int)(e >> 32), so = (int)(e & 0xffffffffu);
    tfirst[g] = mo + so;
    if (g == G - 1) {
        tfirst[G] = n_tiles;
        hdr->n_tiles = n_tiles;
        hdr->n_multi = n_multi;
    }
}

// The tiles themselves, one thread each (a group of many tiles would otherwise be one thread's
// loop): tile t belongs to the last group whose first tile is at most t (every group has one).
__global__ __launch_bounds__(GL_THREADS) void group_tile_fill_kernel(const int32_t *off, const GroupHeader *hdr,
                                                                     const uint64_t *tscan, const int32_t *tfirst,
                                                                     int4 *tiles, int32_t *tl, int Tcap)
{
    const int G = hdr->G, n_tiles = hdr->n_tiles, n_multi = hdr->n_multi;
    if (G <= 0) return;
    for (int t = blockIdx.x * GL_THREADS + threadIdx.x; t < min(n_tiles, Tcap); t += gridDim.x * GL_THREADS) {
        int lo = 0, hi = G - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tfirst[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int g = lo, k = t - tfirst[g];
        const int o = off[g], nb = off[g + 1] - o, nt = (nb + 63) / 64;
        const uint64_t e = tscan[g];
        const int mo = (int)(e >> 32), so = (int)(e & 0xffffffffu);
        tiles[t] = make_int4(g, o + 64 * k, min(64, nb - 64 * k), 0);
        tl[nt > 1 ? mo + k : n_multi + so] = t;
    }
}

int bits_for(uint64_t v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}


// a monotone stand-in for atan2(y, x) on [0, 4)
__device__ __forceinline__ double pseudo_angle(double x, double y)
{
    const double s = fabs(x) + fabs(y);
    if (!(s > 0.0)) return 0.0;
    const double t = y / s; // in [-1, 1]
    return x >= 0.0 ? (y >= 0.0 ? t : 4.0 + t) : 2.0 - t;
}

// The group of layout position p: the last gi with off[gi] <= p (empty groups share their
// offset with the next one and are passed over).
__device__ __forceinline__ int group_of(const int32_t *off, int n_groups, int p)
{
    int lo = 0, hi = n_groups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int ring_body(const int32_t *members, const int32_t *k0, const int32_t *off, int gi,
                                         int p)
{
    const int m = k0[gi] + (p - off[gi]);
    return members ? members[m] : m;
}

__global__ __launch_bounds__(256) void ring_bounds_clear_kernel(int n_groups, uint64_t *bounds)
{
    for (int g = blockIdx.x * 256 + threadIdx.x; g < n_groups; g += gridDim.x * 256) {
        bounds[2 * g] = 0x7ff0000000000000ull; // +inf: the smallest distance so far
        bounds[2 * g + 1] = 0ull;              // +0
    }
}

// Each group's smallest and largest distance to the star over the layout positions: a wave
// whose lanes share one group reduces first; the atomics order the bit patterns, which for
// non-negative doubles is the numeric order, so the result does not depend on the order.
__global__ __launch_bounds__(256) void ring_bounds_kernel(const int32_t *members, const int32_t *k0,
                                                          const int32_t *off, int n_groups, int M, const double *x,
                                                          const double *y, uint64_t *bounds)
{
#pragma clang fp contract(off)
    const int stride = gridDim.x * 256;
    for (int base = blockIdx.x * 256; base < M; base += stride) {
        const int p = base + (int)threadIdx.x;
        const bool on = p < M;
        const int gi = on ? group_of(off, n_groups, p) : 0;
        double r0 = INFINITY, r1 = 0.0;
        if (on) {
            const int bi = ring_body(members, k0, off, gi, p);
            r0 = r1 = sqrt(x[bi] * x[bi] + y[bi] * y[bi]);
        }
        const int g0 = __builtin_amdgcn_readfirstlane(gi);
        const unsigned long long act = __ballot(true);
        if (__ballot(on && gi == g0) == act) {
            for (int d = 32; d > 0; d >>= 1) {
                r0 = fmin(r0, __shfl_xor(r0, d, 64));
                r1 = fmax(r1, __shfl_xor(r1, d, 64));
            }
            if ((threadIdx.x & 63) == 0) {
                atomicMin((unsigned long long *)&bounds[2 * g0], (unsigned long long)__double_as_longlong(r0));
                atomicMax((unsigned long long *)&bounds[2 * g0 + 1], (unsigned long long)__double_as_longlong(r1));
            }
        } else if (on) {
            atomicMin((unsigned long long *)&bounds[2 * gi], (unsigned long long)__double_as_longlong(r0));
            atomicMax((unsigned long long *)&bounds[2 * gi + 1], (unsigned long long)__double_as_longlong(r1));
        }
    }
}

// Per layout position: the member's key (gi, ring, azimuth) and body.  The rings are
// equal-width bands of distance to the star, as many as make a tile of 64 members about as
// wide as long (the band's circumference taken at the middle of the group's range); the
// quantised (ring + azimuth / 4) / rings orders the members.
__global__ __launch_bounds__(256) void ring_keys_kernel(const int32_t *members, const int32_t *k0, const int32_t *off,
                                                        int n_groups, int M, const double *x, const double *y,
                                                        const uint64_t *bounds, uint64_t *key, int32_t *val)
{
#pragma clang fp contract(off)
    for (int p = blockIdx.x * 256 + threadIdx.x; p < M; p += gridDim.x * 256) {
        const int gi = group_of(off, n_groups, p);
        const int bi = ring_body(members, k0, off, gi, p);
        const int nb = off[gi + 1] - off[gi];
        const double r0 = __longlong_as_double((long long)bounds[2 * gi]);
        const double r1 = __longlong_as_double((long long)bounds[2 * gi + 1]);
        const double width = fmax(r1 - r0, 1e-300), rmid = fmax(0.5 * (r0 + r1), 1e-300);
        const double nr = fmin(sqrt(nb * width / (64.0 * 2.0 * M_PI * rmid)), 1048576.0);
        const int rings = max(1, (int)lround(nr));
        const double r = sqrt(x[bi] * x[bi] + y[bi] * y[bi]);
        const int ring = min(rings - 1, (int)((r - r0) / width * rings));
        const double u = (ring + 0.25 * pseudo_angle(x[bi], y[bi])) / rings; // [0, 1]
        const uint64_t q = (uint64_t)fmin(4294967295.0, fmax(0.0, u * 4294967295.0));
        key[p] = (uint64_t)gi << 32 | q;
        val[p] = bi;
    }
}

} // namespace

hipError_t group_work_alloc(GroupWork &w, int cap)
{
    group_work_free(w);
    w.cap = cap > 1 ? cap : 2;
    const size_t n = (size_t)w.cap, ng = n / 2 + 2;
    hipError_t e;
    if ((e = hipMalloc((void **)&w.keys, n * sizeof(uint64_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.keys_sorted, n * sizeof(uint64_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.flag, n * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.gidx, n * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.tv, ng * sizeof(uint64_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.tscan, ng * sizeof(uint64_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.changed, UF_ROUNDS * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.hdr, sizeof(GroupHeader))) != hipSuccess) return e;
    // temporary storage of the sort and the two scans, for the largest sizes
    size_t b0 = 0, b1 = 0, b2 = 0;
    if ((e = rocprim::radix_sort_keys(nullptr, b0, w.keys, w.keys_sorted, (unsigned int)n, 0, 64)) != hipSuccess)
        return e;
    if ((e = rocprim::exclusive_scan(nullptr, b1, w.flag, w.gidx, 0, n, rocprim::plus<int32_t>())) != hipSuccess)
        return e;
    if ((e = rocprim::exclusive_scan(nullptr, b2, w.tv, w.tscan, (uint64_t)0, ng, rocprim::plus<uint64_t>())) !=
        hipSuccess)
        return e;
    w.temp_bytes = std::max(b0, std::max(b1, b2));
    if ((e = hipMalloc(&w.temp, w.temp_bytes ? w.temp_bytes : 1)) != hipSuccess) return e;
    return hipSuccess;
}

void group_work_free(GroupWork &w)
{
    for (void *p : {(void *)w.keys, (void *)w.keys_sorted, (void *)w.flag, (void *)w.gidx, (void *)w.tv,
                    (void *)w.tscan, (void *)w.changed, (void *)w.hdr, w.temp})
        if (p) (void)hipFree(p);
    w = GroupWork{};
}

hipError_t launch_group_layout(const Layout &L, GroupWork &w, const int32_t *pairs, const int32_t *pair_count,
                               int32_t pair_cap, int32_t *lab, const int32_t *pbody, int Mp, const GroupOut &out,
                               hipStream_t stream, bool union_find)
{
    if (Mp > w.cap) return hipErrorInvalidValue;
    group_begin_kernel<<<1, 64, 0, stream>>>(w.hdr, pair_count, w.changed, union_find ? 1 : 0);
    hipError_t e;
    if (union_find) {
        if ((e = launch_uf_init(pairs, pair_count, pair_cap, lab, stream)) != hipSuccess) return e;
        // rounds of two (hook, compress) passes; a round whose predecessor changed nothing is skipped
        for (int r = 0; r < UF_ROUNDS; ++r) {
            const int32_t *run_if = r > 0 ? w.changed + r - 1 : nullptr;
            for (int rep = 0; rep < 2; ++rep) {
                if ((e = launch_uf_hook(pairs, pair_count, pair_cap, lab, w.changed + r, stream, run_if)) !=
                    hipSuccess)
                    return e;
                if ((e = launch_uf_compress(L, lab, stream, run_if)) != hipSuccess) return e;
            }
        }
        group_rounds_kernel<<<1, 64, 0, stream>>>(w.hdr, w.changed);
    }
    if (Mp == 0) return hipGetLastError();
    const uint64_t sentinel = (uint64_t)(uint32_t)L.n_total * (uint64_t)Mp;
    const int nb = (Mp + GL_THREADS - 1) / GL_THREADS;
    group_keys_kernel<<<nb, GL_THREADS, 0, stream>>>(pbody, Mp, lab, sentinel, w.keys);
    size_t bytes = w.temp_bytes;
    if ((e = rocprim::radix_sort_keys(w.temp, bytes, w.keys, w.keys_sorted, (unsigned int)Mp, 0, bits_for(sentinel),
                                      stream)) != hipSuccess)
        return e;
    group_mark_kernel<<<nb, GL_THREADS, 0, stream>>>(w.keys_sorted, Mp, sentinel, pbody, out.body, w.flag);
    bytes = w.temp_bytes;
    if ((e = rocprim::exclusive_scan(w.temp, bytes, w.flag, w.gidx, 0, (size_t)Mp, rocprim::plus<int32_t>(),
                                     stream)) != hipSuccess)
        return e;
    group_offsets_kernel<<<nb, GL_THREADS, 0, stream>>>(w.keys_sorted, Mp, sentinel, w.flag, w.gidx, out.off, w.hdr);
    // groups have at least two members
    const int Gcap = Mp / 2 + 1, ng = (Gcap + GL_THREADS - 1) / GL_THREADS;
    group_sizes_kernel<<<ng, GL_THREADS, 0, stream>>>(out.off, w.hdr, Gcap, w.tv);
    if (out.tiles) {
        bytes = w.temp_bytes;
        if ((e = rocprim::exclusive_scan(w.temp, bytes, w.tv, w.tscan, (uint64_t)0, (size_t)Gcap,
                                         rocprim::plus<uint64_t>(), stream)) != hipSuccess)
            return e;
        group_tiles_kernel<<<ng, GL_THREADS, 0, stream>>>(w.hdr, Gcap, w.tv, w.tscan, out.tfirst);
        // at most one tile per member
        group_tile_fill_kernel<<<std::min(nb, 1024), GL_THREADS, 0, stream>>>(out.off, w.hdr, w.tscan, out.tfirst,
                                                                              out.tiles, out.tl, Mp);
    }
    return hipGetLastError();
}

hipError_t order_work_alloc(OrderWork &w, int cap)
{
    order_work_free(w);
    w.cap = cap > 1 ? cap : 2;
    const size_t n = (size_t)w.cap;
    hipError_t e;
    if ((e = hipMalloc((void **)&w.keys, n * sizeof(uint64_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.keys_sorted, n * sizeof(uint64_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.vals, n * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&w.bounds, 2 * n * sizeof(uint64_t))) != hipSuccess) return e;
    int32_t *out = nullptr;
    if ((e = rocprim::radix_sort_pairs(nullptr, w.temp_bytes, w.keys, w.keys_sorted, w.vals, out, (unsigned int)n, 0,
                                       64)) != hipSuccess)
        return e;
    return hipMalloc(&w.temp, w.temp_bytes ? w.temp_bytes : 1);
}

void order_work_free(OrderWork &w)
{
    for (void *p : {(void *)w.keys, (void *)w.keys_sorted, (void *)w.vals, (void *)w.bounds, w.temp})
        if (p) (void)hipFree(p);
    w = OrderWork{};
}

hipError_t launch_ring_order(const int32_t *members, const int32_t *k0, const int32_t *off, int n_groups, int M,
                             const double *x, const double *y, OrderWork &w, int32_t *body_out, hipStream_t stream)
{
    if (n_groups <= 0 || M <= 0) return hipSuccess;
    if (M > w.cap || n_groups > w.cap) return hipErrorInvalidValue;
    const int grid = std::min((M + 255) / 256, 2048);
    ring_bounds_clear_kernel<<<std::min((n_groups + 255) / 256, 256), 256, 0, stream>>>(n_groups, w.bounds);
    ring_bounds_kernel<<<grid, 256, 0, stream>>>(members, k0, off, n_groups, M, x, y, w.bounds);
    ring_keys_kernel<<<grid, 256, 0, stream>>>(members, k0, off, n_groups, M, x, y, w.bounds, w.keys, w.vals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = w.temp_bytes;
    return rocprim::radix_sort_pairs(w.temp, bytes, w.keys, w.keys_sorted, w.vals, body_out, (unsigned int)M, 0,
                                     32 + bits_for((uint64_t)n_groups), stream);
}

} // namespace genga
