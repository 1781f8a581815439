// Allocation-free long-range accelerations of one system (genga_accel_noalloc): the kick's
// source records, launch plan and split shares live in one file-scope device array instead of
// a context's allocations, for callers that cannot allocate device memory (graph capture,
// serving loops).  The kernels are the kick's own (kick.hip), launched with the shape a
// context picks by default for the same single system, so the results equal genga_accel's.
#include <mutex>

#include "genga_internal.h"

namespace genga {

namespace {

constexpr int NA_MAX_N = GENGA_NOALLOC_MAX_BODIES;
constexpr int NA_MAX_ITEMS = NA_MAX_N / 64;
constexpr int NA_MAX_CHUNKS = NA_MAX_N / CHUNK;
constexpr int NA_MAX_DEVICES = 64;

// byte offsets of the parts of the scratch array (each a multiple of 256)
constexpr size_t align256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t OFF_JREC = 0;                                                 // 32 B per body
constexpr size_t OFF_PART = OFF_JREC + align256((size_t)NA_MAX_N * 32);       // [split][3][n] FP64
constexpr size_t OFF_ITEMS = OFF_PART + align256((size_t)KICK_MAX_SPLIT * 3 * NA_MAX_N * sizeof(double));
constexpr size_t OFF_CHUNKS = OFF_ITEMS + align256((size_t)NA_MAX_ITEMS * sizeof(WorkItem));
constexpr size_t OFF_RC2 = OFF_CHUNKS + align256((size_t)NA_MAX_CHUNKS * sizeof(Chunk));
constexpr size_t OFF_SMALL = OFF_RC2 + align256((size_t)NA_MAX_CHUNKS * sizeof(double)); // sys_off[2], chunk_first[2]
constexpr size_t SCRATCH_BYTES = OFF_SMALL + 256;

// Each GPU the library runs on holds its own copy until the process ends; host code takes its
// address from hipGetSymbolAddress (the name itself is not a device address on the host).
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

struct DeviceScratch {
    unsigned char *ptr = nullptr;
    int n_cu = 0;
};
DeviceScratch g_dev[NA_MAX_DEVICES];
std::mutex g_mu;

// Launch plan of one system of n bodies, all massive: the chunks of the O(N) source-record
// pass and the kick's items of 64 targets; clears the caller's count and status words.
__global__ __launch_bounds__(256) void noalloc_plan_kernel(int n, Chunk *chunks, WorkItem *items, int32_t *small,
                                                           int32_t *d_count, int32_t *d_status)
{
    const int n_chunks = (n + CHUNK - 1) / CHUNK, n_items = (n + 63) / 64;
    for (int k = threadIdx.x; k < n_chunks; k += blockDim.x)
        chunks[k] = Chunk{0, k * CHUNK, min((k + 1) * CHUNK, n), 0};
    for (int k = threadIdx.x; k < n_items; k += blockDim.x)
        items[k] = WorkItem{0, 64 * k, min(64, n - 64 * k), n};
    if (threadIdx.x == 0) {
        small[0] = 0;        // sys_off
        small[1] = n;
        small[2] = 0;        // chunk_first
        small[3] = n_chunks;
        *d_count = 0;
        *d_status = 0;
    }
}

} // namespace

// Address of the scratch array on the current device (looked up once per device).
int noalloc_prepare(int device, unsigned char **ptr_out, int *n_cu_out)
{
    if (device < 0 || device >= NA_MAX_DEVICES) return fail(GENGA_ERR_ARG, "device %d not supported", device);
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceScratch &d = g_dev[device];
    if (!d.ptr) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(GENGA_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        int n_cu = 0;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
        if (e != hipSuccess) return fail(GENGA_ERR_HIP, "device attribute: %s", hipGetErrorString(e));
        d.n_cu = n_cu > 0 ? n_cu : 256;
        d.ptr = (unsigned char *)p;
    }
    if (ptr_out) *ptr_out = d.ptr;
    if (n_cu_out) *n_cu_out = d.n_cu;
    return GENGA_OK;
}

} // namespace genga

using namespace genga;

extern "C" int genga_accel_noalloc(const genga_bodies *b, int32_t n, double *ax, double *ay, double *az,
                                   int32_t *pairs, int32_t pair_cap, int32_t *d_count, int32_t *d_status,
                                   int prec, int acc, void *stream)
{
    if (prec != GENGA_KICK_FP32 && prec != GENGA_KICK_FP64) return fail(GENGA_ERR_ARG, "bad precision %d", prec);
    if (acc != GENGA_ACC_FP64 && acc != GENGA_ACC_KAHAN32) return fail(GENGA_ERR_ARG, "bad accumulator %d", acc);
    if (n < 0 || n > NA_MAX_N)
        return fail(GENGA_ERR_ARG, "n = %d bodies: the allocation-free call takes 0..%d", n, NA_MAX_N);
    if (!d_count || !d_status) return fail(GENGA_ERR_ARG, "null d_count or d_status");
    if (pair_cap < 0 || (pair_cap > 0 && !pairs)) return fail(GENGA_ERR_ARG, "bad pairs buffer");
    if (n > 0) {
        if (!b || !b->x || !b->y || !b->z || !b->m || !b->rcrit)
            return fail(GENGA_ERR_ARG, "null bodies, position, mass or rcrit array");
        if (!ax || !ay || !az) return fail(GENGA_ERR_ARG, "null acceleration array");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GENGA_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    unsigned char *base = nullptr;
    int n_cu = 0;
    int rc = noalloc_prepare(dev, &base, &n_cu);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;

    Chunk *chunks = (Chunk *)(base + OFF_CHUNKS);
    WorkItem *items = (WorkItem *)(base + OFF_ITEMS);
    int32_t *small = (int32_t *)(base + OFF_SMALL);
    noalloc_plan_kernel<<<1, 256, 0, s>>>(n, chunks, items, small, d_count, d_status);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(GENGA_ERR_HIP, "plan launch: %s", hipGetErrorString(e));
    if (n == 0) return GENGA_OK;

    const int fp32 = prec == GENGA_KICK_FP32;
    Layout L;
    L.n_sys = 1;
    L.n_total = n;
    L.n_chunks = (n + CHUNK - 1) / CHUNK;
    L.sys_off = small;
    L.chunks = chunks;
    L.chunk_first = small + 2;
    double *rc2_part = (double *)(base + OFF_RC2);
    void *jrec = base + OFF_JREC;
    e = launch_prep(L, b->x, b->y, b->z, b->m, b->rcrit, jrec, fp32, rc2_part, d_count, nullptr, 0.0, s);
    if (e != hipSuccess) return fail(GENGA_ERR_HIP, "source records: %s", hipGetErrorString(e));

    KickArgs a{};
    a.items = items;
    a.n_items = (n + 63) / 64;
    a.sys_off = small;
    a.x = b->x;
    a.y = b->y;
    a.z = b->z;
    a.m = b->m;
    a.rc = b->rcrit;
    a.jrec = jrec;
    a.rc2_part = rc2_part;
    a.chunk_first = small + 2;
    a.ax = ax;
    a.ay = ay;
    a.az = az;
    a.update_v = 0;
    a.pairs = pairs;
    a.pair_count = d_count;
    a.pair_cap = pair_cap;
    a.flags = d_status;
    a.split = default_kick_split(a.n_items, n_cu);
    a.n_total = n;
    a.part = (double *)(base + OFF_PART);
    e = launch_kick(a, fp32, acc == GENGA_ACC_KAHAN32, default_kick_waves(fp32), 0, s);
    if (e != hipSuccess) return fail(GENGA_ERR_HIP, "kick launch: %s", hipGetErrorString(e));
    return GENGA_OK;
}
