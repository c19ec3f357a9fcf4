/*
 * rd_noalloc.hip -- rd_reaction_step_noalloc (include/rd.h): the reaction
 * step without any device or pinned-host allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid it).
 *
 * Everything the launch needs beyond the caller's states and counters lives
 * in one file-scope device array, `scratch`, of a fixed size: the two 64-bit
 * counters of the persistent kernel (claim position, failed cells), the
 * model's pre-processed parameter block, and the claim-order scratch of the
 * longest-first order.  Each device holds its own copy of the array until the
 * process ends; its device address is looked up once per device with
 * hipGetSymbolAddress and only that address is used from the host.  Every
 * call on a device shares that device's array: the counters are cleared by a
 * kernel at the start of each launch, the parameter block and the claim order
 * are rewritten by each call, and calls that overlap on one device race.
 *
 * The kernels are those of rd_reaction_step_ex (same table, same variants),
 * so the results are bitwise those of the allocating entry point.
 */
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "rd_internal.h"

namespace rd {

/* layout of the array, in bytes */
constexpr size_t kNaCounters = 0;                          /* 2 x u64 */
constexpr size_t kNaParams = 256;                          /* kMaxParamDoubles doubles */
constexpr size_t kNaOrder = kNaParams + ((kMaxParamDoubles * sizeof(double) + 255) & ~(size_t)255);
constexpr int64_t kNaMaxCells = RD_NOALLOC_MAX_CELLS;
/* claim order: an int32 position and one byte per cell, 256-byte aligned
 * each, plus the bucket counters (below 4 KiB) */
constexpr size_t kNaOrderBytes = 4 * (size_t)kNaMaxCells + (size_t)kNaMaxCells + 8192;
constexpr size_t kNaBytes = kNaOrder + kNaOrderBytes;

static __device__ __align__(256) unsigned char scratch[kNaBytes];

struct NaDevice {
    unsigned char* ptr = nullptr; /* device address of this device's scratch */
    int cu_count = 0;
    double* block = nullptr;      /* this device's host copy of the parameter block */
};
static std::mutex g_na_mu;
static NaDevice g_na[64];
/* Host copies of the parameter blocks, one per device: the asynchronous copy
 * into the device array reads from here, which outlives the call (the next
 * call on the device overwrites it). */
static double g_na_block[64][kMaxParamDoubles];

/* The device address of `scratch` on the current device, looked up once per
 * device (with that device current). */
static int na_device(NaDevice* out) {
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    if (dev < 0 || dev >= 64) {
        set_error("device ordinal %d out of range", dev);
        return RD_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_na_mu);
    NaDevice& d = g_na[dev];
    if (!d.ptr) {
        void* p = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)); e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return RD_EDEVICE;
        }
        int cus = 0;
        if (hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            e != hipSuccess || cus < 1) {
            set_error("hipDeviceGetAttribute(compute units): %s", hipGetErrorString(e));
            return RD_EDEVICE;
        }
        d.cu_count = cus;
        d.block = g_na_block[dev];
        d.ptr = (unsigned char*)p;
    }
    *out = d;
    return 0;
}

}  // namespace rd

using namespace rd;

extern "C" {

int64_t rd_reaction_step_noalloc(double* states, int64_t n_cells, int32_t m, double dt,
                                 double rtol, double atol, const rd_model* model,
                                 const rd_options* opts, int32_t* stats, void* hip_stream,
                                 int32_t async) {
    if (opts && (opts->use_graph || opts->h_cells)) {
        set_error("rd_reaction_step_noalloc: use_graph and h_cells are not accepted");
        return RD_EINVAL;
    }
    if (n_cells > kNaMaxCells) {
        set_error("rd_reaction_step_noalloc: %lld cells exceed its fixed scratch of %lld cells",
                  (long long)n_cells, (long long)kNaMaxCells);
        return RD_ETOOBIG;
    }
    if (order_bytes(n_cells) > kNaOrderBytes) {
        set_error("rd_reaction_step_noalloc: claim-order scratch too small");
        return RD_ETOOBIG;
    }
    NaDevice d;
    int r = na_device(&d);
    if (r != 0) return r;
    Prepared pr;
    size_t blen = 0;
    r = prepare_host(states, n_cells, m, dt, rtol, atol, model, opts, stats, &pr, d.block, &blen);
    if (r < 0) return r;
    if (n_cells == 0) return 0;
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned long long* counters = (unsigned long long*)(d.ptr + kNaCounters);
    double* params = (double*)(d.ptr + kNaParams);
    if (hipError_t e = hipMemcpyAsync(params, d.block, blen * sizeof(double), hipMemcpyHostToDevice, s);
        e != hipSuccess) {
        set_error("parameter copy: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    pr.args.params = params;
    pr.args.counter = counters;
    pr.args.nfail = counters + 1;
    pr.grid = pr.entry->schedule == RD_PERSISTENT
                  ? persistent_grid_cu(d.cu_count, pr.entry, n_cells)
                  : (int)((n_cells + pr.entry->cells_per_block - 1) / pr.entry->cells_per_block);
    /* the claim-order kernels (which also clear the counters) with the
     * order scratch of the array, or a clearing kernel */
    bool cleared = false;
    pr.args.order = nullptr;
    if (pr.entry->schedule == RD_PERSISTENT && pr.order && order_bytes(n_cells) != 0) {
        order_fn fn = find_order_fn(pr.entry->kind, m);
        if (fn) {
            unsigned char* ws = d.ptr + kNaOrder;
            const size_t ordb = ((size_t)n_cells * sizeof(int32_t) + 255) & ~(size_t)255;
            if (hipError_t e = fn(pr.args, ws + ordb, (int32_t*)ws, counters, s); e != hipSuccess) {
                set_error("claim-order launch: %s", hipGetErrorString(e));
                return RD_EDEVICE;
            }
            pr.args.order = (const int32_t*)ws;
            cleared = true;
        }
    }
    if (!cleared) {
        if (hipError_t e = launch_reset(counters, 2, s); e != hipSuccess) {
            set_error("counter reset: %s", hipGetErrorString(e));
            return RD_EDEVICE;
        }
    }
    if (hipError_t e = pr.entry->launch(pr.args, pr.grid, s); e != hipSuccess) {
        set_error("reaction-step launch: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    if (async) return 0;
    unsigned long long nfail = 0;
    if (hipError_t e = hipMemcpyAsync(&nfail, counters + 1, sizeof(nfail), hipMemcpyDeviceToHost, s);
        e != hipSuccess) {
        set_error("failure-count copy: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    if (hipError_t e = hipStreamSynchronize(s); e != hipSuccess) {
        set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    return (int64_t)nfail;
}

size_t rd_noalloc_scratch_bytes(void) { return kNaBytes; }

}  // extern "C"
