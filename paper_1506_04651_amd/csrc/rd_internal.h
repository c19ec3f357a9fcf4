/*
 * rd_internal.h -- host-side internals shared by the C-ABI entry points
 * (rd_api.cpp) and the serving session (rd_serving.cpp).
 */
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/rd.h"
#include "rd_launch.h"

namespace rd {

void set_error(const char* fmt, ...);

/* One validated call, ready to launch. */
struct Prepared {
    const KernelEntry* entry = nullptr;
    LaunchArgs args{};
    int grid = 0;
    int device = 0;
    size_t param_key = 0;
    int order = 0; /* claim-order option of the call */
};

/* Per-device state: properties, counter slots, cached parameter blocks. */
struct DevCtx {
    int device = -1;
    int cu_count = 0;
    unsigned long long* slots = nullptr; /* 2 * kSlots counters */
    std::atomic<unsigned> next_slot{0};
    std::mutex mu;
    std::map<std::vector<double>, double*> params; /* key: {kind, m, block...} */
    /* per-stream scratch for the claim order; an outgrown buffer is freed
     * unless a captured graph references it (then it is kept: graphs live as
     * long as the process) */
    std::map<hipStream_t, std::pair<void*, size_t>> order_ws;
    std::set<void*> graph_ws;
    std::vector<void*> retired;
};
constexpr unsigned kSlots = 4096;

/* Context of the current device (created on first use); null on error. */
DevCtx* current_ctx();

/* Validate arguments, transform tolerances, upload (or find) the model's
 * parameter block, select the kernel.  Returns 0 or a negative RD_E* code. */
int prepare(double* states, int64_t n, int32_t m, double dt, double rtol, double atol,
            const rd_model* model, const rd_options* opts, int32_t* stats, Prepared* out);

/* Largest pre-processed model block (the bytecode model: L, C, 32 constants,
 * 4096 instructions), in doubles. */
constexpr size_t kMaxParamDoubles = 2 + RD_BC_REGS + 4096;

/* The host part of prepare: validation, tolerances, kernel choice, and the
 * model's device block written to `block` (kMaxParamDoubles doubles, *blen
 * used); no device work and no allocation.  out->args.params and out->grid
 * are left for the caller. */
int prepare_host(double* states, int64_t n, int32_t m, double dt, double rtol, double atol,
                 const rd_model* model, const rd_options* opts, int32_t* stats, Prepared* out,
                 double* block, size_t* blen);
bool model_block_into(const rd_model* model, int32_t m, double* out, size_t* len);

/* Scratch of at least `bytes` for launches on stream s (claim order). */
void* stream_workspace(DevCtx& c, hipStream_t s, size_t bytes, int* err);

/* Mark stream s's current claim-order scratch as referenced by a captured
 * graph, so that it is never freed. */
void pin_stream_workspace(DevCtx& c, hipStream_t s);

/* Bytes of claim-order scratch a persistent launch over n cells uses (0 when
 * the batch is too small to be ordered). */
size_t order_bytes(int64_t n);

/* Enqueue the claim-order kernels for a prepared persistent launch (when the
 * options ask for it and an order kernel exists); sets pr.args.order.  The
 * order kernels then also clear `counters` (two entries, nullable) and
 * *cleared is set; otherwise the caller clears them.  ws: order_bytes(n)
 * bytes of device scratch, or null for the stream's own scratch. */
int enqueue_order(DevCtx& c, Prepared& pr, hipStream_t s, unsigned long long* counters,
                  bool* cleared, void* ws = nullptr);

/* A prepared reaction step enqueued on stream s with the given counters
 * (claim position, failed cells; cleared by the enqueued work); no host
 * wait, no allocation once ensure_workspace(pr, s) has run.  0 or RD_E*. */
int enqueue_prepared(Prepared& pr, hipStream_t s, unsigned long long* counters);
int ensure_workspace(const Prepared& pr, hipStream_t s);

/* One reaction step enqueued on stream s with its failed-cell count copied,
 * behind it, into this thread's pinned host word `word` (0 or 1); returns 0
 * or a negative call-level error.  reaction_count(word) reads the count once
 * the stream has passed that copy. */
int64_t reaction_enqueue(double* states, int64_t n_cells, int32_t m, double dt, double rtol,
                         double atol, const rd_model* model, const rd_options* opts,
                         int32_t* stats, hipStream_t s, int word);
int64_t reaction_count(int word);

/* Grid for a persistent kernel: resident workgroups on the device, capped by
 * the number of workgroups the cells would fill. */
int persistent_grid(const DevCtx& c, const KernelEntry* e, int64_t n);
int persistent_grid_cu(int cu_count, const KernelEntry* e, int64_t n);

/* Host-side parameter pre-processing shared by direct calls and sessions:
 * returns false when the model is invalid.  block receives the device layout. */
bool model_block(const rd_model* model, int32_t m, std::vector<double>& block);

/* Tolerance transformation and Newton stopping tolerance. */
void make_step_params(double dt, double rtol, double atol, const rd_options& o,
                      StepParams* P);

/* jac: RD_JAC_ANALYTIC / RD_JAC_FD, or -1 for the kind's own Jacobian. */
const KernelEntry* find_kernel(int kind, int m, int precision, int schedule, int fixed,
                               int variant, int jac);

}  // namespace rd
