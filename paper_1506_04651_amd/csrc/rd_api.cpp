/*
 * rd_api.cpp -- the C ABI of librd (declared in include/rd.h): argument
 * validation, tolerance transformation, model-parameter upload, kernel
 * selection, launch (direct or through a cached hipGraph) and completion.
 *
 * The operation is the reaction substep of the Strang splitting scheme
 * (Descombes et al., §2.1) integrated per cell with Radau5 (paper §1 footnote;
 * Hairer & Wanner §IV.8); see include/rd.h for the contract.
 */
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "rd_internal.h"

namespace rd {

const KernelEntry* small_kernel_table(int* count);
const KernelEntry* group_kernel_table(int* count);
const KernelEntry* fd_kernel_table(int* count);
const KernelEntry* group_fd_kernel_table(int* count);

/* ---------------------------------------------------------------- errors */
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                  \
            return RD_EDEVICE;                                                         \
        }                                                                              \
    } while (0)

/* ---------------------------------------------------------------- kernels */
static std::vector<KernelEntry>& all_kernels() {
    static std::vector<KernelEntry> v = [] {
        std::vector<KernelEntry> out;
        int n = 0;
        const KernelEntry* t = small_kernel_table(&n);
        out.insert(out.end(), t, t + n);
        t = group_kernel_table(&n);
        out.insert(out.end(), t, t + n);
        t = fd_kernel_table(&n);
        out.insert(out.end(), t, t + n);
        t = group_fd_kernel_table(&n);
        out.insert(out.end(), t, t + n);
        return out;
    }();
    return v;
}

const KernelEntry* kernel_table(int* count) {
    *count = (int)all_kernels().size();
    return all_kernels().data();
}

static std::mutex g_variant_mu;
static std::map<std::tuple<int, int, int, int>, int> g_default_variant;

static int default_variant(int kind, int m, int precision, int schedule) {
    std::lock_guard<std::mutex> lk(g_variant_mu);
    auto it = g_default_variant.find({kind, m, precision, schedule});
    return it == g_default_variant.end() ? 1 : it->second;
}

/* The kind's own Jacobian: analytic, except for the bytecode model. */
static int native_jac(int kind) { return kind == RD_BYTECODE ? RD_JAC_FD : RD_JAC_ANALYTIC; }

/* Species count under which a request's kernels are registered: kinetics and
 * linear models with 5..8 species run on the 8-column group kernels (m = 8),
 * with 9..16 on the 16-column ones (m = 16), and so do bytecode models with
 * more than 4 species; everything else under its own m.
 * Variant ids and tuned defaults refer to this registry entry. */
static int registry_m(int kind, int m) {
    if ((kind == RD_KINETICS || kind == RD_LINEAR || kind == RD_BYTECODE) && m > 4 && m <= RD_MAX_M)
        return m <= 8 ? 8 : 16;
    return m;
}

const KernelEntry* find_kernel(int kind, int m, int precision, int schedule, int fixed,
                               int variant, int jac) {
    m = registry_m(kind, m);
    if (jac < 0) jac = native_jac(kind);
    /* tuned defaults and variant ids refer to the kind's own Jacobian; the
     * finite-difference kernels of analytic models come in one variant */
    if (fixed || jac != native_jac(kind)) variant = 1;
    else if (variant <= 0) variant = default_variant(kind, m, precision, schedule);
    for (const KernelEntry& e : all_kernels())
        if (e.kind == kind && e.jac == jac && e.m == m && e.precision == precision &&
            e.schedule == schedule && e.fixed == fixed && e.variant == variant)
            return &e;
    return nullptr;
}

/* ---------------------------------------------------------------- devices */
static std::mutex g_ctx_mu;
static DevCtx* g_ctx[64];

DevCtx* current_ctx() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= 64) {
        set_error("device ordinal %d out of range", dev);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (g_ctx[dev]) return g_ctx[dev];
    DevCtx* c = new DevCtx();
    c->device = dev;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) {
        set_error("hipGetDeviceProperties: %s", hipGetErrorString(e));
        delete c;
        return nullptr;
    }
    c->cu_count = prop.multiProcessorCount;
    if ((e = hipMalloc((void**)&c->slots, sizeof(unsigned long long) * 2 * kSlots)) != hipSuccess) {
        set_error("hipMalloc(counter slots): %s", hipGetErrorString(e));
        delete c;
        return nullptr;
    }
    if ((e = hipMemset(c->slots, 0, sizeof(unsigned long long) * 2 * kSlots)) != hipSuccess) {
        set_error("hipMemset(counter slots): %s", hipGetErrorString(e));
        hipFree(c->slots);
        delete c;
        return nullptr;
    }
    g_ctx[dev] = c;
    return c;
}

void* stream_workspace(DevCtx& c, hipStream_t s, size_t bytes, int* err) {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.order_ws.find(s);
    if (it != c.order_ws.end() && it->second.second >= bytes) return it->second.first;
    size_t cap = bytes + bytes / 2;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
        set_error("hipMalloc(workspace of %zu bytes): %s", cap, hipGetErrorString(e));
        *err = RD_ENOMEM;
        return nullptr;
    }
    if (it != c.order_ws.end()) {
        void* old = it->second.first;
        if (c.graph_ws.count(old)) {
            c.retired.push_back(old);
        } else {
            /* only work queued on this stream used it */
            hipStreamSynchronize(s);
            hipFree(old);
        }
        it->second = {p, cap};
    } else {
        c.order_ws[s] = {p, cap};
    }
    return p;
}

void pin_stream_workspace(DevCtx& c, hipStream_t s) {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.order_ws.find(s);
    if (it != c.order_ws.end()) c.graph_ws.insert(it->second.first);
}

/* Below this many cells the claim order is left natural (the sort would cost
 * more than the tail it removes). */
constexpr int64_t kOrderMinCells = 8192;

size_t order_bytes(int64_t n) {
    if (n < kOrderMinCells || n > INT32_MAX) return 0;
    return (((size_t)n * sizeof(int32_t) + 255) & ~(size_t)255) + order_workspace_bytes(n);
}

int enqueue_order(DevCtx& c, Prepared& pr, hipStream_t s, unsigned long long* counters,
                  bool* cleared, void* ws_given) {
    pr.args.order = nullptr;
    if (cleared) *cleared = false;
    if (pr.entry->schedule != RD_PERSISTENT || !pr.order || order_bytes(pr.args.n) == 0)
        return 0;
    /* the 16-lane kernels are registered under m = 16 but serve 5..16:
     * the cost keys use the request's species count */
    order_fn fn = find_order_fn(pr.entry->kind, (int)pr.args.P.m);
    if (!fn) return 0;
    const size_t ordb = ((size_t)pr.args.n * sizeof(int32_t) + 255) & ~(size_t)255;
    int err = 0;
    char* ws = ws_given ? (char*)ws_given : (char*)stream_workspace(c, s, order_bytes(pr.args.n), &err);
    if (!ws) return err ? err : RD_ENOMEM;
    int32_t* order = (int32_t*)ws;
    HIP_TRY(fn(pr.args, ws + ordb, order, counters, s));
    pr.args.order = order;
    if (cleared) *cleared = counters != nullptr;
    return 0;
}

int persistent_grid(const DevCtx& c, const KernelEntry* e, int64_t n) {
    return persistent_grid_cu(c.cu_count, e, n);
}

int persistent_grid_cu(int cu_count, const KernelEntry* e, int64_t n) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, e->func, e->block, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t resident = (int64_t)per_cu * cu_count;
    const int64_t needed = (n + e->cells_per_block - 1) / e->cells_per_block;
    int64_t g = needed < resident ? needed : resident;
    if (g < 1) g = 1;
    return (int)g;
}

/* ---------------------------------------------------------------- models */
static bool all_finite(const double* p, int64_t k) {
    for (int64_t i = 0; i < k; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

/* Bytecode program: check it against the rules of the public header and pack
 * it for the device interpreter: [L, C] as integers in 64-bit slots, the
 * constants, then one slot per instruction holding op | d << 8 | a << 16 |
 * b << 24.  out holds kMaxParamDoubles. */
static bool bytecode_block(const rd_model* md, int32_t m, double* out, size_t* len) {
    const double* p = md->params;
    if (m < 1 || m > RD_MAX_M || md->n_params < 2) return false;
    auto whole = [](double v, double lo, double hi) {
        return std::isfinite(v) && std::floor(v) == v && v >= lo && v <= hi;
    };
    if (!whole(p[0], 1, 4096) || !whole(p[1], 0, RD_BC_REGS)) return false;
    const int L = (int)p[0], C = (int)p[1];
    if (m + C > RD_BC_REGS || md->n_params < 2 + (int64_t)C + 4LL * L) return false;
    if (!all_finite(p + 2, C)) return false;
    auto as_double = [](long long w) {
        double v;
        std::memcpy(&v, &w, sizeof(v));
        return v;
    };
    bool defined[RD_BC_REGS] = {};
    for (int r = 0; r < m + C; ++r) defined[r] = true;
    int out_count[RD_MAX_M] = {};
    size_t k_out = 2 + (size_t)C;
    for (int k = 0; k < L; ++k) {
        const double* ins = p + 2 + C + 4 * k;
        if (!whole(ins[0], RD_BC_ADD, RD_BC_OUT) || !whole(ins[1], 0, RD_BC_REGS - 1) ||
            !whole(ins[2], 0, RD_BC_REGS - 1) || !whole(ins[3], 0, RD_BC_REGS - 1))
            return false;
        const int op = (int)ins[0], d = (int)ins[1], a = (int)ins[2], b = (int)ins[3];
        const bool two = op == RD_BC_ADD || op == RD_BC_SUB || op == RD_BC_MUL ||
                         op == RD_BC_DIV || op == RD_BC_POW;
        if (!defined[a] || (two && !defined[b])) return false;
        if (op == RD_BC_OUT) {
            if (d >= m || out_count[d]++ != 0) return false;
        } else {
            if (d < m + C) return false;
            defined[d] = true;
        }
        out[k_out++] = as_double((long long)(op | (d << 8) | (a << 16) | ((long long)b << 24)));
    }
    for (int i = 0; i < m; ++i)
        if (out_count[i] != 1) return false;
    out[0] = as_double(L);
    out[1] = as_double(C);
    std::memcpy(out + 2, p + 2, sizeof(double) * (size_t)C);
    *len = k_out;
    return true;
}

bool model_block_into(const rd_model* md, int32_t m, double* out, size_t* len) {
    if (!md || md->m != m || !md->params) return false;
    const double* p = md->params;
    auto copy = [&](size_t k) {
        std::memcpy(out, p, sizeof(double) * k);
        *len = k;
        return true;
    };
    switch (md->kind) {
    case RD_OREGONATOR:
        if (m != 3 || md->n_params < 4 || !all_finite(p, 4) || p[0] == 0.0 || p[1] == 0.0) return false;
        /* {eps, mu, f, q} -> {q, f, 1/mu, 1/eps} */
        out[0] = p[3];
        out[1] = p[2];
        out[2] = 1.0 / p[1];
        out[3] = 1.0 / p[0];
        *len = 4;
        return true;
    case RD_ROBERTSON:
        if (m != 3 || md->n_params < 3 || !all_finite(p, 3)) return false;
        return copy(3);
    case RD_NAGUMO:
        if (m != 1 || md->n_params < 1 || !all_finite(p, 1)) return false;
        return copy(1);
    case RD_LINEAR:
        if (m < 1 || m > RD_MAX_M || md->n_params < (int64_t)m * m || !all_finite(p, (int64_t)m * m))
            return false;
        return copy((size_t)m * m);
    case RD_KINETICS:
        if (m < 1 || m > RD_MAX_M || md->n_params < 2LL * m * m || !all_finite(p, 2LL * m * m))
            return false;
        return copy(2 * (size_t)m * m);
    case RD_BYTECODE:
        return bytecode_block(md, m, out, len);
    default:
        return false;
    }
}

bool model_block(const rd_model* md, int32_t m, std::vector<double>& block) {
    block.resize(kMaxParamDoubles);
    size_t len = 0;
    if (!model_block_into(md, m, block.data(), &len)) return false;
    block.resize(len);
    return true;
}

static const double* device_params(DevCtx& c, int kind, int m, const std::vector<double>& block,
                                   int* err) {
    std::vector<double> key;
    key.reserve(block.size() + 2);
    key.push_back((double)kind);
    key.push_back((double)m);
    key.insert(key.end(), block.begin(), block.end());
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.params.find(key);
    if (it != c.params.end()) return it->second;
    double* d = nullptr;
    hipError_t e = hipMalloc((void**)&d, sizeof(double) * (block.size() + 1));
    if (e != hipSuccess) {
        set_error("hipMalloc(params): %s", hipGetErrorString(e));
        *err = RD_ENOMEM;
        return nullptr;
    }
    e = hipMemcpy(d, block.data(), sizeof(double) * block.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error("hipMemcpy(params): %s", hipGetErrorString(e));
        hipFree(d);
        *err = RD_EDEVICE;
        return nullptr;
    }
    c.params.emplace(std::move(key), d);
    return d;
}

/* ---------------------------------------------------------------- tolerances */
void make_step_params(double dt, double rtol, double atol, const rd_options& o, StepParams* P) {
    const double uround = 2.220446049250313e-16;
    double rt = rtol, at = atol;
    if (o.tol_transform) {
        /* the published Radau5 convention: local error test against
         * 0.1 rtol^(2/3), atol scaled by the same factor */
        const double q = atol / rtol;
        rt = 0.1 * std::pow(rtol, 2.0 / 3.0);
        at = rt * q;
    }
    P->dt = dt;
    P->rtol = rt;
    P->atol = at;
    P->newton_tol = std::max(10.0 * uround / rt, std::min(0.03, std::sqrt(rt)));
    P->h0 = o.h0;
    P->h_min = o.h_min > 0.0 ? o.h_min : 1e-14 * dt;
    for (int k = 0; k <= kMaxFacTable; ++k)
        P->fac[k] = 0.9 * (2.0 * o.newton_max + 1.0) / (2.0 * o.newton_max + (double)k);
    P->max_steps = o.max_steps;
    P->kmax = o.newton_max;
    P->fixed_steps = o.fixed_steps;
    P->m = 0;
}

static bool options_valid(const rd_options& o) {
    return (o.precision == RD_FP64 || o.precision == RD_MIXED) &&
           (o.schedule == RD_PERSISTENT || o.schedule == RD_ONE_LAUNCH) && o.max_steps >= 1 &&
           o.newton_max >= 1 && o.newton_max <= 50 && o.fixed_steps >= 0 && o.h0 >= 0.0 &&
           o.h_min >= 0.0 && std::isfinite(o.h0) && std::isfinite(o.h_min) && o.variant >= 0 &&
           (o.order == 0 || o.order == 1) &&
           (o.jacobian == RD_JAC_ANALYTIC || o.jacobian == RD_JAC_FD);
}

int prepare_host(double* states, int64_t n, int32_t m, double dt, double rtol, double atol,
                 const rd_model* model, const rd_options* opts, int32_t* stats, Prepared* out,
                 double* block, size_t* blen) {
    rd_options o;
    rd_default_options(&o);
    if (opts) o = *opts;
    if (n < 0 || m < 1 || m > RD_MAX_M) { set_error("bad n_cells or m"); return RD_EINVAL; }
    if (!std::isfinite(dt) || !(dt > 0.0)) { set_error("dt must be finite and > 0"); return RD_EINVAL; }
    if (!std::isfinite(rtol) || !(rtol > 0.0)) { set_error("rtol must be finite and > 0"); return RD_EINVAL; }
    if (!std::isfinite(atol) || !(atol >= 0.0)) { set_error("atol must be finite and >= 0"); return RD_EINVAL; }
    if (!options_valid(o)) { set_error("invalid rd_options"); return RD_EINVAL; }
    if (!model || model->m != m || !model_block_into(model, m, block, blen)) {
        set_error("invalid model (kind/m/params)");
        return RD_EINVAL;
    }
    if (n > 0 && !states) { set_error("states is null"); return RD_EINVAL; }
    if (o.fixed_steps > 0 && o.precision != RD_FP64) {
        set_error("fixed-step mode is available in FP64 only");
        return RD_EINVAL;
    }
    const int jac = model->kind == RD_BYTECODE ? RD_JAC_FD : o.jacobian;
    const KernelEntry* e = find_kernel(model->kind, m, o.precision, o.schedule, o.fixed_steps > 0,
                                       o.variant, jac);
    if (!e) {
        set_error("no kernel for kind %d, m %d, precision %d, schedule %d, variant %d, jacobian %d",
                  model->kind, m, o.precision, o.schedule, o.variant, jac);
        return RD_EINVAL;
    }
    out->entry = e;
    out->order = o.order;
    make_step_params(dt, rtol, atol, o, &out->args.P);
    out->args.P.m = m;
    out->args.states = states;
    out->args.stats = stats;
    out->args.hcell = o.h_cells;
    out->args.n = n;
    return 0;
}

int prepare(double* states, int64_t n, int32_t m, double dt, double rtol, double atol,
            const rd_model* model, const rd_options* opts, int32_t* stats, Prepared* out) {
    std::vector<double> block(kMaxParamDoubles);
    size_t blen = 0;
    int r = prepare_host(states, n, m, dt, rtol, atol, model, opts, stats, out, block.data(), &blen);
    if (r < 0) return r;
    block.resize(blen);
    if (n == 0) return 0;
    DevCtx* c = current_ctx();
    if (!c) return RD_EDEVICE;
    out->device = c->device;
    int err = 0;
    const double* dp = device_params(*c, model->kind, m, block, &err);
    if (!dp) return err ? err : RD_EDEVICE;
    out->args.params = dp;
    out->grid = out->entry->schedule == RD_PERSISTENT
                    ? persistent_grid(*c, out->entry, n)
                    : (int)((n + out->entry->cells_per_block - 1) / out->entry->cells_per_block);
    return 0;
}

/* ---------------------------------------------------------------- launches */
struct ThreadTiming {
    hipEvent_t a = nullptr, b = nullptr;
    bool valid = false;
    unsigned long long* host = nullptr; /* pinned readback words (2) */
};
static thread_local ThreadTiming g_tt;

static int ensure_thread_objects() {
    if (!g_tt.a) {
        HIP_TRY(hipEventCreate(&g_tt.a));
        HIP_TRY(hipEventCreate(&g_tt.b));
    }
    if (!g_tt.host) HIP_TRY(hipHostMalloc((void**)&g_tt.host, 2 * sizeof(unsigned long long), 0));
    return 0;
}

struct GraphKey {
    hipStream_t stream;
    const KernelEntry* entry;
    double* states;
    int32_t* stats;
    double* hcell;
    const double* params;
    int64_t n;
    int grid;
    StepParams P;
    bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};
struct GraphKeyHash {
    size_t operator()(const GraphKey& k) const {
        const unsigned char* p = (const unsigned char*)&k;
        size_t h = 1469598103934665603ull;
        for (size_t i = 0; i < sizeof(k); ++i) h = (h ^ p[i]) * 1099511628211ull;
        return h;
    }
};
struct GraphVal {
    hipGraphExec_t exec = nullptr;
    unsigned long long* counters = nullptr;
};
static std::mutex g_graph_mu;
static std::unordered_map<GraphKey, GraphVal, GraphKeyHash> g_graphs;

static int launch_prepared(Prepared& pr, hipStream_t s, bool use_graph, unsigned long long** nfail_out) {
    DevCtx* c = current_ctx();
    if (!c) return RD_EDEVICE;
    if (int r = ensure_thread_objects()) return r;
    g_tt.valid = false;
    if (use_graph && s != nullptr) {
        GraphKey key;
        std::memset(&key, 0, sizeof(key));
        key.stream = s;
        key.entry = pr.entry;
        key.states = pr.args.states;
        key.stats = pr.args.stats;
        key.hcell = pr.args.hcell;
        key.params = pr.args.params;
        key.n = pr.args.n;
        key.grid = pr.grid;
        key.P = pr.args.P;
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it == g_graphs.end()) {
            GraphVal v;
            HIP_TRY(hipMalloc((void**)&v.counters, 2 * sizeof(unsigned long long)));
            LaunchArgs a = pr.args;
            a.counter = v.counters;
            a.nfail = v.counters + 1;
            hipGraph_t g = nullptr;
            /* workspace is allocated before the capture starts */
            if (int r = ensure_workspace(pr, s)) {
                hipFree(v.counters);
                return r;
            }
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            bool cleared = false;
            if (int r = enqueue_order(*c, pr, s, v.counters, &cleared)) {
                hipGraph_t dummy = nullptr;
                hipStreamEndCapture(s, &dummy);
                if (dummy) hipGraphDestroy(dummy);
                hipFree(v.counters);
                return r;
            }
            a.order = pr.args.order;
            hipError_t e1 = cleared ? hipSuccess : launch_reset(v.counters, 2, s);
            hipError_t e2 = pr.entry->launch(a, pr.grid, s);
            hipError_t e3 = hipStreamEndCapture(s, &g);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                set_error("graph capture failed: %s / %s / %s", hipGetErrorString(e1),
                          hipGetErrorString(e2), hipGetErrorString(e3));
                if (g) hipGraphDestroy(g);
                hipFree(v.counters);
                return RD_EDEVICE;
            }
            const hipError_t ei = hipGraphInstantiate(&v.exec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            pin_stream_workspace(*c, s);
            if (ei != hipSuccess) {
                set_error("hipGraphInstantiate: %s", hipGetErrorString(ei));
                hipFree(v.counters);
                return RD_EDEVICE;
            }
            it = g_graphs.emplace(key, v).first;
        }
        HIP_TRY(hipEventRecord(g_tt.a, s));
        HIP_TRY(hipGraphLaunch(it->second.exec, s));
        HIP_TRY(hipEventRecord(g_tt.b, s));
        g_tt.valid = true;
        *nfail_out = it->second.counters + 1;
        return 0;
    }
    const unsigned slot = c->next_slot.fetch_add(1) % kSlots;
    unsigned long long* cnt = c->slots + 2 * slot;
    pr.args.counter = cnt;
    pr.args.nfail = cnt + 1;
    bool cleared = false;
    if (int r = enqueue_order(*c, pr, s, cnt, &cleared)) return r;
    if (!cleared) HIP_TRY(launch_reset(cnt, 2, s));
    HIP_TRY(hipEventRecord(g_tt.a, s));
    HIP_TRY(pr.entry->launch(pr.args, pr.grid, s));
    HIP_TRY(hipEventRecord(g_tt.b, s));
    g_tt.valid = true;
    *nfail_out = pr.args.nfail;
    return 0;
}

/* Enqueue a prepared reaction step whose two counters (claim position,
 * failed cells) are `counters`: the claim-order kernels, which also clear
 * them, or a clearing kernel, then the step's kernel.  Nothing is allocated
 * when the stream's claim-order workspace already holds ensure_workspace's
 * size, so it can be recorded into a graph. */
int enqueue_prepared(Prepared& pr, hipStream_t s, unsigned long long* counters) {
    DevCtx* c = current_ctx();
    if (!c) return RD_EDEVICE;
    pr.args.counter = counters;
    pr.args.nfail = counters + 1;
    bool cleared = false;
    if (int r = enqueue_order(*c, pr, s, counters, &cleared)) return r;
    if (!cleared) HIP_TRY(launch_reset(counters, 2, s));
    HIP_TRY(pr.entry->launch(pr.args, pr.grid, s));
    return 0;
}

int ensure_workspace(const Prepared& pr, hipStream_t s) {
    if (pr.entry->schedule != RD_PERSISTENT || !pr.order || order_bytes(pr.args.n) == 0) return 0;
    DevCtx* c = current_ctx();
    if (!c) return RD_EDEVICE;
    int err = 0;
    return stream_workspace(*c, s, order_bytes(pr.args.n), &err) ? 0 : (err ? err : RD_ENOMEM);
}

}  // namespace rd

using namespace rd;

extern "C" {

void rd_default_options(rd_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = RD_FP64;
    o->schedule = RD_PERSISTENT;
    o->tol_transform = 1;
    o->max_steps = 100000;
    o->newton_max = 7;
    o->fixed_steps = 0;
    o->h0 = 0.0;
    o->h_min = 0.0;
    o->variant = 0;
    o->use_graph = 0;
    o->order = 1;
    o->jacobian = RD_JAC_ANALYTIC;
    o->h_cells = nullptr;
}

int64_t rd_reaction_step_ex(double* states, int64_t n_cells, int32_t m, double dt, double rtol,
                            double atol, const rd_model* model, const rd_options* opts,
                            int32_t* stats, void* hip_stream, int32_t async) {
    Prepared pr;
    int r = prepare(states, n_cells, m, dt, rtol, atol, model, opts, stats, &pr);
    if (r < 0) return r;
    if (n_cells == 0) return 0;
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned long long* nfail = nullptr;
    r = launch_prepared(pr, s, opts && opts->use_graph, &nfail);
    if (r < 0) return r;
    if (async) return 0;
    HIP_TRY(hipMemcpyAsync(g_tt.host, nfail, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return (int64_t)*g_tt.host;
}

}  // extern "C"

namespace rd {

/* Enqueue one reaction step and, behind it on the same stream, the copy of
 * its failed-cell count into pinned host word `word` (0 or 1) of this
 * thread; nothing is awaited.  The count is valid once the stream has
 * reached that point (reaction_count). */
int64_t reaction_enqueue(double* states, int64_t n_cells, int32_t m, double dt, double rtol,
                         double atol, const rd_model* model, const rd_options* opts,
                         int32_t* stats, hipStream_t s, int word) {
    Prepared pr;
    int r = prepare(states, n_cells, m, dt, rtol, atol, model, opts, stats, &pr);
    if (r < 0) return r;
    if (int e = ensure_thread_objects()) return e;
    g_tt.host[word] = 0;
    if (n_cells == 0) return 0;
    unsigned long long* nfail = nullptr;
    r = launch_prepared(pr, s, opts && opts->use_graph, &nfail);
    if (r < 0) return r;
    HIP_TRY(hipMemcpyAsync(g_tt.host + word, nfail, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    return 0;
}

int64_t reaction_count(int word) { return (int64_t)g_tt.host[word]; }

}  // namespace rd

extern "C" {

int64_t rd_reaction_step(double* states, int64_t n_cells, int32_t m, double dt, double rtol,
                         double atol, const rd_model* model) {
    return rd_reaction_step_ex(states, n_cells, m, dt, rtol, atol, model, nullptr, nullptr, nullptr, 0);
}

const char* rd_last_error(void) { return g_err; }

double rd_last_kernel_ms(void) {
    if (!g_tt.valid) return -1.0;
    if (hipEventSynchronize(g_tt.b) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_tt.a, g_tt.b) != hipSuccess) return -1.0;
    return (double)ms;
}

int32_t rd_variant_count(int32_t kind, int32_t m, int32_t precision, int32_t schedule) {
    m = registry_m(kind, m);
    int best = 0;
    for (const KernelEntry& e : all_kernels())
        if (e.kind == kind && e.jac == native_jac(kind) && e.m == m && e.precision == precision &&
            e.schedule == schedule && !e.fixed && e.variant > best)
            best = e.variant;
    return best;
}

const char* rd_variant_name(int32_t kind, int32_t m, int32_t precision, int32_t schedule,
                            int32_t variant) {
    const KernelEntry* e =
        find_kernel(kind, m, precision, schedule, 0, variant <= 0 ? 0 : variant, -1);
    return e ? e->name : nullptr;
}

int32_t rd_variant_lanes(int32_t kind, int32_t m, int32_t precision, int32_t schedule,
                         int32_t variant) {
    const KernelEntry* e =
        find_kernel(kind, m, precision, schedule, 0, variant <= 0 ? 0 : variant, -1);
    if (!e) { set_error("no such variant"); return RD_EINVAL; }
    return e->block / e->cells_per_block;
}

int32_t rd_set_default_variant(int32_t kind, int32_t m, int32_t precision, int32_t schedule,
                               int32_t variant) {
    if (variant < 1 || variant > rd_variant_count(kind, m, precision, schedule)) {
        set_error("no variant %d for kind %d m %d precision %d schedule %d", variant, kind, m,
                  precision, schedule);
        return RD_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_variant_mu);
    g_default_variant[{kind, registry_m(kind, m), precision, schedule}] = variant;
    return 0;
}

int32_t rd_persistent_grid(int32_t kind, int32_t m, int32_t precision, int32_t variant,
                           int64_t n_cells) {
    const KernelEntry* e = find_kernel(kind, m, precision, RD_PERSISTENT, 0, variant, -1);
    if (!e) { set_error("no such kernel"); return RD_EINVAL; }
    DevCtx* c = current_ctx();
    if (!c) return RD_EDEVICE;
    return persistent_grid(*c, e, n_cells);
}

}  // extern "C"
