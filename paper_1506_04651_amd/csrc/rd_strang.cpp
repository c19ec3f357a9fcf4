/*
 * rd_strang.cpp -- C ABI of the diffusion step and of the Strang splitting
 * step U_{n+1} = R_{dt/2} D_dt R_{dt/2} U_n (Descombes et al., §2.1) on a
 * uniform grid: argument checks, the RKC stage coefficients, workspace, and
 * the sequence of launches on the caller's stream.
 */
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "rd_diffusion.h"
#include "rd_internal.h"

namespace rd {

/* RKC2 with damping 2/13 (Sommeijer, Shampine & Verwer 1997): w0 = 1 +
 * eps/s^2, w1 = T_s'(w0) / T_s''(w0), b_j = T_j''(w0) / T_j'(w0)^2 for j >= 2,
 * b_0 = b_1 = b_2, a_j = 1 - b_j T_j(w0); stage j >= 2 weights mu_j = 2 b_j w0 /
 * b_{j-1}, nu_j = -b_j / b_{j-2}, mut_j = 2 b_j w1 / b_{j-1}, gamt_j = -a_{j-1}
 * mut_j, and mut_1 = b_1 w1.  T_j and its derivatives at w0 come from the
 * three-term recurrence T_{j+1} = 2 x T_j - T_{j-1}. */
static void rkc_weights(int s, double tau, double& mut1tau, std::vector<RkcStage>& st) {
    const double damp = 2.0 / 13.0;
    const double w0 = 1.0 + damp / ((double)s * s);
    std::vector<double> T(s + 1), dT(s + 1), d2T(s + 1);
    T[0] = 1.0; dT[0] = 0.0; d2T[0] = 0.0;
    T[1] = w0;  dT[1] = 1.0; d2T[1] = 0.0;
    for (int j = 1; j < s; ++j) {
        T[j + 1] = 2.0 * w0 * T[j] - T[j - 1];
        dT[j + 1] = 2.0 * T[j] + 2.0 * w0 * dT[j] - dT[j - 1];
        d2T[j + 1] = 4.0 * dT[j] + 2.0 * w0 * d2T[j] - d2T[j - 1];
    }
    const double w1 = dT[s] / d2T[s];
    std::vector<double> b(s + 1), a(s + 1);
    for (int j = 2; j <= s; ++j) b[j] = d2T[j] / (dT[j] * dT[j]);
    b[0] = b[1] = b[2];
    for (int j = 0; j <= s; ++j) a[j] = 1.0 - b[j] * T[j];
    mut1tau = b[1] * w1 * tau;
    st.assign(s + 1, RkcStage{0, 0, 0, 0, 0});
    for (int j = 2; j <= s; ++j) {
        const double mu = 2.0 * b[j] * w0 / b[j - 1];
        const double nu = -b[j] / b[j - 2];
        const double mut = 2.0 * b[j] * w1 / b[j - 1];
        st[j] = RkcStage{1.0 - mu - nu, mu, nu, mut * tau, -a[j - 1] * mut * tau};
    }
}

/* smallest recommended stage count: 1 + floor(sqrt(1 + 1.54 tau rho)), >= 2 */
static int rkc_stage_count(double tau_rho) {
    const int s = 1 + (int)std::sqrt(1.0 + 1.54 * tau_rho);
    return s < 2 ? 2 : s;
}

/* workspace per (device, stream): 4 state-sized vectors and the eps array;
 * calls on one stream run in order, so they can share it */
struct DiffWork {
    double* buf = nullptr;
    size_t cap = 0; /* doubles */
    std::vector<double*> retired;
};
static std::mutex g_dw_mu;
static std::map<std::pair<int, hipStream_t>, DiffWork> g_dw;

static int diff_workspace(int device, hipStream_t s, size_t doubles, double** out) {
    std::lock_guard<std::mutex> lk(g_dw_mu);
    DiffWork& w = g_dw[{device, s}];
    if (w.cap < doubles) {
        double* p = nullptr;
        const size_t cap = doubles + doubles / 4;
        if (hipMalloc((void**)&p, cap * sizeof(double)) != hipSuccess) {
            set_error("hipMalloc(diffusion workspace of %zu doubles) failed", cap);
            return RD_ENOMEM;
        }
        /* an older buffer may still be in use by queued work on some stream */
        if (w.buf) w.retired.push_back(w.buf);
        w.buf = p;
        w.cap = cap;
    }
    *out = w.buf;
    return 0;
}

static bool grid_valid(const rd_grid* g, int32_t m) {
    if (!g || (g->dim != 2 && g->dim != 3) || g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
    if (g->dim == 2 && g->nz != 1) return false;
    if (!(g->h > 0.0) || !std::isfinite(g->h) || !g->diff) return false;
    for (int i = 0; i < m; ++i)
        if (!(g->diff[i] >= 0.0) || !std::isfinite(g->diff[i])) return false;
    return true;
}

/* One diffusion step, validated and with its RKC stages computed. */
struct DiffPlan {
    int dim = 0, stages = 0;
    double mut1tau = 0.0;
    std::vector<RkcStage> st;
    DiffGrid g{};
    size_t vec = 0; /* m * cells */
};

static int64_t diffusion_plan(int32_t m, const rd_grid* grid, double dt, int32_t stages,
                              DiffPlan* p) {
    if (m < 1 || m > RD_MAX_M || !grid_valid(grid, m)) {
        set_error("invalid grid or species count");
        return RD_EINVAL;
    }
    if (!std::isfinite(dt) || !(dt > 0.0) || stages < 0 || stages > 100000) {
        set_error("dt must be finite and > 0, stages in [0, 100000]");
        return RD_EINVAL;
    }
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    double emax = 0.0;
    for (int i = 0; i < m; ++i) emax = std::fmax(emax, grid->diff[i]);
    const double rho = 4.0 * grid->dim * emax / (grid->h * grid->h); /* Gershgorin */
    p->dim = grid->dim;
    p->stages = stages > 0 ? (stages < 2 ? 2 : stages) : rkc_stage_count(dt * rho);
    rkc_weights(p->stages, dt, p->mut1tau, p->st);
    p->g = DiffGrid{grid->nx, grid->ny, grid->nz, n, 1.0 / (grid->h * grid->h)};
    p->vec = (size_t)m * (size_t)n;
    return 0;
}

/* The stage kernels of a planned step; w: 4 vec doubles of workspace. */
static int diffusion_launch(double* states, int32_t m, const DiffPlan& p, const double* eps_dev,
                            double* w, hipStream_t s) {
    hipError_t e = launch_rkc(p.dim, states, states, w, w + p.vec, w + 2 * p.vec, w + 3 * p.vec, m,
                              p.g, eps_dev, p.mut1tau, p.st.data(), p.stages, s);
    if (e != hipSuccess) {
        set_error("diffusion launch: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    return 0;
}

static int64_t diffusion_enqueue(double* states, int32_t m, const rd_grid* grid, double dt,
                                 int32_t stages, hipStream_t s) {
    DiffPlan p;
    if (int64_t r = diffusion_plan(m, grid, dt, stages, &p)) return r;
    if (!states) { set_error("states is null"); return RD_EINVAL; }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("no current device");
        return RD_EDEVICE;
    }
    double* w = nullptr;
    if (int r = diff_workspace(dev, s, 4 * p.vec + 256, &w)) return r;
    double* eps = w + 4 * p.vec;
    if (hipMemcpyAsync(eps, grid->diff, sizeof(double) * m, hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("hipMemcpyAsync(eps) failed");
        return RD_EDEVICE;
    }
    if (int r = diffusion_launch(states, m, p, eps, w, s)) return r;
    return p.stages;
}

/* ---------------------------------------------------------------- graphs */
/* A whole split step R_{dt/2} D_dt R_{dt/2} recorded as one graph: both
 * reaction halves with counters of their own, the failure counts copied to
 * pinned host words, and the diffusion stages with the coefficients in a
 * device buffer of the graph.  Keyed by everything the recorded work
 * depends on; workspaces are allocated before the capture. */
struct StrangGraph {
    hipGraphExec_t exec = nullptr;
    unsigned long long* counters = nullptr; /* 4: claim + failures, per half */
    unsigned long long* host = nullptr;     /* pinned: failures per half */
    double* eps = nullptr;                  /* device copy of the coefficients */
};
static std::mutex g_sg_mu;
static std::map<std::vector<unsigned char>, StrangGraph> g_sg;

template <class T>
static void put(std::vector<unsigned char>& k, const T& v) {
    const unsigned char* b = (const unsigned char*)&v;
    k.insert(k.end(), b, b + sizeof(T));
}

static void free_strang_graph(StrangGraph& g) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.counters) hipFree(g.counters);
    if (g.host) hipHostFree(g.host);
    if (g.eps) hipFree(g.eps);
    g = StrangGraph{};
}

static int64_t strang_graph_step(double* states, int32_t m, const rd_grid* grid, double dt,
                                 double rtol, double atol, const rd_model* model,
                                 const rd_options* opts, int32_t* stats, hipStream_t s) {
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    Prepared p1, p2;
    int r = prepare(states, n, m, 0.5 * dt, rtol, atol, model, opts, stats, &p1);
    if (r < 0) return r;
    r = prepare(states, n, m, 0.5 * dt, rtol, atol, model, opts,
                stats ? stats + (size_t)RD_NSTATS * n : nullptr, &p2);
    if (r < 0) return r;
    DiffPlan dp;
    if (int64_t e = diffusion_plan(m, grid, dt, 0, &dp)) return e;
    if (n == 0) return 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { set_error("no current device"); return RD_EDEVICE; }

    std::vector<unsigned char> key;
    put(key, dev); put(key, s); put(key, states); put(key, stats); put(key, p1.entry);
    put(key, p1.args.params); put(key, p1.args.P); put(key, p1.grid); put(key, p1.order);
    put(key, grid->dim); put(key, grid->nx); put(key, grid->ny); put(key, grid->nz);
    put(key, grid->h); put(key, dt);
    for (int i = 0; i < m; ++i) put(key, grid->diff[i]);

    StrangGraph run;
    {
        std::lock_guard<std::mutex> lk(g_sg_mu);
        auto it = g_sg.find(key);
        if (it == g_sg.end()) {
            StrangGraph g;
            double* w = nullptr;
            if (hipMalloc((void**)&g.counters, 4 * sizeof(unsigned long long)) != hipSuccess ||
                hipHostMalloc((void**)&g.host, 2 * sizeof(unsigned long long), 0) != hipSuccess ||
                hipMalloc((void**)&g.eps, sizeof(double) * m) != hipSuccess ||
                hipMemcpy(g.eps, grid->diff, sizeof(double) * m, hipMemcpyHostToDevice) != hipSuccess) {
                set_error("allocation of the split-step graph failed");
                free_strang_graph(g);
                return RD_ENOMEM;
            }
            if ((r = ensure_workspace(p1, s)) != 0 || (r = diff_workspace(dev, s, 4 * dp.vec + 256, &w)) != 0) {
                free_strang_graph(g);
                return r;
            }
            if (hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal); e != hipSuccess) {
                set_error("hipStreamBeginCapture: %s", hipGetErrorString(e));
                free_strang_graph(g);
                return RD_EDEVICE;
            }
            int rc = enqueue_prepared(p1, s, g.counters);
            if (rc == 0 && hipMemcpyAsync(g.host, g.counters + 1, sizeof(unsigned long long),
                                          hipMemcpyDeviceToHost, s) != hipSuccess)
                rc = RD_EDEVICE;
            if (rc == 0) rc = diffusion_launch(states, m, dp, g.eps, w, s);
            if (rc == 0) rc = enqueue_prepared(p2, s, g.counters + 2);
            if (rc == 0 && hipMemcpyAsync(g.host + 1, g.counters + 3, sizeof(unsigned long long),
                                          hipMemcpyDeviceToHost, s) != hipSuccess)
                rc = RD_EDEVICE;
            hipGraph_t gr = nullptr;
            const hipError_t ee = hipStreamEndCapture(s, &gr);
            if (rc == 0 && ee != hipSuccess) {
                set_error("hipStreamEndCapture: %s", hipGetErrorString(ee));
                rc = RD_EDEVICE;
            }
            if (rc == 0 && hipGraphInstantiate(&g.exec, gr, nullptr, nullptr, 0) != hipSuccess) {
                set_error("hipGraphInstantiate failed");
                rc = RD_EDEVICE;
            }
            if (gr) hipGraphDestroy(gr);
            if (rc != 0) {
                free_strang_graph(g);
                return rc;
            }
            if (DevCtx* c = current_ctx()) pin_stream_workspace(*c, s);
            it = g_sg.emplace(std::move(key), g).first;
        }
        run = it->second; /* entries are never erased: the handles stay valid */
    }
    if (hipError_t e = hipGraphLaunch(run.exec, s); e != hipSuccess) {
        set_error("hipGraphLaunch: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    if (hipError_t e = hipStreamSynchronize(s); e != hipSuccess) {
        set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    return (int64_t)(run.host[0] + run.host[1]);
}

}  // namespace rd

using namespace rd;

extern "C" {

int64_t rd_diffusion_step(double* states, int32_t m, const rd_grid* grid, double dt,
                          int32_t stages, void* hip_stream) {
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t r = diffusion_enqueue(states, m, grid, dt, stages, s);
    if (r < 0) return r;
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("hipStreamSynchronize failed");
        return RD_EDEVICE;
    }
    return r;
}

int64_t rd_strang_step(double* states, int32_t m, const rd_grid* grid, double dt, double rtol,
                       double atol, const rd_model* model, const rd_options* opts,
                       int32_t* stats, void* hip_stream) {
    if (m < 1 || m > RD_MAX_M || !grid_valid(grid, m)) {
        set_error("invalid grid or species count");
        return RD_EINVAL;
    }
    if (!std::isfinite(dt) || !(dt > 0.0)) { set_error("dt must be finite and > 0"); return RD_EINVAL; }
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    if (opts && opts->h_cells) {
        set_error("per-cell warm start is not supported by the Strang driver");
        return RD_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (opts && opts->use_graph && s != nullptr) {
        if (!states && n > 0) { set_error("states is null"); return RD_EINVAL; }
        return strang_graph_step(states, m, grid, dt, rtol, atol, model, opts, stats, s);
    }
    /* R, D, R in stream order with no host wait in between; the two failure
     * counts land in pinned host words and are read after one synchronization */
    const int64_t r1 = reaction_enqueue(states, n, m, 0.5 * dt, rtol, atol, model, opts, stats, s, 0);
    if (r1 < 0) return r1;
    const int64_t sd = diffusion_enqueue(states, m, grid, dt, 0, s);
    if (sd < 0) return sd;
    const int64_t r2 = reaction_enqueue(states, n, m, 0.5 * dt, rtol, atol, model, opts,
                                        stats ? stats + (size_t)RD_NSTATS * n : nullptr, s, 1);
    if (r2 < 0) return r2;
    if (hipError_t e = hipStreamSynchronize(s); e != hipSuccess) {
        set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
        return RD_EDEVICE;
    }
    return reaction_count(0) + reaction_count(1);
}

}  // extern "C"
