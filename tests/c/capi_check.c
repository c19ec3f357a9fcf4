/*
 * capi_check.c -- the reaction step driven from plain C through the C ABI
 * (include/rd.h), with device memory from the HIP runtime and nothing else:
 * no Python, no torch.
 *
 * Case: the linear model f = K u with K diagonal, whose exact solution over
 * [0, dt] is u_i(dt) = exp(K_ii dt) u_i(0).  The step must return 0 failed
 * cells and every value must lie within the tolerance scale of the exact
 * one; the full entry point with options and counters, an asynchronous call
 * on a created stream, the error returns of invalid calls, and two requests
 * through a serving session are checked too.  Exit status 0 on success, 1 on a failed check, 2 on a HIP error.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "rd.h"

#define HIP_OK(x)                                                        \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));      \
            return 2;                                                    \
        }                                                                \
    } while (0)

static int fails = 0;
static void check(int ok, const char* what) {
    printf("%-60s %s\n", what, ok ? "ok" : "FAILED");
    if (!ok) ++fails;
}

int main(void) {
    enum { N = 4096, M = 2 };
    const double dt = 0.1, rtol = 1e-8, atol = 1e-12;
    const double K[M * M] = {-1.0, 0.0, 0.0, -40.0};
    rd_model model = {RD_LINEAR, M, K, M * M};

    double* h = (double*)malloc(sizeof(double) * M * N);
    double* y = (double*)malloc(sizeof(double) * M * N);
    int32_t* st = (int32_t*)malloc(sizeof(int32_t) * RD_NSTATS * N);
    if (!h || !y || !st) return 2;
    for (int c = 0; c < N; ++c) {
        h[0 * N + c] = 1.0 + (double)c / N;  /* SoA: species-major */
        h[1 * N + c] = 0.5 - 0.25 * (double)c / N;
    }
    double* d = NULL;
    int32_t* dst = NULL;
    HIP_OK(hipMalloc((void**)&d, sizeof(double) * M * N));
    HIP_OK(hipMalloc((void**)&dst, sizeof(int32_t) * RD_NSTATS * N));

    /* 1. simple synchronous form */
    HIP_OK(hipMemcpy(d, h, sizeof(double) * M * N, hipMemcpyHostToDevice));
    int64_t r = rd_reaction_step(d, N, M, dt, rtol, atol, &model);
    check(r == 0, "rd_reaction_step returns 0 failed cells");
    HIP_OK(hipMemcpy(y, d, sizeof(double) * M * N, hipMemcpyDeviceToHost));
    double worst = 0.0;
    for (int i = 0; i < M; ++i)
        for (int c = 0; c < N; ++c) {
            const double ex = exp(K[i * M + i] * dt) * h[i * N + c];
            const double e = fabs(y[i * N + c] - ex) / (atol + rtol * fabs(ex));
            if (e > worst) worst = e;
        }
    printf("  worst error / (atol + rtol |u|) = %.3g\n", worst);
    check(worst <= 100.0, "states match exp(K dt) u0 within the tolerance scale");

    /* 2. full form: options, counters, a stream, asynchronous */
    rd_options o;
    rd_default_options(&o);
    o.schedule = RD_ONE_LAUNCH;
    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));
    HIP_OK(hipMemcpy(d, h, sizeof(double) * M * N, hipMemcpyHostToDevice));
    r = rd_reaction_step_ex(d, N, M, dt, rtol, atol, &model, &o, dst, (void*)s, 1);
    check(r == 0, "rd_reaction_step_ex (async) enqueues");
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(st, dst, sizeof(int32_t) * RD_NSTATS * N, hipMemcpyDeviceToHost));
    int ok_stats = 1;
    for (int c = 0; c < N; ++c) {
        const int32_t status = st[0 * N + c], nstep = st[1 * N + c], nacc = st[2 * N + c],
                      nrej = st[3 * N + c], nfev = st[4 * N + c];
        if (status != 0 || nstep < 1 || nacc < 1 || nacc + nrej > nstep || nfev < 1 + 3 * nacc)
            ok_stats = 0;
    }
    check(ok_stats, "per-cell counters consistent (status 0, nfev >= 1 + 3 naccept)");
    double* y2 = (double*)malloc(sizeof(double) * M * N);
    if (!y2) return 2;
    HIP_OK(hipMemcpy(y2, d, sizeof(double) * M * N, hipMemcpyDeviceToHost));
    int same = 1;
    for (int k = 0; k < M * N; ++k)
        if (y2[k] != y[k]) same = 0;
    check(same, "one-launch schedule gives the persistent schedule's states bitwise");

    /* 3. invalid calls return RD_EINVAL and leave the states untouched */
    rd_model bad = {RD_LINEAR, 3, K, M * M};
    check(rd_reaction_step(d, N, M, dt, rtol, atol, &bad) == RD_EINVAL, "model m mismatch -> RD_EINVAL");
    check(rd_reaction_step(d, N, M, -dt, rtol, atol, &model) == RD_EINVAL, "dt <= 0 -> RD_EINVAL");
    check(rd_reaction_step(NULL, N, M, dt, rtol, atol, &model) == RD_EINVAL, "null states -> RD_EINVAL");
    check(rd_reaction_step(d, 0, M, dt, rtol, atol, &model) == 0, "n_cells == 0 -> 0");
    HIP_OK(hipMemcpy(y2, d, sizeof(double) * M * N, hipMemcpyDeviceToHost));
    same = 1;
    for (int k = 0; k < M * N; ++k)
        if (y2[k] != y[k]) same = 0;
    check(same, "states untouched by the rejected calls");
    check(rd_last_error() != NULL, "rd_last_error available");

    /* 4. the request API: two requests through a session of two streams,
     * each equal to the direct call's result; unknown ids and oversized
     * requests are refused */
    rd_options so;
    rd_default_options(&so);
    so.session_streams = 2;
    rd_session* sess = NULL;
    check(rd_session_create(&sess, 0, (size_t)1 << 22, &so) == 0 && sess != NULL,
          "rd_session_create (4 MiB budget, 2 streams)");
    double* d2 = NULL;
    HIP_OK(hipMalloc((void**)&d2, sizeof(double) * M * N));
    HIP_OK(hipMemcpy(d, h, sizeof(double) * M * N, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d2, h, sizeof(double) * M * N, hipMemcpyHostToDevice));
    uint64_t id1 = 0, id2 = 0;
    int sub1 = rd_submit(sess, d, N, M, dt, rtol, atol, &model, dst, &id1);
    int sub2 = rd_submit_ex(sess, d2, N, M, dt, rtol, atol, &model, NULL, (void*)s, &id2);
    check(sub1 == 0 && sub2 == 0 && id1 != id2, "rd_submit / rd_submit_ex queue two requests");
    rd_request_info info1, info2;
    check(rd_wait(sess, id1, &info1) == 0 && info1.done == 1 && info1.n_failed == 0 &&
              info1.n_cells == N,
          "rd_wait: first request done, no failed cell");
    int pr = 1;
    while (pr == 1) pr = rd_poll(sess, id2, &info2);
    check(pr == 0 && info2.done == 1 && info2.n_failed == 0, "rd_poll: second request done");
    check(info1.t_submit_ns <= info1.t_admit_ns && info1.t_admit_ns <= info1.t_done_ns &&
              info1.kernel_end_ms >= info1.kernel_start_ms && info1.kernel_start_ms >= 0.0,
          "request timestamps ordered");
    check(rd_poll(sess, id1, NULL) == RD_ENOTFOUND, "finished id forgotten -> RD_ENOTFOUND");
    double* y3 = (double*)malloc(sizeof(double) * M * N);
    if (!y3) return 2;
    HIP_OK(hipMemcpy(y3, d, sizeof(double) * M * N, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(y2, d2, sizeof(double) * M * N, hipMemcpyDeviceToHost));
    same = 1;
    for (int k = 0; k < M * N; ++k)
        if (y3[k] != y[k] || y2[k] != y[k]) same = 0;
    check(same, "session results equal the direct call's bitwise");
    uint64_t idb = 0;
    check(rd_submit(sess, d, (int64_t)1 << 22, M, dt, rtol, atol, &model, NULL, &idb) == RD_ETOOBIG,
          "request above the budget -> RD_ETOOBIG");
    check(rd_session_destroy(sess) == 0, "rd_session_destroy");
    HIP_OK(hipFree(d2));
    free(y3);

    HIP_OK(hipStreamDestroy(s));
    HIP_OK(hipFree(d));
    HIP_OK(hipFree(dst));
    free(h);
    free(y);
    free(y2);
    free(st);
    printf("%s (%d failed)\n", fails ? "FAILED" : "all checks passed", fails);
    return fails ? 1 : 0;
}
