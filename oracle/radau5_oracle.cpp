/*
 * radau5_oracle.cpp -- plain, slow, FP64 CPU oracle of the Radau5 reaction
 * substep.
 *
 * TEST INFRASTRUCTURE ONLY: it is loaded by the test-suite, by the smoke check
 * and by the CPU-baseline leg of the benchmark, never by the product path.
 * It shares no code with the GPU library.
 *
 * Source of truth
 *   - Descombes et al., §2.1: Strang splitting U_{n+1} = R_{dt/2} D_dt R_{dt/2}
 *     U_n; in the reaction steps R, every grid point solves its own initial
 *     value problem du/dt = f(u) with Radau5.
 *   - Paper §1 (footnote on Radau5): implicit Runge-Kutta of order five, A- and
 *     L-stable, with time-step adaptation.
 *   - Paper Appendix A: Δt/2 may be split into several sub-steps by the time
 *     stepping, nonlinear systems are solved with a simplified Newton method,
 *     and the minimum work is one sub-step with one Newton iteration.
 *   - Paper §1 (model list): the BZ / Oregonator right-hand side; NAGUMO.
 *   - Hairer & Wanner, Solving ODEs II, §IV.5 (Radau IIA coefficients) and
 *     §IV.8 (simplified Newton on the stage equations, error estimate filtered
 *     by (gamma_hat/h - J)^{-1}, step-size control).  Nothing of the published
 *     Fortran code is used: each step below is written from the mathematics.
 *
 * Deliberately plain: the stage system is solved UNTRANSFORMED, as the
 * 3m x 3m linear system (I - h A (x) J) dZ = -Z + h (A (x) I) F(Z), with a
 * dense Gaussian elimination with partial pivoting.  One cell at a time; cells
 * are shared out to threads by an atomic chunk counter.
 *
 * Pins (tests, CPU): constants against the collocation conditions; the
 * stability function against the (2,3) Pade approximant of exp; order 5;
 * exactness on degree-5 polynomial solutions; the Robertson sum invariant;
 * linear kinetics against the matrix exponential; the Oregonator steady state;
 * tight-tolerance agreement with independent stiff integrators; the error
 * estimate against its definition; model f and J against finite differences.
 * The step-size controller constants and the exact accept/reject sequence are
 * NOT fixed by the paper (it only names Radau5): parity unpinned for the step
 * sequence itself; the results it produces are pinned through accuracy.
 */
#include "rdo.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace {

/* ------------------------------------------------------------------------ */
/* Radau IIA, s = 3 (Hairer & Wanner §IV.5, closed forms of the collocation  */
/* method with the right Radau nodes).                                        */
/* ------------------------------------------------------------------------ */
struct Radau {
    double c[3];
    double A[3][3];
    double gamma_hat; /* real eigenvalue of A^{-1}: root of x^3-9x^2+36x-60 */
    double d[3];      /* embedded estimate weights: d.c = -1, d.c^2 = d.c^3 = 0 */
};

Radau make_radau() {
    const long double r6 = sqrtl(6.0L);
    Radau R;
    R.c[0] = (double)((4.0L - r6) / 10.0L);
    R.c[1] = (double)((4.0L + r6) / 10.0L);
    R.c[2] = 1.0;
    R.A[0][0] = (double)((88.0L - 7.0L * r6) / 360.0L);
    R.A[0][1] = (double)((296.0L - 169.0L * r6) / 1800.0L);
    R.A[0][2] = (double)((-2.0L + 3.0L * r6) / 225.0L);
    R.A[1][0] = (double)((296.0L + 169.0L * r6) / 1800.0L);
    R.A[1][1] = (double)((88.0L + 7.0L * r6) / 360.0L);
    R.A[1][2] = (double)((-2.0L - 3.0L * r6) / 225.0L);
    R.A[2][0] = (double)((16.0L - r6) / 36.0L);
    R.A[2][1] = (double)((16.0L + r6) / 36.0L);
    R.A[2][2] = (double)(1.0L / 9.0L);
    const long double c13 = cbrtl(3.0L);
    R.gamma_hat = (double)(3.0L + c13 * c13 - c13);
    R.d[0] = (double)(-(13.0L + 7.0L * r6) / 3.0L);
    R.d[1] = (double)((-13.0L + 7.0L * r6) / 3.0L);
    R.d[2] = (double)(-1.0L / 3.0L);
    return R;
}

const Radau RK = make_radau();
const double UROUND = 2.220446049250313e-16; /* 2^-52 */

/* ------------------------------------------------------------------------ */
/* Models                                                                     */
/* ------------------------------------------------------------------------ */
struct Model {
    int kind;
    int m;
    std::vector<double> p;
    bool fd = false; /* Jacobian by forward differences */

    /* bytecode model: an interpreter of the documented register program
     * (rdo.h), one instruction at a time */
    void run_bytecode(const double* y, double* out) const {
        double r[RDO_BC_REGS];
        const int L = (int)p[0], C = (int)p[1];
        for (int i = 0; i < m; ++i) r[i] = y[i];
        for (int c = 0; c < C; ++c) r[m + c] = p[2 + c];
        for (int k = 0; k < L; ++k) {
            const double* ins = &p[2 + C + 4 * k];
            const int op = (int)ins[0], d = (int)ins[1], a = (int)ins[2], b = (int)ins[3];
            switch (op) {
            case RDO_BC_ADD: r[d] = r[a] + r[b]; break;
            case RDO_BC_SUB: r[d] = r[a] - r[b]; break;
            case RDO_BC_MUL: r[d] = r[a] * r[b]; break;
            case RDO_BC_DIV: r[d] = r[a] / r[b]; break;
            case RDO_BC_NEG: r[d] = -r[a]; break;
            case RDO_BC_EXP: r[d] = std::exp(r[a]); break;
            case RDO_BC_LOG: r[d] = std::log(r[a]); break;
            case RDO_BC_POW: r[d] = std::pow(r[a], r[b]); break;
            case RDO_BC_OUT: out[d] = r[a]; break;
            }
        }
    }

    /* Forward-difference Jacobian at y, given fy = f(y):
     * column j = (f(y + d_j e_j) - f(y)) / d_j, d_j = sqrt(u max(1e-5, |y_j|)) */
    void jac_fd(const double* y, const double* fy, double* J) const {
        std::vector<double> yp(y, y + m), fp(m);
        for (int j = 0; j < m; ++j) {
            const double dj = std::sqrt(2.220446049250313e-16 * std::max(1e-5, std::fabs(y[j])));
            yp[j] = y[j] + dj;
            f(yp.data(), fp.data());
            for (int i = 0; i < m; ++i) J[i * m + j] = (fp[i] - fy[i]) / dj;
            yp[j] = y[j];
        }
    }

    /* right-hand side f(y) */
    void f(const double* y, double* out) const {
        switch (kind) {
        case RDO_OREGONATOR: {
            /* paper §1, BZ: f1 = (1/mu)(-q a - a b + f c),
             * f2 = (1/eps)(q a - a b + b (1 - b)), f3 = b - c */
            const double eps = p[0], mu = p[1], ff = p[2], q = p[3];
            const double a = y[0], b = y[1], c = y[2];
            out[0] = (-q * a - a * b + ff * c) / mu;
            out[1] = (q * a - a * b + b * (1.0 - b)) / eps;
            out[2] = b - c;
            break;
        }
        case RDO_KINETICS: {
            /* f_i = sum_j K_ij u_j - u_i sum_k G_ik u_k */
            const double* K = p.data();
            const double* G = p.data() + (size_t)m * m;
            for (int i = 0; i < m; ++i) {
                double lin = 0.0, loss = 0.0;
                for (int j = 0; j < m; ++j) {
                    lin += K[i * m + j] * y[j];
                    loss += G[i * m + j] * y[j];
                }
                out[i] = lin - y[i] * loss;
            }
            break;
        }
        case RDO_NAGUMO: {
            /* paper §1, NAGUMO: f = k u^2 (1 - u) */
            const double k = p[0];
            out[0] = k * y[0] * y[0] * (1.0 - y[0]);
            break;
        }
        case RDO_LINEAR: {
            const double* K = p.data();
            for (int i = 0; i < m; ++i) {
                double s = 0.0;
                for (int j = 0; j < m; ++j) s += K[i * m + j] * y[j];
                out[i] = s;
            }
            break;
        }
        case RDO_BYTECODE:
            run_bytecode(y, out);
            break;
        case RDO_ROBERTSON: {
            const double k1 = p[0], k2 = p[1], k3 = p[2];
            out[0] = -k1 * y[0] + k2 * y[1] * y[2];
            out[1] = k1 * y[0] - k2 * y[1] * y[2] - k3 * y[1] * y[1];
            out[2] = k3 * y[1] * y[1];
            break;
        }
        }
    }

    /* analytic Jacobian, J[i*m+j] = d f_i / d y_j */
    void jac(const double* y, double* J) const {
        switch (kind) {
        case RDO_OREGONATOR: {
            const double eps = p[0], mu = p[1], ff = p[2], q = p[3];
            const double a = y[0], b = y[1];
            J[0] = (-q - b) / mu; J[1] = -a / mu;                J[2] = ff / mu;
            J[3] = (q - b) / eps; J[4] = (1.0 - a - 2.0 * b) / eps; J[5] = 0.0;
            J[6] = 0.0;           J[7] = 1.0;                    J[8] = -1.0;
            break;
        }
        case RDO_KINETICS: {
            const double* K = p.data();
            const double* G = p.data() + (size_t)m * m;
            for (int i = 0; i < m; ++i) {
                double gu = 0.0;
                for (int k = 0; k < m; ++k) gu += G[i * m + k] * y[k];
                for (int j = 0; j < m; ++j)
                    J[i * m + j] = K[i * m + j] - y[i] * G[i * m + j]
                                   - (i == j ? gu : 0.0);
            }
            break;
        }
        case RDO_NAGUMO: {
            const double k = p[0];
            J[0] = k * (2.0 * y[0] - 3.0 * y[0] * y[0]);
            break;
        }
        case RDO_LINEAR:
            for (int i = 0; i < m * m; ++i) J[i] = p[i];
            break;
        case RDO_ROBERTSON: {
            const double k1 = p[0], k2 = p[1], k3 = p[2];
            J[0] = -k1; J[1] = k2 * y[2];                      J[2] = k2 * y[1];
            J[3] = k1;  J[4] = -k2 * y[2] - 2.0 * k3 * y[1];   J[5] = -k2 * y[1];
            J[6] = 0.0; J[7] = 2.0 * k3 * y[1];                J[8] = 0.0;
            break;
        }
        }
    }
};

/* Validation of a bytecode program against the rules stated in rdo.h. */
bool bytecode_from_abi(const rdo_model* mm, Model& out) {
    const int m = mm->m;
    if (m < 1 || m > 16 || !mm->params || mm->n_params < 2) return false;
    const double* p = mm->params;
    auto is_int = [](double v, double lo, double hi) {
        return std::isfinite(v) && v == std::floor(v) && v >= lo && v <= hi;
    };
    if (!is_int(p[0], 1, 4096) || !is_int(p[1], 0, RDO_BC_REGS)) return false;
    const int L = (int)p[0], C = (int)p[1];
    if (m + C > RDO_BC_REGS) return false;
    const int64_t need = 2 + (int64_t)C + 4LL * L;
    if (mm->n_params < need) return false;
    for (int c = 0; c < C; ++c)
        if (!std::isfinite(p[2 + c])) return false;
    bool written[RDO_BC_REGS] = {};
    for (int i = 0; i < m + C; ++i) written[i] = true;
    std::vector<int> outs(m, 0);
    for (int k = 0; k < L; ++k) {
        const double* ins = p + 2 + C + 4 * k;
        if (!is_int(ins[0], RDO_BC_ADD, RDO_BC_OUT)) return false;
        for (int f = 1; f < 4; ++f)
            if (!is_int(ins[f], 0, RDO_BC_REGS - 1)) return false;
        const int op = (int)ins[0], d = (int)ins[1], a = (int)ins[2], b = (int)ins[3];
        const bool binary = op == RDO_BC_ADD || op == RDO_BC_SUB || op == RDO_BC_MUL ||
                            op == RDO_BC_DIV || op == RDO_BC_POW;
        if (!written[a] || (binary && !written[b])) return false;
        if (op == RDO_BC_OUT) {
            if (d >= m || outs[d]++) return false;
        } else {
            if (d < m + C) return false;
            written[d] = true;
        }
    }
    for (int i = 0; i < m; ++i)
        if (outs[i] != 1) return false;
    out.kind = RDO_BYTECODE;
    out.m = m;
    out.p.assign(p, p + need);
    out.fd = true;
    return true;
}

bool model_from_abi(const rdo_model* mm, Model& out) {
    if (!mm || mm->m < 1) return false;
    const int m = mm->m;
    int64_t need = 0;
    switch (mm->kind) {
    case RDO_OREGONATOR: if (m != 3) return false; need = 4; break;
    case RDO_KINETICS:   need = 2LL * m * m; break;
    case RDO_NAGUMO:     if (m != 1) return false; need = 1; break;
    case RDO_LINEAR:     need = (int64_t)m * m; break;
    case RDO_ROBERTSON:  if (m != 3) return false; need = 3; break;
    case RDO_BYTECODE:   return bytecode_from_abi(mm, out);
    default: return false;
    }
    if (mm->n_params < need || !mm->params) return false;
    out.kind = mm->kind;
    out.m = m;
    out.p.assign(mm->params, mm->params + need);
    for (double v : out.p)
        if (!std::isfinite(v)) return false;
    return true;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (Gaussian elimination), and its solve.      */
/* Returns false when a pivot is exactly zero.                                */
/* ------------------------------------------------------------------------ */
bool lu_factor(std::vector<double>& a, std::vector<int>& piv, int n) {
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::fabs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            const double v = std::fabs(a[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (a[(size_t)p * n + k] == 0.0) return false;
        if (p != k)
            for (int j = 0; j < n; ++j)
                std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
        const double pk = a[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            const double l = a[(size_t)i * n + k] / pk;
            a[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j)
                a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    return true;
}

void lu_solve(const std::vector<double>& lu, const std::vector<int>& piv,
              int n, double* b) {
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = 1; i < n; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= lu[(size_t)i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= lu[(size_t)i * n + j] * b[j];
        b[i] = s / lu[(size_t)i * n + i];
    }
}

bool all_finite(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

/* ------------------------------------------------------------------------ */
/* Per-call constants                                                         */
/* ------------------------------------------------------------------------ */
struct Tols {
    double rtol, atol;   /* after the optional transformation */
    double newton_tol;   /* kappa*Tol of the Newton stopping test */
};

Tols make_tols(double rtol, double atol, int transform) {
    Tols t;
    if (transform) {
        /* published Radau5 convention: the code is asked for rtol, and runs
         * its local error test against 0.1 rtol^(2/3) (atol scaled alike) */
        const double q = atol / rtol;
        t.rtol = 0.1 * std::pow(rtol, 2.0 / 3.0);
        t.atol = t.rtol * q;
    } else {
        t.rtol = rtol;
        t.atol = atol;
    }
    t.newton_tol = std::max(10.0 * UROUND / t.rtol,
                            std::min(0.03, std::sqrt(t.rtol)));
    return t;
}

struct Opts {
    int max_steps = 100000;
    int kmax = 7;
    int fixed_steps = 0;
    double h0 = 0.0;
    double h_min = 0.0;
    int tol_transform = 1;
    int jacobian = 0;
    double* h_cells = nullptr;
};

/* ------------------------------------------------------------------------ */
/* The integrator for one cell                                                */
/* ------------------------------------------------------------------------ */
struct Stats {
    int status = 0, nstep = 0, naccept = 0, nreject = 0, nfev = 0, njac = 0,
        ndec = 0, nsol = 0, nnewt = 0;
};

class Cell {
public:
    Cell(const Model& md, const Tols& tl, const Opts& op)
        : M(md), T(tl), O(op), m(md.m), n3(3 * md.m),
          J(m * m), E1(m * m), Mbig((size_t)n3 * n3), f0(m), y1(m), sc(m),
          Z(n3), dZ(n3), F(n3), zold(n3), tmp(m), e(m), rhs(n3) {}

    /* Build M = I - h (A (x) J) and E1 = (gamma_hat/h) I - J, factor both. */
    bool factor(double h) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int r = 0; r < m; ++r)
                    for (int s = 0; s < m; ++s) {
                        const size_t row = (size_t)i * m + r;
                        const size_t col = (size_t)j * m + s;
                        double v = -h * RK.A[i][j] * J[r * m + s];
                        if (row == col) v += 1.0;
                        Mbig[row * n3 + col] = v;
                    }
        for (int r = 0; r < m; ++r)
            for (int s = 0; s < m; ++s)
                E1[r * m + s] = (r == s ? RK.gamma_hat / h : 0.0) - J[r * m + s];
        const bool ok1 = lu_factor(Mbig, pivM, n3);
        const bool ok2 = lu_factor(E1, pivE, m);
        return ok1 && ok2;
    }

    /* Start values of the stage increments: zero, or the collocation cubic
     * of the last accepted step continued to the new stage points. */
    void start_values(double h, bool have_old, double h_old) {
        if (!have_old) {
            std::fill(Z.begin(), Z.end(), 0.0);
            return;
        }
        /* Cubic q(s), s measured in units of h_old from the current t:
         * q(-1) = -z3_old, q(c_i - 1) = z_i_old - z3_old (i = 1, 2), q(0) = 0.
         * Lagrange form over the nodes s_k. */
        const double sn[4] = {-1.0, RK.c[0] - 1.0, RK.c[1] - 1.0, 0.0};
        for (int i = 0; i < 3; ++i) {
            const double s = RK.c[i] * h / h_old;
            double w[4];
            for (int k = 0; k < 4; ++k) {
                double l = 1.0;
                for (int j = 0; j < 4; ++j)
                    if (j != k) l *= (s - sn[j]) / (sn[k] - sn[j]);
                w[k] = l;
            }
            for (int r = 0; r < m; ++r) {
                const double z3 = zold[2 * m + r];
                const double v0 = -z3;
                const double v1 = zold[0 * m + r] - z3;
                const double v2 = zold[1 * m + r] - z3;
                Z[(size_t)i * m + r] = w[0] * v0 + w[1] * v1 + w[2] * v2; /* v3 = 0 */
            }
        }
    }

    /* Simplified Newton on the stage equations Z = h (A (x) I) F(y0 + Z).
     * Returns true on convergence; k_used, theta_out filled. */
    bool newton(const double* y0, double h, double& eta, int& k_used,
                double& theta_out, Stats& st) {
        double nprev = 0.0;
        theta_out = 0.0;
        for (int k = 1; k <= O.kmax; ++k) {
            k_used = k;
            st.nnewt++;
            for (int i = 0; i < 3; ++i) {
                for (int r = 0; r < m; ++r) tmp[r] = y0[r] + Z[(size_t)i * m + r];
                M.f(tmp.data(), &F[(size_t)i * m]);
            }
            st.nfev += 3;
            for (int i = 0; i < 3; ++i)
                for (int r = 0; r < m; ++r) {
                    double s = 0.0;
                    for (int j = 0; j < 3; ++j) s += RK.A[i][j] * F[(size_t)j * m + r];
                    rhs[(size_t)i * m + r] = -Z[(size_t)i * m + r] + h * s;
                }
            lu_solve(Mbig, pivM, n3, rhs.data());
            st.nsol++;
            double acc = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int r = 0; r < m; ++r) {
                    const double dz = rhs[(size_t)i * m + r];
                    Z[(size_t)i * m + r] += dz;
                    const double q = dz / sc[r];
                    acc += q * q;
                }
            const double nk = std::sqrt(acc / (double)n3);
            if (!std::isfinite(nk)) return false;
            if (k >= 2) {
                const double theta = nk / nprev;
                theta_out = theta;
                if (theta >= 0.99) return false;
                eta = theta / (1.0 - theta);
                double tp = 1.0;
                for (int j = 0; j < O.kmax - k; ++j) tp *= theta;
                if (tp / (1.0 - theta) * nk > T.newton_tol) return false;
            }
            if (eta * nk <= T.newton_tol) return true;
            nprev = nk;
        }
        return false;
    }

    /* Error estimate: e = E1^{-1} [f(y_base) + (d1 z1 + d2 z2 + d3 z3)/h],
     * returned as the RMS of e/sc; e is left in this->e. */
    double estimate(const double* fbase, double h, Stats& st) {
        for (int r = 0; r < m; ++r) {
            const double dz = RK.d[0] * Z[r] + RK.d[1] * Z[m + r] + RK.d[2] * Z[2 * m + r];
            e[r] = fbase[r] + dz / h;
        }
        lu_solve(E1, pivE, m, e.data());
        st.nsol++;
        double acc = 0.0;
        for (int r = 0; r < m; ++r) {
            const double q = e[r] / sc[r];
            acc += q * q;
        }
        return std::sqrt(acc / (double)m);
    }

    double full_estimate(const double* y0, double h, bool second_allowed, Stats& st) {
        double err = estimate(f0.data(), h, st);
        if (err >= 1.0 && second_allowed) {
            for (int r = 0; r < m; ++r) tmp[r] = y0[r] + e[r];
            std::vector<double> fe(m);
            M.f(tmp.data(), fe.data());
            st.nfev++;
            err = estimate(fe.data(), h, st);
        }
        return err;
    }

    /* J at y (f0 = f(y)): analytic, or forward differences (m more f
     * evaluations) */
    void jacobian(const double* y, Stats& st) {
        if (M.fd) {
            M.jac_fd(y, f0.data(), J.data());
            st.nfev += m;
        } else {
            M.jac(y, J.data());
        }
        st.njac++;
    }

    void scale(const double* y0) {
        for (int r = 0; r < m; ++r) sc[r] = T.atol + T.rtol * std::fabs(y0[r]);
    }

    /* Adaptive integration of one cell over [0, dt]; y is updated in place.
     * h_io: null, or the cell's warm-start step size (in: used as the first
     * trial step when > 0; out: see rdo.h). */
    void integrate(double* y, double dt, Stats& st, double* h_io = nullptr) {
        double h_pre = 0.0;
        integrate_(y, dt, st, h_pre, h_io && *h_io > 0.0 ? *h_io : 0.0);
        if (h_io) *h_io = h_pre;
    }

    void integrate_(double* y, double dt, Stats& st, double& h_pre, double h_in) {
        const double h_min = O.h_min > 0.0 ? O.h_min : 1e-14 * dt;
        M.f(y, f0.data());
        st.nfev++;
        if (!all_finite(y, m) || !all_finite(f0.data(), m)) {
            st.status = RDO_NONFINITE;
            return;
        }
        if (O.fixed_steps > 0) {
            h_pre = dt / O.fixed_steps;
            fixed(y, dt, st);
            return;
        }
        double t = 0.0;
        double h = std::min(h_in > 0.0 ? h_in : (O.h0 > 0.0 ? O.h0 : dt), dt);
        h_pre = h;
        bool first = true, reject = false;
        bool J_stale = true;   /* J must be recomputed before the next attempt */
        bool J_at_y0 = false;  /* J was evaluated at the current y0 */
        bool have_lu = false;
        double h_lu = 0.0;
        double eta = 1.0;
        bool have_old = false;
        double h_old = 0.0;
        bool have_acc = false;
        double h_acc = 0.0, err_acc = 0.0;
        int n_singular = 0;

        while (t < dt) {
            h_pre = h;
            if (st.nstep >= O.max_steps) { st.status = RDO_MAXSTEPS; return; }
            if (h < h_min) { st.status = RDO_H_TOO_SMALL; return; }
            bool last = false;
            if (t + 1.0001 * h >= dt) { h = dt - t; last = true; }
            scale(y);
            if (J_stale) {
                jacobian(y, st);
                J_stale = false;
                J_at_y0 = true;
                have_lu = false;
            }
            if (!have_lu || h != h_lu) {
                st.ndec++;
                if (!factor(h)) {
                    have_lu = false;
                    if (++n_singular >= 5) { st.status = RDO_SINGULAR; return; }
                    h *= 0.5;
                    continue;
                }
                n_singular = 0;
                have_lu = true;
                h_lu = h;
            }
            start_values(h, have_old, h_old);
            int k_used = 0;
            double theta = 0.0;
            if (!newton(y, h, eta, k_used, theta, st)) {
                st.nstep++;
                st.nreject++;
                h *= 0.5;
                reject = true;
                if (!J_at_y0) J_stale = true;
                continue;
            }
            for (int r = 0; r < m; ++r) y1[r] = y[r] + Z[(size_t)2 * m + r];
            const double err = full_estimate(y, h, first || reject, st);
            if (!std::isfinite(err)) { st.status = RDO_NONFINITE; return; }
            st.nstep++;

            const double fac = 0.9 * (2.0 * O.kmax + 1.0) / (2.0 * O.kmax + k_used);
            const double ratio = (err == 0.0)
                ? 8.0 : std::min(8.0, std::max(0.2, fac / std::sqrt(std::sqrt(err))));
            double h_new = h * ratio;

            if (err < 1.0) {
                /* predictive (Gustafsson) controller after the first accepted step */
                if (have_acc) {
                    const double r2 = (err == 0.0)
                        ? 8.0
                        : std::min(8.0, std::max(0.2, fac * (h / h_acc) *
                              std::sqrt(std::sqrt(err_acc)) / std::sqrt(err)));
                    h_new = std::min(h_new, h * r2);
                }
                std::vector<double> f1(m);
                M.f(y1.data(), f1.data());
                st.nfev++;
                if (!all_finite(y1.data(), m) || !all_finite(f1.data(), m)) {
                    st.status = RDO_NONFINITE;
                    return;
                }
                have_acc = true;
                h_acc = h;
                err_acc = std::max(err, 1e-2);
                for (int r = 0; r < m; ++r) { y[r] = y1[r]; f0[r] = f1[r]; }
                t = last ? dt : t + h;
                zold = Z;
                h_old = h;
                have_old = true;
                eta = std::pow(std::max(eta, UROUND), 0.8);
                st.naccept++;
                if (reject) h_new = std::min(h_new, h);
                first = false;
                reject = false;
                J_stale = !(k_used == 1 || theta <= 1e-3);
                J_at_y0 = false;
                if (!J_stale) {
                    const double q = h_new / h;
                    if (q >= 1.0 && q <= 1.2) h_new = h;
                }
                h = std::min(h_new, dt - t);
            } else {
                st.nreject++;
                h = first ? 0.1 * h : h_new;
                reject = true;
            }
        }
    }

    /* N equal steps, every step accepted, no error control (test mode). */
    void fixed(double* y, double dt, Stats& st) {
        const int N = O.fixed_steps;
        const double h = dt / N;
        double eta = 1.0;
        bool have_old = false;
        for (int s = 0; s < N; ++s) {
            scale(y);
            jacobian(y, st);
            st.ndec++;
            if (!factor(h)) { st.status = RDO_SINGULAR; return; }
            start_values(h, have_old, h);
            int k_used = 0;
            double theta = 0.0;
            if (!newton(y, h, eta, k_used, theta, st)) {
                st.status = RDO_NEWTON_FAIL;
                return;
            }
            st.nstep++;
            st.naccept++;
            for (int r = 0; r < m; ++r) y[r] += Z[(size_t)2 * m + r];
            M.f(y, f0.data());
            st.nfev++;
            if (!all_finite(y, m)) { st.status = RDO_NONFINITE; return; }
            zold = Z;
            have_old = true;
            eta = std::pow(std::max(eta, UROUND), 0.8);
        }
    }

    const Model& M;
    const Tols& T;
    const Opts& O;
    const int m, n3;
    std::vector<double> J, E1, Mbig, f0, y1, sc, Z, dZ, F, zold, tmp, e, rhs;
    std::vector<int> pivM, pivE;
};

bool options_from_abi(const rdo_options* o, Opts& out) {
    if (!o) return true;
    out.tol_transform = o->tol_transform;
    out.max_steps = o->max_steps;
    out.kmax = o->newton_max;
    out.fixed_steps = o->fixed_steps;
    out.h0 = o->h0;
    out.h_min = o->h_min;
    out.jacobian = o->jacobian;
    out.h_cells = o->h_cells;
    if (out.max_steps < 1 || out.kmax < 1 || out.kmax > 50 || out.fixed_steps < 0)
        return false;
    if (out.jacobian != 0 && out.jacobian != 1) return false;
    if (!(out.h0 >= 0.0) || !(out.h_min >= 0.0)) return false;
    return true;
}

} // namespace

extern "C" int64_t rdo_reaction_step(double* states, int64_t n, int32_t m,
                                     double dt, double rtol, double atol,
                                     const rdo_model* model,
                                     const rdo_options* opts, int32_t* stats,
                                     int32_t nthreads) {
    if (n < 0 || m < 1 || !model || model->m != m) return RDO_EINVAL;
    if (!std::isfinite(dt) || !(dt > 0.0)) return RDO_EINVAL;
    if (!std::isfinite(rtol) || !(rtol > 0.0)) return RDO_EINVAL;
    if (!std::isfinite(atol) || !(atol >= 0.0)) return RDO_EINVAL;
    Model md;
    if (!model_from_abi(model, md)) return RDO_EINVAL;
    Opts op;
    if (!options_from_abi(opts, op)) return RDO_EINVAL;
    if (op.jacobian) md.fd = true;
    if (n == 0) return 0;
    if (!states) return RDO_EINVAL;
    const Tols tl = make_tols(rtol, atol, op.tol_transform);

    int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if ((int64_t)nt > n) nt = (int)n;
    std::atomic<int64_t> next(0);
    std::atomic<int64_t> failed(0);
    const int64_t chunk = 16;

    auto worker = [&]() {
        Cell cell(md, tl, op);
        std::vector<double> y(m);
        int64_t my_failed = 0;
        for (;;) {
            const int64_t start = next.fetch_add(chunk);
            if (start >= n) break;
            const int64_t end = std::min(n, start + chunk);
            for (int64_t c = start; c < end; ++c) {
                for (int r = 0; r < m; ++r) y[r] = states[(size_t)r * n + c];
                Stats st;
                cell.integrate(y.data(), dt, st, op.h_cells ? op.h_cells + c : nullptr);
                for (int r = 0; r < m; ++r) states[(size_t)r * n + c] = y[r];
                if (st.status != 0) ++my_failed;
                if (stats) {
                    const int v[RDO_NSTATS] = {st.status, st.nstep, st.naccept,
                                               st.nreject, st.nfev, st.njac,
                                               st.ndec, st.nsol, st.nnewt};
                    for (int k = 0; k < RDO_NSTATS; ++k) stats[(size_t)k * n + c] = v[k];
                }
            }
        }
        failed.fetch_add(my_failed);
    };
    if (nt == 1) {
        worker();
    } else {
        std::vector<std::thread> pool;
        pool.reserve(nt);
        for (int i = 0; i < nt; ++i) pool.emplace_back(worker);
        for (auto& th : pool) th.join();
    }
    return failed.load();
}

extern "C" int32_t rdo_single_step(const double* y0, int32_t m, double h,
                                   double rtol, double atol,
                                   int32_t tol_transform, int32_t newton_max,
                                   const rdo_model* model, double* y1,
                                   double* err, int32_t* info) {
    if (!y0 || !y1 || !err || !info || !model || model->m != m || m < 1)
        return RDO_EINVAL;
    if (!(h > 0.0) || !(rtol > 0.0) || !(atol >= 0.0) || newton_max < 1)
        return RDO_EINVAL;
    Model md;
    if (!model_from_abi(model, md)) return RDO_EINVAL;
    Opts op;
    op.kmax = newton_max;
    op.tol_transform = tol_transform;
    const Tols tl = make_tols(rtol, atol, tol_transform);
    Cell cell(md, tl, op);
    Stats st;
    std::vector<double> y(y0, y0 + m);
    md.f(y.data(), cell.f0.data());
    cell.scale(y.data());
    cell.jacobian(y.data(), st);
    if (!cell.factor(h)) return RDO_EINVAL;
    cell.start_values(h, false, h);
    double eta = 1.0, theta = 0.0;
    int k_used = 0;
    const bool ok = cell.newton(y.data(), h, eta, k_used, theta, st);
    for (int r = 0; r < m; ++r) y1[r] = y[r] + cell.Z[(size_t)2 * m + r];
    err[0] = cell.estimate(cell.f0.data(), h, st);
    std::vector<double> tmp(m), fe(m);
    for (int r = 0; r < m; ++r) tmp[r] = y[r] + cell.e[r];
    md.f(tmp.data(), fe.data());
    err[1] = cell.estimate(fe.data(), h, st);
    info[0] = k_used;
    info[1] = ok ? 0 : 1;
    return 0;
}

extern "C" int32_t rdo_start_values(const double* zold, int32_t m, double h,
                                    double h_old, double* z) {
    if (!zold || !z || m < 1 || !(h > 0.0) || !(h_old > 0.0)) return RDO_EINVAL;
    Model md;
    md.kind = RDO_LINEAR;
    md.m = m;
    md.p.assign((size_t)m * m, 0.0);
    const Tols tl = make_tols(1e-6, 1e-6, 1);
    Opts op;
    Cell cell(md, tl, op);
    std::copy(zold, zold + 3 * m, cell.zold.begin());
    cell.start_values(h, true, h_old);
    std::copy(cell.Z.begin(), cell.Z.end(), z);
    return 0;
}

extern "C" int32_t rdo_model_eval(const rdo_model* model, const double* y,
                                  double* f, double* J) {
    Model md;
    if (!model_from_abi(model, md) || !y) return RDO_EINVAL;
    if (f) md.f(y, f);
    if (J) {
        if (md.fd) {
            std::vector<double> fy(md.m);
            md.f(y, fy.data());
            md.jac_fd(y, fy.data(), J);
        } else {
            md.jac(y, J);
        }
    }
    return 0;
}

extern "C" void rdo_constants(double* out) {
    out[0] = RK.c[0]; out[1] = RK.c[1]; out[2] = RK.c[2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[3 + 3 * i + j] = RK.A[i][j];
    out[12] = RK.gamma_hat;
    out[13] = RK.d[0];
    out[14] = RK.d[1];
    out[15] = RK.d[2];
}
