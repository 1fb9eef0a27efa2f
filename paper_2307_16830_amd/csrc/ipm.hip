// Condensed-space interior-point method, Algorithm 1 of the paper, with the
// iterate, slacks, multipliers, derivatives and the Cholesky factor resident
// in HBM.  The host runs only the scalar control flow (barrier update,
// inertia correction, refinement stopping, filter decisions); every vector
// operation is a kernel below, every reduction is a deterministic two-pass
// reduction whose handful of results is copied to pinned host memory.
//
// Steps (Section IV): relaxation of every row into c(x) - s = 0 with slack
// bounds (equality rows [-tol, tol]); Newton step on the barrier KKT
// conditions through the condensed system
//   (W + dw I + Sx + J^T D J) dx = qx + J^T (qs + D qy),   D = Ss + dw I,
// recovery ds = J dx - qy, dy = qs - D ds and of the bound-multiplier steps;
// iterative refinement on the full (unreduced) Newton system; fraction to
// the boundary with separate primal and dual step sizes; filter line search;
// monotone barrier update; scaled optimality error as the stopping test.
// The constants are those of Waechter & Biegler (2006).
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>

#include "model.h"

namespace opf {
void chol_factor_enqueue(chol_sym* C, const double* kval, hipStream_t st, double pivot_tol);
int chol_factor_sync(chol_sym* C, const double* kval, hipStream_t st, double pivot_tol);
int64_t chol_last_negative(const chol_sym* C);
void chol_solve_enqueue(chol_sym* C, const double* b, double* x, hipStream_t st);
int chol_solve_fault(chol_sym* C, hipStream_t st);
void chol_prepare_device(chol_sym* C);
void chol_use_graphs(chol_sym* C, bool on);
void chol_bind_host(chol_sym* C, int64_t* words);
void chol_set_stream(chol_sym* C, hipStream_t st);
}  // namespace opf

using namespace opf;

namespace {

constexpr int EB = 256;
constexpr int RED_BLOCKS = 240;

struct Consts {
    double gamma_theta = 1e-5, gamma_phi = 1e-8, delta = 1.0, s_theta = 1.1, s_phi = 2.3, eta_phi = 1e-4,
           gamma_alpha = 0.05;
    double kappa_eps = 10.0, kappa_mu = 0.2, theta_mu = 1.5, tau_min = 0.99, s_max = 100.0, kappa_sigma = 1e10,
           grad_max = 100.0;
    double dw_first = 1e-4, dw_min = 1e-20, dw_max = 1e40, kw_minus = 1.0 / 3.0, kw_plus_first = 100.0,
           kw_plus = 8.0;
    double ir_stall = 0.9;
    double bound_push = 1e-2, bound_frac = 1e-2;
    int soc_max = 4;          // second-order corrections per iteration (p_max)
    double kappa_soc = 0.99;  // each correction must cut the infeasibility by this factor to continue
};

// distance to a bound: x - lo (lower) or hi - x (upper); absent bounds are +-inf
__device__ __forceinline__ bool fin(double b) { return isfinite(b); }

// ---------------------------------------------------------------- two-pass reductions
enum Comb { SUM = 0, MAX = 1, MIN = 2 };

template <int K>
struct Acc {
    double v[K];
};

__device__ __forceinline__ double comb(int kind, double a, double b) {
    return kind == SUM ? a + b : (kind == MAX ? fmax(a, b) : fmin(a, b));
}
__device__ __forceinline__ double ident(int kind) { return kind == SUM ? 0.0 : (kind == MAX ? -INFINITY : INFINITY); }

template <int K>
__device__ void block_reduce_store(Acc<K>& a, const int* kinds, double* out) {
    __shared__ double sh[K][EB];
    for (int q = 0; q < K; q++) sh[q][threadIdx.x] = a.v[q];
    __syncthreads();
    for (int w = EB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < K; q++) sh[q][threadIdx.x] = comb(kinds[q], sh[q][threadIdx.x], sh[q][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < K; q++) out[q] = sh[q][0];
}

struct KindSet {
    int k[8];
};

template <int K>
__global__ __launch_bounds__(EB) void reduce_final(int nblocks, KindSet ks, const double* __restrict__ part,
                                                   double* __restrict__ out) {
    int kinds[K];
    for (int q = 0; q < K; q++) kinds[q] = ks.k[q];
    Acc<K> a;
    for (int q = 0; q < K; q++) a.v[q] = ident(kinds[q]);
    for (int b = threadIdx.x; b < nblocks; b += EB)
        for (int q = 0; q < K; q++) a.v[q] = comb(kinds[q], a.v[q], part[b * K + q]);
    block_reduce_store<K>(a, kinds, out);
}

struct Vec {
    const double *x, *s, *y, *zl, *zu, *vl, *vu, *xl, *xu, *sl, *su;
};

// (0) max |g - J^T y - zl + zu|, (1) max |y - vl + vu|, (2) max |c - s|,
// (3) max complementarity error for mu, (4) sum |y|, (5) sum |z| (all bound multipliers)
__global__ __launch_bounds__(EB) void red_error(int n, int m, Vec V, const double* __restrict__ g,
                                                const double* __restrict__ jty, const double* __restrict__ c,
                                                double mu, double* __restrict__ part) {
    int kinds[6] = {MAX, MAX, MAX, MAX, SUM, SUM};
    Acc<6> a;
    for (int q = 0; q < 6; q++) a.v[q] = ident(kinds[q]);
    for (int i = blockIdx.x * EB + threadIdx.x; i < n + m; i += gridDim.x * EB) {
        if (i < n) {
            double fx = g[i] - jty[i] - V.zl[i] + V.zu[i];
            a.v[0] = fmax(a.v[0], fabs(fx));
            if (fin(V.xl[i])) a.v[3] = fmax(a.v[3], fabs(V.zl[i] * (V.x[i] - V.xl[i]) - mu));
            if (fin(V.xu[i])) a.v[3] = fmax(a.v[3], fabs(V.zu[i] * (V.xu[i] - V.x[i]) - mu));
            a.v[5] += fabs(V.zl[i]) + fabs(V.zu[i]);
        } else {
            int r = i - n;
            double fs = V.y[r] - V.vl[r] + V.vu[r];
            a.v[1] = fmax(a.v[1], fabs(fs));
            a.v[2] = fmax(a.v[2], fabs(c[r] - V.s[r]));
            if (fin(V.sl[r])) a.v[3] = fmax(a.v[3], fabs(V.vl[r] * (V.s[r] - V.sl[r]) - mu));
            if (fin(V.su[r])) a.v[3] = fmax(a.v[3], fabs(V.vu[r] * (V.su[r] - V.s[r]) - mu));
            a.v[4] += fabs(V.y[r]);
            a.v[5] += fabs(V.vl[r]) + fabs(V.vu[r]);
        }
    }
    block_reduce_store<6>(a, kinds, part + blockIdx.x * 6);
}

// (0) sum |c - s|, (1) sum of log distances to the finite bounds, (2) count of non-positive distances
__global__ __launch_bounds__(EB) void red_merit(int n, int m, const double* __restrict__ x,
                                                const double* __restrict__ s, const double* __restrict__ c,
                                                const double* __restrict__ xl, const double* __restrict__ xu,
                                                const double* __restrict__ sl, const double* __restrict__ su,
                                                double* __restrict__ part) {
    int kinds[3] = {SUM, SUM, SUM};
    Acc<3> a{{0.0, 0.0, 0.0}};
    for (int i = blockIdx.x * EB + threadIdx.x; i < n + m; i += gridDim.x * EB) {
        double v, lo, hi;
        if (i < n) {
            v = x[i];
            lo = xl[i];
            hi = xu[i];
        } else {
            int r = i - n;
            v = s[r];
            lo = sl[r];
            hi = su[r];
            a.v[0] += fabs(c[r] - s[r]);
        }
        if (fin(lo)) {
            double d = v - lo;
            if (d > 0)
                a.v[1] += log(d);
            else
                a.v[2] += 1.0;
        }
        if (fin(hi)) {
            double d = hi - v;
            if (d > 0)
                a.v[1] += log(d);
            else
                a.v[2] += 1.0;
        }
    }
    block_reduce_store<3>(a, kinds, part + blockIdx.x * 3);
}

// (0) g^T dx - mu sum dx/(x-xl) + mu sum dx/(xu-x) - mu sum ds/(s-sl) + mu sum ds/(su-s)
// (1) max |dx|/(1+|x|), |ds|/(1+|s|)
__global__ __launch_bounds__(EB) void red_gphi(int n, int m, const double* __restrict__ g, Vec V,
                                               const double* __restrict__ dx, const double* __restrict__ ds, double mu,
                                               double* __restrict__ part) {
    int kinds[2] = {SUM, MAX};
    Acc<2> a{{0.0, -INFINITY}};
    for (int i = blockIdx.x * EB + threadIdx.x; i < n + m; i += gridDim.x * EB) {
        if (i < n) {
            double t = g[i] * dx[i];
            if (fin(V.xl[i])) t -= mu * dx[i] / (V.x[i] - V.xl[i]);
            if (fin(V.xu[i])) t += mu * dx[i] / (V.xu[i] - V.x[i]);
            a.v[0] += t;
            a.v[1] = fmax(a.v[1], fabs(dx[i]) / (1.0 + fabs(V.x[i])));
        } else {
            int r = i - n;
            double t = 0.0;
            if (fin(V.sl[r])) t -= mu * ds[r] / (V.s[r] - V.sl[r]);
            if (fin(V.su[r])) t += mu * ds[r] / (V.su[r] - V.s[r]);
            a.v[0] += t;
            a.v[1] = fmax(a.v[1], fabs(ds[r]) / (1.0 + fabs(V.s[r])));
        }
    }
    block_reduce_store<2>(a, kinds, part + blockIdx.x * 2);
}

// fraction to the boundary: (0) primal step limit, (1) bound-multiplier step limit
__global__ __launch_bounds__(EB) void red_alpha(int n, int m, Vec V, const double* __restrict__ dx,
                                                const double* __restrict__ ds, const double* __restrict__ dzl,
                                                const double* __restrict__ dzu, const double* __restrict__ dvl,
                                                const double* __restrict__ dvu, double tau,
                                                double* __restrict__ part) {
    int kinds[2] = {MIN, MIN};
    Acc<2> a{{1.0, 1.0}};
    for (int i = blockIdx.x * EB + threadIdx.x; i < n + m; i += gridDim.x * EB) {
        double v, lo, hi, d, zl, zu, dzl_, dzu_;
        if (i < n) {
            v = V.x[i];
            lo = V.xl[i];
            hi = V.xu[i];
            d = dx[i];
            zl = V.zl[i];
            zu = V.zu[i];
            dzl_ = dzl[i];
            dzu_ = dzu[i];
        } else {
            int r = i - n;
            v = V.s[r];
            lo = V.sl[r];
            hi = V.su[r];
            d = ds[r];
            zl = V.vl[r];
            zu = V.vu[r];
            dzl_ = dvl[r];
            dzu_ = dvu[r];
        }
        if (fin(lo)) {
            if (d < 0) a.v[0] = fmin(a.v[0], -tau * (v - lo) / d);
            if (dzl_ < 0) a.v[1] = fmin(a.v[1], -tau * zl / dzl_);
        }
        if (fin(hi)) {
            if (d > 0) a.v[0] = fmin(a.v[0], tau * (hi - v) / d);
            if (dzu_ < 0) a.v[1] = fmin(a.v[1], -tau * zu / dzu_);
        }
    }
    block_reduce_store<2>(a, kinds, part + blockIdx.x * 2);
}

// max |v| over up to 7 blocks of lengths n or m (layout: x-like blocks are n long, others m)
struct Blocks7 {
    const double* p[7];
    int len[7];
};
__global__ __launch_bounds__(EB) void red_maxabs7(Blocks7 B, Blocks7 C, double* __restrict__ part) {
    int kinds[2] = {MAX, MAX};
    Acc<2> a{{0.0, 0.0}};
    for (int q = 0; q < 7; q++) {
        for (int i = blockIdx.x * EB + threadIdx.x; i < B.len[q]; i += gridDim.x * EB) a.v[0] = fmax(a.v[0], fabs(B.p[q][i]));
        for (int i = blockIdx.x * EB + threadIdx.x; i < C.len[q]; i += gridDim.x * EB) a.v[1] = fmax(a.v[1], fabs(C.p[q][i]));
    }
    block_reduce_store<2>(a, kinds, part + blockIdx.x * 2);
}

// ---------------------------------------------------------------- elementwise kernels
// R = -F(mu): right-hand side of the Newton system J_F d = R
__global__ void k_rhs0(int n, int m, Vec V, const double* __restrict__ g, const double* __restrict__ jty,
                       const double* __restrict__ c, double mu, double* Rx, double* Rs, double* Ry, double* Rzl,
                       double* Rzu, double* Rvl, double* Rvu) {
    int i = blockIdx.x * EB + threadIdx.x;
    if (i < n) {
        Rx[i] = -(g[i] - jty[i] - V.zl[i] + V.zu[i]);
        Rzl[i] = fin(V.xl[i]) ? -(V.zl[i] * (V.x[i] - V.xl[i]) - mu) : 0.0;
        Rzu[i] = fin(V.xu[i]) ? -(V.zu[i] * (V.xu[i] - V.x[i]) - mu) : 0.0;
    } else if (i < n + m) {
        int r = i - n;
        Rs[r] = -(V.y[r] - V.vl[r] + V.vu[r]);
        Ry[r] = -(c[r] - V.s[r]);
        Rvl[r] = fin(V.sl[r]) ? -(V.vl[r] * (V.s[r] - V.sl[r]) - mu) : 0.0;
        Rvu[r] = fin(V.su[r]) ? -(V.vu[r] * (V.su[r] - V.s[r]) - mu) : 0.0;
    }
}

// Sx, Ss and the distances; D = Ss + dw
__global__ void k_sigma(int n, int m, Vec V, double* Sx, double* Ss, double* dxl, double* dxu, double* dsl,
                        double* dsu) {
    int i = blockIdx.x * EB + threadIdx.x;
    if (i < n) {
        double a = fin(V.xl[i]) ? V.x[i] - V.xl[i] : 1.0;
        double b = fin(V.xu[i]) ? V.xu[i] - V.x[i] : 1.0;
        dxl[i] = a;
        dxu[i] = b;
        Sx[i] = V.zl[i] / a + V.zu[i] / b;
    } else if (i < n + m) {
        int r = i - n;
        double a = fin(V.sl[r]) ? V.s[r] - V.sl[r] : 1.0;
        double b = fin(V.su[r]) ? V.su[r] - V.s[r] : 1.0;
        dsl[r] = a;
        dsu[r] = b;
        Ss[r] = V.vl[r] / a + V.vu[r] / b;
    }
}

__global__ void k_add_scalar(int m, const double* __restrict__ a, double s, double* __restrict__ out) {
    int i = blockIdx.x * EB + threadIdx.x;
    if (i < m) out[i] = a[i] + s;
}

// reduced right-hand sides: qx = Rx + Rzl/dxl - Rzu/dxu ; qs = ...; v = qs + D qy
__global__ void k_reduce_rhs(int n, int m, Vec V, const double* Rx, const double* Rs, const double* Ry,
                             const double* Rzl, const double* Rzu, const double* Rvl, const double* Rvu,
                             const double* dxl, const double* dxu, const double* dsl, const double* dsu,
                             const double* D, double* qx, double* qs, double* v) {
    int i = blockIdx.x * EB + threadIdx.x;
    if (i < n) {
        double q = Rx[i];
        if (fin(V.xl[i])) q += Rzl[i] / dxl[i];
        if (fin(V.xu[i])) q -= Rzu[i] / dxu[i];
        qx[i] = q;
    } else if (i < n + m) {
        int r = i - n;
        double q = Rs[r];
        if (fin(V.sl[r])) q += Rvl[r] / dsl[r];
        if (fin(V.su[r])) q -= Rvu[r] / dsu[r];
        qs[r] = q;
        v[r] = q + D[r] * Ry[r];
    }
}

// recovery: ds = J dx - qy (Jdx given), dy = qs - D ds, bound-multiplier steps
__global__ void k_recover(int n, int m, Vec V, const double* dx, const double* jdx, const double* Ry,
                          const double* qs, const double* D, const double* Rzl, const double* Rzu, const double* Rvl,
                          const double* Rvu, const double* dxl, const double* dxu, const double* dsl,
                          const double* dsu, double* ds, double* dy, double* dzl, double* dzu, double* dvl,
                          double* dvu) {
    int i = blockIdx.x * EB + threadIdx.x;
    if (i < n) {
        dzl[i] = fin(V.xl[i]) ? (Rzl[i] - V.zl[i] * dx[i]) / dxl[i] : Rzl[i];
        dzu[i] = fin(V.xu[i]) ? (Rzu[i] + V.zu[i] * dx[i]) / dxu[i] : Rzu[i];
    } else if (i < n + m) {
        int r = i - n;
        double d = jdx[r] - Ry[r];
        ds[r] = d;
        dy[r] = qs[r] - D[r] * d;
        dvl[r] = fin(V.sl[r]) ? (Rvl[r] - V.vl[r] * d) / dsl[r] : Rvl[r];
        dvu[r] = fin(V.su[r]) ? (Rvu[r] + V.vu[r] * d) / dsu[r] : Rvu[r];
    }
}

// residual of the full Newton system: res = R - J_F d (W dx, J^T dy and J dx given)
__global__ void k_full_residual(int n, int m, Vec V, double dw, const double* R0x, const double* R0s,
                                const double* R0y, const double* R0zl, const double* R0zu, const double* R0vl,
                                const double* R0vu, const double* dx, const double* ds, const double* dy,
                                const double* dzl, const double* dzu, const double* dvl, const double* dvu,
                                const double* wdx, const double* jtdy, const double* jdx, const double* dxl,
                                const double* dxu, const double* dsl, const double* dsu, double* rx, double* rs,
                                double* ry, double* rzl, double* rzu, double* rvl, double* rvu) {
    int i = blockIdx.x * EB + threadIdx.x;
    if (i < n) {
        rx[i] = R0x[i] - (wdx[i] + dw * dx[i] - jtdy[i] - dzl[i] + dzu[i]);
        rzl[i] = fin(V.xl[i]) ? R0zl[i] - (V.zl[i] * dx[i] + dxl[i] * dzl[i]) : 0.0;
        rzu[i] = fin(V.xu[i]) ? R0zu[i] - (-V.zu[i] * dx[i] + dxu[i] * dzu[i]) : 0.0;
    } else if (i < n + m) {
        int r = i - n;
        rs[r] = R0s[r] - (dw * ds[r] + dy[r] - dvl[r] + dvu[r]);
        ry[r] = R0y[r] - (jdx[r] - ds[r]);
        rvl[r] = fin(V.sl[r]) ? R0vl[r] - (V.vl[r] * ds[r] + dsl[r] * dvl[r]) : 0.0;
        rvu[r] = fin(V.su[r]) ? R0vu[r] - (-V.vu[r] * ds[r] + dsu[r] * dvu[r]) : 0.0;
    }
}

__global__ void k_axpy(int64_t len, double a, const double* __restrict__ x, double* __restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (i < len) y[i] += a * x[i];
}

__global__ void k_trial(int n, int m, double alpha, const double* x, const double* dx, const double* s,
                        const double* ds, double* xt, double* st) {
    int i = blockIdx.x * EB + threadIdx.x;
    if (i < n)
        xt[i] = x[i] + alpha * dx[i];
    else if (i < n + m)
        st[i - n] = s[i - n] + alpha * ds[i - n];
}

// second-order correction: c_soc = a * c_soc + (ct - st) (a = 0: start from ct - st), and its negation into ry
__global__ void k_soc(int m, double a, const double* __restrict__ ct, const double* __restrict__ st,
                      double* __restrict__ csoc, double* __restrict__ ry) {
    int r = blockIdx.x * EB + threadIdx.x;
    if (r < m) {
        const double v = (a == 0.0 ? 0.0 : a * csoc[r]) + (ct[r] - st[r]);
        csoc[r] = v;
        ry[r] = -v;
    }
}

// accept the step and apply the bound-multiplier safeguard
__global__ void k_update(int n, int m, double alpha, double az, double mu, double ksig, double* x, double* s,
                         double* y, double* zl, double* zu, double* vl, double* vu, const double* xl,
                         const double* xu, const double* sl, const double* su, const double* dx, const double* ds,
                         const double* dy, const double* dzl, const double* dzu, const double* dvl,
                         const double* dvu) {
    int i = blockIdx.x * EB + threadIdx.x;
    auto clip = [&](double z, double d) { return fmax(fmin(z, ksig * mu / d), mu / (ksig * d)); };
    if (i < n) {
        double xn = x[i] + alpha * dx[i];
        x[i] = xn;
        double a = zl[i] + az * dzl[i], b = zu[i] + az * dzu[i];
        zl[i] = fin(xl[i]) ? clip(a, xn - xl[i]) : a;
        zu[i] = fin(xu[i]) ? clip(b, xu[i] - xn) : b;
    } else if (i < n + m) {
        int r = i - n;
        double sn = s[r] + alpha * ds[r];
        s[r] = sn;
        y[r] += alpha * dy[r];
        double a = vl[r] + az * dvl[r], b = vu[r] + az * dvu[r];
        vl[r] = fin(sl[r]) ? clip(a, sn - sl[r]) : a;
        vu[r] = fin(su[r]) ? clip(b, su[r] - sn) : b;
    }
}

}  // namespace

// ------------------------------------------------------------------------ state
struct ipm_state {
    opf_model* M = nullptr;
    bool jac_const = false;  // the scaled Jacobian's constant entries are in jac
    chol_sym* C = nullptr;
    ipm_options o{};
    Consts K;
    hipStream_t st = nullptr;
    int n = 0, m = 0;
    double sf = 1.0, mu = 0.1, dw_last = 0.0, theta_max = 0, theta_min = 0;
    int iter = 0;
    int nbounds = 0;
    bool done = false;
    std::vector<std::pair<double, double>> filter;
    // device vectors
    DBuf<double> x, s, y, zl, zu, vl, vu, xl, xu, sl, su, sc;
    DBuf<double> g, c, jac, hess, kval, jty, f;
    DBuf<double> Sx, Ss, D, dxl, dxu, dsl, dsu;
    DBuf<double> R0[7], d[7], cr[7], res[7];
    DBuf<double> qx, qs, v, rhs, tmp_n, tmp_m, wdx, jtdy, jdx;
    DBuf<double> xt, stt, ct, ft;
    DBuf<double> Rs[7], dsoc[7], csoc;  // second-order correction: right-hand side, direction, c_soc
    DBuf<double> part;
    double* host = nullptr;  // pinned scalar outputs
    hipEvent_t ev[10]{};
    bool own_host = true, own_events = true;  // false when lent by the caller (the solve server's slots)
};

namespace {

void fetch(ipm_state* S, int K, double* out) {
    OPF_HIP(hipMemcpyAsync(S->host, S->part.p + RED_BLOCKS * 8, K * sizeof(double), hipMemcpyDeviceToHost, S->st));
    OPF_HIP(hipStreamSynchronize(S->st));
    for (int q = 0; q < K; q++) out[q] = S->host[q];
}

template <int K>
void finish(ipm_state* S, std::initializer_list<int> kinds, double* out) {
    KindSet ks{};
    int q = 0;
    for (int v : kinds) ks.k[q++] = v;
    hipLaunchKernelGGL(reduce_final<K>, dim3(1), dim3(EB), 0, S->st, RED_BLOCKS, ks, S->part.p,
                       S->part.p + RED_BLOCKS * 8);
    OPF_LAUNCH_CHECK();
    fetch(S, K, out);
}

Vec vecs(ipm_state* S) {
    return Vec{S->x.p, S->s.p, S->y.p, S->zl.p, S->zu.p, S->vl.p, S->vu.p, S->xl.p, S->xu.p, S->sl.p, S->su.p};
}

unsigned grid_nm(ipm_state* S) { return ceil_div((size_t)S->n + S->m, EB); }

// E_mu components: dual, primal, compl, and the scaled error
struct ErrInfo {
    double E, dual, primal, compl_;
};

ErrInfo error_mu(ipm_state* S, double mu) {
    hipLaunchKernelGGL(red_error, dim3(RED_BLOCKS), dim3(EB), 0, S->st, S->n, S->m, vecs(S), S->g.p, S->jty.p,
                       S->c.p, mu, S->part.p);
    OPF_LAUNCH_CHECK();
    double r[6];
    finish<6>(S, {MAX, MAX, MAX, MAX, SUM, SUM}, r);
    double dual = std::max(r[0], r[1]), primal = r[2], compl_ = r[3];
    double nb = std::max(S->nbounds, 1);
    double sd = std::max(S->K.s_max, (r[4] + r[5]) / (S->m + nb)) / S->K.s_max;
    double scc = std::max(S->K.s_max, r[5] / nb) / S->K.s_max;
    return {std::max({dual / sd, primal, compl_ / scc}), dual, primal, compl_};
}

// theta and barrier value at (x, s) with constraint values c and scaled objective fval
bool merit(ipm_state* S, const double* x, const double* s, const double* c, double mu, double fval, double* theta,
           double* phi) {
    hipLaunchKernelGGL(red_merit, dim3(RED_BLOCKS), dim3(EB), 0, S->st, S->n, S->m, x, s, c, S->xl.p, S->xu.p,
                       S->sl.p, S->su.p, S->part.p);
    OPF_LAUNCH_CHECK();
    double r[3];
    finish<3>(S, {SUM, SUM, SUM}, r);
    *theta = r[0];
    *phi = fval - mu * r[1];
    return r[2] == 0.0;
}

double read_scalar(ipm_state* S, const double* dptr) {
    OPF_HIP(hipMemcpyAsync(S->host, dptr, sizeof(double), hipMemcpyDeviceToHost, S->st));
    OPF_HIP(hipStreamSynchronize(S->st));
    return S->host[0];
}

void eval_point(ipm_state* S, hipEvent_t after_eval) {
    // scaled gradient, constraints and Jacobian at x, plus J^T y
    // the Jacobian's constant entries (fixed by the row scaling) are written by the first evaluation only
    eval_derivs(S->M, OPF_EVAL_F | OPF_EVAL_C | OPF_EVAL_GRAD | OPF_EVAL_JAC | (S->jac_const ? OPF_EVAL_JAC_VAR : 0),
                S->x.p, S->y.p, S->sf, S->sc.p, S->sf, S->f.p, S->c.p, S->g.p, S->jac.p, nullptr, S->st);
    S->jac_const = true;
    if (after_eval) OPF_HIP(hipEventRecord(after_eval, S->st));
    jt_times(S->M, S->jac.p, S->y.p, nullptr, S->jty.p, S->st);
}

void push_into(std::vector<double>& v, const std::vector<double>& lo, const std::vector<double>& hi, double k1,
               double k2) {
    for (size_t i = 0; i < v.size(); i++) {
        bool fl = std::isfinite(lo[i]), fu = std::isfinite(hi[i]);
        double pl = fl ? k1 * std::max(1.0, std::fabs(lo[i])) : 0.0;
        double pu = fu ? k1 * std::max(1.0, std::fabs(hi[i])) : 0.0;
        if (fl && fu) {
            pl = std::min(pl, k2 * (hi[i] - lo[i]));
            pu = std::min(pu, k2 * (hi[i] - lo[i]));
        }
        if (fl) v[i] = std::max(v[i], lo[i] + pl);
        if (fu) v[i] = std::min(v[i], hi[i] - pu);
    }
}

double relax(double b, double f, double sign) { return std::isfinite(b) ? b + sign * f * std::max(1.0, std::fabs(b)) : b; }

// solve J_F d = R through the condensed system (factor must be current)
void reduce_solve(ipm_state* S, DBuf<double>* R, DBuf<double>* out) {
    const int n = S->n, m = S->m;
    Vec V = vecs(S);
    hipLaunchKernelGGL(k_reduce_rhs, dim3(grid_nm(S)), dim3(EB), 0, S->st, n, m, V, R[0].p, R[1].p, R[2].p, R[3].p,
                       R[4].p, R[5].p, R[6].p, S->dxl.p, S->dxu.p, S->dsl.p, S->dsu.p, S->D.p, S->qx.p, S->qs.p,
                       S->v.p);
    OPF_LAUNCH_CHECK();
    jt_times(S->M, S->jac.p, S->v.p, S->qx.p, S->rhs.p, S->st);
    chol_solve_enqueue(S->C, S->rhs.p, out[0].p, S->st);
    j_times(S->M, S->jac.p, out[0].p, S->jdx.p, S->st);
    hipLaunchKernelGGL(k_recover, dim3(grid_nm(S)), dim3(EB), 0, S->st, n, m, V, out[0].p, S->jdx.p, R[2].p,
                       S->qs.p, S->D.p, R[3].p, R[4].p, R[5].p, R[6].p, S->dxl.p, S->dxu.p, S->dsl.p, S->dsu.p,
                       out[1].p, out[2].p, out[3].p, out[4].p, out[5].p, out[6].p);
    OPF_LAUNCH_CHECK();
}

void maxabs7(ipm_state* S, DBuf<double>* A, DBuf<double>* B, double* na, double* nb) {
    Blocks7 X{}, Y{};
    const int lens[7] = {S->n, S->m, S->m, S->n, S->n, S->m, S->m};
    for (int q = 0; q < 7; q++) {
        X.p[q] = A[q].p;
        X.len[q] = lens[q];
        Y.p[q] = B ? B[q].p : A[q].p;
        Y.len[q] = B ? lens[q] : 0;
    }
    hipLaunchKernelGGL(red_maxabs7, dim3(RED_BLOCKS), dim3(EB), 0, S->st, X, Y, S->part.p);
    OPF_LAUNCH_CHECK();
    double r[2];
    finish<2>(S, {MAX, MAX}, r);
    *na = r[0];
    *nb = r[1];
}

}  // namespace

extern "C" void ipm_default_options(ipm_options* o) {
    o->tol = 1e-4;
    o->max_iter = 500;
    o->max_ir = 10;
    o->ir_tol = 1e-10;
    o->mu_init = 0.1;
    o->bound_relax = 1e-8;
    o->pivot_tol = 1e-12;
    o->graphs = 1;
    o->soc = 0;
}

// ipm_create with optional parts supplied by the caller (internal, used by the solve server): an analysis
// already made for the model's condensed pattern (ownership passes to the state), a pinned buffer of 16
// doubles and 10 events that stay the caller's.  Lets the server run the host analysis before it takes
// pool memory and keep pinned allocations and events per slot instead of per request.
int ipm_create_ex(opf_model* M, const ipm_options* opts, const chol_options* copts, void* stream, chol_sym* prebuilt,
                  double* host, const hipEvent_t* events, ipm_state** out);

extern "C" int ipm_create(opf_model* M, const ipm_options* opts, const chol_options* copts, void* stream,
                          ipm_state** out) {
    return ipm_create_ex(M, opts, copts, stream, nullptr, nullptr, nullptr, out);
}

int ipm_create_ex(opf_model* M, const ipm_options* opts, const chol_options* copts, void* stream, chol_sym* prebuilt,
                  double* host, const hipEvent_t* events, ipm_state** out) {
    return guarded([&] {
        OPF_CHECK(M && out, OPF_E_INVALID, "ipm_create: null argument");
        *out = nullptr;
        auto* S = new ipm_state();
        try {
            S->M = M;
            ipm_default_options(&S->o);
            if (opts) S->o = *opts;
            OPF_CHECK(S->o.tol > 0 && S->o.max_iter >= 0, OPF_E_INVALID, "ipm_create: bad options");
            S->st = (hipStream_t)stream;
            const int n = M->n, m = M->m;
            S->n = n;
            S->m = m;
            if (prebuilt) {
                S->C = prebuilt;
                prebuilt = nullptr;
            } else {
                int rc = chol_analyze(n, M->kcolptr.data(), M->krowind.data(), copts, &S->C);
                if (rc != OPF_OK) throw Error{rc};
            }
            // graphs need a stream of our own to capture on (capture on the null stream is not allowed)
            chol_use_graphs(S->C, S->o.graphs != 0 && S->st != nullptr);
            // pending uploads of the analysis (and of a model created without a stream) run on this stream
            chol_set_stream(S->C, S->st);
            if (!M->dev.done && !M->dev.stream) M->dev.stream = S->st;
            for (DBuf<double>* b : {&S->x, &S->zl, &S->zu, &S->xl, &S->xu, &S->g, &S->jty, &S->Sx, &S->dxl, &S->dxu,
                                    &S->qx, &S->rhs, &S->tmp_n, &S->wdx, &S->jtdy, &S->xt})
                b->alloc(n);
            for (DBuf<double>* b : {&S->s, &S->y, &S->vl, &S->vu, &S->sl, &S->su, &S->sc, &S->c, &S->Ss, &S->D,
                                    &S->dsl, &S->dsu, &S->qs, &S->v, &S->tmp_m, &S->jdx, &S->stt, &S->ct})
                b->alloc(m);
            const int lens[7] = {n, m, m, n, n, m, m};
            for (int q = 0; q < 7; q++) {
                S->R0[q].alloc(lens[q]);
                S->d[q].alloc(lens[q]);
                S->cr[q].alloc(lens[q]);
                S->res[q].alloc(lens[q]);
            }
            if (S->o.soc) {
                for (int q = 0; q < 7; q++) {
                    S->Rs[q].alloc(lens[q]);
                    S->dsoc[q].alloc(lens[q]);
                }
                S->csoc.alloc(m);
            }
            S->jac.alloc(M->nnzj);
            S->hess.alloc(M->nnzh);
            S->kval.alloc(M->nnzk);
            S->f.alloc(1);
            S->ft.alloc(1);
            S->part.alloc(RED_BLOCKS * 8 + 8);
            if (host) {
                S->host = host;
                S->own_host = false;
            } else {
                OPF_HIP(hipHostMalloc((void**)&S->host, 16 * sizeof(double)));
            }
            // the reductions read at most 8 doubles; the last four words carry the factorization's status
            chol_bind_host(S->C, reinterpret_cast<int64_t*>(S->host + 12));
            if (events) {
                for (int q = 0; q < 10; q++) S->ev[q] = events[q];
                S->own_events = false;
            } else {
                for (auto& e : S->ev) OPF_HIP(hipEventCreate(&e));
            }
            // ---- scaling at the user starting point
            std::vector<double> x0 = M->x0;
            OPF_HIP(hipMemcpyAsync(S->x.p, x0.data(), n * 8, hipMemcpyHostToDevice, S->st));
            eval_derivs(M, OPF_EVAL_GRAD | OPF_EVAL_JAC, S->x.p, nullptr, 1.0, nullptr, 1.0, nullptr, nullptr,
                        S->g.p, S->jac.p, nullptr, S->st);
            std::vector<double> g0(n), j0(M->nnzj);
            OPF_HIP(hipMemcpyAsync(g0.data(), S->g.p, n * 8, hipMemcpyDeviceToHost, S->st));
            OPF_HIP(hipMemcpyAsync(j0.data(), S->jac.p, M->nnzj * 8, hipMemcpyDeviceToHost, S->st));
            OPF_HIP(hipStreamSynchronize(S->st));
            double gmax = 0;
            for (double v : g0) gmax = std::max(gmax, std::fabs(v));
            S->sf = gmax > 0 ? std::min(1.0, S->K.grad_max / gmax) : 1.0;
            std::vector<double> rowmax(m, 0.0), sc(m);
            for (int64_t e = 0; e < M->nnzj; e++) rowmax[M->jrow[e]] = std::max(rowmax[M->jrow[e]], std::fabs(j0[e]));
            for (int r = 0; r < m; r++) sc[r] = rowmax[r] > 0 ? std::min(1.0, S->K.grad_max / rowmax[r]) : 1.0;
            // ---- bounds of the relaxed, scaled problem
            const double br = S->o.bound_relax;
            std::vector<double> xl(n), xu(n), sl(m), su(m);
            for (int i = 0; i < n; i++) {
                xl[i] = relax(M->xl[i], br, -1.0);
                xu[i] = relax(M->xu[i], br, +1.0);
            }
            for (int r = 0; r < m; r++) {
                double gl = sc[r] * M->gl[r], gu = sc[r] * M->gu[r];
                if (M->gl[r] == M->gu[r]) {
                    sl[r] = gl - S->o.tol;
                    su[r] = gu + S->o.tol;
                } else {
                    sl[r] = relax(gl, br, -1.0);
                    su[r] = relax(gu, br, +1.0);
                }
            }
            int nb = 0;
            for (int i = 0; i < n; i++) nb += std::isfinite(xl[i]) + std::isfinite(xu[i]);
            for (int r = 0; r < m; r++) nb += std::isfinite(sl[r]) + std::isfinite(su[r]);
            S->nbounds = nb;
            push_into(x0, xl, xu, S->K.bound_push, S->K.bound_frac);
            auto up = [&](DBuf<double>& d, const std::vector<double>& h) {
                OPF_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * 8, hipMemcpyHostToDevice, S->st));
            };
            up(S->x, x0);
            up(S->xl, xl);
            up(S->xu, xu);
            up(S->sl, sl);
            up(S->su, su);
            up(S->sc, sc);
            // slacks from the scaled constraint values at the pushed point
            eval_derivs(M, OPF_EVAL_C, S->x.p, nullptr, 1.0, S->sc.p, 1.0, nullptr, S->c.p, nullptr, nullptr, nullptr,
                        S->st);
            std::vector<double> s0(m);
            OPF_HIP(hipMemcpyAsync(s0.data(), S->c.p, m * 8, hipMemcpyDeviceToHost, S->st));
            OPF_HIP(hipStreamSynchronize(S->st));
            push_into(s0, sl, su, S->K.bound_push, S->K.bound_frac);
            up(S->s, s0);
            std::vector<double> zero_m(m, 0.0), zl(n), zu(n), vl(m), vu(m);
            for (int i = 0; i < n; i++) {
                zl[i] = std::isfinite(xl[i]) ? 1.0 : 0.0;
                zu[i] = std::isfinite(xu[i]) ? 1.0 : 0.0;
            }
            for (int r = 0; r < m; r++) {
                vl[r] = std::isfinite(sl[r]) ? 1.0 : 0.0;
                vu[r] = std::isfinite(su[r]) ? 1.0 : 0.0;
            }
            up(S->y, zero_m);
            up(S->zl, zl);
            up(S->zu, zu);
            up(S->vl, vl);
            up(S->vu, vu);
            S->mu = S->o.mu_init;
            eval_point(S, nullptr);
            double th0 = 0, ph0 = 0;
            merit(S, S->x.p, S->s.p, S->c.p, S->mu, 0.0, &th0, &ph0);
            S->theta_max = 1e4 * std::max(1.0, th0);
            S->theta_min = 1e-4 * std::max(1.0, th0);
        } catch (...) {
            if (prebuilt) chol_destroy(prebuilt);  // not yet handed to the state
            ipm_destroy(S);
            throw;
        }
        *out = S;
    });
}

extern "C" int ipm_destroy(ipm_state* S) {
    if (!S) return OPF_OK;
    if (S->C) chol_destroy(S->C);
    if (S->host && S->own_host) (void)hipHostFree(S->host);
    if (S->own_events)
        for (auto& e : S->ev)
            if (e) (void)hipEventDestroy(e);
    delete S;
    return OPF_OK;
}

extern "C" chol_sym* ipm_chol(ipm_state* S) { return S ? S->C : nullptr; }

// Every device buffer of a state allocated and uploaded now (the analysis's normally wait for the first
// factorization); used by the solve server to count a request's footprint at admission.
int ipm_prepare_device(ipm_state* S) {
    return guarded([&] {
        OPF_CHECK(S, OPF_E_INVALID, "ipm_prepare_device: null state");
        chol_prepare_device(S->C);
        OPF_HIP(hipStreamSynchronize(S->st));
    });
}

// X = J_F^{-1} R through the current factor (condensed solve + recovery) with iterative refinement on the
// full, unreduced system including the regularization dw; returns the refinement steps taken.
static int refined_solve(ipm_state* S, DBuf<double>* R, DBuf<double>* X, double dw) {
    const int n = S->n, m = S->m;
    hipStream_t st = S->st;
    Vec V = vecs(S);
    reduce_solve(S, R, X);
    double nr0, dummy;
    maxabs7(S, R, nullptr, &nr0, &dummy);
    double prev = INFINITY;
    int nir = 0;
    for (int it = 0; it < S->o.max_ir; it++) {
        w_times(S->M, S->hess.p, X[0].p, S->wdx.p, st);
        jt_times(S->M, S->jac.p, X[2].p, nullptr, S->jtdy.p, st);
        j_times(S->M, S->jac.p, X[0].p, S->jdx.p, st);
        hipLaunchKernelGGL(k_full_residual, dim3(grid_nm(S)), dim3(EB), 0, st, n, m, V, dw, R[0].p, R[1].p, R[2].p,
                           R[3].p, R[4].p, R[5].p, R[6].p, X[0].p, X[1].p, X[2].p, X[3].p, X[4].p, X[5].p, X[6].p,
                           S->wdx.p, S->jtdy.p, S->jdx.p, S->dxl.p, S->dxu.p, S->dsl.p, S->dsu.p, S->res[0].p,
                           S->res[1].p, S->res[2].p, S->res[3].p, S->res[4].p, S->res[5].p, S->res[6].p);
        OPF_LAUNCH_CHECK();
        double rn;
        maxabs7(S, S->res, nullptr, &rn, &dummy);
        if (rn <= S->o.ir_tol * std::max(1.0, nr0) || rn > S->K.ir_stall * prev) break;
        prev = rn;
        reduce_solve(S, S->res, S->cr);
        const int lens[7] = {n, m, m, n, n, m, m};
        for (int q = 0; q < 7; q++) {
            hipLaunchKernelGGL(k_axpy, dim3(ceil_div(lens[q], EB)), dim3(EB), 0, st, (int64_t)lens[q], 1.0,
                               S->cr[q].p, X[q].p);
            OPF_LAUNCH_CHECK();
        }
        nir++;
    }
    return nir;
}

// Newton direction at the current iterate for barrier parameter mu: Hessian,
// residuals, diagonals, factorization with inertia correction (primal
// regularization dw), condensed solve + recovery, iterative refinement on the
// full system.  Leaves the direction in S->d.  Returns OPF_OK or OPF_E_NOT_PD.
static int compute_direction(ipm_state* S, double mu, ipm_iter_info& I) {
    const int n = S->n, m = S->m;
    const Consts& K = S->K;
    hipStream_t st = S->st;
    Vec V = vecs(S);
    // ---- Hessian, residuals, diagonals
    OPF_HIP(hipEventRecord(S->ev[0], st));
    eval_derivs(S->M, OPF_EVAL_HESS, S->x.p, S->y.p, S->sf, S->sc.p, S->sf, nullptr, nullptr, nullptr, nullptr,
                S->hess.p, st);
    OPF_HIP(hipEventRecord(S->ev[1], st));
    hipLaunchKernelGGL(k_rhs0, dim3(grid_nm(S)), dim3(EB), 0, st, n, m, V, S->g.p, S->jty.p, S->c.p, mu, S->R0[0].p,
                       S->R0[1].p, S->R0[2].p, S->R0[3].p, S->R0[4].p, S->R0[5].p, S->R0[6].p);
    OPF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sigma, dim3(grid_nm(S)), dim3(EB), 0, st, n, m, V, S->Sx.p, S->Ss.p, S->dxl.p, S->dxu.p,
                       S->dsl.p, S->dsu.p);
    OPF_LAUNCH_CHECK();
    // ---- factorization with inertia correction
    double t_asm = 0, t_fac = 0;
    auto try_factor = [&](double dw) {
        hipLaunchKernelGGL(k_add_scalar, dim3(ceil_div(m, EB)), dim3(EB), 0, st, m, S->Ss.p, dw, S->D.p);
        OPF_HIP(hipEventRecord(S->ev[2], st));
        condense(S->M, S->hess.p, S->jac.p, S->Sx.p, S->D.p, dw, S->kval.p, st);
        OPF_HIP(hipEventRecord(S->ev[3], st));
        int bad = chol_factor_sync(S->C, S->kval.p, st, S->o.pivot_tol);
        OPF_HIP(hipEventRecord(S->ev[4], st));
        OPF_HIP(hipEventSynchronize(S->ev[4]));
        float a = 0, b = 0;
        OPF_HIP(hipEventElapsedTime(&a, S->ev[2], S->ev[3]));
        OPF_HIP(hipEventElapsedTime(&b, S->ev[3], S->ev[4]));
        t_asm += a;
        t_fac += b;
        I.factorizations++;
        // the condensed matrix must be positive definite (Section IV-C); an L D L^T factorization reports it
        // through the signs of its pivots (zero pivots are rejected like non-positive Cholesky pivots)
        return bad < 0 && chol_last_negative(S->C) == 0;
    };
    double dw = 0.0;
    if (!try_factor(0.0)) {
        dw = S->dw_last == 0.0 ? K.dw_first : std::max(K.dw_min, K.kw_minus * S->dw_last);
        while (true) {
            if (dw > K.dw_max) {
                set_error("ipm_step: regularization exceeded its maximum");
                return OPF_E_NOT_PD;
            }
            if (try_factor(dw)) {
                S->dw_last = dw;
                break;
            }
            dw *= S->dw_last == 0.0 ? K.kw_plus_first : K.kw_plus;
        }
    }
    I.delta_w = dw;
    // ---- direction + iterative refinement on the full system
    OPF_HIP(hipEventRecord(S->ev[5], st));
    const int nir = refined_solve(S, S->R0, S->d, dw);
    OPF_HIP(hipEventRecord(S->ev[6], st));
    if (chol_solve_fault(S->C, st)) {
        set_error("ipm_step: a triangular-solve block wait exceeded its bound");
        return OPF_E_DEVICE;
    }
    I.ir_steps = nir;
    I.t_assembly = t_asm;
    I.t_factor = t_fac;
    return OPF_OK;
}

static int ipm_step_impl(ipm_state* S, ipm_iter_info* info) {
    const int n = S->n, m = S->m;
    const Consts& K = S->K;
    hipStream_t st = S->st;
    ipm_iter_info I{};
    I.iter = S->iter;
    auto t_start = std::chrono::steady_clock::now();
    // ---- convergence test at the current point (derivatives already evaluated)
    ErrInfo e0 = error_mu(S, 0.0);
    double fs = read_scalar(S, S->f.p);
    I.obj = fs / S->sf;
    I.e0 = e0.E;
    I.inf_pr = e0.primal;
    I.inf_du = e0.dual;
    I.mu = S->mu;
    if (!std::isfinite(e0.E)) {
        if (info) *info = I;
        set_error("ipm_step: non-finite optimality error");
        return OPF_E_NUMERIC;
    }
    if (e0.E <= S->o.tol) {
        S->done = true;
        if (info) *info = I;
        return 1;
    }
    if (S->iter >= S->o.max_iter) {
        if (info) *info = I;
        set_error("ipm_step: iteration limit reached");
        return OPF_E_MAXITER;
    }
    // ---- barrier update
    const double mu_min = S->o.tol / 10.0;
    while (true) {
        ErrInfo em = error_mu(S, S->mu);
        if (em.E > K.kappa_eps * S->mu || S->mu <= mu_min) break;
        double nm = std::max(mu_min, std::min(K.kappa_mu * S->mu, std::pow(S->mu, K.theta_mu)));
        if (nm >= S->mu) break;
        S->mu = nm;
        S->filter.clear();
    }
    const double mu = S->mu;
    I.mu = mu;
    const double tau = std::max(K.tau_min, 1.0 - mu);
    Vec V = vecs(S);
    {
        int rc = compute_direction(S, mu, I);
        if (rc != OPF_OK) {
            if (info) *info = I;
            return rc;
        }
    }
    // ---- step sizes
    hipLaunchKernelGGL(red_alpha, dim3(RED_BLOCKS), dim3(EB), 0, st, n, m, V, S->d[0].p, S->d[1].p, S->d[3].p,
                       S->d[4].p, S->d[5].p, S->d[6].p, tau, S->part.p);
    OPF_LAUNCH_CHECK();
    double al[2];
    finish<2>(S, {MIN, MIN}, al);
    const double amax = al[0];
    double az = al[1];
    // ---- filter line search
    double th0, ph0;
    merit(S, S->x.p, S->s.p, S->c.p, mu, fs, &th0, &ph0);
    hipLaunchKernelGGL(red_gphi, dim3(RED_BLOCKS), dim3(EB), 0, st, n, m, S->g.p, V, S->d[0].p, S->d[1].p, mu,
                       S->part.p);
    OPF_LAUNCH_CHECK();
    double gp[2];
    finish<2>(S, {SUM, MAX}, gp);
    const double gphi = gp[0];
    const bool tiny = gp[1] < 10.0 * 2.220446049250313e-16;
    double alpha = amax;
    bool accepted = false, augment = false;
    int nls = 0;
    double t_trial = 0;  // derivative evaluations of the line-search trial points (ms)
    int nsoc = 0;        // second-order corrections tried
    if (tiny) {
        accepted = true;
    } else {
        double amin;
        if (gphi < 0) {
            if (th0 <= S->theta_min)
                amin = K.gamma_alpha * std::min({K.gamma_theta, K.gamma_phi * th0 / (-gphi),
                                                 K.delta * std::pow(th0, K.s_theta) / std::pow(-gphi, K.s_phi)});
            else
                amin = K.gamma_alpha * std::min(K.gamma_theta, K.gamma_phi * th0 / (-gphi));
        } else {
            amin = K.gamma_alpha * K.gamma_theta;
        }
        // filter and sufficient-decrease test of a trial point: (accepted, f-type step)
        auto acceptable = [&](double tht, double pht, bool inside, double a, bool* ftype) {
            *ftype = false;
            if (!(inside && std::isfinite(tht) && std::isfinite(pht) && tht < S->theta_max)) return false;
            for (auto& p : S->filter)
                if (!(tht < p.first || pht < p.second)) return false;
            bool switching = gphi < 0 && a * std::pow(-gphi, K.s_phi) > K.delta * std::pow(th0, K.s_theta);
            if (th0 <= S->theta_min && switching) {
                *ftype = true;
                return pht <= ph0 + K.eta_phi * a * gphi;
            }
            return tht <= (1.0 - K.gamma_theta) * th0 || pht <= ph0 - K.gamma_phi * th0;
        };
        // trial point x + a dx, s + a ds: constraint values into ct, returns theta, phi and interiority
        auto trial = [&](double a, const double* dx, const double* ds, double* tht, double* pht) {
            hipLaunchKernelGGL(k_trial, dim3(grid_nm(S)), dim3(EB), 0, st, n, m, a, S->x.p, dx, S->s.p, ds,
                               S->xt.p, S->stt.p);
            OPF_LAUNCH_CHECK();
            OPF_HIP(hipEventRecord(S->ev[8], st));
            eval_derivs(S->M, OPF_EVAL_F | OPF_EVAL_C, S->xt.p, nullptr, 1.0, S->sc.p, S->sf, S->ft.p, S->ct.p,
                        nullptr, nullptr, nullptr, st);
            OPF_HIP(hipEventRecord(S->ev[9], st));
            double ft = read_scalar(S, S->ft.p);
            float tt = 0;
            OPF_HIP(hipEventElapsedTime(&tt, S->ev[8], S->ev[9]));
            t_trial += tt;
            return merit(S, S->xt.p, S->stt.p, S->ct.p, mu, ft, tht, pht);
        };
        const int lens[7] = {n, m, m, n, n, m, m};
        while (true) {
            nls++;
            double tht, pht;
            bool inside = trial(alpha, S->d[0].p, S->d[1].p, &tht, &pht);
            bool ftype = false;
            if (acceptable(tht, pht, inside, alpha, &ftype)) {
                accepted = true;
                augment = !ftype;
                break;
            }
            if (S->o.soc && nls == 1 && !(tht < th0)) {
                // second-order correction: the same Newton matrix with the constraint residual replaced by the
                // accumulated c_soc = alpha0 (c - s) + (c_trial - s_trial)
                const double alpha0 = alpha;
                for (int q = 0; q < 7; q++)
                    if (q != 2)
                        OPF_HIP(hipMemcpyAsync(S->Rs[q].p, S->R0[q].p, lens[q] * 8, hipMemcpyDeviceToDevice, st));
                // c_soc starts as alpha0 (c - s): k_soc with a = 0 on (c, s) gives c - s, scaled on the next call
                hipLaunchKernelGGL(k_soc, dim3(ceil_div(m, EB)), dim3(EB), 0, st, m, 0.0, S->c.p, S->s.p,
                                   S->csoc.p, S->Rs[2].p);
                hipLaunchKernelGGL(k_soc, dim3(ceil_div(m, EB)), dim3(EB), 0, st, m, alpha0, S->ct.p, S->stt.p,
                                   S->csoc.p, S->Rs[2].p);
                OPF_LAUNCH_CHECK();
                double th_old = tht;
                for (int p = 1; p <= K.soc_max; p++) {
                    nsoc++;
                    refined_solve(S, S->Rs, S->dsoc, I.delta_w);
                    hipLaunchKernelGGL(red_alpha, dim3(RED_BLOCKS), dim3(EB), 0, st, n, m, V, S->dsoc[0].p,
                                       S->dsoc[1].p, S->dsoc[3].p, S->dsoc[4].p, S->dsoc[5].p, S->dsoc[6].p, tau,
                                       S->part.p);
                    OPF_LAUNCH_CHECK();
                    double as[2];
                    finish<2>(S, {MIN, MIN}, as);
                    double ths, phs;
                    bool ins = trial(as[0], S->dsoc[0].p, S->dsoc[1].p, &ths, &phs);
                    bool ft2 = false;
                    if (acceptable(ths, phs, ins, alpha0, &ft2)) {
                        for (int q = 0; q < 7; q++)
                            OPF_HIP(hipMemcpyAsync(S->d[q].p, S->dsoc[q].p, lens[q] * 8, hipMemcpyDeviceToDevice,
                                                   st));
                        alpha = as[0];
                        az = as[1];
                        accepted = true;
                        augment = !ft2;
                        break;
                    }
                    if (p == K.soc_max || ths > K.kappa_soc * th_old) break;
                    hipLaunchKernelGGL(k_soc, dim3(ceil_div(m, EB)), dim3(EB), 0, st, m, as[0], S->ct.p, S->stt.p,
                                       S->csoc.p, S->Rs[2].p);
                    OPF_LAUNCH_CHECK();
                    th_old = ths;
                }
                if (accepted) break;
            }
            alpha *= 0.5;
            if (alpha < amin) break;
        }
    }
    I.ls_trials = nls;
    I.soc_steps = nsoc;
    if (!accepted) {
        if (info) *info = I;
        set_error("ipm_step: line search failed at iteration %d", S->iter);
        return OPF_E_LINESEARCH;
    }
    if (augment) S->filter.emplace_back((1.0 - K.gamma_theta) * th0, ph0 - K.gamma_phi * th0);
    hipLaunchKernelGGL(k_update, dim3(grid_nm(S)), dim3(EB), 0, st, n, m, alpha, az, mu, K.kappa_sigma, S->x.p,
                       S->s.p, S->y.p, S->zl.p, S->zu.p, S->vl.p, S->vu.p, S->xl.p, S->xu.p, S->sl.p, S->su.p,
                       S->d[0].p, S->d[1].p, S->d[2].p, S->d[3].p, S->d[4].p, S->d[5].p, S->d[6].p);
    OPF_LAUNCH_CHECK();
    OPF_HIP(hipEventRecord(S->ev[7], st));
    eval_point(S, S->ev[8]);
    OPF_HIP(hipStreamSynchronize(st));
    I.alpha = alpha;
    I.alpha_z = az;
    float tad = 0, tpt = 0, tsol = 0;
    OPF_HIP(hipEventElapsedTime(&tad, S->ev[0], S->ev[1]));
    OPF_HIP(hipEventElapsedTime(&tpt, S->ev[7], S->ev[8]));
    OPF_HIP(hipEventElapsedTime(&tsol, S->ev[5], S->ev[6]));
    // every derivative evaluation of the iteration: Hessian, trial points, new point (c, J, gradient)
    I.t_ad = tad + tpt + t_trial;
    I.t_solve = tsol;
    I.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    S->iter++;
    if (info) *info = I;
    return OPF_OK;
}

extern "C" int ipm_step(ipm_state* S, ipm_iter_info* info) {
    int status = OPF_OK;
    int rc = guarded([&] {
        OPF_CHECK(S, OPF_E_INVALID, "ipm_step: null state");
        status = ipm_step_impl(S, info);
    });
    return rc != OPF_OK ? rc : status;
}

extern "C" int ipm_solve(ipm_state* S, ipm_result* out) {
    int status = OPF_OK;
    ipm_result R{};
    int rc = guarded([&] {
        OPF_CHECK(S, OPF_E_INVALID, "ipm_solve: null state");
        const auto t0 = std::chrono::steady_clock::now();
        ipm_iter_info I{};
        while (true) {
            I = ipm_iter_info{};
            status = ipm_step_impl(S, &I);
            R.factorizations += I.factorizations;
            R.ir_steps += I.ir_steps;
            R.t_ad += I.t_ad;
            R.t_assembly += I.t_assembly;
            R.t_factor += I.t_factor;
            R.t_solve += I.t_solve;
            if (status != OPF_OK) break;
        }
        R.status = status == 1 ? 1 : status;
        R.iterations = S->iter;
        R.objective = I.obj;
        R.e0 = I.e0;
        R.inf_pr = I.inf_pr;
        R.inf_du = I.inf_du;
        R.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        R.x = S->x.p;
        R.s = S->s.p;
        R.y = S->y.p;
        if (status == 1) status = OPF_OK;
    });
    if (rc != OPF_OK) R.status = rc;
    if (out) *out = R;
    return rc != OPF_OK ? rc : status;
}

extern "C" int ipm_get_iterate(const ipm_state* S, double* x, double* s, double* y) {
    return guarded([&] {
        OPF_CHECK(S, OPF_E_INVALID, "ipm_get_iterate: null state");
        // every copy on the state's own stream: an operation on the legacy null stream would have to order
        // itself after other threads' streams, which fails while one of them is capturing a graph
        if (x) OPF_HIP(hipMemcpyAsync(x, S->x.p, S->n * 8, hipMemcpyDeviceToHost, S->st));
        if (s) OPF_HIP(hipMemcpyAsync(s, S->s.p, S->m * 8, hipMemcpyDeviceToHost, S->st));
        if (y) OPF_HIP(hipMemcpyAsync(y, S->y.p, S->m * 8, hipMemcpyDeviceToHost, S->st));
        OPF_HIP(hipStreamSynchronize(S->st));
    });
}

extern "C" int ipm_get_state(const ipm_state* S, double* x, double* s, double* y, double* zl, double* zu, double* vl,
                             double* vu, double* mu, double* dw_last) {
    return guarded([&] {
        OPF_CHECK(S, OPF_E_INVALID, "ipm_get_state: null state");
        auto get = [&](double* h, const DBuf<double>& d, int len) {
            if (h) OPF_HIP(hipMemcpyAsync(h, d.p, (size_t)len * 8, hipMemcpyDeviceToHost, S->st));
        };
        get(x, S->x, S->n);
        get(s, S->s, S->m);
        get(y, S->y, S->m);
        get(zl, S->zl, S->n);
        get(zu, S->zu, S->n);
        get(vl, S->vl, S->m);
        get(vu, S->vu, S->m);
        OPF_HIP(hipStreamSynchronize(S->st));
        if (mu) *mu = S->mu;
        if (dw_last) *dw_last = S->dw_last;
    });
}

extern "C" int ipm_set_state(ipm_state* S, const double* x, const double* s, const double* y, const double* zl,
                             const double* zu, const double* vl, const double* vu, double mu, double dw_last) {
    return guarded([&] {
        OPF_CHECK(S && x && s && y && zl && zu && vl && vu && mu > 0, OPF_E_INVALID, "ipm_set_state: bad argument");
        auto put = [&](DBuf<double>& d, const double* h, int len) {
            OPF_HIP(hipMemcpyAsync(d.p, h, (size_t)len * 8, hipMemcpyHostToDevice, S->st));
        };
        put(S->x, x, S->n);
        put(S->s, s, S->m);
        put(S->y, y, S->m);
        put(S->zl, zl, S->n);
        put(S->zu, zu, S->n);
        put(S->vl, vl, S->m);
        put(S->vu, vu, S->m);
        S->mu = mu;
        S->dw_last = dw_last;
        eval_point(S, nullptr);
        OPF_HIP(hipStreamSynchronize(S->st));
    });
}

extern "C" int ipm_direction(ipm_state* S, double* dx, double* ds, double* dy, double* dzl, double* dzu, double* dvl,
                             double* dvu, double* delta_w, int32_t* ir_steps) {
    int status = OPF_OK;
    int rc = guarded([&] {
        OPF_CHECK(S, OPF_E_INVALID, "ipm_direction: null state");
        ipm_iter_info I{};
        status = compute_direction(S, S->mu, I);
        if (status != OPF_OK) return;
        double* outs[7] = {dx, ds, dy, dzl, dzu, dvl, dvu};
        const int lens[7] = {S->n, S->m, S->m, S->n, S->n, S->m, S->m};
        for (int q = 0; q < 7; q++)
            if (outs[q])
                OPF_HIP(hipMemcpyAsync(outs[q], S->d[q].p, (size_t)lens[q] * 8, hipMemcpyDeviceToHost, S->st));
        OPF_HIP(hipStreamSynchronize(S->st));
        if (delta_w) *delta_w = I.delta_w;
        if (ir_steps) *ir_steps = I.ir_steps;
    });
    return rc != OPF_OK ? rc : status;
}
