// Polar ACOPF templates and their derivatives (Section III of the paper).
//
// The model is written as template instances (Patterns 1-3 of Section II-C):
// every arc evaluates its two flow definitions and its thermal limit, every
// branch its angle difference, every bus its two balance rows (a gather over
// the arcs and generators attached to it: the paper's augmentation, done as a
// precomputed CSR gather instead of a scatter), every generator its cost.
// One fused launch runs all templates: each block knows from its index which
// template family it serves, each work-item owns one instance, reads the
// instance parameters from structure-of-arrays buffers with coalesced loads,
// gathers the bus voltages it needs, and writes its values into fixed,
// family-major slots of c, J and H so that consecutive work-items write
// consecutive addresses.  Each template's nonlinear part is written once, as a
// function of a generic number type (arc_flows, thermal, shunt, cost below):
// instantiated with double it gives the constraint values, instantiated with
// the second-order forward-mode Jet of jet.h it gives the value, the gradient
// (Jacobian entries) and the Hessian over the instance's local inputs in one
// evaluation (Section III-B).  Only the linear parts (the +-1 Jacobian entries
// of the flow variables, arcs and generators in the balances, and the angle
// differences) are written directly.
#include <cmath>
#include <cstdarg>

#include "jet.h"
#include "model.h"

namespace opf {

static thread_local char g_err[1024] = "";

DeviceRegion*& thread_region() {
    static thread_local DeviceRegion* r = nullptr;
    return r;
}

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

struct AdParams {
    int N, E, G, ref;
    unsigned what;
    const double* x;
    const double* y;
    const double* cscale;
    double obj_weight, gscale;
    // template data
    const int32_t *ai, *aj;
    const double *ag, *ab, *abc;
    const double *pd, *qd, *gs, *bs;
    const int32_t *bus_arc_ptr, *bus_arc, *bus_gen_ptr, *bus_gen;
    const double *c2, *c1;
    const int32_t* gbus;
    // outputs
    double *c, *grad, *jac, *hess;
    // block ranges
    int arc_blocks, bus_blocks, gen_blocks;
};

constexpr int AD_BLOCK = 256;

// ---------------------------------------------------------------- template value expressions
// Flow functions of arc i -> j (patterns 3-6) over its local inputs (va_i, va_j, vm_i, vm_j): series
// admittance g + jb, half the line charging bc at each end, tap 1, no shift:
//   phi_p = g vm_i^2 - vm_i vm_j (g cos(va_i - va_j) + b sin(va_i - va_j))
//   phi_q = -(b + bc) vm_i^2 - vm_i vm_j (g sin(va_i - va_j) - b cos(va_i - va_j))
template <class T>
__device__ __forceinline__ void arc_flows(const T& vai, const T& vaj, const T& vi, const T& vj, double g, double b,
                                          double bc, T* phip, T* phiq) {
    T s, c;
    sincos(vai - vaj, &s, &c);
    const T vv = vi * vj;
    const T vi2 = vi * vi;
    *phip = g * vi2 - vv * (g * c + b * s);
    *phiq = -(b + bc) * vi2 - vv * (g * s - b * c);
}

// thermal limit of an arc (patterns 8-9) over (p_a, q_a)
template <class T>
__device__ __forceinline__ T thermal(const T& p, const T& q) {
    return p * p + q * q;
}

// shunt term of a bus balance (patterns 10-11) over vm: coef vm^2 (coef = Gs active, -Bs reactive)
template <class T>
__device__ __forceinline__ T shunt(const T& vm, double coef) {
    return coef * (vm * vm);
}

// generator cost (pattern 1) over pg, without the constant c0 (which the objective adds)
template <class T>
__device__ __forceinline__ T cost(const T& pg, double c2, double c1) {
    return c2 * (pg * pg) + c1 * pg;
}

__device__ __forceinline__ double rs(const double* cscale, int64_t row) { return cscale ? cscale[row] : 1.0; }

__global__ __launch_bounds__(AD_BLOCK) void ad_templates(AdParams P) {
    const int N = P.N, E = P.E, G = P.G;
    const int A = 2 * E;
    const RowLayout R(N, E);
    const JLayout JL(N, E, G);
    const HLayout HL(N, E, G);
    const int ova = 0, ovm = N, opg = 2 * N, oqg = 2 * N + G, op = 2 * N + 2 * G, oq = op + A;
    const bool wc = P.what & OPF_EVAL_C, wj = P.what & OPF_EVAL_JAC, wh = P.what & OPF_EVAL_HESS,
               wg = P.what & OPF_EVAL_GRAD;
    const bool wjc = wj && !(P.what & OPF_EVAL_JAC_VAR);  // constant Jacobian entries too
    int b = blockIdx.x;
    if (b < P.arc_blocks) {
        // ---------------- arc template: patterns 3-6 (flows), 8-9 (thermal), 7 (angle on a < E)
        int a = b * AD_BLOCK + threadIdx.x;
        if (a >= A) return;
        if (wg) {  // the gradient has no arc-flow terms
            P.grad[op + a] = 0.0;
            P.grad[oq + a] = 0.0;
        }
        if (!(wc || wj || wh)) return;
        const int i = P.ai[a], j = P.aj[a];
        const double g = P.ag[a], bb = P.ab[a], bc = P.abc[a];
        const double vai = P.x[ova + i], vaj = P.x[ova + j];
        const double vi = P.x[ovm + i], vj = P.x[ovm + j];
        const double pa = P.x[op + a], qa = P.x[oq + a];
        const int64_t rp = R.p + a, rq = R.q + a, rt = R.th + a;
        const double sp = rs(P.cscale, rp), sq = rs(P.cscale, rq), st = rs(P.cscale, rt);
        if (wc && !(wj || wh)) {
            double phip, phiq;
            arc_flows(vai, vaj, vi, vj, g, bb, bc, &phip, &phiq);
            P.c[rp] = sp * (pa - phip);
            P.c[rq] = sq * (qa - phiq);
            P.c[rt] = st * thermal(pa, qa);
            if (a < E) P.c[R.ang + a] = rs(P.cscale, R.ang + a) * (vai - vaj);
        }
        if (wj || wh) {
            // local inputs 0..3 = (va_i, va_j, vm_i, vm_j); c_p = p_a - phi_p, c_q = q_a - phi_q
            using J4 = Jet<4>;
            J4 phip, phiq;
            arc_flows(J4::input(vai, 0), J4::input(vaj, 1), J4::input(vi, 2), J4::input(vj, 3), g, bb, bc, &phip,
                      &phiq);
            using J2 = Jet<2>;
            const J2 th2 = thermal(J2::input(pa, 0), J2::input(qa, 1));
            if (wc) {
                P.c[rp] = sp * (pa - phip.v);
                P.c[rq] = sq * (qa - phiq.v);
                P.c[rt] = st * th2.v;
                if (a < E) P.c[R.ang + a] = rs(P.cscale, R.ang + a) * (vai - vaj);
            }
            if (wj) {
                double* J = P.jac + JL.flow;
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    J[(1 + k) * (int64_t)A + a] = -sp * phip.g[k];
                    J[(6 + k) * (int64_t)A + a] = -sq * phiq.g[k];
                }
                P.jac[JL.th + a] = st * th2.g[0];
                P.jac[JL.th + A + a] = st * th2.g[1];
                if (wjc) {
                    J[0 * (int64_t)A + a] = sp;
                    J[5 * (int64_t)A + a] = sq;
                    if (a < E) {
                        const double sa = rs(P.cscale, R.ang + a);
                        P.jac[JL.ang + a] = sa;
                        P.jac[JL.ang + E + a] = -sa;
                    }
                    P.jac[JL.bal_parc + a] = rs(P.cscale, R.pb + i);
                    P.jac[JL.bal_qarc + a] = rs(P.cscale, R.qb + i);
                }
            }
            if (wh) {
                // the Lagrangian's -y grad^2 c = +y grad^2 phi over the ten lower entries of (va_i, va_j, vm_i,
                // vm_j), in the Hessian layout's order
                constexpr int slot_i[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
                constexpr int slot_j[10] = {0, 1, 2, 3, 0, 0, 0, 1, 1, 2};
                const double yp = P.y[rp] * sp, yq = P.y[rq] * sq, yt = P.y[rt] * st;
                double* Hp = P.hess + HL.pflow;
                double* Hq = P.hess + HL.qflow;
#pragma unroll
                for (int k = 0; k < 10; k++) {
                    const int q = J4::hi(slot_i[k], slot_j[k]);
                    Hp[k * (int64_t)A + a] = yp * phip.h[q];
                    Hq[k * (int64_t)A + a] = yq * phiq.h[q];
                }
                P.hess[HL.th + a] = -yt * th2.h[J2::hi(0, 0)];
                P.hess[HL.th + A + a] = -yt * th2.h[J2::hi(1, 1)];
            }
        }
        return;
    }
    b -= P.arc_blocks;
    if (b < P.bus_blocks) {
        // ---------------- bus template: patterns 10-15 (balances with arc and generator gathers), 2 (ref)
        int i = b * AD_BLOCK + threadIdx.x;
        if (i >= N) return;
        if (wg) {  // nor voltage terms
            P.grad[ova + i] = 0.0;
            P.grad[ovm + i] = 0.0;
        }
        if (!(wc || wj || wh)) return;
        const double vm = P.x[ovm + i];
        const int64_t rpb = R.pb + i, rqb = R.qb + i;
        const double spb = rs(P.cscale, rpb), sqb = rs(P.cscale, rqb);
        const double gsi = P.gs[i], bsi = P.bs[i];
        if (wc) {
            double sp = 0.0, sq = 0.0;
            for (int k = P.bus_arc_ptr[i]; k < P.bus_arc_ptr[i + 1]; k++) {
                int a = P.bus_arc[k];
                sp += P.x[op + a];
                sq += P.x[oq + a];
            }
            double gp = 0.0, gq = 0.0;
            for (int k = P.bus_gen_ptr[i]; k < P.bus_gen_ptr[i + 1]; k++) {
                int gk = P.bus_gen[k];
                gp += P.x[opg + gk];
                gq += P.x[oqg + gk];
            }
            P.c[rpb] = spb * (sp - gp + P.pd[i] + shunt(vm, gsi));
            P.c[rqb] = sqb * (sq - gq + P.qd[i] + shunt(vm, -bsi));
            if (i == P.ref) P.c[R.ref] = rs(P.cscale, R.ref) * P.x[ova + i];
        }
        if (wj || wh) {
            const Jet<1> shp = shunt(Jet<1>::input(vm, 0), gsi), shq = shunt(Jet<1>::input(vm, 0), -bsi);
            if (wj) {
                P.jac[JL.bal_pvm + i] = spb * shp.g[0];
                P.jac[JL.bal_qvm + i] = sqb * shq.g[0];
                if (wjc && i == P.ref) P.jac[JL.ref] = rs(P.cscale, R.ref);
            }
            if (wh) {
                P.hess[HL.bal_p + i] = -(P.y[rpb] * spb) * shp.h[0];
                P.hess[HL.bal_q + i] = -(P.y[rqb] * sqb) * shq.h[0];
            }
        }
        return;
    }
    b -= P.bus_blocks;
    if (b < P.gen_blocks) {
        // ---------------- generator template: pattern 1 (cost) and the generator columns of 12-13
        int k = b * AD_BLOCK + threadIdx.x;
        if (k >= G) return;
        const double pg = P.x[opg + k];
        const Jet<1> f = cost(Jet<1>::input(pg, 0), P.c2[k], P.c1[k]);
        if (wg) {
            P.grad[opg + k] = P.gscale * f.g[0];
            P.grad[oqg + k] = 0.0;
        }
        if (wjc) {
            const int i = P.gbus[k];
            P.jac[JL.bal_pg + k] = -rs(P.cscale, R.pb + i);
            P.jac[JL.bal_qg + k] = -rs(P.cscale, R.qb + i);
        }
        if (wh) P.hess[HL.gen + k] = P.obj_weight * f.h[0];
    }
}

// f = gscale * sum_g (c2 pg^2 + c1 pg + c0): one block, fixed summation order.
__global__ __launch_bounds__(256) void ad_objective(int N, int G, const double* x, const double* c2, const double* c1,
                                                    const double* c0, double gscale, double* f) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < G; k += 256) {
        double pg = x[2 * N + k];
        acc += cost(pg, c2[k], c1[k]) + c0[k];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) f[0] = gscale * sh[0];
}

void eval_derivs(const opf_model* M, unsigned what, const double* x, const double* y, double obj_weight,
                 const double* cscale, double gscale, double* f, double* c, double* grad, double* jac,
                 double* hess, hipStream_t s) {
    ensure_device(M);
    AdParams P{};
    P.N = M->N;
    P.E = M->E;
    P.G = M->G;
    P.ref = M->ref;
    P.what = what;
    P.x = x;
    P.y = y;
    P.cscale = cscale;
    P.obj_weight = obj_weight;
    P.gscale = gscale;
    P.ai = M->ai.p;
    P.aj = M->aj.p;
    P.ag = M->ag.p;
    P.ab = M->ab.p;
    P.abc = M->abc.p;
    P.pd = M->pd.p;
    P.qd = M->qd.p;
    P.gs = M->gs.p;
    P.bs = M->bs.p;
    P.bus_arc_ptr = M->bus_arc_ptr.p;
    P.bus_arc = M->bus_arc.p;
    P.bus_gen_ptr = M->bus_gen_ptr.p;
    P.bus_gen = M->bus_gen.p;
    P.c2 = M->c2.p;
    P.c1 = M->c1.p;
    P.gbus = M->gbus.p;
    P.c = c;
    P.grad = grad;
    P.jac = jac;
    P.hess = hess;
    unsigned tmpl = what & (OPF_EVAL_C | OPF_EVAL_GRAD | OPF_EVAL_JAC | OPF_EVAL_HESS);
    if (tmpl) {
        // the arc and bus threads also zero their gradient entries (the gradient is the cost's, on pg only)
        P.arc_blocks = ceil_div(2LL * M->E, AD_BLOCK);
        P.bus_blocks = ceil_div(M->N, AD_BLOCK);
        P.gen_blocks = ceil_div(M->G, AD_BLOCK);
        int nb = P.arc_blocks + P.bus_blocks + P.gen_blocks;
        if (nb > 0) {
            hipLaunchKernelGGL(ad_templates, dim3(nb), dim3(AD_BLOCK), 0, s, P);
            OPF_LAUNCH_CHECK();
        }
    }
    if (what & OPF_EVAL_F) {
        hipLaunchKernelGGL(ad_objective, dim3(1), dim3(256), 0, s, M->N, M->G, x, M->c2.p, M->c1.p, M->c0.p, gscale,
                           f);
        OPF_LAUNCH_CHECK();
    }
}

}  // namespace opf

using namespace opf;

extern "C" const char* opf_last_error(void) { return g_err; }

static void build_structure(opf_model* M, const opf_grid* g) {
    const int N = M->N, E = M->E, G = M->G;
    const int64_t A = 2LL * E;
    const RowLayout R(N, E);
    const JLayout JL(N, E, G);
    const HLayout HL(N, E, G);
    const int ova = 0, ovm = N, opg = 2 * N, oqg = 2 * N + G, op = 2 * N + 2 * G, oq = op + (int)A;
    std::vector<int32_t> ai(A), aj(A);
    for (int l = 0; l < E; l++) {
        ai[l] = g->f[l];
        aj[l] = g->t[l];
        ai[E + l] = g->t[l];
        aj[E + l] = g->f[l];
    }
    M->jrow.assign(JL.total, 0);
    M->jcol.assign(JL.total, 0);
    auto setj = [&](int64_t e, int64_t r, int64_t c) {
        M->jrow[e] = (int32_t)r;
        M->jcol[e] = (int32_t)c;
    };
    setj(JL.ref, R.ref, ova + M->ref);
    for (int64_t a = 0; a < A; a++) {
        int i = ai[a], j = aj[a];
        const int64_t cols[5] = {op + a, ova + i, ova + j, ovm + i, ovm + j};
        const int64_t colq[5] = {oq + a, ova + i, ova + j, ovm + i, ovm + j};
        for (int k = 0; k < 5; k++) setj(JL.flow + k * A + a, R.p + a, cols[k]);
        for (int k = 0; k < 5; k++) setj(JL.flow + (5 + k) * A + a, R.q + a, colq[k]);
        setj(JL.th + a, R.th + a, op + a);
        setj(JL.th + A + a, R.th + a, oq + a);
        setj(JL.bal_parc + a, R.pb + i, op + a);
        setj(JL.bal_qarc + a, R.qb + i, oq + a);
    }
    for (int l = 0; l < E; l++) {
        setj(JL.ang + l, R.ang + l, ova + g->f[l]);
        setj(JL.ang + E + l, R.ang + l, ova + g->t[l]);
    }
    for (int i = 0; i < N; i++) {
        setj(JL.bal_pvm + i, R.pb + i, ovm + i);
        setj(JL.bal_qvm + i, R.qb + i, ovm + i);
    }
    for (int k = 0; k < G; k++) {
        setj(JL.bal_pg + k, R.pb + g->gbus[k], opg + k);
        setj(JL.bal_qg + k, R.qb + g->gbus[k], oqg + k);
    }
    M->hrow.assign(HL.total, 0);
    M->hcol.assign(HL.total, 0);
    auto seth = [&](int64_t e, int64_t u, int64_t v) {
        M->hrow[e] = (int32_t)std::max(u, v);
        M->hcol[e] = (int32_t)std::min(u, v);
    };
    for (int64_t a = 0; a < A; a++) {
        int i = ai[a], j = aj[a];
        const int64_t vi = ova + i, vj = ova + j, mi = ovm + i, mj = ovm + j;
        const int64_t pr[10][2] = {{vi, vi}, {vj, vj}, {mi, mi}, {mj, mj}, {vi, vj},
                                   {vi, mi}, {vi, mj}, {vj, mi}, {vj, mj}, {mi, mj}};
        for (int k = 0; k < 10; k++) {
            seth(HL.pflow + k * A + a, pr[k][0], pr[k][1]);
            seth(HL.qflow + k * A + a, pr[k][0], pr[k][1]);
        }
        seth(HL.th + a, op + a, op + a);
        seth(HL.th + A + a, oq + a, oq + a);
    }
    for (int i = 0; i < N; i++) {
        seth(HL.bal_p + i, ovm + i, ovm + i);
        seth(HL.bal_q + i, ovm + i, ovm + i);
    }
    for (int k = 0; k < G; k++) seth(HL.gen + k, opg + k, opg + k);
    M->nnzj = JL.total;
    M->nnzh = HL.total;

    // bounds and starting point
    const int n = M->n, m = M->m;
    const double inf = INFINITY;
    M->xl.assign(n, -inf);
    M->xu.assign(n, inf);
    for (int i = 0; i < N; i++) {
        M->xl[ovm + i] = g->vmin[i];
        M->xu[ovm + i] = g->vmax[i];
    }
    for (int k = 0; k < G; k++) {
        M->xl[opg + k] = g->pmin[k];
        M->xu[opg + k] = g->pmax[k];
        M->xl[oqg + k] = g->qmin[k];
        M->xu[oqg + k] = g->qmax[k];
    }
    for (int64_t a = 0; a < A; a++) {
        double rt = g->rate[a % E];
        M->xl[op + a] = -rt;
        M->xu[op + a] = rt;
        M->xl[oq + a] = -rt;
        M->xu[oq + a] = rt;
    }
    M->gl.assign(m, 0.0);
    M->gu.assign(m, 0.0);
    for (int l = 0; l < E; l++) {
        M->gl[R.ang + l] = g->angmin[l];
        M->gu[R.ang + l] = g->angmax[l];
    }
    for (int64_t a = 0; a < A; a++) {
        double rt = g->rate[a % E];
        M->gl[R.th + a] = -inf;
        M->gu[R.th + a] = rt * rt;
    }
    M->x0.assign(n, 0.0);
    for (int i = 0; i < N; i++) M->x0[ovm + i] = 1.0;
    for (int k = 0; k < G; k++) M->x0[opg + k] = 0.5 * g->pmax[k];
    for (int64_t a = 0; a < A; a++) {
        int l = (int)(a % E);
        double z2 = g->r[l] * g->r[l] + g->x[l] * g->x[l];
        double gg = g->r[l] / z2, bb = -g->x[l] / z2, bc = 0.5 * g->b[l];
        // flat start: vi = vj = 1, theta = 0
        M->x0[op + a] = gg - gg;
        M->x0[oq + a] = -(bb + bc) + bb;
    }

    // device template data
    std::vector<double> ag(A), ab(A), abc(A);
    for (int64_t a = 0; a < A; a++) {
        int l = (int)(a % E);
        double z2 = g->r[l] * g->r[l] + g->x[l] * g->x[l];
        ag[a] = g->r[l] / z2;
        ab[a] = -g->x[l] / z2;
        abc[a] = 0.5 * g->b[l];
    }
    M->dev.upload(M->ai, ai);
    M->dev.upload(M->aj, aj);
    M->dev.upload(M->ag, ag);
    M->dev.upload(M->ab, ab);
    M->dev.upload(M->abc, abc);
    M->dev.upload(M->pd, std::vector<double>(g->pd, g->pd + N));
    M->dev.upload(M->qd, std::vector<double>(g->qd, g->qd + N));
    M->dev.upload(M->gs, std::vector<double>(g->gs, g->gs + N));
    M->dev.upload(M->bs, std::vector<double>(g->bs, g->bs + N));
    std::vector<int32_t> bap(N + 1, 0), ba(A), bgp(N + 1, 0), bg(G);
    for (int64_t a = 0; a < A; a++) bap[ai[a] + 1]++;
    for (int k = 0; k < G; k++) bgp[g->gbus[k] + 1]++;
    for (int i = 0; i < N; i++) {
        bap[i + 1] += bap[i];
        bgp[i + 1] += bgp[i];
    }
    {
        std::vector<int32_t> fa(bap.begin(), bap.end() - 1), fg(bgp.begin(), bgp.end() - 1);
        for (int64_t a = 0; a < A; a++) ba[fa[ai[a]]++] = (int32_t)a;
        for (int k = 0; k < G; k++) bg[fg[g->gbus[k]]++] = k;
    }
    M->dev.upload(M->bus_arc_ptr, bap);
    M->dev.upload(M->bus_arc, ba);
    M->dev.upload(M->bus_gen_ptr, bgp);
    M->dev.upload(M->bus_gen, bg);
    M->dev.upload(M->gbus, std::vector<int32_t>(g->gbus, g->gbus + G));
    const double base = g->base_mva;
    std::vector<double> c2(G), c1(G), c0(G);
    for (int k = 0; k < G; k++) {
        c2[k] = g->c2[k] * base * base;
        c1[k] = g->c1[k] * base;
        c0[k] = g->c0[k];
    }
    M->dev.upload(M->c2, c2);
    M->dev.upload(M->c1, c1);
    M->dev.upload(M->c0, c0);
    M->dev.alloc(M->fpart, 1);
}

extern "C" void opf_default_options(opf_options* o) {
    if (o) o->assembly = 0;
}

namespace opf {
// The grid checks of opf_create (OPF_E_INVALID, with the first problem's message); also used by the solve
// server to reject a bad grid at submission without building the model there.
static void check_grid(const opf_grid* g) {
    OPF_CHECK(g->nbus >= 1 && g->nbranch >= 0 && g->ngen >= 1, OPF_E_INVALID,
              "invalid grid: need nbus >= 1, nbranch >= 0, ngen >= 1");
    OPF_CHECK(g->ref_bus >= 0 && g->ref_bus < g->nbus, OPF_E_INVALID, "invalid grid: ref_bus out of range");
    OPF_CHECK(g->base_mva > 0, OPF_E_INVALID, "invalid grid: base_mva must be positive");
    const int64_t N = g->nbus, E = g->nbranch, G = g->ngen;
    OPF_CHECK(2 * N + 2 * G + 4 * E < INT32_MAX && 2 * N + 1 + 7 * E < INT32_MAX, OPF_E_INVALID,
              "invalid grid: problem too large for int32 indices");
    for (int64_t l = 0; l < E; l++) {
        OPF_CHECK(g->f[l] >= 0 && g->f[l] < N && g->t[l] >= 0 && g->t[l] < N && g->f[l] != g->t[l],
                  OPF_E_INVALID, "invalid grid: branch %lld has invalid endpoints", (long long)l);
        OPF_CHECK(g->r[l] * g->r[l] + g->x[l] * g->x[l] > 0, OPF_E_INVALID,
                  "invalid grid: branch %lld has zero impedance", (long long)l);
        OPF_CHECK(g->rate[l] > 0, OPF_E_INVALID, "invalid grid: branch %lld has non-positive rating",
                  (long long)l);
    }
    for (int64_t k = 0; k < G; k++) {
        OPF_CHECK(g->gbus[k] >= 0 && g->gbus[k] < N, OPF_E_INVALID, "invalid grid: generator %lld bus",
                  (long long)k);
        OPF_CHECK(g->pmin[k] <= g->pmax[k] && g->qmin[k] <= g->qmax[k], OPF_E_INVALID,
                  "invalid grid: generator %lld has inverted limits", (long long)k);
    }
    for (int64_t i = 0; i < N; i++)
        OPF_CHECK(g->vmin[i] <= g->vmax[i] && g->vmin[i] > 0, OPF_E_INVALID, "invalid grid: bus %lld vm bounds",
                  (long long)i);
}

int validate_grid(const opf_grid* g) {
    return guarded([&] {
        OPF_CHECK(g, OPF_E_INVALID, "invalid grid: null pointer");
        check_grid(g);
    });
}
}  // namespace opf

extern "C" int opf_create(const opf_grid* g, const opf_options* opts, void* stream, opf_model** out) {
    return guarded([&] {
        OPF_CHECK(g && out, OPF_E_INVALID, "opf_create: null argument");
        opf_options o{};
        opf_default_options(&o);
        if (opts) o = *opts;
        OPF_CHECK(o.assembly == 0 || o.assembly == 1, OPF_E_INVALID, "opf_create: assembly must be 0 or 1");
        *out = nullptr;
        check_grid(g);
        const int64_t N = g->nbus, E = g->nbranch, G = g->ngen;
        auto* M = new opf_model();
        try {
            M->N = (int)N;
            M->E = (int)E;
            M->G = (int)G;
            M->ref = g->ref_bus;
            M->n = (int)(2 * N + 2 * G + 4 * E);
            M->m = (int)(2 * N + 1 + 7 * E);
            M->dev.stream = (hipStream_t)stream;
            M->per_entry_assembly = o.assembly == 1;
            build_structure(M, g);
            build_kkt_maps(M);
        } catch (...) {
            delete M;
            throw;
        }
        *out = M;
    });
}

extern "C" int opf_destroy(opf_model* M) {
    delete M;
    return OPF_OK;
}

extern "C" int opf_dims(const opf_model* M, int32_t* n, int32_t* m, int64_t* nnzj, int64_t* nnzh, int64_t* nnzk) {
    return guarded([&] {
        OPF_CHECK(M, OPF_E_INVALID, "opf_dims: null model");
        if (n) *n = M->n;
        if (m) *m = M->m;
        if (nnzj) *nnzj = M->nnzj;
        if (nnzh) *nnzh = M->nnzh;
        if (nnzk) *nnzk = M->nnzk;
    });
}

extern "C" int opf_structure(const opf_model* M, int32_t* jrow, int32_t* jcol, int32_t* hrow, int32_t* hcol) {
    return guarded([&] {
        OPF_CHECK(M, OPF_E_INVALID, "opf_structure: null model");
        if (jrow) memcpy(jrow, M->jrow.data(), M->jrow.size() * 4);
        if (jcol) memcpy(jcol, M->jcol.data(), M->jcol.size() * 4);
        if (hrow) memcpy(hrow, M->hrow.data(), M->hrow.size() * 4);
        if (hcol) memcpy(hcol, M->hcol.data(), M->hcol.size() * 4);
    });
}

extern "C" int opf_bounds(const opf_model* M, double* xl, double* xu, double* gl, double* gu) {
    return guarded([&] {
        OPF_CHECK(M, OPF_E_INVALID, "opf_bounds: null model");
        if (xl) memcpy(xl, M->xl.data(), M->xl.size() * 8);
        if (xu) memcpy(xu, M->xu.data(), M->xu.size() * 8);
        if (gl) memcpy(gl, M->gl.data(), M->gl.size() * 8);
        if (gu) memcpy(gu, M->gu.data(), M->gu.size() * 8);
    });
}

extern "C" int opf_initial_point(const opf_model* M, double* x0) {
    return guarded([&] {
        OPF_CHECK(M && x0, OPF_E_INVALID, "opf_initial_point: null argument");
        memcpy(x0, M->x0.data(), M->x0.size() * 8);
    });
}

extern "C" int opf_eval_derivs(opf_model* M, unsigned what, const double* x, const double* y, double obj_weight,
                               double* f, double* c, double* grad, double* jac, double* hess, void* stream) {
    return guarded([&] {
        OPF_CHECK(M && x, OPF_E_INVALID, "opf_eval_derivs: null model or x");
        OPF_CHECK(!(what & ~63u), OPF_E_INVALID, "opf_eval_derivs: unknown flag bits");
        OPF_CHECK(!(what & OPF_EVAL_JAC_VAR) || (what & OPF_EVAL_JAC), OPF_E_INVALID,
                  "opf_eval_derivs: OPF_EVAL_JAC_VAR needs OPF_EVAL_JAC");
        OPF_CHECK(!(what & OPF_EVAL_F) || f, OPF_E_INVALID, "opf_eval_derivs: f is NULL");
        OPF_CHECK(!(what & OPF_EVAL_C) || c, OPF_E_INVALID, "opf_eval_derivs: c is NULL");
        OPF_CHECK(!(what & OPF_EVAL_GRAD) || grad, OPF_E_INVALID, "opf_eval_derivs: grad is NULL");
        OPF_CHECK(!(what & OPF_EVAL_JAC) || jac, OPF_E_INVALID, "opf_eval_derivs: jac is NULL");
        OPF_CHECK(!(what & OPF_EVAL_HESS) || (hess && y), OPF_E_INVALID, "opf_eval_derivs: hess or y is NULL");
        eval_derivs(M, what, x, y, obj_weight, nullptr, 1.0, f, c, grad, jac, hess, (hipStream_t)stream);
    });
}
