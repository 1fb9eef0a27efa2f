// Condensed KKT assembly (Section IV-C): K = W + dw I + Sigma_x + J^T D J.
//
// The paper assembles the condensed matrix with scatter-type operations
// (Pattern 3).  Here every entry of the fixed lower pattern of K owns the
// list of its contributions, computed once on the host when the model is
// created: the Hessian entries that land on it and the Jacobian entry pairs
// (a, b, row r) whose product J_a D_r J_b lands on it.  The assembly kernel
// is then a pure gather (one work-item per entry of K, no atomics, fixed
// summation order, bitwise reproducible).  The same precomputed access paths
// give J x, J^T v and the symmetric Hessian product used by the IPM.
#include <algorithm>
#include <numeric>

#include "model.h"

namespace opf {

constexpr int KB = 256;

__global__ __launch_bounds__(KB) void kkt_gather(int64_t nnzk, const int32_t* __restrict__ hptr,
                                                 const int32_t* __restrict__ hidx, const int32_t* __restrict__ pptr,
                                                 const int32_t* __restrict__ pa, const int32_t* __restrict__ pb,
                                                 const int32_t* __restrict__ pr, const int32_t* __restrict__ kdiag,
                                                 const double* __restrict__ hess, const double* __restrict__ jac,
                                                 const double* __restrict__ sigx, const double* __restrict__ dvec,
                                                 double dw, double* __restrict__ kval) {
    int64_t k = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (k >= nnzk) return;
    double v = 0.0;
    int dcol = kdiag[k];
    if (dcol >= 0) v = sigx[dcol] + dw;
    for (int e = hptr[k]; e < hptr[k + 1]; e++) v += hess[hidx[e]];
    for (int e = pptr[k]; e < pptr[k + 1]; e++) v += jac[pa[e]] * dvec[pr[e]] * jac[pb[e]];
    kval[k] = v;
}

__global__ __launch_bounds__(KB) void csr_gather_mv(int nrows, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ ent, const int32_t* __restrict__ idx,
                                                    const double* __restrict__ val, const double* __restrict__ v,
                                                    const double* __restrict__ base, double* __restrict__ out) {
    int r = blockIdx.x * KB + threadIdx.x;
    if (r >= nrows) return;
    double s = base ? base[r] : 0.0;
    for (int k = ptr[r]; k < ptr[r + 1]; k++) {
        int e = ent[k];
        s += val[e] * v[idx[e]];
    }
    out[r] = s;
}

// Symmetric Hessian product: row i gathers (entry, other index) pairs.
__global__ __launch_bounds__(KB) void sym_gather_mv(int n, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ ent, const int32_t* __restrict__ oth,
                                                    const double* __restrict__ val, const double* __restrict__ v,
                                                    double* __restrict__ out) {
    int r = blockIdx.x * KB + threadIdx.x;
    if (r >= n) return;
    double s = 0.0;
    for (int k = ptr[r]; k < ptr[r + 1]; k++) s += val[ent[k]] * v[oth[k]];
    out[r] = s;
}

void condense(const opf_model* M, const double* hess, const double* jac, const double* sigx, const double* dvec,
              double dw, double* kval, hipStream_t s) {
    ensure_device(M);
    if (M->nnzk == 0) return;
    hipLaunchKernelGGL(kkt_gather, dim3(ceil_div(M->nnzk, KB)), dim3(KB), 0, s, M->nnzk, M->k_hptr.p, M->k_hidx.p,
                       M->k_pptr.p, M->k_pa.p, M->k_pb.p, M->k_pr.p, M->k_diag.p, hess, jac, sigx, dvec, dw, kval);
    OPF_LAUNCH_CHECK();
}

void jt_times(const opf_model* M, const double* jac, const double* v, const double* base, double* out,
              hipStream_t s) {
    ensure_device(M);
    hipLaunchKernelGGL(csr_gather_mv, dim3(ceil_div(M->n, KB)), dim3(KB), 0, s, M->n, M->jt_ptr.p, M->jt_ent.p,
                       M->j_row.p, jac, v, base, out);
    OPF_LAUNCH_CHECK();
}

void j_times(const opf_model* M, const double* jac, const double* x, double* out, hipStream_t s) {
    ensure_device(M);
    hipLaunchKernelGGL(csr_gather_mv, dim3(ceil_div(M->m, KB)), dim3(KB), 0, s, M->m, M->jr_ptr.p, M->jr_ent.p,
                       M->j_col.p, jac, x, (const double*)nullptr, out);
    OPF_LAUNCH_CHECK();
}

void w_times(const opf_model* M, const double* hess, const double* x, double* out, hipStream_t s) {
    ensure_device(M);
    hipLaunchKernelGGL(sym_gather_mv, dim3(ceil_div(M->n, KB)), dim3(KB), 0, s, M->n, M->w_ptr.p, M->w_ent.p,
                       M->w_oth.p, hess, x, out);
    OPF_LAUNCH_CHECK();
}

// Counting sort of items by key into CSR (ptr over nkeys, stable in item order).
static void csr_by_key(int64_t nkeys, const std::vector<int64_t>& key, std::vector<int32_t>& ptr,
                       std::vector<int32_t>& order) {
    ptr.assign(nkeys + 1, 0);
    for (int64_t k : key) ptr[k + 1]++;
    for (int64_t i = 0; i < nkeys; i++) ptr[i + 1] += ptr[i];
    order.assign(key.size(), 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < key.size(); i++) order[fill[key[i]]++] = (int32_t)i;
}

void build_kkt_maps(opf_model* M) {
    const int n = M->n, m = M->m;
    const int64_t nj = M->nnzj, nh = M->nnzh;
    // Jacobian rows (CSR) on the host, entries of each row in entry order
    std::vector<int64_t> key(nj);
    for (int64_t e = 0; e < nj; e++) key[e] = M->jrow[e];
    std::vector<int32_t> jr_ptr, jr_ent;
    csr_by_key(m, key, jr_ptr, jr_ent);
    for (int64_t e = 0; e < nj; e++) key[e] = M->jcol[e];
    std::vector<int32_t> jt_ptr, jt_ent;
    csr_by_key(n, key, jt_ptr, jt_ent);

    // candidate contributions to K entries: (col * n + row) keys
    struct Item {
        int64_t key;
        int32_t kind;  // 0 diag, 1 hessian entry, 2 jacobian pair
        int32_t a, b, r;
    };
    std::vector<Item> items;
    size_t npairs = 0;
    for (int r = 0; r < m; r++) {
        size_t len = jr_ptr[r + 1] - jr_ptr[r];
        npairs += len * (len + 1) / 2;
    }
    items.reserve(n + nh + npairs);
    for (int i = 0; i < n; i++) items.push_back({(int64_t)i * n + i, 0, i, 0, 0});
    for (int64_t e = 0; e < nh; e++)
        items.push_back({(int64_t)M->hcol[e] * n + M->hrow[e], 1, (int32_t)e, 0, 0});
    for (int r = 0; r < m; r++) {
        for (int u = jr_ptr[r]; u < jr_ptr[r + 1]; u++) {
            int ea = jr_ent[u];
            for (int v = u; v < jr_ptr[r + 1]; v++) {
                int eb = jr_ent[v];
                int ca = M->jcol[ea], cb = M->jcol[eb];
                int hi = std::max(ca, cb), lo = std::min(ca, cb);
                items.push_back({(int64_t)lo * n + hi, 2, ea, eb, r});
            }
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) {
        return x.key != y.key ? x.key < y.key : x.kind < y.kind;
    });
    std::vector<int32_t> colptr(n + 1, 0), rowind;
    std::vector<int32_t> hptr{0}, hidx, pptr{0}, pa, pb, pr, kdiag;
    int64_t prev = -1;
    for (const Item& it : items) {
        if (it.key != prev) {
            if (prev >= 0) {
                hptr.push_back((int32_t)hidx.size());
                pptr.push_back((int32_t)pa.size());
            }
            prev = it.key;
            int col = (int)(it.key / n), row = (int)(it.key % n);
            rowind.push_back(row);
            colptr[col + 1]++;
            kdiag.push_back(row == col ? col : -1);
        }
        if (it.kind == 1) hidx.push_back(it.a);
        if (it.kind == 2) {
            pa.push_back(it.a);
            pb.push_back(it.b);
            pr.push_back(it.r);
        }
    }
    hptr.push_back((int32_t)hidx.size());
    pptr.push_back((int32_t)pa.size());
    for (int j = 0; j < n; j++) colptr[j + 1] += colptr[j];
    M->kcolptr = colptr;
    M->krowind = rowind;
    M->nnzk = (int64_t)rowind.size();
    M->dev.upload(M->k_hptr, hptr);
    M->dev.upload(M->k_hidx, hidx);
    M->dev.upload(M->k_pptr, pptr);
    M->dev.upload(M->k_pa, pa);
    M->dev.upload(M->k_pb, pb);
    M->dev.upload(M->k_pr, pr);
    M->dev.upload(M->k_diag, kdiag);
    M->dev.upload(M->j_row, M->jrow);
    M->dev.upload(M->j_col, M->jcol);
    M->dev.upload(M->jt_ptr, jt_ptr);
    M->dev.upload(M->jt_ent, jt_ent);
    M->dev.upload(M->jr_ptr, jr_ptr);
    M->dev.upload(M->jr_ent, jr_ent);
    // symmetric Hessian product map
    std::vector<int64_t> wkey;
    std::vector<int32_t> went_all, woth_all;
    wkey.reserve(2 * nh);
    for (int64_t e = 0; e < nh; e++) {
        wkey.push_back(M->hrow[e]);
        went_all.push_back((int32_t)e);
        woth_all.push_back(M->hcol[e]);
        if (M->hrow[e] != M->hcol[e]) {
            wkey.push_back(M->hcol[e]);
            went_all.push_back((int32_t)e);
            woth_all.push_back(M->hrow[e]);
        }
    }
    std::vector<int32_t> wptr, worder;
    csr_by_key(n, wkey, wptr, worder);
    std::vector<int32_t> went(worder.size()), woth(worder.size());
    for (size_t k = 0; k < worder.size(); k++) {
        went[k] = went_all[worder[k]];
        woth[k] = woth_all[worder[k]];
    }
    M->dev.upload(M->w_ptr, wptr);
    M->dev.upload(M->w_ent, went);
    M->dev.upload(M->w_oth, woth);
}

}  // namespace opf

using namespace opf;

extern "C" int kkt_pattern(const opf_model* M, int32_t* colptr, int32_t* rowind) {
    return guarded([&] {
        OPF_CHECK(M, OPF_E_INVALID, "kkt_pattern: null model");
        if (colptr) memcpy(colptr, M->kcolptr.data(), M->kcolptr.size() * 4);
        if (rowind) memcpy(rowind, M->krowind.data(), M->krowind.size() * 4);
    });
}

extern "C" int kkt_condense(opf_model* M, const double* hess, const double* jac, const double* sigx,
                            const double* dvec, double dw, double* kval, const double* qx, const double* v,
                            double* rhs, void* stream) {
    return guarded([&] {
        OPF_CHECK(M && hess && jac && sigx && dvec && kval, OPF_E_INVALID, "kkt_condense: null argument");
        OPF_CHECK((qx && v && rhs) || (!qx && !v && !rhs), OPF_E_INVALID,
                  "kkt_condense: qx, v and rhs must be all set or all NULL");
        hipStream_t s = (hipStream_t)stream;
        condense(M, hess, jac, sigx, dvec, dw, kval, s);
        if (rhs) jt_times(M, jac, v, qx, rhs, s);
    });
}
