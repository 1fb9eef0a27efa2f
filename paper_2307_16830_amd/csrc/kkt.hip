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

// ---------------------------------------------------------------- segmented wave gathers
// Every output of a gather (an entry of K, a row of J x, ...) is the sum of its terms.  The terms are stored
// sorted by output, 64 to a chunk, so that a wave reads its lanes' term codes with one coalesced load and
// each lane evaluates one term; the lanes of a chunk are then summed per output by a segmented inclusive
// scan (six shuffle steps, fixed order), the partial sum of an output that continues into the next chunk
// is carried to that chunk's lane 0, and the lane holding an output's last term writes it.  Work per wave
// is balanced by term count, not by output, and the summation order is fixed (bitwise reproducible).
constexpr int SEG_CPW = 4;  // chunks per wave range (a range is extended to the next output boundary)

// Condensed-assembly term codes (all fields unsigned): a Jacobian pair term J_a D_r J_b packs a (22 bits),
// b (22 bits), r (20 bits); r = KT_HESS marks a Hessian entry h (44 bits), r = KT_DIAG the diagonal of column
// c (sigma_x[c] + dw).
constexpr uint64_t KT_HESS = 0xFFFFF, KT_DIAG = 0xFFFFE, KT_ZERO = 0xFFFFD;  // KT_ZERO: padding, value 0

// Evaluated without branches: every lane issues its three loads at once (lanes of other kinds read entry 0,
// which every model has, and discard it), so a chunk costs one memory round trip whatever its mix of kinds.
struct KEval {
    const double *jac, *dvec, *hess, *sigx;
    double dw;
    __device__ __forceinline__ double operator()(uint64_t u) const {
        const uint64_t r = u >> 44;
        const bool hs = r == KT_HESS, dg = r == KT_DIAG, pr = r < KT_ZERO;
        const double* p1 = hs ? hess + (u & 0xFFFFFFFFFFFull) : dg ? sigx + (u & 0x3FFFFF) : jac + (pr ? u & 0x3FFFFF : 0);
        const double x1 = *p1;
        const double x2 = dvec[pr ? r : 0];
        const double x3 = jac[pr ? (u >> 22) & 0x3FFFFF : 0];
        asm volatile("" ::"v"(x1), "v"(x2), "v"(x3));  // keeps the compiler from sinking the loads into branches
        const double prod = (x1 * x2) * x3;  // J_a D_r J_b, in that order
        return pr ? prod : dg ? x1 + dw : hs ? x1 : 0.0;
    }
};

// a[lo 32 bits] * b[hi 32 bits]; the code PROD_ZERO (an output without terms) evaluates to 0
constexpr uint64_t PROD_ZERO = ~0ull;
struct ProdEval {
    const double *a, *b;
    __device__ __forceinline__ double operator()(uint64_t u) const {
        const bool z = u == PROD_ZERO;
        const double xa = a[z ? 0u : (uint32_t)u], xb = b[z ? 0u : (uint32_t)(u >> 32)];
        asm volatile("" ::"v"(xa), "v"(xb));  // both loads in flight together, whatever the lane's kind
        return z ? 0.0 : xa * xb;
    }
};

template <class Eval>
__global__ __launch_bounds__(KB) void seg_gather(int nwaves, const int32_t* __restrict__ wptr,
                                                 const uint64_t* __restrict__ term,
                                                 const uint64_t* __restrict__ smask,
                                                 const uint64_t* __restrict__ emask,
                                                 const int32_t* __restrict__ base,
                                                 const int32_t* __restrict__ segout, Eval ev,
                                                 const double* __restrict__ add, double* __restrict__ out) {
    const int w = blockIdx.x * (KB / 64) + threadIdx.x / 64;
    if (w >= nwaves) return;
    const int lane = threadIdx.x % 64;
    const uint64_t below = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // lanes 0..lane
    double carry = 0.0;
    // the chunk range and each chunk's masks and first output are wave-uniform (scalar loads); the next chunk's
    // term codes are fetched while the current chunk's values are gathered, and the output index of a lane
    // that ends a segment is looked up together with those values
    const int c0 = __builtin_amdgcn_readfirstlane(wptr[w]), c1 = __builtin_amdgcn_readfirstlane(wptr[w + 1]);
    uint64_t tn = term[(int64_t)c0 * 64 + lane], smn = smask[c0], emn = emask[c0];
    int bn = base[c0];
    for (int c = c0; c < c1; c++) {
        const uint64_t t = tn, sm = smn, em = emn;
        const int bs = bn;
        if (c + 1 < c1) {
            tn = term[(int64_t)(c + 1) * 64 + lane];
            smn = smask[c + 1];
            emn = emask[c + 1];
            bn = base[c + 1];
        }
        const bool ends = (em >> lane) & 1;
        const int so = bs + __popcll(sm & below & ~1ull);  // segment (output) ordinal
        const int o = segout && ends ? segout[so] : so;
        double v = ev(t);
        int f = (int)((sm >> lane) & 1);
        if (lane == 0 && !f) v += carry;  // the output continued from the previous chunk
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double vp = __shfl_up(v, d);
            const int fp = __shfl_up(f, d);
            if (lane >= d) {
                if (!f) v += vp;
                f |= fp;
            }
        }
        if (ends) out[o] = add ? add[o] + v : v;
        carry = __shfl(v, 63);
    }
}

// Build a SegList from (output, code) pairs grouped by output (consecutive terms of one output form its segment).
// Segments in increasing output order need no map; any other order (chosen for the locality of the terms' reads)
// gets segout, the output of each segment.  Wave ranges are SEG_CPW chunks long and
// begin at a chunk boundary: an output that would straddle a range boundary is moved to the next range, the
// gap filled with `zero_code` terms (value 0, no start or end bit), so no output is split between waves
// except one longer than a whole range, which extends its range.
void build_seglist(SegList& L, const std::vector<int32_t>& outs, const std::vector<uint64_t>& codes,
                   uint64_t zero_code, Deferred& dev) {
    const int64_t n_in = (int64_t)codes.size();
    const int64_t RW = (int64_t)SEG_CPW * 64;  // terms per range
    std::vector<uint64_t> term;
    std::vector<int32_t> tout;     // segment ordinal of each placed term (-1 for padding)
    std::vector<int32_t> segs;     // output of each segment
    bool ordered = true;
    std::vector<char> first, last;  // term starts / ends its output
    term.reserve(n_in + n_in / 8 + 64);
    for (int64_t t = 0; t < n_in;) {
        int64_t u = t;
        while (u < n_in && outs[u] == outs[t]) u++;  // terms [t, u) form one output
        const int64_t len = u - t, pos = (int64_t)term.size(), off = pos % RW;
        if (off != 0 && len <= RW && off + len > RW)
            for (int64_t q = off; q < RW; q++) {
                term.push_back(zero_code);
                tout.push_back(-1);
                first.push_back(0);
                last.push_back(0);
            }
        if (!segs.empty() && outs[t] != segs.back() + 1) ordered = false;
        if (segs.empty() && outs[t] != 0) ordered = false;
        for (int64_t q = t; q < u; q++) {
            term.push_back(codes[q]);
            tout.push_back((int32_t)segs.size());
            first.push_back(q == t);
            last.push_back(q == u - 1);
        }
        segs.push_back(outs[t]);
        t = u;
    }
    const int64_t nt = (int64_t)term.size();
    const int64_t nch = (nt + 63) / 64;
    term.resize(nch * 64, zero_code);
    std::vector<uint64_t> sm(nch, 0), em(nch, 0);
    std::vector<int32_t> base(nch, 0), wptr{0};
    for (int64_t t = 0; t < nt; t++) {
        const int64_t c = t / 64, l = t % 64;
        if (first[t]) sm[c] |= 1ull << l;
        if (last[t]) em[c] |= 1ull << l;
    }
    // a chunk's base is the output of its lane 0 (padding only ever ends a range, so a chunk is either all
    // padding, whose base is never used, or starts with a real term)
    for (int64_t c = 0; c < nch; c++) base[c] = c * 64 < nt && tout[c * 64] >= 0 ? tout[c * 64] : 0;
    for (int64_t c = 0; c < nch;) {
        int64_t e = std::min(nch, c + SEG_CPW);
        while (e < nch && !(sm[e] & 1) && tout[e * 64] >= 0) e++;  // only an output longer than a range
        wptr.push_back((int32_t)e);
        c = e;
    }
    L.nwaves = (int)wptr.size() - 1;
    L.nterms = n_in;
    dev.upload(L.term, term);
    dev.upload(L.smask, sm);
    dev.upload(L.emask, em);
    dev.upload(L.base, base);
    dev.upload(L.wptr, wptr);
    if (!ordered) dev.upload(L.segout, segs);
}

template <class Eval>
static void run_seg(const SegList& L, Eval ev, const double* add, double* out, hipStream_t s) {
    if (L.nwaves == 0) return;
    hipLaunchKernelGGL(seg_gather<Eval>, dim3(ceil_div(L.nwaves, KB / 64)), dim3(KB), 0, s, L.nwaves, L.wptr.p,
                       L.term.p, L.smask.p, L.emask.p, L.base.p, L.segout.p, ev, add, out);
    OPF_LAUNCH_CHECK();
}

void condense(const opf_model* M, const double* hess, const double* jac, const double* sigx, const double* dvec,
              double dw, double* kval, hipStream_t s) {
    ensure_device(M);
    if (M->nnzk == 0) return;
    if (M->seg_k_ok) {
        run_seg(M->seg_k, KEval{jac, dvec, hess, sigx, dw}, nullptr, kval, s);
        return;
    }
    hipLaunchKernelGGL(kkt_gather, dim3(ceil_div(M->nnzk, KB)), dim3(KB), 0, s, M->nnzk, M->k_hptr.p, M->k_hidx.p,
                       M->k_pptr.p, M->k_pa.p, M->k_pb.p, M->k_pr.p, M->k_diag.p, hess, jac, sigx, dvec, dw, kval);
    OPF_LAUNCH_CHECK();
}

void jt_times(const opf_model* M, const double* jac, const double* v, const double* base, double* out,
              hipStream_t s) {
    ensure_device(M);
    if (M->seg_jtv.nwaves) {
        run_seg(M->seg_jtv, ProdEval{jac, v}, base, out, s);
        return;
    }
    hipLaunchKernelGGL(csr_gather_mv, dim3(ceil_div(M->n, KB)), dim3(KB), 0, s, M->n, M->jt_ptr.p, M->jt_ent.p,
                       M->j_row.p, jac, v, base, out);
    OPF_LAUNCH_CHECK();
}

void j_times(const opf_model* M, const double* jac, const double* x, double* out, hipStream_t s) {
    ensure_device(M);
    if (M->seg_jx.nwaves) {
        run_seg(M->seg_jx, ProdEval{jac, x}, nullptr, out, s);
        return;
    }
    hipLaunchKernelGGL(csr_gather_mv, dim3(ceil_div(M->m, KB)), dim3(KB), 0, s, M->m, M->jr_ptr.p, M->jr_ent.p,
                       M->j_col.p, jac, x, (const double*)nullptr, out);
    OPF_LAUNCH_CHECK();
}

void w_times(const opf_model* M, const double* hess, const double* x, double* out, hipStream_t s) {
    ensure_device(M);
    if (M->seg_wx.nwaves) {
        run_seg(M->seg_wx, ProdEval{hess, x}, nullptr, out, s);
        return;
    }
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

    // candidate contributions to K entries, keyed by their (column, row) in the lower triangle
    struct Item {
        int32_t col, row;
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
    for (int i = 0; i < n; i++) items.push_back({i, i, 0, i, 0, 0});
    for (int64_t e = 0; e < nh; e++) items.push_back({M->hcol[e], M->hrow[e], 1, (int32_t)e, 0, 0});
    for (int r = 0; r < m; r++) {
        for (int u = jr_ptr[r]; u < jr_ptr[r + 1]; u++) {
            int ea = jr_ent[u];
            for (int v = u; v < jr_ptr[r + 1]; v++) {
                int eb = jr_ent[v];
                int ca = M->jcol[ea], cb = M->jcol[eb];
                int hi = std::max(ca, cb), lo = std::min(ca, cb);
                items.push_back({lo, hi, 2, ea, eb, r});
            }
        }
    }
    // ordered by (column, row), equal keys by kind (the push order above: diagonal, Hessian entries, pairs):
    // a stable bucketing by column, then each column's few items stably by row (a comparison sort of all the
    // items, and then two scattering passes, dominated the model's host set-up)
    {
        std::vector<int64_t> cptr(n + 1, 0);
        for (const Item& it : items) cptr[it.col + 1]++;
        for (int i = 0; i < n; i++) cptr[i + 1] += cptr[i];
        std::vector<Item> tmp(items.size());
        {
            std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
            for (const Item& it : items) tmp[fill[it.col]++] = it;
        }
        const auto by_row = [](const Item& x, const Item& y) { return x.row < y.row; };
        for (int j = 0; j < n; j++) {
            Item* b = tmp.data() + cptr[j];
            Item* e = tmp.data() + cptr[j + 1];
            if (e - b > 32) {
                std::stable_sort(b, e, by_row);
                continue;
            }
            for (Item* p = b + 1; p < e; p++)  // insertion sort: stable, no allocation
                for (Item* q = p; q > b && by_row(q[0], q[-1]); q--) std::swap(q[0], q[-1]);
        }
        items.swap(tmp);
    }
    std::vector<int32_t> colptr(n + 1, 0), rowind;
    std::vector<int32_t> hptr{0}, hidx, pptr{0}, pa, pb, pr, kdiag;
    int prow = -1, pcol = -1;
    for (const Item& it : items) {
        if (it.col != pcol || it.row != prow) {
            if (pcol >= 0) {
                hptr.push_back((int32_t)hidx.size());
                pptr.push_back((int32_t)pa.size());
            }
            pcol = it.col;
            prow = it.row;
            const int col = it.col, row = it.row;
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

    if (M->per_entry_assembly) return;
    // segmented gathers (an output without terms gets one PROD_ZERO term, so every output is written)
    std::vector<int32_t> outs;
    std::vector<uint64_t> codes;
    auto prod_list = [&](SegList& L, int nout, const std::vector<int32_t>& ptr, auto&& code_of) {
        outs.clear();
        codes.clear();
        for (int o = 0; o < nout; o++) {
            if (ptr[o + 1] == ptr[o]) {
                outs.push_back(o);
                codes.push_back(PROD_ZERO);
            }
            for (int u = ptr[o]; u < ptr[o + 1]; u++) {
                outs.push_back(o);
                codes.push_back(code_of(u));
            }
        }
        build_seglist(L, outs, codes, PROD_ZERO, M->dev);
    };
    auto pack = [](int32_t lo, int32_t hi) { return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32); };
    prod_list(M->seg_jx, m, jr_ptr, [&](int u) { return pack(jr_ent[u], M->jcol[jr_ent[u]]); });
    prod_list(M->seg_jtv, n, jt_ptr, [&](int u) { return pack(jt_ent[u], M->jrow[jt_ent[u]]); });
    prod_list(M->seg_wx, n, wptr, [&](int u) { return pack(went[u], woth[u]); });
    M->seg_k_ok = nj < (int64_t(1) << 22) && n < (1 << 22) && m < (int)KT_ZERO && nh < (int64_t(1) << 44);
    if (M->seg_k_ok) {
        outs.clear();
        codes.clear();
        const int64_t nk = M->nnzk;
        // K slots visited by the smallest constraint row among their Jacobian pair terms (ties by slot): the
        // slots of one row are adjacent, and consecutive rows of a template family read neighbouring J, D and
        // Hessian entries (the family-major layouts), instead of one random line per read
        // (a stable counting sort: slots without pair terms take the last bucket, m)
        std::vector<int64_t> slot(nk);
        std::vector<int32_t> key(nk), cnt(m + 2, 0);
        for (int64_t k = 0; k < nk; k++) {
            int32_t r = m;
            for (int e = pptr[k]; e < pptr[k + 1]; e++) r = std::min(r, pr[e]);
            key[k] = r;
            cnt[r + 1]++;
        }
        for (int r = 0; r <= m; r++) cnt[r + 1] += cnt[r];
        for (int64_t k = 0; k < nk; k++) slot[cnt[key[k]]++] = k;
        for (int64_t k : slot) {
            if (kdiag[k] >= 0) {
                outs.push_back((int32_t)k);
                codes.push_back((uint64_t)kdiag[k] | (KT_DIAG << 44));
            }
            for (int e = hptr[k]; e < hptr[k + 1]; e++) {
                outs.push_back((int32_t)k);
                codes.push_back((uint64_t)hidx[e] | (KT_HESS << 44));
            }
            for (int e = pptr[k]; e < pptr[k + 1]; e++) {
                outs.push_back((int32_t)k);
                codes.push_back((uint64_t)pa[e] | ((uint64_t)pb[e] << 22) | ((uint64_t)pr[e] << 44));
            }
        }
        build_seglist(M->seg_k, outs, codes, KT_ZERO << 44, M->dev);
    }
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
