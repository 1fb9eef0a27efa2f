// Internal layout of an opf_model: template parameter arrays (structure of
// arrays, one entry per template instance), fixed derivative structure and
// the condensed-matrix assembly maps.
#pragma once

#include "common.h"

namespace opf {
// Terms of a gather sorted by their output index, for the segmented wave gathers of kkt.hip: 64 terms per
// chunk (one per lane), a chunk's lanes reduced by a segmented scan, each wave walking a range of chunks that
// starts at an output boundary.  A term is a 64-bit code interpreted by the gather's evaluator.
struct SegList {
    DBuf<uint64_t> term;          // [nchunks * 64]
    DBuf<uint64_t> smask, emask;  // [nchunks]: bit l set if term l is the first / last term of its output
    DBuf<int32_t> base;           // [nchunks]: output (or, with segout, segment ordinal) of the chunk's first term
    DBuf<int32_t> segout;         // [nsegments] output of each segment when segments are not in output order
    DBuf<int32_t> wptr;           // [nwaves + 1]: chunk range of each wave
    int nwaves = 0;
    int64_t nterms = 0;
};
}  // namespace opf

struct opf_model {
    int N = 0, E = 0, G = 0, ref = 0;
    int n = 0, m = 0;
    int64_t nnzj = 0, nnzh = 0, nnzk = 0;

    // ---- host copies of structure and bounds
    std::vector<double> xl, xu, gl, gu, x0;
    std::vector<int32_t> jrow, jcol, hrow, hcol;
    std::vector<int32_t> kcolptr, krowind;  // lower CSC pattern of K

    // ---- device template data
    opf::DBuf<int32_t> ai, aj;        // arc from-end / to-end bus [2E]
    opf::DBuf<double> ag, ab, abc;    // arc series g, b and end charging [2E]
    opf::DBuf<double> pd, qd, gs, bs; // bus data [N]
    opf::DBuf<int32_t> bus_arc_ptr, bus_arc;  // arcs leaving each bus (CSR, [N+1], [2E])
    opf::DBuf<int32_t> bus_gen_ptr, bus_gen;  // generators at each bus (CSR, [N+1], [G])
    opf::DBuf<double> c2, c1, c0;     // generator cost on per-unit pg [G]
    opf::DBuf<int32_t> gbus;          // generator bus [G]
    opf::DBuf<double> fpart;          // objective reduction scratch [1]

    // ---- device condensed-assembly maps (gather form, no atomics)
    opf::DBuf<int32_t> k_hptr, k_hidx;       // K slot -> Hessian entries
    opf::DBuf<int32_t> k_pptr, k_pa, k_pb, k_pr;  // K slot -> Jacobian pair terms (a, b, row)
    opf::DBuf<int32_t> k_diag;               // K slot -> column if diagonal else -1
    // Jacobian access paths
    opf::DBuf<int32_t> j_row, j_col;         // entry -> row / column [nnzj]
    opf::DBuf<int32_t> jt_ptr, jt_ent;       // CSC: column -> entries
    opf::DBuf<int32_t> jr_ptr, jr_ent;       // CSR: row -> entries
    // symmetric Hessian product: row -> (entry, other index)
    opf::DBuf<int32_t> w_ptr, w_ent, w_oth;
    // segmented gathers: condensed assembly (when its codes fit: nnz_jac < 2^22, m < 2^20 - 2), J x, J^T v, W x
    bool per_entry_assembly = false;  // opf_options.assembly == 1: keep the per-entry gather lists only
    bool seg_k_ok = false;
    opf::SegList seg_k, seg_jx, seg_jtv, seg_wx;

    opf::Deferred dev;  // pending uploads, run at the first device use
};

namespace opf {

// Jacobian entry offsets (see opf_structure): ref, flow blocks, angle, thermal, balance.
struct JLayout {
    int64_t ref, flow, ang, th, bal_pvm, bal_qvm, bal_parc, bal_qarc, bal_pg, bal_qg, total;
    __host__ __device__ JLayout(int N, int E, int G) {
        int64_t A = 2LL * E;
        ref = 0;
        flow = 1;              // 10 blocks of 2E: p-row [p, va_i, va_j, vm_i, vm_j], q-row [...]
        ang = flow + 10 * A;   // 2 blocks of E
        th = ang + 2LL * E;    // 2 blocks of 2E
        bal_pvm = th + 2 * A;  // N
        bal_qvm = bal_pvm + N; // N
        bal_parc = bal_qvm + N;   // 2E
        bal_qarc = bal_parc + A;  // 2E
        bal_pg = bal_qarc + A;    // G
        bal_qg = bal_pg + G;      // G
        total = bal_qg + G;
    }
};

// Hessian entry offsets: 10 blocks of 2E per flow kind, thermal, balance, generator.
struct HLayout {
    int64_t pflow, qflow, th, bal_p, bal_q, gen, total;
    __host__ __device__ HLayout(int N, int E, int G) {
        int64_t A = 2LL * E;
        pflow = 0;
        qflow = 10 * A;
        th = 20 * A;
        bal_p = th + 2 * A;
        bal_q = bal_p + N;
        gen = bal_q + N;
        total = gen + G;
    }
};

struct RowLayout {
    int64_t ref, p, q, ang, th, pb, qb;
    __host__ __device__ RowLayout(int N, int E) {
        ref = 0;
        p = 1;
        q = 1 + 2LL * E;
        ang = 1 + 4LL * E;
        th = 1 + 5LL * E;
        pb = 1 + 7LL * E;
        qb = pb + N;
    }
};

// Internal evaluation entry used by the C ABI and the IPM.  cscale (nullable)
// multiplies each constraint row (values, Jacobian rows and the multipliers
// entering the Hessian); gscale multiplies f and its gradient.
void eval_derivs(const opf_model* M, unsigned what, const double* x, const double* y, double obj_weight,
                 const double* cscale, double gscale, double* f, double* c, double* grad, double* jac,
                 double* hess, hipStream_t s);

// Condensed assembly: kval = H + dw I + sigx + J^T diag(dvec) J on the K pattern.
void condense(const opf_model* M, const double* hess, const double* jac, const double* sigx, const double* dvec,
              double dw, double* kval, hipStream_t s);
// out[j] = base[j] (nullable) + sum_e jac[e] v[row(e)]  (J^T v)
void jt_times(const opf_model* M, const double* jac, const double* v, const double* base, double* out,
              hipStream_t s);
// out[r] = sum_e jac[e] x[col(e)]  (J x)
void j_times(const opf_model* M, const double* jac, const double* x, double* out, hipStream_t s);
// out[i] = sum W_ij x_j for the symmetric Hessian given by its lower COO values
void w_times(const opf_model* M, const double* hess, const double* x, double* out, hipStream_t s);

void build_kkt_maps(opf_model* M);
inline void ensure_device(const opf_model* M) { const_cast<opf_model*>(M)->dev.run(); }

}  // namespace opf
