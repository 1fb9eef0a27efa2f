// Pivot-free supernodal (multifrontal) Cholesky of the condensed matrix and
// its triangular solves (Section IV-C: the condensed matrix is factored with a
// fixed pivot sequence because it is positive definite once the inertia is
// right).
//
// Numeric layout: supernode s owns a dense front F_s of m_s x m_s (m_s =
// number of rows of the supernode, its n_s own columns first), of which only
// the lower part is stored, as a block trapezoid of 64-column panels (fcol
// below).  After the partial factorization the first n_s columns hold L's
// panel and the trailing (m_s - n_s) block holds the update matrix passed to
// the parent.
// Fronts are processed by elimination-tree level (leaves first); all fronts
// of a level are independent and run in the same launches:
//   * assembly: one work-group per 64x64 lower tile of a front gathers the
//     entries of K that land in the tile and the children's update-matrix
//     blocks that map into it (relative indices are monotone, so each child
//     contributes one rectangle found by binary search).  No atomics: each
//     tile is owned by one work-group.
//   * fronts with m_s <= 64: the whole front lives in LDS, one work-group
//     factors it (column Cholesky with the Schur update of the trailing block).
//   * larger fronts: right-looking blocked partial factorization with 64-wide
//     panels: diagonal-block Cholesky in LDS, panel triangular solve, and a
//     trailing symmetric rank-64 update on FP64 MFMA (16x16x4) tiles.
// The solves walk the levels upward (each front gathers its children's
// partial results, solves with its diagonal block and forms its own partial
// result for the parent) and then downward (each front gathers the already
// computed solution at its off-diagonal rows).
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "model.h"
#include "symbolic.h"

using namespace opf;

constexpr int NCAT = 6;  // timing categories: assembly, small fronts, diagonal block, panel solve, trailing update,
                         // dense-front tile launch

struct chol_sym {
    Symbolic S;
    chol_options opts{};
    int n = 0;
    int64_t nnzk = 0;
    int nlevels = 0;
    int64_t front_total = 0, nnzl = 0, upd_total = 0;
    double flops = 0;
    bool factored = false;
    // host mirrors
    std::vector<int32_t> h_first, h_ncol, h_mrows, h_level;
    std::vector<int64_t> h_foff, h_roff, h_uoff;
    std::vector<int32_t> lvl_ptr, lvl_sn;           // supernodes by level
    std::vector<int32_t> lvl_small_ptr, lvl_small;  // fronts with m <= 64 by level
    std::vector<int32_t> lvl_small_maxm;            // largest of them, 0 when the level has larger fronts too
    std::vector<int32_t> lvl_small_lda;             // largest of them
    std::vector<int32_t> lvl_narrow_ptr, lvl_narrow;  // fronts solved by one work-group, by level
    std::vector<int32_t> lvl_narrow_maxm;             // largest front of each level's list (<= 64: one-wave sweeps)
    // narrow fronts with many rows below their pivots ("tall"): the sweeps' products with those rows run as
    // separate launches over row blocks (forward) and 16-column blocks (backward), items (front, block)
    std::vector<int32_t> lvl_trow_ptr, lvl_tcol_ptr, trow_it, tcol_it;
    std::vector<int32_t> lvl_wide_ptr, lvl_wide;      // fronts with >= WIDE pivots, by level
    // assembly tile work list (per level)
    std::vector<int32_t> asm_ptr;                  // [nlevels+1] into tiles
    // blocked steps: per (level, step) ranges into the three item lists
    struct Step {
        int level;
        int32_t p0, p1, t0, t1;
        int32_t s0, s1;  // trailing-update tiles of the next panel's 64 columns
        int32_t r0, r1;  // trailing-update tiles of the columns after it
        int32_t kw;      // columns of L applied by the trailing update (64, or up to 128 for a panel pair)
    };
    std::vector<Step> steps;
    std::vector<int32_t> lvl_step_ptr;
    // device
    DBuf<int32_t> first, ncol, mrows, perm;
    DBuf<int32_t> kdiagpos;  // pivot -> position of its diagonal entry in K's values
    DBuf<int64_t> foff, roff, uoff;
    DBuf<int32_t> rows;
    DBuf<int32_t> child_ptr, child;
    DBuf<int64_t> rel_off;
    DBuf<int64_t> gptr, gsrc;  // per front row (roff order): its children's update entries (indices into upd),
                               // children in ascending order
    DBuf<int32_t> rel;
    DBuf<int32_t> tile_sn, tile_rc;  // tile work list: supernode, (tr << 16) | tc
    DBuf<int64_t> tile_cptr;         // per tile: its child rectangles in tile_crec
    DBuf<int32_t> tile_crec;         // (child, ra, rb, ca, cb) per contributing child
    DBuf<int64_t> tile_kptr;
    DBuf<int32_t> tile_k, tile_kpos;
    DBuf<int32_t> lvl_sn_d, lvl_small_d, lvl_narrow_d, lvl_wide_d;
    DBuf<int32_t> trow_d, tcol_d;
    DBuf<int32_t> potrf_it, trsm_it, syrk_it;  // packed items
    DBuf<int32_t> next_slot;  // per trailing-update item: slot of the next panel's diagonal block, or -1

    DBuf<int32_t> status;
    DBuf<int32_t> level_d;    // elimination level of each supernode
    DBuf<int64_t> statwords;  // [0]: first rejected pivot as (level << 32 | pivot), INT64_MAX if none;
                              // [1]: negative pivots of an L D L^T factorization
    DBuf<double> dval;        // L D L^T: the pivots, in pivot order
    int64_t last_nneg = 0;    // negative pivots of the last L D L^T factorization
    // host words the factorization status and the fault words are read into: pinned memory lent by the
    // owning IPM (chol_bind_host), else allocated at the first factorization
    int64_t* hwords = nullptr;
    bool own_hwords = false;
    DBuf<double> fronts, upd, work, ybuf;
    DBuf<double> ldiag, rdiag;  // compact diagonal blocks and reciprocal pivots of one blocked step
    // sync-free solves of wide fronts
    std::vector<int64_t> h_flag_off;  // per supernode (wide fronts only): offset of its blocks in zx
    DBuf<double> zx;                  // solved 64-blocks of the wide fronts' sweeps
    DBuf<double> winv;                // inverses of the wide fronts' 64 x 64 diagonal blocks (4096 doubles each)
    DBuf<int32_t> winv_it;            // per block: (supernode, block, block index in winv)
    int nwinv = 0;
    DBuf<int32_t> sfault;
    Deferred dev;  // pending uploads, run at the first device use
    // optional per-category kernel timing (assemble, small, potrf, trsm, syrk): bit mask of categories
    int timing = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_cat;
    size_t ev_used = 0;
    double t_ms[NCAT] = {};
    int64_t t_launch[NCAT] = {};
    double t_flops[NCAT] = {};
    double t_bytes[NCAT] = {};
    // dense fronts (ncol >= DENSE_MIN): one dependency-driven tile launch per level
    std::vector<int32_t> lvl_dense_ptr;  // [nlevels + 1] task ranges
    std::vector<double> lvl_dense_flops;  // factorization flops of the level's dense fronts
    std::vector<char> is_dense;          // per supernode
    int dense_grid = 0;
    int32_t epoch = 0;
    DBuf<int32_t> dh_s, dh_np, dh_nb, dh_slot0, dtask_h, dtask_rc, dflags, dcounter, ffault;
    DBuf<int64_t> dh_t0;
    DBuf<double> tdiag, trdiag;
    std::vector<double> step_syrk_flops;  // algorithmic flops of each blocked step's trailing update
    std::vector<double> step_syrk_bytes;  // and its algorithmic HBM bytes (C read + written, panel read once)
    // HIP graphs of the factorization and solve launch sequences, replayed instead of re-enqueued (set by the
    // IPM for its own non-null stream): key = (stream, first pointer, second pointer, pivot tolerance)
    struct GraphEntry {
        hipStream_t st;
        const void *a, *b;
        double tol;
        hipGraphExec_t exec;
    };
    bool use_graphs = false;
    std::vector<GraphEntry> graphs;
    ~chol_sym() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        if (own_hwords && hwords) (void)hipHostFree(hwords);
    }
};

namespace {

constexpr int TB = 64;      // tile edge
constexpr int NT = 256;     // threads per work-group

// Front storage.  The columns of an m-row front are cut into 64-column panels; panel p is a column-major
// block of m - 64p rows starting at row 64p, and the panels follow one another.  Entry (r, c) with
// r >= 64 floor(c / 64) (every lower entry; of the strictly upper part only the upper halves of the 64 x 64
// diagonal blocks take memory, and they are never read) is at fcol(m, c) + r, and within a panel column
// c + 1 follows column c at the panel's row count fld(m, c).  A front of at most 64 rows is a plain
// column-major square.
static_assert(TB == 64, "the front layout's panels are the 64-column blocks");
__host__ __device__ __forceinline__ int64_t fcol(int64_t m, int c) {
    const int64_t p = c >> 6;
    return p * (64 * m - 2048 * (p - 1)) + (int64_t)(c - 64 * p) * (m - 64 * p) - 64 * p;
}
__host__ __device__ __forceinline__ int64_t fld(int64_t m, int c) { return m - (c & ~63); }
// doubles of an m-row front
inline int64_t front_doubles(int64_t m) {
    const int64_t P = (m - 1) >> 6, w = m - 64 * P;
    return fcol(m, (int)(64 * P)) + 64 * P + w * w;
}


// ---------------------------------------------------------------- assembly
// One work-group per 64 x 64 lower tile of a front: the tile is built in LDS from the entries of K that land
// in it and from the rectangles of the children's update matrices that map into it (listed per tile at
// analysis time, children in ascending order), then written to the front.  No atomics.
__global__ __launch_bounds__(NT) void front_assemble(int tile0, const int32_t* __restrict__ tile_sn,
                                                     const int32_t* __restrict__ tile_rc,
                                                     const int64_t* __restrict__ tile_kptr,
                                                     const int32_t* __restrict__ tile_k,
                                                     const int32_t* __restrict__ tile_kpos,
                                                     const double* __restrict__ kval, const int32_t* __restrict__ ncol,
                                                     const int32_t* __restrict__ mrows,
                                                     const int64_t* __restrict__ foff,
                                                     const int64_t* __restrict__ tile_cptr,
                                                     const int32_t* __restrict__ tile_crec,
                                                     const int64_t* __restrict__ rel_off,
                                                     const int32_t* __restrict__ rel, double* __restrict__ fronts) {
    __shared__ double T[TB * TB];
    __shared__ int64_t coff[TB];  // per column of the current child rectangle: where its update entries start
    const int item = tile0 + blockIdx.x;
    const int s = tile_sn[item];
    const int tr = tile_rc[item] >> 16, tc = tile_rc[item] & 0xffff;
    const int m = mrows[s];
    const int r0 = tr * TB, c0 = tc * TB;
    for (int e = threadIdx.x; e < TB * TB; e += NT) T[e] = 0.0;
    __syncthreads();
    for (int64_t e = tile_kptr[item] + threadIdx.x; e < tile_kptr[item + 1]; e += NT) T[tile_kpos[e]] = kval[tile_k[e]];
    __syncthreads();
    for (int64_t q = tile_cptr[item]; q < tile_cptr[item + 1]; q++) {
        const int32_t* rec = tile_crec + 5 * q;
        const int c = rec[0], ra = rec[1], rb = rec[2], ca = rec[3], cb = rec[4];
        const int nc = ncol[c], mc = mrows[c];
        const int32_t* rl = rel + rel_off[c];
        const int nr = rb - ra, ncc = cb - ca;  // ncc <= 64: the columns map to distinct columns of the tile
        if (threadIdx.x < ncc) coff[threadIdx.x] = foff[c] + fcol(mc, nc + ca + threadIdx.x) + nc;
        __syncthreads();
        for (int e = threadIdx.x; e < nr * ncc; e += NT) {
            const int ui = ra + e % nr, uj = ca + e / nr;
            if (ui >= uj) {
                const double u = fronts[coff[uj - ca] + ui];
                T[(rl[ui] - r0) + TB * (rl[uj] - c0)] += u;
            }
        }
        __syncthreads();
    }
    double* F = fronts + foff[s] + fcol(m, c0);  // the tile's columns lie in one panel
    const int64_t ld = fld(m, c0);
    for (int e = threadIdx.x; e < TB * TB; e += NT) {
        const int i = r0 + e % TB, j = c0 + e / TB;
        if (i < m && j < m && i >= j) F[i + ld * (j - c0)] = T[e];
    }
}

// Assembly of a level whose fronts all have at most 64 rows (one tile each, a plain square): one wave per
// front and up to `blockDim.x / 64` fronts per work-group, each in its own lda x lda square of dynamic LDS
// (lda = the level's largest front), the K entries first and then the children in order, as in
// front_assemble (so the fronts are bit for bit the same); a wave's LDS accesses are performed in order.
__global__ __launch_bounds__(NT) void front_assemble_tiny(int tile0, int nt, int lda,
                                                          const int32_t* __restrict__ tile_sn,
                                                          const int64_t* __restrict__ tile_kptr,
                                                          const int32_t* __restrict__ tile_k,
                                                          const int32_t* __restrict__ tile_kpos,
                                                          const double* __restrict__ kval,
                                                          const int32_t* __restrict__ ncol,
                                                          const int32_t* __restrict__ mrows,
                                                          const int64_t* __restrict__ foff,
                                                          const int64_t* __restrict__ tile_cptr,
                                                          const int32_t* __restrict__ tile_crec,
                                                          const int64_t* __restrict__ rel_off,
                                                          const int32_t* __restrict__ rel, double* __restrict__ fronts) {
    extern __shared__ double lds_a[];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64, nw = blockDim.x / 64;
    const int q = blockIdx.x * nw + wv;
    if (q >= nt) return;
    double* T = lds_a + (int64_t)wv * lda * lda;
    int64_t* coff = reinterpret_cast<int64_t*>(lds_a + (int64_t)nw * lda * lda) + 64 * wv;
    const int item = tile0 + q;
    const int s = tile_sn[item];
    const int m = mrows[s];
    for (int e = lane; e < lda * lda; e += 64) T[e] = 0.0;
    for (int64_t e = tile_kptr[item] + lane; e < tile_kptr[item + 1]; e += 64) {
        const int pos = tile_kpos[e];  // position in a 64 x 64 tile
        T[(pos % TB) + lda * (pos / TB)] = kval[tile_k[e]];
    }
    for (int64_t c4 = tile_cptr[item]; c4 < tile_cptr[item + 1]; c4++) {
        const int32_t* rec = tile_crec + 5 * c4;
        const int c = rec[0], ra = rec[1], rb = rec[2], ca = rec[3], cb = rec[4];
        const int nc = ncol[c], mc = mrows[c];
        const int32_t* rl = rel + rel_off[c];
        const int nr = rb - ra, ncc = cb - ca;
        if (lane < ncc) coff[lane] = foff[c] + fcol(mc, nc + ca + lane) + nc;
        for (int e = lane; e < nr * ncc; e += 64) {
            const int ui = ra + e % nr, uj = ca + e / nr;
            if (ui >= uj) {
                const double u = fronts[coff[uj - ca] + ui];
                T[rl[ui] + lda * rl[uj]] += u;
            }
        }
    }
    double* F = fronts + foff[s];
    for (int e = lane; e < m * m; e += 64) {
        const int i = e % m, j = e / m;
        if (i >= j) F[e] = T[i + lda * j];
    }
}

// ---------------------------------------------------------------- small fronts in LDS
// A pivot is accepted when it exceeds tol * |K_jj| (tol = 0: when it is positive).
struct PivotRef {
    const double* kval;
    const int32_t* kdiagpos;
    double tol;
    __device__ __forceinline__ double thresh(int pivot) const {
        return tol > 0.0 ? tol * fabs(kval[kdiagpos[pivot]]) : 0.0;
    }
};

// LDL = false: Cholesky, pivot k accepted when d > threshold, column scaled by sqrt(d).  LDL = true: the
// symmetric form L D L^T of the LU factorization with this fixed pivot sequence (U = D L^T): pivot k accepted
// when |d| > threshold (negative pivots are fine), kept on the diagonal and in dval[pivot], the column below
// divided by d, and the trailing block updated with l_i (d l_j) = l_i w_j, w the column before the division.
template <bool LDL>
__device__ __forceinline__ void lds_cholesky(double* A, int lda, int m, int ncols, int* bad_local, PivotRef pr,
                                             int pivot0, double* __restrict__ dval) {
    // A: lower triangle, column-major in LDS.  Factors ncols pivot columns and
    // applies their Schur update to the trailing (m - ncols) block.
    __shared__ double thr[TB];
    __shared__ double lcol[LDL ? TB : 1];
    const int ti = threadIdx.x % 64, tj = threadIdx.x / 64;
    if (threadIdx.x < ncols) thr[threadIdx.x] = pr.thresh(pivot0 + threadIdx.x);
    for (int k = 0; k < ncols; k++) {
        __syncthreads();
        double d = A[k + lda * k];
        if (!(LDL ? fabs(d) > thr[k] : d > thr[k])) {
            if (threadIdx.x == 0 && *bad_local < 0) *bad_local = k;
            d = 1.0;
        }
        if constexpr (LDL) {
            __syncthreads();
            if (threadIdx.x == 0) {
                A[k + lda * k] = d;
                dval[pivot0 + k] = d;
            }
            for (int i = k + 1 + threadIdx.x; i < m; i += NT) lcol[i] = A[i + lda * k] / d;
            __syncthreads();
            for (int j = k + 1 + tj; j < m; j += NT / 64)
                for (int i = j + ti; i < m; i += 64) A[i + lda * j] -= lcol[i] * A[j + lda * k];
            __syncthreads();
            for (int i = k + 1 + threadIdx.x; i < m; i += NT) A[i + lda * k] = lcol[i];
        } else {
            const double r = sqrt(d);
            __syncthreads();
            if (threadIdx.x == 0) A[k + lda * k] = r;
            for (int i = k + 1 + threadIdx.x; i < m; i += NT) A[i + lda * k] /= r;
            __syncthreads();
            for (int j = k + 1 + tj; j < m; j += NT / 64)
                for (int i = j + ti; i < m; i += 64) A[i + lda * j] -= A[i + lda * k] * A[j + lda * k];
        }
    }
    __syncthreads();
}

// The front in lda x lda doubles of dynamic LDS (lda = the level's largest front of at most 64 rows), so that
// a compute unit holds as many of the leaf levels' small fronts as its wave slots allow.
template <bool LDL>
__global__ __launch_bounds__(NT) void front_small(const int32_t* __restrict__ list, const int32_t* __restrict__ first,
                                                  const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                                  const int64_t* __restrict__ foff, double* __restrict__ fronts,
                                                  int32_t* __restrict__ status, PivotRef pr, double* __restrict__ dval,
                                                  int lda) {
    extern __shared__ double A[];
    __shared__ int bad;
    const int s = list[blockIdx.x];
    const int m = mrows[s], nn = ncol[s];
    double* F = fronts + foff[s];  // m <= 64: a plain column-major square
    if (threadIdx.x == 0) bad = -1;
    for (int e = threadIdx.x; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        if (i >= j) A[i + lda * j] = F[e];
    }
    lds_cholesky<LDL>(A, lda, m, nn, &bad, pr, first[s], dval);
    for (int e = threadIdx.x; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        if (i >= j) F[e] = A[i + lda * j];
    }
    if (threadIdx.x == 0) status[s] = bad >= 0 ? first[s] + bad : INT_MAX;
}

// ---------------------------------------------------------------- blocked path for large fronts
// items: potrf (s, k0) packed as two ints; trsm (s, k0, rb); syrk (s, k0, bi, bj)
constexpr int ST = 128;  // trailing-update tile edge

// Value of v held by lane l, read into scalar registers (l is a compile-time constant after unrolling).
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky of the kb x kb diagonal block at (k0, k0) of front s by the NW = 4 waves of a work-group,
// pipelined over the waves.  Lane i holds row i; wave w owns the 16 columns [16w, 16w + 16) in
// registers.  A wave first applies every earlier column of L (produced by the waves before it) to its
// own columns as soon as that column is in LDS, then factors its own 16 pivots: pivot k is read from
// lane k and scaled by a Newton-refined reciprocal square root, and the finished column is written to
// LDS.  Only the next column's update sits on the pivot-to-pivot path (two lane reads); the wave's
// other columns are updated from broadcast LDS reads of the column just written.  Finished columns are
// announced by a counter in LDS, raised after the column writes have completed (every second column and
// at the end of the wave's block), so a consumer reads the counter only when it has caught up.  The
// pivot loop is instantiated per wave so that the lanes it reads are immediates.  A partial block is
// padded with the identity.  Besides writing L_D into the front, the block is left in ldiag slot `slot`
// (64 x 64 column-major, identity padding) with the reciprocal pivots in rdiag (ones past kb) for the
// panel solve, and status[s] is lowered to the first rejected pivot (pivot <= tol |K_jj|, replaced by
// 1).  All NT threads must call it; `colbuf` is 64 x 64 doubles of LDS (16-byte aligned) and `flags`
// two ints of LDS.
constexpr int PW = 16;  // columns per wave in the pipelined diagonal-block Cholesky
constexpr int PUB = 2;  // columns per raise of the column counter

__device__ __forceinline__ double rsqrt_refined(double d) {
    double y = __builtin_amdgcn_rsq(d);  // hardware estimate, then two Newton steps for 1/sqrt(d)
    const double h = 0.5 * d;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

__device__ __forceinline__ double rcp_refined(double d) {
    double y = __builtin_amdgcn_rcp(d);  // hardware estimate, then two Newton steps for 1/d
    y = fma(y, fma(-d, y, 1.0), y);
    y = fma(y, fma(-d, y, 1.0), y);
    return y;
}

constexpr unsigned long long SENTINEL_BITS = 0x7ff4dead00000000ULL;

__device__ __forceinline__ bool is_sentinel(double v) {
    return (unsigned long long)__double_as_longlong(v) == SENTINEL_BITS;
}

// The 16 pivots of wave W (its columns in a[], every earlier column already applied).  thr: lane k holds
// pivot k's acceptance threshold.  Returns the first rejected pivot of the block (INT_MAX: none).
// LDL: the L D L^T form (see lds_cholesky): colbuf receives the column before the division by the pivot
// (w), cinv[k] the pivot's reciprocal, a[] the scaled column with the pivot itself on the diagonal, and the
// updates subtract l_ik w_jk; the lane of pivot k keeps the pivot in myd.
template <int W, bool LDL>
__device__ __forceinline__ int potrf_own(double (&a)[PW], double thr, double* colbuf, double* cinv, int* ready,
                                         double& myrinv, double& myd) {
    const int lane = threadIdx.x % 64;
    int bad = INT_MAX;
    double d = lane_value(a[0], PW * W);
#pragma unroll
    for (int c = 0; c < PW; c++) {
        const int k = PW * W + c;
        if (!(LDL ? fabs(d) > lane_value(thr, k) : d > lane_value(thr, k))) {
            bad = min(bad, k);
            d = 1.0;
        }
        double lik, wik;  // the stored column entry, and the one the updates multiply
        if constexpr (LDL) {
            const double rinv = rcp_refined(d);
            wik = lane == k ? d : a[c];
            lik = lane == k ? d : a[c] * rinv;
            if (lane == k) {
                myrinv = rinv;
                myd = d;
                cinv[k] = rinv;
            }
        } else {
            const double rinv = rsqrt_refined(d);
            lik = lane == k ? d * rinv : a[c] * rinv;
            wik = lik;
            if (lane == k) myrinv = rinv;
        }
        a[c] = lik;
        colbuf[TB * k + lane] = wik;
        if (c + 1 < PW) {
            a[c + 1] = fma(-lik, lane_value(wik, k + 1), a[c + 1]);
            d = lane_value(a[c + 1], k + 1);
        }
        // entries (16 W + c2, k) for c2 > c + 1, read back as broadcasts in aligned pairs (LDS keeps a wave's
        // accesses in order, so the reads see the write above)
#pragma unroll
        for (int q = (c + 2) / 2; q < PW / 2; q++) {
            const double2 u = *reinterpret_cast<const double2*>(&colbuf[TB * k + PW * W + 2 * q]);
            if (2 * q >= c + 2) a[2 * q] = fma(-lik, u.x, a[2 * q]);
            a[2 * q + 1] = fma(-lik, u.y, a[2 * q + 1]);
        }
        if (c % PUB == PUB - 1 || c == PW - 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the column writes have completed
            if (lane == 0) __hip_atomic_store(ready, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    return bad;
}

// Lane k's acceptance threshold for pivot k of the diagonal block at (k0, k0) of front s.  Callers load it
// early (three dependent loads: first pivot, diagonal position, value) so that the latency is off the
// pivot chain.
__device__ __forceinline__ double block_threshold(int s, int k0, const int32_t* __restrict__ first,
                                                  const int32_t* __restrict__ ncol, const PivotRef& pr) {
    const int lane = threadIdx.x % 64;
    return lane < min(TB, ncol[s] - k0) ? pr.thresh(first[s] + k0 + lane) : 0.0;
}

// LDL: the L D L^T form: the front gets L below the diagonal and the pivots on it, the compact copy L with a
// unit diagonal, rdiag the pivots' reciprocals and dval the pivots; `cinv` is 64 doubles of LDS.
template <bool LDL>
__device__ __forceinline__ void potrf_block(int s, int k0, int slot, const int32_t* __restrict__ first,
                                            const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                            const int64_t* __restrict__ foff, double* __restrict__ fronts,
                                            double* __restrict__ ldiag, double* __restrict__ rdiag,
                                            int32_t* __restrict__ status, double thr, double* colbuf,
                                            int* flags, double* cinv, double* __restrict__ dval) {
    const int lane = threadIdx.x % 64;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int m = mrows[s];
    const int kb = min(TB, ncol[s] - k0);
    double* F = fronts + foff[s] + fcol(m, k0) + k0;  // the block's panel, column stride ld
    const int64_t ld = fld(m, k0);
    const int p0 = first[s] + k0;
    int* badmin = flags;
    int* ready = flags + 1;
    if (threadIdx.x == 0) {
        *badmin = INT_MAX;
        *ready = 0;
    }
    double a[PW];
#pragma unroll
    for (int c = 0; c < PW; c++) {
        const int j = PW * w + c;
        a[c] = (j < kb && lane < kb) ? (j <= lane ? F[lane + ld * j] : 0.0) : (j == lane ? 1.0 : 0.0);
    }
    __syncthreads();
    // columns of the waves before this one, in order, each as soon as the counter covers it (bounded: the
    // producing waves belong to this work-group and always progress)
    int avail = 0;
    for (int k = 0; k < PW * w; k++) {
        if (avail <= k) {
            int spins = 0;
            do {
                avail = __hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } while (avail <= k && ++spins < (1 << 22));
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        const double l0 = LDL ? colbuf[TB * k + lane] * cinv[k] : colbuf[TB * k + lane];
#pragma unroll
        for (int q = 0; q < PW / 2; q++) {
            const double2 u = *reinterpret_cast<const double2*>(&colbuf[TB * k + PW * w + 2 * q]);
            a[2 * q] = fma(-l0, u.x, a[2 * q]);
            a[2 * q + 1] = fma(-l0, u.y, a[2 * q + 1]);
        }
    }
    double myrinv = 1.0, myd = 1.0;
    int bad;
    switch (w) {
        case 0: bad = potrf_own<0, LDL>(a, thr, colbuf, cinv, ready, myrinv, myd); break;
        case 1: bad = potrf_own<1, LDL>(a, thr, colbuf, cinv, ready, myrinv, myd); break;
        case 2: bad = potrf_own<2, LDL>(a, thr, colbuf, cinv, ready, myrinv, myd); break;
        default: bad = potrf_own<3, LDL>(a, thr, colbuf, cinv, ready, myrinv, myd); break;
    }
    if (lane == 0 && bad < kb) atomicMin(badmin, bad);
    // results: the front (valid lower part), the compact copy and the reciprocal pivots
    double* Lc = ldiag + (int64_t)slot * TB * TB + lane;
#pragma unroll
    for (int c = 0; c < PW; c++) {
        const int j = PW * w + c;
        if (j < kb && lane < kb && j <= lane) F[lane + ld * j] = a[c];
        if constexpr (LDL)
            Lc[TB * j] = j < lane ? a[c] : j == lane ? 1.0 : 0.0;
        else
            Lc[TB * j] = j <= lane ? a[c] : 0.0;
    }
    // lane i of the wave owning column i holds that pivot's reciprocal
    if (lane >= PW * w && lane < PW * w + PW) {
        rdiag[(int64_t)slot * TB + lane] = myrinv;
        if (LDL && lane < kb) dval[p0 + lane] = myd;
    }
    __syncthreads();
    if (threadIdx.x == 0 && *badmin < INT_MAX) atomicMin(&status[s], p0 + *badmin);
}

// Diagonal blocks of the first blocked step of each front (later steps factor theirs inside the
// trailing update of the step before, see blk_syrk).
template <bool LDL>
__global__ __launch_bounds__(NT) void blk_potrf(const int32_t* __restrict__ it, const int32_t* __restrict__ first,
                                                const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                                const int64_t* __restrict__ foff, double* __restrict__ fronts,
                                                double* __restrict__ ldiag, double* __restrict__ rdiag,
                                                int32_t* __restrict__ status, PivotRef pr, double* __restrict__ dval) {
    __shared__ __attribute__((aligned(16))) double colbuf[TB * TB];
    __shared__ double cinv[LDL ? TB : 1];
    __shared__ int flags[2];
    const int s = it[2 * blockIdx.x], k0 = it[2 * blockIdx.x + 1];
    potrf_block<LDL>(s, k0, blockIdx.x, first, ncol, mrows, foff, fronts, ldiag, rdiag, status,
                     block_threshold(s, k0, first, ncol, pr), colbuf, flags, cinv, dval);
}

constexpr int TR = 64;  // panel rows per work-group of the panel solve

// C(bi, bj) -= P_bi P_bj^T on the trailing matrix, 128 x 128 tiles, FP64 MFMA 16x16x4.
// Four waves in a 2 x 2 arrangement, each computing a 64 x 64 quadrant as 4 x 4 MFMA blocks;
// the panel rows are staged through LDS in chunks of 16 columns.
typedef double double4_t __attribute__((ext_vector_type(4)));

// Panel solve X <- X L_D^{-T} on 64 panel rows per work-group (item: front, k0, row block, slot) with FP64
// MFMA.  L_D (identity padded) is split into 4 x 4 blocks of 16.  Wave b first inverts the diagonal block L_bb into
// LDS (lane q computes column q by forward substitution; L_bb and the reciprocal pivots are uniform, so
// they come through the scalar unit).  Then wave w takes rows [16 w, 16 w + 16) of the work-group's rows
// through the column blocks in order, Y_b = (X_b - sum_{a<b} Y_a L_ba^T) inv(L_bb)^T, computed transposed
// (Y_b^T = inv(L_bb) (X_b - ...)^T) so that every product is a 16x16x4 MFMA.  In this layout a lane holds
// row lane % 16 and columns lane / 16 + 4 r of a 16 x 16 block: that is both the accumulator layout and
// the B-operand layout, so the solved blocks feed the later updates straight from registers, and the
// stores put 16 consecutive rows of a column on each 16-lane group.
// LDL: L_D has a unit diagonal and rdiag holds the pivots' reciprocals: the rows are solved with the unit
// triangle and then scaled column by column, X <- X L_D^{-T} D^{-1}.
template <bool LDL>
__global__ __launch_bounds__(NT) void blk_trsm_mma(const int32_t* __restrict__ it, const int32_t* __restrict__ ncol,
                                                   const int32_t* __restrict__ mrows,
                                                   const int64_t* __restrict__ foff, const double* __restrict__ ldiag,
                                                   const double* __restrict__ rdiag, double* __restrict__ fronts) {
    __shared__ double inv[4][16][17];  // inv[b][p][q] = inv(L_bb)[p][q]
    __shared__ double dg[4][16][17];   // dg[b][t][p] = L_bb(p, t), staged with vector loads
    const int s = it[4 * blockIdx.x], k0 = it[4 * blockIdx.x + 1], rb = it[4 * blockIdx.x + 2];
    const int slot = it[4 * blockIdx.x + 3];
    const int m = mrows[s];
    const int kb = min(TB, ncol[s] - k0);
    const double* Lc = ldiag + (int64_t)slot * TB * TB;  // Lc[t + 64 j] = L_D(t, j)
    const double* rc = rdiag + (int64_t)slot * TB;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    const int li = lane % 16, lk = lane / 16;
    const int row = k0 + kb + rb * TR + 16 * wave + li;
    const bool rowok = row < m;
    const int64_t ld = fld(m, k0);
    double* X = fronts + foff[s] + fcol(m, k0) + (rowok ? row : 0);  // X[ld j] = entry (row, k0 + j)
    // Every global load of the kernel is issued here, before the diagonal blocks are inverted: the wave's
    // diagonal block (rows of a column are contiguous), the reciprocal pivots, the rows' 64 entries and the
    // off-diagonal 16 x 16 blocks of L_D that the substitution's MFMAs take (lof[b (b - 1) / 2 + a] for a < b),
    // so that their latency overlaps the inversion instead of sitting between the substitution's stages.
    double dgv[4];
#pragma unroll
    for (int r = 0; r < 4; r++) dgv[r] = Lc[(16 * wave + li) + TB * (16 * wave + 4 * r + lk)];
    const double rp = lane < 16 ? (LDL ? 1.0 : rc[16 * wave + lane]) : 0.0;
    double4_t xin[4];
#pragma unroll
    for (int b = 0; b < 4; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int j = 16 * b + lk + 4 * r;
            xin[b][r] = (rowok && j < kb) ? X[ld * j] : 0.0;
        }
    double lof[6][4];
#pragma unroll
    for (int b = 1; b < 4; b++)
#pragma unroll
        for (int a = 0; a < b; a++)
#pragma unroll
            for (int kk = 0; kk < 4; kk++) lof[b * (b - 1) / 2 + a][kk] = -Lc[(16 * b + li) + TB * (16 * a + 4 * kk + lk)];
    double dsc[4][4];  // L D L^T: the pivots' reciprocals for the final column scaling
    if constexpr (LDL) {
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) dsc[b][r] = rc[min(16 * b + lk + 4 * r, kb - 1)];
    }
    {
        // the wave's diagonal block into LDS, then the inversion reads it as broadcasts
        const int b = wave, q = li;  // the four 16-lane groups compute the same columns; group 0 stores
#pragma unroll
        for (int r = 0; r < 4; r++) dg[b][4 * r + lk][li] = dgv[r];
        double y[16];
#pragma unroll
        for (int p = 0; p < 16; p++) {
            double acc = p == q ? 1.0 : 0.0;
#pragma unroll
            for (int t = 0; t < p; t++) acc -= dg[b][t][p] * y[t];
            y[p] = acc * lane_value(rp, p);
        }
        if (lk == 0)
#pragma unroll
            for (int p = 0; p < 16; p++) inv[b][p][q] = y[p];
    }
    double4_t y[4];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 4; b++) {
        double4_t acc = xin[b];
#pragma unroll
        for (int a = 0; a < b; a++)
#pragma unroll
            for (int kk = 0; kk < 4; kk++)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(lof[b * (b - 1) / 2 + a][kk], y[a][kk], acc, 0, 0, 0);
        double4_t out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; kk++)
            out = __builtin_amdgcn_mfma_f64_16x16x4f64(inv[b][li][4 * kk + lk], acc[kk], out, 0, 0, 0);
        y[b] = out;
    }
    if (rowok)
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int j = 16 * b + lk + 4 * r;
                if (j < kb) X[ld * j] = LDL ? y[b][r] * dsc[b][r] : y[b][r];
            }
}
constexpr int KC = 16;
constexpr int KH = 16;  // panel columns staged in LDS at a time

// Item: (front, k0, first row ri0, first column rj0) of a tile of up to 128 rows and cw columns.  The
// accumulators start from the tile of C and the row panel is negated on its way into LDS, so the MFMAs
// accumulate C - Pi Pj^T and the tile is read once, at the start, where its latency overlaps the first
// panel loads.
// One launch per blocked step covers the whole trailing update: the first nnext items are 128 x 64 tiles of
// the next panel's 64 columns, the rest 128 x 128 tiles of the columns after it.  The work-group holding
// a front's next-panel diagonal tile goes on to factor that panel's diagonal block, which it has just
// brought up to date, into ldiag slot pslot[item] (-1: no such block), while the other work-groups are
// still updating the rest: the diagonal-block Cholesky of step k+1 hides under the update of step k.
// MFMA part of one tile: each wave computes a (16 RB) x (16 CB) block of the tile, the waves laid out as
// (128 / 16 RB) x (cw / 16 CB); Pi, Pj hold the negated row panel and the column panel (64 columns,
// zero past kb).  RB = CB = 4 for 128 x 128 tiles (2 x 2 waves), RB = 2, CB = 4 for the 128 x 64 tiles
// of the next panel (4 x 1 waves, so the next panel's diagonal block is spread over two waves).
// LDL: the row panel is scaled by the pivots on its way into LDS (each column's pivot is on the front's
// diagonal), so the update is C - (Pi D) Pj^T.
template <int RB, int CB, bool LDL>
__device__ __forceinline__ void tile_mma(double* __restrict__ F, int m, int ri0, int rj0, int nri, int nrj, int k0,
                                         int kb, double* lds) {
    const double(*Pi)[ST + 1] = reinterpret_cast<const double(*)[ST + 1]>(lds);
    const double(*Pj)[ST + 1] = reinterpret_cast<const double(*)[ST + 1]>(lds + KH * (ST + 1));
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    constexpr int WR = ST / (16 * RB);  // waves along the rows
    const int qr = (wave % WR) * 16 * RB, qc = (wave / WR) * 16 * CB;
    const int li = lane % 16, lk = lane / 16;
    // blocks outside the tile's columns or strictly above the diagonal do no MFMA work
    const bool active = qc < nrj && ri0 + qr + 16 * RB - 1 >= rj0 + qc;
    // D layout of the 16x16x4 f64 MFMA: item r of a lane is row (lane / 16) + 4 r, column lane % 16 of the
    // product block; operands are swapped below so the block is C^T: C row = lane % 16, C column =
    // (lane / 16) + 4 r (16 consecutive rows of a column per 16-lane group)
    // The wave's 16 CB <= 64 columns rj0 + qc + jl lie in at most two panels: the first `cut` of them in the
    // panel of column rj0 + qc, the rest at the start of the next one.
    const int cw = rj0 + qc, cut = ((cw | 63) + 1) - cw;
    const int64_t f0 = fcol(m, cw), f1 = fcol(m, cw + cut);
    const int ld0 = (int)fld(m, cw), ld1 = ld0 - 64;
    // Only a front's last blocked step (pivot count not a multiple of 64) has its columns off the panel grid,
    // so the tile's loads and stores take a wave-uniform branch to the form with the per-column choice.
    double4_t acc[RB][CB];
    auto load = [&](auto split) {
#pragma unroll
        for (int a = 0; a < RB; a++)
#pragma unroll
            for (int b = 0; b < CB; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = qr + 16 * a + li;
                    const int jl = 16 * b + lk + 4 * r, j = qc + jl;
                    const int gi = ri0 + i, gj = rj0 + j;
                    const int64_t o = (!decltype(split)::value || jl < cut) ? f0 + jl * ld0 : f1 + (jl - cut) * ld1;
                    acc[a][b][r] = (active && i < nri && j < nrj && gi >= gj) ? F[o + gi] : 0.0;
                }
    };
    if (cut == TB)
        load(std::false_type{});
    else
        load(std::true_type{});
    // the panel slices go through LDS in halves of KH columns (columns past kb are zero; a half that starts
    // at or past kb is skipped).  Each half is fetched into registers while the previous half's MFMAs run,
    // then written to LDS, so the panel loads' latency hides under the arithmetic.
    constexpr int PER = ST * KH / NT;  // panel entries per thread per half (each of Pi and Pj)
    double fa[PER], fb[PER];
    auto fetch = [&](int h0) {
        // the KH columns of a half lie in one panel (k0 and h0 are multiples of KH)
        const int64_t cb = fcol(m, k0 + h0), ld = fld(m, k0 + h0);
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = threadIdx.x + q * NT;
            const int r = e % ST, t = e / ST;
            const bool in = h0 + t < kb;
            const int64_t col = cb + ld * t;
            fa[q] = (in && r < nri) ? F[(int64_t)(ri0 + r) + col] : 0.0;
            fb[q] = (in && r < nrj) ? F[(int64_t)(rj0 + r) + col] : 0.0;
            if constexpr (LDL) fa[q] *= in ? F[col + (k0 + h0 + t)] : 0.0;
        }
    };
    fetch(0);
    for (int h0 = 0; h0 < kb; h0 += KH) {
        __syncthreads();  // earlier readers of LDS (this tile's previous half, or the previous item) are done
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = threadIdx.x + q * NT;
            const int r = e % ST, t = e / ST;
            lds[t * (ST + 1) + r] = -fa[q];
            lds[KH * (ST + 1) + t * (ST + 1) + r] = fb[q];
        }
        __syncthreads();
        if (h0 + KH < kb) fetch(h0 + KH);
        if (active) {
#pragma unroll 2
            for (int t0 = 0; t0 < KH; t0 += KC) {
#pragma unroll
                for (int t = t0; t < t0 + KC; t += 4) {
                    double av[RB], bv[CB];
#pragma unroll
                    for (int a = 0; a < RB; a++) av[a] = Pi[t + lk][qr + 16 * a + li];
#pragma unroll
                    for (int b = 0; b < CB; b++) bv[b] = Pj[t + lk][qc + 16 * b + li];
#pragma unroll
                    for (int a = 0; a < RB; a++)
#pragma unroll
                        for (int b = 0; b < CB; b++)
                            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[b], av[a], acc[a][b], 0, 0, 0);
                }
            }
        }
    }
    auto store = [&](auto split) {
#pragma unroll
        for (int a = 0; a < RB; a++)
#pragma unroll
            for (int b = 0; b < CB; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = qr + 16 * a + li;
                    const int jl = 16 * b + lk + 4 * r, j = qc + jl;
                    const int gi = ri0 + i, gj = rj0 + j;
                    const int64_t o = (!decltype(split)::value || jl < cut) ? f0 + jl * ld0 : f1 + (jl - cut) * ld1;
                    if (i < nri && j < nrj && gi >= gj) F[o + gi] = acc[a][b][r];
                }
    };
    if (active) {
        if (cut == TB)
            store(std::false_type{});
        else
            store(std::true_type{});
    }
}

// One launch per blocked step covers the whole trailing update: the first nnext items are 128 x 64 tiles of
// the next panel's 64 columns, the rest 128 x 128 tiles of the columns after it.  The work-group holding
// a front's next-panel diagonal tile goes on to factor that panel's diagonal block, which it has just
// brought up to date, into ldiag slot pslot[item] (-1: no such block), while the other work-groups are
// still updating the rest: the diagonal-block Cholesky of step k+1 hides under the update of step k.
template <bool LDL>
__global__ __launch_bounds__(NT, 2) void blk_syrk(const int32_t* __restrict__ it, int nitems, int nnext, int kw,
                                               const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                               const int64_t* __restrict__ foff, double* __restrict__ fronts,
                                               const int32_t* __restrict__ pslot,
                                               const int32_t* __restrict__ first, double* __restrict__ ldiag,
                                               double* __restrict__ rdiag, int32_t* __restrict__ status,
                                               PivotRef pr, double* __restrict__ dval) {
    // LDS: both panel slices of the tile, KH columns at a time (66 KB, so two work-groups share a compute
    // unit and one's loads overlap the other's MFMAs), reused by the fused diagonal-block Cholesky as its
    // 64 x 64 column buffer
    __shared__ __attribute__((aligned(16))) double lds[2 * KH * (ST + 1)];
    static_assert(2 * KH * (ST + 1) >= TB * TB, "the column buffer of the diagonal-block Cholesky fits");
    __shared__ int flags[2];
    __shared__ double cinv[LDL ? TB : 1];
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int s = it[4 * item], k0 = it[4 * item + 1];
        const int ri0 = it[4 * item + 2], rj0 = it[4 * item + 3];
        const int m = mrows[s];
        const int kb = min(kw, ncol[s] - k0);
        double* F = fronts + foff[s];
        const int nri = min(ST, m - ri0);
        const int ps = pslot ? pslot[item] : -1;
        const double thr = ps >= 0 ? block_threshold(s, rj0, first, ncol, pr) : 0.0;  // loaded before the tile
        if (item < nnext)
            tile_mma<2, 4, LDL>(F, m, ri0, rj0, nri, min(TB, m - rj0), k0, kb, lds);
        else
            tile_mma<4, 4, LDL>(F, m, ri0, rj0, nri, min(ST, m - rj0), k0, kb, lds);
        if (ps >= 0) {
            __syncthreads();  // the tile's stores are visible to the whole work-group; LDS is free
            potrf_block<LDL>(s, rj0, ps, first, ncol, mrows, foff, fronts, ldiag, rdiag, status, thr, lds, flags,
                             cinv, dval);
        }
    }
}

// ---------------------------------------------------------------- dense fronts: one dependency-driven launch
// Fronts with at least DENSE_MIN pivots (the dense root of an expander-like grid holds almost all the
// factorization's flops) are factored tile by tile in one persistent launch instead of one blocked step at a
// time.  The front's rows are cut into blocks of DT: the pivot columns [0, nn) first (the last pivot block
// may be short), then the update rows [nn, m).  Every lower tile (bi, bj) is a task; tasks are numbered
// column by column (diagonal tile first) and work-groups take them in that order from a counter.  A task
// gathers its tile once, subtracts L(bi, k) L(bj, k)^T for every pivot block k < bj as soon as both tiles are
// final (left-looking, so the tile is read and written once), and then
//   * diagonal tile of a pivot block: factors it (the pipelined diagonal-block Cholesky), leaving L_jj and
//     its reciprocal pivots in the front's slot of tdiag / trdiag;
//   * tile below a diagonal tile: waits for that diagonal tile and solves X L_jj^{-T} (16 x 16 diagonal
//     inverses, block substitution on MFMA, as in the panel solve);
//   * tile of the update block: is left as the update matrix.
// A finished pivot-column tile is published by a release fence and its flag set to the factorization's
// epoch; readers spin (bounded) on the flag and acquire.  Every dependency of a task has a smaller task
// number, and a task is only ever taken by a running work-group, so the smallest unfinished task always
// progresses: no deadlock whatever the residency.  A wait that exceeds its bound raises the fault word and
// proceeds (the factor is then reported invalid).
constexpr int DT = 64;           // tile edge
// Fronts with at least chol_options.tile_min pivots take the tile path; 0 (the default) switches it off: its
// first GPU run did not finish (see the design notes), and it stays off until that is explained.
constexpr int LDT = DT + 1;      // padded LDS row of a staged tile
constexpr int FLAG_SPINS = 1 << 24;  // ~1 s of polling

struct DenseDesc {
    const int32_t* hs;       // supernode of each dense front
    const int32_t* hnp;      // pivot blocks
    const int32_t* hnb;      // all blocks
    const int64_t* htask0;   // first task number of the front
    const int32_t* hslot0;   // first diagonal slot of the front in tdiag / trdiag
    const int32_t* task_h;   // per task: dense-front index
    const int32_t* task_rc;  // per task: (bi << 16) | bj
    int32_t* flags;          // per task: epoch at which the tile became final
    int32_t* counter;        // task counter of the launch
    int32_t* fault;          // raised by a wait past its bound
    double* tdiag;           // 64 x 64 factored diagonal blocks (column-major, identity padding)
    double* trdiag;          // their reciprocal pivots
};

__device__ __forceinline__ int blk_start(int b, int np, int nn) { return b < np ? DT * b : nn + DT * (b - np); }
__device__ __forceinline__ int blk_size(int b, int np, int nn, int m) {
    return b < np ? min(DT, nn - DT * b) : min(DT, m - (nn + DT * (b - np)));
}
// task number of tile (bi, bj), bi >= bj, of a front with nb blocks (column-major lower enumeration)
__device__ __forceinline__ int64_t tile_task(int64_t t0, int nb, int bi, int bj) {
    return t0 + (int64_t)bj * nb - (int64_t)bj * (bj - 1) / 2 + (bi - bj);
}

// Thread 0 waits until the flag holds `epoch` (bounded), then the work-group acquires at agent scope.
__device__ __forceinline__ void wait_final(const int32_t* flag, int epoch, int32_t* fault, int* ok_sh) {
    if (threadIdx.x == 0) {
        int spins = 0, ok = 1;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            ++spins;
            // past the bound, or once any wait of the launch has given up, stop waiting
            if (spins > FLAG_SPINS ||
                ((spins & 255) == 0 && __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                ok = 0;
                __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *ok_sh = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Every thread's stores of the tile reach agent scope, then thread 0 sets the flag.
__device__ __forceinline__ void publish_final(int32_t* flag, int epoch) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(NT, 2) void dense_front(int64_t t0, int64_t t1, DenseDesc D, int epoch,
                                                   const int32_t* __restrict__ first,
                                                   const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                                   const int64_t* __restrict__ foff, double* __restrict__ fronts,
                                                   int32_t* __restrict__ status, PivotRef pr) {
    // two staged tiles (k-major: lds[t][r] = tile entry (r, t)); the first also serves as the diagonal-block
    // Cholesky's 64 x 64 column buffer and as the right-hand side of the triangular solve
    __shared__ __attribute__((aligned(16))) double Pa[DT * LDT];
    __shared__ __attribute__((aligned(16))) double Pb[DT * LDT];
    __shared__ double inv[4][16][17];
    __shared__ int task_sh, ok_sh, flags[2];
    static_assert(DT * LDT >= TB * TB, "the column buffer of the diagonal-block Cholesky fits");
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    const int li = lane % 16, lk = lane / 16;
    const int wr = wave % 2, wc = wave / 2;  // quadrant of the tile owned by this wave in the update
    const int qr = 32 * wr, qc = 32 * wc;
    while (true) {
        if (threadIdx.x == 0) task_sh = (int)(t0 + atomicAdd(D.counter, 1));
        __syncthreads();
        const int64_t t = task_sh;
        __syncthreads();  // every thread has read task_sh before thread 0 may overwrite it
        if (t >= t1) break;
        const int h = D.task_h[t];
        const int bi = D.task_rc[t] >> 16, bj = D.task_rc[t] & 0xffff;
        const int s = D.hs[h], np = D.hnp[h], nb = D.hnb[h];
        const int m = mrows[s], nn = ncol[s];
        const int64_t ht0 = D.htask0[h];
        double* F = fronts + foff[s];
        const int ri0 = blk_start(bi, np, nn), nri = blk_size(bi, np, nn, m);
        const int rj0 = blk_start(bj, np, nn), nrj = blk_size(bj, np, nn, m);
        const bool diag = bi == bj;
        const bool active = !(diag && wc > wr);  // the strictly upper quadrant of a diagonal tile is idle
        double4_t acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = qr + 16 * a + li, j = qc + 16 * b + lk + 4 * r;
                    const bool in = active && i < nri && j < nrj && (!diag || i >= j);
                    acc[a][b][r] = in ? F[fcol(m, rj0 + j) + (ri0 + i)] : 0.0;
                }
        // left-looking: every pivot block before this tile's column
        const int kmax = min(bj, np);
        for (int k = 0; k < kmax; k++) {
            const int kc0 = DT * k, kk = min(DT, nn - kc0);
            wait_final(D.flags + tile_task(ht0, nb, bi, k), epoch, D.fault, &ok_sh);
            if (!diag) wait_final(D.flags + tile_task(ht0, nb, bj, k), epoch, D.fault, &ok_sh);
            for (int e = threadIdx.x; e < DT * DT; e += NT) {
                const int r = e % DT, c = e / DT;
                double av = 0.0, bv = 0.0;
                if (c < kk) {
                    if (r < nri) av = F[fcol(m, kc0 + c) + (ri0 + r)];
                    if (!diag && r < nrj) bv = F[fcol(m, kc0 + c) + (rj0 + r)];
                }
                Pa[c * LDT + r] = -av;
                Pb[c * LDT + r] = bv;
            }
            __syncthreads();
            if (active) {
                const double* Pj = diag ? Pa : Pb;
                const double sg = diag ? -1.0 : 1.0;  // Pa holds the negated rows
#pragma unroll 4
                for (int t4 = 0; t4 < DT; t4 += 4) {
                    double av[2], bv[2];
#pragma unroll
                    for (int a = 0; a < 2; a++) av[a] = Pa[(t4 + lk) * LDT + qr + 16 * a + li];
#pragma unroll
                    for (int b = 0; b < 2; b++) bv[b] = sg * Pj[(t4 + lk) * LDT + qc + 16 * b + li];
#pragma unroll
                    for (int a = 0; a < 2; a++)
#pragma unroll
                        for (int b = 0; b < 2; b++)
                            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[b], av[a], acc[a][b], 0, 0, 0);
                }
            }
            __syncthreads();  // the staged tiles are consumed before the next stage overwrites them
        }
        if (bj >= np) {  // update block: the tile is part of the update matrix
            if (active)
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < 2; b++)
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const int i = qr + 16 * a + li, j = qc + 16 * b + lk + 4 * r;
                            if (i < nri && j < nrj && (!diag || i >= j))
                                F[fcol(m, rj0 + j) + (ri0 + i)] = acc[a][b][r];
                        }
            continue;
        }
        const int slot = D.hslot0[h] + bj;
        int32_t* myflag = D.flags + t;
        if (diag) {
            if (active)
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < 2; b++)
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const int i = qr + 16 * a + li, j = qc + 16 * b + lk + 4 * r;
                            if (i < nri && j < nrj && i >= j) F[fcol(m, rj0 + j) + (ri0 + i)] = acc[a][b][r];
                        }
            __syncthreads();  // the tile's stores are visible to the work-group; LDS is free
            potrf_block<false>(s, rj0, slot, first, ncol, mrows, foff, fronts, D.tdiag, D.trdiag, status,
                               block_threshold(s, rj0, first, ncol, pr), Pa, flags, nullptr, nullptr);
            publish_final(myflag, epoch);
            continue;
        }
        // off-diagonal tile of a pivot column: X L_jj^{-T} once L_jj is final
        if (active)
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int i = qr + 16 * a + li, j = qc + 16 * b + lk + 4 * r;
                        Pb[j * LDT + i] = acc[a][b][r];  // X, k-major like the staged tiles
                    }
        wait_final(D.flags + tile_task(ht0, nb, bj, bj), epoch, D.fault, &ok_sh);
        const double* Lc = D.tdiag + (int64_t)slot * TB * TB;  // Lc[t + 64 j] = L_jj(t, j)
        const double* rc = D.trdiag + (int64_t)slot * TB;
        const int kb = nrj;
        {
            const int b = wave, q = li;  // wave b inverts the diagonal 16 x 16 block b of L_jj
            double y[16];
#pragma unroll
            for (int p = 0; p < 16; p++) {
                double a = p == q ? 1.0 : 0.0;
#pragma unroll
                for (int t2 = 0; t2 < p; t2++) a -= Lc[(16 * b + p) + TB * (16 * b + t2)] * y[t2];
                y[p] = a * rc[16 * b + p];
            }
            if (lk == 0)
#pragma unroll
                for (int p = 0; p < 16; p++) inv[b][p][q] = y[p];
        }
        __syncthreads();
        // wave w solves rows [16 w, 16 w + 16) through the four column blocks
        const int row = 16 * wave + li;
        double4_t yb[4];
#pragma unroll
        for (int b = 0; b < 4; b++) {
            double4_t x;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int j = 16 * b + lk + 4 * r;
                x[r] = j < kb ? Pb[j * LDT + row] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < b; a++)
#pragma unroll
                for (int q4 = 0; q4 < 4; q4++)
                    x = __builtin_amdgcn_mfma_f64_16x16x4f64(-Lc[(16 * b + li) + TB * (16 * a + 4 * q4 + lk)],
                                                             yb[a][q4], x, 0, 0, 0);
            double4_t out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q4 = 0; q4 < 4; q4++)
                out = __builtin_amdgcn_mfma_f64_16x16x4f64(inv[b][li][4 * q4 + lk], x[q4], out, 0, 0, 0);
            yb[b] = out;
        }
        if (row < nri)
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int j = 16 * b + lk + 4 * r;
                    if (j < kb) F[fcol(m, rj0 + j) + (ri0 + row)] = yb[b][r];
                }
        publish_final(myflag, epoch);
    }
}

// ---------------------------------------------------------------- solves
__global__ void permute_in(int n, const int32_t* __restrict__ perm, const double* __restrict__ b,
                           double* __restrict__ y) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = b[perm[k]];
}

__global__ void permute_out(int n, const int32_t* __restrict__ perm, const double* __restrict__ y,
                            double* __restrict__ x) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) x[perm[k]] = y[k];
}

constexpr int WIDE = 256;  // fronts with at least this many pivots use the sync-free solves

// acc + the update entries gsrc[k0..k1) of one front row, added in list order, four loads in flight
__device__ __forceinline__ double row_gather(double acc, int64_t k0, int64_t k1, const int64_t* __restrict__ gsrc,
                                             const double* __restrict__ upd) {
    int64_t k = k0;
    for (; k + 3 < k1; k += 4) {
        const int64_t s0 = gsrc[k], s1 = gsrc[k + 1], s2 = gsrc[k + 2], s3 = gsrc[k + 3];
        const double u0 = upd[s0], u1 = upd[s1], u2 = upd[s2], u3 = upd[s3];
        acc += u0;
        acc += u1;
        acc += u2;
        acc += u3;
    }
    for (; k < k1; k++) acc += upd[gsrc[k]];
    return acc;
}
constexpr int SCB = 16;    // pivot columns per block of the narrow-front sweeps
constexpr int TALL = 512;  // narrow fronts with at least this many rows below their pivots are "tall"

// Forward sweep for one front: w = b(own rows) + children's partial results; solve with the diagonal
// block; keep w on the off-diagonal rows as this front's partial result.  w lives in LDS (dynamic, wcap
// doubles) when the front fits, else in the front's slice of `work`.  The gathers are unrolled by four so
// that four independent index and value loads are in flight per thread.
__global__ __launch_bounds__(NT) void solve_fwd(const int32_t* __restrict__ list, const int32_t* __restrict__ first,
                                                const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                                const int64_t* __restrict__ foff, const int64_t* __restrict__ roff,
                                                const int64_t* __restrict__ uoff, const int64_t* __restrict__ gptr,
                                                const int64_t* __restrict__ gsrc,
                                                const double* __restrict__ fronts, double* __restrict__ work,
                                                double* __restrict__ upd, double* __restrict__ y, int wcap,
                                                int unit) {
    extern __shared__ double wl[];
    const int s = list[blockIdx.x];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    double* w = m <= wcap ? wl : work + roff[s];
    // own right-hand side plus the children's update entries, each row summing its own list (children in
    // ascending order), so no barrier per child
    const int64_t* gp = gptr + roff[s];
    // a tall front's rows below its pivots are gathered and updated by solve_fwd_rows after this launch
    const int mr = m - nn >= TALL ? nn : m;
    for (int t = threadIdx.x; t < mr; t += NT) w[t] = row_gather(t < nn ? y[f + t] : 0.0, gp[t], gp[t + 1], gsrc, upd);
    __syncthreads();
    // blocks of SCB pivot columns: wave 0 solves the diagonal block in registers (solved values to zz), then
    // every thread applies the block's columns to its rows below it, all SCB loads of a row in flight at once.
    // Each w[i] takes the columns in increasing order, one fused multiply-add each, as a column-by-column
    // sweep would.
    __shared__ double zz[WIDE];
    const double* L = fronts + foff[s];
    const int lane = threadIdx.x % 64;
    for (int j0 = 0; j0 < nn; j0 += SCB) {
        const int cb = min(SCB, nn - j0);
        // the block's columns lie in one panel: column j0 + t at Lb + ld t
        const double* Lb = L + fcol(m, j0);
        const int64_t ld = fld(m, j0);
        if (threadIdx.x < 64) {
            const bool act = lane < cb;
            double a[SCB];  // lane p: a[t] = L(j0 + p, j0 + t), t < p
#pragma unroll
            for (int t = 0; t < SCB; t++) a[t] = (act && t < lane) ? Lb[(j0 + lane) + ld * t] : 0.0;
            double wp = act ? w[j0 + lane] : 0.0;
            const double rp = act && !unit ? 1.0 / Lb[(j0 + lane) + ld * lane] : 1.0;
#pragma unroll
            for (int t = 0; t < SCB; t++) {
                const double z = lane_value(wp, t) * lane_value(rp, t);
                if (lane > t) wp = fma(-a[t], z, wp);
                if (lane == t && act) zz[j0 + t] = z;
            }
        }
        __syncthreads();
        for (int i = j0 + cb + threadIdx.x; i < mr; i += NT) {
            double lv[SCB];
#pragma unroll
            for (int t = 0; t < SCB; t++) lv[t] = t < cb ? Lb[i + ld * t] : 0.0;
            double acc = w[i];
#pragma unroll
            for (int t = 0; t < SCB; t++)
                if (t < cb) acc = fma(-lv[t], zz[j0 + t], acc);
            w[i] = acc;
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < mr; t += NT) {
        if (t < nn)
            y[f + t] = zz[t];
        else
            upd[uoff[s] + (t - nn)] = w[t];
    }
}

// Rows below the pivots of a tall front, 256 rows per work-group (item: front, row block): the row's gathered
// update entries, then the pivot columns in increasing order, one fused multiply-add each (the order of the
// single-work-group sweep), 16 loads in flight; the result is the front's partial result for its parent.
__global__ __launch_bounds__(NT) void solve_fwd_rows(const int32_t* __restrict__ items,
                                                     const int32_t* __restrict__ first,
                                                     const int32_t* __restrict__ ncol,
                                                     const int32_t* __restrict__ mrows,
                                                     const int64_t* __restrict__ foff, const int64_t* __restrict__ roff,
                                                     const int64_t* __restrict__ uoff, const int64_t* __restrict__ gptr,
                                                     const int64_t* __restrict__ gsrc,
                                                     const double* __restrict__ fronts, double* __restrict__ upd,
                                                     const double* __restrict__ y) {
    __shared__ double zs[WIDE];
    const int s = items[2 * blockIdx.x], rb = items[2 * blockIdx.x + 1];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    for (int j = threadIdx.x; j < nn; j += NT) zs[j] = y[f + j];
    __syncthreads();
    const int i = nn + rb * NT + threadIdx.x;
    if (i >= m) return;
    const int64_t* gp = gptr + roff[s];
    double acc = row_gather(0.0, gp[i], gp[i + 1], gsrc, upd);
    const double* L = fronts + foff[s] + i;
    for (int j0 = 0; j0 < nn; j0 += SCB) {
        const double* Lb = L + fcol(m, j0);  // the block's columns lie in one panel
        const int64_t ld = fld(m, j0);
        double lv[SCB];
#pragma unroll
        for (int t = 0; t < SCB; t++) lv[t] = j0 + t < nn ? Lb[ld * t] : 0.0;
#pragma unroll
        for (int t = 0; t < SCB; t++)
            if (j0 + t < nn) acc = fma(-lv[t], zs[j0 + t], acc);
    }
    upd[uoff[s] + (i - nn)] = acc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sweeps of levels whose fronts all have m <= 64 rows (plain squares): one wave per front and four fronts per
// work-group, since the leaf levels hold thousands of tiny fronts and a work-group per front costs more to
// dispatch than its work.  Lane i is on row i; every row gets the same operations in the same order as in
// solve_fwd / solve_bwd, so the results are theirs bit for bit.
// Forward: w = b(own rows) + the children's update entries; pivot j: z_j = w_j (1 / L_jj) (unit: L_jj = 1),
// then w_i -= L_ij z_j below it, the loads of 16 pivots' columns in flight together.
__global__ __launch_bounds__(NT) void solve_fwd_tiny(int nf, const int32_t* __restrict__ list,
                                                     const int32_t* __restrict__ first,
                                                     const int32_t* __restrict__ ncol,
                                                     const int32_t* __restrict__ mrows,
                                                     const int64_t* __restrict__ foff, const int64_t* __restrict__ roff,
                                                     const int64_t* __restrict__ uoff,
                                                     const int64_t* __restrict__ gptr, const int64_t* __restrict__ gsrc,
                                                     const double* __restrict__ fronts, double* __restrict__ upd,
                                                     double* __restrict__ y, int unit) {
    const int lane = threadIdx.x % 64;
    const int q = blockIdx.x * (NT / 64) + threadIdx.x / 64;
    if (q >= nf) return;
    const int s = list[q];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    const bool row = lane < m;
    const int64_t* gp = gptr + roff[s];
    const double* L = fronts + foff[s];
    double w = row ? row_gather(lane < nn ? y[f + lane] : 0.0, gp[lane], gp[lane + 1], gsrc, upd) : 0.0;
    const double rp = lane < nn && !unit ? 1.0 / L[lane + m * lane] : 1.0;
    double zl = 0.0;
    for (int j0 = 0; j0 < nn; j0 += SCB) {
        double lv[SCB];  // L(lane, j0 + t)
#pragma unroll
        for (int t = 0; t < SCB; t++) lv[t] = row && lane > j0 + t && j0 + t < nn ? L[lane + m * (j0 + t)] : 0.0;
#pragma unroll
        for (int t = 0; t < SCB; t++) {
            if (j0 + t < nn) {
                const double z = lane_value(w, j0 + t) * lane_value(rp, j0 + t);
                if (lane == j0 + t) zl = z;
                if (row && lane > j0 + t) w = fma(-lv[t], z, w);
            }
        }
    }
    if (lane < nn)
        y[f + lane] = zl;
    else if (row)
        upd[uoff[s] + (lane - nn)] = w;
}

// Backward: w_j = y_j - L(rows below, j)^T x(rows below) (summed across the wave as in solve_bwd: lane t on
// row nn + t), then the pivots from the last: x_t = w_t (1 / L_tt), w_j -= L_tj x_t for j < t.
__global__ __launch_bounds__(NT) void solve_bwd_tiny(int nf, const int32_t* __restrict__ list,
                                                     const int32_t* __restrict__ first,
                                                     const int32_t* __restrict__ ncol,
                                                     const int32_t* __restrict__ mrows,
                                                     const int64_t* __restrict__ foff, const int64_t* __restrict__ roff,
                                                     const int32_t* __restrict__ rows,
                                                     const double* __restrict__ fronts, double* __restrict__ y,
                                                     int unit) {
    const int lane = threadIdx.x % 64;
    const int q = blockIdx.x * (NT / 64) + threadIdx.x / 64;
    if (q >= nf) return;
    const int s = list[q];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    const int32_t* R = rows + roff[s];
    const double* L = fronts + foff[s];
    const int nr = m - nn;
    const double xr = lane < nr ? y[R[nn + lane]] : 0.0;  // solved value of row nn + lane
    double w = lane < nn ? y[f + lane] : 0.0;
    for (int j0 = 0; j0 < nn; j0 += SCB) {
        double lv[SCB];  // L(nn + lane, j0 + t)
#pragma unroll
        for (int t = 0; t < SCB; t++) lv[t] = lane < nr && j0 + t < nn ? L[(nn + lane) + m * (j0 + t)] : 0.0;
#pragma unroll
        for (int t = 0; t < SCB; t++) {
            if (j0 + t < nn) {
                const double acc = wave_sum((lv[t] * xr + 0.0) + (0.0 + 0.0));
                if (lane == j0 + t) w -= acc;
            }
        }
    }
    const double rq = lane < nn && !unit ? 1.0 / L[lane + m * lane] : 1.0;
    double xl = 0.0;
    for (int j1 = nn; j1 > 0; j1 -= SCB) {
        double lv[SCB];  // L(j1 - 1 - t, lane)
#pragma unroll
        for (int t = 0; t < SCB; t++) lv[t] = j1 - 1 - t >= 0 && lane < j1 - 1 - t ? L[(j1 - 1 - t) + m * lane] : 0.0;
#pragma unroll
        for (int t = 0; t < SCB; t++) {
            const int p = j1 - 1 - t;
            if (p >= 0) {
                const double x = lane_value(w, p) * lane_value(rq, p);
                if (lane == p) xl = x;
                if (lane < p) w = fma(-lv[t], x, w);
            }
        }
    }
    if (lane < nn) y[f + lane] = xl;
}

// Backward sweep for one front: x(own) = L11^{-T} (y(own) - L21^T x(rows below)).  The products with
// the rows below run one wave per column (lanes over rows, coalesced) on row chunks staged in LDS.
constexpr int XCH = 1024;  // rows per staged chunk

__global__ __launch_bounds__(NT) void solve_bwd(const int32_t* __restrict__ list, const int32_t* __restrict__ first,
                                                const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                                const int64_t* __restrict__ foff, const int64_t* __restrict__ roff,
                                                const int32_t* __restrict__ rows, const double* __restrict__ fronts,
                                                double* __restrict__ work, double* __restrict__ y, int unit) {
    __shared__ double xb[XCH];
    const int s = list[blockIdx.x];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    const int32_t* R = rows + roff[s];
    const double* L = fronts + foff[s];
    double* w = work + roff[s];
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    // a tall front's products with the rows below were formed by solve_bwd_dots (w of its pivots in work)
    const bool tall = m - nn >= TALL;
    if (!tall)
        for (int j = threadIdx.x; j < nn; j += NT) w[j] = y[f + j];
    for (int r0 = nn; r0 < (tall ? nn : m); r0 += XCH) {
        const int nr = min(XCH, m - r0);
        __syncthreads();
        int t = threadIdx.x;
        for (; t + 3 * NT < nr; t += 4 * NT) {
            const int i0 = R[r0 + t], i1 = R[r0 + t + NT], i2 = R[r0 + t + 2 * NT], i3 = R[r0 + t + 3 * NT];
            xb[t] = y[i0];
            xb[t + NT] = y[i1];
            xb[t + 2 * NT] = y[i2];
            xb[t + 3 * NT] = y[i3];
        }
        for (; t < nr; t += NT) xb[t] = y[R[r0 + t]];
        __syncthreads();
        for (int j = wv; j < nn; j += NT / 64) {
            // four independent partial sums per lane, so that four loads of the column are in flight
            const double* col = L + fcol(m, j) + r0;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int t = ln;
            for (; t + 192 < nr; t += 256) {
                a0 += col[t] * xb[t];
                a1 += col[t + 64] * xb[t + 64];
                a2 += col[t + 128] * xb[t + 128];
                a3 += col[t + 192] * xb[t + 192];
            }
            for (; t < nr; t += 64) a0 += col[t] * xb[t];
            const double acc = wave_sum((a0 + a1) + (a2 + a3));
            if (ln == 0) w[j] -= acc;
        }
    }
    // the pivot block L11^T in blocks of SCB columns from the last: wave 0 solves the diagonal block in
    // registers (solved values to xx), then every thread applies the block's values to its earlier rows,
    // all SCB loads of a row in flight at once.  Each w[i] takes the solved values in decreasing order, one
    // fused multiply-add each, as a pivot-by-pivot sweep would.
    __shared__ double xx[WIDE];
    __syncthreads();  // w of the pivots is complete
    for (int j1 = nn; j1 > 0; j1 -= SCB) {
        const int j0 = max(0, j1 - SCB), cb = j1 - j0;
        if (threadIdx.x < 64) {
            const bool act = ln < cb;
            double a[SCB];  // lane q: a[t] = L(j0 + t, j0 + q), t > q
            const double* Lq = L + fcol(m, j0 + (act ? ln : 0));  // column j0 + ln
#pragma unroll
            for (int t = 0; t < SCB; t++) a[t] = (act && t > ln && t < cb) ? Lq[j0 + t] : 0.0;
            double wq = act ? w[j0 + ln] : 0.0;
            const double rq = act && !unit ? 1.0 / Lq[j0 + ln] : 1.0;
#pragma unroll
            for (int t = SCB - 1; t >= 0; t--) {
                if (t >= cb) continue;
                const double x = lane_value(wq, t) * lane_value(rq, t);
                if (ln < t) wq = fma(-a[t], x, wq);
                if (ln == t) xx[j0 + t] = x;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < j0; i += NT) {
            double lv[SCB];
            const double* Li = L + fcol(m, i) + j0;  // column i from row j0
#pragma unroll
            for (int t = 0; t < SCB; t++) lv[t] = t < cb ? Li[t] : 0.0;
            double acc = w[i];
#pragma unroll
            for (int t = SCB - 1; t >= 0; t--)
                if (t < cb) acc = fma(-lv[t], xx[j0 + t], acc);
            w[i] = acc;
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < nn; j += NT) y[f + j] = xx[j];
}

// Products of a tall front's pivot columns with the solved values at its rows below, 16 columns per work-group
// (item: front, column block): w_j = y_j - L21(:, j)^T x(rows below) for its columns, written to the front's
// slice of work for solve_bwd.  The solved values are staged into LDS up to XBT rows at a time (eight row
// indices, then eight values, in flight per thread); each wave forms four columns' products side by side,
// four partial sums each, combined in a fixed order.
constexpr int XBT = 8192;  // rows of solved values staged per pass (64 KB)
__global__ __launch_bounds__(NT) void solve_bwd_dots(const int32_t* __restrict__ items,
                                                     const int32_t* __restrict__ first,
                                                     const int32_t* __restrict__ ncol,
                                                     const int32_t* __restrict__ mrows,
                                                     const int64_t* __restrict__ foff, const int64_t* __restrict__ roff,
                                                     const int32_t* __restrict__ rows,
                                                     const double* __restrict__ fronts, double* __restrict__ work,
                                                     const double* __restrict__ y) {
    __shared__ double xb[XBT];
    const int s = items[2 * blockIdx.x], cb = items[2 * blockIdx.x + 1];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    const int32_t* R = rows + roff[s];
    const double* L = fronts + foff[s];
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    constexpr int KW = SCB / 4;
    double wj[KW];
    bool on[KW];
#pragma unroll
    for (int k = 0; k < KW; k++) {
        const int j = SCB * cb + wv + 4 * k;
        on[k] = j < nn;
        wj[k] = on[k] ? y[f + j] : 0.0;
    }
    for (int r0 = nn; r0 < m; r0 += XBT) {
        const int nr = min(XBT, m - r0);
        __syncthreads();
        for (int t0 = threadIdx.x; t0 < nr; t0 += 8 * NT) {
            int ri[8];
#pragma unroll
            for (int q = 0; q < 8; q++) ri[q] = t0 + q * NT < nr ? R[r0 + t0 + q * NT] : -1;
#pragma unroll
            for (int q = 0; q < 8; q++)
                if (ri[q] >= 0) xb[t0 + q * NT] = y[ri[q]];
        }
        __syncthreads();
        const double* col[KW];
        double a[KW][4];
#pragma unroll
        for (int k = 0; k < KW; k++) {
            col[k] = L + fcol(m, on[k] ? SCB * cb + wv + 4 * k : 0) + r0;
            a[k][0] = a[k][1] = a[k][2] = a[k][3] = 0.0;
        }
        int t = ln;
        // two steps' loads (32 per lane) issued before their multiply-adds
        for (; t + 448 < nr; t += 512) {
            double v[2][KW][4];
#pragma unroll
            for (int h = 0; h < 2; h++)
#pragma unroll
                for (int k = 0; k < KW; k++)
#pragma unroll
                    for (int p = 0; p < 4; p++) v[h][k][p] = on[k] ? col[k][t + 256 * h + 64 * p] : 0.0;
#pragma unroll
            for (int h = 0; h < 2; h++)
#pragma unroll
                for (int k = 0; k < KW; k++)
#pragma unroll
                    for (int p = 0; p < 4; p++) a[k][p] += v[h][k][p] * xb[t + 256 * h + 64 * p];
        }
        for (; t + 192 < nr; t += 256) {
#pragma unroll
            for (int k = 0; k < KW; k++)
                if (on[k]) {
                    a[k][0] += col[k][t] * xb[t];
                    a[k][1] += col[k][t + 64] * xb[t + 64];
                    a[k][2] += col[k][t + 128] * xb[t + 128];
                    a[k][3] += col[k][t + 192] * xb[t + 192];
                }
        }
        for (; t < nr; t += 64)
#pragma unroll
            for (int k = 0; k < KW; k++)
                if (on[k]) a[k][0] += col[k][t] * xb[t];
#pragma unroll
        for (int k = 0; k < KW; k++)
            if (on[k]) wj[k] -= wave_sum((a[k][0] + a[k][1]) + (a[k][2] + a[k][3]));
    }
    if (ln == 0)
#pragma unroll
        for (int k = 0; k < KW; k++)
            if (on[k]) work[roff[s] + SCB * cb + wv + 4 * k] = wj[k];
}

// ---------------------------------------------------------------- sync-free solves for wide fronts
// A front with many pivots is solved by one launch per sweep whose work-groups each own a 64-row
// (forward) or 64-column (backward) block of the front.  A block's work-group multiplies its part of
// L with every solved block as soon as that block has arrived, then solves with its own diagonal block
// in registers (one wave, pivots read lane by lane) and publishes its block.  Every wait is on a
// lower-numbered work-group, and work-groups are dispatched in index order, so a waiting work-group
// never holds back the one it waits for.  Solved blocks go through device-coherent (agent-scope) stores
// and loads, because the work-groups of a launch sit on dies with separate L2 caches.  A wait is
// bounded: past the spin limit the fault word is raised and the work-group goes on (the result is then
// invalid and reported).
constexpr int WLDS = 8192; // rows of a narrow front's forward vector kept in LDS (64 KB)
constexpr int SB = 64;     // block edge of the sync-free solves

__device__ __forceinline__ void store_coherent(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_coherent(const double* p) {
    return __longlong_as_double((long long)__hip_atomic_load(
        reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// forward, step 0 of a wide front: w = [y(own rows), 0] + the children's update entries, one thread per row
// (children in ascending order), the rows spread over work-groups
__global__ __launch_bounds__(NT) void sfwd_gather(int s, const int32_t* __restrict__ first,
                                                  const int32_t* __restrict__ ncol, const int32_t* __restrict__ mrows,
                                                  const int64_t* __restrict__ roff, const int64_t* __restrict__ gptr,
                                                  const int64_t* __restrict__ gsrc, double* __restrict__ work,
                                                  const double* __restrict__ upd, const double* __restrict__ y) {
    const int m = mrows[s], nn = ncol[s], f = first[s];
    const int t = blockIdx.x * NT + threadIdx.x;
    if (t >= m) return;
    const int64_t* gp = gptr + roff[s];
    work[roff[s] + t] = row_gather(t < nn ? y[f + t] : 0.0, gp[t], gp[t + 1], gsrc, upd);
}

// Solved blocks travel through an exchange buffer zx (64 doubles per pivot block) that is filled with the
// sentinel NaN pattern before each sweep: a block is ready when none of its 64 entries is the sentinel,
// so the data is its own ready flag (one memory round trip per hand-over instead of two).
__global__ void fill_sentinel(int64_t n, double* __restrict__ p) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = __longlong_as_double((long long)SENTINEL_BITS);
}

// The calling wave waits until block c of zx is complete and returns its lane's value of it; every wave
// polls for itself, so a work-group needs neither LDS nor a barrier per block.  Bounded: past the spin
// limit the fault word is raised and the block is taken as it is.
__device__ __forceinline__ double take_block_wave(const double* __restrict__ zx, int c, int32_t* __restrict__ fault,
                                                  bool& alive) {
    const int lane = threadIdx.x % 64;
    double v = load_coherent(zx + SB * c + lane);
    int spins = 0;
    while (alive && __any(is_sentinel(v))) {
        if (++spins > (1 << 20)) {
            alive = false;
            if (lane == 0) __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = load_coherent(zx + SB * c + lane);
    }
    return v;
}

// Inverse of one 64 x 64 diagonal block of a wide front (one wave per block, identity padding past the last
// pivot), column-major into winv: lane j forms column j by forward substitution, the block and its reciprocal
// pivots read as broadcasts from LDS.  The sweeps then solve with a block as one product instead of 64
// dependent steps.
__global__ __launch_bounds__(64) void wide_inverse(const int32_t* __restrict__ items,
                                                   const int32_t* __restrict__ ncol,
                                                   const int32_t* __restrict__ mrows,
                                                   const int64_t* __restrict__ foff, const double* __restrict__ fronts,
                                                   double* __restrict__ winv, int unit) {
    __shared__ __attribute__((aligned(16))) double Ls[SB * SB];  // Ls[i * 64 + k] = L(i, k) of the block
    __shared__ double ri[SB];
    const int s = items[3 * blockIdx.x], g = items[3 * blockIdx.x + 1];
    const int64_t ob = items[3 * blockIdx.x + 2];
    const int m = mrows[s], nn = ncol[s];
    const int r0 = SB * g, nb = min(SB, nn - r0);
    const double* L = fronts + foff[s] + fcol(m, r0) + r0;  // the block's panel, column stride ld
    const int64_t ld = fld(m, r0);
    const int j = threadIdx.x;
    for (int k = 0; k < SB; k++)
        Ls[j * SB + k] = (j < nb && k < nb) ? (j >= k ? L[j + ld * k] : 0.0) : (j == k ? 1.0 : 0.0);
    __syncthreads();
    ri[j] = unit ? 1.0 : 1.0 / Ls[j * SB + j];
    __syncthreads();
    // row i of L is contiguous in LDS (pairs of broadcasts per read); two partial sums per row
    double x[SB];
#pragma unroll
    for (int i = 0; i < SB; i++) {
        double a0 = i == j ? 1.0 : 0.0, a1 = 0.0;
#pragma unroll
        for (int k = 0; k + 1 < i; k += 2) {
            const double2 l = *reinterpret_cast<const double2*>(&Ls[i * SB + k]);
            a0 = fma(-l.x, x[k], a0);
            a1 = fma(-l.y, x[k + 1], a1);
        }
        if (i % 2 == 1) a0 = fma(-Ls[i * SB + i - 1], x[i - 1], a0);
        x[i] = (a0 + a1) * ri[i];
    }
    double* out = winv + ob * SB * SB + (int64_t)SB * j;  // column j
#pragma unroll
    for (int i = 0; i < SB; i++) out[i] = x[i];
}

// forward sweep of one wide front.  Work-group g < nblk owns pivot rows [64g, 64g + 64): it subtracts
// L(rows, block c) z_c for every c < g as soon as z_c is in zx, solves with L(g, g) and publishes z_g
// (to zx, device-coherent, and to y).  The remaining work-groups own 64-row blocks of the rows below
// the pivots and write their partial result to upd.  Thread (i, q) = (row in block, quarter of the 64
// columns of a block).
__global__ __launch_bounds__(NT) void wide_fwd(int s, double* __restrict__ zx, int32_t* __restrict__ fault,
                                               const int32_t* __restrict__ first, const int32_t* __restrict__ ncol,
                                               const int32_t* __restrict__ mrows, const int64_t* __restrict__ foff,
                                               const int64_t* __restrict__ roff, const int64_t* __restrict__ uoff,
                                               const double* __restrict__ fronts, const double* __restrict__ work,
                                               double* __restrict__ upd, double* __restrict__ y,
                                               const double* __restrict__ winv) {
    __shared__ double red[NT / 64][SB];
    __shared__ double wsh[SB];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    const int nblk = (nn + SB - 1) / SB;
    const int g = blockIdx.x;
    const bool piv = g < nblk;
    const int r0 = piv ? SB * g : nn + SB * (g - nblk);
    const int nr = min(SB, (piv ? nn : m) - r0);
    const int ncb = piv ? g : nblk;
    const double* L = fronts + foff[s];
    const int i = threadIdx.x % 64, q = threadIdx.x / 64;
    const bool rowok = i < nr;
    const double* Lr = L + (rowok ? r0 + i : 0);  // row r0 + i
    // row i of the inverse of the own diagonal block (wave 0, read before any wait; zero above the diagonal)
    double v[SB];
    const double* Vi = winv + (int64_t)g * SB * SB + i;  // Vi[64 j] = inv(L_gg)(i, j)
#pragma unroll
    for (int j = 0; j < SB; j++) v[j] = (piv && q == 0 && j <= i) ? Vi[(int64_t)SB * j] : 0.0;
    const double w0 = (q == 0 && rowok) ? work[roff[s] + r0 + i] : 0.0;  // the right-hand side, also early
    double acc = 0.0;
    bool alive = true;
    for (int c = 0; c < ncb; c++) {
        const int c0 = SB * c, kc = min(SB, nn - c0);
        const double* Lc = Lr + fcol(m, c0);  // block c is one panel: column c0 + j at Lc + ld j
        const int64_t ld = fld(m, c0);
        double lv[16];
#pragma unroll
        for (int jj = 0; jj < 16; jj++) {
            const int j = 16 * q + jj;
            lv[jj] = (rowok && j < kc) ? Lc[ld * j] : 0.0;
        }
        const double zv = take_block_wave(zx, c, fault, alive);
#pragma unroll
        for (int jj = 0; jj < 16; jj++) acc += lv[jj] * lane_value(zv, 16 * q + jj);
    }
    red[q][i] = acc;
    __syncthreads();
    if (q != 0) return;
    double wi = rowok ? w0 - ((red[0][i] + red[1][i]) + (red[2][i] + red[3][i])) : 0.0;
    if (!piv) {
        if (rowok) upd[uoff[s] + (r0 - nn) + i] = wi;
        return;
    }
    // z_g = inv(L_gg) w_g (rows past the last pivot carry w = 0 and identity rows of the inverse)
    wsh[i] = wi;  // read back by the other lanes of this wave (LDS keeps a wave's accesses in order)
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
    for (int j = 0; j < SB; j += 4) {
        p0 = fma(v[j], wsh[j], p0);
        p1 = fma(v[j + 1], wsh[j + 1], p1);
        p2 = fma(v[j + 2], wsh[j + 2], p2);
        p3 = fma(v[j + 3], wsh[j + 3], p3);
    }
    const double u = (p0 + p1) + (p2 + p3);
    store_coherent(zx + SB * g + i, rowok ? u : 0.0);
    if (rowok) y[f + r0 + i] = u;
}

// backward sweep of one wide front.  Work-group g owns pivot block b = nblk - 1 - g (columns
// [64b, 64b + 64)): it subtracts L(rows, b)^T x for the rows below the pivots (solved by the
// ancestors) and for every later block c > b as soon as x_c is in zx, then solves with L(b, b)^T
// and publishes x_b (to zx and y).  Thread (j, q) = (column in block, quarter of the 64 rows of a block).
__global__ __launch_bounds__(NT) void wide_bwd(int s, double* __restrict__ zx, int32_t* __restrict__ fault,
                                               const int32_t* __restrict__ first, const int32_t* __restrict__ ncol,
                                               const int32_t* __restrict__ mrows, const int64_t* __restrict__ foff,
                                               const int64_t* __restrict__ roff, const int32_t* __restrict__ rows,
                                               const double* __restrict__ fronts, double* __restrict__ y,
                                               const double* __restrict__ winv) {
    __shared__ double xs[SB];
    __shared__ double tsh[SB];
    __shared__ double red[NT / 64][SB];
    const int m = mrows[s], nn = ncol[s], f = first[s];
    const int nblk = (nn + SB - 1) / SB;
    const int g = blockIdx.x;
    const int b = nblk - 1 - g;
    const int c0 = SB * b, kb = min(SB, nn - c0);
    const int32_t* R = rows + roff[s];
    const int j = threadIdx.x % 64, q = threadIdx.x / 64;
    const bool colok = j < kb;
    const double* Lc = fronts + foff[s] + fcol(m, c0 + (colok ? j : 0));  // column c0 + j
    // column j of the inverse of the own diagonal block (wave 0; zero above the diagonal of the inverse)
    double v[SB];
    const double* Vj = winv + (int64_t)b * SB * SB + (int64_t)SB * j;  // Vj[t] = inv(L_bb)(t, j)
#pragma unroll
    for (int t = 0; t < SB; t++) v[t] = (q == 0 && t >= j) ? Vj[t] : 0.0;
    const double t0 = (q == 0 && colok) ? y[f + c0 + j] : 0.0;  // this block's forward solution, also early
    double acc = 0.0;
    for (int r0 = nn; r0 < m; r0 += SB) {
        const int nr = min(SB, m - r0);
        double lv[16];
#pragma unroll
        for (int ii = 0; ii < 16; ii++) {
            const int r = 16 * q + ii;
            lv[ii] = (colok && r < nr) ? Lc[r0 + r] : 0.0;
        }
        __syncthreads();
        if (threadIdx.x < SB) xs[threadIdx.x] = (int)threadIdx.x < nr ? y[R[r0 + threadIdx.x]] : 0.0;
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < 16; ii++) acc += lv[ii] * xs[16 * q + ii];
    }
    bool alive = true;
    for (int c = nblk - 1; c > b; c--) {
        const int cr0 = SB * c, nr = min(SB, nn - cr0);
        double lv[16];
#pragma unroll
        for (int ii = 0; ii < 16; ii++) {
            const int r = 16 * q + ii;
            lv[ii] = (colok && r < nr) ? Lc[cr0 + r] : 0.0;
        }
        const double xv = take_block_wave(zx, c, fault, alive);
#pragma unroll
        for (int ii = 0; ii < 16; ii++) acc += lv[ii] * lane_value(xv, 16 * q + ii);
    }
    red[q][j] = acc;
    __syncthreads();
    if (q != 0) return;
    double tj = colok ? t0 - ((red[0][j] + red[1][j]) + (red[2][j] + red[3][j])) : 0.0;
    // x_b = inv(L_bb)^T t_b
    tsh[j] = tj;  // read back by the other lanes of this wave
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
    for (int t = 0; t < SB; t += 4) {
        p0 = fma(v[t], tsh[t], p0);
        p1 = fma(v[t + 1], tsh[t + 1], p1);
        p2 = fma(v[t + 2], tsh[t + 2], p2);
        p3 = fma(v[t + 3], tsh[t + 3], p3);
    }
    const double u = (p0 + p1) + (p2 + p3);
    store_coherent(zx + SB * b + j, colok ? u : 0.0);
    if (colok) y[f + c0 + j] = u;
}

// L D L^T solves: y <- D^{-1} y between the forward and the backward sweep.
__global__ void dscale(int n, const double* __restrict__ dval, double* __restrict__ y) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = y[k] / dval[k];
}

// Number of negative pivots of an L D L^T factorization (by Sylvester's law of inertia, the number of negative
// eigenvalues of K when no pivot was rejected), one work-group.
constexpr int CNT_NT = 1024;
__global__ __launch_bounds__(CNT_NT) void count_negative(int n, const double* __restrict__ dval,
                                                         int64_t* __restrict__ out) {
    __shared__ int64_t red[CNT_NT / 64];
    int64_t c = 0;
    for (int k = threadIdx.x; k < n; k += CNT_NT) c += dval[k] < 0.0;
    for (int o = 32; o > 0; o >>= 1) c += (int64_t)__shfl_xor((long long)c, o);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < CNT_NT / 64; w++) c += red[w];
        out[0] = c;
    }
}

}  // namespace

// ------------------------------------------------------------------------ host side
namespace opf {
void chol_set_stream(chol_sym* C, hipStream_t st);
}
static void build_numeric_plan(chol_sym* C, const std::vector<int32_t>& colptr, const std::vector<int32_t>& rowind) {
    const Symbolic& S = C->S;
    const int ns = S.nsuper, n = S.n;
    C->h_first.resize(ns);
    C->h_ncol.resize(ns);
    C->h_mrows.resize(ns);
    C->h_foff.resize(ns + 1);
    C->h_roff.resize(ns + 1);
    C->h_uoff.resize(ns + 1);
    int64_t fo = 0, uo = 0;
    double flops = 0;
    int64_t nnzl = 0;
    for (int s = 0; s < ns; s++) {
        int f = S.snode_ptr[s], nn = S.snode_ptr[s + 1] - f;
        int64_t m = S.rows_ptr[s + 1] - S.rows_ptr[s];
        C->h_first[s] = f;
        C->h_ncol[s] = nn;
        C->h_mrows[s] = (int32_t)m;
        C->h_foff[s] = fo;
        C->h_roff[s] = S.rows_ptr[s];
        C->h_uoff[s] = uo;
        fo += front_doubles(m);
        uo += m - nn;
        nnzl += (int64_t)nn * m - (int64_t)nn * (nn - 1) / 2;
        for (int j = 0; j < nn; j++) {
            double c = (double)(m - j);
            flops += c * c;
        }
    }
    C->h_foff[ns] = fo;
    C->h_roff[ns] = S.rows_ptr[ns];
    C->h_uoff[ns] = uo;
    C->front_total = fo;
    C->upd_total = uo;
    C->nnzl = nnzl;
    C->flops = flops;
    // children lists and relative indices of each child's update rows in its parent
    std::vector<int32_t> cptr(ns + 1, 0), clist;
    for (int s = 0; s < ns; s++)
        if (S.sparent[s] >= 0) cptr[S.sparent[s] + 1]++;
    for (int s = 0; s < ns; s++) cptr[s + 1] += cptr[s];
    clist.resize(cptr[ns]);
    {
        std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
        for (int s = 0; s < ns; s++)
            if (S.sparent[s] >= 0) clist[fill[S.sparent[s]]++] = s;
    }
    std::vector<int64_t> reloff(ns + 1, 0);
    std::vector<int32_t> rel;
    std::vector<int32_t> pos(n, -1);
    for (int s = 0; s < ns; s++) {
        reloff[s] = (int64_t)rel.size();
        int p = S.sparent[s];
        int m = C->h_mrows[s], nn = C->h_ncol[s];
        if (p < 0) continue;
        const int32_t* Rp = S.rows_flat.data() + S.rows_ptr[p];
        int mp = C->h_mrows[p];
        for (int t = 0; t < mp; t++) pos[Rp[t]] = t;
        const int32_t* Rs = S.rows_flat.data() + S.rows_ptr[s];
        for (int t = nn; t < m; t++) rel.push_back(pos[Rs[t]]);
        for (int t = 0; t < mp; t++) pos[Rp[t]] = -1;
    }
    reloff[ns] = (int64_t)rel.size();
    // levels: height above the leaves
    std::vector<int32_t> level(ns, 0);
    for (int s = 0; s < ns; s++)
        if (S.sparent[s] >= 0) level[S.sparent[s]] = std::max(level[S.sparent[s]], level[s] + 1);
    int nl = 0;
    for (int s = 0; s < ns; s++) nl = std::max(nl, level[s] + 1);
    C->nlevels = nl;
    C->h_level = level;
    C->lvl_ptr.assign(nl + 1, 0);
    for (int s = 0; s < ns; s++) C->lvl_ptr[level[s] + 1]++;
    for (int l = 0; l < nl; l++) C->lvl_ptr[l + 1] += C->lvl_ptr[l];
    C->lvl_sn.resize(ns);
    {
        std::vector<int32_t> fill(C->lvl_ptr.begin(), C->lvl_ptr.end() - 1);
        for (int s = 0; s < ns; s++) C->lvl_sn[fill[level[s]]++] = s;
    }
    C->lvl_small_ptr.assign(nl + 1, 0);
    C->lvl_small.clear();
    C->lvl_small_maxm.clear();
    C->lvl_small_lda.clear();
    C->lvl_narrow_ptr.assign(nl + 1, 0);
    C->lvl_narrow_maxm.clear();
    C->lvl_wide_ptr.assign(nl + 1, 0);
    C->lvl_narrow.clear();
    C->lvl_wide.clear();
    for (int l = 0; l < nl; l++) {
        for (int q = C->lvl_ptr[l]; q < C->lvl_ptr[l + 1]; q++) {
            int s = C->lvl_sn[q];
            (C->h_ncol[s] >= WIDE ? C->lvl_wide : C->lvl_narrow).push_back(s);
        }
        C->lvl_narrow_ptr[l + 1] = (int32_t)C->lvl_narrow.size();
        int mx = 0;
        for (int q = C->lvl_narrow_ptr[l]; q < C->lvl_narrow_ptr[l + 1]; q++)
            mx = std::max(mx, C->h_mrows[C->lvl_narrow[q]]);
        C->lvl_narrow_maxm.push_back(mx);
        C->lvl_wide_ptr[l + 1] = (int32_t)C->lvl_wide.size();
    }
    C->lvl_trow_ptr.assign(nl + 1, 0);
    C->lvl_tcol_ptr.assign(nl + 1, 0);
    C->trow_it.clear();
    C->tcol_it.clear();
    for (int l = 0; l < nl; l++) {
        for (int q = C->lvl_narrow_ptr[l]; q < C->lvl_narrow_ptr[l + 1]; q++) {
            const int s = C->lvl_narrow[q], m = C->h_mrows[s], nn = C->h_ncol[s];
            if (m - nn < TALL) continue;
            for (int rb = 0; rb * NT < m - nn; rb++) {
                C->trow_it.push_back(s);
                C->trow_it.push_back(rb);
            }
            for (int cb = 0; cb * SCB < nn; cb++) {
                C->tcol_it.push_back(s);
                C->tcol_it.push_back(cb);
            }
        }
        C->lvl_trow_ptr[l + 1] = (int32_t)C->trow_it.size() / 2;
        C->lvl_tcol_ptr[l + 1] = (int32_t)C->tcol_it.size() / 2;
    }
    // assembly tiles and K entries per tile
    std::vector<int32_t> tsn, trc;
    C->asm_ptr.assign(nl + 1, 0);
    std::vector<int64_t> tile_of_front_start(ns, 0);
    for (int l = 0; l < nl; l++) {
        for (int q = C->lvl_ptr[l]; q < C->lvl_ptr[l + 1]; q++) {
            int s = C->lvl_sn[q];
            int m = C->h_mrows[s];
            if (m <= TB) C->lvl_small.push_back(s);
            int T = (m + TB - 1) / TB;
            tile_of_front_start[s] = (int64_t)tsn.size();
            for (int tc = 0; tc < T; tc++)
                for (int tr = tc; tr < T; tr++) {
                    tsn.push_back(s);
                    trc.push_back((tr << 16) | tc);
                }
        }
        C->lvl_small_ptr[l + 1] = (int32_t)C->lvl_small.size();
        int mx = 1;
        for (int q = C->lvl_small_ptr[l]; q < C->lvl_small_ptr[l + 1]; q++)
            mx = std::max(mx, C->h_mrows[C->lvl_small[q]]);
        const bool all_small = C->lvl_small_ptr[l + 1] - C->lvl_small_ptr[l] == C->lvl_ptr[l + 1] - C->lvl_ptr[l];
        C->lvl_small_maxm.push_back(all_small ? mx : 0);
        C->lvl_small_lda.push_back(mx);
        C->asm_ptr[l + 1] = (int32_t)tsn.size();
    }
    // K entry (original numbering, lower CSC) -> tile and in-tile position
    const int64_t nk = rowind.size();
    std::vector<int64_t> ktile(nk);
    std::vector<int32_t> kpos(nk);
    for (int jo = 0; jo < n; jo++) {
        for (int p = colptr[jo]; p < colptr[jo + 1]; p++) {
            int a = S.iperm[rowind[p]], b = S.iperm[jo];
            int r = std::max(a, b), c = std::min(a, b);
            int s = S.col2sn[c];
            const int32_t* R = S.rows_flat.data() + S.rows_ptr[s];
            int m = C->h_mrows[s], nn = C->h_ncol[s];
            int lc = c - C->h_first[s];
            int lr;
            if (r - C->h_first[s] < nn)
                lr = r - C->h_first[s];
            else
                lr = (int)(std::lower_bound(R + nn, R + m, r) - R);
            int tr = lr / TB, tc = lc / TB;
            int T = (m + TB - 1) / TB;
            // tiles of a front are ordered by column then row (tr >= tc)
            int64_t tidx = tile_of_front_start[s];
            for (int cc = 0; cc < tc; cc++) tidx += T - cc;
            tidx += tr - tc;
            ktile[p] = tidx;
            kpos[p] = (lr - tr * TB) + TB * (lc - tc * TB);
        }
    }
    std::vector<int64_t> tkptr(tsn.size() + 1, 0);
    for (int64_t p = 0; p < nk; p++) tkptr[ktile[p] + 1]++;
    for (size_t t = 0; t < tsn.size(); t++) tkptr[t + 1] += tkptr[t];
    std::vector<int32_t> tk(nk), tkpos(nk);
    {
        std::vector<int64_t> fill(tkptr.begin(), tkptr.end() - 1);
        for (int64_t p = 0; p < nk; p++) {
            int64_t q = fill[ktile[p]]++;
            tk[q] = (int32_t)p;
            tkpos[q] = kpos[p];
        }
    }
    // per tile: the children whose update matrices reach it, each with its row range [ra, rb) and column
    // range [ca, cb) in the child's update-row numbering (relative indices are increasing, so each child
    // contributes one rectangle per tile); children stay in ascending order, which fixes the summation order
    std::vector<int64_t> tcptr(tsn.size() + 1, 0);
    std::vector<int32_t> tcrec;  // 5 ints per entry: child, ra, rb, ca, cb
    for (int pass = 0; pass < 2; pass++) {  // count, then fill
        std::vector<int64_t> fill;
        if (pass == 1) {
            for (size_t t = 0; t < tsn.size(); t++) tcptr[t + 1] += tcptr[t];
            tcrec.resize(5 * tcptr.back());
            fill.assign(tcptr.begin(), tcptr.end() - 1);
        }
        std::vector<int32_t> lo;
        for (int sp = 0; sp < ns; sp++) {
            const int mp = C->h_mrows[sp], T = (mp + TB - 1) / TB;
            for (int ci = cptr[sp]; ci < cptr[sp + 1]; ci++) {
                const int c = clist[ci];
                const int nu = C->h_mrows[c] - C->h_ncol[c];
                const int32_t* rl = rel.data() + reloff[c];
                // start of each row tile of the parent in the child's update rows
                lo.assign(T + 1, nu);
                for (int t = 0, u = 0; t <= T; t++) {
                    while (u < nu && rl[u] < t * TB) u++;
                    lo[t] = u;
                }
                for (int tc = 0; tc < T; tc++) {
                    if (lo[tc + 1] == lo[tc]) continue;
                    for (int tr = tc; tr < T; tr++) {
                        if (lo[tr + 1] == lo[tr]) continue;
                        // tiles of a front are ordered by column then row (tr >= tc)
                        const int64_t tidx = tile_of_front_start[sp] + (int64_t)tc * T - (int64_t)tc * (tc - 1) / 2 +
                                             (tr - tc);
                        if (pass == 0) {
                            tcptr[tidx + 1]++;
                        } else {
                            int32_t* r = tcrec.data() + 5 * fill[tidx]++;
                            r[0] = c;
                            r[1] = lo[tr];
                            r[2] = lo[tr + 1];
                            r[3] = lo[tc];
                            r[4] = lo[tc + 1];
                        }
                    }
                }
            }
        }
    }
    // dense fronts: tile task lists per level (see dense_front)
    C->is_dense.assign(ns, 0);
    for (int s2 = 0; s2 < ns; s2++) C->is_dense[s2] = C->opts.tile_min > 0 && C->h_ncol[s2] >= C->opts.tile_min;
    std::vector<int32_t> dhs, dhnp, dhnb, dhslot0, dth, dtrc;
    std::vector<int64_t> dht0;
    int dslots = 0;
    C->lvl_dense_ptr.assign(nl + 1, 0);
    C->lvl_dense_flops.assign(nl, 0.0);
    for (int l = 0; l < nl; l++) {
        for (int q = C->lvl_ptr[l]; q < C->lvl_ptr[l + 1]; q++) {
            const int s2 = C->lvl_sn[q];
            if (!C->is_dense[s2]) continue;
            const int m = C->h_mrows[s2], nn = C->h_ncol[s2];
            const int np = (nn + DT - 1) / DT, nu = (m - nn + DT - 1) / DT, nb = np + nu;
            OPF_CHECK(nb < 32768, OPF_E_INVALID, "chol_analyze: dense front of %d rows is too large", m);
            const int h = (int)dhs.size();
            dhs.push_back(s2);
            dhnp.push_back(np);
            dhnb.push_back(nb);
            dht0.push_back((int64_t)dth.size());
            dhslot0.push_back(dslots);
            dslots += np;
            for (int bj = 0; bj < nb; bj++)
                for (int bi = bj; bi < nb; bi++) {
                    dth.push_back(h);
                    dtrc.push_back((bi << 16) | bj);
                }
            for (int j = 0; j < nn; j++) C->lvl_dense_flops[l] += (double)(m - j) * (double)(m - j);
        }
        C->lvl_dense_ptr[l + 1] = (int32_t)dth.size();
    }
    OPF_CHECK(dth.size() < (size_t)INT32_MAX, OPF_E_INVALID, "chol_analyze: too many dense-front tiles");
    if (!dhs.empty()) {
        C->dev.upload(C->dh_s, dhs);
        C->dev.upload(C->dh_np, dhnp);
        C->dev.upload(C->dh_nb, dhnb);
        C->dev.upload(C->dh_t0, dht0);
        C->dev.upload(C->dh_slot0, dhslot0);
        C->dev.upload(C->dtask_h, dth);
        C->dev.upload(C->dtask_rc, dtrc);
        C->dev.upload(C->dflags, std::vector<int32_t>(dth.size(), 0));
        C->dev.upload(C->dcounter, std::vector<int32_t>(1, 0));
        C->dev.alloc(C->tdiag, (int64_t)dslots * TB * TB);
        C->dev.alloc(C->trdiag, (int64_t)dslots * TB);
    }
    C->dev.upload(C->ffault, std::vector<int32_t>(1, 0));
    // blocked-path work lists per level and step for the other fronts with m > 64.  A level whose only
    // blocked front has at least chol_options.pair_min pivots (0: never) pairs its 64-column panels: the first panel of a pair
    // updates only the second panel's columns, and the second panel's step applies both panels to the rest
    // of the front as one rank-128 update (half the passes over the trailing matrix).
    std::vector<int32_t> pot, trs, syr, nslot;
    int max_slots = 0;
    C->steps.clear();
    C->lvl_step_ptr.assign(nl + 1, 0);
    for (int l = 0; l < nl; l++) {
        int maxsteps = 0, nblocked = 0, only = -1;
        for (int q = C->lvl_ptr[l]; q < C->lvl_ptr[l + 1]; q++) {
            int s = C->lvl_sn[q];
            if (C->h_mrows[s] > TB && !C->is_dense[s]) {
                maxsteps = std::max(maxsteps, (C->h_ncol[s] + TB - 1) / TB);
                nblocked++;
                only = s;
            }
        }
        const bool paired = nblocked == 1 && C->opts.pair_min > 0 && C->h_ncol[only] >= C->opts.pair_min;
        // pairs cover the leading steps whose pair still leaves at least pair_min rows below it (where the
        // update is bound by passes over a large trailing matrix); the later, latency-bound steps are single
        // groups of G = pair_panels panels (2: pairs); within a group, every step but the last updates only the
        // group's next panel, the last applies the whole group to the rest of the front (rank 64 G)
        const int G = std::max(2, std::min(C->opts.pair_panels, 8));
        int npair_steps = 0;
        if (paired) {
            const int nn = C->h_ncol[only], m = C->h_mrows[only];
            while ((npair_steps + G) * TB < nn && m - (npair_steps + G) * TB >= C->opts.pair_min) npair_steps += G;
        }
        for (int k = 0; k < maxsteps; k++) {
            // step kind 1 = a panel of a group before its last, 2 = the group's last panel (rank-64 G update);
            // gpos = position in the group
            int kind = 0, gpos = 0;
            if (k < npair_steps) {
                gpos = k % G;
                kind = gpos < G - 1 ? 1 : 2;
            }
            chol_sym::Step st{l, (int32_t)pot.size() / 2, 0, (int32_t)trs.size() / 4, 0, 0, 0, 0, 0, TB};
            for (int q = C->lvl_ptr[l]; q < C->lvl_ptr[l + 1]; q++) {
                int s = C->lvl_sn[q];
                int m = C->h_mrows[s], nn = C->h_ncol[s];
                if (m <= TB || C->is_dense[s]) continue;
                int k0 = k * TB;
                if (k0 >= nn) continue;
                int kb = std::min(TB, nn - k0);
                const int slot = (int)pot.size() / 2 - st.p0;  // this item's diagonal-block slot in the step
                pot.push_back(s);
                pot.push_back(k0);
                int rest = m - k0 - kb;
                int Tr = (rest + TR - 1) / TR;
                for (int rb = 0; rb < Tr; rb++) {
                    trs.push_back(s);
                    trs.push_back(k0);
                    trs.push_back(rb);
                    trs.push_back(slot);
                }
            }
            st.p1 = (int32_t)pot.size() / 2;
            st.t1 = (int32_t)trs.size() / 4;
            max_slots = std::max(max_slots, st.p1 - st.p0);
            // trailing update: the next panel's 64 columns (128 x 64 tiles), then the rest (128 x 128); the
            // items carry the first column of the panels applied, the step their total width
            const int kfirst = (k - gpos) * TB;  // first column of the group's panels applied by this step
            if (kind != 0 && only >= 0) st.kw = std::min(k * TB + TB, C->h_ncol[only]) - kfirst;
            for (int pass = 0; pass < 2; pass++) {
                if (pass == 0)
                    st.s0 = (int32_t)syr.size() / 4;
                else
                    st.r0 = (int32_t)syr.size() / 4;
                if (pass == 1 && kind == 1) {  // a panel before the group's last updates the next panel only
                    st.r1 = (int32_t)syr.size() / 4;
                    continue;
                }
                for (int q = C->lvl_ptr[l]; q < C->lvl_ptr[l + 1]; q++) {
                    int s = C->lvl_sn[q];
                    int m = C->h_mrows[s], nn = C->h_ncol[s];
                    int k0 = k * TB;
                    if (m <= TB || C->is_dense[s] || k0 >= nn) continue;
                    int base = k0 + std::min(TB, nn - k0);
                    int c0 = pass == 0 ? base : base + TB;
                    int c1 = pass == 0 ? std::min(base + TB, m) : m;
                    int cw = pass == 0 ? TB : ST;
                    for (int rj0 = c0; rj0 < c1; rj0 += cw)
                        for (int ri0 = rj0; ri0 < m; ri0 += ST) {
                            syr.push_back(s);
                            syr.push_back(kfirst);
                            syr.push_back(ri0);
                            syr.push_back(rj0);
                            // the next panel's diagonal tile factors that panel's diagonal block; its slot is
                            // the front's position among the fronts with a panel at the next step
                            int ns2 = -1;
                            if (pass == 0 && ri0 == base && base < nn) {
                                ns2 = 0;
                                for (int q2 = C->lvl_ptr[l]; q2 < q; q2++) {
                                    int s2 = C->lvl_sn[q2];
                                    if (C->h_mrows[s2] > TB && !C->is_dense[s2] && (k + 1) * TB < C->h_ncol[s2]) ns2++;
                                }
                            }
                            nslot.push_back(ns2);
                        }
                }
                if (pass == 0)
                    st.s1 = (int32_t)syr.size() / 4;
                else
                    st.r1 = (int32_t)syr.size() / 4;
            }
            double fl = 0, by = 0;
            for (int q = C->lvl_ptr[l]; q < C->lvl_ptr[l + 1]; q++) {
                int s = C->lvl_sn[q];
                int m = C->h_mrows[s], nn = C->h_ncol[s];
                if (m <= TB || C->is_dense[s] || k * TB >= nn) continue;
                const double base = k * TB + std::min(TB, nn - k * TB), r = m - base;
                if (kind == 1) {
                    // rank-kw update of the next panel's columns below the diagonal (kw = the group's panels so far)
                    const double w = std::min<double>(TB, r);
                    const double ent = w * r - w * (w - 1) / 2;
                    fl += 2.0 * st.kw * ent;
                    by += 16.0 * ent + 8.0 * st.kw * (r + w);
                } else {
                    const double kw = kind == 2 ? st.kw : std::min(TB, nn - k * TB);
                    fl += r * (r + 1) * kw;  // symmetric rank-kw update of an r x r lower triangle
                    // every lower entry of the r x r block read and written once (16 B); the panel rows read
                    // once by the next-panel tiles and once by the tiles after them
                    const double rest = std::max(0.0, r - TB);
                    by += 16.0 * r * (r + 1) / 2 + 8.0 * kw * (r + rest);
                }
            }
            C->step_syrk_flops.push_back(fl);
            C->step_syrk_bytes.push_back(by);
            C->steps.push_back(st);
        }
        C->lvl_step_ptr[l + 1] = (int32_t)C->steps.size();
    }
    // upload
    C->dev.upload(C->first, C->h_first);
    C->dev.upload(C->ncol, C->h_ncol);
    C->dev.upload(C->mrows, C->h_mrows);
    C->dev.upload(C->perm, S.perm);
    {
        std::vector<int32_t> kdp(n);
        for (int j = 0; j < n; j++) kdp[j] = colptr[S.perm[j]];  // rows ascending: the diagonal comes first
        C->dev.upload(C->kdiagpos, kdp);
    }
    C->dev.upload(C->foff, C->h_foff);
    C->dev.upload(C->roff, C->h_roff);
    C->dev.upload(C->uoff, C->h_uoff);
    C->dev.upload(C->rows, S.rows_flat);
    C->dev.upload(C->child_ptr, cptr);
    C->dev.upload(C->child, clist);
    C->dev.upload(C->rel_off, reloff);
    C->dev.upload(C->rel, rel);
    {
        // extend-add of the solves in gather form: every front row lists the update entries that land on it
        const int64_t nrows = C->h_roff[ns];
        std::vector<int64_t> gp(nrows + 1, 0), gs;
        for (int sn = 0; sn < ns; sn++)
            for (int ci = cptr[sn]; ci < cptr[sn + 1]; ci++) {
                const int c = clist[ci];
                const int nu = C->h_mrows[c] - C->h_ncol[c];
                for (int t = 0; t < nu; t++) gp[C->h_roff[sn] + rel[reloff[c] + t] + 1]++;
            }
        for (int64_t r = 0; r < nrows; r++) gp[r + 1] += gp[r];
        gs.resize(gp[nrows]);
        std::vector<int64_t> fill(gp.begin(), gp.end() - 1);
        for (int sn = 0; sn < ns; sn++)
            for (int ci = cptr[sn]; ci < cptr[sn + 1]; ci++) {
                const int c = clist[ci];
                const int nu = C->h_mrows[c] - C->h_ncol[c];
                for (int t = 0; t < nu; t++) gs[fill[C->h_roff[sn] + rel[reloff[c] + t]]++] = C->h_uoff[c] + t;
            }
        C->dev.upload(C->gptr, gp);
        C->dev.upload(C->gsrc, gs.empty() ? std::vector<int64_t>(1, 0) : gs);
    }
    C->dev.upload(C->tile_sn, tsn);
    C->dev.upload(C->tile_cptr, tcptr);
    C->dev.upload(C->tile_crec, tcrec);
    C->dev.upload(C->tile_rc, trc);
    C->dev.upload(C->tile_kptr, tkptr);
    C->dev.upload(C->tile_k, tk);
    C->dev.upload(C->tile_kpos, tkpos);
    C->dev.upload(C->lvl_sn_d, C->lvl_sn);
    C->dev.upload(C->lvl_small_d, C->lvl_small);
    C->dev.upload(C->lvl_narrow_d, C->lvl_narrow);
    C->dev.upload(C->trow_d, C->trow_it.empty() ? std::vector<int32_t>(2, 0) : C->trow_it);
    C->dev.upload(C->tcol_d, C->tcol_it.empty() ? std::vector<int32_t>(2, 0) : C->tcol_it);
    C->dev.upload(C->lvl_wide_d, C->lvl_wide);
    C->dev.upload(C->potrf_it, pot);
    C->dev.upload(C->trsm_it, trs);
    C->dev.upload(C->syrk_it, syr);
    C->dev.upload(C->next_slot, nslot);
    C->dev.alloc(C->status, std::max(ns, 1));
    C->dev.alloc(C->fronts, std::max<int64_t>(fo, 1));
    C->dev.alloc(C->upd, std::max<int64_t>(uo, 1));
    C->dev.alloc(C->work, std::max<int64_t>(C->h_roff[ns], 1));
    C->dev.alloc(C->ybuf, std::max(n, 1));
    C->dev.alloc(C->ldiag, (int64_t)std::max(max_slots, 1) * TB * TB);
    C->dev.alloc(C->rdiag, (int64_t)std::max(max_slots, 1) * TB);
    C->h_flag_off.assign(ns, -1);
    int64_t nflags = 0;
    for (int s = 0; s < ns; s++)
        if (C->h_ncol[s] >= WIDE) {
            C->h_flag_off[s] = nflags;
            nflags += (C->h_ncol[s] + SB - 1) / SB;
        }
    C->dev.alloc(C->zx, std::max<int64_t>(nflags, 1) * SB);
    // the wide fronts' diagonal-block inverses, refreshed by every factorization for the sweeps
    std::vector<int32_t> wit;
    for (int s = 0; s < ns; s++)
        if (C->h_flag_off[s] >= 0)
            for (int g = 0; g < (C->h_ncol[s] + SB - 1) / SB; g++) {
                wit.push_back(s);
                wit.push_back(g);
                wit.push_back((int32_t)(C->h_flag_off[s] + g));
            }
    C->nwinv = (int)wit.size() / 3;
    C->dev.alloc(C->winv, std::max<int64_t>(nflags, 1) * SB * SB);
    C->dev.upload(C->winv_it, wit.empty() ? std::vector<int32_t>(3, 0) : wit);
    C->dev.upload(C->sfault, std::vector<int32_t>(1, 0));
    C->dev.upload(C->level_d, C->h_level);
    C->dev.alloc(C->statwords, 2);
    C->dev.alloc(C->dval, C->opts.ldlt ? std::max(n, 1) : 1);
}

extern "C" void chol_default_options(chol_options* o) {
    o->dense_frac = 0.5;
    o->dense_abs = INT32_MAX;
    o->max_width = INT32_MAX;
    o->zero_abs = 64;
    o->zero_rel = 0.05;
    o->pivot_tol = 0.0;
    o->tile_min = 0;
    o->pair_min = 2048;
    o->pair_panels = 2;
    o->ldlt = 0;
}

extern "C" int chol_analyze(int32_t n, const int32_t* colptr, const int32_t* rowind, const chol_options* opts,
                            chol_sym** out) {
    return guarded([&] {
        OPF_CHECK(out && colptr && rowind && n >= 1, OPF_E_INVALID, "chol_analyze: bad argument");
        *out = nullptr;
        std::vector<int32_t> cp(colptr, colptr + n + 1);
        OPF_CHECK(cp[0] == 0, OPF_E_INVALID, "chol_analyze: colptr[0] must be 0");
        for (int j = 0; j < n; j++) OPF_CHECK(cp[j + 1] >= cp[j], OPF_E_INVALID, "chol_analyze: colptr not monotone");
        std::vector<int32_t> ri(rowind, rowind + cp[n]);
        for (int j = 0; j < n; j++) {
            bool diag = false;
            for (int p = cp[j]; p < cp[j + 1]; p++) {
                OPF_CHECK(ri[p] >= j && ri[p] < n, OPF_E_INVALID, "chol_analyze: entry (%d,%d) not in the lower triangle",
                          ri[p], j);
                OPF_CHECK(p == cp[j] || ri[p] > ri[p - 1], OPF_E_INVALID, "chol_analyze: rows not strictly ascending");
                diag |= ri[p] == j;
            }
            OPF_CHECK(diag, OPF_E_INVALID, "chol_analyze: column %d has no diagonal entry", j);
        }
        chol_options o;
        chol_default_options(&o);
        if (opts) o = *opts;
        OPF_CHECK(o.ldlt == 0 || o.ldlt == 1, OPF_E_INVALID, "chol_analyze: ldlt must be 0 or 1");
        OPF_CHECK(!(o.ldlt && o.tile_min > 0), OPF_E_INVALID,
                  "chol_analyze: the dependency-driven tile path (tile_min > 0) factors by Cholesky only");
        auto* C = new chol_sym();
        try {
            C->opts = o;
            C->n = n;
            C->nnzk = cp[n];
            C->S = analyze_pattern(n, cp, ri, o);
            build_numeric_plan(C, cp, ri);
        } catch (...) {
            delete C;
            throw;
        }
        *out = C;
    });
}

extern "C" int chol_destroy(chol_sym* C) {
    delete C;
    return OPF_OK;
}

extern "C" int chol_info(const chol_sym* C, int32_t* nsuper, int64_t* nnz_l, double* flops, int64_t* factor_bytes) {
    return guarded([&] {
        OPF_CHECK(C, OPF_E_INVALID, "chol_info: null handle");
        if (nsuper) *nsuper = C->S.nsuper;
        if (nnz_l) *nnz_l = C->nnzl;
        if (flops) *flops = C->flops;
        if (factor_bytes) *factor_bytes = C->front_total * 8;
    });
}

extern "C" int chol_perm(const chol_sym* C, int32_t* perm) {
    return guarded([&] {
        OPF_CHECK(C && perm, OPF_E_INVALID, "chol_perm: null argument");
        memcpy(perm, C->S.perm.data(), C->S.perm.size() * 4);
    });
}

extern "C" int chol_etree(const chol_sym* C, int32_t* parent, int32_t* colcount) {
    return guarded([&] {
        OPF_CHECK(C, OPF_E_INVALID, "chol_etree: null handle");
        if (parent) memcpy(parent, C->S.parent.data(), C->S.parent.size() * 4);
        if (colcount) memcpy(colcount, C->S.colcount.data(), C->S.colcount.size() * 4);
    });
}

extern "C" int chol_supernodes(const chol_sym* C, int32_t* snode_ptr) {
    return guarded([&] {
        OPF_CHECK(C && snode_ptr, OPF_E_INVALID, "chol_supernodes: null argument");
        memcpy(snode_ptr, C->S.snode_ptr.data(), C->S.snode_ptr.size() * 4);
    });
}

extern "C" int chol_supernode_rows(const chol_sym* C, int64_t* rows_ptr, int32_t* rows) {
    return guarded([&] {
        OPF_CHECK(C, OPF_E_INVALID, "chol_supernode_rows: null handle");
        if (rows_ptr) memcpy(rows_ptr, C->S.rows_ptr.data(), C->S.rows_ptr.size() * 8);
        if (rows) memcpy(rows, C->S.rows_flat.data(), C->S.rows_flat.size() * 4);
    });
}

namespace opf {

// Enqueue the numeric factorization (no synchronisation).
static void tmark(chol_sym* C, hipStream_t st, int cat) {
    if (!(C->timing & (1 << cat))) return;
    if (C->ev_used == C->ev_pool.size()) {
        hipEvent_t e;
        OPF_HIP(hipEventCreate(&e));
        C->ev_pool.push_back(e);
        C->ev_cat.push_back(0);
    }
    C->ev_cat[C->ev_used] = cat;
    OPF_HIP(hipEventRecord(C->ev_pool[C->ev_used++], st));
}

// After a synchronisation: fold the recorded (start, end) event pairs into the per-category totals.
static void tcollect(chol_sym* C) {
    if (!C->timing) return;
    for (size_t i = 0; i + 1 < C->ev_used; i += 2) {
        float ms = 0;
        OPF_HIP(hipEventElapsedTime(&ms, C->ev_pool[i], C->ev_pool[i + 1]));
        C->t_ms[C->ev_cat[i]] += ms;
        C->t_launch[C->ev_cat[i]]++;
    }
    C->ev_used = 0;
}

__global__ void reset_words(int32_t* a, int32_t* b) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (a) *a = 0;
        if (b) *b = 0;
    }
}

static int dense_grid(chol_sym* C) {
    if (!C->dense_grid) {
        int dev = 0, cus = 0;
        OPF_HIP(hipGetDevice(&dev));
        OPF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        C->dense_grid = 2 * std::max(cus, 1);  // two work-groups per compute unit (LDS-limited)
    }
    return C->dense_grid;
}

// Run `enqueue` on st, through a captured graph when graphs are enabled: the first call with a key captures
// the launch sequence (stream capture, thread-local mode) and instantiates it, later calls replay it with one
// graph launch.  Every captured node is a kernel (no memset or copy nodes); timing mode and the dependency-
// driven tile path (whose launch carries a per-factorization epoch) run uncaptured.
static std::atomic<int64_t> g_graph_captures{0}, g_graph_fallbacks{0};

template <class F>
static void run_graph(chol_sym* C, hipStream_t st, const void* a, const void* b, double tol, F&& enqueue) {
    const bool tiles = !C->lvl_dense_ptr.empty() && C->lvl_dense_ptr.back() > 0;
    if (!C->use_graphs || !st || C->timing || tiles) {
        enqueue();
        return;
    }
    for (auto& g : C->graphs)
        if (g.st == st && g.a == a && g.b == b && g.tol == tol) {
            OPF_HIP(hipGraphLaunch(g.exec, st));
            return;
        }
    g_graph_captures.fetch_add(1, std::memory_order_relaxed);
    // A capture that fails (another thread's work can invalidate it) is abandoned and the sequence is
    // enqueued directly instead: the graph only saves launch overhead.  Captured work never runs, so the
    // direct enqueue is the only execution.
    auto abandon = [&] {
        g_graph_fallbacks.fetch_add(1, std::memory_order_relaxed);
        hipGraph_t bad = nullptr;
        (void)hipStreamEndCapture(st, &bad);
        if (bad) (void)hipGraphDestroy(bad);
        (void)hipGetLastError();  // clear the thread's error state for the launches that follow
    };
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        abandon();
        enqueue();
        return;
    }
    try {
        enqueue();
    } catch (...) {
        abandon();
        enqueue();  // an error that is not the capture's comes back from the direct enqueue
        return;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(st, &graph) != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        abandon();
        enqueue();
        return;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g_graph_fallbacks.fetch_add(1, std::memory_order_relaxed);
        (void)hipGetLastError();
        enqueue();
        return;
    }
    if (C->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(C->graphs.front().exec);
        C->graphs.erase(C->graphs.begin());
    }
    C->graphs.push_back({st, a, b, tol, exec});
    OPF_HIP(hipGraphLaunch(exec, st));
}

void chol_factor_enqueue(chol_sym* C, const double* kval, hipStream_t st, double pivot_tol) {
    chol_set_stream(C, st);  // first use: the uploads go on the caller's stream
    C->dev.run();
    const PivotRef pr{kval, C->kdiagpos.p, pivot_tol};
    const bool ldl = C->opts.ldlt != 0;
    C->epoch++;
    hipLaunchKernelGGL(reset_words, dim3(1), dim3(64), 0, st, C->ffault.p, (int32_t*)nullptr);
    OPF_LAUNCH_CHECK();
    const DenseDesc DD{C->dh_s.p,   C->dh_np.p,    C->dh_nb.p, C->dh_t0.p,    C->dh_slot0.p, C->dtask_h.p,
                       C->dtask_rc.p, C->dflags.p, C->dcounter.p, C->ffault.p, C->tdiag.p,    C->trdiag.p};
    for (int l = 0; l < C->nlevels; l++) {
        int t0 = C->asm_ptr[l], t1 = C->asm_ptr[l + 1];
        if (t1 > t0) {
            tmark(C, st, 0);
            const int lda = C->lvl_small_maxm[l];
            if (lda > 0) {  // only fronts of at most 64 rows: one wave each, as many per work-group as 64 KB holds
                const size_t per_front = (size_t)lda * lda * sizeof(double) + 64 * sizeof(int64_t);
                const int per = std::max(1, std::min(NT / 64, (int)(65536 / per_front)));
                hipLaunchKernelGGL(front_assemble_tiny, dim3(ceil_div(t1 - t0, per)), dim3(64 * per), per * per_front,
                                   st, t0, t1 - t0, lda, C->tile_sn.p, C->tile_kptr.p, C->tile_k.p, C->tile_kpos.p,
                                   kval, C->ncol.p, C->mrows.p, C->foff.p, C->tile_cptr.p, C->tile_crec.p,
                                   C->rel_off.p, C->rel.p, C->fronts.p);
            } else {
                hipLaunchKernelGGL(front_assemble, dim3(t1 - t0), dim3(NT), 0, st, t0, C->tile_sn.p, C->tile_rc.p,
                                   C->tile_kptr.p, C->tile_k.p, C->tile_kpos.p, kval, C->ncol.p, C->mrows.p,
                                   C->foff.p, C->tile_cptr.p, C->tile_crec.p, C->rel_off.p, C->rel.p, C->fronts.p);
            }
            OPF_LAUNCH_CHECK();
            tmark(C, st, 0);
        }
        int s0 = C->lvl_small_ptr[l], s1 = C->lvl_small_ptr[l + 1];
        if (s1 > s0) {
            tmark(C, st, 1);
            const int lda = C->lvl_small_lda[l];
            hipLaunchKernelGGL(ldl ? front_small<true> : front_small<false>, dim3(s1 - s0), dim3(NT),
                               (size_t)lda * lda * sizeof(double), st, C->lvl_small_d.p + s0, C->first.p, C->ncol.p,
                               C->mrows.p, C->foff.p, C->fronts.p, C->status.p, pr, C->dval.p, lda);
            OPF_LAUNCH_CHECK();
            tmark(C, st, 1);
        }
        const int d0 = C->lvl_dense_ptr[l], d1 = C->lvl_dense_ptr[l + 1];
        if (d1 > d0) {
            hipLaunchKernelGGL(reset_words, dim3(1), dim3(64), 0, st, C->dcounter.p, (int32_t*)nullptr);
            OPF_LAUNCH_CHECK();
            tmark(C, st, 5);
            hipLaunchKernelGGL(dense_front, dim3(std::min(d1 - d0, dense_grid(C))), dim3(NT), 0, st, (int64_t)d0,
                               (int64_t)d1, DD, C->epoch, C->first.p, C->ncol.p, C->mrows.p, C->foff.p, C->fronts.p,
                               C->status.p, pr);
            OPF_LAUNCH_CHECK();
            tmark(C, st, 5);
            if (C->timing & (1 << 5)) C->t_flops[5] += C->lvl_dense_flops[l];
        }
        const int q0 = C->lvl_step_ptr[l], q1 = C->lvl_step_ptr[l + 1];
        for (int q = q0; q < q1; q++) {
            const chol_sym::Step& S = C->steps[q];
            if (q == q0 && S.p1 > S.p0) {  // later steps factor their diagonal blocks in the update before
                tmark(C, st, 2);
                hipLaunchKernelGGL(ldl ? blk_potrf<true> : blk_potrf<false>, dim3(S.p1 - S.p0), dim3(NT), 0, st,
                                   C->potrf_it.p + 2 * S.p0, C->first.p, C->ncol.p, C->mrows.p, C->foff.p,
                                   C->fronts.p, C->ldiag.p, C->rdiag.p, C->status.p, pr, C->dval.p);
                OPF_LAUNCH_CHECK();
                tmark(C, st, 2);
            }
            if (S.t1 > S.t0) {
                tmark(C, st, 3);
                hipLaunchKernelGGL(ldl ? blk_trsm_mma<true> : blk_trsm_mma<false>, dim3(S.t1 - S.t0), dim3(NT), 0, st,
                                   C->trsm_it.p + 4 * S.t0, C->ncol.p, C->mrows.p, C->foff.p, C->ldiag.p, C->rdiag.p,
                                   C->fronts.p);
                OPF_LAUNCH_CHECK();
                tmark(C, st, 3);
            }
            if (S.r1 > S.s0) {
                tmark(C, st, 4);
                hipLaunchKernelGGL(ldl ? blk_syrk<true> : blk_syrk<false>, dim3(S.r1 - S.s0), dim3(NT), 0, st,
                                   C->syrk_it.p + 4 * S.s0, S.r1 - S.s0, S.s1 - S.s0, S.kw, C->ncol.p, C->mrows.p,
                                   C->foff.p, C->fronts.p, C->next_slot.p + S.s0, C->first.p, C->ldiag.p, C->rdiag.p,
                                   C->status.p, pr, C->dval.p);
                OPF_LAUNCH_CHECK();
                tmark(C, st, 4);
            }
            if (C->timing & (1 << 4)) {
                C->t_flops[4] += C->step_syrk_flops[q];
                C->t_bytes[4] += C->step_syrk_bytes[q];
            }
        }
    }
    if (C->nwinv > 0) {  // diagonal-block inverses of the wide fronts for the sweeps
        hipLaunchKernelGGL(wide_inverse, dim3(C->nwinv), dim3(64), 0, st, C->winv_it.p, C->ncol.p, C->mrows.p,
                           C->foff.p, C->fronts.p, C->winv.p, (int)ldl);
        OPF_LAUNCH_CHECK();
    }
    if (ldl) {
        hipLaunchKernelGGL(count_negative, dim3(1), dim3(CNT_NT), 0, st, C->n, C->dval.p, C->statwords.p + 1);
        OPF_LAUNCH_CHECK();
    }
}

__global__ void init_status(int ns, const int32_t* __restrict__ mrows, int32_t* __restrict__ status) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < ns && mrows[s] > TB) status[s] = INT_MAX;
}

// The reported pivot: the smallest (level, pivot) over the supernodes' first rejected pivots (an order-free
// minimum, so the result does not depend on the schedule), one work-group.
constexpr int SMIN_NT = 1024;
__global__ __launch_bounds__(SMIN_NT) void status_min(int ns, const int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ level, int64_t* __restrict__ out) {
    __shared__ int64_t red[SMIN_NT / 64];
    int64_t v = INT64_MAX;
    for (int s = threadIdx.x; s < ns; s += SMIN_NT)
        if (status[s] != INT_MAX) v = min(v, ((int64_t)level[s] << 32) | (uint32_t)status[s]);
    for (int o = 32; o > 0; o >>= 1) v = min(v, (int64_t)__shfl_xor((long long)v, o));
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < SMIN_NT / 64; w++) v = min(v, red[w]);
        out[0] = v;
    }
}

static int64_t* host_words(chol_sym* C) {
    if (!C->hwords) {
        OPF_HIP(hipHostMalloc((void**)&C->hwords, 4 * sizeof(int64_t)));
        C->own_hwords = true;
    }
    return C->hwords;
}

// Factor and report: returns -1 if positive definite, else the bad pivot.
int chol_factor_sync(chol_sym* C, const double* kval, hipStream_t st, double pivot_tol) {
    chol_set_stream(C, st);  // first use: the uploads go on the caller's stream
    C->dev.run();
    const int ns = C->S.nsuper;
    run_graph(C, st, kval, nullptr, pivot_tol, [&] {
        hipLaunchKernelGGL(init_status, dim3(ceil_div(ns, 256)), dim3(256), 0, st, ns, C->mrows.p, C->status.p);
        OPF_LAUNCH_CHECK();
        chol_factor_enqueue(C, kval, st, pivot_tol);
        hipLaunchKernelGGL(status_min, dim3(1), dim3(SMIN_NT), 0, st, ns, C->status.p, C->level_d.p, C->statwords.p);
        OPF_LAUNCH_CHECK();
    });
    int64_t* hw = host_words(C);
    hw[1] = 0;  // the fault word fills its low half
    OPF_HIP(hipMemcpyAsync(hw, C->statwords.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    OPF_HIP(hipMemcpyAsync(hw + 1, C->ffault.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (C->opts.ldlt) OPF_HIP(hipMemcpyAsync(hw + 3, C->statwords.p + 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    OPF_HIP(hipStreamSynchronize(st));
    C->last_nneg = C->opts.ldlt ? hw[3] : 0;
    tcollect(C);
    const int64_t key = hw[0];
    const int32_t ffault = (int32_t)hw[1];
    OPF_CHECK(ffault == 0, OPF_E_DEVICE, "chol_factor: a dense-front tile wait exceeded its bound");
    const int bad = key == INT64_MAX ? -1 : (int)(key & 0xffffffff);
    C->factored = bad < 0;
    return bad;
}

// Device buffers a solve writes besides its output: the permuted working vector y [n], the per-row
// partial results work [roff[ns]], the update vectors passed to parents upd [upd_total], the exchange
// blocks of the wide-front sweeps zx [nflags * SB] and the fault word.
struct SolveBufs {
    double *y, *work, *upd, *zx;
    int32_t* fault;
};

static SolveBufs handle_bufs(chol_sym* C) { return {C->ybuf.p, C->work.p, C->upd.p, C->zx.p, C->sfault.p}; }

static void solve_enqueue(chol_sym* C, const double* b, double* x, hipStream_t st, const SolveBufs& B) {
    const int n = C->n;
    double* y = B.y;
    hipLaunchKernelGGL(permute_in, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, C->perm.p, b, y);
    OPF_LAUNCH_CHECK();
    for (int l = 0; l < C->nlevels; l++) {
        int q0 = C->lvl_narrow_ptr[l], q1 = C->lvl_narrow_ptr[l + 1];
        if (q1 > q0) {
            if (C->lvl_narrow_maxm[l] <= TB) {  // only fronts of at most 64 rows: four to a work-group
                hipLaunchKernelGGL(solve_fwd_tiny, dim3(ceil_div(q1 - q0, NT / 64)), dim3(NT), 0, st, q1 - q0,
                                   C->lvl_narrow_d.p + q0, C->first.p, C->ncol.p, C->mrows.p, C->foff.p, C->roff.p,
                                   C->uoff.p, C->gptr.p, C->gsrc.p, C->fronts.p, B.upd, y, C->opts.ldlt);
            } else {
                const int wcap = std::min(C->lvl_narrow_maxm[l], WLDS);  // fronts up to wcap rows keep w in LDS
                hipLaunchKernelGGL(solve_fwd, dim3(q1 - q0), dim3(NT), (size_t)wcap * sizeof(double), st,
                                   C->lvl_narrow_d.p + q0, C->first.p, C->ncol.p, C->mrows.p, C->foff.p, C->roff.p,
                                   C->uoff.p, C->gptr.p, C->gsrc.p, C->fronts.p, B.work, B.upd, y, wcap,
                                   C->opts.ldlt);
            }
            OPF_LAUNCH_CHECK();
            const int t0 = C->lvl_trow_ptr[l], t1 = C->lvl_trow_ptr[l + 1];
            if (t1 > t0) {  // the tall fronts' rows below their pivots
                hipLaunchKernelGGL(solve_fwd_rows, dim3(t1 - t0), dim3(NT), 0, st, C->trow_d.p + 2 * t0, C->first.p,
                                   C->ncol.p, C->mrows.p, C->foff.p, C->roff.p, C->uoff.p, C->gptr.p, C->gsrc.p,
                                   C->fronts.p, B.upd, y);
                OPF_LAUNCH_CHECK();
            }
        }
        int w0 = C->lvl_wide_ptr[l], w1 = C->lvl_wide_ptr[l + 1];
        if (w1 > w0) {
            for (int q = w0; q < w1; q++) {
                const int s = C->lvl_wide[q];
                const int m = C->h_mrows[s], nn = C->h_ncol[s];
                hipLaunchKernelGGL(sfwd_gather, dim3(ceil_div(m, NT)), dim3(NT), 0, st, s, C->first.p, C->ncol.p,
                                   C->mrows.p, C->roff.p, C->gptr.p, C->gsrc.p, B.work, B.upd, y);
                OPF_LAUNCH_CHECK();
                const int g = (nn + SB - 1) / SB + (m - nn + SB - 1) / SB;
                double* zx = B.zx + C->h_flag_off[s] * SB;
                const int64_t nz = (int64_t)((nn + SB - 1) / SB) * SB;
                hipLaunchKernelGGL(fill_sentinel, dim3(ceil_div(nz, 256)), dim3(256), 0, st, nz, zx);
                OPF_LAUNCH_CHECK();
                hipLaunchKernelGGL(wide_fwd, dim3(g), dim3(NT), 0, st, s, zx, B.fault, C->first.p, C->ncol.p,
                                   C->mrows.p, C->foff.p, C->roff.p, C->uoff.p, C->fronts.p, B.work, B.upd, y,
                                   C->winv.p + C->h_flag_off[s] * SB * SB);
                OPF_LAUNCH_CHECK();
            }
        }
    }
    if (C->opts.ldlt) {  // L D L^T: the forward sweeps solved with the unit triangle; now D
        hipLaunchKernelGGL(dscale, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, C->dval.p, y);
        OPF_LAUNCH_CHECK();
    }
    for (int l = C->nlevels - 1; l >= 0; l--) {
        int w0 = C->lvl_wide_ptr[l], w1 = C->lvl_wide_ptr[l + 1];
        for (int q = w0; q < w1; q++) {
            const int s = C->lvl_wide[q];
            const int nn = C->h_ncol[s];
            double* zx = B.zx + C->h_flag_off[s] * SB;
            const int64_t nz = (int64_t)((nn + SB - 1) / SB) * SB;
            hipLaunchKernelGGL(fill_sentinel, dim3(ceil_div(nz, 256)), dim3(256), 0, st, nz, zx);
            OPF_LAUNCH_CHECK();
            hipLaunchKernelGGL(wide_bwd, dim3((nn + SB - 1) / SB), dim3(NT), 0, st, s, zx, B.fault, C->first.p,
                               C->ncol.p, C->mrows.p, C->foff.p, C->roff.p, C->rows.p, C->fronts.p, y,
                               C->winv.p + C->h_flag_off[s] * SB * SB);
            OPF_LAUNCH_CHECK();
        }
        int q0 = C->lvl_narrow_ptr[l], q1 = C->lvl_narrow_ptr[l + 1];
        const int c0 = C->lvl_tcol_ptr[l], c1 = C->lvl_tcol_ptr[l + 1];
        if (c1 > c0) {  // the tall fronts' products with their rows below
            hipLaunchKernelGGL(solve_bwd_dots, dim3(c1 - c0), dim3(NT), 0, st, C->tcol_d.p + 2 * c0, C->first.p,
                               C->ncol.p, C->mrows.p, C->foff.p, C->roff.p, C->rows.p, C->fronts.p, B.work, y);
            OPF_LAUNCH_CHECK();
        }
        if (q1 > q0) {
            if (C->lvl_narrow_maxm[l] <= TB)
                hipLaunchKernelGGL(solve_bwd_tiny, dim3(ceil_div(q1 - q0, NT / 64)), dim3(NT), 0, st, q1 - q0,
                                   C->lvl_narrow_d.p + q0, C->first.p, C->ncol.p, C->mrows.p, C->foff.p, C->roff.p,
                                   C->rows.p, C->fronts.p, y, C->opts.ldlt);
            else
                hipLaunchKernelGGL(solve_bwd, dim3(q1 - q0), dim3(NT), 0, st, C->lvl_narrow_d.p + q0, C->first.p,
                                   C->ncol.p, C->mrows.p, C->foff.p, C->roff.p, C->rows.p, C->fronts.p, B.work, y,
                                   C->opts.ldlt);
            OPF_LAUNCH_CHECK();
        }
    }
    hipLaunchKernelGGL(permute_out, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, C->perm.p, y, x);
    OPF_LAUNCH_CHECK();
}

void chol_solve_enqueue(chol_sym* C, const double* b, double* x, hipStream_t st) {
    chol_set_stream(C, st);  // first use: the uploads go on the caller's stream
    C->dev.run();
    run_graph(C, st, b, x, -1.0, [&] { solve_enqueue(C, b, x, st, handle_bufs(C)); });
}

void chol_use_graphs(chol_sym* C, bool on) { C->use_graphs = on; }

// Raised by a sync-free solve whose wait exceeded its bound (the solve result is invalid).
// The analysis's device buffers and uploads, normally performed at the first factorization, done now.
void chol_prepare_device(chol_sym* C) { C->dev.run(); }

// The fault word of the last sweeps (0 when no front took the sync-free solves), read through the pinned
// host words when the handle has them (the allocation-free solve must not allocate them).
static int read_fault(const chol_sym* C, const int32_t* fault, hipStream_t st) {
    if (C->h_flag_off.empty()) return 0;
    if (C->hwords) {
        C->hwords[2] = 0;
        OPF_HIP(hipMemcpyAsync(C->hwords + 2, fault, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        OPF_HIP(hipStreamSynchronize(st));
        return (int32_t)C->hwords[2];
    }
    int32_t v = 0;
    OPF_HIP(hipMemcpyAsync(&v, fault, sizeof v, hipMemcpyDeviceToHost, st));
    OPF_HIP(hipStreamSynchronize(st));
    return v;
}

int chol_solve_fault(chol_sym* C, hipStream_t st) { return read_fault(C, C->sfault.p, st); }

// Negative pivots of the last factorization (0 for Cholesky).
int64_t chol_last_negative(const chol_sym* C) { return C->last_nneg; }

// Pending device uploads of the analysis run on st (when they have not run yet).
void chol_set_stream(chol_sym* C, hipStream_t st) {
    if (!C->dev.done) C->dev.stream = st;
}

// Lends the factorization 4 int64 words of pinned host memory (owned by the caller, who outlives C).
void chol_bind_host(chol_sym* C, int64_t* words) {
    if (C->own_hwords && C->hwords) (void)hipHostFree(C->hwords);
    C->hwords = words;
    C->own_hwords = false;
}

__global__ void fill_i32(int n, int32_t v, int32_t* __restrict__ p) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace opf

extern "C" int chol_graph_stats(int64_t* captures, int64_t* fallbacks) {
    return guarded([&] {
        OPF_CHECK(captures && fallbacks, OPF_E_INVALID, "chol_graph_stats: null argument");
        *captures = g_graph_captures.load();
        *fallbacks = g_graph_fallbacks.load();
    });
}

extern "C" int chol_factor(chol_sym* C, const double* kval, void* stream, int32_t* bad_col) {
    return guarded([&] {
        OPF_CHECK(C && kval, OPF_E_INVALID, "chol_factor: null argument");
        int bad = chol_factor_sync(C, kval, (hipStream_t)stream, C->opts.pivot_tol);
        if (bad_col) *bad_col = bad;
        if (bad >= 0) {
            set_error(C->opts.ldlt ? "chol_factor: zero (or below tolerance) pivot at pivot index %d"
                                   : "chol_factor: non-positive pivot at pivot index %d",
                      bad);
            throw Error{OPF_E_NOT_PD};
        }
    });
}

extern "C" int chol_inertia(const chol_sym* C, int64_t* npos, int64_t* nneg) {
    return guarded([&] {
        OPF_CHECK(C && npos && nneg, OPF_E_INVALID, "chol_inertia: null argument");
        OPF_CHECK(C->factored, OPF_E_STATE, "chol_inertia: no successful factorization");
        *nneg = C->last_nneg;
        *npos = C->n - C->last_nneg;
    });
}

extern "C" int chol_solve(chol_sym* C, const double* b, double* x, int32_t nrhs, void* stream) {
    return guarded([&] {
        OPF_CHECK(C && b && x && nrhs >= 0, OPF_E_INVALID, "chol_solve: bad argument");
        OPF_CHECK(C->factored, OPF_E_STATE, "chol_solve: no successful factorization");
        for (int r = 0; r < nrhs; r++)
            chol_solve_enqueue(C, b + (int64_t)r * C->n, x + (int64_t)r * C->n, (hipStream_t)stream);
        OPF_CHECK(chol_solve_fault(C, (hipStream_t)stream) == 0, OPF_E_DEVICE,
                  "chol_solve: a wide-front block wait exceeded its bound");
    });
}

// ---------------------------------------------------------------- allocation-free solve
// Scratch of chol_solve_noalloc: one static device array per GPU, resolved to a device address once per
// device with hipGetSymbolAddress (the array's name is only a host-side stand-in).  Layout, each part
// 256-byte aligned: fault word, y [n], work [row-structure entries], upd [update rows], zx [wide blocks].
static constexpr size_t SOLVE_SCRATCH_BYTES = size_t(64) << 20;
static constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[SOLVE_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES] = {};

static void* scratch_address() {
    int dev = -1;
    OPF_HIP(hipGetDevice(&dev));
    OPF_CHECK(dev >= 0 && dev < MAX_DEVICES, OPF_E_DEVICE, "chol_solve_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        OPF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        OPF_CHECK(p != nullptr, OPF_E_DEVICE, "chol_solve_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

extern "C" int chol_solve_noalloc(chol_sym* C, const double* b, double* x, int32_t nrhs, void* stream) {
    return guarded([&] {
        OPF_CHECK(C && b && x && nrhs >= 0, OPF_E_INVALID, "chol_solve_noalloc: bad argument");
        const int ns = C->S.nsuper;
        int64_t nflags = 0;
        for (int s = 0; s < ns; s++)
            if (C->h_flag_off[s] >= 0) nflags += (C->h_ncol[s] + SB - 1) / SB;
        const size_t o_y = 256;
        const size_t o_work = o_y + align256((size_t)C->n * 8);
        const size_t o_upd = o_work + align256((size_t)C->h_roff[ns] * 8);
        const size_t o_zx = o_upd + align256((size_t)C->upd_total * 8);
        const size_t need = o_zx + align256((size_t)nflags * SB * 8);
        OPF_CHECK(need <= SOLVE_SCRATCH_BYTES, OPF_E_INVALID,
                  "chol_solve_noalloc: this factor needs %zu bytes of solve scratch, more than the %zu available "
                  "(use chol_solve)", need, SOLVE_SCRATCH_BYTES);
        OPF_CHECK(C->factored, OPF_E_STATE, "chol_solve_noalloc: no successful factorization");
        char* base = static_cast<char*>(scratch_address());
        SolveBufs B{reinterpret_cast<double*>(base + o_y), reinterpret_cast<double*>(base + o_work),
                    reinterpret_cast<double*>(base + o_upd), reinterpret_cast<double*>(base + o_zx),
                    reinterpret_cast<int32_t*>(base)};
        hipStream_t st = (hipStream_t)stream;
        // the array keeps the previous call's contents: the fault word must start at zero (the exchange
        // blocks are refilled with their sentinel before every sweep inside the solve)
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, 1, 0, B.fault);
        OPF_LAUNCH_CHECK();
        for (int r = 0; r < nrhs; r++)
            solve_enqueue(C, b + (int64_t)r * C->n, x + (int64_t)r * C->n, st, B);
        OPF_CHECK(read_fault(C, B.fault, st) == 0, OPF_E_DEVICE,
                  "chol_solve_noalloc: a wide-front block wait exceeded its bound");
    });
}

extern "C" int chol_export_factor(chol_sym* C, int64_t* lp, int32_t* li, double* lx) {
    return guarded([&] {
        OPF_CHECK(C && lp && li, OPF_E_INVALID, "chol_export_factor: null argument");
        std::vector<double> F;
        if (lx) {
            OPF_CHECK(C->factored, OPF_E_STATE, "chol_export_factor: no successful factorization");
            C->dev.run();
            F.resize(C->front_total);
            OPF_HIP(hipDeviceSynchronize());
            OPF_HIP(hipMemcpy(F.data(), C->fronts.p, C->front_total * 8, hipMemcpyDeviceToHost));
        }
        const Symbolic& S = C->S;
        int64_t q = 0;
        lp[0] = 0;
        for (int s = 0; s < S.nsuper; s++) {
            int f = C->h_first[s], nn = C->h_ncol[s], m = C->h_mrows[s];
            const int32_t* R = S.rows_flat.data() + S.rows_ptr[s];
            for (int jc = 0; jc < nn; jc++) {
                for (int jr = jc; jr < m; jr++) {
                    li[q] = R[jr];
                    if (lx) lx[q] = F[C->h_foff[s] + fcol(m, jc) + jr];
                    q++;
                }
                lp[f + jc + 1] = q;
            }
        }
    });
}

extern "C" int chol_timing(chol_sym* C, int enable) {
    return guarded([&] {
        OPF_CHECK(C, OPF_E_INVALID, "chol_timing: null handle");
        C->timing = enable & ((1 << NCAT) - 1);
        C->ev_used = 0;
        for (int q = 0; q < NCAT; q++) {
            C->t_ms[q] = 0;
            C->t_launch[q] = 0;
            C->t_flops[q] = 0;
            C->t_bytes[q] = 0;
        }
    });
}

extern "C" int chol_timing_read(const chol_sym* C, double* ms, int64_t* launches, double* flops, double* bytes) {
    return guarded([&] {
        OPF_CHECK(C, OPF_E_INVALID, "chol_timing_read: null handle");
        for (int q = 0; q < NCAT; q++) {
            if (ms) ms[q] = C->t_ms[q];
            if (launches) launches[q] = C->t_launch[q];
            if (flops) flops[q] = C->t_flops[q];
            if (bytes) bytes[q] = C->t_bytes[q];
        }
    });
}
