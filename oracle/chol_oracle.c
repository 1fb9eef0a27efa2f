/*
 * Oracle: symbolic analysis and Cholesky factorization of the condensed KKT
 * matrix, written as plainly as possible (FP64, single thread, no BLAS).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU reference that the HIP
 * path is checked against; the product path never links it.
 *
 * The paper factors the condensed matrix K (Section IV-C, condensed system)
 * with Cholesky under a fixed pivot sequence from a minimum-degree ordering
 * (Section V-A), which is valid because K is positive definite once the
 * inertia is correct (Section IV-C, Sylvester's law).  The paper used an
 * approximate minimum degree code; two independent programs cannot reproduce
 * approximate degrees bit for bit, so the ordering here is fully specified:
 *
 *   ordering   exact minimum degree on the elimination graph of K: at every
 *              step pick the uneliminated vertex of smallest true degree
 *              (number of uneliminated neighbours), ties to the smallest
 *              original index.  Dense-tail rule: before a pick, with r
 *              vertices left and minimum degree d, if d >= dense_frac*(r-1)
 *              or d >= dense_abs, the r remaining vertices are ordered by
 *              ascending original index and the ordering stops.
 *   etree      parent(j) = min{ i > j : L(i,j) != 0 }.
 *   postorder  depth-first, children visited in ascending index, roots in
 *              ascending index; final permutation = ordering o postorder.
 *   supernodes fundamental: column j+1 joins column j's supernode iff
 *              parent(j) = j+1, colcount(j) = colcount(j+1) + 1 and j is
 *              the only child of j+1.  Relaxed amalgamation: visiting
 *              supernodes in ascending order, a supernode c whose last
 *              column is followed directly by the first column of its parent
 *              supernode p is merged into p when the merged width is at most
 *              max_width and its explicit zeros are at most zero_abs or at
 *              most zero_rel times its stored entries.
 *   numeric    left-looking column Cholesky of P K P^T by the definition
 *              L(j,j) = sqrt(A(j,j) - sum_k L(j,k)^2),
 *              L(i,j) = (A(i,j) - sum_k L(i,k) L(j,k)) / L(j,j).
 *   solve      L y = b by columns, then L^T x = y by columns.
 *   LU         the LU factorization of P K P^T with the same fixed pivot
 *              sequence (Section VI names LU refactorization beside
 *              Cholesky), Doolittle's definition: U(k,j) = A(k,j) -
 *              sum_{t<k} L(k,t) U(t,j), L(i,k) = (A(i,k) - sum_{t<k} L(i,t)
 *              U(t,k)) / U(k,k).  For symmetric A, U = D L^T with D = diag(U)
 *              (so U(t,j) = D(t) L(j,t)); the factor keeps L below the
 *              diagonal and D on it.  A pivot is accepted when |D(j)| >
 *              piv_tol * |A(j,j)| (piv_tol = 0: when it is nonzero).  Solve:
 *              L z = b, y = z / D, L^T x = y.
 *
 * Matrices are lower-triangular CSC (column pointers, row indices ascending).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int32_t i32;
typedef int64_t i64;

/* ------------------------------------------------------------------ min-heap of (degree, index) */
typedef struct {
    i64* key; /* degree * (n+1) + index */
    i64 size, cap;
} heap_t;

static int heap_push(heap_t* h, i64 k) {
    if (h->size == h->cap) {
        i64 nc = h->cap ? 2 * h->cap : 1024;
        i64* nk = (i64*)realloc(h->key, (size_t)nc * sizeof(i64));
        if (!nk) return -1;
        h->key = nk;
        h->cap = nc;
    }
    i64 i = h->size++;
    h->key[i] = k;
    while (i > 0) {
        i64 p = (i - 1) / 2;
        if (h->key[p] <= h->key[i]) break;
        i64 t = h->key[p];
        h->key[p] = h->key[i];
        h->key[i] = t;
        i = p;
    }
    return 0;
}

static i64 heap_pop(heap_t* h) {
    i64 top = h->key[0];
    h->key[0] = h->key[--h->size];
    i64 i = 0;
    for (;;) {
        i64 l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->size && h->key[l] < h->key[s]) s = l;
        if (r < h->size && h->key[r] < h->key[s]) s = r;
        if (s == i) break;
        i64 t = h->key[s];
        h->key[s] = h->key[i];
        h->key[i] = t;
        i = s;
    }
    return top;
}

/* ------------------------------------------------------------------ explicit elimination graph */
typedef struct {
    i32* v;
    i32 len, cap;
} set_t; /* sorted vertex list */

static int set_reserve(set_t* s, i32 cap) {
    if (cap <= s->cap) return 0;
    i32 nc = s->cap ? s->cap : 4;
    while (nc < cap) nc *= 2;
    i32* nv = (i32*)realloc(s->v, (size_t)nc * sizeof(i32));
    if (!nv) return -1;
    s->v = nv;
    s->cap = nc;
    return 0;
}

/* dst <- (dst U src) \ {x, y}; buf is scratch of sufficient size */
static int set_union_minus(set_t* dst, const set_t* src, i32 x, i32 y, i32* buf) {
    i32 a = 0, b = 0, k = 0;
    while (a < dst->len || b < src->len) {
        i32 va = a < dst->len ? dst->v[a] : INT32_MAX;
        i32 vb = b < src->len ? src->v[b] : INT32_MAX;
        i32 w;
        if (va < vb) {
            w = va;
            a++;
        } else if (vb < va) {
            w = vb;
            b++;
        } else {
            w = va;
            a++;
            b++;
        }
        if (w != x && w != y) buf[k++] = w;
    }
    if (set_reserve(dst, k) != 0) return -1;
    memcpy(dst->v, buf, (size_t)k * sizeof(i32));
    dst->len = k;
    return 0;
}

/*
 * Minimum-degree ordering of the graph given by the lower CSC pattern
 * (colptr, rowind) of an n x n symmetric matrix.  order[k] = original index
 * of the k-th eliminated vertex.  Returns 0, or -1 on allocation failure.
 */
int oracle_min_degree(i32 n, const i32* colptr, const i32* rowind, double dense_frac, i32 dense_abs,
                      i32* order) {
    set_t* adj = (set_t*)calloc((size_t)n, sizeof(set_t));
    char* done = (char*)calloc((size_t)n, 1);
    i32* buf = (i32*)malloc((size_t)(2 * n + 2) * sizeof(i32));
    i32* cnt = (i32*)calloc((size_t)n, sizeof(i32));
    heap_t h = {0, 0, 0};
    int rc = -1;
    if (!adj || !done || !buf || !cnt) goto out;
    /* adjacency from the off-diagonal pattern, both directions */
    for (i32 j = 0; j < n; j++)
        for (i32 p = colptr[j]; p < colptr[j + 1]; p++)
            if (rowind[p] != j) {
                cnt[j]++;
                cnt[rowind[p]]++;
            }
    for (i32 j = 0; j < n; j++)
        if (set_reserve(&adj[j], cnt[j] + 1) != 0) goto out;
    for (i32 j = 0; j < n; j++)
        for (i32 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 i = rowind[p];
            if (i == j) continue;
            adj[j].v[adj[j].len++] = i;
            adj[i].v[adj[i].len++] = j;
        }
    /* sort + dedupe each list */
    for (i32 j = 0; j < n; j++) {
        set_t* s = &adj[j];
        for (i32 a = 1; a < s->len; a++) { /* insertion sort: lists are short */
            i32 v = s->v[a], b = a - 1;
            while (b >= 0 && s->v[b] > v) {
                s->v[b + 1] = s->v[b];
                b--;
            }
            s->v[b + 1] = v;
        }
        i32 k = 0;
        for (i32 a = 0; a < s->len; a++)
            if (k == 0 || s->v[k - 1] != s->v[a]) s->v[k++] = s->v[a];
        s->len = k;
    }
    const i64 W = (i64)n + 1;
    for (i32 j = 0; j < n; j++)
        if (heap_push(&h, (i64)adj[j].len * W + j) != 0) goto out;
    i32 nel = 0;
    while (nel < n) {
        /* current minimum (skip stale heap entries) */
        i32 v = -1;
        i32 d = 0;
        while (h.size > 0) {
            i64 key = h.key[0];
            i32 cand = (i32)(key % W);
            i32 deg = (i32)(key / W);
            if (done[cand] || adj[cand].len != deg) {
                heap_pop(&h);
                continue;
            }
            v = cand;
            d = deg;
            break;
        }
        i32 r = n - nel;
        if ((double)d >= dense_frac * (double)(r - 1) || d >= dense_abs) {
            for (i32 j = 0; j < n; j++)
                if (!done[j]) order[nel++] = j;
            break;
        }
        heap_pop(&h);
        order[nel++] = v;
        done[v] = 1;
        /* neighbours of v become a clique */
        for (i32 a = 0; a < adj[v].len; a++) {
            i32 u = adj[v].v[a];
            if (set_union_minus(&adj[u], &adj[v], u, v, buf) != 0) goto out;
            if (heap_push(&h, (i64)adj[u].len * W + u) != 0) goto out;
        }
        adj[v].len = 0;
    }
    rc = 0;
out:
    if (adj)
        for (i32 j = 0; j < n; j++) free(adj[j].v);
    free(adj);
    free(done);
    free(buf);
    free(cnt);
    free(h.key);
    return rc;
}

static int cmp_i32(const void* a, const void* b) {
    i32 x = *(const i32*)a, y = *(const i32*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------ permuted pattern */
/* B = P A P^T (lower CSC, rows ascending) where perm[k] = old index of new k. */
static int permute_lower(i32 n, const i32* colptr, const i32* rowind, const double* val, const i32* perm,
                         i32** bptr, i32** bind, double** bval) {
    i32* inv = (i32*)malloc((size_t)n * sizeof(i32));
    i32* cnt = (i32*)calloc((size_t)n + 1, sizeof(i32));
    i32 nnz = colptr[n];
    i32* bi = (i32*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(i32));
    double* bv = val ? (double*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double)) : NULL;
    if (!inv || !cnt || !bi || (val && !bv)) {
        free(inv);
        free(cnt);
        free(bi);
        free(bv);
        return -1;
    }
    for (i32 k = 0; k < n; k++) inv[perm[k]] = k;
    for (i32 j = 0; j < n; j++)
        for (i32 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 a = inv[rowind[p]], b = inv[j];
            i32 c = a < b ? a : b;
            cnt[c + 1]++;
        }
    for (i32 j = 0; j < n; j++) cnt[j + 1] += cnt[j];
    i32* pos = (i32*)malloc((size_t)n * sizeof(i32));
    if (!pos) {
        free(inv);
        free(cnt);
        free(bi);
        free(bv);
        return -1;
    }
    memcpy(pos, cnt, (size_t)n * sizeof(i32));
    for (i32 j = 0; j < n; j++)
        for (i32 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 a = inv[rowind[p]], b = inv[j];
            i32 r = a > b ? a : b, c = a < b ? a : b;
            i32 q = pos[c]++;
            bi[q] = r;
            if (bv) bv[q] = val[p];
        }
    /* sort rows within each column (insertion sort; columns are short) */
    for (i32 j = 0; j < n; j++)
        for (i32 a = cnt[j] + 1; a < cnt[j + 1]; a++) {
            i32 r = bi[a];
            double x = bv ? bv[a] : 0.0;
            i32 b = a - 1;
            while (b >= cnt[j] && bi[b] > r) {
                bi[b + 1] = bi[b];
                if (bv) bv[b + 1] = bv[b];
                b--;
            }
            bi[b + 1] = r;
            if (bv) bv[b + 1] = x;
        }
    free(inv);
    free(pos);
    *bptr = cnt;
    *bind = bi;
    if (bval) *bval = bv;
    return 0;
}

/*
 * Symbolic factorization of a lower CSC pattern by its definition:
 * struct(L_j) = {j} U {i > j : A(i,j) != 0} U (U_{c : parent(c) = j} struct(L_c) \ {c}),
 * parent(j) = min(struct(L_j) \ {j}).  Produces parent[] and, if lp/li are
 * non-NULL, the full L pattern (malloc'd).  Column counts include the diagonal.
 */
static int symbolic_factor(i32 n, const i32* bptr, const i32* bind, i32* parent, i32* colcount, i32** lp_out,
                           i32** li_out) {
    i32* head = (i32*)malloc((size_t)n * sizeof(i32)); /* child lists */
    i32* next = (i32*)malloc((size_t)n * sizeof(i32));
    i32* mark = (i32*)malloc((size_t)n * sizeof(i32));
    i32* lp = (i32*)malloc(((size_t)n + 1) * sizeof(i32));
    i64 cap = (i64)bptr[n] + n + 16;
    i32* li = (i32*)malloc((size_t)cap * sizeof(i32));
    i32* tmp = (i32*)malloc((size_t)n * sizeof(i32));
    if (!head || !next || !mark || !lp || !li || !tmp) goto fail;
    for (i32 j = 0; j < n; j++) {
        head[j] = -1;
        mark[j] = -1;
    }
    lp[0] = 0;
    for (i32 j = 0; j < n; j++) {
        i32 k = 0;
        mark[j] = j;
        tmp[k++] = j;
        for (i32 p = bptr[j]; p < bptr[j + 1]; p++) {
            i32 i = bind[p];
            if (i > j && mark[i] != j) {
                mark[i] = j;
                tmp[k++] = i;
            }
        }
        for (i32 c = head[j]; c != -1; c = next[c])
            for (i32 p = lp[c]; p < lp[c + 1]; p++) {
                i32 i = li[p];
                if (i > j && mark[i] != j) {
                    mark[i] = j;
                    tmp[k++] = i;
                }
            }
        /* sort the column structure */
        qsort(tmp, (size_t)k, sizeof(i32), cmp_i32);
        if ((i64)lp[j] + k > cap) {
            while ((i64)lp[j] + k > cap) cap *= 2;
            i32* nl = (i32*)realloc(li, (size_t)cap * sizeof(i32));
            if (!nl) goto fail;
            li = nl;
        }
        memcpy(li + lp[j], tmp, (size_t)k * sizeof(i32));
        lp[j + 1] = lp[j] + k;
        colcount[j] = k;
        parent[j] = k > 1 ? tmp[1] : -1;
        if (parent[j] >= 0) {
            next[j] = head[parent[j]];
            head[parent[j]] = j;
        }
    }
    free(head);
    free(next);
    free(mark);
    free(tmp);
    if (lp_out) {
        *lp_out = lp;
        *li_out = li;
    } else {
        free(lp);
        free(li);
    }
    return 0;
fail:
    free(head);
    free(next);
    free(mark);
    free(lp);
    free(li);
    free(tmp);
    return -1;
}

/* postorder: post[k] = k-th vertex visited; children in ascending index, roots ascending */
static int postorder(i32 n, const i32* parent, i32* post) {
    i32* head = (i32*)malloc((size_t)n * sizeof(i32));
    i32* next = (i32*)malloc((size_t)n * sizeof(i32));
    i32* stack = (i32*)malloc((size_t)n * sizeof(i32));
    if (!head || !next || !stack) {
        free(head);
        free(next);
        free(stack);
        return -1;
    }
    for (i32 j = 0; j < n; j++) head[j] = -1;
    /* insert in descending order so that lists are ascending */
    for (i32 j = n - 1; j >= 0; j--)
        if (parent[j] >= 0) {
            next[j] = head[parent[j]];
            head[parent[j]] = j;
        }
    i32 k = 0;
    for (i32 root = 0; root < n; root++) {
        if (parent[root] >= 0) continue;
        i32 top = 0;
        stack[top++] = root;
        while (top > 0) {
            i32 v = stack[top - 1];
            i32 c = head[v];
            if (c == -1) {
                top--;
                post[k++] = v;
            } else {
                head[v] = next[c];
                stack[top++] = c;
            }
        }
    }
    free(head);
    free(next);
    free(stack);
    return k == n ? 0 : -1;
}

/*
 * Full analysis.  Inputs: lower CSC pattern of K in original numbering and
 * the ordering/amalgamation parameters.  Outputs (caller-allocated, size n
 * unless noted): perm (perm[k] = original index of pivot k), parent (etree
 * in final numbering), colcount (L column counts incl. diagonal), snode_ptr
 * (size n+1; first column of each supernode, entries 0..nsuper), *nsuper.
 * Returns 0 on success.
 */
int oracle_analyze(i32 n, const i32* colptr, const i32* rowind, double dense_frac, i32 dense_abs, i32 max_width,
                   i64 zero_abs, double zero_rel, i32* perm, i32* parent, i32* colcount, i32* snode_ptr,
                   i32* nsuper) {
    i32* order = (i32*)malloc((size_t)n * sizeof(i32));
    i32* post = (i32*)malloc((size_t)n * sizeof(i32));
    i32* par0 = (i32*)malloc((size_t)n * sizeof(i32));
    i32* cc0 = (i32*)malloc((size_t)n * sizeof(i32));
    i32 *bptr = NULL, *bind = NULL;
    int rc = -1;
    if (!order || !post || !par0 || !cc0) goto out;
    if (oracle_min_degree(n, colptr, rowind, dense_frac, dense_abs, order) != 0) goto out;
    if (permute_lower(n, colptr, rowind, NULL, order, &bptr, &bind, NULL) != 0) goto out;
    if (symbolic_factor(n, bptr, bind, par0, cc0, NULL, NULL) != 0) goto out;
    if (postorder(n, par0, post) != 0) goto out;
    for (i32 k = 0; k < n; k++) perm[k] = order[post[k]];
    free(bptr);
    free(bind);
    bptr = bind = NULL;
    if (permute_lower(n, colptr, rowind, NULL, perm, &bptr, &bind, NULL) != 0) goto out;
    if (symbolic_factor(n, bptr, bind, parent, colcount, NULL, NULL) != 0) goto out;
    /* fundamental supernodes */
    {
        i32* nchild = (i32*)calloc((size_t)n, sizeof(i32));
        if (!nchild) goto out;
        for (i32 j = 0; j < n; j++)
            if (parent[j] >= 0) nchild[parent[j]]++;
        i32 s = 0;
        snode_ptr[0] = 0;
        for (i32 j = 1; j < n; j++) {
            int join = parent[j - 1] == j && colcount[j - 1] == colcount[j] + 1 && nchild[j] == 1;
            if (!join) snode_ptr[++s] = j;
        }
        if (n > 0) snode_ptr[++s] = n;
        free(nchild);
        i32 ns = s;
        /* relaxed amalgamation, supernodes visited in ascending order */
        i32* first = (i32*)malloc((size_t)(ns + 1) * sizeof(i32));
        i32* last = (i32*)malloc((size_t)(ns + 1) * sizeof(i32));
        i32* rows = (i32*)malloc((size_t)(ns + 1) * sizeof(i32)); /* m_s: rows of the supernode */
        i64* zeros = (i64*)calloc((size_t)(ns + 1), sizeof(i64));
        char* dead = (char*)calloc((size_t)(ns + 1), 1);
        i32* owner = (i32*)malloc((size_t)(n > 0 ? n : 1) * sizeof(i32));
        if (!first || !last || !rows || !zeros || !dead || !owner) {
            free(first);
            free(last);
            free(rows);
            free(zeros);
            free(dead);
            free(owner);
            goto out;
        }
        for (i32 t = 0; t < ns; t++) {
            first[t] = snode_ptr[t];
            last[t] = snode_ptr[t + 1] - 1;
            rows[t] = colcount[first[t]];
            for (i32 j = first[t]; j <= last[t]; j++) owner[j] = t;
        }
        for (i32 c = 0; c < ns; c++) {
            i32 pc = parent[last[c]];
            if (pc < 0) continue;
            i32 p = owner[pc];
            if (last[c] + 1 != first[p]) continue;
            i64 nc = last[c] - first[c] + 1, np_ = last[p] - first[p] + 1;
            i64 mc = rows[c], mp = rows[p];
            i64 nm = nc + np_, mm = nc + mp;
            i64 trap_c = nc * mc - nc * (nc - 1) / 2;
            i64 trap_p = np_ * mp - np_ * (np_ - 1) / 2;
            i64 trap_m = nm * mm - nm * (nm - 1) / 2;
            i64 z = zeros[c] + zeros[p] + (trap_m - trap_c - trap_p);
            int ok = nm <= max_width && (z <= zero_abs || (double)z <= zero_rel * (double)trap_m);
            if (!ok) continue;
            first[p] = first[c];
            rows[p] = (i32)mm;
            zeros[p] = z;
            dead[c] = 1;
            for (i32 j = first[c]; j <= last[c]; j++) owner[j] = p;
        }
        i32 k = 0;
        for (i32 t = 0; t < ns; t++)
            if (!dead[t]) snode_ptr[k++] = first[t];
        snode_ptr[k] = n;
        *nsuper = k;
        free(first);
        free(last);
        free(rows);
        free(zeros);
        free(dead);
        free(owner);
    }
    rc = 0;
out:
    free(order);
    free(post);
    free(par0);
    free(cc0);
    free(bptr);
    free(bind);
    return rc;
}

/* ------------------------------------------------------------------ numeric factor and solve */
typedef struct {
    i32 n;
    i32 *lp, *li; /* L pattern, CSC */
    double* lx;
    i32 *rp, *rk, *rpos; /* row structure of L: row j -> columns k<j and position of L(j,k) in lx */
    i32* perm;
    i32 *bptr, *bind; /* permuted A pattern */
    i32* amap;        /* original CSC entry p -> position in permuted (bptr, bind) */
} oracle_chol;

void oracle_chol_free(oracle_chol* f) {
    if (!f) return;
    free(f->lp);
    free(f->li);
    free(f->lx);
    free(f->rp);
    free(f->rk);
    free(f->rpos);
    free(f->perm);
    free(f->bptr);
    free(f->bind);
    free(f->amap);
    free(f);
}

/* Prepare numeric factorization for pattern (colptr,rowind) under permutation perm. */
oracle_chol* oracle_chol_create(i32 n, const i32* colptr, const i32* rowind, const i32* perm) {
    oracle_chol* f = (oracle_chol*)calloc(1, sizeof(oracle_chol));
    if (!f) return NULL;
    f->n = n;
    f->perm = (i32*)malloc((size_t)(n > 0 ? n : 1) * sizeof(i32));
    i32* par = (i32*)malloc((size_t)(n > 0 ? n : 1) * sizeof(i32));
    i32* cc = (i32*)malloc((size_t)(n > 0 ? n : 1) * sizeof(i32));
    if (!f->perm || !par || !cc) goto fail;
    memcpy(f->perm, perm, (size_t)n * sizeof(i32));
    if (permute_lower(n, colptr, rowind, NULL, perm, &f->bptr, &f->bind, NULL) != 0) goto fail;
    if (symbolic_factor(n, f->bptr, f->bind, par, cc, &f->lp, &f->li) != 0) goto fail;
    i64 nnzl = f->lp[n];
    f->lx = (double*)calloc((size_t)(nnzl > 0 ? nnzl : 1), sizeof(double));
    f->rp = (i32*)calloc((size_t)n + 1, sizeof(i32));
    f->rk = (i32*)malloc((size_t)(nnzl > 0 ? nnzl : 1) * sizeof(i32));
    f->rpos = (i32*)malloc((size_t)(nnzl > 0 ? nnzl : 1) * sizeof(i32));
    if (!f->lx || !f->rp || !f->rk || !f->rpos) goto fail;
    for (i32 k = 0; k < n; k++)
        for (i32 p = f->lp[k] + 1; p < f->lp[k + 1]; p++) f->rp[f->li[p] + 1]++;
    for (i32 j = 0; j < n; j++) f->rp[j + 1] += f->rp[j];
    {
        i32* fill = (i32*)malloc((size_t)(n > 0 ? n : 1) * sizeof(i32));
        if (!fill) goto fail;
        memcpy(fill, f->rp, (size_t)n * sizeof(i32));
        for (i32 k = 0; k < n; k++)
            for (i32 p = f->lp[k] + 1; p < f->lp[k + 1]; p++) {
                i32 q = fill[f->li[p]]++;
                f->rk[q] = k;
                f->rpos[q] = p;
            }
        free(fill);
    }
    /* map each original entry to its slot in the permuted pattern */
    {
        i32 nnz = colptr[n];
        f->amap = (i32*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(i32));
        i32* inv = (i32*)malloc((size_t)(n > 0 ? n : 1) * sizeof(i32));
        if (!f->amap || !inv) {
            free(inv);
            goto fail;
        }
        for (i32 k = 0; k < n; k++) inv[perm[k]] = k;
        for (i32 j = 0; j < n; j++)
            for (i32 p = colptr[j]; p < colptr[j + 1]; p++) {
                i32 a = inv[rowind[p]], b = inv[j];
                i32 r = a > b ? a : b, c = a < b ? a : b;
                i32 q = -1;
                for (i32 t = f->bptr[c]; t < f->bptr[c + 1]; t++)
                    if (f->bind[t] == r) {
                        q = t;
                        break;
                    }
                f->amap[p] = q;
            }
        free(inv);
    }
    free(par);
    free(cc);
    return f;
fail:
    free(par);
    free(cc);
    oracle_chol_free(f);
    return NULL;
}

i64 oracle_chol_nnz(const oracle_chol* f) { return f->lp[f->n]; }

/* Copy out the L pattern (CSC) and values. */
void oracle_chol_export(const oracle_chol* f, i32* lp, i32* li, double* lx) {
    memcpy(lp, f->lp, ((size_t)f->n + 1) * sizeof(i32));
    memcpy(li, f->li, (size_t)f->lp[f->n] * sizeof(i32));
    if (lx) memcpy(lx, f->lx, (size_t)f->lp[f->n] * sizeof(double));
}

/*
 * Numeric factorization of P K P^T where K has the pattern given at create
 * time and values val (same CSC order).  A pivot is accepted when it exceeds
 * piv_tol * |A(j,j)| (piv_tol = 0: when it is positive).  Returns 0 if every
 * pivot is accepted, else (1 + j) for the first pivot column j that is not.
 */
int oracle_chol_factor(oracle_chol* f, const double* val, double piv_tol) {
    i32 n = f->n;
    i32 nnz = f->bptr[n];
    double* w = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double* bv = (double*)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(double));
    if (!w || !bv) {
        free(w);
        free(bv);
        return -1;
    }
    /* original entries into the permuted pattern (one entry per (row, col)) */
    for (i32 p = 0; p < nnz; p++) bv[f->amap[p]] = val[p];
    int status = 0;
    for (i32 j = 0; j < n; j++) {
        /* w = A(:, j) on rows >= j */
        for (i32 p = f->bptr[j]; p < f->bptr[j + 1]; p++) w[f->bind[p]] = bv[p];
        /* subtract L(:,k) L(j,k) for every k < j with L(j,k) != 0 */
        for (i32 q = f->rp[j]; q < f->rp[j + 1]; q++) {
            i32 k = f->rk[q];
            i32 pj = f->rpos[q]; /* position of L(j,k) */
            double ljk = f->lx[pj];
            for (i32 p = pj; p < f->lp[k + 1]; p++) w[f->li[p]] -= f->lx[p] * ljk;
        }
        double d = w[j];
        double ajj = bv[f->bptr[j]]; /* diagonal entry: first row of column j */
        if (!(d > piv_tol * fabs(ajj))) {
            status = 1 + j;
            for (i32 p = f->lp[j]; p < f->lp[j + 1]; p++) w[f->li[p]] = 0.0;
            break;
        }
        double ljj = sqrt(d);
        f->lx[f->lp[j]] = ljj;
        w[j] = 0.0;
        for (i32 p = f->lp[j] + 1; p < f->lp[j + 1]; p++) {
            i32 i = f->li[p];
            f->lx[p] = w[i] / ljj;
            w[i] = 0.0;
        }
    }
    free(w);
    free(bv);
    return status;
}

/*
 * LU factorization with the fixed pivot sequence in its symmetric form P K P^T = L D L^T (see the header),
 * left-looking by columns: w = A(:, j) - sum_{k<j, L(j,k) != 0} L(:, k) U(k, j) with U(k, j) = D(k) L(j, k);
 * D(j) = w(j), L(i, j) = w(i) / D(j).  lx holds D(j) at the diagonal position.  Returns 0 if every pivot is
 * accepted, else (1 + j) for the first pivot column j that is not.
 */
int oracle_ldlt_factor(oracle_chol* f, const double* val, double piv_tol) {
    i32 n = f->n;
    i32 nnz = f->bptr[n];
    double* w = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double* bv = (double*)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(double));
    if (!w || !bv) {
        free(w);
        free(bv);
        return -1;
    }
    for (i32 p = 0; p < nnz; p++) bv[f->amap[p]] = val[p];
    int status = 0;
    for (i32 j = 0; j < n; j++) {
        for (i32 p = f->bptr[j]; p < f->bptr[j + 1]; p++) w[f->bind[p]] = bv[p];
        for (i32 q = f->rp[j]; q < f->rp[j + 1]; q++) {
            i32 k = f->rk[q];
            i32 pj = f->rpos[q]; /* position of L(j,k) */
            double ukj = f->lx[f->lp[k]] * f->lx[pj]; /* U(k,j) = D(k) L(j,k) */
            for (i32 p = pj; p < f->lp[k + 1]; p++) w[f->li[p]] -= f->lx[p] * ukj;
        }
        double d = w[j];
        double ajj = bv[f->bptr[j]];
        if (!(fabs(d) > piv_tol * fabs(ajj))) {
            status = 1 + j;
            for (i32 p = f->lp[j]; p < f->lp[j + 1]; p++) w[f->li[p]] = 0.0;
            break;
        }
        f->lx[f->lp[j]] = d;
        w[j] = 0.0;
        for (i32 p = f->lp[j] + 1; p < f->lp[j + 1]; p++) {
            i32 i = f->li[p];
            f->lx[p] = w[i] / d;
            w[i] = 0.0;
        }
    }
    free(w);
    free(bv);
    return status;
}

/* x = K^{-1} b from the L D L^T factor (b and x in original numbering; may alias). */
void oracle_ldlt_solve(const oracle_chol* f, const double* b, double* x) {
    i32 n = f->n;
    double* y = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!y) return;
    for (i32 k = 0; k < n; k++) y[k] = b[f->perm[k]];
    for (i32 j = 0; j < n; j++) {
        double yj = y[j];
        for (i32 p = f->lp[j] + 1; p < f->lp[j + 1]; p++) y[f->li[p]] -= f->lx[p] * yj;
    }
    for (i32 j = 0; j < n; j++) y[j] /= f->lx[f->lp[j]];
    for (i32 j = n - 1; j >= 0; j--) {
        double s = y[j];
        for (i32 p = f->lp[j] + 1; p < f->lp[j + 1]; p++) s -= f->lx[p] * y[f->li[p]];
        y[j] = s;
    }
    for (i32 k = 0; k < n; k++) x[f->perm[k]] = y[k];
    free(y);
}

/* x = K^{-1} b using the last factor (b and x in original numbering; may alias). */
void oracle_chol_solve(const oracle_chol* f, const double* b, double* x) {
    i32 n = f->n;
    double* y = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!y) return;
    for (i32 k = 0; k < n; k++) y[k] = b[f->perm[k]];
    for (i32 j = 0; j < n; j++) {
        y[j] /= f->lx[f->lp[j]];
        double yj = y[j];
        for (i32 p = f->lp[j] + 1; p < f->lp[j + 1]; p++) y[f->li[p]] -= f->lx[p] * yj;
    }
    for (i32 j = n - 1; j >= 0; j--) {
        double s = y[j];
        for (i32 p = f->lp[j] + 1; p < f->lp[j + 1]; p++) s -= f->lx[p] * y[f->li[p]];
        y[j] = s / f->lx[f->lp[j]];
    }
    for (i32 k = 0; k < n; k++) x[f->perm[k]] = y[k];
    free(y);
}
