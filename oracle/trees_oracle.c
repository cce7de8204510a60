/*
 * TREES CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU product path never calls it, and the two
 * share no code, headers, tables or helpers.
 *
 * Two kinds of functions live here:
 *
 *  1. Plain sequential evaluators of what each workload computes: Fibonacci
 *     by iteration and by naive recursion, the N-queens solution count by
 *     backtracking, sorting (the C library qsort, plus a sequential
 *     recursive merge sort), breadth-first search with a FIFO queue,
 *     Dijkstra's shortest paths, and the discrete Fourier transform by its
 *     defining sum (fp64).
 *
 *  2. A step-by-step emulator of the epoch semantics: the Task Vector
 *     Machine of Section 4.3 in the representation TREES uses on the GPU
 *     (Section 5.1.2: one integer per task-vector entry encodes epoch number
 *     and task type as epoch*NumTaskTypes + type, an entry is runnable in the
 *     epoch whose number is CEN when its code lies in
 *     [CEN*NumTaskTypes + 1, (CEN+1)*NumTaskTypes]; Sections 5.2.1-5.2.4:
 *     initialisation, the three epoch phases, the join and NDRange stacks,
 *     nextFreeCore and oldNextFreeCore).
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes of the repository):
 *  - task types are numbered from 1 so that code 0 is the unique
 *    "invalid / finished" value and the root runs in epoch 0;
 *  - the join stack and the NDRange stack are one stack of records
 *    {CEN, b, e, cend}; cend is nextFreeCore at the moment the record was
 *    pushed, and popping a record sets nextFreeCore back to cend (this is
 *    the "nextFreeCore decreases" of Section 5.3, taken so that a join body
 *    never has its unread children overwritten by a new fork);
 *  - a joining task stores (first child index, number of children) in its
 *    own entry (explicit continuation passing, Section 4.1);
 *  - a task that neither emits nor joins marks its entry invalid;
 *  - tasks = valid entry executions, join continuations included; idle
 *    (invalid) lanes in a launched range are counted as launched only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* 1. Plain sequential evaluators                                             */
/* ------------------------------------------------------------------------- */

/* F(n) from its definition F(0)=0, F(1)=1, F(n)=F(n-1)+F(n-2), iteratively. */
int64_t orc_fib_iter(int32_t n) {
    int64_t a = 0, b = 1;
    for (int32_t k = 0; k < n; ++k) { int64_t t = a + b; a = b; b = t; }
    return a;
}

/* Naive recursion: the sequential program the task tree is made from. */
static int64_t fib_rec(int32_t n, int64_t *calls) {
    ++*calls;
    if (n < 2) return n;
    return fib_rec(n - 1, calls) + fib_rec(n - 2, calls);
}
int64_t orc_fib_rec(int32_t n, int64_t *calls) {
    int64_t c = 0;
    int64_t v = fib_rec(n, &c);
    if (calls) *calls = c;
    return v;
}

/* N-queens: number of placements of n non-attacking queens, counted by
 * row-by-row backtracking over column / diagonal occupancy sets. */
static int64_t nq_rec(int32_t n, int32_t row, uint32_t cols, uint32_t ld, uint32_t rd) {
    if (row == n) return 1;
    uint32_t full = (n >= 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
    uint32_t avail = ~(cols | ld | rd) & full;
    int64_t s = 0;
    while (avail) {
        uint32_t bit = avail & (0u - avail);
        avail ^= bit;
        s += nq_rec(n, row + 1, cols | bit, ((ld | bit) << 1) & full, (rd | bit) >> 1);
    }
    return s;
}
int64_t orc_nqueens_rec(int32_t n) { return n <= 0 ? 1 : nq_rec(n, 0, 0, 0, 0); }

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}
/* The plain definition of the sort result: the C library's qsort. */
void orc_sort_u32(uint32_t *keys, int64_t n) {
    if (n > 1) qsort(keys, (size_t)n, sizeof(uint32_t), cmp_u32);
}

/* Sequential recursive merge sort (halves, runs of <= 64 keys insertion
 * sorted): the single-core program the merge-sort task tree comes from. */
static void ins_sort(uint32_t *a, int64_t n) {
    for (int64_t i = 1; i < n; ++i) {
        uint32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
        a[j + 1] = x;
    }
}
static void merge_into(const uint32_t *s, int64_t lo, int64_t mid, int64_t hi, uint32_t *d) {
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) d[k++] = (s[j] < s[i]) ? s[j++] : s[i++];
    while (i < mid) d[k++] = s[i++];
    while (j < hi) d[k++] = s[j++];
}
static void msort_rec(uint32_t *a, uint32_t *t, int64_t lo, int64_t hi) {
    if (hi - lo <= 64) { ins_sort(a + lo, hi - lo); return; }
    int64_t mid = lo + (hi - lo) / 2;
    msort_rec(a, t, lo, mid);
    msort_rec(a, t, mid, hi);
    merge_into(a, lo, mid, hi, t);
    memcpy(a + lo, t + lo, (size_t)(hi - lo) * sizeof(uint32_t));
}
void orc_msort_rec(uint32_t *keys, uint32_t *tmp, int64_t n) { msort_rec(keys, tmp, 0, n); }

/* Unweighted hop distance from src (-1 = unreachable) by FIFO-queue BFS. */
void orc_bfs_queue(int32_t V, const int32_t *row_ptr, const int32_t *col, int32_t src,
                   int32_t *depth) {
    for (int32_t v = 0; v < V; ++v) depth[v] = -1;
    if (V <= 0) return;
    int32_t *q = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    int64_t head = 0, tail = 0;
    depth[src] = 0;
    q[tail++] = src;
    while (head < tail) {
        int32_t v = q[head++];
        for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
            int32_t u = col[k];
            if (depth[u] < 0) { depth[u] = depth[v] + 1; q[tail++] = u; }
        }
    }
    free(q);
}

/* Shortest distances from src over non-negative int32 arc weights
 * (Dijkstra, binary heap with lazy deletion); unreachable = INT32_MAX. */
void orc_dijkstra(int32_t V, const int32_t *row_ptr, const int32_t *col, const int32_t *w,
                  int32_t src, int32_t *dist) {
    for (int32_t v = 0; v < V; ++v) dist[v] = INT32_MAX;
    if (V <= 0) return;
    int64_t cap = (int64_t)row_ptr[V] + 1, n = 0;
    int64_t *hd = (int64_t *)malloc((size_t)cap * sizeof(int64_t));   /* key = dist << 32 | vertex */
    dist[src] = 0;
    hd[n++] = (int64_t)src;
    while (n > 0) {
        const int64_t top = hd[0];
        hd[0] = hd[--n];
        for (int64_t i = 0;;) {                                        /* sift down */
            int64_t l = 2 * i + 1, r = l + 1, m = i;
            if (l < n && hd[l] < hd[m]) m = l;
            if (r < n && hd[r] < hd[m]) m = r;
            if (m == i) break;
            int64_t t = hd[i]; hd[i] = hd[m]; hd[m] = t; i = m;
        }
        const int32_t v = (int32_t)(top & 0xFFFFFFFF), d = (int32_t)(top >> 32);
        if (d > dist[v]) continue;                                     /* stale entry */
        for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
            const int32_t u = col[k];
            const int64_t nd = (int64_t)d + w[k];
            if (nd < dist[u]) {
                dist[u] = (int32_t)nd;
                if (n == cap) { cap *= 2; hd = (int64_t *)realloc(hd, (size_t)cap * sizeof(int64_t)); }
                int64_t i = n++;
                hd[i] = (nd << 32) | (uint32_t)u;
                while (i > 0 && hd[(i - 1) / 2] > hd[i]) {                /* sift up */
                    int64_t t = hd[i]; hd[i] = hd[(i - 1) / 2]; hd[(i - 1) / 2] = t; i = (i - 1) / 2;
                }
            }
        }
    }
    free(hd);
}

/* ------------------------------------------------------------------------- */
/* 2. Epoch-semantics emulator                                                */
/* ------------------------------------------------------------------------- */

enum { ORC_FIB32 = 1, ORC_FIB64 = 2, ORC_MSORT = 3, ORC_NQUEENS = 4, ORC_BFS = 5, ORC_POSTORDER = 6,
       ORC_SSSP = 7, ORC_PREORDER = 8, ORC_FFT = 9 };
enum { ORC_OK = 0, ORC_E_OVERFLOW = -3, ORC_E_ENCODING = -8, ORC_E_ARGS = -1 };

typedef struct {
    int32_t epoch, cen, b, e, launched, valid, forks, joins, nfc;
} orc_rec;

typedef struct {
    int64_t result;
    int64_t epochs, tasks, launched, peak;
    int64_t tasks_by_type[2];
    int32_t status, pad;
} orc_stats;

typedef struct orc_tvm {
    int32_t kind, ntt;
    int64_t cap;          /* 0 = grow on demand */
    int64_t alloc;        /* allocated entries */
    int32_t *code, *a0, *a1, *a2, *a3;
    int64_t *r;
    int32_t (*stk)[4];
    int32_t sp, stkcap;
    int64_t nfc, old, joins;
    int32_t cen;
    /* program parameters and payloads (caller-owned) */
    int32_t p0, p1;
    int32_t p2;           /* SSSP: the bucket width delta (0: none) */
    uint32_t *buf[2];
    const int32_t *row_ptr, *col, *wts;
    int32_t *depth;       /* BFS depth / SSSP distance */
    const int32_t *left, *right;
    int32_t *visit_log, *visit_epoch;
    int64_t nvisit;
    const double *fx;     /* FFT input, interleaved (re, im) */
    double *fy;           /* FFT output */
    orc_stats st;
    orc_rec *recs;
    int64_t nrecs, recs_cap;
} orc_tvm;

static int grow(orc_tvm *m, int64_t need) {
    if (need <= m->alloc) return 1;
    if (m->cap > 0 && need > m->cap) return 0;
    int64_t na = m->alloc ? m->alloc : 64;
    while (na < need) na *= 2;
    if (m->cap > 0 && na > m->cap) na = m->cap;
    m->code = (int32_t *)realloc(m->code, (size_t)na * 4);
    m->a0 = (int32_t *)realloc(m->a0, (size_t)na * 4);
    m->a1 = (int32_t *)realloc(m->a1, (size_t)na * 4);
    m->a2 = (int32_t *)realloc(m->a2, (size_t)na * 4);
    m->a3 = (int32_t *)realloc(m->a3, (size_t)na * 4);
    m->r = (int64_t *)realloc(m->r, (size_t)na * 8);
    for (int64_t i = m->alloc; i < na; ++i) {
        m->code[i] = 0; m->a0[i] = m->a1[i] = m->a2[i] = m->a3[i] = 0; m->r[i] = 0;
    }
    m->alloc = na;
    return 1;
}

static void push(orc_tvm *m, int32_t cen, int32_t b, int32_t e, int32_t cend) {
    if (m->sp == m->stkcap) {
        m->stkcap = m->stkcap ? 2 * m->stkcap : 16;
        m->stk = (int32_t(*)[4])realloc(m->stk, (size_t)m->stkcap * sizeof(*m->stk));
    }
    m->stk[m->sp][0] = cen; m->stk[m->sp][1] = b; m->stk[m->sp][2] = e; m->stk[m->sp][3] = cend;
    m->sp++;
}

/* TVM primitives (Section 4.3.2) ----------------------------------------- */

/* fork: take the next free entry; the child becomes runnable next epoch. */
static int64_t tv_fork(orc_tvm *m, int32_t type, int32_t x0, int32_t x1, int32_t x2, int32_t x3) {
    if (!grow(m, m->nfc + 1)) { m->st.status = ORC_E_OVERFLOW; return -1; }
    int64_t i = m->nfc++;
    m->code[i] = (m->cen + 1) * m->ntt + type;
    m->a0[i] = x0; m->a1[i] = x1; m->a2[i] = x2; m->a3[i] = x3;
    return i;
}
/* join: overwrite the task's own entry with the continuation, same epoch number. */
static void tv_join(orc_tvm *m, int64_t i, int32_t type, int32_t x0, int32_t x1, int32_t x2, int32_t x3) {
    m->code[i] = m->cen * m->ntt + type;
    m->a0[i] = x0; m->a1[i] = x1; m->a2[i] = x2; m->a3[i] = x3;
    m->joins++;
}
/* emit: store the value in the task's own entry; the entry never runs again. */
static void tv_emit(orc_tvm *m, int64_t i, int64_t v) { m->r[i] = v; m->code[i] = 0; }
/* neither emit nor join: the entry is finished. */
static void tv_finish(orc_tvm *m, int64_t i) { m->code[i] = 0; }

/* Task bodies --------------------------------------------------------------- */

static void body_fib(orc_tvm *m, int64_t i, int32_t type) {
    if (type == 1) {                       /* FIB(n) */
        int32_t n = m->a0[i];
        if (n < 2) { tv_emit(m, i, n); return; }
        int64_t c = m->nfc;
        if (tv_fork(m, 1, n - 1, 0, 0, 0) < 0) return;
        if (tv_fork(m, 1, n - 2, 0, 0, 0) < 0) return;
        tv_join(m, i, 2, (int32_t)c, 2, 0, 0);
    } else {                               /* SUM(first child) */
        int64_t c = m->a0[i];
        int64_t v = m->r[c] + m->r[c + 1];
        if (m->kind == ORC_FIB32) v = (int64_t)(int32_t)(uint32_t)((uint64_t)m->r[c] + (uint64_t)m->r[c + 1]);
        tv_emit(m, i, v);
    }
}

static void body_nqueens(orc_tvm *m, int64_t i, int32_t type) {
    if (type == 1) {                       /* Q(row, cols, ld, rd): one partial placement */
        int32_t n = m->p0, row = m->a0[i];
        uint32_t full = (1u << n) - 1u;
        uint32_t cols = (uint32_t)m->a1[i], ld = (uint32_t)m->a2[i], rd = (uint32_t)m->a3[i];
        if (row == n) { tv_emit(m, i, 1); return; }
        uint32_t avail = ~(cols | ld | rd) & full;
        if (!avail) { tv_emit(m, i, 0); return; }
        int64_t c = m->nfc;
        int32_t k = 0;
        while (avail) {
            uint32_t bit = avail & (0u - avail);
            avail ^= bit;
            if (tv_fork(m, 1, row + 1, (int32_t)(cols | bit), (int32_t)(((ld | bit) << 1) & full),
                        (int32_t)((rd | bit) >> 1)) < 0) return;
            ++k;
        }
        tv_join(m, i, 2, (int32_t)c, k, 0, 0);
    } else {                               /* QSUM(first child, k) */
        int64_t c = m->a0[i], s = 0;
        for (int32_t j = 0; j < m->a1[i]; ++j) s += m->r[c + j];
        tv_emit(m, i, s);
    }
}

/* Merge sort, buffers by depth: a run at depth d lives in buf[d & 1]; the
 * root (depth 0) therefore ends in buf[0], the caller's key array. */
static void body_msort(orc_tvm *m, int64_t i, int32_t type) {
    int64_t lo = m->a0[i], hi = m->a1[i];
    int32_t d = m->a2[i];
    if (type == 1) {                       /* MS(lo, hi, d) */
        if (hi - lo <= 64) {
            uint32_t *dst = m->buf[d & 1];
            if (dst != m->buf[0]) memcpy(dst + lo, m->buf[0] + lo, (size_t)(hi - lo) * 4);
            ins_sort(dst + lo, hi - lo);
            tv_finish(m, i);
            return;
        }
        int64_t mid = lo + (hi - lo) / 2;
        if (tv_fork(m, 1, (int32_t)lo, (int32_t)mid, d + 1, 0) < 0) return;
        if (tv_fork(m, 1, (int32_t)mid, (int32_t)hi, d + 1, 0) < 0) return;
        tv_join(m, i, 2, (int32_t)lo, (int32_t)hi, d, 0);
    } else {                               /* MERGE(lo, hi, d) */
        int64_t mid = lo + (hi - lo) / 2;
        merge_into(m->buf[(d + 1) & 1], lo, mid, hi, m->buf[d & 1]);
        tv_finish(m, i);
    }
}

static void body_bfs(orc_tvm *m, int64_t i, int32_t type) {
    (void)type;                            /* VISIT(v) */
    int32_t v = m->a0[i];
    for (int32_t k = m->row_ptr[v]; k < m->row_ptr[v + 1]; ++k) {
        int32_t u = m->col[k];
        if (m->depth[u] == -1) {
            m->depth[u] = m->cen + 1;
            if (tv_fork(m, 1, u, 0, 0, 0) < 0) return;
        }
    }
    tv_finish(m, i);
}

/* SSSP VISIT(v) (Section 6.3's graph workloads, relaxation form): with
 * v's distance as it stands now, lower every out-neighbour's distance that
 * v improves and fork a visit of it; a vertex improved twice is visited
 * twice.  Ends when no distance improves. */
static void body_sssp(orc_tvm *m, int64_t i, int32_t type) {
    (void)type;
    int32_t v = m->a0[i];
    /* With a bucket width delta > 0, a visit whose distance (the one that
     * forked it, a1) is at least (CEN + 1) * delta is not due yet: it forks
     * itself into the next epoch unchanged and relaxes nothing. */
    if (m->p2 > 0 && (int64_t)m->a1[i] >= (int64_t)(m->cen + 1) * m->p2) {
        if (tv_fork(m, 1, v, m->a1[i], 0, 0) < 0) return;
        tv_finish(m, i);
        return;
    }
    const int64_t d = m->depth[v];
    for (int32_t k = m->row_ptr[v]; k < m->row_ptr[v + 1]; ++k) {
        int32_t u = m->col[k];
        const int64_t nd = d + m->wts[k];
        if (nd < m->depth[u]) {
            m->depth[u] = (int32_t)nd;
            if (tv_fork(m, 1, u, (int32_t)nd, 0, 0) < 0) return;
        }
    }
    tv_finish(m, i);
}

/* SSSP's bucket width (before the first epoch; 0 = the plain program). */
void orc_set_delta(orc_tvm *m, int32_t delta) { m->p2 = delta; }

/* Figure 2: postorder(node) forks right then left and joins visitAfter(node). */
static void body_postorder(orc_tvm *m, int64_t i, int32_t type) {
    int32_t node = m->a0[i];
    if (type == 1) {
        if (node < 0) { tv_finish(m, i); return; }
        if (tv_fork(m, 1, m->right[node], 0, 0, 0) < 0) return;
        if (tv_fork(m, 1, m->left[node], 0, 0, 0) < 0) return;
        tv_join(m, i, 2, node, 0, 0, 0);
    } else {
        if (m->visit_log) m->visit_log[m->nvisit] = node;
        if (m->visit_epoch) m->visit_epoch[node] = (int32_t)m->st.epochs;
        m->nvisit++;
        tv_finish(m, i);
    }
}

/* Figure 2: preorder(node) visits node, then forks preorder(right) and
 * preorder(left); nothing joins. */
static void body_preorder(orc_tvm *m, int64_t i) {
    int32_t node = m->a0[i];
    if (node >= 0) {
        if (m->visit_log) m->visit_log[m->nvisit] = node;
        if (m->visit_epoch) m->visit_epoch[node] = (int32_t)m->st.epochs;
        m->nvisit++;
        if (tv_fork(m, 1, m->right[node], 0, 0, 0) < 0) return;
        if (tv_fork(m, 1, m->left[node], 0, 0, 0) < 0) return;
    }
    tv_finish(m, i);
}

/* FFT (Section 6.2): recursive radix-2 decimation in time over N = 2^p0
 * complex values.  FFT(lo, o, ls) transforms the n = N >> ls inputs
 * x[o + j * 2^ls], j < n (the subsequence that recursion level ls reaches),
 * into y[lo, lo + n).  A leaf (n <= 64) writes the DFT of its inputs from the
 * defining sum; otherwise the task forks the even-index half into
 * y[lo, lo + n/2) and the odd-index half into y[lo + n/2, lo + n) and joins
 * COMB(lo, ls), which combines them with one butterfly per k < n/2:
 * y[lo + k] +- exp(-2 pi i k / n) * y[lo + n/2 + k]. */
#define ORC_FFT_LEAF 64
static void dft_strided(const double *x, int64_t o, int64_t s, int64_t n, double *y) {
    for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double a = -2.0 * M_PI * (double)((j * k) % n) / (double)n;
            const double c = cos(a), sn = sin(a);
            const double xr = x[2 * (o + j * s)], xi = x[2 * (o + j * s) + 1];
            sr += xr * c - xi * sn;
            si += xr * sn + xi * c;
        }
        y[2 * k] = sr;
        y[2 * k + 1] = si;
    }
}

static void body_fft(orc_tvm *m, int64_t i, int32_t type) {
    const int32_t lo = m->a0[i], o = m->a1[i], ls = m->a2[i];
    const int64_t n = (int64_t)1 << (m->p0 - ls);
    if (type == 1) {
        if (n <= ORC_FFT_LEAF) {
            dft_strided(m->fx, o, (int64_t)1 << ls, n, m->fy + 2 * (int64_t)lo);
            tv_finish(m, i);
            return;
        }
        if (tv_fork(m, 1, lo, o, ls + 1, 0) < 0) return;
        if (tv_fork(m, 1, (int32_t)(lo + n / 2), o + (1 << ls), ls + 1, 0) < 0) return;
        tv_join(m, i, 2, lo, o, ls, 0);
    } else {
        double *y = m->fy + 2 * (int64_t)lo;
        const int64_t h = n / 2;
        for (int64_t k = 0; k < h; ++k) {
            const double a = -2.0 * M_PI * (double)k / (double)n;
            const double c = cos(a), sn = sin(a);
            const double br = y[2 * (h + k)], bi = y[2 * (h + k) + 1];
            const double tr = br * c - bi * sn, ti = br * sn + bi * c;
            const double ur = y[2 * k], ui = y[2 * k + 1];
            y[2 * k] = ur + tr;           y[2 * k + 1] = ui + ti;
            y[2 * (h + k)] = ur - tr;     y[2 * (h + k) + 1] = ui - ti;
        }
        tv_finish(m, i);
    }
}

/* The DFT of n complex values by its defining sum (the plain definition the
 * FFT program reaches). */
void orc_dft(int64_t n, const double *x, double *y) { dft_strided(x, 0, 1, n, y); }

/* Construction ---------------------------------------------------------------- */

/*
 * kind: ORC_* program.  params:
 *   FIB32/FIB64: p0 = n
 *   NQUEENS:     p0 = n (1..31)
 *   MSORT:       p0 = N; ptr0 = keys (in/out), ptr1 = tmp (N entries)
 *   BFS:         p0 = V, p1 = source; ptr0 = row_ptr, ptr1 = col_idx, ptr2 = depth (out)
 *   POSTORDER,
 *   PREORDER:    p0 = root node (-1 = empty); ptr0 = left, ptr1 = right,
 *                ptr2 = visit log (optional), ptr3 = visit epoch per node (optional)
 *   FFT:         p0 = log2 N (0..24); ptr0 = x, ptr1 = y (2N doubles each)
 * cap: task-vector capacity in entries (0 = unbounded).
 */
orc_tvm *orc_new(int32_t kind, int32_t p0, int32_t p1, void *ptr0, void *ptr1, void *ptr2,
                 void *ptr3, int64_t cap) {
    orc_tvm *m = (orc_tvm *)calloc(1, sizeof(orc_tvm));
    m->kind = kind;
    m->ntt = (kind == ORC_BFS || kind == ORC_SSSP || kind == ORC_PREORDER) ? 1 : 2;
    m->cap = cap;
    m->p0 = p0; m->p1 = p1;
    if (!grow(m, 1)) { m->st.status = ORC_E_OVERFLOW; return m; }
    /* Initialisation (Section 5.2.1): root in entry 0, epoch 0. */
    m->code[0] = 0 * m->ntt + 1;
    switch (kind) {
    case ORC_FIB32: case ORC_FIB64: m->a0[0] = p0; break;
    case ORC_NQUEENS: m->a0[0] = 0; m->a1[0] = m->a2[0] = m->a3[0] = 0; break;
    case ORC_MSORT:
        m->buf[0] = (uint32_t *)ptr0; m->buf[1] = (uint32_t *)ptr1;
        m->a0[0] = 0; m->a1[0] = p0; m->a2[0] = 0;
        break;
    case ORC_BFS:
        m->row_ptr = (const int32_t *)ptr0; m->col = (const int32_t *)ptr1; m->depth = (int32_t *)ptr2;
        for (int32_t v = 0; v < p0; ++v) m->depth[v] = -1;
        m->depth[p1] = 0;
        m->a0[0] = p1;
        break;
    case ORC_POSTORDER: case ORC_PREORDER:
        m->left = (const int32_t *)ptr0; m->right = (const int32_t *)ptr1;
        m->visit_log = (int32_t *)ptr2; m->visit_epoch = (int32_t *)ptr3;
        m->a0[0] = p0;
        break;
    case ORC_SSSP:
        m->row_ptr = (const int32_t *)ptr0; m->col = (const int32_t *)ptr1;
        m->wts = (const int32_t *)ptr2; m->depth = (int32_t *)ptr3;
        for (int32_t v = 0; v < p0; ++v) m->depth[v] = INT32_MAX;
        m->depth[p1] = 0;
        m->a0[0] = p1;
        break;
    case ORC_FFT:
        if (p0 < 0 || p0 > 24) { m->st.status = ORC_E_ARGS; return m; }
        m->fx = (const double *)ptr0; m->fy = (double *)ptr1;
        m->a0[0] = 0; m->a1[0] = 0; m->a2[0] = 0;
        break;
    default: m->st.status = ORC_E_ARGS; return m;
    }
    m->nfc = 1;
    m->st.peak = 1;
    push(m, 0, 0, 1, 1);
    return m;
}

void orc_free(orc_tvm *m) {
    if (!m) return;
    free(m->code); free(m->a0); free(m->a1); free(m->a2); free(m->a3); free(m->r);
    free(m->stk); free(m->recs); free(m);
}

void orc_keep_records(orc_tvm *m, int32_t on) {
    if (on && !m->recs) { m->recs_cap = 64; m->recs = (orc_rec *)malloc(64 * sizeof(orc_rec)); }
}

/*
 * One epoch.  Returns 1 if more epochs remain, 0 when the stacks are empty,
 * negative on error.
 */
int32_t orc_step(orc_tvm *m) {
    if (m->st.status < 0) return m->st.status;
    if (m->sp == 0) return 0;
    /* Phase 1 (Sections 4.3.1, 5.2.2): pop the epoch; remember nextFreeCore. */
    m->sp--;
    int32_t cen = m->stk[m->sp][0], b = m->stk[m->sp][1], e = m->stk[m->sp][2], cend = m->stk[m->sp][3];
    m->cen = cen;
    m->nfc = cend;
    m->old = m->nfc;
    m->joins = 0;
    /* Phase 2 (Sections 4.3.2, 5.2.3): every entry of the range runs. */
    int64_t valid = 0;
    for (int64_t i = b; i < e; ++i) {
        int32_t c = m->code[i];
        if (c == 0) continue;              /* invalid entry: the lane exits */
        int32_t type = c - cen * m->ntt;
        if (type < 1 || type > m->ntt) { m->st.status = ORC_E_ENCODING; return m->st.status; }
        ++valid;
        m->st.tasks_by_type[type - 1]++;
        switch (m->kind) {
        case ORC_FIB32: case ORC_FIB64: body_fib(m, i, type); break;
        case ORC_NQUEENS: body_nqueens(m, i, type); break;
        case ORC_MSORT: body_msort(m, i, type); break;
        case ORC_BFS: body_bfs(m, i, type); break;
        case ORC_POSTORDER: body_postorder(m, i, type); break;
        case ORC_SSSP: body_sssp(m, i, type); break;
        case ORC_PREORDER: body_preorder(m, i); break;
        case ORC_FFT: body_fft(m, i, type); break;
        }
        if (m->st.status < 0) return m->st.status;
    }
    /* Phase 3 (Sections 4.3.3, 5.2.4): joins first, then forks on top. */
    int64_t forks = m->nfc - m->old;
    if (m->joins) push(m, cen, b, e, (int32_t)m->nfc);
    if (forks) push(m, cen + 1, (int32_t)m->old, (int32_t)m->nfc, (int32_t)m->nfc);
    if (m->nfc > m->st.peak) m->st.peak = m->nfc;
    if (m->recs) {
        if (m->nrecs == m->recs_cap) {
            m->recs_cap *= 2;
            m->recs = (orc_rec *)realloc(m->recs, (size_t)m->recs_cap * sizeof(orc_rec));
        }
        orc_rec *q = &m->recs[m->nrecs++];
        q->epoch = (int32_t)m->st.epochs; q->cen = cen; q->b = b; q->e = e;
        q->launched = e - b; q->valid = (int32_t)valid; q->forks = (int32_t)forks;
        q->joins = (int32_t)m->joins; q->nfc = (int32_t)m->nfc;
    }
    m->st.epochs++;
    m->st.tasks += valid;
    m->st.launched += e - b;
    if (m->sp == 0) { m->st.result = m->r[0]; return 0; }
    return 1;
}

/* Run to completion or for at most max_epochs (< 0: no limit). */
int32_t orc_run(orc_tvm *m, int64_t max_epochs) {
    int32_t rc = 1;
    for (int64_t k = 0; (max_epochs < 0 || k < max_epochs) && rc == 1; ++k) rc = orc_step(m);
    return rc;
}

/* Many independent trees in shared global epochs: each global epoch runs one
 * epoch of every tree that is still live.  Returns the number of global
 * epochs executed. */
int64_t orc_run_batch(orc_tvm **ms, int32_t n) {
    int64_t g = 0;
    int32_t live = 1;
    while (live) {
        live = 0;
        int32_t any = 0;
        for (int32_t t = 0; t < n; ++t) {
            if (ms[t]->st.status < 0 || ms[t]->sp == 0) continue;
            any = 1;
            if (orc_step(ms[t]) == 1) live = 1;
        }
        if (any) ++g;
    }
    return g;
}

void orc_get_stats(const orc_tvm *m, orc_stats *out) { *out = m->st; }
int64_t orc_num_records(const orc_tvm *m) { return m->nrecs; }
void orc_get_records(const orc_tvm *m, orc_rec *out) {
    if (m->nrecs) memcpy(out, m->recs, (size_t)m->nrecs * sizeof(orc_rec));
}
int64_t orc_nfc(const orc_tvm *m) { return m->nfc; }
int32_t orc_stack_depth(const orc_tvm *m) { return m->sp; }
int64_t orc_num_visits(const orc_tvm *m) { return m->nvisit; }

/* Checkpoint / resume at an epoch boundary.  The state is exactly the task
 * vector up to the high-water mark, the stack and the counters (Section
 * 4.4.2); the payload arrays are the caller's and are passed again on
 * restore. */
typedef struct {
    int32_t kind, ntt, p0, p1, sp, cen, p2, pad;
    int64_t cap, hw, nfc, nvisit;
    orc_stats st;
} snap_hdr;

int64_t orc_snapshot_size(const orc_tvm *m) {
    int64_t hw = m->st.peak;
    return (int64_t)sizeof(snap_hdr) + hw * (5 * 4 + 8) + (int64_t)m->sp * 16;
}

int64_t orc_snapshot(const orc_tvm *m, void *buf) {
    snap_hdr h;
    memset(&h, 0, sizeof h);
    h.kind = m->kind; h.ntt = m->ntt; h.p0 = m->p0; h.p1 = m->p1; h.sp = m->sp; h.cen = m->cen; h.p2 = m->p2;
    h.cap = m->cap; h.hw = m->st.peak; h.nfc = m->nfc; h.nvisit = m->nvisit; h.st = m->st;
    char *p = (char *)buf;
    memcpy(p, &h, sizeof h); p += sizeof h;
    size_t n4 = (size_t)h.hw * 4;
    memcpy(p, m->code, n4); p += n4;
    memcpy(p, m->a0, n4); p += n4;
    memcpy(p, m->a1, n4); p += n4;
    memcpy(p, m->a2, n4); p += n4;
    memcpy(p, m->a3, n4); p += n4;
    memcpy(p, m->r, (size_t)h.hw * 8); p += (size_t)h.hw * 8;
    memcpy(p, m->stk, (size_t)m->sp * 16); p += (size_t)m->sp * 16;
    return (int64_t)(p - (char *)buf);
}

orc_tvm *orc_restore(const void *buf, void *ptr0, void *ptr1, void *ptr2, void *ptr3) {
    snap_hdr h;
    const char *p = (const char *)buf;
    memcpy(&h, p, sizeof h); p += sizeof h;
    orc_tvm *m = (orc_tvm *)calloc(1, sizeof(orc_tvm));
    m->kind = h.kind; m->ntt = h.ntt; m->p0 = h.p0; m->p1 = h.p1; m->cen = h.cen; m->p2 = h.p2;
    m->cap = h.cap; m->nfc = h.nfc; m->nvisit = h.nvisit; m->st = h.st;
    grow(m, h.hw > 0 ? h.hw : 1);
    size_t n4 = (size_t)h.hw * 4;
    memcpy(m->code, p, n4); p += n4;
    memcpy(m->a0, p, n4); p += n4;
    memcpy(m->a1, p, n4); p += n4;
    memcpy(m->a2, p, n4); p += n4;
    memcpy(m->a3, p, n4); p += n4;
    memcpy(m->r, p, (size_t)h.hw * 8); p += (size_t)h.hw * 8;
    for (int32_t s = 0; s < h.sp; ++s) {
        const int32_t *q = (const int32_t *)(p + 16 * s);
        push(m, q[0], q[1], q[2], q[3]);
    }
    switch (m->kind) {
    case ORC_MSORT: m->buf[0] = (uint32_t *)ptr0; m->buf[1] = (uint32_t *)ptr1; break;
    case ORC_BFS:
        m->row_ptr = (const int32_t *)ptr0; m->col = (const int32_t *)ptr1; m->depth = (int32_t *)ptr2;
        break;
    case ORC_POSTORDER: case ORC_PREORDER:
        m->left = (const int32_t *)ptr0; m->right = (const int32_t *)ptr1;
        m->visit_log = (int32_t *)ptr2; m->visit_epoch = (int32_t *)ptr3;
        break;
    case ORC_SSSP:
        m->row_ptr = (const int32_t *)ptr0; m->col = (const int32_t *)ptr1;
        m->wts = (const int32_t *)ptr2; m->depth = (int32_t *)ptr3;
        break;
    case ORC_FFT: m->fx = (const double *)ptr0; m->fy = (double *)ptr1; break;
    default: break;
    }
    return m;
}
