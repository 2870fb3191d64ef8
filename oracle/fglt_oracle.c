/*
 * fglt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, per-vertex CPU evaluation of the fast graphlet transform
 * of Floros, Pitsianis and Sun ("Fast Graphlet Transform of Sparse Graphs").
 * It exists to check the HIP library; nothing in the product path may link
 * or call it.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the HIP library.
 *
 * What it computes, for every selected vertex i of a simple undirected graph
 * given as a canonical CSR (symmetric, rows strictly increasing, no
 * self-loops):
 *   raw[i][k]  = the raw frequency  \hat d_k(i)  of Table I, k = 0..15;
 *   net[i][k]  = the net frequency  d_k(i) = (U16^{-1} \hat f(i))_k, with
 *                U16 the conversion matrix of Table II, applied by
 *                back-substitution.
 *
 * Each raw frequency is the matrix-vector expression of Table I written out
 * as plain loops over rows of A, in the paper's notation:
 *   p1 = A e (degrees), p2 = A p1 - c2 (eq. of p2, with c2 = p1),
 *   C3 = A .* A^2 (Lemma 2), c3 = C3 e / 2,
 *   p3 = A p2 - p1 .* (p1 - 1) - 2 c3 (Lemma 4),
 *   P2 = A^2 - diag(p1) (eq. of P2), C4,2 = P2 .* (P2 - 1) (Lemma 5),
 *   D4,c = A .* (A (C3 - A)), D4,3 = A .* C4,2, T = A .* [q_ij' A q_ij]
 *   (Section IV-C).
 * Every "-" of Table I is the rectified difference max(b - a, 0), as the
 * paper's notation section and the Table I caption define it; it is applied
 * literally through rdiff().  Divisions are taken after the row sums, where
 * they are exact, and are checked.
 *
 * Parity pins (tests/): the paper's worked example (Fig. 2, both tables),
 * brute-force enumeration of every vertex subset of size <= 4 on tiny graphs,
 * closed forms on cliques, stars, cycles and paths, walk identities
 * (A^3)_ii = 2 c3(i) and (A^4)_ii = 2 c4(i) + d_i^2 + p2(i), orbit-sum
 * invariants, and a library triangle count.  Every orbit is pinned.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;
typedef int32_t i32;

#define NORB 16

/* Rectified difference of the paper's notation: max(b - a, 0). */
static inline i64 rdiff(i64 b, i64 a) { return b > a ? b - a : 0; }

/* Table II: the entries of U16 above its unit diagonal, (row, column, value),
 * with U16 f = \hat f. */
static const int U16_UPPER[][3] = {
    {2, 4, 2},  {3, 4, 1},
    {5, 9, 2},  {5, 10, 1}, {5, 12, 2}, {5, 13, 4}, {5, 14, 2}, {5, 15, 6},
    {6, 10, 1}, {6, 11, 2}, {6, 12, 2}, {6, 13, 2}, {6, 14, 4}, {6, 15, 6},
    {7, 9, 1},  {7, 10, 1}, {7, 13, 2}, {7, 14, 1}, {7, 15, 3},
    {8, 11, 1}, {8, 14, 1}, {8, 15, 1},
    {9, 13, 2}, {9, 15, 3},
    {10, 13, 2}, {10, 14, 2}, {10, 15, 6},
    {11, 14, 2}, {11, 15, 3},
    {12, 13, 1}, {12, 14, 1}, {12, 15, 3},
    {13, 15, 3},
    {14, 15, 3},
};
#define U16_NUPPER ((int)(sizeof(U16_UPPER) / sizeof(U16_UPPER[0])))

/* Copies U16 (Table II) into a dense 16x16 row-major array. */
void oracle_u16(i64* u) {
    memset(u, 0, sizeof(i64) * NORB * NORB);
    for (int k = 0; k < NORB; ++k) u[k * NORB + k] = 1;
    for (int t = 0; t < U16_NUPPER; ++t)
        u[U16_UPPER[t][0] * NORB + U16_UPPER[t][1]] = U16_UPPER[t][2];
}

/* f = U16^{-1} \hat f for each of `rows` vectors, by back-substitution on the
 * unit upper-triangular U16: f_k = \hat f_k - sum_{c > k} U16(k, c) f_c. */
void oracle_raw_to_net(i64 rows, const i64* raw, i64* net) {
    i64 u[NORB * NORB];
    oracle_u16(u);
    for (i64 r = 0; r < rows; ++r) {
        const i64* fr = raw + r * NORB;
        i64 f[NORB];
        for (int k = NORB - 1; k >= 0; --k) {
            i64 s = fr[k];
            for (int c = k + 1; c < NORB; ++c) s -= u[k * NORB + c] * f[c];
            f[k] = s;
        }
        memcpy(net + r * NORB, f, sizeof(f));
    }
}

/* |a ∩ b| for two strictly increasing lists. */
static i64 sorted_intersection_size(const i32* a, i64 na, const i32* b, i64 nb) {
    i64 x = 0, y = 0, c = 0;
    while (x < na && y < nb) {
        if (a[x] < b[y]) ++x;
        else if (a[x] > b[y]) ++y;
        else { ++c; ++x; ++y; }
    }
    return c;
}

typedef struct {
    i64* buf;
    i64 len, cap;
} vec64;

static int vpush(vec64* v, i64 x) {
    if (v->len == v->cap) {
        i64 nc = v->cap ? 2 * v->cap : 1024;
        i64* nb = (i64*)realloc(v->buf, (size_t)nc * sizeof(i64));
        if (!nb) return -1;
        v->buf = nb;
        v->cap = nc;
    }
    v->buf[v->len++] = x;
    return 0;
}

typedef struct {
    i32* buf;
    i64 len, cap;
} vec32;

static int vpush32(vec32* v, i32 x) {
    if (v->len == v->cap) {
        i64 nc = v->cap ? 2 * v->cap : 1024;
        i32* nb = (i32*)realloc(v->buf, (size_t)nc * sizeof(i32));
        if (!nb) return -1;
        v->buf = nb;
        v->cap = nc;
    }
    v->buf[v->len++] = x;
    return 0;
}

/*
 * Raw frequencies (Table I) for the vertices sel[0..nsel) of the graph
 * (n, off, idx); raw is nsel x 16, row-major.  If sel is NULL every vertex is
 * selected in order (nsel must equal n).  Returns 0 on success, -1 on memory
 * exhaustion, -2 if a division that must be exact is not (a broken input).
 */
int oracle_raw(i64 n, const i64* off, const i32* idx, i64 nsel, const i64* sel,
               i64* raw, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    const i64 nnz = off[n];
    int status = 0;

    /* Rows whose C3, p2 and c3 are needed: the selected vertices and their
     * neighbours (Table I reads p2, c3 and C3 of neighbours). */
    unsigned char* need = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    i64* p1 = (i64*)malloc(sizeof(i64) * (size_t)(n > 0 ? n : 1));
    i64* p2 = (i64*)calloc((size_t)(n > 0 ? n : 1), sizeof(i64));
    i64* c3 = (i64*)calloc((size_t)(n > 0 ? n : 1), sizeof(i64));
    i64* C3 = (i64*)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(i64));
    if (!need || !p1 || !p2 || !c3 || !C3) { status = -1; goto done; }

    for (i64 i = 0; i < n; ++i) p1[i] = off[i + 1] - off[i];  /* p1 = A e */
    for (i64 s = 0; s < nsel; ++s) {
        i64 i = sel ? sel[s] : s;
        need[i] = 1;
        for (i64 q = off[i]; q < off[i + 1]; ++q) need[idx[q]] = 1;
    }

    /* Pre-pass over the needed rows j:
     *   p2(j) = (A p1)(j) - c2(j) = sum_{k in N(j)} (p1(k) - 1)   [eq. of p2]
     *   C3(j,k) = (A .* A^2)(j,k) = |N(j) ∩ N(k)| for k in N(j)     [Lemma 2]
     *   c3(j) = (C3 e)(j) / 2                                        [Lemma 2] */
#pragma omp parallel
    {
        unsigned char* mark = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
        if (!mark) {
#pragma omp atomic write
            status = -1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (i64 j = 0; j < n; ++j) {
                if (!need[j]) continue;
                i64 ap1 = 0;
                for (i64 q = off[j]; q < off[j + 1]; ++q) ap1 += p1[idx[q]];
                p2[j] = rdiff(ap1, p1[j]);
                for (i64 q = off[j]; q < off[j + 1]; ++q) mark[idx[q]] = 1;
                i64 rowsum = 0;
                for (i64 q = off[j]; q < off[j + 1]; ++q) {
                    i64 k = idx[q], cnt = 0;
                    for (i64 t = off[k]; t < off[k + 1]; ++t) cnt += mark[idx[t]];
                    C3[q] = cnt;
                    rowsum += cnt;
                }
                for (i64 q = off[j]; q < off[j + 1]; ++q) mark[idx[q]] = 0;
                if (rowsum % 2 != 0) {
#pragma omp atomic write
                    status = -2;
                }
                c3[j] = rowsum / 2;
            }
            free(mark);
        }
    }
    if (status) goto done;

    /* Per selected vertex i: Table I row by row. */
#pragma omp parallel
    {
        i64* pos = (i64*)calloc((size_t)(n > 0 ? n : 1), sizeof(i64));  /* 1 + position in N(i), 0 if absent */
        i64* cnt = (i64*)calloc((size_t)(n > 0 ? n : 1), sizeof(i64));  /* P2(i, k) */
        vec64 touched = {0, 0, 0};
        vec32 qbuf = {0, 0, 0};       /* concatenated q_ij = N(i) ∩ N(j) lists */
        i64* qoff = NULL;             /* start of q_ij in qbuf, per neighbour */
        i64 qoff_cap = 0;
        int local_status = (!pos || !cnt) ? -1 : 0;
#pragma omp for schedule(dynamic, 16)
        for (i64 s = 0; s < nsel; ++s) {
            if (local_status) continue;
            const i64 i = sel ? sel[s] : s;
            const i64 b = off[i], e = off[i + 1], di = e - b;
            i64* r = raw + s * NORB;
            for (i64 q = b; q < e; ++q) pos[idx[q]] = 1 + (q - b);

            /* sigma_0, sigma_1, sigma_2, sigma_3, sigma_4 */
            r[0] = 1;                                   /* \hat d_0 = e        */
            r[1] = p1[i];                               /* \hat d_1 = p1       */
            r[2] = p2[i];                               /* \hat d_2 = p2       */
            r[3] = p1[i] * rdiff(p1[i], 1) / 2;         /* p1 .* (p1 - 1) / 2  */
            r[4] = c3[i];                               /* \hat d_4 = c3       */

            /* sigma_5: p3 = A p2 - p1 .* (p1 - 1) - 2 c3   (Lemma 4) */
            i64 ap2 = 0, ac3 = 0, a7 = 0, c3p = 0;
            for (i64 q = b; q < e; ++q) {
                const i64 j = idx[q];
                ap2 += p2[j];
                ac3 += c3[j];
                a7 += rdiff(p1[j], 1) * rdiff(p1[j], 2);   /* (p1 - 1) .* (p1 - 2) */
                c3p += C3[q] * rdiff(p1[j], 2);            /* C3 (p1 - 2)          */
            }
            r[5] = rdiff(rdiff(ap2, p1[i] * rdiff(p1[i], 1)), 2 * c3[i]);
            /* sigma_6: p2 .* (p1 - 1) - 2 c3 */
            r[6] = rdiff(p2[i] * rdiff(p1[i], 1), 2 * c3[i]);
            /* sigma_7: A ((p1 - 1) .* (p1 - 2)) / 2 */
            if (a7 % 2 != 0) local_status = -2;
            r[7] = a7 / 2;
            /* sigma_8: p1 .* (p1 - 1) .* (p1 - 2) / 6 */
            r[8] = p1[i] * rdiff(p1[i], 1) * rdiff(p1[i], 2) / 6;
            /* sigma_9: A c3 - 2 c3 */
            r[9] = rdiff(ac3, 2 * c3[i]);
            /* sigma_10: C3 (p1 - 2) */
            r[10] = c3p;
            /* sigma_11: (p1 - 2) .* c3 */
            r[11] = rdiff(p1[i], 2) * c3[i];

            /* P2(i, k) for k != i: walks i - j - k with j in N(i)   [eq. of P2] */
            touched.len = 0;
            for (i64 q = b; q < e; ++q) {
                const i64 j = idx[q];
                for (i64 t = off[j]; t < off[j + 1]; ++t) {
                    const i64 k = idx[t];
                    if (k == i) continue;
                    if (cnt[k] == 0 && vpush(&touched, k)) local_status = -1;
                    cnt[k] += 1;
                }
            }
            /* sigma_12: c4 = C4,2 e / 2, C4,2 = P2 .* (P2 - 1)      (Lemma 5) */
            i64 c42 = 0;
            for (i64 t = 0; t < touched.len; ++t) {
                const i64 v = cnt[touched.buf[t]];
                c42 += v * rdiff(v, 1);
            }
            /* sigma_14: D4,3 e / 2, D4,3 = A .* C4,2 */
            i64 d43 = 0;
            for (i64 q = b; q < e; ++q) {
                const i64 v = cnt[idx[q]];
                d43 += v * rdiff(v, 1);
            }
            for (i64 t = 0; t < touched.len; ++t) cnt[touched.buf[t]] = 0;
            if (c42 % 2 != 0 || d43 % 2 != 0) local_status = -2;
            r[12] = c42 / 2;
            r[14] = d43 / 2;

            /* sigma_13: D4,c e / 2, D4,c(i, j) = sum_{k in N(i)} (C3 - A)(k, j)
             * for (i, j) in E; (C3 - A)(k, j) is nonzero only on edges (k, j). */
            i64 d4c = 0;
            /* and the lists q_ij = N(i) ∩ N(j) for sigma_15 */
            qbuf.len = 0;
            if (qoff_cap < di + 1) {
                i64* nq = (i64*)realloc(qoff, sizeof(i64) * (size_t)(di + 1));
                if (!nq) { local_status = -1; continue; }
                qoff = nq;
                qoff_cap = di + 1;
            }
            for (i64 q = b; q < e; ++q) {
                const i64 j = idx[q];
                qoff[q - b] = qbuf.len;
                for (i64 t = off[j]; t < off[j + 1]; ++t) {
                    const i64 k = idx[t];
                    if (!pos[k]) continue;        /* k in N(i) ∩ N(j) */
                    d4c += rdiff(C3[t], 1);       /* (C3 - A)(k, j)    */
                    if (vpush32(&qbuf, (i32)k)) local_status = -1;
                }
            }
            qoff[di] = qbuf.len;
            if (d4c % 2 != 0) local_status = -2;
            r[13] = d4c / 2;

            /* sigma_15: T e / 6, T(i, j) = q_ij' A q_ij = sum_{k in q_ij}
             * |N(k) ∩ q_ij|, and N(k) ∩ q_ij = q_ik ∩ q_ij since q_ij ⊆ N(i). */
            i64 te = 0;
            for (i64 q = b; q < e; ++q) {
                const i64 jj = q - b;
                const i32* qj = qbuf.buf + qoff[jj];
                const i64 nqj = qoff[jj + 1] - qoff[jj];
                for (i64 x = 0; x < nqj; ++x) {
                    const i64 kk = pos[qj[x]] - 1;
                    te += sorted_intersection_size(qj, nqj, qbuf.buf + qoff[kk],
                                                   qoff[kk + 1] - qoff[kk]);
                }
            }
            if (te % 6 != 0) local_status = -2;
            r[15] = te / 6;

            for (i64 q = b; q < e; ++q) pos[idx[q]] = 0;
        }
        if (local_status) {
#pragma omp atomic write
            status = local_status;
        }
        free(pos);
        free(cnt);
        free(touched.buf);
        free(qbuf.buf);
        free(qoff);
    }

done:
    free(need);
    free(p1);
    free(p2);
    free(c3);
    free(C3);
    return status;
}

/* Net frequencies for the selected vertices: Table I, then Table II. */
int oracle_net(i64 n, const i64* off, const i32* idx, i64 nsel, const i64* sel,
               i64* net, int nthreads) {
    i64* raw = (i64*)malloc(sizeof(i64) * NORB * (size_t)(nsel > 0 ? nsel : 1));
    if (!raw) return -1;
    int st = oracle_raw(n, off, idx, nsel, sel, raw, nthreads);
    if (st == 0) oracle_raw_to_net(nsel, raw, net);
    free(raw);
    return st;
}

/* ------------------------------------------------------------------ graph */

static int cmp_i32(const void* a, const void* b) {
    const i32 x = *(const i32*)a, y = *(const i32*)b;
    return (x > y) - (x < y);
}

/*
 * The adjacency of the simple undirected graph on n vertices spanned by the
 * m pairs (src[t], dst[t]) (Section I's graph model): both directions of each
 * pair, self-loops and duplicates dropped, rows sorted.  The definition, in
 * three plain steps for sizes where the numpy route is too slow: every entry
 * is placed in its row, each row is sorted and its repeats are dropped, then
 * the rows are packed.  off (n + 1 entries) and idx (2 m entries, of which
 * off[n] are used) are the caller's.  Returns 0, or -3 for an id outside
 * [0, n), -1 on memory exhaustion.
 */
int oracle_canonical_csr(i64 n, i64 m, const i32* src, const i32* dst, i64* off, i32* idx, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int status = 0;
#pragma omp parallel for schedule(static)
    for (i64 t = 0; t < m; ++t)
        if (src[t] < 0 || src[t] >= n || dst[t] < 0 || dst[t] >= n) {
#pragma omp atomic write
            status = -3;
        }
    if (status) return status;
    i64* fill = (i64*)calloc((size_t)(n + 1), sizeof(i64));
    if (!fill) return -1;
    /* entries per row, both directions, no self-loops */
#pragma omp parallel for schedule(static)
    for (i64 t = 0; t < m; ++t) {
        if (src[t] == dst[t]) continue;
#pragma omp atomic
        fill[src[t]] += 1;
#pragma omp atomic
        fill[dst[t]] += 1;
    }
    off[0] = 0;
    for (i64 i = 0; i < n; ++i) off[i + 1] = off[i] + fill[i];
    for (i64 i = 0; i < n; ++i) fill[i] = off[i];
    /* every entry into its row (in no particular order within the row) */
#pragma omp parallel for schedule(static)
    for (i64 t = 0; t < m; ++t) {
        if (src[t] == dst[t]) continue;
        i64 a, b;
#pragma omp atomic capture
        a = fill[src[t]]++;
#pragma omp atomic capture
        b = fill[dst[t]]++;
        idx[a] = dst[t];
        idx[b] = src[t];
    }
    /* sort each row and drop its repeats; fill[i] = the row's distinct count */
#pragma omp parallel for schedule(dynamic, 1024)
    for (i64 i = 0; i < n; ++i) {
        i32* r = idx + off[i];
        const i64 len = off[i + 1] - off[i];
        qsort(r, (size_t)len, sizeof(i32), cmp_i32);
        i64 k = 0;
        for (i64 q = 0; q < len; ++q)
            if (k == 0 || r[q] != r[k - 1]) r[k++] = r[q];
        fill[i] = k;
    }
    /* pack the rows to the front, in row order */
    i64 pos = 0;
    for (i64 i = 0; i < n; ++i) {
        const i64 b = off[i], k = fill[i];
        off[i] = pos;
        if (pos != b) memmove(idx + pos, idx + b, sizeof(i32) * (size_t)k);
        pos += k;
    }
    off[n] = pos;
    free(fill);
    return 0;
}

/* Number of threads OpenMP will use by default. */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
