/*
 * CPU oracle for the CSRC sparse matrix-vector product -- TEST INFRASTRUCTURE.
 *
 * Plain sequential FP64 C, built with -O2 -ffp-contract=off (no fused
 * multiply-add) so that every product and sum is rounded separately, as in the
 * paper's operation count for machines without FMA (Sec. 4.1).  Nothing here is
 * blocked, fused or reordered.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the GPU library shares no
 * code with it.
 *
 * Format (Sec. 2): A = A_D + A_L + A_U with n x n structurally symmetric A.
 *   ad[i]             diagonal a_ii (0 when not stored)
 *   ia[0..n], ja[k]   row pointers and column indices of the strictly lower
 *                     part, row by row (0-based, ia[0] = 0)
 *   al[k] = a_{i,ja[k]}    lower entry of row i
 *   au[k] = a_{ja[k],i}    its mirror in the upper part (column-wise storage)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * y = A x from the splitting A = A_D + A_L + A_U of Sec. 2, one term after
 * the other, each a plain loop over the stored entries in ascending order:
 *   y   = A_D x          y_i  = ad_i x_i
 *   y  += A_L x          y_i += al_q x_j   for the pair q = (i, j), j < i
 *   y  += A_U x          y_j += au_q x_i   (au_q is a_ji, the mirror of q)
 * The A_U term adds into earlier rows: this is the column-wise traversal of
 * the upper part that CSRC implies.  Every y_i therefore sums, in this
 * order, its diagonal term, its lower products in ascending column and the
 * upper products of the later rows in ascending row.
 */
void oracle_csrc_spmv(int32_t n, const int32_t *ia, const int32_t *ja,
                      const double *ad, const double *al, const double *au,
                      const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = ad[i] * x[i];
    for (int32_t i = 0; i < n; ++i)
        for (int32_t q = ia[i]; q < ia[i + 1]; ++q) y[i] = y[i] + al[q] * x[ja[q]];
    for (int32_t i = 0; i < n; ++i)
        for (int32_t q = ia[i]; q < ia[i + 1]; ++q) y[ja[q]] = y[ja[q]] + au[q] * x[i];
}

/* y = A^T x: A^T = A_D + A_U^T + A_L^T, i.e. the same splitting with the
 * roles of al and au exchanged (Sec. 5). */
void oracle_csrc_spmv_t(int32_t n, const int32_t *ia, const int32_t *ja,
                        const double *ad, const double *al, const double *au,
                        const double *x, double *y)
{
    oracle_csrc_spmv(n, ia, ja, ad, au, al, x, y);
}

/*
 * Y = A X for r right-hand sides stored row-major (X[i*ldx + c]): the
 * product above applied to each column c in turn.
 */
void oracle_csrc_spmm(int32_t n, const int32_t *ia, const int32_t *ja,
                      const double *ad, const double *al, const double *au,
                      int32_t r, const double *X, int64_t ldx, double *Y, int64_t ldy)
{
    for (int32_t c = 0; c < r; ++c) {
#define XC(i) X[(int64_t)(i) * ldx + c]
#define YC(i) Y[(int64_t)(i) * ldy + c]
        for (int32_t i = 0; i < n; ++i) YC(i) = ad[i] * XC(i);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t q = ia[i]; q < ia[i + 1]; ++q) YC(i) = YC(i) + al[q] * XC(ja[q]);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t q = ia[i]; q < ia[i + 1]; ++q) YC(ja[q]) = YC(ja[q]) + au[q] * XC(i);
#undef XC
#undef YC
    }
}

/*
 * Greedy first-fit colouring of the rows (Sec. 3.2), rows visited in ascending
 * index; each row takes the smallest colour used by no earlier row it conflicts
 * with.
 *
 * criterion 0 (write sets): row i writes W(i) = {i} U {ja[k] : k in row i};
 *   rows i and r conflict when W(i) and W(r) intersect.
 * criterion 1 (distance two): rows conflict when adjacent in the pattern graph
 *   (a direct conflict) or when their neighbourhoods in that graph intersect
 *   (the paper's indirect conflicts via a common neighbour).
 *
 * Returns the number of colours, or -1 on allocation failure.
 */
int32_t oracle_csrc_color(int32_t n, const int32_t *ia, const int32_t *ja,
                          int32_t criterion, int32_t *color)
{
    int64_t k = ia[n];
    /* adjacency of the pattern graph (both directions), CSR */
    int64_t *deg = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *mark = malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!deg || !mark) { free(deg); free(mark); return -1; }
    int64_t *ptr = NULL;
    int32_t *adj = NULL;
    int32_t ncolors = 0;

    if (criterion == 0) {
        /* writers[t] = rows whose write set contains t, ascending */
        for (int32_t i = 0; i < n; ++i) {
            deg[i] += 1;
            for (int32_t q = ia[i]; q < ia[i + 1]; ++q) deg[ja[q]] += 1;
        }
        ptr = malloc(sizeof(int64_t) * ((size_t)n + 1));
        adj = malloc(sizeof(int32_t) * ((size_t)(n + k) + 1));
        if (!ptr || !adj) { ncolors = -1; goto done; }
        ptr[0] = 0;
        for (int32_t t = 0; t < n; ++t) ptr[t + 1] = ptr[t] + deg[t];
        for (int32_t t = 0; t < n; ++t) deg[t] = ptr[t];
        for (int32_t i = 0; i < n; ++i) {
            adj[deg[i]++] = i;
            for (int32_t q = ia[i]; q < ia[i + 1]; ++q) adj[deg[ja[q]]++] = i;
        }
        for (int32_t c = 0; c <= n; ++c) mark[c] = -1;
        for (int32_t i = 0; i < n; ++i) {
            /* colours of earlier rows sharing a written entry with row i */
            for (int32_t s = -1; s < ia[i + 1] - ia[i]; ++s) {
                int32_t t = (s < 0) ? i : ja[ia[i] + s];
                for (int64_t p = ptr[t]; p < ptr[t + 1]; ++p) {
                    int32_t r = adj[p];
                    if (r >= i) break;
                    mark[color[r]] = i;
                }
            }
            int32_t c = 0;
            while (mark[c] == i) ++c;
            color[i] = c;
            if (c + 1 > ncolors) ncolors = c + 1;
        }
    } else {
        /* symmetric pattern graph without the diagonal */
        for (int32_t i = 0; i < n; ++i)
            for (int32_t q = ia[i]; q < ia[i + 1]; ++q) { deg[i] += 1; deg[ja[q]] += 1; }
        ptr = malloc(sizeof(int64_t) * ((size_t)n + 1));
        adj = malloc(sizeof(int32_t) * ((size_t)(2 * k) + 1));
        if (!ptr || !adj) { ncolors = -1; goto done; }
        ptr[0] = 0;
        for (int32_t t = 0; t < n; ++t) ptr[t + 1] = ptr[t] + deg[t];
        for (int32_t t = 0; t < n; ++t) deg[t] = ptr[t];
        for (int32_t i = 0; i < n; ++i)
            for (int32_t q = ia[i]; q < ia[i + 1]; ++q) {
                adj[deg[i]++] = ja[q];
                adj[deg[ja[q]]++] = i;
            }
        for (int32_t c = 0; c <= n; ++c) mark[c] = -1;
        for (int32_t i = 0; i < n; ++i) {
            for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
                int32_t v = adj[p];
                if (v < i) mark[color[v]] = i;
                for (int64_t p2 = ptr[v]; p2 < ptr[v + 1]; ++p2) {
                    int32_t w = adj[p2];
                    if (w < i) mark[color[w]] = i;
                }
            }
            int32_t c = 0;
            while (mark[c] == i) ++c;
            color[i] = c;
            if (c + 1 > ncolors) ncolors = c + 1;
        }
    }
done:
    free(deg); free(mark); free(ptr); free(adj);
    return ncolors;
}
