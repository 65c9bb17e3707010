/*
 * lcs_oracle.c -- plain CPU reference for the longest-common-subsequence
 * dynamic program of Dash & Nayak, "Parallel Algorithm for Longest Common
 * Subsequence in a String" (arXiv:1306.4627).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or helper
 * with the HIP library and must never be linked into it.
 *
 * What it computes (paper section I.C, procedure LCS-length; section I.D,
 * procedure Print-LCS):
 *
 *   c[i][0] = c[0][j] = 0                       (borders, including c[0][0])
 *   for i = 1..m (outer), j = 1..n (inner)      (row-major order)
 *     if x_i == y_j:              c = c[i-1][j-1] + 1,  b = DIAG
 *     else if c[i-1][j] >= c[i][j-1]: c = c[i-1][j],    b = UP
 *     else:                       c = c[i][j-1],        b = LEFT
 *   length = c[m][n]
 *
 *   traceback: start at (m, n); while i > 0 and j > 0:
 *     DIAG -> emit x_i, (i-1, j-1);  UP -> (i-1, j);  LEFT -> (i, j-1)
 *   the emitted symbols come out last-first and are reversed.
 *
 * Readings taken where the printed text is garbled (each one is listed with
 * its reason in the design notes of the repository):
 *   - the double loop over (i, j) is missing from the printed procedure; the
 *     text says the table is filled in row-major order, so i is the outer loop;
 *   - the border loops start at 1, so c[0][0] is never set; it is 0;
 *   - the UP branch of Print-LCS is printed as two recursive calls; the
 *     textbook procedure the paper cites moves to (i-1, j) on UP and to
 *     (i, j-1) on LEFT, which is what is implemented;
 *   - the recursion of Print-LCS is written as an iterative walk (same visit
 *     order, no recursion depth limit).
 *
 * Symbols are compared as raw bytes.  Row index i runs over X, column index j
 * over Y.  All functions are single-threaded and re-entrant.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DIAG 1
#define ORC_UP 2
#define ORC_LEFT 3

/* Fill the full tables (section I.C).  c must hold (m+1)*(n+1) uint32 values,
 * row-major with row stride n+1; b must hold (m+1)*(n+1) bytes with the same
 * indexing (row 0 and column 0 of b are set to 0 and never read).
 * Returns c[m][n]. */
uint32_t oracle_lcs_table(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n,
                          uint32_t *c, uint8_t *b)
{
    const int64_t S = n + 1;
    for (int64_t i = 0; i <= m; ++i) { c[i * S + 0] = 0; b[i * S + 0] = 0; }
    for (int64_t j = 0; j <= n; ++j) { c[0 * S + j] = 0; b[0 * S + j] = 0; }
    for (int64_t i = 1; i <= m; ++i) {
        for (int64_t j = 1; j <= n; ++j) {
            if (x[i - 1] == y[j - 1]) {
                c[i * S + j] = c[(i - 1) * S + (j - 1)] + 1;
                b[i * S + j] = ORC_DIAG;
            } else if (c[(i - 1) * S + j] >= c[i * S + (j - 1)]) {
                c[i * S + j] = c[(i - 1) * S + j];
                b[i * S + j] = ORC_UP;
            } else {
                c[i * S + j] = c[i * S + (j - 1)];
                b[i * S + j] = ORC_LEFT;
            }
        }
    }
    return c[m * S + n];
}

/* Walk the b table from (m, n) (section I.D) and write the LCS, in forward
 * order, to out (capacity >= min(m, n)).  Returns the number of symbols. */
int64_t oracle_print_lcs(const uint8_t *b, const uint8_t *x, int64_t m, int64_t n,
                         uint8_t *out)
{
    const int64_t S = n + 1;
    int64_t i = m, j = n, k = 0;
    while (i > 0 && j > 0) {
        uint8_t a = b[i * S + j];
        if (a == ORC_DIAG) { out[k++] = x[i - 1]; --i; --j; }
        else if (a == ORC_UP) { --i; }
        else { --j; }
    }
    for (int64_t p = 0, q = k - 1; p < q; ++p, --q) {
        uint8_t t = out[p]; out[p] = out[q]; out[q] = t;
    }
    return k;
}

/* Length only: the same recurrence in the same row-major order, keeping only
 * the previous row of c (the arithmetic is unchanged; only storage differs).
 * Returns c[m][n], or -1 when memory cannot be allocated. */
int64_t oracle_lcs_length(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n)
{
    if (m == 0 || n == 0) return 0;
    uint32_t *prev = (uint32_t *)calloc((size_t)(n + 1), sizeof(uint32_t));
    uint32_t *cur = (uint32_t *)calloc((size_t)(n + 1), sizeof(uint32_t));
    if (!prev || !cur) { free(prev); free(cur); return -1; }
    for (int64_t i = 1; i <= m; ++i) {
        cur[0] = 0;
        for (int64_t j = 1; j <= n; ++j) {
            if (x[i - 1] == y[j - 1]) cur[j] = prev[j - 1] + 1;
            else if (prev[j] >= cur[j - 1]) cur[j] = prev[j];
            else cur[j] = cur[j - 1];
        }
        uint32_t *t = prev; prev = cur; cur = t;
    }
    int64_t L = prev[n];
    free(prev); free(cur);
    return L;
}

/* Full-table traceback: fill c and b, then walk.  Returns the length, or -1
 * when the tables cannot be allocated. */
int64_t oracle_lcs_traceback(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n,
                             uint8_t *out)
{
    if (m == 0 || n == 0) return 0;
    size_t cells = (size_t)(m + 1) * (size_t)(n + 1);
    uint32_t *c = (uint32_t *)malloc(cells * sizeof(uint32_t));
    uint8_t *b = (uint8_t *)malloc(cells);
    if (!c || !b) { free(c); free(b); return -1; }
    oracle_lcs_table(x, m, y, n, c, b);
    int64_t k = oracle_print_lcs(b, x, m, n, out);
    free(c); free(b);
    return k;
}

/* Checkpointed-row traceback for tables too large to hold.
 *
 * Forward: the recurrence above, row by row, storing row i of c for every i
 * that is a multiple of R (row 0 included).  Backward: the walk of section
 * I.D needs b[i][j] only for rows at or below the current i.  For the row
 * block (i0, i1] that holds the current i (i0 = the checkpoint below), rows
 * i0+1..i1 of c and b are recomputed from checkpoint row i0 with the same
 * recurrence, and the walk proceeds inside the block until i drops to i0;
 * then the next block down is recomputed.  The b entries produced are the
 * ones the full table holds (same recurrence, same inputs), so the walk and
 * its output are identical to oracle_lcs_traceback.
 *
 * Memory: (m/R + 1) * (n+1) uint32 for checkpoints plus R * (n+1) uint32 and
 * R * (n+1) bytes for one block.  Returns the length, -1 on allocation
 * failure, -2 for R < 1. */
int64_t oracle_lcs_traceback_ckpt(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n,
                                  int64_t R, uint8_t *out)
{
    if (R < 1) return -2;
    if (m == 0 || n == 0) return 0;
    const int64_t S = n + 1;
    const int64_t nck = m / R + 1;
    uint32_t *ck = (uint32_t *)malloc((size_t)nck * (size_t)S * sizeof(uint32_t));
    uint32_t *row = (uint32_t *)calloc((size_t)S, sizeof(uint32_t));
    uint32_t *nxt = (uint32_t *)calloc((size_t)S, sizeof(uint32_t));
    uint32_t *bc = (uint32_t *)malloc((size_t)(R + 1) * (size_t)S * sizeof(uint32_t));
    uint8_t *bb = (uint8_t *)malloc((size_t)(R + 1) * (size_t)S);
    if (!ck || !row || !nxt || !bc || !bb) {
        free(ck); free(row); free(nxt); free(bc); free(bb);
        return -1;
    }
    /* forward pass: row 0 is all zero */
    memcpy(ck, row, (size_t)S * sizeof(uint32_t));
    for (int64_t i = 1; i <= m; ++i) {
        nxt[0] = 0;
        for (int64_t j = 1; j <= n; ++j) {
            if (x[i - 1] == y[j - 1]) nxt[j] = row[j - 1] + 1;
            else if (row[j] >= nxt[j - 1]) nxt[j] = row[j];
            else nxt[j] = nxt[j - 1];
        }
        uint32_t *t = row; row = nxt; nxt = t;
        if (i % R == 0) memcpy(ck + (i / R) * S, row, (size_t)S * sizeof(uint32_t));
    }
    /* backward pass */
    int64_t i = m, j = n, k = 0;
    while (i > 0 && j > 0) {
        int64_t i0 = ((i - 1) / R) * R;   /* checkpoint row strictly below i */
        int64_t i1 = i;                   /* rows needed: i0+1 .. i */
        /* local row r = i - i0, r = 0 is the checkpoint row */
        memcpy(bc, ck + (i0 / R) * S, (size_t)S * sizeof(uint32_t));
        for (int64_t r = 1; r <= i1 - i0; ++r) {
            int64_t gi = i0 + r;
            uint32_t *cp = bc + (r - 1) * S, *cc = bc + r * S;
            uint8_t *br = bb + r * S;
            cc[0] = 0; br[0] = 0;
            for (int64_t jj = 1; jj <= n; ++jj) {
                if (x[gi - 1] == y[jj - 1]) { cc[jj] = cp[jj - 1] + 1; br[jj] = ORC_DIAG; }
                else if (cp[jj] >= cc[jj - 1]) { cc[jj] = cp[jj]; br[jj] = ORC_UP; }
                else { cc[jj] = cc[jj - 1]; br[jj] = ORC_LEFT; }
            }
        }
        while (i > i0 && j > 0) {
            uint8_t a = bb[(i - i0) * S + j];
            if (a == ORC_DIAG) { out[k++] = x[i - 1]; --i; --j; }
            else if (a == ORC_UP) { --i; }
            else { --j; }
        }
    }
    for (int64_t p = 0, q = k - 1; p < q; ++p, --q) {
        uint8_t t = out[p]; out[p] = out[q]; out[q] = t;
    }
    free(ck); free(row); free(nxt); free(bc); free(bb);
    return k;
}
