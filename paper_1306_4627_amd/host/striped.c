/* striped.c -- the paper's parallel method on the host: the c (WT) and b
 * (SYM) tables of section I.C filled by Np OpenMP threads, each owning a
 * stripe of consecutive rows (section II, "block-stripped"), then the walk of
 * section I.D from (m, n).
 *
 * A cell needs its left, upper and upper-left neighbours, so the stripes
 * advance as a wavefront over chunks of columns: thread p fills the columns
 * of chunk q of its stripe once thread p-1 has filled chunk q of the stripe
 * above (whose last row is the row above p's first row).  Each thread
 * publishes the number of chunks it has finished with a release store; the
 * thread below waits for it with acquire loads.  The tables are full
 * (m+1) x (n+1) matrices as in the paper (section II.C: Theta(MN) space).
 *
 * Ties: a mismatch takes UP when c[i-1][j] >= c[i][j-1], else LEFT; a match
 * is always DIAG -- the same canonical walk as every other path here.
 */
#include <omp.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { DIAG = 1, UP = 2, LEFT = 3 };

/* Returns 0 on success, -1 on a bad argument, -3 when the tables do not fit
 * in memory.  *len receives c[m][n]; out (capacity >= min(m, n), may be NULL)
 * the LCS bytes of X in order; *fill_seconds the wall time of the table fill
 * (the parallel section) and *total_seconds fill plus walk. */
int striped_lcs(const uint8_t *x, uint64_t m, const uint8_t *y, uint64_t n, int threads,
                int chunk, uint8_t *out, uint64_t *len, double *fill_seconds,
                double *total_seconds) {
    if ((m && !x) || (n && !y) || !len || threads < 1 || chunk < 1) return -1;
    const double t0 = omp_get_wtime();
    const uint64_t W = n + 1;
    uint32_t *c = (uint32_t *)malloc((m + 1) * W * sizeof(uint32_t));
    uint8_t *b = (uint8_t *)malloc((m + 1) * W);
    if (!c || !b) {
        free(c);
        free(b);
        return -3;
    }
    for (uint64_t j = 0; j <= n; ++j) c[j] = 0;
    for (uint64_t i = 0; i <= m; ++i) c[i * W] = 0;
    int np = threads;
    if ((uint64_t)np > (m ? m : 1)) np = (int)(m ? m : 1);
    const uint64_t nchunks = (n + (uint64_t)chunk - 1) / (uint64_t)chunk;
    atomic_ulong *done = (atomic_ulong *)malloc((size_t)np * sizeof(atomic_ulong));
    if (!done) {
        free(c);
        free(b);
        return -3;
    }
    for (int p = 0; p < np; ++p) atomic_init(&done[p], 0);

#pragma omp parallel num_threads(np)
    {
        const int p = omp_get_thread_num();
        /* rows r0+1 .. r1 of the table */
        const uint64_t r0 = m * (uint64_t)p / (uint64_t)np;
        const uint64_t r1 = m * (uint64_t)(p + 1) / (uint64_t)np;
        for (uint64_t q = 0; q < nchunks; ++q) {
            if (p > 0)
                while (atomic_load_explicit(&done[p - 1], memory_order_acquire) <= q) {
                }
            const uint64_t j0 = q * (uint64_t)chunk + 1;
            const uint64_t j1 = (j0 + (uint64_t)chunk - 1 < n) ? j0 + (uint64_t)chunk - 1 : n;
            for (uint64_t i = r0 + 1; i <= r1; ++i) {
                const uint8_t xi = x[i - 1];
                uint32_t *ci = c + i * W, *cu = c + (i - 1) * W;
                uint8_t *bi = b + i * W;
                for (uint64_t j = j0; j <= j1; ++j) {
                    if (xi == y[j - 1]) {
                        ci[j] = cu[j - 1] + 1;
                        bi[j] = DIAG;
                    } else if (cu[j] >= ci[j - 1]) {
                        ci[j] = cu[j];
                        bi[j] = UP;
                    } else {
                        ci[j] = ci[j - 1];
                        bi[j] = LEFT;
                    }
                }
            }
            atomic_store_explicit(&done[p], q + 1, memory_order_release);
        }
    }
    const double t1 = omp_get_wtime();
    *len = c[m * W + n];
    if (out) {
        uint64_t i = m, j = n, k = c[m * W + n];
        while (i > 0 && j > 0) {
            const uint8_t d = b[i * W + j];
            if (d == DIAG) {
                out[--k] = x[i - 1];
                --i;
                --j;
            } else if (d == UP) {
                --i;
            } else {
                --j;
            }
        }
    }
    const double t2 = omp_get_wtime();
    if (fill_seconds) *fill_seconds = t1 - t0;
    if (total_seconds) *total_seconds = t2 - t0;
    free(done);
    free(c);
    free(b);
    return 0;
}
