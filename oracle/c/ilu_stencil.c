/* Oracle (TEST INFRASTRUCTURE ONLY): ILU(0) and the two substitutions of the
 * paper's one-step preconditioner application, on a matrix whose sparsity
 * pattern NZ(M) is a fixed set of offsets clipped to the grid.
 *
 * Alg. 2 (ILU(0)), Alg. 3 (forward substitution, unit lower L) and Alg. 4
 * (backward substitution, upper U), taken in the paper's order: rows in
 * increasing index, and inside a row the lower columns k in increasing order,
 * each followed by the update of the later columns j of the same row.
 * Reading of Alg. 4: the inner loop runs over j = i+1..n (the printed bound
 * would read z(i) before it is set).
 *
 * Storage: H[row * noff + o] is entry (row, row + offset_o); offsets are
 * listed in column order and include (0,0,0); entries whose column falls
 * outside the grid are never read or written. Plain C99, single thread. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int d, n1, noff, diag;
    const int *off;   /* noff x 3: dx, dy, dz */
} grid_t;

static void coords(const grid_t *g, int64_t row, int c[3]) {
    c[0] = (int)(row % g->n1);
    c[1] = g->d > 1 ? (int)((row / g->n1) % g->n1) : 0;
    c[2] = g->d > 2 ? (int)(row / ((int64_t)g->n1 * g->n1)) : 0;
}

static int in_grid(const grid_t *g, const int c[3], int o, int64_t *col,
                   int64_t row) {
    const int *dd = g->off + 3 * o;
    for (int k = 0; k < g->d; ++k) {
        int v = c[k] + dd[k];
        if (v < 0 || v >= g->n1) return 0;
    }
    int64_t n1 = g->n1;
    *col = row + dd[0] + n1 * dd[1] + n1 * n1 * dd[2];
    return 1;
}

/* lookup cube over offset differences: index of an offset in the list, -1
   if absent; R = half-width of the cube */
static int *offset_cube(const grid_t *g, int *R) {
    int h = 0;
    for (int o = 0; o < g->noff; ++o)
        for (int k = 0; k < 3; ++k) {
            int v = g->off[3 * o + k];
            if (v < 0) v = -v;
            if (v > h) h = v;
        }
    *R = 2 * h;
    int W = 2 * (*R) + 1;
    int *cube = (int *)malloc(sizeof(int) * (size_t)W * W * W);
    for (size_t t = 0; t < (size_t)W * W * W; ++t) cube[t] = -1;
    for (int o = 0; o < g->noff; ++o) {
        const int *dd = g->off + 3 * o;
        cube[((size_t)(dd[2] + *R) * W + (dd[1] + *R)) * W + (dd[0] + *R)] = o;
    }
    return cube;
}

/* Alg. 2 in place on H for rows 0..nrows-1 (nrows < 0: all rows). Rows only
   depend on earlier rows, so a prefix is exactly the same computation as in
   the full factorisation. Returns 0, or 1 + row of the first zero pivot. */
int64_t ilu0_stencil(int d, int n1, int noff, const int *off, double *H, int64_t nrows) {
    grid_t g = {d, n1, noff, -1, off};
    for (int o = 0; o < noff; ++o)
        if (off[3 * o] == 0 && off[3 * o + 1] == 0 && off[3 * o + 2] == 0) g.diag = o;
    if (g.diag < 0) return -1;
    /* pair table: for offsets ok (lower) and oj (after ok in column order),
       the offset of column j relative to row k = off[oj] - off[ok] */
    int R;
    int *cube = offset_cube(&g, &R);
    int W = 2 * R + 1;
    /* for each ok: the later offsets oj (oj > ok) with (k, j) in NZ, and the
       offset index of column j relative to row k (CSR) */
    int64_t *ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(noff + 1));
    int64_t cnt = 0;
    for (int ok = 0; ok < noff; ++ok)
        for (int oj = ok + 1; oj < noff; ++oj) {
            const int *a = off + 3 * oj, *b = off + 3 * ok;
            if (cube[((size_t)(a[2] - b[2] + R) * W + (a[1] - b[1] + R)) * W + (a[0] - b[0] + R)] >= 0) ++cnt;
        }
    int *pj = (int *)malloc(sizeof(int) * (size_t)(cnt + 1));
    int *pkj = (int *)malloc(sizeof(int) * (size_t)(cnt + 1));
    cnt = 0;
    for (int ok = 0; ok < noff; ++ok) {
        ptr[ok] = cnt;
        for (int oj = ok + 1; oj < noff; ++oj) {
            const int *a = off + 3 * oj, *b = off + 3 * ok;
            int v = cube[((size_t)(a[2] - b[2] + R) * W + (a[1] - b[1] + R)) * W + (a[0] - b[0] + R)];
            if (v >= 0) { pj[cnt] = oj; pkj[cnt] = v; ++cnt; }
        }
    }
    ptr[noff] = cnt;
    free(cube);
    int64_t n = 1;
    for (int k = 0; k < d; ++k) n *= n1;
    if (nrows >= 0 && nrows < n) n = nrows;
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        coords(&g, i, c);
        double *Hi = H + i * noff;
        for (int ok = 0; ok < g.diag; ++ok) {          /* k < i in NZ(i) */
            int64_t k;
            if (!in_grid(&g, c, ok, &k, i)) continue;
            double *Hk = H + k * noff;
            double pivot = Hk[g.diag];
            if (pivot == 0.0) { free(ptr); free(pj); free(pkj); return 1 + k; }
            Hi[ok] /= pivot;
            double lik = Hi[ok];
            /* j > k in NZ(i) with (k, j) in NZ; other j have H(k,j) = 0 */
            for (int64_t p = ptr[ok]; p < ptr[ok + 1]; ++p) {
                int64_t j;
                if (!in_grid(&g, c, pj[p], &j, i)) continue;
                Hi[pj[p]] -= lik * Hk[pkj[p]];
            }
        }
    }
    free(ptr); free(pj); free(pkj);
    return 0;
}

/* Alg. 3: L y = r with L unit lower (strict part in H), for rows
   0..nrows-1 (nrows < 0: all rows; a prefix only reads earlier rows). */
void forward_stencil_rows(int d, int n1, int noff, const int *off, const double *H,
                          const double *r, double *y, int64_t nrows) {
    grid_t g = {d, n1, noff, -1, off};
    for (int o = 0; o < noff; ++o)
        if (off[3 * o] == 0 && off[3 * o + 1] == 0 && off[3 * o + 2] == 0) g.diag = o;
    int64_t n = 1;
    for (int k = 0; k < d; ++k) n *= n1;
    if (nrows >= 0 && nrows < n) n = nrows;
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        coords(&g, i, c);
        double acc = 0.0;
        for (int o = 0; o < g.diag; ++o) {
            int64_t j;
            if (!in_grid(&g, c, o, &j, i)) continue;
            acc += H[i * noff + o] * y[j];
        }
        y[i] = r[i] - acc;
    }
}

void forward_stencil(int d, int n1, int noff, const int *off, const double *H,
                     const double *r, double *y) {
    forward_stencil_rows(d, n1, noff, off, H, r, y, -1);
}

/* Alg. 4: U z = y with U upper (diagonal and upper part in H). */
void backward_stencil(int d, int n1, int noff, const int *off, const double *H,
                      const double *y, double *z) {
    grid_t g = {d, n1, noff, -1, off};
    for (int o = 0; o < noff; ++o)
        if (off[3 * o] == 0 && off[3 * o + 1] == 0 && off[3 * o + 2] == 0) g.diag = o;
    int64_t n = 1;
    for (int k = 0; k < d; ++k) n *= n1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int c[3];
        coords(&g, i, c);
        double acc = y[i];
        for (int o = g.diag + 1; o < noff; ++o) {
            int64_t j;
            if (!in_grid(&g, c, o, &j, i)) continue;
            acc -= H[i * noff + o] * z[j];
        }
        z[i] = acc / H[i * noff + g.diag];
    }
}
