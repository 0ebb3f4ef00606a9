/*
 * Oracle: plain, slow, element-level FP64 reference for the selected-inversion
 * hot path of "GPU-Accelerated Parallel Selected Inversion for Structured
 * Matrices Using sTiles" (Fattah, Ltaief, Rue, Keyes; arXiv 2504.19171).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file: only tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the HIP path.
 *
 * What it computes (all IEEE binary64, round to nearest, no tiles in the
 * arithmetic):
 *   1. A = L L^T, the Cholesky factor of a symmetric positive-definite
 *      band-plus-arrowhead matrix (Sec. III, opening paragraph; the arrowhead
 *      shape of Sec. I and Sec. IV-A: a band of half-width w over the first
 *      nb = n - a rows and columns, plus a rows/columns that are dense).
 *   2. log det A = 2 * sum_j log L_jj (textbook identity; the paper itself
 *      does not compute it).
 *   3. Sigma = A^{-1} on the tile pattern of L (Sec. III-B, "case 7": the
 *      selected tiles are the non-zero tiles of the Cholesky factor, and whole
 *      tiles are computed), by the element form of the backward recurrence that
 *      follows from L^T Sigma = L^{-1} (Sec. III-A; Takahashi's formula, ref. in
 *      Sec. II).  For column j and every selected row i >= j:
 *          Sigma_ij = ( [i == j] / L_jj  -  sum_{k > j} Sigma_ik L_kj ) / L_jj,
 *      where the sum runs over the non-zeros k of column j of L.  It reaches
 *      the same numbers as the tile relations printed in Sec. III-A (e.g.
 *      Sigma_21 = -Sigma_22 L_21 L_11^{-1}) written for 1 x 1 tiles.
 *   4. Single columns of Sigma = A^{-1} by two triangular solves with L (the
 *      plain definition A Sigma e_j = e_j), for sampled checks at sizes where
 *      the full recurrence is too slow.
 *
 * Storage used by the oracle (element level, all row-major, 0-based):
 *   input A ("canonical band form", shared with the input generator):
 *     ab[d*nb + j] = A[j+d][j]           0 <= d <= w, j+d < nb   (lower band)
 *     P [r*nb + j] = A[nb+r][j]          0 <= r < a,  j < nb     (arrow rows)
 *     C [r*a  + c] = A[nb+r][nb+c]       lower triangle read     (corner)
 *   factor L (same index space, own row-oriented band):
 *     Lr[i*(w+1) + t] = L[i][i-w+t]      t = 0..w, t == w is the diagonal
 *     LP[r*nb + k]    = L[nb+r][k]
 *     LC[r*a + c]     = L[nb+r][nb+c]    c <= r, upper triangle set to 0
 *   selected inverse Sigma (output):
 *     Sb[d*nb + j] = Sigma[j+d][j]       0 <= d <= Wp, rows inside the tile
 *                                        pattern of column j, others 0
 *     SP[r*nb + j] = Sigma[nb+r][j]
 *     SC[r*a + c]  = Sigma[nb+r][nb+c]   full symmetric
 *   Tile pattern (tile size b, tile half-bandwidth Bt = ceil(w/b), capped at
 *   N-1 with N = ceil(nb/b)): for a band column j in tile J = j / b the
 *   selected band rows are j .. min(nb-1, (J+Bt+1)*b - 1); Wp = (Bt+1)*b - 1 is
 *   the largest offset d stored in Sb.  All arrow rows are selected in every
 *   column, and the corner is selected whole.
 *
 * The half-bandwidth passed to these functions must be at most max(nb-1, 0);
 * a wider band is the same matrix, and callers clamp it first.
 *
 * Return codes: 0 = success; k > 0 = the pivot of global column k (1-based) is
 * not positive (or NaN), as LAPACK's potrf reports it; -1 = bad argument;
 * -2 = out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

static i64 imin(i64 x, i64 y) { return x < y ? x : y; }
static i64 imax(i64 x, i64 y) { return x > y ? x : y; }

/* Neumaier (improved Kahan) compensated summation step. */
static void neumaier_add(double* sum, double* comp, double x) {
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

/* A[i][j] for i >= j read from the canonical band form. */
static double a_entry(i64 nb, i64 w, i64 a, const double* ab, const double* P,
                      const double* C, i64 i, i64 j) {
    if (i < nb) {
        i64 d = i - j;
        return (d <= w) ? ab[d * nb + j] : 0.0;
    }
    if (j < nb) return P[(i - nb) * nb + j];
    return C[(i - nb) * a + (j - nb)];
}

/* L[i][k] for a band row i (k <= i); zero outside the band. */
static double l_band(i64 w, const double* Lr, i64 i, i64 k) {
    i64 t = k - (i - w);
    return (t >= 0 && k <= i) ? Lr[i * (w + 1) + t] : 0.0;
}

/*
 * Cholesky factorization A = L L^T, column by column (left-looking):
 *   L_jj = sqrt(A_jj - sum_{k<j} L_jk^2)
 *   L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj      for i > j
 * with the sums restricted to the non-zeros of the rows involved (the band has
 * no fill outside itself, the arrow rows are dense).  Rows i of one column are
 * independent, so they are computed in parallel.
 */
int oracle_cholesky(i64 nb, i64 w, i64 a, const double* ab, const double* P,
                    const double* C, double* Lr, double* LP, double* LC,
                    double* logdet) {
    if (nb < 0 || a < 0 || w < 0 || (nb + a) < 1) return -1;
    if (nb > 0 && w > nb - 1) return -1; /* callers clamp w to nb-1 first */
    memset(Lr, 0, sizeof(double) * (size_t)(nb * (w + 1)));
    if (a > 0) {
        memset(LP, 0, sizeof(double) * (size_t)(a * nb));
        memset(LC, 0, sizeof(double) * (size_t)(a * a));
    }
    double ld_sum = 0.0, ld_comp = 0.0;
    int info = 0;

    /* Band columns. */
    for (i64 j = 0; j < nb && !info; ++j) {
        i64 k0 = imax(0, j - w);
        double s = a_entry(nb, w, a, ab, P, C, j, j);
        for (i64 k = k0; k < j; ++k) {
            double l = Lr[j * (w + 1) + (k - (j - w))];
            s -= l * l;
        }
        if (!(s > 0.0)) { info = (int)(j + 1); break; }
        double ljj = sqrt(s);
        Lr[j * (w + 1) + w] = ljj;
        neumaier_add(&ld_sum, &ld_comp, 2.0 * log(ljj));

        i64 iend = imin(nb - 1, j + w);
#pragma omp parallel for schedule(static)
        for (i64 i = j + 1; i <= iend; ++i) {
            double t = a_entry(nb, w, a, ab, P, C, i, j);
            i64 kk0 = imax(0, i - w); /* row i is zero before i-w */
            for (i64 k = kk0; k < j; ++k)
                t -= Lr[i * (w + 1) + (k - (i - w))] * Lr[j * (w + 1) + (k - (j - w))];
            Lr[i * (w + 1) + (j - (i - w))] = t / ljj;
        }
#pragma omp parallel for schedule(static)
        for (i64 r = 0; r < a; ++r) {
            double t = P[r * nb + j];
            for (i64 k = k0; k < j; ++k)
                t -= LP[r * nb + k] * Lr[j * (w + 1) + (k - (j - w))];
            LP[r * nb + j] = t / ljj;
        }
    }

    /* Corner columns: the trailing a x a block, dense. */
    for (i64 c = 0; c < a && !info; ++c) {
        double s = C[c * a + c];
        for (i64 k = 0; k < nb; ++k) s -= LP[c * nb + k] * LP[c * nb + k];
        for (i64 k = 0; k < c; ++k) s -= LC[c * a + k] * LC[c * a + k];
        if (!(s > 0.0)) { info = (int)(nb + c + 1); break; }
        double lcc = sqrt(s);
        LC[c * a + c] = lcc;
        neumaier_add(&ld_sum, &ld_comp, 2.0 * log(lcc));
#pragma omp parallel for schedule(static)
        for (i64 r = c + 1; r < a; ++r) {
            double t = C[r * a + c];
            for (i64 k = 0; k < nb; ++k) t -= LP[r * nb + k] * LP[c * nb + k];
            for (i64 k = 0; k < c; ++k) t -= LC[r * a + k] * LC[c * a + k];
            LC[r * a + c] = t / lcc;
        }
    }
    if (logdet) *logdet = info ? NAN : ld_sum + ld_comp;
    return info;
}

/* Tile-pattern geometry shared by the functions below. */
typedef struct {
    i64 nb, w, a, b, nt, bt, wp;
} geom_t;

static int make_geom(i64 nb, i64 w, i64 a, i64 b, geom_t* g) {
    if (nb < 0 || w < 0 || a < 0 || b < 1 || nb + a < 1) return -1;
    g->nb = nb; g->w = w; g->a = a; g->b = b;
    g->nt = (nb + b - 1) / b;
    i64 bt = (w + b - 1) / b;
    if (g->nt > 0 && bt > g->nt - 1) bt = g->nt - 1;
    if (g->nt == 0) bt = 0;
    g->bt = bt;
    g->wp = (bt + 1) * b - 1;
    return 0;
}

/* Last selected band row of band column j (tile pattern of L, whole tiles). */
static i64 env_last(const geom_t* g, i64 j) {
    i64 J = j / g->b;
    return imin(g->nb - 1, (J + g->bt + 1) * g->b - 1);
}

i64 oracle_sigma_band_rows(i64 nb, i64 w, i64 a, i64 b) {
    geom_t g;
    if (make_geom(nb, w, a, b, &g)) return -1;
    return g.wp + 1;
}

/*
 * Selected inverse on the tile pattern of L by the backward recurrence
 * (Sec. III-A, L^T Sigma = L^{-1}):
 *   for j = n-1 down to 0:
 *     for selected i > j:  Sigma_ij = -(1/L_jj) sum_{k in nz(j), k > j} Sigma_ik L_kj
 *     then                 Sigma_jj = 1/L_jj^2 - (1/L_jj) sum_{k in nz(j), k > j} Sigma_kj L_kj
 * nz(j) = rows of the non-zeros of column j of L: j+1..min(j+w, nb-1) plus all
 * arrow rows for a band column; j+1..n-1 for a corner column.  Every Sigma_ik
 * the sum needs lies in the tile pattern (it is closed under the recurrence),
 * so no entry outside the pattern is ever formed.
 *
 * Internally Sigma's band part is kept as full symmetric rows
 * W[i][t] = Sigma[i][i - Wp + t], t in [0, 2 Wp], so that Sigma_ik is read the
 * same way for k < i and k > i; it is copied to Sb at the end.
 */
int oracle_selinv(i64 nb, i64 w, i64 a, i64 b, const double* Lr, const double* LP,
                  const double* LC, double* Sb, double* SP, double* SC) {
    geom_t g;
    if (make_geom(nb, w, a, b, &g)) return -1;
    const i64 wp = g.wp, wrow = 2 * wp + 1;
    double* W = NULL;
    if (nb > 0) {
        W = (double*)calloc((size_t)(nb * wrow), sizeof(double));
        if (!W) return -2;
    }
    double* lcol = (double*)malloc(sizeof(double) * (size_t)(w + a + 1 + (a > 0 ? a : 0)));
    if (!lcol) { free(W); return -2; }
    if (a > 0) {
        memset(SP, 0, sizeof(double) * (size_t)(a * nb));
        memset(SC, 0, sizeof(double) * (size_t)(a * a));
    }
#define SIGW(i, k) W[(i) * wrow + ((k) - (i) + wp)]

    /* Corner columns (dense block, no band coupling below it). */
    for (i64 c = a - 1; c >= 0; --c) {
        double lcc = LC[c * a + c];
        /* rows r > c of the corner */
#pragma omp parallel for schedule(static)
        for (i64 r = c + 1; r < a; ++r) {
            double s = 0.0;
            for (i64 k = c + 1; k < a; ++k) s += SC[r * a + k] * LC[k * a + c];
            double v = -s / lcc;
            SC[r * a + c] = v;
            SC[c * a + r] = v;
        }
        double s = 0.0;
        for (i64 k = c + 1; k < a; ++k) s += SC[k * a + c] * LC[k * a + c];
        SC[c * a + c] = 1.0 / (lcc * lcc) - s / lcc;
    }

    /* Band columns, last to first. */
    for (i64 j = nb - 1; j >= 0; --j) {
        double ljj = Lr[j * (w + 1) + w];
        i64 kend = imin(nb - 1, j + w);  /* band non-zeros of column j: j+1..kend */
        i64 nbk = kend - j;
        for (i64 t = 0; t < nbk; ++t) lcol[t] = l_band(w, Lr, j + 1 + t, j);
        for (i64 r = 0; r < a; ++r) lcol[nbk + r] = LP[r * nb + j];
        i64 ilast = env_last(&g, j);

        /* selected band rows i > j */
#pragma omp parallel for schedule(static)
        for (i64 i = j + 1; i <= ilast; ++i) {
            double s = 0.0;
            for (i64 t = 0; t < nbk; ++t) s += SIGW(i, j + 1 + t) * lcol[t];
            for (i64 r = 0; r < a; ++r) s += SP[r * nb + i] * lcol[nbk + r];
            double v = -s / ljj;
            SIGW(i, j) = v;
            SIGW(j, i) = v;
        }
        /* arrow rows */
#pragma omp parallel for schedule(static)
        for (i64 r2 = 0; r2 < a; ++r2) {
            double s = 0.0;
            for (i64 t = 0; t < nbk; ++t) s += SP[r2 * nb + (j + 1 + t)] * lcol[t];
            for (i64 r = 0; r < a; ++r) s += SC[r2 * a + r] * lcol[nbk + r];
            SP[r2 * nb + j] = -s / ljj;
        }
        /* diagonal */
        double s = 0.0;
        for (i64 t = 0; t < nbk; ++t) s += SIGW(j + 1 + t, j) * lcol[t];
        for (i64 r = 0; r < a; ++r) s += SP[r * nb + j] * lcol[nbk + r];
        SIGW(j, j) = 1.0 / (ljj * ljj) - s / ljj;
    }

    /* Copy the band part out: Sb[d][j] = Sigma[j+d][j] inside the pattern. */
    if (nb > 0) memset(Sb, 0, sizeof(double) * (size_t)((wp + 1) * nb));
    for (i64 j = 0; j < nb; ++j) {
        i64 ilast = env_last(&g, j);
        for (i64 i = j; i <= ilast; ++i) Sb[(i - j) * nb + j] = SIGW(i, j);
    }
#undef SIGW
    free(lcol);
    free(W);
    return 0;
}

/*
 * Column j of Sigma = A^{-1}, by the definition A x = e_j solved with the
 * oracle's own factor: L y = e_j (forward), then L^T x = y (backward).  Used to
 * check sampled entries at sizes where the full recurrence is too slow.
 * x has length n = nb + a.
 */
int oracle_sigma_column(i64 nb, i64 w, i64 a, const double* Lr, const double* LP,
                        const double* LC, i64 j, double* x) {
    i64 n = nb + a;
    if (j < 0 || j >= n) return -1;
    double* y = (double*)calloc((size_t)n, sizeof(double));
    if (!y) return -2;
    /* forward: L y = e_j */
    for (i64 i = 0; i < nb; ++i) {
        double s = (i == j) ? 1.0 : 0.0;
        for (i64 k = imax(0, i - w); k < i; ++k) s -= Lr[i * (w + 1) + (k - (i - w))] * y[k];
        y[i] = s / Lr[i * (w + 1) + w];
    }
    for (i64 r = 0; r < a; ++r) {
        i64 i = nb + r;
        double s = (i == j) ? 1.0 : 0.0;
        for (i64 k = 0; k < nb; ++k) s -= LP[r * nb + k] * y[k];
        for (i64 k = 0; k < r; ++k) s -= LC[r * a + k] * y[nb + k];
        y[i] = s / LC[r * a + r];
    }
    /* backward: L^T x = y */
    for (i64 r = a - 1; r >= 0; --r) {
        double s = y[nb + r];
        for (i64 k = r + 1; k < a; ++k) s -= LC[k * a + r] * x[nb + k];
        x[nb + r] = s / LC[r * a + r];
    }
    for (i64 i = nb - 1; i >= 0; --i) {
        double s = y[i];
        i64 kend = imin(nb - 1, i + w);
        for (i64 k = i + 1; k <= kend; ++k) s -= Lr[k * (w + 1) + (i - (k - w))] * x[k];
        for (i64 r = 0; r < a; ++r) s -= LP[r * nb + i] * x[nb + r];
        x[i] = s / Lr[i * (w + 1) + w];
    }
    free(y);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
