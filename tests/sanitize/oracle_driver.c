/*
 * Test driver for a sanitizer build of the oracle (address and undefined
 * behaviour checks on the host; test infrastructure only).
 *
 * Reads one matrix in the oracle's canonical band form from a binary file
 * (int64 nb, w, a, b, then ab [(w+1) nb], P [a nb], C [a a] as doubles),
 * runs oracle_cholesky, oracle_selinv and oracle_sigma_column on every column,
 * and writes log det, info, L, Sigma and the columns to the output file, so
 * the caller can compare them with the ordinary build's results.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef int64_t i64;
int oracle_cholesky(i64 nb, i64 w, i64 a, const double* ab, const double* P, const double* C, double* Lr,
                    double* LP, double* LC, double* logdet);
i64 oracle_sigma_band_rows(i64 nb, i64 w, i64 a, i64 b);
int oracle_selinv(i64 nb, i64 w, i64 a, i64 b, const double* Lr, const double* LP, const double* LC, double* Sb,
                  double* SP, double* SC);
int oracle_sigma_column(i64 nb, i64 w, i64 a, const double* Lr, const double* LP, const double* LC, i64 j,
                        double* x);

static double* take(FILE* f, i64 n) {
    double* p = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!p || (n > 0 && fread(p, sizeof(double), (size_t)n, f) != (size_t)n)) exit(3);
    return p;
}
static void put(FILE* f, const double* p, i64 n) {
    if (n > 0 && fwrite(p, sizeof(double), (size_t)n, f) != (size_t)n) exit(4);
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* in = fopen(argv[1], "rb");
    if (!in) return 2;
    i64 hdr[4];
    if (fread(hdr, sizeof(i64), 4, in) != 4) return 3;
    const i64 nb = hdr[0], w = hdr[1], a = hdr[2], b = hdr[3], n = nb + a;
    double* ab = take(in, (w + 1) * nb);
    double* P = take(in, a * nb);
    double* C = take(in, a * a);
    fclose(in);
    /* exact sizes: any access past them is reported by the sanitizer */
    double* Lr = (double*)calloc((size_t)(nb * (w + 1)), sizeof(double));
    double* LP = (double*)calloc((size_t)(a * nb > 0 ? a * nb : 1), sizeof(double));
    double* LC = (double*)calloc((size_t)(a * a > 0 ? a * a : 1), sizeof(double));
    double logdet = 0.0;
    const int info = oracle_cholesky(nb, w, a, ab, P, C, Lr, LP, LC, &logdet);
    FILE* out = fopen(argv[2], "wb");
    if (!out) return 2;
    const double hd[2] = {logdet, (double)info};
    put(out, hd, 2);
    put(out, Lr, nb * (w + 1));
    put(out, LP, a * nb);
    put(out, LC, a * a);
    if (info == 0) {
        const i64 rows = oracle_sigma_band_rows(nb, w, a, b);
        double* Sb = (double*)calloc((size_t)(rows * nb), sizeof(double));
        double* SP = (double*)calloc((size_t)(a * nb > 0 ? a * nb : 1), sizeof(double));
        double* SC = (double*)calloc((size_t)(a * a > 0 ? a * a : 1), sizeof(double));
        if (oracle_selinv(nb, w, a, b, Lr, LP, LC, Sb, SP, SC) != 0) return 5;
        put(out, Sb, rows * nb);
        put(out, SP, a * nb);
        put(out, SC, a * a);
        double* x = (double*)calloc((size_t)n, sizeof(double));
        for (i64 j = 0; j < n; ++j) {
            if (oracle_sigma_column(nb, w, a, Lr, LP, LC, j, x) != 0) return 6;
            put(out, x, n);
        }
        free(x);
        free(Sb);
        free(SP);
        free(SC);
    }
    fclose(out);
    free(ab);
    free(P);
    free(C);
    free(Lr);
    free(LP);
    free(LC);
    return 0;
}
