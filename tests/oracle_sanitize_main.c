/*
 * Driver of the oracle's C sweep under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_oracle_sanitize.py;
 * CPU only).  It runs every entry point of oracle/sweep.c on a small 2D grid
 * whose lines have their own integer shifts (negative, zero and larger than
 * the line), with and without an output selection, in every storage tier, and
 * checks what the method fixes without any other code:
 *   - alpha = 0 tables (A = I, B = 0) move every cell by s exactly (an exact
 *     permutation along the swept dimension, section II-A update rule);
 *   - the alpha = 1/2 tables of degree 2 (hand-derived fractions, read from
 *     the golden file given as argv[1]) conserve the sum of the cell means;
 *   - the transpose satisfies <M x, y> = <x, M^T y>.
 * Exit status 0 when every check holds; the sanitizers abort on the first
 * invalid access or undefined operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_sweep(int ndim, const int64_t* n, int k, int dim, const int64_t* line_stride,
                  const int32_t* s_tab, const double* ab_tab, int tier,
                  const unsigned char* keep, const int* scale_exp, const double* in,
                  double* out, int64_t n_sel, const int64_t* sel);
void oracle_sweep_adjoint(int ndim, const int64_t* n, int k, int dim,
                          const int64_t* line_stride, const int32_t* s_tab,
                          const double* ab_tab, const double* g_out, double* g_in);
double oracle_round_tier(double x, int tier);
void oracle_round_array(double* x, int64_t n, int tier);

enum { K = 2, O = 3, MODES = 9, N0 = 5, N1 = 4, CELLS = N0 * N1 };

static int failures = 0;

static void check(int ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

/* Reads "A j l p/q" and "B j l p/q" rows into ab[2][O][O]. */
static int read_golden(const char* path, double* ab)
{
    FILE* f = fopen(path, "r");
    if (!f) return 0;
    char line[256];
    int got = 0;
    while (fgets(line, sizeof line, f)) {
        char m;
        int j, l;
        long p, q = 1;
        if (line[0] != 'A' && line[0] != 'B') continue;
        char frac[64];
        if (sscanf(line, "%c %d %d %63s", &m, &j, &l, frac) != 4) continue;
        if (strchr(frac, '/')) {
            if (sscanf(frac, "%ld/%ld", &p, &q) != 2) continue;
        } else {
            p = strtol(frac, NULL, 10);
        }
        if (j < 0 || j >= O || l < 0 || l >= O || q == 0) continue;
        ab[(m == 'B' ? O * O : 0) + j * O + l] = (double)p / (double)q;
        ++got;
    }
    fclose(f);
    return got == 2 * O * O;
}

static int64_t wrapi(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

int main(int argc, char** argv)
{
    if (argc < 2) {
        fprintf(stderr, "usage: %s golden_ab_file\n", argv[0]);
        return 2;
    }
    const int64_t n[2] = {N0, N1};
    /* sweep along dimension 1; every dimension-0 cell has its own line */
    const int64_t stride[2] = {1, 0};
    const int32_t shifts[N0] = {-2, -1, 0, 3, 9};
    double half[2 * O * O];
    if (!read_golden(argv[1], half)) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 2;
    }
    double ident[2 * O * O];
    memset(ident, 0, sizeof ident);
    for (int j = 0; j < O; ++j) ident[j * O + j] = 1.0;

    double* tab_id = malloc(sizeof(double) * N0 * 2 * O * O);
    double* tab_half = malloc(sizeof(double) * N0 * 2 * O * O);
    for (int t = 0; t < N0; ++t) {
        memcpy(tab_id + t * 2 * O * O, ident, sizeof ident);
        memcpy(tab_half + t * 2 * O * O, half, sizeof half);
    }
    double* in = malloc(sizeof(double) * MODES * CELLS);
    double* out = malloc(sizeof(double) * MODES * CELLS);
    double* back = malloc(sizeof(double) * MODES * CELLS);
    double* y = malloc(sizeof(double) * MODES * CELLS);
    unsigned seed = 12345u;
    for (int i = 0; i < MODES * CELLS; ++i) {
        seed = seed * 1664525u + 1013904223u;
        in[i] = ((double)(seed >> 8) / 16777216.0 - 0.5) * (i < CELLS ? 1.0 : 0.01);
        seed = seed * 1664525u + 1013904223u;
        y[i] = (double)(seed >> 8) / 16777216.0 - 0.5;
    }
    unsigned char keep[MODES];
    memset(keep, 0, sizeof keep);
    keep[0] = 1;
    int scale[MODES];
    for (int m = 0; m < MODES; ++m) scale[m] = m % 3;

    for (int tier = 0; tier < 4; ++tier) {
        /* integer shifts: an exact permutation of the cells of each line */
        oracle_sweep(2, n, K, 1, stride, shifts, tab_id, tier, keep, NULL, in, out, 0, NULL);
        int exact = 1;
        for (int m = 0; m < MODES; ++m)
            for (int i1 = 0; i1 < N1; ++i1)
                for (int i0 = 0; i0 < N0; ++i0) {
                    const int64_t src = i0 + N0 * wrapi(i1 - shifts[i0], N1);
                    const double want = keep[m] ? in[m * CELLS + src]
                                                : oracle_round_tier(in[m * CELLS + src], tier);
                    exact &= out[m * CELLS + i0 + N0 * i1] == want;
                }
        check(exact, "integer shift is a permutation");

        /* alpha = 1/2: the sum of the cell means is conserved */
        oracle_sweep(2, n, K, 1, stride, shifts, tab_half, tier, keep, scale, in, out, 0, NULL);
        double m0 = 0.0, m1 = 0.0, a0 = 0.0;
        for (int c = 0; c < CELLS; ++c) {
            m0 += in[c];
            m1 += out[c];
            a0 += fabs(in[c]);
        }
        check(fabs(m1 - m0) <= 1e-14 * a0, "mass conserved at alpha = 1/2");

        /* a selection of output cells (unsorted, repeated) */
        const int64_t sel[6] = {19, 0, 7, 7, 12, 3};
        double osel[MODES * 6];
        oracle_sweep(2, n, K, 1, stride, shifts, tab_half, tier, keep, scale, in, osel, 6, sel);
        int same = 1;
        for (int m = 0; m < MODES; ++m)
            for (int q = 0; q < 6; ++q) same &= osel[m * 6 + q] == out[m * CELLS + sel[q]];
        check(same, "selected cells equal the full sweep");
    }

    /* transpose: <M x, y> = <x, M^T y> (no rounding, FP64 tables) */
    unsigned char keep_all[MODES];
    memset(keep_all, 1, sizeof keep_all);
    oracle_sweep(2, n, K, 1, stride, shifts, tab_half, 0, keep_all, NULL, in, out, 0, NULL);
    oracle_sweep_adjoint(2, n, K, 1, stride, shifts, tab_half, y, back);
    double lhs = 0.0, rhs = 0.0, mag = 0.0;
    for (int i = 0; i < MODES * CELLS; ++i) {
        lhs += out[i] * y[i];
        rhs += in[i] * back[i];
        mag += fabs(out[i] * y[i]) + fabs(in[i] * back[i]);
    }
    check(fabs(lhs - rhs) <= 1e-14 * mag, "dot-product identity of the transpose");

    /* rounding of special values */
    double sp[8] = {0.0, -0.0, 1e-320, -6e-8, 65520.0, 3.4e38, INFINITY, NAN};
    for (int tier = 0; tier < 4; ++tier) {
        double tmp[8];
        memcpy(tmp, sp, sizeof sp);
        oracle_round_array(tmp, 8, tier);
        check(isinf(tmp[6]) && isnan(tmp[7]), "inf and nan pass through rounding");
    }

    free(tab_id);
    free(tab_half);
    free(in);
    free(out);
    free(back);
    free(y);
    if (failures) return 1;
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
