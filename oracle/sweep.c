/*
 * Oracle: plain CPU FP64 projection sweep of the semi-Lagrangian discontinuous
 * Galerkin (sLdG) method.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the CPU-baseline leg of the benchmark use it; the product path never does.
 * It shares no code, header or table with the HIP library.
 *
 * What it computes (Einkemmer, "A mixed precision semi-Lagrangian algorithm and
 * its performance on accelerators", section II-A, update rule): for every
 * output cell i along the swept dimension and every Legendre mode j,
 *
 *     c_new[i][j] = sum_l A[j][l] c[i-s][l] + sum_l B[j][l] c[i-s-1][l]
 *
 * where s = floor(sigma) is the integer part of the displacement in cells and
 * A, B are the (k+1)x(k+1) matrices of the exact L2 projection of the
 * translated piecewise polynomial (they are computed by the Python side of the
 * oracle, exactly, and passed in per line).  In more than one dimension the
 * basis is the tensor product of Legendre polynomials; the sweep mixes only the
 * mode index of the swept dimension, the other mode indices are spectators.
 * The grid is periodic in every dimension.
 *
 * Storage of the oracle state: one FP64 array [mode][cell], mode id
 * m = j_0 + o*(j_1 + o*(j_2 + ...)), cell id = i_0 + N_0*(i_1 + N_1*(...)),
 * dimension 0 fastest.  Mixed precision (section II-A, the paragraph on storing
 * c_0 in double precision; section III-A, where the number of leading
 * coefficients kept in double precision varies) is emulated: every mode not
 * marked `keep` is rounded to nearest-even onto the storage format after each
 * sweep, the kept modes (by default the cell mean m = 0 alone) stay FP64.
 * A narrow mode may also be stored scaled by a power of two 2^e[m] (the
 * per-mode scaling that keeps FP16 away from its underflow range): its value
 * is then round(c * 2^e) * 2^-e, i.e. the rounding onto the format with its
 * exponent range moved by -e; the scaling itself is exact.
 *
 * Plain loops, no blocking, no reordering; OpenMP only splits the independent
 * output cells between threads and does not change any result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { ORACLE_FP64 = 0, ORACLE_FP32 = 1, ORACLE_BF16 = 2, ORACLE_FP16 = 3 };

/* Round x to nearest, ties to even, onto a binary floating-point format with
 * `mant` stored fraction bits, minimum normal exponent emin and maximum exponent
 * emax (IEEE 754 semantics, gradual underflow, overflow to +-inf). */
static double round_format(double x, int mant, int emin, int emax)
{
    if (x == 0.0 || !isfinite(x))
        return x;
    int e;
    frexp(x, &e);          /* x = f * 2^e with 0.5 <= |f| < 1 */
    int ue = e - 1;        /* exponent of the leading bit */
    if (ue < emin)
        ue = emin;         /* subnormal range: the quantum stays 2^(emin-mant) */
    double q = ldexp(1.0, ue - mant);
    double r = nearbyint(x / q) * q;   /* x/q is exact (power-of-two scaling) */
    double maxf = ldexp(2.0 - ldexp(1.0, -mant), emax);
    if (fabs(r) > maxf)
        return r > 0 ? INFINITY : -INFINITY;
    return r;
}

double oracle_round_tier(double x, int tier)
{
    switch (tier) {
    case ORACLE_FP32: return round_format(x, 23, -126, 127);
    case ORACLE_BF16: return round_format(x, 7, -126, 127);
    case ORACLE_FP16: return round_format(x, 10, -14, 15);
    default:          return x;
    }
}

void oracle_round_array(double* x, int64_t n, int tier)
{
    for (int64_t i = 0; i < n; ++i)
        x[i] = oracle_round_tier(x[i], tier);
}

static int64_t wrap(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/*
 * One sweep along dimension `dim`.
 *   ndim, n[ndim]   grid (dimension 0 fastest), periodic
 *   k               polynomial degree, o = k+1 modes per dimension
 *   line_stride     [ndim] stride of dimension e in the per-line tables, 0 when
 *                   the displacement does not depend on e (must be 0 for dim)
 *   s_tab, ab_tab   per table entry t: integer shift s_tab[t] and the matrices
 *                   A = ab_tab[t*2*o*o ...], B = A + o*o, row-major [j][l]
 *   tier            storage emulation of the modes with keep[m] == 0
 *   keep            [o^ndim] 1 for the modes stored (and updated) in FP64
 *   scale_exp       [o^ndim] storage exponent e of every mode, or NULL (all 0)
 *   in              [o^ndim][cells]
 *   out             [o^ndim][n_sel]  (n_sel = cells when sel == NULL)
 *   sel             optional list of output cells to compute
 */
void oracle_sweep(int ndim, const int64_t* n, int k, int dim,
                  const int64_t* line_stride, const int32_t* s_tab,
                  const double* ab_tab, int tier, const unsigned char* keep,
                  const int* scale_exp, const double* in, double* out, int64_t n_sel,
                  const int64_t* sel)
{
    const int o = k + 1;
    int64_t cells = 1, modes = 1, mstride = 1;
    for (int e = 0; e < ndim; ++e) {
        cells *= n[e];
        modes *= o;
        if (e < dim)
            mstride *= o;          /* distance between j_dim and j_dim + 1 */
    }
    int64_t cstride = 1;           /* distance between i_dim and i_dim + 1 */
    for (int e = 0; e < dim; ++e)
        cstride *= n[e];
    const int64_t nout = sel ? n_sel : cells;

#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nout; ++q) {
        const int64_t c = sel ? sel[q] : q;
        /* table entry of the line through c, and the index along dim */
        int64_t rest = c, t = 0, idim = 0;
        for (int e = 0; e < ndim; ++e) {
            int64_t ie = rest % n[e];
            rest /= n[e];
            t += ie * line_stride[e];
            if (e == dim)
                idim = ie;
        }
        const int64_t s = s_tab[t];
        const double* A = ab_tab + t * 2 * o * o;
        const double* B = A + o * o;
        const int64_t base = c - idim * cstride;
        const int64_t ca = base + wrap(idim - s, n[dim]) * cstride;      /* cell i-s   */
        const int64_t cb = base + wrap(idim - s - 1, n[dim]) * cstride;  /* cell i-s-1 */
        for (int64_t m = 0; m < modes; ++m) {
            const int j = (int)((m / mstride) % o);
            const int64_t m0 = m - j * mstride;
            double acc = 0.0;
            for (int l = 0; l < o; ++l)
                acc += A[j * o + l] * in[(m0 + l * mstride) * cells + ca];
            for (int l = 0; l < o; ++l)
                acc += B[j * o + l] * in[(m0 + l * mstride) * cells + cb];
            if (keep[m]) {
                out[m * nout + q] = acc;
            } else {
                const int e = scale_exp ? scale_exp[m] : 0;
                out[m * nout + q] = ldexp(oracle_round_tier(ldexp(acc, e), tier), -e);
            }
        }
    }
}

int oracle_num_threads(void)
{
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            nt = omp_get_num_threads();
#endif
        }
    }
    return nt;
}

/* Sets the OpenMP thread count of later sweeps (n > 0); timing only. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Transpose of oracle_sweep (no rounding): g_in = M^T g_out, M the sweep with
 * the same tables.  Output cell i reads input cells i-s (through A) and
 * i-s-1 (through B), so input cell m is read by output cells m+s (A) and
 * m+s+1 (B):
 *     g_in[l](m) = sum_j A[j][l] g_out[j](m+s) + sum_j B[j][l] g_out[j](m+s+1)
 * for every spectator tuple, periodic along dim.  Arguments as oracle_sweep.
 */
void oracle_sweep_adjoint(int ndim, const int64_t* n, int k, int dim,
                          const int64_t* line_stride, const int32_t* s_tab,
                          const double* ab_tab, const double* g_out, double* g_in)
{
    const int o = k + 1;
    int64_t cells = 1, modes = 1, mstride = 1;
    for (int e = 0; e < ndim; ++e) {
        cells *= n[e];
        modes *= o;
        if (e < dim)
            mstride *= o;
    }
    int64_t cstride = 1;
    for (int e = 0; e < dim; ++e)
        cstride *= n[e];

#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < cells; ++c) {
        int64_t rest = c, t = 0, idim = 0;
        for (int e = 0; e < ndim; ++e) {
            int64_t ie = rest % n[e];
            rest /= n[e];
            t += ie * line_stride[e];
            if (e == dim)
                idim = ie;
        }
        const int64_t s = s_tab[t];
        const double* A = ab_tab + t * 2 * o * o;
        const double* B = A + o * o;
        const int64_t base = c - idim * cstride;
        const int64_t ca = base + wrap(idim + s, n[dim]) * cstride;      /* output m+s   */
        const int64_t cb = base + wrap(idim + s + 1, n[dim]) * cstride;  /* output m+s+1 */
        for (int64_t m = 0; m < modes; ++m) {
            const int l = (int)((m / mstride) % o);
            const int64_t m0 = m - l * mstride;
            double acc = 0.0;
            for (int j = 0; j < o; ++j)
                acc += A[j * o + l] * g_out[(m0 + j * mstride) * cells + ca];
            for (int j = 0; j < o; ++j)
                acc += B[j * o + l] * g_out[(m0 + j * mstride) * cells + cb];
            g_in[m * cells + c] = acc;
        }
    }
}
