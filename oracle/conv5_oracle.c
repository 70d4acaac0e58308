/*
 * conv5_oracle.c -- plain, slow FP64 CPU oracle for the width-5 separable
 * convolution of a multi-plane image.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * What it computes (arXiv 1711.09791):
 *   - Eq. 1 (Section 1): B[y][x] = sum_i sum_j A[y+i][x+j] * K[i][j], written
 *     as a correlation (the kernel is not flipped), with the separable kernel
 *     K[i][j] = k_i * k_j (Section 1, right after Eq. 1), i, j in -2..2
 *     (width 5: Section 1 and the 5x5 Gaussian of Section 4).
 *   - Border convention (Section 5, opening paragraph): only pixels whose whole
 *     5x5 neighbourhood lies inside the image are convolved, starting at pixel
 *     (2,2).  The paper leaves the rest untouched; this oracle fixes it to 0.
 *   - Planes are independent (Section 5.3, the per-plane driver loop).
 *   - The same Eq. 1 at any odd width n with any n x n kernel, separable or
 *     not (oracle_conv_direct_n), for the width-n kernels.
 *   - The two-pass form with its auxiliary array rounded to a 16-bit format
 *     (oracle_conv5_twopass_q), a reduced-precision variant with its own
 *     definition.
 *
 * All arithmetic is IEEE binary64.  The 16-bit helpers decode half and bfloat16
 * storage exactly and round binary64 results to those formats with
 * round-to-nearest-even, written from the IEEE 754 definitions.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define R5 2 /* kernel radius: taps at offsets -2..2 */

#ifdef _OPENMP
/* Threads of one parallel region: nthreads > 0 asks for exactly that many,
 * otherwise the OpenMP default.  The count is set per region (num_threads
 * clause), so a call never changes what later calls get by default; the
 * last region's team is remembered for oracle_last_team(). */
static int g_last_team = 1;
static int team_size(int nthreads)
{
    const int t = nthreads > 0 ? nthreads : omp_get_max_threads();
    g_last_team = t;
    return t;
}
#endif

/*
 * Single-pass form (Section 5.1; Eq. 2 / Eq. 3 of Section 5.2): four nested loops, 25
 * multiply-adds per interior pixel, K[a][b] = k[a] * k[b] evaluated in FP64.
 * A and B are dense [planes][rows][cols]; B is fully written.
 * nthreads <= 0 means "whatever OpenMP picks"; 1 means serial.
 */
void oracle_conv5_direct(const double *A, double *B, const double *k,
                         int64_t planes, int64_t rows, int64_t cols,
                         int nthreads)
{
    const int64_t plane_elems = rows * cols;
    if (plane_elems == 0 || planes == 0)
        return;
    memset(B, 0, sizeof(double) * (size_t)(planes * plane_elems));
    if (rows < 2 * R5 + 1 || cols < 2 * R5 + 1)
        return; /* no pixel has a full neighbourhood */
#ifdef _OPENMP
    const int team = team_size(nthreads);
#pragma omp parallel for collapse(2) schedule(static) num_threads(team)
#endif
    for (int64_t p = 0; p < planes; ++p) {
        for (int64_t y = R5; y < rows - R5; ++y) {
            const double *Ap = A + p * plane_elems;
            double *Bp = B + p * plane_elems;
            for (int64_t x = R5; x < cols - R5; ++x) {
                double acc = 0.0;
                for (int a = -R5; a <= R5; ++a) {
                    for (int b = -R5; b <= R5; ++b) {
                        const double Kab = k[a + R5] * k[b + R5];
                        acc += Ap[(y + a) * cols + (x + b)] * Kab;
                    }
                }
                Bp[y * cols + x] = acc;
            }
        }
    }
}

/*
 * Two-pass form (Section 5.1, the separable algorithm): a horizontal 5-tap
 * pass into an auxiliary array, then a vertical 5-tap pass out of it.  The
 * horizontal pass covers every row, so that the vertical pass at rows 2, 3,
 * H-4 and H-3 reads filtered data.  aux must hold rows*cols doubles.
 */
void oracle_conv5_twopass(const double *A, double *B, double *aux,
                          const double *k, int64_t planes, int64_t rows,
                          int64_t cols)
{
    const int64_t plane_elems = rows * cols;
    if (plane_elems == 0 || planes == 0)
        return;
    memset(B, 0, sizeof(double) * (size_t)(planes * plane_elems));
    if (rows < 2 * R5 + 1 || cols < 2 * R5 + 1)
        return;
    for (int64_t p = 0; p < planes; ++p) {
        const double *Ap = A + p * plane_elems;
        double *Bp = B + p * plane_elems;
        memset(aux, 0, sizeof(double) * (size_t)plane_elems);
        for (int64_t y = 0; y < rows; ++y)            /* horizontal pass */
            for (int64_t x = R5; x < cols - R5; ++x) {
                double t = 0.0;
                for (int b = -R5; b <= R5; ++b)
                    t += Ap[y * cols + x + b] * k[b + R5];
                aux[y * cols + x] = t;
            }
        for (int64_t y = R5; y < rows - R5; ++y)      /* vertical pass */
            for (int64_t x = R5; x < cols - R5; ++x) {
                double s = 0.0;
                for (int a = -R5; a <= R5; ++a)
                    s += aux[(y + a) * cols + x] * k[a + R5];
                Bp[y * cols + x] = s;
            }
    }
}

/*
 * Any odd width n = 2r+1 and any n x n kernel, separable or not: Eq. 1 with
 * K given as a full matrix (Section 5.1 sets the n*n terms of this direct
 * form against the 2n of the separable one).  K is row-major, K[a*n + b]
 * weighting A[y + a - r][x + b - r] (correlation form, as above).  Border of
 * r pixels = 0, the border rule of Section 5 applied to width n.
 */
void oracle_conv_direct_n(const double *A, double *B, const double *K, int n,
                          int64_t planes, int64_t rows, int64_t cols,
                          int nthreads)
{
    const int64_t plane_elems = rows * cols;
    const int r = n / 2;
    if (plane_elems == 0 || planes == 0)
        return;
    memset(B, 0, sizeof(double) * (size_t)(planes * plane_elems));
    if (n < 1 || n % 2 == 0 || rows < n || cols < n)
        return;
#ifdef _OPENMP
    const int team = team_size(nthreads);
#pragma omp parallel for collapse(2) schedule(static) num_threads(team)
#endif
    for (int64_t p = 0; p < planes; ++p) {
        for (int64_t y = r; y < rows - r; ++y) {
            const double *src = A + p * plane_elems;
            double *dst = B + p * plane_elems;
            for (int64_t x = r; x < cols - r; ++x) {
                double acc = 0.0;
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b)
                        acc += src[(y + a - r) * cols + (x + b - r)] * K[a * n + b];
                dst[y * cols + x] = acc;
            }
        }
    }
}

/* ---- exact decoding of the storage formats ------------------------------ */

/* IEEE binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits. */
static double half_bits_to_double(uint16_t h)
{
    const int sign = (h >> 15) & 1;
    const int e = (h >> 10) & 0x1f;
    const int f = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);                  /* subnormal or zero */
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + f), e - 25);      /* (1.f) * 2^(e-15) */
    return sign ? -v : v;
}

/* bfloat16: the upper 16 bits of an IEEE binary32. */
static double bf16_bits_to_double(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

void oracle_decode_f32(const float *src, double *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = (double)src[i];
}

void oracle_decode_f16(const uint16_t *src, double *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = half_bits_to_double(src[i]);
}

void oracle_decode_bf16(const uint16_t *src, double *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = bf16_bits_to_double(src[i]);
}

/* ---- round-to-nearest-even from binary64 ------------------------------- */

/*
 * Round |v| (finite, >= 0) to a binary format with `mbits` fraction bits,
 * minimum normal exponent emin and maximum finite exponent emax, returning
 * the rounded magnitude as a double (or +inf on overflow).  The quantum at
 * exponent e is 2^(e - mbits); below 2^emin the quantum is 2^(emin - mbits).
 * Ties go to the even multiple of the quantum.
 */
static double rne_magnitude(double v, int mbits, int emin, int emax)
{
    if (v == 0.0)
        return 0.0;
    int e;
    frexp(v, &e);           /* v = m * 2^e, m in [0.5, 1): leading bit 2^(e-1) */
    int ex = e - 1;         /* unbiased exponent of v */
    if (ex < emin)
        ex = emin;
    const double q = ldexp(1.0, ex - mbits);        /* quantum */
    const double n = v / q;                         /* exact: power-of-2 scale */
    double fl = floor(n);
    const double rem = n - fl;                      /* exact */
    if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) != 0.0))
        fl += 1.0;
    const double r = fl * q;
    /* largest finite: (2 - 2^-mbits) * 2^emax */
    const double maxf = ldexp(2.0 - ldexp(1.0, -mbits), emax);
    if (r > maxf)
        return INFINITY;
    return r;
}

/* binary64 -> IEEE binary16 bits, RNE, single rounding. */
static uint16_t double_to_half_bits(double v)
{
    if (isnan(v))
        return 0x7e00;
    const uint16_t s = signbit(v) ? 0x8000 : 0;
    const double r = rne_magnitude(fabs(v), 10, -14, 15);
    if (isinf(r))
        return s | 0x7c00;
    if (r == 0.0)
        return s;
    int e;
    frexp(r, &e);
    int ex = e - 1;
    if (ex < -14) {                                  /* subnormal */
        return s | (uint16_t)(r / ldexp(1.0, -24));
    }
    const uint16_t frac = (uint16_t)(r / ldexp(1.0, ex - 10) - 1024.0);
    return s | (uint16_t)((ex + 15) << 10) | frac;
}

/* binary64 -> bfloat16 bits (8 exponent bits, 7 fraction bits), RNE. */
static uint16_t double_to_bf16_bits(double v)
{
    if (isnan(v))
        return 0x7fc0;
    const uint16_t s = signbit(v) ? 0x8000 : 0;
    const double r = rne_magnitude(fabs(v), 7, -126, 127);
    if (isinf(r))
        return s | 0x7f80;
    if (r == 0.0)
        return s;
    int e;
    frexp(r, &e);
    int ex = e - 1;
    if (ex < -126)
        return s | (uint16_t)(r / ldexp(1.0, -133));
    const uint16_t frac = (uint16_t)(r / ldexp(1.0, ex - 7) - 128.0);
    return s | (uint16_t)((ex + 127) << 7) | frac;
}

void oracle_round_f16(const double *src, uint16_t *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = double_to_half_bits(src[i]);
}

void oracle_round_bf16(const double *src, uint16_t *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = double_to_bf16_bits(src[i]);
}

/*
 * Two-pass form with a 16-bit auxiliary array.  The paper's auxiliary array
 * (the intermediate of the two-pass form, Section 7) holds float values; this
 * variant keeps it in a narrower format to halve its memory traffic, which
 * changes the arithmetic, so it has its own definition: the horizontal pass is
 * computed exactly as in oracle_conv5_twopass (binary64, every row, columns
 * 2..cols-3, zero elsewhere); each auxiliary value is then rounded once to the
 * 16-bit format with round-to-nearest-even (tfmt 1: IEEE binary16, 2:
 * bfloat16); the vertical pass reads the rounded values, exactly, in binary64.
 */
void oracle_conv5_twopass_q(const double *A, double *B, double *aux,
                            const double *k, int64_t planes, int64_t rows,
                            int64_t cols, int tfmt)
{
    const int64_t n_plane = rows * cols;
    if (n_plane == 0 || planes == 0)
        return;
    memset(B, 0, sizeof(double) * (size_t)(planes * n_plane));
    if (rows < 2 * R5 + 1 || cols < 2 * R5 + 1)
        return;
    for (int64_t p = 0; p < planes; ++p) {
        const double *in = A + p * n_plane;
        double *out = B + p * n_plane;
        memset(aux, 0, sizeof(double) * (size_t)n_plane);
        /* horizontal pass on every row */
        for (int64_t i = 0; i < rows; ++i)
            for (int64_t j = R5; j < cols - R5; ++j) {
                double h = 0.0;
                for (int d = -R5; d <= R5; ++d)
                    h += in[i * cols + j + d] * k[d + R5];
                aux[i * cols + j] = h;
            }
        /* the auxiliary array in the 16-bit format */
        for (int64_t e = 0; e < n_plane; ++e)
            aux[e] = tfmt == 1 ? half_bits_to_double(double_to_half_bits(aux[e]))
                               : bf16_bits_to_double(double_to_bf16_bits(aux[e]));
        /* vertical pass over the rounded values */
        for (int64_t i = R5; i < rows - R5; ++i)
            for (int64_t j = R5; j < cols - R5; ++j) {
                double v = 0.0;
                for (int d = -R5; d <= R5; ++d)
                    v += aux[(i + d) * cols + j] * k[d + R5];
                out[i * cols + j] = v;
            }
    }
}

/* Number of OpenMP threads a parallel region of the oracle would use. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Team size asked for by the last parallel region (1 before any). */
int oracle_last_team(void)
{
#ifdef _OPENMP
    return g_last_team;
#else
    return 1;
#endif
}
