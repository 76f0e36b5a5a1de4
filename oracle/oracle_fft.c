/*
 * oracle_fft.c -- plain FP64 CPU oracle for the local phases of the pencil
 * 3-D FFT (AccFFT, Gholami et al., Section 2, Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: it exists so that the HIP library can be checked against an
 * independent, slow, obviously correct implementation.  It shares no code,
 * header, table or constant with the HIP sources.
 *
 * What it computes (Section 2, the paragraph that introduces N0, N1, N2 and
 * the Cooley-Tukey operation count; Algorithm 1 for the axis order):
 *
 *   X[k0,k1,k2] = sum_{a,b,c} x[a,b,c] * exp(s*2*pi*i*(k0 a/n0 + k1 b/n1 + k2 c/n2))
 *
 * with s = -1 for the forward and s = +1 for the inverse transform.  Neither
 * direction is scaled, so inverse(forward(x)) = n0*n1*n2 * x (the paper only
 * says the two directions agree up to a scale factor; the footnote on
 * normalisation leaves the choice open -- unscaled is the reading taken).
 * Arrays are C-order [x][y][z], z (n2) fastest, the same layout in both
 * domains (Section 2, slab paragraph: frequency layout equals spatial layout).
 *
 * Evaluation order is the row-column order of Algorithm 1: every z-line,
 * then every y-line, then every x-line.  Because the DFT kernel is separable
 * this equals the triple sum above exactly in exact arithmetic.
 *
 * 1-D transforms use a recursive decimation-in-time mixed-radix Cooley-Tukey
 * split (the reduction the paper credits for the 5 N log N count): a length
 * n = p*m is split into p interleaved subsequences of length m, each
 * transformed recursively, and recombined with twiddles w_n^{q k} followed by
 * a direct length-p DFT.  p is 4 when 4 | n, else the smallest prime factor
 * (2, 3, 5, 7, ...), so any length is handled; a prime length with no
 * smaller factor is done as a direct O(n^2) DFT.
 *
 * Real transforms (Section 1, the list of supported kinds: R2C, C2C, C2R):
 *   R2C: the full complex transform of the real input (imaginary part 0),
 *        keeping k2 = 0 .. floor(n2/2).
 *   C2R: inverse along x, then y, on the n0 x n1 x (floor(n2/2)+1) half
 *        array; then along z each line Y is extended to a Hermitian line F of
 *        length n2 with F[0] = Re Y[0], F[k] = Y[k], F[n2-k] = conj(Y[k]) and,
 *        for even n2, F[n2/2] = Re Y[n2/2]; the output is Re(IDFT(F)).  The
 *        imaginary parts of the k2 = 0 and k2 = n2/2 entries are therefore
 *        discarded, which defines the result for non-Hermitian input too.
 *
 * Spectral Poisson (Section 1 lists "fast spectral operators"; the operator
 * itself is the standard periodic Poisson solve): on the half spectrum,
 *   U[k] = -F[k] / |k|^2, U[0] = 0, with signed wavenumbers
 *   k' = k for k < n/2 else k - n along x and y, and k2 itself along z.
 *
 * Parity status: every exported function is pinned by tests against a brute
 * force DFT, closed forms and invariants; no function is parity unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double kPi = 3.14159265358979323846264338327950288;

typedef struct {
    double re, im;
} cplx;

static cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static cplx c_mul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

/* exp(sign * 2 pi i * j / n), j reduced modulo n first.  The angle is split
 * into a whole number of quarter turns (exact, integer arithmetic) plus a
 * remainder in [0, pi/4], so multiples of a quarter turn come out exact and
 * the libm call only ever sees a small argument. */
static cplx unit_root(int64_t j, int64_t n, int sign)
{
    j %= n;
    if (j < 0) j += n;
    int64_t q = (4 * j) / n;     /* quarter turns */
    int64_t r = 4 * j - q * n;   /* remainder: angle = (q + r/n) * pi/2 */
    double cb, sb;
    if (2 * r <= n) {
        double phi = (kPi / 2.0) * (double)r / (double)n;
        cb = cos(phi);
        sb = sin(phi);
    } else {
        double phi = (kPi / 2.0) * (double)(n - r) / (double)n;
        cb = sin(phi);
        sb = cos(phi);
    }
    double c, s;
    switch (q) {
    case 0: c = cb; s = sb; break;
    case 1: c = -sb; s = cb; break;
    case 2: c = -cb; s = -sb; break;
    default: c = sb; s = -cb; break;
    }
    cplx w = {c, sign < 0 ? -s : s};
    return w;
}

static int smallest_factor(int n)
{
    if (n % 4 == 0) return 4;
    for (int p = 2; (int64_t)p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* The twiddles of every level come from one table of the ntop-th roots of
 * unity, roots[j] = unit_root(j, ntop, sign).  A level of length n (n divides
 * ntop) needs w_n^e = roots[(e mod n) * (ntop / n)]. */
typedef struct {
    const cplx* roots;
    int ntop;
} root_table;

static cplx w_pow(const root_table* t, int64_t e, int n)
{
    e %= n;
    return t->roots[e * (t->ntop / n)];
}

/* Direct DFT of n points read at stride `stride`, written contiguously. */
static void dft_direct(const cplx* x, int64_t stride, cplx* out, int n, const root_table* t)
{
    for (int k = 0; k < n; ++k) {
        cplx acc = {0.0, 0.0};
        for (int j = 0; j < n; ++j)
            acc = c_add(acc, c_mul(x[(int64_t)j * stride], w_pow(t, (int64_t)j * k, n)));
        out[k] = acc;
    }
}

/* Recursive mixed-radix DIT FFT: x read at `stride`, result in out[0..n).
 * `tmp` must hold at least n entries and is clobbered. */
static void fft_rec(const cplx* x, int64_t stride, cplx* out, int n, const root_table* t, cplx* tmp)
{
    if (n == 1) {
        out[0] = x[0];
        return;
    }
    int p = smallest_factor(n);
    if (p == n) {
        dft_direct(x, stride, out, n, t);
        return;
    }
    int m = n / p;
    /* sub-transform q of x[q], x[q+p], ... lands in tmp[q*m .. q*m+m) */
    for (int q = 0; q < p; ++q)
        fft_rec(x + q * stride, stride * p, tmp + (int64_t)q * m, m, t, out);
    /* recombine: X[k + m r] = sum_q w_n^{q k} w_p^{q r} Y_q[k] */
    cplx small[64];
    cplx* tv = (p <= 64) ? small : (cplx*)malloc(sizeof(cplx) * (size_t)p);
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < p; ++q)
            tv[q] = c_mul(tmp[(int64_t)q * m + k], w_pow(t, (int64_t)q * k, n));
        for (int r = 0; r < p; ++r) {
            cplx acc = {0.0, 0.0};
            for (int q = 0; q < p; ++q)
                acc = c_add(acc, c_mul(tv[q], w_pow(t, (int64_t)q * r, p)));
            out[k + (int64_t)m * r] = acc;
        }
    }
    if (tv != small) free(tv);
}

static cplx* make_roots(int n, int sign)
{
    cplx* r = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    for (int j = 0; j < n; ++j) r[j] = unit_root(j, n, sign);
    return r;
}

/* 1-D transform of one contiguous line in place.  work holds 2n entries. */
static void fft_line(cplx* line, int n, const root_table* t, cplx* work)
{
    fft_rec(line, 1, work, n, t, work + n);
    memcpy(line, work, sizeof(cplx) * (size_t)n);
}

/* Transform every line along one axis of a C-order complex array whose shape
 * is (outer, len, inner): element (o, j, i) sits at (o*len + j)*inner + i. */
static void fft_axis(cplx* a, int64_t outer, int len, int64_t inner, int sign)
{
    int64_t lines = outer * inner;
    cplx* roots = make_roots(len, sign);
    root_table t = {roots, len};
#pragma omp parallel
    {
        cplx* line = (cplx*)malloc(sizeof(cplx) * (size_t)len);
        cplx* work = (cplx*)malloc(sizeof(cplx) * (size_t)len * 2);
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; ++l) {
            int64_t o = l / inner, i = l % inner;
            cplx* base = a + o * len * inner + i;
            for (int j = 0; j < len; ++j) line[j] = base[(int64_t)j * inner];
            fft_line(line, len, &t, work);
            for (int j = 0; j < len; ++j) base[(int64_t)j * inner] = line[j];
        }
        free(line);
        free(work);
    }
    free(roots);
}

/* ---- exported entry points (called through ctypes by the test suite) ---- */

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of threads the OpenMP loops above will use. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* 3-D C2C in place on interleaved complex doubles; Algorithm 1 order z,y,x. */
void oracle_fft3d_c2c(double* data, int n0, int n1, int n2, int sign)
{
    cplx* a = (cplx*)data;
    fft_axis(a, (int64_t)n0 * n1, n2, 1, sign);      /* z-lines */
    fft_axis(a, (int64_t)n0, n1, (int64_t)n2, sign); /* y-lines */
    fft_axis(a, 1, n0, (int64_t)n1 * n2, sign);      /* x-lines */
}

/* One axis of a C-order array of shape (outer, len, inner), in place.  Used to
 * build the partial transforms of the pencil share (z only, y only). */
void oracle_fft_axis(double* data, int64_t outer, int len, int64_t inner, int sign)
{
    fft_axis((cplx*)data, outer, len, inner, sign);
}

/* 3-D R2C: real[n0][n1][n2] -> complex[n0][n1][n2/2+1]. */
void oracle_fft3d_r2c(const double* in, double* out, int n0, int n1, int n2)
{
    int n2c = n2 / 2 + 1;
    int64_t lines = (int64_t)n0 * n1;
    cplx* full = (cplx*)malloc(sizeof(cplx) * (size_t)lines * (size_t)n2);
    for (int64_t i = 0; i < lines * n2; ++i) {
        full[i].re = in[i];
        full[i].im = 0.0;
    }
    oracle_fft3d_c2c((double*)full, n0, n1, n2, -1);
    cplx* o = (cplx*)out;
    for (int64_t l = 0; l < lines; ++l)
        for (int k = 0; k < n2c; ++k) o[l * n2c + k] = full[l * n2 + k];
    free(full);
}

/* z-only C2R of `lines` half lines complex[lines][n2/2+1] -> real[lines][n2],
 * unscaled; the imaginary parts at k2 = 0 and (even n2) k2 = n2/2 are
 * discarded.  Definition in the file header. */
void oracle_c2r_z(const double* in, double* out, int64_t lines, int n2)
{
    int n2c = n2 / 2 + 1;
    const cplx* half = (const cplx*)in;
    cplx* roots = make_roots(n2, +1);
    root_table t = {roots, n2};
#pragma omp parallel
    {
        cplx* line = (cplx*)malloc(sizeof(cplx) * (size_t)n2);
        cplx* work = (cplx*)malloc(sizeof(cplx) * (size_t)n2 * 2);
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; ++l) {
            const cplx* y = half + l * n2c;
            for (int k = 0; k < n2; ++k) { line[k].re = 0.0; line[k].im = 0.0; }
            line[0].re = y[0].re;
            for (int k = 1; 2 * k < n2; ++k) {
                line[k] = y[k];
                line[n2 - k].re = y[k].re;
                line[n2 - k].im = -y[k].im;
            }
            if (n2 % 2 == 0 && n2 > 1) line[n2 / 2].re = y[n2 / 2].re;
            fft_line(line, n2, &t, work);
            for (int c = 0; c < n2; ++c) out[l * n2 + c] = line[c].re;
        }
        free(line);
        free(work);
    }
    free(roots);
}

/* 3-D C2R: complex[n0][n1][n2/2+1] -> real[n0][n1][n2], unscaled, the input
 * is left untouched: x- and y-lines inverse, then the z-only C2R. */
void oracle_fft3d_c2r(const double* in, double* out, int n0, int n1, int n2)
{
    int n2c = n2 / 2 + 1;
    int64_t lines = (int64_t)n0 * n1;
    cplx* half = (cplx*)malloc(sizeof(cplx) * (size_t)lines * (size_t)n2c);
    memcpy(half, in, sizeof(cplx) * (size_t)lines * (size_t)n2c);
    fft_axis(half, 1, n0, (int64_t)n1 * n2c, +1);       /* x-lines */
    fft_axis(half, (int64_t)n0, n1, (int64_t)n2c, +1);  /* y-lines */
    oracle_c2r_z((const double*)half, out, lines, n2);
    free(half);
}

/* Spectral Poisson multiply on the half spectrum [n0][n1][n2/2+1] in place:
 * U = -F * scale / |k|^2, U[0,0,0] = 0. */
void oracle_poisson_half(double* data, int n0, int n1, int n2, double scale)
{
    int n2c = n2 / 2 + 1;
    cplx* a = (cplx*)data;
    for (int i0 = 0; i0 < n0; ++i0) {
        int64_t k0 = (2 * i0 < n0) ? i0 : i0 - n0;
        for (int i1 = 0; i1 < n1; ++i1) {
            int64_t k1 = (2 * i1 < n1) ? i1 : i1 - n1;
            for (int k2 = 0; k2 < n2c; ++k2) {
                int64_t kk = k0 * k0 + k1 * k1 + (int64_t)k2 * k2;
                cplx* v = a + ((int64_t)i0 * n1 + i1) * n2c + k2;
                if (kk == 0) {
                    v->re = 0.0;
                    v->im = 0.0;
                } else {
                    double f = -scale / (double)kk;
                    v->re *= f;
                    v->im *= f;
                }
            }
        }
    }
}
