/*
 * Plain FP64 CPU oracle for the array impedance operator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into oracle/_oracle.so and
 * is loaded by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  It shares no code with the GPU library and must never be reached
 * from the library's product path.
 *
 * Everything here is the definition written out, with loops in index order and
 * no blocking or reordering:
 *   - the impedance matrix of eq. (matrixForm): Z = [[A, B^T], [B, C]], where
 *     A is the two-level block-Toeplitz element-element part of eq.
 *     (submatrixAA) and B, C are the rim (margin) couplings;
 *   - y = Z x by rows;
 *   - Gaussian elimination with partial pivoting (Golub & Van Loan,
 *     Matrix Computations, Alg. 3.4.1);
 *   - the brute-force cyclic convolution that circulant embedding computes;
 *   - the 2-D DFT of the placed generators.
 *
 * Conventions (element order of Sec. II-C, x fastest; basis index minor):
 *   unknown (iy*Nx + ix)*b + p is basis p of element (ix, iy); unknown N + r is
 *   rim function r, N = Nx*Ny*b, Nt = N + Nr.
 *   gen[(n+Ny-1)][(m+Nx-1)][p][q] = Z_{m,n}[p][q] couples basis p of element
 *   (ix+m, iy+n) (row) to basis q of element (ix, iy) (column).
 *   rim_re[r][e]: rim row r, element column e.  rim_er[e][r] is the element-rim
 *   block; NULL means reciprocal (rim_er[e][r] = rim_re[r][e]).
 *   Complex numbers are interleaved (re, im) doubles.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int Nx, Ny, b, Nr;
    const cplx *gen, *rim_re, *rim_er, *rim_rr;
} orc_problem;

static long orc_N(const orc_problem *P) { return (long)P->Nx * P->Ny * P->b; }

/* Entry Z[i][j] of the full matrix, straight from eq. (matrixForm). */
static cplx orc_entry(const orc_problem *P, long i, long j)
{
    const long N = orc_N(P);
    const int b = P->b;
    if (i < N && j < N) {
        long ei = i / b, ej = j / b;
        int p = (int)(i % b), q = (int)(j % b);
        int ix = (int)(ei % P->Nx), iy = (int)(ei / P->Nx);
        int lx = (int)(ej % P->Nx), ly = (int)(ej / P->Nx);
        int m = ix - lx, n = iy - ly;
        long blk = (long)(n + P->Ny - 1) * (2 * P->Nx - 1) + (m + P->Nx - 1);
        return P->gen[(blk * b + p) * b + q];
    }
    if (i >= N && j < N)
        return P->rim_re[(i - N) * N + j];
    if (i < N && j >= N)
        return P->rim_er ? P->rim_er[i * P->Nr + (j - N)] : P->rim_re[(j - N) * N + i];
    return P->rim_rr[(i - N) * P->Nr + (j - N)];
}

static orc_problem mkprob(int Nx, int Ny, int b, int Nr, const double *gen, const double *rim_re,
                          const double *rim_er, const double *rim_rr)
{
    orc_problem P = {Nx, Ny, b, Nr, (const cplx *)gen, (const cplx *)rim_re,
                     (const cplx *)rim_er, (const cplx *)rim_rr};
    return P;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Dense Nt x Nt row-major assembly. */
void orc_assemble(int Nx, int Ny, int b, int Nr, const double *gen, const double *rim_re,
                  const double *rim_er, const double *rim_rr, double *Zout)
{
    orc_problem P = mkprob(Nx, Ny, b, Nr, gen, rim_re, rim_er, rim_rr);
    const long Nt = orc_N(&P) + Nr;
    cplx *Z = (cplx *)Zout;
    for (long i = 0; i < Nt; ++i)
        for (long j = 0; j < Nt; ++j) Z[i * Nt + j] = orc_entry(&P, i, j);
}

/*
 * y[r][i] = sum_j Z[i][j] x[r][j] for the listed rows i (all rows if rows ==
 * NULL).  x, y hold R vectors of length Nt back to back (column-major Nt x R).
 * When rows != NULL, y is R x nrows.  The sum over j runs in index order.
 */
void orc_matvec_rows(int Nx, int Ny, int b, int Nr, const double *gen, const double *rim_re,
                     const double *rim_er, const double *rim_rr, const double *xin, int R,
                     const long *rows, long nrows, double *yout, int nthreads)
{
    orc_problem P = mkprob(Nx, Ny, b, Nr, gen, rim_re, rim_er, rim_rr);
    const long Nt = orc_N(&P) + Nr;
    const cplx *x = (const cplx *)xin;
    cplx *y = (cplx *)yout;
    const long nr = rows ? nrows : Nt;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < nr; ++t) {
        long i = rows ? rows[t] : t;
        for (int r = 0; r < R; ++r) {
            cplx s = 0.0;
            for (long j = 0; j < Nt; ++j) s += orc_entry(&P, i, j) * x[(long)r * Nt + j];
            y[(long)r * nr + t] = s;
        }
    }
}

/* Same product with a dense row-major matrix (Nt x Nt), for assembled cases. */
void orc_dense_matvec(long n, const double *Zin, const double *xin, int R, double *yout, int nthreads)
{
    const cplx *Z = (const cplx *)Zin, *x = (const cplx *)xin;
    cplx *y = (cplx *)yout;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i)
        for (int r = 0; r < R; ++r) {
            cplx s = 0.0;
            for (long j = 0; j < n; ++j) s += Z[i * n + j] * x[(long)r * n + j];
            y[(long)r * n + i] = s;
        }
}

/*
 * Gaussian elimination with partial pivoting, in place on the row-major n x n
 * matrix A (Golub & Van Loan Alg. 3.4.1): pivot = largest modulus in the
 * column, ties to the smallest row index.  Then forward and back substitution
 * for the R right-hand sides in B (R x n, overwritten by the solutions).
 * Returns 0, or k+1 if the k-th pivot is exactly zero.
 */
int orc_lu_solve(long n, double *Ain, int R, double *Bin, int nthreads)
{
    cplx *A = (cplx *)Ain, *B = (cplx *)Bin;
    long *piv = (long *)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    set_threads(nthreads);
    for (long k = 0; k < n; ++k) {
        long p = k;
        double best = cabs(A[k * n + k]);
        for (long i = k + 1; i < n; ++i) {
            double a = cabs(A[i * n + k]);
            if (a > best) { best = a; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) { free(piv); return (int)(k + 1); }
        if (p != k)
            for (long j = 0; j < n; ++j) {
                cplx t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
            }
        const cplx akk = A[k * n + k];
#pragma omp parallel for schedule(static)
        for (long i = k + 1; i < n; ++i) {
            cplx l = A[i * n + k] / akk;
            A[i * n + k] = l;
            for (long j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    for (int r = 0; r < R; ++r) {
        cplx *bv = B + (long)r * n;
        for (long k = 0; k < n; ++k)
            if (piv[k] != k) { cplx t = bv[k]; bv[k] = bv[piv[k]]; bv[piv[k]] = t; }
        for (long i = 0; i < n; ++i) {           /* L y = P b, unit diagonal */
            cplx s = bv[i];
            for (long j = 0; j < i; ++j) s -= A[i * n + j] * bv[j];
            bv[i] = s;
        }
        for (long i = n - 1; i >= 0; --i) {      /* U x = y */
            cplx s = bv[i];
            for (long j = i + 1; j < n; ++j) s -= A[i * n + j] * bv[j];
            bv[i] = s / A[i * n + i];
        }
    }
    free(piv);
    return 0;
}

static long pmod(long a, long m) { long r = a % m; return r < 0 ? r + m : r; }

/*
 * Brute-force cyclic convolution of circulant embedding, element part only:
 *   c[(m mod Px), (n mod Py)] = Z_{m,n}, zero elsewhere;
 *   x_pad = x_A zero-padded to the Px x Py grid;
 *   y_c(i) = sum_j c[(i - j) mod P] x_pad(j) over every grid point j;
 *   y_A = y_c cropped to the first Nx x Ny grid points.
 * Requires Px >= 2Nx-1, Py >= 2Ny-1 for the identity with the dense A.
 */
void orc_circulant_product(int Nx, int Ny, int b, const double *genin, int Px, int Py,
                           const double *xin, double *yout)
{
    const cplx *gen = (const cplx *)genin, *x = (const cplx *)xin;
    cplx *y = (cplx *)yout;
    const long bb = (long)b * b;
    cplx *c = (cplx *)calloc((size_t)Px * Py * bb, sizeof(cplx));
    cplx *xp = (cplx *)calloc((size_t)Px * Py * b, sizeof(cplx));
    for (int n = -(Ny - 1); n <= Ny - 1; ++n)
        for (int m = -(Nx - 1); m <= Nx - 1; ++m) {
            const cplx *src = gen + ((long)(n + Ny - 1) * (2 * Nx - 1) + (m + Nx - 1)) * bb;
            cplx *dst = c + (pmod(n, Py) * Px + pmod(m, Px)) * bb;
            for (long t = 0; t < bb; ++t) dst[t] = src[t];
        }
    for (int jy = 0; jy < Ny; ++jy)
        for (int jx = 0; jx < Nx; ++jx)
            for (int q = 0; q < b; ++q)
                xp[((long)jy * Px + jx) * b + q] = x[((long)jy * Nx + jx) * b + q];
    for (int iy = 0; iy < Ny; ++iy)
        for (int ix = 0; ix < Nx; ++ix)
            for (int p = 0; p < b; ++p) {
                cplx s = 0.0;
                for (int jy = 0; jy < Py; ++jy)
                    for (int jx = 0; jx < Px; ++jx) {
                        const cplx *blk = c + (pmod(iy - jy, Py) * Px + pmod(ix - jx, Px)) * bb;
                        const cplx *xv = xp + ((long)jy * Px + jx) * b;
                        for (int q = 0; q < b; ++q) s += blk[(long)p * b + q] * xv[q];
                    }
                y[((long)iy * Nx + ix) * b + p] = s;
            }
    free(c);
    free(xp);
}

/*
 * Spectrum of the placed generators at the listed frequencies:
 *   G[k] = (1/(Px Py)) sum_{gx,gy} c[gx,gy] exp(-2 pi i (kx gx / Px + ky gy / Py))
 * with c the placed grid of orc_circulant_product.  out[t] is the b x b block
 * (row-major) for frequency (kx[t], ky[t]).
 */
void orc_spectrum(int Nx, int Ny, int b, const double *genin, int Px, int Py, const int *kx,
                  const int *ky, long nk, double *outp, int nthreads)
{
    const cplx *gen = (const cplx *)genin;
    cplx *out = (cplx *)outp;
    const long bb = (long)b * b;
    const double two_pi = 6.283185307179586476925286766559;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < nk; ++t) {
        cplx *o = out + t * bb;
        for (long e = 0; e < bb; ++e) o[e] = 0.0;
        for (int gy = 0; gy < Py; ++gy)
            for (int gx = 0; gx < Px; ++gx) {
                /* which generator sits at grid point (gx, gy), if any */
                int m = gx <= Nx - 1 ? gx : gx - Px;
                int n = gy <= Ny - 1 ? gy : gy - Py;
                if (m < -(Nx - 1) || n < -(Ny - 1)) continue;   /* zero padding */
                double ph = two_pi * ((double)pmod((long)kx[t] * gx, Px) / Px +
                                      (double)pmod((long)ky[t] * gy, Py) / Py);
                cplx w = cos(ph) - I * sin(ph);
                const cplx *src = gen + ((long)(n + Ny - 1) * (2 * Nx - 1) + (m + Nx - 1)) * bb;
                for (long e = 0; e < bb; ++e) o[e] += src[e] * w;
            }
        for (long e = 0; e < bb; ++e) o[e] /= (double)Px * (double)Py;
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
