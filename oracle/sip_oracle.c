/*
 * sip_oracle.c -- plain, single-threaded FP64 reference of Stone's strongly
 * implicit procedure (SIP) on one structured 3D block, 7-point stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * GPU implementation.
 *
 * Source of the method: the paper (arXiv:1303.4538) names SIP, a solver
 * built on an approximate (incomplete) LU factorisation, as the linear solver
 * of FASTEST-3D (Sec. 1) and cites Stone (1968) for it; Sec. 4.1 describes the solver structure
 * (factorisation computed once in advance, then forward/backward substitution
 * sweeps, residual computed as part of the forward step).  The paper does not
 * print the equations; they are written here from Stone's construction:
 *
 *   M = L U = A + N, L lower with the B, W, S, P diagonals, U unit upper with
 *   the N, E, T diagonals.  The product L U has six diagonals that A lacks
 *   (positions BN, BE, WN, WT, SE, ST).  N cancels each such entry e at
 *   position Q partially, by the linear extrapolation
 *       phi_Q ~ alpha (phi_Q1 + phi_Q2 - phi_P),
 *   where Q1, Q2 are the two stencil neighbours that span Q (e.g. SE -> S, E).
 *   Matching M = A + N on the seven stencil positions gives, per cell P
 *   visited in lexicographic order (W, S, B before P; X_B means X at cell B):
 *
 *   Lb = A_B / (1 + alpha (Un_B + Ue_B))
 *   Lw = A_W / (1 + alpha (Un_W + Ut_W))
 *   Ls = A_S / (1 + alpha (Ue_S + Ut_S))
 *   P1 = alpha (Lb Un_B + Lw Un_W)   (N-position compensation)
 *   P2 = alpha (Ls Ue_S + Lb Ue_B)   (E-position compensation)
 *   P3 = alpha (Ls Ut_S + Lw Ut_W)   (T-position compensation)
 *   Lp = A_P + P1 + P2 + P3 - Lb Ut_B - Lw Ue_W - Ls Un_S
 *   Un = (A_N - P1) / Lp,  Ue = (A_E - P2) / Lp,  Ut = (A_T - P3) / Lp
 *
 * Iteration (defect correction with the approximate factorisation):
 *   r = b - A x              (FP64)
 *   rho_n = ||r||_2 / ||b||_2
 *   forward  (lexicographic): y_P = (r_P - Lb y_B - Lw y_W - Ls y_S) / Lp
 *   backward (reverse order): d_P = y_P - Un d_N - Ue d_E - Ut d_T
 *   x <- x + d
 *
 * Conventions (readings where the paper is silent):
 *   - signed coefficients: row P reads A_P x_P + sum_nb A_nb x_nb = b_P
 *     (the paper's listing in Sec. 4.1 stores a_nb = -A_nb and su = b);
 *   - arrays hold interior cells only, C order [nk][nj][ni] (i fastest);
 *     a coupling that points out of the block is ignored (treated as 0);
 *   - coefficient array order P, W, E, S, N, B, T; factor array order
 *     Lb, Lw, Ls, Lp, Un, Ue, Ut;
 *   - true IEEE division; built with -ffp-contract=off.
 * Mixed form: factors computed in FP64 then rounded to FP32, r rounded to
 * FP32 before the forward sweep, both sweeps in FP32, d widened to FP64;
 * residual, norm and update stay FP64.
 * All-FP32 form (the single-precision relaxation of Sec. 4.1: b and x are
 * converted to single precision before the sweeps and only x is converted
 * back afterwards): A, the factors (computed in FP64), b and x are rounded
 * to FP32 on entry; residual, both sweeps and the update x += d run in FP32;
 * x is widened to FP64 on exit.  rho_n is the norm of the FP32 residual over
 * the norm of the FP32 b, each summed in FP64 (a reading: the paper does not
 * say how the norm is summed).
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>

enum { AP = 0, AW = 1, AE = 2, AS = 3, AN = 4, AB = 5, AT = 6 };
enum { LB = 0, LW = 1, LS = 2, LP = 3, UN = 4, UE = 5, UT = 6 };

#define IDX(i, j, k) ((size_t)(i) + (size_t)ni * ((size_t)(j) + (size_t)nj * (size_t)(k)))

/* Factorisation, Stone's construction above.  Returns 0, or -1 on a zero /
 * non-finite pivot or a zero denominator.  A and LU are 7*N arrays. */
int oracle_factor(int ni, int nj, int nk, const double *A, double alpha, double *LU)
{
    const size_t n = (size_t)ni * nj * nk;
    const double *aP = A + AP * n, *aW = A + AW * n, *aE = A + AE * n, *aS = A + AS * n,
                 *aN = A + AN * n, *aB = A + AB * n, *aT = A + AT * n;
    double *Lb = LU + LB * n, *Lw = LU + LW * n, *Ls = LU + LS * n, *Lp = LU + LP * n,
           *Un = LU + UN * n, *Ue = LU + UE * n, *Ut = LU + UT * n;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < nj; j++)
            for (int i = 0; i < ni; i++) {
                const size_t p = IDX(i, j, k);
                /* U entries of the W, S, B neighbours; zero outside the block */
                double unB = 0, ueB = 0, utB = 0, unW = 0, ueW = 0, utW = 0, unS = 0, ueS = 0, utS = 0;
                if (k > 0) { size_t q = IDX(i, j, k - 1); unB = Un[q]; ueB = Ue[q]; utB = Ut[q]; }
                if (i > 0) { size_t q = IDX(i - 1, j, k); unW = Un[q]; ueW = Ue[q]; utW = Ut[q]; }
                if (j > 0) { size_t q = IDX(i, j - 1, k); unS = Un[q]; ueS = Ue[q]; utS = Ut[q]; }
                const double cB = (k > 0) ? aB[p] : 0.0;
                const double cW = (i > 0) ? aW[p] : 0.0;
                const double cS = (j > 0) ? aS[p] : 0.0;
                const double cN = (j < nj - 1) ? aN[p] : 0.0;
                const double cE = (i < ni - 1) ? aE[p] : 0.0;
                const double cT = (k < nk - 1) ? aT[p] : 0.0;
                const double denB = 1.0 + alpha * (unB + ueB);
                const double denW = 1.0 + alpha * (unW + utW);
                const double denS = 1.0 + alpha * (ueS + utS);
                if (denB == 0.0 || denW == 0.0 || denS == 0.0) return -1;
                const double lb = cB / denB;
                const double lw = cW / denW;
                const double ls = cS / denS;
                const double p1 = alpha * (lb * unB + lw * unW);
                const double p2 = alpha * (ls * ueS + lb * ueB);
                const double p3 = alpha * (ls * utS + lw * utW);
                const double lp = aP[p] + p1 + p2 + p3 - lb * utB - lw * ueW - ls * unS;
                if (lp == 0.0 || !isfinite(lp)) return -1;
                Lb[p] = lb; Lw[p] = lw; Ls[p] = ls; Lp[p] = lp;
                Un[p] = (cN - p1) / lp;
                Ue[p] = (cE - p2) / lp;
                Ut[p] = (cT - p3) / lp;
            }
    return 0;
}

/* r = b - A x over the 7-point stencil, outward couplings ignored. */
void oracle_residual(int ni, int nj, int nk, const double *A, const double *b, const double *x, double *r)
{
    const size_t n = (size_t)ni * nj * nk;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < nj; j++)
            for (int i = 0; i < ni; i++) {
                const size_t p = IDX(i, j, k);
                double ax = A[AP * n + p] * x[p];
                if (i > 0) ax += A[AW * n + p] * x[IDX(i - 1, j, k)];
                if (i < ni - 1) ax += A[AE * n + p] * x[IDX(i + 1, j, k)];
                if (j > 0) ax += A[AS * n + p] * x[IDX(i, j - 1, k)];
                if (j < nj - 1) ax += A[AN * n + p] * x[IDX(i, j + 1, k)];
                if (k > 0) ax += A[AB * n + p] * x[IDX(i, j, k - 1)];
                if (k < nk - 1) ax += A[AT * n + p] * x[IDX(i, j, k + 1)];
                r[p] = b[p] - ax;
            }
}

/* All-FP32 form: r = b - A x with every product and sum in FP32, the terms
 * added in the order P, W, E, S, N, B, T. */
void oracle_residual_f32(int ni, int nj, int nk, const float *A, const float *b, const float *x, float *r)
{
    const size_t n = (size_t)ni * nj * nk;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < nj; j++)
            for (int i = 0; i < ni; i++) {
                const size_t p = IDX(i, j, k);
                float ax = A[AP * n + p] * x[p];
                if (i > 0) ax += A[AW * n + p] * x[IDX(i - 1, j, k)];
                if (i < ni - 1) ax += A[AE * n + p] * x[IDX(i + 1, j, k)];
                if (j > 0) ax += A[AS * n + p] * x[IDX(i, j - 1, k)];
                if (j < nj - 1) ax += A[AN * n + p] * x[IDX(i, j + 1, k)];
                if (k > 0) ax += A[AB * n + p] * x[IDX(i, j, k - 1)];
                if (k < nk - 1) ax += A[AT * n + p] * x[IDX(i, j, k + 1)];
                r[p] = b[p] - ax;
            }
}

/* Euclidean norm of an FP32 vector, squares summed in FP64. */
static double norm2_f32(const float *v, size_t n)
{
    double s = 0.0;
    for (size_t p = 0; p < n; p++) s += (double)v[p] * (double)v[p];
    return sqrt(s);
}

/* Euclidean norm, summed in lexicographic order. */
double oracle_norm2(const double *v, size_t n)
{
    double s = 0.0;
    for (size_t p = 0; p < n; p++) s += v[p] * v[p];
    return sqrt(s);
}

/* Forward substitution L y = r in lexicographic order. */
void oracle_forward(int ni, int nj, int nk, const double *LU, const double *r, double *y)
{
    const size_t n = (size_t)ni * nj * nk;
    const double *Lb = LU + LB * n, *Lw = LU + LW * n, *Ls = LU + LS * n, *Lp = LU + LP * n;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < nj; j++)
            for (int i = 0; i < ni; i++) {
                const size_t p = IDX(i, j, k);
                double t = r[p];
                if (k > 0) t -= Lb[p] * y[IDX(i, j, k - 1)];
                if (i > 0) t -= Lw[p] * y[IDX(i - 1, j, k)];
                if (j > 0) t -= Ls[p] * y[IDX(i, j - 1, k)];
                y[p] = t / Lp[p];
            }
}

/* Backward substitution U d = y in reverse lexicographic order. */
void oracle_backward(int ni, int nj, int nk, const double *LU, const double *y, double *d)
{
    const size_t n = (size_t)ni * nj * nk;
    const double *Un = LU + UN * n, *Ue = LU + UE * n, *Ut = LU + UT * n;
    for (int k = nk - 1; k >= 0; k--)
        for (int j = nj - 1; j >= 0; j--)
            for (int i = ni - 1; i >= 0; i--) {
                const size_t p = IDX(i, j, k);
                double t = y[p];
                if (j < nj - 1) t -= Un[p] * d[IDX(i, j + 1, k)];
                if (i < ni - 1) t -= Ue[p] * d[IDX(i + 1, j, k)];
                if (k < nk - 1) t -= Ut[p] * d[IDX(i, j, k + 1)];
                d[p] = t;
            }
}

/* Mixed-form sweeps: FP32 factors, FP32 right-hand side, FP32 arithmetic. */
void oracle_forward_f32(int ni, int nj, int nk, const float *LU, const float *r, float *y)
{
    const size_t n = (size_t)ni * nj * nk;
    const float *Lb = LU + LB * n, *Lw = LU + LW * n, *Ls = LU + LS * n, *Lp = LU + LP * n;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < nj; j++)
            for (int i = 0; i < ni; i++) {
                const size_t p = IDX(i, j, k);
                float t = r[p];
                if (k > 0) t -= Lb[p] * y[IDX(i, j, k - 1)];
                if (i > 0) t -= Lw[p] * y[IDX(i - 1, j, k)];
                if (j > 0) t -= Ls[p] * y[IDX(i, j - 1, k)];
                y[p] = t / Lp[p];
            }
}

void oracle_backward_f32(int ni, int nj, int nk, const float *LU, const float *y, float *d)
{
    const size_t n = (size_t)ni * nj * nk;
    const float *Un = LU + UN * n, *Ue = LU + UE * n, *Ut = LU + UT * n;
    for (int k = nk - 1; k >= 0; k--)
        for (int j = nj - 1; j >= 0; j--)
            for (int i = ni - 1; i >= 0; i--) {
                const size_t p = IDX(i, j, k);
                float t = y[p];
                if (j < nj - 1) t -= Un[p] * d[IDX(i, j + 1, k)];
                if (i < ni - 1) t -= Ue[p] * d[IDX(i + 1, j, k)];
                if (k < nk - 1) t -= Ut[p] * d[IDX(i, j, k + 1)];
                d[p] = t;
            }
}

/* All-FP32 driver (mode 2 of the shared driver below). */
static long oracle_run_f32(int ni, int nj, int nk, const double *A, const double *LU, const double *b,
                           double *x, long n_iter, double rtol, double *hist, double *rel_res)
{
    const size_t n = (size_t)ni * nj * nk;
    float *A32 = malloc(7 * n * sizeof(float)), *LU32 = malloc(7 * n * sizeof(float));
    float *b32 = malloc(n * sizeof(float)), *x32 = malloc(n * sizeof(float));
    float *r32 = malloc(n * sizeof(float)), *y32 = malloc(n * sizeof(float)), *d32 = malloc(n * sizeof(float));
    long it = -1;
    if (!A32 || !LU32 || !b32 || !x32 || !r32 || !y32 || !d32) goto out;
    for (size_t q = 0; q < 7 * n; q++) {
        A32[q] = (float)A[q];
        LU32[q] = (float)LU[q];
    }
    for (size_t p = 0; p < n; p++) {
        b32[p] = (float)b[p];
        x32[p] = (float)x[p];
    }
    const double nb = norm2_f32(b32, n);
    if (nb == 0.0) {
        for (size_t p = 0; p < n; p++) x[p] = 0.0;
        if (hist) for (long m = 0; m <= n_iter; m++) hist[m] = 0.0;
        if (rel_res) *rel_res = 0.0;
        it = 0;
        goto out;
    }
    double rho = 0.0;
    for (it = 0;; it++) {
        oracle_residual_f32(ni, nj, nk, A32, b32, x32, r32);
        rho = norm2_f32(r32, n) / nb;
        if (hist) hist[it] = rho;
        if (it >= n_iter) break;
        if (rtol > 0.0 && rho <= rtol) break;
        oracle_forward_f32(ni, nj, nk, LU32, r32, y32);
        oracle_backward_f32(ni, nj, nk, LU32, y32, d32);
        for (size_t p = 0; p < n; p++) x32[p] = x32[p] + d32[p];
    }
    for (size_t p = 0; p < n; p++) x[p] = (double)x32[p];
    if (rel_res) *rel_res = rho;
out:
    free(A32); free(LU32); free(b32); free(x32); free(r32); free(y32); free(d32);
    return it;
}

/* Shared driver.  mode 0: FP64 sweeps; mode 1: mixed form; mode 2: all-FP32
 * form.
 * Stops after n_iter updates, or (rtol > 0) at the first n with
 * rho_n <= rtol, leaving x = x^n.  hist (nullable) receives rho_0..rho_n.
 * Returns the number of updates applied, or -1 on allocation failure.
 * *rel_res receives the relative residual of the returned x. */
static long oracle_run(int ni, int nj, int nk, const double *A, const double *LU, const double *b,
                       double *x, long n_iter, double rtol, int mode, double *hist, double *rel_res)
{
    if (mode == 2) return oracle_run_f32(ni, nj, nk, A, LU, b, x, n_iter, rtol, hist, rel_res);
    const size_t n = (size_t)ni * nj * nk;
    const double nb = oracle_norm2(b, n);
    if (nb == 0.0) {
        for (size_t p = 0; p < n; p++) x[p] = 0.0;
        if (hist) for (long m = 0; m <= n_iter; m++) hist[m] = 0.0;
        if (rel_res) *rel_res = 0.0;
        return 0;
    }
    double *r = malloc(n * sizeof(double));
    double *y = malloc(n * sizeof(double));
    double *d = malloc(n * sizeof(double));
    float *LU32 = NULL, *r32 = NULL, *y32 = NULL, *d32 = NULL;
    if (mode == 1) {
        LU32 = malloc(7 * n * sizeof(float));
        r32 = malloc(n * sizeof(float));
        y32 = malloc(n * sizeof(float));
        d32 = malloc(n * sizeof(float));
    }
    if (!r || !y || !d || (mode == 1 && (!LU32 || !r32 || !y32 || !d32))) {
        free(r); free(y); free(d); free(LU32); free(r32); free(y32); free(d32);
        return -1;
    }
    if (mode == 1)
        for (size_t q = 0; q < 7 * n; q++) LU32[q] = (float)LU[q];
    long it = 0;
    double rho = 0.0;
    for (;;) {
        oracle_residual(ni, nj, nk, A, b, x, r);
        rho = oracle_norm2(r, n) / nb;
        if (hist) hist[it] = rho;
        if (it >= n_iter) break;
        if (rtol > 0.0 && rho <= rtol) break;
        if (mode == 0) {
            oracle_forward(ni, nj, nk, LU, r, y);
            oracle_backward(ni, nj, nk, LU, y, d);
            for (size_t p = 0; p < n; p++) x[p] += d[p];
        } else {
            for (size_t p = 0; p < n; p++) r32[p] = (float)r[p];
            oracle_forward_f32(ni, nj, nk, LU32, r32, y32);
            oracle_backward_f32(ni, nj, nk, LU32, y32, d32);
            for (size_t p = 0; p < n; p++) x[p] += (double)d32[p];
        }
        it++;
    }
    if (rel_res) *rel_res = rho;
    free(r); free(y); free(d); free(LU32); free(r32); free(y32); free(d32);
    return it;
}

/* n_iter plain SIP iterations from x (in/out); hist has n_iter+1 entries.
 * mode: 0 FP64, 1 mixed form, 2 all-FP32 form. */
long oracle_iterate(int ni, int nj, int nk, const double *A, const double *LU, const double *b,
                    double *x, long n_iter, int mode, double *hist)
{
    return oracle_run(ni, nj, nk, A, LU, b, x, n_iter, 0.0, mode, hist, NULL);
}

/* Iterate until rho_n <= rtol or max_iter updates; returns iterations. */
long oracle_solve(int ni, int nj, int nk, const double *A, const double *LU, const double *b,
                  double *x, double rtol, long max_iter, int mode, double *hist, double *rel_res)
{
    return oracle_run(ni, nj, nk, A, LU, b, x, max_iter, rtol, mode, hist, rel_res);
}

/* ------------------------------------------------------------------------
 * Multi-block domain (Sec. 4.2: each block runs its own SIP solver; blocks
 * are coupled only through values at block boundaries exchanged once per
 * iteration, every block receiving the values of the same previous iterate,
 * as with the non-blocking exchange that completes all transfers before any
 * received value is used).  The domain of ni x nj x nk cells is cut into
 * nbi x nbj x nbk blocks at the planes ci[0..nbi] (ci[0] = 0, ci[nbi] = ni),
 * cj, ck.  Each block is factorised on its own (couplings that leave the
 * block are ignored by the factorisation); one iteration computes the
 * residual of the whole domain with every coupling, r = b - A x (this is
 * where neighbour values enter), and each block applies its own forward and
 * backward substitution to its part of r.  mode 0: FP64; mode 1: mixed form
 * (r rounded to FP32, FP32 factors and sweeps).  Returns the number of
 * updates, -1 on allocation failure, -2 on a breakdown in some block.
 * ---------------------------------------------------------------------- */
long oracle_blocks_run(int ni, int nj, int nk, const double *A, double alpha, const double *b, double *x,
                       int nbi, const int *ci, int nbj, const int *cj, int nbk, const int *ck, long n_iter,
                       double rtol, int mode, double *hist, double *rel_res)
{
    const size_t n = (size_t)ni * nj * nk;
    const int nblk = nbi * nbj * nbk;
    double **LU = calloc((size_t)nblk, sizeof(double *));
    float **LU32 = calloc((size_t)nblk, sizeof(float *));
    double *r = malloc(n * sizeof(double)), *rb = malloc(n * sizeof(double)), *yb = malloc(n * sizeof(double));
    double *db = malloc(n * sizeof(double)), *Ab = malloc(7 * n * sizeof(double));
    float *r32 = malloc(n * sizeof(float)), *y32 = malloc(n * sizeof(float)), *d32 = malloc(n * sizeof(float));
    long it = -1;
    if (!LU || !LU32 || !r || !rb || !yb || !db || !Ab || !r32 || !y32 || !d32) goto out;
    /* factorise every block on its own */
    for (int q = 0; q < nblk; q++) {
        const int bi = q % nbi, bj = (q / nbi) % nbj, bk = q / (nbi * nbj);
        const int mi = ci[bi + 1] - ci[bi], mj = cj[bj + 1] - cj[bj], mk = ck[bk + 1] - ck[bk];
        const size_t m = (size_t)mi * mj * mk;
        for (int d = 0; d < 7; d++)
            for (int k = 0; k < mk; k++)
                for (int j = 0; j < mj; j++)
                    for (int i = 0; i < mi; i++)
                        Ab[d * m + ((size_t)k * mj + j) * mi + i] =
                            A[d * n + IDX(ci[bi] + i, cj[bj] + j, ck[bk] + k)];
        LU[q] = malloc(7 * m * sizeof(double));
        if (!LU[q]) goto out;
        if (oracle_factor(mi, mj, mk, Ab, alpha, LU[q]) != 0) {
            it = -2;
            goto out;
        }
        if (mode == 1) {
            LU32[q] = malloc(7 * m * sizeof(float));
            if (!LU32[q]) goto out;
            for (size_t t = 0; t < 7 * m; t++) LU32[q][t] = (float)LU[q][t];
        }
    }
    const double nb = oracle_norm2(b, n);
    if (nb == 0.0) {
        for (size_t p = 0; p < n; p++) x[p] = 0.0;
        if (hist) for (long m = 0; m <= n_iter; m++) hist[m] = 0.0;
        if (rel_res) *rel_res = 0.0;
        it = 0;
        goto out;
    }
    double rho = 0.0;
    for (it = 0;; it++) {
        oracle_residual(ni, nj, nk, A, b, x, r);   /* every coupling: neighbour values enter here */
        rho = oracle_norm2(r, n) / nb;
        if (hist) hist[it] = rho;
        if (it >= n_iter) break;
        if (rtol > 0.0 && rho <= rtol) break;
        for (int q = 0; q < nblk; q++) {
            const int bi = q % nbi, bj = (q / nbi) % nbj, bk = q / (nbi * nbj);
            const int mi = ci[bi + 1] - ci[bi], mj = cj[bj + 1] - cj[bj], mk = ck[bk + 1] - ck[bk];
            const size_t m = (size_t)mi * mj * mk;
            for (int k = 0; k < mk; k++)
                for (int j = 0; j < mj; j++)
                    for (int i = 0; i < mi; i++)
                        rb[((size_t)k * mj + j) * mi + i] = r[IDX(ci[bi] + i, cj[bj] + j, ck[bk] + k)];
            if (mode == 0) {
                oracle_forward(mi, mj, mk, LU[q], rb, yb);
                oracle_backward(mi, mj, mk, LU[q], yb, db);
            } else {
                for (size_t t = 0; t < m; t++) r32[t] = (float)rb[t];
                oracle_forward_f32(mi, mj, mk, LU32[q], r32, y32);
                oracle_backward_f32(mi, mj, mk, LU32[q], y32, d32);
                for (size_t t = 0; t < m; t++) db[t] = (double)d32[t];
            }
            for (int k = 0; k < mk; k++)
                for (int j = 0; j < mj; j++)
                    for (int i = 0; i < mi; i++)
                        x[IDX(ci[bi] + i, cj[bj] + j, ck[bk] + k)] += db[((size_t)k * mj + j) * mi + i];
        }
    }
    if (rel_res) *rel_res = rho;
out:
    if (LU) for (int q = 0; q < nblk; q++) free(LU[q]);
    if (LU32) for (int q = 0; q < nblk; q++) free(LU32[q]);
    free(LU); free(LU32); free(r); free(rb); free(yb); free(db); free(Ab); free(r32); free(y32); free(d32);
    return it;
}
