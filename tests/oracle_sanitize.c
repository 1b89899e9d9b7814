/* Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * CPU oracle (test infrastructure, compiled together with
 * oracle/sip_oracle.c by tests/test_oracle_sanitized.py).  It runs every
 * oracle entry point on small random diagonally dominant 7-point systems,
 * including degenerate shapes (single cells, lines, planes, prime extents)
 * and multi-block cuts, so that any out-of-bounds access, use of freed
 * memory, leak or undefined arithmetic (signed overflow, bad shifts) in the
 * oracle stops the process.  Exit status 0 means every call returned its
 * documented success code. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_factor(int ni, int nj, int nk, const double *A, double alpha, double *LU);
void oracle_residual(int ni, int nj, int nk, const double *A, const double *b, const double *x, double *r);
void oracle_residual_f32(int ni, int nj, int nk, const float *A, const float *b, const float *x, float *r);
double oracle_norm2(const double *v, size_t n);
void oracle_forward(int ni, int nj, int nk, const double *LU, const double *r, double *y);
void oracle_backward(int ni, int nj, int nk, const double *LU, const double *y, double *d);
void oracle_forward_f32(int ni, int nj, int nk, const float *LU, const float *r, float *y);
void oracle_backward_f32(int ni, int nj, int nk, const float *LU, const float *y, float *d);
long oracle_iterate(int ni, int nj, int nk, const double *A, const double *LU, const double *b, double *x,
                    long n_iter, int mode, double *hist);
long oracle_solve(int ni, int nj, int nk, const double *A, const double *LU, const double *b, double *x,
                  double rtol, long max_iter, int mode, double *hist, double *rel_res);
long oracle_blocks_run(int ni, int nj, int nk, const double *A, double alpha, const double *b, double *x,
                       int nbi, const int *ci, int nbj, const int *cj, int nbk, const int *ck, long n_iter,
                       double rtol, int mode, double *hist, double *rel_res);

static uint64_t state = 0x9e3779b97f4a7c15ull;

static double uni(void)   /* xorshift64*, in [0, 1) */
{
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 0x2545f4914f6cdd1dull) >> 11) * (1.0 / 9007199254740992.0);
}

/* Coefficients in the order P, W, E, S, N, B, T; couplings that leave the
 * block are zero, the diagonal exceeds the sum of the couplings. */
static void make_system(int ni, int nj, int nk, double *A, double *b, double *x)
{
    const size_t n = (size_t)ni * nj * nk;
    for (int k = 0; k < nk; k++)
        for (int j = 0; j < nj; j++)
            for (int i = 0; i < ni; i++) {
                const size_t p = ((size_t)k * nj + j) * ni + i;
                const int has[6] = {i > 0, i < ni - 1, j > 0, j < nj - 1, k > 0, k < nk - 1};
                double s = 0.0;
                for (int d = 0; d < 6; d++) {
                    const double a = has[d] ? -(0.2 + uni()) : 0.0;
                    A[(d + 1) * n + p] = a;
                    s -= a;
                }
                A[p] = s + 0.1 + uni();
                b[p] = 2.0 * uni() - 1.0;
                x[p] = 0.5 * uni() - 0.25;
            }
}

static int run_shape(int ni, int nj, int nk)
{
    const size_t n = (size_t)ni * nj * nk;
    double *A = malloc(7 * n * sizeof(double)), *LU = malloc(7 * n * sizeof(double));
    double *b = malloc(n * sizeof(double)), *x = malloc(n * sizeof(double)), *x0 = malloc(n * sizeof(double));
    double *r = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double)), *d = malloc(n * sizeof(double));
    float *A32 = malloc(7 * n * sizeof(float)), *LU32 = malloc(7 * n * sizeof(float));
    float *b32 = malloc(n * sizeof(float)), *x32 = malloc(n * sizeof(float)), *r32 = malloc(n * sizeof(float));
    float *y32 = malloc(n * sizeof(float)), *d32 = malloc(n * sizeof(float));
    double hist[41], rr = 0.0;
    int bad = 0;
    if (!A || !LU || !b || !x || !x0 || !r || !y || !d || !A32 || !LU32 || !b32 || !x32 || !r32 || !y32 || !d32) {
        fprintf(stderr, "allocation failed\n");
        return 1;
    }
    make_system(ni, nj, nk, A, b, x0);
    for (int a = 0; a <= 4; a++) {
        if (oracle_factor(ni, nj, nk, A, 0.25 * a, LU) != 0) {
            fprintf(stderr, "%dx%dx%d alpha %.2f: unexpected breakdown\n", ni, nj, nk, 0.25 * a);
            bad = 1;
        }
    }
    oracle_factor(ni, nj, nk, A, 0.92, LU);
    oracle_residual(ni, nj, nk, A, b, x0, r);
    oracle_forward(ni, nj, nk, LU, r, y);
    oracle_backward(ni, nj, nk, LU, y, d);
    for (size_t t = 0; t < 7 * n; t++) {
        A32[t] = (float)A[t];
        LU32[t] = (float)LU[t];
    }
    for (size_t t = 0; t < n; t++) {
        b32[t] = (float)b[t];
        x32[t] = (float)x0[t];
    }
    oracle_residual_f32(ni, nj, nk, A32, b32, x32, r32);
    oracle_forward_f32(ni, nj, nk, LU32, r32, y32);
    oracle_backward_f32(ni, nj, nk, LU32, y32, d32);
    if (!isfinite(oracle_norm2(d, n))) bad = 1;
    for (int mode = 0; mode < 3; mode++) {
        for (size_t t = 0; t < n; t++) x[t] = x0[t];
        if (oracle_iterate(ni, nj, nk, A, LU, b, x, 40, mode, hist) != 40) bad = 1;
        for (size_t t = 0; t < n; t++) x[t] = x0[t];
        const long it = oracle_solve(ni, nj, nk, A, LU, b, x, mode == 2 ? 1e-4 : 1e-8, 40, mode, hist, &rr);
        if (it < 0 || it > 40) bad = 1;
    }
    /* two blocks along the longest axis, one block when that axis has one cell */
    const int ext[3] = {ni, nj, nk};
    int ax = 0;
    for (int q = 1; q < 3; q++)
        if (ext[q] > ext[ax]) ax = q;
    int cut[3][3];
    int nb[3];
    for (int q = 0; q < 3; q++) {
        cut[q][0] = 0;
        if (q == ax && ext[q] > 1) {
            cut[q][1] = ext[q] / 2;
            cut[q][2] = ext[q];
            nb[q] = 2;
        } else {
            cut[q][1] = ext[q];
            nb[q] = 1;
        }
    }
    for (int mode = 0; mode < 2; mode++) {
        for (size_t t = 0; t < n; t++) x[t] = x0[t];
        if (oracle_blocks_run(ni, nj, nk, A, 0.92, b, x, nb[0], cut[0], nb[1], cut[1], nb[2], cut[2], 20, 0.0, mode,
                              hist, &rr) != 20)
            bad = 1;
    }
    if (bad) fprintf(stderr, "%dx%dx%d: a call did not return its success code\n", ni, nj, nk);
    free(A); free(LU); free(b); free(x); free(x0); free(r); free(y); free(d);
    free(A32); free(LU32); free(b32); free(x32); free(r32); free(y32); free(d32);
    return bad;
}

int main(void)
{
    static const int shapes[][3] = {{1, 1, 1}, {1, 1, 9}, {1, 9, 1}, {9, 1, 1}, {1, 5, 6}, {6, 1, 5}, {5, 6, 1},
                                    {2, 2, 2}, {3, 4, 5}, {17, 5, 3}, {7, 11, 13}, {16, 16, 16}};
    int bad = 0;
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); s++)
        bad |= run_shape(shapes[s][0], shapes[s][1], shapes[s][2]);
    if (!bad) printf("oracle sanitizer run: %zu shapes ok\n", sizeof(shapes) / sizeof(shapes[0]));
    return bad;
}
