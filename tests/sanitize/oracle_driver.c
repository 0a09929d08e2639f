/* Exercises every entry point of the C oracle on small and ragged grids,
 * both boundary rules, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer can report out-of-bounds accesses, leaks and
 * undefined arithmetic in the oracle itself.  Test infrastructure only: it
 * is compiled and run by tests/test_sanitize_oracle.py. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef void (*oracle_step_cb)(int t, const double *u_t, double e_t, double r_t, void *ctx);
int oracle_run(int64_t nx, int64_t ny, int64_t nz, const double *u0, const double *f, double alpha,
               double beta, double gamma, double h, double dt, int bc, int T, double *uT, double *energy,
               double *resid);
int oracle_run_stream(int64_t nx, int64_t ny, int64_t nz, const double *u0, const double *f, double alpha,
                      double beta, double gamma, double h, double dt, int bc, int T, oracle_step_cb cb,
                      void *ctx);
int oracle_run_box(int64_t nx, int64_t ny, int64_t nz, const double *u0, const double *f, double alpha,
                   double beta, double gamma, double h, double dt, int bc, int T, const int64_t blo[3],
                   const int64_t bhi[3], double *out);
int oracle_adjoint(int64_t nx, int64_t ny, int64_t nz, const double *u0, const double *f, const double *lamT,
                   double alpha, double beta, double gamma, double h, double dt, int bc, int T,
                   double *grad_u0, double *grad_ab, double *grad_f, double *grad_gamma);
double oracle_half_sq_dist(int64_t n, const double *a, const double *b);
int oracle_jacobi_1d(int32_t tsteps, int64_t n, double *A, double *B);
int oracle_jacobi_1d_box(int32_t tsteps, int64_t n, int64_t c0, int64_t h1, double *A, double *B);
int oracle_jacobi_2d(int32_t tsteps, int64_t n0, int64_t n1, double *A, double *B);
int oracle_jacobi_2d_box(int32_t tsteps, int64_t n0, int64_t n1, int64_t r0, int64_t c0, int64_t h0, int64_t h1,
                         double *A, double *B);

static uint64_t state = 88172645463325252ull;
static double rnd(void) {  /* xorshift64, uniform in [-1, 1) */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
static double *field(int64_t n) {
    double *p = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) p[i] = rnd();
    return p;
}
static double seen;
static void cb(int t, const double *u, double e, double r, void *ctx) {
    (void)ctx;
    seen += u[0] + e + r + t;
}

int main(void) {
    const int64_t shapes[][3] = {{1, 1, 1}, {2, 1, 3}, {5, 4, 3}, {7, 3, 9}, {4, 6, 2}};
    int bad = 0;
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int64_t nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2], n = nx * ny * nz;
        for (int bc = 0; bc < 2; ++bc) {
            const int T = 4;
            double *u0 = field(n), *f = field(n), *lam = field(n);
            double *uT = field(n), *e = field(T), *r = field(T), *gu = field(n), *gf = field(n);
            double gab[2], gg;
            bad |= oracle_run(nx, ny, nz, u0, f, 1.0, 0.1, 0.5, 1.0, 0.1, bc, T, uT, e, r) != 0;
            bad |= oracle_run_stream(nx, ny, nz, u0, f, 1.0, 0.1, 0.5, 1.0, 0.1, bc, T, cb, NULL) != 0;
            const int64_t lo[3] = {0, 0, nz / 2}, hi[3] = {nx, ny, nz};
            double *box = field(nx * ny * (nz - nz / 2));
            bad |= oracle_run_box(nx, ny, nz, u0, f, 1.0, 0.1, 0.5, 1.0, 0.1, bc, T, lo, hi, box) != 0;
            bad |= oracle_adjoint(nx, ny, nz, u0, f, lam, 1.0, 0.1, 0.5, 1.0, 0.1, bc, T, gu, gab, gf, &gg) != 0;
            bad |= oracle_adjoint(nx, ny, nz, u0, f, lam, 1.0, 0.1, 0.5, 1.0, 0.1, bc, 0, gu, gab, NULL, NULL) != 0;
            seen += oracle_half_sq_dist(n, uT, u0) + gab[0] + gab[1] + gg + box[0] + e[T - 1] + r[T - 1];
            free(u0); free(f); free(lam); free(uT); free(e); free(r); free(gu); free(gf); free(box);
        }
    }
    for (int64_t n = 0; n < 9; ++n) {
        double *A = field(n), *B = field(n);
        bad |= oracle_jacobi_1d(5, n, A, B) != 0;
        if (n >= 3) bad |= oracle_jacobi_1d_box(5, n, 1, n - 2, A, B) != 0;
        free(A); free(B);
    }
    const int64_t sh2[][2] = {{1, 1}, {3, 3}, {4, 7}, {9, 5}};
    for (size_t s = 0; s < sizeof sh2 / sizeof sh2[0]; ++s) {
        const int64_t n0 = sh2[s][0], n1 = sh2[s][1];
        double *A = field(n0 * n1), *B = field(n0 * n1);
        bad |= oracle_jacobi_2d(4, n0, n1, A, B) != 0;
        if (n0 >= 3 && n1 >= 3) bad |= oracle_jacobi_2d_box(4, n0, n1, 1, 1, n0 - 2, n1 - 2, A, B) != 0;
        free(A); free(B);
    }
    printf("oracle driver: %s (checksum %.6g)\n", bad ? "an entry point returned an error" : "ok", seen);
    return bad || !isfinite(seen);
}
