/*
 * jacobi_oracle.c -- plain, serial, FP64 CPU oracle for the two Jacobi
 * stencil programs that the paper lists.
 *
 * TEST INFRASTRUCTURE ONLY.  Like rd3d_oracle.c, this is the slow, obviously
 * correct reference the GPU library is checked against.  It shares no code,
 * header, table or constant with the GPU path, and only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * What it follows:
 *   - Sec. 2.2, "Static symbolic typing": jacobi_1d on two float64 vectors of
 *     length N.  Each pass of its time loop first sets every interior element
 *     of B to 0.33333 times the sum of A's element and its two neighbours
 *     (left, centre, right, added in that order), then sets every interior
 *     element of A the same way from B.  The loop runs for t = 1 .. TSTEPS-1,
 *     that is TSTEPS-1 times (none when TSTEPS <= 1).  Elements 0 and N-1 of
 *     both vectors are never written.
 *   - Sec. 4.3, "Assuming Direct Control via Local Views": jacobi_2d, the
 *     same loop on two float64 N x N arrays with the five-point average:
 *     0.2 times (centre + west + east + south + north), added in that order,
 *     where west/east are the column neighbours j-1/j+1 and south/north the
 *     row neighbours i+1/i-1.  Only the interior [1, N-2] x [1, N-2] is
 *     written.  The array may also be n0 x n1 (the listing's case is square).
 *   - Python evaluates a + b + c left to right and the scale last, so each
 *     new value here is ((..(c0 + c1) + ..) + ck) * w, every operation
 *     rounded once (gcc -ffp-contract=off).  The right-hand side of each
 *     slice assignment reads only the other array, so evaluating it point
 *     by point equals NumPy's whole-slice evaluation bit for bit.
 *
 * Window forms (_box): the arrays hold only the cells [r0, r0+h0) x
 * [c0, c0+h1) of the global n0 x n1 arrays (1D: [c0, c0+h1) of n).  A cell is
 * updated if it is a global interior cell and all its stencil neighbours lie
 * inside the window; the other cells keep their values.  After s half-steps
 * a cell whose distance to every window edge that is not a global edge
 * exceeds s holds exactly the value the full-array program gives it.  With
 * the window equal to the whole array this is the listing itself.
 *
 * Layout: row-major, element (i, j) at i*n1 + j (j contiguous).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)

/* ---- jacobi_1d ---------------------------------------------------------- */

/* dst[i] = 0.33333 * ((src[i-1] + src[i]) + src[i+1]) on the updatable cells
 * of a window of h1 cells starting at global index c0 of a length-n vector. */
static void j1_half(const double *src, double *dst, int64_t n, int64_t c0, int64_t h1) {
    for (int64_t k = 1; k + 1 < h1; ++k) {
        const int64_t i = c0 + k;
        if (i < 1 || i > n - 2) continue;
        const double s = (src[k - 1] + src[k]) + src[k + 1];
        dst[k] = 0.33333 * s;
    }
}

int oracle_jacobi_1d_box(int32_t tsteps, int64_t n, int64_t c0, int64_t h1, double *A, double *B) {
    if (n < 0 || h1 < 0 || c0 < 0 || c0 + h1 > n) return ORC_E_ARG;
    if (h1 > 0 && (!A || !B)) return ORC_E_ARG;
    for (int32_t t = 1; t < tsteps; ++t) {
        j1_half(A, B, n, c0, h1);
        j1_half(B, A, n, c0, h1);
    }
    return ORC_OK;
}

int oracle_jacobi_1d(int32_t tsteps, int64_t n, double *A, double *B) {
    return oracle_jacobi_1d_box(tsteps, n, 0, n, A, B);
}

/* ---- jacobi_2d ---------------------------------------------------------- */

static void j2_half(const double *src, double *dst, int64_t n0, int64_t n1, int64_t r0, int64_t c0,
                    int64_t h0, int64_t h1) {
    for (int64_t a = 1; a + 1 < h0; ++a) {
        const int64_t i = r0 + a;
        if (i < 1 || i > n0 - 2) continue;
        for (int64_t b = 1; b + 1 < h1; ++b) {
            const int64_t j = c0 + b;
            if (j < 1 || j > n1 - 2) continue;
            const double centre = src[a * h1 + b];
            const double west = src[a * h1 + (b - 1)];
            const double east = src[a * h1 + (b + 1)];
            const double south = src[(a + 1) * h1 + b];
            const double north = src[(a - 1) * h1 + b];
            const double s = (((centre + west) + east) + south) + north;
            dst[a * h1 + b] = 0.2 * s;
        }
    }
}

int oracle_jacobi_2d_box(int32_t tsteps, int64_t n0, int64_t n1, int64_t r0, int64_t c0, int64_t h0,
                         int64_t h1, double *A, double *B) {
    if (n0 < 0 || n1 < 0 || h0 < 0 || h1 < 0 || r0 < 0 || c0 < 0) return ORC_E_ARG;
    if (r0 + h0 > n0 || c0 + h1 > n1) return ORC_E_ARG;
    if (h0 > 0 && h1 > 0 && (!A || !B)) return ORC_E_ARG;
    for (int32_t t = 1; t < tsteps; ++t) {
        j2_half(A, B, n0, n1, r0, c0, h0, h1);
        j2_half(B, A, n0, n1, r0, c0, h0, h1);
    }
    return ORC_OK;
}

int oracle_jacobi_2d(int32_t tsteps, int64_t n0, int64_t n1, double *A, double *B) {
    return oracle_jacobi_2d_box(tsteps, n0, n1, 0, 0, n0, n1, A, B);
}
