/*
 * rd3d_oracle.c -- plain, serial, FP64 CPU oracle for the reaction-diffusion
 * array program
 *
 *     u' = u + dt * (alpha * Lap7(u) - beta * u^3 + gamma * f)
 *
 * applied T times on an (nx, ny, nz) grid, and for its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or constant with the GPU path, and only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  The product
 * path never calls it.
 *
 * What it follows:
 *   - Sec. 2.3 ("From Python to DaCe"): the first translation pass splits an
 *     array expression into single-operator statements, one temporary each,
 *     in the order the operators bind.  Every step below materialises those
 *     temporaries exactly (lap, u3, t1..t6) as the unfused NumPy program
 *     would, one full loop per statement, no fusion and no reordering.
 *   - Sec. 2.3, write-conflict resolution: the sums over the grid (norms,
 *     gradient reductions) are plain sums; here they are compensated
 *     (Neumaier) so they are accurate to the last bit or so.
 *   - The program itself (7-point Laplacian with spacing h on all axes,
 *     ghost-zero Dirichlet or periodic boundaries, cubic reaction, source f)
 *     is the element-wise-plus-stencil instance this library implements; the
 *     adjoint is the chain rule applied to it:
 *         J_t = I + dt*alpha*L - diag(3*beta*dt*u_t^2)
 *         lambda_t = J_t^T lambda_{t+1}
 *         dL/dalpha = sum_t dt * <lambda_{t+1}, L u_t>
 *         dL/dbeta  = sum_t -dt * <lambda_{t+1}, u_t^3>
 *         dL/dgamma = sum_t dt * <lambda_{t+1}, f>
 *         dL/df     = gamma * dt * sum_t lambda_{t+1}
 *     (u_{t+1} depends on gamma through dt*gamma*f and on f through
 *     dt*gamma*f, the same at every step)
 *     L^T is applied by a literal scatter (each point sends its value to the
 *     points that read it), so the oracle does not assume L is symmetric.
 *
 * Layout: x is contiguous, linear index p = x + nx*(y + ny*z).
 * Boundary rule per axis: 0 = ghost zero (a neighbour outside [0,n) reads
 * 0.0 and every point is updated), 1 = periodic (neighbour index mod n).
 *
 * Build: gcc -O3 -ffp-contract=off (no FMA contraction, no fast-math), so
 * each operation rounds once, as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NOMEM (-2)

typedef struct {
    int64_t n[3];  /* extents x, y, z */
    int bc[3];     /* per-axis rule: 0 ghost zero, 1 periodic */
} grid_t;

typedef struct {
    double alpha, beta, gamma, h, dt;
} coef_t;

/* ---- compensated summation (Neumaier) ---------------------------------- */
typedef struct {
    double s, c;
} nsum_t;

static void nsum_add(nsum_t *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum_t *a) { return a->s + a->c; }

/* ---- indexing ----------------------------------------------------------- */
static int64_t lin(const grid_t *g, int64_t x, int64_t y, int64_t z) {
    return x + g->n[0] * (y + g->n[1] * z);
}

/* Coordinate of the neighbour c+off along an axis of extent n under rule bc;
 * -1 means "outside the grid" (a ghost cell that reads as zero). */
static int64_t neighbour(int64_t c, int off, int64_t n, int bc) {
    int64_t q = c + off;
    if (q >= 0 && q < n) return q;
    if (bc == 1) return ((q % n) + n) % n;
    return -1;
}

/* Value of u at the face neighbour of (x,y,z) displaced by off along axis. */
static double nb_value(const grid_t *g, const double *u, int64_t x, int64_t y,
                       int64_t z, int axis, int off) {
    int64_t c[3] = {x, y, z};
    int64_t q = neighbour(c[axis], off, g->n[axis], g->bc[axis]);
    if (q < 0) return 0.0;
    c[axis] = q;
    return u[lin(g, c[0], c[1], c[2])];
}

/* Lap7(u) at one point: six face neighbours minus 6u, over h^2, summed in
 * the order x-1, x+1, y-1, y+1, z-1, z+1. */
static double lap7_at(const grid_t *g, const double *u, int64_t x, int64_t y,
                      int64_t z, double h) {
    double xm = nb_value(g, u, x, y, z, 0, -1);
    double xp = nb_value(g, u, x, y, z, 0, +1);
    double ym = nb_value(g, u, x, y, z, 1, -1);
    double yp = nb_value(g, u, x, y, z, 1, +1);
    double zm = nb_value(g, u, x, y, z, 2, -1);
    double zp = nb_value(g, u, x, y, z, 2, +1);
    double uc = u[lin(g, x, y, z)];
    return (xm + xp + ym + yp + zm + zp - 6.0 * uc) / (h * h);
}

/* ---- one time step on a box -------------------------------------------- */
/* Temporaries of one step, each a full grid-sized array. */
enum { T_LAP, T_U3, T_T1, T_T2, T_T3, T_T4, T_T5, T_T6, T_COUNT };

typedef struct {
    int64_t lo[3], hi[3]; /* half-open box [lo, hi) of points to update */
} box_t;

#define FOR_BOX(b, g, p)                                                  \
    for (int64_t z_ = (b)->lo[2]; z_ < (b)->hi[2]; ++z_)                  \
        for (int64_t y_ = (b)->lo[1]; y_ < (b)->hi[1]; ++y_)              \
            for (int64_t x_ = (b)->lo[0], p = lin((g), x_, y_, z_);       \
                 x_ < (b)->hi[0]; ++x_, ++p)

/*
 * u_next = u + dt*(alpha*Lap7(u) - beta*u^3 + gamma*f) on the points of box b,
 * one statement per operator:
 *     lap = Lap7(u)
 *     u3  = (u*u)*u
 *     t1  = alpha*lap
 *     t2  = beta*u3
 *     t3  = t1 - t2
 *     t4  = gamma*f
 *     t5  = t3 + t4
 *     t6  = dt*t5
 *     u_next = u + t6
 * Points of u_next outside b are not written.
 */
static void step_box(const grid_t *g, const box_t *b, const coef_t *c,
                     const double *u, const double *f, double *const tmp[T_COUNT],
                     double *u_next) {
    double *lap = tmp[T_LAP], *u3 = tmp[T_U3], *t1 = tmp[T_T1], *t2 = tmp[T_T2];
    double *t3 = tmp[T_T3], *t4 = tmp[T_T4], *t5 = tmp[T_T5], *t6 = tmp[T_T6];
    FOR_BOX(b, g, p) lap[p] = lap7_at(g, u, x_, y_, z_, c->h);
    FOR_BOX(b, g, p) u3[p] = (u[p] * u[p]) * u[p];
    FOR_BOX(b, g, p) t1[p] = c->alpha * lap[p];
    FOR_BOX(b, g, p) t2[p] = c->beta * u3[p];
    FOR_BOX(b, g, p) t3[p] = t1[p] - t2[p];
    FOR_BOX(b, g, p) t4[p] = c->gamma * f[p];
    FOR_BOX(b, g, p) t5[p] = t3[p] + t4[p];
    FOR_BOX(b, g, p) t6[p] = c->dt * t5[p];
    FOR_BOX(b, g, p) u_next[p] = u[p] + t6[p];
}

static int alloc_fields(double **out, int count, int64_t n) {
    for (int i = 0; i < count; ++i) out[i] = NULL;
    for (int i = 0; i < count; ++i) {
        out[i] = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
        if (!out[i]) return ORC_E_NOMEM;
    }
    return ORC_OK;
}

static void free_fields(double **f, int count) {
    for (int i = 0; i < count; ++i) free(f[i]);
}

static int check_common(int64_t nx, int64_t ny, int64_t nz, int bc, int T,
                        double h) {
    if (nx < 0 || ny < 0 || nz < 0) return ORC_E_ARG;
    if (bc != 0 && bc != 1) return ORC_E_ARG;
    if (T < 0) return ORC_E_ARG;
    if (!(h > 0.0)) return ORC_E_ARG;
    return ORC_OK;
}

/* Observer of a streaming run: called once per step with the new state u_t
 * (valid during the call only) and its two norms. */
typedef void (*oracle_step_cb)(int t, const double *u_t, double e_t,
                               double r_t, void *ctx);

static int run_whole_grid(int64_t nx, int64_t ny, int64_t nz, const double *u0,
                          const double *f, double alpha, double beta,
                          double gamma, double h, double dt, int bc, int T,
                          double *uT, double *energy, double *resid,
                          oracle_step_cb cb, void *ctx);

/*
 * T steps from u0 on the whole grid.
 *   uT     [N]  out: the state after T steps (may be NULL)
 *   energy [T]  out: E_t = sum u_t^2 for t = 1..T (may be NULL)
 *   resid  [T]  out: R_t = sqrt(sum (u_t - u_{t-1})^2) for t = 1..T (may be NULL)
 */
int oracle_run(int64_t nx, int64_t ny, int64_t nz, const double *u0,
               const double *f, double alpha, double beta, double gamma,
               double h, double dt, int bc, int T, double *uT, double *energy,
               double *resid) {
    return run_whole_grid(nx, ny, nz, u0, f, alpha, beta, gamma, h, dt, bc, T,
                          uT, energy, resid, NULL, NULL);
}

/*
 * The same T steps as oracle_run, handing every state u_1 .. u_T to cb as
 * soon as it is computed, so that a caller can compare each step with
 * another evaluation without keeping T fields.  Nothing else differs.
 */
int oracle_run_stream(int64_t nx, int64_t ny, int64_t nz, const double *u0,
                      const double *f, double alpha, double beta,
                      double gamma, double h, double dt, int bc, int T,
                      oracle_step_cb cb, void *ctx) {
    if (!cb) return ORC_E_ARG;
    return run_whole_grid(nx, ny, nz, u0, f, alpha, beta, gamma, h, dt, bc, T,
                          NULL, NULL, NULL, cb, ctx);
}

static int run_whole_grid(int64_t nx, int64_t ny, int64_t nz, const double *u0,
                          const double *f, double alpha, double beta,
                          double gamma, double h, double dt, int bc, int T,
                          double *uT, double *energy, double *resid,
                          oracle_step_cb cb, void *ctx) {
    int rc = check_common(nx, ny, nz, bc, T, h);
    if (rc) return rc;
    grid_t g = {{nx, ny, nz}, {bc, bc, bc}};
    coef_t c = {alpha, beta, gamma, h, dt};
    int64_t n = nx * ny * nz;
    double *tmp[T_COUNT], *st[2];
    if ((rc = alloc_fields(tmp, T_COUNT, n)) || (rc = alloc_fields(st, 2, n))) {
        free_fields(tmp, T_COUNT);
        free_fields(st, 2);
        return rc;
    }
    if (n > 0) memcpy(st[0], u0, (size_t)n * sizeof(double));
    box_t all = {{0, 0, 0}, {nx, ny, nz}};
    for (int t = 0; t < T; ++t) {
        const double *u = st[t & 1];
        double *un = st[(t + 1) & 1];
        step_box(&g, &all, &c, u, f, tmp, un);
        nsum_t e = {0, 0}, r = {0, 0};
        for (int64_t p = 0; p < n; ++p) {
            nsum_add(&e, un[p] * un[p]);
            double d = un[p] - u[p];
            nsum_add(&r, d * d);
        }
        if (energy) energy[t] = nsum_value(&e);
        if (resid) resid[t] = sqrt(nsum_value(&r));
        if (cb) cb(t + 1, un, nsum_value(&e), sqrt(nsum_value(&r)), ctx);
    }
    if (uT && n > 0) memcpy(uT, st[T & 1], (size_t)n * sizeof(double));
    free_fields(tmp, T_COUNT);
    free_fields(st, 2);
    return ORC_OK;
}

/*
 * The state u_T on a small box [blo, bhi) of the grid, without running the
 * whole grid.  After T steps a point depends only on points within distance
 * T of it (per axis), so the same step is evaluated on a window that covers
 * the box plus T points on each side:
 *   - along an axis whose window would cover the whole extent, the whole
 *     axis is used with its true boundary rule;
 *   - otherwise the window is a sub-range (wrapped for periodic, clipped to
 *     the grid for ghost-zero), and the cells beyond its ends read as zero.
 *     Those artificial ends are wrong, but the error moves one point per
 *     step, so it never reaches the box within T steps.
 * Step t (1..T) updates only the points within distance T-t of the box (the
 * points that step T still needs); the rest of the window keeps stale
 * values that are never read.  out[] receives u_T on the box, x fastest.
 */
int oracle_run_box(int64_t nx, int64_t ny, int64_t nz, const double *u0,
                   const double *f, double alpha, double beta, double gamma,
                   double h, double dt, int bc, int T, const int64_t blo[3],
                   const int64_t bhi[3], double *out) {
    int rc = check_common(nx, ny, nz, bc, T, h);
    if (rc) return rc;
    const int64_t n[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d)
        if (blo[d] < 0 || bhi[d] > n[d] || blo[d] >= bhi[d]) return ORC_E_ARG;

    /* window geometry per axis */
    int64_t wlo[3], wlen[3];
    int full[3];
    grid_t w;
    for (int d = 0; d < 3; ++d) {
        int64_t lo = blo[d] - T, hi = bhi[d] + T;
        if (hi - lo >= n[d] || (bc == 0 && lo <= 0 && hi >= n[d])) {
            full[d] = 1;
            wlo[d] = 0;
            wlen[d] = n[d];
            w.bc[d] = bc;
        } else {
            full[d] = 0;
            if (bc == 0) { /* clip to the grid: the clipped side is a true wall */
                if (lo < 0) lo = 0;
                if (hi > n[d]) hi = n[d];
            }
            wlo[d] = lo;
            wlen[d] = hi - lo;
            w.bc[d] = 0;
        }
        w.n[d] = wlen[d];
    }
    int64_t wn = wlen[0] * wlen[1] * wlen[2];
    double *tmp[T_COUNT], *st[2], *wf[1];
    if ((rc = alloc_fields(tmp, T_COUNT, wn)) || (rc = alloc_fields(st, 2, wn)) ||
        (rc = alloc_fields(wf, 1, wn))) {
        free_fields(tmp, T_COUNT);
        free_fields(st, 2);
        free_fields(wf, 1);
        return rc;
    }
    /* gather u0 and f onto the window (window coordinate -> grid coordinate) */
    grid_t gg = {{nx, ny, nz}, {bc, bc, bc}};
    for (int64_t k = 0; k < wlen[2]; ++k)
        for (int64_t j = 0; j < wlen[1]; ++j)
            for (int64_t i = 0; i < wlen[0]; ++i) {
                int64_t wc[3] = {i, j, k}, gc[3];
                for (int d = 0; d < 3; ++d) {
                    int64_t q = wlo[d] + wc[d];
                    gc[d] = ((q % n[d]) + n[d]) % n[d]; /* periodic wrap; in range otherwise */
                }
                int64_t pw = lin(&w, i, j, k), pg = lin(&gg, gc[0], gc[1], gc[2]);
                st[0][pw] = u0[pg];
                wf[0][pw] = f[pg];
            }
    coef_t c = {alpha, beta, gamma, h, dt};
    for (int t = 1; t <= T; ++t) {
        box_t b;
        for (int d = 0; d < 3; ++d) {
            if (full[d] && bc == 1) {
                b.lo[d] = 0;
                b.hi[d] = wlen[d];
            } else {
                int64_t lo = blo[d] - wlo[d] - (T - t), hi = bhi[d] - wlo[d] + (T - t);
                b.lo[d] = lo < 0 ? 0 : lo;
                b.hi[d] = hi > wlen[d] ? wlen[d] : hi;
            }
        }
        step_box(&w, &b, &c, st[(t - 1) & 1], wf[0], tmp, st[t & 1]);
    }
    const double *fin = st[T & 1];
    int64_t o = 0;
    for (int64_t z = blo[2]; z < bhi[2]; ++z)
        for (int64_t y = blo[1]; y < bhi[1]; ++y)
            for (int64_t x = blo[0]; x < bhi[0]; ++x)
                out[o++] = fin[lin(&w, x - wlo[0], y - wlo[1], z - wlo[2])];
    free_fields(tmp, T_COUNT);
    free_fields(st, 2);
    free_fields(wf, 1);
    return ORC_OK;
}

/*
 * Reverse-mode gradient of a loss through T steps.
 *   lamT    [N]  in : dL/du_T (for L = 0.5*||u_T - u_tgt||^2 it is u_T - u_tgt)
 *   grad_u0 [N]  out: dL/du_0 = lambda_0
 *   grad_ab [2]  out: dL/dalpha, dL/dbeta
 * All states u_0..u_{T-1} are kept in host memory.
 * Per step, from t = T-1 down to 0:
 *   LT      = L^T lambda_{t+1}, by scatter: every point p adds lambda[p]/h^2
 *             to each face neighbour it reads and -6*lambda[p]/h^2 to itself
 *   gA     += dt * sum lambda_{t+1} * Lap7(u_t)
 *   gB     += -dt * sum lambda_{t+1} * u_t^3
 *   lambda_t = lambda_{t+1} + dt*(alpha*LT - 3*beta*u_t^2*lambda_{t+1})
 */
/* grad_f (N doubles) and grad_gamma (one double) are optional (NULL). */
int oracle_adjoint(int64_t nx, int64_t ny, int64_t nz, const double *u0,
                   const double *f, const double *lamT, double alpha,
                   double beta, double gamma, double h, double dt, int bc,
                   int T, double *grad_u0, double *grad_ab, double *grad_f,
                   double *grad_gamma) {
    int rc = check_common(nx, ny, nz, bc, T, h);
    if (rc) return rc;
    grid_t g = {{nx, ny, nz}, {bc, bc, bc}};
    coef_t c = {alpha, beta, gamma, h, dt};
    int64_t n = nx * ny * nz;
    int nst = T > 0 ? T : 1;
    double **states = (double **)calloc((size_t)nst, sizeof(double *));
    double *tmp[T_COUNT], *lam[3];
    if (!states) return ORC_E_NOMEM;
    rc = alloc_fields(states, nst, n);
    if (!rc) rc = alloc_fields(tmp, T_COUNT, n);
    else for (int i = 0; i < T_COUNT; ++i) tmp[i] = NULL;
    if (!rc) rc = alloc_fields(lam, 3, n);
    else for (int i = 0; i < 3; ++i) lam[i] = NULL;
    if (rc) {
        free_fields(states, nst);
        free(states);
        free_fields(tmp, T_COUNT);
        free_fields(lam, 3);
        return rc;
    }
    box_t all = {{0, 0, 0}, {nx, ny, nz}};
    if (n > 0) memcpy(states[0], u0, (size_t)n * sizeof(double));
    for (int t = 0; t + 1 < T; ++t) step_box(&g, &all, &c, states[t], f, tmp, states[t + 1]);

    double *lcur = lam[0], *lnext = lam[1], *lt = lam[2];
    if (n > 0) memcpy(lcur, lamT, (size_t)n * sizeof(double));
    nsum_t ga = {0, 0}, gb = {0, 0}, gg = {0, 0};
    /* sum of the lambda_{t+1} seen so far, per point (accumulated in grad_f) */
    if (grad_f)
        for (int64_t p = 0; p < n; ++p) grad_f[p] = 0.0;
    const double inv_h2 = 1.0 / (h * h);
    for (int t = T - 1; t >= 0; --t) {
        const double *u = states[t];
        /* L^T lambda by literal scatter */
        for (int64_t p = 0; p < n; ++p) lt[p] = 0.0;
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t p = lin(&g, x, y, z);
                    double v = lcur[p] * inv_h2;
                    int64_t cc[3] = {x, y, z};
                    for (int axis = 0; axis < 3; ++axis)
                        for (int off = -1; off <= 1; off += 2) {
                            int64_t q = neighbour(cc[axis], off, g.n[axis], g.bc[axis]);
                            if (q < 0) continue;
                            int64_t d[3] = {x, y, z};
                            d[axis] = q;
                            lt[lin(&g, d[0], d[1], d[2])] += v;
                        }
                    lt[p] += -6.0 * v;
                }
        nsum_t sa = {0, 0}, sb = {0, 0};
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t p = lin(&g, x, y, z);
                    double lap = lap7_at(&g, u, x, y, z, h);
                    double u3 = (u[p] * u[p]) * u[p];
                    nsum_add(&sa, lcur[p] * lap);
                    nsum_add(&sb, lcur[p] * u3);
                }
        nsum_add(&ga, dt * nsum_value(&sa));
        nsum_add(&gb, -dt * nsum_value(&sb));
        if (grad_gamma) {
            nsum_t sg = {0, 0};
            for (int64_t p = 0; p < n; ++p) nsum_add(&sg, lcur[p] * f[p]);
            nsum_add(&gg, dt * nsum_value(&sg));
        }
        if (grad_f)
            for (int64_t p = 0; p < n; ++p) grad_f[p] += lcur[p];
        for (int64_t p = 0; p < n; ++p)
            lnext[p] = lcur[p] + dt * (alpha * lt[p] - 3.0 * beta * (u[p] * u[p]) * lcur[p]);
        double *sw = lcur;
        lcur = lnext;
        lnext = sw;
    }
    if (n > 0) memcpy(grad_u0, lcur, (size_t)n * sizeof(double));
    grad_ab[0] = nsum_value(&ga);
    grad_ab[1] = nsum_value(&gb);
    if (grad_gamma) *grad_gamma = nsum_value(&gg);
    if (grad_f)
        for (int64_t p = 0; p < n; ++p) grad_f[p] = (gamma * dt) * grad_f[p];
    free_fields(states, nst);
    free(states);
    free_fields(tmp, T_COUNT);
    free_fields(lam, 3);
    return ORC_OK;
}

/* 0.5 * sum (a - b)^2, compensated. */
double oracle_half_sq_dist(int64_t n, const double *a, const double *b) {
    nsum_t s = {0, 0};
    for (int64_t p = 0; p < n; ++p) {
        double d = a[p] - b[p];
        nsum_add(&s, d * d);
    }
    return 0.5 * nsum_value(&s);
}
