// dcp_api.cpp -- C ABI of libdcp (declared in include/dcp.h): argument
// checks, workspace layout, tile choice and the host drivers of the time
// loop and of the checkpointed adjoint.  All device work is enqueued on the
// caller's stream; nothing here synchronises or allocates device memory.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <vector>

#include "dcp.h"
#include "dcp_internal.h"

using namespace dcp;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Geo {
    int64_t nx = 0, ny = 0, nz = 0, n = 0;
    size_t esz = 8;
    size_t bytes() const { return (size_t)n * esz; }
};

int check_geo(int dtype, int64_t nx, int64_t ny, int64_t nz, Geo *g) {
    if (dtype != DCP_F64 && dtype != DCP_F32) return DCP_E_DTYPE;
    if (nx < 0 || ny < 0 || nz < 0) return DCP_E_SHAPE;
    const int64_t ext_lim = (int64_t)1 << 30;
    if (nx > ext_lim || ny > ext_lim || nz > ext_lim) return DCP_E_SHAPE;
    g->esz = dtype == DCP_F64 ? 8 : 4;
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->n = 0;
    if (nx && ny && nz) {
        const int64_t lim = ((int64_t)1 << 60) / (int64_t)g->esz;
        if (nx > lim / ny) return DCP_E_SHAPE;
        const int64_t nxy = nx * ny;
        if (nxy > lim / nz) return DCP_E_SHAPE;
        g->n = nxy * nz;
    }
    return DCP_OK;
}

int check_coeffs(const dcp_coeffs *c) {
    if (!c) return DCP_E_NULL;
    const double v[5] = {c->alpha, c->beta, c->gamma, c->h, c->dt};
    for (double x : v)
        if (!std::isfinite(x)) return DCP_E_ARG;
    if (!(c->h > 0.0)) return DCP_E_ARG;
    return DCP_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// ------------------------------------------------------------- tile choice
int env_int(const char *name, int def) {
    const char *s = tuning_env(name);
    if (!s || !*s) return def;
    return std::atoi(s);
}

Tile make_tile(const Geo &g, int vec, int shape, int zc) {
    Tile t{};
    const Shape s = shape_at(shape);
    t.vec = vec;
    t.bxw = s.bxw;
    t.by = s.by;
    t.ry = s.ry;
    t.zc = zc;
    const int64_t tx = (g.nx + (int64_t)64 * s.bxw * vec - 1) / ((int64_t)64 * s.bxw * vec);
    const int64_t ty = (g.ny + (int64_t)s.by * s.ry - 1) / ((int64_t)s.by * s.ry);
    const int64_t tz = (g.nz + zc - 1) / zc;
    const int64_t nb = tx * ty * tz;
    t.tiles_x = (int)tx;
    t.tiles_y = (int)ty;
    t.tiles_z = (int)tz;
    t.nblk = nb > INT32_MAX / 1024 ? -1 : (int)nb;
    return t;
}

// Tile for one field operand layout.  The default is tuned for the 512^3
// class of grids; DCP_TILE_SHAPE / DCP_TILE_ZC override it in tuning runs
// (with DCP_TUNING=1).
Tile pick_tile(int dtype, const Geo &g, bool vec_ok) {
    const int wide = dtype == DCP_F64 ? 2 : 4;
    const int vec = vec_ok ? wide : 1;
    int shape = env_int("DCP_TILE_SHAPE", 0);
    if (shape < 0 || shape >= num_shapes()) shape = 0;
    int zc = env_int("DCP_TILE_ZC", 0);
    if (zc <= 0) {
        // enough workgroups to fill 256 CUs several times over, but long
        // z-runs so the two extra planes per run stay a small overhead
        zc = 64;
        while (zc > 8 && make_tile(g, vec, shape, zc).nblk >= 0 &&
               make_tile(g, vec, shape, zc).nblk < 2048)
            zc /= 2;
    }
    if (g.nz > 0 && zc > g.nz) zc = (int)g.nz;
    if (zc < 1) zc = 1;
    return make_tile(g, vec, shape, zc);
}

// Largest workgroup count over both vector widths (workspace sizing must not
// depend on pointer alignment).
int max_blocks(int dtype, const Geo &g) {
    if (g.n == 0) return 0;
    const Tile a = pick_tile(dtype, g, true), b = pick_tile(dtype, g, false);
    if (a.nblk < 0 || b.nblk < 0) return -1;
    return a.nblk > b.nblk ? a.nblk : b.nblk;
}

// ---------------------------------------------------------- workspace layout
struct StepWs {
    size_t temps = 0;     // offset of 3 temporaries (unfused)
    size_t partials = 0;  // offset of partial sums
    size_t total = 0;
};

int layout_step(int dtype, int impl, const Geo &g, bool norms, StepWs *w) {
    size_t off = 0;
    if (impl == DCP_UNFUSED && g.n > 0) {
        w->temps = off;
        off += 3 * align_up(g.bytes());
    }
    if (norms && g.n > 0) {
        const int nb = impl == DCP_UNFUSED ? ew_norm_blocks(g.n) : max_blocks(dtype, g);
        if (nb < 0) return DCP_E_SHAPE;
        w->partials = off;
        off += align_up((size_t)nb * 2 * sizeof(double));
    }
    w->total = off;
    return DCP_OK;
}

struct RunWs {
    size_t field = 0;     // ping-pong field
    size_t temps = 0;     // unfused temporaries
    size_t partials = 0;  // [T][nblk][2]
    int nblk = 0;
    size_t total = 0;
};

// LDS of one workgroup on gfx950, the most a two-step pass may plan for.
constexpr size_t kLdsMax = 160 * 1024;

// Plan of a B-step pass (dcp_tbk.hip): for three steps the ring form (768
// lanes) where a tile fits it, else 1024 lanes; for two steps the reverse.  DCP_TBK_CFG="wc,ty,lanes" restricts the
// planner to segments of wc chunks (a value covering the row: whole rows),
// slabs of ty rows and 768, 1024 or 512 lanes; 0 leaves a choice to the
// planner.  DCP_TBK_SBLK sets the slabs per block of the tile order.
// Tuning overrides only: every choice computes the same states bit for bit
// (the norms' summation order follows the tiles).
bool tbk_for(int dtype, const Geo &g, int B, bool vok, size_t lds_limit, TbkTile *t) {
    int wc = 0, ty = 0, lanes = 0;
    if (const char *e = tuning_env("DCP_TBK_CFG")) {
        int a = 0, b = 0, c = 0;
        if (std::sscanf(e, "%d,%d,%d", &a, &b, &c) == 3) {
            wc = a > 0 ? a : 0;
            ty = b > 0 ? b : 0;
            lanes = c == 512 || c == 768 || c == 1024 ? c : 0;
        }
    }
    // measured at 1024x1024x512 FP64: the ring form is the faster for three
    // steps per pass (22.4 against 24.7 ms for T = 24), the plain form for
    // two (30.7 against 34.4 ms)
    const int first = B == 3 ? 768 : 1024, second = B == 3 ? 1024 : 768;
    bool ok = false;
    if (lanes) ok = tbk_plan(dtype, B, g.nx, g.ny, g.nz, vok, lds_limit, lanes, wc, ty, t);
    else ok = tbk_plan(dtype, B, g.nx, g.ny, g.nz, vok, lds_limit, first, wc, ty, t) ||
              tbk_plan(dtype, B, g.nx, g.ny, g.nz, vok, lds_limit, second, wc, ty, t);
    if (!ok) return false;
    if (const char *e = tuning_env("DCP_TBK_SBLK")) {
        const int h = std::atoi(e);
        if (h > 0) t->sblk = h < t->nslab ? h : t->nslab;
    }
    return true;
}

int layout_run(int dtype, int impl, const Geo &g, int32_t T, int32_t tblock, bool norms, RunWs *w) {
    size_t off = 0;
    if (g.n == 0 || T == 0) {
        w->total = 0;
        return DCP_OK;
    }
    w->field = off;
    off += align_up(g.bytes());
    if (impl == DCP_UNFUSED) {
        w->temps = off;
        off += 3 * align_up(g.bytes());
    }
    if (norms) {
        int nb = impl == DCP_UNFUSED ? ew_norm_blocks(g.n) : max_blocks(dtype, g);
        if (nb < 0) return DCP_E_SHAPE;
        TbTile tb;
        if (impl == DCP_FUSED && tblock >= 2 && tb_plan(dtype, g.nx, g.ny, g.nz, true, kLdsMax, &tb) &&
            tb.nblk > nb)
            nb = tb.nblk;
        for (int B = 2; impl == DCP_FUSED && B <= tblock && B <= 3; ++B) {
            TbkTile tk;
            if (tbk_for(dtype, g, B, true, kLdsMax, &tk) && tk.nblk > nb) nb = tk.nblk;
        }
        w->nblk = nb;
        w->partials = off;
        off += align_up((size_t)T * nb * 2 * sizeof(double));
    }
    w->total = off;
    return DCP_OK;
}

struct AdjWs {
    size_t lam = 0;       // 2 fields
    size_t seg = 0;       // k-1 fields
    size_t partials = 0;  // [T][nblk][2]
    size_t sums = 0;      // [T][2]
    size_t lsum = 0;      // 1 field: running sum of the adjoint inputs (when wanted there)
    size_t dot = 0;       // [ew_norm_blocks][2] + 2: partials of <sum, f>
    int nblk = 0;
    size_t total = 0;
};

// lsum_field: reserve the running-sum field (dL/dgamma without a grad_f buffer).
int layout_adj(int dtype, const Geo &g, int32_t T, int32_t k, int32_t tblock, bool lsum_field, AdjWs *w) {
    size_t off = 0;
    if (T == 0) {
        w->total = 0;
        return DCP_OK;
    }
    if (g.n > 0) {
        int nb = max_blocks(dtype, g);
        if (nb < 0) return DCP_E_SHAPE;
        TbTile tb;
        if (tblock >= 2 && tb_plan(dtype, g.nx, g.ny, g.nz, true, kLdsMax, &tb) && tb.nblk > nb) nb = tb.nblk;
        w->nblk = nb;
        w->lam = off;
        off += 2 * align_up(g.bytes());
        w->seg = off;
        const int32_t kk = k < T ? k : T;
        off += (size_t)(kk - 1) * align_up(g.bytes());
        w->partials = off;
        off += align_up((size_t)T * nb * 2 * sizeof(double));
        if (lsum_field) {
            w->lsum = off;
            off += align_up(g.bytes());
        }
        w->dot = off;
        off += align_up(((size_t)ew_norm_blocks(g.n) * 2 + 2) * sizeof(double));
    }
    w->sums = off;
    off += align_up((size_t)T * 2 * sizeof(double));
    w->total = off;
    return DCP_OK;
}

int check_ws(const void *ws, size_t ws_bytes, size_t need) {
    if (need == 0) return DCP_OK;
    if (ws_bytes < need) return DCP_E_WORKSPACE;
    if (!ws) return DCP_E_NULL;
    return DCP_OK;
}

char *at(void *base, size_t off) { return static_cast<char *>(base) + off; }

int hip_status(hipError_t e) { return e == hipSuccess ? DCP_OK : DCP_E_HIP; }

#define DCP_TRY(expr)                            \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return DCP_E_HIP;  \
    } while (0)

StencilArgs fwd_args(const Geo &g, const dcp_coeffs &c, const Tile &t, const void *u, const void *f,
                     void *out, double *partials) {
    StencilArgs a{};
    a.s = u;
    a.q = f;
    a.out = out;
    a.partials = partials;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.c0 = c.dt * c.alpha / (c.h * c.h);
    a.c1 = c.dt * c.beta;
    a.c2 = c.dt * c.gamma;
    a.tiles_x = t.tiles_x;
    a.tiles_y = t.tiles_y;
    a.zc = t.zc;
    a.nblk = t.nblk;
    return a;
}

// One fused step u -> out (partials may be null).
hipError_t fused_step(int dtype, int bc, const Geo &g, const dcp_coeffs &c, const Tile &t, const void *u,
                      const void *f, void *out, double *partials, hipStream_t st) {
    const StencilArgs a = fwd_args(g, c, t, u, f, out, partials);
    return launch_stencil(dtype, SOP_FWD, bc, partials != nullptr, t, a, st);
}

// One unfused step (the single-operator statements), temporaries in tmp[3].
hipError_t unfused_step(int dtype, int bc, const Geo &g, const dcp_coeffs &c, const Tile &t, bool vec_ok,
                        const void *u, const void *f, void *out, void *const tmp[3], double *partials,
                        hipStream_t st) {
    void *A = tmp[0], *B = tmp[1], *C = tmp[2];
    StencilArgs a{};
    a.s = u;
    a.q = nullptr;
    a.out = A;
    a.partials = nullptr;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.c0 = c.h * c.h;
    a.tiles_x = t.tiles_x;
    a.tiles_y = t.tiles_y;
    a.zc = t.zc;
    a.nblk = t.nblk;
    hipError_t e;
    if ((e = launch_stencil(dtype, SOP_LAP, bc, false, t, a, st)) != hipSuccess) return e;  // lap = Lap7(u)  -> A
    if ((e = launch_ew(dtype, EW_POW3, u, nullptr, B, 0.0, g.n, vec_ok, st))) return e;     // u3 = (u*u)*u  -> B
    if ((e = launch_ew(dtype, EW_SCALE, A, nullptr, C, c.alpha, g.n, vec_ok, st))) return e;  // t1 = alpha*lap -> C
    if ((e = launch_ew(dtype, EW_SCALE, B, nullptr, A, c.beta, g.n, vec_ok, st))) return e;   // t2 = beta*u3  -> A
    if ((e = launch_ew(dtype, EW_SUB, C, A, B, 0.0, g.n, vec_ok, st))) return e;              // t3 = t1 - t2  -> B
    if ((e = launch_ew(dtype, EW_SCALE, f, nullptr, C, c.gamma, g.n, vec_ok, st))) return e;  // t4 = gamma*f  -> C
    if ((e = launch_ew(dtype, EW_ADD, B, C, A, 0.0, g.n, vec_ok, st))) return e;              // t5 = t3 + t4  -> A
    if ((e = launch_ew(dtype, EW_SCALE, A, nullptr, B, c.dt, g.n, vec_ok, st))) return e;     // t6 = dt*t5    -> B
    if ((e = launch_ew(dtype, EW_ADD, u, B, out, 0.0, g.n, vec_ok, st))) return e;            // u' = u + t6
    if (partials) return launch_ew_norms(dtype, out, u, partials, g.n, vec_ok, st);
    return hipSuccess;
}

// A two-step pass u_t -> u_{t+2} (mid receives u_{t+1} when not null).
hipError_t tb_fwd_pass(int dtype, int bc, const Geo &g, const dcp_coeffs &c, const TbTile &tb, const void *u,
                       const void *f, void *out, void *mid, double *part1, double *part2, hipStream_t st) {
    TbArgs ta{};
    ta.u = u;
    ta.f = f;
    ta.out = out;
    ta.mid = mid;
    ta.part1 = part1;
    ta.part2 = part2;
    ta.nx = g.nx;
    ta.ny = g.ny;
    ta.nz = g.nz;
    ta.c0 = c.dt * c.alpha / (c.h * c.h);
    ta.c1 = c.dt * c.beta;
    ta.c2 = c.dt * c.gamma;
    ta.nslab = tb.nslab;
    ta.zc = tb.zc;
    return launch_tb2(dtype, SOP_FWD, bc, part1 != nullptr, tb, ta, st);
}

// LDS one workgroup may use on the current device (gfx950's 160 KiB when no
// device can be asked, for plans made on a host without one).
size_t device_lds() {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0)
        return kLdsMax;
    return (size_t)lds;
}

// Plans a two-step pass when asked for and supported by the grid and device.
bool plan_tb(int dtype, const Geo &g, int32_t tblock, bool vok, TbTile *tb) {
    if (tblock < 2) return false;
    return tb_plan(dtype, g.nx, g.ny, g.nz, vok, device_lds(), tb);
}

// Plans a B-step pass (B = 2, 3) when the grid and the device allow it.
bool plan_tbk(int dtype, const Geo &g, int B, bool vok, TbkTile *t) {
    return tbk_for(dtype, g, B, vok, device_lds(), t);
}

// The passes of a fused dcp_run: three steps where tblock >= 3 and the
// B-step kernel applies; two steps over whole rows where the two-step kernel
// applies, else over x-segments; one step otherwise and for the remainders.
// stride: partial-sum slots per step of the run's workspace (norms only).
struct PassPlan {
    bool use_tb = false, use_k2 = false, use_k3 = false;
    TbTile tb{};
    TbkTile k2{}, k3{};
    // steps in the pass starting at step s of T: three where possible, but
    // four steps left go as two passes of two (cheaper than three and one)
    int32_t len_at(int32_t s, int32_t T) const {
        const bool two = use_tb || use_k2;
        if (use_k3 && s + 3 <= T && !(two && T - s == 4)) return 3;
        if (two && s + 2 <= T) return 2;
        return 1;
    }
};

PassPlan plan_passes(int dtype, int impl, const Geo &g, int32_t T, int32_t tblock, bool vok, bool norms,
                     int stride) {
    PassPlan pp;
    if (impl != DCP_FUSED) return pp;
    pp.use_tb = T >= 2 && plan_tb(dtype, g, tblock, vok, &pp.tb) && (!norms || pp.tb.nblk <= stride);
    pp.use_k2 = !pp.use_tb && T >= 2 && tblock >= 2 && plan_tbk(dtype, g, 2, vok, &pp.k2) &&
                (!norms || pp.k2.nblk <= stride);
    pp.use_k3 = T >= 3 && tblock >= 3 && plan_tbk(dtype, g, 3, vok, &pp.k3) && (!norms || pp.k3.nblk <= stride);
    return pp;
}

// A B-step pass u_t -> u_{t+B}; mid[s-1] receives u_{t+s} when not null;
// part (when not null) holds the B steps' partial-sum arrays.
hipError_t tbk_fwd_pass(int dtype, int bc, const Geo &g, const dcp_coeffs &c, const TbkTile &tk, const void *u,
                        const void *f, void *out, void *const mid[2], double *const part[3], hipStream_t st) {
    TbkArgs a{};
    a.u = u;
    a.f = f;
    a.out = out;
    for (int i = 0; i < 2; ++i) a.mid[i] = mid ? mid[i] : nullptr;
    for (int i = 0; i < 3; ++i) a.part[i] = part ? part[i] : nullptr;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.c0 = c.dt * c.alpha / (c.h * c.h);
    a.c1 = c.dt * c.beta;
    a.c2 = c.dt * c.gamma;
    a.ty = tk.ty;
    a.nslab = tk.nslab;
    a.nseg = tk.nseg;
    a.zc = tk.zc;
    a.wc = tk.wc;
    a.halo = tk.halo;
    a.chf = tk.chf;
    a.sblk = tk.sblk;
    return launch_tbk(dtype, bc, part != nullptr, tk, a, st);
}

// One forward pass of len (1, 2 or 3) steps without norms, u -> out, in the
// kernel `pp` plans for that length; mid[i] (when not null) receives the
// state after i+1 steps of a multi-step pass.
hipError_t fwd_pass(int dtype, int bc, const Geo &g, const dcp_coeffs &c, const Tile &t, const PassPlan &pp,
                    int len, const void *u, const void *f, void *out, void *mid0, void *mid1, hipStream_t st) {
    if (len == 3 || (len == 2 && !pp.use_tb)) {
        void *mid[2] = {mid0, len == 3 ? mid1 : nullptr};
        return tbk_fwd_pass(dtype, bc, g, c, len == 3 ? pp.k3 : pp.k2, u, f, out, mid, nullptr, st);
    }
    if (len == 2) return tb_fwd_pass(dtype, bc, g, c, pp.tb, u, f, out, mid0, nullptr, nullptr, st);
    return fused_step(dtype, bc, g, c, t, u, f, out, nullptr, st);
}

bool vec_ok_for(int dtype, const Geo &g, std::initializer_list<const void *> ptrs) {
    const int wide = dtype == DCP_F64 ? 2 : 4;
    if (g.nx % wide != 0) return false;
    for (const void *p : ptrs)
        if (p && !aligned16(p)) return false;
    return true;
}

int step_common(int impl, int dtype, const void *u, const void *f, void *u_out, int64_t nx, int64_t ny,
                int64_t nz, const dcp_coeffs *coeffs, int bc, double *norms2, void *ws, size_t ws_bytes,
                void *stream) {
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (bc != DCP_DIRICHLET0 && bc != DCP_PERIODIC) return DCP_E_BC;
    if ((rc = check_coeffs(coeffs))) return rc;
    if (g.n > 0 && (!u || !f || !u_out)) return DCP_E_NULL;
    StepWs w;
    if ((rc = layout_step(dtype, impl, g, norms2 != nullptr, &w))) return rc;
    if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
    const size_t fb = g.bytes();
    if (overlaps(u_out, fb, u, fb) || overlaps(u_out, fb, f, fb)) return DCP_E_ALIAS;
    if (overlaps(ws, w.total, u, fb) || overlaps(ws, w.total, f, fb) || overlaps(ws, w.total, u_out, fb))
        return DCP_E_ALIAS;
    if (norms2 && (overlaps(norms2, 16, u, fb) || overlaps(norms2, 16, f, fb) ||
                   overlaps(norms2, 16, u_out, fb) || overlaps(norms2, 16, ws, w.total)))
        return DCP_E_ALIAS;

    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g.n == 0) return norms2 ? hip_status(launch_zero(norms2, 2, st)) : DCP_OK;

    double *partials = norms2 ? reinterpret_cast<double *>(at(ws, w.partials)) : nullptr;
    if (impl == DCP_FUSED) {
        const Tile t = pick_tile(dtype, g, vec_ok_for(dtype, g, {u, f, u_out}));
        DCP_TRY(fused_step(dtype, bc, g, *coeffs, t, u, f, u_out, partials, st));
        if (norms2) DCP_TRY(launch_finalize(partials, t.nblk, t.nblk, 1, norms2, nullptr, 0, st));
    } else {
        void *tmp[3] = {at(ws, w.temps), at(ws, w.temps + align_up(fb)), at(ws, w.temps + 2 * align_up(fb))};
        const bool vok = vec_ok_for(dtype, g, {u, f, u_out, tmp[0], tmp[1], tmp[2]});
        const Tile t = pick_tile(dtype, g, vok);
        DCP_TRY(unfused_step(dtype, bc, g, *coeffs, t, vok, u, f, u_out, tmp, partials, st));
        if (norms2) {
            const int nb = ew_norm_blocks(g.n);
            DCP_TRY(launch_finalize(partials, nb, nb, 1, norms2, nullptr, 0, st));
        }
    }
    return DCP_OK;
}

int32_t num_slots(int32_t T, int32_t k) { return T <= 0 ? 0 : (T + k - 1) / k; }

// ------------------------------------------------ binomial checkpointing
// Workspace of the two revolve calls (kept by the caller between them):
// the saved u_0, nslots snapshot slots, the work state, an advance scratch
// field, two adjoint fields, optionally the running sum of the adjoint
// inputs, and the reduction scratch of the adjoint.
struct RevWs {
    size_t origin = 0, slots = 0, work = 0, scratch = 0, lam = 0, lsum = 0;
    size_t partials = 0, sums = 0, dot = 0;
    int nblk = 0;
    size_t total = 0;
};

int layout_rev(int dtype, const Geo &g, int32_t T, int32_t nslots, bool lsum_field, RevWs *w) {
    size_t off = 0;
    if (T == 0 || g.n == 0) {
        w->total = 0;
        return DCP_OK;
    }
    const size_t fb = align_up(g.bytes());
    const int nb = max_blocks(dtype, g);
    if (nb < 0) return DCP_E_SHAPE;
    w->nblk = nb;
    w->origin = off;
    off += fb;
    w->slots = off;
    off += (size_t)nslots * fb;
    w->work = off;
    off += fb;
    w->scratch = off;
    off += fb;
    w->lam = off;
    off += 2 * fb;
    if (lsum_field) {
        w->lsum = off;
        off += fb;
    }
    w->partials = off;
    off += align_up((size_t)T * nb * 2 * sizeof(double));
    w->sums = off;
    off += align_up((size_t)T * 2 * sizeof(double));
    w->dot = off;
    off += align_up(((size_t)ew_norm_blocks(g.n) * 2 + 2) * sizeof(double));
    w->total = off;
    return DCP_OK;
}

struct RevBufs {
    void *ws;
    const RevWs *w;
    int32_t nslots;
    size_t fb;
    void *buf(int32_t id) const {
        if (id == kRvOrigin) return at(ws, w->origin);
        if (id < nslots) return at(ws, w->slots + (size_t)id * fb);
        return at(ws, w->work);
    }
};

// n fused steps from `from` into `to` (n >= 1; both distinct from the
// scratch field), in the passes of `pp` (up to three steps each where the
// grid allows it), alternating between `to` and the scratch so the last pass
// lands in `to`.
int rev_advance(int dtype, int bc, const Geo &g, const dcp_coeffs &c, const Tile &t, const PassPlan &pp,
                const void *f, const void *from, void *to, void *scratch, int64_t n, hipStream_t st) {
    std::vector<int> lens;
    for (int64_t left = n; left > 0;) {
        const int k = pp.len_at(0, (int32_t)std::min<int64_t>(left, INT32_MAX));
        lens.push_back(k);
        left -= k;
    }
    const void *cur = from;
    const size_t L = lens.size();
    for (size_t i = 0; i < L; ++i) {
        void *out = ((L - 1 - i) % 2 == 0) ? to : scratch;
        if (fwd_pass(dtype, bc, g, c, t, pp, lens[i], cur, f, out, nullptr, nullptr, st) != hipSuccess)
            return DCP_E_HIP;
        cur = out;
    }
    return DCP_OK;
}

}  // namespace

extern "C" {

const char *dcp_status_string(int status) {
    switch (status) {
        case DCP_OK: return "ok";
        case DCP_E_NULL: return "a required pointer is NULL";
        case DCP_E_SHAPE: return "invalid grid shape (negative extent or size overflow)";
        case DCP_E_DTYPE: return "invalid dtype (expected DCP_F64 or DCP_F32)";
        case DCP_E_BC: return "invalid boundary (expected DCP_DIRICHLET0 or DCP_PERIODIC)";
        case DCP_E_ARG: return "invalid argument (T, ckpt_every, tblock, h, impl, op or a non-finite coefficient)";
        case DCP_E_WORKSPACE: return "workspace too small";
        case DCP_E_ALIAS: return "an output overlaps an input";
        case DCP_E_SCRATCH:
            return "the grid needs more than the 1 MiB device scratch of the allocation-free entry point";
        case DCP_E_HIP: return "HIP launch or copy failed";
        default: return "unknown status";
    }
}

int32_t dcp_max_tblock(int dtype) { return (dtype == DCP_F64 || dtype == DCP_F32) ? 3 : 1; }

int dcp_workspace_bytes(int op, int dtype, int impl, int64_t nx, int64_t ny, int64_t nz, int32_t T,
                        int32_t ckpt_every, int32_t tblock, int norms, size_t *bytes) {
    if (!bytes) return DCP_E_NULL;
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    switch (op) {
        case DCP_OP_STEP_FUSED:
        case DCP_OP_STEP_UNFUSED: {
            StepWs w;
            if ((rc = layout_step(dtype, op == DCP_OP_STEP_FUSED ? DCP_FUSED : DCP_UNFUSED, g, norms != 0, &w)))
                return rc;
            *bytes = w.total;
            return DCP_OK;
        }
        case DCP_OP_RUN: {
            if (impl != DCP_FUSED && impl != DCP_UNFUSED) return DCP_E_ARG;
            if (T < 0 || tblock < 1 || tblock > dcp_max_tblock(dtype)) return DCP_E_ARG;
            RunWs w;
            if ((rc = layout_run(dtype, impl, g, T, tblock, norms != 0, &w))) return rc;
            *bytes = w.total;
            return DCP_OK;
        }
        case DCP_OP_ADJOINT: {
            if (T < 0 || ckpt_every < 1) return DCP_E_ARG;
            if (tblock < 1 || tblock > dcp_max_tblock(dtype)) return DCP_E_ARG;
            AdjWs w;
            if ((rc = layout_adj(dtype, g, T, ckpt_every, tblock, norms != 0, &w))) return rc;
            *bytes = w.total;
            return DCP_OK;
        }
        default: return DCP_E_ARG;
    }
}

int dcp_step_fused(int dtype, const void *u, const void *f, void *u_out, int64_t nx, int64_t ny, int64_t nz,
                   const dcp_coeffs *coeffs, int bc, double *norms2, void *ws, size_t ws_bytes, void *stream) {
    return step_common(DCP_FUSED, dtype, u, f, u_out, nx, ny, nz, coeffs, bc, norms2, ws, ws_bytes, stream);
}

// ------------------------------------------------ allocation-free fused step
// Scratch of dcp_step_fused_noalloc: the norms' per-workgroup partial sums.
// Every GPU holds its own copy (with the code object) until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device
// memory: kernels and copies get the address hipGetSymbolAddress returns for
// the current device, fetched once per device.
static __device__ __align__(256) double scratch[DCP_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DCP_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DCP_E_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DCP_OK;
}

}  // namespace

int dcp_step_fused_noalloc(int dtype, const void *u, const void *f, void *u_out, int64_t nx, int64_t ny,
                           int64_t nz, const dcp_coeffs *coeffs, int bc, double *norms2, void *stream) {
    // argument errors first (the same checks as dcp_step_fused), then the size
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (bc != DCP_DIRICHLET0 && bc != DCP_PERIODIC) return DCP_E_BC;
    if ((rc = check_coeffs(coeffs))) return rc;
    if (g.n > 0 && (!u || !f || !u_out)) return DCP_E_NULL;
    StepWs w;
    if ((rc = layout_step(dtype, DCP_FUSED, g, norms2 != nullptr, &w))) return rc;
    if (w.total > DCP_NOALLOC_SCRATCH_BYTES) return DCP_E_SCRATCH;
    const size_t fb = g.bytes();
    if (overlaps(u_out, fb, u, fb) || overlaps(u_out, fb, f, fb)) return DCP_E_ALIAS;
    if (norms2 && (overlaps(norms2, 16, u, fb) || overlaps(norms2, 16, f, fb) || overlaps(norms2, 16, u_out, fb)))
        return DCP_E_ALIAS;
    void *ws = nullptr;
    if (w.total > 0 && (rc = scratch_of_current_device(&ws))) return rc;
    return step_common(DCP_FUSED, dtype, u, f, u_out, nx, ny, nz, coeffs, bc, norms2, ws,
                       w.total > 0 ? (size_t)DCP_NOALLOC_SCRATCH_BYTES : 0, stream);
}

int dcp_step_unfused(int dtype, const void *u, const void *f, void *u_out, int64_t nx, int64_t ny, int64_t nz,
                     const dcp_coeffs *coeffs, int bc, double *norms2, void *ws, size_t ws_bytes, void *stream) {
    return step_common(DCP_UNFUSED, dtype, u, f, u_out, nx, ny, nz, coeffs, bc, norms2, ws, ws_bytes, stream);
}

int dcp_run(int dtype, int impl, void *u, const void *f, int64_t nx, int64_t ny, int64_t nz,
            const dcp_coeffs *coeffs, int bc, int32_t T, int32_t tblock, double *energy, double *resid,
            void *ckpt, int32_t ckpt_every, void *ws, size_t ws_bytes, void *stream) {
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (bc != DCP_DIRICHLET0 && bc != DCP_PERIODIC) return DCP_E_BC;
    if ((rc = check_coeffs(coeffs))) return rc;
    if (impl != DCP_FUSED && impl != DCP_UNFUSED) return DCP_E_ARG;
    if (T < 0 || tblock < 1 || tblock > dcp_max_tblock(dtype)) return DCP_E_ARG;
    if (tblock > 1 && impl != DCP_FUSED) return DCP_E_ARG;
    if (ckpt && ckpt_every < 1) return DCP_E_ARG;
    if (g.n > 0 && (!u || !f)) return DCP_E_NULL;
    const bool norms = energy || resid;
    RunWs w;
    if ((rc = layout_run(dtype, impl, g, T, tblock, norms, &w))) return rc;
    if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
    const size_t fb = g.bytes();
    const int32_t nslots = ckpt ? num_slots(T, ckpt_every) : 0;
    const size_t cb = (size_t)nslots * fb;
    const size_t nb = (size_t)(T > 0 ? T : 0) * sizeof(double);
    if (overlaps(u, fb, f, fb)) return DCP_E_ALIAS;
    if (overlaps(ws, w.total, u, fb) || overlaps(ws, w.total, f, fb)) return DCP_E_ALIAS;
    if (overlaps(ckpt, cb, u, fb) || overlaps(ckpt, cb, f, fb) || overlaps(ckpt, cb, ws, w.total))
        return DCP_E_ALIAS;
    for (const double *o : {energy, resid})
        if (o && (overlaps(o, nb, u, fb) || overlaps(o, nb, f, fb) || overlaps(o, nb, ws, w.total) ||
                  overlaps(o, nb, ckpt, cb)))
            return DCP_E_ALIAS;
    if (energy && resid && overlaps(energy, nb, resid, nb)) return DCP_E_ALIAS;

    hipStream_t st = static_cast<hipStream_t>(stream);
    if (T == 0) return DCP_OK;
    if (g.n == 0) {
        if (energy) DCP_TRY(launch_zero(energy, T, st));
        if (resid) DCP_TRY(launch_zero(resid, T, st));
        return DCP_OK;
    }

    void *buf = at(ws, w.field);
    void *tmp[3] = {nullptr, nullptr, nullptr};
    if (impl == DCP_UNFUSED)
        for (int i = 0; i < 3; ++i) tmp[i] = at(ws, w.temps + i * align_up(fb));
    auto slot = [&](int32_t c) { return static_cast<void *>(static_cast<char *>(ckpt) + (size_t)c * fb); };
    bool vok = vec_ok_for(dtype, g, {u, f, buf, tmp[0], tmp[1], tmp[2]});
    for (int32_t c = 0; c < nslots; ++c) vok = vok && aligned16(slot(c));
    const Tile t = pick_tile(dtype, g, vok);
    const int nblk_one = impl == DCP_UNFUSED ? ew_norm_blocks(g.n) : t.nblk;
    const int stride = w.nblk;  // partial slots per step (>= every kernel's workgroup count)
    double *partials = norms ? reinterpret_cast<double *>(at(ws, w.partials)) : nullptr;

    // passes of several steps where the grid allows them and the device has
    // the LDS: three steps (tblock 3), two steps over whole rows (tblock >= 2,
    // rows that fit the LDS) or over x-segments (longer rows)
    const PassPlan pp = plan_passes(dtype, impl, g, T, tblock, vok, norms, stride);
    const bool use_tb = pp.use_tb;
    const TbTile &tb = pp.tb;
    const TbkTile &tk2 = pp.k2, &tk3 = pp.k3;

    // workgroup count behind each step's partials, for the fixed-order finalize
    std::vector<int> step_nblk;
    if (norms) step_nblk.assign((size_t)T, nblk_one);

    auto is_ckpt = [&](int32_t t) { return nslots > 0 && t % ckpt_every == 0 && t / ckpt_every < nslots; };
    if (nslots > 0) DCP_TRY(launch_ew(dtype, EW_COPY, u, nullptr, slot(0), 0.0, g.n, vok, st));
    const void *cur = u;
    for (int32_t s = 0; s < T;) {
        const int32_t len = pp.len_at(s, T);
        const int32_t se = s + len;
        void *nxt = is_ckpt(se) ? slot(se / ckpt_every) : ((cur == u) ? buf : u);
        double *p = partials ? partials + (size_t)s * stride * 2 : nullptr;
        if (len == 3 || (len == 2 && !use_tb)) {
            // checkpoints at the middle steps are stored by the pass itself
            const TbkTile &tk = len == 3 ? tk3 : tk2;
            void *mid[2] = {is_ckpt(s + 1) ? slot((s + 1) / ckpt_every) : nullptr,
                            len == 3 && is_ckpt(s + 2) ? slot((s + 2) / ckpt_every) : nullptr};
            double *part[3] = {p, p ? p + (size_t)stride * 2 : nullptr, p ? p + (size_t)stride * 4 : nullptr};
            DCP_TRY(tbk_fwd_pass(dtype, bc, g, *coeffs, tk, cur, f, nxt, mid, p ? part : nullptr, st));
            if (norms)
                for (int32_t i = s; i < se; ++i) step_nblk[i] = tk.nblk;
        } else if (len == 2) {
            // a checkpoint at the middle step is stored by the pass itself
            void *mid = is_ckpt(s + 1) ? slot((s + 1) / ckpt_every) : nullptr;
            DCP_TRY(tb_fwd_pass(dtype, bc, g, *coeffs, tb, cur, f, nxt, mid, p,
                                p ? p + (size_t)stride * 2 : nullptr, st));
            if (norms) step_nblk[s] = step_nblk[s + 1] = tb.nblk;
        } else if (impl == DCP_FUSED) {
            DCP_TRY(fused_step(dtype, bc, g, *coeffs, t, cur, f, nxt, p, st));
        } else {
            DCP_TRY(unfused_step(dtype, bc, g, *coeffs, t, vok, cur, f, nxt, tmp, p, st));
        }
        cur = nxt;
        s = se;
    }
    if (cur != u) DCP_TRY(launch_ew(dtype, EW_COPY, cur, nullptr, u, 0.0, g.n, vok, st));
    if (norms) {
        // one fixed-order reduction per run of steps that share a workgroup count
        for (int32_t s0 = 0; s0 < T;) {
            int32_t s1 = s0 + 1;
            while (s1 < T && step_nblk[s1] == step_nblk[s0]) ++s1;
            DCP_TRY(launch_finalize(partials + (size_t)s0 * stride * 2, step_nblk[s0], stride, s1 - s0,
                                    energy ? energy + s0 : nullptr, resid ? resid + s0 : nullptr, 1, st));
            s0 = s1;
        }
    }
    return DCP_OK;
}

int dcp_run_plan(int dtype, int impl, int64_t nx, int64_t ny, int64_t nz, int32_t T, int32_t tblock, int norms,
                 dcp_run_info *info) {
    if (!info) return DCP_E_NULL;
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (impl != DCP_FUSED && impl != DCP_UNFUSED) return DCP_E_ARG;
    if (T < 0 || tblock < 1 || tblock > dcp_max_tblock(dtype)) return DCP_E_ARG;
    if (tblock > 1 && impl != DCP_FUSED) return DCP_E_ARG;
    RunWs w;
    if ((rc = layout_run(dtype, impl, g, T, tblock, norms != 0, &w))) return rc;
    std::memset(info, 0, sizeof(*info));
    if (T == 0 || g.n == 0) return DCP_OK;
    const int wide = dtype == DCP_F64 ? 2 : 4;
    const PassPlan pp = plan_passes(dtype, impl, g, T, tblock, g.nx % wide == 0, norms != 0, w.nblk);
    int32_t most = 0;
    for (int32_t s = 0; s < T;) {
        const int32_t len = pp.len_at(s, T);
        ++info->passes[len - 1];
        most = len > most ? len : most;
        s += len;
    }
    info->steps_per_pass = most;
    if (most >= 2) {
        const bool k = most == 3 || !pp.use_tb;
        const TbkTile &tk = most == 3 ? pp.k3 : pp.k2;
        info->segmented = k && tk.seg ? 1 : 0;
        info->tile_rows = k ? tk.ty : pp.tb.ty;
        info->lanes = k ? tk.nt : 1024;
    }
    return DCP_OK;
}

int dcp_adjoint_run(int dtype, const void *ckpt, int32_t ckpt_every, const void *f, const void *lam_T, int64_t nx,
                    int64_t ny, int64_t nz, const dcp_coeffs *coeffs, int bc, int32_t T, int32_t tblock,
                    void *grad_u0, double *grad_ab, void *grad_f, double *grad_gamma, void *ws, size_t ws_bytes,
                    void *stream) {
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (bc != DCP_DIRICHLET0 && bc != DCP_PERIODIC) return DCP_E_BC;
    if ((rc = check_coeffs(coeffs))) return rc;
    if (T < 0 || ckpt_every < 1 || tblock < 1 || tblock > dcp_max_tblock(dtype)) return DCP_E_ARG;
    if (!grad_ab) return DCP_E_NULL;
    if (g.n > 0 && (!f || !lam_T || !grad_u0 || (T > 0 && !ckpt))) return DCP_E_NULL;
    const bool lsum_field = grad_gamma != nullptr && grad_f == nullptr && g.n > 0;
    AdjWs w;
    if ((rc = layout_adj(dtype, g, T, ckpt_every, tblock, lsum_field, &w))) return rc;
    if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
    const size_t fb = g.bytes();
    const int32_t nslots = num_slots(T, ckpt_every);
    const size_t cb = (size_t)nslots * fb;
    if (overlaps(grad_u0, fb, ckpt, cb) || overlaps(grad_u0, fb, f, fb) || overlaps(grad_u0, fb, lam_T, fb) ||
        overlaps(grad_u0, fb, ws, w.total))
        return DCP_E_ALIAS;
    if (overlaps(ws, w.total, ckpt, cb) || overlaps(ws, w.total, f, fb) || overlaps(ws, w.total, lam_T, fb))
        return DCP_E_ALIAS;
    if (overlaps(grad_ab, 16, grad_u0, fb) || overlaps(grad_ab, 16, ws, w.total) || overlaps(grad_ab, 16, ckpt, cb))
        return DCP_E_ALIAS;
    if (grad_f && (overlaps(grad_f, fb, ckpt, cb) || overlaps(grad_f, fb, f, fb) || overlaps(grad_f, fb, lam_T, fb) ||
                   overlaps(grad_f, fb, grad_u0, fb) || overlaps(grad_f, fb, ws, w.total) ||
                   overlaps(grad_f, fb, grad_ab, 16)))
        return DCP_E_ALIAS;
    if (grad_gamma && (overlaps(grad_gamma, 8, grad_ab, 16) || overlaps(grad_gamma, 8, grad_u0, fb) ||
                       overlaps(grad_gamma, 8, grad_f, grad_f ? fb : 0) || overlaps(grad_gamma, 8, ws, w.total) ||
                       overlaps(grad_gamma, 8, ckpt, cb)))
        return DCP_E_ALIAS;

    hipStream_t st = static_cast<hipStream_t>(stream);
    if (T == 0 || g.n == 0) {
        if (g.n > 0)
            DCP_TRY(launch_ew(dtype, EW_COPY, lam_T, nullptr, grad_u0, 0.0, g.n,
                              vec_ok_for(dtype, g, {lam_T, grad_u0}), st));
        if (grad_f && g.n > 0)
            DCP_TRY(launch_ew(dtype, EW_ZERO, nullptr, nullptr, grad_f, 0.0, g.n, vec_ok_for(dtype, g, {grad_f}), st));
        DCP_TRY(launch_zero(grad_ab, 2, st));
        if (grad_gamma) DCP_TRY(launch_zero(grad_gamma, 1, st));
        return DCP_OK;
    }
    // running sum of the adjoint inputs lambda_T .. lambda_1 (for dL/df and dL/dgamma)
    void *lsum = grad_f ? grad_f : (lsum_field ? static_cast<void *>(at(ws, w.lsum)) : nullptr);

    void *lam[2] = {at(ws, w.lam), at(ws, w.lam + align_up(fb))};
    const int32_t kk = ckpt_every < T ? ckpt_every : T;
    auto seg = [&](int32_t j) { return static_cast<void *>(at(ws, w.seg + (size_t)j * align_up(fb))); };
    auto slot = [&](int32_t c) { return static_cast<const void *>(static_cast<const char *>(ckpt) + (size_t)c * fb); };
    bool vok = vec_ok_for(dtype, g, {f, lam_T, grad_u0, lam[0], lam[1]});
    if (lsum) vok = vok && aligned16(lsum);
    for (int32_t c = 0; c < nslots; ++c) vok = vok && aligned16(slot(c));
    for (int32_t j = 0; j + 1 < kk; ++j) vok = vok && aligned16(seg(j));
    const Tile t = pick_tile(dtype, g, vok);
    double *partials = reinterpret_cast<double *>(at(ws, w.partials));
    double *sums = reinterpret_cast<double *>(at(ws, w.sums));
    const int stride = w.nblk;
    const dcp_coeffs &c = *coeffs;
    TbTile tb{};
    const bool use_tb = plan_tb(dtype, g, tblock, vok, &tb) && tb.nblk <= stride;
    const PassPlan fpp = plan_passes(dtype, DCP_FUSED, g, T, tblock, vok, false, 0);  // recomputation

    StencilArgs aa{};
    aa.nx = g.nx;
    aa.ny = g.ny;
    aa.nz = g.nz;
    aa.c0 = c.dt * c.alpha / (c.h * c.h);
    aa.c1 = 3.0 * c.dt * c.beta;
    aa.tiles_x = t.tiles_x;
    aa.tiles_y = t.tiles_y;
    aa.zc = t.zc;
    aa.nblk = t.nblk;
    TbArgs ta{};
    ta.nx = g.nx;
    ta.ny = g.ny;
    ta.nz = g.nz;
    ta.c0 = aa.c0;
    ta.c1 = aa.c1;
    ta.nslab = tb.nslab;
    ta.zc = tb.zc;

    // Adjoint steps are taken in pairs (2m+1, 2m) by global parity, whatever
    // the checkpoint interval: a pair whose lower step lies in the previous
    // segment waits for that segment (its upper state is a checkpoint slot).
    // Every step's parameter sums therefore come from the same kernel with the
    // same tiling for any k, and the gradient does not depend on k bit for bit.
    std::vector<int> step_nblk((size_t)T, t.nblk);
    const int adj_op = lsum ? SOP_ADJL : SOP_ADJ;
    aa.lam = lsum;
    ta.lam = lsum;
    int lam_first = 1;
    const void *lcur = lam_T;
    int32_t s = T - 1;  // next adjoint step to take
    for (int32_t cs = nslots - 1; cs >= 0; --cs) {
        const int32_t t0 = cs * ckpt_every;
        const int32_t t1 = (t0 + ckpt_every < T) ? t0 + ckpt_every : T;
        // recompute the states u_{t0+1} .. u_{t1-1} of this segment (u_{t0+j}
        // into seg(j-1)), up to three steps per pass, every state stored
        const void *prev = slot(cs);
        for (int32_t j = 1; j < t1 - t0;) {
            const int32_t left = t1 - t0 - j;
            const int len = fpp.len_at(0, left);
            DCP_TRY(fwd_pass(dtype, bc, g, c, t, fpp, len, prev, f, seg(j + len - 2),
                             len >= 2 ? seg(j - 1) : nullptr, len == 3 ? seg(j) : nullptr, st));
            prev = seg(j + len - 2);
            j += len;
        }
        // u_t for t in [t0, t1], the upper end being the next slot
        auto state = [&](int32_t tt) -> const void * {
            if (tt % ckpt_every == 0) return slot(tt / ckpt_every);
            return seg(tt - t0 - 1);
        };
        while (s >= t0) {
            const bool pair = use_tb && (s & 1) && s >= 1;
            if (pair && s - 1 < t0) break;  // the lower step lives in the previous segment
            const int32_t se = pair ? s - 1 : s;
            void *out = (se == 0) ? grad_u0 : (lcur == lam[0] ? lam[1] : lam[0]);
            if (pair) {
                ta.u = lcur;
                ta.f = state(s);
                ta.g2 = state(s - 1);
                ta.out = out;
                ta.mid = nullptr;
                ta.part1 = partials + (size_t)s * stride * 2;
                ta.part2 = partials + (size_t)(s - 1) * stride * 2;
                ta.lam_first = lam_first;
                DCP_TRY(launch_tb2(dtype, adj_op, bc, true, tb, ta, st));
                step_nblk[s] = step_nblk[s - 1] = tb.nblk;
            } else {
                aa.s = lcur;
                aa.q = state(s);
                aa.out = out;
                aa.partials = partials + (size_t)s * stride * 2;
                aa.lam_first = lam_first;
                DCP_TRY(launch_stencil(dtype, adj_op, bc, true, t, aa, st));
            }
            lam_first = 0;
            lcur = out;
            s = se - 1;
        }
    }
    // per-step sums in a fixed order, then over the steps in a fixed order
    for (int32_t s0 = 0; s0 < T;) {
        int32_t s1 = s0 + 1;
        while (s1 < T && step_nblk[s1] == step_nblk[s0]) ++s1;
        DCP_TRY(launch_finalize(partials + (size_t)s0 * stride * 2, step_nblk[s0], stride, s1 - s0,
                                sums + 2 * (size_t)s0, nullptr, 2, st));
        s0 = s1;
    }
    DCP_TRY(launch_grad_finalize(sums, T, c.dt / (c.h * c.h), -c.dt, grad_ab, st));
    if (lsum) {
        // dL/dgamma = dt * <sum, f> (fixed-order double reduction), then
        // dL/df = gamma * dt * sum in place
        if (grad_gamma) {
            double *dp = reinterpret_cast<double *>(at(ws, w.dot));
            const int nb = ew_norm_blocks(g.n);
            double *pair = dp + 2 * (size_t)nb;
            DCP_TRY(launch_ew_dot(dtype, lsum, f, dp, g.n, vec_ok_for(dtype, g, {lsum, f}), st));
            DCP_TRY(launch_finalize(dp, nb, nb, 1, pair, nullptr, 0, st));
            DCP_TRY(launch_scalar_scale(pair, c.dt, grad_gamma, st));
        }
        if (grad_f)
            DCP_TRY(launch_ew(dtype, EW_SCALE, grad_f, nullptr, grad_f, c.gamma * c.dt, g.n,
                              vec_ok_for(dtype, g, {grad_f}), st));
    }
    return DCP_OK;
}

int dcp_revolve_workspace_bytes(int dtype, int64_t nx, int64_t ny, int64_t nz, int32_t T, int32_t nslots,
                                int lsum_field, size_t *bytes) {
    if (!bytes) return DCP_E_NULL;
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (T < 0 || nslots < 0) return DCP_E_ARG;
    RevWs w;
    if ((rc = layout_rev(dtype, g, T, nslots, lsum_field != 0, &w))) return rc;
    *bytes = w.total;
    return DCP_OK;
}

int dcp_revolve_forward(int dtype, void *u, const void *f, int64_t nx, int64_t ny, int64_t nz,
                        const dcp_coeffs *coeffs, int bc, int32_t T, int32_t nslots, int32_t tblock, void *ws,
                        size_t ws_bytes, void *stream) {
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (bc != DCP_DIRICHLET0 && bc != DCP_PERIODIC) return DCP_E_BC;
    if ((rc = check_coeffs(coeffs))) return rc;
    if (T < 0 || nslots < 0 || tblock < 1 || tblock > dcp_max_tblock(dtype)) return DCP_E_ARG;
    if (g.n > 0 && (!u || !f)) return DCP_E_NULL;
    RevWs w;
    if ((rc = layout_rev(dtype, g, T, nslots, false, &w))) return rc;
    // the running-sum field, if any, sits after the fields used here
    if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
    const size_t fb = g.bytes();
    if (overlaps(u, fb, f, fb) || overlaps(ws, ws_bytes, u, fb) || overlaps(ws, ws_bytes, f, fb)) return DCP_E_ALIAS;
    if (T == 0 || g.n == 0) return DCP_OK;
    std::vector<RvOp> ops;
    if (!revolve_schedule(T, nslots, &ops, nullptr)) return DCP_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const RevBufs B{ws, &w, nslots, align_up(fb)};
    void *scratch = at(ws, w.scratch);
    bool vok = vec_ok_for(dtype, g, {u, f, B.buf(kRvOrigin), B.buf(nslots), scratch});
    for (int32_t i = 0; i < nslots; ++i) vok = vok && aligned16(B.buf(i));
    const Tile t = pick_tile(dtype, g, vok);
    const PassPlan pp = plan_passes(dtype, DCP_FUSED, g, T, tblock, vok, false, 0);
    const dcp_coeffs &c = *coeffs;
    DCP_TRY(launch_ew(dtype, EW_COPY, u, nullptr, B.buf(kRvOrigin), 0.0, g.n, vok, st));
    // the schedule's opening chain of advances, u_0 -> ... -> u_{T-1}, stores
    // the snapshots the reverse sweep starts from
    int32_t last = kRvOrigin;
    for (const RvOp &op : ops) {
        if (op.kind != kRvAdvance) break;
        if ((rc = rev_advance(dtype, bc, g, c, t, pp, f, B.buf(op.src), B.buf(op.dst), scratch, op.t1 - op.t0,
                              st)))
            return rc;
        last = op.dst;
    }
    DCP_TRY(fused_step(dtype, bc, g, c, t, B.buf(last), f, u, nullptr, st));  // u_T
    return DCP_OK;
}

int dcp_revolve_adjoint(int dtype, const void *f, const void *lam_T, int64_t nx, int64_t ny, int64_t nz,
                        const dcp_coeffs *coeffs, int bc, int32_t T, int32_t nslots, int32_t tblock,
                        void *grad_u0, double *grad_ab, void *grad_f, double *grad_gamma, void *ws,
                        size_t ws_bytes, void *stream) {
    Geo g;
    int rc = check_geo(dtype, nx, ny, nz, &g);
    if (rc) return rc;
    if (bc != DCP_DIRICHLET0 && bc != DCP_PERIODIC) return DCP_E_BC;
    if ((rc = check_coeffs(coeffs))) return rc;
    if (T < 0 || nslots < 0 || tblock < 1 || tblock > dcp_max_tblock(dtype)) return DCP_E_ARG;
    if (!grad_ab) return DCP_E_NULL;
    if (g.n > 0 && (!f || !lam_T || !grad_u0)) return DCP_E_NULL;
    const bool lsum_field = grad_gamma != nullptr && grad_f == nullptr && g.n > 0;
    RevWs w;
    if ((rc = layout_rev(dtype, g, T, nslots, lsum_field, &w))) return rc;
    if ((rc = check_ws(ws, ws_bytes, w.total))) return rc;
    const size_t fb = g.bytes();
    const size_t wsz = w.total;
    for (const void *p : {f, lam_T})
        if (overlaps(grad_u0, fb, p, fb) || overlaps(ws, wsz, p, fb) || (grad_f && overlaps(grad_f, fb, p, fb)))
            return DCP_E_ALIAS;
    if (overlaps(grad_u0, fb, ws, wsz) || overlaps(grad_ab, 16, ws, wsz) || overlaps(grad_ab, 16, grad_u0, fb))
        return DCP_E_ALIAS;
    if (grad_f && (overlaps(grad_f, fb, ws, wsz) || overlaps(grad_f, fb, grad_u0, fb) ||
                   overlaps(grad_f, fb, grad_ab, 16)))
        return DCP_E_ALIAS;
    if (grad_gamma && (overlaps(grad_gamma, 8, grad_ab, 16) || overlaps(grad_gamma, 8, grad_u0, fb) ||
                       overlaps(grad_gamma, 8, grad_f, grad_f ? fb : 0) || overlaps(grad_gamma, 8, ws, wsz)))
        return DCP_E_ALIAS;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (T == 0 || g.n == 0) {
        if (g.n > 0)
            DCP_TRY(launch_ew(dtype, EW_COPY, lam_T, nullptr, grad_u0, 0.0, g.n,
                              vec_ok_for(dtype, g, {lam_T, grad_u0}), st));
        if (grad_f && g.n > 0)
            DCP_TRY(launch_ew(dtype, EW_ZERO, nullptr, nullptr, grad_f, 0.0, g.n, vec_ok_for(dtype, g, {grad_f}), st));
        DCP_TRY(launch_zero(grad_ab, 2, st));
        if (grad_gamma) DCP_TRY(launch_zero(grad_gamma, 1, st));
        return DCP_OK;
    }
    std::vector<RvOp> ops;
    if (!revolve_schedule(T, nslots, &ops, nullptr)) return DCP_E_ARG;
    const RevBufs B{ws, &w, nslots, align_up(fb)};
    void *scratch = at(ws, w.scratch);
    void *lam[2] = {at(ws, w.lam), at(ws, w.lam + align_up(fb))};
    void *lsum = grad_f ? grad_f : (lsum_field ? static_cast<void *>(at(ws, w.lsum)) : nullptr);
    bool vok = vec_ok_for(dtype, g, {f, lam_T, grad_u0, grad_f, B.buf(kRvOrigin), B.buf(nslots), scratch,
                                     lam[0], lam[1], lsum});
    for (int32_t i = 0; i < nslots; ++i) vok = vok && aligned16(B.buf(i));
    const Tile t = pick_tile(dtype, g, vok);
    const PassPlan pp = plan_passes(dtype, DCP_FUSED, g, T, tblock, vok, false, 0);
    const dcp_coeffs &c = *coeffs;
    double *partials = reinterpret_cast<double *>(at(ws, w.partials));
    double *sums = reinterpret_cast<double *>(at(ws, w.sums));
    const int stride = w.nblk;
    StencilArgs aa{};
    aa.nx = g.nx;
    aa.ny = g.ny;
    aa.nz = g.nz;
    aa.c0 = c.dt * c.alpha / (c.h * c.h);
    aa.c1 = 3.0 * c.dt * c.beta;
    aa.tiles_x = t.tiles_x;
    aa.tiles_y = t.tiles_y;
    aa.zc = t.zc;
    aa.nblk = t.nblk;
    aa.lam = lsum;
    aa.c1f = c.dt * c.beta;  // the forward step's coefficients, for the fused recomputation
    aa.c2f = c.dt * c.gamma;
    // two adjoint steps per pass where both states are at hand (tblock >= 2)
    TbTile tb{};
    const bool use_tb = tblock >= 2 && plan_tb(dtype, g, tblock, vok, &tb) && tb.nblk <= stride;
    TbArgs ta{};
    ta.nx = g.nx;
    ta.ny = g.ny;
    ta.nz = g.nz;
    ta.c0 = aa.c0;
    ta.c1 = aa.c1;
    ta.nslab = tb.nslab;
    ta.zc = tb.zc;
    ta.lam = lsum;
    std::vector<int> step_nblk((size_t)T, t.nblk);
    const int adj_op = lsum ? SOP_ADJL : SOP_ADJ;
    const int adj_rop = lsum ? SOP_ADJLR : SOP_ADJR;
    int lam_first = 1;
    const void *lcur = lam_T;
    // A one-step advance whose result only the next adjoint step reads is
    // folded into that step: the adjoint kernel recomputes u_s at each point
    // from u_{s-1}, with the advance's arithmetic, instead of reading it.
    auto fold = [&](size_t i) {
        const RvOp &a = ops[i];
        if (a.kind != kRvAdvance || a.t1 - a.t0 != 1 || i + 1 >= ops.size()) return false;
        const RvOp &b = ops[i + 1];
        if (b.kind != kRvAdjoint || b.src != a.dst || b.t0 != a.t1) return false;
        for (size_t j = i + 2; j < ops.size(); ++j) {  // is the advance's buffer read again?
            if (ops[j].src == a.dst) return false;
            if (ops[j].kind == kRvAdvance && ops[j].dst == a.dst) break;
        }
        return true;
    };
    // A chain of one-step advances, each from the previous one's state into
    // a buffer of its own, is one pass of two or three steps that stores
    // every state it passes.
    auto chain = [&](size_t i) {
        size_t j = i;
        while (j + 1 < ops.size() && j - i < 2) {
            const RvOp &a = ops[j], &b = ops[j + 1];
            if (b.kind != kRvAdvance || b.t1 - b.t0 != 1 || b.src != a.dst || b.t0 != a.t1) break;
            bool fresh = b.dst != ops[i].src;
            for (size_t k = i; k <= j; ++k) fresh = fresh && ops[k].dst != b.dst;
            if (!fresh) break;
            ++j;
        }
        return j > i ? pp.len_at(0, (int32_t)(j - i + 1)) : 1;
    };
    // the opening chain of advances was run by dcp_revolve_forward
    size_t i0 = 0;
    while (i0 < ops.size() && ops[i0].kind == kRvAdvance) ++i0;
    for (size_t i = i0; i < ops.size(); ++i) {
        const RvOp &op = ops[i];
        if (op.kind == kRvAdvance && op.t1 - op.t0 == 1) {
            const int len = chain(i);
            if (len >= 2) {
                DCP_TRY(fwd_pass(dtype, bc, g, c, t, pp, len, B.buf(op.src), f, B.buf(ops[i + len - 1].dst),
                                 B.buf(op.dst), len == 3 ? B.buf(ops[i + 1].dst) : nullptr, st));
                i += len - 1;
                continue;
            }
        }
        const bool folded = fold(i);
        if (op.kind == kRvAdvance && !folded) {
            if ((rc = rev_advance(dtype, bc, g, c, t, pp, f, B.buf(op.src), B.buf(op.dst), scratch,
                                  op.t1 - op.t0, st)))
                return rc;
            continue;
        }
        // adjoint step s with u_s in buffer src, or recomputed from u_{s-1};
        // or steps s and s - 1 when the next operation is step s - 1
        const RvOp &adj = folded ? ops[i + 1] : op;
        const int64_t s = adj.t0;
        const bool pair = !folded && use_tb && i + 1 < ops.size() && ops[i + 1].kind == kRvAdjoint &&
                          ops[i + 1].t0 == s - 1;
        const int64_t se = pair ? s - 1 : s;
        void *out = (se == 0) ? grad_u0 : (lcur == lam[0] ? lam[1] : lam[0]);
        if (pair) {
            ta.u = lcur;
            ta.f = B.buf(adj.src);
            ta.g2 = B.buf(ops[i + 1].src);
            ta.out = out;
            ta.mid = nullptr;
            ta.part1 = partials + (size_t)s * stride * 2;
            ta.part2 = partials + (size_t)(s - 1) * stride * 2;
            ta.lam_first = lam_first;
            DCP_TRY(launch_tb2(dtype, adj_op, bc, true, tb, ta, st));
            step_nblk[s] = step_nblk[s - 1] = tb.nblk;
        } else {
            aa.s = lcur;
            aa.q = folded ? f : B.buf(adj.src);
            aa.s2 = folded ? B.buf(op.src) : nullptr;
            aa.out = out;
            aa.partials = partials + (size_t)s * stride * 2;
            aa.lam_first = lam_first;
            DCP_TRY(launch_stencil(dtype, folded ? adj_rop : adj_op, bc, true, t, aa, st));
        }
        lam_first = 0;
        lcur = out;
        if (folded || pair) ++i;
    }
    // per-step sums in a fixed order, then over the steps in a fixed order
    for (int32_t s0 = 0; s0 < T;) {
        int32_t s1 = s0 + 1;
        while (s1 < T && step_nblk[s1] == step_nblk[s0]) ++s1;
        DCP_TRY(launch_finalize(partials + (size_t)s0 * stride * 2, step_nblk[s0], stride, s1 - s0,
                                sums + 2 * (size_t)s0, nullptr, 2, st));
        s0 = s1;
    }
    DCP_TRY(launch_grad_finalize(sums, T, c.dt / (c.h * c.h), -c.dt, grad_ab, st));
    if (lsum) {
        if (grad_gamma) {
            double *dp = reinterpret_cast<double *>(at(ws, w.dot));
            const int nb = ew_norm_blocks(g.n);
            double *pair = dp + 2 * (size_t)nb;
            DCP_TRY(launch_ew_dot(dtype, lsum, f, dp, g.n, vec_ok_for(dtype, g, {lsum, f}), st));
            DCP_TRY(launch_finalize(dp, nb, nb, 1, pair, nullptr, 0, st));
            DCP_TRY(launch_scalar_scale(pair, c.dt, grad_gamma, st));
        }
        if (grad_f)
            DCP_TRY(launch_ew(dtype, EW_SCALE, grad_f, nullptr, grad_f, c.gamma * c.dt, g.n,
                              vec_ok_for(dtype, g, {grad_f}), st));
    }
    return DCP_OK;
}

}  // extern "C"
