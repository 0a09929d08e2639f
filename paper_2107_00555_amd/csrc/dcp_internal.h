// dcp_internal.h -- launch interface between the host driver (dcp_api.cpp)
// and the gfx950 kernels (dcp_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

namespace dcp {

// Tuning overrides: environment variables that force a tiling or a pass
// schedule (DCP_TILE_SHAPE, DCP_TILE_ZC, DCP_TB_CFG, DCP_TBK_CFG,
// DCP_TBK_SBLK, DCP_FUSE_ZR, DCP_J1_K, DCP_J2_CFG, DCP_J2_MODE,
// DCP_J2M_CPL).  They are honoured only while DCP_TUNING=1 is also set, so a
// stray variable alone changes nothing.
// Every forced choice computes the same fields; a norm's summation order
// follows the tiles.
inline const char *tuning_env(const char *name) {
    const char *on = getenv("DCP_TUNING");
    if (!on || strcmp(on, "1") != 0) return nullptr;
    return getenv(name);
}

enum StencilOp : int {
    SOP_FWD = 0,  // u' = u + c0*(S6 - 6u) - c1*u^3 + c2*f      (S6 = sum of 6 neighbours)
    SOP_ADJ = 1,  // l' = l + c0*(S6 - 6l) - c1*u^2*l ; sums (S6-6l)*u and l*u^3
    SOP_LAP = 2,  // lap = (((((xm+xp)+ym)+yp)+zm)+zp - 6u) / c0, one rounding per op
    SOP_ADJL = 3, // SOP_ADJ, and lam += l (the adjoint step's input, lambda_{t+1});
                  // lam_first: lam = l + 0 without reading lam
    SOP_ADJR = 4, // SOP_ADJ with u = u_t recomputed at each point from u_{t-1}
                  // (operand s2, stenciled) and f (operand q) by SOP_FWD's
                  // arithmetic with c0, c1f, c2f: one forward step and one
                  // adjoint step in one pass
    SOP_ADJLR = 5,  // SOP_ADJR, and lam += l as in SOP_ADJL
};

// Tile of one workgroup: 64*bxw*vec points along x (bxw waves side by side),
// by*ry rows along y (by waves stacked, ry rows per lane), zc planes along z.
struct Tile {
    int vec;  // elements per lane along x (16-byte vectors, or 1)
    int bxw, by, ry;
    int zc;
    int tiles_x, tiles_y, tiles_z;
    int nblk;
};

struct StencilArgs {
    const void *s;       // stencil operand (u, or lambda_{t+1})
    const void *q;       // point operand (f, or u_t); unused by SOP_LAP
    void *out;           // output field
    double *partials;    // [nblk][2] per-workgroup sums, or null
    void *lam;           // SOP_ADJL, SOP_ADJLR: running sum of the adjoint inputs
    const void *s2;      // SOP_ADJR, SOP_ADJLR: u_{t-1} (stencil operand of the recomputation)
    int64_t nx, ny, nz;
    double c0, c1, c2;
    double c1f, c2f;     // SOP_ADJR, SOP_ADJLR: the forward step's c1 and c2
    int tiles_x, tiles_y, zc, nblk;
    int lam_first;
};

// Tile shapes compiled into the library, in preference order.
struct Shape {
    int bxw, by, ry;
};
int num_shapes();
Shape shape_at(int i);

// Launches the z-marching stencil kernel.  `reduce` selects the variant
// that writes per-workgroup double sums to a.partials.
hipError_t launch_stencil(int dtype, int op, int bc, bool reduce, const Tile &t,
                          const StencilArgs &a, hipStream_t stream);

// Element-wise statements of the unfused program, and a plain copy (o = x)
// used for checkpoint slots and copy-backs.
enum EwOp : int { EW_POW3 = 0, EW_SCALE = 1, EW_SUB = 2, EW_ADD = 3, EW_COPY = 4, EW_ZERO = 5 };
hipError_t launch_ew(int dtype, int op, const void *x, const void *y, void *o,
                     double a, int64_t n, bool vec_ok, hipStream_t stream);

// Per-workgroup sums {sum o^2, sum (o - u)^2} for the unfused program.
int ew_norm_blocks(int64_t n);
hipError_t launch_ew_norms(int dtype, const void *o, const void *u,
                           double *partials, int64_t n, bool vec_ok,
                           hipStream_t stream);
// Per-workgroup sums {sum a*b, 0} in double (ew_norm_blocks(n) workgroups).
hipError_t launch_ew_dot(int dtype, const void *a, const void *b,
                         double *partials, int64_t n, bool vec_ok,
                         hipStream_t stream);
// dst[0] = s * src[0].
hipError_t launch_scalar_scale(const double *src, double s, double *dst,
                               hipStream_t stream);

// Two fused steps per pass (temporal blocking): full-row slabs of ty rows,
// zc planes per run, one 1024-lane workgroup per slab-run.
//   SOP_FWD: u = u_t, f = f, out = u_{t+2}, mid = u_{t+1} or null;
//            part1/part2 = norms of steps t+1 / t+2 (or null)
//   SOP_ADJ: u = lambda_{t+1}, f = u_t, g2 = u_{t-1}, out = lambda_{t-1};
//            part1/part2 = parameter sums of steps t / t-1
//   SOP_ADJL: SOP_ADJ, and lam = (lam + lambda_{t+1}) + lambda_t on the owned
//            points (lam_first: lam is not read, taken as 0)
struct TbArgs {
    const void *u;
    const void *f;
    const void *g2;
    void *out;
    void *mid;
    double *part1;      // [nblk][2]
    double *part2;      // [nblk][2]
    void *lam;
    int64_t nx, ny, nz;
    double c0, c1, c2;
    int nslab, zc;
    int lam_first;
};
struct TbTile {
    int vec, ty, nt, km, zc, nslab, nruns, nblk;
    size_t lds_bytes;
};
// Plans a two-step pass for this grid; false if the kernel does not apply
// (rows too long for the LDS budget, or no 16-byte lanes).
bool tb_plan(int dtype, int64_t nx, int64_t ny, int64_t nz, bool vec_ok, size_t lds_limit,
             TbTile *t);
hipError_t launch_tb2(int dtype, int op, int bc, bool reduce, const TbTile &t, const TbArgs &a,
                      hipStream_t stream);

// B fused forward steps per pass (B = 2 or 3) on tiles of full rows or of
// x-segments with a halo (dcp_tbk.hip).
//   u = u_t, f = f, out = u_{t+B}; mid[s-1] = u_{t+s} (s = 1 .. B-1) on the
//   owned points, or null; part[s-1] = norms of step t+s ([nblk][2]) when
//   the pass reduces.
struct TbkArgs {
    const void *u;
    const void *f;
    void *out;
    void *mid[2];
    double *part[3];
    int64_t nx, ny, nz;
    double c0, c1, c2;
    int ty, nslab, nseg, zc, wc, halo, chf;
    int sblk;  // slabs per block of the tile order (see TbkTile)
};
struct TbkTile {
    int B, vec, ty, nt, km;
    bool seg;             // x-segments with a halo (false: whole rows)
    int wc, halo, chf;    // segment chunks, halo chunks per side, frame chunks per row
    int nseg, nslab, zc, nruns, nblk;
    // Tile order within a z-run: blocks of sblk slabs, each block taking all
    // its segments (slab fastest), so that the tiles one XCD runs together
    // (a contiguous range) are neighbours along x and y.
    int sblk;
    size_t lds_bytes;
};
// Plans a B-step pass; false if the kernel does not apply (no 16-byte lanes,
// or no tile fits the LDS).  lanes: 768 (the ring form, planes under 4
// GiB), 1024 or 512 lanes per workgroup.  When
// force_wc > 0 only segments of that many chunks (or whole rows, if it
// covers the row) are considered; force_ty > 0 fixes the slab height.
bool tbk_plan(int dtype, int B, int64_t nx, int64_t ny, int64_t nz, bool vec_ok, size_t lds_limit, int lanes,
              int force_wc, int force_ty, TbkTile *t);
hipError_t launch_tbk(int dtype, int bc, bool reduce, const TbkTile &t, const TbkArgs &a, hipStream_t stream);

// Fixed-order reduction of [nsteps][stride][2] partials (first nblk used).
//   mode 0: out0[0] = sum k=0, out0[1] = sum k=1          (one step)
//   mode 1: out0[s] = sum k=0, out1[s] = sqrt(sum k=1)   (either may be null)
//   mode 2: out0[2s+k] = sum k                           (per-step sums)
hipError_t launch_finalize(const double *partials, int nblk, int stride, int nsteps,
                           double *out0, double *out1, int mode,
                           hipStream_t stream);

// grad[0] = s0 * sum_t sums[2t], grad[1] = s1 * sum_t sums[2t+1] (t ascending).
hipError_t launch_grad_finalize(const double *sums, int nsteps, double s0,
                                double s1, double *grad, hipStream_t stream);

// dst[0..n) = 0 (doubles), a kernel rather than a memset node.
hipError_t launch_zero(double *dst, int64_t n, hipStream_t stream);

// Binomial checkpointing schedule (dcp_revolve.cpp).  Buffers: kRvOrigin =
// the saved u_0, 0 .. nslots-1 = snapshot slots, nslots = the work state.
//   kRvAdvance: state of buffer src (time t0) advanced to time t1 into dst
//   kRvAdjoint: adjoint step t0 with u_{t0} in buffer src
// Adjoint steps come in the order T-1, T-2, ..., 0.
constexpr int kRvOrigin = -1;
constexpr int kRvAdvance = 0, kRvAdjoint = 1;
struct RvOp {
    int kind;
    int32_t src, dst;
    int64_t t0, t1;
};
bool revolve_schedule(int64_t T, int32_t nslots, std::vector<RvOp> *ops, int64_t *forward_steps);

}  // namespace dcp
