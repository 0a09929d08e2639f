// dcp_jacobi.hip -- the two Jacobi stencil programs the paper lists
// (jacobi_1d, Sec. 2.2; jacobi_2d, Sec. 4.3) on gfx950, and their C ABI.
//
// Each pass of the listings' time loop writes B's interior from A, then A's
// interior from B; the ends (1D) or the outer rows and columns (2D) of both
// arrays are never written.  Every new value is the listing's sum, added left
// to right, times the listing's weight, each operation rounded once (the
// library is built without FP contraction), so the results equal the plain
// serial evaluation bit for bit.
//
// Temporal blocking in registers.  A launch ("pass") applies several
// half-steps to a tile of the arrays plus a halo as wide as the number of
// half-steps, so only the tile's values need to be exact at the end and the
// halo is recomputed redundantly.  The tile's state lives in VGPRs for the
// whole pass: each lane holds a short run of points of both arrays; in-wave
// neighbours come from lane shuffles and (2D) the rows on the edge of a
// wave's band are exchanged through LDS with one barrier per half-step.
// A pass reads A (and B where it is fixed) once and writes both once, so
// the HBM traffic per half-step falls by the number of half-steps per pass.
// Passes read one pair of arrays and write the other (the caller's arrays
// and a workspace copy, in turn); the pass count is even, so the result
// ends in the caller's arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "dcp.h"
#include "dcp_internal.h"

namespace {

constexpr double kW1 = 0.33333;  // jacobi_1d weight, as the listing writes it
constexpr double kW2 = 0.2;      // jacobi_2d weight

// bfix: where B's boundary cells are read (they never change).  write_b:
// 0 = B is not stored (no later pass reads B's interior), 1 = the tile of B
// is stored, 2 = only B's interior cells of the tile are stored (bout is the
// array bfix points to).
struct J1Args {
    const double *ain, *bin, *bfix;
    double *aout, *bout;
    int64_t n, inner;
    int hh, nhalf, phase;  // halo, half-steps in this pass, 1 = first half-step writes A
    int write_b;
};

// vec16: every lane's two columns are one aligned 16-byte pair (n1 and hh
// even, arrays 16-byte aligned), so loads and stores move both at once.
// set: which tiles this launch covers: 0 = all, 1 = the interior rectangle
// [r_lo, r_hi] x [c_lo, c_hi] of tiles whose region holds no boundary cell of
// the array, 2 = the ring of the other tiles (see j2_tile).
struct J2Args {
    const double *ain, *bin, *bfix;
    double *aout, *bout;
    int64_t n0, n1;
    int inner_r, inner_c, tiles_r, tiles_c;
    int hh, nhalf, phase, write_b, vec16;
    int set, r_lo, r_hi, c_lo, c_hi;
};

// Tile (row, column) of workgroup b (after the XCD renumbering).  Tiles run
// column by column, so a tile's upper and lower neighbours (whose halos it
// shares, the larger overlap) are recent in the same XCD's L2.
__device__ __forceinline__ void j2_tile(const J2Args &a, int b, int &tr, int &tc) {
    if (a.set == 0) {
        tr = b % a.tiles_r;
        tc = b / a.tiles_r;
        return;
    }
    if (a.set == 1) {
        const int nr = a.r_hi - a.r_lo + 1;
        tr = a.r_lo + b % nr;
        tc = a.c_lo + b / nr;
        return;
    }
    // ring: the rows above and below the rectangle in full, then the columns
    // left and right of it on the rectangle's rows
    const int top = a.r_lo * a.tiles_c, below = (a.tiles_r - 1 - a.r_hi) * a.tiles_c;
    if (b < top) {
        tr = b / a.tiles_c;
        tc = b % a.tiles_c;
        return;
    }
    b -= top;
    if (b < below) {
        tr = a.r_hi + 1 + b / a.tiles_c;
        tc = b % a.tiles_c;
        return;
    }
    b -= below;
    const int nr = a.r_hi - a.r_lo + 1, left = a.c_lo, right = a.tiles_c - 1 - a.c_hi;
    if (b < nr * left) {
        tr = a.r_lo + b / left;
        tc = b % left;
        return;
    }
    b -= nr * left;
    tr = a.r_lo + b / right;
    tc = a.c_hi + 1 + b % right;
}

__device__ __forceinline__ int j_xcd_remap(int b, int nb) {
    // consecutive workgroups go to different XCDs; number the tiles so that
    // an XCD works on a contiguous run of them (neighbouring halos share L2)
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, j = b >> 3;
    return xcd * per + min(xcd, rem) + j;
}

// Cross-lane moves within a wave as DPP wavefront shifts (full-rate VALU,
// no LDS round trip).  from_lower: lane i receives x of lane i-1 (lane 0
// receives 0); from_upper: lane i receives x of lane i+1 (lane 63: 0).
template <int CTRL>
__device__ __forceinline__ double j_dpp(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_lower(double x) { return j_dpp<0x138>(x); }  // wave_shr:1
__device__ __forceinline__ double from_upper(double x) { return j_dpp<0x130>(x); }  // wave_shl:1

// keep[lane] ? old : nv, as two v_cndmask_b32 (a plain ?: here is turned
// into a branch per cell, which serialises the unrolled update)
__device__ __forceinline__ double j_keep(uint64_t keep, double nv, double old) {
    const uint64_t nb = __builtin_bit_cast(uint64_t, nv), ob = __builtin_bit_cast(uint64_t, old);
    unsigned lo, hi;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(lo) : "v"((unsigned)nb), "v"((unsigned)ob), "s"(keep));
    asm("v_cndmask_b32_e64 %0, %1, %2, %3"
        : "=v"(hi)
        : "v"((unsigned)(nb >> 32)), "v"((unsigned)(ob >> 32)), "s"(keep));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Which cells a half-step may overwrite.  Only the array's own boundary
// cells must keep their values: a cell on the region's edge, or outside the
// array, feeds no cell whose value is still needed once it has been
// recomputed from incomplete neighbours (the exact part of the region
// shrinks by one cell per half-step, and the halo is as wide as the pass),
// and the weights sum to at most 1, so such values stay finite.  A region
// with no boundary cell therefore updates every cell with no mask at all.

// ---------------------------------------------------------------- jacobi_1d
// One wave per workgroup; lane l holds the K consecutive points starting at
// region offset l*K.  The region is 64*K points, the first hh and last hh of
// which are the halo; the rest (inner) is this workgroup's tile.  Loads and
// stores go through LDS so that every global access instruction covers 64
// consecutive elements (the run layout is transposed in LDS, with one pad
// element per run so the lanes' runs fall in different banks).
template <int K>
__global__ void __launch_bounds__(64) j1_kernel(J1Args a) {
    constexpr int R = 64 * K;
    __shared__ double stage[64 * (K + 1)];
    const int lane = threadIdx.x;
    const int64_t n = a.n;
    const int64_t rbase = (int64_t)blockIdx.x * a.inner - a.hh;  // global index of region cell 0
    const int64_t g0 = rbase + (int64_t)lane * K;
    auto pos = [](int i) { return i + i / K; };

    double va[K], vb[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int i = m * 64 + lane;
        const int64_t g = rbase + i;
        stage[pos(i)] = (g >= 0 && g < n) ? a.ain[g] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) va[k] = stage[lane * (K + 1) + k];
    if (a.phase) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int i = m * 64 + lane;
            const int64_t g = rbase + i;
            stage[pos(i)] = (g >= 0 && g < n) ? a.bin[g] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) vb[k] = stage[lane * (K + 1) + k];
    } else {
        // B's interior is written before it is read; only its ends matter
#pragma unroll
        for (int k = 0; k < K; ++k) vb[k] = 0.0;
        if (rbase <= 0 || rbase + R >= n) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t g = g0 + k;
                if (g == 0 || g == n - 1) vb[k] = a.bfix[g];
            }
        }
    }
    // the ends of the array, 0 and n-1, fall in this region only for the
    // first and last workgroups
    const bool edge = rbase <= 0 || rbase + R - 1 >= n - 1;
    auto half = [&](double(&d)[K], const double(&s)[K], auto masked) __attribute__((always_inline)) {
        const double left = from_lower(s[K - 1]);
        const double right = from_upper(s[0]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double l = k == 0 ? left : s[k > 0 ? k - 1 : 0];
            const double r = k == K - 1 ? right : s[k < K - 1 ? k + 1 : k];
            const double nv = kW1 * ((l + s[k]) + r);
            if constexpr (decltype(masked)::value) {
                const int64_t g = g0 + k;
                d[k] = j_keep(__builtin_amdgcn_ballot_w64(g == 0 || g == n - 1), nv, d[k]);
            } else {
                d[k] = nv;
            }
        }
    };
    auto steps = [&](auto masked) __attribute__((always_inline)) {
        int s = 0;
        if (a.phase && a.nhalf > 0) {
            half(va, vb, masked);
            s = 1;
        }
        for (; s + 2 <= a.nhalf; s += 2) {
            half(vb, va, masked);
            half(va, vb, masked);
        }
        if (s < a.nhalf) half(vb, va, masked);
    };
    if (edge) steps(std::true_type{});
    else steps(std::false_type{});

    // write the tile: A, then (if it is needed) B, each through the LDS
    // transpose
    const int nout = a.write_b ? 2 : 1;
    for (int pass = 0; pass < nout; ++pass) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) stage[lane * (K + 1) + k] = pass == 0 ? va[k] : vb[k];
        __syncthreads();
        double *out = pass == 0 ? a.aout : a.bout;
        const int64_t lo = pass == 1 && a.write_b == 2 ? 1 : 0, hi = pass == 1 && a.write_b == 2 ? n - 1 : n;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int i = m * 64 + lane;
            const int64_t g = rbase + i;
            if (i >= a.hh && i < R - a.hh && g >= lo && g < hi) out[g] = stage[pos(i)];
        }
    }
}

// ---------------------------------------------------------------- jacobi_2d
// W waves per workgroup; wave w owns region rows [w*RPL, (w+1)*RPL) and lane
// l the columns 2l and 2l+1, so the region is (W*RPL) x 128 cells.  West and
// east neighbours across lanes come from DPP shifts, the rows above and below
// a wave's band from the neighbouring waves through LDS (two slots, so one
// barrier per half-step suffices).
// MASK = false: every cell is updated; only for tiles whose region holds no
// boundary cell of the array.  MASK = true: boundary cells keep their values;
// any tile.  (One kernel with both paths needs more registers than either.)
template <int W, int RPL, int MINW, bool MASK>
__global__ void __launch_bounds__(64 * W, MINW) j2_kernel(J2Args a) {
    constexpr int VEC = 2;
    constexpr int R = W * RPL, C = 64 * VEC;
    __shared__ double xch[2][W][2][C];
    // the wave index is uniform over a wave: say so, so that everything that
    // depends only on the row (bounds, masks, row addresses) stays scalar
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int tr, tc;
    j2_tile(a, j_xcd_remap(blockIdx.x, gridDim.x), tr, tc);
    const int64_t n0 = a.n0;
    const int n1 = (int)a.n1;  // < 2^30, checked by the host
    const int ri0 = wave * RPL;
    const int64_t gr = (int64_t)tr * a.inner_r - a.hh + ri0;  // global row of r = 0
    const int gc = tc * a.inner_c - a.hh + lane * VEC;         // global column of v = 0

    uint32_t rowin = 0, rowfix = 0;  // bit r: row in the array / a boundary row of the array
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int64_t i = gr + r;
        if (i >= 0 && i < n0) rowin |= 1u << r;
        if (i == 0 || i == n0 - 1) rowfix |= 1u << r;
    }
    unsigned colin = 0;
    uint64_t colfix[VEC];  // lanes whose column v is a boundary column of the array
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const int j = gc + v;
        if (j >= 0 && j < n1) colin |= 1u << v;
        colfix[v] = __builtin_amdgcn_ballot_w64(j == 0 || j == n1 - 1);
    }
    double va[RPL][VEC], vb[RPL][VEC];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int64_t i = gr + r;
        const double *rowa = a.ain + i * n1;
        const double *rowb = (a.phase ? a.bin : a.bfix) + i * n1;
        const bool rfix = (rowfix >> r) & 1u;
        if (a.vec16) {
            // both columns are in the array or neither (gc even, n1 even)
            const bool in = ((rowin >> r) & 1u) && (colin & 1u);
            const double2 x = in ? *reinterpret_cast<const double2 *>(rowa + (unsigned)gc) : double2{0.0, 0.0};
            va[r][0] = x.x;
            va[r][1] = x.y;
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const bool in = ((rowin >> r) & 1u) && ((colin >> v) & 1u);
            const unsigned j = (unsigned)(gc + v);
            const bool fixed = rfix || j == 0 || j == (unsigned)(n1 - 1);
            if (!a.vec16) va[r][v] = in ? rowa[j] : 0.0;
            vb[r][v] = (in && (a.phase || fixed)) ? rowb[j] : 0.0;
        }
    }

    // Edge tiles: the values a half-step must keep.  Boundary rows are kept
    // whole (skipped, a uniform branch); on other rows a lane holds at most
    // one boundary-column cell (the array's first or last column, n1 >= 3
    // when anything is updated), whose A and B values never change, so they
    // are captured once here instead of keeping every old value alive.
    double fixa[RPL], fixb[RPL];
    if constexpr (MASK) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const bool v1 = (colfix[1] >> lane) & 1ull;
            fixa[r] = v1 ? va[r][1] : va[r][0];
            fixb[r] = v1 ? vb[r][1] : vb[r][0];
        }
    }

    int slot = 0;
    auto half = [&](double(&d)[RPL][VEC], const double(&s)[RPL][VEC], const double(&fix)[RPL],
                    auto masked) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            xch[slot][wave][0][lane * VEC + v] = s[0][v];
            xch[slot][wave][1][lane * VEC + v] = s[RPL - 1][v];
        }
        __syncthreads();
        const int wu = wave > 0 ? wave - 1 : 0, wd = wave < W - 1 ? wave + 1 : wave;
        double up0[VEC], dn0[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            // the first and last waves read a slot of their own; the values
            // only feed the region's edge rows
            up0[v] = xch[slot][wu][1][lane * VEC + v];
            dn0[v] = xch[slot][wd][0][lane * VEC + v];
        }
        slot ^= 1;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double wl = from_lower(s[r][VEC - 1]);
            const double er = from_upper(s[r][0]);
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const double c = s[r][v];
                const double w = v == 0 ? wl : s[r][v > 0 ? v - 1 : 0];
                const double e = v == VEC - 1 ? er : s[r][v < VEC - 1 ? v + 1 : v];
                const double so = r == RPL - 1 ? dn0[v] : s[r < RPL - 1 ? r + 1 : r][v];
                const double no = r == 0 ? up0[v] : s[r > 0 ? r - 1 : 0][v];
                const double nv = kW2 * ((((c + w) + e) + so) + no);
                if constexpr (decltype(masked)::value) {
                    // a boundary row keeps all its cells (uniform branch), other
                    // rows keep the lanes on a boundary column
                    if (!((rowfix >> r) & 1u)) d[r][v] = j_keep(colfix[v], nv, fix[r]);
                } else {
                    d[r][v] = nv;
                }
            }
        }
    };
    auto steps = [&](auto masked) __attribute__((always_inline)) {
        int s = 0;
        if (a.phase && a.nhalf > 0) {
            half(va, vb, fixa, masked);
            s = 1;
        }
        for (; s + 2 <= a.nhalf; s += 2) {
            half(vb, va, fixb, masked);
            half(va, vb, fixa, masked);
        }
        if (s < a.nhalf) half(vb, va, fixb, masked);
    };
    steps(std::integral_constant<bool, MASK>{});

#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int ri = ri0 + r;
        if (ri < a.hh || ri >= R - a.hh || !((rowin >> r) & 1u)) continue;
        const int64_t i = gr + r;
        double *rowa = a.aout + i * n1;
        double *rowb = a.bout + i * n1;
        const bool binterior_row = i >= 1 && i <= n0 - 2;
        // with vec16 both columns are inside the tile or neither (hh even)
        if (a.vec16 && lane * VEC >= a.hh && lane * VEC < C - a.hh && (colin & 1u)) {
            *reinterpret_cast<double2 *>(rowa + (unsigned)gc) = double2{va[r][0], va[r][1]};
            if (a.write_b == 1) *reinterpret_cast<double2 *>(rowb + (unsigned)gc) = double2{vb[r][0], vb[r][1]};
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int ci = lane * VEC + v;
            if (ci < a.hh || ci >= C - a.hh || !((colin >> v) & 1u)) continue;
            const unsigned j = (unsigned)(gc + v);
            if (!a.vec16) rowa[j] = va[r][v];
            if ((a.write_b == 1 && !a.vec16) ||
                (a.write_b == 2 && binterior_row && j >= 1 && j <= (unsigned)(n1 - 2)))
                rowb[j] = vb[r][v];
        }
    }
}

// ------------------------------------------- jacobi_2d, marching down rows
// The form for large arrays.  A workgroup is one wave and owns a strip of
// 64*CPL columns (CPL per lane; the first and last hh are halo, recomputed)
// and a segment of rows, and marches down the rows applying NH half-steps in
// one pass: at step q, level s (the arrays after s half-steps; odd levels are
// B, even levels A) is computed for row q - s + 1, from level s - 1 of rows
// q - s .. q - s + 2, the last of which level s - 1 has just computed.  For
// every level each lane keeps three rows of its columns in registers, so the
// rows above and below come from the lane itself and the columns left and
// right from the adjacent lanes (DPP): no LDS exchange and no barrier.  Row x
// of every level lives in register slot x mod 3; the loop is unrolled three
// times, so the slots are fixed at compile time and no register is copied as
// the march advances.  Compared with the region tiles above, only the columns
// carry a halo, and the rows before a segment are recomputed once (NH - 1
// rows per level).
// Loads of level 0 are issued D rows ahead of use.  They read clamped rows
// and columns, so they need no guard: a value read for a row or column
// outside the array only ever feeds a boundary cell of the array, which is
// replaced by its fixed value (a select, so whatever was computed there is
// dropped), or another cell outside the array.  The array's boundary cells
// keep their values at every level: the two boundary rows (both arrays) are
// kept in LDS when the march reads them, and so are the boundary column's
// values (both arrays) of the rows in flight, in a small ring.  Requires n1
// even, hh even and 16-byte aligned arrays.
typedef double j2m_v2 __attribute__((ext_vector_type(2)));

struct J2MArgs {
    const double *ain, *bfix;  // level 0 (A); B's values (its boundary cells never change)
    double *aout, *bout;
    int64_t n0, n1;
    int hh, strips, seg_rows, write_b;
};

template <int NH, int CPL, int D>
__global__ void __launch_bounds__(64) j2m_kernel(J2MArgs a) {
    static_assert(CPL == 2 || CPL == 4, "two or four columns per lane");
    static_assert(D == 1 || D == 3, "the prefetch ring must divide the unroll");
    constexpr int C = 64 * CPL, NP = CPL / 2, RING = NH + 4;
    __shared__ double fixrow[2][2][C];     // [row 0 / row n0-1][A / B][column]
    __shared__ double fixcol[RING][2][2];  // [ring slot][column 0 / n1-1][A / B]
    const int lane = threadIdx.x;
    const int b = j_xcd_remap(blockIdx.x, gridDim.x);
    const int strip = b % a.strips, seg = b / a.strips;  // strips fastest: neighbours share halos in L2
    const int n0 = (int)a.n0;  // < 2^30, checked by the host (so are the row indices below)
    const int n1 = (int)a.n1;
    const int ci = CPL * lane;  // column offset in the strip
    const int gc = strip * (C - 2 * a.hh) - a.hh + ci;  // column of this lane's first value (even)
    // pair p (columns gc+2p, gc+2p+1): in the array both or neither; its load
    // column, clamped into the array; whether this strip stores it
    int colp[NP];
    bool inp[NP], ownp[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int c = gc + 2 * p;
        colp[p] = min(max(c, 0), n1 - 2);
        inp[p] = c >= 0 && c < n1;
        ownp[p] = inp[p] && ci + 2 * p >= a.hh && ci + 2 * p < C - a.hh;
    }
    // boundary columns: column 0 is this lane's value -gc (even) and column
    // n1 - 1 its value n1 - 1 - gc (odd) when that lies in the lane
    const int k0 = -gc;
    const bool bc0 = k0 >= 0 && k0 < CPL;
    const int k1 = n1 - 1 - gc;
    const bool bc1 = k1 >= 1 && k1 < CPL;
    uint64_t keep[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) keep[k] = __builtin_amdgcn_ballot_w64(gc + k == 0 || gc + k == n1 - 1);
    const bool edge = __builtin_amdgcn_ballot_w64(bc0 || bc1) != 0;  // uniform over the wave
    const int R0 = seg * a.seg_rows;
    const int R1 = min(n0, R0 + a.seg_rows);
    const bool rowedge = R0 - NH <= 0 || R1 + NH > n0 - 1;  // rows in flight include a boundary row
    if (R0 >= R1) return;  // a segment past the last row (no barrier below)

    auto row_of = [&](const double *base, int r) {  // uniform row start, the row clamped into the array
        return base + (int64_t)min(max(r, 0), n0 - 1) * n1;
    };
    auto load_row = [&](int r, double (&x)[CPL]) {
        const double *rp = row_of(a.ain, r);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const j2m_v2 v = *reinterpret_cast<const j2m_v2 *>(rp + colp[p]);
            x[2 * p] = v.x;
            x[2 * p + 1] = v.y;
        }
    };
    // record the fixed values of row r (x: its level-0 values; fb0, fb1: B
    // at columns 0 and n1 - 1) in ring slot rs
    auto keep_fixed = [&](int r, int rs, const double (&x)[CPL], double fb0, double fb1) {
        if (edge) {  // uniform
            if (bc0) {
                double v = x[0];
#pragma unroll
                for (int k = 2; k < CPL; k += 2)
                    if (k0 == k) v = x[k];
                fixcol[rs][0][0] = v;
                fixcol[rs][0][1] = fb0;
            }
            if (bc1) {
                double v = x[1];
#pragma unroll
                for (int k = 3; k < CPL; k += 2)
                    if (k1 == k) v = x[k];
                fixcol[rs][1][0] = v;
                fixcol[rs][1][1] = fb1;
            }
        }
        if (rowedge && (r == 0 || r == n0 - 1)) {  // uniform
            const int w = r == 0 ? 0 : 1;
            const double *bp = row_of(a.bfix, r);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const j2m_v2 v = *reinterpret_cast<const j2m_v2 *>(bp + colp[p]);
                fixrow[w][1][ci + 2 * p] = v.x;
                fixrow[w][1][ci + 2 * p + 1] = v.y;
            }
#pragma unroll
            for (int k = 0; k < CPL; ++k) fixrow[w][0][ci + k] = x[k];
        }
    };
    auto wrap = [](int x) { return x >= RING ? x - RING : (x < 0 ? x + RING : x); };

    double S[NH][3][CPL];  // [level][row slot: row mod 3, counted from q0][column]
    double P[D][CPL];      // level-0 rows in flight
    double PB[D][2];       // B at their boundary columns (edge waves)
    const int q0 = R0 - NH + 1, qlast = R1 + NH - 2;
    // level 0: rows q0 - 1 and q0 now, rows q0 + 1 .. q0 + D in flight
    load_row(q0 - 1, S[0][2]);
    load_row(q0, S[0][0]);
    auto load_bfix = [&](int r, double (&fb)[2]) {
        if (edge) {  // uniform
            const double *bp = row_of(a.bfix, r);
            fb[0] = bp[0];
            fb[1] = bp[n1 - 1];
        }
    };
    {
        double fb[2][2] = {};
        load_bfix(q0 - 1, fb[0]);
        load_bfix(q0, fb[1]);
        keep_fixed(q0 - 1, 0, S[0][2], fb[0][0], fb[0][1]);
        keep_fixed(q0, 1, S[0][0], fb[1][0], fb[1][1]);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        load_row(q0 + 1 + d, P[(1 + d) % D]);
        PB[(1 + d) % D][0] = PB[(1 + d) % D][1] = 0.0;
        load_bfix(q0 + 1 + d, PB[(1 + d) % D]);
    }
    int rn = 2;  // ring slot of row q + 1 at step q

    // Step q at phase PH = (q - q0) mod 3.  GENERAL: levels still starting,
    // boundary rows or columns in the wave, rows outside the segment; the
    // plain form drops all of those checks (scalar work that would otherwise
    // take issue slots from the update itself).
    auto step = [&](int q, auto PH, auto GENERAL) {
        constexpr int ph = decltype(PH)::value;
        constexpr bool general = decltype(GENERAL)::value;
        // level 0 takes row q + 1; row q + 1 + D is fetched into its place
        double(&l0)[CPL] = S[0][(ph + 1) % 3];
        double(&pf)[CPL] = P[(ph + 1) % D];
#pragma unroll
        for (int k = 0; k < CPL; ++k) l0[k] = pf[k];
        if (general) keep_fixed(q + 1, rn, l0, PB[(ph + 1) % D][0], PB[(ph + 1) % D][1]);
        load_row(q + 1 + D, pf);
        if (general) load_bfix(q + 1 + D, PB[(ph + 1) % D]);
#pragma unroll
        for (int s = 1; s <= NH; ++s) {
            if (general && q < R0 - NH + 2 * s - 1) break;  // uniform: later levels start later still
            const int r = q - s + 1;
            // level s - 1 rows r - 1, r, r + 1 and the slot of row r
            const int lo = ((ph - s) % 3 + 3) % 3, mid = ((ph - s + 1) % 3 + 3) % 3,
                      hi = ((ph - s + 2) % 3 + 3) % 3;
            const double(&in0)[CPL] = S[s - 1][lo];
            const double(&in1)[CPL] = S[s - 1][mid];
            const double(&in2)[CPL] = S[s - 1][hi];
            const double wl = from_lower(in1[CPL - 1]);
            const double er = from_upper(in1[0]);
            double nv[CPL];
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                const double w = k ? in1[k - 1] : wl;
                const double e = k < CPL - 1 ? in1[k + 1] : er;
                nv[k] = kW2 * ((((in1[k] + w) + e) + in2[k]) + in0[k]);
            }
            const int arr = s & 1;  // 1: B
            if (general) {
                if (rowedge && (r == 0 || r == n0 - 1)) {  // uniform: a boundary row keeps its values
                    const int w = r == 0 ? 0 : 1;
#pragma unroll
                    for (int k = 0; k < CPL; ++k) nv[k] = fixrow[w][arr][ci + k];
                } else if (edge) {  // uniform: the boundary columns keep their values
                    // (column 0 sits at an even place of a lane, column n1 - 1 at an odd one)
                    const int rs = wrap(rn - s);
                    const double f0 = fixcol[rs][0][arr], f1 = fixcol[rs][1][arr];
#pragma unroll
                    for (int k = 0; k < CPL; ++k) nv[k] = j_keep(keep[k], nv[k], (k & 1) ? f1 : f0);
                }
            }
            if (s < NH) {
#pragma unroll
                for (int k = 0; k < CPL; ++k) S[s][mid][k] = nv[k];
            }
            // A's row r is in the segment on the plain path; B's row (the
            // level before) is stored by the last pass only.  With two
            // columns per lane a store covers whole lines and goes out with
            // the streaming hint; with four, the lane's two stores fill each
            // line in halves, which L2 merges when the stores are ordinary
            // (streamed halves reach HBM as separate partial writes: 1.23x
            // the written bytes, measured)
            if (s == NH && (!general || (r >= R0 && r < R1))) {
                const int64_t ro = (int64_t)r * n1 + gc;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (!ownp[p]) continue;
                    j2m_v2 *dst = reinterpret_cast<j2m_v2 *>(a.aout + ro + 2 * p);
                    if constexpr (CPL == 2) __builtin_nontemporal_store(j2m_v2{nv[2 * p], nv[2 * p + 1]}, dst);
                    else *dst = j2m_v2{nv[2 * p], nv[2 * p + 1]};
                }
            }
            if (s == NH - 1 && a.write_b != 0 && r >= R0 && r < R1) {
                const int64_t ro = (int64_t)r * n1 + gc;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (!ownp[p]) continue;
                    const int64_t o = ro + 2 * p;
                    if (a.write_b == 1) {
                        __builtin_nontemporal_store(j2m_v2{nv[2 * p], nv[2 * p + 1]},
                                                    reinterpret_cast<j2m_v2 *>(a.bout + o));
                    } else if (r >= 1 && r <= n0 - 2) {  // B's interior only
                        if (gc + 2 * p >= 1) a.bout[o] = nv[2 * p];
                        if (gc + 2 * p + 1 <= n1 - 2) a.bout[o + 1] = nv[2 * p + 1];
                    }
                }
            }
        }
        if (general) rn = wrap(rn + 1);
    };
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    // The general steps: until every level has started (step q0 + 2 NH - 2,
    // rounded up to a whole group of three), or to the end for waves holding
    // a boundary row or column.  The plain steps carry on from there.  Loops
    // run whole groups and the last one or two steps follow them, so every
    // register keeps its place across the loop's back edge (a copy there
    // would wait for the rows still in flight).
    const int qg = (edge || rowedge) ? qlast + 1 : min(qlast + 1, q0 + (2 * NH - 2 + 2) / 3 * 3);
    int qb = q0;
    for (; qb < qg; qb += 3) {
        step(qb, P0{}, std::true_type{});
        if (qb + 1 < qg) step(qb + 1, P1{}, std::true_type{});
        if (qb + 2 < qg) step(qb + 2, P2{}, std::true_type{});
    }
    if (qg == qlast + 1) return;
    for (; qb + 3 <= qlast + 1; qb += 3) {
        step(qb, P0{}, std::false_type{});
        step(qb + 1, P1{}, std::false_type{});
        step(qb + 2, P2{}, std::false_type{});
    }
    if (qb <= qlast) {
        step(qb, P0{}, std::false_type{});
        if (qb + 1 <= qlast) step(qb + 1, P1{}, std::false_type{});
    }
}

// ------------------------------------------------------------- host side
constexpr int kJ2C = 128;  // region columns (2D)
constexpr int kJ1MaxTb = 256, kJ2MaxTb = 16;
constexpr size_t kJAlign = 256;

// Points per lane in 1D.  Runs of 16 cost the fewest cross-lane moves per
// point without spilling (runs of 32 measured slower); they are used when the
// array gives at least 2048 workgroups with them.  Smaller arrays take the
// shortest admissible run (tile at least half the region), spreading the
// work over more CUs.  DCP_J1_K forces a length (tuning runs only).
int j1_pick_k(int64_t n, int64_t hh) {
    auto admissible = [&](int k) { return 64 * k - 2 * hh >= 32 * k; };
    const char *forced = dcp::tuning_env("DCP_J1_K");
    if (forced && *forced) {
        const int k = std::atoi(forced);
        if ((k == 4 || k == 8 || k == 16 || k == 32) && 64 * k > 2 * hh) return k;
    }
    if (admissible(16) && (n + (64 * 16 - 2 * hh) - 1) / (64 * 16 - 2 * hh) >= 2048) return 16;
    for (int k : {4, 8, 16, 32})
        if (admissible(k)) return k;
    return 32;
}

// 2D workgroup shapes: (waves, rows per lane), all within the 128 VGPRs of
// four waves per SIMD without spilling (a kernel holding both the masked and
// the unmasked update spilled about 64 bytes per lane, which at 46800^2
// wrote about 15 GB per pass to HBM; hence one instantiation per path).
struct J2Cfg {
    int w, rpl;
};
constexpr J2Cfg kJ2Cfgs[] = {{16, 4}, {8, 8}, {16, 8}};

// Launch plan of a 2D pass: a shape and whether the pass is split into the
// ring of edge tiles (masked) and the interior rectangle (unmasked, two
// launches) or run as one masked launch.  Measured at T=1000: large arrays
// (46800^2: 1834 vs 1554 GLUP/s) gain from the split with 16 x 4; small ones
// (1300^2, a fifth of the tiles in the ring, launch-bound) run best as one
// launch of 8 x 8.  DCP_J2_CFG / DCP_J2_MODE (1 = one launch, 2 = split)
// force the choice (tuning runs only).
struct J2Plan {
    int cfg;
    bool split;
};

int64_t j2_interior_tiles(int64_t n0, int64_t n1, int64_t hh, int rows, int64_t *all) {
    const int64_t ir = rows - 2 * hh, ic = 128 - 2 * hh;
    const int64_t tr = (n0 + ir - 1) / ir, tc = (n1 + ic - 1) / ic;
    *all = tr * tc;
    auto span = [&](int64_t n, int64_t inner, int extent, int64_t tiles) {
        const int64_t lo = (hh + 1 + inner - 1) / inner;
        const int64_t num = n - 2 - (extent - 1) + hh;
        const int64_t hi = num < 0 ? -1 : std::min<int64_t>(num / inner, tiles - 1);
        return hi >= lo ? hi - lo + 1 : 0;
    };
    return span(n0, ir, rows, tr) * span(n1, ic, 128, tc);
}

// The row-marching form (j2m_kernel): used for arrays that give it enough
// waves with row segments of at least 8*NH rows, when n1 is even and the
// arrays are 16-byte aligned; passes of 4 to 16 half-steps (even) that start
// with B (whole time-loop iterations).  Four columns per lane (rows fetched
// one ahead) for passes of up to 8 half-steps, else two (rows fetched three
// ahead).  DCP_J2M_CPL = 2 or 4 picks the columns per lane (4 only up to 8
// half-steps), DCP_J2_MODE = 3 forces the form where it applies, 1 or 2 the
// region tiles (tuning runs only).
struct J2MPlan {
    bool use = false;
    int cpl = 2;
    int strips = 0, segs = 0, seg_rows = 0;
};

J2MPlan j2m_pick(int64_t n0, int64_t n1, int64_t hh) {
    J2MPlan m;
    m.cpl = hh <= 8 ? 4 : 2;
    const char *fc = dcp::tuning_env("DCP_J2M_CPL");
    if (fc && *fc) {
        const int c = std::atoi(fc);
        if (c == 2 || (c == 4 && hh <= 8)) m.cpl = c;
    }
    const int64_t C = 64 * m.cpl;
    if (n0 < 3 || n1 < 3 || n0 >= ((int64_t)1 << 30) || n1 % 2 != 0 || hh % 2 != 0 || hh < 4 || hh > 16)
        return m;
    const int64_t strips = (n1 + (C - 2 * hh) - 1) / (C - 2 * hh);
    const int64_t maxsegs = std::max<int64_t>(1, n0 / (8 * hh));
    const int64_t segs = std::max<int64_t>(1, std::min<int64_t>(maxsegs, (16384 + strips - 1) / strips));
    if (strips * segs > INT32_MAX / 2) return m;
    m.strips = (int)strips;
    m.segs = (int)segs;
    m.seg_rows = (int)((n0 + segs - 1) / segs);
    m.use = strips * segs >= 2048;
    const char *fm = dcp::tuning_env("DCP_J2_MODE");
    if (fm && *fm) m.use = std::atoi(fm) == 3;
    return m;
}

// Instantiations: two columns per lane with rows fetched three ahead for
// every pass depth, four columns per lane with rows fetched one ahead up to
// eight half-steps (deeper ones spill).
template <int NH>
void j2m_launch_nh(const J2MPlan &mp, dim3 grid, hipStream_t sm, const J2MArgs &m) {
    if constexpr (NH <= 8) {
        if (mp.cpl == 4) {
            hipLaunchKernelGGL((j2m_kernel<NH, 4, 1>), grid, dim3(64), 0, sm, m);
            return;
        }
    }
    hipLaunchKernelGGL((j2m_kernel<NH, 2, 3>), grid, dim3(64), 0, sm, m);
}

J2Plan j2_pick(int64_t n0, int64_t n1, int64_t hh) {
    J2Plan p{1, false};
    int64_t all = 0;
    const int64_t in = j2_interior_tiles(n0, n1, hh, kJ2Cfgs[0].w * kJ2Cfgs[0].rpl, &all);
    if (all >= 2048 && in * 10 >= all * 9) p = J2Plan{0, true};
    const char *fc = dcp::tuning_env("DCP_J2_CFG");
    if (fc && *fc) {
        const int c = std::atoi(fc);
        if (c >= 0 && c < 3 && kJ2Cfgs[c].w * kJ2Cfgs[c].rpl > 2 * hh) p.cfg = c;
    }
    const char *fm = dcp::tuning_env("DCP_J2_MODE");
    if (fm && *fm) p.split = std::atoi(fm) == 2;
    return p;
}

template <int K>
hipError_t j1_launch(int64_t blocks, const J1Args &a, hipStream_t sm) {
    hipLaunchKernelGGL(j1_kernel<K>, dim3((unsigned)blocks), dim3(64), 0, sm, a);
    return hipGetLastError();
}

size_t j_align(size_t x) { return (x + kJAlign - 1) / kJAlign * kJAlign; }

bool j_overlaps(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

struct JGeo {
    int dims = 1;
    int64_t n0 = 0, n1 = 1, count = 0;
    bool has_interior = false;
};

int j_geo(int dims, int64_t n0, int64_t n1, JGeo *g) {
    if (dims != 1 && dims != 2) return DCP_E_ARG;
    if (n0 < 0 || (dims == 2 && n1 < 0)) return DCP_E_SHAPE;
    const int64_t lim = ((int64_t)1 << 60) / 8;
    g->dims = dims;
    g->n0 = n0;
    g->n1 = dims == 2 ? n1 : 1;
    if (dims == 2 && n1 > 0 && n0 > lim / n1) return DCP_E_SHAPE;
    if (dims == 2 && n1 >= ((int64_t)1 << 30)) return DCP_E_SHAPE;
    if (n0 > lim) return DCP_E_SHAPE;
    g->count = n0 * g->n1;
    g->has_interior = dims == 1 ? n0 >= 3 : (n0 >= 3 && n1 >= 3);
    return DCP_OK;
}

// Half-steps per pass.  The defaults are the measured best on MI355X: in 1D
// 64 for small arrays (the pass count is launch-bound) and 128 for large
// ones; in 2D 8 where the row-marching form applies, else 12 (10-14
// measured within a few percent with the region tiles at 1300^2).
int j_tblock(const JGeo &g, int32_t tblock, int *hp) {
    const int mx = g.dims == 1 ? kJ1MaxTb : kJ2MaxTb;
    if (tblock < 0 || tblock > mx) return DCP_E_ARG;
    if (tblock > 0) *hp = tblock;
    else if (g.dims == 1) *hp = g.count >= ((int64_t)1 << 22) ? 128 : 64;
    else *hp = j2m_pick(g.n0, g.n1, 8).use ? 8 : 12;
    return DCP_OK;
}

// The pass schedule.  Passes alternate between the caller's arrays and the
// workspace copies, and their number is even so the result ends in the
// caller's arrays.  When every pass can hold a whole number of time-loop
// iterations (an even number of half-steps), every pass starts by writing B
// from A, so B's interior is never read across a pass boundary: only the last
// pass stores B, and B's boundary is always read from the caller's B (it
// never changes).  Otherwise (one half-step per pass, or a single iteration)
// passes split at half-steps and store both arrays.
struct JPlan {
    int64_t halves = 0, passes = 0, per = 0, rem = 0, hh = 0;
    bool whole = false;  // pass sizes counted in iterations (2 half-steps each)
    int64_t size(int64_t i) const {
        const int64_t s = per + (i < rem ? 1 : 0);
        return whole ? 2 * s : s;
    }
};

JPlan j_plan(const JGeo &g, int32_t tsteps, int hp) {
    JPlan p;
    if (tsteps <= 1 || !g.has_interior) return p;
    const int64_t iters = (int64_t)tsteps - 1;
    p.halves = 2 * iters;
    if (hp >= 2) {
        int64_t P = (iters + hp / 2 - 1) / (hp / 2);
        if (P & 1) ++P;
        if (P <= iters) {
            p.whole = true;
            p.passes = P;
            p.per = iters / P;
            p.rem = iters % P;
            p.hh = 2 * (p.per + (p.rem ? 1 : 0));
            return p;
        }
    }
    int64_t P = (p.halves + hp - 1) / hp;
    if (P & 1) ++P;
    p.passes = P;
    p.per = p.halves / P;
    p.rem = p.halves % P;
    p.hh = p.per + (p.rem ? 1 : 0);
    return p;
}

size_t j_ws_need(const JGeo &g, const JPlan &p) {
    return p.passes ? 2 * j_align((size_t)g.count * sizeof(double)) : 0;
}

int j_check_buffers(const JGeo &g, const double *A, const double *B, const void *ws, size_t ws_bytes,
                    size_t need) {
    const size_t bytes = (size_t)g.count * sizeof(double);
    if (g.count > 0 && (!A || !B)) return DCP_E_NULL;
    if (j_overlaps(A, bytes, B, bytes)) return DCP_E_ALIAS;
    if (need) {
        if (ws_bytes < need) return DCP_E_WORKSPACE;
        if (!ws) return DCP_E_NULL;
        if (j_overlaps(ws, need, A, bytes) || j_overlaps(ws, need, B, bytes)) return DCP_E_ALIAS;
    }
    return DCP_OK;
}

template <typename Launch>
int j_run_passes(const JGeo &g, const JPlan &p, double *A, double *B, void *ws, Launch launch) {
    const size_t fb = j_align((size_t)g.count * sizeof(double));
    double *WA = reinterpret_cast<double *>(static_cast<char *>(ws));
    double *WB = reinterpret_cast<double *>(static_cast<char *>(ws) + fb);
    int64_t done = 0;
    for (int64_t i = 0; i < p.passes; ++i) {
        const int nh = (int)p.size(i);
        const bool even = (i & 1) == 0;
        const double *ain = even ? A : WA;
        const double *bin = even ? B : WB;
        double *aout = even ? WA : A;
        double *bout = even ? WB : B;
        const bool last = i == p.passes - 1;
        const int write_b = p.whole ? (last ? 2 : 0) : 1;
        const double *bfix = p.whole ? B : bin;
        if (launch(ain, bin, bfix, aout, bout, nh, (int)(done & 1), write_b) != hipSuccess) return DCP_E_HIP;
        done += nh;
    }
    return DCP_OK;
}

}  // namespace

extern "C" {

int dcp_jacobi_workspace_bytes(int dims, int64_t n0, int64_t n1, int32_t tsteps, int32_t tblock,
                               size_t *bytes) {
    if (!bytes) return DCP_E_NULL;
    JGeo g;
    int st = j_geo(dims, n0, n1, &g);
    if (st != DCP_OK) return st;
    int hp = 0;
    st = j_tblock(g, tblock, &hp);
    if (st != DCP_OK) return st;
    *bytes = j_ws_need(g, j_plan(g, tsteps, hp));
    return DCP_OK;
}

int dcp_jacobi_plan(int dims, int64_t n0, int64_t n1, int32_t tsteps, int32_t tblock, int64_t *passes,
                    int32_t *halo) {
    if (!passes || !halo) return DCP_E_NULL;
    JGeo g;
    int st = j_geo(dims, n0, n1, &g);
    if (st != DCP_OK) return st;
    int hp = 0;
    st = j_tblock(g, tblock, &hp);
    if (st != DCP_OK) return st;
    const JPlan p = j_plan(g, tsteps, hp);
    *passes = p.passes;
    *halo = (int32_t)p.hh;
    return DCP_OK;
}

int dcp_jacobi_1d(int32_t tsteps, double *A, double *B, int64_t n, int32_t tblock, void *ws, size_t ws_bytes,
                  void *stream) {
    JGeo g;
    int st = j_geo(1, n, 1, &g);
    if (st != DCP_OK) return st;
    int hp = 0;
    st = j_tblock(g, tblock, &hp);
    if (st != DCP_OK) return st;
    const JPlan p = j_plan(g, tsteps, hp);
    st = j_check_buffers(g, A, B, ws, ws_bytes, j_ws_need(g, p));
    if (st != DCP_OK || p.passes == 0) return st;
    const int K = j1_pick_k(n, p.hh);
    const int64_t inner = 64 * K - 2 * p.hh;
    const int64_t blocks = (n + inner - 1) / inner;
    if (blocks > INT32_MAX) return DCP_E_SHAPE;
    hipStream_t sm = static_cast<hipStream_t>(stream);
    return j_run_passes(g, p, A, B, ws,
                        [&](const double *ain, const double *bin, const double *bfix, double *aout, double *bout,
                            int nh, int ph, int wb) {
                            const J1Args a{ain, bin, bfix, aout, bout, n, inner, (int)p.hh, nh, ph, wb};
                            switch (K) {
                                case 4: return j1_launch<4>(blocks, a, sm);
                                case 8: return j1_launch<8>(blocks, a, sm);
                                case 16: return j1_launch<16>(blocks, a, sm);
                                default: return j1_launch<32>(blocks, a, sm);
                            }
                        });
}

int dcp_jacobi_2d(int32_t tsteps, double *A, double *B, int64_t n0, int64_t n1, int32_t tblock, void *ws,
                  size_t ws_bytes, void *stream) {
    JGeo g;
    int st = j_geo(2, n0, n1, &g);
    if (st != DCP_OK) return st;
    int hp = 0;
    st = j_tblock(g, tblock, &hp);
    if (st != DCP_OK) return st;
    const JPlan p = j_plan(g, tsteps, hp);
    st = j_check_buffers(g, A, B, ws, ws_bytes, j_ws_need(g, p));
    if (st != DCP_OK || p.passes == 0) return st;
    const J2Plan plan = j2_pick(n0, n1, p.hh);
    const int cfg = plan.cfg;
    const int rows = kJ2Cfgs[cfg].w * kJ2Cfgs[cfg].rpl;
    const int inner_r = rows - 2 * (int)p.hh, inner_c = kJ2C - 2 * (int)p.hh;
    const int64_t tiles_r = (n0 + inner_r - 1) / inner_r, tiles_c = (n1 + inner_c - 1) / inner_c;
    if (tiles_c > INT32_MAX || tiles_r > INT32_MAX / tiles_c) return DCP_E_SHAPE;
    // interior rectangle: tiles whose region [t*inner - hh, t*inner - hh + extent)
    // lies in [1, n - 2] on both axes
    auto lo_hi = [&](int64_t n, int inner, int extent, int64_t tiles, int &lo, int &hi) {
        lo = (int)((p.hh + 1 + inner - 1) / inner);
        const int64_t num = n - 2 - (extent - 1) + p.hh;
        hi = num < 0 ? -1 : (int)std::min<int64_t>(num / inner, tiles - 1);
    };
    int r_lo, r_hi, c_lo, c_hi;
    lo_hi(n0, inner_r, rows, tiles_r, r_lo, r_hi);
    lo_hi(n1, inner_c, kJ2C, tiles_c, c_lo, c_hi);
    if (r_lo > r_hi || c_lo > c_hi) {  // no interior tile: everything is ring
        r_lo = (int)tiles_r;
        r_hi = (int)tiles_r - 1;
        c_lo = 0;
        c_hi = -1;
    }
    const int64_t n_in = (int64_t)(r_hi - r_lo + 1) * (c_hi >= c_lo ? c_hi - c_lo + 1 : 0);
    const int64_t n_all = tiles_r * tiles_c, n_ring = n_all - n_in;
    // one masked launch over all tiles, or the ring (masked) and the interior
    // rectangle (unmasked) as two launches
    const bool split = plan.split && n_in > 0;
    hipStream_t sm = static_cast<hipStream_t>(stream);
    auto launch_set = [&](J2Args a, int set, int64_t blocks, bool mask) -> hipError_t {
        a.set = set;
        const dim3 grid((unsigned)blocks);
        if (cfg == 1) {
            if (mask) hipLaunchKernelGGL((j2_kernel<8, 8, 4, true>), grid, dim3(512), 0, sm, a);
            else hipLaunchKernelGGL((j2_kernel<8, 8, 4, false>), grid, dim3(512), 0, sm, a);
        } else if (cfg == 2) {
            if (mask) hipLaunchKernelGGL((j2_kernel<16, 8, 4, true>), grid, dim3(1024), 0, sm, a);
            else hipLaunchKernelGGL((j2_kernel<16, 8, 4, false>), grid, dim3(1024), 0, sm, a);
        } else {
            if (mask) hipLaunchKernelGGL((j2_kernel<16, 4, 4, true>), grid, dim3(1024), 0, sm, a);
            else hipLaunchKernelGGL((j2_kernel<16, 4, 4, false>), grid, dim3(1024), 0, sm, a);
        }
        return hipGetLastError();
    };
    const J2MPlan mp = j2m_pick(n0, n1, p.hh);
    auto launch_march = [&](const J2MArgs &m, int nh) -> hipError_t {
        const dim3 grid((unsigned)((int64_t)mp.strips * mp.segs));
        switch (nh) {
            case 4: j2m_launch_nh<4>(mp, grid, sm, m); break;
            case 6: j2m_launch_nh<6>(mp, grid, sm, m); break;
            case 8: j2m_launch_nh<8>(mp, grid, sm, m); break;
            case 10: j2m_launch_nh<10>(mp, grid, sm, m); break;
            case 12: j2m_launch_nh<12>(mp, grid, sm, m); break;
            case 14: j2m_launch_nh<14>(mp, grid, sm, m); break;
            default: j2m_launch_nh<16>(mp, grid, sm, m); break;
        }
        return hipGetLastError();
    };
    return j_run_passes(g, p, A, B, ws,
                        [&](const double *ain, const double *bin, const double *bfix, double *aout, double *bout,
                            int nh, int ph, int wb) {
                            const bool v16 = (n1 % 2 == 0) && (p.hh % 2 == 0) &&
                                             ((uintptr_t)ain | (uintptr_t)bin | (uintptr_t)bfix |
                                              (uintptr_t)aout | (uintptr_t)bout) % 16 == 0;
                            // whole iterations (B first, B's interior not read):
                            // the row-marching form
                            if (mp.use && v16 && p.whole && ph == 0 && nh >= 4 && nh <= 16 && nh % 2 == 0) {
                                const J2MArgs m{ain, bfix, aout, bout, n0, n1, (int)p.hh, mp.strips, mp.seg_rows,
                                                wb};
                                return launch_march(m, nh);
                            }
                            const J2Args a{ain, bin, bfix, aout, bout, n0, n1, inner_r, inner_c,
                                           (int)tiles_r, (int)tiles_c, (int)p.hh, nh, ph, wb, v16 ? 1 : 0,
                                           0, r_lo, r_hi, c_lo, c_hi};
                            if (!split) return launch_set(a, 0, n_all, true);
                            if (n_ring > 0) {
                                const hipError_t e = launch_set(a, 2, n_ring, true);
                                if (e != hipSuccess) return e;
                            }
                            return launch_set(a, 1, n_in, false);
                        });
}

}  // extern "C"
