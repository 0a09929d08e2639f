// dcp_tbk.hip -- B fused time steps per pass over memory (temporal blocking,
// B = 2 or 3) for the forward reaction-diffusion step on gfx950, on tiles of
// full x-rows or of x-segments.
//
// A pass reads u_t and f once and writes u_{t+B}: 3 fields moved per B steps.
// The paper's fusion (Sec. 3.1) merges the maps of one step; this fuses B
// consecutive steps of the time loop, which is legal because level s (the
// state after s of the B steps) at a point reads level s-1 only within
// distance 1, so level s is recomputed on a halo of B-s points around the
// tile.
//
// Layout of the work:
//   * a workgroup owns a tile of ty rows x one x-range x zc planes; the
//     x-range is either the whole row (no x-halo; the periodic x-wrap stays
//     inside the tile) or a segment of wc 16-byte chunks with `halo` chunks
//     on each side (at least B points), so rows of any length keep B steps
//     per pass;
//   * one workgroup per CU (256 in all, numbered so an XCD holds a
//     contiguous block of slabs across all segments): the tiles of a z-run
//     are resident together and march up z side by side, so their halo rows
//     and chunks are read while the neighbour reads them and are served by
//     the XCD's L2;
//   * each lane owns up to KM chunks of the level-0 frame (ty + 2B rows x the
//     tile's chunks); level 0 (u_t) of the current plane sits in LDS, levels
//     1..B-1 of their two most recent planes sit in LDS (double buffers),
//     the z-neighbours of every level and the next input plane are each
//     lane's registers (register queues);
//   * at iteration q, stage s computes level s at plane q-s+1 (a B-stage
//     z-pipeline), two barriers per plane.
// The ring form (tbr_kernel, 768 lanes, the planner's first choice) keeps
// all z-neighbours in registers and needs one barrier per plane; the form
// above serves the tiles that only fit 1024 or 512 lanes.
// Every point is computed with the same operations, in the same order, as
// the one-step kernel, so a pass equals B one-step launches bit for bit.
// The norms of all B steps are reduced over the owned points only.
#include "dcp_internal.h"

namespace dcp {
namespace {

template <typename T, int N>
struct KVec {
    typedef T type __attribute__((ext_vector_type(N)));
};

template <typename T, int VEC>
__device__ __forceinline__ void k_load(T (&d)[VEC], const T *p) {
    typedef typename KVec<T, VEC>::type V;
    V v = *reinterpret_cast<const V *>(p);
#pragma unroll
    for (int i = 0; i < VEC; ++i) d[i] = v[i];
}

template <typename T, int VEC>
__device__ __forceinline__ void k_store(T *p, const T (&s)[VEC]) {
    typedef typename KVec<T, VEC>::type V;
    V v;
#pragma unroll
    for (int i = 0; i < VEC; ++i) v[i] = s[i];
    *reinterpret_cast<V *>(p) = v;
}

// Streaming (non-temporal) forms for data a pass touches once: f and the
// stored states.  u_t keeps ordinary loads: the neighbouring tiles read its
// halo rows and chunks again through L2.
template <typename T, int VEC>
__device__ __forceinline__ void k_load_nt(T (&d)[VEC], const T *p) {
    typedef typename KVec<T, VEC>::type V;
    V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
    for (int i = 0; i < VEC; ++i) d[i] = v[i];
}

template <typename T, int VEC>
__device__ __forceinline__ void k_store_nt(T *p, const T (&s)[VEC]) {
    typedef typename KVec<T, VEC>::type V;
    V v;
#pragma unroll
    for (int i = 0; i < VEC; ++i) v[i] = s[i];
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
}

template <typename T, int VEC>
__device__ __forceinline__ void k_zero(T (&d)[VEC]) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) d[i] = T(0);
}

template <typename T, int VEC>
__device__ __forceinline__ void k_copy(T (&d)[VEC], const T (&s)[VEC]) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) d[i] = s[i];
}

// lane - 1 (CTRL 0x138, wave_shr:1) or lane + 1 (0x130, wave_shl:1) of the
// wave; zero at the wave's ends
template <int CTRL>
__device__ __forceinline__ float k_dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double k_dpp(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Index i (any integer) under the boundary rule on [0, n); -1 = ghost.
template <int BC>
__device__ __forceinline__ int k_wrap(int i, int n) {
    if (i >= 0 && i < n) return i;
    if constexpr (BC == 1) {
        const int m = i % n;
        return m < 0 ? m + n : m;
    }
    return -1;
}

__device__ __forceinline__ int k_xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, j = b >> 3;
    return xcd * per + min(xcd, rem) + j;
}

// One forward update of a point, operation for operation as in the one-step
// kernel: s6 = ((xm + xp) + (ym + yp)) + (zm + zp), then
// u + c0*(s6 - 6u) - c1*u^3 + c2*f with c1 = dt*beta.
template <typename T>
__device__ __forceinline__ T k_fwd(T c, T xm, T xp, T ym, T yp, T zm, T zp, T fq, T C0, T C1, T C2) {
    const T s6 = ((xm + xp) + (ym + yp)) + (zm + zp);
    const T lapn = fma(T(-6), c, s6);
    T acc = fma(C2, fq, c);
    acc = fma(C0, lapn, acc);
    acc = fma(-(C1 * c) * c, c, acc);
    return acc;
}

// Flag bits of a lane's chunk: bit 0 valid; bit s (1..B) the chunk's row
// carries level s; bit 4 owned (a point of the tile, stored and reduced);
// bit 5 ghost (Dirichlet: outside the grid, every level reads 0); the frame
// column from bit 8 up.
constexpr unsigned kValid = 1u, kOwned = 16u, kGhost = 32u;
constexpr int kColShift = 8;

template <typename T, int VEC, int B, int NT, int KM, int BC, bool SEG, bool RED>
__global__ void __launch_bounds__(NT) tbk_kernel(TbkArgs a) {
    static_assert(B >= 2 && B <= 3, "two or three steps per pass");
    extern __shared__ __align__(16) unsigned char tbk_smem[];
    const int nx = (int)a.nx, ny = (int)a.ny, nz = (int)a.nz;
    const int64_t sz = a.nx * a.ny;
    const int TY = a.ty;
    const int CHF = a.chf;   // chunks per frame row
    const int FW = CHF * VEC;
    const int CH = nx / VEC;  // chunks per grid row
    const int R0 = TY + 2 * B;
    T *const L0 = reinterpret_cast<T *>(tbk_smem);
    // Plane buffer b of level s (1 .. B-1).  Level s lives on frame rows
    // s .. R0-s-1; the buffer is addressed with the level-0 frame offset of
    // a chunk (the base is shifted back by s rows), as an offset from L0 so
    // every access stays an LDS instruction.
    auto LS = [&](int s, int b) -> T * {
        const int r1 = R0 - 2;
        const int off = s == 1 ? R0 + (b & 1) * r1 : R0 + 2 * r1 + (b & 1) * (R0 - 4);
        return L0 + (off - s) * FW;
    };

    const int tid = threadIdx.x;
    const int wlane = tid & 63;
    const int Lb = k_xcd_remap(blockIdx.x, gridDim.x);
    const int ncol = a.nslab * a.nseg;
    const int cb = Lb % ncol;
    const int zrun = Lb / ncol;
    // blocks of sblk slabs (the last may be shorter), segments within a block
    const int blk = cb / (a.nseg * a.sblk);
    const int rem = cb - blk * a.nseg * a.sblk;
    const int hb = min(a.sblk, a.nslab - blk * a.sblk);
    const int seg = rem / hb;
    const int slab = blk * a.sblk + rem % hb;
    const int y0 = slab * TY;
    const int z0 = zrun * a.zc;
    const int z1 = min(nz, z0 + a.zc);
    const int gc0 = SEG ? seg * a.wc - a.halo : 0;  // grid chunk of frame column 0
    const int oc0 = SEG ? a.halo : 0;               // owned frame columns [oc0, oc1)
    const int oc1 = SEG ? a.halo + min(a.wc, CH - seg * a.wc) : CH;

    const T *__restrict__ U = static_cast<const T *>(a.u);
    const T *__restrict__ F = static_cast<const T *>(a.f);
    T *__restrict__ O = static_cast<T *>(a.out);
    const T C0 = (T)a.c0, C1 = (T)a.c1, C2 = (T)a.c2;

    // The lane's chunks: chunk k is frame row r = idx / CHF, column c = idx %
    // CHF; lofs = r*FW + c*VEC (LDS offset), gofs = its offset in a grid
    // plane (-1: ghost row or column), col = c.
    int lofs[KM], gofs[KM];
    unsigned flags[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int idx = tid + k * NT;
        const bool v = idx < R0 * CHF;
        const int r = v ? idx / CHF : 0;
        const int c = v ? idx % CHF : 0;
        const int gy = y0 - B + r;
        const int gyr = k_wrap<BC>(gy, ny);
        const int gcr = SEG ? k_wrap<BC>(gc0 + c, CH) : c;
        lofs[k] = r * FW + c * VEC;
        gofs[k] = (gyr >= 0 && gcr >= 0) ? gyr * nx + gcr * VEC : -1;
        unsigned fl = (v ? kValid : 0u) | ((unsigned)c << kColShift);
#pragma unroll
        for (int s = 1; s <= B; ++s)
            if (v && r >= s && r < R0 - s) fl |= 1u << s;
        if (v && r >= B && r < B + TY && gy < ny && c >= oc0 && c < oc1) fl |= kOwned;
        if (gofs[k] < 0) fl |= kGhost;
        flags[k] = fl;
    }

    auto load_u = [&](int zq, T (&d)[KM][VEC]) {
        const int zr = k_wrap<BC>(zq, nz);
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if ((flags[k] & kValid) && gofs[k] >= 0 && zr >= 0)
                k_load<T, VEC>(d[k], U + (int64_t)zr * sz + gofs[k]);
            else
                k_zero<T, VEC>(d[k]);
        }
    };
    // f at plane zq on the level-1 rows (the rows every level uses)
    auto load_f = [&](int zq, T (&d)[KM][VEC]) {
        const int zr = k_wrap<BC>(zq, nz);
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if ((flags[k] & 2u) && gofs[k] >= 0 && zr >= 0)
                k_load_nt<T, VEC>(d[k], F + (int64_t)zr * sz + gofs[k]);
            else
                k_zero<T, VEC>(d[k]);
        }
    };
    // x-neighbours of the chunk at LDS offset o (frame column c) in the
    // buffer `base`: across the wave where the neighbour chunk is the
    // adjacent lane's, from LDS at the wave's ends; past the frame's ends
    // the whole-row tile wraps (periodic) or reads 0, and a segment reads 0
    // (those points lie in the halo, where the level is not needed)
    auto xnbrs = [&](const T *base, int o, int c, const T (&v)[VEC], T &lft, T &rgt) {
        const T fl = k_dpp<0x138>(v[VEC - 1]);
        const T fu = k_dpp<0x130>(v[0]);
        if (c > 0) lft = wlane != 0 ? fl : base[o - 1];
        else if (!SEG && BC == 1) lft = base[o + FW - 1];
        else lft = T(0);
        if (c < CHF - 1) rgt = wlane != 63 ? fu : base[o + VEC];
        else if (!SEG && BC == 1) rgt = base[o - c * VEC];
        else rgt = T(0);
    };

    // register queues: level 0 at q-1, q+1 and the prefetched q+2; for s = 2..B
    // level s-1 below (zm[s-2]; the level above is the plane stage s-1 has
    // just written to LDS, read back from the lane's own chunk); f at q,
    // q-1, .., q-B+1 and the prefetched q+1
    T am[KM][VEC], ap[KM][VEC], an[KM][VEC];
    T zm[B - 1][KM][VEC];
    T fq[B][KM][VEC], fn[KM][VEC];
    double es[B], rs[B];
#pragma unroll
    for (int s = 0; s < B; ++s) es[s] = rs[s] = 0.0;

    const int q0 = z0 - B + 1;
    {
        T ac0[KM][VEC];
        if (z0 < z1) {
            load_u(q0 - 1, am);
            load_u(q0, ac0);
            load_u(q0 + 1, ap);
            load_f(q0, fq[0]);
        }
#pragma unroll
        for (int k = 0; k < KM; ++k) {
#pragma unroll
            for (int s = 0; s < B - 1; ++s) k_zero<T, VEC>(zm[s][k]);
#pragma unroll
            for (int s = 1; s < B; ++s) k_zero<T, VEC>(fq[s][k]);
            if (flags[k] & kValid) k_store<T, VEC>(L0 + lofs[k], ac0[k]);
        }
    }

    const int qlast = z1 + B - 2;
    for (int q = q0; z0 < z1 && q <= qlast; ++q) {
        const bool more = q < qlast;
        if (more) {
            load_u(q + 2, an);
            load_f(q + 1, fn);
        }
        __syncthreads();

#pragma unroll
        for (int s = 1; s <= B; ++s) {
            const int p = q - s + 1;  // plane of level s in this iteration
            if (q < z0 - B + 2 * s - 1) continue;
            const bool owned_plane = p >= z0 && p < z1;
            const int pr = k_wrap<BC>(p, nz);
            const T *src = s == 1 ? L0 : LS(s - 1, p);
            const T *above = s == 1 ? L0 : LS(s - 1, p + 1);  // level s-1 at p+1 (s >= 2)
            T *dst = s < B ? LS(s, p) : nullptr;
            T *mid = s < B ? static_cast<T *>(a.mid[s - 1]) : nullptr;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const unsigned fl = flags[k];
                // the row test keeps whole frame rows together, so a lane and
                // the neighbours it exchanges x-values with are active
                // together; conditions that depend on the column (owned,
                // ghost) only select results below
                if (!(fl & (1u << s))) continue;
                const int o = lofs[k];
                T c[VEC], res[VEC];
                k_load<T, VEC>(c, src + o);
                T lft, rgt;
                xnbrs(src, o, (int)(fl >> kColShift), c, lft, rgt);
                if (s < B && BC == 0 && (pr < 0 || (fl & kGhost))) {
                    k_zero<T, VEC>(res);
                } else {
                    T ym[VEC], yp[VEC], zp[VEC];
                    k_load<T, VEC>(ym, src + o - FW);
                    k_load<T, VEC>(yp, src + o + FW);
                    if (s == 1) k_copy<T, VEC>(zp, ap[k]);
                    else k_load<T, VEC>(zp, above + o);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const T xm = e == 0 ? lft : c[e > 0 ? e - 1 : 0];
                        const T xp = e == VEC - 1 ? rgt : c[e + 1 < VEC ? e + 1 : e];
                        const T zmv = s == 1 ? am[k][e] : zm[s >= 2 ? s - 2 : 0][k][e];
                        res[e] = k_fwd<T>(c[e], xm, xp, ym[e], yp[e], zmv, zp[e], fq[s - 1][k][e], C0, C1, C2);
                    }
                }
                const bool here = (fl & kOwned) && owned_plane;
                if (s < B) {
                    k_store<T, VEC>(dst + o, res);
                    if (mid && here) k_store_nt<T, VEC>(mid + (int64_t)p * sz + gofs[k], res);
                } else if (fl & kOwned) {
                    k_store_nt<T, VEC>(O + (int64_t)p * sz + gofs[k], res);
                }
                if constexpr (RED) {
                    if (here) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const double d = (double)res[e];
                            es[s - 1] = fma(d, d, es[s - 1]);
                            const double dd = d - (double)c[e];
                            rs[s - 1] = fma(dd, dd, rs[s - 1]);
                        }
                    }
                }
            }
        }

        if (more) {
            // next iteration's lower neighbours: level 0 at q, level s-1 at
            // q-s+1 (stage s's centre in this iteration); each lane reads back
            // only its own chunks
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (flags[k] & kValid) k_load<T, VEC>(am[k], L0 + lofs[k]);
#pragma unroll
                for (int s = 2; s <= B; ++s)
                    if (flags[k] & (1u << s)) k_load<T, VEC>(zm[s - 2][k], LS(s - 1, q - s + 1) + lofs[k]);
            }
        }
        __syncthreads();
        if (more) {
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (flags[k] & kValid) k_store<T, VEC>(L0 + lofs[k], ap[k]);  // level 0 at q+1
                k_copy<T, VEC>(ap[k], an[k]);
#pragma unroll
                for (int s = B - 1; s >= 1; --s) k_copy<T, VEC>(fq[s][k], fq[s - 1][k]);
                k_copy<T, VEC>(fq[0][k], fn[k]);
            }
        }
    }

    if constexpr (RED) {
        double *red = reinterpret_cast<double *>(tbk_smem);
        const int wave = tid >> 6;
        constexpr int NW = NT / 64;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int s = 0; s < B; ++s) {
                es[s] += __shfl_xor(es[s], off, 64);
                rs[s] += __shfl_xor(rs[s], off, 64);
            }
        }
        __syncthreads();
        if (wlane == 0) {
#pragma unroll
            for (int s = 0; s < B; ++s) {
                red[2 * B * wave + 2 * s] = es[s];
                red[2 * B * wave + 2 * s + 1] = rs[s];
            }
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
            for (int s = 0; s < B; ++s) {
                double e = 0.0, r = 0.0;
                for (int w = 0; w < NW; ++w) {
                    e += red[2 * B * w + 2 * s];
                    r += red[2 * B * w + 2 * s + 1];
                }
                a.part[s][2 * (int64_t)Lb] = e;
                a.part[s][2 * (int64_t)Lb + 1] = r;
            }
        }
    }
}

// Ring form of the same pass, compiled for 768 lanes with two chunks each
// (three waves per SIMD, up to 168 VGPRs).  Each lane keeps, for its own
// chunks, the three planes of every level that the next level reads (p-1,
// p, p+1) in registers, so only the y- and x-neighbours of a point come
// from LDS:
//   * level 0 (u) in a ring of three planes, the load of plane q+2 issued as
//     soon as plane q-1 is dead (after stage 1 of iteration q);
//   * level s (1 .. B-1) in a ring of three planes, written by stage s and
//     read by stage s+1 of the same and the next two iterations;
//   * f in a ring of three planes loaded two planes ahead; with B = 3 the
//     plane the last stage needs waits in one LDS plane of the lane's own
//     chunks;
//   * level 0 in two LDS planes (the current plane and the next), so one
//     barrier per plane separates every LDS write from the reads of it and
//     every read from the next write to the same buffer.
// Ring slots are (plane - q0) mod 3, compile-time constants in a plane loop
// unrolled three times, so no register copies rotate the queues.  Every
// point is computed with the one-step kernel's operations, as in tbk_kernel.
template <typename T, int VEC, int B, int NT, int KM, int BC, bool SEG, bool RED>
__global__ void __launch_bounds__(NT) tbr_kernel(TbkArgs a) {
    static_assert(B >= 2 && B <= 3, "two or three steps per pass");
    extern __shared__ __align__(16) unsigned char tbk_smem[];
    const int nx = (int)a.nx, ny = (int)a.ny, nz = (int)a.nz;
    const int64_t sz = a.nx * a.ny;
    const int TY = a.ty;
    const int CHF = a.chf;
    const int FW = CHF * VEC;
    const int CH = nx / VEC;
    const int R0 = TY + 2 * B;
    T *const SM = reinterpret_cast<T *>(tbk_smem);
    // LDS: level 0 at planes of both parities (R0 rows each), then level s =
    // 1 .. B-1 at both parities (frame rows s .. R0-s-1), then (B = 3) f on
    // the level-1 rows; every buffer is addressed with a chunk's level-0
    // frame offset (bases shifted back by the buffer's first row).
    auto L0p = [&](int p) -> T * { return SM + (p & 1) * R0 * FW; };
    auto LSp = [&](int s, int p) -> T * {
        const int off = s == 1 ? 2 * R0 : 4 * R0 - 4;
        return SM + (off + (p & 1) * (R0 - 2 * s) - s) * FW;
    };
    T *const FB = SM + (6 * R0 - 12 - 1) * FW;

    const int tid = threadIdx.x;
    const int wlane = tid & 63;
    const int Lb = k_xcd_remap(blockIdx.x, gridDim.x);
    const int ncol = a.nslab * a.nseg;
    const int cb = Lb % ncol;
    const int zrun = Lb / ncol;
    const int blk = cb / (a.nseg * a.sblk);
    const int rem = cb - blk * a.nseg * a.sblk;
    const int hb = min(a.sblk, a.nslab - blk * a.sblk);
    const int seg = rem / hb;
    const int slab = blk * a.sblk + rem % hb;
    const int y0 = slab * TY;
    const int z0 = zrun * a.zc;
    const int z1 = min(nz, z0 + a.zc);
    const int gc0 = SEG ? seg * a.wc - a.halo : 0;
    const int oc0 = SEG ? a.halo : 0;
    const int oc1 = SEG ? a.halo + min(a.wc, CH - seg * a.wc) : CH;

    const T *__restrict__ U = static_cast<const T *>(a.u);
    const T *__restrict__ F = static_cast<const T *>(a.f);
    T *__restrict__ O = static_cast<T *>(a.out);
    const T C0 = (T)a.c0, C1 = (T)a.c1, C2 = (T)a.c2;

    int lofs[KM], gofs[KM];
    unsigned flags[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int idx = tid + k * NT;
        const bool v = idx < R0 * CHF;
        const int r = v ? idx / CHF : 0;
        const int c = v ? idx % CHF : 0;
        const int gy = y0 - B + r;
        const int gyr = k_wrap<BC>(gy, ny);
        const int gcr = SEG ? k_wrap<BC>(gc0 + c, CH) : c;
        lofs[k] = r * FW + c * VEC;
        gofs[k] = (gyr >= 0 && gcr >= 0) ? gyr * nx + gcr * VEC : -1;
        unsigned fl = (v ? kValid : 0u) | ((unsigned)c << kColShift);
#pragma unroll
        for (int s = 1; s <= B; ++s)
            if (v && r >= s && r < R0 - s) fl |= 1u << s;
        if (v && r >= B && r < B + TY && gy < ny && c >= oc0 && c < oc1) fl |= kOwned;
        if (gofs[k] < 0) fl |= kGhost;
        flags[k] = fl;
    }

    // Every lane loads, from a uniform plane base plus its chunk's 32-bit
    // byte offset in the plane (the planner keeps a plane under 4 GiB for
    // this kernel), so the ring registers have one writer and the loads'
    // waits can be counted instead of drained.  Chunks outside the grid
    // (ghost rows, columns or planes) and lanes past the frame read a valid
    // chunk instead; level 0 of a ghost point is zeroed once, when its plane
    // becomes a lane's upper z-neighbour, so its LDS copy and the x-exchange
    // see zeros, and every higher level of a ghost point is computed as
    // zero; f at a ghost point is never used.
    uint32_t gb[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) gb[k] = gofs[k] >= 0 ? (uint32_t)gofs[k] * (uint32_t)sizeof(T) : 0u;
    auto at = [&](const T *plane, int k) -> const T * {
        return reinterpret_cast<const T *>(reinterpret_cast<const char *>(plane) + gb[k]);
    };
    auto load_u = [&](int zq, T (&d)[KM][VEC]) {
        const int zr = k_wrap<BC>(zq, nz);
        const T *plane = U + (int64_t)(zr >= 0 ? zr : 0) * sz;
#pragma unroll
        for (int k = 0; k < KM; ++k) k_load<T, VEC>(d[k], at(plane, k));
    };
    auto load_f = [&](int zq, T (&d)[KM][VEC]) {
        const int zr = k_wrap<BC>(zq, nz);
        const T *plane = F + (int64_t)(zr >= 0 ? zr : 0) * sz;
#pragma unroll
        for (int k = 0; k < KM; ++k) k_load_nt<T, VEC>(d[k], at(plane, k));
    };
    // Dirichlet: level 0 at plane zq is zero on ghost chunks and planes
    auto ghost0 = [&](int zq, T (&d)[KM][VEC]) {
        if constexpr (BC == 0) {
            const bool gp = zq < 0 || zq >= nz;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const bool g = gp || (flags[k] & kGhost);
#pragma unroll
                for (int e = 0; e < VEC; ++e) d[k][e] = g ? T(0) : d[k][e];
            }
        }
    };
    auto xnbrs = [&](const T *base, int o, int c, const T (&v)[VEC], T &lft, T &rgt) {
        const T fl = k_dpp<0x138>(v[VEC - 1]);
        const T fu = k_dpp<0x130>(v[0]);
        if (c > 0) lft = wlane != 0 ? fl : base[o - 1];
        else if (!SEG && BC == 1) lft = base[o + FW - 1];
        else lft = T(0);
        if (c < CHF - 1) rgt = wlane != 63 ? fu : base[o + VEC];
        else if (!SEG && BC == 1) rgt = base[o - c * VEC];
        else rgt = T(0);
    };

    // rings: slot (plane - q0) mod 3
    T RU[3][KM][VEC];          // level 0
    T RZ[B - 1][3][KM][VEC];   // levels 1 .. B-1
    T RF[3][KM][VEC];          // f
    double es[B], rs[B];
#pragma unroll
    for (int s = 0; s < B; ++s) es[s] = rs[s] = 0.0;

    const int q0 = z0 - B + 1;
    const int qlast = z1 + B - 2;
    // plane q0 + j sits in slot j mod 3; at iteration q (phase ph = (q -
    // q0) mod 3) plane q + d sits in slot rs3(ph + d)
    constexpr auto rs3 = [](int v) constexpr { return ((v % 3) + 3) % 3; };
#pragma unroll
    for (int k = 0; k < KM; ++k) {
#pragma unroll
        for (int s = 0; s < B - 1; ++s)
#pragma unroll
            for (int j = 0; j < 3; ++j) k_zero<T, VEC>(RZ[s][j][k]);
        k_zero<T, VEC>(RF[2][k]);
    }
    if (z0 < z1) {
        load_u(q0 - 1, RU[2]);
        load_u(q0, RU[0]);
        load_u(q0 + 1, RU[1]);
        load_f(q0, RF[0]);
        load_f(q0 + 1, RF[1]);
        ghost0(q0 - 1, RU[2]);
        ghost0(q0, RU[0]);
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (flags[k] & kValid) k_store<T, VEC>(L0p(q0) + lofs[k], RU[0][k]);
    }
    // the prologue's loads have landed: the loop starts with no load in
    // flight on the path from here, so its waits count only its own loads
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    auto iter = [&](auto phc, const int q) {
        constexpr int PH = decltype(phc)::value;
        ghost0(q + 1, RU[rs3(PH + 1)]);
#pragma unroll
        for (int s = 1; s <= B; ++s) {
            if (q < q0 + 2 * (s - 1)) continue;  // stage s starts two planes after stage s-1
            const int p = q - s + 1;               // plane of level s
            const bool owned_plane = p >= z0 && p < z1;
            const int pr = k_wrap<BC>(p, nz);
            const T *src = s == 1 ? L0p(q) : LSp(s - 1, p);
            T *dst = s < B ? LSp(s, p) : nullptr;
            T *mid = s < B ? static_cast<T *>(a.mid[s - 1]) : nullptr;
            // level s-1 at planes p-1, p, p+1 (registers), level s at p (result)
            T(&Lm)[KM][VEC] = s == 1 ? RU[rs3(PH - 1)] : RZ[s >= 2 ? s - 2 : 0][rs3(PH - s)];
            T(&Lc)[KM][VEC] = s == 1 ? RU[rs3(PH)] : RZ[s >= 2 ? s - 2 : 0][rs3(PH + 1 - s)];
            T(&Lp)[KM][VEC] = s == 1 ? RU[rs3(PH + 1)] : RZ[s >= 2 ? s - 2 : 0][rs3(PH + 2 - s)];
            T(&Lo)[KM][VEC] = RZ[s < B ? s - 1 : 0][rs3(PH + 1 - s)];
            // the y- and x-neighbours in the frame plane come from LDS, the
            // z-neighbours and the centre from the rings
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const unsigned fl = flags[k];
                if (!(fl & (1u << s))) continue;
                const int o = lofs[k];
                T ym[VEC], yp[VEC], f3[VEC], lft, rgt;
                k_load<T, VEC>(ym, src + o - FW);
                k_load<T, VEC>(yp, src + o + FW);
                if (s == 3) k_load<T, VEC>(f3, FB + o);
                xnbrs(src, o, (int)(fl >> kColShift), Lc[k], lft, rgt);
                T res[VEC];
                if (s < B && BC == 0 && (pr < 0 || (fl & kGhost))) {
                    k_zero<T, VEC>(res);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const T xm = e == 0 ? lft : Lc[k][e > 0 ? e - 1 : 0];
                        const T xp = e == VEC - 1 ? rgt : Lc[k][e + 1 < VEC ? e + 1 : e];
                        const T fq = s == 1 ? RF[rs3(PH)][k][e] : s == 2 ? RF[rs3(PH - 1)][k][e] : f3[e];
                        res[e] = k_fwd<T>(Lc[k][e], xm, xp, ym[e], yp[e], Lm[k][e], Lp[k][e], fq, C0, C1, C2);
                    }
                }
                const bool here = (fl & kOwned) && owned_plane;
                if (s < B) {
                    k_store<T, VEC>(dst + o, res);
                    k_copy<T, VEC>(Lo[k], res);
                    if (mid && here) k_store_nt<T, VEC>(const_cast<T *>(at(mid + (int64_t)p * sz, k)), res);
                } else if (fl & kOwned) {
                    k_store_nt<T, VEC>(const_cast<T *>(at(O + (int64_t)p * sz, k)), res);
                }
                if constexpr (RED) {
                    if (here) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const double d = (double)res[e];
                            es[s - 1] = fma(d, d, es[s - 1]);
                            const double dd = d - (double)Lc[k][e];
                            rs[s - 1] = fma(dd, dd, rs[s - 1]);
                        }
                    }
                }
            }
            // level 0 at q-1 is dead: fetch plane q+2 into its slot
            if (s == 1) load_u(q + 2, RU[rs3(PH + 2)]);
        }
        // f of plane q-1 is dead after this iteration's stages (B = 2) or
        // waits in LDS for the last stage of the next one (B = 3); its slot
        // takes plane q+2
        if (B == 3) {
#pragma unroll
            for (int k = 0; k < KM; ++k)
                if (flags[k] & 2u) k_store<T, VEC>(FB + lofs[k], RF[rs3(PH - 1)][k]);
        }
        load_f(q + 2, RF[rs3(PH + 2)]);
        if (q + 1 <= qlast) {
#pragma unroll
            for (int k = 0; k < KM; ++k)
                if (flags[k] & kValid) k_store<T, VEC>(L0p(q + 1) + lofs[k], RU[rs3(PH + 1)][k]);
        }
        __syncthreads();
    };

    // whole trips of three planes (one back-edge, no side exits, so each
    // ring slot keeps its registers), then up to two planes
    if (z0 < z1) {
        int q = q0;
        for (; q + 2 <= qlast; q += 3) {
            iter(std::integral_constant<int, 0>{}, q);
            iter(std::integral_constant<int, 1>{}, q + 1);
            iter(std::integral_constant<int, 2>{}, q + 2);
        }
        if (q <= qlast) iter(std::integral_constant<int, 0>{}, q);
        if (q + 1 <= qlast) iter(std::integral_constant<int, 1>{}, q + 1);
    }

    if constexpr (RED) {
        double *red = reinterpret_cast<double *>(tbk_smem);
        const int wave = tid >> 6;
        constexpr int NW = NT / 64;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int s = 0; s < B; ++s) {
                es[s] += __shfl_xor(es[s], off, 64);
                rs[s] += __shfl_xor(rs[s], off, 64);
            }
        }
        __syncthreads();
        if (wlane == 0) {
#pragma unroll
            for (int s = 0; s < B; ++s) {
                red[2 * B * wave + 2 * s] = es[s];
                red[2 * B * wave + 2 * s + 1] = rs[s];
            }
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
            for (int s = 0; s < B; ++s) {
                double e = 0.0, r = 0.0;
                for (int w = 0; w < NW; ++w) {
                    e += red[2 * B * w + 2 * s];
                    r += red[2 * B * w + 2 * s + 1];
                }
                a.part[s][2 * (int64_t)Lb] = e;
                a.part[s][2 * (int64_t)Lb + 1] = r;
            }
        }
    }
}

template <typename T, int VEC, int B, int NT, int KM, int BC, bool SEG, bool RED, bool RING>
auto tbk_fn() {
    if constexpr (RING) return tbr_kernel<T, VEC, B, NT, KM, BC, SEG, RED>;
    else return tbk_kernel<T, VEC, B, NT, KM, BC, SEG, RED>;
}

template <typename T, int VEC, int B, int NT, int KM, bool RING>
hipError_t tbk_launch_t(int bc, bool reduce, const TbkTile &t, const TbkArgs &a, hipStream_t st) {
    const dim3 grid(t.nblk), block(NT);
    const size_t lds = t.lds_bytes;
#define DCP_TBK(BCV, SEGV, REDV)                                                                     \
    do {                                                                                             \
        auto fn = tbk_fn<T, VEC, B, NT, KM, BCV, SEGV, REDV, RING>();                                \
        hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),                      \
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (e_ != hipSuccess) return e_;                                                             \
        hipLaunchKernelGGL(fn, grid, block, lds, st, a);                                             \
    } while (0)
#define DCP_TBK_RED(BCV, SEGV)             \
    do {                                   \
        if (reduce) DCP_TBK(BCV, SEGV, true); \
        else DCP_TBK(BCV, SEGV, false);    \
    } while (0)
    if (bc == 0) {
        if (t.seg) DCP_TBK_RED(0, true);
        else DCP_TBK_RED(0, false);
    } else {
        if (t.seg) DCP_TBK_RED(1, true);
        else DCP_TBK_RED(1, false);
    }
#undef DCP_TBK_RED
#undef DCP_TBK
    return hipGetLastError();
}

// Lane shapes: 1024 lanes with two chunks each (four waves per SIMD, up to
// 128 VGPRs), 512 lanes with four (two waves per SIMD, up to 256 VGPRs), or
// the ring form with 768 lanes of two chunks (three waves per SIMD, up to 168
// VGPRs).
struct TbkLanes {
    int nt, km;
    bool ring;
};
constexpr TbkLanes kTbkLanes[] = {{1024, 2, false}, {512, 4, false}, {768, 2, true}};

// LDS rows of a tile: level 0 (ty + 2B rows), two planes of each level s =
// 1 .. B-1 (ty + 2(B-s) rows each); the ring form adds a second level-0
// plane and, with B = 3, one plane of f on the level-1 rows.
int tbk_lds_rows(int B, int ty, bool ring) {
    const int r0 = ty + 2 * B;
    int rows = ring ? 2 * r0 : r0;
    for (int s = 1; s < B; ++s) rows += 2 * (ty + 2 * (B - s));
    if (ring && B == 3) rows += r0 - 2;
    return rows;
}

}  // namespace

bool tbk_plan(int dtype, int B, int64_t nx, int64_t ny, int64_t nz, bool vec_ok, size_t lds_limit, int lanes,
              int force_wc, int force_ty, TbkTile *t) {
    const int esz = dtype == 0 ? 8 : 4;
    const int vec = 16 / esz;
    if (B < 2 || B > 3) return false;
    if (!vec_ok || nx <= 0 || ny <= 0 || nz <= 0 || nx % vec != 0) return false;
    if (nx > (1 << 24) || nx * ny > (int64_t)INT32_MAX || nz > (1 << 29) || ny > (1 << 29)) return false;
    const int64_t ch = nx / vec;
    const int halo = (B + vec - 1) / vec;
    const TbkLanes ln = kTbkLanes[lanes == 512 ? 1 : lanes == 768 ? 2 : 0];
    // the ring form addresses a chunk as a plane base plus a 32-bit offset
    // (the tile limits below already keep its planes under 1 GiB)
    if (ln.ring && nx * ny * esz > (int64_t)UINT32_MAX) return false;
    // Candidates: whole rows, or segments of 256, 128, 64 or 32 chunks; slabs
    // of 16, 8 or 4 rows.  Each must fit the lanes and the LDS; the planner
    // takes the one that recomputes the fewest points per owned point (the
    // halo rows and chunks of levels 1 .. B-1), whole rows first on a tie.
    double best = 1e30;
    bool found = false;
    const int64_t widths[] = {ch, 256, 128, 64, 32};
    for (int64_t wc : widths) {
        if (wc > ch) continue;
        const bool seg = wc < ch;
        if (force_wc > 0 && (seg ? wc != force_wc : force_wc < ch)) continue;
        const int64_t chf = seg ? wc + 2 * halo : ch;
        for (int ty : {16, 8, 4}) {
            if (force_ty > 0 && ty != force_ty) continue;
            const int r0 = ty + 2 * B;
            if ((int64_t)r0 * chf > (int64_t)ln.nt * ln.km) continue;
            const size_t lds = (size_t)tbk_lds_rows(B, ty, ln.ring) * (size_t)chf * 16;
            if (lds > lds_limit) continue;
            if (lds < (size_t)(ln.nt / 64) * 2 * B * sizeof(double)) continue;
            const int64_t nslab = (ny + ty - 1) / ty;
            const int64_t nseg = (ch + wc - 1) / wc;
            if (nslab * nseg > 65536) continue;
            double work = 0.0;
            for (int s = 1; s <= B; ++s) work += (double)(ty + 2 * (B - s)) * (double)chf;
            const double cost = work / ((double)ty * (double)wc * B);
            if (cost < best - 1e-9) {
                best = cost;
                found = true;
                int64_t cols = nslab * nseg;
                int64_t runs = 256 / cols;
                if (runs < 1) runs = 1;
                if (runs > nz) runs = nz;
                int64_t zc = (nz + runs - 1) / runs;
                runs = (nz + zc - 1) / zc;
                t->B = B;
                t->vec = vec;
                t->ty = ty;
                t->nt = ln.nt;
                t->km = ln.km;
                t->seg = seg;
                t->wc = (int)wc;
                t->halo = seg ? halo : 0;
                t->chf = (int)chf;
                t->nseg = (int)nseg;
                t->nslab = (int)nslab;
                t->zc = (int)zc;
                t->nruns = (int)runs;
                t->nblk = (int)(cols * runs);
                t->lds_bytes = lds;
                // the 256 workgroups go round-robin to the 8 XCDs and are
                // renumbered so each XCD holds a contiguous run of tiles:
                // make that run a block of slabs across all segments, so the
                // halo rows and chunks a tile shares with its neighbours are
                // read through the same L2 (measured at 512^3 FP64: reads per
                // pass 2.55 -> 2.28 GiB, 1.14x the algorithmic 2 GiB)
                int64_t per = (t->nblk + 7) / 8 / nseg;
                t->sblk = (int)(per < 1 ? 1 : per > nslab ? nslab : per);
            }
        }
    }
    return found;
}

hipError_t launch_tbk(int dtype, int bc, bool reduce, const TbkTile &t, const TbkArgs &a, hipStream_t st) {
    const bool n1024 = t.nt == 1024 && t.km == 2, n512 = t.nt == 512 && t.km == 4, n768 = t.nt == 768 && t.km == 2;
    if ((!n1024 && !n512 && !n768) || (t.B != 2 && t.B != 3)) return hipErrorInvalidValue;
#define DCP_TBK_SHAPES(TT, VV, BB)                                                    \
    do {                                                                              \
        if (n1024) return tbk_launch_t<TT, VV, BB, 1024, 2, false>(bc, reduce, t, a, st); \
        if (n768) return tbk_launch_t<TT, VV, BB, 768, 2, true>(bc, reduce, t, a, st);    \
        return tbk_launch_t<TT, VV, BB, 512, 4, false>(bc, reduce, t, a, st);             \
    } while (0)
    if (dtype == 0) {
        if (t.B == 2) DCP_TBK_SHAPES(double, 2, 2);
        DCP_TBK_SHAPES(double, 2, 3);
    }
    if (t.B == 2) DCP_TBK_SHAPES(float, 4, 2);
    DCP_TBK_SHAPES(float, 4, 3);
#undef DCP_TBK_SHAPES
}

}  // namespace dcp
