// dcp_tblock.hip -- two fused time steps per pass over memory (temporal
// blocking) for the reaction-diffusion step on gfx950.
//
// One pass reads u_t and f once and writes u_{t+2}: 3 fields moved per two
// steps instead of per step.  The paper's fusion (Sec. 3.1) merges the maps
// of one step; this goes one step further and fuses two consecutive steps of
// the time loop, which is legal because step t+2 at a point reads step t+1
// only within distance 1, and step t+1 is recomputed on a one-row halo.
//
// Layout of the work:
//   * a workgroup (1024 lanes with two 16-byte chunks each; one workgroup
//     per CU) owns full x-rows: a slab of TY rows x all
//     nx points x zc planes, so there is no x-halo at all and the periodic
//     x-wrap stays inside the slab;
//   * the grid has one workgroup per CU (256), so every slab of a z-run is
//     resident at once and neighbouring slabs march up z together; their
//     two-row y-halos are read while the neighbour reads the same rows, and
//     are served by the XCD's L2 (workgroups are numbered so an XCD holds a
//     contiguous run of slabs);
//   * level 0 (u_t) of the current plane sits in LDS with a two-row halo,
//     level 1 (u_{t+1}) of the two most recent planes sits in LDS with a
//     one-row halo; the z-neighbours of both levels stay in each lane's
//     registers (register queues), and the next input plane is prefetched
//     one iteration ahead;
//   * step t+1 is computed at plane q while step t+2 is computed at plane
//     q-1 (a two-stage z-pipeline), two barriers per plane.
// Every point is computed with exactly the same operations, in the same
// order, as the one-step kernel, so a pass equals two one-step launches bit
// for bit; the two steps' norms are reduced over the owned points only.
#include <cstdlib>

#include "dcp_internal.h"

namespace dcp {
namespace {


template <typename T, int N>
struct TbVec {
    typedef T type __attribute__((ext_vector_type(N)));
};

template <typename T, int VEC>
__device__ __forceinline__ void tb_load(T (&d)[VEC], const T *p) {
    if constexpr (VEC == 1) {
        d[0] = *p;
    } else {
        typedef typename TbVec<T, VEC>::type V;
        V v = *reinterpret_cast<const V *>(p);
#pragma unroll
        for (int i = 0; i < VEC; ++i) d[i] = v[i];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void tb_store(T *p, const T (&s)[VEC]) {
    if constexpr (VEC == 1) {
        *p = s[0];
    } else {
        typedef typename TbVec<T, VEC>::type V;
        V v;
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[i] = s[i];
        *reinterpret_cast<V *>(p) = v;
    }
}

// Streaming (non-temporal) forms for data a pass touches once: the point
// operands, the stored states and the running sum.  The stencil operand
// keeps ordinary loads: neighbouring slabs read its halo rows again
// through L2.
template <typename T, int VEC>
__device__ __forceinline__ void tb_load_nt(T (&d)[VEC], const T *p) {
    if constexpr (VEC == 1) {
        d[0] = __builtin_nontemporal_load(p);
    } else {
        typedef typename TbVec<T, VEC>::type V;
        V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
        for (int i = 0; i < VEC; ++i) d[i] = v[i];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void tb_store_nt(T *p, const T (&s)[VEC]) {
    if constexpr (VEC == 1) {
        __builtin_nontemporal_store(s[0], p);
    } else {
        typedef typename TbVec<T, VEC>::type V;
        V v;
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[i] = s[i];
        __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void tb_zero(T (&d)[VEC]) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) d[i] = T(0);
}

template <typename T, int VEC>
__device__ __forceinline__ void tb_copy(T (&d)[VEC], const T (&s)[VEC]) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) d[i] = s[i];
}

// The value of lane - 1 (CTRL 0x138, wave_shr:1) or lane + 1 (0x130,
// wave_shl:1) of the wave; zero at the wave's ends.
template <int CTRL>
__device__ __forceinline__ float tb_dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double tb_dpp(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Coordinate under the boundary rule for any integer i; -1 = ghost (zero).
template <int BC>
__device__ __forceinline__ int tb_wrap(int i, int n) {
    if (i >= 0 && i < n) return i;
    if constexpr (BC == 1) {
        const int m = i % n;
        return m < 0 ? m + n : m;
    }
    return -1;
}

__device__ __forceinline__ int tb_xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, j = b >> 3;
    return xcd * per + min(xcd, rem) + j;
}

// The one-step updates of a point, operation for operation as in the
// one-step kernel: s6 = ((xm + xp) + (ym + yp)) + (zm + zp).
//   forward: u + c0*(s6 - 6u) - c1*u^3 + c2*f        (c1 = dt*beta)
//   adjoint: l + c0*(s6 - 6l) - c1*u^2*l             (c1 = 3*dt*beta), with the
//            parameter sums (s6 - 6l)*u and l*u^3 accumulated in double by
//            fused multiply-adds when `add` is set
template <typename T>
__device__ __forceinline__ T tb_fwd(T c, T xm, T xp, T ym, T yp, T zm, T zp, T fq, T C0, T C1, T C2) {
    const T s6 = ((xm + xp) + (ym + yp)) + (zm + zp);
    const T lapn = fma(T(-6), c, s6);
    T acc = fma(C2, fq, c);
    acc = fma(C0, lapn, acc);
    acc = fma(-(C1 * c) * c, c, acc);
    return acc;
}

template <typename T>
__device__ __forceinline__ T tb_adj(T c, T xm, T xp, T ym, T yp, T zm, T zp, T uq, T C0, T C1, bool add,
                                    double &sa, double &sb) {
    const T s6 = ((xm + xp) + (ym + yp)) + (zm + zp);
    const T lapn = fma(T(-6), c, s6);
    T acc = fma(C0, lapn, c);
    acc = fma(-(C1 * uq) * uq, c, acc);
    if (add) {
        const double du = (double)uq;
        sa = fma((double)lapn, du, sa);
        sb = fma((double)c, du * du * du, sb);
    }
    return acc;
}

// NT lanes per workgroup; each lane owns up to KM 16-byte chunks of the
// level-0 frame (KM * NT >= (TY + 4) * nx / VEC, checked by the planner).
// OP = SOP_FWD: level 0 = u_t, point operand f at both levels, sums = the
//   norms of steps t+1 and t+2; MID also stores u_{t+1} on the owned points.
// OP = SOP_ADJ: level 0 = lambda_{t+1}, point operands u_t (level 1) and
//   u_{t-1} (level 2), sums = the parameter sums of steps t and t-1.
template <typename T, int VEC, int TY, int NT, int KM, int BC, int OP, bool RED, bool MID>
__global__ void __launch_bounds__(NT) tb2_kernel(TbArgs a) {
    constexpr int kTbThreads = NT;
    constexpr int kTbKmax = KM;
    constexpr bool ADJ = (OP == SOP_ADJ || OP == SOP_ADJL);
    constexpr bool LAM = (OP == SOP_ADJL);
    extern __shared__ __align__(16) unsigned char tb_smem[];
    constexpr int R0 = TY + 4;  // level-0 rows: global rows y0-2 .. y0+TY+1
    constexpr int R1 = TY + 2;  // level-1 rows: global rows y0-1 .. y0+TY
    const int nx = (int)a.nx, ny = (int)a.ny, nz = (int)a.nz;
    const int64_t sz = a.nx * a.ny;
    const int CH = nx / VEC;
    T *L0 = reinterpret_cast<T *>(tb_smem);
    // level-1 buffer b (0 or 1) starts R0 + b*R1 rows into the LDS area; an
    // offset from L0 (not a pointer picked from an array) keeps every access
    // an LDS instruction
    auto L1 = [&](int b) -> T * { return L0 + (R0 + (b & 1) * R1) * nx; };

    const int tid = threadIdx.x;
    const int L = tb_xcd_remap(blockIdx.x, gridDim.x);
    const int slab = L % a.nslab;
    const int zrun = L / a.nslab;
    const int y0 = slab * TY;
    const int z0 = zrun * a.zc;
    const int z1 = min(nz, z0 + a.zc);

    const T *__restrict__ U = static_cast<const T *>(a.u);
    const T *__restrict__ QA = static_cast<const T *>(a.f);   // level-1 point operand
    const T *__restrict__ QB = static_cast<const T *>(a.g2);  // level-2 point operand (adjoint)
    T *__restrict__ O = static_cast<T *>(a.out);
    T *__restrict__ M = static_cast<T *>(a.mid);
    const T C0 = (T)a.c0, C1 = (T)a.c1, C2 = (T)a.c2;

    // The lane's points: chunk k covers level-0 frame row r = idx / CH and
    // x = (idx % CH) * VEC.  lofs = r*nx + x (LDS offset in the level-0 frame,
    // the level-1 buffers use the same frame shifted down one row), gofs = the
    // global offset of (x, row) in a plane, or -1 for a ghost row.
    int lofs[kTbKmax];
    int gofs[kTbKmax];        // < nx*ny <= INT_MAX (checked by the planner)
    unsigned flags[kTbKmax];  // bit 0: valid, bit 1: level 1, bit 2: owned (level 2), x >> 3
#pragma unroll
    for (int k = 0; k < kTbKmax; ++k) {
        const int idx = tid + k * kTbThreads;
        const bool v = idx < R0 * CH;
        const int r = v ? idx / CH : 0;
        const int xo = v ? (idx % CH) * VEC : 0;
        const int gy = y0 - 2 + r;
        const int gyr = tb_wrap<BC>(gy, ny);
        lofs[k] = r * nx + xo;
        gofs[k] = gyr >= 0 ? gyr * nx + xo : -1;
        flags[k] = (v ? 1u : 0u) | ((v && r >= 1 && r <= TY + 2) ? 2u : 0u) |
                   ((v && r >= 2 && r <= TY + 1 && gy < ny) ? 4u : 0u) | ((unsigned)xo << 3);
    }

    auto load_u = [&](int zq, T (&d)[kTbKmax][VEC]) {
        const int zr = tb_wrap<BC>(zq, nz);
#pragma unroll
        for (int k = 0; k < kTbKmax; ++k) {
            if ((flags[k] & 1u) && gofs[k] >= 0 && zr >= 0)
                tb_load<T, VEC>(d[k], U + (int64_t)zr * sz + gofs[k]);
            else
                tb_zero<T, VEC>(d[k]);
        }
    };
    // point operand of level 1 on the level-1 rows, of level 2 on the owned rows
    auto load_qa = [&](int zq, T (&d)[kTbKmax][VEC]) {
        const int zr = tb_wrap<BC>(zq, nz);
#pragma unroll
        for (int k = 0; k < kTbKmax; ++k) {
            if ((flags[k] & 2u) && gofs[k] >= 0 && zr >= 0)
                tb_load_nt<T, VEC>(d[k], QA + (int64_t)zr * sz + gofs[k]);
            else
                tb_zero<T, VEC>(d[k]);
        }
    };
    auto load_qb = [&](int zq, T (&d)[kTbKmax][VEC]) {
#pragma unroll
        for (int k = 0; k < kTbKmax; ++k) {
            if ((flags[k] & 4u) && zq >= 0 && zq < nz)
                tb_load_nt<T, VEC>(d[k], QB + (int64_t)zq * sz + gofs[k]);
            else
                tb_zero<T, VEC>(d[k]);
        }
    };
    // x-neighbours of the chunk at LDS offset o (row start o - xo)
    auto xleft = [&](const T *base, int o, int xo) -> T {
        if (xo > 0) return base[o - 1];
        if constexpr (BC == 1) return base[o - xo + nx - 1];
        return T(0);
    };
    auto xright = [&](const T *base, int o, int xo) -> T {
        if (xo + VEC < nx) return base[o + VEC];
        if constexpr (BC == 1) return base[o - xo];
        return T(0);
    };
    // The neighbouring chunks of a row are held by the neighbouring lanes
    // (chunk idx - 1 by lane - 1, idx + 1 by lane + 1, in the same stage), so
    // the x-neighbours come across the wave; the first and last lane of a
    // wave and the chunks at a row's ends read them from LDS.
    const int wlane = tid & 63;
    auto xnbrs = [&](const T *base, int o, int xo, const T (&c)[VEC], T &lft, T &rgt) {
        const T fl = tb_dpp<0x138>(c[VEC - 1]);
        const T fu = tb_dpp<0x130>(c[0]);
        lft = (wlane != 0 && xo > 0) ? fl : xleft(base, o, xo);
        rgt = (wlane != 63 && xo + VEC < nx) ? fu : xright(base, o, xo);
    };

    // register queues: level 0 at q-1, q+1 and the prefetched q+2; level 1 at
    // q-2 and q; level-1 point operand at q and the prefetched q+1; level-2
    // point operand at q-1 (the forward's is the level-1 operand of the
    // previous plane; the adjoint's is loaded in the same iteration); the
    // centres live in LDS
    T am[kTbKmax][VEC], ap[kTbKmax][VEC], an[kTbKmax][VEC];
    T bm[kTbKmax][VEC], bn[kTbKmax][VEC];
    T qbm[kTbKmax][VEC], qac[kTbKmax][VEC], qan[kTbKmax][VEC];
    double e1 = 0.0, r1 = 0.0, e2 = 0.0, r2 = 0.0;

    T ac0[kTbKmax][VEC];  // level 0 at the first plane, written to LDS in the first iteration
    if (z0 < z1) {
        load_u(z0 - 2, am);
        load_u(z0 - 1, ac0);
        load_u(z0, ap);
        load_qa(z0 - 1, qac);
    }
#pragma unroll
    for (int k = 0; k < kTbKmax; ++k) {
        tb_zero<T, VEC>(bm[k]);
        tb_zero<T, VEC>(qbm[k]);
        if (flags[k] & 1u) tb_store<T, VEC>(L0 + lofs[k], ac0[k]);
    }

    for (int q = z0 - 1; z0 < z1 && q <= z1; ++q) {
        // LDS holds level 0 at plane q (written before the barrier); prefetch
        // level 0 at q+2 and the point operands
        const bool more = q < z1;
        if (more) {
            load_u(q + 2, an);
            load_qa(q + 1, qan);
        }
        // the adjoint's level-2 point operand, u_(t-1) at plane q-1, is loaded
        // here for stage B of this iteration (its latency hides behind stage
        // A) rather than an iteration ahead: one queue slot fewer, so the
        // 1024-lane build stays within 128 VGPRs
        if constexpr (ADJ) load_qb(q - 1, qbm);
        __syncthreads();

        // stage A: level 1 at plane q
        const int qr = tb_wrap<BC>(q, nz);
        const bool owned_plane = q >= z0 && q < z1;
        T *L1w = L1(q);
#pragma unroll
        for (int k = 0; k < kTbKmax; ++k) {
            if (!(flags[k] & 2u)) continue;
            const int o = lofs[k];
            const int xo = (int)(flags[k] >> 3);
            T c[VEC];
            tb_load<T, VEC>(c, L0 + o);
            const bool sum_here = (flags[k] & 4u) && owned_plane;
            if (BC == 0 && (qr < 0 || gofs[k] < 0)) {
                tb_zero<T, VEC>(bn[k]);
            } else {
                T ym[VEC], yp[VEC];
                tb_load<T, VEC>(ym, L0 + o - nx);
                tb_load<T, VEC>(yp, L0 + o + nx);
                T lft, rgt;
                xnbrs(L0, o, xo, c, lft, rgt);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T xm = e == 0 ? lft : c[e > 0 ? e - 1 : 0];
                    const T xp = e == VEC - 1 ? rgt : c[e + 1 < VEC ? e + 1 : e];
                    if constexpr (ADJ) {
                        bn[k][e] = tb_adj<T>(c[e], xm, xp, ym[e], yp[e], am[k][e], ap[k][e], qac[k][e], C0, C1,
                                             sum_here, e1, r1);
                    } else {
                        bn[k][e] = tb_fwd<T>(c[e], xm, xp, ym[e], yp[e], am[k][e], ap[k][e], qac[k][e], C0, C1,
                                             C2);
                    }
                }
            }
            tb_store<T, VEC>(L1w + o - nx, bn[k]);
            if constexpr (MID)
                if (sum_here) tb_store_nt<T, VEC>(M + (int64_t)q * sz + gofs[k], bn[k]);
            if constexpr (RED && !ADJ) {
                if (sum_here) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const double d = (double)bn[k][e];
                        e1 = fma(d, d, e1);
                        const double dd = d - (double)c[e];
                        r1 = fma(dd, dd, r1);
                    }
                }
            }
        }

        // stage B: level 2 at plane q-1, from level 1 at q-2, q-1, q
        if (q - 1 >= z0) {
            const T *L1r = L1(q - 1);
#pragma unroll
            for (int k = 0; k < kTbKmax; ++k) {
                if (!(flags[k] & 4u)) continue;
                const int o = lofs[k] - nx;  // level-1 buffer offset
                const int xo = (int)(flags[k] >> 3);
                T c[VEC], ym[VEC], yp[VEC], res[VEC];
                tb_load<T, VEC>(c, L1r + o);
                tb_load<T, VEC>(ym, L1r + o - nx);
                tb_load<T, VEC>(yp, L1r + o + nx);
                T lft, rgt;
                xnbrs(L1r, o, xo, c, lft, rgt);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T xm = e == 0 ? lft : c[e > 0 ? e - 1 : 0];
                    const T xp = e == VEC - 1 ? rgt : c[e + 1 < VEC ? e + 1 : e];
                    if constexpr (ADJ) {
                        res[e] = tb_adj<T>(c[e], xm, xp, ym[e], yp[e], bm[k][e], bn[k][e], qbm[k][e], C0, C1,
                                           true, e2, r2);
                    } else {
                        res[e] = tb_fwd<T>(c[e], xm, xp, ym[e], yp[e], bm[k][e], bn[k][e], qbm[k][e], C0, C1,
                                           C2);
                    }
                }
                tb_store_nt<T, VEC>(O + (int64_t)(q - 1) * sz + gofs[k], res);
                if constexpr (LAM) {
                    // running sum of the adjoint inputs, in step order:
                    // lam = (lam + lambda_{t+1}) + lambda_t (level 0 at q-1 is in am)
                    T *lp = static_cast<T *>(a.lam) + (int64_t)(q - 1) * sz + gofs[k];
                    T lv[VEC];
                    if (a.lam_first) tb_zero<T, VEC>(lv);
                    else tb_load_nt<T, VEC>(lv, lp);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) lv[e] = (lv[e] + am[k][e]) + c[e];
                    tb_store_nt<T, VEC>(lp, lv);
                }
                if constexpr (RED && !ADJ) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const double d = (double)res[e];
                        e2 = fma(d, d, e2);
                        const double dd = d - (double)c[e];
                        r2 = fma(dd, dd, r2);
                    }
                }
            }
        }

        // rotate: the centres of this iteration become the lower neighbours
        // (each lane reads back only its own points, which no other lane writes)
#pragma unroll
        for (int k = 0; k < kTbKmax; ++k) {
            if (flags[k] & 1u) tb_load<T, VEC>(am[k], L0 + lofs[k]);
            if (flags[k] & 2u) tb_load<T, VEC>(bm[k], L1(q - 1) + lofs[k] - nx);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kTbKmax; ++k) {
            if (flags[k] & 1u) tb_store<T, VEC>(L0 + lofs[k], ap[k]);  // level 0 at q+1
            tb_copy<T, VEC>(ap[k], an[k]);
            if constexpr (!ADJ) tb_copy<T, VEC>(qbm[k], qac[k]);
            tb_copy<T, VEC>(qac[k], qan[k]);
        }
    }

    if constexpr (RED) {
        // reuse the start of the LDS area for the cross-wave sums
        double *red = reinterpret_cast<double *>(tb_smem);
        const int lane = tid & 63, wave = tid >> 6;
        constexpr int NW = kTbThreads / 64;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            e1 += __shfl_xor(e1, off, 64);
            r1 += __shfl_xor(r1, off, 64);
            e2 += __shfl_xor(e2, off, 64);
            r2 += __shfl_xor(r2, off, 64);
        }
        __syncthreads();
        if (lane == 0) {
            red[4 * wave + 0] = e1;
            red[4 * wave + 1] = r1;
            red[4 * wave + 2] = e2;
            red[4 * wave + 3] = r2;
        }
        __syncthreads();
        if (tid == 0) {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            for (int w = 0; w < NW; ++w)
                for (int i = 0; i < 4; ++i) s[i] += red[4 * w + i];
            a.part1[2 * (int64_t)L] = s[0];
            a.part1[2 * (int64_t)L + 1] = s[1];
            a.part2[2 * (int64_t)L] = s[2];
            a.part2[2 * (int64_t)L + 1] = s[3];
        }
    }
}

template <typename T, int VEC, int TY, int NT, int KM>
hipError_t tb_launch_t(int op, int bc, bool reduce, bool mid, const TbTile &t, const TbArgs &a,
                       hipStream_t st) {
    const dim3 grid(t.nblk), block(NT);
    const size_t lds = t.lds_bytes;
#define DCP_TB(BCV, OPV, REDV, MIDV)                                                                  \
    do {                                                                                              \
        auto fn = tb2_kernel<T, VEC, TY, NT, KM, BCV, OPV, REDV, MIDV>;                               \
        hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),                       \
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);    \
        if (e_ != hipSuccess) return e_;                                                              \
        hipLaunchKernelGGL(fn, grid, block, lds, st, a);                                              \
    } while (0)
    if (op == SOP_ADJ) {
        if (bc == 0) DCP_TB(0, SOP_ADJ, true, false);
        else DCP_TB(1, SOP_ADJ, true, false);
    } else if (op == SOP_ADJL) {
        if (bc == 0) DCP_TB(0, SOP_ADJL, true, false);
        else DCP_TB(1, SOP_ADJL, true, false);
    } else if (mid) {
        if (bc == 0) {
            if (reduce) DCP_TB(0, SOP_FWD, true, true);
            else DCP_TB(0, SOP_FWD, false, true);
        } else {
            if (reduce) DCP_TB(1, SOP_FWD, true, true);
            else DCP_TB(1, SOP_FWD, false, true);
        }
    } else if (bc == 0) {
        if (reduce) DCP_TB(0, SOP_FWD, true, false);
        else DCP_TB(0, SOP_FWD, false, false);
    } else {
        if (reduce) DCP_TB(1, SOP_FWD, true, false);
        else DCP_TB(1, SOP_FWD, false, false);
    }
#undef DCP_TB
    return hipGetLastError();
}

// Compiled configurations (slab rows, lanes, chunks per lane), in order of
// preference: taller slabs recompute fewer halo rows.  1024 lanes with two
// chunks each (four waves per SIMD, up to 128 VGPRs; every forward and
// adjoint build stays out of scratch but the float periodic adjoint with the
// running sum, 8 bytes).  512 lanes with four chunks (two waves per SIMD)
// measured slower at 512^3: forward FP64 423 vs 455 GLUP/s, adjoint FP64
// 326 vs 352, FP32 612 vs 689.  8-row slabs fit rows of up to 170 chunks
// (FP32 nx <= 680), 4-row slabs up to 256 chunks (FP64 nx <= 512,
// FP32 nx <= 1024); the LDS budget is checked separately.
struct TbCfg {
    int ty, nt, km;
};
constexpr TbCfg kTbCfgs[] = {{8, 1024, 2}, {4, 1024, 2}};
constexpr int kNumTbCfgs = sizeof(kTbCfgs) / sizeof(kTbCfgs[0]);

}  // namespace

bool tb_plan(int dtype, int64_t nx, int64_t ny, int64_t nz, bool vec_ok, size_t lds_limit, TbTile *t) {
    const int esz = dtype == 0 ? 8 : 4;
    const int vec = 16 / esz;
    if (!vec_ok || nx <= 0 || ny <= 0 || nz <= 0 || nx % vec != 0) return false;
    if (nx > (1 << 24) || nx * ny > (int64_t)INT32_MAX || nz > (1 << 29) || ny > (1 << 29)) return false;
    const int64_t ch = nx / vec;
    const char *forced = tuning_env("DCP_TB_CFG");  // tuning runs only
    const int only = (forced && *forced) ? std::atoi(forced) : -1;
    for (int i = 0; i < kNumTbCfgs; ++i) {
        if (only >= 0 && i != only) continue;
        const TbCfg c = kTbCfgs[i];
        const size_t lds = (size_t)((c.ty + 4) + 2 * (c.ty + 2)) * (size_t)nx * esz;
        if ((c.ty + 4) * ch > (int64_t)c.km * c.nt) continue;
        if (lds > lds_limit) continue;
        if (lds < (size_t)(c.nt / 64) * 4 * sizeof(double)) continue;
        const int64_t nslab = (ny + c.ty - 1) / c.ty;
        if (nslab > 65536) return false;
        // one workgroup per CU: 256 workgroups in all
        int64_t runs = 256 / nslab;
        if (runs < 1) runs = 1;
        if (runs > nz) runs = nz;
        int64_t zc = (nz + runs - 1) / runs;
        runs = (nz + zc - 1) / zc;
        t->vec = vec;
        t->ty = c.ty;
        t->nt = c.nt;
        t->km = c.km;
        t->zc = (int)zc;
        t->nslab = (int)nslab;
        t->nruns = (int)runs;
        t->nblk = (int)(nslab * runs);
        t->lds_bytes = lds;
        return true;
    }
    return false;
}

hipError_t launch_tb2(int dtype, int op, int bc, bool reduce, const TbTile &t, const TbArgs &a, hipStream_t st) {
    const bool mid = op == SOP_FWD && a.mid != nullptr;
    if (t.nt != 1024 || t.km != 2) return hipErrorInvalidValue;
    if (dtype == 0) {
        if (t.ty == 8) return tb_launch_t<double, 2, 8, 1024, 2>(op, bc, reduce, mid, t, a, st);
        return tb_launch_t<double, 2, 4, 1024, 2>(op, bc, reduce, mid, t, a, st);
    }
    if (t.ty == 8) return tb_launch_t<float, 4, 8, 1024, 2>(op, bc, reduce, mid, t, a, st);
    return tb_launch_t<float, 4, 4, 1024, 2>(op, bc, reduce, mid, t, a, st);
}

}  // namespace dcp
