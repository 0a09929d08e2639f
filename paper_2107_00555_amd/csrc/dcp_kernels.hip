// dcp_kernels.hip -- gfx950 kernels of the reaction-diffusion program.
//
// The hot kernel is a z-marching 7-point stencil with the whole point-wise
// expression fused into it (Sec. 3.1: greedy subgraph fusion of maps over
// one iteration space, no transient arrays).  The same kernel, with a
// different point-wise body, applies the adjoint step and, for the unfused
// program of Sec. 2.3, the bare Laplacian statement.
//
// Memory plan (x contiguous, element (x,y,z) at x + nx*(y + ny*z)):
//   * a workgroup owns a tile of 64*BXW*VEC points along x, BY*RY rows along
//     y and zc planes along z, and marches up z through it;
//   * each lane owns VEC consecutive x points (one 16-byte load) in RY
//     consecutive rows; the planes z-1, z, z+1 of those rows sit in
//     registers and move down one slot per step (a register queue), so each
//     plane of the stencil operand is read from memory once per tile;
//   * y-neighbours come from the lane's own rows, except the row above and
//     the row below the lane's rows (two extra row loads per plane, mostly
//     served by L2 because the neighbouring tile reads the same rows);
//   * x-neighbours come from the adjacent lane through a cross-lane
//     permute; only lanes at a wave edge or at the domain edge load one
//     extra element;
//   * the next plane (stencil operand, point operand, halos) is loaded one
//     iteration ahead so its latency overlaps the current plane's work;
//   * workgroups are numbered so that the tiles one XCD runs at a time are
//     neighbours in space (the hardware deals workgroups round-robin to the
//     8 XCDs, each with its own L2), so halo rows hit in that XCD's L2.
// Reductions (norms, gradient sums) are accumulated per lane in double
// (each term added with one fused multiply-add), combined by a fixed
// butterfly within the wave and a fixed order across
// waves, and written as one pair per workgroup; a second kernel adds the
// per-workgroup pairs in a fixed order.  Results are therefore identical
// from run to run (the tiled write-conflict reduction of Sec. 3.1, made
// deterministic).
//
// All code is compiled with -ffp-contract=off; every fused multiply-add is
// written out with fma(), so the arithmetic of a point is the same in every
// instantiation of the kernel.
#include "dcp_internal.h"

namespace dcp {
namespace {

template <typename T, int N>
struct VecT {
    typedef T type __attribute__((ext_vector_type(N)));
};

template <typename T, int VEC>
__device__ __forceinline__ void load_vec(T (&d)[VEC], const T *p) {
    if constexpr (VEC == 1) {
        d[0] = *p;
    } else {
        typedef typename VecT<T, VEC>::type V;
        V v = *reinterpret_cast<const V *>(p);
#pragma unroll
        for (int i = 0; i < VEC; ++i) d[i] = v[i];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec(T *p, const T (&s)[VEC]) {
    if constexpr (VEC == 1) {
        *p = s[0];
    } else {
        typedef typename VecT<T, VEC>::type V;
        V v;
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[i] = s[i];
        *reinterpret_cast<V *>(p) = v;
    }
}

// Non-temporal forms, for data that each launch reads or writes once (the
// point operand, the result, element-wise operands): the loads and stores
// carry the streaming hint, so they do not displace the stencil operand's
// rows, which neighbouring tiles read again through L2.
template <typename T, int VEC>
__device__ __forceinline__ void load_vec_nt(T (&d)[VEC], const T *p) {
    if constexpr (VEC == 1) {
        d[0] = __builtin_nontemporal_load(p);
    } else {
        typedef typename VecT<T, VEC>::type V;
        V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
        for (int i = 0; i < VEC; ++i) d[i] = v[i];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec_nt(T *p, const T (&s)[VEC]) {
    if constexpr (VEC == 1) {
        __builtin_nontemporal_store(s[0], p);
    } else {
        typedef typename VecT<T, VEC>::type V;
        V v;
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[i] = s[i];
        __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void zero_vec(T (&d)[VEC]) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) d[i] = T(0);
}

// Neighbour coordinate i in [-1, n] mapped under the boundary rule;
// -1 means "ghost cell, reads as zero".
template <int BC>
__device__ __forceinline__ int64_t wrap(int64_t i, int64_t n) {
    if (i >= 0 && i < n) return i;
    if constexpr (BC == 1) return i < 0 ? i + n : i - n;
    return -1;
}

// Hardware block b runs on XCD b % 8.  Renumber so that XCD k gets a
// contiguous run of logical tiles, taken in dispatch order.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, j = b >> 3;
    return xcd * per + min(xcd, rem) + j;
}

template <typename T, int VEC, int BXW, int BY, int RY, int BC, int OP, bool RED>
__global__ void __launch_bounds__(64 * BXW * BY) stencil_kernel(StencilArgs a) {
    constexpr int NW = BXW * BY;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wx = wave % BXW;
    const int wy = wave / BXW;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = L % a.tiles_x;
    const int tyz = L / a.tiles_x;
    const int ty = tyz % a.tiles_y;
    const int tz = tyz / a.tiles_y;

    const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t sy = nx, sz = nx * ny;
    const int64_t x0 = ((int64_t)tx * (64 * BXW) + wx * 64 + lane) * VEC;
    const bool xok = x0 < nx;
    const int64_t yf = ((int64_t)ty * BY + wy) * RY;
    const int nrow = (int)max((int64_t)0, min((int64_t)RY, ny - yf));
    const bool active = xok && nrow > 0;
    const int64_t z0 = (int64_t)tz * a.zc;
    const int64_t z1 = min(nz, z0 + (int64_t)a.zc);

    constexpr bool RECOMP = OP == SOP_ADJR || OP == SOP_ADJLR;  // u_t recomputed from u_{t-1}
    constexpr bool LSUM = OP == SOP_ADJL || OP == SOP_ADJLR;    // lam += lambda_{t+1}
    const T *__restrict__ S = static_cast<const T *>(a.s);
    const T *__restrict__ V = static_cast<const T *>(a.s2);
    const T *__restrict__ Q = static_cast<const T *>(a.q);
    T *__restrict__ O = static_cast<T *>(a.out);

    const int64_t ytop = wrap<BC>(yf - 1, ny);
    const int64_t ybot = wrap<BC>(yf + nrow, ny);
    const bool need_l = xok && (lane == 0 || x0 == 0);
    const bool need_r = xok && (lane == 63 || x0 + VEC >= nx);
    const int64_t xl = wrap<BC>(x0 - 1, nx);
    const int64_t xr = wrap<BC>(x0 + VEC, nx);

    const T C0 = (T)a.c0, C1 = (T)a.c1, C2 = (T)a.c2;
    const T C1F = (T)a.c1f, C2F = (T)a.c2f;

    // loaders for a resolved plane index zr (-1 = ghost plane) of a stencil
    // operand P (S, or V)
    auto load_rows_of = [&](const T *P, int64_t zr, T (&d)[RY][VEC]) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (active && zr >= 0 && r < nrow)
                load_vec<T, VEC>(d[r], P + zr * sz + (yf + r) * sy + x0);
            else
                zero_vec<T, VEC>(d[r]);
        }
    };
    auto load_rows = [&](int64_t zr, T (&d)[RY][VEC]) { load_rows_of(S, zr, d); };
    auto load_point = [&](int64_t z, T (&d)[RY][VEC]) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (active && r < nrow)
                load_vec_nt<T, VEC>(d[r], Q + z * sz + (yf + r) * sy + x0);
            else
                zero_vec<T, VEC>(d[r]);
        }
    };
    auto load_halo_of = [&](const T *P, int64_t z, T (&ht)[VEC], T (&hb)[VEC], T (&el)[RY], T (&er)[RY]) {
        if (active && ytop >= 0)
            load_vec<T, VEC>(ht, P + z * sz + ytop * sy + x0);
        else
            zero_vec<T, VEC>(ht);
        if (active && ybot >= 0)
            load_vec<T, VEC>(hb, P + z * sz + ybot * sy + x0);
        else
            zero_vec<T, VEC>(hb);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            el[r] = (need_l && xl >= 0 && r < nrow) ? P[z * sz + (yf + r) * sy + xl] : T(0);
            er[r] = (need_r && xr >= 0 && r < nrow) ? P[z * sz + (yf + r) * sy + xr] : T(0);
        }
    };
    auto load_halo = [&](int64_t z, T (&ht)[VEC], T (&hb)[VEC], T (&el)[RY], T (&er)[RY]) {
        load_halo_of(S, z, ht, hb, el, er);
    };

    T um[RY][VEC], uc[RY][VEC], up[RY][VEC], qc[RY][VEC];
    T ht[VEC], hb[VEC], el[RY], er[RY];
    // the recomputation's stencil operand u_{t-1} (RECOMP only; otherwise unused)
    T vm[RY][VEC], vc[RY][VEC], vp[RY][VEC];
    T vht[VEC], vhb[VEC], vel[RY], ver[RY];
    double acc0 = 0.0, acc1 = 0.0;

    if (z0 < z1) {
        load_rows(wrap<BC>(z0 - 1, nz), um);
        load_rows(z0, uc);
        load_halo(z0, ht, hb, el, er);
        if constexpr (OP != SOP_LAP) load_point(z0, qc);
        load_rows(wrap<BC>(z0 + 1, nz), up);
        if constexpr (RECOMP) {
            load_rows_of(V, wrap<BC>(z0 - 1, nz), vm);
            load_rows_of(V, z0, vc);
            load_halo_of(V, z0, vht, vhb, vel, ver);
            load_rows_of(V, wrap<BC>(z0 + 1, nz), vp);
        }
    }

    for (int64_t z = z0; z < z1; ++z) {
        T un[RY][VEC], qn[RY][VEC], htn[VEC], hbn[VEC], eln[RY], ern[RY];
        T vn[RY][VEC], vhtn[VEC], vhbn[VEC], veln[RY], vern[RY];
        const bool more = z + 1 < z1;
        if (more) {
            load_rows(wrap<BC>(z + 2, nz), un);
            if constexpr (OP != SOP_LAP) load_point(z + 1, qn);
            load_halo(z + 1, htn, hbn, eln, ern);
            if constexpr (RECOMP) {
                load_rows_of(V, wrap<BC>(z + 2, nz), vn);
                load_halo_of(V, z + 1, vhtn, vhbn, veln, vern);
            }
        }

        // x-neighbours of each row's first and last element
        T lft[RY], rgt[RY], vlft[RY], vrgt[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            lft[r] = __shfl_up(uc[r][VEC - 1], 1, 64);
            rgt[r] = __shfl_down(uc[r][0], 1, 64);
            if (need_l) lft[r] = el[r];
            if (need_r) rgt[r] = er[r];
            if constexpr (RECOMP) {
                vlft[r] = __shfl_up(vc[r][VEC - 1], 1, 64);
                vrgt[r] = __shfl_down(vc[r][0], 1, 64);
                if (need_l) vlft[r] = vel[r];
                if (need_r) vrgt[r] = ver[r];
            }
        }

        if (active) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                if (r < nrow) {
                    T res[VEC];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const T c = uc[r][e];
                        const T xm = e == 0 ? lft[r] : uc[r][e > 0 ? e - 1 : 0];
                        const T xp = e == VEC - 1 ? rgt[r] : uc[r][e + 1 < VEC ? e + 1 : e];
                        const T ym = r == 0 ? ht[e] : uc[r > 0 ? r - 1 : 0][e];
                        const T yp = (r == nrow - 1) ? hb[e] : uc[r + 1 < RY ? r + 1 : r][e];
                        const T zm = um[r][e], zp = up[r][e];
                        if constexpr (OP == SOP_LAP) {
                            T s = xm + xp;
                            s = s + ym;
                            s = s + yp;
                            s = s + zm;
                            s = s + zp;
                            const T six = T(6) * c;
                            res[e] = (s - six) / C0;
                        } else {
                            const T s6 = ((xm + xp) + (ym + yp)) + (zm + zp);
                            const T lapn = fma(T(-6), c, s6);  // h^2 * Lap7 at this point
                            T qv = qc[r][e];
                            if constexpr (RECOMP) {
                                // u_t = u_{t-1} + c0*(S6 - 6u) - c1f*u^3 + c2f*f, as SOP_FWD
                                const T v = vc[r][e];
                                const T vxm = e == 0 ? vlft[r] : vc[r][e > 0 ? e - 1 : 0];
                                const T vxp = e == VEC - 1 ? vrgt[r] : vc[r][e + 1 < VEC ? e + 1 : e];
                                const T vym = r == 0 ? vht[e] : vc[r > 0 ? r - 1 : 0][e];
                                const T vyp = (r == nrow - 1) ? vhb[e] : vc[r + 1 < RY ? r + 1 : r][e];
                                const T vs6 = ((vxm + vxp) + (vym + vyp)) + (vm[r][e] + vp[r][e]);
                                const T vlap = fma(T(-6), v, vs6);
                                T ut = fma(C2F, qv, v);
                                ut = fma(C0, vlap, ut);
                                ut = fma(-(C1F * v) * v, v, ut);
                                qv = ut;
                            }
                            if constexpr (OP == SOP_FWD) {
                                T acc = fma(C2, qv, c);
                                acc = fma(C0, lapn, acc);
                                acc = fma(-(C1 * c) * c, c, acc);
                                res[e] = acc;
                                if constexpr (RED) {
                                    const double d = (double)acc;
                                    acc0 = fma(d, d, acc0);
                                    const double dd = d - (double)c;
                                    acc1 = fma(dd, dd, acc1);
                                }
                            } else {  // the adjoint ops: c = lambda_{t+1}, qv = u_t
                                T acc = fma(C0, lapn, c);
                                acc = fma(-(C1 * qv) * qv, c, acc);
                                res[e] = acc;
                                if constexpr (RED) {
                                    const double du = (double)qv;
                                    acc0 = fma((double)lapn, du, acc0);
                                    acc1 = fma((double)c, du * du * du, acc1);
                                }
                            }
                        }
                    }
                    store_vec_nt<T, VEC>(O + z * sz + (yf + r) * sy + x0, res);
                    if constexpr (LSUM) {
                        // running sum of the adjoint inputs: lam += lambda_{t+1}
                        T *lp = static_cast<T *>(a.lam) + z * sz + (yf + r) * sy + x0;
                        T lv[VEC];
                        if (a.lam_first) zero_vec<T, VEC>(lv);
                        else load_vec_nt<T, VEC>(lv, lp);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) lv[e] = lv[e] + uc[r][e];
                        store_vec_nt<T, VEC>(lp, lv);
                    }
                }
            }
        }

        if (more) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    um[r][e] = uc[r][e];
                    uc[r][e] = up[r][e];
                    up[r][e] = un[r][e];
                    if constexpr (OP != SOP_LAP) qc[r][e] = qn[r][e];
                    if constexpr (RECOMP) {
                        vm[r][e] = vc[r][e];
                        vc[r][e] = vp[r][e];
                        vp[r][e] = vn[r][e];
                    }
                }
                el[r] = eln[r];
                er[r] = ern[r];
                if constexpr (RECOMP) {
                    vel[r] = veln[r];
                    ver[r] = vern[r];
                }
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                ht[e] = htn[e];
                hb[e] = hbn[e];
                if constexpr (RECOMP) {
                    vht[e] = vhtn[e];
                    vhb[e] = vhbn[e];
                }
            }
        }
    }

    if constexpr (RED) {
        __shared__ double red[2][NW];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            acc0 += __shfl_xor(acc0, off, 64);
            acc1 += __shfl_xor(acc1, off, 64);
        }
        if (lane == 0) {
            red[0][wave] = acc0;
            red[1][wave] = acc1;
        }
        __syncthreads();
        if (tid == 0) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                s0 += red[0][w];
                s1 += red[1][w];
            }
            a.partials[2 * (int64_t)L] = s0;
            a.partials[2 * (int64_t)L + 1] = s1;
        }
    }
}

// ----------------------------------------------------------------- dispatch
constexpr Shape kShapes[] = {
    {1, 4, 4},  // 256 threads, tile 64*vec x 16
    {1, 4, 2},  // 256 threads, tile 64*vec x 8
    {2, 2, 4},  // 256 threads, tile 128*vec x 8
    {1, 8, 2},  // 512 threads, tile 64*vec x 16
    {1, 2, 8},  // 128 threads, tile 64*vec x 16
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

template <typename T, int VEC, int BXW, int BY, int RY>
hipError_t launch_shape(int op, int bc, bool reduce, int nblk, const StencilArgs &a,
                        hipStream_t st) {
    const dim3 grid(nblk), block(64 * BXW * BY);
#define DCP_L(BCV, OPV, REDV) \
    hipLaunchKernelGGL((stencil_kernel<T, VEC, BXW, BY, RY, BCV, OPV, REDV>), grid, block, 0, st, a)
    if (bc == 0) {
        if (op == SOP_FWD) {
            if (reduce) DCP_L(0, SOP_FWD, true);
            else DCP_L(0, SOP_FWD, false);
        } else if (op == SOP_ADJ) {
            DCP_L(0, SOP_ADJ, true);
        } else if (op == SOP_ADJL) {
            DCP_L(0, SOP_ADJL, true);
        } else if (op == SOP_ADJR) {
            DCP_L(0, SOP_ADJR, true);
        } else if (op == SOP_ADJLR) {
            DCP_L(0, SOP_ADJLR, true);
        } else {
            DCP_L(0, SOP_LAP, false);
        }
    } else {
        if (op == SOP_FWD) {
            if (reduce) DCP_L(1, SOP_FWD, true);
            else DCP_L(1, SOP_FWD, false);
        } else if (op == SOP_ADJ) {
            DCP_L(1, SOP_ADJ, true);
        } else if (op == SOP_ADJL) {
            DCP_L(1, SOP_ADJL, true);
        } else if (op == SOP_ADJR) {
            DCP_L(1, SOP_ADJR, true);
        } else if (op == SOP_ADJLR) {
            DCP_L(1, SOP_ADJLR, true);
        } else {
            DCP_L(1, SOP_LAP, false);
        }
    }
#undef DCP_L
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t launch_vec(int shape, int op, int bc, bool reduce, int nblk, const StencilArgs &a,
                      hipStream_t st) {
    switch (shape) {
        case 0: return launch_shape<T, VEC, 1, 4, 4>(op, bc, reduce, nblk, a, st);
        case 1: return launch_shape<T, VEC, 1, 4, 2>(op, bc, reduce, nblk, a, st);
        case 2: return launch_shape<T, VEC, 2, 2, 4>(op, bc, reduce, nblk, a, st);
        case 3: return launch_shape<T, VEC, 1, 8, 2>(op, bc, reduce, nblk, a, st);
        case 4: return launch_shape<T, VEC, 1, 2, 8>(op, bc, reduce, nblk, a, st);
        default: return hipErrorInvalidValue;
    }
}

int shape_index(const Tile &t) {
    for (int i = 0; i < kNumShapes; ++i)
        if (kShapes[i].bxw == t.bxw && kShapes[i].by == t.by && kShapes[i].ry == t.ry) return i;
    return -1;
}

// ------------------------------------------------------ element-wise kernels
template <typename T, int VEC, int OPC>
__device__ __forceinline__ void ew_apply(T (&o)[VEC], const T (&x)[VEC], const T (&y)[VEC], T a) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
        if constexpr (OPC == EW_POW3) o[i] = (x[i] * x[i]) * x[i];
        else if constexpr (OPC == EW_SCALE) o[i] = a * x[i];
        else if constexpr (OPC == EW_SUB) o[i] = x[i] - y[i];
        else if constexpr (OPC == EW_ADD) o[i] = x[i] + y[i];
        else if constexpr (OPC == EW_ZERO) o[i] = T(0);
        else o[i] = x[i];
    }
}

// Element-wise statement over n elements.  Workgroup b streams the
// contiguous vectors [b*per, min(nv, (b+1)*per)), four 16-byte vectors in
// flight per lane (contiguous chunks stream faster than a grid-stride walk).
template <typename T, int VEC, int OPC>
__global__ void __launch_bounds__(256)
    ew_kernel(const T *__restrict__ x, const T *__restrict__ y, T *__restrict__ o, T a, int64_t n, int64_t per) {
    constexpr bool BIN = (OPC == EW_SUB || OPC == EW_ADD);
    constexpr int U = 4;
    const int64_t nv = n / VEC;
    const int64_t beg = (int64_t)blockIdx.x * per;
    const int64_t end = min(nv, beg + per);
    for (int64_t j = beg + threadIdx.x; j < end; j += 256 * U) {
        T xv[U][VEC], yv[U][VEC], ov[U][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = j + u * 256;
            if (i < end) {
                if constexpr (OPC != EW_ZERO) load_vec_nt<T, VEC>(xv[u], x + i * VEC);
                else zero_vec<T, VEC>(xv[u]);
                if constexpr (BIN) load_vec_nt<T, VEC>(yv[u], y + i * VEC);
                else zero_vec<T, VEC>(yv[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = j + u * 256;
            if (i < end) {
                ew_apply<T, VEC, OPC>(ov[u], xv[u], yv[u], a);
                store_vec_nt<T, VEC>(o + i * VEC, ov[u]);
            }
        }
    }
    if (blockIdx.x == 0) {
        const int64_t t = nv * VEC + threadIdx.x;
        if (t < n) {
            T xs[1] = {OPC == EW_ZERO ? T(0) : x[t]}, ys[1] = {BIN ? y[t] : T(0)}, os[1];
            ew_apply<T, 1, OPC>(os, xs, ys, a);
            o[t] = os[0];
        }
    }
}

__device__ __forceinline__ void block_sum2_256(double &a0, double &a1, double (*red)[4]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off, 64);
        a1 += __shfl_xor(a1, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = a0;
        red[1][w] = a1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a0 = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        a1 = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

// DOT = false: {sum o^2, sum (o - u)^2};  DOT = true: {sum o*u, 0}.
template <typename T, int VEC, bool DOT>
__global__ void __launch_bounds__(256)
    ew_norms_kernel(const T *__restrict__ o, const T *__restrict__ u, double *__restrict__ partials,
                    int64_t n) {
    __shared__ double red[2][4];
    const int64_t nv = n / VEC;
    const int64_t stride = (int64_t)gridDim.x * 256;
    double a0 = 0.0, a1 = 0.0;
    auto term = [&](T ov, T uv) {
        const double d = (double)ov;
        if constexpr (DOT) {
            a0 += d * (double)uv;
        } else {
            a0 += d * d;
            const double dd = d - (double)uv;
            a1 += dd * dd;
        }
    };
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += stride) {
        T ov[VEC], uv[VEC];
        load_vec_nt<T, VEC>(ov, o + i * VEC);
        load_vec_nt<T, VEC>(uv, u + i * VEC);
#pragma unroll
        for (int e = 0; e < VEC; ++e) term(ov[e], uv[e]);
    }
    const int64_t t = nv * VEC + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) term(o[t], u[t]);
    block_sum2_256(a0, a1, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = a0;
        partials[2 * blockIdx.x + 1] = a1;
    }
}

__global__ void __launch_bounds__(256)
    finalize_kernel(const double *__restrict__ partials, int nblk, int stride, double *out0, double *out1,
                    int mode) {
    __shared__ double red[2][4];
    const int s = blockIdx.x;
    const double *p = partials + (int64_t)s * stride * 2;
    double a0 = 0.0, a1 = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) {
        a0 += p[2 * i];
        a1 += p[2 * i + 1];
    }
    block_sum2_256(a0, a1, red);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            out0[0] = a0;
            out0[1] = a1;
        } else if (mode == 1) {
            if (out0) out0[s] = a0;
            if (out1) out1[s] = sqrt(a1);
        } else {
            out0[2 * s] = a0;
            out0[2 * s + 1] = a1;
        }
    }
}

// Compensated (Neumaier) sum over the steps, one thread, ascending t.
__global__ void grad_finalize_kernel(const double *__restrict__ sums, int nsteps, double s0, double s1,
                                     double *grad) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double sa = 0.0, ca = 0.0, sb = 0.0, cb = 0.0;
    for (int t = 0; t < nsteps; ++t) {
        const double va = sums[2 * t], vb = sums[2 * t + 1];
        double ta = sa + va;
        ca += fabs(sa) >= fabs(va) ? (sa - ta) + va : (va - ta) + sa;
        sa = ta;
        double tb = sb + vb;
        cb += fabs(sb) >= fabs(vb) ? (sb - tb) + vb : (vb - tb) + sb;
        sb = tb;
    }
    grad[0] = s0 * (sa + ca);
    grad[1] = s1 * (sb + cb);
}

__global__ void scalar_scale_kernel(const double *src, double s, double *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = s * src[0];
}

__global__ void zero_kernel(double *dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = 0.0;
}

template <typename T>
hipError_t launch_ew_t(int op, const void *x, const void *y, void *o, double a, int64_t n, bool vec_ok,
                       hipStream_t st) {
    constexpr int W = 16 / sizeof(T);
    const int vec = vec_ok ? W : 1;
    const int64_t nv = n / vec;
    // about eight workgroups per CU, each a contiguous run of 1024-vector strips
    const int64_t strip = 256 * 4;
    int64_t per = (nv + 2047) / 2048;
    per = (per + strip - 1) / strip * strip;
    if (per < strip) per = strip;
    int64_t blocks = (nv + per - 1) / per;
    if (blocks < 1) blocks = 1;
    const T *X = static_cast<const T *>(x);
    const T *Y = static_cast<const T *>(y);
    T *O = static_cast<T *>(o);
    const T A = (T)a;
#define DCP_EW(V, OPC) \
    hipLaunchKernelGGL((ew_kernel<T, V, OPC>), dim3(blocks), dim3(256), 0, st, X, Y, O, A, n, per)
    if (vec_ok) {
        switch (op) {
            case EW_POW3: DCP_EW(W, EW_POW3); break;
            case EW_SCALE: DCP_EW(W, EW_SCALE); break;
            case EW_SUB: DCP_EW(W, EW_SUB); break;
            case EW_ADD: DCP_EW(W, EW_ADD); break;
            case EW_ZERO: DCP_EW(W, EW_ZERO); break;
            default: DCP_EW(W, EW_COPY); break;
        }
    } else {
        switch (op) {
            case EW_POW3: DCP_EW(1, EW_POW3); break;
            case EW_SCALE: DCP_EW(1, EW_SCALE); break;
            case EW_SUB: DCP_EW(1, EW_SUB); break;
            case EW_ADD: DCP_EW(1, EW_ADD); break;
            case EW_ZERO: DCP_EW(1, EW_ZERO); break;
            default: DCP_EW(1, EW_COPY); break;
        }
    }
#undef DCP_EW
    return hipGetLastError();
}

}  // namespace

int num_shapes() { return kNumShapes; }
Shape shape_at(int i) { return kShapes[i]; }

hipError_t launch_stencil(int dtype, int op, int bc, bool reduce, const Tile &t, const StencilArgs &a,
                          hipStream_t st) {
    const int shape = shape_index(t);
    if (shape < 0 || t.nblk <= 0) return hipErrorInvalidValue;
    if (dtype == 0) {
        if (t.vec == 2) return launch_vec<double, 2>(shape, op, bc, reduce, t.nblk, a, st);
        if (t.vec == 1) return launch_vec<double, 1>(shape, op, bc, reduce, t.nblk, a, st);
    } else {
        if (t.vec == 4) return launch_vec<float, 4>(shape, op, bc, reduce, t.nblk, a, st);
        if (t.vec == 1) return launch_vec<float, 1>(shape, op, bc, reduce, t.nblk, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ew(int dtype, int op, const void *x, const void *y, void *o, double a, int64_t n,
                     bool vec_ok, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    return dtype == 0 ? launch_ew_t<double>(op, x, y, o, a, n, vec_ok, st)
                      : launch_ew_t<float>(op, x, y, o, a, n, vec_ok, st);
}

int ew_norm_blocks(int64_t n) {
    int64_t b = (n + 256 * 8 - 1) / (256 * 8);
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int)b;
}

template <bool DOT>
hipError_t launch_ew_red(int dtype, const void *o, const void *u, double *partials, int64_t n, bool vec_ok,
                         hipStream_t st) {
    const int nb = ew_norm_blocks(n);
    if (dtype == 0) {
        const double *O = static_cast<const double *>(o), *U = static_cast<const double *>(u);
        if (vec_ok)
            hipLaunchKernelGGL((ew_norms_kernel<double, 2, DOT>), dim3(nb), dim3(256), 0, st, O, U, partials, n);
        else
            hipLaunchKernelGGL((ew_norms_kernel<double, 1, DOT>), dim3(nb), dim3(256), 0, st, O, U, partials, n);
    } else {
        const float *O = static_cast<const float *>(o), *U = static_cast<const float *>(u);
        if (vec_ok)
            hipLaunchKernelGGL((ew_norms_kernel<float, 4, DOT>), dim3(nb), dim3(256), 0, st, O, U, partials, n);
        else
            hipLaunchKernelGGL((ew_norms_kernel<float, 1, DOT>), dim3(nb), dim3(256), 0, st, O, U, partials, n);
    }
    return hipGetLastError();
}

hipError_t launch_ew_norms(int dtype, const void *o, const void *u, double *partials, int64_t n,
                           bool vec_ok, hipStream_t st) {
    return launch_ew_red<false>(dtype, o, u, partials, n, vec_ok, st);
}

hipError_t launch_ew_dot(int dtype, const void *a, const void *b, double *partials, int64_t n, bool vec_ok,
                         hipStream_t st) {
    return launch_ew_red<true>(dtype, a, b, partials, n, vec_ok, st);
}

hipError_t launch_scalar_scale(const double *src, double s, double *dst, hipStream_t st) {
    hipLaunchKernelGGL(scalar_scale_kernel, dim3(1), dim3(64), 0, st, src, s, dst);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nblk, int stride, int nsteps, double *out0, double *out1,
                           int mode, hipStream_t st) {
    if (nsteps <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(nsteps), dim3(256), 0, st, partials, nblk, stride, out0, out1, mode);
    return hipGetLastError();
}

hipError_t launch_grad_finalize(const double *sums, int nsteps, double s0, double s1, double *grad,
                                hipStream_t st) {
    hipLaunchKernelGGL(grad_finalize_kernel, dim3(1), dim3(64), 0, st, sums, nsteps, s0, s1, grad);
    return hipGetLastError();
}

hipError_t launch_zero(double *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, dst, n);
    return hipGetLastError();
}

}  // namespace dcp
