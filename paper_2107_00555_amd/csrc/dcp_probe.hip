// dcp_probe.hip -- streaming kernels that measure what HBM bandwidth a plain
// streaming kernel reaches on this GPU (the practical ceiling the stencil
// kernels are compared with).  Not part of the reaction-diffusion program.
//
// Each kernel walks its buffers in 16-byte vectors with a grid-stride loop
// (65536 workgroups of 1024 lanes); `nt` selects loads and stores with the
// streaming (non-temporal) hint, the form the stencil kernels use for data
// they touch once.
#include <hip/hip_runtime.h>

#include "dcp.h"

namespace {

typedef double probe_v2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ probe_v2 pload(const probe_v2 *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void pstore(probe_v2 *p, probe_v2 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// kind 0: out = a; 1: out = a + b; 2: read a (one flag written per
// workgroup only if a value never produced by the generator appears); 3: out = c
template <int KIND, bool NT>
__global__ void __launch_bounds__(1024)
    probe_kernel(const probe_v2 *__restrict__ a, const probe_v2 *__restrict__ b, probe_v2 *__restrict__ o,
                 int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    probe_v2 acc = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if constexpr (KIND == 0) pstore<NT>(o + i, pload<NT>(a + i));
        else if constexpr (KIND == 1) pstore<NT>(o + i, pload<NT>(a + i) + pload<NT>(b + i));
        else if constexpr (KIND == 2) acc += pload<NT>(a + i);
        else pstore<NT>(o + i, probe_v2{1.0, 2.0});
    }
    if constexpr (KIND == 2) {
        // keeps the loads; the condition never holds for finite inputs
        if (acc.x != acc.x && threadIdx.x == 0) o[blockIdx.x] = acc;
    }
}

template <int KIND>
hipError_t probe_launch(bool nt, const void *a, const void *b, void *o, int64_t n, hipStream_t st) {
    const dim3 grid(65536), block(1024);
    const auto *A = static_cast<const probe_v2 *>(a);
    const auto *Bp = static_cast<const probe_v2 *>(b);
    auto *O = static_cast<probe_v2 *>(o);
    if (nt) hipLaunchKernelGGL((probe_kernel<KIND, true>), grid, block, 0, st, A, Bp, O, n);
    else hipLaunchKernelGGL((probe_kernel<KIND, false>), grid, block, 0, st, A, Bp, O, n);
    return hipGetLastError();
}

}  // namespace

extern "C" int dcp_stream_probe(int kind, int nt, const void *a, const void *b, void *out, size_t bytes,
                                void *stream) {
    if (kind < 0 || kind > 3 || bytes == 0 || bytes % 16 != 0) return DCP_E_ARG;
    const bool need_a = kind <= 2, need_b = kind == 1, need_o = kind != 2;
    if ((need_a && !a) || (need_b && !b) || !out) return DCP_E_NULL;
    const uintptr_t mis = (uintptr_t)a | (uintptr_t)b | (uintptr_t)out;
    if (mis & 15u) return DCP_E_ARG;
    if (kind == 2 && bytes / 16 < 65536) return DCP_E_ARG;  // one flag slot per workgroup in out
    const size_t o_bytes = kind == 2 ? (size_t)65536 * 16 : bytes;
    auto ov = [](const void *p, size_t np, const void *q, size_t nq) {
        if (!p || !q) return false;
        const uintptr_t p0 = (uintptr_t)p, q0 = (uintptr_t)q;
        return p0 < q0 + nq && q0 < p0 + np;
    };
    if ((need_a && ov(out, o_bytes, a, bytes)) || (need_b && ov(out, o_bytes, b, bytes))) return DCP_E_ALIAS;
    const int64_t n = (int64_t)(bytes / 16);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    switch (kind) {
        case 0: e = probe_launch<0>(nt != 0, a, b, out, n, st); break;
        case 1: e = probe_launch<1>(nt != 0, a, b, out, n, st); break;
        case 2: e = probe_launch<2>(nt != 0, a, b, out, n, st); break;
        default: e = probe_launch<3>(nt != 0, a, b, out, n, st); break;
    }
    return e == hipSuccess ? DCP_OK : DCP_E_HIP;
}
