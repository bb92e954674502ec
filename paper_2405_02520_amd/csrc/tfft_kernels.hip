// Dispatch of the pass, correction and reset launches over the element type
// and the pass length; the kernels themselves are instantiated per
// (type, length) in tfft_inst.hip.
#include <algorithm>

#include "tfft_persist.h"

namespace tfft {

TFFT_FOR_EACH_M(TFFT_EXTERN_M, float)
TFFT_FOR_EACH_M(TFFT_EXTERN_M, double)
TFFT_PERSIST_EXTERN(float, FT_NONE)
TFFT_PERSIST_EXTERN(float, FT_BLOCK)
TFFT_PERSIST_EXTERN(double, FT_NONE)
TFFT_PERSIST_EXTERN(double, FT_BLOCK)

__global__ void reset_kernel(DevReport *rep) {
    if (threadIdx.x == 0) {
        rep->n_flag = 0;
        rep->corrected = 0;
        rep->benign = 0;
        rep->uncorrectable = 0;
    }
}

template <typename R, typename F>
static hipError_t by_m(int M, F &&f) {
    switch (M) {
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 32: return f(std::integral_constant<int, 32>{});
        case 64: return f(std::integral_constant<int, 64>{});
        case 128: return f(std::integral_constant<int, 128>{});
        case 256: return f(std::integral_constant<int, 256>{});
        case 512: return f(std::integral_constant<int, 512>{});
        case 1024: return f(std::integral_constant<int, 1024>{});
        case 2048: return f(std::integral_constant<int, 2048>{});
        case 4096: return f(std::integral_constant<int, 4096>{});
        case 8192: return f(std::integral_constant<int, 8192>{});
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(int fp64, int M, int kind, int ft, const PassArgs &a, int grid, hipStream_t st) {
    if (fp64)
        return by_m<double>(M, [&](auto m) { return launch_m<double, decltype(m)::value>(kind, ft, a, grid, st); });
    return by_m<float>(M, [&](auto m) { return launch_m<float, decltype(m)::value>(kind, ft, a, grid, st); });
}

hipError_t launch_correct(int fp64, int M, int kind, const PassArgs &a, int grid, hipStream_t st) {
    if (fp64) return by_m<double>(M, [&](auto m) { return correct_m<double, decltype(m)::value>(kind, a, grid, st); });
    return by_m<float>(M, [&](auto m) { return correct_m<float, decltype(m)::value>(kind, a, grid, st); });
}

int pass_occupancy(int fp64, int M, int kind, int ft) {
    int r = 0;
    auto f = [&](auto m) {
        r = fp64 ? occ_m<double, decltype(m)::value>(kind, ft) : occ_m<float, decltype(m)::value>(kind, ft);
        return hipSuccess;
    };
    if (fp64) by_m<double>(M, f);
    else by_m<float>(M, f);
    return r;
}

// Streaming copy (measurement instrument): 16-byte non-temporal loads and
// stores, four in flight per thread, a grid-stride loop over whole 16-byte
// elements and a byte tail.
__global__ void __launch_bounds__(512) stream_copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                          size_t n16, const unsigned char *__restrict__ tsrc,
                                                          unsigned char *__restrict__ tdst, size_t ntail) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const v4u *s = reinterpret_cast<const v4u *>(src);
    v4u *d = reinterpret_cast<v4u *>(dst);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        v4u v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(s + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], d + i + u * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tdst[threadIdx.x] = tsrc[threadIdx.x];
}

hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;
    const size_t ntail = bytes % 16;
    const unsigned char *ts = static_cast<const unsigned char *>(src) + n16 * 16;
    unsigned char *td = static_cast<unsigned char *>(dst) + n16 * 16;
    size_t want = (n16 / 4 + 511) / 512;
    const unsigned grid = (unsigned)std::max<size_t>(1, std::min<size_t>(want, TFFT_COPY_GRID));
    hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(512), 0, st, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), n16, ts, td, ntail);
    return hipGetLastError();
}

hipError_t launch_persist(int fp64, int ft, const PQueue &q, int grid, hipStream_t st) {
    if (fp64) return ft ? persist_launch<double, FT_BLOCK>(q, grid, st) : persist_launch<double, FT_NONE>(q, grid, st);
    return ft ? persist_launch<float, FT_BLOCK>(q, grid, st) : persist_launch<float, FT_NONE>(q, grid, st);
}

int persist_occupancy(int fp64, int ft) {
    if (fp64) return ft ? persist_occ<double, FT_BLOCK>() : persist_occ<double, FT_NONE>();
    return ft ? persist_occ<float, FT_BLOCK>() : persist_occ<float, FT_NONE>();
}

// Queue state of one persistent execution cleared by a kernel (no memset
// node in a captured graph): the head, the release counts, the error flag
// and the report counters.
__global__ void persist_reset_kernel(PQueue q, int n_done, DevReport *rep) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_done) q.done[i] = 0;
    if (i < kPQueues) q.head[i] = 0;
    if (i == 0) {
        *q.err = 0;
        rep->n_flag = 0;
        rep->corrected = 0;
        rep->benign = 0;
        rep->uncorrectable = 0;
    }
}

hipError_t launch_persist_reset(const PQueue &q, int n_done, DevReport *rep, hipStream_t st) {
    const int threads = 256;
    const int blocks = std::max(1, (n_done + threads - 1) / threads);
    hipLaunchKernelGGL(persist_reset_kernel, dim3(blocks), dim3(threads), 0, st, q, n_done, rep);
    return hipGetLastError();
}

hipError_t launch_reset(DevReport *rep, hipStream_t st) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, rep);
    return hipGetLastError();
}

}  // namespace tfft
