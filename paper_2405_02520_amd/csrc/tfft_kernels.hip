// Dispatch of the pass, correction and reset launches over the element type
// and the pass length; the kernels themselves are instantiated per
// (type, length) in tfft_inst.hip.
#include "tfft_kernels.h"

namespace tfft {

TFFT_FOR_EACH_M(TFFT_EXTERN_M, float)
TFFT_FOR_EACH_M(TFFT_EXTERN_M, double)

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

hipError_t launch_reset(DevReport *rep, hipStream_t st) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, rep);
    return hipGetLastError();
}

}  // namespace tfft
