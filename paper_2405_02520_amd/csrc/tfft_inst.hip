// One (element type, pass length) instantiation of the kernels: the build
// compiles this file once per pair with -DTFFT_INST_R=<float|double> and
// -DTFFT_INST_M=<length>.
#include "tfft_kernels.h"

namespace tfft {
TFFT_INSTANTIATE_M(TFFT_INST_R, TFFT_INST_M)
}  // namespace tfft
