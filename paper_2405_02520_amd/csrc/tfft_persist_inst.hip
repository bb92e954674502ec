// One (element type, checksum scheme) instantiation of the persistent ragged
// kernel: the build compiles this file once per pair with
// -DTFFT_INST_R=<float|double> and -DTFFT_INST_FT=<FT_NONE|FT_BLOCK>.
#include "tfft_persist.h"

namespace tfft {
TFFT_PERSIST_INSTANTIATE(TFFT_INST_R, TFFT_INST_FT)
}  // namespace tfft
