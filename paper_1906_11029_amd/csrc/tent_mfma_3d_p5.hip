// Instantiation of the matrix-core tent kernels for one group of (dimension, degree,
// precision); the kernel code is in tent_mfma.h.
#include "tent_mfma.h"
#include "tent_mfma_configs.h"

namespace mtp {
namespace mfk {
MTP_MFMA_CONFIGS_3D_P5(MTP_MFMA_INSTANTIATE)
}  // namespace mfk
}  // namespace mtp
