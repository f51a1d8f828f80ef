// Dispatch of the matrix-core tent kernels on (dimension, degree, precision, patch size);
// the kernels are instantiated in tent_mfma_*.hip (one translation unit per group, so that
// the build runs them in parallel).
#include "tent_mfma.h"
#include "tent_mfma_configs.h"

namespace mtp {
namespace mfk {

MTP_MFMA_CONFIGS(MTP_MFMA_EXTERN)

template <typename T>
hipError_t launch_dt(const PersistentArgs& a, int d, int p, int max_patch, hipStream_t s, int* resident) {
  if (d == 2) {
    switch (p) {
      case 1: return launch_mdp<2, 1, T>(a, max_patch, s, resident);
      case 2: return launch_mdp<2, 2, T>(a, max_patch, s, resident);
      case 3: return launch_mdp<2, 3, T>(a, max_patch, s, resident);
      case 4: return launch_mdp<2, 4, T>(a, max_patch, s, resident);
      case 5: return launch_mdp<2, 5, T>(a, max_patch, s, resident);
    }
  } else {
    switch (p) {
      case 1: return launch_mdp<3, 1, T>(a, max_patch, s, resident);
      case 2: return launch_mdp<3, 2, T>(a, max_patch, s, resident);
      case 3: return launch_mdp<3, 3, T>(a, max_patch, s, resident);
      case 4: return launch_mdp<3, 4, T>(a, max_patch, s, resident);
      case 5: return launch_mdp<3, 5, T>(a, max_patch, s, resident);
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_bt(const BatchLaunch& bl, hipStream_t s) {
  if (bl.d == 2) {
    switch (bl.p) {
      case 1: return launch_mbp<2, 1, T>(bl, s);
      case 2: return launch_mbp<2, 2, T>(bl, s);
      case 3: return launch_mbp<2, 3, T>(bl, s);
      case 4: return launch_mbp<2, 4, T>(bl, s);
      case 5: return launch_mbp<2, 5, T>(bl, s);
    }
  } else {
    switch (bl.p) {
      case 1: return launch_mbp<3, 1, T>(bl, s);
      case 2: return launch_mbp<3, 2, T>(bl, s);
      case 3: return launch_mbp<3, 3, T>(bl, s);
      case 4: return launch_mbp<3, 4, T>(bl, s);
      case 5: return launch_mbp<3, 5, T>(bl, s);
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_t(const KernelParams& kp, int64_t first, int64_t count, hipStream_t s) {
  if (kp.d == 2) {
    switch (kp.p) {
      case 1: return launch_mp<2, 1, T>(kp, first, count, s);
      case 2: return launch_mp<2, 2, T>(kp, first, count, s);
      case 3: return launch_mp<2, 3, T>(kp, first, count, s);
      case 4: return launch_mp<2, 4, T>(kp, first, count, s);
      case 5: return launch_mp<2, 5, T>(kp, first, count, s);
    }
  } else {
    switch (kp.p) {
      case 1: return launch_mp<3, 1, T>(kp, first, count, s);
      case 2: return launch_mp<3, 2, T>(kp, first, count, s);
      case 3: return launch_mp<3, 3, T>(kp, first, count, s);
      case 4: return launch_mp<3, 4, T>(kp, first, count, s);
      case 5: return launch_mp<3, 5, T>(kp, first, count, s);
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
size_t lds_t(int d, int p, int max_patch, int system) {
  if (d == 2) {
    switch (p) {
      case 1: return lds_mp<2, 1, T>(max_patch, system);
      case 2: return lds_mp<2, 2, T>(max_patch, system);
      case 3: return lds_mp<2, 3, T>(max_patch, system);
      case 4: return lds_mp<2, 4, T>(max_patch, system);
      case 5: return lds_mp<2, 5, T>(max_patch, system);
    }
  } else {
    switch (p) {
      case 1: return lds_mp<3, 1, T>(max_patch, system);
      case 2: return lds_mp<3, 2, T>(max_patch, system);
      case 3: return lds_mp<3, 3, T>(max_patch, system);
      case 4: return lds_mp<3, 4, T>(max_patch, system);
      case 5: return lds_mp<3, 5, T>(max_patch, system);
    }
  }
  return (size_t)-1;
}

template <typename T>
size_t opg_t(int d, int p, int max_patch, int system) {
  if (d == 2) {
    switch (p) {
      case 1: return opg_mp<2, 1, T>(max_patch, system);
      case 2: return opg_mp<2, 2, T>(max_patch, system);
      case 3: return opg_mp<2, 3, T>(max_patch, system);
      case 4: return opg_mp<2, 4, T>(max_patch, system);
      case 5: return opg_mp<2, 5, T>(max_patch, system);
    }
  } else {
    switch (p) {
      case 1: return opg_mp<3, 1, T>(max_patch, system);
      case 2: return opg_mp<3, 2, T>(max_patch, system);
      case 3: return opg_mp<3, 3, T>(max_patch, system);
      case 4: return opg_mp<3, 4, T>(max_patch, system);
      case 5: return opg_mp<3, 5, T>(max_patch, system);
    }
  }
  return 0;
}

template <typename T>
hipError_t stage_t(const KernelParams& kp, hipStream_t s) {
  if (kp.d == 2) {
    switch (kp.p) {
      case 1: return stage_mp<2, 1, T>(kp, s);
      case 2: return stage_mp<2, 2, T>(kp, s);
      case 3: return stage_mp<2, 3, T>(kp, s);
      case 4: return stage_mp<2, 4, T>(kp, s);
      case 5: return stage_mp<2, 5, T>(kp, s);
    }
  } else {
    switch (kp.p) {
      case 1: return stage_mp<3, 1, T>(kp, s);
      case 2: return stage_mp<3, 2, T>(kp, s);
      case 3: return stage_mp<3, 3, T>(kp, s);
      case 4: return stage_mp<3, 4, T>(kp, s);
      case 5: return stage_mp<3, 5, T>(kp, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace mfk

using namespace mfk;

size_t tent_mfma_opg_bytes(int d, int p, int max_patch, int fp32, int system) {
  return fp32 ? opg_t<float>(d, p, max_patch, system) : opg_t<double>(d, p, max_patch, system);
}

size_t tent_mfma_frg_bytes(int d, int p, int max_patch, int fp32, int system) {
  if (d != 3 || (p != 4 && p != 5)) return 0;   // only P4 and P5 in 3D have the extra-large class
  if (p == 5) return fp32 ? frg_mp<3, 5, float>(max_patch, system) : frg_mp<3, 5, double>(max_patch, system);
  return fp32 ? frg_mp<3, 4, float>(max_patch, system) : frg_mp<3, 4, double>(max_patch, system);
}

hipError_t stage_tent_operator_mfma(const KernelParams& kp, int fp32, hipStream_t s) {
  return fp32 ? stage_t<float>(kp, s) : stage_t<double>(kp, s);
}

hipError_t launch_tent_dag_mfma(const KernelParams& kp, int fp32, hipStream_t s) {
  const PersistentArgs a{&kp, nullptr, nullptr};
  return fp32 ? launch_dt<float>(a, kp.d, kp.p, kp.max_patch, s, nullptr)
              : launch_dt<double>(a, kp.d, kp.p, kp.max_patch, s, nullptr);
}

int tent_dag_grid(const KernelParams& kp, int fp32) {
  int resident = 0;
  const PersistentArgs a{&kp, nullptr, nullptr};
  const hipError_t e = fp32 ? launch_dt<float>(a, kp.d, kp.p, kp.max_patch, nullptr, &resident)
                            : launch_dt<double>(a, kp.d, kp.p, kp.max_patch, nullptr, &resident);
  return e == hipSuccess ? resident : 0;
}

hipError_t launch_tent_batch_dag_mfma(const KernelParams* kps, const BatchDag& bd, int d, int p, int max_patch,
                                      int fp32, hipStream_t s) {
  const PersistentArgs a{nullptr, kps, &bd};
  return fp32 ? launch_dt<float>(a, d, p, max_patch, s, nullptr) : launch_dt<double>(a, d, p, max_patch, s, nullptr);
}

int tent_batch_dag_grid(int d, int p, int max_patch, int fp32, int system, int method) {
  int resident = 0;
  BatchDag bd{};
  bd.system = system;
  bd.method = method;
  const PersistentArgs a{nullptr, nullptr, &bd};
  const hipError_t e = fp32 ? launch_dt<float>(a, d, p, max_patch, nullptr, &resident)
                            : launch_dt<double>(a, d, p, max_patch, nullptr, &resident);
  return e == hipSuccess ? resident : 0;
}

size_t tent_mfma_lds_bytes(int d, int p, int max_patch, int fp32, int system) {
  return fp32 ? lds_t<float>(d, p, max_patch, system) : lds_t<double>(d, p, max_patch, system);
}

hipError_t launch_tent_batch_mfma(const BatchLaunch& bl, int fp32, hipStream_t s) {
  return fp32 ? launch_bt<float>(bl, s) : launch_bt<double>(bl, s);
}

hipError_t launch_tent_layer_mfma(const KernelParams& kp, int64_t first, int64_t count, int fp32, hipStream_t s) {
  if (count == 0) return hipSuccess;
  return fp32 ? launch_t<float>(kp, first, count, s) : launch_t<double>(kp, first, count, s);
}

}  // namespace mtp
