// The (dimension, degree, precision) groups of the matrix-core tent kernels and the
// translation unit that instantiates each (its launchers and, through them, its kernels).
#pragma once

#define MTP_MFMA_INSTANTIATE(D, P, T)                                                                     \
  template hipError_t launch_mdp<D, P, T>(const PersistentArgs&, int, hipStream_t, int*);                 \
  template hipError_t launch_mbp<D, P, T>(const BatchLaunch&, hipStream_t);                               \
  template hipError_t launch_mp<D, P, T>(const KernelParams&, int64_t, int64_t, hipStream_t);             \
  template size_t lds_mp<D, P, T>(int, int);                                                              \
  template size_t opg_mp<D, P, T>(int, int);                                                              \
  template size_t frg_mp<D, P, T>(int, int);                                                              \
  template hipError_t stage_mp<D, P, T>(const KernelParams&, hipStream_t);
#define MTP_MFMA_EXTERN(D, P, T)                                                                          \
  extern template hipError_t launch_mdp<D, P, T>(const PersistentArgs&, int, hipStream_t, int*);          \
  extern template hipError_t launch_mbp<D, P, T>(const BatchLaunch&, hipStream_t);                        \
  extern template hipError_t launch_mp<D, P, T>(const KernelParams&, int64_t, int64_t, hipStream_t);      \
  extern template size_t lds_mp<D, P, T>(int, int);                                                       \
  extern template size_t opg_mp<D, P, T>(int, int);                                                       \
  extern template size_t frg_mp<D, P, T>(int, int);                                                       \
  extern template hipError_t stage_mp<D, P, T>(const KernelParams&, hipStream_t);

// tent_mfma_2d_p12.hip, tent_mfma_2d_p3.hip, tent_mfma_2d_p4.hip, tent_mfma_2d_p5.hip
#define MTP_MFMA_CONFIGS_2D_P12(X) X(2, 1, double) X(2, 1, float) X(2, 2, double) X(2, 2, float)
#define MTP_MFMA_CONFIGS_2D_P3(X) X(2, 3, double) X(2, 3, float)
#define MTP_MFMA_CONFIGS_2D_P4(X) X(2, 4, double) X(2, 4, float)
#define MTP_MFMA_CONFIGS_2D_P5(X) X(2, 5, double) X(2, 5, float)
// tent_mfma_3d_p1.hip, tent_mfma_3d_p2.hip, tent_mfma_3d_p3.hip, tent_mfma_3d_p4_f64.hip,
// tent_mfma_3d_p4_f32.hip
#define MTP_MFMA_CONFIGS_3D_P1(X) X(3, 1, double) X(3, 1, float)
#define MTP_MFMA_CONFIGS_3D_P2(X) X(3, 2, double) X(3, 2, float)
#define MTP_MFMA_CONFIGS_3D_P3(X) X(3, 3, double) X(3, 3, float)
#define MTP_MFMA_CONFIGS_3D_P4_F64(X) X(3, 4, double)
#define MTP_MFMA_CONFIGS_3D_P4_F32(X) X(3, 4, float)
// tent_mfma_3d_p5.hip
#define MTP_MFMA_CONFIGS_3D_P5(X) X(3, 5, double) X(3, 5, float)

#define MTP_MFMA_CONFIGS(X)                                                                               \
  MTP_MFMA_CONFIGS_2D_P12(X) MTP_MFMA_CONFIGS_2D_P3(X) MTP_MFMA_CONFIGS_2D_P4(X) MTP_MFMA_CONFIGS_2D_P5(X)  \
  MTP_MFMA_CONFIGS_3D_P1(X) MTP_MFMA_CONFIGS_3D_P2(X) MTP_MFMA_CONFIGS_3D_P3(X) MTP_MFMA_CONFIGS_3D_P4_F64(X) \
  MTP_MFMA_CONFIGS_3D_P4_F32(X) MTP_MFMA_CONFIGS_3D_P5(X)
