// HIP kernels for gfx950: the per-tent SAT evolution of mapped-tent DG Maxwell, and
// the set / read-out conversions of the state.
//
// One workgroup advances one tent (one launch per layer; the tents of a layer have
// element-disjoint patches, section 2).  For a tent at vertex V with height H:
//   - every patch element is renumbered so that V is its local vertex 0 (node gather
//     through a permutation table), so all elements share the reference operators
//     S_l (volume) and L_j (lift) staged once in LDS;
//   - per element: grad phi_b = sum_i tau_i grad lambda_i, b' = grad delta = H grad lambda_V,
//     b_i = grad phi_b + (i/m) b'  (the tent map's gradient at the sub-interval start);
//   - SAT (section 4, eqs. coeff_rec and recursion-init) with the state w = nodal values
//     of g(u) - f(u) grad phi (Y with the element mass divided out):
//       U_{i,0} = K(b_i)^{-1} W                                (closed form, FP64)
//       Y_{i,n} = H [ sum_l A(grad lambda_l) S_l U - sum_j L_j G_j(U) ]   n = 1..q
//       U_{i,n} = K(b_i)^{-1} (Y_{i,n} + n A(b') U_{i,n-1})    n = 1..q-1 (M'U = -A(b')U)
//       W <- sum_n Y_{i,n} / (m^n n!)                          (Taylor sum, FP64)
//     where G_j is the upwind flux times |grad lambda_j| at the face nodes of the faces
//     containing V (faces of the patch boundary carry delta = 0 and are skipped);
//   - scatter W back and set tau_V = t_top.
// The patch state U lives in LDS; each thread owns (element, node) pairs and keeps the
// Taylor accumulator in registers.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"
#include "tent_common.h"

namespace mtp {

namespace {

template <int D, int P>
struct Shape {
  static constexpr int NC = Dims<D>::NC;
  static constexpr int NP = binom_c(P + D, D);
  static constexpr int NF = binom_c(P + D - 1, D - 1);
  static constexpr int NV = D + 1;
};

// LDS layout (doubles first, then ints), per workgroup
template <int D, int P>
struct Lds {
  using SH = Shape<D, P>;
  static __host__ __device__ size_t doubles(int nt) {
    return (size_t)D * SH::NP * SH::NP          // S
           + (size_t)D * SH::NF * SH::NP        // L
           + (size_t)nt * SH::NC * SH::NP       // U
           + (size_t)nt * D * SH::NC * SH::NF   // G
           + (size_t)nt * SH::NV * D            // permuted grad lambda
           + (size_t)nt * D                     // grad phi_b
           + (size_t)nt * 2;                    // eps, mu
  }
  static __host__ __device__ size_t ints(int nt) {
    return (size_t)D * 2 * SH::NF + (size_t)nt * (2 + D);
  }
  static __host__ __device__ size_t bytes(int nt) { return doubles(nt) * 8 + ints(nt) * 4; }
};

template <int D, int P, int BLOCK, int MAXPAIR>
__global__ void __launch_bounds__(BLOCK) tent_kernel(KernelParams kp, int64_t first, int64_t count) {
  using SH = Shape<D, P>;
  constexpr int NC = SH::NC, NP = SH::NP, NF = SH::NF, NV = SH::NV;
  extern __shared__ double lds[];
  const int nt_max = kp.max_patch;
  double* sS = lds;
  double* sL = sS + D * NP * NP;
  double* sU = sL + D * NF * NP;
  double* sG = sU + (size_t)nt_max * NC * NP;
  double* sGL = sG + (size_t)nt_max * D * NC * NF;
  double* sBb = sGL + (size_t)nt_max * NV * D;
  double* sEM = sBb + (size_t)nt_max * D;
  int* sFn = reinterpret_cast<int*>(sEM + (size_t)nt_max * 2);
  int* sElem = sFn + D * 2 * NF;   // [e]: element id
  int* sK = sElem + nt_max;        // [e]: local index of V
  int* sF = sK + nt_max;           // [e][j]: face codes

  const int tid = threadIdx.x;
  for (int i = tid; i < D * NP * NP; i += BLOCK) sS[i] = kp.S[i];
  for (int i = tid; i < D * NF * NP; i += BLOCK) sL[i] = kp.L[i];
  for (int i = tid; i < D * 2 * NF; i += BLOCK) sFn[i] = kp.fnode[i];

  const double invm = 1.0 / kp.m;

  for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
    const int32_t V = kp.tent_vertex[first + t];
    const double t_top = kp.slab[0] + kp.tent_top[first + t];
    const int32_t p0 = kp.patch_ptr[V];
    const int nT = kp.patch_ptr[V + 1] - p0;
    const double t_bot = kp.tau[V];
    const double H = t_top - t_bot;

    // element setup
    for (int e = tid; e < nT; e += BLOCK) {
      const int el = kp.patch_elem[p0 + e];
      const int32_t* info = kp.patch_info + (size_t)(p0 + e) * (1 + D);
      const int k = info[0];
      int order[NV];
      vertex_order_dev<D>(k, order);
      const double* gl = kp.grad_lam + (size_t)el * NV * D;
      double gb[D];
#pragma unroll
      for (int i = 0; i < D; ++i) gb[i] = 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double tv = kp.tau[kp.cells[(size_t)el * NV + v]];
#pragma unroll
        for (int i = 0; i < D; ++i) gb[i] += tv * gl[v * D + i];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int i = 0; i < D; ++i) sGL[(e * NV + v) * D + i] = gl[order[v] * D + i];
#pragma unroll
      for (int i = 0; i < D; ++i) sBb[e * D + i] = gb[i];
      sEM[2 * e] = kp.eps[el];
      sEM[2 * e + 1] = kp.mu[el];
      sElem[e] = el;
      sK[e] = k;
#pragma unroll
      for (int j = 0; j < D; ++j) sF[e * D + j] = info[1 + j];
    }
    __syncthreads();

    // gather W for the owned (element, node) pairs
    const int npairs = nT * NP;
    double acc[MAXPAIR][NC];
    double unew[MAXPAIR][NC];
#pragma unroll
    for (int r = 0; r < MAXPAIR; ++r) {
      const int P_ = tid + r * BLOCK;
      if (P_ < npairs) {
        const int e = P_ / NP, b = P_ - e * NP;
        const int nold = kp.perm[sK[e] * NP + b];
        const double* Wp = kp.W + (size_t)sElem[e] * NC * NP + nold;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = Wp[c * NP];
      }
    }
    bool ok = true;
    // U_{0,0} = K(b_0)^{-1} W
#pragma unroll
    for (int r = 0; r < MAXPAIR; ++r) {
      const int P_ = tid + r * BLOCK;
      if (P_ < npairs) {
        const int e = P_ / NP, b = P_ - e * NP;
        double u[NC];
        ok &= kinv<D>(&sBb[e * D], sEM[2 * e], sEM[2 * e + 1], acc[r], u);
#pragma unroll
        for (int c = 0; c < NC; ++c) sU[(e * NC + c) * NP + b] = u[c];
      }
    }
    __syncthreads();

    for (int i = 0; i < kp.m; ++i) {
      const double th = i * invm;
      double coef = 1.0;
      for (int n = 1; n <= kp.q; ++n) {
        coef *= invm / n;
        // ---- face fluxes G_j at the face nodes of the faces containing V
        for (int it = tid; it < nT * D * NF; it += BLOCK) {
          const int e = it / (D * NF);
          const int rem = it - e * (D * NF);
          const int j = rem / NF;
          const int s = rem - j * NF;
          const int nin = sFn[(j * 2) * NF + s];
          double um[NC], up[NC], G[NC], g[D];
#pragma unroll
          for (int c = 0; c < NC; ++c) um[c] = sU[(e * NC + c) * NP + nin];
#pragma unroll
          for (int x = 0; x < D; ++x) g[x] = -sGL[(e * NV + j + 1) * D + x];
          const int code = sF[e * D + j];
          if (code >= 0) {
            const int pe = code >> 4, jn = (code >> 1) & 7, o = code & 1;
            const int nout = sFn[((jn - 1) * 2 + o) * NF + s];
#pragma unroll
            for (int c = 0; c < NC; ++c) up[c] = sU[(pe * NC + c) * NP + nout];
          } else {
            ghost_state<D, P>(kp, -1 - code, um, up, sElem[e], sK[e], nin, H, th, n);
          }
          flux<D>(g, kp.alpha, um, up, G);
#pragma unroll
          for (int c = 0; c < NC; ++c) sG[((e * D + j) * NC + c) * NF + s] = G[c];
        }
        __syncthreads();

        // ---- volume + lift for the owned pairs, Taylor accumulation, next U
#pragma unroll
        for (int r = 0; r < MAXPAIR; ++r) {
          const int P_ = tid + r * BLOCK;
          if (P_ < npairs) {
            const int e = P_ / NP, b = P_ - e * NP;
            const double* Ue = sU + (size_t)e * NC * NP;
            double Y[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) Y[c] = 0.0;
#pragma unroll
            for (int l = 0; l < D; ++l) {
              double tl[NC];
#pragma unroll
              for (int c = 0; c < NC; ++c) tl[c] = 0.0;
              const double* Sl = sS + l * NP * NP + b;
              for (int a = 0; a < NP; ++a) {
                const double sv = Sl[a * NP];
#pragma unroll
                for (int c = 0; c < NC; ++c) tl[c] = fma(sv, Ue[c * NP + a], tl[c]);
              }
              double gl[D], at[NC];
#pragma unroll
              for (int x = 0; x < D; ++x) gl[x] = sGL[(e * NV + l + 1) * D + x];
              applyA<D>(gl, tl, at);
#pragma unroll
              for (int c = 0; c < NC; ++c) Y[c] += at[c];
            }
            const double* Ge = sG + (size_t)e * D * NC * NF;
#pragma unroll
            for (int j = 0; j < D; ++j) {
              const double* Lj = sL + j * NF * NP + b;
              for (int s = 0; s < NF; ++s) {
                const double lv = Lj[s * NP];
#pragma unroll
                for (int c = 0; c < NC; ++c) Y[c] = fma(-lv, Ge[(j * NC + c) * NF + s], Y[c]);
              }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              Y[c] *= H;
              acc[r][c] = fma(coef, Y[c], acc[r][c]);
            }
            const double* gv = &sGL[(e * NV + 0) * D];
            if (n < kp.q) {
              // U_n = K(b_i)^{-1} (Y_n + n A(b') U_{n-1}),  b' = H grad lambda_V
              double bi[D], bp[D], uo[NC], au[NC], rhs[NC];
#pragma unroll
              for (int x = 0; x < D; ++x) {
                bp[x] = H * gv[x];
                bi[x] = sBb[e * D + x] + th * bp[x];
              }
#pragma unroll
              for (int c = 0; c < NC; ++c) uo[c] = Ue[c * NP + b];
              applyA<D>(bp, uo, au);
#pragma unroll
              for (int c = 0; c < NC; ++c) rhs[c] = Y[c] + n * au[c];
              ok &= kinv<D>(bi, sEM[2 * e], sEM[2 * e + 1], rhs, unew[r]);
            } else if (i + 1 < kp.m) {
              // next sub-interval: U_{i+1,0} = K(b_{i+1})^{-1} W
              double bi[D];
              const double th1 = (i + 1) * invm;
#pragma unroll
              for (int x = 0; x < D; ++x) bi[x] = sBb[e * D + x] + th1 * H * gv[x];
              ok &= kinv<D>(bi, sEM[2 * e], sEM[2 * e + 1], acc[r], unew[r]);
            }
          }
        }
        __syncthreads();
        if (n < kp.q || i + 1 < kp.m) {
#pragma unroll
          for (int r = 0; r < MAXPAIR; ++r) {
            const int P_ = tid + r * BLOCK;
            if (P_ < npairs) {
              const int e = P_ / NP, b = P_ - e * NP;
#pragma unroll
              for (int c = 0; c < NC; ++c) sU[(e * NC + c) * NP + b] = unew[r][c];
            }
          }
          __syncthreads();
        }
      }
    }

    // scatter the tent top
#pragma unroll
    for (int r = 0; r < MAXPAIR; ++r) {
      const int P_ = tid + r * BLOCK;
      if (P_ < npairs) {
        const int e = P_ / NP, b = P_ - e * NP;
        const int nold = kp.perm[sK[e] * NP + b];
        double* Wp = kp.W + (size_t)sElem[e] * NC * NP + nold;
#pragma unroll
        for (int c = 0; c < NC; ++c) Wp[c * NP] = acc[r][c];
      }
    }
    if (!ok) kp.err[0] = ERRF_CAUSALITY;
    __syncthreads();
    if (tid == 0) kp.tau[V] = t_top;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ conversions
// set: W[e][c][node] = K(grad tau_e) u[e][node][c]   (w = g(u) - f(u) grad tau)
template <int D, int SYS>
__global__ void set_fields_kernel(KernelParams kp, int64_t ne, const double* u) {
  using PH = Phys<D, SYS>;
  constexpr int NC = PH::NC, NV = D + 1;
  const int np = kp.np;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne * np) return;
  const int64_t e = idx / np;
  const int a = (int)(idx - e * np);
  double g[D];
  for (int i = 0; i < D; ++i) g[i] = 0.0;
  for (int v = 0; v < NV; ++v) {
    const double tv = kp.tau[kp.cells[e * NV + v]];
    for (int i = 0; i < D; ++i) g[i] += tv * kp.grad_lam[(e * NV + v) * D + i];
  }
  double uu[NC], fu[NC];
  bool fin = true;
  for (int c = 0; c < NC; ++c) {
    uu[c] = u[(e * np + a) * NC + c];
    fin &= isfinite(uu[c]);
  }
  PH::A(g, uu, fu);
  const double eps = kp.eps[e], mu = kp.mu[e];
  for (int c = 0; c < NC; ++c) {
    const double gm = (c < PH::NE) ? eps : mu;
    kp.W[(e * NC + c) * np + a] = gm * uu[c] - fu[c];
  }
  if (!fin) kp.err[1] = ERRF_NONFINITE;
}

template <int D, int SYS>
__global__ void get_fields_kernel(KernelParams kp, int64_t ne, double* out, int raw) {
  using PH = Phys<D, SYS>;
  constexpr int NC = PH::NC, NV = D + 1;
  const int np = kp.np;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne * np) return;
  const int64_t e = idx / np;
  const int a = (int)(idx - e * np);
  double w[NC], u[NC];
  bool fin = true;
  for (int c = 0; c < NC; ++c) {
    w[c] = kp.W[(e * NC + c) * np + a];
    fin &= isfinite(w[c]);
  }
  if (raw) {
    for (int c = 0; c < NC; ++c) out[(e * np + a) * NC + c] = w[c];
  } else {
    double g[D];
    for (int i = 0; i < D; ++i) g[i] = 0.0;
    for (int v = 0; v < NV; ++v) {
      const double tv = kp.tau[kp.cells[e * NV + v]];
      for (int i = 0; i < D; ++i) g[i] += tv * kp.grad_lam[(e * NV + v) * D + i];
    }
    if (!PH::inv(g, kp.eps[e], kp.mu[e], w, u)) kp.err[0] = ERRF_CAUSALITY;
    for (int c = 0; c < NC; ++c) out[(e * np + a) * NC + c] = u[c];
  }
  if (!fin) kp.err[1] = ERRF_NONFINITE;
}

__global__ void slab_reset_kernel(double* slab, double t0, double height) {
  if (threadIdx.x == 0) {
    slab[0] = t0;
    slab[1] = height;
    slab[2] = t0;
    slab[3] = 0.0;
  }
}
__global__ void slab_begin_kernel(double* slab) {
  if (threadIdx.x == 0) slab[0] = slab[2] + slab[3] * slab[1];
}
__global__ void slab_end_kernel(double* slab) {
  if (threadIdx.x == 0) slab[3] += 1.0;
}

__global__ void batch_slab_kernel(const KernelParams* kps, int n, int end) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double* slab = kps[i].slab;
    if (end) slab[3] += 1.0;
    else slab[0] = slab[2] + slab[3] * slab[1];
  }
}

// Persistent-schedule state for one slab: in-degrees from the pristine copy, the tents
// without predecessor (the first nready) in the first queue slots, every other slot
// empty, claim counter 0, fill counter nready, abort clear.
__global__ void dag_reset_kernel(int32_t* indeg, const int32_t* indeg0, int32_t* queue, int32_t* ctl, int n,
                                 int nready) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    indeg[i] = indeg0[i];
    queue[i] = i < nready ? i : -1;
  }
  if (i == 0) {
    ctl[0] = 0;
    ctl[1] = nready;
    ctl[2] = 0;
  }
}

// Batch version: slot / global id i; in-degrees of every solver's tents from their pristine
// copies, the first-layer tents of every solver in the leading queue slots.
__device__ __forceinline__ int last_le(const int32_t* a, int n, int x) {   // last k < n with a[k] <= x
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__global__ void batch_dag_reset_kernel(const KernelParams* kps, BatchDag bd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < bd.n) {
    const int s = last_le(bd.off, bd.nsolv, i);
    const int t = i - bd.off[s];
    kps[s].dag_indeg[t] = kps[s].dag_indeg0[t];
    const int nr = bd.roff[bd.nsolv];
    if (i < nr) {
      const int r = last_le(bd.roff, bd.nsolv, i);
      bd.queue[i] = bd.off[r] + (i - bd.roff[r]);
    } else {
      bd.queue[i] = -1;
    }
  }
  if (i == 0) {
    bd.ctl[0] = 0;
    bd.ctl[1] = bd.roff[bd.nsolv];
    bd.ctl[2] = 0;
  }
}

__global__ void fill_kernel(double* x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ------------------------------------------------------------------ dispatch
template <int D, int P, int BLOCK, int MAXPAIR>
hipError_t launch_tp(const KernelParams& kp, int64_t first, int64_t count, hipStream_t s) {
  const size_t lds = Lds<D, P>::bytes(kp.max_patch);
  auto kfn = tent_kernel<D, P, BLOCK, MAXPAIR>;
  if (count < 0) {   // prepare: allow the dynamic LDS size (done once, outside graph capture)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
  }
  hipLaunchKernelGGL(kfn, dim3((unsigned)count), dim3(BLOCK), lds, s, kp, first, count);
  return hipGetLastError();
}

template <int D, int P, int BLOCK>
hipError_t launch_dp(const KernelParams& kp, int64_t first, int64_t count, hipStream_t s) {
  const int need = (kp.max_patch * Shape<D, P>::NP + BLOCK - 1) / BLOCK;
  if (need <= 1) return launch_tp<D, P, BLOCK, 1>(kp, first, count, s);
  if (need <= 2) return launch_tp<D, P, BLOCK, 2>(kp, first, count, s);
  if (need <= 4) return launch_tp<D, P, BLOCK, 4>(kp, first, count, s);
  if (need <= 8) return launch_tp<D, P, BLOCK, 8>(kp, first, count, s);
  return hipErrorInvalidValue;
}

}  // namespace

bool tent_kernel_supported(int d, int p) {
  return (d == 2 && p >= 1 && p <= 5) || (d == 3 && p >= 1 && p <= 4);
}

size_t tent_kernel_lds_bytes(int d, int p, int nt) {
  if (d == 2) {
    switch (p) {
      case 1: return Lds<2, 1>::bytes(nt);
      case 2: return Lds<2, 2>::bytes(nt);
      case 3: return Lds<2, 3>::bytes(nt);
      case 4: return Lds<2, 4>::bytes(nt);
      case 5: return Lds<2, 5>::bytes(nt);
    }
  } else {
    switch (p) {
      case 1: return Lds<3, 1>::bytes(nt);
      case 2: return Lds<3, 2>::bytes(nt);
      case 3: return Lds<3, 3>::bytes(nt);
      case 4: return Lds<3, 4>::bytes(nt);
    }
  }
  return 0;
}

// maximum (element, node) pairs a workgroup can own
int tent_kernel_max_pairs(int d) { return d == 2 ? 128 * 8 : 256 * 8; }

hipError_t launch_tent_layer(const KernelParams& kp, int64_t first, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (kp.d == 2) {
    switch (kp.p) {
      case 1: return launch_dp<2, 1, 128>(kp, first, count, s);
      case 2: return launch_dp<2, 2, 128>(kp, first, count, s);
      case 3: return launch_dp<2, 3, 128>(kp, first, count, s);
      case 4: return launch_dp<2, 4, 128>(kp, first, count, s);
      case 5: return launch_dp<2, 5, 128>(kp, first, count, s);
    }
  } else {
    switch (kp.p) {
      case 1: return launch_dp<3, 1, 256>(kp, first, count, s);
      case 2: return launch_dp<3, 2, 256>(kp, first, count, s);
      case 3: return launch_dp<3, 3, 256>(kp, first, count, s);
      case 4: return launch_dp<3, 4, 256>(kp, first, count, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_slab_reset(const KernelParams& kp, double t0, double height, hipStream_t s) {
  hipLaunchKernelGGL(slab_reset_kernel, dim3(1), dim3(64), 0, s, kp.slab, t0, height);
  return hipGetLastError();
}
hipError_t launch_batch_slab(const KernelParams* kps, int n, int end, hipStream_t s) {
  hipLaunchKernelGGL(batch_slab_kernel, dim3((n + 63) / 64), dim3(64), 0, s, kps, n, end);
  return hipGetLastError();
}

hipError_t launch_dag_reset(const KernelParams& kp, hipStream_t s) {
  const int n = kp.dag_n > 0 ? kp.dag_n : 1;
  hipLaunchKernelGGL(dag_reset_kernel, dim3((n + 255) / 256), dim3(256), 0, s, kp.dag_indeg, kp.dag_indeg0,
                     kp.dag_queue, kp.dag_ctl, kp.dag_n, kp.dag_nready);
  return hipGetLastError();
}

hipError_t launch_batch_dag_reset(const KernelParams* kps, const BatchDag& bd, hipStream_t s) {
  const int n = bd.n > 0 ? bd.n : 1;
  hipLaunchKernelGGL(batch_dag_reset_kernel, dim3((n + 255) / 256), dim3(256), 0, s, kps, bd);
  return hipGetLastError();
}

hipError_t launch_slab_begin(const KernelParams& kp, hipStream_t s) {
  hipLaunchKernelGGL(slab_begin_kernel, dim3(1), dim3(64), 0, s, kp.slab);
  return hipGetLastError();
}
hipError_t launch_slab_end(const KernelParams& kp, hipStream_t s) {
  hipLaunchKernelGGL(slab_end_kernel, dim3(1), dim3(64), 0, s, kp.slab);
  return hipGetLastError();
}

hipError_t prepare_tent_kernel(const KernelParams& kp, int kernel) {
  if (kernel == 0) return launch_tent_layer(kp, 0, -1, nullptr);
  return launch_tent_layer_mfma(kp, 0, -1, kernel == 2, nullptr);
}

hipError_t launch_set_fields(const KernelParams& kp, int64_t ne, const double* u_nodal, double t0,
                             int64_t nv, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, kp.tau, nv, t0);
  const int64_t n = ne * kp.np;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (kp.d == 2) {
    auto fn = kp.system ? set_fields_kernel<2, 1> : set_fields_kernel<2, 0>;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, kp, ne, u_nodal);
  } else {
    auto fn = kp.system ? set_fields_kernel<3, 1> : set_fields_kernel<3, 0>;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, kp, ne, u_nodal);
  }
  return hipGetLastError();
}

hipError_t launch_get_fields(const KernelParams& kp, int64_t ne, double* out, int raw, hipStream_t s) {
  const int64_t n = ne * kp.np;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (kp.d == 2) {
    auto fn = kp.system ? get_fields_kernel<2, 1> : get_fields_kernel<2, 0>;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, kp, ne, out, raw);
  } else {
    auto fn = kp.system ? get_fields_kernel<3, 1> : get_fields_kernel<3, 0>;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, kp, ne, out, raw);
  }
  return hipGetLastError();
}

}  // namespace mtp
