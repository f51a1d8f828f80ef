// Tents whose patch holds a curved (quadratic) triangle, 2D TE Maxwell, FP64 on the vector
// ALUs (section 4: the structure-aware Taylor recursion; on curved elements the field is
// recovered from the mapped variable by the pointwise closed-form inverse followed by a
// projection with an approximation of the inverse mass matrix).
//
// Every patch element runs on quadrature (the curved path does not use the shared
// reference operator of the affine kernels): per element, in its own node numbering, the
// state W holds the nodal values of the mapped variable w = g(u) - f(u) grad phi, and a
// stage applies
//   R = H [ int lambda_V grad phi_b . f(U) - sum_{faces F containing V} int_F lambda_V phi_b f_n(U-, U+) ]
//   W_n = Minv R,   Minv = Mhat^{-1} M_{1/J} Mhat^{-1}   (the weight-adjusted inverse mass)
// and the recovery of the field from a W-space vector w at sub-interval time th is
//   U = Minv int phi K(b(x, th))^{-1} w(x) dx          (closed form at each quadrature point),
// with b(x, th) = grad phi(x, th) = J^{-T} sum_k tau_k(th) gradhat lambdahat_k.  The
// sub-interval start is U_{i,0} = recovery of W; the correction of stage n < q is
// U_{i,n} = recovery of W_n + n Minv int phi A(b') U, b' = H grad lambda_V.  The Taylor sum
// W <- sum_n W_n / (m^n n!) and the layout of W are those of the affine kernels.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "tent_common.h"

namespace mtp {
namespace {

// 4 waves per tent (one workgroup each); a layer's few hundred curved tents are resident at
// once.  The kernel is bound by LDS traffic (the phases re-read the point values and tables
// per output node), not by the lanes per tent: 8 or 16 waves per tent run no faster.
constexpr int CBLOCK = 256;
// the long reductions (over the volume points) run on teams of TEAM consecutive lanes, each
// summing every TEAM-th point, combined by lane exchanges
constexpr int TEAM = 4;

template <int P>
struct CShape {
  static constexpr int NP = (P + 1) * (P + 2) / 2;
  static constexpr int NQ = (P + 4) * (P + 4);
  static constexpr int NFQ = P + 4;
  static constexpr int NC = 3;
  // LDS per patch element: doubles (S, U, W_n, R, values at the points, face fluxes,
  // eps, mu, the three vertex times) and ints (element, k, zone, 2 x (face, neighbour, code))
  static constexpr int DBL = 4 * NC * NP + NQ * NC + 2 * NFQ * NC + 5;
  static constexpr int INT = 9;
  // reference tables (V, Gr, Lam, Vf, Lamf) and the geometry block of one zone element
  // (Q, Minv, face data), both staged in LDS
  static constexpr int REF = NQ * NP * 3 + NQ * 3 + 3 * NFQ * (NP + 3);
  static constexpr int PER = NQ * 5 + NP * NP + 3 * NFQ * 3;
};

template <int P>
size_t lds_bytes(int max_patch, bool geo) {
  using CS = CShape<P>;
  return (size_t)max_patch * ((size_t)CS::DBL * 8 + (size_t)CS::INT * 4) + 8 + (size_t)CS::REF * 8 +
         (geo ? (size_t)max_patch * CS::PER * 8 : 0);
}

__device__ __forceinline__ double team_sum(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  return v;
}

template <int P>
__global__ void __launch_bounds__(CBLOCK) tent_curved_kernel(KernelParams kp, CurvedParams cp, int64_t first) {
  using CS = CShape<P>;
  constexpr int NP = CS::NP, NQ = CS::NQ, NFQ = CS::NFQ, NC = CS::NC, PER = CS::PER;
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int64_t t = first + blockIdx.x;
  const int32_t V = kp.tent_vertex[t];
  const double t_top = kp.slab[0] + kp.tent_top[t];
  const int32_t p0 = kp.patch_ptr[V];
  const int nT = kp.patch_ptr[V + 1] - p0;
  const double H = t_top - kp.tau[V];
  const double invm = 1.0 / kp.m;
  const int MT = cp.max_patch;

  double* sS = lds;                          // [e][c][a]  W at the sub-interval start / Taylor sum
  double* sU = sS + MT * NC * NP;            // [e][c][a]  stage input U
  double* sWn = sU + MT * NC * NP;           // [e][c][a]  W_n, then the corrected W
  double* sR = sWn + MT * NC * NP;           // [e][c][a]  tested integrals / projection input
  double* sQ = sR + MT * NC * NP;            // [e][q][c]  values at the volume points
  double* sFx = sQ + MT * NQ * NC;           // [e][s][q][c]  lifted face fluxes
  double* sEM = sFx + MT * 2 * NFQ * NC;     // [e][2]  eps, mu
  double* sTau = sEM + MT * 2;               // [e][3]  vertex times at the tent bottom
  int* sEl = reinterpret_cast<int*>(sTau + MT * 3);
  int* sK = sEl + MT;                        // local index of V
  int* sZ = sK + MT;                         // zone index
  int* sFf = sZ + MT;                        // [e][2]  the two local faces containing V
  int* sNb = sFf + MT * 2;                   // [e][2]  patch index of the neighbour, or -1 - kind
  int* sNc = sNb + MT * 2;                   // [e][2]  neighbour face | reversed << 2
  // reference tables, then (if the patch fits) the geometry blocks of its elements
  double* sRef = reinterpret_cast<double*>(sNc + MT * 2 + (MT & 1));   // 8-byte aligned
  double* sGeo = sRef + CS::REF;

  const double* V_ = sRef;                                   // [q][a]
  const double* Gr = V_ + NQ * NP;                           // [q][a][l]
  const double* Lam = Gr + NQ * NP * 2;                      // [q][k]
  const double* Vf = Lam + NQ * 3;                           // [f][q][a]
  const double* Lamf = Vf + 3 * NFQ * NP;                    // [f][q][k]
  // geometry block of patch element e: Q [q][5], Minv [b][a], face data [f][q][3]
  auto geo_of = [&](int e) -> const double* {
    return cp.geo_lds ? sGeo + (size_t)e * PER : cp.geo + (size_t)sZ[e] * PER;
  };
  // gradhat lambdahat_k: (-1, -1), (1, 0), (0, 1)
  auto hat = [](int k, int l) -> double { return k == 0 ? -1.0 : (k == l + 1 ? 1.0 : 0.0); };

  // ---- patch set-up and gather
  for (int i = tid; i < CS::REF; i += CBLOCK) sRef[i] = cp.ref[i];
  for (int e = tid; e < nT; e += CBLOCK) {
    const int el = kp.patch_elem[p0 + e];
    const int k = kp.patch_info[(size_t)(p0 + e) * 3];
    sEl[e] = el;
    sK[e] = k;
    sZ[e] = cp.zone[el];
    sEM[2 * e] = kp.eps[el];
    sEM[2 * e + 1] = kp.mu[el];
    for (int v = 0; v < 3; ++v) sTau[e * 3 + v] = kp.tau[kp.cells[(size_t)el * 3 + v]];
  }
  for (int i = tid; i < nT * NC * NP; i += CBLOCK) {
    const int e = i / (NC * NP), r = i - e * NC * NP;
    sS[i] = kp.W[(size_t)kp.patch_elem[p0 + e] * NC * NP + r];
  }
  if (cp.geo_lds) {
    for (int i = tid; i < nT * PER; i += CBLOCK) {
      const int e = i / PER, r = i - e * PER;
      sGeo[i] = cp.geo[(size_t)cp.zone[kp.patch_elem[p0 + e]] * PER + r];
    }
  }
  __syncthreads();
  for (int e = tid; e < nT; e += CBLOCK) {
    const int z = sZ[e], k = sK[e];
    int s = 0;
    for (int f = 0; f < 3; ++f) {
      if (f == k) continue;   // the face opposite V lies on the patch boundary (delta = 0)
      const int nb = cp.nbr[z * 6 + f];
      int pe = nb;            // -1 - kind on the domain boundary
      if (nb >= 0) {
        pe = -100;
        for (int j = 0; j < nT; ++j)
          if (sEl[j] == nb) pe = j;
      }
      sFf[e * 2 + s] = f;
      sNb[e * 2 + s] = pe;
      sNc[e * 2 + s] = cp.nbr[z * 6 + 3 + f];
      ++s;
    }
  }
  __syncthreads();

  bool ok = true;
  // grad phi(x_q, th) of patch element e: the bottom front with V lifted by th H
  auto front_grad = [&](int e, int q, double th, const double* Q, double* b) {
    double g0 = 0.0, g1 = 0.0;
    for (int kk = 0; kk < 3; ++kk) {
      const double tk = sTau[e * 3 + kk] + (kk == sK[e] ? th * H : 0.0);
      g0 += tk * hat(kk, 0);
      g1 += tk * hat(kk, 1);
    }
    // (J^{-T} g)_r = sum_l Jinv[l][r] g_l
    b[0] = Q[1] * g0 + Q[3] * g1;
    b[1] = Q[2] * g0 + Q[4] * g1;
  };
  // src [e][c][a] -> sQ [e][q][c]: values at the volume points
  auto interp = [&](const double* src) {
    for (int i = tid; i < nT * NQ; i += CBLOCK) {
      const int e = i / NQ, q = i - e * NQ;
      double v[NC] = {0.0, 0.0, 0.0};
      for (int a = 0; a < NP; ++a) {
        const double ph = V_[q * NP + a];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = fma(ph, src[(e * NC + c) * NP + a], v[c]);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) sQ[(e * NQ + q) * NC + c] = v[c];
    }
  };
  // sR = V^T sQ (the weights are already in sQ), then dst = Minv sR (+ scale * into dst)
  auto project = [&](double* dst, bool add, double scale) {
    for (int base = 0; base < nT * NP; base += CBLOCK / TEAM) {
      const int i = base + tid / TEAM, part = tid % TEAM;
      if (i < nT * NP) {   // uniform over the team
        const int e = i / NP, a = i - e * NP;
        double v[NC] = {0.0, 0.0, 0.0};
        for (int q = part; q < NQ; q += TEAM) {
          const double ph = V_[q * NP + a];
#pragma unroll
          for (int c = 0; c < NC; ++c) v[c] = fma(ph, sQ[(e * NQ + q) * NC + c], v[c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = team_sum(v[c]);
        if (part == 0) {
#pragma unroll
          for (int c = 0; c < NC; ++c) sR[(e * NC + c) * NP + a] = v[c];
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < nT * NP; i += CBLOCK) {
      const int e = i / NP, b = i - e * NP;
      const double* Mi = geo_of(e) + NQ * 5 + b * NP;
      double v[NC] = {0.0, 0.0, 0.0};
      for (int a = 0; a < NP; ++a) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = fma(Mi[a], sR[(e * NC + c) * NP + a], v[c]);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double& d = dst[(e * NC + c) * NP + b];
        d = add ? fma(scale, v[c], d) : v[c];
      }
    }
    __syncthreads();
  };
  // U = Minv int phi K(b(x, th))^{-1} w(x) dx for w = src (W space)
  auto recover = [&](const double* src, double th) {
    interp(src);
    __syncthreads();
    for (int i = tid; i < nT * NQ; i += CBLOCK) {
      const int e = i / NQ, q = i - e * NQ;
      const double* Q = geo_of(e) + q * 5;
      double b[2], w[NC], u[NC];
      front_grad(e, q, th, Q, b);
#pragma unroll
      for (int c = 0; c < NC; ++c) w[c] = sQ[(e * NQ + q) * NC + c];
      ok &= kinv<2>(b, sEM[2 * e], sEM[2 * e + 1], w, u);
#pragma unroll
      for (int c = 0; c < NC; ++c) sQ[(e * NQ + q) * NC + c] = Q[0] * u[c];
    }
    __syncthreads();
    project(sU, false, 0.0);
  };

  for (int i = 0; i < kp.m; ++i) {
    const double th = i * invm;
    recover(sS, th);
    double coef = 1.0;
    for (int n = 1; n <= kp.q; ++n) {
      coef *= invm / n;
      // ---- R = A U: values at the volume points and the face fluxes
      interp(sU);
      for (int i2 = tid; i2 < nT * 2 * NFQ; i2 += CBLOCK) {
        const int e = i2 / (2 * NFQ), r = i2 - e * 2 * NFQ, s = r / NFQ, q = r - s * NFQ;
        const int f = sFf[e * 2 + s], pe = sNb[e * 2 + s], code = sNc[e * 2 + s];
        const double* Fq = geo_of(e) + NQ * 5 + NP * NP + (f * NFQ + q) * 3;
        double um[NC] = {0.0, 0.0, 0.0}, up[NC] = {0.0, 0.0, 0.0}, G[NC];
        for (int a = 0; a < NP; ++a) {
          const double ph = Vf[(f * NFQ + q) * NP + a];
#pragma unroll
          for (int c = 0; c < NC; ++c) um[c] = fma(ph, sU[(e * NC + c) * NP + a], um[c]);
        }
        if (pe >= 0) {
          const int fn = code & 3, qn = (code & 4) ? NFQ - 1 - q : q;
          for (int a = 0; a < NP; ++a) {
            const double ph = Vf[(fn * NFQ + qn) * NP + a];
#pragma unroll
            for (int c = 0; c < NC; ++c) up[c] = fma(ph, sU[(pe * NC + c) * NP + a], up[c]);
          }
        } else if (pe == -1 - 1) {   // PMC mirror: E_out = E_in, H_out = -H_in
          up[0] = um[0];
          up[1] = um[1];
          up[2] = -um[2];
        } else {                     // PEC mirror: E_out = -E_in, H_out = H_in
          up[0] = -um[0];
          up[1] = -um[1];
          up[2] = um[2];
        }
        const double nrm[2] = {Fq[1], Fq[2]};
        flux<2>(nrm, kp.alpha, um, up, G);
        const double wl = H * Fq[0] * Lamf[(f * NFQ + q) * 3 + sK[e]];
#pragma unroll
        for (int c = 0; c < NC; ++c) sFx[((e * 2 + s) * NFQ + q) * NC + c] = wl * G[c];
      }
      __syncthreads();
      // volume and lift into sR
      for (int base = 0; base < nT * NP; base += CBLOCK / TEAM) {
        const int i2 = base + tid / TEAM, part = tid % TEAM;
        if (i2 < nT * NP) {   // uniform over the team
          const int e = i2 / NP, b = i2 - e * NP;
          const double* Qe = geo_of(e);
          const int k = sK[e];
          double R[NC] = {0.0, 0.0, 0.0};
          for (int q = part; q < NQ; q += TEAM) {
            const double* Q = Qe + q * 5;
            const double gl0 = Gr[(q * NP + b) * 2], gl1 = Gr[(q * NP + b) * 2 + 1];
            const double g[2] = {Q[1] * gl0 + Q[3] * gl1, Q[2] * gl0 + Q[4] * gl1};   // grad phi_b
            double AU[NC];
            applyA<2>(g, &sQ[(e * NQ + q) * NC], AU);
            const double w = H * Q[0] * Lam[q * 3 + k];
#pragma unroll
            for (int c = 0; c < NC; ++c) R[c] = fma(w, AU[c], R[c]);
          }
          for (int r = part; r < 2 * NFQ; r += TEAM) {
            const int s = r / NFQ, q = r - s * NFQ;
            const double ph = Vf[(sFf[e * 2 + s] * NFQ + q) * NP + b];
#pragma unroll
            for (int c = 0; c < NC; ++c) R[c] = fma(-ph, sFx[((e * 2 + s) * NFQ + q) * NC + c], R[c]);
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) R[c] = team_sum(R[c]);
          if (part == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) sR[(e * NC + c) * NP + b] = R[c];
          }
        }
      }
      __syncthreads();
      // ---- W_n = Minv R, Taylor sum
      for (int i2 = tid; i2 < nT * NP; i2 += CBLOCK) {
        const int e = i2 / NP, b = i2 - e * NP;
        const double* Mi = geo_of(e) + NQ * 5 + b * NP;
        double v[NC] = {0.0, 0.0, 0.0};
        for (int a = 0; a < NP; ++a) {
#pragma unroll
          for (int c = 0; c < NC; ++c) v[c] = fma(Mi[a], sR[(e * NC + c) * NP + a], v[c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          sWn[(e * NC + c) * NP + b] = v[c];
          sS[(e * NC + c) * NP + b] = fma(coef, v[c], sS[(e * NC + c) * NP + b]);
        }
      }
      __syncthreads();
      if (n < kp.q) {
        // W_n + n Minv int phi A(b') U, then the recovery at th
        for (int i2 = tid; i2 < nT * NQ; i2 += CBLOCK) {
          const int e = i2 / NQ, q = i2 - e * NQ;
          const double* Q = geo_of(e) + q * 5;
          const int k = sK[e];
          const double bp[2] = {H * (Q[1] * hat(k, 0) + Q[3] * hat(k, 1)),
                                H * (Q[2] * hat(k, 0) + Q[4] * hat(k, 1))};
          double AU[NC];
          applyA<2>(bp, &sQ[(e * NQ + q) * NC], AU);
#pragma unroll
          for (int c = 0; c < NC; ++c) sQ[(e * NQ + q) * NC + c] = Q[0] * AU[c];
        }
        __syncthreads();
        project(sWn, true, (double)n);
        recover(sWn, th);
      }
    }
  }

  // ---- scatter the tent top
  for (int i = tid; i < nT * NC * NP; i += CBLOCK) {
    const int e = i / (NC * NP), r = i - e * NC * NP;
    kp.W[(size_t)sEl[e] * NC * NP + r] = sS[i];
  }
  if (!ok) kp.err[0] = ERRF_CAUSALITY;
  __syncthreads();
  if (tid == 0) kp.tau[V] = t_top;
}

template <int P>
hipError_t launch_p(const KernelParams& kp, const CurvedParams& cp, int64_t first, int64_t count, hipStream_t s) {
  if (count < 0) {   // set the kernel's dynamic LDS limit
    return hipFuncSetAttribute(reinterpret_cast<const void*>(tent_curved_kernel<P>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)cp.lds);
  }
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(tent_curved_kernel<P>, dim3((unsigned)count), dim3(CBLOCK), cp.lds, s, kp, cp, first);
  return hipGetLastError();
}

}  // namespace

size_t tent_curved_lds_bytes(int p, int max_patch, bool geo) {
  switch (p) {
    case 1: return lds_bytes<1>(max_patch, geo);
    case 2: return lds_bytes<2>(max_patch, geo);
    case 3: return lds_bytes<3>(max_patch, geo);
    case 4: return lds_bytes<4>(max_patch, geo);
    default: return 0;
  }
}

// count < 0: only set the kernel attributes
hipError_t launch_tent_curved(const KernelParams& kp, const CurvedParams& cp, int64_t first, int64_t count,
                              hipStream_t s) {
  switch (cp.p) {
    case 1: return launch_p<1>(kp, cp, first, count, s);
    case 2: return launch_p<2>(kp, cp, first, count, s);
    case 3: return launch_p<3>(kp, cp, first, count, s);
    case 4: return launch_p<4>(kp, cp, first, count, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mtp
