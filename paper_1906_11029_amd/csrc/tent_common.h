// Device helpers shared by the tent kernels: the Maxwell flux matrix A(g), the
// closed-form inverse of the tent-map mass form, the upwind flux and the boundary ghosts.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace mtp {

template <int D> struct Dims;
template <> struct Dims<2> { static constexpr int NC = 3; };
template <> struct Dims<3> { static constexpr int NC = 6; };

__host__ __device__ constexpr int binom_c(int n, int k) {
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// A(g) u = f(u) g : 3D (H x g, g x E);  2D TE (-g_y Hz, g_x Hz, g_x Ey - g_y Ex)
template <int D>
__device__ __forceinline__ void applyA(const double* g, const double* u, double* out);
template <>
__device__ __forceinline__ void applyA<3>(const double* g, const double* u, double* out) {
  const double Ex = u[0], Ey = u[1], Ez = u[2], Hx = u[3], Hy = u[4], Hz = u[5];
  out[0] = Hy * g[2] - Hz * g[1];
  out[1] = Hz * g[0] - Hx * g[2];
  out[2] = Hx * g[1] - Hy * g[0];
  out[3] = g[1] * Ez - g[2] * Ey;
  out[4] = g[2] * Ex - g[0] * Ez;
  out[5] = g[0] * Ey - g[1] * Ex;
}
template <>
__device__ __forceinline__ void applyA<2>(const double* g, const double* u, double* out) {
  out[0] = -g[1] * u[2];
  out[1] = g[0] * u[2];
  out[2] = g[0] * u[1] - g[1] * u[0];
}

// Closed-form inverse of u -> g(u) - f(u) b  (section 4):
//   E = s (I - b b^T/(eps mu)) (mu w_E + w_H x b),  H = s (I - b b^T/(eps mu)) (eps w_H - w_E x b),
//   s = 1/(eps mu - |b|^2).  Returns false if eps mu - |b|^2 <= 0 (causality violated).
// The two scalars of the inverse depend only on b and the medium: f = (s, 1/(eps mu)).
// Returns false if eps mu - |b|^2 <= 0 (causality violated).
template <int D>
__device__ __forceinline__ bool kinv_fac(const double* b, double eps, double mu, double* f) {
  const double em = eps * mu;
  double bb = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) bb += b[i] * b[i];
  const double den = em - bb;
  f[0] = 1.0 / den;
  f[1] = 1.0 / em;
  return den > 0.0;
}
template <int D>
__device__ __forceinline__ void kinv_apply(const double* b, double eps, double mu, const double* f, const double* w,
                                           double* u);
template <>
__device__ __forceinline__ void kinv_apply<3>(const double* b, double eps, double mu, const double* f, const double* w,
                                              double* u) {
  const double s = f[0], iem = f[1];
  double rE[3], rH[3];
  rE[0] = mu * w[0] + (w[4] * b[2] - w[5] * b[1]);
  rE[1] = mu * w[1] + (w[5] * b[0] - w[3] * b[2]);
  rE[2] = mu * w[2] + (w[3] * b[1] - w[4] * b[0]);
  rH[0] = eps * w[3] - (w[1] * b[2] - w[2] * b[1]);
  rH[1] = eps * w[4] - (w[2] * b[0] - w[0] * b[2]);
  rH[2] = eps * w[5] - (w[0] * b[1] - w[1] * b[0]);
  const double pE = (b[0] * rE[0] + b[1] * rE[1] + b[2] * rE[2]) * iem;
  const double pH = (b[0] * rH[0] + b[1] * rH[1] + b[2] * rH[2]) * iem;
  for (int i = 0; i < 3; ++i) {
    u[i] = s * (rE[i] - b[i] * pE);
    u[3 + i] = s * (rH[i] - b[i] * pH);
  }
}
template <>
__device__ __forceinline__ void kinv_apply<2>(const double* b, double eps, double mu, const double* f, const double* w,
                                              double* u) {
  const double s = f[0], iem = f[1];
  const double rx = mu * w[0] - w[2] * b[1];
  const double ry = mu * w[1] + w[2] * b[0];
  const double pE = (b[0] * rx + b[1] * ry) * iem;
  u[0] = s * (rx - b[0] * pE);
  u[1] = s * (ry - b[1] * pE);
  u[2] = s * (eps * w[2] - (w[0] * b[1] - w[1] * b[0]));
}
template <int D>
__device__ __forceinline__ bool kinv(const double* b, double eps, double mu, const double* w, double* u) {
  double f[2];
  const bool ok = kinv_fac<D>(b, eps, mu, f);
  kinv_apply<D>(b, eps, mu, f, w, u);
  return ok;
}

// Upwind flux times |g| for the outward direction g = -grad lambda_j (unnormalised):
//   G = 1/2 A(g)(u_in + u_out) + alpha |g| P_t (u_in - u_out),   P_t = tangential part.
template <int D>
__device__ __forceinline__ void flux(const double* g, double alpha, const double* um, const double* up, double* G);
// The face scalars fs = (|g|, 1/|g|^2) depend only on the face: face_scalars forms them once.
template <int D>
__device__ __forceinline__ void face_scalars(const double* g, double* fs) {
  double gg = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) gg += g[i] * g[i];
  fs[0] = sqrt(gg);
  fs[1] = 1.0 / gg;
}
template <int D>
__device__ __forceinline__ void flux_f(const double* g, const double* fs, double alpha, const double* um,
                                       const double* up, double* G);
template <int D>
__device__ __forceinline__ void flux(const double* g, double alpha, const double* um, const double* up, double* G) {
  double fs[2];
  face_scalars<D>(g, fs);
  flux_f<D>(g, fs, alpha, um, up, G);
}
template <>
__device__ __forceinline__ void flux_f<3>(const double* g, const double* fs, double alpha, const double* um,
                                          const double* up, double* G) {
  double s[6], dlt[6];
  for (int c = 0; c < 6; ++c) { s[c] = 0.5 * (um[c] + up[c]); dlt[c] = um[c] - up[c]; }
  applyA<3>(g, s, G);
  const double gn = fs[0];
  const double ig = fs[1];
  const double nE = (g[0] * dlt[0] + g[1] * dlt[1] + g[2] * dlt[2]) * ig;
  const double nH = (g[0] * dlt[3] + g[1] * dlt[4] + g[2] * dlt[5]) * ig;
  const double ag = alpha * gn;
  for (int i = 0; i < 3; ++i) {
    G[i] += ag * (dlt[i] - nE * g[i]);
    G[3 + i] += ag * (dlt[3 + i] - nH * g[i]);
  }
}
template <>
__device__ __forceinline__ void flux_f<2>(const double* g, const double* fs, double alpha, const double* um,
                                          const double* up, double* G) {
  double s[3], dlt[3];
  for (int c = 0; c < 3; ++c) { s[c] = 0.5 * (um[c] + up[c]); dlt[c] = um[c] - up[c]; }
  applyA<2>(g, s, G);
  const double gn = fs[0];
  const double nE = (g[0] * dlt[0] + g[1] * dlt[1]) * fs[1];
  const double ag = alpha * gn;
  G[0] += ag * (dlt[0] - nE * g[0]);
  G[1] += ag * (dlt[1] - nE * g[1]);
  G[2] += ag * dlt[2];
}

// Impedance-matched upwind flux across a material interface: G = A(g) u* with u* the
// interface state of the one-dimensional Riemann problem along n = g/|g| (tangential E
// and H continuous, each side's incoming wave from its own state), impedances
// zm = sqrt(mu/eps) of the "in" side and zp of the other:
//   E* = (zp E_in + zm E_out - zm zp n x (H_in - H_out)) / (zm + zp)
//   H* = (zm H_in + zp H_out + n x (E_in - E_out)) / (zm + zp)
// (normal parts of E*, H* drop out of A(g)).  zm = zp = 1 gives the alpha = 1/2 flux.
template <int D>
__device__ __forceinline__ void flux_imp(const double* g, const double* fs, double zm, double zp, const double* um,
                                         const double* up, double* G);
template <>
__device__ __forceinline__ void flux_imp<3>(const double* g, const double* fs, double zm, double zp,
                                            const double* um, const double* up, double* G) {
  const double in = fs[0] * fs[1];   // 1/|g|
  const double n[3] = {g[0] * in, g[1] * in, g[2] * in};
  const double dE[3] = {um[0] - up[0], um[1] - up[1], um[2] - up[2]};
  const double dH[3] = {um[3] - up[3], um[4] - up[4], um[5] - up[5]};
  const double nxdH[3] = {n[1] * dH[2] - n[2] * dH[1], n[2] * dH[0] - n[0] * dH[2], n[0] * dH[1] - n[1] * dH[0]};
  const double nxdE[3] = {n[1] * dE[2] - n[2] * dE[1], n[2] * dE[0] - n[0] * dE[2], n[0] * dE[1] - n[1] * dE[0]};
  const double is = 1.0 / (zm + zp), zz = zm * zp;
  double us[6];
  for (int i = 0; i < 3; ++i) {
    us[i] = (zp * um[i] + zm * up[i] - zz * nxdH[i]) * is;
    us[3 + i] = (zm * um[3 + i] + zp * up[3 + i] + nxdE[i]) * is;
  }
  applyA<3>(g, us, G);
}
template <>
__device__ __forceinline__ void flux_imp<2>(const double* g, const double* fs, double zm, double zp,
                                            const double* um, const double* up, double* G) {
  // TE: E in the plane, H = Hz e_z; n x (Hz e_z) = Hz (n_y, -n_x), (n x E)_z = n_x Ey - n_y Ex
  const double in = fs[0] * fs[1];
  const double nx = g[0] * in, ny = g[1] * in;
  const double dHz = um[2] - up[2];
  const double nxdE = nx * (um[1] - up[1]) - ny * (um[0] - up[0]);
  const double is = 1.0 / (zm + zp), zz = zm * zp;
  const double us[3] = {(zp * um[0] + zm * up[0] - zz * ny * dHz) * is,
                        (zp * um[1] + zm * up[1] + zz * nx * dHz) * is,
                        (zm * um[2] + zp * up[2] + nxdE) * is};
  applyA<2>(g, us, G);
}

// ---------------------------------------------------------------- acoustics
// Linear acoustics kappa p_t + div v = 0, rho v_t + grad p = 0 in the same conservation form
// d_t g(u) + div f(u) = 0: u = (p, v), g(u) = (kappa p, rho v), f(u) n = A(n) u = (v.n, p n).
// The two per-element coefficients are (kappa, rho) in the slots of (eps, mu); the wave
// speed is 1/sqrt(kappa rho) and the impedance Z = sqrt(rho/kappa), as for Maxwell.
template <int D>
__device__ __forceinline__ void applyA_ac(const double* g, const double* u, double* out) {
  double vg = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    vg += g[i] * u[1 + i];
    out[1 + i] = g[i] * u[0];
  }
  out[0] = vg;
}

// Closed-form inverse of u -> g(u) - f(u) b = (kappa p - v.b, rho v - p b):
//   p = (rho w_p + b.w_v) / (kappa rho - |b|^2),  v = (w_v + p b) / rho.
template <int D>
__device__ __forceinline__ bool kinv_ac_fac(const double* b, double kappa, double rho, double* f) {
  double bb = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) bb += b[i] * b[i];
  const double den = kappa * rho - bb;
  f[0] = 1.0 / den;
  f[1] = 1.0 / rho;
  return den > 0.0;
}
template <int D>
__device__ __forceinline__ void kinv_ac_apply(const double* b, double kappa, double rho, const double* f,
                                              const double* w, double* u) {
  double bw = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) bw += b[i] * w[1 + i];
  const double p = (rho * w[0] + bw) * f[0];
  u[0] = p;
#pragma unroll
  for (int i = 0; i < D; ++i) u[1 + i] = (w[1 + i] + p * b[i]) * f[1];
}
template <int D>
__device__ __forceinline__ bool kinv_ac(const double* b, double kappa, double rho, const double* w, double* u) {
  double f[2];
  const bool ok = kinv_ac_fac<D>(b, kappa, rho, f);
  kinv_ac_apply<D>(b, kappa, rho, f, w, u);
  return ok;
}

// Upwind flux times |g|:  1/2 A(g)(u_in + u_out) + alpha |g| (dp, (dv.n) n),  d = in - out
// (alpha = 1/2: the exact upwind flux for unit impedance).
template <int D>
__device__ __forceinline__ void flux_ac(const double* g, const double* fs, double alpha, const double* um,
                                        const double* up, double* G) {
  double s[D + 1];
#pragma unroll
  for (int c = 0; c <= D; ++c) s[c] = 0.5 * (um[c] + up[c]);
  applyA_ac<D>(g, s, G);
  double dvg = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) dvg += g[i] * (um[1 + i] - up[1 + i]);
  const double gn = fs[0], ign = fs[0] * fs[1];   // |g|, 1/|g|
  G[0] += alpha * gn * (um[0] - up[0]);
#pragma unroll
  for (int i = 0; i < D; ++i) G[1 + i] += alpha * (dvg * ign) * g[i];
}

// Impedance-matched upwind flux: A(g) u* with the interface state of the Riemann problem
// along n = g/|g|:  p* = (zp p_in + zm p_out + zm zp (v_in - v_out).n) / (zm + zp),
// v*.n = (zm v_in.n + zp v_out.n + p_in - p_out) / (zm + zp).
template <int D>
__device__ __forceinline__ void flux_imp_ac(const double* g, const double* fs, double zm, double zp,
                                            const double* um, const double* up, double* G) {
  double vmg = 0.0, vpg = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    vmg += g[i] * um[1 + i];
    vpg += g[i] * up[1 + i];
  }
  const double gn = fs[0], ign = fs[0] * fs[1], is = 1.0 / (zm + zp);
  const double ps = (zp * um[0] + zm * up[0] + zm * zp * (vmg - vpg) * ign) * is;
  const double vns = (zm * vmg + zp * vpg) * ign * is + (um[0] - up[0]) * is;
  G[0] = gn * vns;
#pragma unroll
  for (int i = 0; i < D; ++i) G[1 + i] = ps * g[i];
}

// ---------------------------------------------------------------- physics trait
// SYS 0: Maxwell, u = (E, H); SYS 1: acoustics, u = (p, v).  NC fields, the first NE of
// which form the first group (E, or p: negated by a kind-0 wall, the second group by a
// kind-1 wall); component c of A(g) u = sum over NTERM terms s g[q] u[p].
template <int D, int SYS> struct Phys;
template <int D> struct Phys<D, 0> {
  static constexpr int NC = (D == 3) ? 6 : 3, NE = (D == 3) ? 3 : 2, NTERM = 2;
  static __device__ __forceinline__ void A(const double* g, const double* u, double* o) { applyA<D>(g, u, o); }
  static __device__ __forceinline__ bool inv(const double* b, double c1, double c2, const double* w, double* u) {
    return kinv<D>(b, c1, c2, w, u);
  }
  // the inverse in two steps: its scalars at b (once per element and time), then the map
  static __device__ __forceinline__ bool inv_fac(const double* b, double c1, double c2, double* f) {
    return kinv_fac<D>(b, c1, c2, f);
  }
  static __device__ __forceinline__ void inv_apply(const double* b, double c1, double c2, const double* f,
                                                   const double* w, double* u) {
    kinv_apply<D>(b, c1, c2, f, w, u);
  }
  // fluxes with the face scalars fs = (|g|, 1/|g|^2) of face_scalars
  static __device__ __forceinline__ void fl(const double* g, const double* fs, double a, const double* um,
                                            const double* up, double* G) {
    flux_f<D>(g, fs, a, um, up, G);
  }
  static __device__ __forceinline__ void fl_imp(const double* g, const double* fs, double zm, double zp,
                                                const double* um, const double* up, double* G) {
    flux_imp<D>(g, fs, zm, zp, um, up, G);
  }
};
template <int D> struct Phys<D, 1> {
  static constexpr int NC = D + 1, NE = 1, NTERM = D;
  static __device__ __forceinline__ void A(const double* g, const double* u, double* o) { applyA_ac<D>(g, u, o); }
  static __device__ __forceinline__ bool inv(const double* b, double c1, double c2, const double* w, double* u) {
    return kinv_ac<D>(b, c1, c2, w, u);
  }
  static __device__ __forceinline__ bool inv_fac(const double* b, double c1, double c2, double* f) {
    return kinv_ac_fac<D>(b, c1, c2, f);
  }
  static __device__ __forceinline__ void inv_apply(const double* b, double c1, double c2, const double* f,
                                                   const double* w, double* u) {
    kinv_ac_apply<D>(b, c1, c2, f, w, u);
  }
  static __device__ __forceinline__ void fl(const double* g, const double* fs, double a, const double* um,
                                            const double* up, double* G) {
    flux_ac<D>(g, fs, a, um, up, G);
  }
  static __device__ __forceinline__ void fl_imp(const double* g, const double* fs, double zm, double zp,
                                                const double* um, const double* up, double* G) {
    flux_imp_ac<D>(g, fs, zm, zp, um, up, G);
  }
};

template <int D>
__device__ __forceinline__ void vertex_order_dev(int k, int* order) {
  order[0] = k;
  int c = 1;
#pragma unroll
  for (int i = 0; i <= D; ++i)
    if (i != k) order[c++] = i;
}



// Ghost state on a boundary face of kind 0 (PEC mirror: E_out = -E_in, H_out = H_in;
// acoustics: pressure release, p_out = -p_in), 1 (PMC mirror: E_out = E_in, H_out = -H_in;
// acoustics: rigid wall, v_out = -v_in) or 2 (data: the plane wave
// u_ex(x, phi(x, th)), whose (n-1)-th th-derivative is delta^(n-1) d_t^(n-1) u_ex with
// delta = H lambda_V, evaluated at the face node nin of element el).
template <int D, int P, int SYS = 0>
__device__ __forceinline__ void ghost_state(const KernelParams& kp, int kind, const double* um, double* up,
                                            int el, int kloc, int nin, double H, double th, int n) {
  constexpr int NC = Phys<D, SYS>::NC, NV = D + 1, NE = Phys<D, SYS>::NE;
  if (kind == 2 && kp.has_data) {
    // every multiply-add written as an explicit fma and no other contraction, so that the
    // data do not depend on how a kernel instantiation schedules this code
#pragma clang fp contract(off)
    int order[NV];
    vertex_order_dev<D>(kloc, order);
    double x[D], phib = 0.0;
#pragma unroll
    for (int xx = 0; xx < D; ++xx) x[xx] = 0.0;
    const int* alpha = kp.mi + nin * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int gv = kp.cells[(size_t)el * NV + order[v]];
      const double lam = (double)alpha[v] / P;
      phib = fma(lam, kp.tau[gv], phib);
#pragma unroll
      for (int xx = 0; xx < D; ++xx) x[xx] = fma(lam, kp.coords[(size_t)gv * D + xx], x[xx]);
    }
    const double delta = H * ((double)alpha[0] / P);
    const double phi = fma(th, delta, phib);
    double psi = fma(-kp.pw_omega, phi, kp.pw_phase);
#pragma unroll
    for (int xx = 0; xx < D; ++xx) psi = fma(kp.pw_k[xx], x[xx], psi);
    const int kd = n - 1;
    double scale = 1.0;
    for (int z = 0; z < kd; ++z) scale *= delta * kp.pw_omega;
    // d_t^k cos = omega^k cos(. - k pi/2)
    const double val = scale * cos(fma(-(double)kd, 1.5707963267948966, psi));
#pragma unroll
    for (int c = 0; c < NC; ++c) up[c] = kp.pw_amp[c] * val;
  } else if (kind == 1) {
#pragma unroll
    for (int c = 0; c < NC; ++c) up[c] = (c < NE) ? um[c] : -um[c];
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) up[c] = (c < NE) ? -um[c] : um[c];
  }
}

}  // namespace mtp
