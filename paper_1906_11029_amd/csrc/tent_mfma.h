// MFMA tent kernel for gfx950: the same per-tent SAT evolution as the VALU kernel, with
// the per-stage contraction of every patch element done as one matrix product on the
// matrix cores:
//
//   R = [ S_1 .. S_d | -L_1 .. -L_d ] . [ A(grad lambda_1) U ; .. ; A(grad lambda_d) U ; F ]
//        (np x (d np + d nf))              ((d np + d nf) x (nc nT))
//
// with U the patch state (node-major, one column per (element, component)), F the upwind
// face fluxes at the face nodes of the faces containing the tent vertex, and R the mass-
// divided right-hand side dY/dth / H of every node.  A(grad lambda_l) U is formed while
// loading the B operand (two LDS reads and two multiply-adds per value: A(g) is a cross
// product), so only U and F are stored.  Accumulators stay in registers until every wave
// has finished reading F, then R overwrites F in LDS.  The plain path (T = double) runs
// every product on v_mfma_f64_16x16x4f64, and at most 4 rows beyond the full 16-row tiles
// on v_mfma_f64_4x4x4f64.  The mixed path (T = float) keeps the same FP64 storage (plus an
// FP32 copy of the operator's volume part) and FP64 first stage of every sub-interval,
// and runs the products of the later stages, which act on the small Taylor coefficients
// U_{i,n} (n >= 1), on v_mfma_f32_16x16x4f32 / v_mfma_f32_4x4x1f32; the closed-form
// inverses, fluxes and the Taylor sum stay FP64.
//
// Internal header: the kernel templates and their launchers.  Every (dimension, degree,
// precision) is instantiated in exactly one translation unit (tent_mfma_<d>d*.hip, see
// MTP_MFMA_CONFIGS); tent_mfma.hip holds the dispatch on (d, p, precision).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "kernels.h"
#include "tent_common.h"

namespace mtp {
namespace mfk {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc_t = v4d;
  // output value r of lane l sits in row l/16 + 4 r (measured lane layout)
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // 4-row product on v_mfma_f64_4x4x4f64 (4 blocks of 4 columns, a quarter of the 16x16x4
  // cycles): lane l supplies A(row l%4, k = l/16) and the same B value as for the 16x16x4
  // shape (k = l/16, column l%16); lane l receives (row l/16, column l%16)  (measured)
  using mini_t = double;
  static __device__ __forceinline__ mini_t mini(double a, double b, mini_t c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ double mini_out(mini_t c, int) { return c; }
};
template <> struct Mfma<float> {
  using acc_t = v4f;
  // output value r of lane l sits in row 4 (l/16) + r
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // 4-row product on v_mfma_f32_4x4x1f32 (16 blocks of 4 x 4 x 1, a quarter of the 16x16x4
  // cycles): block l/4 takes A(row l%4) and B from lane l, so with the 16x16x4 operands
  // (k = l/16, column l%16) block (k, column group) accumulates the part of the sum over
  // k = l/16 mod 4; value r of lane l is (row r, column l%16) of that part  (measured).
  // The four parts are added across lanes l, l^16, l^32, l^48 at the end.
  using mini_t = v4f;
  static __device__ __forceinline__ mini_t mini(float a, float b, mini_t c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
  }
  // row lane/16, column lane%16 of the 4-row product.  The cross-lane sums use the
  // register swaps of gfx950 (v_permlane16_swap / v_permlane32_swap: the two results hold
  // x[l] and x[l ^ 16], resp. x[l ^ 32], in some order; measured), not LDS permutes.
  static __device__ __forceinline__ float xor_sum(float x, bool by32) {
    const unsigned u = __float_as_uint(x);
    const auto p = by32 ? __builtin_amdgcn_permlane32_swap(u, u, false, false)
                        : __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
  static __device__ __forceinline__ double mini_out(mini_t c, int lane) {
#pragma unroll
    for (int r = 0; r < 4; ++r) c[r] = xor_sum(xor_sum(c[r], false), true);
    const int r = lane >> 4;
    return (double)(r == 0 ? c[0] : r == 1 ? c[1] : r == 2 ? c[2] : c[3]);
  }
};

// component c of A(g) u = sum_t s[t] g[q[t]] u[p[t]] over the system's NTERM terms, from
// nibble tables (no branches)
template <int D, int SYS> struct ACoef;
template <> struct ACoef<3, 0> {
  // Maxwell, g x H and -(g x E) with u = (E, H):  P1 = {4,5,3,2,0,1}, Q1 = {2,0,1,1,2,0},
  // P2 = {5,3,4,1,2,0}, Q2 = {1,2,0,2,0,1}, s1 = +1, s2 = -1
  static __device__ __forceinline__ void get(int c, int* p, int* q, double* s) {
    p[0] = (0x102354 >> (4 * c)) & 15;
    q[0] = (0x021102 >> (4 * c)) & 15;
    p[1] = (0x021435 >> (4 * c)) & 15;
    q[1] = (0x102021 >> (4 * c)) & 15;
    s[0] = 1.0;
    s[1] = -1.0;
  }
};
template <> struct ACoef<2, 0> {
  // Maxwell TE, (-g1 Hz, g0 Hz, g0 Ey - g1 Ex) with u = (Ex, Ey, Hz)
  static __device__ __forceinline__ void get(int c, int* p, int* q, double* s) {
    p[0] = (0x122 >> (4 * c)) & 15;
    q[0] = (0x001 >> (4 * c)) & 15;
    p[1] = (0x022 >> (4 * c)) & 15;
    q[1] = (0x110 >> (4 * c)) & 15;
    s[0] = (c == 0) ? -1.0 : 1.0;
    s[1] = (c == 2) ? -1.0 : 0.0;
  }
};
template <int D> struct ACoef<D, 1> {
  // acoustics, (g.v, g_0 p, .., g_{D-1} p) with u = (p, v)
  static __device__ __forceinline__ void get(int c, int* p, int* q, double* s) {
#pragma unroll
    for (int t = 0; t < D; ++t) {
      p[t] = (c == 0) ? 1 + t : 0;
      q[t] = (c == 0) ? t : c - 1;
      s[t] = (c == 0 || t == 0) ? 1.0 : 0.0;
    }
  }
};

// Threads per workgroup: 3D, 8 waves (2 per SIMD), one tent per CU; 2D tents are small
// (a few triangles): 2 waves, so that several tents share a CU.
template <int D>
__host__ __device__ constexpr int tent_block() { return D == 2 ? 128 : 512; }

template <int D, int P, int NTMAX, int SYS = 0>
struct MShape {
  static constexpr int NC = Phys<D, SYS>::NC;
  static constexpr int NP = binom_c(P + D, D);
  static constexpr int NF = binom_c(P + D - 1, D - 1);
  static constexpr int NV = D + 1;
  static constexpr int NPK = (NP + 3) / 4 * 4;            // one volume block of K (padded)
  static constexpr int KV = D * NPK;                      // volume part of K
  static constexpr int KF = D * NF;                       // lift part of K
  static constexpr int KFP = (KF + 3) / 4 * 4;            // lift part padded to the MFMA depth
  static constexpr int KT = KV + KFP;
  static constexpr int MT = (NP + 15) / 16;               // 16-row tiles of R
  static constexpr int MP = MT * 16;
  // a last M-tile of at most 4 rows (P4 and P3 in 3D) runs on the 4-row MFMA shape, in the
  // same pass as the last full tile of its column block (same B operand)
  static constexpr bool MINI = NP > 16 && NP % 16 >= 1 && NP % 16 <= 4;
  static constexpr int MTF = MINI ? NP / 16 : MT;         // 16-row tiles run as such
  static constexpr int NCOL = (NC * NTMAX + 15) / 16 * 16;  // columns (element, component)
  static constexpr int RS = NCOL + 1;   // row stride of U and F/R: odd, so that threads owning
                                        // consecutive nodes of one element hit distinct banks
  static constexpr int NTILE_MAX = NCOL / 16;
  // F during the product (KF rows: the lift part's last K step clamps its rows beyond KF,
  // which meet zero operator columns), R after (up to MP rows, 16 MTF + 4 with the 4-row part)
  static constexpr int RROWS = MINI ? MTF * 16 + 4 : MP;
  static constexpr int FROWS = (KF > RROWS) ? KF : RROWS;
  static constexpr int BLOCK = tent_block<D>();
  static constexpr int WAVES = BLOCK / 64;
  static constexpr int TILES_PER_WAVE = (MTF * NTILE_MAX + WAVES - 1) / WAVES;
  static constexpr int MAXPAIR = (NTMAX * NP + BLOCK - 1) / BLOCK;
  // P4 patches of more than 24 tets and P5 in 3D (up to 28 or 36 product tiles on 8 waves): each wave takes whole
  // column blocks and writes their R at once, so only one column block's row tiles hold
  // accumulators (4 tiles per wave do not fit the registers), and the Taylor sum of each
  // (element, node) pair stays in the tent's own entries of W (the pair belongs to one
  // thread for the whole tent) instead of registers
  static constexpr bool COLB = D == 3 && ((P == 4 && NTMAX > 24) || P >= 5);
  static constexpr bool ACCG = COLB;
};

// The capacity classes of the patch size: 8, 24, and a large class of 48 tets, or 36 for
// P4 in 3D (the largest whose tent region fits the LDS once the operator block is moved out)
// and 24 for P5 in 3D; these two have a further, extra-large class of 48 (F/R in device
// memory, and at P5 the operator block too).
template <int D, int P>
__host__ __device__ constexpr int big_class() { return D == 3 ? (P == 4 ? 36 : P >= 5 ? 24 : 48) : 48; }
template <int D, int P>
__host__ __device__ constexpr int xl_class() { return D == 3 && (P == 4 || P == 5) ? 48 : -1; }

// LDS layout, identical for both variants (state, fluxes and operators stored in FP64; the
// mixed variant only changes the precision of the products of stages n >= 2): an operator
// block (FP64 operator, in the mixed kernel the FP32 copy of its volume part, the face-node
// tables), which depends on the degree only, then the region of one tent (U, F/R, geometry).
template <int D, int P, typename T, int NTMAX, int SYS = 0>
struct MLds {
  using SH = MShape<D, P, NTMAX, SYS>;
  static constexpr int OPS = SH::RROWS;   // operator rows read by the products
  // FP64 operator, then (mixed kernel) the FP32 copy of its volume part, in doubles
  static constexpr size_t opf_floats = sizeof(T) == 4 ? (size_t)SH::KV * OPS : 0;
  static constexpr size_t op_elems = (size_t)SH::KT * OPS + (opf_floats + 1) / 2;
  static constexpr size_t face_ints = (size_t)D * 2 * SH::NF + SH::NF;
  static constexpr size_t op_block = op_elems + (face_ints + 1) / 2;   // doubles
  static constexpr size_t u_elems = (size_t)SH::NPK * SH::RS;
  static constexpr size_t f_elems = (size_t)SH::FROWS * SH::RS;
  static constexpr size_t geo_doubles =
      (size_t)NTMAX * (SH::NV * D + D + 2) + 3 * (size_t)NTMAX * D + 4 * (size_t)NTMAX;
  static constexpr size_t tent_ints = (size_t)NTMAX * (2 + D) + (size_t)NTMAX * D;
  static constexpr size_t common = u_elems + f_elems + geo_doubles + (tent_ints + 1) / 2;   // doubles
  // An operator block that does not fit beside the tent region (P4 patches of more than 24
  // tets) stays in device memory, written once per solver (KernelParams::opg); the products
  // then read their A operand through the caches.
  static constexpr size_t LDS_LIMIT = 160 * 1024;
  // The extra-large class (P4 patches of 37-48 tets in 3D) keeps the operator block in LDS
  // and moves F/R instead, a slot of f_elems doubles per workgroup (KernelParams::frg): F/R
  // is the B operand of the lift part only and the input of the pointwise update, read far
  // less often than the operator.
  static constexpr bool FRG = NTMAX == xl_class<D, P>();
  static constexpr size_t lds_common = common - (FRG ? f_elems : 0);   // the tent region in LDS
  static constexpr bool OPG = (op_block + lds_common) * 8 > LDS_LIMIT && lds_common * 8 <= LDS_LIMIT;
  static constexpr size_t frg_doubles = FRG ? f_elems : 0;
  static constexpr size_t bytes = ((OPG ? 0 : op_block) + lds_common) * 8;
};

// LDS pointers of one degree's operator block and of the tent region
struct TentLds {
  double* sOp;     // [k][m], m fastest
  float* sOpF;     // mixed: FP32 copy of the volume rows k < KV
  int* sFn;        // face node -> volume node, [j][o][s]
  int* sFsw;       // [s]: face node with the two non-V vertices exchanged
  double* sU;      // [node][col]
  double* sFR;     // [row][col]: F, then R
  double* sGL;     // [e][v][x]
  double* sBb;     // [e][x]
  double* sEM;     // [e][2]
  double* sRat;    // [face]: -|grad lambda_jn| / |grad lambda_j|
  double* sFs;     // [face][2]: |g|, 1/|g|^2 of the face direction g
  double* sFac;    // [slot][e][2]: scalars of K(b(th))^{-1}, th = i / m
  int* sElem;
  int* sK;
  int* sF;
  int* sPF;        // [face]: patch face code (element << 2 | face)
};

// op: the operator block; common: the tent region in LDS; fr: the workgroup's F/R slot in
// device memory (classes with MLds::FRG only)
template <int D, int P, typename T, int NTMAX, int SYS>
__device__ __forceinline__ TentLds tent_lds(double* op, double* common, double* fr) {
  using SH = MShape<D, P, NTMAX, SYS>;
  using LD = MLds<D, P, T, NTMAX, SYS>;
  constexpr int NV = SH::NV;
  TentLds L;
  L.sOp = op;
  L.sOpF = reinterpret_cast<float*>(op + SH::KT * LD::OPS);
  L.sFn = reinterpret_cast<int*>(op + LD::op_elems);
  L.sFsw = L.sFn + D * 2 * SH::NF;
  L.sU = common;
  L.sFR = LD::FRG ? fr : L.sU + LD::u_elems;
  L.sGL = L.sU + LD::u_elems + (LD::f_elems - LD::frg_doubles);
  L.sBb = L.sGL + NTMAX * NV * D;
  L.sEM = L.sBb + NTMAX * D;
  L.sRat = L.sEM + NTMAX * 2;
  L.sFs = L.sRat + NTMAX * D;
  L.sFac = L.sFs + 2 * NTMAX * D;
  L.sElem = reinterpret_cast<int*>(L.sFac + 4 * NTMAX);
  L.sK = L.sElem + NTMAX;
  L.sF = L.sK + NTMAX;
  L.sPF = L.sF + NTMAX * D;
  return L;
}

// The operator block of degree P: A operand [k][m] with S_l[m][a] at k = l NPK + a (a < NP),
// -L_j[m][s] at k = KV + j NF + s, zero in the padding rows and columns; the face-node tables.
template <int D, int P, typename T, int NTMAX, int SYS>
__device__ __forceinline__ void stage_operator(const KernelParams& kp0, const TentLds& L, int tid) {
  using SH = MShape<D, P, NTMAX, SYS>;
  constexpr bool MIXED = sizeof(T) == 4;
  constexpr int NP = SH::NP, NF = SH::NF, NPK = SH::NPK, KV = SH::KV, KF = SH::KF, KT = SH::KT;
  constexpr int OPS = MLds<D, P, T, NTMAX, SYS>::OPS, BLOCK = SH::BLOCK;
  for (int i = tid; i < KT * OPS; i += BLOCK) {
    const int k = i / OPS, m = i - k * OPS;
    double v = 0.0;
    if (m < NP) {
      if (k < KV) {
        const int l = k / NPK, a = k - l * NPK;
        if (a < NP) v = kp0.S[(l * NP + a) * NP + m];
      } else if (k < KV + KF) {
        const int j = (k - KV) / NF, s = (k - KV) - j * NF;
        v = -kp0.L[(j * NF + s) * NP + m];
      }
    }
    L.sOp[i] = v;
    if constexpr (MIXED) {
      if (k < KV) L.sOpF[i] = (float)v;
    }
  }
  for (int i = tid; i < D * 2 * NF; i += BLOCK) L.sFn[i] = kp0.fnode[i];
  for (int i = tid; i < NF; i += BLOCK) L.sFsw[i] = kp0.fswap[i];
}


// R = [S | -L] [A(grad lambda) U ; F] for this wave's tiles with TM-precision products
// (operands converted from the FP64 LDS values as they are loaded), written back to
// sFR as FP64 once every wave has finished reading F.  The volume part of K runs node
// block major: the two U values a lane needs for node block `as` serve the D products
// (l = 1..D) of that block, which differ only in the coefficients of A(grad lambda_l).
// The raw LDS operands of the next node block are loaded before the current block's
// products are issued (register ring, no code motion across blocks).  Tiles are numbered
// from the last full M-tile down; when the rows beyond the full tiles are at most 4, the
// tiles of the last full M-tile also run those rows on the 4-row shape with the same B.
// Every wave runs the volume part of K (U only) for all its tiles, then waits for F and
// runs the lift part.
// sOpF (mixed kernel): an FP32 copy of the volume part of the operator (KV rows of OPS);
// the FP32 products read their volume operands from it (half the LDS bytes, no
// conversion), everything else reads the FP64 operator sOp.
// The product's tiles (row block mr, column block nt) = mr * ntiles + nt run by this wave,
// slot by slot (MTF * ntiles, or more, for an empty slot), by the tuned assignment `order`
// (wave-uniform, worked out once per tent; results do not depend on it):
//   0: round robin, except for the full P4 patch (9 column blocks, 9 tiles with the 4-row
//      part and 9 without), where a fixed assignment evens the matrix-core time of the
//      four SIMDs (waves w and w + 4 share one): 5.25 / 5.25 / 5 / 4.75 tile units
//      instead of 5.75 / 5.5 / 4.5 / 4.5 (5-bit entries, 31 = none)
//   1: round robin over the tiles numbered row block first
//   2: blocked, each wave a run of consecutive tiles of that numbering
//   3: round robin over the tiles numbered column block first
template <int D, int P, int NTMAX, int SYS>
__device__ __forceinline__ void tile_assign(int order, int wave, int ntiles,
                                            int (&tiles)[MShape<D, P, NTMAX, SYS>::TILES_PER_WAVE]) {
  using SH = MShape<D, P, NTMAX, SYS>;
  constexpr int MTF = SH::MTF, WAVES = SH::WAVES, TPW = SH::TILES_PER_WAVE;
  constexpr bool MINI = SH::MINI;
  const int ntot = MTF * ntiles;
#pragma unroll
  for (int ts = 0; ts < TPW; ++ts) {
    int t = wave + WAVES * ts;
    if (order == 2) {
      const int per = (ntot + WAVES - 1) / WAVES;
      t = ts < per ? wave * per + ts : ntot;
    } else if (order == 3) {
      const int j = wave + WAVES * ts;
      t = j < ntot ? (j % MTF) * ntiles + j / MTF : ntot;
    } else if (order == 0) {
      if constexpr (MINI && MTF == 2 && WAVES == 8 && TPW == 3) {
        if (ntiles == 9) {
          constexpr uint64_t T0 = 0ull | 1ull << 5 | 2ull << 10 | 4ull << 15 | 13ull << 20 | 15ull << 25 |
                                  6ull << 30 | 8ull << 35;
          constexpr uint64_t T1 = 9ull | 11ull << 5 | 3ull << 10 | 5ull << 15 | 14ull << 20 | 16ull << 25 |
                                  7ull << 30 | 17ull << 35;
          constexpr uint64_t T2 = 10ull | 12ull << 5 | 31ull << 10 | 31ull << 15 | 31ull << 20 | 31ull << 25 |
                                  31ull << 30 | 31ull << 35;
          const uint64_t tab = ts == 0 ? T0 : ts == 1 ? T1 : T2;
          t = (int)((tab >> (5 * wave)) & 31);
        }
      }
    }
    tiles[ts] = __builtin_amdgcn_readfirstlane(t);
  }
}

template <typename TM, int D, int P, int NTMAX, int SYS>
__device__ __forceinline__ void tile_product(const double* sOp, const float* sOpF, const double* sU, double* sFR,
                                             const double* sGL, int wave, int lane, int ncols, int ntiles,
                                             const int (&tiles)[MShape<D, P, NTMAX, SYS>::TILES_PER_WAVE]) {
  using SH = MShape<D, P, NTMAX, SYS>;
  constexpr int NT = Phys<D, SYS>::NTERM;
  using MM = Mfma<TM>;
  constexpr int NC = SH::NC, NV = SH::NV, NPK = SH::NPK, KV = SH::KV, KF = SH::KF, KFP = SH::KFP, MTF = SH::MTF,
                RS = SH::RS, WAVES = SH::WAVES, TPW = SH::TILES_PER_WAVE;
  constexpr bool MINI = SH::MINI;
  constexpr int OPS = MLds<D, P, double, NTMAX, SYS>::OPS;
  constexpr int NB = NPK / 4;              // node blocks of the volume part
  constexpr int NG = NB + KFP / 4;         // K groups: node blocks, then lift steps
  constexpr int PDG = 2;                   // ring depth in K groups
  constexpr bool F32 = sizeof(TM) == 4;
  constexpr bool FRGM = MLds<D, P, double, NTMAX, SYS>::FRG;   // F/R in device memory
  typename MM::acc_t accs[TPW];
  typename MM::mini_t accm[TPW];
#pragma unroll
  for (int ts = 0; ts < TPW; ++ts) {
    accs[ts] = typename MM::acc_t{0, 0, 0, 0};
    accm[ts] = typename MM::mini_t{};
  }
  auto tile_of = [&](int ts) -> int { return tiles[ts]; };
  // K groups [G0, G1) of `tile` into (acc, accmini): the volume part (U only) or the lift part (F)
  auto part = [&](int tile, typename MM::acc_t& acc, typename MM::mini_t& accmini, auto lift) {
    constexpr bool LIFT = decltype(lift)::value;
    constexpr int G0 = LIFT ? NB : 0, G1 = LIFT ? NG : NB;
    if (tile < MTF * ntiles) {
      const int mr = tile / ntiles, nt = tile - mr * ntiles;
      const int mt = MTF - 1 - mr;
      const bool with_mini = MINI && mr == 0;   // wave-uniform
      const int col = nt * 16 + (lane & 15);
      const bool live = col < ncols;
      const int e = live ? col / NC : 0;
      const int c = live ? col - e * NC : 0;
      int pt[NT], qt[NT];
      double st[NT];
      ACoef<D, SYS>::get(c, pt, qt, st);
      TM cf[NT][D];
#pragma unroll
      for (int l = 0; l < D; ++l) {
        const double* gl = &sGL[(e * NV + l + 1) * D];
#pragma unroll
        for (int k = 0; k < NT; ++k) cf[k][l] = (TM)(live ? st[k] * gl[qt[k]] : 0.0);
      }
      const TM fm = live ? (TM)1 : (TM)0;
      const int kq = lane >> 4;
      // operand rows of this tile (lane & 15) and of the rows beyond the full tiles (lane & 3):
      // the volume part of an FP32 product from the FP32 copy, the rest from the FP64 operator
      using araw = std::conditional_t<F32 && !LIFT, float, double>;
      const araw* opb;
      if constexpr (F32 && !LIFT) opb = sOpF; else opb = sOp;
      const araw* acol = opb + mt * 16 + (lane & 15) + kq * OPS;
      const araw* acolm = opb + MTF * 16 + (lane & 3) + kq * OPS;
      const double* ut[NT];
#pragma unroll
      for (int k = 0; k < NT; ++k) ut[k] = sU + kq * RS + e * NC + pt[k];
      const int colp = live ? col : 0;
      const double* fr = sFR + kq * RS + colp;
      // the K loop, without branches: WM (compile time) adds the 4-row product
      auto kloop = [&](auto wm) {
        constexpr bool WM = decltype(wm)::value;
        constexpr int DM = WM ? D : 1;
        if constexpr (LIFT && FRGM) {
          // F in device memory: every F value of the lift part is loaded first (one round
          // trip instead of one per K step), the operator read from LDS as the steps go
          constexpr int NL = NG - NB;
          double fb[NL];
#pragma unroll
          for (int i = 0; i < NL; ++i)
            fb[i] = (4 * i + 3 < KF) ? fr[4 * i * RS] : sFR[min(4 * i + kq, KF - 1) * RS + colp];
#pragma unroll
          for (int i = 0; i < NL; ++i) {
            const TM b = fm * (TM)fb[i];
            acc = MM::mma((TM)acol[(KV + 4 * i) * OPS], b, acc);
            if constexpr (WM) accmini = MM::mini((TM)acolm[(KV + 4 * i) * OPS], b, accmini);
          }
          return;
        }
        araw ra[PDG][D], rm[PDG][DM];
        double ru[PDG][NT];
        auto load = [&](int g, int slot) {
          if (g < NB) {
#pragma unroll
            for (int l = 0; l < D; ++l) ra[slot][l] = acol[(l * NPK + 4 * g) * OPS];
            if constexpr (WM) {
#pragma unroll
              for (int l = 0; l < D; ++l) rm[slot][l] = acolm[(l * NPK + 4 * g) * OPS];
            }
#pragma unroll
            for (int k = 0; k < NT; ++k) ru[slot][k] = ut[k][4 * g * RS];
          } else {
            ra[slot][0] = acol[(KV + 4 * (g - NB)) * OPS];
            if constexpr (WM) rm[slot][0] = acolm[(KV + 4 * (g - NB)) * OPS];
            if (4 * (g - NB) + 3 < KF)
              ru[slot][0] = fr[4 * (g - NB) * RS];
            else   // rows beyond KF meet zero operator columns: read row KF - 1 instead
              ru[slot][0] = sFR[min(4 * (g - NB) + kq, KF - 1) * RS + colp];
          }
        };
        // operator value of ring slot `slot`, index l, in the product precision
        auto aval = [&](int slot, int l) -> TM { return (TM)ra[slot][l]; };
        auto amval = [&](int slot, int l) -> TM { return (TM)rm[slot][l]; };
#pragma unroll
        for (int g = G0; g < G0 + PDG && g < G1; ++g) load(g, g % PDG);
#pragma unroll
        for (int g = G0; g < G1; ++g) {
          const int slot = g % PDG;
          TM a[D], am[DM];
          double x[NT];
#pragma unroll
          for (int l = 0; l < D; ++l) a[l] = aval(slot, l);
          if constexpr (WM) {
#pragma unroll
            for (int l = 0; l < D; ++l) am[l] = amval(slot, l);
          }
#pragma unroll
          for (int k = 0; k < NT; ++k) x[k] = ru[slot][k];
          if (g + PDG < G1) load(g + PDG, slot);
          if (g < NB) {
            TM v[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) v[k] = (TM)x[k];
#pragma unroll
            for (int l = 0; l < D; ++l) {
              TM b = cf[0][l] * v[0];
#pragma unroll
              for (int k = 1; k < NT; ++k) b += cf[k][l] * v[k];
              acc = MM::mma(a[l], b, acc);
              if constexpr (WM) accmini = MM::mini(am[l], b, accmini);
            }
          } else {
            const TM b = fm * (TM)x[0];
            acc = MM::mma(a[0], b, acc);
            if constexpr (WM) accmini = MM::mini(am[0], b, accmini);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      if (with_mini)
        kloop(std::true_type{});
      else
        kloop(std::false_type{});
    }
  };
  // R of `tile` from its accumulators into sFR (FP64)
  auto write_r = [&](int tile, const typename MM::acc_t& acc, const typename MM::mini_t& accmini) {
    if (tile < MTF * ntiles) {
      const int mr = tile / ntiles, nt = tile - mr * ntiles;
      const int mt = MTF - 1 - mr;
      const int col = nt * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) sFR[(mt * 16 + MM::row(lane, r)) * RS + col] = (double)acc[r];
      if (MINI && mr == 0) sFR[(MTF * 16 + (lane >> 4)) * RS + col] = MM::mini_out(accmini, lane);
    }
  };
  if constexpr (SH::COLB) {
    // whole column blocks per wave: the volume and lift parts of the block's row tiles, then
    // its R, which overwrites F only in the block's own columns (read by this wave alone; a
    // wave's LDS operations complete in order)
    __syncthreads();   // F is complete
    for (int nt = wave; nt < ntiles; nt += WAVES) {
      typename MM::acc_t ac[MTF];
      typename MM::mini_t am[MTF];
#pragma unroll
      for (int mr = 0; mr < MTF; ++mr) {
        ac[mr] = typename MM::acc_t{0, 0, 0, 0};
        am[mr] = typename MM::mini_t{};
      }
#pragma unroll
      for (int mr = 0; mr < MTF; ++mr) part(mr * ntiles + nt, ac[mr], am[mr], std::false_type{});
      if constexpr (FRGM) {
        // F in device memory: the lift part of every row tile of the block in one loop over
        // K, the block's F values (the B operand the row tiles share) loaded once, in one
        // round trip, the operator (the A operands) read from LDS as the steps go
        constexpr int NL = NG - NB;
        const int kq = lane >> 4;
        const int col = nt * 16 + (lane & 15);
        const bool live = col < ncols;
        const int colp = live ? col : 0;
        const TM fm = live ? (TM)1 : (TM)0;
        const double* fr = sFR + kq * RS + colp;
        double fb[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i)
          fb[i] = (4 * i + 3 < KF) ? fr[4 * i * RS] : sFR[min(4 * i + kq, KF - 1) * RS + colp];
#pragma unroll
        for (int i = 0; i < NL; ++i) {
          const TM b = fm * (TM)fb[i];
#pragma unroll
          for (int mr = 0; mr < MTF; ++mr) {
            const double* acol = sOp + (MTF - 1 - mr) * 16 + (lane & 15) + kq * OPS;
            ac[mr] = MM::mma((TM)acol[(KV + 4 * i) * OPS], b, ac[mr]);
            if constexpr (MINI) {
              if (mr == 0) {
                const double* acolm = sOp + MTF * 16 + (lane & 3) + kq * OPS;
                am[0] = MM::mini((TM)acolm[(KV + 4 * i) * OPS], b, am[0]);
              }
            }
          }
        }
      } else {
#pragma unroll
        for (int mr = 0; mr < MTF; ++mr) part(mr * ntiles + nt, ac[mr], am[mr], std::true_type{});
      }
#pragma unroll
      for (int mr = 0; mr < MTF; ++mr) write_r(mr * ntiles + nt, ac[mr], am[mr]);
    }
    __syncthreads();
    return;
  }
  // every wave runs the volume part of all its tiles first: it needs U only, so it may
  // overlap the end of the face-flux phase (the caller does not synchronise after it)
#pragma unroll
  for (int ts = 0; ts < TPW; ++ts) part(tile_of(ts), accs[ts], accm[ts], std::false_type{});
  __syncthreads();   // F is complete
#pragma unroll
  for (int ts = 0; ts < TPW; ++ts) part(tile_of(ts), accs[ts], accm[ts], std::true_type{});
  __syncthreads();   // every wave is done reading F and U
#pragma unroll
  for (int ts = 0; ts < TPW; ++ts) write_r(tile_of(ts), accs[ts], accm[ts]);
  __syncthreads();
}

// ---- persistent schedule over the tent DAG
// Claim the next queue slot and wait (bounded) until a released tent fills it.  Returns the
// tent, or -1 when every slot is claimed, on abort, or when the wait bound is exceeded
// (which sets ERRF_DAG_WAIT and the abort word, so that every workgroup leaves).  Thread 0's
// acquire fence after the claim makes the predecessors' W and tau visible: it invalidates the
// CU's L1 and its XCD's L2, which every wave of the workgroup reads through after the
// barrier, so one fence per workgroup suffices.
__device__ __forceinline__ int dag_claim(const KernelParams& kp, int* sh, int tid) {
  if (tid == 0) {
    int t = -1;
    if (__hip_atomic_load(&kp.dag_ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      const int slot = __hip_atomic_fetch_add(&kp.dag_ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (slot < kp.dag_n) {
        const uint64_t t0 = wall_clock64();
        for (;;) {
          t = __hip_atomic_load(&kp.dag_queue[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          if (t >= 0) break;
          if (__hip_atomic_load(&kp.dag_ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
          if ((int64_t)(wall_clock64() - t0) > kp.dag_wait_ticks) {
            atomicOr(&kp.err[2], (int32_t)ERRF_DAG_WAIT);
            __hip_atomic_store(&kp.dag_ctl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
    }
    if (t >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *sh = t;
  }
  __syncthreads();
  return *sh;
}

// Wave 0 of a workgroup whose tent is done: after the release fence, one lane per successor
// counts its predecessor count down (in parallel, not one round trip after another); the
// successors that reach zero get consecutive queue slots from one reservation, ranked by lane.
// Queue entries are base + successor (base: the solver's first global id in a batch).
__device__ __forceinline__ void dag_push_successors(const int32_t* succ, int nsucc, int32_t* indeg, int32_t* queue,
                                                    int32_t* ctl, int base, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  for (int i0 = 0; i0 < nsucc; i0 += 64) {
    const int i = i0 + lane;
    int s = -1;
    bool ready = false;
    if (i < nsucc) {
      s = succ[i];
      ready = __hip_atomic_fetch_add(&indeg[s], -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 1;
    }
    const unsigned long long mask = __ballot(ready);
    if (mask) {
      const int leader = __ffsll((long long)mask) - 1;
      int slot0 = 0;
      if (lane == leader)
        slot0 = __hip_atomic_fetch_add(&ctl[1], __popcll(mask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      slot0 = __shfl(slot0, leader);
      if (ready) {
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        __hip_atomic_store(&queue[slot0 + rank], base + s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Tent t is done: make its W and tau visible device-wide, then count down its successors;
// a successor whose count reaches zero goes into the next queue slot.  The caller's barrier
// has completed every wave's stores (they sit in the XCD's L2); wave 0's release fence
// writes the L2 back for the other XCDs, one fence per workgroup.
__device__ __forceinline__ void dag_release(const KernelParams& kp, int t, int tid) {
  if (tid < 64) dag_push_successors(kp.dag_succ + kp.dag_succ_ptr[t], kp.dag_succ_ptr[t + 1] - kp.dag_succ_ptr[t],
                                     kp.dag_indeg, kp.dag_queue, kp.dag_ctl, 0, tid);
}

// Tent sources of the body: next() yields the next tent (false: the workgroup is done),
// params() the parameter block of its solver (kp0, the kernel's own block, for a single
// solve: the body reads it through a reference to the kernel argument, which the compiler
// lowers to scalar loads of the argument segment; a batch's blocks live in device memory),
// done() runs after the tent's scatter.
struct SchedRange {   // tents first + it, it = begin, begin + step, ... < count
  int64_t first, count, it, step;
  __device__ bool next(const KernelParams&, int*, int, int64_t& t) {
    if (it >= count) return false;
    t = first + it;
    it += step;
    return true;
  }
  __device__ const KernelParams& params(const KernelParams& kp0) const { return kp0; }
  __device__ void done(const KernelParams&, int64_t, int) {}
};

struct SchedBatchRange {   // the tents of a batched launch's segments: it, it + step, ... < total
  const KernelParams* kps;
  const BatchSeg* segs;
  int nseg;
  int64_t total, it, step;
  int solver;
  __device__ bool next(const KernelParams&, int*, int, int64_t& t) {
    if (it >= total) return false;
    int lo = 0, hi = nseg - 1;   // last segment with block0 <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].block0 <= it) lo = mid; else hi = mid - 1;
    }
    const BatchSeg sg = segs[lo];
    t = sg.first + (it - sg.block0);
    solver = sg.solver;
    it += step;
    return true;
  }
  __device__ const KernelParams& params(const KernelParams&) const { return kps[solver]; }
  __device__ void done(const KernelParams&, int64_t, int) {}
};

struct SchedDag {     // one solver's tent DAG
  __device__ bool next(const KernelParams& kp0, int* sh, int tid, int64_t& t) {
    const int c = dag_claim(kp0, sh, tid);
    if (c < 0) return false;
    t = c;
    return true;
  }
  __device__ const KernelParams& params(const KernelParams& kp0) const { return kp0; }
  __device__ void done(const KernelParams& k, int64_t t, int tid) { dag_release(k, (int)t, tid); }
};

struct SchedBatchDag {   // the tent DAGs of a batch of solvers, one queue of global ids
  const KernelParams* kps;
  BatchDag bd;
  int solver;
  __device__ bool next(const KernelParams&, int* sh, int tid, int64_t& t) {
    if (tid == 0) {
      int g = -1;
      if (__hip_atomic_load(&bd.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        const int slot = __hip_atomic_fetch_add(&bd.ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (slot < bd.n) {
          const uint64_t t0 = wall_clock64();
          for (;;) {
            g = __hip_atomic_load(&bd.queue[slot], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (g >= 0) break;
            if (__hip_atomic_load(&bd.ctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
            if ((int64_t)(wall_clock64() - t0) > bd.wait_ticks) {
              for (int i = 0; i < bd.nsolv; ++i) atomicOr(&kps[i].err[2], (int32_t)ERRF_DAG_WAIT);
              __hip_atomic_store(&bd.ctl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
      }
      int s = 0;
      if (g >= 0) {   // solver of g: last s with off[s] <= g
        int lo = 0, hi = bd.nsolv - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (bd.off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        s = lo;
      }
      if (g >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // once per workgroup, as dag_claim
      sh[0] = g;
      sh[1] = s;
    }
    __syncthreads();
    const int g = sh[0];
    solver = sh[1];
    if (g < 0) return false;
    t = g - bd.off[solver];
    return true;
  }
  __device__ const KernelParams& params(const KernelParams&) const { return kps[solver]; }
  __device__ void done(const KernelParams& k, int64_t t, int tid) {   // after the body's barrier, as dag_release
    if (tid < 64)
      dag_push_successors(k.dag_succ + k.dag_succ_ptr[t], k.dag_succ_ptr[t + 1] - k.dag_succ_ptr[t], k.dag_indeg,
                          bd.queue, bd.ctl, bd.off[solver], tid);
  }
};

// Body shared by every entry point: tents from the Sched source, the operator staged from
// kp0 (all solvers of a batch share dimension and degree, hence the reference operator).
// T = double: every product in FP64.  T = float (mixed): the first stage of every
// sub-interval, whose U_{i,0} has the full size of the fields, stays FP64; the later
// stages act on the small Taylor coefficients U_{i,n}, n >= 1, and run on the FP32 cores.
// RK4: the classical RK4 variant instead of SAT (FP64 only).
// One tent of degree P in the LDS regions L: gather, m sub-intervals of the SAT recursion
// (or classical RK4), scatter, and the tent vertex's new time.
template <int D, int P, typename T, int NTMAX, bool RK4, int SYS>
__device__ __forceinline__ void tent_run(const KernelParams& kp, int64_t t, const TentLds& L, int tid, int lane,
                                         int wave) {
  using SH = MShape<D, P, NTMAX, SYS>;
  using PH = Phys<D, SYS>;
  constexpr bool MIXED = sizeof(T) == 4;
  constexpr int NC = SH::NC, NP = SH::NP, NF = SH::NF, NV = SH::NV;
  constexpr int RS = SH::RS;
  constexpr int MAXPAIR = SH::MAXPAIR, BLOCK = SH::BLOCK;
  double* const sOp = L.sOp;
  float* const sOpF = L.sOpF;
  double* const sU = L.sU;
  double* const sFR = L.sFR;
  double* const sGL = L.sGL;
  double* const sBb = L.sBb;
  double* const sEM = L.sEM;
  double* const sRat = L.sRat;
  double* const sFs = L.sFs;
  double* const sFac = L.sFac;
  const int* const sFn = L.sFn;
  const int* const sFsw = L.sFsw;
  int* const sElem = L.sElem;
  int* const sK = L.sK;
  int* const sF = L.sF;
  int* const sPF = L.sPF;
  const double invm = 1.0 / kp.m;
  const int32_t V = kp.tent_vertex[t];
  const double t_top = kp.slab[0] + kp.tent_top[t];
  const int32_t p0 = kp.patch_ptr[V];
  const int nT = kp.patch_ptr[V + 1] - p0;
  const double H = t_top - kp.tau[V];
  const int ncols = nT * NC;
  const int ntiles = (ncols + 15) / 16;
  int tiles[SH::TILES_PER_WAVE];
  tile_assign<D, P, NTMAX, SYS>(kp.tile_order, wave, ntiles, tiles);
  const int32_t f0 = kp.pface_ptr[V];
  const int nFace = kp.pface_ptr[V + 1] - f0;

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

  // gather W (FP64, registers) and U_{0,0} = K(b_0)^{-1} W (closed form in FP64)
  const int npairs = nT * NP;
  constexpr bool ACCG = SH::ACCG;
  double acc[MAXPAIR][NC];   // the Taylor sum of each owned pair (registers)
  double* wp[MAXPAIR];       // ACCG: the pair's entries of W (stride NP per component)
  // Taylor sum of owned pair r, component c
  auto A = [&](int r, int c) -> double& {
    if constexpr (ACCG) return wp[r][c * NP];
    else return acc[r][c];
  };
  bool ok = true;
#pragma unroll
  for (int r = 0; r < MAXPAIR; ++r) {
    const int P_ = tid + r * BLOCK;
    if (P_ < npairs) {
      const int e = P_ / NP, b = P_ - e * NP;
      const int nold = kp.perm[sK[e] * NP + b];
      double* Wp = kp.W + (size_t)sElem[e] * NC * NP + nold;
      double w0[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) w0[c] = Wp[c * NP];
      if constexpr (ACCG) {
        wp[r] = Wp;
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = w0[c];
      }
      double u[NC];
      ok &= PH::inv(&sBb[e * D], sEM[2 * e], sEM[2 * e + 1], w0, u);
#pragma unroll
      for (int c = 0; c < NC; ++c) sU[b * RS + e * NC + c] = u[c];
    }
  }
  // per face, once per tent: the face code and, for an interior face, the factor that
  // carries the flux to the other side
  for (int fi = tid; fi < nFace; fi += BLOCK) {
    const int fc = kp.pface[f0 + fi];
    const int e = fc >> 2, j = fc & 3;
    const int code = sF[e * D + j];
    face_scalars<D>(&sGL[(e * NV + j + 1) * D], &sFs[2 * fi]);
    double ratio = 0.0;
    if (code >= 0) {
      const int pe = code >> 4, jn = (code >> 1) & 7;
      double gg = 0.0, gn = 0.0;
#pragma unroll
      for (int x = 0; x < D; ++x) {
        const double a = sGL[(e * NV + j + 1) * D + x];
        gg += a * a;
        const double h = sGL[(pe * NV + jn) * D + x];
        gn += h * h;
      }
      ratio = -sqrt(gn / gg);
    }
    sPF[fi] = fc;
    sRat[fi] = ratio;
  }
  // scalars of the inverse at th_0 and th_1 (slot i & 1 holds th_i); the recursion then
  // computes th_{i+2} into the slot th_i leaves, in the last stage of sub-interval i.  Only
  // th_i with i < m are used (the tent top is never inverted), and only those are formed,
  // so that the causality flag covers exactly the inversions the method makes
  auto fac_at = [&](int ib, int slot) {
    for (int e = BLOCK - 1 - tid; e < nT; e += BLOCK) {
      const double thb = ib * invm;
      const double* gv = &sGL[(e * NV + 0) * D];
      double bi[D];
#pragma unroll
      for (int x = 0; x < D; ++x) bi[x] = sBb[e * D + x] + thb * (H * gv[x]);
      ok &= PH::inv_fac(bi, sEM[2 * e], sEM[2 * e + 1], &sFac[(slot * NTMAX + e) * 2]);
    }
  };
  if constexpr (!RK4) {
    fac_at(0, 0);
    if (kp.m > 1) fac_at(1, 1);
  }
  __syncthreads();

  // ---- face fluxes for stage input U at sub-interval time th (data ghosts: derivative
  //      n - 1 of the boundary data)
  auto face_fluxes = [&](double th, int n) {
    // ---- face fluxes (times |grad lambda_j|) into F[j nf + s][col], each face once:
    //      the other side of an interior face gets -(|grad lambda_jn| / |grad lambda_j|) G
    //      at its own face-node order (exchanged when the two orders differ)
    // items from the last thread down: a short last round falls on the last wave, which
    // has the fewest product tiles and so the most slack in the product's volume part
    for (int it = BLOCK - 1 - tid; it < nFace * NF; it += BLOCK) {
      const int fi = it / NF;
      const int s = it - fi * NF;
      const int fc = sPF[fi];
      const int e = fc >> 2, j = fc & 3;
      const int nin = sFn[(j * 2) * NF + s];
      double um[NC], up[NC], G[NC], g[D];
#pragma unroll
      for (int c = 0; c < NC; ++c) um[c] = sU[nin * RS + e * NC + c];
#pragma unroll
      for (int x = 0; x < D; ++x) g[x] = -sGL[(e * NV + j + 1) * D + x];
      const int code = sF[e * D + j];
      if (code >= 0) {
        const int pe = code >> 4, jn = (code >> 1) & 7, o = code & 1;
        const int nout = sFn[((jn - 1) * 2 + o) * NF + s];
#pragma unroll
        for (int c = 0; c < NC; ++c) up[c] = sU[nout * RS + pe * NC + c];
        if (kp.flux_kind == 1)
          PH::fl_imp(g, &sFs[2 * fi], sqrt(sEM[2 * e + 1] / sEM[2 * e]), sqrt(sEM[2 * pe + 1] / sEM[2 * pe]), um,
                     up, G);
        else
          PH::fl(g, &sFs[2 * fi], kp.alpha, um, up, G);
        const double ratio = sRat[fi];
        const int s2 = o ? sFsw[s] : s;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          sFR[(j * NF + s) * RS + e * NC + c] = G[c];
          sFR[((jn - 1) * NF + s2) * RS + pe * NC + c] = ratio * G[c];
        }
      } else {
        ghost_state<D, P, SYS>(kp, -1 - code, um, up, sElem[e], sK[e], nin, H, th, n);
        if (kp.flux_kind == 1) {   // walls and data: the element's own medium on both sides
          const double z = sqrt(sEM[2 * e + 1] / sEM[2 * e]);
          PH::fl_imp(g, &sFs[2 * fi], z, z, um, up, G);
        } else {
          PH::fl(g, &sFs[2 * fi], kp.alpha, um, up, G);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) sFR[(j * NF + s) * RS + e * NC + c] = G[c];
      }
    }
    // no barrier: the product reads F only after its volume part and a barrier
  };

  if constexpr (RK4) {
    // classical RK4 on dW/dth = H R(K(b(th))^{-1} W) + data source, the naive variant the
    // paper contrasts with SAT: four evaluations per sub-interval, each with the pointwise
    // inverse at its own time; FP64 step-start state (acc) and stage sum (ks)
    double ks[MAXPAIR][NC];
    for (int i = 0; i < kp.m; ++i) {
      for (int s = 0; s < 4; ++s) {
        const double th = (i + (s == 0 ? 0.0 : (s == 3 ? 1.0 : 0.5))) * invm;
        face_fluxes(th, 1);
        tile_product<double, D, P, NTMAX, SYS>(sOp, sOpF, sU, sFR, sGL, wave, lane, ncols, ntiles, tiles);
        const double thn = (s == 3) ? (i + 1) * invm : (i + (s == 2 ? 1.0 : 0.5)) * invm;
        const double a = (s == 2) ? invm : 0.5 * invm;   // weight of k_s in the next stage input
        const double wk = (s == 0 || s == 3) ? 1.0 : 2.0;
#pragma unroll
        for (int r = 0; r < MAXPAIR; ++r) {
          const int P_ = tid + r * BLOCK;
          if (P_ < npairs) {
            const int e = P_ / NP, b = P_ - e * NP;
            double wst[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              const double k = H * sFR[b * RS + e * NC + c];
              ks[r][c] = (s == 0) ? k : fma(wk, k, ks[r][c]);
              if (s < 3) {
                wst[c] = fma(a, k, A(r, c));
              } else {
                A(r, c) = fma(invm / 6.0, ks[r][c], A(r, c));
                wst[c] = A(r, c);
              }
            }
            if (s < 3 || i + 1 < kp.m) {
              const double* gv = &sGL[(e * NV + 0) * D];
              double bi[D], un[NC];
#pragma unroll
              for (int x = 0; x < D; ++x) bi[x] = sBb[e * D + x] + thn * H * gv[x];
              ok &= PH::inv(bi, sEM[2 * e], sEM[2 * e + 1], wst, un);
#pragma unroll
              for (int c = 0; c < NC; ++c) sU[b * RS + e * NC + c] = un[c];
            }
          }
        }
        __syncthreads();
      }
    }
  } else
  for (int i = 0; i < kp.m; ++i) {
    const double th = i * invm;
    double coef = 1.0;
    for (int n = 1; n <= kp.q; ++n) {
      coef *= invm / n;
      face_fluxes(th, n);

      // ---- R = [S | -L] [A(grad lambda) U ; F] on the matrix cores
      if (MIXED && n >= 2)
        tile_product<float, D, P, NTMAX, SYS>(sOp, sOpF, sU, sFR, sGL, wave, lane, ncols, ntiles, tiles);
      else
        tile_product<double, D, P, NTMAX, SYS>(sOp, sOpF, sU, sFR, sGL, wave, lane, ncols, ntiles, tiles);

      // ---- Taylor accumulation (FP64) and the next U for the owned (element, node) pairs
#pragma unroll
      for (int r = 0; r < MAXPAIR; ++r) {
        const int P_ = tid + r * BLOCK;
        if (P_ < npairs) {
          const int e = P_ / NP, b = P_ - e * NP;
          double Y[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            Y[c] = H * sFR[b * RS + e * NC + c];
            A(r, c) = fma(coef, Y[c], A(r, c));
          }
          const double* gv = &sGL[(e * NV + 0) * D];
          double un[NC];
          bool write = false;
          if (n < kp.q) {
            double bi[D], bp[D], uo[NC], au[NC], rhs[NC];
#pragma unroll
            for (int x = 0; x < D; ++x) {
              bp[x] = H * gv[x];
              bi[x] = sBb[e * D + x] + th * bp[x];
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) uo[c] = sU[b * RS + e * NC + c];
            PH::A(bp, uo, au);
#pragma unroll
            for (int c = 0; c < NC; ++c) rhs[c] = Y[c] + n * au[c];
            PH::inv_apply(bi, sEM[2 * e], sEM[2 * e + 1], &sFac[((i & 1) * NTMAX + e) * 2], rhs, un);
            write = true;
          } else if (i + 1 < kp.m) {
            double bi[D], wsum[NC];
            const double th1 = (i + 1) * invm;
#pragma unroll
            for (int x = 0; x < D; ++x) bi[x] = sBb[e * D + x] + th1 * (H * gv[x]);
#pragma unroll
            for (int c = 0; c < NC; ++c) wsum[c] = A(r, c);
            PH::inv_apply(bi, sEM[2 * e], sEM[2 * e + 1], &sFac[(((i + 1) & 1) * NTMAX + e) * 2], wsum, un);
            write = true;
          }
          if (write) {
#pragma unroll
            for (int c = 0; c < NC; ++c) sU[b * RS + e * NC + c] = un[c];
          }
        }
      }
      if (n == kp.q && i + 2 < kp.m) fac_at(i + 2, i & 1);   // read again in sub-interval i + 1's last stage
      __syncthreads();
    }
  }

  // scatter the tent top (ACCG: the sum is already in W)
  if constexpr (!ACCG) {
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
  }
  if (!ok) kp.err[0] = ERRF_CAUSALITY;
  __syncthreads();
  if (tid == 0) kp.tau[V] = t_top;
  __syncthreads();
}

// Body shared by every single-degree entry point: the operator of degree P staged once,
// then tents from the Sched source (all solvers of a batch share dimension and degree).
// T = double: every product in FP64.  T = float (mixed): the first stage of every
// sub-interval, whose U_{i,0} has the full size of the fields, stays FP64; the later
// stages act on the small Taylor coefficients U_{i,n}, n >= 1, and run on the FP32 cores.
// RK4: the classical RK4 variant instead of SAT (FP64 only).
template <int D, int P, typename T, int NTMAX, class Sched, bool RK4 = false, int SYS = 0>
__device__ __forceinline__ void tent_mfma_body(const KernelParams& kp0, Sched sched) {
  using SH = MShape<D, P, NTMAX, SYS>;
  using LD = MLds<D, P, T, NTMAX, SYS>;
  extern __shared__ double lds_d[];
  // the operator block in LDS (staged here), or in device memory (staged once per solver;
  // all solvers of a batch share dimension and degree, hence its contents)
  // F/R slot of this workgroup (FRG classes): the launches keep the grid within kp0.frg_slots.
  // Taken through a global-address-space pointer, so that its loads and stores are global
  // (not flat) memory instructions and do not wait on the LDS counter.
  double* fr = nullptr;
  if constexpr (LD::FRG) {
    using gdouble = __attribute__((address_space(1))) double;
    gdouble* g = (gdouble*)(kp0.frg + (size_t)blockIdx.x * LD::frg_doubles);
    fr = (double*)g;
  }
  const TentLds L = LD::OPG ? tent_lds<D, P, T, NTMAX, SYS>(kp0.opg, lds_d, fr)
                            : tent_lds<D, P, T, NTMAX, SYS>(lds_d, lds_d + LD::op_block, fr);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (scalar registers)
  if constexpr (!LD::OPG) stage_operator<D, P, T, NTMAX, SYS>(kp0, L, tid);
  // padding rows of U and F are read by the product (times zero): keep them finite
  for (int i = tid; i < (SH::NPK - SH::NP) * SH::RS; i += SH::BLOCK) L.sU[SH::NP * SH::RS + i] = 0.0;
  for (int i = tid; i < (SH::FROWS - SH::KF) * SH::RS; i += SH::BLOCK) L.sFR[SH::KF * SH::RS + i] = 0.0;
  __syncthreads();
  __shared__ int sh_tent[2];
  for (;;) {
    int64_t t;
    if (!sched.next(kp0, sh_tent, tid, t)) break;
    const KernelParams& kp = sched.params(kp0);
    tent_run<D, P, T, NTMAX, RK4, SYS>(kp, t, L, tid, lane, wave);
    sched.done(kp, t, tid);
  }
}

// One workgroup writes the operator block of a class whose block stays in device memory
// (kp.opg, MLds::op_block doubles) in the layout the products read.
template <int D, int P, typename T, int NTMAX, int SYS>
__global__ void __launch_bounds__(tent_block<D>()) stage_operator_kernel(KernelParams kp) {
  const TentLds L = tent_lds<D, P, T, NTMAX, SYS>(kp.opg, kp.opg, nullptr);   // only the operator block is written
  stage_operator<D, P, T, NTMAX, SYS>(kp, L, threadIdx.x);
}

template <int D, int P, typename T, int NTMAX, int WPE, bool RK4 = false, int SYS = 0>
__global__ void __launch_bounds__(tent_block<D>()) __attribute__((amdgpu_waves_per_eu(WPE)))
tent_mfma_kernel(KernelParams kp, int64_t first, int64_t count) {
  tent_mfma_body<D, P, T, NTMAX, SchedRange, RK4, SYS>(
      kp, SchedRange{first, count, (int64_t)blockIdx.x, (int64_t)gridDim.x});
}

// Persistent entry point: every tent of the slab, in DAG order, by kp.dag_grid workgroups.
template <int D, int P, typename T, int NTMAX, int WPE, bool RK4 = false, int SYS = 0>
__global__ void __launch_bounds__(tent_block<D>()) __attribute__((amdgpu_waves_per_eu(WPE)))
tent_mfma_dag_kernel(KernelParams kp) {
  tent_mfma_body<D, P, T, NTMAX, SchedDag, RK4, SYS>(kp, SchedDag{});
}

// Persistent entry point of a batch: every tent of every solver's slab, in DAG order.
template <int D, int P, typename T, int NTMAX, int WPE, int SYS = 0, bool RK4 = false>
__global__ void __launch_bounds__(tent_block<D>()) __attribute__((amdgpu_waves_per_eu(WPE)))
tent_mfma_batch_dag_kernel(const KernelParams* kps, BatchDag bd) {
  tent_mfma_body<D, P, T, NTMAX, SchedBatchDag, RK4, SYS>(kps[0], SchedBatchDag{kps, bd, 0});
}

// Batched entry point: workgroup b runs tent b - seg.block0 of segment seg, i.e. of the
// layer slice (first, count) of solver seg.solver; all solvers share (D, P, T).
template <int D, int P, typename T, int NTMAX, int WPE, int SYS = 0, bool RK4 = false>
__global__ void __launch_bounds__(tent_block<D>()) __attribute__((amdgpu_waves_per_eu(WPE)))
tent_mfma_batch_kernel(const KernelParams* kps, const BatchSeg* segs, int nseg) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = nseg - 1;   // last segment with block0 <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].block0 <= b) lo = mid; else hi = mid - 1;
  }
  const BatchSeg sg = segs[lo];
  tent_mfma_body<D, P, T, NTMAX, SchedRange, RK4, SYS>(kps[sg.solver],
                                                       SchedRange{sg.first, sg.count, b - sg.block0, (int64_t)1 << 62});
}

// Batched entry point with a capped grid (classes with F/R in device memory: one slot per
// workgroup): workgroup b runs tents b, b + gridDim.x, ... of the launch's segments; the
// operator and the slots come from the first segment's solver (one degree per launch, and
// every solver of the batch points at the batch's slots).
template <int D, int P, typename T, int NTMAX, int WPE, int SYS = 0, bool RK4 = false>
__global__ void __launch_bounds__(tent_block<D>()) __attribute__((amdgpu_waves_per_eu(WPE)))
tent_mfma_batch_range_kernel(const KernelParams* kps, const BatchSeg* segs, int nseg, int64_t total) {
  tent_mfma_body<D, P, T, NTMAX, SchedBatchRange, RK4, SYS>(
      kps[segs[0].solver], SchedBatchRange{kps, segs, nseg, total, (int64_t)blockIdx.x, (int64_t)gridDim.x, 0});
}

template <int D, int P, typename T, int NTMAX>
hipError_t launch_m(const KernelParams& kp, int64_t first, int64_t count, hipStream_t s) {
  const size_t lds = MLds<D, P, T, NTMAX>::bytes;
  const size_t lds_ac = MLds<D, P, T, NTMAX, 1>::bytes;
  constexpr int WPE = 2;   // 8 waves per workgroup, one workgroup per CU
  constexpr int BLOCK = MShape<D, P, NTMAX>::BLOCK;
  auto kfn = tent_mfma_kernel<D, P, T, NTMAX, WPE>;
  // RK4 runs in FP64 only: in the FP32 instantiation this names the plain kernel (never
  // launched as RK4), so no kernel is instantiated by two translation units
  auto kfn_rk4 = tent_mfma_kernel<D, P, T, NTMAX, WPE, sizeof(T) == 8>;
  auto kfn_ac = tent_mfma_kernel<D, P, T, NTMAX, WPE, false, 1>;
  auto kfn_ac_rk4 = tent_mfma_kernel<D, P, T, NTMAX, WPE, sizeof(T) == 8, 1>;   // FP64 only, as above
  if (count < 0) {   // prepare: allow the dynamic LDS size (done once, outside graph capture)
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && sizeof(T) == 8)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn_rk4), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e == hipSuccess && lds_ac <= 160 * 1024)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn_ac), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_ac);
    if (e == hipSuccess && sizeof(T) == 8 && lds_ac <= 160 * 1024)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn_ac_rk4),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_ac);
    return e;
  }
  // one workgroup per tent; a class with F/R in device memory runs at most kp.frg_slots
  // workgroups (one slot each), every workgroup then taking every grid-th tent of the range
  int64_t grid = count;
  if constexpr (MLds<D, P, T, NTMAX>::FRG) {
    if (!kp.frg || kp.frg_slots <= 0) return hipErrorInvalidValue;
    grid = std::min<int64_t>(count, kp.frg_slots);
  }
  if (grid <= 0) return hipSuccess;
  if (kp.system == 1) {
    if (kp.method == 1) {
      if (sizeof(T) != 8) return hipErrorInvalidValue;
      hipLaunchKernelGGL(kfn_ac_rk4, dim3((unsigned)grid), dim3(BLOCK), lds_ac, s, kp, first, count);
    } else {
      hipLaunchKernelGGL(kfn_ac, dim3((unsigned)grid), dim3(BLOCK), lds_ac, s, kp, first, count);
    }
  } else if (kp.method == 1) {
    if (sizeof(T) != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kfn_rk4, dim3((unsigned)grid), dim3(BLOCK), lds, s, kp, first, count);
  } else {
    hipLaunchKernelGGL(kfn, dim3((unsigned)grid), dim3(BLOCK), lds, s, kp, first, count);
  }
  return hipGetLastError();
}

// Workgroups of a persistent kernel that are resident at once on the device (also sets the
// kernel's dynamic LDS attribute).
inline hipError_t resident_grid(const void* kfn, int block, size_t lds, int* resident) {
  hipError_t e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0, dev = 0, cus = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, block, lds)) != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  *resident = per_cu * cus;
  return hipSuccess;
}

// Persistent launches.  resident != null: only report the resident grid (and set the
// LDS attribute, outside graph capture); otherwise launch the stated grid.
struct PersistentArgs {
  const KernelParams* kp;    // single solve (by value in the launch)
  const KernelParams* kps;   // batch: device array
  const BatchDag* bd;
};

template <int D, int P, typename T, int NTMAX>
hipError_t launch_md(const PersistentArgs& a, hipStream_t s, int* resident) {
  const size_t lds = MLds<D, P, T, NTMAX>::bytes;
  constexpr int BLOCK = MShape<D, P, NTMAX>::BLOCK;
  if (a.bd) {   // a batch of one system (the acoustic variant when a.bd->system == 1)
    // RK4 runs in FP64 only: in the FP32 instantiation the RK4 names are the plain kernels
    // (never launched as RK4).  Classes with F/R in device memory: the host keeps the grid
    // within the batch's slots.
    constexpr bool R = sizeof(T) == 8;
    const bool ac = a.bd->system == 1, rk = a.bd->method == 1;
    if (rk && !R) return hipErrorInvalidValue;
    const void* kf = ac ? (rk ? reinterpret_cast<const void*>(tent_mfma_batch_dag_kernel<D, P, T, NTMAX, 2, 1, R>)
                              : reinterpret_cast<const void*>(tent_mfma_batch_dag_kernel<D, P, T, NTMAX, 2, 1>))
                        : (rk ? reinterpret_cast<const void*>(tent_mfma_batch_dag_kernel<D, P, T, NTMAX, 2, 0, R>)
                              : reinterpret_cast<const void*>(tent_mfma_batch_dag_kernel<D, P, T, NTMAX, 2, 0>));
    const size_t lds_b = ac ? MLds<D, P, T, NTMAX, 1>::bytes : lds;
    if (resident) return resident_grid(kf, BLOCK, lds_b, resident);
    if (a.bd->n <= 0) return hipSuccess;
    if (a.bd->grid <= 0) return hipErrorInvalidValue;
    const KernelParams* kps = a.kps;
    BatchDag bd = *a.bd;
    void* args[] = {&kps, &bd};
    return hipLaunchKernel(kf, dim3((unsigned)a.bd->grid), dim3(BLOCK), args, lds_b, s);
  }
  auto kfn = tent_mfma_dag_kernel<D, P, T, NTMAX, 2>;
  auto kfn_rk4 = tent_mfma_dag_kernel<D, P, T, NTMAX, 2, sizeof(T) == 8>;   // FP64 only, as above
  auto kfn_ac = tent_mfma_dag_kernel<D, P, T, NTMAX, 2, false, 1>;
  auto kfn_ac_rk4 = tent_mfma_dag_kernel<D, P, T, NTMAX, 2, sizeof(T) == 8, 1>;   // FP64 only, as above
  const size_t lds_ac = MLds<D, P, T, NTMAX, 1>::bytes;
  if (resident) {   // the residency of the variant the solver runs (all: the smallest)
    if (a.kp && a.kp->system == 1) {
      hipError_t e = resident_grid(reinterpret_cast<const void*>(kfn_ac), BLOCK, lds_ac, resident);
      if (e == hipSuccess && sizeof(T) == 8) {
        int r2 = 0;
        e = resident_grid(reinterpret_cast<const void*>(kfn_ac_rk4), BLOCK, lds_ac, &r2);
        *resident = std::min(*resident, r2);
      }
      return e;
    }
    hipError_t e = resident_grid(reinterpret_cast<const void*>(kfn), BLOCK, lds, resident);
    if (e == hipSuccess && sizeof(T) == 8) {
      int r2 = 0;
      e = resident_grid(reinterpret_cast<const void*>(kfn_rk4), BLOCK, lds, &r2);
      *resident = std::min(*resident, r2);
    }
    return e;
  }
  if (a.kp->dag_n <= 0) return hipSuccess;
  if (a.kp->dag_grid <= 0) return hipErrorInvalidValue;
  if (MLds<D, P, T, NTMAX>::FRG && (!a.kp->frg || a.kp->dag_grid > a.kp->frg_slots)) return hipErrorInvalidValue;
  if (a.kp->system == 1) {
    if (a.kp->method == 1) {
      if (sizeof(T) != 8) return hipErrorInvalidValue;
      hipLaunchKernelGGL(kfn_ac_rk4, dim3((unsigned)a.kp->dag_grid), dim3(BLOCK), lds_ac, s, *a.kp);
    } else {
      hipLaunchKernelGGL(kfn_ac, dim3((unsigned)a.kp->dag_grid), dim3(BLOCK), lds_ac, s, *a.kp);
    }
  } else if (a.kp->method == 1) {
    if (sizeof(T) != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kfn_rk4, dim3((unsigned)a.kp->dag_grid), dim3(BLOCK), lds, s, *a.kp);
  } else {
    hipLaunchKernelGGL(kfn, dim3((unsigned)a.kp->dag_grid), dim3(BLOCK), lds, s, *a.kp);
  }
  return hipGetLastError();
}

template <int D, int P, typename T>
hipError_t launch_mdp(const PersistentArgs& a, int max_patch, hipStream_t s, int* resident) {
  constexpr int NB = big_class<D, P>();
  if (max_patch <= 8) return launch_md<D, P, T, 8>(a, s, resident);
  if (max_patch <= 24) return launch_md<D, P, T, 24>(a, s, resident);
  if (max_patch <= NB) return launch_md<D, P, T, NB>(a, s, resident);
  constexpr int XL = xl_class<D, P>();
  if constexpr (XL > 0)
    if (max_patch <= XL) return launch_md<D, P, T, XL>(a, s, resident);
  return hipErrorInvalidValue;
}

template <int D, int P, typename T, int NTMAX>
hipError_t launch_mb(const BatchLaunch& bl, hipStream_t s) {
  constexpr int WPE = 2;
  constexpr int BLOCK = MShape<D, P, NTMAX>::BLOCK;
  // RK4 runs in FP64 only: in the FP32 instantiation the RK4 names are the plain kernels
  constexpr bool R = sizeof(T) == 8;
  const bool ac = bl.system == 1, rk = bl.method == 1;
  if (rk && !R) return hipErrorInvalidValue;
  const size_t lds = ac ? MLds<D, P, T, NTMAX, 1>::bytes : MLds<D, P, T, NTMAX>::bytes;
  if constexpr (MLds<D, P, T, NTMAX>::FRG) {
    // F/R in device memory: at most bl.frg_slots workgroups, each taking every grid-th tent
    const void* kr = ac ? (rk ? reinterpret_cast<const void*>(tent_mfma_batch_range_kernel<D, P, T, NTMAX, WPE, 1, R>)
                              : reinterpret_cast<const void*>(tent_mfma_batch_range_kernel<D, P, T, NTMAX, WPE, 1>))
                        : (rk ? reinterpret_cast<const void*>(tent_mfma_batch_range_kernel<D, P, T, NTMAX, WPE, 0, R>)
                              : reinterpret_cast<const void*>(tent_mfma_batch_range_kernel<D, P, T, NTMAX, WPE, 0>));
    if (bl.blocks < 0) return hipFuncSetAttribute(kr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (bl.blocks == 0) return hipSuccess;
    if (bl.frg_slots <= 0) return hipErrorInvalidValue;
    const KernelParams* kps = bl.kps;
    const BatchSeg* segs = bl.segs;
    int nseg = bl.nseg;
    int64_t total = bl.blocks;
    void* args[] = {&kps, &segs, &nseg, &total};
    return hipLaunchKernel(kr, dim3((unsigned)std::min<int64_t>(bl.blocks, bl.frg_slots)), dim3(BLOCK), args, lds, s);
  } else {
    const void* kf = ac ? (rk ? reinterpret_cast<const void*>(tent_mfma_batch_kernel<D, P, T, NTMAX, WPE, 1, R>)
                              : reinterpret_cast<const void*>(tent_mfma_batch_kernel<D, P, T, NTMAX, WPE, 1>))
                        : (rk ? reinterpret_cast<const void*>(tent_mfma_batch_kernel<D, P, T, NTMAX, WPE, 0, R>)
                              : reinterpret_cast<const void*>(tent_mfma_batch_kernel<D, P, T, NTMAX, WPE, 0>));
    if (bl.blocks < 0) return hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (bl.blocks == 0) return hipSuccess;
    const KernelParams* kps = bl.kps;
    const BatchSeg* segs = bl.segs;
    int nseg = bl.nseg;
    void* args[] = {&kps, &segs, &nseg};
    return hipLaunchKernel(kf, dim3((unsigned)bl.blocks), dim3(BLOCK), args, lds, s);
  }
}

template <int D, int P, typename T>
hipError_t launch_mbp(const BatchLaunch& bl, hipStream_t s) {
  constexpr int NB = big_class<D, P>();
  if (bl.max_patch <= 8) return launch_mb<D, P, T, 8>(bl, s);
  if (bl.max_patch <= 24) return launch_mb<D, P, T, 24>(bl, s);
  if (bl.max_patch <= NB) return launch_mb<D, P, T, NB>(bl, s);
  constexpr int XL = xl_class<D, P>();
  if constexpr (XL > 0)
    if (bl.max_patch <= XL) return launch_mb<D, P, T, XL>(bl, s);
  return hipErrorInvalidValue;
}

template <int D, int P, typename T>
hipError_t launch_mp(const KernelParams& kp, int64_t first, int64_t count, hipStream_t s) {
  constexpr int NB = big_class<D, P>();
  if (kp.max_patch <= 8) return launch_m<D, P, T, 8>(kp, first, count, s);
  if (kp.max_patch <= 24) return launch_m<D, P, T, 24>(kp, first, count, s);
  if (kp.max_patch <= NB) return launch_m<D, P, T, NB>(kp, first, count, s);
  constexpr int XL = xl_class<D, P>();
  if constexpr (XL > 0)
    if (kp.max_patch <= XL) return launch_m<D, P, T, XL>(kp, first, count, s);
  return hipErrorInvalidValue;
}

// Device-memory operator block of the class kp.max_patch falls in: its size in bytes (0 if
// the class stages the operator in LDS), and the launch that writes it to kp.opg.
template <int D, int P, typename T, int NTMAX>
size_t opg_m(int system) {
  return system == 1 ? (MLds<D, P, T, NTMAX, 1>::OPG ? MLds<D, P, T, NTMAX, 1>::op_block * 8 : 0)
                     : (MLds<D, P, T, NTMAX, 0>::OPG ? MLds<D, P, T, NTMAX, 0>::op_block * 8 : 0);
}

template <int D, int P, typename T>
size_t opg_mp(int max_patch, int system) {
  constexpr int NB = big_class<D, P>();
  if (max_patch <= 8) return opg_m<D, P, T, 8>(system);
  if (max_patch <= 24) return opg_m<D, P, T, 24>(system);
  if (max_patch <= NB) return opg_m<D, P, T, NB>(system);
  constexpr int XL = xl_class<D, P>();
  if constexpr (XL > 0)
    if (max_patch <= XL) return opg_m<D, P, T, XL>(system);
  return 0;
}

// Bytes of one workgroup's F/R slot in device memory for the class max_patch falls in (0 if
// the class keeps F/R in LDS).
template <int D, int P, typename T>
size_t frg_mp(int max_patch, int system) {
  constexpr int NB = big_class<D, P>(), XL = xl_class<D, P>();
  if constexpr (XL > 0) {
    if (max_patch > NB && max_patch <= XL)
      return (system == 1 ? MLds<D, P, T, XL, 1>::frg_doubles : MLds<D, P, T, XL>::frg_doubles) * 8;
  }
  return 0;
}

template <int D, int P, typename T, int NTMAX>
hipError_t stage_m(const KernelParams& kp, hipStream_t s) {
  constexpr int BLOCK = MShape<D, P, NTMAX>::BLOCK;
  if (kp.system == 1) {
    if constexpr (MLds<D, P, T, NTMAX, 1>::OPG) {
      hipLaunchKernelGGL((stage_operator_kernel<D, P, T, NTMAX, 1>), dim3(1), dim3(BLOCK), 0, s, kp);
      return hipGetLastError();
    }
    return hipSuccess;
  }
  if constexpr (MLds<D, P, T, NTMAX, 0>::OPG) {
    hipLaunchKernelGGL((stage_operator_kernel<D, P, T, NTMAX, 0>), dim3(1), dim3(BLOCK), 0, s, kp);
    return hipGetLastError();
  }
  return hipSuccess;
}

template <int D, int P, typename T>
hipError_t stage_mp(const KernelParams& kp, hipStream_t s) {
  constexpr int NB = big_class<D, P>();
  if (kp.max_patch <= 8) return stage_m<D, P, T, 8>(kp, s);
  if (kp.max_patch <= 24) return stage_m<D, P, T, 24>(kp, s);
  if (kp.max_patch <= NB) return stage_m<D, P, T, NB>(kp, s);
  constexpr int XL = xl_class<D, P>();
  if constexpr (XL > 0)
    if (kp.max_patch <= XL) return stage_m<D, P, T, XL>(kp, s);
  return hipErrorInvalidValue;
}

template <int D, int P, typename T>
size_t lds_mp(int max_patch, int system) {
  constexpr int NB = big_class<D, P>();
  if (system == 1) {
    if (max_patch <= 8) return MLds<D, P, T, 8, 1>::bytes;
    if (max_patch <= 24) return MLds<D, P, T, 24, 1>::bytes;
    if (max_patch <= NB) return MLds<D, P, T, NB, 1>::bytes;
    if constexpr (xl_class<D, P>() > 0)
      if (max_patch <= xl_class<D, P>()) return MLds<D, P, T, xl_class<D, P>(), 1>::bytes;
    return (size_t)-1;
  }
  if (max_patch <= 8) return MLds<D, P, T, 8>::bytes;
  if (max_patch <= 24) return MLds<D, P, T, 24>::bytes;
  if (max_patch <= NB) return MLds<D, P, T, NB>::bytes;
  if constexpr (xl_class<D, P>() > 0)
    if (max_patch <= xl_class<D, P>()) return MLds<D, P, T, xl_class<D, P>()>::bytes;
  return (size_t)-1;
}

}  // namespace mfk
}  // namespace mtp
