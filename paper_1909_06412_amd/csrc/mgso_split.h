// mgso_split.h -- three-pass transforms of 16^8 complex64 grids.
//
// The radix-16 plan of a 16^8 grid takes four passes per transform direction:
// axes 5-7 (a contiguous 4096-point tile), then 3-4, 1-2 and 0 (strided tiles).
// A strided tile can hold 16384 complex64 points (128 KiB of LDS); with runs of 16
// consecutive points that leaves 10 transform bits per tile, and 12 + 10 + 10
// covers the 32 bits of the grid in three passes once one axis (axis 2) is split
// into two 4-point digits, n = n0 + 4 n1.  A 16-point DFT is a 4-point DFT over
// the high digit n1 (giving k0), the twiddle W16^(n0 k0), and a 4-point DFT over
// the low digit n0 (giving k1), with X[k0 + 4 k1] left at the digit positions of
// (k1, k0): a swapped order that only momentum-space work sees, and that work
// stays in registers (the second pass is the turning pass of the kinetic substep).
//   pass B: axis 3 (X, bits 16-19), the high digit of axis 2 (Y, bits 22-23),
//           axis 0 (Z, bits 28-31)
//   pass C: axis 4 (X, bits 12-15), the low digit of axis 2 (Y, bits 20-21),
//           axis 1 (Z, bits 24-27)
// (run: bits 0-3, axis 7).  Each pass pairs a middle axis with an outer one: tiles
// whose transform bits all sit in the top bits of the address measured a quarter
// slower.  Kinetic substep (Sec. II.G.2, Eq. (55)): sweep 0 forward, B forward, C
// forward reduced to the momentum moments (nothing stored), finalize, C round trip
// (forward DFTs, the kinetic factor M, inverse DFTs), B inverse, sweep 0 inverse.
// The round trip goes axis by axis (Z, then X, then the Y digit: M is a product of
// per-axis factors and DFTs along different axes commute), so it needs the same two
// LDS transposes as a one-way pass.  Every pass loads its tile as Z lines and stores
// it from Y lines (pass B inverse applies its pointwise factors first and then the
// inverse DFTs in the order Z, X, Y): loaded as Y lines it took 5% longer.
//
// Tables (built by the finalize kernel at G.gtab_len in AG / MG, 1024 + 1024 + 16
// entries each, then 48): AG[tB + g] = A_X A_Z d(Y) for pass B, with d(n1) the
// high-digit part of axis 2's A factor (that factor is a linear phase with a sign
// (-1)^n, so A_2(n0 + 4 n1) = c(n0) d(n1)), AG[tC + g] = A_X A_Z for pass C, AG[tS +
// 4 n0 + k0] = c(n0) W16^(n0 k0); MG[tB + g] = M_X M_Z of pass B, MG[tS + k] =
// M_2(k) and, for pass C's per-axis round trips, MG[tS + 16 + k] = M_X(k) and
// MG[tS + 32 + k] = M_Z(k).  g = X + 16 Y + 64 Z.
#pragma once
#include "mgso_sweep16.h"

namespace mgk {

enum : int { SPL_B_FWD = 0, SPL_B_INV = 1, SPL_C_MOM = 2, SPL_C_RT = 3 };

// Axis assignment: pass p transforms axes SPL_AX[p][0] (X) and SPL_AX[p][1] (Z)
// and one digit of axis SPL_SPLIT_AXIS (p = 0: the high digit, p = 1: the low one).
constexpr int SPL_AX[2][2] = {{3, 0}, {4, 1}};
constexpr int SPL_SPLIT_AXIS = 2;
constexpr int SPL_NT = 1024;
constexpr uint32_t SPL_TILE = 16384;
constexpr uint32_t SPL_TILE_LDS = SPL_TILE + SPL_TILE / 16;  // pad16 gaps
constexpr int SPL_TAB = 2 * 1024 + 48;                        // split entries appended to AG / MG
constexpr size_t SPL_LDS_BYTES = (size_t)(SPL_TILE_LDS + 2 * 1024 + 48) * sizeof(float2);

struct SplitDesc {
  int32_t pX, pY, pZ;  // flat bit positions of the in-tile fields X (4 bits), Y (2), Z (4)
  int32_t pYc;         // flat bit position of the split axis' other digit (tile constant)
  int32_t axX, axY, axZ;
  int32_t nf;          // tile-index fields, low first: flat position and width
  int32_t flo[4], fw[4];
  uint32_t ntiles;
  int32_t tab;         // this pass's 1024-entry tables in AG / MG
  int32_t small;       // the 16-entry table (AG for pass B, MG for pass C)
};

struct SplArgs {
  const PacketGeom* geom;
  const float2* src;
  float2* dst;
  const float2* AG;
  const float2* MG;
  double* partials;
  SplitDesc d;
};

template <int KIND>
__global__ __launch_bounds__(SPL_NT) void k_split(SplArgs a) {
  typedef float2 C;
  constexpr bool HAS_M = KIND == SPL_B_INV;

  extern __shared__ __align__(16) unsigned char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  C* __restrict__ ltab = lds + SPL_TILE_LDS;
  C* __restrict__ lmt = ltab + 1024;
  C* __restrict__ lsm = lmt + 1024;  // the 16-entry table(s) (read once per tile)
  const SplitDesc d = a.d;
  const PacketGeom& G = *a.geom;
  const uint64_t off = G.off;
  const C* __restrict__ src = a.src + off;
  C* __restrict__ dst = a.dst + off;
  const uint32_t t = threadIdx.x;
  for (uint32_t i = t; i < 1024u; i += SPL_NT) {
    ltab[i] = a.AG[d.tab + i];
    if (HAS_M) lmt[i] = a.MG[d.tab + i];
    if (i < 48u) lsm[i] = KIND == SPL_C_RT ? a.MG[d.small + i] : i < 16u ? a.AG[d.small + i] : C{0.f, 0.f};
  }
  __syncthreads();

  const uint32_t run = t & 15u;
  // In the Z- and Y-line layouts a lane's (run, X) = (t & 15, (t >> 4) & 15) and
  // the rest of its position, t >> 8, is the same across a wave (64 lanes): HBM
  // addresses are a wave-uniform base plus a 32-bit lane offset.
  const uint32_t lX = (t >> 4) & 15u;
  const uint32_t w8 = __builtin_amdgcn_readfirstlane(t >> 8);
  const uint32_t loff = run | (lX << d.pX);
  // Z lines: thread (run, X, Y = t >> 8), point k at Z = k
  const uint32_t zbase = w8 << d.pY;
  const uint32_t zg = lX + 16u * (t >> 8);  // + 64 k
  // X lines: thread (run, Y, Z), point k at X = k
  const uint32_t xY = (t >> 4) & 3u, xZ = t >> 6;
  const uint32_t xl = pad16(run + 256u * xY + 1024u * xZ);  // + 17 k
  // Y lines: thread (run, X, Zb + i), Zb = 4 (t >> 8), point 4 i + j at Y = j
  const uint32_t yZb = 4u * w8;
  const uint32_t yl = pad16(run + 16u * lX + 1024u * (4u * (t >> 8)));  // + 272 j + 1088 i
  const uint32_t yg = lX + 64u * (4u * (t >> 8));                    // + 16 j + 64 i
  const uint32_t zl = pad16(t);                                       // + 1088 k

  auto tile_base = [&](uint32_t tl) -> uint32_t {
    uint32_t b = 0, sh = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (f < d.nf) {
        b |= ((tl >> sh) & ((1u << d.fw[f]) - 1u)) << d.flo[f];
        sh += (uint32_t)d.fw[f];
      }
    }
    return b;
  };
  // wave-uniform element offsets of the Y-line point (i, j) and the Z-line point k
  auto ybase = [&](uint32_t base, int i, int j) -> size_t {
    return (size_t)(base | ((uint32_t)j << d.pY) | ((yZb + (uint32_t)i) << d.pZ));
  };
  auto zbase_k = [&](uint32_t base, int k) -> size_t {
    return (size_t)(base | zbase | ((uint32_t)k << d.pZ));
  };
  C xn[16];
  auto load = [&](uint32_t tl) {
    const uint32_t base = tile_base(tl);
#pragma unroll
    for (int k = 0; k < 16; ++k) xn[k] = (src + zbase_k(base, k))[loff];
  };
  if (blockIdx.x < d.ntiles) load(blockIdx.x);

  double acc[MGK_NACC];
#pragma unroll
  for (int k = 0; k < MGK_NACC; ++k) acc[k] = 0.0;

  // LDS moves between the three line layouts (each followed by a barrier pair)
  // (pad16 of u + 16 m is pad16(u) + 17 m when u's low four bits stay below 16)
  auto z_to_lds = [&](C* x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) lds[zl + 1088u * k] = x[k];
  };
  auto x_to_lds = [&](C* x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) lds[xl + 17u * k] = x[k];
  };
  auto lds_to_x = [&](C* x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = lds[xl + 17u * k];
  };
  auto lds_to_y = [&](C* x) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) x[4 * i + j] = lds[yl + 272u * j + 1088u * i];
  };

  for (uint32_t tile = blockIdx.x; tile < d.ntiles; tile += gridDim.x) {
    const uint32_t base = tile_base(tile);
    const uint32_t oth = (base >> d.pYc) & 3u;  // the split axis' other digit (B: n0, C: k0)
    C x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = xn[k];
    if (tile + gridDim.x < d.ntiles) load(tile + gridDim.x);

    if constexpr (KIND == SPL_B_INV) {
      // Z lines as loaded, each at a fixed stored digit k0 = t >> 8: undo the twiddle
      // and c(n0) and apply M of X and Z (all pointwise), inverse DFTs along Z and X,
      // then along the Y digit in the Y-line layout, conj(A), store from there
      const C s0 = lsm[4u * oth + (t >> 8)];
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = cmul(cmulc(x[k], s0), lmt[zg + 64u * k]);
      dft16<float, true>(x);
      z_to_lds(x);
      __syncthreads();
      lds_to_x(x);
      __syncthreads();
      dft16<float, true>(x);
      x_to_lds(x);
      __syncthreads();
      lds_to_y(x);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) dft4(&x[4 * i], true);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = cmulc(x[4 * i + j], ltab[yg + 16u * j + 64u * i]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) (dst + ybase(base, i, j))[loff] = x[4 * i + j];
    } else if constexpr (KIND == SPL_C_RT) {
      // per-axis round trips: A of X and Z, then along Z: DFT, M_Z, inverse DFT; the
      // X lines the same with M_X; the Y digit with M_2 at k = k0 + 4 k1; conj(A)
      const C* __restrict__ m2 = lsm;
      const C* __restrict__ mx = lsm + 16;
      const C* __restrict__ mz = lsm + 32;
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = cmul(x[k], ltab[zg + 64u * k]);
      dft16<float, false>(x);
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = cmul(x[k], mz[k]);
      dft16<float, true>(x);
      z_to_lds(x);
      __syncthreads();
      lds_to_x(x);
      __syncthreads();
      dft16<float, false>(x);
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = cmul(x[k], mx[k]);
      dft16<float, true>(x);
      x_to_lds(x);
      __syncthreads();
      lds_to_y(x);
      __syncthreads();
      C m[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) m[j] = m2[oth + 4 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dft4(&x[4 * i], false);
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = cmul(x[4 * i + j], m[j]);
        dft4(&x[4 * i], true);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = cmulc(x[4 * i + j], ltab[yg + 16u * j + 64u * i]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) (dst + ybase(base, i, j))[loff] = x[4 * i + j];
    } else {
      // forward half: A factors, DFT along Z, X, then the 4-point Y digit
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = cmul(x[k], ltab[zg + 64u * k]);
      dft16<float, false>(x);
      z_to_lds(x);
      __syncthreads();
      lds_to_x(x);
      __syncthreads();
      dft16<float, false>(x);
      x_to_lds(x);
      __syncthreads();
      lds_to_y(x);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) dft4(&x[4 * i], false);
      if constexpr (KIND == SPL_B_FWD) {
        // k0 = j: twiddle W16^(n0 k0) and the low digit's A factor c(n0)
        C s[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] = lsm[4 * oth + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) x[4 * i + j] = cmul(x[4 * i + j], s[j]);
      }
      if constexpr (KIND == SPL_C_MOM) {
        // momentum moments: every axis is transformed; axis axY has k = k0 + 4 k1
        // (k0 = oth, k1 = j), the run is axis D-1, the other axes are tile constants
        double wi[4] = {0.0, 0.0, 0.0, 0.0}, wj[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const C v = x[4 * i + j];
            const double w = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            wi[i] += w;
            wj[j] += w;
          }
        constexpr int AX = SPL_AX[1][0], AZ = SPL_AX[1][1], AY = SPL_SPLIT_AXIS;
        const double ws = (wi[0] + wi[1]) + (wi[2] + wi[3]);
        acc[0] += ws;
        acc[1 + 7] += ws * ((double)run - 8.0);
        acc[1 + AX] += ws * ((double)lX - 8.0);
        double mz = 0.0, my = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) mz += wi[i] * ((double)(yZb + i) - 8.0);
#pragma unroll
        for (int j = 0; j < 4; ++j) my += wj[j] * ((double)(oth + 4u * j) - 8.0);
        acc[1 + AZ] += mz;
        acc[1 + AY] += my;
#pragma unroll
        for (int l = 0; l < 7; ++l)
          if (l != AX && l != AY && l != AZ)
            acc[1 + l] += ws * ((double)((base >> (4 * (7 - l))) & 15u) - 8.0);
        continue;
      }
    }
    if constexpr (KIND == SPL_B_FWD) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) (dst + ybase(base, i, j))[loff] = x[4 * i + j];
    }
  }
  if constexpr (KIND == SPL_C_MOM)
    block_reduce<SPL_NT>(acc, G.D + 2, a.partials + (size_t)blockIdx.x * MGK_NACC, (double*)lds_raw);
}

}  // namespace mgk
