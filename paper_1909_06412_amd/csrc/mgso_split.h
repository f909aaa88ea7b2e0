// mgso_split.h -- three-pass transforms of 16^8 grids.
//
// The radix-16 plan of a 16^8 grid takes four passes per transform direction:
// axes 5-7 (a contiguous 4096-point tile), then 3-4, 1-2 and 0 (strided tiles).
// A strided tile can hold 16384 complex64 points or 8192 complex128 points (128
// KiB of LDS); with runs of 128 bytes (16 or 8 consecutive points) that leaves 10
// transform bits per tile, and 12 + 10 + 10
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
// (run: bits 0-3, complex128 bits 0-2, of axis 7).  Each pass pairs a middle axis with
// an outer one: tiles
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
// Tables (built by the finalize kernel at G.gtab_len in AG / MG: 1024 + 1024 + 80
// entries each): AG[tB + g] = A_X A_Z d(Y) for pass B, with d(n1) the high-digit
// part of axis 2's A factor (that factor is a linear phase with a sign (-1)^n, so
// A_2(n0 + 4 n1) = c(n0) d(n1)), AG[tC + g] = A_X A_Z for pass C, AG[tS + 4 n0 + k0] =
// c(n0) W16^(n0 k0); per-axis kinetic factors MG[tS + k] = M_2(k), MG[tS + 16 + k]
// and MG[tS + 32 + k] = M of pass C's X and Z axes, MG[tS + 48 + k] and MG[tS + 64 +
// k] = M of pass B's X and Z axes.  g = X + 16 Y + 64 Z.
#pragma once
#include "mgso_sweep16.h"

namespace mgk {

enum : int { SPL_B_FWD = 0, SPL_B_INV = 1, SPL_C_MOM = 2, SPL_C_RT = 3 };

// Axis assignment: pass p transforms axes SPL_AX[p][0] (X) and SPL_AX[p][1] (Z)
// and one digit of axis SPL_SPLIT_AXIS (p = 0: the high digit, p = 1: the low one).
constexpr int SPL_AX[2][2] = {{3, 0}, {4, 1}};
constexpr int SPL_SPLIT_AXIS = 2;
// Tile geometry: a run of R = 2^LR consecutive points (128 bytes), 1024 R points,
// 64 R threads with 16 points each.
template <typename T> constexpr int spl_lr() { return sizeof(T) == 4 ? 4 : 3; }
template <typename T> constexpr int spl_nt() { return 64 << spl_lr<T>(); }
template <typename T> constexpr uint32_t spl_tile_lds() {
  return (1024u << spl_lr<T>()) + (64u << spl_lr<T>());  // the tile and its pad16 gaps
}
constexpr int SPL_SMALL = 80;                 // 16-entry tables: twiddles or M_2, then four per-axis M
constexpr int SPL_TAB = 2 * 1024 + SPL_SMALL;  // split entries appended to AG / MG
template <typename T> constexpr size_t spl_lds_bytes() {
  // the tile in complex elements, then the tables in 16-byte table entries
  return (size_t)spl_tile_lds<T>() * 2 * sizeof(T) + (size_t)(1024 + SPL_SMALL) * 16;
}

struct SplitDesc {
  int32_t pX, pY, pZ;  // flat bit positions of the in-tile fields X (4 bits), Y (2), Z (4)
  int32_t pYc;         // flat bit position of the split axis' other digit (tile constant)
  int32_t axX, axY, axZ;
  int32_t nf;          // tile-index fields (tile index bits low first): flat position and width
  int32_t flo[4], fw[4];
  uint32_t ntiles;
  int32_t tab;         // this pass's 1024-entry tables in AG / MG
  int32_t small;       // the 16-entry tables (tS)
};

template <typename T> struct SplArgs {
  const PacketGeom* geom;
  const typename CT<T>::type* src;
  typename CT<T>::type* dst;
  const typename TE<T>::type* AG;
  const typename TE<T>::type* MG;
  double* partials;
  SplitDesc d;
};

template <typename T, int KIND>
__global__ __launch_bounds__(spl_nt<T>()) void k_split(SplArgs<T> a) {
  typedef typename CT<T>::type C;
  constexpr int LR = spl_lr<T>(), R = 1 << LR, NT = spl_nt<T>();

  extern __shared__ __align__(16) unsigned char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  typedef typename TE<T>::type E;
  E* __restrict__ ltab = reinterpret_cast<E*>(lds + spl_tile_lds<T>());
  E* __restrict__ lsm = ltab + 1024;  // the 16-entry tables (read once per tile)
  const SplitDesc d = a.d;
  const PacketGeom& G = *a.geom;
  const uint64_t off = G.off;
  const C* __restrict__ src = a.src + off;
  C* __restrict__ dst = a.dst + off;
  const uint32_t t = threadIdx.x;
  for (uint32_t i = t; i < 1024u; i += NT) {
    ltab[i] = a.AG[d.tab + i];
    if (i < (uint32_t)SPL_SMALL) lsm[i] = (i < 16u && KIND != SPL_C_RT) ? a.AG[d.small + i] : a.MG[d.small + i];
  }
  __syncthreads();

  // Tile index u = run + R X + 16 R Y + 64 R Z.  In the Z- and Y-line layouts a
  // lane's (run, X) = (t & (R-1), (t >> LR) & 15) and the rest of its position,
  // t >> (LR+4), is the same across a wave (64 lanes): HBM addresses are a
  // wave-uniform base plus a 32-bit lane offset.
  const uint32_t run = t & (uint32_t)(R - 1);
  const uint32_t lX = (t >> LR) & 15u;
  const uint32_t wY = t >> (LR + 4);
  const uint32_t wYs = __builtin_amdgcn_readfirstlane(wY);
  const uint32_t loff = run | (lX << d.pX);
  // Z lines: thread (run, X, Y = wY), point k at Z = k: u = t + NT k
  const uint32_t zbase = wYs << d.pY;
  const uint32_t zg = lX + 16u * wY;  // + 64 k
  const uint32_t zl = pad16(t);       // + (NT + NT/16) k
  // X lines: thread (run, Y, Z), point k at X = k (pad16 of u + R k is pad16(u) + R k +
  // (R k >> 4), as run + R (k mod (16/R)) stays below 16)
  const uint32_t xY = (t >> LR) & 3u, xZ = t >> (LR + 2);
  const uint32_t xl = pad16(run + 16u * R * xY + 64u * R * xZ);
  // Y lines: thread (run, X, Zb + i), Zb = 4 wY, point 4 i + j at Y = j
  const uint32_t yZb = 4u * wYs;
  const uint32_t yl = pad16(run + R * lX + 256u * R * wY);  // + 17 R j + 68 R i
  const uint32_t yg = lX + 256u * wY;                       // + 16 j + 64 i
  // complex128 round trip: a thread's A factors (pass C's A_X A_Z at its fixed X; Z = k
  // on load, Zb + i on store) are the same in every tile and stay in registers for the
  // launch (complex64 has no registers to spare at 1024 threads)
  constexpr bool AREG = KIND == SPL_C_RT && sizeof(T) == 8;
  E areg[AREG ? 16 : 1], creg[AREG ? 4 : 1];
  if constexpr (AREG) {
#pragma unroll
    for (int k = 0; k < 16; ++k) areg[k] = ltab[zg + 64u * k];
#pragma unroll
    for (int i = 0; i < 4; ++i) creg[i] = ltab[yg + 64u * i];
  }

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
  // The first tile's loads complete here, once: left in flight, they meet the
  // loop's back edge at its header, and the compiler's wait there (sized for this
  // entry) then also drains the previous tile's stores on every iteration, so
  // that no store overlaps the next tile's work.
  __builtin_amdgcn_s_waitcnt(0);

  double acc[MGK_NACC];
#pragma unroll
  for (int k = 0; k < MGK_NACC; ++k) acc[k] = 0.0;

  // LDS moves between the three line layouts.  A barrier follows each move into
  // LDS and each read of the Y lines (the next tile's Z-line writes land on other
  // threads' slots); none is needed between reading the X lines and writing them
  // back, since a thread writes exactly the slots it read (the X-line slots of
  // (thread, point) cover the tile once).
  // (pad16 of u + 16 m is pad16(u) + 17 m when u's low four bits stay below 16)
  constexpr uint32_t ZS = NT + NT / 16;
  auto z_to_lds = [&](C* x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) lds[zl + ZS * k] = x[k];
  };
  auto x_to_lds = [&](C* x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) lds[xl + R * k + ((R * k) >> 4)] = x[k];
  };
  auto lds_to_x = [&](C* x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = lds[xl + R * k + ((R * k) >> 4)];
  };
  auto lds_to_y = [&](C* x) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) x[4 * i + j] = lds[yl + 17u * R * j + 68u * R * i];
  };

  for (uint32_t tile = blockIdx.x; tile < d.ntiles; tile += gridDim.x) {
    const uint32_t base = tile_base(tile);
    const uint32_t oth = (base >> d.pYc) & 3u;  // the split axis' other digit (B: n0, C: k0)
    C x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = xn[k];
    if (tile + gridDim.x < d.ntiles) load(tile + gridDim.x);

    if constexpr (KIND == SPL_B_INV) {
      // Z lines as loaded, each at a fixed stored digit k0 = wY: undo the twiddle and
      // c(n0) and apply M of X and Z (all pointwise), inverse DFTs along Z and X, then
      // along the Y digit in the Y-line layout, conj(A), store from there
      const E sx = te_prod<T>(lsm[48u + lX], lsm[4u * oth + wY], true);
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = tmul<T>(tmul<T>(x[k], sx), lsm[64 + k]);
      dft16<T, true>(x);
      z_to_lds(x);
      __syncthreads();
      lds_to_x(x);
      dft16<T, true>(x);
      x_to_lds(x);
      __syncthreads();
      lds_to_y(x);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) dft4(&x[4 * i], true);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = tmul<T>(x[4 * i + j], ltab[yg + 16u * j + 64u * i], true);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) (dst + ybase(base, i, j))[loff] = x[4 * i + j];
    } else if constexpr (KIND == SPL_C_RT) {
      // per-axis round trips: A of X and Z, then along Z: DFT, M_Z, inverse DFT; the
      // X lines the same with M_X; the Y digit with M_2 at k = k0 + 4 k1; conj(A)
      const E* __restrict__ m2 = lsm;
      const E* __restrict__ mx = lsm + 16;
      const E* __restrict__ mz = lsm + 32;
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = tmul<T>(x[k], AREG ? areg[AREG ? k : 0] : ltab[zg + 64u * k]);
      dft16<T, false>(x);
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = tmul<T>(x[k], mz[k]);
      dft16<T, true>(x);
      z_to_lds(x);
      __syncthreads();
      lds_to_x(x);
      dft16<T, false>(x);
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = tmul<T>(x[k], mx[k]);
      dft16<T, true>(x);
      x_to_lds(x);
      __syncthreads();
      lds_to_y(x);
      __syncthreads();
      // Y lines one at a time, each stored as soon as it is done (its stores then
      // overlap the next lines' work: complex128 30.5 -> 30.1 ms, complex64 15.2 ->
      // 14.9 ms per launch; pass B's inverse, with less work per line, measured
      // slower that way in complex64 and keeps its stores at the end)
      E m[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) m[j] = m2[oth + 4 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dft4(&x[4 * i], false);
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = tmul<T>(x[4 * i + j], m[j]);
        dft4(&x[4 * i], true);
        // pass C's A table is A_X A_Z, the same for every Y: one entry per Z line
        const E ca = AREG ? creg[AREG ? i : 0] : ltab[yg + 64u * i];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          x[4 * i + j] = tmul<T>(x[4 * i + j], ca, true);
          (dst + ybase(base, i, j))[loff] = x[4 * i + j];
        }
      }
    } else if constexpr (KIND == SPL_C_MOM && sizeof(T) == 8) {
      // momentum moments (complex128).  Each axis' moment needs only that axis transformed (the
      // sum of |c|^2 over the other axes is the same in either representation), so
      // the Z lines after their DFT give the total weight and the moments of Z, of
      // the run (axis D-1) and of the tile constants; the X lines and the Y lines
      // are both read from one LDS copy of that Z-transformed tile (one LDS write
      // and two barriers per tile; complex128 13.9 -> 13.5 ms per launch, while the
      // complex64 pass measured 8.1 -> 8.5 ms that way and keeps the layout of pass B
      // below).  Axis axY has k = k0 + 4 k1 (k0 = oth, k1 = j).
      constexpr int AX = SPL_AX[1][0], AZ = SPL_AX[1][1], AY = SPL_SPLIT_AXIS;
      auto w2 = [](const C v) -> double { return (double)v.x * (double)v.x + (double)v.y * (double)v.y; };
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = tmul<T>(x[k], ltab[zg + 64u * k]);
      dft16<T, false>(x);
      // The unnormalised DFTs scale the weights by 16 (dft16) and 4 (dft4): each sum
      // is brought to that of the fully transformed tile (Z, X and Y done) by an exact
      // power of two, 64 (Z lines), 4 (X lines) or 16 (Y lines), and goes into acc
      // at once (fewer values live across the LDS moves).
      {
        double ws = 0.0, mz = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const double w = w2(x[k]);
          ws += w;
          mz += w * ((double)k - 8.0);
        }
        ws *= 64.0;
        acc[0] += ws;
        acc[1 + 7] += ws * ((double)(run | (base & 15u)) - 8.0);  // axis 7: the run and (complex128) bit 3
        acc[1 + AZ] += 64.0 * mz;
#pragma unroll
        for (int l = 0; l < 7; ++l)
          if (l != AX && l != AY && l != AZ)
            acc[1 + l] += ws * ((double)((base >> (4 * (7 - l))) & 15u) - 8.0);
      }
      z_to_lds(x);
      __syncthreads();
      lds_to_x(x);
      dft16<T, false>(x);
      {
        double mx = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) mx += w2(x[k]) * ((double)k - 8.0);
        acc[1 + AX] += 4.0 * mx;
      }
      lds_to_y(x);
      __syncthreads();
      double wj[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dft4(&x[4 * i], false);
#pragma unroll
        for (int j = 0; j < 4; ++j) wj[j] += w2(x[4 * i + j]);
      }
      double my = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) my += wj[j] * ((double)(oth + 4u * j) - 8.0);
      acc[1 + AY] += 16.0 * my;
    } else {
      // forward half (pass B, and the complex64 moments): A factors, DFT along Z, X,
      // then the 4-point Y digit
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = tmul<T>(x[k], ltab[zg + 64u * k]);
      dft16<T, false>(x);
      z_to_lds(x);
      __syncthreads();
      lds_to_x(x);
      dft16<T, false>(x);
      x_to_lds(x);
      __syncthreads();
      lds_to_y(x);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) dft4(&x[4 * i], false);
      if constexpr (KIND == SPL_B_FWD) {
        // k0 = j: twiddle W16^(n0 k0) and the low digit's A factor c(n0)
        E s[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] = lsm[4 * oth + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) x[4 * i + j] = tmul<T>(x[4 * i + j], s[j]);
      }
      if constexpr (KIND == SPL_C_MOM) {
        // momentum moments of the fully transformed tile: axis axY has k = k0 + 4 k1
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
        acc[1 + 7] += ws * ((double)(run | (base & 15u)) - 8.0);  // axis 7: the run and (complex128) bit 3
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
    block_reduce<NT>(acc, G.D + 2, a.partials + (size_t)blockIdx.x * MGK_NACC, (double*)lds_raw);
}

}  // namespace mgk
