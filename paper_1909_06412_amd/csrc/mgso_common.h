// mgso_common.h -- descriptors shared by the host runtime and the gfx950 kernels.
//
// Layout of one wavepacket on the device: N = prod_l N_l complex values, C-ordered
// (the last axis contiguous), c_J = psi(q^J) sqrt(prod_l dq_l).
//
// A "sweep" transforms a contiguous range of axes [a, b) of the array viewed as
// [O][L_G][I] (O = prod_{l<a} N_l, L_G = prod_{a<=l<b} N_l, I = prod_{l>=b} N_l).
// One tile is staged in LDS:
//   kind 0 (b == D):  ob consecutive outer rows x L_G        (contiguous in HBM)
//   kind 1 (b <  D):  L_G x a run of r consecutive inner indices (runs of r*S bytes)
// Every axis of the group is transformed inside the tile by radix-2/3/4/5/8
// Stockham passes; ragged last tiles are zero-padded in LDS and not stored.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#define __forceinline__ inline
#endif

#define MGK_MAXD 8
#define MGK_MAXPASS 12
#define MGK_TMAX 4096           // complex elements per LDS tile
#define MGK_NACC (MGK_MAXD + 2) // reduction slots: sum w, sum w*x_l (D), sum w*e

// Exact unsigned division by an invariant d for x*d < 2^32 (all in-tile indices).
struct Div32 {
  uint32_t d, m;
};
__host__ __device__ __forceinline__ uint32_t div32(uint32_t x, Div32 v) {
#ifdef __HIP_DEVICE_COMPILE__
  return v.d == 1 ? x : __umulhi(x, v.m);
#else
  return v.d == 1 ? x : (uint32_t)(((uint64_t)x * v.m) >> 32);
#endif
}
static inline Div32 make_div32(uint32_t d) {
  Div32 v;
  v.d = d;
  v.m = d <= 1 ? 0u : (uint32_t)((((uint64_t)1) << 32) / d + 1);
  return v;
}

// Exact division of 32-bit values by d using a 64-bit magic (x*d < 2^64 always).
struct DivW {
  uint32_t d;
  uint32_t pad;
  uint64_t m;
};
__host__ __device__ __forceinline__ uint32_t divw(uint32_t x, DivW v) {
  if (v.d == 1) return x;
#ifdef __HIP_DEVICE_COMPILE__
  return (uint32_t)__umul64hi((uint64_t)x, v.m);
#else
  return (uint32_t)(((unsigned __int128)x * v.m) >> 64);
#endif
}
static inline DivW make_divw(uint32_t d) {
  DivW v;
  v.d = d;
  v.pad = 0;
  v.m = d <= 1 ? 0ull : (uint64_t)((((unsigned __int128)1) << 64) / d + 1);
  return v;
}

struct PassDesc {
  uint16_t R;       // radix of this pass
  uint16_t Ns;      // product of the radices of the earlier passes
  uint16_t tws;     // n / (Ns R): twiddle index step
  uint16_t pad;
  Div32 dNs;        // division by Ns
  Div32 dNbl;       // division by n / R (butterflies per line)
};

struct AxisDesc {
  int32_t n;        // points on this axis
  int32_t tw_off;   // offset of exp(-2 pi i m / n), m < n, in the twiddle table
  int32_t tab_off;  // offset of this axis in the per-packet A / M tables
  int32_t npass;
  PassDesc pass[MGK_MAXPASS];
  DivW dn;          // division by n (index decode)
  double dq, dp, minv;
};

struct SweepDesc {
  int32_t a, b;           // axes [a, b)
  int32_t kind;           // 0: rows x L_G, 1: L_G x run
  uint32_t O, LG, I;      // outer, group and inner extents
  uint32_t ob, r;         // rows per tile (kind 0) / run length (kind 1)
  uint32_t T;             // elements in a full tile
  uint32_t tiles_i;       // tiles along the inner extent (kind 1)
  uint32_t ntiles;        // tiles in the sweep
  Div32 dLG, dr;          // in-tile decode of (row, g) or (g, ii)
  DivW dtiles_i;          // tile -> (o, inner block)
  uint32_t S[MGK_MAXD];   // LDS stride of each axis of the group (index l - a)
  Div32 dS[MGK_MAXD];
  int32_t gtab_off;       // offset of the group-combined phase tables (16-point path)
  int32_t pad;
};

struct PacketGeom {
  int32_t D;
  int32_t nsweeps;
  uint64_t N_total;       // points (<= 2^32; 16^8 = 2^32 needs 64 bits)
  uint64_t off;           // element offset of this packet in the state buffer
  int32_t tab_len;        // sum_l N_l (A and M tables)
  int32_t fast16;         // every axis has 16 points and D >= 3: 16-point sweep kernels
  int32_t gtab_len;       // sum over sweeps of the group sizes (combined tables)
  int32_t split;          // 1: the three-pass plan of 16^8 complex64 grids (tables at gtab_len)
  double hbar;
  AxisDesc ax[MGK_MAXD];
  SweepDesc sw[MGK_MAXD];
};

// Per-packet dynamic state (FP64), updated on the device by the finalize steps.
struct PacketState {
  double q_c[MGK_MAXD];
  double p_c[MGK_MAXD];
  double delta[MGK_MAXD];
  double last[MGK_NACC];  // last reduced moments of a substep
  double obs[2 * MGK_NACC]; // observables: position-grid then momentum-grid sums
  double t;
  double scale;           // renormalisation factor for the next pointwise pass
  int32_t err;
  int32_t fixed;          // 1: grid centres held (fixed grid; the naive scheme between re-centrings)
};

#define MGK_POT_MAXPAR 24
struct PotDesc {
  int32_t kind;           // mg_pot
  int32_t D;
  double p[MGK_POT_MAXPAR];
};

// Stockham index helpers (shared with a host-side checker).
// Butterfly bf of a pass over an axis of length n and LDS stride S:
//   lo = bf % S, rest = bf / S, j = rest % (n/R), hi = rest / (n/R)
//   base = hi*n*S + lo; inputs at base + (j + r n/R) S, outputs at base + ((j-k)R + k + r Ns) S
//   with k = j % Ns; twiddle exp(-+2 pi i r k / (Ns R)) = tw[r k n / (Ns R)].
__host__ __device__ __forceinline__ void bfly_index(uint32_t bf, uint32_t n, uint32_t S, Div32 dS,
                                                     Div32 dNbl, uint32_t* base, uint32_t* j) {
  uint32_t rest = div32(bf, dS);
  uint32_t lo = bf - rest * S;
  uint32_t hi = div32(rest, dNbl);
  *j = rest - hi * dNbl.d;
  *base = hi * n * S + lo;
}
