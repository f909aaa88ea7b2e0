// mgso_sweep16.h -- sweep kernel for packets whose axes all have 16 points
// (the 8-D Henon-Heiles grid 16^8 and any 16^D, D >= 3).
//
// A contiguous tile (K = 3, the innermost three axes) holds 16^3 = 4096 points and
// is worked by 256 threads; a strided tile holds the K < 3 group axes of the sweep
// (16^K points) times a run of r = 8192 / 16^K consecutive inner indices and is
// worked by 512 threads (the longer runs, 256 bytes and up, keep the memory
// system busier at large strides).  For every group axis there is exactly one
// line of 16 points per thread, transformed by a radix-16 DFT in registers.
// Axes are taken outermost first: the first one is loaded straight from HBM into
// registers (lanes run along its large stride, so a wave reads whole 128-byte
// lines); the others go through LDS; the last one is stored straight from
// registers when its stride is >= 16 points, else through one more LDS transpose
// so that a wave writes 512 contiguous bytes.
//
// The per-axis phase factors of the kinetic substep (Sec. II.G.2, Eq. (55)) are
// applied once per point from tables combined over the sweep's group axes:
//   AG[g] = prod_{l in group} A_l(j_l)   (forward: on load; inverse: conj on store)
//   MG[g] = prod_{l in group} M_l(k_l)   (inverse: on load)
// built in FP64 (one sincos of the summed angle) and rounded once.
#pragma once
#include "mgso_kernels.h"

namespace mgk {

struct S16Desc {
  int32_t K;          // group axes (1..3)
  int32_t a;          // first group axis
  int32_t kind;       // 0: tile = 16^K contiguous points (r = 1), 1: 16^K x r
  int32_t lr;         // log2 r
  int32_t lI;         // log2 I (inner extent)
  int32_t lLG;        // log2 16^K
  int32_t lS[3];      // log2 of the tile stride of group axis e (e = 0 outermost)
  uint32_t tiles_i;   // tiles along the inner extent (kind 1)
  int32_t ltiles_i;   // log2 tiles_i
  uint32_t ntiles;
  int32_t gtab_off;   // offset of this sweep's AG / MG tables
};

template <typename T> struct S16Args {
  const PacketGeom* geom;
  const PacketState* st;
  const PotDesc* pot;
  const typename CT<T>::type* src;
  typename CT<T>::type* dst;
  const typename TE<T>::type* AG;
  const typename TE<T>::type* MG;
  double* partials;
  S16Desc d;
  double h;
};

// 16-point DFT in registers, natural order in and out (4 x 4 decomposition).
// The twiddles are applied with compensated constants in complex64 (kmul, crotk):
// each acts as the exact root of unity, so the DFT keeps the norm on average.
template <typename T, bool INV, typename C> __device__ __forceinline__ void dft16(C* x) {
  const double c1 = 0.92387953251128675612818318939679;  // cos(pi/8)
  const double s1 = 0.38268343236508977172845998403040;  // sin(pi/8)
  const double r2 = 0.70710678118654752440084436210485;
  C y[16];
  // DFT4 over n1 for each n2: inputs x[4 n1 + n2]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C v[4] = {x[n2], x[4 + n2], x[8 + n2], x[12 + n2]};
    dft4(v, INV);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[4 * n2 + k1] = v[k1];
  }
  // twiddles W16^(n2 k1), W16 = exp(-+ 2 pi i / 16)
  auto tw = [&](C v, int m) -> C {
    // exp(-i pi m / 8) for forward, conjugate for inverse
    const double sg = INV ? 1.0 : -1.0;
    switch (m) {
      case 1: return crotk<T>(v, c1, sg * s1);
      case 3: return crotk<T>(v, s1, sg * c1);
      case 9: return crotk<T>(v, -c1, -sg * s1);  // cos(9pi/8) = -c1, sin(9pi/8) = -s1
      case 2: {  // r2 (1 -+ i)
        const T a = INV ? v.x - v.y : v.x + v.y, b = INV ? v.x + v.y : v.y - v.x;
        return C{kmul<T>(a, r2), kmul<T>(b, r2)};
      }
      default: {  // m = 6: r2 (-1 -+ i)
        const T a = INV ? -v.x - v.y : v.y - v.x, b = INV ? v.x - v.y : -v.x - v.y;
        return C{kmul<T>(a, r2), kmul<T>(b, r2)};
      }
    }
  };
  y[4 * 1 + 1] = tw(y[5], 1);
  y[4 * 1 + 2] = tw(y[6], 2);
  y[4 * 1 + 3] = tw(y[7], 3);
  y[4 * 2 + 1] = tw(y[9], 2);
  y[4 * 2 + 2] = rot(y[10], INV);  // W^4 = -+ i
  y[4 * 2 + 3] = tw(y[11], 6);
  y[4 * 3 + 1] = tw(y[13], 3);
  y[4 * 3 + 2] = tw(y[14], 6);
  y[4 * 3 + 3] = tw(y[15], 9);
  // DFT4 over n2 for each k1: X[k1 + 4 k2]
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C v[4] = {y[k1], y[4 + k1], y[8 + k1], y[12 + k1]};
    dft4(v, INV);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = v[k2];
  }
}

__device__ __forceinline__ uint32_t pad16(uint32_t t) { return t + (t >> 4); }

// Potentials that are polynomials of degree <= 3 in each coordinate (free,
// harmonic, quadratic, Henon-Heiles): along a line of 16 points V is a cubic of
// the line coordinate and each dV/dq_m a quadratic, so a Taylor expansion at the
// line centre is exact.  (These are the only kinds a 16^D grid with D >= 3 can
// carry.)
static inline bool pot_is_cubic(int kind) { return kind != 2; }

// v exp(-i phi): complex64 by mul_phase_f32, complex128 by the FP64 series.
template <typename T, typename C> __device__ __forceinline__ C mul_phase16(C v, double phi) {
  if constexpr (sizeof(T) == 4) return mul_phase_f32(v, phi);
  else return cmul(v, phase_poly64(phi));
}

// Potential part of the line epilogue (Sec. II.G.1, Eqs. (45), (47)) for a line
// along packet axis L whose other indices are jfix.  With u = x - x_c (x_c the
// centre q_ctr,L, line point 8) and s = u / dq_L = k - 8, the moments of the
// weights M0 = sum w, M1 = sum w s, M2 = sum w s^2 give
//   sum_k w_k dV/dq_m(x_k) = b0_m M0 + b1_m dq M1 + b2_m dq^2 M2,
// where dV/dq_m = b0_m + b1_m u + b2_m u^2 along the line, and
//   V(s) = c0 + c1 s + c2 s^2 + c3 s^3,  c0 = V(x_c), c1 = b0_L dq,
//   c2 = b1_L dq^2 / 2, c3 = b2_L dq^3 / 3.
// b0 is the gradient at the line centre; b1, b2 are nonzero only where the
// gradient depends on x (one entry for the harmonic kind, one column of K for
// the quadratic kind, axes L-1, L, L+1 for Henon-Heiles).
// Packet constants the epilogue needs, staged in LDS once per workgroup: reads of
// global memory inside the tile loop cannot use the scalar cache (the loop
// stores to the state), so each would be a vector load waited on in turn.
struct LineCst {
  double qc[MGK_MAXD], dq[MGK_MAXD], pc[MGK_MAXD];
  double ihb;
  PotDesc pot;
};

__device__ __forceinline__ void stage_line_cst(LineCst& lc, const PacketGeom& G, const PacketState& st,
                                               const PotDesc& P) {
  const uint32_t t = threadIdx.x;
  if (t < MGK_MAXD) {
    lc.qc[t] = st.q_c[t];
    lc.dq[t] = G.ax[t].dq;
    lc.pc[t] = st.p_c[t];
  }
  if (t < MGK_POT_MAXPAR) lc.pot.p[t] = P.p[t];
  if (t == 0) {
    lc.ihb = 1.0 / G.hbar;
    lc.pot.kind = P.kind;
    lc.pot.D = P.D;
  }
  __syncthreads();
}

template <int PK>
__device__ __forceinline__ void line_model(int L, const int* jfix, double M0, double M1, double M2, int D,
                                           const LineCst& lc, double* acc, double* cp) {
  const PotDesc& P = lc.pot;
  double q[MGK_MAXD], g[MGK_MAXD];
#pragma unroll
  for (int l = 0; l < MGK_MAXD; ++l)
    if (l < D) q[l] = l == L ? lc.qc[l] : lc.qc[l] + (double)(jfix[l] - 8) * lc.dq[l];
  const double V0 = pot_eval<PK>(P, D, q, g);
  const double d = lc.dq[L];
  const double S1 = d * M1, S2 = d * d * M2;
  double b0L = 0.0, b1L = 0.0, b2L = 0.0;
  if (PK == 1) b1L = P.p[L];
  if (PK == 4) b1L = P.p[L * D + L];
  double xc = 0.0, ym = 0.0, yp = 0.0;
  if (PK == 3) {
#pragma unroll
    for (int l = 0; l < MGK_MAXD; ++l) {
      if (l == L) xc = q[l];
      if (l + 1 == L) ym = q[l];
      if (l == L + 1 && l < D) yp = q[l];
    }
    const double ka = P.p[0], la = P.p[1];
    b1L = ka;
    if (L + 1 < D) b1L += 2.0 * la * yp;
    if (L >= 1) {
      b1L -= 2.0 * la * xc;
      b2L = -la;
    }
  }
#pragma unroll
  for (int m = 0; m < MGK_MAXD; ++m) {
    if (m >= D) continue;
    double v = g[m] * M0;
    if (m == L) {
      b0L = g[m];
      v += b1L * S1 + b2L * S2;
    }
    if (PK == 4 && m != L) v += P.p[m * D + L] * S1;
    if (PK == 3) {
      const double la = P.p[1];
      if (m + 1 == L) v += 2.0 * la * ym * S1;
      if (m == L + 1) v += 2.0 * la * xc * S1 + la * S2;
    }
    acc[1 + m] += v;
  }
  cp[0] = V0;
  cp[1] = b0L * d;
  cp[2] = 0.5 * b1L * d * d;
  cp[3] = b2L * (1.0 / 3.0) * d * d * d;
}

// Henon-Heiles (Sec. III.C) on a contiguous tile, which holds the innermost three
// axes L, L+1, L+2 (= D-3..D-1): every term of V and of dV/dq_m that involves only
// the outer axes is the same for the whole tile and comes from LDS (tcs: per outer
// axis m its share of V, its gradient component without the x-dependent pair
// (L-1, L), and q_{L-1}); the line along axis L adds the terms of its own axes.
// Same quantities as line_model, in two parts: the line's terms (which give the
// cubic V(s), s = k - 8, before the weights are known) and, once the weight moments
// are summed, their gradient sums into acc.
struct HHTile {
  double V0, gL, gL1, gL2, b1L, b2L, qm, xc;
};
__device__ __forceinline__ HHTile hh_tile_terms(int L, int j1, int j2, const LineCst& lc, const double* tcs) {
  const double ka = lc.pot.p[0], la = lc.pot.p[1];
  HHTile h;
  h.xc = lc.qc[L];
  const double xc = h.xc;
  const double y = lc.qc[L + 1] + (double)(j1 - 8) * lc.dq[L + 1];
  const double z = lc.qc[L + 2] + (double)(j2 - 8) * lc.dq[L + 2];
  const bool hasm = L >= 1;
  h.qm = hasm ? tcs[2 * MGK_MAXD] : 0.0;
  const double qm = h.qm;
  double tout = 0.0;
#pragma unroll
  for (int m = 0; m < MGK_MAXD; ++m)
    if (m < L) tout += tcs[m];
  h.V0 = tout + (hasm ? la * (qm * qm * xc - xc * xc * xc * (1.0 / 3.0)) : 0.0) +
         0.5 * ka * (xc * xc + y * y + z * z) + la * (xc * xc * y - y * y * y * (1.0 / 3.0)) +
         la * (y * y * z - z * z * z * (1.0 / 3.0));
  h.gL = ka * xc + (hasm ? la * (qm * qm - xc * xc) : 0.0) + 2.0 * la * xc * y;
  h.gL1 = ka * y + la * (xc * xc - y * y) + 2.0 * la * y * z;
  h.gL2 = ka * z + la * (y * y - z * z);
  h.b1L = ka + 2.0 * la * y - (hasm ? 2.0 * la * xc : 0.0);
  h.b2L = hasm ? -la : 0.0;
  return h;
}
__device__ __forceinline__ void hh_tile_cp(const HHTile& h, int L, const LineCst& lc, double* cp) {
  const double d = lc.dq[L];
  cp[0] = h.V0;
  cp[1] = h.gL * d;
  cp[2] = 0.5 * h.b1L * d * d;
  cp[3] = h.b2L * (1.0 / 3.0) * d * d * d;
}
__device__ __forceinline__ void hh_tile_acc(const HHTile& h, int L, int D, double M0, double M1, double M2,
                                            const LineCst& lc, const double* tcs, double* acc) {
  const double la = lc.pot.p[1];
  const double d = lc.dq[L];
  const double S1 = d * M1, S2 = d * d * M2;
#pragma unroll
  for (int m = 0; m < MGK_MAXD; ++m) {
    if (m >= D) continue;
    double v;
    if (m < L - 1) v = tcs[MGK_MAXD + m] * M0;
    else if (m == L - 1) v = (tcs[MGK_MAXD + m] + 2.0 * la * h.qm * h.xc) * M0 + 2.0 * la * h.qm * S1;
    else if (m == L) v = h.gL * M0 + h.b1L * S1 + h.b2L * S2;
    else if (m == L + 1) v = h.gL1 * M0 + 2.0 * la * h.xc * S1 + la * S2;
    else v = h.gL2 * M0;
    acc[1 + m] += v;
  }
}

// Epilogue on a line held in registers (strided tiles): moments (REDP) or the
// potential substep (V) with weights w_k = |x_k|^2.
template <typename T, int EPI, int PK>
__device__ __forceinline__ void line_epilogue(typename CT<T>::type* x, int L, uint64_t f, int D, const LineCst& lc,
                                              double hh, double* acc) {
  int jfix[MGK_MAXD];
#pragma unroll
  for (int l = 0; l < MGK_MAXD; ++l)
    if (l < D) jfix[l] = (int)((f >> (4 * (D - 1 - l))) & 15);
  double wl = 0.0, ml = 0.0, m2 = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const double w = (double)x[k].x * (double)x[k].x + (double)x[k].y * (double)x[k].y;
    wl += w;
    ml += w * (double)(k - 8);
    if (EPI == EPI_V) m2 += w * (double)((k - 8) * (k - 8));
  }
  acc[0] += wl;
  if (EPI == EPI_REDP) {
#pragma unroll
    for (int l = 0; l < MGK_MAXD; ++l)
      if (l < D) acc[1 + l] += (l == L) ? ml : wl * (double)(jfix[l] - 8);
  }
  if (EPI == EPI_V) {
    double cp[4];
    line_model<PK>(L, jfix, wl, ml, m2, D, lc, acc, cp);
#pragma unroll
    for (int i = 0; i < 4; ++i) cp[i] *= hh;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double sk = (double)(k - 8);
      const double phi = cp[0] + sk * cp[1] + (sk * sk) * cp[2] + (sk * sk * sk) * cp[3];
      x[k] = mul_phase16<T>(x[k], phi);
    }
  }
}

// Dynamic LDS of k_sweep16, in complex elements: the tile (with the pad16 gaps)
// when there are transposes, then (strided tiles) the group tables of the sweep:
// the pre-multiplication (forward A, inverse M) and, inverse, the conj(A) factors
// of the store.  The final FP64 reduction reuses the start of the buffer.
// Threads of a k_sweep16 workgroup and points of its tile (16 per thread).
__host__ __device__ constexpr int k16_threads(int K) { return K < 3 ? 512 : 256; }
// Padded tile (pad16 gaps) when there are transposes through LDS.
__host__ __device__ constexpr uint32_t k16_tile_lds(int K) {
  return K > 1 ? (uint32_t)(16 * k16_threads(K)) + (uint32_t)k16_threads(K) : 0u;
}
__host__ __device__ constexpr uint32_t k16_lds_tab(int K, bool INV) {
  return K < 3 ? (1u << (4 * K)) * (INV ? 2u : 1u) : 0u;
}
// complex64 contiguous tiles alternate between two tile buffers (the transposes'
// reads then need no barrier of their own): 68 KiB, two workgroups per CU
template <typename T> __host__ __device__ constexpr bool k16_pingpong(int K) { return K == 3 && sizeof(T) == 4; }
template <typename T> __host__ __device__ constexpr size_t k16_lds_bytes(int K, bool INV) {
  // the tile(s) in complex elements, then the tables in 16-byte table entries
  const size_t b = (size_t)k16_tile_lds(K) * (k16_pingpong<T>(K) ? 2 : 1) * 2 * sizeof(T) +
                   (size_t)k16_lds_tab(K, INV) * 16;
  const size_t red = (size_t)(k16_threads(K) / 64) * MGK_NACC * sizeof(double);
  return b > red ? b : red;
}

// Sweep modes (profile classes): SW_SPLIT / SW_SPLIT_MOM are the passes of the
// three-pass 16^8 plan (the latter reduced to the momentum moments, no store).
enum : int { SW_FULL = 0, SW_MOMENTS = 1, SW_ROUNDTRIP = 2, SW_SPLIT = 3, SW_SPLIT_MOM = 4 };

// MODE (strided one-axis sweeps only) splits a kinetic substep differently at its
// turning point, where the last forward sweep meets the first inverse sweep on the
// same axis group: SW_MOMENTS is that forward sweep reduced to its momentum moments
// (nothing is stored, the axis stays untransformed in memory), SW_ROUNDTRIP the inverse
// sweep that then does the forward DFT, the M factor and the inverse DFT of the axis
// in registers.  Same arithmetic as the two full sweeps, one HBM write and one read
// fewer.
// DT > 0 fixes the packet dimension at compile time (contiguous tiles only, where the
// tile's first axis is a = DT - 3), so that the per-axis loops of the epilogue unroll
// without tests on D.
template <typename T, int K, bool INV, int EPI, int PK = -1, int MODE = 0, int DT = 0>
__global__ __launch_bounds__(k16_threads(K)) __attribute__((amdgpu_waves_per_eu(2)))
void k_sweep16(S16Args<T> a) {
  static_assert(DT == 0 || (K == 3 && DT >= 3 && DT <= MGK_MAXD), "a fixed dimension needs a contiguous tile");
  static_assert(MODE == SW_FULL || (K == 1 && (MODE == SW_MOMENTS) == (!INV && EPI == EPI_REDP) &&
                                    (MODE == SW_ROUNDTRIP) == (INV && EPI == 0)),
                "moments-only and round-trip sweeps are one-axis strided sweeps");
  constexpr int NT = k16_threads(K);
  typedef typename CT<T>::type C;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  // Ping-pong (complex64 contiguous tiles): the three transposes of a tile use
  // buffers b0, b1, b0 and the next tile starts on b1.  Every write to a buffer then
  // follows a barrier that comes after all reads of that buffer, so only the
  // barrier after each write is needed (three per tile instead of six).
  constexpr bool PP = k16_pingpong<T>(K);
  C* lb0 = lds;
  C* lb1 = lds + (PP ? k16_tile_lds(K) : 0u);
  const PacketGeom& G = *a.geom;
  const S16Desc d = a.d;
  // every 16^D plan has contiguous 16^3 tiles for K = 3 and strided tiles below
  constexpr int KIND = K == 3 ? 0 : 1;
  const int D = DT ? DT : G.D;
  const uint32_t t = threadIdx.x;
  double acc[MGK_NACC];
#pragma unroll
  for (int k = 0; k < MGK_NACC; ++k) acc[k] = 0.0;
  const double hh = a.h / G.hbar;
  const uint64_t off = G.off;  // read once: stores to dst must not force reloads
  const C* __restrict__ src = a.src + off;
  C* __restrict__ dst = a.dst + off;
  typedef typename TE<T>::type E;
  const E* __restrict__ AG = a.AG + d.gtab_off;
  const E* __restrict__ MG = a.MG + d.gtab_off;
  __shared__ LineCst lc;
  __shared__ double tcs[2 * MGK_MAXD + 1];  // per-tile outer-axis terms (Henon-Heiles, contiguous tiles)
  if (EPI == EPI_V) stage_line_cst(lc, G, *a.st, *a.pot);
  // Strided tiles keep the sweep's group tables (16^K entries) in LDS for the
  // whole launch; the table index of a thread's points is the same in every tile.
  E* __restrict__ ltab = reinterpret_cast<E*>(lds + k16_tile_lds(K));
  E* __restrict__ lsto = ltab + (1u << (4 * K));
  if constexpr (KIND == 1) {
    for (uint32_t i = t; i < (1u << (4 * K)); i += NT) {
      ltab[i] = INV ? MG[i] : AG[i];
      if (INV) lsto[i] = AG[i];
    }
    __syncthreads();
  }
  // Loads are software-pipelined: the first-axis loads of the next tile are in
  // flight while the current tile is transformed (strided tiles: issued as soon
  // as the current tile's data has arrived; contiguous tiles: once the tile sits
  // in LDS, so that they overlap the epilogue and the stores).  Each tile is read
  // and written by one workgroup only, so this is safe in place.
  // log2 of the tile stride of group axis e; a contiguous 16^3 tile has the strides
  // 256, 16, 1 as constants, so that its LDS addresses below are one per-thread base
  // plus immediate offsets
  auto lS_of = [&](int e_) -> int { return KIND == 0 ? 4 * (K - 1 - e_) : d.lS[e_]; };
  // LDS slot of point k of a line at tile position tau with stride S: pad16(tau + k S),
  // which is pad16(tau) + k (S + S/16) when S is a multiple of 16 or tau is (S = 1)
  auto lslot = [&](uint32_t tau, uint32_t S_, int k) -> uint32_t {
    return KIND == 0 ? pad16(tau) + (uint32_t)k * (S_ + (S_ >> 4)) : pad16(tau + (uint32_t)k * S_);
  };
  auto tile_flat0 = [&](uint32_t tl) -> uint64_t {
    if (KIND == 0) return (uint64_t)tl << 12;
    const uint32_t o = tl >> d.ltiles_i;
    const uint32_t ib = tl & (d.tiles_i - 1);
    return ((uint64_t)o << (d.lLG + d.lI)) + ((uint64_t)ib << d.lr);
  };
  // (complex64 only: the complex128 kernels have no registers to spare)
  constexpr bool PIPE = sizeof(T) == 4;
  C xn[16];
  auto load_first = [&](uint32_t tl) {
    const uint32_t S0 = 1u << lS_of(0);
    const uint32_t tau = ((t >> lS_of(0)) << (lS_of(0) + 4)) + (t & (S0 - 1));
    const uint64_t ms0 = KIND == 0 ? (uint64_t)S0 : ((uint64_t)(S0 >> d.lr) << d.lI);
    const uint32_t lane0 =
        KIND == 0 ? tau : (uint32_t)(((uint64_t)(tau >> d.lr) << d.lI) + (tau & ((1u << d.lr) - 1)));
    const C* __restrict__ ts0 = src + tile_flat0(tl);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const C* __restrict__ bk = ts0 + (uint64_t)k * ms0;
      xn[k] = KIND == 0 ? ntload(bk + lane0) : bk[lane0];
    }
  };
  if (PIPE && blockIdx.x < d.ntiles) load_first(blockIdx.x);
  // A contiguous tile's first-axis factors (point k of thread t: entry t + 256 k of the
  // group table) are the same in every tile: each thread keeps its sixteen in registers.
  // The inverse potential sweep folds the store's conj(AG) into its epilogue: its sign
  // (-1)^m into the phase, its magnitude 4^-K (a power of two, exact) into these factors.
  constexpr bool FOLD = KIND == 0 && INV && EPI == EPI_V;
  E preg[KIND == 0 ? 16 : 1];
  if constexpr (KIND == 0) {
    const E* __restrict__ pre0 = INV ? MG : AG;
    const T mag = FOLD ? (T)(1.0 / (double)(1 << (2 * K))) : (T)1;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      preg[k] = pre0[256 * k + t];
      if constexpr (FOLD) {
        if constexpr (sizeof(T) == 4) preg[k] = E{preg[k].x * mag, preg[k].y * mag, preg[k].z * mag, preg[k].w * mag};
        else preg[k] = E{preg[k].x * mag, preg[k].y * mag};
      }
    }
  }

  for (uint32_t tile = blockIdx.x; tile < d.ntiles; tile += gridDim.x) {
    const uint64_t flat0 = tile_flat0(tile);
    auto flat_of = [&](uint32_t tau) -> uint64_t {
      if (KIND == 0) return flat0 + tau;
      return flat0 + ((uint64_t)(tau >> d.lr) << d.lI) + (tau & ((1u << d.lr) - 1));
    };
    auto g_of = [&](uint32_t tau) -> uint32_t { return KIND == 0 ? tau : (tau >> d.lr); };
    // Along a line of axis e the tile stride S >= r, so consecutive points are a
    // uniform distance apart in memory and in the group tables.
    auto mem_stride = [&](uint32_t S_) -> uint64_t {
      return KIND == 0 ? (uint64_t)S_ : ((uint64_t)(S_ >> d.lr) << d.lI);
    };
    auto tab_stride = [&](uint32_t S_) -> uint32_t { return KIND == 0 ? S_ : (S_ >> d.lr); };

    C x[16];
    E pv[KIND == 1 ? 16 : 1];  // strided inverse: the conj(A) factors of the store
    // ---- first axis: the outermost group axis (largest tile stride), coalesced
    int e = 0;
    uint32_t S = 1u << lS_of(0);
    uint32_t tau0 = ((t >> lS_of(0)) << (lS_of(0) + 4)) + (t & (S - 1));
    {
      // uniform (scalar) base per point k + a 32-bit per-lane offset: the loads
      // use scalar-base addressing and stay in flight together
      const E* __restrict__ pre = KIND == 1 ? ltab : (INV ? MG : AG);
      const uint32_t ts = tab_stride(S);
      const uint32_t glane = g_of(tau0);
      if (!PIPE) load_first(tile);
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = xn[k];
      if (PIPE && KIND == 1 && tile + gridDim.x < d.ntiles) load_first(tile + gridDim.x);
      if constexpr (MODE == SW_ROUNDTRIP) {
        // forward half of the round trip: A factor, DFT (the A table also gives the
        // conj(A) of the store below)
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          pv[k] = lsto[k * ts + glane];
          x[k] = tmul<T>(x[k], pv[k]);
        }
        dft16<T, false>(x);
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = tmul<T>(x[k], KIND == 0 ? preg[k] : pre[k * ts + glane]);
      dft16<T, INV>(x);
    }
    // ---- inner axes through LDS
#pragma unroll
    for (int ee = 1; ee < K; ++ee) {
      C* const lb = (ee & 1) ? lb0 : lb1;
#pragma unroll
      for (int k = 0; k < 16; ++k) lb[lslot(tau0, S, k)] = x[k];
      __syncthreads();
      e = ee;
      S = 1u << lS_of(e);
      tau0 = ((t >> lS_of(e)) << (lS_of(e) + 4)) + (t & (S - 1));
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = lb[lslot(tau0, S, k)];
      if (!PP) __syncthreads();
      if (ee < K - 1) dft16<T, INV>(x);
    }
    // inverse: fetch the conj(A) factors of the store now, so that their latency
    // overlaps the last DFT and the epilogue
    // (a contiguous tile fetches them after the epilogue instead, to keep the
    // epilogue's registers free; they then overlap the LDS transpose)
    if (INV && KIND == 1 && MODE != SW_ROUNDTRIP) {
      const uint32_t ts = tab_stride(S);
      const uint32_t glane = g_of(tau0);
#pragma unroll
      for (int k = 0; k < 16; ++k) pv[k] = lsto[k * ts + glane];
    }
    if (K > 1) dft16<T, INV>(x);
    if constexpr (KIND == 1) {
      // ---- strided tile: epilogue on the thread's line (packet axis L), store
      // 128-byte segments straight from registers
      const int L = d.a + e;
      if (EPI) line_epilogue<T, EPI, PK>(x, L, flat_of(tau0), D, lc, hh, acc);
      if (MODE == SW_MOMENTS) continue;
      const uint64_t ms = mem_stride(S);
      const uint32_t lane = (uint32_t)(flat_of(tau0) - flat0);
      C* __restrict__ tdst = dst + flat0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        C v = x[k];
        if (INV) v = tmul<T>(v, pv[k], true);
        C* __restrict__ bk = tdst + (uint64_t)k * ms;
        bk[lane] = v;
      }
    } else {
      // ---- contiguous tile: the last axis is contiguous.  Transpose through LDS;
      // thread t then owns positions t + 256 m, a line along the outermost group
      // axis (packet axis a), and streams it in one pass: reduces, applies the phase
      // and the conj(A) factor and stores 512 contiguous bytes per wave.
      if constexpr (EPI == EPI_V && PK == 3) {
        // Henon-Heiles terms of the outer axes of this tile (one thread per axis)
        const int L = DT ? DT - 3 : d.a;
        if (t < (uint32_t)L) {
          const double ka = lc.pot.p[0], la = lc.pot.p[1];
          auto qo = [&](int l) {
            return lc.qc[l] + (double)((int)((flat0 >> (4 * (D - 1 - l))) & 15u) - 8) * lc.dq[l];
          };
          const int m = (int)t;
          const double qv = qo(m);
          double term = 0.5 * ka * qv * qv, g = ka * qv;
          if (m >= 1) {
            const double qp = qo(m - 1);
            term += la * (qp * qp * qv - qv * qv * qv * (1.0 / 3.0));
            g += la * (qp * qp - qv * qv);
          }
          if (m + 1 <= L - 1) g += 2.0 * la * qv * qo(m + 1);
          tcs[m] = term;
          tcs[MGK_MAXD + m] = g;
          if (m == L - 1) tcs[2 * MGK_MAXD] = qv;
        }
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) lb0[lslot(tau0, S, k)] = x[k];
      __syncthreads();
      if (PIPE && KIND == 0 && tile + gridDim.x < d.ntiles) load_first(tile + gridDim.x);
      // One pass over the line: per point the weight moments (REDP, V), the phase
      // (V) or the store factor (plain inverse), and the store.  The potential's
      // cubic along the line depends only on the line's position, so its phase is
      // known before the weights; the moments' gradient sums go into acc after.
      const int L = DT ? DT - 3 : d.a;
      const int j1 = (int)((t >> 4) & 15u), j2 = (int)(t & 15u);  // fixed indices on axes L+1, L+2
      int jfix[MGK_MAXD];
      if (EPI) {
        const uint64_t f = flat0 + t;
#pragma unroll
        for (int l = 0; l < MGK_MAXD; ++l)
          if (l < D) jfix[l] = (int)((f >> (4 * (D - 1 - l))) & 15);
      }
      double cp[4] = {0.0, 0.0, 0.0, 0.0};
      HHTile hht{};
      if (EPI == EPI_V) {
        if constexpr (PK == 3) {
          hht = hh_tile_terms(L, j1, j2, lc, tcs);
          hh_tile_cp(hht, L, lc, cp);
        } else {
          double unused[MGK_NACC];
          line_model<PK>(L, jfix, 0.0, 0.0, 0.0, D, lc, unused, cp);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) cp[i] *= hh;
        if (INV) {
          // conj(AG) of the store folded into the same phase: along the line
          // (axis L, index m = s + 8) its angle is ang_t + beta m, times (-1)^m =
          // exp(-i pi s) (its magnitude is in the first-axis factors)
          const double ang_t = M_PI * (double)((j1 & 1) + (j2 & 1)) -
                               (lc.pc[L + 1] * lc.dq[L + 1] * (double)j1 +
                                lc.pc[L + 2] * lc.dq[L + 2] * (double)j2) * lc.ihb;
          const double beta = -lc.pc[L] * lc.dq[L] * lc.ihb;
          cp[0] += ang_t + 8.0 * beta;
          cp[1] += beta + M_PI;
        }
      }
      C* __restrict__ tdst = dst + flat0;
      // the cubic phase at s = m - 8 through its forward differences: the value at
      // s = -8 and the first three differences
      double ph = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
      if (EPI == EPI_V) {
        ph = cp[0] - 8.0 * cp[1] + 64.0 * cp[2] - 512.0 * cp[3];
        d1 = cp[1] - 15.0 * cp[2] + 169.0 * cp[3];
        d2 = 2.0 * cp[2] - 42.0 * cp[3];
        d3 = 6.0 * cp[3];
      }
      // complex128: the factors exp(-i phi(s)) themselves by the same differences,
      // as products: w = exp(-i phi(s)), u = exp(-i dphi(s)), y = exp(-i d2phi(s)),
      // z = exp(-i d3phi) (constant): four FP64 sine/cosine evaluations per line
      // instead of sixteen, three complex products per point (rounding ~1e-15 after
      // the 16 points, unbiased)
      C w{}, u{}, y{}, z{};
      if constexpr (EPI == EPI_V && sizeof(T) == 8) {
        w = phase_poly64(ph);
        u = phase_poly64(d1);
        y = phase_poly64(d2);
        z = phase_poly64(d3);
      }
      double wl = 0.0, ml = 0.0, m2 = 0.0;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        C v = lb0[pad16(t) + 272 * m];
        if (EPI) {
          const double wv = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
          wl += wv;
          ml += wv * (double)(m - 8);
          if (EPI == EPI_V) m2 += wv * (double)((m - 8) * (m - 8));
        }
        if (EPI == EPI_V) {
          if constexpr (sizeof(T) == 4) {
            // complex64: the phase argument itself by forward differences (three FP64
            // adds per point; the 16-step drift is ~16 ulp of |phi|, far below the
            // FP32 rounding of the storage)
            v = mul_phase16<T>(v, ph);
            ph += d1;
            d1 += d2;
            d2 += d3;
          } else {
            v = cmul(v, w);
            if (m < 15) {
              w = cmul(w, u);
              u = cmul(u, y);
              y = cmul(y, z);
            }
          }
        } else if (INV) {
          v = tmul<T>(v, AG[t + 256 * m], true);
        }
        ntstore(tdst + 256 * m + t, v);
      }
      if (EPI) {
        acc[0] += wl;
        if (EPI == EPI_REDP) {
#pragma unroll
          for (int l = 0; l < MGK_MAXD; ++l)
            if (l < D) acc[1 + l] += (l == L) ? ml : wl * (double)(jfix[l] - 8);
        }
        if (EPI == EPI_V) {
          if constexpr (PK == 3) {
            hh_tile_acc(hht, L, D, wl, ml, m2, lc, tcs, acc);
          } else {
            double unused[4];
            line_model<PK>(L, jfix, wl, ml, m2, D, lc, acc, unused);
          }
        }
      }
      if (PP) {
        C* const sw = lb0;
        lb0 = lb1;
        lb1 = sw;
      } else {
        __syncthreads();
      }
    }
  }
  if (EPI) {
    if (PP) __syncthreads();  // the last tile's reads before the reduction reuses LDS
    // the inverse tables carry 1/sqrt(16) per axis: the sums above miss 16^-K
    // (except where the first-axis factors carry it)
    if (INV && !FOLD) {
      const double sc = ldexp(1.0, -4 * K);
#pragma unroll
      for (int k = 0; k < MGK_NACC; ++k) acc[k] *= sc;
    }
    block_reduce<NT>(acc, D + 2, a.partials + (size_t)blockIdx.x * MGK_NACC, (double*)lds_raw);
  }
}

}  // namespace mgk
