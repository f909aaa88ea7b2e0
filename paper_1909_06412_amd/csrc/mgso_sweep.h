// mgso_sweep.h -- tile processing shared by the grid-wide sweep kernels and the
// one-workgroup-per-packet persistent engine.
#pragma once
#include "mgso_kernels.h"

namespace mgk {

// Direction / table use of a sweep.
enum : int { DIR_FWD = 0, DIR_INV = 1 };

// Per-axis tables of a packet, table entries of the storage precision (make_te):
//   Atab[l][j] = (-1)^j exp(-i p_ctr,l j dq_l / hbar) / sqrt(N_l)   (forward pre, inverse post conj)
//   Mtab[l][k] = exp(-i [h p_l^2 / (2 m_l) - delta_l p_l] / hbar)  (inverse pre)
template <typename T> struct Tables {
  const typename TE<T>::type* tw;   // twiddles (shared, offsets per axis length)
  const typename TE<T>::type* A;
  const typename TE<T>::type* M;
};

// Load one tile of sweep `sw` into LDS (zero padding outside a ragged tile).
// Returns the base element offsets needed for the store.
struct TileOrigin {
  uint64_t base;       // element offset of the tile origin in the buffer
  uint32_t o;          // outer index (kind 1) or first outer row (kind 0)
  uint32_t i0;         // first inner index (kind 1)
  uint32_t lim;        // rows (kind 0) or run elements (kind 1) inside the array
};

__device__ __forceinline__ TileOrigin tile_origin(const PacketGeom& G, const SweepDesc& sw, uint32_t tile) {
  TileOrigin t;
  if (sw.kind == 0) {
    t.o = tile * sw.ob;
    t.i0 = 0;
    t.lim = min(sw.ob, sw.O - t.o);
    t.base = G.off + (uint64_t)t.o * sw.LG;
  } else {
    t.o = divw(tile, sw.dtiles_i);
    const uint32_t ib = tile - t.o * sw.tiles_i;
    t.i0 = ib * sw.r;
    t.lim = min(sw.r, sw.I - t.i0);
    t.base = G.off + ((uint64_t)t.o * sw.LG) * sw.I + t.i0;
  }
  return t;
}

// In-tile decode constants of a sweep, read once into registers before the
// element loops of a tile.
struct TileDec {
  int32_t kind;
  uint32_t LG, r, I;
  Div32 dLG, dr;
};
__device__ __forceinline__ TileDec tile_dec(const SweepDesc& sw) {
  return TileDec{sw.kind, sw.LG, sw.r, sw.I, sw.dLG, sw.dr};
}

// Element t of the tile -> (global offset, valid, group index g, outer o, inner i)
__device__ __forceinline__ bool tile_elem(const TileDec& sw, const TileOrigin& to, uint32_t t, uint64_t* gofs,
                                          uint32_t* g, uint32_t* o, uint32_t* i) {
  if (sw.kind == 0) {
    const uint32_t row = div32(t, sw.dLG);
    *g = t - row * sw.LG;
    *o = to.o + row;
    *i = 0;
    *gofs = to.base + t;
    return row < to.lim;
  } else {
    const uint32_t gg = div32(t, sw.dr);
    const uint32_t ii = t - gg * sw.r;
    *g = gg;
    *o = to.o;
    *i = to.i0 + ii;
    *gofs = to.base + (uint64_t)gg * sw.I + ii;
    return ii < to.lim;
  }
}

// Process one tile: load from src, transform the sweep's axes (forward with A pre-
// multiplication, or inverse with M pre- and conj(A) post-multiplication), run the
// pointwise epilogue and store to dst.  acc collects the epilogue's FP64 sums.
// PP: the transforms ping-pong between lds[0, TM) and lds[TM, 2 TM) (out-of-place
// Stockham passes); the tile is back in lds[0, TM) after the epilogue.
// LCH: loads issued per thread before the first is waited for (1: one at a time,
// for kernels whose registers are already full).
template <typename T, int NTHR, int TM = MGK_TMAX, bool PP = false, int DT = 0, bool WIDE = false, int LCH = 1>
__device__ __forceinline__ void process_tile(typename CT<T>::type* lds, const PacketGeom& G, int si, uint32_t tile,
                                             const typename CT<T>::type* src, typename CT<T>::type* dst,
                                             const Tables<T>& tb, int dir, int epi, double h,
                                             const PacketState& st, const PotDesc& P, double* acc,
                                             bool do_load, bool do_store, const double* mtab = nullptr) {
  typedef typename CT<T>::type C;
  const SweepDesc& sw = G.sw[si];
  const TileOrigin to = tile_origin(G, sw, tile);
  const uint32_t Tn = sw.T;
  const TileDec td = tile_dec(sw);
  if (do_load) {
    // loads in groups of CH per thread, all issued before the first is waited for
    // (a loop that stores each value to LDS as it arrives waits once per element)
    constexpr int CH = LCH;
    for (uint32_t t0 = threadIdx.x; t0 < Tn; t0 += CH * NTHR) {
      C v[CH];
#pragma unroll
      for (int m = 0; m < CH; ++m) {
        const uint32_t t = t0 + (uint32_t)(m * NTHR);
        v[m] = C{(T)0, (T)0};
        if (t < Tn) {
          uint64_t gofs;
          uint32_t g, o, i;
          if (tile_elem(td, to, t, &gofs, &g, &o, &i)) v[m] = gload(src, gofs);
        }
      }
#pragma unroll
      for (int m = 0; m < CH; ++m) {
        const uint32_t t = t0 + (uint32_t)(m * NTHR);
        if (t < Tn) lds[t] = v[m];
      }
    }
    __syncthreads();
  }
  const bool inv = dir == DIR_INV;
  int cur = 0;
  for (int ai = 0; ai < sw.b - sw.a; ++ai) {
    const AxisDesc& ax = G.ax[sw.a + ai];
    const typename TE<T>::type* tw = tb.tw + ax.tw_off;
    if constexpr (PP) {
      if (!inv)
        tile_axis_fft_pp<T, NTHR>(lds, lds + TM, &cur, Tn, ax, sw.S[ai], sw.dS[ai], false, tw, tb.A + ax.tab_off,
                                  nullptr, false);
      else
        tile_axis_fft_pp<T, NTHR>(lds, lds + TM, &cur, Tn, ax, sw.S[ai], sw.dS[ai], true, tw, tb.M + ax.tab_off,
                                  tb.A + ax.tab_off, true);
    } else if (!inv) {
      tile_axis_fft<T, NTHR, TM, WIDE>(lds, Tn, ax, sw.S[ai], sw.dS[ai], false, tw, tb.A + ax.tab_off, nullptr,
                                       false);
    } else {
      tile_axis_fft<T, NTHR, TM, WIDE>(lds, Tn, ax, sw.S[ai], sw.dS[ai], true, tw, tb.M + ax.tab_off,
                                       tb.A + ax.tab_off, true);
    }
  }
  // after an odd number of ping-pong passes the tile sits in the second buffer;
  // the epilogue reads it from there and writes each point back to lds[t]
  const C* res = (PP && cur) ? lds + TM : lds;
  const int D = DT > 0 ? DT : G.D, sa = sw.a, sb = sw.b;
  const AxDec ad = load_axdec(G, D);
  for (uint32_t t = threadIdx.x; t < Tn; t += NTHR) {
    uint64_t gofs;
    uint32_t g, o, i;
    const bool ok = tile_elem(td, to, t, &gofs, &g, &o, &i);
    if (!ok) continue;
    C x = res[t];
    if (epi) {
      int j[MGK_MAXD];
      decode_index(ad, D, sa, sb, o, g, i, j);
      x = epilogue_point<T, DT>(x, j, G, st, P, epi, h, acc, mtab);
    }
    if (do_store) gstore(dst, gofs, x);
    else lds[t] = x;
  }
  __syncthreads();
}

}  // namespace mgk

namespace mgk {

// ---------------------------------------------------------------------------
// Substep bookkeeping shared by the finalize kernel and the persistent batch
// engine (one thread for the scalar part, the whole workgroup for the tables).
// ---------------------------------------------------------------------------

// Kinetic substep (Sec. II.G.2, Eqs. (49), (52)): <p> from the momentum-grid
// sums tot = (sum w, sum w (k_l - N_l/2)), delta = h m^-1 <p>, q_ctr += delta.
// With st.fixed the grid stays where it is (delta = 0): the fixed-grid propagation
// that the naive scheme (Sec. II.F, Eqs. (29)-(34)) re-centres after each step.
__device__ __forceinline__ void fin_kinetic(const PacketGeom& G, PacketState& st, const double* tot, double h) {
  const double n = tot[0];
  bool bad = !(n > 0.0) || !isfinite(n);
  if (st.fixed) {
    for (int l = 0; l < G.D; ++l) st.delta[l] = 0.0;
    for (int k = 0; k < G.D + 2; ++k) st.last[k] = tot[k];
    if (bad) st.err = 1;
    return;
  }
  for (int l = 0; l < G.D; ++l) {
    const double pbar = st.p_c[l] + G.ax[l].dp * (tot[1 + l] / n);
    const double d = h * G.ax[l].minv * pbar;
    if (!isfinite(d) || fabs(d) > 0.5 * G.ax[l].n * G.ax[l].dq) bad = true;
    st.delta[l] = d;
    st.q_c[l] += d;
  }
  for (int k = 0; k < G.D + 2; ++k) st.last[k] = tot[k];
  if (bad) st.err = 1;
}

// Potential substep (Sec. II.G.1, Eq. (47)): p_ctr -= h <dV/dq> from
// tot = (sum w, sum w dV/dq_l).
__device__ __forceinline__ void fin_potential(const PacketGeom& G, PacketState& st, const double* tot, double h) {
  const double n = tot[0];
  bool bad = !(n > 0.0) || !isfinite(n);
  for (int l = 0; l < G.D; ++l) {
    const double gl = tot[1 + l] / n;
    if (!isfinite(gl)) bad = true;
    if (!st.fixed) st.p_c[l] -= h * gl;
  }
  for (int k = 0; k < G.D + 2; ++k) st.last[k] = tot[k];
  if (bad) st.err = 1;
}

// M_l(k) = exp(-i [h p^2 / (2 m_l) - delta_l p] / hbar), p = p_ctr + (k - N/2) dp
// (sgn = -1 builds conj(M), used by the adjoint of the kinetic substep)
template <typename T, int NT>
__device__ __forceinline__ void build_M_tables(const PacketGeom& G, const PacketState& st, double h,
                                               typename TE<T>::type* M, double sgn = 1.0) {
  for (int l = 0; l < G.D; ++l) {
    const AxisDesc& ax = G.ax[l];
    for (int k = threadIdx.x; k < ax.n; k += NT) {
      const double p = st.p_c[l] + (double)(k - ax.n / 2) * ax.dp;
      const double phi = sgn * (h * 0.5 * ax.minv * p * p - st.delta[l] * p) / G.hbar;
      double s, c;
      sincos(phi, &s, &c);
      M[ax.tab_off + k] = make_te<T>(c, -s);
    }
  }
}

// A_l(j) = (-1)^j exp(-i p_ctr,l j dq_l / hbar) / sqrt(N_l)
template <typename T, int NT>
__device__ __forceinline__ void build_A_tables(const PacketGeom& G, const PacketState& st, typename TE<T>::type* A) {
  for (int l = 0; l < G.D; ++l) {
    const AxisDesc& ax = G.ax[l];
    const double inv_sqrt = 1.0 / sqrt((double)ax.n);
    for (int j = threadIdx.x; j < ax.n; j += NT) {
      const double phi = st.p_c[l] * (double)j * ax.dq / G.hbar;
      double s, c;
      sincos(phi, &s, &c);
      const double sg = (j & 1) ? -inv_sqrt : inv_sqrt;
      A[ax.tab_off + j] = make_te<T>(sg * c, -sg * s);
    }
  }
}

}  // namespace mgk
