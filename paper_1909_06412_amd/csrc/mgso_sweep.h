// mgso_sweep.h -- tile processing shared by the grid-wide sweep kernels and the
// one-workgroup-per-packet persistent engine.
#pragma once
#include "mgso_kernels.h"

namespace mgk {

// Direction / table use of a sweep.
enum : int { DIR_FWD = 0, DIR_INV = 1 };

// Per-axis tables of a packet in the storage precision:
//   Atab[l][j] = (-1)^j exp(-i p_ctr,l j dq_l / hbar) / sqrt(N_l)   (forward pre, inverse post conj)
//   Mtab[l][k] = exp(-i [h p_l^2 / (2 m_l) - delta_l p_l] / hbar)  (inverse pre)
template <typename T> struct Tables {
  const typename CT<T>::type* tw;   // twiddles (shared, offsets per axis length)
  const typename CT<T>::type* A;
  const typename CT<T>::type* M;
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

// Element t of the tile -> (global offset, valid, group index g, outer o, inner i)
__device__ __forceinline__ bool tile_elem(const SweepDesc& sw, const TileOrigin& to, uint32_t t, uint64_t* gofs,
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
template <typename T, int NTHR>
__device__ __forceinline__ void process_tile(typename CT<T>::type* lds, const PacketGeom& G, int si, uint32_t tile,
                                             const typename CT<T>::type* src, typename CT<T>::type* dst,
                                             const Tables<T>& tb, int dir, int epi, double h,
                                             const PacketState& st, const PotDesc& P, double* acc,
                                             bool do_load, bool do_store) {
  typedef typename CT<T>::type C;
  const SweepDesc& sw = G.sw[si];
  const TileOrigin to = tile_origin(G, sw, tile);
  const uint32_t Tn = sw.T;
  if (do_load) {
    for (uint32_t t = threadIdx.x; t < Tn; t += NTHR) {
      uint64_t gofs;
      uint32_t g, o, i;
      const bool ok = tile_elem(sw, to, t, &gofs, &g, &o, &i);
      lds[t] = ok ? src[gofs] : C{(T)0, (T)0};
    }
    __syncthreads();
  }
  const bool inv = dir == DIR_INV;
  for (int ai = 0; ai < sw.b - sw.a; ++ai) {
    const AxisDesc& ax = G.ax[sw.a + ai];
    const C* tw = tb.tw + ax.tw_off;
    if (!inv) {
      tile_axis_fft<T, NTHR>(lds, Tn, ax, sw.S[ai], sw.dS[ai], false, tw, tb.A + ax.tab_off, nullptr, false);
    } else {
      tile_axis_fft<T, NTHR>(lds, Tn, ax, sw.S[ai], sw.dS[ai], true, tw, tb.M + ax.tab_off,
                             tb.A + ax.tab_off, true);
    }
  }
  for (uint32_t t = threadIdx.x; t < Tn; t += NTHR) {
    uint64_t gofs;
    uint32_t g, o, i;
    const bool ok = tile_elem(sw, to, t, &gofs, &g, &o, &i);
    if (!ok) continue;
    C x = lds[t];
    if (epi) {
      int j[MGK_MAXD];
      decode_index(G, sw.a, sw.b, o, g, i, j);
      x = epilogue_point<T>(x, j, G, st, P, epi, h, acc);
    }
    if (do_store) dst[gofs] = x;
    else lds[t] = x;
  }
  __syncthreads();
}

}  // namespace mgk
