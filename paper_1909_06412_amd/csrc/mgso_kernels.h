// mgso_kernels.h -- gfx950 device code of the moving-grid split-operator step.
//
// Method: Choi & Vanicek, arXiv:1909.06412 (equation numbers count the paper's
// displayed equations in order of appearance).  One TVT stage is, per packet,
//
//   kinetic substep U_T,adpt(h)  (Sec. II.G.2, Eq. (55) with Eqs. (49), (52)):
//     X = DFT[A c] / sqrt(N),  A_J = prod_l (-1)^{j_l} exp(-i p_ctr,l j_l dq_l / hbar)
//     <p> = p_ctr + dp * sum |X|^2 (k - N/2) / sum |X|^2,   delta = h m^-1 <p>
//     c  <- conj(A) IDFT[M X] / sqrt(N),  M_K = exp(-i [h T(p^K) - delta . p^K] / hbar)
//     q_ctr += delta
//   (the centre-dependent post-phase and constant of the paper's f(q,p) in Eq. (19)
//   cancel between f~(q_h, p) and f(q, p) except for the delta . p^K term kept in M)
//
//   potential substep U_V,adpt(h)  (Sec. II.G.1, Eqs. (45)-(47)):
//     p_ctr -= h sum |c|^2 dV/dq(q^J) / sum |c|^2,   c <- c exp(-i h V(q^J) / hbar)
//
// A, M are separable, so each axis' factor is applied inside the sweep that
// transforms that axis, from per-axis tables built in FP64 and rounded once.
// Reductions are FP64, per thread -> wave -> workgroup -> fixed-order finalize.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "mgso_common.h"

namespace mgk {

template <typename T> struct CT;
template <> struct CT<float> { typedef float2 type; };
template <> struct CT<double> { typedef double2 type; };

// Loads and stores of the wavepacket state through global-address-space pointers.
// The state always lives in device memory; saying so lets the compiler keep the
// LDS-staged plan, state and potential in registers across loops that store the
// state (a generic store might alias LDS, so every descriptor field would be
// re-read, one LDS round trip each, per element), and emit global rather than flat
// memory instructions.
// (The host pass only parses these; address spaces exist in the device pass.)
template <typename C> __device__ __forceinline__ C gload(const C* p, uint64_t i) {
#ifdef __HIP_DEVICE_COMPILE__
  typedef __attribute__((address_space(1))) const C GC;
  C r;
  __builtin_memcpy(&r, (const void*)((const GC*)p + i), sizeof(C));
  return r;
#else
  return p[i];
#endif
}
template <typename C> __device__ __forceinline__ void gstore(C* p, uint64_t i, C v) {
#ifdef __HIP_DEVICE_COMPILE__
  typedef __attribute__((address_space(1))) C GC;
  ((GC*)p)[i] = v;
#else
  p[i] = v;
#endif
}

// Streaming loads and stores of the state in the contiguous-tile sweeps: every point
// is read once and written once per pass, so they carry the nontemporal hint
// (measured on 16^8: those sweeps 3-5% faster; the split passes' 128-byte runs were
// slower with it and keep plain accesses).
template <typename C> struct NTVec;
template <> struct NTVec<float2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct NTVec<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename C> __device__ __forceinline__ C ntload(const C* p) {
  typedef typename NTVec<C>::type V;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return C{v.x, v.y};
}
template <typename C> __device__ __forceinline__ void ntstore(C* p, C c) {
  typedef typename NTVec<C>::type V;
  V v;
  v.x = c.x;
  v.y = c.y;
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// a * (-i) when fwd, a * (+i) when inverse
template <typename C> __device__ __forceinline__ C rot(C a, bool inv) {
  return inv ? C{-a.y, a.x} : C{a.y, -a.x};
}

// Multiplication by a real constant k of the DFTs.  complex64: k is carried as
// hi + lo (hi = k rounded to FP32, lo = the FP32 rounding of what is left), so the
// product is k x rounded once.  With k alone rounded to FP32, every root of unity
// (c, s) built from rounded constants has c^2 + s^2 != 1 by a few 1e-8, always with
// the same sign: a 16-point DFT then loses 2.3e-8 of the norm on average, every
// transform of every step, which adds up to a steady norm decay (norm preservation,
// Sec. II.G, is the property the moving grid must keep).  complex128: plain product.
template <typename T> __device__ __forceinline__ T kmul(T x, double k);
template <> __device__ __forceinline__ float kmul<float>(float x, double k) {
  const float hi = (float)k, lo = (float)(k - (double)hi);
  return __builtin_fmaf(x, hi, x * lo);
}
template <> __device__ __forceinline__ double kmul<double>(double x, double k) { return x * k; }

// v * (c + i s) with c, s given in FP64; complex64 as hi + lo pairs (see kmul).
template <typename T, typename C> __device__ __forceinline__ C crotk(C v, double c, double s) {
  if constexpr (sizeof(T) == 4) {
    const float ch = (float)c, cl = (float)(c - (double)ch);
    const float sh = (float)s, sl = (float)(s - (double)sh);
    const float tr = __builtin_fmaf(-v.y, sl, v.x * cl);
    const float ti = __builtin_fmaf(v.y, cl, v.x * sl);
    return C{__builtin_fmaf(v.x, ch, __builtin_fmaf(-v.y, sh, tr)),
             __builtin_fmaf(v.y, ch, __builtin_fmaf(v.x, sh, ti))};
  } else {
    return C{v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// Twiddle of a table: v * w (or v * conj(w) when conj) with w = hi, plus its
// complex64 remainder lo (the table stores both, see the twiddle tables' layout).
template <typename T, typename C> __device__ __forceinline__ C cmul_tw(C v, C w, C wl, bool conj) {
  if constexpr (sizeof(T) == 4) {
    const float wy = conj ? -w.y : w.y, ly = conj ? -wl.y : wl.y;
    const float tr = __builtin_fmaf(-v.y, ly, v.x * wl.x);
    const float ti = __builtin_fmaf(v.y, wl.x, v.x * ly);
    return C{__builtin_fmaf(v.x, w.x, __builtin_fmaf(-v.y, wy, tr)),
             __builtin_fmaf(v.y, w.x, __builtin_fmaf(v.x, wy, ti))};
  } else {
    return conj ? cmulc(v, w) : cmul(v, w);
  }
}

// Table entries (twiddles, the per-axis and group phase tables): a root of unity
// or phase factor computed in FP64 and rounded to the storage precision.  complex64
// entries are float4 {hi.x, hi.y, lo.x, lo.y}: the rounded value and the rounded
// remainder, multiplied in with cmul_tw.  A complex64 table entry rounded once has
// |w|^2 - 1 of about 3e-8, fixed for as long as the table stays; a packet only a few
// grid points wide weights a handful of entries per axis, so these errors do not
// average out, and every substep would scale the norm by a random 1e-7 or so.
// complex128 entries are the plain double2 value.
template <typename T> struct TE;
template <> struct TE<float> { typedef float4 type; };
template <> struct TE<double> { typedef double2 type; };

template <typename T> __host__ __device__ __forceinline__ typename TE<T>::type make_te(double c, double s);
template <> __host__ __device__ __forceinline__ float4 make_te<float>(double c, double s) {
  const float ch = (float)c, sh = (float)s;
  return float4{ch, sh, (float)(c - (double)ch), (float)(s - (double)sh)};
}
template <> __host__ __device__ __forceinline__ double2 make_te<double>(double c, double s) {
  return double2{c, s};
}
// The FP64 value of an entry (hi + lo).
__device__ __forceinline__ double2 te_value(float4 e) {
  return double2{(double)e.x + (double)e.z, (double)e.y + (double)e.w};
}
__device__ __forceinline__ double2 te_value(double2 e) { return e; }

// v * e (or v * conj(e))
template <typename T, typename C> __device__ __forceinline__ C tmul(C v, typename TE<T>::type e, bool conj = false) {
  if constexpr (sizeof(T) == 4) {
    return cmul_tw<T>(v, C{e.x, e.y}, C{e.z, e.w}, conj);
  } else {
    return conj ? cmulc(v, e) : cmul(v, e);
  }
}
// The entry a * b (or a * conj(b)), formed in FP64 and rounded once.
template <typename T> __device__ __forceinline__ typename TE<T>::type te_prod(typename TE<T>::type a,
                                                                            typename TE<T>::type b, bool conjb) {
  const double2 x = te_value(a), y = te_value(b);
  const double yi = conjb ? -y.y : y.y;
  return make_te<T>(x.x * y.x - x.y * yi, x.x * yi + x.y * y.x);
}

// ---------------------------------------------------------------------------
// Small DFTs in registers: forward sign exp(-2 pi i nk/R), inverse exp(+...)
// ---------------------------------------------------------------------------
template <typename C> __device__ __forceinline__ void dft2(C* v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename C> __device__ __forceinline__ void dft4(C* v, bool inv) {
  C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  C t2 = cadd(v[1], v[3]), t3 = rot(csub(v[1], v[3]), inv);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T, typename C> __device__ __forceinline__ void dft8(C* v, bool inv) {
  const double h = 0.70710678118654752440084436210485;
  C b[4], c[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    b[n] = cadd(v[n], v[n + 4]);
    c[n] = csub(v[n], v[n + 4]);
  }
  // c_n *= w8^n, w8 = exp(-+ i pi / 4)
  {
    C x = c[1];
    const T d = x.x - x.y, e = x.x + x.y;
    c[1] = inv ? C{kmul<T>(d, h), kmul<T>(e, h)} : C{kmul<T>(e, h), kmul<T>(-d, h)};
    c[2] = rot(c[2], inv);
    x = c[3];
    const T f = x.x + x.y, g = x.x - x.y;
    c[3] = inv ? C{kmul<T>(-f, h), kmul<T>(g, h)} : C{kmul<T>(-g, h), kmul<T>(-f, h)};
  }
  dft4(b, inv);
  dft4(c, inv);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    v[2 * m] = b[m];
    v[2 * m + 1] = c[m];
  }
}

template <typename T, typename C> __device__ __forceinline__ void dft3(C* v, bool inv) {
  const double s = 0.86602540378443864676372317075294;  // sin(2 pi / 3)
  C t = cadd(v[1], v[2]);
  C u = csub(v[1], v[2]);
  C y0 = cadd(v[0], t);
  C m = C{v[0].x - (T)0.5 * t.x, v[0].y - (T)0.5 * t.y};
  C su = rot(C{kmul<T>(u.x, s), kmul<T>(u.y, s)}, inv);  // -+ i s u
  v[0] = y0;
  v[1] = cadd(m, su);
  v[2] = csub(m, su);
}

template <typename T, typename C> __device__ __forceinline__ void dft5(C* v, bool inv) {
  const double c1 = 0.30901699437494742410229341718282;   // cos(2 pi / 5)
  const double c2 = -0.80901699437494742410229341718282;  // cos(4 pi / 5)
  const double s1 = 0.95105651629515357211643933337938;   // sin(2 pi / 5)
  const double s2 = 0.58778525229247312916870595463907;   // sin(4 pi / 5)
  C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  C u1 = csub(v[1], v[4]), u2 = csub(v[2], v[3]);
  C y0 = C{v[0].x + t1.x + t2.x, v[0].y + t1.y + t2.y};
  C m1 = C{v[0].x + kmul<T>(t1.x, c1) + kmul<T>(t2.x, c2), v[0].y + kmul<T>(t1.y, c1) + kmul<T>(t2.y, c2)};
  C m2 = C{v[0].x + kmul<T>(t1.x, c2) + kmul<T>(t2.x, c1), v[0].y + kmul<T>(t1.y, c2) + kmul<T>(t2.y, c1)};
  C n1 = rot(C{kmul<T>(u1.x, s1) + kmul<T>(u2.x, s2), kmul<T>(u1.y, s1) + kmul<T>(u2.y, s2)}, inv);
  C n2 = rot(C{kmul<T>(u1.x, s2) - kmul<T>(u2.x, s1), kmul<T>(u1.y, s2) - kmul<T>(u2.y, s1)}, inv);
  v[0] = y0;
  v[1] = cadd(m1, n1);
  v[4] = csub(m1, n1);
  v[2] = cadd(m2, n2);
  v[3] = csub(m2, n2);
}

// Roots of unity of the composite radices (exact where the angle is a multiple of
// pi/2, pi/4 or pi/6; otherwise the double nearest the reduced-angle value).
template <int R> struct Unity;
template <> struct Unity<9> {
  static constexpr double c[9] = {1.0, 0.766044443118978, 0.17364817766693033, -0.5, -0.9396926207859084, -0.9396926207859084, -0.5, 0.17364817766693033, 0.766044443118978};
  static constexpr double s[9] = {0.0, 0.6427876096865393, 0.984807753012208, 0.8660254037844386, 0.3420201433256687, -0.3420201433256687, -0.8660254037844386, -0.984807753012208, -0.6427876096865393};
};
template <> struct Unity<10> {
  static constexpr double c[10] = {1.0, 0.8090169943749475, 0.3090169943749474, -0.3090169943749474, -0.8090169943749475, -1.0, -0.8090169943749475, -0.3090169943749474, 0.3090169943749474, 0.8090169943749475};
  static constexpr double s[10] = {0.0, 0.5877852522924731, 0.9510565162951535, 0.9510565162951535, 0.5877852522924731, 0.0, -0.5877852522924731, -0.9510565162951535, -0.9510565162951535, -0.5877852522924731};
};
template <> struct Unity<12> {
  static constexpr double c[12] = {1.0, 0.8660254037844386, 0.5, 0.0, -0.5, -0.8660254037844386, -1.0, -0.8660254037844386, -0.5, 0.0, 0.5, 0.8660254037844386};
  static constexpr double s[12] = {0.0, 0.5, 0.8660254037844386, 1.0, 0.8660254037844386, 0.5, 0.0, -0.5, -0.8660254037844386, -1.0, -0.8660254037844386, -0.5};
};
template <> struct Unity<15> {
  static constexpr double c[15] = {1.0, 0.9135454576426009, 0.6691306063588582, 0.3090169943749474, -0.10452846326765346, -0.5, -0.8090169943749475, -0.9781476007338057, -0.9781476007338057, -0.8090169943749475, -0.5, -0.10452846326765346, 0.3090169943749474, 0.6691306063588582, 0.9135454576426009};
  static constexpr double s[15] = {0.0, 0.40673664307580015, 0.7431448254773942, 0.9510565162951535, 0.9945218953682733, 0.8660254037844386, 0.5877852522924731, 0.20791169081775931, -0.20791169081775931, -0.5877852522924731, -0.8660254037844386, -0.9945218953682733, -0.9510565162951535, -0.7431448254773942, -0.40673664307580015};
};
template <> struct Unity<16> {
  static constexpr double c[16] = {1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898, 0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867};
  static constexpr double s[16] = {0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867, 1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898};
};

template <typename T, int R, typename C> __device__ __forceinline__ void dftR(C* v, bool inv);

// Composite radix R = A B in registers (Cooley-Tukey inside the butterfly):
// input n = B a + b, output k = k1 + A k2; A-point DFTs over a for each b,
// multiplication by w_R^(b k1), then B-point DFTs over b for each k1.
template <typename T, int A, int B, typename C> __device__ __forceinline__ void dft_ab(C* v, bool inv) {
  constexpr int R = A * B;
  C t[R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    C u[A];
#pragma unroll
    for (int a = 0; a < A; ++a) u[a] = v[B * a + b];
    dftR<T, A>(u, inv);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      C x = u[k1];
      const int m = (b * k1) % R;
      if (m != 0) {
        // forward w = c - i sn, inverse w = c + i sn
        x = crotk<T>(x, Unity<R>::c[m], inv ? Unity<R>::s[m] : -Unity<R>::s[m]);
      }
      t[b * A + k1] = x;
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    C u[B];
#pragma unroll
    for (int b = 0; b < B; ++b) u[b] = t[b * A + k1];
    dftR<T, B>(u, inv);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = u[k2];
  }
}

template <typename T, int R, typename C> __device__ __forceinline__ void dftR(C* v, bool inv) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 3) dft3<T>(v, inv);
  else if constexpr (R == 4) dft4(v, inv);
  else if constexpr (R == 5) dft5<T>(v, inv);
  else if constexpr (R == 8) dft8<T>(v, inv);
  else if constexpr (R == 9) dft_ab<T, 3, 3>(v, inv);
  else if constexpr (R == 10) dft_ab<T, 2, 5>(v, inv);
  else if constexpr (R == 12) dft_ab<T, 4, 3>(v, inv);
  else if constexpr (R == 15) dft_ab<T, 3, 5>(v, inv);
  else if constexpr (R == 16) dft_ab<T, 4, 4>(v, inv);
}

// ---------------------------------------------------------------------------
// One Stockham pass of radix R over every line of one axis of the LDS tile.
// Reads all of a thread's butterflies into registers, barrier, writes them back.
// pre (first pass) multiplies inputs by a per-axis table at the natural index;
// post (last pass) multiplies outputs by a per-axis table (or its conjugate).
// ---------------------------------------------------------------------------
template <typename T, int R, int NTHR, int TM = MGK_TMAX>
__device__ __forceinline__ void stockham_pass(typename CT<T>::type* lds, uint32_t Tn, uint32_t n,
                                              uint32_t S, Div32 dS, const PassDesc& pd, bool inv,
                                              const typename TE<T>::type* __restrict__ tw,
                                              const typename TE<T>::type* __restrict__ pre,
                                              const typename TE<T>::type* __restrict__ post,
                                              bool post_conj) {
  typedef typename CT<T>::type C;
  constexpr int MB = (TM + R * NTHR - 1) / (R * NTHR);
  const uint32_t nbl = n / R;
  const uint32_t nb = Tn / R;
  const uint32_t Ns = pd.Ns;
  C v[MB][R];
  uint32_t base[MB], jj[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const uint32_t bf = threadIdx.x + m * NTHR;
    if (bf < nb) {
      uint32_t b0, j;
      bfly_index(bf, n, S, dS, pd.dNbl, &b0, &j);
      base[m] = b0;
      jj[m] = j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[m][r] = lds[b0 + (j + r * nbl) * S];
      if (pre) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[m][r] = tmul<T>(v[m][r], pre[j + r * nbl]);
      }
      if (Ns > 1) {
        const uint32_t k = j - div32(j, pd.dNs) * Ns;
        const uint32_t step = k * pd.tws;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[m][r] = tmul<T>(v[m][r], tw[r * step], inv);
        }
      }
      dftR<T, R>(v[m], inv);
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const uint32_t bf = threadIdx.x + m * NTHR;
    if (bf < nb) {
      const uint32_t j = jj[m];
      const uint32_t k = j - div32(j, pd.dNs) * Ns;
      const uint32_t o0 = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t p = o0 + r * Ns;
        C x = v[m][r];
        if (post) x = tmul<T>(x, post[p], post_conj);
        lds[base[m] + p * S] = x;
      }
    }
  }
  __syncthreads();
}

// The same pass out of place (Stockham ping-pong between two LDS buffers): each
// butterfly reads from `in` and writes to `out` at once, so a thread holds only
// its R values and a pass needs one barrier, at the price of a second tile of LDS.
template <typename T, int R, int NTHR>
__device__ __forceinline__ void stockham_pass_pp(const typename CT<T>::type* __restrict__ in,
                                                 typename CT<T>::type* __restrict__ out, uint32_t Tn, uint32_t n,
                                                 uint32_t S, Div32 dS, const PassDesc& pd, bool inv,
                                                 const typename TE<T>::type* __restrict__ tw,
                                                 const typename TE<T>::type* __restrict__ pre,
                                                 const typename TE<T>::type* __restrict__ post, bool post_conj) {
  typedef typename CT<T>::type C;
  const uint32_t nbl = n / R;
  const uint32_t nb = Tn / R;
  const uint32_t Ns = pd.Ns;
  for (uint32_t bf = threadIdx.x; bf < nb; bf += NTHR) {
    uint32_t b0, j;
    bfly_index(bf, n, S, dS, pd.dNbl, &b0, &j);
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[b0 + (j + r * nbl) * S];
    if (pre) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = tmul<T>(v[r], pre[j + r * nbl]);
    }
    const uint32_t k = j - div32(j, pd.dNs) * Ns;
    if (Ns > 1) {
      const uint32_t step = k * pd.tws;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        v[r] = tmul<T>(v[r], tw[r * step], inv);
      }
    }
    dftR<T, R>(v, inv);
    const uint32_t o0 = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t p = o0 + r * Ns;
      C x = v[r];
      if (post) x = tmul<T>(x, post[p], post_conj);
      out[b0 + p * S] = x;
    }
  }
  __syncthreads();
}

// All passes of axis `ax` with the ping-pong pass; *cur selects the buffer that
// holds the data (0: a, 1: b) on entry and on return.  Besides 2, 3, 4, 5 and 8
// this pass takes the composite radices 9, 10, 12, 15 and 16 (plans made with
// wide radices), so most 5-smooth lengths up to 256 need two passes.
template <typename T, int NTHR>
__device__ __forceinline__ void tile_axis_fft_pp(typename CT<T>::type* a, typename CT<T>::type* b, int* cur,
                                                 uint32_t Tn, const AxisDesc& ax, uint32_t S, Div32 dS, bool inv,
                                                 const typename TE<T>::type* tw, const typename TE<T>::type* pre,
                                                 const typename TE<T>::type* post, bool post_conj) {
  const int np = ax.npass;
  for (int p = 0; p < np; ++p) {
    const PassDesc& pd = ax.pass[p];
    const typename TE<T>::type* pr = p == 0 ? pre : nullptr;
    const typename TE<T>::type* po = p == np - 1 ? post : nullptr;
    typename CT<T>::type* src = *cur ? b : a;
    typename CT<T>::type* dst = *cur ? a : b;
    switch (pd.R) {
      case 2: stockham_pass_pp<T, 2, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 3: stockham_pass_pp<T, 3, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 4: stockham_pass_pp<T, 4, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 5: stockham_pass_pp<T, 5, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 9: stockham_pass_pp<T, 9, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 10: stockham_pass_pp<T, 10, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 12: stockham_pass_pp<T, 12, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 15: stockham_pass_pp<T, 15, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 16: stockham_pass_pp<T, 16, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      default: stockham_pass_pp<T, 8, NTHR>(src, dst, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
    }
    *cur ^= 1;
  }
}

// FFT of every line of axis `ax` in the tile (all passes of that axis).  WIDE
// adds the composite radices 9, 10, 12, 15 and 16 (plans made with wide radices).
template <typename T, int NTHR, int TM = MGK_TMAX, bool WIDE = false>
__device__ __forceinline__ void tile_axis_fft(typename CT<T>::type* lds, uint32_t Tn,
                                              const AxisDesc& ax, uint32_t S, Div32 dS, bool inv,
                                              const typename TE<T>::type* tw,
                                              const typename TE<T>::type* pre,
                                              const typename TE<T>::type* post, bool post_conj) {
  const int np = ax.npass;
  for (int p = 0; p < np; ++p) {
    const PassDesc& pd = ax.pass[p];
    const typename TE<T>::type* pr = p == 0 ? pre : nullptr;
    const typename TE<T>::type* po = p == np - 1 ? post : nullptr;
    switch (pd.R) {
      case 2: stockham_pass<T, 2, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 3: stockham_pass<T, 3, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 4: stockham_pass<T, 4, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 5: stockham_pass<T, 5, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
      case 9:
        if constexpr (WIDE) stockham_pass<T, 9, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj);
        break;
      case 10:
        if constexpr (WIDE) stockham_pass<T, 10, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj);
        break;
      case 12:
        if constexpr (WIDE) stockham_pass<T, 12, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj);
        break;
      case 15:
        if constexpr (WIDE) stockham_pass<T, 15, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj);
        break;
      case 16:
        if constexpr (WIDE) stockham_pass<T, 16, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj);
        break;
      default: stockham_pass<T, 8, NTHR, TM>(lds, Tn, ax.n, S, dS, pd, inv, tw, pr, po, post_conj); break;
    }
  }
}

// ---------------------------------------------------------------------------
// Potentials (FP64): value and gradient at one grid point.
// ---------------------------------------------------------------------------
// PK >= 0 fixes the kind at compile time (specialised kernels); PK < 0 dispatches
// on P.kind at run time.
template <int PK = -1>
__device__ __forceinline__ double pot_eval(const PotDesc& P, int D, const double* q, double* g) {
  double V = 0.0;
  switch (PK >= 0 ? PK : P.kind) {
    case 1: {  // harmonic: k[D], s[D]
#pragma unroll
      for (int l = 0; l < MGK_MAXD; ++l) {
        if (l >= D) break;
        const double x = q[l] - P.p[D + l];
        V += 0.5 * P.p[l] * x * x;
        if (g) g[l] = P.p[l] * x;
      }
      break;
    }
    case 2: {  // Morse + repulsion: De, a, re, A, b, c
      const double e = exp(-P.p[1] * (q[0] - P.p[2]));
      V = P.p[0] * (1.0 - e) * (1.0 - e);
      double g0 = 2.0 * P.p[0] * P.p[1] * e * (1.0 - e);
      if (D > 1) {
        const double rep = P.p[3] * exp(-P.p[4] * (q[1] - P.p[5] * q[0]));
        V += rep;
        g0 += P.p[4] * P.p[5] * rep;
        if (g) g[1] = -P.p[4] * rep;
      }
      if (g) g[0] = g0;
      break;
    }
    case 3: {  // Henon-Heiles: kappa, lam
      const double ka = P.p[0], la = P.p[1];
#pragma unroll
      for (int l = 0; l < MGK_MAXD; ++l) {
        if (l >= D) break;
        V += 0.5 * ka * q[l] * q[l];
        if (g) g[l] = ka * q[l];
      }
#pragma unroll
      for (int l = 0; l + 1 < MGK_MAXD; ++l) {
        if (l + 1 >= D) break;
        const double a = q[l], b = q[l + 1];
        V += la * (a * a * b - b * b * b / 3.0);
        if (g) {
          g[l] += 2.0 * la * a * b;
          g[l + 1] += la * (a * a - b * b);
        }
      }
      break;
    }
    case 4: {  // quadratic: K[D*D], s[D]  (D <= 4)
      double x[4];
#pragma unroll
      for (int l = 0; l < 4; ++l) x[l] = l < D ? q[l] - P.p[D * D + l] : 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a >= D) break;
        double row = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (b < D) row += P.p[a * D + b] * x[b];
        V += 0.5 * x[a] * row;
        if (g) g[a] = row;
      }
      break;
    }
    default:
      if (g) {
#pragma unroll
        for (int l = 0; l < MGK_MAXD; ++l)
          if (l < D) g[l] = 0.0;
      }
      break;
  }
  return V;
}

// Hessian-vector product out = (d^2 V / dq dq) v at one point (FP64).
__device__ __forceinline__ void pot_hess_vec(const PotDesc& P, int D, const double* q, const double* v,
                                             double* out) {
  for (int l = 0; l < D; ++l) out[l] = 0.0;
  switch (P.kind) {
    case 1:
      for (int l = 0; l < D; ++l) out[l] = P.p[l] * v[l];
      break;
    case 2: {
      const double De = P.p[0], a = P.p[1], re = P.p[2], A = P.p[3], b = P.p[4], c = P.p[5];
      const double e = exp(-a * (q[0] - re));
      double h00 = 2.0 * De * a * a * e * (2.0 * e - 1.0);
      if (D > 1) {
        const double rep = A * exp(-b * (q[1] - c * q[0]));
        h00 += b * b * c * c * rep;
        const double h01 = -b * b * c * rep, h11 = b * b * rep;
        out[0] = h00 * v[0] + h01 * v[1];
        out[1] = h01 * v[0] + h11 * v[1];
      } else {
        out[0] = h00 * v[0];
      }
      break;
    }
    case 3: {
      const double ka = P.p[0], la = P.p[1];
      for (int l = 0; l < D; ++l) out[l] = ka * v[l];
      for (int l = 0; l + 1 < D; ++l) {
        const double x = q[l], y = q[l + 1];
        // V_l = la (x^2 y - y^3/3): d2/dx2 = 2 la y, d2/dxdy = 2 la x, d2/dy2 = -2 la y
        out[l] += 2.0 * la * y * v[l] + 2.0 * la * x * v[l + 1];
        out[l + 1] += 2.0 * la * x * v[l] - 2.0 * la * y * v[l + 1];
      }
      break;
    }
    case 4:
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) out[a] += P.p[a * D + b] * v[b];
      break;
    default:
      break;
  }
}

// Derivatives with respect to potential parameter `id` (index into the
// mg_set_potential list): returns dV/dtheta and fills dg = d(dV/dq)/dtheta.
// Supported: harmonic k_l (ids 0..D-1); Morse+repulsion A (3) and b (4).
__device__ __forceinline__ double pot_dtheta(const PotDesc& P, int D, const double* q, int id, double* dg) {
  for (int l = 0; l < D; ++l) dg[l] = 0.0;
  if (P.kind == 1 && id >= 0 && id < D) {
    const double x = q[id] - P.p[D + id];
    dg[id] = x;
    return 0.5 * x * x;
  }
  if (P.kind == 2 && D == 2 && (id == 3 || id == 4)) {
    const double A = P.p[3], b = P.p[4], c = P.p[5];
    const double R = q[1] - c * q[0];
    const double E = exp(-b * R);
    if (id == 3) {  // V_rep = A E, grad = (b c A E, -b A E)
      dg[0] = b * c * E;
      dg[1] = -b * E;
      return E;
    }
    // d/db: V -> -R A E; grad -> (c A E (1 - b R), -A E (1 - b R))
    dg[0] = c * A * E * (1.0 - b * R);
    dg[1] = -A * E * (1.0 - b * R);
    return -R * A * E;
  }
  return 0.0;
}

// x exp(-i phi) for the complex64 path without branches: quadrant reduction in FP64
// (n = rint(2 phi / pi), r = phi - n pi/2 with pi/2 split in two parts so that the
// reduction error stays near 1e-16 for |phi| < 1e6), sin r and cm = cos r - 1 by
// their Taylor series (sin to r^9, cos to r^10) in FP32 with explicit FMAs, then
// x + x cm - i x sin r with the 1 kept exact, then the quarter turns (-i)^n as exact
// swaps and sign flips.  Keeping cos r as 1 + cm makes the
// factor unitary to ~r^2 1e-7: cos r rounded to FP32 near 1 would instead leave
// |exp(-i r)|^2 - 1 = r^2 exactly for every |r| < 2.4e-4 (cos r rounds to 1), a
// steady norm gain wherever the potential phase is small.  On |r| <= pi/4 the
// truncation is below 2e-9 (sin) and 1.2e-10 (cos), the FP32 evaluation error about
// 5e-8; the x^4 coefficient of cos is 1/24 rounded up (one FP32 step above the
// nearest value), which makes the mean of |factor|^2 - 1 over the reduced range
// +8e-11 instead of -3.7e-10.
__device__ __forceinline__ float2 mul_phase_f32(float2 v, double phi) {
  const double two_over_pi = 0.63661977236758134307553505349006;
  // pi/2 split so that n * pio2_hi is exact (32-bit mantissa) (Cody-Waite)
  const double pio2_hi = 1.5707963267341256;
  const double pio2_lo = 6.077100506506192e-11;
  const double n = rint(phi * two_over_pi);
  const float r = (float)((phi - n * pio2_hi) - n * pio2_lo);
  const float r2 = r * r;
  // sin r = r + r^3 (-1/6 + r^2 (1/120 + r^2 (-1/5040 + r^2 / 362880)))
  float ps = __builtin_fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = __builtin_fmaf(ps, r2, 1.0f / 120.0f);
  ps = __builtin_fmaf(ps, r2, -1.0f / 6.0f);
  const float sn = __builtin_fmaf(r, r2 * ps, r);
  // cos r - 1 = r^2 (-1/2 + r^2 (1/24 + r^2 (-1/720 + r^2 (1/40320 - r^2 / 3628800))))
  float pc = __builtin_fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = __builtin_fmaf(pc, r2, -1.0f / 720.0f);
  pc = __builtin_fmaf(pc, r2, 0x1.555558p-5f);  // 1/24, one FP32 step up
  pc = __builtin_fmaf(pc, r2, -0.5f);
  const float cm = r2 * pc;
  // v exp(-i r) = (x + (x cm + y sn), y + (y cm - x sn)): the two small terms are summed
  // before they meet x, so the one rounding to x's precision sees the whole change.
  // (Rounded first as x + x cm, the decrement x cm < 0 is lost whenever it is below half
  // an FP32 step of x, and |result|^2 gains sn^2: on a packet whose phases are mostly
  // below 1e-3, a norm gain of about 7e-9 per potential substep.)
  const float a = v.x + __builtin_fmaf(v.x, cm, v.y * sn);
  const float b = v.y + __builtin_fmaf(v.y, cm, -v.x * sn);
  // times (-i)^q: q = 1 maps (a, b) to (b, -a), q = 2 to (-a, -b), q = 3 to (-b, a)
  const int q = (int)n & 3;
  const bool odd = (q & 1) != 0;
  const float u = odd ? b : a, w = odd ? a : b;
  const uint32_t su = (uint32_t)(q & 2) << 30, sw = (uint32_t)((q + 1) & 2) << 30;
  return float2{__uint_as_float(__float_as_uint(u) ^ su), __uint_as_float(__float_as_uint(w) ^ sw)};
}

// The same in FP64 for the complex128 path: Taylor series to x^17 / x^16 on
// |r| <= pi/4 (truncation below 1e-19).
__device__ __forceinline__ double2 phase_poly64(double phi) {
  const double two_over_pi = 0.63661977236758134307553505349006;
  const double pio2_hi = 1.5707963267341256;   // as in mul_phase_f32
  const double pio2_lo = 6.077100506506192e-11;
  const double n = rint(phi * two_over_pi);
  const double r = (phi - n * pio2_hi) - n * pio2_lo;
  const double r2 = r * r;
  // sin r = r - r^3 P(r^2), P = 1/3! - r^2/5! + ... - r^14/17!  (Horner from the top)
  const double ps =
      ((((((((-1.0 / 355687428096000.0) * r2 + 1.0 / 1307674368000.0) * r2 - 1.0 / 6227020800.0) * r2 +
           1.0 / 39916800.0) * r2 - 1.0 / 362880.0) * r2 + 1.0 / 5040.0) * r2 - 1.0 / 120.0) * r2 + 1.0 / 6.0);
  const double sn = r - r * r2 * ps;              // r - r^3/6 + r^5/120 - ...
  // cos r = 1 + r^2 Q(r^2), Q = -1/2! + r^2/4! - ... + r^14/16!
  const double pc = ((((((((1.0 / 20922789888000.0) * r2 - 1.0 / 87178291200.0) * r2 + 1.0 / 479001600.0) * r2 -
                   1.0 / 3628800.0) * r2 + 1.0 / 40320.0) * r2 - 1.0 / 720.0) * r2 + 1.0 / 24.0) * r2 - 0.5);
  const double cs = 1.0 + r2 * pc;
  // exp(i phi) = exp(i q pi/2) (cs + i sn): odd q swaps the pair, q = 1, 2 negate
  // the cosine, q = 2, 3 the sine (selects and sign flips on the high word: no
  // branches, which would diverge across a wave)
  const int q = (int)n & 3;
  const bool odd = (q & 1) != 0;
  const double c0 = odd ? sn : cs, s0 = odd ? cs : sn;
  const uint64_t sc = (uint64_t)((q + 1) & 2) << 62, ss = (uint64_t)(q & 2) << 62;
  const double c = __longlong_as_double(__double_as_longlong(c0) ^ (long long)sc);
  const double ms = __longlong_as_double(__double_as_longlong(s0) ^ (long long)(ss ^ 0x8000000000000000ull));
  return double2{c, ms};
}

// x exp(-i phi) with phi in FP64: complex64 through mul_phase_f32, complex128 with
// the FP64 sine and cosine.
template <typename T, typename C> __device__ __forceinline__ C mul_phase(C v, double phi) {
  if constexpr (sizeof(T) == 4) {
    return mul_phase_f32(v, phi);
  } else {
    double s, c;
    sincos(phi, &s, &c);
    return cmul(v, C{c, -s});
  }
}

// ---------------------------------------------------------------------------
// Workgroup reduction of nacc FP64 values to out[0..nacc) (fixed order).
// ---------------------------------------------------------------------------
// `red` is LDS scratch of (NTHR/64) * MGK_NACC doubles (the caller's tile buffer
// once the tile work is done).
template <int NTHR>
__device__ __forceinline__ void block_reduce(double* acc, int nacc, double* out, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < MGK_NACC; ++k) {
    if (k >= nacc) break;
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wv * MGK_NACC + k] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < nacc) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NTHR / 64; ++w) s += red[w * MGK_NACC + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Per-axis index-decode constants read once into registers before an element
// loop (read inside it, each would cost an LDS or memory round trip per element).
struct AxDec {
  uint32_t n[MGK_MAXD];
  DivW dn[MGK_MAXD];
};
__device__ __forceinline__ AxDec load_axdec(const PacketGeom& G, int D) {
  AxDec A;
#pragma unroll
  for (int l = 0; l < MGK_MAXD; ++l) {
    A.n[l] = l < D ? (uint32_t)G.ax[l].n : 1u;
    A.dn[l] = l < D ? G.ax[l].dn : DivW{1u, 0u, 0ull};
  }
  return A;
}

// Decode the multi-index of a point from (outer, group, inner) parts of a sweep.
__device__ __forceinline__ void decode_index(const AxDec& A, int D, int a, int b, uint32_t o, uint32_t g,
                                             uint32_t i, int* j) {
  // unrolled over MGK_MAXD so that j[] (and the caller's per-axis arrays) keep
  // static indices and live in registers
#pragma unroll
  for (int l = MGK_MAXD - 1; l >= 0; --l) {
    if (l >= D) continue;
    const uint32_t v = l >= b ? i : (l >= a ? g : o);
    const uint32_t qq = divw(v, A.dn[l]);
    j[l] = (int)(v - qq * A.n[l]);
    if (l >= b) i = qq;
    else if (l >= a) g = qq;
    else o = qq;
  }
}
__device__ __forceinline__ void decode_index(const PacketGeom& G, int a, int b, uint32_t o, uint32_t g,
                                             uint32_t i, int* j) {
  decode_index(load_axdec(G, G.D), G.D, a, b, o, g, i, j);
}

// Epilogue modes of a sweep / pointwise pass (bit flags).
enum : int {
  EPI_REDP = 1,    // sums w, w (k_l - N_l/2)                      (momentum moments)
  EPI_EKIN = 2,    // + sum w T(p^K)                                (observables)
  EPI_V = 4,       // potential substep: phase exp(-i h V / hbar) and sums w, w dV/dq_l
  EPI_REDQ = 8,    // sums w, w (j_l - N_l/2), w V(q^J)             (observables)
  EPI_SCALE = 16   // multiply by PacketState.scale
};

// Per-line factors of the two-dimensional atom-diatom potential (kind 2, D = 2:
// a Morse well along axis 0 plus the repulsion A exp(-b (q_1 - c q_0))).  With
// x_0 = q_0 - q_c,0 the repulsion factors into exp(b c x_0) exp(-b (q_1 - c q_c,0)),
// so a grid needs 2 N_0 + N_1 exponentials instead of two per point:
//   tab[j0] = exp(-a (q_0 - r_e)),  tab[N_0 + j0] = exp(b c x_0),
//   tab[2 N_0 + j1] = exp(-b (q_1 - c q_c,0))
// (the exponents stay within b c times half the span, whatever the centres).
// Built by the whole workgroup; q_l as in epilogue_point.
template <int NTHR>
__device__ __forceinline__ void build_morse_tab(const PacketGeom& G, const PacketState& st, const PotDesc& P,
                                                double* tab) {
  const int n0 = G.ax[0].n, n1 = G.ax[1].n;
  const double a = P.p[1], re = P.p[2], b = P.p[4], c = P.p[5];
  for (int i = threadIdx.x; i < 2 * n0 + n1; i += NTHR) {
    double v;
    if (i < n0) {
      const double q0 = st.q_c[0] + (double)(i - n0 / 2) * G.ax[0].dq;
      v = exp(-a * (q0 - re));
    } else if (i < 2 * n0) {
      v = exp(b * c * ((double)(i - n0 - n0 / 2) * G.ax[0].dq));
    } else {
      const double q1 = st.q_c[1] + (double)(i - 2 * n0 - n1 / 2) * G.ax[1].dq;
      v = exp(-b * (q1 - c * st.q_c[0]));
    }
    tab[i] = v;
  }
}

// Pointwise work on one element with full multi-index j; returns the new value.
// DT > 0 fixes the number of axes at compile time (specialised batch kernels).
// mtab: the atom-diatom line factors of build_morse_tab (potential kind 2, D = 2),
// or null to evaluate the potential point by point.
template <typename T, int DT = 0>
__device__ __forceinline__ typename CT<T>::type epilogue_point(typename CT<T>::type x, const int* j,
                                                               const PacketGeom& G, const PacketState& st,
                                                               const PotDesc& P, int mode, double h,
                                                               double* acc, const double* mtab = nullptr) {
  const int D = DT > 0 ? DT : G.D;
  if (mode & EPI_SCALE) {
    const T s = (T)st.scale;
    x.x *= s;
    x.y *= s;
  }
  const double w = (double)x.x * (double)x.x + (double)x.y * (double)x.y;
  if (mode & (EPI_REDP | EPI_REDQ)) {
    acc[0] += w;
#pragma unroll
    for (int l = 0; l < MGK_MAXD; ++l)
      if (l < D) acc[1 + l] += w * (double)(j[l] - G.ax[l].n / 2);
    if (mode & EPI_EKIN) {
      double e = 0.0;
#pragma unroll
      for (int l = 0; l < MGK_MAXD; ++l) {
        if (l >= D) break;
        const double p = st.p_c[l] + (double)(j[l] - G.ax[l].n / 2) * G.ax[l].dp;
        e += 0.5 * G.ax[l].minv * p * p;
      }
      // slot D + 1 by select-adds over fixed indices: a dynamic index would put the
      // whole accumulator array in scratch memory for every epilogue of the kernel
      const double we = w * e;
#pragma unroll
      for (int k = 2; k < MGK_NACC; ++k) acc[k] += (k == D + 1) ? we : 0.0;
    }
    if (mode & EPI_REDQ) {
      double q[MGK_MAXD];
#pragma unroll
      for (int l = 0; l < MGK_MAXD; ++l) q[l] = l < D ? st.q_c[l] + (double)(j[l] - G.ax[l].n / 2) * G.ax[l].dq : 0.0;
      const double Vq = w * pot_eval(P, D, q, nullptr);
#pragma unroll
      for (int k = 2; k < MGK_NACC; ++k) acc[k] += (k == D + 1) ? Vq : 0.0;
    }
  }
  if (mode & EPI_V) {
    double q[MGK_MAXD], g[MGK_MAXD];
    double V;
    if (mtab) {
      // the terms of pot_eval's kind 2 in its order, the exponentials from the table
      const int n0 = G.ax[0].n;
      const double e = mtab[j[0]];
      const double rep = P.p[3] * (mtab[n0 + j[0]] * mtab[2 * n0 + j[1]]);
      V = P.p[0] * (1.0 - e) * (1.0 - e);
      double g0 = 2.0 * P.p[0] * P.p[1] * e * (1.0 - e);
      V += rep;
      g0 += P.p[4] * P.p[5] * rep;
      g[0] = g0;
      g[1] = -P.p[4] * rep;
#pragma unroll
      for (int l = 2; l < MGK_MAXD; ++l) g[l] = 0.0;
    } else {
#pragma unroll
      for (int l = 0; l < MGK_MAXD; ++l) q[l] = l < D ? st.q_c[l] + (double)(j[l] - G.ax[l].n / 2) * G.ax[l].dq : 0.0;
      V = pot_eval(P, D, q, g);
    }
    acc[0] += w;
#pragma unroll
    for (int l = 0; l < MGK_MAXD; ++l)
      if (l < D) acc[1 + l] += w * g[l];
    x = mul_phase<T>(x, h * V / G.hbar);
  }
  return x;
}

}  // namespace mgk
