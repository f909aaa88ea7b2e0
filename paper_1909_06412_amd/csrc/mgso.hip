// mgso.hip -- kernels and host runtime behind include/mgso.h (gfx950).
//
// Method: Choi & Vanicek, arXiv:1909.06412 (equation numbers count the paper's
// displayed equations in order of appearance).  See mgso_kernels.h for the
// arithmetic of one substep and mgso_sweep.h for the tiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mgso.h"
#include "mgso_sweep.h"
#include "mgso_sweep16.h"
#include "mgso_split.h"

using namespace mgk;

#define NTHR 256
#define MAX_BLOCKS 2048

// ===========================================================================
// Kernels
// ===========================================================================
// Finalize modes.
enum : int {
  FIN_T = 1,        // <p> -> delta = h m^-1 <p>, q_ctr += delta, then the M tables
  FIN_V = 2,        // <dV/dq> -> p_ctr -= h <dV/dq>, then the A tables
  FIN_REGRID = 3,   // delta forced (h = 0), q_ctr += delta, then the M tables
  FIN_OBSQ = 4,     // store position-grid sums
  FIN_OBSP = 5,     // store momentum-grid sums
  FIN_BUILD_A = 6,  // only rebuild the A tables from p_ctr
  FIN_NORM = 7,     // scale = 1/sqrt(sum w) for a following renormalisation pass
  FIN_NAIVE_A = 8,  // naive re-centring: p_ctr = <p>, delta = <q> - q_ctr (from the obs sums), A tables
  FIN_NAIVE_M = 9   // naive re-centring: q_ctr += delta, M tables of the shift (h = 0)
};

template <typename T> struct FinArgs {
  const PacketGeom* geom;
  PacketState* st;
  const double* partials;
  int nblk;
  int mode;
  double h;
  double forced[MGK_MAXD];
  typename TE<T>::type* A;
  typename TE<T>::type* M;
  typename TE<T>::type* AG;   // group-combined tables (16-point path), may be null
  typename TE<T>::type* MG;
};

// Body of the finalize (one workgroup of NTHR threads); also run at the end of a
// one-workgroup sweep (k_sweep<T, true>), which saves a launch per substep on grids
// that fit one tile.
template <typename T> __device__ __forceinline__ void finalize_body(const FinArgs<T>& a);

template <typename T> struct SweepArgs {
  const PacketGeom* geom;
  const PacketState* st;
  const PotDesc* pot;
  const typename CT<T>::type* src;
  typename CT<T>::type* dst;
  Tables<T> tb;
  double* partials;  // [gridDim.x][MGK_NACC] when epi != 0
  int si, dir, epi;
  double h;
  FinArgs<T> fin;    // FIN: the finalize this one-workgroup sweep ends with
};

// One sweep of one packet over all its tiles (grid-stride over tiles).  FIN: a
// launch of one workgroup that then runs the finalize of its reduction itself.
template <typename T, bool FIN = false>
__global__ __launch_bounds__(NTHR) void k_sweep(SweepArgs<T> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  typedef typename CT<T>::type C;
  C* lds = reinterpret_cast<C*>(lds_raw);
  const PacketGeom& G = *a.geom;
  const SweepDesc& sw = G.sw[a.si];
  double acc[MGK_NACC];
#pragma unroll
  for (int k = 0; k < MGK_NACC; ++k) acc[k] = 0.0;
  for (uint32_t tile = blockIdx.x; tile < sw.ntiles; tile += gridDim.x)
    process_tile<T, NTHR, MGK_TMAX, false, 0, false, 8>(lds, G, a.si, tile, a.src, a.dst, a.tb, a.dir, a.epi, a.h,
                                                        *a.st, *a.pot, acc, true, true);
  if (a.epi) block_reduce<NTHR>(acc, G.D + 2, a.partials + (size_t)blockIdx.x * MGK_NACC, (double*)lds_raw);
  if constexpr (FIN) {
    __syncthreads();  // the partial sums and every read of the tables before they are rebuilt
    finalize_body<T>(a.fin);
  }
}

// Pointwise pass over all points of a packet (standalone potential substep,
// observables on the position grid, renormalisation).
template <typename T> struct PointArgs {
  const PacketGeom* geom;
  const PacketState* st;
  const PotDesc* pot;
  typename CT<T>::type* psi;
  double* partials;
  int epi;
  double h;
};

template <typename T>
__global__ __launch_bounds__(NTHR) void k_pointwise(PointArgs<T> a) {
  typedef typename CT<T>::type C;
  const PacketGeom& G = *a.geom;
  double acc[MGK_NACC];
#pragma unroll
  for (int k = 0; k < MGK_NACC; ++k) acc[k] = 0.0;
  const uint64_t N = G.N_total;
  for (uint64_t e = (uint64_t)blockIdx.x * NTHR + threadIdx.x; e < N; e += (uint64_t)gridDim.x * NTHR) {
    int j[MGK_MAXD];
    decode_index(G, G.D, G.D, (uint32_t)e, 0, 0, j);
    C x = gload(a.psi, G.off + e);
    x = epilogue_point<T>(x, j, G, *a.st, *a.pot, a.epi, a.h, acc);
    if (a.epi & (EPI_V | EPI_SCALE)) gstore(a.psi, G.off + e, x);
  }
  __shared__ double red[(NTHR / 64) * MGK_NACC];
  if (a.epi & (EPI_V | EPI_REDQ | EPI_REDP))
    block_reduce<NTHR>(acc, G.D + 2, a.partials + (size_t)blockIdx.x * MGK_NACC, red);
}

template <typename T>
__global__ __launch_bounds__(NTHR) void k_finalize(FinArgs<T> a) {
  finalize_body<T>(a);
}

template <typename T> __device__ __forceinline__ void finalize_body(const FinArgs<T>& a) {
  typedef typename CT<T>::type C;
  const PacketGeom& G = *a.geom;
  PacketState& st = *a.st;
  const int D = G.D;
  const int nacc = D + 2;
  __shared__ double tot[MGK_NACC];
  __shared__ double red[(NTHR / 64) * MGK_NACC];
  if (a.mode != FIN_BUILD_A && a.mode != FIN_REGRID && a.mode != FIN_NAIVE_A && a.mode != FIN_NAIVE_M) {
    double acc[MGK_NACC];
    for (int k = 0; k < nacc; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < a.nblk; b += NTHR)
      for (int k = 0; k < nacc; ++k) acc[k] += a.partials[(size_t)b * MGK_NACC + k];
    block_reduce<NTHR>(acc, nacc, tot, red);
  }
  if (threadIdx.x == 0) {
    if (a.mode == FIN_T) {
      fin_kinetic(G, st, tot, a.h);
    } else if (a.mode == FIN_REGRID) {
      for (int l = 0; l < D; ++l) {
        st.delta[l] = a.forced[l];
        st.q_c[l] += a.forced[l];
      }
    } else if (a.mode == FIN_V) {
      fin_potential(G, st, tot, a.h);
    } else if (a.mode == FIN_OBSQ) {
      for (int k = 0; k < nacc; ++k) st.obs[k] = tot[k];
    } else if (a.mode == FIN_OBSP) {
      for (int k = 0; k < nacc; ++k) st.obs[MGK_NACC + k] = tot[k];
    } else if (a.mode == FIN_NORM) {
      for (int k = 0; k < nacc; ++k) st.last[k] = tot[k];
      st.scale = tot[0] > 0.0 ? 1.0 / sqrt(tot[0]) : 1.0;
    } else if (a.mode == FIN_NAIVE_A) {
      // Eqs. (29)-(34): the new centres are the expectation values of the state
      // propagated on the frozen grid (position sums in obs[0..], momentum sums,
      // taken on the p-grid at the old p_ctr, in obs[MGK_NACC..])
      const double nq = st.obs[0], np_ = st.obs[MGK_NACC];
      bool bad = !(nq > 0.0) || !(np_ > 0.0);
      for (int l = 0; l < D; ++l) {
        const double dl = G.ax[l].dq * st.obs[1 + l] / nq;
        const double pl = st.p_c[l] + G.ax[l].dp * st.obs[MGK_NACC + 1 + l] / np_;
        if (!isfinite(dl) || !isfinite(pl) || fabs(dl) > 0.5 * G.ax[l].n * G.ax[l].dq) bad = true;
        st.delta[l] = dl;
        st.p_c[l] = pl;
      }
      if (bad) st.err = 1;
    } else if (a.mode == FIN_NAIVE_M) {
      for (int l = 0; l < D; ++l) st.q_c[l] += st.delta[l];
    }
  }
  __syncthreads();
  const double hbar = G.hbar;
  const bool doM = a.mode == FIN_T || a.mode == FIN_REGRID || a.mode == FIN_NAIVE_M;
  const bool doA = a.mode == FIN_V || a.mode == FIN_BUILD_A || a.mode == FIN_NAIVE_A;
  if (doM) build_M_tables<T, NTHR>(G, st, a.mode == FIN_T ? a.h : 0.0, a.M);
  if (doA) build_A_tables<T, NTHR>(G, st, a.A);
  // Group-combined tables of the 16-point path: one FP64 angle sum per entry.
  if (G.fast16 && a.AG) {
    if (doA || doM) {
      const double h = a.mode == FIN_T ? a.h : 0.0;
      for (int si = 0; si < G.nsweeps; ++si) {
        const SweepDesc& sw = G.sw[si];
        const int K = sw.b - sw.a;
        const double mag = doA ? ldexp(1.0, -2 * K) : 1.0;   // prod 1/sqrt(16)
        for (uint32_t g = threadIdx.x; g < sw.LG; g += NTHR) {
          double ang = 0.0;
          for (int l = sw.b - 1, sh = 0; l >= sw.a; --l, sh += 4) {
            const int j = (int)((g >> sh) & 15u);
            const AxisDesc& ax = G.ax[l];
            if (doA) {
              ang += M_PI * (double)(j & 1) - st.p_c[l] * (double)j * ax.dq / hbar;
            } else {
              const double p = st.p_c[l] + (double)(j - 8) * ax.dp;
              ang -= (h * 0.5 * ax.minv * p * p - st.delta[l] * p) / hbar;
            }
          }
          double s, c;
          sincos(ang, &s, &c);
          const typename TE<T>::type v = make_te<T>(mag * c, mag * s);
          if (doA) a.AG[sw.gtab_off + g] = v;
          else a.MG[sw.gtab_off + g] = v;
        }
      }
      if (G.split) {
        // tables of the three-pass 16^8 plan (mgso_split.h): per-axis angles summed
        // in FP64, as above; A_l(j) carries (-1)^j and 1/4, M_l(k) the momentum
        // p = p_ctr + (k - 8) dp of Eq. (55)
        auto angA = [&](int l, int j) {
          return M_PI * (double)(j & 1) - st.p_c[l] * (double)j * G.ax[l].dq / hbar;
        };
        auto angM = [&](int l, int k) {
          const double p = st.p_c[l] + (double)(k - 8) * G.ax[l].dp;
          return -(h * 0.5 * G.ax[l].minv * p * p - st.delta[l] * p) / hbar;
        };
        const int ys = SPL_SPLIT_AXIS;
        for (int e = threadIdx.x; e < SPL_TAB; e += NTHR) {
          double ang, mag = 1.0;
          if (e < 2048) {
            // A products of the passes (the kinetic factors go per axis below)
            if (!doA) continue;
            const int pass = e >> 10, g = e & 1023;
            const int X = g & 15, Y = (g >> 4) & 3, Z = g >> 6;
            const int ax = SPL_AX[pass][0], az = SPL_AX[pass][1];
            ang = angA(ax, X) + angA(az, Z);
            mag = 1.0 / 16.0;
            if (pass == 0) {
              // high digit n1 = Y of the split axis: its index 4 n1 is even
              ang -= st.p_c[ys] * (double)(4 * Y) * G.ax[ys].dq / hbar;
              mag = 1.0 / 64.0;
            }
          } else if (e < 2064) {
            const int k = e - 2048;
            if (doA) {
              // c(n0) W16^(n0 k0) at 4 n0 + k0
              const int n0 = k >> 2, k0 = k & 3;
              ang = angA(ys, n0) - 2.0 * M_PI * (double)(n0 * k0) / 16.0;
            } else {
              ang = angM(ys, k);
            }
          } else {
            // per-axis M: pass C's X and Z axes, then pass B's (the A side is unused)
            const int q = (e - 2064) >> 4, k = (e - 2064) & 15;
            ang = doA ? 0.0 : angM(SPL_AX[q < 2 ? 1 : 0][q & 1], k);
          }
          double sn, cs;
          sincos(ang, &sn, &cs);
          const typename TE<T>::type v = make_te<T>(mag * cs, mag * sn);
          if (doA) a.AG[G.gtab_len + e] = v;
          else a.MG[G.gtab_len + e] = v;
        }
      }
    }
  }
}

// Initial Gaussian (FP64), one factor per axis, scaled by sqrt(prod dq).
struct GaussArgs {
  const PacketGeom* geom;
  const PacketState* st;
  double q0[MGK_MAXD], p0[MGK_MAXD], sigma[MGK_MAXD];
};

template <typename T>
__global__ __launch_bounds__(NTHR) void k_init_gaussian(GaussArgs a, typename CT<T>::type* psi) {
  typedef typename CT<T>::type C;
  const PacketGeom& G = *a.geom;
  const int D = G.D;
  double lognorm = 0.0;
  for (int l = 0; l < D; ++l)
    lognorm += -0.25 * log(M_PI * a.sigma[l] * a.sigma[l]) + 0.5 * log(G.ax[l].dq);
  for (uint64_t e = (uint64_t)blockIdx.x * NTHR + threadIdx.x; e < G.N_total; e += (uint64_t)gridDim.x * NTHR) {
    int j[MGK_MAXD];
    decode_index(G, D, D, (uint32_t)e, 0, 0, j);
    double re = lognorm, ph = 0.0;
    for (int l = 0; l < D; ++l) {
      const double q = a.st->q_c[l] + (double)(j[l] - G.ax[l].n / 2) * G.ax[l].dq;
      const double x = q - a.q0[l];
      re -= x * x / (2.0 * a.sigma[l] * a.sigma[l]);
      ph += a.p0[l] * x / G.hbar;
    }
    const double amp = exp(re);
    double s, c;
    sincos(ph, &s, &c);
    psi[G.off + e] = C{(decltype(C().x))(amp * c), (decltype(C().x))(amp * s)};
  }
}

// Autocorrelation <psi_0|psi_t> (Sec. III.C) with psi_0 the Gaussian of Eq. (62)
// evaluated analytically on the current grid.  psi_0 is a product of per-axis
// factors: tab[l][j] = (pi sigma_l^2)^(-1/4) sqrt(dq_l) exp(-x^2/(2 sigma_l^2) + i p0_l x / hbar),
// x = q_ctr,l + (j - N_l/2) dq_l - q0_l (FP64, built by k_acf_tables).
__global__ __launch_bounds__(NTHR) void k_acf_tables(GaussArgs a, double2* tab) {
  const PacketGeom& G = *a.geom;
  for (int l = 0; l < G.D; ++l) {
    const AxisDesc& ax = G.ax[l];
    const double lg = -0.25 * log(M_PI * a.sigma[l] * a.sigma[l]) + 0.5 * log(ax.dq);
    for (int j = threadIdx.x; j < ax.n; j += NTHR) {
      const double x = a.st->q_c[l] + (double)(j - ax.n / 2) * ax.dq - a.q0[l];
      const double amp = exp(lg - x * x / (2.0 * a.sigma[l] * a.sigma[l]));
      double sn, cs;
      sincos(a.p0[l] * x / G.hbar, &sn, &cs);
      tab[ax.tab_off + j] = double2{amp * cs, amp * sn};
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NTHR) void k_acf(const PacketGeom* geom, const typename CT<T>::type* psi,
                                              const double2* tab, double* partials) {
  const PacketGeom& G = *geom;
  const int D = G.D;
  double acc[MGK_NACC];
#pragma unroll
  for (int k = 0; k < MGK_NACC; ++k) acc[k] = 0.0;
  for (uint64_t e = (uint64_t)blockIdx.x * NTHR + threadIdx.x; e < G.N_total; e += (uint64_t)gridDim.x * NTHR) {
    int j[MGK_MAXD];
    decode_index(G, D, D, (uint32_t)e, 0, 0, j);
    double2 f = tab[G.ax[0].tab_off + j[0]];
    for (int l = 1; l < D; ++l) {
      const double2 g = tab[G.ax[l].tab_off + j[l]];
      f = double2{f.x * g.x - f.y * g.y, f.x * g.y + f.y * g.x};
    }
    const auto x = psi[G.off + e];
    // conj(f) * x
    acc[0] += f.x * (double)x.x + f.y * (double)x.y;
    acc[1] += f.x * (double)x.y - f.y * (double)x.x;
  }
  __shared__ double red[(NTHR / 64) * MGK_NACC];
  block_reduce<NTHR>(acc, D + 2, partials + (size_t)blockIdx.x * MGK_NACC, red);
}

// ===========================================================================
// Host runtime
// ===========================================================================
namespace {

struct Packet {
  PacketGeom geom;  // host copy
};

bool is_smooth(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}

std::vector<int> radices(int n) {
  std::vector<int> r;
  while (n % 8 == 0 && n > 8) { r.push_back(8); n /= 8; }
  if (n % 8 == 0) { r.push_back(8); n /= 8; }
  while (n % 4 == 0) { r.push_back(4); n /= 4; }
  while (n % 2 == 0) { r.push_back(2); n /= 2; }
  while (n % 3 == 0) { r.push_back(3); n /= 3; }
  while (n % 5 == 0) { r.push_back(5); n /= 5; }
  return r;
}

// Passes for the ping-pong pass, which also has the composite radices 9, 10, 12,
// 15 and 16: fewest passes, then the smallest largest radix (fewer registers per
// butterfly), larger radices first.
static bool wide_better(const std::vector<int>& a, const std::vector<int>& b) {
  if (a.size() != b.size()) return a.size() < b.size();
  const int ma = *std::max_element(a.begin(), a.end()), mb = *std::max_element(b.begin(), b.end());
  if (ma != mb) return ma < mb;
  return std::lexicographical_compare(b.begin(), b.end(), a.begin(), a.end());
}
std::vector<int> radices_wide(int n) {
  static const int kR[] = {16, 15, 12, 10, 9, 8, 5, 4, 3, 2};
  std::map<int, std::vector<int>> best;  // m | n -> plan for m
  best[1] = {};
  std::vector<int> divs;
  for (int m = 2; m <= n; ++m)
    if (n % m == 0) divs.push_back(m);
  for (int m : divs) {  // increasing: every proper divisor of m is already planned
    bool have = false;
    std::vector<int> pick;
    for (int r : kR) {
      if (m % r) continue;
      auto it = best.find(m / r);
      if (it == best.end()) continue;
      std::vector<int> c = it->second;
      c.push_back(r);
      std::sort(c.begin(), c.end(), std::greater<int>());
      if (!have || wide_better(c, pick)) {
        pick = c;
        have = true;
      }
    }
    if (have) best[m] = pick;
  }
  return best.count(n) ? best[n] : radices(n);
}

// Build the per-axis passes and the sweep plan of one packet.
bool build_geom(int D, const int32_t* N, const double* dq, const double* minv, double hbar, int tw_base,
                std::map<int, int>& tw_offsets, int& tw_total, PacketGeom& G, std::string& err,
                uint32_t tmax = MGK_TMAX, bool wide = false) {
  memset(&G, 0, sizeof(G));
  G.D = D;
  G.hbar = hbar;
  uint64_t tot = 1;
  int tab = 0;
  for (int l = 0; l < D; ++l) {
    const int n = N[l];
    if (n < 2 || n % 2 || n > MG_MAX_AXIS || !is_smooth(n)) {
      err = "N_l must be even, 2.." + std::to_string(MG_MAX_AXIS) + " and of the form 2^a 3^b 5^c";
      return false;
    }
    if (!(dq[l] > 0.0) || !std::isfinite(dq[l]) || !std::isfinite(minv[l])) {
      err = "dq must be positive and finite, inv_mass finite";
      return false;
    }
    AxisDesc& ax = G.ax[l];
    ax.n = n;
    ax.dq = dq[l];
    ax.dp = 2.0 * M_PI * hbar / (n * dq[l]);
    ax.minv = minv[l];
    ax.dn = make_divw(n);
    ax.tab_off = tab;
    tab += n;
    auto it = tw_offsets.find(n);
    if (it == tw_offsets.end()) {
      tw_offsets[n] = tw_base + tw_total;
      ax.tw_off = tw_base + tw_total;
      tw_total += n;
    } else {
      ax.tw_off = it->second;
    }
    std::vector<int> rs = wide ? radices_wide(n) : radices(n);
    ax.npass = (int)rs.size();
    int Ns = 1;
    for (size_t p = 0; p < rs.size(); ++p) {
      PassDesc& pd = ax.pass[p];
      pd.R = (uint16_t)rs[p];
      pd.Ns = (uint16_t)Ns;
      pd.tws = (uint16_t)(n / (Ns * rs[p]));
      pd.dNs = make_div32(Ns);
      pd.dNbl = make_div32(n / rs[p]);
      Ns *= rs[p];
    }
    tot *= (uint64_t)n;
  }
  if (tot > (1ull << 32)) {
    err = "more than 2^32 grid points";
    return false;
  }
  G.N_total = tot;
  G.tab_len = tab;
  // sweeps, from the innermost axis outward
  const uint32_t RUN = 16;
  int b = D, ns = 0;
  while (b > 0) {
    SweepDesc& s = G.sw[ns];
    uint64_t I = 1;
    for (int l = b; l < D; ++l) I *= N[l];
    int a = b - 1;
    uint64_t LG = N[a];
    const uint64_t need = b == D ? 1 : std::min<uint64_t>(I, RUN);
    while (a > 0 && LG * N[a - 1] * need <= tmax) {
      --a;
      LG *= N[a];
    }
    uint64_t O = 1;
    for (int l = 0; l < a; ++l) O *= N[l];
    s.a = a;
    s.b = b;
    s.O = (uint32_t)O;
    s.LG = (uint32_t)LG;
    s.I = (uint32_t)I;
    if (b == D) {
      s.kind = 0;
      s.ob = (uint32_t)std::min<uint64_t>(O, tmax / LG);
      s.r = 1;
      s.T = s.ob * s.LG;
      s.tiles_i = 1;
      s.ntiles = (uint32_t)((O + s.ob - 1) / s.ob);
    } else {
      s.kind = 1;
      s.ob = 1;
      s.r = (uint32_t)std::min<uint64_t>(I, tmax / LG);
      s.T = s.LG * s.r;
      s.tiles_i = (uint32_t)((I + s.r - 1) / s.r);
      s.ntiles = (uint32_t)(O * s.tiles_i);
    }
    s.dLG = make_div32(s.LG);
    s.dr = make_div32(s.r);
    s.dtiles_i = make_divw(s.tiles_i);
    // LDS strides: tile is [ob][N_a..N_{b-1}][r]
    uint32_t stride = s.kind == 1 ? s.r : 1;
    for (int l = b - 1; l >= a; --l) {
      s.S[l - a] = stride;
      s.dS[l - a] = make_div32(stride);
      stride *= N[l];
    }
    ++ns;
    b = a;
  }
  G.nsweeps = ns;
  return true;
}

struct Unit {
  bool hasT, hasV;
  double hT, hV;
};

// Expand a scheme into merged substeps and pair each kinetic substep with the
// potential substep that follows it.
std::vector<Unit> lower_scheme(int split, const std::vector<double>& gam, double dt, int64_t nsteps) {
  std::vector<std::pair<char, double>> subs;
  for (int64_t s = 0; s < nsteps; ++s)
    for (double g : gam) {
      const double h = g * dt;
      if (split == MG_TVT) {
        subs.push_back({'T', h / 2});
        subs.push_back({'V', h});
        subs.push_back({'T', h / 2});
      } else {
        subs.push_back({'V', h / 2});
        subs.push_back({'T', h});
        subs.push_back({'V', h / 2});
      }
    }
  std::vector<std::pair<char, double>> merged;
  for (auto& x : subs) {
    if (!merged.empty() && merged.back().first == x.first) merged.back().second += x.second;
    else merged.push_back(x);
  }
  std::vector<Unit> units;
  for (size_t i = 0; i < merged.size(); ++i) {
    Unit u{false, false, 0.0, 0.0};
    if (merged[i].first == 'T') {
      u.hasT = true;
      u.hT = merged[i].second;
      if (i + 1 < merged.size() && merged[i + 1].first == 'V') {
        u.hasV = true;
        u.hV = merged[i + 1].second;
        ++i;
      }
    } else {
      u.hasV = true;
      u.hV = merged[i].second;
    }
    units.push_back(u);
  }
  return units;
}

std::vector<double> composition(int comp, int order, const double* user, int nuser, std::string& err) {
  std::vector<double> g{1.0};
  if (comp == MG_COMP_USER) {
    if (!user || nuser < 1) { err = "user gammas missing"; return {}; }
    std::vector<double> u(user, user + nuser);
    double s = 0;
    for (int i = 0; i < nuser; ++i) {
      s += u[i];
      if (std::fabs(u[i] - u[nuser - 1 - i]) > 1e-12) { err = "gammas must be palindromic"; return {}; }
    }
    if (std::fabs(s - 1.0) > 1e-12) { err = "gammas must sum to one"; return {}; }
    return u;
  }
  if (order < 2 || order > 10 || order % 2) { err = "order must be even, 2..10"; return {}; }
  if (comp == MG_COMP_STRANG || order == 2) return g;
  for (int n = 1; n < order / 2; ++n) {
    std::vector<double> ng;
    if (comp == MG_COMP_SUZUKI) {
      const double x = std::pow(4.0, 1.0 / (2 * n + 1));
      const double a = 1.0 / (4.0 - x);
      const double c[5] = {a, a, 1.0 - 4.0 * a, a, a};
      for (double cc : c)
        for (double gg : g) ng.push_back(cc * gg);
    } else if (comp == MG_COMP_TRIPLE_JUMP) {
      const double x = std::pow(2.0, 1.0 / (2 * n + 1));
      const double a = 1.0 / (2.0 - x);
      const double c[3] = {a, 1.0 - 2.0 * a, a};
      for (double cc : c)
        for (double gg : g) ng.push_back(cc * gg);
    } else {
      err = "unknown composition";
      return {};
    }
    g.swap(ng);
  }
  return g;
}

}  // namespace

// ===========================================================================
// Context
// ===========================================================================
struct ProfEntry {
  hipEvent_t e0, e1;
  int cls;
};

#define MG_MAGIC_CTX 0x4d474358u
#define MG_MAGIC_BATCH 0x4d474258u

struct mg_ctx {
  uint32_t magic = MG_MAGIC_CTX;
  std::string err;
  int D = 0;
  mg_precision prec = MG_C128;
  hipStream_t stream = nullptr;
  size_t csize = 16;
  PacketGeom geom{};
  PacketGeom* d_geom = nullptr;
  PacketState* d_st = nullptr;
  PotDesc pot{};
  PotDesc* d_pot = nullptr;
  void* d_tw = nullptr;
  void* d_A = nullptr;
  void* d_M = nullptr;
  void* d_AG = nullptr;
  void* d_MG = nullptr;
  S16Desc s16[MGK_MAXD];
  SplitDesc spl[2];  // passes B and C of the three-pass 16^8 plan (geom.split)
  int n_cu = 0;      // compute units of the device (grid of the split passes)
  double* d_part = nullptr;
  void* psi = nullptr;
  bool psi_owned = false;
  void* work = nullptr;
  bool work_owned = false;
  bool has_state = false, has_pot = false;
  int split = MG_TVT;
  std::vector<double> gam{1.0};
  int opt_graph = 0, opt_profile = 0, opt_renorm = 0, opt_engine = 0;
  double2* d_acf = nullptr;  // per-axis factors of the autocorrelation reference (sum N_l)
  int grid_mode = 0;  // MG_OPT_GRID: 0 moving (Sec. II.G), 1 fixed, 2 naive re-centring (Sec. II.F)
  std::vector<ProfEntry> prof_pending;
  std::map<int, std::pair<int64_t, double>> prof;  // class -> (launches, ms)
  // captured step (MG_OPT_GRAPH): replayed while (dt, nsteps, version) match
  uint64_t version = 0;  // bumped by everything that changes the launch sequence or its pointers
  hipGraphExec_t gexec = nullptr;
  hipStream_t gcap = nullptr;
  double g_dt = 0.0;
  int64_t g_n = -1;
  uint64_t g_ver = ~0ull;
};

static thread_local std::string g_create_err;
static const char* batch_error(const void* p);

static mg_status fail(mg_ctx* c, mg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail((ctx), MG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Twiddle table of each axis length n: exp(-2 pi i m / n) for m < n at off + m, as
// table entries (make_te: complex64 keeps the remainder of the rounding as well).
template <typename T> static void build_twiddles(const std::map<int, int>& offs, int total,
                                                 std::vector<typename mgk::TE<T>::type>& out) {
  out.assign((size_t)total, mgk::make_te<T>(0.0, 0.0));
  for (auto& kv : offs) {
    const int n = kv.first, off = kv.second;
    for (int m = 0; m < n; ++m) {
      const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)n;
      out[off + m] = mgk::make_te<T>((double)cosl(ang), (double)sinl(ang));
    }
  }
}

static int grid_for(uint64_t work_items) {
  uint64_t b = std::max<uint64_t>(1, work_items);
  return (int)std::min<uint64_t>(b, MAX_BLOCKS);
}

template <typename T> static Tables<T> tables_of(mg_ctx* c) {
  typedef typename TE<T>::type E;
  return Tables<T>{(const E*)c->d_tw, (const E*)c->d_A, (const E*)c->d_M};
}

template <typename T> static FinArgs<T> fin_args(mg_ctx* c, int mode, double h, int nblk, const double* forced) {
  FinArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.geom = c->d_geom;
  a.st = c->d_st;
  a.partials = c->d_part;
  a.nblk = nblk;
  a.mode = mode;
  a.h = h;
  if (forced)
    for (int l = 0; l < c->D; ++l) a.forced[l] = forced[l];
  typedef typename TE<T>::type E;
  a.A = (E*)c->d_A;
  a.M = (E*)c->d_M;
  a.AG = (E*)c->d_AG;
  a.MG = (E*)c->d_MG;
  return a;
}

template <typename T> static mg_status launch_finalize(mg_ctx* c, int mode, double h, int nblk, const double* forced) {
  const FinArgs<T> a = fin_args<T>(c, mode, h, nblk, forced);
  hipLaunchKernelGGL(k_finalize<T>, dim3(1), dim3(NTHR), 0, c->stream, a);
  HIPCHK(c, hipGetLastError());
  return MG_OK;
}

template <typename T, int K, bool INV, int EPI> static void launch16(mg_ctx* c, const S16Args<T>& a, int grid,
                                                                     int mode) {
  typedef typename CT<T>::type C;
  const size_t lds = k16_lds_bytes<T>(K, INV);
  const dim3 nt(k16_threads(K));
  if constexpr (K == 1 && !INV && EPI == EPI_REDP) {
    if (mode == SW_MOMENTS) {
      hipLaunchKernelGGL((k_sweep16<T, 1, false, EPI_REDP, -1, SW_MOMENTS>), dim3(grid), nt, lds, c->stream, a);
      return;
    }
  }
  if constexpr (K == 1 && INV && EPI == 0) {
    if (mode == SW_ROUNDTRIP) {
      hipLaunchKernelGGL((k_sweep16<T, 1, true, 0, -1, SW_ROUNDTRIP>), dim3(grid), nt, lds, c->stream, a);
      return;
    }
  }
  if constexpr (EPI == EPI_V) {
    switch (c->pot.kind) {
      case MG_POT_FREE: hipLaunchKernelGGL((k_sweep16<T, K, INV, EPI, 0>), dim3(grid), nt, lds, c->stream, a); break;
      case MG_POT_HARMONIC: hipLaunchKernelGGL((k_sweep16<T, K, INV, EPI, 1>), dim3(grid), nt, lds, c->stream, a); break;
      case MG_POT_HENON_HEILES:
        // the 8-D model's contiguous tile (axes 5-7) with the dimension fixed
        if (K == 3 && c->D == 8 && a.d.a == 5)
          hipLaunchKernelGGL((k_sweep16<T, K, INV, EPI, 3, 0, K == 3 ? 8 : 0>), dim3(grid), nt, lds, c->stream, a);
        else
          hipLaunchKernelGGL((k_sweep16<T, K, INV, EPI, 3>), dim3(grid), nt, lds, c->stream, a);
        break;
      default: hipLaunchKernelGGL((k_sweep16<T, K, INV, EPI, 4>), dim3(grid), nt, lds, c->stream, a); break;
    }
  } else {
    hipLaunchKernelGGL((k_sweep16<T, K, INV, EPI>), dim3(grid), nt, lds, c->stream, a);
  }
}

template <typename T, bool INV, int EPI>
static void launch16_k(mg_ctx* c, const S16Args<T>& a, int grid, int mode) {
  switch (a.d.K) {
    case 1: launch16<T, 1, INV, EPI>(c, a, grid, mode); break;
    case 2: launch16<T, 2, INV, EPI>(c, a, grid, mode); break;
    default: launch16<T, 3, INV, EPI>(c, a, grid, mode); break;
  }
}

// The 16-point kernels run a propagation step's sweeps (plain, REDP and V epilogues).
static bool fast16_step(const mg_ctx* c) {
  return c->opt_engine != 1 && c->geom.fast16 && pot_is_cubic(c->pot.kind);
}
// A kinetic substep of such a step turns round on its outermost sweep (moments-only
// forward, round-trip inverse) when that sweep is a one-axis strided sweep.
static bool fast16_turn(const mg_ctx* c) {
  const int ns = c->geom.nsweeps;
  return fast16_step(c) && ns >= 2 && c->s16[ns - 1].K == 1 && c->s16[ns - 1].kind == 1;
}

// Launch sweep si; returns the number of blocks (for the finalize).  fast = use
// the 16-point kernel when the packet qualifies (only plain, REDP and V epilogues);
// mode SW_MOMENTS / SW_ROUNDTRIP only where fast16_turn holds.
// fin_mode != 0: the finalize that follows this sweep; a generic sweep of one
// workgroup runs it itself (*fused = true) and the caller skips its launch.
template <typename T>
static mg_status launch_sweep(mg_ctx* c, int si, int dir, int epi, double h, const void* src, void* dst, int* nblk,
                              bool fast = false, int mode = SW_FULL, int fin_mode = 0, double fin_h = 0.0,
                              bool* fused = nullptr) {
  if (fused) *fused = false;
  typedef typename CT<T>::type C;
  if (mode != SW_FULL &&
      !(fast && fast16_turn(c) && si == c->geom.nsweeps - 1 &&
        (mode == SW_MOMENTS ? dir == DIR_FWD && epi == EPI_REDP : dir == DIR_INV && epi == 0)))
    return fail(c, MG_EINVAL, "internal: turning sweep requested where the plan has none");
  if (fast && fast16_step(c) && (epi == 0 || epi == EPI_REDP || epi == EPI_V)) {
    S16Args<T> a;
    a.geom = c->d_geom;
    a.st = c->d_st;
    a.pot = c->d_pot;
    a.src = (const C*)src;
    a.dst = (C*)dst;
    a.AG = (const typename TE<T>::type*)c->d_AG;
    a.MG = (const typename TE<T>::type*)c->d_MG;
    a.partials = c->d_part;
    a.d = c->s16[si];
    a.h = h;
    const int grid = grid_for(a.d.ntiles);
    *nblk = grid;
    ProfEntry pe{};
    if (c->opt_profile) {
      HIPCHK(c, hipEventCreate(&pe.e0));
      HIPCHK(c, hipEventCreate(&pe.e1));
      HIPCHK(c, hipEventRecord(pe.e0, c->stream));
    }
    const bool inv = dir == DIR_INV;
    if (!inv) {
      if (epi == EPI_REDP) launch16_k<T, false, EPI_REDP>(c, a, grid, mode);
      else launch16_k<T, false, 0>(c, a, grid, mode);
    } else {
      if (epi == EPI_V) launch16_k<T, true, EPI_V>(c, a, grid, mode);
      else launch16_k<T, true, 0>(c, a, grid, mode);
    }
    HIPCHK(c, hipGetLastError());
    if (c->opt_profile) {
      HIPCHK(c, hipEventRecord(pe.e1, c->stream));
      pe.cls = mode * 4096 + si * 64 + dir * 32 + epi;
      c->prof_pending.push_back(pe);
    }
    return MG_OK;
  }
  SweepArgs<T> a;
  a.geom = c->d_geom;
  a.st = c->d_st;
  a.pot = c->d_pot;
  a.src = (const C*)src;
  a.dst = (C*)dst;
  a.tb = tables_of<T>(c);
  a.partials = c->d_part;
  a.si = si;
  a.dir = dir;
  a.epi = epi;
  a.h = h;
  const int grid = grid_for(c->geom.sw[si].ntiles);
  *nblk = grid;
  const bool fuse = fin_mode != 0 && grid == 1 && fused;
  if (fuse) a.fin = fin_args<T>(c, fin_mode, fin_h, 1, nullptr);
  else memset(&a.fin, 0, sizeof(a.fin));
  const size_t lds = (size_t)MGK_TMAX * sizeof(C);
  ProfEntry pe{};
  if (c->opt_profile) {
    HIPCHK(c, hipEventCreate(&pe.e0));
    HIPCHK(c, hipEventCreate(&pe.e1));
    HIPCHK(c, hipEventRecord(pe.e0, c->stream));
  }
  if (fuse) {
    hipLaunchKernelGGL((k_sweep<T, true>), dim3(grid), dim3(NTHR), lds, c->stream, a);
    *fused = true;
  } else {
    hipLaunchKernelGGL((k_sweep<T, false>), dim3(grid), dim3(NTHR), lds, c->stream, a);
  }
  HIPCHK(c, hipGetLastError());
  if (c->opt_profile) {
    HIPCHK(c, hipEventRecord(pe.e1, c->stream));
    pe.cls = si * 64 + dir * 32 + epi;
    c->prof_pending.push_back(pe);
  }
  return MG_OK;
}

template <typename T> static mg_status launch_pointwise(mg_ctx* c, int epi, double h, int* nblk) {
  typedef typename CT<T>::type C;
  PointArgs<T> a;
  a.geom = c->d_geom;
  a.st = c->d_st;
  a.pot = c->d_pot;
  a.psi = (C*)c->psi;
  a.partials = c->d_part;
  a.epi = epi;
  a.h = h;
  const int grid = grid_for((c->geom.N_total + NTHR - 1) / NTHR);
  *nblk = grid;
  hipLaunchKernelGGL(k_pointwise<T>, dim3(grid), dim3(NTHR), 0, c->stream, a);
  HIPCHK(c, hipGetLastError());
  return MG_OK;
}

// Forward transform of src into dst (dst may equal src); the last sweep reduces
// the momentum moments with epilogue `epi_last`.
// The three-pass plan runs a 16^8 step's kinetic substeps (engine 0).
static bool split_step(const mg_ctx* c) { return c->opt_engine == 0 && c->geom.split && fast16_turn(c); }

template <typename T, int KIND> static void launch_split_k(mg_ctx* c, const SplArgs<T>& a, int grid) {
  hipLaunchKernelGGL((k_split<T, KIND>), dim3(grid), dim3(spl_nt<T>()), spl_lds_bytes<T>(), c->stream, a);
}

// One pass of the three-pass plan on buf (in place); kind SPL_*.  One workgroup
// per compute unit (the tile takes most of the LDS), each looping over its tiles.
template <typename T> static mg_status launch_split(mg_ctx* c, int kind, void* buf, int* nblk) {
  typedef typename CT<T>::type C;
  SplArgs<T> a;
  a.geom = c->d_geom;
  a.src = (const C*)buf;
  a.dst = (C*)buf;
  a.AG = (const typename TE<T>::type*)c->d_AG;
  a.MG = (const typename TE<T>::type*)c->d_MG;
  a.partials = c->d_part;
  a.d = c->spl[kind >= SPL_C_MOM ? 1 : 0];
  const int grid = std::min<int>(c->n_cu > 0 ? c->n_cu : 256, MAX_BLOCKS);
  *nblk = grid;
  ProfEntry pe{};
  if (c->opt_profile) {
    HIPCHK(c, hipEventCreate(&pe.e0));
    HIPCHK(c, hipEventCreate(&pe.e1));
    HIPCHK(c, hipEventRecord(pe.e0, c->stream));
  }
  switch (kind) {
    case SPL_B_FWD: launch_split_k<T, SPL_B_FWD>(c, a, grid); break;
    case SPL_B_INV: launch_split_k<T, SPL_B_INV>(c, a, grid); break;
    case SPL_C_MOM: launch_split_k<T, SPL_C_MOM>(c, a, grid); break;
    default: launch_split_k<T, SPL_C_RT>(c, a, grid); break;
  }
  HIPCHK(c, hipGetLastError());
  if (c->opt_profile) {
    HIPCHK(c, hipEventRecord(pe.e1, c->stream));
    const int mode = kind == SPL_C_MOM ? SW_SPLIT_MOM : SW_SPLIT;
    const int si = kind >= SPL_C_MOM ? 2 : 1;
    const int dir = (kind == SPL_B_INV || kind == SPL_C_RT) ? DIR_INV : DIR_FWD;
    pe.cls = mode * 4096 + si * 64 + dir * 32 + (kind == SPL_C_MOM ? EPI_REDP : 0);
    c->prof_pending.push_back(pe);
  }
  return MG_OK;
}

// turn: the last sweep only reduces (dst keeps that axis group untransformed; the
// next inverse_transform must turn too).
template <typename T>
static mg_status forward_transform(mg_ctx* c, const void* src, void* dst, int epi_last, int* nblk_last,
                                   bool fast = false, bool turn = false, int fin_mode = 0, double fin_h = 0.0,
                                   bool* fused = nullptr) {
  if (fused) *fused = false;
  const int ns = c->geom.nsweeps;
  if (fast && turn && split_step(c)) {
    if (epi_last != EPI_REDP) return fail(c, MG_EINVAL, "internal: the three-pass plan reduces momentum moments");
    int nb;
    mg_status r = launch_sweep<T>(c, 0, DIR_FWD, 0, 0.0, src, dst, &nb, fast);
    if (!r) r = launch_split<T>(c, SPL_B_FWD, dst, &nb);
    if (!r) r = launch_split<T>(c, SPL_C_MOM, dst, nblk_last);
    return r;
  }
  for (int s = 0; s < ns; ++s) {
    int nb;
    const int mode = turn && s == ns - 1 ? SW_MOMENTS : SW_FULL;
    mg_status r = launch_sweep<T>(c, s, DIR_FWD, s == ns - 1 ? epi_last : 0, 0.0, s == 0 ? src : dst, dst, &nb,
                                  fast, mode, s == ns - 1 ? fin_mode : 0, fin_h, s == ns - 1 ? fused : nullptr);
    if (r) return r;
    if (s == ns - 1) *nblk_last = nb;
  }
  return MG_OK;
}

template <typename T>
static mg_status inverse_transform(mg_ctx* c, void* buf, int epi_first_sweep, double hV, int* nblk_last,
                                   bool fast = false, bool turn = false, int fin_mode = 0, bool* fused = nullptr) {
  if (fused) *fused = false;
  const int ns = c->geom.nsweeps;
  if (fast && turn && split_step(c)) {
    int nb;
    mg_status r = launch_split<T>(c, SPL_C_RT, buf, &nb);
    if (!r) r = launch_split<T>(c, SPL_B_INV, buf, &nb);
    if (!r) r = launch_sweep<T>(c, 0, DIR_INV, epi_first_sweep, hV, buf, buf, nblk_last, fast);
    return r;
  }
  for (int s = ns - 1; s >= 0; --s) {
    int nb;
    const int mode = turn && s == ns - 1 ? SW_ROUNDTRIP : SW_FULL;
    mg_status r = launch_sweep<T>(c, s, DIR_INV, s == 0 ? epi_first_sweep : 0, hV, buf, buf, &nb, fast, mode,
                                  s == 0 ? fin_mode : 0, hV, s == 0 ? fused : nullptr);
    if (r) return r;
    if (s == 0) *nblk_last = nb;
  }
  return MG_OK;
}

template <typename T> static mg_status run_unit(mg_ctx* c, const Unit& u) {
  mg_status r;
  int nb = 0;
  if (u.hasT) {
    const bool turn = fast16_turn(c);
    bool fused = false;
    if ((r = forward_transform<T>(c, c->psi, c->psi, EPI_REDP, &nb, true, turn, FIN_T, u.hT, &fused))) return r;
    if (!fused && (r = launch_finalize<T>(c, FIN_T, u.hT, nb, nullptr))) return r;
    if ((r = inverse_transform<T>(c, c->psi, u.hasV ? EPI_V : 0, u.hV, &nb, true, turn, u.hasV ? FIN_V : 0,
                                  &fused)))
      return r;
    if (u.hasV && !fused && (r = launch_finalize<T>(c, FIN_V, u.hV, nb, nullptr))) return r;
  } else if (u.hasV) {
    if ((r = launch_pointwise<T>(c, EPI_V, u.hV, &nb))) return r;
    if ((r = launch_finalize<T>(c, FIN_V, u.hV, nb, nullptr))) return r;
  }
  if (u.hasV && c->opt_renorm) {
    if ((r = launch_pointwise<T>(c, EPI_REDQ, 0.0, &nb))) return r;
    if ((r = launch_finalize<T>(c, FIN_NORM, 0.0, nb, nullptr))) return r;
    if ((r = launch_pointwise<T>(c, EPI_SCALE, 0.0, &nb))) return r;
  }
  return MG_OK;
}

static mg_status collect_profile(mg_ctx* c) {
  for (auto& pe : c->prof_pending) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, pe.e0, pe.e1));
    auto& e = c->prof[pe.cls];
    e.first += 1;
    e.second += ms;
    hipEventDestroy(pe.e0);
    hipEventDestroy(pe.e1);
  }
  c->prof_pending.clear();
  return MG_OK;
}

// One-dimensional grids of at most 64 points: the whole call in one wave (mgso_small.inc).
static bool small_path(const mg_ctx* c);
template <typename T> static mg_status launch_small(mg_ctx* c, double dt, int64_t nsteps);

template <typename T> static mg_status step_impl(mg_ctx* c, double dt, int64_t nsteps) {
  if (small_path(c)) return launch_small<T>(c, dt, nsteps);
  mg_status r;
  if ((r = launch_finalize<T>(c, FIN_BUILD_A, 0.0, 0, nullptr))) return r;
  std::vector<Unit> units = lower_scheme(c->split, c->gam, dt, nsteps);
  for (const Unit& u : units)
    if ((r = run_unit<T>(c, u))) return r;
  return MG_OK;
}

// The naive adaptive grid (Sec. II.F, Eqs. (29)-(34)): each step runs on the
// frozen grid, then the grid is re-centred on the new expectation values: p_ctr
// moves to <p> (taken on the p-grid at the old p_ctr) and the state is shifted by
// <q> - q_ctr by trigonometric interpolation on the p-grid at the new p_ctr.
template <typename T> static mg_status naive_recentre(mg_ctx* c) {
  mg_status r;
  int nb = 0;
  if ((r = launch_pointwise<T>(c, EPI_REDQ, 0.0, &nb))) return r;
  if ((r = launch_finalize<T>(c, FIN_OBSQ, 0.0, nb, nullptr))) return r;
  if ((r = launch_finalize<T>(c, FIN_BUILD_A, 0.0, 0, nullptr))) return r;
  if ((r = forward_transform<T>(c, c->psi, c->work, EPI_REDP, &nb))) return r;
  if ((r = launch_finalize<T>(c, FIN_OBSP, 0.0, nb, nullptr))) return r;
  if ((r = launch_finalize<T>(c, FIN_NAIVE_A, 0.0, 0, nullptr))) return r;
  if ((r = forward_transform<T>(c, c->psi, c->psi, 0, &nb))) return r;
  if ((r = launch_finalize<T>(c, FIN_NAIVE_M, 0.0, 0, nullptr))) return r;
  return inverse_transform<T>(c, c->psi, 0, 0.0, &nb);
}

// The launches of mg_step(dt, nsteps) for the context's grid mode.
template <typename T> static mg_status step_body(mg_ctx* c, double dt, int64_t nsteps) {
  if (c->grid_mode != 2) return step_impl<T>(c, dt, nsteps);
  mg_status r;
  for (int64_t s = 0; s < nsteps; ++s)
    if ((r = step_impl<T>(c, dt, 1)) || (r = naive_recentre<T>(c))) return r;
  return MG_OK;
}

// MG_OPT_GRAPH: capture the launches of mg_step(dt, nsteps) once (on a private
// stream: the caller's may be the null stream, which cannot be captured) and
// replay the instantiated graph on the caller's stream.  The sequence has only
// kernel launches (no memset or copy nodes).
static mg_status step_graph(mg_ctx* c, double dt, int64_t nsteps) {
  if (!c->gexec || c->g_dt != dt || c->g_n != nsteps || c->g_ver != c->version) {
    if (c->gexec) {
      HIPCHK(c, hipGraphExecDestroy(c->gexec));
      c->gexec = nullptr;
    }
    if (!c->gcap) HIPCHK(c, hipStreamCreateWithFlags(&c->gcap, hipStreamNonBlocking));
    // the capture must not overtake work already queued on the caller's stream
    HIPCHK(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    hipStream_t user = c->stream;
    c->stream = c->gcap;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->gcap, hipStreamCaptureModeThreadLocal);
    mg_status r = MG_OK;
    if (e == hipSuccess) {
      r = c->prec == MG_C64 ? step_body<float>(c, dt, nsteps) : step_body<double>(c, dt, nsteps);
      e = hipStreamEndCapture(c->gcap, &g);
    }
    c->stream = user;
    if (r == MG_OK && e == hipSuccess) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (r) return r;
    if (e != hipSuccess) {
      c->gexec = nullptr;
      return fail(c, MG_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    c->g_dt = dt;
    c->g_n = nsteps;
    c->g_ver = c->version;
  }
  HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  return MG_OK;
}

static mg_status sync_and_check(mg_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->opt_profile) {
    mg_status r = collect_profile(c);
    if (r) return r;
  }
  int32_t err = 0;
  HIPCHK(c, hipMemcpy(&err, &c->d_st->err, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (err) {
    c->has_state = false;
    return fail(c, MG_EUNSTABLE,
                "non-finite moments or a grid shift beyond half the grid span (Verlet instability of the centres)");
  }
  return MG_OK;
}

static mg_status ensure_psi(mg_ctx* c) {
  if (!c->psi) {
    HIPCHK(c, hipMalloc(&c->psi, mg_state_bytes(c)));
    c->psi_owned = true;
  }
  return MG_OK;
}

static mg_status ensure_work(mg_ctx* c) {
  if (!c->work) {
    HIPCHK(c, hipMalloc(&c->work, mg_workspace_bytes(c)));
    c->work_owned = true;
  }
  return MG_OK;
}

static mg_status upload_state_scalars(mg_ctx* c, const double* q, const double* p, double t) {
  PacketState st;
  memset(&st, 0, sizeof(st));
  for (int l = 0; l < c->D; ++l) {
    st.q_c[l] = q[l];
    st.p_c[l] = p[l];
  }
  st.t = t;
  st.scale = 1.0;
  st.fixed = c->grid_mode != 0;
  HIPCHK(c, hipMemcpyAsync(c->d_st, &st, sizeof(st), hipMemcpyHostToDevice, c->stream));
  return MG_OK;
}

// Dynamic-LDS limit of every 16-point kernel instantiation of one precision.
template <typename T, int K, bool INV, int EPI, int PK = -1, int DT = 0> static hipError_t lds_attr16() {
  return hipFuncSetAttribute((const void*)k_sweep16<T, K, INV, EPI, PK, 0, DT>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)k16_lds_bytes<T>(K, INV));
}
template <typename T, int K> static hipError_t lds_attr16_k() {
  hipError_t e = lds_attr16<T, K, false, 0>();
  if (e == hipSuccess) e = lds_attr16<T, K, false, EPI_REDP>();
  if (e == hipSuccess) e = lds_attr16<T, K, true, 0>();
  if (e == hipSuccess) e = lds_attr16<T, K, true, EPI_V, 0>();
  if (e == hipSuccess) e = lds_attr16<T, K, true, EPI_V, 1>();
  if (e == hipSuccess) e = lds_attr16<T, K, true, EPI_V, 3>();
  if (e == hipSuccess) e = lds_attr16<T, K, true, EPI_V, 4>();
  if (K == 3 && e == hipSuccess) e = lds_attr16<T, K, true, EPI_V, 3, K == 3 ? 8 : 0>();
  return e;
}
template <typename T> static hipError_t set_lds_attr16() {
  hipError_t e = lds_attr16_k<T, 1>();
  if (e == hipSuccess) e = lds_attr16_k<T, 2>();
  if (e == hipSuccess) e = lds_attr16_k<T, 3>();
  return e;
}

template <typename T> static hipError_t set_lds_attr_split() {
  const int b = (int)spl_lds_bytes<T>();
  const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipFuncSetAttribute((const void*)k_split<T, SPL_B_FWD>, at, b);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_split<T, SPL_B_INV>, at, b);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_split<T, SPL_C_MOM>, at, b);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_split<T, SPL_C_RT>, at, b);
  return e;
}

static int ilog2u(uint64_t v) {
  int l = 0;
  while ((1ull << l) < v) ++l;
  return (1ull << l) == v ? l : -1;
}

static void setup_fast16(mg_ctx* c) {
  PacketGeom& G = c->geom;
  G.fast16 = 0;
  G.gtab_len = 0;
  if (G.D < 3) return;
  for (int l = 0; l < G.D; ++l)
    if (G.ax[l].n != 16) return;
  int off = 0;
  for (int si = 0; si < G.nsweeps; ++si) {
    SweepDesc& sw = G.sw[si];
    S16Desc& d = c->s16[si];
    memset(&d, 0, sizeof(d));
    d.K = sw.b - sw.a;
    d.a = sw.a;
    d.kind = sw.kind;
    if (sw.T != 4096 || d.K < 1 || d.K > 3) return;
    if (sw.kind == 0 && (sw.ob != 1 || sw.LG != 4096)) return;
    if (sw.kind != (d.K == 3 ? 0 : 1)) return;  // the kernels fix the tile kind by K
    d.lr = ilog2u(sw.kind == 0 ? 1 : sw.r);
    d.lI = ilog2u(sw.I);
    d.lLG = ilog2u(sw.LG);
    d.ltiles_i = ilog2u(sw.tiles_i);
    if (d.lr < 0 || d.lI < 0 || d.lLG < 0 || d.ltiles_i < 0) return;
    if (sw.kind == 1 && sw.I % sw.r) return;
    d.tiles_i = sw.tiles_i;
    d.ntiles = sw.ntiles;
    if (sw.kind == 1) {
      // the 16-point kernels take strided tiles of 8192 points: twice the run of
      // the generic 4096-point plan (the group tables do not depend on the run)
      if (sw.I % (2 * sw.r) || sw.tiles_i % 2) return;
      d.lr += 1;
      d.tiles_i = sw.tiles_i / 2;
      d.ltiles_i -= 1;
      d.ntiles = sw.ntiles / 2;
    }
    for (int e = 0; e < d.K; ++e) d.lS[e] = 4 * (d.K - 1 - e) + d.lr;
    d.gtab_off = off;
    sw.gtab_off = off;
    off += (int)sw.LG;
  }
  G.gtab_len = off;
  G.fast16 = 1;
}

// The three-pass plan of 16^8 grids (mgso_split.h): the radix-16 plan must be
// sweep 0 over axes 5-7 (contiguous tile) and three strided sweeps.
static void setup_split(mg_ctx* c) {
  PacketGeom& G = c->geom;
  G.split = 0;
  if (!G.fast16 || G.D != 8 || G.nsweeps != 4) return;
  const int lr = c->prec == MG_C64 ? spl_lr<float>() : spl_lr<double>();  // log2 of the run
  if (c->s16[0].K != 3 || c->s16[0].a != 5 || c->s16[0].kind != 0) return;
  const int p2 = 4 * (7 - SPL_SPLIT_AXIS);
  for (int p = 0; p < 2; ++p) {
    SplitDesc& d = c->spl[p];
    memset(&d, 0, sizeof(d));
    d.axX = SPL_AX[p][0];
    d.axZ = SPL_AX[p][1];
    d.axY = SPL_SPLIT_AXIS;
    d.pX = 4 * (7 - d.axX);
    d.pZ = 4 * (7 - d.axZ);
    d.pY = p == 0 ? p2 + 2 : p2;
    d.pYc = p == 0 ? p2 : p2 + 2;
    const uint32_t in = ((1u << lr) - 1u) | (0xFu << d.pX) | (0x3u << d.pY) | (0xFu << d.pZ);
    // the tile index fills the other bits: maximal runs of them, low first
    int nf = 0, nb = 0;
    for (int b = 0; b < 32;) {
      if ((in >> b) & 1u) {
        ++b;
        continue;
      }
      int w = 0;
      while (b + w < 32 && !((in >> (b + w)) & 1u)) ++w;
      if (nf == 4) return;
      d.flo[nf] = b;
      d.fw[nf] = w;
      ++nf;
      nb += w;
      b += w;
    }
    if (nb != 22 - lr || __builtin_popcount(in) != 10 + lr) return;
    if (p == 1) {
      // pass C takes its tiles high fields first, so that the tiles in flight at once
      // lie far apart rather than on neighbouring 128-byte runs: measured on 16^8,
      // its round trip 34.1 -> 30.4 ms (complex128) and 16.8 -> 15.3 ms (complex64);
      // pass B is fastest low fields first
      std::reverse(d.flo, d.flo + nf);
      std::reverse(d.fw, d.fw + nf);
    }
    d.nf = nf;
    d.ntiles = 1u << (22 - lr);
    d.tab = G.gtab_len + 1024 * p;
    d.small = G.gtab_len + 2048;
  }
  G.split = 1;
}

// Tile size of a single grid.  Each tile of a sweep is one workgroup, so a small
// grid (a few tiles of 4096 points) leaves most of the device idle and every
// launch waits for a few long workgroups: halve the tile (not below 512 points
// nor below the longest axis) until a sweep has 128 tiles, as long as the plan
// keeps its number of sweeps.  Grids of 16-point axes keep 4096 (the 16-point
// kernels' tile).
static uint32_t single_tile_points(int D, const int32_t* N, const double* dq, const double* minv, double hbar) {
  uint64_t tot = 1;
  int32_t maxn = 1;
  bool all16 = D >= 3;
  for (int l = 0; l < D; ++l) {
    tot *= (uint64_t)std::max(N[l], 1);
    maxn = std::max(maxn, N[l]);
    if (N[l] != 16) all16 = false;
  }
  uint32_t t = MGK_TMAX;
  if (all16) return t;
  auto sweeps = [&](uint32_t tm) -> int {
    std::map<int, int> offs;
    int total = 0;
    std::string e;
    PacketGeom g;
    return build_geom(D, N, dq, minv, hbar, 0, offs, total, g, e, tm) ? g.nsweeps : -1;
  };
  const int ns = sweeps(t);
  while (t > 512 && tot / t < 128 && (int32_t)(t / 2) >= maxn && sweeps(t / 2) == ns) t /= 2;
  return t;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

mg_status mg_create(int D, const int32_t* N, const double* dq, const double* inv_mass, double hbar,
                    mg_precision prec, void* hip_stream, mg_ctx** out) {
  if (!out) return MG_EINVAL;
  *out = nullptr;
  if (D < 1 || D > MG_MAX_DIM || !N || !dq || !inv_mass || !(hbar > 0.0) || (prec != MG_C128 && prec != MG_C64))
    return MG_EINVAL;
  mg_ctx* c = new mg_ctx();
  c->D = D;
  c->prec = prec;
  c->stream = (hipStream_t)hip_stream;
  c->csize = prec == MG_C64 ? 8 : 16;
  std::map<int, int> tw_offs;
  int tw_total = 0;
  if (!build_geom(D, N, dq, inv_mass, hbar, 0, tw_offs, tw_total, c->geom, c->err,
                  single_tile_points(D, N, dq, inv_mass, hbar))) {
    g_create_err = c->err;
    delete c;
    return MG_EINVAL;
  }
  c->geom.off = 0;
  setup_fast16(c);
  setup_split(c);
  c->pot.kind = MG_POT_FREE;
  c->pot.D = D;
  hipError_t e = hipSuccess;
  const char* where = "hipMalloc";
  e = hipMalloc(&c->d_geom, sizeof(PacketGeom));
  if (e == hipSuccess) e = hipMalloc(&c->d_st, sizeof(PacketState));
  if (e == hipSuccess) e = hipMalloc(&c->d_pot, sizeof(PotDesc));
  // table entries are 16 bytes in both precisions (make_te)
  if (e == hipSuccess) e = hipMalloc(&c->d_tw, (size_t)tw_total * 16);
  if (e == hipSuccess) e = hipMalloc(&c->d_A, (size_t)c->geom.tab_len * 16);
  if (e == hipSuccess) e = hipMalloc(&c->d_M, (size_t)c->geom.tab_len * 16);
  if (e == hipSuccess) e = hipMalloc(&c->d_part, (size_t)MAX_BLOCKS * MGK_NACC * sizeof(double));
  const size_t gtab = (size_t)c->geom.gtab_len + (c->geom.split ? SPL_TAB : 0);
  if (e == hipSuccess && c->geom.fast16) e = hipMalloc(&c->d_AG, gtab * 16);
  if (e == hipSuccess && c->geom.fast16) e = hipMalloc(&c->d_MG, gtab * 16);
  if (e == hipSuccess && c->geom.fast16) {
    where = "hipFuncSetAttribute";
    e = prec == MG_C128 ? set_lds_attr16<double>() : set_lds_attr16<float>();
  }
  if (e == hipSuccess && c->geom.split)
    e = prec == MG_C128 ? set_lds_attr_split<double>() : set_lds_attr_split<float>();
  if (e == hipSuccess && c->geom.split) {
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  }
  if (e == hipSuccess) where = "hipMemcpy";
  if (e == hipSuccess) e = hipMemcpy(c->d_geom, &c->geom, sizeof(PacketGeom), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_pot, &c->pot, sizeof(PotDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->d_st, 0, sizeof(PacketState));
  if (e == hipSuccess) {
    if (prec == MG_C64) {
      std::vector<float4> tw;
      build_twiddles<float>(tw_offs, tw_total, tw);
      e = hipMemcpy(c->d_tw, tw.data(), tw.size() * sizeof(float4), hipMemcpyHostToDevice);
    } else {
      std::vector<double2> tw;
      build_twiddles<double>(tw_offs, tw_total, tw);
      e = hipMemcpy(c->d_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice);
    }
  }
  if (e != hipSuccess) {
    g_create_err = std::string(where) + ": " + hipGetErrorString(e);
    mg_destroy(c);
    return e == hipErrorOutOfMemory ? MG_ENOMEM : MG_EDEVICE;
  }
  *out = c;
  return MG_OK;
}

void mg_destroy(mg_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  for (auto& pe : c->prof_pending) {
    hipEventDestroy(pe.e0);
    hipEventDestroy(pe.e1);
  }
  if (c->psi_owned) hipFree(c->psi);
  if (c->work_owned) hipFree(c->work);
  hipFree(c->d_geom);
  hipFree(c->d_st);
  hipFree(c->d_pot);
  hipFree(c->d_tw);
  hipFree(c->d_A);
  hipFree(c->d_M);
  hipFree(c->d_part);
  if (c->d_AG) hipFree(c->d_AG);
  if (c->d_MG) hipFree(c->d_MG);
  if (c->d_acf) (void)hipFree(c->d_acf);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->gcap) (void)hipStreamDestroy(c->gcap);
  delete c;
}

size_t mg_state_bytes(const mg_ctx* c) { return c ? (size_t)c->geom.N_total * c->csize : 0; }
size_t mg_workspace_bytes(const mg_ctx* c) { return c ? (size_t)c->geom.N_total * c->csize : 0; }
void* mg_state_ptr(mg_ctx* c) { return c ? c->psi : nullptr; }

mg_status mg_bind_buffers(mg_ctx* c, void* psi_dev, void* work_dev) {
  if (!c || !psi_dev) return fail(c, MG_EINVAL, "psi_dev is NULL");
  ++c->version;
  if (((uintptr_t)psi_dev & 255) || ((uintptr_t)work_dev & 255)) return fail(c, MG_EINVAL, "buffers must be 256-byte aligned");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->psi_owned) hipFree(c->psi);
  if (c->work_owned && work_dev) hipFree(c->work);
  c->psi = psi_dev;
  c->psi_owned = false;
  if (work_dev) {
    c->work = work_dev;
    c->work_owned = false;
  }
  c->has_state = false;
  return MG_OK;
}

mg_status mg_set_gaussian(mg_ctx* c, const double* q0, const double* p0, const double* sigma) {
  if (!c || !q0 || !p0 || !sigma) return fail(c, MG_EINVAL, "null argument");
  for (int l = 0; l < c->D; ++l)
    if (!(sigma[l] > 0.0) || !std::isfinite(q0[l]) || !std::isfinite(p0[l]))
      return fail(c, MG_EINVAL, "sigma must be positive, q0/p0 finite");
  mg_status r;
  if ((r = ensure_psi(c))) return r;
  if ((r = upload_state_scalars(c, q0, p0, 0.0))) return r;
  GaussArgs a;
  memset(&a, 0, sizeof(a));
  a.geom = c->d_geom;
  a.st = c->d_st;
  for (int l = 0; l < c->D; ++l) {
    a.q0[l] = q0[l];
    a.p0[l] = p0[l];
    a.sigma[l] = sigma[l];
  }
  const int grid = grid_for((c->geom.N_total + NTHR - 1) / NTHR);
  if (c->prec == MG_C64)
    hipLaunchKernelGGL(k_init_gaussian<float>, dim3(grid), dim3(NTHR), 0, c->stream, a, (float2*)c->psi);
  else
    hipLaunchKernelGGL(k_init_gaussian<double>, dim3(grid), dim3(NTHR), 0, c->stream, a, (double2*)c->psi);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->has_state = true;
  return MG_OK;
}

mg_status mg_set_state(mg_ctx* c, const double* psi_phys, const double* q, const double* p, double t) {
  if (!c || !psi_phys || !q || !p) return fail(c, MG_EINVAL, "null argument");
  mg_status r;
  if ((r = ensure_psi(c))) return r;
  double sc = 1.0;
  for (int l = 0; l < c->D; ++l) sc *= c->geom.ax[l].dq;
  sc = std::sqrt(sc);
  const size_t n2 = 2 * (size_t)c->geom.N_total;
  if (c->prec == MG_C64) {
    std::vector<float> h(n2);
    for (size_t i = 0; i < n2; ++i) h[i] = (float)(psi_phys[i] * sc);
    HIPCHK(c, hipMemcpyAsync(c->psi, h.data(), n2 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::vector<double> h(n2);
    for (size_t i = 0; i < n2; ++i) h[i] = psi_phys[i] * sc;
    HIPCHK(c, hipMemcpyAsync(c->psi, h.data(), n2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if ((r = upload_state_scalars(c, q, p, t))) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->has_state = true;
  return MG_OK;
}

mg_status mg_get_state(mg_ctx* c, double* psi_phys, double* q, double* p, double* t) {
  if (!c) return MG_EINVAL;
  if (!c->psi) return fail(c, MG_ESTATE, "no state");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  PacketState st;
  HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof(st), hipMemcpyDeviceToHost));
  if (q)
    for (int l = 0; l < c->D; ++l) q[l] = st.q_c[l];
  if (p)
    for (int l = 0; l < c->D; ++l) p[l] = st.p_c[l];
  if (t) *t = st.t;
  if (psi_phys) {
    double sc = 1.0;
    for (int l = 0; l < c->D; ++l) sc *= c->geom.ax[l].dq;
    sc = 1.0 / std::sqrt(sc);
    const size_t n2 = 2 * (size_t)c->geom.N_total;
    if (c->prec == MG_C64) {
      std::vector<float> h(n2);
      HIPCHK(c, hipMemcpy(h.data(), c->psi, n2 * sizeof(float), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < n2; ++i) psi_phys[i] = (double)h[i] * sc;
    } else {
      HIPCHK(c, hipMemcpy(psi_phys, c->psi, n2 * sizeof(double), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < n2; ++i) psi_phys[i] *= sc;
    }
  }
  return MG_OK;
}

mg_status mg_set_potential(mg_ctx* c, mg_pot kind, const double* params, int np) {
  if (!c) return MG_EINVAL;
  ++c->version;
  PotDesc P;
  memset(&P, 0, sizeof(P));
  P.kind = kind;
  P.D = c->D;
  const int D = c->D;
  int need = -1;
  switch (kind) {
    case MG_POT_FREE: need = 0; break;
    case MG_POT_HARMONIC: need = 2 * D; break;
    case MG_POT_MORSE_REP: need = 6; if (D > 2) return fail(c, MG_EINVAL, "Morse+repulsion needs D <= 2"); break;
    case MG_POT_HENON_HEILES: need = 2; break;
    case MG_POT_QUADRATIC: need = D * D + D; if (D > 4) return fail(c, MG_EINVAL, "quadratic needs D <= 4"); break;
    default: return fail(c, MG_EINVAL, "unknown potential kind");
  }
  if (np != need || (need > 0 && !params)) return fail(c, MG_EINVAL, "wrong number of potential parameters");
  for (int i = 0; i < np; ++i) {
    if (!std::isfinite(params[i])) return fail(c, MG_EINVAL, "non-finite potential parameter");
    P.p[i] = params[i];
  }
  c->pot = P;
  HIPCHK(c, hipMemcpyAsync(c->d_pot, &c->pot, sizeof(PotDesc), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->has_pot = true;
  return MG_OK;
}

mg_status mg_set_scheme(mg_ctx* c, mg_split split, mg_comp comp, int order, const double* gammas, int ns) {
  if (!c) return MG_EINVAL;
  ++c->version;
  if (split != MG_TVT && split != MG_VTV) return fail(c, MG_EINVAL, "unknown split");
  std::string e;
  std::vector<double> g = composition(comp, order, gammas, ns, e);
  if (g.empty()) return fail(c, MG_EINVAL, e);
  c->split = split;
  c->gam = g;
  return MG_OK;
}

mg_status mg_step(mg_ctx* c, double dt, int64_t nsteps) {
  if (!c) return MG_EINVAL;
  if (!c->has_state) return fail(c, MG_ESTATE, "no valid state (set_gaussian / set_state first)");
  if (!std::isfinite(dt) || nsteps < 0) return fail(c, MG_EINVAL, "bad dt or nsteps");
  if (nsteps == 0) return MG_OK;
  mg_status r;
  if (c->opt_graph && !c->opt_profile) r = step_graph(c, dt, nsteps);
  else r = c->prec == MG_C64 ? step_body<float>(c, dt, nsteps) : step_body<double>(c, dt, nsteps);
  if (r) return r;
  if ((r = sync_and_check(c))) return r;
  // advance t on the host side of the state (device copy kept consistent)
  PacketState st;
  HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof(st), hipMemcpyDeviceToHost));
  st.t += dt * (double)nsteps;
  HIPCHK(c, hipMemcpy(&c->d_st->t, &st.t, sizeof(double), hipMemcpyHostToDevice));
  return MG_OK;
}

mg_status mg_observables(mg_ctx* c, double* out) {
  if (!c || !out) return MG_EINVAL;
  if (!c->has_state) return fail(c, MG_ESTATE, "no valid state");
  mg_status r;
  if ((r = ensure_work(c))) return r;
  int nb = 0;
  if (c->prec == MG_C64) {
    if ((r = launch_finalize<float>(c, FIN_BUILD_A, 0.0, 0, nullptr))) return r;
    if ((r = launch_pointwise<float>(c, EPI_REDQ, 0.0, &nb))) return r;
    if ((r = launch_finalize<float>(c, FIN_OBSQ, 0.0, nb, nullptr))) return r;
    if ((r = forward_transform<float>(c, c->psi, c->work, EPI_REDP | EPI_EKIN, &nb))) return r;
    if ((r = launch_finalize<float>(c, FIN_OBSP, 0.0, nb, nullptr))) return r;
  } else {
    if ((r = launch_finalize<double>(c, FIN_BUILD_A, 0.0, 0, nullptr))) return r;
    if ((r = launch_pointwise<double>(c, EPI_REDQ, 0.0, &nb))) return r;
    if ((r = launch_finalize<double>(c, FIN_OBSQ, 0.0, nb, nullptr))) return r;
    if ((r = forward_transform<double>(c, c->psi, c->work, EPI_REDP | EPI_EKIN, &nb))) return r;
    if ((r = launch_finalize<double>(c, FIN_OBSP, 0.0, nb, nullptr))) return r;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  PacketState st;
  HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof(st), hipMemcpyDeviceToHost));
  const int D = c->D;
  const double* sq = st.obs;
  const double* sp = st.obs + MGK_NACC;
  out[0] = sq[0];
  for (int l = 0; l < D; ++l) {
    out[1 + l] = st.q_c[l] + c->geom.ax[l].dq * sq[1 + l] / sq[0];
    out[1 + D + l] = st.p_c[l] + c->geom.ax[l].dp * sp[1 + l] / sp[0];
    out[1 + 2 * D + l] = st.q_c[l];
    out[1 + 3 * D + l] = st.p_c[l];
  }
  out[1 + 4 * D] = sp[D + 1] / sp[0];
  out[2 + 4 * D] = sq[D + 1] / sq[0];
  out[3 + 4 * D] = st.t;
  return MG_OK;
}

mg_status mg_autocorrelation(mg_ctx* c, const double* q0, const double* p0, const double* sigma, double* out) {
  if (!c || !q0 || !p0 || !sigma || !out) return MG_EINVAL;
  if (!c->has_state) return fail(c, MG_ESTATE, "no valid state");
  GaussArgs a;
  memset(&a, 0, sizeof(a));
  a.geom = c->d_geom;
  a.st = c->d_st;
  for (int l = 0; l < c->D; ++l) {
    if (!(sigma[l] > 0.0) || !std::isfinite(q0[l]) || !std::isfinite(p0[l]))
      return fail(c, MG_EINVAL, "bad Gaussian parameters");
    a.q0[l] = q0[l];
    a.p0[l] = p0[l];
    a.sigma[l] = sigma[l];
  }
  if (!c->d_acf) HIPCHK(c, hipMalloc(&c->d_acf, sizeof(double2) * (size_t)c->geom.tab_len));
  hipLaunchKernelGGL(k_acf_tables, dim3(1), dim3(NTHR), 0, c->stream, a, c->d_acf);
  HIPCHK(c, hipGetLastError());
  const int grid = grid_for((c->geom.N_total + NTHR - 1) / NTHR);
  if (c->prec == MG_C64) {
    hipLaunchKernelGGL(k_acf<float>, dim3(grid), dim3(NTHR), 0, c->stream, c->d_geom, (const float2*)c->psi,
                       (const double2*)c->d_acf, c->d_part);
  } else {
    hipLaunchKernelGGL(k_acf<double>, dim3(grid), dim3(NTHR), 0, c->stream, c->d_geom, (const double2*)c->psi,
                       (const double2*)c->d_acf, c->d_part);
  }
  HIPCHK(c, hipGetLastError());
  mg_status r = c->prec == MG_C64 ? launch_finalize<float>(c, FIN_OBSQ, 0.0, grid, nullptr)
                                  : launch_finalize<double>(c, FIN_OBSQ, 0.0, grid, nullptr);
  if (r) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  PacketState st;
  HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof(st), hipMemcpyDeviceToHost));
  out[0] = st.obs[0];
  out[1] = st.obs[1];
  return MG_OK;
}

mg_status mg_spectrum(const double* times, const double* acf, int n, const double* energies, int ne,
                      double t_damp, double hbar, double* out) {
  if (!times || !acf || !energies || !out || n < 2 || ne < 0 || !(t_damp > 0.0) || !(hbar > 0.0))
    return MG_EINVAL;
  for (int k = 0; k < ne; ++k) {
    double s = 0.0, prev = 0.0;
    for (int i = 0; i < n; ++i) {
      const double t = times[i], f = exp(-(t / t_damp) * (t / t_damp));
      const double ph = energies[k] * t / hbar;
      const double v = f * (acf[2 * i] * cos(ph) - acf[2 * i + 1] * sin(ph));  // Re[acf e^{i E t}]
      if (i > 0) s += 0.5 * (t - times[i - 1]) * (v + prev);
      prev = v;
    }
    out[k] = s;
  }
  return MG_OK;
}

mg_status mg_regrid(mg_ctx* c, const double* new_q) {
  if (!c || !new_q) return MG_EINVAL;
  if (!c->has_state) return fail(c, MG_ESTATE, "no valid state");
  PacketState st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof(st), hipMemcpyDeviceToHost));
  double d[MGK_MAXD];
  for (int l = 0; l < c->D; ++l) d[l] = new_q[l] - st.q_c[l];
  mg_status r;
  int nb = 0;
  if (c->prec == MG_C64) {
    if ((r = launch_finalize<float>(c, FIN_BUILD_A, 0.0, 0, nullptr))) return r;
    if ((r = forward_transform<float>(c, c->psi, c->psi, 0, &nb))) return r;
    if ((r = launch_finalize<float>(c, FIN_REGRID, 0.0, 0, d))) return r;
    if ((r = inverse_transform<float>(c, c->psi, 0, 0.0, &nb))) return r;
  } else {
    if ((r = launch_finalize<double>(c, FIN_BUILD_A, 0.0, 0, nullptr))) return r;
    if ((r = forward_transform<double>(c, c->psi, c->psi, 0, &nb))) return r;
    if ((r = launch_finalize<double>(c, FIN_REGRID, 0.0, 0, d))) return r;
    if ((r = inverse_transform<double>(c, c->psi, 0, 0.0, &nb))) return r;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // the forced shift lands exactly on new_q
  HIPCHK(c, hipMemcpy(c->d_st->q_c, new_q, sizeof(double) * c->D, hipMemcpyHostToDevice));
  return MG_OK;
}

mg_status mg_set_option(mg_ctx* c, int option, int64_t value) {
  if (!c) return MG_EINVAL;
  ++c->version;
  switch (option) {
    case MG_OPT_ENGINE: if (value < 0 || value > 2) return fail(c, MG_EINVAL, "engine 0..2"); c->opt_engine = (int)value; break;
    case MG_OPT_GRAPH: c->opt_graph = value != 0; break;
    case MG_OPT_PROFILE: c->opt_profile = value != 0; break;
    case MG_OPT_RENORMALIZE: c->opt_renorm = value != 0; break;
    case MG_OPT_GRID: {
      if (value < 0 || value > 2) return fail(c, MG_EINVAL, "grid mode 0..2");
      if (value == 2) {
        mg_status r = ensure_work(c);
        if (r) return r;
      }
      c->grid_mode = (int)value;
      const int32_t fx = value != 0;
      HIPCHK(c, hipMemcpy(&c->d_st->fixed, &fx, sizeof(fx), hipMemcpyHostToDevice));
      break;
    }
    default: return fail(c, MG_EINVAL, "unknown option");
  }
  return MG_OK;
}

mg_status mg_profile_class(const mg_ctx* c, int* sweep, int* dir, int* epi, int* group_axes, int* mode) {
  if (!c) return MG_EINVAL;
  int best = -1;
  double best_ms = -1;
  for (auto& kv : c->prof)
    if (kv.second.second > best_ms) {
      best_ms = kv.second.second;
      best = kv.first;
    }
  const int si = best < 0 ? -1 : (best & 4095) / 64;
  if (sweep) *sweep = si;
  if (dir) *dir = best < 0 ? -1 : (best / 32) & 1;
  if (epi) *epi = best < 0 ? -1 : best & 31;
  if (group_axes) *group_axes = si < 0 ? -1 : best / 4096 >= SW_SPLIT ? 3 : c->geom.sw[si].b - c->geom.sw[si].a;
  if (mode) *mode = best < 0 ? -1 : best / 4096;
  return MG_OK;
}

mg_status mg_profile_read(mg_ctx* c, int64_t* launches, double* total_ms, double* bytes, int reset) {
  if (!c) return MG_EINVAL;
  int best = -1;
  double best_ms = -1;
  for (auto& kv : c->prof)
    if (kv.second.second > best_ms) {
      best_ms = kv.second.second;
      best = kv.first;
    }
  if (launches) *launches = best < 0 ? 0 : c->prof[best].first;
  if (total_ms) *total_ms = best < 0 ? 0.0 : best_ms;
  // a moments-only sweep reads the state once; every other sweep reads and writes it
  const int md = best / 4096;
  if (bytes) *bytes = (md == SW_MOMENTS || md == SW_SPLIT_MOM ? 1.0 : 2.0) * (double)c->geom.N_total * (double)c->csize;
  if (reset) c->prof.clear();
  return MG_OK;
}

#ifndef MGSO_SOURCE_SHA256
#define MGSO_SOURCE_SHA256 "unknown"
#endif
const char* mg_build_hash(void) { return MGSO_SOURCE_SHA256; }

const char* mg_last_error(const void* p) {
  if (!p) return g_create_err.empty() ? "null context" : g_create_err.c_str();
  const uint32_t magic = *(const uint32_t*)p;
  if (magic == MG_MAGIC_CTX) return ((const mg_ctx*)p)->err.c_str();
  if (magic == MG_MAGIC_BATCH) return batch_error(p);
  return "unknown handle";
}

}  // extern "C"

// ===========================================================================
// Entry points completed in mgso_batch.hip / mgso_adjoint.hip
// ===========================================================================
#include "mgso_batch.inc"
#include "mgso_adjoint.inc"
#include "mgso_small.inc"
#include "mgso_noalloc.inc"
