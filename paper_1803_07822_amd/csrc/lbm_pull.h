// Streamed values of one fluid node, read from the pull layout; shared by
// the two-pass step, the state conversions, the force kernels and the
// re-projection.
//
// Layout: pop[l][x] holds the post-collision deviation f*_l(x) - w_l, except
// on links that leave through a wall or the interior plate, where it holds
// the bounced value destined to come back to x as direction opp(l).  The
// streamed deviation at x is pop[l][x - c_l], or pop[opp(l)][x] when the link
// from x - c_l is cut.  With open ends in x (Sec. VI.A) the values that
// would stream in from outside the end columns are extrapolated from the
// inner columns instead.
#pragma once

#include "lbm_device.h"

namespace lbm {

struct Pos {
  int i, jf, k;
  long long n;
};

__device__ __forceinline__ int wrapd(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ Pos pos_at(const Grid& g, int i, int jf, int k) {
  Pos p;
  p.i = i;
  p.jf = jf;
  p.k = k;
  p.n = ((long long)k * g.H + jf) * g.nx + i;
  return p;
}

// Regular pull: walls, plate and periodic x.  The cut test selects the
// address, not a branch, so that the pulls of all directions are issued
// together instead of each waiting for its own round trip.
template <class T, int l>
__device__ __forceinline__ T pull(const T* __restrict__ pop, const Grid& g, const Pos& p) {
  constexpr int x = cx(l), y = cy(l), z = cz(l);
  const bool cut = (y > 0 && p.jf == 0) || (y < 0 && p.jf == g.H - 1) || plate_cut(g, p.i, p.jf, -x, -y);
  const int is = x ? wrapd(p.i - x, g.nx) : p.i;
  const int ks = z ? wrapd(p.k - z, g.nz) : p.k;
  const int js = p.jf - y;
  const long long e = cut ? (long long)opp(l) * g.N + p.n : (long long)l * g.N + ((long long)ks * g.H + js) * g.nx + is;
  return pop[e];
}

// rho and rho u of the streamed state at an interior node p (regular pulls):
// rho = sqrt g (1 + sum g~) + A/2, rho u = sqrt g sum g~ c + B/2.
template <class T>
__device__ __forceinline__ void pulled_moments(const T* __restrict__ pop, const T* __restrict__ hist,
                                               const T* __restrict__ geo, const Grid& g, const Pos& p, T& r,
                                               T j[3]) {
  T s = 0, j0 = 0, j1 = 0, j2 = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    const T v = pull<T, l>(pop, g, p);
    s += v;
    if (cx(l)) j0 += T(cx(l)) * v;
    if (cy(l)) j1 += T(cy(l)) * v;
    if (cz(l)) j2 += T(cz(l)) * v;
  });
  const T sg = T(1) + geo[G_SG * g.N + p.n];
  r = sg * (T(1) + s) + T(0.5) * hist[H_A * g.N + p.n];
  j[0] = sg * j0 + T(0.5) * hist[(H_B + 0) * g.N + p.n];
  j[1] = sg * j1 + T(0.5) * hist[(H_B + 1) * g.N + p.n];
  j[2] = sg * j2 + T(0.5) * hist[(H_B + 2) * g.N + p.n];
}

// All 19 streamed deviations g~_l of node p.  Open ends: at the outlet
// (column nx - 1) the values arriving from outside are extrapolated linearly
// from columns nx - 2 and nx - 3; at the inlet (column 0) from columns 1
// and 2, plus the equilibrium difference f^eq(rho_e, j_in) - f^eq(rho_e, j_e)
// at the extrapolated moments (rho_e, j_e), with j_in = rho_e v_in and v_in
// the prescribed inlet velocity in the chart components of the inlet node.
template <class T>
__device__ __forceinline__ void pull_all(const T* __restrict__ pop, const T* __restrict__ hist,
                                         const T* __restrict__ geo, const T* __restrict__ vin, const Grid& g,
                                         const Pos& p, T gv[Q]) {
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    gv[l] = pull<T, l>(pop, g, p);
  });
  if (!g.open) return;
  if (p.i == g.nx - 1) {
    const Pos a = pos_at(g, g.nx - 2, p.jf, p.k), b = pos_at(g, g.nx - 3, p.jf, p.k);
    for_q([&](auto L) {
      constexpr int l = decltype(L)::value;
      if constexpr (cx(l) < 0) gv[l] = T(2) * pull<T, l>(pop, g, a) - pull<T, l>(pop, g, b);
    });
  } else if (p.i == 0) {
    const Pos a = pos_at(g, 1, p.jf, p.k), b = pos_at(g, 2, p.jf, p.k);
    T ra, rb, ja[3], jb[3];
    pulled_moments(pop, hist, geo, g, a, ra, ja);
    pulled_moments(pop, hist, geo, g, b, rb, jb);
    const T re = T(2) * ra - rb;
    const T* v = vin + ((long long)p.k * g.H + p.jf) * 3;
    T je[3], jin[3], da1[3], da2[6];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      je[q] = T(2) * ja[q] - jb[q];
      jin[q] = re * v[q];
      da1[q] = jin[q] - je[q];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int s = q; s < 3; ++s) da2[sym(q, s)] = (jin[q] * jin[s] - je[q] * je[s]) / re;
    const T isg = T(1) / (T(1) + geo[G_SG * g.N + p.n]);
    for_q([&](auto L) {
      constexpr int l = decltype(L)::value;
      if constexpr (cx(l) > 0)
        gv[l] = T(2) * pull<T, l>(pop, g, a) - pull<T, l>(pop, g, b) +
                T(wgt(l)) * isg * hermite_term<T, l>(T(0), da1, da2);
    });
  }
}

}  // namespace lbm
