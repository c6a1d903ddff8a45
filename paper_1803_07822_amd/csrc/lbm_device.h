// Device-side core of the curved-space D3Q19 lattice Boltzmann library:
// lattice constants, grid indexing, the state layout in HBM, and the per-node
// arithmetic of one step (equilibrium, stress, forcing, collision) in
// deviation variables.
//
// Deviation variables keep FP32 accurate: populations are stored as f - w_l,
// sqrt g as sqrt g - 1, g^ij as g^ij - delta^ij.  The same code serves FP64
// (T = double) and FP32 (T = float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ------------------------------------------------------------------ lattice
// D3Q19: 0 rest; 1..6 faces; 7..18 edges; opposite pairs adjacent.
constexpr int Q = 19;
__host__ __device__ constexpr int cx(int l) {
  constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return v[l];
}
__host__ __device__ constexpr int cy(int l) {
  constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return v[l];
}
__host__ __device__ constexpr int cz(int l) {
  constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return v[l];
}
__host__ __device__ constexpr int cc(int l, int a) { return a == 0 ? cx(l) : (a == 1 ? cy(l) : cz(l)); }
__host__ __device__ constexpr double wgt(int l) {
  return l == 0 ? 1.0 / 3.0 : (l <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr int opp(int l) { return l == 0 ? 0 : ((l & 1) ? l + 1 : l - 1); }

// Symmetric 3x3 packing: xx, xy, xz, yy, yz, zz.
__host__ __device__ constexpr int sym(int a, int b) {
  return (a < b ? a : b) == 0 ? (a < b ? b : a) : ((a < b ? a : b) == 1 ? 2 + (a < b ? b : a) : 5);
}

// ------------------------------------------------------------- grid / layout
struct Grid {
  int nx, ny, nz, H;  // H = ny - 2 fluid layers
  long long N;        // fluid nodes
  // Interior plate on the half row between fluid rows pj - 1 and pj over
  // columns pi0..pi1 and every z (pj = 0: none).
  int pj, pi0, pi1;
  // Open ends in x: inlet at column 0, outlet at column nx - 1 (0: periodic).
  int open;
};

// J = dh/dxi at fluid node n from its [9][N] planes.  A chart that moves the
// nodes along y only (Y) has the rows (1, 0, 0) and (0, 0, 1), which are then
// not read.
template <bool Y>
__device__ __forceinline__ void jac_at(const double* __restrict__ jac, long long N, long long n, double J[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = (!Y || a == 1) ? jac[(a * 3 + b) * N + n] : (a == b ? 1.0 : 0.0);
}

// g = J^T J, packed (xx, xy, xz, yy, yz, zz).
__device__ __forceinline__ void metric_of(const double J[3][3], double gq[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) gq[sym(a, b)] = J[0][a] * J[0][b] + J[1][a] * J[1][b] + J[2][a] * J[2][b];
}

// g = J^T J of a chart that moves the nodes along y only, from J's varying
// row r (rows (1, 0, 0) and (0, 0, 1) exact): six products instead of the
// general form's 18 and their sums, which the compiler may not shorten by
// itself (adding a zero product is not a no-op for a signed zero).
__device__ __forceinline__ void metric_of_row(double r0, double r1, double r2, double gq[6]) {
  gq[0] = 1.0 + r0 * r0;
  gq[1] = r0 * r1;
  gq[2] = r0 * r2;
  gq[3] = r1 * r1;
  gq[4] = r1 * r2;
  gq[5] = 1.0 + r2 * r2;
}

// The link from fluid node (i, jf) along (x, y) crosses the plate: it joins
// rows pj - 1 and pj and crosses the half row at i + x/2 within
// [pi0 - 1/2, pi1 + 1/2] on the periodic x axis, where the seam point
// -1/2 = nx - 1/2 belongs to a plate that reaches column 0 or column nx - 1
// (so a link and its reverse are cut alike).  Such links bounce back
// halfway, as at the walls.
__device__ __forceinline__ bool plate_cut(const Grid& g, int i, int jf, int x, int y) {
  if (y == 0 || g.pj == 0) return false;
  if (y > 0 ? jf != g.pj - 1 : jf != g.pj) return false;
  const int s2 = 2 * i + x;
  if (s2 == -1 || s2 == 2 * g.nx - 1) return g.pi0 == 0 || g.pi1 == g.nx - 1;
  return s2 >= 2 * g.pi0 - 1 && s2 <= 2 * g.pi1 + 1;
}

// Geometry field indices in the per-node geometry block (28 planes):
// 0: sqrt g - 1; 1..6: g^ij - delta^ij; 7..24: Gamma^i_jk (i major, jk sym);
// 25..27: F^i.
enum { G_SG = 0, G_GI = 1, G_GAM = 7, G_F = 25, G_N = 28 };
// History coefficients: A, B (3), C (6 sym).
enum { H_A = 0, H_B = 1, H_C = 4, H_N = 10 };

template <class T> struct State {
  T* pop;         // [19][N]  post-collision deviations (pull layout, see step kernel)
  T* hist;        // [10][N]  forcing coefficients of the last step
  const T* geo;   // [28][N]
  T* mom;         // [4][N]   rho - 1, j^x, j^y, j^z of the current state
  const T* uw;    // [2][nz][nx][3] wall velocity, chart components at the adjacent fluid node
  int moving[2];  // wall moves (nonzero velocity somewhere)
};

// ------------------------------------------------------------ node math
template <class T> struct Coef {
  T A, B[3], C[6];
};

// Hermite recomposition to second order (Eq. expansion-equilibrium, App. B):
// (w_l/sqrt g) [a0 + a1.c/c_s^2 + a2:(cc - c_s^2 I)/(2 c_s^4)]
//   = (w_l/sqrt g) [a0 + 3 a1.c + 4.5 a2:cc - 1.5 tr a2].
template <class T, int l>
__device__ __forceinline__ T hermite_term(const T a0, const T a1[3], const T a2[6]) {
  constexpr int x = cx(l), y = cy(l), z = cz(l);
  T s = a0 - T(1.5) * (a2[0] + a2[3] + a2[5]);
  if (x) s += T(3 * x) * a1[0];
  if (y) s += T(3 * y) * a1[1];
  if (z) s += T(3 * z) * a1[2];
  if (x) s += T(4.5) * a2[0];
  if (y) s += T(4.5) * a2[3];
  if (z) s += T(4.5) * a2[5];
  if (x && y) s += T(9.0 * x * y) * a2[1];
  if (x && z) s += T(9.0 * x * z) * a2[2];
  if (y && z) s += T(9.0 * y * z) * a2[4];
  return s;
}

template <class T, int l> struct Unroll {
  template <class F> __device__ __forceinline__ static void run(F&& f) {
    Unroll<T, l - 1>::run(f);
    f(std::integral_constant<int, l - 1>());
  }
};
template <class T> struct Unroll<T, 0> {
  template <class F> __device__ __forceinline__ static void run(F&&) {}
};
template <class F> __device__ __forceinline__ void for_q(F&& f) { Unroll<int, Q>::run(f); }

// Forcing populations F_l from coefficients (Eq. forcing2 with b0 = A,
// b1 = B, b2 = C - c_s^2 delta A), in units of w_l/sqrt g already applied.
template <class T>
__device__ __forceinline__ void forcing_pops(const Coef<T>& c, T isg, T out[Q]) {
  T a2[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) a2[q] = c.C[q];
  a2[0] -= T(1.0 / 3.0) * c.A;
  a2[3] -= T(1.0 / 3.0) * c.A;
  a2[5] -= T(1.0 / 3.0) * c.A;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    out[l] = T(wgt(l)) * isg * hermite_term<T, l>(c.A, c.B, a2);
  });
}

// Geometry of one node, loaded from the SoA planes.
template <class T> struct NodeGeo {
  T sgd;       // sqrt g - 1
  T gid[6];    // g^ij - delta^ij
  T gam[18];   // Gamma^i_jk, [i][sym(j,k)]
  T F[3];
};

template <class T>
__device__ __forceinline__ void load_geo(const T* __restrict__ geo, long long N, long long n, NodeGeo<T>& G) {
  G.sgd = geo[G_SG * N + n];
#pragma unroll
  for (int q = 0; q < 6; ++q) G.gid[q] = geo[(G_GI + q) * N + n];
#pragma unroll
  for (int q = 0; q < 18; ++q) G.gam[q] = geo[(G_GAM + q) * N + n];
#pragma unroll
  for (int q = 0; q < 3; ++q) G.F[q] = geo[(G_F + q) * N + n];
}

template <class T> __device__ __forceinline__ T Gm(const NodeGeo<T>& G, int i, int j, int k) {
  return G.gam[i * 6 + sym(j, k)];
}

// Equilibrium deviations feq_l - w_l for density deviation dr = rho - 1 and
// momentum j (Eq. expansion-equilibrium with a2 = rho theta (g^ij - delta^ij)
// + j j / rho, theta = c_s^2).
template <class T>
__device__ __forceinline__ void equilibrium_dev(const NodeGeo<T>& G, T dr, const T j[3], T out[Q]) {
  const T sg = T(1) + G.sgd;
  const T isg = T(1) / sg;
  const T rho = T(1) + dr;
  const T irho = T(1) / rho;
  T a2[6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) a2[sym(a, b)] = rho * T(1.0 / 3.0) * G.gid[sym(a, b)] + j[a] * j[b] * irho;
  // rho/sqrt g - 1 = (dr - sgd)/sqrt g
  const T a0 = dr - G.sgd;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    out[l] = T(wgt(l)) * isg * hermite_term<T, l>(a0, j, a2);
  });
}

// Non-equilibrium part ne = f - feq and the energy-momentum tensor of
// Eq. (fields3), T = rho theta g^ij + j j / rho + (1 - 1/(2 tau)) sqrt g
// sum_l (f - feq) c c, from the populations' deviations f~ = f - w and the
// node moments (dr = rho - 1, j).
template <class T>
__device__ __forceinline__ void node_stress(const NodeGeo<T>& G, const T ft[Q], T dr, const T j[3], T tau,
                                            T ne[Q], T Tm[6]) {
  const T sg = T(1) + G.sgd;
  const T rho = T(1) + dr;
  const T irho = T(1) / rho;
  T feq[Q];
  equilibrium_dev(G, dr, j, feq);
  T pn[6] = {0, 0, 0, 0, 0, 0};
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    ne[l] = ft[l] - feq[l];
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    if (x) pn[0] += ne[l];
    if (y) pn[3] += ne[l];
    if (z) pn[5] += ne[l];
    if (x && y) pn[1] += T(x * y) * ne[l];
    if (x && z) pn[2] += T(x * z) * ne[l];
    if (y && z) pn[4] += T(y * z) * ne[l];
  });
  const T kneq = (T(1) - T(0.5) / tau) * sg;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      const int q = sym(a, b);
      Tm[q] = rho * T(1.0 / 3.0) * ((a == b ? T(1) : T(0)) + G.gid[q]) + j[a] * j[b] * irho + kneq * pn[q];
    }
}

// Forcing coefficients of Eqs. (forcing-A), (forcing-B), (forcing-C) from
// the momentum j, the stress T and the lattice gradient dj[k][i] = d_k j^i.
template <class T>
__device__ __forceinline__ void forcing_coef(const NodeGeo<T>& G, const T j[3], const T Tm[6], const T dj[3][3],
                                             Coef<T>& c) {
  // tr[b] = Gamma^i_ib
  T tr[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) tr[b] = Gm(G, 0, 0, b) + Gm(G, 1, 1, b) + Gm(G, 2, 2, b);
  // A = -Gamma^i_ij j^j - Gamma^j_ij j^i = -2 tr . j
  c.A = -T(2) * (tr[0] * j[0] + tr[1] * j[1] + tr[2] * j[2]);
  // B^i = -Gamma^k_jk T^ij - Gamma^i_jk T^jk - Gamma^j_jk T^ki + F^i
  //     = -2 tr_j T^ij - Gamma^i_jk T^jk + F^i  (T symmetric)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T s = G.F[i];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      s -= T(2) * tr[jj] * Tm[sym(i, jj)];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) s -= Gm(G, i, jj, kk) * Tm[sym(jj, kk)];
    }
    c.B[i] = s;
  }
  // dbar_k j^i = d_k j^i - Gamma^l_kl j^i ; nab_k j^i = d_k j^i + Gamma^i_kl j^l
  T dbar[3][3], nab[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dbar[k][i] = dj[k][i] - tr[k] * j[i];
      nab[k][i] = dj[k][i] + Gm(G, i, k, 0) * j[0] + Gm(G, i, k, 1) * j[1] + Gm(G, i, k, 2) * j[2];
    }
  const T divbar = dbar[0][0] + dbar[1][1] + dbar[2][2];
  const T divnab = nab[0][0] + nab[1][1] + nab[2][2];
  // C^ij = c_s^2 (dbar_j j^i + dbar_i j^j + delta^ij dbar_k j^k)
  //      - theta (g^jk nab_k j^i + g^ik nab_k j^j + g^ij nab_k j^k),
  // g^ij = delta^ij + gid^ij, theta = c_s^2 = 1/3.
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj) {
      T s = dbar[jj][i] + dbar[i][jj] + (i == jj ? divbar : T(0));
      T t = nab[jj][i] + nab[i][jj] + (i == jj ? divnab : T(0));
#pragma unroll
      for (int k = 0; k < 3; ++k) t += G.gid[sym(jj, k)] * nab[k][i] + G.gid[sym(i, k)] * nab[k][jj];
      t += G.gid[sym(i, jj)] * divnab;
      c.C[sym(i, jj)] = T(1.0 / 3.0) * (s - t);
    }
}

}  // namespace lbm
