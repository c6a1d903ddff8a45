// Oracle for the second-order curved-space D3Q19 lattice Boltzmann method of
// Flouris et al., "Fluid structure interaction with curved space lattice
// Boltzmann" (arXiv 1803.07822).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 CPU statement
// of what the GPU path computes.  Only the tests, the smoke check and the CPU
// baseline leg of the benchmark load it.  It shares no code, header, table or
// helper with the HIP library; the two meet only through seeded input arrays.
//
// Everything is written as node loops in the order the paper gives the steps.
// The scalar type is a template parameter so that the same code, instantiated
// with a dual number, yields exact directional derivatives (forward mode) for
// checking the hand-written adjoint of the GPU path.
//
// Conventions (the paper leaves them open; each is a stated reading):
//   * lattice units dx = dt = 1 (Sec. II), c_s^2 = theta = 1/3.
//   * D3Q19: rest, 6 faces, 12 edges; weights 1/3, 1/18, 1/36 (Sec. II, App. B).
//     Order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = edge pairs
//     (+x+y,-x-y), (+x-y,-x+y), (+x+z,-x-z), (+x-z,-x+z), (+y+z,-y-z),
//     (+y-z,-y+z).  Opposite directions are adjacent (1<->2, 3<->4, ...).
//   * Grid nodes (i,j,k), x fastest; j = 0 and j = ny-1 are solid wall layers,
//     fluid layers are 1..ny-2 (H = ny-2 of them); x and z are periodic.
//   * Fluid arrays are [.][nz][H][nx]; chart arrays are [3][nz][ny][nx].
//   * Forcing history per node: A, B^x, B^y, B^z, C^xx, C^xy, C^xz, C^yy,
//     C^yz, C^zz (Eqs. forcing-A/B/C).
//   * Interior plate (Sec. IV.A.1 (ii), Sec. VI.A): a thin plate on the half
//     row between fluid rows jp-1 and jp, over columns i0..i1 and all z.  A
//     link between those rows is cut when its crossing point x lies in
//     [i0 - 1/2, i1 + 1/2] (periodically); cut links bounce back halfway,
//     like the walls.
//   * Open ends in x (Sec. VI.A), when set: x stops being periodic.  The
//     populations that would stream in from outside are extrapolated from
//     the inner neighbours: at the outlet (last column) the streamed part
//     f - F/2 linearly from the two next columns in; at the inlet (column 0)
//     the same linear extrapolation plus the equilibrium difference for the
//     prescribed inlet velocity, f^eq(rho_e, u_in) - f^eq(rho_e, u_e) at the
//     extrapolated moments (density and non-equilibrium part extrapolated,
//     velocity imposed).  The lattice gradient takes the end
//     column's own momentum beyond each end (zero gradient).
//   * Geometry export per fluid node (28 values): sqrt g, g^xx, g^xy, g^xz,
//     g^yy, g^yz, g^zz, Gamma^i_jk for i = x,y,z and jk in
//     (xx,xy,xz,yy,yz,zz), then F^x, F^y, F^z.

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------- constants
static const int QN = 19;
static const int CV[QN][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W0 = 1.0 / 3.0, W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;
static const double WV[QN] = {W0, W1, W1, W1, W1, W1, W1, W2, W2, W2, W2,
                              W2, W2, W2, W2, W2, W2, W2, W2};
static const double CS2 = 1.0 / 3.0;   // lattice speed of sound squared
static const double THETA = 1.0 / 3.0; // normalised temperature (= c_s^2)

static inline int opposite(int l) { return l == 0 ? 0 : ((l & 1) ? l + 1 : l - 1); }
static inline int wrapi(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

// ---------------------------------------------------------- dual numbers
// Forward-mode dual number: value v and derivative d along one direction.
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
static inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
static inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
static inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
static inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
static inline double val(double x) { return x; }
static inline double val(const Dual& x) { return x.v; }
using std::sqrt;

// ------------------------------------------------------------- 3x3 algebra
template <class T> static T det3(const T m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
         m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}
// Inverse by the adjugate: r = m^{-1}.
template <class T> static void inv3(const T m[3][3], T r[3][3]) {
  T d = det3(m);
  r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / d;
  r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / d;
  r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / d;
  r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / d;
  r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / d;
  r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / d;
  r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / d;
  r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / d;
  r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / d;
}

// --------------------------------------------------------- per-node geometry
// Everything the scheme needs at one fluid node (App. A).
template <class T> struct Geo {
  T J[3][3];       // J[a][i] = d h^a / d xi^i, the basis vectors e_i as columns
  T Ji[3][3];      // inverse of J: Ji[i][a]
  T g[3][3];       // g_ij = e_i . e_j
  T gi[3][3];      // g^ij
  T sg;            // sqrt(det g) = det J
  T Gam[3][3][3];  // Gam[i][j][k] = Gamma^i_jk
  T Fb[3];         // contravariant body force F^i = (J^{-1} F_cart)^i
};

// Scalar field on the y-extended grid, layers j = -3 .. ny+2.
struct Ext {
  int nx, ny, nz, ne;
  Ext(int x, int y, int z) : nx(x), ny(y), nz(z), ne(y + 6) {}
  long at(int i, int j, int k) const {
    return ((long)wrapi(k, nz) * ne + (j + 3)) * nx + wrapi(i, nx);
  }
  long size() const { return (long)nz * ne * nx; }
};

// Second-order isotropic lattice gradient G_i f = (1/c_s^2) sum_l w_l c_l^i f(x+c_l)
// and Laplacian L f = (2/c_s^2) sum_l w_l (f(x+c_l) - f(x))  (App. D).
template <class T>
static T iso_grad(const std::vector<T>& F, const Ext& E, int i, int j, int k, int dir) {
  T s = 0.0;
  for (int l = 1; l < QN; ++l)
    if (CV[l][dir] != 0)
      s += WV[l] * CV[l][dir] * F[E.at(i + CV[l][0], j + CV[l][1], k + CV[l][2])];
  return s / CS2;
}
template <class T>
static T iso_lap(const std::vector<T>& F, const Ext& E, int i, int j, int k) {
  T s = 0.0, c = F[E.at(i, j, k)];
  for (int l = 1; l < QN; ++l)
    s += WV[l] * (F[E.at(i + CV[l][0], j + CV[l][1], k + CV[l][2])] - c);
  return 2.0 * s / CS2;
}

// Geometry of a chart given as node positions chart[3][nz][ny][nx].
// The chart is written h = xi + u with u periodic in x and z; the lattice
// operators are exact on the linear part, so J = I + D u.  In y the
// displacement is continued 3 layers beyond each wall layer by the cubic
// through the 4 nearest layers (exact for the linearly blended charts).
// D is the fourth-order derivative D_i f = G_i[f - (c_s^2/2) L f] (App. D),
// used for J and for the metric derivatives in the Christoffel symbols.
template <class T>
static void compute_geometry(int nx, int ny, int nz, const T* chart, const T Fc[3],
                             std::vector<Geo<T>>& geo) {
  const int H = ny - 2;
  Ext E(nx, ny, nz);
  std::vector<T> u[3], v[3];
  for (int a = 0; a < 3; ++a) {
    u[a].assign(E.size(), T(0.0));
    v[a].assign(E.size(), T(0.0));
  }
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double xi = (a == 0) ? i : (a == 1 ? j : k);
          u[a][E.at(i, j, k)] = chart[(((long)a * nz + k) * ny + j) * nx + i] - xi;
        }
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        for (int j = -1; j >= -3; --j)
          u[a][E.at(i, j, k)] = 4.0 * u[a][E.at(i, j + 1, k)] - 6.0 * u[a][E.at(i, j + 2, k)] +
                                4.0 * u[a][E.at(i, j + 3, k)] - u[a][E.at(i, j + 4, k)];
        for (int j = ny; j <= ny + 2; ++j)
          u[a][E.at(i, j, k)] = 4.0 * u[a][E.at(i, j - 1, k)] - 6.0 * u[a][E.at(i, j - 2, k)] +
                                4.0 * u[a][E.at(i, j - 3, k)] - u[a][E.at(i, j - 4, k)];
      }
  // v = u - (c_s^2/2) L u on layers -2 .. ny+1
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < nz; ++k)
      for (int j = -2; j <= ny + 1; ++j)
        for (int i = 0; i < nx; ++i)
          v[a][E.at(i, j, k)] = u[a][E.at(i, j, k)] - 0.5 * CS2 * iso_lap(u[a], E, i, j, k);
  // J and g on layers -1 .. ny
  std::vector<T> gl[6], wl[6];
  for (int c = 0; c < 6; ++c) {
    gl[c].assign(E.size(), T(0.0));
    wl[c].assign(E.size(), T(0.0));
  }
  static const int PA[6] = {0, 0, 0, 1, 1, 2}, PB[6] = {0, 1, 2, 1, 2, 2};
  std::vector<T> Jf(9 * E.size(), T(0.0));
  for (int k = 0; k < nz; ++k)
    for (int j = -1; j <= ny; ++j)
      for (int i = 0; i < nx; ++i) {
        T J[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            J[a][b] = (a == b ? 1.0 : 0.0) + iso_grad(v[a], E, i, j, k, b);
        for (int c = 0; c < 6; ++c) {
          T s = 0.0;
          for (int a = 0; a < 3; ++a) s += J[a][PA[c]] * J[a][PB[c]];
          gl[c][E.at(i, j, k)] = s;
        }
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) Jf[(a * 3 + b) * E.size() + E.at(i, j, k)] = J[a][b];
      }
  for (int c = 0; c < 6; ++c)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j <= ny - 1; ++j)
        for (int i = 0; i < nx; ++i)
          wl[c][E.at(i, j, k)] = gl[c][E.at(i, j, k)] - 0.5 * CS2 * iso_lap(gl[c], E, i, j, k);
  geo.assign((long)nz * H * nx, Geo<T>());
  for (int k = 0; k < nz; ++k)
    for (int jf = 0; jf < H; ++jf)
      for (int i = 0; i < nx; ++i) {
        const int j = jf + 1;
        Geo<T>& G = geo[((long)k * H + jf) * nx + i];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) G.J[a][b] = Jf[(a * 3 + b) * E.size() + E.at(i, j, k)];
        for (int c = 0; c < 6; ++c) {
          G.g[PA[c]][PB[c]] = gl[c][E.at(i, j, k)];
          G.g[PB[c]][PA[c]] = gl[c][E.at(i, j, k)];
        }
        inv3(G.g, G.gi);
        inv3(G.J, G.Ji);
        G.sg = det3(G.J);
        // dg[l][a][b] = D_l g_ab
        T dg[3][3][3];
        for (int l = 0; l < 3; ++l)
          for (int c = 0; c < 6; ++c) {
            T d = iso_grad(wl[c], E, i, j, k, l);
            dg[l][PA[c]][PB[c]] = d;
            dg[l][PB[c]][PA[c]] = d;
          }
        // Gamma^i_jk = 1/2 g^il (D_j g_kl + D_k g_jl - D_l g_jk)  (App. A)
        for (int ii = 0; ii < 3; ++ii)
          for (int jj = 0; jj < 3; ++jj)
            for (int kk = 0; kk < 3; ++kk) {
              T s = 0.0;
              for (int l = 0; l < 3; ++l)
                s += G.gi[ii][l] * (dg[jj][kk][l] + dg[kk][jj][l] - dg[l][jj][kk]);
              G.Gam[ii][jj][kk] = 0.5 * s;
            }
        for (int ii = 0; ii < 3; ++ii) {
          T s = 0.0;
          for (int a = 0; a < 3; ++a) s += G.Ji[ii][a] * Fc[a];
          G.Fb[ii] = s;
        }
      }
}

// ------------------------------------------------------ Hermite evaluation
// (w_l / sqrt g) [a0 + a1.c/c_s^2 + a2:(c c - c_s^2 I)/(2 c_s^4)], the
// expansion of Eq. (expansion-equilibrium) and Eq. (forcing2) truncated at n = 2.
template <class T>
static T hermite(int l, const T& sg, const T& a0, const T a1[3], const T a2[3][3]) {
  const int* c = CV[l];
  T s1 = a1[0] * (double)c[0] + a1[1] * (double)c[1] + a1[2] * (double)c[2];
  T s2 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      s2 += a2[a][b] * ((double)(c[a] * c[b]) - (a == b ? CS2 : 0.0));
  return WV[l] / sg * (a0 + s1 / CS2 + s2 / (2.0 * CS2 * CS2));
}

// Forcing history coefficients of one node.
template <class T> struct Coef {
  T A, B[3], C[3][3];
};

template <class T> static void coef_load(const std::vector<T>& Fp, long N, long n, Coef<T>& c) {
  c.A = Fp[0 * N + n];
  for (int a = 0; a < 3; ++a) c.B[a] = Fp[(1 + a) * N + n];
  static const int PA[6] = {0, 0, 0, 1, 1, 2}, PB[6] = {0, 1, 2, 1, 2, 2};
  for (int q = 0; q < 6; ++q) {
    c.C[PA[q]][PB[q]] = Fp[(4 + q) * N + n];
    c.C[PB[q]][PA[q]] = Fp[(4 + q) * N + n];
  }
}
template <class T> static void coef_store(std::vector<T>& Fp, long N, long n, const Coef<T>& c) {
  Fp[0 * N + n] = c.A;
  for (int a = 0; a < 3; ++a) Fp[(1 + a) * N + n] = c.B[a];
  static const int PA[6] = {0, 0, 0, 1, 1, 2}, PB[6] = {0, 1, 2, 1, 2, 2};
  for (int q = 0; q < 6; ++q) Fp[(4 + q) * N + n] = c.C[PA[q]][PB[q]];
}

// Forcing term F_l from its coefficients: b0 = A, b1 = B, b2 = C - c_s^2 delta A.
template <class T> static T forcing_pop(int l, const T& sg, const Coef<T>& c) {
  T b2[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) b2[a][b] = c.C[a][b] - (a == b ? CS2 : 0.0) * c.A;
  return hermite(l, sg, c.A, c.B, b2);
}

// Equilibrium (App. B): a0 = rho, a1 = rho u, a2 = rho(theta g^ij - c_s^2 delta) + rho u u.
template <class T>
static void equilibrium(const Geo<T>& G, const T& rho, const T j[3], T feq[QN]) {
  T a2[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      a2[a][b] = rho * (THETA * G.gi[a][b] - (a == b ? CS2 : 0.0)) + j[a] * j[b] / rho;
  for (int l = 0; l < QN; ++l) feq[l] = hermite(l, G.sg, rho, j, a2);
}

// Energy-momentum tensor, Eq. (fields3):
//   T = Pi_eq + (1 - 1/(2 tau)) sqrt g sum_l (f_l - feq_l) c c.
template <class T>
static void stress(const Geo<T>& G, const T f[QN], const T feq[QN], const T& rho, const T j[3],
                   const T& tau, T Tm[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      T s = 0.0;
      for (int l = 0; l < QN; ++l)
        if (CV[l][a] * CV[l][b] != 0) s += (f[l] - feq[l]) * (double)(CV[l][a] * CV[l][b]);
      Tm[a][b] = rho * THETA * G.gi[a][b] + j[a] * j[b] / rho + (1.0 - 0.5 / tau) * G.sg * s;
    }
}

// Forcing coefficients, Eqs. (forcing-A), (forcing-B), (forcing-C).
// dj[k][i] = d_k (rho u^i).
template <class T>
static void forcing_coefficients(const Geo<T>& G, const T j[3], const T Tm[3][3],
                                 const T dj[3][3], Coef<T>& c) {
  T tr[3];  // tr[j] = Gamma^i_ij
  for (int b = 0; b < 3; ++b) tr[b] = G.Gam[0][0][b] + G.Gam[1][1][b] + G.Gam[2][2][b];
  // A = -Gamma^i_ij rho u^j - Gamma^j_ij rho u^i
  T A = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A -= G.Gam[a][a][b] * j[b] + G.Gam[b][a][b] * j[a];
  c.A = A;
  // B^i = -Gamma^k_jk T^ij - Gamma^i_jk T^jk - Gamma^j_jk T^ki + F^i
  for (int i = 0; i < 3; ++i) {
    T s = G.Fb[i];
    for (int jj = 0; jj < 3; ++jj)
      for (int kk = 0; kk < 3; ++kk)
        s -= G.Gam[kk][jj][kk] * Tm[i][jj] + G.Gam[i][jj][kk] * Tm[jj][kk] +
             G.Gam[jj][jj][kk] * Tm[kk][i];
    c.B[i] = s;
  }
  // dbar_k (rho u^i) = d_k (rho u^i) - Gamma^l_kl rho u^i
  // nabla_k (rho u^i) = d_k (rho u^i) + Gamma^i_kl rho u^l
  T dbar[3][3], nab[3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) {
      dbar[k][i] = dj[k][i] - tr[k] * j[i];
      T s = dj[k][i];
      for (int l = 0; l < 3; ++l) s += G.Gam[i][k][l] * j[l];
      nab[k][i] = s;
    }
  T divbar = dbar[0][0] + dbar[1][1] + dbar[2][2];
  T divnab = nab[0][0] + nab[1][1] + nab[2][2];
  for (int i = 0; i < 3; ++i)
    for (int jj = 0; jj < 3; ++jj) {
      T s = CS2 * (dbar[jj][i] + dbar[i][jj] + (i == jj ? divbar : T(0.0)));
      T t = G.gi[i][jj] * divnab;
      for (int k = 0; k < 3; ++k) t += G.gi[jj][k] * nab[k][i] + G.gi[i][k] * nab[k][jj];
      c.C[i][jj] = s - THETA * t;
    }
}

// ------------------------------------------------------------------ solver
template <class T> struct Sim {
  int nx, ny, nz, H;
  long N;  // fluid nodes
  T tau;
  T Fc[3];                          // Cartesian body-force density
  std::vector<T> chart;             // [3][nz][ny][nx]
  std::vector<Geo<T>> geo;          // per fluid node
  std::vector<T> f;                 // [19][N]: state f_l(x,t) as in Eq. (streaming)
  std::vector<T> Fp;                // [10][N]: coefficients of F(x, t-1)
  std::vector<T> disp[2];           // wall displacements [nz][nx] (bottom, top)
  std::vector<T> vwall[2];          // Cartesian wall velocity [nz][nx][3]
  std::vector<T> uwall[2];          // chart components at the adjacent fluid node
  int pj = 0, pi0 = 0, pi1 = -1;    // interior plate (pj = 0: none)
  bool open_x = false;              // open ends in x (inlet at column 0, outlet at nx-1)
  std::vector<T> uin;               // Cartesian inlet velocity [nz][H][3]
  std::vector<T> dplate;            // plate y-displacement [nz][nx] (cross-section row)
  std::vector<T> vplate;            // Cartesian plate velocity per column [nz][nx][3]
  std::vector<T> uplate[2];         // chart components at the node below (0) / above (1)
  bool have_geo = false, have_state = false;
  // Diagnostic ablation (tests only): drop the velocity-gradient coefficient
  // C^ij of Eq. (forcing-C) from every forcing term.  Not part of the method.
  bool drop_C = false;
  void ablate(Coef<T>& c) const {
    if (!drop_C) return;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) c.C[a][b] = T(0.0);
  }

  Sim(int x, int y, int z, double t) : nx(x), ny(y), nz(z), H(y - 2), tau(t) {
    N = (long)nz * H * nx;
    Fc[0] = Fc[1] = Fc[2] = 0.0;
    for (int w = 0; w < 2; ++w) {
      disp[w].assign((long)nz * nx, T(0.0));
      vwall[w].assign((long)nz * nx * 3, T(0.0));
      uwall[w].assign((long)nz * nx * 3, T(0.0));
      uplate[w].assign((long)nz * nx * 3, T(0.0));
    }
    dplate.assign((long)nz * nx, T(0.0));
    vplate.assign((long)nz * nx * 3, T(0.0));
  }

  // The link from fluid node (i, jf) along (cx, cy) crosses the plate: it
  // joins rows jp-1 and jp and crosses the half row at x = i + cx/2 within
  // [i0 - 1/2, i1 + 1/2] on the periodic x axis.  The seam point
  // x = -1/2 = nx - 1/2 lies on the plate when the plate reaches column 0 or
  // column nx - 1; a link and its reverse are then cut alike.
  bool plate_cut(int i, int jf, int cx, int cy) const {
    if (pj == 0 || cy == 0) return false;
    if (cy > 0 ? jf != pj - 1 : jf != pj) return false;
    const int s2 = 2 * i + cx;
    if (s2 == -1 || s2 == 2 * nx - 1) return pi0 == 0 || pi1 == nx - 1;
    return s2 >= 2 * pi0 - 1 && s2 <= 2 * pi1 + 1;
  }
  long nid(int i, int jf, int k) const { return ((long)k * H + jf) * nx + i; }
  // Column of a neighbour in x: periodic, or with open ends the end column
  // itself beyond each end.
  int colx(int i) const { return open_x ? (i < 0 ? 0 : (i > nx - 1 ? nx - 1 : i)) : wrapi(i, nx); }

  void update_wall_velocity() {
    for (int w = 0; w < 2; ++w)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
          const Geo<T>& G = geo[nid(i, w == 0 ? 0 : H - 1, k)];
          for (int a = 0; a < 3; ++a) {
            T s = 0.0;
            for (int b = 0; b < 3; ++b) s += G.Ji[a][b] * vwall[w][((long)k * nx + i) * 3 + b];
            uwall[w][((long)k * nx + i) * 3 + a] = s;
          }
        }
  }

  // Plate velocity in the chart components of the nodes next to the plate:
  // column i takes the velocity of the nearest plate column.
  void update_plate_velocity() {
    if (pj == 0) return;
    for (int s = 0; s < 2; ++s)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
          const Geo<T>& G = geo[nid(i, pj - 1 + s, k)];
          const int ic = i < pi0 ? pi0 : (i > pi1 ? pi1 : i);
          for (int a = 0; a < 3; ++a) {
            T v = 0.0;
            for (int b = 0; b < 3; ++b) v += G.Ji[a][b] * vplate[((long)k * nx + ic) * 3 + b];
            uplate[s][((long)k * nx + i) * 3 + a] = v;
          }
        }
  }

  // Open ends in x with the Cartesian inlet velocity u_in [nz][H][3]
  // (nullptr: periodic x again).
  bool set_open_x(const T* u) {
    if (!u) {
      open_x = false;
      return true;
    }
    if (nx < 4 || (pj > 0 && (pi0 < 3 || pi1 > nx - 4))) return false;
    open_x = true;
    uin.assign(u, u + (long)nz * H * 3);
    return true;
  }

  // The open-end rule on a state fv whose forcing history is Fp: the
  // populations arriving from outside at the two end columns are derived
  // from the inner neighbours (see the header).
  void apply_open_ends(std::vector<T>& fv) const {
    if (!open_x) return;
    // g~ = f - F/2, the part carried by streaming
    auto gs = [&](int l, long n) {
      Coef<T> c;
      coef_load(Fp, N, n, c);
      return fv[l * N + n] - 0.5 * forcing_pop(l, geo[n].sg, c);
    };
    auto half_f = [&](int l, long n) {
      Coef<T> c;
      coef_load(Fp, N, n, c);
      return 0.5 * forcing_pop(l, geo[n].sg, c);
    };
    for (int k = 0; k < nz; ++k)
      for (int jf = 0; jf < H; ++jf) {
        // outlet: g~ extrapolated linearly from columns nx-2 and nx-3
        {
          const long nb = nid(nx - 1, jf, k), n1 = nid(nx - 2, jf, k), n2 = nid(nx - 3, jf, k);
          for (int l = 0; l < QN; ++l)
            if (CV[l][0] < 0) fv[l * N + nb] = 2.0 * gs(l, n1) - gs(l, n2) + half_f(l, nb);
        }
        // inlet: g~ extrapolated linearly from columns 1 and 2, plus
        // f^eq(rho_e, u_in) - f^eq(rho_e, u_e) at the extrapolated moments
        {
          const long n0 = nid(0, jf, k), n1 = nid(1, jf, k), n2 = nid(2, jf, k);
          T re = 0.0, je[3] = {0.0, 0.0, 0.0};
          for (int q = 0; q < 2; ++q) {
            const long n = q == 0 ? n1 : n2;
            const double wq = q == 0 ? 2.0 : -1.0;
            T r = 0.0, jv[3] = {0.0, 0.0, 0.0};
            for (int l = 0; l < QN; ++l) {
              const T fl = fv[l * N + n];
              r += fl;
              for (int a = 0; a < 3; ++a)
                if (CV[l][a]) jv[a] += fl * (double)CV[l][a];
            }
            re += wq * geo[n].sg * r;
            for (int a = 0; a < 3; ++a) je[a] += wq * geo[n].sg * jv[a];
          }
          T jin[3];
          for (int a = 0; a < 3; ++a) {
            T v = 0.0;
            for (int b = 0; b < 3; ++b) v += geo[n0].Ji[a][b] * uin[((long)k * H + jf) * 3 + b];
            jin[a] = re * v;
          }
          T da1[3], da2[3][3];
          for (int a = 0; a < 3; ++a) da1[a] = jin[a] - je[a];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) da2[a][b] = (jin[a] * jin[b] - je[a] * je[b]) / re;
          for (int l = 0; l < QN; ++l)
            if (CV[l][0] > 0)
              fv[l * N + n0] = 2.0 * gs(l, n1) - gs(l, n2) + half_f(l, n0) + hermite(l, geo[n0].sg, T(0.0), da1, da2);
        }
      }
  }

  void set_body_force(const double F[3]) {
    for (int a = 0; a < 3; ++a) Fc[a] = F[a];
    if (have_geo)
      for (long n = 0; n < N; ++n)
        for (int i = 0; i < 3; ++i) {
          T s = 0.0;
          for (int a = 0; a < 3; ++a) s += geo[n].Ji[i][a] * Fc[a];
          geo[n].Fb[i] = s;
        }
  }

  void set_metric(const T* ch, bool reproject) {
    std::vector<T> newchart(ch, ch + 3L * nz * ny * nx);
    std::vector<Geo<T>> newgeo;
    compute_geometry(nx, ny, nz, newchart.data(), Fc, newgeo);
    const bool moved = reproject && have_state && have_geo;
    if (moved) reproject_state(newchart, newgeo);
    chart.swap(newchart);
    geo.swap(newgeo);
    have_geo = true;
    update_wall_velocity();
    update_plate_velocity();
    // the re-projected state lives on the new chart: its open-end
    // populations are derived with the new geometry
    if (moved) apply_open_ends(f);
  }

  // Linear blending of the two wall displacements into the interior
  // (Sec. IV.A.1 (i)): h = (xi_x, xi_y + (1 - eta/H) d_bot + (eta/H) d_top, xi_z),
  // eta = xi_y - 1/2, so the halfway walls sit at eta = 0 and eta = H.
  void set_wall_displacement(int wall, const T* d, bool reproject) {
    for (long q = 0; q < (long)nz * nx; ++q) disp[wall][q] = d ? d[q] : T(0.0);
    build_chart(reproject);
  }

  // Natural cubic spline along the normal of the plate (Sec. IV.A.1 (ii)):
  // the shape S(eta) through (0, 0), (eta_p, 1), (H, 0) with S'' = 0 at both
  // walls.  With knot spacings a = eta_p and b = H - eta_p, continuity of S'
  // at the plate gives its second derivative there, M = -3 (1/a + 1/b) / H;
  // each piece is the cubic with end values and end second derivatives.
  double plate_shape(double eta) const {
    const double a = pj, b = H - pj, M = -3.0 * (1.0 / a + 1.0 / b) / H;
    if (eta <= a) {
      const double t = eta;  // distance from the bottom wall
      return M * t * t * t / (6.0 * a) + (1.0 - M * a * a / 6.0) * t / a;
    }
    const double t = H - eta;  // distance from the top wall
    return M * t * t * t / (6.0 * b) + (1.0 - M * b * b / 6.0) * t / b;
  }

  // Chart of the walls and the plate: the two wall displacements blended
  // linearly across the channel (Sec. IV.A.1 (i)) plus the plate's
  // cross-section displacement D(x, z) carried by the spline shape:
  // h = (xi_x, xi_y + (1 - eta/H) d_bot + (eta/H) d_top + D S(eta), xi_z),
  // eta = xi_y - 1/2, so the halfway walls sit at eta = 0 and eta = H and the
  // plate at eta = jp.
  void build_chart(bool reproject) {
    std::vector<T> ch(3L * nz * ny * nx);
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double eta = j - 0.5;
          long q = (long)k * nx + i;
          long p = ((long)k * ny + j) * nx + i;
          ch[0L * nz * ny * nx + p] = (double)i;
          T y = (double)j + (1.0 - eta / H) * disp[0][q] + (eta / H) * disp[1][q];
          if (pj > 0) y += dplate[q] * plate_shape(eta);
          ch[1L * nz * ny * nx + p] = y;
          ch[2L * nz * ny * nx + p] = (double)k;
        }
    set_metric(ch.data(), reproject);
  }

  // Interior plate on the half row between fluid rows jp-1 and jp, columns
  // i0..i1 (the plate's displacement and velocity start at zero).
  bool set_plate(int jp, int i0, int i1) {
    if (jp == 0) {
      pj = 0;
      return true;
    }
    if (jp < 1 || jp > H - 1 || i0 < 0 || i1 < i0 || i1 > nx - 1) return false;
    if (open_x && (i0 < 3 || i1 > nx - 4)) return false;
    pj = jp;
    pi0 = i0;
    pi1 = i1;
    dplate.assign((long)nz * nx, T(0.0));
    vplate.assign((long)nz * nx * 3, T(0.0));
    if (have_geo) update_plate_velocity();
    return true;
  }

  void set_plate_displacement(const T* d, bool reproject) {
    for (long q = 0; q < (long)nz * nx; ++q) dplate[q] = d ? d[q] : T(0.0);
    build_chart(reproject);
  }

  void set_plate_velocity(const T* v) {
    for (long q = 0; q < (long)nz * nx * 3; ++q) vplate[q] = v ? v[q] : T(0.0);
    if (have_geo) update_plate_velocity();
  }

  void set_wall_velocity(int wall, const T* v) {
    for (long q = 0; q < (long)nz * nx * 3; ++q) vwall[wall][q] = v ? v[q] : T(0.0);
    if (have_geo) update_wall_velocity();
  }

  // Fields rho = sqrt g sum f and rho u = sqrt g sum f c (Eqs. fields1-2).
  void moments_raw(std::vector<T>& rho, std::vector<T>& jv) const {
    rho.assign(N, T(0.0));
    jv.assign(3 * N, T(0.0));
    for (long n = 0; n < N; ++n) {
      T s = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
      for (int l = 0; l < QN; ++l) {
        T fl = f[l * N + n];
        s += fl;
        if (CV[l][0]) sx += fl * (double)CV[l][0];
        if (CV[l][1]) sy += fl * (double)CV[l][1];
        if (CV[l][2]) sz += fl * (double)CV[l][2];
      }
      rho[n] = geo[n].sg * s;
      jv[0 * N + n] = geo[n].sg * sx;
      jv[1 * N + n] = geo[n].sg * sy;
      jv[2 * N + n] = geo[n].sg * sz;
    }
  }

  // rho u at grid node (i, j, k) with j in 0..ny-1; the wall layers carry the
  // mirror ghost j_g = 2 rho_m u_w - j_m of the adjacent fluid node m.
  T jat(const std::vector<T>& rho, const std::vector<T>& jv, int i, int j, int k, int a) const {
    i = colx(i);
    k = wrapi(k, nz);
    if (j >= 1 && j <= ny - 2) return jv[a * N + nid(i, j - 1, k)];
    int w = (j <= 0) ? 0 : 1;
    long m = nid(i, w == 0 ? 0 : H - 1, k);
    return 2.0 * rho[m] * uwall[w][((long)k * nx + i) * 3 + a] - jv[a * N + m];
  }

  // Forcing coefficients of the current state at every node; optional outputs
  // of the per-node intermediate quantities used by the collision.
  void forcing_all(const std::vector<T>& rho, const std::vector<T>& jv, std::vector<T>& coef) const {
    coef.assign(10 * N, T(0.0));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int jf = 0; jf < H; ++jf)
        for (int i = 0; i < nx; ++i) {
          long n = nid(i, jf, k);
          const Geo<T>& G = geo[n];
          T fl[QN], feq[QN], jl[3], Tm[3][3], dj[3][3];
          for (int l = 0; l < QN; ++l) fl[l] = f[l * N + n];
          for (int a = 0; a < 3; ++a) jl[a] = jv[a * N + n];
          equilibrium(G, rho[n], jl, feq);
          stress(G, fl, feq, rho[n], jl, tau, Tm);
          node_gradient(rho, jv, i, jf + 1, k, dj);
          Coef<T> c;
          forcing_coefficients(G, jl, Tm, dj, c);
          ablate(c);
          coef_store(coef, N, n, c);
        }
  }

  // d_k (rho u^i) by the second-order isotropic gradient (App. D).
  // A neighbour across the plate is replaced by the mirror ghost of the node
  // m on this side in the neighbour's column, j_g = 2 rho_m u_p - j_m, as at
  // the walls.
  void node_gradient(const std::vector<T>& rho, const std::vector<T>& jv, int i, int j, int k,
                     T dj[3][3]) const {
    for (int kk = 0; kk < 3; ++kk)
      for (int a = 0; a < 3; ++a) {
        T s = 0.0;
        for (int l = 1; l < QN; ++l)
          if (CV[l][kk] != 0) {
            T jn;
            if (plate_cut(i, j - 1, CV[l][0], CV[l][1])) {
              const int im = colx(i + CV[l][0]), km = wrapi(k + CV[l][2], nz);
              const long m = nid(im, j - 1, km);
              const int side = (j - 1 == pj) ? 1 : 0;
              jn = 2.0 * rho[m] * uplate[side][((long)km * nx + im) * 3 + a] - jv[a * N + m];
            } else {
              jn = jat(rho, jv, i + CV[l][0], j + CV[l][1], k + CV[l][2], a);
            }
            s += WV[l] * (double)CV[l][kk] * jn;
          }
        dj[kk][a] = s / CS2;
      }
  }

  // Initial state: f = f_eq(rho0, u0) with u0 = J^{-1} u_cart, and the
  // forcing history set to the forcing of that state, F(x, -1) := F(x, 0).
  void init_equilibrium(const T* rho0, const T* ucart) {
    f.assign(QN * N, T(0.0));
    for (long n = 0; n < N; ++n) {
      const Geo<T>& G = geo[n];
      T r = rho0 ? rho0[n] : T(1.0);
      T uc[3], j[3], feq[QN];
      for (int a = 0; a < 3; ++a) uc[a] = ucart ? ucart[a * N + n] : T(0.0);
      for (int a = 0; a < 3; ++a) {
        T s = 0.0;
        for (int b = 0; b < 3; ++b) s += G.Ji[a][b] * uc[b];
        j[a] = r * s;
      }
      equilibrium(G, r, j, feq);
      for (int l = 0; l < QN; ++l) f[l * N + n] = feq[l];
    }
    reset_history();
    apply_open_ends(f);
    have_state = true;
  }

  // The history is formed from the state as given; with open ends the
  // populations arriving from outside are then derived from it.
  void set_populations(const T* fin) {
    f.assign(fin, fin + QN * N);
    reset_history();
    apply_open_ends(f);
    have_state = true;
  }

  void reset_history() {
    std::vector<T> rho, jv;
    moments_raw(rho, jv);
    forcing_all(rho, jv, Fp);
  }

  // One time step: collision Eq. (collision) with the leading f_l restored,
  //   f* = f - (f - f_eq)/tau + F(t) - F(t-1)/2,
  // then streaming Eq. (streaming), f(x+c, t+1) = f*(x, t) + F(x+c, t)/2,
  // with halfway bounce-back (moving-wall term) at the solid layers.
  void step() {
    std::vector<T> rho, jv;
    moments_raw(rho, jv);
    std::vector<T> fs(QN * N), Fl(QN * N), coef(10 * N);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int jf = 0; jf < H; ++jf)
        for (int i = 0; i < nx; ++i) {
          long n = nid(i, jf, k);
          const Geo<T>& G = geo[n];
          T fl[QN], feq[QN], jl[3], Tm[3][3], dj[3][3];
          for (int l = 0; l < QN; ++l) fl[l] = f[l * N + n];
          for (int a = 0; a < 3; ++a) jl[a] = jv[a * N + n];
          equilibrium(G, rho[n], jl, feq);
          stress(G, fl, feq, rho[n], jl, tau, Tm);
          node_gradient(rho, jv, i, jf + 1, k, dj);
          Coef<T> c, cp;
          forcing_coefficients(G, jl, Tm, dj, c);
          ablate(c);
          coef_store(coef, N, n, c);
          coef_load(Fp, N, n, cp);
          for (int l = 0; l < QN; ++l) {
            T Fn = forcing_pop(l, G.sg, c);
            T Fo = forcing_pop(l, G.sg, cp);
            Fl[l * N + n] = Fn;
            fs[l * N + n] = fl[l] - (fl[l] - feq[l]) / tau + Fn - 0.5 * Fo;
          }
        }
    std::vector<T> fn(QN * N, T(0.0));
    for (int k = 0; k < nz; ++k)
      for (int jf = 0; jf < H; ++jf)
        for (int i = 0; i < nx; ++i) {
          long n = nid(i, jf, k);
          for (int l = 0; l < QN; ++l) {
            int jd = jf + 1 + CV[l][1];
            const bool cut = plate_cut(i, jf, CV[l][0], CV[l][1]);
            if (jd >= 1 && jd <= ny - 2 && !cut) {
              const int id = i + CV[l][0];
              if (open_x && (id < 0 || id > nx - 1)) continue;  // leaves through an open end
              long d = nid(wrapi(id, nx), jd - 1, wrapi(k + CV[l][2], nz));
              fn[l * N + d] = fs[l * N + n];
            } else {
              int w = (jd <= 0) ? 0 : 1;
              const T* uw = cut ? &uplate[jf == pj ? 1 : 0][((long)k * nx + i) * 3]
                                : &uwall[w][((long)k * nx + i) * 3];
              T cu = uw[0] * (double)CV[l][0] + uw[1] * (double)CV[l][1] + uw[2] * (double)CV[l][2];
              fn[opposite(l) * N + n] = fs[l * N + n] - 2.0 * WV[l] / geo[n].sg * rho[n] * cu / CS2;
            }
          }
        }
    for (long q = 0; q < QN * N; ++q) fn[q] += 0.5 * Fl[q];
    f.swap(fn);
    Fp.swap(coef);
    apply_open_ends(f);
  }

  // Moments output: rho and u (chart components, or Cartesian u_c = J u).
  void moments(T* rho_out, T* u_out, bool cartesian) const {
    std::vector<T> rho, jv;
    moments_raw(rho, jv);
    for (long n = 0; n < N; ++n) {
      T u[3];
      for (int a = 0; a < 3; ++a) u[a] = jv[a * N + n] / rho[n];
      if (rho_out) rho_out[n] = rho[n];
      if (u_out)
        for (int a = 0; a < 3; ++a) {
          if (cartesian) {
            T s = 0.0;
            for (int b = 0; b < 3; ++b) s += geo[n].J[a][b] * u[b];
            u_out[a * N + n] = s;
          } else {
            u_out[a * N + n] = u[a];
          }
        }
    }
  }

  // Momentum-exchange force on a wall at rest (a diagnostic beside the
  // node-exact traction): every population that streamed into the wall in the
  // last step came back reversed, handing the wall 2 f*_l c_l, with f* the
  // post-collision value.  f* is recovered from the streamed state: the
  // reversed population is f_opp(l) = f*_l + F_opp(l)/2 (the half force added
  // at streaming, from the history).  Cartesian force sqrt g J c_l per link,
  // summed per column.  Returns false for a moving wall.
  bool wall_force_mem(int wall, T total[3], T* per_node) const {
    for (long q = 0; q < (long)nz * nx * 3; ++q)
      if (val(vwall[wall][q]) != 0.0) return false;
    total[0] = total[1] = total[2] = 0.0;
    const int jf = (wall == 0) ? 0 : H - 1;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        const long n = nid(i, jf, k);
        const Geo<T>& G = geo[n];
        Coef<T> c;
        coef_load(Fp, N, n, c);
        T col[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < QN; ++l) {
          const int cy = CV[l][1];
          if (!((wall == 1 && cy > 0) || (wall == 0 && cy < 0))) continue;  // links into this wall
          const int o = opposite(l);
          const T fstar = f[o * N + n] - 0.5 * forcing_pop(o, G.sg, c);
          for (int a = 0; a < 3; ++a) {
            T v = 0.0;
            for (int b = 0; b < 3; ++b) v += G.J[a][b] * (double)CV[l][b];
            col[a] += 2.0 * G.sg * fstar * v;
          }
        }
        for (int a = 0; a < 3; ++a) {
          total[a] += col[a];
          if (per_node) per_node[((long)k * nx + i) * 3 + a] = col[a];
        }
      }
    return true;
  }

  // Node-exact wall traction (Sec. IV.A.2): at the fluid layer next to the
  // wall, the Cartesian force sqrt g T^{i y} e_i per column; n dA = sqrt g e^y.
  // The bottom wall's outward normal points to -y, hence the sign.
  void wall_force(int wall, T total[3], T* per_node) const {
    std::vector<T> rho, jv;
    moments_raw(rho, jv);
    total[0] = total[1] = total[2] = 0.0;
    const int jf = (wall == 0) ? 0 : H - 1;
    const double sgn = (wall == 0) ? -1.0 : 1.0;
    for (int k = 0; k < nz; ++k)
      for (int i = 0; i < nx; ++i) {
        long n = nid(i, jf, k);
        const Geo<T>& G = geo[n];
        T fl[QN], feq[QN], jl[3], Tm[3][3];
        for (int l = 0; l < QN; ++l) fl[l] = f[l * N + n];
        for (int a = 0; a < 3; ++a) jl[a] = jv[a * N + n];
        equilibrium(G, rho[n], jl, feq);
        stress(G, fl, feq, rho[n], jl, tau, Tm);
        for (int a = 0; a < 3; ++a) {
          T s = 0.0;
          for (int i2 = 0; i2 < 3; ++i2) s += G.sg * Tm[i2][1] * G.J[a][i2];
          s = sgn * s;
          total[a] += s;
          if (per_node) per_node[((long)k * nx + i) * 3 + a] = s;
        }
      }
  }

  // Force on the plate: the node-exact traction of both faces over the plate
  // columns, + sqrt g T^{iy} J e_i at the node below (whose outward normal is
  // +y) and - sqrt g T^{iy} J e_i at the node above.  per_col [nz][nx][3] is
  // zero outside i0..i1.
  void plate_force(T total[3], T* per_col) const {
    std::vector<T> rho, jv;
    moments_raw(rho, jv);
    total[0] = total[1] = total[2] = 0.0;
    if (per_col)
      for (long q = 0; q < (long)nz * nx * 3; ++q) per_col[q] = 0.0;
    if (pj == 0) return;
    for (int k = 0; k < nz; ++k)
      for (int i = pi0; i <= pi1; ++i) {
        T col[3] = {0.0, 0.0, 0.0};
        for (int s = 0; s < 2; ++s) {
          long n = nid(i, pj - 1 + s, k);
          const Geo<T>& G = geo[n];
          T fl[QN], feq[QN], jl[3], Tm[3][3];
          for (int l = 0; l < QN; ++l) fl[l] = f[l * N + n];
          for (int a = 0; a < 3; ++a) jl[a] = jv[a * N + n];
          equilibrium(G, rho[n], jl, feq);
          stress(G, fl, feq, rho[n], jl, tau, Tm);
          const double sgn = s == 0 ? 1.0 : -1.0;
          for (int a = 0; a < 3; ++a) {
            T v = 0.0;
            for (int i2 = 0; i2 < 3; ++i2) v += G.sg * Tm[i2][1] * G.J[a][i2];
            col[a] += sgn * v;
          }
        }
        for (int a = 0; a < 3; ++a) {
          total[a] += col[a];
          if (per_col) per_col[((long)k * nx + i) * 3 + a] = col[a];
        }
      }
  }

  // --------------------------------------------------------- re-projection
  // Old chart displacement on the y-extended grid (same continuation as the
  // geometry), used to locate psi(x~) = h^{-1}(h~(x~)).
  void extended_displacement(const std::vector<T>& ch, std::vector<double> u[3], Ext& E) const {
    for (int a = 0; a < 3; ++a) u[a].assign(E.size(), 0.0);
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            double xi = (a == 0) ? i : (a == 1 ? j : k);
            u[a][E.at(i, j, k)] = val(ch[(((long)a * nz + k) * ny + j) * nx + i]) - xi;
          }
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
          for (int j = -1; j >= -3; --j)
            u[a][E.at(i, j, k)] = 4.0 * u[a][E.at(i, j + 1, k)] - 6.0 * u[a][E.at(i, j + 2, k)] +
                                  4.0 * u[a][E.at(i, j + 3, k)] - u[a][E.at(i, j + 4, k)];
          for (int j = ny; j <= ny + 2; ++j)
            u[a][E.at(i, j, k)] = 4.0 * u[a][E.at(i, j - 1, k)] - 6.0 * u[a][E.at(i, j - 2, k)] +
                                  4.0 * u[a][E.at(i, j - 3, k)] - u[a][E.at(i, j - 4, k)];
        }
  }

  // Trilinear interpolation of an extended-grid field and its gradient at xi.
  // With side >= 0 a cell spanning the plate is moved to that side, as in
  // trilin_clamped, so that the position search and the moment interpolation
  // of a node use the same cell.
  double trilin(const std::vector<double>& F, const Ext& E, const double p[3], double grad[3], int side) const {
    double fl[3];
    int b[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) fl[a] = std::floor(p[a]);
    b[0] = (int)fl[0];
    b[2] = (int)fl[2];
    b[1] = (int)fl[1];
    if (b[1] < -3) b[1] = -3;
    if (b[1] > E.ny + 1) b[1] = E.ny + 1;
    if (side >= 0 && b[1] == pj) {
      const int c0 = wrapi(b[0], nx), c1 = wrapi(b[0] + 1, nx);
      if ((c0 >= pi0 && c0 <= pi1) || (c1 >= pi0 && c1 <= pi1)) b[1] = side ? pj + 1 : pj - 1;
    }
    for (int a = 0; a < 3; ++a) fr[a] = p[a] - b[a];
    double v = 0.0;
    if (grad) grad[0] = grad[1] = grad[2] = 0.0;
    for (int c = 0; c < 8; ++c) {
      int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
      double wx = ox ? fr[0] : 1.0 - fr[0];
      double wy = oy ? fr[1] : 1.0 - fr[1];
      double wz = oz ? fr[2] : 1.0 - fr[2];
      double fv = F[E.at(b[0] + ox, b[1] + oy, b[2] + oz)];
      v += wx * wy * wz * fv;
      if (grad) {
        grad[0] += (ox ? 1.0 : -1.0) * wy * wz * fv;
        grad[1] += wx * (oy ? 1.0 : -1.0) * wz * fv;
        grad[2] += wx * wy * (oz ? 1.0 : -1.0) * fv;
      }
    }
    return v;
  }

  // Re-projection of f and of the forcing history onto a new chart
  // (Sec. IV.B): Hermite moments at the old nodes, pushed to Cartesian
  // components with J, interpolated at psi(x~), pulled back with J~^{-1}, and
  // recomposed to second order.  The second moment is moved as the momentum
  // flux Pi = sqrt g sum f c c (a tensor); a2 = Pi - c_s^2 rho I is formed in
  // the new chart.
  void reproject_state(const std::vector<T>& newchart, const std::vector<Geo<T>>& newgeo) {
    // This step is not differentiated; it runs on values only.
    std::vector<T> rho, jv;
    moments_raw(rho, jv);
    // Cartesian fields on the old full grid (layers 0..ny-1, extended storage):
    // 0 rho, 1-3 j_c, 4-9 Pi_c, 10 A, 11-13 B_c, 14-19 C_c.
    const int NF = 20;
    Ext E(nx, ny, nz);
    std::vector<double> fld[NF];
    for (int q = 0; q < NF; ++q) fld[q].assign(E.size(), 0.0);
    static const int PA[6] = {0, 0, 0, 1, 1, 2}, PB[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < nz; ++k)
      for (int jf = 0; jf < H; ++jf)
        for (int i = 0; i < nx; ++i) {
          long n = nid(i, jf, k);
          const Geo<T>& G = geo[n];
          double Pi[3][3], jl[3], J[3][3];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
              double s = 0.0;
              for (int l = 0; l < QN; ++l) s += val(f[l * N + n]) * CV[l][a] * CV[l][b];
              Pi[a][b] = val(G.sg) * s;
              J[a][b] = val(G.J[a][b]);
            }
          for (int a = 0; a < 3; ++a) jl[a] = val(jv[a * N + n]);
          Coef<T> c;
          coef_load(Fp, N, n, c);
          double Bv[3], Cm[3][3];
          for (int a = 0; a < 3; ++a) Bv[a] = val(c.B[a]);
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Cm[a][b] = val(c.C[a][b]);
          long e = E.at(i, jf + 1, k);
          fld[0][e] = val(rho[n]);
          fld[10][e] = val(c.A);
          for (int a = 0; a < 3; ++a) {
            double sj = 0.0, sb = 0.0;
            for (int b = 0; b < 3; ++b) {
              sj += J[a][b] * jl[b];
              sb += J[a][b] * Bv[b];
            }
            fld[1 + a][e] = sj;
            fld[11 + a][e] = sb;
          }
          for (int q = 0; q < 6; ++q) {
            int a = PA[q], b = PB[q];
            double sp = 0.0, sc = 0.0;
            for (int p = 0; p < 3; ++p)
              for (int r = 0; r < 3; ++r) {
                sp += J[a][p] * Pi[p][r] * J[b][r];
                sc += J[a][p] * Cm[p][r] * J[b][r];
              }
            fld[4 + q][e] = sp;
            fld[14 + q][e] = sc;
          }
        }
    // Ghost layers: momentum by the mirror rule about rho v_w (so that linear
    // interpolation gives the wall momentum at the halfway wall), the other
    // moments by linear extrapolation from the two nearest fluid layers.
    for (int w = 0; w < 2; ++w)
      for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
          long eg = E.at(i, w == 0 ? 0 : ny - 1, k);
          long em = E.at(i, w == 0 ? 1 : ny - 2, k);
          long em2 = E.at(i, w == 0 ? 2 : ny - 3, k);
          for (int q = 0; q < NF; ++q) fld[q][eg] = 2.0 * fld[q][em] - fld[q][em2];
          for (int a = 0; a < 3; ++a)
            fld[1 + a][eg] = 2.0 * fld[0][em] * val(vwall[w][((long)k * nx + i) * 3 + a]) - fld[1 + a][em];
        }
    std::vector<double> uo[3];
    extended_displacement(chart, uo, E);
    std::vector<T> fnew(QN * N), Fnew(10 * N);
    for (int k = 0; k < nz; ++k)
      for (int jf = 0; jf < H; ++jf)
        for (int i = 0; i < nx; ++i) {
          long n = nid(i, jf, k);
          long p3 = ((long)k * ny + (jf + 1)) * nx + i, plane = (long)nz * ny * nx;
          double p[3] = {val(newchart[p3]), val(newchart[plane + p3]), val(newchart[2 * plane + p3])};
          // psi: solve xi + u_old(xi) = p by Newton on the trilinear interpolant
          // (cells on the node's side of the plate)
          const int side = (pj > 0) ? (jf >= pj ? 1 : 0) : -1;
          double xi[3] = {(double)i, (double)(jf + 1), (double)k};
          for (int it = 0; it < 50; ++it) {
            double r[3], Jm[3][3], Jinv[3][3];
            for (int a = 0; a < 3; ++a) {
              double gr[3];
              r[a] = xi[a] + trilin(uo[a], E, xi, gr, side) - p[a];
              for (int b = 0; b < 3; ++b) Jm[a][b] = (a == b ? 1.0 : 0.0) + gr[b];
            }
            inv3(Jm, Jinv);
            double dmax = 0.0;
            for (int a = 0; a < 3; ++a) {
              double d = Jinv[a][0] * r[0] + Jinv[a][1] * r[1] + Jinv[a][2] * r[2];
              xi[a] -= d;
              dmax = std::fmax(dmax, std::fabs(d));
            }
            if (dmax <= 1e-13 * (1.0 + std::fabs(xi[0]) + std::fabs(xi[1]) + std::fabs(xi[2]))) break;
          }
          // Interpolation inside the old moment grid, layers 0..ny-1.
          double q[3] = {xi[0], xi[1], xi[2]};
          if (q[1] < 0.0) q[1] = 0.0;
          if (q[1] > ny - 1.0) q[1] = ny - 1.0;
          double m[NF];
          for (int c = 0; c < NF; ++c) m[c] = trilin_clamped(fld[c], E, q, side);
          const Geo<T>& Gn = newgeo[n];
          double Ji[3][3];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Ji[a][b] = val(Gn.Ji[a][b]);
          double jt[3], Bt[3], Pc[3][3], Cc[3][3], Pt[3][3], Ct[3][3];
          for (int qd = 0; qd < 6; ++qd) {
            Pc[PA[qd]][PB[qd]] = Pc[PB[qd]][PA[qd]] = m[4 + qd];
            Cc[PA[qd]][PB[qd]] = Cc[PB[qd]][PA[qd]] = m[14 + qd];
          }
          for (int a = 0; a < 3; ++a) {
            jt[a] = Ji[a][0] * m[1] + Ji[a][1] * m[2] + Ji[a][2] * m[3];
            Bt[a] = Ji[a][0] * m[11] + Ji[a][1] * m[12] + Ji[a][2] * m[13];
          }
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
              double sp = 0.0, sc = 0.0;
              for (int p1 = 0; p1 < 3; ++p1)
                for (int r1 = 0; r1 < 3; ++r1) {
                  sp += Ji[a][p1] * Pc[p1][r1] * Ji[b][r1];
                  sc += Ji[a][p1] * Cc[p1][r1] * Ji[b][r1];
                }
              Pt[a][b] = sp;
              Ct[a][b] = sc;
            }
          T a0 = m[0], a1[3], a2[3][3];
          for (int a = 0; a < 3; ++a) a1[a] = jt[a];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) a2[a][b] = Pt[a][b] - (a == b ? CS2 * m[0] : 0.0);
          for (int l = 0; l < QN; ++l) fnew[l * N + n] = hermite(l, Gn.sg, a0, a1, a2);
          Coef<T> c;
          c.A = m[10];
          for (int a = 0; a < 3; ++a) c.B[a] = Bt[a];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) c.C[a][b] = Ct[a][b];
          coef_store(Fnew, N, n, c);
        }
    f.swap(fnew);
    Fp.swap(Fnew);
  }

  // Trilinear interpolation with x, z periodic and y limited to layers 0..ny-1.
  // A cell that spans the plate (layers jp and jp+1, i.e. fluid rows jp-1 and
  // jp, in a column pair touching a plate column) is moved to the side of
  // the node being built (side 0 below, 1 above): the moments are then
  // extrapolated linearly from that side instead of mixed across the plate.
  double trilin_clamped(const std::vector<double>& F, const Ext& E, const double p[3], int side) const {
    int bx = (int)std::floor(p[0]), bz = (int)std::floor(p[2]);
    int by = (int)std::floor(p[1]);
    if (by > ny - 2) by = ny - 2;
    if (by < 0) by = 0;
    if (side >= 0 && by == pj) {
      const int c0 = wrapi(bx, nx), c1 = wrapi(bx + 1, nx);
      if ((c0 >= pi0 && c0 <= pi1) || (c1 >= pi0 && c1 <= pi1)) by = side ? pj + 1 : pj - 1;
    }
    double fx = p[0] - bx, fy = p[1] - by, fz = p[2] - bz;
    double v = 0.0;
    for (int c = 0; c < 8; ++c) {
      int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
      double w = (ox ? fx : 1.0 - fx) * (oy ? fy : 1.0 - fy) * (oz ? fz : 1.0 - fz);
      v += w * F[E.at(bx + ox, by + oy, bz + oz)];
    }
    return v;
  }

  void geometry_export(double* out) const {
    static const int PA[6] = {0, 0, 0, 1, 1, 2}, PB[6] = {0, 1, 2, 1, 2, 2};
    for (long n = 0; n < N; ++n) {
      const Geo<T>& G = geo[n];
      out[0 * N + n] = val(G.sg);
      for (int q = 0; q < 6; ++q) out[(1 + q) * N + n] = val(G.gi[PA[q]][PB[q]]);
      for (int i = 0; i < 3; ++i)
        for (int q = 0; q < 6; ++q) out[(7 + 6 * i + q) * N + n] = val(G.Gam[i][PA[q]][PB[q]]);
      for (int i = 0; i < 3; ++i) out[(25 + i) * N + n] = val(G.Fb[i]);
    }
  }
  void jacobian_export(double* out) const {
    for (long n = 0; n < N; ++n)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) out[(a * 3 + b) * N + n] = val(geo[n].J[a][b]);
  }
};

}  // namespace orc

// ------------------------------------------------------------------ C API
using orc::Dual;
using orc::Sim;

extern "C" {

// Threads the node loops use (OpenMP over z-planes).
int orc_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads for the following node loops (n >= 1); returns the count in effect.
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

void* orc_create(int nx, int ny, int nz, double tau) {
  if (nx < 1 || nz < 1 || ny < 4 || !(tau > 0.5)) return nullptr;
  return new Sim<double>(nx, ny, nz, tau);
}
void orc_destroy(void* s) { delete (Sim<double>*)s; }
long orc_fluid_nodes(void* s) { return ((Sim<double>*)s)->N; }
void orc_set_body_force(void* s, const double* F) { ((Sim<double>*)s)->set_body_force(F); }
void orc_set_metric(void* s, const double* chart, int reproject) {
  ((Sim<double>*)s)->set_metric(chart, reproject != 0);
}
void orc_set_wall_displacement(void* s, int wall, const double* d, int reproject) {
  ((Sim<double>*)s)->set_wall_displacement(wall, d, reproject != 0);
}
void orc_set_wall_velocity(void* s, int wall, const double* v) {
  ((Sim<double>*)s)->set_wall_velocity(wall, v);
}
void orc_init_equilibrium(void* s, const double* rho, const double* ucart) {
  ((Sim<double>*)s)->init_equilibrium(rho, ucart);
}
void orc_set_populations(void* s, const double* f) { ((Sim<double>*)s)->set_populations(f); }
void orc_get_populations(void* s, double* f) {
  Sim<double>* S = (Sim<double>*)s;
  std::memcpy(f, S->f.data(), sizeof(double) * S->f.size());
}
void orc_get_history(void* s, double* c) {
  Sim<double>* S = (Sim<double>*)s;
  std::memcpy(c, S->Fp.data(), sizeof(double) * S->Fp.size());
}
void orc_step(void* s, int n) {
  for (int t = 0; t < n; ++t) ((Sim<double>*)s)->step();
}
void orc_moments(void* s, double* rho, double* u, int cartesian) {
  ((Sim<double>*)s)->moments(rho, u, cartesian != 0);
}
int orc_wall_force_mem(void* s, int wall, double* total, double* per_node) {
  return ((Sim<double>*)s)->wall_force_mem(wall, total, per_node) ? 0 : -1;
}
void orc_wall_force(void* s, int wall, double* total, double* per_node) {
  ((Sim<double>*)s)->wall_force(wall, total, per_node);
}
int orc_set_plate(void* s, int jp, int i0, int i1) { return ((Sim<double>*)s)->set_plate(jp, i0, i1) ? 0 : -1; }
void orc_set_plate_displacement(void* s, const double* d, int reproject) {
  ((Sim<double>*)s)->set_plate_displacement(d, reproject != 0);
}
void orc_set_plate_velocity(void* s, const double* v) { ((Sim<double>*)s)->set_plate_velocity(v); }
// Diagnostic ablation for tests (bit 0: drop C^ij of Eq. forcing-C).
void orc_set_ablation(void* s, int flags) { ((Sim<double>*)s)->drop_C = (flags & 1) != 0; }
int orc_set_open_x(void* s, const double* uin) { return ((Sim<double>*)s)->set_open_x(uin) ? 0 : -1; }
void orc_plate_force(void* s, double* total, double* per_col) { ((Sim<double>*)s)->plate_force(total, per_col); }
void orc_geometry(void* s, double* out28) { ((Sim<double>*)s)->geometry_export(out28); }
void orc_chart(void* s, double* out) {
  Sim<double>* S = (Sim<double>*)s;
  std::memcpy(out, S->chart.data(), sizeof(double) * S->chart.size());
}
void orc_jacobian(void* s, double* out9) { ((Sim<double>*)s)->jacobian_export(out9); }

// Forces on `wall` at states 1..K after the initial state given by f0, for the
// top-wall displacement d (bottom wall flat) and the Cartesian wall velocities
// vwall [2][nz][nx][3] (NULL: walls at rest).
void orc_run_forces(int nx, int ny, int nz, double tau, const double* Fc, const double* d_top,
                    const double* f0, int K, int wall, double* forces, const double* vwall) {
  Sim<double> S(nx, ny, nz, tau);
  S.set_body_force(Fc);
  if (vwall)
    for (int w = 0; w < 2; ++w) S.set_wall_velocity(w, vwall + (long)w * nz * nx * 3);
  S.set_wall_displacement(1, d_top, false);
  S.set_populations(f0);
  for (int t = 0; t < K; ++t) {
    S.step();
    S.wall_force(wall, forces + 3 * t, nullptr);
  }
}

// The same run in dual numbers: forces and their derivatives along the
// direction (dd_top, df0), exact to rounding (forward-mode differentiation).
void orc_dual_forces(int nx, int ny, int nz, double tau, const double* Fc, const double* d_top,
                     const double* dd_top, const double* f0, const double* df0, int K, int wall,
                     double* forces, double* dforces, const double* vwall) {
  Sim<Dual> S(nx, ny, nz, tau);
  S.set_body_force(Fc);
  long ncol = (long)nz * nx;
  if (vwall) {
    std::vector<Dual> v(3 * ncol);
    for (int w = 0; w < 2; ++w) {
      for (long q = 0; q < 3 * ncol; ++q) v[q] = Dual(vwall[w * 3 * ncol + q], 0.0);
      S.set_wall_velocity(w, v.data());
    }
  }
  std::vector<Dual> d(ncol);
  for (long q = 0; q < ncol; ++q) d[q] = Dual(d_top[q], dd_top ? dd_top[q] : 0.0);
  S.set_wall_displacement(1, d.data(), false);
  std::vector<Dual> f(19 * S.N);
  for (long q = 0; q < 19 * S.N; ++q) f[q] = Dual(f0[q], df0 ? df0[q] : 0.0);
  S.set_populations(f.data());
  for (int t = 0; t < K; ++t) {
    S.step();
    Dual tot[3];
    S.wall_force(wall, tot, nullptr);
    for (int a = 0; a < 3; ++a) {
      forces[3 * t + a] = tot[a].v;
      dforces[3 * t + a] = tot[a].d;
    }
  }
}

}  // extern "C"
