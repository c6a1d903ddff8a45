// Per-node forward arithmetic of one step in full-population form (FP64) and
// its hand-written vector-Jacobian product, for the adjoint sweep.
//
// Forward (one fluid node, inputs f_l, history coefficients Fp, geometry,
// lattice gradient dj[k][i] = d_k j^i of the neighbours' momentum):
//   rho = sqrt g sum f, j = sqrt g sum f c                       (Eqs. fields1-2)
//   feq = (w/sqrt g) [rho + 3 j.c + 4.5 a2:cc - 1.5 tr a2],
//         a2 = rho theta (g^ij - delta) + j j / rho              (App. B)
//   ne = f - feq, P = sum ne c c, T = rho theta g^ij + j j/rho + kappa sqrt g P
//   A, B, C of Eqs. (forcing-A/B/C); F = H(A, B, C - theta A delta)
//   f* = f - ne/tau + F - Fo/2, Fo = H(Fp)                        (Eq. collision)
// with theta = c_s^2 = 1/3 and kappa = 1 - 1/(2 tau).  Symmetric tensors are
// packed (xx, xy, xz, yy, yz, zz); Gamma is [i][sym(j,k)].
#pragma once

#include "lbm_device.h"

namespace lbm {

struct AGeo {
  double sg, gi[6], gam[18], F[3];  // sqrt g, g^ij (full), Gamma, F^i
};

struct AGeoBar {
  double sg, gi[6], gam[18], F[3];
};

// Second-order Hermite recomposition (w_l/sqrt g)[a0 + 3 a1.c + 4.5 a2:cc -
// 1.5 tr a2] with a2 packed.
__host__ __device__ inline double hermite_eval(int l, double isg, double a0, const double a1[3], const double a2[6]) {
  const int x = cx(l), y = cy(l), z = cz(l);
  double s = a0 - 1.5 * (a2[0] + a2[3] + a2[5]);
  s += 3.0 * (x * a1[0] + y * a1[1] + z * a1[2]);
  s += 4.5 * (x * x * a2[0] + y * y * a2[3] + z * z * a2[5]);
  s += 9.0 * (x * y * a2[1] + x * z * a2[2] + y * z * a2[4]);
  return wgt(l) * isg * s;
}

// VJP of out_l = hermite_eval(l, 1/sg, a0, a1, a2): accumulates into the
// coefficient adjoints and the adjoint of sg.
__host__ __device__ inline void hermite_vjp(const double hb[Q], const double out[Q], double sg, double& a0b,
                                            double a1b[3], double a2b[6], double& sgb) {
  const double isg = 1.0 / sg;
  double s0 = 0, s1[3] = {0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0}, so = 0;
  for (int l = 0; l < Q; ++l) {
    const double wb = wgt(l) * isg * hb[l];
    const int x = cx(l), y = cy(l), z = cz(l);
    s0 += wb;
    s1[0] += 3.0 * x * wb;
    s1[1] += 3.0 * y * wb;
    s1[2] += 3.0 * z * wb;
    s2[0] += (4.5 * x * x - 1.5) * wb;
    s2[3] += (4.5 * y * y - 1.5) * wb;
    s2[5] += (4.5 * z * z - 1.5) * wb;
    s2[1] += 9.0 * x * y * wb;
    s2[2] += 9.0 * x * z * wb;
    s2[4] += 9.0 * y * z * wb;
    so += out[l] * hb[l];
  }
  a0b += s0;
  for (int a = 0; a < 3; ++a) a1b[a] += s1[a];
  for (int q = 0; q < 6; ++q) a2b[q] += s2[q];
  sgb -= so * isg;
}

// Forward intermediates kept for the VJP.
struct NodeFwd {
  double rho, j[3], S0, S1[3];
  double a2[6], feq[Q], ne[Q], P[6], T[6];
  double tr[3], dbar[3][3], nab[3][3];
  double A, B[3], C[6], b2[6], F[Q];
  double bp[6], Fo[Q];
};

// Forward of one node.  with_old: include the F(t-1) term (false for the
// history of an initial state, which only needs A, B, C).
__host__ __device__ inline void node_fwd(const double f[Q], const double Fp[10], const AGeo& G,
                                         const double dj[3][3], double tau, bool with_old, NodeFwd& o) {
  const double th = 1.0 / 3.0, isg = 1.0 / G.sg;
  o.S0 = 0;
  o.S1[0] = o.S1[1] = o.S1[2] = 0;
  for (int l = 0; l < Q; ++l) {
    o.S0 += f[l];
    o.S1[0] += cx(l) * f[l];
    o.S1[1] += cy(l) * f[l];
    o.S1[2] += cz(l) * f[l];
  }
  o.rho = G.sg * o.S0;
  for (int a = 0; a < 3; ++a) o.j[a] = G.sg * o.S1[a];
  const double ir = 1.0 / o.rho;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b)
      o.a2[sym(a, b)] = o.rho * th * (G.gi[sym(a, b)] - (a == b ? 1.0 : 0.0)) + o.j[a] * o.j[b] * ir;
  for (int l = 0; l < Q; ++l) {
    o.feq[l] = hermite_eval(l, isg, o.rho, o.j, o.a2);
    o.ne[l] = f[l] - o.feq[l];
  }
  for (int q = 0; q < 6; ++q) o.P[q] = 0;
  for (int l = 0; l < Q; ++l) {
    const int c[3] = {cx(l), cy(l), cz(l)};
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) o.P[sym(a, b)] += c[a] * c[b] * o.ne[l];
  }
  const double kap = 1.0 - 0.5 / tau;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      const int q = sym(a, b);
      o.T[q] = o.rho * th * G.gi[q] + o.j[a] * o.j[b] * ir + kap * G.sg * o.P[q];
    }
  for (int b = 0; b < 3; ++b) o.tr[b] = G.gam[0 * 6 + sym(0, b)] + G.gam[1 * 6 + sym(1, b)] + G.gam[2 * 6 + sym(2, b)];
  o.A = -2.0 * (o.tr[0] * o.j[0] + o.tr[1] * o.j[1] + o.tr[2] * o.j[2]);
  for (int i = 0; i < 3; ++i) {
    double s = G.F[i];
    for (int jj = 0; jj < 3; ++jj) {
      s -= 2.0 * o.tr[jj] * o.T[sym(i, jj)];
      for (int kk = 0; kk < 3; ++kk) s -= G.gam[i * 6 + sym(jj, kk)] * o.T[sym(jj, kk)];
    }
    o.B[i] = s;
  }
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) {
      o.dbar[k][i] = dj[k][i] - o.tr[k] * o.j[i];
      double s = dj[k][i];
      for (int l = 0; l < 3; ++l) s += G.gam[i * 6 + sym(k, l)] * o.j[l];
      o.nab[k][i] = s;
    }
  const double divbar = o.dbar[0][0] + o.dbar[1][1] + o.dbar[2][2];
  const double divnab = o.nab[0][0] + o.nab[1][1] + o.nab[2][2];
  for (int i = 0; i < 3; ++i)
    for (int jj = i; jj < 3; ++jj) {
      const double s = o.dbar[jj][i] + o.dbar[i][jj] + (i == jj ? divbar : 0.0);
      double t = G.gi[sym(i, jj)] * divnab;
      for (int k = 0; k < 3; ++k) t += G.gi[sym(jj, k)] * o.nab[k][i] + G.gi[sym(i, k)] * o.nab[k][jj];
      o.C[sym(i, jj)] = th * (s - t);
    }
  for (int q = 0; q < 6; ++q) o.b2[q] = o.C[q];
  o.b2[0] -= th * o.A;
  o.b2[3] -= th * o.A;
  o.b2[5] -= th * o.A;
  for (int l = 0; l < Q; ++l) o.F[l] = hermite_eval(l, isg, o.A, o.B, o.b2);
  if (with_old) {
    for (int q = 0; q < 6; ++q) o.bp[q] = Fp[4 + q];
    o.bp[0] -= th * Fp[0];
    o.bp[3] -= th * Fp[0];
    o.bp[5] -= th * Fp[0];
    for (int l = 0; l < Q; ++l) o.Fo[l] = hermite_eval(l, isg, Fp[0], Fp + 1, o.bp);
  }
}

// VJP of one node.  Inputs: fsb = adjoint of f* (with_old only), Fb = adjoint
// of F (added to what flows from f*), cb = adjoint of the new coefficients
// (A, B, C).  Outputs (accumulated): fb = direct adjoint of f (through ne and
// f*), rb/jb = adjoint of rho and j (local uses), djb = adjoint of dj, Fpb =
// adjoint of the old coefficients, gb = geometry adjoint.
__host__ __device__ inline void node_vjp(const double f[Q], const double Fp[10], const AGeo& G, const double dj[3][3],
                                         double tau, bool with_old, const NodeFwd& o, const double fsb[Q],
                                         const double Fbin[Q], const double cb[10], const double* Tbin, double fb[Q],
                                         double& rb, double jb[3], double djb[3][3], double Fpb[10], AGeoBar& gb) {
  (void)f;
  (void)dj;
  const double th = 1.0 / 3.0, itau = 1.0 / tau, kap = 1.0 - 0.5 / tau;
  double neb[Q], Fb[Q], Fob[Q];
  for (int l = 0; l < Q; ++l) {
    const double s = with_old ? fsb[l] : 0.0;
    fb[l] += s;
    neb[l] = -s * itau;
    Fb[l] = s + Fbin[l];
    Fob[l] = -0.5 * s;
  }
  // F(t-1) = H(Fp) -> old coefficients
  if (with_old) {
    double a0b = 0, a1b[3] = {0, 0, 0}, a2b[6] = {0, 0, 0, 0, 0, 0};
    hermite_vjp(Fob, o.Fo, G.sg, a0b, a1b, a2b, gb.sg);
    Fpb[0] += a0b - th * (a2b[0] + a2b[3] + a2b[5]);
    for (int a = 0; a < 3; ++a) Fpb[1 + a] += a1b[a];
    for (int q = 0; q < 6; ++q) Fpb[4 + q] += a2b[q];
  }
  // F = H(A, B, C - theta A delta)
  double Ab = cb[0], Bb[3] = {cb[1], cb[2], cb[3]}, Cb[6];
  for (int q = 0; q < 6; ++q) Cb[q] = cb[4 + q];
  {
    double a0b = 0, a1b[3] = {0, 0, 0}, a2b[6] = {0, 0, 0, 0, 0, 0};
    hermite_vjp(Fb, o.F, G.sg, a0b, a1b, a2b, gb.sg);
    Ab += a0b - th * (a2b[0] + a2b[3] + a2b[5]);
    for (int a = 0; a < 3; ++a) Bb[a] += a1b[a];
    for (int q = 0; q < 6; ++q) Cb[q] += a2b[q];
  }
  double jbar[3] = {0, 0, 0}, Tb[6] = {0, 0, 0, 0, 0, 0}, trb[3] = {0, 0, 0};
  if (Tbin)
    for (int q = 0; q < 6; ++q) Tb[q] = Tbin[q];
  double dbarb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, nabb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  // C^ij = theta (s_ij - t_ij)
  double divbarb = 0, divnabb = 0;
  for (int i = 0; i < 3; ++i)
    for (int jj = i; jj < 3; ++jj) {
      const double cbq = th * Cb[sym(i, jj)];
      // s = dbar[jj][i] + dbar[i][jj] + delta divbar
      dbarb[jj][i] += cbq;
      dbarb[i][jj] += cbq;
      if (i == jj) divbarb += cbq;
      // t = g^{i jj} divnab + sum_k g^{jj k} nab[k][i] + g^{i k} nab[k][jj]
      const double tbq = -cbq;
      gb.gi[sym(i, jj)] += tbq * (o.nab[0][0] + o.nab[1][1] + o.nab[2][2]);
      divnabb += tbq * G.gi[sym(i, jj)];
      for (int k = 0; k < 3; ++k) {
        gb.gi[sym(jj, k)] += tbq * o.nab[k][i];
        nabb[k][i] += tbq * G.gi[sym(jj, k)];
        gb.gi[sym(i, k)] += tbq * o.nab[k][jj];
        nabb[k][jj] += tbq * G.gi[sym(i, k)];
      }
    }
  for (int k = 0; k < 3; ++k) {
    dbarb[k][k] += divbarb;
    nabb[k][k] += divnabb;
  }
  // nab[k][i] = dj[k][i] + Gamma^i_kl j^l ; dbar[k][i] = dj[k][i] - tr_k j^i
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) {
      djb[k][i] += nabb[k][i] + dbarb[k][i];
      for (int l = 0; l < 3; ++l) {
        gb.gam[i * 6 + sym(k, l)] += nabb[k][i] * o.j[l];
        jbar[l] += nabb[k][i] * G.gam[i * 6 + sym(k, l)];
      }
      trb[k] -= dbarb[k][i] * o.j[i];
      jbar[i] -= dbarb[k][i] * o.tr[k];
    }
  // B^i = F^i - 2 tr_j T^ij - Gamma^i_jk T^jk
  for (int i = 0; i < 3; ++i) {
    gb.F[i] += Bb[i];
    for (int jj = 0; jj < 3; ++jj) {
      trb[jj] -= 2.0 * Bb[i] * o.T[sym(i, jj)];
      Tb[sym(i, jj)] -= 2.0 * Bb[i] * o.tr[jj];
      for (int kk = 0; kk < 3; ++kk) {
        gb.gam[i * 6 + sym(jj, kk)] -= Bb[i] * o.T[sym(jj, kk)];
        Tb[sym(jj, kk)] -= Bb[i] * G.gam[i * 6 + sym(jj, kk)];
      }
    }
  }
  // A = -2 tr . j
  for (int a = 0; a < 3; ++a) {
    trb[a] -= 2.0 * Ab * o.j[a];
    jbar[a] -= 2.0 * Ab * o.tr[a];
  }
  // tr_b = sum_i Gamma^i_ib
  for (int b = 0; b < 3; ++b)
    for (int i = 0; i < 3; ++i) gb.gam[i * 6 + sym(i, b)] += trb[b];
  // T = rho theta g^ij + j j / rho + kappa sqrt g P
  double rbar = 0, Pb[6];
  const double ir = 1.0 / o.rho;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      const int q = sym(a, b);
      rbar += Tb[q] * (th * G.gi[q] - o.j[a] * o.j[b] * ir * ir);
      gb.gi[q] += Tb[q] * o.rho * th;
      jbar[a] += Tb[q] * o.j[b] * ir;
      jbar[b] += Tb[q] * o.j[a] * ir;
      gb.sg += Tb[q] * kap * o.P[q];
      Pb[q] = Tb[q] * kap * G.sg;
    }
  // P = sum ne c c
  for (int l = 0; l < Q; ++l) {
    const int c[3] = {cx(l), cy(l), cz(l)};
    double s = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) s += c[a] * c[b] * Pb[sym(a, b)];
    neb[l] += s;
  }
  // ne = f - feq
  double feqb[Q];
  for (int l = 0; l < Q; ++l) {
    fb[l] += neb[l];
    feqb[l] = -neb[l];
  }
  // feq = H(rho, j, a2)
  double a2b[6] = {0, 0, 0, 0, 0, 0};
  {
    double a0b = 0, a1b[3] = {0, 0, 0};
    hermite_vjp(feqb, o.feq, G.sg, a0b, a1b, a2b, gb.sg);
    rbar += a0b;
    for (int a = 0; a < 3; ++a) jbar[a] += a1b[a];
  }
  // a2 = rho theta (g^ij - delta) + j j / rho
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      const int q = sym(a, b);
      rbar += a2b[q] * (th * (G.gi[q] - (a == b ? 1.0 : 0.0)) - o.j[a] * o.j[b] * ir * ir);
      gb.gi[q] += a2b[q] * o.rho * th;
      jbar[a] += a2b[q] * o.j[b] * ir;
      jbar[b] += a2b[q] * o.j[a] * ir;
    }
  rb += rbar;
  for (int a = 0; a < 3; ++a) jb[a] += jbar[a];
}

// Moments rho = sg S0, j = sg S1 -> adjoint into f and sg.
__host__ __device__ inline void moments_vjp(double sg, double S0, const double S1[3], double rb, const double jb[3],
                                            double fb[Q], double& sgb) {
  for (int l = 0; l < Q; ++l) fb[l] += sg * (rb + cx(l) * jb[0] + cy(l) * jb[1] + cz(l) * jb[2]);
  sgb += S0 * rb + S1[0] * jb[0] + S1[1] * jb[1] + S1[2] * jb[2];
}

}  // namespace lbm
