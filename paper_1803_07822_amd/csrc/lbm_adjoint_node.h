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
//
// Every loop over the 19 directions is unrolled at compile time and no
// per-direction intermediate is stored, so a node's working set stays in
// registers: the Hermite recompositions are linear in their coefficients, so
// the VJP of one needs only ten basis sums of the incoming adjoint, and the
// forward value it would multiply is a0 s0 + a1.s1 + a2:s2 of those sums.
#pragma once

#include "lbm_device.h"

namespace lbm {

struct AGeo {
  double sg, gi[6], gam[18], F[3];  // sqrt g, g^ij (full), Gamma, F^i
};

// Adjoint of the geometry of one node, accumulated in registers.  The VJPs
// add into it through add_* so that an accumulator in LDS (LdsGeoBar) can
// stand in for it where registers are short.
struct AGeoBar {
  double sg, gi[6], gam[18], F[3];
  __device__ __forceinline__ void add_sg(double v) { sg += v; }
  __device__ __forceinline__ void add_gi(int q, double v) { gi[q] += v; }
  __device__ __forceinline__ void add_gam(int q, double v) { gam[q] += v; }
  __device__ __forceinline__ void add_F(int i, double v) { F[i] += v; }
};

// The same accumulator in LDS: 28 slots per lane at base[slot * stride], each
// addition one LDS atomic add (no return value), so that no register holds
// the 28 sums between the additions.  Slot order: sqrt g, g^ij (6), Gamma
// (18), F^i (3).
struct LdsGeoBar {
  double* base;
  int stride;
  __device__ __forceinline__ void add(int slot, double v) {
    __hip_atomic_fetch_add(base + slot * stride, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ __forceinline__ void add_sg(double v) { add(0, v); }
  __device__ __forceinline__ void add_gi(int q, double v) { add(1 + q, v); }
  __device__ __forceinline__ void add_gam(int q, double v) { add(7 + q, v); }
  __device__ __forceinline__ void add_F(int i, double v) { add(25 + i, v); }
};

// Basis sums of an adjoint hb_l over the directions (lattice weight included,
// 1/sqrt g not): s0 = sum w hb, s1 = sum w hb 3c, s2 = sum w hb (4.5 cc -
// 1.5 I) packed, with off-diagonal entries 9 c_a c_b.
struct HSum {
  double s0, s1[3], s2[6];
};

__device__ __forceinline__ void hsum_zero(HSum& h) {
  h.s0 = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) h.s1[a] = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) h.s2[q] = 0;
}

template <int l> __device__ __forceinline__ void hsum_add(HSum& h, double hb) {
  constexpr int x = cx(l), y = cy(l), z = cz(l);
  const double wb = wgt(l) * hb;
  h.s0 += wb;
  if (x) h.s1[0] += (3.0 * x) * wb;
  if (y) h.s1[1] += (3.0 * y) * wb;
  if (z) h.s1[2] += (3.0 * z) * wb;
  h.s2[0] += (4.5 * x * x - 1.5) * wb;
  h.s2[3] += (4.5 * y * y - 1.5) * wb;
  h.s2[5] += (4.5 * z * z - 1.5) * wb;
  if (x && y) h.s2[1] += (9.0 * x * y) * wb;
  if (x && z) h.s2[2] += (9.0 * x * z) * wb;
  if (y && z) h.s2[4] += (9.0 * y * z) * wb;
}

// Second-order Hermite recomposition (w_l/sqrt g)[a0 + 3 a1.c + 4.5 a2:cc -
// 1.5 tr a2] with a2 packed.
template <int l>
__device__ __forceinline__ double hermite_val(double isg, double a0, const double a1[3], const double a2[6]) {
  return wgt(l) * isg * hermite_term<double, l>(a0, a1, a2);
}

// VJP of out_l = (w_l/sg) H_l(a0, a1, a2) from the basis sums h of its
// adjoint: accumulates into the coefficient adjoints and the adjoint of sg
// (out is proportional to 1/sg).
__device__ __forceinline__ void hermite_vjp(const HSum& h, double isg, double a0, const double a1[3], const double a2[6],
                                            double& a0b, double a1b[3], double a2b[6], double& sgb) {
  a0b += isg * h.s0;
  double so = a0 * h.s0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    a1b[a] += isg * h.s1[a];
    so += a1[a] * h.s1[a];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    a2b[q] += isg * h.s2[q];
    so += a2[q] * h.s2[q];
  }
  sgb -= so * isg * isg;
}

// Forward intermediates kept for the VJP.
struct NodeFwd {
  double isg, rho, j[3], S0, S1[3];
  double a2[6], P[6], T[6];
  double tr[3], dbar[3][3], nab[3][3];
  double A, B[3], C[6], b2[6];
  double bp[6];
};

__device__ __forceinline__ void node_fwd_rest(const double Fp[10], const AGeo& G, const double dj[3][3], double tau,
                                              bool with_old, NodeFwd& o);

// Forward of one node.  with_old: include the F(t-1) term (false for the
// history of an initial state, which only needs A, B, C).
__device__ __forceinline__ void node_fwd(const double f[Q], const double Fp[10], const AGeo& G, const double dj[3][3],
                                         double tau, bool with_old, NodeFwd& o) {
  const double th = 1.0 / 3.0;
  o.isg = 1.0 / G.sg;
  o.S0 = 0;
  o.S1[0] = o.S1[1] = o.S1[2] = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    o.S0 += f[l];
    if (cx(l)) o.S1[0] += cx(l) * f[l];
    if (cy(l)) o.S1[1] += cy(l) * f[l];
    if (cz(l)) o.S1[2] += cz(l) * f[l];
  });
  o.rho = G.sg * o.S0;
#pragma unroll
  for (int a = 0; a < 3; ++a) o.j[a] = G.sg * o.S1[a];
  const double ir = 1.0 / o.rho;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
      o.a2[sym(a, b)] = o.rho * th * (G.gi[sym(a, b)] - (a == b ? 1.0 : 0.0)) + o.j[a] * o.j[b] * ir;
  // P = sum (f - feq) c c
#pragma unroll
  for (int q = 0; q < 6; ++q) o.P[q] = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    constexpr int x = cx(l), y = cy(l), z = cz(l);
    const double ne = f[l] - hermite_val<l>(o.isg, o.rho, o.j, o.a2);
    if (x) o.P[0] += ne;
    if (y) o.P[3] += ne;
    if (z) o.P[5] += ne;
    if (x && y) o.P[1] += (x * y) * ne;
    if (x && z) o.P[2] += (x * z) * ne;
    if (y && z) o.P[4] += (y * z) * ne;
  });
  node_fwd_rest(Fp, G, dj, tau, with_old, o);
}

// The rest of the forward of one node, from o.isg, o.rho, o.j, o.a2 and o.P:
// the stress T, the forcing coefficients and the old forcing's b2.
__device__ __forceinline__ void node_fwd_rest(const double Fp[10], const AGeo& G, const double dj[3][3], double tau,
                                              bool with_old, NodeFwd& o) {
  const double th = 1.0 / 3.0;
  const double ir = 1.0 / o.rho;
  const double kap = 1.0 - 0.5 / tau;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      const int q = sym(a, b);
      o.T[q] = o.rho * th * G.gi[q] + o.j[a] * o.j[b] * ir + kap * G.sg * o.P[q];
    }
#pragma unroll
  for (int b = 0; b < 3; ++b) o.tr[b] = G.gam[0 * 6 + sym(0, b)] + G.gam[1 * 6 + sym(1, b)] + G.gam[2 * 6 + sym(2, b)];
  o.A = -2.0 * (o.tr[0] * o.j[0] + o.tr[1] * o.j[1] + o.tr[2] * o.j[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = G.F[i];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      s -= 2.0 * o.tr[jj] * o.T[sym(i, jj)];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) s -= G.gam[i * 6 + sym(jj, kk)] * o.T[sym(jj, kk)];
    }
    o.B[i] = s;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      o.dbar[k][i] = dj[k][i] - o.tr[k] * o.j[i];
      double s = dj[k][i];
#pragma unroll
      for (int l = 0; l < 3; ++l) s += G.gam[i * 6 + sym(k, l)] * o.j[l];
      o.nab[k][i] = s;
    }
  const double divbar = o.dbar[0][0] + o.dbar[1][1] + o.dbar[2][2];
  const double divnab = o.nab[0][0] + o.nab[1][1] + o.nab[2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj) {
      const double s = o.dbar[jj][i] + o.dbar[i][jj] + (i == jj ? divbar : 0.0);
      double t = G.gi[sym(i, jj)] * divnab;
#pragma unroll
      for (int k = 0; k < 3; ++k) t += G.gi[sym(jj, k)] * o.nab[k][i] + G.gi[sym(i, k)] * o.nab[k][jj];
      o.C[sym(i, jj)] = th * (s - t);
    }
#pragma unroll
  for (int q = 0; q < 6; ++q) o.b2[q] = o.C[q];
  o.b2[0] -= th * o.A;
  o.b2[3] -= th * o.A;
  o.b2[5] -= th * o.A;
  if (with_old) {
#pragma unroll
    for (int q = 0; q < 6; ++q) o.bp[q] = Fp[4 + q];
    o.bp[0] -= th * Fp[0];
    o.bp[3] -= th * Fp[0];
    o.bp[5] -= th * Fp[0];
  }
}

// VJP of the old forcing Fo = H(Fp) (F(t-1) in Eq. collision, b2 = bp) from
// the basis sums h of its adjoint: into the old coefficients Fpb and sg.
__device__ __forceinline__ void old_forcing_vjp(const HSum& h, double isg, const double Fp[10], const double bp[6],
                                                double Fpb[10], double& sgb) {
  const double th = 1.0 / 3.0;
  double a0b = 0, a1b[3] = {0, 0, 0}, a2b[6] = {0, 0, 0, 0, 0, 0};
  hermite_vjp(h, isg, Fp[0], Fp + 1, bp, a0b, a1b, a2b, sgb);
  Fpb[0] += a0b - th * (a2b[0] + a2b[3] + a2b[5]);
#pragma unroll
  for (int a = 0; a < 3; ++a) Fpb[1 + a] += a1b[a];
#pragma unroll
  for (int q = 0; q < 6; ++q) Fpb[4 + q] += a2b[q];
}

// The P-dependent part of the adjoint of f_l: the adjoint Pb of
// P = sum_l ne_l c_l c_l (packed) seen by direction l.
template <int l> __device__ __forceinline__ double pb_term(const double Pb[6]) {
  constexpr int x = cx(l), y = cy(l), z = cz(l);
  double v = 0.0;
  if (x) v += Pb[0];
  if (y) v += Pb[3];
  if (z) v += Pb[5];
  if (x && y) v += (x * y) * Pb[1];
  if (x && z) v += (x * z) * Pb[2];
  if (y && z) v += (y * z) * Pb[4];
  return v;
}

// VJP of one node, with the per-direction adjoints entering only through
// their Hermite basis sums.  Inputs: hs = basis sums of the adjoint s_l of
// f*_l (with_old only), hb = basis sums of the adjoint of F_l (added to what
// flows from f*), cb = adjoint of the new coefficients (A, B, C), Tbin =
// adjoint of T (or null).  Outputs (accumulated): Pb = adjoint of P, so that
// the direct adjoint of f_l is (1 - 1/tau) s_l + pb_term<l>(Pb) (formed where
// s_l is read again); rb/jb = adjoint of rho and j (local uses); djb =
// adjoint of dj; Fpb = adjoint of the old coefficients; gb = geometry
// adjoint.
template <class GB>
__device__ __forceinline__ void node_vjp(const double Fp[10], const AGeo& G, double tau, bool with_old,
                                         const NodeFwd& o, const HSum& hs, const HSum& hb, const double cb[10],
                                         const double* Tbin, double Pb[6], double& rb, double jb[3],
                                         double djb[3][3], double Fpb[10], GB& gb) {
  const double th = 1.0 / 3.0, itau = 1.0 / tau, kap = 1.0 - 0.5 / tau;
  double sgl = 0;  // adjoint of sqrt g, added to gb at the end
  // f* = f - ne/tau + F - Fo/2: basis sums of the adjoints of Fo and F
  HSum hFo, hF;
  {
    const double w = with_old ? 1.0 : 0.0;
    hFo.s0 = -0.5 * w * hs.s0;
    hF.s0 = w * hs.s0 + hb.s0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      hFo.s1[a] = -0.5 * w * hs.s1[a];
      hF.s1[a] = w * hs.s1[a] + hb.s1[a];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      hFo.s2[q] = -0.5 * w * hs.s2[q];
      hF.s2[q] = w * hs.s2[q] + hb.s2[q];
    }
  }
  // (Fp null: the caller has reversed the old forcing already)
  if (with_old && Fp) old_forcing_vjp(hFo, o.isg, Fp, o.bp, Fpb, sgl);
  // F = H(A, B, C - theta A delta)
  double Ab = cb[0], Bb[3] = {cb[1], cb[2], cb[3]}, Cb[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) Cb[q] = cb[4 + q];
  {
    double a0b = 0, a1b[3] = {0, 0, 0}, a2b[6] = {0, 0, 0, 0, 0, 0};
    hermite_vjp(hF, o.isg, o.A, o.B, o.b2, a0b, a1b, a2b, sgl);
    Ab += a0b - th * (a2b[0] + a2b[3] + a2b[5]);
#pragma unroll
    for (int a = 0; a < 3; ++a) Bb[a] += a1b[a];
#pragma unroll
    for (int q = 0; q < 6; ++q) Cb[q] += a2b[q];
  }
  double jbar[3] = {0, 0, 0}, Tb[6] = {0, 0, 0, 0, 0, 0}, trb[3] = {0, 0, 0};
  if (Tbin)
#pragma unroll
    for (int q = 0; q < 6; ++q) Tb[q] = Tbin[q];
  double dbarb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, nabb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  // C^ij = theta (s_ij - t_ij)
  double divbarb = 0, divnabb = 0;
  const double divnab = o.nab[0][0] + o.nab[1][1] + o.nab[2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj) {
      const double cbq = th * Cb[sym(i, jj)];
      // s = dbar[jj][i] + dbar[i][jj] + delta divbar
      dbarb[jj][i] += cbq;
      dbarb[i][jj] += cbq;
      if (i == jj) divbarb += cbq;
      // t = g^{i jj} divnab + sum_k g^{jj k} nab[k][i] + g^{i k} nab[k][jj]
      const double tbq = -cbq;
      gb.add_gi(sym(i, jj), tbq * divnab);
      divnabb += tbq * G.gi[sym(i, jj)];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gb.add_gi(sym(jj, k), tbq * o.nab[k][i]);
        nabb[k][i] += tbq * G.gi[sym(jj, k)];
        gb.add_gi(sym(i, k), tbq * o.nab[k][jj]);
        nabb[k][jj] += tbq * G.gi[sym(i, k)];
      }
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dbarb[k][k] += divbarb;
    nabb[k][k] += divnabb;
  }
  // nab[k][i] = dj[k][i] + Gamma^i_kl j^l ; dbar[k][i] = dj[k][i] - tr_k j^i
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      djb[k][i] += nabb[k][i] + dbarb[k][i];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        gb.add_gam(i * 6 + sym(k, l), nabb[k][i] * o.j[l]);
        jbar[l] += nabb[k][i] * G.gam[i * 6 + sym(k, l)];
      }
      trb[k] -= dbarb[k][i] * o.j[i];
      jbar[i] -= dbarb[k][i] * o.tr[k];
    }
  // B^i = F^i - 2 tr_j T^ij - Gamma^i_jk T^jk
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gb.add_F(i, Bb[i]);
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      trb[jj] -= 2.0 * Bb[i] * o.T[sym(i, jj)];
      Tb[sym(i, jj)] -= 2.0 * Bb[i] * o.tr[jj];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        gb.add_gam(i * 6 + sym(jj, kk), -(Bb[i] * o.T[sym(jj, kk)]));
        Tb[sym(jj, kk)] -= Bb[i] * G.gam[i * 6 + sym(jj, kk)];
      }
    }
  }
  // A = -2 tr . j
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    trb[a] -= 2.0 * Ab * o.j[a];
    jbar[a] -= 2.0 * Ab * o.tr[a];
  }
  // tr_b = sum_i Gamma^i_ib
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i) gb.add_gam(i * 6 + sym(i, b), trb[b]);
  // T = rho theta g^ij + j j / rho + kappa sqrt g P
  double rbar = 0;
  const double ir = 1.0 / o.rho;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      const int q = sym(a, b);
      rbar += Tb[q] * (th * G.gi[q] - o.j[a] * o.j[b] * ir * ir);
      gb.add_gi(q, Tb[q] * o.rho * th);
      jbar[a] += Tb[q] * o.j[b] * ir;
      jbar[b] += Tb[q] * o.j[a] * ir;
      sgl += Tb[q] * kap * o.P[q];
      Pb[q] = Tb[q] * kap * G.sg;
    }
  // P = sum ne c c, ne = f - feq; f* = f - ne/tau + ...: the adjoint of ne_l
  // is -s_l/tau + pb_term<l>(Pb), and feq_l = f_l - ne_l takes minus that
  // (basis sums: hs/tau minus those of the pb_term)
  HSum hfeq;
  hsum_zero(hfeq);
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    hsum_add<l>(hfeq, -pb_term<l>(Pb));
  });
  if (with_old) {
    hfeq.s0 += itau * hs.s0;
#pragma unroll
    for (int a = 0; a < 3; ++a) hfeq.s1[a] += itau * hs.s1[a];
#pragma unroll
    for (int q = 0; q < 6; ++q) hfeq.s2[q] += itau * hs.s2[q];
  }
  // feq = H(rho, j, a2)
  double a2b[6] = {0, 0, 0, 0, 0, 0};
  {
    double a0b = 0, a1b[3] = {0, 0, 0};
    hermite_vjp(hfeq, o.isg, o.rho, o.j, o.a2, a0b, a1b, a2b, sgl);
    rbar += a0b;
#pragma unroll
    for (int a = 0; a < 3; ++a) jbar[a] += a1b[a];
  }
  // a2 = rho theta (g^ij - delta) + j j / rho
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      const int q = sym(a, b);
      rbar += a2b[q] * (th * (G.gi[q] - (a == b ? 1.0 : 0.0)) - o.j[a] * o.j[b] * ir * ir);
      gb.add_gi(q, a2b[q] * o.rho * th);
      jbar[a] += a2b[q] * o.j[b] * ir;
      jbar[b] += a2b[q] * o.j[a] * ir;
    }
  rb += rbar;
#pragma unroll
  for (int a = 0; a < 3; ++a) jb[a] += jbar[a];
  gb.add_sg(sgl);
}

// Moments rho = sg S0, j = sg S1 -> adjoint into f and sg.
__device__ __forceinline__ void moments_vjp(double sg, double S0, const double S1[3], double rb, const double jb[3],
                                            double fb[Q], double& sgb) {
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    double v = rb;
    if (cx(l)) v += cx(l) * jb[0];
    if (cy(l)) v += cy(l) * jb[1];
    if (cz(l)) v += cz(l) * jb[2];
    fb[l] += sg * v;
  });
  sgb += S0 * rb + S1[0] * jb[0] + S1[1] * jb[1] + S1[2] * jb[2];
}

}  // namespace lbm
