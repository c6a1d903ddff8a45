// Adjoint of K steps (FP64): trajectory storage and entry points.
#pragma once

#include "lbm_internal.h"

namespace lbm {

struct AdjointBuffers {
  double* ckpt = nullptr;  // nckpt states (pop 19 + history 10 per node, pull layout)
  double* traj = nullptr;  // ckpt_every states of one segment
  double* tmom = nullptr;  // [ckpt_every][4][N] rho, rho u of the segment's states, from the recompute steps
  double* lf[2] = {nullptr, nullptr};  // [19][N] adjoint of f (current / next)
  double* lp[2] = {nullptr, nullptr};  // [10][N] adjoint of the history coefficients
  double* lpb = nullptr;   // [6][N]  adjoint of the non-equilibrium flux P (direct part of the f adjoint)
  double* lml = nullptr;   // [4][N]  local adjoint of (rho, j)
  double* ldj = nullptr;   // [9][N]  adjoint of the lattice gradient
  double* lg = nullptr;    // [28][N] adjoint of the stored geometry fields
  double* lj = nullptr;    // [9][N]  adjoint of J (wall force)
  double* ldg = nullptr;   // [18][N] adjoint of the metric derivatives D_l g
  double* lue = nullptr;   // [3][NE]
  double* lve = nullptr;   // [3][NE]
  double* lJe = nullptr;   // [9][NE]
  double* lge = nullptr;   // [6][NE]
  double* lwe = nullptr;   // [6][NE]
  double* gc = nullptr;    // [3][NC] adjoint of the chart
  double* ub = nullptr;    // [2][nz][nx][3] adjoint of the walls' chart-component velocity
  int nckpt = 0;
};

inline void carve_adjoint(Carver& c, const Grid& g, int K, int N, AdjointBuffers& A) {
  const size_t Nn = (size_t)g.N;
  const size_t NE = (size_t)g.nz * (g.ny + 6) * g.nx, NC = (size_t)g.nz * g.ny * g.nx;
  const size_t state = sizeof(double) * (19 + H_N) * Nn;
  A.nckpt = (K + N - 1) / N + 1;  // segment starts plus the final state
  A.ckpt = (double*)c.take(state * A.nckpt);
  A.traj = (double*)c.take(state * N);
  A.tmom = (double*)c.take(sizeof(double) * 4 * Nn * N);
  for (int b = 0; b < 2; ++b) {
    A.lf[b] = (double*)c.take(sizeof(double) * 19 * Nn);
    A.lp[b] = (double*)c.take(sizeof(double) * H_N * Nn);
  }
  A.lpb = (double*)c.take(sizeof(double) * 6 * Nn);
  A.lml = (double*)c.take(sizeof(double) * 4 * Nn);
  A.ldj = (double*)c.take(sizeof(double) * 9 * Nn);
  A.lg = (double*)c.take(sizeof(double) * G_N * Nn);
  A.lj = (double*)c.take(sizeof(double) * 9 * Nn);
  A.ldg = (double*)c.take(sizeof(double) * 18 * Nn);
  A.lue = (double*)c.take(sizeof(double) * 3 * NE);
  A.lve = (double*)c.take(sizeof(double) * 3 * NE);
  A.lJe = (double*)c.take(sizeof(double) * 9 * NE);
  A.lge = (double*)c.take(sizeof(double) * 6 * NE);
  A.lwe = (double*)c.take(sizeof(double) * 6 * NE);
  A.gc = (double*)c.take(sizeof(double) * 3 * NC);
  A.ub = (double*)c.take(sizeof(double) * 2 * 3 * (size_t)g.nz * g.nx);
}

hipError_t adjoint_forward(Fields& F, AdjointBuffers& A, hipStream_t s, int K, int N, int wall, double tau,
                           double* forces);
hipError_t adjoint_backward(Fields& F, AdjointBuffers& A, hipStream_t s, int K, int N, int wall, double tau,
                            const double Fc[3], const double* dLdF, double* grad_disp, double* grad_chart,
                            double* grad_f0);

}  // namespace lbm
