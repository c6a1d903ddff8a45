// Adjoint of K steps (FP64): trajectory storage and entry points.
#pragma once

#include "lbm_internal.h"

namespace lbm {

struct AdjointBuffers {
  double* ckpt = nullptr;  // (K/N + 1) checkpoints of (pop, hist) in the FP64 pull layout
  double* traj = nullptr;  // N states of one segment
  int nckpt = 0;
};

inline void carve_adjoint(Carver& c, const Grid& g, int K, int N, AdjointBuffers& A) {
  const size_t state = sizeof(double) * (19 + H_N) * (size_t)g.N;
  A.nckpt = K / N + 1;
  A.ckpt = (double*)c.take(state * A.nckpt);
  A.traj = (double*)c.take(state * (N + 1));
}

hipError_t adjoint_forward(Fields& F, AdjointBuffers& A, hipStream_t s, int K, int N, int wall, double tau,
                           double* forces);
hipError_t adjoint_backward(Fields& F, AdjointBuffers& A, hipStream_t s, int K, int N, int wall, double tau,
                            const double Fc[3], const double* dLdF, double* grad_disp, double* grad_chart,
                            double* grad_f0);

}  // namespace lbm
