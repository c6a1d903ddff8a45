// C-ABI of liblbm: context, argument checks, call order, workspace carving and
// launch orchestration.  All device memory comes from the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_adjoint.h"
#include "lbm_internal.h"

using lbm::Fields;
using lbm::Grid;

struct lbm_ctx {
  Fields F;
  lbm::AdjointBuffers adj;
  int precision = 0;
  double tau = 0.8;
  double Fc[3] = {0, 0, 0};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t bytes = 0, used = 0;
  int have_geo = 0, have_state = 0;
  int sticky = LBM_OK;
  int adjK = 0, adjN = 0, recorded = 0, rec_wall = 1;
  void* scratch = nullptr;  // the device's allocation-free scratch (lbm_wall_force_noalloc)
  int scratch_rc = 0;       // hipError_t of resolving it
  std::string err;
};

namespace {

using lbm::ALIGN;
using lbm::Carver;

// The step kernels address a pair of population planes from one base with
// 32-bit byte offsets: 2 * fluid nodes * 8 bytes must stay below 4 GiB.
constexpr long long MAX_FLUID_NODES = 1LL << 28;

bool grid_ok(const lbm_grid* g) {
  if (!g || g->nx < 1 || g->nz < 1 || g->ny < 4) return false;
  return (long long)g->nx * (g->ny - 2) * g->nz < MAX_FLUID_NODES;
}

Grid make_grid(const lbm_grid* h) {
  Grid g;
  g.nx = h->nx;
  g.ny = h->ny;
  g.nz = h->nz;
  g.H = h->ny - 2;
  g.N = (long long)g.nx * g.H * g.nz;
  g.pj = 0;
  g.pi0 = 0;
  g.pi1 = -1;
  g.open = 0;
  return g;
}

// Staging of pulled populations in the fused step that measured fastest:
// registers in FP32; in FP64 the collision leaves no registers for a second
// plane.
int default_stage(int precision) { return precision == LBM_FP64 ? 0 : 1; }

void carve_core(Carver& c, const Grid& g, int precision, Fields& F) {
  const size_t sz = precision == LBM_FP64 ? sizeof(double) : sizeof(float);
  const long long NE = (long long)g.nz * (g.ny + 6) * g.nx, NC = (long long)g.nz * g.ny * g.nx, N = g.N;
  F.g = g;
  F.NE = NE;
  F.NC = NC;
  F.chart = (double*)c.take(sizeof(double) * 3 * NC);
  F.uext[0] = (double*)c.take(sizeof(double) * 3 * NE);
  F.uext[1] = (double*)c.take(sizeof(double) * 3 * NE);
  F.vtmp = (double*)c.take(sizeof(double) * 3 * NE);
  F.gext = (double*)c.take(sizeof(double) * 6 * NE);
  F.wext = (double*)c.take(sizeof(double) * 6 * NE);
  F.jac = (double*)c.take(sizeof(double) * 9 * N);
  F.geo = c.take(sz * lbm::G_N * N);
  F.pop[0] = c.take(sz * 19 * N);
  F.pop[1] = c.take(sz * 19 * N);
  F.hist[0] = c.take(sz * lbm::H_N * N);
  F.hist[1] = c.take(sz * lbm::H_N * N);
  F.mom = c.take(sz * 4 * N);
  F.uw = c.take(sz * 2 * 3 * (size_t)g.nz * g.nx);
  F.up = c.take(sz * 2 * 3 * (size_t)g.nz * g.nx);
  F.vplate = (double*)c.take(sizeof(double) * 3 * (size_t)g.nz * g.nx);
  F.dplate = (double*)c.take(sizeof(double) * (size_t)g.nz * g.nx);
  F.uin = (double*)c.take(sizeof(double) * 3 * (size_t)g.nz * g.H);
  F.vin = c.take(sz * 3 * (size_t)g.nz * g.H);
  F.disp = (double*)c.take(sizeof(double) * 2 * (size_t)g.nz * g.nx);
  F.vwall = (double*)c.take(sizeof(double) * 2 * 3 * (size_t)g.nz * g.nx);
  F.full = (double*)c.take(sizeof(double) * 19 * N);
  F.mf = c.take(sz * 20 * NC);
  F.part = (double*)c.take(sizeof(double) * 3 * (size_t)lbm::wall_force_blocks(g));
  F.count = (unsigned*)c.take(ALIGN);
  F.fpart = (double*)c.take(sizeof(double) * 2 * 3 * (size_t)((g.nx + lbm::BX - 1) / lbm::BX) * g.nz);
  F.flag = (int*)c.take(ALIGN);
  F.cur = 0;
  F.uext_cur = 0;
  F.moving[0] = F.moving[1] = 0;
}

// Clears n doubles with a kernel: the setters a time loop repeats use it in
// place of a memset, so that a caller capturing them into a HIP graph records
// kernels and device-to-device copies only.
__global__ void k_zero(double* __restrict__ p, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) p[e] = 0.0;
}

hipError_t zero_async(double* p, size_t n, hipStream_t s) {
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

int fail(lbm_ctx* c, int code, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (code == LBM_EHIP || code == LBM_EUNSTABLE) c->sticky = code;
  }
  return code;
}

int hip_check(lbm_ctx* c, hipError_t e, const char* where) {
  if (e == hipSuccess) return LBM_OK;
  return fail(c, LBM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define LBM_GUARD(c)                                                          \
  do {                                                                        \
    if (!(c)) return LBM_EINVAL;                                              \
    if ((c)->sticky != LBM_OK) return (c)->sticky;                            \
  } while (0)

#define LBM_HIP(c, expr)                                                      \
  do {                                                                        \
    int _r = hip_check((c), (expr), #expr);                                   \
    if (_r != LBM_OK) return _r;                                              \
  } while (0)

template <class T> int geometry_path(lbm_ctx* c, int reproject) {
  Fields& F = c->F;
  if (reproject)
    LBM_HIP(c, lbm::launch_reproject<T>(F, c->stream, c->Fc, (T)c->tau));
  else
    LBM_HIP(c, lbm::launch_geometry<T>(F, c->stream, c->Fc));
  LBM_HIP(c, lbm::launch_wall_velocity<T>(F, c->stream));
  if (F.g.pj) LBM_HIP(c, lbm::launch_plate_velocity<T>(F, c->stream));
  if (F.g.open) LBM_HIP(c, lbm::launch_inlet_velocity<T>(F, c->stream));
  c->have_geo = 1;
  return LBM_OK;
}

int geometry_dispatch(lbm_ctx* c, int reproject) {
  if (reproject && !c->have_state) return fail(c, LBM_ESTATE, "re-projection needs a state");
  return c->precision == LBM_FP64 ? geometry_path<double>(c, reproject) : geometry_path<float>(c, reproject);
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_grid* h_grid, int lattice, int precision, int adjoint_K, int ckpt_every) {
  if (!grid_ok(h_grid) || lattice != LBM_D3Q19) return 0;
  if (precision != LBM_FP64 && precision != LBM_FP32_DEV) return 0;
  if (adjoint_K < 0 || (adjoint_K > 0 && (ckpt_every < 1 || ckpt_every > adjoint_K))) return 0;
  Carver c(nullptr);
  Fields F;
  carve_core(c, make_grid(h_grid), precision, F);
  if (adjoint_K > 0) {
    lbm::AdjointBuffers A;
    lbm::carve_adjoint(c, make_grid(h_grid), adjoint_K, ckpt_every, A);
  }
  return c.off + ALIGN;
}

int lbm_create(lbm_ctx** out, const lbm_grid* h_grid, int lattice, double tau, int precision, void* d_workspace,
               size_t bytes, void* hip_stream) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!grid_ok(h_grid) || lattice != LBM_D3Q19 || !(tau > 0.5) || !std::isfinite(tau) || !d_workspace)
    return LBM_EINVAL;
  if (precision != LBM_FP64 && precision != LBM_FP32_DEV) return LBM_EINVAL;
  if (((uintptr_t)d_workspace) % ALIGN) return LBM_EINVAL;
  const size_t need = lbm_workspace_bytes(h_grid, lattice, precision, 0, 0);
  if (bytes < need) return LBM_ENOMEM;
  lbm_ctx* c = new lbm_ctx();
  c->precision = precision;
  c->F.stage = default_stage(precision);
  c->tau = tau;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)d_workspace;
  c->bytes = bytes;
  Carver cv(c->ws);
  carve_core(cv, make_grid(h_grid), precision, c->F);
  c->used = cv.off;
  Fields& F = c->F;
  const size_t sz = precision == LBM_FP64 ? sizeof(double) : sizeof(float);
  hipError_t e = hipMemsetAsync(F.disp, 0, sizeof(double) * 2 * (size_t)F.g.nz * F.g.nx, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.vwall, 0, sizeof(double) * 6 * (size_t)F.g.nz * F.g.nx, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.uw, 0, sz * 6 * (size_t)F.g.nz * F.g.nx, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.up, 0, sz * 6 * (size_t)F.g.nz * F.g.nx, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.vplate, 0, sizeof(double) * 3 * (size_t)F.g.nz * F.g.nx, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.dplate, 0, sizeof(double) * (size_t)F.g.nz * F.g.nx, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.uin, 0, sizeof(double) * 3 * (size_t)F.g.nz * F.g.H, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.vin, 0, sz * 3 * (size_t)F.g.nz * F.g.H, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.flag, 0, ALIGN, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(F.count, 0, ALIGN, c->stream);
  if (e != hipSuccess) {
    delete c;
    return LBM_EHIP;
  }
  // address of the static scratch array on this (the current) device, for
  // lbm_wall_force_noalloc; a failure is reported by that call only
  int dev = 0;
  hipError_t de = hipGetDevice(&dev);
  if (de == hipSuccess) de = lbm::noalloc_scratch_init(dev, &c->scratch);
  c->scratch_rc = (int)de;
  *out = c;
  return LBM_OK;
}

int lbm_reserve_adjoint(lbm_ctx* c, int adjoint_K, int ckpt_every) {
  LBM_GUARD(c);
  if (adjoint_K < 1 || ckpt_every < 1 || ckpt_every > adjoint_K) return fail(c, LBM_EINVAL, "bad adjoint sizes");
  if (c->precision != LBM_FP64) return fail(c, LBM_EUNSUPPORTED, "the adjoint needs the FP64 form");
  Carver cv(c->ws);
  cv.off = c->used;
  lbm::AdjointBuffers A;
  lbm::carve_adjoint(cv, c->F.g, adjoint_K, ckpt_every, A);
  if (cv.off + ALIGN > c->bytes) return fail(c, LBM_ENOMEM, "workspace too small for the adjoint");
  c->adj = A;
  c->adjK = adjoint_K;
  c->adjN = ckpt_every;
  c->recorded = 0;
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  delete c;
  return LBM_OK;
}

int lbm_set_body_force(lbm_ctx* c, const double* F) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  if (!F || !std::isfinite(F[0]) || !std::isfinite(F[1]) || !std::isfinite(F[2]))
    return fail(c, LBM_EINVAL, "body force must be 3 finite numbers");
  for (int a = 0; a < 3; ++a) c->Fc[a] = F[a];
  if (c->have_geo) {
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_body_force<double>(c->F, c->stream, c->Fc));
    else
      LBM_HIP(c, lbm::launch_body_force<float>(c->F, c->stream, c->Fc));
  }
  return LBM_OK;
}

int lbm_set_metric(lbm_ctx* c, const double* d_chart, int reproject) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  if (!d_chart) return fail(c, LBM_EINVAL, "chart is NULL");
  if (reproject && !c->have_state) return fail(c, LBM_ESTATE, "re-projection needs a state");
  LBM_HIP(c, hipMemcpyAsync(c->F.chart, d_chart, sizeof(double) * 3 * c->F.NC, hipMemcpyDeviceToDevice, c->stream));
  c->F.chart_yonly = 0;
  return geometry_dispatch(c, reproject);
}

int lbm_set_wall_displacement(lbm_ctx* c, int wall, const double* d_disp, int reproject) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  if (wall != LBM_WALL_YMIN && wall != LBM_WALL_YMAX) return fail(c, LBM_EINVAL, "bad wall");
  if (reproject && !c->have_state) return fail(c, LBM_ESTATE, "re-projection needs a state");
  // the chart kernel takes the displacement from d_disp and stores it
  LBM_HIP(c, lbm::launch_chart_from_disp(c->F, c->stream, wall, d_disp));
  return geometry_dispatch(c, reproject);
}

int lbm_set_wall_velocity(lbm_ctx* c, int wall, const double* d_vcart) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  if (wall != LBM_WALL_YMIN && wall != LBM_WALL_YMAX) return fail(c, LBM_EINVAL, "bad wall");
  c->F.moving[wall] = d_vcart != nullptr;
  if (c->have_geo) {
    // the kernel takes the velocity from d_vcart, stores it and forms its
    // chart components
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_wall_velocity<double>(c->F, c->stream, wall, d_vcart));
    else
      LBM_HIP(c, lbm::launch_wall_velocity<float>(c->F, c->stream, wall, d_vcart));
    return LBM_OK;
  }
  const size_t n = (size_t)c->F.g.nz * c->F.g.nx * 3;
  double* dst = c->F.vwall + (size_t)wall * n;
  if (d_vcart)
    LBM_HIP(c, hipMemcpyAsync(dst, d_vcart, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  else
    LBM_HIP(c, zero_async(dst, n, c->stream));
  return LBM_OK;
}

int lbm_set_plate(lbm_ctx* c, int jp, int i0, int i1) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  Fields& F = c->F;
  if (jp == 0) {
    F.g.pj = 0;
    F.g.pi0 = 0;
    F.g.pi1 = -1;
    return LBM_OK;
  }
  if (jp < 1 || jp > F.g.H - 1 || i0 < 0 || i1 < i0 || i1 > F.g.nx - 1)
    return fail(c, LBM_EINVAL, "plate must lie between fluid rows 1..H-1 over columns 0..nx-1");
  if (F.g.open && (i0 < 3 || i1 > F.g.nx - 4))
    return fail(c, LBM_EINVAL, "with open ends the plate keeps 3 columns from each end");
  if (c->have_state) return fail(c, LBM_ESTATE, "set the plate before the state");
  F.g.pj = jp;
  F.g.pi0 = i0;
  F.g.pi1 = i1;
  const size_t ncol = (size_t)F.g.nz * F.g.nx;
  LBM_HIP(c, hipMemsetAsync(F.dplate, 0, sizeof(double) * ncol, c->stream));
  LBM_HIP(c, hipMemsetAsync(F.vplate, 0, sizeof(double) * 3 * ncol, c->stream));
  if (c->have_geo) {
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_plate_velocity<double>(F, c->stream));
    else
      LBM_HIP(c, lbm::launch_plate_velocity<float>(F, c->stream));
  }
  return LBM_OK;
}

int lbm_set_plate_displacement(lbm_ctx* c, const double* d_disp, int reproject) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  if (!c->F.g.pj) return fail(c, LBM_ESTATE, "no plate");
  if (reproject && !c->have_state) return fail(c, LBM_ESTATE, "re-projection needs a state");
  // the chart kernel takes the plate displacement from d_disp and stores it
  LBM_HIP(c, lbm::launch_chart_from_disp(c->F, c->stream, 2, d_disp));
  return geometry_dispatch(c, reproject);
}

int lbm_set_plate_velocity(lbm_ctx* c, const double* d_vcart) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  if (!c->F.g.pj) return fail(c, LBM_ESTATE, "no plate");
  if (c->have_geo) {
    // the kernel takes the velocity from d_vcart, stores it and forms its
    // chart components
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_plate_velocity<double>(c->F, c->stream, 1, d_vcart));
    else
      LBM_HIP(c, lbm::launch_plate_velocity<float>(c->F, c->stream, 1, d_vcart));
    return LBM_OK;
  }
  const size_t n = (size_t)c->F.g.nz * c->F.g.nx * 3;
  if (d_vcart)
    LBM_HIP(c, hipMemcpyAsync(c->F.vplate, d_vcart, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  else
    LBM_HIP(c, zero_async(c->F.vplate, n, c->stream));
  return LBM_OK;
}

int lbm_plate_force(lbm_ctx* c, double* d_total3, double* d_per_column) {
  LBM_GUARD(c);
  if (!c->F.g.pj) return fail(c, LBM_ESTATE, "no plate");
  if (!d_total3) return fail(c, LBM_EINVAL, "total output is NULL");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  if (c->precision == LBM_FP64)
    LBM_HIP(c, lbm::launch_wall_force<double>(c->F, c->stream, 2, c->tau, d_total3, d_per_column));
  else
    LBM_HIP(c, lbm::launch_wall_force<float>(c->F, c->stream, 2, (float)c->tau, d_total3, d_per_column));
  return LBM_OK;
}

int lbm_set_open_x(lbm_ctx* c, const double* d_uin) {
  LBM_GUARD(c);
  c->recorded = 0;  // a recorded trajectory no longer matches the fields
  Fields& F = c->F;
  if (c->have_state) return fail(c, LBM_ESTATE, "set the ends before the state");
  if (!d_uin) {
    F.g.open = 0;
    return LBM_OK;
  }
  if (F.g.nx < 4) return fail(c, LBM_EINVAL, "open ends need nx >= 4");
  if (F.g.pj && (F.g.pi0 < 3 || F.g.pi1 > F.g.nx - 4))
    return fail(c, LBM_EINVAL, "with open ends the plate keeps 3 columns from each end");
  F.g.open = 1;
  LBM_HIP(c, hipMemcpyAsync(F.uin, d_uin, sizeof(double) * 3 * (size_t)F.g.nz * F.g.H, hipMemcpyDeviceToDevice,
                            c->stream));
  if (c->have_geo) {
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_inlet_velocity<double>(F, c->stream));
    else
      LBM_HIP(c, lbm::launch_inlet_velocity<float>(F, c->stream));
  }
  return LBM_OK;
}

int lbm_init_equilibrium(lbm_ctx* c, const double* d_rho, const double* d_ucart) {
  LBM_GUARD(c);
  if (!c->have_geo) return fail(c, LBM_ESTATE, "set a metric first");
  if (c->precision == LBM_FP64) {
    LBM_HIP(c, lbm::launch_feq_full<double>(c->F, c->stream, d_rho, d_ucart));
    LBM_HIP(c, lbm::launch_set_state<double>(c->F, c->stream, c->F.full, c->tau));
  } else {
    LBM_HIP(c, lbm::launch_feq_full<float>(c->F, c->stream, d_rho, d_ucart));
    LBM_HIP(c, lbm::launch_set_state<float>(c->F, c->stream, c->F.full, (float)c->tau));
  }
  c->have_state = 1;
  c->recorded = 0;
  return LBM_OK;
}

int lbm_set_populations(lbm_ctx* c, const double* d_f) {
  LBM_GUARD(c);
  if (!d_f) return fail(c, LBM_EINVAL, "populations are NULL");
  if (!c->have_geo) return fail(c, LBM_ESTATE, "set a metric first");
  if (c->precision == LBM_FP64)
    LBM_HIP(c, lbm::launch_set_state<double>(c->F, c->stream, d_f, c->tau));
  else
    LBM_HIP(c, lbm::launch_set_state<float>(c->F, c->stream, d_f, (float)c->tau));
  c->have_state = 1;
  c->recorded = 0;
  return LBM_OK;
}

int lbm_get_populations(lbm_ctx* c, double* d_f) {
  LBM_GUARD(c);
  if (!d_f) return fail(c, LBM_EINVAL, "output is NULL");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  if (c->precision == LBM_FP64)
    LBM_HIP(c, lbm::launch_get_pops<double>(c->F, c->stream, d_f));
  else
    LBM_HIP(c, lbm::launch_get_pops<float>(c->F, c->stream, d_f));
  return LBM_OK;
}

int lbm_get_history(lbm_ctx* c, double* d_coef) {
  LBM_GUARD(c);
  if (!d_coef) return fail(c, LBM_EINVAL, "output is NULL");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  if (c->precision == LBM_FP64)
    LBM_HIP(c, lbm::launch_get_hist<double>(c->F, c->stream, d_coef));
  else
    LBM_HIP(c, lbm::launch_get_hist<float>(c->F, c->stream, d_coef));
  return LBM_OK;
}

int lbm_get_geometry(lbm_ctx* c, double* d_geo28, double* d_jac9) {
  LBM_GUARD(c);
  if (!c->have_geo) return fail(c, LBM_ESTATE, "no metric");
  if (d_geo28) {
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_get_geo<double>(c->F, c->stream, d_geo28));
    else
      LBM_HIP(c, lbm::launch_get_geo<float>(c->F, c->stream, d_geo28));
  }
  if (d_jac9)
    LBM_HIP(c, hipMemcpyAsync(d_jac9, c->F.jac, sizeof(double) * 9 * c->F.g.N, hipMemcpyDeviceToDevice, c->stream));
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int n) {
  LBM_GUARD(c);
  if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  for (int t = 0; t < n; ++t) {
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_step<double>(c->F, c->stream, c->tau));
    else
      LBM_HIP(c, lbm::launch_step<float>(c->F, c->stream, (float)c->tau));
  }
  if (n > 0) c->recorded = 0;
  return LBM_OK;
}

int lbm_step_force(lbm_ctx* c, int n, int wall, double* d_forces) {
  LBM_GUARD(c);
  if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
  if (wall != LBM_WALL_YMIN && wall != LBM_WALL_YMAX) return fail(c, LBM_EINVAL, "bad wall");
  if (n > 0 && !d_forces) return fail(c, LBM_EINVAL, "forces output is NULL");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  hipError_t e = c->precision == LBM_FP64
                     ? lbm::launch_steps_fused_force<double>(c->F, c->stream, c->tau, wall, n, d_forces)
                     : lbm::launch_steps_fused_force<float>(c->F, c->stream, (float)c->tau, wall, n, d_forces);
  if (e == hipErrorNotSupported) {
    // plate, open ends or the two-pass step: the force kernel, then the step
    for (int t = 0; t < n; ++t) {
      double* out = d_forces + 3 * (size_t)t;
      if (c->precision == LBM_FP64) {
        LBM_HIP(c, lbm::launch_wall_force<double>(c->F, c->stream, wall, c->tau, out, nullptr, 0));
        LBM_HIP(c, lbm::launch_step<double>(c->F, c->stream, c->tau));
      } else {
        LBM_HIP(c, lbm::launch_wall_force<float>(c->F, c->stream, wall, (float)c->tau, out, nullptr, 0));
        LBM_HIP(c, lbm::launch_step<float>(c->F, c->stream, (float)c->tau));
      }
    }
  } else {
    LBM_HIP(c, e);
  }
  if (n > 0) c->recorded = 0;
  return LBM_OK;
}

int lbm_step_profiled(lbm_ctx* c, int n, double* h_ms, int nslots) {
  LBM_GUARD(c);
  if (n < 1 || !h_ms || nslots < lbm::STEP_KERNELS) return fail(c, LBM_EINVAL, "bad profiling arguments");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  const int NK = lbm::STEP_KERNELS;
  std::vector<hipEvent_t> ev((size_t)n * (NK + 1), nullptr);
  int rc = LBM_OK;
  for (auto& e : ev)
    if (rc == LBM_OK) rc = hip_check(c, hipEventCreate(&e), "hipEventCreate");
  for (int t = 0; t < n && rc == LBM_OK; ++t) {
    hipError_t e = c->precision == LBM_FP64
                       ? lbm::launch_step<double>(c->F, c->stream, c->tau, &ev[(size_t)t * (NK + 1)])
                       : lbm::launch_step<float>(c->F, c->stream, (float)c->tau, &ev[(size_t)t * (NK + 1)]);
    rc = hip_check(c, e, "launch_step");
  }
  if (rc == LBM_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  for (int k = 0; k < nslots; ++k) h_ms[k] = 0.0;
  for (int t = 0; t < n && rc == LBM_OK; ++t)
    for (int k = 0; k < NK && rc == LBM_OK; ++k) {
      float ms = 0.f;
      rc = hip_check(c, hipEventElapsedTime(&ms, ev[(size_t)t * (NK + 1) + k], ev[(size_t)t * (NK + 1) + k + 1]),
                     "hipEventElapsedTime");
      h_ms[k] += ms / n;
    }
  for (auto& e : ev) {
    if (!e) continue;
    const hipError_t d = hipEventDestroy(e);
    if (rc == LBM_OK) rc = hip_check(c, d, "hipEventDestroy");
  }
  if (n > 0) c->recorded = 0;
  return rc;
}

int lbm_set_tuning(lbm_ctx* c, int zchunk, int variant, int stage) {
  LBM_GUARD(c);
  if (zchunk < 0 || variant < 0 || variant > 1 || stage < -1 || stage > 1)
    return fail(c, LBM_EINVAL, "bad tuning arguments");
  c->F.zc = zchunk;
  c->F.variant = variant;
  c->F.stage = stage >= 0 ? stage : default_stage(c->precision);
  return LBM_OK;
}

int lbm_get_tuning(lbm_ctx* c, int* zchunk, int* variant, int* stage) {
  LBM_GUARD(c);
  if (!zchunk || !variant || !stage) return fail(c, LBM_EINVAL, "null output pointer");
  int zc = 0;
  const bool two_pass = !lbm::step_is_fused(c->F);
  if (!two_pass)
    LBM_HIP(c, c->precision == LBM_FP64 ? lbm::fused_step_chunk<double>(c->F, &zc)
                                        : lbm::fused_step_chunk<float>(c->F, &zc));
  *zchunk = zc;
  *variant = two_pass ? 1 : 0;
  *stage = c->precision == LBM_FP64 ? 0 : c->F.stage;
  return LBM_OK;
}

int lbm_stream_probe(int precision, long long n, const void* d_in, void* d_out, void* hip_stream) {
  if (n < 1 || n >= MAX_FLUID_NODES || !d_in || !d_out || (precision != LBM_FP64 && precision != LBM_FP32_DEV))
    return LBM_EINVAL;
  return lbm::launch_stream_probe(precision == LBM_FP64 ? 0 : 1, n, d_in, d_out, (hipStream_t)hip_stream) ==
                 hipSuccess
             ? LBM_OK
             : LBM_EHIP;
}

int lbm_sync(lbm_ctx* c) {
  LBM_GUARD(c);
  LBM_HIP(c, hipStreamSynchronize(c->stream));
  int flag = 0;
  LBM_HIP(c, hipMemcpy(&flag, c->F.flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) return fail(c, LBM_EUNSTABLE, "instability guard: non-finite population, rho <= 0 or |u|^2 > 0.1");
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* d_rho, double* d_u, int cartesian) {
  LBM_GUARD(c);
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  if (d_rho || d_u) {
    if (c->precision == LBM_FP64)
      LBM_HIP(c, lbm::launch_moments_out<double>(c->F, c->stream, d_rho, d_u, cartesian));
    else
      LBM_HIP(c, lbm::launch_moments_out<float>(c->F, c->stream, d_rho, d_u, cartesian));
  }
  return lbm_sync(c);
}

int lbm_wall_force(lbm_ctx* c, int wall, int method, double* d_total3, double* d_per_node) {
  LBM_GUARD(c);
  if (wall != LBM_WALL_YMIN && wall != LBM_WALL_YMAX) return fail(c, LBM_EINVAL, "bad wall");
  if (method != LBM_FORCE_STRESS && method != LBM_FORCE_MEM) return fail(c, LBM_EINVAL, "bad force method");
  if (!d_total3) return fail(c, LBM_EINVAL, "total output is NULL");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  const int mem = method == LBM_FORCE_MEM;
  if (mem && c->F.moving[wall])
    return fail(c, LBM_EUNSUPPORTED, "the momentum-exchange force is provided for a wall at rest");
  if (c->precision == LBM_FP64)
    LBM_HIP(c, lbm::launch_wall_force<double>(c->F, c->stream, wall, c->tau, d_total3, d_per_node, mem));
  else
    LBM_HIP(c, lbm::launch_wall_force<float>(c->F, c->stream, wall, (float)c->tau, d_total3, d_per_node, mem));
  return LBM_OK;
}

int lbm_wall_force_noalloc(lbm_ctx* c, int wall, int method, double* d_total3, double* d_per_node) {
  LBM_GUARD(c);
  if (wall != LBM_WALL_YMIN && wall != LBM_WALL_YMAX) return fail(c, LBM_EINVAL, "bad wall");
  if (method != LBM_FORCE_STRESS && method != LBM_FORCE_MEM) return fail(c, LBM_EINVAL, "bad force method");
  if (!d_total3) return fail(c, LBM_EINVAL, "total output is NULL");
  if (lbm::wall_force_blocks(c->F.g) > lbm::NOALLOC_MAX_BLOCKS)
    return fail(c, LBM_EINVAL, "lbm_wall_force_noalloc: nx * nz exceeds LBM_NOALLOC_MAX_COLUMNS");
  if (c->scratch_rc != (int)hipSuccess || !c->scratch)
    return hip_check(c, c->scratch_rc != (int)hipSuccess ? (hipError_t)c->scratch_rc : hipErrorInvalidValue,
                     "lbm_wall_force_noalloc: static scratch address");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  const int mem = method == LBM_FORCE_MEM;
  if (mem && c->F.moving[wall])
    return fail(c, LBM_EUNSUPPORTED, "the momentum-exchange force is provided for a wall at rest");
  if (c->precision == LBM_FP64)
    LBM_HIP(c, lbm::launch_wall_force_noalloc<double>(c->F, c->stream, wall, c->tau, d_total3, d_per_node, mem,
                                                      c->scratch));
  else
    LBM_HIP(c, lbm::launch_wall_force_noalloc<float>(c->F, c->stream, wall, (float)c->tau, d_total3, d_per_node,
                                                     mem, c->scratch));
  return LBM_OK;
}

int lbm_couple(lbm_ctx* c, int wall, const double* d_disp, const double* d_vcart, int n, double* d_total3,
               double* d_per_node) {
  LBM_GUARD(c);
  if (wall != LBM_WALL_YMIN && wall != LBM_WALL_YMAX) return fail(c, LBM_EINVAL, "bad wall");
  if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
  if (!d_total3) return fail(c, LBM_EINVAL, "total output is NULL");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  int rc = LBM_OK;
  if (d_disp) rc = lbm_set_wall_displacement(c, wall, d_disp, 1);
  if (rc == LBM_OK) rc = lbm_set_wall_velocity(c, wall, d_vcart);
  if (rc == LBM_OK) rc = lbm_step(c, n);
  if (rc == LBM_OK) rc = lbm_wall_force(c, wall, LBM_FORCE_STRESS, d_total3, d_per_node);
  return rc;
}

int lbm_forward_record(lbm_ctx* c, int K, int ckpt_every, int wall, int method, double* d_forces) {
  LBM_GUARD(c);
  if (c->precision != LBM_FP64) return fail(c, LBM_EUNSUPPORTED, "the adjoint needs the FP64 form");
  if (K != c->adjK || ckpt_every != c->adjN || K < 1) return fail(c, LBM_EINVAL, "K / ckpt_every do not match the reservation");
  if (wall != LBM_WALL_YMIN && wall != LBM_WALL_YMAX) return fail(c, LBM_EINVAL, "bad wall");
  if (method != LBM_FORCE_STRESS) return fail(c, LBM_EUNSUPPORTED, "only the stress method is provided");
  if (!d_forces) return fail(c, LBM_EINVAL, "forces output is NULL");
  if (!c->have_state) return fail(c, LBM_ESTATE, "no state");
  if (c->F.g.pj) return fail(c, LBM_EUNSUPPORTED, "the adjoint does not cover an interior plate");
  if (c->F.g.open) return fail(c, LBM_EUNSUPPORTED, "the adjoint does not cover open ends");
  {
    hipError_t e = lbm::adjoint_forward(c->F, c->adj, c->stream, K, ckpt_every, wall, c->tau, d_forces);
    if (e == hipErrorNotSupported) return fail(c, LBM_EUNSUPPORTED, "adjoint not available in this build");
    LBM_HIP(c, e);
  }
  c->recorded = 1;
  c->rec_wall = wall;
  return LBM_OK;
}

int lbm_backward(lbm_ctx* c, const double* d_dL_dF, double* d_grad_disp, double* d_grad_chart, double* d_grad_f0) {
  LBM_GUARD(c);
  if (!c->recorded) return fail(c, LBM_ESTATE, "backward needs a prior forward_record");
  if (!d_dL_dF) return fail(c, LBM_EINVAL, "dL/dF is NULL");
  {
    hipError_t e = lbm::adjoint_backward(c->F, c->adj, c->stream, c->adjK, c->adjN, c->rec_wall, c->tau, c->Fc,
                                         d_dL_dF, d_grad_disp, d_grad_chart, d_grad_f0);
    if (e == hipErrorNotSupported) return fail(c, LBM_EUNSUPPORTED, "adjoint not available in this build");
    LBM_HIP(c, e);
  }
  return lbm_sync(c);
}

const char* lbm_last_error(const lbm_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

}  // extern "C"
