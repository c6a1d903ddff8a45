// A caller of liblbm that uses only the C-ABI in include/lbm.h, with device
// memory from the HIP runtime: no Python and no torch.  It runs the sheared
// 32x16x16 channel (tau 0.8, body force 1e-6 along x, the top wall's
// displacement read from a file) in FP64, and writes rho [fluid], the
// Cartesian u [3][fluid], the top-wall force [3] and then the top-wall forces
// of 4 more steps taken with lbm_step_force [4][3] to an output file, so a
// test can compare them with the same calls made through the Python binding.
//
// Usage: lbm_c_caller DISP.bin STEPS OUT.bin   (DISP.bin: nz*nx doubles)
// Prints one JSON line; exit status 0 when every call returned LBM_OK.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lbm.h"

namespace {

int first_error = LBM_OK;
const char* first_call = "";

// Record the first failing call (its name and status).
void check(int rc, const char* what) {
  if (rc != LBM_OK && first_error == LBM_OK) {
    first_error = rc;
    first_call = what;
  }
}

bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return false;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: %s DISP.bin STEPS OUT.bin\n", argv[0]);
    return 2;
  }
  const int nx = 32, ny = 16, nz = 16, H = ny - 2;
  const lbm_grid grid = {nx, ny, nz};
  const size_t ncol = (size_t)nz * nx, nf = (size_t)nx * H * nz;
  const int steps = std::atoi(argv[2]);

  std::vector<double> disp(ncol);
  FILE* fin = std::fopen(argv[1], "rb");
  if (!fin || std::fread(disp.data(), sizeof(double), ncol, fin) != ncol) {
    std::fprintf(stderr, "cannot read %zu doubles from %s\n", ncol, argv[1]);
    return 2;
  }
  std::fclose(fin);

  const size_t bytes = lbm_workspace_bytes(&grid, LBM_D3Q19, LBM_FP64, 0, 0);
  void* ws = nullptr;
  double *d_disp = nullptr, *d_rho = nullptr, *d_u = nullptr, *d_force = nullptr, *d_forces = nullptr;
  const int nsf = 4;  // steps of lbm_step_force
  if (!hip_ok(hipMalloc(&ws, bytes), "hipMalloc workspace") ||
      !hip_ok(hipMalloc((void**)&d_disp, sizeof(double) * ncol), "hipMalloc disp") ||
      !hip_ok(hipMalloc((void**)&d_rho, sizeof(double) * nf), "hipMalloc rho") ||
      !hip_ok(hipMalloc((void**)&d_u, sizeof(double) * 3 * nf), "hipMalloc u") ||
      !hip_ok(hipMalloc((void**)&d_force, sizeof(double) * 3), "hipMalloc force") ||
      !hip_ok(hipMalloc((void**)&d_forces, sizeof(double) * 3 * nsf), "hipMalloc forces") ||
      !hip_ok(hipMemcpy(d_disp, disp.data(), sizeof(double) * ncol, hipMemcpyHostToDevice), "hipMemcpy disp"))
    return 1;

  lbm_ctx* ctx = nullptr;
  check(lbm_create(&ctx, &grid, LBM_D3Q19, 0.8, LBM_FP64, ws, bytes, nullptr), "lbm_create");
  if (!ctx) {
    std::printf("{\"status\": %d, \"failed\": \"%s\"}\n", first_error, first_call);
    return 1;
  }
  // the call order is enforced: a step before any state is refused
  const int early = lbm_step(ctx, 1);
  const char* early_msg = lbm_last_error(ctx);
  std::printf("# early step: %d (%s)\n", early, early_msg);

  const double body[3] = {1e-6, 0.0, 0.0};
  check(lbm_set_body_force(ctx, body), "lbm_set_body_force");
  check(lbm_set_wall_displacement(ctx, LBM_WALL_YMAX, d_disp, 0), "lbm_set_wall_displacement");
  check(lbm_init_equilibrium(ctx, nullptr, nullptr), "lbm_init_equilibrium");
  check(lbm_step(ctx, steps), "lbm_step");
  check(lbm_moments(ctx, d_rho, d_u, 1), "lbm_moments");
  check(lbm_wall_force(ctx, LBM_WALL_YMAX, LBM_FORCE_STRESS, d_force, nullptr), "lbm_wall_force");
  check(lbm_step_force(ctx, nsf, LBM_WALL_YMAX, d_forces), "lbm_step_force");
  check(lbm_sync(ctx), "lbm_sync");

  std::vector<double> out(nf + 3 * nf + 3 + 3 * nsf);
  if (!hip_ok(hipMemcpy(out.data(), d_rho, sizeof(double) * nf, hipMemcpyDeviceToHost), "hipMemcpy rho") ||
      !hip_ok(hipMemcpy(out.data() + nf, d_u, sizeof(double) * 3 * nf, hipMemcpyDeviceToHost), "hipMemcpy u") ||
      !hip_ok(hipMemcpy(out.data() + 4 * nf, d_force, sizeof(double) * 3, hipMemcpyDeviceToHost), "hipMemcpy force") ||
      !hip_ok(hipMemcpy(out.data() + 4 * nf + 3, d_forces, sizeof(double) * 3 * nsf, hipMemcpyDeviceToHost),
              "hipMemcpy forces"))
    return 1;
  FILE* fout = std::fopen(argv[3], "wb");
  if (!fout || std::fwrite(out.data(), sizeof(double), out.size(), fout) != out.size()) {
    std::fprintf(stderr, "cannot write %s\n", argv[3]);
    return 1;
  }
  std::fclose(fout);

  double mass = 0.0;
  for (size_t n = 0; n < nf; ++n) mass += out[n];
  std::printf("{\"status\": %d, \"failed\": \"%s\", \"early_step\": %d, \"steps\": %d, \"mass\": %.17g, "
              "\"force\": [%.17g, %.17g, %.17g]}\n",
              first_error, first_call, early, steps, mass, out[4 * nf], out[4 * nf + 1], out[4 * nf + 2]);
  check(lbm_destroy(ctx), "lbm_destroy");
  hipFree(d_forces);
  hipFree(d_force);
  hipFree(d_u);
  hipFree(d_rho);
  hipFree(d_disp);
  hipFree(ws);
  return first_error == LBM_OK ? 0 : 1;
}
