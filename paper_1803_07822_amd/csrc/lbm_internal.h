// Host-side launchers shared between the kernel translation units and the
// C-ABI implementation.  Every launcher enqueues on the given stream and
// returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

// Device buffers of one context, carved from the caller's workspace.
struct Fields {
  Grid g;
  long long NE;   // nodes of the y-extended grid, nz * (ny + 6) * nx
  long long NC;   // nodes of the full grid, nz * ny * nx
  double* chart;  // [3][NC] current chart
  double* uext[2];// [3][NE] chart displacement on the extended grid (current / previous)
  double* vtmp;   // [3][NE]
  double* gext;   // [6][NE]
  double* wext;   // [6][NE]
  double* jac;    // [9][N] J = dh/dxi at fluid nodes
  void* geo;      // [28][N] T
  void* pop[2];   // [19][N] T
  void* hist[2];  // [10][N] T forcing history, flips with the populations
  void* mom;      // [4][N] T
  void* uw;       // [2][nz][nx][3] T
  void* up;       // [2][nz][nx][3] T plate velocity, chart components at the node below (0) / above (1)
  double* vplate; // [nz][nx][3] Cartesian plate velocity per column
  double* dplate; // [nz][nx] y-displacement of the plate's cross-section row
  double* uin;    // [nz][H][3] Cartesian inlet velocity (open ends)
  void* vin;      // [nz][H][3] T inlet velocity in the chart components of the inlet nodes
  double* disp;   // [2][nz][nx]
  double* vwall;  // [2][nz][nx][3] Cartesian wall velocity
  double* full;   // [19][N] FP64 scratch
  void* mf;       // [NC][20] T: Cartesian moment fields for re-projection, deviations from rest
  double* part;   // wall-force reduction: 3 doubles per block
  unsigned* count;// wall-force reduction: blocks done (zero between launches)
  double* fpart;  // wall force of the fused step: two halves of 3 doubles per (tile column, z chunk), nx/64 * nz each
  int* flag;      // instability guard
  int cur;        // index of the current population and history buffers
  int uext_cur;   // index of the current extended displacement
  // The chart, and the chart each extended displacement was built from, moves
  // the nodes along y only (it was built from wall and plate displacements):
  // their x and z displacements are exactly zero.  A chart given whole counts
  // as general.
  int chart_yonly = 0;
  int uext_yonly[2] = {0, 0};
  // the x and z components of the smoothed displacement (vtmp) are zero
  int vtmp_xz_zero = 0;
  // jac holds the rows (1, 0, 0) and (0, 0, 1) of such a chart
  int jac_rows_exact = 0;
  int moving[2];
  int zc = 0;        // planes per block of the fused step (0 = automatic)
  int variant = -1;  // -1: automatic (step_is_fused); 0: fused step; 1: two-pass step (moments pass + collision pass)
  int stage = 1;     // FP32 fused step keeps pulled populations in registers
  // resident blocks on the device of the fused-step instances used so far
  // (key of the instance, count), so that alternating lbm_step and
  // lbm_step_force query the device once per instance
  int slots_key[4] = {-1, -1, -1, -1};
  long long slots[4] = {0, 0, 0, 0};
};

constexpr int BX = 64, BY = 4;

// Open ends run the fused step followed by two small passes over the end
// columns; those passes cost a fixed few tens of microseconds, so below this
// many fluid nodes the automatic choice is the two-pass step.
constexpr long long OPEN_FUSED_MIN_NODES = 1LL << 20;

// The step a launch runs: the fused kernel, or the two-pass kernels.
inline bool step_is_fused(const Fields& F) {
  if (F.variant >= 0) return F.variant == 0;
  return !F.g.open || F.g.N >= OPEN_FUSED_MIN_NODES;
}
constexpr size_t ALIGN = 256;

// Carves the caller's workspace into aligned buffers; with base == nullptr it
// only counts bytes (used by lbm_workspace_bytes).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(char* b) : base(b) {}
  void* take(size_t n) {
    off = (off + ALIGN - 1) / ALIGN * ALIGN;
    void* p = base ? base + off : nullptr;
    off += n;
    return p;
  }
};

inline dim3 fluid_grid(const Grid& g) { return dim3((g.nx + BX - 1) / BX, (g.H + BY - 1) / BY, g.nz); }
inline dim3 ext_grid(const Grid& g) { return dim3((g.nx + BX - 1) / BX, (g.ny + 6 + BY - 1) / BY, g.nz); }
inline dim3 col_grid(const Grid& g) { return dim3((g.nx + BX - 1) / BX, (g.nz + BY - 1) / BY, 1); }

// XCD-aware numbering of the fluid-grid blocks (64 x 4 tiles, one z-plane
// each).  The hardware deals blocks round-robin over the 8 XCDs; with a 1D
// launch padded to a multiple of 8 * XCD_TILES blocks, each XCD takes groups
// of XCD_TILES consecutive tiles in x-fastest order, the XCDs taking
// consecutive groups in turn: the neighbour rows a node reads mostly sit in
// its own L2, and all XCDs stream neighbouring memory (one contiguous range
// per XCD was 2.6 % slower for the re-projection at 512x256x256).
constexpr int XCD_TILES = 32;
inline dim3 xcd_fluid_grid(const Grid& g) {
  const long long nb = (long long)((g.nx + BX - 1) / BX) * ((g.H + BY - 1) / BY) * g.nz, sweep = 8LL * XCD_TILES;
  return dim3((unsigned)((nb + sweep - 1) / sweep * sweep));
}

__device__ __forceinline__ bool xcd_fluid_node(const Grid& g, int& i, int& jf, int& k) {
  const int ntx = (g.nx + BX - 1) / BX, nty = (g.H + BY - 1) / BY;
  const int nb = ntx * nty * g.nz;
  const int xs = (int)(blockIdx.x % 8), sl = (int)(blockIdx.x / 8);
  const int t = ((sl / XCD_TILES) * 8 + xs) * XCD_TILES + sl % XCD_TILES;
  if (t >= nb) return false;
  i = (t % ntx) * BX + threadIdx.x;
  jf = ((t / ntx) % nty) * BY + threadIdx.y;
  k = t / (ntx * nty);
  return i < g.nx && jf < g.H;
}

// bandwidth calibration: 57 planes of n read, 29 written (precision 0 = FP64)
hipError_t launch_stream_probe(int precision, long long n, const void* in, void* out, hipStream_t s);

// geometry (FP64 precompute; writes geo in precision T)
template <class T> hipError_t launch_geometry(Fields& F, hipStream_t s, const double Fc[3]);
template <class T> hipError_t launch_body_force(Fields& F, hipStream_t s, const double Fc[3]);
// The velocity and chart launchers can also take a new input for one field
// (which: wall 0 or 1, for the chart 2 = plate; -1 none) straight from the
// caller's device array (NULL: zero): the kernel stores it into the context's
// copy, in place of a separate copy launch.
template <class T> hipError_t launch_wall_velocity(Fields& F, hipStream_t s, int which = -1, const double* src = nullptr);
template <class T> hipError_t launch_plate_velocity(Fields& F, hipStream_t s, int in = 0, const double* src = nullptr);
template <class T> hipError_t launch_inlet_velocity(Fields& F, hipStream_t s);
hipError_t launch_chart_from_disp(Fields& F, hipStream_t s, int which = -1, const double* src = nullptr);

// state
template <class T> hipError_t launch_feq_full(Fields& F, hipStream_t s, const double* rho, const double* uc);
template <class T> hipError_t launch_set_state(Fields& F, hipStream_t s, const double* f, T tau);
template <class T> hipError_t launch_get_pops(Fields& F, hipStream_t s, double* out);
template <class T> hipError_t launch_get_hist(Fields& F, hipStream_t s, double* out);
template <class T> hipError_t launch_get_geo(Fields& F, hipStream_t s, double* out);
constexpr int STEP_KERNELS = 2;  // at most this many kernels per step (timed separately by lbm_step_profiled)
template <class T> hipError_t launch_step(Fields& F, hipStream_t s, T tau, hipEvent_t* ev = nullptr);
template <class T> hipError_t launch_step_fused(Fields& F, hipStream_t s, T tau, int zc);
// Output of the fused step's wall force (WF instantiation): the wall, J at
// the fluid nodes, this step's partial sums, and the previous step's partial
// sums (count and destination of their total; prev_part null for none).
struct WallOut {
  int wall;
  const double* jac;
  double* part;
  const double* prev_part;
  int prev_n;
  double* prev_out;
};
// n fused steps (automatic z chunk) that also write the stress-method force on
// `wall` of each state stepped from to out[3 t]; hipErrorNotSupported (before
// any launch) for grids with a plate or open ends or with the two-pass step
// selected.
template <class T> hipError_t launch_steps_fused_force(Fields& F, hipStream_t s, T tau, int wall, int n, double* out);
// Fused step (64x4 tiles, no staging) that also writes rho and rho u of the
// state it steps from to mout [4][N]; periodic grids without a plate only.
template <class T> hipError_t launch_step_fused_moments(Fields& F, hipStream_t s, T tau, T* mout);
// Planes per block the fused step runs with (F.zc, or the automatic choice).
template <class T> hipError_t fused_step_chunk(Fields& F, int* zc);
template <class T> hipError_t launch_moments_out(Fields& F, hipStream_t s, double* rho, double* u, int cart);
// Wall force: one column per thread, blocks of WF_THREADS.
constexpr int WF_THREADS = 256;
inline long long wall_force_blocks(const Grid& g) { return ((long long)g.nx * g.nz + WF_THREADS - 1) / WF_THREADS; }
// wall 0 / 1: the walls; wall 2: the interior plate (both faces, plate
// columns).  mem != 0: momentum exchange (walls at rest) instead of traction.
// The reduction scratch is part [3 * wall_force_blocks] and count (zero on
// entry, zero again on exit), the context's own unless part is given.
template <class T> hipError_t launch_wall_force(Fields& F, hipStream_t s, int wall, T tau, double* total,
                                                double* per_node, int mem = 0, double* part = nullptr,
                                                unsigned* count = nullptr);
template <class T> hipError_t launch_reproject(Fields& F, hipStream_t s, const double Fc[3], T tau);

// Allocation-free wall force: the reduction scratch is a static device array
// of the library (at most NOALLOC_MAX_BLOCKS blocks, i.e.
// WF_THREADS * NOALLOC_MAX_BLOCKS wall columns).  noalloc_scratch_init resolves its
// address on device dev (which must be current) once and returns it;
// launch_wall_force_noalloc takes that address.
constexpr long long NOALLOC_MAX_BLOCKS = 2048;
hipError_t noalloc_scratch_init(int dev, void** out);
template <class T> hipError_t launch_wall_force_noalloc(Fields& F, hipStream_t s, int wall, T tau, double* total,
                                                        double* per_node, int mem, void* scratch);

}  // namespace lbm
