// Fused single-kernel time step (plane marching).
//
// A block owns a TX x TY tile of the (x, y) plane and marches along a chunk of
// ZC planes in z.  The lattice gradient d_k(rho u^i) needs the momentum of all
// 18 neighbours before any collision, so the block keeps the moments
// (rho - 1, rho u) of consecutive planes of its tile plus a one-node halo in
// an LDS ring: at plane z it forms the moments of plane z+1, then collides
// plane z (which reads planes z-1, z, z+1).  In FP32 each thread keeps the 19 pulled populations of
// its own node in registers from the moment pass to the collision one
// iteration later; in FP64 (no register room) the collision pulls them again,
// from the caches.  The halo entries are pulled by the block as well, and
// those reads mostly hit L2.
// Blocks are numbered so that each XCD gets groups of consecutive tiles,
// which keeps the halo reads of neighbouring tiles in one L2.
//
// The population layout, the streamed value g_l and the collision are those
// of the two-pass form (pull layout with bounce-back slots, deviation
// variables); see the state kernels for the layout.
#include "lbm_internal.h"

namespace lbm {

namespace {

// Tiles per XCD group of the fused step's block order (XCD_TILES).  A
// contiguous range of tiles per XCD (each XCD on its own z chunks) was 8 %
// slower at 512x256x256 (2.79 against 2.59 ms per FP32 step); groups of 16 or
// 32 tiles are as fast as plain block order there and as fast as the
// contiguous ranges at 256x128x128, where plain order was 12 % slower.
constexpr int XCD_GROUP = XCD_TILES;

template <int TX, int TY> struct Tile {
  static constexpr int NT = TX * TY;
  static constexpr int HX = TX + 2;
  static constexpr int HY = TY + 2;
  static constexpr int HN = HX * HY;  // haloed tile
};

__device__ __forceinline__ int wrapf(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Neighbour offsets of one fluid node in 32-bit element units: the source of
// a pull in direction l is n + ox[x] + oz[z] - y*nx (periodic wraps folded in),
// and every plane l is addressed as a uniform base plus that offset.
struct NodeIdx {
  unsigned n;         // fluid index
  int oxm, oxp;       // offset to i-1 and to i+1 (wrapped)
  int ozm, ozp;       // offset to k-1 and to k+1 (wrapped), in whole planes
  int jf;
  unsigned cut;       // plate: bit cut_bit(x, y) set when the link arriving along (x, y) is cut
};

// Bit of the link arriving along (x, y), y != 0, in NodeIdx::cut.
__host__ __device__ constexpr int cut_bit(int x, int y) { return (y > 0 ? 0 : 3) + x + 1; }

// PL: the grid has an interior plate (the links it cuts are found once per
// node); without it the mask stays zero and the pulls do not test it.
template <bool PL = false>
__device__ __forceinline__ NodeIdx node_idx(const Grid& g, int i, int jf, int k) {
  NodeIdx r;
  r.cut = 0;
  if constexpr (PL) {
#pragma unroll
    for (int x = -1; x <= 1; ++x) {
      if (plate_cut(g, i, jf, -x, -1)) r.cut |= 1u << cut_bit(x, 1);
      if (plate_cut(g, i, jf, -x, 1)) r.cut |= 1u << cut_bit(x, -1);
    }
  }
  const int plane = g.H * g.nx;
  r.n = (unsigned)(k * plane + jf * g.nx + i);
  r.oxm = i == 0 ? g.nx - 1 : -1;
  r.oxp = i == g.nx - 1 ? 1 - g.nx : 1;
  r.ozm = k == 0 ? (g.nz - 1) * plane : -plane;
  r.ozp = k == g.nz - 1 ? (1 - g.nz) * plane : plane;
  r.jf = jf;
  return r;
}

// Element e of a plane given by a uniform base pointer: the byte offset is
// formed in 32 bits so that loads and stores use a scalar base register plus
// one 32-bit vector offset.
template <class T> __device__ __forceinline__ const T& at(const T* __restrict__ base, unsigned e) {
  return *(const T*)((const char*)base + (e * (unsigned)sizeof(T)));
}
// Streaming store: the step's outputs are not read again within the step.
template <class T> __device__ __forceinline__ void stw(T* __restrict__ base, unsigned e, T v) {
  __builtin_nontemporal_store(v, base + (size_t)e);
}

// Pulled deviation g~_l: the population that left x - c_l in direction l,
// or the bounce-back slot opp(l) of this node when the link from x - c_l
// crosses a wall or the plate.
// Both candidate planes (l and opp(l)) are addressed from the lower of the
// two as one uniform base, so the per-lane choice is a choice of 32-bit
// offset and every load keeps the scalar-base form.
template <class T, int l, bool PL = false>
__device__ __forceinline__ T pullf(const T* __restrict__ pop, const Grid& g, const NodeIdx& p) {
  constexpr int x = cx(l), y = cy(l), z = cz(l);
  constexpr int lo = l < opp(l) ? l : opp(l);
  const T* base = pop + (size_t)lo * g.N;
  int off = -y * g.nx;
  if (x > 0) off += p.oxm;
  if (x < 0) off += p.oxp;
  if (z > 0) off += p.ozm;
  if (z < 0) off += p.ozp;
  const unsigned e = (unsigned)(l - lo) * (unsigned)g.N + (unsigned)((int)p.n + off);
  if constexpr (y == 0) {
    return at(base, e);
  } else {
    bool wall = y > 0 ? p.jf == 0 : p.jf == g.H - 1;
    if constexpr (PL) wall = wall || ((p.cut >> cut_bit(x, y)) & 1u);
    const unsigned eb = (unsigned)(opp(l) - lo) * (unsigned)g.N + p.n;
    return at(base, wall ? eb : e);
  }
}

template <class T> __device__ __forceinline__ T fld(const T* __restrict__ a, int q, const Grid& g, unsigned n) {
  return at(a + (size_t)q * g.N, n);
}
// Streaming load of a field read once per step.
template <class T> __device__ __forceinline__ T fldnt(const T* __restrict__ a, int q, const Grid& g, unsigned n) {
  const T* plane = a + (size_t)q * g.N;
  return __builtin_nontemporal_load(plane + (size_t)n);
}

// Discards the pulled deviations of a node.
struct NoKeep {
  template <class L, class T> __device__ void operator()(L, T) const {}
};

// rho - 1 and rho u of the streamed state at a fluid node; each pulled
// deviation g~_l is also handed to keep(l, g~_l).
template <class T, bool PL, class Keep = NoKeep>
__device__ __forceinline__ void node_moments(const T* __restrict__ pop, const T* __restrict__ hist,
                                             const T* __restrict__ geo, const Grid& g, int i, int jf, int k, T m[4],
                                             const Keep& keep = Keep()) {
  const NodeIdx p = node_idx<PL>(g, i, jf, k);
  T s = 0, j0 = 0, j1 = 0, j2 = 0;
  for_q([&](auto L) {
    constexpr int l = decltype(L)::value;
    const T v = pullf<T, l, PL>(pop, g, p);
    keep(L, v);
    s += v;
    if (cx(l)) j0 += T(cx(l)) * v;
    if (cy(l)) j1 += T(cy(l)) * v;
    if (cz(l)) j2 += T(cz(l)) * v;
  });
  const T sgd = fld(geo, G_SG, g, p.n);
  const T sg = T(1) + sgd;
  m[0] = sgd + sg * s + T(0.5) * fld(hist, H_A, g, p.n);
  m[1] = sg * j0 + T(0.5) * fld(hist, H_B + 0, g, p.n);
  m[2] = sg * j1 + T(0.5) * fld(hist, H_B + 1, g, p.n);
  m[3] = sg * j2 + T(0.5) * fld(hist, H_B + 2, g, p.n);
}

// Moments of entry e of the haloed tile at plane k into the ring slot.  Wall
// layers (jf = -1, H) get the mirror ghost of the adjacent fluid node.  A
// fluid entry hands its pulled deviations to `keep`.
template <class T, int TX, int TY, bool PL, class Keep = NoKeep>
__device__ __forceinline__ void fill_entry(T (*ring)[(TX + 2) * (TY + 2)], const T* __restrict__ pop,
                                           const T* __restrict__ hist, const T* __restrict__ geo,
                                           const T* __restrict__ uw, int mv0, int mv1, const Grid& g, int i0,
                                           int j0, int k, int e, const Keep& keep = Keep()) {
  constexpr int HX = Tile<TX, TY>::HX;
  const int hx = e % HX, hy = e / HX;
  const int i = i0 - 1 + hx, jf = j0 - 1 + hy;
  if (i > g.nx || jf > g.H) return;  // beyond a ragged tile edge: never read
  const int iw = wrapf(i, g.nx);
  T m[4];
  if (jf >= 0 && jf < g.H) {
    node_moments<T, PL>(pop, hist, geo, g, iw, jf, k, m, keep);
  } else {
    const int w = jf < 0 ? 0 : 1;
    T mm[4];
    node_moments<T, PL>(pop, hist, geo, g, iw, w == 0 ? 0 : g.H - 1, k, mm);
    m[0] = mm[0];
    m[1] = -mm[1];
    m[2] = -mm[2];
    m[3] = -mm[3];
    if (w == 0 ? mv0 : mv1) {
      const T r2 = T(2) * (T(1) + mm[0]);
      const long long c = (((long long)w * g.nz + k) * g.nx + iw) * 3;
      m[1] += r2 * uw[c];
      m[2] += r2 * uw[c + 1];
      m[3] += r2 * uw[c + 2];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) ring[q][e] = m[q];
}

// Fill one ring slot with the moments of plane k over the haloed tile.
template <class T, int TX, int TY, bool PL>
__device__ __forceinline__ void fill_plane(T (*ring)[(TX + 2) * (TY + 2)], const T* __restrict__ pop, const T* __restrict__ hist,
                                           const T* __restrict__ geo, const T* __restrict__ uw, int mv0, int mv1,
                                           const Grid& g, int i0, int j0, int k) {
  k = wrapf(k, g.nz);
  for (int e = threadIdx.x; e < Tile<TX, TY>::HN; e += Tile<TX, TY>::NT)
    fill_entry<T, TX, TY, PL>(ring, pop, hist, geo, uw, mv0, mv1, g, i0, j0, k, e);
}

// Staged fill: each thread fills the entry of its own node (handing that
// node's pulled deviations to `keep`, for the collision one iteration later);
// the 2*(TX+2) + 2*TY halo entries are shared out over the block.
template <class T, int TX, int TY, bool PL, class Keep>
__device__ __forceinline__ void fill_plane_staged(T (*ring)[(TX + 2) * (TY + 2)], const T* __restrict__ pop,
                                                  const T* __restrict__ hist, const T* __restrict__ geo,
                                                  const T* __restrict__ uw, int mv0, int mv1, const Grid& g, int i0,
                                                  int j0, int k, int tx, int ty, const Keep& keep) {
  constexpr int HX = Tile<TX, TY>::HX;
  k = wrapf(k, g.nz);
  fill_entry<T, TX, TY, PL>(ring, pop, hist, geo, uw, mv0, mv1, g, i0, j0, k, (ty + 1) * HX + (tx + 1), keep);
  constexpr int NH = 2 * HX + 2 * TY;
  for (int h = threadIdx.x; h < NH; h += Tile<TX, TY>::NT) {
    int e;
    if (h < HX)
      e = h;
    else if (h < 2 * HX)
      e = (TY + 1) * HX + (h - HX);
    else if (h < 2 * HX + TY)
      e = (1 + h - 2 * HX) * HX;
    else
      e = (1 + h - 2 * HX - TY) * HX + (HX - 1);
    fill_entry<T, TX, TY, PL>(ring, pop, hist, geo, uw, mv0, mv1, g, i0, j0, k, e);
  }
}

// Where the pulled deviations of a plane wait between its moment pass and its
// collision one iteration later.
enum Stage {
  STAGE_NONE = 0,  // nowhere: the collision pulls them again (cache hits)
  STAGE_REG = 1,   // registers (two planes live across the collision)
};

// Sum of v over the 64 lanes of a wave by a butterfly of lane exchanges
// (every lane ends with the same value).
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// MO: also write each node's rho and rho u (the streamed moments the step
// collides with) to mout [4][N], for the adjoint's recompute steps.
// WF: also the force of the fluid on wall wo.wall at the state the step
// collides (the traction sqrt g T^{iy} J[.][i] at the fluid layer next to the
// wall, Sec. IV.A.2, from the T the collision forms anyway): each block whose
// tile holds that layer sums its columns over its planes into
// wo.part[tile column, z chunk].  No block waits for another: block 0 of the
// next step (or k_sum_force after the last one) adds the previous step's
// partial sums, wo.prev_part[0 .. wo.prev_n), in index order into
// wo.prev_out[3]; the kernel boundary orders them.
__device__ __forceinline__ void sum_force_partials(const double* __restrict__ part, int np, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  double sp[3] = {0.0, 0.0, 0.0};
  for (int q = lane; q < np; q += 64)
#pragma unroll
    for (int a = 0; a < 3; ++a) sp[a] += part[(size_t)q * 3 + a];
#pragma unroll
  for (int a = 0; a < 3; ++a) sp[a] = wave_sum64(sp[a]);
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = sp[a];
}

// The last step's force of an lbm_step_force call: one wave.
__global__ __launch_bounds__(64) void k_sum_force(const double* __restrict__ part, int np, double* __restrict__ out) {
  sum_force_partials(part, np, out);
}

template <class T, int TX, int TY, int STAGE, bool PL, bool MO = false, bool WF = false>
__global__ __launch_bounds__(TX * TY) void k_step_fused(Grid g, int ntx, int nty, int nzc, int zc,
                                                   const T* __restrict__ pin, T* __restrict__ pout,
                                                   const T* __restrict__ hist, T* __restrict__ hout,
                                                   const T* __restrict__ geo,
                                                   const T* __restrict__ uw, int mv0, int mv1,
                                                   const T* __restrict__ up, T tau,
                                                   int* __restrict__ flag, T* __restrict__ mout, WallOut wo) {
  constexpr int HN = Tile<TX, TY>::HN, HX = Tile<TX, TY>::HX;
  // Four ring slots: the fill of plane k+1 overwrites plane k-3, whose last
  // reader (the collision of plane k-2) every thread has finished before
  // passing the barrier of the previous iteration, so one barrier per plane
  // suffices and waves of a block may drift by a plane.
  __shared__ T ring[4][4][HN];
  auto rslot = [](int k) { return (k + 4) & 3; };
  // XCD-aware tile order: hardware deals blocks round-robin over 8 XCDs;
  // each XCD takes groups of XCD_GROUP consecutive tiles (x fastest, then y,
  // then z chunk), the XCDs taking consecutive groups in turn, so a tile's
  // neighbours mostly share its L2 while all XCDs stream neighbouring memory.
  if constexpr (WF) {
    if (blockIdx.x == 0 && wo.prev_part && threadIdx.x < 64) sum_force_partials(wo.prev_part, wo.prev_n, wo.prev_out);
  }
  const int nb = ntx * nty * nzc;
  const int b = blockIdx.x;
  const int xcd = b % 8, slot = b / 8;
  const int tile = ((slot / XCD_GROUP) * 8 + xcd) * XCD_GROUP + slot % XCD_GROUP;
  if (tile >= nb) return;  // whole block exits together (no barrier skipped)
  const int tzc = tile / (ntx * nty);
  const int rem = tile % (ntx * nty);
  const int ty0 = rem / ntx, tx0 = rem % ntx;
  const int i0 = tx0 * TX, j0 = ty0 * TY;
  const int z0 = tzc * zc;
  const int z1 = min(z0 + zc, g.nz);
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = i0 + tx, jf = j0 + ty;
  const bool active = i < g.nx && jf < g.H;

  // wall force: the fluid layer next to the wall and its sign
  [[maybe_unused]] const int wrow = wo.wall == 0 ? 0 : g.H - 1;
  [[maybe_unused]] const double wsgn = wo.wall == 0 ? -1.0 : 1.0;
  [[maybe_unused]] double tw[3] = {0.0, 0.0, 0.0};

  T cur[Q], nxt[Q];
  bool own = active;  // this thread's node is collided later in the chunk
  auto to_cur = [&](auto L, T v) {
    if (own) cur[decltype(L)::value] = v;
  };
  auto to_next = [&](auto L, T v) {
    if (own) nxt[decltype(L)::value] = v;
  };
  fill_plane<T, TX, TY, PL>(ring[rslot(z0 - 1)], pin, hist, geo, uw, mv0, mv1, g, i0, j0, z0 - 1);
  if constexpr (STAGE == STAGE_NONE)
    fill_plane<T, TX, TY, PL>(ring[rslot(z0)], pin, hist, geo, uw, mv0, mv1, g, i0, j0, z0);
  else
    fill_plane_staged<T, TX, TY, PL>(ring[rslot(z0)], pin, hist, geo, uw, mv0, mv1, g, i0, j0, z0, tx, ty, to_cur);
  const T itau = T(1) / tau;
  for (int k = z0; k < z1; ++k) {
    own = active && k + 1 < z1;
    if constexpr (STAGE == STAGE_NONE)
      fill_plane<T, TX, TY, PL>(ring[rslot(k + 1)], pin, hist, geo, uw, mv0, mv1, g, i0, j0, k + 1);
    else
      fill_plane_staged<T, TX, TY, PL>(ring[rslot(k + 1)], pin, hist, geo, uw, mv0, mv1, g, i0, j0, k + 1, tx, ty, to_next);
    __syncthreads();
    if (active) {
      const NodeIdx p = node_idx<PL>(g, i, jf, k);
      const unsigned n = p.n;
      const int c0 = (ty + 1) * HX + (tx + 1);
      const T(*rc)[HN] = ring[rslot(k)];
      const T dr = rc[0][c0];
      const T j[3] = {rc[1][c0], rc[2][c0], rc[3][c0]};
      if constexpr (MO) {
        mout[n] = T(1) + dr;
#pragma unroll
        for (int a = 0; a < 3; ++a) mout[(size_t)(1 + a) * g.N + n] = j[a];
      }
      // lattice gradient from the ring
      T dj[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) dj[a][bb] = T(0);
      for_q([&](auto L) {
        constexpr int l = decltype(L)::value;
        if (l == 0) return;
        constexpr int x = cx(l), y = cy(l), z = cz(l);
        const T(*rs)[HN] = ring[rslot(k + z)];
        const int e = (ty + 1 + y) * HX + (tx + 1 + x);
        constexpr T f = T(3.0 * wgt(l));
        // across the plate: mirror ghost of the entry on this side
        bool cut = false;
        T r2 = T(0);
        const T* um = nullptr;
        if constexpr (PL && y != 0) {
          cut = (p.cut >> cut_bit(-x, -y)) & 1u;
          if (cut) {
            const int em = (ty + 1) * HX + (tx + 1 + x);
            r2 = T(2) * (T(1) + rs[0][em]);
            const int im = x ? wrapf(i + x, g.nx) : i, km = z ? wrapf(k + z, g.nz) : k;
            um = up + ((unsigned)((jf == g.pj ? g.nz : 0) + km) * g.nx + im) * 3;
          }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          T v = rs[1 + q][e];
          if constexpr (PL && y != 0)
            if (cut) v = r2 * um[q] - rs[1 + q][(ty + 1) * HX + (tx + 1 + x)];
          if (x) dj[0][q] += T(x) * f * v;
          if (y) dj[1][q] += T(y) * f * v;
          if (z) dj[2][q] += T(z) * f * v;
        }
      });
      // Streamed deviations g~_l and their second moment.
      T gv[Q];
      T sgc[6] = {0, 0, 0, 0, 0, 0};
      for_q([&](auto L) {
        constexpr int l = decltype(L)::value;
        const T v = STAGE == STAGE_NONE ? pullf<T, l, PL>(pin, g, p) : cur[l];
        gv[l] = v;
        constexpr int x = cx(l), y = cy(l), z = cz(l);
        if (x) sgc[0] += v;
        if (y) sgc[3] += v;
        if (z) sgc[5] += v;
        if (x && y) sgc[1] += T(x * y) * v;
        if (x && z) sgc[2] += T(x * z) * v;
        if (y && z) sgc[4] += T(y * z) * v;
      });
      NodeGeo<T> G;
      G.sgd = fld(geo, G_SG, g, n);
#pragma unroll
      for (int q = 0; q < 6; ++q) G.gid[q] = fldnt(geo, G_GI + q, g, n);
#pragma unroll
      for (int q = 0; q < 18; ++q) G.gam[q] = fldnt(geo, G_GAM + q, g, n);
#pragma unroll
      for (int q = 0; q < 3; ++q) G.F[q] = fldnt(geo, G_F + q, g, n);
      Coef<T> cp;
      cp.A = fld(hist, H_A, g, n);
#pragma unroll
      for (int a = 0; a < 3; ++a) cp.B[a] = fld(hist, H_B + a, g, n);
#pragma unroll
      for (int q = 0; q < 6; ++q) cp.C[q] = fldnt(hist, H_C + q, g, n);
      // J at a wall-force node, loaded with the geometry so that its latency
      // is not a round trip of its own (FP32; FP64 has no register room for
      // it there and reads J after the node's stores)
      [[maybe_unused]] double Jw[9];
      if constexpr (WF && sizeof(T) == 4) {
        if (jf == wrow)
#pragma unroll
          for (int q = 0; q < 9; ++q) Jw[q] = __builtin_nontemporal_load(wo.jac + (size_t)q * g.N + n);
      }
      const T sg = T(1) + G.sgd, isg = T(1) / sg;
      const T rho = T(1) + dr, irho = T(1) / rho;
      // equilibrium coefficients (deviation form): a0 = rho - sqrt g,
      // a1 = rho u, a2 = rho theta (g^ij - delta) + rho u u
      const T a0e = dr - G.sgd;
      T ae[6];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int bb = a; bb < 3; ++bb) ae[sym(a, bb)] = rho * T(1.0 / 3.0) * G.gid[sym(a, bb)] + j[a] * j[bb] * irho;
      // sum_l (f - feq) c c, with sum_l F_l c c = C/sqrt g and
      // sum_l feq~_l c c = (a0 delta/3 + a2)/sqrt g (D3Q19 quadrature)
      const T kneq = (T(1) - T(0.5) * itau) * sg;
      T Tm[6];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int bb = a; bb < 3; ++bb) {
          const int q = sym(a, bb);
          const T pn = sgc[q] + isg * (T(0.5) * cp.C[q] - ae[q] - (a == bb ? a0e * T(1.0 / 3.0) : T(0)));
          Tm[q] = rho * T(1.0 / 3.0) * ((a == bb ? T(1) : T(0)) + G.gid[q]) + j[a] * j[bb] * irho + kneq * pn;
        }
      // T^{iy} for the wall force, applied after this node's stores
      [[maybe_unused]] T tiy[3];
      if constexpr (WF) {
#pragma unroll
        for (int i2 = 0; i2 < 3; ++i2) tiy[i2] = Tm[sym(i2, 1)];
      }
      Coef<T> c;
      forcing_coef(G, j, Tm, dj, c);
      // f*_l - w_l = (1 - 1/tau) g~_l + (w_l/sqrt g) h_l(a_eq/tau + a_F - a_Fprev/(2 tau))
      const T hf = T(0.5) * itau;
      const T A0 = a0e * itau + c.A - hf * cp.A;
      T A1[3], A2[6];
#pragma unroll
      for (int a = 0; a < 3; ++a) A1[a] = j[a] * itau + c.B[a] - hf * cp.B[a];
#pragma unroll
      for (int q = 0; q < 6; ++q) A2[q] = ae[q] * itau + c.C[q] - hf * cp.C[q];
      {
        const T dA = T(1.0 / 3.0) * (c.A - hf * cp.A);  // b2 = C - c_s^2 A delta
        A2[0] -= dA;
        A2[3] -= dA;
        A2[5] -= dA;
      }
      const T keep = T(1) - itau;
      const T* u = uw + ((unsigned)((jf == 0 ? 0 : g.nz) + k) * g.nx + i) * 3;
      const bool mv = (jf == 0 && mv0) || (jf == g.H - 1 && mv1);
      T chk = T(0);
      for_q([&](auto L) {
        constexpr int l = decltype(L)::value;
        const T wl = T(wgt(l)) * isg;
        T v = keep * gv[l] + wl * hermite_term<T, l>(A0, A1, A2);
        constexpr int y = cy(l);
        if ((y > 0 && jf == g.H - 1) || (y < 0 && jf == 0)) {
          if (mv) {
            T cu = T(y) * u[1];
            if (cx(l)) cu += T(cx(l)) * u[0];
            if (cz(l)) cu += T(cz(l)) * u[2];
            v -= T(6) * wl * rho * cu;
          }
        }
        if constexpr (PL && y != 0) {
          // the link leaving along c_l is the one arriving along -c_l at the
          // node across: cut exactly when this node's mask has (-x, -y)
          if ((p.cut >> cut_bit(-cx(l), -y)) & 1u) {
            const T* upn = up + ((unsigned)((jf == g.pj ? g.nz : 0) + k) * g.nx + i) * 3;
            T cu = T(y) * upn[1];
            if (cx(l)) cu += T(cx(l)) * upn[0];
            if (cz(l)) cu += T(cz(l)) * upn[2];
            v -= T(6) * wl * rho * cu;
          }
        }
        chk += v;
        stw(pout + (size_t)l * g.N, n, v);
      });
      stw(hout + (size_t)H_A * g.N, n, c.A);
#pragma unroll
      for (int a = 0; a < 3; ++a) stw(hout + (size_t)(H_B + a) * g.N, n, c.B[a]);
#pragma unroll
      for (int q = 0; q < 6; ++q) stw(hout + (size_t)(H_C + q) * g.N, n, c.C[q]);
      const T uu = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
      if (!(rho > T(0)) || !(uu < T(0.1) * rho * rho) || !isfinite(chk)) atomicOr(flag, 1);
      if constexpr (WF) {
        if (jf == wrow) {
          const double sgw = 1.0 + (double)G.sgd;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            double sa = 0.0;
#pragma unroll
            for (int i2 = 0; i2 < 3; ++i2) {
              double ja;
              if constexpr (sizeof(T) == 4)
                ja = Jw[a * 3 + i2];
              else
                ja = wo.jac[(size_t)(a * 3 + i2) * g.N + n];
              sa += (double)tiy[i2] * ja;
            }
            tw[a] += wsgn * sgw * sa;
          }
        }
      }
    }
    if constexpr (STAGE == STAGE_REG)
      if (own)
        for_q([&](auto L) {
          constexpr int l = decltype(L)::value;
          cur[l] = nxt[l];
        });
  }
  if constexpr (WF) {
    if (ty0 != wrow / TY) return;  // uniform per block: the tile holds no wall column
    __shared__ double red[TX * TY / 64][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) tw[a] = wave_sum64(tw[a]);
    if (lane == 0)
#pragma unroll
      for (int a = 0; a < 3; ++a) red[wave][a] = tw[a];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double sa = red[0][a];
#pragma unroll
        for (int w = 1; w < TX * TY / 64; ++w) sa += red[w][a];
        wo.part[(size_t)(tzc * ntx + tx0) * 3 + a] = sa;
      }
  }
}

}  // namespace

// Register staging for FP32 only: FP64 has no register room for a second
// plane of pulled populations.
template <class T> constexpr int reg_stage() { return sizeof(T) == 4 ? STAGE_REG : STAGE_NONE; }

// Planes per block when the caller leaves it open.  Blocks run in rounds of
// `slots` (resident blocks on the whole device); a chunk of zc planes costs
// about zc + 1 plane-times (its two halo planes get moments only).  Take the
// zc with the least rounds * (zc + 1); ties go to the smaller zc.  Chunks are
// capped at zc_max<T>() planes: longer ones spread each block's 86 streams
// over more of every array at once, which costs more than the model's saved
// halo planes (512x256x256 FP32: 256 planes 2.88 ms per step, 32 planes 2.59,
// 16 planes 2.57; 256x128x128 FP32: 32 planes 0.298 ms, 16 planes 0.295).  In
// FP64 32 planes stay (256x128x128: 0.599 ms against 0.610 with 16).
template <class T> constexpr int zc_max() { return sizeof(T) == 4 ? 16 : 32; }
inline int choose_zc(long long tiles, int nz, long long slots, int zc_cap) {
  const int top = nz < zc_cap ? nz : zc_cap;
  int best = top;
  long long best_cost = -1;
  for (int zc = 1; zc <= top; ++zc) {
    const long long nb = tiles * ((nz + zc - 1) / zc);
    const long long cost = ((nb + slots - 1) / slots) * (zc + 1);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zc;
    }
  }
  return best;
}

// Planes per block for kernel k_step_fused<T, TX, TY, ST, PL>: zc if
// positive, else the choice above for this device.
template <class T, int TX, int TY, int ST, bool PL, bool MO = false, bool WF = false>
hipError_t fused_chunk(Fields& F, int zc, int* out) {
  const Grid g = F.g;
  if (zc <= 0) {
    const int key = ((((int)sizeof(T) * 1000 + TX) * 100 + TY * 10 + ST) * 8) + (PL ? 1 : 0) + (MO ? 2 : 0) + (WF ? 4 : 0);
    int hit = -1;
    for (int q = 0; q < 4; ++q)
      if (F.slots_key[q] == key) hit = q;
    if (hit < 0) {
      int dev = 0, cus = 0, per_cu = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_fused<T, TX, TY, ST, PL, MO, WF>,
                                                         Tile<TX, TY>::NT, 0);
      if (e != hipSuccess) return e;
      hit = 0;
      while (hit < 3 && F.slots_key[hit] >= 0) ++hit;  // a free entry, else the last
      F.slots[hit] = (long long)cus * (per_cu > 0 ? per_cu : 1);
      F.slots_key[hit] = key;
    }
    const long long tiles = (long long)((g.nx + TX - 1) / TX) * ((g.H + TY - 1) / TY);
    zc = choose_zc(tiles, g.nz, F.slots[hit], zc_max<T>());
  }
  *out = zc < g.nz ? zc : g.nz;
  return hipSuccess;
}

template <class T, int TX, int TY, int ST, bool PL, bool MO = false, bool WF = false>
hipError_t fused_launch(Fields& F, hipStream_t s, T tau, int zc, T* mout = nullptr, WallOut wo = WallOut{}) {
  const Grid g = F.g;
  const hipError_t e = fused_chunk<T, TX, TY, ST, PL, MO, WF>(F, zc, &zc);
  if (e != hipSuccess) return e;
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.H + TY - 1) / TY;
  const int nzc = (g.nz + zc - 1) / zc;
  const long long sweep = 8LL * XCD_GROUP;
  const unsigned nblk = (unsigned)(((long long)ntx * nty * nzc + sweep - 1) / sweep * sweep);
  hipLaunchKernelGGL((k_step_fused<T, TX, TY, ST, PL, MO, WF>), dim3(nblk), dim3(Tile<TX, TY>::NT), 0, s, g, ntx,
                     nty, nzc, zc, (const T*)F.pop[F.cur], (T*)F.pop[F.cur ^ 1], (const T*)F.hist[F.cur],
                     (T*)F.hist[F.cur ^ 1], (const T*)F.geo, (const T*)F.uw, F.moving[0], F.moving[1],
                     (const T*)F.up, tau, F.flag, mout, wo);
  F.cur ^= 1;
  return hipGetLastError();
}

template <class T, int TX, int TY, bool PL = false> hipError_t launch_fused_tile(Fields& F, hipStream_t s, T tau, int zc) {
  if (F.stage == STAGE_REG) return fused_launch<T, TX, TY, reg_stage<T>(), PL>(F, s, tau, zc);
  return fused_launch<T, TX, TY, STAGE_NONE, PL>(F, s, tau, zc);
}

template <class T, int TX, int TY, bool PL = false> hipError_t chunk_tile(Fields& F, int* zc) {
  if (F.stage == STAGE_REG) return fused_chunk<T, TX, TY, reg_stage<T>(), PL>(F, F.zc, zc);
  return fused_chunk<T, TX, TY, STAGE_NONE, PL>(F, F.zc, zc);
}

// The fused step runs on 64x4 tiles (x by y nodes per block); a grid with an
// interior plate runs the plate-aware instantiation.
template <class T> hipError_t launch_step_fused(Fields& F, hipStream_t s, T tau, int zc) {
  if (F.g.pj) return launch_fused_tile<T, 64, 4, true>(F, s, tau, zc);
  return launch_fused_tile<T, 64, 4>(F, s, tau, zc);
}

// The fused step on 64x4 tiles without register staging that also writes
// rho and rho u of the state it steps from to mout [4][N] (rho in full, not
// as a deviation): the adjoint's recompute steps keep them for the reverse
// sweep.  Grids with a plate or open ends are not served (hipErrorNotSupported).
template <class T> hipError_t launch_step_fused_moments(Fields& F, hipStream_t s, T tau, T* mout) {
  if (F.g.pj || F.g.open || !mout) return hipErrorNotSupported;
  return fused_launch<T, 64, 4, STAGE_NONE, false, true>(F, s, tau, F.zc, mout);
}

// n fused steps, each also giving the force on a wall of the state it steps
// from (stress method) into out[3 t]: grids without a plate or open ends, with
// the fused step selected (hipErrorNotSupported otherwise, before any launch;
// the caller then takes lbm_wall_force and a plain step).  Step t writes its
// partial sums into one half of F.fpart, step t+1 (or k_sum_force after the
// last step) adds them up.
template <class T> hipError_t launch_steps_fused_force(Fields& F, hipStream_t s, T tau, int wall, int n, double* out) {
  if (F.g.pj || F.g.open || !step_is_fused(F) || !out) return hipErrorNotSupported;
  if (n <= 0) return hipSuccess;
  constexpr int ST = reg_stage<T>();
  const bool staged = F.stage == STAGE_REG;
  int zc = 0;
  hipError_t e = staged ? fused_chunk<T, 64, 4, ST, false, false, true>(F, F.zc, &zc)
                        : fused_chunk<T, 64, 4, STAGE_NONE, false, false, true>(F, F.zc, &zc);
  if (e != hipSuccess) return e;
  const int np = ((F.g.nx + 63) / 64) * ((F.g.nz + zc - 1) / zc);  // blocks holding the wall layer
  const size_t half = 3 * (size_t)((F.g.nx + 63) / 64) * F.g.nz;
  for (int t = 0; t < n; ++t) {
    WallOut wo{wall, F.jac, F.fpart + half * (t & 1), nullptr, np, nullptr};
    if (t > 0) {
      wo.prev_part = F.fpart + half * ((t - 1) & 1);
      wo.prev_out = out + 3 * (size_t)(t - 1);
    }
    e = staged ? fused_launch<T, 64, 4, ST, false, false, true>(F, s, tau, F.zc, nullptr, wo)
               : fused_launch<T, 64, 4, STAGE_NONE, false, false, true>(F, s, tau, F.zc, nullptr, wo);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sum_force, dim3(1), dim3(64), 0, s, (const double*)(F.fpart + half * ((n - 1) & 1)), np,
                     out + 3 * (size_t)(n - 1));
  return hipGetLastError();
}

template <class T> hipError_t fused_step_chunk(Fields& F, int* zc) {
  if (F.g.pj) return chunk_tile<T, 64, 4, true>(F, zc);
  return chunk_tile<T, 64, 4>(F, zc);
}

template hipError_t fused_step_chunk<double>(Fields&, int*);
template hipError_t fused_step_chunk<float>(Fields&, int*);
template hipError_t launch_step_fused<double>(Fields&, hipStream_t, double, int);
template hipError_t launch_steps_fused_force<double>(Fields&, hipStream_t, double, int, int, double*);
template hipError_t launch_steps_fused_force<float>(Fields&, hipStream_t, float, int, int, double*);
template hipError_t launch_step_fused<float>(Fields&, hipStream_t, float, int);
template hipError_t launch_step_fused_moments<double>(Fields&, hipStream_t, double, double*);

}  // namespace lbm
