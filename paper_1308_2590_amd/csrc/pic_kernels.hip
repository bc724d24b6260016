// HIP kernels (gfx950) of the implicit 2D3V PIC particle stage.
//
// Field solve (FP64, one thread per node / cell):
//   k_solve_e   Eq. (4) per node: E_new = (I + S)^{-1}[(I - S)E + dt(curl H - dj)] with curl H
//               from the 2x2 neighbouring cells (Sec. 3.3 Step 5); on an absorbing x axis the
//               thread of the inner node next to a boundary node also applies the first-order
//               Mur condition to E - E_inc there (Steps 3, 4, 6); writes E-bar.  Moments are
//               read, then cleared for the next deposit, only in tiles the deposit reached.
//   k_update_h  Eq. (5) at cell centres with curl E from the 4 corner nodes (Steps 8-9), and
//               clears the deposit flags of the tiles.
// Particles (one block per tile of cells, one wavefront per row of the tile):
//   k_particles gather E-bar (bilinear from the 4 corner nodes) and B (the particle's cell),
//               implicit push (Eq. (2a) solved for the time-centred momentum), position
//               advance, move code, then deposit of S-hat, delta-j and density (Step 1,
//               Eq. (3)) at the new position into LDS accumulators covering the tile plus a
//               halo, folded once per tile into the FP64 moment planes with global atomics.
//               It also counts the particles leaving each cell per move code and arriving in
//               each cell.  Instantiated for FP64 and for the mixed form (FP32 particles).
// Sort (stable by cell, removed particles dropped):
//   k_scan_counts / k_scan_apply  exclusive scan of the arrival counts -> next cell start
//               offsets (per block, then the block totals added), the tiles holding particles
//               in the next order as flags and, from one extra block, as an ordered list;
//   k_tile_flags / k_tile_compact  the same flags and list from cell starts (after loads);
//   kb_scan1 / kb_scan2  the same two passes for every run of a batch;
//   k_rank      stable destination of every particle: cell start + particles arriving from
//               source cells with a smaller key + rank within (source cell, move code),
//               written as the next cycle's slot -> location permutation.
// Positions never move more than one cell per cycle because dt <= min(dx, dz) and |v| < c,
// which is what keeps the sort a 3x3 neighbourhood redistribution.
//
// The file is compiled with -ffp-contract=off: fused multiply-adds appear only where written.
// The FP64 mover evaluates the same expressions as a plain implementation of the method up to
// rounding (vector form of the response, Newton-refined reciprocals), so FP64 results agree
// with the oracle to about 1e-15 relative per cycle.

#include <algorithm>
#include <type_traits>

#include "pic_internal.h"

namespace pic {
namespace {

constexpr uint32_t kFlagOrder = PIC_FLAG_ORDER;
constexpr uint32_t kFlagNonFinite = PIC_FLAG_NONFINITE;
constexpr uint32_t kFlagJump = PIC_FLAG_JUMP;
constexpr uint32_t kFlagSlot = PIC_FLAG_SLOT;

__device__ __forceinline__ int wrap1(int i, int n) {
  if (i < 0) return i + n;
  if (i >= n) return i - n;
  return i;
}

__device__ __forceinline__ int wrap_any(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Wrap onto [0, n): one conditional add or subtract when i is known to lie in [-n, 2n) (near:
// a tile and its ring fit in the grid), the general remainder otherwise (grids smaller than a
// tile).  near is the same for the whole block.
__device__ __forceinline__ int wrap_t(int i, int n, bool near) {
  return near ? wrap1(i, n) : wrap_any(i, n);
}

// Quotient e / d of non-negative integers (e < 2^22, 0 < d < 2^12) from one multiply:
// (e + 1/2) / d lies at least 1 / (2 d) away from every integer, and the float product is
// within a relative 2^-23 of it, i.e. within (e + 1/2) / d 2^-23 < 1 / (2 d) absolutely, so
// truncating it gives the exact quotient.  Grid coordinates (below 2^22 by the grid's limits)
// and tile-local indices both qualify.
struct SmallDiv {
  float r;
  __device__ __forceinline__ explicit SmallDiv(int d) : r(1.0f / (float)d) {}
  __device__ __forceinline__ int q(int e) const { return (int)(((float)e + 0.5f) * r); }
};

// The tile handled by this block, taken from the ordered list of tiles that hold particles:
// blocks are dealt round-robin to the 8 XCDs, so each XCD gets a contiguous band of the list
// (neighbouring tiles share halo nodes and field cache lines).  Surplus blocks return.
__device__ __forceinline__ int block_tile(const TileArgs &t, const int32_t *list) {
  const int count = list[t.ntiles];
  const int per = (count + 7) >> 3;
  const int b = blockIdx.x;
  if ((b >> 3) >= per) return -1;
  const int idx = (b & 7) * per + (b >> 3);
  return idx < count ? list[idx] : -1;
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }

// Reciprocal and reciprocal square root.  FP64: the hardware estimate refined by two
// Newton-Raphson steps (each squares the relative error), which leaves an error of about one
// unit in the last place.  FP32: the hardware results, accurate to about one unit in the last
// place, are used as they are.  Arguments here are >= 1, far from denormals and overflow.
__device__ __forceinline__ double rcpT(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float rcpT(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsqT(double x) {
  // y' = y + (y / 2)(1 - x y^2)
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}
__device__ __forceinline__ float rsqT(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float floorT(float a) { return floorf(a); }  // the mixed carry (FP64 uses floor)

// ------------------------------------------------------------------------------------------
// Field solve
// ------------------------------------------------------------------------------------------

__device__ double incident_ey(const LaserArgs &L, double t, double x, double z) {
  if (L.a0 == 0.0) return 0.0;
  double tau = t - x;
  double st = (tau - L.t_center) / L.fwhm_t;
  double sz = (z - L.z_center) / L.sigma_z;
  return L.a0 * sin(L.omega * tau) * exp(-0.5 * sz * sz) * exp(-2.0 * 0.6931471805599453 * st * st);
}

// Whether the moment planes of node n can hold a deposit: the flag of its run of kFlagNodes
// nodes.  Elsewhere the planes are zero.
__device__ __forceinline__ bool node_deposited(const FieldArgs &a, int64_t n) {
  return !a.mflag || a.mflag[n / kFlagNodes] != 0;
}

// Zero every moment plane of node n once its values have been read, so the next deposit
// starts from zero.  Each node is read and cleared by one thread.
__device__ __forceinline__ void clear_node_moments(const FieldArgs &a, int64_t n) {
  for (int p = 0; p < a.g.n_planes; ++p) a.M[p * a.g.nnodes + n] = 0.0;
}

// Inputs of Eq. (4) at the node (i, k), i an interior column: curl H from the 2x2 cells
// around the node, E^n, and S-hat and delta-j where a deposit can have reached the node (zero
// elsewhere).  Loads only: a thread gathers the inputs of all its nodes before its first
// store (the compiler cannot tell the planes apart, so a load after a store waits for it).
struct NodeIn {
  double curl[3], e[3], S[9], J[3];
  int64_t n;
  bool dep;
};

__device__ __forceinline__ void node_load(const FieldArgs &a, int i, int k, NodeIn &in) {
  const GridArgs &g = a.g;
  const int nx = g.nx, nz = g.nz;
  const int64_t nn = g.nnodes, nc = g.ncells;
  int iR = wrap1(i, nx), iL = wrap1(i - 1, nx);
  int kU = wrap1(k, nz), kD = wrap1(k - 1, nz);
  int64_t cUR = (int64_t)kU * nx + iR, cUL = (int64_t)kU * nx + iL;
  int64_t cDR = (int64_t)kD * nx + iR, cDL = (int64_t)kD * nx + iL;
  const double *Hx = a.H, *Hy = a.H + nc, *Hz = a.H + 2 * nc;
  double dHx_dz = ((Hx[cUR] + Hx[cUL]) - (Hx[cDR] + Hx[cDL])) * a.r2dz;
  double dHy_dz = ((Hy[cUR] + Hy[cUL]) - (Hy[cDR] + Hy[cDL])) * a.r2dz;
  double dHy_dx = ((Hy[cUR] + Hy[cDR]) - (Hy[cUL] + Hy[cDL])) * a.r2dx;
  double dHz_dx = ((Hz[cUR] + Hz[cDR]) - (Hz[cUL] + Hz[cDL])) * a.r2dx;
  in.curl[0] = -dHy_dz;
  in.curl[1] = dHx_dz - dHz_dx;
  in.curl[2] = dHy_dx;
  const int64_t n = (int64_t)k * g.nxn + i;
  in.n = n;
#pragma unroll
  for (int r = 0; r < 3; ++r) in.e[r] = a.E[r * nn + n];
  in.dep = node_deposited(a, n);
  if (in.dep) {
#pragma unroll
    for (int r = 0; r < 9; ++r) in.S[r] = a.M[r * nn + n];
#pragma unroll
    for (int r = 0; r < 3; ++r) in.J[r] = a.M[(9 + r) * nn + n];
  } else {
#pragma unroll
    for (int r = 0; r < 9; ++r) in.S[r] = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) in.J[r] = 0.0;
  }
}

// Eq. (4): E^{n+1} = (I + S)^{-1} [(I - S) E^n + dt (curl H - delta-j)].
__device__ __forceinline__ void node_solve(const FieldArgs &a, const NodeIn &in, double out[3]) {
  const double dt = a.g.dt;
  const double *S = in.S, *e = in.e;
  double rhs[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double se = S[3 * r] * e[0] + S[3 * r + 1] * e[1] + S[3 * r + 2] * e[2];
    rhs[r] = (e[r] - se) + dt * (in.curl[r] - in.J[r]);
  }
  double A[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) A[r] = S[r] + ((r % 4 == 0) ? 1.0 : 0.0);
  // Cramer's rule; I + S has a positive-definite symmetric part, so det > 0.
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  double c10 = A[2] * A[7] - A[1] * A[8];
  double c11 = A[0] * A[8] - A[2] * A[6];
  double c12 = A[1] * A[6] - A[0] * A[7];
  double c20 = A[1] * A[5] - A[2] * A[4];
  double c21 = A[2] * A[3] - A[0] * A[5];
  double c22 = A[0] * A[4] - A[1] * A[3];
  const double rdet = 1.0 / det;
  out[0] = (c00 * rhs[0] + c10 * rhs[1] + c20 * rhs[2]) * rdet;
  out[1] = (c01 * rhs[0] + c11 * rhs[1] + c21 * rhs[2]) * rdet;
  out[2] = (c02 * rhs[0] + c12 * rhs[1] + c22 * rhs[2]) * rdet;
}

// E^{n+1} of node n.  (The particle kernel forms E-bar = (E^n + E^{n+1}) / 2 where it reads
// the fields.)
__device__ __forceinline__ void write_e(const FieldArgs &a, int64_t n, const double en[3]) {
  const int64_t nn = a.g.nnodes;
#pragma unroll
  for (int r = 0; r < 3; ++r) a.E_new[r * nn + n] = en[r];
}

// Mur boundary (Step 3) at the column i = 0 or i = nx of an absorbing axis, from E^n (eo_in)
// and the new E (ein) of the inner column next to it; the x = 0 column takes the source of
// Step 4 on E_y.
__device__ void mur_node(const FieldArgs &a, double tE, int i, int k, const double eo_in[3],
                         const double ein[3]) {
  const GridArgs &g = a.g;
  const int64_t nn = g.nnodes;
  const double kappa = (g.dt - g.dx) / (g.dt + g.dx);
  const double t0 = tE, t1 = tE + g.dt;
  const double z = (double)k * g.dz;
  const int64_t nb = (int64_t)k * g.nxn + i;
  double en[3], eo[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) eo[r] = a.E[r * nn + nb];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double Eo_b = eo[r], Eo_in = eo_in[r];
    if (i == 0) {
      double i10 = 0.0, i01 = 0.0, i11 = 0.0, i00 = 0.0;
      if (r == 1) {
        i10 = incident_ey(a.laser, t1, 0.0, z);
        i01 = incident_ey(a.laser, t0, g.dx, z);
        i11 = incident_ey(a.laser, t1, g.dx, z);
        i00 = incident_ey(a.laser, t0, 0.0, z);
      }
      en[r] = i10 + (Eo_in - i01) + kappa * ((ein[r] - i11) - (Eo_b - i00));
    } else {
      en[r] = Eo_in + kappa * (ein[r] - Eo_b);
    }
  }
  write_e(a, nb, en);
  // the boundary node takes deposits too; its planes are not used by the solve
  if (node_deposited(a, nb)) clear_node_moments(a, nb);
}

// Nodes n0, n0 + stride, ... of the E solve (kSolveNodes per thread, their inputs loaded
// together).  On an absorbing axis the thread of the inner column next to a boundary column
// also writes that column, so every node's moments are read and cleared by a single thread (an
// absorbing axis has nx >= 2).

__device__ __forceinline__ void solve_e_body(const FieldArgs &a, double tE, int64_t n0,
                                             int64_t stride) {
  const GridArgs &g = a.g;
  const bool absorbing = g.bc_x == PIC_BC_ABSORBING;
  NodeIn in[kSolveNodes];
  bool live[kSolveNodes];
  int ii[kSolveNodes], kk[kSolveNodes];
#pragma unroll
  for (int q = 0; q < kSolveNodes; ++q) {
    const int64_t n = n0 + q * stride;
    const int k = (int)(n / g.nxn), i = (int)(n - (int64_t)k * g.nxn);
    ii[q] = i;
    kk[q] = k;
    live[q] = n < g.nnodes && !(absorbing && (i == 0 || i == g.nx));
    if (live[q]) node_load(a, i, k, in[q]);
  }
  double en[kSolveNodes][3];
#pragma unroll
  for (int q = 0; q < kSolveNodes; ++q)
    if (live[q]) node_solve(a, in[q], en[q]);
#pragma unroll
  for (int q = 0; q < kSolveNodes; ++q) {
    if (!live[q]) continue;
    if (in[q].dep) clear_node_moments(a, in[q].n);
    write_e(a, in[q].n, en[q]);
    if (absorbing) {
      if (ii[q] == 1) mur_node(a, tE, 0, kk[q], in[q].e, en[q]);
      if (ii[q] == g.nx - 1) mur_node(a, tE, g.nx, kk[q], in[q].e, en[q]);
    }
  }
}

// Block b of a grid of 8 * per blocks runs on XCD b % 8 (round-robin dispatch); give the
// blocks of one XCD a contiguous band of the grid, so the neighbouring rows a stencil reads
// are mostly in the same L2.  Returns -1 for the padding blocks.
__device__ __forceinline__ int64_t xcd_band_block(int64_t nblocks) {
  const int64_t per = (nblocks + 7) >> 3;
  const int64_t b = blockIdx.x;
  const int64_t idx = (b & 7) * per + (b >> 3);
  return idx < nblocks ? idx : -1;
}

__global__ __launch_bounds__(kBlock) void k_solve_e(const FieldArgs a, int64_t nblocks) {
  const int64_t blk = xcd_band_block(nblocks);
  if (blk < 0) return;
  solve_e_body(a, a.t, blk * (kSolveNodes * kBlock) + threadIdx.x, kBlock);
}

// Cells c0, c0 + stride, ... of the H update (kHCells per thread, all loads before the
// stores).
__device__ __forceinline__ void update_h_body(const FieldArgs &a, int64_t c0, int64_t stride) {
  const GridArgs &g = a.g;
  const int nx = g.nx, nz = g.nz, nxn = g.nxn;
  const int64_t nn = g.nnodes, nc = g.ncells;
  const double *Ex = a.E_new, *Ey = a.E_new + nn, *Ez = a.E_new + 2 * nn;
  double hn[kHCells][3];
  bool live[kHCells];
#pragma unroll
  for (int q = 0; q < kHCells; ++q) {
    const int64_t c = c0 + q * stride;
    live[q] = c < nc;
    if (!live[q]) continue;
    int k = (int)(c / nx), i = (int)(c - (int64_t)k * nx);
    int i1 = (g.bc_x == PIC_BC_PERIODIC) ? wrap1(i + 1, nx) : i + 1;
    int k1 = wrap1(k + 1, nz);
    int64_t na = (int64_t)k * nxn + i, nb = (int64_t)k * nxn + i1;
    int64_t ncn = (int64_t)k1 * nxn + i, nd = (int64_t)k1 * nxn + i1;
    double dEx_dz = ((Ex[ncn] + Ex[nd]) - (Ex[na] + Ex[nb])) * a.r2dz;
    double dEy_dz = ((Ey[ncn] + Ey[nd]) - (Ey[na] + Ey[nb])) * a.r2dz;
    double dEy_dx = ((Ey[nb] + Ey[nd]) - (Ey[na] + Ey[ncn])) * a.r2dx;
    double dEz_dx = ((Ez[nb] + Ez[nd]) - (Ez[na] + Ez[ncn])) * a.r2dx;
    hn[q][0] = a.H[c] - g.dt * (-dEy_dz);
    hn[q][1] = a.H[nc + c] - g.dt * (dEx_dz - dEz_dx);
    hn[q][2] = a.H[2 * nc + c] - g.dt * dEy_dx;
  }
#pragma unroll
  for (int q = 0; q < kHCells; ++q) {
    if (!live[q]) continue;
    const int64_t c = c0 + q * stride;
    a.H_new[c] = hn[q][0];
    a.H_new[nc + c] = hn[q][1];
    a.H_new[2 * nc + c] = hn[q][2];
    // The E solve has read the deposit flags: clear them for the next deposit (there are
    // fewer flags than cells: nodes <= 2 cells).
    if (a.mflag && c < (nn + kFlagNodes - 1) / kFlagNodes) a.mflag[c] = 0;
    // the next order's tile flags, set again by the sort's scan (batched cycle; there are no
    // more tiles than cells)
    if (a.tact_next && c < (int64_t)a.ntiles_next) a.tact_next[c] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_update_h(const FieldArgs a, int64_t nblocks) {
  const int64_t blk = xcd_band_block(nblocks);
  if (blk < 0) return;
  update_h_body(a, blk * (kHCells * kBlock) + threadIdx.x, kBlock);
}

// ------------------------------------------------------------------------------------------
// Particles
// ------------------------------------------------------------------------------------------

// The value of the lane below (lane 0 gets its own): a DPP wave shift by one lane, which
// stays in the VALU instead of the LDS crossbar.
__device__ __forceinline__ int lane_before(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}

// The value of the lane above (lane 63 gets its own), by DPP wave shifts of 32-bit halves.
__device__ __forceinline__ int lane_after(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ float lane_after(float v) {
  return __int_as_float(lane_after(__float_as_int(v)));
}
__device__ __forceinline__ double lane_after(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_after((int)(b & 0xffffffffll)), hi = lane_after((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Stores of the particle kernel as raw buffer stores: a lane without a value passes an offset
// past the buffer's range, which the hardware drops, so the store needs no branch.  Every array
// gets the same range, 2^31 bytes (a species holds fewer than 2^28 particles).
constexpr int kStoreDrop = (int)0xFFFFFF00u;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t store_rsrc(void *p) {
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)0x80000000u, 0x00020000);
}
__device__ __forceinline__ void store_or_drop(double *p, int i, bool on, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), store_rsrc(p), on ? i * 8 : kStoreDrop, 0, 0);
}
__device__ __forceinline__ void store_or_drop(uint32_t *p, int i, bool on, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, store_rsrc(p), on ? i * 4 : kStoreDrop, 0, 0);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Compact moments of one particle in the field B of its cell.  With s = beta / gamma and
// b = s B, R = (I + s [B]x + s^2 B B^T) / (1 + s^2 B.B), so
//   S-hat = a0 I + a1 [B]x + a2 B B^T,  a0 = w q^2 dt^2 / (4 m gamma (1 + s^2 B.B)),
//   a1 = a0 s, a2 = a1 s,
//   delta-j = (w q / gamma) R u = (w q / (gamma (1 + s^2 B.B))) (u + s u x B + s^2 (B.u) B).
// Particles sharing a cell share B, so their S-hat deposits add up through three scalars.
template <typename T>
struct Compact {
  T a0, a1, a2, j0, j1, j2;
};

// Species constants in the arithmetic type of the kernel.
template <typename T>
struct SpConst {
  T beta, cS, kJ, w;
};

template <typename T>
__device__ __forceinline__ Compact<T> compact_moments(const SpConst<T> &k, T ginv, T u0, T u1,
                                                      T u2, T B0, T B1, T B2) {
  const T s = k.beta * ginv;
  const T BB = fmaT(B2, B2, fmaT(B1, B1, B0 * B0));
  const T inv = rcpT(fmaT(s * s, BB, T(1)));
  Compact<T> m;
  m.a0 = k.cS * ginv * inv;
  m.a1 = m.a0 * s;
  m.a2 = m.a1 * s;
  const T kk = k.kJ * ginv * inv;
  const T bu = fmaT(B2, u2, fmaT(B1, u1, B0 * u0));
  const T s2bu = s * s * bu;
  m.j0 = kk * fmaT(s2bu, B0, fmaT(s, fmaT(u1, B2, -(u2 * B1)), u0));
  m.j1 = kk * fmaT(s2bu, B1, fmaT(s, fmaT(u2, B0, -(u0 * B2)), u1));
  m.j2 = kk * fmaT(s2bu, B2, fmaT(s, fmaT(u0, B1, -(u1 * B0)), u2));
  return m;
}

// The compact moments of unit density scaled to a particle's density w.
template <typename T>
__device__ __forceinline__ void scale_compact(Compact<T> &m, T w) {
  m.a0 *= w;
  m.a1 *= w;
  m.a2 *= w;
  m.j0 *= w;
  m.j1 *= w;
  m.j2 *= w;
}

// Add one corner's share of compact moments (one particle's, weighted, or a lane's sum):
// delta-j and the density to the node planes at node o, and the three S-hat scalars to the
// planes of that corner of cell rc.  S-hat is expanded with each cell's B only when the tile is
// folded, so a flush does no arithmetic.  The LDS accumulators are FP64 in both precisions
// (FP32 LDS atomic adds are far slower than FP64 ones on gfx950).
struct AccLds {
  double *node;  // [3 + species][plane]: delta-j x, y, z, then one density plane per species
  double *cell;  // [3 scalars][4 corners][npl]: S-hat scalars a0, a1, a2 per cell corner
  int plane, npl, LW, NW;
};

template <typename T>
__device__ __forceinline__ void corner_add(const AccLds &A, int o, int rc, int corner, T A0, T A1,
                                           T A2, T J0, T J1, T J2, T D, int dplane) {
  atomicAdd(&A.node[0 * A.plane + o], (double)J0);
  atomicAdd(&A.node[1 * A.plane + o], (double)J1);
  atomicAdd(&A.node[2 * A.plane + o], (double)J2);
  atomicAdd(&A.node[dplane * A.plane + o], (double)D);
  atomicAdd(&A.cell[(0 * 4 + corner) * A.npl + rc], (double)A0);
  atomicAdd(&A.cell[(1 * 4 + corner) * A.npl + rc], (double)A1);
  atomicAdd(&A.cell[(2 * 4 + corner) * A.npl + rc], (double)A2);
}

// Per-lane running sum of the compact moments of consecutive particles that stay in one
// cell, per corner (order (i,k), (i+1,k), (i,k+1), (i+1,k+1)).
template <typename T>
struct CellAcc {
  T A0[4], A1[4], A2[4], J0[4], J1[4], J2[4], D[4];
  int cell;  // tile-local column of the cell being accumulated, -1 when empty

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int c = 0; c < 4; ++c) A0[c] = A1[c] = A2[c] = J0[c] = J1[c] = J2[c] = D[c] = T(0);
  }
  __device__ __forceinline__ void add(T fx, T fz, const Compact<T> &m, T w) {
    const T one = T(1);
    const T W[4] = {(one - fx) * (one - fz), fx * (one - fz), (one - fx) * fz, fx * fz};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      A0[c] = fmaT(W[c], m.a0, A0[c]);
      A1[c] = fmaT(W[c], m.a1, A1[c]);
      A2[c] = fmaT(W[c], m.a2, A2[c]);
      J0[c] = fmaT(W[c], m.j0, J0[c]);
      J1[c] = fmaT(W[c], m.j1, J1[c]);
      J2[c] = fmaT(W[c], m.j2, J2[c]);
      D[c] = fmaT(W[c], w, D[c]);
    }
  }
  // The accumulated cell is (cell, lz - 1) of the tile: ring cell (cell + 1, lz), whose
  // lower-left node is (cell + 1, lz) locally (the layout with the ring).
  __device__ __forceinline__ void flush(const AccLds &acc, int lz, int dplane) {
    const int b = lz * acc.LW + cell + 1, rc = lz * acc.NW + cell + 1;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      corner_add(acc, b + (c & 1) + (c >> 1) * acc.LW, rc, c, A0[c], A1[c], A2[c], J0[c], J1[c],
                 J2[c], D[c], dplane);
  }
  // End of a row: every lane flushes at once, and the lanes whose runs end in one cell are
  // neighbours.  Their sums are first added up across lanes (a segmented reduction with
  // shuffles towards the first lane of each cell), so that one lane per cell issues the LDS
  // atomics; same-address atomics from many lanes of one instruction are serialised.  All 64
  // lanes must be active.
  __device__ __forceinline__ void flush_row_end(const AccLds &acc, int lz, int dplane, int lane) {
    const int prev = lane_before(cell);
    const bool head = lane == 0 || prev != cell;
    const uint64_t heads = __ballot(head);
    const uint64_t above = heads & ~((2ull << lane) - 1ull);
    const int seg_end = above ? __ffsll((unsigned long long)above) - 1 : 64;
    {
      // first step (neighbour one lane up) by DPP; the wider steps go through the LDS crossbar
      const bool take = lane + 1 < seg_end;
      if (!__any(take)) {
        if (head && cell >= 0) flush(acc, lz, dplane);
        return;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T v;
        v = lane_after(A0[c]); A0[c] += take ? v : T(0);
        v = lane_after(A1[c]); A1[c] += take ? v : T(0);
        v = lane_after(A2[c]); A2[c] += take ? v : T(0);
        v = lane_after(J0[c]); J0[c] += take ? v : T(0);
        v = lane_after(J1[c]); J1[c] += take ? v : T(0);
        v = lane_after(J2[c]); J2[c] += take ? v : T(0);
        v = lane_after(D[c]); D[c] += take ? v : T(0);
      }
    }
    for (int d = 2; d < 64; d <<= 1) {
      const bool take = lane + d < seg_end;
      if (!__any(take)) break;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T v;
        v = __shfl_down(A0[c], d); A0[c] += take ? v : T(0);
        v = __shfl_down(A1[c], d); A1[c] += take ? v : T(0);
        v = __shfl_down(A2[c], d); A2[c] += take ? v : T(0);
        v = __shfl_down(J0[c], d); J0[c] += take ? v : T(0);
        v = __shfl_down(J1[c], d); J1[c] += take ? v : T(0);
        v = __shfl_down(J2[c], d); J2[c] += take ? v : T(0);
        v = __shfl_down(D[c], d); D[c] += take ? v : T(0);
      }
    }
    if (head && cell >= 0) flush(acc, lz, dplane);
  }
};

// Particles that change cell deposit into a different cell (and field) from the lane's run,
// so they are queued per wavefront in LDS and deposited 64 at a time, one per lane.
constexpr int kMqCap = 64;
// fx fz a0 a1 a2 j0 j1 j2, and the particle's density when densities are per particle
__host__ __device__ constexpr int mq_words(bool pw) { return pw ? 9 : 8; }

template <typename T>
struct MoverQ {
  T *v;      // [mq_words][kMqCap]
  int *idx;  // [2][kMqCap]: lower-left accumulator node, ring cell of the destination
};

template <typename T, bool PW>
__device__ __forceinline__ void drain_movers(const MoverQ<T> &q, int count, int lane,
                                             const AccLds &acc, int dplane, T w_uniform) {
  if (lane < count) {
    const T fx = q.v[0 * kMqCap + lane], fz = q.v[1 * kMqCap + lane];
    const T a0 = q.v[2 * kMqCap + lane], a1 = q.v[3 * kMqCap + lane];
    const T a2 = q.v[4 * kMqCap + lane], j0 = q.v[5 * kMqCap + lane];
    const T j1 = q.v[6 * kMqCap + lane], j2 = q.v[7 * kMqCap + lane];
    const T w = PW ? q.v[8 * kMqCap + lane] : w_uniform;
    const int o = q.idx[lane], rc = q.idx[kMqCap + lane];
#pragma unroll 1
    for (int c = 0; c < 4; ++c) {
      const int cx = c & 1, cz = c >> 1;
      const T W = (cx ? fx : T(1) - fx) * (cz ? fz : T(1) - fz);
      corner_add(acc, o + cx + cz * acc.LW, rc, c, W * a0, W * a1, W * a2, W * j0, W * j1, W * j2,
                 W * w, dplane);
    }
  }
}

// One particle's compact moments added to the LDS accumulators of its cell (lower-left
// accumulator node o, ring cell rc), corner by corner.  Lanes of odd index take the corners in
// the order (i,k+1), (i+1,k+1), (i,k), (i+1,k): neighbouring lanes often hold particles of one
// cell, and same-address atomics of one instruction are serialised (different rows cost less).
template <typename T>
__device__ __forceinline__ void deposit_one(const AccLds &acc, int o, int rc, T fx, T fz,
                                            const Compact<T> &m, T w, int dplane) {
  // odd lanes take the upper row of corners first (corners 2, 3, 0, 1)
  const bool odd = threadIdx.x & 1;
  const T gx[2] = {T(1) - fx, fx};
  const T gz[2] = {odd ? fz : T(1) - fz, odd ? T(1) - fz : fz};
  const int orow[2] = {o + (odd ? acc.LW : 0), o + (odd ? 0 : acc.LW)};
  const int crow[2] = {odd ? 2 : 0, odd ? 0 : 2};
#pragma unroll
  for (int c0 = 0; c0 < 4; ++c0) {
    const int cx = c0 & 1, row = c0 >> 1;
    const T W = gx[cx] * gz[row];
    corner_add(acc, orow[row] + cx, rc, crow[row] + cx, W * m.a0, W * m.a1, W * m.a2, W * m.j0,
               W * m.j1, W * m.j2, W * w, dplane);
  }
}

// Chunk-of-2 form: a particle whose new cell (gi, gk) lies outside the tile adds its moments to
// the global moment planes at once, at the cell's 4 corner nodes: the same products as an LDS
// deposit, with S-hat expanded with that cell's B as the fold expands the per-cell sums.  At
// a few particles per cell about one in three hundred leaves its tile in a cycle, and the
// tile's LDS then holds the nodes and cells of the tile alone.
template <typename T>
__device__ void deposit_global(const StepArgs &a, int gi, int gk, T fx, T fz, const Compact<T> &m,
                               T w, T B0t, T B1t, T B2t, int dplane) {
  const GridArgs &g = a.g;
  const int64_t nn = g.nnodes;
  const int gi1 = (g.bc_x == PIC_BC_PERIODIC && gi + 1 == g.nx) ? 0 : gi + 1;
  const int gk1 = gk + 1 == g.nz ? 0 : gk + 1;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const int cx = c & 1, cz = c >> 1;
    const T W = (cx ? fx : T(1) - fx) * (cz ? fz : T(1) - fz);
    const double A0 = (double)(W * m.a0), A1 = (double)(W * m.a1), A2 = (double)(W * m.a2);
    const double B0 = (double)B0t, B1 = (double)B1t, B2 = (double)B2t;
    double *M = a.M + ((int64_t)(cz ? gk1 : gk) * g.nxn + (cx ? gi1 : gi));
    unsafeAtomicAdd(M, fma(A2, B0 * B0, A0));
    unsafeAtomicAdd(M + nn, fma(A2, B0 * B1, A1 * B2));
    unsafeAtomicAdd(M + 2 * nn, fma(A2, B0 * B2, -A1 * B1));
    unsafeAtomicAdd(M + 3 * nn, fma(A2, B1 * B0, -A1 * B2));
    unsafeAtomicAdd(M + 4 * nn, fma(A2, B1 * B1, A0));
    unsafeAtomicAdd(M + 5 * nn, fma(A2, B1 * B2, A1 * B0));
    unsafeAtomicAdd(M + 6 * nn, fma(A2, B2 * B0, A1 * B1));
    unsafeAtomicAdd(M + 7 * nn, fma(A2, B2 * B1, -A1 * B0));
    unsafeAtomicAdd(M + 8 * nn, fma(A2, B2 * B2, A0));
    unsafeAtomicAdd(M + 9 * nn, (double)(W * m.j0));
    unsafeAtomicAdd(M + 10 * nn, (double)(W * m.j1));
    unsafeAtomicAdd(M + 11 * nn, (double)(W * m.j2));
    unsafeAtomicAdd(M + (9 + dplane) * nn, (double)(W * w));
    if (a.mflag) a.mflag[((int64_t)(cz ? gk1 : gk) * g.nxn + (cx ? gi1 : gi)) / kFlagNodes] = 1;
  }
}

// LDS layout of the particle kernel (byte offsets): the moment accumulators (delta-j and
// density per node, S-hat scalars per cell corner), the fields the tile's particles read (E-bar
// on the tile's nodes, H^{n+1/2} on its cells, H^{n+3/2} on its cells plus the one-cell ring a
// particle can move into), the per-wave mover queues, per species the int move counters of the
// tile's cells and the arrival counts of the tile's cells and their ring, and the first and
// end slot of every tile row of every species slot.  Two layouts: with mover queues
// (qwords > 0) the accumulators cover the tile and its ring; without (the chunk-of-2 form) they
// cover the tile's own nodes and cells, particles leaving the tile deposit to the global
// planes, and the arrivals are summed from the move counters (no arrival array), which brings
// a 32 x 4 tile of two species to 40 KB: four blocks per CU.  Accumulators are FP64; fields
// and queues use the kernel's arithmetic type.
struct TileLds {
  int LW, LH, plane;          // accumulator node grid (tx + 3) x (tz + 3), or (tx + 1) x (tz + 1)
  int EW, EPL;                // E-bar node grid (tx + 1) x (tz + 1)
  int HPL;                    // H^{n+1/2} cells tx x tz
  int NW, NPL;                // H^{n+3/2} cells (tx + 2) x (tz + 2)
  int CPL;                    // pitch of the S-hat corner planes: NPL, or HPL padded
  int n_node;                 // node accumulator planes: 3 + species
  size_t acc, accc, eb, ho, hn, mq, cnt, arr, rows;  // byte offsets
  size_t bytes;
  __host__ __device__ TileLds(int n_planes, int tx, int tz, int tsize, int qwords) {
    const int ring = qwords ? 1 : 0;
    LW = tx + 1 + 2 * ring;
    LH = tz + 1 + 2 * ring;
    plane = LW * LH;
    EW = tx + 1;
    EPL = EW * (tz + 1);
    HPL = tx * tz;
    NW = tx + 2;
    NPL = NW * (tz + 2);
    // without the ring the corner-plane pitch is padded to 4 (mod 8) doubles: the two lanes of
    // one cell, whose corners are two planes apart, then use complementary LDS banks
    CPL = ring ? NPL : HPL + ((4 - HPL % 8) + 8) % 8;
    n_node = 3 + (n_planes - 12);
    acc = 0;
    accc = acc + (size_t)n_node * plane * sizeof(double);
    eb = accc + (size_t)12 * CPL * sizeof(double);
    ho = eb + 3 * (size_t)EPL * tsize;
    hn = ho + 3 * (size_t)HPL * tsize;
    mq = (hn + 3 * (size_t)NPL * tsize + 7) & ~(size_t)7;
    cnt = mq + (qwords ? (size_t)(kBlock / 64) * kMqCap * ((size_t)qwords * tsize + 2 * sizeof(int)) : 0);
    arr = cnt + (size_t)(n_node - 3) * tx * tz * kMoveCodes * sizeof(int);
    rows = arr + (ring ? (size_t)(n_node - 3) * (tx + 2) * (tz + 2) * sizeof(int) : 0);
    bytes = rows + (size_t)(n_node - 3) * tz * 2 * sizeof(int);
  }
};

// Particle state in either form, as the kernel's arithmetic type: cell (i, k), in-cell offsets
// (fx, fz) and momentum.  FP64 keeps positions in cell units; the mixed form keeps the cell key
// and FP32 offsets.  Src holds the species' source arrays in registers for the whole species.
template <bool MIXED>
struct Pstate;
template <>
struct Pstate<false> {
  double x, z, u0, u1, u2;
  struct Src {
    const double *a[5];
    __device__ __forceinline__ explicit Src(const SpeciesArgs &sp) {
#pragma unroll
      for (int v = 0; v < 5; ++v) a[v] = sp.src[v];
    }
  };
  __device__ __forceinline__ void load(const Src &s, int p) {
    x = s.a[0][p];
    z = s.a[1][p];
    u0 = s.a[2][p];
    u1 = s.a[3][p];
    u2 = s.a[4][p];
  }
};
template <>
struct Pstate<true> {
  int cell;
  float x, z, u0, u1, u2;  // x, z: in-cell offsets
  struct Src {
    const int32_t *c;
    const float *a[5];
    __device__ __forceinline__ explicit Src(const SpeciesArgs &sp) {
      c = sp.msrc_cell;
#pragma unroll
      for (int v = 0; v < 5; ++v) a[v] = sp.msrc[v];
    }
  };
  __device__ __forceinline__ void load(const Src &s, int p) {
    cell = s.c[p];
    x = s.a[0][p];
    z = s.a[1][p];
    u0 = s.a[2][p];
    u1 = s.a[3][p];
    u2 = s.a[4][p];
  }
};

// One block per tile of cells (tile rows are cell rows), one wavefront per tile row (or per
// part of a row when the tile has fewer rows than wavefronts).  The row's particles (a
// contiguous range of the cell-sorted order) are split into 64 contiguous runs, one per lane;
// run lengths differ by at most one.  A lane accumulates the deposits of
// particles that stay in their cell in registers and adds them to the LDS tile when its run
// enters the next cell, so LDS atomics are issued once per (lane, cell) instead of once per
// particle; particles changing cell go through a per-wave queue.  The pushed state of the
// particle at iteration `it` of lane `l` is written to location row_start + 64 it + l, which
// makes the stores (and next cycle's loads through the permutation) coalesced.
// MIXED selects the mixed-precision form: FP32 state, gather, push and per-lane partial sums,
// added into FP64 LDS accumulators and the FP64 moment planes.  With chunks of 4 the FP64 form
// needs about 230 VGPRs (two waves per SIMD) and the FP32 form about 150 (three); the
// chunk-of-2 form needs about 120 and 105 (four).  IDS adds the copy of particle ids
// (tests only).  PW selects per-particle densities: each particle's moments are those of unit
// density times its own density, which is read with the state and written with the pushed
// state (a species with one density reads it from a one-element array with stride 0).  CH is
// the chunk of particles a lane loads at once: 4, or 2 where a lane holds about two particles
// per row.  The chunk-of-2 form deposits each particle into LDS at once (no register sums or
// mover queue), reads the fields for every particle, keeps accumulators for the tile's own
// nodes and cells only and sends the moments of a particle that leaves the tile to the global
// planes: about 120 VGPRs (FP64) and 40 KB of LDS at 32 x 4, four blocks per CU.
template <bool PUSH, bool MIXED, bool IDS, bool PW, int CH = 4>
__device__ __forceinline__ void particles_body(const StepArgs &a, int tile) {
  using T = typename std::conditional<MIXED, float, double>::type;
  const GridArgs &g = a.g;
  const TileArgs &t = a.t;
  const int tzi = tile / t.ntx, txi = tile - tzi * t.ntx;
  const int i0 = txi * t.tx, k0 = tzi * t.tz;
  const int i1 = min(i0 + t.tx, g.nx), k1 = min(k0 + t.tz, g.nz);
  const int ntc = t.tx * t.tz;
  const int64_t nn = g.nnodes, nc = g.ncells;

  extern __shared__ double lds[];
  char *ldsb = reinterpret_cast<char *>(lds);
  constexpr int kQw = mq_words(PW);
  const TileLds Lo(g.n_planes, t.tx, t.tz, (int)sizeof(T), (PUSH && CH == 2) ? 0 : kQw);
  const AccLds acc{reinterpret_cast<double *>(ldsb + Lo.acc),
                   reinterpret_cast<double *>(ldsb + Lo.accc), Lo.plane, Lo.CPL, Lo.LW, Lo.NW};
  T *Eb = reinterpret_cast<T *>(ldsb + Lo.eb);
  T *Ho = reinterpret_cast<T *>(ldsb + Lo.ho);
  T *Hn = reinterpret_cast<T *>(ldsb + Lo.hn);
  int *cntL = reinterpret_cast<int *>(ldsb + Lo.cnt);
  int *arrL = reinterpret_cast<int *>(ldsb + Lo.arr);  // the layout with the ring
  const int LW = Lo.LW, plane = Lo.plane;
  const int n_acc = Lo.n_node * plane + 12 * Lo.CPL;  // node planes, then cell-corner planes

  for (int e = threadIdx.x; e < n_acc; e += blockDim.x) acc.node[e] = 0.0;
  // the chunk-of-2 form: accumulators over the tile's own nodes and cells (no ring)
  constexpr bool kTileOnly = PUSH && CH == 2;
  const int AW = t.tx + 2, AH = t.tz + 2;  // arrival counts: the tile's cells and their ring
  if (PUSH) {
    const int nsl = Lo.n_node - 3;
    for (int e = threadIdx.x; e < nsl * ntc * kMoveCodes; e += blockDim.x) cntL[e] = 0;
    if constexpr (!kTileOnly)
      for (int e = threadIdx.x; e < nsl * AW * AH; e += blockDim.x) arrL[e] = 0;
  }
  const int cw = i1 - i0, chh = k1 - k0;  // the tile's cells inside the grid
  // a tile and its two-cell ring fit in the grid along an axis: wraps need one compare there
  const bool nearx = g.nx >= t.tx + 3, nearz = g.nz >= t.tz + 3;
  // Stage the fields of the tile and the slot range of every tile row of every species in one
  // pass: a thread issues all its loads (at clamped, valid addresses) before it stores any, so
  // the block waits for one memory round trip instead of one per array.
  const int nrows_t = k1 - k0;
  int *rowsL = reinterpret_cast<int *>(ldsb + Lo.rows);  // [species][row]: first, end slot
  const int n_stage = max(max(Lo.HPL, nrows_t), PUSH ? max(Lo.EPL, Lo.NPL) : 0);
  for (int e = threadIdx.x; e < n_stage; e += blockDim.x) {
    // H^{n+1/2} on the tile's cells
    const int eh = min(e, Lo.HPL - 1);
    const int hk = SmallDiv(t.tx).q(eh), hi = eh - hk * t.tx;
    const bool h_in = e < Lo.HPL && i0 + hi < g.nx && k0 + hk < g.nz;
    const int64_t ch = (int64_t)min(k0 + hk, g.nz - 1) * g.nx + min(i0 + hi, g.nx - 1);
    double ho[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) ho[q] = a.Hold[q * nc + ch];
    // first and end slot of tile row e of every species (threads e < rows of the tile)
    const bool r_th = e < nrows_t;
    const int64_t rowc = (int64_t)(k0 + min(e, nrows_t - 1)) * g.nx;
    int rbv[kMaxSpecies], rev[kMaxSpecies];
#pragma unroll
    for (int q = 0; q < kMaxSpecies; ++q) {
      rbv[q] = 0;
      rev[q] = 0;
      if (q < a.nsp && a.sp[q].active && r_th) {
        rbv[q] = a.sp[q].cs[rowc + i0];
        rev[q] = a.sp[q].cs[rowc + i1];
      }
    }
    double eo[3], en[3], hn[3];
    bool e_in = false, n_in = false;
    if (PUSH) {
      // E-bar on the tile's nodes
      const int ee = min(e, Lo.EPL - 1);
      const int ek = SmallDiv(Lo.EW).q(ee), ei = ee - ek * Lo.EW;
      int gi = i0 + ei;
      const int gk = wrap_t(k0 + ek, g.nz, nearz);
      e_in = e < Lo.EPL;
      if (g.bc_x == PIC_BC_PERIODIC) gi = wrap_t(gi, g.nx, nearx); else e_in = e_in && gi <= g.nx;
      const int64_t n = (int64_t)gk * g.nxn + min(gi, g.nxn - 1);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        eo[q] = a.Eold[q * nn + n];
        en[q] = a.Enew[q * nn + n];
      }
      // H^{n+3/2} on the tile's cells and their ring
      const int en_ = min(e, Lo.NPL - 1);
      const int nk = SmallDiv(Lo.NW).q(en_), ni = en_ - nk * Lo.NW;
      int gi2 = i0 - 1 + ni;
      const int gk2 = wrap_t(k0 - 1 + nk, g.nz, nearz);
      n_in = e < Lo.NPL;
      if (g.bc_x == PIC_BC_PERIODIC) gi2 = wrap_t(gi2, g.nx, nearx); else n_in = n_in && gi2 >= 0 && gi2 < g.nx;
      const int64_t c2 = (int64_t)gk2 * g.nx + min(max(gi2, 0), g.nx - 1);
#pragma unroll
      for (int q = 0; q < 3; ++q) hn[q] = a.Hnew[q * nc + c2];
    }
    if (e < Lo.HPL) {
#pragma unroll
      for (int q = 0; q < 3; ++q) Ho[q * Lo.HPL + e] = h_in ? (T)ho[q] : T(0);
    }
    if (r_th) {
#pragma unroll
      for (int q = 0; q < kMaxSpecies; ++q) {
        if (q < a.nsp) {
          rowsL[2 * (q * nrows_t + e)] = rbv[q];
          rowsL[2 * (q * nrows_t + e) + 1] = rev[q];
        }
      }
    }
    if (PUSH && e < Lo.EPL) {
#pragma unroll
      for (int q = 0; q < 3; ++q) Eb[q * Lo.EPL + e] = e_in ? (T)(0.5 * (eo[q] + en[q])) : T(0);
    }
    if (PUSH && e < Lo.NPL) {
#pragma unroll
      for (int q = 0; q < 3; ++q) Hn[q * Lo.NPL + e] = n_in ? (T)hn[q] : T(0);
    }
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  MoverQ<T> mq;
  {
    char *qb = ldsb + Lo.mq + (size_t)wave * kMqCap * ((size_t)kQw * sizeof(T) + 2 * sizeof(int));
    mq.v = reinterpret_cast<T *>(qb);
    mq.idx = reinterpret_cast<int *>(qb + (size_t)kMqCap * kQw * sizeof(T));
  }
  const T cxT = (T)g.cx, czT = (T)g.cz;

  for (int s = 0; s < a.nsp; ++s) {
    const SpeciesArgs &sp = a.sp[s];
    if (!sp.active) continue;
    int *const cntS = cntL + s * ntc * kMoveCodes;  // the species' move counters
    const SpConst<T> K{(T)sp.beta, (T)(PW ? sp.cS1 : sp.cS), (T)(PW ? sp.kJ1 : sp.kJ), (T)sp.w};
    const typename Pstate<MIXED>::Src src(sp);
    // per-particle densities: index p * wstride (stride 0 reads a species' single density)
    const T *wsrc = nullptr;
    T *wdst = nullptr;
    if constexpr (MIXED) {
      wsrc = sp.msrc_w;
      wdst = sp.mdst_w;
    } else {
      wsrc = sp.src_w;
      wdst = sp.dst_w;
    }
    const int wstride = sp.w_stride;
    const int32_t *perm = sp.perm;
    const int dplane = 3 + s;  // density plane of the species in the node accumulators
    // A tile with fewer rows than wavefronts splits each row's particles into wpr contiguous
    // parts, one per wavefront, so short tiles keep every wavefront busy.
    const int nrows = k1 - k0;
    const int wpr = nrows < nwaves ? nwaves / nrows : 1;  // 1, 2 or 4 (four wavefronts)
    const int wsh = wpr == 4 ? 2 : (wpr == 2 ? 1 : 0);
    const int part = wave % wpr;
    for (int r = k0 + wave / wpr; r < k1; r += nwaves / wpr) {
      const int rb = rowsL[2 * (s * nrows_t + (r - k0))], re = rowsL[2 * (s * nrows_t + (r - k0)) + 1];
      const int jb = rb + (int)(((uint32_t)(re - rb) * (uint32_t)part) >> wsh);
      const int je = rb + (int)(((uint32_t)(re - rb) * (uint32_t)(part + 1)) >> wsh);
      const int L = je - jb;
      if (L == 0) continue;
      const int q = L >> 6, rr = L & 63;
      const int my_n = q + (lane < rr ? 1 : 0);
      const int start = jb + lane * q + min(lane, rr);
      const int iters = q + (rr > 0 ? 1 : 0);
      const int lz = r - k0 + 1;
      const int lk = r - k0;
      CellAcc<T> ca;
      ca.clear();
      ca.cell = -1;
      int nq = 0;  // movers queued by this wavefront (uniform)
      // fields of the cell the lane's run is in, kept in registers while the run stays in it:
      // H^{n+1/2} (fB) and E-bar at its 4 nodes (fE, the push)
      T fB0 = T(0), fB1 = T(0), fB2 = T(0), fE[12];
      // The run is processed in chunks of kChunk particles: the chunk's state loads are issued
      // together (with the next chunk's permutation entries), then its particles are pushed
      // from registers in an unrolled sequence.  Global stores share the vector-memory counter
      // with loads, so a load whose value is still in flight across a loop iteration makes
      // the compiler wait for all earlier stores too; keeping every loaded value inside one
      // iteration lets it wait for the loads alone.  Loads are issued unconditionally (slots
      // past a lane's run read a location inside the state arrays, and their values go
      // unused): a load under a divergent branch also forces a full wait.
      constexpr int kChunk = CH;
      // two particles per chunk: the form for about two particles per lane and row, where a
      // lane's register sums would hold one or two particles; it deposits each particle into
      // LDS directly (no register sums, row-end reduction or mover queue: fewer registers)
      constexpr bool kDirect = PUSH && CH == 2;
      Pstate<MIXED> cb[kChunk];
      int cp_[kChunk], np_[kChunk];
      T cw_[kChunk];
      // A chunk's permutation entries come in one 16-byte load per lane (the array is padded
      // so the load stays inside it); entries past the lane's run are clamped to a location
      // inside the state arrays and their particles go unused.
      static_assert((kChunk == 4 || kChunk == 2) && kPermPad >= 2 * kChunk,
                    "one int4 or int2 of entries per chunk");
      const uint32_t loc_max = (uint32_t)(sp.cap - 1);
      auto perm4 = [&](int first, int out[kChunk]) {
        if constexpr (kChunk == 4) {
          int4 v;
          __builtin_memcpy(&v, perm + first, sizeof(v));
          out[0] = (int)min((uint32_t)v.x, loc_max);
          out[1] = (int)min((uint32_t)v.y, loc_max);
          out[2] = (int)min((uint32_t)v.z, loc_max);
          out[3] = (int)min((uint32_t)v.w, loc_max);
        } else {
          int2 v;
          __builtin_memcpy(&v, perm + first, sizeof(v));
          out[0] = (int)min((uint32_t)v.x, loc_max);
          out[1] = (int)min((uint32_t)v.y, loc_max);
        }
      };
      perm4(start, np_);
      // all lanes run the same number of iterations so the mover queue stays wave-uniform
      for (int c0 = 0; c0 < iters; c0 += kChunk) {
#pragma unroll
        for (int kk = 0; kk < kChunk; ++kk) {
          cp_[kk] = np_[kk];
          cb[kk].load(src, cp_[kk]);
          if constexpr (PW) cw_[kk] = wsrc[cp_[kk] * wstride];
        }
        perm4(start + c0 + kChunk, np_);
#pragma unroll
        for (int kk = 0; kk < kChunk; ++kk) {
          const int it = c0 + kk;
          if (it >= iters) break;
          const bool act = it < my_n;
          const int j = start + it;
          const int p = cp_[kk];
          const Pstate<MIXED> &ps = cb[kk];
          int i, k;
          T fx, fz;
          if constexpr (MIXED) {
            k = r;
            i = ps.cell - r * g.nx;
            fx = ps.x;
            fz = ps.z;
          } else {
            i = (int)floor(ps.x);
            k = (int)floor(ps.z);
            fx = ps.x - (double)i;
            fz = ps.z - (double)k;
          }
          const T u0 = ps.u0, u1 = ps.u1, u2 = ps.u2;
          const T wp = PW ? cw_[kk] : K.w;  // the particle's density
          const bool ok = act && k == r && i >= i0 && i < i1;
          if (act && !ok) {
            atomicOr(a.flags, kFlagOrder);
            if (PUSH) sp.locode[j] = ((uint32_t)(jb + it * 64 + lane) << 4) | kAbsorbed;
          }
          // Lanes without a valid particle run the arithmetic on a valid cell of the tile and
          // discard the results, so the main path has no branches around it.
          const int li = ok ? i - i0 : max(ca.cell, 0);
          const int hc = lk * t.tx + li;
          // On entering a new cell: read its fields, use them, and only then flush the previous
          // cell's accumulator.  LDS operations complete in order, so a read issued after the
          // flush's atomics (or consumed while they are in flight) would wait for all of them.
          // The chunk-of-2 form reads them for every particle (a lane holds about two per row,
          // and fields kept across particles would hold about 30 registers).
          const bool newcell = kDirect || (ok && li != ca.cell);
          if (newcell) {
            fB0 = Ho[hc];
            fB1 = Ho[Lo.HPL + hc];
            fB2 = Ho[2 * Lo.HPL + hc];
            if (PUSH) {
              const int e00 = lk * Lo.EW + li;
#pragma unroll
              for (int qq = 0; qq < 3; ++qq) {
                const T *f = Eb + qq * Lo.EPL + e00;
                fE[4 * qq] = f[0];
                fE[4 * qq + 1] = f[1];
                fE[4 * qq + 2] = f[Lo.EW];
                fE[4 * qq + 3] = f[Lo.EW + 1];
              }
            }
          }
          const T one = T(1);
          const T ginv = rsqT(fmaT(u2, u2, fmaT(u1, u1, fmaT(u0, u0, one))));  // 1 / gamma(u^n)
          if (!PUSH) {
            Compact<T> m0 = compact_moments(K, ginv, u0, u1, u2, fB0, fB1, fB2);
            if constexpr (PW) scale_compact(m0, wp);
            if (newcell) {
              if (ca.cell >= 0) ca.flush(acc, lz, dplane);
              ca.clear();
              ca.cell = li;
            }
            if (ok) ca.add(fx, fz, m0, wp);
          } else {
            bool mover = false;
            int mo = 0, mh = 0;
            T fx2, fz2;
            Compact<T> m;
            {
              // gather E-bar at x^{n+1/2} from the 4 corner nodes (linear weights)
              const T W0 = (one - fx) * (one - fz), W1 = fx * (one - fz);
              const T W2 = (one - fx) * fz, W3 = fx * fz;
              T Ep[3];
#pragma unroll
              for (int qq = 0; qq < 3; ++qq)
                Ep[qq] = fmaT(W3, fE[4 * qq + 3],
                              fmaT(W2, fE[4 * qq + 2], fmaT(W1, fE[4 * qq + 1], W0 * fE[4 * qq])));
              // implicit push: with a = u + beta E and b = beta B / gamma,
              // u-bar = R a = (a + a x b + (a.b) b) / (1 + b.b), and u' = 2 u-bar - u
              const T bg = K.beta * ginv;
              const T bx = bg * fB0, by = bg * fB1, bz = bg * fB2;
              const T a0 = fmaT(K.beta, Ep[0], u0), a1 = fmaT(K.beta, Ep[1], u1);
              const T a2 = fmaT(K.beta, Ep[2], u2);
              const T inv = rcpT(fmaT(bz, bz, fmaT(by, by, fmaT(bx, bx, one))));
              const T ab = fmaT(a2, bz, fmaT(a1, by, a0 * bx));
              const T n0 = fmaT(T(2), fmaT(ab, bx, a0 + fmaT(a1, bz, -(a2 * by))) * inv, -u0);
              const T n1 = fmaT(T(2), fmaT(ab, by, a1 + fmaT(a2, bx, -(a0 * bz))) * inv, -u1);
              const T n2 = fmaT(T(2), fmaT(ab, bz, a2 + fmaT(a0, by, -(a1 * bx))) * inv, -u2);
              const T g1sq = fmaT(n2, n2, fmaT(n1, n1, fmaT(n0, n0, one)));
              const T rg1 = rsqT(g1sq);  // 1 / gamma(u^{n+1})
              const T vx = n0 * rg1, vz = n2 * rg1;
              // position advance: FP64 in cell units; mixed as FP32 offset with integer carry
              T xn, zn;
              int i2, k2;
              bool alive = ok;
              bool finite;
              if constexpr (MIXED) {
                xn = fx + cxT * vx;
                zn = fz + czT * vz;
                finite = isfinite(g1sq) && isfinite(xn) && isfinite(zn);
                const int cxi = finite ? (int)floorT(xn) : 0, czi = finite ? (int)floorT(zn) : 0;
                xn -= (T)cxi;
                zn -= (T)czi;
                int ci = i + cxi, ck = k + czi;
                if (xn >= one) { xn = T(0); ci += 1; }
                if (zn >= one) { zn = T(0); ck += 1; }
                if (g.bc_x == PIC_BC_PERIODIC) {
                  ci = wrap1(ci, g.nx);
                } else if (ci < 0 || ci >= g.nx) {
                  alive = false;
                }
                ck = wrap1(ck, g.nz);
                i2 = ci;
                k2 = ck;
              } else {
                xn = ps.x + g.cx * vx;
                zn = ps.z + g.cz * vz;
                if (g.bc_x == PIC_BC_PERIODIC) {
                  if (xn < 0.0) xn += (double)g.nx;
                  if (xn >= (double)g.nx) xn -= (double)g.nx;
                } else if (xn < 0.0 || xn >= (double)g.nx) {
                  alive = false;
                }
                if (zn < 0.0) zn += (double)g.nz;
                if (zn >= (double)g.nz) zn -= (double)g.nz;
                finite = isfinite(g1sq) && isfinite(xn) && isfinite(zn);
                i2 = finite ? (int)floor(xn) : i;
                k2 = finite ? (int)floor(zn) : k;
              }
              if (ok && !finite) atomicOr(a.flags, kFlagNonFinite);
              alive = alive && finite;
              int di = i2 - i, dk = k2 - k;
              if (di > 1) di -= g.nx;
              if (di < -1) di += g.nx;
              if (dk > 1) dk -= g.nz;
              if (dk < -1) dk += g.nz;
              const bool jump = di < -1 || di > 1 || dk < -1 || dk > 1;
              if (alive && jump) atomicOr(a.flags, kFlagJump);
              alive = alive && !jump;
              if (!alive) {
                di = 0;
                dk = 0;
              }
              const uint32_t code = alive ? (uint32_t)((dk + 1) * 3 + (di + 1)) : kAbsorbed;
              // moments M^{n+3/2} at x^{n+3/2} with u^{n+1}, 1/gamma(u^{n+1}) and H^{n+3/2}
              // of the new cell (read before any LDS atomic of this particle is issued)
              const int hn = (lk + dk + 1) * Lo.NW + (li + di + 1);
              m = compact_moments(K, rg1, n0, n1, n2, Hn[hn], Hn[Lo.NPL + hn], Hn[2 * Lo.NPL + hn]);
              // the new cell, tile-local (a dead particle stays, unused)
              const int ldx = li + di, ldz = lk + dk;
              const bool inside = ldx >= 0 && ldx < cw && ldz >= 0 && ldz < chh;
              if constexpr (PW) scale_compact(m, wp);
              if constexpr (MIXED) {
                fx2 = xn;
                fz2 = zn;
              } else {
                fx2 = xn - (double)i2;
                fz2 = zn - (double)k2;
              }
              if (newcell) {
                if constexpr (!kDirect) {
                  if (ca.cell >= 0) ca.flush(acc, lz, dplane);
                  ca.clear();
                }
                ca.cell = li;
              }
              if constexpr (MIXED) {
                if (ok) {
                  const int loc = jb + it * 64 + lane;
                  sp.mdst_cell[loc] = k2 * g.nx + i2;
                  sp.mdst[0][loc] = xn;
                  sp.mdst[1][loc] = zn;
                  sp.mdst[2][loc] = n0;
                  sp.mdst[3][loc] = n1;
                  sp.mdst[4][loc] = n2;
                  if (PW && wstride) wdst[loc] = wp;
                  sp.locode[j] = ((uint32_t)loc << 4) | code;
                }
              } else {
                // FP64: every lane issues the stores, without a branch (a lane without a
                // particle passes an offset the hardware drops), so the compiler knows how many
                // stores each particle issues and waits for the next particle's loads alone.
                // (The mixed form measured no gain from this and keeps plain stores.)
                const int loc = jb + it * 64 + lane;
                store_or_drop(sp.dst[0], loc, ok, xn);
                store_or_drop(sp.dst[1], loc, ok, zn);
                store_or_drop(sp.dst[2], loc, ok, n0);
                store_or_drop(sp.dst[3], loc, ok, n1);
                store_or_drop(sp.dst[4], loc, ok, n2);
                if constexpr (PW) store_or_drop(wdst, loc, ok && wstride != 0, wp);
                store_or_drop(sp.locode, j, ok, ((uint32_t)loc << 4) | code);
              }
              if (ok) {
                // particle ids (tests only): a separate instantiation, so that its load, which
                // is waited for at once, does not enter the wait counts of the kernel without ids
                if (IDS && sp.dst_id) sp.dst_id[jb + it * 64 + lane] = sp.src_id[p];
                if (code != kAbsorbed) atomicAdd(&cntS[hc * kMoveCodes + code], 1);
              }
              // stayers add to the lane's accumulator, movers go through the queue (with few
              // particles per lane every particle goes to the LDS accumulators at once, or to
              // the global planes if it leaves the tile)
              if constexpr (kDirect) {
                if (alive && inside)
                  deposit_one(acc, ldz * LW + ldx, ldz * t.tx + ldx, fx2, fz2, m, wp, dplane);
                if (alive && !inside)
                  deposit_global(a, i2, k2, fx2, fz2, m, wp, Hn[hn], Hn[Lo.NPL + hn],
                                 Hn[2 * Lo.NPL + hn], dplane);
              } else if (alive && code == 4u) {
                ca.add(fx2, fz2, m, wp);
              } else if (alive) {
                mover = true;
                mo = (lz + dk) * LW + (li + 1 + di);
                mh = hn;
              }
            }
            // queue this iteration's movers; drain first if they would not fit
            const uint64_t mmask = __ballot(mover);
            const int nm = __popcll(mmask);
            if (nq + nm > kMqCap) {
              wave_sync();
              drain_movers<T, PW>(mq, nq, lane, acc, dplane, K.w);
              wave_sync();
              nq = 0;
            }
            if (mover) {
              const int e = nq + __popcll(mmask & lt_mask);
              mq.v[0 * kMqCap + e] = fx2;
              mq.v[1 * kMqCap + e] = fz2;
              mq.v[2 * kMqCap + e] = m.a0;
              mq.v[3 * kMqCap + e] = m.a1;
              mq.v[4 * kMqCap + e] = m.a2;
              mq.v[5 * kMqCap + e] = m.j0;
              mq.v[6 * kMqCap + e] = m.j1;
              mq.v[7 * kMqCap + e] = m.j2;
              if constexpr (PW) mq.v[8 * kMqCap + e] = wp;
              mq.idx[e] = mo;
              mq.idx[kMqCap + e] = mh;
            }
            nq += nm;
          }
        }
      }
      if constexpr (!kDirect) ca.flush_row_end(acc, lz, dplane, lane);
      if (PUSH && nq > 0) {
        wave_sync();
        drain_movers<T, PW>(mq, nq, lane, acc, dplane, K.w);
        wave_sync();
      }
    }
  }
  __syncthreads();
  // Move counts of the tile's cells, for the ranking.  The counts of every species are kept
  // until here, so the species need no barriers between them.
  for (int s = 0; s < a.nsp; ++s) {
    const SpeciesArgs &sp = a.sp[s];
    if (!PUSH || !sp.active) continue;
    const int *cntS = cntL + s * ntc * kMoveCodes;
    int *arrS = arrL + s * AW * AH;
    {
      const SmallDiv div_cw(cw);
      for (int e = threadIdx.x; e < chh * cw; e += blockDim.x) {
        const int lkk = div_cw.q(e), li = e - lkk * cw;
        const int64_t cg = (int64_t)(k0 + lkk) * g.nx + (i0 + li);
        const int *cl = cntS + (lkk * t.tx + li) * kMoveCodes;
        uint32_t mask = 0;
#pragma unroll
        for (int d = 0; d < kMoveCodes; ++d) {
          const int v = cl[d];
          // with code masks only the nonzero counts are written (most cells send all their
          // particles with one code)
          if (!a.count_masks || v) sp.cnt[(int64_t)d * nc + cg] = v;
          if (v) {
            mask |= 1u << d;
            if constexpr (!kTileOnly) atomicAdd(&arrS[(lkk + d / 3) * AW + (li + d % 3)], v);
          }
        }
        if (a.count_masks) sp.cmask[cg] = (uint16_t)mask;
      }
    }
  }
  // Fold the tile's accumulators into the global FP64 moment planes, one node per thread:
  // delta-j and the densities as they are; S-hat from the S-hat scalars of the (up to) four
  // cells around the node, each expanded with its cell's B (H^{n+3/2} after a push, H^{n+1/2}
  // for a deposit of the current state): S-hat = a0 I + a1 [B]x + a2 B B^T.
  const SmallDiv div_lw(LW);
  for (int idx = threadIdx.x; idx < plane; idx += blockDim.x) {
    const int lzz = div_lw.q(idx), lx = idx - lzz * LW;
    constexpr int kOff = kTileOnly ? 0 : 1;  // the ring's column and row before the tile
    int gx = i0 - kOff + lx;
    bool in = true;
    if (g.bc_x == PIC_BC_PERIODIC) gx = wrap_t(gx, g.nx, nearx); else in = gx >= 0 && gx <= g.nx;
    const int gz = wrap_t(k0 - kOff + lzz, g.nz, nearz);
    const int64_t node = (int64_t)gz * g.nxn + gx;
    // the field solve reads and clears the moment planes only under a set deposit flag: set
    // the flag of every node this fold adds to
    bool wrote = false;
    for (int pp = 0; pp < Lo.n_node; ++pp) {
      const double v = acc.node[pp * plane + idx];
      const int gp = pp < 3 ? 9 + pp : 12 + (pp - 3);
      if (in && v != 0.0) {
        unsafeAtomicAdd(&a.M[(int64_t)gp * nn + node], v);
        wrote = true;
      }
    }
    double S[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool any = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // the cell whose corner c is this node, tile-local (-1 and tx, tz: the ring)
      const int cx = lx - kOff - (c & 1), cz = lzz - kOff - (c >> 1);
      if (cx < -kOff || cx >= t.tx + kOff || cz < -kOff || cz >= t.tz + kOff) continue;
      const int rc = (cz + 1) * Lo.NW + (cx + 1);                 // in the ring's numbering
      const int ac = kTileOnly ? cz * t.tx + cx : rc;             // in the corner planes
      const double A0 = acc.cell[(0 * 4 + c) * Lo.CPL + ac];
      const double A1 = acc.cell[(1 * 4 + c) * Lo.CPL + ac];
      const double A2 = acc.cell[(2 * 4 + c) * Lo.CPL + ac];
      if (A0 == 0.0 && A1 == 0.0 && A2 == 0.0) continue;
      double B0 = 0.0, B1 = 0.0, B2 = 0.0;
      if (PUSH) {
        B0 = (double)Hn[rc];
        B1 = (double)Hn[Lo.NPL + rc];
        B2 = (double)Hn[2 * Lo.NPL + rc];
      } else if (cx >= 0 && cx < t.tx && cz >= 0 && cz < t.tz) {
        const int hc = cz * t.tx + cx;
        B0 = (double)Ho[hc];
        B1 = (double)Ho[Lo.HPL + hc];
        B2 = (double)Ho[2 * Lo.HPL + hc];
      }
      S[0] += fma(A2, B0 * B0, A0);
      S[1] += fma(A2, B0 * B1, A1 * B2);
      S[2] += fma(A2, B0 * B2, -A1 * B1);
      S[3] += fma(A2, B1 * B0, -A1 * B2);
      S[4] += fma(A2, B1 * B1, A0);
      S[5] += fma(A2, B1 * B2, A1 * B0);
      S[6] += fma(A2, B2 * B0, A1 * B1);
      S[7] += fma(A2, B2 * B1, -A1 * B0);
      S[8] += fma(A2, B2 * B2, A0);
      any = true;
    }
    if (any && in) {
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        if (S[r] != 0.0) {
          unsafeAtomicAdd(&a.M[(int64_t)r * nn + node], S[r]);
          wrote = true;
        }
      }
    }
    if (wrote && a.mflag) a.mflag[node / kFlagNodes] = 1;
  }
  if (PUSH) {
    // The particles the tile's cells send to each cell of the tile and its ring (the cell
    // (x - dx, z - dz) sends count[code (dx, dz)]), added to the per-cell arrival counts: the
    // sort's scan reads those instead of gathering nine counts per cell.
    // (the layout with the ring sums them in LDS during the count pass)
    if constexpr (!kTileOnly) __syncthreads();
    for (int s = 0; s < a.nsp; ++s) {
      const SpeciesArgs &sp = a.sp[s];
      if (!sp.active) continue;
      const int *cntS = cntL + s * ntc * kMoveCodes;
      const int *arrS = arrL + s * AW * AH;
      for (int e = threadIdx.x; e < AW * AH; e += blockDim.x) {
        const int az = SmallDiv(AW).q(e), ax = e - az * AW;
        int v = 0;
        if constexpr (kTileOnly) {
#pragma unroll
          for (int d = 0; d < kMoveCodes; ++d) {
            const int sx = ax - d % 3, sz = az - d / 3;  // the source cell, tile-local
            if (sx >= 0 && sx < cw && sz >= 0 && sz < chh) v += cntS[(sz * t.tx + sx) * kMoveCodes + d];
          }
        } else {
          v = arrS[e];
        }
        if (v == 0) continue;
        int gi = i0 - 1 + ax;
        const int gk = wrap1(k0 - 1 + az, g.nz);
        if (g.bc_x == PIC_BC_PERIODIC) gi = wrap1(gi, g.nx);
        atomicAdd(&sp.arr[(int64_t)gk * g.nx + gi], v);
      }
    }
  }
}

// Waves per SIMD: the register sums of the chunks of 4 hold two FP64 waves (three mixed); the
// chunk-of-2 form, without them, holds four in both precisions (at 32 x 4 cells and two
// species its LDS also lets four blocks share a CU).
template <bool PUSH, bool MIXED, bool IDS, bool PW, int CH = 4>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(CH == 2 ? 4 : 2 + MIXED, CH == 2 ? 4 : 2 + MIXED)))
void k_particles(const StepArgs a) {
  // clear the next order's tile flags (set by the scan of this cycle's sort); the grid has a
  // block for every tile index
  if (threadIdx.x == 0 && (int)blockIdx.x < a.t.ntiles) a.tile_active_next[blockIdx.x] = 0;
  const int tile = block_tile(a.t, a.tile_list);
  if (tile < 0) return;
  particles_body<PUSH, MIXED, IDS, PW, CH>(a, tile);
}

// ------------------------------------------------------------------------------------------
// Sort
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total too.
__device__ int block_excl_scan(int v, int *sh, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int inc = wave_incl_scan(v, lane);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wave) off += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Stable destinations of one tile's particles.  The destination base of every (cell, move
// code) of the tile is computed once into LDS; then one wavefront per tile row (or part of a
// row) walks the row's slots in order, 64 at a time: particles with the same (cell, code) in a
// group of 64 get consecutive ranks from ballots of the code's bits, and a per-wave LDS
// counter carries the rank across groups.
__device__ __forceinline__ void rank_body(const StepArgs &a, int tile, int species) {
  const GridArgs &g = a.g;
  const TileArgs &t = a.t;
  const int tzi = tile / t.ntx, txi = tile - tzi * t.ntx;
  const int i0 = txi * t.tx, k0 = tzi * t.tz;
  const int i1 = min(i0 + t.tx, g.nx), k1 = min(k0 + t.tz, g.nz);
  const int cw = i1 - i0, ch = k1 - k0;
  const int ntc = t.tx * t.tz;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
  extern __shared__ int ldsi[];
  const int ring_cells = (t.tx + 4) * (t.tz + 4);
  int *btab = ldsi;                                                   // [ntc][9]
  int *rowcs = ldsi + ntc * 9 + wave * (t.tx + 1);                    // [tx + 1] per wave
  int *ctr = ldsi + ntc * 9 + nwaves * (t.tx + 1) + wave * (t.tx * 10);  // [tx][10] per wave
  int *rcnt = ldsi + ntc * 9 + nwaves * (t.tx + 1 + t.tx * 10);       // [9][ring_cells]
  int *rcsn = rcnt + kMoveCodes * ring_cells;                         // [ring_cells]
  int *rkey = rcsn + ring_cells;                                      // [ring_cells]
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  // one block per (tile, species): twice the blocks of a per-tile launch, to overlap the
  // memory latency of the staging and walking phases
  {
    const int s = species;
    const SpeciesArgs &sp = a.sp[s];
    if (!sp.active) return;
    // A tile with fewer rows than wavefronts splits each row's slots into wpr contiguous
    // parts, one per wavefront.  A part that starts inside a cell first counts, per move code,
    // that cell's slots before the part, so its ranks continue the ones of the parts before.
    const int nrows = k1 - k0;
    const int wpr = nrows < nwaves ? nwaves / nrows : 1;
    const int part = wave % wpr;
    const int r_first = k0 + wave / wpr;
    // the first row's cell starts and counters, loaded together with the staging below
    if (r_first < k1) {
      for (int q = lane; q <= cw; q += 64) rowcs[q] = sp.cs[(int64_t)r_first * g.nx + i0 + q];
      for (int q = lane; q < cw * 10; q += 64) ctr[q] = 0;
    }
    const int total = sp.cs_new[g.ncells];
    // counts of the tile and a one-cell ring (sources of the destinations reached from the
    // tile), and next-order starts of the same region, staged in LDS
    const int RW = t.tx + 4, RH = t.tz + 4;  // ring of two cells: destinations +-1, their sources +-1
    // a tile and its ring fit in the grid along an axis: wraps need one compare there
    const bool nearx = g.nx >= t.tx + 4, nearz = g.nz >= t.tz + 4;
    const SmallDiv div_rw(RW), div_tx(t.tx), div_tz(t.tz);
    for (int e = threadIdx.x; e < RW * RH; e += blockDim.x) {
      const int rz = div_rw.q(e), rx = e - rz * RW;
      int gi = i0 - 2 + rx;
      const int gk = wrap_t(k0 - 2 + rz, g.nz, nearz);
      bool in = true;
      if (g.bc_x == PIC_BC_PERIODIC) gi = wrap_t(gi, g.nx, nearx); else in = gi >= 0 && gi < g.nx;
      // The counts are valid only in tiles that held particles (the tile flag); they are
      // loaded together with the flag (from a cell inside the grid) and kept or dropped after.
      const int gic = min(max(gi, 0), g.nx - 1);
      const int64_t c = (int64_t)gk * g.nx + gic;
      const bool act = in && a.tile_active[div_tz.q(gk) * t.ntx + div_tx.q(gic)] != 0;
      int v[kMoveCodes];
#pragma unroll
      for (int d = 0; d < kMoveCodes; ++d) v[d] = sp.cnt[(int64_t)d * g.ncells + c];
      const int csn_c = sp.cs_new[c];
#pragma unroll
      for (int d = 0; d < kMoveCodes; ++d) rcnt[d * RW * RH + e] = act ? v[d] : 0;
      rcsn[e] = in ? csn_c : 0;
      rkey[e] = in ? (int)c : -1;  // sort key of the cell; -1 outside an absorbing axis
    }
    __syncthreads();
    // (a tile without particles of this species has no counts: its table stays zero and its
    // rows are empty)
    // one (code, cell) pair per thread, consecutive threads on consecutive cells of one code
    // (so their LDS reads of the staged counts fall in different banks)
    const SmallDiv div_cells(ch * cw), div_cw(cw);
    for (int e = threadIdx.x; e < ch * cw * kMoveCodes; e += blockDim.x) {
      const int d = div_cells.q(e), cell = e - d * (ch * cw);
      const int lk = div_cw.q(cell), li = cell - lk * cw;
      // First slot, in the next order, of the particles moving from this cell with code d:
      // the start of the destination cell plus the particles arriving there from source
      // cells earlier in the current (cell-sorted) order.  Destination and sources lie in
      // the ring, so they are found by ring offsets; the order uses the cells' sort keys.
      const int rc = (lk + 2) * RW + (li + 2);
      int b = 0;
      if (rcnt[d * RW * RH + rc] > 0) {
        const int rd = rc + (d / 3 - 1) * RW + (d % 3 - 1);  // destination
        if (rkey[rd] >= 0) {
          const int key_c = rkey[rc];
          b = rcsn[rd];
#pragma unroll
          for (int d2 = 0; d2 < kMoveCodes; ++d2) {
            const int rs = rd - (d2 / 3 - 1) * RW - (d2 % 3 - 1);  // source sending d2 to rd
            const int ks = rkey[rs];
            if (ks >= 0 && ks < key_c) b += rcnt[d2 * RW * RH + rs];
          }
        }
      }
      btab[(lk * t.tx + li) * kMoveCodes + d] = b;
    }
    __syncthreads();
    for (int r = r_first; r < k1; r += nwaves / wpr) {
      const int64_t rowc = (int64_t)r * g.nx;
      const int lk = r - k0;
      if (r != r_first) {
        for (int q = lane; q <= cw; q += 64) rowcs[q] = sp.cs[rowc + i0 + q];
        for (int q = lane; q < cw * 10; q += 64) ctr[q] = 0;
      }
      wave_sync();
      const int rb = rowcs[0], re = rowcs[cw];
      const int jb = rb + (int)((int64_t)(re - rb) * part / wpr);
      const int je = rb + (int)((int64_t)(re - rb) * (part + 1) / wpr);
      int clb = 0;  // the cell of the next group's first slot, or a cell before it
      if (part > 0 && jb < je) {
        int lo = 0, hi = cw - 1;  // the cell holding slot jb
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rowcs[mid] <= jb) lo = mid; else hi = mid - 1;
        }
        clb = lo;
        int before[kMoveCodes] = {};
        for (int b0 = rowcs[lo]; b0 < jb; b0 += 64) {
          const int j = b0 + lane;
          const int d = j < jb ? (int)(sp.locode[j] & 15u) : kAbsorbed;
#pragma unroll
          for (int dd = 0; dd < kMoveCodes; ++dd) before[dd] += __popcll(__ballot(d == dd));
        }
        if (lane < kMoveCodes) {
#pragma unroll
          for (int dd = 0; dd < kMoveCodes; ++dd)
            if (lane == dd) ctr[lo * 10 + dd] = before[dd];
        }
        wave_sync();
      }
      // the row's move codes are loaded kGroups groups of 64 at a time (indices clamped into
      // the row), then ranked group by group
      constexpr int kGroups = 8;
      constexpr int kProbe = 4;
      for (int b0 = jb; b0 < je; b0 += 64 * kGroups) {
        uint32_t lcs[kGroups];
#pragma unroll
        for (int q = 0; q < kGroups; ++q) lcs[q] = sp.locode[min(b0 + q * 64 + lane, je - 1)];
#pragma unroll
        for (int q = 0; q < kGroups; ++q) {
          const int base = b0 + q * 64;
          if (base >= je) break;
          const int j = base + lane;
          const bool act = j < je;
          int d = kAbsorbed, cl = 0, loc = 0;
          // the largest cl with rowcs[cl] <= j: the group's slots are consecutive, so it is
          // one of the few cells after clb (independent probes, one LDS round trip); a lane
          // past them searches
          {
            int cnt = 0;
#pragma unroll
            for (int t = 1; t <= kProbe; ++t) cnt += (clb + t < cw && rowcs[min(clb + t, cw)] <= j) ? 1 : 0;
            cl = clb + cnt;
            if (act && cnt == kProbe && cl + 1 < cw && rowcs[cl + 1] <= j) {
              int lo = cl + 1, hi = cw - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rowcs[mid] <= j) lo = mid; else hi = mid - 1;
              }
              cl = lo;
            }
            clb = __builtin_amdgcn_readlane(cl, min(63, je - 1 - base));  // cell of the group's last slot
          }
          if (act) {
            const uint32_t lc = lcs[q];
            d = (int)(lc & 15u);
            loc = (int)(lc >> 4);
          }
          const bool valid = act && d < kMoveCodes;
          // The group's slots are in cell order, so the lanes of one cell are contiguous:
          // [cstart, cend).  A particle's rank within its (cell, code) in this group is the
          // number of lanes of its cell below it with the same code.
          const int prevcl = lane_before(cl);
          const uint64_t heads = __ballot(act && (lane == 0 || prevcl != cl));
          const uint64_t upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
          const int cstart = upto ? 63 - __clzll((long long)upto) : 0;
          const uint64_t above = heads & ~(lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
          const int cend = above ? __ffsll((unsigned long long)above) - 1 : 64;
          const uint64_t cellm = (cend == 64 ? ~0ull : ((1ull << cend) - 1ull)) & ~((1ull << cstart) - 1ull);
          // the lanes with the same move code: one ballot per bit of the code
          uint64_t same = __ballot(valid);
#pragma unroll
          for (int bit = 0; bit < 4; ++bit) {
            const bool on = (d >> bit) & 1;
            const uint64_t m = __ballot(valid && on);
            same &= on ? m : ~m;
          }
          same &= cellm;
          if (valid) {
            const int key = cl * 10 + d;
            const int before = ctr[key];
            const int rank = __popcll(same & lt_mask);
            const int slot = btab[(lk * t.tx + cl) * kMoveCodes + d] + before + rank;
            if (slot >= 0 && slot < total) {
              sp.perm_new[slot] = loc;
            } else {
              atomicOr(a.flags, kFlagSlot);
            }
            // the last lane of each (cell, code) carries the count to the next group
            if ((same >> lane) == 1ull) ctr[key] = before + rank + 1;
          }
          wave_sync();
        }
      }
      wave_sync();
    }
  }
}

// Stable destinations with one thread per cell of an active tile (one species per block,
// wavefronts over runs of 64 cells).  A cell's particles that move with code d go, in the
// next order, to the start of the destination cell, plus the particles arriving there from
// source cells with a smaller key, plus their rank among the cell's earlier slots with code d.
// The thread computes that first slot for each code its cell uses, from the destination's
// next-order start and the counts of the destination's sources (read only for a source that
// holds particles in the current order: the counts of a cell without particles may be left
// from an earlier cycle), then walks its cell's slots in order.  Move codes are canonical
// after the wrap (one code per source and destination pair), so on grids one or two cells
// wide a source listed under two codes has a zero count under the other.  No LDS and no
// cross-lane work: for few particles per cell the row walk's per-tile staging costs more.
// MASKS: the particle kernel wrote each cell's mask of used codes and only the nonzero counts
// (most cells send every particle with one code), so a cell's own codes come from its mask
// and a source's count is read only where the source's mask has the code.
template <bool MASKS>
__device__ __forceinline__ void rank_cells_body(const StepArgs &a, int tile, int species) {
  const GridArgs &g = a.g;
  const TileArgs &t = a.t;
  const SpeciesArgs &sp = a.sp[species];
  if (!sp.active) return;
  const int tzi = tile / t.ntx, txi = tile - tzi * t.ntx;
  const int i0 = txi * t.tx, k0 = tzi * t.tz;
  const int cw = min(i0 + t.tx, g.nx) - i0, ch = min(k0 + t.tz, g.nz) - k0;
  const int ncell = cw * ch;
  const int total = sp.cs_new[g.ncells];
  const bool periodic_x = g.bc_x == PIC_BC_PERIODIC;
  const SmallDiv div_cw(cw);
  // the count a source cell sent with code d2, valid only if the source holds particles now
  // (with masks, read only where its mask has the code: the other counts are not written)
  auto source_count = [&](int sc, int d2) -> int {
    const int sb = sp.cs[sc], se = sp.cs[sc + 1];
    if constexpr (MASKS) {
      const uint32_t m = sp.cmask[sc];
      return (se > sb && ((m >> d2) & 1u)) ? sp.cnt[(int64_t)d2 * g.ncells + sc] : 0;
    } else {
      const int v = sp.cnt[(int64_t)d2 * g.ncells + sc];
      return se > sb ? v : 0;
    }
  };
  for (int e = threadIdx.x; e < ncell; e += blockDim.x) {
    const int lk = div_cw.q(e), li = e - lk * cw;
    const int ci = i0 + li, ck = k0 + lk;
    const int c = ck * g.nx + ci;
    // Issued together: the cell's slot range and used codes, its own next-order start, and
    // what the sources that precede it among the sources of its own cell as a destination
    // (code 4, the particles that stay) sent it: in key order these are the row below and the
    // left neighbour (codes 5 to 8); codes 0 to 3 come before it only through a wrap.
    const int cb = sp.cs[c], ce = sp.cs[c + 1];
    int cur[kMoveCodes];
    if constexpr (MASKS) {
      const uint32_t mc = sp.cmask[c];
#pragma unroll
      for (int d = 0; d < kMoveCodes; ++d) cur[d] = (int)((mc >> d) & 1u);
    } else {
#pragma unroll
      for (int d = 0; d < kMoveCodes; ++d) cur[d] = sp.cnt[(int64_t)d * g.ncells + c];
    }
    int stay = sp.cs_new[c];
    int pv[4], pb[4], pe[4];
    uint32_t pmk[4];
    bool pm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d2 = 5 + q;
      int si = ci - (d2 % 3 - 1), sk = ck - (d2 / 3 - 1);
      bool in = true;
      if (periodic_x) {
        if (si < 0) si += g.nx;
        if (si >= g.nx) si -= g.nx;
      } else {
        in = si >= 0 && si < g.nx;
      }
      if (sk < 0) sk += g.nz;
      const int sc = in ? sk * g.nx + si : c;
      pm[q] = in && sc < c;
      pb[q] = sp.cs[sc];
      pe[q] = sp.cs[sc + 1];
      if constexpr (MASKS) {
        pmk[q] = sp.cmask[sc];
        pv[q] = sc;
      } else {
        pmk[q] = ~0u;
        pv[q] = sp.cnt[(int64_t)d2 * g.ncells + sc];
      }
    }
    if (cb >= ce) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (pm[q] && pe[q] > pb[q] && ((pmk[q] >> (5 + q)) & 1u)) {
        if constexpr (MASKS)
          stay += sp.cnt[(int64_t)(5 + q) * g.ncells + pv[q]];
        else
          stay += pv[q];
      }
    }
    if (ck == g.nz - 1 || (periodic_x && ci == g.nx - 1)) {
#pragma unroll
      for (int d2 = 0; d2 < 4; ++d2) {
        int si = ci - (d2 % 3 - 1), sk = ck - (d2 / 3 - 1);
        bool in = true;
        if (periodic_x) {
          if (si < 0) si += g.nx;
          if (si >= g.nx) si -= g.nx;
        } else {
          in = si >= 0 && si < g.nx;
        }
        if (sk >= g.nz) sk -= g.nz;
        const int sc = sk * g.nx + si;
        if (in && sc < c) stay += source_count(sc, d2);
      }
    }
    // the other codes a cell uses (particles that change cell: few per cycle)
#pragma unroll
    for (int d = 0; d < kMoveCodes; ++d) {
      if (d == 4) {
        cur[d] = stay;
        continue;
      }
      if (cur[d] <= 0) continue;
      // destination (inside the grid: an absorbed particle has its own code)
      int di = ci + (d % 3 - 1), dk = ck + (d / 3 - 1);
      if (di < 0) di += g.nx;
      if (di >= g.nx) di -= g.nx;
      if (dk < 0) dk += g.nz;
      if (dk >= g.nz) dk -= g.nz;
      const int dc = dk * g.nx + di;
      int b = sp.cs_new[dc];
#pragma unroll
      for (int d2 = 0; d2 < kMoveCodes; ++d2) {
        // the source that sends code d2 to the destination
        int si = di - (d2 % 3 - 1), sk = dk - (d2 / 3 - 1);
        bool in = true;
        if (periodic_x) {
          if (si < 0) si += g.nx;
          if (si >= g.nx) si -= g.nx;
        } else {
          in = si >= 0 && si < g.nx;
        }
        if (sk < 0) sk += g.nz;
        if (sk >= g.nz) sk -= g.nz;
        const int sc = sk * g.nx + si;
        if (in && sc < c) b += source_count(sc, d2);
      }
      cur[d] = b;
    }
    // the cell's slots in order, four move codes loaded at a time
    for (int j = cb; j < ce; j += 4) {
      uint32_t lc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) lc[q] = sp.locode[min(j + q, ce - 1)];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (j + q >= ce) break;
        const int d = (int)(lc[q] & 15u);
        int slot = -1;
#pragma unroll
        for (int dd = 0; dd < kMoveCodes; ++dd) {
          if (d == dd) {
            slot = cur[dd];
            cur[dd] = slot + 1;
          }
        }
        if (d < kMoveCodes) {
          if (slot >= 0 && slot < total) {
            sp.perm_new[slot] = (int)(lc[q] >> 4);
          } else {
            atomicOr(a.flags, kFlagSlot);
          }
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_rank_cells(const StepArgs a) {
  const int tile = block_tile(a.t, a.tile_list);
  if (tile < 0) return;
  if (a.count_masks)
    rank_cells_body<true>(a, tile, blockIdx.y);
  else
    rank_cells_body<false>(a, tile, blockIdx.y);
}

__global__ __launch_bounds__(kBlock) void k_rank(const StepArgs a) {
  const int tile = block_tile(a.t, a.tile_list);
  if (tile < 0) return;
  rank_body(a, tile, blockIdx.y);
}

// Flag per tile: does it hold particles of any species in the order given by the cell starts
// (the current order, or the next one when from_next is set).  One thread per tile.
__device__ __forceinline__ void tile_flags_body(const StepArgs &a, int tile, int from_next) {
  const GridArgs &g = a.g;
  const TileArgs &t = a.t;
  if (tile >= t.ntiles) return;
  const int tzi = tile / t.ntx, txi = tile - tzi * t.ntx;
  const int i0 = txi * t.tx, k0 = tzi * t.tz;
  const int i1 = min(i0 + t.tx, g.nx), k1 = min(k0 + t.tz, g.nz);
  int act = 0;
  for (int s = 0; s < a.nsp; ++s) {
    const SpeciesArgs &sp = a.sp[s];
    if (!sp.active) continue;
    const int32_t *cs = from_next ? sp.cs_new : sp.cs;
    for (int r = k0; r < k1; ++r) act |= cs[(int64_t)r * g.nx + i1] > cs[(int64_t)r * g.nx + i0];
  }
  a.tile_active_next[tile] = (uint8_t)act;
}

__global__ __launch_bounds__(kBlock) void k_tile_flags(const StepArgs a, int from_next) {
  tile_flags_body(a, blockIdx.x * blockDim.x + threadIdx.x, from_next);
}

// Ordered list of the flagged tiles, count at [ntiles].  One block; each thread takes a run of
// kPer consecutive flags (loaded together), one block-wide scan per pass places the runs.  The
// list order decides which block takes which tile: in tile order, the blocks of one XCD take
// neighbouring tiles.
__device__ __forceinline__ void tile_compact_body(const StepArgs &a) {
  __shared__ int sh[1024 / 64];
  // A pass takes 64 flags per thread (four 16-byte words; tb is a multiple of 64), counts them
  // with popcounts (flags are 0 or 1), places them with one block scan and writes the active
  // tiles in order.
  constexpr int kPer = 64;
  const int ntiles = a.t.ntiles;
  const uint8_t *flags = a.tile_active_next;
  int carry = 0;
  for (int pbase = 0; pbase < ntiles; pbase += (int)blockDim.x * kPer) {
    const int tb = pbase + (int)threadIdx.x * kPer;
    uint32_t w[kPer / 4];
#pragma unroll
    for (int h = 0; h < kPer / 16; ++h) {
      const int w0 = tb + 16 * h;
      if (w0 + 16 <= ntiles) {
        const uint4 v = *reinterpret_cast<const uint4 *>(flags + w0);
        w[4 * h] = v.x;
        w[4 * h + 1] = v.y;
        w[4 * h + 2] = v.z;
        w[4 * h + 3] = v.w;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t x = 0u;
          for (int b = 0; b < 4; ++b) {
            const int t = w0 + 4 * q + b;
            if (t < ntiles) x |= (uint32_t)flags[t] << (8 * b);
          }
          w[4 * h + q] = x;
        }
      }
    }
    int n = 0;
#pragma unroll
    for (int q = 0; q < kPer / 4; ++q) n += __popc(w[q]);
    int total;
    int pos = carry + block_excl_scan(n, sh, &total);
#pragma unroll
    for (int q = 0; q < kPer / 4; ++q) {
      uint32_t x = w[q];
      while (x) {
        const int bit = __ffs(x) - 1;  // the set bit is bit 0 of byte bit / 8
        a.tile_list_next[pos++] = tb + 4 * q + (bit >> 3);
        x &= x - 1u;
      }
    }
    carry += total;
  }
  if (threadIdx.x == 0) a.tile_list_next[ntiles] = carry;
}

__global__ __launch_bounds__(1024) void k_tile_compact(const StepArgs a) { tile_compact_body(a); }

// ---- two-pass scan of a cycle's sort --------------------------------------------------------
// Pass 1 (k_scan_counts): per block of kScan1Block cells, the exclusive scan of the arrival
// counts within the block (cleared for the next cycle), the block total, and the next order's
// tile flags (a tile is active when particles arrive in one of its cells; the particle kernel
// of the cycle cleared the flags).  Pass 2 (k_scan_apply): every block adds the totals of the
// blocks before it; one extra block compacts the tile flags into the ordered tile list.
__device__ __forceinline__ void scan1_body(const StepArgs &a, int bx, int s) {
  __shared__ int sh[kBlock / 64];
  const SpeciesArgs &sp = a.sp[s];
  if (!sp.active) return;
  const GridArgs &g = a.g;
  const int64_t c0 = (int64_t)bx * kScan1Block + (int64_t)threadIdx.x * kScan1Items;
  int in[kScan1Items];
  if (c0 + kScan1Items <= g.ncells) {
    int4 *p4 = reinterpret_cast<int4 *>(sp.arr + c0);
#pragma unroll
    for (int q = 0; q < kScan1Items / 4; ++q) {
      const int4 v = p4[q];
      in[4 * q] = v.x;
      in[4 * q + 1] = v.y;
      in[4 * q + 2] = v.z;
      in[4 * q + 3] = v.w;
      if (v.x | v.y | v.z | v.w) p4[q] = make_int4(0, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int q = 0; q < kScan1Items; ++q) {
      const int64_t c = c0 + q;
      int v = 0;
      if (c < g.ncells) {
        v = sp.arr[c];
        if (v) sp.arr[c] = 0;
      }
      in[q] = v;
    }
  }
  int sum = 0;
#pragma unroll
  for (int q = 0; q < kScan1Items; ++q) sum += in[q];
  if (sum) {
    int k = (int)(c0 / g.nx), i = (int)(c0 - (int64_t)k * g.nx);
    const SmallDiv div_tx(a.t.tx), div_tz(a.t.tz);
#pragma unroll
    for (int q = 0; q < kScan1Items; ++q) {
      if (in[q] && k < g.nz) a.tile_active_next[div_tz.q(k) * a.t.ntx + div_tx.q(i)] = 1;
      if (++i == g.nx) {
        i = 0;
        ++k;
      }
    }
  }
  int total;
  int run = block_excl_scan(sum, sh, &total);
  if (c0 + kScan1Items <= g.ncells) {
    int4 *o4 = reinterpret_cast<int4 *>(sp.cs_new + c0);
#pragma unroll
    for (int q = 0; q < kScan1Items / 4; ++q) {
      int4 v;
      v.x = run;
      run += in[4 * q];
      v.y = run;
      run += in[4 * q + 1];
      v.z = run;
      run += in[4 * q + 2];
      v.w = run;
      run += in[4 * q + 3];
      o4[q] = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kScan1Items; ++q) {
      const int64_t c = c0 + q;
      if (c < g.ncells) sp.cs_new[c] = run;
      run += in[q];
    }
  }
  if (threadIdx.x == 0) sp.bsum[bx] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_counts(const StepArgs a) {
  scan1_body(a, blockIdx.x, blockIdx.y);
}

// Pass 2 for block bx of species s (bx < n_scan1_blocks).
__device__ __forceinline__ void scan2_body(const StepArgs &a, int bx, int s) {
  __shared__ int sh[kBlock / 64];
  const int nb = a.n_scan1_blocks;
  const SpeciesArgs &sp = a.sp[s];
  if (!sp.active) return;
  // the totals of the blocks before this one (up to 16 per thread on a 2048 x 2048 grid):
  // unrolled so that a thread's loads are issued together
  int part = 0;
#pragma unroll 8
  for (int b = threadIdx.x; b < bx; b += blockDim.x) part += sp.bsum[b];
  int prefix;
  (void)block_excl_scan(part, sh, &prefix);
  const GridArgs &g = a.g;
  const int64_t c0 = (int64_t)bx * kScan1Block + (int64_t)threadIdx.x * kScan1Items;
  if (c0 + kScan1Items <= g.ncells) {
    int4 *o4 = reinterpret_cast<int4 *>(sp.cs_new + c0);
#pragma unroll
    for (int q = 0; q < kScan1Items / 4; ++q) {
      int4 v = o4[q];
      v.x += prefix;
      v.y += prefix;
      v.z += prefix;
      v.w += prefix;
      o4[q] = v;
    }
  } else {
    for (int q = 0; q < kScan1Items; ++q)
      if (c0 + q < g.ncells) sp.cs_new[c0 + q] += prefix;
  }
  if (bx == nb - 1 && threadIdx.x == 0) sp.cs_new[g.ncells] = prefix + sp.bsum[bx];
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const StepArgs a) {
  const int s = blockIdx.y, bx = blockIdx.x;
  if (bx == a.n_scan1_blocks) {
    if (s == 0) tile_compact_body(a);
    return;
  }
  scan2_body(a, bx, s);
}

// ------------------------------------------------------------------------------------------
// Batched cycle: every kernel launched once for all runs of a batch, one block per work item
// of all runs (a run's items are numbered after the previous runs'); the run of an item is
// found in the exclusive prefix of item counts.
// ------------------------------------------------------------------------------------------

// The run owning work item w: the largest r with pre[r] <= w (runs without items are skipped
// because their prefix equals the next run's).
// The run owning work item w: the last r with pre[r] <= w (pre is the exclusive prefix of the
// runs' item counts, non-decreasing, pre[0] = 0; a run without items is skipped).  The 64
// lanes of the wavefront each load one pivot, spaced evenly over the range left, and a ballot
// keeps the interval of the last pivot <= w: one memory round trip per factor 64 of runs
// (the item index is uniform across the wavefront, which must be whole).
__device__ __forceinline__ int find_run(const int32_t *pre, int nruns, int w) {
  const int lane = threadIdx.x & 63;
  int lo = 0, n = nruns;
  while (n > 1) {
    const int step = (n + 63) >> 6;
    const int idx = lo + lane * step;
    const bool le = idx < lo + n && pre[idx] <= w;
    const uint64_t m = __ballot(le);
    const int last = 63 - __clzll((long long)m);  // lane 0 holds pre[lo] <= w
    const int nlo = lo + last * step;
    n = min(step, lo + n - nlo);
    lo = nlo;
  }
  return lo;
}

// The argument tables are read through the constant address space: they do not change during
// a launch, so their fields can be loaded into scalar registers like kernel arguments.
__device__ __forceinline__ const StepArgs &run_step(const BatchArgs &b, int r) {
  const int p = b.par[r];
  const StepArgs __attribute__((address_space(4))) *t =
      (const StepArgs __attribute__((address_space(4))) *)(b.step);
  return *(const StepArgs *)(t + 2 * r + p);
}
__device__ __forceinline__ const FieldArgs &run_field(const BatchArgs &b, int r) {
  const int p = b.par[r];
  const FieldArgs __attribute__((address_space(4))) *t =
      (const FieldArgs __attribute__((address_space(4))) *)(b.field);
  return *(const FieldArgs *)(t + 2 * r + p);
}

// The field kernels' items (node and cell blocks of every run) do not change between
// rebuilds of the batch, so these launch one block per item, with the items of each XCD a
// contiguous band (as in a single run) instead of a persistent loop.
__global__ __launch_bounds__(kBlock) void kb_solve_e(const BatchArgs b, int total) {
  const int w = (int)xcd_band_block(total);
  if (w < 0) return;
  const int r = find_run(b.pre_nodes, b.nruns, w);
  const FieldArgs &fa = run_field(b, r);
  const double tE = (double)b.step_ctr[r] * fa.g.dt;
  solve_e_body(fa, tE, (int64_t)(w - b.pre_nodes[r]) * (kSolveNodes * kBlock) + threadIdx.x, kBlock);
}

__global__ __launch_bounds__(kBlock) void kb_update_h(const BatchArgs b, int total) {
  const int w = (int)xcd_band_block(total);
  if (w < 0) return;
  const int r = find_run(b.pre_cells, b.nruns, w);
  update_h_body(run_field(b, r), (int64_t)(w - b.pre_cells[r]) * (kHCells * kBlock) + threadIdx.x, kBlock);
}

// Work prefixes of the active tiles of every run's current order (one block).
__global__ __launch_bounds__(1024) void kb_prefix(const BatchArgs b) {
  __shared__ int sh[1024 / 64];
  int carry_t = 0, carry_r = 0;
  for (int base = 0; base < b.nruns; base += blockDim.x) {
    const int r = base + threadIdx.x;
    int nt = 0, nr = 0;
    if (r < b.nruns) {
      const StepArgs &sa = run_step(b, r);
      nt = sa.tile_list[sa.t.ntiles];
      nr = nt * sa.nsp;
    }
    int tot_t, tot_r;
    const int off_t = block_excl_scan(nt, sh, &tot_t);
    const int off_r = block_excl_scan(nr, sh, &tot_r);
    if (r < b.nruns) {
      b.pre_tiles[r] = carry_t + off_t;
      b.pre_rank[r] = carry_r + off_r;
    }
    carry_t += tot_t;
    carry_r += tot_r;
  }
  if (threadIdx.x == 0) {
    b.pre_tiles[b.nruns] = carry_t;
    b.pre_rank[b.nruns] = carry_r;
  }
}

// The particle and rank kernels' items (active tiles, and tiles x species) change every cycle;
// they launch one block per item any run could have, and the blocks past the cycle's items
// return at once, so the hardware hands the items, of very unequal cost, to the CUs as they
// free up.  Block b takes item b: consecutive items (the tiles of one run) go to different
// XCDs.  (Contiguous bands of items per XCD, as in a single run, were measured slower: runs
// differ in cost, so the bands load the XCDs unequally.)
__device__ __forceinline__ int batch_item(int total) {
  const int w = (int)blockIdx.x;
  return w < total ? w : -1;
}

template <bool MIXED, bool IDS, bool PW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2 + MIXED, 2 + MIXED)))
void kb_particles(const BatchArgs b) {
  const int w = batch_item(b.pre_tiles[b.nruns]);
  if (w < 0) return;
  const int r = find_run(b.pre_tiles, b.nruns, w);
  const StepArgs &sa = run_step(b, r);
  particles_body<true, MIXED, IDS, PW>(sa, sa.tile_list[w - b.pre_tiles[r]]);
}

// The two-pass scan of every run's sort, as in a single run: pass 1 over (run, species, block
// of cells) items; pass 2 over the same items, then one tile-list compaction item per run.
// The next order's tile flags were cleared by the H update of the cycle.
__global__ __launch_bounds__(kBlock) void kb_scan1(const BatchArgs b) {
  const int total = b.pre_scan[b.nruns];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int r = find_run(b.pre_scan, b.nruns, w);
    const StepArgs &sa = run_step(b, r);
    const int li = w - b.pre_scan[r];
    const int s = li / sa.n_scan1_blocks;
    scan1_body(sa, li - s * sa.n_scan1_blocks, s);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void kb_scan2(const BatchArgs b) {
  const int nscan = b.pre_scan[b.nruns];
  const int total = nscan + b.nruns;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    if (w >= nscan) {
      tile_compact_body(run_step(b, w - nscan));
    } else {
      const int r = find_run(b.pre_scan, b.nruns, w);
      const StepArgs &sa = run_step(b, r);
      const int li = w - b.pre_scan[r];
      const int s = li / sa.n_scan1_blocks;
      scan2_body(sa, li - s * sa.n_scan1_blocks, s);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void kb_rank(const BatchArgs b) {
  const int w = batch_item(b.pre_rank[b.nruns]);
  if (w < 0) return;
  const int r = find_run(b.pre_rank, b.nruns, w);
  const StepArgs &sa = run_step(b, r);
  const int li = w - b.pre_rank[r];
  const int idx = li / sa.nsp;
  if (sa.rank_cells && sa.count_masks)
    rank_cells_body<true>(sa, sa.tile_list[idx], li - idx * sa.nsp);
  else if (sa.rank_cells)
    rank_cells_body<false>(sa, sa.tile_list[idx], li - idx * sa.nsp);
  else
    rank_body(sa, sa.tile_list[idx], li - idx * sa.nsp);
}

// End of a cycle: flip every run's buffer parity and count the cycle.
__global__ void kb_end(const BatchArgs b) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < b.nruns) {
    b.par[r] ^= 1;
    b.step_ctr[r] += 1;
  }
}

__global__ void k_iota(int32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

}  // namespace

size_t particle_lds_bytes(const GridArgs &g, const TileArgs &t, bool mixed, bool pw, bool queues) {
  return TileLds(g.n_planes, t.tx, t.tz, mixed ? (int)sizeof(float) : (int)sizeof(double),
                 queues ? mq_words(pw) : 0).bytes;
}

size_t rank_lds_bytes(const TileArgs &t) {
  const int nw = kBlock / 64;
  const size_t ring = (size_t)(t.tx + 4) * (t.tz + 4);
  return ((size_t)t.tx * t.tz * kMoveCodes + (size_t)nw * ((t.tx + 1) + t.tx * 10) +
          ring * (kMoveCodes + 2)) * sizeof(int);
}

hipError_t launch_field_solve(const FieldArgs &a, hipStream_t s) {
  const int64_t nb_nodes = (a.g.nnodes + kSolveNodes * kBlock - 1) / (kSolveNodes * kBlock);
  const int64_t nb_cells = (a.g.ncells + kHCells * kBlock - 1) / (kHCells * kBlock);
  hipLaunchKernelGGL(k_solve_e, dim3(8u * (unsigned)((nb_nodes + 7) / 8)), dim3(kBlock), 0, s, a, nb_nodes);
  hipLaunchKernelGGL(k_update_h, dim3(8u * (unsigned)((nb_cells + 7) / 8)), dim3(kBlock), 0, s, a, nb_cells);
  return hipGetLastError();
}

// The kernel instantiation for a cycle (push) or a deposit of the current state (no push):
// precision, particle-id copy (push only) and per-particle densities.
template <bool PUSH, bool MIXED>
static void launch_particles_t(const StepArgs &a, bool ids, bool pw, dim3 grid, size_t lds,
                               hipStream_t s) {
  // the pushing kernels without ids in the two-particle chunk form (few particles per lane)
  if constexpr (PUSH) {
    if (!ids && a.chunk2) {
      if (pw)
        hipLaunchKernelGGL((k_particles<PUSH, MIXED, false, true, 2>), grid, dim3(kBlock), lds, s, a);
      else
        hipLaunchKernelGGL((k_particles<PUSH, MIXED, false, false, 2>), grid, dim3(kBlock), lds, s, a);
      return;
    }
  }
  if (PUSH && ids && pw)
    hipLaunchKernelGGL((k_particles<PUSH, MIXED, PUSH, true>), grid, dim3(kBlock), lds, s, a);
  else if (PUSH && ids)
    hipLaunchKernelGGL((k_particles<PUSH, MIXED, PUSH, false>), grid, dim3(kBlock), lds, s, a);
  else if (pw)
    hipLaunchKernelGGL((k_particles<PUSH, MIXED, false, true>), grid, dim3(kBlock), lds, s, a);
  else
    hipLaunchKernelGGL((k_particles<PUSH, MIXED, false, false>), grid, dim3(kBlock), lds, s, a);
}

hipError_t launch_particles(const StepArgs &a, bool push, hipStream_t s) {
  bool ids = false, pw = false;
  for (int q = 0; q < a.nsp; ++q) {
    ids = ids || a.sp[q].dst_id != nullptr;
    pw = pw || (a.sp[q].active && a.sp[q].w_stride != 0);
  }
  // the chunk-of-2 pushing form has no mover queues
  const size_t lds = particle_lds_bytes(a.g, a.t, a.mixed != 0, pw, !(push && a.chunk2 && !ids));
  const dim3 grid(8u * (unsigned)a.t.per_xcd);
  if (a.mixed) {
    if (push) launch_particles_t<true, true>(a, ids, pw, grid, lds, s);
    else launch_particles_t<false, true>(a, ids, pw, grid, lds, s);
  } else {
    if (push) launch_particles_t<true, false>(a, ids, pw, grid, lds, s);
    else launch_particles_t<false, false>(a, ids, pw, grid, lds, s);
  }
  return hipGetLastError();
}

hipError_t launch_sort(const StepArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_counts, dim3((unsigned)a.n_scan1_blocks, (unsigned)a.nsp), dim3(kBlock), 0,
                     s, a);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)a.n_scan1_blocks + 1u, (unsigned)a.nsp), dim3(kBlock),
                     0, s, a);
  const dim3 grid(8u * (unsigned)a.t.per_xcd, (unsigned)a.nsp);
  if (a.rank_cells) {
    // one thread per cell of a tile, at most a full block
    const int cells = a.t.tx * a.t.tz;
    const int rounded = (cells + 63) / 64 * 64;
    const unsigned threads = (unsigned)(rounded < kBlock ? rounded : kBlock);
    hipLaunchKernelGGL(k_rank_cells, grid, dim3(threads), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_rank, grid, dim3(kBlock), rank_lds_bytes(a.t), s, a);
  }
  return hipGetLastError();
}

hipError_t launch_tile_list(const StepArgs &a, bool from_next_order, hipStream_t s) {
  const unsigned ntb = (unsigned)((a.t.ntiles + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_tile_flags, dim3(ntb), dim3(kBlock), 0, s, a, from_next_order ? 1 : 0);
  hipLaunchKernelGGL(k_tile_compact, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

typedef void (*BatchParticlesKernel)(BatchArgs);

// The batched particle kernel instantiation: precision, particle-id copy, per-particle densities.
static BatchParticlesKernel batch_particles_kernel(bool mixed, bool ids, bool pw) {
  if (mixed) {
    if (ids) return pw ? kb_particles<true, true, true> : kb_particles<true, true, false>;
    return pw ? kb_particles<true, false, true> : kb_particles<true, false, false>;
  }
  if (ids) return pw ? kb_particles<false, true, true> : kb_particles<false, true, false>;
  return pw ? kb_particles<false, false, true> : kb_particles<false, false, false>;
}

hipError_t launch_batch_cycle(const BatchArgs &b, const BatchLaunch &l, hipStream_t s) {
  const dim3 blk(kBlock);
  hipLaunchKernelGGL(kb_solve_e, dim3(8u * (unsigned)std::max(1, (l.items_nodes + 7) / 8)), blk, 0,
                     s, b, l.items_nodes);
  hipLaunchKernelGGL(kb_update_h, dim3(8u * (unsigned)std::max(1, (l.items_cells + 7) / 8)), blk, 0,
                     s, b, l.items_cells);
  hipLaunchKernelGGL(kb_prefix, dim3(1), dim3(1024), 0, s, b);
  const dim3 gp((unsigned)l.grid_particles);
  hipLaunchKernelGGL(batch_particles_kernel(l.mixed, l.ids, l.pw), gp, blk, l.lds_particles, s, b);
  // the scans' items are fixed between rebuilds: a block per item (the kernels' loops then run
  // once per block)
  hipLaunchKernelGGL(kb_scan1, dim3((unsigned)std::max(1, l.items_scan)), blk, 0, s, b);
  hipLaunchKernelGGL(kb_scan2, dim3((unsigned)std::max(1, l.items_scan + b.nruns)), blk, 0, s, b);
  hipLaunchKernelGGL(kb_rank, dim3((unsigned)l.grid_rank), blk, l.lds_rank, s, b);
  hipLaunchKernelGGL(kb_end, dim3((unsigned)((b.nruns + kBlock - 1) / kBlock)), blk, 0, s, b);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace pic
