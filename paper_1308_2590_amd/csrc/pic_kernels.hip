// HIP kernels (gfx950) of the implicit 2D3V PIC particle stage.
//
// Field solve (FP64, one thread per node / cell):
//   k_solve_e   Eq. (4) per node: E_new = (I + S)^{-1}[(I - S)E + dt(curl H - dj)] with curl H
//               from the 2x2 neighbouring cells (Sec. 3.3 Step 5); on an absorbing x axis the
//               thread of a boundary node recomputes its inner neighbour and applies the
//               first-order Mur condition to E - E_inc (Steps 3, 4, 6); writes E-bar.
//   k_update_h  Eq. (5) at cell centres with curl E from the 4 corner nodes (Steps 8-9), and
//               clears the moment planes for the next deposit.
// Particles (one block per tile of cells, one wavefront per row of the tile):
//   k_particles gather E-bar (bilinear from the 4 corner nodes) and B (the particle's cell),
//               implicit push (Eq. (2a) solved for the time-centred momentum), position
//               advance, move code, then deposit of S-hat, delta-j and density (Step 1,
//               Eq. (3)) at the new position into LDS accumulators covering the tile plus a
//               halo, folded once per tile into the FP64 moment planes with global atomics.
// Sort (stable by cell, removed particles dropped):
//   k_scan_counts / k_scan_blocks / k_scan_finish  particles arriving in each cell from its
//               3x3 neighbourhood, exclusive scan -> next cell start offsets;
//   k_rank      stable destination of every particle: cell start + particles arriving from
//               source cells with a smaller key + rank within (source cell, move code),
//               written as the next cycle's slot -> location permutation.
// Positions never move more than one cell per cycle because dt <= min(dx, dz) and |v| < c,
// which is what keeps the sort a 3x3 neighbourhood redistribution.
//
// The file is compiled with -ffp-contract=off: the mover performs the same IEEE-754
// operations in the same order as a plain scalar implementation, so particles pushed in the
// same fields land bit-for-bit in the same cell.
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

// The tile handled by this block: blocks are dealt round-robin to the 8 XCDs, so hand each
// XCD a contiguous band of tiles (neighbouring tiles share halo nodes and field cache lines).
__device__ __forceinline__ int block_tile(const TileArgs &t) {
  int b = blockIdx.x;
  return (b & 7) * t.per_xcd + (b >> 3);
}

// Implicit response of a particle: R = (I + [b]x + b b^T) / (1 + b.b) with b = (beta/gamma) B,
// [b]x a = a x b.  It solves u-bar = a + u-bar x b, the time-centred Eq. (2a).
__device__ __forceinline__ void response(double beta, double g, double B0, double B1, double B2,
                                         double R[9]) {
  double bg = beta / g;
  double bx = bg * B0, by = bg * B1, bz = bg * B2;
  double inv = 1.0 / (1.0 + bx * bx + by * by + bz * bz);
  R[0] = (1.0 + bx * bx) * inv;
  R[1] = (bz + bx * by) * inv;
  R[2] = (-by + bx * bz) * inv;
  R[3] = (-bz + by * bx) * inv;
  R[4] = (1.0 + by * by) * inv;
  R[5] = (bx + by * bz) * inv;
  R[6] = (by + bz * bx) * inv;
  R[7] = (-bx + bz * by) * inv;
  R[8] = (1.0 + bz * bz) * inv;
}

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

// Eq. (4) at the node (i, k), i an interior column.
__device__ void solve_node(const FieldArgs &a, int i, int k, double out[3]) {
  const GridArgs &g = a.g;
  const int nx = g.nx, nz = g.nz;
  const int64_t nn = g.nnodes, nc = g.ncells;
  int iR = wrap1(i, nx), iL = wrap1(i - 1, nx);
  int kU = wrap1(k, nz), kD = wrap1(k - 1, nz);
  int64_t cUR = (int64_t)kU * nx + iR, cUL = (int64_t)kU * nx + iL;
  int64_t cDR = (int64_t)kD * nx + iR, cDL = (int64_t)kD * nx + iL;
  const double *Hx = a.H, *Hy = a.H + nc, *Hz = a.H + 2 * nc;
  double dHx_dz = ((Hx[cUR] + Hx[cUL]) - (Hx[cDR] + Hx[cDL])) / (2.0 * g.dz);
  double dHy_dz = ((Hy[cUR] + Hy[cUL]) - (Hy[cDR] + Hy[cDL])) / (2.0 * g.dz);
  double dHy_dx = ((Hy[cUR] + Hy[cDR]) - (Hy[cUL] + Hy[cDL])) / (2.0 * g.dx);
  double dHz_dx = ((Hz[cUR] + Hz[cDR]) - (Hz[cUL] + Hz[cDL])) / (2.0 * g.dx);
  double curl[3] = {-dHy_dz, dHx_dz - dHz_dx, dHy_dx};
  int64_t n = (int64_t)k * g.nxn + i;
  double S[9], e[3], rhs[3];
#pragma unroll
  for (int r = 0; r < 9; ++r) S[r] = a.M[r * nn + n];
#pragma unroll
  for (int r = 0; r < 3; ++r) e[r] = a.E[r * nn + n];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double se = S[3 * r] * e[0] + S[3 * r + 1] * e[1] + S[3 * r + 2] * e[2];
    rhs[r] = (e[r] - se) + g.dt * (curl[r] - a.M[(9 + r) * nn + n]);
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
  out[0] = (c00 * rhs[0] + c10 * rhs[1] + c20 * rhs[2]) / det;
  out[1] = (c01 * rhs[0] + c11 * rhs[1] + c21 * rhs[2]) / det;
  out[2] = (c02 * rhs[0] + c12 * rhs[1] + c22 * rhs[2]) / det;
}

__global__ __launch_bounds__(kBlock) void k_solve_e(const FieldArgs a) {
  const GridArgs &g = a.g;
  int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nnodes) return;
  int k = (int)(n / g.nxn), i = (int)(n - (int64_t)k * g.nxn);
  const int64_t nn = g.nnodes;
  double en[3];
  if (g.bc_x == PIC_BC_ABSORBING && (i == 0 || i == g.nx)) {
    // Mur boundary (Step 3), the x = 0 column taking the source of Step 4 on E_y.
    const int inner = (i == 0) ? 1 : g.nx - 1;
    double ein[3];
    if (g.nx >= 2) {
      solve_node(a, inner, k, ein);
    } else {
      for (int r = 0; r < 3; ++r) ein[r] = a.E[r * nn + (int64_t)k * g.nxn + inner];
    }
    const double kappa = (g.dt - g.dx) / (g.dt + g.dx);
    const double t0 = a.t, t1 = a.t + g.dt;
    const double z = (double)k * g.dz;
    int64_t nb = (int64_t)k * g.nxn + i, nin = (int64_t)k * g.nxn + inner;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double Eo_b = a.E[r * nn + nb], Eo_in = a.E[r * nn + nin];
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
  } else {
    solve_node(a, i, k, en);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double eo = a.E[r * nn + n];
    a.E_new[r * nn + n] = en[r];
    a.Ebar[r * nn + n] = 0.5 * (eo + en[r]);
  }
}

__global__ __launch_bounds__(kBlock) void k_update_h(const FieldArgs a) {
  const GridArgs &g = a.g;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncells) return;
  const int nx = g.nx, nz = g.nz, nxn = g.nxn;
  int k = (int)(c / nx), i = (int)(c - (int64_t)k * nx);
  int i1 = (g.bc_x == PIC_BC_PERIODIC) ? wrap1(i + 1, nx) : i + 1;
  int k1 = wrap1(k + 1, nz);
  const int64_t nn = g.nnodes, nc = g.ncells;
  int64_t na = (int64_t)k * nxn + i, nb = (int64_t)k * nxn + i1;
  int64_t ncn = (int64_t)k1 * nxn + i, nd = (int64_t)k1 * nxn + i1;
  const double *Ex = a.E_new, *Ey = a.E_new + nn, *Ez = a.E_new + 2 * nn;
  double dEx_dz = ((Ex[ncn] + Ex[nd]) - (Ex[na] + Ex[nb])) / (2.0 * g.dz);
  double dEy_dz = ((Ey[ncn] + Ey[nd]) - (Ey[na] + Ey[nb])) / (2.0 * g.dz);
  double dEy_dx = ((Ey[nb] + Ey[nd]) - (Ey[na] + Ey[ncn])) / (2.0 * g.dx);
  double dEz_dx = ((Ez[nb] + Ez[nd]) - (Ez[na] + Ez[ncn])) / (2.0 * g.dx);
  a.H_new[c] = a.H[c] - g.dt * (-dEy_dz);
  a.H_new[nc + c] = a.H[nc + c] - g.dt * (dEx_dz - dEz_dx);
  a.H_new[2 * nc + c] = a.H[2 * nc + c] - g.dt * dEy_dx;
  if (a.M_clear) {
    // Node (i, k) belongs to cell (i, k); the extra x column of an absorbing axis to i = nx-1.
    for (int p = 0; p < g.n_planes; ++p) a.M_clear[p * nn + na] = 0.0;
    if (g.bc_x == PIC_BC_ABSORBING && i == nx - 1)
      for (int p = 0; p < g.n_planes; ++p) a.M_clear[p * nn + na + 1] = 0.0;
  }
}

// ------------------------------------------------------------------------------------------
// Particles
// ------------------------------------------------------------------------------------------

// Add the 12 implicit moments and the density of one particle, spread by the four linear
// weights of its cell, to the tile's LDS accumulators (corner (lx, lz) is the cell's lower
// left node in tile-local coordinates).
__device__ __forceinline__ void deposit_lds(double *acc, int plane, int LW, int lx, int lz,
                                            double fx, double fz, const double val[12],
                                            int dens_plane, double w) {
  const double W[4] = {(1.0 - fx) * (1.0 - fz), fx * (1.0 - fz), (1.0 - fx) * fz, fx * fz};
  const int b = lz * LW + lx;
  const int o[4] = {b, b + 1, b + LW, b + LW + 1};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int p = 0; p < 12; ++p) atomicAdd(&acc[p * plane + o[c]], W[c] * val[p]);
    atomicAdd(&acc[dens_plane * plane + o[c]], W[c] * w);
  }
}

// The 12 moment values of one particle with momentum u, Lorentz factor g and field B:
// S-hat = w q^2 dt^2 R / (4 m g), delta-j = (w q / g) R u (the split of Eq. (3)).
__device__ __forceinline__ void moment_values(const SpeciesArgs &sp, double g, double u0,
                                              double u1, double u2, double B0, double B1,
                                              double B2, double val[12]) {
  double R[9];
  response(sp.beta, g, B0, B1, B2, R);
  double kS = sp.cS / g, kJ = sp.kJ / g;
#pragma unroll
  for (int r = 0; r < 9; ++r) val[r] = kS * R[r];
#pragma unroll
  for (int r = 0; r < 3; ++r) val[9 + r] = kJ * (R[3 * r] * u0 + R[3 * r + 1] * u1 + R[3 * r + 2] * u2);
}

template <bool PUSH>
__global__ __launch_bounds__(kBlock) void k_particles(const StepArgs a) {
  const GridArgs &g = a.g;
  const TileArgs &t = a.t;
  const int tile = block_tile(t);
  if (tile >= t.ntiles) return;
  const int tzi = tile / t.ntx, txi = tile - tzi * t.ntx;
  const int i0 = txi * t.tx, k0 = tzi * t.tz;
  const int i1 = min(i0 + t.tx, g.nx), k1 = min(k0 + t.tz, g.nz);
  const int LW = t.tx + 3, LH = t.tz + 3, plane = LW * LH;
  const int ntc = t.tx * t.tz;

  extern __shared__ double lds[];
  double *acc = lds;
  int *cntL = reinterpret_cast<int *>(lds + (size_t)g.n_planes * plane);

  for (int e = threadIdx.x; e < g.n_planes * plane; e += blockDim.x) acc[e] = 0.0;
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
  const int64_t nn = g.nnodes, nc = g.ncells;

  for (int s = 0; s < a.nsp; ++s) {
    const SpeciesArgs &sp = a.sp[s];
    if (!sp.active) continue;
    if (PUSH) {
      for (int e = threadIdx.x; e < ntc * 10; e += blockDim.x) cntL[e] = 0;
      __syncthreads();
    }
    for (int r = k0 + wave; r < k1; r += nwaves) {
      const int64_t rowc = (int64_t)r * g.nx;
      const int jb = sp.cs[rowc + i0], je = sp.cs[rowc + i1];
      for (int j = jb + lane; j < je; j += 64) {
        const int p = sp.perm[j];
        const double x = sp.src[0][p], z = sp.src[1][p];
        const double u0 = sp.src[2][p], u1 = sp.src[3][p], u2 = sp.src[4][p];
        const int i = (int)floor(x), k = (int)floor(z);
        if (k != r || i < i0 || i >= i1) {
          atomicOr(a.flags, kFlagOrder);
          if (PUSH) sp.code[j] = kAbsorbed;
          continue;
        }
        const double fx = x - (double)i, fz = z - (double)k;
        const int64_t c = (int64_t)k * g.nx + i;
        const double B0 = a.Hold[c], B1 = a.Hold[nc + c], B2 = a.Hold[2 * nc + c];
        const double gam = sqrt(1.0 + u0 * u0 + u1 * u1 + u2 * u2);
        const int lx = i - i0 + 1, lz = k - k0 + 1;
        if (!PUSH) {
          double val[12];
          moment_values(sp, gam, u0, u1, u2, B0, B1, B2, val);
          deposit_lds(acc, plane, LW, lx, lz, fx, fz, val, 12 + s, sp.w);
          continue;
        }
        // gather E-bar at x^{n+1/2} from the 4 corner nodes (linear weights)
        const int in1 = (g.bc_x == PIC_BC_PERIODIC) ? wrap1(i + 1, g.nx) : i + 1;
        const int kn1 = wrap1(k + 1, g.nz);
        const int64_t n00 = (int64_t)k * g.nxn + i, n10 = (int64_t)k * g.nxn + in1;
        const int64_t n01 = (int64_t)kn1 * g.nxn + i, n11 = (int64_t)kn1 * g.nxn + in1;
        const double W0 = (1.0 - fx) * (1.0 - fz), W1 = fx * (1.0 - fz);
        const double W2 = (1.0 - fx) * fz, W3 = fx * fz;
        double Ep[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double *f = a.Ebar + q * nn;
          Ep[q] = W0 * f[n00] + W1 * f[n10] + W2 * f[n01] + W3 * f[n11];
        }
        // implicit push: u-bar = R (u + beta E), u' = 2 u-bar - u
        double R[9];
        response(sp.beta, gam, B0, B1, B2, R);
        const double av0 = u0 + sp.beta * Ep[0], av1 = u1 + sp.beta * Ep[1], av2 = u2 + sp.beta * Ep[2];
        const double n0 = 2.0 * (R[0] * av0 + R[1] * av1 + R[2] * av2) - u0;
        const double n1 = 2.0 * (R[3] * av0 + R[4] * av1 + R[5] * av2) - u1;
        const double n2 = 2.0 * (R[6] * av0 + R[7] * av1 + R[8] * av2) - u2;
        const double g1 = sqrt(1.0 + n0 * n0 + n1 * n1 + n2 * n2);
        double xn = x + g.cx * (n0 / g1);
        double zn = z + g.cz * (n2 / g1);
        bool alive = true;
        if (g.bc_x == PIC_BC_PERIODIC) {
          if (xn < 0.0) xn += (double)g.nx;
          if (xn >= (double)g.nx) xn -= (double)g.nx;
        } else if (xn < 0.0 || xn >= (double)g.nx) {
          alive = false;
        }
        if (zn < 0.0) zn += (double)g.nz;
        if (zn >= (double)g.nz) zn -= (double)g.nz;
        if (!(isfinite(g1) && isfinite(xn) && isfinite(zn))) {
          atomicOr(a.flags, kFlagNonFinite);
          alive = false;
        }
        uint8_t code = kAbsorbed;
        int i2 = 0, k2 = 0, di = 0, dk = 0;
        if (alive) {
          i2 = (int)floor(xn);
          k2 = (int)floor(zn);
          di = i2 - i;
          dk = k2 - k;
          if (di > 1) di -= g.nx;
          if (di < -1) di += g.nx;
          if (dk > 1) dk -= g.nz;
          if (dk < -1) dk += g.nz;
          if (di < -1 || di > 1 || dk < -1 || dk > 1) {
            atomicOr(a.flags, kFlagJump);
            alive = false;
          } else {
            code = (uint8_t)((dk + 1) * 3 + (di + 1));
          }
        }
        sp.dst[0][j] = xn;
        sp.dst[1][j] = zn;
        sp.dst[2][j] = n0;
        sp.dst[3][j] = n1;
        sp.dst[4][j] = n2;
        if (sp.dst_id) sp.dst_id[j] = sp.src_id[p];
        sp.code[j] = code;
        atomicAdd(&cntL[((k - k0) * t.tx + (i - i0)) * 10 + code], 1);
        if (alive) {
          // deposit M^{n+3/2} at x^{n+3/2} with u^{n+1}, gamma(u^{n+1}) and H^{n+3/2} there
          const int64_t c2 = (int64_t)k2 * g.nx + i2;
          double val[12];
          moment_values(sp, g1, n0, n1, n2, a.Hnew[c2], a.Hnew[nc + c2], a.Hnew[2 * nc + c2], val);
          deposit_lds(acc, plane, LW, lx + di, lz + dk, xn - (double)i2, zn - (double)k2, val,
                      12 + s, sp.w);
        }
      }
    }
    if (PUSH) {
      __syncthreads();
      const int cw = i1 - i0;
      for (int e = threadIdx.x; e < (k1 - k0) * cw * kMoveCodes; e += blockDim.x) {
        const int d = e / ((k1 - k0) * cw);
        const int rem = e - d * ((k1 - k0) * cw);
        const int lk = rem / cw, li = rem - lk * cw;
        sp.cnt[(int64_t)d * nc + (int64_t)(k0 + lk) * g.nx + (i0 + li)] = cntL[(lk * t.tx + li) * 10 + d];
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // fold the tile's accumulators into the global moment planes
  for (int e = threadIdx.x; e < g.n_planes * plane; e += blockDim.x) {
    const double v = acc[e];
    if (v == 0.0) continue;
    const int p = e / plane, idx = e - p * plane;
    const int lz = idx / LW, lx = idx - lz * LW;
    int gx = i0 - 1 + lx, gz = k0 - 1 + lz;
    if (g.bc_x == PIC_BC_PERIODIC) {
      gx = wrap_any(gx, g.nx);
    } else if (gx < 0 || gx > g.nx) {
      continue;
    }
    gz = wrap_any(gz, g.nz);
    unsafeAtomicAdd(&a.M[(int64_t)p * nn + (int64_t)gz * g.nxn + gx], v);
  }
}

// ------------------------------------------------------------------------------------------
// Sort
// ------------------------------------------------------------------------------------------

// Source cell of destination cell (iK, kK) for move code d, or -1 if it does not exist.
__device__ __forceinline__ int64_t source_cell(const GridArgs &g, int iK, int kK, int d) {
  const int di = d % 3 - 1, dk = d / 3 - 1;
  int is = iK - di, ks = kK - dk;
  if (g.bc_x == PIC_BC_PERIODIC) {
    is = wrap_any(is, g.nx);
  } else if (is < 0 || is >= g.nx) {
    return -1;
  }
  ks = wrap_any(ks, g.nz);
  return (int64_t)ks * g.nx + is;
}

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

__global__ __launch_bounds__(kBlock) void k_scan_counts(const StepArgs a) {
  __shared__ int sh[kBlock / 64];
  const SpeciesArgs &sp = a.sp[blockIdx.y];
  if (!sp.active) return;
  const GridArgs &g = a.g;
  const int64_t c0 = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int in[kScanItems];
  int sum = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t c = c0 + q;
    int v = 0;
    if (c < g.ncells) {
      const int kK = (int)(c / g.nx), iK = (int)(c - (int64_t)kK * g.nx);
      for (int d = 0; d < kMoveCodes; ++d) {
        const int64_t src = source_cell(g, iK, kK, d);
        if (src >= 0) v += sp.cnt[(int64_t)d * g.ncells + src];
      }
    }
    in[q] = v;
    sum += v;
  }
  int total;
  int off = block_excl_scan(sum, sh, &total);
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int64_t c = c0 + q;
    if (c < g.ncells) sp.cs_new[c] = off;
    off += in[q];
  }
  if (threadIdx.x == 0) sp.bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(const StepArgs a, int nblocks) {
  __shared__ int sh[1024 / 64];
  const SpeciesArgs &sp = a.sp[blockIdx.x];
  if (!sp.active) return;
  int carry = 0;
  for (int base = 0; base < nblocks; base += blockDim.x) {
    const int b = base + threadIdx.x;
    const int v = b < nblocks ? sp.bsum[b] : 0;
    int total;
    const int off = block_excl_scan(v, sh, &total);
    if (b < nblocks) sp.bsum[b] = carry + off;
    carry += total;
  }
  if (threadIdx.x == 0) sp.cs_new[a.g.ncells] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_finish(const StepArgs a) {
  const SpeciesArgs &sp = a.sp[blockIdx.y];
  if (!sp.active) return;
  const int add = sp.bsum[blockIdx.x];
  const int64_t c0 = (int64_t)blockIdx.x * kScanBlock;
  for (int q = threadIdx.x; q < kScanBlock; q += blockDim.x) {
    const int64_t c = c0 + q;
    if (c < a.g.ncells) sp.cs_new[c] += add;
  }
}

// First slot, in the next order, of the particles moving from cell c with move code d:
// start of the destination cell plus everything arriving there from source cells that come
// earlier in the current (cell-sorted) order.
__device__ int64_t dest_base(const GridArgs &g, const SpeciesArgs &sp, int ic, int kc, int d) {
  const int di = d % 3 - 1, dk = d / 3 - 1;
  int iK = ic + di, kK = wrap_any(kc + dk, g.nz);
  if (g.bc_x == PIC_BC_PERIODIC) iK = wrap_any(iK, g.nx);
  const int64_t K = (int64_t)kK * g.nx + iK;
  const int64_t key_c = (int64_t)kc * g.nx + ic;
  int64_t base = sp.cs_new[K];
  for (int d2 = 0; d2 < kMoveCodes; ++d2) {
    const int64_t src = source_cell(g, iK, kK, d2);
    if (src >= 0 && src < key_c) base += sp.cnt[(int64_t)d2 * g.ncells + src];
  }
  return base;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(kBlock) void k_rank(const StepArgs a) {
  const GridArgs &g = a.g;
  const TileArgs &t = a.t;
  const int tile = block_tile(t);
  if (tile >= t.ntiles) return;
  const int tzi = tile / t.ntx, txi = tile - tzi * t.ntx;
  const int i0 = txi * t.tx, k0 = tzi * t.tz;
  const int i1 = min(i0 + t.tx, g.nx), k1 = min(k0 + t.tz, g.nz);
  const int cw = i1 - i0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
  extern __shared__ int ldsi[];
  int *rowcs = ldsi + wave * (t.tx + 1);                           // [tx + 1] per wave
  int *ctr = ldsi + nwaves * (t.tx + 1) + wave * (t.tx * 10);      // [tx][10] per wave
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  for (int s = 0; s < a.nsp; ++s) {
    const SpeciesArgs &sp = a.sp[s];
    if (!sp.active) continue;
    const int total = sp.cs_new[g.ncells];
    for (int r = k0 + wave; r < k1; r += nwaves) {
      const int64_t rowc = (int64_t)r * g.nx;
      for (int q = lane; q <= cw; q += 64) rowcs[q] = sp.cs[rowc + i0 + q];
      for (int q = lane; q < cw * 10; q += 64) ctr[q] = 0;
      wave_sync();
      const int jb = rowcs[0], je = rowcs[cw];
      for (int base = jb; base < je; base += 64) {
        const int j = base + lane;
        const bool act = j < je;
        int d = kAbsorbed, cl = 0;
        if (act) {
          d = sp.code[j];
          int lo = 0, hi = cw - 1;  // largest cl with rowcs[cl] <= j
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rowcs[mid] <= j) lo = mid; else hi = mid - 1;
          }
          cl = lo;
        }
        const bool valid = act && d < kMoveCodes;
        const int key = cl * 10 + d;
        uint64_t todo = __ballot(valid);
        while (todo) {
          const int leader = __ffsll((unsigned long long)todo) - 1;
          const int lkey = __shfl(key, leader, 64);
          const uint64_t grp = __ballot(valid && key == lkey);
          const int lcl = lkey / 10, ld = lkey - lcl * 10;
          const int before = ctr[lkey];
          const int64_t b0 = dest_base(g, sp, i0 + lcl, r, ld) + before;
          if ((grp >> lane) & 1ull) {
            const int64_t slot = b0 + __popcll(grp & lt_mask);
            if (slot >= 0 && slot < total) {
              sp.perm_new[slot] = j;
            } else {
              atomicOr(a.flags, kFlagSlot);
            }
          }
          wave_sync();
          if (lane == leader) ctr[lkey] = before + __popcll(grp);
          wave_sync();
          todo &= ~grp;
        }
      }
      wave_sync();
    }
  }
}

__global__ void k_iota(int32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

}  // namespace

size_t particle_lds_bytes(const GridArgs &g, const TileArgs &t) {
  return (size_t)g.n_planes * (t.tx + 3) * (t.tz + 3) * sizeof(double) +
         (size_t)t.tx * t.tz * 10 * sizeof(int);
}

size_t rank_lds_bytes(const TileArgs &t) {
  const int nw = kBlock / 64;
  return (size_t)nw * ((t.tx + 1) + t.tx * 10) * sizeof(int);
}

hipError_t launch_field_solve(const FieldArgs &a, hipStream_t s) {
  const int64_t nb_nodes = (a.g.nnodes + kBlock - 1) / kBlock;
  const int64_t nb_cells = (a.g.ncells + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_solve_e, dim3((unsigned)nb_nodes), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_update_h, dim3((unsigned)nb_cells), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_particles(const StepArgs &a, bool push, hipStream_t s) {
  const size_t lds = particle_lds_bytes(a.g, a.t);
  const dim3 grid(8u * (unsigned)a.t.per_xcd);
  if (push)
    hipLaunchKernelGGL(k_particles<true>, grid, dim3(kBlock), lds, s, a);
  else
    hipLaunchKernelGGL(k_particles<false>, grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_sort(const StepArgs &a, int32_t n_scan_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_counts, dim3((unsigned)n_scan_blocks, (unsigned)a.nsp), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)a.nsp), dim3(1024), 0, s, a, n_scan_blocks);
  hipLaunchKernelGGL(k_scan_finish, dim3((unsigned)n_scan_blocks, (unsigned)a.nsp), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_rank, dim3(8u * (unsigned)a.t.per_xcd), dim3(kBlock), rank_lds_bytes(a.t), s, a);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace pic
