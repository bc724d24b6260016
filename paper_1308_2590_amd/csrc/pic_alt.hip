// HIP kernels (gfx950) for the mover options and the energy diagnostic.
//
//   k_particles_alt  the particle stage of a cycle with a mover option (FP64): one thread per
//                    sorted slot; gather E-bar (bilinear from the 4 corner nodes), B at the
//                    particle (its cell's H, or bilinear from the 4 surrounding cell centres),
//                    gamma-bar (gamma(u^n), or gamma(u^n + beta E^n) with E^n interpolated at
//                    the particle), the implicit push of Eq. (2), position advance and move
//                    code, then the deposit of S-hat, delta-j and density (Step 1, Eq. (3)) at
//                    the new position with the same options, into the global moment planes with
//                    FP64 atomics, each first summed over the lanes of a wavefront that
//                    deposit into the same cell.  It writes the move codes, counts and arrivals
//                    the cycle's sort reads, exactly as the tile kernel does.  Without push it
//                    deposits the current state.
//   k_energy         field energy (1/2)(sum |E|^2 over nodes + sum |H|^2 over cells) dx dz and
//                    kinetic energy sum w m (gamma - 1) dx dz per species.
//
// The options are two readings of what the paper leaves open (the Lorentz factor inside the
// linearised mover and B at a particle when H is cell-centred).  Per-particle B makes S-hat
// differ from particle to particle, so these kernels deposit each particle's expanded moments
// instead of per-cell sums; they trade speed for the choice.

#include <mutex>

#include "pic_internal.h"

namespace pic {
namespace {

constexpr uint32_t kFlagNonFiniteA = PIC_FLAG_NONFINITE;
constexpr uint32_t kFlagJumpA = PIC_FLAG_JUMP;
constexpr uint32_t kFlagOrderA = PIC_FLAG_ORDER;

__device__ __forceinline__ int wrapc(int i, int n) {
  if (i < 0) return i + n;
  if (i >= n) return i - n;
  return i;
}

// The four corner nodes of cell (i, k) (order (i,k), (i+1,k), (i,k+1), (i+1,k+1)) and the
// linear weights of offsets (fx, fz).
__device__ __forceinline__ void corners(const GridArgs &g, int i, int k, double fx, double fz,
                                        int64_t node[4], double W[4]) {
  const int i1 = g.bc_x == PIC_BC_PERIODIC ? wrapc(i + 1, g.nx) : i + 1;
  const int k1 = wrapc(k + 1, g.nz);
  node[0] = (int64_t)k * g.nxn + i;
  node[1] = (int64_t)k * g.nxn + i1;
  node[2] = (int64_t)k1 * g.nxn + i;
  node[3] = (int64_t)k1 * g.nxn + i1;
  W[0] = (1.0 - fx) * (1.0 - fz);
  W[1] = fx * (1.0 - fz);
  W[2] = (1.0 - fx) * fz;
  W[3] = fx * fz;
}

__device__ __forceinline__ double at_nodes(const double *f, const int64_t node[4], const double W[4]) {
  return W[0] * f[node[0]] + W[1] * f[node[1]] + W[2] * f[node[2]] + W[3] * f[node[3]];
}

// B at position (x, z) in cell (i, k) from the cell-centred planes H.
__device__ void b_at(const GridArgs &g, const double *H, int mover, double x, double z, int i,
                     int k, double B[3]) {
  const int64_t nc = g.ncells;
  if (!(mover & PIC_MOVER_B_BILINEAR)) {
    const int64_t c = (int64_t)k * g.nx + i;
    for (int r = 0; r < 3; ++r) B[r] = H[r * nc + c];
    return;
  }
  const double sx = x - 0.5, sz = z - 0.5;
  const int ic = (int)floor(sx), kc = (int)floor(sz);
  const double gx = sx - (double)ic, gz = sz - (double)kc;
  int ci[2], ck[2];
  for (int t = 0; t < 2; ++t) {
    const int ii = ic + t;
    ci[t] = g.bc_x == PIC_BC_PERIODIC ? wrapc(ii, g.nx) : min(max(ii, 0), g.nx - 1);
    ck[t] = wrapc(kc + t, g.nz);
  }
  const double Wc[4] = {(1.0 - gx) * (1.0 - gz), gx * (1.0 - gz), (1.0 - gx) * gz, gx * gz};
  const int64_t c4[4] = {(int64_t)ck[0] * g.nx + ci[0], (int64_t)ck[0] * g.nx + ci[1],
                         (int64_t)ck[1] * g.nx + ci[0], (int64_t)ck[1] * g.nx + ci[1]};
  for (int r = 0; r < 3; ++r)
    B[r] = Wc[0] * H[r * nc + c4[0]] + Wc[1] * H[r * nc + c4[1]] + Wc[2] * H[r * nc + c4[2]] +
           Wc[3] * H[r * nc + c4[3]];
}

// gamma-bar for momentum u at a particle with corner nodes/weights: gamma(u), or with the
// predictor gamma(u + beta E) for E interpolated from the planes En.
__device__ double gamma_bar(const GridArgs &g, const double *En, int mover, double beta,
                            const double u[3], const int64_t node[4], const double W[4]) {
  if (!(mover & PIC_MOVER_GAMMA_PREDICT)) return sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double um[3];
  for (int r = 0; r < 3; ++r) um[r] = u[r] + beta * at_nodes(En + r * g.nnodes, node, W);
  return sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
}

// One particle's S-hat (9), delta-j (3) and density: with s = beta / gamma-bar and
// D = 1 + s^2 B.B, S-hat = (w q^2 dt^2 / (4 m gamma-bar D)) (I + s [B]x + s^2 B B^T) and
// delta-j = (w q / (gamma-bar D)) (u + s u x B + s^2 (B.u) B), w the particle's density (wp
// when the species carries one per particle).
__device__ void moments13(const SpeciesArgs &sp, double gam, const double u[3], const double B[3],
                          double wp, double v[13]) {
  const double sg = sp.beta / gam;
  const double inv = 1.0 / (1.0 + sg * sg * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]));
  const double cS = sp.w_stride ? sp.cS1 * wp : sp.cS;
  const double kJ = sp.w_stride ? sp.kJ1 * wp : sp.kJ;
  const double a0 = cS / gam * inv, a1 = a0 * sg, a2 = a1 * sg;
  const double kk = kJ / gam * inv;
  const double bu = B[0] * u[0] + B[1] * u[1] + B[2] * u[2];
  v[0] = a2 * B[0] * B[0] + a0;
  v[1] = a2 * B[0] * B[1] + a1 * B[2];
  v[2] = a2 * B[0] * B[2] - a1 * B[1];
  v[3] = a2 * B[1] * B[0] - a1 * B[2];
  v[4] = a2 * B[1] * B[1] + a0;
  v[5] = a2 * B[1] * B[2] + a1 * B[0];
  v[6] = a2 * B[2] * B[0] + a1 * B[1];
  v[7] = a2 * B[2] * B[1] - a1 * B[0];
  v[8] = a2 * B[2] * B[2] + a0;
  v[9] = kk * (u[0] + sg * (u[1] * B[2] - u[2] * B[1]) + sg * sg * bu * B[0]);
  v[10] = kk * (u[1] + sg * (u[2] * B[0] - u[0] * B[2]) + sg * sg * bu * B[1]);
  v[11] = kk * (u[2] + sg * (u[0] * B[1] - u[1] * B[0]) + sg * sg * bu * B[2]);
  v[12] = sp.w_stride ? wp : sp.w;
}

// The threads of a wavefront follow the cell-sorted order, so lanes that add to the same
// addresses (one cell's nodes, counter or arrival count) are neighbours.  Their values are
// summed over each run of equal keys (a segmented reduction towards the run's first lane) and
// the first lane issues one global atomic per value: same-address atomics from the lanes of
// one cell would otherwise be serialised.  All 64 lanes take part; a lane without a value has
// a key of its own (negative).
struct Seg {
  int lane, seg_end, steps;
  bool head;
};

__device__ __forceinline__ Seg seg_of(int64_t key) {
  const int lane = threadIdx.x & 63;
  const int64_t prev = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || prev != key;
  const uint64_t heads = __ballot(head);
  const uint64_t above = heads & ~((2ull << lane) - 1ull);
  Seg sg{lane, above ? __ffsll((unsigned long long)above) - 1 : 64, 0, head};
  while (sg.steps < 6 && __any(lane + (1 << sg.steps) < sg.seg_end)) ++sg.steps;
  return sg;
}

template <typename V>
__device__ __forceinline__ V seg_sum(const Seg &sg, V v) {
  for (int q = 0; q < sg.steps; ++q) {
    const int d = 1 << q;
    const V t = __shfl_down(v, d, 64);
    if (sg.lane + d < sg.seg_end) v += t;
  }
  return v;
}

template <bool PUSH>
__global__ __launch_bounds__(kBlock) void k_particles_alt(const StepArgs a, int mover) {
  const GridArgs &g = a.g;
  // the next order's tile flags are set by the sort's scan; every node may hold deposits
  if (blockIdx.y == 0) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (PUSH)
      for (int64_t t = t0; t < a.t.ntiles; t += stride) a.tile_active_next[t] = 0;
    if (a.mflag)
      for (int64_t f = t0; f < (a.g.nnodes + kFlagNodes - 1) / kFlagNodes; f += stride) a.mflag[f] = 1;
  }
  const int s = blockIdx.y;
  const SpeciesArgs &sp = a.sp[s];
  if (!sp.active) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = sp.cs[g.ncells];
  if ((int)(blockIdx.x * blockDim.x) >= n) return;  // the whole block past the particles
  const int lane = threadIdx.x & 63;
  // what the lane adds: moments at 4 nodes (dep), a move count (cnt_on), an arrival
  bool dep = false, cnt_on = false;
  int64_t dkey = 0, ckey = 0, cidx = 0;
  int64_t node[4] = {0, 0, 0, 0};
  double W[4] = {0.0, 0.0, 0.0, 0.0}, v[13];
  for (int r = 0; r < 13; ++r) v[r] = 0.0;
  if (j < n) {
    const int p = sp.perm[j];
    const double x = sp.src[0][p], z = sp.src[1][p];
    const double u[3] = {sp.src[2][p], sp.src[3][p], sp.src[4][p]};
    const double wp = sp.w_stride ? sp.src_w[p] : sp.w;
    const int i = (int)floor(x), k = (int)floor(z);
    if (i < 0 || i >= g.nx || k < 0 || k >= g.nz) {
      atomicOr(a.flags, kFlagOrderA);
      if (PUSH) sp.locode[j] = ((uint32_t)j << 4) | kAbsorbed;
    } else {
      corners(g, i, k, x - (double)i, z - (double)k, node, W);
      double B[3];
      b_at(g, a.Hold, mover, x, z, i, k, B);
      const double gam = gamma_bar(g, a.Eold, mover, sp.beta, u, node, W);
      if (!PUSH) {
        moments13(sp, gam, u, B, wp, v);
        dep = true;
        dkey = (int64_t)k * g.nx + i;
      } else {
        // E-bar at the particle and the implicit push: a = u + beta E-bar, b = beta B / gamma-bar,
        // u-bar = (a + a x b + (a.b) b) / (1 + b.b), u' = 2 u-bar - u
        const int64_t nn = g.nnodes;
        double Eb[3];
        for (int r = 0; r < 3; ++r) {
          const double *eo = a.Eold + r * nn, *en = a.Enew + r * nn;
          double acc = 0.0;
          for (int c = 0; c < 4; ++c) acc += W[c] * (0.5 * (eo[node[c]] + en[node[c]]));
          Eb[r] = acc;
        }
        const double bx = sp.beta / gam * B[0], by = sp.beta / gam * B[1], bz = sp.beta / gam * B[2];
        const double a0 = u[0] + sp.beta * Eb[0], a1 = u[1] + sp.beta * Eb[1], a2 = u[2] + sp.beta * Eb[2];
        const double inv = 1.0 / (1.0 + bx * bx + by * by + bz * bz);
        const double ab = a0 * bx + a1 * by + a2 * bz;
        double un[3];
        un[0] = 2.0 * ((a0 + (a1 * bz - a2 * by) + ab * bx) * inv) - u[0];
        un[1] = 2.0 * ((a1 + (a2 * bx - a0 * bz) + ab * by) * inv) - u[1];
        un[2] = 2.0 * ((a2 + (a0 * by - a1 * bx) + ab * bz) * inv) - u[2];
        const double g1 = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
        double xn = x + g.cx * (un[0] / g1), zn = z + g.cz * (un[2] / g1);
        bool alive = true;
        if (g.bc_x == PIC_BC_PERIODIC) {
          if (xn < 0.0) xn += (double)g.nx;
          if (xn >= (double)g.nx) xn -= (double)g.nx;
        } else if (xn < 0.0 || xn >= (double)g.nx) {
          alive = false;
        }
        if (zn < 0.0) zn += (double)g.nz;
        if (zn >= (double)g.nz) zn -= (double)g.nz;
        const bool finite = isfinite(g1) && isfinite(xn) && isfinite(zn);
        if (!finite) atomicOr(a.flags, kFlagNonFiniteA);
        alive = alive && finite;
        const int i2 = finite ? (int)floor(xn) : i, k2 = finite ? (int)floor(zn) : k;
        int di = i2 - i, dk = k2 - k;
        if (di > 1) di -= g.nx;
        if (di < -1) di += g.nx;
        if (dk > 1) dk -= g.nz;
        if (dk < -1) dk += g.nz;
        const bool jump = di < -1 || di > 1 || dk < -1 || dk > 1;
        if (alive && jump) atomicOr(a.flags, kFlagJumpA);
        alive = alive && !jump;
        const uint32_t code = alive ? (uint32_t)((dk + 1) * 3 + (di + 1)) : kAbsorbed;
        // the pushed state goes to location j of the other buffer; the sort reads the codes
        sp.dst[0][j] = xn;
        sp.dst[1][j] = zn;
        sp.dst[2][j] = un[0];
        sp.dst[3][j] = un[1];
        sp.dst[4][j] = un[2];
        if (sp.dst_id) sp.dst_id[j] = sp.src_id[p];
        if (sp.w_stride) sp.dst_w[j] = wp;
        sp.locode[j] = ((uint32_t)j << 4) | code;
        if (alive) {
          const int64_t src_cell = (int64_t)k * g.nx + i;
          cnt_on = true;
          ckey = (src_cell << 4) | code;
          cidx = (int64_t)code * g.ncells + src_cell;
          // the moments at x^{n+3/2} with u^{n+1}, B = H^{n+3/2} at the new position and
          // E^{n+1}
          corners(g, i2, k2, xn - (double)i2, zn - (double)k2, node, W);
          double B2[3];
          b_at(g, a.Hnew, mover, xn, zn, i2, k2, B2);
          const double gam2 = gamma_bar(g, a.Enew, mover, sp.beta, un, node, W);
          moments13(sp, gam2, un, B2, wp, v);
          dep = true;
          dkey = (int64_t)k2 * g.nx + i2;
        }
      }
    }
  }
  // move counts and arrivals, then the moments, each summed over the lanes' runs
  const Seg sd = seg_of(dep ? dkey : -1 - (int64_t)lane);
  if (PUSH) {
    const Seg sc = seg_of(cnt_on ? ckey : -1 - (int64_t)lane);
    const int nc_ = seg_sum(sc, cnt_on ? 1 : 0);
    if (cnt_on && sc.head) atomicAdd(&sp.cnt[cidx], nc_);
    const int na_ = seg_sum(sd, dep ? 1 : 0);
    if (dep && sd.head) atomicAdd(&sp.arr[dkey], na_);
  }
  const int64_t nn = g.nnodes;
  for (int c = 0; c < 4; ++c) {
    for (int r = 0; r < 13; ++r) {
      const double t = seg_sum(sd, W[c] * v[r]);
      if (dep && sd.head) unsafeAtomicAdd(&a.M[(int64_t)(r < 12 ? r : 12 + s) * nn + node[c]], t);
    }
  }
}

// Energies: out[0] field, out[1 + s] kinetic of species s (both times dx dz), summed over
// blocks with FP64 atomics.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kBlock) void k_energy(const StepArgs a, const double *E,
                                                   const double *H, double *out) {
  __shared__ double sh[kBlock / 64];
  const GridArgs &g = a.g;
  const double area = g.dx * g.dz;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double f = 0.0;
  for (int64_t e = tid; e < 3 * g.nnodes; e += stride) f += E[e] * E[e];
  for (int64_t e = tid; e < 3 * g.ncells; e += stride) f += H[e] * H[e];
  const double fs = block_sum(f, sh);
  if (threadIdx.x == 0) unsafeAtomicAdd(&out[0], 0.5 * fs * area);
  for (int s = 0; s < a.nsp; ++s) {
    const SpeciesArgs &sp = a.sp[s];
    if (!sp.active) continue;
    const int n = sp.cs[g.ncells];
    double kin = 0.0;
    for (int64_t j = tid; j < n; j += stride) {
      const int p = sp.perm[j];
      double u0, u1, u2;
      if (a.mixed) {
        u0 = (double)sp.msrc[2][p];
        u1 = (double)sp.msrc[3][p];
        u2 = (double)sp.msrc[4][p];
      } else {
        u0 = sp.src[2][p];
        u1 = sp.src[3][p];
        u2 = sp.src[4][p];
      }
      // the particle's density (one per species unless carried per particle)
      double wp = 1.0;
      if (sp.w_stride) wp = a.mixed ? (double)sp.msrc_w[p] : sp.src_w[p];
      kin += wp * (sqrt(1.0 + u0 * u0 + u1 * u1 + u2 * u2) - 1.0);
    }
    const double ks = block_sum(kin, sh);
    const double wsp = sp.w_stride ? 1.0 : sp.w;
    if (threadIdx.x == 0) unsafeAtomicAdd(&out[1 + s], ks * wsp * sp.m * area);
  }
}

// ---- energy without device allocation ----------------------------------------------------
// The same sums as k_energy, reduced in a fixed order: every block writes its partial sums
// (field, then each species slot) to its own row of a fixed buffer, and one block adds the rows
// in block order.  Every value is written before it is read, so nothing needs clearing, and
// the result does not depend on the timing of the blocks.

__global__ __launch_bounds__(kBlock) void k_energy_partials(const StepArgs a, const double *E,
                                                            const double *H, double *part) {
  __shared__ double sh[kBlock / 64];
  const GridArgs &g = a.g;
  const double area = g.dx * g.dz;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double *row = part + (size_t)blockIdx.x * kEnergyVals;
  double f = 0.0;
  for (int64_t e = tid; e < 3 * g.nnodes; e += stride) f += E[e] * E[e];
  for (int64_t e = tid; e < 3 * g.ncells; e += stride) f += H[e] * H[e];
  const double fs = block_sum(f, sh);
  if (threadIdx.x == 0) row[0] = 0.5 * fs * area;
  for (int s = 0; s < kMaxSpecies; ++s) {
    if (s >= a.nsp || !a.sp[s].active) {
      if (threadIdx.x == 0) row[1 + s] = 0.0;
      continue;
    }
    const SpeciesArgs &sp = a.sp[s];
    const int n = sp.cs[g.ncells];
    double kin = 0.0;
    for (int64_t j = tid; j < n; j += stride) {
      const int p = sp.perm[j];
      double u0, u1, u2, wp = 1.0;
      if (a.mixed) {
        u0 = (double)sp.msrc[2][p];
        u1 = (double)sp.msrc[3][p];
        u2 = (double)sp.msrc[4][p];
        if (sp.w_stride) wp = (double)sp.msrc_w[p];
      } else {
        u0 = sp.src[2][p];
        u1 = sp.src[3][p];
        u2 = sp.src[4][p];
        if (sp.w_stride) wp = sp.src_w[p];
      }
      kin += wp * (sqrt(1.0 + u0 * u0 + u1 * u1 + u2 * u2) - 1.0);
    }
    const double ks = block_sum(kin, sh);
    const double wsp = sp.w_stride ? 1.0 : sp.w;
    if (threadIdx.x == 0) row[1 + s] = ks * wsp * sp.m * area;
  }
}

// Totals: thread v adds column v of the kEnergyBlocks rows in row order.
__global__ void k_energy_total(const double *part, double *total) {
  const int v = threadIdx.x;
  if (v >= kEnergyVals) return;
  double t = 0.0;
  for (int b = 0; b < kEnergyBlocks; ++b) t += part[(size_t)b * kEnergyVals + v];
  total[v] = t;
}

// The fixed buffer: kEnergyBlocks rows of partial sums, then the kEnergyVals totals.  One copy
// per GPU, kept until the process ends; every call on a GPU uses that GPU's copy.
static __device__ __align__(256) double scratch[kEnergyScratchDoubles];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

}  // namespace

hipError_t energy_scratch(int32_t device, double **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    // the address of this device's copy, looked up once with the device current (the array's
    // name in host code is not a device address)
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_energy_scratch(const StepArgs &a, const double *E, const double *H,
                                 double *scratch_ptr, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_partials, dim3(kEnergyBlocks), dim3(kBlock), 0, s, a, E, H,
                     scratch_ptr);
  hipLaunchKernelGGL(k_energy_total, dim3(1), dim3(64), 0, s, scratch_ptr,
                     scratch_ptr + kEnergyBlocks * kEnergyVals);
  return hipGetLastError();
}

hipError_t launch_particles_alt(const StepArgs &a, bool push, int mover, int32_t max_n,
                                hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(
      1, std::max<int64_t>((max_n + kBlock - 1) / kBlock, (a.t.ntiles + kBlock - 1) / kBlock));
  const dim3 grid(nb, (unsigned)a.nsp);
  if (push)
    hipLaunchKernelGGL(k_particles_alt<true>, grid, dim3(kBlock), 0, s, a, mover);
  else
    hipLaunchKernelGGL(k_particles_alt<false>, grid, dim3(kBlock), 0, s, a, mover);
  return hipGetLastError();
}

hipError_t launch_energy(const StepArgs &a, const double *E, const double *H, double *out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_energy, dim3(1024), dim3(kBlock), 0, s, a, E, H, out);
  return hipGetLastError();
}

}  // namespace pic
