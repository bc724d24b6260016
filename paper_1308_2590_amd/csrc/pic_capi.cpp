// Host side of the C ABI declared in include/pic.h: context life cycle, device buffers,
// particle loading, the per-cycle kernel sequence and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_ctx.h"
#include "pic_internal.h"

using pic::ProfEvents;
using pic::SpeciesState;

namespace {

thread_local std::string g_init_error;

// The allocator hook of pic_set_allocator (process-wide; each context and batch copies it when
// it is created).
std::mutex g_alloc_mu;
pic_alloc_fn g_alloc = nullptr;
pic_free_fn g_free = nullptr;
void *g_alloc_user = nullptr;

}  // namespace

namespace pic {

DevAlloc current_allocator(int32_t device) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  DevAlloc a;
  a.alloc = g_alloc;
  a.free = g_free;
  a.user = g_alloc_user;
  a.device = device;
  return a;
}

hipError_t DevAlloc::get(void **p, size_t n) {
  *p = nullptr;
  if (alloc) {
    *p = alloc((uint64_t)n, device, user);
    if (!*p) return hipErrorOutOfMemory;
  } else {
    const hipError_t e = hipMalloc(p, n);
    if (e != hipSuccess) {
      *p = nullptr;
      return e;
    }
  }
  live[*p] = n;
  bytes += (int64_t)n;
  return hipSuccess;
}

void DevAlloc::put(void *p) {
  if (!p) return;
  auto it = live.find(p);
  const size_t n = it == live.end() ? 0 : it->second;
  if (it != live.end()) live.erase(it);
  bytes -= (int64_t)n;
  if (free)
    free(p, (uint64_t)n, device, user);
  else
    (void)hipFree(p);
}

void DevAlloc::put_all() {
  std::vector<void *> ps;
  for (auto &kv : live) ps.push_back(kv.first);
  for (void *p : ps) put(p);
}

}  // namespace pic

namespace {

pic_status fail(pic_ctx *c, pic_status st, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_init_error = msg;
  return st;
}

pic_status hip_fail(pic_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? PIC_ERR_OOM : PIC_ERR_DEVICE, m);
}

#define HIP_TRY(ctx, expr, what)                 \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

template <typename T>
pic_status dalloc(pic_ctx *c, T **p, size_t count, const char *what) {
  *p = nullptr;
  if (count == 0) count = 1;
  void *q = nullptr;
  hipError_t e = c->mem.get(&q, count * sizeof(T));
  if (e != hipSuccess) {
    if (c->mem.alloc && e == hipErrorOutOfMemory)
      return fail(c, PIC_ERR_OOM, std::string(what) + ": the allocator returned no memory for " +
                                       std::to_string(count * sizeof(T)) + " bytes");
    return hip_fail(c, e, what);
  }
  *p = static_cast<T *>(q);
  return PIC_OK;
}

// Host <-> device copies and fills run on the context's stream and the host waits for it.  The
// null stream is not used: it would wait for every blocking stream's unrelated work, and an
// operation on it invalidates a graph capture another thread has under way (a serving loop
// loads new runs on one thread while it captures the batch's cycle on another).
hipError_t copy_wait(pic_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
  const hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, c->stream);
  return e == hipSuccess ? hipStreamSynchronize(c->stream) : e;
}

hipError_t fill_wait(pic_ctx *c, void *dst, int value, size_t bytes) {
  const hipError_t e = hipMemsetAsync(dst, value, bytes, c->stream);
  return e == hipSuccess ? hipStreamSynchronize(c->stream) : e;
}

// Release a block of the context (its size is known to the allocator record).
void dfree(pic_ctx *c, void *p, size_t /*bytes*/) { c->mem.put(p); }

void free_species(pic_ctx *c, SpeciesState &s) {
  const size_t cap = (size_t)std::max<int64_t>(s.cap, 1);
  const size_t nc = (size_t)c->g.ncells;
  for (int b = 0; b < 2; ++b) {
    for (int v = 0; v < 5; ++v) dfree(c, s.buf[b][v], cap * sizeof(double)), s.buf[b][v] = nullptr;
    for (int v = 0; v < 5; ++v) dfree(c, s.mbuf[b][v], cap * sizeof(float)), s.mbuf[b][v] = nullptr;
    dfree(c, s.mcell[b], cap * sizeof(int32_t)), s.mcell[b] = nullptr;
    dfree(c, s.ids[b], cap * sizeof(int64_t)), s.ids[b] = nullptr;
    dfree(c, s.wbuf[b], cap * sizeof(double)), s.wbuf[b] = nullptr;
    dfree(c, s.mwbuf[b], cap * sizeof(float)), s.mwbuf[b] = nullptr;
    dfree(c, s.perm[b], (cap + pic::kPermPad) * sizeof(int32_t)), s.perm[b] = nullptr;
    dfree(c, s.cs[b], (nc + 1) * sizeof(int32_t)), s.cs[b] = nullptr;
  }
  dfree(c, s.locode, cap * sizeof(uint32_t)), s.locode = nullptr;
  dfree(c, s.cnt, (size_t)pic::kMoveCodes * nc * sizeof(int32_t)), s.cnt = nullptr;
  dfree(c, s.cmask, nc * sizeof(uint16_t)), s.cmask = nullptr;
  dfree(c, s.arr, nc * sizeof(int32_t)), s.arr = nullptr;
  dfree(c, s.bsum, (size_t)c->n_scan_blocks * sizeof(int32_t)), s.bsum = nullptr;
  s.loaded = false;
  s.pw = false;
  s.cap = 0;
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

bool mixed(const pic_ctx *c) { return c->d.precision == PIC_PREC_MIXED; }

// Whether some loaded species carries per-particle densities (the kernels with them run).
bool any_pw(const pic_ctx *c) {
  for (int s = 0; s < c->S; ++s)
    if (c->sp[s].loaded && c->sp[s].pw) return true;
  return false;
}

// Tile size from the load.  One wavefront handles one row of a tile, each lane a contiguous
// run of that row's particles.  The rule follows what timing every candidate shape measured on
// uniform and slab loads: tiles 16 cells wide where the occupied part of a row is at most 16
// cells (a narrow slab), otherwise 32, or 8 in mixed precision above 16 particles per occupied
// cell and species (three wavefronts per SIMD want more, smaller blocks); and as many rows (1 to 4) as
// bring a tile to about 4096 particles per species (mixed: 2048), counting only the occupied
// cells of a row.
// Shrunk in x until two blocks fit in the LDS of a CU (half the LDS a block may use).
// ppc: particles per occupied cell and species; width: occupied cells per occupied row.
void choose_tiles(pic_ctx *c, double ppc, double width) {
  int tx = c->d.tile_x, tz = c->d.tile_z;
  if (tx <= 0 || tz <= 0) {
    const bool mx = mixed(c);
    tx = width <= 16.0 ? 16 : (mx && ppc > 16.0) ? 8 : 32;
    const double per_row = std::max(1.0, std::min((double)tx, width) * ppc);
    tz = (int)std::lround((mx ? 2048.0 : 4096.0) / per_row);
    tz = std::min(4, std::max(1, tz));
    while (tx > 4 &&
           pic::particle_lds_bytes(c->g, pic::TileArgs{tx, tz, 0, 0, 0, 0}, mixed(c), any_pw(c)) >
               c->lds_max / 2)
      tx /= 2;
  }
  c->tiles.tx = tx;
  c->tiles.tz = tz;
  c->tiles.ntx = (c->g.nx + tx - 1) / tx;
  c->tiles.ntz = (c->g.nz + tz - 1) / tz;
  c->tiles.ntiles = c->tiles.ntx * c->tiles.ntz;
  c->tiles.per_xcd = (c->tiles.ntiles + 7) / 8;
}

// The sort's ranker: one thread per cell up to this many particles per occupied cell and
// species, the row walk above.
constexpr double kRankCellsMaxPerCell = 16.0;

bool rank_cells(const pic_ctx *c) {
  if (c->rank_mode == PIC_RANK_CELLS) return true;
  if (c->rank_mode == PIC_RANK_ROWS) return false;
  return c->rank_cells_auto;
}

pic::StepArgs step_args(pic_ctx *c, bool push) {
  pic::StepArgs a{};
  a.g = c->g;
  a.t = c->tiles;
  a.mixed = mixed(c) ? 1 : 0;
  a.rank_cells = rank_cells(c) ? 1 : 0;
  a.chunk2 = c->chunk2 ? 1 : 0;
  // the per-cell ranker reads code masks, which the tile kernel writes (not the per-particle
  // kernel of the mover options, which accumulates full counts)
  a.count_masks = (a.rank_cells && !c->mover) ? 1 : 0;
  a.n_scan_blocks = c->n_scan_blocks;
  a.n_scan1_blocks = c->n_scan1_blocks;
  a.nsp = c->S;
  const int cur = c->cur, nxt = 1 - c->cur;
  for (int s = 0; s < c->S; ++s) {
    SpeciesState &st = c->sp[s];
    pic::SpeciesArgs &x = a.sp[s];
    x.active = st.loaded ? 1 : 0;
    if (!st.loaded) continue;
    x.cap = (int32_t)st.cap;
    x.q = st.q;
    x.m = st.m;
    x.w = st.w;
    x.beta = st.q * c->g.dt / (2.0 * st.m);
    x.cS = st.w * st.q * st.q * c->g.dt * c->g.dt / (4.0 * st.m);
    x.kJ = st.w * st.q;
    x.cS1 = st.q * st.q * c->g.dt * c->g.dt / (4.0 * st.m);
    x.kJ1 = st.q;
    if (st.pw) {
      x.w_stride = 1;
      x.src_w = st.wbuf[cur];
      x.dst_w = push ? st.wbuf[nxt] : nullptr;
      x.msrc_w = st.mwbuf[cur];
      x.mdst_w = push ? st.mwbuf[nxt] : nullptr;
    } else {
      // the species' single density, read with stride 0 and never written
      x.w_stride = 0;
      x.src_w = c->wconst64 + s;
      x.dst_w = c->wconst64 + s;
      x.msrc_w = c->wconst32 + s;
      x.mdst_w = c->wconst32 + s;
    }
    for (int v = 0; v < 5; ++v) {
      x.src[v] = st.buf[cur][v];
      x.dst[v] = push ? st.buf[nxt][v] : nullptr;
      x.msrc[v] = st.mbuf[cur][v];
      x.mdst[v] = push ? st.mbuf[nxt][v] : nullptr;
    }
    x.msrc_cell = st.mcell[cur];
    x.mdst_cell = push ? st.mcell[nxt] : nullptr;
    x.src_id = st.ids[cur];
    x.dst_id = push ? st.ids[nxt] : nullptr;
    x.perm = st.perm[cur];
    x.perm_new = st.perm[nxt];
    x.cs = st.cs[cur];
    x.cs_new = st.cs[nxt];
    x.locode = st.locode;
    x.cnt = st.cnt;
    x.cmask = st.cmask;
    x.arr = st.arr;
    x.bsum = st.bsum;
  }
  a.flags = c->flags;
  a.tile_active = c->tact[cur];
  a.tile_list = c->tlist[cur];
  a.tile_active_next = c->tact[nxt];
  a.tile_list_next = c->tlist[nxt];
  a.mflag = c->mflag;
  return a;
}

// (Re)allocate the active-tile arrays for the current tile decomposition.
pic_status alloc_tiles(pic_ctx *c) {
  const int32_t nt = c->tiles.ntiles;
  if (nt == c->tiles_alloc && c->tiles.tx == c->tiles_tx && c->tiles.tz == c->tiles_tz) return PIC_OK;
  c->tiles_tx = c->tiles.tx;
  c->tiles_tz = c->tiles.tz;
  for (int b = 0; b < 2; ++b) {
    dfree(c, c->tact[b], (size_t)std::max(c->tiles_alloc, 1));
    dfree(c, c->tlist[b], ((size_t)c->tiles_alloc + 1) * sizeof(int32_t));
    c->tact[b] = nullptr;
    c->tlist[b] = nullptr;
  }
  c->tiles_alloc = 0;
  pic_status st;
  for (int b = 0; b < 2; ++b) {
    if ((st = dalloc(c, &c->tact[b], (size_t)nt, "alloc tile flags")) != PIC_OK) return st;
    if ((st = dalloc(c, &c->tlist[b], (size_t)nt + 1, "alloc tile list")) != PIC_OK) return st;
  }
  c->tiles_alloc = nt;
  return PIC_OK;
}

// Active-tile flags and list of the current order (after loads).
pic_status build_tile_list(pic_ctx *c) {
  pic::StepArgs a = step_args(c, false);
  a.tile_active_next = c->tact[c->cur];
  a.tile_list_next = c->tlist[c->cur];
  HIP_TRY(c, pic::launch_tile_list(a, false, c->stream), "tile list");
  return PIC_OK;
}

// Largest particle capacity of the loaded species (bounds the per-particle kernel's grid).
int32_t max_particles(const pic_ctx *c) {
  int64_t m = 0;
  for (int s = 0; s < c->S; ++s)
    if (c->sp[s].loaded) m = std::max<int64_t>(m, c->sp[s].cap);
  return (int32_t)m;
}

// Deposit M^{k+1/2} of the current state (used after loads).
pic_status redeposit(pic_ctx *c) {
  HIP_TRY(c, hipMemsetAsync(c->M, 0, (size_t)c->g.n_planes * c->g.nnodes * sizeof(double), c->stream),
          "clear moments");
  bool any = false;
  for (int s = 0; s < c->S; ++s) any = any || c->sp[s].loaded;
  if (!any) return PIC_OK;
  pic_status rs = alloc_tiles(c);
  if (rs != PIC_OK) return rs;
  if ((rs = build_tile_list(c)) != PIC_OK) return rs;
  pic::StepArgs a = step_args(c, false);
  a.Eold = a.Enew = c->E[c->ecur];  // E^n: read by the gamma-bar predictor of the options only
  a.Hold = c->H[c->hcur];
  a.Hnew = c->H[c->hcur];
  a.M = c->M;
  if (c->mover)
    HIP_TRY(c, pic::launch_particles_alt(a, false, c->mover, max_particles(c), c->stream), "deposit kernel");
  else
    HIP_TRY(c, pic::launch_particles(a, false, c->stream), "deposit kernel");
  return PIC_OK;
}

// The particle stage of one cycle: the tile kernel, or with mover options the per-particle
// kernel (whose move counts are accumulated from zero).
pic_status particle_stage(pic_ctx *c, const pic::StepArgs &a) {
  if (!c->mover) {
    HIP_TRY(c, pic::launch_particles(a, true, c->stream), "particle kernel");
    return PIC_OK;
  }
  for (int s = 0; s < c->S; ++s)
    if (c->sp[s].loaded)
      HIP_TRY(c, hipMemsetAsync(c->sp[s].cnt, 0, (size_t)pic::kMoveCodes * c->g.ncells * sizeof(int32_t),
                                c->stream), "clear move counts");
  HIP_TRY(c, pic::launch_particles_alt(a, true, c->mover, max_particles(c), c->stream), "particle kernel");
  return PIC_OK;
}

// Tile shape from the descriptor's tile_x / tile_z, or from the load when those are 0: the
// particles per occupied cell and species, and the occupied cells per occupied row.  Waits
// for the stream (reads the cell starts).
pic_status retile(pic_ctx *c) {
  const int64_t nc = c->g.ncells;
  std::vector<uint8_t> occ((size_t)nc, 0);
  std::vector<int32_t> csh((size_t)nc + 1);
  int64_t total = 0;
  int nloaded = 0;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  for (int ss = 0; ss < c->S; ++ss) {
    if (!c->sp[ss].loaded) continue;
    ++nloaded;
    HIP_TRY(c, copy_wait(c, csh.data(), c->sp[ss].cs[c->cur], ((size_t)nc + 1) * sizeof(int32_t),
                         hipMemcpyDeviceToHost), "read cell starts");
    for (int64_t cc = 0; cc < nc; ++cc)
      if (csh[cc + 1] > csh[cc]) occ[cc] = 1;
    total += csh[nc];
  }
  int64_t occupied = 0, rows = 0;
  for (int64_t k = 0; k < c->g.nz; ++k) {
    int64_t in_row = 0;
    for (int64_t i = 0; i < c->g.nx; ++i) in_row += occ[(size_t)(k * c->g.nx + i)];
    occupied += in_row;
    rows += in_row > 0 ? 1 : 0;
  }
  const double ppc = occupied > 0 ? (double)total / (double)occupied / std::max(nloaded, 1) : 1.0;
  const double width = rows > 0 ? (double)occupied / (double)rows : (double)c->g.nx;
  choose_tiles(c, ppc, width);
  c->rank_cells_auto = occupied > 0 && ppc <= kRankCellsMaxPerCell;
  // particles per lane in a tile row (a row splits over the wavefronts when the tile has fewer
  // rows than the block has wavefronts): chunks of 2 up to 2.5 of them
  {
    const int waves_per_row = c->tiles.tz >= 4 ? 1 : 4 / c->tiles.tz;
    const double per_lane = std::min((double)c->tiles.tx, width) * ppc / (64.0 * waves_per_row);
    c->chunk2 = occupied > 0 && per_lane <= 2.5;
  }
  if (pic::particle_lds_bytes(c->g, c->tiles, mixed(c), any_pw(c)) > c->lds_max)
    return fail(c, PIC_ERR_ARG, "tile too large: its LDS accumulators exceed the LDS of a block");
  return PIC_OK;
}

void prof_accumulate(pic_ctx *c) {
  for (size_t q = 0; q < c->prof_used; ++q) {
    ProfEvents &p = c->prof_ev[q];
    float t_field = 0, t_part = 0, t_sort = 0, t_step = 0;
    (void)hipEventElapsedTime(&t_field, p.ev[0], p.ev[1]);
    (void)hipEventElapsedTime(&t_part, p.ev[1], p.ev[2]);
    (void)hipEventElapsedTime(&t_sort, p.ev[2], p.ev[3]);
    (void)hipEventElapsedTime(&t_step, p.ev[0], p.ev[3]);
    c->prof_acc.steps += 1;
    c->prof_acc.field_launches += 1;
    c->prof_acc.particle_launches += 1;
    c->prof_acc.sort_launches += 1;
    c->prof_acc.field_ms += t_field;
    c->prof_acc.particle_ms += t_part;
    c->prof_acc.sort_ms += t_sort;
    c->prof_acc.step_ms += t_step;
  }
  c->prof_used = 0;
}

}  // namespace

namespace pic {

StepArgs cycle_step_args(pic_ctx *c, int p) {
  const int saved = c->cur;
  c->cur = p;
  StepArgs a = step_args(c, true);
  c->cur = saved;
  a.Eold = c->E[p];
  a.Enew = c->E[1 - p];
  a.Hold = c->H[p];
  a.Hnew = c->H[1 - p];
  a.M = c->M;
  return a;
}

FieldArgs cycle_field_args(pic_ctx *c, int p) {
  FieldArgs fa{};
  fa.g = c->g;
  fa.laser = c->laser;
  fa.t = (double)c->step * c->g.dt;
  fa.M = c->M;
  fa.E = c->E[p];
  fa.H = c->H[p];
  fa.E_new = c->E[1 - p];
  fa.H_new = c->H[1 - p];
  fa.mflag = c->mflag;
  fa.ntiles_next = c->tiles.ntiles;
  fa.r2dx = 1.0 / (2.0 * c->g.dx);
  fa.r2dz = 1.0 / (2.0 * c->g.dz);
  return fa;
}

}  // namespace pic

extern "C" {

pic_status pic_init_grid(const pic_grid_desc *d, pic_ctx **out) {
  if (!out) return fail(nullptr, PIC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!d) return fail(nullptr, PIC_ERR_ARG, "descriptor is NULL");
  for (int r = 0; r < 7; ++r)
    if (d->reserved[r] != 0) return fail(nullptr, PIC_ERR_ARG, "reserved fields must be zero");
  if (d->nx < 1 || d->nz < 1) return fail(nullptr, PIC_ERR_ARG, "nx and nz must be >= 1");
  if ((int64_t)d->nx * d->nz > 0x7fffffffLL - 1) return fail(nullptr, PIC_ERR_ARG, "too many cells");
  // the kernels find a cell's tile by a float-reciprocal quotient, exact below 2^22
  if (d->nx >= (1 << 22) || d->nz >= (1 << 22))
    return fail(nullptr, PIC_ERR_ARG, "nx and nz must be below 2^22");
  if (!(d->dx > 0 && d->dz > 0 && d->dt > 0) || !std::isfinite(d->dx) || !std::isfinite(d->dz) ||
      !std::isfinite(d->dt))
    return fail(nullptr, PIC_ERR_ARG, "dx, dz, dt must be positive and finite");
  if (d->bc_x != PIC_BC_PERIODIC && d->bc_x != PIC_BC_ABSORBING)
    return fail(nullptr, PIC_ERR_ARG, "bc_x must be periodic or absorbing");
  if (d->bc_z != PIC_BC_PERIODIC) return fail(nullptr, PIC_ERR_ARG, "bc_z must be periodic");
  if (d->bc_x == PIC_BC_ABSORBING && d->nx < 2)
    return fail(nullptr, PIC_ERR_ARG, "an absorbing x axis needs nx >= 2");
  if (d->precision != PIC_PREC_FP64 && d->precision != PIC_PREC_MIXED)
    return fail(nullptr, PIC_ERR_ARG, "precision must be PIC_PREC_FP64 or PIC_PREC_MIXED");
  if (d->n_species < 1 || d->n_species > PIC_MAX_SPECIES)
    return fail(nullptr, PIC_ERR_ARG, "n_species must be in 1..8");
  if (d->allow_cfl_violation != 0 || d->dt > std::min(d->dx, d->dz))
    return fail(nullptr, PIC_ERR_ARG,
                "dt must not exceed min(dx, dz): the explicit curls are unstable beyond it and the "
                "cell sort relies on particles moving less than one cell per cycle");
  if (d->track_ids != 0 && d->track_ids != 1) return fail(nullptr, PIC_ERR_ARG, "track_ids must be 0 or 1");
  if (d->tile_x < 0 || d->tile_z < 0 || d->tile_x > 64 || d->tile_z > 64 ||
      ((d->tile_x == 0) != (d->tile_z == 0)))
    return fail(nullptr, PIC_ERR_ARG, "tile_x, tile_z must both be 0 or both in 1..64");
  if (!finite3(d->e0) || !finite3(d->h0)) return fail(nullptr, PIC_ERR_ARG, "e0, h0 must be finite");
  const double lz[6] = {d->laser_a0, d->laser_omega, d->laser_sigma_z, d->laser_z_center,
                        d->laser_fwhm_t, d->laser_t_center};
  for (double v : lz)
    if (!std::isfinite(v)) return fail(nullptr, PIC_ERR_ARG, "laser parameters must be finite");
  if (d->laser_a0 != 0.0) {
    if (d->bc_x != PIC_BC_ABSORBING)
      return fail(nullptr, PIC_ERR_ARG, "the x = 0 source needs an absorbing x axis");
    if (!(d->laser_sigma_z > 0 && d->laser_fwhm_t > 0))
      return fail(nullptr, PIC_ERR_ARG, "laser sigma_z and fwhm_t must be positive");
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) return fail(nullptr, PIC_ERR_DEVICE, "no HIP device available");
  if (d->device < 0 || d->device >= ndev) return fail(nullptr, PIC_ERR_ARG, "device ordinal out of range");
  e = hipSetDevice(d->device);
  if (e != hipSuccess) return fail(nullptr, PIC_ERR_DEVICE, "hipSetDevice failed");
  int lds_max = 0;
  e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, d->device);
  if (e != hipSuccess || lds_max <= 0) return fail(nullptr, PIC_ERR_DEVICE, "cannot read the LDS size");

  pic_ctx *c = new pic_ctx();
  c->d = *d;
  c->mem = pic::current_allocator(d->device);
  c->lds_max = (size_t)lds_max;
  c->S = d->n_species;
  pic::GridArgs &g = c->g;
  g.nx = d->nx;
  g.nz = d->nz;
  g.nxn = d->nx + (d->bc_x == PIC_BC_ABSORBING ? 1 : 0);
  g.nzn = d->nz;
  g.bc_x = d->bc_x;
  g.n_planes = 12 + c->S;
  g.ncells = (int64_t)d->nx * d->nz;
  g.nnodes = (int64_t)g.nxn * g.nzn;
  g.dx = d->dx;
  g.dz = d->dz;
  g.dt = d->dt;
  g.cx = d->dt / d->dx;
  g.cz = d->dt / d->dz;
  c->laser = pic::LaserArgs{d->laser_a0, d->laser_omega, d->laser_sigma_z, d->laser_z_center,
                            d->laser_fwhm_t, d->laser_t_center};
  c->n_scan_blocks = (int32_t)((g.ncells + pic::kScanBlock - 1) / pic::kScanBlock);
  c->n_scan1_blocks = (int32_t)((g.ncells + pic::kScan1Block - 1) / pic::kScan1Block);
  choose_tiles(c, 1.0, (double)g.nx);

  pic_status st = PIC_OK;
  auto bail = [&](pic_status s2) {
    g_init_error = c->err;
    pic_destroy(c);
    return s2;
  };
  e = hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(hip_fail(c, e, "hipStreamCreate"));
  c->stream = c->own_stream;
  const size_t nn = (size_t)g.nnodes, nc = (size_t)g.ncells;
  for (int b = 0; b < 2; ++b) {
    if ((st = dalloc(c, &c->E[b], 3 * nn, "alloc E")) != PIC_OK) return bail(st);
    if ((st = dalloc(c, &c->H[b], 3 * nc, "alloc H")) != PIC_OK) return bail(st);
  }
  if ((st = dalloc(c, &c->M, (size_t)g.n_planes * nn, "alloc moments")) != PIC_OK) return bail(st);
  if ((st = dalloc(c, &c->flags, 1, "alloc flags")) != PIC_OK) return bail(st);
  const size_t nflag = (nn + pic::kFlagNodes - 1) / pic::kFlagNodes;
  if ((st = dalloc(c, &c->mflag, nflag, "alloc deposit flags")) != PIC_OK) return bail(st);
  // 8 doubles, then 8 floats
  if ((st = dalloc(c, &c->wconst64, 12, "alloc densities")) != PIC_OK) return bail(st);
  c->wconst32 = reinterpret_cast<float *>(c->wconst64 + PIC_MAX_SPECIES);
  e = fill_wait(c, c->wconst64, 0, 12 * sizeof(double));
  if (e != hipSuccess) return bail(hip_fail(c, e, "clear densities"));
  std::vector<double> host(3 * std::max(nn, nc));
  for (int r = 0; r < 3; ++r) std::fill(host.begin() + r * nn, host.begin() + (r + 1) * nn, d->e0[r]);
  e = copy_wait(c, c->E[0], host.data(), 3 * nn * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(hip_fail(c, e, "upload E"));
  for (int r = 0; r < 3; ++r) std::fill(host.begin() + r * nc, host.begin() + (r + 1) * nc, d->h0[r]);
  e = copy_wait(c, c->H[0], host.data(), 3 * nc * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(hip_fail(c, e, "upload H"));
  e = fill_wait(c, c->M, 0, (size_t)g.n_planes * nn * sizeof(double));
  // the moments start at zero: no node holds a deposit
  if (e == hipSuccess) e = fill_wait(c, c->mflag, 0, nflag);
  if (e != hipSuccess) return bail(hip_fail(c, e, "clear moments"));
  e = fill_wait(c, c->flags, 0, sizeof(uint32_t));
  if (e != hipSuccess) return bail(hip_fail(c, e, "clear flags"));
  *out = c;
  return PIC_OK;
}

pic_status pic_load_particles(pic_ctx *c, int32_t s, double q, double m, int64_t n,
                              const double *xi_x, const double *xi_z, const double *ux,
                              const double *uy, const double *uz, const double *w,
                              double w_uniform) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (s < 0 || s >= c->S) return fail(c, PIC_ERR_ARG, "species index out of range");
  if (n < 0 || n >= (1LL << 28)) return fail(c, PIC_ERR_ARG, "n out of range (at most 2^28 - 1 per species)");
  if (!std::isfinite(q) || !std::isfinite(w_uniform) || !(m > 0) || !std::isfinite(m))
    return fail(c, PIC_ERR_ARG, "q, w_uniform must be finite and m positive");
  if (n > 0 && (!xi_x || !xi_z || !ux || !uy || !uz)) return fail(c, PIC_ERR_ARG, "NULL particle array");
  const pic::GridArgs &g = c->g;
  const int64_t nc = g.ncells;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  // validate and sort by cell (stable counting sort; input order breaks ties)
  std::vector<int32_t> key((size_t)n);
  std::vector<int32_t> start((size_t)nc + 1, 0);
  for (int64_t a = 0; a < n; ++a) {
    const double x = xi_x[a], z = xi_z[a];
    if (!(x >= 0.0 && x < (double)g.nx && z >= 0.0 && z < (double)g.nz))
      return fail(c, PIC_ERR_RANGE, "particle " + std::to_string(a) + " lies outside the domain");
    if (!std::isfinite(ux[a]) || !std::isfinite(uy[a]) || !std::isfinite(uz[a]))
      return fail(c, PIC_ERR_RANGE, "particle " + std::to_string(a) + " has a non-finite momentum");
    if (w && !std::isfinite(w[a]))
      return fail(c, PIC_ERR_RANGE, "particle " + std::to_string(a) + " has a non-finite density");
    const int32_t i = (int32_t)std::floor(x), k = (int32_t)std::floor(z);
    key[a] = k * g.nx + i;
    start[(size_t)key[a] + 1] += 1;
  }
  for (int64_t cc = 0; cc < nc; ++cc) start[cc + 1] += start[cc];
  std::vector<int32_t> order((size_t)n);
  {
    std::vector<int32_t> pos(start.begin(), start.end() - 1);
    for (int64_t a = 0; a < n; ++a) order[pos[key[a]]++] = (int32_t)a;
  }
  SpeciesState &st = c->sp[s];
  free_species(c, st);
  st.q = q;
  st.m = m;
  st.pw = w != nullptr;
  // with per-particle densities the kernels scale unit-density moments by each particle's own
  st.w = st.pw ? 1.0 : w_uniform;
  st.cap = n;
  st.n_loaded = n;
  const size_t cap = (size_t)std::max<int64_t>(n, 1);
  // on any failure below the species is left without particles
  auto bail = [&](pic_status r) {
    const std::string msg = c->err;
    free_species(c, st);
    c->err = msg;
    return r;
  };
  pic_status rs;
  for (int b = 0; b < 2; ++b) {
    if (mixed(c)) {
      if ((rs = dalloc(c, &st.mcell[b], cap, "alloc particles")) != PIC_OK) return bail(rs);
      for (int v = 0; v < 5; ++v)
        if ((rs = dalloc(c, &st.mbuf[b][v], cap, "alloc particles")) != PIC_OK) return bail(rs);
      if (st.pw && (rs = dalloc(c, &st.mwbuf[b], cap, "alloc densities")) != PIC_OK) return bail(rs);
    } else {
      for (int v = 0; v < 5; ++v)
        if ((rs = dalloc(c, &st.buf[b][v], cap, "alloc particles")) != PIC_OK) return bail(rs);
      if (st.pw && (rs = dalloc(c, &st.wbuf[b], cap, "alloc densities")) != PIC_OK) return bail(rs);
    }
    if (c->d.track_ids)
      if ((rs = dalloc(c, &st.ids[b], cap, "alloc ids")) != PIC_OK) return bail(rs);
    // padded: the particle kernel reads the permutation 4 entries at a time, up to 7 past
    // the last slot of a row part
    if ((rs = dalloc(c, &st.perm[b], cap + pic::kPermPad, "alloc perm")) != PIC_OK) return bail(rs);
    if (fill_wait(c, st.perm[b], 0, (cap + pic::kPermPad) * sizeof(int32_t)) != hipSuccess)
      return bail(fail(c, PIC_ERR_DEVICE, "clear perm"));
    if ((rs = dalloc(c, &st.cs[b], (size_t)nc + 1, "alloc cell starts")) != PIC_OK) return bail(rs);
  }
  if ((rs = dalloc(c, &st.locode, cap, "alloc codes")) != PIC_OK) return bail(rs);
  if ((rs = dalloc(c, &st.cnt, (size_t)pic::kMoveCodes * nc, "alloc counts")) != PIC_OK) return bail(rs);
  if ((rs = dalloc(c, &st.cmask, (size_t)nc, "alloc code masks")) != PIC_OK) return bail(rs);
  if ((rs = dalloc(c, &st.arr, (size_t)nc, "alloc arrivals")) != PIC_OK) return bail(rs);
  if (fill_wait(c, st.arr, 0, (size_t)nc * sizeof(int32_t)) != hipSuccess)
    return bail(fail(c, PIC_ERR_DEVICE, "clear arrivals"));
  if ((rs = dalloc(c, &st.bsum, (size_t)c->n_scan_blocks, "alloc scan sums")) != PIC_OK) return bail(rs);
  {
    auto up = [&](void *dst, const void *src, size_t bytes) {
      const hipError_t e = copy_wait(c, dst, src, bytes, hipMemcpyHostToDevice);
      return e == hipSuccess ? PIC_OK : hip_fail(c, e, "upload particles");
    };
    const double *srcs[5] = {xi_x, xi_z, ux, uy, uz};
    if (mixed(c)) {
      // cell key and FP32 offsets in [0, 1) (an offset that rounds up to 1 is taken as the
      // largest float below 1, so the particle stays in its cell), FP32 momenta and densities
      std::vector<int32_t> kc((size_t)n);
      std::vector<float> tmp((size_t)n);
      for (int64_t j = 0; j < n; ++j) kc[j] = key[order[j]];
      if ((rs = up(st.mcell[c->cur], kc.data(), (size_t)n * sizeof(int32_t))) != PIC_OK) return bail(rs);
      for (int v = 0; v < 6; ++v) {
        if (v == 5 && !st.pw) break;
        for (int64_t j = 0; j < n; ++j) {
          const double x = v < 5 ? srcs[v][order[j]] : w[order[j]];
          if (v < 2) {
            float f = (float)(x - std::floor(x));
            if (f >= 1.0f) f = std::nextafter(1.0f, 0.0f);
            tmp[j] = f;
          } else {
            tmp[j] = (float)x;
          }
        }
        float *dst = v < 5 ? st.mbuf[c->cur][v] : st.mwbuf[c->cur];
        if ((rs = up(dst, tmp.data(), (size_t)n * sizeof(float))) != PIC_OK) return bail(rs);
      }
    } else {
      std::vector<double> tmp((size_t)n);
      for (int v = 0; v < 6; ++v) {
        if (v == 5 && !st.pw) break;
        for (int64_t j = 0; j < n; ++j) tmp[j] = v < 5 ? srcs[v][order[j]] : w[order[j]];
        double *dst = v < 5 ? st.buf[c->cur][v] : st.wbuf[c->cur];
        if ((rs = up(dst, tmp.data(), (size_t)n * sizeof(double))) != PIC_OK) return bail(rs);
      }
    }
    if (c->d.track_ids) {
      std::vector<int64_t> idv((size_t)n);
      for (int64_t j = 0; j < n; ++j) idv[j] = order[j];
      if ((rs = up(st.ids[c->cur], idv.data(), (size_t)n * sizeof(int64_t))) != PIC_OK) return bail(rs);
    }
    // the species' single density, read with stride 0 by kernels with per-particle densities
    const double wd = st.w;
    const float wf = (float)st.w;
    if ((rs = up(c->wconst64 + s, &wd, sizeof(double))) != PIC_OK) return bail(rs);
    if ((rs = up(c->wconst32 + s, &wf, sizeof(float))) != PIC_OK) return bail(rs);
    if ((rs = up(st.cs[c->cur], start.data(), ((size_t)nc + 1) * sizeof(int32_t))) != PIC_OK)
      return bail(rs);
  }
  if (pic::launch_iota(st.perm[c->cur], n, c->stream) != hipSuccess)
    return bail(fail(c, PIC_ERR_DEVICE, "identity permutation"));
  st.loaded = true;
  {
    const pic_status rt = retile(c);
    if (rt != PIC_OK) return rt;
  }
  HIP_TRY(c, hipMemsetAsync(c->flags, 0, sizeof(uint32_t), c->stream), "clear flags");
  pic::batch_touch(c);
  return redeposit(c);
}

pic_status pic_load_fields(pic_ctx *c, const double *e, const double *h) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  const size_t nn = (size_t)c->g.nnodes, nc = (size_t)c->g.ncells;
  if (e)
    for (size_t q = 0; q < 3 * nn; ++q)
      if (!std::isfinite(e[q])) return fail(c, PIC_ERR_RANGE, "non-finite E");
  if (h)
    for (size_t q = 0; q < 3 * nc; ++q)
      if (!std::isfinite(h[q])) return fail(c, PIC_ERR_RANGE, "non-finite H");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  if (e) HIP_TRY(c, copy_wait(c, c->E[c->ecur], e, 3 * nn * sizeof(double), hipMemcpyHostToDevice), "upload E");
  if (h) HIP_TRY(c, copy_wait(c, c->H[c->hcur], h, 3 * nc * sizeof(double), hipMemcpyHostToDevice), "upload H");
  HIP_TRY(c, hipMemsetAsync(c->flags, 0, sizeof(uint32_t), c->stream), "clear flags");
  pic::batch_touch(c);
  return redeposit(c);
}

pic_status pic_set_tiles(pic_ctx *c, int32_t tile_x, int32_t tile_z) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (tile_x < 0 || tile_z < 0 || tile_x > 64 || tile_z > 64 || ((tile_x == 0) != (tile_z == 0)))
    return fail(c, PIC_ERR_ARG, "tile_x, tile_z must both be 0 or both in 1..64");
  bool any = false;
  for (int s = 0; s < c->S; ++s) any = any || c->sp[s].loaded;
  if (!any) return fail(c, PIC_ERR_STATE, "no particles loaded");
  const int32_t ox = c->d.tile_x, oz = c->d.tile_z;
  c->d.tile_x = tile_x;
  c->d.tile_z = tile_z;
  pic_status st = retile(c);
  if (st != PIC_OK) {
    const std::string msg = c->err;
    c->d.tile_x = ox;
    c->d.tile_z = oz;
    (void)retile(c);
    c->err = msg;
    return st;
  }
  if ((st = alloc_tiles(c)) != PIC_OK) return st;
  if ((st = build_tile_list(c)) != PIC_OK) return st;
  pic::batch_touch(c);
  return PIC_OK;
}

pic_status pic_set_rank_mode(pic_ctx *c, int32_t mode) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (mode != PIC_RANK_AUTO && mode != PIC_RANK_ROWS && mode != PIC_RANK_CELLS)
    return fail(c, PIC_ERR_ARG, "mode must be PIC_RANK_AUTO, PIC_RANK_ROWS or PIC_RANK_CELLS");
  c->rank_mode = mode;
  pic::batch_touch(c);
  return PIC_OK;
}

pic_status pic_set_step(pic_ctx *c, int64_t step) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (step < 0) return fail(c, PIC_ERR_ARG, "step must be >= 0");
  c->step = step;
  pic::batch_touch(c);
  return PIC_OK;
}

pic_status pic_step(pic_ctx *c, int32_t nsteps) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (nsteps < 0) return fail(c, PIC_ERR_ARG, "nsteps must be >= 0");
  if (c->batch) return fail(c, PIC_ERR_STATE, "the context is stepped by a batch");
  bool any = false;
  for (int s = 0; s < c->S; ++s) any = any || c->sp[s].loaded;
  if (!any) return fail(c, PIC_ERR_STATE, "no particles loaded");
  for (int32_t it = 0; it < nsteps; ++it) {
    ProfEvents *pe = nullptr;
    if (c->prof_on && (c->prof_count++ % c->prof_every) == 0) {
      if (c->prof_used == c->prof_ev.size()) {
        if (c->prof_ev.size() >= 4096) {
          HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
          prof_accumulate(c);
        } else {
          ProfEvents p{};
          for (int q = 0; q < 4; ++q) HIP_TRY(c, hipEventCreate(&p.ev[q]), "event create");
          c->prof_ev.push_back(p);
        }
      }
      pe = &c->prof_ev[c->prof_used++];
      HIP_TRY(c, hipEventRecord(pe->ev[0], c->stream), "event record");
    }
    const pic::FieldArgs fa = pic::cycle_field_args(c, c->cur);
    HIP_TRY(c, pic::launch_field_solve(fa, c->stream), "field solve");
    if (pe) HIP_TRY(c, hipEventRecord(pe->ev[1], c->stream), "event record");
    const pic::StepArgs a = pic::cycle_step_args(c, c->cur);
    pic_status ps = particle_stage(c, a);
    if (ps != PIC_OK) return ps;
    if (pe) HIP_TRY(c, hipEventRecord(pe->ev[2], c->stream), "event record");
    HIP_TRY(c, pic::launch_sort(a, c->stream), "sort kernels");
    if (pe) HIP_TRY(c, hipEventRecord(pe->ev[3], c->stream), "event record");
    c->ecur ^= 1;
    c->hcur ^= 1;
    c->cur ^= 1;
    c->step += 1;
  }
  return PIC_OK;
}

pic_status pic_read_moments(pic_ctx *c, double *out, int64_t len) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  const int64_t need = (int64_t)c->g.n_planes * c->g.nnodes;
  if (!out || len < need) return fail(c, PIC_ERR_ARG, "output buffer too small");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  HIP_TRY(c, copy_wait(c, out, c->M, (size_t)need * sizeof(double), hipMemcpyDeviceToHost), "read moments");
  return PIC_OK;
}

pic_status pic_read_fields(pic_ctx *c, double *e, double *h) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  if (e) HIP_TRY(c, copy_wait(c, e, c->E[c->ecur], 3 * (size_t)c->g.nnodes * sizeof(double), hipMemcpyDeviceToHost), "read E");
  if (h) HIP_TRY(c, copy_wait(c, h, c->H[c->hcur], 3 * (size_t)c->g.ncells * sizeof(double), hipMemcpyDeviceToHost), "read H");
  return PIC_OK;
}

static pic_status alive_count(pic_ctx *c, int s, int64_t *n) {
  *n = 0;
  if (!c->sp[s].loaded) return PIC_OK;
  int32_t v = 0;
  HIP_TRY(c, copy_wait(c, &v, c->sp[s].cs[c->cur] + c->g.ncells, sizeof(int32_t), hipMemcpyDeviceToHost),
          "read count");
  *n = v;
  return PIC_OK;
}

pic_status pic_read_particles(pic_ctx *c, int32_t s, int64_t *n_inout, double *xi_x, double *xi_z,
                              double *ux, double *uy, double *uz, double *w, int64_t *id) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (s < 0 || s >= c->S || !n_inout) return fail(c, PIC_ERR_ARG, "bad species or n_inout");
  if (id && !c->d.track_ids) return fail(c, PIC_ERR_ARG, "ids need track_ids");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  int64_t n = 0;
  pic_status rs = alive_count(c, s, &n);
  if (rs != PIC_OK) return rs;
  if (*n_inout < n) {
    *n_inout = n;
    return fail(c, PIC_ERR_ARG, "particle arrays too small");
  }
  *n_inout = n;
  if (n == 0) return PIC_OK;
  SpeciesState &st = c->sp[s];
  std::vector<int32_t> perm((size_t)n);
  HIP_TRY(c, copy_wait(c, perm.data(), st.perm[c->cur], (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost),
          "read perm");
  double *outs[5] = {xi_x, xi_z, ux, uy, uz};
  if (mixed(c)) {
    // positions come back as cell index + offset, exact in FP64
    std::vector<int32_t> kc((size_t)st.cap);
    std::vector<float> tmp((size_t)st.cap);
    HIP_TRY(c, copy_wait(c, kc.data(), st.mcell[c->cur], (size_t)st.cap * sizeof(int32_t), hipMemcpyDeviceToHost),
            "read particles");
    for (int v = 0; v < 5; ++v) {
      if (!outs[v]) continue;
      HIP_TRY(c, copy_wait(c, tmp.data(), st.mbuf[c->cur][v], (size_t)st.cap * sizeof(float), hipMemcpyDeviceToHost),
              "read particles");
      for (int64_t j = 0; j < n; ++j) {
        const int32_t loc = perm[j];
        double val = (double)tmp[loc];
        if (v == 0) val += (double)(kc[loc] % c->g.nx);
        if (v == 1) val += (double)(kc[loc] / c->g.nx);
        outs[v][j] = val;
      }
    }
  } else {
    std::vector<double> tmp((size_t)st.cap);
    for (int v = 0; v < 5; ++v) {
      if (!outs[v]) continue;
      HIP_TRY(c, copy_wait(c, tmp.data(), st.buf[c->cur][v], (size_t)st.cap * sizeof(double), hipMemcpyDeviceToHost),
              "read particles");
      for (int64_t j = 0; j < n; ++j) outs[v][j] = tmp[perm[j]];
    }
  }
  if (w) {
    if (!st.pw) {
      std::fill(w, w + n, st.w);
    } else if (mixed(c)) {
      std::vector<float> tw((size_t)st.cap);
      HIP_TRY(c, copy_wait(c, tw.data(), st.mwbuf[c->cur], (size_t)st.cap * sizeof(float), hipMemcpyDeviceToHost),
              "read densities");
      for (int64_t j = 0; j < n; ++j) w[j] = (double)tw[perm[j]];
    } else {
      std::vector<double> tw((size_t)st.cap);
      HIP_TRY(c, copy_wait(c, tw.data(), st.wbuf[c->cur], (size_t)st.cap * sizeof(double), hipMemcpyDeviceToHost),
              "read densities");
      for (int64_t j = 0; j < n; ++j) w[j] = tw[perm[j]];
    }
  }
  if (id) {
    std::vector<int64_t> t2((size_t)st.cap);
    HIP_TRY(c, copy_wait(c, t2.data(), st.ids[c->cur], (size_t)st.cap * sizeof(int64_t), hipMemcpyDeviceToHost),
            "read ids");
    for (int64_t j = 0; j < n; ++j) id[j] = t2[perm[j]];
  }
  return PIC_OK;
}

pic_status pic_get_info(pic_ctx *c, pic_info *info) {
  if (!c || !info) return fail(c, PIC_ERR_ARG, "NULL argument");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  pic_info r{};
  r.step = c->step;
  r.t = (double)c->step * c->g.dt;
  r.n_species = c->S;
  r.nodes_x = c->g.nxn;
  r.nodes_z = c->g.nzn;
  r.cells_x = c->g.nx;
  r.cells_z = c->g.nz;
  r.tile_x = c->tiles.tx;
  r.tile_z = c->tiles.tz;
  r.precision = c->d.precision;
  for (int s = 0; s < c->S; ++s) {
    int64_t n = 0;
    pic_status rs = alive_count(c, s, &n);
    if (rs != PIC_OK) return rs;
    r.alive[s] = n;
    r.absorbed[s] = c->sp[s].loaded ? c->sp[s].n_loaded - n : 0;
  }
  HIP_TRY(c, copy_wait(c, &r.overflow_flags, c->flags, sizeof(uint32_t), hipMemcpyDeviceToHost), "read flags");
  r.rank_mode = rank_cells(c) ? PIC_RANK_CELLS : PIC_RANK_ROWS;
  r.device_bytes = c->mem.bytes;
  *info = r;
  return PIC_OK;
}

pic_status pic_set_stream(pic_ctx *c, void *stream) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (c->batch) return fail(c, PIC_ERR_STATE, "the context runs on its batch's stream");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  c->stream = stream ? static_cast<hipStream_t>(stream) : c->own_stream;
  return PIC_OK;
}

pic_status pic_sync(pic_ctx *c) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  return PIC_OK;
}

pic_status pic_profile_enable(pic_ctx *c, int32_t on) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (on < 0) return fail(c, PIC_ERR_ARG, "on must be >= 0");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  if (on) {
    c->prof_used = 0;
    c->prof_acc = pic_profile{};
    c->prof_on = true;
    c->prof_every = on;
    c->prof_count = 0;
  } else {
    prof_accumulate(c);
    c->prof_on = false;
  }
  return PIC_OK;
}

pic_status pic_profile_read(pic_ctx *c, pic_profile *out) {
  if (!c || !out) return fail(c, PIC_ERR_ARG, "NULL argument");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  prof_accumulate(c);
  *out = c->prof_acc;
  return PIC_OK;
}

pic_status pic_set_mover(pic_ctx *c, int32_t options) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (options & ~(PIC_MOVER_GAMMA_PREDICT | PIC_MOVER_B_BILINEAR))
    return fail(c, PIC_ERR_ARG, "unknown mover option bits");
  if (options && mixed(c)) return fail(c, PIC_ERR_ARG, "mover options are for FP64 contexts only");
  if (c->batch) return fail(c, PIC_ERR_STATE, "the context is stepped by a batch");
  c->mover = options;
  return redeposit(c);
}

pic_status pic_energy(pic_ctx *c, double *out, int32_t len) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (!out || len < 1 + c->S) return fail(c, PIC_ERR_ARG, "out must hold 1 + n_species values");
  double *d = nullptr;
  pic_status st = dalloc(c, &d, (size_t)1 + c->S, "alloc energy");
  if (st != PIC_OK) return st;
  pic::StepArgs a = step_args(c, false);
  hipError_t e = hipMemsetAsync(d, 0, (1 + (size_t)c->S) * sizeof(double), c->stream);
  if (e == hipSuccess) e = pic::launch_energy(a, c->E[c->ecur], c->H[c->hcur], d, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = copy_wait(c, out, d, (1 + (size_t)c->S) * sizeof(double), hipMemcpyDeviceToHost);
  dfree(c, d, (1 + (size_t)c->S) * sizeof(double));
  if (e != hipSuccess) return hip_fail(c, e, "energy");
  return PIC_OK;
}

pic_status pic_set_allocator(pic_alloc_fn alloc, pic_free_fn free_fn, void *user) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(nullptr, PIC_ERR_ARG, "alloc and free must both be given or both be NULL");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = alloc;
  g_free = free_fn;
  g_alloc_user = alloc ? user : nullptr;
  return PIC_OK;
}

pic_status pic_energy_noalloc(pic_ctx *c, double *out, int32_t len) {
  if (!c) return fail(nullptr, PIC_ERR_ARG, "ctx is NULL");
  if (!out || len < 1 + c->S) return fail(c, PIC_ERR_ARG, "out must hold 1 + n_species values");
  if (1 + c->S > pic::kEnergyVals)
    return fail(c, PIC_ERR_ARG, "more species than the fixed energy buffer holds");
  double *buf = nullptr;
  HIP_TRY(c, pic::energy_scratch(c->d.device, &buf), "energy buffer address");
  const pic::StepArgs a = step_args(c, false);
  HIP_TRY(c, pic::launch_energy_scratch(a, c->E[c->ecur], c->H[c->hcur], buf, c->stream), "energy");
  HIP_TRY(c, hipMemcpyAsync(out, buf + (size_t)pic::kEnergyBlocks * pic::kEnergyVals,
                            (1 + (size_t)c->S) * sizeof(double), hipMemcpyDeviceToHost, c->stream),
          "read energy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  return PIC_OK;
}

const char *pic_last_error(const pic_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void pic_destroy(pic_ctx *c) {
  if (!c) return;
  pic::batch_detach(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int s = 0; s < PIC_MAX_SPECIES; ++s) free_species(c, c->sp[s]);
  const size_t nn = (size_t)c->g.nnodes, nc = (size_t)c->g.ncells;
  for (int b = 0; b < 2; ++b) {
    dfree(c, c->E[b], 3 * nn * sizeof(double));
    dfree(c, c->H[b], 3 * nc * sizeof(double));
  }
  dfree(c, c->M, (size_t)c->g.n_planes * nn * sizeof(double));
  dfree(c, c->flags, sizeof(uint32_t));
  dfree(c, c->wconst64, 12 * sizeof(double));
  for (int b = 0; b < 2; ++b) {
    dfree(c, c->tact[b], (size_t)std::max(c->tiles_alloc, 1));
    dfree(c, c->tlist[b], ((size_t)c->tiles_alloc + 1) * sizeof(int32_t));
  }
  dfree(c, c->mflag, (size_t)(c->g.nnodes + pic::kFlagNodes - 1) / pic::kFlagNodes);
  c->mem.put_all();
  for (auto &p : c->prof_ev)
    for (int q = 0; q < 4; ++q) (void)hipEventDestroy(p.ev[q]);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

}  // extern "C"
