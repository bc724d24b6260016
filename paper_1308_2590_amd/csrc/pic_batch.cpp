// Host side of the batch API declared in include/pic.h: many independent runs stepped with one
// launch of each kernel per cycle.  The batch keeps, in device memory, the step and field
// arguments of every member for both buffer parities, each member's current parity and cycle
// count, and the prefix sums over members of each kernel's work items.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_ctx.h"
#include "pic_internal.h"

struct pic_batch {
  int32_t device = 0;
  int32_t precision = PIC_PREC_FP64;
  hipStream_t stream = nullptr;
  std::vector<pic_ctx *> runs;
  // device tables (capacity cap runs)
  size_t cap = 0;
  pic::StepArgs *d_step = nullptr;   // [2 cap]
  pic::FieldArgs *d_field = nullptr; // [2 cap]
  int32_t *d_par = nullptr;          // [cap]
  int64_t *d_ctr = nullptr;          // [cap]
  int32_t *d_pre = nullptr;          // [6][cap + 1]
  pic::BatchArgs args{};
  pic::BatchLaunch launch{};
  bool dirty = true;
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string err;
  pic::DevAlloc mem;  // device memory of the tables (hipMalloc or the allocator hook)
};

namespace {

thread_local std::string g_batch_error;

pic_status bfail(pic_batch *b, pic_status st, const std::string &msg) {
  if (b)
    b->err = msg;
  else
    g_batch_error = msg;
  return st;
}

pic_status bhip(pic_batch *b, hipError_t e, const char *what) {
  return bfail(b, e == hipErrorOutOfMemory ? PIC_ERR_OOM : PIC_ERR_DEVICE,
               std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIP(b, expr, what)                         \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return bhip(b, e_, what); \
  } while (0)

void drop_graph(pic_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

void free_tables(pic_batch *b) {
  b->mem.put(b->d_step);
  b->mem.put(b->d_field);
  b->mem.put(b->d_par);
  b->mem.put(b->d_ctr);
  b->mem.put(b->d_pre);
  b->d_step = nullptr;
  b->d_field = nullptr;
  b->d_par = nullptr;
  b->d_ctr = nullptr;
  b->d_pre = nullptr;
  b->cap = 0;
}

pic_status grow(pic_batch *b, size_t n) {
  if (n <= b->cap) return PIC_OK;
  size_t cap = std::max<size_t>(n, 2 * b->cap);
  free_tables(b);
  BHIP(b, b->mem.get((void **)&b->d_step, 2 * cap * sizeof(pic::StepArgs)), "batch tables");
  BHIP(b, b->mem.get((void **)&b->d_field, 2 * cap * sizeof(pic::FieldArgs)), "batch tables");
  BHIP(b, b->mem.get((void **)&b->d_par, cap * sizeof(int32_t)), "batch tables");
  BHIP(b, b->mem.get((void **)&b->d_ctr, cap * sizeof(int64_t)), "batch tables");
  BHIP(b, b->mem.get((void **)&b->d_pre, 6 * (cap + 1) * sizeof(int32_t)), "batch tables");
  b->cap = cap;
  return PIC_OK;
}

// Rebuild the device tables and the launch configuration from the members' current state.
pic_status rebuild(pic_batch *b) {
  drop_graph(b);
  const size_t n = b->runs.size();
  pic_status st = grow(b, std::max<size_t>(n, 1));
  if (st != PIC_OK) return st;
  std::vector<pic::StepArgs> steps(2 * n);
  std::vector<pic::FieldArgs> fields(2 * n);
  std::vector<int32_t> par(n);
  std::vector<int64_t> ctr(n);
  std::vector<int32_t> pre(6 * (n + 1), 0);
  size_t lds_p = 0, lds_r = 0;
  bool ids = false, pw = false;
  for (size_t r = 0; r < n; ++r) {
    pic_ctx *c = b->runs[r];
    ids = ids || c->d.track_ids != 0;
    for (int q = 0; q < c->S; ++q) pw = pw || (c->sp[q].loaded && c->sp[q].pw);
  }
  for (size_t r = 0; r < n; ++r) {
    pic_ctx *c = b->runs[r];
    for (int p = 0; p < 2; ++p) {
      steps[2 * r + p] = pic::cycle_step_args(c, p);
      fields[2 * r + p] = pic::cycle_field_args(c, p);
      // the batched cycle clears the next order's tile flags in the H update
      fields[2 * r + p].tact_next = c->tact[1 - p];
    }
    par[r] = c->cur;
    ctr[r] = c->step;
    const pic::GridArgs &g = c->g;
    const int32_t items[4] = {
        (int32_t)((g.nnodes + pic::kSolveNodes * pic::kBlock - 1) / (pic::kSolveNodes * pic::kBlock)),
        (int32_t)((g.ncells + pic::kHCells * pic::kBlock - 1) / (pic::kHCells * pic::kBlock)),
        c->n_scan1_blocks * c->S,
        1};
    for (int k = 0; k < 4; ++k) pre[k * (n + 1) + r + 1] = pre[k * (n + 1) + r] + items[k];
    lds_p = std::max(lds_p, pic::particle_lds_bytes(c->g, c->tiles, b->precision == PIC_PREC_MIXED, pw));
    lds_r = std::max(lds_r, pic::rank_lds_bytes(c->tiles));
  }
  if (n > 0) {
    // on the batch's stream (not the null stream: see the context's copies), then wait, since
    // the host tables go out of scope
    auto up = [&](void *dst, const void *src, size_t bytes) {
      return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream);
    };
    BHIP(b, up(b->d_step, steps.data(), steps.size() * sizeof(pic::StepArgs)), "upload batch tables");
    BHIP(b, up(b->d_field, fields.data(), fields.size() * sizeof(pic::FieldArgs)), "upload batch tables");
    BHIP(b, up(b->d_par, par.data(), n * sizeof(int32_t)), "upload batch tables");
    BHIP(b, up(b->d_ctr, ctr.data(), n * sizeof(int64_t)), "upload batch tables");
    BHIP(b, up(b->d_pre, pre.data(), pre.size() * sizeof(int32_t)), "upload batch tables");
    BHIP(b, hipStreamSynchronize(b->stream), "upload batch tables");
  }
  pic::BatchArgs &a = b->args;
  a.step = b->d_step;
  a.field = b->d_field;
  a.par = b->d_par;
  a.step_ctr = b->d_ctr;
  a.nruns = (int32_t)n;
  const size_t stride = n + 1;
  a.pre_nodes = b->d_pre + 0 * stride;
  a.pre_cells = b->d_pre + 1 * stride;
  a.pre_scan = b->d_pre + 2 * stride;
  a.pre_one = b->d_pre + 3 * stride;
  a.pre_tiles = b->d_pre + 4 * stride;
  a.pre_rank = b->d_pre + 5 * stride;
  pic::BatchLaunch &l = b->launch;
  l.mixed = b->precision == PIC_PREC_MIXED;
  l.ids = ids;
  l.pw = pw;
  l.lds_particles = lds_p;
  l.lds_rank = lds_r;
  // one block per tile that any run could have active (the blocks past the cycle's active
  // tiles return at once)
  int64_t tiles_max = 0, rank_max = 0;
  for (size_t r = 0; r < n; ++r) {
    tiles_max += b->runs[r]->tiles.ntiles;
    rank_max += (int64_t)b->runs[r]->tiles.ntiles * b->runs[r]->S;
  }
  l.grid_particles = (int32_t)std::max<int64_t>(1, tiles_max);
  l.grid_rank = (int32_t)std::max<int64_t>(1, rank_max);
  l.items_nodes = n > 0 ? pre[0 * (n + 1) + n] : 0;
  l.items_cells = n > 0 ? pre[1 * (n + 1) + n] : 0;
  l.items_scan = n > 0 ? pre[2 * (n + 1) + n] : 0;
  b->dirty = false;
  return PIC_OK;
}

pic_status capture(pic_batch *b) {
  drop_graph(b);
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "graph capture");
  hipError_t le = pic::launch_batch_cycle(b->args, b->launch, b->stream);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(b->stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bhip(b, le, "graph capture");
  }
  if (ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bhip(b, ee, "graph capture");
  }
  b->graph = g;
  BHIP(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0), "graph instantiate");
  return PIC_OK;
}

}  // namespace

namespace pic {

void batch_touch(pic_ctx *c) {
  if (c && c->batch) c->batch->dirty = true;
}

void batch_detach(pic_ctx *c) {
  if (c && c->batch) (void)pic_batch_remove(c->batch, c);
}

}  // namespace pic

extern "C" {

pic_status pic_batch_create(int32_t device, int32_t precision, pic_batch **out) {
  if (!out) return bfail(nullptr, PIC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (precision != PIC_PREC_FP64 && precision != PIC_PREC_MIXED)
    return bfail(nullptr, PIC_ERR_ARG, "precision must be PIC_PREC_FP64 or PIC_PREC_MIXED");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return bfail(nullptr, PIC_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return bfail(nullptr, PIC_ERR_ARG, "device ordinal out of range");
  if (hipSetDevice(device) != hipSuccess) return bfail(nullptr, PIC_ERR_DEVICE, "hipSetDevice failed");
  pic_batch *b = new pic_batch();
  b->device = device;
  b->precision = precision;
  b->mem = pic::current_allocator(device);
  hipDeviceProp_t prop;  // checks the device ordinal
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    g_batch_error = std::string("batch set-up: ") + hipGetErrorString(e);
    delete b;
    return PIC_ERR_DEVICE;
  }
  *out = b;
  return PIC_OK;
}

pic_status pic_batch_add(pic_batch *b, pic_ctx *c) {
  if (!b) return bfail(nullptr, PIC_ERR_ARG, "batch is NULL");
  if (!c) return bfail(b, PIC_ERR_ARG, "ctx is NULL");
  if (c->batch) return bfail(b, PIC_ERR_ARG, "the context is already in a batch");
  if (c->d.device != b->device) return bfail(b, PIC_ERR_ARG, "the context is on another device");
  if (c->d.precision != b->precision) return bfail(b, PIC_ERR_ARG, "the context has another precision");
  if (c->mover != 0) return bfail(b, PIC_ERR_ARG, "contexts with mover options are not batched");
  bool any = false;
  for (int s = 0; s < c->S; ++s) any = any || c->sp[s].loaded;
  if (!any) return bfail(b, PIC_ERR_ARG, "the context has no particles");
  // the context's queued work must finish before the batch's stream takes over
  BHIP(b, hipStreamSynchronize(c->stream), "sync");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  c->stream_before_batch = c->stream;
  c->stream = b->stream;
  c->batch = b;
  b->runs.push_back(c);
  b->dirty = true;
  return PIC_OK;
}

pic_status pic_batch_remove(pic_batch *b, pic_ctx *c) {
  if (!b) return bfail(nullptr, PIC_ERR_ARG, "batch is NULL");
  auto it = std::find(b->runs.begin(), b->runs.end(), c);
  if (!c || it == b->runs.end()) return bfail(b, PIC_ERR_ARG, "the context is not in this batch");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  b->runs.erase(it);
  c->stream = c->stream_before_batch ? c->stream_before_batch : c->own_stream;
  c->stream_before_batch = nullptr;
  c->batch = nullptr;
  b->dirty = true;
  return PIC_OK;
}

pic_status pic_batch_step(pic_batch *b, int32_t nsteps) {
  if (!b) return bfail(nullptr, PIC_ERR_ARG, "batch is NULL");
  if (nsteps < 0) return bfail(b, PIC_ERR_ARG, "nsteps must be >= 0");
  if (b->runs.empty() || nsteps == 0) return PIC_OK;
  BHIP(b, hipSetDevice(b->device), "hipSetDevice");
  if (b->dirty) {
    // the tables are read by queued cycles: wait before rewriting them
    BHIP(b, hipStreamSynchronize(b->stream), "sync");
    pic_status st = rebuild(b);
    if (st != PIC_OK) return st;
  }
  if (b->use_graph && !b->gexec) {
    pic_status st = capture(b);
    if (st != PIC_OK) return st;
  }
  for (int32_t it = 0; it < nsteps; ++it) {
    if (b->gexec) {
      BHIP(b, hipGraphLaunch(b->gexec, b->stream), "graph launch");
    } else {
      BHIP(b, pic::launch_batch_cycle(b->args, b->launch, b->stream), "batch cycle");
    }
  }
  // the host view of every member follows the device counters
  for (pic_ctx *c : b->runs) {
    if (nsteps & 1) {
      c->cur ^= 1;
      c->ecur ^= 1;
      c->hcur ^= 1;
    }
    c->step += nsteps;
  }
  return PIC_OK;
}

pic_status pic_batch_set_graph(pic_batch *b, int32_t on) {
  if (!b) return bfail(nullptr, PIC_ERR_ARG, "batch is NULL");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  b->use_graph = on != 0;
  drop_graph(b);
  return PIC_OK;
}

pic_status pic_batch_sync(pic_batch *b) {
  if (!b) return bfail(nullptr, PIC_ERR_ARG, "batch is NULL");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  return PIC_OK;
}

pic_status pic_batch_size(const pic_batch *b, int32_t *n) {
  if (!b || !n) return bfail(nullptr, PIC_ERR_ARG, "NULL argument");
  *n = (int32_t)b->runs.size();
  return PIC_OK;
}

const char *pic_batch_last_error(const pic_batch *b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

void pic_batch_destroy(pic_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  while (!b->runs.empty()) (void)pic_batch_remove(b, b->runs.back());
  drop_graph(b);
  free_tables(b);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
