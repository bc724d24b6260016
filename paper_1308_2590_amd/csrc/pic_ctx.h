// Private: the context structure shared by the host files of the library (pic_capi.cpp and
// pic_batch.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <unordered_map>
#include <vector>

#include "pic.h"
#include "pic_internal.h"

namespace pic {

// Device memory of a context or batch: hipMalloc / hipFree, or the allocator hook installed by
// pic_set_allocator when the context or batch was created.  Every block's size is recorded so
// the hook's free gets the size it allocated.
struct DevAlloc {
  pic_alloc_fn alloc = nullptr;
  pic_free_fn free = nullptr;
  void *user = nullptr;
  int32_t device = 0;
  std::unordered_map<void *, size_t> live;
  int64_t bytes = 0;
  // hipErrorOutOfMemory when the hook returns NULL
  hipError_t get(void **p, size_t bytes);
  void put(void *p);
  void put_all();
};
// The hook pair installed at this moment (empty for hipMalloc / hipFree).
DevAlloc current_allocator(int32_t device);

struct SpeciesState {
  bool loaded = false;
  bool pw = false;         // per-particle densities (wbuf / mwbuf); otherwise w for all
  double q = 0, m = 1, w = 0;
  int64_t cap = 0;         // slots allocated
  int64_t n_loaded = 0;    // particles given at the last load
  double *buf[2][5] = {};  // FP64 form: two copies of the state; perm maps sorted slot -> location
  int32_t *mcell[2] = {};  // mixed form: cell key k * nx + i
  float *mbuf[2][5] = {};  // mixed form: in-cell offsets f_x, f_z and u_x, u_y, u_z
  int64_t *ids[2] = {};
  double *wbuf[2] = {};    // per-particle densities, FP64 form (addressed like buf)
  float *mwbuf[2] = {};    // the same, mixed form (FP32)
  int32_t *perm[2] = {};
  int32_t *cs[2] = {};     // cell start offsets [ncells + 1]
  uint32_t *locode = nullptr;
  int32_t *cnt = nullptr;  // [9][ncells]
  uint16_t *cmask = nullptr;  // [ncells] move codes used per cell (with the per-cell ranker)
  int32_t *arr = nullptr;  // [ncells] arrivals per cell, zero between cycles
  int32_t *bsum = nullptr;
};

struct ProfEvents {
  hipEvent_t ev[4];  // step start, after field solve, after particles, after sort
};


}  // namespace pic

struct pic_ctx {
  pic_grid_desc d{};
  pic::GridArgs g{};
  pic::LaserArgs laser{};
  pic::TileArgs tiles{};
  int S = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  double *E[2] = {}, *H[2] = {}, *M = nullptr;
  int ecur = 0, hcur = 0, cur = 0;  // flip together every cycle
  pic::SpeciesState sp[PIC_MAX_SPECIES];
  uint32_t *flags = nullptr;
  // each species' single density (kernels with per-particle densities read it with stride 0
  // for species loaded without per-particle values): FP64 at [0, 8), FP32 at wconst32
  double *wconst64 = nullptr;
  float *wconst32 = nullptr;
  pic::DevAlloc mem;       // device memory of the context
  uint8_t *tact[2] = {};   // active-tile flags of the current / next order
  int32_t *tlist[2] = {};  // ordered active-tile lists, count at [ntiles]
  uint8_t *mflag = nullptr;  // deposit flags, one per kFlagNodes nodes (moments can be nonzero)
  int32_t tiles_alloc = 0, tiles_tx = 0, tiles_tz = 0;
  int64_t step = 0;
  size_t lds_max = 65536;  // LDS a block may use on the context's device
  int32_t mover = 0;       // PIC_MOVER_* options; 0: the tile kernel's default mover
  int32_t rank_mode = PIC_RANK_AUTO;
  bool rank_cells_auto = false;  // the automatic choice, made with the tile shape
  bool chunk2 = false;           // particle kernel chunk of 2 (about 2 particles per lane and row)
  int32_t n_scan_blocks = 0;
  int32_t n_scan1_blocks = 0;  // blocks of the scan of a cycle's sort
  std::string err;
  // profiling
  bool prof_on = false;
  int32_t prof_every = 1;  // time every prof_every-th cycle
  int64_t prof_count = 0;  // cycles since profiling started
  std::vector<pic::ProfEvents> prof_ev;
  size_t prof_used = 0;
  pic_profile prof_acc{};
  // batch membership: a context in a batch is stepped by it, on the batch's stream
  pic_batch *batch = nullptr;
  hipStream_t stream_before_batch = nullptr;
};

namespace pic {

// Step arguments of a context for buffer parity p (p = the current copy), as pic_step builds
// them for a cycle, and the field-solve arguments of the same cycle.
StepArgs cycle_step_args(pic_ctx *c, int p);
FieldArgs cycle_field_args(pic_ctx *c, int p);
// Mark the batch holding c (if any) for a rebuild of its tables.
void batch_touch(pic_ctx *c);
// Remove c from its batch (if any); used by pic_destroy.
void batch_detach(pic_ctx *c);

}  // namespace pic
