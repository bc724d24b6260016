/*
 * pic.h -- C ABI of the MI355X (gfx950) implicit 2D3V particle-in-cell particle stage.
 *
 * The library implements one cycle of the implicit PIC method of Petrov & Davis
 * ("Parallelization of an implicit algorithm for multi-dimensional particle-in-cell
 * simulations"), Sec. 2 and Sec. 3.3, on one GPU:
 *   field solve   Eq. (4) per node with the x-boundary conditions and the x = 0 source
 *                 (Steps 3-6), E-bar = (E^n + E^{n+1})/2, then Eq. (5) (Steps 8-9);
 *   particles     gather E-bar and B, implicit relativistic push (Eq. (2) solved for the
 *                 momentum, particles pushed once per cycle), position advance, and the
 *                 deposit of the implicit source moments S-hat and delta-j of Eq. (3)
 *                 (Step 1) plus the species densities, at the new positions;
 *   sort          stable sort of every species by cell, dropping particles that left an
 *                 absorbing boundary (the one-GPU counterpart of moving particles to the
 *                 processor that owns them, Sec. 3.1 and the end of Sec. 3.3).
 *
 * Conventions shared by every call:
 *   - the simulation plane is (x, z) with d/dy = 0 and three momentum components;
 *   - units c = eps0 = mu0 = 1 (so B = H); time in 1/omega_r, length in c/omega_r,
 *     momentum u = p/(m c), charge in e, mass in m_e;
 *   - positions are in cell units: cell (i, k) covers [i, i+1) x [k, k+1);
 *   - E lives on grid nodes and H at cell centres (Sec. 2, last paragraph; Sec. 3.2 (3));
 *     a periodic axis with N cells has N nodes (node N is node 0), an absorbing axis N + 1;
 *   - every 2D array is stored with x fastest: node (i, k) at k * nodes_x + i, cell (i, k)
 *     at k * nx + i;
 *   - moment planes (Step 1 and Fig. 1: S-hat and delta-j on the nodes), each one node
 *     array: 0..8 S-hat row-major (S_xx S_xy S_xz S_yx ... S_zz), 9..11 delta-j,
 *     12 + s density of species s;
 *   - state after k cycles: positions x^{k+1/2}, momenta u^k, E^k, H^{k+1/2}, t = k dt.
 *
 * Precision.  PIC_PREC_FP64 holds and pushes particles in FP64.  PIC_PREC_MIXED stores each
 * particle as an int32 cell key (k * nx + i), FP32 offsets within the cell in [0, 1) and FP32
 * momenta; the gather, the push and each particle's moments are computed in FP32, and a
 * lane's FP32 partial sums are added into FP64 accumulators and the FP64 moment planes.  The
 * field solve, E, E-bar, H and the moments stay FP64 in both forms.  Loading rounds offsets
 * and momenta to FP32 (an offset that would round to 1 becomes the largest float below 1);
 * positions read back as i + offset, exactly.  An offset carried past a face by the push
 * moves the particle to the neighbouring cell (offset minus one), and one that rounds to 1
 * becomes offset 0 of the next cell, so every particle's cell and offset stay consistent.
 *
 * Ownership: every pointer argument is a HOST pointer owned by the caller; the library
 * copies from or into it during the call and keeps nothing.  The context owns all device
 * memory.  Every call returns a pic_status; on failure pic_last_error() gives a message and
 * the context state is unchanged unless stated.  One context must not be used from two host
 * threads at once; separate contexts are independent.
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
  PIC_OK = 0,
  PIC_ERR_ARG = 1,      /* invalid argument or descriptor (includes dt > min(dx, dz)) */
  PIC_ERR_OOM = 2,      /* device allocation failed */
  PIC_ERR_DEVICE = 3,   /* a HIP call failed */
  PIC_ERR_STATE = 4,    /* call out of order (e.g. step before any particles were loaded) */
  PIC_ERR_RANGE = 5,    /* particle position outside the domain or non-finite input */
  PIC_ERR_OVERFLOW = 6  /* the device raised an overflow flag during a step (see pic_info) */
} pic_status;

enum { PIC_BC_PERIODIC = 0, PIC_BC_ABSORBING = 1 };
enum { PIC_PREC_FP64 = 0, PIC_PREC_MIXED = 1 };
/* How the cell sort finds each particle's slot in the next order (pic_set_rank_mode). */
enum { PIC_RANK_AUTO = 0, PIC_RANK_ROWS = 1, PIC_RANK_CELLS = 2 };

/* Mover options (bits of pic_set_mover's argument), two readings of what the paper leaves
 * open, for comparing their energy behaviour:
 *   PIC_MOVER_GAMMA_PREDICT  the Lorentz factor inside the linearised mover is
 *                            gamma(u^n + beta E^n), E^n interpolated at the particle (a
 *                            Boris-style predictor), instead of gamma(u^n);
 *   PIC_MOVER_B_BILINEAR     B at the particle is interpolated bilinearly from the four
 *                            surrounding cell centres (the edge cell repeated beyond an
 *                            absorbing x boundary), instead of its own cell's H. */
enum { PIC_MOVER_GAMMA_PREDICT = 1, PIC_MOVER_B_BILINEAR = 2 };
enum { PIC_MAX_SPECIES = 8 };

/* Device overflow flags reported in pic_info.overflow_flags. */
enum {
  PIC_FLAG_ORDER = 1u,      /* a particle was not in the cell its sorted slot says */
  PIC_FLAG_NONFINITE = 2u,  /* a pushed momentum or position was not finite */
  PIC_FLAG_JUMP = 4u,       /* a particle moved by more than one cell in one cycle */
  PIC_FLAG_SLOT = 8u        /* a sort destination fell outside the particle array */
};

typedef struct {
  int32_t nx, nz;            /* cells along x and z, each in 1 .. 2^22 - 1, nx nz < 2^31 - 1 */
  double dx, dz, dt;         /* cell sizes and time step; dt <= min(dx, dz) is required */
  int32_t bc_x, bc_z;        /* PIC_BC_*; bc_z must be PIC_BC_PERIODIC */
  int32_t precision;         /* PIC_PREC_FP64 or PIC_PREC_MIXED (see below) */
  int32_t n_species;         /* number of species slots S, 1..PIC_MAX_SPECIES */
  double e0[3], h0[3];       /* uniform initial E (nodes) and H (cell centres) */
  /* E_y source at x = 0 (absorbing x only; a0 = 0 switches it off):
   *   a0 sin(omega (t - x)) exp(-(z - z_center)^2 / (2 sigma_z^2))
   *      exp(-2 ln 2 ((t - x - t_center) / fwhm_t)^2)                                  */
  double laser_a0, laser_omega, laser_sigma_z, laser_z_center, laser_fwhm_t, laser_t_center;
  int32_t allow_cfl_violation; /* must be 0: the cell sort relies on moves of < 1 cell */
  int32_t track_ids;         /* 1: carry a 64-bit label per particle through every sort */
  int32_t tile_x, tile_z;    /* cells per particle tile; 0 picks them from the load */
  int32_t device;            /* HIP device ordinal */
  int32_t reserved[7];       /* must be zero */
} pic_grid_desc;

typedef struct {
  int64_t step;              /* cycles done */
  double t;                  /* step * dt */
  int32_t n_species, nodes_x, nodes_z, cells_x, cells_z;
  int32_t tile_x, tile_z, precision;
  int64_t alive[PIC_MAX_SPECIES];     /* particles held per species */
  int64_t absorbed[PIC_MAX_SPECIES];  /* particles removed at absorbing boundaries */
  uint32_t overflow_flags;   /* PIC_FLAG_* raised since the last pic_load_* call */
  int32_t rank_mode;         /* PIC_RANK_ROWS or PIC_RANK_CELLS: the ranker the sort uses */
  int64_t device_bytes;      /* device memory held by the context */
} pic_info;

typedef struct {
  int64_t steps;             /* cycles timed since profiling was enabled */
  int64_t particle_launches; /* launches of the fused gather-push-deposit kernel */
  double particle_ms;        /* their summed duration (HIP events on the context's stream) */
  int64_t field_launches;    /* field-solve kernel pairs */
  double field_ms;
  int64_t sort_launches;     /* scan + rank/scatter kernel sequences */
  double sort_ms;
  double step_ms;            /* whole cycles, first kernel start to last kernel end */
} pic_profile;

/* Create a context: validate the descriptor, allocate E and H (two time levels each) and
 * the moment planes on the device, and set E = e0, H = h0, t = 0 (Sec. 3.2 (1), (3)).
 * Errors: PIC_ERR_ARG for an invalid descriptor, PIC_ERR_OOM, PIC_ERR_DEVICE.  On error
 * *out is NULL. */
pic_status pic_init_grid(const pic_grid_desc *desc, pic_ctx **out);

/* Place n particles of species s (Sec. 3.2 (2)): charge q, mass m, positions x^{k+1/2} in
 * cell units and momenta u^k, each array n doubles.  Every particle carries its own density
 * (the n_alpha of the current j_alpha = n_alpha q_alpha v_alpha, Sec. 2 Eqs. (2)-(3)): w[a]
 * when w is not NULL, otherwise w_uniform for every particle of the species.  Per-particle
 * densities travel with their particles through every cycle (8 more bytes read and written
 * per particle and cycle in FP64, 4 in the mixed form, which stores them as FP32).
 * Replaces whatever species s held.  The particles are stably sorted by cell (input order
 * breaks ties), and the moments M^{k+1/2} of all species are deposited again.  When
 * track_ids is set, particle a gets label a.  Errors: PIC_ERR_ARG (s out of range, n < 0,
 * m <= 0, q or w_uniform not finite, NULL position or momentum array with n > 0),
 * PIC_ERR_RANGE (a position outside [0, nx) x [0, nz), or a non-finite momentum or w[a]),
 * PIC_ERR_OOM.  At most 2^28 - 1 particles per species. */
pic_status pic_load_particles(pic_ctx *ctx, int32_t species, double q, double m, int64_t n,
                              const double *xi_x, const double *xi_z, const double *ux,
                              const double *uy, const double *uz, const double *w,
                              double w_uniform);

/* Replace E^k ([3][nodes]) and H^{k+1/2} ([3][cells]); either may be NULL to keep it.
 * The moments are deposited again since they depend on H at the particles.
 * Errors: PIC_ERR_RANGE for a non-finite value. */
pic_status pic_load_fields(pic_ctx *ctx, const double *e, const double *h);

/* Change the tile shape (cells per particle tile; 0, 0 picks it from the particles per
 * occupied cell).  The tiling only distributes work: results are unchanged up to the order of
 * floating-point atomic additions.  Waits for the stream.  Errors: PIC_ERR_ARG (sizes outside
 * 1..64, or the tile's LDS accumulators would exceed the LDS a block may use on the device;
 * the old shape is kept),
 * PIC_ERR_STATE (no particles loaded). */
pic_status pic_set_tiles(pic_ctx *ctx, int32_t tile_x, int32_t tile_z);

/* Choose how the cell sort ranks the particles (the result is the same stable order either
 * way).  PIC_RANK_ROWS: per tile, the destination of every (cell, move code) is staged in LDS
 * and one wavefront per tile row ranks 64 slots at a time with ballots (many particles per
 * cell).  PIC_RANK_CELLS: one thread per cell computes its destinations from its neighbours'
 * counts and walks its own slots (few particles per cell).  PIC_RANK_AUTO (the default)
 * picks by the particles per occupied cell at the last load or re-tiling.
 * Errors: PIC_ERR_ARG for another mode. */
pic_status pic_set_rank_mode(pic_ctx *ctx, int32_t mode);

/* Set the cycle counter and time t = step * dt (used by the x = 0 source). */
pic_status pic_set_step(pic_ctx *ctx, int64_t step);

/* Advance nsteps cycles (Sec. 3.3): field solve, gather-push-deposit, sort.  Work is queued
 * on the context's stream; the call returns without waiting.  Errors: PIC_ERR_STATE if no
 * species is loaded, PIC_ERR_ARG for nsteps < 0, PIC_ERR_DEVICE. */
pic_status pic_step(pic_ctx *ctx, int32_t nsteps);

/* Copy the moment planes M^{k+1/2} ((12 + S) * nodes doubles) into out; len is the size of
 * out in doubles.  Waits for the stream.  Errors: PIC_ERR_ARG if len is too small. */
pic_status pic_read_moments(pic_ctx *ctx, double *out, int64_t len);

/* Copy E^k ([3][nodes]) and H^{k+1/2} ([3][cells]); either pointer may be NULL. */
pic_status pic_read_fields(pic_ctx *ctx, double *e, double *h);

/* Copy species s in its current (cell-sorted) order.  *n_inout holds the capacity of the
 * arrays on entry and the particle count on return; PIC_ERR_ARG if the capacity is too
 * small (then *n_inout is the count needed).  Any output array may be NULL.  w receives each
 * particle's density (w_uniform for a species loaded without per-particle values); id needs
 * track_ids. */
pic_status pic_read_particles(pic_ctx *ctx, int32_t species, int64_t *n_inout, double *xi_x,
                              double *xi_z, double *ux, double *uy, double *uz, double *w,
                              int64_t *id);

/* Sizes, counters and device flags (waits for the stream). */
pic_status pic_get_info(pic_ctx *ctx, pic_info *info);

/* Queue the context's work on an existing HIP stream (hipStream_t passed as void *), or on
 * the context's own stream when NULL.  The stream must outlive its use by the context. */
pic_status pic_set_stream(pic_ctx *ctx, void *stream);

/* Wait until all queued work of the context has finished. */
pic_status pic_sync(pic_ctx *ctx);

/* Per-kernel timing with HIP events recorded on the context's stream.  on = n > 0 starts a
 * new measurement that times every n-th cycle (the first cycle after the call, then every
 * n-th: each event pair leaves the GPU idle for a few microseconds between kernels, so
 * n > 1 keeps most cycles free of them); 0 stops; negative is an error.  Read the sums, over
 * the timed cycles only, with pic_profile_read (waits for the stream). */
pic_status pic_profile_enable(pic_ctx *ctx, int32_t on);
pic_status pic_profile_read(pic_ctx *ctx, pic_profile *out);

/* Select the mover options (PIC_MOVER_* bits; 0 restores the default mover).  Both the
 * deposit (Step 1) and the push of every later cycle use them.  With any option set, the
 * particle stage of a cycle runs in a kernel with one thread per particle that deposits each
 * particle's expanded moments with global atomics, summed first over the lanes of a wavefront
 * that share a cell (per-particle B makes S-hat differ from particle to particle): about three
 * times slower than the default tile kernel.  If particles are loaded, the
 * moments of the current state are deposited again with the new options.  Errors:
 * PIC_ERR_ARG (unknown bits, or a mixed-precision context: the options are FP64 only),
 * PIC_ERR_STATE (the context is in a batch). */
pic_status pic_set_mover(pic_ctx *ctx, int32_t options);

/* Energies of the current state, computed on the device: out[0] = field energy
 * (1/2)(sum over nodes of |E^n|^2 + sum over cells of |H^{n+1/2}|^2) dx dz, out[1 + s] =
 * kinetic energy of species s, sum over its particles of w m (gamma(u^n) - 1) dx dz (0 for a
 * species without particles).  len >= 1 + n_species.  Waits for the stream.  Errors:
 * PIC_ERR_ARG (out NULL or len too small). */
pic_status pic_energy(pic_ctx *ctx, double *out, int32_t len);

/* pic_energy for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same energies, computed without
 * any allocation.  Partial sums go to a fixed buffer in the library's device memory, one copy
 * per GPU held until the process ends ((1024 + 1) x 9 doubles, 73,800 bytes, the largest
 * species count included), and are added in a fixed order, so repeated calls on the same
 * state give the same bits.  Calls that overlap on one GPU (other host threads, other
 * contexts on the device) race on that buffer and must be serialised by the caller.  Waits for
 * the context's stream.  Errors: as pic_energy (PIC_ERR_ARG for out NULL or len < 1 +
 * n_species), PIC_ERR_DEVICE. */
pic_status pic_energy_noalloc(pic_ctx *ctx, double *out, int32_t len);

/* Device memory.  By default a context (and a batch) allocates with hipMalloc and releases
 * with hipFree.  pic_set_allocator installs a process-wide pair of functions used instead by
 * every context and batch created after the call (each keeps the pair it was created with):
 * alloc(bytes, device, user) returns device memory of at least bytes bytes on the given HIP
 * device, aligned to 256 bytes, or NULL when it cannot; the library call then fails with
 * PIC_ERR_OOM (pic_init_grid returns no context, pic_load_particles leaves the species
 * without particles, pic_set_tiles keeps the old tiles).  free(ptr, bytes, device, user)
 * releases a block with the size it was allocated with.  This is how a framework such as
 * PyTorch lends the library its caching allocator.  The library frees memory only after the
 * work queued on it has finished.  Passing NULL for both restores hipMalloc / hipFree.
 * Errors: PIC_ERR_ARG if exactly one of alloc and free is NULL. */
typedef void *(*pic_alloc_fn)(uint64_t bytes, int32_t device, void *user);
typedef void (*pic_free_fn)(void *ptr, uint64_t bytes, int32_t device, void *user);
pic_status pic_set_allocator(pic_alloc_fn alloc, pic_free_fn free_fn, void *user);

/* Message for the last failed call on this context (or of pic_init_grid, pic_set_allocator
 * or another call without a context when ctx is NULL). */
const char *pic_last_error(const pic_ctx *ctx);

/* Release the context and all its device memory (removing it from its batch first).  NULL is
 * allowed. */
void pic_destroy(pic_ctx *ctx);

/* ---- Batches: many independent runs stepped together ----------------------------------------
 *
 * A batch steps its member contexts with one launch of each kernel per cycle for all members
 * together (persistent blocks over the work items of every member), optionally replaying a
 * captured HIP graph of one cycle.  This is the same cycle as pic_step (Sec. 3.3), so each
 * member's results are those of stepping it alone, up to the order of floating-point atomic
 * additions.  Members keep their own device memory and stay readable (pic_read_*,
 * pic_get_info) between batch steps; while in a batch they run on the batch's stream and
 * pic_step / pic_set_stream on them return PIC_ERR_STATE.  Loading particles or fields into a
 * member, or pic_set_step, is allowed and takes effect at the next batch step.  All members
 * must be on the batch's device, use the batch's precision and have particles loaded. */
typedef struct pic_batch pic_batch;

/* Create an empty batch on a HIP device for contexts of the given precision (PIC_PREC_*).
 * Errors: PIC_ERR_ARG, PIC_ERR_DEVICE. */
pic_status pic_batch_create(int32_t device, int32_t precision, pic_batch **out);

/* Add a context (PIC_ERR_ARG if it is NULL, already in a batch, on another device, of another
 * precision, or has no particles) / remove it (PIC_ERR_ARG if it is not a member).  Removal
 * waits for the batch's queued work and returns the context to its own stream. */
pic_status pic_batch_add(pic_batch *b, pic_ctx *ctx);
pic_status pic_batch_remove(pic_batch *b, pic_ctx *ctx);

/* Advance every member nsteps cycles.  Work is queued on the batch's stream; the call returns
 * without waiting.  An empty batch is a no-op.  Errors: PIC_ERR_ARG (nsteps < 0),
 * PIC_ERR_DEVICE, PIC_ERR_OOM (growing the batch tables). */
pic_status pic_batch_step(pic_batch *b, int32_t nsteps);

/* on = 1: capture one cycle of all members in a HIP graph (again after every change of the
 * membership or of a member's load) and replay it for each cycle; 0: launch the kernels
 * directly (the default). */
pic_status pic_batch_set_graph(pic_batch *b, int32_t on);

/* Wait for the batch's queued work. */
pic_status pic_batch_sync(pic_batch *b);

/* Number of member contexts. */
pic_status pic_batch_size(const pic_batch *b, int32_t *n);

/* Message for the last failed call on this batch (or of pic_batch_create when b is NULL). */
const char *pic_batch_last_error(const pic_batch *b);

/* Release the batch (members are removed and stay valid).  NULL is allowed. */
void pic_batch_destroy(pic_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
