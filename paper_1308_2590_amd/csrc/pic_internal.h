// Internal interface between the host side of the library (pic_capi.cpp) and the HIP
// kernels (pic_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

namespace pic {

constexpr int kMaxSpecies = PIC_MAX_SPECIES;
constexpr int kMoveCodes = 9;      // destination cell relative to the source: 3 x 3 block
constexpr uint8_t kAbsorbed = 9;   // move code of a particle that left an absorbing boundary
constexpr int kBlock = 256;        // threads per block of the tile kernels (4 wavefronts)
constexpr int kPermPad = 8;        // padding entries after each permutation array
constexpr int kSolveNodes = 2;     // nodes per thread in the E solve
constexpr int kHCells = 2;         // cells per thread in the H update
constexpr int kScanItems = 4;      // cells per thread in the count scan
constexpr int kFlagNodes = 8;      // consecutive nodes per deposit flag
constexpr int kScanBlock = kBlock * kScanItems;
constexpr int kScan1Items = 4;      // cells per thread in the scan of a cycle's sort
constexpr int kScan1Block = kBlock * kScan1Items;

struct GridArgs {
  int32_t nx, nz, nxn, nzn;  // cells and nodes per axis
  int32_t bc_x;              // PIC_BC_PERIODIC or PIC_BC_ABSORBING (z is periodic)
  int32_t n_planes;          // 12 + S moment planes
  int64_t ncells, nnodes;
  double dx, dz, dt;
  double cx, cz;             // dt / dx, dt / dz
};

struct LaserArgs {
  double a0, omega, sigma_z, z_center, fwhm_t, t_center;
};

struct TileArgs {
  int32_t tx, tz;            // cells per tile
  int32_t ntx, ntz, ntiles;  // tiles per axis and in total
  int32_t per_xcd;           // tiles per XCD band: launch grid is 8 * per_xcd blocks
};

// FP64 particle state: structure of arrays, 5 planes (xi_x, xi_z, u_x, u_y, u_z).
struct SpeciesArgs {
  double q, m, w;
  double beta;               // q dt / (2 m)
  double cS;                 // w q^2 dt^2 / (4 m)  (uniform w)
  double kJ;                 // w q
  double cS1, kJ1;           // q^2 dt^2 / (4 m) and q: per-particle densities multiply these
  const double *src[5];      // current state, addressed through perm (FP64 form)
  double *dst[5];            // pushed state, written in the kernel's processing order
  // Per-particle densities (NULL for a species with one density w): FP64 form src_w / dst_w,
  // mixed form msrc_w / mdst_w (FP32), addressed like the state arrays.
  const double *src_w;
  double *dst_w;
  const float *msrc_w;
  float *mdst_w;
  int32_t w_stride;          // 1: per-particle densities; 0: src_w / msrc_w hold the single w
  const int32_t *msrc_cell;  // mixed form: cell key k * nx + i
  const float *msrc[5];      // mixed form: offsets f_x, f_z in [0, 1) and u_x, u_y, u_z
  int32_t *mdst_cell;
  float *mdst[5];
  const int64_t *src_id;
  int64_t *dst_id;
  const int32_t *perm;       // sorted slot -> location in src
  int32_t *perm_new;         // next cycle's sorted slot -> location in dst
  const int32_t *cs;         // cell start offsets of the current order [ncells + 1]
  int32_t *cs_new;           // cell start offsets of the next order [ncells + 1]
  uint32_t *locode;          // per sorted slot: (location written << 4) | move code
  int32_t *cnt;              // [9][ncells] particles leaving each cell per move code
  // [ncells] bit d set when the cell sent particles with move code d; with count masks only
  // the counts of set bits are written (the others keep values from earlier cycles)
  uint16_t *cmask;
  int32_t *arr;              // [ncells] particles arriving in each cell; zero between cycles
  int32_t *bsum;             // block sums of the count scan
  int32_t cap;               // particle capacity of the state arrays
  int32_t active;
};

struct StepArgs {
  GridArgs g;
  TileArgs t;
  int32_t mixed;             // 1: mixed-precision particle state and arithmetic
  int32_t rank_cells;        // 1: destinations ranked one thread per cell, 0: by tile rows
  int32_t chunk2;            // 1: the particle kernel loads 2 particles per lane at a time, 0: 4
  int32_t count_masks;       // 1: the particle kernel writes code masks and nonzero counts only
  int32_t n_scan_blocks;     // blocks of the count scan per species
  int32_t nsp;               // species slots
  SpeciesArgs sp[kMaxSpecies];
  const double *Eold, *Enew; // E^n, E^{n+1} [3][nodes]: E-bar is their mean
  const double *Hold;        // H^{n+1/2} [3][cells]
  const double *Hnew;        // H^{n+3/2} [3][cells]
  double *M;                 // moment planes [12 + S][nodes]
  uint32_t *flags;
  // tiles holding particles of the current order (flag per tile; ordered list, count at
  // [ntiles]) and the same for the next order, built after the count scan
  const uint8_t *tile_active;
  const int32_t *tile_list;
  uint8_t *tile_active_next;
  int32_t *tile_list_next;
  uint8_t *mflag;            // deposit flags (see FieldArgs): set for every node the fold adds to
  int32_t n_scan1_blocks;   // blocks of kScan1Block cells in a cycle's sort scan
};

struct FieldArgs {
  GridArgs g;
  LaserArgs laser;
  double t;                  // time of E^n
  double *M;                 // moment planes: read, then zeroed, where deposits can be
  const double *E;           // E^n
  const double *H;           // H^{n+1/2}
  double *E_new, *H_new;
  // Deposit flags, one per kFlagNodes consecutive nodes (node index n: flag n / kFlagNodes):
  // a node's moments are read (and cleared) only where its flag is set, since the deposit sets
  // the flag of every node it adds to; the H update clears the flags for the next deposit.
  // NULL: every node is read and cleared.
  uint8_t *mflag;
  uint8_t *tact_next;        // batched cycle: the next order's tile flags, cleared here (or NULL)
  int32_t ntiles_next;       // their count
  double r2dx, r2dz;         // 1 / (2 dx), 1 / (2 dz) of the centred differences
};

// Many independent runs stepped together, each kernel launched once for all of them (a block
// per work item for the field, particle and rank kernels, persistent blocks looping over the
// items of the scans).  Per run, the step and field arguments for both
// buffer parities live in device memory, and the run's current parity and cycle count are
// device counters, so one captured cycle can be replayed for any mix of runs.
struct BatchArgs {
  const StepArgs *step;      // [2 * nruns]: run r, parity p at 2 r + p
  const FieldArgs *field;    // [2 * nruns]
  int32_t *par;              // [nruns] buffer parity of the current cycle
  int64_t *step_ctr;         // [nruns] cycles done (E^n is at step * dt)
  int32_t nruns;
  // exclusive prefix sums over runs ([nruns + 1]) of the work items of each kernel
  const int32_t *pre_nodes;  // blocks of kSolveNodes * kBlock nodes
  const int32_t *pre_cells;  // blocks of kHCells * kBlock cells
  const int32_t *pre_scan;   // scan blocks x species slots (both passes of the sort's scan)
  const int32_t *pre_one;    // one item per run
  int32_t *pre_tiles;        // active tiles of the current order (written each cycle)
  int32_t *pre_rank;         // active tiles x species slots (written each cycle)
};

struct BatchLaunch {
  int32_t grid_particles;    // blocks of the particle kernel: every tile of every run
  int32_t grid_rank;         // blocks of the rank kernel: tiles x species of every run
  int32_t items_nodes;       // node blocks of all runs (one block each in the E solve)
  int32_t items_cells;       // cell blocks of all runs (one block each in the H update)
  int32_t items_scan;        // scan blocks x species of all runs (one block each in the scans)
  size_t lds_particles, lds_rank;
  bool mixed;
  bool ids;                  // some run copies particle ids (the kernel instantiation with ids)
  bool pw;                   // some run carries per-particle densities
};

// LDS of the particle kernel's block for a tile; pw: the instantiation with per-particle
// densities (one more word per queued mover); queues: with the per-wavefront mover queues.
size_t particle_lds_bytes(const GridArgs &g, const TileArgs &t, bool mixed, bool pw, bool queues = true);
size_t rank_lds_bytes(const TileArgs &t);

hipError_t launch_field_solve(const FieldArgs &a, hipStream_t s);
// launch_particles also clears the next order's tile flags, which the sort's scan sets again;
// launch_sort is the sort of a cycle (two-pass scan with tile flags and list, then ranks).
hipError_t launch_particles(const StepArgs &a, bool push, hipStream_t s);
hipError_t launch_sort(const StepArgs &a, hipStream_t s);
// The particle stage with mover options (PIC_MOVER_* bits), one thread per slot: max_n bounds
// the particles of every species; the move counts must be zero on entry.
hipError_t launch_particles_alt(const StepArgs &a, bool push, int mover, int32_t max_n,
                                hipStream_t s);
// Field and kinetic energies into out[1 + nsp] (accumulated: zero it first).
hipError_t launch_energy(const StepArgs &a, const double *E, const double *H, double *out,
                         hipStream_t s);
// The same energies without device allocation: partial sums of kEnergyBlocks blocks in a
// fixed per-device buffer, added in block order; the totals (field, then kMaxSpecies species
// slots) end at scratch_ptr + kEnergyBlocks * kEnergyVals.
constexpr int kEnergyBlocks = 1024;
constexpr int kEnergyVals = 1 + kMaxSpecies;
constexpr int kEnergyScratchDoubles = (kEnergyBlocks + 1) * kEnergyVals;  // 73,800 bytes
constexpr int kMaxScratchDevices = 64;
// Device address of that buffer on a HIP device (looked up once per device).
hipError_t energy_scratch(int32_t device, double **ptr);
hipError_t launch_energy_scratch(const StepArgs &a, const double *E, const double *H,
                                 double *scratch_ptr, hipStream_t s);
hipError_t launch_iota(int32_t *p, int64_t n, hipStream_t s);
// One cycle of every run of a batch (field solve, particles, sort, counters).
hipError_t launch_batch_cycle(const BatchArgs &b, const BatchLaunch &l, hipStream_t s);
// Build the active-tile flags and list of the order described by sp[].cs (into
// tile_active_next / tile_list_next).
hipError_t launch_tile_list(const StepArgs &a, bool from_next_order, hipStream_t s);

}  // namespace pic
