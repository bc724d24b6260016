/*
 * CPU oracle for the implicit 2D3V particle-in-cell particle stage (Petrov & Davis,
 * "Parallelization of an implicit algorithm for multi-dimensional particle-in-cell
 * simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64, single-threaded implementation
 * written straight from the paper's equations so that the GPU library can be checked
 * against it.  Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or constant with the GPU library.
 *
 * Conventions (readings of the paper, listed with their reasons in the design notes):
 *   - plane (x, z) with d/dy = 0 and three momentum components (2D3V, abstract);
 *   - units c = eps0 = mu0 = 1, so B = H (Sec. 2, Eqs. 1a-1b);
 *   - E on grid nodes, H at cell centres, S-hat and delta-j on nodes (end of Sec. 2,
 *     Sec. 3.2 item 3, Fig. 1 caption);
 *   - positions in cell units: cell (i, k) spans [i, i+1) x [k, k+1); node (i, k) sits at
 *     integer coordinates; arrays are stored with x fastest;
 *   - a periodic axis with N cells has N nodes (node N is node 0); an absorbing axis has
 *     N + 1 nodes;
 *   - moment planes, each [nodes_z][nodes_x]:
 *       0..8   S_xx S_xy S_xz S_yx S_yy S_yz S_zx S_zy S_zz  (row-major 3x3)
 *       9..11  dj_x dj_y dj_z
 *       12+s   density of species s
 *   - the whole file is compiled with -ffp-contract=off (no fused multiply-add), so each
 *     operation is one IEEE-754 double rounding in the order written.
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_ABSORBING = 1 };

/* Mover options (readings R1 and R5 of the paper; 0 is the default of both):
 *   ORC_GAMMA_PREDICT  gamma-bar = gamma(u^n + beta E^n) instead of gamma(u^n);
 *   ORC_B_BILINEAR     B at the particle interpolated from the four surrounding cell centres
 *                      instead of the particle's own cell. */
enum { ORC_GAMMA_PREDICT = 1, ORC_B_BILINEAR = 2 };

typedef struct {
  int32_t nx, nz;          /* cells along x and z */
  double dx, dz, dt;
  int32_t bc_x, bc_z;      /* bc_z must be periodic */
  int32_t n_species;       /* S: number of density planes */
  double laser_a0, laser_omega, laser_sigma_z, laser_z_center, laser_fwhm_t, laser_t_center;
} orc_grid;

typedef struct {
  double q, m;             /* charge (units of e) and mass (units of m_e) */
  int64_t n;               /* particles held */
  double *xi_x, *xi_z;     /* position in cell units */
  double *ux, *uy, *uz;    /* momentum p / (m c) */
  double *w;               /* density carried by each particle */
  int64_t *id;             /* label carried through the sort (may be NULL) */
} orc_species;

int32_t orc_nodes_x(const orc_grid *g);
int32_t orc_nodes_z(const orc_grid *g);

/* Implicit response of one particle: R = (I + [b]x + b b^T) / (1 + b.b), b = beta B / gamma,
 * for a given gamma-bar (orc_response_g) or gamma-bar = gamma(u) (orc_response). */
void orc_response_g(double q, double m, double dt, double gamma, const double B[3], double R[9]);
void orc_response(double q, double m, double dt, const double u[3], const double B[3],
                  double R[9], double *gamma);

/* Add species s's implicit source moments S-hat, delta-j and density to M (Sec. 3.3 Step 1).
 * E = E^n (read with ORC_GAMMA_PREDICT only); mode = ORC_* mover options. */
void orc_deposit(const orc_grid *g, int32_t s, const orc_species *sp, const double *H,
                 const double *E, int32_t mode, double *M);

/* Linear (bilinear) interpolation of ncomp node planes to n particle positions. */
void orc_gather(const orc_grid *g, const double *F, int32_t ncomp, int64_t n,
                const double *xi_x, const double *xi_z, double *out);

/* B at n particle positions as the mover sees it (mode & ORC_B_BILINEAR selects the
 * interpolation), out[3][n]. */
void orc_particle_B(const orc_grid *g, const double *H, int32_t mode, int64_t n,
                    const double *xi_x, const double *xi_z, double *out);

/* Incident laser E_y at time t and point (x, z) (the source added at x = 0, Step 4). */
double orc_incident_ey(const orc_grid *g, double t, double x, double z);

/* Field solve: Eq. (4) per node, x-boundary conditions and source, E-bar, Eq. (5). */
void orc_field_solve(const orc_grid *g, double t, const double *M, const double *E,
                     const double *H, double *E_new, double *Ebar, double *H_new);

/* Implicit push of one species in E-bar and H^{n+1/2}; alive[p] = 0 if absorbed.  E = E^n
 * (read with ORC_GAMMA_PREDICT only); mode = ORC_* mover options. */
void orc_push(const orc_grid *g, orc_species *sp, const double *Ebar, const double *H,
              const double *E, int32_t mode, uint8_t *alive);

/* Stable counting sort of alive particles by cell key k*nx + i; returns the new count.
 * perm_out (may be NULL) receives, for each new position, the old index. */
int64_t orc_sort(const orc_grid *g, orc_species *sp, const uint8_t *alive, int64_t *perm_out);

#ifdef __cplusplus
}
#endif
#endif
