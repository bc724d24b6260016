/*
 * CPU oracle for the implicit 2D3V PIC particle stage.  TEST INFRASTRUCTURE ONLY: see orc.h.
 *
 * Each function follows one passage of the paper; the reconstruction of the pieces the paper
 * leaves to its Ref. [19] is done from Eqs. (2)-(5) alone:
 *
 *   Time-centred form of Eq. (2a) in normalised units, with u = p/(m c), gamma-bar taken at
 *   u^n, B at the particle's cell and u-bar = (u^n + u^{n+1})/2:
 *       u-bar = u^n + beta E-bar + u-bar x b,     beta = q dt / (2 m),  b = beta B / gamma-bar.
 *   Its solution is u-bar = R (u^n + beta E-bar) with R = (I + [b]x + b b^T) / (1 + b.b),
 *   where [b]x a = a x b.  The particle current n_a q u-bar / gamma-bar is then
 *       j_a = (w q / gamma) R u^n  +  (w q^2 dt / (2 m gamma)) R E-bar,
 *   i.e. the split of Eq. (3) into delta-j and a conductivity.  Putting the time-centred
 *   current into Eq. (1a) gives Eq. (4) with S-hat = dt/2 times that conductivity:
 *       S-hat_a = w q^2 dt^2 R / (4 m gamma).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int32_t orc_nodes_x(const orc_grid *g) { return g->nx + (g->bc_x == ORC_ABSORBING ? 1 : 0); }
int32_t orc_nodes_z(const orc_grid *g) { return g->nz + (g->bc_z == ORC_ABSORBING ? 1 : 0); }

/* Node index along an axis with wrap on a periodic axis. */
static int32_t wrap_node(int32_t i, int32_t ncell, int32_t bc) {
  if (bc == ORC_PERIODIC) {
    if (i < 0) return i + ncell;
    if (i >= ncell) return i - ncell;
  }
  return i;
}

/* Cell index along an axis with wrap (used by the stencils; absorbing axes never wrap). */
static int32_t wrap_cell(int32_t i, int32_t ncell) {
  if (i < 0) return i + ncell;
  if (i >= ncell) return i - ncell;
  return i;
}

/* Eq. (2a) solved for the time-centred momentum: the 3x3 matrix R for a given gamma-bar. */
void orc_response_g(double q, double m, double dt, double g, const double B[3], double R[9]) {
  double beta = q * dt / (2.0 * m);
  double bg = beta / g;
  double bx = bg * B[0], by = bg * B[1], bz = bg * B[2];
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

/* The same with gamma-bar = gamma(u^n), the lagged Lorentz factor. */
void orc_response(double q, double m, double dt, const double u[3], const double B[3],
                  double R[9], double *gamma) {
  double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  orc_response_g(q, m, dt, g, B, R);
  *gamma = g;
}

/* The particle's cell, in-cell offsets and the four linear shape weights (Sec. 3.3, last
 * paragraph: linear interpolation, all quantities collected within the cell).  Corner order:
 * (i,k), (i+1,k), (i,k+1), (i+1,k+1). */
static void cell_weights(const orc_grid *g, double xi_x, double xi_z, int32_t node[4],
                         double W[4], int32_t *cell_i, int32_t *cell_k) {
  int32_t i = (int32_t)floor(xi_x);
  int32_t k = (int32_t)floor(xi_z);
  double fx = xi_x - (double)i;
  double fz = xi_z - (double)k;
  int32_t nxn = orc_nodes_x(g);
  int32_t i1 = wrap_node(i + 1, g->nx, g->bc_x);
  int32_t k1 = wrap_node(k + 1, g->nz, g->bc_z);
  node[0] = k * nxn + i;
  node[1] = k * nxn + i1;
  node[2] = k1 * nxn + i;
  node[3] = k1 * nxn + i1;
  W[0] = (1.0 - fx) * (1.0 - fz);
  W[1] = fx * (1.0 - fz);
  W[2] = (1.0 - fx) * fz;
  W[3] = fx * fz;
  *cell_i = i;
  *cell_k = k;
}

/* B at the particle from the cell-centred H (R5).  Default: H of the particle's own cell.
 * ORC_B_BILINEAR: bilinear interpolation between the four cell centres around the particle
 * (centres at i + 1/2, k + 1/2); periodic axes wrap; on an absorbing x axis a centre index
 * beyond the edge is clamped to the edge cell. */
static void particle_B(const orc_grid *g, const double *H, double xi_x, double xi_z, int32_t mode,
                       double B[3]) {
  int64_t ncells = (int64_t)g->nx * g->nz;
  if (!(mode & ORC_B_BILINEAR)) {
    int64_t c = (int64_t)floor(xi_z) * g->nx + (int64_t)floor(xi_x);
    for (int r = 0; r < 3; ++r) B[r] = H[r * ncells + c];
    return;
  }
  double sx = xi_x - 0.5, sz = xi_z - 0.5;
  int32_t ic = (int32_t)floor(sx), kc = (int32_t)floor(sz);
  double gx = sx - (double)ic, gz = sz - (double)kc;
  int32_t ci[2], ck[2];
  for (int t = 0; t < 2; ++t) {
    int32_t i = ic + t, k = kc + t;
    if (g->bc_x == ORC_PERIODIC) {
      ci[t] = wrap_cell(i, g->nx);
    } else {
      ci[t] = i < 0 ? 0 : (i >= g->nx ? g->nx - 1 : i);
    }
    ck[t] = wrap_cell(k, g->nz);
  }
  double Wc[4] = {(1.0 - gx) * (1.0 - gz), gx * (1.0 - gz), (1.0 - gx) * gz, gx * gz};
  int64_t c4[4] = {(int64_t)ck[0] * g->nx + ci[0], (int64_t)ck[0] * g->nx + ci[1],
                   (int64_t)ck[1] * g->nx + ci[0], (int64_t)ck[1] * g->nx + ci[1]};
  for (int r = 0; r < 3; ++r)
    B[r] = Wc[0] * H[r * ncells + c4[0]] + Wc[1] * H[r * ncells + c4[1]] +
           Wc[2] * H[r * ncells + c4[2]] + Wc[3] * H[r * ncells + c4[3]];
}

void orc_particle_B(const orc_grid *g, const double *H, int32_t mode, int64_t n,
                    const double *xi_x, const double *xi_z, double *out) {
  for (int64_t a = 0; a < n; ++a) {
    double B[3];
    particle_B(g, H, xi_x[a], xi_z[a], mode, B);
    for (int r = 0; r < 3; ++r) out[r * n + a] = B[r];
  }
}

/* gamma-bar of the linearised mover (R1).  Default: gamma(u^n).  ORC_GAMMA_PREDICT: the
 * Boris-style predictor gamma(u^n + beta E^n), E^n (the field before the solve) interpolated
 * linearly at the particle; the deposit and the push of a cycle use the same value. */
static double particle_gamma(const orc_grid *g, const double *E, double q, double m,
                             const double u[3], const int32_t node[4], const double W[4],
                             int32_t mode) {
  if (!(mode & ORC_GAMMA_PREDICT))
    return sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  int64_t nnodes = (int64_t)orc_nodes_x(g) * orc_nodes_z(g);
  double beta = q * g->dt / (2.0 * m);
  double um[3];
  for (int r = 0; r < 3; ++r) {
    const double *f = E + r * nnodes;
    double e = W[0] * f[node[0]] + W[1] * f[node[1]] + W[2] * f[node[2]] + W[3] * f[node[3]];
    um[r] = u[r] + beta * e;
  }
  return sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
}

/* Sec. 3.3 Step 1 with Eq. (3): S-hat and delta-j accumulated on the nodes from the particles
 * at x^{n+1/2} with u^n and B = H^{n+1/2} at the particle; plus the species density.  E is E^n
 * (read by ORC_GAMMA_PREDICT only; may be NULL otherwise). */
void orc_deposit(const orc_grid *g, int32_t s, const orc_species *sp, const double *H,
                 const double *E, int32_t mode, double *M) {
  int64_t nnodes = (int64_t)orc_nodes_x(g) * orc_nodes_z(g);
  double cS = sp->q * sp->q * g->dt * g->dt / (4.0 * sp->m);
  for (int64_t a = 0; a < sp->n; ++a) {
    int32_t node[4], ci, ck;
    double W[4];
    cell_weights(g, sp->xi_x[a], sp->xi_z[a], node, W, &ci, &ck);
    double B[3];
    particle_B(g, H, sp->xi_x[a], sp->xi_z[a], mode, B);
    double u[3] = {sp->ux[a], sp->uy[a], sp->uz[a]};
    double R[9];
    double gam = particle_gamma(g, E, sp->q, sp->m, u, node, W, mode);
    orc_response_g(sp->q, sp->m, g->dt, gam, B, R);
    double w = sp->w[a];
    double kS = w * cS / gam;
    double kJ = w * sp->q / gam;
    double val[13];
    for (int r = 0; r < 9; ++r) val[r] = kS * R[r];
    for (int r = 0; r < 3; ++r)
      val[9 + r] = kJ * (R[3 * r] * u[0] + R[3 * r + 1] * u[1] + R[3 * r + 2] * u[2]);
    val[12] = w;
    for (int v = 0; v < 4; ++v) {
      for (int r = 0; r < 12; ++r) M[r * nnodes + node[v]] += W[v] * val[r];
      M[(12 + s) * nnodes + node[v]] += W[v] * val[12];
    }
  }
}

void orc_gather(const orc_grid *g, const double *F, int32_t ncomp, int64_t n,
                const double *xi_x, const double *xi_z, double *out) {
  int64_t nnodes = (int64_t)orc_nodes_x(g) * orc_nodes_z(g);
  for (int64_t a = 0; a < n; ++a) {
    int32_t node[4], ci, ck;
    double W[4];
    cell_weights(g, xi_x[a], xi_z[a], node, W, &ci, &ck);
    for (int c = 0; c < ncomp; ++c) {
      const double *f = F + c * nnodes;
      out[c * n + a] = W[0] * f[node[0]] + W[1] * f[node[1]] + W[2] * f[node[2]] + W[3] * f[node[3]];
    }
  }
}

/* Sec. 3.3 Step 4: the source field injected at x = 0, an E_y wave travelling in +x with a
 * Gaussian transverse profile and a Gaussian envelope in retarded time. */
double orc_incident_ey(const orc_grid *g, double t, double x, double z) {
  if (g->laser_a0 == 0.0) return 0.0;
  double tau = t - x;
  double st = (tau - g->laser_t_center) / g->laser_fwhm_t;
  double sz = (z - g->laser_z_center) / g->laser_sigma_z;
  return g->laser_a0 * sin(g->laser_omega * tau) * exp(-0.5 * sz * sz) *
         exp(-2.0 * log(2.0) * st * st);
}

/* Solve the 3x3 system A x = b by Cramer's rule (adjugate over determinant). */
static void solve3(const double A[9], const double b[3], double x[3]) {
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
  /* x = adj(A) b / det, adj(A)_{rc} = cofactor_{cr} */
  x[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) / det;
  x[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) / det;
  x[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) / det;
}

/*
 * Field solve of one cycle (Sec. 2 Eqs. (4)-(5); Sec. 3.3 Steps 3-9 without communication).
 *   E_new = (I + S)^{-1} [ (I - S) E + dt (curl H - delta-j) ]   at every node (Step 5);
 *   on an absorbing x axis the columns x = 0 and x = L_x take a first-order Mur condition
 *   (Step 3), applied to the scattered field E - E_inc at x = 0 so the source of Step 4
 *   enters there;  E-bar = (E + E_new)/2;  H_new = H - dt curl E_new at cell centres
 *   (Eq. (5), Steps 8-9).  curl H at a node and curl E at a cell centre both use central
 *   differences over the 2x2 block of neighbours, averaged across the other axis.
 */
void orc_field_solve(const orc_grid *g, double t, const double *M, const double *E,
                     const double *H, double *E_new, double *Ebar, double *H_new) {
  const int32_t nx = g->nx, nz = g->nz;
  const int32_t nxn = orc_nodes_x(g), nzn = orc_nodes_z(g);
  const int64_t nn = (int64_t)nxn * nzn, nc = (int64_t)nx * nz;
  const double dt = g->dt;
  const int absorbing = (g->bc_x == ORC_ABSORBING);
  const double *Hx = H, *Hy = H + nc, *Hz = H + 2 * nc;

  for (int32_t k = 0; k < nzn; ++k) {
    int32_t kU = wrap_cell(k, nz), kD = wrap_cell(k - 1, nz);
    for (int32_t i = 0; i < nxn; ++i) {
      int64_t n = (int64_t)k * nxn + i;
      if (absorbing && (i == 0 || i == nx)) continue; /* boundary columns: Mur below */
      int32_t iR = wrap_cell(i, nx), iL = wrap_cell(i - 1, nx);
      int64_t cUR = (int64_t)kU * nx + iR, cUL = (int64_t)kU * nx + iL;
      int64_t cDR = (int64_t)kD * nx + iR, cDL = (int64_t)kD * nx + iL;
      double dHx_dz = ((Hx[cUR] + Hx[cUL]) - (Hx[cDR] + Hx[cDL])) / (2.0 * g->dz);
      double dHy_dz = ((Hy[cUR] + Hy[cUL]) - (Hy[cDR] + Hy[cDL])) / (2.0 * g->dz);
      double dHy_dx = ((Hy[cUR] + Hy[cDR]) - (Hy[cUL] + Hy[cDL])) / (2.0 * g->dx);
      double dHz_dx = ((Hz[cUR] + Hz[cDR]) - (Hz[cUL] + Hz[cDL])) / (2.0 * g->dx);
      double curl[3] = {-dHy_dz, dHx_dz - dHz_dx, dHy_dx};
      double S[9], A[9], e[3], rhs[3], x[3];
      for (int r = 0; r < 9; ++r) S[r] = M[r * nn + n];
      for (int r = 0; r < 3; ++r) e[r] = E[r * nn + n];
      for (int r = 0; r < 3; ++r) {
        double se = S[3 * r] * e[0] + S[3 * r + 1] * e[1] + S[3 * r + 2] * e[2];
        rhs[r] = (e[r] - se) + dt * (curl[r] - M[(9 + r) * nn + n]);
      }
      for (int r = 0; r < 9; ++r) A[r] = S[r] + ((r % 4 == 0) ? 1.0 : 0.0);
      solve3(A, rhs, x);
      for (int r = 0; r < 3; ++r) E_new[r * nn + n] = x[r];
    }
  }

  if (absorbing) {
    const double kappa = (dt - g->dx) / (dt + g->dx);
    const double t1 = t + dt;
    for (int32_t k = 0; k < nzn; ++k) {
      double z = (double)k * g->dz;
      int64_t n0 = (int64_t)k * nxn, n1 = n0 + 1, nb = n0 + nx, nb1 = nb - 1;
      for (int r = 0; r < 3; ++r) {
        const double *Eo = E + r * nn;
        double *En = E_new + r * nn;
        double inc_t1_0 = 0.0, inc_t0_1 = 0.0, inc_t1_1 = 0.0, inc_t0_0 = 0.0;
        if (r == 1) {
          inc_t1_0 = orc_incident_ey(g, t1, 0.0, z);
          inc_t0_1 = orc_incident_ey(g, t, g->dx, z);
          inc_t1_1 = orc_incident_ey(g, t1, g->dx, z);
          inc_t0_0 = orc_incident_ey(g, t, 0.0, z);
        }
        En[n0] = inc_t1_0 + (Eo[n1] - inc_t0_1) + kappa * ((En[n1] - inc_t1_1) - (Eo[n0] - inc_t0_0));
        En[nb] = Eo[nb1] + kappa * (En[nb1] - Eo[nb]);
      }
    }
  }

  for (int64_t q = 0; q < 3 * nn; ++q) Ebar[q] = 0.5 * (E[q] + E_new[q]);

  const double *Ex = E_new, *Ey = E_new + nn, *Ez = E_new + 2 * nn;
  for (int32_t k = 0; k < nz; ++k) {
    int32_t k1 = wrap_node(k + 1, nz, g->bc_z);
    for (int32_t i = 0; i < nx; ++i) {
      int32_t i1 = wrap_node(i + 1, nx, g->bc_x);
      int64_t a = (int64_t)k * nxn + i, b = (int64_t)k * nxn + i1;
      int64_t c = (int64_t)k1 * nxn + i, d = (int64_t)k1 * nxn + i1;
      double dEx_dz = ((Ex[c] + Ex[d]) - (Ex[a] + Ex[b])) / (2.0 * g->dz);
      double dEy_dz = ((Ey[c] + Ey[d]) - (Ey[a] + Ey[b])) / (2.0 * g->dz);
      double dEy_dx = ((Ey[b] + Ey[d]) - (Ey[a] + Ey[c])) / (2.0 * g->dx);
      double dEz_dx = ((Ez[b] + Ez[d]) - (Ez[a] + Ez[c])) / (2.0 * g->dx);
      int64_t cell = (int64_t)k * nx + i;
      H_new[cell] = H[cell] - dt * (-dEy_dz);
      H_new[nc + cell] = H[nc + cell] - dt * (dEx_dz - dEz_dx);
      H_new[2 * nc + cell] = H[2 * nc + cell] - dt * dEy_dx;
    }
  }
}

/*
 * The implicit mover (Sec. 2, Eq. (2); pushed once per cycle, Sec. 1): with E-bar gathered at
 * x^{n+1/2} and B = H^{n+1/2} at the particle (its cell's, or bilinear with ORC_B_BILINEAR),
 * u-bar = R (u^n + beta E-bar), u^{n+1} = 2 u-bar - u^n, then
 * x^{n+3/2} = x^{n+1/2} + dt u^{n+1} / gamma(u^{n+1}) (Eqs. 2b-2c).  E is E^n, read for the
 * gamma-bar predictor only (ORC_GAMMA_PREDICT; may be NULL otherwise).
 * Periodic axes wrap; a particle leaving an absorbing x axis is removed (it leaves the domain,
 * as particles leaving a processor's strip leave that processor, Sec. 3.3).
 */
void orc_push(const orc_grid *g, orc_species *sp, const double *Ebar, const double *H,
              const double *E, int32_t mode, uint8_t *alive) {
  int64_t nnodes = (int64_t)orc_nodes_x(g) * orc_nodes_z(g);
  double beta = sp->q * g->dt / (2.0 * sp->m);
  double cx = g->dt / g->dx, cz = g->dt / g->dz;
  for (int64_t a = 0; a < sp->n; ++a) {
    int32_t node[4], ci, ck;
    double W[4];
    cell_weights(g, sp->xi_x[a], sp->xi_z[a], node, W, &ci, &ck);
    double B[3];
    particle_B(g, H, sp->xi_x[a], sp->xi_z[a], mode, B);
    double u[3] = {sp->ux[a], sp->uy[a], sp->uz[a]};
    double R[9];
    double gam = particle_gamma(g, E, sp->q, sp->m, u, node, W, mode);
    orc_response_g(sp->q, sp->m, g->dt, gam, B, R);
    double Ep[3];
    for (int r = 0; r < 3; ++r) {
      const double *f = Ebar + r * nnodes;
      Ep[r] = W[0] * f[node[0]] + W[1] * f[node[1]] + W[2] * f[node[2]] + W[3] * f[node[3]];
    }
    double av[3] = {u[0] + beta * Ep[0], u[1] + beta * Ep[1], u[2] + beta * Ep[2]};
    double un[3];
    for (int r = 0; r < 3; ++r) {
      double ub = R[3 * r] * av[0] + R[3 * r + 1] * av[1] + R[3 * r + 2] * av[2];
      un[r] = 2.0 * ub - u[r];
    }
    double g1 = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
    double x = sp->xi_x[a] + cx * (un[0] / g1);
    double z = sp->xi_z[a] + cz * (un[2] / g1);
    uint8_t ok = 1;
    if (g->bc_x == ORC_PERIODIC) {
      if (x < 0.0) x += (double)g->nx;
      if (x >= (double)g->nx) x -= (double)g->nx;
    } else if (x < 0.0 || x >= (double)g->nx) {
      ok = 0;
    }
    if (z < 0.0) z += (double)g->nz;
    if (z >= (double)g->nz) z -= (double)g->nz;
    sp->xi_x[a] = x;
    sp->xi_z[a] = z;
    sp->ux[a] = un[0];
    sp->uy[a] = un[1];
    sp->uz[a] = un[2];
    alive[a] = ok;
  }
}

/* Stable counting sort by cell key; removed particles are dropped. */
int64_t orc_sort(const orc_grid *g, orc_species *sp, const uint8_t *alive, int64_t *perm_out) {
  int64_t ncells = (int64_t)g->nx * g->nz;
  int64_t n = sp->n;
  int64_t *start = (int64_t *)calloc((size_t)ncells + 1, sizeof(int64_t));
  int64_t *key = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t *perm = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  for (int64_t a = 0; a < n; ++a) {
    if (alive && !alive[a]) {
      key[a] = -1;
      continue;
    }
    int64_t i = (int64_t)floor(sp->xi_x[a]);
    int64_t k = (int64_t)floor(sp->xi_z[a]);
    key[a] = k * g->nx + i;
    start[key[a] + 1] += 1;
  }
  for (int64_t c = 0; c < ncells; ++c) start[c + 1] += start[c];
  int64_t n_new = start[ncells];
  for (int64_t a = 0; a < n; ++a) {
    if (key[a] < 0) continue;
    perm[start[key[a]]++] = a;
  }
  double *tmp = (double *)malloc((size_t)(n_new > 0 ? n_new : 1) * sizeof(double));
  double *arrs[6] = {sp->xi_x, sp->xi_z, sp->ux, sp->uy, sp->uz, sp->w};
  for (int v = 0; v < 6; ++v) {
    for (int64_t j = 0; j < n_new; ++j) tmp[j] = arrs[v][perm[j]];
    memcpy(arrs[v], tmp, (size_t)n_new * sizeof(double));
  }
  if (sp->id) {
    int64_t *tid = (int64_t *)malloc((size_t)(n_new > 0 ? n_new : 1) * sizeof(int64_t));
    for (int64_t j = 0; j < n_new; ++j) tid[j] = sp->id[perm[j]];
    memcpy(sp->id, tid, (size_t)n_new * sizeof(int64_t));
    free(tid);
  }
  if (perm_out) memcpy(perm_out, perm, (size_t)n_new * sizeof(int64_t));
  sp->n = n_new;
  free(tmp);
  free(perm);
  free(key);
  free(start);
  return n_new;
}
