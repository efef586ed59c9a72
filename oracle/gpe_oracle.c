/*
 * gpe_oracle.c -- plain CPU FP64 reference of the GPE + Cahn-Hilliard time
 * step of arXiv 2011.00814 (J.-J. Huang).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU library.  Shares no
 * code with it.
 *
 * Everything is written as plain loops over cells and faces, in the order the
 * paper presents the method:
 *   Sec. 2  mixture laws rho(phi), eta(phi), nu = eta/rho; chemical potential
 *           mu = 4 a phi (phi^2 - 1) - kappa lap(phi), a = 3/(4W), kappa = 3W/8;
 *           surface-tension force -sigma phi grad(mu); buoyancy (rho - rho_ref) g;
 *           bulk viscosity eta_b = eta.
 *   Sec. 3  staggered second-order differences for div u, variable-nu pressure
 *           diffusion, momentum convection with 4-point averaged transverse
 *           velocity, the four variable-viscosity stress sub-stencils with
 *           corner-averaged eta, the face surface-tension term and the
 *           transversely averaged pressure gradient ([1,4,1]/6 in 2-D, the
 *           3x3 [16,4,1]/36 weights in 3-D); TVD-RK3 for (p, u) with phi and
 *           mu frozen; space-time-averaged centre velocity; isotropic lattice
 *           stencils for the CH derivatives; TVD-RK2 (2-D) / RK4 (3-D) for phi.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - u[i] is the low-x face of cell i (divergence stencil index convention).
 *   - rho at a velocity point is the mean of the two adjacent cells.
 *   - the bulk term d/dx(eta D) pairs eta_i with D_i (same cell).
 *   - the factor 2 of d/dx(2 eta du/dx) multiplies the printed sub-stencil.
 *   - stencils are evaluated difference-first (sum of w (f_nb - f_c)), and
 *     the Runge-Kutta combinations in increment form (see orc_run).
 *   - boundaries sit on cell faces; normal velocity there is 0; ghosts mirror
 *     scalars, negate the normal velocity, and negate (no-slip wall) or keep
 *     (symmetry plane, axis) the tangential velocity.
 *   - CH transport in conservative form: minus the isotropic divergence of
 *     phi * u_hat (identical to the advective form for uniform u_hat).
 *   - phi is clamped to [-1, 1] inside rho(phi), eta(phi) only.
 *   - axisymmetric terms in exact cylindrical finite-volume form; the CH
 *     Laplacian weights every lattice link by its mid-point radius, the CH
 *     flux is the isotropic divergence of r * phi * u_hat over r.
 */
#include "gpe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Lattice velocity sets for the isotropic CH stencils (textbook weights,    */
/* classified by the number of non-zero components of the lattice vector).   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int q;
  int e[27][3];
  double w[27];
} lattice_t;

static int build_lattice(int which, int dim, lattice_t* L) {
  double wt[4];
  if (which == 9 && dim == 2) {
    wt[0] = 4.0 / 9.0; wt[1] = 1.0 / 9.0; wt[2] = 1.0 / 36.0; wt[3] = 0.0;
  } else if (which == 15 && dim == 3) {
    wt[0] = 2.0 / 9.0; wt[1] = 1.0 / 9.0; wt[2] = 0.0; wt[3] = 1.0 / 72.0;
  } else if (which == 19 && dim == 3) {
    wt[0] = 1.0 / 3.0; wt[1] = 1.0 / 18.0; wt[2] = 1.0 / 36.0; wt[3] = 0.0;
  } else if (which == 27 && dim == 3) {
    wt[0] = 8.0 / 27.0; wt[1] = 2.0 / 27.0; wt[2] = 1.0 / 54.0; wt[3] = 1.0 / 216.0;
  } else {
    return -1;
  }
  int q = 0;
  int zr = (dim == 3) ? 1 : 0;
  for (int ez = -zr; ez <= zr; ++ez)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ex = -1; ex <= 1; ++ex) {
        int nnz = (ex != 0) + (ey != 0) + (ez != 0);
        if (wt[nnz] == 0.0) continue;
        L->e[q][0] = ex; L->e[q][1] = ey; L->e[q][2] = ez;
        L->w[q] = wt[nnz];
        ++q;
      }
  L->q = q;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Grid, index maps and ghost rules                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_params* P;
  int n[3];
  int dim;
} grid_t;

typedef struct { int v[3]; } ix3;

static ix3 mk(int i, int j, int k) { ix3 x; x.v[0] = i; x.v[1] = j; x.v[2] = k; return x; }
static ix3 sh(ix3 x, int a, int d) { x.v[a] += d; return x; }

static size_t lin(const grid_t* g, int i, int j, int k) {
  return ((size_t)k * g->n[1] + j) * g->n[0] + i;
}

/* Cell index c along an axis of n cells; *refl receives the BC of the mirror
 * crossed (0 when none). */
static int map_cell(int c, int n, int lo, int hi, int* refl) {
  *refl = 0;
  if (c < 0) {
    if (lo == ORC_BC_PERIODIC) return ((c % n) + n) % n;
    *refl = lo;
    return -1 - c;
  }
  if (c >= n) {
    if (hi == ORC_BC_PERIODIC) return c % n;
    *refl = hi;
    return 2 * n - 1 - c;
  }
  return c;
}

/* Face index f (the low face of cell f) along its own normal axis.  Returns
 * -1 when the face lies on a wall / symmetry plane (value 0); flips *sign
 * for a mirrored face. */
static int map_face(int f, int n, int lo, int hi, int* sign) {
  if (lo == ORC_BC_PERIODIC) return ((f % n) + n) % n;
  if (f <= 0) {
    if (f == 0) return -1;
    *sign = -*sign;
    return -f;
  }
  if (f >= n) {
    if (f == n) return -1;
    (void)hi;
    *sign = -*sign;
    return 2 * n - f;
  }
  return f;
}

/* Scalar at a cell centre (p, phi, mu, rho, eta, nu, D): even mirror. */
static double Sc(const grid_t* g, const double* f, ix3 x) {
  int idx[3] = {0, 0, 0}, r;
  for (int a = 0; a < g->dim; ++a)
    idx[a] = map_cell(x.v[a], g->n[a], g->P->bc[2 * a], g->P->bc[2 * a + 1], &r);
  return f[lin(g, idx[0], idx[1], idx[2])];
}

/* Component c of the face-staggered velocity at face index x. */
static double Fv(const grid_t* g, const double* f, int c, ix3 x) {
  int idx[3] = {0, 0, 0}, sign = 1, r;
  for (int a = 0; a < g->dim; ++a) {
    int lo = g->P->bc[2 * a], hi = g->P->bc[2 * a + 1];
    if (a == c) {
      idx[a] = map_face(x.v[a], g->n[a], lo, hi, &sign);
      if (idx[a] < 0) return 0.0;
    } else {
      idx[a] = map_cell(x.v[a], g->n[a], lo, hi, &r);
      if (r == ORC_BC_WALL) sign = -sign;
    }
  }
  return sign * f[lin(g, idx[0], idx[1], idx[2])];
}

/* Component c of a cell-centred vector (the centre velocity). */
static double Cv(const grid_t* g, const double* f, int c, ix3 x) {
  int idx[3] = {0, 0, 0}, sign = 1, r;
  for (int a = 0; a < g->dim; ++a) {
    idx[a] = map_cell(x.v[a], g->n[a], g->P->bc[2 * a], g->P->bc[2 * a + 1], &r);
    if (r != 0 && (a == c || r == ORC_BC_WALL)) sign = -sign;
  }
  return sign * f[lin(g, idx[0], idx[1], idx[2])];
}

static int is_boundary_face(const grid_t* g, int a, ix3 x) {
  return g->P->bc[2 * a] != ORC_BC_PERIODIC && x.v[a] == 0;
}

/* Axisymmetric radii: cell centre r_j = j + 1/2, low radial face of row j at
 * R_j = j. */
static double rc(int j) { return j + 0.5; }
static double rf(int j) { return (double)j; }

static int setup(const orc_params* P, grid_t* g) {
  if (!P || (P->dim != 2 && P->dim != 3)) return -1;
  g->P = P;
  g->dim = P->dim;
  for (int a = 0; a < 3; ++a) g->n[a] = P->n[a];
  if (P->dim == 2 && P->n[2] != 1) return -1;
  for (int a = 0; a < P->dim; ++a) {
    if (P->n[a] < 2) return -1;
    if ((P->bc[2 * a] == ORC_BC_PERIODIC) != (P->bc[2 * a + 1] == ORC_BC_PERIODIC)) return -1;
  }
  if (P->axisym && (P->dim != 2 || P->bc[2] != ORC_BC_SYMMETRY)) return -1;
  return 0;
}

static size_t ncells(const grid_t* g) { return (size_t)g->n[0] * g->n[1] * g->n[2]; }

/* ------------------------------------------------------------------------ */
/* Material laws (Sec. 2, mixture density and viscosity)                     */
/* ------------------------------------------------------------------------ */
static double clamp1(double x) { return x < -1.0 ? -1.0 : (x > 1.0 ? 1.0 : x); }
static double rho_of(const orc_params* P, double phi) {
  double f = clamp1(phi);
  return 0.5 * (P->rho_l * (1.0 + f) + P->rho_g * (1.0 - f));
}
static double eta_of(const orc_params* P, double phi) {
  double f = clamp1(phi);
  return 0.5 * (P->eta_l * (1.0 + f) + P->eta_g * (1.0 - f));
}

/* ------------------------------------------------------------------------ */
/* Chemical potential (Sec. 2) with the isotropic Laplacian (Sec. 3)         */
/* ------------------------------------------------------------------------ */
int orc_mu(const orc_params* P, const double* phi, double* mu) {
  grid_t g;
  lattice_t L;
  if (setup(P, &g) || build_lattice(P->lattice, P->dim, &L)) return -1;
  const double a = 3.0 / (4.0 * P->width);
  const double kappa = 3.0 * P->width / 8.0;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        double pc = phi[lin(&g, i, j, k)];
        double lap = 0.0;
        for (int q = 0; q < L.q; ++q) {
          if (!L.e[q][0] && !L.e[q][1] && !L.e[q][2]) continue;
          ix3 y = mk(i + L.e[q][0], j + L.e[q][1], k + L.e[q][2]);
          double rr = P->axisym ? (rc(j) + 0.5 * L.e[q][1]) / rc(j) : 1.0;
          lap += L.w[q] * rr * (Sc(&g, phi, y) - pc);
        }
        lap *= 6.0;
        mu[lin(&g, i, j, k)] = 4.0 * a * pc * (pc * pc - 1.0) - kappa * lap;
      }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Flow right-hand sides (Sec. 3, semi-discrete pressure/momentum system)    */
/* ------------------------------------------------------------------------ */
static double face_rhs(const grid_t* g, int a, ix3 x, const double* p,
                       const double* const vel[3], const double* rho,
                       const double* eta, const double* D, const double* phi,
                       const double* mu) {
  const orc_params* P = g->P;
  const int dim = g->dim;
  const int axi = P->axisym;
  const ix3 lo = sh(x, a, -1); /* the cell below the face along a */
  const double ua = Fv(g, vel[a], a, x);
  const double rho_f = 0.5 * (Sc(g, rho, lo) + Sc(g, rho, x));

  /* convection: u_a d_a u_a + sum_b ubar_b d_b u_a */
  double C = ua * (Fv(g, vel[a], a, sh(x, a, 1)) - Fv(g, vel[a], a, sh(x, a, -1))) * 0.5;
  for (int b = 0; b < dim; ++b) {
    if (b == a) continue;
    double ub = 0.25 * (Fv(g, vel[b], b, x) + Fv(g, vel[b], b, lo) +
                        Fv(g, vel[b], b, sh(x, b, 1)) + Fv(g, vel[b], b, sh(lo, b, 1)));
    C += ub * (Fv(g, vel[a], a, sh(x, b, 1)) - Fv(g, vel[a], a, sh(x, b, -1))) * 0.5;
  }

  /* viscous stress divergence */
  double V;
  const double eta_hi = Sc(g, eta, x), eta_lo = Sc(g, eta, lo);
  const double ua_p = Fv(g, vel[a], a, sh(x, a, 1)), ua_m = Fv(g, vel[a], a, sh(x, a, -1));
  const int printed = axi && (P->flags & ORC_AXI_PRINTED);
  if (axi && a == 1 && printed) {
    /* radial face, the r-equation as printed: d_r(2 eta d_r u_r) plus
     * (eta/r)(d_r u_r - u_r/r), d_r u_r by the central difference of the
     * two neighbouring radial faces, eta of the face the mean of its cells */
    const double R = rf(x.v[1]);
    V = 2.0 * (eta_hi * (ua_p - ua) - eta_lo * (ua - ua_m));
    V += 0.5 * (eta_lo + eta_hi) / R * (0.5 * (ua_p - ua_m) - ua / R);
  } else if (axi && a == 1) {
    /* radial face at radius R_j: (1/r) d_r(r 2 eta d_r u_r) - 2 eta u_r / r^2 */
    const int j = x.v[1];
    const double R = rf(j);
    V = (rc(j) * 2.0 * eta_hi * (ua_p - ua) - rc(j - 1) * 2.0 * eta_lo * (ua - ua_m)) / R;
    V -= 2.0 * 0.5 * (eta_lo + eta_hi) * ua / (R * R);
  } else {
    V = 2.0 * (eta_hi * (ua_p - ua) - eta_lo * (ua - ua_m));
  }
  for (int b = 0; b < dim; ++b) {
    if (b == a) continue;
    double ep = 0.25 * (eta_hi + Sc(g, eta, sh(x, b, 1)) + eta_lo + Sc(g, eta, sh(lo, b, 1)));
    double em = 0.25 * (eta_hi + Sc(g, eta, sh(x, b, -1)) + eta_lo + Sc(g, eta, sh(lo, b, -1)));
    double fp = ep * ((Fv(g, vel[a], a, sh(x, b, 1)) - ua) +
                      (Fv(g, vel[b], b, sh(x, b, 1)) - Fv(g, vel[b], b, sh(lo, b, 1))));
    double fm = em * ((ua - Fv(g, vel[a], a, sh(x, b, -1))) +
                      (Fv(g, vel[b], b, x) - Fv(g, vel[b], b, lo)));
    if (axi && b == 1 && printed) {
      /* axial face, the z-equation as printed: d_r[eta (d_r u_z + d_z u_r)]
       * plus (eta/r) d_r u_z, d_r u_z by the central difference of the two
       * radial neighbours, eta of the face the mean of its cells */
      V += fp - fm;
      V += 0.5 * (eta_lo + eta_hi) / rc(x.v[1]) * 0.5 *
           (Fv(g, vel[a], a, sh(x, b, 1)) - Fv(g, vel[a], a, sh(x, b, -1)));
    } else if (axi && b == 1) {
      /* axial face: (1/r) d_r [ r eta (d_r u_z + d_z u_r) ] */
      const int j = x.v[1];
      V += (rf(j + 1) * fp - rf(j) * fm) / rc(j);
    } else {
      V += fp - fm;
    }
  }
  if (!(P->flags & ORC_NO_BULK)) V += eta_hi * Sc(g, D, x) - eta_lo * Sc(g, D, lo);

  /* averaged pressure gradient */
  double G;
#define DP(y) (Sc(g, p, (y)) - Sc(g, p, sh((y), a, -1)))
  if (P->flags & ORC_NO_PAVG) {
    G = DP(x);
  } else if (dim == 2) {
    const int b = 1 - a;
    G = (4.0 * DP(x) + DP(sh(x, b, 1)) + DP(sh(x, b, -1))) / 6.0;
  } else {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    G = (16.0 * DP(x) +
         4.0 * (DP(sh(x, b, 1)) + DP(sh(x, b, -1)) + DP(sh(x, c, 1)) + DP(sh(x, c, -1))) +
         (DP(sh(sh(x, b, 1), c, 1)) + DP(sh(sh(x, b, -1), c, -1)) +
          DP(sh(sh(x, b, -1), c, 1)) + DP(sh(sh(x, b, 1), c, -1)))) / 36.0;
  }
#undef DP

  /* surface tension -sigma phi d_a mu, buoyancy (rho - rho_ref) g_a */
  const double S = -P->sigma * (Sc(g, phi, x) + Sc(g, phi, lo)) *
                   (Sc(g, mu, x) - Sc(g, mu, lo)) * 0.5;
  const double B = (rho_f - P->rho_ref) * P->g[a];

  return -C + (-G + V + S + B) / rho_f;
}

int orc_flow_rhs(const orc_params* P, const double* p, const double* u,
                 const double* v, const double* w, const double* phi,
                 double* Lp, double* Lu, double* Lv, double* Lw) {
  grid_t g;
  if (setup(P, &g)) return -1;
  if (P->dim == 3 && (!w || !Lw)) return -1;
  const size_t N = ncells(&g);
  double* rho = malloc(N * sizeof(double));
  double* eta = malloc(N * sizeof(double));
  double* nu = malloc(N * sizeof(double));
  double* mu = malloc(N * sizeof(double));
  double* D = malloc(N * sizeof(double));
  const double* vel[3] = {u, v, w};
  double* out[3] = {Lu, Lv, Lw};
  int rcode = 0;
  if (!rho || !eta || !nu || !mu || !D) { rcode = -1; goto done; }

  /* frozen material fields (phi and mu fixed during the flow step) */
  for (size_t c = 0; c < N; ++c) {
    rho[c] = rho_of(P, phi[c]);
    eta[c] = eta_of(P, phi[c]);
    nu[c] = eta[c] / rho[c];
  }
  if (orc_mu(P, phi, mu)) { rcode = -1; goto done; }

  /* velocity divergence at cell centres */
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        ix3 x = mk(i, j, k);
        double d = 0.0;
        for (int a = 0; a < g.dim; ++a) {
          if (P->axisym && a == 1)
            d += (rf(j + 1) * Fv(&g, v, 1, sh(x, 1, 1)) - rf(j) * Fv(&g, v, 1, x)) / rc(j);
          else
            d += Fv(&g, vel[a], a, sh(x, a, 1)) - Fv(&g, vel[a], a, x);
        }
        D[lin(&g, i, j, k)] = d;
      }

  /* pressure equation: dp/dt = -rho cs^2 D + div(nu grad p) */
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        ix3 x = mk(i, j, k);
        size_t c = lin(&g, i, j, k);
        double pc = p[c], nc = nu[c];
        double diff = 0.0;
        for (int a = 0; a < g.dim; ++a) {
          double np = 0.5 * (nc + Sc(&g, nu, sh(x, a, 1)));
          double nm = 0.5 * (nc + Sc(&g, nu, sh(x, a, -1)));
          double fp = np * (Sc(&g, p, sh(x, a, 1)) - pc);
          double fm = nm * (pc - Sc(&g, p, sh(x, a, -1)));
          if (P->axisym && a == 1)
            diff += (rf(j + 1) * fp - rf(j) * fm) / rc(j);
          else
            diff += fp - fm;
        }
        Lp[c] = -rho[c] * P->cs2 * D[c] + diff;
      }

  /* momentum equations at the faces */
  for (int a = 0; a < g.dim; ++a) {
    double* La = out[a];
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          ix3 x = mk(i, j, k);
          size_t c = lin(&g, i, j, k);
          if (is_boundary_face(&g, a, x))
            La[c] = 0.0;
          else
            La[c] = face_rhs(&g, a, x, p, vel, rho, eta, D, phi, mu);
        }
  }

done:
  free(rho); free(eta); free(nu); free(mu); free(D);
  return rcode;
}

/* ------------------------------------------------------------------------ */
/* Cahn-Hilliard right-hand side (Sec. 2 CH equation, Sec. 3 isotropic       */
/* stencils), conservative transport of phi by the frozen centre velocity    */
/* ------------------------------------------------------------------------ */
int orc_ch_rhs(const orc_params* P, const double* phi, const double* uc,
               const double* vc, const double* wc, double* Lphi) {
  grid_t g;
  lattice_t L;
  if (setup(P, &g) || build_lattice(P->lattice, P->dim, &L)) return -1;
  const size_t N = ncells(&g);
  double* mu = malloc(N * sizeof(double));
  if (!mu) return -1;
  if (orc_mu(P, phi, mu)) { free(mu); return -1; }
  const double* vel[3] = {uc, vc, wc};
  const int advective = (P->flags & ORC_ADVECTIVE_CH) != 0;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        size_t c = lin(&g, i, j, k);
        double flux = 0.0, lap = 0.0;
        double grad[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < L.q; ++q) {
          if (!L.e[q][0] && !L.e[q][1] && !L.e[q][2]) continue;
          ix3 y = mk(i + L.e[q][0], j + L.e[q][1], k + L.e[q][2]);
          double rr = P->axisym ? (rc(j) + 0.5 * L.e[q][1]) / rc(j) : 1.0;
          lap += L.w[q] * rr * (Sc(&g, mu, y) - mu[c]);
          if (advective) {
            double py = Sc(&g, phi, y);
            for (int a = 0; a < g.dim; ++a) grad[a] += L.w[q] * L.e[q][a] * py;
          } else {
            double py = Sc(&g, phi, y);
            double ef = 0.0;
            for (int a = 0; a < g.dim; ++a) ef += L.e[q][a] * py * Cv(&g, vel[a], a, y);
            if (P->axisym) {
              /* isotropic divergence of r * phi * u_hat, divided by r_j; the
               * neighbour's radius is that of the in-domain cell it mirrors */
              int refl;
              int jm = map_cell(j + L.e[q][1], g.n[1], P->bc[2], P->bc[3], &refl);
              flux += L.w[q] * (rc(jm) / rc(j)) * ef;
            } else {
              flux += L.w[q] * ef;
            }
          }
        }
        if (advective) {
          flux = 0.0;
          for (int a = 0; a < g.dim; ++a) flux += vel[a][c] * grad[a];
        }
        Lphi[c] = -3.0 * flux + 6.0 * P->mob * lap;
      }
  free(mu);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One full time step (Sec. 3): flow TVD-RK3 with phi frozen, centre         */
/* velocity averaged in space and time, then the CH sub-step.                */
/* ------------------------------------------------------------------------ */
int orc_run(const orc_params* P, double* p, double* u, double* v, double* w,
            double* phi, long nsteps) {
  grid_t g;
  lattice_t L;
  if (setup(P, &g) || build_lattice(P->lattice, P->dim, &L)) return -1;
  if (P->dim == 3 && !w) return -1;
  const int dim = g.dim;
  const size_t N = ncells(&g);
  const double dt = P->dt;
  const int ch_rk = P->ch_rk ? P->ch_rk : (dim == 2 ? 2 : 4);
  if (ch_rk != 2 && ch_rk != 4) return -1;

  /* scratch: 3 RHS sets and 2 stage sets of (p, u, v, w); 3 centre
   * velocities; 5 phi-sized arrays */
  const int nq = 1 + dim;
  double* buf = calloc(N * (size_t)(3 * nq + 3 + 5 + 3), sizeof(double));
  if (!buf) return -1;
  double* q0[4] = {p, u, v, w};
  double *q1[4], *q2[4], *Lq[4];
  for (int f = 0; f < nq; ++f) {
    q1[f] = buf + (size_t)f * N;
    q2[f] = buf + (size_t)(nq + f) * N;
    Lq[f] = buf + (size_t)(2 * nq + f) * N;
  }
  double* uh[3];
  for (int a = 0; a < 3; ++a) uh[a] = buf + (size_t)(3 * nq + a) * N;
  double* ph1 = buf + (size_t)(3 * nq + 3) * N;
  double* ph2 = ph1 + N;
  double* Lph = ph2 + N;
  double* acc = Lph + N;
  double* uold = acc + N; /* 3 arrays: u^n saved for the centre velocity */
  /* map (p, u, v, w) slot f -> q arrays; slot 0 is p, slot 1+a is velocity a */
#define QV(qs, a) ((qs)[1 + (a)])

  for (long step = 0; step < nsteps; ++step) {
    for (int a = 0; a < dim; ++a) memcpy(uold + (size_t)a * N, QV(q0, a), N * sizeof(double));

    /* ---- flow: TVD-RK3 (or the RK2 ablation), phi frozen ---- */
    if (orc_flow_rhs(P, q0[0], QV(q0, 0), QV(q0, 1), dim == 3 ? QV(q0, 2) : NULL, phi,
                     Lq[0], QV(Lq, 0), QV(Lq, 1), dim == 3 ? QV(Lq, 2) : NULL)) {
      free(buf);
      return -1;
    }
    for (int f = 0; f < nq; ++f)
      for (size_t c = 0; c < N; ++c) q1[f][c] = q0[f][c] + dt * Lq[f][c];
    if (orc_flow_rhs(P, q1[0], QV(q1, 0), QV(q1, 1), dim == 3 ? QV(q1, 2) : NULL, phi,
                     Lq[0], QV(Lq, 0), QV(Lq, 1), dim == 3 ? QV(Lq, 2) : NULL)) {
      free(buf);
      return -1;
    }
    /* The Shu-Osher combinations a q^n + (1 - a)(q^(s) + dt L) are written
     * in the algebraically identical increment form
     * q^n + (1 - a)((q^(s) - q^n) + dt L), which returns q^n exactly when
     * the right-hand side vanishes (a steady state stays bitwise steady). */
    if (P->flags & ORC_FLOW_RK2) {
      for (int f = 0; f < nq; ++f)
        for (size_t c = 0; c < N; ++c)
          q0[f][c] = q0[f][c] + 0.5 * ((q1[f][c] - q0[f][c]) + dt * Lq[f][c]);
    } else {
      for (int f = 0; f < nq; ++f)
        for (size_t c = 0; c < N; ++c)
          q2[f][c] = q0[f][c] + 0.25 * ((q1[f][c] - q0[f][c]) + dt * Lq[f][c]);
      if (orc_flow_rhs(P, q2[0], QV(q2, 0), QV(q2, 1), dim == 3 ? QV(q2, 2) : NULL, phi,
                       Lq[0], QV(Lq, 0), QV(Lq, 1), dim == 3 ? QV(Lq, 2) : NULL)) {
        free(buf);
        return -1;
      }
      for (int f = 0; f < nq; ++f)
        for (size_t c = 0; c < N; ++c)
          q0[f][c] = q0[f][c] + 2.0 / 3.0 * ((q2[f][c] - q0[f][c]) + dt * Lq[f][c]);
    }

    /* ---- centre velocity at t^{n+1/2}: mean over the two faces of the cell
     *      and over the old and new time levels ---- */
    for (int a = 0; a < dim; ++a) {
      const double* un = uold + (size_t)a * N;
      const double* unew = QV(q0, a);
#pragma omp parallel for collapse(2) schedule(static)
      for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
          for (int i = 0; i < g.n[0]; ++i) {
            ix3 x = mk(i, j, k);
            uh[a][lin(&g, i, j, k)] =
                0.25 * ((Fv(&g, un, a, x) + Fv(&g, un, a, sh(x, a, 1))) +
                        (Fv(&g, unew, a, x) + Fv(&g, unew, a, sh(x, a, 1))));
          }
    }

    /* ---- CH sub-step with the centre velocity frozen ---- */
    const double* w3 = dim == 3 ? uh[2] : NULL;
    if (ch_rk == 2) {
      /* TVD-RK2 as phi* + (a + b)/2 with the increments a = dt L(phi*),
       * b = dt L(phi* + a): the stage-1 increment is kept rather than
       * recovered as (phi* + a) - phi* (the same form as RK4 below) */
      double* ka = acc;
      orc_ch_rhs(P, phi, uh[0], uh[1], w3, Lph);
      for (size_t c = 0; c < N; ++c) { ka[c] = dt * Lph[c]; ph1[c] = phi[c] + ka[c]; }
      orc_ch_rhs(P, ph1, uh[0], uh[1], w3, Lph);
      for (size_t c = 0; c < N; ++c) phi[c] = phi[c] + 0.5 * (ka[c] + dt * Lph[c]);
    } else {
      /* classic RK4: a, b, c, d increments; the sum (a + 2b + 2c + d)/6 */
      double* ka = acc;              /* a, then running weighted sum */
      orc_ch_rhs(P, phi, uh[0], uh[1], w3, Lph);
      for (size_t c = 0; c < N; ++c) { ka[c] = dt * Lph[c]; ph1[c] = phi[c] + 0.5 * ka[c]; }
      orc_ch_rhs(P, ph1, uh[0], uh[1], w3, Lph);            /* b */
      for (size_t c = 0; c < N; ++c) { ph2[c] = dt * Lph[c]; }
      for (size_t c = 0; c < N; ++c) { ka[c] += 2.0 * ph2[c]; ph1[c] = phi[c] + 0.5 * ph2[c]; }
      orc_ch_rhs(P, ph1, uh[0], uh[1], w3, Lph);            /* c */
      for (size_t c = 0; c < N; ++c) { ph2[c] = dt * Lph[c]; }
      for (size_t c = 0; c < N; ++c) { ka[c] += 2.0 * ph2[c]; ph1[c] = phi[c] + ph2[c]; }
      orc_ch_rhs(P, ph1, uh[0], uh[1], w3, Lph);            /* d */
      for (size_t c = 0; c < N; ++c) {
        ka[c] += dt * Lph[c];
        phi[c] = phi[c] + ka[c] / 6.0;
      }
    }
  }
#undef QV
  free(buf);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */
int orc_diagnostics(const orc_params* P, const double* p, const double* u,
                    const double* v, const double* w, const double* phi,
                    double* out) {
  grid_t g;
  if (setup(P, &g)) return -1;
  const double* vel[3] = {u, v, w};
  double mass = 0.0, ke = 0.0, maxdiv = 0.0, pmin = INFINITY, pmax = -INFINITY, umax = 0.0;
  int finite = 1;
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        ix3 x = mk(i, j, k);
        size_t c = lin(&g, i, j, k);
        double wr = P->axisym ? rc(j) : 1.0;
        mass += wr * phi[c];
        if (phi[c] < pmin) pmin = phi[c];
        if (phi[c] > pmax) pmax = phi[c];
        if (!isfinite(phi[c]) || !isfinite(p[c])) finite = 0;
        double d = 0.0;
        for (int a = 0; a < g.dim; ++a) {
          double ua = vel[a][c];
          if (!isfinite(ua)) finite = 0;
          if (fabs(ua) > umax) umax = fabs(ua);
          double rho_f = 0.5 * (rho_of(P, Sc(&g, phi, sh(x, a, -1))) + rho_of(P, phi[c]));
          double wf = (P->axisym && a == 1) ? rf(j) : wr;
          ke += 0.5 * rho_f * ua * ua * wf;
          if (P->axisym && a == 1)
            d += (rf(j + 1) * Fv(&g, v, 1, sh(x, 1, 1)) - rf(j) * Fv(&g, v, 1, x)) / rc(j);
          else
            d += Fv(&g, vel[a], a, sh(x, a, 1)) - Fv(&g, vel[a], a, x);
        }
        if (fabs(d) > maxdiv) maxdiv = fabs(d);
      }
  out[0] = mass; out[1] = ke; out[2] = maxdiv; out[3] = pmin; out[4] = pmax;
  out[5] = umax; out[6] = finite;
  (void)p;
  return 0;
}
