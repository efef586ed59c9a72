/*
 * gpe_oracle.h -- CPU FP64 reference ("oracle") of one time step of the
 * general-pressure-equation (GPE) + Cahn-Hilliard two-phase method of
 * J.-J. Huang, "Numerical simulation of two-phase incompressible viscous
 * flows using general pressure equation" (arXiv 2011.00814).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference the GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Units: lattice units, grid spacing dx = 1.  All arrays are caller-owned,
 * double precision, shape (nz, ny, nx) with x fastest (nz = 1 in 2D).
 * Face arrays have the same shape as cell arrays: u[k][j][i] is the
 * x-velocity on the LOW-x face of cell (i,j,k) (Sec. 3, staggered layout and
 * the index convention of the divergence stencil); v and w likewise.
 *
 * Axisymmetric geometry (Sec. 2, axisymmetric equation set): x is the axial
 * coordinate z, y is the radial coordinate r (cell centre r_j = j + 1/2),
 * u = u_z, v = u_r; the y-low boundary is the axis and must be SYMMETRY.
 */
#ifndef GPE_ORACLE_H
#define GPE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1, ORC_BC_SYMMETRY = 2 };

/* Ablation switches (oracle only; the paper's own ablation studies). */
enum {
  ORC_NO_PAVG      = 1,  /* pressure gradient without transverse averaging  */
  ORC_NO_BULK      = 2,  /* bulk viscosity eta_b = 0 instead of eta          */
  ORC_FLOW_RK2     = 4,  /* TVD-RK2 instead of TVD-RK3 for (p, u)            */
  ORC_ADVECTIVE_CH = 8,  /* CH transport in advective form u.grad(phi)       */
  ORC_AXI_PRINTED  = 16  /* axisymmetric viscous terms in the form printed in
                            Sec. 2 (Cartesian stress differences plus
                            (eta/r) d_r u_z and (eta/r)(d_r u_r - u_r/r))
                            instead of the exact cylindrical form            */
};

typedef struct {
  int dim;        /* 2 or 3                                                  */
  int axisym;     /* 1: 2-D axisymmetric (x axial, y radial)                 */
  int n[3];       /* cells along x, y, z (n[2] = 1 in 2-D)                   */
  int bc[6];      /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi                      */
  int lattice;    /* isotropic CH stencil: 9 (D2Q9), 15, 19, 27 (D3Qb)       */
  int flags;      /* ORC_* ablation switches, 0 for the published method     */
  int ch_rk;      /* CH integrator: 2 (TVD-RK2) or 4 (RK4); 0 = 2 in 2-D, 4 in 3-D */
  double dt;      /* time step                                               */
  double cs2;     /* squared sound speed c_s^2                               */
  double rho_l, rho_g, eta_l, eta_g;
  double sigma;   /* physical surface tension (force -sigma phi grad mu)     */
  double mob;     /* Cahn-Hilliard mobility M                                */
  double width;   /* interface width W: a = 3/(4W), kappa = 3W/8            */
  double g[3];    /* body force                                              */
  double rho_ref; /* reference density of the buoyancy term                  */
} orc_params;

/* Advance (p, u, v, w, phi) by nsteps full time steps in place.
 * w may be NULL in 2-D.  Returns 0, or -1 on invalid parameters. */
int orc_run(const orc_params* P, double* p, double* u, double* v, double* w,
            double* phi, long nsteps);

/* Right-hand sides of the semi-discrete flow system for a given state with
 * phi frozen (dp/dt, du/dt, dv/dt, dw/dt).  Boundary-normal faces of
 * walls / symmetry planes get 0.  Lw / w may be NULL in 2-D. */
int orc_flow_rhs(const orc_params* P, const double* p, const double* u,
                 const double* v, const double* w, const double* phi,
                 double* Lp, double* Lu, double* Lv, double* Lw);

/* Chemical potential mu(phi) at every cell. */
int orc_mu(const orc_params* P, const double* phi, double* mu);

/* Right-hand side of the CH equation for phase field phi and frozen
 * cell-centre velocity (uc, vc, wc); wc may be NULL in 2-D. */
int orc_ch_rhs(const orc_params* P, const double* phi, const double* uc,
               const double* vc, const double* wc, double* L);

/* Diagnostics of a state (FP64 sums in a fixed order).
 * out[0] mass = sum phi (sum r_j phi in axisymmetric geometry)
 * out[1] kinetic energy 1/2 sum_faces rho_f u_f^2 (radius-weighted if axisym)
 * out[2] max |div u|     out[3] min phi   out[4] max phi
 * out[5] max |u_f| over all face components
 * out[6] 1 if every value of p, u, v, w, phi is finite, else 0 */
int orc_diagnostics(const orc_params* P, const double* p, const double* u,
                    const double* v, const double* w, const double* phi,
                    double* out);

#ifdef __cplusplus
}
#endif
#endif
