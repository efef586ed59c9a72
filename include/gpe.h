/*
 * gpe.h -- C-ABI of libgpe, an MI355X (gfx950) implementation of the fully
 * explicit time step of the general-pressure-equation (GPE) + Cahn-Hilliard
 * two-phase solver of J.-J. Huang, "Numerical simulation of two-phase
 * incompressible viscous flows using general pressure equation"
 * (arXiv 2011.00814).
 *
 * One time step (Sec. 3) = three TVD-RK3 stages of the pressure equation and
 * the momentum equations on a staggered grid with the phase field frozen,
 * the space-time averaged cell-centre velocity, then the Cahn-Hilliard
 * sub-step (TVD-RK2 in 2-D and axisymmetric geometry, classic RK4 in 3-D).
 *
 * Conventions shared by every call:
 *  - Lattice units: grid spacing dx = 1.  dt and cs2 are free parameters
 *    (the paper fixes cs = dx / (sqrt(3) dt), Sec. 2, general pressure eq.).
 *  - Layout: every field has the cells of shape (nz, ny, nx), x fastest
 *    (nz = 1 in 2-D).  Host arrays (gpe_copy_field, the initial fields) are
 *    dense.  On the device each x row takes gpe_field_pitch elements: in
 *    FP32 with nx >= 64, nx rounded up to a multiple of 64, so that every
 *    row starts on a 256-byte boundary; otherwise nx.  Row j of plane k
 *    starts at element (k ny + j) pitch; the padding is zero and is never
 *    read.  Velocity components are stored on the LOW face of
 *    their cell: u[k][j][i] sits between cells i-1 and i (Sec. 3, index
 *    convention of the divergence stencil).  For walls and symmetry planes
 *    the boundary-normal face of cell 0 is on the boundary and is always 0.
 *  - Axisymmetric geometry (Sec. 2, axisymmetric equations): x is the axial
 *    coordinate z, y the radial coordinate r (cell centres r = j + 1/2),
 *    u = u_z, v = u_r; the y-low boundary is the axis (GPE_BC_SYMMETRY).
 *  - Ownership: the caller owns all device memory (one workspace buffer)
 *    and the HIP stream.  The library never allocates or frees device
 *    memory; gpe_destroy frees host metadata only.
 *  - Errors: every int-returning call returns GPE_OK (0) or a negative
 *    gpe_error code; no exception crosses the ABI.  gpe_strerror names them.
 *  - Threading: one handle per stream; a handle is not thread-safe.
 *  - Precision: GPE_FP64 (reference) or GPE_FP32 (fast).  Reductions of
 *    gpe_diagnostics accumulate in FP64 in both modes.
 */
#ifndef GPE_H
#define GPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum gpe_error {
  GPE_OK = 0,
  GPE_EINVAL = -1,       /* invalid argument or parameter set              */
  GPE_EUNSTABLE = -2,    /* a linear stability estimate is exceeded         */
  GPE_EWORKSPACE = -3,   /* workspace too small or misaligned               */
  GPE_EHIP = -4,         /* a HIP runtime call failed                       */
  GPE_ENONFINITE = -5    /* the state holds NaN / Inf (sticky per handle)   */
};

enum gpe_geometry { GPE_GEOM_2D = 0, GPE_GEOM_AXISYM = 1, GPE_GEOM_3D = 2 };
enum gpe_precision { GPE_FP64 = 0, GPE_FP32 = 1 };
enum gpe_bc { GPE_BC_PERIODIC = 0, GPE_BC_WALL = 1, GPE_BC_SYMMETRY = 2 };
/* isotropic lattice of the CH derivatives (Sec. 3, isotropic schemes) */
enum gpe_lattice { GPE_D2Q9 = 9, GPE_D3Q15 = 15, GPE_D3Q19 = 19, GPE_D3Q27 = 27 };
enum gpe_field { GPE_FIELD_P = 0, GPE_FIELD_U = 1, GPE_FIELD_V = 2, GPE_FIELD_W = 3,
                 GPE_FIELD_PHI = 4 };
enum gpe_copy_dir { GPE_H2D = 0, GPE_D2H = 1 };
/* in-kernel initial phase field, used when gpe_init_state gets h_phi0 = NULL */
enum gpe_init_kind {
  GPE_INIT_NONE = 0,     /* phi = init_amp everywhere                                  */
  GPE_INIT_DROP = 1,     /* phi = tanh(2 (R - r) / init_width): liquid sphere/disc     */
  GPE_INIT_BUBBLE = 2,   /* phi = tanh(2 (r - R) / init_width): gas sphere/disc        */
  GPE_INIT_LAYER = 3,    /* phi = tanh(2 (y - y0(x)) / init_width) (2-D) or in z (3-D),
                            y0 = init_center[1 or 2] + init_amp cos(2 pi x_c / nx)     */
  GPE_INIT_ELLIPSE = 4   /* phi = tanh(2 R (1 - rho) / init_width), R = init_radius,
                            rho = |((x-x0)/a, (y-y0)/b[, (z-z0)/R])|,
                            a = R (1 + init_amp), b = R (1 - init_amp), |init_amp| < 1 */
};

/* Convection term of the Cahn-Hilliard equation (Sec. 2), with the frozen
 * space-time averaged centre velocity u_hat and the isotropic first
 * derivative (Sec. 3):
 *  - GPE_CH_CONSERVATIVE: div(phi u_hat), the isotropic divergence of the
 *    product.  The phase mass sum(phi) is conserved to round-off.  It
 *    differs from the advective form by phi div(u_hat), which couples phi to
 *    the acoustic divergence in the bulk phases; with a light gas phase
 *    (density ratio ~50) that coupling grows at the grid scale.
 *  - GPE_CH_ADVECTIVE: u_hat . grad(phi), the equation as printed; the
 *    phase mass then drifts by O(sum phi div u_hat).
 * The batched ensemble (gpe_ensemble_*) supports the conservative form only. */
enum gpe_ch_transport { GPE_CH_CONSERVATIVE = 0, GPE_CH_ADVECTIVE = 1 };

/* Ablation switches of the 3-D flow discretisation, OR-ed together; 0 is the
 * scheme of the paper.  The paper (Sec. 4, drop coalescence in 3-D) names
 * both the transverse pressure average of the momentum equations' pressure
 * gradient and the bulk viscosity eta_b = eta as needed for stable 3-D runs
 * and demonstrates it by switching each off:
 *  - GPE_SCHEME_NO_PAVG: the pressure gradient at a face is the plain
 *    difference of the two cell pressures (no transverse average);
 *  - GPE_SCHEME_NO_BULK: eta_b = 0, i.e. the term grad(eta_b div u) is
 *    dropped from the momentum equations.
 * Accepted for 3-D geometry only (GPE_EINVAL otherwise) and not by the
 * batched ensemble. */
enum gpe_scheme { GPE_SCHEME_PAPER = 0, GPE_SCHEME_NO_PAVG = 1, GPE_SCHEME_NO_BULK = 2 };

/* Physical and numerical parameters in lattice units (dx = 1). */
typedef struct gpe_params {
  int32_t geometry;        /* gpe_geometry                                             */
  int32_t precision;       /* gpe_precision                                            */
  int32_t n[3];            /* cells along x, y, z; n[2] = 1 unless 3-D; each >= 3;
                              total <= 4e9 cells, and one x-row (2-D) or one x-y
                              plane (3-D) < 2^32 bytes                              */
  int32_t bc[6];           /* gpe_bc of x-lo, x-hi, y-lo, y-hi, z-lo, z-hi; an axis is
                              periodic on both sides or on neither                      */
  int32_t lattice;         /* GPE_D2Q9 in 2-D/axisym; GPE_D3Q15/19/27 in 3-D           */
  int32_t allow_unstable;  /* 1: skip the GPE_EUNSTABLE check of gpe_init_state        */
  int32_t ch_transport;    /* gpe_ch_transport: form of the CH convection term          */
  double dt;               /* time step                                                */
  double cs2;              /* c_s^2 of the pressure equation                          */
  double rho_l, rho_g;     /* densities of liquid (phi = +1) and gas (phi = -1)       */
  double eta_l, eta_g;     /* dynamic viscosities (bulk viscosity eta_b = eta unless
                              GPE_SCHEME_NO_BULK)                                      */
  double sigma;            /* surface tension of the force -sigma phi grad(mu)        */
  double mobility;         /* Cahn-Hilliard mobility M                                */
  double width;            /* interface width W: a = 3/(4W), kappa = 3W/8              */
  double g[3];             /* body force; buoyancy (rho(phi) - rho_ref) g              */
  double rho_ref;          /* reference density absorbed into the pressure            */
  int32_t init_kind;       /* gpe_init_kind (only when h_phi0 == NULL)                 */
  int32_t scheme;          /* gpe_scheme flags; 0 = the paper's scheme                  */
  int32_t zchunk;          /* planes per work-group along the marching axis (z in 3-D,
                              y in 2-D); 0 = chosen by the library.  The work split
                              never changes the result (bitwise).  Single grids only:
                              the batched ensemble chooses its own                     */
  int32_t reserved;        /* 0                                                        */
  double init_center[3];   /* cell-centre coordinates (x_c = i + 1/2)                  */
  double init_radius;
  double init_width;       /* profile width (usually = width)                          */
  double init_amp;
} gpe_params;

/* The paper's problem statement (Sec. 4 set-ups).  The characteristic
 * length L_c is resolved by N_L cells and the characteristic time
 * T_c = L_c / U_c by N_t steps, so that dx = dt = 1 in lattice units,
 * U_c = N_L / N_t and c_s^2 = 1/3 (c_s = dx / (sqrt(3) dt), Sec. 2);
 * rho_L = 1 and sigma_ref = 1 (Sec. 2, chemical potential).  The groups
 * that fix eta_L, sigma and g come in the alternatives below; the length
 * in Oh, Eo and Mo is L_g = L_g_factor L_c (the paper uses the drop
 * diameter 2 L_c in some set-ups and the radius in others). */
enum gpe_time_scale {
  GPE_TIME_NT = 0,       /* U_c = N_L / N_t                                           */
  GPE_TIME_MA = 1        /* U_c = Ma c_s (Mach number of the characteristic velocity) */
};
enum gpe_visc_group {
  GPE_VISC_RE = 0,       /* Re = rho_L U_c L_c / eta_L                                */
  GPE_VISC_OH = 1,       /* Oh = eta_L / sqrt(rho_L sigma L_g)                        */
  GPE_VISC_MO = 2,       /* Mo = g (rho_L - rho_G) eta_L^4 / (rho_L^2 sigma^3)        */
  GPE_VISC_CAPILLARY = 3 /* U_c = sigma / eta_L: eta_L = sigma / U_c                  */
};
enum gpe_st_group {
  GPE_ST_NONE = 0,       /* sigma = 0                                                 */
  GPE_ST_WE = 1,         /* We = rho_L U_c^2 L_c / sigma                              */
  GPE_ST_EO = 2,         /* Eo = g (rho_L - rho_G) L_g^2 / sigma                      */
  GPE_ST_SIGMA = 3,      /* sigma given in lattice units (field sigma)                */
  GPE_ST_CAPILLARY = 4   /* U_c = sigma / eta_L: sigma = U_c eta_L                    */
};
enum gpe_gravity {
  GPE_GRAV_G = 0,        /* g = G U_c^2 / L_c (G dimensionless, may be 0)             */
  GPE_GRAV_FR = 1,       /* |g| = U_c^2 / (Fr^2 L_c) along the direction of G        */
  GPE_GRAV_EO = 2        /* |g| = Eo sigma / ((rho_L - rho_G) L_g^2) along G          */
};
enum gpe_rho_ref_kind {
  GPE_RHO_REF_ZERO = 0, GPE_RHO_REF_LIQUID = 1, GPE_RHO_REF_GAS = 2,
  GPE_RHO_REF_VALUE = 3  /* rho_ref = rho_ref_value rho_L                             */
};

typedef struct gpe_problem {
  int32_t geometry, precision;
  int32_t n[3];
  int32_t bc[6];
  int32_t lattice;
  int32_t ch_transport;    /* gpe_ch_transport, copied to gpe_params                    */
  int32_t scheme;          /* gpe_scheme flags, copied to gpe_params                    */
  int32_t time_scale;      /* gpe_time_scale                                           */
  int32_t visc_group;      /* gpe_visc_group                                           */
  int32_t st_group;        /* gpe_st_group                                             */
  int32_t gravity;         /* gpe_gravity                                              */
  int32_t rho_ref_kind;    /* gpe_rho_ref_kind                                         */
  int32_t reserved;        /* 0                                                        */
  double N_L;              /* cells per characteristic length L_c                     */
  double N_t;              /* steps per T_c (GPE_TIME_NT)                              */
  double Ma;               /* U_c / c_s (GPE_TIME_MA)                                  */
  double L_g_factor;       /* L_g / L_c of Oh, Eo, Mo (0 means 1)                      */
  double r_rho;            /* rho_L / rho_G                                            */
  double r_eta;            /* eta_L / eta_G                                            */
  double Re, Oh, Mo;       /* the one visc_group selects                               */
  double We, Eo, sigma;    /* the one st_group selects; Eo also for GPE_GRAV_EO        */
  double Pe;               /* U_c L_c^2 / (M sigma_ref); 0: M = 0                      */
  double Cn;               /* W / L_c                                                  */
  double G[3];             /* GPE_GRAV_G: body force in U_c^2 / L_c; else direction    */
  double Fr;               /* U_c / sqrt(|g| L_c) (GPE_GRAV_FR)                        */
  double rho_ref_value;    /* GPE_RHO_REF_VALUE: rho_ref / rho_L                       */
} gpe_problem;

/* Diagnostics (FP64 reductions in a fixed order: bitwise reproducible). */
typedef struct gpe_diag {
  int64_t step;            /* completed time steps                                     */
  double t;                /* step * dt (or the value set by gpe_set_step_time)        */
  double mass;             /* sum phi (sum r_j phi in axisymmetric geometry)           */
  double mass_abs0;        /* sum |phi| (r-weighted) of the initial state: normaliser  */
  double ke;               /* 1/2 sum over faces of rho_f u_f^2 (r-weighted if axisym) */
  double max_div;          /* max |div u| over cells                                   */
  double phi_min, phi_max;
  double umax;             /* max |u_f| over all face components                       */
  int32_t finite;          /* 1 if p, u, v, w, phi are all finite                      */
  int32_t reserved;
} gpe_diag;

typedef struct gpe_state gpe_state;

/* Map the problem statement (Sec. 4 parameter choices: dx = L_c / N_L,
 * dt = T_c / N_t, rho_L = 1, sigma_ref = 1, W = Cn L_c, M = U_c L_c^2 / Pe)
 * to lattice-unit parameters, in this order: U_c; g when given by G or Fr;
 * sigma when it does not depend on eta_L; eta_L; sigma = U_c eta_L
 * (GPE_ST_CAPILLARY); g when given by Eo.  With GPE_ST_CAPILLARY, Oh and Mo
 * are solved for eta_L in closed form (eta_L = Oh^2 rho_L U_c L_g,
 * eta_L = Mo rho_L^2 U_c^3 / (g (rho_L - rho_G))).  init_* fields of *out are
 * zeroed.  Returns GPE_EINVAL for a missing or non-positive group, a
 * combination that leaves a quantity undetermined (GPE_VISC_CAPILLARY with
 * GPE_ST_CAPILLARY, Eo used for both sigma and g, Eo or Mo with
 * rho_L <= rho_G or without gravity) or parameters gpe_init_state would
 * reject as invalid; GPE_OK otherwise. */
int gpe_params_from_dimensionless(const gpe_problem* in, gpe_params* out);

/* Bytes of the caller-owned device workspace needed for *p: every resident
 * field (state, two RK stage sets, phase-field stage buffers, face velocity
 * sums) plus reduction scratch, each 256-byte aligned.  0 if *p is invalid. */
size_t gpe_workspace_bytes(const gpe_params* p);

/* Validate *p, lay the fields out in d_workspace (device pointer, >= bytes
 * from gpe_workspace_bytes, 256-byte aligned) and set the initial state on
 * hip_stream (a hipStream_t; NULL = the null stream): u = v = w = 0,
 * p = h_p0 or 0, phi = h_phi0 or the in-kernel profile of p->init_kind.
 * h_phi0 / h_p0 are host arrays of n[0]*n[1]*n[2] doubles or NULL.
 * Returns GPE_EUNSTABLE when an estimate of the linear stability limits of
 * the acoustic, viscous, pressure-diffusion or CH parts is exceeded and
 * p->allow_unstable == 0.  On success *out receives a new handle. */
int gpe_init_state(const gpe_params* p, void* d_workspace, size_t bytes, void* hip_stream,
                   const double* h_phi0, const double* h_p0, gpe_state** out);

/* One full time step (Sec. 3): three flow TVD-RK3 stages with phi frozen,
 * the space-time averaged centre velocity, the CH sub-step.  Asynchronous. */
int gpe_rk3_step(gpe_state* s);

/* n time steps, replayed from a captured HIP graph of one step when the
 * stream is not the null stream.  Asynchronous.  n >= 0. */
int gpe_run_n(gpe_state* s, int64_t n);

/* Reduce the current state into *out (synchronises the stream).  Sets the
 * sticky GPE_ENONFINITE on the handle and returns it if the state is not
 * finite; *out is filled either way. */
int gpe_diagnostics(gpe_state* s, gpe_diag* out);

/* Experiment diagnostics (Sec. 4: the falling drop's centroid velocity
 * U_drop and aspect ratio, the coalescing drops' radius R_r / half length
 * R_x and centroid velocity, the Rayleigh-Taylor bubble and spike fronts).
 * Positions are cell-centre coordinates in lattice units (cell i spans
 * [i, i+1], its centre is i + 1/2); axes are those of gpe_params.n (2-D and
 * axisymmetric: axis 0 = x or z, axis 1 = y or r; entries of a missing
 * third axis are NaN).  FP64 reductions in a fixed order.  Each call
 * synchronises the stream.  Returns GPE_OK, GPE_EINVAL or GPE_EHIP. */

/* The liquid region, the cells with phi > 0, each weighted by w = r (its
 * centre radius, axisymmetric geometry: integrals r dr dz per radian) or 1:
 * out[0] = sum w, out[1..3] = its centroid sum w x / sum w per axis,
 * out[4..6] = the mean of the cell-centre velocity (the mean of the cell's
 * two faces) sum w u / sum w per axis.  out[1..6] are NaN if no cell has
 * phi > 0. */
int gpe_phase_stats(gpe_state* s, double out[7]);

/* Extent of the interface along each axis a: over every pair of
 * neighbouring cells along a (both inside the grid) whose phi lie on
 * different sides of 0 (phi > 0 on exactly one), the crossing
 * x_i + phi_i / (phi_i - phi_{i+1}) (linear between the centres);
 * out[2a] = the smallest, out[2a+1] = the largest, NaN if there is none. */
int gpe_interface_extent(gpe_state* s, double out[6]);

/* The same crossings on one grid line parallel to axis `axis` (0 <= axis <
 * dimension), through the cells whose indices along the other axes are
 * (i0, i1) in increasing axis order (i1 = 0 in 2-D): out[0] = the first
 * (smallest), out[1] = the last (largest), NaN if none.  GPE_EINVAL for an
 * index outside the grid. */
int gpe_line_crossings(gpe_state* s, int32_t axis, int32_t i0, int32_t i1, double out[2]);

/* Copy one field between the device state and a dense host array of
 * n[0]*n[1]*n[2] doubles (converted from/to the state precision), in the
 * layout above (the device rows are padded, the host rows are not).  GPE_FIELD_W is valid in 3-D only; for walls and symmetry
 * planes the boundary-normal faces written by GPE_H2D must be 0.
 * bytes must equal n[0]*n[1]*n[2]*8.  Synchronous. */
int gpe_copy_field(gpe_state* s, int field, int dir, void* host, size_t bytes);

/* Byte offset of a state field inside the workspace (elements of the state
 * precision, layout above), or (size_t)-1 for an invalid field. */
size_t gpe_field_offset(const gpe_state* s, int field);

/* Device address of a field of the state (layout above; the same address
 * as the workspace plus gpe_field_offset), or NULL for an invalid field.
 * For callers that run their own kernels on the fields. */
void* gpe_field_pointer(const gpe_state* s, int field);

/* Elements from one x row of a device field to the next (layout above):
 * in FP32 with n[0] >= 64, n[0] rounded up to a multiple of 64, else n[0];
 * or GPE_EINVAL for a null handle.
 * Callers that address the fields themselves (gpe_field_pointer) use it as
 * the row stride; a plane holds n[1] such rows (1 in 2-D, where the rows
 * are the y lines). */
int64_t gpe_field_pitch(const gpe_state* s);

/* Overwrite the step counter and time (checkpoint restart). */
int gpe_set_step_time(gpe_state* s, int64_t step, double t);

/* Average device duration of every kernel of the step, measured with HIP
 * events around each launch over nsteps eager steps on the handle's stream
 * (the state advances by nsteps).  The steps are enqueued back to back with
 * one event before each step and one after every kernel, and the call
 * blocks until they have run; the per-kernel means therefore add up to the
 * device time per step.  names[i] receives a static string,
 * ms[i] the mean duration in milliseconds, bytes[i] the algorithmic HBM
 * bytes of one launch (each field read once and written once).  Returns
 * the number of kernels (<= max) or a negative gpe_error. */
int gpe_kernel_times(gpe_state* s, int64_t nsteps, int max, const char** names,
                     double* ms, double* bytes);

/* As gpe_kernel_times, with events only at the boundaries of the kernels
 * selected by mask (bit q: the q-th kernel of a step, in the order of the
 * names; bits beyond the step's kernel count are ignored).  The other
 * launches run back to back without events between them, so the steps run
 * as they do untimed except around the selected kernels.  ms[q] is 0 for a
 * kernel not selected; names and bytes are filled for all.  Returns the
 * number of kernels, or GPE_EINVAL when no kernel of the step is selected
 * (or for the argument errors of gpe_kernel_times). */
int gpe_kernel_times_masked(gpe_state* s, int64_t nsteps, uint32_t mask, int max,
                            const char** names, double* ms, double* bytes);

/* ------------------------------------------------------------------------
 * Batched ensemble: many independent 2-D (or many axisymmetric) grids of
 * different sizes and parameters advanced together, one kernel launch per
 * time-step stage for the whole batch (the per-stage launches of one step
 * are replayed as one HIP graph).  Every case runs the same kernels and
 * arithmetic as a single grid: its state after n steps is bitwise the state
 * gpe_run_n gives for that case alone.  All cases share one precision and
 * one geometry (GPE_GEOM_2D or GPE_GEOM_AXISYM); each has its own size,
 * boundary conditions, dt and material parameters.  The caller owns the
 * workspace (256-byte aligned) and the stream, as for a single grid.
 * ------------------------------------------------------------------------ */
typedef struct gpe_ensemble gpe_ensemble;

/* Workspace bytes for the batch (0 for an invalid batch). */
size_t gpe_ensemble_workspace_bytes(const gpe_params* cases, int32_t count);

/* Set up `count` cases (1 <= count <= 65535) in d_workspace and initialise
 * each from its init_kind fields (as gpe_init_state with h_phi0 = NULL).
 * Work-group tiles are 32 rows high until gpe_ensemble_autotune.
 * Returns GPE_EINVAL for an invalid case, a mixed batch or a 3-D case,
 * GPE_EUNSTABLE if a case without allow_unstable exceeds the stability
 * estimate, GPE_EWORKSPACE, GPE_EHIP. */
int gpe_ensemble_create(const gpe_params* cases, int32_t count, void* d_workspace, size_t bytes,
                        void* hip_stream, gpe_ensemble** out);

/* Advance every case by nsteps time steps (enqueued on the stream). */
int gpe_ensemble_run_n(gpe_ensemble* e, int64_t nsteps);

/* Tile autotuner: for every group of cases with the same number of rows,
 * try work-group tile heights of 1, 2, 4, 8, 16, 32, 64 and 128 rows (clamped to the
 * grid) and keep the one with the shortest batch step, timed over
 * trial_steps graph-replayed steps per candidate (one size group at a time,
 * the others held fixed).  The trial steps are real steps: every case
 * advances by them, and results do not depend on the tile height.  h_rows
 * (NULL or count entries) receives each case's chosen height.  Needs a
 * non-null stream; blocks until the trials have run. */
int gpe_ensemble_autotune(gpe_ensemble* e, int32_t trial_steps, int32_t* h_rows);

/* Per-case finite flag (1: p, u, v, phi all finite; 0 otherwise) into
 * h_flags[count]; blocks until the stream reaches this point. */
int gpe_ensemble_finite(gpe_ensemble* e, int32_t* h_flags);

/* Borrowed handle of case i (0 <= i < count) for gpe_diagnostics,
 * gpe_copy_field, gpe_set_step_time or stepping that case alone; valid until
 * gpe_ensemble_destroy and never passed to gpe_destroy.  NULL if invalid. */
gpe_state* gpe_ensemble_case(gpe_ensemble* e, int32_t i);

/* Free the host-side ensemble handle and its case handles (never the
 * workspace).  NULL is ignored. */
void gpe_ensemble_destroy(gpe_ensemble* e);

/* ------------------------------------------------------------------------
 * HBM streaming probe (a measurement aid, not part of the method): the
 * bandwidth a plain streaming kernel reaches on this device, the practical
 * ceiling the stencil kernels are compared with.  One launch that streams
 * `bytes` (a multiple of 16; both pointers 16-byte aligned) with 16-byte
 * accesses, grid-strided over `workgroups` work-groups of 256 threads
 * (0: 8 per CU):
 *  - GPE_STREAM_READ: reads d_src (d_dst, >= 4 bytes, receives nothing: a
 *    sum is stored only if it equals a value it never takes);
 *  - GPE_STREAM_WRITE: writes a constant into d_dst;
 *  - GPE_STREAM_COPY: copies d_src to d_dst (non-overlapping).
 * Asynchronous on the stream; the caller times it.  Returns GPE_OK,
 * GPE_EINVAL or GPE_EHIP.
 * ------------------------------------------------------------------------ */
enum gpe_stream_mode { GPE_STREAM_READ = 0, GPE_STREAM_WRITE = 1, GPE_STREAM_COPY = 2 };
int gpe_hbm_stream(int32_t mode, void* d_dst, const void* d_src, size_t bytes, int32_t workgroups, void* stream);

/* Free the host-side handle (never the workspace). NULL is ignored. */
void gpe_destroy(gpe_state* s);

const char* gpe_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* GPE_H */
