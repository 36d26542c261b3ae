/* Oracle of the Cartesian cut-cell discrete-velocity method
 * (Dechriste & Mieussens, "A Cartesian cut cell method for rarefied flow
 * simulations around moving obstacles", 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, serial-order FP64 CPU
 * implementation that follows the paper's steps in the paper's order.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the solver
 * library; the two meet only through the seeded inputs.
 *
 * Layout of the oracle's own arrays: cell c = (k*ny + j)*nx + i, velocity
 * p = (p3*N + p2)*N + p1, f[c*nvel + p].  2D carries f and g; 3D carries F.
 *
 * Status codes: 0 ok, -1 bad argument, -3 geometry rejected (saddle cell,
 * master search cycle or no gas neighbour), -2 out of memory.
 */
#ifndef CCDVM_ORACLE_H
#define CCDVM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int dim;                 /* 2 or 3 */
  int n[3];                /* cells per axis (n[2] = 1 in 2D) */
  double lo[3], hi[3];     /* domain box */
  int nv;                  /* velocity nodes per axis */
  double vmin, vmax;       /* velocity box, same on every axis */
  double kn, lref;         /* Knudsen number (<= 0: collisionless), length */
  double cfl, dt;          /* dt <= 0: dt from cfl */
  double inflow[5];        /* rho, ux, uy, uz, T of the farfield Maxwellian */
  int body_kind;           /* 0 none 1 circle 2 ellipse 3 cavity 4 halfplane 5 sphere 6 vane */
  double center[3], axes[3], theta, t_wall;
  double mass, inertia;
  int motion;              /* 0 fixed 1 free rotation 2 imposed */
  double vel[3], omega;    /* rigid body velocity at t = 0 */
  int maxwellian;          /* 0 direct moments, 1 conservative (Newton) */
  int scheme;              /* 0 explicit (ExSchemeDD), 1 semi-implicit (ImpSchemeDD) */
  int model;               /* 0 BGK, 1 Shakhov */
  double prandtl;          /* Prandtl number of the Shakhov model */
  int amr_depth;           /* octree (3D): finest depth below the coarse grid n, 0 = uniform */
  double amr_band;         /* octree refinement band in coarse spacings (<= 0: 2 sqrt 2) */
} orc_cfg;

typedef struct orc2d orc2d;

int  orc2d_create(const orc_cfg *cfg, orc2d **out);
void orc2d_destroy(orc2d *o);
double orc2d_dt(const orc2d *o);
void orc2d_velocity(const orc2d *o, double *v);     /* N nodes */
/* geometry export: per-cell arrays of length ncell */
void orc2d_geometry(const orc2d *o, int *type, int *master, double *lxm,
                    double *lxp, double *lym, double *lyp, double *lw,
                    double *nwx, double *nwy, double *rwx, double *rwy,
                    double *sbar, double *scv);
void orc2d_init(const orc2d *o, double *f, double *g);
/* in-place merge over control volumes (FusionDD) */
void orc2d_merge(const orc2d *o, double *f, double *g);
/* scheme + redistribution for the listed cells (their control volumes);
   input must be merged.  Output rows are written for the listed cells only,
   in list order: fo[k*nvel + p]. */
void orc2d_update_cells(const orc2d *o, const double *fm, const double *gm,
                        const int *cells, int ncells, double *fo, double *go);
/* one complete fixed-geometry step: merge, scheme, redistribution.
   diag (nullable) receives Fx, Fy, torque, mass of the state at t^n. */
int  orc2d_step(orc2d *o, const double *f, const double *g, double *fo,
                double *go, double *diag);
/* force, torque and mass of a merged state */
void orc2d_force(const orc2d *o, const double *fm, const double *gm, double *diag);
/* per-cell moments rho, ux, uy, T, Sxx, Sxy, Syy, qx, qy (9 per cell) */
void orc2d_moments(const orc2d *o, const double *f, const double *g, double *out);
/* body state: centre (2), theta, velocity (2), omega */
void orc2d_body_state(const orc2d *o, double *state);
/* adjoint (fixed bodies): nsteps from the inflow Maxwellian, objective
   0 = drag, 1 = torque of the final state; out = J, dJ/dT_w, dJ/dKn,
   dJ/du_x, dJ/du_y of the farfield velocity */
int  orc2d_adjoint(orc2d *o, int nsteps, int objective, double *out);
/* triplet (rho, ux, uy, T) of the equilibrium used by the relaxation of
   one cell's (f, g): the direct moments, or the conservative solution;
   returns the Newton iterations taken (0 for direct), -1 if no convergence */
int  orc2d_equilibrium(const orc2d *o, const double *f, const double *g, double *out);
/* equilibria (f_eq, g_eq) of one cell's (f, g) at every velocity: eq. (BGKDD)
   or eq. (ShakhovDD), with the triplet of orc2d_equilibrium */
void orc2d_equilibrium_values(const orc2d *o, const double *f, const double *g, double *fe,
                              double *ge);
int  orc_threads(void);
void orc_set_threads(int n);

typedef struct orc3d orc3d;
int  orc3d_create(const orc_cfg *cfg, orc3d **out);
void orc3d_destroy(orc3d *o);
double orc3d_dt(const orc3d *o);
void orc3d_velocity(const orc3d *o, double *v);
/* geometry export: type, master, S (6 per cell: x-, x+, y-, y+, z-, z+ gas
   areas), wall area, wall normal (3 per cell, into the solid), wall centre
   (3 per cell), virtual-cell volume, control-volume volume */
void orc3d_geometry(const orc3d *o, int *type, int *master, double *S6, double *sw,
                    double *nw3, double *rw3, double *vbar, double *vcv);
void orc3d_init(const orc3d *o, double *F);
void orc3d_merge(const orc3d *o, double *F);
void orc3d_update_cells(const orc3d *o, const double *Fm, const int *cells, int ncells,
                        double *out);
/* one fixed-geometry step; diag (nullable) = Fx, Fy, Fz, mass of F^n */
int  orc3d_step(orc3d *o, const double *F, double *Fo, double *diag);
void orc3d_force(const orc3d *o, const double *Fm, double *diag);
/* 14 moments per cell (see orc3d_moments) */
void orc3d_moments(const orc3d *o, const double *F, double *out);
/* triplet (rho, ux, uy, uz, T) of the equilibrium of one cell's F (direct
   or conservative); returns the Newton iterations, -1 if no convergence */
int  orc3d_equilibrium(const orc3d *o, const double *F, double *out);
/* equilibrium of one cell's F at every velocity: the Maxwellian of Section
   2.1, or the Shakhov equilibrium given there */
void orc3d_equilibrium_values(const orc3d *o, const double *F, double *Fe);

/* 3D octree mesh (Section 5.1, octree procedure): leaves in Z-order; state
   F[leaf][p].  A body with motion != 0 turns about the z axis through its
   centre (pure rotation, Section 5 steps 1-7): orc3a_step then leaves the
   state at t^{n+1} on the mesh of t^n, orc3a_adapt rebuilds the mesh for the
   new angle and orc3a_remap carries the state over to it. */
typedef struct orc3a orc3a;
int  orc3a_create(const orc_cfg *cfg, orc3a **out);
void orc3a_destroy(orc3a *o);
double orc3a_dt(const orc3a *o);
int  orc3a_nleaf(const orc3a *o);
int  orc3a_nface(const orc3a *o);
void orc3a_velocity(const orc3a *o, double *v);
/* per leaf: depth, coordinates at that depth (3), type, master, gas volume,
   control-volume volume, wall area, the 6 face gas areas */
void orc3a_leaves(const orc3a *o, int *lvl, int *ijk, int *type, int *master, double *vbar,
                  double *vcv, double *sw, double *S6);
/* face lists: fptr (nleaf + 1), neighbour leaf or -1, direction 0..5
   (x-, x+, y-, y+, z-, z+), gas area */
void orc3a_faces(const orc3a *o, int *fptr, int *fnb, int *fdir, double *farea);
void orc3a_init(const orc3a *o, double *F);
void orc3a_merge(const orc3a *o, double *F);
/* diag = Fx, Fy, Fz, mass of F^n (fixed body) or Fx, Fy, torque about
   the z axis, mass (turning body) */
int  orc3a_step(orc3a *o, const double *F, double *Fo, double *diag);
int  orc3a_adapt(orc3a *o);
void orc3a_remap(const orc3a *o, const double *Fold, double *Fnew);
void orc3a_body(const orc3a *o, double *out);   /* angle, angular velocity */
double orc3a_levelset(const orc3a *o, double th, double x, double y, double z);

#ifdef __cplusplus
}
#endif
#endif
