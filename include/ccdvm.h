/* ccdvm -- Cartesian cut-cell discrete-velocity solver for rarefied gas flow
 * around obstacles, on AMD Instinct MI355X (gfx950).
 *
 * Method: Dechriste & Mieussens, "A Cartesian cut cell method for rarefied
 * flow simulations around moving obstacles" (2015).  One time step is the
 * sweep over cells x discrete velocities of Section 3.3: merge of small
 * virtual cells into control volumes (eq. FusionDD), first-order explicit
 * scheme with upwind fluxes on Cartesian and wall edges (eqs. ExSchemeDD,
 * FluxDD), diffuse-reflection wall distribution whose density makes the net
 * mass flux zero (eq. BoundaryDDv), BGK relaxation toward the local
 * Maxwellian built from the discrete moments (eqs. MacroscopicDDv, BGKDD),
 * redistribution to the virtual cells (eq. UpdateDD); the force and torque
 * on the body from the wall stress (eqs. eq-force, eq-torque,
 * StressTensorDD); the rigid-body update (eqs. motionDD_posit, motionDD_vit,
 * uwDD).  The 3D variant follows Section 5 (eq. eq-schema3D).
 *
 * Units: nondimensional, R = T0 = rho0 = 1.  All floating point is FP64.
 *
 * Memory ownership: the caller owns every device buffer.  It queries sizes
 * with cc_workspace_bytes, allocates them (for example as torch tensors on
 * the GPU) and hands them to cc_bind together with the HIP stream to use.
 * The library keeps only host metadata and never allocates device memory
 * after cc_bind; cc_step launches kernels only (no host synchronisation
 * unless a status flag is read back).
 *
 * Device layouts (velocity innermost, so consecutive lanes read consecutive
 * addresses):
 *   cell index   c = (k*ny + j)*nx + i          (i fastest)
 *   velocity     p = p2*N + p1 (2D), p = (p3*N + p2)*N + p1 (3D), p1 fastest;
 *                node v = vmin + (idx + 1/2) dv, dv = (vmax - vmin)/N
 *   2D state     double2 state[c][p] = {f, g} (16 bytes per cell-velocity)
 *   3D state     double  state[c][p] = F      (8 bytes per cell-velocity)
 *   "plane" arrays used by cc_load_state / cc_store_state: double f[c][p]
 *   (and g[c][p] in 2D), 8-byte aligned device pointers.
 *
 * Errors: every call returns a cc_status; no exception crosses the ABI.
 * cc_last_error returns a message for the last failure on that context.
 * Threading: one context per host thread at a time; a context is bound to
 * one stream.
 */
#ifndef CCDVM_H
#define CCDVM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cc_ctx cc_ctx;

typedef enum {
  CC_OK = 0,
  CC_EINVAL = -1,     /* bad argument or unsupported size */
  CC_ENOMEM = -2,     /* host allocation failed (no entry point lets an
                         exception out) or a workspace is too small */
  CC_EGEOM = -3,      /* geometry rejected: a cell cut twice by the boundary,
                         a master search that cycles or needs more than 4 hops */
  CC_ECFL = -4,       /* positivity condition (eq-CFL) violated in strict mode */
  CC_EHIP = -5,       /* a HIP runtime call failed */
  CC_ESTATE = -6      /* call out of order (e.g. cc_step before cc_bind) */
} cc_status;

enum { CC_BODY_NONE = 0, CC_BODY_CIRCLE = 1, CC_BODY_ELLIPSE = 2,
       CC_BODY_CAVITY = 3, CC_BODY_HALFPLANE = 4, CC_BODY_SPHERE = 5, CC_BODY_VANE = 6 };
enum { CC_MOTION_FIXED = 0, CC_MOTION_FREE_ROTATION = 1, CC_MOTION_IMPOSED = 2 };
/* Equilibrium of the relaxation term: the Maxwellian of the directly
 * computed moments (eq. MacroscopicDDv), or the conservative one of
 * Section 3.1, whose triplet (rho, u, T) solves, by Newton iterations from
 * the direct moments, "discrete mass, momentum and energy of the sampled
 * Maxwellian (and of T/2 M in 2D) = those of the state", so that the
 * discrete relaxation conserves them exactly.  The whole triplet, rho in the
 * relaxation time included, comes from that solution.  A cell whose
 * iteration does not converge in 50 steps keeps the direct triplet. */
enum { CC_MAXW_DIRECT = 0, CC_MAXW_CONSERVATIVE = 1 };
/* Time scheme: explicit (eq. ExSchemeDD) or the first-order semi-implicit
 * scheme of eq. ImpSchemeDD: explicit transport, then the relaxation taken
 * implicitly toward the equilibrium of the transported value,
 * f^{n+1} = (f* + (dt/tau^n) E*)/(1 + dt/tau^n), tau^n from the density of
 * the state at t^n.  Stable for dt >> tau.  In 2D with the direct
 * equilibrium and up to 8 velocity chunks per half-row the relaxation runs
 * inside the streaming kernel, which then reads and writes the state once,
 * as the explicit step does; otherwise a second pass relaxes in place. */
enum { CC_SCHEME_EXPLICIT = 0, CC_SCHEME_IMEX = 1 };
/* Relaxation model: BGK (eq. BGKDD; 3D: the Maxwellian) or the Shakhov
 * model (eq. ShakhovDD; 3D: the Shakhov equilibrium of Section 2.1), whose
 * equilibrium multiplies the Maxwellian by a polynomial in v - u carrying
 * the heat flux q of eq. MacroscopicDDv, so that the model has the Prandtl
 * number `prandtl`.  q is taken about the directly computed mean velocity;
 * with the conservative equilibrium the Newton triplet fills the rest of
 * the formula.  Pr = 1 is BGK. */
enum { CC_MODEL_BGK = 0, CC_MODEL_SHAKHOV = 1 };

/* Flow set-up.  dim = 2 selects the reduced plane-flow model with the two
 * distributions f, g (Section 2.2); dim = 3 the full model with F
 * (Section 2.1).  n[2] = 1 in 2D.  kn <= 0 selects pure transport (no
 * collisions).  dt <= 0: dt = cfl / sum_d (max_p |v_d| / dx_d).  inflow =
 * (rho, ux, uy, uz, T) of the Maxwellian carried by every outer face (farfield)
 * and used as the initial state. */
typedef struct {
  int dim;
  int n[3];
  double lo[3], hi[3];
  int nv;                 /* velocity nodes per axis, N */
  double vmin, vmax;
  double kn, lref;
  double cfl, dt;
  double inflow[5];
  int maxwellian;         /* CC_MAXW_DIRECT or CC_MAXW_CONSERVATIVE (fixed bodies,
                             no adjoint or batch) */
  int scheme;             /* CC_SCHEME_EXPLICIT or CC_SCHEME_IMEX (fixed bodies,
                             no adjoint or batch) */
  int model;              /* CC_MODEL_BGK or CC_MODEL_SHAKHOV (no adjoint or batch) */
  double prandtl;         /* Shakhov: Prandtl number, finite and > 0 */
  int amr_depth;          /* 3D octree mesh (Section 5.1): finest depth below the
                             coarse grid n; 0 = uniform grid; at most 8 */
  double amr_band;        /* refinement band in coarse spacings (<= 0: 2 sqrt 2) */
  int cfl_strict;         /* 1: cc_bind returns CC_ECFL when the positivity number of
                             eq. eq-CFL exceeds 1 (0: it only warns on stderr) */
} cc_config;

/* Obstacle given by an analytic signed distance, gas side positive
 * (Appendix A).  circle: axes[0] = radius; ellipse: semi-axes axes[0],
 * axes[1], rotated by theta about center; cavity: gas inside a circle of
 * radius axes[0]; halfplane: gas where (x - center).(cos theta, sin theta) > 0;
 * sphere (3D): axes[0] = radius; vane (3D): the points within
 * r = min(axes) of the box of half-sizes axes - r (a plate with rounded
 * edges), turned by theta about the z axis through center (exact signed
 * distance).  t_wall: wall temperature.  motion: fixed, free rotation about
 * the centre driven by the gas torque (inertia), or imposed constant
 * velocity vel / angular velocity omega.  In 3D a moving body turns about
 * the z axis through its centre (pure rotation, Section 5: vel must be 0);
 * its walls move with omega e_z x (x - center). */
typedef struct {
  int kind;
  double center[3], axes[3], theta, t_wall;
  double mass, inertia;
  int motion;
  double vel[3], omega;
} cc_body;

/* Validates the set-up, computes dt and the sizes of the device buffers.
 * No device work.  *out receives a new context (free with cc_destroy).
 * Returns CC_EINVAL for an unsupported set-up; in 3D the velocity box must
 * be symmetric about 0 and N one of 4, 6, 8, 12, 16, and the body a sphere
 * or a vane (or none).  A turning 3D body runs on the octree mesh (any
 * amr_depth; 0 is the uniform grid), whose buffers are sized here for the
 * largest mesh over a half turn plus a quarter. */
cc_status cc_create(const cc_config* cfg, const cc_body* body, cc_ctx** out);
void cc_destroy(cc_ctx* ctx);
const char* cc_last_error(const cc_ctx* ctx);

/* Bytes of the two state buffers (each), of the geometry buffer and of the
 * scratch buffer.  All must be 256-byte aligned device allocations. */
cc_status cc_workspace_bytes(const cc_ctx* ctx, size_t* state_bytes,
                             size_t* geom_bytes, size_t* scratch_bytes);

/* Binds caller-owned device buffers and a HIP stream (hipStream_t passed as
 * void*, NULL = default stream), then builds the geometry on the device
 * (Appendix A: level set, cell types, edge lengths, wall normal, areas,
 * master search, control volumes).  Synchronises the stream once to read
 * the geometry status; returns CC_EGEOM when the geometry is rejected. */
cc_status cc_bind(cc_ctx* ctx, void* state0, void* state1, void* geom,
                  void* scratch, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cc_bind
 * without the scratch buffer.  The context's per-step records (moments of
 * the current state, force and mass partials, rigid-body state, moving-body
 * lists) are kept in a static device array of the library, 32 MiB, one copy
 * on each GPU, held until the process ends; state0, state1 and geom are the
 * caller's buffers as for cc_bind, hip_stream must belong to the current
 * device.  Allocates no device memory (the side stream and events of a
 * context are created on its first bind, as with cc_bind).  Returns
 * CC_EINVAL when the set-up needs more scratch than the array holds (the
 * scratch size of cc_workspace_bytes; a 2D 512 x 256 grid with 32^2
 * velocities needs 22 MiB).  The array serves one bound context per GPU:
 * binding another context to it waits for the previous owner's stream, keeps
 * its body state on the host and unbinds it (its calls then return
 * CC_ESTATE until it is bound again); calls that overlap on one GPU race.
 * cc_bind or cc_destroy releases the array. */
cc_status cc_bind_noalloc(cc_ctx* ctx, void* state0, void* state1, void* geom,
                          void* hip_stream);

/* Positivity condition of the explicit scheme (Section 3.4.1, eqs. eq-CFL
 * and phiCFL), evaluated by cc_bind on the bound geometry:
 *   out[0] = dt max_{CV, p} phi_{CV,p} / S_CV, phi the outflow rate of a
 *            control volume at velocity p summed over its members' Cartesian
 *            and wall edges (faces in 3D) as printed, with the wall velocity
 *            of the initial body state;
 *   out[1] = dt max 1/tau at the inflow density (the state is not known at
 *            bind; 0 without collisions and for the semi-implicit scheme,
 *            whose condition does not involve tau);
 *   out[2] = out[0] + out[1], the number that must not exceed 1.
 * phi is convex in v, so its largest value on the velocity grid is taken at
 * one of the grid's corner nodes.  CC_ESTATE before cc_bind. */
cc_status cc_cfl_number(const cc_ctx* ctx, double out[3]);

/* Fills the current state with the inflow Maxwellian in every non-solid
 * cell (g = T/2 f in 2D), zero in solid cells.  Asynchronous. */
cc_status cc_init_maxwellian(cc_ctx* ctx);

/* Copies a state given as plane arrays (device pointers, layout above; g is
 * ignored in 3D) into the current state, sets solid cells to zero and merges
 * every control volume (eq. FusionDD).  Asynchronous. */
cc_status cc_load_state(cc_ctx* ctx, const double* f, const double* g);

/* Copies the current state out as plane arrays (device pointers). */
cc_status cc_store_state(const cc_ctx* ctx, double* f, double* g);

/* Advances nsteps time steps.  diag (nullable device pointer, nsteps*4
 * doubles) receives, for each step n, the force (Fx, Fy), the torque about
 * the body centre and the total mass, all of the state at t^n (eqs.
 * eq-force, eq-torque, def-masse); in 3D the entries are (Fx, Fy, Fz, mass),
 * for a turning body (Fx, Fy, torque about the z axis through the centre,
 * mass).  Asynchronous for fixed bodies; for a moving 2D body the
 * rigid-body update of every step runs on the device as well.  A turning
 * 3D body (Section 5, steps 1-7, then the mesh adapted to the body) is
 * driven by the host: each step plans the step on the mesh of t^n, runs the
 * kernels, reads the torque back (one synchronisation per step), builds the
 * mesh of t^{n+1} and carries the state over to it (0th-order
 * prolongation, gas-volume weighted restriction); the leaf count may
 * change (cc_amr_counts).  CC_EGEOM when the body leaves the refined band
 * within one step or a leaf appearing at t^{n+1} finds no control volume;
 * CC_ENOMEM when the adapted mesh outgrows the buffers. */
cc_status cc_step(cc_ctx* ctx, int nsteps, double* diag);

/* Moments of every cell of the current state, eq. (MacroscopicDDv):
 * 2D: out[c][9] = rho, ux, uy, T, Sxx, Sxy, Syy, qx, qy;
 * 3D: out[c][14] = rho, ux, uy, uz, T, Sxx, Sxy, Sxz, Syy, Syz, Szz, qx, qy, qz.
 * Solid cells get zeros.  out is a device pointer.  Asynchronous. */
cc_status cc_moments(cc_ctx* ctx, double* out);

/* Force and torque on the body for the current state (synchronous), from
 * the wall stress of eq. (StressTensorDD) summed over every wall edge (face)
 * of every virtual cell, eqs. (eq-force) and (eq-torque), the wall density
 * of eq. (BoundaryDDv) taken from the current state: out[0..3] = Fx, Fy,
 * torque about the body centre (counter-clockwise positive), mass
 * sum_CV S_CV rho (2D) or Fx, Fy, Fz, mass (3D, Section 5). */
cc_status cc_body_force(cc_ctx* ctx, double out[4]);

/* Rigid-body state at the current time (synchronous): centre x, y,
 * angle, velocity x, y, angular velocity (a turning 3D body: its angle and
 * angular velocity about the z axis). */
cc_status cc_body_state(cc_ctx* ctx, double out[6]);

/* Applies one explicit Euler update of the body velocity with a given
 * force and torque, eq. (motionDD_vit), honouring the motion mode (free
 * rotation updates only the angular velocity).  Synchronous. */
cc_status cc_rigid_update(cc_ctx* ctx, const double force[3], double torque);

/* Time step in use. */
cc_status cc_dt(const cc_ctx* ctx, double* dt);

/* Copies the geometry tables to host arrays of ncell entries each (any
 * pointer may be NULL): type (0 gas, 1 cut, 2 solid), master (-1 for solid),
 * then 2D: lxm, lxp, lym, lyp, lw, nwx, nwy, rwx, rwy, sbar, scv.
 * Synchronous.  3D: see cc_geometry_export3d. */
cc_status cc_geometry_export(cc_ctx* ctx, int* type, int* master,
                             double* lxm, double* lxp, double* lym, double* lyp,
                             double* lw, double* nwx, double* nwy, double* rwx,
                             double* rwy, double* sbar, double* scv);

/* 3D geometry tables (Section 5 with the face, wall and volume rules
 * stated in the library's geometry source) to host arrays of ncell entries
 * each (any pointer may be NULL): type, master, gas areas of the faces x-,
 * x+, y-, y+, z-, z+, wall area, wall normal (into the solid), wall centre,
 * virtual-cell volume, control-volume volume.  Synchronous. */
cc_status cc_geometry_export3d(cc_ctx* ctx, int* type, int* master, double* sxm, double* sxp,
                               double* sym, double* syp, double* szm, double* szp, double* aw,
                               double* nwx, double* nwy, double* nwz, double* rwx, double* rwy,
                               double* rwz, double* vbar, double* vcv);

/* Number of control volumes handled by the cut-cell kernel (masters that
 * are cut cells or own merged cells) and of non-master non-solid cells. */
cc_status cc_geometry_counts(cc_ctx* ctx, int* n_irregular, int* n_members,
                             int* n_solid);

/* Octree mesh (3D, amr_depth > 0 or a turning body; Section 5.1, octree
 * procedure).  The
 * coarse grid n is refined near the boundary: a cell of depth d is divided
 * in 8 while the distance from its centre to the boundary is below
 * amr_band * dx / 2^d (dx = largest coarse spacing) and d < amr_depth.  The
 * mesh is built on the host by cc_create (CC_EGEOM if a cut cell lies above
 * the finest depth, neighbours differ by more than one depth, or the master
 * search fails) and uploaded by cc_bind.  The cells of every other call are
 * then the leaves, in Z-order of their lower corner: the state is
 * F[leaf][p]; cc_moments, cc_geometry_counts and the diag rows of cc_step
 * (force and mass of the state entering each step) work as on a uniform
 * grid; cc_body_force and cc_geometry_export3d are not available.  The
 * octree runs the explicit BGK scheme with the direct equilibrium; dt comes
 * from the finest spacing.
 * With a turning body the mesh follows the body and these report the mesh
 * of the current state.
 * cc_amr_counts: leaves and face-list entries.
 * cc_amr_export (host arrays, each nullable): per leaf its depth, its
 * integer coordinates at that depth (3), type (0 gas, 1 cut, 2 solid),
 * master leaf (-1 solid), gas volume, control-volume volume, wall area and
 * the gas areas of its six faces (x-, x+, y-, y+, z-, z+).
 * cc_amr_faces (host arrays): fptr (nleaf + 1) into the face entries, the
 * leaf across each face (-1: farfield), its direction 0..5 and gas area
 * (across a change of depth the finer leaf's face).
 * All three return CC_EINVAL on a uniform grid. */
cc_status cc_amr_counts(cc_ctx* ctx, int* nleaf, int* nface);
cc_status cc_amr_export(cc_ctx* ctx, int* lvl, int* ijk, int* type, int* master, double* vbar,
                        double* vcv, double* aw, double* S6);
cc_status cc_amr_faces(cc_ctx* ctx, int* fptr, int* fnb, int* fdir, double* farea);

/* Rows of cells per tile of the regular-cell pass (each tile is 4 adjacent
 * columns; one wave per column marches up the rows).  0 = automatic.
 * Changes performance only, never results. */
cc_status cc_set_tile_rows(cc_ctx* ctx, int rows);

/* Per-kernel timing with HIP events recorded on the bound stream.
 * cc_profile_enable(ctx, 1) starts recording (cleared); cc_profile_read
 * returns, for kernel id k (0 = regular-cell step kernel, 1 = cut-cell
 * kernel, 2 = force/mass reduction, 3 = merge, 4 = pass between steps:
 * 3D moments and the conservative Newton solve, a turning body's remap
 * to the adapted mesh, or a moving 2D body's geometry rebuild (pose, level
 * set, cells, masters, control volumes and step lists of t^{n+1}),
 * 5 = implicit relaxation of the semi-implicit
 * scheme), the summed milliseconds and the number of launches since
 * enabling (at most 4096 launches per kernel are recorded); ids 6, 7 and
 * 8 return the host time of a turning body's steps: the step planning
 * (with its upload), the wall time from the launch of the step kernels to
 * the remap map, and the build of the new mesh alone (it runs on a host
 * thread while the device runs the step).  Reading synchronises the
 * stream. */
cc_status cc_profile_enable(cc_ctx* ctx, int on);
cc_status cc_profile_read(cc_ctx* ctx, int kernel, double* total_ms, int* launches);

/* ------------------------------------------------------------------ */
/* Adjoint (2D fixed bodies).  Starting from the inflow Maxwellian, runs
 * nsteps and returns out = {J, dJ/dT_w, dJ/dKn, dJ/dMa}, J = drag
 * (objective 0) or torque (objective 1) of the final state, by a
 * hand-written adjoint of every step (transposed upwind fluxes, wall density,
 * BGK Jacobian) with checkpointed recomputation: the state is saved every
 * ckpt_every steps and each segment is recomputed once during the backward
 * sweep.  Mach derivative: u_inflow = Ma sqrt(gamma T_inflow) along the
 * inflow direction, gamma = 5/3.  pool: caller-owned 256-byte aligned device
 * buffer of cc_adjoint_workspace_bytes bytes (checkpoints, one segment of
 * states and moments, two sensitivity buffers, partial sums).  Leaves the
 * context at the final state.  Synchronous. */
cc_status cc_adjoint_workspace_bytes(const cc_ctx* ctx, int nsteps, int ckpt_every, size_t* bytes);
cc_status cc_adjoint(cc_ctx* ctx, int nsteps, int ckpt_every, int objective, void* pool,
                     double out[4]);

/* ------------------------------------------------------------------ */
/* Batched instances.  Many independent 2D fixed-body problems (each its own
 * context: grid, velocity grid, Kn, T_w, inflow), all bound to the same
 * stream, advanced together: per step one kernel walks the cut/merged
 * control volumes of every instance and one kernel per velocity-grid size
 * walks the regular-cell tiles of every instance of that size.  A step is
 * captured once as a HIP graph (one per ping-pong parity), so cc_batch_step
 * issues one graph launch per step.  Results are bitwise identical to
 * stepping each context with cc_step. */
typedef struct cc_batch cc_batch;

/* ctxs: n distinct bound 2D fixed-body contexts on the same stream.  The
 * batch refers to them; they must outlive it. */
cc_status cc_batch_create(cc_ctx* const* ctxs, int n, cc_batch** out);
/* Bytes of the device workspace (descriptor tables and work lists). */
cc_status cc_batch_workspace_bytes(const cc_batch* b, size_t* bytes);
/* Binds a caller-owned 256-byte aligned device workspace, builds the tables
 * and captures the step graphs.  Synchronises the stream. */
cc_status cc_batch_bind(cc_batch* b, void* workspace);
/* Picks, for each velocity-grid size, the tile height (rows) with the
 * fastest tile kernel over trial_steps timed launches; rows_out (nullable)
 * receives one entry per group.  The states are not advanced.  Synchronous. */
cc_status cc_batch_autotune(cc_batch* b, int trial_steps, int* rows_out);
/* Groups (velocity-grid sizes): count, chunks of 64 velocities per half-row
 * and tile rows in use, arrays of ngroups entries (at most 16 groups). */
cc_status cc_batch_groups(const cc_batch* b, int* ngroups, int* chunks, int* rows);
/* Advances every instance by nsteps (asynchronous).  Stepping an instance
 * on its own in between is allowed; the tables are rebuilt when needed. */
cc_status cc_batch_step(cc_batch* b, int nsteps);
/* Adjoint of every instance at once: what cc_adjoint returns for each
 * context (from the inflow Maxwellian, nsteps steps, J = drag or torque of
 * the final state, checkpoint every ckpt_every steps), with each step of
 * each phase one launch over all instances (forward steps and segment
 * recomputations through the batched step kernels, adjoint steps through
 * batched adjoint kernels, checkpoint copies through one copy kernel).
 * Results are bitwise those of cc_adjoint on each context.  out: n x 4
 * doubles {J, dJ/dT_w, dJ/dKn, dJ/dMa} per instance, in the batch order.
 * workspace: caller-owned 256-byte aligned device buffer of
 * cc_batch_adjoint_workspace_bytes bytes (every instance's adjoint pool and
 * the step tables).  Leaves every context at its final state.
 * Synchronous. */
cc_status cc_batch_adjoint_workspace_bytes(const cc_batch* b, int nsteps, int ckpt_every, size_t* bytes);
cc_status cc_batch_adjoint(cc_batch* b, int nsteps, int ckpt_every, int objective, void* workspace,
                           double* out);
const char* cc_batch_last_error(const cc_batch* b);
void cc_batch_destroy(cc_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* CCDVM_H */
