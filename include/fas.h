/*
 * fas.h - C ABI of the MI355X library for preconditioned FAS smoothers of
 * the 2-D cell-centred finite-volume Euler / Baldwin-Lomax RANS equations
 * (Birken, Bull, Jameson, "Preconditioned smoothers for the full
 * approximation scheme for the RANS equations").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns fas_status (FAS_OK = 0, negative on error) and never
 *   throws.  fas_last_error() returns a message for the calling thread.
 * - Grid node arrays are HOST pointers, (nj+1) x (ni+1), I fastest.
 * - Every other array argument is a DEVICE pointer on the state's device,
 *   laid out as [4][nj][ni] (component, j, i with i fastest; components
 *   rho, rho*u, rho*v, rho*E) for per-cell vectors, [nj][ni] for scalars.
 *   Caller arrays are read or written during the call (or the stream work it
 *   enqueues) and never retained.
 * - Work is enqueued on the stream given to fas_state_create; a call returns
 *   once its work is enqueued unless it returns host values (n_done, ...),
 *   which synchronise that stream.
 * - Level 0 is the finest level; level l has ni/2^l x nj/2^l cells.
 * - Nondimensionalisation: rho_inf = 1, p_inf = 1, |v_inf| = M sqrt(gamma),
 *   chord 1 (it reproduces the paper's physical time step 0.486822 of
 *   Section 6.4).
 */
#ifndef FAS_H
#define FAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FAS_OK = 0,
    FAS_EINVAL = -1,          /* bad argument, shape or parameter */
    FAS_ENOMEM = -2,          /* device allocation failed */
    FAS_EDEVICE = -3,         /* HIP runtime error */
    FAS_DIVERGED = -4,        /* non-finite or grown residual norm (state rolled back) */
    FAS_STALLED = -5,         /* too little residual drop over the stall window */
    FAS_NOT_CONVERGED = -6    /* cycle cap reached before the requested drop */
} fas_status;

enum { FAS_BOX = 0, FAS_CGRID = 1 };          /* grid topology */
enum { FAS_EULER = 0, FAS_RANS_BL = 1 };       /* model */
enum {                                         /* smoother (Table "RK smoothers") */
    FAS_AW3 = 0, FAS_PARK3J = 1, FAS_AW5J = 2, FAS_AW51 = 3, FAS_AW52 = 4, FAS_PARK51 = 5
};

#define FAS_PARAMS_VERSION 4

typedef struct {
    int32_t version;        /* FAS_PARAMS_VERSION */
    int32_t model;          /* FAS_EULER | FAS_RANS_BL */
    int32_t scheme;         /* FAS_AW3 ... */
    int32_t n_ramp;         /* cycles run at c* = cfl_ramp at the start of a solve */
    double  eta;            /* W ~ I + eta dt* J (Section 4.2) */
    double  d_cut;          /* eigenvalue cutoff fraction d of eq. "cutoff" */
    double  cfl;            /* pseudo CFL number c* */
    double  cfl_ramp;       /* start-up c* (Section 6: 20 for two iterations) */
    double  ramp_growth;    /* >1: c* grows by this factor per cycle after the ramp */
    double  kappa2c;        /* coarse-level first-order dissipation coefficient */
    double  mach, alpha_deg, reynolds, prandtl, prandtl_t;
    int32_t n_levels;       /* multigrid levels (1 = single grid) */
    int32_t cycle_gamma;    /* 1: V-cycle, 2: W-cycle (Section 3) */
    int32_t nu1;            /* pre-smoothing iterations per level */
    int32_t precond_fp32;   /* 1: SGS blocks and sweeps in FP32 */
    /* 0: the preconditioner blocks hold the convective flux-vector
     * splitting alone, as printed (eqs. "d-l-u-matrices-W",
     * "d-l-u-matrices-J"); 1: on RANS levels every face also adds the
     * thin-layer scalar v_f = (mu + mu_t)_f (gamma / Pr) |S_f|^2 /
     * (rho_f Omega_f) to D and subtracts it from the neighbour block (an
     * extension for high-Reynolds-number boundary layers; no effect on
     * Euler) */
    int32_t viscous_blocks;
    /* pseudo time step of Section 4.1 ("c* times the local mesh width"):
     * 0: dt* = c* Omega / (r_xi + r_eta); 1: dt* = c* Omega / max(r_xi,
     * r_eta), i.e. c* times the smaller of the two directional CFL steps,
     * which on a Cartesian cell at alpha = 0 is c* dx / (|v_1| + a), the
     * step of the Fourier analysis section */
    int32_t dt_form;
    /* stall test of fas_cycle / fas_batch_solve: a solve whose fine
     * residual norm gained fewer than stall_orders orders over the last
     * stall_window cycles stops with FAS_STALLED (stall_window 0: off) */
    int32_t stall_window;
    double  stall_orders;
    /* growth test: a norm above growth_limit times the norm before the
     * first cycle counts as divergence (0: off; non-finite norms always
     * do).  A diverged solve restores the fine-level solution from before
     * the cycle that diverged (the last iterate with a finite, not grown
     * norm) */
    double  growth_limit;
    /* levels of the adjoint GMRES preconditioner (0: all n_levels, or
     * 1 .. n_levels): 1 is the transposed smoother increment of the fine
     * level; L adds, for every coarser level l < L, the coarse correction
     * R^T M_l^T P^T built from the transposes of the FAS transfers
     * (Section 3: P the bilinear prolongation, R the volume-weighted
     * agglomeration) and the level's own transposed increment M_l^T (its
     * SGS blocks and dt* at its state from the last cycle).  The
     * preconditioner changes the iteration count, not the solution */
    int32_t adjoint_levels;
    /* 1: the fine level's Baldwin-Lomax eddy viscosity is not evaluated
     * again and keeps the values of its last evaluation (frozen
     * turbulence: the model the adjoint differentiates); 0: evaluated at
     * every residual evaluation's state, as in Section 2 */
    int32_t freeze_mut;
} fas_params;

typedef struct fas_grid_s *fas_grid;     /* opaque, library owned */
typedef struct fas_state_s *fas_state;   /* opaque, bound to one device and stream */

/* Fill *p with defaults: AW3, robust mode (eta 0.5, d 0.5, c* 1e4), the
 * printed convective blocks (viscous_blocks 0), dt_form 1, no stall test,
 * growth limit 1e8, an adjoint preconditioner over every level. */
void fas_params_default(fas_params *p);

/*
 * Grid of ni x nj cells from host node arrays (Section 2: structured
 * cell-centred finite volumes; Section 3: n_levels of 2x2 agglomeration).
 * topology FAS_CGRID: i runs lower wake -> airfoil -> upper wake, j from
 * the wall / wake cut outward, cells (i,0) and (ni-1-i,0) are neighbours
 * across the cut for i < n_wake or i >= ni - n_wake.  FAS_BOX: slip wall at
 * j = 0, far field elsewhere.  ni, nj (and n_wake) must be divisible by
 * 2^(n_levels-1); nj <= 512 (one sweep row per thread); the fine level's
 * preconditioner blocks (640 bytes per padded cell) must stay below 2 GiB,
 * about (ni + nj) * nj < 3.3e6.  The grid is bound to the current HIP
 * device.  Errors: FAS_EINVAL, FAS_ENOMEM.
 */
fas_status fas_grid_create(int32_t topology, int32_t ni, int32_t nj, int32_t n_wake,
                           const double *x_nodes, const double *y_nodes,
                           int32_t n_levels, fas_grid *out);
void fas_grid_destroy(fas_grid g);
/* Move the grid's nodes (host arrays as for fas_grid_create): every level's
 * metrics are recomputed; states on the grid use them from their next call
 * (a moving state's rotated copy from its next rotation).  Synchronises the
 * device.  Errors: FAS_EINVAL (null, other device, non-positive volume),
 * FAS_EDEVICE. */
fas_status fas_grid_set_nodes(fas_grid g, const double *x_nodes, const double *y_nodes);

/*
 * State of one flow case on grid g, initialised with the fine-level
 * solution u0 (device, [4][nj][ni]).  stream is a hipStream_t (NULL: the
 * default stream).  p->n_levels must not exceed the grid's levels.
 */
fas_status fas_state_create(fas_grid g, const fas_params *p, const double *u0,
                            void *stream, fas_state *out);
void fas_state_destroy(fas_state s);
fas_status fas_state_set_params(fas_state s, const fas_params *p);

/*
 * Checkpoint and resume.  A state is its fine-level solution u, the
 * physical time levels of dual time stepping (eq. "nonlin-eq": u^n and
 * u^{n-1} of the BDF2 step in progress), the clock (time t, step dt,
 * physical steps taken) and the count of FAS cycles of the current solve
 * (it sets c* on the start-up ramp).  Flow parameters and mesh motion are
 * the caller's (fas_state_set_params, fas_set_motion).
 *
 * fas_set_state: step = 0 makes the state steady (un, unm1, t, dt
 * ignored); step = 1 restores the first physical step (implicit Euler,
 * un required, unm1 ignored); step >= 2 a BDF2 step (un and unm1
 * required).  dt must be > 0 when step > 0.  The coarse levels' time
 * levels are restricted from the fine ones, as fas_dual_time_step does,
 * so a state restored from fas_get_state / fas_get_time_levels continues
 * bitwise as the uninterrupted one would.  n_cycles >= 0.
 * fas_get_state: u and (nullable) the eddy viscosity of the last
 * fine-level smoother iteration ([nj][ni]).
 * fas_get_time_levels: un, unm1 (device [4][nj][ni], nullable; written
 * only when the state holds them) and the clock (host, nullable).
 * Errors: FAS_EINVAL, FAS_EDEVICE.
 */
fas_status fas_set_state(fas_state s, const double *u, const double *un, const double *unm1, double t,
                         double dt, int32_t step, int32_t n_cycles);
fas_status fas_get_state(fas_state s, double *u, double *mu_t);
fas_status fas_get_time_levels(fas_state s, double *un, double *unm1, double *t, double *dt, int32_t *step,
                               int32_t *n_cycles);
/* Solution and FAS source term of any level ([4][nj_l][ni_l]; source may be NULL). */
fas_status fas_get_level(fas_state s, int32_t level, double *u, double *source);

/* Diagnostic of the banded sweeps (row bands hand their boundary rows on
 * through a per-level device array whose slots hold a sentinel between
 * launches): *n_pending = number of 32-bit words of a level's array that
 * do not hold the sentinel; 0 whenever no sweep is running.  Synchronises
 * the state's stream.  Errors: FAS_EINVAL, FAS_EDEVICE. */
fas_status fas_handoff_pending(fas_state s, int32_t level, int64_t *n_pending);

/*
 * F_l(u_l) - s_l per unit volume on a level (eqs. "nonlin-eq",
 * "nonlin-eq-steady" and "coarse-nonlin-eq"; s = 0 on level 0), with the
 * eddy viscosity evaluated at u_l.  F_out: device [4][nj_l][ni_l].
 */
fas_status fas_residual(fas_state s, int32_t level, double *F_out);

/*
 * n_iter smoother iterations on one level (Section 4: low-storage additive
 * W / preconditioned ARK stages with the block SGS preconditioner of
 * Section 4.4).  c* follows the ramp of the state's cycle counter.
 */
fas_status fas_smooth(fas_state s, int32_t level, int32_t n_iter);

/*
 * x = P^-1 r with the SGS preconditioner built at the current state of a
 * level (eq. "sgs-precon"), r and x device [4][nj_l][ni_l].  For tests and
 * analysis.
 */
fas_status fas_sgs_apply(fas_state s, int32_t level, const double *r, double *x);

/*
 * FAS cycles (Section 3) until the RMS of the density component of the
 * fine residual has dropped by drop_orders (<= 0: run max_cycles) or
 * max_cycles were run.  res_hist (host, may be NULL) receives the norm
 * before the first and after every cycle (max_cycles + 1 entries).
 * Returns FAS_OK, FAS_NOT_CONVERGED, FAS_STALLED (the params' stall test)
 * or FAS_DIVERGED (a non-finite norm, or one above growth_limit times the
 * first; the fine-level solution is then restored to the iterate before
 * the cycle that diverged); *n_done cycles ran, the diverged one included.
 */
fas_status fas_cycle(fas_state s, int32_t max_cycles, double drop_orders,
                     double *res_hist, int32_t *n_done);

/*
 * One physical time step of BDF2 dual time stepping (eq. "nonlin-eq";
 * implicit Euler on the first step, Section 6), with the far-field angle
 * of attack set to alpha_deg, inner FAS cycles as in fas_cycle.
 */
fas_status fas_dual_time_step(fas_state s, double dt, double alpha_deg, int32_t max_inner,
                              double drop_orders, double *res_hist, int32_t *n_inner);

/*
 * Rigid-body pitching on a moving mesh (arbitrary Lagrangian-Eulerian
 * finite volumes; the paper's pitching airfoils, Section 6; the grid-motion
 * terms are a reading, Section 2 does not print them).  The body is turned
 * nose-up by dalpha_deg about (pivot_x, pivot_y), i.e. the whole mesh of
 * every level rotates by -dalpha_deg, turning at -rate_deg (degrees per
 * unit time); the free stream keeps the angle of the parameters.  Face
 * fluxes gain -(w . S) (u_L + u_R) / 2 with w the grid velocity at the face
 * midpoint, spectral radii, far-field Riemann states and the split
 * Jacobians use velocities relative to the mesh, walls move with it (a
 * moving wall does the pressure work p_w (w . S)); volumes are unchanged.
 * Call before fas_dual_time_step for the state at t_{n+1} (with alpha_deg
 * of that call kept at the free-stream angle).  The first call allocates
 * per-state geometry.  The adjoint entry points and batches reject moving
 * meshes.  Errors: FAS_EINVAL, FAS_ENOMEM, FAS_EDEVICE.
 */
fas_status fas_set_motion(fas_state s, double dalpha_deg, double rate_deg, double pivot_x, double pivot_y);

/*
 * Opt-in timing of kernel classes with HIP events recorded on the state's
 * stream around each launch (adds a little launch overhead while on).
 * fas_profile resets the counters and switches timing on (enable = 1) or
 * off; fas_profile_read synchronises the stream and returns, per class,
 * the summed kernel time in ms and the number of launches (arrays of
 * FAS_PROF_NCLASS entries, either may be NULL).
 */
enum { FAS_PROF_SWEEP = 0, FAS_PROF_RESIDUAL = 1, FAS_PROF_BLOCKS = 2, FAS_PROF_NCLASS = 3 };
fas_status fas_profile(fas_state s, int32_t enable);
fas_status fas_profile_read(fas_state s, double *ms, int64_t *count);

/*
 * Batched steady solves: n independent flow cases, possibly on grids of
 * different sizes and with different flow conditions, advanced together by
 * the FAS cycle of Section 3 with the smoother of Section 4 (each case
 * keeps its own exact SGS order).  Every kernel of a cycle is one launch
 * over all cases; converged cases are masked by a device flag.
 *
 * fas_batch_create: the states must be on one device and share model,
 * scheme, n_levels, cycle_gamma, nu1 and precond_fp32, and must be steady
 * (no fas_dual_time_step taken).  The batch reads each state's flow
 * parameters at creation and works in place on the states' device buffers:
 * the states must outlive the batch and must not be used while a batch
 * call runs.  stream: hipStream_t for the batch's work (NULL: the batch
 * creates its own non-blocking stream).  autotune = 1 times every sweep
 * configuration that covers the tallest grid of each level on the batch
 * itself and keeps the fastest; 0 picks one by grid height.  groups > 1
 * splits the cases into that many groups (at most n; the cases in
 * descending order of ni + nj, dealt to the groups in turn), each a batch of
 * its own with its own stream, autotuning and captured cycle; fas_batch_solve
 * then runs the groups' cycles concurrently, so kernels of one group fill
 * the compute units another group's long sweep chains leave idle.  Every
 * case's iterates are those of a solve on its own whatever the grouping.
 * groups 0 or 1: one group.
 * Errors: FAS_EINVAL, FAS_ENOMEM, FAS_EDEVICE.
 */
typedef struct fas_batch_s *fas_batch;
fas_status fas_batch_create(int32_t n, const fas_state *states, void *stream, int32_t autotune,
                            int32_t groups, fas_batch *out);
void fas_batch_destroy(fas_batch b);

/*
 * Up to max_cycles FAS cycles for every case, each case stopping on its own
 * when its fine residual norm (as in fas_cycle) has dropped by drop_orders
 * (<= 0: run max_cycles), is not finite, or the cap is reached.
 * use_graph = 1 captures one batched cycle (cycle, norm, status update) in a
 * HIP graph once and replays it; 0 launches the same kernels directly.
 * Outputs (host, nullable): n_done[n] cycles run per case, status[n]
 * (FAS_OK, FAS_NOT_CONVERGED, FAS_STALLED, FAS_DIVERGED, with the
 * diverged case rolled back as in fas_cycle), res_hist[n][max_cycles + 1]
 * norms before the first and after every cycle (entries after n_done are
 * unspecified).  Returns the worst per-case status.
 */
fas_status fas_batch_solve(fas_batch b, int32_t max_cycles, double drop_orders, int32_t use_graph,
                           int32_t *n_done, int32_t *status, double *res_hist);

/* Sweep configuration chosen for a level (index, and rows one launch covers
 * per case), and a manual override (cfg -1: pick by grid height; FAS_EINVAL
 * if the configuration covers fewer rows than the level's tallest grid).
 * With groups, the query reports the group holding the level's tallest
 * grid and the override applies to every group.
 * Configurations 0 .. fas_sweep_config_count() - 1: one workgroup per case
 * (four or eight threads per row, or one thread per row), or row bands of one
 * workgroup each, several per case, handing the band-boundary rows on
 * through device memory (the forward and backward sweeps of Section 4.4 keep
 * their exact order).  A banded configuration whose workgroups cannot all
 * be resident at once runs as the height-based default instead. */
fas_status fas_batch_sweep_config(fas_batch b, int32_t level, int32_t *cfg, int32_t *rows);
fas_status fas_batch_set_sweep_config(fas_batch b, int32_t level, int32_t cfg);
int32_t fas_sweep_config_count(void);
/* Configuration cfg: kind (0: four threads per row, one workgroup per
 * case; 1: one thread per row; 2: row bands of four-thread rows; 3: eight
 * threads per row, one workgroup per case; 4: row bands of eight-thread
 * rows), threads per workgroup, rows
 * per workgroup, prefetch depth (hyperplanes per batch) for FP64 and FP32
 * blocks.  Errors: FAS_EINVAL. */
fas_status fas_sweep_config_info(int32_t cfg, int32_t *kind, int32_t *threads, int32_t *rows_per_workgroup,
                                 int32_t *depth_fp64, int32_t *depth_fp32);

/* Kernel-class timing of the batch's direct launches (as fas_profile;
 * launches replayed from a graph are not timed).  With groups, the sums
 * over the groups, whose launches overlap in time. */
fas_status fas_batch_profile(fas_batch b, int32_t enable);
fas_status fas_batch_profile_read(fas_batch b, double *ms, int64_t *count);

/*
 * Discrete adjoint of the steady fine-level residual F(u) (Section 2
 * discretisation; eq. "nonlin-eq-steady").  Derivatives are exact
 * derivatives of the discrete F with the eddy viscosity frozen at the
 * current state (frozen-turbulence adjoint); they do not include the
 * Baldwin-Lomax model's own dependence on u.  All arrays are device
 * [4][nj][ni] on the fine level.
 *
 * fas_forces: lift and drag coefficients of the wall pressure force of
 * the current solution (the residual's wall flux p_w S summed over the
 * solid-wall faces, q_inf = rho_inf |v_inf|^2 / 2, chord 1; host values),
 * and, if dcl_du is not NULL, dC_L/du.
 * fas_vjp: out = (dF/du)^T lam.
 * fas_param_partials: dF/dalpha (per degree) and dF/dM at fixed u (either
 * may be NULL), and dcl_dparam (host [2], may be NULL): the explicit
 * partials of C_L with respect to alpha (per degree) and M at fixed u.
 * fas_sgs_apply_transpose: x = P^-T r for the SGS preconditioner built at
 * the current state (transpose of fas_sgs_apply).
 * fas_adjoint_solve: (dF/du)^T lam = rhs by the transposed smoother (the
 * stages of the state's scheme with the transposed increments), starting
 * from lam (in/out), until the RMS of the adjoint residual has dropped by
 * drop_orders or max_iter iterations ran; res_hist (host, may be NULL,
 * max_iter + 1 entries).  Returns FAS_OK, FAS_NOT_CONVERGED or
 * FAS_DIVERGED.
 * fas_lift_gradient: at a converged state, dC_L/dalpha (per degree) and
 * dC_L/dM into grad (host [2]) by the adjoint, dC_L/dq = dC_L/dq|_u +
 * lam^T dF/dq with (dF/du)^T lam = -dC_L/du; cl (host, may be NULL).
 */
fas_status fas_forces(fas_state s, double *cl, double *cd, double *dcl_du);
fas_status fas_vjp(fas_state s, const double *lam, double *out);
/*
 * out = (dS/du)^T lam for the map S: u -> one fine-level smoother
 * iteration from u (Section 4: the stages of the state's scheme with the
 * split f^c / f^v blending of Section 4.1), with the quantities a smoother
 * iteration freezes at its starting state held fixed: dt*, the SGS blocks
 * and the eddy viscosity.  The transpose runs the stages backwards: each
 * stage applies P^-T (the transposed sweeps of eq. "sgs-precon") and the
 * transposed Jacobians of f^c and f^v at the stored stage states.  Steady
 * fixed-mesh states only; the state's solution is left unchanged.  lam,
 * out: device [4][nj][ni].  Errors: FAS_EINVAL (null, moving mesh, a dual
 * time step taken), FAS_ENOMEM, FAS_EDEVICE.
 */
fas_status fas_vjp_smooth(fas_state s, const double *lam, double *out);
fas_status fas_param_partials(fas_state s, double *dF_dalpha, double *dF_dmach, double *dcl_dparam);
fas_status fas_sgs_apply_transpose(fas_state s, const double *r, double *x);
fas_status fas_adjoint_solve(fas_state s, const double *rhs, double *lam, int32_t max_iter,
                             double drop_orders, double *res_hist, int32_t *n_iter);
fas_status fas_lift_gradient(fas_state s, int32_t max_iter, double drop_orders, double *cl,
                             double *grad, double *res_hist, int32_t *n_iter);

/*
 * Discrete adjoint of dual time stepping (eq. "nonlin-eq", implicit Euler on
 * the first step and BDF2 after it) on a fixed mesh, with checkpointing.
 * Functional: the time-averaged lift J = (1/N) sum_{n=1..N} C_L(u^n) of
 * N = n_steps physical steps of size dt started from the state's current
 * solution u^0, which must be the converged steady solution at
 * alpha_deg[0] (fas_cycle first); step n sets the far-field angle to
 * alpha_deg[n] (host, n_steps + 1 entries) and runs inner FAS cycles as
 * fas_dual_time_step (max_inner, inner_drop).  The adjoint runs backwards
 * through the steps and the steady start, each step an adjoint solve of
 * (dF/du + tau I)^T (tau = 1/dt, then 3/(2 dt); 0 for the steady start) as
 * in fas_adjoint_solve (adj_max_iter, adj_drop) with the eddy viscosity
 * frozen at that step's state (frozen turbulence).  Only every
 * checkpoint_every-th step's state is kept (with its previous time level):
 * the reverse pass recomputes the steps in between from the checkpoint
 * before them (checkpoint_every = 1 keeps every state, larger values trade
 * recomputation for memory).  Outputs (host): J, dJ/dM, dJ/dalpha_n per
 * degree for n = 0..N (dJ_dalpha, n_steps + 1 entries; entry 0 through the
 * steady start), the adjoint iterations per step and the orders of adjoint
 * residual drop each reached (adj_iters, adj_orders, nullable, n_steps + 1
 * entries; a step short of adj_drop leaves its gradient terms unconverged)
 * and the number of recomputed steps (nullable).  The adjoint solves use the
 * preconditioner at the full c*.  On
 * return the state holds the last step's solution and time levels, as after
 * fas_dual_time_step.  Errors: FAS_EINVAL (bad arguments, a moving mesh, a
 * state that has taken dual time steps), FAS_ENOMEM, FAS_DIVERGED,
 * FAS_EDEVICE.
 */
fas_status fas_unsteady_lift_gradient(fas_state s, int32_t n_steps, double dt, const double *alpha_deg,
                                      int32_t max_inner, double inner_drop, int32_t checkpoint_every,
                                      int32_t adj_max_iter, double adj_drop, double *J, double *dJ_dmach,
                                      double *dJ_dalpha, int32_t *adj_iters, double *adj_orders,
                                      int32_t *recomputed_steps);

/*
 * Grid-node sensitivities of the steady fine-level residual and the lift.
 * The residual depends on the nodes through the metrics of Section 2 (face
 * vectors, mean face vectors, volumes, cell centres, and the ghost cells'
 * centres reflected across the boundary faces); the eddy viscosity is
 * frozen, so the turbulence model's wall distance is not differentiated.
 * Node arrays: device [(nj+1)][(ni+1)], i fastest, every node an
 * independent coordinate (the coinciding wake-cut nodes included).
 * fas_vjp_nodes: dx = (dF/dx)^T lam, dy = (dF/dy)^T lam (overwritten), lam
 * device [4][nj][ni].
 * fas_lift_gradient_nodes: fas_lift_gradient, plus dC_L/dx and dC_L/dy of
 * every node: dC_L/dX = dC_L/dX|_u + lam^T dF/dX with the same adjoint
 * solution.  Errors as fas_lift_gradient; moving meshes: FAS_EINVAL.
 */
fas_status fas_vjp_nodes(fas_state s, const double *lam, double *dx, double *dy);
fas_status fas_lift_gradient_nodes(fas_state s, int32_t max_iter, double drop_orders, double *cl,
                                   double *grad, double *dcl_dx, double *dcl_dy, double *res_hist,
                                   int32_t *n_iter);

/*
 * Discrete Fourier analysis of the smoothers (Section "Discrete Fourier
 * Analysis"): amplification and smoothing factors of one AW or
 * preconditioned ARK iteration for the Euler equations linearised about a
 * constant state, JST scheme (the constant state's pressure sensor is zero:
 * fourth differences only, eps4 = (|v_k| + a)/32) and the SGS preconditioner
 * with the cutoff splitting, on a periodic Cartesian mesh; every pair of
 * phase angles gives one 4x4 complex iteration matrix.
 * cases: host array of n_cases descriptors.  Mesh: nx cells of width 1/nx
 * in x, dy = ar dx (or dx / ar); nx and ny (phase angles in y, normally
 * nx ar) even and >= 2; phase angles 2 pi k / n, k = -n/2 + 1 .. n/2.
 * Steps: dt* = cstar b and, with unsteady = 1, the BDF2 terms 3/(2 dt)
 * with dt = c b, b = min(dx / (|v_1| + a), dy / (|v_2| + a)) (the smaller
 * directional CFL step).  Preconditioner P: the SGS factorisation (eq.
 * "sgs-precon"), the exact first-order operator D + L + U, or none.  The amplification factor is the largest
 * spectral radius over all pairs, the smoothing factor over the pairs with
 * max(|Theta_x|, |Theta_y|) >= pi/2.
 * amp, smooth: device [n_cases]; radius: device, nullable, the spectral
 * radius of every pair, case after case, Theta_x slowest (sum of nx ny
 * values).  Enqueued on stream; returns once the results are written.
 * Errors: FAS_EINVAL (sizes or parameters), FAS_EDEVICE.
 */
typedef struct {
    double u[4];            /* linearisation state (rho, rho v1, rho v2, rho E), rho, p > 0 */
    int32_t scheme;         /* FAS_AW3 ... FAS_PARK51 */
    int32_t nx, ny;
    int32_t unsteady;       /* 1: dual time stepping (BDF2 terms), 0: steady */
    double cstar;           /* pseudo CFL c* (> 0) */
    double d;               /* eigenvalue cutoff (>= 0) */
    double eta;             /* W parameter (additive W schemes) */
    double ar;              /* aspect ratio (> 0), see mesh */
    double c;               /* physical CFL (> 0 when unsteady) */
    int32_t precond;        /* FAS_DFA_SGS, FAS_DFA_EXACT (P = D + L + U, the
                             * tables' exact-preconditioner columns) or
                             * FAS_DFA_NONE (P = I, the explicit schemes) */
    int32_t unsplit;        /* 1: every beta = 1 (the unsplit ERK / W forms) */
    int32_t mesh;           /* FAS_DFA_MESH_AR_DX: dy = ar dx; FAS_DFA_MESH_DX_OVER_AR:
                             * dy = dx / ar (the ny cells fill the unit height) */
    int32_t reserved;       /* 0 */
} fas_dfa_case;
enum { FAS_DFA_SGS = 0, FAS_DFA_EXACT = 1, FAS_DFA_NONE = 2 };
enum { FAS_DFA_MESH_AR_DX = 0, FAS_DFA_MESH_DX_OVER_AR = 1 };
fas_status fas_dfa(const fas_dfa_case *cases, int32_t n_cases, double *amp, double *smooth, double *radius,
                   void *stream);

/*
 * fas_dfa for callers that cannot allocate device memory (serving loops
 * and harnesses that forbid hipMalloc): the same analysis with no
 * hipMalloc, hipFree or other allocating call.  The per-case descriptor
 * table lives in a fixed device array of FAS_DFA_NOALLOC_MAX_CASES entries
 * (about 190 KiB, held by each GPU the library runs on until the process
 * ends); n_cases above that limit gives FAS_EINVAL.  Arguments, outputs and
 * synchronisation as fas_dfa.  Every call on a GPU shares that GPU's table:
 * the library serialises its own calls until their results are written;
 * calls that overlap through other means (another copy of the library in
 * the process) race.
 */
#define FAS_DFA_NOALLOC_MAX_CASES 1024
fas_status fas_dfa_noalloc(const fas_dfa_case *cases, int32_t n_cases, double *amp, double *smooth,
                           double *radius, void *stream);

/*
 * Launch-size rule of the residual and preconditioner-block kernels: a
 * launch of at most max_cells cells (over all cases of a batch) runs the
 * four-lanes-per-cell variants (one face per lane), a larger one the
 * one-lane-per-cell variants.  Both give bitwise the same results.
 * max_cells < 0 restores the default (65536).  Process-wide; takes
 * effect for launches enqueued after the call (graphs captured earlier
 * keep their kernels).  Returns the previous value.
 */
int64_t fas_set_four_lane_limit(int64_t max_cells);

/* Message of the last failing call on this thread (never NULL). */
const char *fas_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FAS_H */
