/*
 * lgsim.h -- C-ABI of the MI355X (gfx950) local-global hyperelastic solver with
 * frictional contact (liblgsim_hip.so).
 *
 * The solver implements Algorithm 4 of "Fast But Accurate: A Real-Time
 * Hyperelastic Simulator with Robust Frictional Contact" (arXiv 2503.15078):
 * per frame, collision detection, the Delassus operator W = H S^T S H^T and the
 * predicted state; per local-global iteration, the per-tet local projections
 * (Eq. PD local), the right-hand side b (Eq. PD global), the non-smooth
 * Fischer-Burmeister contact terms (Sec. 5.2, App. B), a Conjugate Residual
 * solve of the Schur system (Sec. 5.2-5.3, Sec. 6) and the constrained global
 * step q = S^T S (b + h^2 J^T lambda) (Sec. 4.2, Eq. rhs correction).
 *
 * Conventions for every call:
 *  - Arrays passed in are host memory owned by the caller; they are read during
 *    the call and copied (never retained).  Arrays passed out are host memory
 *    owned by the caller and sized as documented.  The handle owns all device
 *    memory it allocates.
 *  - Node and tet arrays are in the caller's order; the library renumbers nodes
 *    internally and converts back on every read.
 *  - Every call returns SIM_OK (0) or a negative SIM_E_* code; on error the
 *    message is available from sim_last_error() (thread-local) and the handle's
 *    simulation state is unchanged unless stated otherwise.  No C++ exception
 *    crosses the ABI.
 *  - One handle must not be used by two threads at once.  Work is enqueued on the
 *    handle's HIP stream; calls that return host data synchronise that stream.
 */
#ifndef LGSIM_H
#define LGSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SIM_OK = 0,
  SIM_E_ARG = -1,       /* invalid argument                                        */
  SIM_E_MESH = -2,      /* empty mesh, index out of range, unused node, volume <= 0 */
  SIM_E_NOT_SPD = -3,   /* system matrix not positive definite                     */
  SIM_E_NOMEM = -4,     /* host or device allocation failed                        */
  SIM_E_DEVICE = -5,    /* HIP runtime error                                       */
  SIM_E_STATE = -6,     /* call out of order                                       */
  SIM_E_DIVERGED = -7,  /* non-finite state produced; state rolled back to frame start */
  SIM_E_CAPACITY = -8   /* more contacts than sim_options.max_contacts             */
};

enum { SIM_ARAP = 0, SIM_COROT = 1, SIM_STABLE_NH = 2, SIM_MOONEY_RIVLIN = 3 };
enum { SIM_OBST_HALFSPACE = 0, SIM_OBST_BOX = 1, SIM_OBST_CYLINDER = 2, SIM_OBST_BINDING = 3 };
enum { SIM_WARM_ZERO = 0, SIM_WARM_PREV = 1, SIM_WARM_MLP = 2, SIM_WARM_MLP_PERSIST = 3 };

typedef struct lgsim* sim_t; /* opaque, library-owned */

/* Tetrahedral mesh (Sec. 3.1: positions q, velocities v; Sec. 3.3: one local
 * constraint per tet).  rest_xyz [n][3] and tets [m][4] are required; tets must be
 * positively oriented.  init_xyz/init_vel [n][3] default to the rest shape and 0.
 * Pinned nodes (positional constraints, Sec. 3.3 local step) carry a group index;
 * the target of group g moves rigidly (sim_set_pin_motion). */
typedef struct {
  int32_t n_nodes, n_tets;
  const double* rest_xyz;
  const int32_t* tets;
  const double* init_xyz;
  const double* init_vel;
  int32_t n_pins;
  const int32_t* pin_nodes;
  const int32_t* pin_group;
} sim_mesh;

/* Material (Sec. 3.3 local energies; models per Sec. 7.4): model is one of SIM_ARAP,
 * SIM_COROT, SIM_STABLE_NH, SIM_MOONEY_RIVLIN.  Per-tet arrays [m] override the
 * defaults when non-null. */
typedef struct {
  int32_t model;
  double E, nu, rho;
  const int32_t* tet_model;
  const double* tet_E;
  const double* tet_nu;
} sim_material;

/* Options.  cr_iters: Conjugate Residual iterations per L-G iteration (Sec. 7.1: 10).
 * warm: initial impulse of a frame (SIM_WARM_*).  ncp_tol/max_iters: stopping rule of
 * sim_step with iters == 0.  max_contacts: contact capacity (device buffers).
 * hip_stream: a hipStream_t to enqueue on (null: the library creates its own).
 * ncp / precond: NCP function and complementarity preconditioner of the contact rows
 * (SIM_NCP_*, SIM_PRECOND_*; the defaults are the method's).  global_step: SIM_GLOBAL_*.
 * lg_form: SIM_LG_*. */
typedef struct {
  double gravity[3];
  double pin_weight_scale; /* h^2 w_pin = 1e3 * scale * [A_n]_vv                */
  double contact_margin;   /* metres; contact iff min(sdf(q_t), sdf(q~)) < margin */
  int32_t cr_iters;        /* at most 1024                                        */
  int32_t warm;
  double ncp_tol;          /* metres */
  int32_t max_iters;
  int32_t max_contacts;
  void* hip_stream;
  double cr_tol;           /* > 0: CR also stops once |r| <= cr_tol |r_0| (0: fixed count) */
  int32_t cr_variant;      /* SIM_CR_TEXTBOOK (default) or SIM_CR_PIPELINED */
  int32_t graph;           /* 1 (default): fixed-iteration frames replay a captured hipGraph */
  int32_t ncp;             /* SIM_NCP_FB (default) or SIM_NCP_MINMAP */
  int32_t precond;         /* SIM_PRECOND_DELASSUS (default) or SIM_PRECOND_MASS */
  int32_t global_step;     /* SIM_GLOBAL_DIRECT (default) or SIM_GLOBAL_JACOBI */
  int32_t lg_form;         /* SIM_LG_PD (default) or SIM_LG_ADMM */
  int32_t self_contact;    /* 1: vertex-triangle self-contact rows (single-scene handles)  */
  double self_mu;          /* friction coefficient of the self-contact rows                */
} sim_options;

/* Forms of the Conjugate Residual iteration; both give the same iterates in exact
 * arithmetic.  TEXTBOOK exchanges data between the solver's blocks twice per step
 * (the residual, then the inner products) and reaches float32 accuracy when run to
 * convergence.  PIPELINED carries M r and M p by recurrence, with M r replaced by its
 * true value after every exchange, and exchanges once per step: about half the
 * synchronisation, with a relative accuracy floor near 1e-4 of the solution when run
 * to convergence (fine for a fixed handful of steps or a loose tolerance). */
enum { SIM_CR_TEXTBOOK = 0, SIM_CR_PIPELINED = 1 };
/* NCP functions of the contact rows (App. B): Fischer-Burmeister (the method's) or the
 * minimum map.  Min-map rows: phi_n = delta_n with omega_n = 1, E_n = 0 where
 * delta_n <= r_n lambda_n, else phi_n = r_n lambda_n with omega_n = 0, E_n = r_n; friction
 * rows with lambda_n > 0 (and mu > 0): omega_f = 1 and E_f = 0 while
 * |vdot_f| <= r_f (mu lambda_n - |lambda_f|), else E_f = (|vdot_f| - r_f (mu lambda_n -
 * |lambda_f|)) / (mu lambda_n); otherwise omega_f = 0, E_f = 1. */
enum { SIM_NCP_FB = 0, SIM_NCP_MINMAP = 1 };
/* Complementarity preconditioner (Sec. 5.4): r_n = h^2 W_jj, r_f = h W_jj from the
 * Delassus diagonal (the method's), or the mass-inverse form r_n = h^2 / m_v,
 * r_f = h / m_v that Sec. 7's stick-sliding test compares against (m_v: lumped mass of
 * the contact node). */
enum { SIM_PRECOND_DELASSUS = 0, SIM_PRECOND_MASS = 1 };
/* Global step of each L-G iteration: the direct solve q = A^-1 b through S^T S (Sec. 4,
 * the method), or the incomplete solution that Sec. 7's convergence comparison uses as
 * its baseline, one Jacobi sweep q <- q + D^-1 (b - A q) from the current iterate
 * (D = diag A).  The Jacobi step is implemented for scenes without obstacles: sim_step
 * and sim_run_iterations return SIM_E_STATE when a Jacobi handle has obstacles.
 * Currently switched off (SIM_E_STATE from sim_step, sim_run_iterations and
 * sim_lg_energy): a device run that included it ended in a GPU fault whose cause has not
 * been established. */
enum { SIM_GLOBAL_DIRECT = 0, SIM_GLOBAL_JACOBI = 1 };
/* Local-global form: projective dynamics (the local step projects F_t = G_t q), or
 * ADMM-PD, the paper's other implementation (local step of the cited ADMM-PD method):
 * per-tet dual variables u_t, zero at every frame start; the local step takes
 * p_t = prox(F_t + u_t), updates u_t += F_t - p_t, and the global step uses p_t - u_t.
 * ADMM-PD's converged iterate is stationary for the hyperelastic incremental potential
 * itself; PD's minimises its quadratic-penalty relaxation.  ARAP takes its energy
 * mu |F - R|^2 (prox s* = (sigma + 1) / 2) in the ADMM form instead of the SO(3)
 * indicator of the PD form. */
enum { SIM_LG_PD = 0, SIM_LG_ADMM = 1 };

/* Obstacles (App. A: analytic contact partners).  geom by type:
 *   HALFSPACE [px,py,pz, nx,ny,nz]        solid where n.(x-p) < 0
 *   BOX       [cx,cy,cz, hx,hy,hz]        axis-aligned box, half extents
 *   CYLINDER  [ax,ay,az, bx,by,bz, r]     capped cylinder
 *   BINDING   [px,py,pz, cx,cy,cz, e, v]  bilateral row at node v (caller order, within
 *                                         its scene): c.x_v = c.p^ with compliance e >= 0
 *                                         (Sec. 3.2 binding contact, App. A bilateral items:
 *                                         phi_b = delta_b + e lambda_b; e = 0 hard), active
 *                                         at every frame, no friction (mu, vel ignored)
 * mu is the Coulomb coefficient; vel is the obstacle velocity u^ entering d_f. */
typedef struct {
  int32_t type;
  double geom[10];
  double mu;
  double vel[3];
} sim_obstacle;

/* Surface triangles of a self-contact handle: the faces that belong to exactly one
 * tet, each oriented with its normal pointing away from its tet's fourth vertex, as
 * caller node triples [n][3] sorted by their sorted triple; *n = count (SIM_E_CAPACITY
 * when count > cap, nothing copied; 0 triangles without self contact).
 * A pair (v, i) of a surface vertex and a triangle that v is not a corner of is a
 * self contact iff, at q_t and at q~, v projects into the triangle (all barycentric
 * weights >= 0), its signed distance along the normal at q_t exceeds -margin, v faces the
 * triangle at q_t (the sum of the cross products of v's surface triangles has a negative
 * dot product with the triangle's normal) and the smaller of the two distances is below
 * the margin; evaluated in float64 from the float32 state with the dot products summed
 * left to right. */
int sim_surface_triangles(sim_t s, int32_t* tris, int32_t cap, int32_t* n);

/* Per-frame statistics.  ms_phase: 0 frame setup (predict, collision, Delassus,
 * warm start), 1 local step + RHS, 2 S pass, 3 contact evaluation, 4 CR solve,
 * 5 correction + S^T pass, 6 integrate, 7 residual. */
typedef struct {
  int32_t iters_done, n_contacts;
  double ncp_res;
  float ms_frame;
  float ms_phase[8];
} sim_stats;

/* A contact: caller node id, obstacle index, frame rows (n, f1, f2), impulse
 * (lambda_n, lambda_f1, lambda_f2) in that frame, signed distance at q_t.
 * Self-contact rows (sim_options.self_contact; Sec. 6 collision detection: H may couple
 * degrees of freedom of one object; the row of App. A on the gap between surface vertex
 * `node` and the point sum_a w_a x_a of surface triangle i, with barycentric weights w
 * and the triangle's outward normal n, taken at q_t) carry obstacle = -1 - i, i the
 * index into the list of sim_surface_triangles; their gap is n . (x_v - p) at q_t. */
typedef struct {
  int32_t node, obstacle;
  double frame[9];
  double lambda[3];
  double gap;
} sim_contact;

/* Fill *opt with defaults: gravity (0,0,-9.81), pin scale 1, margin 0, 10 CR
 * iterations, previous-frame warm start, ncp_tol 1e-6, max_iters 200,
 * max_contacts 2048, null stream. */
int sim_options_default(sim_options* opt);

/* Build a solver (Algorithm 4, first two lines): validates the mesh, assembles the
 * constant system matrix A = M + h^2 sum w G^T G (Eq. PD global), factors it in
 * float64 and forms S = L^-1 (Theorem 1, Algorithm 2), then uploads everything.
 * h > 0 is the time step.  opt may be null (defaults).  On success *out owns the
 * device state.  Errors: SIM_E_ARG, SIM_E_MESH, SIM_E_NOT_SPD, SIM_E_NOMEM,
 * SIM_E_DEVICE. */
int sim_create(const sim_mesh* mesh, const sim_material* mat, double h, const sim_options* opt,
               sim_t* out);

/* Change the Conjugate Residual settings of the constraint solve (Sec. 6) between
 * frames: at most cr_iters iterations (<= 1024), stopping early per scene once
 * |r| <= cr_tol |r_0| when cr_tol > 0, in the form cr_variant (SIM_CR_*). */
int sim_set_solver(sim_t s, int32_t cr_iters, double cr_tol, int32_t cr_variant);

/* Measurement: average duration (ms) of `reps` back-to-back launches of one kernel pass
 * on the handle's stream between a single pair of HIP events, on the current buffers
 * (which = 0: y = S b, which = 1: u = q~ + S^T y, the result going to a scratch buffer;
 * which = 2: the local step at the current iterate, rewriting its per-tet corner forces
 * with the same values; SIM_E_STATE for ADMM-PD handles, whose local step updates the
 * duals).  The state is unchanged. */
int sim_time_kernel(sim_t s, int32_t which, int32_t reps, float* ms_avg);

/* Measurement of the constraint solve (Sec. 6, CR) on the current contact state: one
 * untimed launch, then `reps` (1..SIM_PROFILE_MAX_REPS, else SIM_E_ARG) launches back to
 * back on the handle's stream between one pair of HIP events, each with barrier flags
 * of its own zeroed before the first; then one launch from the saved impulses that
 * records wall-clock stamps of its first block.  A launch adds its increment to the
 * impulses only at its end, so every launch does the same work.  out[6]: [0] ms per
 * launch (events), [1] the stamped launch's in-kernel duration (us), [2] set-up until the
 * first exchange (us), [3] mean exchange (us per device-wide exchange: publishing,
 * waiting at the barrier, reading the other blocks' data), [4] mean barrier wait alone
 * (us), [5] exchanges.  Call after a frame or sim_run_iterations (contacts evaluated);
 * impulses are restored, other state is unchanged.  Its buffers are allocated on the
 * first call. */
#define SIM_PROFILE_MAX_REPS 64
int sim_profile_cr(sim_t s, int32_t reps, float* out);

/* Measurement: the wall-clock stamps (ticks at hipDeviceAttributeWallClockRate kHz) of
 * the last sim_profile_cr's stamped launch, taken by the first block: [0] start, [1] end,
 * then for each device-wide barrier b = 1, 2, ...: entry, exit, end of the read of the
 * data the other blocks published before it, end of the products with the Delassus rows
 * that follow (0 where none follow).  Copies min(cap, count) values; *n receives the
 * count (0 before the first sim_profile_cr). */
int sim_read_cr_stamps(sim_t s, uint64_t* out, int32_t cap, int32_t* n);

/* Frames with a fixed iteration count are recorded once into a hipGraph (frame setup,
 * the iterations, integration: one launch per frame) and replayed; the graph is
 * re-recorded when a setting or the device state layout changes.  on = 0 launches the
 * kernels one by one (needed for per-phase timing in sim_stats.ms_phase, which is zero
 * for replayed frames). */
int sim_set_graph(sim_t s, int32_t on);

/* Launch configuration: CR blocks (one per CU at most), CR form (SIM_CR_*), S-pass
 * segment length in floats (multiple of 4, >= 64), element-kernel block size (64, 128,
 * 192 or 256 threads), the most rows of S that share one S-pass wavefront (consecutive
 * rows stored from the same column quad) and the most columns that share one S^T-pass
 * wavefront (consecutive columns of one elimination-tree chain), each 1, 2, 4 or 8;
 * ms_frame: the autotuner's measured time of the chosen one. */
typedef struct {
  int32_t cr_blocks, cr_variant, seg_floats, elem_block;
  int32_t row_group, col_group;
  float ms_frame;
} sim_tuning;
int sim_get_tuning(sim_t s, sim_tuning* t);
int sim_set_tuning(sim_t s, const sim_tuning* t);
/* Autotuner, from the current state (restored afterwards).  The S-pass row group and
 * segment length (1/2/4/8 x 1024/2048/4096) and the S^T-pass column group (1/2/4/8) are
 * chosen by the times of 30 back-to-back launches of those kernels; then the element
 * block (64/128/256), CR blocks (16..256) and both CR forms if allow_pipelined are chosen
 * by coordinate search over the time of `frames` frames of `iters` iterations.  The
 * fastest configuration is kept and reported in *best.  The candidates that change
 * rounding (groups, segment length, CR form) stay within the parity tolerances. */
int sim_autotune(sim_t s, int32_t frames, int32_t iters, int32_t allow_pipelined, sim_tuning* best);

/* Replace the obstacle set of a single-scene handle (n >= 0; at most 64), e.g. to move
 * obstacles between frames.  Obstacles are the analytic contact partners of App. A (their
 * surface velocity enters the friction rows as h d_f) plus the bilateral rows of Sec. 3.2
 * (binding type).  obs is borrowed for the call and copied.  SIM_E_ARG for a bad count,
 * type, non-finite geometry, a zero normal, a degenerate cylinder or a binding node out of
 * range; SIM_E_STATE on a batch handle.  Takes effect at the next frame start. */
int sim_set_obstacles(sim_t s, int32_t n, const sim_obstacle* obs);

/* Rigid motion of each pin group (the moving positional constraints of Sec. 3.3's local
 * step, e.g. the twisted ends of Sec. 7's bar): target(t) = pivot + lin_vel t +
 * R(ang_vel t)(x0 - pivot), x0 the pinned node's initial position, R the rotation by the
 * vector ang_vel t.  Arrays [n_groups][3], borrowed and copied; n_groups must cover every
 * group index used by the mesh (SIM_E_ARG), non-finite values are SIM_E_ARG, a batch
 * handle is SIM_E_STATE.  The pin weights stay those fixed at creation (they are part of
 * the constant system matrix of Sec. 4); only targets move. */
int sim_set_pin_motion(sim_t s, int32_t n_groups, const double* lin_vel, const double* ang_vel,
                       const double* pivot);

/* Advance `frames` frames (Algorithm 4 outer loop).  iters > 0: that many L-G
 * iterations per frame; iters == 0: iterate until the NCP residual (max-norm, metres)
 * is <= opt.ncp_tol or opt.max_iters is reached.  With graphs on (the default), such a
 * frame runs its iterations in replayed chunks of 4, each iteration followed by the
 * residual and a convergence check on the device, and the host reads the outcome once per
 * chunk; iterations after convergence return at once on the device.  With graphs off the
 * host reads the residual after every iteration (and per-phase times are resolved).
 * stats: null or [frames].
 * Errors: SIM_E_CAPACITY (contacts beyond max_contacts; frame not advanced),
 * SIM_E_DIVERGED (non-finite state; rolled back), SIM_E_DEVICE. */
int sim_step(sim_t s, int32_t frames, int32_t iters, sim_stats* stats);

/* Copy the state to the host: q_t and v_t of Algorithm 4 after the last frame, xyz/vel
 * [n][3] float64 in caller order (each may be null), and the last frame's contacts in
 * canonical (node, obstacle) order into contacts[cap] (may be null): frame rows n, f1, f2
 * (Sec. 3.2), the impulse lambda in that frame and the float64 gap at the frame start;
 * *n_contacts (may be null) receives the total count (more than cap is not an error: the
 * first cap are copied).  Buffers are caller-owned; the call synchronises the handle's
 * stream. */
int sim_read_state(sim_t s, double* xyz, double* vel, sim_contact* contacts, int32_t cap,
                   int32_t* n_contacts);

/* Enqueue a device-to-device copy of the positions, float32 structure-of-arrays
 * [3][n] in caller order, into d_xyz_soa (device memory owned by the caller, e.g. a
 * torch tensor) on hip_stream (null: the handle's stream). */
int sim_read_state_device(sim_t s, float* d_xyz_soa, void* hip_stream);

/* Checkpoint / resume on the device: sim_save_state copies the frame state (positions,
 * velocities, time, previous-frame contacts and impulses) into a device-side snapshot
 * owned by the handle; sim_restore_state copies it back.  Both are stream-ordered
 * device-to-device copies (no host synchronisation).  Restore before any save:
 * SIM_E_STATE. */
int sim_save_state(sim_t s);
int sim_restore_state(sim_t s);

/* Release everything owned by the handle (null is accepted). */
int sim_destroy(sim_t s);

/* Thread-local message of the last failing call ("" if none). */
const char* sim_last_error(void);

/* ---- batching (many independent scenes in one set of launches) -------------------
 * Build a batch solver from several scene descriptions.  Scenes are concatenated:
 * the block-diagonal system has one elimination forest, so every kernel of
 * Algorithm 4 runs once per stage for all scenes, and the Conjugate Residual solves
 * run per scene inside one persistent launch.  All scenes share h and options.
 * obstacles[i] / n_obstacles[i] describe scene i.  count must lie in [1, 256] (the
 * constraint solver keeps per-scene slots in fixed on-chip tables): SIM_E_ARG otherwise,
 * before any device work. */
int sim_create_batch(int32_t count, const sim_mesh* meshes, const sim_material* mats,
                     const int32_t* n_obstacles, const sim_obstacle* const* obstacles, double h,
                     const sim_options* opt, sim_t* out);
/* Scene count and per-scene node offsets ([count+1]) of a handle. */
int sim_batch_info(sim_t s, int32_t* count, int32_t* node_offsets);

/* ---- parity hooks (tests) --------------------------------------------------------
 * Set a complete iterate state: frame start q_t, v_t [n][3], current iterate q_k
 * [n][3] (caller order; NULL: q^0 = q~, the predicted state of Algorithm 4),
 * simulation time t (frame start), and a contact list of c
 * entries (node, obstacle, lambda in the frame of that contact; frame rows and gap
 * are recomputed from q_t).  Recomputes the predicted state, frames, d_n, the
 * Delassus operator and the preconditioner exactly as a frame start does, but keeps
 * the given contact list and impulses. */
int sim_set_iterate_state(sim_t s, const double* q_t, const double* v_t, const double* q_k,
                          double t, int32_t c, const sim_contact* contacts);
/* Run k L-G iterations from the current iterate state without ending the frame. */
int sim_run_iterations(sim_t s, int32_t k);
/* The objective the L-G iteration minimises, at the current iterate q and the frame's
 * q~ and pin targets, with the local variables at their optimum (Eq. PD local and PD
 * global; Sec. 7's relative error is measured on it):
 *   1/2 (q - q~)^T M (q - q~) + h^2 sum_t [w_t/2 |F_t - p_t|^2 + V_t psi(p_t)]
 *   + 1/2 sum_pins h^2 w_pin |q_v - target|^2,
 * p_t the prox of F_t (ARAP: the rotation of F_t).  Float32 positions and per-tet terms,
 * float64 sums in a fixed order.  Contact terms are not included. */
int sim_lg_energy(sim_t s, double* energy);
/* Read the current iterate q_k [n][3] (caller order) and the impulses [c][3] of the
 * contact list, in canonical (node, obstacle) order. */
int sim_read_iterate(sim_t s, double* q_k, double* lambda);
/* u = S^T S b on the device (the global step, Algorithm 2): b, u [n][3] caller order. */
int sim_global_solve(sim_t s, const double* b, double* u);
/* Delta-form right-hand side of the current iterate: b - A q~ [n][3] (caller order),
 * i.e. h^2 sum_t w_t G_t^T (p_t - G_t q~) + pin terms (Eq. PD local / PD global). */
int sim_debug_rhs(sim_t s, double* rhs);
/* Delassus block K = B^T A_n^-1 B of the current contact list ([c][c], canonical
 * order), from which W_(j,k) = K_jk C_j C_k^T (Sec. 5.3). */
int sim_debug_delassus(sim_t s, double* K);

/* ---- learned warm start (not part of the paper: the paper leaves the initial impulse
 * of a frame open; the plain start re-uses the previous frame's impulse per contact
 * key).  A network 12 -> 128 -> 128 -> 3 (GELU; inputs padded to 16) predicts the
 * frame's converged impulse from per-contact features, all computed on the device at
 * the frame start, with l the mean rest edge length of the scene:
 *   f0 (n . x~ - d_n) / l     normal gap at the predicted position (App. A frame)
 *   f1..3 n                   contact normal, world frame
 *   f4..6 h C (v_t - u) / l   velocity relative to the obstacle, contact frame
 *   f7..9 h^2 K_jj lambda_prev / l   previous-frame impulse, contact frame
 *   f10 log K_jj              Delassus diagonal (r_n = h^2 K_jj, Sec. 5.4)
 *   f11 mu, f12..15 0
 * and its output y gives lambda = y l / (h^2 K_jj), projected onto the friction cone;
 * a contact whose prediction is not finite keeps the previous-frame impulse.  The
 * prediction is a candidate: a judge (sim_read_warm_judge) keeps the previous-frame
 * start of a scene wherever the prediction does not lower the NCP residual.
 * SIM_WARM_MLP predicts every contact; SIM_WARM_MLP_PERSIST only contacts with a
 * non-zero previous-frame impulse (new or released contacts start at zero, as with
 * the previous-frame start).
 * Parameters: float32, SIM_MLP_N_PARAMS values in the order W1 [128][16], b1 [128],
 * W2 [128][128], b2 [128], W3 [16][128] (rows 3..15 unused), b3 [16]; the device uses
 * bf16 copies of the weights and bf16 activations with float32 accumulation. */
#define SIM_MLP_N_PARAMS 20752
#define SIM_MLP_N_FEATURES 16
#define SIM_MLP_MAX_BATCH 16384

/* Upload the network used by SIM_WARM_MLP frames (copied; n_params must equal
 * SIM_MLP_N_PARAMS, else SIM_E_ARG).  Stepping in SIM_WARM_MLP mode without a model is
 * SIM_E_STATE. */
int sim_set_warm_model(sim_t s, const float* params, int32_t n_params);
/* Switch the warm start between frames (SIM_WARM_*). */
int sim_set_warm_mode(sim_t s, int32_t warm);
/* on != 0: compute the contact features at every frame start (needed by
 * sim_read_training_pairs in modes other than SIM_WARM_MLP). */
int sim_record_training_pairs(sim_t s, int32_t on);
/* Features [c][16] of the last frame's contacts, taken at that frame's start, and their
 * scaled impulses at its end, h^2 K_jj lambda / l [c][3] (contact frame), into host
 * buffers of cap rows, in the canonical contact order of sim_read_state (node and
 * obstacle keys as there; both nullable); *n = c.  SIM_E_CAPACITY when c > cap
 * (nothing copied), SIM_E_STATE when features are not recorded. */
int sim_read_training_pairs(sim_t s, int32_t* node, int32_t* obstacle, float* feat, float* target, int32_t cap,
                            int32_t* n);

/* Judge of the learned start (not part of the paper, which leaves the start impulse
 * open): each frame start with a learned warm start has two candidates, the
 * previous-frame impulse and the network's.  Each is scored by the NCP residual (the
 * metres measure of sim_step) that it leaves in the frame start's linear contact
 * problem, positions x_v = q~_v + h^2 sum_k K_jk C_k^T lambda_k (the predicted state
 * moved by the impulses through A^-1, Sec. 5.3), velocities (x - q_t) / h; per scene
 * the network's candidate is used only if its score is strictly lower.  Read the last
 * frame's scores: res [2][count] float32 (res[s]: previous-frame start of scene s,
 * res[count + s]: the network's), and, if cap > 0, the network's candidate impulses
 * [c][3] (contact frame, canonical contact order) into lam_learned; *n = c.
 * SIM_E_STATE when the warm start is not learned, SIM_E_CAPACITY when c > cap. */
int sim_read_warm_judge(sim_t s, float* res, float* lam_learned, int32_t cap, int32_t* n);

/* ---- trainer of the warm-start network ------------------------------------------
 * Device-resident float32 parameters with Adam moments (beta1 0.9, beta2 0.999, eps
 * 1e-8, bias-corrected; Kingma and Ba 2015).  Batches are device pointers: d_x [n][16]
 * float32 features (16-byte aligned, else SIM_E_ARG), d_t [n][3] float32 targets, loss = mean over n x 3 of (y - t)^2;
 * a training or gradient batch holds at most SIM_MLP_MAX_BATCH samples.
 * Work is enqueued on hip_stream (null: the default stream).  The gradient is a sum of
 * per-block partial sums added in block order, so results are deterministic. */
typedef struct lg_mlp* mlp_t;
int mlp_create(const float* params, int32_t n_params, mlp_t* out);
/* Replace the parameters (host, SIM_MLP_N_PARAMS) and reset the Adam state. */
int mlp_set_params(mlp_t m, const float* params, int32_t n_params);
/* Copy the parameters to a host buffer (waits for the device). */
int mlp_get_params(mlp_t m, float* params, int32_t n_params);
/* d_y [n][3] = network(d_x) (device pointers). */
int mlp_forward(mlp_t m, const float* d_x, float* d_y, int32_t n, void* hip_stream);
/* One Adam step with learning rate lr on the batch; if loss is not null the batch loss
 * before the step is copied to *loss (waits for the stream). */
int mlp_train_step(mlp_t m, const float* d_x, const float* d_t, int32_t n, float lr, void* hip_stream,
                   float* loss);
/* Gradient [SIM_MLP_N_PARAMS] (host) and loss of the batch, parameters unchanged. */
int mlp_gradient(mlp_t m, const float* d_x, const float* d_t, int32_t n, void* hip_stream, float* grad,
                 float* loss);
int mlp_destroy(mlp_t m);

/* ---- no-allocation gradient --------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * training loops, harnesses that forbid hipMalloc.  The gradient and loss of
 * mlp_gradient, without a trainer handle: its per-block partial sums go to a fixed
 * scratch array inside the library, (SIM_MLP_NOALLOC_MAX_BATCH / 64) x
 * (SIM_MLP_N_PARAMS + 1) floats = 5.3 MB on each GPU it runs on, held until the
 * process ends.
 *   d_params  [SIM_MLP_N_PARAMS] float32 parameters (layout of sim_set_warm_model),
 *             16-byte aligned
 *   d_x [n][16] features (16-byte aligned), d_t [n][3] targets (float32, as mlp_gradient)
 *   d_out     [SIM_MLP_N_PARAMS + 1] float32: the gradient, then the loss
 * All pointers are device memory of the current device (any allocator), borrowed for
 * the work enqueued on hip_stream (null: the default stream); the call does not wait.
 * 1 <= n <= SIM_MLP_NOALLOC_MAX_BATCH and the alignments hold, else SIM_E_ARG before
 * any device work; a failed
 * lookup of the scratch array is SIM_E_DEVICE.  No allocating routine is called (the
 * first call on a device looks the array's address up once).  Every call on one GPU
 * uses that GPU's one scratch array, so calls that overlap in time on one GPU (other
 * streams, other threads) race and give wrong results; calls on one stream are safe. */
#define SIM_MLP_NOALLOC_MAX_BATCH 4096
int mlp_gradient_noalloc(const float* d_params, const float* d_x, const float* d_t, int32_t n, float* d_out,
                         void* hip_stream);

/* ---- host-only precompute inspection (no device needed) -------------------------
 * Run only the host precomputation of sim_create and keep its products. */
typedef struct lg_host* lg_host_t;
int lg_host_create(const sim_mesh* mesh, const sim_material* mat, double h, double pin_weight_scale,
                   int32_t want_dense_S, lg_host_t* out);
/* info[0..7] = n, m, nnz(S), nnz(L), stored row floats, max depth, chains, 0. */
int lg_host_info(lg_host_t hs, int64_t* info);
/* perm[orig] = internal index; parent [n] etree in internal order (-1 for roots). */
int lg_host_ordering(lg_host_t hs, int32_t* perm, int32_t* parent);
/* Node-level A_n [n][n] dense, internal order (small meshes). */
int lg_host_dense_A(lg_host_t hs, double* A);
/* S = L^-1 [n][n] dense, internal order: float64 values if requested at creation. */
int lg_host_dense_S(lg_host_t hs, double* S);
/* S^T S b for b [n][3] internal order, using the float32 row and column storages on
 * the host (checks both layouts). */
int lg_host_apply_StS(lg_host_t hs, const double* b, double* u);
int lg_host_destroy(lg_host_t hs);

#ifdef __cplusplus
}
#endif

#endif /* LGSIM_H */
