/*
 * mabd.h -- C ABI of libmabd, an MI355X (gfx950) implementation of the
 * per-time-step solve of M-ABD: co-rotated affine bodies joined by ball,
 * hinge, universal and prismatic joints, one implicit-Euler Newton step per
 * call (or several) with the joints enforced exactly through the KKT system
 * (arXiv 2603.08079, Secs. 3-5).
 *
 * One step does, on the GPU:
 *   (a) per body: polar rotation R = A (A^T A)^{-1/2} (Eq. polar), force
 *       f_A (Eq. variation_energy, Eq. reduced_K) and the unconstrained local
 *       solve with the constant pre-factorised Hbar (Eq. abd_final), or for
 *       bodies without joints optionally the polar-free solve of Alg. 1;
 *   (b) the dual (Schur) system  grad C H^{-1} grad C^T  with right-hand side
 *       grad C H^{-1} f_A + C  (Eq. dual; -C as in the footnote of Eq. kkt);
 *   (c) its solution: block cyclic reduction on ball chains (Eq. chain-btd),
 *       a rake/compress elimination on trees and hinge chains (Sec. 5.3), a
 *       spanning tree plus a dense Schur system over the loop-closing joints
 *       for components with a few loops (Sec. 5, Case III, Eq. loop), and
 *       preconditioned CG on networks (Secs. 5.4-5.5);
 *   (d) the primal back-projection dq = H^{-1}(f_A - grad C^T dlambda)
 *       (Eq. primal) and the state update q += dq, qdot = dq / h.
 *
 * Conventions
 *   - Every pointer in a struct passed to mabd_create is a HOST pointer; the
 *     data are copied during the call, the caller keeps ownership.
 *   - The context owns all device memory; results go to caller buffers.
 *   - Every call returns a status; mabd_last_error() gives a message.  Nothing
 *     aborts or throws across the ABI.
 *   - A context is not thread-safe; several contexts may coexist.  Work is
 *     issued on the stream given in mabd_options.stream (a hipStream_t), or on
 *     a stream of the library's own when that is NULL.  mabd_step returns as
 *     soon as its steps are queued (unless the assembly has a network
 *     component, whose solve runs under host control, or kernel timing is
 *     on); the outcome of queued steps is read by the next call that waits
 *     for the stream: mabd_state, mabd_multipliers, mabd_residual, mabd_stats,
 *     mabd_set_state, mabd_set_wrenches, the learned-start calls, or a later
 *     mabd_step once that outcome has arrived.
 *   - Units are SI.  q per body = [a1; a2; a3; t] (12 doubles), a_c the c-th
 *     column of the affine matrix A, t the translation (Sec. 3.1, Eq. abd_dof);
 *     qdot has the same layout.
 */
#ifndef MABD_H
#define MABD_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mabd_ctx mabd_ctx;

typedef enum {
  MABD_OK = 0,
  MABD_ERR_INVALID_ARG = -1,  /* bad index, size, non-finite input, bad option   */
  MABD_ERR_TOPOLOGY = -2,     /* joint graph the library cannot solve            */
  MABD_ERR_DEVICE = -3,       /* HIP runtime error, or a kernel's internal size check   */
  MABD_ERR_OOM = -4,          /* device allocation failed                        */
  MABD_ERR_NONFINITE = -5,    /* non-finite state or det A <= 0 during a step    */
  MABD_ERR_NOT_CONVERGED = -6,/* PCG reached max_iters, or precision-1 refinement ran
                                 out of sweeps, above kkt_tol                        */
  MABD_ERR_SINGULAR = -7      /* a dual pivot block was not positive definite    */
} mabd_status;

/* n bodies, all boxes with the rest frame at the centre of mass and axes along
   the box edges (so the generalised mass J^T M J is diagonal, Eq. newton_abd). */
typedef struct {
  int32_t n;
  const double *dims;      /* n*3  box edge lengths, > 0                                  */
  const double *density;   /* n    kg/m^3, > 0                                            */
  const double *k_orth;    /* n    k_A of Eq. EA (material 0) or Young's modulus (1)      */
  const double *poisson;   /* n    Poisson ratio (material 1 only; may be NULL otherwise) */
  const uint8_t *pinned;   /* n    1 = kinematic body held at q0 (may be NULL: none)      */
  const double *q0, *qd0;  /* n*12 initial state (qd0 may be NULL: zero)                  */
} mabd_bodies;

/* m joints.  type 0: ball joint, 3 rows (Eq. ball): the points P1 of both
   bodies coincide.  The other types are rows of a rotated frame owned by body
   a, R_J = dR R_a^T (R_a the polar rotation of a, dR the joint's frame at
   rest), each row one local component of R_J (y_X - y_Y) for control points
   X, Y (Secs. 4.3-4.5; gradient with the A-linearised rotation term of Eq.
   r_gradient):
     type 1, hinge, 5 rows (Eq. hinge): dR = Rod(axis) (rows r_x, axis, r_z);
       P2 = P1 + cp_len * axis on both bodies; rows x, y, z of P1a - P1b and
       x, z of P2a - P2b;
     type 2, universal, 4 rows (Eq. universal): dR rows (a1 x a2, a1, a2) for
       axis = a1 and axis2 = a2 (orthogonal); b's P2 = P1 + cp_len * a2; rows
       x, y, z of P1a - P1b and y of P2b - P1b (b's second axis stays normal
       to a's first);
     type 3, prismatic, 5 rows (Eq. prismatic): dR = Rod(axis); b's P2 = P1 +
       cp_len * axis and P3 = P1 + cp_len * n, n the frame's local z at rest;
       rows x, z of P1a - P1b, x, z of P2b - P1b and x of P3b - P1b (b slides
       along the axis and may not turn).
   Directions given in a's rest frame enter b's as the same world direction
   at creation.  The paper's six-row linear hinge (an edge-edge constraint)
   is two ball joints at the two points of its axis. */
typedef struct {
  int32_t m;
  const uint8_t *type;     /* m    0 ball, 1 hinge, 2 universal, 3 prismatic             */
  const int32_t *a, *b;    /* m    body indices, -1 = world; a != b; one side dynamic      */
  const double *pa, *pb;   /* m*3  P1 in the rest frame of a / b (world coords if -1)     */
  const double *axis;      /* m*3  hinge / prismatic axis, universal a1, in a's rest frame
                                   (world if a = -1); may be NULL if all joints are balls */
  const double *cp_len;    /* m    spacing of the further control points (> 0 except for
                                   ball joints; may be NULL if all joints are balls)      */
  const double *axis2;     /* m*3  universal a2, orthogonal to axis (a's rest frame);
                                   may be NULL if there is no universal joint            */
} mabd_joints;

typedef struct {
  double gravity[3];       /* m/s^2, default (0, 0, -9.8)                                 */
  int32_t precision;       /* 0 FP64 throughout; 1 on chain components: FP32 body solve and
                              dual assembly, FP64 dual factor, then FP64 KKT residual
                              checks and correction sweeps until max(rho_p, rho_d) <=
                              kkt_tol; a sweep that no longer halves it has reached the
                              FP64 rounding floor and ends the step, accepted
                              (stats.ir_stalled = 1) if the residual is within 10
                              kkt_tol, or if rho_p is and |G dq + C| is within 64
                              units of rounding of the size of the summands it is
                              formed from (where the dual right-hand side all but
                              vanishes, as for a freely falling chain, rho_d is O(1)
                              for any FP64 solution);
                              NOT_CONVERGED otherwise.  Tree components (contexts with
                              newton_iters = 1 and no loop or network component): the
                              force and local solve (the polar rotation stays FP64)
                              and the clique matrices L Hbar^{-1} L^T in FP32, the
                              contraction in FP64, then the FP64 residual of the tree
                              bodies and joints and correction sweeps (the tree solve
                              with Hbar^{-1} R^T r_p and r_d as right-hand sides)
                              under the same rules except the rounding test, checked
                              on the host: such steps wait.  Loops and networks stay
                              FP64                                                      */
  double kkt_tol;          /* PCG stop: |r - S lam| <= kkt_tol |r|; precision-1 target of
                              the chain KKT residual; default 1e-10                      */
  int32_t max_iters;       /* PCG iteration cap, default 200000                           */
  int32_t warm_start;      /* PCG start: 0 zero, 1 previous step's multipliers, 2 learned
                              (ball networks with weights; otherwise zero)              */
  int32_t newton_iters;    /* Newton iterations per step, default 1                       */
  int32_t hinge_grad;      /* 0 frozen frame + A-linearised rotation term, 2 frozen only  */
  int32_t material;        /* 0: mu = 4 k_A, lambda = 0 (Eq. EA linearised); 1: Lame     */
  int32_t diagnostics;     /* bit 0: evaluate on the device, after every step, the FP64
                              KKT residual of the step (every Newton iteration's when
                              newton_iters > 1) and the joint values at the new state
                              (stats rho_p, rho_d, kkt, c_ball, c_hinge, kkt_newton);
                              bit 1: time every kernel group with HIP events (phase_ms)  */
  int32_t use_graph;       /* 1 (default): replay each step as a captured hipGraph when
                              the assembly has no PCG component and bit 1 is off        */
  int32_t autotune;        /* 1 (default): at the first step of a context with at least
                              20,000 chain rows, time the chain tile forms (packed
                              60-row tiles; 64, 128, 256 threads) and keep the fastest;
                              with at least 20,000 tree-contraction slots and no
                              network component, also the tree schedules (threshold
                              above which a round's 16-row cliques launch apart: 1,500,
                              6,000 or never; clique classes largest or smallest first
                              in a launch); schedules change no result.  Without it
                              packed tiles, 6,000 and largest first.  The environment
                              variable MABD_CHAIN_TILE_THREADS = 64p, 64, 128 or 256
                              fixes the form at mabd_create instead, and
                              MABD_CHAIN_TOP_GLOBAL=1 sends every chain's top system
                              through the global-memory reduction that chains beyond
                              ~3.9M rows need (both for testing)                         */
  int32_t ir_max_sweeps;   /* precision 1: correction sweeps before NOT_CONVERGED, 0..16,
                              default 4                                                 */
  int32_t body_solve;      /* 0 (default): every body rotates its forces and increment by
                              its polar rotation R (Eqs. polar, abd_final); 1: bodies
                              without joints take the polar-free solve of Alg. 1 instead:
                              R^T x and R y replaced block by block by A^T x and A y
                              scaled to the lengths of x and y (Eq. len_preserving),
                              also in the rotated elastic force.  Exact where A is a
                              scaled rotation, first order in the deformation otherwise;
                              such bodies are left out of rho_p (diagnostics)          */
  int32_t path_solver;     /* 1 (default): tree components whose bodies carry at most two
                              joints each (paths: chains with hinge, universal or
                              prismatic joints, free-floating chains) are solved as
                              block-tridiagonal systems over their joints: segments of
                              up to 16 joints, each eliminated by a team of 16 lanes
                              that forms the joints' blocks from the joint rows, then
                              level by level over the segments' last joints (segments
                              of 4, one lane each); the solve runs on a second stream
                              beside the tree contraction when both are large.  0: by
                              the tree contraction like every other tree.  Both are exact
                              (Sec. 5.3) and agree to rounding.  The environment
                              variable MABD_PATH_SEGMENT = T or T0,T1 sets the segment
                              length (T0 = 2..16 at the first level, T1 = 2..64 above)
                              and MABD_PATH_FORK = n the number of forward contraction
                              rounds left when the second stream forks (default 3), at
                              mabd_create (for testing)                                */
  const char *tune_cache;  /* path of a tuning cache file, or NULL (default): with
                              autotune on, a context whose device and schedule shape
                              (chain rows and count, tree slots and rounds) have an
                              entry takes that entry's choices at mabd_create instead
                              of timing them; a context that times them appends its
                              entry.  Text, one "key = values" line per entry; an
                              unreadable file counts as empty, a failed append is
                              ignored (the choices still apply).  Copied at create.  */
  void *stream;            /* hipStream_t, or NULL for a library-owned stream             */
} mabd_options;

#define MABD_NPHASES 10
#define MABD_NEWTON_DIAG 8  /* Newton iterations whose KKT residual the stats keep */

typedef struct {
  int64_t steps_done;      /* steps completed since create                               */
  int32_t last_status;     /* status of the last mabd_step                               */
  int32_t pcg_iters;       /* PCG iterations of the last step (max over components)      */
  /* FP64 KKT residual of the last step (Eq. kkt with the -C right-hand side):
     r_p = f_A - H dq - G^T lambda, r_d = G dq + C.  With diagnostics bit 0 all
     five values come from the device evaluation; otherwise rho_d is the PCG's
     true residual (network components), rho_p, rho_d and kkt the form-1
     refinement's (chains, precision 1), and -1 / 0 where nothing evaluated them */
  double rho_p, rho_d;     /* |H^-1 r_p|/|H^-1 f_A|, |r_d|/|G H^-1 f_A + C|                */
  double kkt;              /* max(rho_p, rho_d)                                           */
  double c_ball, c_hinge;  /* max |C| at the new state of the ball joints and of the other
                              (rotated-frame) joints (diagnostics bit 0)                 */
  int32_t ir_sweeps;       /* refinement sweeps of the last step (precision 1)           */
  int32_t warm_accepted;   /* 1 if the GNN warm start was kept                            */
  int32_t n_chain, n_tree, n_graph;  /* components per solver class                     */
  int32_t n_dyn;           /* dynamic bodies                                              */
  /* With diagnostics bit 1: GPU time of each kernel group summed over the last
     mabd_step call, and its launch count.  Groups: 0 chain tile reduce, 1 chain
     interface solve, 2 chain tile apply, 3 generic bodies, 4 generic joints,
     5 tree elimination, 6 generic back-projection, 7 PCG, 8 chain FP64 KKT
     residual check (precision 1), 9 chain state update (precision 1). */
  double phase_ms[MABD_NPHASES];
  int64_t phase_calls[MABD_NPHASES];
  int32_t tile_threads;    /* workgroup size of the chain tile kernels in use            */
  int32_t graph_replay;    /* 1 if the last mabd_step replayed captured step graphs       */
  int32_t tree_rounds;     /* rounds of the tree contraction (rake + compress)          */
  int32_t tile_packed;     /* 1 if the chain tiles are packed: 60-row tiles whose last
                              four cyclic-reduction levels run four tiles to a wave     */
  int32_t ir_stalled;      /* precision 1: the refinement of the last step ended at the
                              rounding floor (see precision) instead of below kkt_tol    */
  double kkt_newton[MABD_NEWTON_DIAG]; /* diagnostics bit 0: KKT residual of each Newton
                              iteration of the last step (a ninth and later iterations
                              share the last entry), -1 where not evaluated             */
  int32_t n_loop;          /* components with a few closed loops, solved by the loop-
                              breaker Schur complement (Sec. 5, Case III): a spanning
                              tree by the tree contraction, the loop-closing joints (at
                              most 48 rows per component) by a dense Schur system;
                              components with more loop rows are networks (PCG)       */
  int32_t tree_split;      /* tree schedule in use: 16-row classes launch apart above
                              this many operations per round (INT32_MAX: never)      */
  int32_t tree_order;      /* 0 clique classes largest first in a launch, 1 smallest   */
  int32_t tune_source;     /* 0 default schedules, 1 timed by the autotuner, 2 read from
                              the tuning cache                                        */
  int32_t n_path;          /* tree components solved as paths (path_solver; counted in
                              n_tree too)                                             */
  int32_t path_levels;     /* levels of the path solve (0: none)                      */
} mabd_step_stats;

/* Fills *opt with the defaults listed above. */
void mabd_options_default(mabd_options *opt);

/* Validates and copies the assembly, classifies every connected component of
   dynamic bodies (chain: the dual graph of Fig. dual_mat is a path with only
   ball joints; tree: body/joint incidence graph acyclic, a path when every
   body carries at most two joints (path_solver); loop: a spanning tree plus
   loop-closing joints of at most 48 rows (Case III); graph: otherwise),
   builds the solve schedules and uploads state and schedules to the device.
   Pinned bodies become constant world-side anchors.  opt may be NULL
   (defaults).  On success *out receives a context to free with mabd_destroy.
   Errors: INVALID_ARG (bad sizes, indices, non-finite or non-positive inputs,
   zero hinge axis), TOPOLOGY, DEVICE, OOM. */
mabd_status mabd_create(const mabd_bodies *bodies, const mabd_joints *joints,
                        const mabd_options *opt, mabd_ctx **out);

/* Advances n >= 1 steps of size h > 0 (implicit Euler, Eq. variation_energy;
   newton_iters Newton iterations per step, Eq. kkt).  If h differs from the
   previous call the per-shape factors Hbar^{-1} are rebuilt first (Eq.
   abd_final).  Asynchronous on the context's stream: it returns once the
   steps are queued, except for assemblies with a network component (PCG under
   host control), precision-1 tree components (refinement under host control)
   and kernel timing (diagnostics bit 1), which wait.  A step
   that fails (NONFINITE, NOT_CONVERGED, SINGULAR) makes the later queued
   steps do nothing and leaves the state at the last completed step; the
   failure is returned by the next call that reads the outcome (mabd_state,
   mabd_multipliers, mabd_residual, a learned-start call, or mabd_step itself
   once the outcome has arrived) and recorded in mabd_stats' last_status,
   also where mabd_set_state or mabd_set_wrenches read it.  The state
   written by mabd_state_device is the last completed step's in every case. */
mabd_status mabd_step(mabd_ctx *ctx, double h, int32_t n);

/* Copies the state to host buffers q, qd (n*12 doubles each, input body
   order; either may be NULL).  Synchronises the stream and returns the
   failure of a queued step, if one failed (the state copied is then the last
   completed step's). */
mabd_status mabd_state(const mabd_ctx *ctx, double *q, double *qd);

/* Writes the state into device buffers (n*12 doubles each, input body order)
   on the context's stream, without synchronising. */
mabd_status mabd_state_device(const mabd_ctx *ctx, void *q_dev, void *qd_dev);

/* Replaces the state (host buffers, n*12 doubles each, input order).  Pinned
   bodies keep q0.  Bitwise continuation: set_state(state()) changes nothing.
   Waits for queued steps first; the multipliers stop being a warm start. */
mabd_status mabd_set_state(mabd_ctx *ctx, const double *q, const double *qd);

/* External spatial wrenches W = [tau; f] per body (host, n*6 doubles in input
   body order: torque then force, world frame, about the body's centre of
   mass), applied at every following step until replaced; w = NULL removes
   them.  Each enters the body force as f_A,ext = G(A)^T W (Eqs.
   module1-G-twist, module1-wrench-map): 1/2 tau x a_c on column c of A and f
   on the translation, evaluated at the current Newton iterate.  Entries of
   pinned bodies are ignored.  Synchronises the stream.  Errors: INVALID_ARG
   (NULL ctx, non-finite entries), OOM, DEVICE. */
mabd_status mabd_set_wrenches(mabd_ctx *ctx, const double *w);

/* Multipliers dlambda of the last step's dual solve (Eq. dual) in input joint
   order, 3 doubles per ball joint and 5 per hinge, concatenated.  lam must hold
   mabd_rows(ctx) doubles.  Synchronises the stream; returns the failure of a
   queued step, if one failed. */
mabd_status mabd_multipliers(const mabd_ctx *ctx, double *lam);
int64_t mabd_rows(const mabd_ctx *ctx);

/* FP64 KKT residual of the last completed step, evaluated on the device
   from the state it started from, its increment dq = h qdot_new and its
   multipliers (Eq. kkt with the -C of its footnote):
     out[0] rho_p = |H^-1 (f_A - H dq - G^T lambda)| / |H^-1 f_A|,
     out[1] rho_d = |G dq + C| / |G H^-1 f_A + C|,
     out[2] max(rho_p, rho_d),
     out[3], out[4] largest |C| of the ball joints / hinges at the new state
   (out: 5 host doubles).  Partial sums go to a buffer of the library's,
   allocated at the first call (diag_blocks x 6 doubles, diag_blocks = chain
   tiles + ceil(generic bodies / 256) + ceil(generic joints / 256)) and kept
   until mabd_destroy.  Synchronises the stream.  Errors: the failure of a
   queued step; INVALID_ARG if no step completed since create, mabd_set_state,
   mabd_set_wrenches or a learned-start call, or if newton_iters > 1
   (diagnostics bit 0 evaluates every iteration instead); OOM; DEVICE. */
mabd_status mabd_residual(mabd_ctx *ctx, double *out);

/* mabd_residual for callers that cannot allocate device memory or wait for
   the stream: code under HIP graph capture, serving loops that forbid
   allocation.  The five values (as mabd_residual's out) are written to
   out_dev, a DEVICE buffer of 5 doubles, by kernels queued on the context's
   stream; the call returns without waiting.  The partial sums go to a fixed
   device array of the library's instead of a buffer allocated at the first
   call: 65,536 records of 6 doubles (3 MiB), one copy on every device the
   library runs on, held until the process ends; nothing is allocated.  Every
   call on one device shares that array and its records are rewritten by
   each call: calls that overlap on one device (other host threads, or
   streams not ordered with this context's) race.  Errors (host-side, nothing
   queued): INVALID_ARG if the assembly needs more than 65,536 records (chain
   tiles of 60 rows + ceil(generic bodies / 256) + ceil(generic joints /
   256)), if no step completed since create, mabd_set_state, mabd_set_wrenches
   or a learned-start call, or if newton_iters > 1; DEVICE.  If a queued step
   fails, out_dev is not meaningful (it may be left unchanged); the failure is
   reported by the next call that reads the outcome. */
mabd_status mabd_residual_noalloc(mabd_ctx *ctx, double *out_dev);

/* Spatial twist of every body at the current state (Eq. module1-G-twist):
   V = G(A) qdot = [omega; v], omega = 1/2 sum_c a_c x adot_c (a_c the c-th
   column of A), v = tdot; world frame.  V: host, n*6 doubles in input body
   order, zero for pinned bodies.  Synchronises the stream; returns the
   failure of a queued step, if one failed. */
mabd_status mabd_twists(const mabd_ctx *ctx, double *V);

/* Joint wrench on every body from the last step: the spatial wrench W =
   [tau; f] (world frame, about the centre of mass) that does the same
   virtual work on rigid motions as the body's generalised joint force
   -sum_k G_kb^T dlambda_k (the primal rows of Eq. kkt), W = E(A)^T (-G^T
   dlambda) with the rigid-motion embedding E(A) of Eq. module2-E, taken at
   the state the step started from (single-body comparison of Sec. 6: the
   spatial wrench of a generalised force).  For a ball joint this is the
   point force at the anchor and its moment.  W: host, n*6 doubles in input
   body order, zero for pinned bodies.  Synchronises the stream.  Errors: the
   failure of a queued step; INVALID_ARG if no step completed since create,
   mabd_set_state, mabd_set_wrenches or a learned-start call, or if
   newton_iters > 1. */
mabd_status mabd_joint_wrenches(const mabd_ctx *ctx, double *W);

/* Diagnostics of the last step.  Synchronises the stream; the outcome of
   queued steps goes to st->last_status (the call itself returns MABD_OK). */
mabd_status mabd_stats(const mabd_ctx *ctx, mabd_step_stats *st);

/* ---------------------------------------------------------------------------
   Learned warm start of the ball-network PCG (warm_start = 2).  Not part of
   the paper's method: it only supplies the PCG start value.  A
   message-passing network over the joints (3 layers of width 64, FP32,
   mabd_gnn_size() parameters) predicts a correction of the base start (the
   previous step's multipliers, or zero on a first step) from per-joint
   features (block-Jacobi step of the base residual, base multipliers,
   degrees, world sides).  The solve keeps the corrected start only if it
   lowers the dual energy 1/2 l^T S l - b^T l below the base start's (then its
   S-norm error is smaller; stats.warm_accepted says which start was used).
   Training minimises that energy decrease, normalised by the energy of a
   block-Jacobi step, over the dual systems of the states the caller steps
   through; everything runs on the context's stream.  All calls need a
   ball-joint network component (INVALID_ARG otherwise) and, except init and
   set, weights (INVALID_ARG otherwise).
   --------------------------------------------------------------------------- */

/* Number of network parameters (float32). */
int32_t mabd_gnn_size(void);

/* Allocates the network's device buffers (about 1.6 KB per joint) and draws
   Glorot-uniform weights from `seed`; resets the Adam state. */
mabd_status mabd_gnn_init(mabd_ctx *ctx, uint64_t seed);

/* Copies the weights to `get` and/or replaces them from `set` (both host,
   n = mabd_gnn_size() floats, either may be NULL; `set` resets Adam). */
mabd_status mabd_gnn_params(mabd_ctx *ctx, float *get, const float *set, int32_t n);

/* Gradient (host, mabd_gnn_size() floats; may be NULL) and loss of the dual
   system of the current state for time step h; the state is unchanged. */
mabd_status mabd_gnn_grad(mabd_ctx *ctx, double h, float *grad, double *loss);

/* `iters` Adam steps (learning rate lr) on the dual system of the current
   state for time step h; the loss before the first and after the last step
   go to loss_first / loss_last (may be NULL).  The state is unchanged. */
mabd_status mabd_gnn_train(mabd_ctx *ctx, double h, int32_t iters, float lr, double *loss_first,
                           double *loss_last);

/* The network's start multipliers for the current state (host, 3 per joint
   in input order; joints outside ball networks get 0). */
mabd_status mabd_gnn_predict(mabd_ctx *ctx, double h, double *lam0);

/* Writes / reads the weights (8-byte tag, int32 count, float32 values).
   Errors: INVALID_ARG on an unreadable file or a wrong tag or count. */
mabd_status mabd_gnn_save(const mabd_ctx *ctx, const char *path);
mabd_status mabd_gnn_load(mabd_ctx *ctx, const char *path);

/* Message of the last error on ctx (or of the last failed create if ctx is
   NULL).  Valid until the next call on the same context. */
const char *mabd_last_error(const mabd_ctx *ctx);

/* Releases device memory and the owned stream.  NULL is allowed. */
void mabd_destroy(mabd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
