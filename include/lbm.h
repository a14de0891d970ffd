/*
 * lbm.h - C interface of the MI355X (gfx950) library for the coupled
 * lattice-Boltzmann / dynamic immersed-boundary step of Coclite, de Tullio,
 * Pascazio and Politi, "Characterization of micro-Capsules Deformation in
 * Branching Channels" (arXiv 2207.06043), Section "Numerical method and
 * computational procedure".
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice units: dx = dt = 1.  Node (x, y, z) sits at position (x, y, z) and
 * has the linear index n = x + nx*(y + ny*z) (x fastest); N = nx*ny*nz.
 * Per-node scalar fields are [N]; per-node vector fields are component-major
 * [3][N]; populations are [19][N] in the order of the D3Q19 velocity set
 * printed in the paper's fluid-evolution section (Eq. e_i).  Point lists
 * (markers, vertices) are [n][3].  All floating-point arguments are double.
 *
 * Ownership: every pointer in lbm_desc / lbm_body_desc is host memory that is
 * copied during the call.  Arguments named d_* are caller-owned device
 * pointers on the context's device; they must stay valid until the work the
 * call enqueued on the context's stream has completed.  The library never
 * frees or retains them.
 *
 * Errors: every call returns an lbm_status and never throws.
 * lbm_last_error() gives a message for the last failure on a context.  A HIP
 * runtime failure is sticky: the call returns LBM_E_HIP and every later call
 * on the context returns LBM_E_STATE.  LBM_E_UNSTABLE and LBM_E_DAMAGED are
 * reported by lbm_sync() (and the calls that synchronise) once the device
 * has seen them; the state is then left at the last completed step and
 * further steps do nothing.
 *
 * Threads: one context per host thread; no internal locking.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_INVAL = 1,       /* bad argument, size, geometry or mesh            */
  LBM_E_NOMEM = 2,       /* device or host allocation failed               */
  LBM_E_HIP = 3,         /* HIP runtime error (sticky)                      */
  LBM_E_UNSTABLE = 4,    /* |u| > 0.3 or NaN in the fluid or a body         */
  LBM_E_DAMAGED = 5,     /* a membrane link reached twice its rest length   */
  LBM_E_STATE = 6,       /* context unusable after an earlier HIP error     */
  LBM_E_UNSUPPORTED = 7  /* feature not available in this build            */
} lbm_status;

typedef enum {
  LBM_F64 = 0,  /* populations stored and collided in double                  */
  LBM_F32 = 1,  /* populations stored as float deviations f_i - w_i, float math */
  LBM_F16S = 2  /* populations stored as half deviations f_i - w_i, float math  */
} lbm_precision;

enum { LBM_NODE_FLUID = 0, LBM_NODE_SOLID = 1, LBM_NODE_INLET = 2, LBM_NODE_OUTLET = 3 };

/* The fluid problem (sections "Fluid evolution", "Dirichlet conditions for
 * external boundaries" and "No-slip boundary conditions for stationary
 * immersed boundaries").
 *  node_type [N]: LBM_NODE_*.  INLET nodes carry a velocity Dirichlet
 *    condition, OUTLET nodes a density Dirichlet condition (Zou-He); both
 *    must lie on exactly one non-periodic face of the box.  Every other
 *    non-solid node must have all its neighbours inside the box (or across
 *    a periodic face).
 *  Wall links (link_node[k], link_dir[k], link_q[k]): link_node + e_dir is a
 *    solid node and the wall crosses that link at fraction q in [0, 1]
 *    (Eq. qbouzidi).  Every solid neighbour of a non-solid node needs one.
 *  inlet_u [n_inlet][3]: wall velocity of the INLET nodes in increasing
 *    linear index order.  outlet_rho: density imposed on OUTLET nodes.
 *  init_rho [N], init_u [3][N]: initial fields (NULL: rho = 1, u = 0); the
 *    populations start at the equilibrium (Eq. eqfunc) of these fields.
 *  tau > 1/2: BGK relaxation time (nu = (tau - 1/2)/3).
 *  body_force [3]: uniform force density added to the immersed-boundary
 *    force on every non-solid node (Eq. forcing).
 *  u_max: characteristic flow velocity used by the inter-body repulsion
 *    (Eq. collision). */
typedef struct {
  int32_t nx, ny, nz;
  int32_t periodic[3];
  double tau;
  double u_max;
  double body_force[3];
  int32_t precision; /* lbm_precision */
  const uint8_t *node_type;
  int64_t n_links;
  const int64_t *link_node;
  const uint8_t *link_dir;
  const double *link_q;
  const double *inlet_u;
  double outlet_rho;
  const double *init_rho;
  const double *init_u;
} lbm_desc;

/* A capsule (section "Immersed-Structure Transport"): a closed triangle mesh
 * with counter-clockwise faces seen from outside.  Its face centroids are
 * the Lagrangian markers of the direct forcing.
 *  rigid: Newton-Euler motion of the whole body; fixed: held at rest.
 *  ca: capillary number Ca = rho nu u_ref / k_s0 (rho = 1) giving the
 *    membrane modulus; eb: bending number Eb = k_b / (k_s,l r_ref^2);
 *  kv: volume-penalty constant (<= 0: 10 k_s0 / r_ref);
 *  rho_ratio: solid-to-fluid density ratio (mass = rho_ratio * enclosed volume);
 *  v0 [nv][3]: initial vertex velocities (NULL: at rest). */
typedef struct {
  int32_t nv, nf;
  const double *x;
  const int32_t *faces;
  int32_t rigid, fixed;
  double ca, eb, kv, rho_ratio, r_ref, u_ref;
  const double *v0;
} lbm_body_desc;

/* Sizes and counters of a context. */
typedef struct {
  int64_t n_nodes, n_fluid, n_bulk, n_general, n_links;
  int64_t n_bodies, n_vertices, n_faces;
  int64_t steps_done;
  int64_t bytes_per_step_alg;   /* 2 * 19 * sizeof(stored population) * n_fluid */
  int32_t precision;
  int32_t mls_singular;         /* markers whose moment matrix was singular */
  int32_t fluid_launch;         /* 1: one fused fluid kernel per step (small grids);
                                   2: bulk and boundary-record kernels on two streams */
  int32_t pad;
} lbm_info_t;

/* Create a context on the current HIP device; work is enqueued on
 * hip_stream (a hipStream_t; NULL = the default stream).  Validates the
 * geometry (LBM_E_INVAL with a message on failure).  The kernels index
 * nodes with 32-bit integers: a grid whose padded node count with one guard
 * plane on each side, px ny (nz + 2) with px = nx rounded up to a multiple
 * of 8, reaches 2^31 is refused with LBM_E_INVAL ("grid too large"). */
lbm_status lbm_create(const lbm_desc *desc, void *hip_stream, lbm_ctx **out);
lbm_status lbm_destroy(lbm_ctx *ctx);
const char *lbm_last_error(const lbm_ctx *ctx);
lbm_status lbm_info(lbm_ctx *ctx, lbm_info_t *out);

/* Add a capsule (host data copied).  Rest lengths, areas, angles and volume
 * are taken from the given positions.  LBM_E_INVAL for an open or
 * inconsistently oriented mesh, or a vertex in more than 10 faces.  The
 * faces may be given in any order and each in any rotation of its
 * (counter-clockwise) vertices: the library keeps them in a canonical order
 * (turned to start at the smallest vertex id, sorted by vertex triple), and
 * its results do not depend on the order given.  The forcing markers
 * (Eq. bodyforce) are processed in blocks of 64 faces taken along the
 * Hilbert curve of their stencil bases, sorted on the device when the body
 * is added, after lbm_load and every 512 steps, so that a block's support
 * nodes form one compact box in on-chip memory. */
lbm_status lbm_add_body(lbm_ctx *ctx, const lbm_body_desc *body, int32_t *body_id);

/* Advance n_steps coupled steps (asynchronous on the context's stream):
 * streaming with interpolated bounce-back and Zou-He, dynamic-IB direct
 * forcing, forced BGK collision, membrane and hydrodynamic forces, body
 * motion.  The step is replayed from a captured HIP graph. */
lbm_status lbm_step(lbm_ctx *ctx, int32_t n_steps);

/* Wait for the context's stream and report LBM_E_UNSTABLE / LBM_E_DAMAGED
 * if the device raised them. */
lbm_status lbm_sync(lbm_ctx *ctx);

/* Macroscopic fields of the last completed step: d_rho [N], d_u [3][N]
 * (u = (sum f e + F/2)/rho with the step's total force F); solid nodes 0. */
lbm_status lbm_get_fields(lbm_ctx *ctx, double *d_rho, double *d_u);
/* Post-collision populations [19][N] (solid nodes 0). */
lbm_status lbm_get_populations(lbm_ctx *ctx, double *d_f);
/* The inverse: the current state's post-collision populations become d_f
 * ([19][N] FP64 device array, x fastest; entries at solid nodes ignored),
 * stored as f - w_i rounded to the context's storage (the state the next
 * lbm_step starts from, as Eq. evoleq's f* of the last step).  The step
 * count, the force field and the bodies are not changed.  Asynchronous on
 * the context's stream (d_f must stay valid until it completes). */
lbm_status lbm_set_populations(lbm_ctx *ctx, const double *d_f);
/* Immersed-boundary force density [3][N] of the last completed step. */
lbm_status lbm_get_force(lbm_ctx *ctx, double *d_fib);
/* Vertex positions and velocities [nv][3] of a body. */
lbm_status lbm_get_body(lbm_ctx *ctx, int32_t body_id, double *d_x, double *d_v);

/* Moving-least-squares interpolation (Eqs. uLag, l2norm, intKernel) of the
 * vector field d_field [3][N] at n points d_pts [n][3] into d_u [n][3].
 * d_field = NULL interpolates the fluid velocity of the last completed step.
 * Support: the 3x3x3 nodes around the nearest node, solid nodes and nodes
 * outside a non-periodic face excluded.  A point whose support is
 * degenerate gets 0. */
lbm_status ib_interpolate(lbm_ctx *ctx, int64_t n, const double *d_pts, const double *d_field,
                          double *d_u);

/* Spreading (Eq. bodyforce): d_fib [3][N] += sum_l c_l phi_k^l F_l for the
 * n points d_pts [n][3] with forces d_F [n][3] and weights d_c [n].  The sum
 * is accumulated in 64-bit fixed point (unit 2^-57, up to +-64 per node), so
 * it is bitwise reproducible whatever the thread order.  Each contribution
 * c_l phi_k^l F_l must lie in [-1, 1]: one that does not is dropped and the
 * call returns LBM_E_INVAL after the rest was added.  Synchronises the
 * context's stream. */
lbm_status ib_spread(lbm_ctx *ctx, int64_t n, const double *d_pts, const double *d_F,
                     const double *d_c, double *d_fib);

/* ib_spread without allocating: for callers that cannot allocate device
 * memory (code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and errors as
 * ib_spread, bitwise the same d_fib; it allocates nothing (no hipMalloc,
 * hipFree or allocating library call).  Its fixed-point sums live in a
 * fixed device scratch array of 48 MiB plus 256 bytes that every GPU the
 * library runs on holds until the process ends; the call clears the part it
 * uses first.  Lattices of more than 2^21 padded nodes (rows padded to a
 * multiple of 8: px ny nz > 2097152) are refused with LBM_E_INVAL.  All calls
 * on one GPU share that array: calls that overlap on one GPU (other streams,
 * other host threads, other contexts) race and must be serialised by the
 * caller.  Synchronises the context's stream. */
lbm_status ib_spread_noalloc(lbm_ctx *ctx, int64_t n, const double *d_pts, const double *d_F,
                             const double *d_c, double *d_fib);

/* Discrete adjoint of the coupled step (Eqs. evoleq, forcing, bbouzidi,
 * extbound for the fluid; with a soft body, the direct forcing, spreading
 * and MLS interpolation (Eqs. uLag, l2norm, intKernel, bodyforce), the
 * membrane forces (Eqs. strainFor, bendFor, volFor), the probe tractions
 * (Eqs. hydroForP, hydroForNu) and the Verlet update (Eqs. verletPos,
 * verletVel, verletPosC) taken with the step as one map of the state (g, P,
 * Q, V): post-collision deviations g = f - w_i, vertex positions x^n and
 * x^{n-1}, vertex velocities).  For the n_steps-step trajectory that starts
 * from the context's current state and the objective
 *   J = <lambda, g^n> + sum_{t=1..n} <w, g^t>
 * (lambda, w: [19][N] FP64 device arrays, N = nx ny nz, x fastest; w may be
 * NULL), it returns in d_lambda (overwritten) dJ/dg^0 and in d_grad (5
 * doubles, device) dJ/ds, dJ/dFx, dJ/dFy, dJ/dFz, dJ/dtau: s scales the wall
 * velocity of every velocity-face (inlet) node, F is the uniform body force,
 * tau the relaxation time (Eq. evoleq; the viscosity, also in the probes'
 * stress; the membrane modulus k_s0 held fixed), all held fixed over the n
 * steps, derivatives at the context's current values.  The trajectory is
 * recomputed in the context's precision (its storage and arithmetic, as
 * lbm_step runs it); the adjoint is FP64: the transposes of the collision
 * and of Zou-He written out at each node's state, exact transposes of the
 * streaming and bounce-back, and, with a body, the transposes of the IB
 * operations including the derivatives of the MLS weights, face areas and
 * normals with respect to the moving points (for an FP32 or FP16S context,
 * the derivative of the step in exact arithmetic at its states).  Entries of
 * w and lambda at solid nodes are ignored; dJ/dg^0 is zero there.
 * checkpoint_every (K) >= 1; d_w may be NULL; every other pointer is
 * required (else LBM_E_INVAL).
 * Checkpoints: the state is kept every checkpoint_every steps and each
 * segment is recomputed once in the reverse sweep (device memory: 6 FP64
 * fields and ceil(n/K) + max(K, 2) states of 19 x plane values, plus K x 19
 * doubles per boundary record; with a body, eleven FP64 [Np] fields, a
 * state and 9 nv doubles per checkpoint and per step of a segment;
 * allocated and freed by the call; LBM_E_NOMEM if it does not fit).  The
 * context's state and step count are not changed.  Contexts with rigid or
 * fixed bodies, or with more than one body (the repulsion), give
 * LBM_E_UNSUPPORTED; a trajectory on which a capsule is damaged or the flow
 * becomes unstable gives LBM_E_DAMAGED / LBM_E_UNSTABLE.  Synchronises the
 * context's stream. */
lbm_status lbm_adjoint_step(lbm_ctx *ctx, int32_t n_steps, int32_t checkpoint_every,
                            const double *d_w, double *d_lambda, double *d_grad);

/* The same sweep with the capsule objective of the differentiation form and
 * the membrane-stiffness gradient: J adds taylor_weight times the sum over
 * the n steps of the Taylor deformation D = (sqrt(l1) - sqrt(l3)) /
 * (sqrt(l1) + sqrt(l3)) of body taylor_body after each step (l1, l3 the
 * largest and smallest eigenvalues of the second-moment tensor of its vertex
 * positions about their mean).  d_grad takes 6 doubles: the 5 of
 * lbm_adjoint_step, then dJ/dkappa, kappa scaling the membrane modulus k_s0
 * of every body (stretching, bending and the default volume constant follow
 * it; Eqs. strainFor, bendFor, volFor), at the context's current scale
 * (lbm_set_scales; dJ/dk_s0 = dJ/dkappa / k_s0).  d_body_grad (device,
 * [3][nv][3] over all vertices, or NULL): dJ/dx^0, dJ/dx^{-1} and dJ/du_v^0
 * of the initial body state.  J (host, 2 doubles, or NULL): the value of
 * <lambda, g^n> + sum_t <w, g^t>, and the unweighted sum over the steps of
 * the Taylor deformation (0 without bodies), from the recomputed trajectory.
 * taylor_body is ignored when taylor_weight is 0. */
lbm_status lbm_adjoint_run(lbm_ctx *ctx, int32_t n_steps, int32_t checkpoint_every, const double *d_w,
                           double taylor_weight, int32_t taylor_body, double *d_lambda, double *d_grad,
                           double *d_body_grad, double *J);

/* Parameter scales of the problem, relative to the context as created: every
 * inlet (velocity-face) wall velocity times inlet_scale (Eq. extbound), and
 * the membrane modulus k_s0 of every body times stiffness_scale (> 0; the
 * stretching and bending constants and the default volume constant follow;
 * the capillary number becomes Ca / stiffness_scale).  Applies to the steps
 * enqueued after the call; the adjoint's parameter derivatives are taken at
 * these values.  Synchronises the context's stream. */
lbm_status lbm_set_scales(lbm_ctx *ctx, double inlet_scale, double stiffness_scale);

/* Checkpoint / restart of the full state (populations, force field, body
 * state) to a binary file; lbm_load requires a context created with the
 * same geometry and bodies.  lbm_save returns LBM_E_INVAL if the file
 * cannot be opened or fully written.  lbm_load reads and checks the whole
 * file before it changes anything: a file that does not match the context,
 * is truncated or is longer than its state gives LBM_E_INVAL and leaves the
 * context as it was. */
lbm_status lbm_save(lbm_ctx *ctx, const char *path);
lbm_status lbm_load(lbm_ctx *ctx, const char *path);

/* Timing support: average duration in milliseconds of one launch of the
 * fused stream-collide phase, over n_steps full steps launched one kernel
 * at a time (not from the graph).  In each of them the phase is launched 8
 * times back to back between two HIP events on the context's stream (it
 * rewrites the next populations and the macro field from the same inputs,
 * so the step's result is unchanged) and the span is divided by 8. */
lbm_status lbm_time_fluid_kernel(lbm_ctx *ctx, int32_t n_steps, double *avg_ms);

/* FP64 diagnostics of the last completed step (the checks the paper runs on
 * its simulations: conservation, capsule volume and surface, damage):
 * out[0] total mass (sum over non-solid nodes of sum_i f_i), out[1..3] total
 * momentum (sum of f_i e_i) of the post-collision populations, reduced in a
 * fixed order (bitwise reproducible); then per body b, out[4 + 3b ..]: its
 * enclosed volume V, surface S and largest link stretch l/l0 at the current
 * positions.  out is host memory of 4 + 3 * n_bodies doubles.  Synchronises
 * the context's stream. */
lbm_status lbm_diagnostics(lbm_ctx *ctx, double *out);

/* Replay steps from captured HIP graphs (default 1) or launch kernels one by one (0). */
lbm_status lbm_set_graph(lbm_ctx *ctx, int32_t enable);

/* Launch shape of the stream-collide kernel: bulk_v consecutive nodes per
 * thread of a tile (FP64: 1, 2; FP32: 1, 2, 4; FP16S: 2, 4, 8), or 0 for
 * the list form (one bulk node per thread, from the ordered list of bulk
 * nodes: no idle lanes on sparse geometries), and block threads per block
 * (64, 128, 256).  The arithmetic per node does not depend on it, so
 * results are bitwise unchanged.  Synchronises the context's stream;
 * LBM_E_INVAL for an unsupported shape. */
lbm_status lbm_set_launch_shape(lbm_ctx *ctx, int32_t bulk_v, int32_t block);

/* ------------------------------------------------------------------------
 * Batching form: many independent instances (contexts of any size, e.g. the
 * bifurcations of a parameter sweep) advanced together.  Every phase of a
 * coupled step (forcing, stream-collide, probes and vertex velocities,
 * membrane and motion, close) is ONE launch over the work units of all
 * instances -- block g takes unit (instance, block of that instance's own
 * launch) from a device map -- and 16 steps are one HIP graph launch.  Each
 * instance computes exactly what its own lbm_step computes (bitwise).
 * ---------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* Fluid-phase launch shape of a batch: bulk_v and block as for
 * lbm_set_launch_shape; mode 0 runs boundary records and bulk tiles in one
 * launch, mode 1 runs all records, then all bulk tiles; per_xcd > 0 runs the
 * merged units (mode 0) or the bulk tiles (mode 1) in a persistent grid of
 * per_xcd blocks on each of the 8 XCDs, which load an instance's arguments
 * once per run of its units.  fluid_ms: measured duration of the phase (tuner output). */
typedef struct {
  int32_t bulk_v, block, mode, per_xcd;
  double fluid_ms;
} lbm_batch_shape;

/* Groups n contexts (n >= 1, all distinct, same precision, same stream,
 * none periodic along x) into a batch.  The contexts stay owned by the
 * caller, must outlive the batch, and keep working on their own (lbm_sync,
 * lbm_get_*, lbm_step); adding a body or stepping one context alone is
 * picked up by the next batch call.  *out is set even on failure (read
 * lbm_batch_last_error, then lbm_batch_destroy).  LBM_E_UNSUPPORTED for a
 * periodic-x context. */
lbm_status lbm_batch_create(lbm_ctx *const *ctxs, int32_t n, lbm_batch **out);
lbm_status lbm_batch_destroy(lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);

/* n_steps coupled steps of every instance, enqueued on the shared stream.
 * Status bits (unstable, damaged) are per instance: read them with lbm_sync
 * on each context.  An instance that stopped is skipped by every phase. */
lbm_status lbm_batch_step(lbm_batch *b, int32_t n_steps);

/* The autotuner: times the batched stream-collide phase (reps launches after
 * two untimed ones, HIP events on the shared stream) for every shape the
 * precision supports, keeps the fastest, and writes up to max_out of the
 * tried shapes with their times to out (may be NULL) and their count to
 * *n_out.  Timing the phase leaves the run unchanged (it rewrites only what
 * the next step rewrites from the same inputs). */
lbm_status lbm_batch_tune(lbm_batch *b, int32_t reps, lbm_batch_shape *out, int32_t max_out,
                          int32_t *n_out);
lbm_status lbm_batch_set_shape(lbm_batch *b, const lbm_batch_shape *shape);
lbm_status lbm_batch_get_shape(lbm_batch *b, lbm_batch_shape *shape);
/* Average duration (ms) of the batched stream-collide phase over reps launches. */
lbm_status lbm_batch_time_fluid(lbm_batch *b, int32_t reps, double *avg_ms);
/* Graph replay (default 1) or one launch at a time (0). */
lbm_status lbm_batch_set_graph(lbm_batch *b, int32_t enable);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
