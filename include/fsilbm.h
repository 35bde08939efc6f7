/*
 * fsilbm.h -- C ABI of the MI355X (gfx950) library for the two-population
 * compressible lattice Boltzmann fluid-structure step of Bhadauria, Dorschner
 * and Karlin (arXiv 2107.01370).
 *
 * What one step computes (paper Sec. II-IV; staggered weak coupling, Sec. III):
 *   1. surface force F^n and moment M_EA^n from the populations at t^n
 *      (sigma = -p I - (1 - omega/2) P^(1), Sec. III);
 *   2. rigid-body state s^{n+1}: RK4 of the 1DOF / 2DOF spring-mass ODEs with
 *      the load frozen (Sec. IV), or a prescribed motion;
 *   3. blended mesh x^{n+1} = r X + (1 - r) G'(X) (Sec. II.D) and its velocity
 *      V_G = (x^{n+1} - x^n) / dt;
 *   4. collision of f and g with the momentum correction phi and the energy
 *      correction Psi (Sec. II.C, kinetic equations);
 *   5. ALE semi-Lagrangian streaming of all nine populations: departure
 *      points X - dt c^ with c^ = (dx/dX)^{-1}(c - V_G), bilinear inverse
 *      map, 9-node quadratic Lagrange interpolation (Sec. II.A-B); the rest
 *      populations (c = 0) move where the mesh moves (c^_0 = -(dx/dX)^{-1} V_G)
 *      and keep their value where it does not;
 *   6. Grad wall populations and far-field equilibria (Sec. III.A).
 *
 * Conventions
 *   - Lattice units, gas constant R = 1, C_v = 1/(gamma - 1).
 *   - Node (i, j), i fastest; host arrays are row-major [nj][ni].
 *   - Velocity order 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1)
 *     6:(-1,1) 7:(-1,-1) 8:(1,-1); population arrays are [9][nj][ni].
 *   - Every call returns fsi_status (0 = OK, < 0 = error); nothing throws
 *     across the ABI.  On error, fsi_last_error() holds a message.
 *
 * Ownership
 *   - Host inputs are copied during the call that receives them.
 *   - Device memory is owned by the caller: fsi_workspace_bytes() says how
 *     much, fsi_bind_workspace() lends it to the context.  It must stay
 *     allocated, and untouched by the caller, until fsi_destroy().
 *   - Host outputs go to caller-owned buffers of the stated sizes.
 *   - All device work is enqueued on the HIP stream given at creation
 *     (fsi_step() on an O-grid whose step streams more than the 256 MiB
 *     Infinity Cache also forks a second stream of the library's own inside
 *     its captured graph and joins it back before the step ends, so work the
 *     caller enqueues after it on the given stream still follows the step).
 *     fsi_step() is asynchronous; a sticky device error word is checked and
 *     reported by the next synchronising call (fsi_synchronize, fsi_get_*,
 *     fsi_dump_macro, fsi_save).
 *
 * Threading: a context may be used from one host thread at a time.
 */
#ifndef FSILBM_H
#define FSILBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSI_OK = 0,
    FSI_E_ARG = -1,     /* invalid argument or size */
    FSI_E_MESH = -2,    /* det(dX/dxi) <= 0, bad topology, wall cell thinner than dt */
    FSI_E_CFL = -3,     /* a departure point left the cells around its node */
    FSI_E_STATE = -4,   /* rho <= 0, T <= 0, T + u_a^2 >= 1, or NaN */
    FSI_E_HIP = -5,     /* HIP runtime error */
    FSI_E_NOMEM = -6,   /* host allocation failed */
    FSI_E_UNBOUND = -7  /* workspace not bound / state not initialised */
} fsi_status;

typedef struct fsi_ctx fsi_ctx;

/* Storage precision of the populations (arithmetic is FP32 in both). */
enum { FSI_STORE_FP32 = 0, FSI_STORE_FP16_SHIFTED = 1 };

/* Fluid parameters (Sec. II.C): mu = (1/omega - 1/2) p dt with constant mu,
 * Pr = (1/omega - 1/2)/(1/omega_1 - 1/2); free-stream state for the far field. */
typedef struct {
    double gamma;       /* adiabatic exponent (> 1) */
    double Pr;          /* Prandtl number */
    double mu;          /* dynamic viscosity (lattice units) */
    double rho_inf;     /* free-stream density */
    double T_inf;       /* free-stream temperature */
    double u_inf[2];    /* free-stream velocity */
    double dt;          /* time step */
    int storage;        /* FSI_STORE_FP32 or FSI_STORE_FP16_SHIFTED */
} fsi_fluid_params;

/* Mesh topologies.
 *   PERIODIC2: periodic in i and j; crossing a seam adds shift_i / shift_j to
 *              the coordinates.  No wall, no far field.
 *   OGRID:     periodic in i (no shift); row j = 0 is the body wall, row
 *              j = nj - 1 the far field.  dX/dxi must have a positive
 *              determinant (i runs clockwise when j points outward).
 *   CGRID:     C-grid round a section with a wake cut.  i runs from the lower
 *              exit along the lower side of the cut, round the section
 *              (clockwise) and along the upper side of the cut to the upper
 *              exit; n_wake nodes lie on each side of the cut.  Row 0 holds
 *              every cut point and the trailing edge twice: (i, 0) and
 *              (ni - 1 - i, 0) must coincide for i <= n_wake, and node (i, -m)
 *              is node (ni - 1 - i, m).  The wall is row 0 between the two
 *              trailing-edge copies (columns [n_wake, ni - n_wake)); row nj - 1
 *              and the exit columns i = 0, ni - 1 are far field.  The
 *              duplicated nodes are kept single-valued: the two trailing-edge
 *              copies merge (per population, the streamed value of the copy
 *              whose cells hold the departure point, else their mean) and the
 *              upper copy of each cut node takes the lower copy's state.
 *   TWIN:      O-grid round two bodies joined by a slit (a cut of zero
 *              thickness; for several bodies in one flow, Sec. II.D and the
 *              tandem cases of Sec. V).  i is periodic (no shift); row
 *              nj - 1 is far field.  Row 0 runs round the first body (columns
 *              0 .. nA, both ends being the same junction point), along one
 *              side of the slit (n_wake cells), round the second body
 *              (n_wall2 cells: columns nA + n_wake .. nA + n_wake + n_wall2,
 *              both ends the other junction point) and back along the other
 *              side of the slit; nA = ni - 2 n_wake - n_wall2.  Node (i, -m)
 *              is node ((nA - i) mod ni, m), and (i, 0) must coincide with
 *              ((nA - i) mod ni, 0) for nA <= i <= nA + n_wake.  Wall column
 *              segment 0 belongs to body 0, segment 1 to body 1 (nbodies must
 *              be 2).  Junction copies merge and slit copies are kept
 *              single-valued as on a C-grid.
 *   Q9:        unstructured mesh of 9-node quadrilateral elements (the
 *              paper's own discretisation, Sec. II.B): periodic and static
 *              (period shift_i[0] along x, shift_j[1] along y, shifts used by
 *              `elem_shifts`), or bounded, round one body: `wall_nodes` the
 *              body polygon, clockwise (a +90 degree rotation of its tangent
 *              points into the fluid), `far_nodes` the outer boundary.  A
 *              boundary node's population whose departure point lies in none
 *              of the node's elements is missing: far-field nodes take the
 *              free-stream equilibrium, wall nodes Grad's populations (u = the
 *              wall node's mesh velocity, 0 for FSI_DOF_FIXED; rho, T
 *              interpolated at B = X + dt n in the undeformed element of the
 *              node that holds it, the wall nodes there at their previous
 *              values; gradients by the nodal finite-element derivative on the
 *              mesh of the new level with the wall nodes at their targets).
 *              The force is sigma . (n ds) summed over the wall polygon,
 *              (n ds)_k = rot90(x_{k+1} - x_{k-1}) / 2 on the mesh of the
 *              level, the moment about the body's displaced `ea`.  A moving
 *              body (any dof but FSI_DOF_FIXED; radial or distance blending)
 *              needs a rigid zone that holds every element at the wall
 *              (FSI_E_ARG otherwise); nodes move by the blending of Sec. II.D
 *              and each step locates the departure points
 *              X - dt g^{-1}(c - V_G) (the rest direction c = 0 included,
 *              where the node moves) anew among the node's undeformed
 *              elements (g = dx/dX, V_G the node's mesh velocity), trying the
 *              previous step's element first; an interior point outside its
 *              elements is reported as FSI_E_CFL at the next synchronising
 *              call.  ni = number of nodes, nj = 1; X holds the
 *              node coordinates; `elems` [n_elems][9] the nodes of each
 *              element in the order corners (-1,-1), (1,-1), (1,1), (-1,1),
 *              edge midpoints (0,-1), (1,0), (0,1), (-1,0), centre (0,0),
 *              counter-clockwise; `elem_shifts` [n_elems][9][2] the periods
 *              to add to each node's coordinates to place it next to the
 *              element's other nodes.  Edge and centre nodes must sit where
 *              the corners' bilinear map puts them (straight-sided elements):
 *              departure points are located with that map and interpolated
 *              with the nine shape functions.  Nodal derivatives are the mean
 *              over a node's elements of the element derivatives there.
 *              Number nodes along a space-filling curve: each step collides
 *              and interpolates blocks of 256 consecutive nodes through LDS,
 *              so a compact block keeps its halo small (a mesh whose largest
 *              block halo does not fit 64 KiB of LDS, or a context created
 *              with the environment variable FSILBM_UNSTRUCTURED_GATHER set to
 *              "device", gathers through device memory instead; the two agree
 *              to FP32 rounding).                                          */
typedef enum { FSI_TOPO_PERIODIC2 = 0, FSI_TOPO_OGRID = 1, FSI_TOPO_CGRID = 2,
               FSI_TOPO_TWIN = 3, FSI_TOPO_Q9 = 4 } fsi_topo;

/* Most bodies one mesh carries (TWIN: exactly this many). */
#define FSI_MAX_BODIES 2

typedef struct {
    int ni, nj;             /* nodes in i (fast) and j; ni >= 8, nj >= 8 */
    int topo;               /* fsi_topo */
    const double *X;        /* host, [nj][ni][2] undeformed coordinates, FP64; copied */
    double shift_i[2];      /* PERIODIC2 only */
    double shift_j[2];      /* PERIODIC2 only */
    int n_wake;             /* CGRID: cut nodes on each side (>= 2); TWIN: slit cells (>= 2) */
    int n_wall2;            /* TWIN only: wall cells round the second body (>= 8) */
    int n_elems;            /* Q9 only: elements */
    const int32_t *elems;   /* Q9 only: host, [n_elems][9] node indices; copied */
    const int8_t *elem_shifts;  /* Q9 only: host, [n_elems][9][2] periods (-1, 0, 1); copied */
    int n_wall_nodes;       /* Q9 only: nodes of the body's wall polygon (0: no body) */
    const int32_t *wall_nodes;  /* Q9 only: host, [n_wall_nodes], clockwise round the body; copied */
    int n_far_nodes;        /* Q9 only: nodes of the outer boundary (0: periodic mesh) */
    const int32_t *far_nodes;   /* Q9 only: host, [n_far_nodes]; copied */
} fsi_mesh_desc;

/* Rigid-body degrees of freedom (Sec. IV). */
enum { FSI_DOF_PRESCRIBED = 0, FSI_DOF_HEAVE = 1, FSI_DOF_PITCH_PLUNGE = 2,
       FSI_DOF_FIXED = 3 };

/* One body: spring-mass parameters (m h'' + S_a a'' + k_h h = F_y,
 * S_a h'' + I_a a'' + k_a a = M_EA), the blending region of influence
 * (rigid inside r_rigid, r_5 blend out to r_blend, Sec. II.D), the elastic
 * axis `ea` (rotation centre), the initial state and, for FSI_DOF_PRESCRIBED,
 * h(t) = heave_amp sin(2 pi heave_freq t), alpha(t) = pitch_amp sin(2 pi
 * pitch_freq t).  h is along +y, alpha is counter-clockwise.
 *   blend_mode 0: r_rigid, r_blend are radii from `center` (the paper's
 *     choice); 1: distances to the wall (the mesh's wall polygon in the
 *     undeformed frame, computed once per node at creation; meshes with a
 *     wall only, at most 4e9 node-edge pairs), the variant the paper suggests
 *     for slender bodies.
 *   release_time > 0 (FSI_DOF_HEAVE, FSI_DOF_PITCH_PLUNGE): the body follows
 *     the prescribed motion above while t^{n+1} <= release_time and its ODE
 *     afterwards, starting from the state reached (the forced-then-free
 *     protocol of the paper's airfoil case, Sec. V).
 *   Several bodies (Sec. II.D): each moves the nodes of its own region of
 *     influence; the regions may not overlap (FSI_E_ARG names a node that
 *     lies in two).  Distance blending measures from the body's own wall.
 *   link >= 0 (an earlier body that is not linked itself): the body is part
 *     of a rigid assembly with that body (the paper's linked tandem
 *     cylinders): it has no equation of its own, moves with that body's
 *     rigid map (its elastic axis and state; this body's dof, masses,
 *     stiffnesses, ea, initial state and motion are ignored), and its load
 *     joins that body's equation (forces summed, moment about that body's
 *     elastic axis).  Its history reports its own load.  -1: own equation. */
typedef struct {
    int dof;
    double m, S_a, I_a, k_h, k_a;
    double center[2], ea[2];
    double r_rigid, r_blend;
    double h0, a0, hd0, ad0;
    double heave_amp, heave_freq, pitch_amp, pitch_freq;
    double release_time;     /* see above; 0: no forced start */
    int blend_mode;          /* 0 radial, 1 distance to the wall */
    int link;                /* -1, or the body this one moves with */
} fsi_body_desc;

/* Create a context for one structured mesh with its moving bodies: 0 or 1 on
 * a PERIODIC2, OGRID or CGRID mesh, FSI_MAX_BODIES on a TWIN mesh (body k
 * owns wall segment k).  `hip_stream` is a hipStream_t (NULL = default
 * stream).  Validates the mesh (FSI_E_MESH) and precomputes the static
 * boundary geometry on the host.  No device memory is allocated. */
fsi_status fsi_create(const fsi_fluid_params *fluid, const fsi_mesh_desc *mesh,
                      const fsi_body_desc *bodies, int nbodies, void *hip_stream,
                      fsi_ctx **out);

/* Bytes of device workspace the context needs (populations ping-pong,
 * coordinates, boundary and body buffers). */
fsi_status fsi_workspace_bytes(const fsi_ctx *ctx, size_t *bytes);

/* Lend `bytes` of device memory at `dev_ptr` (256-byte aligned) to the
 * context and upload the static data.  Synchronises the stream.  Q9 meshes:
 * also locates every departure point of the undeformed mesh once (a moving
 * body relocates them every step); FSI_E_CFL if one lies outside the
 * elements of its node (dt too large for the mesh). */
fsi_status fsi_bind_workspace(fsi_ctx *ctx, void *dev_ptr, size_t bytes);

/* Initial populations = equilibria (f^eq, g^eq with Psi) of the given host
 * fields [nj][ni] (NULL = free-stream values), body state from the body
 * description, step counter 0; computes the initial load F^0 and s^1.
 * Synchronises. */
fsi_status fsi_init_equilibrium(fsi_ctx *ctx, const double *rho, const double *ux,
                                const double *uy, const double *T);

/* Enqueue `nsteps` coupled steps: replays of a captured HIP graph of 16
 * steps, then of one step for the remainder (both captured on first use).
 * Asynchronous.  On an O-grid whose step streams more than the Infinity
 * Cache, the first call creates a second stream (and two events) of the
 * context's own, released by fsi_destroy(): each captured step runs the
 * interior tiles of the collision-streaming kernel there, beside the tiles
 * next to the wall and the far field and the boundary kernels, and joins
 * before the body kernel (results are those of one launch, bit for bit). */
fsi_status fsi_step(fsi_ctx *ctx, int nsteps);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same `nsteps` coupled
 * steps as fsi_step, with the same kernels and results, but launched directly
 * on the context's stream (no graph is captured or instantiated, nothing is
 * allocated, no memset is recorded, no second stream: the collision-streaming
 * kernel runs as one launch over every tile).  The step's temporaries (wall masks,
 * wall targets, per-node tractions, cut staging: 52 * ni bytes plus
 * 72 * (cut columns) bytes, each part rounded up to 256) live in a static
 * device array of 1 MiB per GPU, held until the process ends, instead of the
 * workspace; its address on the device current at fsi_bind_workspace is
 * looked up there.  Structured meshes only (FSI_E_ARG for 9-node meshes and
 * for meshes whose temporaries exceed 1 MiB).  Every call on one GPU shares
 * the array: calls on different contexts that overlap in time on one GPU
 * race (serialise them, e.g. on one stream).  No entry of the array needs to
 * start at zero (each step writes every entry before reading it).
 * Asynchronous, like fsi_step; the inputs and outputs are the context's bound
 * state. */
fsi_status fsi_step_noalloc(fsi_ctx *ctx, int nsteps);

/* Wait for the stream and report the sticky device error word
 * (FSI_E_CFL, FSI_E_STATE, FSI_E_MESH). */
fsi_status fsi_synchronize(fsi_ctx *ctx);

/* Number of completed steps (synchronises). */
fsi_status fsi_get_step(fsi_ctx *ctx, int64_t *step);

/* History records of body `body` for steps first .. first+count-1, each
 * {n, F_x, F_y, M_EA, h, alpha} at the start of step n (F from f^n).  The
 * library keeps the last `fsi_history_capacity()` records.  Synchronises. */
fsi_status fsi_get_forces(fsi_ctx *ctx, int body, int64_t first, int count, double *out);
int64_t fsi_history_capacity(void);

/* Current body state {h, alpha, hdot, alphadot}.  Synchronises. */
fsi_status fsi_get_body_state(fsi_ctx *ctx, int body, double out[4]);

/* Macroscopic fields of the current populations, host [nj][ni] each
 * (any pointer may be NULL).  Synchronises. */
fsi_status fsi_dump_macro(fsi_ctx *ctx, double *rho, double *ux, double *uy, double *T);

/* Current populations as FP32 host arrays [9][nj][ni] (decoded from the
 * storage precision).  Synchronises. */
fsi_status fsi_get_populations(fsi_ctx *ctx, float *f, float *g);

/* Overwrite the current populations from FP32 host arrays [9][nj][ni]
 * (encoded to the storage precision).  Does not change the body state. */
fsi_status fsi_set_populations(fsi_ctx *ctx, const float *f, const float *g);

/* Checkpoint: populations (storage precision), body states, step counter and
 * parameters; with a moving body on a Q9 mesh also the departure table
 * (element and local coordinates per node and direction) that each step's
 * relocation starts from, so that a restart repeats the run bitwise.
 * fsi_state_bytes() gives the buffer size. */
fsi_status fsi_state_bytes(const fsi_ctx *ctx, size_t *bytes);
fsi_status fsi_save(fsi_ctx *ctx, void *host_buf, size_t bytes);
fsi_status fsi_load(fsi_ctx *ctx, const void *host_buf, size_t bytes);

/* Strong coupling by sub-iterations (Sec. III names it as the alternative to
 * the staggered scheme for small solid-to-fluid mass ratios; the paper gives
 * no algorithm).  Each step starts from the staggered predictor (the body
 * advanced with the load of t^n frozen); each of the first subiterations - 1
 * passes streams the post-collision populations of t^n onto the mesh of the
 * current body estimate, applies the boundary conditions, takes the new load,
 * re-solves the body equation over the step with the load varying linearly
 * from F^n to it, and moves the estimate that fraction `relaxation` of the way
 * to the solution; the last pass is accepted (populations and the body state
 * they were computed with).  1 sub-iteration = the staggered scheme (the
 * default).  Each pass costs one collision-streaming launch.  FSI_E_ARG unless
 * 1 <= subiterations <= 64 and 0 < relaxation <= 1.  On a Q9 mesh each pass
 * after the first first forms again the level-n moments and wall values that
 * the previous pass overwrote.  Invalidates the captured graph; the state is
 * kept. */
fsi_status fsi_set_coupling(fsi_ctx *ctx, int subiterations, double relaxation);

/* Largest change |solution - estimate| of body `body`'s state components in
 * the last pass of the latest step (how far the sub-iterations are from
 * converged; 0 with one sub-iteration).  Synchronises. */
fsi_status fsi_get_coupling_residual(fsi_ctx *ctx, int body, double *residual);

/* Time each kernel of one coupled step with HIP events on the context's
 * stream: `reps` back-to-back launches of the collision-streaming kernel, of
 * the two wall kernels and of the body kernel, at the current step (every
 * launch recomputes the same values, so the state is unchanged).  out_ms[4]
 * receives the mean milliseconds per launch, in that order (0 for kernels the
 * topology does not use).  On a Q9 mesh the first entry covers the element
 * derivatives, nodal means and collision-interpolation of a step (without
 * the mesh motion and relocation of a moving body, which are left alone);
 * the moments of the next step are formed again afterwards.  Synchronises. */
fsi_status fsi_time_kernels(fsi_ctx *ctx, int reps, double out_ms[4]);

/* ---------------------------------------------------------------------------
 * Batches: many independent instances (each one mesh with its bodies, of any
 * sizes) advanced together.  Every step is ONE launch of each kernel over
 * the concatenated work items of all instances, captured in one HIP graph.
 * Instances keep their own parameters, state, history and error word.
 * ------------------------------------------------------------------------- */
typedef struct fsi_batch fsi_batch;

/* Create a batch of n instances: fluids[n], meshes[n]; instance k has
 * nbodies[k] bodies (nbodies may be NULL: no bodies), stored back to back in
 * `bodies` in instance order.  All instances must use the same storage
 * precision.  Validation as fsi_create; the failing instance is named in
 * fsi_batch_last_error(). */
fsi_status fsi_batch_create(int n, const fsi_fluid_params *fluids, const fsi_mesh_desc *meshes,
                            const fsi_body_desc *bodies, const int *nbodies, void *hip_stream,
                            fsi_batch **out);
fsi_status fsi_batch_workspace_bytes(const fsi_batch *b, size_t *bytes);
fsi_status fsi_batch_bind_workspace(fsi_batch *b, void *dev_ptr, size_t bytes);
/* Initial equilibria of instance k (NULL fields = its free stream). */
fsi_status fsi_batch_init_equilibrium(fsi_batch *b, int k, const double *rho, const double *ux,
                                      const double *uy, const double *T);
/* Work distribution of the collision-streaming launch: `grid` workgroups (0 =
 * one per work item; otherwise a persistent grid, rounded to a multiple of 8),
 * `order` of the work items (0: instance after instance, 1: instances by
 * decreasing size) and the tile `shape` of the arrival nodes one workgroup owns
 * (0: 32 x 16, the default, 1: 64 x 8, 2: 16 x 32, 3: 16 x 16 with 256-thread
 * workgroups).  The shape applies to the instances without a cut; C-grid, TWIN
 * and two-body instances always run on 32 x 16 tiles, in a launch of their own.
 * Invalidates the captured graph.  FSI_E_ARG on values out of range. */
fsi_status fsi_batch_set_schedule(fsi_batch *b, int grid, int order, int shape);
/* Time candidate schedules on the current state and keep the fastest: after
 * warm-up launches, each (shape, order, grid) candidate is timed twice over
 * `reps` launches of the collision-streaming kernel (each recomputes the same
 * values, so the state is unchanged) and its faster pass counts;
 * best[4] = {grid, order, shape, mean ms per launch}.  Synchronises. */
fsi_status fsi_batch_autotune(fsi_batch *b, int reps, double best[4]);
/* The same coupling for every instance, as fsi_set_coupling. */
fsi_status fsi_batch_set_coupling(fsi_batch *b, int subiterations, double relaxation);
fsi_status fsi_batch_step(fsi_batch *b, int nsteps);
fsi_status fsi_batch_synchronize(fsi_batch *b);
/* Per-instance queries, as the single-instance calls. */
fsi_status fsi_batch_get_forces(fsi_batch *b, int k, int body, int64_t first, int count,
                                double *out);
fsi_status fsi_batch_get_body_state(fsi_batch *b, int k, int body, double out[4]);
fsi_status fsi_batch_dump_macro(fsi_batch *b, int k, double *rho, double *ux, double *uy,
                                double *T);
fsi_status fsi_batch_get_populations(fsi_batch *b, int k, float *f, float *g);
/* Mean ms per launch of the batched kernels, as fsi_time_kernels. */
fsi_status fsi_batch_time_kernels(fsi_batch *b, int reps, double out_ms[4]);
int64_t fsi_batch_nodes(const fsi_batch *b);
const char *fsi_batch_last_error(const fsi_batch *b);
/* Waits for queued work, then releases the batch (not the workspace). */
void fsi_batch_destroy(fsi_batch *b);

/* Message of the last error on this context (static storage of the context). */
const char *fsi_last_error(const fsi_ctx *ctx);

/* Wait for the work queued on the context's stream, then release the context
 * (not the caller's workspace, which may be freed once this returns). */
void fsi_destroy(fsi_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FSILBM_H */
