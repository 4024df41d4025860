/*
 * iblb.h -- C ABI of libiblb, one immersed-boundary / lattice-Boltzmann
 * (IB-LB) time step on an AMD Instinct MI355X (gfx950).
 *
 * Method: Pelusi, Guglietta, Sega, Aouane, Harting, "A sharp interface
 * approach for wetting dynamics of hydrophobic coated droplets and soft
 * particles", arXiv:2305.18919.  One call of iblb_step advances the coupled
 * system by one lattice time step in the order of the algorithm listed at the
 * end of the "Numerical implementation" section:
 *   1. nodal forces phi_i = phi^S + phi^V + phi^W       (Eq. total_nodal_force)
 *        phi^S = -dW/dq, W = sum_faces A0 w_S(I1, I2)    (Eqs. generalised_energy1,
 *                                                         nodal_force_S)
 *        phi^V = -d/dq [k_V (V - V0)^2 / (2 V0)]         (Eq. nodal_force_V)
 *        phi^W = face-centroid Lennard-Jones wall force   (Eq. LJ_interaction)
 *   2. spreading F(x) = sum_i phi_i delta_D(x - q_i)     (Eq. ibm-governing_eq2)
 *   3. D3Q19 BGK collision with Guo forcing, streaming   (Eqs. LBeq, feq)
 *   4. fluid velocity u = (sum c f + F/2)/rho            (Guo velocity)
 *   5. interpolation qdot_i = sum_x u(x) delta_D(x - q_i) (Eq. ibm-governing_eq1)
 *   6. q_i <- q_i + qdot_i                               (Eq. ibm_update_pos)
 * with delta_D the product of three 4-point stencils phi4
 * (Eq. ibm-interpolation_stencil), periodic x and y, and half-way bounce-back
 * walls in z (the paragraph after the algorithm).
 *
 * Conventions shared by every call
 *  - Lattice units: dx = dt = 1, c_s^2 = 1/3.  Node (x, y, z) sits at integer
 *    coordinates.  With IBLB_WALLS_Z the layers z = 0 and z = nz-1 are solid,
 *    the fluid is z = 1 .. nz-2 and the wall planes are z = 0.5 and z = nz-1.5.
 *  - Field arrays on the host are [component][z_fluid][y][x], x fastest,
 *    z_fluid = z - 1 with walls (z with IBLB_PERIODIC_ALL).  N = nx*ny*nz_fluid.
 *  - Populations are exchanged as deviations f_i - w_i rho0 in the canonical
 *    D3Q19 order: i = 0 rest; 1,2 = (+-1,0,0); 3,4 = (0,+-1,0); 5,6 = (0,0,+-1);
 *    7,8 = +-(1,1,0); 9,10 = +-(1,-1,0); 11,12 = +-(1,0,1); 13,14 = +-(1,0,-1);
 *    15,16 = +-(0,1,1); 17,18 = +-(0,1,-1); weights 1/3, 1/18 (1..6), 1/36.
 *  - Vertex arrays on the host are [vertex][xyz] doubles, unwrapped
 *    coordinates (x and y are not folded back into the box).
 *  - Every function returns IBLB_OK (0) or a negative IBLB_E_* code and never
 *    aborts or throws; iblb_last_error() then holds a message.  Errors raised
 *    inside kernels (non-finite state, list overflow) are reported by the next
 *    call that synchronises (iblb_sync and every getter).
 *  - Host pointers passed in are read during the call only (inputs are
 *    copied).  Output buffers belong to the caller.
 *  - One context per host thread; calls on one context are not thread-safe.
 */
#ifndef IBLB_H
#define IBLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    IBLB_OK = 0,
    IBLB_E_INVAL = -1,    /* bad argument or size */
    IBLB_E_DEVICE = -2,   /* HIP runtime error */
    IBLB_E_MESH = -3,     /* mesh not closed / not consistently oriented / degenerate */
    IBLB_E_UNSTABLE = -4, /* non-finite or runaway state found on the device */
    IBLB_E_STATE = -5     /* call not valid in the current state */
};

enum {                                            /* population storage and LB arithmetic */
    IBLB_FP64 = 0,
    IBLB_FP32_DEV = 1,
    IBLB_FP16_DEV = 2,
    IBLB_BF16_DEV = 3
};
enum { IBLB_WALLS_Z = 0, IBLB_PERIODIC_ALL = 1 };   /* z boundary */

typedef struct iblb_ctx iblb_ctx;

typedef struct {
    int32_t nx, ny, nz;        /* lattice size incl. the two solid layers when IBLB_WALLS_Z; each >= 8 */
    int32_t wall_mode;         /* IBLB_WALLS_Z or IBLB_PERIODIC_ALL */
    int32_t precision;         /* IBLB_FP64: FP64 populations and LB arithmetic;
                                  IBLB_FP32_DEV: FP32 deviations f - w rho0, FP32 LB and
                                  interface arithmetic; positions, volume and area stay FP64;
                                  IBLB_FP16_DEV / IBLB_BF16_DEV: as FP32_DEV, but each
                                  population is stored in 16 bits as (f - w rho0) / w,
                                  times 2^12 for FP16 (|(f - w rho0) / w| < 16), rounded to
                                  nearest even; the arithmetic stays FP32 */
    int32_t init_couette;      /* 0: fluid at rest; 1: f = f^eq(rho0, u linear between the walls) */
    double tau;                /* BGK relaxation time (> 1/2); viscosity (tau - 1/2)/3 */
    double rho0;               /* initial and reference density */
    double u_wall_lo[3];       /* velocity of the wall at z = 0.5 (tangential) */
    double u_wall_hi[3];       /* velocity of the wall at z = nz - 1.5 */
    double body_force[3];      /* uniform force density added to F on every node */
} iblb_domain_desc;

typedef struct {
    int32_t n_vertices, n_faces; /* 4 <= n_vertices <= 65536 */
    const double *vertices;     /* host [n_vertices][3]: initial positions q(0) */
    const double *ref_vertices; /* host [n_vertices][3]: stress-free shape; NULL => vertices */
    const int32_t *faces;       /* host [n_faces][3]: closed surface, outward counter-clockwise */
    double alpha[3];            /* (alpha1, alpha2, alpha3) of Eq. generalised_energy1 */
    double k_v;                 /* volume stiffness k_V of Eq. nodal_force_V (paper: 1) */
    double eps_wall_lo;         /* LJ strength of the wall at z = 0.5 (0: off) */
    double eps_wall_hi;         /* LJ strength of the wall at z = nz - 1.5 (0: off) */
    double xi_wall;             /* LJ length xi (paper: 0.5) */
    double r_cut_wall;          /* LJ cut-off distance from the wall plane */
} iblb_mesh_desc;

/* Device bytes needed by a context for this domain and (optional, may be NULL)
 * mesh, for callers that pass their own workspace to iblb_create. */
int iblb_workspace_bytes(const iblb_domain_desc *dom, const iblb_mesh_desc *mesh, size_t *bytes);

/* Create a context on the current HIP device.
 * dev_workspace: device buffer of >= iblb_workspace_bytes(dom, NULL) bytes that
 *   the caller owns and keeps alive until iblb_destroy (e.g. a torch uint8
 *   tensor); NULL => the library allocates and frees its own memory.  A
 *   workspace of iblb_workspace_bytes(dom, mesh) bytes also holds the mesh
 *   arrays of iblb_add_mesh; a smaller one makes iblb_add_mesh allocate them.
 * hip_stream: hipStream_t all work is enqueued on; NULL => a private stream.
 * Initialises the populations (rest, or Couette when init_couette = 1). */
int iblb_create(const iblb_domain_desc *dom, void *dev_workspace, size_t workspace_bytes,
                void *hip_stream, iblb_ctx **out);

/* Attach the (single) mesh.  Validates that the surface is closed and
 * consistently oriented, copies the inputs, precomputes per-face reference
 * data (metric inverse, area) and the reference volume V0 (volume of
 * ref_vertices), and bins the vertices for the first step.  V - V0 is later
 * evaluated face by face, expanded exactly in the displacements from
 * ref_vertices.  *mesh_id = 0.  Fails with IBLB_E_STATE if a mesh exists or a
 * debug force field is set, IBLB_E_INVAL above 65536 vertices (the spreading
 * keeps one bit per vertex for every tile of the lattice, see
 * iblb_tile_shape: tiles x ceil(n_vertices / 64) x 8 bytes of device
 * memory). */
int iblb_add_mesh(iblb_ctx *ctx, const iblb_mesh_desc *mesh, int32_t *mesh_id);

/* Enqueue n_steps full IB-LB steps on the context stream; returns without
 * waiting.  In graph mode (default) a captured hipGraph of 16 steps that
 * starts at an even time is replayed; the remaining steps are launched
 * directly. */
int iblb_step(iblb_ctx *ctx, int32_t n_steps);

/* Wait for the context stream and report device-side errors. */
int iblb_sync(iblb_ctx *ctx);

/* Number of completed steps (host count of enqueued steps). */
int iblb_step_count(const iblb_ctx *ctx, int64_t *t);

/* Vertex positions q(t) -> host [n_vertices][3] (synchronises). */
int iblb_get_vertices(iblb_ctx *ctx, int32_t mesh_id, double *host_out);

/* Device pointer to the FP64 positions, structure-of-arrays [3][n_vertices]
 * (all x, then all y, then all z).  Valid until the next step is enqueued;
 * the caller must order its reads after the context stream. */
int iblb_vertices_device(iblb_ctx *ctx, int32_t mesh_id, const double **dev_ptr);

/* Enclosed volume V and surface area A of the current mesh, FP64 reductions
 * (V from signed tetrahedra, Eq. nodal_force_V's V = sum_j V_j). */
int iblb_volume(iblb_ctx *ctx, int32_t mesh_id, double *V, double *A);

/* Shape in the x-z shear plane: Taylor deformation D = (r1 - r3)/(r1 + r3)
 * (Eq. taylor_deform) and inclination Theta of r1 from +x in (-pi/2, pi/2],
 * with r1, r3 from the central second-moment tensor of the enclosed volume read
 * as an ellipsoid (M = V/5 diag(r^2)); centroid = volume centroid. */
int iblb_shape(iblb_ctx *ctx, int32_t mesh_id, double *D, double *Theta, double centroid[3]);

/* Contact angle against a wall (0: lower, 1: upper), FP64, from vertices at
 * least 2 lattice units away from that wall plane.
 *   method 1: the paper's measurement (appendix on the resolution test), a
 *     circle cut by the wall chord fitted by algebraic least squares in the
 *     (x, z) plane to a slice of the mesh: the K = round((4 / 3^(1/4))
 *     sqrt(pi N_f)) vertices nearest the plane y = y of the volume centroid,
 *     ties to the lower vertex index (K capped at the vertex count).
 *   method 0: an algebraic least-squares sphere fit of all those vertices
 *     (the three-dimensional form of the same cap).
 * Returns the angle in degrees measured inside the liquid, the contact radius
 * and the height of the fitted cap above the wall plane.  IBLB_E_INVAL for
 * another wall or method, IBLB_E_STATE without walls or with too few vertices
 * (4 for the sphere, 3 for the circle) away from the wall. */
int iblb_contact_angle(iblb_ctx *ctx, int32_t mesh_id, int32_t wall, int32_t method,
                       double *theta_deg, double *contact_radius, double *height);

/* rho [N] and u [3][N] on the fluid nodes at the current time, with the force
 * density of the last step in the Guo velocity (zero before the first step). */
int iblb_get_fields(iblb_ctx *ctx, double *rho, double *u);

/* Allocation-free form of iblb_get_fields, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * iblb_get_fields, which allocates a device staging buffer of 32 bytes per
 * fluid node on every call; this one stages through a fixed device array of
 * IBLB_NOALLOC_MAX_NODES * 32 bytes (64 MiB) that the library holds on every
 * GPU it runs on until the process ends.  Lattices with more fluid nodes get
 * IBLB_E_INVAL; IBLB_E_DEVICE if the array could not be located on the
 * context's device.  All calls on one GPU share that array: calls that
 * overlap on one GPU (from several threads) race. */
#define IBLB_NOALLOC_MAX_NODES 2097152
int iblb_get_fields_noalloc(iblb_ctx *ctx, double *rho, double *u);

/* The cost of ordering two phases of a step across the whole GPU, two ways:
 * `rounds` back-to-back launches of a kernel of `blocks` 256-thread blocks,
 * replayed from a captured graph (kernel boundaries), against one
 * cooperative kernel of `blocks` blocks passing `rounds` grid-wide barriers
 * (an atomic arrival count and generation).  Each block writes one word per
 * phase in both.  Outputs: microseconds per boundary and per barrier, the
 * median of 5 repetitions.  This is the measurement behind the batched
 * step's dispatch-per-phase design.  Allocates its own stream and buffer.
 * IBLB_E_INVAL for rounds outside [1, 100000], or blocks beyond what the GPU
 * holds at once; IBLB_E_UNSTABLE if a barrier wait gave up (the kernel ends
 * in any case); IBLB_E_DEVICE for runtime errors. */
int iblb_probe_phase_sync(int32_t blocks, int32_t rounds, double *boundary_us, double *barrier_us);

/* Debug / validation calls. */
/* Fixed external force density [3][N] added every step; only without a mesh. */
int iblb_debug_set_force(iblb_ctx *ctx, const double *F);
/* Force density of the last step [3][N] (IB + body + external; zero before the first step). */
int iblb_debug_get_force(iblb_ctx *ctx, double *F);
/* Population deviations f_i - w_i rho0 at the current time, [19][N] canonical order. */
int iblb_debug_get_populations(iblb_ctx *ctx, double *f);
int iblb_debug_set_populations(iblb_ctx *ctx, const double *f);
/* Nodal forces phi_i of the last step, host [n_vertices][3]. */
int iblb_debug_get_nodal_forces(iblb_ctx *ctx, int32_t mesh_id, double *phi);

/* Checkpoint: host_buf == NULL => *bytes receives the size; else the complete
 * state (populations, positions, last force field, step count) is written.
 * iblb_load_state accepts only a buffer from a context of identical shape,
 * precision and mesh size. */
int iblb_save_state(iblb_ctx *ctx, void *host_buf, size_t *bytes);
int iblb_load_state(iblb_ctx *ctx, const void *host_buf, size_t bytes);

/* Execution controls.  graph != 0: iblb_step replays captured hipGraphs
 * (default) of 16 steps and of one step, for either parity of the start
 * time; iblb_set_graph(ctx, 1) captures them at once (they are captured on
 * first use otherwise), so that no later call of iblb_step captures.  0:
 * plain launches.  timing != 0: plain launches of the same dispatches, each
 * bracketed by hipEvents on the context stream, accumulated until read.
 * Capture errors return IBLB_E_DEVICE. */
int iblb_set_graph(iblb_ctx *ctx, int32_t graph);
int iblb_set_timing(iblb_ctx *ctx, int32_t timing);
/* Launch shape of the LB of the nodes outside the active tiles (for
 * accounting): blocks of block_x x (256 / block_x) nodes of one z layer,
 * numbered x fastest, the first share_forces of them run by the forces
 * dispatch and the rest by the spreading dispatch.  Either output may be
 * NULL. */
int iblb_get_lb_split(const iblb_ctx *ctx, int32_t *block_x, double *share_forces);
/* Per-dispatch accumulated event time.  names: "forces" (interface forces,
 * the list of active tiles, and their share of the LB outside the active
 * tiles), "spread" (spreading, the LB of the active tiles, and the rest of
 * that LB), "moments" (u(t+1) on the active tiles), "move" (interpolation
 * and move), "lb" (the step without a mesh).  Returns total milliseconds and
 * launch count; resets nothing. */
int iblb_kernel_time(iblb_ctx *ctx, const char *name, double *total_ms, int64_t *launches);
int iblb_reset_timing(iblb_ctx *ctx);

/* Fluid nodes in the active tiles of the last completed step, the tiles
 * reached by some vertex's 4^3 stencil (Eq. ibm-interpolation_stencil; their LB
 * runs with the spreading, the "lb" kernel updates the rest); 0 without a mesh
 * or before the first step.  Synchronises. */
int iblb_active_nodes(iblb_ctx *ctx, int64_t *n);

/* Extents in fluid nodes along x, y and z of the tiles the lattice is cut
 * into for the spreading (product 64, one wavefront's lanes; tile (i, j, k)
 * holds the nodes x in [i tx, (i + 1) tx), y and z likewise, z counted in
 * fluid layers; tiles at the lattice's far faces are partial).  Any pointer
 * may be null; never fails. */
void iblb_tile_shape(int32_t *tx, int32_t *ty, int32_t *tz);

const char *iblb_last_error(const iblb_ctx *ctx);
int iblb_destroy(iblb_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Batches of independent domains
 *
 * Parameter sweeps (the contact-angle campaigns of the "Results" section, the
 * capillary-number sweep of the shear benchmark) run many small, independent
 * domains.  A batch advances several contexts together: each step launches
 * each step kernel once for all members, every block working on one member's
 * arrays, so the members share the per-kernel launch and cache-flush costs
 * that dominate a small domain's step.  Each member computes what iblb_step
 * computes for it, in the same operation order: the batched kernels are
 * compiled from the same code, so a member agrees with the same context
 * stepped alone to rounding (the compiler fuses a different set of
 * multiply-adds).  Every launch shape of iblb_batch_config gives
 * bit-identical results, except vertices_per_wave, which changes the order of
 * the interpolation sums.
 *
 * Members are contexts created with iblb_create / iblb_add_mesh on the
 * current device: each has a mesh, all have the same precision and step
 * parity.  They stay owned by the caller, must outlive the batch and keep
 * answering every query (vertices, volume, shape, contact angle, fields,
 * checkpoints).  Work is ordered against each member's stream with events,
 * so queries on a member see the batch's steps.  Stepping a member on its own
 * while it is in a batch is allowed, but the next batch call then fails with
 * IBLB_E_STATE if the members' step parities differ.
 * ------------------------------------------------------------------------- */
typedef struct iblb_batch iblb_batch;

typedef struct {
    int32_t lb_block_x;           /* LB blocks of lb_block_x x (256 / lb_block_x) nodes of one z
                                     layer: 16, 32 or 64 (capped per member by its nx); 0 = the
                                     single-context rule (64 if nx >= 64, 32 if nx >= 32, else 16) */
    int32_t spread_blocks_per_cu; /* spreading blocks of the whole batch per compute unit, 1..8,
                                     shared out in proportion to the members' active tiles; the
                                     blocks are two wavefronts (four while a stepped member has
                                     more than 32768 vertices); 0 = eight wavefronts per compute
                                     unit (four with FP64) */
    int32_t vertices_per_wave;    /* interpolation and move: 1 or 2 vertices per 64-lane wavefront;
                                     0 = 1 while the batch has at most 32 vertices per compute unit */
    int32_t reserved;             /* 0 */
    double lb_share_forces;       /* fraction of each member's LB blocks (nodes outside the active
                                     tiles) run in the forces dispatch, [0, 1]; default 0.6 */
} iblb_batch_config;

/* Groups n (1..256) distinct contexts.  hip_stream: the stream the batch's
 * launches go to (NULL => a stream of its own).  Errors: IBLB_E_INVAL (null or
 * repeated member, n out of range), IBLB_E_STATE (a member without mesh, or
 * precisions or step parities that differ), IBLB_E_DEVICE. */
int iblb_batch_create(iblb_ctx *const *members, int32_t n, void *hip_stream, iblb_batch **out);
/* n_steps steps of every member that is not frozen (asynchronous; replays a
 * captured hipGraph of 16 steps from even times).  Each member's step count
 * advances by n_steps.  A member whose device error bits are set stops at
 * once: its blocks return without work until iblb_batch_check freezes it, so
 * the garbage state of an unstable member costs the others nothing. */
int iblb_batch_step(iblb_batch *b, int32_t n_steps);
int iblb_batch_sync(iblb_batch *b);
/* Synchronises, reads every member's device error bits and freezes each
 * member that reports one: later batch steps leave it where it is.
 * status (NULL or n entries): IBLB_OK, or IBLB_E_UNSTABLE for a frozen member
 * (iblb_batch_member_error gives the reason); *n_frozen: frozen members. */
int iblb_batch_check(iblb_batch *b, int32_t *status, int32_t *n_frozen);
const char *iblb_batch_member_error(const iblb_batch *b, int32_t member);
/* Launch shape of the batch's dispatches; get returns the resolved values. */
int iblb_batch_get_config(const iblb_batch *b, iblb_batch_config *cfg);
int iblb_batch_set_config(iblb_batch *b, iblb_batch_config const *cfg);
/* Autotuner: times trial_steps (rounded up to a multiple of 16) graph-replayed
 * steps of the batch for each launch shape visited by two passes of
 * coordinate descent over lb_block_x {16, 32, 64}, lb_share_forces {0.3,
 * 0.45, 0.6, 0.75, 0.9}, spread_blocks_per_cu {2, 4, 6} ({1, 2, 3} with
 * four-wavefront spreading blocks) and vertices_per_wave
 * {1, 2}, keeps the fastest and writes its time per step (ms).  The members'
 * device state is copied aside first and restored afterwards (needs that much
 * free device memory), so the trial steps leave no trace. */
int iblb_batch_tune(iblb_batch *b, int32_t trial_steps, double *best_ms_per_step);
const char *iblb_batch_last_error(const iblb_batch *b);
/* Synchronises and frees the batch; the members are untouched. */
int iblb_batch_destroy(iblb_batch *b);

/* ---- Discrete adjoint of the step (reverse mode)
 * Gradients of an observable J(q(t0 + n)) of the mesh's final vertex
 * positions, after n steps from t0, with respect to the mesh parameters of
 * the nodal forces (alpha_1, alpha_2, alpha_3 of Eq. generalised_energy1, k_V
 * of Eq. nodal_force_V, eps of the lower wall in Eq. LJ_interaction), the
 * relaxation time tau of Eq. LBeq and the positions q(t0).  The reverse sweep
 * takes the transpose of every operation of the step (the algorithm at the end
 * of the "Numerical implementation" section) in reverse order; the adjoint of
 * the populations is kept in FP64 arithmetic.  J itself is the caller's: it
 * passes dJ/dq(t0 + n).  Requires a mesh (IBLB_E_STATE otherwise).
 *
 * Steps the context n times (like iblb_step) and records what the reverse
 * sweep needs:
 *  every = 0: every time level and the forward's own fields of each step in
 *    device memory, in the step's arithmetic precision (FP64 for FP64
 *    storage, FP32 otherwise): per step 25 x N values (populations, force
 *    density, velocity), 6 x n_vertices values (nodal force parts, dV/dq),
 *    3 x n_vertices + 1 doubles (positions, V - V0), and the step's tile
 *    vertex masks and active-tile list (tiles x (8 ceil(n_vertices / 64) + 4)
 *    bytes, tiles = ceil(nx/tx) ceil(ny/ty) ceil(N / (nx ny) / tz) with the
 *    extents of iblb_tile_shape); the sweep
 *    then recomputes nothing.  Its adjoint populations are stored in the same
 *    precision.
 *  every > 0: a device copy of the whole context state every `every` steps;
 *    the sweep restores each segment's checkpoint, records the segment again
 *    as above and walks it backwards.  It holds two such recordings (2 x
 *    (every + 1) levels and 2 x every steps of fields in device memory): the
 *    segment before is recorded on the context's stream while the segment
 *    after it is swept on a second stream the library owns, ordered with
 *    events; iblb_adjoint_backward returns once both are done.
 * Replaces any earlier recording.  The context is left at t0 + n.  Errors:
 * IBLB_E_INVAL (null context, n < 1, every < 0), IBLB_E_STATE (no mesh),
 * IBLB_E_DEVICE (the recording does not fit in device memory, or a HIP
 * error). */
int iblb_adjoint_record(iblb_ctx *ctx, int32_t n_steps, int32_t every);
/* Reverse sweep over the recorded window.
 * dJdq: [n_vertices][3] host doubles, dJ/dq at the window's end (read only).
 * grads: 6 host doubles written with dJ/d(alpha_1, alpha_2, alpha_3, k_V,
 *   eps_lo, tau).  dJdq0: NULL or [n_vertices][3] host doubles, written with
 *   dJ/dq at the window's start.
 * May be called again (another J over the same window).  The context must not
 * have been stepped since iblb_adjoint_record (IBLB_E_STATE), and is left at
 * the window's end.  IBLB_E_INVAL for a null pointer, IBLB_E_STATE with no
 * recording, IBLB_E_UNSTABLE / IBLB_E_DEVICE from the device. */
int iblb_adjoint_backward(iblb_ctx *ctx, const double *dJdq, double *grads, double *dJdq0);
/* Frees the recording (also done by iblb_destroy). */
int iblb_adjoint_release(iblb_ctx *ctx);
/* Host-side, FP64: the sphere fit of the contact-angle measurement
 * (iblb_contact_angle, method 0) and its gradient.  Least-squares sphere
 * |p|^2 = 2 c.p + k through the vertices at least `exclude` from the wall
 * plane z = z_wall (wall 0: lower, the droplet above; 1: upper), coordinates
 * relative to the selected vertices' x-y centroid and to the plane.  Writes
 * h = height of the fitted sphere's top above the plane (NULL to skip), r2 =
 * R^2 - c_z^2 (the squared contact radius when positive; NULL to skip) and
 * their gradients with respect to q (NULL to skip; [nv][3], zero for vertices
 * left out), differentiating the normal equations.  q: [nv][3] host doubles.
 * IBLB_E_INVAL for bad arguments, IBLB_E_STATE with fewer than 4 vertices
 * selected or singular normal equations. */
int iblb_sphere_fit_grad(int32_t nv, const double *q, int32_t wall, double z_wall, double exclude, double *h,
                         double *r2, double *dh_dq, double *dr2_dq);

#ifdef __cplusplus
}
#endif
#endif /* IBLB_H */
