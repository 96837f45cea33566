/*
 * grid.h -- C ABI of the MI355X batched gradient-of-forward-dynamics library.
 *
 * The calls follow the problem statement of GRiD (arXiv 2109.06976): a robot model
 * plus arrays of joint positions q, velocities qd and torques tau go in; the joint
 * accelerations qdd, the inverse mass matrix M^-1 and the gradients dqdd/dq and
 * dqdd/dqd come out (Sec. IV-B, the last item of the feature list:
 * dqdd/du = -M^-1 dRNEA(q, qd, qdd)/du, and dqdd/dtau = M^-1).
 *
 * Conventions shared by every call
 *   - Bodies are numbered 0..n-1 with parent[i] < i; parent -1 is the fixed base
 *     (Sec. III-B). Outputs use the caller's numbering.
 *   - Joints move along a unit axis a_i of their joint frame (+z unless `axis` is given):
 *     a revolute joint rotates about it (S_i = (a_i, 0), q_i in radians), a prismatic joint
 *     slides along it (S_i = (0, a_i), q_i in metres), and a fixed joint does not move
 *     (GRiD's three joint types, Sec. IV). The joint transform is iX_lambda(q_i) =
 *     X_J(q_i) * X_T,i with X_J the coordinate rotation by q_i about a_i (revolute) or
 *     the translation by q_i a_i (prismatic), and X_T,i given by tree_rot (rotation from
 *     the parent frame to the joint frame) and tree_pos (the joint origin in parent
 *     coordinates) (Sec. III-B). The library rotates every body frame so that its joint
 *     axis becomes z before generating the kernel (a change of body coordinates that
 *     leaves every joint-space quantity unchanged).
 *   - Spatial vectors are ordered [angular; linear] (Eq. 2). SI units: radians for revolute
 *     joints, metres for prismatic ones (and N m or N for tau).
 *   - Fixed base, fully actuated (B = I in Eq. 1), no external forces (F = 0).
 *   - Batched arrays are knot-major and row-major float32:
 *       q, qd, tau, qdd       [N][n]
 *       Minv, dqdd_dq, dqdd_dqd  [N][n][n],  dqdd_dq[k][i][j] = d qdd_i / d q_j at knot k.
 *     M^-1 is returned exactly symmetric.
 *   - Arithmetic is float32 throughout.
 *
 * Errors: every call returns a grid_status. Arguments are validated on the host
 * before any device work, so on error nothing has been enqueued. N = 0 is a no-op that
 * returns GRID_OK. A call takes at most GRID_MAX_KNOTS knots (2^24; a larger N is EINVAL).
 * NaN or Inf inputs are not checked and propagate to the outputs. A
 * fault of an asynchronous launch surfaces as GRID_EDEVICE at the next call that
 * synchronises. grid_last_error() returns a thread-local description of the last
 * failure on the calling thread. No C++ exception crosses this interface.
 *
 * Ownership: a grid_model owns its device constants and compiled kernels and is not
 * modified by launches, so several threads may launch with one model. A
 * grid_workspace belongs to one stream (or one thread) at a time. The caller owns all
 * input and output buffers.
 */
#ifndef GRID_H
#define GRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t grid_status;
#define GRID_OK 0
#define GRID_EINVAL (-1)        /* bad argument or model description */
#define GRID_ENOMEM (-2)        /* device or host allocation failed */
#define GRID_EDEVICE (-3)       /* HIP runtime error, no device, or a kernel fault */
#define GRID_EUNSUPPORTED (-4)  /* valid request the library does not implement */
#define GRID_ECOMPILE (-5)      /* generating or compiling the robot's kernel failed */
#define GRID_EBUSY (-6)         /* a request larger than the server's admission budget */
#define GRID_ETIMEDOUT (-7)     /* the wait ended before the request completed */
#define GRID_ECANCELED (-8)     /* the server was destroyed before the request ran */

/* The largest knot count N of one call (and max_knots of a workspace): 2^24. */
#define GRID_MAX_KNOTS (1 << 24)

#define GRID_JOINT_REVOLUTE 0
#define GRID_JOINT_PRISMATIC 1
#define GRID_JOINT_FIXED 2

/*
 * A fixed joint welds its body to the parent. The library merges every such body into its
 * nearest ancestor with a movable (revolute or prismatic) joint (its inertia re-expressed
 * there; dropped if welded to the base) and attaches the children to that ancestor through
 * the composed transform (a fixed joint's transform is X_T alone). All arrays of every call
 * then hold the movable joints only, in increasing body order: n_dof of them
 * (grid_model_info reports n_dof); at least one joint must be movable.
 */
typedef struct grid_model_desc {
    int32_t n;                   /* number of bodies, 1..32 (and of movable joints, when
                                    joint_type is NULL) */
    const int32_t* parent;       /* [n], -1 <= parent[i] < i */
    const int32_t* joint_type;   /* [n] GRID_JOINT_REVOLUTE, GRID_JOINT_PRISMATIC or
                                    GRID_JOINT_FIXED; NULL for all revolute */
    const double* axis;          /* [n][3] unit joint axis in the joint frame (norm within
                                    1e-6 of 1, normalised); NULL = +z for every joint */
    const double* tree_rot;      /* [n][3][3] E_T, row-major, parent frame -> joint frame */
    const double* tree_pos;      /* [n][3] joint origin in parent coordinates (m) */
    const double* mass;          /* [n] link mass (kg), > 0 */
    const double* com;           /* [n][3] centre of mass in the body frame (m) */
    const double* inertia_com;   /* [n][6] xx yy zz xy xz yz about the centre of mass (kg m^2) */
    double gravity[3];           /* gravity in base coordinates (m/s^2) */
} grid_model_desc;

typedef struct grid_model_s* grid_model;
typedef struct grid_workspace_s* grid_workspace;

typedef struct grid_timing {
    float h2d_ms;      /* host -> device copy of q, qd, tau */
    float kernel_ms;   /* device compute */
    float d2h_ms;      /* device -> host copy of the four outputs */
    float total_ms;    /* first copy start to last copy end */
} grid_timing;

/* Name of a status code (static string). */
const char* grid_status_string(grid_status s);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* grid_last_error(void);

/*
 * Validate a model description and obtain the robot's kernel on `device`: the library
 * writes the topology out as compile-time structures and the constants as literals
 * (Sec. IV-C code generation), compiles it for gfx950 or loads the code object from
 * the kernel cache (directory GRID_KERNEL_CACHE, else the package's _kcache), and
 * loads it on the device.
 * flags: reserved, must be 0. On success *out owns the loaded code object until
 * grid_model_destroy. Errors: EINVAL (bad description, an axis not of unit length),
 * EUNSUPPORTED (n > 32), ECOMPILE, EDEVICE, ENOMEM.
 */
grid_status grid_model_create(const grid_model_desc* desc, int32_t device, uint32_t flags,
                              grid_model* out);

/* Release a model (NULL is accepted). Waits for nothing: the caller must not destroy a
 * model that still has launches in flight. */
grid_status grid_model_destroy(grid_model m);

/* n (the movable joints the arrays hold), bytes moved per knot by the host-pointer call
 * (inputs + outputs), and the number of wavefront lanes one knot occupies (summed over its
 * base branches). Any pointer may be NULL. */
grid_status grid_model_info(grid_model m, int32_t* n, size_t* io_bytes_per_knot,
                            int32_t* lanes);

/* A 64-bit FNV-1a hash of the machine code of the model's two loaded code objects (every
 * kernel generated for the robot, then the role-split kernel's own module: their .text,
 * .rodata and .note sections), so that measurements taken on a kernel can be matched to the
 * exact machine code they ran; the same robot, sources and compiler give the same hash, and
 * an edit that leaves the machine code alone (a comment) does not change it.
 * Errors: EINVAL (NULL argument). */
grid_status grid_model_code_hash(grid_model m, uint64_t* hash);

/*
 * The batched path, one fused kernel launch (per knot and per branch of the tree at
 * the fixed base: transforms, RNEA, M, its sparse factorisation, qdd, RNEA at qdd,
 * dRNEA forward/backward, -M^-1 dtau and M^-1). All pointers are device
 * pointers in the layouts above; `stream` is a hipStream_t (NULL = default stream).
 * Asynchronous: returns after the launch is enqueued. Errors: EINVAL (N < 0, a NULL
 * pointer with N > 0, N > GRID_MAX_KNOTS), EDEVICE (launch failure).
 */
grid_status grid_fd_grad(grid_model m, int32_t N, const float* q, const float* qd,
                         const float* tau, float* qdd, float* Minv, float* dqdd_dq,
                         float* dqdd_dqd, void* stream);

/*
 * Vector-Jacobian product of forward dynamics, qdd = FD(q, qd, tau), for reverse-mode
 * differentiation: given the outputs of grid_fd_grad and an output cotangent gbar [N][n],
 *   qbar = (dqdd/dq)^T gbar,  qdbar = (dqdd/dqd)^T gbar,  taubar = M^-1 gbar
 * (dqdd/dtau = M^-1 is symmetric; Sec. IV-B). Device pointers, [N][n] vectors and
 * [N][n][n] matrices as above; asynchronous on `stream`. Errors: EINVAL (N < 0, NULL
 * pointers, N > GRID_MAX_KNOTS), EDEVICE.
 */
grid_status grid_fd_vjp(grid_model m, int32_t N, const float* dqdd_dq, const float* dqdd_dqd,
                        const float* Minv, const float* gbar, float* qbar, float* qdbar,
                        float* taubar, void* stream);

/*
 * Workspace for the host-pointer and staged calls: device buffers, pinned host staging
 * and the staged pipeline's intermediates for up to max_knots knots, plus a private
 * stream and events.
 */
grid_status grid_workspace_create(grid_model m, int32_t max_knots, grid_workspace* out);
grid_status grid_workspace_destroy(grid_workspace ws);

/*
 * Host-pointer variant (the paper's CPU-side call, Sec. IV-A): copies q, qd, tau to
 * the device, runs grid_fd_grad, copies the outputs back and waits. Host buffers are
 * ordinary (pageable) memory in the layouts above; they are staged through the
 * workspace's pinned buffers. `timing` (may be NULL) receives HIP-event times of the
 * three phases. Errors: EINVAL (N > max_knots of the workspace, NULL pointers, a
 * workspace made for another model), EDEVICE.
 */
grid_status grid_fd_grad_host(grid_model m, grid_workspace ws, int32_t N, const float* q,
                              const float* qd, const float* tau, float* qdd, float* Minv,
                              float* dqdd_dq, float* dqdd_dqd, grid_timing* timing);

/*
 * The workspace's pinned host buffers, for callers that write the inputs and read the outputs
 * in place (no pageable staging; the I/O of Sec. V-B without host-side copies). For a call on
 * N knots the arrays are packed one after the other in the layouts above:
 *   in  = q [N][n] | qd [N][n] | tau [N][n]
 *   out = qdd [N][n] | Minv [N][n][n] | dqdd_dq [N][n][n] | dqdd_dqd [N][n][n]
 * Both are sized for max_knots and belong to the workspace (valid until it is destroyed).
 * Errors: EINVAL (a NULL argument).
 */
grid_status grid_workspace_host_buffers(grid_workspace ws, float** in, float** out);

/*
 * The host call on the workspace's pinned buffers: copies the inputs of N knots from `in` to
 * the device, runs grid_fd_grad's fused kernel, copies the outputs into `out` and waits.
 * pieces = 1: one copy each way around one launch, timed per phase (timing as in
 * grid_fd_grad_host). pieces > 1: the batch is split into that many contiguous ranges of knots
 * whose copies and launches go to two streams in turn, so that one range's copies overlap
 * another's kernel; only timing->total_ms (first copy start to last copy end) is set. Each
 * launch runs the build grid_fd_grad picks for its own knot count, and its results equal
 * grid_fd_grad's on those knots bit for bit. Errors: EINVAL (N > max_knots of the workspace, a
 * workspace of another model, pieces outside 1..64), EDEVICE.
 */
grid_status grid_fd_grad_pinned(grid_model m, grid_workspace ws, int32_t N, int32_t pieces,
                                grid_timing* timing);

/*
 * The host call on the workspace's pinned buffers without copy-engine transfers (the I/O of
 * Sec. V-B as part of the device work): the fused kernel reads q, qd, tau of N knots from the
 * pinned input buffer through the device's mapping of it, and the outputs reach the pinned
 * output buffer (layouts as in grid_workspace_host_buffers) either
 *   GRID_IO_COPY_KERNEL  through the workspace's device buffer and one copy kernel with 16-byte
 *                        stores into the mapping, or
 *   GRID_IO_DIRECT       straight from the fused kernel's own stores into the mapping.
 * Waits for the results. timing (may be NULL: no events are then recorded): kernel_ms = the
 * fused kernel with its input reads, d2h_ms = the copy kernel (0 for DIRECT), total_ms = both;
 * h2d_ms = 0. Results equal
 * grid_fd_grad's on the same inputs bit for bit. Errors: EINVAL (NULL, a workspace of another
 * model, N > its max_knots, an unknown mode), EUNSUPPORTED (the runtime maps no pinned buffer
 * into the device's address space), EDEVICE.
 */
#define GRID_IO_COPY_KERNEL 0
#define GRID_IO_DIRECT 1
grid_status grid_fd_grad_mapped(grid_model m, grid_workspace ws, int32_t N, int32_t out_mode,
                                grid_timing* timing);

/*
 * The plain staged pipeline, for comparison with the fused launch: the same steps in
 * five launches on `stream` (transforms + RNEA -> c; M and its factor -> M^-1;
 * qdd; RNEA at qdd + dRNEA -> dtau/du; -M^-1 dtau/du), each intermediate going through
 * the workspace in device memory. Device pointers as in grid_fd_grad; N <= max_knots of
 * the workspace. Results equal grid_fd_grad's up to float rounding. Errors: as
 * grid_fd_grad, plus EINVAL for a workspace of another model or too small.
 */
grid_status grid_fd_grad_staged(grid_model m, grid_workspace ws, int32_t N, const float* q,
                                const float* qd, const float* tau, float* qdd, float* Minv,
                                float* dqdd_dq, float* dqdd_dqd, void* stream);

/*
 * For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): grid_fd_grad_staged without a workspace. The five
 * stage kernels keep their intermediates in the library's own static device array of
 * GRID_NOALLOC_SCRATCH_BYTES (one per device, held until the process ends; its address is
 * taken when the first model on that device is created). The call allocates nothing. Same
 * arguments, layouts and results as grid_fd_grad_staged (bit for bit), asynchronous on
 * `stream`. The array is shared by every call on the device and keeps the last call's
 * contents: calls that overlap in time on one device race and must be ordered by the caller
 * (one stream, or events). Errors: EINVAL (NULL model, N < 0, a NULL data pointer with N > 0,
 * N times the model's per-knot scratch above GRID_NOALLOC_SCRATCH_BYTES; the message states
 * the limit in knots), EDEVICE.
 */
#define GRID_NOALLOC_SCRATCH_BYTES (16u << 20)
grid_status grid_fd_grad_staged_noalloc(grid_model m, int32_t N, const float* q,
                                        const float* qd, const float* tau, float* qdd,
                                        float* Minv, float* dqdd_dq, float* dqdd_dqd,
                                        void* stream);

/*
 * Code generation without a device: write the generated HIP source for a model (its
 * topology as compile-time structures, its constants as float literals) into buf (len
 * in: capacity, out: bytes needed including the terminating NUL; buf may be NULL to
 * query), or compile it into the kernel cache. Used by the build step and by tests.
 * A model has two code objects: every kernel, and the role-split fused kernel (the build
 * grid_fd_grad picks for small batches) alone, compiled with an instruction-level-
 * parallelism schedule. grid_codegen_source returns the first, or with
 * GRID_CODEGEN_PIPE_MODULE the second; grid_codegen_precompile (flags 0) compiles both.
 * Errors: as grid_model_create's description checks; EINVAL if buf is too small or a flag
 * bit is unknown.
 */
#define GRID_CODEGEN_PIPE_MODULE (1u << 16)
grid_status grid_codegen_source(const grid_model_desc* desc, uint32_t flags, char* buf,
                                size_t* len);
grid_status grid_codegen_precompile(const grid_model_desc* desc, uint32_t flags);

/* ------------------------------------------------------------------ mixed batches
 *
 * A batch item is one model's knots with their own device buffers (layouts as in
 * grid_fd_grad). Items of different robots and uneven N run as independent launches.
 */
typedef struct grid_item {
    grid_model model;
    int32_t N;
    const float *q, *qd, *tau;
    float *qdd, *Minv, *dqdd_dq, *dqdd_dqd;
} grid_item;

typedef struct grid_graph_s* grid_graph;

/* Launch every item's fused kernel on `stream`, one after the other. Errors: as
 * grid_graph_create's item checks. */
grid_status grid_fd_grad_batch(const grid_item* items, int32_t count, void* stream);

/* Capture the items into one hipGraph (their kernels as a chain of kernel nodes, in item
 * order), instantiate it, and return it. All models must be on one device. Errors: EINVAL
 * (NULL, count < 1 or > 64, N < 0 or > GRID_MAX_KNOTS), EDEVICE. */
grid_status grid_graph_create(const grid_item* items, int32_t count, grid_graph* out);

/* Replay the graph on `stream` (one launch call for the whole mixed batch). */
grid_status grid_graph_launch(grid_graph g, void* stream);

/* Point the graph at new items (other N, other buffers; same count): the graph is
 * re-captured and the executable updated in place, or re-instantiated if the update is
 * refused. */
grid_status grid_graph_update(grid_graph g, const grid_item* items, int32_t count);

grid_status grid_graph_destroy(grid_graph g);

/* ------------------------------------------------------------------ one launch, several robots
 *
 * The whole path of grid_fd_grad (Sec. IV: RNEA, dRNEA, M^-1 and dFD = -M^-1 dID, fused) for
 * a table of items of different robots and uneven N in ONE kernel launch. A mixed module is
 * compiled for a fixed list of robot models (at most 16); it holds the fused kernel build that
 * runs each base branch of a knot on one workgroup of role-split wavefronts (the build
 * grid_fd_grad picks for small batches), instantiated for every branch of every robot. A launch
 * splits its grid into segments, one per (item, branch): the workgroups of item 0's branches
 * first, then item 1's, and so on; each workgroup finds its segment in a table passed with the
 * kernel arguments. Results are those of that build run on each item alone.
 */
typedef struct grid_mixed_s* grid_mixed;

typedef struct grid_mixed_item {
    int32_t robot;      /* index into the descs the module was created from */
    int32_t N;          /* knots, >= 0 (0: the item is skipped) */
    const float *q, *qd, *tau;                  /* device, layouts as in grid_fd_grad */
    float *qdd, *Minv, *dqdd_dq, *dqdd_dqd;     /* device, written for the item's N knots */
} grid_mixed_item;

/* Validate `count` (1..16) robot descriptions, generate and compile (or take from the kernel
 * cache) their common module, and load it on `device`, together with each robot's own modules
 * (as grid_model_create; the per-robot mode below). The descriptions are read during the
 * call only. Errors: EINVAL (a description invalid, as grid_model_create), ECOMPILE, EDEVICE,
 * EUNSUPPORTED (not a gfx950 device). */
grid_status grid_mixed_create(const grid_model_desc* descs, int32_t count, int32_t device,
                              grid_mixed* out);

/* Launch the items (1..16, any robot of the module, in any order, a robot more than once) on
 * `stream`, in the mode grid_mixed_tune chose for a batch of this size (one kernel when
 * untuned; see the modes below). Items must not share output buffers. At most 64 (item, branch)
 * segments per launch (an item has as many branches as its robot has bodies on the fixed
 * base). Errors: EINVAL (NULL, a robot index out of range, N < 0 or > GRID_MAX_KNOTS, a NULL
 * data pointer of an item with N > 0, too many segments), EDEVICE. Nothing is launched when
 * every N is 0. */
grid_status grid_mixed_launch(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                              void* stream);

/*
 * The three ways a mixed batch can run (the heterogeneous-batch choice the module's tuner
 * makes with each measured):
 *   GRID_MIXED_ONE_LAUNCH   one kernel, one workgroup per block of knots of a segment;
 *   GRID_MIXED_PERSISTENT   one kernel whose workgroups (as many as the device holds at once)
 *                           stride over the blocks, the segments of the largest branches
 *                           first; each block's arithmetic is the one-launch form's;
 *   GRID_MIXED_PER_ROBOT    one launch per item on its robot's own module, with the build
 *                           grid_fd_grad picks for the item's N (robots whose kernels need
 *                           fewer registers keep their own occupancy).
 * The first two give bitwise the same outputs (the three-role build of grid_fd_grad run on
 * each item alone); the third gives the outputs of the build the robot's tuning picks.
 */
#define GRID_MIXED_ONE_LAUNCH 0
#define GRID_MIXED_PERSISTENT 1
#define GRID_MIXED_PER_ROBOT 2

/* grid_mixed_launch in a given mode. Errors: as grid_mixed_launch, EINVAL for an unknown
 * mode. */
grid_status grid_mixed_launch_mode(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                                   int32_t mode, void* stream);

/*
 * One mixed launch captured in a hipGraph (the uneven mix of robots and knot counts as one
 * replayable launch): `mode` as above, or -1 for the mode grid_mixed_launch picks for this
 * batch size at capture time. The result is a grid_graph: replay it with grid_graph_launch,
 * free it with grid_graph_destroy (before the mixed module). grid_mixed_graph_update
 * re-captures it for other items (any count 1..16; the executable is updated in place or
 * re-instantiated). Outputs equal those of grid_mixed_launch_mode in the same mode. Errors: as
 * grid_mixed_launch, EINVAL for an unknown mode, or for grid_mixed_graph_update on a graph
 * that grid_graph_create made (and grid_graph_update on one made here), EDEVICE.
 */
grid_status grid_mixed_graph_create(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                                    int32_t mode, grid_graph* out);
grid_status grid_mixed_graph_update(grid_graph g, const grid_mixed_item* items, int32_t count);

/*
 * Tune each robot's own model for the knot counts it has among the items (grid_tune, so that
 * the per-robot mode runs the builds that tuning picks), then time the three modes on these
 * items (3 warm-up and 20 timed launches per trial, median of 5 trials, HIP events on a
 * stream of the library's; the items' outputs are written) and keep
 * the fastest for launches of this size: from then on grid_mixed_launch runs a batch of B
 * blocks in the mode tuned for the smallest tuned size >= B (the largest beyond; one launch
 * when nothing is tuned). *chosen (may be NULL) receives the mode; us (may be NULL) receives
 * the three median times per launch in microseconds, indexed by mode. Errors: as
 * grid_mixed_launch, EINVAL when the items hold no knots, EDEVICE.
 */
grid_status grid_mixed_tune(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                            int32_t* chosen, float* us);

grid_status grid_mixed_destroy(grid_mixed mx);

/* The generated source of a mixed module and its compilation into the kernel cache, without
 * a device (buffer protocol as grid_codegen_source). */
grid_status grid_mixed_source(const grid_model_desc* descs, int32_t count, char* buf,
                              size_t* len);
grid_status grid_mixed_precompile(const grid_model_desc* descs, int32_t count);

/*
 * Jacobians of the discrete-time dynamics of one semi-implicit Euler step of length dt,
 * qd' = qd + dt qdd(q, qd, tau), q' = q + dt qd', the form trajectory optimisation uses
 * (Sec. I: dFD feeds the optimiser's knot points). From the outputs of grid_fd_grad:
 *   A[k] = d(q', qd')/d(q, qd) = [[1 + dt^2 Dq, dt 1 + dt^2 Dqd], [dt Dq, 1 + dt Dqd]]
 *   B[k] = d(q', qd')/dtau     = [[dt^2 M^-1], [dt M^-1]]
 * with Dq = dqdd/dq, Dqd = dqdd/dqd; A is [N][2n][2n] and B [N][2n][n], row-major, device
 * pointers, asynchronous on `stream`. Errors: EINVAL (N < 0, dt not positive and finite,
 * NULL pointers, N > GRID_MAX_KNOTS, 6 N n^2 > 2^31 - 256), EDEVICE.
 */
grid_status grid_dt_jacobians(grid_model m, int32_t N, float dt, const float* dqdd_dq,
                              const float* dqdd_dqd, const float* Minv, float* A, float* B,
                              void* stream);

/* ------------------------------------------------------------------ the other algorithms
 *
 * The paper's other rigid-body algorithms on the same batched layout (Sec. IV-B), one
 * kernel launch each, per knot and per base branch; device pointers, `stream` a
 * hipStream_t, asynchronous. Arrays: q, qd, qdd, tau [N][n]; Minv, dtau_dq, dtau_dqd
 * [N][n][n] row-major (dtau_dq[k][i][j] = d tau_i / d q_j). Errors: EINVAL (N < 0, a
 * required pointer NULL with N > 0, N > GRID_MAX_KNOTS), EDEVICE (launch failure).
 */

/* Inverse dynamics tau = ID(q, qd, qdd) by RNEA with gravity (Sec. IV-B, Eq. 1). */
grid_status grid_id(grid_model m, int32_t N, const float* q, const float* qd, const float* qdd,
                    float* tau, void* stream);

/* Forward dynamics qdd = M^-1 (tau - RNEA(q, qd, 0)) (Sec. IV-B, Eq. 1). */
grid_status grid_fd(grid_model m, int32_t N, const float* q, const float* qd, const float* tau,
                    float* qdd, void* stream);

/* The mass-matrix inverse M(q)^-1 (Sec. IV-B), exactly symmetric. */
grid_status grid_minv(grid_model m, int32_t N, const float* q, float* Minv, void* stream);

/* M(q)^-1 by a chosen route, to compare the paper's direct inverse with the factorisation
 * the fused kernels use (Sec. IV-B lists the direct inverse of Carpentier and Mansard):
 *   GRID_MINV_QUAD         grid_minv itself (quad layout: columns of M, L^T L, solves);
 *   GRID_MINV_LANE_LTL     one lane per knot and branch: M by composite rigid bodies,
 *                          M = L^T L along ancestor paths, B triangular solve pairs;
 *   GRID_MINV_LANE_DIRECT  one lane per knot and branch: the direct articulated-body
 *                          recursion (zero velocity and gravity, the identity as its right-hand
 *                          sides; inward articulated inertias, outward rows of M^-1).
 * All three write Minv [N][n][n] row-major, exactly symmetric (upper triangle mirrored),
 * device pointers, asynchronous on `stream`. Errors: EINVAL (unknown route, N < 0, NULL
 * pointer with N > 0, N > GRID_MAX_KNOTS), EDEVICE. */
#define GRID_MINV_QUAD 0
#define GRID_MINV_LANE_LTL 1
#define GRID_MINV_LANE_DIRECT 2
grid_status grid_minv_route(grid_model m, int32_t N, const float* q, float* Minv, int32_t route,
                            void* stream);

/* The gradient of inverse dynamics at the given qdd: dtau/dq and dtau/dqd (Sec. IV-B,
 * Algorithm 1 and its backward pass). */
grid_status grid_id_grad(grid_model m, int32_t N, const float* q, const float* qd,
                         const float* qdd, float* dtau_dq, float* dtau_dqd, void* stream);

/* The vector-Jacobian product of forward dynamics without forming its Jacobians: from
 * q, qd and the forward result qdd = FD(q, qd, tau), and a cotangent gbar [N][n],
 *   taubar = M^-1 gbar,  qbar = -(dtau/dq)^T taubar,  qdbar = -(dtau/dqd)^T taubar
 * (the same values as grid_fd_vjp, Sec. IV-B: dqdd/du = -M^-1 dRNEA/du). The transposed
 * products come from one reverse sweep over RNEA, O(n) per knot instead of the n^2
 * columns: with the virtual displacement u_i = X_i u_lambda + S_i taubar_i,
 * taubar^T tau = sum_i u_i . f_i, differentiated backwards through the sweep. Writes
 * [N][n] vectors qbar, qdbar, taubar. */
grid_status grid_fd_vjp_adjoint(grid_model m, int32_t N, const float* q, const float* qd,
                                const float* qdd, const float* gbar, float* qbar, float* qdbar,
                                float* taubar, void* stream);

/* ------------------------------------------------------------------ autotuning
 *
 * The fused kernel exists in eight builds. Build 0 spreads each spatial vector over the
 * four lanes of a quad and gives every derivative column its own quad (few instructions per
 * lane: low latency). Builds 1, 2, 3 give every column one lane that runs the shared
 * sweeps itself (fewest instructions per knot: the highest throughput), allowed 1, 2 or 4
 * resident wavefronts per SIMD. Build 4 is build 0 split over three roles on different
 * wavefronts of a workgroup (RNEA and dtau/du at qdd = 0; M, qdd and the qdd-dependent part
 * of dtau/dq; M^-1), the shortest dependency chain. Build 5
 * gives each (knot, branch) problem
 * one lane (no repeated work: the fewest instructions per knot, the longest latency). Build 6
 * is build 5 with four lanes per problem that share the columns of M^-1 and the derivative
 * columns (each repeats the rest): four times the wavefronts of build 5 for the same batch.
 * Build 7 is the same with two lanes per problem (twice the wavefronts of build 5).
 * Untuned, a batch runs build 4 while its wavefronts fit one per SIMD of the device, build 1
 * beyond, build 6 from 64 knots per compute unit and build 5 from 128, except for a robot
 * with a base branch of more than 8 bodies: build 4 up to 4096 knots, build 6 beyond.
 * grid_tune times each build on the model's
 * device for every knot count in Ns (synthetic inputs, HIP events, median of repeats),
 * keeps the fastest per count, and from then on grid_fd_grad uses, for a batch of N
 * knots, the choice made for the smallest tuned count >= N (the largest otherwise).
 * chosen[i] (may be NULL) receives the build index (0..7) picked for Ns[i]. The
 * result is also appended to `table_path` (may be NULL) as one JSON line keyed by the
 * hash of the model's code objects (grid_model_code_hash), so a table is applied only to
 * the machine code it was tuned on; grid_model_create reads the file named by GRID_TUNE_TABLE,
 * if set, and applies the last matching line. Errors: EINVAL, ENOMEM, EDEVICE.
 */
grid_status grid_tune(grid_model m, const int32_t* Ns, int32_t count, const char* table_path,
                      int32_t* chosen);

/* Apply a tuning table from memory: a batch of N knots runs build builds[i] for the
 * smallest Ns[i] >= N (builds[count - 1] beyond the largest). Ns must be ascending
 * (1..2^22, 1 <= count <= 64); count = 0 returns the model to the untuned choice.
 * EUNSUPPORTED if a build index is outside 0..7, EINVAL otherwise. */
grid_status grid_tune_apply(grid_model m, const int32_t* Ns, const int32_t* builds,
                            int32_t count);

/* The build (0..7) a batch of N >= 1 knots runs with the model's current tuning. */
grid_status grid_build_for(grid_model m, int32_t N, int32_t* build);

/* ------------------------------------------------------------------ serving
 *
 * A server accepts dFD requests (a model index, N knots, host arrays) from any number of
 * client threads and runs them with continuous batching: a scheduler thread admits
 * requests while the device bytes they need fit the budget, packs the admitted requests of
 * one model into the next free batch context (up to max_batch_knots knots per launch), and
 * issues H2D copy, one fused launch and D2H copy on that context's stream. Several batch
 * contexts per model are in flight at once, so requests that arrive while others run are
 * packed into the next launch (the batching policy of the config decides how long a batch
 * waits for company) and their work overlaps on the device. Each context has a thread that
 * waits for its batch on the device and copies the outputs to the callers' buffers; no
 * thread of the server spins while it waits (condition variables, and an event wait that
 * polls only for the first tens of microseconds). Model constants live in the models' code
 * objects on the device. Each knot's arithmetic does not depend on the other knots of its
 * launch, so a request's results are the same alone and in a mix.
 */
typedef struct grid_server_s* grid_server;

#define GRID_SERVER_PER_REQUEST 1   /* baseline: one staged (plain) launch per request */
/* Batches read their inputs from, and write their outputs to, the contexts' pinned staging
 * through the device's mapping of it (no copy-engine H2D and D2H; as grid_fd_grad_mapped with
 * GRID_IO_DIRECT). The loadgen's H2D and D2H phases are then empty. */
#define GRID_SERVER_MAPPED_IO 2
/* A request whose seven arrays all lie inside pinned host ranges registered with
 * grid_server_pin_range and that forms a batch alone is computed in place: the kernel reads
 * the caller's inputs and writes the caller's outputs through the device's mapping, with no
 * staging copy in and no copy-out (the loadgen's copy-out phase is then empty). Requests
 * packed with others, and other arrays, take the staged path. */
#define GRID_SERVER_DIRECT_PINNED 4

typedef struct grid_server_config {
    size_t device_budget_bytes;  /* admission budget of in-flight request bytes (inputs+outputs) */
    int32_t max_batch_knots;     /* knots per launch, >= the largest request */
    int32_t contexts_per_model;  /* batch contexts (streams) per model, >= 1 */
    uint32_t flags;              /* 0, or any of GRID_SERVER_PER_REQUEST, GRID_SERVER_MAPPED_IO,
                                    GRID_SERVER_DIRECT_PINNED */
    /* Batching policy. While a model has no batch in flight, its admitted requests launch as
     * soon as a context is free. While one is in flight, the next batch of that model waits
     * until it holds min_batch_knots knots or its oldest request has waited batch_window_us
     * microseconds, so that requests arriving meanwhile share a launch. 0 and 0: never wait.
     * Ignored with GRID_SERVER_PER_REQUEST. */
    int32_t batch_window_us;     /* 0 .. 1000000 */
    int32_t min_batch_knots;     /* 0 .. max_batch_knots */
} grid_server_config;

typedef struct grid_server_stats {
    uint64_t submitted, completed, canceled;
    uint64_t knots_completed;
    uint64_t launches;           /* device launches issued (fused, or staged pipelines) */
    uint64_t max_inflight_bytes;
    uint64_t inplace_launches;   /* launches run in place on a request's own pinned arrays */
} grid_server_stats;

/* Create a server over `count` models (all on one device; the models must outlive the
 * server). Errors: EINVAL (bad config, NULL models, models on different devices), ENOMEM,
 * EDEVICE. */
grid_status grid_server_create(const grid_model* models, int32_t count,
                               const grid_server_config* config, grid_server* out);

/* Queue a request. Host buffers in the layouts of grid_fd_grad; inputs are read and
 * outputs written by the server until grid_server_wait reports completion, so they must
 * stay valid until then. *ticket identifies the request. Errors: EINVAL (bad index, N < 1,
 * N > max_batch_knots, NULL pointers), EBUSY (the request alone exceeds the admission
 * budget), ECANCELED (the server is shutting down). */
grid_status grid_server_submit(grid_server s, int32_t model_index, int32_t N, const float* q,
                               const float* qd, const float* tau, float* qdd, float* Minv,
                               float* dqdd_dq, float* dqdd_dqd, uint64_t* ticket);

/* Wait up to timeout_us microseconds (< 0: no limit) for a request. GRID_OK once its outputs
 * are written (the ticket is then released); ETIMEDOUT if still running (the ticket stays
 * valid); ECANCELED if the server dropped it; EINVAL for an unknown ticket. */
grid_status grid_server_wait(grid_server s, uint64_t ticket, int64_t timeout_us);

grid_status grid_server_stats_get(grid_server s, grid_server_stats* out);

/* Stop accepting requests, finish the ones already launched, cancel the queued ones (their
 * waiters get ECANCELED) and release everything. Waiters must not call into the server
 * after this returns. */
grid_status grid_server_destroy(grid_server s);

/*
 * Register (unregister) a range of pinned host memory for in-place requests on a
 * GRID_SERVER_DIRECT_PINNED server: a request runs in place when each of its seven arrays lies
 * inside a registered range and its batch holds it alone. The range must lie inside one
 * allocation of pinned host memory mapped into the device (checked with the runtime's pointer
 * queries when registering; EINVAL otherwise). The caller keeps the memory allocated until it
 * unregisters the range and no request using it is in flight. At most 64 ranges per server;
 * grid_server_unpin_range takes the pointer the range was registered with. Errors: EINVAL.
 */
grid_status grid_server_pin_range(grid_server s, const void* p, size_t bytes);
grid_status grid_server_unpin_range(grid_server s, const void* p);

/* Open-loop load generator for measurement: Poisson arrivals at `rate_per_s` for
 * `warmup_s + duration_s` seconds; each request picks model k with probability
 * model_prob[k] and N uniformly in [n_min, n_max]; inputs are drawn once per model
 * (q ~ U[-pi, pi], qd ~ N(0,1), tau ~ N(0,25)) and requests take windows of them.
 * Latency = completion (outputs in host memory) - scheduled arrival; requests arriving
 * in the warm-up are not counted. */
typedef struct grid_loadgen_config {
    double rate_per_s, duration_s, warmup_s;
    const double* model_prob;    /* [count of server models], sums to 1 */
    int32_t n_min, n_max;
    uint64_t seed;
    int32_t pinned;              /* nonzero: the clients' arrays are pinned host memory mapped
                                    into the device (hipHostMalloc) rather than ordinary memory */
} grid_loadgen_config;

/* Where a request's latency goes (microseconds): queue = scheduled arrival to the launch of
 * its batch (admission, waiting for a context or the batch window); h2d, kernel, d2h = the
 * batch's device phases (HIP events); complete = launch to the server seeing the batch done
 * (device queueing, the three phases and the wake-up); copyout = copying its outputs from the
 * pinned staging into the caller's buffers. */
typedef struct grid_latency_split {
    double queue_us, h2d_us, kernel_us, d2h_us, complete_us, copyout_us;
} grid_latency_split;

#define GRID_LOADGEN_MODELS 8       /* models with their own latency percentiles below */

typedef struct grid_loadgen_result {
    uint64_t requests, knots;    /* completed in the measured window */
    double seconds;              /* measured window */
    double p50_us, p90_us, p99_us, max_us, mean_us;
    double offered_rate_per_s;
    double requests_per_launch;  /* over the whole run */
    grid_latency_split p50, p99; /* per phase, over the measured requests */
    /* per model (index < GRID_LOADGEN_MODELS; 0 for a model without requests) */
    uint64_t model_requests[GRID_LOADGEN_MODELS];
    double model_p50_us[GRID_LOADGEN_MODELS], model_p99_us[GRID_LOADGEN_MODELS];
} grid_loadgen_result;

grid_status grid_server_loadgen(grid_server s, const grid_loadgen_config* cfg,
                                grid_loadgen_result* out);

#ifdef __cplusplus
}
#endif
#endif /* GRID_H */
