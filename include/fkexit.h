/*
 * fkexit.h -- C ABI of the MI355X (gfx950) library for the backward
 * Feynman-Kac scheme of the exit-time probability (Yang, Zhang,
 * del-Castillo-Negrete, Stoyanov: "A Feynman-Kac based numerical method for
 * the exit time probability of a class of transport problems").
 *
 * Problem (paper Section 2, Eq. (e1)-(e2)): an SDE dX = b(t,X) dt + sigma dW
 * on a Cartesian grid over a box, sigma = sqrt(2 D) I, an exit region, a
 * tensor Gauss-Hermite rule of Q* nodes per dimension, a time step dt and a
 * step count N.  Output: the fields u^n, n = N..0, of Scheme 1 (Section 3.1),
 *   u^N = chi;  u^n_j = sum_q w_q * (z_jq exits ? 1 : I[u^{n+1}](z_jq)),
 *   z_jq = x_j + b(t_n, x_j) dt + sigma sqrt(2 dt) a_q            (Eq. (e31))
 * with I the tensor cubic Hermite interpolant whose nodal slopes are the PCHIP
 * slopes of Eq. (e300) (value and first-derivative basis functions, Eq. (Lag11)),
 * i.e. u^n = Q Psi^n F^n u^{n+1} of Eq. (e36) plus the exit mass.  For an
 * autonomous problem u^n = P(T - t_n, x); in general u^n_j is the probability
 * of exiting in (t_n, T] from x_j at t_n.
 *
 * Conventions shared by every call:
 *  - All calls return fk_status; nothing is thrown across the ABI.  On error
 *    fk_last_error() (thread-local) holds a message and outputs are undefined.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are host memory owned by the caller.  The library never
 *    allocates device memory: every device buffer it uses lives in the caller's
 *    workspace (fk_plan_set_workspace) or in the caller's outputs.
 *  - stream is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously; outputs are valid after the stream has synchronised.
 *  - Field layout: one field is the concatenation of the instances of a plan,
 *    instance i at node offset off[i] (fk_plan_layout), each instance in
 *    C order over its grid (axis d-1 fastest).  Element type is double for
 *    FK_PREC_F64 and float for FK_PREC_F32.
 *  - A plan is not thread-safe; distinct plans are.
 */
#ifndef FKEXIT_H
#define FKEXIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FK_ABI_VERSION 2
#define FK_MAX_DIM 3
#define FK_MAX_THETA 8
/* Bytes of the library's static device buffer used by fk_forward_static. */
#define FK_STATIC_SCRATCH_BYTES (64u << 20)

typedef enum {
    FK_OK = 0,
    FK_ERR_ARG = -1,          /* invalid argument */
    FK_ERR_UNSUPPORTED = -2,  /* valid request outside what this build implements */
    FK_ERR_WORKSPACE = -3,    /* workspace missing or too small */
    FK_ERR_HIP = -4,          /* HIP runtime error */
    FK_ERR_NONFINITE = -5,    /* non-finite parameter, state or result */
    FK_ERR_STATE = -6         /* call out of order */
} fk_status;

/* Drift b(t, x); theta = (coef[0..np-1], D) are the differentiable parameters.
 *  FK_COEF_CONST       b = (coef[0], .., coef[d-1]);                 np = d
 *  FK_COEF_CELLULAR2D  stream function psi = A sin(pi (x + eps sin(omega t))) sin(pi y),
 *                      b = (-dpsi/dy, dpsi/dx), coef = (A, eps, omega); np = 3
 *                      (cellular flow of Section 4.2, the paper's sign convention)
 *  FK_COEF_ABC3D       b = f(t) (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x),
 *                      f(t) = 1 + amp sin t, coef = (A, B, C, amp); np = 4
 *  FK_COEF_ROLLS2D     the paper's own 2D example (Section 4.2, Eq. (ex3)): b = Pe v,
 *                      v_1 = -pi cos(pi y) (sin(n x) + e(t) cos(n x)),
 *                      v_2 = n sin(pi y) (cos(n x) - e(t) sin(n x)), e(t) = eps cos(omega t)
 *                      (2n Rayleigh-Benard rolls on x in [-pi, pi], periodic, exit
 *                      through y = 0, 1 with a box region); coef = (Pe, eps, omega, n);
 *                      np = 3 (n, a count, is not differentiated)
 *  FK_COEF_RUNAWAY3D   the runaway-electron model of Section 4.3, Eq. (ex32d): state
 *                      (p, xi, r), drift and diagonal diffusion both depend on the node
 *                      (sigma = (sqrt(2 C_A(p)), sqrt(2 C_B(p))/p sqrt(1 - xi^2),
 *                      sqrt(2 D(r, p))); D of fk_problem is not used); coef = (E, tau, Z,
 *                      delta, nu_ee, v_T, r_D, W, Delta_p, V_0, D_0, t_*, That_0, That_f,
 *                      Ttilde, m c^2); t_* > 0: the thermal-quench model of Section 4.3
 *                      (coef[0] is then E_0).  Forward calls only (no adjoint) */
enum { FK_COEF_CONST = 0, FK_COEF_CELLULAR2D = 1, FK_COEF_ABC3D = 2, FK_COEF_ROLLS2D = 3,
       FK_COEF_RUNAWAY3D = 4 };

/* Face kinds of the box (fk_problem.face[a][side], side 0 the low face):
 * FK_FACE_EXIT1 (default): a point on or beyond the face exits with value 1;
 * FK_FACE_EXIT0: it exits with value 0 (absorbed without counting);
 * FK_FACE_REFLECT: it is mirrored back into the domain, z -> lo + (lo - z).
 * Exit nodes hold their face's value for every n; at a corner the lowest axis
 * decides (low face before high face), then the ball.  Plans with a face other
 * than FK_FACE_EXIT1 (and FK_COEF_RUNAWAY3D plans) run the fused form and the
 * forward calls only, in the thread-per-node step layouts (fk_options
 * .step_kernel 0, 1 or 3; 4 falls back to 1) or the lane-group one (2, and
 * with FK_HERMITE_R2). */
enum { FK_FACE_EXIT1 = 0, FK_FACE_EXIT0 = 1, FK_FACE_REFLECT = 2 };

/* Exit region (paper Section 2: D is an open box; a disc or ball target, such
 * as the cellular-flow workload's disc, adds a ball).  FK_REGION_BOX: a point exits when a coordinate on a non-periodic
 * axis is <= the first or >= the last node.  FK_REGION_BALL: it also exits
 * when |z - center|^2 >= radius^2 (evaluated as sum over axes of
 * (z_i - c_i)*(z_i - c_i), axis 0 first, no fused multiply-add).  Nodes that
 * lie in the exit region hold u = 1 for every n. */
enum { FK_REGION_BOX = 0, FK_REGION_BALL = 1 };

/* FK_PREC_F64: everything in FP64.
 * FK_PREC_F32: landing points, exit tests, cells and in-cell positions in FP64
 * (classification needs it); Hermite weights, gathers, accumulation and the
 * stored fields in FP32. */
enum { FK_PREC_F64 = 0, FK_PREC_F32 = 1 };

/* Interpolant (Section 3.1.2, a tensor product of cubic Hermite bases).
 * FK_HERMITE_R1: values and first derivatives (the nodal slopes of Eq. (e300)
 * along each axis; the column blocks of Psi^n in Eq. (e34)).
 * FK_HERMITE_R2: also the mixed derivatives, the twist field of an axis set
 * composed from the one-dimensional rule in increasing axis order
 * (u_xy = D_y(D_x u)); exact on tensor products of cubics given exact fields.
 * In 3D the four twist fields (axis sets {0,1}, {0,2}, {1,2}, {0,1,2}) sit in
 * a second record per node in the workspace.  R2 is built for d = 1 (the
 * same as R1), 2 and 3, the fused form and the forward pass (fk_forward,
 * fk_forward_from, fk_step, fk_forward_horizons); in 3D with the
 * thread-per-node step only (fk_options.step_kernel 0, 1 or 3; a gh_q with
 * such a kernel compiled) and exit-1 faces.  Other combinations are
 * FK_ERR_UNSUPPORTED. */
enum { FK_HERMITE_R1 = 0, FK_HERMITE_R2 = 1 };

/* FK_FORM_FUSED: matrix-free step (landing, weights and contraction in one
 * kernel).  FK_FORM_ELL: the step operator A_n = Q Psi^n (Eq. (e36)) is
 * assembled each step into ELL-like storage and then applied as a sparse
 * matrix-vector product, the paper's own GPU formulation (Section 3.2.1).
 * Internally each row is stored as the dense box of nodes its landing cells
 * can cover (columns implicit in the box origin), its values in 16-byte
 * blocks of consecutive box nodes of one field; fk_export_ell writes the
 * plain (column, value) layout. */
enum { FK_FORM_FUSED = 0, FK_FORM_ELL = 1 };

typedef struct {
    int n;                /* number of nodes, >= 4 */
    const double *nodes;  /* host: n strictly increasing coordinates (copied) */
    int periodic;         /* nonzero: nodes[n-1] is the image of nodes[0] */
} fk_axis;

typedef struct {
    int d;                 /* 1..3 */
    fk_axis ax[FK_MAX_DIM];
    int coef_kind;         /* FK_COEF_* */
    double coef[16];       /* drift parameters, see FK_COEF_* */
    double D;              /* diffusion coefficient, sigma = sqrt(2 D) I, D >= 0 */
    int region_kind;       /* FK_REGION_* */
    double center[FK_MAX_DIM];
    double radius;
    int gh_q;              /* Q*, Gauss-Hermite nodes per Brownian dimension */
    double dt;             /* > 0 */
    int n_steps;           /* N >= 1 */
    double t0;             /* step n evaluates coefficients at t0 + n dt */
    int force_f64;         /* nonzero in an FK_PREC_F32 plan: this instance is
                              computed entirely in FP64 (its fields are still
                              delivered and taken in FP32); ignored in FP64
                              plans.  fk_probe_precision picks the instances
                              whose FP32 result misses a tolerance. */
    int face[FK_MAX_DIM][2];  /* FK_FACE_* per non-periodic axis, low and high face */
} fk_problem;

typedef struct {
    int precision;   /* FK_PREC_* */
    int form;        /* FK_FORM_* */
    int use_graph;   /* nonzero: capture the N-step loop once and replay it */
    int ckpt_every;  /* adjoint checkpoint interval K (0 = no adjoint storage) */
    int block;       /* threads per workgroup, 0 = library default */
    int step_kernel; /* fused step layout: 0 = auto; 1 = one thread per node;
                        2 = a lane group per node over the tensor points (any gh_q);
                        3 = Q* lanes per node over the outermost axis;
                        4 = separable box form for nodes whose landing points
                        cannot reach a ball boundary (footprint up to 8 nodes
                        per axis; d >= 2 on affine axes), one thread per node
                        for the others.  1, 3 and 4 exist for d=1: gh_q
                        2..8,10,12,16; d=2: 2..8; d=3: 2..6
                        (FK_ERR_UNSUPPORTED otherwise).  auto picks 4 for 3D
                        plans with many active nodes, 1 for other large plans,
                        3 for small ones, 2 when the others are not compiled
                        for gh_q; fk_tune measures them instead.  Plans with
                        faces other than exit-1 (or the runaway model) take 4
                        as 1, and with FK_HERMITE_R2 always run 2 */
    int columns;     /* fk_forward_horizons: most columns one launch of the
                        FK_FORM_ELL product takes (1..4; 0 = 1); the workspace
                        holds that many record planes */
    int hermite;     /* FK_HERMITE_R1 (default) | FK_HERMITE_R2 */
} fk_options;

typedef struct {
    int n_inst;
    int d;
    int gh_q;
    int n_quad;             /* Q = Q*^d */
    int n_steps;
    int n_theta;            /* theta per instance (drift params + D) */
    int64_t n_nodes;        /* nodes of all instances */
    int64_t n_active;       /* active nodes of all instances */
    int64_t ell_width;      /* ELL row width (FK_FORM_ELL), else 0; the widest instance */
    size_t workspace_bytes;
    int64_t ell_entries;    /* ELL entries, sum over instances of width x active rows (block padding not counted) */
    int64_t adj_point_nodes;  /* adjoint (ckpt_every > 0): active nodes transposed per landing point */
    int64_t adj_box_nodes;    /* adjoint: active nodes transposed in separable box form */
} fk_plan_info;

typedef struct fk_plan fk_plan;

/* Result of fk_tune: the fastest step layout and the measured mean duration
 * of one backward step (slope pass + step pass) per layout, in milliseconds
 * (0 where the layout was not timed: not compiled for the plan, or the same
 * lists as one already timed). */
typedef struct {
    int step_kernel;          /* value for fk_options.step_kernel */
    double ms_per_step[5];    /* indexed by step_kernel 0..4 (0 unused) */
} fk_tune_result;

/* Message of the last error on this thread ("" if none).  Library plumbing:
 * no passage of the paper defines it. */
const char *fk_last_error(void);

/* FK_ABI_VERSION of the loaded library (plumbing, as fk_last_error). */
int fk_version(void);

/* Gauss-Hermite rule for the normalised Gaussian weight pi^{-1/2} e^{-xi^2}
 * (paper Eq. (expec)-(quad)): q nodes ascending and weights summing to 1,
 * symmetric about 0.  host outputs of length q; 1 <= q <= 64. */
fk_status fk_gh_rule(int q, double *nodes, double *weights);

/* Validates n_inst >= 1 problems and builds a plan (host work only).  The
 * inputs are the paper's problem statement: the SDE's drift and diffusion
 * (Section 2, Eq. (e1)), the exit region (Section 2; the ball is this
 * library's addition), the Cartesian grid S (Section 3.1.2), the quadrature
 * order Q* (Eq. (expec)-(quad)), dt and N (Section 3.1, Scheme 1).  The plan
 * classifies every node (active, exit, periodic image: the terminal condition
 * chi of Scheme 1) and builds the work lists of the step kernels.  All
 * instances must share d, gh_q, dt, n_steps, t0, coef_kind and region_kind;
 * grids and parameters may differ (batched, uneven grids).  Host arrays are
 * copied.  opt may be NULL (defaults: F64, fused, no graph, no adjoint).
 * Errors: FK_ERR_ARG (invalid problem: its message names the instance and the
 * field), FK_ERR_UNSUPPORTED (a step layout not compiled for gh_q; instances
 * forced to FP64 in an FK_FORM_ELL plan).  An FP32 plan with instances forced
 * to FP64 computes them in an internal FP64 plan that reads and writes this
 * plan's fields (every call below handles both, in stream order). */
fk_status fk_plan_create(const fk_problem *probs, int n_inst, const fk_options *opt,
                         fk_plan **out);

/* Frees the plan's host memory and its captured graph; the caller's
 * workspace is not touched (the caller frees it).  NULL is ignored. */
void fk_plan_destroy(fk_plan *p);

/* Sizes of a plan (host output): node and active-node counts, Q = Q*^d
 * (Eq. (quad) over d dimensions), workspace bytes.  FK_ERR_ARG on NULL. */
fk_status fk_plan_get_info(const fk_plan *p, fk_plan_info *info);

/* Packed field layout (host outputs): node_offset[n_inst + 1] (instance i
 * owns nodes node_offset[i] .. node_offset[i+1]-1 of every field) and
 * active_count[n_inst] (its active nodes, the rows of A_n of Eq. (e36)). */
fk_status fk_plan_layout(const fk_plan *p, int64_t *node_offset, int64_t *active_count);

/* Attaches caller-owned device memory of at least workspace_bytes bytes
 * (256-byte aligned) and uploads the plan's tables into it; synchronises
 * stream before returning.  The memory must stay valid until the plan is
 * destroyed or another workspace is set.  Plumbing (the library allocates no
 * device memory itself); it holds the fields of Scheme 1's ping-pong, the
 * records [u, F^n u] of Eq. (e36) and, for the adjoint, the checkpoints.
 * Errors: FK_ERR_ARG (NULL or misaligned), FK_ERR_WORKSPACE (too small). */
fk_status fk_plan_set_workspace(fk_plan *p, void *dev_ptr, size_t bytes, void *stream);

/* Backward pass of Scheme 1 (Section 3.1; matrix form Eq. (e36)-(e37)):
 * from u^N = chi, u^n = A_n u^{n+1} + exit mass for n = N-1 .. 0.  u_out
 * (device, caller-owned) receives n_snap fields, u_out[s] = u^{snap_steps[s]}
 * (0 <= snap_steps[s] <= N, host array).  A non-finite value in a produced
 * field is reported by fk_check_flags.  Errors: FK_ERR_STATE (no workspace),
 * FK_ERR_ARG (snapshot outside [0, N], null output with n_snap > 0),
 * FK_ERR_HIP. */
fk_status fk_forward(fk_plan *p, const int *snap_steps, int n_snap, void *u_out,
                     void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): fk_forward without
 * a caller workspace.  The plan's tables, the ping-pong fields and the node
 * records live in one static device array of FK_STATIC_SCRATCH_BYTES bytes
 * per device, held until the process ends; the call allocates and frees
 * nothing.  Same outputs as fk_forward (u_out device, caller-owned; snapshot
 * rules alike) and the same kernels, without a graph and without adjoint
 * checkpoints; a plan workspace, if set, is neither needed nor touched.  The
 * tables are copied from host memory on every call (the array keeps the last
 * call's contents, and every plan on the device shares it), so calls that
 * overlap on one device race: serialise them (one stream, or
 * synchronisation).  Non-finite values are not reported (fk_check_flags reads
 * the workspace's flags).  Errors: FK_ERR_WORKSPACE when the plan's forward
 * workspace exceeds FK_STATIC_SCRATCH_BYTES, FK_ERR_ARG as fk_forward,
 * FK_ERR_UNSUPPORTED (a plan with instances forced to FP64), FK_ERR_HIP. */
fk_status fk_forward_static(fk_plan *p, const int *snap_steps, int n_snap, void *u_out,
                            void *stream);

/* Algorithm 1 (Section 3.2): the exit probabilities p^m of Eq. (e37) for
 * several horizons in one backward sweep.  horizons (host, n_h >= 1 entries,
 * each in [1, N], repeats allowed): horizon m is the time t0 + m dt.  Column h
 * starts as chi; at sweep index n = M .. 1 (M the largest horizon) every
 * column with horizons[h] >= n takes one step with the coefficients at
 * t0 + (n-1) dt, the same operator A_{n-1} for all of them, so that
 * u_out[h] = P(exit by t0 + horizons[h] dt | X_{t0} = x) (device, n_h fields,
 * caller-owned, also the working storage).  FK_FORM_ELL plans assemble
 * A_{n-1} once per sweep index and apply it to up to fk_options.columns
 * columns per launch (a sparse matrix times a dense block of columns); fused
 * plans run the matrix-free step once per active column.  Errors:
 * FK_ERR_ARG (horizon outside [1, N], null arguments), FK_ERR_UNSUPPORTED
 * (plans with instances forced to FP64), FK_ERR_HIP. */
fk_status fk_forward_horizons(fk_plan *p, const int *horizons, int n_h, void *u_out,
                              void *stream);

/* Backward pass of Scheme 1 (Section 3.1) resumed from a caller state
 * u_start = u^{start_step} (device, one field, read only); snapshots with
 * snap_steps[s] <= start_step.  Errors as fk_forward. */
fk_status fk_forward_from(fk_plan *p, const void *u_start, int start_step,
                          const int *snap_steps, int n_snap, void *u_out, void *stream);

/* One step of Scheme 1 (Section 3.1), u^n = Q Psi^n F^n u^{n+1} + exit mass
 * (Eq. (e36)), from an arbitrary state u_next (device, one field) into u_out
 * (device, one field).  Exit nodes of the result are 1, periodic images copy
 * their originals.  Errors: FK_ERR_ARG (n outside [0, N-1], null field). */
fk_status fk_step(fk_plan *p, int n, const void *u_next, void *u_out, void *stream);

/* The step operator A_n = Q Psi^n of Eq. (e34)-(e36) as a linear map, and its
 * transpose (the reverse sweep's scatter, Eq. (e36) transposed), on caller
 * data: a test hook for the adjoint identity <A_n x, y> = <x, A_n^T y>.
 * Columns: the (d + 1) fields [u; g_0; ..; g_{d-1}] (values and nodal slopes
 * along each axis, the column blocks of Psi^n), each one packed field, field
 * f at element offset f * n_nodes.  Rows: the active nodes; the exit mass
 * (the landing points that leave, value 1) is not part of A_n.
 *   transpose = 0: x = (d + 1) fields (device, read), y = one field (device,
 *     written): y_j = sum_q w_q I[x](z_jq) over the inside landing points of
 *     active node j, y = 0 on every other node.  The coefficient tables of
 *     step n are used (times t0 + n dt); the slopes are taken from x, not from
 *     Eq. (e300).  FK_FORM_ELL plans assemble and apply A_n, fused plans
 *     apply it matrix-free.
 *   transpose = 1: x = one field (device, read; its values off the active
 *     nodes are ignored), y = (d + 1) fields (device, written) = A_n^T x.
 *     Needs a plan created with ckpt_every > 0 (FK_ERR_STATE otherwise).
 * Uses the plan's ping-pong and record buffers: adjoint checkpoints stay
 * valid.  Errors: FK_ERR_ARG (n outside [0, N-1], null field),
 * FK_ERR_STATE, FK_ERR_UNSUPPORTED (a plan with instances forced to FP64),
 * FK_ERR_HIP. */
fk_status fk_apply_step(fk_plan *p, int n, int transpose, const void *x, void *y, void *stream);

/* Landing points of step n (Eq. (e31)) located in the grid, for instance
 * inst (device outputs, caller-owned): cells[Ja][Q][d] int32, the cell
 * max{k : x_k <= z} of each coordinate clamped to [0, n-2] (Section 3.1.2;
 * -1 where the landing point exits), and exit_flags[Ja][Q] uint8 (1: the point
 * lies in the exit region, Section 2), active nodes in increasing linear
 * index, tensor points in lexicographic order (last axis fastest).  Errors:
 * FK_ERR_ARG (inst or n out of range, null output). */
fk_status fk_export_cells(fk_plan *p, int inst, int n, int *cells,
                          unsigned char *exit_flags, void *stream);

/* Assembled step operator A_n = Q Psi^n of step n (Eq. (e34)-(e36); the
 * paper's own GPU formulation assembles it, Section 3.2.1), FK_FORM_ELL plans
 * only (FK_ERR_STATE otherwise): for every active
 * node (all instances, packed order) a row of ell_width (column, value) pairs,
 * column = (d + 1) * node + field (field 0: u, field 1 + a: slope along a,
 * node = packed node index), padding has value 0; exit_mass[row] = sum of
 * w_q over exiting landing points.  Layout: cols[k * n_active + row]
 * (column-major ELL), vals likewise, element type of the plan precision. */
fk_status fk_export_ell(fk_plan *p, int n, int *cols, void *vals, void *exit_mass,
                        void *stream);

/* Reads and clears the device status flags (synchronises stream); plumbing,
 * no passage of the paper defines it.  *flags bit 0: a non-finite value was
 * produced since the last check (returns FK_ERR_NONFINITE); bit 1: a landing
 * cell fell outside an assembled row box (FK_ERR_UNSUPPORTED). */
fk_status fk_check_flags(fk_plan *p, void *stream, int *flags);

/* Adjoint of the whole backward pass of Scheme 1 (the reverse sweep of the
 * matrix form Eq. (e36): lam^{n+1} = F^n' ^T (Q Psi^n)^T lam^n, plus the
 * derivatives of the landing points Eq. (e31) and of the Hermite weights with
 * respect to theta), the exit classification of landing points held fixed.
 * lam0 (device, one field) = dJ/du^0.  Outputs: grad (device, double,
 * n_inst * FK_MAX_THETA, overwritten; entry [i * FK_MAX_THETA + k] is dJ/dtheta_k
 * of instance i for k < n_theta, theta = (coef[0..np-1], D)) and, if lamN is
 * not NULL, dJ/du^N (device, one field; zero on exit nodes).
 * u is checkpointed every ckpt_every steps (fk_options) and recomputed.
 * With ckpt_every > 0, fk_forward stores these checkpoints on its way, and an
 * fk_adjoint enqueued after it on the same stream starts from them instead of
 * running the forward pass again (same values: the pass is deterministic);
 * any other stream, or a workspace change, makes fk_adjoint recompute them. */
fk_status fk_adjoint(fk_plan *p, const void *lam0, double *grad, void *lamN,
                     void *stream);

/* Autotuner for batched plans (an engineering addition; the paper has no
 * counterpart): builds a trial plan for each step layout
 * (fk_options.step_kernel 1..4) of the problems with n_steps replaced by
 * trial_steps (the cost of a step does not depend on n), runs its backward
 * pass twice on stream with the caller's other options, and returns the
 * layout with the shortest second run in out (host).  workspace (device,
 * 256-byte aligned, caller-owned, contents destroyed) must hold the largest
 * trial plan: the workspace_bytes of a plan over the full problems suffices.
 * Synchronises stream.  Errors: FK_ERR_ARG (bad arguments), FK_ERR_WORKSPACE
 * (workspace too small for a trial plan), plan-creation and HIP errors. */
fk_status fk_tune(const fk_problem *probs, int n_inst, const fk_options *opt, int trial_steps,
                  void *workspace, size_t workspace_bytes, void *stream, fk_tune_result *out);

/* Measurement hook (hardware, no passage of the paper): the lane-level rate of
 * LDS floating-point atomic adds of the device, FP64 (f32 = 0) or FP32
 * (f32 = 1), with conflict-free addresses: 2048 workgroups x 256 lanes x
 * 4096 adds each, the best of three timed launches after a warm-up, HIP
 * events on stream.  *adds_per_s (host) receives the rate.  workspace
 * (device, caller-owned, >= 16 KiB) receives one value per workgroup.
 * The transposed step accumulates in FP64 LDS atomics; this is its ceiling.
 * Synchronises stream.  Errors: FK_ERR_ARG, FK_ERR_WORKSPACE, FK_ERR_HIP. */
fk_status fk_probe_lds_atomics(int f32, double *adds_per_s, void *workspace, size_t workspace_bytes,
                               void *stream);

/* Precision probe for FP32 plans (the precision split is an engineering
 * addition; the error of every FP32 result against FP64 is what it bounds):
 * runs the backward pass of the problems once in FP64 and once with
 * FK_PREC_F32 (fused form, opt's graph use and step layout) and returns per
 * instance diff[i] = max over the instance's nodes of |u^0 (FP64) - u^0 (FP32)|.
 * With a cotangent lam0 (device, double, one field of the problems' packed
 * layout; NULL: fields only) it also runs both adjoints (checkpoints every 32
 * steps; the FP32 one with lam0 rounded to FP32) and returns grad_diff[i] =
 * max_k |dJ/dtheta_k (FP64) - (FP32)| / max_k |dJ/dtheta_k (FP64)| (if
 * grad_diff is not NULL).  force_f64[i] = (diff[i] > tol / 2) or, with lam0,
 * (grad_diff[i] > grad_tol / 2) (host outputs of length n_inst), ready for
 * fk_problem.force_f64: an instance whose scheme amplifies the FP32 rounding
 * beyond half a tolerance is then computed in FP64 (the other half is left for
 * the FP64 evaluation's own rounding).  force_f64 of the inputs is ignored.
 * With workspace == NULL only *bytes_needed is written (device bytes for the
 * same call with a cotangent); otherwise workspace (device, 256-byte aligned,
 * caller-owned, contents destroyed) must hold that many.  Synchronises stream.
 * Errors: FK_ERR_ARG, FK_ERR_WORKSPACE, plan-creation and HIP errors. */
fk_status fk_probe_precision(const fk_problem *probs, int n_inst, const fk_options *opt,
                             double tol, const double *lam0, double grad_tol, void *workspace,
                             size_t workspace_bytes, void *stream, size_t *bytes_needed,
                             int *force_f64, double *diff, double *grad_diff);

/* Measurement hook (Scheme 1, Section 3.1, timed; the cost model of
 * Section 3.2.1 names assembly and product; instances forced to FP64 are not
 * timed): runs one backward pass from chi without a graph on
 * stream, with HIP events around every kernel launch, and returns the mean
 * duration in milliseconds per launch of each pass kind in ms[4] (host):
 * [0] slope pass, [1] fused step pass, [2] ELL assembly, [3] ELL product
 * (0 for kinds the plan's form does not launch); counts[4] (host) receives the
 * number of launches timed.  Synchronises stream. */
fk_status fk_profile_pass(fk_plan *p, double *ms, int *counts, void *stream);

/* Measurement hook for the adjoint (the reverse sweep of Eq. (e36), timed):
 * runs fk_adjoint(p, lam0, grad, NULL,
 * stream) with HIP events around every kernel group of the reverse sweep and
 * returns the mean duration in milliseconds per step of each group in ms[5]
 * (host): [0] slope pass of u^{n+1}, [1] transposed step of the nodes
 * handled per landing point (the scatter of A_n^T lam^n and the
 * theta-gradient), [2] transposed slope pass with the image fold, [3] forward
 * step recomputed inside a checkpoint segment, [4] transposed step of the
 * nodes handled in separable box form; counts[5] (host) receives the number of
 * steps timed.
 * Arguments and errors as fk_adjoint.  Synchronises stream. */
fk_status fk_profile_adjoint(fk_plan *p, const void *lam0, double *grad, double *ms,
                             int *counts, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FKEXIT_H */
