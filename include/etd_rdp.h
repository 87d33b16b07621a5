/*
 * etd_rdp.h -- C ABI of the MI355X (gfx950) ETD-RDP-IF reaction-diffusion
 * stepper.
 *
 * The library advances   u_t = D Lap(u) + F(u)   (Section 2 of Asante-Asamani,
 * Kleefeld and Wade, "A second-order exponential time differencing scheme for
 * non-linear reaction-diffusion systems with dimensional splitting") with the
 * second-order L-stable ETD-RDP-IF scheme: the d-dimensional frame of
 * Section 6 (eq. donedone for d = 3, eq. done for d = 2, its general-d form
 * for d = 4 .. ETD_MAX_DIM; for d = 1 the unsplit ETD-RDP, eq. finalle).  Every split factor
 * (I + (k/gamma) A_i)^{-1}, gamma in {1, 3, 4}, is applied as a batch of exact
 * 1-D line solves (Section 7) fused with the pointwise reaction.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arithmetic is IEEE FP64 unless a context is created with another
 *    etd_scheme_t.precision (FP32, or complex FP64 for complex species).
 *  - A state is a contiguous, caller-owned device array of s * N doubles
 *    (floats, or interleaved complex pairs, for the other precisions),
 *    N = n[0] * ... * n[d-1], laid out species-planar:
 *        u[sigma][i_d]...[i_2][i_1],  i_1 (axis 1) fastest.
 *    Axis i is the axis of the paper's A_i (eq. Ai): axis 1 carries B_p in the
 *    innermost spatial Kronecker position, axis d in the outermost one.  The
 *    scheme treats axis d differently from the others (its T/S solves come
 *    after f*), so this ordering is part of the contract.  The paper's own
 *    vector puts the species index innermost; that is a permutation of the
 *    same data.
 *  - Boundary conditions are homogeneous, one per axis (Section 2):
 *    Dirichlet, Neumann or periodic, with the grids of Example 1.
 *  - The library never allocates device memory.  Device data (tables and
 *    carried intermediates) live in a caller-provided workspace whose size
 *    etd_rdp_workspace_bytes() reports; it must be 256-byte aligned.
 *  - Every call returns an int status: ETD_OK (0) or a negative ETD_ERR_*.
 *    No C++ exception crosses the ABI.  Kernel faults surface at the caller's
 *    next synchronisation; launch errors are reported as ETD_ERR_HIP and the
 *    HIP code is kept in the context (etd_rdp_last_hip_error).
 *  - A context may be used by one host thread / one stream at a time.
 *  - Streams are passed as void* (a hipStream_t, or NULL for the null stream).
 */
#ifndef ETD_RDP_H_
#define ETD_RDP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ETD_OK 0
#define ETD_ERR_ARG (-1)          /* invalid argument (see etd_rdp_init)    */
#define ETD_ERR_UNSUPPORTED (-2)  /* valid problem the library does not run */
#define ETD_ERR_WORKSPACE (-3)    /* workspace NULL, too small, misaligned  */
#define ETD_ERR_HIP (-4)          /* a HIP runtime call failed              */
#define ETD_ERR_INTERNAL (-5)     /* a table self-check failed              */

/* ---- boundary conditions (Section 2, Example 1) ------------------------ */
#define ETD_BC_DIRICHLET 0
#define ETD_BC_NEUMANN 1
#define ETD_BC_PERIODIC 2

/* ---- reaction models F(u) --------------------------------------------- */
/* params[] meaning per model; F is evaluated at (u + shift).               */
#define ETD_RX_LINEAR 0       /* F = C u, C = params[0..s*s) row-major      */
#define ETD_RX_ENZYME 1       /* s=1: F = -u/(1+u)            (Section 8.1) */
#define ETD_RX_BRUSSELATOR 2  /* s=2: params a,b: a-(b+1)u+u^2v, bu-u^2v    */
#define ETD_RX_GRAY_SCOTT 3   /* s=2: params F,kappa: -uv^2+F(1-u),
                                 uv^2-(F+kappa)v                            */
#define ETD_RX_SCHNAKENBERG 4 /* s=2: params a,b,gamma: g(a-u+u^2v),
                                 g(b-u^2v)                                  */
#define ETD_RX_CGL 5          /* s=2 (Re,Im), alpha=0: params beta:
                                 u - (1+i beta) u |u|^2        (Section 8.3) */
/* Models of one complex species (ETD_PRECISION_C128 contexts only):        */
#define ETD_RX_CGL_Z 6        /* s=1 complex, D = 1 + i alpha: params beta:
                                 u - (1+i beta) u |u|^2        (Section 8.3) */
#define ETD_RX_NLS_Z 7        /* s=1 complex, D = i (cubic Schroedinger
                                 i u_t + Lap u = q u): params B, C:
                                 F = -i (B + C |u|^2) u        (Section 8.4) */

/* ---- time-stepping scheme --------------------------------------------- */
#define ETD_SCHEME_RDP 0   /* ETD-RDP-IF, second order (Section 6)          */
#define ETD_SCHEME_ETD1 1  /* predictor only: ETD1-IF with Pade-(0,1),
                              first order (eq. duhamel3t)                    */

#define ETD_MAX_DIM 8
#define ETD_MAX_SPECIES 2
#define ETD_MAX_PARAMS 16

typedef struct etd_grid_t {
  int32_t d;                  /* spatial dimension: 1 to ETD_MAX_DIM         */
  int32_t s;                  /* number of species: 1 or 2                   */
  int64_t n[ETD_MAX_DIM];     /* unknowns per axis, n[0] = axis 1 (fastest)  */
  double h[ETD_MAX_DIM];      /* spacing per axis; 0 selects the unit-domain
                                 default of Example 1: Dirichlet 1/(n+1),
                                 Neumann 1/(n-1), periodic 1/n               */
} etd_grid_t;

typedef struct etd_reaction_t {
  int32_t model;                    /* ETD_RX_*                              */
  int32_t field;                    /* 1: a per-cell field b(x) is added to
                                       ETD_RX_NLS_Z's B (Section 8.4's 2-D
                                       example), set with etd_rdp_set_field;
                                       0 otherwise (other models: must be 0) */
  double params[ETD_MAX_PARAMS];    /* model parameters (see ETD_RX_*)       */
  double shift[ETD_MAX_SPECIES];    /* F evaluated at u + shift              */
} etd_reaction_t;

/* Line lengths.  A line of n rows is cut into at most 64 chunks solved by
 * the lanes of one wavefront.  Where some m <= 8 divides n with n/m <= 64
 * the chunks are equal ("regular" lines).  Any other n <= 1024 (n prime or
 * with no such divisor, or n > 512) is a "general" line: m = ceil(n/64)
 * rows per chunk, C = ceil(n/m) chunks, the last one shorter when m does
 * not divide n.  The forward step runs general lines with kernels of their
 * own (one line per wavefront); the reverse-mode step, the single solves
 * and the ensembles take regular lines only.
 *
 * Lines per wavefront of the forward passes (etd_scheme_t.lines_per_wave).
 * A wavefront solves one grid line with up to 64 chunks, or two lines of
 * 32 chunks each when the line length is n = 32 m with 2 <= m <= 8 (fewer
 * cross-lane reduction levels per line, 32-line tiles), four lines of 16
 * chunks when n = 16 m (64-line tiles), or eight lines of 8 chunks when
 * n = 8 m (128-line tiles), again with 2 <= m <= 8.
 * Results agree with the one-line form to rounding (the chunking differs). */
#define ETD_LINES_AUTO 0   /* on passes of >= 8192 lines eight, else four,
                              else two where n allows; on passes of <= 128
                              lines two where n allows; else one               */
#define ETD_LINES_ONE 1    /* always one                                       */
#define ETD_LINES_TWO 2    /* two wherever n allows                            */
#define ETD_LINES_FOUR 4   /* four lines of 16 chunks where n = 16 m (2 <= m <=
                              8, n <= 128), else as ETD_LINES_TWO              */
#define ETD_LINES_EIGHT 8  /* eight lines of 8 chunks where n = 8 m (2 <= m <=
                              8, n <= 64), else as ETD_LINES_FOUR              */

/* Element type of the state and of the carried arrays
 * (etd_scheme_t.precision).  The line-solve tables are built and held in
 * FP64 either way; an FP32 context converts them when its kernels load them.
 * FP32 contexts step with etd_rdp_step_f32 / etd_rdp_run_pass_f32, FP32
 * ensembles with etd_rdp_batch_step_f32; the reverse-mode step, the single
 * solves and debug_passes are FP64 only (ETD_ERR_UNSUPPORTED). */
#define ETD_PRECISION_F64 0
#define ETD_PRECISION_F32 1
/* Complex species (a complex diffusion coefficient, Sections 8.3 and 8.4):
 * u holds s*N complex FP64 values as interleaved (re, im) pairs, D holds s
 * (re, im) pairs with Re D >= 0, the model is ETD_RX_CGL_Z or ETD_RX_NLS_Z
 * (and those models need this precision), shift must be 0.  Every solve is
 * a complex line solve.  Lines run one per wavefront (ETD_LINES_TWO and
 * ETD_LINES_FOUR are
 * ETD_ERR_UNSUPPORTED), with the same line lengths as real species.  Step
 * with etd_rdp_step_z /
 * etd_rdp_run_pass_z; the other entry points return ETD_ERR_ARG or
 * ETD_ERR_UNSUPPORTED for such a context. */
#define ETD_PRECISION_C128 2

typedef struct etd_scheme_t {
  int32_t scheme;                   /* ETD_SCHEME_RDP or ETD_SCHEME_ETD1     */
  int32_t lines_per_wave;           /* ETD_LINES_*; ignored by the batch API */
  int32_t precision;                /* ETD_PRECISION_*                       */
  int32_t reserved;                 /* must be 0                             */
} etd_scheme_t;

typedef struct etd_rdp_ctx etd_rdp_ctx;

/*
 * etd_rdp_init -- validate a problem and build its line-solve tables on the
 * host.  Makes no HIP call, so it runs on machines without a GPU.
 *
 *  grid  : dimension, species, sizes, spacings (above).
 *  bc    : bc[i] for axis i+1, one of ETD_BC_*.
 *  D     : s diffusion coefficients, finite and >= 0 (diagonal D, Section 2);
 *          for ETD_PRECISION_C128, s complex ones as (re, im) pairs.
 *  k     : time step, finite and > 0.
 *  scheme: NULL selects ETD_SCHEME_RDP with ETD_LINES_AUTO.
 *  rx    : reaction model and parameters; must match s.
 *  out   : receives the new context (owned by the library; free it with
 *          etd_rdp_destroy).
 *
 * Errors: ETD_ERR_ARG for a NULL pointer, d not in 1..ETD_MAX_DIM, s not in {1,2},
 * n below the minimum of its BC (Dirichlet 1, Neumann 2, periodic 3), a
 * non-finite or non-positive h or k, a negative or non-finite D, an unknown
 * model or one whose species count differs from s, lines_per_wave not one of
 * ETD_LINES_*, precision not one of ETD_PRECISION_*.  ETD_ERR_UNSUPPORTED for
 * a line length n > 1024 (longer than 64 chunks of 16 rows), complex
 * species with two, four or eight lines per wavefront.  ETD_ERR_INTERNAL if
 * a table self-check fails.
 */
int etd_rdp_init(const etd_grid_t* grid, const int32_t* bc, const double* D,
                 double k, const etd_scheme_t* scheme,
                 const etd_reaction_t* rx, etd_rdp_ctx** out);

/* Frees a context (NULL is allowed).  Device memory is the caller's. */
int etd_rdp_destroy(etd_rdp_ctx* ctx);

/*
 * Bytes of device workspace a step needs: the factor tables plus the
 * carried FP64 arrays of s*N values each (the passes' intermediates): one
 * triple (c1, c2, w) written by pass 1 and, for d >= 3, a second triple
 * written by pass 2 (six arrays for d >= 3, three in 2-D; later passes
 * alternate between the two triples, odd passes writing the first).
 */
int etd_rdp_workspace_bytes(const etd_rdp_ctx* ctx, size_t* bytes);

/*
 * etd_rdp_workspace_layout -- where pass `pass` (1..d-1) leaves its carried
 * triple (c1, c2, w): byte offsets of the three arrays inside the workspace
 * and, in strides[0..d-1], the element stride (in doubles) of axes 1..d
 * inside each species plane (species planes are N doubles apart).  Each
 * pass writes the layout the next pass reads line by line: pass 1 writes
 * axis 2 fastest, then axis 1, then axis 3 ([z][x][y]); pass 2 writes axis 3
 * fastest, then axis 2, then axis 1 ([x][y][z]).  With d >= 4 the layouts
 * are cyclic: pass p writes axis p+1 fastest, then p+2, ..., d, 1, ..., p
 * (odd passes into the first triple's arrays, even ones into the second's).
 * After a full step the
 * contents are unspecified; etd_rdp_debug_passes leaves defined values.
 * Errors: ETD_ERR_ARG (NULL pointer, pass outside 1..d-1).
 */
int etd_rdp_workspace_layout(const etd_rdp_ctx* ctx, int32_t pass,
                             size_t* off_c1, size_t* off_c2, size_t* off_w,
                             int64_t* strides);

/*
 * etd_rdp_step -- advance u in place by nsteps time steps on `stream`.
 *
 *  u        : device, s*N doubles, caller-owned, read and overwritten.
 *  ws       : device workspace of at least etd_rdp_workspace_bytes bytes,
 *             256-byte aligned; its first use (or a change of ws) uploads
 *             the tables with an asynchronous copy on `stream`.  Calls that
 *             pass the address of the last workspace reuse the tables it
 *             holds: after freeing or overwriting that buffer, call
 *             etd_rdp_forget_workspace first.
 *  nsteps   : >= 0; 0 is a no-op.
 *  stream   : hipStream_t (NULL = null stream).  The call only enqueues work;
 *             it does not synchronise.
 * Errors: ETD_ERR_ARG (NULL ctx/u, nsteps < 0), ETD_ERR_WORKSPACE,
 * ETD_ERR_HIP.
 */
int etd_rdp_step(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes,
                 int64_t nsteps, void* stream);

/*
 * etd_rdp_step_static -- etd_rdp_step without a caller workspace, for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * device array of ETD_STATIC_SCRATCH_BYTES inside the library, one per
 * device, which each device holds until the process ends; the call makes no
 * allocation.  u, nsteps and stream as etd_rdp_step; FP64 contexts only.
 *
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other host threads, other streams) race and give wrong
 * results; calls ordered on one stream do not.  The tables are uploaded
 * (an asynchronous copy on `stream`) whenever another context used the
 * array last; nothing else in it needs clearing.
 * Errors: ETD_ERR_ARG (NULL ctx/u, nsteps < 0, not an FP64 context),
 * ETD_ERR_WORKSPACE (etd_rdp_workspace_bytes of the context exceeds
 * ETD_STATIC_SCRATCH_BYTES: use etd_rdp_step), ETD_ERR_UNSUPPORTED (a
 * context with a reaction field; a device index above 63), ETD_ERR_HIP.
 */
#define ETD_STATIC_SCRATCH_BYTES (64u << 20)
int etd_rdp_step_static(etd_rdp_ctx* ctx, double* u, int64_t nsteps, void* stream);

/*
 * etd_rdp_step_f32 -- etd_rdp_step for a context created with
 * ETD_PRECISION_F32: u holds s*N floats (same layout), the carried arrays
 * are FP32 and every solve and reaction evaluation runs in FP32 arithmetic
 * (tables converted from FP64).  The workspace size is
 * etd_rdp_workspace_bytes of that context.  ETD_ERR_ARG if the context is
 * FP64 (and etd_rdp_step returns ETD_ERR_ARG for an FP32 context).
 */
int etd_rdp_step_f32(etd_rdp_ctx* ctx, float* u, void* ws, size_t ws_bytes,
                     int64_t nsteps, void* stream);

/*
 * etd_rdp_step_z -- etd_rdp_step for a context created with
 * ETD_PRECISION_C128 (Sections 8.3 and 8.4: complex diffusion coefficient).
 *  u : device, s*N complex values as 2*s*N doubles, (re, im) interleaved,
 *      16-byte aligned; otherwise the layout of etd_rdp_step.
 * The carried arrays are complex.  ETD_ERR_ARG if the context is not
 * complex or u is misaligned; other errors as etd_rdp_step.
 */
int etd_rdp_step_z(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes,
                   int64_t nsteps, void* stream);

/*
 * etd_rdp_debug_passes -- run only the first `npasses` passes (1..d) of one
 * step and stop, leaving the carried arrays in the workspace (see
 * etd_rdp_workspace_layout).  Pass 1's triple holds c1 = R_1 U,
 * c2 = R_1 f(U), w = P_1 (U + k f); pass 2's (d = 3) holds c1 = R_2 R_1 U,
 * c2 = R_2 R_1 f, w = P_2 P_1 (U + k f).
 * npasses = d is a full step (u is overwritten).  For testing each pass
 * against the oracle's intermediates.
 */
int etd_rdp_debug_passes(etd_rdp_ctx* ctx, double* u, void* ws,
                         size_t ws_bytes, int32_t npasses, void* stream);

/*
 * etd_rdp_run_pass -- run pass `pass` (1..d) of a step on its own, reading
 * and writing the same arrays as inside a full step (pass 1 reads u and
 * writes its triple, pass 2 of a 3-D step reads that and writes its own,
 * pass d reads the last triple and writes u).  For timing the kernels one
 * by one.
 */
int etd_rdp_run_pass(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes,
                     int32_t pass, void* stream);

/* etd_rdp_run_pass for an ETD_PRECISION_F32 context (u holds floats). */
int etd_rdp_run_pass_f32(etd_rdp_ctx* ctx, float* u, void* ws, size_t ws_bytes,
                         int32_t pass, void* stream);

/* etd_rdp_run_pass for an ETD_PRECISION_C128 context (u as etd_rdp_step_z). */
int etd_rdp_run_pass_z(etd_rdp_ctx* ctx, double* u, void* ws, size_t ws_bytes,
                       int32_t pass, void* stream);

/*
 * etd_rdp_set_field -- store the per-cell reaction field b (Section 8.4:
 * q = B + b(x) + C |u|^2) of a context created with etd_reaction_t.field = 1
 * in the workspace ws, on `stream`.
 *  b  : device, N doubles in the layout of one species of u; read only
 *       during the call's stream work (the library keeps two copies in ws,
 *       one in the layout each reading pass uses).
 * Steps on that context must use this workspace afterwards (another
 * workspace: ETD_ERR_ARG until set_field is called for it).
 * Errors: ETD_ERR_ARG (NULL pointers, a context without a field),
 * ETD_ERR_WORKSPACE, ETD_ERR_HIP.
 */
int etd_rdp_set_field(etd_rdp_ctx* ctx, void* ws, size_t ws_bytes, const double* b,
                      void* stream);

/*
 * etd_rdp_apply_solve -- x <- (I + (k/gamma) D_sigma A_axis)^{-1} x for a
 * single-species grid array x of N doubles (layout as one species of u),
 * gamma = 1, 3 or 4 (Section 7: the systems the scheme solves).  axis is
 * 1-based.  Exposes the line solver alone for testing.  FP64 contexts with
 * a regular line length on the axis only (ETD_ERR_UNSUPPORTED otherwise).
 */
int etd_rdp_apply_solve(etd_rdp_ctx* ctx, double* x, void* ws, size_t ws_bytes,
                        int32_t axis, int32_t sigma, int32_t gamma,
                        void* stream);

/*
 * etd_rdp_forget_workspace -- the workspace this context last used may no
 * longer hold its tables (it was freed and reallocated, possibly at the same
 * address, or written by something else).  A context uploads its tables
 * into a workspace on first use and skips the upload while later calls pass
 * the same address; it cannot tell a new buffer at an old address from the
 * old one, so the caller must call this whenever that can happen.  The next
 * call that takes a workspace uploads the tables again; a reaction field
 * must be stored again with etd_rdp_set_field.
 * Errors: ETD_ERR_ARG (NULL).
 */
int etd_rdp_forget_workspace(etd_rdp_ctx* ctx);

/*
 * etd_rdp_set_slab -- schedule of a 3-D step: with planes > 0, passes 1 and 2
 * run slab by slab, `planes` planes of axis 3 at a time (pass 2 of a slab
 * reads what pass 1 of the same slab has just written, while much of it is
 * still in the device's caches); pass 3 runs over the whole grid.  0 (the
 * default, and any value >= n[2]) runs each pass over the whole grid.  The
 * result is the same bit for bit; only the launch order changes (2 launches
 * per slab instead of 2 per step).  Contexts with a reaction field ignore it.
 * etd_rdp_get_slab reads it back.  Errors: ETD_ERR_ARG (NULL, planes < 0),
 * ETD_ERR_UNSUPPORTED (planes > 0 and d != 3).
 */
int etd_rdp_set_slab(etd_rdp_ctx* ctx, int64_t planes);
int etd_rdp_get_slab(const etd_rdp_ctx* ctx, int64_t* planes);

/*
 * etd_rdp_set_graph -- on = 1: etd_rdp_step (and _f32, _z) records the
 * launches of its nsteps steps into a HIP graph, on a private capture
 * stream, and launches the graph on the caller's stream; the graph is kept
 * and replayed while (u, ws, nsteps) stay the same (a new triple records a
 * new one).  Removes the per-launch host overhead of small problems; the
 * results are the same bit for bit.  on = 0 (the default) launches the
 * kernels one by one.  A recorded graph holds the workspace address: after
 * freeing that buffer call etd_rdp_forget_workspace, which also drops the
 * graph.  Errors: ETD_ERR_ARG (NULL, on not 0 or 1).
 */
int etd_rdp_set_graph(etd_rdp_ctx* ctx, int32_t on);

/* Record the graph of nsteps steps on (u, ws) without running it (graph
 * mode only), so that the next etd_rdp_step with the same arguments only
 * replays it.  The tables must already be in ws (a step on ws uploads
 * them).  Errors: ETD_ERR_ARG (NULL, nsteps < 1, graph mode off),
 * ETD_ERR_WORKSPACE, ETD_ERR_HIP. */
int etd_rdp_record_graph(etd_rdp_ctx* ctx, void* u, void* ws, size_t ws_bytes, int64_t nsteps);

/* Human-readable text of a status code (static storage). */
const char* etd_rdp_status_string(int status);

/* Last HIP error code seen by ctx (0 if none). */
int etd_rdp_last_hip_error(const etd_rdp_ctx* ctx);

/* Name of the kernel pass `pass` (1..d) launches, as profilers print it
 * without the namespace and arguments (for example
 * "k_mid_s<8, 2, 32, 2, true, double>"),
 * written NUL-terminated into name[0..size).  For reports.  Errors:
 * ETD_ERR_ARG (NULL, pass out of range, buffer too small). */
int etd_rdp_pass_kernel(const etd_rdp_ctx* ctx, int32_t pass, char* name,
                        size_t size);

/* Chunk length m and chunk count C = ceil(n/m) the line solver uses on an
 * axis (1-based); for tests and tuning. */
int etd_rdp_line_split(const etd_rdp_ctx* ctx, int32_t axis, int32_t* m,
                       int32_t* chunks);

/* ======================================================================
 * Reverse mode (gradients through a time step).
 *
 * The scheme is differentiated exactly, step by step, as a function of the
 * state U_n, the diffusion coefficients D and the reaction parameters theta
 * (the chain rule of the frame of Section 6, eqs. done / donedone; the paper
 * itself gives no adjoint).  A gradient vector holds etd_rdp_grad_size()
 * doubles: dL/dD_0 .. dL/dD_{s-1}, then dL/dtheta for the model's parameters
 * in params[] order (linear: C row-major; enzyme: none; Brusselator: a, b;
 * Gray-Scott: F, kappa; Schnakenberg: a, b, gamma; CGL: beta).  The shift is
 * a constant, not a parameter.
 * ====================================================================== */

/* Number of gradient entries, s + (number of reaction parameters). */
int etd_rdp_grad_size(const etd_rdp_ctx* ctx, int32_t* n);

/* Device workspace bytes etd_rdp_adjoint needs: the tables, 9 (d = 3) or 6
 * (d = 2) carried arrays of s*N doubles and the gradient block sums.  It is
 * at least etd_rdp_workspace_bytes, and etd_rdp_step accepts the same buffer
 * (its carried arrays come first, in the same places), so one workspace
 * serves a forward sweep and its reverse sweep. */
int etd_rdp_adjoint_workspace_bytes(const etd_rdp_ctx* ctx, size_t* bytes);

/*
 * etd_rdp_adjoint -- one reverse step.  With U_{n+1} = Phi(U_n; D, theta)
 * the step etd_rdp_step takes:
 *   lam_n = (dPhi/dU_n)^T lam_np1,
 *   grad += (dPhi/d(D, theta))^T lam_np1   (accumulated, not overwritten).
 *
 *  u_n     : device, s*N doubles (layout of u), the state the step started
 *            from; read only.
 *  lam_np1 : device, s*N doubles, dL/dU_{n+1}; read only.
 *  lam_n   : device, s*N doubles, receives dL/dU_n.  May be lam_np1 (the
 *            update is then in place); must not overlap u_n.
 *  grad    : device, etd_rdp_grad_size() doubles, caller-initialised.
 *  ws      : device workspace of etd_rdp_adjoint_workspace_bytes, 256-byte
 *            aligned; its carried arrays are overwritten.
 * The result is bitwise reproducible for a given device (fixed reduction
 * order).  Asynchronous on `stream`.
 * Errors: ETD_ERR_ARG (NULL pointer, u_n == lam_n), ETD_ERR_UNSUPPORTED
 * (scheme ETD1, d = 1 or d >= 4, FP32 or complex contexts, a general line length
 * on some axis), ETD_ERR_WORKSPACE,
 * ETD_ERR_HIP.
 */
int etd_rdp_adjoint(etd_rdp_ctx* ctx, const double* u_n, const double* lam_np1,
                    double* lam_n, double* grad, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * Kept steps: a forward step that leaves its carried arrays in caller
 * memory, and the reverse step that reads them instead of recomputing them
 * (the reverse step's own forward passes 1..d-1).  The arrays are exactly
 * what etd_rdp_adjoint recomputes, so results are bitwise those of
 * etd_rdp_adjoint.  For trajectories whose carried arrays fit in device
 * memory (at 128^3 with two species, 201 MB per step).
 *
 * etd_rdp_keep_bytes: bytes of one step's kept arrays: 3 (d = 2) or 6
 *   (d = 3) arrays of s*N doubles, each 256-byte aligned.
 *   ETD_ERR_UNSUPPORTED wherever etd_rdp_adjoint is (d not 2 or 3, FP32,
 *   complex, the first-order scheme, a general axis, a reaction field).
 * etd_rdp_step_keep: one step from u_in to u_out (device states in u's
 *   layout; the same pointer steps in place, as etd_rdp_step with nsteps = 1,
 *   same arithmetic, also on the slab schedule; distinct states must not
 *   overlap), its carried arrays written to keep (device, at least
 *   keep_bytes, 256-byte aligned, caller-owned) instead of the workspace.
 *   Out of place, a caller that keeps every state needs no copy.  ws: a
 *   forward or adjoint workspace.  Errors as etd_rdp_keep_bytes and
 *   etd_rdp_step; ETD_ERR_ARG for a missing, small or misaligned keep and
 *   for overlapping distinct states.
 * etd_rdp_adjoint_kept: etd_rdp_adjoint for the step that started from u_n,
 *   with that step's kept arrays (read only).  ws: an adjoint workspace as
 *   for etd_rdp_adjoint (its two carried triples are not used).  Errors as
 *   etd_rdp_adjoint; ETD_ERR_ARG for a missing, small or misaligned keep.
 */
int etd_rdp_keep_bytes(const etd_rdp_ctx* ctx, size_t* bytes);
int etd_rdp_step_keep(etd_rdp_ctx* ctx, const double* u_in, double* u_out, void* ws,
                      size_t ws_bytes, void* keep, size_t keep_bytes, void* stream);
int etd_rdp_adjoint_kept(etd_rdp_ctx* ctx, const double* u_n, const void* keep,
                         size_t keep_bytes, const double* lam_np1, double* lam_n,
                         double* grad, void* ws, size_t ws_bytes, void* stream);

/* ======================================================================
 * Ensembles: many independent 2-D problems of uneven size advanced together.
 * All instances share the number of species s, the reaction model, the time
 * step k and the scheme; each has its own grid, boundary conditions,
 * diffusion coefficients and reaction parameters.  The states are packed
 * back to back in one device array, instance i at the offset (in elements:
 * doubles, or floats for an FP32 ensemble) that etd_rdp_batch_offsets
 * reports, each laid out like a single problem's state.
 * ====================================================================== */

typedef struct etd_instance_t {
  int64_t n[2];                     /* unknowns on axis 1 (fastest), axis 2 */
  double h[2];                      /* spacing; 0 = unit-domain default     */
  int32_t bc[2];                    /* ETD_BC_* per axis                    */
  double D[ETD_MAX_SPECIES];        /* diffusion coefficients               */
  double params[ETD_MAX_PARAMS];    /* reaction parameters (see ETD_RX_*)   */
  double shift[ETD_MAX_SPECIES];    /* F evaluated at u + shift             */
} etd_instance_t;

typedef struct etd_rdp_batch etd_rdp_batch;

/*
 * etd_rdp_batch_init -- validate ninst >= 1 instances and build their tables
 * on the host (no HIP call).  s and model as in etd_rdp_init; every instance
 * obeys etd_rdp_init's rules for d = 2.  scheme (may be NULL: ETD-RDP, FP64)
 * selects ETD_SCHEME_RDP or ETD_SCHEME_ETD1 and ETD_PRECISION_F64 or
 * ETD_PRECISION_F32 (complex: ETD_ERR_UNSUPPORTED); its other fields are
 * ignored.  Errors as etd_rdp_init; ETD_ERR_UNSUPPORTED also for an instance
 * with a general line length (regular lines only).
 */
int etd_rdp_batch_init(int32_t ninst, const etd_instance_t* inst, int32_t s,
                       int32_t model, double k, const etd_scheme_t* scheme,
                       etd_rdp_batch** out);

int etd_rdp_batch_destroy(etd_rdp_batch* b);

/* offsets[0..ninst]: start of instance i in the packed state (elements);
 * offsets[ninst] is the total length.  Offsets are multiples of 32.
 * Instances of one grid shape sit next to each other (see the groups below),
 * so the offsets are not in instance order. */
int etd_rdp_batch_offsets(const etd_rdp_batch* b, int64_t* offsets);

/* Device workspace bytes (tables, instance descriptors, tile maps and the
 * three carried arrays); 256-byte aligned. */
int etd_rdp_batch_workspace_bytes(const etd_rdp_batch* b, size_t* bytes);

/*
 * etd_rdp_batch_step -- advance every instance by nsteps steps on `stream`.
 * use_graph != 0 records the whole nsteps sequence of launches into one HIP
 * graph (on a private capture stream) and launches that graph on `stream`;
 * the graph is kept and replayed while (u, ws, nsteps) stay the same.
 * Otherwise the kernels are launched one by one.  Asynchronous.
 * ETD_ERR_ARG for an FP32 ensemble.
 */
int etd_rdp_batch_step(etd_rdp_batch* b, double* u_packed, void* ws,
                       size_t ws_bytes, int64_t nsteps, int32_t use_graph,
                       void* stream);

/*
 * etd_rdp_batch_step_f32 -- etd_rdp_batch_step for an ensemble created with
 * ETD_PRECISION_F32: u_packed holds offsets[ninst] floats, the carried
 * arrays are FP32 and every solve and reaction evaluation runs in FP32
 * (tables converted from FP64), as etd_rdp_step_f32 does for one problem.
 * ETD_ERR_ARG for an FP64 ensemble.
 */
int etd_rdp_batch_step_f32(etd_rdp_batch* b, float* u_packed, void* ws,
                           size_t ws_bytes, int64_t nsteps, int32_t use_graph,
                           void* stream);

/* etd_rdp_forget_workspace for an ensemble: the next step uploads the
 * tables, instance descriptors and tile maps again and records a new graph.
 * Errors: ETD_ERR_ARG (NULL). */
int etd_rdp_batch_forget_workspace(etd_rdp_batch* b);

/* Number of kernel launches of one step (for tests and reports): two per
 * group. */
int etd_rdp_batch_launches_per_step(const etd_rdp_batch* b, int32_t* n);

/* ----------------------------------------------------------------------
 * Groups, plans and the autotuner.
 *
 * Instances of the same grid shape (n1, n2) form a group, stored next to
 * each other at equal spacing (so etd_rdp_batch_offsets is not in instance
 * order); a step is one launch per (group, pass).  Each (group, pass) runs
 * one of three kernel forms, its plan entry:
 *   ETD_FORM_UNSPLIT   all solves of a species at once; 16-line tiles for
 *                      chunks of up to 4 rows, 8-line tiles otherwise;
 *   ETD_FORM_STREAMED  solves in phases of at most two, 16-line tiles
 *                      (chunks of at least 3 rows; not pass 1 of ETD1);
 *   ETD_FORM_TWO_LINE  streamed with two lines of 32 chunks per wavefront,
 *                      32-line tiles (lines of n = 32 m rows, 2 <= m <= 8;
 *                      not pass 1 of ETD1).
 * A plan is an int32 array of 2 * ngroups entries: plan[2 g + p] is the form
 * of pass p (0: axis 1, 1: axis 2) of group g.  Every form computes the same
 * step up to rounding (the chunking of the two-line form differs).
 * ---------------------------------------------------------------------- */
#define ETD_FORM_UNSPLIT 0
#define ETD_FORM_STREAMED 1
#define ETD_FORM_TWO_LINE 2

/* Number of groups; if shapes is not NULL, shapes[2 g], shapes[2 g + 1] get
 * group g's (n1, n2); if counts is not NULL, counts[g] its instance count.
 * Errors: ETD_ERR_ARG (NULL b or ngroups). */
int etd_rdp_batch_groups(const etd_rdp_batch* b, int32_t* ngroups, int64_t* shapes,
                         int32_t* counts);

/* The current plan (2 * ngroups entries).  A new ensemble starts with a
 * default plan from the single-problem rules.  Errors: ETD_ERR_ARG. */
int etd_rdp_batch_get_plan(const etd_rdp_batch* b, int32_t* plan);

/* Replace the plan (e.g. one etd_rdp_batch_tune found earlier and a caller
 * kept).  ETD_ERR_ARG (and no change) if any entry is not a form that
 * (group, pass) allows.  Drops a recorded graph. */
int etd_rdp_batch_set_plan(etd_rdp_batch* b, const int32_t* plan);

/* *allowed = 1 if (group, pass) may run `form`, else 0.  Errors:
 * ETD_ERR_ARG (NULL, index out of range). */
int etd_rdp_batch_form_allowed(const etd_rdp_batch* b, int32_t group, int32_t pass,
                               int32_t form, int32_t* allowed);

/*
 * etd_rdp_batch_tune -- the autotuner: for every group and pass, time `reps`
 * launches (after one untimed launch) of every form it allows, on `stream`
 * with HIP events, and keep the fastest in the plan.  Works on the caller's
 * state: u (device, offsets[ninst] elements of the ensemble's precision) is
 * advanced by exactly one step of the new plan.  times (may be NULL):
 * 2 * ngroups * 3 doubles, times[(2 g + p) * 3 + form] = milliseconds per
 * launch, or -1 for a form the (group, pass) does not allow.  Synchronises
 * the stream before returning.  Errors: ETD_ERR_ARG, ETD_ERR_WORKSPACE,
 * ETD_ERR_HIP.
 */
int etd_rdp_batch_tune(etd_rdp_batch* b, void* u, void* ws, size_t ws_bytes, int32_t reps,
                       void* stream, double* times);

/* Launch pass `pass` of group `group` alone in form `form` (-1: the plan's),
 * on the same arrays as inside a step (pass 0 reads u and writes the carried
 * arrays, pass 1 reads them and writes u).  For timing and tests.  Errors:
 * ETD_ERR_ARG (bad index, a form the group does not allow), ETD_ERR_WORKSPACE,
 * ETD_ERR_HIP. */
int etd_rdp_batch_group_pass(etd_rdp_batch* b, void* u, void* ws, size_t ws_bytes,
                             int32_t group, int32_t pass, int32_t form, void* stream);

/* ======================================================================
 * Bandwidth calibration (for reports; not part of the scheme).
 * ====================================================================== */

/*
 * etd_calib_stream -- one streaming sweep over `bytes` bytes of device
 * memory on `stream`, with `blocks` workgroups (of 256 threads unless
 * stated):
 *   kind 0: copy src -> dst (reads and writes `bytes`),
 *   kind 1: read src (dst: device, at least 8 bytes; written only if the
 *           sum of src is -1e308, which finite data never reaches),
 *   kind 2: write dst (src unused, may be NULL),
 *   kind 3, 4: kinds 0 and 2 with non-temporal stores,
 *   kind 5: copy with workgroups of 1024 threads, each streaming one
 *           contiguous range of the buffers, non-temporal stores.
 * Timing these against the passes gives the rate simple streaming code
 * reaches on this device.  bytes must be a multiple of 16 and the pointers
 * 16-byte aligned; the buffers are the caller's.
 * Errors: ETD_ERR_ARG (bad kind, size, alignment or NULL), ETD_ERR_HIP.
 */
int etd_calib_stream(int32_t kind, const void* src, void* dst, size_t bytes,
                     int32_t blocks, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ETD_RDP_H_ */
