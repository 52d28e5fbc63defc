/*
 * mrtfd -- the time step of the energy-conserving multiple-relaxation-time
 * finite-difference lattice Boltzmann model of Chen, Xu, Zhang and Li
 * ("Multiple-relaxation-time lattice Boltzmann model for compressible
 * fluids", arXiv:0908.3749) on AMD MI355X (gfx950).
 *
 * One step, for every interior node of a 2D grid with the paper's 16
 * discrete velocities (Sect. III, Eq. 4):
 *   f-hat = M f (Eq. 5), equilibria f-hat^eq of the nonconserved moments
 *   (Eq. 14), relaxation by the diagonal S-hat and the map back with M^-1
 *   (Eq. 3), then forward Euler in time with the per-axis Lax-Wendroff
 *   difference in space (appendix, Eq. A.1a-b), collision and advection both
 *   evaluated at the old time level (Sect. IV, the update behind G).
 * Boundary nodes carry f = f^eq of a macroscopic state chosen by a rule
 * (Sect. V: prescribed, periodic, reflecting, linearly extrapolated, moving
 * isothermal wall).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int32 status: MRTFD_OK (0) or a negative
 *    MRTFD_ERR_* code; mrtfd_status_string() names it and
 *    mrtfd_last_error() gives the context's last message.  No C++ exception
 *    crosses this interface.  A failing call leaves the context usable.
 *  - Pointers named d_* are device pointers (HBM of the GPU the context was
 *    created on); all other pointers are host pointers.
 *  - The caller owns all device memory: the library works inside one
 *    caller-provided workspace and never allocates or frees device memory.
 *    The context object itself is host memory owned by the library and
 *    released by mrtfd_destroy().
 *  - Every GPU operation is enqueued on the stream given at creation, in
 *    call order.  Only calls returning host data (mrtfd_sums) synchronise
 *    that stream.  Memory is cleared by kernels, never by memset nodes.
 *  - Debugging: with MRTFD_POISON_PADDING=1 in the environment when a
 *    context is created, its two copies of f start filled with NaN instead
 *    of zeros.  Only interior nodes are ever written or read as state, so
 *    results are unchanged; a read outside the interior would show as NaN.
 *  - Macroscopic fields are FP32, row-major [ny][nx] over the interior
 *    nodes, node (i, j) at x = (i + 1/2) dx, y = (j + 1/2) dy.
 *  - Populations are numbered as in Eq. (4): 0-3 = cyc(+-1,0) in the order
 *    (+,0),(0,+),(-,0),(0,-); 4-7 the same times 6; 8-11 = sqrt2(+-1,+-1) in
 *    the order (+,+),(-,+),(-,-),(+,-); 12-15 the same times 3/sqrt2.
 */
#ifndef MRTFD_H
#define MRTFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MRTFD_OK 0
#define MRTFD_ERR_ARG (-1)         /* a bad argument or parameter           */
#define MRTFD_ERR_HIP (-2)         /* a HIP runtime call failed             */
#define MRTFD_ERR_UNSTABLE (-3)    /* dt*s > 1 or Courant number > 1        */
#define MRTFD_ERR_NONFINITE (-4)   /* NaN/Inf met in the state              */
#define MRTFD_ERR_STATE (-5)       /* call out of order (e.g. step before init) */
#define MRTFD_ERR_UNSUPPORTED (-6) /* a mode the library does not provide  */

/* ---- boundary rules (Sect. V) ------------------------------------------ */
#define MRTFD_BC_PERIODIC 0    /* copy of the opposite interior edge (V.A)      */
#define MRTFD_BC_DIRICHLET 1   /* f^eq of the prescribed state (V.A, V.B)       */
#define MRTFD_BC_REFLECT 2     /* adjacent interior state, normal velocity
                                  reversed (V.B(a))                             */
#define MRTFD_BC_EXTRAPOLATE 3 /* 2 q1 - q2 on (rho,u1,u2,T) from the first two
                                  interior nodes, q1 if that gives rho <= 0 or
                                  T <= 0 (V.B(a), "linear extrapolation")       */
#define MRTFD_BC_WALL 4        /* (rho of the adjacent node, u1, u2, T of the
                                  state): constant speed and temperature
                                  walls (V.D)                                   */

/* ---- arithmetic of the moment transforms ------------------------------- */
#define MRTFD_FP32 0  /* FP32 everywhere (FP64 only in mrtfd_sums)            */
#define MRTFD_BF16X3 1 /* the collision's transforms (the 4x4 blocks of the
                          factored M and M^-1) on the matrix cores in BF16
                          parts, FP32 accumulation: M's blocks, exact in
                          BF16 (a sqrt 2 factor of two columns moved onto
                          the inputs), against inputs split exactly into
                          three parts; the back-map's FP32 weights split
                          exactly into three parts against the
                          nonequilibrium moments split into two.  The
                          butterflies, equilibria and stencil FP32 (a last
                          grid column alone in its 64-column wave takes the
                          FP32 collision)                                   */
#define MRTFD_FP64 2   /* the whole step in FP64, populations stored in FP64
                          (the rows kernel at one row per wave, or the
                          simple kernel; 256 bytes of populations per node
                          update): for states
                          whose populations sum to far more than rho (hot
                          gas: the 16-velocity equilibrium sums to about
                          0.7 T^2 rho), where FP32 storage rounds rho by that
                          factor more than u (Sect. V.A(c), (d)).  Outputs
                          of mrtfd_read_macro are FP32 roundings;
                          mrtfd_get_f64 / mrtfd_set_f64 exchange the stored
                          values exactly                                     */

/* ---- collision operator ------------------------------------------------ */
#define MRTFD_COLLISION_MRT 0 /* Eq. (3): M^-1 S-hat (f-hat - f-hat^eq)            */
#define MRTFD_COLLISION_SRT 1 /* single relaxation time S = I/tau (Sect. II):
                                 s_6..s_16 must equal s_5 = 1/tau; computed
                                 as Eq. (3) with equal rates, which keeps
                                 the conserved moments out of the update
                                 exactly (f - f^eq evaluated in velocity
                                 space in FP32 does not)                     */

/* ---- device order of the populations (internal copies of f) ------------ */
#define MRTFD_LAYOUT_ROWS 0   /* per grid row, the 16 population rows side by
                                 side                                          */
#define MRTFD_LAYOUT_PLANES 1 /* 16 whole-grid population planes             */
#define MRTFD_LAYOUT_TILES 2  /* per grid row and 64-column piece, the 16
                                 population pieces side by side (4 KiB)        */

/* ---- kernel choice for the step ---------------------------------------- */
#define MRTFD_KERNEL_AUTO 0   /* autotuned among the variants below            */
#define MRTFD_KERNEL_SIMPLE 1 /* one thread per node, 64x4 tiles, neighbours
                                 read from memory                              */
#define MRTFD_KERNEL_ROWS 2   /* each wave: `rows` rows of 64 columns loaded
                                 once, west/east neighbours by lane shifts     */
#define MRTFD_KERNEL_MFMA 3   /* reported only: the rows kernel with the
                                 split-BF16 matrix-core collision, which
                                 MRTFD_BF16X3 always uses (rows per wave, store
                                 kind and tile order autotuned)                */

/* One side of the grid.  The rule is kind_lo at ghost nodes whose
 * along-side coordinate (x for the south/north sides, y for west/east) is
 * <= split0 + split_rate * t, and kind_hi beyond; set kind_lo == kind_hi for
 * a single rule.  state_* = (rho, u1, u2, T) for DIRICHLET, (ignored, u1,
 * u2, T) for WALL, unused otherwise.  A PERIODIC side needs the opposite
 * side PERIODIC too, on both parts. */
typedef struct mrtfd_side {
    int32_t kind_lo, kind_hi;
    double state_lo[4];
    double state_hi[4];
    double split0, split_rate;
} mrtfd_side;

/* Problem parameters.  s[k] is s_{k+1} of S-hat (Eq. 3); s[0..3] act on
 * conserved moments and are ignored.  side[] = west (i = -1), east (i = nx),
 * south (j = -1), north (j = ny).  Validation: nx, ny >= 3; dx, dy, dt > 0;
 * 0 <= dt*s_k <= 1 for k >= 5 (the paper never goes beyond); 6 dt / min(dx,
 * dy) <= 1 (Courant number of the fastest velocity). */
typedef struct mrtfd_params {
    int32_t nx, ny;
    double dx, dy, dt;
    double s[16];
    mrtfd_side side[4];
    int32_t precision;  /* MRTFD_FP32, MRTFD_BF16X3 or MRTFD_FP64             */
    int32_t kernel;     /* MRTFD_KERNEL_*                                    */
    int32_t rows;       /* rows per wave for MRTFD_KERNEL_ROWS (1 or 2),
                           0 = auto                                          */
    int32_t graph_steps;/* steps per captured HIP graph, 0 = no graph        */
    int32_t collision;  /* MRTFD_COLLISION_MRT or _SRT                        */
    int32_t layout;     /* MRTFD_LAYOUT_ROWS or _PLANES (device order of f)   */
    int32_t flux_budget;/* 1: every step also adds the FP64 outflow through
                           each side to a running total (mrtfd_outflow):
                           in extra blocks of the step kernel's own grid
                           (rows kernel, one row per wave), else a small
                           kernel on a library-owned stream that runs
                           beside the step kernel. 0: off                */
    double ref_rho, ref_T;
                        /* reference state at rest, both > 0, or both 0 for
                           none.  With a reference the copies of f hold
                           g = f - f_ref, f_ref = f^eq(ref_rho, 0, 0, ref_T)
                           (Eq. 14 mapped back by M^-1; the reference values
                           are rounded to FP32 first): the difference
                           scheme (Eq. A.1b) is linear and f_ref uniform, so
                           it acts on g alone, and the collision (Eq. 3)
                           adds back the reference's conserved moments and
                           takes out its one nonzero nonconserved
                           equilibrium.  The FP32 rounding of every step
                           then scales with |f - f_ref| rather than |f|:
                           near the reference state (smooth, slow flow) the
                           error against exact arithmetic falls by the
                           ratio.  mrtfd_get_f / mrtfd_set_f exchange g;
                           mrtfd_ref_populations gives f_ref.           */
} mrtfd_params;

typedef struct mrtfd_ctx mrtfd_ctx;

/* Size in bytes of the device workspace a context with these parameters
 * needs (two FP32 copies of f with a ghost ring plus reduction scratch).
 * Returns 0 if the parameters are invalid. */
size_t mrtfd_workspace_bytes(const mrtfd_params *p);

/* Validate parameters without touching the GPU.  Writes a message into msg
 * (host buffer of msg_len bytes, may be NULL).  Returns MRTFD_OK,
 * MRTFD_ERR_ARG or MRTFD_ERR_UNSTABLE. */
int32_t mrtfd_check_params(const mrtfd_params *p, char *msg, size_t msg_len);

/* Create a context.  Builds M from Eq. (5) on the host, inverts it in FP64
 * and uploads the FP32 constants.  d_workspace: device buffer of at least
 * mrtfd_workspace_bytes(p) bytes, 256-byte aligned, owned by the caller and
 * kept alive until mrtfd_destroy.  stream: a hipStream_t (NULL = default
 * stream).  On success *out receives the context.  Errors: the codes of
 * mrtfd_check_params; MRTFD_ERR_ARG for a NULL, short or misaligned
 * workspace; MRTFD_ERR_HIP if a runtime call fails; MRTFD_ERR_UNSUPPORTED
 * with MRTFD_BF16X3 if the factored transform's blocks are not held exactly
 * by their BF16 parts (a consistency check of the model, which the
 * 16-velocity M of Eq. 5 passes). */
int32_t mrtfd_create(const mrtfd_params *p, void *d_workspace, size_t workspace_bytes,
                     void *stream, mrtfd_ctx **out);

/* Release the context (host memory, graphs).  The workspace is untouched. */
int32_t mrtfd_destroy(mrtfd_ctx *ctx);

/* Initialise f = M^-1 f-hat^eq(rho, rho u, rho (T + |u|^2/2)) at every
 * interior node (the equilibrium of the macroscopic initial condition, as
 * the paper's boundary and initial states are set) and reset the clock to
 * step 0.  Inputs: four device [ny][nx] FP32 arrays.  rho > 0 and T > 0 are
 * required; a violation (or a non-finite input) is reported by the next
 * mrtfd_sums as MRTFD_ERR_ARG. */
int32_t mrtfd_init_macro(mrtfd_ctx *ctx, const float *d_rho, const float *d_ux,
                         const float *d_uy, const float *d_T);

/* Advance nsteps >= 0 time steps (each: boundary nodes at time t_n = n dt
 * from f^n, then the fused collision + Lax-Wendroff + Euler update of every
 * interior node).  While the kernel choice is open (see mrtfd_kernel_info)
 * the first steps of a long enough call time the candidate variants. */
int32_t mrtfd_step(mrtfd_ctx *ctx, int64_t nsteps);

/* Macroscopic fields of the current state: rho = f-hat_1, u = j / rho,
 * T = (e - rho |u|^2 / 2) / rho, p = rho T (R = 1).  Outputs are device
 * [ny][nx] FP32 arrays; any of them may be NULL. */
int32_t mrtfd_read_macro(mrtfd_ctx *ctx, float *d_rho, float *d_ux, float *d_uy,
                         float *d_T, float *d_p);

/* FP64 sums over the interior of rho, j_x, j_y, e (host array out[4]).
 * Deterministic (fixed reduction order).  Synchronises the stream.  Returns
 * MRTFD_ERR_NONFINITE if any sum is not finite. */
int32_t mrtfd_sums(mrtfd_ctx *ctx, double out[4]);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the FP64 sums of
 * mrtfd_sums written to the caller's device array d_out[4] (rho, j_x, j_y,
 * e), enqueued on the context's stream with no synchronisation, no host
 * copy and no allocation of any kind.  The reduction's partial sums go to a
 * library-held device array of 4096 doubles (32 KiB, one per GPU, held until
 * the process ends; a reduction uses at most 1024 x 4 of them, so every grid
 * fits and larger needs would be refused with MRTFD_ERR_ARG).  Same kernels
 * and summation order as mrtfd_sums: the same bits.  The caller checks the
 * values for finiteness.  All contexts on one GPU share that array: calls
 * whose kernels can overlap (different streams on the same GPU without
 * ordering between them) race and give wrong sums; calls on one stream, or
 * ordered by events, are safe. */
int32_t mrtfd_sums_noalloc(mrtfd_ctx *ctx, double *d_out);

/* Copy the interior populations out of / into the context as a packed
 * device FP32 array [16][ny][nx] (checkpoint / restart, seeded states).
 * These are the populations as stored: f itself, or g = f - f_ref when the
 * parameters set a reference state (ref_rho, ref_T), so that a checkpoint
 * taken with mrtfd_get_f restarts bit for bit. */
int32_t mrtfd_get_f(mrtfd_ctx *ctx, float *d_f);
int32_t mrtfd_set_f(mrtfd_ctx *ctx, const float *d_f);

/* The same exchange as a packed device FP64 array [16][ny][nx]: exact for
 * MRTFD_FP64 contexts (checkpoint and restart bit for bit); for FP32-stored
 * contexts get widens exactly and set rounds to nearest FP32 (mrtfd_get_f /
 * mrtfd_set_f do the reverse for MRTFD_FP64 contexts). */
int32_t mrtfd_get_f64(mrtfd_ctx *ctx, double *d_f);
int32_t mrtfd_set_f64(mrtfd_ctx *ctx, const double *d_f);

/* f_ref = M^-1 f-hat^eq(ref_rho, 0, 0, ref_rho ref_T) (Eq. 14, FP64, from
 * the FP32 roundings of ref_rho and ref_T) of these parameters into the host
 * array out[16]; zeros when no reference state is set.  f = g + f_ref for the
 * arrays of mrtfd_get_f / mrtfd_set_f.  Needs no GPU. */
int32_t mrtfd_ref_populations(const mrtfd_params *p, double out[16]);

/* Current step index and time t = step * dt (host outputs, may be NULL). */
int32_t mrtfd_time(mrtfd_ctx *ctx, int64_t *step, double *t);

/* Outflow budget (needs flux_budget = 1).  Over the interior the
 * difference of Eq. (A.1b) is a difference of face values, so the node sums
 * of rho, j1, j2, e (mrtfd_sums) change in each step by minus the face
 * values summed over the outer faces (the collision, Eq. 3, conserves them).
 * out[4*side + k] (host, 16 doubles) = the FP64 outflow of moment k (rho,
 * j1, j2, e) through side (west, east, south, north) summed over the steps
 * since the last mrtfd_init_macro / mrtfd_set_f: face values taken in FP64
 * from the FP32 populations of each step, with the step's boundary ghosts
 * (periodic sides: the periodic image, equal and opposite on the two sides).
 * Then sums(now) - sums(start) + sum over sides of out = 0 up to the FP32
 * rounding of the updates.  Synchronises the stream; MRTFD_ERR_STATE if the
 * budget is off, MRTFD_ERR_NONFINITE if a total is not finite. */
int32_t mrtfd_outflow(mrtfd_ctx *ctx, double out[16]);

/* Set the clock to step index `step` >= 0 (t = step * dt), e.g. after
 * mrtfd_set_f on a restart, so that time-dependent boundary rules carry on
 * where they stopped. */
int32_t mrtfd_set_step(mrtfd_ctx *ctx, int64_t step);

/* The step kernel in use (MRTFD_KERNEL_SIMPLE, _ROWS or _MFMA), its rows
 * per wave, 1 if it writes with streaming (non-temporal) stores, else 0, and
 * the order in which tiles go to the chip's eight L2 domains: 0 = each takes
 * a band of whole tile rows, 1 = a band of tile columns (host outputs, each
 * may be NULL).  With MRTFD_KERNEL_AUTO, or _ROWS and
 * rows = 0, the choice is made by timing the candidates (rows per wave,
 * store kind, tile order, and the simple kernel) on the first steps of the
 * first mrtfd_step call long enough for a fair trial (two passes over the
 * candidates, up to about 600 steps; results are bit-identical whichever
 * runs) and is cached per grid size, precision and flux_budget for later
 * contexts; before that the rows kernel with one row per wave and plain
 * stores runs.  With MRTFD_BF16X3 the same trial picks the split-BF16 rows
 * kernel's rows per wave, store kind and tile order. */
int32_t mrtfd_kernel_info(mrtfd_ctx *ctx, int32_t *kernel, int32_t *rows, int32_t *streaming,
                          int32_t *tile_order);

/* Von Neumann screen of Sect. IV.  For the uniform state (rho, u1, u2, T) =
 * state[0..3] (host array; rho > 0, T > 0) and the spacing, time step and
 * rates of p (dx, dy, dt > 0 and rates >= 0, finite; dt s_k may exceed 1,
 * which mrtfd_create refuses; the grid and boundary fields are not used), the
 * amplification matrix of one Fourier mode of the scheme (Eq. A.1a-b with the
 * collision of Eq. 3 linearised about the state, the equilibria of Eq. 14
 * differentiated through rho, j and e) is
 *   G_ij(theta) = delta_ij (1 - i a_i sin theta_x + a_i^2 (cos theta_x - 1)
 *                 - i b_i sin theta_y + b_i^2 (cos theta_y - 1))
 *                 - dt [M^-1 S (M - d f-hat^eq / d f)]_ij,
 * a_i = v_i1 dt / dx, b_i = v_i2 dt / dy, theta = (k_x dx, k_y dy); the scheme
 * is stable at the state when every eigenvalue omega of G has |omega| <= 1
 * over all phases.  For n phase pairs d_theta[2 p], d_theta[2 p + 1] (device
 * array of 2 n doubles) computes the 16 eigenvalues of G in FP64 (balancing,
 * Householder reduction to Hessenberg form and the shifted QR algorithm, four
 * phase pairs per wave) and writes them, largest modulus first, as (re, im)
 * pairs to d_eig[32 p .. 32 p + 31], and the largest modulus to d_rho[p]
 * (device arrays of 32 n and n doubles; either may be NULL, not both).  They
 * are the exact eigenvalues of some G + E with ||E|| a small multiple of u
 * ||G|| (u = 2^-53), so an eigenvalue with condition number kappa (1 / |y^H x|
 * for unit left and right eigenvectors y, x) is accurate to about kappa u
 * ||G||: near 1e-12 at moderate states, but ~1e-4 at hot or fast ones, where
 * ||G|| and kappa both reach ~1e6.  A phase whose iteration does not converge
 * in 480 QR steps gets NaN.  Enqueued on `stream` (a hipStream_t, NULL =
 * default); nothing is allocated.  MRTFD_ERR_ARG for p NULL, dx, dy or dt not
 * positive and finite, a negative or non-finite rate, a state with rho <= 0, T
 * <= 0 or non-finite values, n < 0, d_theta NULL or both outputs NULL with n >
 * 0; MRTFD_ERR_HIP if the launch fails. */
int32_t mrtfd_screen(const mrtfd_params *p, const double state[4], const double *d_theta, int32_t n,
                     double *d_eig, double *d_rho, void *stream);

/* The von Neumann screen of Sect. IV over many parameter sets at once, for
 * searches over states and rates.  Set q (0 <= q < nsets) has the uniform
 * state d_states[4 q .. 4 q + 3] = (rho, u1, u2, T) and the 16 rates
 * d_rates[16 q .. 16 q + 15] (device arrays); the spacing and time step come
 * from p (dx, dy, dt > 0, finite; its rates, grid and boundary fields are not
 * used).  For the n phase pairs d_theta (device, 2 n doubles) shared by all
 * sets, writes max |omega| of G (as mrtfd_screen) for set q at pair j to
 * d_rho[q n + j] (device, nsets n doubles) and the largest over j to d_max[q]
 * (device, nsets doubles); either may be NULL, not both.  Each set's
 * coefficients are formed on the GPU (the Jacobian of Eq. 14 by dual numbers),
 * so the values differ from mrtfd_screen's by the rounding of the
 * coefficients, amplified as there by the eigenvalues' condition numbers
 * (far below 1e-9 at moderate states, 4e-6 at the high-Mach tube's west
 * state).  A
 * set with rho <= 0, T <= 0 or a non-finite state or rate, and a non-finite
 * phase pair, give NaN (and NaN as that set's maximum).  Enqueued on `stream`;
 * the first call on a device uploads the model (M, M^-1, velocities: 4.3 KB)
 * to a static device array, synchronously; nothing is allocated.
 * MRTFD_ERR_ARG for p NULL, dx, dy or dt not positive and finite, nsets < 0, n
 * < 0, nsets n >= 2^31, or NULL arrays with nsets n > 0; MRTFD_ERR_HIP if the
 * upload or a launch fails; nsets n = 0 writes nothing. */
int32_t mrtfd_screen_sets(const mrtfd_params *p, int32_t nsets, const double *d_states, const double *d_rates,
                          const double *d_theta, int32_t n, double *d_rho, double *d_max, void *stream);

/* The library's FP64 model on the host: velocity set v[16][2] (Eq. 4), M
 * [16][16] (Eq. 5, row-major, M[k][i] = m_{k+1}(v_i)) and its inverse, as
 * used to build the kernels' constants.  Host arrays; any may be NULL. */
int32_t mrtfd_model(double *v, double *M, double *Minv);

/* sizeof(mrtfd_params) and sizeof(mrtfd_side) as compiled into the library,
 * so that language bindings can check their struct layouts. */
int32_t mrtfd_struct_sizes(size_t *params_size, size_t *side_size);

const char *mrtfd_status_string(int32_t status);
const char *mrtfd_last_error(const mrtfd_ctx *ctx);

/* ---- batches of independent shock tubes ----------------------------------
 * Many one-dimensional Riemann problems (Sect. V.A) of different lengths run
 * together.  Tube k has n[k] columns and 4 rows, periodic in y, and its two
 * ends carry f = f^eq of its left / right state (as the paper sets its tube
 * ends); its initial state is the left state for columns x < n[k]/2 and the
 * right state beyond.  Every tube advances its own number of steps.  The
 * work is split into items of seg_cols columns that advance round_steps
 * steps per launch inside on-chip memory (temporal blocking); the launch of
 * a round covers the items of all tubes still running.  Each node's update
 * is the same arithmetic as the single-grid step, so tube k ends bit for bit
 * where a single grid with the same parameters would. */
typedef struct mrtfd_batch mrtfd_batch;

typedef struct mrtfd_batch_params {
    int32_t ntubes;      /* >= 1                                                */
    double dx, dt;       /* node spacing (dx = dy) and time step, all tubes     */
    double s[16];        /* relaxation rates as in mrtfd_params, all tubes      */
    int32_t seg_cols;    /* columns per work item, 0 = autotune; built pairs
                            (seg_cols, round_steps): (32,16) (48,8) (56,4)   */
    int32_t round_steps; /* steps per round (4, 8 or 16), 0 = autotune       */
    int32_t use_graph;   /* 1: replay all rounds as one captured HIP graph      */
} mrtfd_batch_params;

/* Device workspace bytes for a batch with tube lengths n[ntubes] (host
 * array); 0 if the parameters are invalid. */
size_t mrtfd_batch_workspace_bytes(const mrtfd_batch_params *p, const int32_t *n);

/* Create a batch.  Host arrays: n[ntubes] (>= 3 columns), steps[ntubes]
 * (>= 0), left[ntubes][4] and right[ntubes][4] = (rho, u1, u2, T) with
 * rho > 0, T > 0.  d_workspace: caller-owned device buffer of
 * mrtfd_batch_workspace_bytes bytes, 256-byte aligned.  stream as for
 * mrtfd_create.  Validation as for mrtfd_params (dt s_k <= 1, 6 dt / dx <= 1). */
int32_t mrtfd_batch_create(const mrtfd_batch_params *p, const int32_t *n, const int64_t *steps,
                           const double *left, const double *right, void *d_workspace,
                           size_t workspace_bytes, void *stream, mrtfd_batch **out);

/* Set every tube to its initial Riemann state (step 0). */
int32_t mrtfd_batch_init(mrtfd_batch *b);

/* Advance every tube by its own number of steps (after mrtfd_batch_init;
 * once per initialisation).  The first call on a batch shape autotunes
 * seg_cols and round_steps unless given. */
int32_t mrtfd_batch_run(mrtfd_batch *b);

/* Macroscopic fields (device [4][n[tube]] FP32 arrays, any may be NULL) or
 * the packed populations (device [16][4][n[tube]]) of one tube's current
 * state. */
int32_t mrtfd_batch_read_macro(mrtfd_batch *b, int32_t tube, float *d_rho, float *d_ux,
                               float *d_uy, float *d_T, float *d_p);
int32_t mrtfd_batch_get_f(mrtfd_batch *b, int32_t tube, float *d_f);

/* Chosen work-item width, steps per round and number of rounds (host
 * outputs, may be NULL). */
int32_t mrtfd_batch_info(mrtfd_batch *b, int32_t *seg_cols, int32_t *round_steps,
                         int32_t *rounds);

int32_t mrtfd_batch_destroy(mrtfd_batch *b);
const char *mrtfd_batch_last_error(const mrtfd_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* MRTFD_H */
