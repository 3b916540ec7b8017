/*
 * rte.h -- C ABI of librte: MgNet-preconditioned flexible GMRES for the steady
 * discrete-ordinates radiative transfer equation on one AMD Instinct MI355X
 * (gfx950).
 *
 * Problem (paper Sec. 1, eq. (RTE), eq. (hg), eq. (boundary_condition); Sec. 2.1,
 * eq. (DORTE_2d)): on the unit square or cube with I cubic cells per axis,
 * find psi_{m,c} (direction m, cell c) with
 *
 *   sum_a |u_{m,a}|/h (psi_{m,c} - psi_{m,c-s_a e_a}) + sT_c psi_{m,c}
 *        - sS_c sum_n S_mn psi_{n,c} = b_{m,c}
 *
 * (first-order upwind finite volumes, s_a = sign(u_{m,a})), sT = sigma_T/eps,
 * sS = sigma_T/eps - eps sigma_a, b = eps q plus the inflow carried in across
 * boundary faces, and S = K W the Henyey-Greenstein kernel matrix, scaled
 * symmetrically so that its quadrature-weighted rows and columns sum to one.
 * The learned preconditioner is the CoeffNet + MgNet pair of Sec. 3.
 *
 * Conventions for every function:
 *   - the return value is an rte_status; RTE_OK is 0; on any other value a
 *     message is available from rte_last_error() on the calling thread;
 *   - no output is modified on error, except where a function says otherwise;
 *   - "device" pointers are HIP device memory on the current device (for
 *     example a torch tensor's data_ptr()); "host" pointers are ordinary
 *     memory; the library never takes ownership of caller memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     functions that take a stream enqueue their work on it and return
 *     without waiting unless they say otherwise;
 *   - vectors over the discretisation are direction-major: element
 *     [m * cells + c], with cells ordered x fastest then y then z.
 */
#ifndef RTE_H
#define RTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RTE_OK = 0,
  RTE_EINVAL = -1,      /* invalid argument or input data                    */
  RTE_ENOMEM = -2,      /* workspace too small, allocation failed, budget   */
  RTE_EDEVICE = -3,     /* a HIP runtime call failed                         */
  RTE_ENOCONV = -4,     /* solve stopped before the tolerance; x and stats valid */
  RTE_EBREAKDOWN = -5,  /* non-finite values appeared in the Krylov process  */
  RTE_EAGAIN = -6,      /* poll: not finished yet / submit: server full      */
  RTE_EFORMAT = -7,     /* malformed MGN1 weights blob                       */
  RTE_ENOTFOUND = -8    /* unknown ticket                                    */
} rte_status;

/* Scattering kernel choice (eq. (hg)).  FLATLAND: (1-g^2)/(1+g^2-2g mu), the
 * circle analogue, whose mean cosine is g.  SPHERE: eq. (hg) as printed,
 * (1-g^2)/(1+g^2-2g mu)^{3/2}.  AUTO: FLATLAND when every direction has
 * z = 0, else SPHERE. */
enum { RTE_HG_AUTO = 0, RTE_HG_FLATLAND = 1, RTE_HG_SPHERE = 2 };
enum { RTE_FP32 = 0, RTE_FP64 = 1 };
/* Preconditioner of rte_solve: none, MgNet with BF16 MFMA convolutions,
 * MgNet with FP32 MFMA convolutions (FP32 accumulation in both), or the
 * cell-wise Block-Jacobi comparator of the paper's experiments (Sec. 4):
 * per cell the N x N block of L coupling that cell's directions,
 * diag_m(sum_a |u_{m,a}|/h) + sT_c I - sS_c S, solved in FP32 (up to
 * RTE_BJ_MAX_DIRS directions; no model needed). */
enum { RTE_PC_NONE = 0, RTE_PC_MGNET_BF16 = 1, RTE_PC_MGNET_FP32 = 2, RTE_PC_BLOCK_JACOBI = 3 };
enum { RTE_BJ_MAX_DIRS = 112 };

typedef struct rte_operator rte_operator;
typedef struct mgnet_model mgnet_model;
typedef struct rte_server rte_server;
typedef struct rte_atfps rte_atfps;

/* Spatial scheme of an operator.
 * UPWIND: cell-centred first-order upwind finite volumes (the equation at the
 *   top of this file); unknowns psi, direction-major [ndir][cells].
 * TFPS: the tailored finite point scheme of Sec. 2.2 (2D only): in every cell
 *   the exact exponential solutions of the cell's constant-coefficient
 *   discrete-ordinates equation, eq. (2D_eigenfunc), 2 N of them with
 *   eigenvectors normalised to max-norm 1 (sign: the first entry within 1e-8
 *   of the largest magnitude is positive) in the order x-type decaying from
 *   the left edge, x-type decaying from the right edge, y-type from the bottom,
 *   y-type from the top, eigenvalue ascending within each group, plus the
 *   constant particular solution eps q / (eps sigma_a).  Unknowns: the
 *   coefficients, cell-major [cells][2 N].  Equations, cell-major [cells][2][N]:
 *   for cell (i, j), row [0][m] is continuity of psi_m at the midpoint of its
 *   left face, eq. (2DTFPS_continuity_cond), written psi(cell i-1) -
 *   psi(cell i) = particular-solution jump (i >= 1), or for i = 0 the inflow
 *   condition, eq. (2DTFPS_boundary_cond), of the x = 0 face (u_x > 0) or of
 *   the x = 1 face of cell (I-1, j) (u_x < 0); row [1][m] the same along y.
 *   Needs sigma_a > 0 in every cell, every direction with nonzero x and y
 *   components, half of them positive along each axis, and no MgNet model
 *   (the preconditioners of rte_solve that apply: RTE_PC_NONE). */
enum { RTE_SCHEME_UPWIND = 0, RTE_SCHEME_TFPS = 1 };

/* Angular and spatial discretisation (Sec. 2.1; Sec. 2.2 first paragraph). */
typedef struct {
  int dim;                /* 2 or 3; domain [0,1]^dim                            */
  int n[3];               /* cells per axis x, y, z (n[2] = 1 in 2D); all equal  */
  int ndir;               /* number of directions N, 1..256                      */
  const double* dirs;     /* host [ndir][3] unit vectors (z ignored in 2D)        */
  const double* weights;  /* host [ndir], positive, summing to 1 (+-1e-12)        */
  double g;               /* HG anisotropy, |g| < 1                              */
  int kernel;             /* RTE_HG_*                                            */
  int scheme;             /* RTE_SCHEME_* (0: upwind)                             */
} rte_geometry;

/* Per-cell medium (eq. (RTE): sigma_T, sigma_a, q, eps; Sec. 2.2 cell values).
 * All arrays are host [cells] in cell order.  The library copies what it
 * needs before rte_build_operator returns. */
typedef struct {
  const double* sigma_t;  /* > 0                                                 */
  const double* sigma_a;  /* >= 0, with sigma_t/eps - eps*sigma_a >= 0           */
  const double* q;        /* >= 0                                                */
  const double* eps;      /* 0 < eps <= 1, or NULL to use eps_scalar everywhere  */
  double eps_scalar;
  /* Inflow data Psi (eq. (boundary_condition_2d)): host array
   * [2*dim faces][ndir][face_stride] doubles, faces x-, x+, y-, y+, z-, z+;
   * face cells ordered with the lower remaining axis fastest.  Only entries
   * of directions entering through that face (u.n < 0) are read.  NULL means
   * zero inflow.  face_stride = 0 means the largest face's cell count. */
  const double* inflow;
  size_t inflow_face_stride;
} rte_medium;

typedef struct {
  int dim, nx, ny, nz, ndir;
  int kernel;             /* resolved RTE_HG_FLATLAND or RTE_HG_SPHERE            */
  int64_t cells, n;       /* n = ndir * cells                                    */
  double h, g;
  int has_fields;         /* CoeffNet fields were built for a model              */
  int scheme;             /* RTE_SCHEME_*; n = 2 ndir cells for TFPS              */
  int64_t nbasis;         /* TFPS: distinct per-cell eigen-bases (one per medium
                             ratio), each 2 ndir (ndir + 1) doubles; else 0      */
} rte_operator_info;

/* Build the operator: validate inputs, form S, the scaled coefficients and
 * the right-hand side b in FP64 on the host, upload them, and -- when
 * `model` is not NULL -- run CoeffNet on the device to produce the per-level
 * fields a^[l], a^{-1,[l]} that MgNet reads (Sec. 3.2).  The model must
 * match the geometry (dim, ndir; every extent divisible by 2^(levels-1)).
 * The returned handle is immutable and may be shared by concurrent solves;
 * the model must outlive it.  Errors: RTE_EINVAL (bad geometry or medium),
 * RTE_ENOMEM, RTE_EDEVICE.  Synchronises `stream` before returning. */
rte_status rte_build_operator(const rte_geometry* geom, const rte_medium* med,
                              const mgnet_model* model, void* stream, rte_operator** out);
rte_status rte_operator_free(rte_operator* op);
rte_status rte_operator_get_info(const rte_operator* op, rte_operator_info* info);

/* Copy an internal array of the operator into caller device memory, for
 * inspection and testing.  which / layout / bytes:
 *   RTE_ARR_RHS     b,            FP64 [ndir][cells]
 *   RTE_ARR_SCATTER S,            FP64 [ndir][ndir] row-major
 *   RTE_ARR_SIGMA   (sT, sA),     FP64 [2][cells]   (sA = eps sigma_a)
 *   RTE_ARR_FIELD_A a^[level],    FP32 [cells_l][C_l] (channels fastest)
 *   RTE_ARR_FIELD_AINV a^{-1,[level]}, same layout
 * `bytes` must equal the array size.  Errors: RTE_EINVAL. */
enum { RTE_ARR_RHS = 0, RTE_ARR_SCATTER = 1, RTE_ARR_SIGMA = 2,
       RTE_ARR_FIELD_A = 3, RTE_ARR_FIELD_AINV = 4 };
rte_status rte_operator_copy_array(const rte_operator* op, int which, int level,
                                   void* dst, size_t bytes, void* stream);

/* Parse and validate an MGN1 weights blob (CoeffNet + MgNet of Sec. 3.2-3.3;
 * FP32 tensors; layout documented with the weights writer).  Host-only: the
 * weights are uploaded to a device on first use.  The blob may be freed
 * after return.  Errors: RTE_EFORMAT (bad magic, version, truncation,
 * missing/duplicate/misshapen tensors, trailing bytes), RTE_EINVAL. */
rte_status mgnet_load(const void* blob, size_t bytes, mgnet_model** out);
rte_status mgnet_free(mgnet_model* model);
/* dims_out[8] = {dim, ndir, c0, levels, nu_pre, nu_post, nu_coarse, coef_ch}. */
rte_status mgnet_describe(const mgnet_model* model, int* dims_out);

/* y = L x (paper eq. (DORTE_2d), discretised as above).  precision RTE_FP32:
 * x, y are float [n]; RTE_FP64: double [n].  x and y must not overlap.
 * Errors: RTE_EINVAL. */
rte_status rte_apply(const rte_operator* op, const void* x, void* y, int precision, void* stream);

/* r = b - L x in FP64 (double [n] each; may not overlap).  Errors: RTE_EINVAL. */
rte_status rte_residual(const rte_operator* op, const double* x, double* r, void* stream);

/* psi_m at every cell centre from a solution x of the operator's system:
 * device double [ndir][cells] (direction-major).  UPWIND: a copy of x.  TFPS:
 * eq. (2DTFPS_sol) evaluated at the centres, sum_k x_k chi^k + the particular
 * solution.  x (device double [n]) and psi must not overlap.  Errors:
 * RTE_EINVAL. */
rte_status rte_cell_values(const rte_operator* op, const double* x, double* psi, void* stream);

/* Adaptive tailored finite point scheme (Sec. 2.3) on a TFPS operator (scheme
 * RTE_SCHEME_TFPS, 2D).  rte_atfps_build selects, per cell, the basis functions
 * whose value at the cell centre exp(-|xi| sigma_T h / 2) exceeds delta (eq.
 * (def_V_delta)), builds every face's interface basis (the kept functions
 * centred on the face orthonormalised by a QR factorisation and scaled to
 * max-norm 1, first near-largest entry positive; then the dropped functions'
 * eigenvectors scaled to max-norm 1), and assembles in FP64 on the host:
 *   - the compressed system A_d alpha = b_d of eq. (2DAdaptiveTFPS_linear_sys):
 *     per face, the projections of the continuity (or inflow) condition onto
 *     the face's kept basis vectors, with the kept functions of both cells;
 *   - the layer reconstruction of eq. (2DAdaptive_TFPS_layer1) and
 *     (2DAdaptive_TFPS_layer2): each dropped coefficient is the projection of
 *     the jump of the smooth solution across its face (or of the inflow data
 *     minus the smooth solution) onto its own basis vector;
 *   - the filtered loss of eq. (loss_delta), ||b_d - A_d D_d psi||_2, with D_d
 *     the per-cell minimum-norm least-squares fit of the cell-centre values
 *     minus the particular solution by the kept functions.
 * Rows: x faces x_0..x_I of each grid row (i fastest), then y faces y_0..y_I
 * of each grid column; within a face its kept basis vectors in order.
 * Unknowns alpha (n_kept = n_rows of them): the kept coefficients cell by cell
 * (x fastest), each cell's kept local indices ascending (local order of the
 * TFPS operator).  The maps are uploaded as sparse rows to the current
 * device; the evaluations below launch on `stream` and do not synchronise.
 * delta in [0, 1); delta = 0 keeps every function.  When nothing is kept
 * (n_kept = 0) alpha and rho may be NULL.  The operator must outlive the
 * handle.  Errors: RTE_EINVAL (not a TFPS operator, bad delta,
 * singular face basis), RTE_ENOMEM, RTE_EDEVICE. */
rte_status rte_atfps_build(const rte_operator* op, double delta, rte_atfps** out);
rte_status rte_atfps_free(rte_atfps* a);
/* n_kept: unknowns, n_rows: rows of A_d (equal), nnz: stored entries of A_d.
 * Any output may be NULL. */
rte_status rte_atfps_get_info(const rte_atfps* a, int64_t* n_kept, int64_t* n_rows, int64_t* nnz);
/* r = b_d - A_d alpha.  alpha, r: device double [n_kept]; must not overlap. */
rte_status rte_atfps_residual(const rte_atfps* a, const double* alpha, double* r, void* stream);
/* All 2 ndir coefficients of every cell from the kept ones: the kept ones
 * copied, the dropped ones by layer reconstruction.  alpha: device double
 * [n_kept]; coef: device double [cells][2 ndir] (the TFPS operator's unknown
 * layout, so rte_cell_values evaluates it); must not overlap. */
rte_status rte_atfps_reconstruct(const rte_atfps* a, const double* alpha, double* coef, void* stream);
/* rho = b_d - A_d D_d psi and *loss = ||rho||_2 (eq. (loss_delta)).  psi:
 * device double [ndir][cells] cell-centre values (direction-major, the layout
 * of rte_cell_values); rho: device double [n_rows]; loss: device double [1].
 * psi and rho must not overlap. */
rte_status rte_atfps_filtered_loss(const rte_atfps* a, const double* psi, double* rho, double* loss,
                                   void* stream);

/* z = M(v): one MgNet V-cycle (Sec. 3.3) with the operator's CoeffNet
 * fields (precond RTE_PC_MGNET_BF16 or RTE_PC_MGNET_FP32), or the
 * Block-Jacobi solve (RTE_PC_BLOCK_JACOBI; model, workspace may be NULL).
 * v: device double [n]; z: device float [n].  The workspace (device memory
 * of at least rte_precond_workspace_bytes) holds the level activations.
 * Errors: RTE_EINVAL (no fields built, model mismatch, more than
 * RTE_BJ_MAX_DIRS directions for Block-Jacobi), RTE_ENOMEM (small workspace). */
rte_status rte_precond_workspace_bytes(const rte_operator* op, const mgnet_model* model,
                                       size_t* bytes);
rte_status rte_precond_apply(const rte_operator* op, const mgnet_model* model, int precond,
                             const double* v, float* z, void* workspace, size_t ws_bytes,
                             void* stream);

/* Environment switches read by the library (for comparisons and profiling;
 * results do not depend on them): RTE_GRAPHS=0 runs the Arnoldi steps of
 * rte_solve and the server eagerly instead of as HIP graphs captured per
 * step shape; RTE_T_BF16=0 stores every intermediate t of the BF16 V-cycle
 * (the tensors that only feed convolutions) in FP32 instead of bfloat16;
 * RTE_APPLY64_VEC=1 runs the FP64 apply and residual on the vector kernel
 * instead of the FP64 matrix cores (16, 32, 64 or 96 directions). */
/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the MgNet
 * V-cycle of rte_precond_apply (precond RTE_PC_MGNET_BF16 or
 * RTE_PC_MGNET_FP32 only), with the level activations in a device array
 * owned by the library instead of a caller workspace.  The array holds
 * 64 MiB (RTE_NOALLOC_SCRATCH_BYTES) on each device the library runs on,
 * kept until the process ends; a V-cycle whose rte_precond_workspace_bytes
 * exceeds it is rejected with RTE_ENOMEM.  The call allocates no device
 * memory: the model's weights must already be on the current device (they
 * are once an operator has been built with the model on it).  Every call on
 * one device uses that device's one array, so calls that overlap on one
 * device (concurrent streams or threads) race and give undefined results;
 * serialise them.  Nothing in the array needs to start at zero (each
 * V-cycle writes every activation before reading it).  v: device double
 * [n]; z: device float [n]; results equal rte_precond_apply's bit for bit.
 * Errors: RTE_EINVAL (null argument, other preconditioner, operator not
 * built with this model, weights not on the current device), RTE_ENOMEM,
 * RTE_EDEVICE. */
#define RTE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rte_status rte_precond_apply_noalloc(const rte_operator* op, const mgnet_model* model, int precond,
                                     const double* v, float* z, void* stream);

/* One convolution of the MgNet V-cycle (Sec. 3.3) with its fused pointwise
 * epilogue, run over `nslots` independent inputs in one launch exactly as
 * the V-cycle runs it: an inspection and test hook for the convolution
 * kernels.
 *   which, level, index select the weights: MGN_W_A (A_level), MGN_W_BPRE
 *     (B_level^(index), before the restriction), MGN_W_BPOST (after the
 *     prolongation), MGN_W_BCOARSE (coarsest level, B^(index)), MGN_W_R
 *     (R_level: kernel 3, stride 2, channels C -> 2C), MGN_W_PR (Pr_level:
 *     kernel 4, stride 2, transposed, 2C -> C, input on level + 1's grid);
 *   precond: RTE_PC_MGNET_BF16 (input and weights rounded to bfloat16, nearest
 *     even, products accumulated in FP32) or RTE_PC_MGNET_FP32;
 *   in_dim: the input grid (cells along x, y, z; 1 for an unused z);
 *   epilogue, with conv the convolution of `in` (zero padding outside the grid):
 *     MGN_EPI_STORE    out = conv
 *     MGN_EPI_ACCUM    out = out + conv
 *     MGN_EPI_STORE_T  out = conv, out2 = ainv (.) conv
 *     MGN_EPI_RESID_R  out = f - conv - a (.) in          (3x3 stride 1 only)
 *     MGN_EPI_RESID_T  out = ainv (.) (f - conv - a (.) in) (3x3 stride 1 only)
 *   Every array is device FP32, channels-last [pixels][channels] with pixels
 *   x fastest; f, a, ainv and out2 have the output's shape (NULL where the
 *   epilogue does not read them).  Slot s's arrays begin s * slot_stride
 *   bytes after slot 0's (one stride for every array; slot_stride is ignored
 *   when nslots is 1).
 *   table: device memory of at least 128 * nslots bytes for the launch's slot
 *   table, or NULL when nslots is 1.
 * Synchronises `stream` before returning.  Errors: RTE_EINVAL (unknown
 * weights or epilogue, grid not matching the level, null array). */
enum { MGN_W_A = 0, MGN_W_BPRE = 1, MGN_W_BPOST = 2, MGN_W_BCOARSE = 3, MGN_W_R = 4, MGN_W_PR = 5 };
enum { MGN_EPI_STORE = 0, MGN_EPI_ACCUM = 1, MGN_EPI_STORE_T = 2, MGN_EPI_RESID_R = 3,
       MGN_EPI_RESID_T = 4 };
rte_status mgnet_conv_apply(const mgnet_model* model, int precond, int which, int level, int index,
                            int epilogue, const int* in_dim, int nslots, size_t slot_stride,
                            const float* in, float* out, float* out2, const float* f, const float* a,
                            const float* ainv, void* table, void* stream);

typedef struct {
  int restart;            /* Krylov cycle length k, 1..64 (paper: GMRES)          */
  double rtol;            /* stop when ||b - L x||_2 <= rtol ||b||_2, checked in FP64 */
  int max_iters;          /* total inner iterations, >= 1                         */
  int precond;            /* RTE_PC_*                                             */
  const double* x0;       /* device double [n] initial guess, or NULL for zero    */
  const double* b;        /* device double [n] right-hand side, or NULL for the built b */
} rte_solve_opts;

typedef struct {
  int iterations;         /* inner FGMRES steps taken                             */
  int restarts;           /* completed cycles                                     */
  int converged;          /* 1 if the FP64 true residual met rtol                 */
  int status;             /* the rte_status the solve ended with                  */
  double rel_residual;    /* ||b - L x||_2 / ||b||_2 in FP64 at exit              */
  double ms_total;        /* wall time of the solve                               */
} rte_solve_stats;

/* Workspace for rte_solve: a one-slot batch table, the iterate and right-hand
 * side (FP64), Krylov bases V (FP64, k+1 vectors), Z (FP32, k vectors),
 * reduction scratch and, for MgNet, the level activations.
 * Errors: RTE_EINVAL. */
rte_status rte_workspace_bytes(const rte_operator* op, const mgnet_model* model,
                               const rte_solve_opts* opts, size_t* bytes);

/* Right-preconditioned flexible GMRES(k) (Krylov solve of Sec. 3 and Sec. 4.2,
 * flexible because the preconditioner runs in reduced precision): inner
 * operator applies and preconditioning in FP32 (or BF16 convolutions),
 * orthogonalisation (classical Gram-Schmidt with reorthogonalisation, the second
 * correction of each basis vector completed in the next step), Hessenberg least
 * squares and the restart residual b - L x in FP64 on the device.
 * psi_out: device double [n], the solution x (written when the solve ends;
 * the iterate lives in the workspace, so x0 may alias psi_out).
 * stats (host) is filled on RTE_OK, RTE_ENOCONV and RTE_EBREAKDOWN.
 * Blocks the calling thread until the solve ends.
 * Errors: RTE_EINVAL (also when psi_out, x0 or b is not device memory),
 * RTE_ENOMEM (workspace smaller than required), RTE_ENOCONV, RTE_EBREAKDOWN,
 * RTE_EDEVICE. */
rte_status rte_solve(const rte_operator* op, const mgnet_model* model, const rte_solve_opts* opts,
                     void* workspace, size_t ws_bytes, double* psi_out, rte_solve_stats* stats,
                     void* stream);

/* ---- serving: continuous batching of independent solves ----
 * A server owns a worker thread.  Requests are admitted in arrival order
 * while fewer than `max_slots` solves are active and the request's
 * workspace fits in the caller-provided device arena (admission by HBM
 * footprint).  Admitted requests of one shape (grid, directions, model,
 * restart length, preconditioner) form a batch: every kernel launch of a
 * batch covers all of its solves, each solve runs its own restart cycles
 * (the restart decision is taken on the device), a request that arrives
 * while the batch runs joins at the batch's next Arnoldi step, and a solve
 * that meets its tolerance stops taking steps without a host round trip.
 * Batches of
 * different shapes run on streams of their own and overlap on the device.
 * Finished solves free their arena range for the next request.  Each solve
 * performs exactly the arithmetic rte_solve performs, so its result does not
 * depend on what else is in flight (bitwise). */
typedef struct {
  int64_t submitted, completed, active, queued;
  size_t arena_bytes, arena_in_use, arena_peak;
} rte_server_stats;

/* arena: device memory of arena_bytes owned by the caller, which must
 * outlive the server; per-solve workspaces and each batch's slot table come
 * from it.  max_slots: 1..64, the most solves active at once and the width
 * of a batch.  Errors: RTE_EINVAL, RTE_EDEVICE. */
rte_status rte_server_create(void* arena, size_t arena_bytes, int max_slots, rte_server** out);
/* Queue a solve.  op, model and psi_out (device double [n]) must stay valid
 * until the ticket is polled as finished.  Errors: RTE_EINVAL, RTE_ENOMEM
 * (the request can never fit the arena), RTE_EAGAIN (queue of 4096 full). */
rte_status rte_submit(rte_server* srv, const rte_operator* op, const mgnet_model* model,
                      const rte_solve_opts* opts, double* psi_out, uint64_t* ticket);
/* Queue `count` solves at once, all or none: they become visible to the
 * worker together, so a burst of requests is admitted in the same tick
 * instead of trickling in one call at a time.  ops[i], models[i] (models may
 * be NULL, or an entry NULL, for no model), opts[i] (host array of count
 * option structs), psi_out[i] as for rte_submit; tickets (host uint64 [count])
 * receives the tickets in order.  Errors: as rte_submit, for the first
 * request that fails validation; then no request is queued. */
rte_status rte_submit_many(rte_server* srv, int count, const rte_operator* const* ops,
                           const mgnet_model* const* models, const rte_solve_opts* opts, double* const* psi_out,
                           uint64_t* tickets);
/* RTE_EAGAIN while queued or running; once finished, fills *stats (host,
 * may be NULL), forgets the ticket and returns the solve's own status
 * (RTE_EINVAL when psi_out, x0 or b turned out not to be device memory).
 * Errors: RTE_ENOTFOUND for an unknown or already collected ticket. */
rte_status rte_poll(rte_server* srv, uint64_t ticket, rte_solve_stats* stats);
rte_status rte_server_query(rte_server* srv, rte_server_stats* out);
/* Finish every queued and running request, then free the server. */
rte_status rte_server_destroy(rte_server* srv);

/* ---- kernel timing: HIP events around launches of one kernel class ----
 * rte_prof_enable(cls, every): every > 0 brackets every `every`-th launch of
 * the class with an event pair stamped by its dispatch (1 = all launches;
 * sampling keeps the events' own cost out of the timed work); 0 disables.
 * Enabling creates a pool of 8192 events up front, so that the timed launches
 * do not create them.
 * Solves replay their Arnoldi steps as HIP graphs, whose launches cannot be
 * bracketed; while any class is enabled a solve runs one step in `every`
 * without its graph and times every launch of the enabled classes in it.  rte_prof_query synchronises the recorded events and returns,
 * since the last reset, the summed duration, the number of timed launches,
 * their summed algorithmic work -- FLOPs for RTE_K_CONV
 * (2 x rows x cout x cin x taps), bytes for the bandwidth-bound classes,
 * 0 for RTE_K_PRECOND (a composite: the whole V-cycle) -- and their summed
 * algorithmic bytes (every operand read once, every result written once;
 * for RTE_K_CONV: input tensor, weights, output and epilogue tensors).
 * Any output pointer may be NULL. */
enum { RTE_K_APPLY = 0, RTE_K_RESIDUAL = 1, RTE_K_CONV = 2, RTE_K_ORTH = 3,
       RTE_K_PRECOND = 4, RTE_K_COUNT = 5 };
rte_status rte_prof_enable(int kernel_class, int every);
rte_status rte_prof_query(int kernel_class, double* total_ms, int64_t* launches, double* work,
                          double* bytes);
/* The same sums restricted to the launches of one key: for RTE_K_CONV the key
 * is floor(log2(output channels)) of the convolution (so the levels of a
 * V-cycle separate: C_l = C_0 2^l); for RTE_K_ORTH 1 = boundary dot products,
 * 2 = their second reduction stage, 3 = the lagged-CGS2 first pass (completes
 * V_j, forms V^T w), 4 = the second pass (w -= V h, V^T w), 5 = the Givens step;
 * for every other class 0.  Errors: RTE_EINVAL (class or key out of range). */
#define RTE_PROF_KEYS 16
rte_status rte_prof_query_key(int kernel_class, int key, double* total_ms, int64_t* launches, double* work,
                              double* bytes);
rte_status rte_prof_reset(void);

/* Message of the last failing call on this thread ("" if none). */
const char* rte_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTE_H */
