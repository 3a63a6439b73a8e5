/*
 * hexla.h - C ABI of an MI355X (gfx950) evaluator for compound linear-algebra
 * expressions.
 *
 * The library implements the expression-optimisation method of Sanderson &
 * Curtin, "Armadillo: An Efficient Framework for Numerical Linear Algebra"
 * (arXiv 2502.03000), on one GPU:
 *   - an expression is described first and evaluated only when asked for
 *     (delayed evaluation, Sec. II): builder calls record markers that hold
 *     references to matrices and copies of scalars, and nothing runs until
 *     hexla_execute;
 *   - element-wise sub-expressions of any length are fused into one pass with
 *     no temporaries (Sec. II, the Z = 0.4*X + 0.6*Y example);
 *   - sizes are checked when the expression is built (Sec. II);
 *   - inv(A)*B is solved by LU with partial pivoting without forming the
 *     inverse (Sec. I, Sec. II; expression (9) of Sec. III);
 *   - a product of one matrix with its own transpose runs as a symmetric
 *     rank-k update (Sec. II; expression (8) of Sec. III);
 *   - matrix chains are reordered by cost (Sec. II; expression (6) of
 *     Sec. III): by exact dynamic programming over multiply-add counts by
 *     default, or by the paper's own smallest-result-first rule.
 *
 * Conventions
 *   - Matrices are column-major with a leading dimension ld >= rows (ld >= 1
 *     when rows == 0), the storage of the BLAS/LAPACK routines the paper maps
 *     expressions onto. A vector is an n x 1 matrix.
 *   - Every function returns hexla_status. Out-parameters come last.
 *   - Operands, results and workspaces are always owned by the caller. The
 *     library never allocates device memory while executing. Its own
 *     allocations are a 256-byte status block per context
 *     (hexla_ctx_create), the code of generated element-wise kernels, a
 *     pinned host copy of each batch plan's instance table, and a learned
 *     cost model's parameters and scratch (hexla_model_*).
 *   - A context is used by one host thread at a time.
 *   - Plans, batch plans and models belong to the context that made them.
 *     Destroying the context first detaches them: afterwards they may only
 *     be destroyed (any other call returns HEXLA_E_INVALID_ARG), so the
 *     objects can be released in any order.
 *   - Errors left behind by HIP calls made outside the library are cleared
 *     when a call makes the context's device current; they are not
 *     reported as the library's.
 */
#ifndef HEXLA_H
#define HEXLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hexla_status {
  HEXLA_OK = 0,
  HEXLA_E_INVALID_ARG = 1,     /* null pointer, bad ld, aliasing, short workspace */
  HEXLA_E_DIM = 2,             /* non-conforming sizes (Sec. II size checks)      */
  HEXLA_E_DTYPE = 3,           /* mixed storage types in one expression           */
  HEXLA_E_NOT_SQUARE = 4,      /* inv()/solve() of a non-square matrix            */
  HEXLA_E_SINGULAR = 5,        /* deferred: exact zero pivot met during LU        */
  HEXLA_E_NO_CONVERGENCE = 6,  /* deferred: refinement hit its iteration cap      */
  HEXLA_E_UNSUPPORTED = 7,     /* expression form this library does not evaluate */
  HEXLA_E_DEVICE = 8           /* HIP error; text in hexla_last_error             */
} hexla_status;

typedef enum hexla_dtype { HEXLA_F64 = 0, HEXLA_F32 = 1 } hexla_dtype;

typedef enum hexla_op {
  /* unary */
  HEXLA_OP_TRANS = 1,  /* transpose (Op<.., op_htrans>, Fig. 3)                */
  HEXLA_OP_NEG = 2,    /* element-wise negation                                */
  HEXLA_OP_EXP = 3,    /* element-wise exponential                             */
  HEXLA_OP_INV = 4,    /* inverse marker (Op<.., op_inv>, Sec. II)             */
  HEXLA_OP_DIAG = 5,   /* main diagonal as a column vector, min(m,n) x 1
                          (diag(A*B) of expression (4), Sec. III)              */
  HEXLA_OP_DIAGMAT = 6,/* diagonal matrix: a vector v (n x 1 or 1 x n) gives
                          the n x n matrix with v on its diagonal; a matrix
                          keeps its diagonal, zeros elsewhere (expressions
                          (3), (4), (7))                                      */
  HEXLA_OP_TRACE = 7,  /* sum of the main diagonal, a 1 x 1 result
                          (expression (5))                                    */
  HEXLA_OP_SUBMAT = 8, /* submatrix view (made by hexla_submatrix only)       */
  /* binary */
  HEXLA_OP_TIMES = 16, /* matrix product, or scaling when one side is a scalar */
  HEXLA_OP_PLUS = 17,  /* element-wise sum (Glue<.., glue_plus>, Sec. II)      */
  HEXLA_OP_MINUS = 18, /* element-wise difference                              */
  HEXLA_OP_SCHUR = 19, /* element-wise product ("%")                           */
  HEXLA_OP_DIV = 20,   /* element-wise division                                */
  HEXLA_OP_SOLVE = 21  /* solve(A, B): X with A X = B                          */
} hexla_op;

typedef uint32_t hexla_node;            /* index into the context's node arena */
typedef struct hexla_ctx hexla_ctx;
typedef struct hexla_plan hexla_plan;
typedef struct hexla_model hexla_model;

/* ------------------------------------------------------------------ context */

/* device >= 0: a HIP device ordinal; kernels run on `stream` (a hipStream_t,
 * NULL = the default stream). device == -1: a dry-run context that builds and
 * plans without a GPU (hexla_execute then returns HEXLA_E_UNSUPPORTED).
 * Errors: HEXLA_E_INVALID_ARG (out NULL, device < -1), HEXLA_E_DEVICE. */
hexla_status hexla_ctx_create(int device, void* stream, hexla_ctx** out);
/* Frees nodes, the status block and every plan still owned by the context. */
hexla_status hexla_ctx_destroy(hexla_ctx* ctx);
hexla_status hexla_ctx_set_stream(hexla_ctx* ctx, void* stream);
/* Drops every node (plans already created stay valid). */
hexla_status hexla_ctx_clear_nodes(hexla_ctx* ctx);
/* Text of the last error on this context; valid until the next call on it. */
const char* hexla_last_error(const hexla_ctx* ctx);

/* ------------------------------------------------------------- IR builder
 * Markers hold references to matrices and copies of scalars (Sec. II).      */

/* A leaf BORROWS `ptr` (device memory, column-major, rows x cols, leading
 * dimension ld). The memory must stay valid until the last hexla_execute that
 * reads it has completed in stream order. Two leaves with the same
 * (ptr, rows, cols, ld, dtype) are the same matrix (this identity is what the
 * symmetric-product rewrite checks; equal values in distinct buffers are not
 * detected). Errors: HEXLA_E_INVALID_ARG (rows/cols < 0, ld < max(rows,1),
 * ptr NULL with rows*cols > 0, bad dtype). */
hexla_status hexla_leaf(hexla_ctx* ctx, const void* ptr, int64_t rows, int64_t cols,
                        int64_t ld, hexla_dtype dtype, hexla_node* out);
/* A scalar, copied. It broadcasts in element-wise operations and scales in
 * products. */
hexla_status hexla_scalar(hexla_ctx* ctx, double value, hexla_node* out);
/* Errors: HEXLA_E_INVALID_ARG (bad node or op), HEXLA_E_NOT_SQUARE (INV of a
 * non-square matrix). */
hexla_status hexla_unary(hexla_ctx* ctx, hexla_op op, hexla_node a, hexla_node* out);
/* Sizes are checked here (Sec. II): HEXLA_E_DIM for non-conforming operands,
 * HEXLA_E_NOT_SQUARE for solve() with a non-square left side, HEXLA_E_DTYPE
 * when the operands' storage types differ. */
hexla_status hexla_binary(hexla_ctx* ctx, hexla_op op, hexla_node a, hexla_node b,
                          hexla_node* out);
/* Submatrix view (expression (2) of Sec. III: columns and rows accessed in
 * place): rows [r0, r0 + rows) and columns [c0, c0 + cols) of `a` (0-based;
 * a column A(:, j) is (0, j, m, 1), a row B(i, :) is (i, 0, 1, n)). A view of
 * a leaf borrows the leaf's storage with its leading dimension; a view of
 * any other node views its evaluated value. Errors: HEXLA_E_DIM (the range
 * leaves the operand), HEXLA_E_INVALID_ARG (negative sizes, scalar). */
hexla_status hexla_submatrix(hexla_ctx* ctx, hexla_node a, int64_t r0, int64_t c0,
                             int64_t rows, int64_t cols, hexla_node* out);
/* Shape of a node (a scalar is 1 x 1 with *is_scalar = 1). */
hexla_status hexla_node_shape(const hexla_ctx* ctx, hexla_node n, int64_t* rows,
                              int64_t* cols, int32_t* is_scalar);

/* ---------------------------------------------------------------- planner */

typedef enum hexla_planner {
  HEXLA_PLANNER_DP = 0,      /* exact minimum multiply-adds over all bracketings */
  HEXLA_PLANNER_GREEDY = 1,  /* Sec. II rule: smallest-result pair first, leftmost on ties */
  HEXLA_PLANNER_NAIVE = 2,   /* Sec. III "naive": left to right, no rewrites     */
  HEXLA_PLANNER_LEARNED = 3, /* predicted-time DP with the context's cost model,
                                checked by the DP (see hexla_ctx_set_model)     */
  HEXLA_PLANNER_ROOFLINE = 4 /* exact minimum over all bracketings of the summed
                                roofline times max(flops / peak, bytes / 8 TB/s)
                                of the products (peak: the MFMA rate of the
                                product precision); not in the paper        */
} hexla_planner;

typedef enum hexla_product_precision {
  HEXLA_PRODUCT_PLAIN = 0,   /* products in the storage type                     */
  HEXLA_PRODUCT_BF16X3 = 1,  /* FP32 products as 3 BF16 MFMA products (hi/lo split) */
  HEXLA_PRODUCT_BF16X6 = 2   /* FP32 products as 6 BF16 MFMA products (3-term split) */
} hexla_product_precision;

/* Mixed-precision forms apply to FP64 systems (iterative refinement with a
 * low-precision factorisation; the paper names reduced-precision types as
 * future work, Sec. IV). The LU is stored in FP32 and its panels are factored
 * in FP32 (IR_FP32) or in FP64, pivots chosen on FP64 values and the panel
 * rounded to FP32 when stored (IR_FP16, IR_BF16X3, IR_BF16X6). The trailing
 * updates run in the form's product precision with FP32 accumulation, except
 * the next panel's 64 columns, which the next panel waits for: those are
 * updated in FP32 (about 96 / n of the update's products). The residual
 * R = B - S X and the update X += D are FP64, D solved on the low-precision
 * factors. The loop stops when ||R||inf <= ir_tol_scale * 2^-53 * ||S||inf *
 * ||X||inf (ir_tol_scale 0: 1; converged), when ir_max_iter is reached, when
 * a correction is larger than the previous one (it is dropped) or when it is
 * larger than half the previous one (it is applied: stagnation). A stagnated
 * solve whose last residual's backward error ||R||/(||S|| ||X||) exceeds
 * n * 2^-53, a diverging one and a capped one raise the deferred
 * HEXLA_E_NO_CONVERGENCE; hexla_sync reports the iterations and that
 * backward error. The loop reads a small status block after every step, so
 * hexla_execute of such a plan returns only when the solve is done and the
 * plan cannot be captured. */
typedef enum hexla_solve_precision {
  HEXLA_SOLVE_PLAIN = 0,     /* LU and substitution in the storage type          */
  HEXLA_SOLVE_IR_FP32 = 1,   /* FP32 LU (FP32 panels), FP32 trailing updates      */
  HEXLA_SOLVE_IR_FP16 = 2,   /* FP32 LU, FP64 panels, FP16-MFMA trailing updates
                                (FP32 accumulation)                              */
  HEXLA_SOLVE_IR_BF16X3 = 3, /* FP32 LU, FP64 panels, split-BF16 (x3) MFMA
                                trailing updates                                 */
  HEXLA_SOLVE_IR_BF16X6 = 4  /* FP32 LU, FP64 panels, split-BF16 (x6) MFMA
                                trailing updates                                 */
} hexla_solve_precision;

typedef struct hexla_plan_opts {
  int32_t planner;            /* hexla_planner                                   */
  int32_t product_precision;  /* hexla_product_precision                         */
  int32_t solve_precision;    /* hexla_solve_precision                           */
  int32_t fuse;               /* 1: fuse element-wise subtrees (default); 0: one
                                 kernel and one temporary per operation          */
  int32_t syrk;               /* 1: X^T X / X X^T on one leaf -> SYRK (default)  */
  int32_t ir_max_iter;        /* refinement cap (default 30; 0: none; < 0: 30)   */
  double ir_tol_scale;        /* stop when ||R||inf <= scale*2^-53*||S||inf*||X||inf;
                                 0 = 1                                           */
  int32_t solve_structure;    /* 0: solve() examines the system matrix when the
                                 plan runs and picks a solver for its structure
                                 (hexla_solver; default); 1: LU always. Plain
                                 precision only; a plan that examines cannot be
                                 captured                                        */
  int32_t codegen;            /* 1: element-wise passes run as kernels generated
                                 for the expression (hipRTC, default); 0: the
                                 program interpreter kernel                     */
  int32_t reserved[6];
} hexla_plan_opts;

/* Fills the defaults: DP, plain precision, fusion on, SYRK on, cap 30,
 * generated element-wise kernels on. */
hexla_status hexla_plan_opts_default(hexla_plan_opts* opts);

/* Plans the evaluation of `root` (opts NULL = defaults). Host only: nothing
 * is launched. The plan copies every leaf descriptor it needs, so nodes may
 * be cleared afterwards. Errors: HEXLA_E_INVALID_ARG, HEXLA_E_UNSUPPORTED
 * (e.g. a scalar-valued root), HEXLA_E_DTYPE. */
hexla_status hexla_plan_create(hexla_ctx* ctx, hexla_node root, const hexla_plan_opts* opts,
                               hexla_plan** out);

typedef struct hexla_plan_info {
  int64_t rows, cols;         /* shape of the result                             */
  int32_t dtype;              /* hexla_dtype of the result                       */
  int32_t n_steps;            /* kernels launched per execute (upper bound)       */
  uint64_t workspace_bytes;   /* workspace hexla_execute needs (may be 0)        */
  double flops;               /* algorithmic flops of the chosen plan            */
  double bytes;               /* algorithmic HBM bytes (each operand once)       */
  double chain_macs;          /* multiply-adds of the chosen chain orders        */
} hexla_plan_info;

hexla_status hexla_plan_get_info(const hexla_plan* plan, hexla_plan_info* out);
/* JSON description of the plan (the analogue of the paper's call trace,
 * Fig. 3): steps, kernels, shapes, flops, bytes. Writes at most cap bytes
 * (NUL-terminated when cap > 0) and the full length (without NUL) to *needed. */
hexla_status hexla_plan_describe(const hexla_plan* plan, char* buf, size_t cap, size_t* needed);
hexla_status hexla_plan_destroy(hexla_plan* plan);

/* -------------------------------------------------------------- evaluator */

/* Evaluates the plan on the context's stream, asynchronously. `out` is
 * caller-owned device memory for the rows x cols result with leading dimension
 * ld_out >= max(rows,1); `workspace` is caller-owned device memory of at least
 * workspace_bytes (256-byte aligned), or NULL when that is 0. The workspace
 * and out must not overlap each other or any leaf read by a product, solve or
 * transpose of the plan (element-wise-only plans may write in place).
 * Errors (synchronous): HEXLA_E_INVALID_ARG, HEXLA_E_DEVICE,
 * HEXLA_E_UNSUPPORTED (dry-run context). Numerical failures are deferred to
 * hexla_sync. */
hexla_status hexla_execute(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                           size_t workspace_bytes);

/* Evaluates the plan like hexla_execute, with its intermediates in a static
 * device array of the library instead of a caller-provided workspace: for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation). No device memory
 * is allocated or freed by this call. The array holds
 * hexla_static_scratch_bytes() bytes (64 MiB) on each device, kept until the
 * process ends; a plan whose workspace_bytes exceeds it is rejected with
 * HEXLA_E_INVALID_ARG. All calls on one device share that device's array:
 * calls that overlap in time on one device (two streams or threads) race.
 * `out` and ld_out, ownership, aliasing rules and errors are those of
 * hexla_execute. */
hexla_status hexla_execute_static(hexla_plan* plan, void* out, int64_t ld_out);
hexla_status hexla_static_scratch_bytes(size_t* bytes);

/* Solvers a structure-aware solve chooses (expression (10) of Sec. III: the
 * matrix is analysed and a tailored solver used): S diagonal -> division;
 * lower / upper triangular -> blocks of 64 rows, each solved as the product
 * with its diagonal block's inverse (the inverse's error grows with the
 * condition number of that 64 x 64 block, as in GPU BLAS triangular
 * solves); tridiagonal -> elimination with partial pivoting between
 * adjacent rows, back substitution by the pivots' reciprocals; symmetric
 * (S_ij and S_ji within n u max|S|, u the unit roundoff: the rounding
 * differences of a product X X^T formed by a general GEMM; the
 * factorisation reads the lower triangle) with a positive diagonal, or
 * S = X X^T known from the expression (the solve of Sec. IV's call trace) -> Cholesky by blocks
 * of 64 (each diagonal block inverted for the block column below it and for
 * the substitutions), falling back to LU if a pivot is not positive;
 * anything else -> LU with partial pivoting. */
typedef enum hexla_solver {
  HEXLA_SOLVER_LU = 0,
  HEXLA_SOLVER_CHOLESKY = 1,
  HEXLA_SOLVER_LOWER = 2,
  HEXLA_SOLVER_UPPER = 3,
  HEXLA_SOLVER_TRIDIAGONAL = 4,
  HEXLA_SOLVER_DIAGONAL = 5
} hexla_solver;

typedef struct hexla_report {
  int32_t status;             /* deferred hexla_status of the work since the last sync */
  int32_t ir_iterations;      /* refinement iterations of the last refined solve */
  int64_t singular_column;    /* first zero-pivot column (or -1)                 */
  double ir_backward_error;   /* ||R||inf / (||S||inf ||X||inf) of the last
                                 residual that refined solve formed            */
  int32_t solver;             /* hexla_solver of the last structure-aware solve,
                                 -1 if none ran since the last sync             */
  int32_t reserved;
} hexla_report;

/* Waits for the context's stream, then reports (and clears) the deferred
 * status: HEXLA_E_SINGULAR (exact zero pivot; the result is unspecified),
 * HEXLA_E_NO_CONVERGENCE (a refined solve hit its cap, its correction grew,
 * or it stagnated with a backward error above n * 2^-53). `report` may be NULL. The
 * return value is HEXLA_E_DEVICE on a HIP error, else HEXLA_OK. */
hexla_status hexla_sync(hexla_ctx* ctx, hexla_report* report);

/* The bfloat16 terms the split-BF16 products use (BF16 as a type for
 * higher-precision results: Sec. IV). For FP32 x[i] (device memory):
 * t0 = rne(x), t1 = rne(x - t0) and, when terms == 3, t2 = rne(x - t0 - t1),
 * rne = round to nearest, ties to even; outputs are raw bfloat16 bit
 * patterns (device memory, n entries each). Asynchronous on the context's
 * stream. Errors: HEXLA_E_INVALID_ARG (terms not 2 or 3, null pointers),
 * HEXLA_E_UNSUPPORTED (dry-run context), HEXLA_E_DEVICE. */
hexla_status hexla_split_bf16(hexla_ctx* ctx, const float* x, int64_t n, uint16_t* t0,
                              uint16_t* t1, uint16_t* t2, int32_t terms);

/* ------------------------------------------------------- tuning and graphs */

/* Times every candidate tile / split-K configuration of each matrix product
 * of the plan on these buffers (valid as for hexla_execute; their contents
 * are overwritten), keeps the fastest in the plan and records it in the
 * context's tuning table, which later hexla_plan_create calls consult.
 * reps: timed launches per candidate (<= 0: 5). Synchronous. Errors: as
 * hexla_execute. */
hexla_status hexla_plan_autotune(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                                 size_t workspace_bytes, int32_t reps);
/* Writes / reads the tuning table as text, one "gfx950 key tile split" line
 * per entry. Loading rejects a table made for another target
 * (HEXLA_E_INVALID_ARG). */
hexla_status hexla_tune_save(const hexla_ctx* ctx, const char* path);
hexla_status hexla_tune_load(hexla_ctx* ctx, const char* path);

/* Records the plan's launches, bound to these buffers, into a HIP graph owned
 * by the plan (replacing any earlier capture); hexla_plan_replay launches it
 * on the context's stream. Useful when the same expression is evaluated on
 * the same buffers many times. Errors: as hexla_execute. */
hexla_status hexla_plan_capture(hexla_plan* plan, void* out, int64_t ld_out, void* workspace,
                                size_t workspace_bytes);
hexla_status hexla_plan_replay(hexla_plan* plan);

/* ---------------------------------------------------------------- batches
 * Many small instances of one vector expression, evaluated by one persistent
 * launch: each workgroup takes instances, largest first, from a queue and
 * runs the whole expression on one instance with its intermediate vectors in
 * on-chip memory. This is the same delayed evaluation (Sec. II) applied to a
 * batch: one plan, made once from a template expression, evaluates every
 * instance.
 *
 * The template is an expression over leaves of two shapes, t x t (matrices)
 * and t x 1 (vectors) for one t >= 2 (the template leaves' pointers are not
 * read), whose result is t x 1. Instance i binds every template leaf to an
 * n_i x n_i or n_i x 1 matrix, 1 <= n_i <= 512 (n_i == 0: nothing is written).
 * Supported forms:
 *   - products whose last factor is vector-valued; the other factors are
 *     matrix leaves, trans(leaf), inv(leaf) and scalars. They run right to
 *     left as matrix-vector products (with square factors that is the
 *     order the chain-cost minimisation of Sec. II picks: any other
 *     bracketing multiplies two n x n matrices);
 *   - solve(leaf, v) and inv(leaf) * v: LU with partial pivoting of the
 *     instance's matrix (Sec. I, Sec. II), without forming the inverse;
 *   - element-wise + - % / exp, unary minus and scalars over vectors, fused
 *     into one pass (Sec. II).
 * Other forms give HEXLA_E_UNSUPPORTED at creation. */
typedef struct hexla_batch hexla_batch;

typedef struct hexla_batch_info {
  int64_t count;              /* instances                                       */
  int64_t max_n;              /* largest instance size                          */
  int32_t dtype;              /* hexla_dtype                                     */
  int32_t n_ops;              /* operations of the per-instance program          */
  int32_t panel;              /* LU panel width of the chosen configuration      */
  int32_t threads;            /* threads per workgroup                           */
  int32_t grid;               /* workgroups of the persistent launch             */
  int32_t reserved;
  uint64_t workspace_bytes;   /* workspace hexla_batch_execute needs             */
  double flops;               /* algorithmic flops of all instances              */
  double bytes;               /* algorithmic HBM bytes (each operand once)       */
} hexla_batch_info;

/* Creates a batch plan. `leaves` lists the template's leaf nodes (n_leaves <=
 * 8); leaf_ptrs[i * n_leaves + l] is instance i's device pointer for leaf l,
 * with leading dimension lds[i * n_leaves + l] (lds NULL: n_i for every
 * leaf); outs[i] receives instance i's n_i x 1 result; sizes[i] = n_i. All
 * arrays are host memory, read during this call only; the device pointers
 * are borrowed and must stay valid while the plan is used. Outputs may not
 * overlap each other or any input. Host only apart from the plan's pinned
 * host copy of the instance table. opts: planner and precision fields are
 * ignored. Errors: HEXLA_E_INVALID_ARG (null pointers, ld < n_i, overlapping
 * outputs, a template leaf listed twice or missing), HEXLA_E_DIM (template
 * shapes), HEXLA_E_UNSUPPORTED (form or n_i > 512), HEXLA_E_DTYPE. */
hexla_status hexla_batch_create(hexla_ctx* ctx, hexla_node root, const hexla_node* leaves,
                                int32_t n_leaves, int64_t count, const int64_t* sizes,
                                const void* const* leaf_ptrs, const int64_t* lds,
                                void* const* outs, const hexla_plan_opts* opts,
                                hexla_batch** out);
hexla_status hexla_batch_get_info(const hexla_batch* batch, hexla_batch_info* out);
/* JSON description: the per-instance program and the launch configuration. */
hexla_status hexla_batch_describe(const hexla_batch* batch, char* buf, size_t cap,
                                  size_t* needed);
/* Evaluates every instance on the context's stream, asynchronously: copies
 * the instance table into the workspace (caller-owned device memory of at
 * least workspace_bytes, 256-byte aligned), then one persistent launch. An
 * exact zero pivot is deferred to hexla_sync as HEXLA_E_SINGULAR, with the
 * index of a singular instance in singular_column. Errors: HEXLA_E_INVALID_ARG
 * (short workspace), HEXLA_E_UNSUPPORTED (dry-run context), HEXLA_E_DEVICE. */
hexla_status hexla_batch_execute(hexla_batch* batch, void* workspace, size_t workspace_bytes);
/* Times every launch configuration (LU panel width, threads per workgroup,
 * workgroups) on this workspace (reps timed launches each, <= 0: 3) and keeps
 * the fastest. Synchronous. Errors: as hexla_batch_execute. */
hexla_status hexla_batch_autotune(hexla_batch* batch, void* workspace, size_t workspace_bytes,
                                  int32_t reps);
/* Selects the launch configuration by hand: LU panel width and threads per
 * workgroup name one of the compiled variants (hexla_batch_describe lists the
 * chosen one), grid is 1..the largest grid the workspace was sized for
 * (768). A captured graph is dropped. Host only. Errors: HEXLA_E_INVALID_ARG
 * (no such variant, grid out of range). */
hexla_status hexla_batch_set_config(hexla_batch* batch, int32_t panel, int32_t threads,
                                    int32_t grid);
/* Copies the instance table into the workspace, waits for it, then records
 * the launches into a HIP graph owned by the batch (replacing any earlier
 * capture); hexla_batch_replay launches the graph on the context's stream.
 * Between capture and the last replay the workspace keeps the instance table
 * and must not be written by the caller. Errors: as hexla_batch_execute. */
hexla_status hexla_batch_capture(hexla_batch* batch, void* workspace, size_t workspace_bytes);
hexla_status hexla_batch_replay(hexla_batch* batch);
hexla_status hexla_batch_destroy(hexla_batch* batch);

/* ------------------------------------------------------- learned planner
 * A small FP32 network (32 features -> 64 -> 64 -> 64 -> 1, ReLU) predicts
 * the log of a matrix product's run time in microseconds from its shape,
 * type, transposes and launch configuration (tile, split-K). It is trained on
 * the GPU by the library's own kernels (MSE loss, Adam) on timings the
 * evaluator measures itself: hexla_timing_log makes hexla_plan_autotune
 * append every configuration it times to a file. Nothing of this is in the
 * paper, whose chain rule is the greedy heuristic of Sec. II; it is a
 * planner variant beside the cost-count DP.
 *
 * With a model set on the context, HEXLA_PLANNER_LEARNED plans each chain by
 * a DP over predicted times (each product at its predicted-fastest
 * configuration; one inference launch per chain, on the context's stream,
 * waited for by hexla_plan_create). The multiply-add DP has the last word: the
 * learned order is kept only when its multiply-adds are at most twice the
 * DP's and its predicted time is below the predicted time of the DP order;
 * otherwise the DP order is used. Configurations in the context's tuning
 * table (measured) take precedence over predicted ones. Without a model the
 * learned planner is the DP planner. A model holds its parameters and Adam
 * state in device memory allocated at creation (about 126 KB), and
 * inference scratch grown on demand. */
#define HEXLA_MODEL_FEATURES 32

typedef struct hexla_train_opts {
  int32_t epochs;             /* passes over the data (default 200)              */
  int32_t batch;              /* samples per Adam step (default 256)             */
  float lr;                   /* Adam step size (default 1e-3; betas 0.9, 0.999) */
  int32_t reserved0;
  uint64_t seed;              /* shuffling seed                                  */
  int32_t reserved[8];
} hexla_train_opts;

/* The feature vector (HEXLA_MODEL_FEATURES floats, host memory) of a product
 * C = op(A) op(B), op(A) m x k, op(B) k x n, in configuration (tile, split)
 * of the kernel family of (dtype, precision); mode 1 = symmetric (SYRK).
 * Errors: HEXLA_E_INVALID_ARG. */
hexla_status hexla_product_features(int32_t dtype, int32_t precision, int32_t mode, int32_t ta,
                                    int32_t tb, int64_t m, int64_t n, int64_t k, int32_t tile,
                                    int32_t split, float* out);
/* A network with He-normal weights drawn from `seed`, zero biases. */
hexla_status hexla_model_create(hexla_ctx* ctx, uint64_t seed, hexla_model** out);
hexla_status hexla_model_destroy(hexla_model* model);
hexla_status hexla_model_param_count(int64_t* n);
/* Parameters as one flat host array of param_count floats: W1 (64 x 32,
 * row-major: out x in), b1, W2 (64 x 64), b2, W3, b3, W4 (1 x 64), b4, and
 * the target standardisation (predictions are y_mean + y_std * network).
 * set_params also clears the Adam state. */
hexla_status hexla_model_get_params(hexla_model* model, float* host, int64_t n, float* y_mean,
                                    float* y_std);
hexla_status hexla_model_set_params(hexla_model* model, const float* host, int64_t n,
                                    float y_mean, float y_std);
/* Gradient (host, param_count floats) and value of the raw network's loss
 * (1/count) sum_i (network(x_i) - t_i)^2 over x (device, row-major count x
 * HEXLA_MODEL_FEATURES) and t (device, count). Synchronous. */
hexla_status hexla_model_grad(hexla_model* model, const float* x, const float* t, int64_t count,
                              float* grad, double* loss);
/* One Adam step of the raw network on this batch. Synchronous. */
hexla_status hexla_model_step(hexla_model* model, const float* x, const float* t, int64_t count,
                              float lr, double* loss);
/* Trains on (x, t) with t = log(microseconds) (device arrays): targets are
 * standardised, then minibatch Adam over shuffled epochs; final_loss is the
 * MSE over all samples in standardised units. Synchronous. */
hexla_status hexla_model_train(hexla_model* model, const float* x, const float* t, int64_t count,
                               const hexla_train_opts* opts, double* final_loss);
/* y (device, count) = predicted log(microseconds) of x (device). Asynchronous
 * on the context's stream. */
hexla_status hexla_model_predict(hexla_model* model, const float* x, int64_t count, float* y);
/* Text file: a "hexla-mlp 1 gfx950 32 P" header, y_mean y_std, then the
 * parameters. Loading rejects other layouts and targets (HEXLA_E_INVALID_ARG). */
hexla_status hexla_model_save(hexla_model* model, const char* path);
hexla_status hexla_model_load(hexla_ctx* ctx, const char* path, hexla_model** out);
/* The model HEXLA_PLANNER_LEARNED consults (borrowed; NULL clears). */
hexla_status hexla_ctx_set_model(hexla_ctx* ctx, hexla_model* model);
/* Appends every configuration hexla_plan_autotune times to `path`, one JSON
 * object per line: dtype, precision, mode, ta, tb, m, n, k, tile, split, us
 * (microseconds per launch). NULL stops logging. */
hexla_status hexla_timing_log(hexla_ctx* ctx, const char* path);

/* Library version string (static storage). */
const char* hexla_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HEXLA_H */
