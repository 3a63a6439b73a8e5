// Launch interface of the gfx950 kernels. Host code (planner, evaluator)
// includes this header only; every argument is a plain pointer or integer.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace hexla {
namespace k {

// ------------------------------------------------------------ element-wise
// A post-order program for a 4-deep value stack, evaluated per element with
// uniform (scalar) control flow: the fused loop of Sec. II, with no temporaries.
enum EwOp : uint8_t {
  EW_LEAF = 0,   // push leaf[arg] at this element
  EW_EXTRA = 1,  // push the producing kernel's value (GEMV epilogue)
  EW_CONST = 2,  // push cst[arg]
  EW_IDENT = 3,  // push (i == j) ? 1 : 0 (general path only)
  EW_ADD = 4,    // b = pop, a = pop, push a + b
  EW_SUB = 5,    //                    push a - b
  EW_MUL = 6,    //                    push a * b
  EW_DIV = 7,    //                    push a / b
  EW_RSUB = 8,   //                    push b - a
  EW_RDIV = 9,   //                    push b / a
  EW_NEG = 10,   // top = -top
  EW_EXP = 11,   // top = exp(top)
  EW_SCALE = 12, // top = top * cst[arg]
  EW_ADDC = 13,  // top = top + cst[arg]
  EW_LEAFMUL = 14,  // top = top * leaf[arg]
  EW_LEAFADD = 15   // top = top + leaf[arg]
};

constexpr int kEwMaxInstr = 32;
constexpr int kEwMaxLeaf = 8;
constexpr int kEwMaxConst = 8;
constexpr int kEwMaxDepth = 4;

struct EwLeaf {
  const void* ptr;
  int64_t si, sj;  // element (i, j) of the view is ptr[i*si + j*sj]
};

struct EwProgram {
  int32_t n_instr;
  int32_t n_leaf;
  int32_t contiguous;  // every leaf is dense in flat column-major order
  int32_t uses_ident;
  int64_t rows, cols;  // shape of the evaluated view
  uint8_t op[kEwMaxInstr];
  uint8_t arg[kEwMaxInstr];
  double cst[kEwMaxConst];
  EwLeaf leaf[kEwMaxLeaf];
};

// out element (i, j) is written to out[i*osi + j*osj].
hipError_t ew_launch(int dtype, const EwProgram& p, void* out, int64_t osi, int64_t osj,
                     hipStream_t s);

// -------------------------------------------------------------------- GEMV
// y = alpha * op(A) x (+ epilogue), A stored ms x ns column-major (lda).
// trans = 0: y has ms entries; trans = 1: y has ns entries. With an epilogue,
// y_i = program(extra = alpha * (op(A) x)_i) evaluated at flat index i.
hipError_t gemv_launch(int dtype, int trans, int64_t ms, int64_t ns, double alpha,
                       const void* A, int64_t lda, const void* x, int64_t incx,
                       void* y, int64_t incy, const EwProgram* epi, hipStream_t s);

// -------------------------------------------------------------------- GEMM
// C = alpha * op(A) op(B) + beta * C, op(A) m x k, op(B) k x n, all
// column-major. mode 0: full product; mode 1: symmetric result, only
// lower-triangle tiles are computed and mirrored (SYRK). split > 1 runs
// split-K into `partial` (split * m * n elements) followed by a fixed-order
// reduction (deterministic).
struct GemmConfig {
  int tile;   // index into the tile table of the kernel family
  int split;  // K splits
};
enum GemmPrecision { GEMM_PLAIN = 0, GEMM_BF16X3 = 1, GEMM_BF16X6 = 2, GEMM_F16 = 3 };

GemmConfig gemm_choose(int dtype, int precision, int mode, int64_t m, int64_t n, int64_t k);
// tile table access for the autotuner
int gemm_tile_count(int dtype);
void gemm_tile_shape(int dtype, int precision, int tile, int* bm, int* bn, int* bk);
bool gemm_tile_valid(int dtype, int tile, int mode);
int64_t gemm_tiles_for(int dtype, int tile, int mode, int64_t m, int64_t n);  // output tiles
int gemm_split_for(int dtype, int tile, int mode, int64_t m, int64_t n, int64_t k, int64_t target,
                   int64_t min_steps);
size_t gemm_partial_bytes(int dtype, const GemmConfig& cfg, int64_t m, int64_t n);
// split-BF16 family (FP32 storage only), used by gemm_choose / gemm_launch
GemmConfig gemm_choose_split(int dtype, int precision, int mode, int64_t m, int64_t n, int64_t k);
hipError_t gemm_split_launch(int dtype, int precision, int mode, int ta, int tb, int64_t m,
                             int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
                             const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                             void* partial, const GemmConfig& cfg, hipStream_t s);
hipError_t gemm_launch(int dtype, int precision, int mode, int ta, int tb, int64_t m, int64_t n,
                       int64_t k, double alpha, const void* A, int64_t lda, const void* B,
                       int64_t ldb, double beta, void* C, int64_t ldc, void* partial,
                       const GemmConfig& cfg, hipStream_t s);

// The bfloat16 terms of FP32 values (raw bit patterns): t0 = rne(x),
// t1 = rne(x - t0), t2 = rne(x - t0 - t1) (written when terms == 3).
// C -= A B with K <= 64 in split terms (precision GEMM_BF16X3, GEMM_BF16X6 or
// GEMM_F16), FP32 operands, column-major: the LU's low-precision trailing
// update.
hipError_t rank_update_split_launch(int precision, int64_t m, int64_t n, int64_t K,
                                    const float* A, int64_t lda, const float* B, int64_t ldb,
                                    float* C, int64_t ldc, hipStream_t s);
hipError_t split_bf16_launch(const float* x, int64_t n, uint16_t* t0, uint16_t* t1, uint16_t* t2,
                             int terms, hipStream_t s);

// ---------------------------------------------------------------- diagonals
// d[i * incd] = alpha * sum_k op(A)(i, k) op(B)(k, i) for i < nd (op(A) is
// nd x kk or wider, op(B) kk x nd or wider; ta / tb: transposed operands),
// or with sum: d[0] = alpha * sum_i of the same. `partial` (device,
// diagprod_partial_bytes) holds the split-contraction partial sums.
size_t diagprod_partial_bytes(int dtype, int64_t nd, int64_t kk, bool sum);
hipError_t diagprod_launch(int dtype, int ta, int tb, int64_t nd, int64_t kk, double alpha,
                           const void* A, int64_t lda, const void* B, int64_t ldb, void* d,
                           int64_t incd, bool sum, void* partial, hipStream_t s);
// out[0] = alpha * sum of the program over its p.rows x p.cols elements (any
// leaf strides); `partial`: ew_sum_partial_bytes(count) bytes.
size_t ew_sum_partial_bytes(int dtype, int64_t count);
hipError_t ew_sum_launch(int dtype, const EwProgram& p, double alpha, void* out, void* partial,
                         hipStream_t s);

// ------------------------------------------------------ structured solves
// Lookahead for the factorisations (Cholesky, LU): a second stream, default priority like the caller's, and two events, owned
// by the caller: the trailing update beyond the next panel's columns runs
// there while the next panel is factored (the factorisation makes the
// caller's stream wait for it before it returns).
struct Lookahead {
  hipStream_t s = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
};

// Blocked triangular solves in one launch per direction and 1024 columns (the
// one-launch MFMA solve of lu_solve_launch): X <- op(M)^-1 X in place, for
// mode 0 the lower triangle of M (forward), 1 its upper triangle (backward),
// 2 the transpose of its lower triangle (backward); the diagonal blocks'
// inverses (64 x 64, column-major, identity-padded) at inv + block * stride.
// mode2 (or -1) is a second direction applied after the first, per 1024
// columns. work: tri_chain_work_bytes, 256-byte aligned. A wait that timed
// out raises status[1].
size_t tri_chain_work_bytes(int dtype, int64_t n, int64_t nrhs);
hipError_t tri_chain_launch(int dtype, int64_t n, int64_t nrhs, const void* M, int64_t ldm,
                            int mode1, const void* inv1, int64_t stride1, int mode2,
                            const void* inv2, int64_t stride2, void* X, int64_t ldx, void* work,
                            int32_t* status, hipStream_t s);
// info (16 ints, 8-byte aligned, cleared here): [0] lower bandwidth, [1]
// upper bandwidth, [2] 1 if S != S^T bitwise, [3] 1 if a diagonal entry is
// not > 0, [5] 1 if a diagonal entry is zero, 64-bit words at [8] max |S_ij|
// and [10] max |S_ij - S_ji| (FP64 values). One pass over the n x n S (lds).
hipError_t structure_launch(int dtype, int64_t n, const void* S, int64_t lds, int32_t* info,
                            hipStream_t s);
// In-place Cholesky A = L L^T (lower triangle of A, lda), blocks of 64.
// A pivot that is not > 0 sets info[4] (A is then not positive definite and
// its contents are unspecified). With side, each next diagonal block is
// factored while the rest of the trailing update runs on side->s. work: the
// inverses of the diagonal blocks of L, laid out as tri_solve_launch's work
// (which then may skip computing them).
hipError_t chol_factor_launch(int dtype, int64_t n, void* A, int64_t lda, int32_t* info,
                              void* work, hipStream_t s, const Lookahead* side = nullptr);
// The lower-triangle 64 x 64 tiles (diagonal tiles whole) of the n x n C
// (ldc) take C -= W W^T, W n x K (ldw), K <= 64: the Cholesky factorisation's
// trailing update, C tile held in the MFMA accumulators.
hipError_t syrk_lower_update_launch(int dtype, int64_t n, int64_t K, const void* W, int64_t ldw,
                                   void* C, int64_t ldc, hipStream_t s);
// C (m x n, ldc) -= A Bt^T, A m x K (lda), Bt n x K (ldbt), K <= 64, with
// the same kernel (every tile).
hipError_t rank_update_bt_launch(int dtype, int64_t m, int64_t n, int64_t K, const void* A,
                                 int64_t lda, const void* Bt, int64_t ldbt, void* C, int64_t ldc,
                                 hipStream_t s);
// X <- M^-1 X in place (n x nrhs, ldx), by blocks of 64 with the inverses
// of the diagonal blocks: which 0: M = L L^T (L the lower triangle of M),
// 1: M = L (lower), 2: M = U (upper); non-unit diagonals; n <= kLuMaxN.
// work: tri_solve_workspace_bytes (the inverses, then the blocked solve's
// tickets and exchange), 256-byte aligned; have_inv: work already holds the
// inverses (left there by chol_factor_launch). A wait that timed out raises
// status[1].
size_t tri_solve_workspace_bytes(int dtype, int64_t n, int64_t nrhs);
hipError_t tri_solve_launch(int dtype, int which, int64_t n, int64_t nrhs, const void* M,
                            int64_t ldm, void* X, int64_t ldx, void* work, bool have_inv,
                            int32_t* status, hipStream_t s);
// Tridiagonal part of S with partial pivoting; X (ldx) holds the right-hand
// sides and receives the solution; work: 6 n elements of scratch; a zero
// pivot sets info[5].
hipError_t gtsv_launch(int dtype, int64_t n, int64_t nrhs, const void* S, int64_t lds, void* X,
                       int64_t ldx, void* work, int32_t* info, hipStream_t s);

// ---------------------------------------------------------------------- LU
// In-place LU with partial pivoting of the n x n column-major matrix A (lda),
// A = P^T L U. rowid (n ints) receives the original row held at each final
// position (row i of L U is row rowid[i] of A). status[0] gets HEXLA_E_SINGULAR
// and status[2..3] the first zero-pivot column on an exact zero pivot.
// update_precision: GemmPrecision of the trailing updates (FP32 storage only
// for the non-plain values). panel_fp64 (FP32 storage only): each panel is
// factored in FP64 (pivot search and elimination on FP64 values) and rounded
// to FP32 when it is stored.
// n <= kLuMaxN (larger n: hipErrorInvalidValue). The workspace also keeps the
// inverses of the 64 x 64 diagonal blocks, which lu_solve_launch applies, and
// (nrhs > 0) the solve's exchange of solved blocks for nrhs right-hand sides.
constexpr int64_t kLuMaxN = 16384;
size_t lu_workspace_bytes(int dtype, int64_t n, int64_t nrhs = 0);
hipError_t lu_factor_launch(int dtype, int64_t n, void* A, int64_t lda, int32_t* rowid,
                            void* work, int32_t* status, hipStream_t s, const Lookahead* side,
                            int update_precision = 0, bool panel_fp64 = false);
// X (n x nrhs, ldx) <- U^{-1} L^{-1} B[rowid], B with ldb; work: the
// factorisation's workspace, sized for at least nrhs right-hand sides. Two
// launches per 1024 right-hand sides (forward, backward); a wait that timed
// out raises status[1]. X may not alias B.
hipError_t lu_solve_launch(int dtype, int64_t n, int64_t nrhs, const void* LU, int64_t lda,
                           const int32_t* rowid, void* work, const void* B, int64_t ldb, void* X,
                           int64_t ldx, int32_t* status, hipStream_t s);

// ------------------------------------------------------ mixed precision
// b(i, j) = a(i, j) converted between types (0 FP64, 1 FP32); a(i, j) at
// a[i*asi + j*asj].
hipError_t cast_launch(int from, int to, int64_t rows, int64_t cols, const void* a, int64_t asi,
                       int64_t asj, void* b, int64_t ldb, hipStream_t s);
// *out = max_i sum_j |a_ij| (FP64), scratch holds norm_scratch_elems(rows) doubles.
size_t norm_scratch_elems(int64_t rows);
hipError_t norm_inf_launch(int dtype, int64_t rows, int64_t cols, const void* a, int64_t lda,
                           double* scratch, double* out, hipStream_t s);
// x(i, j) += d(i, j), x FP64, d of type dtype_d.
hipError_t add_mixed_launch(int dtype_d, int64_t rows, int64_t cols, double* x, int64_t ldx,
                            const void* d, int64_t ldd, hipStream_t s);

// ---------------------------------------------------------------- batches
// A per-instance program over vector slots held in LDS. Instances are
// square (n x n matrices, n x 1 vectors), n <= kBMaxN.
constexpr int kBMaxN = 512;
constexpr int kBMaxSlots = 6;
constexpr int kBMaxOps = 16;
constexpr int kBMaxLeaf = 8;
constexpr int kBMaxEw = 48;
constexpr int kBMaxConst = 8;
constexpr uint8_t kBSlotBit = 0x80;  // element-wise operand names a slot
constexpr uint8_t kBOut = 0xff;      // destination: the instance's output

enum BOpKind : uint8_t {
  B_LOAD = 0,   // slot[dst] = vector leaf
  B_GEMV = 1,   // slot[dst] = alpha * op(matrix leaf) slot[src]; dst != src
  B_SOLVE = 2,  // slot[dst] = (matrix leaf)^-1 slot[src] (LU with partial pivoting)
  B_EW = 3      // slot[dst] (or output) = element-wise program ew[begin, end)
};

struct BOp {
  uint8_t kind, dst, src, leaf, trans, ew_begin, ew_end, pad;
  double alpha;
};

struct BProgram {
  int32_t n_ops;
  int32_t out_slot;  // slot copied to the output at the end, or kBOut
  BOp ops[kBMaxOps];
  uint8_t ew_op[kBMaxEw];   // EwOp codes (EW_EXTRA and EW_IDENT excluded)
  uint8_t ew_arg[kBMaxEw];  // leaf index, kBSlotBit | slot, or constant index
  double cst[kBMaxConst];
};

struct BInst {
  const void* leaf[kBMaxLeaf];
  int64_t ld[kBMaxLeaf];
  void* out;
  int64_t n;
};

// Launch configurations: LU panel width x threads per workgroup.
struct BatchConfig {
  int variant;  // index into the variant table of the dtype
  int grid;     // workgroups of the persistent launch
};
int batch_variant_count(int dtype);
void batch_variant_shape(int dtype, int variant, int* panel, int* threads);
BatchConfig batch_default(int dtype, int64_t count);
// scratch elements per workgroup for instances up to max_n
int64_t batch_scratch_stride(int64_t max_n);
// Resets the queue counter, then runs every instance (order: instance indices,
// largest first). status[0] <- HEXLA_E_SINGULAR and status[2] <- instance on
// an exact zero pivot.
hipError_t batch_launch(int dtype, const BatchConfig& cfg, const BProgram* p, const BInst* inst,
                        const int32_t* order, int64_t count, unsigned* queue, void* scratch,
                        int64_t scratch_stride, int32_t* status, hipStream_t s);

// ------------------------------------------------------- learned cost model
// FP32 ReLU network kMlpFeatures -> 64 -> 64 -> 64 -> 1 over a flat
// parameter vector of kMlpParams floats (W1 row-major, b1, W2, b2, W3, b3, W4,
// b4). x is row-major [count][kMlpFeatures].
constexpr int kMlpFeatures = 32;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpHidden * kMlpFeatures + kMlpHidden +
                           2 * (kMlpHidden * kMlpHidden + kMlpHidden) + kMlpHidden + 1;
int64_t mlp_blocks(int64_t count);
// Per-block gradient partials of L = (1/count) sum (y - t)^2 (partial:
// mlp_blocks(count) x kMlpParams floats; loss_partial: sum of squares per
// block). idx (optional) maps sample positions to rows of x and t.
hipError_t mlp_grad_launch(const float* params, const float* x, const float* t,
                           const int32_t* idx, int64_t count, float* partial,
                           float* loss_partial, hipStream_t s);
// grad (optional) <- sum of the partials; with params: one Adam step (step >= 1).
hipError_t mlp_reduce_launch(const float* partial, int64_t nblocks, float* grad, float* params,
                             float* m, float* v, float lr, float beta1, float beta2, float eps,
                             int64_t step, hipStream_t s);
// y = shift + scale * network(x)
hipError_t mlp_predict_launch(const float* params, const float* x, int64_t count, float scale,
                              float shift, float* y, hipStream_t s);

// ------------------------------------------------------------------- utils
hipError_t fill_i32_launch(int32_t* p, int64_t count, int32_t value, hipStream_t s);

}  // namespace k
}  // namespace hexla
