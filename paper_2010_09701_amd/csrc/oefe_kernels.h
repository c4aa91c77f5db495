// Launchers of the HIP kernels (device code in oefe_ops.hip and oefe_linalg.hip).
#pragma once

#include "oefe_internal.h"

namespace oefe {

// Work layout for the operator step of a block with `ncv` vectors (complex or real).
struct StepWork {
  void* ycell;    // [n_cells * nd * ldc] real columns, element T
  int ldc;        // real columns per cell node (padded)
  void* zo;       // [n_enr * ncr] S X^O
  void* part;     // [tile_slots * ncr] per-tile partials of (m^-1/2 H^co)^* X
  void* part2;    // [n_enr * n_rchunks * ncr] partials folded over chunks of tiles
  void* wp;       // [n_enr * ncr]
};

// Allows a kernel `dynamic_bytes` of dynamic LDS (above the 64 KB default the
// attribute must be raised; the limit is the CU's 160 KB including static LDS).
// Returns hipSuccess or the error of hipFuncSetAttribute.
inline hipError_t allow_dynamic_lds(const void* kernel, size_t dynamic_bytes) {
  if (dynamic_bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dynamic_bytes);
}

size_t step_work_bytes(const oefe_op_s* op, int elem_bytes, bool cplx, int nv, int* ldc_out);
StepWork carve_step_work(const oefe_op_s* op, int elem_bytes, bool cplx, int nv, void* work);

// Overlap of a recurrence: the enrichment side of step k (the coupling kernel, then
// the partial fold, W', the enrichment rows of out and Z^O of step k+1) runs on `side`
// beside the cell stage of step k; the node assembly of step k waits for the coupling
// kernel (ev_k1), and the side work of step k+1 waits for that assembly (ev_node).
// first: this step computes its own Z^O; last: the main stream waits for the side
// chain (ev_zo) at the end of the step.
struct Overlap {
  hipStream_t side;
  hipEvent_t ev_node, ev_k1, ev_zo;
  bool first, last;
};

// out = alpha (Ht x - c x) - beta prev   (prev may be null when beta == 0)
// T = double or float; x: [n_tot x ld], prev and out: [n_tot x ldo] (complex: interleaved, leading
// dimensions in complex elements).  prev may alias out.
// sc (device, optional): (alpha, c, beta) of the step, read by the kernels in place of the
// host values (which then only say whether prev is read: beta != 0)
template <typename T>
int apply_step(const oefe_op_s* op, bool bf16, const T* x, int64_t ld, const T* prev, T* out, int64_t ldo, int nv,
               double alpha, double c, double beta, const StepWork& w, hipStream_t s,
               const Overlap* ov = nullptr, const double* sc = nullptr);
// the m steps' (alpha, c, beta) of a filter from device bounds (a, b, a0) into out [m][3]
int cheb_scalars(const double* bounds, int m, double* out, int32_t* status, hipStream_t s);
// Batched steps of nk operators sharing one mesh / enrichment layout (k-points), in lockstep.
template <typename T>
int apply_step_batch(const oefe_op_s* const* ops, int nk, bool bf16, const T* const* x, const int64_t* ld,
                     const T* const* prev, T* const* out, const int64_t* ldo, const int* nv, const double* alpha,
                     const double* c, const double* beta, const StepWork* w, hipStream_t s,
                     const Overlap* ov = nullptr);
// Z^O = S X^O only (for the density)
template <typename T>
int zo_only(const oefe_op_s* op, const T* x, int64_t ld, int nv, T* zo, int ncr, hipStream_t s);
// density partials per 64-column block: dens[blk][e][q] = sum_cols f_v psi_col(x_eq)^2
template <typename T>
int density_partial(const oefe_op_s* op, const T* x, int64_t ld, int nv, const double* f, const T* zo, int ncr,
                    double* dens, hipStream_t s);
// dEdV[e][q] = W_eq sum_blk dens[blk][e][q]
int density_final(const oefe_op_s* op, const double* dens, int nblk, double* dEdV, hipStream_t s, int mode = 0);

// ---- dense linear algebra (float64, real or complex-interleaved), oefe_linalg.hip
// G[i][j] = sum_g conj(A[g][i]) B[g][j]  (na x nb, row-major ldg), rows 0..n-1.
int gram(bool cplx, const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb, int64_t n,
         double* G, int ldg, double* scratch, size_t scratch_bytes, hipStream_t s);
size_t gram_scratch_bytes(bool cplx, int na, int nb, int64_t n);
// C = A * B, A [n x k] (lda), B [k x m] (ldb, small), C [n x m] (ldc)
int gemm_nn(bool cplx, const double* A, int64_t lda, const double* B, int ldb, double* C, int64_t ldc, int64_t n,
            int k, int m, hipStream_t s);
// X <- X R in place on the matrix cores, X [n x nv] (ldx), R [nv x nv] row-major; real, nv <= 80
bool rowmul_on_mfma(bool cplx, int nv);
// (gate: device int; the product is skipped when it holds 0)
int rowmul_inplace(double* X, int64_t ldx, int64_t n, int nv, const double* R, hipStream_t s,
                   const int32_t* gate = nullptr);
// in-place Cholesky of Jacobi-scaled Hermitian G (n x n): writes Rinv = (D^-1 L)^-* ... see linalg source
// gate (device int, optional): skipped when it holds 0; go (device int, optional): 1 after a
// successful factorization, else 0.  Gates need cholgs_device_gated(cplx, n).
int chol_factor_inverse(bool cplx, double* G, int ldg, int n, double* Rinv, int32_t* status, hipStream_t s,
                        const int32_t* gate = nullptr, int32_t* go = nullptr);
// CholGS of nv columns can run without host round trips: the factor inverse takes gates and
// X R^-1 runs in place on the matrix cores
bool cholgs_device_gated(bool cplx, int nv);
// Hermitian eigensolver (cyclic Jacobi, one workgroup): A overwritten; lam ascending, U columns.
// status: {0, sweeps} or {OEFE_ENOCONV, sweeps} when max_sweeps (0: built-in limit) ended the
// iteration before the off-diagonal part vanished to rounding
int jacobi_eig(bool cplx, double* A, int n, double* lam, double* U, double* scratch, int32_t* status,
               hipStream_t s, int max_sweeps = 0);
size_t jacobi_scratch_bytes(bool cplx, int n);
// max |G - I| into *err (device double)
// with repeat (device int): repeat = (status[0] == 0 && max |G - I| > tol)
int max_offdiag_identity(bool cplx, const double* G, int n, double* err, hipStream_t s,
                         const int32_t* status = nullptr, int32_t* repeat = nullptr, double tol = 0.0);
// symmetrize (Hermitian part) in place
int hermitian_part(bool cplx, double* G, int n, hipStream_t s, const int32_t* gate = nullptr);
// copies / casts between blocks [n_rows x ld] (only the first ncols real columns)
int copy_block(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n_rows, int ncols, hipStream_t s);
// out = sum_j f_j Re sum_g conj(A[g][j]) B[g][j]  (f may be null: all ones), accumulated in float64
template <typename T>
int dot_columns(bool cplx, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n, int nv, const double* f,
                double* out, double* scratch, hipStream_t s);
// the one-column dot product of dot_columns in two parts, for kernels that form its chunk
// partials themselves: the number of row chunks (each cdiv(n, chunks) rows; the partial of a chunk
// sums rows t, t + 2048, ... and t + 1024, t + 3072, ... of thread t of 1024, then the 16 wave
// sums of fixed butterflies in order), and the final sum of the partials into *out
int dot1_chunk_count(int64_t n);
int dot1_final(const double* part, int nch, double* out, hipStream_t s);
// dst (ldd) <- src (lds), n_rows x ncols real elements, with float/double conversion
int cast_block(const void* src, bool src_f32, void* dst, bool dst_f32, int64_t n_rows, int64_t lds, int64_t ldd,
               int ncols, hipStream_t s);
// dE/dX = 2 f_j (H x)_j in place
int scale_grad(bool cplx, void* g, int64_t ld, int64_t n, int nv, const double* f, bool f32, hipStream_t s);
// Lanczos helpers (float64, vectors [n] packed or strided by ldv complex elements)
int lanczos_axpy(bool cplx, double* w, const double* v, const double* vprev, const double* alpha,
                 const double* beta, int64_t n, int64_t ldv, hipStream_t s);
int lanczos_scale(bool cplx, double* dst, int64_t ldd, const double* w, const double* beta, int64_t n,
                  hipStream_t s);
int sub_block(bool cplx, double* w, const double* t, int64_t n, hipStream_t s);
int sqrt_inplace(double* x, hipStream_t s);

}  // namespace oefe
