// Dense float64 linear algebra for Cholesky-Gram-Schmidt, Rayleigh-Ritz and
// Lanczos (gfx950): tall-skinny Gram products, tall x small products, a
// one-workgroup Cholesky with triangular inverse, and a one-workgroup cyclic
// Jacobi eigensolver for Hermitian matrices.  Complex data is interleaved.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "oefe_kernels.h"

namespace oefe {

namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Z {
  double r, i;
};
__device__ __forceinline__ Z zmul(Z a, Z b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ Z zcjmul(Z a, Z b) { return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r}; }

// ---- Gram: partial[chunk][i][j] = sum_{g in chunk} conj(A[g][i]) B[g][j]; 16x16 tile per block
template <bool CPLX>
__global__ __launch_bounds__(256) void gram_partial_kernel(const double* __restrict__ A, int64_t lda, int na,
                                                           const double* __restrict__ B, int64_t ldb, int nb,
                                                           int64_t n, int64_t rows_per_chunk,
                                                           double* __restrict__ part) {
  constexpr int TS = 16, KB = 32;
  constexpr int E = CPLX ? 2 : 1;
  __shared__ double As[KB][TS * E + 1];
  __shared__ double Bs[KB][TS * E + 1];
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  const int i0 = blockIdx.y * TS, j0 = blockIdx.z * TS;
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t g1 = min(n, g0 + rows_per_chunk);
  double ar = 0, ai = 0;
  for (int64_t gb = g0; gb < g1; gb += KB) {
    for (int t = threadIdx.x; t < KB * TS * E; t += 256) {
      const int r = t / (TS * E), cc = t % (TS * E);
      const int64_t g = gb + r;
      const int col = cc / E;
      double va = 0, vb = 0;
      if (g < g1) {
        if (i0 + col < na) va = A[g * lda * E + (int64_t)(i0 + col) * E + cc % E];
        if (j0 + col < nb) vb = B[g * ldb * E + (int64_t)(j0 + col) * E + cc % E];
      }
      As[r][cc] = va;
      Bs[r][cc] = vb;
    }
    __syncthreads();
    const int kmax = (int)min<int64_t>(KB, g1 - gb);
    if constexpr (!CPLX) {
      for (int k = 0; k < kmax; ++k) ar += As[k][ty] * Bs[k][tx];
    } else {
      for (int k = 0; k < kmax; ++k) {
        Z t = zcjmul(Z{As[k][2 * ty], As[k][2 * ty + 1]}, Z{Bs[k][2 * tx], Bs[k][2 * tx + 1]});
        ar += t.r;
        ai += t.i;
      }
    }
    __syncthreads();
  }
  const int i = i0 + ty, j = j0 + tx;
  if (i < na && j < nb) {
    double* o = part + ((int64_t)blockIdx.x * na * nb + (int64_t)i * nb + j) * E;
    o[0] = ar;
    if (CPLX) o[1] = ai;
  }
}

template <bool CPLX>
__global__ void gram_reduce_kernel(const double* __restrict__ part, int nchunks, int na, int nb,
                                   double* __restrict__ G, int ldg) {
  constexpr int E = CPLX ? 2 : 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= na * nb) return;
  const int i = idx / nb, j = idx % nb;
  double sr = 0, si = 0;
  for (int c = 0; c < nchunks; ++c) {
    const double* p = part + ((int64_t)c * na * nb + idx) * E;
    sr += p[0];
    if (CPLX) si += p[1];
  }
  G[((int64_t)i * ldg + j) * E] = sr;
  if (CPLX) G[((int64_t)i * ldg + j) * E + 1] = si;
}

// ---- Gram on the matrix cores (16x16x4 float64 MFMA), real, for 16 <= na, nb <= 16 kGramNBMax:
// partial[chunk][i][j] = sum over the chunk's rows g of A[g][i] B[g][j].  One workgroup
// (one wave per SIMD) per (row chunk, group of NBI 16-row blocks of G); each wave takes
// every fourth k-step of 4 rows and accumulates the NBI x NBJ output blocks of 16x16, with the fragments of the next k-step
// loaded while the MFMAs of the current one run (lane: row 4 k + lane / 16, column
// 16 ib + lane % 16).  The four waves' sums are then added through one LDS buffer in a
// fixed order and the workgroup's partial is written.
typedef double dv4 __attribute__((ext_vector_type(4)));
constexpr int kGramNBMax = 5;   // 16-column blocks per operand
constexpr int kGramChunks = 256;

// One workgroup's share: 16-row blocks ib0 .. ib0 + NBI - 1 of G = A^T B over rows g0 .. g1 - 1,
// written to out (row-major na x nb).  gsm: [NBI * NBJ * 4][64] doubles of LDS.
template <int NBI, int NBJ>
__device__ __forceinline__ void gram_mfma_body(const double* __restrict__ A, int64_t lda, int na,
                                               const double* __restrict__ B, int64_t ldb, int nb, int64_t g0,
                                               int64_t g1, int ib0, double* __restrict__ out, double* gsm) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int ca[NBI], cb[NBJ];
  double ma[NBI], mb[NBJ];
#pragma unroll
  for (int i = 0; i < NBI; ++i) {
    const int c = (ib0 + i) * 16 + li;
    ma[i] = c < na ? 1.0 : 0.0;
    ca[i] = min(c, na - 1);
  }
#pragma unroll
  for (int j = 0; j < NBJ; ++j) {
    const int c = j * 16 + li;
    mb[j] = c < nb ? 1.0 : 0.0;
    cb[j] = min(c, nb - 1);
  }
  dv4 acc[NBI][NBJ];
#pragma unroll
  for (int i = 0; i < NBI; ++i)
#pragma unroll
    for (int j = 0; j < NBJ; ++j) acc[i][j] = dv4{0, 0, 0, 0};
  // fragments of the k-step at rows gk .. gk + 3 (rows past the chunk: clamped, zeroed)
  auto load = [&](int64_t gk, double (&a)[NBI], double (&b)[NBJ]) {
    const int64_t r = gk + lk;
    const double m = r < g1 ? 1.0 : 0.0;
    const int64_t rc = r < g1 ? r : g1 - 1;
    const double* Ar = A + rc * lda;
    const double* Br = B + rc * ldb;
#pragma unroll
    for (int i = 0; i < NBI; ++i) a[i] = Ar[ca[i]] * (m * ma[i]);
#pragma unroll
    for (int j = 0; j < NBJ; ++j) b[j] = Br[cb[j]] * mb[j];
  };
  auto mma = [&](const double (&a)[NBI], const double (&b)[NBJ]) {
#pragma unroll
    for (int i = 0; i < NBI; ++i)
#pragma unroll
      for (int j = 0; j < NBJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  };
  double a0[NBI], b0[NBJ], a1[NBI], b1[NBJ];
  int64_t gk = g0 + 4 * w;
  if (gk < g1) load(gk, a0, b0);
  for (; gk < g1; gk += 32) {
    load(gk + 16, a1, b1);
    mma(a0, b0);
    if (gk + 16 >= g1) break;
    load(gk + 32, a0, b0);
    mma(a1, b1);
  }
  // combine the four waves in a fixed order through one LDS buffer: ((w3 + w2) + w1) + w0
  auto slot = [&](int i, int j, int v) -> double& { return gsm[((size_t)(i * NBJ + j) * 4 + v) * 64 + lane]; };
  for (int step = 3; step >= 0; --step) {
    if (w == step) {
#pragma unroll
      for (int i = 0; i < NBI; ++i)
#pragma unroll
        for (int j = 0; j < NBJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double t = step == 3 ? acc[i][j][v] : slot(i, j, v) + acc[i][j][v];
            if (step > 0) {
              slot(i, j, v) = t;
            } else {
              const int row = (ib0 + i) * 16 + lk + 4 * v, col = j * 16 + li;
              if (row < na && col < nb) out[(int64_t)row * nb + col] = t;
            }
          }
    }
    if (step > 0) __syncthreads();
  }
}

template <int NBI, int NBJ>
__global__ __launch_bounds__(256, NBI == 1 ? 4 : 1) void gram_mfma_kernel(const double* __restrict__ A, int64_t lda, int na,
                                                           const double* __restrict__ B, int64_t ldb, int nb,
                                                           int64_t n, int64_t rows_per_chunk,
                                                           double* __restrict__ part) {
  extern __shared__ double gsm[];
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_chunk, g1 = min(n, g0 + rows_per_chunk);
  gram_mfma_body<NBI, NBJ>(A, lda, na, B, ldb, nb, g0, g1, blockIdx.y * NBI, part + (int64_t)blockIdx.x * na * nb,
                           gsm);
}

// Gram matrices of blocks wider than 16 kGramNBMax columns in one launch: G is cut into
// column groups of at most 16 kGramNBMax (near-equal), and each (I, J) pair of groups is one
// matrix-core Gram as above.  Pair p covers rows i0[p] .. i0[p] + ni[p] - 1 of G (columns of A)
// and columns j0[p] .. of G (columns of B); with A = B only the pairs I <= J are computed and
// the rest of G is their mirror image.
constexpr int kGramPairsMax = 64;
struct GramPairs {
  int np, gs;  // pairs; partial-block stride (gs x gs doubles, gs = the largest group)
  int i0[kGramPairsMax], ni[kGramPairsMax], j0[kGramPairsMax], nj[kGramPairsMax];
};

// workgroup L (after the XCD remap) = ((chunk np + pair) rbs + row block): the workgroups of one
// row chunk are contiguous in L, so each XCD (workgroups bk = x mod 8, a contiguous range of L)
// reads a chunk's rows of A and B from HBM once for all pairs and row blocks
__global__ __launch_bounds__(256, 4) void gram_mfma_pairs_kernel(const double* __restrict__ A, int64_t lda,
                                                                 const double* __restrict__ B, int64_t ldb, int64_t n,
                                                                 int64_t rows_per_chunk, int nch, GramPairs gp,
                                                                 double* __restrict__ part) {
  extern __shared__ double gsm[];
  const int nbk = gridDim.x, bk = blockIdx.x, nb8 = nbk & ~7;
  const int L = bk < nb8 ? (bk & 7) * (nb8 >> 3) + (bk >> 3) : bk;
  const int rbs = (gp.gs + 15) >> 4;
  const int rb = L % rbs, rest = L / rbs;
  const int p = rest % gp.np, chunk = rest / gp.np;
  const int na = gp.ni[p], nb = gp.nj[p];
  if (rb * 16 >= na) return;  // whole workgroup: no barrier is pending
  const int64_t g0 = (int64_t)chunk * rows_per_chunk, g1 = min(n, g0 + rows_per_chunk);
  gram_mfma_body<1, kGramNBMax>(A + gp.i0[p], lda, na, B + gp.j0[p], ldb, nb, g0, g1, rb,
                                part + ((int64_t)p * nch + chunk) * gp.gs * gp.gs, gsm);
}

// G entries of pair blockIdx.y = sum over the chunks, one wave per entry (lane-strided chunks in
// order, then a fixed butterfly); mirror != 0 also writes the transposed entry of an off-diagonal pair
__global__ __launch_bounds__(256) void gram_reduce_pairs_kernel(const double* __restrict__ part, int nch, GramPairs gp,
                                                                double* __restrict__ G, int ldg, int mirror) {
  const int p = blockIdx.y;
  const int na = gp.ni[p], nb = gp.nj[p];
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (idx >= na * nb) return;
  const double* pp = part + (int64_t)p * nch * gp.gs * gp.gs;
  double s = 0.0;
  for (int c = lane; c < nch; c += 64) s += pp[(int64_t)c * gp.gs * gp.gs + idx];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) {
    const int i = gp.i0[p] + idx / nb, j = gp.j0[p] + idx % nb;
    G[(int64_t)i * ldg + j] = s;
    if (mirror && gp.i0[p] != gp.j0[p]) G[(int64_t)j * ldg + i] = s;
  }
}

// G[i][j] = sum over the chunks, one wave per entry: lane l adds chunks l, l + 64, ... in
// order, then a fixed butterfly over the 64 lanes
template <bool CPLX>
__global__ __launch_bounds__(256) void gram_reduce_wave_kernel(const double* __restrict__ part, int nchunks, int na,
                                                               int nb, double* __restrict__ G, int ldg) {
  constexpr int E = CPLX ? 2 : 1;
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (idx >= na * nb) return;
  double s[E];
#pragma unroll
  for (int e = 0; e < E; ++e) s[e] = 0.0;
  for (int c = lane; c < nchunks; c += 64)
#pragma unroll
    for (int e = 0; e < E; ++e) s[e] += part[((int64_t)c * na * nb + idx) * E + e];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int e = 0; e < E; ++e) s[e] += __shfl_xor(s[e], o);
  if (lane == 0) {
    const int i = idx / nb, j = idx - i * nb;
#pragma unroll
    for (int e = 0; e < E; ++e) G[((int64_t)i * ldg + j) * E + e] = s[e];
  }
}

// ---- C = A * B : A [n x k], B [k x m] (small); 64x64 output tile, 4x4 per thread
template <bool CPLX>
__global__ __launch_bounds__(256) void gemm_nn_kernel(const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                      int64_t ldc, int64_t n, int k, int m) {
  constexpr int E = CPLX ? 2 : 1;
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ double As[TK][TM * E + E];
  __shared__ double Bs[TK][TN * E + E];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t r0 = (int64_t)blockIdx.x * TM;
  const int c0 = blockIdx.y * TN;
  double acc[4][4][E];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[a][b][e] = 0;
  for (int k0 = 0; k0 < k; k0 += TK) {
    for (int t = threadIdx.x; t < TM * TK * E; t += 256) {
      const int rr = t / (TK * E), kk = (t % (TK * E)) / E, e = t % E;
      const int64_t g = r0 + rr;
      As[kk][rr * E + e] = (g < n && k0 + kk < k) ? A[g * lda * E + (int64_t)(k0 + kk) * E + e] : 0.0;
    }
    for (int t = threadIdx.x; t < TK * TN * E; t += 256) {
      const int kk = t / (TN * E), cc = (t % (TN * E)) / E, e = t % E;
      Bs[kk][cc * E + e] = (k0 + kk < k && c0 + cc < m) ? B[((int64_t)(k0 + kk) * ldb + c0 + cc) * E + e] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      double a[4][E], b[4][E];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          a[q][e] = As[kk][(ty + 16 * q) * E + e];
          b[q][e] = Bs[kk][(tx + 16 * q) * E + e];
        }
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
          if constexpr (!CPLX) {
            acc[qa][qb][0] += a[qa][0] * b[qb][0];
          } else {
            acc[qa][qb][0] += a[qa][0] * b[qb][0] - a[qa][E - 1] * b[qb][E - 1];
            acc[qa][qb][E - 1] += a[qa][0] * b[qb][E - 1] + a[qa][E - 1] * b[qb][0];
          }
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int qa = 0; qa < 4; ++qa)
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
      const int64_t g = r0 + ty + 16 * qa;
      const int cc = c0 + tx + 16 * qb;
      if (g < n && cc < m)
#pragma unroll
        for (int e = 0; e < E; ++e) C[g * ldc * E + (int64_t)cc * E + e] = acc[qa][qb][e];
    }
}

// ---- C = A B on the matrix cores (real, float64): A [n x k] (row stride lda), B [k x m] (row
// stride ldb, small), C [n x m] (row stride ldc), for the wide blocks' products X R (CholGS) and
// Q U (Rayleigh-Ritz).  A workgroup takes 128 rows (32 per wave: two 16-row blocks) and 16 NBJ
// output columns; the column blocks of the same rows are consecutive in the remapped launch
// index and each XCD takes a contiguous range, so they read those rows of A through one L2.  B
// is staged in LDS in chunks of kGemmKC rows (row stride 16 NBJ + 1); the A fragments of the
// next k-step are loaded during the current one's MFMAs.  Fragment layouts as in
// rowmul_mfma_kernel below.
constexpr int kGemmKC = 64;

template <int NBJ>
__global__ __launch_bounds__(256) void gemm_nn_mfma_kernel(const double* __restrict__ A, int64_t lda,
                                                           const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                           int64_t ldc, int64_t n, int k, int m, int ncb) {
  constexpr int RS = 16 * NBJ + 1;
  __shared__ double bs[kGemmKC * RS];
  const int nbk = gridDim.x, bk = blockIdx.x, nb8 = nbk & ~7;
  const int64_t L = bk < nb8 ? (int64_t)(bk & 7) * (nb8 >> 3) + (bk >> 3) : bk;
  const int64_t rt = L / ncb;
  const int c0 = (int)(L - rt * ncb) * 16 * NBJ;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = rt * 128 + w * 32;
  const double* ar[2];
  double mrow[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int64_t r = r0 + 16 * b + li;
    mrow[b] = r < n ? 1.0 : 0.0;
    ar[b] = A + (r < n ? r : n - 1) * lda;
  }
  dv4 acc[2][NBJ];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int j = 0; j < NBJ; ++j) acc[b][j] = dv4{0, 0, 0, 0};
  for (int k0 = 0; k0 < k; k0 += kGemmKC) {
    const int kc = min(kGemmKC, k - k0), nks = (kc + 3) / 4;
    __syncthreads();  // the previous chunk's reads of bs are done
    for (int t = threadIdx.x; t < nks * 4 * 16 * NBJ; t += 256) {
      const int kk = t / (16 * NBJ), cc = t - kk * (16 * NBJ);
      bs[kk * RS + cc] = (kk < kc && c0 + cc < m) ? B[(int64_t)(k0 + kk) * ldb + c0 + cc] : 0.0;
    }
    __syncthreads();
    // A fragments of k-step s of this chunk (columns past k: clamped, zeroed)
    auto load = [&](int s, double (&a)[2]) {
      const int c = k0 + 4 * s + lk;
      const double mk = c < k ? 1.0 : 0.0;
      const int cc = c < k ? c : k - 1;
#pragma unroll
      for (int b = 0; b < 2; ++b) a[b] = ar[b][cc] * (mk * mrow[b]);
    };
    auto mma = [&](int s, const double (&a)[2]) {
      const double* bk4 = bs + (4 * s + lk) * RS + li;
#pragma unroll
      for (int j = 0; j < NBJ; ++j) {
        const double bj = bk4[16 * j];
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[b][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[b], bj, acc[b][j], 0, 0, 0);
      }
    };
    double a0[2], a1[2];
    load(0, a0);
    int s = 0;
    for (; s + 1 < nks; s += 2) {
      load(s + 1, a1);
      mma(s, a0);
      if (s + 2 < nks) load(s + 2, a0);
      mma(s + 1, a1);
    }
    if (s < nks) mma(s, a0);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int j = 0; j < NBJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + 16 * b + lk + 4 * v;
        const int c = c0 + 16 * j + li;
        if (r < n && c < m) C[r * ldc + c] = acc[b][j][v];
      }
}

// ---- X <- X R in place on the matrix cores (real, X [n x nv] with nv <= 80, R [nv x nv]).
// Row-local: each wave owns 16 * RB rows and accumulates all nv output columns (NBJ blocks
// of 16) over the k-steps of 4; every k-step of its rows is read before the wave stores, so
// the result overwrites X.  R, zero-padded to a multiple of 4 rows and 16 NBJ columns, is
// staged in LDS once per workgroup (row stride 16 NBJ + 1).  MFMA f64 16x16x4 layouts: the
// A fragment of lane (li, lk) = (lane % 16, lane / 16) is X[row li][k lk], the B fragment
// R[k lk][col li], and element v of the result is (row lane / 16 + 4 v, col lane % 16).
constexpr int kRowMulRB = 2;  // 16-row blocks per wave

template <int NBJ>
__global__ __launch_bounds__(256) void rowmul_mfma_kernel(double* __restrict__ X, int64_t ldx, int64_t n, int nv,
                                                          const double* __restrict__ R,
                                                          const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;  // the device-side gate (set by an earlier kernel) says skip
  extern __shared__ double rsm[];  // [nks * 4][16 NBJ + 1]
  constexpr int RS = 16 * NBJ + 1;
  const int nks = (nv + 3) / 4;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int t = threadIdx.x; t < nks * 4 * 16 * NBJ; t += 256) {
    const int k = t / (16 * NBJ), c = t - k * (16 * NBJ);
    rsm[k * RS + c] = (k < nv && c < nv) ? R[(int64_t)k * nv + c] : 0.0;
  }
  __syncthreads();
  // persistent: the workgroup keeps R in LDS and takes tasks of 64 RB rows in turn
  const int64_t ntask = (n + 64 * kRowMulRB - 1) / (64 * kRowMulRB);
  for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
  const int64_t r0 = (task * 4 + w) * 16 * kRowMulRB;
  if (r0 >= n) continue;
  const double* xr[kRowMulRB];
  double mrow[kRowMulRB];
#pragma unroll
  for (int b = 0; b < kRowMulRB; ++b) {
    const int64_t r = r0 + 16 * b + li;
    mrow[b] = r < n ? 1.0 : 0.0;
    xr[b] = X + (r < n ? r : n - 1) * ldx;
  }
  dv4 acc[kRowMulRB][NBJ];
#pragma unroll
  for (int b = 0; b < kRowMulRB; ++b)
#pragma unroll
    for (int j = 0; j < NBJ; ++j) acc[b][j] = dv4{0, 0, 0, 0};
  // A fragments of k-step s (columns past nv: clamped, zeroed)
  auto load = [&](int s, double (&a)[kRowMulRB]) {
    const int c = 4 * s + lk;
    const double m = c < nv ? 1.0 : 0.0;
    const int cc = c < nv ? c : nv - 1;
#pragma unroll
    for (int b = 0; b < kRowMulRB; ++b) a[b] = xr[b][cc] * (m * mrow[b]);
  };
  auto mma = [&](int s, const double (&a)[kRowMulRB]) {
    const double* rk = rsm + (4 * s + lk) * RS + li;
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
      const double bj = rk[16 * j];
#pragma unroll
      for (int b = 0; b < kRowMulRB; ++b) acc[b][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[b], bj, acc[b][j], 0, 0, 0);
    }
  };
  double a0[kRowMulRB], a1[kRowMulRB];
  load(0, a0);
  int s = 0;
  for (; s + 1 < nks; s += 2) {
    load(s + 1, a1);
    mma(s, a0);
    if (s + 2 < nks) load(s + 2, a0);
    mma(s + 1, a1);
  }
  if (s < nks) mma(s, a0);
  // every k-step of these rows has been read: store the result over them
#pragma unroll
  for (int b = 0; b < kRowMulRB; ++b)
#pragma unroll
    for (int j = 0; j < NBJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + 16 * b + lk + 4 * v;
        const int c = 16 * j + li;
        if (r < n && c < nv) X[r * ldx + c] = acc[b][j][v];
      }
  }
}

// Same method for small n, in two kernels.
// jacobi_rot_kernel (one workgroup): the matrix in LDS, upper triangle only (the lower
// one is its conjugate transpose and is never read).  One round of the round-robin
// ordering rotates n/2 disjoint pairs at once, so A <- G^* A G factors into independent
// 2x2 blocks: block (k1, k2) of rows (p1, q1) and columns (p2, q2) becomes
// G_k1^* B G_k2, and block (k2, k1) is its conjugate transpose, so only the blocks
// k1 <= k2 are computed.  A round is two barrier-separated phases: (a) the rotations,
// which are also written to a record, (b) the block updates.  The eigenvalues are the
// diagonal, ranked ascending.
// jacobi_vec_kernel (n/4 workgroups, one wave per row of V): applies the recorded
// rotations of every round in order to its row of V = I, then writes the row to U with
// the columns in rank order.  Rows of V evolve independently, so the accumulation of
// the eigenvectors leaves the single-workgroup kernel.
constexpr int kJacobiRecSweeps = 40;  // sweeps the rotation record holds
constexpr int kJacobiGlobalSweeps = 60;  // sweep limit of the global-memory version (jbig_eig)

__device__ __forceinline__ void jacobi_pair(int st, int k, int m, int& p, int& q) {
  if (k == 0) {
    p = 0;
    q = 1 + st % m;
  } else {
    p = 1 + (st + k) % m;
    q = 1 + (st - k + m) % m;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// ---- Parallel cyclic Jacobi in one workgroup, the matrix moved along the pairing ring.
// The round-robin pairing of jacobi_pair is realised physically: the matrix sits in LDS in
// full storage over NN = n + (n odd) positions, positions 2k and 2k + 1 hold pair k of the
// current round, and after every round each index moves to the next position of a fixed
// ring, which makes the next round's pairs adjacent again.  Index 0 stays at position 0; the
// other NN - 1 positions form one cycle, so after NN - 1 rounds (one sweep) every index is
// back where it started.  Every thread therefore updates 2x2 blocks at fixed positions.  The
// padding index of odd n has a zero row and column and is never rotated.

// position that the index at position j moves to after a round
__device__ __forceinline__ int jacobi_ring_next(int j, int npair) {
  const int k = j >> 1;
  if ((j & 1) == 0) return k == 0 ? 0 : (k == 1 ? 1 : 2 * (k - 1));
  return k == npair - 1 ? (npair == 1 ? 1 : 2 * (npair - 1)) : 2 * (k + 1) + 1;
}
// index at position j at the start of a sweep (round 0 of jacobi_pair)
__device__ __forceinline__ int jacobi_ring_index(int j, int m) {
  const int k = j >> 1;
  if ((j & 1) == 0) return k == 0 ? 0 : 1 + k;
  return k == 0 ? 1 : 1 + m - k;
}
// position of index i at the start of a sweep
__device__ __forceinline__ int jacobi_ring_pos(int i, int npair, int m) {
  return i <= 1 ? i : (i <= npair ? 2 * (i - 1) : 2 * (1 + m - i) + 1);
}
// position that the index at position j held in the previous round (inverse of jacobi_ring_next)
__device__ __forceinline__ int jacobi_ring_prev(int j, int npair) {
  const int k = j >> 1;
  if (j <= 1) return j == 0 ? 0 : (npair >= 2 ? 2 : 1);
  if ((j & 1) == 0) return k <= npair - 2 ? 2 * (k + 1) : 2 * (npair - 1) + 1;
  return 2 * (k - 1) + 1;
}

// 1/x and 1/sqrt(x) for x in [1/4, 4]: the hardware estimate refined by two Newton steps
// (each step squares the relative error of the estimate).
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// One plane rotation of a Jacobi round: c, s and the phase er + i ei of a_pq (real: er = sign
// of a_pq); the identity (c = 1, s = 0, er = 1, ei = 0) when the pair is not rotated.
struct JacobiRot {
  double c, s, er, ei;
  bool on;
};

// The rotation that annihilates a_pq = b of the Hermitian 2x2 pivot [al, b; conj(b), ga]:
// t = tan(phi) = sgn(d) 2|b| / (|d| + sqrt(d^2 + 4|b|^2)) with d = ga - al (the smaller root
// of t^2 + (d/|b|) t - 1 = 0), c = 1/sqrt(1 + t^2), s = t c.  d and 2|b| are first scaled
// by a power of two that brings the larger into [1/2, 1), so t needs no unscaling and every
// reciprocal and square root sees an argument in [1/4, 4].  The pair is rotated only when
// |b| lies above float64 rounding, measured on its diagonal entries or on the matrix norm
// (whichever is larger).  No branches: the identity is selected when the pair is not rotated.
template <bool CPLX>
__device__ __forceinline__ JacobiRot jacobi_rotation(double al, double ga, double br, double bi, double nrm_n) {
  const double r = CPLX ? sqrt(br * br + bi * bi) : fabs(br);
  const bool on = r > 1e-300 && r > 2.220446049250313e-16 * fmax(sqrt(fabs(al * ga)), nrm_n);
  const double d = ga - al;
  const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(d), 2.0 * r));
  const double ds = ldexp(d, -ex), rs2 = ldexp(2.0 * r, -ex);  // max(|ds|, rs2) in [1/2, 1)
  const double x = fma(ds, ds, rs2 * rs2);                     // [1/4, 2]
  const double w = x * rsq_refined(x);                         // sqrt(x)
  const double t = (d >= 0 ? rs2 : -rs2) * rcp_refined(fabs(ds) + w);
  const double c = rsq_refined(fma(t, t, 1.0));
  JacobiRot R;
  R.on = on;
  R.c = on ? c : 1.0;
  R.s = on ? t * c : 0.0;
  if constexpr (CPLX) {
    const double ir = 1.0 / r;
    R.er = on ? br * ir : 1.0;
    R.ei = on ? bi * ir : 0.0;
  } else {
    R.er = on ? (br >= 0 ? 1.0 : -1.0) : 1.0;
    R.ei = 0.0;
  }
  return R;
}

template <bool CPLX>
__device__ __forceinline__ Z jz_load(const double* a) {
  if constexpr (CPLX) return Z{a[0], a[1]};
  else return Z{a[0], 0.0};
}
template <bool CPLX>
__device__ __forceinline__ void jz_store(double* a, Z v) {
  a[0] = v.r;
  if constexpr (CPLX) a[1] = v.i;
}
template <bool CPLX>
__device__ __forceinline__ Z jz_mul(Z a, Z b) {
  if constexpr (CPLX) return zmul(a, b);
  else return Z{a.r * b.r, 0.0};
}
template <bool CPLX>
__device__ __forceinline__ Z jz_fma(Z a, Z b, Z c) {  // a b + c
  if constexpr (CPLX) return Z{fma(a.r, b.r, fma(-a.i, b.i, c.r)), fma(a.r, b.i, fma(a.i, b.r, c.i))};
  else return Z{fma(a.r, b.r, c.r), 0.0};
}
__device__ __forceinline__ Z jz_conj(Z a) { return Z{a.r, -a.i}; }
// entry (a, b) of G1^* B G2 for 2x2 matrices stored row-major
template <bool CPLX>
__device__ __forceinline__ Z jz_entry(const Z* G1, const Z* B, const Z* G2, int a, int b) {
  // columns a of G1 and b of G2 by selects (a, b may vary per lane)
  const Z g1a0 = a ? G1[1] : G1[0], g1a1 = a ? G1[3] : G1[2];
  const Z g2b0 = b ? G2[1] : G2[0], g2b1 = b ? G2[3] : G2[2];
  const Z c0 = jz_fma<CPLX>(B[1], g2b1, jz_mul<CPLX>(B[0], g2b0));  // (B G2)[0][b]
  const Z c1 = jz_fma<CPLX>(B[3], g2b1, jz_mul<CPLX>(B[2], g2b0));  // (B G2)[1][b]
  return jz_fma<CPLX>(jz_conj(g1a1), c1, jz_mul<CPLX>(jz_conj(g1a0), c0));
}

size_t jacobi_rot_lds_bytes(bool cplx, int n) {
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, E = cplx ? 2 : 1;
  const size_t nblk = (size_t)npair * (npair + 1) / 2;
  return ((size_t)NN * (NN + 1) * E + 4 * (size_t)E * npair + 32) * sizeof(double) + nblk * sizeof(uint16_t);
}

// Rotations of all sweeps are recorded (c, s, er, ei per pair and round, in the orientation
// p < q of jacobi_pair) for jacobi_vec_kernel; eigenvalues come out in ascending order with
// the rank of every index.
template <bool CPLX, int KB>
__global__ __launch_bounds__(1024) void jacobi_rot_kernel(const double* __restrict__ A, int n,
                                                          double* __restrict__ lam, int32_t* __restrict__ rank_out,
                                                          double* __restrict__ rec, int32_t* __restrict__ status, int max_sweeps) {
  constexpr int E = CPLX ? 2 : 1;
  extern __shared__ double sm[];
  const int NN = (n % 2) ? n + 1 : n;  // padded size for the schedule
  const int npair = NN / 2, m = NN - 1;
  const int nblk = npair * (npair + 1) / 2;
  // storage as in jacobi_ring1_kernel: slot-major rows / columns with an odd row stride, the
  // rotation table as four arrays
  const int ld = NN + 1;
  double* As = sm;
  double* gph = As + (size_t)NN * ld * E;       // [4][npair]: the 2x2 transforms by position
  double* red = gph + 4 * (size_t)E * npair;    // 2 per wave (<= 32)
  uint16_t* blk = reinterpret_cast<uint16_t*>(red + 32);  // k1 | k2 << 8, k1 <= k2
  __shared__ int anyrot;  // a rotation was applied in the current sweep
  const int tid = threadIdx.x, nth = blockDim.x;
  auto slot = [npair](int j) { return (j & 1) * npair + (j >> 1); };
  auto at = [&](int pi, int pj) { return slot(pi) * ld + slot(pj); };
  auto gtab = [&](int e) { return gph + (size_t)e * npair * E; };
  // A (Hermitian; its upper triangle is read) at the ring positions of a sweep's start
  for (int t = tid; t < NN * NN; t += nth) {
    const int pi = t / NN, pj = t - pi * NN;
    const int i = jacobi_ring_index(pi, m), j = jacobi_ring_index(pj, m);
    double vr = 0.0, vi = 0.0;
    if (i < n && j < n) {
      const double* a = A + ((size_t)min(i, j) * n + max(i, j)) * E;
      vr = a[0];
      if (CPLX) vi = i == j ? 0.0 : (i < j ? a[E - 1] : -a[E - 1]);
    }
    As[(size_t)at(pi, pj) * E] = vr;
    if (CPLX) As[(size_t)at(pi, pj) * E + 1] = vi;
  }
  for (int b = tid; b < nblk; b += nth) {
    int k1 = 0, bb = b;
    while (bb >= npair - k1) {
      bb -= npair - k1;
      ++k1;
    }
    blk[b] = (uint16_t)(k1 | ((k1 + bb) << 8));
  }
  __syncthreads();
  // this thread's blocks (k1, k2), k1 <= k2: where their four entries are, and where the
  // entries and their mirror images move to
  int myblk[KB], src[KB][4], dst[KB][4], mir[KB][4];
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    const int bb = tid + i * nth;
    myblk[i] = bb < nblk ? (int)blk[bb] : -1;
    const int kk = myblk[i] < 0 ? 0 : myblk[i];
    const int k1 = kk & 255, k2 = kk >> 8;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int r = jacobi_ring_next(2 * k1 + a, npair), q = jacobi_ring_next(2 * k2 + c, npair);
        src[i][2 * a + c] = at(2 * k1 + a, 2 * k2 + c);
        dst[i][2 * a + c] = at(r, q);
        mir[i][2 * a + c] = at(q, r);
      }
  }
  const int kp = tid < npair ? tid : 0;
  const int opiv = at(2 * kp, 2 * kp), opiv1 = at(2 * kp + 1, 2 * kp + 1), opq = at(2 * kp, 2 * kp + 1);
  int sweep = 0, nrec = 0;
  bool conv = false;
  for (; sweep < min(kJacobiRecSweeps, max_sweeps); ++sweep) {
    // convergence test: squared Frobenius norms of the off-diagonal and diagonal parts
    double off = 0, dia = 0;
    for (int t = tid; t < NN * NN; t += nth) {
      const int i = t / NN, j = t - i * NN;
      const double* a = As + ((size_t)i * ld + j) * E;
      const double v = a[0] * a[0] + (CPLX ? a[1] * a[1] : 0.0);
      if (i == j) dia += v;
      else off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dia += __shfl_xor(dia, o);
    }
    if ((tid & 63) == 0) {
      red[2 * (tid >> 6)] = off;
      red[2 * (tid >> 6) + 1] = dia;
    }
    __syncthreads();
    double offs = 0, dias = 0;
    for (int w = 0; w < nth / 64; ++w) {
      offs += red[2 * w];
      dias += red[2 * w + 1];
    }
    const double nrm_n = sqrt(offs + dias) / n;  // Frobenius norm / n
    if (tid == 0) anyrot = 0;
    __syncthreads();
    if (offs <= 1e-30 * dias || offs == 0.0) {
      conv = true;
      break;
    }
    double* rrec = rec + (size_t)nrec * m * npair * 4;
    // schedule positions (st + k) mod m and (st - k) mod m of pair k = tid
    int sa = kp % m, sb = (m - kp % m) % m;
    for (int st = 0; st < m; ++st) {
      // (a) one thread per pair forms the rotation of the pair at positions (2k, 2k+1); every
      // thread reads its blocks (the previous round has finished moving them)
      if (tid < npair) {
        const int k = tid;
        const double a00 = As[(size_t)opiv * E], a11 = As[(size_t)opiv1 * E];
        const Z b = jz_load<CPLX>(As + (size_t)opq * E);
        const bool sw = k >= 1 && sa > sb;  // position 2k holds q
        const JacobiRot g = jacobi_rotation<CPLX>(sw ? a11 : a00, sw ? a00 : a11, b.r, sw ? -b.i : b.i, nrm_n);
        double* R = rrec + ((size_t)st * npair + k) * 4;
        R[0] = g.c; R[1] = g.s; R[2] = g.er; R[3] = g.ei;
        // columns (p, q) <- (p, q) G with G = [c, s; -s conj(e), c conj(e)], e = er + i ei;
        // by position the rows and columns of G are swapped when position 2k holds q
        const Z g00{g.c, 0.0}, g01{g.s, 0.0}, g10{-g.s * g.er, g.s * g.ei}, g11{g.c * g.er, -g.c * g.ei};
        jz_store<CPLX>(gtab(0) + (size_t)k * E, sw ? g11 : g00);
        jz_store<CPLX>(gtab(1) + (size_t)k * E, sw ? g10 : g01);
        jz_store<CPLX>(gtab(2) + (size_t)k * E, sw ? g01 : g10);
        jz_store<CPLX>(gtab(3) + (size_t)k * E, sw ? g00 : g11);
        if (g.on) anyrot = 1;
        sa = sa + 1 == m ? 0 : sa + 1;
        sb = sb + 1 == m ? 0 : sb + 1;
      }
      Z bl[KB][4];
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        if (myblk[i] < 0) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) bl[i][e] = jz_load<CPLX>(As + (size_t)src[i][e] * E);
      }
      __syncthreads();
      // (b) B <- G_k1^* B G_k2, written to the positions of the next round
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        if (myblk[i] < 0) break;
        const int k1 = myblk[i] & 255, k2 = myblk[i] >> 8;
        Z u[4], v[4], d[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          u[e] = jz_load<CPLX>(gtab(e) + (size_t)k1 * E);
          v[e] = jz_load<CPLX>(gtab(e) + (size_t)k2 * E);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] = jz_entry<CPLX>(u, bl[i], v, e >> 1, e & 1);
        if (k1 == k2) {
          if (u[1].r != 0.0 || u[1].i != 0.0) {  // the rotated pair; its diagonal stays real
            d[1] = d[2] = Z{0.0, 0.0};
            d[0].i = 0.0;
            d[3].i = 0.0;
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) jz_store<CPLX>(As + (size_t)dst[i][e] * E, d[e]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            jz_store<CPLX>(As + (size_t)dst[i][e] * E, d[e]);
            jz_store<CPLX>(As + (size_t)mir[i][e] * E, jz_conj(d[e]));
          }
        }
      }
      __syncthreads();
    }
    // a sweep that found no pair coupled above rounding: converged (its record is the identity)
    if (anyrot == 0) {
      ++sweep;
      conv = true;
      break;
    }
    ++nrec;
  }
  if (tid == 0) {
    status[0] = conv ? 0 : OEFE_ENOCONV;
    status[1] = sweep;
    rank_out[n] = nrec;
  }
  // the layout is that of a sweep's start: eigenvalue of index i at position jacobi_ring_pos(i)
  double* dg = gph;  // NN <= 4 E npair doubles
  for (int i = tid; i < n; i += nth) {
    const int q = jacobi_ring_pos(i, npair, m);
    dg[i] = As[(size_t)at(q, q) * E];
  }
  __syncthreads();
  // ascending order by rank
  for (int i = tid; i < n; i += nth) {
    const double li = dg[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = dg[j];
      if (lj < li || (lj == li && j < i)) ++rank;
    }
    lam[rank] = li;
    rank_out[i] = rank;
  }
}

// The same Jacobi with one barrier per round (real or small n: the matrix is double
// buffered in LDS and every block fits one thread).  Within a round every block thread reads
// the current matrix and rotation table and writes the moved blocks to the other buffer,
// while one thread per pair, in waves of their own, forms the rotation of the NEXT round: the
// two indices that pair k meets at positions (2k, 2k+1) next round sit at positions
// u = jacobi_ring_prev(2k) and v = jacobi_ring_prev(2k+1) now, in different pairs, so the
// next pivot entries are entries of G_u^* B G_v for blocks B of the current matrix.
// Storage is slot-major: position j is kept at row / column (j odd) * npair + j / 2, so a
// ring step moves an entry by one column, and the blocks of neighbouring lanes (neighbouring
// k2) are read and written at neighbouring addresses; the odd row stride spreads the mirror
// images, written along a column, over the LDS banks.  The rotation table is kept as four
// arrays (one per entry of the 2x2 transform).
size_t jacobi_ring1_lds_bytes(bool cplx, int n) {
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, E = cplx ? 2 : 1;
  const size_t nblk = (size_t)npair * (npair + 1) / 2;
  return (2 * (size_t)NN * (NN + 1) * E + 8 * (size_t)E * npair + 32) * sizeof(double) + nblk * sizeof(uint16_t);
}
// block threads (one block each) and the waves of rotation threads fit 1024 threads
bool jacobi_ring1_fits(int n) {
  const int npair = (n + 1) / 2;
  return npair * (npair + 1) / 2 <= 1024 - 64 * ((npair + 63) / 64);
}

template <bool CPLX>
__global__ __launch_bounds__(1024) void jacobi_ring1_kernel(const double* __restrict__ A, int n,
                                                            double* __restrict__ lam, int32_t* __restrict__ rank_out,
                                                            double* __restrict__ rec, int32_t* __restrict__ status, int max_sweeps) {
  constexpr int E = CPLX ? 2 : 1;
  extern __shared__ double sm[];
  const int NN = (n % 2) ? n + 1 : n;  // padded size for the schedule
  const int npair = NN / 2, m = NN - 1;
  const int nblk = npair * (npair + 1) / 2;
  const int ld = NN + 1;
  const size_t msz = (size_t)NN * ld * E;
  double* Gt0 = sm + 2 * msz;                    // two rotation tables [4][npair]
  double* red = Gt0 + 8 * (size_t)E * npair;     // 2 per wave (<= 32)
  uint16_t* blk = reinterpret_cast<uint16_t*>(red + 32);  // k1 | k2 << 8, k1 <= k2
  __shared__ int anyrot;  // a rotation was applied in the current sweep
  const int tid = threadIdx.x, nth = blockDim.x;
  const int rbase = nth - 64 * ((npair + 63) / 64);  // rotation threads: pair kr = tid - rbase
  const int kr = tid - rbase;
  const bool is_rot = kr >= 0 && kr < npair;
  auto slot = [npair](int j) { return (j & 1) * npair + (j >> 1); };  // storage row / column of position j
  auto at = [&](int pi, int pj) { return slot(pi) * ld + slot(pj); };  // entry offset of (pi, pj)
  for (int t = tid; t < NN * NN; t += nth) {
    const int pi = t / NN, pj = t - pi * NN;
    const int i = jacobi_ring_index(pi, m), j = jacobi_ring_index(pj, m);
    double vr = 0.0, vi = 0.0;
    if (i < n && j < n) {
      const double* a = A + ((size_t)min(i, j) * n + max(i, j)) * E;
      vr = a[0];
      if (CPLX) vi = i == j ? 0.0 : (i < j ? a[E - 1] : -a[E - 1]);
    }
    sm[(size_t)at(pi, pj) * E] = vr;
    if (CPLX) sm[(size_t)at(pi, pj) * E + 1] = vi;
  }
  for (int b = tid; b < nblk; b += nth) {
    int k1 = 0, bb = b;
    while (bb >= npair - k1) {
      bb -= npair - k1;
      ++k1;
    }
    blk[b] = (uint16_t)(k1 | ((k1 + bb) << 8));
  }
  __syncthreads();
  const int myb = tid < nblk ? (int)blk[tid] : -1;
  const int k1 = myb < 0 ? 0 : (myb & 255), k2 = myb < 0 ? 0 : (myb >> 8);
  int src[4], dst[4], mir[4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int r = jacobi_ring_next(2 * k1 + a, npair), q = jacobi_ring_next(2 * k2 + c, npair);
      src[2 * a + c] = at(2 * k1 + a, 2 * k2 + c);
      dst[2 * a + c] = at(r, q);
      mir[2 * a + c] = at(q, r);
    }
  const int krc = is_rot ? kr : 0;
  const int pu = jacobi_ring_prev(2 * krc, npair), pv = jacobi_ring_prev(2 * krc + 1, npair);
  const int ku = pu >> 1, ul = pu & 1, kv = pv >> 1, vl = pv & 1;
  int ouu[4], ovv[4], ouv[4];  // blocks (ku, ku), (kv, kv), (ku, kv)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      ouu[2 * a + c] = at(2 * ku + a, 2 * ku + c);
      ovv[2 * a + c] = at(2 * kv + a, 2 * kv + c);
      ouv[2 * a + c] = at(2 * ku + a, 2 * kv + c);
    }
  const int opiv = at(2 * krc, 2 * krc), opiv1 = at(2 * krc + 1, 2 * krc + 1), opq = at(2 * krc, 2 * krc + 1);
  int cb = 0, gb = 0;  // current matrix buffer and rotation table
  int sweep = 0, nrec = 0;
  bool conv = false;
  auto gtab = [&](int g, int e) { return Gt0 + ((size_t)(g * 4 + e) * npair) * E; };
  // pair kr's rotation from its pivot entries as stored at positions (2kr, 2kr+1): record it and
  // put its transform by position into table g
  auto form = [&](double a00, double a11, Z b, int sa, int sb, double nrm_n, int g, double* R) {
    const bool sw = kr >= 1 && sa > sb;  // position 2kr holds q
    const JacobiRot q = jacobi_rotation<CPLX>(sw ? a11 : a00, sw ? a00 : a11, b.r, sw ? -b.i : b.i, nrm_n);
    R[0] = q.c; R[1] = q.s; R[2] = q.er; R[3] = q.ei;
    const Z g00{q.c, 0.0}, g01{q.s, 0.0}, g10{-q.s * q.er, q.s * q.ei}, g11{q.c * q.er, -q.c * q.ei};
    jz_store<CPLX>(gtab(g, 0) + (size_t)kr * E, sw ? g11 : g00);
    jz_store<CPLX>(gtab(g, 1) + (size_t)kr * E, sw ? g10 : g01);
    jz_store<CPLX>(gtab(g, 2) + (size_t)kr * E, sw ? g01 : g10);
    jz_store<CPLX>(gtab(g, 3) + (size_t)kr * E, sw ? g00 : g11);
    if (q.on) anyrot = 1;
  };
  auto ldblk = [&](const double* Ab, const int* o, Z* B) {
#pragma unroll
    for (int e = 0; e < 4; ++e) B[e] = jz_load<CPLX>(Ab + (size_t)o[e] * E);
  };
  auto ldrot = [&](int g, int k, Z* G) {
#pragma unroll
    for (int e = 0; e < 4; ++e) G[e] = jz_load<CPLX>(gtab(g, e) + (size_t)k * E);
  };
  for (; sweep < min(kJacobiRecSweeps, max_sweeps); ++sweep) {
    const double* Ac = sm + cb * msz;
    double off = 0, dia = 0;
    for (int t = tid; t < NN * NN; t += nth) {
      const int i = t / NN, j = t - i * NN;
      const double* a = Ac + ((size_t)i * ld + j) * E;
      const double v = a[0] * a[0] + (CPLX ? a[1] * a[1] : 0.0);
      if (i == j) dia += v;
      else off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dia += __shfl_xor(dia, o);
    }
    if ((tid & 63) == 0) {
      red[2 * (tid >> 6)] = off;
      red[2 * (tid >> 6) + 1] = dia;
    }
    __syncthreads();
    double offs = 0, dias = 0;
    for (int w = 0; w < nth / 64; ++w) {
      offs += red[2 * w];
      dias += red[2 * w + 1];
    }
    const double nrm_n = sqrt(offs + dias) / n;  // Frobenius norm / n
    if (tid == 0) anyrot = 0;
    __syncthreads();
    if (offs <= 1e-30 * dias || offs == 0.0) {
      conv = true;
      break;
    }
    double* rrec = rec + (size_t)nrec * m * npair * 4;
    int sa = krc % m, sb = (m - krc % m) % m;  // (round + kr) mod m, (round - kr) mod m
    if (is_rot) {  // rotations of round 0 from the pivots
      form(Ac[(size_t)opiv * E], Ac[(size_t)opiv1 * E], jz_load<CPLX>(Ac + (size_t)opq * E), sa, sb, nrm_n, gb,
           rrec + (size_t)kr * 4);
      sa = sa + 1 == m ? 0 : sa + 1;
      sb = sb + 1 == m ? 0 : sb + 1;
    }
    __syncthreads();
    for (int st = 0; st < m; ++st) {
      const double* Acur = sm + cb * msz;
      double* Anext = sm + (cb ^ 1) * msz;
      if (myb >= 0) {  // B <- G_k1^* B G_k2, written to the positions of the next round
        Z u[4], v[4], B[4];
        ldrot(gb, k1, u);
        ldrot(gb, k2, v);
        ldblk(Acur, src, B);
        Z d[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] = jz_entry<CPLX>(u, B, v, e >> 1, e & 1);
        if (k1 == k2) {
          if (u[1].r != 0.0 || u[1].i != 0.0) {  // the rotated pair; its diagonal stays real
            d[1] = d[2] = Z{0.0, 0.0};
            d[0].i = 0.0;
            d[3].i = 0.0;
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) jz_store<CPLX>(Anext + (size_t)dst[e] * E, d[e]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            jz_store<CPLX>(Anext + (size_t)dst[e] * E, d[e]);
            jz_store<CPLX>(Anext + (size_t)mir[e] * E, jz_conj(d[e]));
          }
        }
      }
      if (is_rot && st + 1 < m) {  // rotation of pair kr in the next round
        Z gu[4], gv[4], Buu[4], Bvv[4], Buv[4];
        ldrot(gb, ku, gu);
        ldrot(gb, kv, gv);
        ldblk(Acur, ouu, Buu);
        ldblk(Acur, ovv, Bvv);
        ldblk(Acur, ouv, Buv);
        const double xuu = jz_entry<CPLX>(gu, Buu, gu, ul, ul).r;
        const double xvv = jz_entry<CPLX>(gv, Bvv, gv, vl, vl).r;
        const Z xuv = jz_entry<CPLX>(gu, Buv, gv, ul, vl);
        form(xuu, xvv, xuv, sa, sb, nrm_n, gb ^ 1, rrec + ((size_t)(st + 1) * npair + kr) * 4);
        sa = sa + 1 == m ? 0 : sa + 1;
        sb = sb + 1 == m ? 0 : sb + 1;
      }
      __syncthreads();
      cb ^= 1;
      gb ^= 1;
    }
    // a sweep that found no pair coupled above rounding: converged (its record is the identity)
    if (anyrot == 0) {
      ++sweep;
      conv = true;
      break;
    }
    ++nrec;
  }
  if (tid == 0) {
    status[0] = conv ? 0 : OEFE_ENOCONV;
    status[1] = sweep;
    rank_out[n] = nrec;
  }
  // the layout is that of a sweep's start: eigenvalue of index i at position jacobi_ring_pos(i)
  const double* Af = sm + cb * msz;
  double* dg = Gt0;  // NN <= 8 E npair doubles
  for (int i = tid; i < n; i += nth) {
    const int q = jacobi_ring_pos(i, npair, m);
    dg[i] = Af[(size_t)at(q, q) * E];
  }
  __syncthreads();
  for (int i = tid; i < n; i += nth) {
    const double li = dg[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = dg[j];
      if (lj < li || (lj == li && j < i)) ++rank;
    }
    lam[rank] = li;
    rank_out[i] = rank;
  }
}

constexpr int kJacobiVecChunk = 8192;  // doubles of the rotation record staged in LDS at a time

size_t jacobi_vec_lds_bytes(bool cplx, int n) {
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, m = NN - 1;
  return ((size_t)kJacobiVecChunk + 4 * (size_t)n * (cplx ? 2 : 1)) * sizeof(double) +
         (size_t)m * npair * sizeof(int);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void jacobi_vec_kernel(const double* __restrict__ rec,
                                                         const int32_t* __restrict__ rank, int n,
                                                         double* __restrict__ U) {
  constexpr int E = CPLX ? 2 : 1;
  extern __shared__ double sm[];
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, m = NN - 1;
  double* chunk = sm;                                      // kJacobiVecChunk
  double* vall = chunk + kJacobiVecChunk;                  // [4][n][E]
  int* sched = reinterpret_cast<int*>(vall + 4 * n * E);   // [m][npair]: p | q << 16
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = blockIdx.x * 4 + w;  // row of V (waves past n idle along)
  double* v = vall + (size_t)w * n * E;
  const int nround = rank[n] * m;
  const int cr = max(1, kJacobiVecChunk / (4 * npair));  // rounds per chunk
  for (int t = tid; t < m * npair; t += 256) {
    int p, q;
    jacobi_pair(t / npair, t - (t / npair) * npair, m, p, q);
    sched[t] = p | (q << 16);
  }
  for (int i = lane; i < n; i += 64) {
    v[(size_t)i * E] = i == r ? 1.0 : 0.0;
    if (CPLX) v[(size_t)i * E + 1] = 0.0;
  }
  for (int s0 = 0; s0 < nround; s0 += cr) {
    const int ns = min(cr, nround - s0);
    __syncthreads();  // the previous chunk is no longer read
    const double* src = rec + (size_t)s0 * npair * 4;
    for (int t = tid; t < ns * npair * 4; t += 256) chunk[t] = src[t];
    __syncthreads();
    if (r < n && npair <= 64) {
      // one pair per lane: the next round's rotation and pair are read while this round's
      // entries are updated
      const int k = min(lane, npair - 1);
      const bool act = lane < npair;
      int rr = s0 % m;
      double c = chunk[k * 4], sn = chunk[k * 4 + 1], e2 = chunk[k * 4 + 2], e3 = chunk[k * 4 + 3];
      int pq = sched[rr * npair + k];
      for (int j = 0; j < ns; ++j) {
        const double cc = c, ss = sn, f2 = e2, f3 = e3;
        const int pqc = pq;
        if (j + 1 < ns) {
          rr = rr + 1 == m ? 0 : rr + 1;
          const double* R = chunk + ((size_t)(j + 1) * npair + k) * 4;
          c = R[0]; sn = R[1]; e2 = R[2]; e3 = R[3];
          pq = sched[rr * npair + k];
        }
        const int p = pqc & 0xffff, q = pqc >> 16;
        if (act && q < n && ss != 0.0) {
          double* vp = v + (size_t)p * E;
          double* vq = v + (size_t)q * E;
          if constexpr (!CPLX) {
            const double x = vp[0], y = vq[0] * f2;
            vp[0] = x * cc - y * ss;
            vq[0] = x * ss + y * cc;
          } else {
            const Z emi{f2, -f3};
            const Z x{vp[0], vp[1]}, y{vq[0], vq[1]};
            const Z ye = zmul(y, emi);
            vp[0] = x.r * cc - ye.r * ss; vp[1] = x.i * cc - ye.i * ss;
            vq[0] = x.r * ss + ye.r * cc; vq[1] = x.i * ss + ye.i * cc;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
    } else if (r < n) {
      for (int j = 0; j < ns; ++j) {
        const int* sp = sched + (size_t)((s0 + j) % m) * npair;
        for (int k = lane; k < npair; k += 64) {
          const double* R = chunk + ((size_t)j * npair + k) * 4;
          const double c = R[0], sn = R[1];
          const int pq = sp[k], p = pq & 0xffff, q = pq >> 16;
          if (q >= n || sn == 0.0) continue;
          double* vp = v + (size_t)p * E;
          double* vq = v + (size_t)q * E;
          if constexpr (!CPLX) {
            const double x = vp[0], y = vq[0] * R[2];
            vp[0] = x * c - y * sn;
            vq[0] = x * sn + y * c;
          } else {
            const Z emi{R[2], -R[3]};
            const Z x{vp[0], vp[1]}, y{vq[0], vq[1]};
            const Z ye = zmul(y, emi);
            vp[0] = x.r * c - ye.r * sn; vp[1] = x.i * c - ye.i * sn;
            vq[0] = x.r * sn + ye.r * c; vq[1] = x.i * sn + ye.i * c;
          }
        }
        // the next round reads entries this round's other lanes wrote
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
    }
  }
  if (r < n) {
    for (int i = lane; i < n; i += 64) {
      const int c = rank[i];
      U[((int64_t)r * n + c) * E] = v[(size_t)i * E];
      if (CPLX) U[((int64_t)r * n + c) * E + 1] = v[(size_t)i * E + 1];
    }
  }
}

// Eigenvectors from the rotation record by the pairing ring (npair <= 64): one wave holds
// RPW rows of V in registers by position, lane k the entries at positions 2k and 2k + 1 (the
// pair k of the round).  A round applies the pair's 2x2 transform by position and then moves
// the entries along the ring with two lane shifts: slot 0 of lane k comes from slot 0 of lane
// k + 1 and slot 1 from slot 1 of lane k - 1, except slot 0 of lane 0 (stays), slot 1 of
// lane 0 (from slot 0 of lane 1) and slot 0 of the last pair (from its own slot 1).  The
// rotations of the next kJacobiVecAhead rounds are loaded ahead from the record.
constexpr int kJacobiVecAhead = 4;
constexpr int kJacobiVecRows = 1;  // rows of V per wave

template <bool CPLX>
__global__ __launch_bounds__(64) void jacobi_vec_ring_kernel(const double* __restrict__ rec,
                                                             const int32_t* __restrict__ rank, int n,
                                                             double* __restrict__ U) {
  constexpr int E = CPLX ? 2 : 1, RPW = kJacobiVecRows, D = kJacobiVecAhead;
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, m = NN - 1;
  const int k = threadIdx.x;
  const int kc = k < npair ? k : npair - 1;
  const int r0 = blockIdx.x * RPW;
  const int i0 = jacobi_ring_index(2 * kc, m), i1 = jacobi_ring_index(2 * kc + 1, m);
  // positions 2k, 2k + 1 of rows r0 .. r0 + RPW - 1, real and imaginary parts (V starts as I)
  double v0r[RPW], v0i[RPW], v1r[RPW], v1i[RPW];
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    v0r[q] = i0 == r0 + q ? 1.0 : 0.0;
    v1r[q] = i1 == r0 + q ? 1.0 : 0.0;
    v0i[q] = v1i[q] = 0.0;
  }
  const int nround = rank[n] * m;
  int sa = kc % m, sb = (m - kc % m) % m;  // (round + k) mod m, (round - k) mod m
  const double* rk = rec + (size_t)kc * 4;
  const size_t rstride = (size_t)npair * 4;
  double bufa[D][4], bufb[D][4];
  auto fetch = [&](int t0, double (&bf)[D][4]) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int t = min(t0 + d, max(nround - 1, 0));
      const double* R = rk + (size_t)t * rstride;
      // real rotations have ei = 0: no load is issued for it (a loaded, unused register
      // would be reused while its load is in flight)
#pragma unroll
      for (int e = 0; e < 4; ++e) bf[d][e] = (CPLX || e < 3) ? R[e] : 0.0;
    }
  };
  // rounds tb .. tb + D - 1 (those below nround) with the rotations in bf
  auto run = [&](int tb, const double (&bf)[D][4]) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (tb + d < nround) {
        const double c = bf[d][0], sn = bf[d][1], er = bf[d][2], ei = bf[d][3];
        const bool sw = kc >= 1 && sa > sb;  // position 2k holds q
        // (p, q) columns <- (p, q) G, G = [c, s; -s conj(e), c conj(e)]; by position the rows
        // and columns of G are swapped when position 2k holds q
        const Z g00{c, 0.0}, g01{sn, 0.0}, g10{-sn * er, sn * ei}, g11{c * er, -c * ei};
        const Z h00 = sw ? g11 : g00, h01 = sw ? g10 : g01, h10 = sw ? g01 : g10, h11 = sw ? g00 : g11;
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
          const Z a{v0r[q], v0i[q]}, b{v1r[q], v1i[q]};
          const Z n0 = jz_fma<CPLX>(b, h10, jz_mul<CPLX>(a, h00));
          const Z n1 = jz_fma<CPLX>(b, h11, jz_mul<CPLX>(a, h01));
          v0r[q] = n0.r; v1r[q] = n1.r;
          if constexpr (CPLX) { v0i[q] = n0.i; v1i[q] = n1.i; }
        }
        if (npair > 1) {
          const int ka = k + 1, kb = k - 1 < 0 ? 0 : k - 1;
          const bool first = k == 0, last = k == npair - 1;
#pragma unroll
          for (int q = 0; q < RPW; ++q) {
            const double ar = __shfl(v0r[q], ka), br = __shfl(v1r[q], kb);
            const double n0r = first ? v0r[q] : (last ? v1r[q] : ar), n1r = first ? ar : br;
            v0r[q] = n0r;
            v1r[q] = n1r;
            if constexpr (CPLX) {
              const double ai = __shfl(v0i[q], ka), bi = __shfl(v1i[q], kb);
              const double n0i = first ? v0i[q] : (last ? v1i[q] : ai), n1i = first ? ai : bi;
              v0i[q] = n0i;
              v1i[q] = n1i;
            }
          }
        }
        sa = sa + 1 == m ? 0 : sa + 1;
        sb = sb + 1 == m ? 0 : sb + 1;
      }
    }
  };
  if (nround > 0) fetch(0, bufa);
  for (int t0 = 0; t0 < nround; t0 += 2 * D) {
    fetch(t0 + D, bufb);
    run(t0, bufa);
    fetch(t0 + 2 * D, bufa);
    run(t0 + D, bufb);
  }
  // back at the sweep-start layout: position 2k + h holds index jacobi_ring_index(2k + h)
  if (k < npair) {
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const int r = r0 + q;
      if (r >= n) break;
      if (i0 < n) jz_store<CPLX>(U + ((int64_t)r * n + rank[i0]) * E, Z{v0r[q], v0i[q]});
      if (i1 < n) jz_store<CPLX>(U + ((int64_t)r * n + rank[i1]) * E, Z{v1r[q], v1i[q]});
    }
  }
}

// ---- Inverse Cholesky factor by elimination (one workgroup, small n).  Gaussian elimination
// without pivoting of C = [A | I], A the Jacobi-scaled Gram matrix in full storage: step k
// subtracts (c_ik / c_kk) times row k from every row i > k over the columns k < j <= n + k
// (the rest of row k is zero).  That leaves the pivots D = diag(c_kk) of A = L_1 D L_1^*
// (L_1 unit lower) and L_1^-1 in the right half; the Cholesky factor is L = L_1 D^1/2, so
// L^-1 = D^-1/2 L_1^-1.  Step k reads only column k and row k, both final after step k - 1,
// and writes neither, so one barrier per step suffices.  Thread t keeps column k + 1 + t % n
// of the window and the rows k + 1 + t / n + r nth / n.  Same scaling, pivots and breakdown
// rule as chol_lds_kernel; G is only read.
size_t chol_elim_lds_bytes(bool cplx, int n) { return ((size_t)n * (2 * n + 1) * (cplx ? 2 : 1) + n) * sizeof(double); }
bool chol_elim_fits(bool cplx, int n) { return n <= 512 && chol_elim_lds_bytes(cplx, n) <= 158 * 1024; }

// With a gate, the kernel runs only when *gate != 0; go (optional) receives 1 after a
// successful factorization and 0 otherwise (also when the gate skipped it).
template <bool CPLX>
__global__ __launch_bounds__(1024) void chol_elim_kernel(const double* __restrict__ G, int ldg, int n,
                                                         double* __restrict__ Rinv, double* __restrict__ dsc,
                                                         int32_t* __restrict__ status, const int32_t* __restrict__ gate,
                                                         int32_t* __restrict__ go) {
  constexpr int E = CPLX ? 2 : 1;
  if (gate && *gate == 0) {
    if (go && threadIdx.x == 0) *go = 0;
    return;
  }
  extern __shared__ double sm[];
  const int ld = 2 * n + 1;             // odd row stride
  double* C = sm;                       // [n][ld]: [A | I]
  double* d = C + (size_t)n * ld * E;   // [n]: Jacobi scaling
  __shared__ int bad;
  const int tid = threadIdx.x, nth = blockDim.x;
  if (tid == 0) bad = -1;
  __syncthreads();
  for (int i = tid; i < n; i += nth) {
    const double gii = G[((int64_t)i * ldg + i) * E];
    if (!(gii > 0.0)) atomicMax(&bad, i);
    d[i] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
    dsc[i] = d[i];
  }
  __syncthreads();
  if (bad >= 0) {
    if (tid == 0) {
      status[0] = OEFE_ENOTSPD;
      status[1] = bad;
      if (go) *go = 0;
    }
    return;
  }
  for (int t = tid; t < n * n; t += nth) {
    const int i = t / n, j = t - i * n;
    const double sc = d[i] * d[j];
    const double* g = G + ((int64_t)i * ldg + j) * E;
    double* a = C + ((size_t)i * ld + j) * E;
    double* mm = C + ((size_t)i * ld + n + j) * E;
    a[0] = g[0] * sc;
    mm[0] = i == j ? 1.0 : 0.0;
    if (CPLX) {
      a[1] = g[E - 1] * sc;
      mm[1] = 0.0;
    }
  }
  const int cc = tid % n, ro = tid / n, rstep = nth / n;  // threads past rstep * n idle
  __syncthreads();
  auto at = [&](int i, int j) { return C + ((size_t)i * ld + j) * E; };
  for (int k = 0; k < n; ++k) {
    // breakdown: a pivot of the unit-diagonal (Jacobi-scaled) Gram matrix at or below
    // n * 2^-52, i.e. numerically rank deficient in float64 (every thread sees the same value)
    const double dk = at(k, k)[0];
    if (!(dk > n * 2.220446049250313e-16) || !isfinite(dk)) {
      if (tid == 0) bad = k;
      break;
    }
    if (ro < rstep) {
      const double rk = 1.0 / dk;
      const int j = k + 1 + cc;
      const double* sk = at(k, j);
      const Z src{sk[0], CPLX ? sk[E - 1] : 0.0};
      for (int i = k + 1 + ro; i < n; i += rstep) {
        const double* ci = at(i, k);
        const Z f{ci[0] * rk, CPLX ? ci[E - 1] * rk : 0.0};
        double* c0 = at(i, j);
        if constexpr (!CPLX) {
          c0[0] = fma(-f.r, src.r, c0[0]);
        } else {
          const Z pr = zmul(f, src);
          c0[0] -= pr.r;
          c0[1] -= pr.i;
        }
      }
    }
    __syncthreads();
  }
  if (bad >= 0) {
    if (tid == 0) {
      status[0] = OEFE_ENOTSPD;
      status[1] = bad;
      if (go) *go = 0;
    }
    return;
  }
  // Rinv = diag(d) L^-*, L^-1 = D^-1/2 L_1^-1: Rinv[i][j] = d_i conj(m_ji) / sqrt(c_jj), j >= i
  for (int t = tid; t < n * n; t += nth) {
    const int i = t / n, j = t - i * n;
    double vr = 0.0, vi = 0.0;
    if (j >= i) {
      const double sc = d[i] / sqrt(at(j, j)[0]);
      const double* mm = at(j, n + i);
      vr = sc * mm[0];
      if (CPLX) vi = -sc * mm[E - 1];
    }
    Rinv[(int64_t)t * E] = vr;
    if (CPLX) Rinv[(int64_t)t * E + 1] = vi;
  }
  if (tid == 0) {
    status[0] = 0;
    status[1] = -1;
    if (go) *go = 1;
  }
}

// ---- Cholesky of the Jacobi-scaled Gram matrix and triangular inverse in LDS (small n).
// Jacobi scaling of the Gram matrix, pivots, and breakdown when a pivot of the scaled
// (unit-diagonal) matrix is at or below n 2^-52; G is only read.
template <bool CPLX>
__global__ __launch_bounds__(512) void chol_lds_kernel(const double* __restrict__ G, int ldg, int n,
                                                       double* __restrict__ Rinv, double* __restrict__ dsc,
                                                       int32_t* __restrict__ status) {
  constexpr int E = CPLX ? 2 : 1;
  extern __shared__ double sm[];
  double* L = sm;                        // [n][n] lower factor (row-major)
  double* Li = L + (size_t)n * n * E;    // [n][n] its inverse (lower)
  double* d = Li + (size_t)n * n * E;    // [n] Jacobi scaling
  __shared__ int bad;
  const int tid = threadIdx.x, nth = blockDim.x;
  if (tid == 0) bad = -1;
  __syncthreads();
  for (int i = tid; i < n; i += nth) {
    const double gii = G[((int64_t)i * ldg + i) * E];
    if (!(gii > 0.0)) atomicMax(&bad, i);
    d[i] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
    dsc[i] = d[i];
  }
  __syncthreads();
  if (bad >= 0) {
    if (tid == 0) { status[0] = OEFE_ENOTSPD; status[1] = bad; }
    return;
  }
  for (int t = tid; t < n * n; t += nth) {
    const int i = t / n, j = t - i * n;
    const double sc = d[i] * d[j];
    L[(int64_t)t * E] = G[((int64_t)i * ldg + j) * E] * sc;
    if (CPLX) L[(int64_t)t * E + 1] = G[((int64_t)i * ldg + j) * E + 1] * sc;
    Li[(int64_t)t * E] = 0.0;
    if (CPLX) Li[(int64_t)t * E + 1] = 0.0;
  }
  __syncthreads();
  auto re = [&](int i, int j) -> double& { return L[((int64_t)i * n + j) * E]; };
  auto im = [&](int i, int j) -> double& { return L[((int64_t)i * n + j) * E + (E - 1)]; };
  for (int k = 0; k < n; ++k) {
    // breakdown: a pivot of the unit-diagonal (Jacobi-scaled) Gram matrix at or below
    // n * 2^-52, i.e. numerically rank deficient in float64 (every thread sees the same value)
    const double dk = re(k, k);
    if (!(dk > n * 2.220446049250313e-16) || !isfinite(dk)) {
      if (tid == 0) bad = k;
      break;
    }
    const double l = sqrt(dk);
    for (int i = k + 1 + tid; i < n; i += nth) {
      re(i, k) /= l;
      if (CPLX) im(i, k) /= l;
    }
    __syncthreads();
    const int m = n - k - 1;
    for (int t = tid; t < m * m; t += nth) {
      const int ii = t / m, jj = t - ii * m;
      if (jj > ii) continue;
      const int i = k + 1 + ii, j = k + 1 + jj;
      if constexpr (!CPLX) {
        re(i, j) -= re(i, k) * re(j, k);
      } else {
        const double ar = re(i, k), ai = im(i, k), br = re(j, k), bi = im(j, k);
        re(i, j) -= ar * br + ai * bi;
        im(i, j) -= ai * br - ar * bi;
      }
    }
    if (tid == 0) {
      re(k, k) = l;
      if (CPLX) im(k, k) = 0.0;
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad >= 0) {
    if (tid == 0) { status[0] = OEFE_ENOTSPD; status[1] = bad; }
    return;
  }
  // L^-1 row by row: Li[i][j] = -(sum_{k=j}^{i-1} L[i][k] Li[k][j]) / L[i][i], Li[i][i] = 1 / L[i][i];
  // 8 lanes per entry, partial sums combined by lane shuffles
  const int sub = tid & 7;
  for (int i = 0; i < n; ++i) {
    const double lii = re(i, i);
    for (int j0 = 0; j0 <= i; j0 += nth / 8) {
      const int j = j0 + (tid >> 3);
      double sr = 0.0, si = 0.0;
      if (j < i)
        for (int k = j + sub; k < i; k += 8) {
          const double lr = re(i, k), lm = CPLX ? im(i, k) : 0.0;
          const double yr = Li[((int64_t)k * n + j) * E], yi = CPLX ? Li[((int64_t)k * n + j) * E + 1] : 0.0;
          sr += lr * yr - lm * yi;
          si += lr * yi + lm * yr;
        }
      for (int o = 4; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o, 8);
        si += __shfl_xor(si, o, 8);
      }
      if (sub == 0 && j <= i) {
        Li[((int64_t)i * n + j) * E] = (j == i ? 1.0 : -sr) / lii;
        if (CPLX) Li[((int64_t)i * n + j) * E + 1] = (j == i ? 0.0 : -si) / lii;
      }
    }
    __syncthreads();
  }
  // Rinv = diag(d) Linv^*: Rinv[i][j] = d_i conj(Li[j][i]) (upper triangular)
  for (int t = tid; t < n * n; t += nth) {
    const int i = t / n, j = t - i * n;
    const double* y = Li + ((int64_t)j * n + i) * E;
    Rinv[(int64_t)t * E] = d[i] * y[0];
    if (CPLX) Rinv[(int64_t)t * E + 1] = -d[i] * y[1];
  }
  if (tid == 0) { status[0] = 0; status[1] = -1; }
}

template <bool CPLX>
__global__ void max_dev_identity_kernel(const double* __restrict__ G, int n, double* __restrict__ err,
                                        const int32_t* __restrict__ status, int32_t* __restrict__ repeat, double tol) {
  constexpr int E = CPLX ? 2 : 1;
  __shared__ double red[256];
  double mx = 0;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t % n;
    const double r = G[(int64_t)t * E] - (i == j ? 1.0 : 0.0);
    const double im = CPLX ? G[(int64_t)t * E + 1] : 0.0;
    mx = fmax(mx, sqrt(r * r + im * im));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *err = red[0];
    // repeat the factorization when the last one succeeded and left |Q^* Q - I| above tol
    if (repeat) *repeat = (status[0] == 0 && red[0] > tol) ? 1 : 0;
  }
}

template <bool CPLX>
__global__ void hermitian_part_kernel(double* __restrict__ G, int n, const int32_t* __restrict__ gate) {
  constexpr int E = CPLX ? 2 : 1;
  if (gate && *gate == 0) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int i = t / n, j = t % n;
  if (i > j) return;
  double* a = G + ((int64_t)i * n + j) * E;
  double* b = G + ((int64_t)j * n + i) * E;
  const double r = 0.5 * (a[0] + b[0]);
  a[0] = r;
  b[0] = r;
  if (CPLX) {
    const double im = 0.5 * (a[1] - b[1]);
    a[1] = (i == j) ? 0.0 : im;
    b[1] = (i == j) ? 0.0 : -im;
  }
}

__global__ void copy_block_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst, int64_t ldd,
                                  int64_t n, int ncols) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ncols) return;
  const int64_t r = t / ncols;
  const int c = (int)(t % ncols);
  dst[r * ldd + c] = src[r * lds + c];
}

// per-column partial dot products: part[chunk][j] = sum_g Re(conj(A[g][j]) B[g][j]) in float64
template <typename T, bool CPLX>
__global__ void dot_partial_kernel(const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
                                   int64_t n, int nv, int64_t rows_per_chunk, double* __restrict__ part) {
  constexpr int E = CPLX ? 2 : 1;
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= nv) return;
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t g1 = min(n, g0 + rows_per_chunk);
  double s = 0;
  for (int64_t g = g0; g < g1; ++g) {
    const T* a = A + (g * lda + j) * E;
    const T* b = B + (g * ldb + j) * E;
    s += (double)a[0] * (double)b[0] + (CPLX ? (double)a[E - 1] * (double)b[E - 1] : 0.0);
  }
  part[(int64_t)blockIdx.x * nv + j] = s;
}

// one column: workgroup b sums the rows of its contiguous chunk (thread-strided, then a fixed tree)
// One column's dot product over a chunk of rows: 1024 threads, each adding rows t, t + 2048, ...
// and t + 1024, t + 3072, ... into two sums (two loads in flight), then a fixed butterfly per
// wave and the 16 wave sums in order by one thread
template <typename T, bool CPLX>
__global__ __launch_bounds__(1024) void dot1_partial_kernel(const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                                            int64_t ldb, int64_t n, int64_t rows_per_chunk,
                                                            double* __restrict__ part) {
  constexpr int E = CPLX ? 2 : 1;
  __shared__ double red[16];
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_chunk, g1 = min(n, g0 + rows_per_chunk);
  auto term = [&](int64_t g) {
    const T* a = A + g * lda * E;
    const T* b = B + g * ldb * E;
    return (double)a[0] * (double)b[0] + (CPLX ? (double)a[E - 1] * (double)b[E - 1] : 0.0);
  };
  double s0 = 0, s1 = 0;
  int64_t g = g0 + threadIdx.x;
  for (; g + 1024 < g1; g += 2048) {
    s0 += term(g);
    s1 += term(g + 1024);
  }
  if (g < g1) s0 += term(g);
  double s = s0 + s1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// out = sum_j f_j sum_c part[c][j]: one thread per column, the chunks in order; a single column
// (the conjugate-gradient and Lanczos dots) spreads its chunks over the threads instead (thread t
// adds chunks t, t + 256, ... in order), both followed by the same fixed tree
__global__ void dot_final_kernel(const double* __restrict__ part, int nchunks, int nv, const double* __restrict__ f,
                                 double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0;
  if (nv == 1) {
    for (int c = threadIdx.x; c < nchunks; c += blockDim.x) s += part[c];
  } else {
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
      double cs = 0;
      for (int c = 0; c < nchunks; ++c) cs += part[(int64_t)c * nv + j];
      s += (f ? f[j] : 1.0) * cs;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = (int)blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = nv == 1 && f ? f[0] * red[0] : red[0];
}

template <typename S, typename D>
__global__ void cast_block_kernel(const S* __restrict__ src, int64_t lds, D* __restrict__ dst, int64_t ldd, int64_t n,
                                  int ncols) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ncols) return;
  const int64_t r = t / ncols;
  const int c = (int)(t % ncols);
  dst[r * ldd + c] = (D)src[r * lds + c];
}

template <typename T, bool CPLX>
__global__ void scale_grad_kernel(T* __restrict__ g, int64_t ld, int64_t n, int nv, const double* __restrict__ f) {
  constexpr int E = CPLX ? 2 : 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nv * E) return;
  const int64_t r = t / (nv * E);
  const int c = (int)(t % (nv * E));
  const int v = c / E;
  g[r * ld * E + c] = (T)(2.0 * f[v]) * g[r * ld * E + c];
}

// w -= alpha v + beta vprev  (v, vprev strided by ldv complex elements; w packed)
template <bool CPLX>
__global__ void lanczos_axpy_kernel(double* __restrict__ w, const double* __restrict__ v,
                                    const double* __restrict__ vprev, const double* __restrict__ alpha,
                                    const double* __restrict__ beta, int64_t n, int64_t ldv) {
  constexpr int E = CPLX ? 2 : 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * E) return;
  const int64_t r = t / E;
  const int e = (int)(t % E);
  double x = w[t] - alpha[0] * v[r * ldv * E + e];
  if (vprev) x -= beta[0] * vprev[r * ldv * E + e];
  w[t] = x;
}

template <bool CPLX>
__global__ void lanczos_scale_kernel(double* __restrict__ dst, int64_t ldd, const double* __restrict__ w,
                                     const double* __restrict__ beta, int64_t n) {
  constexpr int E = CPLX ? 2 : 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * E) return;
  const int64_t r = t / E;
  const int e = (int)(t % E);
  // w may be strided like dst when dst == w (in-place normalization of a strided column)
  dst[r * ldd * E + e] = w[(dst == w ? r * ldd * E : r * E) + e] / beta[0];
}

__global__ void sub_kernel(double* __restrict__ w, const double* __restrict__ t, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] -= t[i];
}

__global__ void sqrt_kernel(double* x) { x[0] = sqrt(x[0]); }

int check() { return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE; }

int gram_chunks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(128, cdiv(n, 512))); }

}  // namespace

static bool gram_on_mfma(bool cplx, int na, int nb) {
  return !cplx && na >= 16 && nb >= 16 && na <= 16 * kGramNBMax && nb <= 16 * kGramNBMax;
}
static int gram_mfma_chunks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kGramChunks, cdiv(n, 64))); }
// chunks of one launch: at most gram_mfma_chunks(n) (the scratch bound), and few enough that the
// chunks x row blocks workgroups fit the device's resident slots (four per CU) in one round, so
// no partial second round of full-length workgroups follows
static int gram_mfma_chunks_launch(int64_t n, int nbi) {
  static int slots[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (!slots[dev]) {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
    slots[dev] = 4 * ncu;
  }
  return std::max(1, std::min(gram_mfma_chunks(n), slots[dev] / std::max(1, nbi)));
}

// real blocks wider than one matrix-core Gram launch takes: tiled over column groups
static bool gram_mfma_tiled(bool cplx, int na, int nb) {
  return !cplx && na >= 16 && nb >= 16 && (na > 16 * kGramNBMax || nb > 16 * kGramNBMax);
}

// column groups of a tiled Gram and the chunks of its pairs launch: every workgroup of the launch
// resident in one round of 1024 slots (four per CU on 256 CUs); fixed, so that the summation order
// does not depend on the device
static int gram_pairs_chunks(int64_t n, int np, int gs) {
  return std::max(1, std::min(gram_mfma_chunks(n), 1024 / std::max(1, np * (int)cdiv(gs, 16))));
}
static bool gram_pairs(const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb, GramPairs& gp,
                       bool& sym) {
  const int gi = (int)cdiv(na, 16 * kGramNBMax), gj = (int)cdiv(nb, 16 * kGramNBMax);
  sym = A == B && lda == ldb && na == nb;
  gp.np = 0;
  gp.gs = 0;
  for (int I = 0; I < gi; ++I)
    for (int J = sym ? I : 0; J < gj; ++J) {
      if (gp.np == kGramPairsMax) return false;
      const int q = gp.np++;
      gp.i0[q] = (int)((int64_t)na * I / gi);
      gp.ni[q] = (int)((int64_t)na * (I + 1) / gi) - gp.i0[q];
      gp.j0[q] = (int)((int64_t)nb * J / gj);
      gp.nj[q] = (int)((int64_t)nb * (J + 1) / gj) - gp.j0[q];
      gp.gs = std::max(gp.gs, std::max(gp.ni[q], gp.nj[q]));
    }
  return true;
}

size_t gram_scratch_bytes(bool cplx, int na, int nb, int64_t n) {
  if (gram_mfma_tiled(cplx, na, nb)) {
    const int gi = (int)cdiv(na, 16 * kGramNBMax), gj = (int)cdiv(nb, 16 * kGramNBMax);
    const int bi = (int)cdiv(na, gi), bj = (int)cdiv(nb, gj), gs = std::max(bi, bj);
    size_t bytes = (size_t)gram_mfma_chunks(n) * bi * bj * sizeof(double);  // one pair per launch
    // one launch for all pairs (the symmetric case has fewer pairs, possibly more chunks)
    for (int np : {gi * gj, gi * (gi + 1) / 2})
      if (np <= kGramPairsMax) bytes = std::max(bytes, (size_t)np * gram_pairs_chunks(n, np, gs) * gs * gs * sizeof(double));
    return bytes;
  }
  const int nch = gram_on_mfma(cplx, na, nb) ? gram_mfma_chunks(n) : gram_chunks(n);
  return (size_t)nch * na * nb * (cplx ? 2 : 1) * sizeof(double);
}

static void launch_gram_mfma(const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb, int64_t n,
                             double* G, int ldg, double* scratch, hipStream_t s) {
  const int nbi = (int)cdiv(na, 16), nbj = (int)cdiv(nb, 16);
  const int nch = gram_mfma_chunks_launch(n, nbi);
  const int64_t rpc = cdiv(cdiv(n, nch), 4) * 4;
  // one row block per workgroup (up to four workgroups per CU), column blocks rounded up to {2, 3, 5}:
  // fragments past na / nb are zero
  const int bi = 1, bj = nbj <= 2 ? 2 : (nbj <= 3 ? 3 : 5);
  const dim3 g2((unsigned)nch, (unsigned)cdiv(nbi, bi));
  auto go2 = [&](auto kern) {
    const size_t lds = (size_t)bi * bj * 4 * 64 * sizeof(double);
    if (allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds) != hipSuccess) return;
    hipLaunchKernelGGL(kern, g2, dim3(256), lds, s, A, lda, na, B, ldb, nb, n, rpc, scratch);
  };
  if (bi == 1) { if (bj == 2) go2(gram_mfma_kernel<1, 2>); else if (bj == 3) go2(gram_mfma_kernel<1, 3>); else go2(gram_mfma_kernel<1, 5>); }
  else if (bi == 2) { if (bj == 2) go2(gram_mfma_kernel<2, 2>); else if (bj == 3) go2(gram_mfma_kernel<2, 3>); else go2(gram_mfma_kernel<2, 5>); }
  else { if (bj == 2) go2(gram_mfma_kernel<3, 2>); else if (bj == 3) go2(gram_mfma_kernel<3, 3>); else go2(gram_mfma_kernel<3, 5>); }
  hipLaunchKernelGGL((gram_reduce_wave_kernel<false>), dim3((unsigned)cdiv((int64_t)na * nb, 4)), dim3(256), 0, s,
                     scratch, nch, na, nb, G, ldg);
}

int gram(bool cplx, const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb, int64_t n, double* G,
         int ldg, double* scratch, size_t scratch_bytes, hipStream_t s) {
  if (gram_scratch_bytes(cplx, na, nb, n) > scratch_bytes) return OEFE_EINVAL;
  if (gram_on_mfma(cplx, na, nb)) {
    launch_gram_mfma(A, lda, na, B, ldb, nb, n, G, ldg, scratch, s);
    return check();
  }
  if (gram_mfma_tiled(cplx, na, nb)) {
    // wide real blocks: the matrix-core Gram on every pair of column groups of at most
    // 16 kGramNBMax columns (near-equal groups, each of at least 16 columns), all pairs in one
    // launch where the pair table holds them
    GramPairs gp;
    bool sym = false;
    if (gram_pairs(A, lda, na, B, ldb, nb, gp, sym)) {
      const int nch = gram_pairs_chunks(n, gp.np, gp.gs);
      const int64_t rpc = cdiv(cdiv(n, nch), 4) * 4;
      const int rbs = (int)cdiv(gp.gs, 16);
      const size_t lds = (size_t)kGramNBMax * 4 * 64 * sizeof(double);
      if (allow_dynamic_lds(reinterpret_cast<const void*>(&gram_mfma_pairs_kernel), lds) != hipSuccess) return OEFE_EDEVICE;
      hipLaunchKernelGGL(gram_mfma_pairs_kernel, dim3((unsigned)((int64_t)nch * gp.np * rbs)), dim3(256), lds, s, A, lda,
                         B, ldb, n, rpc, nch, gp, scratch);
      hipLaunchKernelGGL(gram_reduce_pairs_kernel, dim3((unsigned)cdiv((int64_t)gp.gs * gp.gs, 4), (unsigned)gp.np),
                         dim3(256), 0, s, scratch, nch, gp, G, ldg, sym ? 1 : 0);
      return check();
    }
    const int gi = (int)cdiv(na, 16 * kGramNBMax), gj = (int)cdiv(nb, 16 * kGramNBMax);
    for (int I = 0; I < gi; ++I) {
      const int i0 = (int)((int64_t)na * I / gi), i1 = (int)((int64_t)na * (I + 1) / gi);
      for (int J = 0; J < gj; ++J) {
        const int j0 = (int)((int64_t)nb * J / gj), j1 = (int)((int64_t)nb * (J + 1) / gj);
        launch_gram_mfma(A + i0, lda, i1 - i0, B + j0, ldb, j1 - j0, n, G + (size_t)i0 * ldg + j0, ldg, scratch, s);
      }
    }
    return check();
  }
  const int nch = gram_chunks(n);
  const int64_t rpc = cdiv(n, nch);
  dim3 grid(nch, (unsigned)cdiv(na, 16), (unsigned)cdiv(nb, 16));
  if (cplx) {
    hipLaunchKernelGGL(gram_partial_kernel<true>, grid, dim3(256), 0, s, A, lda, na, B, ldb, nb, n, rpc, scratch);
    hipLaunchKernelGGL(gram_reduce_kernel<true>, dim3((unsigned)cdiv((int64_t)na * nb, 256)), dim3(256), 0, s,
                       scratch, nch, na, nb, G, ldg);
  } else {
    hipLaunchKernelGGL(gram_partial_kernel<false>, grid, dim3(256), 0, s, A, lda, na, B, ldb, nb, n, rpc, scratch);
    hipLaunchKernelGGL(gram_reduce_kernel<false>, dim3((unsigned)cdiv((int64_t)na * nb, 256)), dim3(256), 0, s,
                       scratch, nch, na, nb, G, ldg);
  }
  return check();
}

int gemm_nn(bool cplx, const double* A, int64_t lda, const double* B, int ldb, double* C, int64_t ldc, int64_t n,
            int k, int m, hipStream_t s) {
  if (!cplx && k >= 16 && m >= 64 && n >= 4096) {  // real wide blocks: on the matrix cores
    const int nbj = m >= 80 ? 5 : cdiv(m, 16);
    const int ncb = cdiv(m, 16 * nbj);
    const dim3 g((unsigned)(cdiv(n, 128) * ncb));
    switch (nbj) {
      case 4: hipLaunchKernelGGL(gemm_nn_mfma_kernel<4>, g, dim3(256), 0, s, A, lda, B, ldb, C, ldc, n, k, m, ncb); break;
      default: hipLaunchKernelGGL(gemm_nn_mfma_kernel<5>, g, dim3(256), 0, s, A, lda, B, ldb, C, ldc, n, k, m, ncb); break;
    }
    return check();
  }
  dim3 grid((unsigned)cdiv(n, 64), (unsigned)cdiv(m, 64));
  if (cplx)
    hipLaunchKernelGGL(gemm_nn_kernel<true>, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, n, k, m);
  else
    hipLaunchKernelGGL(gemm_nn_kernel<false>, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, n, k, m);
  return check();
}

bool rowmul_on_mfma(bool cplx, int nv) { return !cplx && nv >= 1 && nv <= 80; }

bool cholgs_device_gated(bool cplx, int nv) { return rowmul_on_mfma(cplx, nv) && chol_elim_fits(cplx, nv); }

int rowmul_inplace(double* X, int64_t ldx, int64_t n, int nv, const double* R, hipStream_t s, const int32_t* gate) {
  if (n <= 0) return 0;
  const int nbj = cdiv(nv, 16), nks = cdiv(nv, 4);
  const size_t lds = (size_t)nks * 4 * (16 * nbj + 1) * sizeof(double);
  // persistent grid: as many workgroups as are resident at once
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  auto go = [&](auto kern) {
    if (allow_dynamic_lds(reinterpret_cast<const void*>(kern), lds) != hipSuccess) return;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    const dim3 grid((unsigned)std::min<int64_t>(cdiv(n, 64 * kRowMulRB), (int64_t)per_cu * cus));
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, X, ldx, n, nv, R, gate);
  };
  switch (nbj) {
    case 1: go(rowmul_mfma_kernel<1>); break;
    case 2: go(rowmul_mfma_kernel<2>); break;
    case 3: go(rowmul_mfma_kernel<3>); break;
    case 4: go(rowmul_mfma_kernel<4>); break;
    default: go(rowmul_mfma_kernel<5>); break;
  }
  return check();
}

// ---- Cholesky factor inverse for matrices above the LDS size: the elimination of [A | I]
// (A the Jacobi-scaled Gram matrix) with one launch per step.  Step k subtracts multiples of
// row k from the rows below: columns k+1 .. n-1 of the left part (kept in G) and columns
// 0 .. k of the right part (kept in Rinv, where the unit lower-triangular L_1^-1 builds up);
// column k itself is not rewritten, so every thread reads the multiplier A_ik and row k
// unchanged by the other threads of the launch.  The pivots D_k are A = L_1 D L_1^*'s, so
// L^-1 = D^-1/2 L_1^-1 and R^-1 = diag(d) L^-*.  Breakdown rule as in the other Cholesky
// kernels (a pivot of the unit-diagonal matrix at or below n 2^-52, or a non-positive
// diagonal before scaling); flag[0] holds the first failing index (INT32_MAX: none).
template <bool CPLX>
__global__ __launch_bounds__(256) void cholbig_scale_kernel(double* __restrict__ G, int ldg, int n,
                                                            double* __restrict__ Rinv, double* __restrict__ dsc,
                                                            int32_t* __restrict__ flag) {
  constexpr int E = CPLX ? 2 : 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t - (int64_t)i * n);
  const double gii = G[((int64_t)i * ldg + i) * E], gjj = G[((int64_t)j * ldg + j) * E];
  if (j == 0) {
    if (!(gii > 0.0)) atomicMin(flag, i);
    dsc[i] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
  }
  const double f = (gii > 0.0 && gjj > 0.0) ? 1.0 / (sqrt(gii) * sqrt(gjj)) : 0.0;
  double* g = G + ((int64_t)i * ldg + j) * E;
  g[0] = i == j ? (gii > 0.0 ? 1.0 : 0.0) : g[0] * f;
  if (CPLX) g[1] = i == j ? 0.0 : g[1] * f;
  double* r = Rinv + ((int64_t)i * n + j) * E;
  r[0] = i == j ? 1.0 : 0.0;
  if (CPLX) r[1] = 0.0;
}

template <bool CPLX>
__global__ __launch_bounds__(256) void cholbig_step_kernel(double* __restrict__ G, int ldg, int n,
                                                           double* __restrict__ Rinv, int k, int32_t* __restrict__ flag) {
  constexpr int E = CPLX ? 2 : 1;
  if (*flag != INT32_MAX) return;
  const double d = G[((int64_t)k * ldg + k) * E];
  if (!(d > n * 2.220446049250313e-16) || !isfinite(d)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) atomicMin(flag, k);
    return;
  }
  const int i = k + 1 + (int)blockIdx.y;  // row
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);  // 0 .. n-1: left columns k+1.., then right 0..k
  if (i >= n || c >= n) return;
  const double* gik = G + ((int64_t)i * ldg + k) * E;
  const double fr = gik[0] / d, fi = CPLX ? gik[1] / d : 0.0;  // multiplier A_ik / D_k
  double* dst;
  const double* src;
  if (c < n - 1 - k) {
    const int col = k + 1 + c;
    dst = G + ((int64_t)i * ldg + col) * E;
    src = G + ((int64_t)k * ldg + col) * E;
  } else {
    const int col = c - (n - 1 - k);  // 0 .. k
    dst = Rinv + ((int64_t)i * n + col) * E;
    src = Rinv + ((int64_t)k * n + col) * E;
  }
  if constexpr (!CPLX) {
    dst[0] -= fr * src[0];
  } else {
    dst[0] -= fr * src[0] - fi * src[1];
    dst[1] -= fr * src[1] + fi * src[0];
  }
}

// R^-1[i][j] = d_i conj(L^-1[j][i]) = d_i conj(L_1^-1[j][i]) / sqrt(D_j) (i <= j), 0 below
template <bool CPLX>
__global__ __launch_bounds__(256) void cholbig_final_kernel(const double* __restrict__ G, int ldg, int n,
                                                            double* __restrict__ Rinv, const double* __restrict__ dsc,
                                                            const int32_t* __restrict__ flag, int32_t* __restrict__ status) {
  constexpr int E = CPLX ? 2 : 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int bad = *flag;
  if (t == 0) {
    status[0] = bad != INT32_MAX ? OEFE_ENOTSPD : 0;
    status[1] = bad != INT32_MAX ? bad : -1;
  }
  if (bad != INT32_MAX || t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t - (int64_t)i * n);
  if (i > j) return;
  double* a = Rinv + ((int64_t)i * n + j) * E;
  double* b = Rinv + ((int64_t)j * n + i) * E;
  const double sj = 1.0 / sqrt(G[((int64_t)j * ldg + j) * E]);
  const double lr = b[0], li = CPLX ? b[1] : 0.0;  // L_1^-1[j][i]
  a[0] = dsc[i] * lr * sj;
  if (CPLX) a[1] = -dsc[i] * li * sj;
  if (i != j) {
    b[0] = 0.0;
    if (CPLX) b[1] = 0.0;
  }
}

__global__ void cholbig_init_kernel(int32_t* flag) { *flag = INT32_MAX; }

static int chol_big(bool cplx, double* G, int ldg, int n, double* Rinv, double* dsc, int32_t* status, hipStream_t s) {
  int32_t* flag = status + 2;  // the status block has room beyond {code, column}
  hipLaunchKernelGGL(cholbig_init_kernel, dim3(1), dim3(1), 0, s, flag);
  const unsigned g1 = (unsigned)cdiv((int64_t)n * n, 256);
  if (cplx)
    hipLaunchKernelGGL(cholbig_scale_kernel<true>, dim3(g1), dim3(256), 0, s, G, ldg, n, Rinv, dsc, flag);
  else
    hipLaunchKernelGGL(cholbig_scale_kernel<false>, dim3(g1), dim3(256), 0, s, G, ldg, n, Rinv, dsc, flag);
  for (int k = 0; k < n; ++k) {
    const dim3 g((unsigned)cdiv(n, 256), (unsigned)std::max(n - 1 - k, 1));
    if (cplx)
      hipLaunchKernelGGL(cholbig_step_kernel<true>, g, dim3(256), 0, s, G, ldg, n, Rinv, k, flag);
    else
      hipLaunchKernelGGL(cholbig_step_kernel<false>, g, dim3(256), 0, s, G, ldg, n, Rinv, k, flag);
  }
  if (cplx)
    hipLaunchKernelGGL(cholbig_final_kernel<true>, dim3(g1), dim3(256), 0, s, G, ldg, n, Rinv, dsc, flag, status);
  else
    hipLaunchKernelGGL(cholbig_final_kernel<false>, dim3(g1), dim3(256), 0, s, G, ldg, n, Rinv, dsc, flag, status);
  return check();
}

int chol_factor_inverse(bool cplx, double* G, int ldg, int n, double* Rinv, int32_t* status, hipStream_t s,
                        const int32_t* gate, int32_t* go) {
  if ((gate || go) && !chol_elim_fits(cplx, n)) return OEFE_EUNSUPPORTED;
  // dsc stored after Rinv (caller reserves n extra doubles)
  double* dsc = Rinv + (size_t)n * n * (cplx ? 2 : 1);
  if (chol_elim_fits(cplx, n)) {
    const size_t lds = chol_elim_lds_bytes(cplx, n);
    const void* fn = cplx ? (const void*)chol_elim_kernel<true> : (const void*)chol_elim_kernel<false>;
    if (allow_dynamic_lds(fn, lds) != hipSuccess) return OEFE_EDEVICE;
    if (cplx)
      hipLaunchKernelGGL(chol_elim_kernel<true>, dim3(1), dim3(1024), lds, s, G, ldg, n, Rinv, dsc, status, gate, go);
    else
      hipLaunchKernelGGL(chol_elim_kernel<false>, dim3(1), dim3(1024), lds, s, G, ldg, n, Rinv, dsc, status, gate, go);
    return check();
  }
  const size_t lds = ((size_t)2 * n * n * (cplx ? 2 : 1) + n) * sizeof(double);
  if (lds <= 150 * 1024) {
    const void* fn = cplx ? (const void*)chol_lds_kernel<true> : (const void*)chol_lds_kernel<false>;
    if (allow_dynamic_lds(fn, lds) != hipSuccess) return OEFE_EDEVICE;
    if (cplx)
      hipLaunchKernelGGL(chol_lds_kernel<true>, dim3(1), dim3(512), lds, s, G, ldg, n, Rinv, dsc, status);
    else
      hipLaunchKernelGGL(chol_lds_kernel<false>, dim3(1), dim3(512), lds, s, G, ldg, n, Rinv, dsc, status);
    return check();
  }
  return chol_big(cplx, G, ldg, n, Rinv, dsc, status, s);
}

// LDS version: the rotation record (kJacobiRecSweeps sweeps of m rounds x n/2 pairs x 4
// doubles) and the ranks (+ the recorded sweep count); global version: V and the rotations.
// ---- The same cyclic Jacobi for matrices above the LDS size, one launch per round.
// The matrix and the eigenvector matrix live in global memory, each double buffered, in the
// ring-position storage of the LDS kernels (position j holds index jacobi_ring_index(j) at a
// sweep's start; pair k of every round sits at positions 2k, 2k + 1).  A round launch reads
// the current buffers and writes the next ones: every thread of the matrix part takes one
// 2x2 block (k1 <= k2), forms the rotations of its two pairs itself from the current pivot
// entries (the same branch-free formula as the LDS kernels), and writes G_k1^* B G_k2 (and
// its mirror) to the positions of the next round; every thread of the vector part rotates
// the entries (2k, 2k + 1) of one row of V and moves them along the ring.  A control block
// carries the sweep state: a norm kernel at every sweep start sets the rotation threshold,
// and declares convergence when the off-diagonal part fell to rounding or the previous sweep
// rotated nothing; later launches then return at once.
struct JacobiCtl {
  double nrm_n;     // Frobenius norm / n at the current sweep's start
  int32_t done;     // no more rounds
  int32_t conv;     // converged (else the sweep limit ended it)
  int32_t buf;      // buffer that holds the matrix and V when done was set
  int32_t sweeps;   // sweeps started
  int32_t anyrot;   // a pair was rotated in the current sweep
  int32_t pad;
};

template <bool CPLX>
__global__ __launch_bounds__(256) void jbig_init_kernel(const double* __restrict__ A, int n, double* __restrict__ A0,
                                                        double* __restrict__ V0, JacobiCtl* __restrict__ ctl) {
  constexpr int E = CPLX ? 2 : 1;
  const int NN = (n % 2) ? n + 1 : n, m = NN - 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ctl->nrm_n = 0.0;
    ctl->done = 0;
    ctl->conv = 0;
    ctl->buf = 0;
    ctl->sweeps = 0;
    ctl->anyrot = 1;
  }
  if (t < (int64_t)NN * NN) {
    const int pi = (int)(t / NN), pj = (int)(t - (int64_t)pi * NN);
    const int i = jacobi_ring_index(pi, m), j = jacobi_ring_index(pj, m);
    double vr = 0.0, vi = 0.0;
    if (i < n && j < n) {
      const double* a = A + ((size_t)min(i, j) * n + max(i, j)) * E;
      vr = a[0];
      if (CPLX) vi = i == j ? 0.0 : (i < j ? a[E - 1] : -a[E - 1]);
    }
    A0[t * E] = vr;
    if (CPLX) A0[t * E + 1] = vi;
  }
  if (t < (int64_t)n * NN) {  // V = I by ring position: V[r][pos] = (index at pos == r)
    const int r = (int)(t / NN), pj = (int)(t - (int64_t)r * NN);
    V0[t * E] = jacobi_ring_index(pj, m) == r ? 1.0 : 0.0;
    if (CPLX) V0[t * E + 1] = 0.0;
  }
}

// sweep start: convergence test and the rotation threshold; one workgroup
template <bool CPLX>
__global__ __launch_bounds__(1024) void jbig_norm_kernel(const double* __restrict__ A0, const double* __restrict__ A1,
                                                         int n, int cur, int max_sweeps, JacobiCtl* __restrict__ ctl) {
  constexpr int E = CPLX ? 2 : 1;
  __shared__ double red[32];
  if (ctl->done) return;
  const int NN = (n % 2) ? n + 1 : n;
  const double* Ac = cur ? A1 : A0;
  const int tid = threadIdx.x;
  double off = 0, dia = 0;
  for (int t = tid; t < NN * NN; t += blockDim.x) {
    const int i = t / NN, j = t - i * NN;
    const double* a = Ac + (size_t)t * E;
    const double v = a[0] * a[0] + (CPLX ? a[1] * a[1] : 0.0);
    if (i == j) dia += v;
    else off += v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    off += __shfl_xor(off, o);
    dia += __shfl_xor(dia, o);
  }
  if ((tid & 63) == 0) {
    red[2 * (tid >> 6)] = off;
    red[2 * (tid >> 6) + 1] = dia;
  }
  __syncthreads();
  if (tid != 0) return;
  double offs = 0, dias = 0;
  for (int w = 0; w < (int)blockDim.x / 64; ++w) {
    offs += red[2 * w];
    dias += red[2 * w + 1];
  }
  // a sweep that found no pair coupled above rounding, or an off-diagonal part at rounding:
  // converged; the sweep limit: stopped
  const bool conv = (ctl->sweeps > 0 && ctl->anyrot == 0) || offs <= 1e-30 * dias || offs == 0.0;
  if (conv || ctl->sweeps >= max_sweeps) {
    ctl->done = 1;
    ctl->conv = conv ? 1 : 0;
    ctl->buf = cur;
    return;
  }
  ctl->nrm_n = sqrt(offs + dias) / n;
  ctl->anyrot = 0;
  ctl->sweeps += 1;
}

// The 2 x 2 diagonal block of pair k (entries 2k and 2k+1 of the current matrix)
template <bool CPLX>
struct PairBlock {
  double a00, a11;
  Z b;
};
template <bool CPLX>
__device__ __forceinline__ PairBlock<CPLX> jbig_pair_load(const double* __restrict__ Ac, int NN, int k) {
  constexpr int E = CPLX ? 2 : 1;
  const int p0 = 2 * k, p1 = 2 * k + 1;
  return {Ac[((size_t)p0 * NN + p0) * E], Ac[((size_t)p1 * NN + p1) * E], jz_load<CPLX>(Ac + ((size_t)p0 * NN + p1) * E)};
}

// The rotation of pair k at round st from its diagonal block
template <bool CPLX>
__device__ __forceinline__ void jbig_table(const PairBlock<CPLX>& pb, int m, int st, int k, double nrm_n, Z* g,
                                           bool& on) {
  // position 2k holds the larger index q of the pair at this round (as in the LDS kernels)
  const int sa = (k + st) % m, sb = (m - k + st) % m;
  const bool sw = k >= 1 && sa > sb;
  const JacobiRot R = jacobi_rotation<CPLX>(sw ? pb.a11 : pb.a00, sw ? pb.a00 : pb.a11, pb.b.r, sw ? -pb.b.i : pb.b.i, nrm_n);
  const Z g00{R.c, 0.0}, g01{R.s, 0.0}, g10{-R.s * R.er, R.s * R.ei}, g11{R.c * R.er, -R.c * R.ei};
  g[0] = sw ? g11 : g00;
  g[1] = sw ? g10 : g01;
  g[2] = sw ? g01 : g10;
  g[3] = sw ? g00 : g11;
  on = R.on;
}

// One round: every 2 x 2 block (k1, k2) of the matrix (one thread each, k1 <= k2, from a
// square index range of npair^2 threads of which those with k2 < k1 do nothing) and every
// (row, pair) of V.  Each thread issues all its loads (the sweep state, the diagonal blocks
// of its pairs, its own block or V entries) before any arithmetic: the round is a chain of
// memory latencies, not of work.
template <bool CPLX>
__global__ __launch_bounds__(256) void jbig_round_kernel(const double* __restrict__ Ac, double* __restrict__ An,
                                                         const double* __restrict__ Vc, double* __restrict__ Vn,
                                                         int n, int st, JacobiCtl* __restrict__ ctl) {
  constexpr int E = CPLX ? 2 : 1;
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, m = NN - 1;
  const int nsq = npair * npair;
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t < nsq) {
    const int k1 = t / npair, k2 = t - k1 * npair;
    if (k2 < k1) return;
    const PairBlock<CPLX> p1 = jbig_pair_load<CPLX>(Ac, NN, k1), p2 = jbig_pair_load<CPLX>(Ac, NN, k2);
    Z bl[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      bl[e] = jz_load<CPLX>(Ac + ((size_t)(2 * k1 + (e >> 1)) * NN + 2 * k2 + (e & 1)) * E);
    const double nrm_n = ctl->nrm_n;
    if (ctl->done) return;
    Z u[4], v[4], d[4];
    bool on1, on2;
    jbig_table<CPLX>(p1, m, st, k1, nrm_n, u, on1);
    jbig_table<CPLX>(p2, m, st, k2, nrm_n, v, on2);
#pragma unroll
    for (int e = 0; e < 4; ++e) d[e] = jz_entry<CPLX>(u, bl, v, e >> 1, e & 1);
    if (k1 == k2) {
      if (on1) {  // the rotated pair; its diagonal stays real
        d[1] = d[2] = Z{0.0, 0.0};
        d[0].i = 0.0;
        d[3].i = 0.0;
        ctl->anyrot = 1;  // benign race: every writer stores 1
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = jacobi_ring_next(2 * k1 + (e >> 1), npair), q = jacobi_ring_next(2 * k2 + (e & 1), npair);
      jz_store<CPLX>(An + ((size_t)r * NN + q) * E, d[e]);
      if (k1 != k2) jz_store<CPLX>(An + ((size_t)q * NN + r) * E, jz_conj(d[e]));
    }
    return;
  }
  const int tv = t - nsq;
  if (tv >= n * npair) return;
  // row r of V, pair k: (v_2k, v_2k+1) <- (v_2k, v_2k+1) G_k, moved along the ring
  const int r = tv / npair, k = tv - r * npair;
  const PairBlock<CPLX> pk = jbig_pair_load<CPLX>(Ac, NN, k);
  const double* vr = Vc + (size_t)r * NN * E;
  const Z v0 = jz_load<CPLX>(vr + (size_t)(2 * k) * E), v1 = jz_load<CPLX>(vr + (size_t)(2 * k + 1) * E);
  const double nrm_n = ctl->nrm_n;
  if (ctl->done) return;
  Z g[4];
  bool on;
  jbig_table<CPLX>(pk, m, st, k, nrm_n, g, on);
  const Z w0 = jz_fma<CPLX>(v1, g[2], jz_mul<CPLX>(v0, g[0]));
  const Z w1 = jz_fma<CPLX>(v1, g[3], jz_mul<CPLX>(v0, g[1]));
  double* vn = Vn + (size_t)r * NN * E;
  jz_store<CPLX>(vn + (size_t)jacobi_ring_next(2 * k, npair) * E, w0);
  jz_store<CPLX>(vn + (size_t)jacobi_ring_next(2 * k + 1, npair) * E, w1);
}

// eigenvalues (ascending), U[r][rank(i)] = V[r][pos(i)], status; one workgroup
template <bool CPLX>
__global__ __launch_bounds__(1024) void jbig_final_kernel(const double* __restrict__ A0, const double* __restrict__ A1,
                                                          const double* __restrict__ V0, const double* __restrict__ V1,
                                                          int n, double* __restrict__ lam, double* __restrict__ U,
                                                          int32_t* __restrict__ rankbuf, const JacobiCtl* __restrict__ ctl,
                                                          int32_t* __restrict__ status) {
  constexpr int E = CPLX ? 2 : 1;
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, m = NN - 1;
  const int buf = ctl->buf;
  const double* Af = buf ? A1 : A0;
  const double* Vf = buf ? V1 : V0;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += blockDim.x) {
    const int q = jacobi_ring_pos(i, npair, m);
    const double li = Af[((size_t)q * NN + q) * E];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const int qj = jacobi_ring_pos(j, npair, m);
      const double lj = Af[((size_t)qj * NN + qj) * E];
      if (lj < li || (lj == li && j < i)) ++rank;
    }
    lam[rank] = li;
    rankbuf[i] = rank;
  }
  __syncthreads();
  for (int t = tid; t < n * n; t += blockDim.x) {
    const int r = t / n, i = t - r * n;
    const int q = jacobi_ring_pos(i, npair, m);
    const double* src = Vf + ((size_t)r * NN + q) * E;
    double* dst = U + ((size_t)r * n + rankbuf[i]) * E;
    dst[0] = src[0];
    if (CPLX) dst[1] = src[1];
  }
  if (tid == 0) {
    status[0] = ctl->conv ? 0 : OEFE_ENOCONV;
    status[1] = ctl->sweeps;
  }
}

size_t jbig_scratch_bytes(bool cplx, int n) {
  const int NN = (n % 2) ? n + 1 : n, E = cplx ? 2 : 1;
  const size_t a = (size_t)NN * NN * E * sizeof(double), v = (size_t)n * NN * E * sizeof(double);
  return 2 * ((a + 255) / 256 * 256) + 2 * ((v + 255) / 256 * 256) + 256 + ((size_t)n * sizeof(int32_t) + 255) / 256 * 256;
}

int jbig_eig(bool cplx, double* A, int n, double* lam, double* U, double* scratch, int32_t* status, hipStream_t s,
             int max_sweeps) {
  const int NN = (n % 2) ? n + 1 : n, npair = NN / 2, m = NN - 1, E = cplx ? 2 : 1;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  char* p = (char*)scratch;
  double* Ab[2];
  double* Vb[2];
  Ab[0] = (double*)p; p += al((size_t)NN * NN * E * sizeof(double));
  Ab[1] = (double*)p; p += al((size_t)NN * NN * E * sizeof(double));
  Vb[0] = (double*)p; p += al((size_t)n * NN * E * sizeof(double));
  Vb[1] = (double*)p; p += al((size_t)n * NN * E * sizeof(double));
  JacobiCtl* ctl = (JacobiCtl*)p; p += 256;
  int32_t* rankbuf = (int32_t*)p;
  const int64_t ninit = std::max<int64_t>((int64_t)NN * NN, (int64_t)n * NN);
  if (cplx)
    hipLaunchKernelGGL(jbig_init_kernel<true>, dim3((unsigned)cdiv(ninit, 256)), dim3(256), 0, s, A, n, Ab[0], Vb[0], ctl);
  else
    hipLaunchKernelGGL(jbig_init_kernel<false>, dim3((unsigned)cdiv(ninit, 256)), dim3(256), 0, s, A, n, Ab[0], Vb[0], ctl);
  const unsigned grid = (unsigned)cdiv((int64_t)npair * npair + (int64_t)n * npair, 256);
  // a pinned host word per host thread for the convergence flag (allocated once, kept)
  static thread_local int32_t* done_h = nullptr;
  if (!done_h && hipHostMalloc((void**)&done_h, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) done_h = nullptr;
  int cur = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (cplx)
      hipLaunchKernelGGL(jbig_norm_kernel<true>, dim3(1), dim3(1024), 0, s, Ab[0], Ab[1], n, cur, max_sweeps, ctl);
    else
      hipLaunchKernelGGL(jbig_norm_kernel<false>, dim3(1), dim3(1024), 0, s, Ab[0], Ab[1], n, cur, max_sweeps, ctl);
    // after the first sweeps, look whether the sweep start found convergence before queueing
    // its rounds (later launches would return at once, but each costs a launch)
    if (sw >= 2 && done_h) {
      if (hipMemcpyAsync(done_h, &ctl->done, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        break;
      if (*done_h) break;
    }
    for (int st = 0; st < m; ++st) {
      if (cplx)
        hipLaunchKernelGGL(jbig_round_kernel<true>, dim3(grid), dim3(256), 0, s, Ab[cur], Ab[cur ^ 1], Vb[cur],
                           Vb[cur ^ 1], n, st, ctl);
      else
        hipLaunchKernelGGL(jbig_round_kernel<false>, dim3(grid), dim3(256), 0, s, Ab[cur], Ab[cur ^ 1], Vb[cur],
                           Vb[cur ^ 1], n, st, ctl);
      cur ^= 1;
    }
  }
  // the state after the last sweep (the limit, or a convergence not yet declared)
  if (cplx)
    hipLaunchKernelGGL(jbig_norm_kernel<true>, dim3(1), dim3(1024), 0, s, Ab[0], Ab[1], n, cur, 0, ctl);
  else
    hipLaunchKernelGGL(jbig_norm_kernel<false>, dim3(1), dim3(1024), 0, s, Ab[0], Ab[1], n, cur, 0, ctl);
  if (cplx)
    hipLaunchKernelGGL(jbig_final_kernel<true>, dim3(1), dim3(1024), 0, s, Ab[0], Ab[1], Vb[0], Vb[1], n, lam, U,
                       rankbuf, ctl, status);
  else
    hipLaunchKernelGGL(jbig_final_kernel<false>, dim3(1), dim3(1024), 0, s, Ab[0], Ab[1], Vb[0], Vb[1], n, lam, U,
                       rankbuf, ctl, status);
  return check();
}

static bool jacobi_in_lds(bool cplx, int n) {
  const int npair = (n + 1) / 2;
  return jacobi_rot_lds_bytes(cplx, n) <= 158 * 1024 && npair * (npair + 1) / 2 <= 3 * 1024;  // 160 KB of LDS per workgroup
}

size_t jacobi_scratch_bytes(bool cplx, int n) {
  const int NN = (n % 2) ? n + 1 : n;
  if (!jacobi_in_lds(cplx, n)) return jbig_scratch_bytes(cplx, n);
  const size_t recb = (size_t)kJacobiRecSweeps * (NN - 1) * (NN / 2) * 4 * sizeof(double) +
                      ((size_t)n + 1) * sizeof(int32_t) + 256;
  return recb;
}

int jacobi_eig(bool cplx, double* A, int n, double* lam, double* U, double* scratch, int32_t* status, hipStream_t s,
               int max_sweeps) {
  if (jacobi_in_lds(cplx, n)) {
    const int NN = (n % 2) ? n + 1 : n;
    double* rec = scratch;
    int32_t* rank = reinterpret_cast<int32_t*>(rec + (size_t)kJacobiRecSweeps * (NN - 1) * (NN / 2) * 4);
    const size_t lds2 = jacobi_vec_lds_bytes(cplx, n);
    // one barrier per round where the double-buffered matrix fits, else blocks of the upper
    // triangle per thread of the two-barrier kernel
    const int npair = NN / 2, kb = cdiv(npair * (npair + 1) / 2, 1024);
    using RotFn = void (*)(const double*, int, double*, int32_t*, double*, int32_t*, int);
    const bool one = jacobi_ring1_fits(n) && jacobi_ring1_lds_bytes(cplx, n) <= 158 * 1024;
    size_t lds = one ? jacobi_ring1_lds_bytes(cplx, n) : jacobi_rot_lds_bytes(cplx, n);
    RotFn rot = one ? (cplx ? jacobi_ring1_kernel<true> : jacobi_ring1_kernel<false>)
              : cplx ? (kb == 1 ? jacobi_rot_kernel<true, 1> : kb == 2 ? jacobi_rot_kernel<true, 2> : jacobi_rot_kernel<true, 3>)
                     : (kb == 1 ? jacobi_rot_kernel<false, 1> : kb == 2 ? jacobi_rot_kernel<false, 2> : jacobi_rot_kernel<false, 3>);
    const void* fn2 = cplx ? (const void*)jacobi_vec_kernel<true> : (const void*)jacobi_vec_kernel<false>;
    if (allow_dynamic_lds((const void*)rot, lds) != hipSuccess || allow_dynamic_lds(fn2, lds2) != hipSuccess)
      return OEFE_EDEVICE;
    const dim3 g2((unsigned)cdiv(n, 4));
    hipLaunchKernelGGL(rot, dim3(1), dim3(1024), lds, s, A, n, lam, rank, rec, status,
                       max_sweeps > 0 ? max_sweeps : kJacobiRecSweeps);
    if (npair <= 64) {  // eigenvectors in registers, moved along the ring by lane shifts
      const dim3 g3((unsigned)cdiv(n, kJacobiVecRows));
      if (cplx)
        hipLaunchKernelGGL(jacobi_vec_ring_kernel<true>, g3, dim3(64), 0, s, rec, rank, n, U);
      else
        hipLaunchKernelGGL(jacobi_vec_ring_kernel<false>, g3, dim3(64), 0, s, rec, rank, n, U);
    } else if (cplx) {
      hipLaunchKernelGGL(jacobi_vec_kernel<true>, g2, dim3(256), lds2, s, rec, rank, n, U);
    } else {
      hipLaunchKernelGGL(jacobi_vec_kernel<false>, g2, dim3(256), lds2, s, rec, rank, n, U);
    }
    return check();
  }
  return jbig_eig(cplx, A, n, lam, U, scratch, status, s, max_sweeps > 0 ? max_sweeps : kJacobiGlobalSweeps);
}

int max_offdiag_identity(bool cplx, const double* G, int n, double* err, hipStream_t s, const int32_t* status,
                         int32_t* repeat, double tol) {
  if (cplx)
    hipLaunchKernelGGL(max_dev_identity_kernel<true>, dim3(1), dim3(256), 0, s, G, n, err, status, repeat, tol);
  else
    hipLaunchKernelGGL(max_dev_identity_kernel<false>, dim3(1), dim3(256), 0, s, G, n, err, status, repeat, tol);
  return check();
}

int hermitian_part(bool cplx, double* G, int n, hipStream_t s, const int32_t* gate) {
  dim3 grid((unsigned)cdiv((int64_t)n * n, 256));
  if (cplx)
    hipLaunchKernelGGL(hermitian_part_kernel<true>, grid, dim3(256), 0, s, G, n, gate);
  else
    hipLaunchKernelGGL(hermitian_part_kernel<false>, grid, dim3(256), 0, s, G, n, gate);
  return check();
}

int copy_block(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n_rows, int ncols, hipStream_t s) {
  hipLaunchKernelGGL(copy_block_kernel, dim3((unsigned)cdiv(n_rows * ncols, 256)), dim3(256), 0, s, src, lds, dst,
                     ldd, n_rows, ncols);
  return check();
}

template <typename T>
int dot_columns(bool cplx, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n, int nv, const double* f,
                double* out, double* scratch, hipStream_t s) {
  if (nv == 1) {
    // a single column: 1024 threads per chunk (the per-column kernel would use one lane of 64)
    const int nch = gram_chunks(n);
    const int64_t rpc = cdiv(n, nch);
    if (cplx)
      hipLaunchKernelGGL((dot1_partial_kernel<T, true>), dim3(nch), dim3(1024), 0, s, A, lda, B, ldb, n, rpc, scratch);
    else
      hipLaunchKernelGGL((dot1_partial_kernel<T, false>), dim3(nch), dim3(1024), 0, s, A, lda, B, ldb, n, rpc, scratch);
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, scratch, nch, 1, f, out);
    return check();
  }
  const int nch = gram_chunks(n);
  const int64_t rpc = cdiv(n, nch);
  dim3 grid(nch, (unsigned)cdiv(nv, 64));
  if (cplx)
    hipLaunchKernelGGL((dot_partial_kernel<T, true>), grid, dim3(64), 0, s, A, lda, B, ldb, n, nv, rpc, scratch);
  else
    hipLaunchKernelGGL((dot_partial_kernel<T, false>), grid, dim3(64), 0, s, A, lda, B, ldb, n, nv, rpc, scratch);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, scratch, nch, nv, f, out);
  return check();
}
int dot1_chunk_count(int64_t n) { return gram_chunks(n); }

int dot1_final(const double* part, int nch, double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, part, nch, 1, nullptr, out);
  return check();
}

template int dot_columns<double>(bool, const double*, int64_t, const double*, int64_t, int64_t, int, const double*,
                                 double*, double*, hipStream_t);
template int dot_columns<float>(bool, const float*, int64_t, const float*, int64_t, int64_t, int, const double*,
                                double*, double*, hipStream_t);

int cast_block(const void* src, bool src_f32, void* dst, bool dst_f32, int64_t n_rows, int64_t lds, int64_t ldd,
               int ncols, hipStream_t s) {
  dim3 grid((unsigned)cdiv(n_rows * ncols, 256));
  if (src_f32 && dst_f32)
    hipLaunchKernelGGL((cast_block_kernel<float, float>), grid, dim3(256), 0, s, (const float*)src, lds, (float*)dst, ldd, n_rows, ncols);
  else if (src_f32)
    hipLaunchKernelGGL((cast_block_kernel<float, double>), grid, dim3(256), 0, s, (const float*)src, lds, (double*)dst, ldd, n_rows, ncols);
  else if (dst_f32)
    hipLaunchKernelGGL((cast_block_kernel<double, float>), grid, dim3(256), 0, s, (const double*)src, lds, (float*)dst, ldd, n_rows, ncols);
  else
    hipLaunchKernelGGL((cast_block_kernel<double, double>), grid, dim3(256), 0, s, (const double*)src, lds, (double*)dst, ldd, n_rows, ncols);
  return check();
}

int scale_grad(bool cplx, void* g, int64_t ld, int64_t n, int nv, const double* f, bool f32, hipStream_t s) {
  dim3 grid((unsigned)cdiv(n * nv * (cplx ? 2 : 1), 256));
  if (f32) {
    if (cplx) hipLaunchKernelGGL((scale_grad_kernel<float, true>), grid, dim3(256), 0, s, (float*)g, ld, n, nv, f);
    else hipLaunchKernelGGL((scale_grad_kernel<float, false>), grid, dim3(256), 0, s, (float*)g, ld, n, nv, f);
  } else {
    if (cplx) hipLaunchKernelGGL((scale_grad_kernel<double, true>), grid, dim3(256), 0, s, (double*)g, ld, n, nv, f);
    else hipLaunchKernelGGL((scale_grad_kernel<double, false>), grid, dim3(256), 0, s, (double*)g, ld, n, nv, f);
  }
  return check();
}

int lanczos_axpy(bool cplx, double* w, const double* v, const double* vprev, const double* alpha,
                 const double* beta, int64_t n, int64_t ldv, hipStream_t s) {
  dim3 grid((unsigned)cdiv(n * (cplx ? 2 : 1), 256));
  if (cplx) hipLaunchKernelGGL(lanczos_axpy_kernel<true>, grid, dim3(256), 0, s, w, v, vprev, alpha, beta, n, ldv);
  else hipLaunchKernelGGL(lanczos_axpy_kernel<false>, grid, dim3(256), 0, s, w, v, vprev, alpha, beta, n, ldv);
  return check();
}

int lanczos_scale(bool cplx, double* dst, int64_t ldd, const double* w, const double* beta, int64_t n,
                  hipStream_t s) {
  dim3 grid((unsigned)cdiv(n * (cplx ? 2 : 1), 256));
  if (cplx) hipLaunchKernelGGL(lanczos_scale_kernel<true>, grid, dim3(256), 0, s, dst, ldd, w, beta, n);
  else hipLaunchKernelGGL(lanczos_scale_kernel<false>, grid, dim3(256), 0, s, dst, ldd, w, beta, n);
  return check();
}

int sub_block(bool cplx, double* w, const double* t, int64_t n, hipStream_t s) {
  const int64_t m = n * (cplx ? 2 : 1);
  hipLaunchKernelGGL(sub_kernel, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, s, w, t, m);
  return check();
}

int sqrt_inplace(double* x, hipStream_t s) {
  hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(1), 0, s, x);
  return check();
}

}  // namespace oefe
