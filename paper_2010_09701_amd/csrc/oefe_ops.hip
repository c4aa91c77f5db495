// HIP kernels of the OEFE operator application Ht X = M^-1/2 H M^-1/2 X and the
// scaled Chebyshev recurrence step built on it (gfx950, wave64).
//
// One operator step (out = alpha (Ht x - c x) - beta prev) is:
//   1. zo       Z^O = S X^O                                   (small dense)
//   2. cell     per cell: z_e = m^-1/2 (theta o X)|_e, y_e = K_e z_e + B^T diag(W V) B z_e
//               (sum-factorized, see fe_cell_kernel) -> per-cell buffer
//   3. partial  per 64-row tile: conj(m^-1/2 H^co)^T X over the tile's rows
//   4. node     per FE node: fixed-order sum of the (up to 8) cell results sharing it
//               (no atomics), times m^-1/2, + (m^-1/2 H^co) Z^O, recurrence epilogue
//   5. reduce   W' = sum of the tile partials of each function (fixed order)
//   6. gemm     W' += H^oo Z^O ;  enrichment rows alpha (S W' - c x) - beta prev
// Every launch can cover several operators of one mesh at once (k-points): the
// per-operator arguments travel in a KBatch and blockIdx.z selects the operator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "oefe_kernels.h"

namespace oefe {

namespace {

template <typename T>
struct C2 {
  T r, i;
};
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__device__ __forceinline__ C2<T> cjmul(C2<T> a, C2<T> b) {  // conj(a) * b
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}

template <typename T>
struct Phase3 {
  T re[3], im[3];
};

constexpr int KMAX = 8;  // operators per batched launch

// Per-operator arguments of one recurrence step (leading dimensions in elements of T).
template <typename T>
struct KP {
  const T* x;
  const T* prev;
  T* out;
  int64_t ldx, ldo;
  int nv, ncr;  // vectors (complex elements when complex) and real columns
  T* ycell;
  int ldc;
  T* zo;
  T* part;
  T* part2;
  int nch;  // chunks per function in part2
  T* wp;
  const T* wv;  // W (V + the form's constant shift) of this operator at its quadrature points
  const T* tv;
  const T* S;
  const T* Hoo;
  T alpha, c, beta;
  const double* sc;  // device (alpha, c, beta) of the step in place of the three above, or null
  Phase3<T> ph;
  T uk[3];  // periodic-function k-point form: (h/2)^3 (2/h) k_d (zero otherwise)
};

// the step's scalars: from device memory when the filter's bounds live on the device
template <typename T>
__device__ __forceinline__ void step_scalars(const KP<T>& P, T& alpha, T& c, T& beta) {
  if (P.sc) {
    alpha = (T)P.sc[0];
    c = (T)P.sc[1];
    beta = (T)P.sc[2];
  } else {
    alpha = P.alpha;
    c = P.c;
    beta = P.beta;
  }
}

template <typename T>
struct KBatch {
  int nk;
  KP<T> k[KMAX];
};


// ---------------------------------------------------------------------------
// 1D passes of the sum-factorized cell operator, shared by the cell kernels so that every
// launch shape does the same arithmetic.  EO (degree 4): each 5-point contraction through
// the even and odd halves of its matrix (EO5); otherwise plain sums in index order.
// ---------------------------------------------------------------------------
// out(q, (M v)_q) for q < 5 from in(a) = v_a, M given by its halves
template <typename T, typename In, typename Out>
__device__ __forceinline__ void eo5_apply(const EO5<T>& m, In in, Out out) {
  const T v0 = in(0), v1 = in(1), v2 = in(2), v3 = in(3), v4 = in(4);
  const T e0 = v0 + v4, e1 = v1 + v3, o0 = v0 - v4, o1 = v1 - v3;
  const T E0 = m.e[0][0] * e0 + m.e[0][1] * e1 + m.e[0][2] * v2;
  const T E1 = m.e[1][0] * e0 + m.e[1][1] * e1 + m.e[1][2] * v2;
  const T E2 = m.e[2][0] * e0 + m.e[2][1] * e1 + m.e[2][2] * v2;
  const T O0 = m.o[0][0] * o0 + m.o[0][1] * o1;
  const T O1 = m.o[1][0] * o0 + m.o[1][1] * o1;
  out(0, E0 + O0);
  out(1, E1 + O1);
  out(2, E2);
  out(3, E1 - O1);
  out(4, E0 - O0);
}

// x- then y-pass with B1 on a z-plane: v[ay][ax] -> v[qy][qx] (t is scratch)
template <typename T, int P1, bool EO>
__device__ __forceinline__ void cell_pass_xy(const CellCoef<T>& cf, T (&v)[P1 * P1], T (&t)[P1 * P1]) {
  if constexpr (EO) {
#pragma unroll
    for (int ay = 0; ay < P1; ++ay)
      eo5_apply(cf.eB1, [&](int a) { return v[ay * P1 + a]; }, [&](int q, T r) { t[ay * P1 + q] = r; });
#pragma unroll
    for (int qx = 0; qx < P1; ++qx)
      eo5_apply(cf.eB1, [&](int a) { return t[a * P1 + qx]; }, [&](int q, T r) { v[q * P1 + qx] = r; });
  } else {
#pragma unroll
    for (int ay = 0; ay < P1; ++ay)
#pragma unroll
      for (int qx = 0; qx < P1; ++qx) {
        T s = 0;
#pragma unroll
        for (int ax = 0; ax < P1; ++ax) s += cf.B1[qx][ax] * v[ay * P1 + ax];
        t[ay * P1 + qx] = s;
      }
#pragma unroll
    for (int qy = 0; qy < P1; ++qy)
#pragma unroll
      for (int qx = 0; qx < P1; ++qx) {
        T s = 0;
#pragma unroll
        for (int ay = 0; ay < P1; ++ay) s += cf.B1[qy][ay] * t[ay * P1 + qx];
        v[qy * P1 + qx] = s;
      }
  }
}

// z-pass with B1 on an x-plane: t[az][qy] -> u[qz][qy]
template <typename T, int P1, bool EO>
__device__ __forceinline__ void cell_pass_z(const CellCoef<T>& cf, const T (&t)[P1 * P1], T (&u)[P1 * P1]) {
  if constexpr (EO) {
#pragma unroll
    for (int qy = 0; qy < P1; ++qy)
      eo5_apply(cf.eB1, [&](int a) { return t[a * P1 + qy]; }, [&](int q, T r) { u[q * P1 + qy] = r; });
  } else {
#pragma unroll
    for (int qz = 0; qz < P1; ++qz)
#pragma unroll
      for (int qy = 0; qy < P1; ++qy) {
        T s = 0;
#pragma unroll
        for (int az = 0; az < P1; ++az) s += cf.B1[qz][az] * t[az * P1 + qy];
        u[qz * P1 + qy] = s;
      }
  }
}

// t' = (B^T)_y (B^T)_z t: t[qz][qy] -> tp[az][ay] (v is scratch)
template <typename T, int P1, bool EO>
__device__ __forceinline__ void cell_back_yz(const CellCoef<T>& cf, const T (&t)[P1 * P1], T (&v)[P1 * P1],
                                             T (&tp)[P1 * P1]) {
  if constexpr (EO) {
#pragma unroll
    for (int qz = 0; qz < P1; ++qz)
      eo5_apply(cf.eB1t, [&](int q) { return t[qz * P1 + q]; }, [&](int ay, T r) { v[qz * P1 + ay] = r; });
#pragma unroll
    for (int ay = 0; ay < P1; ++ay)
      eo5_apply(cf.eB1t, [&](int q) { return v[q * P1 + ay]; }, [&](int az, T r) { tp[az * P1 + ay] = r; });
  } else {
#pragma unroll
    for (int qz = 0; qz < P1; ++qz)
#pragma unroll
      for (int ay = 0; ay < P1; ++ay) {
        T s = 0;
#pragma unroll
        for (int qy = 0; qy < P1; ++qy) s += cf.B1[qy][ay] * t[qz * P1 + qy];
        v[qz * P1 + ay] = s;
      }
#pragma unroll
    for (int az = 0; az < P1; ++az)
#pragma unroll
      for (int ay = 0; ay < P1; ++ay) {
        T s = 0;
#pragma unroll
        for (int qz = 0; qz < P1; ++qz) s += cf.B1[qz][az] * v[qz * P1 + ay];
        tp[az * P1 + ay] = s;
      }
  }
}

// the x kinetic term before its x-pass: u <- kappa (B^T W)_y (B^T W)_z u (v is scratch)
template <typename T, int P1, bool EO>
__device__ __forceinline__ void cell_xkin_yz(const CellCoef<T>& cf, T (&u)[P1 * P1], T (&v)[P1 * P1]) {
  if constexpr (EO) {
#pragma unroll
    for (int qz = 0; qz < P1; ++qz)
      eo5_apply(cf.eBtW, [&](int q) { return u[qz * P1 + q]; }, [&](int ay, T r) { v[qz * P1 + ay] = r; });
#pragma unroll
    for (int ay = 0; ay < P1; ++ay)
      eo5_apply(cf.ekBtW, [&](int q) { return v[q * P1 + ay]; }, [&](int az, T r) { u[az * P1 + ay] = r; });
  } else {
#pragma unroll
    for (int qz = 0; qz < P1; ++qz)
#pragma unroll
      for (int ay = 0; ay < P1; ++ay) {
        T s = 0;
#pragma unroll
        for (int qy = 0; qy < P1; ++qy) s += cf.BtW[ay][qy] * u[qz * P1 + qy];
        v[qz * P1 + ay] = s;
      }
#pragma unroll
    for (int az = 0; az < P1; ++az)
#pragma unroll
      for (int ay = 0; ay < P1; ++ay) {
        T s = 0;
#pragma unroll
        for (int qz = 0; qz < P1; ++qz) s += cf.BtW[az][qz] * v[qz * P1 + ay];
        u[az * P1 + ay] = cf.kappa * s;
      }
  }
}

// the quadrature-point terms: t = W V u + kappa w_x (w_z L1_y u + w_y L1_z u); wvq(qz, qy) is
// W V at the point (qx, qy, qz) of this plane
template <typename T, int P1, bool EO, typename WV>
__device__ __forceinline__ void cell_point_terms(const CellCoef<T>& cf, const T (&u)[P1 * P1], T (&t)[P1 * P1],
                                                 WV wvq, T kx) {
#pragma unroll
  for (int qz = 0; qz < P1; ++qz) {
    T ly[P1];
    if constexpr (EO) {
      eo5_apply(cf.eL1, [&](int k) { return u[qz * P1 + k]; }, [&](int q, T r) { ly[q] = r; });
    } else {
#pragma unroll
      for (int qy = 0; qy < P1; ++qy) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < P1; ++k) s += cf.L1[qy][k] * u[qz * P1 + k];
        ly[qy] = s;
      }
    }
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) {
      T lz = 0;
#pragma unroll
      for (int k = 0; k < P1; ++k) lz += cf.L1[qz][k] * u[k * P1 + qy];
      t[qz * P1 + qy] = wvq(qz, qy) * u[qz * P1 + qy] + kx * (cf.w[qz] * ly[qy] + cf.w[qy] * lz);
    }
  }
}

// x-pass with B^T of one row: y[ax] = sum_q B1[q][ax] r[q]
template <typename T, int P1, bool EO>
__device__ __forceinline__ void cell_back_x(const CellCoef<T>& cf, const T (&r)[P1], T* y) {
  if constexpr (EO) {
    eo5_apply(cf.eB1t, [&](int q) { return r[q]; }, [&](int ax, T o) { y[ax] = o; });
  } else {
#pragma unroll
    for (int ax = 0; ax < P1; ++ax) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < P1; ++q) s += cf.B1[q][ax] * r[q];
      y[ax] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Cell kernel.
//
// Workgroup = P1 waves; wave w owns "plane" w of the (p+1)^3 cell tensor, lane l
// owns column l of a 64-column tile (CPT = 64 / CW cells x CW real columns).
// The x- and y-direction 1D passes run in registers on z-planes; a transpose
// through LDS gives x-planes for the z-pass and the quadrature-point work.
// In quadrature space the cell operator is
//   t = W V u + kappa [ (W (x) L1 (x) W) + (W (x) W (x) L1) ] u      (y-, z- kinetic terms)
//   y = B^T t + kappa (B^T L1) (x) (B^T W) (x) (B^T W) u                (x kinetic term)
// with u = B z, L1 the Gauss-point collocation Laplacian, kappa = h/4, which
// equals K_e z + B^T diag(W V) B z with the exact (Gauss) cell stiffness.
// ---------------------------------------------------------------------------
template <typename T, int P1, int CW, bool CPLX>
__global__ __launch_bounds__(64 * P1) void fe_cell_kernel(KBatch<T> kb, CellCoef<T> cf, int nc, int p, int n,
                                                          int64_t n_cells) {
  constexpr int NP = P1 * P1;
  constexpr int CPT = 64 / CW;
  constexpr bool EO = P1 == 5;  // the same passes as the planes-in-lanes kernel
  __shared__ T lds[NP * P1][64];
  const KP<T>& P = kb.k[blockIdx.z];
  const int ncr = P.ncr;
  if ((int)blockIdx.y * CW >= ncr) return;  // column block beyond this operator's width
  const T* __restrict__ X = P.x;
  const int64_t ldx = P.ldx;
  T* __restrict__ Yc = P.ycell;
  const int ldc = P.ldc;
  const Phase3<T> ph = P.ph;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int cl = lane / CW, col = lane % CW;
  const int64_t e = (int64_t)blockIdx.x * CPT + cl;
  const int j = blockIdx.y * CW + col;
  const bool valid = (e < n_cells) && (j < ncr);
  const int64_t ee = valid ? e : 0;
  const int cx = (int)(ee % nc), cy = (int)((ee / nc) % nc), cz = (int)(ee / ((int64_t)nc * nc));

  // 1. gather plane az = w with the m^-1/2 pre-scale (and Bloch phase)
  T v[NP];
  {
    const int az = w;
    int iz = cz * p + az;
    bool wz = iz >= n;
    if (wz) iz -= n;
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) {
      int iy = cy * p + ay;
      bool wy = iy >= n;
      if (wy) iy -= n;
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) {
        int ix = cx * p + ax;
        bool wx = ix >= n;
        if (wx) ix -= n;
        const int64_t g = ix + (int64_t)n * (iy + (int64_t)n * iz);
        const T sc = cf.mscale * cf.om[ax] * cf.om[ay] * cf.om[az];
        T val = 0;
        if (valid) {
          if constexpr (!CPLX) {
            val = X[g * ldx + j];
          } else {
            const T* px = X + g * ldx + (j & ~1);
            C2<T> z{px[0], px[1]};
            if (wx) z = cmul(z, C2<T>{ph.re[0], ph.im[0]});
            if (wy) z = cmul(z, C2<T>{ph.re[1], ph.im[1]});
            if (wz) z = cmul(z, C2<T>{ph.re[2], ph.im[2]});
            val = (j & 1) ? z.i : z.r;
          }
        }
        v[ay * P1 + ax] = sc * val;
      }
    }
  }
  // 2. x- then y-pass with B1 (in registers)
  T t[NP];
  cell_pass_xy<T, P1, EO>(cf, v, t);
  // 3. transpose z-planes -> x-planes: lds[(az*P1 + qy)*P1 + qx]
#pragma unroll
  for (int qy = 0; qy < P1; ++qy)
#pragma unroll
    for (int qx = 0; qx < P1; ++qx) lds[(w * P1 + qy) * P1 + qx][lane] = v[qy * P1 + qx];
  __syncthreads();
  // this wave now owns qx = w; u[az][qy]
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) t[az * P1 + qy] = lds[(az * P1 + qy) * P1 + w][lane];
  // 4. z-pass -> u[qz][qy]
  T u[NP];
  cell_pass_z<T, P1, EO>(cf, t, u);
  // 5. quadrature-point terms: potential + y/z kinetic
  const int qx = w;
  const T kx = cf.kappa * cf.w[qx];
  const T* wv = P.wv + ee * (NP * P1);
  cell_point_terms<T, P1, EO>(cf, u, t, [&](int qz, int qy) { return wv[(qz * P1 + qy) * P1 + qx]; }, kx);
  // 6. t' = (B^T)_y (B^T)_z t  -> indexed [az][ay]
  T tp[NP];
  cell_back_yz<T, P1, EO>(cf, t, v, tp);
  // 7. s = kappa (B^T W)_y (B^T W)_z u  (the x kinetic term before its x-pass)
  cell_xkin_yz<T, P1, EO>(cf, u, v);
  // 8. transpose t' back to z-planes, x-pass with B^T
  __syncthreads();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) lds[(az * P1 + ay) * P1 + w][lane] = tp[az * P1 + ay];
  __syncthreads();
  T y[NP];
#pragma unroll
  for (int ay = 0; ay < P1; ++ay) {
    T r[P1];
#pragma unroll
    for (int q = 0; q < P1; ++q) r[q] = lds[(w * P1 + ay) * P1 + q][lane];
    cell_back_x<T, P1, EO>(cf, r, y + ay * P1);
  }
  // 9. transpose s, x-pass with B^T L1, accumulate
  __syncthreads();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) lds[(az * P1 + ay) * P1 + w][lane] = u[az * P1 + ay];
  __syncthreads();
#pragma unroll
  for (int ay = 0; ay < P1; ++ay) {
    T r[P1];
#pragma unroll
    for (int q = 0; q < P1; ++q) r[q] = lds[(w * P1 + ay) * P1 + q][lane];
#pragma unroll
    for (int ax = 0; ax < P1; ++ax) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < P1; ++q) s += cf.BtL[ax][q] * r[q];
      y[ay * P1 + ax] += s;
    }
  }
  // 10. store plane az = w of y_e into the node-slot grid: local node a of cell c
  //     goes to slot (c (p+1) + a + 1) mod S per dimension, S = nc (p+1)
  if (valid) {
    const int S = nc * P1;
    int sz = cz * P1 + w + 1;
    if (sz >= S) sz -= S;
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) {
      int sy = cy * P1 + ay + 1;
      if (sy >= S) sy -= S;
      const int64_t rowyz = (int64_t)S * (sy + (int64_t)S * sz);
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) {
        int sx = cx * P1 + ax + 1;
        if (sx >= S) sx -= S;
        Yc[(rowyz + sx) * ldc + j] = y[ay * P1 + ax];
      }
    }
  }
}

// Cell kernel with the planes in the lanes of one wave: lane = r * CWc + g holds plane r of
// the cell tensor for column g of a CWc-column block (CWc = 64 / P1 rounded down to even;
// the 64 - P1 CWc spare lanes repeat the last plane's work and store nothing).  A wave
// owns one (cell, column block) and its own LDS region, so the three transposes need no
// workgroup barrier and the four waves of a workgroup carry equal work.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P1>
constexpr int lanes_cw() { return (64 / P1) & ~1; }

// UF: the periodic-function k-point form's first-derivative term -i k . int N grad N is added
// (complex columns only): k . grad u at the Gauss points (derivatives of the interpolant of the
// Gauss values, the x-derivative taken on the x-y plane before the transpose), weighted, from
// the complex partner lane (real <-> imaginary part) with the sign of -i, into the values that
// the backward passes project.
template <typename T, int P1, bool CPLX, bool UF = false>
__global__ __launch_bounds__(256, 3) void fe_cell_lanes_kernel(KBatch<T> kb, CellCoef<T> cf, int nc, int p, int n,
                                                            int64_t n_cells, int nch) {
  static_assert(!UF || CPLX, "the first-derivative term acts on complex columns");
  constexpr int NP = P1 * P1;
  constexpr int CWc = lanes_cw<P1>();
  // degree 4: the even-odd passes (the periodic-function form, which runs in this kernel only,
  // keeps the plain sums in float64: there its first-derivative term needs the registers)
  constexpr bool EO = P1 == 5 && (!UF || sizeof(T) == 4);
  // launch order: the column chunks of a group of 4 cells are consecutive in L, and each
  // XCD (workgroups bk = x mod 8) takes a contiguous range of L, so that the chunks reading
  // the same node rows, and neighbouring cells, share one L2
  const int nbk = gridDim.x, bk = blockIdx.x, nb8 = nbk & ~7;
  const int L = bk < nb8 ? (bk & 7) * (nb8 >> 3) + (bk >> 3) : bk;
  const int chunk = L % nch, cgrp = L / nch;
  __shared__ T lds_all[4][NP * P1 * CWc];
  __shared__ T wv_all[4][128];  // W V of the wave's cell at its quadrature points
  const KP<T>& P = kb.k[blockIdx.z];
  const int ncr = P.ncr;
  if (chunk * CWc >= ncr) return;  // column block beyond this operator's width
  const T* __restrict__ X = P.x;
  const int64_t ldx = P.ldx;
  T* __restrict__ Yc = P.ycell;
  const int ldc = P.ldc;
  const Phase3<T> ph = P.ph;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const bool active = lane < P1 * CWc;
  const int w = min(lane / CWc, P1 - 1);  // plane of this lane
  const int g = active ? lane % CWc : lane - P1 * CWc;  // spare lanes repeat a last-plane lane
  T* lds = lds_all[wid];
  const int64_t e = (int64_t)cgrp * 4 + wid;
  const int j = chunk * CWc + g;
  const bool valid = (e < n_cells) && (j < ncr);
  // the wave's cell (uniform: scalar arithmetic); a wave past the last cell addresses the last
  // cell's nodes and stores nothing
  const int eu = (int)(e < n_cells ? e : n_cells - 1);  // n_cells < 2^31
  const int cx = eu % nc, cy = (eu / nc) % nc, cz = eu / (nc * nc);
  // W V of the wave's cell: loaded now, parked in LDS after the first passes, read in step 5
  constexpr int NQ3 = NP * P1;
  const T* __restrict__ wvg = P.wv + (e < n_cells ? e : n_cells - 1) * NQ3;
  const T wv0 = wvg[min(lane, NQ3 - 1)], wv1 = wvg[min(lane + 64, NQ3 - 1)];

  // 1. gather plane az = w with the m^-1/2 pre-scale (and Bloch phase)
  const int jc = min(j, ncr - 1);
  const T vmask = valid ? T(1) : T(0);
  T v[NP];
  {
    const int az = w;
    int iz = cz * p + az;
    bool wz = iz >= n;
    if (wz) iz -= n;
    // addresses: one 64-bit base per lane for its z-plane, then 32-bit row offsets from
    // full-rate 24-bit products (iy n ldx + ix ldx < n^2 ldx < 2^31, checked at launch)
    const T* __restrict__ Xz = X + (int64_t)iz * n * n * ldx + (CPLX ? (jc & ~1) : jc);
    const unsigned ldx32 = (unsigned)ldx, ldxn = (unsigned)ldx * (unsigned)n;
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) {
      int iy = cy * p + ay;
      bool wy = iy >= n;
      if (wy) iy -= n;
      const unsigned oy = __umul24((unsigned)iy, ldxn);
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) {
        int ix = cx * p + ax;
        bool wx = ix >= n;
        if (wx) ix -= n;
        const unsigned off = oy + __umul24((unsigned)ix, ldx32);
        const T sc = cf.mscale * cf.om[ax] * cf.om[ay] * cf.om[az];
        // unconditional in-bounds loads (column clamped), zeroed by a multiply for lanes
        // outside the block: no branch around the load
        T val;
        if constexpr (!CPLX) {
          val = Xz[off];
        } else {
          const T* px = Xz + off;
          C2<T> z{px[0], px[1]};
          if (wx) z = cmul(z, C2<T>{ph.re[0], ph.im[0]});
          if (wy) z = cmul(z, C2<T>{ph.re[1], ph.im[1]});
          if (wz) z = cmul(z, C2<T>{ph.re[2], ph.im[2]});
          val = (jc & 1) ? z.i : z.r;
        }
        v[ay * P1 + ax] = sc * (val * vmask);
      }
    }
  }
  // 2. x- then y-pass with B1 (in registers)
  T t[NP];
  cell_pass_xy<T, P1, EO>(cf, v, t);
  // UF: x-derivative of the x-y plane (transposed after step 3, z-interpolated after step 4)
  T dxv[UF ? NP : 1];
  if constexpr (UF) {
#pragma unroll
    for (int qy = 0; qy < P1; ++qy)
#pragma unroll
      for (int qx = 0; qx < P1; ++qx) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < P1; ++k) s += cf.Dh[qx][k] * v[qy * P1 + k];
        dxv[qy * P1 + qx] = s;
      }
  }
  // 3. transpose z-planes -> x-planes: lds[(az*P1 + qy)*P1 + qx]
  T* wvs = wv_all[wid];
  if (lane < NQ3) wvs[lane] = wv0;
  if (lane + 64 < NQ3) wvs[lane + 64] = wv1;
#pragma unroll
  for (int qy = 0; qy < P1; ++qy)
#pragma unroll
    for (int qx = 0; qx < P1; ++qx) lds[((w * P1 + qy) * P1 + qx) * CWc + g] = v[qy * P1 + qx];
  wave_sync();
  // this wave now owns qx = w; u[az][qy]
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) t[az * P1 + qy] = lds[((az * P1 + qy) * P1 + w) * CWc + g];
  if constexpr (UF) {
    wave_sync();  // every lane has read the transpose
#pragma unroll
    for (int qy = 0; qy < P1; ++qy)
#pragma unroll
      for (int qx = 0; qx < P1; ++qx) lds[((w * P1 + qy) * P1 + qx) * CWc + g] = dxv[qy * P1 + qx];
    wave_sync();
  }
  // 4. z-pass -> u[qz][qy]
  T u[NP];
  cell_pass_z<T, P1, EO>(cf, t, u);
  // UF: t = W' uk . grad u at this lane's Gauss points (W' the product of the 1D weights; t is
  // free after step 4), taken from the complex partner with the sign of -i: real part
  // += (k.G) imag, imag -= (k.G) real; the x-derivative read from the transposed plane in LDS
  if constexpr (UF) {
    const T k0 = P.uk[0], k1 = P.uk[1], k2 = P.uk[2];
    const T sg = (g & 1) ? T(-1) : T(1);
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) {
      T dt[P1];
#pragma unroll
      for (int k = 0; k < P1; ++k) dt[k] = lds[((k * P1 + qy) * P1 + w) * CWc + g];
#pragma unroll
      for (int qz = 0; qz < P1; ++qz) {
        T dx = 0, dy = 0, dz = 0;
#pragma unroll
        for (int k = 0; k < P1; ++k) {
          dx += cf.B1[qz][k] * dt[k];
          dy += cf.Dh[qy][k] * u[qz * P1 + k];
          dz += cf.Dh[qz][k] * u[k * P1 + qy];
        }
        const T tg = cf.w[w] * cf.w[qy] * cf.w[qz] * (k0 * dx + k1 * dy + k2 * dz);
        t[qz * P1 + qy] = sg * __shfl_xor(tg, 1);
      }
    }
  }
  // 5. quadrature-point terms: potential + y/z kinetic
  const int qx = w;
  const T kx = cf.kappa * cf.w[qx];
  if constexpr (UF) {
#pragma unroll
    for (int qz = 0; qz < P1; ++qz)
#pragma unroll
      for (int qy = 0; qy < P1; ++qy) {
        T ly = 0, lz = 0;
#pragma unroll
        for (int k = 0; k < P1; ++k) {
          ly += cf.L1[qy][k] * u[qz * P1 + k];
          lz += cf.L1[qz][k] * u[k * P1 + qy];
        }
        const T tq = wvs[(qz * P1 + qy) * P1 + qx] * u[qz * P1 + qy] + kx * (cf.w[qz] * ly + cf.w[qy] * lz);
        t[qz * P1 + qy] = tq + t[qz * P1 + qy];
      }
  } else {
    cell_point_terms<T, P1, EO>(cf, u, t, [&](int qz, int qy) { return wvs[(qz * P1 + qy) * P1 + qx]; }, kx);
  }
  // 6. t' = (B^T)_y (B^T)_z t  -> indexed [az][ay]
  T tp[NP];
  cell_back_yz<T, P1, EO>(cf, t, v, tp);
  // 7. s = kappa (B^T W)_y (B^T W)_z u  (the x kinetic term before its x-pass)
  cell_xkin_yz<T, P1, EO>(cf, u, v);
  // 8. transpose t' back to z-planes, x-pass with B^T
  wave_sync();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) lds[((az * P1 + ay) * P1 + w) * CWc + g] = tp[az * P1 + ay];
  wave_sync();
  T y[NP];
#pragma unroll
  for (int ay = 0; ay < P1; ++ay) {
    T r[P1];
#pragma unroll
    for (int q = 0; q < P1; ++q) r[q] = lds[((w * P1 + ay) * P1 + q) * CWc + g];
    cell_back_x<T, P1, EO>(cf, r, y + ay * P1);
  }
  // 9. transpose s, x-pass with B^T L1, accumulate
  wave_sync();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) lds[((az * P1 + ay) * P1 + w) * CWc + g] = u[az * P1 + ay];
  wave_sync();
#pragma unroll
  for (int ay = 0; ay < P1; ++ay) {
    T r[P1];
#pragma unroll
    for (int q = 0; q < P1; ++q) r[q] = lds[((w * P1 + ay) * P1 + q) * CWc + g];
#pragma unroll
    for (int ax = 0; ax < P1; ++ax) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < P1; ++q) s += cf.BtL[ax][q] * r[q];
      y[ay * P1 + ax] += s;
    }
  }
  // 10. store plane az = w of y_e into the node-slot grid: local node a of cell c
  //     goes to slot (c (p+1) + a + 1) mod S per dimension, S = nc (p+1)
  if (valid && active) {
    const int S = nc * P1;
    int sz = cz * P1 + w + 1;
    if (sz >= S) sz -= S;
    // one 64-bit base per lane for its slot plane, 32-bit offsets below S^2 ldc < 2^31
    T* __restrict__ Ycz = Yc + (int64_t)sz * S * S * ldc + j;
    const unsigned ldc32 = (unsigned)ldc, ldcs = (unsigned)ldc * (unsigned)S;
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) {
      int sy = cy * P1 + ay + 1;
      if (sy >= S) sy -= S;
      const unsigned oy = __umul24((unsigned)sy, ldcs);
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) {
        int sx = cx * P1 + ax + 1;
        if (sx >= S) sx -= S;
        Ycz[oy + __umul24((unsigned)sx, ldc32)] = y[ay * P1 + ax];
      }
    }
  }
}

// Cell stage at one real column (the auxiliary potential's conjugate gradients, Lanczos): the
// planes-in-lanes kernel with cells in the place of columns, lane = plane x CWc + cell of the
// wave, where the column layout would leave 11 of its 12 lane groups idle.  Every lane forms its
// own cell's addresses (64-bit), reads W V of its cell's points from device memory, and runs the
// same passes in the same order, so each cell's values equal the column layout's bit for bit.
template <typename T, int P1>
__global__ __launch_bounds__(256, 3) void fe_cell_cells_kernel(KBatch<T> kb, CellCoef<T> cf, int nc, int p, int n,
                                                               int64_t n_cells) {
  constexpr int NP = P1 * P1;
  constexpr int CWc = lanes_cw<P1>();
  constexpr bool EO = P1 == 5;
  __shared__ T lds_all[4][NP * P1 * CWc];
  const KP<T>& P = kb.k[blockIdx.z];
  const T* __restrict__ X = P.x;
  const int64_t ldx = P.ldx, ldc = P.ldc;
  T* __restrict__ Yc = P.ycell;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const bool active = lane < P1 * CWc;
  const int w = min(lane / CWc, P1 - 1);                // plane of this lane
  const int g = active ? lane % CWc : lane - P1 * CWc;  // cell of the wave; spare lanes repeat a last-plane lane
  T* lds = lds_all[wid];
  const int64_t e = ((int64_t)blockIdx.x * 4 + wid) * CWc + g;
  const bool valid = e < n_cells;
  const int64_t eu = valid ? e : n_cells - 1;  // a lane past the last cell works on the last cell and stores nothing
  const int cx = (int)(eu % nc), cy = (int)((eu / nc) % nc), cz = (int)(eu / ((int64_t)nc * nc));
  const T vmask = valid ? T(1) : T(0);

  // 1. gather plane az = w with the m^-1/2 pre-scale
  T v[NP];
  {
    const int az = w;
    int iz = cz * p + az;
    if (iz >= n) iz -= n;
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) {
      int iy = cy * p + ay;
      if (iy >= n) iy -= n;
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) {
        int ix = cx * p + ax;
        if (ix >= n) ix -= n;
        const T sc = cf.mscale * cf.om[ax] * cf.om[ay] * cf.om[az];
        const T val = X[(ix + (int64_t)n * (iy + (int64_t)n * iz)) * ldx];
        v[ay * P1 + ax] = sc * (val * vmask);
      }
    }
  }
  // 2. x- then y-pass
  T t[NP];
  cell_pass_xy<T, P1, EO>(cf, v, t);
  // 3. transpose z-planes -> x-planes
#pragma unroll
  for (int qy = 0; qy < P1; ++qy)
#pragma unroll
    for (int qx = 0; qx < P1; ++qx) lds[((w * P1 + qy) * P1 + qx) * CWc + g] = v[qy * P1 + qx];
  wave_sync();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) t[az * P1 + qy] = lds[((az * P1 + qy) * P1 + w) * CWc + g];
  // 4. z-pass
  T u[NP];
  cell_pass_z<T, P1, EO>(cf, t, u);
  // 5. quadrature-point terms (W V of this lane's cell at the points of its plane)
  const int qx = w;
  const T kx = cf.kappa * cf.w[qx];
  const T* __restrict__ wvc = P.wv + eu * (NP * P1);
  cell_point_terms<T, P1, EO>(cf, u, t, [&](int qz, int qy) { return wvc[(qz * P1 + qy) * P1 + qx]; }, kx);
  // 6. t' = (B^T)_y (B^T)_z t; 7. the x kinetic term before its x-pass
  T tp[NP];
  cell_back_yz<T, P1, EO>(cf, t, v, tp);
  cell_xkin_yz<T, P1, EO>(cf, u, v);
  // 8. transpose t' back to z-planes, x-pass with B^T
  wave_sync();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) lds[((az * P1 + ay) * P1 + w) * CWc + g] = tp[az * P1 + ay];
  wave_sync();
  T y[NP];
#pragma unroll
  for (int ay = 0; ay < P1; ++ay) {
    T r[P1];
#pragma unroll
    for (int q = 0; q < P1; ++q) r[q] = lds[((w * P1 + ay) * P1 + q) * CWc + g];
    cell_back_x<T, P1, EO>(cf, r, y + ay * P1);
  }
  // 9. transpose s, x-pass with B^T L1, accumulate
  wave_sync();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) lds[((az * P1 + ay) * P1 + w) * CWc + g] = u[az * P1 + ay];
  wave_sync();
#pragma unroll
  for (int ay = 0; ay < P1; ++ay) {
    T r[P1];
#pragma unroll
    for (int q = 0; q < P1; ++q) r[q] = lds[((w * P1 + ay) * P1 + q) * CWc + g];
#pragma unroll
    for (int ax = 0; ax < P1; ++ax) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < P1; ++q) s += cf.BtL[ax][q] * r[q];
      y[ay * P1 + ax] += s;
    }
  }
  // 10. store plane az = w of the cell's result into the node-slot grid (column 0)
  if (valid && active) {
    const int S = nc * P1;
    int sz = cz * P1 + w + 1;
    if (sz >= S) sz -= S;
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) {
      int sy = cy * P1 + ay + 1;
      if (sy >= S) sy -= S;
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) {
        int sx = cx * P1 + ax + 1;
        if (sx >= S) sx -= S;
        Yc[(sx + (int64_t)S * (sy + (int64_t)S * sz)) * ldc] = y[ay * P1 + ax];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 cell kernel (real operators, float32 vectors): the cell operator in dense form
//   U = B Z,  T = (W V) o U,  Y = K Z + B^T T
// on the matrix cores (16x16x32 bf16 MFMA, float32 accumulation), with B, K, B^T
// (128 x 128, zero-padded) held in LDS in A-fragment order.  Z (nodes x 16 columns of
// one cell, m^-1/2 pre-scaled) and T are rounded to bf16; U and Y stay float32.  The
// lane layout of the result of B Z is the operand layout of B^T T up to a fixed
// permutation of each 32-point block, which is built into the stored B^T.  Each wave
// takes (cell, 16-column block) tasks in turn; Y goes to the node-slot grid.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBf16MatElems = 8 * 4 * 64 * 8;  // one 128 x 128 matrix in fragment order

__global__ __launch_bounds__(768) void fe_cell_bf16_kernel(KBatch<float> kb, const uint16_t* __restrict__ mats,
                                                           CellCoef<float> cf, int nc, int p, int n, int P1,
                                                           int64_t n_cells) {
  extern __shared__ unsigned char smem_raw[];
  bf16x8* frag = reinterpret_cast<bf16x8*>(smem_raw);  // [3][8][4][64]
  // per local node a < 128: (ax, ay, az) packed in 8-bit fields, and the m^-1/2 factor
  int* ncode = reinterpret_cast<int*>(smem_raw + 3 * kBf16MatElems * sizeof(uint16_t));
  float* nscale = reinterpret_cast<float*>(ncode + 128);
  // offsets of local node a from the cell's first node (global rows) and first slot (grid
  // rows), valid for cells that do not touch the upper periodic boundary
  int* noff = reinterpret_cast<int*>(nscale + 128);
  int* soff = noff + 128;
  const int nd = P1 * P1 * P1;
  {
    const uint4* src = reinterpret_cast<const uint4*>(mats);
    uint4* dst = reinterpret_cast<uint4*>(smem_raw);
    for (int i = threadIdx.x; i < 3 * kBf16MatElems / 8; i += blockDim.x) dst[i] = src[i];
    if (threadIdx.x < 128) {
      const int a = threadIdx.x;
      const int ax = a % P1, ay = (a / P1) % P1, az = a / (P1 * P1);
      float om[kMaxP1];
#pragma unroll
      for (int i = 0; i < kMaxP1; ++i) om[i] = cf.om[i];
      float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
      for (int i = 0; i < kMaxP1; ++i) {
        sx = i == ax ? om[i] : sx;
        sy = i == ay ? om[i] : sy;
        sz = i == az ? om[i] : sz;
      }
      ncode[a] = a < nd ? (ax | (ay << 8) | (az << 16)) : 0;
      nscale[a] = a < nd ? cf.mscale * sx * sy * sz : 0.0f;
      noff[a] = a < nd ? ax + n * (ay + n * az) : 0;
      soff[a] = a < nd ? ax + nc * P1 * (ay + nc * P1 * az) : 0;
    }
  }
  __syncthreads();
  const bf16x8* fB = frag;
  const bf16x8* fK = frag + kBf16MatElems / 8;
  const bf16x8* fBT = frag + 2 * kBf16MatElems / 8;
  const KP<float>& P = kb.k[blockIdx.z];
  const int ncr = P.ncr;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int ncb = (ncr + 15) / 16;
  const int64_t ntask = n_cells * ncb;
  const float* __restrict__ X = P.x;
  const int64_t ldx = P.ldx;
  float* __restrict__ Yc = P.ycell;
  const int64_t ldc = P.ldc;
  const int S = nc * P1;
  // workgroups of one XCD (blockIdx.x = x mod 8) take a contiguous range of task groups,
  // so that the column blocks of a cell and neighbouring cells share one L2
  const int nbk = gridDim.x, bk = blockIdx.x, nb8 = nbk & ~7;
  const int wg = bk < nb8 ? (bk & 7) * (nb8 >> 3) + (bk >> 3) : bk;
  for (int64_t task = (int64_t)wg * nw + w; task < ntask; task += (int64_t)gridDim.x * nw) {
    const int64_t e = task / ncb;
    const int col = (int)(task - e * ncb) * 16 + c;
    const bool cok = col < ncr;
    const int cc = cok ? col : ncr - 1;
    const int cx = (int)(e % nc), cy = (int)((e / nc) % nc), cz = (int)(e / ((int64_t)nc * nc));
    const int bx = cx * p, by = cy * p, bz = cz * p;
    // Z: node 32 k4 + 8 g + t of the cell, column col, scaled by m^-1/2 (one batch of loads);
    // a cell away from the upper periodic boundary (wave-uniform) indexes by table offsets
    const bool interior = cx < nc - 1 && cy < nc - 1 && cz < nc - 1;
    const int64_t gbase = bx + (int64_t)n * (by + (int64_t)n * bz);
    // W V of this lane's quadrature points, loaded with the gather (used after U = B Z)
    const float* wv = P.wv + e * nd;
    float wq[4][8];
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q0 = 32 * k4 + 4 * g + v, q1 = q0 + 16;
        wq[k4][v] = wv[q0 < nd ? q0 : 0];
        wq[k4][4 + v] = wv[q1 < nd ? q1 : 0];
      }
    bf16x8 z[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // two batches of 16 loads
      float zv[16];
      if (interior) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int a = 32 * (2 * h + (i >> 3)) + 8 * g + (i & 7);
          zv[i] = X[(gbase + noff[a]) * ldx + cc];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int a = 32 * (2 * h + (i >> 3)) + 8 * g + (i & 7);
          const int code = ncode[a];
          int ix = bx + (code & 255), iy = by + ((code >> 8) & 255), iz = bz + (code >> 16);
          ix -= ix >= n ? n : 0;
          iy -= iy >= n ? n : 0;
          iz -= iz >= n ? n : 0;
          zv[i] = X[(ix + (int64_t)n * (iy + (int64_t)n * iz)) * ldx + cc];
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i)
        z[2 * h + (i >> 3)][i & 7] = (__bf16)(zv[i] * nscale[32 * (2 * h + (i >> 3)) + 8 * g + (i & 7)]);
      __builtin_amdgcn_sched_barrier(0);
    }
    // U = B Z
    f32x4 u[8];
#pragma unroll
    for (int mb = 0; mb < 8; ++mb) {
      u[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4)
        u[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fB[(mb * 4 + k4) * 64 + lane], z[k4], u[mb], 0, 0, 0);
    }
    // T = (W V) o U, as the operand of B^T T (point 16 mb + 4 g + v of U sits in lane g, element v)
    bf16x8 tq[4];
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q0 = 32 * k4 + 4 * g + v, q1 = q0 + 16;
        tq[k4][v] = (__bf16)(q0 < nd ? wq[k4][v] * u[2 * k4][v] : 0.0f);
        tq[k4][4 + v] = (__bf16)(q1 < nd ? wq[k4][4 + v] * u[2 * k4 + 1][v] : 0.0f);
      }
    // Y = K Z + B^T T, stored to the node-slot grid
#pragma unroll 2
    for (int mb = 0; mb < 8; ++mb) {
      f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fK[(mb * 4 + k4) * 64 + lane], z[k4], y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fBT[(mb * 4 + k4) * 64 + lane], tq[k4], y, 0, 0, 0);
      }
      if (interior) {
        const int64_t sbase = (cx * P1 + 1) + (int64_t)S * ((cy * P1 + 1) + (int64_t)S * (cz * P1 + 1));
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * mb + 4 * g + v;
          if (cok && a < nd) Yc[(sbase + soff[a]) * ldc + col] = y[v];
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * mb + 4 * g + v;
          if (cok && a < nd) {
            const int code = ncode[a];
            int sx = cx * P1 + (code & 255) + 1, sy = cy * P1 + ((code >> 8) & 255) + 1,
                sz = cz * P1 + (code >> 16) + 1;
            sx -= sx >= S ? S : 0;
            sy -= sy >= S ? S : 0;
            sz -= sz >= S ? S : 0;
            Yc[(sx + (int64_t)S * (sy + (int64_t)S * sz)) * ldc + col] = y[v];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Node stage, split in two kernels so that the dense coupling work leaves the
// critical path:
//
// fe_coupling_kernel (side stream, beside the cell stage; needs only X and Z^O):
//   for each coupling tile t of kTileRows FE rows (tile_node) and each group of 16 NBW real columns
//     part_t = Ht_t^* X_t              -> per-tile partial of W' (reduced later)
//     out_t  = alpha Ht_t Z^O - beta prev_t
//   (Ht_t: the tile's dense block of m^-1/2 H^co) on the matrix cores (16x16x4 MFMA,
//   float64 or float32).  One wave per (tile, column group), no LDS and no barriers: the
//   tile's block and Z^O are read through the caches, shared by the waves of a tile.
//
// fe_assemble_kernel (main stream, after the cell stage), one element per thread:
//   out = alpha (m^-1/2 sum_slots(Y) - c x) + base,  base = out (the coupling kernel's
//   result) or -beta prev when the operator has no enrichment.
//   sum_slots adds, in a fixed order, the (up to 8) cell results stored for the node in
//   the node-slot grid (no atomics).
//
// Complex columns are interleaved (re, im); a complex product is two real MFMA passes
// over the real and imaginary parts of Ht with the matching (swapped, signed) columns.
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held by lane l in element v (column l % 16)
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

constexpr int kCoupleNBWMax = 2;  // 16-column blocks per coupling wave

// LDS of the coupling kernel: the tile's block, one plane per real / imaginary part, rows
// of FP + 1 (odd) elements so that 16 lanes reading 16 consecutive functions of a row, or
// one function of 16 consecutive rows, touch 16 distinct bank pairs; then the function list.
__host__ __device__ constexpr int coupling_row_stride(int fp) { return fp + 1; }

template <typename T, bool CPLX>
constexpr size_t coupling_lds_bytes(int fpmax) {
  return (size_t)(CPLX ? 2 : 1) * kTileRows * coupling_row_stride(fpmax) * sizeof(T) + (size_t)fpmax * sizeof(int32_t);
}

// part columns of NQ blocks of 16 functions (from function m0) over the tile's TR rows:
// pc[q][nb] += Ht_t[r][m0 + 16 q + .]^* x[r][cols of block nb], k-steps of 4 rows with the
// x loads of 4 k-steps issued ahead of their MFMAs; Ht_t from LDS (planes hs[e])
template <typename T, int NQ, int NBW, bool CPLX>
__device__ __forceinline__ void coupling_part(const T* hs, int HS, const T* __restrict__ x, int64_t ldx, int tx0,
                                              int ty0, int tz0, int n, int tm, int FP, int m0, const int (&colc)[NBW], int li,
                                              int lk,
                                              typename Mfma<T>::V4 (&pc)[4][NBW]) {
  using M = Mfma<T>;
  constexpr int TR = kTileRows, E = CPLX ? 2 : 1, KB = 4;
  const T sgn = (li & 1) ? T(-1) : T(1);
  int fcl[NQ];
  bool fok[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int f = m0 + q * 16 + li;
    fok[q] = f < FP;
    fcl[q] = fok[q] ? f : FP - 1;
  }
  for (int ks0 = 0; ks0 < TR / 4; ks0 += KB) {
    T b[KB][E][NBW];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int r = (ks0 + j) * 4 + lk;
      const int gt = tile_row_node(tx0, ty0, tz0, r, n, tm);
      const bool rok = gt >= 0;
      const int64_t g = rok ? gt : 0;
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        // multiply by 1 or 0 rather than select: keeps the load unconditional and batched
        b[j][0][nb] = x[g * ldx + colc[nb]] * (rok ? T(1) : T(0));
      }
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int r = (ks0 + j) * 4 + lk;
      if constexpr (CPLX) {
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) b[j][1][nb] = sgn * __shfl_xor(b[j][0][nb], 1);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const T av = hs[(e * TR + r) * HS + fcl[q]];
          const T a = fok[q] ? av : T(0);
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb) pc[q][nb] = M::op(a, b[j][e][nb], pc[q][nb]);
        }
    }
  }
}

template <typename T, int NBW, bool CPLX>
__global__ __launch_bounds__(256, NBW == 1 ? 2 : 1) void fe_coupling_kernel(KBatch<T> kb, const int32_t* __restrict__ tile_fptr,
                                                          const int32_t* __restrict__ tile_fns, int n, int tm) {
  using M = Mfma<T>;
  using V4 = typename M::V4;
  constexpr int TR = kTileRows, E = CPLX ? 2 : 1, RB = TR / 16, HPT = 8;
  extern __shared__ unsigned char smem_raw[];
  const KP<T>& P = kb.k[blockIdx.z];
  const int ncr = P.ncr;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int t = blockIdx.x;
  int tx0, ty0, tz0;
  tile_origin(t, n, tm, tx0, ty0, tz0);
  const int f0 = tile_fptr[t], FP = tile_fptr[t + 1] - f0;  // FP: a multiple of 4
  const int HS = coupling_row_stride(FP);
  T* hs = reinterpret_cast<T*>(smem_raw);                   // [E][TR][HS]
  int32_t* fs = reinterpret_cast<int32_t*>(hs + E * TR * HS);  // [FP]
  const T* __restrict__ tv = P.tv + (int64_t)f0 * TR * E;   // [TR][FP][E], zero rows past the mesh
  const T* __restrict__ x = P.x;
  const T* __restrict__ zo = P.zo;  // [n_enr][ncr]
  const int64_t ldx = P.ldx, ldo = P.ldo;
  const int ngrp = (ncr + 16 * NBW - 1) / (16 * NBW);

  // ---- stage the tile's block (batches of HPT coalesced loads per thread) and its function list
  const int nh = TR * FP * E;
  for (int q0 = 0; q0 < nh; q0 += 256 * HPT) {
    T hv[HPT];
#pragma unroll
    for (int i = 0; i < HPT; ++i) hv[i] = tv[min(q0 + (int)threadIdx.x + 256 * i, nh - 1)];
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const int q = q0 + threadIdx.x + 256 * i;
      if (q < nh) {
        const int r = q / (FP * E), rem = q - r * FP * E, f = rem / E, e = rem - f * E;
        hs[(e * TR + r) * HS + f] = hv[i];
      }
    }
  }
  for (int f = threadIdx.x; f < FP; f += 256) fs[f] = tile_fns[f0 + f];
  __syncthreads();

  // ---- each wave: column groups w, w + 4, ...
  for (int grp = w; grp < ngrp; grp += 4) {
    const int cb0 = grp * 16 * NBW;
    // Loads are unconditional, from clamped in-bounds addresses, with unwanted values
    // replaced by selects, so that each batch is issued at once.
    int colc[NBW];
    bool colok[NBW];
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      const int col = cb0 + nb * 16 + li;
      colok[nb] = col < ncr;
      colc[nb] = colok[nb] ? col : ncr - 1;
    }

    // part = Ht_t^* X_t, up to 4 blocks of 16 functions at a time
    // (complex: e = 1 pairs Im(H) with the partner column, signed)
    for (int m0 = 0; m0 < FP; m0 += 64) {
      V4 pc[4][NBW];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) pc[q][nb] = V4{0, 0, 0, 0};
      const int nq = min(4, (FP - m0 + 15) / 16);
      switch (nq) {
        case 4: coupling_part<T, 4, NBW, CPLX>(hs, HS, x, ldx, tx0, ty0, tz0, n, tm, FP, m0, colc, li, lk, pc); break;
        case 3: coupling_part<T, 3, NBW, CPLX>(hs, HS, x, ldx, tx0, ty0, tz0, n, tm, FP, m0, colc, li, lk, pc); break;
        case 2: coupling_part<T, 2, NBW, CPLX>(hs, HS, x, ldx, tx0, ty0, tz0, n, tm, FP, m0, colc, li, lk, pc); break;
        default: coupling_part<T, 1, NBW, CPLX>(hs, HS, x, ldx, tx0, ty0, tz0, n, tm, FP, m0, colc, li, lk, pc); break;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q >= nq) break;
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb) {
          if (!colok[nb]) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int fi = m0 + q * 16 + M::row(lane, v);
            if (fi < FP) P.part[(int64_t)(f0 + fi) * ncr + colc[nb]] = pc[q][nb][v];
          }
        }
      }
    }

    // en = Ht_t Z^O for the RB 16-row blocks of the tile, k-steps of 4 functions with the
    // Z^O loads of KB k-steps issued ahead (a k-step past the list multiplies zero columns)
    V4 acc[RB][NBW];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) acc[rb][nb] = V4{0, 0, 0, 0};
    {
      constexpr int KB = 4;
      const T sgn = (li & 1) ? T(1) : T(-1);
      for (int k0 = 0; k0 < FP; k0 += 4 * KB) {
        T b[KB][E][NBW];
#pragma unroll
        for (int j = 0; j < KB; ++j) {
          const int f = k0 + 4 * j + lk;
          const int fn = f < FP ? fs[f] : -1;
          const T* __restrict__ zr = zo + (int64_t)max(fn, 0) * ncr;
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb) b[j][0][nb] = zr[colc[nb]] * (fn >= 0 ? T(1) : T(0));
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) {
          const int f = min(k0 + 4 * j + lk, FP - 1);
          if constexpr (CPLX) {
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) b[j][1][nb] = sgn * __shfl_xor(b[j][0][nb], 1);
          }
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int e = 0; e < E; ++e) {
              const T a = hs[(e * TR + rb * 16 + li) * HS + f];
#pragma unroll
              for (int nb = 0; nb < NBW; ++nb) acc[rb][nb] = M::op(a, b[j][e][nb], acc[rb][nb]);
            }
        }
      }
    }

    // out = alpha en - beta prev (prev may be the same array as out: all of this lane's
    // elements are read before any is written)
    T alpha, cst, beta;
    step_scalars(P, alpha, cst, beta);
    T pv[RB][4][NBW];
    if (beta != T(0)) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t g = max(tile_row_node(tx0, ty0, tz0, rb * 16 + M::row(lane, v), n, tm), 0);
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb) pv[rb][v][nb] = beta * P.prev[g * ldo + colc[nb]];
        }
    } else {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb) pv[rb][v][nb] = T(0);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gv = tile_row_node(tx0, ty0, tz0, rb * 16 + M::row(lane, v), n, tm);
        if (gv < 0) continue;
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
          if (colok[nb]) P.out[(int64_t)gv * ldo + colc[nb]] = alpha * acc[rb][nb][v] - pv[rb][v][nb];
      }
  }
}

// Flat element index -> (row, column) for rows of nel elements, without a 64-bit
// integer division: a float64 quotient corrected by one step.
__device__ __forceinline__ int64_t row_of(int64_t i, int nel, double rnel) {
  int64_t g = (int64_t)((double)i * rnel);
  const int64_t r = i - g * nel;
  g += r < 0 ? -1 : (r >= nel ? 1 : 0);
  return g;
}

// floor(a / d) for 0 <= a < 2^31, 1 <= d, from rd = 1 / d in float64 (the product is within one
// of the quotient; one correction step), instead of an integer division sequence
__device__ __forceinline__ int div_rcp(int a, int d, double rd) {
  int q = (int)((double)a * rd);
  const int r = a - q * d;
  q += r < 0 ? -1 : (r >= d ? 1 : 0);
  return q;
}
// a / p for the supported element degrees p = 2, 3, 4 (a >= 0): constant divisors
__device__ __forceinline__ int div_p(int a, int p) { return p == 4 ? a >> 2 : (p == 2 ? a >> 1 : a / 3); }

template <typename T, bool CPLX>
__device__ __forceinline__ void assemble_one(const KP<T>& P, int64_t i, int nel, double rnel, int nc, int p, int n,
                                             int P1, const CellCoef<T>& cf, int base_in_out);

template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void fe_assemble_kernel(KBatch<T> kb, int nc, int p, int n, int P1, CellCoef<T> cf,
                                                          int N, int base_in_out) {
  const KP<T>& P = kb.k[blockIdx.z];
  const int nel = CPLX ? P.nv : P.ncr;  // elements per row: complex pairs or real columns
  const int64_t total = (int64_t)N * nel;
  const double rnel = 1.0 / nel;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
    assemble_one<T, CPLX>(P, i, nel, rnel, nc, p, n, P1, cf, base_in_out);
}

template <typename T, bool CPLX>
__device__ __forceinline__ void assemble_one(const KP<T>& P, int64_t i, int nel, double rnel, int nc, int p, int n,
                                             int P1, const CellCoef<T>& cf, int base_in_out) {
  const int64_t g = row_of(i, nel, rnel);
  const int j = (int)(i - g * nel);
  const int gi = (int)g;
  const int nn = n * n;
  const int iz = div_rcp(gi, nn, 1.0 / nn), rem = gi - iz * nn, iy = div_rcp(rem, n, 1.0 / n), ix = rem - iy * n;
  const int qx = div_p(ix, p), rx = ix - qx * p, qy = div_p(iy, p), ry = iy - qy * p, qz = div_p(iz, p),
            rz = iz - qz * p;
  const int S = nc * P1;
  const int bx = qx * P1 + (rx ? rx + 1 : 0), by = qy * P1 + (ry ? ry + 1 : 0), bz = qz * P1 + (rz ? rz + 1 : 0);
  const T msc = cf.mscale * cf.om[rx] * cf.om[ry] * cf.om[rz];
  const T* __restrict__ Yc = P.ycell;
  const int64_t ldc = P.ldc;
  T alpha, c, beta;
  step_scalars(P, alpha, c, beta);
  // (ky, kz) slot pairs in a fixed order, each the lower-x slot then (shared x node) the next one
  if constexpr (!CPLX) {
    T s = 0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int ky = kk & 1, kz = kk >> 1;
      if ((ky && ry) || (kz && rz)) continue;
      const int64_t r0 = bx + (int64_t)S * (by + ky + (int64_t)S * (bz + kz));
      T add = Yc[r0 * ldc + j];
      if (rx == 0) add += Yc[(r0 + 1) * ldc + j];
      s += add;
    }
    const int64_t io = g * P.ldo + j;
    const T base = base_in_out ? P.out[io] : (beta != T(0) ? -beta * P.prev[io] : T(0));
    P.out[io] = alpha * (msc * s - c * P.x[g * P.ldx + j]) + base;
  } else {
    const Phase3<T> ph = P.ph;
    C2<T> s{0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int ky = kk & 1, kz = kk >> 1;
      if ((ky && ry) || (kz && rz)) continue;
      const int sy = by + ky, sz = bz + kz;
      const int64_t r0 = bx + (int64_t)S * (sy + (int64_t)S * sz);
      C2<T> z0{Yc[r0 * ldc + 2 * j], Yc[r0 * ldc + 2 * j + 1]};
      C2<T> z1{0, 0};
      if (rx == 0) z1 = C2<T>{Yc[(r0 + 1) * ldc + 2 * j], Yc[(r0 + 1) * ldc + 2 * j + 1]};
      // periodic images: slot 0 of a dimension came from the last cell
      if (bx == 0) z0 = cjmul(C2<T>{ph.re[0], ph.im[0]}, z0);
      if (sy == 0) {
        z0 = cjmul(C2<T>{ph.re[1], ph.im[1]}, z0);
        z1 = cjmul(C2<T>{ph.re[1], ph.im[1]}, z1);
      }
      if (sz == 0) {
        z0 = cjmul(C2<T>{ph.re[2], ph.im[2]}, z0);
        z1 = cjmul(C2<T>{ph.re[2], ph.im[2]}, z1);
      }
      s.r += z0.r + z1.r;
      s.i += z0.i + z1.i;
    }
    const int64_t io = g * P.ldo + 2 * j, ix2 = g * P.ldx + 2 * j;
    C2<T> base{0, 0};
    if (base_in_out) base = C2<T>{P.out[io], P.out[io + 1]};
    else if (beta != T(0)) base = C2<T>{-beta * P.prev[io], -beta * P.prev[io + 1]};
    P.out[io] = alpha * (msc * s.r - c * P.x[ix2]) + base.r;
    P.out[io + 1] = alpha * (msc * s.i - c * P.x[ix2 + 1]) + base.i;
  }
}

// Node stage of real operators in one kernel, fe_node_fused_kernel: one workgroup (4
// waves) per coupling tile of kTileRows FE rows (tile_node) x 16 NB real columns computes part, the slot
// gather and out = alpha (m^-1/2 sum_slots(Y) + Ht_t Z^O - c x) - beta prev.  Order within
// the workgroup: one batch of loads (x tile, H tile, function list; float32 also the
// first slot pair of the gather, which lands during the matrix-core phase), part on the
// matrix cores, the gather, acc = m^-1/2 sum - c x, then Ht_t Z^O accumulated onto acc
// from Z^O rows staged in LDS, with the previous iterate loaded beside them.
// LDS of the node kernel: the tile's rows of X (its column block; reused afterwards
// for chunks of up to kTileRows rows of Z^O), its dense block of m^-1/2 H^co, and the
// tile's function list.
// Row strides (in elements) of the node kernel's LDS tiles, padded to 16 mod 32 so that the
// two row groups of a half-wave in the MFMA operand reads fall into disjoint banks.
constexpr int lds_row_stride(int w) { return w + (((16 - w % 32) % 32) + 32) % 32; }

constexpr int kNodeNBMax = 5;  // 16-column blocks per fused node workgroup (80 real columns: no spills)

// Row stride of the coupling block in LDS for a tile of FP functions: padded to 16 mod 32
// (lds_row_stride) unless that would keep two workgroups from sharing a CU's 160 KB of LDS;
// then the largest odd stride that fits (hs_cap, at least FP).
template <typename T, int NB>
constexpr int node_hs_cap(int fpmax) {
  const int budget = (80 * 1024 - 512) / (int)sizeof(T);  // elements per workgroup
  const int cap = (budget - kTileRows * lds_row_stride(NB * 16) - fpmax * (int)sizeof(int32_t) / (int)sizeof(T)) /
                  kTileRows;
  return (cap & 1) ? cap : cap - 1;
}
__host__ __device__ constexpr int node_hs(int fp, int hs_cap) {
  return lds_row_stride(fp) <= hs_cap || hs_cap < fp ? lds_row_stride(fp) : hs_cap;
}
template <typename T, int NB>
constexpr size_t node_lds_bytes(int fpmax) {
  return (size_t)kTileRows * (lds_row_stride(NB * 16) + node_hs(fpmax, node_hs_cap<T, NB>(fpmax))) * sizeof(T) +
         (size_t)fpmax * sizeof(int32_t);
}

template <typename T, int NB>
__global__ __launch_bounds__(256, NB == 4 ? 3 : 2) void fe_node_fused_kernel(KBatch<T> kb, int nc, int p, int n, int P1,
                                                               CellCoef<T> cf, const int32_t* __restrict__ tile_fptr,
                                                               const int32_t* __restrict__ tile_fns, int N, int ncb,
                                                               int hs_cap, int tm) {
  using M = Mfma<T>;
  using V4 = typename M::V4;
  constexpr int TR = kTileRows, CBW = NB * 16, XS = lds_row_stride(CBW);
  constexpr int XPT = TR * CBW / 256;  // staged elements per thread of one TR x CBW block
  extern __shared__ unsigned char smem_raw[];
  const KP<T>& P = kb.k[blockIdx.z];
  const int ncr = P.ncr;
  // launch order: the column blocks of a tile are consecutive in L, and each XCD (workgroups
  // bk = x mod 8) takes a contiguous range of L, so the column blocks that read the same
  // coupling block and x rows share one L2
  const int nbk = gridDim.x, bk = blockIdx.x, nb8 = nbk & ~7;
  const int L = bk < nb8 ? (bk & 7) * (nb8 >> 3) + (bk >> 3) : bk;
  const int t = L / ncb;
  const int cb0 = (L - t * ncb) * CBW;
  if (cb0 >= ncr) return;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int f0 = tile_fptr ? tile_fptr[t] : 0, FP = tile_fptr ? tile_fptr[t + 1] - f0 : 0;
  const int HS = node_hs(FP, hs_cap);
  T* xs = reinterpret_cast<T*>(smem_raw);  // [TR][XS]: x rows of the tile (zero past the mesh), later Z^O rows
  T* hs = xs + TR * XS;                     // [TR][HS]: the tile's block
  int32_t* fs = reinterpret_cast<int32_t*>(hs + __umul24(TR, HS));  // [FP]: enrichment function of each tile column
  const T* __restrict__ tv = P.tv + (int64_t)f0 * TR;  // [TR][FP]
  const T* __restrict__ zo = P.zo;                         // [n_enr][ncr]
  const T* __restrict__ x = P.x;
  const int64_t ldx = P.ldx;
  const int64_t ldc = P.ldc;
  T alpha, c, beta;
  step_scalars(P, alpha, c, beta);
  const T* prev = P.prev;  // may be the same array as out (each element is read before it is written)
  T* out = P.out;
  const int64_t ldo = P.ldo;
  const int S = nc * P1;
  // Global loads below are unconditional, from clamped in-bounds addresses, with
  // unwanted values replaced by selects, so that each batch is issued at once.
  int colc[NB];
  bool colok[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int col = cb0 + nb * 16 + li;
    colok[nb] = col < ncr;
    colc[nb] = colok[nb] ? col : ncr - 1;
  }
  // node-slot grid columns, not clamped: a row of the grid (ldc >= ncr; a multiple of 8, or 1) is
  // followed by the next row or by the grid's padding (one row plus 16 kNodeNBMax elements,
  // slot_grid_elems), so every column this block reads, below ncr + 16 NB, stays in the
  // allocation; values past ncr only reach lanes whose output is not stored.  The loads of a
  // row then differ by constant offsets.
  const T* __restrict__ Ycl = P.ycell + cb0 + li;

  // slots of node i per dimension: a shared node (i mod p == 0) has two, the one from
  // the lower cell first; slot 0 holds the periodic image of the last cell
  int bx[4], by[4], bz[4], gc[4];
  bool x2[4], y2[4], z2[4], ok[4];
  T msc[4];
  int tx0, ty0, tz0;  // the tile's first node (uniform)
  tile_origin(t, n, tm, tx0, ty0, tz0);
  // consecutive rows (mode 0): the node of the tile's first row (uniform), the others by stepping
  // along x from it, without a division per row
  int sx0 = 0, sy0 = 0, sz0 = 0;
  if (tm == 0) {
    sz0 = tx0 / (n * n);
    const int rem = tx0 - sz0 * n * n;
    sy0 = rem / n;
    sx0 = rem - sy0 * n;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = w * 16 + M::row(lane, v);
    int ix, iy, iz, gv;
    if (tm == 0) {
      gv = tx0 + r;
      ix = sx0 + r;
      iy = sy0;
      iz = sz0;
      while (ix >= n) {
        ix -= n;
        if (++iy == n) {
          iy = 0;
          ++iz;
        }
      }
      if (gv >= N) gv = -1, ix = iy = iz = 0;
    } else {
      gv = tile_row_coords(tx0, ty0, tz0, r, n, tm, ix, iy, iz);
    }
    ok[v] = gv >= 0;
    gc[v] = ok[v] ? gv : 0;
    const int qx = div_p(ix, p), rx = ix - qx * p, qy = div_p(iy, p), ry = iy - qy * p, qz = div_p(iz, p),
              rz = iz - qz * p;
    bx[v] = qx * P1 + (rx ? rx + 1 : 0);
    by[v] = qy * P1 + (ry ? ry + 1 : 0);
    bz[v] = qz * P1 + (rz ? rz + 1 : 0);
    x2[v] = rx == 0;
    y2[v] = ry == 0;
    z2[v] = rz == 0;
    msc[v] = cf.mscale * cf.om[rx] * cf.om[ry] * cf.om[rz];
  }
  // element offset of each row's first slot in the node-slot grid (one 64-bit product per
  // row); the other slots of a node lie S ldc (y) and S^2 ldc (z) further (and ldc in x)
  const int64_t Sl = (int64_t)S * ldc, S2l = Sl * S;
  int64_t yoff[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) yoff[v] = (bx[v] + (int64_t)S * (by[v] + (int64_t)S * bz[v])) * ldc;

  // ---- one batch of loads: the x tile, the first part of the H tile, the function list
  // and (real columns) the first slot pair of the gather, which lands during the
  // matrix-core phase below
  constexpr bool kEarly = sizeof(T) == 4;
  // the whole H tile in the first batch for up to 48 (float64) / 32 (float32: its registers
  // also hold the first gather loads) functions
  constexpr int HPT = sizeof(T) == 8 ? 12 : 8;
  const int nh = TR * FP;
  T gA[4][NB], gB[4][NB];
  // staging of a [TR][CBW] block: thread (tr, tc) = (threadIdx.x / 16, threadIdx.x % 16) takes
  // rows tr + 16 i (i < TR / 16) and columns tc + 16 j (j < NB), element i NB + j
  static_assert(TR == 64 && XPT == 4 * NB, "staging layout assumes 64-row tiles");
  const int tr = (int)threadIdx.x >> 4, tc = (int)threadIdx.x & 15;
  // tile rows past the mesh and columns past ncr are clamped for the loads (their values are
  // not used); the staging rows of this thread: tr + 16 i
  const int cmax = ncr - 1 - cb0;
  const T* xrow[4];
  bool rowok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gr = tile_row_node(tx0, ty0, tz0, tr + 16 * i, n, tm);
    rowok[i] = gr >= 0;
    xrow[i] = x + (int64_t)(rowok[i] ? gr : 0) * ldx + cb0;
  }
  // the H tile [TR][FP] on the same map, HJ 16-column groups per batch: rows tr + 16 i,
  // columns jc0 + tc + 16 j (past FP: clamped loads, no store)
  constexpr int HJ = HPT / 4;
  auto hload = [&](int jc0, T (&hv)[HPT]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ro = (int)__umul24((unsigned)(tr + 16 * i), (unsigned)FP);
#pragma unroll
      for (int j = 0; j < HJ; ++j) hv[i * HJ + j] = tv[min(ro + jc0 + tc + 16 * j, nh - 1)];
    }
  };
  auto hstore = [&](int jc0, const T (&hv)[HPT]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ro = (int)__umul24((unsigned)(tr + 16 * i), (unsigned)HS);
#pragma unroll
      for (int j = 0; j < HJ; ++j) {
        const int col = jc0 + tc + 16 * j;
        if (col < FP) hs[ro + col] = hv[i * HJ + j];
      }
    }
  };
  {
    T xv[XPT], hv[HPT];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < NB; ++j) xv[i * NB + j] = xrow[i][min(tc + 16 * j, cmax)];
    }
    if (FP > 0) hload(0, hv);
    const int32_t fv = (int)threadIdx.x < FP ? tile_fns[f0 + threadIdx.x] : 0;
    if constexpr (kEarly) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T* ya = Ycl + yoff[v];
        const T* yb = x2[v] ? ya + ldc : ya;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          gA[v][nb] = ya[nb * 16];
          gB[v][nb] = yb[nb * 16];
        }
      }
    }
    if ((int)threadIdx.x < FP) fs[threadIdx.x] = fv;
    for (int f = threadIdx.x + 256; f < FP; f += 256) fs[f] = tile_fns[f0 + f];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) xs[(tr + 16 * i) * XS + tc + 16 * j] = rowok[i] ? xv[i * NB + j] : T(0);
    if (FP > 0) hstore(0, hv);
  }
  // the rest of the H tile
  for (int jc0 = 16 * HJ; jc0 < FP; jc0 += 16 * HJ) {
    T hv[HPT];
    hload(jc0, hv);
    hstore(jc0, hv);
  }
  __syncthreads();

  // ---- part = Ht_t^* X_t from LDS: (function block mb, column block nb) pairs over the 4 waves
  if (FP > 0) {
    const int MB = (FP + 15) / 16;
    // two (mb, nb) blocks per wave at a time: independent accumulator chains
    for (int q0 = w; q0 < MB * NB; q0 += 8) {
      const bool two = q0 + 4 < MB * NB;
      int fcs[2], cls[2];
      bool foks[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = (h == 0 || two) ? q0 + 4 * h : q0;
        const int mb = q / NB, nb = q - mb * NB;
        const int f = mb * 16 + li;
        foks[h] = f < FP;
        fcs[h] = foks[h] ? f : FP - 1;
        cls[h] = nb * 16 + li;  // LDS column; past ncr it holds a duplicate, never stored
      }
      V4 pc[2] = {V4{0, 0, 0, 0}, V4{0, 0, 0, 0}};
#pragma unroll 4
      for (int ks = 0; ks < TR / 4; ++ks) {
        const int r = ks * 4 + lk;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const T av = hs[__umul24(r, HS) + fcs[h]];
          const T a = foks[h] ? av : T(0);
          pc[h] = M::op(a, xs[__umul24(r, XS) + cls[h]], pc[h]);
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && !two) break;
        const int q = q0 + 4 * h;
        const int mb = q / NB;
        const int col = cb0 + cls[h];
        if (col < ncr) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int fi = mb * 16 + M::row(lane, v);
            if (fi < FP) P.part[(int64_t)(f0 + fi) * ncr + col] = pc[h][v];
          }
        }
      }
    }
  }

  // ---- node-slot gather: sum over the (up to 8) cell results stored for the node
  T sum[4][NB];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) sum[v][nb] = 0;
  // masks as factors (the gathered values are finite): fma(v, 1, s) = v + s and fma(v, 0, s) = s
  // exactly, so the sums equal those of the selects, without the selects
  T m2[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) m2[v] = x2[v] ? T(1) : T(0);
  if constexpr (kEarly) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T mo = ok[v] ? T(1) : T(0);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) sum[v][nb] = fma(fma(gB[v][nb], m2[v], gA[v][nb]), mo, sum[v][nb]);
    }
  }
  // (ky, kz) slot pairs in a fixed order; a pair is visited when some lane of the
  // wave needs it, lanes that do not need it reload their first slot (in bounds,
  // cached) and discard it
#pragma unroll
  for (int kk = kEarly ? 1 : 0; kk < 4; ++kk) {
    const int ky = kk & 1, kz = kk >> 1;
    bool need[4];
    int anyv = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      need[v] = ok[v] && (ky == 0 || y2[v]) && (kz == 0 || z2[v]);
      anyv |= need[v];
    }
    if (kk > 0 && !__any(anyv)) continue;
    const int64_t kofs = ky * Sl + kz * S2l;  // slot offset of the pair (uniform)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T* ya = Ycl + yoff[v] + (need[v] ? kofs : 0);
      const T* yb = x2[v] ? ya + ldc : ya;
      const T mn = need[v] ? T(1) : T(0);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const T v0 = ya[nb * 16];
        const T v1 = yb[nb * 16];
        sum[v][nb] = fma(fma(v1, m2[v], v0), mn, sum[v][nb]);
      }
    }
  }

  // ---- acc = m^-1/2 sum - c x on the MFMA result layout, then acc += Ht_t Z^O
  V4 acc[NB];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rl = w * 16 + M::row(lane, v);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb][v] = msc[v] * sum[v][nb] - c * xs[__umul24(rl, XS) + nb * 16 + li];
  }
  // the previous iterate is read here, before any element of out is written
  T pv[4][NB];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const T* pr = prev + (int64_t)gc[v] * ldo;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) pv[v][nb] = beta != T(0) ? pr[colc[nb]] : T(0);
  }

  // Z^O rows of the tile's functions, in chunks of TR rows staged over the x tile
  const int rA = w * 16 + li;
  for (int fc0 = 0; fc0 < FP; fc0 += TR) {
    const int FC = min(TR, FP - fc0);  // a multiple of 4, as FP is
    __syncthreads();                   // the x tile (or the previous chunk) is no longer read
    {
      T zv[XPT];
      int fnv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = tr + 16 * i;
        fnv[i] = r < FC ? fs[fc0 + r] : -1;
        const unsigned ro = __umul24((unsigned)max(fnv[i], 0), (unsigned)ncr) + (unsigned)cb0;
#pragma unroll
        for (int j = 0; j < NB; ++j) zv[i * NB + j] = zo[ro + (unsigned)min(tc + 16 * j, cmax)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) xs[(tr + 16 * i) * XS + tc + 16 * j] = fnv[i] >= 0 ? zv[i * NB + j] : T(0);
    }
    __syncthreads();
#pragma unroll 2
    for (int k0 = 0; k0 < FC; k0 += 4) {
      const int f = k0 + lk;
      const T a = hs[__umul24(rA, HS) + fc0 + f];
      T b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = xs[__umul24(f, XS) + nb * 16 + li];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = M::op(a, b[nb], acc[nb]);
    }
  }

  // ---- out = alpha acc - beta prev
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T* orow = out + (int64_t)gc[v] * ldo;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      T r = alpha * acc[nb][v];
      if (beta != T(0)) r -= beta * pv[v][nb];
      if (ok[v] && colok[nb]) orow[colc[nb]] = r;
    }
  }
}

// Node stage of real operators at one column (the auxiliary-potential conjugate gradients,
// Lanczos): one wave per coupling tile, lane = tile row, no LDS.  The slot gather takes the
// same slots in the same order as fe_node_fused_kernel; the tile's coupling row is applied with
// one product per function in list order, and each function's partial of H^co* x is a fixed
// butterfly over the 64 rows.  Launched when every operator of the step has one column and the
// tiles couple to at most kCol1MaxFunctions functions (per-function butterflies cost more than
// the matrix-core products beyond that).
constexpr int kCol1MaxFunctions = 24;  // functions per tile up to which one column takes fe_node_col1_kernel
template <typename T>
__global__ __launch_bounds__(256) void fe_node_col1_kernel(KBatch<T> kb, int nc, int p, int n, int P1, CellCoef<T> cf,
                                                           const int32_t* __restrict__ tile_fptr,
                                                           const int32_t* __restrict__ tile_fns, int ntiles, int tm) {
  constexpr int TR = kTileRows;
  const KP<T>& P = kb.k[blockIdx.z];
  const int t = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform per wave
  if (t >= ntiles) return;  // the whole wave
  const int r = (int)threadIdx.x & 63;
  int x0, y0, z0, ix, iy, iz;
  tile_origin(t, n, tm, x0, y0, z0);
  const int gv = tile_row_coords(x0, y0, z0, r, n, tm, ix, iy, iz);
  const bool ok = gv >= 0;
  const int g = ok ? gv : 0;
  T alpha, c, beta;
  step_scalars(P, alpha, c, beta);
  const T xv = ok ? P.x[(int64_t)g * P.ldx] : T(0);
  const T pv = beta != T(0) ? P.prev[(int64_t)g * P.ldo] : T(0);
  // slots of the node: (bx + {0, x2}) x (by + {0, y2}) x (bz + {0, z2}), as in the fused kernel
  const int qx = div_p(ix, p), rx = ix - qx * p, qy = div_p(iy, p), ry = iy - qy * p, qz = div_p(iz, p),
            rz = iz - qz * p;
  const int bx = qx * P1 + (rx ? rx + 1 : 0), by = qy * P1 + (ry ? ry + 1 : 0), bz = qz * P1 + (rz ? rz + 1 : 0);
  const bool x2 = rx == 0, y2 = ry == 0, z2 = rz == 0;
  const T msc = cf.mscale * cf.om[rx] * cf.om[ry] * cf.om[rz];
  const int S = nc * P1;
  const int64_t ldc = P.ldc, Sl = (int64_t)S * ldc, S2l = Sl * S;
  const T* __restrict__ Y0 = P.ycell + (bx + (int64_t)S * (by + (int64_t)S * bz)) * ldc;
  const T m2 = x2 ? T(1) : T(0);
  T sum = 0;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int ky = kk & 1, kz = kk >> 1;
    const bool need = ok && (ky == 0 || y2) && (kz == 0 || z2);
    const T* ya = Y0 + (need ? ky * Sl + kz * S2l : 0);
    const T* yb = x2 ? ya + ldc : ya;
    const T mn = need ? T(1) : T(0);
    sum = fma(fma(yb[0], m2, ya[0]), mn, sum);
  }
  T acc = msc * sum - c * xv;
  if (tile_fptr) {
    const int f0 = tile_fptr[t], FP = tile_fptr[t + 1] - f0;  // a multiple of 4 (padded list)
    const T* __restrict__ tv = P.tv + (int64_t)f0 * TR + (int64_t)r * FP;  // this row of the [TR][FP] block
    // four functions at a time: their loads issued together, their butterflies interleaved
    for (int fb = 0; fb < FP; fb += 4) {
      T h[4], z[4], q[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // padding entries of the list hold -1 (and zero coupling values): Z^O row 0, replaced by 0
        const int fn = tile_fns[f0 + fb + i];
        h[i] = tv[fb + i];
        const T zl = P.zo[(int64_t)max(fn, 0) * P.ncr];
        z[i] = fn >= 0 ? zl : T(0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc = fma(h[i], z[i], acc);
        q[i] = h[i] * xv;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] += __shfl_xor(q[i], o);
      if (r == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) P.part[(int64_t)(f0 + fb + i) * P.ncr] = q[i];
      }
    }
  }
  if (ok) {
    T o = alpha * acc;
    if (beta != T(0)) o -= beta * pv;
    P.out[(int64_t)g * P.ldo] = o;
  }
}

// First fold of the tile partials: part2[nu][ch][j] = sum of the partials of function
// nu with list positions in chunk ch (kReduceChunk entries), in list order within
// 4 interleaved groups and a fixed 4-way tree.  Chunks past the list hold 0.
constexpr int kReduceChunk = 64;

template <typename T>
__global__ __launch_bounds__(256) void enr_reduce1_kernel(KBatch<T> kb, int nch, const int32_t* __restrict__ fn_pptr,
                                                          const int32_t* __restrict__ fn_poff) {
  __shared__ T red[4][64];
  const KP<T>& P = kb.k[blockIdx.z];
  const int ncr = P.ncr;
  if ((int)blockIdx.y * 64 >= ncr) return;
  const T* __restrict__ part = P.part;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int nu = blockIdx.x / nch, ch = blockIdx.x - nu * nch;
  const int j = blockIdx.y * 64 + lane;
  const int e1 = fn_pptr[nu + 1];
  const int es = fn_pptr[nu] + ch * kReduceChunk, ee = min(e1, es + kReduceChunk);
  // this wave's entries es + grp + 4 i, all loads issued at once; summed as two
  // interleaved chains (even i, odd i) in list order
  constexpr int EPG = kReduceChunk / 4;
  const int eg = __builtin_amdgcn_readfirstlane(es + grp);
  T v[EPG];
  if (ee > es) {
    const int jc = min(j, ncr - 1);
#pragma unroll
    for (int i = 0; i < EPG; ++i) {
      const int e = eg + 4 * i;
      const T pv = part[(int64_t)fn_poff[min(e, ee - 1)] * ncr + jc];  // clamped in-bounds entry
      // a multiply by 1 or 0 (not a select, which the compiler would turn into a branch
      // around the load) keeps all loads of the batch in flight together
      v[i] = pv * ((e < ee && j < ncr) ? T(1) : T(0));
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPG; ++i) v[i] = T(0);
  }
  T s0 = 0, s1 = 0;
#pragma unroll
  for (int i = 0; i < EPG; i += 2) {
    s0 += v[i];
    s1 += v[i + 1];
  }
  red[grp][lane] = s0 + s1;
  __syncthreads();
  if (grp == 0 && j < ncr)
    P.part2[((int64_t)nu * nch + ch) * ncr + j] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Small dense products on the enrichment rows (n = n_enr; complex interleaved when
// CPLX), 16x16 output tile per workgroup, LDS-staged K tiles.
//   mode 0: zo = S x^O       mode 1: wp = (sum of the folded tile partials) + H^oo zo
//   mode 2: out^O = alpha (S wp - c x^O) - beta prev^O
//   mode 3: zo = S out^O      (Z^O of the next recurrence step)
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void small_gemm_kernel(KBatch<T> kb, int mode, int64_t N, int n) {
  constexpr int E = CPLX ? 2 : 1;
  constexpr int TS = 16;
  __shared__ T As[TS][TS * E + 1];
  __shared__ T Bs[TS][TS * E + 1];
  const KP<T>& P = kb.k[blockIdx.z];
  const int m = P.nv;
  if ((int)blockIdx.x * TS >= m) return;
  const int k = n;
  const T* __restrict__ A = mode == 1 ? P.Hoo : P.S;
  const T* __restrict__ B = mode == 0 ? P.x + N * P.ldx
                           : mode == 3 ? P.out + N * P.ldo
                                       : (mode == 1 ? P.zo : P.wp);
  const int64_t ldb = mode == 0 ? P.ldx : mode == 3 ? P.ldo : (int64_t)P.ncr;
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  const int i = blockIdx.y * TS + ty;   // row
  const int jc = blockIdx.x * TS + tx;  // column (complex element)
  T sr = 0, si = 0;
  for (int k0 = 0; k0 < k; k0 += TS) {
    for (int e = 0; e < E; ++e) {
      const int ka = k0 + tx, kr = k0 + ty;
      As[ty][tx * E + e] = (i < n && ka < k) ? A[((int64_t)i * k + ka) * E + e] : T(0);
      Bs[ty][tx * E + e] = (kr < k && jc < m) ? B[(int64_t)kr * ldb + (int64_t)jc * E + e] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TS; ++kk) {
      if constexpr (!CPLX) {
        sr += As[ty][kk] * Bs[kk][tx];
      } else {
        const C2<T> t = cmul(C2<T>{As[ty][2 * kk], As[ty][2 * kk + 1]}, C2<T>{Bs[kk][2 * tx], Bs[kk][2 * tx + 1]});
        sr += t.r;
        si += t.i;
      }
    }
    __syncthreads();
  }
  if (i >= n || jc >= m) return;
  if (mode == 0 || mode == 3) {
    P.zo[(int64_t)i * P.ncr + (int64_t)jc * E] = sr;
    if (CPLX) P.zo[(int64_t)i * P.ncr + (int64_t)jc * E + 1] = si;
  } else if (mode == 1) {
    const T* p2 = P.part2 + (int64_t)i * P.nch * P.ncr + (int64_t)jc * E;
    T wr = 0, wi = 0;
    for (int ch = 0; ch < P.nch; ++ch) {
      wr += p2[(int64_t)ch * P.ncr];
      if (CPLX) wi += p2[(int64_t)ch * P.ncr + 1];
    }
    P.wp[(int64_t)i * P.ncr + (int64_t)jc * E] = wr + sr;
    if (CPLX) P.wp[(int64_t)i * P.ncr + (int64_t)jc * E + 1] = wi + si;
  } else {
    const int64_t ox = (N + i) * P.ldx + (int64_t)jc * E, oo = (N + i) * P.ldo + (int64_t)jc * E;
    T alpha, cst, beta;
    step_scalars(P, alpha, cst, beta);
    T r = alpha * (sr - cst * P.x[ox]);
    if (beta != T(0)) r -= beta * P.prev[oo];
    P.out[oo] = r;
    if (CPLX) {
      T r2 = alpha * (si - cst * P.x[ox + 1]);
      if (beta != T(0)) r2 -= beta * P.prev[oo + 1];
      P.out[oo + 1] = r2;
    }
  }
}

// The three products of small_gemm modes 1, 2 and 3 in one launch: every product is
// (n x n) times (n x columns), so one workgroup per block of kChainCols columns computes
//   W' = (sum of the folded tile partials) + H^oo Z^O,
//   out^O = alpha (S W' - c x^O) - beta prev^O,
//   Z^O of the next step = S out^O (when next),
// with S, H^oo and the block's Z^O, W' and out^O in LDS (1024 threads: one output of a phase
// per thread for n kChainCols <= 1024).  Sums run in the same order as in
// small_gemm (chunk partials first, then the products in k order); the chunk partials are
// loaded in batches of 8.
constexpr int kChainCols = 16;

template <typename T, bool CPLX>
constexpr size_t enr_chain_lds_bytes(int n) {
  return (2 * (size_t)n * n + 3 * (size_t)n * kChainCols) * (CPLX ? 2 : 1) * sizeof(T);
}

template <typename T, bool CPLX>
__global__ __launch_bounds__(1024) void enr_chain_kernel(KBatch<T> kb, int64_t N, int n, int next) {
  constexpr int E = CPLX ? 2 : 1, TC = kChainCols;
  extern __shared__ unsigned char chain_raw[];
  T* Ss = reinterpret_cast<T*>(chain_raw);  // [n][n] S
  T* Hs = Ss + (size_t)n * n * E;           // [n][n] H^oo
  T* Zs = Hs + (size_t)n * n * E;           // [n][TC] Z^O of this step
  T* Ws = Zs + (size_t)n * TC * E;          // [n][TC] W'
  T* Os = Ws + (size_t)n * TC * E;          // [n][TC] out^O
  const KP<T>& P = kb.k[blockIdx.z];
  const int m = P.nv, ncr = P.ncr;
  const int j0 = blockIdx.x * TC;
  if (j0 >= m) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int t = tid; t < n * n * E; t += nth) {
    Ss[t] = P.S[t];
    Hs[t] = P.Hoo[t];
  }
  for (int t = tid; t < n * TC; t += nth) {
    const int i = t / TC, jl = t - i * TC, j = min(j0 + jl, m - 1);
#pragma unroll
    for (int e = 0; e < E; ++e) Zs[(size_t)t * E + e] = P.zo[(int64_t)i * ncr + (int64_t)j * E + e];
  }
  __syncthreads();
  // sum_k A[i][k] B[k][jl] over LDS tiles, in k order
  auto dot = [&](const T* A, const T* B, int i, int jl, T& sr, T& si) {
    sr = 0;
    si = 0;
#pragma unroll 8
    for (int k = 0; k < n; ++k) {
      const T* a = A + ((size_t)i * n + k) * E;
      const T* b = B + ((size_t)k * TC + jl) * E;
      if constexpr (!CPLX) {
        sr += a[0] * b[0];
      } else {
        const C2<T> q = cmul(C2<T>{a[0], a[1]}, C2<T>{b[0], b[1]});
        sr += q.r;
        si += q.i;
      }
    }
  };
  // W'
  if (m == 1) {
    // one column: the TC threads of a row, which would all compute the same entry, split its
    // chunks (thread jl adds chunks jl, jl + TC, ... in order) into Os, then add them in order
    for (int t = tid; t < n * TC; t += nth) {
      const int i = t / TC, jl = t - i * TC;
      const T* p2 = P.part2 + (int64_t)i * P.nch * ncr;
      T wr = 0, wi = 0;
      for (int ch = jl; ch < P.nch; ch += TC) {
        wr += p2[(int64_t)ch * ncr];
        if (CPLX) wi += p2[(int64_t)ch * ncr + 1];
      }
      Os[(size_t)t * E] = wr;
      if (CPLX) Os[(size_t)t * E + 1] = wi;
    }
    __syncthreads();
    for (int t = tid; t < n * TC; t += nth) {
      const int i = t / TC, jl = t - i * TC;
      T wr = 0, wi = 0;
      for (int q = 0; q < TC; ++q) {
        wr += Os[((size_t)i * TC + q) * E];
        if (CPLX) wi += Os[((size_t)i * TC + q) * E + 1];
      }
      T sr, si;
      dot(Hs, Zs, i, jl, sr, si);
      Ws[(size_t)t * E] = wr + sr;
      if (CPLX) Ws[(size_t)t * E + 1] = wi + si;
    }
  } else {
  for (int t = tid; t < n * TC; t += nth) {
    const int i = t / TC, jl = t - i * TC, j = min(j0 + jl, m - 1);
    const T* p2 = P.part2 + (int64_t)i * P.nch * ncr + (int64_t)j * E;
    T wr = 0, wi = 0;
    int ch = 0;
    for (; ch + 8 <= P.nch; ch += 8) {
      T vr[8], vi[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        vr[q] = p2[(int64_t)(ch + q) * ncr];
        vi[q] = CPLX ? p2[(int64_t)(ch + q) * ncr + 1] : T(0);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        wr += vr[q];
        if (CPLX) wi += vi[q];
      }
    }
    for (; ch < P.nch; ++ch) {
      wr += p2[(int64_t)ch * ncr];
      if (CPLX) wi += p2[(int64_t)ch * ncr + 1];
    }
    T sr, si;
    dot(Hs, Zs, i, jl, sr, si);
    Ws[(size_t)t * E] = wr + sr;
    if (CPLX) Ws[(size_t)t * E + 1] = wi + si;
  }
  }
  __syncthreads();
  // out^O
  for (int t = tid; t < n * TC; t += nth) {
    const int i = t / TC, jl = t - i * TC, j = j0 + jl;
    T sr, si;
    dot(Ss, Ws, i, jl, sr, si);
    const int64_t ox = (N + i) * P.ldx + (int64_t)min(j, m - 1) * E, oo = (N + i) * P.ldo + (int64_t)min(j, m - 1) * E;
    T alpha, cst, beta;
    step_scalars(P, alpha, cst, beta);
    T r = alpha * (sr - cst * P.x[ox]);
    if (beta != T(0)) r -= beta * P.prev[oo];
    T r2 = 0;
    if (CPLX) {
      r2 = alpha * (si - cst * P.x[ox + 1]);
      if (beta != T(0)) r2 -= beta * P.prev[oo + 1];
    }
    Os[(size_t)t * E] = r;
    if (CPLX) Os[(size_t)t * E + 1] = r2;
    if (j < m) {
      P.out[oo] = r;
      if (CPLX) P.out[oo + 1] = r2;
    }
  }
  if (!next) return;
  __syncthreads();
  // Z^O of the next step
  for (int t = tid; t < n * TC; t += nth) {
    const int i = t / TC, jl = t - i * TC, j = j0 + jl;
    T sr, si;
    dot(Ss, Os, i, jl, sr, si);
    if (j < m) {
      P.zo[(int64_t)i * ncr + (int64_t)j * E] = sr;
      if (CPLX) P.zo[(int64_t)i * ncr + (int64_t)j * E + 1] = si;
    }
  }
}

// diagonal test operator: out = alpha (lambda x - c x) - beta prev
template <typename T>
__global__ void diag_step_kernel(const T* __restrict__ lam, const T* __restrict__ x, const T* __restrict__ prev,
                                 T* __restrict__ out, int64_t ldx, int64_t ldo, int nv, int64_t N, T alpha, T c,
                                 T beta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nv) return;
  const int64_t g = idx / nv;
  const int vv = (int)(idx % nv);
  const int64_t o = g * ldx + vv;
  const int64_t oo = g * ldo + vv;
  T r = alpha * (lam[g] * x[o] - c * x[o]);
  if (beta != T(0)) r -= beta * prev[oo];
  out[oo] = r;
}

// ---------------------------------------------------------------------------
// Density at the quadrature points for the potential gradient:
//   dens[blk][e][q] = sum over the 64 real columns of this block of f_v psi_col(x_eq)^2,
//   psi = B (m^-1/2 theta o x)|_e + sum_nu N^O_nu(x_eq) (S x^O)_nu.
// Same plane layout as fe_cell_kernel (one cell x 64 real columns per workgroup).
// ---------------------------------------------------------------------------
template <typename T, int P1, bool CPLX>
__global__ __launch_bounds__(64 * P1) void density_kernel(
    const T* __restrict__ X, int64_t ldx, int ncr, const double* __restrict__ fw, const T* __restrict__ zo,
    CellCoef<T> cf, int nc, int p, int n, Phase3<T> ph, const int64_t* __restrict__ cph_ptr,
    const int32_t* __restrict__ cph_blk, const int64_t* __restrict__ cph_off, const int32_t* __restrict__ blk_fn0,
    const int32_t* __restrict__ blk_nf, const double* __restrict__ phi, int FMAX, int n_enr,
    double* __restrict__ dens, int64_t n_cells) {
  constexpr int NP = P1 * P1;
  constexpr int NQ = NP * P1;
  __shared__ T lds[NQ][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t e = blockIdx.x;
  const int j = blockIdx.y * 64 + lane;
  const bool valid = j < ncr;
  const int cx = (int)(e % nc), cy = (int)((e / nc) % nc), cz = (int)(e / ((int64_t)nc * nc));
  T v[NP], t[NP];
  {
    const int az = w;
    int iz = cz * p + az;
    const bool wz = iz >= n;
    if (wz) iz -= n;
#pragma unroll
    for (int ay = 0; ay < P1; ++ay) {
      int iy = cy * p + ay;
      const bool wy = iy >= n;
      if (wy) iy -= n;
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) {
        int ix = cx * p + ax;
        const bool wx = ix >= n;
        if (wx) ix -= n;
        const int64_t g = ix + (int64_t)n * (iy + (int64_t)n * iz);
        T val = 0;
        if (valid) {
          if constexpr (!CPLX) {
            val = X[g * ldx + j];
          } else {
            const T* px = X + g * ldx + (j & ~1);
            C2<T> z{px[0], px[1]};
            if (wx) z = cmul(z, C2<T>{ph.re[0], ph.im[0]});
            if (wy) z = cmul(z, C2<T>{ph.re[1], ph.im[1]});
            if (wz) z = cmul(z, C2<T>{ph.re[2], ph.im[2]});
            val = (j & 1) ? z.i : z.r;
          }
        }
        v[ay * P1 + ax] = cf.mscale * cf.om[ax] * cf.om[ay] * cf.om[az] * val;
      }
    }
  }
#pragma unroll
  for (int ay = 0; ay < P1; ++ay)
#pragma unroll
    for (int qx = 0; qx < P1; ++qx) {
      T s = 0;
#pragma unroll
      for (int ax = 0; ax < P1; ++ax) s += cf.B1[qx][ax] * v[ay * P1 + ax];
      t[ay * P1 + qx] = s;
    }
#pragma unroll
  for (int qy = 0; qy < P1; ++qy)
#pragma unroll
    for (int qx = 0; qx < P1; ++qx) {
      T s = 0;
#pragma unroll
      for (int ay = 0; ay < P1; ++ay) s += cf.B1[qy][ay] * t[ay * P1 + qx];
      lds[(w * P1 + qy) * P1 + qx][lane] = s;
    }
  __syncthreads();
#pragma unroll
  for (int az = 0; az < P1; ++az)
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) t[az * P1 + qy] = lds[(az * P1 + qy) * P1 + w][lane];
  const int qx = w;
  double psi[NP];
#pragma unroll
  for (int qz = 0; qz < P1; ++qz)
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) {
      T s = 0;
#pragma unroll
      for (int az = 0; az < P1; ++az) s += cf.B1[qz][az] * t[az * P1 + qy];
      psi[qz * P1 + qy] = (double)s;
    }
  // enrichment part: the support blocks of the cell in turn; a block's values at the cell's points
  // (all its functions) are staged in LDS by the whole workgroup, double-buffered: the next
  // block's values and Z^O entries are loaded while this block's are summed; the sums run in the
  // same order as one function after the other
  {
    constexpr int E = CPLX ? 2 : 1;
    constexpr int kFn = 8;                                     // enrichment functions per atom at most
    constexpr int kPer = (NQ * kFn * E + 64 * P1 - 1) / (64 * P1);  // staged values per thread at most
    // two buffers of NQ FMAX E doubles: 2 x 125 x 8 x 2 x 8 B <= NQ x 64 x sizeof(T) for float and double
    double* stg = reinterpret_cast<double*>(&lds[0][0]);
    const int64_t k0 = cph_ptr[e], k1 = cph_ptr[e + 1];
    const int cnt = NQ * FMAX * E, nth = 64 * P1, tid = (int)threadIdx.x;
    double pre[kPer], zr[kFn], zi[kFn], zrn[kFn], zin[kFn];
    int fn_next0 = 0, nf_next = 0;
    auto fetch = [&](int64_t k) {  // block k's values into pre[], its Z^O entries into zrn / zin
      const int b = cph_blk[k];
      const int64_t off = cph_off[k];
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int idx = tid + i * nth;
        pre[i] = idx < cnt ? phi[off * cnt + idx] : 0.0;
      }
      fn_next0 = blk_fn0[b];
      nf_next = blk_nf[b];
#pragma unroll
      for (int f = 0; f < kFn; ++f) {
        zrn[f] = zin[f] = 0.0;
        if (valid && f < nf_next) {
          if constexpr (!CPLX) {
            zrn[f] = (double)zo[(int64_t)(fn_next0 + f) * ncr + j];
          } else {
            zrn[f] = (double)zo[(int64_t)(fn_next0 + f) * ncr + (j & ~1)];
            zin[f] = (double)zo[(int64_t)(fn_next0 + f) * ncr + (j & ~1) + 1];
          }
        }
      }
    };
    auto park = [&](double* buf) {
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int idx = tid + i * nth;
        if (idx < cnt) buf[idx] = pre[i];
      }
    };
    if (k0 < k1) fetch(k0);
    __syncthreads();  // the transpose is no longer read
    if (k0 < k1) park(stg);
    for (int64_t k = k0; k < k1; ++k) {
      double* cur = stg + ((k - k0) & 1) * cnt;
      const int nf = nf_next;
#pragma unroll
      for (int f = 0; f < kFn; ++f) {
        zr[f] = zrn[f];
        zi[f] = zin[f];
      }
      __syncthreads();  // block k's values parked; the other buffer (block k - 1) no longer read
      if (k + 1 < k1) fetch(k + 1);
      if (valid) {
#pragma unroll
        for (int f = 0; f < kFn; ++f) {
          if (f >= nf) break;
          if constexpr (!CPLX) {
            const double z = zr[f];
#pragma unroll
            for (int qz = 0; qz < P1; ++qz)
#pragma unroll
              for (int qy = 0; qy < P1; ++qy) {
                const int q = (qz * P1 + qy) * P1 + qx;
                psi[qz * P1 + qy] += cur[q * FMAX + f] * z;
              }
          } else {
#pragma unroll
            for (int qz = 0; qz < P1; ++qz)
#pragma unroll
              for (int qy = 0; qy < P1; ++qy) {
                const int q = (qz * P1 + qy) * P1 + qx;
                const double pr = cur[2 * (q * FMAX + f)];
                const double pi = cur[2 * (q * FMAX + f) + 1];
                psi[qz * P1 + qy] += (j & 1) ? (pr * zi[f] + pi * zr[f]) : (pr * zr[f] - pi * zi[f]);
              }
          }
        }
      }
      if (k + 1 < k1) park(stg + ((k + 1 - k0) & 1) * cnt);
    }
  }
  const double fv = valid ? fw[CPLX ? (j >> 1) : j] : 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    double s = valid ? fv * psi[k] * psi[k] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    psi[k] = s;
  }
  if (lane == 0) {
    double* out = dens + ((int64_t)blockIdx.y * n_cells + e) * NQ;
#pragma unroll
    for (int qz = 0; qz < P1; ++qz)
#pragma unroll
      for (int qy = 0; qy < P1; ++qy) out[(qz * P1 + qy) * P1 + qx] = psi[qz * P1 + qy];
  }
}

struct GW {
  double w[8];
};
// mode 0: out = W s (the potential gradient); 1: out = s (the density); 2: out += s
__global__ void density_final_kernel2(const double* __restrict__ dens, int nblk, int64_t total, int P1, GW gw,
                                      double h3, double* __restrict__ out, int mode) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int nq = P1 * P1 * P1;
  const int q = (int)(t % nq);
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += dens[(int64_t)b * total + t];
  if (mode == 0) {
    const double W = h3 * gw.w[q % P1] * gw.w[(q / P1) % P1] * gw.w[q / (P1 * P1)];
    out[t] = W * s;
  } else if (mode == 1) {
    out[t] = s;
  } else {
    out[t] += s;
  }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T>
const CellCoef<T>& coef(const oefe_op_s* op);
template <>
const CellCoef<double>& coef<double>(const oefe_op_s* op) { return op->cd; }
template <>
const CellCoef<float>& coef<float>(const oefe_op_s* op) { return op->cf; }

template <typename T>
struct DevPtrs {
  const T *WV, *S, *Hoo, *lambda, *tv;
};
template <typename T>
DevPtrs<T> devptrs(const oefe_op_s* op);
template <>
DevPtrs<double> devptrs<double>(const oefe_op_s* op) {
  return {op->d.WV, op->d.S, op->d.Hoo, op->d.lambda, op->d.tile_val};
}
template <>
DevPtrs<float> devptrs<float>(const oefe_op_s* op) {
  return {op->d.WVf, op->d.Sf, op->d.Hoof, op->d.lambdaf, op->d.tile_valf};
}

template <typename T, int P1, int CW, bool CPLX>
void launch_cell_cw(const oefe_op_s* op, const KBatch<T>& kb, int max_ncr, hipStream_t s) {
  constexpr int CPT = 64 / CW;
  dim3 grid((unsigned)cdiv(op->n_cells, CPT), (unsigned)cdiv(max_ncr, CW), (unsigned)kb.nk);
  hipLaunchKernelGGL((fe_cell_kernel<T, P1, CW, CPLX>), grid, dim3(64 * P1), 0, s, kb, coef<T>(op), op->nc, op->p,
                     op->n, op->n_cells);
}

template <typename T, int P1, bool CPLX>
void launch_cell_p(const oefe_op_s* op, const KBatch<T>& kb, int max_ncr, int cw, hipStream_t s) {
  switch (cw) {
    case 64: launch_cell_cw<T, P1, 64, CPLX>(op, kb, max_ncr, s); break;
    case 32: launch_cell_cw<T, P1, 32, CPLX>(op, kb, max_ncr, s); break;
    case 16: launch_cell_cw<T, P1, 16, CPLX>(op, kb, max_ncr, s); break;
    default: launch_cell_cw<T, P1, 8, CPLX>(op, kb, max_ncr, s); break;
  }
}

template <typename T, int P1, bool CPLX>
void launch_cell_lanes(const oefe_op_s* op, const KBatch<T>& kb, int max_ncr, hipStream_t s) {
  constexpr int CWc = lanes_cw<P1>();
  const int nch = (int)cdiv(max_ncr, CWc);
  dim3 grid((unsigned)(cdiv(op->n_cells, 4) * nch), 1, (unsigned)kb.nk);
  if constexpr (CPLX) {
    if (op->uform) {  // the operators of a batch share the form (checked by the batched entry points)
      hipLaunchKernelGGL((fe_cell_lanes_kernel<T, P1, true, true>), grid, dim3(256), 0, s, kb, coef<T>(op), op->nc,
                         op->p, op->n, op->n_cells, nch);
      return;
    }
  }
  hipLaunchKernelGGL((fe_cell_lanes_kernel<T, P1, CPLX>), grid, dim3(256), 0, s, kb, coef<T>(op), op->nc, op->p, op->n,
                     op->n_cells, nch);
}

// The planes-in-lanes kernel forms row offsets within a z-plane of X and of the node-slot
// grid in 32 bits from 24-bit products: n^2 ldx and S^2 ldc below 2^31 (S = nc (p+1)).
template <typename T>
bool lanes_offsets_fit(const oefe_op_s* op, const KBatch<T>& kb) {
  const int64_t S = (int64_t)op->nc * op->P1, n = op->n;
  for (int q = 0; q < kb.nk; ++q) {
    const int64_t ldx = kb.k[q].ldx, ldc = kb.k[q].ldc;
    if (ldx * n * n >= (int64_t(1) << 31) || ldc * S * S >= (int64_t(1) << 31)) return false;
  }
  return true;
}

// cw = 0: planes-in-lanes kernel; 8, 16, 32, 64: plane-per-wave kernel with cw columns per cell
template <typename T, int P1>
void launch_cell_cells(const oefe_op_s* op, const KBatch<T>& kb, hipStream_t s) {
  constexpr int CWc = lanes_cw<P1>();
  hipLaunchKernelGGL((fe_cell_cells_kernel<T, P1>), dim3((unsigned)cdiv(op->n_cells, 4 * CWc), 1, (unsigned)kb.nk),
                     dim3(256), 0, s, kb, coef<T>(op), op->nc, op->p, op->n, op->n_cells);
}

template <typename T, bool CPLX>
void launch_cell(const oefe_op_s* op, const KBatch<T>& kb, int max_ncr, int cw, hipStream_t s) {
  if constexpr (!CPLX) {
    if (max_ncr == 1) {  // one real column: cells in the lanes, whatever the tuned shape
      switch (op->P1) {
        case 3: launch_cell_cells<T, 3>(op, kb, s); break;
        case 4: launch_cell_cells<T, 4>(op, kb, s); break;
        default: launch_cell_cells<T, 5>(op, kb, s); break;
      }
      return;
    }
  }
  if (op->uform) {
    // only the planes-in-lanes kernel carries the periodic-function form's first-derivative
    // term; oefe_op_create_uform checks that its 32-bit offsets fit the mesh
    cw = 0;
  } else if (cw == 0 && !lanes_offsets_fit(op, kb)) {
    cw = 16;
  }
  if (cw == 0) {
    switch (op->P1) {
      case 3: launch_cell_lanes<T, 3, CPLX>(op, kb, max_ncr, s); break;
      case 4: launch_cell_lanes<T, 4, CPLX>(op, kb, max_ncr, s); break;
      default: launch_cell_lanes<T, 5, CPLX>(op, kb, max_ncr, s); break;
    }
    return;
  }
  switch (op->P1) {
    case 3: launch_cell_p<T, 3, CPLX>(op, kb, max_ncr, cw, s); break;
    case 4: launch_cell_p<T, 4, CPLX>(op, kb, max_ncr, cw, s); break;
    default: launch_cell_p<T, 5, CPLX>(op, kb, max_ncr, cw, s); break;
  }
}

template <typename T, int NBW, bool CPLX>
void launch_coupling_w(const oefe_op_s* op, const KBatch<T>& kb, hipStream_t s) {
  const size_t lds = coupling_lds_bytes<T, CPLX>(op->tile_fpmax);
  if (allow_dynamic_lds(reinterpret_cast<const void*>(&fe_coupling_kernel<T, NBW, CPLX>), lds) != hipSuccess) return;
  hipLaunchKernelGGL((fe_coupling_kernel<T, NBW, CPLX>), dim3((unsigned)op->n_tiles, 1, (unsigned)kb.nk), dim3(256),
                     lds, s, kb, op->d.tile_fptr, op->d.tile_fns, op->n, op->tile_mode);
}

// nbw: 16-column blocks per coupling wave (1 or 2)
template <typename T, bool CPLX>
void launch_coupling(const oefe_op_s* op, const KBatch<T>& kb, int nbw, hipStream_t s) {
  switch (nbw) {
    case 2: launch_coupling_w<T, 2, CPLX>(op, kb, s); break;
    default: launch_coupling_w<T, 1, CPLX>(op, kb, s); break;
  }
}

template <typename T, bool CPLX>
void launch_assemble(const oefe_op_s* op, const KBatch<T>& kb, int max_ncr, bool base_in_out, hipStream_t s) {
  const int64_t nel = CPLX ? max_ncr / 2 : max_ncr;
  const int64_t blocks = std::min<int64_t>(cdiv(op->N * nel, 256), int64_t(1) << 22);
  hipLaunchKernelGGL((fe_assemble_kernel<T, CPLX>), dim3((unsigned)blocks, 1, (unsigned)kb.nk),
                     dim3(256), 0, s, kb, op->nc, op->p, op->n, op->P1, coef<T>(op), (int)op->N,
                     base_in_out ? 1 : 0);
}

template <typename T, int NB>
void launch_node_fused_nb(const oefe_op_s* op, const KBatch<T>& kb, int ncb, hipStream_t s) {
  const size_t lds = node_lds_bytes<T, NB>(op->n_enr > 0 ? op->tile_fpmax : 0);
  if (allow_dynamic_lds(reinterpret_cast<const void*>(&fe_node_fused_kernel<T, NB>), lds) != hipSuccess) return;
  hipLaunchKernelGGL((fe_node_fused_kernel<T, NB>), dim3((unsigned)((int64_t)tile_count(op->n, op->tile_mode) * ncb), 1u,
                     (unsigned)kb.nk), dim3(256), lds, s, kb, op->nc, op->p, op->n, op->P1, coef<T>(op),
                     op->n_enr > 0 ? op->d.tile_fptr : nullptr, op->d.tile_fns, (int)op->N, ncb,
                     node_hs_cap<T, NB>(op->n_enr > 0 ? op->tile_fpmax : 0), op->tile_mode);
}

template <typename T>
void launch_node_fused(const oefe_op_s* op, const KBatch<T>& kb, int NB, int ncb, hipStream_t s) {
  switch (NB) {
    case 1: launch_node_fused_nb<T, 1>(op, kb, ncb, s); break;
    case 2: launch_node_fused_nb<T, 2>(op, kb, ncb, s); break;
    case 3: launch_node_fused_nb<T, 3>(op, kb, ncb, s); break;
    case 4: launch_node_fused_nb<T, 4>(op, kb, ncb, s); break;
    default: launch_node_fused_nb<T, 5>(op, kb, ncb, s); break;
  }
}

inline int reduce_chunks(const oefe_op_s* op) { return std::max(1, (int)cdiv(op->fn_smax, kReduceChunk)); }

// Steps of several operators sharing one mesh and enrichment layout, in lockstep.
void launch_cell_bf16(const oefe_op_s* op, const KBatch<float>& kb, hipStream_t s) {
  const size_t lds = 3 * (size_t)kBf16MatElems * sizeof(uint16_t) + 128 * (3 * sizeof(int) + sizeof(float));
  if (allow_dynamic_lds(reinterpret_cast<const void*>(&fe_cell_bf16_kernel), lds) != hipSuccess) return;
  int cus = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipLaunchKernelGGL(fe_cell_bf16_kernel, dim3((unsigned)std::max(1, cus / kb.nk), 1, (unsigned)kb.nk), dim3(768),
                     lds, s, kb, op->d.bf_mats, op->cf, op->nc, op->p, op->n, op->P1, op->n_cells);
}

template <typename T, bool CPLX>
int apply_step_batch_impl(const oefe_op_s* const* ops, const KBatch<T>& kb, hipStream_t s, const Overlap* ov,
                          bool bf16) {
  const oefe_op_s* op = ops[0];
  int max_ncr = 0, max_nv = 0;
  for (int q = 0; q < kb.nk; ++q) {
    max_ncr = std::max(max_ncr, kb.k[q].ncr);
    max_nv = std::max(max_nv, kb.k[q].nv);
    if (ops[q]->uform != op->uform) return OEFE_EINVAL;  // one form per batch
  }
  // the periodic-function form runs on the planes-in-lanes cell kernel only
  if (op->uform && !lanes_offsets_fit(op, kb)) return OEFE_EUNSUPPORTED;
  const unsigned nk = (unsigned)kb.nk;
  const int nO = op->n_enr;
  const bool ovl = ov != nullptr && nO > 0;
  // optional HIP events around one stage (oefe_kernel_timer), on the stream it runs on
  auto timed = [&](int kind, hipStream_t st, auto&& launch) {
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool on = op->timer_kind == kind && hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess;
    if (on) (void)hipEventRecord(ev0, st);
    launch();
    if (on) {
      (void)hipEventRecord(ev1, st);
      op->timer_events.emplace_back(ev0, ev1);
    }
  };
  auto cell_stage = [&] {
    timed(OEFE_TIMER_CELL, s, [&] {
      if constexpr (std::is_same<T, float>::value && !CPLX) {
        if (bf16) {
          launch_cell_bf16(op, kb, s);
          return;
        }
      }
      launch_cell<T, CPLX>(op, kb, max_ncr, op->tune_cw, s);
    });
  };
  const dim3 gg((unsigned)cdiv(max_nv, 16), (unsigned)cdiv(nO, 16), nk);
  // the chain that folds the tile partials into W' and writes the enrichment rows of out
  // (and, in an overlapped recurrence, Z^O of the next step), on stream se
  auto side_chain = [&](hipStream_t se) {
    const int nch = reduce_chunks(op);
    hipLaunchKernelGGL((enr_reduce1_kernel<T>), dim3((unsigned)(nO * nch), (unsigned)cdiv(max_ncr, 64), nk),
                       dim3(256), 0, se, kb, nch, op->d.fn_pptr, op->d.fn_poff);
    const size_t clds = enr_chain_lds_bytes<T, CPLX>(nO);
    if (clds <= 96 * 1024 &&
        allow_dynamic_lds(reinterpret_cast<const void*>(&enr_chain_kernel<T, CPLX>), clds) == hipSuccess) {
      hipLaunchKernelGGL((enr_chain_kernel<T, CPLX>), dim3((unsigned)cdiv(max_nv, kChainCols), 1, nk), dim3(1024), clds,
                         se, kb, op->N, nO, (ovl && !ov->last) ? 1 : 0);
    } else {
      hipLaunchKernelGGL((small_gemm_kernel<T, CPLX>), gg, dim3(256), 0, se, kb, 1, op->N, nO);
      hipLaunchKernelGGL((small_gemm_kernel<T, CPLX>), gg, dim3(256), 0, se, kb, 2, op->N, nO);
      if (ovl && !ov->last) hipLaunchKernelGGL((small_gemm_kernel<T, CPLX>), gg, dim3(256), 0, se, kb, 3, op->N, nO);
    }
    if (ovl) (void)hipEventRecord(ov->ev_zo, se);
  };
  if constexpr (!CPLX) {
    // Real operators: fused node kernel after the cell stage; the chain of step k runs on
    // the side stream beside the cell stage of step k+1, whose node stage waits for it.
    if (nO > 0 && (!ovl || ov->first)) hipLaunchKernelGGL((small_gemm_kernel<T, CPLX>), gg, dim3(256), 0, s, kb, 0, op->N, nO);
    cell_stage();
    // node workgroup width: 16-column blocks, all real columns up to the cap, else near-equal
    // parts.  Built-in cap: 4 blocks in float64 (diamond meshes of 110 k and 885 k nodes: node
    // stage 112 / 3650 us against 127 / 4470 us with 5), 5 in float32.
    const int nbdef = sizeof(T) == 8 ? 4 : kNodeNBMax;
    const int nbcap = std::max(1, std::min(kNodeNBMax, op->tune_cb > 0 ? op->tune_cb / 16 : nbdef));
    const int nb_all = (int)cdiv(max_ncr, 16);
    const int ncb = (int)cdiv(nb_all, nbcap);
    const int NB = (int)cdiv(nb_all, ncb);
    if (ovl && !ov->first) (void)hipStreamWaitEvent(s, ov->ev_zo, 0);  // this step's Z^O
    // one column: the flat kernel where tiles couple to few functions (the auxiliary-potential
    // operator, one function per atom: 23 % less time per conjugate-gradient iteration on
    // diamond64); the Kohn-Sham operator's ~50 functions per tile stay on the matrix cores
    if (max_ncr == 1 && op->tile_fpmax <= kCol1MaxFunctions) {
      const int ntiles = tile_count(op->n, op->tile_mode);
      timed(OEFE_TIMER_NODE, s, [&] {
        hipLaunchKernelGGL((fe_node_col1_kernel<T>), dim3((unsigned)cdiv(ntiles, 4), 1u, (unsigned)kb.nk), dim3(256), 0, s,
                           kb, op->nc, op->p, op->n, op->P1, coef<T>(op), op->n_enr > 0 ? op->d.tile_fptr : nullptr,
                           op->d.tile_fns, ntiles, op->tile_mode);
      });
    } else {
      timed(OEFE_TIMER_NODE, s, [&] { launch_node_fused<T>(op, kb, NB, ncb, s); });
    }
    if (nO > 0) {
      hipStream_t se = s;
      if (ovl) {
        (void)hipEventRecord(ov->ev_node, s);
        (void)hipStreamWaitEvent(ov->side, ov->ev_node, 0);
        se = ov->side;
      }
      side_chain(se);
      if (ovl && ov->last) (void)hipStreamWaitEvent(s, ov->ev_zo, 0);
    }
  } else {
    // Bloch operators: the coupling kernel (and then the chain) on the side stream, after
    // the previous step's node assembly and beside this step's cell stage; the assembly
    // adds onto the coupling kernel's result in out.
    if (nO > 0) {
      hipStream_t se = s;
      if (ovl) {
        if (ov->first) (void)hipEventRecord(ov->ev_node, s);
        (void)hipStreamWaitEvent(ov->side, ov->ev_node, 0);
        se = ov->side;
      }
      if (!ovl || ov->first) hipLaunchKernelGGL((small_gemm_kernel<T, CPLX>), gg, dim3(256), 0, se, kb, 0, op->N, nO);
      const int cb = op->tune_cb;
      const int nbw = cb >= 32 ? kCoupleNBWMax : 1;
      timed(OEFE_TIMER_COUPLING, se, [&] { launch_coupling<T, CPLX>(op, kb, nbw, se); });
      if (ovl) (void)hipEventRecord(ov->ev_k1, se);
      side_chain(se);
    }
    cell_stage();
    if (ovl) (void)hipStreamWaitEvent(s, ov->ev_k1, 0);
    timed(OEFE_TIMER_NODE, s, [&] { launch_assemble<T, CPLX>(op, kb, max_ncr, nO > 0, s); });
    if (ovl) {
      (void)hipEventRecord(ov->ev_node, s);
      if (ov->last) (void)hipStreamWaitEvent(s, ov->ev_zo, 0);
    }
  }
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
}

template <typename T>
KP<T> make_kp(const oefe_op_s* op, const T* x, int64_t ld, const T* prev, T* out, int64_t ldout, int nv,
              double alpha, double c, double beta, const StepWork& w) {
  const bool cx = op->cplx;
  const DevPtrs<T> dp = devptrs<T>(op);
  KP<T> P{};
  P.x = x;
  P.prev = prev;
  P.out = out;
  P.ldx = cx ? 2 * ld : ld;
  P.ldo = cx ? 2 * ldout : ldout;
  P.nv = nv;
  P.ncr = cx ? 2 * nv : nv;
  P.ycell = (T*)w.ycell;
  P.ldc = w.ldc;
  P.zo = (T*)w.zo;
  P.part = (T*)w.part;
  P.part2 = (T*)w.part2;
  P.nch = reduce_chunks(op);
  P.wp = (T*)w.wp;
  P.wv = dp.WV;
  P.tv = dp.tv;
  P.S = dp.S;
  P.Hoo = dp.Hoo;
  P.alpha = (T)alpha;
  P.c = (T)c;
  P.beta = (T)beta;
  P.sc = nullptr;
  for (int d = 0; d < 3; ++d) {
    P.ph.re[d] = (T)op->phase[d][0];
    P.ph.im[d] = (T)op->phase[d][1];
    P.uk[d] = (T)op->uk[d];
  }
  return P;
}

template <typename T, int P1, bool CPLX>
void launch_density(const oefe_op_s* op, const T* x, int64_t ldx, int ncr, const double* f, const T* zo, double* dens,
                    hipStream_t s) {
  Phase3<T> ph;
  for (int d = 0; d < 3; ++d) {
    ph.re[d] = (T)op->phase[d][0];
    ph.im[d] = (T)op->phase[d][1];
  }
  dim3 grid((unsigned)op->n_cells, (unsigned)cdiv(ncr, 64));
  hipLaunchKernelGGL((density_kernel<T, P1, CPLX>), grid, dim3(64 * P1), 0, s, x, ldx, ncr, f, zo, coef<T>(op),
                     op->nc, op->p, op->n, ph, op->d.cph_ptr, op->d.cph_blk, op->d.cph_off, op->d.blk_fn0,
                     op->d.blk_nf, op->d.phi, op->FMAX, op->n_enr, dens, op->n_cells);
}

}  // namespace

// Node-slot grid elements: n_cells nd rows of ldc, then a padding of one row plus 16 kNodeNBMax
// elements.  The fused node kernel reads the columns of a row without clamping them to ncr:
// at most cb0 + 16 NB - 1 < ncr + 16 kNodeNBMax - 1 for a column block that starts below ncr,
// so the reads past the last row's end stay inside the padding (ncr <= ldc).
static size_t slot_grid_elems(const oefe_op_s* op, int ldc) {
  return (size_t)op->n_cells * op->nd * ldc + (size_t)ldc + 16 * kNodeNBMax;
}

size_t step_work_bytes(const oefe_op_s* op, int elem_bytes, bool cplx, int nv, int* ldc_out) {
  const int ncr = cplx ? 2 * nv : nv;
  // rows of the node-slot grid: a multiple of 8 columns, except one real column, whose slots
  // are then contiguous (every cell kernel stores only columns below ncr; the node kernels'
  // reads past the column stay inside the grid's padding)
  const int ldc = ncr == 1 ? 1 : (int)cdiv(ncr, 8) * 8;
  if (ldc_out) *ldc_out = ldc;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t bytes = 0;
  if (!op->diagonal) bytes += al(slot_grid_elems(op, ldc) * elem_bytes);
  bytes += al((size_t)std::max(op->n_enr, 1) * ncr * elem_bytes);                 // zo
  bytes += al((size_t)std::max<int64_t>(op->tile_slots, 1) * ncr * elem_bytes);  // part
  bytes += al((size_t)std::max(op->n_enr, 1) * reduce_chunks(op) * ncr * elem_bytes);  // part2
  bytes += al((size_t)std::max(op->n_enr, 1) * ncr * elem_bytes);                 // wp
  return bytes;
}

StepWork carve_step_work(const oefe_op_s* op, int elem_bytes, bool cplx, int nv, void* work) {
  StepWork w{};
  const int ncr = cplx ? 2 * nv : nv;
  int ldc;
  step_work_bytes(op, elem_bytes, cplx, nv, &ldc);
  w.ldc = ldc;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  char* p = (char*)work;
  if (!op->diagonal) {
    w.ycell = p;
    p += al(slot_grid_elems(op, ldc) * elem_bytes);
  }
  w.zo = p;
  p += al((size_t)std::max(op->n_enr, 1) * ncr * elem_bytes);
  w.part = p;
  p += al((size_t)std::max<int64_t>(op->tile_slots, 1) * ncr * elem_bytes);
  w.part2 = p;
  p += al((size_t)std::max(op->n_enr, 1) * reduce_chunks(op) * ncr * elem_bytes);
  w.wp = p;
  return w;
}

template <typename T>
int apply_step(const oefe_op_s* op, bool bf16, const T* x, int64_t ld, const T* prev, T* out, int64_t ldo, int nv,
               double alpha, double c, double beta, const StepWork& w, hipStream_t s, const Overlap* ov,
               const double* sc) {
  // BF16 cell stage: real operators with float32 vectors and the dense-cell matrices
  if (bf16 && (sizeof(T) != 4 || op->cplx || op->diagonal || !op->d.bf_mats)) return OEFE_EUNSUPPORTED;
  if (!x || !out || (beta != 0.0 && !prev)) return OEFE_EINVAL;  // prev is read only when beta != 0
  if (sc && op->diagonal) return OEFE_EUNSUPPORTED;
  if (op->diagonal) {
    const DevPtrs<T> dp = devptrs<T>(op);
    const int64_t tot = op->N * nv;
    hipLaunchKernelGGL((diag_step_kernel<T>), dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, dp.lambda, x, prev,
                       out, ld, ldo, nv, op->N, (T)alpha, (T)c, (T)beta);
    return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
  }
  KBatch<T> kb{};
  kb.nk = 1;
  kb.k[0] = make_kp<T>(op, x, ld, prev, out, ldo, nv, alpha, c, beta, w);
  kb.k[0].sc = sc;
  const oefe_op_s* ops[1] = {op};
  if (op->cplx) return apply_step_batch_impl<T, true>(ops, kb, s, ov, false);
  return apply_step_batch_impl<T, false>(ops, kb, s, ov, bf16);
}

template int apply_step<double>(const oefe_op_s*, bool, const double*, int64_t, const double*, double*, int64_t, int,
                                double, double, double, const StepWork&, hipStream_t, const Overlap*, const double*);
template int apply_step<float>(const oefe_op_s*, bool, const float*, int64_t, const float*, float*, int64_t, int,
                               double, double, double, const StepWork&, hipStream_t, const Overlap*, const double*);

// The scalars of an m-step filter from device bounds (a, b, a0), in the order and arithmetic
// of the host recurrence: step 0 (s1 / e, c, 0), step k (2 s_k+1 / e, c, s_k s_k+1) with
// e = (b - a) / 2, c = (b + a) / 2, s1 = e / (a0 - c), s_k+1 = 1 / (2 / s1 - s_k).  Bounds
// that violate a0 < a < b give zero scalars and status {OEFE_EINVAL, 0}; else {0, -1}.
__global__ void cheb_scalars_kernel(const double* __restrict__ bounds, int m, double* __restrict__ out,
                                    int32_t* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double a = bounds[0], b = bounds[1], a0 = bounds[2];
  const bool ok = a < b && a0 < a && isfinite(a) && isfinite(b) && isfinite(a0);
  const double e = (b - a) / 2.0, c = (b + a) / 2.0;
  const double s1 = e / (a0 - c);
  out[0] = ok ? s1 / e : 0.0;
  out[1] = ok ? c : 0.0;
  out[2] = 0.0;
  double sig = s1;
  for (int k = 1; k < m; ++k) {
    const double sn = 1.0 / (2.0 / s1 - sig);
    out[3 * k] = ok ? 2.0 * sn / e : 0.0;
    out[3 * k + 1] = ok ? c : 0.0;
    out[3 * k + 2] = ok ? sig * sn : 0.0;
    sig = sn;
  }
  if (status) {
    status[0] = ok ? 0 : OEFE_EINVAL;
    status[1] = ok ? -1 : 0;
  }
}

int cheb_scalars(const double* bounds, int m, double* out, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(cheb_scalars_kernel, dim3(1), dim3(64), 0, s, bounds, m, out, status);
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
}

template <typename T>
int apply_step_batch(const oefe_op_s* const* ops, int nk, bool bf16, const T* const* x, const int64_t* ld,
                     const T* const* prev, T* const* out, const int64_t* ldo, const int* nv, const double* alpha,
                     const double* c, const double* beta, const StepWork* w, hipStream_t s, const Overlap* ov) {
  if (bf16)
    for (int q = 0; q < nk; ++q)
      if (sizeof(T) != 4 || ops[q]->cplx || ops[q]->diagonal || !ops[q]->d.bf_mats) return OEFE_EUNSUPPORTED;
  for (int q = 0; q < nk; ++q)  // the kernels read prev only when beta is nonzero
    if (!x[q] || !out[q] || (beta[q] != 0.0 && !prev[q])) return OEFE_EINVAL;
  for (int q0 = 0; q0 < nk; q0 += KMAX) {
    KBatch<T> kb{};
    kb.nk = std::min(KMAX, nk - q0);
    for (int q = 0; q < kb.nk; ++q)
      kb.k[q] = make_kp<T>(ops[q0 + q], x[q0 + q], ld[q0 + q], prev[q0 + q], out[q0 + q], ldo[q0 + q], nv[q0 + q],
                           alpha[q0 + q], c[q0 + q], beta[q0 + q], w[q0 + q]);
    // overlap only when the whole batch is one launch group
    const Overlap* o = nk <= KMAX ? ov : nullptr;
    const int rc = ops[0]->cplx ? apply_step_batch_impl<T, true>(ops + q0, kb, s, o, false)
                                : apply_step_batch_impl<T, false>(ops + q0, kb, s, o, bf16);
    if (rc) return rc;
  }
  return OEFE_OK;
}

template int apply_step_batch<double>(const oefe_op_s* const*, int, bool, const double* const*, const int64_t*,
                                      const double* const*, double* const*, const int64_t*, const int*, const double*,
                                      const double*, const double*, const StepWork*, hipStream_t, const Overlap*);
template int apply_step_batch<float>(const oefe_op_s* const*, int, bool, const float* const*, const int64_t*,
                                     const float* const*, float* const*, const int64_t*, const int*, const double*,
                                     const double*, const double*, const StepWork*, hipStream_t, const Overlap*);

template <typename T>
int zo_only(const oefe_op_s* op, const T* x, int64_t ld, int nv, T* zo, int ncr, hipStream_t s) {
  if (op->n_enr == 0) return OEFE_OK;
  StepWork w{};
  w.zo = zo;
  KBatch<T> kb{};
  kb.nk = 1;
  kb.k[0] = make_kp<T>(op, x, ld, nullptr, nullptr, ld, nv, 0, 0, 0, w);
  kb.k[0].ncr = ncr;
  if (op->cplx)
    hipLaunchKernelGGL((small_gemm_kernel<T, true>), dim3((unsigned)cdiv(nv, 16), (unsigned)cdiv(op->n_enr, 16), 1),
                       dim3(256), 0, s, kb, 0, op->N, op->n_enr);
  else
    hipLaunchKernelGGL((small_gemm_kernel<T, false>), dim3((unsigned)cdiv(nv, 16), (unsigned)cdiv(op->n_enr, 16), 1),
                       dim3(256), 0, s, kb, 0, op->N, op->n_enr);
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
}

template int zo_only<double>(const oefe_op_s*, const double*, int64_t, int, double*, int, hipStream_t);
template int zo_only<float>(const oefe_op_s*, const float*, int64_t, int, float*, int, hipStream_t);

template <typename T>
int density_partial(const oefe_op_s* op, const T* x, int64_t ld, int nv, const double* f, const T* zo, int ncr,
                    double* dens, hipStream_t s) {
  const bool c = op->cplx;
  const int64_t ldx = c ? 2 * ld : ld;
  switch (op->P1) {
    case 3: c ? launch_density<T, 3, true>(op, x, ldx, ncr, f, zo, dens, s) : launch_density<T, 3, false>(op, x, ldx, ncr, f, zo, dens, s); break;
    case 4: c ? launch_density<T, 4, true>(op, x, ldx, ncr, f, zo, dens, s) : launch_density<T, 4, false>(op, x, ldx, ncr, f, zo, dens, s); break;
    default: c ? launch_density<T, 5, true>(op, x, ldx, ncr, f, zo, dens, s) : launch_density<T, 5, false>(op, x, ldx, ncr, f, zo, dens, s); break;
  }
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
}

int density_final(const oefe_op_s* op, const double* dens, int nblk, double* dEdV, hipStream_t s, int mode) {
  const int64_t total = op->n_cells * op->nq;
  GW gw;
  for (int i = 0; i < 8; ++i) gw.w[i] = i < op->P1 ? op->gauss_w[i] : 0.0;
  const double h3 = (op->h / 2) * (op->h / 2) * (op->h / 2);
  hipLaunchKernelGGL(density_final_kernel2, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, dens, nblk, total,
                     op->P1, gw, h3, dEdV, mode);
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
}

template int density_partial<double>(const oefe_op_s*, const double*, int64_t, int, const double*, const double*, int,
                                     double*, hipStream_t);
template int density_partial<float>(const oefe_op_s*, const float*, int64_t, int, const double*, const float*, int,
                                    double*, hipStream_t);

}  // namespace oefe
