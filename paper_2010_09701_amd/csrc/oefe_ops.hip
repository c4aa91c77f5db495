// HIP kernels of the OEFE operator application Ht X = M^-1/2 H M^-1/2 X and the
// scaled Chebyshev recurrence step built on it (gfx950, wave64).
//
// One operator step (out = alpha (Ht x - c x) - beta prev) is:
//   1. zo      Z^O = S X^O                                   (small dense)
//   2. cell    per cell: z_e = m^-1/2 (theta o X)|_e, y_e = K_e z_e + B^T diag(W V) B z_e
//              (sum-factorized, see fe_cell_kernel) -> per-cell buffer
//   3. partial per atom block / row chunk: sum_r conj(H^co[r, f]) m_r^-1/2 X[r]
//   4. node    per FE node: sum of the (up to 8) cell results sharing it (fixed order,
//              no atomics), + H^co Z^O, times m^-1/2, recurrence epilogue
//   5. wprime  W' = sum of partials + H^oo Z^O ;  6. final  S W', recurrence epilogue
#include <hip/hip_runtime.h>

#include <algorithm>

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
__global__ __launch_bounds__(64 * P1) void fe_cell_kernel(const T* __restrict__ X, int64_t ldx, int ncr,
                                                          T* __restrict__ Yc, int ldc, const T* __restrict__ WV,
                                                          CellCoef<T> cf, int nc, int p, int n, int64_t n_cells,
                                                          Phase3<T> ph) {
  constexpr int NP = P1 * P1;
  constexpr int CPT = 64 / CW;
  __shared__ T lds[NP * P1][64];
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
#pragma unroll
  for (int qz = 0; qz < P1; ++qz)
#pragma unroll
    for (int qy = 0; qy < P1; ++qy) {
      T s = 0;
#pragma unroll
      for (int az = 0; az < P1; ++az) s += cf.B1[qz][az] * t[az * P1 + qy];
      u[qz * P1 + qy] = s;
    }
  // 5. quadrature-point terms: potential + y/z kinetic
  const int qx = w;
  const T kx = cf.kappa * cf.w[qx];
  const T* wv = WV + ee * (NP * P1);
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
      t[qz * P1 + qy] = wv[(qz * P1 + qy) * P1 + qx] * u[qz * P1 + qy] + kx * (cf.w[qz] * ly + cf.w[qy] * lz);
    }
  // 6. t' = (B^T)_y (B^T)_z t  -> indexed [az][ay]
  T tp[NP];
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
  // 7. s = kappa (B^T W)_y (B^T W)_z u  (the x kinetic term before its x-pass)
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
#pragma unroll
    for (int ax = 0; ax < P1; ++ax) {
      T s = 0;
#pragma unroll
      for (int q = 0; q < P1; ++q) s += cf.B1[q][ax] * r[q];
      y[ay * P1 + ax] = s;
    }
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
  // 10. store plane az = w of y_e
  if (valid) {
    T* out = Yc + (e * (NP * P1) + w * NP) * (int64_t)ldc + j;
#pragma unroll
    for (int a = 0; a < NP; ++a) out[(int64_t)a * ldc] = y[a];
  }
}

// ---------------------------------------------------------------------------
// Node kernel: FE rows.  Workgroup = RB nodes x NVB vector lanes (2D), thread
// per (FE node g, vector v): fixed-order sum of the (up to 8) cell results that
// share g, times m_g^-1/2, plus the enrichment term sum_nu (m^-1/2 H^co)[g,nu]
// Z^O[nu][v] (pre-scaled per-row CSR), then the recurrence epilogue.
// Z^O is staged in LDS when it fits.
// ---------------------------------------------------------------------------
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void fe_node_kernel(
    const T* __restrict__ Yc, int ldc, const T* __restrict__ X, const T* __restrict__ prev, T* __restrict__ out,
    int64_t ldx, int64_t ldo, int nv, int nvb, int nc, int p, int n, int P1, CellCoef<T> cf, Phase3<T> ph,
    const T* __restrict__ zo, int ncr, int nO, int zo_in_lds, const int64_t* __restrict__ fr_ptr,
    const int32_t* __restrict__ fr_fn, const T* __restrict__ fr_val, T alpha, T c, T beta, int N) {
  extern __shared__ unsigned char smem_raw[];
  T* zs = reinterpret_cast<T*>(smem_raw);
  const int tx = threadIdx.x % nvb, ty = threadIdx.x / nvb;
  const int RB = blockDim.x / nvb;
  if (zo_in_lds) {
    const int tot = nO * ncr;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) zs[t] = zo[t];
    __syncthreads();
  }
  const T* zsrc = zo_in_lds ? zs : zo;
  const int g = blockIdx.x * RB + ty;
  const int vv = blockIdx.y * nvb + tx;
  if (ty >= RB || g >= N || vv >= nv) return;
  const int ix = g % n, iy = (g / n) % n, iz = g / (n * n);
  const int nd = P1 * P1 * P1;
  int cxs[2], axs[2], wxs[2], nxs = 1;
  int cys[2], ays[2], wys[2], nys = 1;
  int czs[2], azs[2], wzs[2], nzs = 1;
  cxs[0] = ix / p; axs[0] = ix % p; wxs[0] = 0;
  if (axs[0] == 0) { cxs[1] = (cxs[0] + nc - 1) % nc; axs[1] = p; wxs[1] = (cxs[1] == nc - 1); nxs = 2; }
  cys[0] = iy / p; ays[0] = iy % p; wys[0] = 0;
  if (ays[0] == 0) { cys[1] = (cys[0] + nc - 1) % nc; ays[1] = p; wys[1] = (cys[1] == nc - 1); nys = 2; }
  czs[0] = iz / p; azs[0] = iz % p; wzs[0] = 0;
  if (azs[0] == 0) { czs[1] = (czs[0] + nc - 1) % nc; azs[1] = p; wzs[1] = (czs[1] == nc - 1); nzs = 2; }
  const T msc = cf.mscale * cf.om[ix % p] * cf.om[iy % p] * cf.om[iz % p];
  const int64_t k0 = fr_ptr[g], k1 = fr_ptr[g + 1];
  if constexpr (!CPLX) {
    T acc = 0;
    for (int kz = 0; kz < nzs; ++kz)
      for (int ky = 0; ky < nys; ++ky)
        for (int kx = 0; kx < nxs; ++kx) {
          const int64_t e = cxs[kx] + (int64_t)nc * (cys[ky] + (int64_t)nc * czs[kz]);
          const int a = axs[kx] + P1 * (ays[ky] + P1 * azs[kz]);
          acc += Yc[(e * nd + a) * (int64_t)ldc + vv];
        }
    T en = 0;
#pragma unroll 8
    for (int64_t k = k0; k < k1; ++k) en += fr_val[k] * zsrc[fr_fn[k] * ncr + vv];
    const T hx = msc * acc + en;
    const int64_t gi = (int64_t)g;
    const T xv = X[gi * ldx + vv];
    T r = alpha * (hx - c * xv);
    if (beta != T(0)) r -= beta * prev[gi * ldo + vv];
    out[gi * ldo + vv] = r;
  } else {
    C2<T> acc{0, 0};
    for (int kz = 0; kz < nzs; ++kz)
      for (int ky = 0; ky < nys; ++ky)
        for (int kx = 0; kx < nxs; ++kx) {
          const int64_t e = cxs[kx] + (int64_t)nc * (cys[ky] + (int64_t)nc * czs[kz]);
          const int a = axs[kx] + P1 * (ays[ky] + P1 * azs[kz]);
          const T* py = Yc + (e * nd + a) * (int64_t)ldc + 2 * vv;
          C2<T> z{py[0], py[1]};
          // scatter phase conj(theta)
          if (wxs[kx]) z = cjmul(C2<T>{ph.re[0], ph.im[0]}, z);
          if (wys[ky]) z = cjmul(C2<T>{ph.re[1], ph.im[1]}, z);
          if (wzs[kz]) z = cjmul(C2<T>{ph.re[2], ph.im[2]}, z);
          acc.r += z.r;
          acc.i += z.i;
        }
    C2<T> en{0, 0};
#pragma unroll 4
    for (int64_t k = k0; k < k1; ++k) {
      const T* pz = zsrc + fr_fn[k] * ncr + 2 * vv;
      const C2<T> zz = cmul(C2<T>{fr_val[2 * k], fr_val[2 * k + 1]}, C2<T>{pz[0], pz[1]});
      en.r += zz.r;
      en.i += zz.i;
    }
    const int64_t gi = (int64_t)g;
    const T* px = X + gi * ldx + 2 * vv;
    T rr = alpha * (msc * acc.r + en.r - c * px[0]);
    T ri = alpha * (msc * acc.i + en.i - c * px[1]);
    if (beta != T(0)) {
      const T* pp = prev + gi * ldo + 2 * vv;
      rr -= beta * pp[0];
      ri -= beta * pp[1];
    }
    T* po = out + gi * ldo + 2 * vv;
    po[0] = rr;
    po[1] = ri;
  }
}

// ---------------------------------------------------------------------------
// Tiled node kernel: FE rows.  Workgroup = one tile of kTileRows consecutive FE
// rows x CB real columns, 4 row groups.  For each output (row g, column j):
//   fixed-order sum of the (up to 8) cell results sharing g, times m_g^-1/2,
//   + sum_f Ht[g][f] Z^O[fn_f][j]  (dense tile block of m^-1/2 H^co, LDS-staged
//     16 functions at a time together with the matching Z^O rows),
//   then the recurrence epilogue alpha (y - c x) - beta prev.
// ---------------------------------------------------------------------------
template <typename T, bool CPLX>
__global__ __launch_bounds__(512) void fe_node_tile_kernel(
    const T* __restrict__ Yc, int ldc, const T* __restrict__ X, const T* __restrict__ prev, T* __restrict__ out,
    int64_t ldx, int64_t ldo, int ncr, int CB, int nc, int p, int n, int P1, CellCoef<T> cf, Phase3<T> ph,
    const T* __restrict__ zo, const int32_t* __restrict__ tile_fptr, const int32_t* __restrict__ tile_fns,
    const T* __restrict__ tile_val, T alpha, T c, T beta, int N) {
  constexpr int TR = kTileRows, RG = 4, RPT = TR / RG, JC = 16;
  constexpr int E = CPLX ? 2 : 1;
  extern __shared__ unsigned char smem_raw[];
  T* Hs = reinterpret_cast<T*>(smem_raw);  // [TR][JC][E]
  T* zs = Hs + TR * JC * E;                // [JC][CB]
  const int cl = threadIdx.x % CB, rg = threadIdx.x / CB;
  const int t = blockIdx.x;
  const int j = blockIdx.y * CB + cl;  // real column
  // no enrichment: tile_fptr is null and the tile couples to no function
  const int f0 = tile_fptr ? tile_fptr[t] : 0, FP = tile_fptr ? tile_fptr[t + 1] - f0 : 0;
  const T* tv = tile_val + (int64_t)f0 * TR * E;
  T en[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) en[i] = 0;
  for (int j0 = 0; j0 < FP; j0 += JC) {
    const int jn = min(JC, FP - j0);
    for (int q = threadIdx.x; q < TR * JC * E; q += blockDim.x) {
      const int r = q / (JC * E), jj = (q / E) % JC, e = q % E;
      Hs[q] = jj < jn ? tv[((int64_t)r * FP + j0 + jj) * E + e] : T(0);
    }
    for (int q = threadIdx.x; q < JC * CB; q += blockDim.x) {
      const int jj = q / CB, cc = q % CB;
      const int fn = jj < jn ? tile_fns[f0 + j0 + jj] : -1;
      const int col = blockIdx.y * CB + cc;
      zs[q] = (fn >= 0 && col < ncr) ? zo[(int64_t)fn * ncr + col] : T(0);
    }
    __syncthreads();
    for (int jj = 0; jj < jn; ++jj) {
      if constexpr (!CPLX) {
        const T z = zs[jj * CB + cl];
#pragma unroll
        for (int i = 0; i < RPT; ++i) en[i] += Hs[(rg + RG * i) * JC + jj] * z;
      } else {
        const T zr = zs[jj * CB + (cl & ~1)], zi = zs[jj * CB + (cl | 1)];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const T hr = Hs[((rg + RG * i) * JC + jj) * 2], hi = Hs[((rg + RG * i) * JC + jj) * 2 + 1];
          en[i] += (cl & 1) ? (hr * zi + hi * zr) : (hr * zr - hi * zi);
        }
      }
    }
    __syncthreads();
  }
  if (j >= ncr) return;
  const int nd = P1 * P1 * P1;
#pragma unroll 1
  for (int i = 0; i < RPT; ++i) {
    const int g = t * TR + rg + RG * i;
    if (g >= N) break;
    const int ix = g % n, iy = (g / n) % n, iz = g / (n * n);
    int cxs[2], axs[2], wxs[2], nxs = 1;
    int cys[2], ays[2], wys[2], nys = 1;
    int czs[2], azs[2], wzs[2], nzs = 1;
    cxs[0] = ix / p; axs[0] = ix % p; wxs[0] = 0;
    if (axs[0] == 0) { cxs[1] = (cxs[0] + nc - 1) % nc; axs[1] = p; wxs[1] = (cxs[1] == nc - 1); nxs = 2; }
    cys[0] = iy / p; ays[0] = iy % p; wys[0] = 0;
    if (ays[0] == 0) { cys[1] = (cys[0] + nc - 1) % nc; ays[1] = p; wys[1] = (cys[1] == nc - 1); nys = 2; }
    czs[0] = iz / p; azs[0] = iz % p; wzs[0] = 0;
    if (azs[0] == 0) { czs[1] = (czs[0] + nc - 1) % nc; azs[1] = p; wzs[1] = (czs[1] == nc - 1); nzs = 2; }
    const T msc = cf.mscale * cf.om[ix % p] * cf.om[iy % p] * cf.om[iz % p];
    T acc = 0;
    for (int kz = 0; kz < nzs; ++kz)
      for (int ky = 0; ky < nys; ++ky)
        for (int kx = 0; kx < nxs; ++kx) {
          const int64_t e = cxs[kx] + (int64_t)nc * (cys[ky] + (int64_t)nc * czs[kz]);
          const int a = axs[kx] + P1 * (ays[ky] + P1 * azs[kz]);
          if constexpr (!CPLX) {
            acc += Yc[(e * nd + a) * (int64_t)ldc + j];
          } else {
            const T* py = Yc + (e * nd + a) * (int64_t)ldc + (j & ~1);
            C2<T> z{py[0], py[1]};
            if (wxs[kx]) z = cjmul(C2<T>{ph.re[0], ph.im[0]}, z);
            if (wys[ky]) z = cjmul(C2<T>{ph.re[1], ph.im[1]}, z);
            if (wzs[kz]) z = cjmul(C2<T>{ph.re[2], ph.im[2]}, z);
            acc += (j & 1) ? z.i : z.r;
          }
        }
    const int64_t gi = (int64_t)g;
    T r = alpha * (msc * acc + en[i] - c * X[gi * ldx + j]);
    if (beta != T(0)) r -= beta * prev[gi * ldo + j];
    out[gi * ldo + j] = r;
  }
}

// Transposed enrichment product per tile:
//   part[(tile_fptr[t] + s)][j] = sum_{r in tile} conj(Ht[r][s]) x[r][j]
// Workgroup = one tile x CB real columns, 4 slot groups; rows staged 16 at a time.
template <typename T, bool CPLX>
__global__ __launch_bounds__(512) void enr_tile_partial_kernel(
    const T* __restrict__ x, int64_t ldx, int ncr, int CB, const int32_t* __restrict__ tile_fptr,
    const T* __restrict__ tile_val, T* __restrict__ part, int N) {
  constexpr int TR = kTileRows, SG = 4, RC = 16, SMAX = 16;
  constexpr int E = CPLX ? 2 : 1;
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);  // [RC][CB]
  T* Hs = xs + RC * CB;                     // [RC][FP][E]
  const int cl = threadIdx.x % CB, sg = threadIdx.x / CB;
  const int t = blockIdx.x;
  const int j = blockIdx.y * CB + cl;
  const int f0 = tile_fptr[t], FP = tile_fptr[t + 1] - f0;
  const T* tv = tile_val + (int64_t)f0 * TR * E;
  for (int s0 = 0; s0 < FP; s0 += SG * SMAX) {  // slots in groups of 64
    T acc[SMAX];
#pragma unroll
    for (int i = 0; i < SMAX; ++i) acc[i] = 0;
    for (int r0 = 0; r0 < TR; r0 += RC) {
      for (int q = threadIdx.x; q < RC * CB; q += blockDim.x) {
        const int rr = q / CB, cc = q % CB;
        const int g = t * TR + r0 + rr;
        const int col = blockIdx.y * CB + cc;
        xs[q] = (g < N && col < ncr) ? x[(int64_t)g * ldx + col] : T(0);
      }
      for (int q = threadIdx.x; q < RC * FP * E; q += blockDim.x) Hs[q] = tv[(int64_t)r0 * FP * E + q];
      __syncthreads();
      for (int rr = 0; rr < RC; ++rr) {
        if constexpr (!CPLX) {
          const T xv = xs[rr * CB + cl];
#pragma unroll
          for (int i = 0; i < SMAX; ++i) {
            const int sl = s0 + sg + SG * i;
            if (sl < FP) acc[i] += Hs[rr * FP + sl] * xv;
          }
        } else {
          const T xr = xs[rr * CB + (cl & ~1)], xi = xs[rr * CB + (cl | 1)];
#pragma unroll
          for (int i = 0; i < SMAX; ++i) {
            const int sl = s0 + sg + SG * i;
            if (sl < FP) {
              const T hr = Hs[(rr * FP + sl) * 2], hi = Hs[(rr * FP + sl) * 2 + 1];
              acc[i] += (cl & 1) ? (hr * xi - hi * xr) : (hr * xr + hi * xi);
            }
          }
        }
      }
      __syncthreads();
    }
    if (j < ncr) {
#pragma unroll
      for (int i = 0; i < SMAX; ++i) {
        const int sl = s0 + sg + SG * i;
        if (sl < FP) part[(int64_t)(f0 + sl) * ncr + j] = acc[i];
      }
    }
  }
}

// W'[nu][j] = sum over the tiles coupling to nu of their partial slot, in tile order.
// Workgroup per (nu, 64 real columns): 16 groups sum strided subsets, fixed LDS tree.
template <typename T>
__global__ __launch_bounds__(1024) void enr_tile_reduce_kernel(const T* __restrict__ part,
                                                               const int32_t* __restrict__ fn_pptr,
                                                               const int32_t* __restrict__ fn_poff, int ncr,
                                                               T* __restrict__ wp) {
  __shared__ T red[16][64];
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int nu = blockIdx.x;
  const int j = blockIdx.y * 64 + lane;
  const int e0 = fn_pptr[nu], e1 = fn_pptr[nu + 1];
  T s0 = 0, s1 = 0;
  if (j < ncr) {
    int e = e0 + grp;
    for (; e + 16 < e1; e += 32) {
      s0 += part[(int64_t)fn_poff[e] * ncr + j];
      s1 += part[(int64_t)fn_poff[e + 16] * ncr + j];
    }
    if (e < e1) s0 += part[(int64_t)fn_poff[e] * ncr + j];
  }
  red[grp][lane] = s0 + s1;
  __syncthreads();
  for (int st = 8; st > 0; st >>= 1) {
    if (grp < st) red[grp][lane] += red[grp + st][lane];
    __syncthreads();
  }
  if (grp == 0 && j < ncr) wp[(int64_t)nu * ncr + j] = red[0][lane];
}

// Partial transposed enrichment product per row chunk of an atom block:
//   part[c][f][v] = sum_{r in chunk} conj((m^-1/2 H^co)[r, f]) x[row_r][v]
// Workgroup = RG row groups x NVB vector lanes; the row groups are reduced in LDS.
template <typename T, bool CPLX>
__global__ __launch_bounds__(512) void enr_partial_kernel(
    const T* __restrict__ x, int64_t ldx, int nv, int nvb, const int32_t* __restrict__ chunk_blk,
    const int64_t* __restrict__ chunk_r0, const int64_t* __restrict__ chunk_r1, const int32_t* __restrict__ blk_nf,
    const int64_t* __restrict__ blk_rptr, const int32_t* __restrict__ rows, const T* __restrict__ hv, int FMAX,
    T* __restrict__ part, int ncr) {
  constexpr int FM = 8;
  constexpr int E = CPLX ? 2 : 1;
  extern __shared__ unsigned char smem_raw[];
  T* red = reinterpret_cast<T*>(smem_raw);  // [RG][FMAX][nvb][E]
  const int tx = threadIdx.x % nvb, ty = threadIdx.x / nvb;
  const int RG = blockDim.x / nvb;
  const int c = blockIdx.x;
  const int vv = blockIdx.y * nvb + tx;
  const bool active = ty < RG && vv < nv;
  const int b = chunk_blk[c];
  const int nf = blk_nf[b];
  const int64_t base = blk_rptr[b];
  T ar[FM], ai[FM];
#pragma unroll
  for (int f = 0; f < FM; ++f) ar[f] = ai[f] = 0;
  if (active) {
    const int64_t r1 = chunk_r1[c];
#pragma unroll 4
    for (int64_t r = chunk_r0[c] + ty; r < r1; r += RG) {
      const int64_t g = rows[base + r];
      const T* h = hv + (base + r) * FMAX * E;
      if constexpr (!CPLX) {
        const T z = x[g * ldx + vv];
#pragma unroll
        for (int f = 0; f < FM; ++f)
          if (f < nf) ar[f] += h[f] * z;
      } else {
        const T* px = x + g * ldx + 2 * vv;
        const C2<T> z{px[0], px[1]};
#pragma unroll
        for (int f = 0; f < FM; ++f)
          if (f < nf) {
            const C2<T> t = cjmul(C2<T>{h[2 * f], h[2 * f + 1]}, z);
            ar[f] += t.r;
            ai[f] += t.i;
          }
      }
    }
  }
  if (ty < RG) {
    for (int f = 0; f < nf; ++f) {
      red[((ty * FMAX + f) * nvb + tx) * E] = ar[f];
      if (CPLX) red[((ty * FMAX + f) * nvb + tx) * E + (E - 1)] = ai[f];
    }
  }
  __syncthreads();
  if (ty == 0 && vv < nv) {
    for (int f = 0; f < nf; ++f) {
      T sr = 0, si = 0;
      for (int g2 = 0; g2 < RG; ++g2) {
        sr += red[((g2 * FMAX + f) * nvb + tx) * E];
        if (CPLX) si += red[((g2 * FMAX + f) * nvb + tx) * E + (E - 1)];
      }
      part[((int64_t)c * FMAX + f) * ncr + E * vv] = sr;
      if (CPLX) part[((int64_t)c * FMAX + f) * ncr + E * vv + 1] = si;
    }
  }
}

// W'[nu][j] = sum over the chunks of nu's block of part, in a fixed order.
// Workgroup per (nu, 64 real columns): 16 groups of 64 lanes each sum a strided
// subset of the chunks, then a fixed LDS tree combines the groups.
template <typename T>
__global__ __launch_bounds__(1024) void enr_reduce_kernel(const T* __restrict__ part,
                                                          const int32_t* __restrict__ fn_blk,
                                                          const int32_t* __restrict__ blk_fn0,
                                                          const int32_t* __restrict__ blk_chunk0, int FMAX, int nO,
                                                          int ncr, T* __restrict__ wp) {
  __shared__ T red[16][64];
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int nu = blockIdx.x;
  const int j = blockIdx.y * 64 + lane;
  const int b = fn_blk[nu];
  const int f = nu - blk_fn0[b];
  const int c0 = blk_chunk0[b], c1 = blk_chunk0[b + 1];
  T s0 = 0, s1 = 0;
  if (j < ncr) {
    int c = c0 + grp;
    for (; c + 16 < c1; c += 32) {
      s0 += part[((int64_t)c * FMAX + f) * ncr + j];
      s1 += part[((int64_t)(c + 16) * FMAX + f) * ncr + j];
    }
    if (c < c1) s0 += part[((int64_t)c * FMAX + f) * ncr + j];
  }
  red[grp][lane] = s0 + s1;
  __syncthreads();
  for (int st = 8; st > 0; st >>= 1) {
    if (grp < st) red[grp][lane] += red[grp + st][lane];
    __syncthreads();
  }
  if (grp == 0 && j < ncr) wp[(int64_t)nu * ncr + j] = red[0][lane];
}

// Small dense products on the enrichment rows (n x k times k x m, complex
// interleaved when CPLX), 16x16 output tile per workgroup, LDS-staged K tiles.
//   mode 0: C = A B        mode 1: C += A B
//   mode 2: recurrence epilogue  out[N+i][j] = alpha (A B - c x[N+i][j]) - beta prev[N+i][j]
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void small_gemm_kernel(const T* __restrict__ A, const T* __restrict__ B, int64_t ldb,
                                                         T* __restrict__ C, int64_t ldc, int n, int k, int m, int mode,
                                                         const T* __restrict__ x, const T* __restrict__ prev,
                                                         int64_t ldx, int64_t ldo, T alpha, T cc, T beta) {
  constexpr int E = CPLX ? 2 : 1;
  constexpr int TS = 16;
  __shared__ T As[TS][TS * E + 1];
  __shared__ T Bs[TS][TS * E + 1];
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  const int i = blockIdx.y * TS + ty;  // row of C
  const int j = blockIdx.x * TS + tx;  // column of C (complex element)
  T sr = 0, si = 0;
  for (int k0 = 0; k0 < k; k0 += TS) {
    for (int e = 0; e < E; ++e) {
      const int ka = k0 + tx, kb = k0 + ty;
      As[ty][tx * E + e] = (i < n && ka < k) ? A[((int64_t)i * k + ka) * E + e] : T(0);
      Bs[ty][tx * E + e] = (kb < k && j < m) ? B[(int64_t)kb * ldb + (int64_t)j * E + e] : T(0);
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
  if (i >= n || j >= m) return;
  if (mode == 0) {
    C[(int64_t)i * ldc + (int64_t)j * E] = sr;
    if (CPLX) C[(int64_t)i * ldc + (int64_t)j * E + 1] = si;
  } else if (mode == 1) {
    C[(int64_t)i * ldc + (int64_t)j * E] += sr;
    if (CPLX) C[(int64_t)i * ldc + (int64_t)j * E + 1] += si;
  } else {
    const int64_t ox = (int64_t)i * ldx + (int64_t)j * E, oo = (int64_t)i * ldo + (int64_t)j * E;
    T r = alpha * (sr - cc * x[ox]);
    if (beta != T(0)) r -= beta * prev[oo];
    C[oo] = r;
    if (CPLX) {
      T r2 = alpha * (si - cc * x[ox + 1]);
      if (beta != T(0)) r2 -= beta * prev[oo + 1];
      C[oo + 1] = r2;
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
  // enrichment part
  if (valid) {
    for (int64_t k = cph_ptr[e]; k < cph_ptr[e + 1]; ++k) {
      const int b = cph_blk[k];
      const int64_t off = cph_off[k];
      const int f0 = blk_fn0[b], nf = blk_nf[b];
      for (int f = 0; f < nf; ++f) {
        if constexpr (!CPLX) {
          const double z = (double)zo[(int64_t)(f0 + f) * ncr + j];
#pragma unroll
          for (int qz = 0; qz < P1; ++qz)
#pragma unroll
            for (int qy = 0; qy < P1; ++qy) {
              const int q = (qz * P1 + qy) * P1 + qx;
              psi[qz * P1 + qy] += phi[(off * NQ + q) * FMAX + f] * z;
            }
        } else {
          const int v2 = j & ~1;
          const double zr = (double)zo[(int64_t)(f0 + f) * ncr + v2];
          const double zi = (double)zo[(int64_t)(f0 + f) * ncr + v2 + 1];
#pragma unroll
          for (int qz = 0; qz < P1; ++qz)
#pragma unroll
            for (int qy = 0; qy < P1; ++qy) {
              const int q = (qz * P1 + qy) * P1 + qx;
              const double pr = phi[2 * ((off * NQ + q) * FMAX + f)];
              const double pi = phi[2 * ((off * NQ + q) * FMAX + f) + 1];
              psi[qz * P1 + qy] += (j & 1) ? (pr * zi + pi * zr) : (pr * zr - pi * zi);
            }
        }
      }
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
__global__ void density_final_kernel2(const double* __restrict__ dens, int nblk, int64_t total, int P1, GW gw,
                                      double h3, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int nq = P1 * P1 * P1;
  const int q = (int)(t % nq);
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += dens[(int64_t)b * total + t];
  const double W = h3 * gw.w[q % P1] * gw.w[(q / P1) % P1] * gw.w[q / (P1 * P1)];
  out[t] = W * s;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int pick_cw(int ncr) {
  if (ncr >= 64 && ncr % 64 == 0) return 64;
  if (ncr >= 48) return (ncr % 32 == 0) ? 32 : (ncr % 16 == 0 ? 16 : (ncr >= 128 ? 64 : 8));
  if (ncr >= 32 && ncr % 32 == 0) return 32;
  if (ncr >= 16 && ncr % 16 == 0) return 16;
  return 8;
}

template <typename T, int P1, int CW, bool CPLX>
void launch_cell_cw(const oefe_op_s* op, const T* x, int64_t ldx, int ncr, T* yc, int ldc, const T* wv,
                    const CellCoef<T>& cf, const Phase3<T>& ph, hipStream_t s) {
  constexpr int CPT = 64 / CW;
  dim3 grid((unsigned)cdiv(op->n_cells, CPT), (unsigned)cdiv(ncr, CW));
  hipLaunchKernelGGL((fe_cell_kernel<T, P1, CW, CPLX>), grid, dim3(64 * P1), 0, s, x, ldx, ncr, yc, ldc, wv, cf,
                     op->nc, op->p, op->n, op->n_cells, ph);
}

template <typename T, int P1, bool CPLX>
void launch_cell_p(const oefe_op_s* op, const T* x, int64_t ldx, int ncr, T* yc, int ldc, const T* wv,
                   const CellCoef<T>& cf, const Phase3<T>& ph, hipStream_t s) {
  switch (pick_cw(ncr)) {
    case 64: launch_cell_cw<T, P1, 64, CPLX>(op, x, ldx, ncr, yc, ldc, wv, cf, ph, s); break;
    case 32: launch_cell_cw<T, P1, 32, CPLX>(op, x, ldx, ncr, yc, ldc, wv, cf, ph, s); break;
    case 16: launch_cell_cw<T, P1, 16, CPLX>(op, x, ldx, ncr, yc, ldc, wv, cf, ph, s); break;
    default: launch_cell_cw<T, P1, 8, CPLX>(op, x, ldx, ncr, yc, ldc, wv, cf, ph, s); break;
  }
}

template <typename T, bool CPLX>
void launch_cell(const oefe_op_s* op, const T* x, int64_t ldx, int ncr, T* yc, int ldc, const T* wv,
                 const CellCoef<T>& cf, const Phase3<T>& ph, hipStream_t s) {
  switch (op->P1) {
    case 3: launch_cell_p<T, 3, CPLX>(op, x, ldx, ncr, yc, ldc, wv, cf, ph, s); break;
    case 4: launch_cell_p<T, 4, CPLX>(op, x, ldx, ncr, yc, ldc, wv, cf, ph, s); break;
    default: launch_cell_p<T, 5, CPLX>(op, x, ldx, ncr, yc, ldc, wv, cf, ph, s); break;
  }
}

template <typename T>
const CellCoef<T>& coef(const oefe_op_s* op);
template <>
const CellCoef<double>& coef<double>(const oefe_op_s* op) { return op->cd; }
template <>
const CellCoef<float>& coef<float>(const oefe_op_s* op) { return op->cf; }

template <typename T>
struct DevPtrs {
  const T *WV, *hv, *S, *Hoo, *lambda, *frv, *tv;
};
template <typename T>
DevPtrs<T> devptrs(const oefe_op_s* op);
template <>
DevPtrs<double> devptrs<double>(const oefe_op_s* op) {
  return {op->d.WV, op->d.hv, op->d.S, op->d.Hoo, op->d.lambda, op->d.fr_val, op->d.tile_val};
}
template <>
DevPtrs<float> devptrs<float>(const oefe_op_s* op) {
  return {op->d.WVf, op->d.hvf, op->d.Sf, op->d.Hoof, op->d.lambdaf, op->d.fr_valf, op->d.tile_valf};
}

template <typename T, bool CPLX>
void small_gemm(const T* A, const T* B, int64_t ldb, T* C, int64_t ldc, int n, int k, int m, int mode, const T* x,
                const T* prev, int64_t ldx, int64_t ldo, double alpha, double c, double beta, hipStream_t s) {
  dim3 grid((unsigned)cdiv(m, 16), (unsigned)cdiv(n, 16));
  hipLaunchKernelGGL((small_gemm_kernel<T, CPLX>), grid, dim3(256), 0, s, A, B, ldb, C, ldc, n, k, m, mode, x, prev,
                     ldx, ldo, (T)alpha, (T)c, (T)beta);
}

template <typename T, bool CPLX>
int apply_step_impl(const oefe_op_s* op, const T* x, int64_t ld, const T* prev, T* out, int64_t ldout, int nv,
                    double alpha, double c, double beta, const StepWork& w, hipStream_t s) {
  const DevPtrs<T> dp = devptrs<T>(op);
  const int64_t ldx = CPLX ? 2 * ld : ld;
  const int64_t ldo = CPLX ? 2 * ldout : ldout;
  const int ncr = CPLX ? 2 * nv : nv;
  if (op->diagonal) {
    const int64_t tot = op->N * nv;
    hipLaunchKernelGGL((diag_step_kernel<T>), dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, dp.lambda, x, prev,
                       out, ldx, ldo, nv, op->N, (T)alpha, (T)c, (T)beta);
    return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
  }
  Phase3<T> ph;
  for (int d = 0; d < 3; ++d) {
    ph.re[d] = (T)op->phase[d][0];
    ph.im[d] = (T)op->phase[d][1];
  }
  const CellCoef<T>& cf = coef<T>(op);
  const int nO = op->n_enr;
  T* zo = (T*)w.zo;
  T* part = (T*)w.part;
  T* wp = (T*)w.wp;
  // Z^O = S X^O
  if (nO > 0)
    small_gemm<T, CPLX>(dp.S, x + op->N * ldx, ldx, zo, ncr, nO, nO, nv, 0, nullptr, nullptr, 0, 0, 0, 0, 0, s);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (op->timer_on && hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess)
    (void)hipEventRecord(ev0, s);
  launch_cell<T, CPLX>(op, x, ldx, ncr, (T*)w.ycell, w.ldc, dp.WV, cf, ph, s);
  if (ev1) {
    (void)hipEventRecord(ev1, s);
    op->timer_events.emplace_back(ev0, ev1);
  }
  // column block of the tiled kernels: all real columns up to 128, else near-equal blocks
  int CB = ncr <= 128 ? ncr : (int)cdiv(ncr, cdiv(ncr, 128));
  CB = (int)cdiv(CB, 8) * 8;
  const int ncb = (int)cdiv(ncr, CB);
  if (nO > 0) {
    const size_t lds = (size_t)(16 * CB + 16 * op->tile_fpmax * (CPLX ? 2 : 1)) * sizeof(T);
    hipLaunchKernelGGL((enr_tile_partial_kernel<T, CPLX>), dim3((unsigned)op->n_tiles, (unsigned)ncb), dim3(4 * CB),
                       lds, s, x, ldx, ncr, CB, op->d.tile_fptr, dp.tv, part, (int)op->N);
  }
  {
    const size_t lds = (size_t)(kTileRows * 16 * (CPLX ? 2 : 1) + 16 * CB) * sizeof(T);
    hipLaunchKernelGGL((fe_node_tile_kernel<T, CPLX>), dim3((unsigned)cdiv(op->N, kTileRows), (unsigned)ncb),
                       dim3(4 * CB), lds, s, (const T*)w.ycell, w.ldc, x, prev, out, ldx, ldo, ncr, CB, op->nc,
                       op->p, op->n, op->P1, cf, ph, zo, op->d.tile_fptr, op->d.tile_fns, dp.tv, (T)alpha, (T)c,
                       (T)beta, (int)op->N);
  }
  if (nO > 0) {
    hipLaunchKernelGGL((enr_tile_reduce_kernel<T>), dim3((unsigned)nO, (unsigned)cdiv(ncr, 64)), dim3(1024), 0, s,
                       part, op->d.fn_pptr, op->d.fn_poff, ncr, wp);
    // W' += H^oo Z^O ;  enrichment rows: alpha (S W' - c x) - beta prev
    small_gemm<T, CPLX>(dp.Hoo, zo, ncr, wp, ncr, nO, nO, nv, 1, nullptr, nullptr, 0, 0, 0, 0, 0, s);
    small_gemm<T, CPLX>(dp.S, wp, ncr, out + op->N * ldo, ldo, nO, nO, nv, 2, x + op->N * ldx,
                        prev ? prev + op->N * ldo : nullptr, ldx, ldo, alpha, c, beta, s);
  }
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
}

}  // namespace

size_t step_work_bytes(const oefe_op_s* op, int elem_bytes, bool cplx, int nv, int* ldc_out) {
  const int ncr = cplx ? 2 * nv : nv;
  const int ldc = (int)cdiv(ncr, 64) * 64;
  if (ldc_out) *ldc_out = ldc;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t bytes = 0;
  if (!op->diagonal) bytes += al((size_t)op->n_cells * op->nd * ldc * elem_bytes);
  bytes += al((size_t)std::max(op->n_enr, 1) * ncr * elem_bytes);                      // zo
  bytes += al((size_t)std::max<int64_t>(op->tile_slots, 1) * ncr * elem_bytes);  // part
  bytes += al((size_t)std::max(op->n_enr, 1) * ncr * elem_bytes);                      // wp
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
    p += al((size_t)op->n_cells * op->nd * ldc * elem_bytes);
  }
  w.zo = p;
  p += al((size_t)std::max(op->n_enr, 1) * ncr * elem_bytes);
  w.part = p;
  p += al((size_t)std::max<int64_t>(op->tile_slots, 1) * ncr * elem_bytes);
  w.wp = p;
  return w;
}

template <typename T>
int apply_step(const oefe_op_s* op, bool bf16, const T* x, int64_t ld, const T* prev, T* out, int64_t ldo, int nv,
               double alpha, double c, double beta, const StepWork& w, hipStream_t s) {
  if (bf16) return OEFE_EUNSUPPORTED;
  if (op->cplx) return apply_step_impl<T, true>(op, x, ld, prev, out, ldo, nv, alpha, c, beta, w, s);
  return apply_step_impl<T, false>(op, x, ld, prev, out, ldo, nv, alpha, c, beta, w, s);
}

template int apply_step<double>(const oefe_op_s*, bool, const double*, int64_t, const double*, double*, int64_t, int,
                                double, double, double, const StepWork&, hipStream_t);
template int apply_step<float>(const oefe_op_s*, bool, const float*, int64_t, const float*, float*, int64_t, int,
                               double, double, double, const StepWork&, hipStream_t);

template <typename T>
int zo_only(const oefe_op_s* op, const T* x, int64_t ld, int nv, T* zo, int ncr, hipStream_t s) {
  if (op->n_enr == 0) return OEFE_OK;
  const DevPtrs<T> dp = devptrs<T>(op);
  const int nO = op->n_enr;
  if (op->cplx)
    small_gemm<T, true>(dp.S, x + op->N * 2 * ld, 2 * ld, zo, ncr, nO, nO, nv, 0, nullptr, nullptr, 0, 0, 0, 0, 0, s);
  else
    small_gemm<T, false>(dp.S, x + op->N * ld, ld, zo, ncr, nO, nO, nv, 0, nullptr, nullptr, 0, 0, 0, 0, 0, s);
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
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

int density_final(const oefe_op_s* op, const double* dens, int nblk, double* dEdV, hipStream_t s) {
  const int64_t total = op->n_cells * op->nq;
  GW gw;
  for (int i = 0; i < 8; ++i) gw.w[i] = i < op->P1 ? op->gauss_w[i] : 0.0;
  const double h3 = (op->h / 2) * (op->h / 2) * (op->h / 2);
  hipLaunchKernelGGL(density_final_kernel2, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, dens, nblk, total,
                     op->P1, gw, h3, dEdV);
  return hipGetLastError() == hipSuccess ? OEFE_OK : OEFE_EDEVICE;
}

template int zo_only<double>(const oefe_op_s*, const double*, int64_t, int, double*, int, hipStream_t);
template int zo_only<float>(const oefe_op_s*, const float*, int64_t, int, float*, int, hipStream_t);
template int density_partial<double>(const oefe_op_s*, const double*, int64_t, int, const double*, const double*, int,
                                     double*, hipStream_t);
template int density_partial<float>(const oefe_op_s*, const float*, int64_t, int, const double*, const float*, int,
                                    double*, hipStream_t);

}  // namespace oefe
