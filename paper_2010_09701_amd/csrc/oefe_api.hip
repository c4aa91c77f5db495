// C ABI entry points (include/oefe.h): operator handles, device upload, and the
// compute calls built from the kernels in oefe_ops.hip / oefe_linalg.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "oefe_kernels.h"

// Scratch of the allocation-free entry point (cholgs_noalloc), 14 MiB per device.
constexpr size_t kScratchBytes = (size_t)14 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace oefe {

namespace {
thread_local std::string g_last_error;

template <typename T>
int dalloc(T** p, size_t count, std::string& err) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    err = std::string("hipMalloc failed: ") + hipGetErrorString(e);
    return OEFE_ENOMEM;
  }
  return OEFE_OK;
}
template <typename T>
int dput(T** p, const std::vector<T>& h, std::string& err) {
  int rc = dalloc(p, h.size(), err);
  if (rc) return rc;
  if (!h.empty()) {
    hipError_t e = hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      err = std::string("hipMemcpy failed: ") + hipGetErrorString(e);
      return OEFE_EDEVICE;
    }
  }
  return OEFE_OK;
}
template <typename T>
int dset(T* p, const std::vector<T>& h, std::string& err) {
  if (h.empty()) return OEFE_OK;
  hipError_t e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    err = std::string("hipMemcpy failed: ") + hipGetErrorString(e);
    return OEFE_EDEVICE;
  }
  return OEFE_OK;
}
template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

std::vector<float> to_float(const std::vector<double>& v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
  return o;
}

// complex host vector -> interleaved doubles (or real parts only)
std::vector<double> flatten(const std::vector<cplx>& v, bool cplx) {
  std::vector<double> o(v.size() * (cplx ? 2 : 1));
  for (size_t i = 0; i < v.size(); ++i) {
    if (cplx) {
      o[2 * i] = v[i].real();
      o[2 * i + 1] = v[i].imag();
    } else {
      o[i] = v[i].real();
    }
  }
  return o;
}

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return OEFE_EDEVICE;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

bool prec_real(int prec) { return prec == OEFE_F64 || prec == OEFE_F32 || prec == OEFE_BF16; }
bool prec_fp32(int prec) { return prec == OEFE_F32 || prec == OEFE_BF16 || prec == OEFE_C64; }

int check_prec(const oefe_op_s* op, int prec) {
  if (prec < OEFE_F64 || prec > OEFE_C64) return fail(OEFE_EINVAL, "unknown precision");
  if (op->cplx && prec_real(prec)) return fail(OEFE_EINVAL, "Bloch operator needs a complex precision (C128/C64)");
  if (!op->cplx && !prec_real(prec)) return fail(OEFE_EINVAL, "Gamma-point operator needs a real precision");
  return OEFE_OK;
}

// ---- layout of `work` beyond the operator step
struct Layout {
  StepWork step;
  size_t step_bytes;
  char* vecA;  // [n_tot x nv] complex-or-real doubles (E)
  char* vecB;
  double* G;       // nv*nv*E
  double* Rinv;    // nv*nv*E + nv
  double* U;       // nv*nv*E
  double* lam;     // nv
  double* gscr;    // gram scratch
  double* jscr;    // jacobi scratch
  double* misc;    // 512 doubles
  int32_t* status; // 4 ints
  double* dens;    // density partials
  size_t total;
};

int ncols_blocks(int ncr) { return (ncr + 63) / 64; }

Layout layout(const oefe_op_s* op, int prec, int nv, void* work) {
  Layout L{};
  const bool cplx = op->cplx;
  const int E = cplx ? 2 : 1;
  const int eb = prec_fp32(prec) ? 4 : 8;
  char* p = (char*)work;
  int ldc;
  L.step_bytes = al256(step_work_bytes(op, eb, cplx, nv, &ldc));
  if (work) L.step = carve_step_work(op, eb, cplx, nv, work);
  p += L.step_bytes;
  const size_t vb = al256((size_t)op->n_tot * nv * E * sizeof(double));
  L.vecA = p; p += vb;
  L.vecB = p; p += vb;
  const size_t sq = al256((size_t)nv * nv * E * sizeof(double));
  L.G = (double*)p; p += sq;
  L.Rinv = (double*)p; p += sq + al256(nv * sizeof(double));
  L.U = (double*)p; p += sq;
  L.lam = (double*)p; p += al256(nv * sizeof(double));
  const size_t gs = al256(std::max(gram_scratch_bytes(cplx, nv, nv, op->n_tot),
                                   (size_t)128 * nv * sizeof(double)));
  L.gscr = (double*)p; p += gs;
  L.jscr = (double*)p; p += al256(jacobi_scratch_bytes(cplx, nv));
  L.misc = (double*)p; p += 512 * sizeof(double);
  L.status = (int32_t*)p; p += 256;
  const size_t db = op->diagonal ? 256 : al256((size_t)ncols_blocks(cplx ? 2 * nv : nv) * op->n_cells * op->nq * sizeof(double));
  L.dens = (double*)p; p += db;
  L.total = (size_t)(p - (char*)work);
  return L;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

int upload_potential_parts(oefe_op_s* op, std::string& err) {
  const bool cplx = op->cplx;
  // W V at quadrature points
  std::vector<double> wv(op->V.size());
  for (size_t i = 0; i < wv.size(); ++i) wv[i] = op->W[i] * op->V[i];
  int rc;
  if (!op->d.WV) {
    if ((rc = dalloc(&op->d.WV, wv.size(), err))) return rc;
    if ((rc = dalloc(&op->d.WVf, wv.size(), err))) return rc;
  }
  if ((rc = dset(op->d.WV, wv, err))) return rc;
  if ((rc = dset(op->d.WVf, to_float(wv), err))) return rc;
  if (op->n_enr == 0) return OEFE_OK;
  // H^co values, scaled by m_g^-1/2 of their FE row: block-row layout and per-row CSR
  const int E = cplx ? 2 : 1;
  std::vector<double> hv((size_t)op->n_hrows * op->FMAX * E, 0.0);
  std::vector<double> frv((size_t)op->fr_nnz * E, 0.0);
  int64_t base = 0;
  for (size_t bi = 0; bi < op->blocks.size(); ++bi) {
    auto& b = op->blocks[bi];
    std::vector<std::complex<double>> vals;
    block_hco_values(op, b, vals);
    for (size_t r = 0; r < b.rows.size(); ++r) {
      const double ms = 1.0 / std::sqrt(op->mdiag[b.rows[r]]);
      for (int f = 0; f < b.nf; ++f) {
        const std::complex<double> v = ms * vals[r * b.nf + f];
        const size_t o = ((size_t)(base + r) * op->FMAX + f) * E;
        hv[o] = v.real();
        if (cplx) hv[o + 1] = v.imag();
        const size_t k = (size_t)(op->fr_pos[bi][r] + f) * E;
        frv[k] = v.real();
        if (cplx) frv[k + 1] = v.imag();
      }
    }
    base += (int64_t)b.rows.size();
  }
  if (!op->d.hv) {
    if ((rc = dalloc(&op->d.hv, hv.size(), err))) return rc;
    if ((rc = dalloc(&op->d.hvf, hv.size(), err))) return rc;
    if ((rc = dalloc(&op->d.fr_val, frv.size(), err))) return rc;
    if ((rc = dalloc(&op->d.fr_valf, frv.size(), err))) return rc;
    if ((rc = dalloc(&op->d.Hoo, (size_t)op->n_enr * op->n_enr * E, err))) return rc;
    if ((rc = dalloc(&op->d.Hoof, (size_t)op->n_enr * op->n_enr * E, err))) return rc;
  }
  if ((rc = dset(op->d.hv, hv, err))) return rc;
  if ((rc = dset(op->d.hvf, to_float(hv), err))) return rc;
  if ((rc = dset(op->d.fr_val, frv, err))) return rc;
  if ((rc = dset(op->d.fr_valf, to_float(frv), err))) return rc;
  {
    std::vector<double> tv((size_t)op->tile_slots * kTileRows * E, 0.0);
    for (int64_t k = 0; k < op->fr_nnz; ++k)
      for (int e = 0; e < E; ++e) tv[(size_t)op->csr_to_tile[k] * E + e] = frv[(size_t)k * E + e];
    if (!op->d.tile_val) {
      if ((rc = dalloc(&op->d.tile_val, tv.size(), err))) return rc;
      if ((rc = dalloc(&op->d.tile_valf, tv.size(), err))) return rc;
    }
    if ((rc = dset(op->d.tile_val, tv, err))) return rc;
    if ((rc = dset(op->d.tile_valf, to_float(tv), err))) return rc;
  }
  std::vector<double> hoo = flatten(op->Hoo, cplx);
  if ((rc = dset(op->d.Hoo, hoo, err))) return rc;
  if ((rc = dset(op->d.Hoof, to_float(hoo), err))) return rc;
  return OEFE_OK;
}

// Round-to-nearest-even float -> bf16 bit pattern (finite inputs).
uint16_t to_bf16_bits(double x) {
  const float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Dense cell matrices of the BF16 cell stage, padded to 128 x 128, in the A-fragment
// order of the 16x16x32 bf16 MFMA: entry (mb, kb, lane, t) = A[16 mb + lane % 16][32 kb + 8 (lane / 16) + t].
//   0: B   [q][a] = B1[qx][ax] B1[qy][ay] B1[qz][az]          (values at Gauss points)
//   1: K   [a][b] = kappa (S1 x M1 x M1 + M1 x S1 x M1 + M1 x M1 x S1)   (exact Gauss stiffness)
//   2: B^T [a][q] with the quadrature index of each 32-block in the order the MFMA
//      result of B Z leaves it in the lanes: position 8g + t is point 4g + t (t < 4)
//      or 16 + 4g + t - 4 (t >= 4) of the block.
std::vector<uint16_t> bf16_cell_matrices(const oefe_op_s* op) {
  const int P1 = op->P1, nd = P1 * P1 * P1;
  double M1[8][8] = {}, S1[8][8] = {};
  for (int a = 0; a < P1; ++a)
    for (int b = 0; b < P1; ++b)
      for (int q = 0; q < P1; ++q) {
        M1[a][b] += op->gauss_w[q] * op->B1[q][a] * op->B1[q][b];
        S1[a][b] += op->gauss_w[q] * op->D1[q][a] * op->D1[q][b];
      }
  const double kappa = op->h / 4.0;
  auto dec = [&](int a, int& x, int& y, int& z) { x = a % P1; y = (a / P1) % P1; z = a / (P1 * P1); };
  auto Bm = [&](int q, int a) {
    if (q >= nd || a >= nd) return 0.0;
    int qx, qy, qz, ax, ay, az;
    dec(q, qx, qy, qz);
    dec(a, ax, ay, az);
    return op->B1[qx][ax] * op->B1[qy][ay] * op->B1[qz][az];
  };
  auto Km = [&](int a, int b) {
    if (a >= nd || b >= nd) return 0.0;
    int ax, ay, az, bx, by, bz;
    dec(a, ax, ay, az);
    dec(b, bx, by, bz);
    return kappa * (S1[ax][bx] * M1[ay][by] * M1[az][bz] + M1[ax][bx] * S1[ay][by] * M1[az][bz] +
                    M1[ax][bx] * M1[ay][by] * S1[az][bz]);
  };
  std::vector<uint16_t> out(3 * 8 * 4 * 64 * 8);
  for (int w = 0; w < 3; ++w)
    for (int mb = 0; mb < 8; ++mb)
      for (int kb = 0; kb < 4; ++kb)
        for (int l = 0; l < 64; ++l)
          for (int t = 0; t < 8; ++t) {
            const int i = 16 * mb + l % 16, g = l / 16;
            const int k = 32 * kb + 8 * g + t;
            double v;
            if (w == 0) v = Bm(i, k);
            else if (w == 1) v = Km(i, k);
            else v = Bm(32 * kb + (t < 4 ? 4 * g + t : 16 + 4 * g + t - 4), i);
            out[((((size_t)w * 8 + mb) * 4 + kb) * 64 + l) * 8 + t] = to_bf16_bits(v);
          }
  return out;
}

int upload_operator(oefe_op_s* op, std::string& err) {
  int rc;
  const bool cplx = op->cplx;
  const int E = cplx ? 2 : 1;
  if (!cplx) {
    if ((rc = dput(&op->d.bf_mats, bf16_cell_matrices(op), err))) return rc;
  }
  if (op->n_enr > 0) {
    const int nb = (int)op->blocks.size();
    std::vector<int32_t> fn0(nb), nf(nb), fn_blk(op->n_enr), blk_chunk0(nb + 1);
    std::vector<int64_t> rptr(nb + 1, 0);
    std::vector<int32_t> rows;
    std::vector<int32_t> chunk_blk;
    std::vector<int64_t> chunk_r0, chunk_r1;
    for (int b = 0; b < nb; ++b) {
      auto& B = op->blocks[b];
      fn0[b] = B.fn0;
      nf[b] = B.nf;
      for (int f = 0; f < B.nf; ++f) fn_blk[B.fn0 + f] = b;
      rptr[b + 1] = rptr[b] + (int64_t)B.rows.size();
      rows.insert(rows.end(), B.rows.begin(), B.rows.end());
      blk_chunk0[b] = (int32_t)chunk_blk.size();
      for (int64_t r = 0; r < (int64_t)B.rows.size(); r += op->chunk_rows) {
        chunk_blk.push_back(b);
        chunk_r0.push_back(r);
        chunk_r1.push_back(std::min<int64_t>((int64_t)B.rows.size(), r + op->chunk_rows));
      }
    }
    blk_chunk0[nb] = (int32_t)chunk_blk.size();
    op->n_hrows = rptr[nb];
    op->n_chunks = (int64_t)chunk_blk.size();
    // forward CSR by FE row: entries ordered by block, then function
    std::vector<int64_t> fr_ptr(op->N + 1, 0);
    for (int b = 0; b < nb; ++b)
      for (int32_t g : op->blocks[b].rows) fr_ptr[g + 1] += op->blocks[b].nf;
    for (int64_t g = 0; g < op->N; ++g) fr_ptr[g + 1] += fr_ptr[g];
    op->fr_nnz = fr_ptr[op->N];
    std::vector<int32_t> fr_fn(op->fr_nnz);
    std::vector<int64_t> fill(fr_ptr.begin(), fr_ptr.end() - 1);
    op->fr_pos.assign(nb, {});
    for (int b = 0; b < nb; ++b) {
      auto& B = op->blocks[b];
      op->fr_pos[b].resize(B.rows.size());
      for (size_t r = 0; r < B.rows.size(); ++r) {
        const int64_t k = fill[B.rows[r]];
        fill[B.rows[r]] += B.nf;
        op->fr_pos[b][r] = k;
        for (int f = 0; f < B.nf; ++f) fr_fn[k + f] = B.fn0 + f;
      }
    }
    // enrichment tiles: union of functions over the rows of each tile (tile_node).  The block
    // shape (mode 1) is taken when it needs clearly fewer (tile, function) slots than runs of
    // consecutive rows (mode 0): where atoms are dense relative to the mesh.
    {
      struct Tiling {
        std::vector<int32_t> tfptr, tfns;
        std::vector<int64_t> csr_to_tile;
        int fpmax = 0;
      };
      auto build_tiles = [&](int mode, Tiling& T) {
        const int nt = tile_count(op->n, mode);
        T.tfptr.assign(nt + 1, 0);
        T.tfns.clear();
        T.csr_to_tile.assign(op->fr_nnz, 0);
        T.fpmax = 0;
        std::vector<int32_t> slot(op->n_enr, -1);
        for (int t = 0; t < nt; ++t) {
          std::vector<int32_t> fl;
          for (int r = 0; r < kTileRows; ++r) {
            const int g = tile_node(t, r, op->n, mode);
            if (g < 0) continue;
            for (int64_t k = fr_ptr[g]; k < fr_ptr[g + 1]; ++k)
              if (slot[fr_fn[k]] < 0) {
                slot[fr_fn[k]] = 0;
                fl.push_back(fr_fn[k]);
              }
          }
          std::sort(fl.begin(), fl.end());
          const int F = (int)fl.size(), FP = (F + 3) / 4 * 4;
          for (int j = 0; j < F; ++j) slot[fl[j]] = j;
          for (int r = 0; r < kTileRows; ++r) {
            const int g = tile_node(t, r, op->n, mode);
            if (g < 0) continue;
            for (int64_t k = fr_ptr[g]; k < fr_ptr[g + 1]; ++k)
              T.csr_to_tile[k] = (int64_t)T.tfptr[t] * kTileRows + (int64_t)r * FP + slot[fr_fn[k]];
          }
          for (int j = 0; j < FP; ++j) T.tfns.push_back(j < F ? fl[j] : -1);
          for (int32_t f : fl) slot[f] = -1;
          T.tfptr[t + 1] = T.tfptr[t] + FP;
          T.fpmax = std::max(T.fpmax, FP);
        }
      };
      Tiling T0, T1;
      build_tiles(0, T0);
      build_tiles(1, T1);
      const bool blocks_win = (double)T1.tfptr.back() <= 0.85 * (double)T0.tfptr.back();
      Tiling& T = blocks_win ? T1 : T0;
      op->tile_mode = blocks_win ? 1 : 0;
      op->n_tiles = tile_count(op->n, op->tile_mode);
      std::vector<int32_t> tfptr = std::move(T.tfptr), tfns = std::move(T.tfns);
      op->csr_to_tile = std::move(T.csr_to_tile);
      const int fpmax = T.fpmax;
      op->tile_slots = tfptr[op->n_tiles];
      op->tile_fpmax = fpmax;
      // the node-stage kernels hold one tile's dense block in LDS
      if (fpmax > kTileFunctionsMax) {
        err = "enrichment too dense for the node stage: a tile of " + std::to_string(kTileRows) +
              " FE nodes couples to " + std::to_string(fpmax) + " functions (at most " +
              std::to_string(kTileFunctionsMax) + ")";
        return OEFE_EINVAL;
      }
      // per function: its (tile, slot) partial positions, in tile order
      std::vector<int32_t> fpp(op->n_enr + 1, 0);
      for (int32_t f : tfns)
        if (f >= 0) fpp[f + 1]++;
      for (int f = 0; f < op->n_enr; ++f) fpp[f + 1] += fpp[f];
      std::vector<int32_t> fpo(fpp[op->n_enr]);
      std::vector<int32_t> ff(fpp.begin(), fpp.end() - 1);
      for (size_t q = 0; q < tfns.size(); ++q)
        if (tfns[q] >= 0) fpo[ff[tfns[q]]++] = (int32_t)q;
      op->fn_smax = 0;
      for (int f = 0; f < op->n_enr; ++f) op->fn_smax = std::max(op->fn_smax, fpp[f + 1] - fpp[f]);
      if ((rc = dput(&op->d.tile_fptr, tfptr, err))) return rc;
      if ((rc = dput(&op->d.tile_fns, tfns, err))) return rc;
      if ((rc = dput(&op->d.fn_pptr, fpp, err))) return rc;
      if ((rc = dput(&op->d.fn_poff, fpo, err))) return rc;
    }
    // N^O at quadrature points by cell
    std::vector<int64_t> cph_ptr(op->n_cells + 1, 0);
    for (auto& B : op->blocks)
      for (int64_t e : B.cells) cph_ptr[e + 1]++;
    for (int64_t e = 0; e < op->n_cells; ++e) cph_ptr[e + 1] += cph_ptr[e];
    std::vector<int32_t> cph_blk(cph_ptr[op->n_cells]);
    std::vector<int64_t> cph_off(cph_ptr[op->n_cells]);
    std::vector<int64_t> cfill(cph_ptr.begin(), cph_ptr.end() - 1);
    int64_t total_cells = 0;
    for (auto& B : op->blocks) total_cells += (int64_t)B.cells.size();
    std::vector<double> phi((size_t)total_cells * op->nq * op->FMAX * E, 0.0);
    int64_t off = 0;
    for (int b = 0; b < nb; ++b) {
      auto& B = op->blocks[b];
      for (size_t ci = 0; ci < B.cells.size(); ++ci) {
        const int64_t k = cfill[B.cells[ci]]++;
        cph_blk[k] = b;
        cph_off[k] = off + (int64_t)ci;
        for (int q = 0; q < op->nq; ++q)
          for (int f = 0; f < B.nf; ++f) {
            const std::complex<double> v = B.phi[(ci * op->nq + q) * B.nf + f];
            const size_t o = (((size_t)(off + ci) * op->nq + q) * op->FMAX + f) * E;
            phi[o] = v.real();
            if (cplx) phi[o + 1] = v.imag();
          }
      }
      off += (int64_t)B.cells.size();
    }
    // ---- structure of the device potential rebuild (oefe_op_set_potential)
    {
      const int P1 = op->P1, p = op->p, n = op->n, nc = op->nc;
      std::vector<int64_t> boff(nb + 1, 0);
      for (int b = 0; b < nb; ++b) boff[b + 1] = boff[b] + (int64_t)op->blocks[b].cells.size();
      std::vector<int32_t> cf_cell(boff[nb]);
      for (int b = 0; b < nb; ++b)
        for (size_t ci = 0; ci < op->blocks[b].cells.size(); ++ci) cf_cell[boff[b] + ci] = (int32_t)op->blocks[b].cells[ci];
      // block row -> (flattened support cell, local node) pairs, ordered by cell then node
      std::vector<int32_t> row_blk(op->n_hrows);
      std::vector<int64_t> rpos(op->n_hrows), rr_ptr(op->n_hrows + 1, 0);
      std::vector<int32_t> local(op->N, -1);
      for (int b = 0; b < nb; ++b) {
        auto& B = op->blocks[b];
        for (size_t r = 0; r < B.rows.size(); ++r) {
          row_blk[rptr[b] + r] = b;
          rpos[rptr[b] + r] = op->fr_pos[b][r];
        }
      }
      auto node_of = [&](int64_t e, int a) {
        const int cx = (int)(e % nc), cy = (int)((e / nc) % nc), cz = (int)(e / ((int64_t)nc * nc));
        const int ix = (cx * p + a % P1) % n, iy = (cy * p + (a / P1) % P1) % n, iz = (cz * p + a / (P1 * P1)) % n;
        return (int64_t)ix + (int64_t)n * (iy + (int64_t)n * iz);
      };
      for (int b = 0; b < nb; ++b) {  // count
        auto& B = op->blocks[b];
        for (size_t r = 0; r < B.rows.size(); ++r) local[B.rows[r]] = (int32_t)r;
        for (size_t ci = 0; ci < B.cells.size(); ++ci)
          for (int a = 0; a < op->nd; ++a) rr_ptr[rptr[b] + local[node_of(B.cells[ci], a)] + 1]++;
        for (size_t r = 0; r < B.rows.size(); ++r) local[B.rows[r]] = -1;
      }
      for (int64_t R = 0; R < op->n_hrows; ++R) rr_ptr[R + 1] += rr_ptr[R];
      {
        std::vector<int32_t> rr_ent(rr_ptr[op->n_hrows]);
        std::vector<int64_t> fillp(rr_ptr.begin(), rr_ptr.end() - 1);
        for (int b = 0; b < nb; ++b) {  // fill
          auto& B = op->blocks[b];
          for (size_t r = 0; r < B.rows.size(); ++r) local[B.rows[r]] = (int32_t)r;
          for (size_t ci = 0; ci < B.cells.size(); ++ci)
            for (int a = 0; a < op->nd; ++a) {
              const int64_t R = rptr[b] + local[node_of(B.cells[ci], a)];
              rr_ent[fillp[R]++] = (int32_t)((boff[b] + (int64_t)ci) * 128 + a);
            }
          for (size_t r = 0; r < B.rows.size(); ++r) local[B.rows[r]] = -1;
        }
        if ((rc = dput(&op->d.rr_ent, rr_ent, err))) return rc;
      }
      // kinetic part of H^co by block row
      std::vector<double> hkin((size_t)op->n_hrows * op->FMAX * E, 0.0);
      for (int b = 0; b < nb; ++b) {
        auto& B = op->blocks[b];
        for (size_t r = 0; r < B.rows.size(); ++r)
          for (int f = 0; f < B.nf; ++f) {
            const size_t o = ((size_t)(rptr[b] + r) * op->FMAX + f) * E;
            hkin[o] = B.hkin[r * B.nf + f].real();
            if (cplx) hkin[o + 1] = B.hkin[r * B.nf + f].imag();
          }
      }
      // common support cells of every pair of atom blocks (ascending cell index)
      std::vector<int64_t> hp_ptr((size_t)nb * nb + 1, 0);
      std::vector<int32_t> hp_i, hp_j;
      for (int bi = 0; bi < nb; ++bi)
        for (int bj = 0; bj < nb; ++bj) {
          auto& ci = op->blocks[bi].cells;
          auto& cj = op->blocks[bj].cells;
          size_t i = 0, j = 0;
          while (i < ci.size() && j < cj.size()) {
            if (ci[i] < cj[j]) { ++i; continue; }
            if (ci[i] > cj[j]) { ++j; continue; }
            hp_i.push_back((int32_t)(boff[bi] + (int64_t)i));
            hp_j.push_back((int32_t)(boff[bj] + (int64_t)j));
            ++i;
            ++j;
          }
          hp_ptr[(size_t)bi * nb + bj + 1] = (int64_t)hp_i.size();
        }
      if (hp_i.empty()) hp_i.push_back(0), hp_j.push_back(0);
      std::vector<double> msq(op->N);
      for (int64_t g = 0; g < op->N; ++g) msq[g] = 1.0 / std::sqrt(op->mdiag[g]);
      if ((rc = dput(&op->d.cf_cell, cf_cell, err))) return rc;
      if ((rc = dput(&op->d.row_blk, row_blk, err))) return rc;
      if ((rc = dput(&op->d.rpos, rpos, err))) return rc;
      if ((rc = dput(&op->d.rr_ptr, rr_ptr, err))) return rc;
      if ((rc = dput(&op->d.hkin, hkin, err))) return rc;
      if ((rc = dput(&op->d.hp_ptr, hp_ptr, err))) return rc;
      if ((rc = dput(&op->d.hp_i, hp_i, err))) return rc;
      if ((rc = dput(&op->d.hp_j, hp_j, err))) return rc;
      if ((rc = dput(&op->d.msq, msq, err))) return rc;
      std::vector<double> hook = flatten(op->Hoo_kin, cplx);
      if ((rc = dput(&op->d.Hoo_kin, hook, err))) return rc;
      if ((rc = dput(&op->d.csr2tile, op->csr_to_tile, err))) return rc;
      if (op->poisson && (rc = dput(&op->d.blk_cf0, boff, err))) return rc;
      // adaptive rule (oefe_op_create_adaptive): points, leaves, N^O at the points of every
      // flattened support cell, and the partials of the potential part of H^co
      if (op->adaptive) {
        std::vector<int32_t> cf_acell(boff[nb]);
        std::vector<int64_t> cf_aoff(boff[nb] + 1, 0);
        for (int b = 0; b < nb; ++b) {
          auto& B = op->blocks[b];
          for (size_t ci = 0; ci < B.cells.size(); ++ci) {
            const int64_t cf = boff[b] + (int64_t)ci;
            cf_acell[cf] = op->ad_index[B.cells[ci]];
            cf_aoff[cf + 1] = cf_aoff[cf] + (B.aoff[ci + 1] - B.aoff[ci]);
          }
        }
        std::vector<double> phiA((size_t)cf_aoff[boff[nb]] * op->FMAX * E, 0.0);
        for (int b = 0; b < nb; ++b) {
          auto& B = op->blocks[b];
          for (size_t ci = 0; ci < B.cells.size(); ++ci) {
            const int64_t cf = boff[b] + (int64_t)ci;
            for (int64_t r = 0; r < B.aoff[ci + 1] - B.aoff[ci]; ++r)
              for (int f = 0; f < B.nf; ++f) {
                const std::complex<double> v = B.phiA[(size_t)(B.aoff[ci] + r) * B.nf + f];
                const size_t o = ((size_t)(cf_aoff[cf] + r) * op->FMAX + f) * E;
                phiA[o] = v.real();
                if (cplx) phiA[o + 1] = v.imag();
              }
          }
        }
        if ((rc = dput(&op->d.a_w, op->ad_w, err))) return rc;
        if ((rc = dput(&op->d.a_V, op->ad_V, err))) return rc;
        if ((rc = dput(&op->d.a_leafB, op->ad_B, err))) return rc;
        if ((rc = dput(&op->d.a_off, op->ad_off, err))) return rc;
        if ((rc = dput(&op->d.cf_acell, cf_acell, err))) return rc;
        if ((rc = dput(&op->d.cf_aoff, cf_aoff, err))) return rc;
        if ((rc = dput(&op->d.phiA, phiA, err))) return rc;
        if (op->poisson && (rc = dput(&op->d.a_b, op->ad_b, err))) return rc;
      }
      // partials of the potential part of H^co per (flattened support cell, local node, function)
      if ((rc = dalloc(&op->d.hpart, (size_t)boff[nb] * op->nd * op->FMAX * E, err))) return rc;
      op->n_cf = boff[nb];
      // H^oo's potential part in chunks of each block pair's common cells: about 2048 workgroups
      op->hoo_nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(64, 2048 / ((int64_t)nb * nb)));
      if ((rc = dalloc(&op->d.hoo_part, (size_t)nb * nb * op->hoo_nchunk * op->FMAX * op->FMAX * E, err))) return rc;
    }
    if ((rc = dput(&op->d.blk_fn0, fn0, err))) return rc;
    if ((rc = dput(&op->d.blk_nf, nf, err))) return rc;
    if ((rc = dput(&op->d.fn_blk, fn_blk, err))) return rc;
    if ((rc = dput(&op->d.blk_rptr, rptr, err))) return rc;
    if ((rc = dput(&op->d.blk_rows, rows, err))) return rc;
    if ((rc = dput(&op->d.blk_chunk0, blk_chunk0, err))) return rc;
    if ((rc = dput(&op->d.chunk_blk, chunk_blk, err))) return rc;
    if ((rc = dput(&op->d.chunk_r0, chunk_r0, err))) return rc;
    if ((rc = dput(&op->d.chunk_r1, chunk_r1, err))) return rc;
    if ((rc = dput(&op->d.fr_ptr, fr_ptr, err))) return rc;
    if ((rc = dput(&op->d.fr_fn, fr_fn, err))) return rc;
    if ((rc = dput(&op->d.cph_ptr, cph_ptr, err))) return rc;
    if ((rc = dput(&op->d.cph_blk, cph_blk, err))) return rc;
    if ((rc = dput(&op->d.cph_off, cph_off, err))) return rc;
    if ((rc = dput(&op->d.phi, phi, err))) return rc;
    std::vector<double> S = flatten(op->S, cplx);
    if ((rc = dput(&op->d.S, S, err))) return rc;
    std::vector<float> Sf = to_float(S);
    if ((rc = dput(&op->d.Sf, Sf, err))) return rc;
  } else {
    // empty row lists so the node kernel can run without enrichment
    std::vector<int64_t> fr_ptr(op->N + 1, 0);
    if ((rc = dput(&op->d.fr_ptr, fr_ptr, err))) return rc;
  }
  if ((rc = dput(&op->d.W, op->W, err))) return rc;
  if ((rc = dput(&op->d.V, op->V, err))) return rc;
  if (op->poisson && (rc = dput(&op->d.bsmear, op->bsmear, err))) return rc;
  return upload_potential_parts(op, err);
}

void free_device(oefe_op_s* op) {
  auto& d = op->d;
  dfree(d.WV); dfree(d.WVf); dfree(d.blk_fn0); dfree(d.blk_nf); dfree(d.blk_rptr); dfree(d.blk_rows);
  dfree(d.tile_fptr); dfree(d.tile_fns); dfree(d.tile_val); dfree(d.tile_valf); dfree(d.fn_pptr);
  dfree(d.fn_poff); dfree(d.hv); dfree(d.hvf); dfree(d.fr_ptr); dfree(d.fr_fn); dfree(d.fr_val); dfree(d.fr_valf); dfree(d.chunk_blk);
  dfree(d.chunk_r0); dfree(d.chunk_r1); dfree(d.blk_chunk0); dfree(d.fn_blk); dfree(d.S); dfree(d.Hoo);
  dfree(d.Sf); dfree(d.Hoof); dfree(d.cph_ptr); dfree(d.cph_blk); dfree(d.cph_off); dfree(d.phi);
  dfree(d.lambda); dfree(d.lambdaf); dfree(d.bf_mats);
  dfree(d.W); dfree(d.V); dfree(d.msq); dfree(d.hkin); dfree(d.Hoo_kin); dfree(d.row_blk); dfree(d.rpos);
  dfree(d.a_w); dfree(d.a_V); dfree(d.a_leafB); dfree(d.a_off); dfree(d.cf_acell); dfree(d.cf_aoff);
  dfree(d.phiA); dfree(d.hpart); dfree(d.hoo_part); dfree(d.a_b);
  dfree(d.bsmear); dfree(d.blk_cf0); dfree(d.rr_ptr); dfree(d.rr_ent); dfree(d.cf_cell); dfree(d.csr2tile); dfree(d.hp_ptr); dfree(d.hp_i);
  dfree(d.hp_j);
}

}  // namespace oefe

using namespace oefe;

namespace {

// Achievable HBM rate: a grid-stride copy of 16-byte elements, four loads in flight per
// thread before their stores, non-temporal (streaming) loads and stores, and a grid of 64x the
// resident workgroups (the fastest of the shapes measured on this device: 5.3-5.5 TB/s).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void stream_copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                          int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Side stream and events of the overlapped recurrence (created once per operator).  The
// events only order kernels of the two streams on this device, so they skip the
// system-scope cache write-back and invalidation (no host or peer reads what they guard).
int overlap_setup(const oefe_op_s* op, Overlap* ov) {
  if (!op->side_stream) {
    const unsigned fl = hipEventDisableTiming | hipEventDisableSystemFence;
    hipError_t e = hipStreamCreateWithFlags(&op->side_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&op->ev_node, fl);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&op->ev_k1, fl);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&op->ev_zo, fl);
    if (e != hipSuccess) return hip_fail(e, "overlap stream setup");
  }
  ov->side = op->side_stream;
  ov->ev_node = op->ev_node;
  ov->ev_k1 = op->ev_k1;
  ov->ev_zo = op->ev_zo;
  ov->first = ov->last = false;
  return OEFE_OK;
}

// the device-bounds filter keeps its [m][3] scalars in the work buffer's misc area (512 doubles)
constexpr int kFilterDevMaxDegree = 160;

// ---- Potential-dependent operator data rebuilt on the device (oefe_op_set_potential).
// W V at the quadrature points (float64 and float32 copies)
__global__ void shift_kernel(double* __restrict__ v, double c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] += c;
}

__global__ void wv_kernel(const double* __restrict__ W, const double* __restrict__ V, double* __restrict__ WV,
                          float* __restrict__ WVf, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = W[i] * V[i];
  WV[i] = v;
  WVf[i] = (float)v;
}

// H^co (eqnHOEFEelelements, FE row g, enrichment function nu) = kinetic part (fixed) +
// sum over the (cell e, local node a) pairs of row g of conj(theta_ea) sum_q B[q, a] W_eq V_eq
// N^O_nu(x_eq), pre-scaled by m_g^-1/2 as the node stage uses it; one thread per (block row,
// function), pairs in ascending cell order, written to the block-row, CSR and tile layouts.
struct HcoRebuild {
  const double *W, *V, *phi, *msq, *hkin;
  const double* hpart;  // adaptive rule: the (support cell, local node, f) partials, else null
  const int64_t *rr_ptr, *rpos, *csr2tile;
  const int32_t *rr_ent, *cf_cell, *row_blk, *blk_nf, *blk_rows;
  double *hv, *fr_val, *tile_val;
  float *hvf, *fr_valf, *tile_valf;
  int64_t n_hrows;
  int FMAX, nq, P1, p, nc, n, nd;
  double ph[3][2];
};

// The potential part of H^co per (flattened support cell cf, local node a, function f): the sum
// over the cell's quadrature points x of ell_a(x) w V(x) N^O_f(x), over the cell's Gauss points or
// the leaves of the adaptive rule (Sec. III.B).  Per leaf: w V N^O staged in LDS, then the
// tensor contractions with the leaf's 1D Lagrange values, x, y, z in turn; one workgroup per cf
// accumulating its (a, f) items over the leaves in rule order (a fixed summation order).
struct HcoPart {
  const double *W, *V, *phi;  // the Gauss rule: weights, potential, N^O [cf][nq][FMAX]
  const int32_t* cf_cell;
  const double *a_w, *a_V, *a_leafB, *phiA;  // the adaptive rule (a_off null: the Gauss rule)
  const int64_t *a_off, *cf_aoff;
  const int32_t* cf_acell;
  double* hpart;
  int nd, P1, FMAX;
};

constexpr int kHcoItemsPerThread = 4;  // nd FMAX <= 125 * 8 items over 256 threads

template <bool CPLX>
__global__ __launch_bounds__(256) void hco_partial_kernel(HcoPart a, CellCoef<double> cd) {
  constexpr int E = CPLX ? 2 : 1;
  constexpr int kQ = kMaxP1 * kMaxP1 * kMaxP1;
  __shared__ double T[kQ * 8 * E], U[kQ * 8 * E];
  __shared__ double Bl[3][kMaxP1][kMaxP1];
  const int64_t cf = blockIdx.x;
  const int P1 = a.P1, nq = P1 * P1 * P1, F = a.FMAX;
  const int nitem = nq * F;  // (point or node, function)
  const bool adapt = a.a_off != nullptr;
  int64_t l0 = 0, l1 = 1, p0 = 0, r0 = cf * nq;
  int64_t e = 0;
  if (adapt) {
    const int k = a.cf_acell[cf];
    p0 = a.a_off[k];
    l0 = p0 / nq;
    l1 = a.a_off[k + 1] / nq;
    r0 = a.cf_aoff[cf];
  } else {
    e = a.cf_cell[cf];
  }
  double acc[kHcoItemsPerThread][E];
  for (int j = 0; j < kHcoItemsPerThread; ++j)
    for (int c = 0; c < E; ++c) acc[j][c] = 0.0;
  for (int64_t l = l0; l < l1; ++l) {
    __syncthreads();  // the previous leaf's last reads of T and Bl are done
    for (int i = threadIdx.x; i < 3 * P1 * P1; i += blockDim.x) {
      const int d = i / (P1 * P1), q = (i / P1) % P1, an = i % P1;
      Bl[d][q][an] = adapt ? a.a_leafB[((l * 3 + d) * P1 + q) * P1 + an] : cd.B1[q][an];
    }
    for (int i = threadIdx.x; i < nitem; i += blockDim.x) {
      const int q = i / F, f = i - q * F;
      double wv;
      const double* ph;
      if (adapt) {
        const int64_t gp = l * nq + q;
        wv = a.a_w[gp] * a.a_V[gp];
        ph = a.phiA + ((r0 + (gp - p0)) * F + f) * E;
      } else {
        wv = a.W[e * nq + q] * a.V[e * nq + q];
        ph = a.phi + ((r0 + q) * F + f) * E;
      }
      T[i * E] = wv * ph[0];
      if (CPLX) T[i * E + 1] = wv * ph[1];
    }
    __syncthreads();
    // x: U[(qz, qy, ax), f] = sum_qx B[qx][ax] T[(qz, qy, qx), f]
    for (int i = threadIdx.x; i < nitem; i += blockDim.x) {
      const int idx = i / F, f = i - idx * F;
      const int ax = idx % P1, qyz = idx / P1;
      double sr = 0.0, si = 0.0;
      for (int qx = 0; qx < P1; ++qx) {
        const double b = Bl[0][qx][ax];
        const int j = ((qyz * P1 + qx) * F + f) * E;
        sr += b * T[j];
        if (CPLX) si += b * T[j + 1];
      }
      U[i * E] = sr;
      if (CPLX) U[i * E + 1] = si;
    }
    __syncthreads();
    // y: T[(qz, ay, ax), f] = sum_qy B[qy][ay] U[(qz, qy, ax), f]
    for (int i = threadIdx.x; i < nitem; i += blockDim.x) {
      const int idx = i / F, f = i - idx * F;
      const int ax = idx % P1, ay = (idx / P1) % P1, qz = idx / (P1 * P1);
      double sr = 0.0, si = 0.0;
      for (int qy = 0; qy < P1; ++qy) {
        const double b = Bl[1][qy][ay];
        const int j = (((qz * P1 + qy) * P1 + ax) * F + f) * E;
        sr += b * U[j];
        if (CPLX) si += b * U[j + 1];
      }
      T[i * E] = sr;
      if (CPLX) T[i * E + 1] = si;
    }
    __syncthreads();
    // z: acc[(az, ay, ax), f] += sum_qz B[qz][az] T[(qz, ay, ax), f]
    int slot = 0;
    for (int i = threadIdx.x; i < nitem; i += blockDim.x, ++slot) {
      const int idx = i / F, f = i - idx * F;
      const int ax = idx % P1, ay = (idx / P1) % P1, az = idx / (P1 * P1);
      double sr = 0.0, si = 0.0;
      for (int qz = 0; qz < P1; ++qz) {
        const double b = Bl[2][qz][az];
        const int j = (((qz * P1 + ay) * P1 + ax) * F + f) * E;
        sr += b * T[j];
        if (CPLX) si += b * T[j + 1];
      }
      acc[slot][0] += sr;
      if (CPLX) acc[slot][E - 1] += si;
    }
  }
  int slot = 0;
  for (int i = threadIdx.x; i < nitem; i += blockDim.x, ++slot) {
    double* o = a.hpart + (cf * nitem + i) * E;  // (cf, local node, f): nitem = nd FMAX
    o[0] = acc[slot][0];
    if (CPLX) o[1] = acc[slot][E - 1];
  }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void hco_rebuild_kernel(HcoRebuild a) {
  constexpr int E = CPLX ? 2 : 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_hrows * a.FMAX) return;
  const int64_t R = t / a.FMAX;
  const int f = (int)(t - R * a.FMAX);
  if (f >= a.blk_nf[a.row_blk[R]]) return;
  const int P1 = a.P1;
  double sr = 0.0, si = 0.0;
  for (int64_t k = a.rr_ptr[R]; k < a.rr_ptr[R + 1]; ++k) {
    const int cf = a.rr_ent[k] >> 7, an = a.rr_ent[k] & 127;
    const int e = a.cf_cell[cf];
    const int ax = an % P1, ay = (an / P1) % P1, az = an / (P1 * P1);
    // the partial of this (support cell, local node, function) (hco_partial_kernel)
    const double* hp = a.hpart + (((int64_t)cf * a.nd + an) * a.FMAX + f) * E;
    const double vr = hp[0], vi = CPLX ? hp[1] : 0.0;
    if constexpr (CPLX) {
      // conj(theta) of the periodic image the node is reached through
      const int cx = e % a.nc, cy = (e / a.nc) % a.nc, cz = e / (a.nc * a.nc);
      double tr = 1.0, ti = 0.0;
      const bool wr[3] = {cx * a.p + ax >= a.n, cy * a.p + ay >= a.n, cz * a.p + az >= a.n};
      for (int d = 0; d < 3; ++d)
        if (wr[d]) {
          const double nr = tr * a.ph[d][0] - ti * a.ph[d][1], ni = tr * a.ph[d][1] + ti * a.ph[d][0];
          tr = nr;
          ti = ni;
        }
      sr += tr * vr + ti * vi;
      si += tr * vi - ti * vr;
    } else {
      sr += vr;
    }
  }
  const int g = a.blk_rows[R];
  const double ms = a.msq[g];
  const double* hk = a.hkin + (R * a.FMAX + f) * E;
  const double hr = ms * (hk[0] + sr), hi = CPLX ? ms * (hk[1] + si) : 0.0;
  const int64_t ob = (R * a.FMAX + f) * E, k = a.rpos[R] + f, tp = a.csr2tile[k] * E;
  a.hv[ob] = hr;
  a.hvf[ob] = (float)hr;
  a.fr_val[k * E] = hr;
  a.fr_valf[k * E] = (float)hr;
  a.tile_val[tp] = hr;
  a.tile_valf[tp] = (float)hr;
  if (CPLX) {
    a.hv[ob + 1] = hi;
    a.hvf[ob + 1] = (float)hi;
    a.fr_val[k * E + 1] = hi;
    a.fr_valf[k * E + 1] = (float)hi;
    a.tile_val[tp + 1] = hi;
    a.tile_valf[tp + 1] = (float)hi;
  }
}

// H^oo = kinetic part + sum over the common support cells (ascending) of two blocks and their
// quadrature points (the Gauss points, or the adaptive rule's points) of w V conj(N^O_i) N^O_j.
// One workgroup per (block pair (bi, bj), chunk of their common cells): thread t takes the entry
// item = t mod (nf_i nf_j) and the point lane t / (nf_i nf_j), lanes striding over each cell's
// points; the lanes' sums are added in lane order into the chunk's partial, and
// hoo_sum_kernel adds the chunks in order (a fixed summation order throughout).
struct HooPair {
  const double *W, *V, *phi;  // the Gauss rule
  const int32_t* cf_cell;
  const double *a_w, *a_V, *phiA;  // the adaptive rule (a_off null: the Gauss rule)
  const int64_t *a_off, *cf_aoff;
  const int32_t* cf_acell;
  const double* Hoo_kin;
  const int64_t* hp_ptr;
  const int32_t *hp_i, *hp_j, *blk_fn0, *blk_nf, *fn_blk;
  double* Hoo;
  float* Hoof;
  double* part;  // [pair][chunk][FMAX^2] (complex: x2)
  int nO, nb, FMAX, nq, nchunk;
};

template <bool CPLX>
__global__ __launch_bounds__(256) void hoo_pair_kernel(HooPair a) {
  constexpr int E = CPLX ? 2 : 1;
  __shared__ double red[256][E];
  const int pair = blockIdx.x / a.nchunk, chunk = blockIdx.x - pair * a.nchunk;
  const int bi = pair / a.nb, bj = pair - bi * a.nb;
  const int nfi = a.blk_nf[bi], nfj = a.blk_nf[bj], nit = nfi * nfj;
  const int lanes = (int)blockDim.x / nit;
  const int t = threadIdx.x, item = t % nit, lane = t / nit;
  const int f = item / nfj, g = item - f * nfj;
  const bool adapt = a.a_off != nullptr;
  const int F = a.FMAX;
  double sr = 0.0, si = 0.0;
  if (lane < lanes) {
    const int64_t pr = (int64_t)bi * a.nb + bj;
    const int64_t k0 = a.hp_ptr[pr], nk = a.hp_ptr[pr + 1] - k0;
    for (int64_t k = k0 + nk * chunk / a.nchunk; k < k0 + nk * (chunk + 1) / a.nchunk; ++k) {
      const int ci = a.hp_i[k], cj = a.hp_j[k];
      int64_t np, p0 = 0, e = 0;
      const double *pa, *pb;
      if (adapt) {
        const int kc = a.cf_acell[ci];
        p0 = a.a_off[kc];
        np = a.a_off[kc + 1] - p0;
        pa = a.phiA + (a.cf_aoff[ci] * F + f) * E;
        pb = a.phiA + (a.cf_aoff[cj] * F + g) * E;
      } else {
        e = a.cf_cell[ci];
        np = a.nq;
        pa = a.phi + ((int64_t)ci * a.nq * F + f) * E;
        pb = a.phi + ((int64_t)cj * a.nq * F + g) * E;
      }
      for (int64_t q = lane; q < np; q += lanes) {
        const double wv = adapt ? a.a_w[p0 + q] * a.a_V[p0 + q] : a.W[e * a.nq + q] * a.V[e * a.nq + q];
        const double ar = pa[q * F * E], ai = CPLX ? -pa[q * F * E + 1] : 0.0;
        const double br = pb[q * F * E], bim = CPLX ? pb[q * F * E + 1] : 0.0;
        const double xr = wv * ar, xi = wv * ai;
        sr += xr * br - xi * bim;
        if (CPLX) si += xr * bim + xi * br;
      }
    }
  }
  red[t][0] = sr;
  if (CPLX) red[t][E - 1] = si;
  __syncthreads();
  if (lane == 0) {
    double tr = 0.0, ti = 0.0;
    for (int l = 0; l < lanes; ++l) {
      tr += red[l * nit + item][0];
      if (CPLX) ti += red[l * nit + item][E - 1];
    }
    double* o = a.part + (((int64_t)pair * a.nchunk + chunk) * a.FMAX * a.FMAX + item) * E;
    o[0] = tr;
    if (CPLX) o[1] = ti;
  }
}

// H^oo[i][j] = kinetic part + the chunks' partials of the entry, in chunk order; one thread per entry.
template <bool CPLX>
__global__ __launch_bounds__(256) void hoo_sum_kernel(HooPair a) {
  constexpr int E = CPLX ? 2 : 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nO * a.nO) return;
  const int i = t / a.nO, j = t - i * a.nO;
  const int bi = a.fn_blk[i], bj = a.fn_blk[j];
  const int f = i - a.blk_fn0[bi], g = j - a.blk_fn0[bj];
  const int item = f * a.blk_nf[bj] + g;
  const int64_t pair = (int64_t)bi * a.nb + bj;
  double tr = a.Hoo_kin[(int64_t)t * E], ti = CPLX ? a.Hoo_kin[(int64_t)t * E + 1] : 0.0;
  for (int c = 0; c < a.nchunk; ++c) {
    const double* p = a.part + ((pair * a.nchunk + c) * a.FMAX * a.FMAX + item) * E;
    tr += p[0];
    if (CPLX) ti += p[1];
  }
  a.Hoo[(int64_t)t * E] = tr;
  a.Hoof[(int64_t)t * E] = (float)tr;
  if (CPLX) {
    a.Hoo[(int64_t)t * E + 1] = ti;
    a.Hoof[(int64_t)t * E + 1] = (float)ti;
  }
}

// ---- Occupations and Fermi level (eqnfd, eqnne) for the Ritz values of nk k-points, one
// workgroup: bisection on mu for 2 sum_k w_k sum f(theta, mu) = N_e (the count increases with
// mu), every count summed in a fixed order (each thread a fixed strided share, then a fixed
// tree), so the result is reproducible; then f and E_band = 2 sum_k w_k sum f theta.
constexpr int kOccMaxK = 64;
struct OccArgs {
  int nk;
  int off[kOccMaxK + 1];  // value offsets of the k-points in theta
  double w2[kOccMaxK];    // 2 w_k
};

__device__ double occ_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

__device__ double occ_count(const double* __restrict__ th, const OccArgs& a, double mu, double kT, double* red) {
  double s = 0.0;
  for (int k = 0; k < a.nk; ++k)
    for (int i = a.off[k] + (int)threadIdx.x; i < a.off[k + 1]; i += blockDim.x)
      s += a.w2[k] / (1.0 + exp((th[i] - mu) / kT));
  return occ_block_sum(s, red);
}

__global__ __launch_bounds__(1024) void occupations_kernel(const double* __restrict__ th, OccArgs a, double n_elec,
                                                           double kT, double* __restrict__ f, double* __restrict__ out,
                                                           int32_t* __restrict__ status) {
  __shared__ double red[16];
  const int ntot = a.off[a.nk];
  double lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < ntot; i += blockDim.x) {
    lo = fmin(lo, th[i]);
    hi = fmax(hi, th[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
  }
  __shared__ double mm[2][16];
  if ((threadIdx.x & 63) == 0) {
    mm[0][threadIdx.x >> 6] = lo;
    mm[1][threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  lo = INFINITY;
  hi = -INFINITY;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    lo = fmin(lo, mm[0][i]);
    hi = fmax(hi, mm[1][i]);
  }
  lo -= 50.0 * kT;
  hi += 50.0 * kT;
  const double cmax = occ_count(th, a, hi, kT, red);
  if (!(n_elec > 0.0 && n_elec < cmax)) {
    if (threadIdx.x == 0) {
      status[0] = OEFE_EINVAL;
      status[1] = 0;
    }
    return;
  }
  int it = 0;
  for (; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(mid))) break;
    if (occ_count(th, a, mid, kT, red) < n_elec) lo = mid;
    else hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  double eb = 0.0;
  for (int k = 0; k < a.nk; ++k)
    for (int i = a.off[k] + (int)threadIdx.x; i < a.off[k + 1]; i += blockDim.x) {
      const double fi = 1.0 / (1.0 + exp((th[i] - mu) / kT));
      f[i] = fi;
      eb += a.w2[k] * fi * th[i];
    }
  eb = occ_block_sum(eb, red);
  const double cnt = occ_count(th, a, mu, kT, red);
  if (threadIdx.x == 0) {
    out[0] = mu;
    out[1] = eb;
    out[2] = cnt;
    status[0] = 0;
    status[1] = it;
  }
}

// ---- allocation-free CholGS: its Gram, factor and flag scratch in the file-scope device
// array `scratch` (each device holds its own copy until the process ends).  Host code never
// passes the array's name to a kernel or a copy: its device address is taken once per device
// with hipGetSymbolAddress and kept in scratch_ptr.
constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kScratchDevices] = {};

// device address of `scratch` on the current device (nullptr and a message on failure)
void* scratch_address(std::string& err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) {
    err = "no usable HIP device";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

// Rayleigh-Ritz epilogue: the eigensolver status {code, sweeps} and the next pass's filter
// bounds (a = theta_nv, a0 = theta_1; b unchanged) from the ascending Ritz values.
__global__ void rr_finish_kernel(const double* __restrict__ lam, int nv, const int32_t* __restrict__ jst,
                                 int32_t* __restrict__ dev_status, double* __restrict__ next_bounds) {
  if (threadIdx.x != 0) return;
  if (dev_status) {
    dev_status[0] = jst[0];
    dev_status[1] = jst[1];
  }
  if (next_bounds) {
    next_bounds[0] = lam[nv - 1];
    next_bounds[2] = lam[0];
  }
}

template <typename T>
int filter_impl(oefe_op_s* op, bool bf16, T* X, int64_t ld, int nv, int m, double a, double b, double a0,
                const Layout& L, hipStream_t s, const double* dsc = nullptr) {
  // dsc (device [m][3], optional): the steps' scalars, computed on the device from device
  // bounds; a, b, a0 are then not used
  const double e = (b - a) / 2.0, c = (b + a) / 2.0;
  const double s1 = e / (a0 - c);
  const int64_t ldw = nv;  // second buffer is packed
  T* B = (T*)L.vecA;
  // the recurrence runs on (X, B) with in-place overwrite of the older iterate.
  // Buffers hold blocks with leading dimensions ld (X) and ldw (B); to keep one ld per
  // step, copy X into B's layout when ld != nv.
  T* cur;
  T* old;
  int64_t ldu;
  T* C = (T*)L.vecB;
  if (ld == ldw) {
    cur = X;
    old = B;
    ldu = ld;
  } else {
    // pack X into C
    const int E = op->cplx ? 2 : 1;
    int rc = cast_block(X, sizeof(T) == 4, C, sizeof(T) == 4, op->n_tot, ld * E, ldw * E, nv * E, s);
    if (rc) return rc;
    cur = C;
    old = B;
    ldu = ldw;
  }
  Overlap ov;
  if (int rc = overlap_setup(op, &ov)) return rc;
  // on an error the main stream still waits for the side chain already queued
  auto bail = [&](int rc) {
    if (rc != OEFE_EINVAL) (void)hipStreamWaitEvent(s, ov.ev_zo, 0);
    return rc;
  };
  // Y_1 = (s1/e)(H x - c x)  -> old buffer
  ov.first = true;
  ov.last = m == 1;
  int rc = apply_step<T>(op, bf16, cur, ldu, nullptr, old, ldu, nv, s1 / e, c, 0.0, L.step, s, &ov, dsc);
  if (rc) return bail(rc);
  std::swap(cur, old);  // cur = Y1, old = Y0
  double sig = s1;
  for (int k = 1; k < m; ++k) {
    const double sn = 1.0 / (2.0 / s1 - sig);
    ov.first = false;
    ov.last = k == m - 1;
    // (device scalars: the host beta only marks that prev is read)
    rc = apply_step<T>(op, bf16, cur, ldu, old, old, ldu, nv, 2.0 * sn / e, c, dsc ? 1.0 : sig * sn, L.step, s, &ov,
                       dsc ? dsc + 3 * k : nullptr);
    if (rc) return bail(rc);
    std::swap(cur, old);
    sig = sn;
  }
  if (cur != X) {
    const int E = op->cplx ? 2 : 1;
    rc = cast_block(cur, sizeof(T) == 4, X, sizeof(T) == 4, op->n_tot, ldu * E, ld * E, nv * E, s);
    if (rc) return rc;
  }
  return OEFE_OK;
}

}  // namespace

extern "C" {

const char* oefe_strerror(int code) {
  switch (code) {
    case OEFE_OK: return "ok";
    case OEFE_EINVAL: return "invalid argument";
    case OEFE_ENOMEM: return "out of device memory";
    case OEFE_EDEVICE: return "HIP runtime error";
    case OEFE_ENOTSPD: return "Gram matrix not positive definite (Cholesky breakdown)";
    case OEFE_ENOCONV: return "dense eigensolver did not converge";
    case OEFE_EUNSUPPORTED: return "unsupported precision, degree or operator kind";
    default: return "unknown status";
  }
}

const char* oefe_last_error(void) { return g_last_error.c_str(); }

int oefe_kernel_timer(oefe_op op, int which) {
  if (!op) return fail(OEFE_EINVAL, "null operator");
  if (which < OEFE_TIMER_OFF || which > OEFE_TIMER_COUPLING) return fail(OEFE_EINVAL, "unknown timer kind");
  for (auto& pr : op->timer_events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  op->timer_events.clear();
  op->timer_kind = which;
  return OEFE_OK;
}

int oefe_kernel_timer_read(oefe_op op, int64_t* launches, double* total_ms) {
  if (!op || !launches || !total_ms) return fail(OEFE_EINVAL, "null argument");
  double tot = 0.0;
  int64_t n = 0;
  int rc = OEFE_OK;
  for (auto& pr : op->timer_events) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(pr.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) rc = hip_fail(e, "oefe_kernel_timer_read");
    tot += ms;
    ++n;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  op->timer_events.clear();
  *launches = n;
  *total_ms = tot;
  return rc;
}

int oefe_copy_rate(const void* src, void* dst, size_t bytes, int32_t reps, double* gbs, oefe_stream stream) {
  if (!src || !dst || !gbs || bytes == 0 || reps < 1 || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
    return fail(OEFE_EINVAL, "oefe_copy_rate: bytes and both addresses must be positive multiples of 16");
  const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
  if (s0 < d0 + bytes && d0 < s0 + bytes) return fail(OEFE_EINVAL, "oefe_copy_rate: buffers overlap");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&stream_copy_kernel), 256, 0);
  if (e != hipSuccess) return hip_fail(e, "oefe_copy_rate");
  const int64_t n = (int64_t)(bytes / 16);
  const unsigned grid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * std::max(per_cu, 1) * 64, (n + 255) / 256));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::vector<float> ms;
  auto launch = [&] {
    hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n);
    return hipGetLastError();
  };
  if (e == hipSuccess) e = launch();  // warm-up
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    float t = 0.f;
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    ms.push_back(t);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "oefe_copy_rate");
  std::sort(ms.begin(), ms.end());
  const double med = ms[ms.size() / 2];
  *gbs = med > 0 ? 2.0 * (double)bytes / (med * 1e-3) / 1e9 : 0.0;
  return OEFE_OK;
}

static int rebuild_potential_device(oefe_op op, hipStream_t s);

// Arguments shared by the finite-element operators' create calls.
static int check_desc(const oefe_system_desc* desc, oefe_op* out) {
  if (!desc || !out) return fail(OEFE_EINVAL, "null argument");
  *out = nullptr;
  if (desc->n_atoms < 0 || desc->n_enr < 0 || (desc->n_atoms > 0 && (!desc->pos || !desc->Z)) ||
      (desc->n_enr > 0 && (!desc->enr_atom || !desc->enr_power || !desc->enr_zeta || !desc->enr_axis)))
    return fail(OEFE_EINVAL, "inconsistent system description");
  for (int nu = 0; nu < desc->n_enr; ++nu)
    if (desc->enr_power[nu] < 0 || desc->enr_axis[nu] < -1 || desc->enr_axis[nu] > 2 || !(desc->enr_zeta[nu] > 0))
      return fail(OEFE_EINVAL, "bad enrichment function parameters");
  return OEFE_OK;
}

// Host construction, upload and (adaptive rule) the potential parts on the device; frees `op`
// on failure.
static int finish_create(oefe_op_s* op, const oefe_system_desc* desc, oefe_op* out) {
  std::string err;
  int rc = build_operator(op, desc, err);
  if (rc == OEFE_OK && hipGetDevice(&op->device) != hipSuccess) {
    rc = OEFE_EDEVICE;
    err = "no HIP device";
  }
  if (rc == OEFE_OK) rc = upload_operator(op, err);
  // the allocation-free calls' scratch address on this device, taken at set-up
  if (rc == OEFE_OK && !scratch_address(err)) rc = OEFE_EDEVICE;
  if (rc == OEFE_OK && op->adaptive && op->n_enr > 0) {
    // the potential parts of the enrichment blocks under the adaptive rule
    rc = rebuild_potential_device(op, nullptr);
    if (rc == OEFE_OK && hipDeviceSynchronize() != hipSuccess) {
      rc = OEFE_EDEVICE;
      err = "potential rebuild failed";
    } else if (rc != OEFE_OK) {
      err = oefe_last_error();
    }
  }
  if (rc != OEFE_OK) {
    free_device(op);
    delete op;
    return fail(rc, err);
  }
  *out = op;
  return OEFE_OK;
}

int oefe_op_create(const oefe_system_desc* desc, oefe_op* out) {
  if (int rc = check_desc(desc, out)) return rc;
  oefe_op_s* op = new (std::nothrow) oefe_op_s();
  if (!op) return fail(OEFE_ENOMEM, "host allocation failed");
  return finish_create(op, desc, out);
}

int oefe_op_create_uform(const oefe_system_desc* desc, oefe_op* out) {
  if (int rc = check_desc(desc, out)) return rc;
  if (!desc->kvec) return fail(OEFE_EINVAL, "the periodic-function form needs a Bloch wavevector (kvec)");
  oefe_op_s* op = new (std::nothrow) oefe_op_s();
  if (!op) return fail(OEFE_ENOMEM, "host allocation failed");
  op->uform = true;
  return finish_create(op, desc, out);
}

int oefe_op_create_uform_adaptive(const oefe_system_desc* desc, double tol, int32_t max_depth, oefe_op* out) {
  if (int rc = check_desc(desc, out)) return rc;
  if (!desc->kvec) return fail(OEFE_EINVAL, "the periodic-function form needs a Bloch wavevector (kvec)");
  if (!(tol > 0.0 && tol < 1.0) || max_depth < 0 || max_depth > kAdaptMaxDepth)
    return fail(OEFE_EINVAL, "adaptive rule: need 0 < tol < 1 and 0 <= max_depth <= 5");
  if (desc->n_enr < 1) return fail(OEFE_EINVAL, "adaptive rule: no enrichment functions");
  oefe_op_s* op = new (std::nothrow) oefe_op_s();
  if (!op) return fail(OEFE_ENOMEM, "host allocation failed");
  op->uform = true;
  op->adaptive = true;
  op->ad_tol = tol;
  op->ad_depth = max_depth;
  return finish_create(op, desc, out);
}

int oefe_op_create_adaptive(const oefe_system_desc* desc, double tol, int32_t max_depth, oefe_op* out) {
  if (int rc = check_desc(desc, out)) return rc;
  if (!(tol > 0.0 && tol < 1.0) || max_depth < 0 || max_depth > kAdaptMaxDepth)
    return fail(OEFE_EINVAL, "adaptive rule: need 0 < tol < 1 and 0 <= max_depth <= 5");
  if (desc->n_enr < 1) return fail(OEFE_EINVAL, "adaptive rule: no enrichment functions");
  oefe_op_s* op = new (std::nothrow) oefe_op_s();
  if (!op) return fail(OEFE_ENOMEM, "host allocation failed");
  op->adaptive = true;
  op->ad_tol = tol;
  op->ad_depth = max_depth;
  return finish_create(op, desc, out);
}

int oefe_op_create_diagonal(const double* lambda, int64_t n, oefe_op* out) {
  if (!lambda || !out || n <= 0) return fail(OEFE_EINVAL, "bad diagonal operator arguments");
  oefe_op_s* op = new (std::nothrow) oefe_op_s();
  if (!op) return fail(OEFE_ENOMEM, "host allocation failed");
  op->diagonal = true;
  op->N = n;
  op->n_tot = n;
  std::vector<double> l(lambda, lambda + n);
  std::string err;
  int rc = dput(&op->d.lambda, l, err);
  if (!rc) rc = dput(&op->d.lambdaf, to_float(l), err);
  if (rc) {
    free_device(op);
    delete op;
    return fail(rc, err);
  }
  (void)hipGetDevice(&op->device);
  *out = op;
  return OEFE_OK;
}

int oefe_op_destroy(oefe_op op) {
  if (!op) return OEFE_OK;
  if (op->side_stream) {
    (void)hipStreamSynchronize(op->side_stream);
    (void)hipStreamDestroy(op->side_stream);
    (void)hipEventDestroy(op->ev_node);
    (void)hipEventDestroy(op->ev_k1);
    (void)hipEventDestroy(op->ev_zo);
  }
  free_device(op);
  delete op;
  return OEFE_OK;
}

int oefe_op_dims(oefe_op op, int64_t* dims) {
  if (!op || !dims) return fail(OEFE_EINVAL, "null argument");
  dims[0] = op->N;
  dims[1] = op->n_enr;
  dims[2] = op->n_tot;
  dims[3] = op->n_cells;
  dims[4] = op->nq;
  dims[5] = op->nc;
  dims[6] = op->p;
  dims[7] = op->cplx ? 1 : 0;
  dims[8] = op->n_enr > 0 ? op->tile_slots : 0;
  dims[9] = kTileRows;
  dims[10] = op->n_enr > 0 ? op->fr_nnz : 0;
  return OEFE_OK;
}

// The potential parts on the device from d.V (and, with the adaptive rule, d.a_V), queued on s:
// W V for the cell stage, H^co in every layout the kernels read, and H^oo.
static int rebuild_potential_device(oefe_op op, hipStream_t s) {
  const int64_t nqt = op->n_cells * op->nq;
  hipLaunchKernelGGL(wv_kernel, dim3((unsigned)((nqt + 255) / 256)), dim3(256), 0, s, op->d.W, op->d.V, op->d.WV,
                     op->d.WVf, nqt);
  if (op->n_enr > 0) {
    const bool ad = op->adaptive;
    HcoPart h{};
    h.W = op->d.W; h.V = op->d.V; h.phi = op->d.phi; h.cf_cell = op->d.cf_cell;
    if (ad) {
      h.a_w = op->d.a_w; h.a_V = op->d.a_V; h.a_leafB = op->d.a_leafB; h.phiA = op->d.phiA;
      h.a_off = op->d.a_off; h.cf_aoff = op->d.cf_aoff; h.cf_acell = op->d.cf_acell;
    }
    h.hpart = op->d.hpart;
    h.nd = op->nd; h.P1 = op->P1; h.FMAX = op->FMAX;
    if (op->cplx)
      hipLaunchKernelGGL(hco_partial_kernel<true>, dim3((unsigned)op->n_cf), dim3(256), 0, s, h, op->cd);
    else
      hipLaunchKernelGGL(hco_partial_kernel<false>, dim3((unsigned)op->n_cf), dim3(256), 0, s, h, op->cd);
    HcoRebuild a{};
    a.W = op->d.W; a.V = op->d.V; a.phi = op->d.phi; a.msq = op->d.msq; a.hkin = op->d.hkin;
    a.hpart = op->d.hpart;
    a.rr_ptr = op->d.rr_ptr; a.rpos = op->d.rpos; a.csr2tile = op->d.csr2tile;
    a.rr_ent = op->d.rr_ent; a.cf_cell = op->d.cf_cell; a.row_blk = op->d.row_blk; a.blk_nf = op->d.blk_nf;
    a.blk_rows = op->d.blk_rows;
    a.hv = op->d.hv; a.fr_val = op->d.fr_val; a.tile_val = op->d.tile_val;
    a.hvf = op->d.hvf; a.fr_valf = op->d.fr_valf; a.tile_valf = op->d.tile_valf;
    a.n_hrows = op->n_hrows;
    a.FMAX = op->FMAX; a.nq = op->nq; a.P1 = op->P1; a.p = op->p; a.nc = op->nc; a.n = op->n; a.nd = op->nd;
    for (int d = 0; d < 3; ++d) {
      a.ph[d][0] = op->phase[d][0];
      a.ph[d][1] = op->phase[d][1];
    }
    const unsigned g1 = (unsigned)((op->n_hrows * op->FMAX + 255) / 256);
    if (op->cplx)
      hipLaunchKernelGGL(hco_rebuild_kernel<true>, dim3(g1), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(hco_rebuild_kernel<false>, dim3(g1), dim3(256), 0, s, a);
    HooPair o{};
    o.W = op->d.W; o.V = op->d.V; o.phi = op->d.phi; o.cf_cell = op->d.cf_cell;
    if (ad) {
      o.a_w = op->d.a_w; o.a_V = op->d.a_V; o.phiA = op->d.phiA;
      o.a_off = op->d.a_off; o.cf_aoff = op->d.cf_aoff; o.cf_acell = op->d.cf_acell;
    }
    o.Hoo_kin = op->d.Hoo_kin; o.hp_ptr = op->d.hp_ptr; o.hp_i = op->d.hp_i; o.hp_j = op->d.hp_j;
    o.blk_fn0 = op->d.blk_fn0; o.blk_nf = op->d.blk_nf; o.fn_blk = op->d.fn_blk; o.Hoo = op->d.Hoo; o.Hoof = op->d.Hoof;
    o.part = op->d.hoo_part;
    const int nb = (int)op->blocks.size();
    o.nO = op->n_enr; o.nb = nb; o.FMAX = op->FMAX; o.nq = op->nq; o.nchunk = op->hoo_nchunk;
    const unsigned g3 = (unsigned)(((int64_t)op->n_enr * op->n_enr + 255) / 256);
    if (op->cplx) {
      hipLaunchKernelGGL(hoo_pair_kernel<true>, dim3((unsigned)(nb * nb * op->hoo_nchunk)), dim3(256), 0, s, o);
      hipLaunchKernelGGL(hoo_sum_kernel<true>, dim3(g3), dim3(256), 0, s, o);
    } else {
      hipLaunchKernelGGL(hoo_pair_kernel<false>, dim3((unsigned)(nb * nb * op->hoo_nchunk)), dim3(256), 0, s, o);
      hipLaunchKernelGGL(hoo_sum_kernel<false>, dim3(g3), dim3(256), 0, s, o);
    }
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "potential rebuild");
  return OEFE_OK;
}

int oefe_op_set_potential(oefe_op op, const double* V, oefe_stream stream) {
  if (!op || !V || op->diagonal) return fail(OEFE_EINVAL, "bad arguments");
  if (op->adaptive) return fail(OEFE_EINVAL, "an operator with the adaptive rule takes V at its points too (oefe_op_set_potential_adaptive)");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nqt = op->n_cells * op->nq;
  if (hipMemcpyAsync(op->d.V, V, (size_t)nqt * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(OEFE_EDEVICE, "oefe_op_set_potential: copy of V failed");
  if (op->vshift != 0.0)  // the periodic-function form's |k|^2/2 rides on V
    hipLaunchKernelGGL(shift_kernel, dim3((unsigned)((nqt + 255) / 256)), dim3(256), 0, s, op->d.V, op->vshift, nqt);
  return rebuild_potential_device(op, s);
}

int oefe_op_set_potential_adaptive(oefe_op op, const double* V, const double* V_adapt, oefe_stream stream) {
  if (!op || !V || !V_adapt || op->diagonal || !op->adaptive) return fail(OEFE_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nqt = op->n_cells * op->nq, np = op->ad_off.back();
  if (hipMemcpyAsync(op->d.V, V, (size_t)nqt * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(op->d.a_V, V_adapt, (size_t)np * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(OEFE_EDEVICE, "oefe_op_set_potential_adaptive: copy of V failed");
  if (op->vshift != 0.0) {  // the periodic-function form's |k|^2/2 rides on V
    hipLaunchKernelGGL(shift_kernel, dim3((unsigned)((nqt + 255) / 256)), dim3(256), 0, s, op->d.V, op->vshift, nqt);
    hipLaunchKernelGGL(shift_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, op->d.a_V, op->vshift, np);
  }
  return rebuild_potential_device(op, s);
}

int oefe_op_adaptive_points(oefe_op op, int64_t* n_points, double* xyz_host, double* w_host) {
  if (!op || !n_points || !op->adaptive) return fail(OEFE_EINVAL, "bad arguments");
  *n_points = op->ad_off.back();
  if (xyz_host) std::memcpy(xyz_host, op->ad_x.data(), op->ad_x.size() * sizeof(double));
  if (w_host) std::memcpy(w_host, op->ad_w.data(), op->ad_w.size() * sizeof(double));
  return OEFE_OK;
}

int oefe_op_get_potential(oefe_op op, double* V_host, double* W_host) {
  if (!op || op->diagonal) return fail(OEFE_EINVAL, "bad arguments");
  const size_t bytes = (size_t)op->n_cells * op->nq * sizeof(double);
  hipError_t e = hipDeviceSynchronize();  // after the set_potential calls queued on any stream
  if (e == hipSuccess && V_host) e = hipMemcpy(V_host, op->d.V, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess && W_host) e = hipMemcpy(W_host, op->d.W, bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "oefe_op_get_potential");
  if (V_host && op->vshift != 0.0)  // report the caller's V (without the form's |k|^2/2)
    for (size_t i = 0; i < bytes / sizeof(double); ++i) V_host[i] -= op->vshift;
  return OEFE_OK;
}

int oefe_op_get_enrichment(oefe_op op, double* S_host, double* eig_host) {
  if (!op || op->diagonal) return fail(OEFE_EINVAL, "bad arguments");
  const int n = op->n_enr;
  if (S_host)
    for (size_t i = 0; i < (size_t)n * n; ++i) {
      if (op->cplx) {
        S_host[2 * i] = op->S[i].real();
        S_host[2 * i + 1] = op->S[i].imag();
      } else {
        S_host[i] = op->S[i].real();
      }
    }
  if (eig_host) std::copy(op->Moo_eigs.begin(), op->Moo_eigs.end(), eig_host);
  return OEFE_OK;
}

size_t oefe_work_size(oefe_op op, oefe_prec prec, int32_t nv) {
  if (!op || nv <= 0) return 0;
  return layout(op, prec, nv, nullptr).total + 256;
}

int ham_apply(oefe_op op, oefe_prec prec, const void* X, void* Y, int64_t ld, int32_t nv, void* work,
              oefe_stream stream) {
  if (!op || !X || !Y || !work || nv <= 0 || ld < nv) return fail(OEFE_EINVAL, "bad arguments");
  if (int rc = check_prec(op, prec)) return rc;
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (prec_fp32(prec))
    rc = apply_step<float>(op, prec == OEFE_BF16, (const float*)X, ld, nullptr, (float*)Y, ld, nv, 1.0, 0.0, 0.0,
                           L.step, s);
  else
    rc = apply_step<double>(op, false, (const double*)X, ld, nullptr, (double*)Y, ld, nv, 1.0, 0.0, 0.0, L.step, s);
  if (rc == OEFE_EUNSUPPORTED) return fail(rc, "precision not supported by ham_apply");
  if (rc) return fail(rc, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
  return OEFE_OK;
}

int chebyshev_filter(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, int32_t m, double a, double b,
                     double a0, void* work, oefe_stream stream) {
  if (!op || !X || !work || nv <= 0 || ld < nv || m < 1) return fail(OEFE_EINVAL, "bad arguments");
  if (!(a < b) || !(a0 < a) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(a0))
    return fail(OEFE_EINVAL, "need a0 < a < b (finite)");
  if (int rc = check_prec(op, prec)) return rc;
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (prec_fp32(prec))
    rc = filter_impl<float>(op, prec == OEFE_BF16, (float*)X, ld, nv, m, a, b, a0, L, s);
  else
    rc = filter_impl<double>(op, false, (double*)X, ld, nv, m, a, b, a0, L, s);
  if (rc == OEFE_EUNSUPPORTED) return fail(rc, "precision not supported by chebyshev_filter");
  if (rc) return fail(rc, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
  return OEFE_OK;
}

int chebyshev_filter_dev(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, int32_t m,
                         const double* bounds, void* work, int32_t* dev_status, oefe_stream stream) {
  if (!op || !X || !work || !bounds || nv <= 0 || ld < nv || m < 1) return fail(OEFE_EINVAL, "bad arguments");
  if (m > kFilterDevMaxDegree) return fail(OEFE_EINVAL, "degree above the device-bounds limit");
  if (op->diagonal) return fail(OEFE_EUNSUPPORTED, "device bounds need a finite-element operator");
  if (int rc = check_prec(op, prec)) return rc;
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  double* dsc = L.misc + 32;  // [m][3]
  int rc = cheb_scalars(bounds, m, dsc, dev_status, s);
  // finite placeholders for the host-side recurrence (its values are not used)
  if (!rc) {
    if (prec_fp32(prec))
      rc = filter_impl<float>(op, prec == OEFE_BF16, (float*)X, ld, nv, m, 0.0, 2.0, -1.0, L, s, dsc);
    else
      rc = filter_impl<double>(op, false, (double*)X, ld, nv, m, 0.0, 2.0, -1.0, L, s, dsc);
  }
  if (rc == OEFE_EUNSUPPORTED) return fail(rc, "precision not supported by chebyshev_filter_dev");
  if (rc) return fail(rc, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
  return OEFE_OK;
}

int chebyshev_filter_mixed(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, int32_t m, double a,
                           double b, double a0, void* work, oefe_stream stream) {
  if (!op || !X || !work || nv <= 0 || ld < nv || m < 1) return fail(OEFE_EINVAL, "bad arguments");
  if (!(a < b) || !(a0 < a) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(a0))
    return fail(OEFE_EINVAL, "need a0 < a < b (finite)");
  if (!prec_fp32(prec)) return fail(OEFE_EINVAL, "chebyshev_filter_mixed needs a float32 filter precision");
  if (int rc = check_prec(op, prec)) return rc;
  const int E = op->cplx ? 2 : 1;
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  float* Xf = (float*)L.vecB;  // packed float32 copy
  int rc = cast_block(X, false, Xf, true, op->n_tot, ld * E, (int64_t)nv * E, nv * E, s);
  if (!rc) rc = filter_impl<float>(op, prec == OEFE_BF16, Xf, nv, nv, m, a, b, a0, L, s);
  if (!rc) rc = cast_block(Xf, true, X, false, op->n_tot, (int64_t)nv * E, ld * E, nv * E, s);
  if (rc == OEFE_EUNSUPPORTED) return fail(rc, "precision not supported by chebyshev_filter_mixed");
  if (rc) return fail(rc, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
  return OEFE_OK;
}

size_t oefe_batched_work_size(int32_t nk, const oefe_op* ops, oefe_prec prec, const int32_t* nv) {
  if (nk <= 0 || !ops || !nv) return 0;
  const int eb = prec_fp32(prec) ? 4 : 8;
  size_t tot = 0;
  for (int q = 0; q < nk; ++q) {
    if (!ops[q] || nv[q] <= 0) return 0;
    const int E = ops[q]->cplx ? 2 : 1;
    tot += al256(step_work_bytes(ops[q], eb, ops[q]->cplx, nv[q], nullptr));
    tot += 2 * al256((size_t)ops[q]->n_tot * nv[q] * E * eb);
  }
  return tot + 256;
}

int oefe_set_launch_shape(oefe_op op, int32_t cw, int32_t cb) {
  if (!op) return fail(OEFE_EINVAL, "null operator");
  if (!(cw == 0 || cw == 8 || cw == 16 || cw == 32 || cw == 64)) return fail(OEFE_EINVAL, "cw must be 0, 8, 16, 32 or 64");
  if (cb < 0 || cb > 128 || cb % 16) return fail(OEFE_EINVAL, "cb must be a multiple of 16 in [0, 128]");
  op->tune_cw = cw;
  op->tune_cb = cb;
  return OEFE_OK;
}

}  // extern "C"

namespace {
// Launch-shape tuner: times one batched operator step (out = alpha (Ht x - c x) - beta out,
// the filter's access pattern and stream overlap, bounded values) for each candidate
// cell-tile width cw and node-stage column width cb, and keeps the fastest on every operator.
template <typename T>
int autotune_impl(int nk, const oefe_op* ops, bool bf16, void* const* X, const int64_t* ld, const int32_t* nv,
                  int reps, void* work, int32_t* cw_out, int32_t* cb_out, double* ms_out, hipStream_t s) {
  const int eb = sizeof(T);
  std::vector<StepWork> sw(nk);
  std::vector<const T*> xin(nk), pin(nk);
  std::vector<T*> outp(nk);
  std::vector<int> nvv(nk);
  std::vector<int64_t> ldp(nk);
  std::vector<double> al(nk, 1e-3), cc(nk, 0.0), be(nk, 0.5);
  char* p = (char*)work;
  for (int q = 0; q < nk; ++q) {
    const int E = ops[q]->cplx ? 2 : 1;
    sw[q] = carve_step_work(ops[q], eb, ops[q]->cplx, nv[q], p);
    p += al256(step_work_bytes(ops[q], eb, ops[q]->cplx, nv[q], nullptr));
    T* A = (T*)p;
    p += al256((size_t)ops[q]->n_tot * nv[q] * E * eb);
    T* B = (T*)p;
    p += al256((size_t)ops[q]->n_tot * nv[q] * E * eb);
    int rc = cast_block(X[q], eb == 4, A, eb == 4, ops[q]->n_tot, ld[q] * E, (int64_t)nv[q] * E, nv[q] * E, s);
    if (!rc) rc = cast_block(X[q], eb == 4, B, eb == 4, ops[q]->n_tot, ld[q] * E, (int64_t)nv[q] * E, nv[q] * E, s);
    if (rc) return rc;
    xin[q] = A;
    pin[q] = B;
    outp[q] = B;
    nvv[q] = nv[q];
    ldp[q] = nv[q];
  }
  const oefe_op_s* const* opp = (const oefe_op_s* const*)ops;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return OEFE_EDEVICE;
  const int cws[5] = {0, 8, 16, 32, 64};
  const int cbs[4] = {16, 32, 64, 128};
  Overlap ov;
  if (int e = overlap_setup(opp[0], &ov)) return e;
  ov.first = ov.last = true;  // each timed step is a whole overlapped step
  double best = 1e300;
  int bcw = 0, bcb = 0, rc = OEFE_OK;
  // the periodic-function form runs on the planes-in-lanes cell kernel (cw = 0) only
  const int n_cw = opp[0]->uform ? 1 : 5;
  for (int a = 0; a < n_cw && !rc; ++a)
    for (int b = 0; b < 4 && !rc; ++b) {
      for (int q = 0; q < nk; ++q) {
        ops[q]->tune_cw = cws[a];
        ops[q]->tune_cb = cbs[b];
      }
      auto step = [&] {
        return apply_step_batch<T>(opp, nk, bf16, xin.data(), ldp.data(), pin.data(), outp.data(), ldp.data(),
                                   nvv.data(), al.data(), cc.data(), be.data(), sw.data(), s, &ov);
      };
      rc = step();  // warm-up (first launch of this instantiation)
      if (rc) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && !rc; ++r) rc = step();
      (void)hipEventRecord(e1, s);
      float ms = 0.f;
      if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = OEFE_EDEVICE;
      if (!rc && ms / reps < best) {
        best = ms / reps;
        bcw = cws[a];
        bcb = cbs[b];
      }
    }
  (void)hipStreamWaitEvent(s, ov.ev_zo, 0);  // side work of a step that stopped early
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int q = 0; q < nk; ++q) {
    ops[q]->tune_cw = rc ? 0 : bcw;
    ops[q]->tune_cb = rc ? 0 : bcb;
  }
  if (rc) return rc;
  if (cw_out) *cw_out = bcw;
  if (cb_out) *cb_out = bcb;
  if (ms_out) *ms_out = best;
  return OEFE_OK;
}

template <typename T>
int filter_batched_impl(int nk, const oefe_op* ops, bool bf16, void* const* X, const int64_t* ld, const int32_t* nv,
                        int m, const double* abc, void* work, hipStream_t s) {
  const int eb = sizeof(T);
  std::vector<StepWork> sw(nk);
  std::vector<T*> A(nk), B(nk);
  std::vector<int> nvv(nk);
  std::vector<int64_t> ldp(nk);
  char* p = (char*)work;
  for (int q = 0; q < nk; ++q) {
    const int E = ops[q]->cplx ? 2 : 1;
    sw[q] = carve_step_work(ops[q], eb, ops[q]->cplx, nv[q], p);
    p += al256(step_work_bytes(ops[q], eb, ops[q]->cplx, nv[q], nullptr));
    A[q] = (T*)p;
    p += al256((size_t)ops[q]->n_tot * nv[q] * E * eb);
    B[q] = (T*)p;
    p += al256((size_t)ops[q]->n_tot * nv[q] * E * eb);
    nvv[q] = nv[q];
    ldp[q] = nv[q];
    int rc = cast_block(X[q], eb == 4, A[q], eb == 4, ops[q]->n_tot, ld[q] * E, (int64_t)nv[q] * E, nv[q] * E, s);
    if (rc) return rc;
  }
  std::vector<double> e(nk), c(nk), s1(nk), sig(nk), al(nk), be(nk);
  for (int q = 0; q < nk; ++q) {
    const double a = abc[3 * q], b = abc[3 * q + 1], a0 = abc[3 * q + 2];
    e[q] = (b - a) / 2.0;
    c[q] = (b + a) / 2.0;
    s1[q] = e[q] / (a0 - c[q]);
    sig[q] = s1[q];
  }
  std::vector<const T*> xin(nk), pin(nk);
  std::vector<T*> outp(nk);
  const oefe_op_s* const* opp = (const oefe_op_s* const*)ops;
  // Y_1 = (s1/e)(H x - c x): cur = A, result into B
  for (int q = 0; q < nk; ++q) {
    xin[q] = A[q];
    pin[q] = nullptr;
    outp[q] = B[q];
    al[q] = s1[q] / e[q];
    be[q] = 0.0;
  }
  Overlap ov;
  if (int rc = overlap_setup(opp[0], &ov)) return rc;
  auto bail = [&](int rc) {
    if (rc != OEFE_EINVAL) (void)hipStreamWaitEvent(s, ov.ev_zo, 0);
    return rc;
  };
  ov.first = true;
  ov.last = m == 1;
  int rc = apply_step_batch<T>(opp, nk, bf16, xin.data(), ldp.data(), pin.data(), outp.data(), ldp.data(), nvv.data(),
                               al.data(), c.data(), be.data(), sw.data(), s, &ov);
  if (rc) return bail(rc);
  T** cur = B.data();
  T** old = A.data();
  for (int k = 1; k < m; ++k) {
    ov.first = false;
    ov.last = k == m - 1;
    for (int q = 0; q < nk; ++q) {
      const double sn = 1.0 / (2.0 / s1[q] - sig[q]);
      xin[q] = cur[q];
      pin[q] = old[q];
      outp[q] = old[q];
      al[q] = 2.0 * sn / e[q];
      be[q] = sig[q] * sn;
      sig[q] = sn;
    }
    rc = apply_step_batch<T>(opp, nk, bf16, xin.data(), ldp.data(), pin.data(), outp.data(), ldp.data(), nvv.data(),
                             al.data(), c.data(), be.data(), sw.data(), s, &ov);
    if (rc) return bail(rc);
    std::swap(cur, old);
  }
  for (int q = 0; q < nk; ++q) {
    const int E = ops[q]->cplx ? 2 : 1;
    rc = cast_block(cur[q], eb == 4, X[q], eb == 4, ops[q]->n_tot, (int64_t)nv[q] * E, ld[q] * E, nv[q] * E, s);
    if (rc) return rc;
  }
  return OEFE_OK;
}
}  // namespace

extern "C" {

int chebyshev_filter_batched(int32_t nk, const oefe_op* ops, oefe_prec prec, void* const* X, const int64_t* ld,
                             const int32_t* nv, int32_t m, const double* abc, void* work, oefe_stream stream) {
  if (nk <= 0 || !ops || !X || !ld || !nv || !abc || !work || m < 1) return fail(OEFE_EINVAL, "bad arguments");
  for (int q = 0; q < nk; ++q) {
    if (!ops[q] || !X[q] || nv[q] <= 0 || ld[q] < nv[q]) return fail(OEFE_EINVAL, "bad per-operator arguments");
    if (int rc = check_prec(ops[q], prec)) return rc;
    const oefe_op_s* a = ops[0];
    const oefe_op_s* b = ops[q];
    if (b->diagonal || a->diagonal || b->nc != a->nc || b->p != a->p || b->L != a->L || b->n_enr != a->n_enr ||
        b->n_tiles != a->n_tiles || b->tile_mode != a->tile_mode || b->tile_slots != a->tile_slots ||
        b->tile_fpmax != a->tile_fpmax)
      return fail(OEFE_EINVAL, "batched operators must share the mesh and the enrichment layout");
    const double aa = abc[3 * q], bb = abc[3 * q + 1], a0 = abc[3 * q + 2];
    if (!(aa < bb) || !(a0 < aa)) return fail(OEFE_EINVAL, "need a0 < a < b for every operator");
  }
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (prec_fp32(prec))
    rc = filter_batched_impl<float>(nk, ops, prec == OEFE_BF16, X, ld, nv, m, abc, work, s);
  else
    rc = filter_batched_impl<double>(nk, ops, false, X, ld, nv, m, abc, work, s);
  if (rc == OEFE_EUNSUPPORTED) return fail(rc, "precision not supported by chebyshev_filter_batched");
  if (rc) return fail(rc, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
  return OEFE_OK;
}

int oefe_autotune(int32_t nk, const oefe_op* ops, oefe_prec prec, void* const* X, const int64_t* ld, const int32_t* nv,
                  int32_t reps, void* work, int32_t* cw_out, int32_t* cb_out, double* ms_per_step,
                  oefe_stream stream) {
  if (nk <= 0 || !ops || !X || !ld || !nv || !work || reps <= 0) return fail(OEFE_EINVAL, "bad arguments");
  for (int q = 0; q < nk; ++q) {
    if (!ops[q] || ops[q]->diagonal || !X[q] || nv[q] <= 0 || ld[q] < nv[q]) return fail(OEFE_EINVAL, "bad block");
    if (int rc = check_prec(ops[q], prec)) return rc;
    const oefe_op_s* a = ops[0];
    const oefe_op_s* b = ops[q];
    if (b->nc != a->nc || b->p != a->p || b->L != a->L || b->n_enr != a->n_enr || b->cplx != a->cplx ||
        b->n_tiles != a->n_tiles || b->tile_mode != a->tile_mode || b->tile_slots != a->tile_slots ||
        b->tile_fpmax != a->tile_fpmax)
      return fail(OEFE_EINVAL, "operators must share mesh and enrichment layout");
  }
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (prec_fp32(prec))
    rc = autotune_impl<float>(nk, ops, prec == OEFE_BF16, X, ld, nv, reps, work, cw_out, cb_out, ms_per_step, s);
  else
    rc = autotune_impl<double>(nk, ops, false, X, ld, nv, reps, work, cw_out, cb_out, ms_per_step, s);
  if (rc == OEFE_EUNSUPPORTED) return fail(rc, "precision not supported by oefe_autotune");
  if (rc) return fail(rc, "oefe_autotune failed");
  return OEFE_OK;
}

// CholGS on the matrix-core path without host round trips (the Gram matrix of X is in L.G):
// device flags decide (status[2]: pass 1 factored, status[3]: repeat wanted, status[4]: pass 2
// factored); {code, column} ends in L.status[0..1] and, when given, in dev_status.
static int cholgs_gated_enqueue(oefe_op op, const Layout& L, bool cplx, double* Xd, int64_t ld, int32_t nv,
                                int32_t* dev_status, hipStream_t s) {
  int32_t* st = L.status;
  int rc = hermitian_part(cplx, L.G, nv, s);
  if (!rc) rc = chol_factor_inverse(cplx, L.G, nv, nv, L.Rinv, st, s, nullptr, st + 2);
  if (!rc) rc = rowmul_inplace(Xd, ld, op->n_tot, nv, L.Rinv, s, st + 2);
  if (!rc) rc = gram(cplx, Xd, ld, nv, Xd, ld, nv, op->n_tot, L.G, nv, L.gscr, (size_t)1 << 62, s);
  if (!rc) rc = max_offdiag_identity(cplx, L.G, nv, L.misc, s, st, st + 3, 1e-12);
  if (!rc) rc = hermitian_part(cplx, L.G, nv, s, st + 3);
  if (!rc) rc = chol_factor_inverse(cplx, L.G, nv, nv, L.Rinv, st, s, st + 3, st + 4);
  if (!rc) rc = rowmul_inplace(Xd, ld, op->n_tot, nv, L.Rinv, s, st + 4);
  if (!rc && dev_status && hipMemcpyAsync(dev_status, st, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
    rc = OEFE_EDEVICE;
  return rc;
}

int cholgs(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, void* work, int32_t* dev_status,
           oefe_stream stream) {
  if (!op || !X || !work || nv <= 0 || ld < nv) return fail(OEFE_EINVAL, "bad arguments");
  if (prec != OEFE_F64 && prec != OEFE_C128) return fail(OEFE_EINVAL, "cholgs runs in float64 (F64 or C128)");
  if (int rc = check_prec(op, prec)) return rc;
  const bool cplx = op->cplx;
  const int E = cplx ? 2 : 1;
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  double* Xd = (double*)X;
  double* tmp = (double*)L.vecA;
  // Pass 1 factors the Gram matrix of X; its orthogonality check computes Q^* Q, which is
  // exactly the Gram matrix the (at most one) repeated pass factors.
  int rc = gram(cplx, Xd, ld, nv, Xd, ld, nv, op->n_tot, L.G, nv, L.gscr, (size_t)1 << 62, s);
  if (rc) return fail(rc, "cholgs: kernel launch failed");
  if (cholgs_device_gated(cplx, nv)) {
    rc = cholgs_gated_enqueue(op, L, cplx, Xd, ld, nv, dev_status, s);
    if (rc) return fail(rc, "cholgs: kernel launch failed");
    int32_t* st = L.status;
    int32_t h[2];
    hipError_t he = hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "cholgs");
    if (h[0] != 0)
      return fail(OEFE_ENOTSPD, "cholgs: Gram matrix not positive definite at column " + std::to_string(h[1]));
    return OEFE_OK;
  }
  for (int it = 0; it < 2; ++it) {
    rc = hermitian_part(cplx, L.G, nv, s);
    if (!rc) rc = chol_factor_inverse(cplx, L.G, nv, nv, L.Rinv, L.status, s);
    if (rc) return fail(rc, "cholgs: kernel launch failed");
    int32_t st[2];
    hipError_t he = hipMemcpyAsync(st, L.status, sizeof(st), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "cholgs");
    if (st[0] != 0) {
      if (dev_status) (void)hipMemcpyAsync(dev_status, L.status, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
      (void)hipStreamSynchronize(s);
      return fail(OEFE_ENOTSPD, "cholgs: Gram matrix not positive definite at column " + std::to_string(st[1]));
    }
    if (rowmul_on_mfma(cplx, nv)) {
      rc = rowmul_inplace(Xd, ld, op->n_tot, nv, L.Rinv, s);
    } else {
      rc = gemm_nn(cplx, Xd, ld, L.Rinv, nv, tmp, nv, op->n_tot, nv, nv, s);
      if (!rc) rc = copy_block(tmp, (int64_t)nv * E, Xd, ld * E, op->n_tot, nv * E, s);
    }
    if (rc) return fail(rc, "cholgs: kernel launch failed");
    if (it == 1) break;  // repeated once at most
    // orthogonality check on Q^* Q
    rc = gram(cplx, Xd, ld, nv, Xd, ld, nv, op->n_tot, L.G, nv, L.gscr, (size_t)1 << 62, s);
    if (!rc) rc = max_offdiag_identity(cplx, L.G, nv, L.misc, s);
    if (rc) return fail(rc, "cholgs: kernel launch failed");
    double errv = 0;
    he = hipMemcpyAsync(&errv, L.misc, sizeof(double), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "cholgs");
    if (!(errv > 1e-12)) break;
  }
  if (dev_status) {
    int32_t ok[2] = {0, -1};
    (void)hipMemcpyAsync(dev_status, ok, sizeof(ok), hipMemcpyHostToDevice, s);
    (void)hipStreamSynchronize(s);
  }
  return OEFE_OK;
}

int cholgs_async(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, void* work, int32_t* dev_status,
                 oefe_stream stream) {
  if (!op || !X || !work || !dev_status || nv <= 0 || ld < nv) return fail(OEFE_EINVAL, "bad arguments");
  if (prec != OEFE_F64 && prec != OEFE_C128) return fail(OEFE_EINVAL, "cholgs runs in float64 (F64 or C128)");
  if (int rc = check_prec(op, prec)) return rc;
  const bool cplx = op->cplx;
  if (!cholgs_device_gated(cplx, nv)) return cholgs(op, prec, X, ld, nv, work, dev_status, stream);
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  double* Xd = (double*)X;
  int rc = gram(cplx, Xd, ld, nv, Xd, ld, nv, op->n_tot, L.G, nv, L.gscr, (size_t)1 << 62, s);
  if (!rc) rc = cholgs_gated_enqueue(op, L, cplx, Xd, ld, nv, dev_status, s);
  if (rc) return fail(rc, "cholgs_async: kernel launch failed");
  return OEFE_OK;
}

int cholgs_noalloc(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, int32_t* dev_status,
                   oefe_stream stream) {
  if (!op || !X || !dev_status || nv <= 0 || ld < nv) return fail(OEFE_EINVAL, "bad arguments");
  if (prec != OEFE_F64) return fail(OEFE_EUNSUPPORTED, "cholgs_noalloc takes real float64 blocks (F64)");
  if (int rc = check_prec(op, prec)) return rc;
  if (op->diagonal || !cholgs_device_gated(false, nv))
    return fail(OEFE_EUNSUPPORTED, "cholgs_noalloc takes 1..80 columns of a finite-element operator");
  // scratch layout: G [nv^2], factor inverse [nv^2 + nv], Gram chunk partials, 512 doubles, flags
  const size_t sq = al256((size_t)nv * nv * sizeof(double));
  const size_t gs = al256(gram_scratch_bytes(false, nv, nv, op->n_tot));
  const size_t need = sq + sq + al256((size_t)nv * sizeof(double)) + gs + 512 * sizeof(double) + 256;
  if (need > kScratchBytes)
    return fail(OEFE_EINVAL, "cholgs_noalloc: the block needs " + std::to_string(need) +
                                 " bytes of scratch, more than the " + std::to_string(kScratchBytes) + " available");
  std::string err;
  char* base = (char*)scratch_address(err);
  if (!base) return fail(OEFE_EDEVICE, err);
  Layout L{};
  char* p = base;
  L.G = (double*)p; p += sq;
  L.Rinv = (double*)p; p += sq + al256((size_t)nv * sizeof(double));
  L.gscr = (double*)p; p += gs;
  L.misc = (double*)p; p += 512 * sizeof(double);
  L.status = (int32_t*)p;
  hipStream_t s = (hipStream_t)stream;
  double* Xd = (double*)X;
  int rc = gram(false, Xd, ld, nv, Xd, ld, nv, op->n_tot, L.G, nv, L.gscr, gs, s);
  if (!rc) rc = cholgs_gated_enqueue(op, L, false, Xd, ld, nv, dev_status, s);
  if (rc) return fail(rc, "cholgs_noalloc: kernel launch failed");
  return OEFE_OK;
}

int rayleigh_ritz(oefe_op op, oefe_prec prec, void* Q, int64_t ld, int32_t nv, double* eigvals, void* work,
                  int32_t* dev_status, double* next_bounds, oefe_stream stream) {
  if (!op || !Q || !eigvals || !work || nv <= 0 || ld < nv) return fail(OEFE_EINVAL, "bad arguments");
  if (prec != OEFE_F64 && prec != OEFE_C128) return fail(OEFE_EINVAL, "rayleigh_ritz runs in float64 (F64 or C128)");
  if (int rc = check_prec(op, prec)) return rc;
  const bool cplx = op->cplx;
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  double* Qd = (double*)Q;
  double* W = (double*)L.vecA;  // packed [n_tot x nv]
  // W = Ht Q
  int rc = apply_step<double>(op, false, Qd, ld, nullptr, W, nv, nv, 1.0, 0.0, 0.0, L.step, s);
  if (rc) return fail(rc, "rayleigh_ritz: operator step failed");
  // Hq = Q^* W (Hermitian part), Hq = U diag(theta) U^*
  rc = gram(cplx, Qd, ld, nv, W, nv, nv, op->n_tot, L.G, nv, L.gscr, (size_t)1 << 62, s);
  if (!rc) rc = hermitian_part(cplx, L.G, nv, s);
  if (!rc) rc = jacobi_eig(cplx, L.G, nv, eigvals, L.U, L.jscr, L.status, s, op->eig_sweeps);
  // Q <- Q U  (in place on the matrix cores, else through the packed buffer)
  if (!rc && rowmul_on_mfma(cplx, nv)) {
    rc = rowmul_inplace(Qd, ld, op->n_tot, nv, L.U, s);
  } else if (!rc) {
    rc = gemm_nn(cplx, Qd, ld, L.U, nv, W, nv, op->n_tot, nv, nv, s);
    if (!rc) rc = copy_block(W, (int64_t)nv * (cplx ? 2 : 1), Qd, ld * (cplx ? 2 : 1), op->n_tot, nv * (cplx ? 2 : 1), s);
  }
  // the eigensolver's status and the next pass's filter bounds, in stream order
  if (!rc && (dev_status || next_bounds)) {
    hipLaunchKernelGGL(rr_finish_kernel, dim3(1), dim3(64), 0, s, eigvals, nv, L.status, dev_status, next_bounds);
    if (hipGetLastError() != hipSuccess) rc = OEFE_EDEVICE;
  }
  if (rc) return fail(rc, "rayleigh_ritz: kernel launch failed");
  return OEFE_OK;
}

int oefe_set_eig_sweep_limit(oefe_op op, int32_t sweeps) {
  if (!op || sweeps < 0) return fail(OEFE_EINVAL, "bad arguments");
  op->eig_sweeps = sweeps;
  return OEFE_OK;
}

int lanczos_bounds(oefe_op op, int32_t k, const double* v0, double* out, void* work, double* dev_bounds,
                   oefe_stream stream) {
  if (!op || !v0 || !out || !work || k < 1 || k > 64) return fail(OEFE_EINVAL, "bad arguments");
  const bool cplx = op->cplx;
  const int E = cplx ? 2 : 1;
  const int prec = cplx ? OEFE_C128 : OEFE_F64;
  const int kb = k + 2;  // block width of the Lanczos basis
  Layout L = layout(op, prec, kb, work);
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = op->n_tot;
  double* Vb = (double*)L.vecA;  // [n x kb]
  double* w = (double*)L.vecB;   // [n x 1] (uses the first n*E doubles)
  double* t = w + n * E;         // [n x 1]
  StepWork sw = carve_step_work(op, 8, cplx, 1, work);
  double* a_d = L.misc;       // alpha_j at misc[2 j] (complex slot), beta_j at misc[256 + j], norm at misc[511]
  double* h = L.G;            // reorth coefficients [kb]
  // v_1 = v0 / ||v0||
  int rc = copy_block(v0, E, Vb, (int64_t)kb * E, n, E, s);
  if (!rc) rc = dot_columns<double>(cplx, Vb, kb, Vb, kb, n, 1, nullptr, a_d + 511, L.gscr, s);
  if (!rc) rc = sqrt_inplace(a_d + 511, s);
  if (!rc) rc = lanczos_scale(cplx, Vb, kb, Vb, a_d + 511, n, s);
  if (rc) return fail(rc, "lanczos: kernel launch failed");
  std::vector<double> alpha, beta;
  double scale = 0;
  for (int j = 0; j < k; ++j) {
    rc = apply_step<double>(op, false, Vb + (int64_t)j * E, kb, nullptr, w, 1, 1, 1.0, 0.0, 0.0, sw, s);
    if (rc) return fail(rc, "lanczos: operator step failed");
    // alpha_j = Re(v_j^* w)
    if (!rc) rc = gram(cplx, Vb + (int64_t)j * E, kb, 1, w, 1, 1, n, a_d + 2 * j, 1, L.gscr, (size_t)1 << 62, s);
    // w -= alpha_j v_j + beta_{j-1} v_{j-1}
    if (!rc)
      rc = lanczos_axpy(cplx, w, Vb + (int64_t)j * E, j > 0 ? Vb + (int64_t)(j - 1) * E : nullptr, a_d + 2 * j,
                        j > 0 ? a_d + 256 + (j - 1) : nullptr, n, kb, s);
    // full reorthogonalization, twice: w -= V (V^* w)
    for (int r = 0; r < 2 && !rc; ++r) {
      rc = gram(cplx, Vb, kb, j + 1, w, 1, 1, n, h, 1, L.gscr, (size_t)1 << 62, s);
      if (!rc) rc = gemm_nn(cplx, Vb, kb, h, 1, t, 1, n, j + 1, 1, s);
      if (!rc) rc = sub_block(cplx, w, t, n, s);
    }
    // beta_j = ||w||
    if (!rc) rc = dot_columns<double>(cplx, w, 1, w, 1, n, 1, nullptr, a_d + 256 + j, L.gscr, s);
    if (!rc) rc = sqrt_inplace(a_d + 256 + j, s);
    if (rc) return fail(rc, "lanczos: kernel launch failed");
    double ab[2];
    hipError_t he = hipMemcpyAsync(&ab[0], a_d + 2 * j, sizeof(double), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipMemcpyAsync(&ab[1], a_d + 256 + j, sizeof(double), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "lanczos");
    alpha.push_back(ab[0]);
    beta.push_back(ab[1]);
    for (double x : alpha) scale = std::max(scale, std::fabs(x));
    for (double x : beta) scale = std::max(scale, std::fabs(x));
    if (ab[1] < 1e-14 * scale || j == k - 1) break;
    rc = lanczos_scale(cplx, Vb + (int64_t)(j + 1) * E, kb, w, a_d + 256 + j, n, s);
    if (rc) return fail(rc, "lanczos: kernel launch failed");
  }
  // eigenvalues of the tridiagonal T (float64 Jacobi on the device)
  const int m = (int)alpha.size();
  std::vector<double> T((size_t)m * m * E, 0.0);
  for (int i = 0; i < m; ++i) {
    T[((size_t)i * m + i) * E] = alpha[i];
    if (i + 1 < m) {
      T[((size_t)i * m + i + 1) * E] = beta[i];
      T[((size_t)(i + 1) * m + i) * E] = beta[i];
    }
  }
  hipError_t he = hipMemcpyAsync(L.Rinv, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (he != hipSuccess) return hip_fail(he, "lanczos");
  rc = jacobi_eig(cplx, L.Rinv, m, L.lam, L.U, L.jscr, L.status, s, op->eig_sweeps);
  if (rc) return fail(rc, "lanczos: eigensolver launch failed");
  std::vector<double> th(m);
  int32_t jst[2] = {0, 0};
  he = hipMemcpyAsync(th.data(), L.lam, m * sizeof(double), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipMemcpyAsync(jst, L.status, sizeof(jst), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return hip_fail(he, "lanczos");
  if (jst[0] != 0)
    return fail(OEFE_ENOCONV, "lanczos: eigensolver of T_k stopped after " + std::to_string(jst[1]) + " sweeps");
  // a0 = smallest Ritz value of T_k, b = largest + beta_k; the first pass cuts the spectrum
  // at the midpoint of [a0, b]
  out[0] = th[0];
  out[1] = th[m - 1] + beta[m - 1];
  out[2] = 0.5 * (out[0] + out[1]);
  if (dev_bounds) {
    const double abc[3] = {out[2], out[1], out[0]};
    he = hipMemcpyAsync(dev_bounds, abc, sizeof(abc), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_fail(he, "lanczos");
  }
  return OEFE_OK;
}

int band_energy_grad(oefe_op op, oefe_prec prec, const void* X, int64_t ld, int32_t nv, const double* f, double* E,
                     double* dE_dV, void* dE_dX, void* work, oefe_stream stream) {
  if (!op || !X || !f || !E || !work || nv <= 0 || ld < nv) return fail(OEFE_EINVAL, "bad arguments");
  if (int rc = check_prec(op, prec)) return rc;
  if (op->diagonal && dE_dV) return fail(OEFE_EINVAL, "diagonal operator has no potential");
  if (op->adaptive && dE_dV)  // V also enters at the adaptive rule's points
    return fail(OEFE_EUNSUPPORTED, "dE/dV at the Gauss points is not the whole derivative under the adaptive rule");
  const bool cplx = op->cplx;
  const bool f32 = prec_fp32(prec);
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  // H X (precision of X) into dE_dX (leading dimension ld) or into packed scratch
  void* HX = dE_dX ? dE_dX : (void*)L.vecA;
  const int64_t ldh = dE_dX ? ld : nv;
  int rc;
  if (f32)
    rc = apply_step<float>(op, prec == OEFE_BF16, (const float*)X, ld, nullptr, (float*)HX, ldh, nv, 1.0, 0.0, 0.0,
                           L.step, s);
  else
    rc = apply_step<double>(op, false, (const double*)X, ld, nullptr, (double*)HX, ldh, nv, 1.0, 0.0, 0.0, L.step, s);
  if (rc) return fail(rc, "band_energy_grad: operator step failed");
  // E = sum_i f_i Re(x_i^* (H x)_i), accumulated in float64
  if (f32)
    rc = dot_columns<float>(cplx, (const float*)X, ld, (const float*)HX, ldh, op->n_tot, nv, f, E, L.gscr, s);
  else
    rc = dot_columns<double>(cplx, (const double*)X, ld, (const double*)HX, ldh, op->n_tot, nv, f, E, L.gscr, s);
  if (rc) return fail(rc, "band_energy_grad: reduction failed");
  if (dE_dV) {
    const int ncr = cplx ? 2 * nv : nv;
    if (f32) {
      rc = zo_only<float>(op, (const float*)X, ld, nv, (float*)L.step.zo, ncr, s);
      if (!rc) rc = density_partial<float>(op, (const float*)X, ld, nv, f, (const float*)L.step.zo, ncr, L.dens, s);
    } else {
      rc = zo_only<double>(op, (const double*)X, ld, nv, (double*)L.step.zo, ncr, s);
      if (!rc) rc = density_partial<double>(op, (const double*)X, ld, nv, f, (const double*)L.step.zo, ncr, L.dens, s);
    }
    if (!rc) rc = density_final(op, L.dens, ncols_blocks(ncr), dE_dV, s);
    if (rc) return fail(rc, "band_energy_grad: density kernels failed");
  }
  if (dE_dX) {
    rc = scale_grad(cplx, dE_dX, ld, op->n_tot, nv, f, f32, s);
    if (rc) return fail(rc, "band_energy_grad: scaling failed");
  }
  return OEFE_OK;
}

int oefe_fermi_occupations(int32_t nk, const int32_t* nv, const double* wk, const double* theta, double n_elec,
                           double kT, double* f, double* out, int32_t* dev_status, oefe_stream stream) {
  if (nk < 1 || nk > kOccMaxK || !nv || !wk || !theta || !f || !out || !dev_status || !(kT > 0.0))
    return fail(OEFE_EINVAL, "bad arguments (1 <= nk <= 64, kT > 0, non-null pointers)");
  OccArgs a{};
  a.nk = nk;
  a.off[0] = 0;
  for (int k = 0; k < nk; ++k) {
    if (nv[k] < 1 || !(wk[k] >= 0.0)) return fail(OEFE_EINVAL, "bad block width or weight");
    a.off[k + 1] = a.off[k] + nv[k];
    a.w2[k] = 2.0 * wk[k];
  }
  hipLaunchKernelGGL(occupations_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, theta, a, n_elec, kT, f, out,
                     dev_status);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "oefe_fermi_occupations");
  return OEFE_OK;
}

}  // extern "C"

// ---- The auxiliary-potential Poisson problem (eqnpoissonaux, eqnpoissX) on the device.
// The operator of oefe_poisson_create applies At = P^T A P with P = diag(m^-1/2, S),
// S = (A^oo)^-1/2 (the same kernels as Ht: no potential, the Laplacian 1/(4 pi) grad . grad,
// the phi enrichment).  A phi = c becomes At y = P^T c, phi = P y, solved by conjugate gradients:
// CG on At is CG on A preconditioned by the diagonal GLL mass on the FE rows and A^oo on the
// enrichment rows.
namespace {
constexpr int kPoisPartials = 256;

// per workgroup, in a fixed order: sum W (b + rho) and sum W over a contiguous range
__global__ __launch_bounds__(256) void pois_charge_partial_kernel(const double* __restrict__ W,
                                                                  const double* __restrict__ b,
                                                                  const double* __restrict__ rho, int64_t n,
                                                                  int64_t per, double* __restrict__ part) {
  __shared__ double s0[256], s1[256];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
  double a = 0.0, w = 0.0;
  for (int64_t i = i0 + t; i < i1; i += 256) {
    a += W[i] * (b[i] + rho[i]);
    w += W[i];
  }
  s0[t] = a;
  s1[t] = w;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s0[t] += s0[t + o];
      s1[t] += s1[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

// sc[0] = (sum W (b + rho)) / (sum W): the uniform background removed from the charge
__global__ void pois_mean_kernel(const double* __restrict__ part, int G, double* __restrict__ sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, w = 0.0;
  for (int g = 0; g < G; ++g) {
    a += part[2 * g];
    w += part[2 * g + 1];
  }
  sc[0] = a / w;
}

// f = b + rho - background (eqnDiscForceVec's charge, made neutral)
__global__ void pois_neutral_kernel(const double* __restrict__ b, const double* __restrict__ rho,
                                    const double* __restrict__ sc, double* __restrict__ f, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = b[i] + rho[i] - sc[0];
}

// right-hand side on the FE rows: yb[g] = m_g^-1/2 c_g, c_g = int f N_g = sum over the (up to 8)
// cells of node g of sum_q W_q f_q B[q, a] (B the tensor-product values of the GLL basis at the
// Gauss points), cells and points in a fixed order; z[g] = m_g^1/2 (the null vector of At)
__global__ __launch_bounds__(256) void pois_rhs_fe_kernel(const double* __restrict__ f, const double* __restrict__ W,
                                                          CellCoef<double> cf, const double* __restrict__ msq,
                                                          int nc, int p, int n, int P1, int nq, int64_t N,
                                                          double* __restrict__ yb, double* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int nn = n * n;
  const int iz = (int)(g / nn), rem = (int)(g - (int64_t)iz * nn), iy = rem / n, ix = rem - iy * n;
  const int id[3] = {ix, iy, iz};
  int cc[3][2], aa[3][2], na[3];
  for (int d = 0; d < 3; ++d) {
    const int c = id[d] / p, a = id[d] - c * p;
    na[d] = 1;
    cc[d][0] = c;
    aa[d][0] = a;
    if (a == 0) {  // also the last local node of the previous cell (periodic)
      na[d] = 2;
      cc[d][1] = c == 0 ? nc - 1 : c - 1;
      aa[d][1] = p;
    }
  }
  double c = 0.0;
  for (int kz = 0; kz < na[2]; ++kz)
    for (int ky = 0; ky < na[1]; ++ky)
      for (int kx = 0; kx < na[0]; ++kx) {
        const int64_t e = cc[0][kx] + (int64_t)nc * (cc[1][ky] + (int64_t)nc * cc[2][kz]);
        const int ax = aa[0][kx], ay = aa[1][ky], az = aa[2][kz];
        const double* fe = f + e * nq;
        const double* We = W + e * nq;
        double se = 0.0;
        for (int qz = 0; qz < P1; ++qz) {
          double sy = 0.0;
          for (int qy = 0; qy < P1; ++qy) {
            double sx = 0.0;
            for (int qx = 0; qx < P1; ++qx) {
              const int q = qx + P1 * (qy + P1 * qz);
              sx += cf.B1[qx][ax] * (We[q] * fe[q]);
            }
            sy += cf.B1[qy][ay] * sx;
          }
          se += cf.B1[qz][az] * sy;
        }
        c += se;
      }
  yb[g] = msq[g] * c;
  z[g] = 1.0 / msq[g];
}

// enrichment rows of c: c_I = sum over the support cells of block I and their points of W f N^O_I
// (one workgroup per block, one function per block, fixed order)
// Adaptive rule: the enrichment rows c_I = sum over atom I's support cells and their rule points of
// w (b + rho - background) N^O_I, with b and rho at the points (a_b, rho_a) and the background sc[0];
// one workgroup per atom, threads striding over each cell's points, a fixed tree at the end.
__global__ __launch_bounds__(256) void pois_rhs_enr_adapt_kernel(const double* __restrict__ a_b,
                                                                 const double* __restrict__ rho_a,
                                                                 const double* __restrict__ a_w,
                                                                 const double* __restrict__ phiA,
                                                                 const int64_t* __restrict__ a_off,
                                                                 const int64_t* __restrict__ cf_aoff,
                                                                 const int32_t* __restrict__ cf_acell,
                                                                 const int64_t* __restrict__ blk_cf0,
                                                                 const double* __restrict__ sc, double* __restrict__ cO) {
  __shared__ double red[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const double bg = sc[0];
  double a = 0.0;
  for (int64_t cf = blk_cf0[b]; cf < blk_cf0[b + 1]; ++cf) {
    const int k = cf_acell[cf];
    const int64_t p0 = a_off[k], np = a_off[k + 1] - p0, r0 = cf_aoff[cf];
    for (int64_t q = t; q < np; q += 256) a += a_w[p0 + q] * (a_b[p0 + q] + rho_a[p0 + q] - bg) * phiA[r0 + q];
  }
  red[t] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) cO[b] = red[0];
}

__global__ __launch_bounds__(256) void pois_rhs_enr_kernel(const double* __restrict__ f, const double* __restrict__ W,
                                                           const double* __restrict__ phi,
                                                           const int32_t* __restrict__ cf_cell,
                                                           const int64_t* __restrict__ blk_cf0, int nq,
                                                           double* __restrict__ cO) {
  __shared__ double red[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const int64_t j0 = blk_cf0[b] * nq, j1 = blk_cf0[b + 1] * nq;
  double a = 0.0;
  for (int64_t j = j0 + t; j < j1; j += 256) {
    const int64_t e = cf_cell[j / nq];
    const int q = (int)(j % nq);
    a += W[e * nq + q] * f[e * nq + q] * phi[j];
  }
  red[t] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) cO[b] = red[0];
}

// y[i] = sum_j S[i][j] x[j] (S symmetric, nO x nO), one thread per row
__global__ void pois_small_mv_kernel(const double* __restrict__ S, const double* __restrict__ x, int nO,
                                     double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nO) return;
  double a = 0.0;
  for (int j = 0; j < nO; ++j) a += S[(size_t)i * nO + j] * x[j];
  y[i] = a;
}

// v[0..N) -= (num / den) z  (the component along the null vector z; num, den device scalars)
__global__ void pois_project_kernel(double* __restrict__ v, const double* __restrict__ z, const double* __restrict__ num,
                                    const double* __restrict__ den, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) v[i] -= (num[0] / den[0]) * z[i];
}

// x = 0, r = p = v
__global__ void pois_start_kernel(const double* __restrict__ v, double* __restrict__ x, double* __restrict__ r,
                                  double* __restrict__ pv, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = 0.0;
  r[i] = v[i];
  pv[i] = v[i];
}

// x += alpha p, r -= alpha q with alpha = rr / pq (0 when pq <= 0), and the chunk partials of
// r_new . r_new in the chunking and summation order of the one-column dot product
// (dot1_chunk_count, dot1_final): the step and the dot in one pass over r, the dot's bits
__global__ __launch_bounds__(1024) void pois_step_rr_kernel(double* __restrict__ x, double* __restrict__ r,
                                                            const double* __restrict__ pv, const double* __restrict__ q,
                                                            const double* __restrict__ rr, const double* __restrict__ pq,
                                                            int64_t n, int64_t rows_per_chunk, double* __restrict__ part) {
  __shared__ double red[16];
  const double al = pq[0] > 0.0 ? rr[0] / pq[0] : 0.0;
  const int64_t g0 = (int64_t)blockIdx.x * rows_per_chunk, g1 = min(n, g0 + rows_per_chunk);
  auto step = [&](int64_t g) {
    x[g] += al * pv[g];
    const double rn = r[g] - al * q[g];
    r[g] = rn;
    return rn * rn + 0.0;  // the dot kernel's term, written the same way
  };
  double s0 = 0, s1 = 0;
  int64_t g = g0 + threadIdx.x;
  for (; g + 1024 < g1; g += 2048) {
    s0 += step(g);
    s1 += step(g + 1024);
  }
  if (g < g1) s0 += step(g);
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

// p = r + beta p with beta = rr_new / rr
__global__ void pois_dir_kernel(double* __restrict__ pv, const double* __restrict__ r,
                                const double* __restrict__ rr_new, const double* __restrict__ rr, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double be = rr[0] > 0.0 ? rr_new[0] / rr[0] : 0.0;
  pv[i] = r[i] + be * pv[i];
}

// phi = P y with the FE part's GLL-mass-weighted mean removed: phi_g = m_g^-1/2 y_g - (z . y) / (z . z)
__global__ void pois_finish_fe_kernel(const double* __restrict__ y, const double* __restrict__ msq,
                                      const double* __restrict__ zy, const double* __restrict__ zz,
                                      double* __restrict__ phi, int64_t N) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) phi[g] = msq[g] * y[g] - zy[0] / zz[0];
}

struct PoisLayout {
  StepWork step;
  double *x, *r, *p, *q, *v, *z, *f, *cO, *dscr, *sc, *part;
  size_t total;
};

PoisLayout pois_layout(const oefe_op_s* op, void* work) {
  PoisLayout L{};
  char* p = (char*)work;
  const size_t sb = al256(step_work_bytes(op, 8, false, 1, nullptr));
  if (work) L.step = carve_step_work(op, 8, false, 1, work);
  p += sb;
  const size_t vb = al256((size_t)op->n_tot * sizeof(double));
  auto take = [&](size_t bytes) {
    double* r = (double*)p;
    p += al256(bytes);
    return r;
  };
  L.x = take(vb);
  L.r = take(vb);
  L.p = take(vb);
  L.q = take(vb);
  L.v = take(vb);
  L.z = take((size_t)op->N * sizeof(double));
  L.f = take((size_t)op->n_cells * op->nq * sizeof(double));
  L.cO = take((size_t)std::max(op->n_enr, 1) * sizeof(double));
  L.dscr = take(256 * sizeof(double));
  L.sc = take(16 * sizeof(double));
  L.part = take(2 * kPoisPartials * sizeof(double));
  L.total = (size_t)(p - (char*)work);
  return L;
}
}  // namespace

extern "C" {

int oefe_poisson_create(const oefe_system_desc* desc, oefe_op* out) {
  if (!desc || !out) return fail(OEFE_EINVAL, "null argument");
  *out = nullptr;
  if (desc->n_atoms < 1 || !desc->pos || !desc->Z) return fail(OEFE_EINVAL, "the Poisson operator needs atoms");
  if (desc->kvec) return fail(OEFE_EINVAL, "the Poisson operator is real (no Bloch wavevector)");
  for (int I = 0; I < desc->n_atoms; ++I)
    if (!(desc->Z[I] > 0)) return fail(OEFE_EINVAL, "atomic numbers must be positive");
  oefe_op_s* op = new (std::nothrow) oefe_op_s();
  if (!op) return fail(OEFE_ENOMEM, "host allocation failed");
  op->poisson = true;
  std::string err;
  int rc = build_operator(op, desc, err);
  if (rc == OEFE_OK && hipGetDevice(&op->device) != hipSuccess) {
    rc = OEFE_EDEVICE;
    err = "no HIP device";
  }
  if (rc == OEFE_OK) rc = upload_operator(op, err);
  if (rc == OEFE_OK && !scratch_address(err)) rc = OEFE_EDEVICE;
  if (rc != OEFE_OK) {
    free_device(op);
    delete op;
    return fail(rc, err);
  }
  *out = op;
  return OEFE_OK;
}

size_t oefe_poisson_work_size(oefe_op pop) {
  if (!pop || !pop->poisson) return 0;
  return pois_layout(pop, nullptr).total + 256;
}

static int poisson_solve_impl(oefe_op pop, const double* rho, const double* rho_adapt, double* phi, double tol,
                              int32_t max_iter, double* info, void* work, oefe_stream stream);

int oefe_poisson_solve(oefe_op pop, const double* rho, double* phi, double tol, int32_t max_iter, double* info,
                       void* work, oefe_stream stream) {
  if (pop && pop->adaptive) return fail(OEFE_EINVAL, "an operator with the adaptive rule takes rho at its points (oefe_poisson_solve_adaptive)");
  return poisson_solve_impl(pop, rho, nullptr, phi, tol, max_iter, info, work, stream);
}

int oefe_poisson_solve_adaptive(oefe_op pop, const double* rho, const double* rho_adapt, double* phi, double tol,
                                int32_t max_iter, double* info, void* work, oefe_stream stream) {
  if (!pop || !pop->adaptive || !rho_adapt) return fail(OEFE_EINVAL, "bad arguments");
  return poisson_solve_impl(pop, rho, rho_adapt, phi, tol, max_iter, info, work, stream);
}

int oefe_poisson_create_adaptive(const oefe_system_desc* desc, double tol, int32_t max_depth, oefe_op* out) {
  if (!desc || !out) return fail(OEFE_EINVAL, "null argument");
  *out = nullptr;
  if (desc->n_atoms < 1 || !desc->pos || !desc->Z) return fail(OEFE_EINVAL, "the Poisson operator needs atoms");
  if (desc->kvec) return fail(OEFE_EINVAL, "the Poisson operator is real (no Bloch wavevector)");
  for (int I = 0; I < desc->n_atoms; ++I)
    if (!(desc->Z[I] > 0)) return fail(OEFE_EINVAL, "atomic numbers must be positive");
  if (!(tol > 0.0 && tol < 1.0) || max_depth < 0 || max_depth > kAdaptMaxDepth)
    return fail(OEFE_EINVAL, "adaptive rule: need 0 < tol < 1 and 0 <= max_depth <= 5");
  oefe_op_s* op = new (std::nothrow) oefe_op_s();
  if (!op) return fail(OEFE_ENOMEM, "host allocation failed");
  op->poisson = true;
  op->adaptive = true;
  op->ad_tol = tol;
  op->ad_depth = max_depth;
  return finish_create(op, desc, out);
}

static int poisson_solve_impl(oefe_op pop, const double* rho, const double* rho_adapt, double* phi, double tol,
                              int32_t max_iter, double* info, void* work, oefe_stream stream) {
  if (!pop || !rho || !phi || !work || !info || max_iter < 1 || !(tol > 0.0))
    return fail(OEFE_EINVAL, "bad arguments");
  if (!pop->poisson) return fail(OEFE_EINVAL, "not an operator of oefe_poisson_create");
  const oefe_op_s* op = pop;
  hipStream_t s = (hipStream_t)stream;
  PoisLayout L = pois_layout(op, work);
  const int64_t N = op->N, n = op->n_tot, nqt = op->n_cells * op->nq;
  const int nO = op->n_enr;
  auto blocks = [](int64_t m) { return dim3((unsigned)((m + 255) / 256)); };
  // charge: f = b + rho - background
  const int64_t per = (nqt + kPoisPartials - 1) / kPoisPartials;
  hipLaunchKernelGGL(pois_charge_partial_kernel, dim3(kPoisPartials), dim3(256), 0, s, op->d.W, op->d.bsmear, rho, nqt,
                     per, L.part);
  hipLaunchKernelGGL(pois_mean_kernel, dim3(1), dim3(64), 0, s, L.part, kPoisPartials, L.sc + 8);
  hipLaunchKernelGGL(pois_neutral_kernel, blocks(nqt), dim3(256), 0, s, op->d.bsmear, rho, L.sc + 8, L.f, nqt);
  // v = P^T c, projected off the null vector z = (m^1/2, 0)
  hipLaunchKernelGGL(pois_rhs_fe_kernel, blocks(N), dim3(256), 0, s, L.f, op->d.W, op->cd, op->d.msq, op->nc, op->p,
                     op->n, op->P1, op->nq, N, L.v, L.z);
  if (rho_adapt)  // the enrichment rows on the adaptive rule, the charge at its points
    hipLaunchKernelGGL(pois_rhs_enr_adapt_kernel, dim3((unsigned)nO), dim3(256), 0, s, op->d.a_b, rho_adapt, op->d.a_w,
                       op->d.phiA, op->d.a_off, op->d.cf_aoff, op->d.cf_acell, op->d.blk_cf0, L.sc + 8, L.cO);
  else
    hipLaunchKernelGGL(pois_rhs_enr_kernel, dim3((unsigned)nO), dim3(256), 0, s, L.f, op->d.W, op->d.phi,
                       op->d.cf_cell, op->d.blk_cf0, op->nq, L.cO);
  hipLaunchKernelGGL(pois_small_mv_kernel, blocks(nO), dim3(256), 0, s, op->d.S, L.cO, nO, L.v + N);
  int rc = dot_columns<double>(false, L.z, 1, L.v, 1, N, 1, nullptr, L.sc + 4, L.dscr, s);  // z . v
  if (!rc) rc = dot_columns<double>(false, L.z, 1, L.z, 1, N, 1, nullptr, L.sc + 5, L.dscr, s);  // z . z
  if (rc) return fail(rc, "oefe_poisson_solve: kernel launch failed");
  hipLaunchKernelGGL(pois_project_kernel, blocks(N), dim3(256), 0, s, L.v, L.z, L.sc + 4, L.sc + 5, N);
  // conjugate gradients on At y = v from y = 0; rr of iteration k in sc[k & 1], pq in sc[2],
  // the starting residual in sc[3]
  hipLaunchKernelGGL(pois_start_kernel, blocks(n), dim3(256), 0, s, L.v, L.x, L.r, L.p, n);
  rc = dot_columns<double>(false, L.r, 1, L.r, 1, n, 1, nullptr, L.sc + 0, L.dscr, s);
  if (!rc) rc = dot_columns<double>(false, L.r, 1, L.r, 1, n, 1, nullptr, L.sc + 3, L.dscr, s);
  if (rc) return fail(rc, "oefe_poisson_solve: kernel launch failed");
  thread_local double* hbuf = nullptr;
  if (!hbuf && hipHostMalloc((void**)&hbuf, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    hbuf = nullptr;
    return fail(OEFE_EDEVICE, "oefe_poisson_solve: pinned host buffer");
  }
  int it = 0;
  double rel = 1.0;
  bool done = false;
  const int nch1 = dot1_chunk_count(n);  // the r . r partials of pois_step_rr_kernel fill nch1 <= 128 of dscr
  while (!done && it < max_iter) {
    const int k = it & 1;
    rc = apply_step<double>(op, false, L.p, 1, nullptr, L.q, 1, 1, 1.0, 0.0, 0.0, L.step, s);
    if (!rc) rc = dot_columns<double>(false, L.p, 1, L.q, 1, n, 1, nullptr, L.sc + 2, L.dscr, s);
    if (rc) return fail(rc, "oefe_poisson_solve: kernel launch failed");
    hipLaunchKernelGGL(pois_step_rr_kernel, dim3((unsigned)nch1), dim3(1024), 0, s, L.x, L.r, L.p, L.q, L.sc + k,
                       L.sc + 2, n, (n + nch1 - 1) / nch1, L.dscr);
    rc = dot1_final(L.dscr, nch1, L.sc + (k ^ 1), s);
    if (rc) return fail(rc, "oefe_poisson_solve: kernel launch failed");
    hipLaunchKernelGGL(pois_dir_kernel, blocks(n), dim3(256), 0, s, L.p, L.r, L.sc + (k ^ 1), L.sc + k, n);
    ++it;
    if (it % 8 == 0 || it == max_iter) {  // convergence test: one host read every 8 iterations
      hipError_t e = hipMemcpyAsync(hbuf, L.sc, 4 * sizeof(double), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_fail(e, "oefe_poisson_solve");
      rel = hbuf[3] > 0.0 ? std::sqrt(std::max(hbuf[it & 1], 0.0) / hbuf[3]) : 0.0;
      done = rel <= tol;
    }
  }
  // phi = P y (FE part with zero mass-weighted mean)
  rc = dot_columns<double>(false, L.z, 1, L.x, 1, N, 1, nullptr, L.sc + 6, L.dscr, s);
  if (rc) return fail(rc, "oefe_poisson_solve: kernel launch failed");
  hipLaunchKernelGGL(pois_finish_fe_kernel, blocks(N), dim3(256), 0, s, L.x, op->d.msq, L.sc + 6, L.sc + 5, phi, N);
  hipLaunchKernelGGL(pois_small_mv_kernel, blocks(nO), dim3(256), 0, s, op->d.S, L.x + N, nO, phi + N);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "oefe_poisson_solve");
  info[0] = it;
  info[1] = rel;
  return done ? OEFE_OK : fail(OEFE_ENOCONV, "oefe_poisson_solve: residual above the tolerance after max_iter");
}

int oefe_density(oefe_op op, oefe_prec prec, const void* X, int64_t ld, int32_t nv, const double* weights, double* rho,
                 int32_t accumulate, void* work, oefe_stream stream) {
  if (!op || !X || !weights || !rho || !work || nv <= 0 || ld < nv) return fail(OEFE_EINVAL, "bad arguments");
  if (int rc = check_prec(op, prec)) return rc;
  if (op->diagonal) return fail(OEFE_EINVAL, "diagonal operator has no density");
  const bool cplx = op->cplx;
  Layout L = layout(op, prec, nv, work);
  hipStream_t s = (hipStream_t)stream;
  const int ncr = cplx ? 2 * nv : nv;
  int rc;
  if (prec_fp32(prec)) {
    rc = zo_only<float>(op, (const float*)X, ld, nv, (float*)L.step.zo, ncr, s);
    if (!rc) rc = density_partial<float>(op, (const float*)X, ld, nv, weights, (const float*)L.step.zo, ncr, L.dens, s);
  } else {
    rc = zo_only<double>(op, (const double*)X, ld, nv, (double*)L.step.zo, ncr, s);
    if (!rc) rc = density_partial<double>(op, (const double*)X, ld, nv, weights, (const double*)L.step.zo, ncr, L.dens, s);
  }
  if (!rc) rc = density_final(op, L.dens, ncols_blocks(ncr), rho, s, accumulate ? 2 : 1);
  if (rc) return fail(rc, "oefe_density: kernel launch failed");
  return OEFE_OK;
}

}  // extern "C"
