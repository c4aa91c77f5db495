// Internal definitions shared by the host setup and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/oefe.h"

namespace oefe {

constexpr int kMaxP1 = 5;  // supported GLL nodes per edge: 3, 4, 5 (degree 2..4)
constexpr int kTileRows = 64;  // FE rows per enrichment tile
constexpr int kAdaptMaxDepth = 5;  // deepest subdivision of the adaptive rule (8^5 leaves per cell at most)

// Enrichment coupling tiles of kTileRows FE rows, in one of two shapes chosen per operator:
//  mode 0: 64 consecutive FE rows, g = 64 t + r;
//  mode 1: the block of 16 x 2 x 2 FE nodes starting at node (16 bx, 2 by, 2 bz),
//          t = bx + nbx (by + nby bz), nbx = ceil(n / 16), nby = ceil(n / 2) (n nodes per edge),
//          row r = the node (16 bx + r % 16, 2 by + (r / 16) % 2, 2 bz + r / 32).
// A block couples to fewer enrichment functions than 64 nodes of one x-line where atoms are
// dense relative to the mesh, and each 16-row group (one wave of the node stage) still lies on
// one x-line, where every node has the same slots in y and z.  Rows past the mesh: none (-1).
__host__ __device__ inline int tile_count(int n, int mode) {
  if (mode == 0) return (int)(((int64_t)n * n * n + 63) / 64);
  const int nbx = (n + 15) >> 4, nby = (n + 1) >> 1;
  return nbx * nby * nby;
}
// first node of tile t: (x0, y0, z0) in mode 1; in mode 0 x0 = 64 t (the first row)
__host__ __device__ inline void tile_origin(int t, int n, int mode, int& x0, int& y0, int& z0) {
  if (mode == 0) {
    x0 = 64 * t;
    y0 = z0 = 0;
    return;
  }
  const int nbx = (n + 15) >> 4, nby = (n + 1) >> 1;
  const int rest = t / nbx;
  x0 = 16 * (t - rest * nbx);
  y0 = 2 * (rest % nby);
  z0 = 2 * (rest / nby);
}
// FE row of row r of the tile with origin (x0, y0, z0) and its node (ix, iy, iz), or -1 past the
// mesh (then ix = iy = iz = 0)
__host__ __device__ inline int tile_row_coords(int x0, int y0, int z0, int r, int n, int mode, int& ix, int& iy,
                                               int& iz) {
  if (mode == 0) {
    const int g = x0 + r, nn = n * n;
    if (g >= nn * n) {
      ix = iy = iz = 0;
      return -1;
    }
    iz = g / nn;
    const int rem = g - iz * nn;
    iy = rem / n;
    ix = rem - iy * n;
    return g;
  }
  ix = x0 + (r & 15);
  iy = y0 + ((r >> 4) & 1);
  iz = z0 + (r >> 5);
  if (ix < n && iy < n && iz < n) return ix + n * (iy + n * iz);
  ix = iy = iz = 0;
  return -1;
}
// FE row of row r of the tile with origin (x0, y0, z0), or -1 past the mesh
__host__ __device__ inline int tile_row_node(int x0, int y0, int z0, int r, int n, int mode) {
  if (mode == 0) {
    const int g = x0 + r;
    return g < n * n * n ? g : -1;
  }
  const int ix = x0 + (r & 15), iy = y0 + ((r >> 4) & 1), iz = z0 + (r >> 5);
  return (ix < n && iy < n && iz < n) ? ix + n * (iy + n * iz) : -1;
}
__host__ __device__ inline int tile_node(int t, int r, int n, int mode) {
  int x0, y0, z0;
  tile_origin(t, n, mode, x0, y0, z0);
  return tile_row_node(x0, y0, z0, r, n, mode);
}
// enrichment functions one tile may couple to: the node-stage kernels stage a tile's dense
// block (complex: two planes of kTileRows x (F + 1) float64) in 150 KB of LDS
constexpr int kTileFunctionsMax = 144;

using cplx = std::complex<double>;

// A 5 x 5 matrix M that a reflection of both indices leaves unchanged (M[4-q][4-a] = M[q][a]:
// the 1D operators of degree 4 on the symmetric GLL nodes and Gauss points), by its even and
// odd halves: e[q][a] = (M[q][a] + M[q][4-a]) / 2 for a < 2 and e[q][2] = M[q][2] (q <= 2),
// o[q][a] = (M[q][a] - M[q][4-a]) / 2 (q, a < 2).  Then, with e_a = v_a + v_4-a and
// o_a = v_a - v_4-a, (M v)_q = E_q + O_q and (M v)_4-q = E_q - O_q, E = e (e_0, e_1, v_2) and
// O = o (o_0, o_1): 13 products and 8 additions in place of 25 products.
template <typename T>
struct EO5 {
  T e[3][3];
  T o[2][2];
};

// 1D reference data in the form the cell kernel uses (q = p + 1 Gauss points).
//  B1[qi][a]   Lagrange basis on GLL nodes at Gauss point qi
//  L1[qi][qj]  collocation Laplacian at Gauss points: Dh^T diag(w) Dh, Dh = D1 B1^-1
//  BtL[a][qj]  sum_k B1[k][a] L1[k][qj]
//  BtW[a][qi]  B1[qi][a] w[qi]
//  w[q]        Gauss weights
//  om[a]       1/sqrt(w'_{a mod p}) with w'_0 = 2 what_0 (lumped-mass factor per local index)
template <typename T>
struct CellCoef {
  T B1[kMaxP1][kMaxP1];
  T L1[kMaxP1][kMaxP1];
  T BtL[kMaxP1][kMaxP1];
  T BtW[kMaxP1][kMaxP1];
  T w[kMaxP1];
  T om[kMaxP1];
  T kappa;  // h / 4: scale of the reference kinetic form
  T mscale; // (h/2)^(-3/2): scale of m^-1/2
  // the derivative at the Gauss points of the interpolant of values there (reference
  // coordinates): the first-derivative term of the periodic-function k-point form
  T Dh[kMaxP1][kMaxP1];
  // degree 4 only: the halves of B1, B1^T, L1, BtW and kappa BtW
  EO5<T> eB1, eB1t, eL1, eBtW, ekBtW;
};

struct DeviceArrays {
  // potential times weight at quadrature points [n_cells * nq]
  double* WV = nullptr;
  float* WVf = nullptr;
  // enrichment, atom-blocked H^co: block b has nf[b] functions starting at fn0[b],
  // rows rows[rptr[b] .. rptr[b+1]) (global FE index) and values
  // hv[(rptr[b] + r) * FMAX + f] (complex: 2 doubles per entry)
  int32_t* blk_fn0 = nullptr;
  int32_t* blk_nf = nullptr;
  int64_t* blk_rptr = nullptr;
  int32_t* blk_rows = nullptr;
  double* hv = nullptr;
  float* hvf = nullptr;
  // forward product by FE row (CSR): row g has entries fr_ptr[g]..fr_ptr[g+1]) of
  // (function fr_fn[k], value fr_val[k] = m_g^-1/2 H^co[g, fn]); hv above is scaled the same way
  int64_t* fr_ptr = nullptr;
  int32_t* fr_fn = nullptr;
  double* fr_val = nullptr;
  float* fr_valf = nullptr;
  // tile-dense enrichment coupling: FE rows in tiles of kTileRows; tile t couples to the
  // functions tile_fns[tile_fptr[t] .. tile_fptr[t+1]) (padded to a multiple of 4 with -1)
  // with dense values tile_val[(tile_fptr[t] * kTileRows + r * FP_t + j)] (complex: x2),
  // pre-scaled by m_g^-1/2.  Transposed partials are reduced per function over the list
  // fn_poff[fn_pptr[nu] .. fn_pptr[nu+1]) of (tile_fptr[t] + j) slots.
  int32_t* tile_fptr = nullptr;
  int32_t* tile_fns = nullptr;
  double* tile_val = nullptr;
  float* tile_valf = nullptr;
  // the three dense cell matrices of the BF16 cell stage (B, K, B^T with permuted
  // quadrature order), bf16 bit patterns in MFMA A-fragment order, 3 x 8 x 4 x 64 x 8
  uint16_t* bf_mats = nullptr;
  int32_t* fn_pptr = nullptr;
  int32_t* fn_poff = nullptr;
  // transposed-product chunks: chunk c covers block chunk_blk[c], rows [chunk_r0[c], chunk_r1[c])
  int32_t* chunk_blk = nullptr;
  int64_t* chunk_r0 = nullptr;
  int64_t* chunk_r1 = nullptr;
  int32_t* blk_chunk0 = nullptr;  // first chunk of each block [nblk + 1]
  int32_t* fn_blk = nullptr;      // block of each enrichment function [n_enr]
  // dense enrichment matrices (n_enr^2, complex interleaved when complex)
  double* S = nullptr;
  double* Hoo = nullptr;
  float* Sf = nullptr;
  float* Hoof = nullptr;
  // N^O at quadrature points by cell: cell e has entries cph_ptr[e]..cph_ptr[e+1]),
  // entry j: block cph_blk[j], values phi[(cph_off[j] * nq + q) * FMAX + f]
  int64_t* cph_ptr = nullptr;
  int32_t* cph_blk = nullptr;
  int64_t* cph_off = nullptr;
  double* phi = nullptr;
  // diagonal test operator
  double* lambda = nullptr;
  float* lambdaf = nullptr;
  // potential rebuild on the device (oefe_op_set_potential)
  double* W = nullptr;          // quadrature weights [n_cells * nq]
  double* V = nullptr;          // current potential [n_cells * nq]
  double* msq = nullptr;        // m_g^-1/2 [N]
  double* hkin = nullptr;       // kinetic part of H^co by block row [n_hrows][FMAX] (complex: x2), unscaled
  double* Hoo_kin = nullptr;    // kinetic part of H^oo [n_enr^2] (complex: x2)
  int32_t* row_blk = nullptr;   // block of each block row [n_hrows]
  int64_t* rpos = nullptr;      // CSR position of each block row's first function [n_hrows]
  int64_t* rr_ptr = nullptr;    // block row -> its (support cell, local node) pairs [n_hrows + 1]
  int32_t* rr_ent = nullptr;    // pair: 128 * (flattened support cell) + local node
  int32_t* cf_cell = nullptr;   // cell of each flattened support cell (index into phi)
  int64_t* csr2tile = nullptr;  // CSR entry -> tile_val position [fr_nnz]
  int64_t* hp_ptr = nullptr;    // atom-block pair (bi nb + bj) -> common support cells [nb^2 + 1]
  int32_t* hp_i = nullptr;      // flattened support cell of bi for each common cell
  int32_t* hp_j = nullptr;      // flattened support cell of bj
  // auxiliary-potential Poisson operator (oefe_poisson_create)
  double* bsmear = nullptr;     // smeared nuclear charge at the quadrature points [n_cells * nq]
  int64_t* blk_cf0 = nullptr;   // first flattened support cell of each block [nblk + 1]
  // adaptive quadrature of the enrichment integrals (oefe_op_create_adaptive): the rule's
  // points by rule cell (whole leaves of P1^3 points each), the 1D basis of every leaf, and
  // N^O at the points of every flattened support cell
  double* a_w = nullptr;        // weights [n_points]
  double* a_V = nullptr;        // potential at the points [n_points]
  double* a_leafB = nullptr;    // leaf l, direction d: ell_a(t_q) at [(l * 3 + d) * P1 + q] * P1 + a
  int64_t* a_off = nullptr;     // rule cell -> first point [n_rule_cells + 1]
  int32_t* cf_acell = nullptr;  // flattened support cell -> rule cell
  int64_t* cf_aoff = nullptr;   // flattened support cell -> first row of phiA
  double* phiA = nullptr;       // N^O: phiA[(row * FMAX + f)] (complex: x2)
  double* hpart = nullptr;      // potential part of H^co per (flattened support cell, local node, f)
  double* hoo_part = nullptr;   // potential part of H^oo per (block pair, chunk of common cells, f, g)
  double* a_b = nullptr;        // Poisson operator: the smeared nuclear charge at the rule's points
};

struct AtomBlock {
  int atom;
  int fn0, nf;
  std::vector<int64_t> cells;      // sorted, N^O support (dilated)
  std::vector<cplx> phi;           // [ncell][nq][nf]
  std::vector<cplx> gphi;          // [ncell][nq][nf][3]
  std::vector<int32_t> rows;       // sorted FE rows where H^co is nonzero
  std::vector<cplx> hkin;          // kinetic part of H^co on rows [rows][nf]
  // adaptive quadrature: N^O and its gradient at the rule's points of each support cell
  std::vector<int64_t> aoff;       // support cell -> first row (its points) [ncell + 1]
  std::vector<cplx> phiA;          // [rows][nf]
  std::vector<cplx> gphiA;         // [rows][nf][3] (set-up only)
};

}  // namespace oefe

struct oefe_op_s {
  bool diagonal = false;
  bool cplx = false;
  // operator of the auxiliary-potential Poisson problem: one phi-enrichment function per
  // atom, no potential, the Laplacian 1/(4 pi) int grad . grad in place of the kinetic
  // 1/2 int grad . grad, and S = (A^oo)^-1/2 (the enrichment block's Jacobi factor)
  bool poisson = false;
  // k-point operator in the periodic-function form (oefe_op_create_uform): periodic FE functions
  // (no Bloch phase), the k terms of the Hamiltonian (-i k . grad in the cell stage, |k|^2/2
  // added to the potential: vshift) and the k-dependent enrichment
  bool uform = false;
  double vshift = 0.0;
  double uk[3] = {0, 0, 0};  // (h/2)^3 (2/h) k_d: the cell stage's first-derivative coefficients
  int device = 0;
  // geometry
  double L = 0, h = 0;
  int nc = 0, p = 0, P1 = 0, n = 0, nd = 0, nq = 0;
  int64_t N = 0, n_cells = 0, n_tot = 0;
  int n_enr = 0;
  double kvec[3] = {0, 0, 0};
  double phase[3][2] = {{1, 0}, {1, 0}, {1, 0}};  // exp(i k_d L)
  // 1D data
  oefe::CellCoef<double> cd;
  oefe::CellCoef<float> cf;
  double gll_w[8], gauss_x[8], gauss_w[8];
  double B1[8][8], D1[8][8];
  // host copies
  std::vector<double> V, W;  // [n_cells * nq]
  std::vector<double> mdiag;
  std::vector<oefe::AtomBlock> blocks;
  std::vector<oefe::cplx> Moo, Hoo_kin, Hoo, S;
  std::vector<double> Moo_eigs;
  std::vector<double> bsmear, rc_smear;  // Poisson operator: smeared charge, smearing radii
  // adaptive quadrature of the enrichment integrals (Sec. III.B; oefe_op_create_adaptive):
  // rule cells ascending, their points (whole leaves of P1^3 tensor Gauss points), weights,
  // the potential there, and per leaf the 1D Lagrange values and derivatives at its points
  bool adaptive = false;
  double ad_tol = 0.0;
  int ad_depth = 0;
  std::vector<int64_t> ad_cells;    // rule cell -> mesh cell
  std::vector<int32_t> ad_index;    // mesh cell -> rule cell or -1 [n_cells]
  std::vector<int64_t> ad_off;      // rule cell -> first point [n_rule_cells + 1]
  std::vector<double> ad_x, ad_w, ad_V;
  std::vector<double> ad_b;         // Poisson operator: the smeared nuclear charge at the points
  std::vector<double> ad_B, ad_D;   // leaf l, direction d: [(l * 3 + d) * P1 + q] * P1 + a
  int64_t n_cf = 0;                 // flattened (block, support cell) pairs
  int hoo_nchunk = 1;               // chunks of each block pair's common cells (H^oo rebuild)
  int FMAX = 1;
  int64_t n_hrows = 0;  // total rows over blocks
  int64_t n_chunks = 0;
  int chunk_rows = 256;
  int64_t fr_nnz = 0;
  std::vector<std::vector<int64_t>> fr_pos;  // per block, per row: CSR position of its first function
  std::vector<int64_t> csr_to_tile;           // CSR entry -> index into tile_val
  int64_t n_tiles = 0, tile_slots = 0;        // tiles, total padded (tile, function) slots
  int tile_mode = 0;                           // coupling-tile shape (tile_count)
  int tile_fpmax = 0;
  int fn_smax = 0;  // most tile partials of one enrichment function
  oefe::DeviceArrays d;
  // launch shape overrides (autotuner): cell-kernel column width, node/partial column block
  int tune_cw = 0, tune_cb = 0;
  // sweep limit of the dense Hermitian eigensolver (0: built-in); oefe_set_eig_sweep_limit
  int eig_sweeps = 0;
  // instrumentation (oefe_kernel_timer)
  int timer_kind = 0;  // oefe_timer_kind
  // side stream and events of the overlapped recurrence (created on first use)
  mutable hipStream_t side_stream = nullptr;
  mutable hipEvent_t ev_node = nullptr, ev_k1 = nullptr, ev_zo = nullptr;
  mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> timer_events;
};

namespace oefe {
// host setup (oefe_setup.cpp)
int build_operator(oefe_op_s* op, const oefe_system_desc* desc, std::string& err);
int rebuild_potential_parts(oefe_op_s* op, std::string& err);
void hermitian_eig(int n, std::vector<cplx>& A, std::vector<double>& lam, std::vector<cplx>& U);
void block_hco_values(const oefe_op_s* op, const AtomBlock& b, std::vector<cplx>& out);
// device upload (oefe_api.hip)
int upload_operator(oefe_op_s* op, std::string& err);
int upload_potential_parts(oefe_op_s* op, std::string& err);
void set_error(const std::string& msg);
}  // namespace oefe
