// Host-side construction of the OEFE operator data (untimed setup).
//
// Everything here follows Sec. III.A of the paper: spectral Lagrange elements
// on GLL nodes with a diagonal GLL mass (eqnMcc, eqnorthCGLL), atomic
// enrichment functions with a smooth cutoff (eqnUOEFEAtomic,
// eqnKSAtomicTrunc, eqnCutoffProperties), their orthogonalization against the
// FE space (eqnUOEFEOrtho, eqnorthC, eqnorthCGLL), and the enrichment blocks
// M^oo (eqnMoo), H^co and H^oo (eqnHOEFEelelements).  Integrals of H use one
// tensor Gauss rule with p + 1 points per direction; the numerator of c uses
// the same rule and the denominator the GLL mass.  Cell-level transforms are
// sum-factorized (tensor-product 1D passes).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>

#include "oefe_internal.h"

namespace oefe {

namespace {

constexpr double kPi = 3.14159265358979323846;

// P_n(x) and P_{n-1}(x) by the three-term recurrence.
void legendre_pair(int n, double x, double& pn, double& pn1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { pn = 1.0; pn1 = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

// GLL nodes: -1, 1 and the zeros of x P_p - P_{p-1} (equivalently of P_p');
// weights 2 / (p (p+1) P_p^2).
void gll_rule(int p, double* x, double* w) {
  for (int j = 0; j <= p; ++j) x[j] = -std::cos(kPi * j / p);
  for (int j = 1; j < p; ++j) {
    for (int it = 0; it < 100; ++it) {
      double pn, pn1;
      legendre_pair(p, x[j], pn, pn1);
      double f = x[j] * pn - pn1;
      double dx = f / ((p + 1) * pn);
      x[j] -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
  }
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 0; j <= p; ++j) {
    double pn, pn1;
    legendre_pair(p, x[j], pn, pn1);
    w[j] = 2.0 / (p * (p + 1) * pn * pn);
  }
}

// Gauss-Legendre: zeros of P_q, weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss_rule(int q, double* x, double* w) {
  for (int j = 0; j < q; ++j) {
    double z = -std::cos(kPi * (j + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, pn1;
      legendre_pair(q, z, pn, pn1);
      double dp = q * (z * pn - pn1) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double pn, pn1;
    legendre_pair(q, z, pn, pn1);
    double dp = q * (z * pn - pn1) / (z * z - 1.0);
    x[j] = z;
    w[j] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Lagrange basis on `nodes` (count n): value and derivative of ell_a at t.
void lagrange(int n, const double* nodes, int a, double t, double& val, double& der) {
  double denom = 1.0, num = 1.0;
  for (int j = 0; j < n; ++j)
    if (j != a) {
      denom *= nodes[a] - nodes[j];
      num *= t - nodes[j];
    }
  val = num / denom;
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    if (k == a) continue;
    double pr = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != a && j != k) pr *= t - nodes[j];
    s += pr;
  }
  der = s / denom;
}

// In-place inverse of a small dense matrix (Gauss-Jordan, partial pivoting).
bool invert(int n, double* A) {
  std::vector<double> M(2 * n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) M[i * 2 * n + j] = A[i * n + j];
    M[i * 2 * n + n + i] = 1.0;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * 2 * n + c]) > std::fabs(M[piv * 2 * n + c])) piv = r;
    if (M[piv * 2 * n + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(M[c * 2 * n + j], M[piv * 2 * n + j]);
    double d = M[c * 2 * n + c];
    for (int j = 0; j < 2 * n; ++j) M[c * 2 * n + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = M[r * 2 * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < 2 * n; ++j) M[r * 2 * n + j] -= f * M[c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[i * n + j] = M[i * 2 * n + n + j];
  return true;
}

// erf(r/sigma)/r with its small-r series.
double erf_over_r(double r, double sigma) {
  if (r < 1e-6 * sigma) {
    double x = r / sigma;
    return 2.0 / (sigma * std::sqrt(kPi)) * (1.0 - x * x / 3.0 + x * x * x * x / 10.0);
  }
  return std::erf(r / sigma) / r;
}

// Smooth cutoff h(r) and h'(r): 1 below r0, 0 above r1, 1/(1 + exp(1/x - 1/(1-x))) between.
void cutoff(double r, double r0, double r1, double& h, double& dh) {
  if (r <= r0) { h = 1.0; dh = 0.0; return; }
  if (r >= r1) { h = 0.0; dh = 0.0; return; }
  double x = (r1 - r) / (r1 - r0);
  double u = 1.0 / x - 1.0 / (1.0 - x);
  double s;
  if (u > 0) {
    double e = std::exp(-u);
    s = e / (1.0 + e);
  } else {
    s = 1.0 / (1.0 + std::exp(u));
  }
  h = s;
  double dsdx = s * (1.0 - s) * (1.0 / (x * x) + 1.0 / ((1.0 - x) * (1.0 - x)));
  dh = -dsdx / (r1 - r0);
}

// Atomic function r^pw exp(-zeta r) [d_axis] h(r) and its gradient at displacement d.
void atomic_fn(const double d[3], int pw, double zeta, int axis, double r0, double r1, double& val,
               double grad[3]) {
  double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double e = std::exp(-zeta * r);
  double rp = pw == 0 ? 1.0 : std::pow(r, pw);
  double f = rp * e;
  double fp = (pw == 0 ? 0.0 : pw * std::pow(r, pw - 1)) * e - zeta * f;
  double h, dh;
  cutoff(r, r0, r1, h, dh);
  double radial = fp * h + f * dh;  // d/dr of f h
  if (axis < 0) {
    val = f * h;
    for (int k = 0; k < 3; ++k) grad[k] = radial * d[k] / r;
  } else {
    double P = d[axis];
    val = P * f * h;
    for (int k = 0; k < 3; ++k) grad[k] = P * radial * d[k] / r;
    grad[axis] += f * h;
  }
}

// Unit smeared charge g(r, rc) (eqngr) and its potential v_g(r, rc) with dv_g/dr (eqnvg).
double smeared_g(double r, double rc) {
  if (r > rc) return 0.0;
  const double t = r - rc;
  return -21.0 * t * t * t * (6.0 * r * r + 3.0 * r * rc + rc * rc) / (5.0 * kPi * std::pow(rc, 8));
}
void smeared_v(double r, double rc, double& v, double& dv) {
  if (r > rc) {
    v = 1.0 / r;
    dv = -1.0 / (r * r);
    return;
  }
  const double r2 = r * r, r4 = r2 * r2, c2 = rc * rc, c5 = c2 * c2 * rc, c8 = std::pow(rc, 8);
  v = (9.0 * r4 * r2 * r - 30.0 * r4 * r2 * rc + 28.0 * r4 * r * c2 - 14.0 * r2 * c5 + 12.0 * c5 * c2) / (5.0 * c8);
  dv = (63.0 * r4 * r2 - 180.0 * r4 * r * rc + 140.0 * r4 * c2 - 28.0 * r * c5) / (5.0 * c8);
}

// Hartree potential of the model atom density Z alpha^3 / (8 pi) exp(-alpha r) (the isolated-atom
// Hartree potential of the auxiliary-potential enrichment, which an atomic solver would supply):
// V = Z (1 - (1 + alpha r / 2) exp(-alpha r)) / r, with its series below alpha r = 1e-3.
void model_hartree(double r, double Z, double alpha, double& v, double& dv) {
  const double x = alpha * r;
  if (x < 1e-3) {
    v = Z * alpha * (0.5 - x * x / 12.0 + x * x * x / 24.0);
    dv = Z * alpha * alpha * (-x / 6.0 + x * x / 8.0);
    return;
  }
  const double e = std::exp(-x), u = 1.0 - (1.0 + 0.5 * x) * e;
  v = Z * alpha * u / x;
  dv = Z * alpha * alpha * ((0.5 + 0.5 * x) * e * x - u) / (x * x);
}

// Atomic part of the auxiliary-potential enrichment (eqnPhiAuxAtomic, eqnEnrichedPhiAux):
// (V_H(r) - Z v_g(r, rc)) h(r) and its gradient at displacement d.
void phi_aux_fn(const double d[3], double Z, double alpha, double rc, double r0, double r1, double& val,
                double grad[3]) {
  const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double vh, dvh, vg, dvg, h, dh;
  model_hartree(r, Z, alpha, vh, dvh);
  smeared_v(r, rc, vg, dvg);
  cutoff(r, r0, r1, h, dh);
  const double f = vh - Z * vg, fp = dvh - Z * dvg;
  val = f * h;
  const double radial = fp * h + f * dh;
  for (int k = 0; k < 3; ++k) grad[k] = r > 0.0 ? radial * d[k] / r : 0.0;
}

// Tensor-product transforms on one cell (P1 = q = p + 1 points per direction).
// fwd: out[qz][qy][qx] = sum Mz[qz][az] My[qy][ay] Mx[qx][ax] in[az][ay][ax]
template <typename S>
void tp_forward(int P1, const double* Mx, const double* My, const double* Mz, const S* in, S* out) {
  S t1[125], t2[125];
  for (int az = 0; az < P1; ++az)
    for (int ay = 0; ay < P1; ++ay)
      for (int qx = 0; qx < P1; ++qx) {
        S s = 0;
        for (int ax = 0; ax < P1; ++ax) s += Mx[qx * 8 + ax] * in[(az * P1 + ay) * P1 + ax];
        t1[(az * P1 + ay) * P1 + qx] = s;
      }
  for (int az = 0; az < P1; ++az)
    for (int qy = 0; qy < P1; ++qy)
      for (int qx = 0; qx < P1; ++qx) {
        S s = 0;
        for (int ay = 0; ay < P1; ++ay) s += My[qy * 8 + ay] * t1[(az * P1 + ay) * P1 + qx];
        t2[(az * P1 + qy) * P1 + qx] = s;
      }
  for (int qz = 0; qz < P1; ++qz)
    for (int qy = 0; qy < P1; ++qy)
      for (int qx = 0; qx < P1; ++qx) {
        S s = 0;
        for (int az = 0; az < P1; ++az) s += Mz[qz * 8 + az] * t2[(az * P1 + qy) * P1 + qx];
        out[(qz * P1 + qy) * P1 + qx] = s;
      }
}

// bwd (transpose): out[az][ay][ax] = sum Mz[qz][az] My[qy][ay] Mx[qx][ax] in[qz][qy][qx]
template <typename S>
void tp_backward(int P1, const double* Mx, const double* My, const double* Mz, const S* in, S* out) {
  S t1[125], t2[125];
  for (int qz = 0; qz < P1; ++qz)
    for (int qy = 0; qy < P1; ++qy)
      for (int ax = 0; ax < P1; ++ax) {
        S s = 0;
        for (int qx = 0; qx < P1; ++qx) s += Mx[qx * 8 + ax] * in[(qz * P1 + qy) * P1 + qx];
        t1[(qz * P1 + qy) * P1 + ax] = s;
      }
  for (int qz = 0; qz < P1; ++qz)
    for (int ay = 0; ay < P1; ++ay)
      for (int ax = 0; ax < P1; ++ax) {
        S s = 0;
        for (int qy = 0; qy < P1; ++qy) s += My[qy * 8 + ay] * t1[(qz * P1 + qy) * P1 + ax];
        t2[(qz * P1 + ay) * P1 + ax] = s;
      }
  for (int az = 0; az < P1; ++az)
    for (int ay = 0; ay < P1; ++ay)
      for (int ax = 0; ax < P1; ++ax) {
        S s = 0;
        for (int qz = 0; qz < P1; ++qz) s += Mz[qz * 8 + az] * t2[(qz * P1 + ay) * P1 + ax];
        out[(az * P1 + ay) * P1 + ax] = s;
      }
}

struct Geo {
  const oefe_op_s* op;
  int64_t cell_of(int cx, int cy, int cz) const {
    int nc = op->nc;
    cx = ((cx % nc) + nc) % nc;
    cy = ((cy % nc) + nc) % nc;
    cz = ((cz % nc) + nc) % nc;
    return cx + (int64_t)nc * (cy + (int64_t)nc * cz);
  }
  // global FE index and Bloch phase of local node a of cell e
  void dof(int64_t e, int a, int64_t& g, cplx& th) const {
    int nc = op->nc, p = op->p, P1 = op->P1, n = op->n;
    int cx = e % nc, cy = (e / nc) % nc, cz = e / ((int64_t)nc * nc);
    int ax = a % P1, ay = (a / P1) % P1, az = a / (P1 * P1);
    int ix = cx * p + ax, iy = cy * p + ay, iz = cz * p + az;
    th = cplx(1.0, 0.0);
    if (ix >= n) { ix -= n; th *= cplx(op->phase[0][0], op->phase[0][1]); }
    if (iy >= n) { iy -= n; th *= cplx(op->phase[1][0], op->phase[1][1]); }
    if (iz >= n) { iz -= n; th *= cplx(op->phase[2][0], op->phase[2][1]); }
    g = ix + (int64_t)n * (iy + (int64_t)n * iz);
  }
  void quad_point(int64_t e, int q, double x[3]) const {
    int nc = op->nc, P1 = op->P1;
    int c[3] = {(int)(e % nc), (int)((e / nc) % nc), (int)(e / ((int64_t)nc * nc))};
    int qq[3] = {q % P1, (q / P1) % P1, q / (P1 * P1)};
    for (int d = 0; d < 3; ++d) x[d] = c[d] * op->h + (op->gauss_x[qq[d]] + 1.0) * op->h / 2.0;
  }
};

// ---- adaptive quadrature of the enrichment integrals (Sec. III.B)
//
constexpr int kSetupThreads = 16;  // host threads of the rule's refinement
//
// Whole-space integrals A = int psi~^2 and B = int |grad psi~|^2 of an atomic function
// psi~ = g(r) (axis < 0) or d_axis g(r), g = r^pw exp(-zeta r) h(r), after the angular
// integration: s-type 4 pi r^2 g^2 and 4 pi r^2 g'^2; p-type 4 pi r^4 g^2 / 3 and
// 4 pi r^2 (g^2 + 2/3 r g g' + r^2 g'^2 / 3); radial integrals by 64 panels of 20-point
// Gauss-Legendre on [0, r1] (g vanishes beyond r1).
// The radial function g(r), g'(r) of a trial function (gfun), vanishing beyond r1.
using RadialFn = std::function<void(double r, double& g, double& gp)>;
// The value and gradient of trial function fn of atom I at displacement d.
using TrialEval = std::function<void(int I, int fn, const double d[3], double& v, double g[3])>;

void radial_scales(const RadialFn& gfun, int axis, double r1, double& A, double& B) {
  constexpr int kPanels = 64, kOrder = 20;
  double x[kOrder], w[kOrder];
  gauss_rule(kOrder, x, w);
  A = 0.0;
  B = 0.0;
  for (int k = 0; k < kPanels; ++k) {
    const double a = r1 * k / kPanels, b = r1 * (k + 1) / kPanels;
    for (int j = 0; j < kOrder; ++j) {
      const double r = 0.5 * (b - a) * (x[j] + 1.0) + a, wr = 0.5 * (b - a) * w[j];
      double g, gp;
      gfun(r, g, gp);
      if (axis < 0) {
        A += wr * 4.0 * kPi * r * r * g * g;
        B += wr * 4.0 * kPi * r * r * gp * gp;
      } else {
        A += wr * 4.0 * kPi * r * r * r * r * g * g / 3.0;
        B += wr * 4.0 * kPi * r * r * (g * g + 2.0 / 3.0 * r * g * gp + r * r * gp * gp / 3.0);
      }
    }
  }
}

// Trial integrals of one box [lo, lo + size]^3 of the cell with origin org under the box's
// tensor Gauss rule (P1 points per direction), for each function fl[j] = (atom, enrichment
// function), psi~ at the displacement from the atom's nearest image: out[j * nt + 0] =
// int psi~^2, [1] = int |grad psi~|^2, [2 + a] = int psi~ N_a, [2 + nd + a] =
// int grad psi~ . grad^ N_a (grad^: the gradient in the cell's reference coordinates), a over
// the cell's nd local nodes; nt = 2 + 2 nd.
void box_trials(const oefe_op_s* op, const oefe_system_desc* desc, const TrialEval& eval, const double* xi,
                const double org[3], const double lo[3], double size, const std::vector<std::pair<int, int>>& fl,
                std::vector<double>& out) {
  const int P1 = op->P1, nd = op->nd, nt = 2 + 2 * nd;
  const double h = op->h;
  double t[3][8], wt[3][8], Lv[3][8][8], Ld[3][8][8];
  for (int d = 0; d < 3; ++d)
    for (int q = 0; q < P1; ++q) {
      t[d][q] = lo[d] + 0.5 * size * (op->gauss_x[q] + 1.0);
      wt[d][q] = 0.5 * size * op->gauss_w[q];
      const double ref = 2.0 * (t[d][q] - org[d]) / h - 1.0;
      for (int a = 0; a < P1; ++a) lagrange(P1, xi, a, ref, Lv[d][q][a], Ld[d][q][a]);
    }
  out.assign(fl.size() * nt, 0.0);
  for (int qz = 0; qz < P1; ++qz)
    for (int qy = 0; qy < P1; ++qy)
      for (int qx = 0; qx < P1; ++qx) {
        const double x[3] = {t[0][qx], t[1][qy], t[2][qz]};
        const double w = wt[0][qx] * wt[1][qy] * wt[2][qz];
        for (size_t j = 0; j < fl.size(); ++j) {
          const int I = fl[j].first, fn = fl[j].second;
          double dd[3];
          for (int k = 0; k < 3; ++k) {
            const double dr = x[k] - desc->pos[3 * I + k];
            dd[k] = dr - op->L * std::nearbyint(dr / op->L);
          }
          double v, g[3];
          eval(I, fn, dd, v, g);
          double* o = &out[j * nt];
          o[0] += w * v * v;
          o[1] += w * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
          if (v == 0.0 && g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
          for (int az = 0; az < P1; ++az)
            for (int ay = 0; ay < P1; ++ay)
              for (int ax = 0; ax < P1; ++ax) {
                const int a = ax + P1 * (ay + P1 * az);
                const double na = Lv[0][qx][ax] * Lv[1][qy][ay] * Lv[2][qz][az];
                const double gn = g[0] * Ld[0][qx][ax] * Lv[1][qy][ay] * Lv[2][qz][az] +
                                  g[1] * Lv[0][qx][ax] * Ld[1][qy][ay] * Lv[2][qz][az] +
                                  g[2] * Lv[0][qx][ax] * Lv[1][qy][ay] * Ld[2][qz][az];
                o[2 + a] += w * v * na;
                o[2 + nd + a] += w * gn;
              }
        }
      }
}

// A box that meets the ball of radius r1 around one of the atoms of fl (nearest image) while
// none of its Gauss points lies inside that ball: its rule cannot see the functions there.
bool blind_box(const oefe_op_s* op, const oefe_system_desc* desc, const std::vector<std::pair<int, int>>& fl,
               const double lo[3], double size) {
  const int P1 = op->P1;
  const double r1 = desc->r1;
  int last = -1;
  for (const auto& pr : fl) {
    const int I = pr.first;
    if (I == last) continue;
    last = I;
    const double* R = &desc->pos[3 * I];
    double ex2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double c = lo[k] + 0.5 * size - R[k];
      c -= op->L * std::nearbyint(c / op->L);
      const double ex = std::max(std::fabs(c) - 0.5 * size, 0.0);
      ex2 += ex * ex;
    }
    if (!(std::sqrt(ex2) < r1)) continue;
    bool inside = false;
    for (int qz = 0; qz < P1 && !inside; ++qz)
      for (int qy = 0; qy < P1 && !inside; ++qy)
        for (int qx = 0; qx < P1 && !inside; ++qx) {
          const int qq[3] = {qx, qy, qz};
          double d2 = 0.0;
          for (int k = 0; k < 3; ++k) {
            double dr = lo[k] + 0.5 * size * (op->gauss_x[qq[k]] + 1.0) - R[k];
            dr -= op->L * std::nearbyint(dr / op->L);
            d2 += dr * dr;
          }
          inside = std::sqrt(d2) < r1;
        }
    if (!inside) return true;
  }
  return false;
}

// Leaves of one cell: a box blind to an atom's support (blind_box) is split; otherwise it is
// kept when, for every trial integral, its own rule and the sum of its 8 half-size children's
// rules (children in the order cx + 2 cy + 4 cz) differ by at most bound[], else its children
// are refined in that order; at max_depth levels boxes are kept.  Leaves are appended depth
// first as {lo_x, lo_y, lo_z, size}.
void refine_box(const oefe_op_s* op, const oefe_system_desc* desc, const TrialEval& eval, const double* xi,
                const double org[3], const std::vector<std::pair<int, int>>& fl, const std::vector<double>& bound,
                const double lo[3], double size, int depth, std::vector<std::array<double, 4>>& leaves) {
  if (depth == op->ad_depth) {
    leaves.push_back({lo[0], lo[1], lo[2], size});
    return;
  }
  double clo[8][3];
  for (int c = 0; c < 8; ++c) {
    const int off[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    for (int d = 0; d < 3; ++d) clo[c][d] = lo[d] + 0.5 * size * off[d];
  }
  bool split = blind_box(op, desc, fl, lo, size);
  if (!split) {
    std::vector<double> own, kid, ksum;
    box_trials(op, desc, eval, xi, org, lo, size, fl, own);
    ksum.assign(own.size(), 0.0);
    for (int c = 0; c < 8; ++c) {
      box_trials(op, desc, eval, xi, org, clo[c], 0.5 * size, fl, kid);
      for (size_t j = 0; j < kid.size(); ++j) ksum[j] += kid[j];
    }
    for (size_t j = 0; j < own.size() && !split; ++j) split = !(std::fabs(own[j] - ksum[j]) <= bound[j]);
  }
  if (!split) {
    leaves.push_back({lo[0], lo[1], lo[2], size});
    return;
  }
  for (int c = 0; c < 8; ++c) refine_box(op, desc, eval, xi, org, fl, bound, clo[c], 0.5 * size, depth + 1, leaves);
}

// The adaptive rule on the union of the blocks' support cells (cells ascending): leaves, their
// points and weights, the 1D GLL Lagrange values and derivatives at each leaf's points (in the
// cell's reference coordinates), and the potential at the points.
int build_adaptive_rule(oefe_op_s* op, const oefe_system_desc* desc, const double* xi, const TrialEval& eval,
                        const std::vector<double>& scaleA, const std::vector<double>& scaleB, std::string& err) {
  const int P1 = op->P1, nq = op->nq;
  const double h = op->h;
  std::vector<std::vector<std::pair<int, int>>> fns_of(op->n_cells);
  for (auto& b : op->blocks)
    for (int64_t e : b.cells)
      for (int f = 0; f < b.nf; ++f) fns_of[e].push_back({b.atom, b.fn0 + f});
  op->ad_cells.clear();
  op->ad_index.assign(op->n_cells, -1);
  for (int64_t e = 0; e < op->n_cells; ++e)
    if (!fns_of[e].empty()) {
      op->ad_index[e] = (int32_t)op->ad_cells.size();
      op->ad_cells.push_back(e);
    }
  op->ad_off.assign(1, 0);
  op->ad_x.clear();
  op->ad_w.clear();
  op->ad_B.clear();
  op->ad_D.clear();
  const int nc = op->nc;
  // scales of the trial integrals: A, B for the quadratic ones, their Cauchy-Schwarz bounds
  // sqrt(A v), sqrt(B v) (v = 4/3 pi r1^3) for the ones with the FE functions
  const int nd = op->nd, nt = 2 + 2 * nd;
  const double vol = 4.0 / 3.0 * kPi * desc->r1 * desc->r1 * desc->r1;
  // cells are refined independently: contiguous ranges of rule cells on host threads, each
  // collecting its leaves, then appended in cell order (the rule does not depend on the split)
  const int64_t nrc = (int64_t)op->ad_cells.size();
  std::vector<std::vector<std::array<double, 4>>> cell_leaves(nrc);
  auto work = [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t e = op->ad_cells[k];
      const auto& fl = fns_of[e];
      std::vector<double> bound(nt * fl.size());
      for (size_t j = 0; j < fl.size(); ++j) {
        const double A = scaleA[fl[j].second], B = scaleB[fl[j].second];
        bound[j * nt] = op->ad_tol * A;
        bound[j * nt + 1] = op->ad_tol * B;
        for (int a = 0; a < nd; ++a) {
          bound[j * nt + 2 + a] = op->ad_tol * std::sqrt(A * vol);
          bound[j * nt + 2 + nd + a] = op->ad_tol * std::sqrt(B * vol);
        }
      }
      const double org[3] = {(double)(e % nc) * h, (double)((e / nc) % nc) * h, (double)(e / ((int64_t)nc * nc)) * h};
      refine_box(op, desc, eval, xi, org, fl, bound, org, h, 0, cell_leaves[k]);
    }
  };
  const int nth = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kSetupThreads,
                                                              (int64_t)std::max(1u, std::thread::hardware_concurrency()),
                                                              nrc}));
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(work, nrc * t / nth, nrc * (t + 1) / nth);
  work(0, nrc / nth);
  for (auto& th : pool) th.join();
  for (int64_t k = 0; k < nrc; ++k) {
    const int64_t e = op->ad_cells[k];
    const double org[3] = {(double)(e % nc) * h, (double)((e / nc) % nc) * h, (double)(e / ((int64_t)nc * nc)) * h};
    const auto& leaves = cell_leaves[k];
    for (const auto& lf : leaves) {
      double t[3][8], wt[3][8];
      for (int d = 0; d < 3; ++d)
        for (int q = 0; q < P1; ++q) {
          t[d][q] = lf[d] + 0.5 * lf[3] * (op->gauss_x[q] + 1.0);
          wt[d][q] = 0.5 * lf[3] * op->gauss_w[q];
          const double ref = 2.0 * (t[d][q] - org[d]) / h - 1.0;
          for (int a = 0; a < P1; ++a) {
            double v, dv;
            lagrange(P1, xi, a, ref, v, dv);
            op->ad_B.push_back(v);
            op->ad_D.push_back(dv);
          }
        }
      for (int qz = 0; qz < P1; ++qz)
        for (int qy = 0; qy < P1; ++qy)
          for (int qx = 0; qx < P1; ++qx) {
            op->ad_x.push_back(t[0][qx]);
            op->ad_x.push_back(t[1][qy]);
            op->ad_x.push_back(t[2][qz]);
            op->ad_w.push_back(wt[0][qx] * wt[1][qy] * wt[2][qz]);
          }
    }
    op->ad_off.push_back(op->ad_off.back() + (int64_t)leaves.size() * nq);
  }
  const int64_t np = op->ad_off.back();
  if (np >= (int64_t(1) << 31)) {
    err = "adaptive rule has 2^31 points or more";
    return OEFE_EUNSUPPORTED;
  }
  op->ad_V.assign(np, 0.0);
  if (op->poisson) {  // no potential; the smeared nuclear charge at the points (eqnsmeared)
    op->ad_b.assign(np, 0.0);
    for (int64_t i = 0; i < np; ++i) {
      double b = 0.0;
      for (int I = 0; I < desc->n_atoms; ++I) {
        double d2 = 0;
        for (int k = 0; k < 3; ++k) {
          double dd = op->ad_x[3 * i + k] - desc->pos[3 * I + k];
          dd -= op->L * std::nearbyint(dd / op->L);
          d2 += dd * dd;
        }
        b -= desc->Z[I] * smeared_g(std::sqrt(d2), op->rc_smear[I]);
      }
      op->ad_b[i] = b;
    }
    return OEFE_OK;
  }
  for (int64_t i = 0; i < np; ++i) {
    double v = 0.0;
    for (int I = 0; I < desc->n_atoms; ++I) {
      double d2 = 0;
      for (int k = 0; k < 3; ++k) {
        double dd = op->ad_x[3 * i + k] - desc->pos[3 * I + k];
        dd -= op->L * std::nearbyint(dd / op->L);
        d2 += dd * dd;
      }
      v -= desc->Z[I] * erf_over_r(std::sqrt(d2), desc->sigma);
    }
    op->ad_V[i] = v + op->vshift;  // the periodic-function form's |k|^2/2 rides on V
  }
  return OEFE_OK;
}

// 1D matrices of leaf l in the stride-8 layout of tp_forward / tp_backward (rows: the leaf's
// points, columns: nodes), values (D = false) or derivatives (D = true) in direction d.
void leaf_matrix(const oefe_op_s* op, int64_t l, int d, bool D, double* M) {
  const int P1 = op->P1;
  const double* src = (D ? op->ad_D.data() : op->ad_B.data()) + ((size_t)l * 3 + d) * P1 * P1;
  for (int q = 0; q < P1; ++q)
    for (int a = 0; a < P1; ++a) M[q * 8 + a] = src[q * P1 + a];
}

}  // namespace

// Hermitian eigendecomposition by cyclic complex Jacobi: A = U diag(lam) U^*, ascending.
void hermitian_eig(int n, std::vector<cplx>& A, std::vector<double>& lam, std::vector<cplx>& U) {
  U.assign((size_t)n * n, cplx(0, 0));
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> cplx& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (i == j) diag += std::norm(a(i, j));
        else off += std::norm(a(i, j));
      }
    if (off <= 1e-30 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        cplx b = a(p, q);
        double r = std::abs(b);
        if (r == 0.0) continue;
        double al = a(p, p).real(), ga = a(q, q).real();
        if (r < 1e-300) continue;
        cplx eph = b / r;  // e^{i phi}
        double tau = (ga - al) / (2.0 * r);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        cplx emi = std::conj(eph);  // e^{-i phi}
        // A <- A G (columns p, q), G = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
        for (int k = 0; k < n; ++k) {
          cplx akp = a(k, p), akq = a(k, q);
          a(k, p) = akp * c - akq * s * emi;
          a(k, q) = akp * s + akq * c * emi;
        }
        // A <- G^* A (rows p, q)
        for (int k = 0; k < n; ++k) {
          cplx apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * eph * aqk;
          a(q, k) = s * apk + c * eph * aqk;
        }
        a(p, q) = 0.0;
        a(q, p) = 0.0;
        a(p, p) = al - t * r;
        a(q, q) = ga + t * r;
        for (int k = 0; k < n; ++k) {
          cplx ukp = U[(size_t)k * n + p], ukq = U[(size_t)k * n + q];
          U[(size_t)k * n + p] = ukp * c - ukq * s * emi;
          U[(size_t)k * n + q] = ukp * s + ukq * c * emi;
        }
      }
  }
  lam.resize(n);
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x).real() < a(y, y).real(); });
  std::vector<cplx> U2((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    lam[j] = a(idx[j], idx[j]).real();
    for (int k = 0; k < n; ++k) U2[(size_t)k * n + j] = U[(size_t)k * n + idx[j]];
  }
  U.swap(U2);
}

int build_operator(oefe_op_s* op, const oefe_system_desc* desc, std::string& err) {
  const int p = desc->p;
  if (p < 2 || p > 4) { err = "degree p must be 2, 3 or 4"; return OEFE_EUNSUPPORTED; }
  if (desc->nc < 2 || desc->L <= 0) { err = "need nc >= 2 and L > 0"; return OEFE_EINVAL; }
  if (desc->n_enr > 0 && !(desc->r1 > desc->r0 && desc->r0 > 0 && desc->r1 < 0.5 * desc->L)) {
    err = "need 0 < r0 < r1 < L/2";
    return OEFE_EINVAL;
  }
  op->L = desc->L;
  op->nc = desc->nc;
  op->p = p;
  op->P1 = p + 1;
  op->n = op->nc * p;
  op->nd = op->P1 * op->P1 * op->P1;
  op->nq = op->nd;
  op->h = op->L / op->nc;
  op->N = (int64_t)op->n * op->n * op->n;
  op->n_cells = (int64_t)op->nc * op->nc * op->nc;
  const bool pois = op->poisson;
  op->n_enr = pois ? desc->n_atoms : desc->n_enr;
  op->n_tot = op->N + op->n_enr;
  op->cplx = desc->kvec != nullptr;
  const bool uf = op->uform;
  if (uf && !op->cplx) {
    err = "the periodic-function form needs a Bloch wavevector";
    return OEFE_EINVAL;
  }
  if (pois && (op->cplx || desc->n_atoms < 1)) {
    err = "the auxiliary-potential operator needs atoms and no Bloch wavevector";
    return OEFE_EINVAL;
  }
  if (pois && !(desc->r1 > desc->r0 && desc->r0 > 0 && desc->r1 < 0.5 * desc->L)) {
    err = "need 0 < r0 < r1 < L/2";
    return OEFE_EINVAL;
  }
  // Laplacian scale: 1/2 for the Kohn-Sham kinetic term, 1/(4 pi) for the Poisson problem
  const double kin = pois ? 1.0 / (4.0 * kPi) : 0.5;
  if (op->cplx) {
    for (int d = 0; d < 3; ++d) {
      op->kvec[d] = desc->kvec[d];
      // the periodic-function form's FE functions are periodic: no phase across the cell boundary
      op->phase[d][0] = uf ? 1.0 : std::cos(desc->kvec[d] * op->L);
      op->phase[d][1] = uf ? 0.0 : std::sin(desc->kvec[d] * op->L);
    }
  }
  op->vshift = uf ? 0.5 * (op->kvec[0] * op->kvec[0] + op->kvec[1] * op->kvec[1] + op->kvec[2] * op->kvec[2]) : 0.0;
  const int P1 = op->P1;
  const double h = op->h;
  // ---- 1D data
  double xi[8], what[8];
  gll_rule(p, xi, what);
  gauss_rule(P1, op->gauss_x, op->gauss_w);
  for (int j = 0; j <= p; ++j) op->gll_w[j] = what[j];
  for (int qi = 0; qi < P1; ++qi)
    for (int a = 0; a < P1; ++a) lagrange(P1, xi, a, op->gauss_x[qi], op->B1[qi][a], op->D1[qi][a]);
  double Binv[25], Dh[25], L1[25];
  for (int i = 0; i < P1; ++i)
    for (int j = 0; j < P1; ++j) Binv[i * P1 + j] = op->B1[i][j];
  if (!invert(P1, Binv)) { err = "singular interpolation matrix"; return OEFE_EINVAL; }
  for (int i = 0; i < P1; ++i)
    for (int j = 0; j < P1; ++j) {
      double s = 0;
      for (int k = 0; k < P1; ++k) s += op->D1[i][k] * Binv[k * P1 + j];
      Dh[i * P1 + j] = s;
    }
  for (int i = 0; i < P1; ++i)
    for (int j = 0; j < P1; ++j) {
      double s = 0;
      for (int k = 0; k < P1; ++k) s += Dh[k * P1 + i] * op->gauss_w[k] * Dh[k * P1 + j];
      L1[i * P1 + j] = s;
    }
  std::memset(&op->cd, 0, sizeof(op->cd));
  for (int i = 0; i < P1; ++i) {
    op->cd.w[i] = op->gauss_w[i];
    double wp = what[i % p] * (i % p == 0 ? 2.0 : 1.0);
    op->cd.om[i] = 1.0 / std::sqrt(wp);
    for (int j = 0; j < P1; ++j) {
      op->cd.B1[i][j] = op->B1[i][j];
      op->cd.L1[i][j] = L1[i * P1 + j];
      op->cd.BtW[i][j] = op->B1[j][i] * op->gauss_w[j];
      double s = 0;
      for (int k = 0; k < P1; ++k) s += op->B1[k][i] * L1[k * P1 + j];
      op->cd.BtL[i][j] = s;
    }
  }
  op->cd.kappa = kin * h / 2.0;  // kin (2/h)^2 (h/2)^3
  op->cd.mscale = std::pow(h / 2.0, -1.5);
  for (int i = 0; i < P1; ++i)
    for (int j = 0; j < P1; ++j) op->cd.Dh[i][j] = Dh[i * P1 + j];
  if (P1 == 5) {
    // even and odd halves for the degree-4 cell kernel; the matrices are unchanged by the
    // reflection of both indices up to rounding (symmetric nodes and points)
    auto halves = [&](auto at, double scale, EO5<double>& r) {
      double big = 0, asym = 0;
      for (int q = 0; q < 5; ++q)
        for (int a = 0; a < 5; ++a) {
          big = std::max(big, std::fabs(at(q, a)));
          asym = std::max(asym, std::fabs(at(q, a) - at(4 - q, 4 - a)));
        }
      for (int q = 0; q < 3; ++q) {
        for (int a = 0; a < 2; ++a) r.e[q][a] = scale * 0.5 * (at(q, a) + at(q, 4 - a));
        r.e[q][2] = scale * at(q, 2);
      }
      for (int q = 0; q < 2; ++q)
        for (int a = 0; a < 2; ++a) r.o[q][a] = scale * 0.5 * (at(q, a) - at(q, 4 - a));
      return asym <= 1e-12 * big;
    };
    auto& c = op->cd;
    const bool sym = halves([&](int q, int a) { return c.B1[q][a]; }, 1.0, c.eB1) &&
                     halves([&](int q, int a) { return c.B1[a][q]; }, 1.0, c.eB1t) &&
                     halves([&](int q, int a) { return c.L1[q][a]; }, 1.0, c.eL1) &&
                     halves([&](int q, int a) { return c.BtW[q][a]; }, 1.0, c.eBtW) &&
                     halves([&](int q, int a) { return c.BtW[q][a]; }, c.kappa, c.ekBtW);
    if (!sym) {
      err = "the 1D cell matrices of degree 4 are not reflection-symmetric";
      return OEFE_EINVAL;
    }
  }
  for (int d = 0; d < 3; ++d) op->uk[d] = uf ? std::pow(h / 2.0, 3) * (2.0 / h) * op->kvec[d] : 0.0;
  {
    auto& f = op->cf;
    auto& c = op->cd;
    for (int i = 0; i < kMaxP1; ++i) {
      f.w[i] = (float)c.w[i];
      f.om[i] = (float)c.om[i];
      for (int j = 0; j < kMaxP1; ++j) {
        f.B1[i][j] = (float)c.B1[i][j];
        f.L1[i][j] = (float)c.L1[i][j];
        f.BtL[i][j] = (float)c.BtL[i][j];
        f.BtW[i][j] = (float)c.BtW[i][j];
      }
    }
    f.kappa = (float)c.kappa;
    f.mscale = (float)c.mscale;
    for (int i = 0; i < kMaxP1; ++i)
      for (int j = 0; j < kMaxP1; ++j) f.Dh[i][j] = (float)c.Dh[i][j];
    auto to_f = [](const EO5<double>& d, EO5<float>& r) {
      for (int q = 0; q < 3; ++q)
        for (int a = 0; a < 3; ++a) r.e[q][a] = (float)d.e[q][a];
      for (int q = 0; q < 2; ++q)
        for (int a = 0; a < 2; ++a) r.o[q][a] = (float)d.o[q][a];
    };
    to_f(c.eB1, f.eB1);
    to_f(c.eB1t, f.eB1t);
    to_f(c.eL1, f.eL1);
    to_f(c.eBtW, f.eBtW);
    to_f(c.ekBtW, f.ekBtW);
  }
  // ---- lumped GLL mass m_g = (h/2)^3 prod_d w'(i_d mod p)
  const int n = op->n;
  op->mdiag.resize(op->N);
  for (int64_t g = 0; g < op->N; ++g) {
    int ix = g % n, iy = (g / n) % n, iz = g / ((int64_t)n * n);
    double m = std::pow(h / 2.0, 3);
    int ii[3] = {ix % p, iy % p, iz % p};
    for (int d = 0; d < 3; ++d) m *= what[ii[d]] * (ii[d] == 0 ? 2.0 : 1.0);
    op->mdiag[g] = m;
  }
  Geo geo{op};
  const int nq = op->nq;
  // ---- quadrature weights and potential
  op->W.resize(op->n_cells * nq);
  op->V.resize(op->n_cells * nq);
  const double h3 = std::pow(h / 2.0, 3);
  for (int64_t e = 0; e < op->n_cells; ++e)
    for (int q = 0; q < nq; ++q) {
      int qx = q % P1, qy = (q / P1) % P1, qz = q / (P1 * P1);
      op->W[e * nq + q] = h3 * op->gauss_w[qx] * op->gauss_w[qy] * op->gauss_w[qz];
      double x[3];
      geo.quad_point(e, q, x);
      double v = 0.0;
      for (int I = 0; I < (pois ? 0 : desc->n_atoms); ++I) {
        double d2 = 0;
        for (int k = 0; k < 3; ++k) {
          double dd = x[k] - desc->pos[3 * I + k];
          dd -= op->L * std::nearbyint(dd / op->L);
          d2 += dd * dd;
        }
        v -= desc->Z[I] * erf_over_r(std::sqrt(d2), desc->sigma);
      }
      op->V[e * nq + q] = v + op->vshift;  // the periodic-function form's |k|^2/2 rides on V
    }
  // ---- Poisson operator: smearing radii (half the distance to the nearest other atom or
  // periodic image, the largest radii without overlap) and the smeared nuclear charge
  // b = -sum_I Z_I g(|x - R_I|, rc_I) at the quadrature points (eqnsmeared, nearest image)
  std::vector<double> alpha_m;
  if (pois) {
    const int na = desc->n_atoms;
    op->rc_smear.assign(na, 0.0);
    alpha_m.assign(na, 0.0);
    for (int I = 0; I < na; ++I) {
      double best = 1e300;
      for (int J = 0; J < na; ++J)
        for (int sz = -1; sz <= 1; ++sz)
          for (int sy = -1; sy <= 1; ++sy)
            for (int sx = -1; sx <= 1; ++sx) {
              if (J == I && sx == 0 && sy == 0 && sz == 0) continue;
              const int sh[3] = {sx, sy, sz};
              double d2 = 0;
              for (int k = 0; k < 3; ++k) {
                const double dd = desc->pos[3 * J + k] + op->L * sh[k] - desc->pos[3 * I + k];
                d2 += dd * dd;
              }
              best = std::min(best, std::sqrt(d2));
            }
      op->rc_smear[I] = 0.5 * best;
      alpha_m[I] = 2.0 * std::cbrt(desc->Z[I]);
    }
    op->bsmear.assign(op->n_cells * nq, 0.0);
    for (int64_t e = 0; e < op->n_cells; ++e)
      for (int q = 0; q < nq; ++q) {
        double x[3];
        geo.quad_point(e, q, x);
        double b = 0.0;
        for (int I = 0; I < na; ++I) {
          double d2 = 0;
          for (int k = 0; k < 3; ++k) {
            double dd = x[k] - desc->pos[3 * I + k];
            dd -= op->L * std::nearbyint(dd / op->L);
            d2 += dd * dd;
          }
          b -= desc->Z[I] * smeared_g(std::sqrt(d2), op->rc_smear[I]);
        }
        op->bsmear[e * nq + q] = b;
      }
  }
  // ---- enrichment blocks (one per atom with functions; the Poisson operator: one per atom)
  op->blocks.clear();
  if (pois) {
    for (int I = 0; I < desc->n_atoms; ++I) {
      AtomBlock b;
      b.atom = I;
      b.fn0 = I;
      b.nf = 1;
      op->blocks.push_back(std::move(b));
    }
  } else if (op->n_enr > 0) {
    for (int nu = 0; nu < op->n_enr; ++nu) {
      int I = desc->enr_atom[nu];
      if (I < 0 || I >= desc->n_atoms) { err = "enrichment atom index out of range"; return OEFE_EINVAL; }
      if (nu > 0 && desc->enr_atom[nu] < desc->enr_atom[nu - 1]) {
        err = "enrichment list must be grouped by atom in ascending order";
        return OEFE_EINVAL;
      }
    }
    int nu = 0;
    while (nu < op->n_enr) {
      AtomBlock b;
      b.atom = desc->enr_atom[nu];
      b.fn0 = nu;
      while (nu < op->n_enr && desc->enr_atom[nu] == b.atom) ++nu;
      b.nf = nu - b.fn0;
      op->blocks.push_back(std::move(b));
    }
  }
  int FMAX = 1;
  for (auto& b : op->blocks) FMAX = std::max(FMAX, b.nf);
  if (FMAX > 8) { err = "at most 8 enrichment functions per atom are supported"; return OEFE_EUNSUPPORTED; }
  op->FMAX = FMAX;
  // matrices for the sum-factorized transforms (stride 8)
  double Bm[64], Dm[64];
  for (int i = 0; i < P1; ++i)
    for (int j = 0; j < P1; ++j) {
      Bm[i * 8 + j] = op->B1[i][j];
      Dm[i * 8 + j] = op->D1[i][j];
    }
  const double s2h = 2.0 / h;
  for (auto& b : op->blocks) {
    const double* R = &desc->pos[3 * b.atom];
    // core cells: box within r1 of the atom (nearest image); support: core dilated by one layer
    std::vector<char> core(op->n_cells, 0), sup(op->n_cells, 0);
    for (int64_t e = 0; e < op->n_cells; ++e) {
      int c[3] = {(int)(e % op->nc), (int)((e / op->nc) % op->nc), (int)(e / ((int64_t)op->nc * op->nc))};
      double dist2 = 0;
      for (int k = 0; k < 3; ++k) {
        double dd = R[k] - (c[k] + 0.5) * h;
        dd -= op->L * std::nearbyint(dd / op->L);
        double ex = std::max(std::fabs(dd) - h / 2.0, 0.0);
        dist2 += ex * ex;
      }
      if (dist2 < desc->r1 * desc->r1) core[e] = 1;
    }
    for (int64_t e = 0; e < op->n_cells; ++e) {
      if (!core[e]) continue;
      int cx = e % op->nc, cy = (e / op->nc) % op->nc, cz = e / ((int64_t)op->nc * op->nc);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) sup[geo.cell_of(cx + dx, cy + dy, cz + dz)] = 1;
    }
    for (int64_t e = 0; e < op->n_cells; ++e)
      if (sup[e]) b.cells.push_back(e);
  }
  // ---- adaptive quadrature of the enrichment integrals: the rule on the union of the supports
  const bool ad = op->adaptive;
  if (ad) {
    // trial functions: the atomic functions without phase, or the auxiliary-potential enrichment
    std::vector<double> sA(op->n_enr), sB(op->n_enr);
    TrialEval eval;
    if (pois) {
      eval = [&](int I, int, const double d[3], double& v, double g[3]) {
        phi_aux_fn(d, desc->Z[I], alpha_m[I], op->rc_smear[I], desc->r0, desc->r1, v, g);
      };
      for (int I = 0; I < op->n_enr; ++I)
        radial_scales(
            [&](double r, double& g, double& gp) {
              const double d[3] = {r, 0.0, 0.0};
              double gr[3];
              phi_aux_fn(d, desc->Z[I], alpha_m[I], op->rc_smear[I], desc->r0, desc->r1, g, gr);
              gp = gr[0];
            },
            -1, desc->r1, sA[I], sB[I]);
    } else {
      eval = [&](int, int fn, const double d[3], double& v, double g[3]) {
        atomic_fn(d, desc->enr_power[fn], desc->enr_zeta[fn], desc->enr_axis[fn], desc->r0, desc->r1, v, g);
      };
      for (int fn = 0; fn < op->n_enr; ++fn)
        radial_scales(
            [&](double r, double& g, double& gp) {
              const double d[3] = {r, 0.0, 0.0};
              double gr[3];
              atomic_fn(d, desc->enr_power[fn], desc->enr_zeta[fn], -1, desc->r0, desc->r1, g, gr);
              gp = gr[0];
            },
            desc->enr_axis[fn], desc->r1, sA[fn], sB[fn]);
    }
    if (int rc = build_adaptive_rule(op, desc, xi, eval, sA, sB, err)) return rc;
  }
  const int nq3 = nq;
  // blocks are independent: host threads over contiguous block ranges, each with its own scratch
  auto block_work = [&](size_t b0, size_t b1) {
    std::vector<cplx> dacc;   // [N][nf] accumulation of d (reused)
    std::vector<char> touched;
    for (size_t ib = b0; ib < b1; ++ib) {
      auto& b = op->blocks[ib];
      const double* R = &desc->pos[3 * b.atom];
      const int nf = b.nf;
      const size_t ncb = b.cells.size();
      // N^A and grad N^A at the quadrature points of the support cells
      std::vector<cplx> NA(ncb * nq * nf), gNA(ncb * nq * nf * 3);
      for (size_t ci = 0; ci < ncb; ++ci) {
        int64_t e = b.cells[ci];
        for (int q = 0; q < nq; ++q) {
          double x[3], d[3], t[3];
          geo.quad_point(e, q, x);
          for (int k = 0; k < 3; ++k) {
            double dr = x[k] - R[k];
            t[k] = std::nearbyint(dr / op->L);
            d[k] = dr - op->L * t[k];
          }
          cplx ph(1.0, 0.0);
          if (uf) {  // exp(-i k . (x - R^x)) (eqnUOEFEAtomic)
            double arg = -(op->kvec[0] * d[0] + op->kvec[1] * d[1] + op->kvec[2] * d[2]);
            ph = cplx(std::cos(arg), std::sin(arg));
          } else if (op->cplx) {
            double arg = op->L * (op->kvec[0] * t[0] + op->kvec[1] * t[1] + op->kvec[2] * t[2]);
            ph = cplx(std::cos(arg), std::sin(arg));
          }
          for (int f = 0; f < nf; ++f) {
            int fn = b.fn0 + f;
            double val, gr[3];
            if (pois)
              phi_aux_fn(d, desc->Z[b.atom], alpha_m[b.atom], op->rc_smear[b.atom], desc->r0, desc->r1, val, gr);
            else
              atomic_fn(d, desc->enr_power[fn], desc->enr_zeta[fn], desc->enr_axis[fn], desc->r0, desc->r1, val, gr);
            NA[(ci * nq + q) * nf + f] = ph * val;
            for (int k = 0; k < 3; ++k)  // the periodic-function form: grad (e^{-ik.d} f) = e^{-ik.d} (grad f - i k f)
              gNA[((ci * nq + q) * nf + f) * 3 + k] = ph * (uf ? cplx(gr[k], -op->kvec[k] * val) : cplx(gr[k], 0.0));
          }
        }
      }
      // adaptive rule: N^A and grad N^A at the rule's points of the support cells
      std::vector<cplx> NAa, gNAa;
      if (ad) {
        b.aoff.assign(ncb + 1, 0);
        for (size_t ci = 0; ci < ncb; ++ci) {
          const int32_t k = op->ad_index[b.cells[ci]];
          b.aoff[ci + 1] = b.aoff[ci] + (op->ad_off[k + 1] - op->ad_off[k]);
        }
        NAa.assign((size_t)b.aoff[ncb] * nf, cplx(0, 0));
        gNAa.assign((size_t)b.aoff[ncb] * nf * 3, cplx(0, 0));
        for (size_t ci = 0; ci < ncb; ++ci) {
          const int32_t k = op->ad_index[b.cells[ci]];
          for (int64_t i = op->ad_off[k]; i < op->ad_off[k + 1]; ++i) {
            const int64_t row = b.aoff[ci] + (i - op->ad_off[k]);
            double d[3], t[3];
            for (int kk = 0; kk < 3; ++kk) {
              const double dr = op->ad_x[3 * i + kk] - R[kk];
              t[kk] = std::nearbyint(dr / op->L);
              d[kk] = dr - op->L * t[kk];
            }
            cplx ph(1.0, 0.0);
            if (uf) {  // exp(-i k . (x - R^x)) (eqnUOEFEAtomic)
              const double arg = -(op->kvec[0] * d[0] + op->kvec[1] * d[1] + op->kvec[2] * d[2]);
              ph = cplx(std::cos(arg), std::sin(arg));
            } else if (op->cplx) {
              const double arg = op->L * (op->kvec[0] * t[0] + op->kvec[1] * t[1] + op->kvec[2] * t[2]);
              ph = cplx(std::cos(arg), std::sin(arg));
            }
            for (int f = 0; f < nf; ++f) {
              const int fn = b.fn0 + f;
              double val, gr[3];
              if (pois)
                phi_aux_fn(d, desc->Z[b.atom], alpha_m[b.atom], op->rc_smear[b.atom], desc->r0, desc->r1, val, gr);
              else
                atomic_fn(d, desc->enr_power[fn], desc->enr_zeta[fn], desc->enr_axis[fn], desc->r0, desc->r1, val, gr);
              NAa[(size_t)row * nf + f] = ph * val;
              for (int kk = 0; kk < 3; ++kk)  // the periodic-function form: e^{-ik.d} (grad f - i k f)
                gNAa[((size_t)row * nf + f) * 3 + kk] = ph * (uf ? cplx(gr[kk], -op->kvec[kk] * val) : cplx(gr[kk], 0.0));
            }
          }
        }
      }
      // d_g = sum_{(e,a)->g} conj(theta_ea) sum_q W B[q,a] N^A ; c_g = d_g / m_g (the adaptive
      // rule's points and weights in place of the cell's Gauss rule when it is in use)
      dacc.assign((size_t)op->N * nf, cplx(0, 0));
      std::vector<cplx> tin(nq), tout(nq);
      for (size_t ci = 0; ad && ci < ncb; ++ci) {
        const int64_t e = b.cells[ci];
        const int32_t k = op->ad_index[e];
        for (int f = 0; f < nf; ++f) {
          std::vector<cplx> acc(op->nd, cplx(0, 0));
          for (int64_t l = op->ad_off[k] / nq3; l < op->ad_off[k + 1] / nq3; ++l) {
            double Mx[64], My[64], Mz[64];
            leaf_matrix(op, l, 0, false, Mx);
            leaf_matrix(op, l, 1, false, My);
            leaf_matrix(op, l, 2, false, Mz);
            const int64_t row0 = b.aoff[ci] + (l * nq3 - op->ad_off[k]);
            for (int q = 0; q < nq; ++q) tin[q] = op->ad_w[l * nq3 + q] * NAa[(size_t)(row0 + q) * nf + f];
            tp_backward<cplx>(P1, Mx, My, Mz, tin.data(), tout.data());
            for (int a = 0; a < op->nd; ++a) acc[a] += tout[a];
          }
          for (int a = 0; a < op->nd; ++a) {
            int64_t g;
            cplx th;
            geo.dof(e, a, g, th);
            dacc[(size_t)g * nf + f] += std::conj(th) * acc[a];
          }
        }
      }
      for (size_t ci = 0; !ad && ci < ncb; ++ci) {
        int64_t e = b.cells[ci];
        for (int f = 0; f < nf; ++f) {
          for (int q = 0; q < nq; ++q) tin[q] = op->W[e * nq + q] * NA[(ci * nq + q) * nf + f];
          tp_backward<cplx>(P1, Bm, Bm, Bm, tin.data(), tout.data());
          for (int a = 0; a < op->nd; ++a) {
            int64_t g;
            cplx th;
            geo.dof(e, a, g, th);
            dacc[(size_t)g * nf + f] += std::conj(th) * tout[a];
          }
        }
      }
      // orthogonalized values and gradients
      b.phi.assign(ncb * nq * nf, cplx(0, 0));
      b.gphi.assign(ncb * nq * nf * 3, cplx(0, 0));
      std::vector<cplx> ce(op->nd), o(nq);
      for (size_t ci = 0; ci < ncb; ++ci) {
        int64_t e = b.cells[ci];
        for (int f = 0; f < nf; ++f) {
          for (int a = 0; a < op->nd; ++a) {
            int64_t g;
            cplx th;
            geo.dof(e, a, g, th);
            ce[a] = th * (dacc[(size_t)g * nf + f] / op->mdiag[g]);
          }
          tp_forward<cplx>(P1, Bm, Bm, Bm, ce.data(), o.data());
          for (int q = 0; q < nq; ++q) b.phi[(ci * nq + q) * nf + f] = NA[(ci * nq + q) * nf + f] - o[q];
          for (int dd = 0; dd < 3; ++dd) {
            const double* Mx = dd == 0 ? Dm : Bm;
            const double* My = dd == 1 ? Dm : Bm;
            const double* Mz = dd == 2 ? Dm : Bm;
            tp_forward<cplx>(P1, Mx, My, Mz, ce.data(), o.data());
            for (int q = 0; q < nq; ++q)
              b.gphi[((ci * nq + q) * nf + f) * 3 + dd] = gNA[((ci * nq + q) * nf + f) * 3 + dd] - s2h * o[q];
          }
        }
      }
      // adaptive rule: N^O and grad N^O at its points with the same coefficients
      if (ad) {
        b.phiA.assign((size_t)b.aoff[ncb] * nf, cplx(0, 0));
        b.gphiA.assign((size_t)b.aoff[ncb] * nf * 3, cplx(0, 0));
        for (size_t ci = 0; ci < ncb; ++ci) {
          const int64_t e = b.cells[ci];
          const int32_t k = op->ad_index[e];
          for (int f = 0; f < nf; ++f) {
            for (int a = 0; a < op->nd; ++a) {
              int64_t g;
              cplx th;
              geo.dof(e, a, g, th);
              ce[a] = th * (dacc[(size_t)g * nf + f] / op->mdiag[g]);
            }
            for (int64_t l = op->ad_off[k] / nq3; l < op->ad_off[k + 1] / nq3; ++l) {
              double Bx[64], By[64], Bz[64], Dx[64], Dy[64], Dz[64];
              leaf_matrix(op, l, 0, false, Bx);
              leaf_matrix(op, l, 1, false, By);
              leaf_matrix(op, l, 2, false, Bz);
              leaf_matrix(op, l, 0, true, Dx);
              leaf_matrix(op, l, 1, true, Dy);
              leaf_matrix(op, l, 2, true, Dz);
              const int64_t row0 = b.aoff[ci] + (l * nq3 - op->ad_off[k]);
              tp_forward<cplx>(P1, Bx, By, Bz, ce.data(), o.data());
              for (int q = 0; q < nq; ++q) b.phiA[(size_t)(row0 + q) * nf + f] = NAa[(size_t)(row0 + q) * nf + f] - o[q];
              for (int dd = 0; dd < 3; ++dd) {
                tp_forward<cplx>(P1, dd == 0 ? Dx : Bx, dd == 1 ? Dy : By, dd == 2 ? Dz : Bz, ce.data(), o.data());
                for (int q = 0; q < nq; ++q)
                  b.gphiA[((size_t)(row0 + q) * nf + f) * 3 + dd] = gNAa[((size_t)(row0 + q) * nf + f) * 3 + dd] - s2h * o[q];
              }
            }
          }
        }
      }
      // rows of H^co: all FE nodes of the support cells
      touched.assign(op->N, 0);
      for (size_t ci = 0; ci < ncb; ++ci)
        for (int a = 0; a < op->nd; ++a) {
          int64_t g;
          cplx th;
          geo.dof(b.cells[ci], a, g, th);
          touched[g] = 1;
        }
      b.rows.clear();
      for (int64_t g = 0; g < op->N; ++g)
        if (touched[g]) b.rows.push_back((int32_t)g);
      // kinetic part of H^co: sum_q W kin (2/h) G_d[q,a] dPhi_d (the adaptive rule's points when in use)
      dacc.assign((size_t)op->N * nf, cplx(0, 0));
      for (size_t ci = 0; ad && ci < ncb; ++ci) {
        const int64_t e = b.cells[ci];
        const int32_t k = op->ad_index[e];
        for (int f = 0; f < nf; ++f) {
          std::vector<cplx> acc(op->nd, cplx(0, 0));
          for (int64_t l = op->ad_off[k] / nq3; l < op->ad_off[k + 1] / nq3; ++l) {
            double Bx[64], By[64], Bz[64], Dx[64], Dy[64], Dz[64];
            leaf_matrix(op, l, 0, false, Bx);
            leaf_matrix(op, l, 1, false, By);
            leaf_matrix(op, l, 2, false, Bz);
            leaf_matrix(op, l, 0, true, Dx);
            leaf_matrix(op, l, 1, true, Dy);
            leaf_matrix(op, l, 2, true, Dz);
            const int64_t row0 = b.aoff[ci] + (l * nq3 - op->ad_off[k]);
            for (int dd = 0; dd < 3; ++dd) {
              const double* Mx = dd == 0 ? Dx : Bx;
              const double* My = dd == 1 ? Dy : By;
              const double* Mz = dd == 2 ? Dz : Bz;
              for (int q = 0; q < nq; ++q)
                tin[q] = kin * s2h * op->ad_w[l * nq3 + q] * b.gphiA[((size_t)(row0 + q) * nf + f) * 3 + dd];
              tp_backward<cplx>(P1, Mx, My, Mz, tin.data(), tout.data());
              for (int a = 0; a < op->nd; ++a) acc[a] += tout[a];
              if (uf) {  // the first-derivative term in Hermitian form, on the rule's points
                const cplx mi(0.0, -0.5 * op->kvec[dd]), pi(0.0, 0.5 * op->kvec[dd]);
                for (int q = 0; q < nq; ++q)
                  tin[q] = mi * op->ad_w[l * nq3 + q] * b.gphiA[((size_t)(row0 + q) * nf + f) * 3 + dd];
                tp_backward<cplx>(P1, Bx, By, Bz, tin.data(), tout.data());
                for (int a = 0; a < op->nd; ++a) acc[a] += tout[a];
                for (int q = 0; q < nq; ++q) tin[q] = pi * s2h * op->ad_w[l * nq3 + q] * b.phiA[(size_t)(row0 + q) * nf + f];
                tp_backward<cplx>(P1, Mx, My, Mz, tin.data(), tout.data());
                for (int a = 0; a < op->nd; ++a) acc[a] += tout[a];
              }
            }
          }
          for (int a = 0; a < op->nd; ++a) {
            int64_t g;
            cplx th;
            geo.dof(e, a, g, th);
            dacc[(size_t)g * nf + f] += std::conj(th) * acc[a];
          }
        }
      }
      for (size_t ci = 0; !ad && ci < ncb; ++ci) {
        int64_t e = b.cells[ci];
        for (int f = 0; f < nf; ++f) {
          std::vector<cplx> acc(op->nd, cplx(0, 0));
          for (int dd = 0; dd < 3; ++dd) {
            for (int q = 0; q < nq; ++q)
              tin[q] = kin * s2h * op->W[e * nq + q] * b.gphi[((ci * nq + q) * nf + f) * 3 + dd];
            const double* Mx = dd == 0 ? Dm : Bm;
            const double* My = dd == 1 ? Dm : Bm;
            const double* Mz = dd == 2 ? Dm : Bm;
            tp_backward<cplx>(P1, Mx, My, Mz, tin.data(), tout.data());
            for (int a = 0; a < op->nd; ++a) acc[a] += tout[a];
            if (uf) {
              // the first-derivative term in Hermitian form (the enrichment function is not a
              // polynomial): -i/2 k_d int N^C d_d Phi + i/2 k_d int (d_d N^C) Phi
              const cplx mi(0.0, -0.5 * op->kvec[dd]), pi(0.0, 0.5 * op->kvec[dd]);
              for (int q = 0; q < nq; ++q) tin[q] = mi * op->W[e * nq + q] * b.gphi[((ci * nq + q) * nf + f) * 3 + dd];
              tp_backward<cplx>(P1, Bm, Bm, Bm, tin.data(), tout.data());
              for (int a = 0; a < op->nd; ++a) acc[a] += tout[a];
              for (int q = 0; q < nq; ++q) tin[q] = pi * s2h * op->W[e * nq + q] * b.phi[(ci * nq + q) * nf + f];
              tp_backward<cplx>(P1, Mx, My, Mz, tin.data(), tout.data());
              for (int a = 0; a < op->nd; ++a) acc[a] += tout[a];
            }
          }
          for (int a = 0; a < op->nd; ++a) {
            int64_t g;
            cplx th;
            geo.dof(e, a, g, th);
            dacc[(size_t)g * nf + f] += std::conj(th) * acc[a];
          }
        }
      }
      b.hkin.resize(b.rows.size() * nf);
      for (size_t r = 0; r < b.rows.size(); ++r)
        for (int f = 0; f < nf; ++f) b.hkin[r * nf + f] = dacc[(size_t)b.rows[r] * nf + f];
    }
  };
  {
    const size_t nbk = op->blocks.size();
    const size_t nth = std::max<size_t>(1, std::min<size_t>({(size_t)kSetupThreads,
                                                            (size_t)std::max(1u, std::thread::hardware_concurrency()), nbk}));
    std::vector<std::thread> pool;
    for (size_t t = 1; t < nth; ++t) pool.emplace_back(block_work, nbk * t / nth, nbk * (t + 1) / nth);
    block_work(0, nbk / nth);
    for (auto& th : pool) th.join();
  }
  // ---- M^oo and the kinetic part of H^oo over common support cells
  const int nO = op->n_enr;
  op->Moo.assign((size_t)nO * nO, cplx(0, 0));
  op->Hoo_kin.assign((size_t)nO * nO, cplx(0, 0));
  // one block's rows at a time (disjoint rows of M^oo and H^oo_kin: host threads over the blocks,
  // every entry summed in the same order as on one thread)
  auto pair_rows = [&](size_t b0, size_t b1) {
    for (size_t ib = b0; ib < b1; ++ib) {
      auto& bi = op->blocks[ib];
      for (auto& bj : op->blocks) {
        size_t i = 0, j = 0;
        while (i < bi.cells.size() && j < bj.cells.size()) {
          if (bi.cells[i] < bj.cells[j]) { ++i; continue; }
          if (bi.cells[i] > bj.cells[j]) { ++j; continue; }
          int64_t e = bi.cells[i];
          if (ad) {  // the adaptive rule's points of cell e (the same rows for both blocks' functions)
            const int32_t k = op->ad_index[e];
            const int64_t npt = op->ad_off[k + 1] - op->ad_off[k];
            for (int64_t pt = 0; pt < npt; ++pt) {
              const double Wq = op->ad_w[op->ad_off[k] + pt];
              const int64_t ri = bi.aoff[i] + pt, rj = bj.aoff[j] + pt;
              for (int f = 0; f < bi.nf; ++f) {
                const cplx a = std::conj(bi.phiA[(size_t)ri * bi.nf + f]);
                const cplx* ga = &bi.gphiA[((size_t)ri * bi.nf + f) * 3];
                for (int g2 = 0; g2 < bj.nf; ++g2) {
                  const cplx bb = bj.phiA[(size_t)rj * bj.nf + g2];
                  const cplx* gb = &bj.gphiA[((size_t)rj * bj.nf + g2) * 3];
                  const size_t ix = (size_t)(bi.fn0 + f) * nO + (bj.fn0 + g2);
                  op->Moo[ix] += Wq * a * bb;
                  op->Hoo_kin[ix] +=
                      kin * Wq * (std::conj(ga[0]) * gb[0] + std::conj(ga[1]) * gb[1] + std::conj(ga[2]) * gb[2]);
                  if (uf) {  // -i/2 k . int (Phi_i^* grad Phi_j - grad Phi_i^* Phi_j)
                    cplx t(0.0, 0.0);
                    for (int kk = 0; kk < 3; ++kk) t += op->kvec[kk] * (a * gb[kk] - std::conj(ga[kk]) * bb);
                    op->Hoo_kin[ix] += cplx(0.0, -0.5) * Wq * t;
                  }
                }
              }
            }
            ++i;
            ++j;
            continue;
          }
          for (int q = 0; q < nq; ++q) {
            double Wq = op->W[e * nq + q];
            for (int f = 0; f < bi.nf; ++f) {
              cplx a = std::conj(bi.phi[(i * nq + q) * bi.nf + f]);
              const cplx* ga = &bi.gphi[((i * nq + q) * bi.nf + f) * 3];
              for (int g2 = 0; g2 < bj.nf; ++g2) {
                cplx bb = bj.phi[(j * nq + q) * bj.nf + g2];
                const cplx* gb = &bj.gphi[((j * nq + q) * bj.nf + g2) * 3];
                size_t ix = (size_t)(bi.fn0 + f) * nO + (bj.fn0 + g2);
                op->Moo[ix] += Wq * a * bb;
                op->Hoo_kin[ix] +=
                    kin * Wq * (std::conj(ga[0]) * gb[0] + std::conj(ga[1]) * gb[1] + std::conj(ga[2]) * gb[2]);
                if (uf) {  // -i/2 k . int (Phi_i^* grad Phi_j - grad Phi_i^* Phi_j)
                  cplx t(0.0, 0.0);
                  for (int k = 0; k < 3; ++k) t += op->kvec[k] * (a * gb[k] - std::conj(ga[k]) * bb);
                  op->Hoo_kin[ix] += cplx(0.0, -0.5) * Wq * t;
                }
              }
            }
          }
          ++i;
          ++j;
        }
      }
    }
  };
  {
    const size_t nbk = op->blocks.size();
    const size_t nth = std::max<size_t>(1, std::min<size_t>({(size_t)kSetupThreads,
                                                            (size_t)std::max(1u, std::thread::hardware_concurrency()), nbk}));
    std::vector<std::thread> pool;
    for (size_t t = 1; t < nth; ++t) pool.emplace_back(pair_rows, nbk * t / nth, nbk * (t + 1) / nth);
    pair_rows(0, nbk / nth);
    for (auto& th : pool) th.join();
  }
  for (auto& b : op->blocks) std::vector<cplx>().swap(b.gphiA);  // set-up only
  // ---- S = (M^oo)^-1/2; for the Poisson operator the block's own metric is A^oo, so that
  // S A^oo S = I (the enrichment rows' Jacobi factor of the preconditioned Laplacian)
  if (pois) op->Moo = op->Hoo_kin;
  if (nO > 0) {
    std::vector<cplx> A(op->Moo), U;
    for (int i = 0; i < nO; ++i)
      for (int j = 0; j < nO; ++j) A[(size_t)i * nO + j] = 0.5 * (op->Moo[(size_t)i * nO + j] + std::conj(op->Moo[(size_t)j * nO + i]));
    hermitian_eig(nO, A, op->Moo_eigs, U);
    if (op->Moo_eigs[0] <= 0.0) { err = "enrichment overlap M^oo is not positive definite"; return OEFE_EINVAL; }
    op->S.assign((size_t)nO * nO, cplx(0, 0));
    for (int i = 0; i < nO; ++i)
      for (int j = 0; j < nO; ++j) {
        cplx s = 0;
        for (int k = 0; k < nO; ++k) s += U[(size_t)i * nO + k] * (1.0 / std::sqrt(op->Moo_eigs[k])) * std::conj(U[(size_t)j * nO + k]);
        op->S[(size_t)i * nO + j] = s;
      }
  }
  return rebuild_potential_parts(op, err);
}

// Potential-dependent parts: H^oo = H^oo_kin + sum W V conj(Phi) Phi and the H^co values are
// recomputed by the upload step from the stored kinetic part plus sum_q B[q,a] W V Phi.
int rebuild_potential_parts(oefe_op_s* op, std::string& err) {
  (void)err;
  const int nO = op->n_enr, nq = op->nq, P1 = op->P1;
  op->Hoo = op->Hoo_kin;
  for (auto& bi : op->blocks)
    for (auto& bj : op->blocks) {
      size_t i = 0, j = 0;
      while (i < bi.cells.size() && j < bj.cells.size()) {
        if (bi.cells[i] < bj.cells[j]) { ++i; continue; }
        if (bi.cells[i] > bj.cells[j]) { ++j; continue; }
        int64_t e = bi.cells[i];
        for (int q = 0; q < nq; ++q) {
          double wv = op->W[e * nq + q] * op->V[e * nq + q];
          for (int f = 0; f < bi.nf; ++f) {
            cplx a = std::conj(bi.phi[(i * nq + q) * bi.nf + f]);
            for (int g2 = 0; g2 < bj.nf; ++g2)
              op->Hoo[(size_t)(bi.fn0 + f) * nO + (bj.fn0 + g2)] += wv * a * bj.phi[(j * nq + q) * bj.nf + g2];
          }
        }
        ++i;
        ++j;
      }
    }
  (void)P1;
  return OEFE_OK;
}

// H^co values on the rows of block b: kinetic part + potential part.
void block_hco_values(const oefe_op_s* op, const AtomBlock& b, std::vector<cplx>& out) {
  const int nq = op->nq, P1 = op->P1, nf = b.nf;
  double Bm[64];
  for (int i = 0; i < P1; ++i)
    for (int j = 0; j < P1; ++j) Bm[i * 8 + j] = op->B1[i][j];
  Geo geo{op};
  std::vector<cplx> acc((size_t)op->N * 0 + 1);
  // local row index of every global row of this block
  std::vector<int32_t> local(op->N, -1);
  for (size_t r = 0; r < b.rows.size(); ++r) local[b.rows[r]] = (int32_t)r;
  out.assign(b.rows.size() * nf, cplx(0, 0));
  std::vector<cplx> tin(nq), tout(nq);
  for (size_t ci = 0; ci < b.cells.size(); ++ci) {
    int64_t e = b.cells[ci];
    for (int f = 0; f < nf; ++f) {
      for (int q = 0; q < nq; ++q) tin[q] = op->W[e * nq + q] * op->V[e * nq + q] * b.phi[(ci * nq + q) * nf + f];
      tp_backward<cplx>(P1, Bm, Bm, Bm, tin.data(), tout.data());
      for (int a = 0; a < op->nd; ++a) {
        int64_t g;
        cplx th;
        geo.dof(e, a, g, th);
        out[(size_t)local[g] * nf + f] += std::conj(th) * tout[a];
      }
    }
  }
  for (size_t k = 0; k < out.size(); ++k) out[k] += b.hkin[k];
}

}  // namespace oefe
