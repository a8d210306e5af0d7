// swe_nh_dg1d.hip -- the paper's own 1D discretisation on one workgroup
// (gfx950): second-order Runge-Kutta discontinuous Galerkin with P1 elements
// for the hydrostatic predictor (Sec. 3.1, Eqs. 6-9), the local DG (LDG) P1
// solution of the elliptic system of Eqs. 14-15 with the alternating
// ("flip-flop") flux of Eqs. 16-17 (Sec. 3.2), and the correction of
// Eqs. 10-11; the global model or the adaptive one of Sec. 5 on elements,
// reflective walls.
//
// The paper's setups have a few hundred elements, so one workgroup holds a
// whole channel: thread i owns element i (its node values in registers;
// channels of at most 256 or 512 elements run on 256 or 512 threads, whose
// register budget holds nearly the whole step), neighbours' values pass
// through LDS, and a launch runs many steps with nothing but workgroup
// barriers between the phases.  A batch of independent channels runs one
// workgroup per channel, which is how the method fills the chip.
//
// Discretisation (as the FP64 reference of the same method):
//   * nodal Lagrange P1 on [i dx, (i + 1) dx], nodes at the element ends;
//     consistent mass M = dx/6 [[2, 1], [1, 2]], so M^-1 = 2/dx [[2, -1],
//     [-1, 2]];
//   * element integrals of the flux (h u, h u^2 + g h^2 / 2, h u w) and of
//     the bed source g h d_x by three-point Gauss-Legendre quadrature of the
//     P1 state, d_x the slope of the bottom's P1 interpolant (well balanced);
//   * Rusanov flux at the element faces, mirror states at the walls; Heun
//     with the bottom at t^{n+1} in the second stage;
//   * LDG: p* = p+ and (hu)* = (hu)- inside; p* = 0 at both walls, and at
//     the left wall (hu)* = (hu)+ - c11 p+ with c11 = 1 / (s12 dx); the
//     products of the elliptic system interpolated at the nodes;
//   * hw corrected with the bottom pressure of Eqs. 10-11, node by node.
//
// The LDG system couples element i only through q1_{i-1} (hu at the left
// neighbour's right node, in the row of q0_i) and p0_{i+1} (in the row of
// p1_i).  Each element's 4 x 4 block is solved for its right-hand side and
// those two couplings, u_i = g_i + a_i q1_{i-1} + b_i p0_{i+1}; the pairs
// (q1_{k-1}, p0_k) at the n - 1 interior faces then satisfy a block
// tridiagonal system with 2 x 2 blocks, solved by parallel cyclic reduction
// in LDS, and each element recovers its four unknowns.
//
// Adaptive model: an element outside the non-hydrostatic set publishes its
// fixed values instead of a solved block (q1 = hu~ at its right node, p0 = 0
// at its left node, no couplings), so the interface system carries them as
// identity rows and a marked neighbour's rows see exactly the zero Dirichlet
// datum of the restricted system; the element then keeps the predictor's
// state.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "swe_nh.h"
#include "swe_nh_common.h"

namespace swenh {
namespace {

// threads of the workgroup, one per element: 512 (no register spills) or
// SWE_NH_DG_MAX_ELEMS
constexpr int NTD_SMALL = 512;
// channels of at most 256 elements: two such workgroups fit on a compute unit
// where one of 512 threads (8 wavefronts of 256 VGPRs) fills it
constexpr int NTD_TINY = 256;

struct DgArgs {
  int n, nsteps;
  double dx, dt, g, rho, ds, t0;
  Chan body;
  double *h, *hu, *hw, *p;
  int* status;
  int adaptive, crit, enlarge, first_global;
  double k_nh;
  int* marked;
};

template <int NTD>
struct DgSmem {
  union {
    struct {
      double q[3][NTD][2];  // node values of a stage's input
      double F[3][NTD + 1];  // Rusanov fluxes at the faces
    } s;
    struct {
      double v[3][NTD];  // (g, a, b) components at the right node's q of each element
    } c;
    struct {
      double A[4][NTD], B[4][NTD], C[4][NTD], d[2][NTD];  // interface rows, 2 x 2 row-major
    } r[NTD <= 512 ? 2 : 1];  // two buffers (one barrier per reduction level) where LDS allows
  } u;
  int status;
  unsigned char raw[NTD];  // criterion exceeded (adaptive model)
};

__device__ __forceinline__ void phys_flux(double g, double h, double m, double k, double (&F)[3]) {
  const double r = 1.0 / h;
  F[0] = m;
  F[1] = m * m * r + 0.5 * g * h * h;
  F[2] = m * k * r;
}

// H(Q) of the semi-discrete form for this thread's element (all threads
// call: the barriers are the workgroup's)
template <int NTD>
__device__ void dg_operator(DgSmem<NTD>& S, const DgArgs& A, int i, bool on, const double (&Q)[3][2],
                            double slope, double (&H)[3][2]) {
  const int n = A.n;
  const double g = A.g;
  if (on) {
    for (int a = 0; a < 3; a++) {
      S.u.s.q[a][i][0] = Q[a][0];
      S.u.s.q[a][i][1] = Q[a][1];
    }
    if (!(Q[0][0] > 0.0) || !(Q[0][1] > 0.0)) atomicOr(&S.status, ST_DRY);
  }
  __syncthreads();
  // Rusanov flux at face f between states qm (left) and qp (right)
  auto face = [&](const double (&qm)[3], const double (&qp)[3], int f) {
    double fm[3], fp[3];
    phys_flux(g, qm[0], qm[1], qm[2], fm);
    phys_flux(g, qp[0], qp[1], qp[2], fp);
    const double lam = fmax(fabs(qm[1] / qm[0]) + sqrt(g * qm[0]),
                            fabs(qp[1] / qp[0]) + sqrt(g * qp[0]));
    for (int a = 0; a < 3; a++) S.u.s.F[a][f] = 0.5 * (fm[a] + fp[a]) - 0.5 * lam * (qp[a] - qm[a]);
  };
  if (on) {
    // the element's right face; element 0 also takes the left wall
    const double qm[3] = {Q[0][1], Q[1][1], Q[2][1]};
    if (i + 1 < n) {
      const double qp[3] = {S.u.s.q[0][i + 1][0], S.u.s.q[1][i + 1][0], S.u.s.q[2][i + 1][0]};
      face(qm, qp, i + 1);
    } else {
      const double qp[3] = {Q[0][1], -Q[1][1], Q[2][1]};
      face(qm, qp, n);
    }
    if (i == 0) {
      const double wl[3] = {Q[0][0], -Q[1][0], Q[2][0]}, q0[3] = {Q[0][0], Q[1][0], Q[2][0]};
      face(wl, q0, 0);
    }
  }
  __syncthreads();
  if (on) {
    // Gauss-Legendre points of [0, 1] and their weights
    const double s6 = 0.5 * sqrt(0.6);
    const double xg[3] = {0.5 - s6, 0.5, 0.5 + s6};
    const double wg[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    double fint[3] = {0.0, 0.0, 0.0}, src[2] = {0.0, 0.0};
    for (int k = 0; k < 3; k++) {
      const double hq = (1.0 - xg[k]) * Q[0][0] + xg[k] * Q[0][1];
      const double mq = (1.0 - xg[k]) * Q[1][0] + xg[k] * Q[1][1];
      const double kq = (1.0 - xg[k]) * Q[2][0] + xg[k] * Q[2][1];
      double F[3];
      phys_flux(g, hq, mq, kq, F);
      for (int a = 0; a < 3; a++) fint[a] += wg[k] * F[a];
      const double s = wg[k] * g * hq * slope;
      src[0] += s * (1.0 - xg[k]);
      src[1] += s * xg[k];
    }
    const double c = 2.0 / A.dx;
    for (int a = 0; a < 3; a++) {
      double r0 = -fint[a] + S.u.s.F[a][i], r1 = fint[a] - S.u.s.F[a][i + 1];
      if (a == 1) {
        r0 += A.dx * src[0];
        r1 += A.dx * src[1];
      }
      H[a][0] = c * (2.0 * r0 - r1);
      H[a][1] = c * (2.0 * r1 - r0);
    }
  }
  __syncthreads();
}

// the bottom at x and time t: d, and (through Shape and BedRate) its
// derivatives; flat static depth ds
struct Bed {
  double d, dx_, dxx, dt_, dtt, dxt;
};
__device__ __forceinline__ Bed bed_at(const DgArgs& A, const Motion& M, double x) {
  const Shape s = body_shape(A.body, x - M.X, 0.0);
  const BedRate r = bed_rate(M, s);
  return Bed{A.ds - s.B, -s.Bx, -s.Bxx, r.d_t, r.d_tt, r.d_xt};
}

// x of A x = b for a 4 x 4 system with three right-hand sides (Gaussian
// elimination with partial pivoting; the columns of b are overwritten)
__device__ void solve4(double (&M)[4][4], double (&b)[4][3]) {
  for (int c = 0; c < 4; c++) {
    int piv = c;
    for (int r = c + 1; r < 4; r++)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < 4; k++) {
        const double t = M[c][k];
        M[c][k] = M[piv][k];
        M[piv][k] = t;
      }
      for (int k = 0; k < 3; k++) {
        const double t = b[c][k];
        b[c][k] = b[piv][k];
        b[piv][k] = t;
      }
    }
    const double inv = 1.0 / M[c][c];
    for (int r = c + 1; r < 4; r++) {
      const double f = M[r][c] * inv;
      for (int k = c; k < 4; k++) M[r][k] -= f * M[c][k];
      for (int k = 0; k < 3; k++) b[r][k] -= f * b[c][k];
    }
  }
  for (int c = 3; c >= 0; c--) {
    const double inv = 1.0 / M[c][c];
    for (int k = 0; k < 3; k++) {
      double s = b[c][k];
      for (int j = c + 1; j < 4; j++) s -= M[c][j] * b[j][k];
      b[c][k] = s * inv;
    }
  }
}

// 2 x 2 helpers (row-major [a b; c d])
__device__ __forceinline__ void inv2(const double (&m)[4], double (&r)[4]) {
  const double id = 1.0 / (m[0] * m[3] - m[1] * m[2]);
  r[0] = m[3] * id;
  r[1] = -m[1] * id;
  r[2] = -m[2] * id;
  r[3] = m[0] * id;
}
__device__ __forceinline__ void mul2(const double (&a)[4], const double (&b)[4], double (&r)[4]) {
  r[0] = a[0] * b[0] + a[1] * b[2];
  r[1] = a[0] * b[1] + a[1] * b[3];
  r[2] = a[2] * b[0] + a[3] * b[2];
  r[3] = a[2] * b[1] + a[3] * b[3];
}

// the element's criterion of Sec. 5.1 on the predictor's node values: the
// larger node value of |eta/d|, |u| or |w|, or the magnitude of the P1 slope
// of eta, u or w; d0, d1 the depths at the nodes at t^{n+1}
__device__ __forceinline__ double element_indicator(int crit, const double (&Qt)[3][2], double d0,
                                                    double d1, double dx) {
  const double h0 = Qt[0][0], h1 = Qt[0][1];
  switch (crit) {
    case SWE_NH_CRIT_ETA_D:
      return fmax(fabs((h0 - d0) / d0), fabs((h1 - d1) / d1));
    case SWE_NH_CRIT_U:
      return fmax(fabs(Qt[1][0] / h0), fabs(Qt[1][1] / h1));
    case SWE_NH_CRIT_W:
      return fmax(fabs(Qt[2][0] / h0), fabs(Qt[2][1] / h1));
    case SWE_NH_CRIT_ETA_X:
      return fabs(((h1 - d1) - (h0 - d0)) / dx);
    case SWE_NH_CRIT_U_X:
      return fabs((Qt[1][1] / h1 - Qt[1][0] / h0) / dx);
    default:  // SWE_NH_CRIT_W_X
      return fabs((Qt[2][1] / h1 - Qt[2][0] / h0) / dx);
  }
}

// whether element i is non-hydrostatic in this step (all threads call: the
// barriers are the workgroup's); thread 0 records the count
template <int NTD>
__device__ bool element_marked(DgSmem<NTD>& S, const DgArgs& A, int i, bool on, int step,
                               const double (&Qt)[3][2], double d0, double d1) {
  const int crit = A.crit;
  bool nh;
  if (crit == SWE_NH_CRIT_GLOBAL ||
      (A.first_global && step == 0 && (crit == SWE_NH_CRIT_W || crit == SWE_NH_CRIT_W_X))) {
    nh = on;
  } else if (crit == SWE_NH_CRIT_NONE) {
    nh = false;
  } else {
    if (on) S.raw[i] = element_indicator(crit, Qt, d0, d1, A.dx) > A.k_nh;
    __syncthreads();
    nh = false;
    if (on) {
      const int lo = max(0, i - A.enlarge), hi = min(A.n - 1, i + A.enlarge);
      for (int k = lo; k <= hi; k++) nh = nh || S.raw[k];
    }
    __syncthreads();  // raw is rewritten in the next step
  }
  const int cnt = __syncthreads_count(nh);
  if (i == 0 && A.marked) A.marked[step] = cnt;
  return nh;
}

// a whole run of one channel on this workgroup; ADAPT: the adaptive model
// (the global model's kernel carries none of it)
template <int NTD, bool ADAPT>
__device__ __forceinline__ void dg1d_channel(DgSmem<NTD>& S, const DgArgs& A) {
  const int i = threadIdx.x, n = A.n;
  const bool on = i < n;
  const double dx = A.dx, dt = A.dt, g = A.g, rho = A.rho;
  if (i == 0) S.status = 0;
  double Q[3][2] = {{1.0, 1.0}, {0.0, 0.0}, {0.0, 0.0}};
  double P[2] = {0.0, 0.0};
  if (on) {
    Q[0][0] = A.h[2 * i];
    Q[0][1] = A.h[2 * i + 1];
    Q[1][0] = A.hu[2 * i];
    Q[1][1] = A.hu[2 * i + 1];
    Q[2][0] = A.hw[2 * i];
    Q[2][1] = A.hw[2 * i + 1];
  }
  const double x0 = i * dx, x1 = (i + 1) * dx;
  for (int step = 0; step < A.nsteps; step++) {
    const double t = A.t0 + step * dt, t1 = t + dt;
    const Motion M0 = body_motion(A.body, t), M1 = body_motion(A.body, t1);
    const Bed b00 = bed_at(A, M0, x0), b01 = bed_at(A, M0, x1);
    const Bed b10 = bed_at(A, M1, x0), b11 = bed_at(A, M1, x1);
    // ---- predictor: Heun over two DG stages (Eqs. 8-9) ----
    double H0[3][2], H1[3][2], Qs[3][2];
    dg_operator(S, A, i, on, Q, (b01.d - b00.d) / dx, H0);
    for (int a = 0; a < 3; a++)
      for (int k = 0; k < 2; k++) Qs[a][k] = Q[a][k] + dt * H0[a][k];
    dg_operator(S, A, i, on, Qs, (b11.d - b10.d) / dx, H1);
    double Qt[3][2];
    for (int a = 0; a < 3; a++)
      for (int k = 0; k < 2; k++) Qt[a][k] = Q[a][k] + 0.5 * dt * (H0[a][k] + H1[a][k]);
    // ---- coefficients of Eqs. 12-15 at the nodes, at t^{n+1} ----
    const Bed bn[2] = {b10, b11};
    const double hx = (Qt[0][1] - Qt[0][0]) / dx;
    const double ex = ((Qt[0][1] - b11.d) - (Qt[0][0] - b10.d)) / dx;
    double s11[2], s12[2], s21[2], s22[2], f1[2], f2[2], al[2], phi[2];
    for (int k = 0; k < 2; k++) {
      const double h = Qt[0][k], m = Qt[1][k], kk = Qt[2][k], ih = 1.0 / h;
      const Bed& b = bn[k];
      const double u = m * ih;
      al[k] = 4.0 + b.dx_ * b.dx_;
      phi[k] = rho * h / al[k] * (g * b.dx_ * ex - b.dtt - 2.0 * u * b.dxt - u * u * b.dxx);
      s11[k] = (2.0 * hx - 3.0 * b.dx_) * 0.5 * ih;
      s12[k] = rho * al[k] / (4.0 * dt * h);
      f1[k] = al[k] / (4.0 * h) * (phi[k] * b.dx_ + rho / dt * m);
      s21[k] = -s11[k];
      s22[k] = 3.0 * dt / (rho * h);
      f2[k] = -2.0 * b.dt_ - 2.0 * kk * ih - b.dx_ * m * 0.5 * ih -
              dt * al[k] * phi[k] / (2.0 * rho * h);
    }
    // ---- the element's LDG block (unknowns p0, p1, q0, q1) ----
    const double Ml[2][2] = {{dx / 3.0, dx / 6.0}, {dx / 6.0, dx / 3.0}};
    const double Dt[2][2] = {{0.5, 0.5}, {-0.5, -0.5}};  // - int (phi_j)_x phi_k, row j, col k
    double Bm[4][4], rh[4][3];
    for (int j = 0; j < 2; j++) {
      for (int k = 0; k < 2; k++) {
        Bm[j][k] = Dt[j][k] + Ml[j][k] * s11[k];
        Bm[j][2 + k] = Ml[j][k] * s12[k];
        Bm[2 + j][2 + k] = Dt[j][k] + Ml[j][k] * s21[k];
        Bm[2 + j][k] = Ml[j][k] * s22[k];
      }
      rh[j][0] = Ml[j][0] * f1[0] + Ml[j][1] * f1[1];
      rh[2 + j][0] = Ml[j][0] * f2[0] + Ml[j][1] * f2[1];
    }
    Bm[3][3] += 1.0;  // + q*_r = q- (own right node; at the right wall too)
    if (i > 0) {
      Bm[0][0] -= 1.0;  // - p*_l = p+ (own left node)
    } else {
      Bm[2][2] -= 1.0;  // left wall: q*_l = q+ - c11 p+, p*_l = 0
      Bm[2][0] += 1.0 / (s12[0] * dx);
    }
    for (int r = 0; r < 4; r++) {
      rh[r][1] = 0.0;
      rh[r][2] = 0.0;
    }
    if (i > 0) rh[2][1] = 1.0;      // the row of q0 holds - q1_{i-1}
    if (i + 1 < n) rh[1][2] = -1.0;  // the row of p1 holds + p0_{i+1}
    const bool nh = ADAPT ? element_marked(S, A, i, on, step, Qt, b10.d, b11.d) : on;
    if (on && nh) {
      solve4(Bm, rh);
    } else if (ADAPT) {
      // fixed unknowns: p = 0, q = hu~ (no couplings)
      for (int r = 0; r < 4; r++) {
        rh[r][0] = r < 2 ? 0.0 : Qt[1][r - 2];
        rh[r][1] = 0.0;
        rh[r][2] = 0.0;
      }
    }
    // u = g + a q1_{i-1} + b p0_{i+1}; the interface rows need the q1
    // components of the left neighbour
    if (on) {
      S.u.c.v[0][i] = rh[3][0];
      S.u.c.v[1][i] = rh[3][1];
      S.u.c.v[2][i] = rh[3][2];
    }
    __syncthreads();
    // interface k = i (between elements k - 1 and k), unknowns (x_k, y_k) =
    // (q1_{k-1}, p0_k), row j = k - 1 of the m = n - 1 rows
    const int m = n - 1, j = i - 1;
    const bool row = i >= 1 && i < n;
    double Ar[4] = {0.0, 0.0, 0.0, 0.0}, Br[4] = {1.0, 0.0, 0.0, 1.0}, Cr[4] = {0.0, 0.0, 0.0, 0.0};
    double dr[2] = {0.0, 0.0};
    if (row) {
      const double gl = S.u.c.v[0][i - 1], al3 = S.u.c.v[1][i - 1], bl3 = S.u.c.v[2][i - 1];
      Br[1] = -bl3;
      Br[2] = -rh[0][1];
      Ar[0] = -al3;
      Cr[3] = -rh[0][2];
      dr[0] = gl;
      dr[1] = rh[0][0];
    }
    __syncthreads();
    constexpr bool TWO = NTD <= 512;  // the level reads one buffer and writes the other
    int cur = 0;
    auto put = [&](int bf) {
      if (!row) return;
      for (int e = 0; e < 4; e++) {
        S.u.r[bf].A[e][j] = Ar[e];
        S.u.r[bf].B[e][j] = Br[e];
        S.u.r[bf].C[e][j] = Cr[e];
      }
      S.u.r[bf].d[0][j] = dr[0];
      S.u.r[bf].d[1][j] = dr[1];
    };
    put(0);
    __syncthreads();
    for (int s = 1; s < m; s *= 2) {
      const auto& R = S.u.r[cur];
      double An[4], Bn[4] = {Br[0], Br[1], Br[2], Br[3]}, Cn[4], dn[2] = {dr[0], dr[1]};
      if (row) {
        double al_[4] = {0.0, 0.0, 0.0, 0.0}, ga_[4] = {0.0, 0.0, 0.0, 0.0};
        double Am[4] = {0.0, 0.0, 0.0, 0.0}, Cp[4] = {0.0, 0.0, 0.0, 0.0};
        if (j - s >= 0) {
          double Bm_[4], Bi[4], Cm[4];
          for (int e = 0; e < 4; e++) {
            Bm_[e] = R.B[e][j - s];
            Am[e] = R.A[e][j - s];
            Cm[e] = R.C[e][j - s];
          }
          inv2(Bm_, Bi);
          mul2(Ar, Bi, al_);
          double t[4];
          mul2(al_, Cm, t);
          for (int e = 0; e < 4; e++) Bn[e] -= t[e];
          dn[0] -= al_[0] * R.d[0][j - s] + al_[1] * R.d[1][j - s];
          dn[1] -= al_[2] * R.d[0][j - s] + al_[3] * R.d[1][j - s];
        }
        if (j + s < m) {
          double Bp[4], Bi[4], Ap[4];
          for (int e = 0; e < 4; e++) {
            Bp[e] = R.B[e][j + s];
            Ap[e] = R.A[e][j + s];
            Cp[e] = R.C[e][j + s];
          }
          inv2(Bp, Bi);
          mul2(Cr, Bi, ga_);
          double t[4];
          mul2(ga_, Ap, t);
          for (int e = 0; e < 4; e++) Bn[e] -= t[e];
          dn[0] -= ga_[0] * R.d[0][j + s] + ga_[1] * R.d[1][j + s];
          dn[1] -= ga_[2] * R.d[0][j + s] + ga_[3] * R.d[1][j + s];
        }
        double t[4];
        mul2(al_, Am, t);
        for (int e = 0; e < 4; e++) An[e] = -t[e];
        mul2(ga_, Cp, t);
        for (int e = 0; e < 4; e++) Cn[e] = -t[e];
      }
      if (!TWO) __syncthreads();  // one buffer: every read of this level first
      if (row) {
        for (int e = 0; e < 4; e++) {
          Ar[e] = An[e];
          Br[e] = Bn[e];
          Cr[e] = Cn[e];
        }
        dr[0] = dn[0];
        dr[1] = dn[1];
      }
      if (TWO) cur ^= 1;
      put(cur);
      __syncthreads();
    }
    // every row is decoupled: (x_k, y_k) = B^-1 d, published through d
    if (row) {
      double Bi[4];
      inv2(Br, Bi);
      const double xk = Bi[0] * dr[0] + Bi[1] * dr[1], yk = Bi[2] * dr[0] + Bi[3] * dr[1];
      S.u.r[cur].d[0][j] = xk;
      S.u.r[cur].d[1][j] = yk;
    }
    __syncthreads();
    const double ql = (on && i >= 1) ? S.u.r[cur].d[0][i - 1] : 0.0;  // q1_{i-1} = x_i
    const double pr = (on && i + 1 < n) ? S.u.r[cur].d[1][i] : 0.0;   // p0_{i+1} = y_{i+1}
    double U[4];
    for (int r = 0; r < 4; r++) U[r] = rh[r][0] + rh[r][1] * ql + rh[r][2] * pr;
    __syncthreads();
    // ---- correction (Eqs. 10-11): hu = q, hw from the bottom pressure;
    // the hydrostatic elements keep the predictor's state ----
    for (int k = 0; k < 2; k++) {
      const double pk = U[k], qk = U[2 + k];
      const double Pb = 1.5 * pk - rho * bn[k].dx_ * (qk - Qt[1][k]) / (4.0 * dt) +
                        al[k] * phi[k] / 4.0;
      const bool keep = ADAPT && !nh;
      Q[0][k] = Qt[0][k];
      Q[1][k] = keep ? Qt[1][k] : qk;
      Q[2][k] = keep ? Qt[2][k] : Qt[2][k] + dt / rho * Pb;
      P[k] = keep ? 0.0 : pk;
    }
  }
  if (on) {
    for (int k = 0; k < 2; k++) {
      A.h[2 * i + k] = Q[0][k];
      A.hu[2 * i + k] = Q[1][k];
      A.hw[2 * i + k] = Q[2][k];
      A.p[2 * i + k] = P[k];
      bool fin = true;
      for (int a = 0; a < 3; a++) fin = fin && isfinite(Q[a][k]);
      if (!fin || !isfinite(P[k])) atomicOr(&S.status, ST_NAN);
    }
  }
  __syncthreads();
  if (i == 0 && S.status) atomicOr(A.status, S.status);
}

// batches: two wavefronts per SIMD at least, so that two 256-thread
// workgroups share a compute unit (the register budget of the 512-thread one)
constexpr int dg_min_waves(int ntd) { return ntd / 256 > 2 ? ntd / 256 : 2; }

// one channel per launch: the workgroup has its compute unit to itself, so
// its registers are bounded by its own size only
template <int NTD, bool ADAPT>
__global__ void __launch_bounds__(NTD) k_dg1d_run(DgArgs A) {
  __shared__ DgSmem<NTD> S;
  dg1d_channel<NTD, ADAPT>(S, A);
}

// one workgroup per channel of a batch
template <int NTD, bool ADAPT>
__global__ void __launch_bounds__(NTD, dg_min_waves(NTD)) k_dg1d_batch(const DgArgs* __restrict__ As) {
  __shared__ DgSmem<NTD> S;
  const DgArgs A = As[blockIdx.x];
  dg1d_channel<NTD, ADAPT>(S, A);
}

}  // namespace
}  // namespace swenh

using namespace swenh;

namespace {
bool dg_config_ok(const swe_nh_dg1d_config* c) {
  if (!c || c->n < 1 || c->n > SWE_NH_DG_MAX_ELEMS || !(c->dx > 0.0) || !(c->dt > 0.0) ||
      !(c->g > 0.0) || !(c->rho > 0.0) || !(c->d_static > 0.0))
    return false;
  return !c->adaptive || (c->crit >= SWE_NH_CRIT_ETA_D && c->crit <= SWE_NH_CRIT_NONE &&
                          c->enlarge >= 0 && c->enlarge <= SWE_NH_DG_MAX_ENLARGE &&
                          c->k_nh >= 0.0);
}

// the kernel arguments of one channel whose node values start at h, hu, hw, p;
// in a kernel with the adaptive model, a channel of the global model takes
// the criterion that marks every element
DgArgs dg_args(const swe_nh_dg1d_config* c, double t0, int nsteps, double* h, double* hu,
               double* hw, double* p, int32_t* status) {
  DgArgs A;
  A.n = c->n;
  A.nsteps = nsteps;
  A.dx = c->dx;
  A.dt = c->dt;
  A.g = c->g;
  A.rho = c->rho;
  A.ds = c->d_static;
  A.t0 = t0;
  Chan& b = A.body;
  b.off = 0;
  b.n = c->n;
  b.kind = c->body.kind;
  b.law = c->body.law;
  b.pad = 0;
  b.amp = c->body.amp;
  b.len = c->body.len;
  b.x0 = c->body.x0;
  b.y0 = c->body.y0;
  b.dir = c->body.dir;
  for (int k = 0; k < 5; k++) b.q[k] = c->body.q[k];
  A.h = h;
  A.hu = hu;
  A.hw = hw;
  A.p = p;
  A.status = status;
  A.adaptive = c->adaptive ? 1 : 0;
  A.crit = c->adaptive ? c->crit : SWE_NH_CRIT_GLOBAL;
  A.enlarge = c->adaptive ? c->enlarge : 0;
  A.first_global = c->adaptive ? c->first_global : 0;
  A.k_nh = c->adaptive ? c->k_nh : 0.0;
  A.marked = c->adaptive ? c->marked : nullptr;
  return A;
}

// threads of the workgroup that runs channels of at most n elements
int dg_threads(int n) {
  return n <= NTD_TINY ? NTD_TINY : (n <= NTD_SMALL ? NTD_SMALL : SWE_NH_DG_MAX_ELEMS);
}

// waits for the stream and maps the status bits
int dg_finish(int32_t* status, hipStream_t s) {
  int bits = 0;
  if (hipMemcpyAsync(&bits, status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SWE_NH_EHIP;
  if (bits & ST_DRY) return SWE_NH_EDRY;  // a dry node also makes the values non-finite
  if (bits & ST_NAN) return SWE_NH_ENAN;
  return SWE_NH_OK;
}
}  // namespace

extern "C" int swe_nh_dg1d_run(const swe_nh_dg1d_config* c, double t0, int32_t nsteps, double* h,
                               double* hu, double* hw, double* p, int32_t* status, void* stream) {
  if (!dg_config_ok(c) || !h || !hu || !hw || !p || !status || nsteps < 0) return SWE_NH_EINVAL;
  if (nsteps == 0) return SWE_NH_OK;
  const DgArgs A = dg_args(c, t0, nsteps, h, hu, hw, p, status);
  hipStream_t s = (hipStream_t)stream;
  const int nt = dg_threads(c->n);
  void (*kern)(DgArgs);
  if (nt == NTD_TINY)
    kern = A.adaptive ? k_dg1d_run<NTD_TINY, true> : k_dg1d_run<NTD_TINY, false>;
  else if (nt == NTD_SMALL)
    kern = A.adaptive ? k_dg1d_run<NTD_SMALL, true> : k_dg1d_run<NTD_SMALL, false>;
  else
    kern = A.adaptive ? k_dg1d_run<SWE_NH_DG_MAX_ELEMS, true>
                      : k_dg1d_run<SWE_NH_DG_MAX_ELEMS, false>;
  if (hipMemsetAsync(status, 0, sizeof(int32_t), s) != hipSuccess) return SWE_NH_EHIP;
  hipLaunchKernelGGL(kern, dim3(1), dim3(nt), 0, s, A);
  if (hipGetLastError() != hipSuccess) return SWE_NH_EHIP;
  return dg_finish(status, s);
}

extern "C" int swe_nh_dg1d_run_batch(const swe_nh_dg1d_config* cfgs, int32_t nch, double t0,
                                     int32_t nsteps, double* h, double* hu, double* hw, double* p,
                                     int32_t* status, void* stream) {
  if (!cfgs || nch < 1 || nch > SWE_NH_DG_MAX_BATCH || !h || !hu || !hw || !p || !status ||
      nsteps < 0)
    return SWE_NH_EINVAL;
  int nmax = 0;
  bool adapt = false;
  for (int c = 0; c < nch; c++) {
    if (!dg_config_ok(&cfgs[c])) return SWE_NH_EINVAL;
    nmax = cfgs[c].n > nmax ? cfgs[c].n : nmax;
    adapt = adapt || cfgs[c].adaptive;
  }
  if (nsteps == 0) return SWE_NH_OK;
  std::vector<DgArgs> host(nch);
  int64_t e0 = 0;  // first element of the channel
  for (int c = 0; c < nch; c++) {
    const int64_t o = 2 * e0;
    host[c] = dg_args(&cfgs[c], t0, nsteps, h + o, hu + o, hw + o, p + o, status);
    e0 += cfgs[c].n;
  }
  hipStream_t s = (hipStream_t)stream;
  DgArgs* dev = nullptr;
  if (hipMalloc((void**)&dev, sizeof(DgArgs) * (size_t)nch) != hipSuccess) return SWE_NH_EHIP;
  int rc = SWE_NH_OK;
  if (hipMemcpyAsync(dev, host.data(), sizeof(DgArgs) * (size_t)nch, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemsetAsync(status, 0, sizeof(int32_t), s) != hipSuccess) {
    rc = SWE_NH_EHIP;
  } else {
    const int nt = dg_threads(nmax);
    void (*kern)(const DgArgs*);
    if (nt == NTD_TINY)
      kern = adapt ? k_dg1d_batch<NTD_TINY, true> : k_dg1d_batch<NTD_TINY, false>;
    else if (nt == NTD_SMALL)
      kern = adapt ? k_dg1d_batch<NTD_SMALL, true> : k_dg1d_batch<NTD_SMALL, false>;
    else
      kern = adapt ? k_dg1d_batch<SWE_NH_DG_MAX_ELEMS, true>
                   : k_dg1d_batch<SWE_NH_DG_MAX_ELEMS, false>;
    hipLaunchKernelGGL(kern, dim3(nch), dim3(nt), 0, s, (const DgArgs*)dev);
    rc = hipGetLastError() != hipSuccess ? SWE_NH_EHIP : dg_finish(status, s);
  }
  // the host copy is pageable: the stream has finished with both buffers
  if (rc == SWE_NH_EHIP) (void)hipStreamSynchronize(s);
  (void)hipFree(dev);
  return rc;
}
