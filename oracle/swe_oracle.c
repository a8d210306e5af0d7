/*
 * swe_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see
 * swe_oracle.h).  Deliberately slow and literal: whole-array passes in the
 * order the method states them, ghost cells materialised explicitly, no
 * blocking, no fusion, no reordering of sums.
 *
 * Paper passages followed (Firdaus & Behrens):
 *   model and quadratic pressure relation ........ Sec. 2, Eqs. 1-5
 *   hydrostatic predictor, Rusanov flux, Heun ..... Sec. 3.1, Eqs. 6-9
 *   backward-Euler correction ..................... Sec. 3.2, Eqs. 10-11
 *   elliptic first-order system, s11+s21=0 ........ Sec. 3.2, Eqs. 12-15
 *   LDG fluxes with the flip-flop constant 1/2 .... Sec. 3.2, Eqs. 16-17
 *   criteria and threshold k_nh ................... Sec. 5.1
 *   global first step for |w|, |w_x| ............. Sec. 5.1.2
 *   one-element enlargement ....................... Sec. 5.2
 *   quartic slide shape, slide kinematics ......... Sec. 4.3, Eqs. 20-21
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - spatial operator: second-order finite volume (MUSCL with minmod limiter
 *     on eta, hu, hw and d) with the hydrostatic reconstruction of Audusse,
 *     Bouchut, Bristeau, Klein and Perthame (2004) and the Rusanov flux;
 *   - elliptic system at polynomial degree zero: with the flip-flop choice
 *     (hu)* = (hu)^- and p* = p^+ the momentum unknown of a cell sits on its
 *     right face, the discrete gradient G is a forward difference with s11
 *     averaged onto the face, and the divergence is -G^T, so that the Schur
 *     complement A = diag(s22) + G^T diag(1/s12) G is symmetric positive
 *     definite because s22 > 0 and s12 > 0;
 *   - derivatives of eta, u, w and d at cells: central differences with
 *     mirrored ghost cells at walls; d_t, d_tt, d_xt: chain rule of the rigid
 *     body translation;
 *   - walls: reflective ghosts for the predictor, zero Dirichlet for p.
 */
#include "swe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI_ 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* forcing: d(x, t) = d_s(x) - B(x - X(t), y - y0)                           */
/* ------------------------------------------------------------------------ */

void orc_body_motion(const orc_body* b, double t, double* X, double* Xd, double* Xdd) {
  double s = 0.0, sd = 0.0, sdd = 0.0;
  if (b->law == ORC_LAW_CONST_VEL) {
    s = b->q[0] * t;
    sd = b->q[0];
  } else if (b->law == ORC_LAW_SIN_RAMP) {
    /* s(t) = (s_f/2)(1 - cos(pi t / T_s)) for t <= T_s, then s_f */
    double sf = b->q[0], Ts = b->q[1];
    if (t <= Ts) {
      s = 0.5 * sf * (1.0 - cos(PI_ * t / Ts));
      sd = 0.5 * sf * (PI_ / Ts) * sin(PI_ * t / Ts);
      sdd = 0.5 * sf * (PI_ / Ts) * (PI_ / Ts) * cos(PI_ * t / Ts);
    } else {
      s = sf;
    }
  } else if (b->law == ORC_LAW_PIECEWISE) {
    /* Eq. 21: accelerate with a0 up to t1, coast at u_t to t2, decelerate to t3 */
    double a0 = b->q[0], ut = b->q[1], t1 = b->q[2], t2 = b->q[3], t3 = b->q[4];
    if (t <= t1) {
      s = 0.5 * a0 * t * t;
      sd = a0 * t;
      sdd = a0;
    } else if (t <= t2) {
      s = 0.5 * a0 * t1 * t1 + ut * (t - t1);
      sd = ut;
    } else if (t <= t3) {
      s = 0.5 * a0 * t1 * t1 + ut * (t - t1) - 0.5 * a0 * (t - t2) * (t - t2);
      sd = ut - a0 * (t - t2);
      sdd = -a0;
    } else {
      s = 0.5 * a0 * t1 * t1 + ut * (t3 - t1) - 0.5 * a0 * (t3 - t2) * (t3 - t2);
    }
  }
  *X = b->x0 + b->dir * s;
  *Xd = b->dir * sd;
  *Xdd = b->dir * sdd;
}

/* shape B and its derivatives with respect to xi = x - X and zeta = y - y0 */
static void body_shape(const orc_body* b, double xi, double zeta, double* B, double* Bx,
                       double* Bxx, double* Bxy) {
  *B = *Bx = *Bxx = *Bxy = 0.0;
  if (b->kind == ORC_BODY_QUARTIC) {
    /* Eq. 20: H_s (1 - (2 xi / L_s)^4) on |xi| < L_s / 2 */
    double L = b->len, H = b->amp;
    if (fabs(xi) < 0.5 * L) {
      double z = 2.0 * xi / L;
      *B = H * (1.0 - z * z * z * z);
      *Bx = -H * 4.0 * z * z * z * (2.0 / L);
      *Bxx = -H * 12.0 * z * z * (2.0 / L) * (2.0 / L);
    }
  } else if (b->kind == ORC_BODY_GAUSS) {
    double w2 = b->len * b->len;
    double e = b->amp * exp(-(xi * xi + zeta * zeta) / w2);
    *B = e;
    *Bx = -2.0 * xi / w2 * e;
    *Bxx = (4.0 * xi * xi / (w2 * w2) - 2.0 / w2) * e;
    *Bxy = 4.0 * xi * zeta / (w2 * w2) * e;
  }
}

void orc_forcing_1d(int32_t n, double dx, const double* ds, const orc_body* b, double t,
                    double* d, double* d_t, double* d_tt, double* d_xt) {
  double X, Xd, Xdd;
  orc_body_motion(b, t, &X, &Xd, &Xdd);
  for (int32_t i = 0; i < n; i++) {
    double x = (i + 0.5) * dx;
    double B, Bx, Bxx, Bxy;
    body_shape(b, x - X, 0.0, &B, &Bx, &Bxx, &Bxy);
    if (d) d[i] = ds[i] - B;
    if (d_t) d_t[i] = Xd * Bx;
    if (d_tt) d_tt[i] = Xdd * Bx - Xd * Xd * Bxx;
    if (d_xt) d_xt[i] = Xd * Bxx;
  }
}

void orc_forcing_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                    const orc_body* b, double t, double* d, double* d_t, double* d_tt,
                    double* d_xt, double* d_yt) {
  double X, Xd, Xdd;
  orc_body_motion(b, t, &X, &Xd, &Xdd);
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      double x = (i + 0.5) * dx, y = (j + 0.5) * dy;
      double B, Bx, Bxx, Bxy;
      body_shape(b, x - X, y - b->y0, &B, &Bx, &Bxx, &Bxy);
      int64_t c = (int64_t)j * nx + i;
      if (d) d[c] = ds[c] - B;
      if (d_t) d_t[c] = Xd * Bx;
      if (d_tt) d_tt[c] = Xdd * Bx - Xd * Xd * Bxx;
      if (d_xt) d_xt[c] = Xd * Bxx;
      if (d_yt) d_yt[c] = Xd * Bxy;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (fabs(a) < fabs(b)) ? a : b;
}

/* reflective ghost: cell index outside [0, n) mirrors into the domain */
static int32_t mirror(int32_t i, int32_t n) {
  if (i < 0) return -1 - i;
  if (i >= n) return 2 * n - 1 - i;
  return i;
}

static double* dalloc(size_t count) { return (double*)calloc(count ? count : 1, sizeof(double)); }

/* Rusanov flux across one face of the hydrostatically reconstructed states
 * (Sec. 3.1: F(Q) = (hu, hu^2 + g h^2 / 2, huw)).  Inputs are the MUSCL face
 * values of eta, normal momentum, tangential momenta and d on the two sides.
 * Outputs: flux of h, normal momentum (without the Audusse correction),
 * tangential momentum(s), and the reconstructed h on both sides. */
typedef struct {
  double Fh, Fm, Ft1, Ft2;
  double hL, hR, hsL, hsR;
} face_flux;

static int rusanov(double g, double etaL, double mL, double t1L, double t2L, double dL,
                   double etaR, double mR, double t1R, double t2R, double dR, face_flux* f) {
  double hL = etaL + dL, hR = etaR + dR;
  if (!(hL > 0.0) || !(hR > 0.0)) return ORC_EDRY;
  double uL = mL / hL, uR = mR / hR;
  double aL = t1L / hL, aR = t1R / hR; /* tangential velocity 1 (w in 1D, v or u in 2D) */
  double bL = t2L / hL, bR = t2R / hR; /* tangential velocity 2 (w in 2D) */
  double df = fmin(dL, dR);
  double hsL = fmax(0.0, etaL + df), hsR = fmax(0.0, etaR + df);
  double lam = fmax(fabs(uL) + sqrt(g * hsL), fabs(uR) + sqrt(g * hsR));
  f->Fh = 0.5 * (hsL * uL + hsR * uR) - 0.5 * lam * (hsR - hsL);
  f->Fm = 0.5 * (hsL * uL * uL + 0.5 * g * hsL * hsL + hsR * uR * uR + 0.5 * g * hsR * hsR) -
          0.5 * lam * (hsR * uR - hsL * uL);
  f->Ft1 = 0.5 * (hsL * uL * aL + hsR * uR * aR) - 0.5 * lam * (hsR * aR - hsL * aL);
  f->Ft2 = 0.5 * (hsL * uL * bL + hsR * uR * bR) - 0.5 * lam * (hsR * bR - hsL * bL);
  f->hL = hL;
  f->hR = hR;
  f->hsL = hsL;
  f->hsR = hsR;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 1D predictor                                                             */
/* ------------------------------------------------------------------------ */

double orc_max_speed_1d(int32_t n, const double* h, const double* m, double g) {
  double s = 0.0;
  for (int32_t i = 0; i < n; i++) {
    double c = fabs(m[i] / h[i]) + sqrt(g * h[i]);
    if (!(c <= 1e300)) return NAN; /* NaN or infinite state */
    if (c > s) s = c;
  }
  return s;
}

/* hydrostatic finite-volume operator L(Q; d) of the 1D SWE without the NH
 * terms (Eqs. 1-3 with p = 0, P_b = 0) */
int orc_operator_1d(int32_t n, double dx, double g, const double* d, const double* h,
                    const double* m, const double* k, double* Lh, double* Lm, double* Lk) {
  int32_t ne = n + 4; /* two ghost cells on each side */
  double *eta = dalloc(ne), *M = dalloc(ne), *K = dalloc(ne), *D = dalloc(ne);
  double *se = dalloc(ne), *sm = dalloc(ne), *sk = dalloc(ne), *sd = dalloc(ne);
  double *Fh = dalloc(n + 1), *FmL = dalloc(n + 1), *FmR = dalloc(n + 1), *Fk = dalloc(n + 1);
  double *hLf = dalloc(n + 1), *hRf = dalloc(n + 1);
  int st = ORC_OK;
  for (int32_t e = 0; e < ne; e++) {
    int32_t i = e - 2, s = mirror(i, n);
    double sign = (i == s) ? 1.0 : -1.0; /* normal momentum is odd at a wall */
    eta[e] = h[s] - d[s];
    M[e] = sign * m[s];
    K[e] = k[s];
    D[e] = d[s];
  }
  for (int32_t e = 1; e < ne - 1; e++) {
    se[e] = minmod(eta[e] - eta[e - 1], eta[e + 1] - eta[e]);
    sm[e] = minmod(M[e] - M[e - 1], M[e + 1] - M[e]);
    sk[e] = minmod(K[e] - K[e - 1], K[e + 1] - K[e]);
    sd[e] = minmod(D[e] - D[e - 1], D[e + 1] - D[e]);
  }
  for (int32_t j = 0; j <= n; j++) { /* face j between cells j-1 and j */
    int32_t l = j + 1, r = j + 2;
    face_flux f;
    st = rusanov(g, eta[l] + 0.5 * se[l], M[l] + 0.5 * sm[l], K[l] + 0.5 * sk[l], 0.0,
                 D[l] + 0.5 * sd[l], eta[r] - 0.5 * se[r], M[r] - 0.5 * sm[r],
                 K[r] - 0.5 * sk[r], 0.0, D[r] - 0.5 * sd[r], &f);
    if (st != ORC_OK) goto done;
    Fh[j] = f.Fh;
    Fk[j] = f.Ft1;
    /* hydrostatic reconstruction: each side sees its own pressure correction */
    FmL[j] = f.Fm + 0.5 * g * (f.hL * f.hL - f.hsL * f.hsL);
    FmR[j] = f.Fm + 0.5 * g * (f.hR * f.hR - f.hsR * f.hsR);
    hLf[j] = f.hL;
    hRf[j] = f.hR;
  }
  for (int32_t i = 0; i < n; i++) {
    int32_t e = i + 2;
    /* centred source g h d_x over the cell: d jumps by the reconstructed slope */
    double src = g * 0.5 * (hLf[i + 1] + hRf[i]) * sd[e] / dx;
    Lh[i] = -(Fh[i + 1] - Fh[i]) / dx;
    Lm[i] = -(FmL[i + 1] - FmR[i]) / dx + src;
    Lk[i] = -(Fk[i + 1] - Fk[i]) / dx;
  }
done:
  free(eta); free(M); free(K); free(D); free(se); free(sm); free(sk); free(sd);
  free(Fh); free(FmL); free(FmR); free(Fk); free(hLf); free(hRf);
  return st;
}

/* Heun (Eqs. 8-9): Q* = Q^n + dt L(Q^n, t^n);
 *                  Q~ = Q^n + dt/2 (L(Q^n, t^n) + L(Q*, t^n + dt)) */
int orc_predict_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                   double t, double dt, const double* h, const double* m, const double* k,
                   double* ht, double* mt, double* kt) {
  double *d0 = dalloc(n), *d1 = dalloc(n);
  double *L1h = dalloc(n), *L1m = dalloc(n), *L1k = dalloc(n);
  double *L2h = dalloc(n), *L2m = dalloc(n), *L2k = dalloc(n);
  double *hs = dalloc(n), *ms = dalloc(n), *ks = dalloc(n);
  int st;
  orc_forcing_1d(n, dx, ds, b, t, d0, NULL, NULL, NULL);
  orc_forcing_1d(n, dx, ds, b, t + dt, d1, NULL, NULL, NULL);
  st = orc_operator_1d(n, dx, ph->g, d0, h, m, k, L1h, L1m, L1k);
  if (st != ORC_OK) goto done;
  for (int32_t i = 0; i < n; i++) {
    hs[i] = h[i] + dt * L1h[i];
    ms[i] = m[i] + dt * L1m[i];
    ks[i] = k[i] + dt * L1k[i];
  }
  st = orc_operator_1d(n, dx, ph->g, d1, hs, ms, ks, L2h, L2m, L2k);
  if (st != ORC_OK) goto done;
  for (int32_t i = 0; i < n; i++) {
    ht[i] = h[i] + 0.5 * dt * (L1h[i] + L2h[i]);
    mt[i] = m[i] + 0.5 * dt * (L1m[i] + L2m[i]);
    kt[i] = k[i] + 0.5 * dt * (L1k[i] + L2k[i]);
  }
done:
  free(d0); free(d1); free(L1h); free(L1m); free(L1k); free(L2h); free(L2m); free(L2k);
  free(hs); free(ms); free(ks);
  return st;
}

/* ------------------------------------------------------------------------ */
/* 1D criterion (Sec. 5.1) and enlargement (Sec. 5.2)                       */
/* ------------------------------------------------------------------------ */

int orc_indicator_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                     double t1, const double* ht, const double* mt, const double* kt, double* ind) {
  double *d = dalloc(n), *eta = dalloc(n), *u = dalloc(n), *w = dalloc(n);
  orc_forcing_1d(n, dx, ds, b, t1, d, NULL, NULL, NULL);
  for (int32_t i = 0; i < n; i++) {
    eta[i] = ht[i] - d[i];
    u[i] = mt[i] / ht[i];
    w[i] = kt[i] / ht[i];
  }
  for (int32_t i = 0; i < n; i++) {
    int32_t il = mirror(i - 1, n), ir = mirror(i + 1, n);
    double su_l = (il == i - 1) ? 1.0 : -1.0, su_r = (ir == i + 1) ? 1.0 : -1.0;
    double v = 0.0;
    switch (ph->crit) {
      case ORC_CRIT_ETA_D: v = fabs(eta[i] / d[i]); break;
      case ORC_CRIT_ETA_X: v = fabs((eta[ir] - eta[il]) / (2.0 * dx)); break;
      case ORC_CRIT_U: v = fabs(u[i]); break;
      case ORC_CRIT_U_X: v = fabs((su_r * u[ir] - su_l * u[il]) / (2.0 * dx)); break;
      case ORC_CRIT_W: v = fabs(w[i]); break;
      case ORC_CRIT_W_X: v = fabs((w[ir] - w[il]) / (2.0 * dx)); break;
      default: v = 0.0;
    }
    ind[i] = v;
  }
  free(d); free(eta); free(u); free(w);
  return ORC_OK;
}

int orc_mask_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                double t1, int32_t first_step, const double* ht, const double* mt, const double* kt,
                uint8_t* mask) {
  int32_t crit = ph->crit, count = 0;
  if (crit < 0 || crit > ORC_CRIT_NONE || ph->enlarge < 0) return ORC_EINVAL;
  int global = (crit == ORC_CRIT_GLOBAL) ||
               ((crit == ORC_CRIT_W || crit == ORC_CRIT_W_X) && first_step && ph->first_global);
  if (global || crit == ORC_CRIT_NONE) {
    for (int32_t i = 0; i < n; i++) mask[i] = (uint8_t)(global ? 1 : 0);
    return global ? n : 0;
  }
  double* ind = dalloc(n);
  uint8_t* raw = (uint8_t*)calloc(n ? n : 1, 1);
  orc_indicator_1d(n, dx, ds, b, ph, t1, ht, mt, kt, ind);
  for (int32_t i = 0; i < n; i++) raw[i] = (uint8_t)(ind[i] > ph->k_nh); /* strict: "exceeds" */
  for (int32_t i = 0; i < n; i++) {
    uint8_t v = 0;
    for (int32_t j = i - ph->enlarge; j <= i + ph->enlarge; j++)
      if (j >= 0 && j < n && raw[j]) v = 1;
    mask[i] = v;
    count += v;
  }
  free(ind); free(raw);
  return count;
}

/* ------------------------------------------------------------------------ */
/* 1D elliptic system (Sec. 3.2)                                            */
/* ------------------------------------------------------------------------ */

/* cell rows: 0 D=d_x, 1 alpha=4+d_x^2, 2 phi, 3 s22, 4 f2, 5 d_t, 6 eta_x, 7 u
 * face rows (face j between cells j-1 and j, j = 0..n):
 *   0 h_f, 1 d_x,f, 2 s11_f, 3 K_f = 1/s12_f, 4 a_f, 5 b_f, 6 q_pred,f,
 *   7 (dt/rho) phi_f d_x,f
 * with the discrete gradient (G p)_f = a_f p_{j-1} + b_f p_j. */
int orc_nh_coeffs_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                     double t1, double dt, const double* ht, const double* mt, const double* kt,
                     double* cell, double* face) {
  const double g = ph->g, rho = ph->rho;
  double *d = dalloc(n), *dtc = dalloc(n), *dtt = dalloc(n), *dxt = dalloc(n);
  double *D = cell, *al = cell + n, *phi = cell + 2 * n, *s22 = cell + 3 * n, *f2 = cell + 4 * n,
         *dtv = cell + 5 * n, *etx = cell + 6 * n, *uu = cell + 7 * n;
  int32_t nf = n + 1;
  orc_forcing_1d(n, dx, ds, b, t1, d, dtc, dtt, dxt);
  for (int32_t i = 0; i < n; i++) {
    if (!(ht[i] > 0.0)) { free(d); free(dtc); free(dtt); free(dxt); return ORC_EDRY; }
  }
  for (int32_t i = 0; i < n; i++) {
    int32_t il = mirror(i - 1, n), ir = mirror(i + 1, n);
    double Dx = (d[ir] - d[il]) / (2.0 * dx);
    double dxx = (d[ir] - 2.0 * d[i] + d[il]) / (dx * dx);
    double ex = ((ht[ir] - d[ir]) - (ht[il] - d[il])) / (2.0 * dx);
    double u = mt[i] / ht[i];
    double a = 4.0 + Dx * Dx;
    /* Eq. 5: phi = rho h / (4 + d_x^2) (g d_x eta_x - d_tt - 2 u d_xt - u^2 d_xx) */
    double ph_ = rho * ht[i] / a * (g * Dx * ex - dtt[i] - 2.0 * u * dxt[i] - u * u * dxx);
    D[i] = Dx;
    al[i] = a;
    phi[i] = ph_;
    s22[i] = 3.0 * dt / (rho * ht[i]);                                  /* Eq. 13 */
    f2[i] = -2.0 * dtc[i] - 2.0 * kt[i] / ht[i] - Dx * mt[i] / (2.0 * ht[i]) -
            dt * a * ph_ / (2.0 * rho * ht[i]);                         /* Eq. 13 */
    dtv[i] = dtc[i];
    etx[i] = ex;
    uu[i] = u;
  }
  for (int32_t j = 0; j < nf; j++) {
    int32_t il = mirror(j - 1, n), ir = mirror(j, n);
    double sl = (il == j - 1) ? 1.0 : -1.0, sr = (ir == j) ? 1.0 : -1.0;
    double hf = 0.5 * (ht[il] + ht[ir]);
    double Df = (d[ir] - d[il]) / dx;
    double hx = (ht[ir] - ht[il]) / dx;
    double phif = 0.5 * (phi[il] + phi[ir]);
    double qf = 0.5 * (sl * mt[il] + sr * mt[ir]);
    double af = 4.0 + Df * Df;
    double s11 = (2.0 * hx - 3.0 * Df) / (2.0 * hf);      /* Eq. 12 */
    double K = 4.0 * dt * hf / (rho * af);                /* 1 / s12, Eq. 12 */
    double fd = dt / rho * phif * Df;
    face[0 * nf + j] = hf;
    face[1 * nf + j] = Df;
    face[2 * nf + j] = s11;
    face[3 * nf + j] = K;
    face[4 * nf + j] = -1.0 / dx + 0.5 * s11;
    face[5 * nf + j] = 1.0 / dx + 0.5 * s11;
    face[6 * nf + j] = qf + fd;                           /* K f1 at the face */
    face[7 * nf + j] = fd;
  }
  free(d); free(dtc); free(dtt); free(dxt);
  return ORC_OK;
}

/* A p = f2 + G^T q_pred on the NH cells, identity rows elsewhere (p = 0) */
int orc_nh_system_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                     double t1, double dt, const double* ht, const double* mt, const double* kt,
                     const uint8_t* mask, double* diag, double* upper, double* rhs) {
  int32_t nf = n + 1;
  double *cell = dalloc(8 * (size_t)n), *face = dalloc(8 * (size_t)nf);
  int st = orc_nh_coeffs_1d(n, dx, ds, b, ph, t1, dt, ht, mt, kt, cell, face);
  if (st == ORC_OK) {
    const double *s22 = cell + 3 * n, *f2 = cell + 4 * n;
    const double *K = face + 3 * nf, *a = face + 4 * nf, *bb = face + 5 * nf, *qp = face + 6 * nf;
    for (int32_t i = 0; i < n; i++) {
      if (!mask[i]) {
        diag[i] = 1.0;
        upper[i] = 0.0;
        rhs[i] = 0.0;
        continue;
      }
      /* cell i is the right cell of face i and the left cell of face i+1 */
      diag[i] = s22[i] + K[i] * bb[i] * bb[i] + K[i + 1] * a[i + 1] * a[i + 1];
      upper[i] = (i + 1 < n && mask[i + 1]) ? K[i + 1] * a[i + 1] * bb[i + 1] : 0.0;
      rhs[i] = f2[i] + bb[i] * qp[i] + a[i + 1] * qp[i + 1];
    }
  }
  free(cell); free(face);
  return st;
}

/* Thomas algorithm for a symmetric tridiagonal matrix (upper[i] couples i, i+1) */
int orc_tridiag_solve(int32_t n, const double* diag, const double* upper, const double* rhs,
                      double* x) {
  if (n <= 0) return ORC_OK;
  double *c = dalloc(n), *y = dalloc(n);
  double den = diag[0];
  if (!(fabs(den) > 0.0)) { free(c); free(y); return ORC_EINVAL; }
  c[0] = upper[0] / den;
  y[0] = rhs[0] / den;
  for (int32_t i = 1; i < n; i++) {
    den = diag[i] - upper[i - 1] * c[i - 1];
    if (!(fabs(den) > 0.0)) { free(c); free(y); return ORC_EINVAL; }
    c[i] = (i + 1 < n) ? upper[i] / den : 0.0;
    y[i] = (rhs[i] - upper[i - 1] * y[i - 1]) / den;
  }
  x[n - 1] = y[n - 1];
  for (int32_t i = n - 2; i >= 0; i--) x[i] = y[i] - c[i] * x[i + 1];
  free(c); free(y);
  return ORC_OK;
}

/* Eqs. 10-11 on the NH cells: the face momenta m_f = q_pred,f - K_f (G p)_f,
 * hu = m~ + mean of the two face increments, and
 * P_b = 3p/2 - rho d_x (hu - m~) / (4 dt) + (4 + d_x^2) phi / 4 (Eq. 5 with
 * (h p)_x eliminated through Eq. 10), hw = k~ + dt P_b / rho. */
int orc_nh_correct_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                      double t1, double dt, const double* ht, const double* mt, const double* kt,
                      const uint8_t* mask, const double* p, double* m_out, double* k_out) {
  int32_t nf = n + 1;
  double rho = ph->rho;
  double *cell = dalloc(8 * (size_t)n), *face = dalloc(8 * (size_t)nf), *dq = dalloc(nf);
  int st = orc_nh_coeffs_1d(n, dx, ds, b, ph, t1, dt, ht, mt, kt, cell, face);
  if (st == ORC_OK) {
    const double *D = cell, *al = cell + n, *phi = cell + 2 * n;
    const double *K = face + 3 * nf, *a = face + 4 * nf, *bb = face + 5 * nf, *fd = face + 7 * nf;
    for (int32_t j = 0; j < nf; j++) {
      double pl = (j - 1 >= 0 && mask[j - 1]) ? p[j - 1] : 0.0;
      double pr = (j < n && mask[j]) ? p[j] : 0.0;
      dq[j] = fd[j] - K[j] * (a[j] * pl + bb[j] * pr);
    }
    for (int32_t i = 0; i < n; i++) {
      if (!mask[i]) {
        m_out[i] = mt[i];
        k_out[i] = kt[i];
        continue;
      }
      double dm = 0.5 * (dq[i] + dq[i + 1]);
      double Pb = 1.5 * p[i] - rho * D[i] * dm / (4.0 * dt) + al[i] * phi[i] / 4.0;
      m_out[i] = mt[i] + dm;
      k_out[i] = kt[i] + dt * Pb / rho;
    }
  }
  free(cell); free(face); free(dq);
  return st;
}

int orc_step_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                double cfl, double dt_fixed, int32_t step_index, double* t, double* h, double* m,
                double* k, double* p, uint8_t* mask, double* dt_used, int32_t* n_active) {
  if (n < 3 || !(dx > 0.0)) return ORC_EINVAL;
  /* state check: non-finite values first, then dry cells */
  int bad_nan = 0, bad_dry = 0;
  for (int32_t i = 0; i < n; i++) {
    if (!isfinite(h[i]) || !isfinite(m[i]) || !isfinite(k[i])) bad_nan = 1;
    else if (!(h[i] > 0.0)) bad_dry = 1;
  }
  if (bad_nan) return ORC_ENAN;
  if (bad_dry) return ORC_EDRY;
  double smax = orc_max_speed_1d(n, h, m, ph->g);
  if (!(smax <= 1e300)) return ORC_ENAN;
  double dt = (cfl > 0.0) ? cfl * dx / smax : dt_fixed;
  if (!(dt > 0.0)) return ORC_EINVAL;
  double *ht = dalloc(n), *mt = dalloc(n), *kt = dalloc(n);
  double *dg = dalloc(n), *up = dalloc(n), *rh = dalloc(n);
  int st = orc_predict_1d(n, dx, ds, b, ph, *t, dt, h, m, k, ht, mt, kt);
  int32_t na = 0;
  if (st != ORC_OK) goto done;
  na = orc_mask_1d(n, dx, ds, b, ph, *t + dt, step_index == 0, ht, mt, kt, mask);
  if (na < 0) { st = na; goto done; }
  if (na > 0) {
    st = orc_nh_system_1d(n, dx, ds, b, ph, *t + dt, dt, ht, mt, kt, mask, dg, up, rh);
    if (st != ORC_OK) goto done;
    st = orc_tridiag_solve(n, dg, up, rh, p);
    if (st != ORC_OK) goto done;
    st = orc_nh_correct_1d(n, dx, ds, b, ph, *t + dt, dt, ht, mt, kt, mask, p, m, k);
    if (st != ORC_OK) goto done;
  } else {
    for (int32_t i = 0; i < n; i++) { p[i] = 0.0; m[i] = mt[i]; k[i] = kt[i]; }
  }
  for (int32_t i = 0; i < n; i++) h[i] = ht[i]; /* no correction of the mass, Sec. 3.2 */
  *t += dt;
done:
  if (dt_used) *dt_used = dt;
  if (n_active) *n_active = na;
  free(ht); free(mt); free(kt); free(dg); free(up); free(rh);
  return st;
}

/* ------------------------------------------------------------------------ */
/* 2D (the paper's stated future work; read from the vector form of Eqs.    */
/* 1-5: see the design notes)                                                */
/* ------------------------------------------------------------------------ */

#define IDX(j, i) ((int64_t)(j) * nx + (i))

double orc_max_rate_2d(int32_t nx, int32_t ny, double dx, double dy, const double* h,
                       const double* m, const double* n_, double g) {
  double s = 0.0;
  for (int64_t c = 0; c < (int64_t)nx * ny; c++) {
    double a = sqrt(g * h[c]);
    double r = (fabs(m[c] / h[c]) + a) / dx + (fabs(n_[c] / h[c]) + a) / dy;
    if (!(r <= 1e300)) return NAN;
    if (r > s) s = r;
  }
  return s;
}

/* unsplit 2D hydrostatic operator: x-sweep and y-sweep of the 1D face
 * treatment, each with its own reconstruction along its direction */
int orc_operator_2d(int32_t nx, int32_t ny, double dx, double dy, double g, const double* d,
                    const double* h, const double* m, const double* n_, const double* k,
                    double* Lh, double* Lm, double* Ln, double* Lk) {
  int st = ORC_OK;
  int64_t N = (int64_t)nx * ny;
  for (int64_t c = 0; c < N; c++) Lh[c] = Lm[c] = Ln[c] = Lk[c] = 0.0;
  /* x direction, one row at a time */
  {
    int32_t ne = nx + 4;
    double *eta = dalloc(ne), *M = dalloc(ne), *T1 = dalloc(ne), *T2 = dalloc(ne), *D = dalloc(ne);
    double *se = dalloc(ne), *sm = dalloc(ne), *s1 = dalloc(ne), *s2 = dalloc(ne), *sd = dalloc(ne);
    double *Fh = dalloc(nx + 1), *FmL = dalloc(nx + 1), *FmR = dalloc(nx + 1), *F1 = dalloc(nx + 1),
           *F2 = dalloc(nx + 1), *hLf = dalloc(nx + 1), *hRf = dalloc(nx + 1);
    for (int32_t j = 0; j < ny && st == ORC_OK; j++) {
      for (int32_t e = 0; e < ne; e++) {
        int32_t i = e - 2, s = mirror(i, nx);
        double sign = (i == s) ? 1.0 : -1.0;
        eta[e] = h[IDX(j, s)] - d[IDX(j, s)];
        M[e] = sign * m[IDX(j, s)];
        T1[e] = n_[IDX(j, s)];
        T2[e] = k[IDX(j, s)];
        D[e] = d[IDX(j, s)];
      }
      for (int32_t e = 1; e < ne - 1; e++) {
        se[e] = minmod(eta[e] - eta[e - 1], eta[e + 1] - eta[e]);
        sm[e] = minmod(M[e] - M[e - 1], M[e + 1] - M[e]);
        s1[e] = minmod(T1[e] - T1[e - 1], T1[e + 1] - T1[e]);
        s2[e] = minmod(T2[e] - T2[e - 1], T2[e + 1] - T2[e]);
        sd[e] = minmod(D[e] - D[e - 1], D[e + 1] - D[e]);
      }
      for (int32_t f = 0; f <= nx; f++) {
        int32_t l = f + 1, r = f + 2;
        face_flux ff;
        st = rusanov(g, eta[l] + 0.5 * se[l], M[l] + 0.5 * sm[l], T1[l] + 0.5 * s1[l],
                     T2[l] + 0.5 * s2[l], D[l] + 0.5 * sd[l], eta[r] - 0.5 * se[r],
                     M[r] - 0.5 * sm[r], T1[r] - 0.5 * s1[r], T2[r] - 0.5 * s2[r],
                     D[r] - 0.5 * sd[r], &ff);
        if (st != ORC_OK) break;
        Fh[f] = ff.Fh;
        F1[f] = ff.Ft1;
        F2[f] = ff.Ft2;
        FmL[f] = ff.Fm + 0.5 * g * (ff.hL * ff.hL - ff.hsL * ff.hsL);
        FmR[f] = ff.Fm + 0.5 * g * (ff.hR * ff.hR - ff.hsR * ff.hsR);
        hLf[f] = ff.hL;
        hRf[f] = ff.hR;
      }
      if (st != ORC_OK) break;
      for (int32_t i = 0; i < nx; i++) {
        int64_t c = IDX(j, i);
        double src = g * 0.5 * (hLf[i + 1] + hRf[i]) * sd[i + 2] / dx;
        Lh[c] += -(Fh[i + 1] - Fh[i]) / dx;
        Lm[c] += -(FmL[i + 1] - FmR[i]) / dx + src;
        Ln[c] += -(F1[i + 1] - F1[i]) / dx;
        Lk[c] += -(F2[i + 1] - F2[i]) / dx;
      }
    }
    free(eta); free(M); free(T1); free(T2); free(D); free(se); free(sm); free(s1); free(s2);
    free(sd); free(Fh); free(FmL); free(FmR); free(F1); free(F2); free(hLf); free(hRf);
  }
  if (st != ORC_OK) return st;
  /* y direction, one column at a time; normal momentum is hv */
  {
    int32_t ne = ny + 4;
    double *eta = dalloc(ne), *M = dalloc(ne), *T1 = dalloc(ne), *T2 = dalloc(ne), *D = dalloc(ne);
    double *se = dalloc(ne), *sm = dalloc(ne), *s1 = dalloc(ne), *s2 = dalloc(ne), *sd = dalloc(ne);
    double *Fh = dalloc(ny + 1), *FmL = dalloc(ny + 1), *FmR = dalloc(ny + 1), *F1 = dalloc(ny + 1),
           *F2 = dalloc(ny + 1), *hLf = dalloc(ny + 1), *hRf = dalloc(ny + 1);
    for (int32_t i = 0; i < nx && st == ORC_OK; i++) {
      for (int32_t e = 0; e < ne; e++) {
        int32_t j = e - 2, s = mirror(j, ny);
        double sign = (j == s) ? 1.0 : -1.0;
        eta[e] = h[IDX(s, i)] - d[IDX(s, i)];
        M[e] = sign * n_[IDX(s, i)];
        T1[e] = m[IDX(s, i)];
        T2[e] = k[IDX(s, i)];
        D[e] = d[IDX(s, i)];
      }
      for (int32_t e = 1; e < ne - 1; e++) {
        se[e] = minmod(eta[e] - eta[e - 1], eta[e + 1] - eta[e]);
        sm[e] = minmod(M[e] - M[e - 1], M[e + 1] - M[e]);
        s1[e] = minmod(T1[e] - T1[e - 1], T1[e + 1] - T1[e]);
        s2[e] = minmod(T2[e] - T2[e - 1], T2[e + 1] - T2[e]);
        sd[e] = minmod(D[e] - D[e - 1], D[e + 1] - D[e]);
      }
      for (int32_t f = 0; f <= ny; f++) {
        int32_t l = f + 1, r = f + 2;
        face_flux ff;
        st = rusanov(g, eta[l] + 0.5 * se[l], M[l] + 0.5 * sm[l], T1[l] + 0.5 * s1[l],
                     T2[l] + 0.5 * s2[l], D[l] + 0.5 * sd[l], eta[r] - 0.5 * se[r],
                     M[r] - 0.5 * sm[r], T1[r] - 0.5 * s1[r], T2[r] - 0.5 * s2[r],
                     D[r] - 0.5 * sd[r], &ff);
        if (st != ORC_OK) break;
        Fh[f] = ff.Fh;
        F1[f] = ff.Ft1;
        F2[f] = ff.Ft2;
        FmL[f] = ff.Fm + 0.5 * g * (ff.hL * ff.hL - ff.hsL * ff.hsL);
        FmR[f] = ff.Fm + 0.5 * g * (ff.hR * ff.hR - ff.hsR * ff.hsR);
        hLf[f] = ff.hL;
        hRf[f] = ff.hR;
      }
      if (st != ORC_OK) break;
      for (int32_t j = 0; j < ny; j++) {
        int64_t c = IDX(j, i);
        double src = g * 0.5 * (hLf[j + 1] + hRf[j]) * sd[j + 2] / dy;
        Lh[c] += -(Fh[j + 1] - Fh[j]) / dy;
        Ln[c] += -(FmL[j + 1] - FmR[j]) / dy + src;
        Lm[c] += -(F1[j + 1] - F1[j]) / dy;
        Lk[c] += -(F2[j + 1] - F2[j]) / dy;
      }
    }
    free(eta); free(M); free(T1); free(T2); free(D); free(se); free(sm); free(s1); free(s2);
    free(sd); free(Fh); free(FmL); free(FmR); free(F1); free(F2); free(hLf); free(hRf);
  }
  return st;
}

int orc_predict_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                   const orc_body* b, const orc_phys* ph, double t, double dt, const double* h,
                   const double* m, const double* n_, const double* k, double* ht, double* mt,
                   double* nt, double* kt) {
  int64_t N = (int64_t)nx * ny;
  double *d0 = dalloc(N), *d1 = dalloc(N);
  double *L1[4], *L2[4], *S[4];
  for (int q = 0; q < 4; q++) { L1[q] = dalloc(N); L2[q] = dalloc(N); S[q] = dalloc(N); }
  int st;
  orc_forcing_2d(nx, ny, dx, dy, ds, b, t, d0, NULL, NULL, NULL, NULL);
  orc_forcing_2d(nx, ny, dx, dy, ds, b, t + dt, d1, NULL, NULL, NULL, NULL);
  st = orc_operator_2d(nx, ny, dx, dy, ph->g, d0, h, m, n_, k, L1[0], L1[1], L1[2], L1[3]);
  if (st == ORC_OK) {
    for (int64_t c = 0; c < N; c++) {
      S[0][c] = h[c] + dt * L1[0][c];
      S[1][c] = m[c] + dt * L1[1][c];
      S[2][c] = n_[c] + dt * L1[2][c];
      S[3][c] = k[c] + dt * L1[3][c];
    }
    st = orc_operator_2d(nx, ny, dx, dy, ph->g, d1, S[0], S[1], S[2], S[3], L2[0], L2[1], L2[2],
                         L2[3]);
  }
  if (st == ORC_OK) {
    for (int64_t c = 0; c < N; c++) {
      ht[c] = h[c] + 0.5 * dt * (L1[0][c] + L2[0][c]);
      mt[c] = m[c] + 0.5 * dt * (L1[1][c] + L2[1][c]);
      nt[c] = n_[c] + 0.5 * dt * (L1[2][c] + L2[2][c]);
      kt[c] = k[c] + 0.5 * dt * (L1[3][c] + L2[3][c]);
    }
  }
  for (int q = 0; q < 4; q++) { free(L1[q]); free(L2[q]); free(S[q]); }
  free(d0); free(d1);
  return st;
}

/* 2D indicators: magnitudes of the vector quantities (|grad eta|, |(u,v)|,
 * Frobenius norm of grad(u,v), |grad w|), central differences, mirrored ghosts */
int orc_indicator_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                     const orc_body* b, const orc_phys* ph, double t1, const double* ht,
                     const double* mt, const double* nt, const double* kt, double* ind) {
  int64_t N = (int64_t)nx * ny;
  double *d = dalloc(N), *eta = dalloc(N), *u = dalloc(N), *v = dalloc(N), *w = dalloc(N);
  orc_forcing_2d(nx, ny, dx, dy, ds, b, t1, d, NULL, NULL, NULL, NULL);
  for (int64_t c = 0; c < N; c++) {
    eta[c] = ht[c] - d[c];
    u[c] = mt[c] / ht[c];
    v[c] = nt[c] / ht[c];
    w[c] = kt[c] / ht[c];
  }
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      int32_t il = mirror(i - 1, nx), ir = mirror(i + 1, nx);
      int32_t jl = mirror(j - 1, ny), jr = mirror(j + 1, ny);
      double sxl = (il == i - 1) ? 1.0 : -1.0, sxr = (ir == i + 1) ? 1.0 : -1.0;
      double syl = (jl == j - 1) ? 1.0 : -1.0, syr = (jr == j + 1) ? 1.0 : -1.0;
      int64_t c = IDX(j, i);
      double val = 0.0;
      switch (ph->crit) {
        case ORC_CRIT_ETA_D: val = fabs(eta[c] / d[c]); break;
        case ORC_CRIT_ETA_X: {
          double ex = (eta[IDX(j, ir)] - eta[IDX(j, il)]) / (2.0 * dx);
          double ey = (eta[IDX(jr, i)] - eta[IDX(jl, i)]) / (2.0 * dy);
          val = sqrt(ex * ex + ey * ey);
        } break;
        case ORC_CRIT_U: val = sqrt(u[c] * u[c] + v[c] * v[c]); break;
        case ORC_CRIT_U_X: {
          /* u is odd across x-walls, v across y-walls */
          double ux = (sxr * u[IDX(j, ir)] - sxl * u[IDX(j, il)]) / (2.0 * dx);
          double uy = (u[IDX(jr, i)] - u[IDX(jl, i)]) / (2.0 * dy);
          double vx = (v[IDX(j, ir)] - v[IDX(j, il)]) / (2.0 * dx);
          double vy = (syr * v[IDX(jr, i)] - syl * v[IDX(jl, i)]) / (2.0 * dy);
          val = sqrt(ux * ux + uy * uy + vx * vx + vy * vy);
        } break;
        case ORC_CRIT_W: val = fabs(w[c]); break;
        case ORC_CRIT_W_X: {
          double wx = (w[IDX(j, ir)] - w[IDX(j, il)]) / (2.0 * dx);
          double wy = (w[IDX(jr, i)] - w[IDX(jl, i)]) / (2.0 * dy);
          val = sqrt(wx * wx + wy * wy);
        } break;
        default: val = 0.0;
      }
      ind[c] = val;
    }
  }
  free(d); free(eta); free(u); free(v); free(w);
  return ORC_OK;
}

int orc_mask_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds, const orc_body* b,
                const orc_phys* ph, double t1, int32_t first_step, const double* ht,
                const double* mt, const double* nt, const double* kt, uint8_t* mask) {
  int64_t N = (int64_t)nx * ny;
  int32_t crit = ph->crit, e = ph->enlarge;
  if (crit < 0 || crit > ORC_CRIT_NONE || e < 0) return ORC_EINVAL;
  int global = (crit == ORC_CRIT_GLOBAL) ||
               ((crit == ORC_CRIT_W || crit == ORC_CRIT_W_X) && first_step && ph->first_global);
  if (global || crit == ORC_CRIT_NONE) {
    for (int64_t c = 0; c < N; c++) mask[c] = (uint8_t)(global ? 1 : 0);
    return global ? (int32_t)N : 0;
  }
  double* ind = dalloc(N);
  uint8_t* raw = (uint8_t*)calloc(N ? N : 1, 1);
  orc_indicator_2d(nx, ny, dx, dy, ds, b, ph, t1, ht, mt, nt, kt, ind);
  for (int64_t c = 0; c < N; c++) raw[c] = (uint8_t)(ind[c] > ph->k_nh);
  int32_t count = 0;
  /* enlargement by e cells in both directions: a (2e+1) x (2e+1) box */
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      uint8_t val = 0;
      for (int32_t jj = j - e; jj <= j + e; jj++)
        for (int32_t ii = i - e; ii <= i + e; ii++)
          if (jj >= 0 && jj < ny && ii >= 0 && ii < nx && raw[IDX(jj, ii)]) val = 1;
      mask[IDX(j, i)] = val;
      count += val;
    }
  }
  free(ind); free(raw);
  return count;
}

/* cell rows: 0 d_x, 1 d_y, 2 alpha = 4 + |grad d|^2, 3 phi, 4 s22, 5 f2, 6 d_t
 * x-face (j, f), f = 0..nx between cells (j, f-1) and (j, f); y-face (f, i)
 * between (f-1, i) and (f, i).  Face rows: 0 K, 1 a, 2 b, 3 q_pred, 4 (dt/rho) phi_f d_n,f
 * K on an x-face is the xx entry of S12^{-1} = (dt h / rho)(I - grad d grad d^T / alpha);
 * the off-diagonal d_x d_y / alpha coupling of the tensor is dropped here and
 * added pair by pair by orc_nh_pairs_2d for the exact-tensor operator. */
int orc_nh_coeffs_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                     const orc_body* b, const orc_phys* ph, double t1, double dt, const double* ht,
                     const double* mt, const double* nt, const double* kt, double* cell,
                     double* xface, double* yface) {
  const double g = ph->g, rho = ph->rho;
  int64_t N = (int64_t)nx * ny, NX = (int64_t)ny * (nx + 1), NY = (int64_t)(ny + 1) * nx;
  double *d = dalloc(N), *dtc = dalloc(N), *dtt = dalloc(N), *dxt = dalloc(N), *dyt = dalloc(N);
  orc_forcing_2d(nx, ny, dx, dy, ds, b, t1, d, dtc, dtt, dxt, dyt);
  for (int64_t c = 0; c < N; c++) {
    if (!(ht[c] > 0.0)) { free(d); free(dtc); free(dtt); free(dxt); free(dyt); return ORC_EDRY; }
  }
  double *Dx = cell, *Dy = cell + N, *al = cell + 2 * N, *phi = cell + 3 * N, *s22 = cell + 4 * N,
         *f2 = cell + 5 * N, *dtv = cell + 6 * N;
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      int32_t il = mirror(i - 1, nx), ir = mirror(i + 1, nx);
      int32_t jl = mirror(j - 1, ny), jr = mirror(j + 1, ny);
      int64_t c = IDX(j, i);
      double ddx = (d[IDX(j, ir)] - d[IDX(j, il)]) / (2.0 * dx);
      double ddy = (d[IDX(jr, i)] - d[IDX(jl, i)]) / (2.0 * dy);
      double dxx = (d[IDX(j, ir)] - 2.0 * d[c] + d[IDX(j, il)]) / (dx * dx);
      double dyy = (d[IDX(jr, i)] - 2.0 * d[c] + d[IDX(jl, i)]) / (dy * dy);
      double dxy = (d[IDX(jr, ir)] - d[IDX(jl, ir)] - d[IDX(jr, il)] + d[IDX(jl, il)]) /
                   (4.0 * dx * dy);
      double ex = ((ht[IDX(j, ir)] - d[IDX(j, ir)]) - (ht[IDX(j, il)] - d[IDX(j, il)])) / (2.0 * dx);
      double ey = ((ht[IDX(jr, i)] - d[IDX(jr, i)]) - (ht[IDX(jl, i)] - d[IDX(jl, i)])) / (2.0 * dy);
      double u = mt[c] / ht[c], v = nt[c] / ht[c];
      double a = 4.0 + ddx * ddx + ddy * ddy;
      double ph_ = rho * ht[c] / a *
                   (g * (ddx * ex + ddy * ey) - dtt[c] - 2.0 * (u * dxt[c] + v * dyt[c]) -
                    (u * u * dxx + 2.0 * u * v * dxy + v * v * dyy));
      Dx[c] = ddx;
      Dy[c] = ddy;
      al[c] = a;
      phi[c] = ph_;
      s22[c] = 3.0 * dt / (rho * ht[c]);
      f2[c] = -2.0 * dtc[c] - 2.0 * kt[c] / ht[c] - (ddx * mt[c] + ddy * nt[c]) / (2.0 * ht[c]) -
              dt * a * ph_ / (2.0 * rho * ht[c]);
      dtv[c] = dtc[c];
    }
  }
  /* x-faces */
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t f = 0; f <= nx; f++) {
      int32_t il = mirror(f - 1, nx), ir = mirror(f, nx);
      double sl = (il == f - 1) ? 1.0 : -1.0, sr = (ir == f) ? 1.0 : -1.0;
      int64_t cl = IDX(j, il), cr = IDX(j, ir), o = (int64_t)j * (nx + 1) + f;
      double hf = 0.5 * (ht[cl] + ht[cr]);
      double Dn = (d[cr] - d[cl]) / dx;
      double Dt = 0.5 * (Dy[cl] + Dy[cr]);
      double hn = (ht[cr] - ht[cl]) / dx;
      double phif = 0.5 * (phi[cl] + phi[cr]);
      double qf = 0.5 * (sl * mt[cl] + sr * mt[cr]);
      double af = 4.0 + Dn * Dn + Dt * Dt;
      double s11 = (2.0 * hn - 3.0 * Dn) / (2.0 * hf);
      double K = dt * hf / rho * (1.0 - Dn * Dn / af);
      double fd = dt / rho * phif * Dn;
      xface[0 * NX + o] = K;
      xface[1 * NX + o] = -1.0 / dx + 0.5 * s11;
      xface[2 * NX + o] = 1.0 / dx + 0.5 * s11;
      xface[3 * NX + o] = qf + fd;
      xface[4 * NX + o] = fd;
    }
  }
  /* y-faces */
  for (int32_t f = 0; f <= ny; f++) {
    for (int32_t i = 0; i < nx; i++) {
      int32_t jl = mirror(f - 1, ny), jr = mirror(f, ny);
      double sl = (jl == f - 1) ? 1.0 : -1.0, sr = (jr == f) ? 1.0 : -1.0;
      int64_t cl = IDX(jl, i), cr = IDX(jr, i), o = (int64_t)f * nx + i;
      double hf = 0.5 * (ht[cl] + ht[cr]);
      double Dn = (d[cr] - d[cl]) / dy;
      double Dt = 0.5 * (Dx[cl] + Dx[cr]);
      double hn = (ht[cr] - ht[cl]) / dy;
      double phif = 0.5 * (phi[cl] + phi[cr]);
      double qf = 0.5 * (sl * nt[cl] + sr * nt[cr]);
      double af = 4.0 + Dn * Dn + Dt * Dt;
      double s11 = (2.0 * hn - 3.0 * Dn) / (2.0 * hf);
      double K = dt * hf / rho * (1.0 - Dn * Dn / af);
      double fd = dt / rho * phif * Dn;
      yface[0 * NY + o] = K;
      yface[1 * NY + o] = -1.0 / dy + 0.5 * s11;
      yface[2 * NY + o] = 1.0 / dy + 0.5 * s11;
      yface[3 * NY + o] = qf + fd;
      yface[4 * NY + o] = fd;
    }
  }
  free(d); free(dtc); free(dtt); free(dxt); free(dyt);
  return ORC_OK;
}

/* The exact-tensor operator (a reading of the 2D extension, which the paper
 * leaves to future work): the flux correction at the faces is the tensor
 * S12^{-1} = (dt h / rho)(I - grad d grad d^T / alpha) applied to the face
 * gradients (G p)_f.  Its diagonal is the face coefficient K of
 * orc_nh_coeffs_2d.  Its off-diagonal couples an x-face with a y-face, so the
 * faces are paired: cell o owns the x-face east of it and the y-face north of
 * it, and the pair's 2 x 2 block is [[K_e, k], [k, K_n]] with
 *   k = -sqrt(K_e K_n) S_x S_y / sqrt((4 + S_x^2)(4 + S_y^2)),
 * S_x, S_y the normal bottom slopes of the two faces.  Where the face values
 * agree (a planar bottom under uniform h) the block is the tensor exactly:
 * K_e = c (4 + S_y^2) / alpha, K_n = c (4 + S_x^2) / alpha, k = -c S_x S_y / alpha
 * with c = dt h / rho.  |k| < sqrt(K_e K_n) always, so every block and the
 * operator stay symmetric positive definite.  Wall faces have a zero normal
 * slope (mirrored depth), so pairs with a wall face have k = 0. */
int orc_nh_pairs_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                    const orc_body* b, double t1, const double* xface, const double* yface,
                    double* kxy) {
  int64_t N = (int64_t)nx * ny;
  double *d = dalloc(N), *w1 = dalloc(N), *w2 = dalloc(N), *w3 = dalloc(N), *w4 = dalloc(N);
  orc_forcing_2d(nx, ny, dx, dy, ds, b, t1, d, w1, w2, w3, w4);
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      int64_t c = IDX(j, i);
      double Sx = (d[IDX(j, mirror(i + 1, nx))] - d[c]) / dx;
      double Sy = (d[IDX(mirror(j + 1, ny), i)] - d[c]) / dy;
      double Ke = xface[(int64_t)j * (nx + 1) + i + 1];
      double Kn = yface[(int64_t)(j + 1) * nx + i];
      kxy[c] = -sqrt(Ke * Kn) * Sx * Sy / sqrt((4.0 + Sx * Sx) * (4.0 + Sy * Sy));
    }
  }
  free(d); free(w1); free(w2); free(w3); free(w4);
  return ORC_OK;
}

/* p at (j, i), read as 0 off the grid and off the mask */
static double p_at(int32_t nx, int32_t ny, const uint8_t* mask, const double* p, int32_t j,
                   int32_t i) {
  if (i < 0 || i >= nx || j < 0 || j >= ny || !mask[IDX(j, i)]) return 0.0;
  return p[IDX(j, i)];
}

/* (G p) on the x-face east of cell (j, i) and on the y-face north of it */
static double grad_east(int32_t nx, int32_t ny, const double* xface, const uint8_t* mask,
                        const double* p, int32_t j, int32_t i) {
  int64_t NX = (int64_t)ny * (nx + 1), f = (int64_t)j * (nx + 1) + i + 1;
  return xface[NX + f] * p_at(nx, ny, mask, p, j, i) +
         xface[2 * NX + f] * p_at(nx, ny, mask, p, j, i + 1);
}
static double grad_north(int32_t nx, int32_t ny, const double* yface, const uint8_t* mask,
                         const double* p, int32_t j, int32_t i) {
  int64_t NY = (int64_t)(ny + 1) * nx, f = (int64_t)(j + 1) * nx + i;
  return yface[NY + f] * p_at(nx, ny, mask, p, j, i) +
         yface[2 * NY + f] * p_at(nx, ny, mask, p, j + 1, i);
}

/* (A p)_c = s22_c p_c + sum over the four faces of G_{f,c} (flux correction)_f
 * on NH cells (p read as 0 off the mask); identity on the other cells.  The
 * flux correction at a face is K_f (G p)_f, plus with the tensor k of the
 * face's pair times (G p) on the pair's other face. */
int orc_nh_apply7_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                     const double* yface, const double* kxy, const uint8_t* mask,
                     const double* p, double* Ap) {
  int64_t N = (int64_t)nx * ny, NX = (int64_t)ny * (nx + 1), NY = (int64_t)(ny + 1) * nx;
  const double* s22 = cell + 4 * N;
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      int64_t c = IDX(j, i);
      if (!mask[c]) { Ap[c] = p[c]; continue; }
      double pc = p[c];
      double pw = p_at(nx, ny, mask, p, j, i - 1), pe = p_at(nx, ny, mask, p, j, i + 1);
      double ps = p_at(nx, ny, mask, p, j - 1, i), pn = p_at(nx, ny, mask, p, j + 1, i);
      int64_t fw = (int64_t)j * (nx + 1) + i, fe = fw + 1;
      int64_t fs = (int64_t)j * nx + i, fn = fs + nx;
      /* flux corrections of the four faces, diagonal part */
      double qw = xface[fw] * (xface[NX + fw] * pw + xface[2 * NX + fw] * pc);
      double qe = xface[fe] * (xface[NX + fe] * pc + xface[2 * NX + fe] * pe);
      double qs = yface[fs] * (yface[NY + fs] * ps + yface[2 * NY + fs] * pc);
      double qn = yface[fn] * (yface[NY + fn] * pc + yface[2 * NY + fn] * pn);
      if (kxy) {
        /* east and north faces: the pair of this cell; west face: the pair of
         * the cell to the west (its x-face); south face: the pair of the cell
         * to the south (its y-face) */
        qe += kxy[c] * grad_north(nx, ny, yface, mask, p, j, i);
        qn += kxy[c] * grad_east(nx, ny, xface, mask, p, j, i);
        if (i > 0) qw += kxy[c - 1] * grad_north(nx, ny, yface, mask, p, j, i - 1);
        if (j > 0) qs += kxy[c - nx] * grad_east(nx, ny, xface, mask, p, j - 1, i);
      }
      /* west face: c is its right cell (coefficient b); east face: left cell (a) */
      Ap[c] = s22[c] * pc + xface[2 * NX + fw] * qw + xface[NX + fe] * qe +
              yface[2 * NY + fs] * qs + yface[NY + fn] * qn;
    }
  }
  return ORC_OK;
}

int orc_nh_apply_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                    const double* yface, const uint8_t* mask, const double* p, double* Ap) {
  return orc_nh_apply7_2d(nx, ny, cell, xface, yface, NULL, mask, p, Ap);
}

int orc_nh_rhs_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                  const double* yface, const uint8_t* mask, double* rhs) {
  int64_t N = (int64_t)nx * ny, NX = (int64_t)ny * (nx + 1), NY = (int64_t)(ny + 1) * nx;
  const double* f2 = cell + 5 * N;
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      int64_t c = IDX(j, i);
      if (!mask[c]) { rhs[c] = 0.0; continue; }
      int64_t fw = (int64_t)j * (nx + 1) + i, fe = fw + 1;
      int64_t fs = (int64_t)j * nx + i, fn = fs + nx;
      rhs[c] = f2[c] + xface[2 * NX + fw] * xface[3 * NX + fw] +
               xface[NX + fe] * xface[3 * NX + fe] + yface[2 * NY + fs] * yface[3 * NY + fs] +
               yface[NY + fn] * yface[3 * NY + fn];
    }
  }
  return ORC_OK;
}

static double dot_masked(int64_t N, const uint8_t* mask, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t c = 0; c < N; c++)
    if (mask[c]) s += a[c] * b[c];
  return s;
}

/* plain conjugate gradients on the NH cells, starting from x (warm start);
 * stops when ||rhs - A x|| <= tol ||rhs|| */
int orc_cg7_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
               const double* yface, const double* kxy, const uint8_t* mask, const double* rhs,
               double tol, int32_t max_iter, double* x, int32_t* iters, double* rel_res) {
  int64_t N = (int64_t)nx * ny;
  double *r = dalloc(N), *pp = dalloc(N), *q = dalloc(N);
  for (int64_t c = 0; c < N; c++)
    if (!mask[c]) x[c] = 0.0;
  orc_nh_apply7_2d(nx, ny, cell, xface, yface, kxy, mask, x, q);
  for (int64_t c = 0; c < N; c++) {
    r[c] = mask[c] ? rhs[c] - q[c] : 0.0;
    pp[c] = r[c];
  }
  double bn = sqrt(dot_masked(N, mask, rhs, rhs));
  double rr = dot_masked(N, mask, r, r);
  int32_t it = 0;
  int st = ORC_OK;
  if (bn == 0.0) {
    for (int64_t c = 0; c < N; c++) x[c] = 0.0;
    rr = 0.0;
  }
  while (bn > 0.0 && sqrt(rr) > tol * bn) {
    if (it >= max_iter) { st = ORC_ENOCONV; break; }
    orc_nh_apply7_2d(nx, ny, cell, xface, yface, kxy, mask, pp, q);
    double pq = dot_masked(N, mask, pp, q);
    double alpha = rr / pq;
    for (int64_t c = 0; c < N; c++) {
      if (!mask[c]) continue;
      x[c] += alpha * pp[c];
      r[c] -= alpha * q[c];
    }
    double rr_new = dot_masked(N, mask, r, r);
    double beta = rr_new / rr;
    rr = rr_new;
    for (int64_t c = 0; c < N; c++) pp[c] = mask[c] ? r[c] + beta * pp[c] : 0.0;
    it++;
  }
  /* true residual of the returned iterate */
  orc_nh_apply7_2d(nx, ny, cell, xface, yface, kxy, mask, x, q);
  double tr = 0.0;
  for (int64_t c = 0; c < N; c++)
    if (mask[c]) tr += (rhs[c] - q[c]) * (rhs[c] - q[c]);
  if (iters) *iters = it;
  if (rel_res) *rel_res = (bn > 0.0) ? sqrt(tr) / bn : 0.0;
  free(r); free(pp); free(q);
  return st;
}

int orc_cg_2d(int32_t nx, int32_t ny, const double* cell, const double* xface, const double* yface,
              const uint8_t* mask, const double* rhs, double tol, int32_t max_iter, double* x,
              int32_t* iters, double* rel_res) {
  return orc_cg7_2d(nx, ny, cell, xface, yface, NULL, mask, rhs, tol, max_iter, x, iters, rel_res);
}

int orc_nh_correct7_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                       const double* yface, const double* kxy, double dt, double rho,
                       const double* mt, const double* nt, const double* kt,
                       const uint8_t* mask, const double* p, double* m_out, double* n_out,
                       double* k_out) {
  int64_t N = (int64_t)nx * ny, NX = (int64_t)ny * (nx + 1), NY = (int64_t)(ny + 1) * nx;
  const double *Dx = cell, *Dy = cell + N, *al = cell + 2 * N, *phi = cell + 3 * N;
#define PV(jj, ii) (((ii) >= 0 && (ii) < nx && (jj) >= 0 && (jj) < ny && mask[IDX(jj, ii)]) ? p[IDX(jj, ii)] : 0.0)
  for (int32_t j = 0; j < ny; j++) {
    for (int32_t i = 0; i < nx; i++) {
      int64_t c = IDX(j, i);
      if (!mask[c]) {
        m_out[c] = mt[c];
        n_out[c] = nt[c];
        k_out[c] = kt[c];
        continue;
      }
      int64_t fw = (int64_t)j * (nx + 1) + i, fe = fw + 1;
      int64_t fs = (int64_t)j * nx + i, fn = fs + nx;
      double dqw = xface[4 * NX + fw] - xface[fw] * (xface[NX + fw] * PV(j, i - 1) + xface[2 * NX + fw] * PV(j, i));
      double dqe = xface[4 * NX + fe] - xface[fe] * (xface[NX + fe] * PV(j, i) + xface[2 * NX + fe] * PV(j, i + 1));
      double dqs = yface[4 * NY + fs] - yface[fs] * (yface[NY + fs] * PV(j - 1, i) + yface[2 * NY + fs] * PV(j, i));
      double dqn = yface[4 * NY + fn] - yface[fn] * (yface[NY + fn] * PV(j, i) + yface[2 * NY + fn] * PV(j + 1, i));
      if (kxy) { /* the tensor's off-diagonal part, pair by pair as in orc_nh_apply7_2d */
        dqe -= kxy[c] * grad_north(nx, ny, yface, mask, p, j, i);
        dqn -= kxy[c] * grad_east(nx, ny, xface, mask, p, j, i);
        if (i > 0) dqw -= kxy[c - 1] * grad_north(nx, ny, yface, mask, p, j, i - 1);
        if (j > 0) dqs -= kxy[c - nx] * grad_east(nx, ny, xface, mask, p, j - 1, i);
      }
      double dm = 0.5 * (dqw + dqe), dn = 0.5 * (dqs + dqn);
      double Pb = 1.5 * p[c] - rho * (Dx[c] * dm + Dy[c] * dn) / (4.0 * dt) + al[c] * phi[c] / 4.0;
      m_out[c] = mt[c] + dm;
      n_out[c] = nt[c] + dn;
      k_out[c] = kt[c] + dt * Pb / rho;
    }
  }
#undef PV
  return ORC_OK;
}

int orc_nh_correct_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                      const double* yface, double dt, double rho, const double* mt,
                      const double* nt, const double* kt, const uint8_t* mask, const double* p,
                      double* m_out, double* n_out, double* k_out) {
  return orc_nh_correct7_2d(nx, ny, cell, xface, yface, NULL, dt, rho, mt, nt, kt, mask, p, m_out,
                            n_out, k_out);
}

int orc_step_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds, const orc_body* b,
                const orc_phys* ph, double cfl, double dt_fixed, int32_t step_index, double* t,
                double* h, double* m, double* n_, double* k, double* p, uint8_t* mask,
                double* dt_used, int32_t* n_active, int32_t* iters, double* rel_res) {
  if (nx < 3 || ny < 3 || !(dx > 0.0) || !(dy > 0.0)) return ORC_EINVAL;
  int64_t N = (int64_t)nx * ny, NX = (int64_t)ny * (nx + 1), NY = (int64_t)(ny + 1) * nx;
  int bad_nan = 0, bad_dry = 0;
  for (int64_t c = 0; c < N; c++) {
    if (!isfinite(h[c]) || !isfinite(m[c]) || !isfinite(n_[c]) || !isfinite(k[c])) bad_nan = 1;
    else if (!(h[c] > 0.0)) bad_dry = 1;
  }
  if (bad_nan) return ORC_ENAN;
  if (bad_dry) return ORC_EDRY;
  double rate = orc_max_rate_2d(nx, ny, dx, dy, h, m, n_, ph->g);
  if (!(rate <= 1e300)) return ORC_ENAN;
  double dt = (cfl > 0.0) ? cfl / rate : dt_fixed;
  if (!(dt > 0.0)) return ORC_EINVAL;
  double *ht = dalloc(N), *mt = dalloc(N), *nt = dalloc(N), *kt = dalloc(N), *rh = dalloc(N);
  double *cell = dalloc(7 * N), *xf = dalloc(5 * NX), *yf = dalloc(5 * NY);
  double* kxy = ph->tensor ? dalloc(N) : NULL;
  int32_t na = 0, it = 0;
  double rr = 0.0;
  int st = orc_predict_2d(nx, ny, dx, dy, ds, b, ph, *t, dt, h, m, n_, k, ht, mt, nt, kt);
  if (st != ORC_OK) goto done;
  na = orc_mask_2d(nx, ny, dx, dy, ds, b, ph, *t + dt, step_index == 0, ht, mt, nt, kt, mask);
  if (na < 0) { st = na; goto done; }
  if (na > 0) {
    st = orc_nh_coeffs_2d(nx, ny, dx, dy, ds, b, ph, *t + dt, dt, ht, mt, nt, kt, cell, xf, yf);
    if (st != ORC_OK) goto done;
    if (kxy) orc_nh_pairs_2d(nx, ny, dx, dy, ds, b, *t + dt, xf, yf, kxy);
    orc_nh_rhs_2d(nx, ny, cell, xf, yf, mask, rh);
    st = orc_cg7_2d(nx, ny, cell, xf, yf, kxy, mask, rh, ph->tol, ph->max_iter, p, &it, &rr);
    if (st != ORC_OK) goto done;
    orc_nh_correct7_2d(nx, ny, cell, xf, yf, kxy, dt, ph->rho, mt, nt, kt, mask, p, m, n_, k);
  } else {
    for (int64_t c = 0; c < N; c++) { p[c] = 0.0; m[c] = mt[c]; n_[c] = nt[c]; k[c] = kt[c]; }
  }
  for (int64_t c = 0; c < N; c++) h[c] = ht[c];
  *t += dt;
done:
  if (dt_used) *dt_used = dt;
  if (n_active) *n_active = na;
  if (iters) *iters = it;
  if (rel_res) *rel_res = rr;
  free(ht); free(mt); free(nt); free(kt); free(rh); free(cell); free(xf); free(yf); free(kxy);
  return st;
}
