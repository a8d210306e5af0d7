/*
 * swe_oracle.h -- plain FP64 CPU oracle of the locally adaptive non-hydrostatic
 * shallow water step (Firdaus & Behrens, "Locally Adaptive Non-Hydrostatic
 * Shallow Water Extension for Moving Bottom-Generated Waves").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product (the HIP
 * library under paper_2505_17025_amd/) never calls it and shares no code,
 * header, table or helper with it.
 *
 * Every routine is a direct, unblocked, unfused transcription of the method in
 * the paper's order: Heun predictor over a finite-volume hydrostatic operator
 * (Sec. 3.1, Eqs. 6-9 read with a finite-volume spatial operator), the
 * adaptivity criterion and its one-element enlargement (Sec. 5.1, 5.2), the
 * elliptic system of Eqs. 12-17 at degree zero with the flip-flop flux, solved
 * with zero Dirichlet data outside the non-hydrostatic area (Sec. 3.2), and the
 * backward-Euler projection of Eqs. 10-11.
 *
 * Conventions: SI units, cell-centred values, cell i of a 1D grid has centre
 * x_i = (i + 1/2) dx; 2D arrays are [ny][nx] with x fastest.  d is the still
 * water depth (positive downward, bottom at z = -d), h = eta + d the water
 * column thickness, m = hu, n = hv, k = hw.
 */
#ifndef SWE_ORACLE_H
#define SWE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOCONV = -2, ORC_EDRY = -3, ORC_ENAN = -4 };

/* Sec. 5.1: the six indicators, plus "everywhere" (global model) and
 * "nowhere" (pure hydrostatic SWE). */
enum { ORC_CRIT_ETA_D = 0, ORC_CRIT_ETA_X = 1, ORC_CRIT_U = 2, ORC_CRIT_U_X = 3,
       ORC_CRIT_W = 4, ORC_CRIT_W_X = 5, ORC_CRIT_GLOBAL = 6, ORC_CRIT_NONE = 7 };

/* Moving body subtracted from the static depth: d(x,t) = d_s(x) - B(x - X(t)). */
enum { ORC_BODY_NONE = 0, ORC_BODY_QUARTIC = 1, ORC_BODY_GAUSS = 2 };
/* Travel law s(t); X(t) = x0 + dir * s(t). */
enum { ORC_LAW_FIXED = 0, ORC_LAW_CONST_VEL = 1, ORC_LAW_SIN_RAMP = 2, ORC_LAW_PIECEWISE = 3 };

typedef struct {
  int32_t kind;   /* ORC_BODY_* */
  int32_t law;    /* ORC_LAW_* */
  double amp;     /* quartic: height H_s; gauss: amplitude A */
  double len;     /* quartic: length L_s; gauss: e-folding width w */
  double x0;      /* centre at t = 0 */
  double y0;      /* gauss (2D): fixed y of the centre */
  double dir;     /* horizontal projection of the travel (cos of the slope) */
  double q[5];    /* law parameters: CONST_VEL q0=v; SIN_RAMP q0=s_f q1=T_s;
                     PIECEWISE (Eq. 21) q0=a0 q1=u_t q2=t1 q3=t2 q4=t3 */
} orc_body;

typedef struct {
  double g, rho;
  double k_nh;          /* criterion threshold, Sec. 5.1 */
  int32_t crit;         /* ORC_CRIT_* */
  int32_t enlarge;      /* dilation of the NH area in cells, Sec. 5.2 */
  int32_t first_global; /* |w|, |w_x| criteria: global on the first step (Sec. 5.1.2) */
  double tol;           /* 2D CG: stop when ||b - A p|| <= tol ||b|| */
  int32_t max_iter;
  int32_t tensor;       /* 2D: 1 = the exact-tensor (7-point) operator, 0 = its diagonal */
} orc_phys;

/* ---- forcing ---- */
void orc_body_motion(const orc_body* b, double t, double* X, double* Xd, double* Xdd);
/* depth and analytic time derivatives of the moving bottom at the cell centres */
void orc_forcing_1d(int32_t n, double dx, const double* ds, const orc_body* b, double t,
                    double* d, double* d_t, double* d_tt, double* d_xt);
void orc_forcing_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                    const orc_body* b, double t, double* d, double* d_t, double* d_tt,
                    double* d_xt, double* d_yt);

/* ---- 1D ---- */
double orc_max_speed_1d(int32_t n, const double* h, const double* m, double g);
int orc_operator_1d(int32_t n, double dx, double g, const double* d, const double* h,
                    const double* m, const double* k, double* Lh, double* Lm, double* Lk);
int orc_predict_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                   double t, double dt, const double* h, const double* m, const double* k,
                   double* ht, double* mt, double* kt);
int orc_indicator_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                     double t1, const double* ht, const double* mt, const double* kt, double* ind);
int orc_mask_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                double t1, int32_t first_step, const double* ht, const double* mt, const double* kt,
                uint8_t* mask);
int orc_nh_coeffs_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                     double t1, double dt, const double* ht, const double* mt, const double* kt,
                     double* cell /* [8][n] */, double* face /* [8][n+1] */);
int orc_nh_system_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                     double t1, double dt, const double* ht, const double* mt, const double* kt,
                     const uint8_t* mask, double* diag, double* upper, double* rhs);
int orc_tridiag_solve(int32_t n, const double* diag, const double* upper, const double* rhs,
                      double* x);
int orc_nh_correct_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                      double t1, double dt, const double* ht, const double* mt, const double* kt,
                      const uint8_t* mask, const double* p, double* m_out, double* k_out);
int orc_step_1d(int32_t n, double dx, const double* ds, const orc_body* b, const orc_phys* ph,
                double cfl, double dt_fixed, int32_t step_index, double* t, double* h, double* m,
                double* k, double* p, uint8_t* mask, double* dt_used, int32_t* n_active);

/* ---- 2D ---- */
double orc_max_rate_2d(int32_t nx, int32_t ny, double dx, double dy, const double* h,
                       const double* m, const double* n_, double g);
int orc_operator_2d(int32_t nx, int32_t ny, double dx, double dy, double g, const double* d,
                    const double* h, const double* m, const double* n_, const double* k,
                    double* Lh, double* Lm, double* Ln, double* Lk);
int orc_predict_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                   const orc_body* b, const orc_phys* ph, double t, double dt, const double* h,
                   const double* m, const double* n_, const double* k, double* ht, double* mt,
                   double* nt, double* kt);
int orc_indicator_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                     const orc_body* b, const orc_phys* ph, double t1, const double* ht,
                     const double* mt, const double* nt, const double* kt, double* ind);
int orc_mask_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds, const orc_body* b,
                const orc_phys* ph, double t1, int32_t first_step, const double* ht,
                const double* mt, const double* nt, const double* kt, uint8_t* mask);
int orc_nh_coeffs_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                     const orc_body* b, const orc_phys* ph, double t1, double dt, const double* ht,
                     const double* mt, const double* nt, const double* kt,
                     double* cell /* [7][ny*nx] */, double* xface /* [5][ny*(nx+1)] */,
                     double* yface /* [5][(ny+1)*nx] */);
int orc_nh_apply_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                    const double* yface, const uint8_t* mask, const double* p, double* Ap);
int orc_nh_rhs_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                  const double* yface, const uint8_t* mask, double* rhs);
int orc_cg_2d(int32_t nx, int32_t ny, const double* cell, const double* xface, const double* yface,
              const uint8_t* mask, const double* rhs, double tol, int32_t max_iter, double* x,
              int32_t* iters, double* rel_res);
int orc_nh_correct_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                      const double* yface, double dt, double rho, const double* mt,
                      const double* nt, const double* kt, const uint8_t* mask, const double* p,
                      double* m_out, double* n_out, double* k_out);
/* the exact-tensor operator: per owner cell (j, i) the off-diagonal entry of
 * the face tensor that pairs the x-face east of the cell with the y-face north
 * of it; kxy == NULL in the routines below means the diagonal (5-point) form */
int orc_nh_pairs_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds,
                    const orc_body* b, double t1, const double* xface, const double* yface,
                    double* kxy /* [ny*nx] */);
int orc_nh_apply7_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                     const double* yface, const double* kxy, const uint8_t* mask,
                     const double* p, double* Ap);
int orc_cg7_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
               const double* yface, const double* kxy, const uint8_t* mask, const double* rhs,
               double tol, int32_t max_iter, double* x, int32_t* iters, double* rel_res);
int orc_nh_correct7_2d(int32_t nx, int32_t ny, const double* cell, const double* xface,
                       const double* yface, const double* kxy, double dt, double rho,
                       const double* mt, const double* nt, const double* kt,
                       const uint8_t* mask, const double* p, double* m_out, double* n_out,
                       double* k_out);
int orc_step_2d(int32_t nx, int32_t ny, double dx, double dy, const double* ds, const orc_body* b,
                const orc_phys* ph, double cfl, double dt_fixed, int32_t step_index, double* t,
                double* h, double* m, double* n_, double* k, double* p, uint8_t* mask,
                double* dt_used, int32_t* n_active, int32_t* iters, double* rel_res);

#ifdef __cplusplus
}
#endif
#endif
