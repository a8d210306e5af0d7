// swe_nh_2d.h -- 2D path (structured [ny][nx] grid): context and entry points
// used by the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swe_nh.h"
#include "swe_nh_kernels.h"

namespace swenh {

constexpr int TX2 = 32;  // tile width (cells along x) of the 2D kernels
constexpr int TY2 = 16;  // tile height
constexpr int PCG_NVEC = 10;  // inner vectors of the 2D solver
constexpr int CMAX2 = 128;     // most active tiles for which the solver adds the coarse space

constexpr int MG_MAXL = 12;    // most levels of the multigrid preconditioner (global extension)
constexpr int MG_BUDGET = 32;  // iterations of the multigrid-preconditioned CG in a step
// the same for the exact-tensor operator, which no other solver continues: a
// first solve of MG_TENSOR_FIRST iterations, then a restart from the true
// residual of its iterate (for a recursive residual that drifted from the
// true one, or more iterations) up to MG_BUDGET_TENSOR in all.  Every
// iteration's launches are paid whether or not it is needed (about 2 us
// each), which is why the restart's share is small
constexpr int MG_TENSOR_FIRST = 40;
constexpr int MG_BUDGET_TENSOR = 48;
constexpr int MG_COARSE_MAX = 4096;  // most cells of the multigrid's coarsest level (one block)
// active tiles above which an adaptive step's system goes to the multigrid CG
// on the active tiles' bounding box: up to CMAX2 tiles the tile solver has
// its coarse space and its pipelined iterations (7-9 us each) cost less than
// the multigrid's launches (about 90 us per iteration however small the box);
// beyond, its iteration count grows with the marked area (on the 2048^2
// shelf: 3-12 ms per step against 2.5-3.1 ms with the multigrid)
constexpr int MG_MIN_TILES = CMAX2;

// scalars of the multigrid-preconditioned CG (device)
struct MgState {
  int done;    // 0 running, 1 converged, 2 stopped on a non-finite residual
  int it;      // iterations taken
  int use;     // 1: this step's system is solved by the multigrid CG
  int ok;      // 1: the multigrid CG met the tolerance (its true residual)
  int box[4];  // x0, y0, x1, y1: the cells it works on (multiples of 2^levels)
  double rho, beta, alpha, rr, bb;
};

// the FP64 vectors and outputs of that CG
struct MgArgs {
  int nx = 0, ny = 0;
  const double *dg = nullptr, *ce = nullptr, *cn = nullptr, *b = nullptr;
  // the exact-tensor operator: coupling of each cell with (i+1, j-1) (nullptr:
  // the 5-point operator)
  const double* cd = nullptr;
  double* x = nullptr;
  double *r = nullptr, *q = nullptr, *p[2] = {nullptr, nullptr};
  float* z = nullptr;      // the preconditioned residual (output of the FP32 V-cycle)
  double* part = nullptr;  // block partial sums [2][npart]
  int npart = 0;
  MgState* st = nullptr;
  double tol = 0.0;      // on the true residual of the final iterate
  double tol_rec = 0.0;  // on the recursively updated residual (the stopping test)
  int restart = 0;       // a second solve from the true residual of the first one's iterate
  int* iters = nullptr;
  long long* iters_sum = nullptr;
  double* rel = nullptr;
  int* status = nullptr;
};

struct Ctx2D {
  int nx = 0, ny = 0, tiles_x = 0, tiles_y = 0, ntiles = 0;
  int grid_pcg = 0;          // blocks of the persistent solver (Chronopoulos-Gear form)
  int grid_pipe = 0;         // blocks of the persistent solver (pipelined form)
  // predictor output
  double *ht = nullptr, *mt = nullptr, *nt = nullptr, *kt = nullptr;
  uint8_t* mask_ws = nullptr;
  // tiles
  int* tile_cnt = nullptr;   // marked cells per tile
  double* tspeed = nullptr;  // per tile: max (|u| + c)/dx + (|v| + c)/dy of the new state
  int* tile_list = nullptr;  // active tiles
  int* tile_pos = nullptr;   // per tile: position in tile_list, -1 when inactive
  // coarse space of the preconditioner (one constant per active tile)
  double* crow = nullptr;    // [ntiles][5] coarse operator rows: self, E, W, N, S
  double* cinv = nullptr;    // [CMAX2 * CMAX2] inverse of the coarse operator
  int* cused = nullptr;      // [CMAX2 + 3] tiles, age and use of that inverse
  int* n_tiles_act = nullptr;
  int* n_act = nullptr;      // marked cells
  // operator (FP64 and FP32 copies), neighbour flags, right-hand side, solution
  double *dg = nullptr, *ce = nullptr, *cn = nullptr, *b = nullptr, *x = nullptr;
  float *dg32 = nullptr, *ce32 = nullptr, *cn32 = nullptr;
  uint8_t* nb = nullptr;
  // the exact-tensor operator (tensor2d): each cell's coupling with (i+1, j-1)
  // (dg, ce, cn then hold the 7-point operator's entries; the FP32 copy, the
  // multigrid's level 0, stays the 5-point operator, which preconditions it)
  double* cd = nullptr;
  int tensor = 0;
  // an adaptive 5-point step captured without the multigrid's launches (the
  // tile solver takes every step): chosen by the host while few tiles are
  // active, where the multigrid would not be used and its idle launches cost
  // more than the solve
  int mg_off = 0;
  // inner Krylov vectors, FP32 (precision 1) or FP64 (precision 0):
  // r, u, w, z, q, s, p, e, m[2] of the pipelined CG
  float* v32[PCG_NVEC] = {};
  double* v64[PCG_NVEC] = {};
  unsigned* tflag = nullptr;  // per tile: neighbour-sync stamp
  double* part = nullptr;    // [2][4][PCG_GMAX] block partial sums
  // tagged words of the pipelined solver: M^-1 w by tag parity (1 word per
  // value in FP32, 2 in FP64) and the block partials [2][4][PCG_GMAX][2]
  unsigned long long* mtag[2] = {nullptr, nullptr};
  unsigned long long* pt = nullptr;
  size_t tag_bytes = 0;
  unsigned* tag_base = nullptr;  // first tag of the next solve
  unsigned long long* bar = nullptr;  // grid barrier arrival counter
  int* iters = nullptr;
  long long* iters_sum = nullptr;
  double* rel = nullptr;
  // multigrid-preconditioned CG of the global extension (mg_levels > 0):
  // level l has mg_nx[l] x mg_ny[l] cells; operator C, E, N (level 0: the
  // FP32 copy dg32, ce32, cn32), right-hand side b and output z (l >= 1),
  // all FP32
  int mg_levels = 0;
  int mg_nx[MG_MAXL] = {}, mg_ny[MG_MAXL] = {};
  float *mg_c[MG_MAXL] = {}, *mg_e[MG_MAXL] = {}, *mg_n[MG_MAXL] = {};
  float *mg_b[MG_MAXL] = {}, *mg_z[MG_MAXL] = {};
  MgArgs mg_args;
  // learned warm start (warm = 2)
  char* cnn_ws = nullptr;
  size_t cnn_bytes = 0;
  uint16_t* feat = nullptr;
  double* guess = nullptr;
  int crop_w = 0, crop_h = 0;  // window of the grid the network sees (cells, multiples of 16)
  int* crop_org = nullptr;     // its origin (i0, j0), placed over the active tiles each step
  const float* net = nullptr;
  double fscale[4] = {1.0, 1.0, 1.0, 1.0};  // input scales of eta, hu, hv, -d_t
  double p_scale = 1.0;
  // shared scalars from the 1D block (time, dt, speed, status, step)
  double* t = nullptr;
  double* dt = nullptr;
  unsigned long long* smax = nullptr;
  int* status = nullptr;
  int* step = nullptr;
  const Chan* ch = nullptr;
};

// levels of the multigrid for an nx x ny grid (2 x 2 aggregation while both
// extents are even and the level has more than MG_COARSE_MAX cells); the
// number of coarsenings, 0 when the grid does not reach MG_COARSE_MAX cells
// that way
int mg_plan_levels(int nx, int ny, int* lnx, int* lny);
// block partial sums one reduction of that solver needs at most
int mg_partials(int nx, int ny);
// this step's box and choice: the whole grid (global), or the bounding box of
// the active tiles when there are more than min_tiles of them; the cells of
// inactive tiles inside the box get identity rows
void launch_mg_box2d(Ctx2D* x, bool global, int min_tiles, hipStream_t s);
// the global extension's solve of A x = b (x holds the initial guess): CG in
// FP64 preconditioned by one FP32 V-cycle, at most budget iterations.  With
// last, a solve that misses the tolerance sets the no-convergence status;
// otherwise another solver continues (launch_mg_account2d after it adds the
// multigrid iterations to the statistics)
// With restart, it continues a previous solve that missed the tolerance from
// the true residual of its iterate (and does nothing after one that met it);
// the coarse operators are that solve's, the iteration counts add up.
void launch_mg_solve2d(Ctx2D* x, double tol, int budget, bool last, bool restart, hipStream_t s);
void launch_mg_account2d(Ctx2D* x, hipStream_t s);

void plan2d(const swe_nh_config* c, char* base, size_t* off, Ctx2D* x);
int init2d(const swe_nh_config* c, Ctx2D* x, const K1D& k1, hipStream_t s);
// the warm-start network's weights packed for the convolution kernels
void pack_net2d(Ctx2D* x, hipStream_t s);
// speed of the caller's state -> dt of the first step of a call
void launch_speed2d_prologue(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* h,
                             const double* hu, const double* hv, const double* hw);
void enqueue_step2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, double* h, double* hu,
                    double* hv, double* hw, double* p, uint8_t* mask);
void launch_pred2d_stage(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* h,
                         const double* hu, const double* hv, const double* hw, const double* t_in,
                         const double* dt_in, double* ht, double* mt, double* nt, double* kt);
void launch_mask2d_stage(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
                         const double* mt, const double* nt, const double* kt,
                         const double* t_in, const double* dt_in, int mode, uint8_t* mask);
void solve_pressure2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
                      const double* mt, const double* nt, const double* kt, const uint8_t* mask,
                      const double* t_in, const double* dt_in, double* p);
void correct2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
               const double* mt, const double* nt, const double* kt, const uint8_t* mask,
               const double* p, const double* t_in, const double* dt_in, double* m_out,
               double* n_out, double* k_out);
void time_stage2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, int stage, double* h,
                  double* hu, double* hv, double* hw, double* p);

}  // namespace swenh
