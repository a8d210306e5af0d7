// swe_nh_kernels.h -- kernel parameter blocks and host-side launchers shared
// between the kernel translation units and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swe_nh_common.h"

namespace swenh {

constexpr int TILE_MAX = 512;   // largest 1D tile (cells per block of the stencil kernels)
constexpr int ONEPASS_TILES = 512;  // most tiles of the one-kernel fused step
constexpr int TRI_ROWS = 1024;  // rows per block in the tridiagonal solver
constexpr int TRI_MAX_LEVELS = 6;
// The maximum wave speed of a channel is gathered in nslot partial maxima
// (nslot a power of two <= SPEED_SLOTS_MAX): block b folds its maximum into
// slot b % nslot, each slot on its own 128-byte line, so that the blocks of
// a long channel do not all queue on one address; readers take the maximum
// of the slots.  Slot k of channel ch, buffer q lies at
// smax[speed_at(q * batch + ch, k, nslot)].
constexpr int SPEED_SLOTS_MAX = 32;
constexpr int SPEED_PAD = 16;  // unsigned long long per slot
__host__ __device__ constexpr size_t speed_at(int qch, int k, int nslot) {
  return ((size_t)qch * nslot + k) * SPEED_PAD;
}

// parameter block of the 1D kernels (passed by value)
struct K1D {
  const Chan* ch;          // [batch]
  const int4* tiles;       // [ntiles] (channel, first cell, channel offset, channel cells)
  const int* first_tile;   // [batch]
  const double* ds;        // static depth [cells]
  double dx, g, rho, cfl, dt_fixed, k_nh;
  int crit, enlarge, first_global, ntiles;
  int tile;                // cells per 1D tile, at most cap
  int cap;                 // capacity of the tile kernels' LDS windows: 128, 256 or 512
  double* t;               // [batch] time at the start of the step (fused: [2][batch] by parity)
  double* dt;              // [batch] step of the current step
  unsigned long long* smax;  // [batch] slotted bit patterns of the max wave speed (speed_at)
  int nslot;               // speed slots in use per channel (power of two, <= SPEED_SLOTS_MAX)
  int* status;             // ST_* bits
  int* step;               // steps taken (fused: [2] by parity)
  int* tile_cnt;           // [ntiles]
  int* tile_off;           // [ntiles]
  int* n_act;              // marked cells
  int* act_cell;           // [cells] packed row -> global cell
  int* act_chan;           // [cells] packed row -> channel
  // tile-fused step (FP64): smax is then [2][batch], selected by step parity
  int fused;
  int nch;
  int max_ch_tiles;  // most tiles of one channel
  int* n_acc;              // [2] marked cells counted during a step, by step parity
  double* zw;              // [ZW_N][ntiles * cap] per marked row, tile-padded
  double *dg1, *up1, *rh1; // level-1 rows: first and last marked row of each tile
  double* x1;              // level-1 solution
  // one-kernel step (onepass, at most ONEPASS_TILES tiles): the tiles publish
  // their marked counts and level-1 rows as tagged words, each marked tile
  // solves the level-1 system itself (beyond 64 marked tiles block 0 solves
  // it and publishes the solution), and the marked tiles project in the same
  // kernel.  tw: [ntiles] counts, [ntiles][12] rows (F and L:
  // dg, up, rh), [ntiles][4] solution (F, L); tag1: tag of the last step;
  // l1s: [2][2 ntiles] scratch of block 0's sequential solve
  int onepass;
  int keep_speed;  // stage timing: block 0 leaves the speed buffer the step read in place
  // FP32 inner solve with FP64 refinement in the tile-fused step (refine = 1):
  // each tile's interior system is reduced in FP32 and refined with FP64
  // residuals until its componentwise backward error is at most tol, in at
  // most max_sweeps sweeps; sweeps / berr: [2] by step parity, the largest
  // sweep count and backward error (bit pattern) of the step's tiles;
  // iters_out / rel_out receive the last step's at the end of a run
  int refine;
  int max_sweeps;
  double tol;
  int* sweeps;
  unsigned long long* berr;
  int* iters_out;
  double* rel_out;
  unsigned long long* tw;
  unsigned* tag1;
  // two-kernel step: per channel, the step's dt and the body's motion at t^n
  // and t^{n+1} ([batch][CTAB_N]), written by k_chan_step before the step kernel
  double* ctab;
  // two-kernel step: the marked tiles of the step (appended by the step
  // kernel in any order; mcount reset by k_chan_step), walked by the projection
  int* mlist;
  int* mcount;
  double* l1s;
};

// per marked row of the tile-fused step: solution basis of the tile's
// interior system (x = z + u x_first + v x_last) and the projection data
enum {
  ZW_Z, ZW_U, ZW_V,                  // x = z + u x_first + v x_last
  ZW_KL, ZW_AL, ZW_BL, ZW_FL,        // left face: K, a, b, (dt / rho) phi d_x
  ZW_KR, ZW_AR, ZW_BR, ZW_FR,        // right face
  ZW_D, ZW_P,                        // cell: d_x, (4 + d_x^2) phi / 4
  ZW_HT, ZW_MT, ZW_KT,               // h~, hu~, hw~
  ZW_N
};

// per-channel step table of the two-kernel step (doubles per channel)
enum { CT_DT, CT_X0, CT_V0, CT_A0, CT_X1, CT_V1, CT_A1, CTAB_N = 8 };

// ---- 1D stencil / mask / projection ----
void launch_speed1d(const K1D& P, const double* h, const double* hu, const double* hw,
                    hipStream_t s);
void launch_pred1d(const K1D& P, const double* h, const double* hu, const double* hw, double* ht,
                   double* mt, double* kt, const double* t_in, const double* dt_in,
                   int dt_from_speed, hipStream_t s);
void launch_mask1d(const K1D& P, const double* ht, const double* mt, const double* kt,
                   const double* t_in, const double* dt_in, int mode_override, uint8_t* mask,
                   double* h, double* hu, double* hw, double* p, int write_state, hipStream_t s);
void launch_count1d(const K1D& P, const uint8_t* mask, hipStream_t s);
void launch_scan(const int* cnt, int* off, int n, int* total, hipStream_t s);
void launch_compact1d(const K1D& P, const uint8_t* mask, hipStream_t s);
void launch_assemble1d(const K1D& P, int64_t max_rows, const double* ht, const double* mt,
                       const double* kt, const uint8_t* mask, const double* t_in,
                       const double* dt_in, double* dg, double* up, double* rh, hipStream_t s);
void launch_correct1d(const K1D& P, int64_t max_rows, const double* ht, const double* mt,
                      const double* kt, const uint8_t* mask, const double* t_in,
                      const double* dt_in, const double* x, double* hu, double* hw, double* p,
                      hipStream_t s);
void launch_advance(const K1D& P, int nch, hipStream_t s);
// fused FP64 step: predictor + criterion + assembly + tile reduction from the
// state (h, hu, hw) into a second state buffer (hn, hun, hwn), and the
// projection from the level-1 solution (plus next-step speed and advance)
void launch_step1d(const K1D& P, const double* h, const double* hu, const double* hw, double* hn,
                   double* hun, double* hwn, uint8_t* mask, double* p, int par, hipStream_t s);
void launch_apply1d(const K1D& P, const uint8_t* mask, double* hun, double* hwn, double* p,
                    int par, hipStream_t s);
void launch_run_end(const K1D& P, int last_par, hipStream_t s);
bool level1_local(const K1D& P);  // the projection kernel solves the level-1 system itself
// else one block per channel solves it when every channel's part is small enough
bool level1_per_channel(const K1D& P);
void launch_level1_chan(const K1D& P, hipStream_t s);
int onepass_resident(const K1D& P);  // blocks of the one-kernel step that fit at once (0: error)
int fused_max_enlarge();
void launch_speed_prologue(const K1D& P, const double* h, const double* hu, const double* hw,
                           hipStream_t s);
void launch_fill(double* a, int64_t n, double v, hipStream_t s);
void launch_fill_i32(int* a, int64_t n, int v, hipStream_t s);
void launch_copy(const double* a, double* b, int64_t n, hipStream_t s);
void launch_gather_packed(const int* act_cell, const int* n_act, int64_t max_rows,
                          const double* full, double* packed, hipStream_t s);
void launch_scatter_packed(const int* act_cell, const int* n_act, int64_t max_rows,
                           const double* packed, double* full, hipStream_t s);

// ---- tridiagonal solver over a packed symmetric tridiagonal system ----
// level l has n_l rows (device count); rows l+1 = 2 * ceil(n_l / TRI_ROWS)
template <typename R>
struct TriLevels {
  int nlev;                          // number of levels (>= 1)
  int64_t nmax[TRI_MAX_LEVELS];      // host bound on the rows of each level
  R* dg[TRI_MAX_LEVELS];
  R* up[TRI_MAX_LEVELS];
  R* rh[TRI_MAX_LEVELS];
  R* x[TRI_MAX_LEVELS];
  int* n;                            // device [TRI_MAX_LEVELS]; n[0] is the caller's count
};
// solves level 0 (dg[0], up[0], rh[0], count *n0) into x[0]; conv (may be
// NULL): skip everything when *conv != 0
template <typename R>
void launch_tri_solve(const TriLevels<R>& T, const int* n0, const int* conv, hipStream_t s);

// ---- FP64 residual / FP32 refinement of the packed 1D system ----
void launch_resid1d(const double* dg, const double* up, const double* rh, const double* x,
                    const int* n, int64_t max_rows, float* r32, double* part, int with_b,
                    double* part_b, const int* conv, hipStream_t s);
void launch_resid_final(const double* part, const double* part_b, int nparts, int sweep,
                        double tol, double* norms /*[0]=rr,[1]=bb*/, double* rel, int* iters,
                        int* conv, int is_first, hipStream_t s);
void launch_refine_update(const float* e, double* x, const int* n, int64_t max_rows, int first,
                          const int* conv, hipStream_t s);
void launch_cast_sys(const double* dg, const double* up, const double* rh, const int* n,
                     int64_t max_rows, float* dg32, float* up32, float* rh32, hipStream_t s);
void launch_flag_noconv(const int* conv, int* status, hipStream_t s);

int resid_blocks(int64_t max_rows);

}  // namespace swenh
