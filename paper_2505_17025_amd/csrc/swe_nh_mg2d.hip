// swe_nh_mg2d.hip -- conjugate gradients with a geometric multigrid
// preconditioner for the 2D elliptic system of the global extension (every
// cell marked), gfx950.
//
// The operator is the 5-point matrix of the 2D elliptic system (diagonal dg,
// east and north couplings ce, cn; the west and south couplings are the
// neighbours' east and north ones).  Its pressure decays over h / sqrt(3), so
// with dx << h the Krylov iteration with a local preconditioner needs
// hundreds of iterations; a multigrid V-cycle removes the smooth error on
// coarser grids.
//
// Levels: cells aggregated 2 x 2 while both extents stay even and the grid
// holds more than MG_COARSE_MAX cells, with the coarse operators of
// k_mg_coarsen (5-point, computed once per solve).  One V-cycle: on each
// level one red-black Gauss-Seidel sweep from zero, restriction of the
// residual (R = sum over the four children), the coarser level's correction
// added piecewise constant (P = R^T), then one black-red sweep, so that the
// V-cycle is a symmetric operator; on the coarsest level (at most
// MG_COARSE_MAX cells, one block, in LDS) MG_COARSE_SWEEPS symmetric sweeps
// from zero.  The V-cycle runs in FP32; the Krylov vectors, the operator of
// the iteration and every dot product are FP64, so the solution is an FP64
// solution whatever the precision of the preconditioner.
//
// The smoothing kernels work on LDS tiles with a ring of two cells.  Red
// cells ((i + j) even) are updated first: from zero their value is b / C and
// needs no neighbour, so the way down (sweep, residual, restriction) is one
// kernel per level without storing the smoothed values, and the way up
// recomputes them.

// The iteration count is data-dependent while the step is a captured graph:
// the solve is a fixed budget of iterations whose kernels return at once
// when a device flag says the residual has met the tolerance.  Dot products
// are block partial sums reduced by one block in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "swe_nh_2d.h"
#include "swe_nh_common.h"

namespace swenh {

namespace {

constexpr int NTM = 256;             // threads per block of the level kernels
constexpr int MG_GRID_MAX = 2048;    // most blocks of a level kernel (grid-stride)
constexpr int MG_COARSE_SWEEPS = 4;  // symmetric sweeps on the coarsest level

struct Lvl {
  int nx, ny, l;  // cells, level
  const float *C, *E, *N;
};

// the cells of level l the solve works on: the level-0 box (multiples of
// 2^levels) halved l times
struct Box {
  int x0, y0, x1, y1;
  __device__ bool in(int i, int j) const { return i >= x0 && j >= y0 && i < x1 && j < y1; }
};
__device__ __forceinline__ Box box_of(const MgState* st, int l) {
  return Box{st->box[0] >> l, st->box[1] >> l, st->box[2] >> l, st->box[3] >> l};
}

// the kernels of an iteration return at once when the multigrid CG is not
// this step's solver or has converged
__device__ __forceinline__ bool idle(const MgState* s) { return !s->use || s->done != 0; }

// block sum of v (every thread of the block calls) -> part[blockIdx.x]
template <int NT = NTM>
__device__ void block_partial(double v, double* part) {
  __shared__ double red[NT / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; w++) t += red[w];
    part[blockIdx.x] = t;
  }
  __syncthreads();
}

int blocks_for(int64_t n) {
  const int64_t b = (n + NTM - 1) / NTM;
  return (int)(b < MG_GRID_MAX ? (b > 0 ? b : 1) : MG_GRID_MAX);
}

// ---------------------------------------------------------------------------
// level operators
// ---------------------------------------------------------------------------
// Coarse operator of the aggregates of 2 x 2 cells.  The Galerkin product
// R A P with piecewise-constant P keeps the mass-like part of A (its
// diagonal excess over the couplings, M = C + sum of the row's couplings,
// which are negative) exactly, but weighs the Laplacian-like rest about
// twice too strongly for smooth error, so the coarse correction would come
// out about half as large as it should.  The coarse operator is therefore
// (R A P + diag(R M+ P)) / 2, M+ = max(M, 0): couplings half the Galerkin
// ones, diagonal half the Galerkin diagonal plus half the children's mass.
// It is symmetric positive definite (half an SPD matrix plus a non-negative
// diagonal), so the V-cycle is an SPD preconditioner without any scaling of
// its coarse correction.
__global__ void __launch_bounds__(NTM) k_mg_coarsen(int nxf, const float* __restrict__ Cf,
                                                     const float* __restrict__ Ef,
                                                     const float* __restrict__ Nf, int nxc,
                                                     int lc, float* __restrict__ Cc,
                                                     float* __restrict__ Ec,
                                                     float* __restrict__ Nc, const MgState* st) {
  if (!st->use) return;
  const Box Bc = box_of(st, lc);
  const int bw = Bc.x1 - Bc.x0;
  const int64_t n = (int64_t)bw * (Bc.y1 - Bc.y0);
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    const int I = Bc.x0 + (int)(o % bw), J = Bc.y0 + (int)(o / bw);
    const int64_t c = (int64_t)J * nxc + I;
    const int64_t f00 = (int64_t)(2 * J) * nxf + 2 * I, f01 = f00 + 1, f10 = f00 + nxf,
                  f11 = f10 + 1;
    const bool w = I > Bc.x0, e = I + 1 < Bc.x1, s = J > Bc.y0, nn = J + 1 < Bc.y1;
    // the children's couplings: inside the aggregate, and across its edges
    const float ei0 = Ef[f00], ei1 = Ef[f10], ni0 = Nf[f00], ni1 = Nf[f01];
    const float ee0 = e ? Ef[f01] : 0.0f, ee1 = e ? Ef[f11] : 0.0f;
    const float ew0 = w ? Ef[f00 - 1] : 0.0f, ew1 = w ? Ef[f10 - 1] : 0.0f;
    const float nn0 = nn ? Nf[f10] : 0.0f, nn1 = nn ? Nf[f11] : 0.0f;
    const float ns0 = s ? Nf[f00 - nxf] : 0.0f, ns1 = s ? Nf[f01 - nxf] : 0.0f;
    const float c00 = Cf[f00], c01 = Cf[f01], c10 = Cf[f10], c11 = Cf[f11];
    const float gal = c00 + c01 + c10 + c11 + 2.0f * (ei0 + ei1) + 2.0f * (ni0 + ni1);
    const float mass = fmaxf(c00 + ew0 + ei0 + ns0 + ni0, 0.0f) +
                       fmaxf(c01 + ei0 + ee0 + ns1 + ni1, 0.0f) +
                       fmaxf(c10 + ew1 + ei1 + ni0 + nn0, 0.0f) +
                       fmaxf(c11 + ei1 + ee1 + ni1 + nn1, 0.0f);
    Cc[c] = 0.5f * (gal + mass);
    Ec[c] = 0.5f * (ee0 + ee1);
    Nc[c] = 0.5f * (nn0 + nn1);
  }
}

// ---------------------------------------------------------------------------
// smoothing sweeps on LDS tiles
// ---------------------------------------------------------------------------
// A block takes MTX x MTY cells of a level plus a ring of two cells (the
// right-hand side and the operator, FP32, in LDS; cells outside the box have
// C = 1 and no couplings, so their values stay 0) and one thread per 2 x 2
// aggregate of the tile; blocks whose tile misses the box return at once.  The pre-smoothing sweep from zero is never stored:
// its red values are b / C and its black values follow from those, so the
// kernel of the way up recomputes them.
constexpr int MTX = 64, MTY = 32;                // cells of a tile (even)
constexpr int MNT = (MTX / 2) * (MTY / 2);       // threads: one per aggregate
constexpr int RX = MTX + 4, RY = MTY + 4, RN = RX * RY;

struct MgTile {
  float b[RN], C[RN], E[RN], N[RN], v[RN];
};

__device__ __forceinline__ int tiles_x_of(int nx) { return (nx + MTX - 1) / MTX; }

// The tile's right-hand side and operator into LDS, and the red cells'
// starting values: b / C from zero, plus the coarse correction e of their
// aggregate on the way up (UP).  Every load of a thread is issued
// before its first store.
template <bool UP, typename B>
__device__ void load_tile(MgTile& T, const Lvl& L, const Box& Bx, const B* __restrict__ b, int i0,
                          int j0, int nxc, const float* __restrict__ e) {
  constexpr int KN = (RN + MNT - 1) / MNT;
  float bb[KN], cc[KN], ee[KN], nn[KN], cor[KN];
#pragma unroll
  for (int k = 0; k < KN; k++) {
    const int w = threadIdx.x + k * MNT;
    const int i = i0 - 2 + w % RX, j = j0 - 2 + w / RX;
    bb[k] = 0.0f;
    cc[k] = 1.0f;
    ee[k] = 0.0f;
    nn[k] = 0.0f;
    cor[k] = 0.0f;
    if (w < RN && Bx.in(i, j)) {
      const int64_t o = (int64_t)j * L.nx + i;
      bb[k] = (float)b[o];
      cc[k] = L.C[o];
      ee[k] = L.E[o];
      nn[k] = L.N[o];
      if (UP && ((i + j) & 1) == 0) cor[k] = e[(int64_t)(j >> 1) * nxc + (i >> 1)];
    }
  }
#pragma unroll
  for (int k = 0; k < KN; k++) {
    const int w = threadIdx.x + k * MNT;
    if (w >= RN) continue;
    T.b[w] = bb[k];
    T.C[w] = cc[k];
    T.E[w] = ee[k];
    T.N[w] = nn[k];
    if ((((w % RX) + (w / RX)) & 1) == 0) T.v[w] = bb[k] / cc[k] + (UP ? cor[k] : 0.0f);
  }
}

// off-diagonal part of row w applied to the values in LDS (w not on the
// region's outer ring)
__device__ __forceinline__ float off_sum(const MgTile& T, int w) {
  return T.E[w - 1] * T.v[w - 1] + T.E[w] * T.v[w + 1] + T.N[w - RX] * T.v[w - RX] +
         T.N[w] * T.v[w + RX];
}

// black cells of the tile and its first ring from the red values in LDS
__device__ __forceinline__ void black_sweep(MgTile& T) {
  for (int w = threadIdx.x; w < RN; w += MNT) {
    const int rx = w % RX, ry = w / RX;
    if (((rx + ry) & 1) && rx >= 1 && rx <= RX - 2 && ry >= 1 && ry <= RY - 2)
      T.v[w] = (T.b[w] - off_sum(T, w)) / T.C[w];
  }
}

// region index of the red cell (0, 0) of this thread's aggregate
__device__ __forceinline__ int agg_w00() {
  const int ax = threadIdx.x % (MTX / 2), ay = threadIdx.x / (MTX / 2);
  return (2 * ay + 2) * RX + 2 * ax + 2;
}

// pre-smoothing from zero (red, then black) and the residual of the tile's
// aggregates restricted to the coarse right-hand side bc (the residual is
// zero on the black cells, just updated)
template <typename B>
__global__ void __launch_bounds__(MNT) k_mg_down(Lvl L, const B* __restrict__ b, int nxc,
                                                  float* __restrict__ bc, const MgState* st) {
  if (idle(st)) return;
  const Box Bx = box_of(st, L.l), Bc = box_of(st, L.l + 1);
  const int tx = tiles_x_of(L.nx);
  const int i0 = (blockIdx.x % tx) * MTX, j0 = (blockIdx.x / tx) * MTY;
  if (i0 >= Bx.x1 || j0 >= Bx.y1 || i0 + MTX <= Bx.x0 || j0 + MTY <= Bx.y0) return;
  __shared__ MgTile T;
  load_tile<false>(T, L, Bx, b, i0, j0, 0, nullptr);
  __syncthreads();
  black_sweep(T);
  __syncthreads();
  const int I = i0 / 2 + threadIdx.x % (MTX / 2), J = j0 / 2 + threadIdx.x / (MTX / 2);
  if (Bc.in(I, J)) {
    const int w00 = agg_w00(), w11 = w00 + RX + 1;
    const float r00 = T.b[w00] - T.C[w00] * T.v[w00] - off_sum(T, w00);
    const float r11 = T.b[w11] - T.C[w11] * T.v[w11] - off_sum(T, w11);
    bc[(int64_t)J * nxc + I] = r00 + r11;
  }
}

// the way up: the pre-smoothed red values plus the coarse correction e of
// their aggregate, post-smoothing (black, then red), the
// result to z; on the finest level (part != null) also the block's partial
// sum of r . z with the FP64 residual r = b
template <typename B>
__global__ void __launch_bounds__(MNT) k_mg_up(Lvl L, const B* __restrict__ b, int nxc,
                                                const float* __restrict__ e, float* __restrict__ z,
                                                double* __restrict__ part, const MgState* st) {
  if (idle(st)) return;
  const Box Bx = box_of(st, L.l);
  const int tx = tiles_x_of(L.nx);
  const int i0 = (blockIdx.x % tx) * MTX, j0 = (blockIdx.x / tx) * MTY;
  if (i0 >= Bx.x1 || j0 >= Bx.y1 || i0 + MTX <= Bx.x0 || j0 + MTY <= Bx.y0) {
    if (part && threadIdx.x == 0) part[blockIdx.x] = 0.0;  // a tile with no work adds nothing
    return;
  }
  __shared__ MgTile T;
  load_tile<true>(T, L, Bx, b, i0, j0, nxc, e);
  __syncthreads();
  black_sweep(T);
  __syncthreads();
  const int ax = threadIdx.x % (MTX / 2), ay = threadIdx.x / (MTX / 2);
  const int i = i0 + 2 * ax, j = j0 + 2 * ay;
  double acc = 0.0;
  if (Bx.in(i, j)) {
    const int w00 = agg_w00(), w11 = w00 + RX + 1;
    const float z00 = (T.b[w00] - off_sum(T, w00)) / T.C[w00];
    const float z11 = (T.b[w11] - off_sum(T, w11)) / T.C[w11];
    const float z10 = T.v[w00 + 1], z01 = T.v[w00 + RX];
    const int64_t c00 = (int64_t)j * L.nx + i, c01 = c00 + L.nx;
    z[c00] = z00;
    z[c00 + 1] = z10;
    z[c01] = z01;
    z[c01 + 1] = z11;
    if (part)
      acc = (double)b[c00] * z00 + (double)b[c00 + 1] * z10 + (double)b[c01] * z01 +
            (double)b[c01 + 1] * z11;
  }
  if (part) block_partial<MNT>(acc, part);
}

// the coarsest level (n <= MG_COARSE_MAX cells, one block): symmetric
// red-black Gauss-Seidel from zero, the values in LDS, each thread's rows
// (right-hand side, reciprocal diagonal, couplings, neighbour positions) in
// registers
constexpr int NTC = 1024;
constexpr int KC = MG_COARSE_MAX / NTC;
static_assert(MG_COARSE_MAX % NTC == 0, "the coarsest level's cells split evenly over its threads");
__global__ void __launch_bounds__(NTC) k_mg_coarsest(Lvl L, const float* __restrict__ b,
                                                      float* __restrict__ x, const MgState* st) {
  if (idle(st)) return;
  __shared__ float sx[MG_COARSE_MAX];
  const int n = L.nx * L.ny;
  const Box Bx = box_of(st, L.l);
  float rb[KC], ic[KC], cw[KC], ce[KC], cs[KC], cn[KC];
  int nw[KC], ne[KC], ns[KC], nn[KC], col[KC];
#pragma unroll
  for (int k = 0; k < KC; k++) {
    const int o = threadIdx.x + k * NTC;
    const int i = o < n ? o % L.nx : 0, j = o < n ? o / L.nx : 0;
    const bool in = o < n && Bx.in(i, j);
    const bool w = in && i > Bx.x0, e = in && i + 1 < Bx.x1, s = in && j > Bx.y0,
               nr = in && j + 1 < Bx.y1;
    rb[k] = in ? b[o] : 0.0f;
    ic[k] = in ? 1.0f / L.C[o] : 0.0f;
    cw[k] = w ? L.E[o - 1] : 0.0f;
    ce[k] = e ? L.E[o] : 0.0f;
    cs[k] = s ? L.N[o - L.nx] : 0.0f;
    cn[k] = nr ? L.N[o] : 0.0f;
    // a missing neighbour points at the cell itself (with a zero coupling):
    // every value read is one the block has written
    nw[k] = w ? o - 1 : o;
    ne[k] = e ? o + 1 : o;
    ns[k] = s ? o - L.nx : o;
    nn[k] = nr ? o + L.nx : o;
    col[k] = in ? (i + j) & 1 : 2;
    sx[o] = 0.0f;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 2 * MG_COARSE_SWEEPS; sweep++) {
    const bool fwd = sweep < MG_COARSE_SWEEPS;
    for (int h = 0; h < 2; h++) {
      const int c = fwd ? h : 1 - h;  // forward sweeps red then black, backward black then red
#pragma unroll
      for (int k = 0; k < KC; k++)
        if (col[k] == c)
          sx[threadIdx.x + k * NTC] = (rb[k] - (cw[k] * sx[nw[k]] + ce[k] * sx[ne[k]] +
                                                cs[k] * sx[ns[k]] + cn[k] * sx[nn[k]])) * ic[k];
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < KC; k++)
    if (col[k] < 2) x[threadIdx.x + k * NTC] = sx[threadIdx.x + k * NTC];
}

// ---------------------------------------------------------------------------
// this step's box and choice
// ---------------------------------------------------------------------------
// The multigrid CG solves the system on a box of whole aggregates of the
// coarsest level: the whole grid in the global extension, else the bounding
// box of the active tiles when there are more than min_tiles of them (below
// that, the tile solver's iterations cost less than the levels' launches).
// One block.
__global__ void __launch_bounds__(1024) k_mg_box(MgState* st, const int* __restrict__ tile_list,
                                                 const int* n_list, int tiles_x, int tx2, int ty2,
                                                 int nx, int ny, int align, int global,
                                                 int min_tiles) {
  __shared__ int red[4][1024 / 64];
  const int nl = *n_list;
  int v[4] = {1 << 30, 1 << 30, -1, -1};  // tile x0, y0, x1, y1
  if (!global)
    for (int t = threadIdx.x; t < nl; t += 1024) {
      const int tile = tile_list[t], tx = tile % tiles_x, ty = tile / tiles_x;
      v[0] = min(v[0], tx);
      v[1] = min(v[1], ty);
      v[2] = max(v[2], tx);
      v[3] = max(v[3], ty);
    }
  for (int o = 32; o > 0; o >>= 1) {
    v[0] = min(v[0], __shfl_xor(v[0], o));
    v[1] = min(v[1], __shfl_xor(v[1], o));
    v[2] = max(v[2], __shfl_xor(v[2], o));
    v[3] = max(v[3], __shfl_xor(v[3], o));
  }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; k++) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < 1024 / 64; w++) {
    v[0] = min(v[0], red[0][w]);
    v[1] = min(v[1], red[1][w]);
    v[2] = max(v[2], red[2][w]);
    v[3] = max(v[3], red[3][w]);
  }
  int b[4] = {0, 0, nx, ny};
  int use = 1;
  if (!global) {
    use = nl > min_tiles ? 1 : 0;
    if (use) {
      b[0] = (v[0] * tx2) / align * align;
      b[1] = (v[1] * ty2) / align * align;
      b[2] = min(((v[2] + 1) * tx2 + align - 1) / align * align, nx);
      b[3] = min(((v[3] + 1) * ty2 + align - 1) / align * align, ny);
    }
  }
  for (int k = 0; k < 4; k++) st->box[k] = b[k];
  st->use = use;
  st->ok = 0;
  st->done = 0;
  st->it = 0;
}

// identity rows (and a zero right-hand side and guess) on the cells of the
// box whose tiles hold no marked cell: the assembly visits only the active
// tiles.  One block per tile.
__global__ void __launch_bounds__(256) k_mg_identity(const MgState* st,
                                                     const int* __restrict__ tile_pos,
                                                     int tiles_x, int tx2, int ty2, int nx,
                                                     double* dg, double* ce, double* cn, double* b,
                                                     double* x, float* dg32, float* ce32,
                                                     float* cn32, uint8_t* nb, double* cd) {
  if (!st->use || tile_pos[blockIdx.x] >= 0) return;
  const Box Bx = box_of(st, 0);
  const int i0 = (blockIdx.x % tiles_x) * tx2, j0 = (blockIdx.x / tiles_x) * ty2;
  for (int c = threadIdx.x; c < tx2 * ty2; c += 256) {
    const int i = i0 + c % tx2, j = j0 + c / tx2;
    if (!Bx.in(i, j)) continue;
    const int64_t o = (int64_t)j * nx + i;
    dg[o] = 1.0;
    ce[o] = 0.0;
    cn[o] = 0.0;
    b[o] = 0.0;
    x[o] = 0.0;
    dg32[o] = 1.0f;
    ce32[o] = 0.0f;
    cn32[o] = 0.0f;
    nb[o] = 0;
    if (cd) cd[o] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// conjugate gradients (FP64)
// ---------------------------------------------------------------------------
// the exact-tensor operator's two more couplings of cell (i, j) with v: to
// (i+1, j-1), stored at the cell, and to (i-1, j+1), stored at that cell
template <typename V>
__device__ __forceinline__ double apply_diag(const MgArgs& A, const Box& Bx, V v, int64_t o,
                                             int i, int j) {
  double a = 0.0;
  if (i + 1 < Bx.x1 && j > Bx.y0) a += A.cd[o] * v(o - A.nx + 1);
  if (i > Bx.x0 && j + 1 < Bx.y1) a += A.cd[o + A.nx - 1] * v(o + A.nx - 1);
  return a;
}

// A x at cell (i, j) of the box (couplings across the box's edge are zero:
// the cells beyond it hold no marked cell)
__device__ __forceinline__ double apply_64(const MgArgs& A, const Box& Bx, const double* v,
                                           int64_t o, int i, int j) {
  double a = A.dg[o] * v[o];
  if (i > Bx.x0) a += A.ce[o - 1] * v[o - 1];
  if (i + 1 < Bx.x1) a += A.ce[o] * v[o + 1];
  if (j > Bx.y0) a += A.cn[o - A.nx] * v[o - A.nx];
  if (j + 1 < Bx.y1) a += A.cn[o] * v[o + A.nx];
  if (A.cd) a += apply_diag(A, Bx, [&](int64_t u) { return v[u]; }, o, i, j);
  return a;
}

// grid-stride loop over the cells of the box: f(o, i, j) with o = j nx + i
template <typename F>
__device__ __forceinline__ void for_box(const MgArgs& A, const Box& Bx, F f) {
  const int bw = Bx.x1 - Bx.x0;
  const int64_t n = (int64_t)bw * (Bx.y1 - Bx.y0);
  for (int64_t k = blockIdx.x * (int64_t)NTM + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * NTM) {
    const int i = Bx.x0 + (int)(k % bw), j = Bx.y0 + (int)(k / bw);
    f((int64_t)j * A.nx + i, i, j);
  }
}

// r = b - A x, partial sums of r.r and b.b
// a restarted solve does nothing after a first solve that met the tolerance
__device__ __forceinline__ bool restart_done(const MgArgs& A) { return A.restart && A.st->ok; }

__global__ void __launch_bounds__(NTM) k_cg_init(MgArgs A) {
  if (!A.st->use || restart_done(A)) return;
  const Box Bx = box_of(A.st, 0);
  double rr = 0.0, bb = 0.0;
  for_box(A, Bx, [&](int64_t o, int i, int j) {
    const double r = A.b[o] - apply_64(A, Bx, A.x, o, i, j);
    A.r[o] = r;
    rr += r * r;
    bb += A.b[o] * A.b[o];
  });
  block_partial(rr, A.part);
  block_partial(bb, A.part + A.npart);
}

// p = z + beta p_old (p alternates between two buffers by iteration parity),
// q = A p, partial sums of p.q
__global__ void __launch_bounds__(NTM) k_cg_pq(MgArgs A) {
  const MgState* st = A.st;
  if (idle(st)) return;
  const Box Bx = box_of(st, 0);
  const int par = st->it & 1;
  const double* po = A.p[par ^ 1];
  double* pn = A.p[par];
  const double beta = st->beta;
  // the first direction is z itself (p_old is not read: it may hold anything)
  const bool first = st->it == 0;
  auto pv = [&](int64_t o) { return first ? (double)A.z[o] : (double)A.z[o] + beta * po[o]; };
  double pq = 0.0;
  for_box(A, Bx, [&](int64_t o, int i, int j) {
    const double pc = pv(o);
    double q = A.dg[o] * pc;
    if (i > Bx.x0) q += A.ce[o - 1] * pv(o - 1);
    if (i + 1 < Bx.x1) q += A.ce[o] * pv(o + 1);
    if (j > Bx.y0) q += A.cn[o - A.nx] * pv(o - A.nx);
    if (j + 1 < Bx.y1) q += A.cn[o] * pv(o + A.nx);
    if (A.cd) q += apply_diag(A, Bx, pv, o, i, j);
    pn[o] = pc;
    A.q[o] = q;
    pq += pc * q;
  });
  block_partial(pq, A.part);
}

// x += alpha p, r -= alpha q, partial sums of r.r
__global__ void __launch_bounds__(NTM) k_cg_update(MgArgs A) {
  const MgState* st = A.st;
  if (idle(st)) return;
  const Box Bx = box_of(st, 0);
  const double* p = A.p[st->it & 1];
  const double alpha = st->alpha;
  double rr = 0.0;
  for_box(A, Bx, [&](int64_t o, int, int) {
    A.x[o] += alpha * p[o];
    const double r = A.r[o] - alpha * A.q[o];
    A.r[o] = r;
    rr += r * r;
  });
  block_partial(rr, A.part);
}

// one block: the fixed-order sum of nb partial sums
__device__ double sum_partials(const double* part, int nb) {
  __shared__ double red[1024 / 64];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) s += part[k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)blockDim.x / 64; w++) t += red[w];
  __syncthreads();
  return t;
}

// the scalars of the iteration (one block); what: 0 after the initial
// residual, 1 after r.z (rho, beta), 2 after p.q (alpha), 3 after r.r (the
// convergence test, the iteration count)
__global__ void __launch_bounds__(1024) k_cg_scalars(MgArgs A, int what, int nb) {
  MgState* st = A.st;
  if (!st->use || (what != 0 && st->done) || restart_done(A)) return;
  const double s = sum_partials(A.part, nb);
  if (what == 0) {
    const double bb = sum_partials(A.part + A.npart, nb);
    if (threadIdx.x == 0) {
      st->bb = bb;
      st->rr = s;
      st->it = 0;
      st->done = (bb == 0.0 || s <= A.tol_rec * A.tol_rec * bb) ? 1 : 0;
    }
    return;
  }
  if (threadIdx.x != 0) return;
  if (what == 1) {
    st->beta = st->it == 0 ? 0.0 : s / st->rho;
    st->rho = s;
  } else if (what == 2) {
    st->alpha = s != 0.0 ? st->rho / s : 0.0;
  } else {
    st->rr = s;
    st->it += 1;
    if (!(s == s)) st->done = 2;  // not a number: stop, reported as no convergence
    else if (s <= A.tol_rec * A.tol_rec * st->bb) st->done = 1;
  }
}

// partial sums of the true residual ||b - A x||^2 of the final iterate
__global__ void __launch_bounds__(NTM) k_cg_true(MgArgs A) {
  if (!A.st->use || restart_done(A)) return;
  const Box Bx = box_of(A.st, 0);
  double rr = 0.0;
  for_box(A, Bx, [&](int64_t o, int i, int j) {
    const double r = A.b[o] - apply_64(A, Bx, A.x, o, i, j);
    rr += r * r;
  });
  block_partial(rr, A.part);
}

// statistics of the solve: iterations, relative true residual; a solve
// whose true residual misses the tolerance (the recursive one met it) counts
// as not converged: the continuing solver then takes over, or (last) the
// no-convergence status is set.  Nothing when the tile solver has the step.
__global__ void __launch_bounds__(1024) k_cg_finish(MgArgs A, int nb, int last) {
  MgState* st = A.st;
  if (!st->use) {  // nothing marked (the tile solver, if any, has the step)
    if (last && threadIdx.x == 0) {
      *A.iters = 0;
      *A.rel = 0.0;
    }
    return;
  }
  if (restart_done(A)) return;
  const double rr = sum_partials(A.part, nb);
  if (threadIdx.x != 0) return;
  const bool ok = st->done == 1 && (st->bb == 0.0 || rr <= A.tol * A.tol * st->bb);
  st->ok = ok ? 1 : 0;
  *A.iters = A.restart ? *A.iters + st->it : st->it;
  *A.iters_sum += st->it;
  *A.rel = st->bb > 0.0 ? sqrt(rr / st->bb) : 0.0;
  if (last && !ok) atomicOr(A.status, ST_NOCONV);
}

// after a continuing solver (which wrote its own iteration count): the step's
// count is the sum of both
__global__ void k_cg_account(MgArgs A) {
  if (A.st->use && !A.st->ok) *A.iters += A.st->it;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int mg_plan_levels(int nx, int ny, int* lnx, int* lny) {
  int L = 0;
  lnx[0] = nx;
  lny[0] = ny;
  while (L + 1 < MG_MAXL && (lnx[L] & 1) == 0 && (lny[L] & 1) == 0 &&
         (int64_t)lnx[L] * lny[L] > MG_COARSE_MAX) {
    lnx[L + 1] = lnx[L] / 2;
    lny[L + 1] = lny[L] / 2;
    L++;
  }
  if ((int64_t)lnx[L] * lny[L] > MG_COARSE_MAX || L < 1) return 0;  // no multigrid for this grid
  return L;
}

static int tiles_of(int nx, int ny) {
  return ((nx + MTX - 1) / MTX) * ((ny + MTY - 1) / MTY);
}

int mg_partials(int nx, int ny) { return std::max(MG_GRID_MAX, tiles_of(nx, ny)); }

void launch_mg_solve2d(Ctx2D* x, double tol, int budget, bool last, bool restart,
                       hipStream_t s) {
  const int L = x->mg_levels;
  const int64_t n0 = (int64_t)x->nx * x->ny;
  MgArgs A = x->mg_args;
  A.tol = tol;
  // the recursive residual stops the iteration; the true residual of the
  // final iterate must then meet tol.  With no solver to continue (last), the
  // recursion aims at half the tolerance, so that its drift from the true
  // residual cannot fail a converged solve
  A.tol_rec = last ? 0.5 * tol : tol;
  A.restart = restart ? 1 : 0;
  auto lvl = [&](int l) {
    return Lvl{x->mg_nx[l], x->mg_ny[l], l, x->mg_c[l], x->mg_e[l], x->mg_n[l]};
  };
  auto tiles = [&](int l) { return tiles_of(x->mg_nx[l], x->mg_ny[l]); };
  // the coarse operators of this solve (level 0 is the FP32 copy of the
  // operator written by the assembly)
  for (int l = 0; l < L && !restart; l++) {
    const int64_t nc = (int64_t)x->mg_nx[l + 1] * x->mg_ny[l + 1];
    hipLaunchKernelGGL(k_mg_coarsen, dim3(blocks_for(nc)), dim3(NTM), 0, s, x->mg_nx[l],
                       (const float*)x->mg_c[l], (const float*)x->mg_e[l],
                       (const float*)x->mg_n[l], x->mg_nx[l + 1], l + 1, x->mg_c[l + 1],
                       x->mg_e[l + 1], x->mg_n[l + 1], (const MgState*)A.st);
  }
  const int g0 = blocks_for(n0);
  hipLaunchKernelGGL(k_cg_init, dim3(g0), dim3(NTM), 0, s, A);
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 0, g0);
  const MgState* st = A.st;
  for (int it = 0; it < budget; it++) {
    // z = V-cycle(r)
    hipLaunchKernelGGL(k_mg_down<double>, dim3(tiles(0)), dim3(MNT), 0, s, lvl(0),
                       (const double*)A.r, x->mg_nx[1], x->mg_b[1], st);
    for (int l = 1; l < L; l++)
      hipLaunchKernelGGL(k_mg_down<float>, dim3(tiles(l)), dim3(MNT), 0, s, lvl(l),
                         (const float*)x->mg_b[l], x->mg_nx[l + 1], x->mg_b[l + 1], st);
    hipLaunchKernelGGL(k_mg_coarsest, dim3(1), dim3(NTC), 0, s, lvl(L),
                       (const float*)x->mg_b[L], x->mg_z[L], st);
    for (int l = L - 1; l >= 1; l--)
      hipLaunchKernelGGL(k_mg_up<float>, dim3(tiles(l)), dim3(MNT), 0, s, lvl(l),
                         (const float*)x->mg_b[l], x->mg_nx[l + 1], (const float*)x->mg_z[l + 1],
                         x->mg_z[l], (double*)nullptr, st);
    hipLaunchKernelGGL(k_mg_up<double>, dim3(tiles(0)), dim3(MNT), 0, s, lvl(0),
                       (const double*)A.r, x->mg_nx[1], (const float*)x->mg_z[1], A.z, A.part,
                       st);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 1, tiles(0));
    hipLaunchKernelGGL(k_cg_pq, dim3(g0), dim3(NTM), 0, s, A);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 2, g0);
    hipLaunchKernelGGL(k_cg_update, dim3(g0), dim3(NTM), 0, s, A);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 3, g0);
  }
  hipLaunchKernelGGL(k_cg_true, dim3(g0), dim3(NTM), 0, s, A);
  hipLaunchKernelGGL(k_cg_finish, dim3(1), dim3(1024), 0, s, A, g0, (int)last);
}

void launch_mg_box2d(Ctx2D* x, bool global, int min_tiles, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_box, dim3(1), dim3(1024), 0, s, x->mg_args.st,
                     (const int*)x->tile_list, (const int*)x->n_tiles_act, x->tiles_x, TX2, TY2,
                     x->nx, x->ny, 1 << x->mg_levels, global ? 1 : 0, min_tiles);
  hipLaunchKernelGGL(k_mg_identity, dim3(x->ntiles), dim3(256), 0, s,
                     (const MgState*)x->mg_args.st, (const int*)x->tile_pos, x->tiles_x, TX2, TY2,
                     x->nx, x->dg, x->ce, x->cn, x->b, x->x, x->dg32, x->ce32, x->cn32, x->nb,
                     x->cd);
}

void launch_mg_account2d(Ctx2D* x, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_account, dim3(1), dim3(1), 0, s, x->mg_args);
}

}  // namespace swenh
