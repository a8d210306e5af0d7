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
// holds more than MG_COARSE_MAX cells.  Coarse operators by Galerkin
// projection with piecewise-constant transfers (R = sum over the four
// children, P = R^T): again 5-point, computed once per solve.  One V-cycle:
// on each level one red-black Gauss-Seidel sweep from zero, restriction of
// the residual, correction from the coarser level scaled by MG_OMEGA
// (piecewise-constant prolongation under-corrects smooth error by about half;
// over-correction restores the convergence rate), then one black-red sweep,
// so that the V-cycle is a symmetric operator; on the coarsest level (at most
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
constexpr float MG_OMEGA = 1.8f;     // coarse-correction scale
constexpr int MG_COARSE_SWEEPS = 1;  // symmetric sweeps on the coarsest level

struct Lvl {
  int nx, ny;
  const float *C, *E, *N;
};

__device__ __forceinline__ bool done_of(const MgState* s) { return s->done != 0; }

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
// Galerkin coarse operator R A P of the aggregates of 2 x 2 cells: the
// children's diagonals plus twice the couplings inside the aggregate; the
// couplings across its east and north edges.
__global__ void __launch_bounds__(NTM) k_mg_coarsen(int nxf, const float* __restrict__ Cf,
                                                     const float* __restrict__ Ef,
                                                     const float* __restrict__ Nf, int nxc,
                                                     int nyc, float* __restrict__ Cc,
                                                     float* __restrict__ Ec,
                                                     float* __restrict__ Nc) {
  const int64_t n = (int64_t)nxc * nyc;
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    const int I = (int)(o % nxc), J = (int)(o / nxc);
    const int64_t f00 = (int64_t)(2 * J) * nxf + 2 * I, f01 = f00 + 1, f10 = f00 + nxf,
                  f11 = f10 + 1;
    Cc[o] = Cf[f00] + Cf[f01] + Cf[f10] + Cf[f11] + 2.0f * (Ef[f00] + Ef[f10]) +
            2.0f * (Nf[f00] + Nf[f01]);
    Ec[o] = I + 1 < nxc ? Ef[f01] + Ef[f11] : 0.0f;
    Nc[o] = J + 1 < nyc ? Nf[f10] + Nf[f11] : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// smoothing sweeps on LDS tiles
// ---------------------------------------------------------------------------
// A block takes MTX x MTY cells of a level plus a ring of two cells (the
// right-hand side and the operator, FP32, in LDS; cells off the grid have
// C = 1 and no couplings, so their values stay 0) and one thread per 2 x 2
// aggregate of the tile.  The pre-smoothing sweep from zero is never stored:
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
// starting values: b / C from zero, plus omega times the coarse correction e
// of their aggregate on the way up (UP).  Every load of a thread is issued
// before its first store.
template <bool UP, typename B>
__device__ void load_tile(MgTile& T, const Lvl& L, const B* __restrict__ b, int i0, int j0,
                          int nxc, const float* __restrict__ e) {
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
    if (w < RN && i >= 0 && j >= 0 && i < L.nx && j < L.ny) {
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
    if ((((w % RX) + (w / RX)) & 1) == 0) T.v[w] = bb[k] / cc[k] + (UP ? MG_OMEGA * cor[k] : 0.0f);
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
__global__ void __launch_bounds__(MNT) k_mg_down(Lvl L, const B* __restrict__ b, int nxc, int nyc,
                                                  float* __restrict__ bc, const MgState* st) {
  if (done_of(st)) return;
  __shared__ MgTile T;
  const int tx = tiles_x_of(L.nx);
  const int i0 = (blockIdx.x % tx) * MTX, j0 = (blockIdx.x / tx) * MTY;
  load_tile<false>(T, L, b, i0, j0, 0, nullptr);
  __syncthreads();
  black_sweep(T);
  __syncthreads();
  const int I = i0 / 2 + threadIdx.x % (MTX / 2), J = j0 / 2 + threadIdx.x / (MTX / 2);
  if (I < nxc && J < nyc) {
    const int w00 = agg_w00(), w11 = w00 + RX + 1;
    const float r00 = T.b[w00] - T.C[w00] * T.v[w00] - off_sum(T, w00);
    const float r11 = T.b[w11] - T.C[w11] * T.v[w11] - off_sum(T, w11);
    bc[(int64_t)J * nxc + I] = r00 + r11;
  }
}

// the way up: the pre-smoothed red values plus omega times the coarse
// correction e of their aggregate, post-smoothing (black, then red), the
// result to z; on the finest level (part != null) also the block's partial
// sum of r . z with the FP64 residual r = b
template <typename B>
__global__ void __launch_bounds__(MNT) k_mg_up(Lvl L, const B* __restrict__ b, int nxc,
                                                const float* __restrict__ e, float* __restrict__ z,
                                                double* __restrict__ part, const MgState* st) {
  if (done_of(st)) return;
  __shared__ MgTile T;
  const int tx = tiles_x_of(L.nx);
  const int i0 = (blockIdx.x % tx) * MTX, j0 = (blockIdx.x / tx) * MTY;
  load_tile<true>(T, L, b, i0, j0, nxc, e);
  __syncthreads();
  black_sweep(T);
  __syncthreads();
  const int ax = threadIdx.x % (MTX / 2), ay = threadIdx.x / (MTX / 2);
  const int i = i0 + 2 * ax, j = j0 + 2 * ay;
  double acc = 0.0;
  if (i < L.nx && j < L.ny) {
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
  if (done_of(st)) return;
  __shared__ float sx[MG_COARSE_MAX];
  const int n = L.nx * L.ny;
  float rb[KC], ic[KC], cw[KC], ce[KC], cs[KC], cn[KC];
  int nw[KC], ne[KC], ns[KC], nn[KC], col[KC];
#pragma unroll
  for (int k = 0; k < KC; k++) {
    const int o = threadIdx.x + k * NTC;
    const bool in = o < n;
    const int i = in ? o % L.nx : 0, j = in ? o / L.nx : 0;
    const bool w = in && i > 0, e = in && i + 1 < L.nx, s = in && j > 0, nr = in && j + 1 < L.ny;
    rb[k] = in ? b[o] : 0.0f;
    ic[k] = in ? 1.0f / L.C[o] : 0.0f;
    cw[k] = w ? L.E[o - 1] : 0.0f;
    ce[k] = e ? L.E[o] : 0.0f;
    cs[k] = s ? L.N[o - L.nx] : 0.0f;
    cn[k] = nr ? L.N[o] : 0.0f;
    nw[k] = w ? o - 1 : 0;
    ne[k] = e ? o + 1 : 0;
    ns[k] = s ? o - L.nx : 0;
    nn[k] = nr ? o + L.nx : 0;
    col[k] = in ? (i + j) & 1 : 2;
    if (in) sx[o] = 0.0f;
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
// conjugate gradients (FP64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double apply5_64(const double* dg, const double* ce, const double* cn,
                                            const double* v, int64_t o, int i, int j, int nx,
                                            int ny) {
  double a = dg[o] * v[o];
  if (i > 0) a += ce[o - 1] * v[o - 1];
  if (i + 1 < nx) a += ce[o] * v[o + 1];
  if (j > 0) a += cn[o - nx] * v[o - nx];
  if (j + 1 < ny) a += cn[o] * v[o + nx];
  return a;
}

// r = b - A x, partial sums of r.r and b.b
__global__ void __launch_bounds__(NTM) k_cg_init(MgArgs A) {
  const int64_t n = (int64_t)A.nx * A.ny;
  double rr = 0.0, bb = 0.0;
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    const int i = (int)(o % A.nx), j = (int)(o / A.nx);
    const double r = A.b[o] - apply5_64(A.dg, A.ce, A.cn, A.x, o, i, j, A.nx, A.ny);
    A.r[o] = r;
    rr += r * r;
    bb += A.b[o] * A.b[o];
  }
  block_partial(rr, A.part);
  block_partial(bb, A.part + A.npart);
}

// p = z + beta p_old (p alternates between two buffers by iteration parity),
// q = A p, partial sums of p.q
__global__ void __launch_bounds__(NTM) k_cg_pq(MgArgs A) {
  const MgState* st = A.st;
  if (done_of(st)) return;
  const int par = st->it & 1;
  const double* po = A.p[par ^ 1];
  double* pn = A.p[par];
  const double beta = st->beta;
  const int64_t n = (int64_t)A.nx * A.ny;
  // the first direction is z itself (p_old is not read: it may hold anything)
  const bool first = st->it == 0;
  auto pv = [&](int64_t o) { return first ? (double)A.z[o] : (double)A.z[o] + beta * po[o]; };
  double pq = 0.0;
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    const int i = (int)(o % A.nx), j = (int)(o / A.nx);
    const double pc = pv(o);
    double q = A.dg[o] * pc;
    if (i > 0) q += A.ce[o - 1] * pv(o - 1);
    if (i + 1 < A.nx) q += A.ce[o] * pv(o + 1);
    if (j > 0) q += A.cn[o - A.nx] * pv(o - A.nx);
    if (j + 1 < A.ny) q += A.cn[o] * pv(o + A.nx);
    pn[o] = pc;
    A.q[o] = q;
    pq += pc * q;
  }
  block_partial(pq, A.part);
}

// x += alpha p, r -= alpha q, partial sums of r.r
__global__ void __launch_bounds__(NTM) k_cg_update(MgArgs A) {
  const MgState* st = A.st;
  if (done_of(st)) return;
  const double* p = A.p[st->it & 1];
  const double alpha = st->alpha;
  const int64_t n = (int64_t)A.nx * A.ny;
  double rr = 0.0;
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    A.x[o] += alpha * p[o];
    const double r = A.r[o] - alpha * A.q[o];
    A.r[o] = r;
    rr += r * r;
  }
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
  if (what != 0 && st->done) return;
  const double s = sum_partials(A.part, nb);
  if (what == 0) {
    const double bb = sum_partials(A.part + A.npart, nb);
    if (threadIdx.x == 0) {
      st->bb = bb;
      st->rr = s;
      st->it = 0;
      st->done = (bb == 0.0 || s <= A.tol * A.tol * bb) ? 1 : 0;
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
    else if (s <= A.tol * A.tol * st->bb) st->done = 1;
  }
}

// partial sums of the true residual ||b - A x||^2 of the final iterate
__global__ void __launch_bounds__(NTM) k_cg_true(MgArgs A) {
  const int64_t n = (int64_t)A.nx * A.ny;
  double rr = 0.0;
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    const int i = (int)(o % A.nx), j = (int)(o / A.nx);
    const double r = A.b[o] - apply5_64(A.dg, A.ce, A.cn, A.x, o, i, j, A.nx, A.ny);
    rr += r * r;
  }
  block_partial(rr, A.part);
}

// statistics of the solve: iterations, relative true residual; a solve
// whose true residual misses the tolerance (the recursive one met it) counts
// as not converged: the continuing solver then takes over, or (last) the
// no-convergence status is set
__global__ void __launch_bounds__(1024) k_cg_finish(MgArgs A, int nb, int last) {
  MgState* st = A.st;
  const double rr = sum_partials(A.part, nb);
  if (threadIdx.x != 0) return;
  const bool ok = st->done == 1 && (st->bb == 0.0 || rr <= A.tol * A.tol * st->bb);
  if (!ok && st->done == 1) st->done = 0;
  *A.iters = st->it;
  *A.iters_sum += st->it;
  *A.rel = st->bb > 0.0 ? sqrt(rr / st->bb) : 0.0;
  if (last && !ok) atomicOr(A.status, ST_NOCONV);
}

// after a continuing solver (which wrote its own iteration count): the step's
// count is the sum of both
__global__ void k_cg_account(MgArgs A) {
  if (A.st->done != 1) *A.iters += A.st->it;
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

void launch_mg_solve2d(Ctx2D* x, double tol, int budget, bool last, hipStream_t s) {
  const int L = x->mg_levels;
  const int64_t n0 = (int64_t)x->nx * x->ny;
  MgArgs A = x->mg_args;
  A.tol = tol;
  auto lvl = [&](int l) {
    return Lvl{x->mg_nx[l], x->mg_ny[l], x->mg_c[l], x->mg_e[l], x->mg_n[l]};
  };
  auto tiles = [&](int l) { return tiles_of(x->mg_nx[l], x->mg_ny[l]); };
  // the coarse operators of this solve (level 0 is the FP32 copy of the
  // operator written by the assembly)
  for (int l = 0; l < L; l++) {
    const int64_t nc = (int64_t)x->mg_nx[l + 1] * x->mg_ny[l + 1];
    hipLaunchKernelGGL(k_mg_coarsen, dim3(blocks_for(nc)), dim3(NTM), 0, s, x->mg_nx[l],
                       (const float*)x->mg_c[l], (const float*)x->mg_e[l],
                       (const float*)x->mg_n[l], x->mg_nx[l + 1], x->mg_ny[l + 1], x->mg_c[l + 1],
                       x->mg_e[l + 1], x->mg_n[l + 1]);
  }
  const int g0 = blocks_for(n0);
  hipLaunchKernelGGL(k_cg_init, dim3(g0), dim3(NTM), 0, s, A);
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 0, g0);
  const MgState* st = A.st;
  for (int it = 0; it < budget; it++) {
    // z = V-cycle(r)
    hipLaunchKernelGGL(k_mg_down<double>, dim3(tiles(0)), dim3(MNT), 0, s, lvl(0),
                       (const double*)A.r, x->mg_nx[1], x->mg_ny[1], x->mg_b[1], st);
    for (int l = 1; l < L; l++)
      hipLaunchKernelGGL(k_mg_down<float>, dim3(tiles(l)), dim3(MNT), 0, s, lvl(l),
                         (const float*)x->mg_b[l], x->mg_nx[l + 1], x->mg_ny[l + 1],
                         x->mg_b[l + 1], st);
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

void launch_mg_account2d(Ctx2D* x, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_account, dim3(1), dim3(1), 0, s, x->mg_args);
}

}  // namespace swenh
