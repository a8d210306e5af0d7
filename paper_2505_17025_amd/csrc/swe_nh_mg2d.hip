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
// holds more than 1024 cells.  Coarse operators by Galerkin projection with
// piecewise-constant transfers (R = sum over the four children, P = R^T):
// again 5-point, computed once per solve.  One V-cycle: on each level one
// red-black Gauss-Seidel sweep from zero, restriction of the residual,
// correction from the coarser level scaled by MG_OMEGA (piecewise-constant
// prolongation under-corrects smooth error by about half; over-correction
// restores the convergence rate), then one black-red sweep, so that the
// V-cycle is a symmetric operator; on the coarsest level (at most 1024 cells,
// one block, in LDS) MG_COARSE_SWEEPS symmetric sweeps from zero.  The V-cycle
// runs in FP32; the Krylov vectors, the operator of the iteration and every
// dot product are FP64, so the solution is an FP64 solution whatever the
// precision of the preconditioner.
//
// Each thread of a smoothing kernel owns one 2 x 2 aggregate.  Red cells
// ((i + j) even) are updated first: from zero their value is b / C and needs
// no neighbour, so a black cell's update and a red cell's residual can be
// recomputed from the arrays by whichever thread needs them, and one kernel
// does a whole sweep plus the residual and its restriction without a grid
// barrier.  The same holds for the post-smoothing sweep.
//
// The iteration count is data-dependent while the step is a captured graph:
// the solve is a fixed budget of iterations whose kernels return at once
// when a device flag says the residual has met the tolerance.  Dot products
// are block partial sums reduced by one block in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swe_nh_2d.h"
#include "swe_nh_common.h"

namespace swenh {

namespace {

constexpr int NTM = 256;             // threads per block of the level kernels
constexpr int MG_GRID_MAX = 2048;    // most blocks of a level kernel (grid-stride)
constexpr float MG_OMEGA = 1.6f;     // coarse-correction scale
constexpr int MG_COARSE_SWEEPS = 4;  // symmetric sweeps on the coarsest level

struct Lvl {
  int nx, ny;
  const float *C, *E, *N;
};

__device__ __forceinline__ bool done_of(const MgState* s) { return s->done != 0; }

// block sum of v (every thread of the block calls) -> part[blockIdx.x]
__device__ void block_partial(double v, double* part) {
  __shared__ double red[NTM / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NTM / 64; w++) t += red[w];
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
// smoothing sweeps of one aggregate
// ---------------------------------------------------------------------------
// values of the level's arrays at (i, j), zero off the grid (where the
// couplings towards it vanish anyway)
template <typename B>
struct Cells {
  const Lvl& L;
  const B* b;
  __device__ bool in(int i, int j) const { return i >= 0 && j >= 0 && i < L.nx && j < L.ny; }
  __device__ int64_t at(int i, int j) const { return (int64_t)j * L.nx + i; }
  __device__ float rhs(int i, int j) const { return (float)b[at(i, j)]; }
  // off-diagonal part of row (i, j) applied to the values v(., .)
  template <typename V>
  __device__ float off(int i, int j, V v) const {
    const int64_t o = at(i, j);
    float a = 0.0f;
    if (i > 0) a += L.E[o - 1] * v(i - 1, j);
    if (i + 1 < L.nx) a += L.E[o] * v(i + 1, j);
    if (j > 0) a += L.N[o - L.nx] * v(i, j - 1);
    if (j + 1 < L.ny) a += L.N[o] * v(i, j + 1);
    return a;
  }
};

// pre-smoothing from zero (red, then black), the residual of the four cells
// of aggregate (I, J) (zero on the black cells, just updated), the smoothed
// values to x and the aggregate's residual sum to bc
template <typename B>
__global__ void __launch_bounds__(NTM) k_mg_down(Lvl L, const B* __restrict__ b,
                                                  float* __restrict__ x, int nxc, int nyc,
                                                  float* __restrict__ bc, const MgState* st) {
  if (done_of(st)) return;
  const Cells<B> Q{L, b};
  auto red = [&](int i, int j) { return Q.in(i, j) ? Q.rhs(i, j) / L.C[Q.at(i, j)] : 0.0f; };
  auto blk = [&](int i, int j) {
    if (!Q.in(i, j)) return 0.0f;
    return (Q.rhs(i, j) - Q.off(i, j, red)) / L.C[Q.at(i, j)];
  };
  const int64_t n = (int64_t)nxc * nyc;
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    const int i0 = 2 * (int)(o % nxc), j0 = 2 * (int)(o / nxc);
    const float r00 = red(i0, j0), r11 = red(i0 + 1, j0 + 1);
    const float b10 = blk(i0 + 1, j0), b01 = blk(i0, j0 + 1);
    // red residuals: every neighbour of a red cell is black
    auto bl = [&](int i, int j) {
      if (i == i0 + 1 && j == j0) return b10;
      if (i == i0 && j == j0 + 1) return b01;
      return blk(i, j);
    };
    const float res00 = Q.rhs(i0, j0) - L.C[Q.at(i0, j0)] * r00 - Q.off(i0, j0, bl);
    const float res11 =
        Q.rhs(i0 + 1, j0 + 1) - L.C[Q.at(i0 + 1, j0 + 1)] * r11 - Q.off(i0 + 1, j0 + 1, bl);
    x[Q.at(i0, j0)] = r00;
    x[Q.at(i0 + 1, j0)] = b10;
    x[Q.at(i0, j0 + 1)] = b01;
    x[Q.at(i0 + 1, j0 + 1)] = r11;
    bc[o] = res00 + res11;
  }
}

// correction from the coarser level (omega e of the parent aggregate), then
// post-smoothing (black, then red); Z: the level's output (FP32 on coarse
// levels, the FP64 preconditioned residual on the finest, where the partial
// sums of r . z are also formed)
template <typename B, typename Z>
__global__ void __launch_bounds__(NTM) k_mg_up(Lvl L, const B* __restrict__ b,
                                                const float* __restrict__ x, int nxc,
                                                const float* __restrict__ e, Z* __restrict__ z,
                                                double* __restrict__ part, const MgState* st) {
  if (done_of(st)) return;
  const Cells<B> Q{L, b};
  auto y = [&](int i, int j) {  // corrected value (red neighbours of the black cells)
    if (!Q.in(i, j)) return 0.0f;
    return x[Q.at(i, j)] + MG_OMEGA * e[(int64_t)(j >> 1) * nxc + (i >> 1)];
  };
  auto blk = [&](int i, int j) {
    if (!Q.in(i, j)) return 0.0f;
    return (Q.rhs(i, j) - Q.off(i, j, y)) / L.C[Q.at(i, j)];
  };
  const int nyc = L.ny / 2;
  const int64_t n = (int64_t)nxc * nyc;
  double acc = 0.0;
  for (int64_t o = blockIdx.x * (int64_t)NTM + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * NTM) {
    const int i0 = 2 * (int)(o % nxc), j0 = 2 * (int)(o / nxc);
    const float b10 = blk(i0 + 1, j0), b01 = blk(i0, j0 + 1);
    auto bl = [&](int i, int j) {
      if (i == i0 + 1 && j == j0) return b10;
      if (i == i0 && j == j0 + 1) return b01;
      return blk(i, j);
    };
    const float r00 = (Q.rhs(i0, j0) - Q.off(i0, j0, bl)) / L.C[Q.at(i0, j0)];
    const float r11 = (Q.rhs(i0 + 1, j0 + 1) - Q.off(i0 + 1, j0 + 1, bl)) /
                      L.C[Q.at(i0 + 1, j0 + 1)];
    const int64_t c00 = Q.at(i0, j0), c10 = c00 + 1, c01 = c00 + L.nx, c11 = c01 + 1;
    z[c00] = (Z)r00;
    z[c10] = (Z)b10;
    z[c01] = (Z)b01;
    z[c11] = (Z)r11;
    if (part)
      acc += (double)b[c00] * (double)r00 + (double)b[c10] * (double)b10 +
             (double)b[c01] * (double)b01 + (double)b[c11] * (double)r11;
  }
  if (part) block_partial(acc, part);
}

// the coarsest level (n <= 1024 cells, one block): symmetric red-black
// Gauss-Seidel from zero in LDS
__global__ void __launch_bounds__(1024) k_mg_coarsest(Lvl L, const float* __restrict__ b,
                                                       float* __restrict__ x, const MgState* st) {
  if (done_of(st)) return;
  __shared__ float sC[1024], sE[1024], sN[1024], sb[1024], sx[1024];
  const int n = L.nx * L.ny;
  const int o = threadIdx.x;
  if (o < n) {
    sC[o] = L.C[o];
    sE[o] = L.E[o];
    sN[o] = L.N[o];
    sb[o] = b[o];
    sx[o] = 0.0f;
  }
  __syncthreads();
  const int i = o % L.nx, j = o / L.nx;
  const int colour = (i + j) & 1;
  for (int sweep = 0; sweep < 2 * MG_COARSE_SWEEPS; sweep++) {
    const bool fwd = sweep < MG_COARSE_SWEEPS;
    for (int h = 0; h < 2; h++) {
      const int c = fwd ? h : 1 - h;  // forward sweeps red then black, backward black then red
      if (o < n && colour == c) {
        float a = 0.0f;
        if (i > 0) a += sE[o - 1] * sx[o - 1];
        if (i + 1 < L.nx) a += sE[o] * sx[o + 1];
        if (j > 0) a += sN[o - L.nx] * sx[o - L.nx];
        if (j + 1 < L.ny) a += sN[o] * sx[o + L.nx];
        sx[o] = (sb[o] - a) / sC[o];
      }
      __syncthreads();
    }
  }
  if (o < n) x[o] = sx[o];
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
  block_partial(bb, A.part + MG_GRID_MAX);
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
  auto pv = [&](int64_t o) { return first ? A.z[o] : A.z[o] + beta * po[o]; };
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
    const double bb = sum_partials(A.part + MG_GRID_MAX, nb);
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

// statistics of the solve: iterations, relative true residual, no-convergence
__global__ void __launch_bounds__(1024) k_cg_finish(MgArgs A, int nb) {
  const MgState* st = A.st;
  const double rr = sum_partials(A.part, nb);
  if (threadIdx.x != 0) return;
  *A.iters = st->it;
  *A.iters_sum += st->it;
  *A.rel = st->bb > 0.0 ? sqrt(rr / st->bb) : 0.0;
  if (st->done != 1) atomicOr(A.status, ST_NOCONV);
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
         (int64_t)lnx[L] * lny[L] > 1024) {
    lnx[L + 1] = lnx[L] / 2;
    lny[L + 1] = lny[L] / 2;
    L++;
  }
  if ((int64_t)lnx[L] * lny[L] > 1024 || L < 1) return 0;  // no multigrid for this grid
  return L;
}

void launch_mg_solve2d(Ctx2D* x, double tol, int budget, hipStream_t s) {
  const int L = x->mg_levels;
  const int64_t n0 = (int64_t)x->nx * x->ny;
  MgArgs A = x->mg_args;
  A.tol = tol;
  auto lvl = [&](int l) { return Lvl{x->mg_nx[l], x->mg_ny[l], x->mg_c[l], x->mg_e[l], x->mg_n[l]}; };
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
    for (int l = 0; l < L; l++) {
      const int64_t nc = (int64_t)x->mg_nx[l + 1] * x->mg_ny[l + 1];
      if (l == 0)
        hipLaunchKernelGGL((k_mg_down<double>), dim3(blocks_for(nc)), dim3(NTM), 0, s, lvl(0),
                           (const double*)A.r, x->mg_x[0], x->mg_nx[1], x->mg_ny[1], x->mg_b[1],
                           st);
      else
        hipLaunchKernelGGL((k_mg_down<float>), dim3(blocks_for(nc)), dim3(NTM), 0, s, lvl(l),
                           (const float*)x->mg_b[l], x->mg_x[l], x->mg_nx[l + 1],
                           x->mg_ny[l + 1], x->mg_b[l + 1], st);
    }
    hipLaunchKernelGGL(k_mg_coarsest, dim3(1), dim3(1024), 0, s, lvl(L),
                       (const float*)x->mg_b[L], x->mg_z[L], st);
    for (int l = L - 1; l >= 0; l--) {
      const int64_t nc = (int64_t)x->mg_nx[l + 1] * x->mg_ny[l + 1];
      if (l == 0)
        hipLaunchKernelGGL((k_mg_up<double, double>), dim3(blocks_for(nc)), dim3(NTM), 0, s,
                           lvl(0), (const double*)A.r, (const float*)x->mg_x[0], x->mg_nx[1],
                           (const float*)x->mg_z[1], A.z, A.part, st);
      else
        hipLaunchKernelGGL((k_mg_up<float, float>), dim3(blocks_for(nc)), dim3(NTM), 0, s,
                           lvl(l), (const float*)x->mg_b[l], (const float*)x->mg_x[l],
                           x->mg_nx[l + 1], (const float*)x->mg_z[l + 1], x->mg_z[l],
                           (double*)nullptr, st);
    }
    const int gz = blocks_for((int64_t)x->mg_nx[1] * x->mg_ny[1]);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 1, gz);
    hipLaunchKernelGGL(k_cg_pq, dim3(g0), dim3(NTM), 0, s, A);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 2, g0);
    hipLaunchKernelGGL(k_cg_update, dim3(g0), dim3(NTM), 0, s, A);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1024), 0, s, A, 3, g0);
  }
  hipLaunchKernelGGL(k_cg_true, dim3(g0), dim3(NTM), 0, s, A);
  hipLaunchKernelGGL(k_cg_finish, dim3(1), dim3(1024), 0, s, A, g0);
}

}  // namespace swenh
