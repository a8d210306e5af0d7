// swe_nh_tri.hip -- packed symmetric tridiagonal solver for the 1D elliptic
// system (all marked runs of all channels in one system; a run ends where
// the coupling to the next row is zero).
//
// Block-recursive Schur complement, no pivoting (every Schur complement of
// the SPD matrix is SPD):
//   * a chunk is TRI_ROWS = 1024 consecutive rows, 4 per thread of the block
//     that walks it (a level's grid is capped, so a block may walk several);
//   * each thread eliminates its two interior rows (closed 2x2 inverse),
//     leaving a 512-row tridiagonal system of the threads' end rows in LDS;
//   * reduce: that system, with its first and last rows pinned, is solved by
//     parallel cyclic reduction for three right-hand sides, which yields the
//     chunk's Schur complement on its first and last rows -> 2 rows per chunk
//     of the next level;
//   * the last level (<= 1024 rows) is solved by one block;
//   * back-substitution re-runs each chunk with its end rows known.
#include "swe_nh_common.h"
#include "swe_nh_kernels.h"

namespace swenh {
namespace {

constexpr int RROWS = TRI_ROWS / 2;  // rows of the in-LDS reduced system
constexpr int TPB = TRI_ROWS / 4;    // threads per block

template <typename R, int NR>
struct TriSmem {
  R a[RROWS], b[RROWS], c[RROWS];
  R d[NR][RROWS];
};

struct Four {
  double d[4], u[4], b[4];
};

template <typename R>
struct Rows4 {
  R d[4], u[4], b[4], lo;
};

// load the thread's four rows (identity beyond n) and its coupling to the row before
template <typename R>
__device__ __forceinline__ Rows4<R> load4(const R* dg, const R* up, const R* rh, int n, int r) {
  Rows4<R> q;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int row = r + j;
    const bool in = row < n;
    q.d[j] = in ? dg[row] : R(1);
    q.u[j] = (in && row + 1 < n) ? up[row] : R(0);
    q.b[j] = in ? rh[row] : R(0);
  }
  q.lo = (r > 0 && r - 1 < n) ? up[r - 1] : R(0);
  return q;
}

// eliminate rows 1, 2 of the thread's block: writes reduced rows 2t (first)
// and 2t + 1 (last) into S (coefficients and right-hand side 0)
template <typename R, int NR>
__device__ __forceinline__ void reduce4(const Rows4<R>& q, TriSmem<R, NR>& S, int t) {
  const R det = q.d[1] * q.d[2] - q.u[1] * q.u[1];
  const R z1 = (q.d[2] * q.b[1] - q.u[1] * q.b[2]) / det;
  const R z2 = (q.d[1] * q.b[2] - q.u[1] * q.b[1]) / det;
  const R sff = q.d[0] - q.u[0] * q.u[0] * q.d[2] / det;
  const R sll = q.d[3] - q.u[2] * q.u[2] * q.d[1] / det;
  const R sfl = q.u[0] * q.u[1] * q.u[2] / det;
  S.a[2 * t] = q.lo;
  S.b[2 * t] = sff;
  S.c[2 * t] = sfl;
  S.d[0][2 * t] = q.b[0] - q.u[0] * z1;
  S.a[2 * t + 1] = sfl;
  S.b[2 * t + 1] = sll;
  S.c[2 * t + 1] = q.u[3];
  S.d[0][2 * t + 1] = q.b[3] - q.u[2] * z2;
}

// parallel cyclic reduction on the RROWS-row system in LDS; afterwards row i
// reads b[i] x_i = d[.][i]
template <typename R, int NR>
__device__ void pcr(TriSmem<R, NR>& S) {
  const int t = threadIdx.x;
  for (int s = 1; s < RROWS; s <<= 1) {
    R na[2], nb[2], nc[2], nd[2][NR];
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const int i = 2 * t + j;
      const int im = i - s, ip = i + s;
      R bi = S.b[i], ai = R(0), ci = R(0);
      R di[NR];
#pragma unroll
      for (int r = 0; r < NR; r++) di[r] = S.d[r][i];
      if (im >= 0) {
        const R k1 = S.a[i] / S.b[im];
        ai = -S.a[im] * k1;
        bi -= S.c[im] * k1;
#pragma unroll
        for (int r = 0; r < NR; r++) di[r] -= S.d[r][im] * k1;
      }
      if (ip < RROWS) {
        const R k2 = S.c[i] / S.b[ip];
        ci = -S.c[ip] * k2;
        bi -= S.a[ip] * k2;
#pragma unroll
        for (int r = 0; r < NR; r++) di[r] -= S.d[r][ip] * k2;
      }
      na[j] = ai;
      nb[j] = bi;
      nc[j] = ci;
#pragma unroll
      for (int r = 0; r < NR; r++) nd[j][r] = di[r];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const int i = 2 * t + j;
      S.a[i] = na[j];
      S.b[i] = nb[j];
      S.c[i] = nc[j];
#pragma unroll
      for (int r = 0; r < NR; r++) S.d[r][i] = nd[j][r];
    }
    __syncthreads();
  }
}

template <typename R>
__global__ void __launch_bounds__(TPB) k_tri_reduce(const R* __restrict__ dg,
                                                    const R* __restrict__ up,
                                                    const R* __restrict__ rh, const int* n_in,
                                                    R* __restrict__ dg2, R* __restrict__ up2,
                                                    R* __restrict__ rh2, int* n_out,
                                                    const int* conv) {
  if (conv && *conv) return;
  const int n = *n_in;
  const int nchunks = (n + TRI_ROWS - 1) / TRI_ROWS;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = 2 * nchunks;
  __shared__ TriSmem<R, 3> S;
  const int t = threadIdx.x;
  for (int cb = blockIdx.x; cb < nchunks; cb += gridDim.x) {  // the block's chunks
    const int row0 = cb * TRI_ROWS;
    const Rows4<R> q = load4(dg, up, rh, n, row0 + 4 * t);
    reduce4(q, S, t);
    __syncthreads();
    // keep the block's end rows, then pin them: x_0 and x_last are parameters
    const R b0 = S.b[0], c0 = S.c[0], d0 = S.d[0][0];
    const R aL = S.a[RROWS - 1], bL = S.b[RROWS - 1], dL = S.d[0][RROWS - 1];
    __syncthreads();
    for (int j = 0; j < 2; j++) {
      const int i = 2 * t + j;
      const bool first = (i == 0), last = (i == RROWS - 1);
      if (first || last) {
        S.a[i] = R(0);
        S.c[i] = R(0);
        S.b[i] = R(1);
        S.d[0][i] = R(0);
      }
      S.d[1][i] = first ? R(1) : R(0);
      S.d[2][i] = last ? R(1) : R(0);
    }
    __syncthreads();
    pcr<R, 3>(S);
    if (t == 0) {
      const R z1 = S.d[0][1] / S.b[1], u1 = S.d[1][1] / S.b[1], v1 = S.d[2][1] / S.b[1];
      const R zL = S.d[0][RROWS - 2] / S.b[RROWS - 2];
      const R vL = S.d[2][RROWS - 2] / S.b[RROWS - 2];
      const int o = 2 * cb;
      dg2[o] = b0 + c0 * u1;
      up2[o] = c0 * v1;
      rh2[o] = d0 - c0 * z1;
      dg2[o + 1] = bL + aL * vL;
      rh2[o + 1] = dL - aL * zL;
      const int lastrow = row0 + TRI_ROWS - 1;
      up2[o + 1] = (lastrow + 1 < n) ? up[lastrow] : R(0);
    }
    __syncthreads();  // S is rewritten by the next chunk
  }
}

// xnext == nullptr: the whole system fits one chunk (top level); otherwise
// chunk c has end values xnext[2c], xnext[2c + 1]
template <typename R>
__global__ void __launch_bounds__(TPB) k_tri_solve(const R* __restrict__ dg,
                                                   const R* __restrict__ up,
                                                   const R* __restrict__ rh, const int* n_in,
                                                   const R* __restrict__ xnext, R* __restrict__ x,
                                                   const int* conv) {
  if (conv && *conv) return;
  const int n = *n_in;
  const int nchunks = (n + TRI_ROWS - 1) / TRI_ROWS;
  __shared__ TriSmem<R, 1> S;
  const int t = threadIdx.x;
  for (int cb = blockIdx.x; cb < nchunks; cb += gridDim.x) {  // the block's chunks
    const int row0 = cb * TRI_ROWS;
    const Rows4<R> q = load4(dg, up, rh, n, row0 + 4 * t);
    reduce4(q, S, t);
    __syncthreads();
    if (xnext) {
      if (t == 0) {
        S.a[0] = R(0);
        S.c[0] = R(0);
        S.b[0] = R(1);
        S.d[0][0] = xnext[2 * cb];
        S.a[RROWS - 1] = R(0);
        S.c[RROWS - 1] = R(0);
        S.b[RROWS - 1] = R(1);
        S.d[0][RROWS - 1] = xnext[2 * cb + 1];
      }
      __syncthreads();
    }
    pcr<R, 1>(S);
    const R xf = S.d[0][2 * t] / S.b[2 * t];
    const R xl = S.d[0][2 * t + 1] / S.b[2 * t + 1];
    const R det = q.d[1] * q.d[2] - q.u[1] * q.u[1];
    const R r1 = q.b[1] - q.u[0] * xf, r2 = q.b[2] - q.u[2] * xl;
    const R x1 = (q.d[2] * r1 - q.u[1] * r2) / det;
    const R x2 = (q.d[1] * r2 - q.u[1] * r1) / det;
    const int r = row0 + 4 * t;
    if (r < n) x[r] = xf;
    if (r + 1 < n) x[r + 1] = x1;
    if (r + 2 < n) x[r + 2] = x2;
    if (r + 3 < n) x[r + 3] = xl;
    __syncthreads();  // S is rewritten by the next chunk
  }
}

}  // namespace

// blocks of a level: the row count lives on the device and the host only
// knows its bound, so a block walks several chunks rather than the grid
// holding one block per possible chunk (most of which would only load the
// count and exit)
static int tri_grid(int64_t nmax) {
  const int64_t b = (nmax + TRI_ROWS - 1) / TRI_ROWS;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

template <typename R>
void launch_tri_solve(const TriLevels<R>& T, const int* n0, const int* conv, hipStream_t s) {
  // n of level 0 lives with the caller; levels >= 1 in T.n
  const int* nl[TRI_MAX_LEVELS];
  nl[0] = n0;
  for (int l = 1; l < T.nlev; l++) nl[l] = T.n + l;
  for (int l = 0; l + 1 < T.nlev; l++) {
    const int blocks = tri_grid(T.nmax[l]);
    hipLaunchKernelGGL(k_tri_reduce<R>, dim3(blocks), dim3(TPB), 0, s, T.dg[l], T.up[l], T.rh[l],
                       nl[l], T.dg[l + 1], T.up[l + 1], T.rh[l + 1], T.n + l + 1, conv);
  }
  const int top = T.nlev - 1;
  hipLaunchKernelGGL(k_tri_solve<R>, dim3(1), dim3(TPB), 0, s, T.dg[top], T.up[top], T.rh[top],
                     nl[top], (const R*)nullptr, T.x[top], conv);
  for (int l = T.nlev - 2; l >= 0; l--) {
    const int blocks = tri_grid(T.nmax[l]);
    hipLaunchKernelGGL(k_tri_solve<R>, dim3(blocks), dim3(TPB), 0, s, T.dg[l], T.up[l], T.rh[l],
                       nl[l], (const R*)T.x[l + 1], T.x[l], conv);
  }
}

template void launch_tri_solve<double>(const TriLevels<double>&, const int*, const int*,
                                       hipStream_t);
template void launch_tri_solve<float>(const TriLevels<float>&, const int*, const int*,
                                      hipStream_t);

// ---------------------------------------------------------------------------
// FP64 residual and FP32 refinement of the packed 1D system
// ---------------------------------------------------------------------------
namespace {
constexpr int RB = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += sh[w];
  return s;
}

__global__ void __launch_bounds__(RB) k_resid1d(const double* __restrict__ dg,
                                                const double* __restrict__ up,
                                                const double* __restrict__ rh,
                                                const double* __restrict__ x, const int* n_in,
                                                float* __restrict__ r32, double* part, int with_b,
                                                double* part_b, const int* conv) {
  if (conv && *conv) return;
  __shared__ double sh[RB / 64];
  const int n = *n_in;
  double rr = 0.0, bb = 0.0;
  for (int k = blockIdx.x * RB + threadIdx.x; k < n; k += gridDim.x * RB) {
    double ax = 0.0;  // x == nullptr stands for x = 0
    if (x) {
      ax = dg[k] * x[k];
      if (k > 0) ax += up[k - 1] * x[k - 1];
      if (k + 1 < n) ax += up[k] * x[k + 1];
    }
    const double r = rh[k] - ax;
    if (r32) r32[k] = (float)r;
    rr += r * r;
    if (with_b) bb += rh[k] * rh[k];
  }
  const double s = block_sum(rr, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  if (with_b) {
    __syncthreads();
    const double sb = block_sum(bb, sh);
    if (threadIdx.x == 0) part_b[blockIdx.x] = sb;
  }
}

// fixed-order sum of the block partials -> relative residual and convergence
__global__ void k_resid_final(const double* part, const double* part_b, int nparts, int sweep,
                              double tol, double* norms, double* rel, int* iters, int* conv,
                              int is_first) {
  if (conv && *conv && !is_first) return;
  // one wavefront: strided partial sums, then a shuffle reduction
  double rr = 0.0, bsum = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) {
    rr += part[i];
    if (part_b) bsum += part_b[i];
  }
  rr = wave_sum(rr);
  bsum = wave_sum(bsum);
  if (threadIdx.x != 0) return;
  if (part_b) norms[1] = bsum;
  norms[0] = rr;
  const double bb = norms[1];
  const double r = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  *rel = r;
  if (iters) *iters = sweep;
  if (conv) *conv = (r <= tol) ? 1 : 0;
}

__global__ void __launch_bounds__(RB) k_refine_update(const float* __restrict__ e,
                                                      double* __restrict__ x, const int* n_in,
                                                      int first, const int* conv) {
  if (conv && *conv) return;
  const int n = *n_in;
  for (int k = blockIdx.x * RB + threadIdx.x; k < n; k += gridDim.x * RB)
    x[k] = first ? (double)e[k] : x[k] + (double)e[k];
}

__global__ void __launch_bounds__(RB) k_cast_sys(const double* __restrict__ dg,
                                                 const double* __restrict__ up,
                                                 const double* __restrict__ rh, const int* n_in,
                                                 float* __restrict__ dg32,
                                                 float* __restrict__ up32,
                                                 float* __restrict__ rh32) {
  const int n = *n_in;
  for (int k = blockIdx.x * RB + threadIdx.x; k < n; k += gridDim.x * RB) {
    dg32[k] = (float)dg[k];
    up32[k] = (float)up[k];
    rh32[k] = (float)rh[k];
  }
}

__global__ void k_flag_noconv(const int* conv, int* status) {
  if (threadIdx.x == 0 && !*conv) atomicOr(status, ST_NOCONV);
}
}  // namespace

int resid_blocks(int64_t max_rows) {
  int64_t b = (max_rows + RB - 1) / RB;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_resid1d(const double* dg, const double* up, const double* rh, const double* x,
                    const int* n, int64_t max_rows, float* r32, double* part, int with_b,
                    double* part_b, const int* conv, hipStream_t s) {
  hipLaunchKernelGGL(k_resid1d, dim3(resid_blocks(max_rows)), dim3(RB), 0, s, dg, up, rh, x, n,
                     r32, part, with_b, part_b, conv);
}

void launch_resid_final(const double* part, const double* part_b, int nparts, int sweep,
                        double tol, double* norms, double* rel, int* iters, int* conv,
                        int is_first, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(64), 0, s, part, part_b, nparts, sweep, tol,
                     norms, rel, iters, conv, is_first);
}

void launch_refine_update(const float* e, double* x, const int* n, int64_t max_rows, int first,
                          const int* conv, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_update, dim3(resid_blocks(max_rows)), dim3(RB), 0, s, e, x, n,
                     first, conv);
}

void launch_cast_sys(const double* dg, const double* up, const double* rh, const int* n,
                     int64_t max_rows, float* dg32, float* up32, float* rh32, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_sys, dim3(resid_blocks(max_rows)), dim3(RB), 0, s, dg, up, rh, n,
                     dg32, up32, rh32);
}

void launch_flag_noconv(const int* conv, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_noconv, dim3(1), dim3(64), 0, s, conv, status);
}

}  // namespace swenh
