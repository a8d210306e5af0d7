// swe_nh_2d.hip -- 2D kernels of the non-hydrostatic SWE step (gfx950).
//
// Grid [ny][nx], x fastest, tiles of TX2 x TY2 cells (one block of 256
// threads per tile).  Walls on all four sides: reflected ghosts (the normal
// momentum changes sign), zero Dirichlet data for the NH pressure.
//
//   k_speed2d      max (|u| + c)/dx + (|v| + c)/dy and state checks -> dt
//   k_pred2d       both Heun stages of the unsplit hydrostatic FV operator in
//                  LDS (4-cell halo); face fluxes computed once per direction
//   k_mask2d       criterion + (2e+1)^2 box enlargement, tile counts
//   k_tiles2d      list of tiles holding marked cells
//   k_assemble2d   5-point (or exact-tensor 7-point) operator of the elliptic
//                  system (FP64 + FP32 copy)
//   k_pcg2d<R>     persistent CG preconditioned by tile-block symmetric
//                  red-black SOR (pipelined form when each block owns one
//                  tile, Chronopoulos-Gear otherwise), in precision R with
//                  FP64 residuals and FP64 refinement of the solution,
//                  deterministic fixed-order dot products, arrival-counter
//                  grid barrier, bounded waits
//   k_correct2d    projection of hu, hv and hw on the marked cells
#include "swe_nh_2d.h"
#include "swe_nh_cnn.h"
#include "swe_nh_common.h"

namespace swenh {

namespace {

constexpr int NT2 = 256;
constexpr int H2 = 4;
constexpr int WX = TX2 + 2 * H2, WY = TY2 + 2 * H2, WN = WX * WY;
constexpr int R1X = TX2 + 4, R1Y = TY2 + 4, R1N = R1X * R1Y;
constexpr int NFACE = ((R1X + 1) * R1Y > R1X * (R1Y + 1)) ? (R1X + 1) * R1Y : R1X * (R1Y + 1);
constexpr int NTP = 512;  // threads of the predictor kernel
constexpr int QMAX = (R1N + NTP - 1) / NTP;
// slope cells of one direction of a stage: the region widened by one cell
// across the faces' direction
constexpr int NSLOPE = ((R1X + 2) * R1Y > R1X * (R1Y + 2)) ? (R1X + 2) * R1Y : R1X * (R1Y + 2);
constexpr int TN = TX2 * TY2;
constexpr int MAXE2 = 64;

struct G2 {
  int nx, ny, tiles_x;
  double dx, dy, g, rho, cfl, dt_fixed, k_nh;
  int crit, enlarge, first_global;
  int tensor;  // the exact-tensor (7-point) elliptic operator
  const double* ds;
  const Chan* ch;
  double* t;
  double* dt;
  unsigned long long* smax;
  double* tspeed;  // [ntiles] max speed term of each tile's new state
  int* status;
  int* step;
};

G2 make_g2(const swe_nh_config* c, const Ctx2D* x) {
  G2 g;
  g.nx = c->nx;
  g.ny = c->ny;
  g.tiles_x = x->tiles_x;
  g.dx = c->dx;
  g.dy = c->dy;
  g.g = c->g;
  g.rho = c->rho;
  g.cfl = c->cfl;
  g.dt_fixed = c->dt_fixed;
  g.k_nh = c->k_nh;
  g.crit = c->crit;
  g.enlarge = c->enlarge;
  g.first_global = c->first_global;
  g.tensor = c->tensor2d;
  g.ds = c->depth_static;
  g.ch = x->ch;
  g.t = x->t;
  g.dt = x->dt;
  g.smax = x->smax;
  g.tspeed = x->tspeed;
  g.status = x->status;
  g.step = x->step;
  return g;
}

__device__ __forceinline__ double depth2(const G2& G, const Chan& c, const Motion& M, int i,
                                         int j) {
  const double x = (i + 0.5) * G.dx, y = (j + 0.5) * G.dy;
  return G.ds[(int64_t)j * G.nx + i] - body_B(c, x - M.X, y - c.y0);
}

// ---------------------------------------------------------------------------
// wave speed
// ---------------------------------------------------------------------------
// Each tile keeps the largest (|u| + c)/dx + (|v| + c)/dy of its state in
// tspeed[tile] (plain stores by the block that owns the tile: the step's mask
// pass for the unmarked cells, the projection for the marked ones); one block
// reduces the tiles at the end of the step.  Thousands of blocks taking the
// maximum on one address would serialise on it.

// one cell's speed term (s) and state checks (flags)
__device__ __forceinline__ void cell_speed2d(const G2& G, double idx, double idy, double hh,
                                             double m, double n, double k, double& s,
                                             int& flags) {
  if (!isfinite(hh) || !isfinite(m) || !isfinite(n) || !isfinite(k)) {
    flags |= ST_NAN;
  } else if (!(hh > 0.0)) {
    flags |= ST_DRY;
  } else {
    const double a = sqrt64(G.g * hh), r = rcp64(hh);
    s = fmax(s, (fabs(m * r) + a) * idx + (fabs(n * r) + a) * idy);
  }
}

// block maximum of s into *slot (max with its value when combine), flags into
// the status word
__device__ void flush_tile_speed(const G2& G, double* slot, double s, int flags, bool combine) {
  __shared__ double red[NT2 / 64];
  __shared__ int fl;
  s = wave_max(s);
  if (threadIdx.x == 0) fl = 0;
  __syncthreads();
  if (flags) atomicOr(&fl, flags);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < NT2 / 64; w++) m = fmax(m, red[w]);
    *slot = combine ? fmax(m, *slot) : m;
    if (fl) atomicOr(G.status, fl);
  }
}

__global__ void __launch_bounds__(NT2) k_speed2d(G2 G, const double* __restrict__ h,
                                                 const double* __restrict__ hu,
                                                 const double* __restrict__ hv,
                                                 const double* __restrict__ hw) {
  const int i0 = (blockIdx.x % G.tiles_x) * TX2, j0 = (blockIdx.x / G.tiles_x) * TY2;
  const double idx = 1.0 / G.dx, idy = 1.0 / G.dy;
  double s = 0.0;
  int flags = 0;
  for (int c = threadIdx.x; c < TN; c += NT2) {
    const int i = i0 + c % TX2, j = j0 + c / TX2;
    if (i >= G.nx || j >= G.ny) continue;
    const int64_t o = (int64_t)j * G.nx + i;
    cell_speed2d(G, idx, idy, h[o], hu[o], hv[o], hw[o], s, flags);
  }
  flush_tile_speed(G, &G.tspeed[blockIdx.x], s, flags, false);
}

// maximum over the tiles -> *smax; with advance, also the end of a step:
// t += dt and the step counter
__global__ void __launch_bounds__(1024) k_speed_reduce2d(G2 G, int ntiles, int advance) {
  __shared__ double red[1024 / 64];
  double m = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += 1024) m = fmax(m, G.tspeed[t]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < 1024 / 64; w++) r = fmax(r, red[w]);
    *G.smax = pos_bits(r);
    if (advance) {
      G.t[0] += G.dt[0];
      *G.step += 1;
    }
  }
}

// ---------------------------------------------------------------------------
// predictor
// ---------------------------------------------------------------------------
struct Flux2 {
  double Fh, FmL, FmR, Ft1, Ft2;
  bool dry;
};

// Rusanov flux across a face with normal momentum m and tangential
// momenta a, b, hydrostatic reconstruction of the bed (Audusse et al. 2004)
__device__ __forceinline__ Flux2 rusanov2d(double g, double eL, double mL, double aL, double bL,
                                           double dL, double eR, double mR, double aR, double bR,
                                           double dR) {
  Flux2 f;
  const double hL = eL + dL, hR = eR + dR;
  f.dry = !(hL > 0.0) || !(hR > 0.0);
  const double rL = rcp64(hL), rR = rcp64(hR);
  const double uL = mL * rL, uR = mR * rR;
  const double vL = aL * rL, vR = aR * rR;
  const double wL = bL * rL, wR = bR * rR;
  const double db = fmin(dL, dR);
  const double sL = fmax(0.0, eL + db), sR = fmax(0.0, eR + db);
  const double lam = fmax(fabs(uL) + sqrt64(g * sL), fabs(uR) + sqrt64(g * sR));
  const double qL = sL * uL, qR = sR * uR;
  f.Fh = 0.5 * (qL + qR) - 0.5 * lam * (sR - sL);
  const double Fm = 0.5 * (qL * uL + 0.5 * g * sL * sL + qR * uR + 0.5 * g * sR * sR) -
                    0.5 * lam * (qR - qL);
  f.FmL = Fm + 0.5 * g * (hL * hL - sL * sL);
  f.FmR = Fm + 0.5 * g * (hR * hR - sR * sR);
  f.Ft1 = 0.5 * (qL * vL + qR * vR) - 0.5 * lam * (sR * vR - sL * vL);
  f.Ft2 = 0.5 * (qL * wL + qR * wR) - 0.5 * lam * (sR * wR - sL * wL);
  return f;
}

struct P2 {
  double e[WN], m[WN], n[WN], k[WN], d0[WN], d1[WN];
  // minmod slopes of one direction (eta, normal and tangential momentum, hw,
  // depth) on the slope cells, then, in the same space, the face fluxes
  union {
    double sl[5][NSLOPE];
    double F[5][NFACE];
  } u;
};

__device__ __forceinline__ int W(int i, int j) { return j * WX + i; }

// L of one stage on the region of RXs x RYs cells at window offset O; the
// thread's cells are region cells r = threadIdx.x + NTP q (stage 1 layout);
// only cells with `want` set are evaluated.  Per direction: the minmod
// slopes of every cell once, the face fluxes from the cells' reconstructed
// values, then each cell's update from its two faces.
template <int RXs, int RYs, int O>
__device__ void stage2d(P2& S, const double* d, const G2& G, int i0, int j0, double (&L)[QMAX][4],
                        int* flags) {
  const double idx = 1.0 / G.dx, idy = 1.0 / G.dy;
  const int wi0 = i0 - H2, wj0 = j0 - H2;  // domain coords of window cell (0, 0)
  auto dom = [&](int wi, int wj) {
    const int i = wi0 + wi, j = wj0 + wj;
    return i >= 0 && i < G.nx && j >= 0 && j < G.ny;
  };
  auto inreg = [&](int wi, int wj) {
    return wi >= O && wi < O + RXs && wj >= O && wj < O + RYs;
  };
  constexpr int FPT = ((RXs + 1) * RYs > RXs * (RYs + 1) ? (RXs + 1) * RYs : RXs * (RYs + 1));
  constexpr int FQ = (FPT + NTP - 1) / NTP;  // faces per thread
#pragma unroll
  for (int dir = 0; dir < 2; dir++) {
    const bool xd = dir == 0;
    const int s = xd ? 1 : WX;
    const double* nm = xd ? S.m : S.n;  // normal momentum
    const double* t1 = xd ? S.n : S.m;  // tangential momentum
    // slope cells: xd: (RXs + 2) x RYs from (O - 1, O); else RXs x (RYs + 2) from (O, O - 1)
    const int SX = xd ? RXs + 2 : RXs, SY = xd ? RYs : RYs + 2;
    const int sw0 = xd ? W(O - 1, O) : W(O, O - 1);
    for (int c = threadIdx.x; c < SX * SY; c += NTP) {
      const int w = sw0 + (c / SX) * WX + c % SX;
      S.u.sl[0][c] = minmod(S.e[w] - S.e[w - s], S.e[w + s] - S.e[w]);
      S.u.sl[1][c] = minmod(nm[w] - nm[w - s], nm[w + s] - nm[w]);
      S.u.sl[2][c] = minmod(t1[w] - t1[w - s], t1[w + s] - t1[w]);
      S.u.sl[3][c] = minmod(S.k[w] - S.k[w - s], S.k[w + s] - S.k[w]);
      S.u.sl[4][c] = minmod(d[w] - d[w - s], d[w + s] - d[w]);
    }
    __syncthreads();
    // faces: xd: (RXs + 1) x RYs, face fi between region cells fi - 1 and fi
    const int NF = xd ? (RXs + 1) * RYs : RXs * (RYs + 1);
    double fv[FQ][5];
#pragma unroll
    for (int q = 0; q < FQ; q++) {
      const int f = threadIdx.x + NTP * q;
      if (f >= NF) continue;
      int wl, cl;  // window cell and slope cell left of (below) the face
      if (xd) {
        const int fi = f % (RXs + 1), rj = f / (RXs + 1);
        wl = W(O + fi - 1, O + rj);
        cl = rj * SX + fi;
      } else {
        const int ri = f % RXs, fj = f / RXs;
        wl = W(O + ri, O + fj - 1);
        cl = fj * SX + ri;
      }
      const int wr = wl + s, cr = cl + (xd ? 1 : SX);
      const double eL = S.e[wl] + 0.5 * S.u.sl[0][cl], dL = d[wl] + 0.5 * S.u.sl[4][cl];
      const double eR = S.e[wr] - 0.5 * S.u.sl[0][cr], dR = d[wr] - 0.5 * S.u.sl[4][cr];
      Flux2 F = rusanov2d(G.g, eL, nm[wl] + 0.5 * S.u.sl[1][cl], t1[wl] + 0.5 * S.u.sl[2][cl],
                          S.k[wl] + 0.5 * S.u.sl[3][cl], dL, eR, nm[wr] - 0.5 * S.u.sl[1][cr],
                          t1[wr] - 0.5 * S.u.sl[2][cr], S.k[wr] - 0.5 * S.u.sl[3][cr], dR);
      // the centred bed source g h (d slope) / 2 of each side's cell with its
      // reconstructed depth at this face: a cell's normal-momentum update is
      // then the difference of its two faces' values
      fv[q][0] = F.Fh;
      fv[q][1] = F.FmL - 0.5 * G.g * (eL + dL) * S.u.sl[4][cl];
      fv[q][2] = F.FmR + 0.5 * G.g * (eR + dR) * S.u.sl[4][cr];
      fv[q][3] = F.Ft1;
      fv[q][4] = F.Ft2;
      if (F.dry) {
        const int li = (wl % WX), lj = (wl / WX), ri2 = (wr % WX), rj2 = (wr / WX);
        const bool used = (inreg(li, lj) && dom(li, lj)) || (inreg(ri2, rj2) && dom(ri2, rj2));
        if (used) *flags |= ST_DRY;
      }
    }
    __syncthreads();  // the slopes are read: the fluxes take their space
#pragma unroll
    for (int q = 0; q < FQ; q++) {
      const int f = threadIdx.x + NTP * q;
      if (f >= NF) continue;
#pragma unroll
      for (int v = 0; v < 5; v++) S.u.F[v][f] = fv[q][v];
    }
    __syncthreads();
    const double id = xd ? idx : idy;
#pragma unroll
    for (int q = 0; q < QMAX; q++) {
      const int r = threadIdx.x + NTP * q;
      if (r >= R1N) break;
      const int wi = 2 + r % R1X, wj = 2 + r / R1X;  // stage-1 layout
      if (!inreg(wi, wj)) continue;
      const int ri = wi - O, rj = wj - O;
      const int fl = xd ? rj * (RXs + 1) + ri : rj * RXs + ri;
      const int fr = fl + (xd ? 1 : RXs);
      const double a0 = -(S.u.F[0][fr] - S.u.F[0][fl]) * id;
      const double an = -(S.u.F[1][fr] - S.u.F[2][fl]) * id;  // normal momentum
      const double at = -(S.u.F[3][fr] - S.u.F[3][fl]) * id;  // tangential
      const double ak = -(S.u.F[4][fr] - S.u.F[4][fl]) * id;
      if (xd) {
        L[q][0] = a0;
        L[q][1] = an;
        L[q][2] = at;
        L[q][3] = ak;
      } else {
        L[q][0] += a0;
        L[q][2] += an;
        L[q][1] += at;
        L[q][3] += ak;
      }
    }
    __syncthreads();
  }
}

// The workgroups of a launch go to the 8 XCDs in turn (workgroup b to XCD
// b % 8), each with its own L2.  Tile of workgroup b such that every XCD
// walks one contiguous band of the row-major tiles: the neighbours whose
// windows overlap a tile's (the next tile along x, the tile row above) are
// then read through the same L2.  A bijection of [0, n) for any n.
__device__ __forceinline__ int xcd_band_tile(int b, int n) {
  constexpr int NX = 8;
  const int x = b % NX, k = b / NX, per = n / NX, rem = n % NX;
  return x * per + min(x, rem) + k;
}

__global__ void __launch_bounds__(NTP) k_pred2d(G2 G, const double* __restrict__ h,
                                                const double* __restrict__ hu,
                                                const double* __restrict__ hv,
                                                const double* __restrict__ hw,
                                                double* __restrict__ ht, double* __restrict__ mt,
                                                double* __restrict__ nt, double* __restrict__ kt,
                                                const double* t_in, const double* dt_in,
                                                int dt_from_speed) {
  __shared__ P2 S;
  __shared__ int sflags;
  const Chan c = G.ch[0];
  const int tb = xcd_band_tile(blockIdx.x, gridDim.x);
  const int i0 = (tb % G.tiles_x) * TX2, j0 = (tb / G.tiles_x) * TY2;
  const int wi0 = i0 - H2, wj0 = j0 - H2;
  const double t0 = t_in[0];
  double dt;
  if (dt_from_speed) {
    dt = (G.cfl > 0.0) ? G.cfl / __longlong_as_double((long long)*G.smax) : G.dt_fixed;
    if (blockIdx.x == 0 && threadIdx.x == 0) G.dt[0] = dt;
  } else {
    dt = dt_in[0];
  }
  const Motion M0 = body_motion(c, t0), M1 = body_motion(c, t0 + dt);
  if (threadIdx.x == 0) sflags = 0;
  int flags = 0;
  for (int w = threadIdx.x; w < WN; w += NTP) {
    const int ii = wi0 + w % WX, jj = wj0 + w / WX;
    const int si = reflect(min(max(ii, -H2), G.nx + H2 - 1), G.nx);
    const int sj = reflect(min(max(jj, -H2), G.ny + H2 - 1), G.ny);
    const int64_t o = (int64_t)sj * G.nx + si;
    const double a0 = depth2(G, c, M0, si, sj), a1 = depth2(G, c, M1, si, sj);
    S.e[w] = h[o] - a0;
    S.m[w] = (si == ii ? 1.0 : -1.0) * hu[o];
    S.n[w] = (sj == jj ? 1.0 : -1.0) * hv[o];
    S.k[w] = hw[o];
    S.d0[w] = a0;
    S.d1[w] = a1;
  }
  __syncthreads();
  double Qn[QMAX][4], L1[QMAX][4], L2[QMAX][4];
#pragma unroll
  for (int q = 0; q < QMAX; q++)
#pragma unroll
    for (int v = 0; v < 4; v++) Qn[q][v] = L1[q][v] = L2[q][v] = 0.0;
  stage2d<R1X, R1Y, 2>(S, S.d0, G, i0, j0, L1, &flags);
  // Q* = Q^n + dt L(Q^n) on the stage-1 region, then ghosts reflected from Q*
#pragma unroll
  for (int q = 0; q < QMAX; q++) {
    const int r = threadIdx.x + NTP * q;
    if (r >= R1N) break;
    const int wi = 2 + r % R1X, wj = 2 + r / R1X, w = W(wi, wj);
    const int i = wi0 + wi, j = wj0 + wj;
    if (i < 0 || i >= G.nx || j < 0 || j >= G.ny) continue;
    Qn[q][0] = S.e[w] + S.d0[w];
    Qn[q][1] = S.m[w];
    Qn[q][2] = S.n[w];
    Qn[q][3] = S.k[w];
    S.e[w] = Qn[q][0] + dt * L1[q][0] - S.d1[w];
    S.m[w] = Qn[q][1] + dt * L1[q][1];
    S.n[w] = Qn[q][2] + dt * L1[q][2];
    S.k[w] = Qn[q][3] + dt * L1[q][3];
  }
  __syncthreads();
  for (int r = threadIdx.x; r < R1N; r += NTP) {
    const int wi = 2 + r % R1X, wj = 2 + r / R1X, w = W(wi, wj);
    const int i = wi0 + wi, j = wj0 + wj;
    if (i >= 0 && i < G.nx && j >= 0 && j < G.ny) continue;
    const int si = reflect(min(max(i, -H2), G.nx + H2 - 1), G.nx);
    const int sj = reflect(min(max(j, -H2), G.ny + H2 - 1), G.ny);
    const int swi = si - wi0, swj = sj - wj0;
    double ev = 0.0, mv = 0.0, nv = 0.0, kv = 0.0;
    if (swi >= 2 && swi < 2 + R1X && swj >= 2 && swj < 2 + R1Y) {
      const int sw = W(swi, swj);
      ev = S.e[sw];
      mv = (si == i ? 1.0 : -1.0) * S.m[sw];
      nv = (sj == j ? 1.0 : -1.0) * S.n[sw];
      kv = S.k[sw];
    }
    S.e[w] = ev;
    S.m[w] = mv;
    S.n[w] = nv;
    S.k[w] = kv;
  }
  __syncthreads();
  stage2d<TX2, TY2, H2>(S, S.d1, G, i0, j0, L2, &flags);
#pragma unroll
  for (int q = 0; q < QMAX; q++) {
    const int r = threadIdx.x + NTP * q;
    if (r >= R1N) break;
    const int wi = 2 + r % R1X, wj = 2 + r / R1X;
    if (wi < H2 || wi >= H2 + TX2 || wj < H2 || wj >= H2 + TY2) continue;
    const int i = wi0 + wi, j = wj0 + wj;
    if (i >= G.nx || j >= G.ny) continue;
    const int64_t o = (int64_t)j * G.nx + i;
    ht[o] = Qn[q][0] + 0.5 * dt * (L1[q][0] + L2[q][0]);
    mt[o] = Qn[q][1] + 0.5 * dt * (L1[q][1] + L2[q][1]);
    nt[o] = Qn[q][2] + 0.5 * dt * (L1[q][2] + L2[q][2]);
    kt[o] = Qn[q][3] + 0.5 * dt * (L1[q][3] + L2[q][3]);
  }
  if (flags) atomicOr(&sflags, flags);
  __syncthreads();
  if (threadIdx.x == 0 && sflags) atomicOr(G.status, sflags);
}

// ---------------------------------------------------------------------------
// criterion and enlargement
// ---------------------------------------------------------------------------
__device__ double indicator2d(const G2& G, const Chan& c, const Motion& M, const double* ht,
                              const double* mt, const double* nt, const double* kt, int i, int j) {
  const int nx = G.nx, ny = G.ny;
  const int il = reflect(i - 1, nx), ir = reflect(i + 1, nx);
  const int jl = reflect(j - 1, ny), jr = reflect(j + 1, ny);
  const double sxl = (il == i - 1) ? 1.0 : -1.0, sxr = (ir == i + 1) ? 1.0 : -1.0;
  const double syl = (jl == j - 1) ? 1.0 : -1.0, syr = (jr == j + 1) ? 1.0 : -1.0;
  auto O = [&](int a, int b) { return (int64_t)b * nx + a; };
  const int64_t o = O(i, j);
  switch (G.crit) {
    case SWE_NH_CRIT_ETA_D: {
      const double d = depth2(G, c, M, i, j);
      return fabs((ht[o] - d) / d);
    }
    case SWE_NH_CRIT_ETA_X: {
      const double ex = ((ht[O(ir, j)] - depth2(G, c, M, ir, j)) -
                         (ht[O(il, j)] - depth2(G, c, M, il, j))) / (2.0 * G.dx);
      const double ey = ((ht[O(i, jr)] - depth2(G, c, M, i, jr)) -
                         (ht[O(i, jl)] - depth2(G, c, M, i, jl))) / (2.0 * G.dy);
      return sqrt(ex * ex + ey * ey);
    }
    case SWE_NH_CRIT_U: {
      const double u = mt[o] / ht[o], v = nt[o] / ht[o];
      return sqrt(u * u + v * v);
    }
    case SWE_NH_CRIT_U_X: {
      const double ux = (sxr * mt[O(ir, j)] / ht[O(ir, j)] - sxl * mt[O(il, j)] / ht[O(il, j)]) /
                        (2.0 * G.dx);
      const double uy = (mt[O(i, jr)] / ht[O(i, jr)] - mt[O(i, jl)] / ht[O(i, jl)]) / (2.0 * G.dy);
      const double vx = (nt[O(ir, j)] / ht[O(ir, j)] - nt[O(il, j)] / ht[O(il, j)]) / (2.0 * G.dx);
      const double vy = (syr * nt[O(i, jr)] / ht[O(i, jr)] - syl * nt[O(i, jl)] / ht[O(i, jl)]) /
                        (2.0 * G.dy);
      return sqrt(ux * ux + uy * uy + vx * vx + vy * vy);
    }
    case SWE_NH_CRIT_W:
      return fabs(kt[o] / ht[o]);
    default: {
      const double wx = (kt[O(ir, j)] / ht[O(ir, j)] - kt[O(il, j)] / ht[O(il, j)]) / (2.0 * G.dx);
      const double wy = (kt[O(i, jr)] / ht[O(i, jr)] - kt[O(i, jl)] / ht[O(i, jl)]) / (2.0 * G.dy);
      return sqrt(wx * wx + wy * wy);
    }
  }
}

__global__ void __launch_bounds__(NT2) k_mask2d(G2 G, const double* __restrict__ ht,
                                                const double* __restrict__ mt,
                                                const double* __restrict__ nt,
                                                const double* __restrict__ kt, const double* t_in,
                                                const double* dt_in, int mode_override,
                                                uint8_t* __restrict__ mask, int* tile_cnt,
                                                double* h, double* hu, double* hv, double* hw,
                                                double* p, int write_state) {
  __shared__ uint8_t raw[(TX2 + 2 * MAXE2) * (TY2 + 2 * MAXE2)];
  __shared__ uint8_t rowor[TX2 * (TY2 + 2 * MAXE2)];
  __shared__ int cnt[NT2 / 64];
  const Chan c = G.ch[0];
  const int i0 = (blockIdx.x % G.tiles_x) * TX2, j0 = (blockIdx.x / G.tiles_x) * TY2;
  const int e = G.enlarge;
  int mode = mode_override;
  if (mode < 0) {
    const bool wcrit = (G.crit == SWE_NH_CRIT_W || G.crit == SWE_NH_CRIT_W_X);
    if (G.crit == SWE_NH_CRIT_GLOBAL || (wcrit && G.first_global && *G.step == 0))
      mode = 1;
    else if (G.crit == SWE_NH_CRIT_NONE)
      mode = 2;
    else
      mode = 0;
  }
  const int RW = TX2 + 2 * e, RH = TY2 + 2 * e;
  if (mode == 0) {
    const Motion M = body_motion(c, t_in[0] + dt_in[0]);
    for (int w = threadIdx.x; w < RW * RH; w += NT2) {
      const int i = i0 - e + w % RW, j = j0 - e + w / RW;
      uint8_t r = 0;
      if (i >= 0 && i < G.nx && j >= 0 && j < G.ny)
        r = indicator2d(G, c, M, ht, mt, nt, kt, i, j) > G.k_nh;
      raw[w] = r;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < TX2 * RH; w += NT2) {
      const int ti = w % TX2, rj = w / TX2;
      uint8_t v = 0;
      for (int a = 0; a <= 2 * e; a++) v |= raw[rj * RW + ti + a];
      rowor[w] = v;
    }
    __syncthreads();
  }
  int local = 0;
  const double idx = 1.0 / G.dx, idy = 1.0 / G.dy;
  double sp = 0.0;
  int flags = 0;
  for (int cc = threadIdx.x; cc < TN; cc += NT2) {
    const int ti = cc % TX2, tj = cc / TX2;
    const int i = i0 + ti, j = j0 + tj;
    if (i >= G.nx || j >= G.ny) continue;
    uint8_t v;
    if (mode == 1) {
      v = 1;
    } else if (mode == 2) {
      v = 0;
    } else {
      v = 0;
      for (int a = 0; a <= 2 * e; a++) v |= rowor[(tj + a) * TX2 + ti];
    }
    const int64_t o = (int64_t)j * G.nx + i;
    mask[o] = v;
    local += v;
    if (write_state) {
      const double hh = ht[o], mm = mt[o], nn = nt[o], kk = kt[o];
      h[o] = hh;
      hu[o] = mm;
      hv[o] = nn;
      hw[o] = kk;
      if (!v) {
        p[o] = 0.0;
        cell_speed2d(G, idx, idy, hh, mm, nn, kk, sp, flags);  // final: no projection follows
      }
    }
  }
  if (write_state) flush_tile_speed(G, &G.tspeed[blockIdx.x], sp, flags, false);
  local = wave_sum_i(local);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < NT2 / 64; w++) s += cnt[w];
    tile_cnt[blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(NT2) k_count2d(G2 G, const uint8_t* __restrict__ mask,
                                                 int* tile_cnt) {
  __shared__ int cnt[NT2 / 64];
  const int i0 = (blockIdx.x % G.tiles_x) * TX2, j0 = (blockIdx.x / G.tiles_x) * TY2;
  int local = 0;
  for (int cc = threadIdx.x; cc < TN; cc += NT2) {
    const int i = i0 + cc % TX2, j = j0 + cc / TX2;
    if (i < G.nx && j < G.ny) local += mask[(int64_t)j * G.nx + i] ? 1 : 0;
  }
  local = wave_sum_i(local);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < NT2 / 64; w++) s += cnt[w];
    tile_cnt[blockIdx.x] = s;
  }
}

// list of tiles holding marked cells, in tile order; total marked cells
__global__ void __launch_bounds__(1024) k_tiles2d(const int* __restrict__ tile_cnt, int ntiles,
                                                  int* __restrict__ tile_list, int* n_list,
                                                  int* n_cells, int* __restrict__ tile_pos) {
  __shared__ int part[1024];
  __shared__ long long cells[1024];
  const int per = (ntiles + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(b + per, ntiles);
  int s = 0;
  long long cs = 0;
  for (int i = b; i < e; i++) {
    s += tile_cnt[i] > 0;
    cs += tile_cnt[i];
  }
  part[threadIdx.x] = s;
  cells[threadIdx.x] = cs;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
    const long long w = threadIdx.x >= (unsigned)o ? cells[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    cells[threadIdx.x] += w;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int i = b; i < e; i++) {
    const bool on = tile_cnt[i] > 0;
    tile_pos[i] = on ? run : -1;
    if (on) tile_list[run++] = i;
  }
  if (threadIdx.x == 1023) {
    *n_list = part[1023];
    *n_cells = (int)cells[1023];
  }
}

// ---------------------------------------------------------------------------
// elliptic system (Eqs. 12-17 on the 2D grid, the diagonal part of
// S12^{-1} = (dt h / rho)(I - grad d grad d^T / alpha) on each face)
// ---------------------------------------------------------------------------
constexpr int RGX = TX2 + 2, RGY = TY2 + 2, RGN = RGX * RGY;

struct Ring {
  double h[RGN], m[RGN], n[RGN], d[RGN], Dx[RGN], Dy[RGN], phi[RGN];
};

struct Face2 {
  double K, a, b, qp, fd, Dn;  // Dn: the bottom's normal slope at the face
};

// fills the ring (tile +- 1) with the quantities the faces need
__device__ void fill_ring(Ring& R, const G2& G, const Chan& c, const Motion& M, const double* ht,
                          const double* mt, const double* nt, int i0, int j0) {
  const int nx = G.nx, ny = G.ny;
  for (int w = threadIdx.x; w < RGN; w += NT2) {
    const int ii = i0 - 1 + w % RGX, jj = j0 - 1 + w / RGX;
    const int i = reflect(min(max(ii, -1), nx), nx), j = reflect(min(max(jj, -1), ny), ny);
    auto O = [&](int a, int b) { return (int64_t)b * nx + a; };
    const int il = reflect(i - 1, nx), ir = reflect(i + 1, nx);
    const int jl = reflect(j - 1, ny), jr = reflect(j + 1, ny);
    const double d = depth2(G, c, M, i, j);
    const double dw = depth2(G, c, M, il, j), de = depth2(G, c, M, ir, j);
    const double ds_ = depth2(G, c, M, i, jl), dn = depth2(G, c, M, i, jr);
    const double Dx = (de - dw) / (2.0 * G.dx), Dy = (dn - ds_) / (2.0 * G.dy);
    const double dxx = (de - 2.0 * d + dw) / (G.dx * G.dx);
    const double dyy = (dn - 2.0 * d + ds_) / (G.dy * G.dy);
    const double dxy = (depth2(G, c, M, ir, jr) - depth2(G, c, M, ir, jl) -
                        depth2(G, c, M, il, jr) + depth2(G, c, M, il, jl)) /
                       (4.0 * G.dx * G.dy);
    const int64_t o = O(i, j);
    const double hs = ht[o];
    const double ex = ((ht[O(ir, j)] - de) - (ht[O(il, j)] - dw)) / (2.0 * G.dx);
    const double ey = ((ht[O(i, jr)] - dn) - (ht[O(i, jl)] - ds_)) / (2.0 * G.dy);
    const double u = mt[o] / hs, v = nt[o] / hs;
    const double x = (i + 0.5) * G.dx, y = (j + 0.5) * G.dy;
    const BedRate br = bed_rate(M, body_shape(c, x - M.X, y - c.y0));
    const double al = 4.0 + Dx * Dx + Dy * Dy;
    R.h[w] = hs;
    R.m[w] = (i == ii ? 1.0 : -1.0) * mt[o];
    R.n[w] = (j == jj ? 1.0 : -1.0) * nt[o];
    R.d[w] = d;
    R.Dx[w] = Dx;
    R.Dy[w] = Dy;
    R.phi[w] = G.rho * hs / al *
               (G.g * (Dx * ex + Dy * ey) - br.d_tt - 2.0 * (u * br.d_xt + v * br.d_yt) -
                (u * u * dxx + 2.0 * u * v * dxy + v * v * dyy));
  }
}

// face between ring cells l and r; xdir selects the normal
__device__ __forceinline__ Face2 face_coef(const Ring& R, const G2& G, double dt, int l, int r,
                                           bool xdir) {
  const double del = xdir ? G.dx : G.dy;
  const double hf = 0.5 * (R.h[l] + R.h[r]);
  const double Dn = (R.d[r] - R.d[l]) / del;
  const double Dt = xdir ? 0.5 * (R.Dy[l] + R.Dy[r]) : 0.5 * (R.Dx[l] + R.Dx[r]);
  const double hn = (R.h[r] - R.h[l]) / del;
  const double qf = xdir ? 0.5 * (R.m[l] + R.m[r]) : 0.5 * (R.n[l] + R.n[r]);
  const double af = 4.0 + Dn * Dn + Dt * Dt;
  const double s11 = (2.0 * hn - 3.0 * Dn) / (2.0 * hf);
  Face2 f;
  f.K = dt * hf / G.rho * (1.0 - Dn * Dn / af);
  f.a = -1.0 / del + 0.5 * s11;
  f.b = 1.0 / del + 0.5 * s11;
  f.fd = dt / G.rho * (0.5 * (R.phi[l] + R.phi[r])) * Dn;
  f.qp = qf + f.fd;
  f.Dn = Dn;
  return f;
}

// The exact-tensor operator pairs the x-face east of a cell (fx) with the
// y-face north of it (fy): the face tensor's off-diagonal entry of the pair,
// -d_x d_y / alpha times dt h / rho, taken as the geometric mean of the two
// faces' diagonal entries times the tensor's correlation of their normal
// slopes, -S_x S_y / sqrt((4 + S_x^2)(4 + S_y^2)).  That is the tensor itself
// where the faces' values agree, and |k| < sqrt(K_x K_y) always, so the
// operator stays symmetric positive definite.  A wall face has S = 0.
__device__ __forceinline__ double pair_k(const Face2& fx, const Face2& fy) {
  return -sqrt(fx.K * fy.K) * fx.Dn * fy.Dn /
         sqrt((4.0 + fx.Dn * fx.Dn) * (4.0 + fy.Dn * fy.Dn));
}

enum : uint8_t { NB_W = 1, NB_E = 2, NB_S = 4, NB_N = 8, NB_SELF = 16 };

__device__ __forceinline__ uint8_t nbr_flags(const G2& G, const uint8_t* mask, int i, int j) {
  const int64_t o = (int64_t)j * G.nx + i;
  uint8_t f = mask[o] ? NB_SELF : 0;
  if (!f) return 0;
  if (i > 0 && mask[o - 1]) f |= NB_W;
  if (i + 1 < G.nx && mask[o + 1]) f |= NB_E;
  if (j > 0 && mask[o - G.nx]) f |= NB_S;
  if (j + 1 < G.ny && mask[o + G.nx]) f |= NB_N;
  return f;
}

struct Sys2 {
  double *dg, *ce, *cn, *b, *x;
  float *dg32, *ce32, *cn32;
  uint8_t* nb;
  double* cd;  // the exact-tensor operator's coupling with (i+1, j-1), or nullptr
};

__global__ void __launch_bounds__(NT2) k_assemble2d(G2 G, const double* __restrict__ ht,
                                                    const double* __restrict__ mt,
                                                    const double* __restrict__ nt,
                                                    const double* __restrict__ kt,
                                                    const uint8_t* __restrict__ mask,
                                                    const int* tile_list, const int* n_list,
                                                    const double* t_in, const double* dt_in,
                                                    Sys2 Y, const double* p_prev, int warm) {
  if ((int)blockIdx.x >= *n_list) return;
  __shared__ Ring R;
  const int tile = tile_list[blockIdx.x];
  const int i0 = (tile % G.tiles_x) * TX2, j0 = (tile / G.tiles_x) * TY2;
  const Chan c = G.ch[0];
  const double dt = dt_in[0];
  const Motion M = body_motion(c, t_in[0] + dt);
  fill_ring(R, G, c, M, ht, mt, nt, i0, j0);
  __syncthreads();
  for (int cc = threadIdx.x; cc < TN; cc += NT2) {
    const int ti = cc % TX2, tj = cc / TX2;
    const int i = i0 + ti, j = j0 + tj;
    if (i >= G.nx || j >= G.ny) continue;
    const int64_t o = (int64_t)j * G.nx + i;
    const uint8_t nb = nbr_flags(G, mask, i, j);
    Y.nb[o] = nb;
    if (!(nb & NB_SELF)) {
      Y.dg[o] = 1.0;
      Y.ce[o] = 0.0;
      Y.cn[o] = 0.0;
      Y.b[o] = 0.0;
      Y.x[o] = 0.0;
      Y.dg32[o] = 1.0f;
      Y.ce32[o] = 0.0f;
      Y.cn32[o] = 0.0f;
      if (Y.cd) Y.cd[o] = 0.0;
      continue;
    }
    const int w = (tj + 1) * RGX + (ti + 1);
    const Face2 fw = face_coef(R, G, dt, w - 1, w, true), fe = face_coef(R, G, dt, w, w + 1, true);
    const Face2 fs = face_coef(R, G, dt, w - RGX, w, false);
    const Face2 fn = face_coef(R, G, dt, w, w + RGX, false);
    const double hs = R.h[w];
    const double x = (i + 0.5) * G.dx, y = (j + 0.5) * G.dy;
    const BedRate br = bed_rate(M, body_shape(c, x - M.X, y - c.y0));
    const double al = 4.0 + R.Dx[w] * R.Dx[w] + R.Dy[w] * R.Dy[w];
    const double s22 = 3.0 * dt / (G.rho * hs);
    const double f2 = -2.0 * br.d_t - 2.0 * kt[o] / hs -
                      (R.Dx[w] * mt[o] + R.Dy[w] * nt[o]) / (2.0 * hs) -
                      dt * al * R.phi[w] / (2.0 * G.rho * hs);
    const double dg = s22 + fw.K * fw.b * fw.b + fe.K * fe.a * fe.a + fs.K * fs.b * fs.b +
                      fn.K * fn.a * fn.a;
    const double ce = (nb & NB_E) ? fe.K * fe.a * fe.b : 0.0;
    const double cn = (nb & NB_N) ? fn.K * fn.a * fn.b : 0.0;
    // the FP32 copy (the multigrid's level 0) is the 5-point operator in both
    // forms: with the exact tensor it preconditions the 7-point operator
    Y.dg32[o] = (float)dg;
    Y.ce32[o] = (float)ce;
    Y.cn32[o] = (float)cn;
    if (G.tensor) {
      // this cell's pair (its east and north faces) adds to its diagonal and
      // to its couplings with E and N; the pair of the cell below couples
      // this cell with (i+1, j-1), stored here (the coupling with (i-1, j+1)
      // is stored at that cell)
      const double k0 = pair_k(fe, fn);
      const Face2 feS = face_coef(R, G, dt, w - RGX, w - RGX + 1, true);
      const bool se = i + 1 < G.nx && j > 0 && mask[o - G.nx + 1];
      Y.dg[o] = dg + 2.0 * k0 * fe.a * fn.a;
      Y.ce[o] = (nb & NB_E) ? ce + k0 * fn.a * fe.b : 0.0;
      Y.cn[o] = (nb & NB_N) ? cn + k0 * fe.a * fn.b : 0.0;
      Y.cd[o] = se ? pair_k(feS, fs) * feS.b * fs.b : 0.0;
    } else {
      Y.dg[o] = dg;
      Y.ce[o] = ce;
      Y.cn[o] = cn;
    }
    Y.b[o] = f2 + fw.b * fw.qp + fe.a * fe.qp + fs.b * fs.qp + fn.a * fn.qp;
    Y.x[o] = warm ? p_prev[o] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// persistent PCG with FP64 refinement
// ---------------------------------------------------------------------------
// An inner solve also ends when its recursively updated residual has not
// fallen by 10% for STALL_ITERS iterations: rounding in the recurrences
// (pipelined CG in FP32 above all) can hold it above the inner target for
// good, and the FP64 residual of the next refinement sweep then restarts it.
constexpr int STALL_ITERS = 50;

// The inner solve is pipelined CG with a tile-block preconditioner
// (symmetric red-black SOR on each tile's own block of A); see k_pcg2d.
//
// Bounded waits: a wait longer than WAIT_TICKS aborts the solve (status bit)
// so that the kernel always ends; wall_clock64 ticks at 100 MHz.
constexpr unsigned long long WAIT_TICKS = 50000000ull;
constexpr int PCG_GMAX = 1024;  // most blocks of the persistent solver

struct Bar {
  unsigned long long* count;  // arrivals, increasing over the whole solve
  int* status;
};

__device__ __forceinline__ bool aborted(const Bar& B) {
  return (__hip_atomic_load(B.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_ABORT) != 0;
}

// waits until *B.count >= target (relaxed polls, no cache maintenance per
// poll); false when the wait timed out or another block aborted
__device__ bool wait_count(const Bar& B, unsigned long long target) {
  const unsigned long long t0 = wall_clock64();
  unsigned polls = 0;
  while (__hip_atomic_load(B.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if ((++polls & 255u) == 0u) {
      if (aborted(B)) return false;
      if (wall_clock64() - t0 > WAIT_TICKS) {
        atomicOr(B.status, ST_ABORT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// grid-wide barrier over the G co-resident blocks of the solve: one arrival
// counter (release on arrival, acquire after the wait).  Barrier number k
// (1, 2, ...) completes when the counter reaches k G.  Returns false in every
// thread of the block when the solve was aborted.
__device__ bool grid_sync(const Bar& B, unsigned k, int G) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(B.count, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = wait_count(B, (unsigned long long)k * (unsigned long long)G) ? 1 : 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

// The pipelined solver publishes each value of a pass with the pass's tag
// (tagged words, put_tagged / try_tagged): a reader polls until every word
// it needs carries the tag it expects.  The values validate themselves, so a
// pass needs neither the arrival counter nor the cache write-back and
// invalidation of the barrier's fences.  Tags grow over the context's life
// (never reused while a word could still hold them).
template <typename R>
constexpr int tag_words() {
  return sizeof(R) / 4;  // 64-bit words per tagged value
}

// LDS rows for the solver's reductions: up to 9 rows of NT2 doubles, shared
// by the block partials and the grid totals (they are separated by barriers)
__device__ __forceinline__ double (*red_rows())[NT2] {
  __shared__ double rows[9][NT2];
  return rows;
}

// fixed-order sum of the first nrow rows of NT2 values in `rows`: 16 lanes
// per row each add 16 consecutive values, then a butterfly over the 16
// lanes; the sums land in out[row] (all threads synchronised on return)
__device__ __forceinline__ void sum_rows(const double (*rows)[NT2], int nrow, double* out) {
  if (threadIdx.x < nrow * 16) {
    const int k = threadIdx.x >> 4, s = threadIdx.x & 15;
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < 16; i++) a += rows[k][16 * s + i];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) a += __shfl_xor(a, o, 16);
    if (s == 0) out[k] = a;
  }
  __syncthreads();
}

// block partial sums (fixed order) of NV values -> part[v][vb]
template <int NV>
__device__ void block_partials(double (&v)[NV], double* part, int vb, int G) {
  static_assert(NV <= 4, "one wavefront sums the rows");
  double (*rows)[NT2] = red_rows();
#pragma unroll
  for (int k = 0; k < NV; k++) rows[k][threadIdx.x] = v[k];
  __syncthreads();
  if (threadIdx.x < NV * 16) {
    const int k = threadIdx.x >> 4, s = threadIdx.x & 15;
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < 16; i++) a += rows[k][16 * s + i];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) a += __shfl_xor(a, o, 16);
    if (s == 0) part[(int64_t)k * G + vb] = a;
  }
}

// The same fixed-order totals of the G partial sums in every block; with
// `on`, also the coarse correction: rows `crow` (5 rows of the coarse
// inverse, one entry per block = per active tile) times the last partial
// row (the tile sums).  Thread t adds the partials b = t, t + NT2, ...
template <int NV>
__device__ void grid_totals_rows(const double* part, int G, double (&tot)[NV], bool on,
                                 const double (*crow)[CMAX2], double (&c)[5]) {
  static_assert(NV + 5 <= 9, "reduction rows");
  __shared__ double out[NV + 5];
  double (*rows)[NT2] = red_rows();
  double a[NV + 5];
#pragma unroll
  for (int k = 0; k < NV + 5; k++) a[k] = 0.0;
  for (int b = threadIdx.x; b < G; b += NT2) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
      const double v =
          __hip_atomic_load(&part[(int64_t)k * G + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a[k] += v;
      if (k == NV - 1 && on) {
#pragma unroll
        for (int r = 0; r < 5; r++) a[NV + r] += crow[r][b] * v;
      }
    }
  }
  const int nrow = on ? NV + 5 : NV;
#pragma unroll
  for (int k = 0; k < NV + 5; k++)
    if (k < nrow) rows[k][threadIdx.x] = a[k];
  __syncthreads();
  sum_rows(rows, nrow, out);
#pragma unroll
  for (int k = 0; k < NV; k++) tot[k] = out[k];
#pragma unroll
  for (int r = 0; r < 5; r++) c[r] = on ? out[NV + r] : 0.0;
}

template <int NV>
__device__ void grid_totals(const double* part, int G, double (&tot)[NV]) {
  double c[5];
  grid_totals_rows<NV>(part, G, tot, false, nullptr, c);
}

// block_partials with tagged words: pt[(k G + vb) 2 + {0, 1}]
template <int NV>
__device__ void block_partials_tagged(double (&v)[NV], unsigned long long* pt, int vb, int G,
                                      unsigned tag) {
  static_assert(NV <= 4, "one wavefront sums the rows");
  double (*rows)[NT2] = red_rows();
#pragma unroll
  for (int k = 0; k < NV; k++) rows[k][threadIdx.x] = v[k];
  __syncthreads();
  if (threadIdx.x < NV * 16) {
    const int k = threadIdx.x >> 4, s = threadIdx.x & 15;
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < 16; i++) a += rows[k][16 * s + i];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) a += __shfl_xor(a, o, 16);
    if (s == 0) put_tagged(pt + ((int64_t)k * G + vb) * 2, a, tag);
  }
}

// partial sums of the phase that ends with barrier k: two buffers, so that a
// block already writing the next phase's partials cannot overwrite values
// another block is still reading
__device__ __forceinline__ double* part_buf(double* part, unsigned k) {
  return part + (k & 1u) * 4 * PCG_GMAX;
}

template <typename R>
struct PcgArgs {
  int nx, ny, tiles_x, tiles_y;
  const int* tile_list;
  const int* n_list;
  const int* tile_cnt;  // marked cells per tile (0: the tile holds no unknowns)
  const uint8_t* nb;
  const double *dg, *ce, *cn, *b;
  double* x;
  const R *dgR, *ceR, *cnR;
  R *r, *u, *w, *z, *q, *s, *p, *e;
  R* m[2];          // M^-1 w, double-buffered by pass parity (unused by the tagged form)
  unsigned long long* mt[2];  // tagged M^-1 w on the tiles' edge cells, by tag parity
  unsigned long long* pt;     // tagged block partials [2][4][PCG_GMAX][2], by tag parity
  unsigned* tag_base;         // first tag of the next solve
  int pipe_blocks;  // grid of the pipelined form (decides which form runs)
  const int* tile_pos;  // per tile: position in tile_list (-1: inactive)
  const double* cinv;   // (Z^T A Z)^-1 of the active tiles (coarse space), or null
  const int* cused;     // [2]: 1 when cinv is to be used
  unsigned* tflag;  // per tile: last neighbour-sync stamp passed (Chronopoulos-Gear form)
  double* part;
  Bar bar;
  int* iters;
  long long* iters_sum;  // iterations summed over all solves
  double* rel;
  double tol, tol_in;
  int max_iter;
  const int* skip;  // the solve returns at once when *skip == 1 (null: never)
  const int* used;  // iterations another solver already spent on this system (null: none)
};

template <typename T, typename V>
__device__ __forceinline__ V apply5(const T* dg, const T* ce, const T* cn, const V* v, uint8_t nb,
                                    int64_t o, int nx) {
  V a = (V)dg[o] * v[o];
  if (nb & NB_E) a += (V)ce[o] * v[o + 1];
  if (nb & NB_W) a += (V)ce[o - 1] * v[o - 1];
  if (nb & NB_N) a += (V)cn[o] * v[o + nx];
  if (nb & NB_S) a += (V)cn[o - nx] * v[o - nx];
  return a;
}

// Block-to-tile map of the solver: the G participating blocks take
// contiguous, equal shares of the active-tile list, ordered so that the
// blocks of one XCD (blocks are dispatched round-robin over the 8 XCDs) hold
// neighbouring shares.
struct Share {
  int vb;      // position of this block among the G shares
  int t0, t1;  // active-list range [t0, t1)
};

__device__ __forceinline__ Share share_of(int G, int nlist) {
  const int b = blockIdx.x, x = b & 7, l = b >> 3;
  const int vb = x * (G >> 3) + min(x, G & 7) + l;
  Share S;
  S.vb = vb;
  S.t0 = (int)(((int64_t)nlist * vb) / G);
  S.t1 = (int)(((int64_t)nlist * (vb + 1)) / G);
  return S;
}

// calls f(o, nb) for each marked cell of the block's share
template <typename F>
__device__ __forceinline__ void for_cells(int nx, int ny, int tiles_x, const int* tile_list,
                                          const Share& S, const uint8_t* nbf, F f) {
  for (int t = S.t0; t < S.t1; t++) {
    const int tile = tile_list[t];
    const int i0 = (tile % tiles_x) * TX2, j0 = (tile / tiles_x) * TY2;
    for (int cc = threadIdx.x; cc < TN; cc += NT2) {
      const int i = i0 + cc % TX2, j = j0 + cc / TX2;
      if (i >= nx || j >= ny) continue;
      const int64_t o = (int64_t)j * nx + i;
      const uint8_t nb = nbf[o];
      if (nb & NB_SELF) f(o, nb);
    }
  }
}

// Preconditioner: per active tile, symmetric red-black SOR on the tile's own
// block of A (couplings that leave the tile dropped), from zero: half-sweeps
// red, black, ..., red (GS_HALF of them, a palindrome, so the preconditioner
// is symmetric), over-relaxation GS_OMEGA.  Thread t owns the tile cells 2t
// and 2t + 1 (row-major), one of each colour.
constexpr int GS_HALF = 9;
constexpr int PCG_K = 1;  // tiles per block of the pipelined solver (2 halves the barrier
                          // participants but doubles the registers: slower here)
constexpr double GS_OMEGA = 1.5;

template <typename R>
struct TileCells {
  int64_t o[2];
  uint8_t nb[2];  // neighbour flags restricted to the tile (NB_SELF: a cell of the system)
  int li[2], lj[2];
};

template <typename R>
__device__ __forceinline__ TileCells<R> tile_cells(const PcgArgs<R>& A, int tile) {
  TileCells<R> C;
  const int i0 = (tile % A.tiles_x) * TX2, j0 = (tile / A.tiles_x) * TY2;
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const int cc = 2 * threadIdx.x + q;
    const int li = cc % TX2, lj = cc / TX2;
    const int i = i0 + li, j = j0 + lj;
    C.li[q] = li;
    C.lj[q] = lj;
    C.o[q] = (int64_t)min(j, A.ny - 1) * A.nx + min(i, A.nx - 1);
    uint8_t f = 0;
    if (i < A.nx && j < A.ny) {
      f = A.nb[C.o[q]];
      if (li == TX2 - 1) f &= ~NB_E;
      if (li == 0) f &= ~NB_W;
      if (lj == TY2 - 1) f &= ~NB_N;
      if (lj == 0) f &= ~NB_S;
    }
    C.nb[q] = f;
  }
  return C;
}

// the tile's own block of A at the thread's cells (couplings that leave the
// tile dropped)
template <typename R>
struct TileOp {
  R wdg[2];  // GS_OMEGA / diagonal
  R cE[2], cW[2], cN[2], cS[2];
};

template <typename R>
__device__ __forceinline__ TileOp<R> tile_op(const PcgArgs<R>& A, const TileCells<R>& C) {
  TileOp<R> T;
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const int64_t o = C.o[q];
    const uint8_t f = C.nb[q];
    T.wdg[q] = (R)GS_OMEGA / ((f & NB_SELF) ? A.dgR[o] : R(1));
    T.cE[q] = (f & NB_E) ? A.ceR[o] : R(0);
    T.cW[q] = (f & NB_W) ? A.ceR[o - 1] : R(0);
    T.cN[q] = (f & NB_N) ? A.cnR[o] : R(0);
    T.cS[q] = (f & NB_S) ? A.cnR[o - A.nx] : R(0);
  }
  return T;
}

// u = M^-1 r on one tile; rc[q]: r of the thread's cells (0 off the system);
// z: LDS [TY2][TX2]; result in z (all threads synchronised on return)
template <typename R, int K>
__device__ void tile_precond_k(const TileCells<R> (&C)[K], const TileOp<R> (&T)[K],
                               const R (&rc)[K][2], R (*z)[TY2][TX2]);

template <typename R>
__device__ void tile_precond(const TileCells<R>& C, const TileOp<R>& T, const R (&rc)[2],
                             R (*z)[TX2]) {
  const TileCells<R> Ck[1] = {C};
  const TileOp<R> Tk[1] = {T};
  const R rk[1][2] = {{rc[0], rc[1]}};
  tile_precond_k<R, 1>(Ck, Tk, rk, reinterpret_cast<R(*)[TY2][TX2]>(z));
}

// The full operator at the thread's cells (couplings across tile edges kept)
template <typename R>
struct FullOp {
  uint8_t nf[2];
  R dg[2], cE[2], cW[2], cN[2], cS[2];
};

template <typename R>
__device__ __forceinline__ FullOp<R> full_op(const PcgArgs<R>& A, const TileCells<R>& C) {
  FullOp<R> F;
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const int64_t o = C.o[q];
    const uint8_t f = (C.nb[q] & NB_SELF) ? A.nb[o] : 0;
    F.nf[q] = f;
    F.dg[q] = (f & NB_SELF) ? A.dgR[o] : R(1);
    F.cE[q] = (f & NB_E) ? A.ceR[o] : R(0);
    F.cW[q] = (f & NB_W) ? A.ceR[o - 1] : R(0);
    F.cN[q] = (f & NB_N) ? A.cnR[o] : R(0);
    F.cS[q] = (f & NB_S) ? A.cnR[o - A.nx] : R(0);
  }
  return F;
}

// its restriction to the tile's own block
template <typename R>
__device__ __forceinline__ TileOp<R> restrict_op(const FullOp<R>& F, const TileCells<R>& C) {
  TileOp<R> T;
#pragma unroll
  for (int q = 0; q < 2; q++) {
    T.wdg[q] = (R)GS_OMEGA / F.dg[q];
    T.cE[q] = (C.nb[q] & NB_E) ? F.cE[q] : R(0);
    T.cW[q] = (C.nb[q] & NB_W) ? F.cW[q] : R(0);
    T.cN[q] = (C.nb[q] & NB_N) ? F.cN[q] : R(0);
    T.cS[q] = (C.nb[q] & NB_S) ? F.cS[q] : R(0);
  }
  return T;
}

// (A v) at the thread's cell q: v of the tile from LDS (lds) or memory, v
// across the tile edges from memory
template <typename R>
__device__ __forceinline__ R apply_at(const FullOp<R>& F, const TileCells<R>& C, int q, const R* v,
                                      const R (*zt)[TX2], bool lds, int nx) {
  const int64_t o = C.o[q];
  const int li = C.li[q], lj = C.lj[q];
  const uint8_t f = F.nf[q];
  R a = F.dg[q] * (lds ? zt[lj][li] : v[o]);
  if (f & NB_E) a += F.cE[q] * ((lds && li + 1 < TX2) ? zt[lj][li + 1] : v[o + 1]);
  if (f & NB_W) a += F.cW[q] * ((lds && li > 0) ? zt[lj][li - 1] : v[o - 1]);
  if (f & NB_N) a += F.cN[q] * ((lds && lj + 1 < TY2) ? zt[lj + 1][li] : v[o + nx]);
  if (f & NB_S) a += F.cS[q] * ((lds && lj > 0) ? zt[lj - 1][li] : v[o - nx]);
  return a;
}

// inner vectors of the thread's two cells
template <typename R>
struct Cells {
  R r[2], u[2], w[2], z[2], q[2], s[2], p[2], e[2];
};

// Neighbour sync: every block stamps its tiles, then waits until the four
// face neighbours of each of its tiles that hold unknowns carry the stamp.
template <typename R>
__device__ bool neighbour_sync(const PcgArgs<R>& A, const Share& S, unsigned stamp) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (int t = S.t0; t < S.t1; t++)
      __hip_atomic_store(&A.tflag[A.tile_list[t]], stamp, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 4 * (S.t1 - S.t0); q += NT2) {
    const int tile = A.tile_list[S.t0 + (q >> 2)];
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    int nx_ = tx, ny_ = ty;
    switch (q & 3) {
      case 0: nx_ = tx + 1; break;
      case 1: nx_ = tx - 1; break;
      case 2: ny_ = ty + 1; break;
      default: ny_ = ty - 1;
    }
    if (nx_ < 0 || nx_ >= A.tiles_x || ny_ < 0 || ny_ >= A.tiles_y) continue;
    const int nt = ny_ * A.tiles_x + nx_;
    if (A.tile_cnt[nt] == 0) continue;
    const unsigned long long t0 = wall_clock64();
    unsigned polls = 0;
    while (__hip_atomic_load(&A.tflag[nt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < stamp) {
      if ((++polls & 255u) == 0u) {
        if (aborted(A.bar) || wall_clock64() - t0 > WAIT_TICKS) {
          atomicOr(A.bar.status, ST_ABORT);
          ok = 0;
          break;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return ok != 0;
}

// Preconditioned CG in the Chronopoulos-Gear form (u = M^-1 r, w = A u; one
// grid reduction of (r,u), (w,u), (r,r) per iteration) for blocks that own
// several tiles: vectors in memory.  Each iteration: phase 1 (recurrences of
// p, s, e, r, then u = M^-1 r on the block's tiles), a neighbour-tile sync
// (w needs the neighbours' u), phase 2 (w = A u), one grid barrier.
template <typename R>
__device__ void pcg_cg(const PcgArgs<R>& A, const Share& S, int G, R (*zt)[TX2]) {
  const int nx = A.nx;
  unsigned k = 0;      // grid barriers passed
  unsigned stamp = 0;  // neighbour syncs passed
  double bb = 0.0, rr = 0.0;
  int total = 0, sweep = 0;
  for (;;) {
    // FP64 residual of the current solution -> r in precision R
    {
      double v[2] = {0.0, 0.0};
      for_cells(nx, A.ny, A.tiles_x, A.tile_list, S, A.nb, [&](int64_t o, uint8_t nb) {
        const double rv = A.b[o] - apply5<double, double>(A.dg, A.ce, A.cn, A.x, nb, o, nx);
        A.r[o] = (R)rv;
        v[0] += rv * rv;
        if (sweep == 0) v[1] += A.b[o] * A.b[o];
      });
      block_partials<2>(v, part_buf(A.part, k + 1), S.vb, G);
      if (!grid_sync(A.bar, ++k, G)) return;
      double tt[2];
      grid_totals<2>(part_buf(A.part, k), G, tt);
      rr = tt[0];
      if (sweep == 0) bb = tt[1];
    }
    const double rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (rel <= A.tol) {
      if (blockIdx.x == 0 && threadIdx.x == 0) *A.rel = rel;
      break;
    }
    if (total >= A.max_iter) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        *A.rel = rel;
        atomicOr(A.bar.status, ST_NOCONV);
      }
      break;
    }
    // inner solve of A_R e = r stopped at ||r_k|| <= tol_abs.  FP32 reduces
    // the residual by tol_in (what FP32 can deliver) but never further than
    // the outer target; FP64 goes straight to the outer target.
    const double tol_abs = (sizeof(R) == 4) ? fmax(A.tol_in * sqrt(rr), 0.5 * A.tol * sqrt(bb))
                                            : 0.5 * A.tol * sqrt(bb);
    double gam = 0.0, alpha = 0.0, beta = 0.0;
    double rbest = 0.0;  // stall guard, as in the pipelined solver
    int ibest = 0;
    for (int it = 0;; it++) {
      const R al = (R)alpha, bt = (R)beta;
      double v[3] = {0.0, 0.0, 0.0};  // (r,u), (r,r), (w,u)
      // phase 1
      for (int t = S.t0; t < S.t1; t++) {
        const TileCells<R> C = tile_cells(A, A.tile_list[t]);
        R rc[2];
#pragma unroll
        for (int q = 0; q < 2; q++) {
          rc[q] = R(0);
          if (!(C.nb[q] & NB_SELF)) continue;
          const int64_t o = C.o[q];
          if (it == 0) {
            A.e[o] = R(0);
            rc[q] = A.r[o];
          } else {
            const R pv = it == 1 ? A.u[o] : fma(bt, A.p[o], A.u[o]);
            const R sv = it == 1 ? A.w[o] : fma(bt, A.s[o], A.w[o]);
            A.p[o] = pv;
            A.s[o] = sv;
            A.e[o] = fma(al, pv, A.e[o]);
            rc[q] = fma(-al, sv, A.r[o]);
            A.r[o] = rc[q];
          }
        }
        tile_precond(C, tile_op(A, C), rc, zt);
#pragma unroll
        for (int q = 0; q < 2; q++) {
          if (!(C.nb[q] & NB_SELF)) continue;
          const R uv = zt[C.lj[q]][C.li[q]];
          A.u[C.o[q]] = uv;
          v[0] += (double)rc[q] * (double)uv;
          v[1] += (double)rc[q] * (double)rc[q];
        }
        __syncthreads();  // zt is reused by the next tile
      }
      if (!neighbour_sync(A, S, ++stamp)) return;
      // phase 2: w = A u
      for_cells(nx, A.ny, A.tiles_x, A.tile_list, S, A.nb, [&](int64_t o, uint8_t nb) {
        const R a = apply5<R, R>(A.dgR, A.ceR, A.cnR, A.u, nb, o, nx);
        A.w[o] = a;
        v[2] += (double)a * (double)A.u[o];
      });
      block_partials<3>(v, part_buf(A.part, k + 1), S.vb, G);
      if (!grid_sync(A.bar, ++k, G)) return;
      double tt[3];
      grid_totals<3>(part_buf(A.part, k), G, tt);
      const double gn = tt[0], rn = tt[1], dn = tt[2];
      if (it == 0 || rn < 0.81 * rbest) {
        rbest = rn;
        ibest = it;
      }
      if (it > 0) {
        total++;
        if (sqrt(rn) <= tol_abs || total >= A.max_iter || !(gn == gn)) break;
        if (it - ibest >= STALL_ITERS) break;
      }
      if (it == 0) {
        alpha = dn != 0.0 ? gn / dn : 0.0;
        beta = 0.0;
      } else {
        const double bn = gam != 0.0 ? gn / gam : 0.0;
        const double den = dn - bn * gn / alpha;
        if (!(den != 0.0)) break;
        beta = bn;
        alpha = gn / den;
      }
      gam = gn;
    }
    // x += e (FP64)
    for_cells(nx, A.ny, A.tiles_x, A.tile_list, S, A.nb,
              [&](int64_t o, uint8_t nb) { A.x[o] += (double)A.e[o]; });
    if (!grid_sync(A.bar, ++k, G)) return;
    sweep++;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *A.iters = total;
    *A.iters_sum += total;
  }
}


// u = M^-1 r on the K tiles of a block at once (the sweeps of all K tiles
// share the block's barriers); slot k of zt holds tile k
// one cell of a thread in the red-black sweeps
template <typename R>
struct SorCell {
  int li, lj;
  uint8_t f;
  R r, wdg, cE, cW, cN, cS;
};

template <typename R>
__device__ __forceinline__ SorCell<R> sor_cell(const TileCells<R>& C, const TileOp<R>& T,
                                               const R (&rc)[2], int q) {
  SorCell<R> X;
  X.li = q ? C.li[1] : C.li[0];
  X.lj = C.lj[0];
  X.f = q ? C.nb[1] : C.nb[0];
  X.r = q ? rc[1] : rc[0];
  X.wdg = q ? T.wdg[1] : T.wdg[0];
  X.cE = q ? T.cE[1] : T.cE[0];
  X.cW = q ? T.cW[1] : T.cW[0];
  X.cN = q ? T.cN[1] : T.cN[0];
  X.cS = q ? T.cS[1] : T.cS[0];
  return X;
}

template <typename R>
__device__ __forceinline__ void sor_relax(const SorCell<R>& X, R (*z)[TX2], R om) {
  if (!(X.f & NB_SELF)) return;
  R a = X.r;
  if (X.f & NB_E) a -= X.cE * z[X.lj][X.li + 1];
  if (X.f & NB_W) a -= X.cW * z[X.lj][X.li - 1];
  if (X.f & NB_N) a -= X.cN * z[X.lj + 1][X.li];
  if (X.f & NB_S) a -= X.cS * z[X.lj - 1][X.li];
  z[X.lj][X.li] = (R(1) - om) * z[X.lj][X.li] + X.wdg * a;
}

// The thread's two cells 2t, 2t + 1 are neighbours in one row, so one is red
// and one black: each half-sweep relaxes exactly one cell per thread.  The
// first (red) half-sweep starts from z = 0, where a red cell's neighbours
// are all zero: it takes wdg r, and the black cells are cleared with it.
template <typename R, int K>
__device__ void tile_precond_k(const TileCells<R> (&C)[K], const TileOp<R> (&T)[K],
                               const R (&rc)[K][2], R (*z)[TY2][TX2]) {
  SorCell<R> X[K][2];  // [tile][colour]
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int q0 = (C[k].li[0] + C[k].lj[0]) & 1;  // colour of cell 0
    X[k][0] = sor_cell(C[k], T[k], rc[k], q0);      // red: (i + j) even
    X[k][1] = sor_cell(C[k], T[k], rc[k], q0 ^ 1);
    const SorCell<R>& Rd = X[k][0];
    z[k][Rd.lj][Rd.li] = (Rd.f & NB_SELF) ? Rd.wdg * Rd.r : R(0);
    z[k][X[k][1].lj][X[k][1].li] = R(0);
  }
  __syncthreads();
  const R om = (R)GS_OMEGA;
#pragma unroll
  for (int hs = 1; hs < GS_HALF; hs++) {
#pragma unroll
    for (int k = 0; k < K; k++) sor_relax(X[k][hs & 1], z[k], om);
    __syncthreads();
  }
}

// Coarse correction of the block's tile and of its four face neighbours:
// c = (Z^T A Z)^-1 sig restricted to those tiles, where sig holds the tile
// sums of the vector being preconditioned (one per active tile, list order).
template <typename R>
struct Coarse {
  R own, e, w, n, s;
};

// the rows of (Z^T A Z)^-1 of the block's tile and its face neighbours (zero
// rows for missing or inactive neighbours) -> rows[5][CMAX2]; returns whether
// the coarse space is used (the block's tile at list position t, nc tiles)
template <typename R>
__device__ bool coarse_rows(const PcgArgs<R>& A, int t, int nc, double (*rows)[CMAX2]) {
  const bool on = A.cinv != nullptr && nc <= CMAX2 && A.cused[2] == 1;
  if (!on) return false;
  const int tile = A.tile_list[t], tx = tile % A.tiles_x, ty = tile / A.tiles_x;
  int pos[5];
  pos[0] = t;
  pos[1] = tx + 1 < A.tiles_x ? A.tile_pos[tile + 1] : -1;
  pos[2] = tx > 0 ? A.tile_pos[tile - 1] : -1;
  pos[3] = ty + 1 < A.tiles_y ? A.tile_pos[tile + A.tiles_x] : -1;
  pos[4] = ty > 0 ? A.tile_pos[tile - A.tiles_x] : -1;
  for (int e = threadIdx.x; e < 5 * CMAX2; e += NT2) {
    const int r = e / CMAX2, j = e % CMAX2;
    rows[r][j] = (pos[r] >= 0 && j < nc) ? A.cinv[(int64_t)pos[r] * nc + j] : 0.0;
  }
  __syncthreads();
  return true;
}

// grid_totals plus the coarse correction from the last of the NV partial
// rows (the tile sums: one per block = one per active tile, list order)
template <int NV, typename R>
__device__ void grid_totals_coarse(const double* part, int G, double (&tot)[NV], bool on,
                                   const double (*rows)[CMAX2], Coarse<R>& cc) {
  double c[5];
  grid_totals_rows<NV>(part, G, tot, on, rows, c);
  cc.own = (R)c[0];
  cc.e = (R)c[1];
  cc.w = (R)c[2];
  cc.n = (R)c[3];
  cc.s = (R)c[4];
}

// (A v) at the thread's cell q where v = (tile-local part) + (coarse
// constant of the tile the cell lies in): the tile's local part from LDS, the
// neighbours' from memory
template <typename R>
__device__ __forceinline__ R apply_coarse(const FullOp<R>& F, const TileCells<R>& C, int q,
                                          const R* v, const R (*zt)[TX2], int nx,
                                          const Coarse<R>& K) {
  const int64_t o = C.o[q];
  const int li = C.li[q], lj = C.lj[q];
  const uint8_t f = F.nf[q];
  R a = F.dg[q] * (zt[lj][li] + K.own);
  if (f & NB_E) a += F.cE[q] * (li + 1 < TX2 ? zt[lj][li + 1] + K.own : v[o + 1] + K.e);
  if (f & NB_W) a += F.cW[q] * (li > 0 ? zt[lj][li - 1] + K.own : v[o - 1] + K.w);
  if (f & NB_N) a += F.cN[q] * (lj + 1 < TY2 ? zt[lj + 1][li] + K.own : v[o + nx] + K.n);
  if (f & NB_S) a += F.cS[q] * (lj > 0 ? zt[lj - 1][li] + K.own : v[o - nx] + K.s);
  return a;
}

// whether the thread's cell q couples to a cell outside its tile in
// direction d (0 E, 1 W, 2 N, 3 S), and that cell's offset from it
template <typename R>
__device__ __forceinline__ bool off_tile(const FullOp<R>& F, const TileCells<R>& C, int q, int d) {
  const uint8_t f = F.nf[q];
  const int li = C.li[q], lj = C.lj[q];
  switch (d) {
    case 0: return (f & NB_E) && li + 1 == TX2;
    case 1: return (f & NB_W) && li == 0;
    case 2: return (f & NB_N) && lj + 1 == TY2;
    default: return (f & NB_S) && lj == 0;
  }
}
__device__ __forceinline__ int64_t dir_offset(int d, int nx) {
  return d == 0 ? 1 : d == 1 ? -1 : d == 2 ? (int64_t)nx : -(int64_t)nx;
}

// The end of a pass: one polling loop gathers both the pass's block partials
// (all G of them, thread t taking b = t, t + NT2, ...) and the values of the
// vector just published (mt) outside the thread's tiles, for the next pass's
// product, so that the two waits overlap; then the fixed-order totals as in
// grid_totals_rows.  Returns false in every thread when the solve aborted.
template <int NV, typename R, int K>
__device__ bool pass_end_tagged(const unsigned long long* pt, int G, unsigned tag,
                                double (&tot)[NV], bool on, const double (*crow)[CMAX2],
                                double (&c)[5], const FullOp<R> (&F)[K],
                                const TileCells<R> (&C)[K], const unsigned long long* mt, int nx,
                                R (&hv)[K][2][4], const Bar& B, int* abort_flag) {
  static_assert(NV + 5 <= 9, "reduction rows");
  constexpr int NBT = PCG_GMAX / NT2;  // partials per thread
  static_assert(NBT * NV <= 32 && 8 * K <= 32, "poll masks");
  constexpr int W = tag_words<R>();
  __shared__ double out[NV + 5];
  unsigned nh = 0, np = 0;
#pragma unroll
  for (int k = 0; k < K; k++)
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
      for (int d = 0; d < 4; d++) {
        hv[k][q][d] = R(0);
        if (off_tile(F[k], C[k], q, d)) nh |= 1u << (8 * k + 4 * q + d);
      }
  double pv[NBT][NV];
#pragma unroll
  for (int i = 0; i < NBT; i++)
#pragma unroll
    for (int k = 0; k < NV; k++) {
      pv[i][k] = 0.0;
      if ((int)threadIdx.x + NT2 * i < G) np |= 1u << (NV * i + k);
    }
  bool ok = true;
  const unsigned long long t0 = wall_clock64();
  unsigned polls = 0;
  while (nh | np) {
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
      for (int q = 0; q < 2; q++)
#pragma unroll
        for (int d = 0; d < 4; d++) {
          const unsigned bit = 1u << (8 * k + 4 * q + d);
          if ((nh & bit) &&
              try_tagged(mt + (C[k].o[q] + dir_offset(d, nx)) * W, tag, hv[k][q][d]))
            nh &= ~bit;
        }
#pragma unroll
    for (int i = 0; i < NBT; i++)
#pragma unroll
      for (int k = 0; k < NV; k++) {
        const unsigned bit = 1u << (NV * i + k);
        const int b = threadIdx.x + NT2 * i;
        if ((np & bit) && try_tagged(pt + ((int64_t)k * G + b) * 2, tag, pv[i][k])) np &= ~bit;
      }
    if (!(nh | np)) break;
    if ((++polls & 255u) == 0u) {
      if (aborted(B) || wall_clock64() - t0 > WAIT_TICKS) {
        if (!aborted(B)) atomicOr(B.status, ST_ABORT);
        ok = false;
        break;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (!ok) *abort_flag = 1;
  double a[NV + 5];
#pragma unroll
  for (int k = 0; k < NV + 5; k++) a[k] = 0.0;
#pragma unroll
  for (int i = 0; i < NBT; i++) {
    const int b = threadIdx.x + NT2 * i;
    if (b >= G) continue;
#pragma unroll
    for (int k = 0; k < NV; k++) a[k] += pv[i][k];
    if (on) {
#pragma unroll
      for (int r = 0; r < 5; r++) a[NV + r] += crow[r][b] * pv[i][NV - 1];
    }
  }
  double (*rows)[NT2] = red_rows();
  const int nrow = on ? NV + 5 : NV;
  __syncthreads();  // the block partials' reads of the rows are done
#pragma unroll
  for (int k = 0; k < NV + 5; k++)
    if (k < nrow) rows[k][threadIdx.x] = a[k];
  __syncthreads();
  sum_rows(rows, nrow, out);
#pragma unroll
  for (int k = 0; k < NV; k++) tot[k] = out[k];
#pragma unroll
  for (int r = 0; r < 5; r++) c[r] = on ? out[NV + r] : 0.0;
  return *abort_flag == 0;
}

// (A v) at the thread's cell q with v's tile-local part from LDS, its values
// outside the tile from hv (E, W, N, S), plus the coarse constants
template <typename R>
__device__ __forceinline__ R apply_halo(const FullOp<R>& F, const TileCells<R>& C, int q,
                                        const R (&hv)[4], const R (*zt)[TX2],
                                        const Coarse<R>& K) {
  const int li = C.li[q], lj = C.lj[q];
  const uint8_t f = F.nf[q];
  R a = F.dg[q] * (zt[lj][li] + K.own);
  if (f & NB_E) a += F.cE[q] * (li + 1 < TX2 ? zt[lj][li + 1] + K.own : hv[0] + K.e);
  if (f & NB_W) a += F.cW[q] * (li > 0 ? zt[lj][li - 1] + K.own : hv[1] + K.w);
  if (f & NB_N) a += F.cN[q] * (lj + 1 < TY2 ? zt[lj + 1][li] + K.own : hv[2] + K.n);
  if (f & NB_S) a += F.cS[q] * (lj > 0 ? zt[lj - 1][li] + K.own : hv[3] + K.s);
  return a;
}

// Preconditioned CG in the pipelined form of Ghysels and Vanroose (2014)
// for blocks that own up to K tiles each: per iteration one pass and one
// grid barrier, which both completes the reduction of (r,u), (w,u), (r,r)
// and publishes m = M^-1 w (tile-local) for the neighbours' n = A m of the
// next pass (m double-buffered by pass parity).  The vectors stay in
// registers and the tiles' m stays in LDS for the whole solve.
template <typename R, int K>
__device__ unsigned pcg_pipelined(const PcgArgs<R>& A, const Share& S, int G, R (*zt)[TY2][TX2],
                                  double (*crows)[CMAX2], unsigned base) {
  const int nx = A.nx;
  __shared__ int s_abort;  // set by any thread whose poll of a pass timed out or saw an abort
  if (threadIdx.x == 0) s_abort = 0;
  __syncthreads();
  unsigned tp = 0;  // tags used: the pass with tag base + tp is the latest
  TileCells<R> C[K];
  FullOp<R> F[K];
  TileOp<R> T[K];
  Cells<R> X[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const bool has = S.t0 + k < S.t1;
    C[k] = tile_cells(A, has ? A.tile_list[S.t0 + k] : A.tile_list[S.t0]);
    if (!has) C[k].nb[0] = C[k].nb[1] = 0;  // an empty slot: no cells of the system
    F[k] = full_op(A, C[k]);
    T[k] = restrict_op(F[k], C[k]);
    X[k] = Cells<R>{};
  }
  // the coarse space needs one tile per block (its tile sums are the blocks'
  // partial sums)
  const bool coarse = (K == 1) && coarse_rows(A, S.t0, G, crows);
  Coarse<R> cu{}, cm{};  // coarse constants of u_0 and of the last m
  unsigned bk = 0;  // grid barriers passed
  double bb = 0.0, rr = 0.0;
  int total = 0, sweep = 0;
  for (;;) {
    // FP64 residual of the current solution -> r_0 (precision R), u_0 = M^-1 r_0
    {
      double v[3] = {0.0, 0.0, 0.0};  // (r,r), (b,b), tile sum of r
      R rc[K][2];
#pragma unroll
      for (int k = 0; k < K; k++)
#pragma unroll
        for (int q = 0; q < 2; q++) {
          rc[k][q] = R(0);
          if (!(F[k].nf[q] & NB_SELF)) continue;
          const int64_t o = C[k].o[q];
          const double rv =
              A.b[o] - apply5<double, double>(A.dg, A.ce, A.cn, A.x, F[k].nf[q], o, nx);
          rc[k][q] = (R)rv;
          X[k].r[q] = rc[k][q];
          X[k].e[q] = R(0);
          v[0] += rv * rv;
          if (sweep == 0) v[1] += A.b[o] * A.b[o];
          v[2] += (double)rc[k][q];
        }
      tile_precond_k<R, K>(C, T, rc, zt);
#pragma unroll
      for (int k = 0; k < K; k++)
#pragma unroll
        for (int q = 0; q < 2; q++) {
          if (!(F[k].nf[q] & NB_SELF)) continue;
          A.u[C[k].o[q]] = zt[k][C[k].lj[q]][C[k].li[q]];  // the tile-local part
        }
      block_partials<3>(v, part_buf(A.part, bk + 1), S.vb, G);
      if (!grid_sync(A.bar, ++bk, G)) return tp;
      double tt[3];
      grid_totals_coarse<3, R>(part_buf(A.part, bk), G, tt, coarse, crows, cu);
      rr = tt[0];
      if (sweep == 0) bb = tt[1];
#pragma unroll
      for (int k = 0; k < K; k++)
#pragma unroll
        for (int q = 0; q < 2; q++)
          if (F[k].nf[q] & NB_SELF) X[k].u[q] = zt[k][C[k].lj[q]][C[k].li[q]] + cu.own;
    }
    const double rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (rel <= A.tol) {
      if (blockIdx.x == 0 && threadIdx.x == 0) *A.rel = rel;
      break;
    }
    if (total >= A.max_iter) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        *A.rel = rel;
        atomicOr(A.bar.status, ST_NOCONV);
      }
      break;
    }
    // inner solve of A_R e = r stopped at ||r_j|| <= tol_abs.  FP32 reduces
    // the residual by tol_in (what FP32 can deliver) but never further than
    // the outer target; FP64 goes straight to the outer target.
    const double tol_abs = (sizeof(R) == 4) ? fmax(A.tol_in * sqrt(rr), 0.5 * A.tol * sqrt(bb))
                                            : 0.5 * A.tol * sqrt(bb);
    double gam = 0.0, alpha = 0.0, beta = 0.0;
    double rbest = 0.0;  // stall guard: the smallest ||r_j||^2 that cut the last best by 10%
    int jbest = 0;
    R hv[K][2][4];  // m of the last pass outside the tiles (gathered at its end)
    for (int j = 0;; j++) {
      // pass j: (j >= 1) n = A m_{j-1} and the recurrences with alpha_{j-1},
      // beta_{j-1}; (j == 0) w_0 = A u_0.  Then the partial sums of pass j
      // and m_j = M^-1 w_j: its tile-local part published for the
      // neighbours, its coarse part from the tile sums of w_j after the
      // barrier.  zt holds the tile-local part of u_0 (j == 0) or of m_{j-1}
      // on entry.
      const R al = (R)alpha, bt = (R)beta;
      const unsigned tag = base + (++tp);
      double v[4] = {0.0, 0.0, 0.0, 0.0};  // (r,u), (w,u), (r,r), tile sum of w
      R wc[K][2];
#pragma unroll
      for (int k = 0; k < K; k++)
#pragma unroll
        for (int q = 0; q < 2; q++) {
          wc[k][q] = R(0);
          if (!(F[k].nf[q] & NB_SELF)) continue;
          Cells<R>& Y = X[k];
          if (j == 0) {
            Y.w[q] = coarse ? apply_coarse(F[k], C[k], q, A.u, zt[k], nx, cu)
                            : apply_at(F[k], C[k], q, A.u, zt[k], true, nx);
          } else {
            const R n = apply_halo(F[k], C[k], q, hv[k][q], zt[k], cm);
            const R m = zt[k][C[k].lj[q]][C[k].li[q]] + cm.own;
            const bool first = j == 1;
            Y.z[q] = first ? n : fma(bt, Y.z[q], n);
            Y.q[q] = first ? m : fma(bt, Y.q[q], m);
            Y.s[q] = first ? Y.w[q] : fma(bt, Y.s[q], Y.w[q]);
            Y.p[q] = first ? Y.u[q] : fma(bt, Y.p[q], Y.u[q]);
            Y.e[q] = fma(al, Y.p[q], Y.e[q]);
            Y.r[q] = fma(-al, Y.s[q], Y.r[q]);
            Y.u[q] = fma(-al, Y.q[q], Y.u[q]);
            Y.w[q] = fma(-al, Y.z[q], Y.w[q]);
          }
          wc[k][q] = Y.w[q];
          v[0] += (double)Y.r[q] * (double)Y.u[q];
          v[1] += (double)Y.w[q] * (double)Y.u[q];
          v[2] += (double)Y.r[q] * (double)Y.r[q];
          v[3] += (double)Y.w[q];
        }
      __syncthreads();  // the tiles' LDS values are read before the sweeps overwrite them
      if (s_abort) return tp;
      tile_precond_k<R, K>(C, T, wc, zt);
      // m_j on the tiles' edge cells, for the neighbours' next pass
      unsigned long long* mw = A.mt[tag & 1];
#pragma unroll
      for (int k = 0; k < K; k++)
#pragma unroll
        for (int q = 0; q < 2; q++) {
          const int li = C[k].li[q], lj = C[k].lj[q];
          const bool edge = li == 0 || li == TX2 - 1 || lj == 0 || lj == TY2 - 1;
          if (edge && (F[k].nf[q] & NB_SELF))
            put_tagged(mw + C[k].o[q] * tag_words<R>(), zt[k][lj][li], tag);
        }
      unsigned long long* pw = A.pt + (size_t)(tag & 1u) * (8 * PCG_GMAX);
      block_partials_tagged<4>(v, pw, S.vb, G, tag);
      double tt[4], c5[5];
      if (!pass_end_tagged<4, R, K>(pw, G, tag, tt, coarse, crows, c5, F, C, mw, nx, hv, A.bar,
                                    &s_abort))
        return tp;
      cm.own = (R)c5[0];
      cm.e = (R)c5[1];
      cm.w = (R)c5[2];
      cm.n = (R)c5[3];
      cm.s = (R)c5[4];
      const double gn = tt[0], dn = tt[1], rn = tt[2];
      if (j == 0 || rn < 0.81 * rbest) {
        rbest = rn;
        jbest = j;
      }
      if (j > 0) {
        total++;
        if (sqrt(rn) <= tol_abs || total >= A.max_iter || !(gn == gn)) break;
        // the recursively updated residual has stalled (rounding in the
        // recurrences, worst in FP32): end this inner solve, and the FP64
        // residual of the next sweep restarts it
        if (j - jbest >= STALL_ITERS) break;
      }
      if (j == 0) {
        alpha = dn != 0.0 ? gn / dn : 0.0;
        beta = 0.0;
      } else {
        const double bn = gam != 0.0 ? gn / gam : 0.0;
        const double den = dn - bn * gn / alpha;
        if (!(den != 0.0)) break;
        beta = bn;
        alpha = gn / den;
      }
      gam = gn;
    }
    // x += e (FP64)
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
      for (int q = 0; q < 2; q++)
        if (F[k].nf[q] & NB_SELF) A.x[C[k].o[q]] += (double)X[k].e[q];
    if (!grid_sync(A.bar, ++bk, G)) return tp;
    sweep++;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *A.iters = total;
    *A.iters_sum += total;
  }
  return tp;
}

// Persistent preconditioned CG (M^-1: the tile-block symmetric red-black SOR
// above), two kernels launched one after the other of which exactly one
// works: pipelined when the active tiles fit PCG_K per block of its grid,
// Chronopoulos-Gear with a neighbour-tile sync otherwise (separate kernels,
// so that each gets its own register budget and grid).  The inner solve runs
// in precision R; the outer loop refines the FP64 solution with FP64
// residuals until ||b - A x|| <= tol ||b||.
template <typename R>
__global__ void __launch_bounds__(NT2) k_pcg2d_pipe(PcgArgs<R> A) {
  __shared__ R zt[PCG_K][TY2][TX2];
  __shared__ double crows[5][CMAX2];
  if (A.skip && *A.skip == 1) return;
  const int nlist = *A.n_list;
  if (nlist < 1 || nlist > PCG_K * A.pipe_blocks) return;  // the other form's case
  const int G = (nlist + PCG_K - 1) / PCG_K;
  if ((int)blockIdx.x >= G) return;
  PcgArgs<R> B = A;
  if (B.used) B.max_iter -= *B.used;
  // every block reads the tag base before block 0 can pass its first pass
  const unsigned base = *A.tag_base;
  const unsigned used = pcg_pipelined<R, PCG_K>(B, share_of(G, nlist), G, zt, crows, base);
  // no block is more than one pass ahead of block 0, even after an abort
  if (blockIdx.x == 0 && threadIdx.x == 0) *A.tag_base = base + used + 2;
}

template <typename R>
__global__ void __launch_bounds__(NT2) k_pcg2d_cg(PcgArgs<R> A) {
  __shared__ R zt[TY2][TX2];
  if (A.skip && *A.skip == 1) return;
  const int nlist = *A.n_list;
  if (nlist >= 1 && nlist <= PCG_K * A.pipe_blocks) return;  // the pipelined form's case
  const int G = max(1, min((int)gridDim.x, nlist));
  if ((int)blockIdx.x >= G) return;
  PcgArgs<R> B = A;
  if (B.used) B.max_iter -= *B.used;
  pcg_cg(B, share_of(G, nlist), G, zt);
}

// ---- coarse space of the preconditioner ----
// Two-level additive Schwarz (Nicolaides' coarse space): with Z the matrix
// whose column k is the indicator of active tile k's unknowns, the
// preconditioner is M^-1 = (tile-block SSOR) + Z (Z^T A Z)^-1 Z^T.  Z^T A Z is
// symmetric positive definite (A is, and Z has full column rank); it couples
// each tile with its four face neighbours.  The pipelined solver applies the
// coarse part with the tile sums of w, which travel with the partial sums of
// its one grid barrier per iteration; when more tiles are active than CMAX2
// the solver runs without it.

// row of Z^T A Z of active tile blockIdx.x (list order): sum of A over the
// tile's own block, and of the couplings to each face-neighbour tile
__global__ void __launch_bounds__(NT2) k_coarse2d(int nx, int ny, int tiles_x,
                                                  const int* tile_list, const int* n_list,
                                                  const uint8_t* __restrict__ nbf,
                                                  const double* __restrict__ dg,
                                                  const double* __restrict__ ce,
                                                  const double* __restrict__ cn,
                                                  double* __restrict__ crow) {
  if ((int)blockIdx.x >= *n_list) return;
  const int tile = tile_list[blockIdx.x];
  const int i0 = (tile % tiles_x) * TX2, j0 = (tile / tiles_x) * TY2;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // self, E, W, N, S
  for (int cc = threadIdx.x; cc < TN; cc += NT2) {
    const int li = cc % TX2, lj = cc / TX2, i = i0 + li, j = j0 + lj;
    if (i >= nx || j >= ny) continue;
    const int64_t o = (int64_t)j * nx + i;
    const uint8_t f = nbf[o];
    if (!(f & NB_SELF)) continue;
    v[0] += dg[o];
    if (f & NB_E) v[li + 1 < TX2 ? 0 : 1] += ce[o];
    if (f & NB_W) v[li > 0 ? 0 : 2] += ce[o - 1];
    if (f & NB_N) v[lj + 1 < TY2 ? 0 : 3] += cn[o];
    if (f & NB_S) v[lj > 0 ? 0 : 4] += cn[o - nx];
  }
  __shared__ double sh[5][NT2 / 64];
#pragma unroll
  for (int k = 0; k < 5; k++) {
    const double t = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = t;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double t = 0.0;
    for (int w = 0; w < NT2 / 64; w++) t += sh[threadIdx.x][w];
    crow[5 * (int64_t)blockIdx.x + threadIdx.x] = t;
  }
}

// (Z^T A Z)^-1 of the nc <= CMAX2 active tiles: the dense matrix in LDS,
// inverted in place by Gauss-Jordan elimination without pivoting (an SPD
// matrix needs none), written to cinv[nc][nc].  One block.
//
// The inverse is kept while the active tiles stay the same, for up to
// CINV_AGE solves: any SPD matrix in its place still gives an SPD
// preconditioner, and the operator changes little from one step to the next.
//
// The coarse space pays off when the operator couples the tiles strongly,
// i.e. when the pressure's decay length (the screening of the s22 term) spans
// several tiles; when it is shorter than a tile the tile-local part already
// holds the solution's structure and the additive coarse term only adds to
// the spectrum.  Measure: rho = max over tiles of (sum of the couplings to
// the neighbour tiles) / (diagonal) of Z^T A Z, which tends to 1 as the
// screening vanishes; the coarse space is used when rho >= CRHO.
//
// used[0] = nc of the stored inverse (-1: none), used[1] = solves since it was
// made, used[2] = 1 when the solver uses it, used[3 ..] = its tile list.
constexpr int CINV_AGE = 16;
constexpr double CRHO = 0.95;

__global__ void __launch_bounds__(1024) k_coarse_inv2d(int tiles_x, int tiles_y,
                                                       const int* tile_list, const int* n_list,
                                                       const int* tile_pos,
                                                       const double* __restrict__ crow,
                                                       double* __restrict__ cinv, int* used) {
  const int nc = *n_list;
  if (nc < 1 || nc > CMAX2) {
    if (threadIdx.x == 0) {
      used[0] = -1;
      used[2] = 0;
    }
    return;
  }
  __shared__ int keep;
  if (threadIdx.x == 0) keep = (used[0] == nc && used[1] + 1 < CINV_AGE) ? 1 : 0;
  __syncthreads();
  if (keep) {
    if ((int)threadIdx.x < nc && used[3 + threadIdx.x] != tile_list[threadIdx.x]) keep = 0;
    __syncthreads();
    if (keep) {
      if (threadIdx.x == 0) used[1] += 1;
      return;
    }
  }
  __shared__ double M[CMAX2][CMAX2];
  __shared__ double col[CMAX2];
  __shared__ double rho_w[1024 / 64];
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) M[e / nc][e % nc] = 0.0;
  __syncthreads();
  double rho = 0.0;
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const int tile = tile_list[i], tx = tile % tiles_x, ty = tile / tiles_x;
    const double* r = crow + 5 * (int64_t)i;
    M[i][i] = r[0];
    double off = 0.0;
    if (tx + 1 < tiles_x && tile_pos[tile + 1] >= 0) {
      M[i][tile_pos[tile + 1]] = r[1];
      off += fabs(r[1]);
    }
    if (tx > 0 && tile_pos[tile - 1] >= 0) {
      M[i][tile_pos[tile - 1]] = r[2];
      off += fabs(r[2]);
    }
    if (ty + 1 < tiles_y && tile_pos[tile + tiles_x] >= 0) {
      M[i][tile_pos[tile + tiles_x]] = r[3];
      off += fabs(r[3]);
    }
    if (ty > 0 && tile_pos[tile - tiles_x] >= 0) {
      M[i][tile_pos[tile - tiles_x]] = r[4];
      off += fabs(r[4]);
    }
    rho = fmax(rho, off / r[0]);
  }
  rho = wave_max(rho);
  if ((threadIdx.x & 63) == 0) rho_w[threadIdx.x >> 6] = rho;
  __syncthreads();
  rho = rho_w[0];
  for (int w = 1; w < 1024 / 64; w++) rho = fmax(rho, rho_w[w]);
  if (!(rho >= CRHO)) {  // the coarse space would not help: recorded, not inverted
    if ((int)threadIdx.x < nc) used[3 + threadIdx.x] = tile_list[threadIdx.x];
    if (threadIdx.x == 0) {
      used[0] = nc;
      used[1] = 0;
      used[2] = 0;
    }
    return;
  }
  // thread (ty, tx) of a 32 x 32 layout updates rows ty + 32 a, columns tx + 32 b
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = 0; k < nc; k++) {
    const double inv = 1.0 / M[k][k];
    // column k kept, row k scaled (off the pivot)
    if ((int)threadIdx.x < nc) {
      const int e = threadIdx.x;
      col[e] = M[e][k];
      if (e != k) M[k][e] *= inv;
    }
    __syncthreads();
    for (int i = ty; i < nc; i += 32) {
      const double ci = col[i];
      for (int j = tx; j < nc; j += 32) {
        if (i == k) {
          if (j == k) M[k][k] = inv;
        } else if (j == k) {
          M[i][k] = -ci * inv;
        } else {
          M[i][j] -= ci * M[k][j];
        }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) cinv[e] = M[e / nc][e % nc];
  if ((int)threadIdx.x < nc) used[3 + threadIdx.x] = tile_list[threadIdx.x];
  if (threadIdx.x == 0) {
    used[0] = nc;
    used[1] = 0;
    used[2] = 1;
  }
}

__global__ void k_bar_reset(unsigned long long* count, unsigned* tflag, int ntiles) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0ull;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x)
    tflag[t] = 0u;
}

// ---------------------------------------------------------------------------
// projection
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT2) k_correct2d(G2 G, const double* __restrict__ ht,
                                                   const double* __restrict__ mt,
                                                   const double* __restrict__ nt,
                                                   const double* __restrict__ kt,
                                                   const uint8_t* __restrict__ mask,
                                                   const int* tile_list, const int* n_list,
                                                   const double* t_in, const double* dt_in,
                                                   const double* __restrict__ x, double* hu,
                                                   double* hv, double* hw, double* p,
                                                   int fold_speed) {
  if ((int)blockIdx.x >= *n_list) return;
  __shared__ Ring R;
  const int tile = tile_list[blockIdx.x];
  const int i0 = (tile % G.tiles_x) * TX2, j0 = (tile / G.tiles_x) * TY2;
  const Chan c = G.ch[0];
  const double dt = dt_in[0];
  const Motion M = body_motion(c, t_in[0] + dt);
  fill_ring(R, G, c, M, ht, mt, nt, i0, j0);
  __syncthreads();
  const int nx = G.nx;
  const double idx = 1.0 / G.dx, idy = 1.0 / G.dy;
  double sp = 0.0;
  int flags = 0;
  for (int cc = threadIdx.x; cc < TN; cc += NT2) {
    const int ti = cc % TX2, tj = cc / TX2;
    const int i = i0 + ti, j = j0 + tj;
    if (i >= G.nx || j >= G.ny) continue;
    const int64_t o = (int64_t)j * nx + i;
    if (!mask[o]) continue;
    auto pv = [&](int a, int b) -> double {
      if (a < 0 || a >= G.nx || b < 0 || b >= G.ny) return 0.0;
      const int64_t u = (int64_t)b * nx + a;
      return mask[u] ? x[u] : 0.0;
    };
    const int w = (tj + 1) * RGX + (ti + 1);
    const Face2 fw = face_coef(R, G, dt, w - 1, w, true), fe = face_coef(R, G, dt, w, w + 1, true);
    const Face2 fs = face_coef(R, G, dt, w - RGX, w, false);
    const Face2 fn = face_coef(R, G, dt, w, w + RGX, false);
    const double pc = x[o];
    double dqw = fw.fd - fw.K * (fw.a * pv(i - 1, j) + fw.b * pc);
    double dqe = fe.fd - fe.K * (fe.a * pc + fe.b * pv(i + 1, j));
    double dqs = fs.fd - fs.K * (fs.a * pv(i, j - 1) + fs.b * pc);
    double dqn = fn.fd - fn.K * (fn.a * pc + fn.b * pv(i, j + 1));
    if (G.tensor) {
      // the off-diagonal flux of each face's pair: east and north faces pair
      // with each other, the west face with the north face of the cell to the
      // west, the south face with the east face of the cell below
      const double k0 = pair_k(fe, fn);
      dqe -= k0 * (fn.a * pc + fn.b * pv(i, j + 1));
      dqn -= k0 * (fe.a * pc + fe.b * pv(i + 1, j));
      if (i > 0) {
        const Face2 fnW = face_coef(R, G, dt, w - 1, w - 1 + RGX, false);
        dqw -= pair_k(fw, fnW) * (fnW.a * pv(i - 1, j) + fnW.b * pv(i - 1, j + 1));
      }
      if (j > 0) {
        const Face2 feS = face_coef(R, G, dt, w - RGX, w - RGX + 1, true);
        dqs -= pair_k(feS, fs) * (feS.a * pv(i, j - 1) + feS.b * pv(i + 1, j - 1));
      }
    }
    const double dm = 0.5 * (dqw + dqe), dn = 0.5 * (dqs + dqn);
    const double al = 4.0 + R.Dx[w] * R.Dx[w] + R.Dy[w] * R.Dy[w];
    const double Pb = 1.5 * pc - G.rho * (R.Dx[w] * dm + R.Dy[w] * dn) / (4.0 * dt) +
                      al * R.phi[w] / 4.0;
    const double mn = mt[o] + dm, nn = nt[o] + dn, kn = kt[o] + dt * Pb / G.rho;
    hu[o] = mn;
    hv[o] = nn;
    hw[o] = kn;
    if (p) p[o] = pc;
    if (fold_speed) cell_speed2d(G, idx, idy, ht[o], mn, nn, kn, sp, flags);
  }
  // the tile's speed: its unmarked cells were taken by the mask pass
  if (fold_speed) flush_tile_speed(G, &G.tspeed[tile], sp, flags, true);
}



Sys2 sys_of(Ctx2D* x) {
  Sys2 Y;
  Y.dg = x->dg;
  Y.ce = x->ce;
  Y.cn = x->cn;
  Y.b = x->b;
  Y.x = x->x;
  Y.dg32 = x->dg32;
  Y.ce32 = x->ce32;
  Y.cn32 = x->cn32;
  Y.nb = x->nb;
  Y.cd = x->cd;
  return Y;
}

template <typename R>
PcgArgs<R> pcg_common(const swe_nh_config* c, Ctx2D* x) {
  PcgArgs<R> A;
  A.nx = x->nx;
  A.ny = x->ny;
  A.tiles_x = x->tiles_x;
  A.tiles_y = x->tiles_y;
  A.tile_list = x->tile_list;
  A.n_list = x->n_tiles_act;
  A.tile_cnt = x->tile_cnt;
  A.tflag = x->tflag;
  A.nb = x->nb;
  A.dg = x->dg;
  A.ce = x->ce;
  A.cn = x->cn;
  A.b = x->b;
  A.x = x->x;
  A.part = x->part;
  A.bar.count = x->bar;
  A.bar.status = x->status;
  A.iters = x->iters;
  A.iters_sum = x->iters_sum;
  A.rel = x->rel;
  A.tol = c->tol;
  A.max_iter = c->max_iter;
  A.pipe_blocks = x->grid_pipe;
  A.tile_pos = x->tile_pos;
  A.cinv = x->cinv;
  A.cused = x->cused;
  A.mt[0] = x->mtag[0];
  A.mt[1] = x->mtag[1];
  A.pt = x->pt;
  A.tag_base = x->tag_base;
  A.skip = nullptr;
  A.used = nullptr;
  return A;
}

template <typename R>
void set_vectors(PcgArgs<R>& A, R* const* v) {
  A.r = v[0];
  A.u = v[1];
  A.w = v[2];
  A.z = v[3];
  A.q = v[4];
  A.s = v[5];
  A.p = v[6];
  A.e = v[7];
  A.m[0] = v[8];
  A.m[1] = v[9];
}

PcgArgs<float> pcg_args32(const swe_nh_config* c, Ctx2D* x) {
  PcgArgs<float> A = pcg_common<float>(c, x);
  A.dgR = x->dg32;
  A.ceR = x->ce32;
  A.cnR = x->cn32;
  set_vectors(A, x->v32);
  A.tol_in = 1e-4;  // each FP32 solve reduces the FP64 residual by this factor
  return A;
}

PcgArgs<double> pcg_args64(const swe_nh_config* c, Ctx2D* x) {
  PcgArgs<double> A = pcg_common<double>(c, x);
  A.dgR = x->dg;
  A.ceR = x->ce;
  A.cnR = x->cn;
  set_vectors(A, x->v64);
  A.tol_in = 0.0;
  return A;
}

__global__ void k_copy_masked2d(const double* __restrict__ x, const uint8_t* __restrict__ mask,
                                double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = mask[i] ? x[i] : 0.0;
}

// the tile solver on the system in x (its initial guess in x->x); with
// skip, it returns at once when *skip == 1; it runs at most max_iter
// iterations less *used (when given)
void launch_tile_solve2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, bool coarse,
                         const int* skip, const int* used) {
  hipLaunchKernelGGL(k_bar_reset, dim3((x->ntiles + 255) / 256), dim3(256), 0, s, x->bar, x->tflag,
                     x->ntiles);
  if (coarse) {
    // coarse operator of the active tiles (the inversion exits when there are
    // more than CMAX2 of them, and then the solver does without)
    hipLaunchKernelGGL(k_coarse2d, dim3(std::min(x->ntiles, CMAX2)), dim3(NT2), 0, s, x->nx,
                       x->ny, x->tiles_x, (const int*)x->tile_list, (const int*)x->n_tiles_act,
                       (const uint8_t*)x->nb, (const double*)x->dg, (const double*)x->ce,
                       (const double*)x->cn, x->crow);
    hipLaunchKernelGGL(k_coarse_inv2d, dim3(1), dim3(1024), 0, s, x->tiles_x, x->tiles_y,
                       (const int*)x->tile_list, (const int*)x->n_tiles_act,
                       (const int*)x->tile_pos, (const double*)x->crow, x->cinv, x->cused);
  }
  if (c->precision == 1) {
    PcgArgs<float> A = pcg_args32(c, x);
    A.skip = skip;
    A.used = used;
    hipLaunchKernelGGL(k_pcg2d_pipe<float>, dim3(x->grid_pipe), dim3(NT2), 0, s, A);
    hipLaunchKernelGGL(k_pcg2d_cg<float>, dim3(x->grid_pcg), dim3(NT2), 0, s, A);
  } else {
    PcgArgs<double> A = pcg_args64(c, x);
    A.skip = skip;
    A.used = used;
    hipLaunchKernelGGL(k_pcg2d_pipe<double>, dim3(x->grid_pipe), dim3(NT2), 0, s, A);
    hipLaunchKernelGGL(k_pcg2d_cg<double>, dim3(x->grid_pcg), dim3(NT2), 0, s, A);
  }
}

void launch_solve2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s) {
  const bool mg_off = x->mg_off && !x->tensor && c->crit != SWE_NH_CRIT_GLOBAL;
  if (x->mg_levels > 0 && !mg_off) {
    // the multigrid CG on its box (the whole grid in the global extension,
    // the active tiles' bounding box when they are many) for up to MG_BUDGET
    // iterations (a captured step cannot size a launch sequence by the
    // iteration count); the tile solver takes the step when the multigrid
    // is not chosen, and continues from its iterate when it has not met the
    // tolerance by then
    const bool global = c->crit == SWE_NH_CRIT_GLOBAL;
    if (x->tensor) {
      // the exact-tensor operator: the multigrid CG at every active-tile
      // count (the tile solver's blocks exchange no corner values); a solve
      // that misses the tolerance within MG_TENSOR_FIRST iterations, or whose
      // recursive residual drifted from the true one, is restarted from the
      // true residual of its iterate for the rest of MG_BUDGET_TENSOR
      launch_mg_box2d(x, global, 0, s);
      const int b1 = std::min(c->max_iter, MG_TENSOR_FIRST);
      launch_mg_solve2d(x, c->tol, b1, false, false, s);
      launch_mg_solve2d(x, c->tol, std::min(c->max_iter, MG_BUDGET_TENSOR) - b1, true, true, s);
      return;
    }
    launch_mg_box2d(x, global, MG_MIN_TILES, s);
    launch_mg_solve2d(x, c->tol, std::min(c->max_iter, MG_BUDGET), false, false, s);
    launch_tile_solve2d(c, x, s, !global, &x->mg_args.st->ok, &x->mg_args.st->it);
    launch_mg_account2d(x, s);
    return;
  }
  launch_tile_solve2d(c, x, s, true, nullptr, nullptr);
}

}  // namespace

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
void plan2d(const swe_nh_config* c, char* base, size_t* off, Ctx2D* x) {
  auto take = [&](size_t bytes) -> char* {
    *off = (*off + 255) & ~size_t(255);
    char* p = base ? base + *off : nullptr;
    *off += bytes ? bytes : 1;
    return p;
  };
  const int64_t N = (int64_t)c->nx * c->ny;
  x->nx = c->nx;
  x->ny = c->ny;
  x->tiles_x = (c->nx + TX2 - 1) / TX2;
  x->tiles_y = (c->ny + TY2 - 1) / TY2;
  x->ntiles = x->tiles_x * x->tiles_y;
  x->grid_pcg = x->ntiles < PCG_GMAX ? x->ntiles : PCG_GMAX;
  x->ht = (double*)take(8 * N);
  x->mt = (double*)take(8 * N);
  x->nt = (double*)take(8 * N);
  x->kt = (double*)take(8 * N);
  x->mask_ws = (uint8_t*)take(N);
  x->tile_cnt = (int*)take(4 * x->ntiles);
  x->tspeed = (double*)take(8 * (size_t)x->ntiles);
  x->tile_list = (int*)take(4 * x->ntiles);
  x->tile_pos = (int*)take(4 * x->ntiles);
  x->crow = (double*)take(8 * 5 * (size_t)x->ntiles);
  x->cinv = (double*)take(8 * (size_t)CMAX2 * CMAX2);
  x->cused = (int*)take(4 * (size_t)(CMAX2 + 3));
  x->n_tiles_act = (int*)take(4);
  x->n_act = (int*)take(4);
  x->dg = (double*)take(8 * N);
  x->ce = (double*)take(8 * N);
  x->cn = (double*)take(8 * N);
  x->b = (double*)take(8 * N);
  x->x = (double*)take(8 * N);
  x->nb = (uint8_t*)take(N);
  x->dg32 = (float*)take(4 * N);
  x->ce32 = (float*)take(4 * N);
  x->cn32 = (float*)take(4 * N);
  x->tensor = c->tensor2d;
  x->cd = c->tensor2d ? (double*)take(8 * N) : nullptr;
  for (int k = 0; k < PCG_NVEC; k++) {
    if (c->precision == 1)
      x->v32[k] = (float*)take(4 * N);
    else
      x->v64[k] = (double*)take(8 * N);
  }
  x->part = (double*)take(8 * 2 * 4 * (size_t)PCG_GMAX);
  const size_t tw = c->precision == 1 ? 1 : 2;  // 64-bit words per tagged value
  x->tag_bytes = 8 * (2 * tw * N + 2 * 4 * 2 * (size_t)PCG_GMAX) + 256;
  x->mtag[0] = (unsigned long long*)take(x->tag_bytes);
  x->mtag[1] = x->mtag[0] + tw * N;
  x->pt = x->mtag[1] + tw * N;
  x->tag_base = (unsigned*)take(4);
  x->bar = (unsigned long long*)take(8);
  x->tflag = (unsigned*)take(4 * (size_t)x->ntiles);
  x->iters = (int*)take(4);
  x->iters_sum = (long long*)take(8);
  x->rel = (double*)take(8);
  x->mg_levels = 0;
  if (c->crit != SWE_NH_CRIT_NONE) {
    // CG with a multigrid preconditioner for the global extension and for
    // large active areas, when the grid coarsens to at most MG_COARSE_MAX
    // cells by 2 x 2 aggregation
    x->mg_levels = mg_plan_levels(c->nx, c->ny, x->mg_nx, x->mg_ny);
    const int L = x->mg_levels;
    for (int l = 1; l <= L; l++) {
      const int64_t n = (int64_t)x->mg_nx[l] * x->mg_ny[l];
      x->mg_c[l] = (float*)take(4 * n);
      x->mg_e[l] = (float*)take(4 * n);
      x->mg_n[l] = (float*)take(4 * n);
      x->mg_b[l] = (float*)take(4 * n);
      x->mg_z[l] = (float*)take(4 * n);
    }
    if (L > 0) {
      x->mg_c[0] = x->dg32;
      x->mg_e[0] = x->ce32;
      x->mg_n[0] = x->cn32;
      MgArgs& A = x->mg_args;
      A.nx = c->nx;
      A.ny = c->ny;
      A.dg = x->dg;
      A.ce = x->ce;
      A.cn = x->cn;
      A.cd = x->cd;
      A.b = x->b;
      A.x = x->x;
      A.r = (double*)take(8 * N);
      A.z = (float*)take(4 * N);
      A.q = (double*)take(8 * N);
      A.p[0] = (double*)take(8 * N);
      A.p[1] = (double*)take(8 * N);
      A.npart = mg_partials(c->nx, c->ny);
      A.part = (double*)take(8 * 2 * (size_t)A.npart);
      A.st = (MgState*)take(sizeof(MgState));
      A.iters = x->iters;
      A.iters_sum = x->iters_sum;
      A.rel = x->rel;
    }
  }
  if (c->warm == 2) {
    // the network runs on a window of at most 256 x 256 cells over the active
    // tiles: the pressure's support plus the network's receptive field
    x->crop_w = std::min(c->nx, 256);
    x->crop_h = std::min(c->ny, 256);
    x->cnn_bytes = cnn_layout(1, x->crop_h, x->crop_w).bytes;
    x->cnn_ws = take(x->cnn_bytes);
    x->feat = (uint16_t*)take(2 * 16 * (size_t)x->crop_w * x->crop_h);
    x->guess = (double*)take(8 * N);
    x->crop_org = (int*)take(6 * sizeof(int));
  }
}

int init2d(const swe_nh_config* c, Ctx2D* x, const K1D& k1, hipStream_t s) {
  if (c->warm == 2 && (c->nx % 16 || c->ny % 16)) return SWE_NH_EINVAL;
  x->t = k1.t;
  x->dt = k1.dt;
  x->smax = k1.smax;
  x->status = k1.status;
  x->step = k1.step;
  x->ch = k1.ch;
  x->mg_args.status = k1.status;
  // the persistent solver needs all its blocks resident at once
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SWE_NH_EHIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SWE_NH_EHIP;
  hipError_t e = c->precision == 1
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pcg2d_cg<float>, NT2, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pcg2d_cg<double>, NT2, 0);
  if (e != hipSuccess || per_cu < 1) return SWE_NH_EHIP;
  const int cap = cus * per_cu;
  if (x->grid_pcg > cap) x->grid_pcg = cap;
  int per_cu_p = 0;
  e = c->precision == 1
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_p, k_pcg2d_pipe<float>, NT2, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_p, k_pcg2d_pipe<double>, NT2, 0);
  if (e != hipSuccess || per_cu_p < 1) return SWE_NH_EHIP;
  // the pipelined grid: enough blocks for every active tile at PCG_K per block
  // when possible, never more than fit at once
  x->grid_pipe = std::min(cus * per_cu_p, std::min(PCG_GMAX, (x->ntiles + PCG_K - 1) / PCG_K));
  int zi[2] = {0, 0};
  if (hipMemcpy(x->n_tiles_act, zi, 4, hipMemcpyHostToDevice) != hipSuccess) return SWE_NH_EHIP;
  if (hipMemcpy(x->n_act, zi, 4, hipMemcpyHostToDevice) != hipSuccess) return SWE_NH_EHIP;
  if (hipMemcpy(x->iters, zi, 4, hipMemcpyHostToDevice) != hipSuccess) return SWE_NH_EHIP;
  // the network's buffers start at zero: tiles of the window it skips keep
  // finite values
  if (x->cnn_ws && hipMemset(x->cnn_ws, 0, x->cnn_bytes) != hipSuccess) return SWE_NH_EHIP;
  const long long zl = 0;
  if (hipMemcpy(x->iters_sum, &zl, 8, hipMemcpyHostToDevice) != hipSuccess) return SWE_NH_EHIP;
  // tagged words start with tag 0, which no pass uses (tags start at 2)
  if (hipMemset(x->mtag[0], 0, x->tag_bytes) != hipSuccess) return SWE_NH_EHIP;
  const unsigned one = 1;
  if (hipMemcpy(x->tag_base, &one, 4, hipMemcpyHostToDevice) != hipSuccess) return SWE_NH_EHIP;
  const int none[3] = {-1, 0, 0};  // no coarse inverse yet
  if (hipMemcpy(x->cused, none, sizeof(none), hipMemcpyHostToDevice) != hipSuccess)
    return SWE_NH_EHIP;
  (void)s;
  return SWE_NH_OK;
}

// origin of the network's w x h window, centred on the bounding box of the
// active tiles and inside the grid, and the part of the window the network
// computes: that box, widened by 16 cells (more than the 6-cell receptive
// field of the six 3 x 3 layers, so the values on the active tiles are those
// of the whole window).  org = (i0, j0, x0, y0, x1, y1).  One block.
__global__ void __launch_bounds__(256) k_crop2d(const int* tile_list, const int* n_list,
                                                int tiles_x, int nx, int ny, int w, int h,
                                                int* org) {
  __shared__ int lo[2][256 / 64], hi[2][256 / 64];
  const int nl = *n_list;
  int bx0 = 1 << 30, by0 = 1 << 30, bx1 = -1, by1 = -1;
  for (int t = threadIdx.x; t < nl; t += 256) {
    const int tile = tile_list[t], tx = tile % tiles_x, ty = tile / tiles_x;
    bx0 = min(bx0, tx);
    bx1 = max(bx1, tx);
    by0 = min(by0, ty);
    by1 = max(by1, ty);
  }
  for (int o = 32; o > 0; o >>= 1) {
    bx0 = min(bx0, __shfl_xor(bx0, o));
    by0 = min(by0, __shfl_xor(by0, o));
    bx1 = max(bx1, __shfl_xor(bx1, o));
    by1 = max(by1, __shfl_xor(by1, o));
  }
  if ((threadIdx.x & 63) == 0) {
    lo[0][threadIdx.x >> 6] = bx0;
    lo[1][threadIdx.x >> 6] = by0;
    hi[0][threadIdx.x >> 6] = bx1;
    hi[1][threadIdx.x >> 6] = by1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 256 / 64; k++) {
      bx0 = min(bx0, lo[0][k]);
      by0 = min(by0, lo[1][k]);
      bx1 = max(bx1, hi[0][k]);
      by1 = max(by1, hi[1][k]);
    }
    int i0 = 0, j0 = 0;
    if (nl > 0) {
      const int cx = ((bx0 + bx1 + 1) * TX2) / 2, cy = ((by0 + by1 + 1) * TY2) / 2;
      i0 = min(max(cx - w / 2, 0), nx - w);
      j0 = min(max(cy - h / 2, 0), ny - h);
    }
    org[0] = i0;
    org[1] = j0;
    if (nl > 0) {
      org[2] = max(bx0 * TX2 - 16 - i0, 0);
      org[3] = max(by0 * TY2 - 16 - j0, 0);
      org[4] = min((bx1 + 1) * TX2 + 16 - i0, w);
      org[5] = min((by1 + 1) * TY2 + 16 - j0, h);
    } else {
      org[2] = org[3] = org[4] = org[5] = 0;
    }
  }
}

// the guess on the marked cells of the active tiles: scale * network output
// inside the window, 0 outside it
__global__ void __launch_bounds__(NT2) k_guess2d(const float* __restrict__ out,
                                                 const int* org, int w, int h,
                                                 const uint8_t* __restrict__ mask,
                                                 const int* tile_list, const int* n_list,
                                                 int tiles_x, int nx, int ny, double scale,
                                                 double* __restrict__ guess) {
  if ((int)blockIdx.x >= *n_list) return;
  const int tile = tile_list[blockIdx.x];
  const int i0 = (tile % tiles_x) * TX2, j0 = (tile / tiles_x) * TY2;
  const int ox = org[0], oy = org[1];
  for (int cc = threadIdx.x; cc < TN; cc += NT2) {
    const int i = i0 + cc % TX2, j = j0 + cc / TX2;
    if (i >= nx || j >= ny) continue;
    const int64_t g = (int64_t)j * nx + i;
    if (!mask[g]) continue;
    const int li = i - ox, lj = j - oy;
    guess[g] = (li >= 0 && li < w && lj >= 0 && lj < h)
                   ? scale * (double)out[(int64_t)lj * w + li] : 0.0;
  }
}

static void enqueue_nh2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
                         const double* mt, const double* nt, const double* kt,
                         const uint8_t* mask, const double* t_in, const double* dt_in,
                         const double* p_prev, double* hu, double* hv, double* hw, double* p,
                         bool tiles_ready = false) {
  const G2 G = make_g2(c, x);
  if (!tiles_ready)
    hipLaunchKernelGGL(k_tiles2d, dim3(1), dim3(1024), 0, s, x->tile_cnt, x->ntiles, x->tile_list,
                       x->n_tiles_act, x->n_act, x->tile_pos);
  hipLaunchKernelGGL(k_assemble2d, dim3(x->ntiles), dim3(NT2), 0, s, G, ht, mt, nt, kt, mask,
                     x->tile_list, x->n_tiles_act, t_in, dt_in, sys_of(x), p_prev,
                     (int)(p_prev != nullptr));
  launch_solve2d(c, x, s);
  if (hu)
    hipLaunchKernelGGL(k_correct2d, dim3(x->ntiles), dim3(NT2), 0, s, G, ht, mt, nt, kt, mask,
                       x->tile_list, x->n_tiles_act, t_in, dt_in, x->x, hu, hv, hw, p, 1);
}

void enqueue_step2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, double* h, double* hu,
                    double* hv, double* hw, double* p, uint8_t* mask) {
  const G2 G = make_g2(c, x);
  uint8_t* M = mask ? mask : x->mask_ws;
  hipLaunchKernelGGL(k_pred2d, dim3(x->ntiles), dim3(NTP), 0, s, G, h, hu, hv, hw, x->ht, x->mt,
                     x->nt, x->kt, (const double*)x->t, (const double*)x->dt, 1);
  // the mask pass clears p only off the new marked area: p keeps the previous
  // pressure where it is needed as the initial guess
  hipLaunchKernelGGL(k_mask2d, dim3(x->ntiles), dim3(NT2), 0, s, G, x->ht, x->mt, x->nt, x->kt,
                     (const double*)x->t, (const double*)x->dt, -1, M, x->tile_cnt, h, hu, hv,
                     hw, p, 1);
  if (c->crit != SWE_NH_CRIT_NONE) {
    const double* guess = c->warm == 1 ? p : nullptr;
    bool tiles_ready = false;
    if (c->warm == 2 && x->net) {
      // the network on its window over the active tiles; the guess is read
      // only on their marked cells
      hipLaunchKernelGGL(k_tiles2d, dim3(1), dim3(1024), 0, s, x->tile_cnt, x->ntiles,
                         x->tile_list, x->n_tiles_act, x->n_act, x->tile_pos);
      tiles_ready = true;
      const int w = x->crop_w, hh = x->crop_h;
      hipLaunchKernelGGL(k_crop2d, dim3(1), dim3(256), 0, s, (const int*)x->tile_list,
                         (const int*)x->n_tiles_act, x->tiles_x, x->nx, x->ny, w, hh, x->crop_org);
      const CnnLayout L = cnn_layout(1, hh, w);
      cnn_features(x->ch, c->depth_static, x->nx, x->ny, c->dx, c->dy, x->fscale, x->t, x->dt,
                   x->ht, x->mt, x->nt, M, x->feat, s, x->crop_org, w, hh);
      float* out = reinterpret_cast<float*>(x->cnn_ws + L.out);
      cnn_forward(x->net, x->feat, 1, hh, w, x->cnn_ws, L, out, s, x->crop_org + 2);
      hipLaunchKernelGGL(k_guess2d, dim3(x->ntiles), dim3(NT2), 0, s, (const float*)out,
                         (const int*)x->crop_org, w, hh, (const uint8_t*)M,
                         (const int*)x->tile_list, (const int*)x->n_tiles_act, x->tiles_x, x->nx,
                         x->ny, x->p_scale, x->guess);
      guess = x->guess;
    }
    enqueue_nh2d(c, x, s, x->ht, x->mt, x->nt, x->kt, M, x->t, x->dt, guess, hu, hv, hw, p,
                 tiles_ready);
  } else {
    hipLaunchKernelGGL(k_tiles2d, dim3(1), dim3(1024), 0, s, x->tile_cnt, x->ntiles, x->tile_list,
                       x->n_tiles_act, x->n_act, x->tile_pos);
  }
  // the new state's speed (tiles written by the mask pass and the projection)
  // -> dt of the next step; time and step counter advance
  hipLaunchKernelGGL(k_speed_reduce2d, dim3(1), dim3(1024), 0, s, G, x->ntiles, 1);
}

void pack_net2d(Ctx2D* x, hipStream_t s) {
  if (x->net && x->cnn_ws)
    cnn_pack_weights(x->net, x->cnn_ws, cnn_layout(1, x->crop_h, x->crop_w), false, s);
}

void launch_speed2d_prologue(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* h,
                             const double* hu, const double* hv, const double* hw) {
  const G2 G = make_g2(c, x);
  hipLaunchKernelGGL(k_speed2d, dim3(x->ntiles), dim3(NT2), 0, s, G, h, hu, hv, hw);
  hipLaunchKernelGGL(k_speed_reduce2d, dim3(1), dim3(1024), 0, s, G, x->ntiles, 0);
}

void launch_pred2d_stage(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* h,
                         const double* hu, const double* hv, const double* hw, const double* t_in,
                         const double* dt_in, double* ht, double* mt, double* nt, double* kt) {
  hipLaunchKernelGGL(k_pred2d, dim3(x->ntiles), dim3(NTP), 0, s, make_g2(c, x), h, hu, hv, hw, ht,
                     mt, nt, kt, t_in, dt_in, 0);
}

void launch_mask2d_stage(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
                         const double* mt, const double* nt, const double* kt,
                         const double* t_in, const double* dt_in, int mode, uint8_t* mask) {
  const G2 G = make_g2(c, x);
  hipLaunchKernelGGL(k_mask2d, dim3(x->ntiles), dim3(NT2), 0, s, G, ht, mt, nt, kt, t_in,
                     dt_in, mode, mask, x->tile_cnt, nullptr, nullptr, nullptr, nullptr, nullptr,
                     0);
  hipLaunchKernelGGL(k_tiles2d, dim3(1), dim3(1024), 0, s, x->tile_cnt, x->ntiles, x->tile_list,
                     x->n_tiles_act, x->n_act, x->tile_pos);
}

void solve_pressure2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
                      const double* mt, const double* nt, const double* kt, const uint8_t* mask,
                      const double* t_in, const double* dt_in, double* p) {
  const G2 G = make_g2(c, x);
  const int64_t N = (int64_t)x->nx * x->ny;
  hipLaunchKernelGGL(k_count2d, dim3(x->ntiles), dim3(NT2), 0, s, G, mask, x->tile_cnt);
  enqueue_nh2d(c, x, s, ht, mt, nt, kt, mask, t_in, dt_in, c->warm == 1 ? p : nullptr, nullptr,
               nullptr, nullptr, nullptr);
  // p = x on the marked cells, 0 elsewhere
  hipLaunchKernelGGL(k_copy_masked2d, dim3(2048), dim3(256), 0, s, (const double*)x->x, mask, p,
                     N);
}

void correct2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, const double* ht,
               const double* mt, const double* nt, const double* kt, const uint8_t* mask,
               const double* p, const double* t_in, const double* dt_in, double* m_out,
               double* n_out, double* k_out) {
  const G2 G = make_g2(c, x);
  const int64_t N = (int64_t)x->nx * x->ny;
  hipLaunchKernelGGL(k_count2d, dim3(x->ntiles), dim3(NT2), 0, s, G, mask, x->tile_cnt);
  hipLaunchKernelGGL(k_tiles2d, dim3(1), dim3(1024), 0, s, x->tile_cnt, x->ntiles, x->tile_list,
                     x->n_tiles_act, x->n_act, x->tile_pos);
  launch_copy(mt, m_out, N, s);
  launch_copy(nt, n_out, N, s);
  launch_copy(kt, k_out, N, s);
  hipLaunchKernelGGL(k_correct2d, dim3(x->ntiles), dim3(NT2), 0, s, G, ht, mt, nt, kt, mask,
                     x->tile_list, x->n_tiles_act, t_in, dt_in, p, m_out, n_out, k_out, nullptr,
                     0);
}

void time_stage2d(const swe_nh_config* c, Ctx2D* x, hipStream_t s, int stage, double* h,
                  double* hu, double* hv, double* hw, double* p) {
  const G2 G = make_g2(c, x);
  switch (stage) {
    case 0:
      hipLaunchKernelGGL(k_pred2d, dim3(x->ntiles), dim3(NTP), 0, s, G, h, hu, hv, hw, x->ht,
                         x->mt, x->nt, x->kt, (const double*)x->t, (const double*)x->dt, 0);
      break;
    case 1:
      hipLaunchKernelGGL(k_mask2d, dim3(x->ntiles), dim3(NT2), 0, s, G, x->ht, x->mt, x->nt, x->kt,
                         (const double*)x->t, (const double*)x->dt, 0, x->mask_ws, x->tile_cnt,
                         nullptr, nullptr, nullptr, nullptr, nullptr, 0);
      break;
    case 2:
      launch_solve2d(c, x, s);
      break;
    default:
      hipLaunchKernelGGL(k_correct2d, dim3(x->ntiles), dim3(NT2), 0, s, G, x->ht, x->mt, x->nt,
                         x->kt, x->mask_ws, x->tile_list, x->n_tiles_act, (const double*)x->t,
                         (const double*)x->dt, x->x, hu, hv, hw, p, 0);
  }
}

}  // namespace swenh
