// swe_nh_1d.hip -- 1D kernels of the non-hydrostatic SWE step (gfx950).
//
// Layout: all channels packed back to back in one FP64 array per field; a
// launch tile is 32..512 consecutive cells of one channel (tile table built on
// the host).  Kernels never read across a channel end: the two ghost cells
// on each side are reflections of the channel's own cells.
//
//   k_speed1d   max |u| + sqrt(g h) per channel (atomic max on the bit
//               pattern into the channel's speed slots, exact) and state
//               checks -> dt (Sec. 3.1 CFL rule)
//   k_pred1d    both Heun stages (Eqs. 8-9) of the hydrostatic FV operator
//               fused in LDS with a 4-cell halo
//   k_mask1d    criterion (Sec. 5.1) + enlargement (Sec. 5.2), tile counts
//   k_scan      exclusive scan of tile counts (single block)
//   k_compact1d packed list of marked cells (wave ballots)
//   k_assemble1d / k_correct1d  elliptic system of Eqs. 12-17 and the
//               projection of Eqs. 10-11 on the packed rows
#include "swe_nh_common.h"
#include "swe_nh_kernels.h"

namespace swenh {

// maximum wave speed of channel ch in speed buffer q: the maximum of its
// slots, returned to every lane of the calling wavefront
__device__ __forceinline__ double read_speed(const K1D& P, int q, int ch) {
  const unsigned long long* s = P.smax + speed_at(q * P.nch + ch, 0, P.nslot);
  const int k = (threadIdx.x & 63) & (P.nslot - 1);
  double v = __longlong_as_double((long long)s[(size_t)k * SPEED_PAD]);
  for (int o = P.nslot >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// wave speed and state check
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_speed1d(K1D P, const double* __restrict__ h,
                                                 const double* __restrict__ hu,
                                                 const double* __restrict__ hw) {
  const int4 tl = P.tiles[blockIdx.x];
  const Chan c = P.ch[tl.x];
  const int end = min(tl.y + P.tile, c.n);
  double s = 0.0;
  int flags = 0;
  for (int i = tl.y + threadIdx.x; i < end; i += blockDim.x) {
    const int64_t gi = c.off + i;
    const double hh = h[gi], mm = hu[gi], kk = hw[gi];
    if (!isfinite(hh) || !isfinite(mm) || !isfinite(kk)) {
      flags |= ST_NAN;
    } else if (!(hh > 0.0)) {
      flags |= ST_DRY;
    } else {
      s = fmax(s, fabs(mm / hh) + sqrt64(P.g * hh));
    }
  }
  s = wave_max(s);
  __shared__ double red[4];
  __shared__ int fl;
  if (threadIdx.x == 0) fl = 0;
  __syncthreads();
  if (flags) atomicOr(&fl, flags);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(&P.smax[speed_at(tl.x, blockIdx.x & (P.nslot - 1), P.nslot)], pos_bits(m));
    if (fl) atomicOr(P.status, fl);
  }
}

// ---------------------------------------------------------------------------
// hydrostatic predictor
// ---------------------------------------------------------------------------
struct Flux {
  double Fh, FmL, FmR, Fk, hL, hR;
  bool dry;
};

// Rusanov flux between hydrostatically reconstructed states (Audusse et al.
// 2004 reconstruction; Rusanov solver as in Sec. 3.1)
__device__ __forceinline__ Flux rusanov1d(double g, double eL, double mL, double kL, double dL,
                                          double eR, double mR, double kR, double dR) {
  Flux f;
  const double hL = eL + dL, hR = eR + dR;
  f.dry = !(hL > 0.0) || !(hR > 0.0);
  const double rL = rcp64(hL), rR = rcp64(hR);
  const double uL = mL * rL, uR = mR * rR;
  const double wL = kL * rL, wR = kR * rR;
  const double db = fmin(dL, dR);
  const double sL = fmax(0.0, eL + db), sR = fmax(0.0, eR + db);
  const double lam = fmax(fabs(uL) + sqrt64(g * sL), fabs(uR) + sqrt64(g * sR));
  const double qL = sL * uL, qR = sR * uR;
  const double pL = 0.5 * g * sL * sL, pR = 0.5 * g * sR * sR;
  f.Fh = 0.5 * (qL + qR) - 0.5 * lam * (sR - sL);
  const double Fm = 0.5 * (qL * uL + pL + qR * uR + pR) - 0.5 * lam * (qR - qL);
  f.FmL = Fm + 0.5 * g * (hL * hL - sL * sL);
  f.FmR = Fm + 0.5 * g * (hR * hR - sR * sR);
  f.Fk = 0.5 * (qL * wL + qR * wR) - 0.5 * lam * (sR * wR - sL * wL);
  f.hL = hL;
  f.hR = hR;
  return f;
}

namespace {
constexpr int HALO = 4;

// LDS of the fused predictor for a tile of T cells (window of T + 8)
template <int T>
struct PredSmem {
  static constexpr int WIN = T + 2 * HALO;
  double e[WIN], m[WIN], k[WIN], d0[WIN], d1[WIN];  // working state, depth at t^n and t^n+1
  double Fh[WIN], FmL[WIN], FmR[WIN], Fk[WIN], hL[WIN], hR[WIN];  // face fluxes
};

// face fluxes of one stage for faces f in [f0, f1) (face f between window
// cells f-1 and f); d: depth of the stage
template <int T>
__device__ __forceinline__ void stage_faces(PredSmem<T>& S, const double* d, double g, int f0,
                                            int f1, int lo_cell, int hi_cell, int base,
                                            int* flags) {
  for (int f = f0 + threadIdx.x; f < f1; f += blockDim.x) {
    const int l = f - 1, r = f;
    const double se_l = minmod(S.e[l] - S.e[l - 1], S.e[l + 1] - S.e[l]);
    const double sm_l = minmod(S.m[l] - S.m[l - 1], S.m[l + 1] - S.m[l]);
    const double sk_l = minmod(S.k[l] - S.k[l - 1], S.k[l + 1] - S.k[l]);
    const double sd_l = minmod(d[l] - d[l - 1], d[l + 1] - d[l]);
    const double se_r = minmod(S.e[r] - S.e[r - 1], S.e[r + 1] - S.e[r]);
    const double sm_r = minmod(S.m[r] - S.m[r - 1], S.m[r + 1] - S.m[r]);
    const double sk_r = minmod(S.k[r] - S.k[r - 1], S.k[r + 1] - S.k[r]);
    const double sd_r = minmod(d[r] - d[r - 1], d[r + 1] - d[r]);
    const Flux F = rusanov1d(g, S.e[l] + 0.5 * se_l, S.m[l] + 0.5 * sm_l, S.k[l] + 0.5 * sk_l,
                             d[l] + 0.5 * sd_l, S.e[r] - 0.5 * se_r, S.m[r] - 0.5 * sm_r,
                             S.k[r] - 0.5 * sk_r, d[r] - 0.5 * sd_r);
    S.Fh[f] = F.Fh;
    S.FmL[f] = F.FmL;
    S.FmR[f] = F.FmR;
    S.Fk[f] = F.Fk;
    S.hL[f] = F.hL;
    S.hR[f] = F.hR;
    // only faces touching a channel cell of this stage's range count
    const int il = base + l, ir = base + r;
    const bool used = (il >= lo_cell && il < hi_cell) || (ir >= lo_cell && ir < hi_cell);
    if (F.dry && used) *flags |= ST_DRY;
  }
}

template <int T>
__device__ __forceinline__ void stage_cell(const PredSmem<T>& S, const double* d, double g,
                                           double idx, int e, double& Lh, double& Lm,
                                           double& Lk) {
  const double sd = minmod(d[e] - d[e - 1], d[e + 1] - d[e]);
  Lh = -(S.Fh[e + 1] - S.Fh[e]) * idx;
  Lm = -(S.FmL[e + 1] - S.FmR[e]) * idx + g * 0.5 * (S.hL[e + 1] + S.hR[e]) * sd * idx;
  Lk = -(S.Fk[e + 1] - S.Fk[e]) * idx;
}
}  // namespace

namespace {
// The body's motion at t0 and t1, evaluated by the first and the second
// wavefront of the block and shared through LDS: it is the same for every
// cell of a tile, so a block needs one evaluation per time, not one per
// wavefront.  Contains a block barrier; needs at least two wavefronts.
__device__ __forceinline__ void block_motions(const Chan& c, double t0, double t1, Motion& M0,
                                              Motion& M1) {
  __shared__ Motion slot[2];
  const int wv = threadIdx.x >> 6;
  if (wv < 2) {
    const Motion m = body_motion(c, wv == 0 ? t0 : t1);
    if ((threadIdx.x & 63) == 0) slot[wv] = m;
  }
  __syncthreads();
  M0 = slot[0];
  M1 = slot[1];
}

// the fused step's time step (from the channel's speed slots) and the body's
// motion at t^n (wavefront 0) and t^{n+1} (wavefront 1, which also reduces
// the speed slots), shared through LDS; needs at least two wavefronts
__device__ __forceinline__ void block_step_motions(const K1D& P, int par, int ch, const Chan& c,
                                                   double t0, double& dt, Motion& M0,
                                                   Motion& M1) {
  __shared__ Motion slot[2];
  __shared__ double sdt;
  const int wv = threadIdx.x >> 6;
  if (wv < 2) {
    double d = 0.0;
    if (wv == 1) d = (P.cfl > 0.0) ? P.cfl * P.dx / read_speed(P, par, ch) : P.dt_fixed;
    const Motion m = body_motion(c, wv == 0 ? t0 : t0 + d);
    if ((threadIdx.x & 63) == 0) {
      slot[wv] = m;
      if (wv == 1) sdt = d;
    }
  }
  __syncthreads();
  dt = sdt;
  M0 = slot[0];
  M1 = slot[1];
}

}  // namespace

// Both Heun stages for a tile of at most T cells.  Thread t owns the window
// cells e = 2 + t + NT q of the stage-1 range [2, tile + 6): their Q^n and stage-1
// operator stay in registers for the final combination on the tile cells.
template <int T, int NT>
__global__ void __launch_bounds__(NT) k_pred1d(K1D P, const double* __restrict__ h,
                                               const double* __restrict__ hu,
                                               const double* __restrict__ hw,
                                               double* __restrict__ ht, double* __restrict__ mt,
                                               double* __restrict__ kt, const double* t_in,
                                               const double* dt_in, int dt_from_speed) {
  constexpr int R1 = T + 4;  // stage-1 cells at most: window [2, tile + 6)
  constexpr int Q = (R1 + NT - 1) / NT;
  __shared__ PredSmem<T> S;
  __shared__ int sflags;
  const int4 tl = P.tiles[blockIdx.x];
  const Chan c = P.ch[tl.x];
  const int n = c.n, start = tl.y, base = start - HALO;  // window cell e <-> channel cell base+e
  const int end = min(start + P.tile, n);
  const int WIN = P.tile + 2 * HALO;  // window of this tile length
  const double t0 = t_in[tl.x];
  double dt;
  if (dt_from_speed) {
    dt = (P.cfl > 0.0) ? P.cfl * P.dx / read_speed(P, 0, tl.x) : P.dt_fixed;
    if (blockIdx.x == P.first_tile[tl.x] && threadIdx.x == 0) P.dt[tl.x] = dt;
  } else {
    dt = dt_in[tl.x];
  }
  const double t1 = t0 + dt;
  Motion M0, M1;
  block_motions(c, t0, t1, M0, M1);
  const double idx = 1.0 / P.dx;
  if (threadIdx.x == 0) sflags = 0;
  int flags = 0;

  // load Q^n on the window with reflected ghosts; depth at both stage times
  for (int e = threadIdx.x; e < WIN; e += NT) {
    const int i = min(base + e, n + HALO - 1);
    const int s = reflect(i, n);
    const int64_t gi = c.off + s;
    const double x = (s + 0.5) * P.dx;
    const double ds = P.ds[gi];
    const double dA = ds - body_shape(c, x - M0.X, 0.0).B;
    S.e[e] = h[gi] - dA;
    S.m[e] = (s == i ? 1.0 : -1.0) * hu[gi];
    S.k[e] = hw[gi];
    S.d0[e] = dA;
    S.d1[e] = ds - body_shape(c, x - M1.X, 0.0).B;
  }
  __syncthreads();

  double Qn[Q][3], L1[Q][3];
  // stage 1: faces [2, WIN - 1), cells [2, WIN - 2)
  const int lo1 = max(0, start - 2), hi1 = min(n, start + P.tile + 2);
  stage_faces<T>(S, S.d0, P.g, 2, WIN - 1, lo1, hi1, base, &flags);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const int e = 2 + threadIdx.x + NT * q;
    Qn[q][0] = Qn[q][1] = Qn[q][2] = 0.0;
    L1[q][0] = L1[q][1] = L1[q][2] = 0.0;
    if (e < WIN - 2) {
      stage_cell<T>(S, S.d0, P.g, idx, e, L1[q][0], L1[q][1], L1[q][2]);
      Qn[q][0] = S.e[e] + S.d0[e];
      Qn[q][1] = S.m[e];
      Qn[q][2] = S.k[e];
    }
  }
  __syncthreads();
  // Q* = Q^n + dt L(Q^n, t^n) on the channel cells of the range
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const int e = 2 + threadIdx.x + NT * q;
    const int i = base + e;
    if (e < WIN - 2 && i >= 0 && i < n) {
      S.e[e] = Qn[q][0] + dt * L1[q][0] - S.d1[e];
      S.m[e] = Qn[q][1] + dt * L1[q][1];
      S.k[e] = Qn[q][2] + dt * L1[q][2];
    }
  }
  __syncthreads();
  // ghosts of Q*: reflections of channel cells (h and hw even, hu odd)
  for (int e = threadIdx.x; e < WIN; e += NT) {
    const int i = base + e;
    if (i >= 0 && i < n) continue;
    const int s = reflect(min(i, n + HALO - 1), n);
    const int es = s - base;
    double ev = 0.0, mv = 0.0, kv = 0.0;
    if (es >= 2 && es < WIN - 2) {
      ev = S.e[es];
      mv = -S.m[es];
      kv = S.k[es];
    }
    S.e[e] = ev;
    S.m[e] = mv;
    S.k[e] = kv;
  }
  __syncthreads();

  // stage 2 on the tile cells: faces [HALO, HALO + tile + 1)
  stage_faces<T>(S, S.d1, P.g, HALO, HALO + P.tile + 1, start, end, base, &flags);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const int e = 2 + threadIdx.x + NT * q;
    const int i = base + e;
    if (e < HALO || e >= HALO + P.tile || i >= end) continue;
    double a, b, k2;
    stage_cell<T>(S, S.d1, P.g, idx, e, a, b, k2);
    const int64_t gi = c.off + i;
    ht[gi] = Qn[q][0] + 0.5 * dt * (L1[q][0] + a);
    mt[gi] = Qn[q][1] + 0.5 * dt * (L1[q][1] + b);
    kt[gi] = Qn[q][2] + 0.5 * dt * (L1[q][2] + k2);
  }
  if (flags) atomicOr(&sflags, flags);
  __syncthreads();
  if (threadIdx.x == 0 && sflags) atomicOr(P.status, sflags);
}

// ---------------------------------------------------------------------------
// criterion, enlargement, tile counts
// ---------------------------------------------------------------------------
namespace {
constexpr int MAXE = 64;  // largest supported enlargement

__device__ __forceinline__ double eta_at(const K1D& P, const Chan& c, const Motion& M,
                                         const double* ht, int i) {
  const int s = reflect(i, c.n);
  const double x = (s + 0.5) * P.dx;
  return ht[c.off + s] - (P.ds[c.off + s] - body_shape(c, x - M.X, 0.0).B);
}

// indicator of Sec. 5.1 at channel cell i (central differences, reflected ghosts)
__device__ double indicator1d(const K1D& P, const Chan& c, const Motion& M, const double* ht,
                              const double* mt, const double* kt, int i, int crit) {
  const int n = c.n;
  const int64_t o = c.off;
  switch (crit) {
    case SWE_NH_CRIT_ETA_D: {
      const double x = (i + 0.5) * P.dx;
      const double d = P.ds[o + i] - body_shape(c, x - M.X, 0.0).B;
      return fabs((ht[o + i] - d) / d);
    }
    case SWE_NH_CRIT_ETA_X:
      return fabs((eta_at(P, c, M, ht, i + 1) - eta_at(P, c, M, ht, i - 1)) / (2.0 * P.dx));
    case SWE_NH_CRIT_U:
      return fabs(mt[o + i] / ht[o + i]);
    case SWE_NH_CRIT_U_X: {
      const int l = reflect(i - 1, n), r = reflect(i + 1, n);
      const double ul = (l == i - 1 ? 1.0 : -1.0) * mt[o + l] / ht[o + l];
      const double ur = (r == i + 1 ? 1.0 : -1.0) * mt[o + r] / ht[o + r];
      return fabs((ur - ul) / (2.0 * P.dx));
    }
    case SWE_NH_CRIT_W:
      return fabs(kt[o + i] / ht[o + i]);
    default: {
      const int l = reflect(i - 1, n), r = reflect(i + 1, n);
      return fabs((kt[o + r] / ht[o + r] - kt[o + l] / ht[o + l]) / (2.0 * P.dx));
    }
  }
}
}  // namespace

// mode: 0 criterion, 1 every cell, 2 no cell.  When write_state != 0 the
// step's defaults are written too: h = h~, hu = hu~, hw = hw~ everywhere and
// p = 0 off the marked area (the projection then overwrites marked cells).
__global__ void __launch_bounds__(256) k_mask1d(K1D P, const double* __restrict__ ht,
                                                const double* __restrict__ mt,
                                                const double* __restrict__ kt,
                                                const double* t_in, const double* dt_in,
                                                int mode_override, uint8_t* __restrict__ mask,
                                                double* h, double* hu, double* hw, double* p,
                                                int write_state) {
  __shared__ uint8_t raw[TILE_MAX + 2 * MAXE];
  __shared__ int cnt[4];
  const int4 tl = P.tiles[blockIdx.x];
  const Chan c = P.ch[tl.x];
  const int n = c.n, start = tl.y, end = min(start + P.tile, n);
  const int e = P.enlarge;
  int mode = mode_override;
  if (mode < 0) {  // step: decide from the criterion and the step counter
    const bool wcrit = (P.crit == SWE_NH_CRIT_W || P.crit == SWE_NH_CRIT_W_X);
    if (P.crit == SWE_NH_CRIT_GLOBAL || (wcrit && P.first_global && *P.step == 0))
      mode = 1;
    else if (P.crit == SWE_NH_CRIT_NONE)
      mode = 2;
    else
      mode = 0;
  }
  if (mode == 0) {
    const double t1 = t_in[tl.x] + dt_in[tl.x];
    const Motion M = body_motion(c, t1);
    for (int w = threadIdx.x; w < P.tile + 2 * e; w += blockDim.x) {
      const int i = start - e + w;
      uint8_t r = 0;
      if (i >= 0 && i < n) r = indicator1d(P, c, M, ht, mt, kt, i, P.crit) > P.k_nh;
      raw[w] = r;
    }
    __syncthreads();
  }
  int local = 0;
  for (int i = start + threadIdx.x; i < end; i += blockDim.x) {
    uint8_t v;
    if (mode == 1) {
      v = 1;
    } else if (mode == 2) {
      v = 0;
    } else {
      v = 0;
      const int w0 = i - start;  // raw index of cell i - e
      for (int j = 0; j <= 2 * e; j++) v |= raw[w0 + j];
    }
    const int64_t gi = c.off + i;
    mask[gi] = v;
    local += v;
    if (write_state) {
      h[gi] = ht[gi];
      hu[gi] = mt[gi];
      hw[gi] = kt[gi];
      if (!v) p[gi] = 0.0;
    }
  }
  local = wave_sum_i(local);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) P.tile_cnt[blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// tile counts of a caller-supplied mask
__global__ void __launch_bounds__(256) k_count1d(K1D P, const uint8_t* __restrict__ mask) {
  __shared__ int cnt[4];
  const int4 tl = P.tiles[blockIdx.x];
  const Chan c = P.ch[tl.x];
  const int end = min(tl.y + P.tile, c.n);
  int local = 0;
  for (int i = tl.y + threadIdx.x; i < end; i += blockDim.x) local += mask[c.off + i] ? 1 : 0;
  local = wave_sum_i(local);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) P.tile_cnt[blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// exclusive scan of cnt[0..n) into off, total into *total: one block of 1024
// threads walks the array in chunks of 4096 (each thread scans 4 consecutive
// counts, the wavefronts scan the thread sums with shuffles, 16 wavefront
// sums are scanned by the first wavefront) and a running carry joins them
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ cnt, int* __restrict__ off,
                                               int n, int* total) {
  __shared__ int wsum[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += 4096) {
    const int i0 = base + 4 * (int)threadIdx.x;
    int v[4];
#pragma unroll
    for (int j = 0; j < 4; j++) v[j] = i0 + j < n ? cnt[i0 + j] : 0;
    const int ts = v[0] + v[1] + v[2] + v[3];
    int x = ts;  // inclusive scan of the thread sums within the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (wv == 0) {
      int w = lane < 16 ? wsum[lane] : 0;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const int y = __shfl_up(w, o, 64);
        if (lane >= o) w += y;
      }
      if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    int run = carry + (wv > 0 ? wsum[wv - 1] : 0) + x - ts;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (i0 + j < n) off[i0 + j] = run;
      run += v[j];
    }
    carry += wsum[15];
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (threadIdx.x == 0) *total = carry;
}

// packed list of marked cells in cell order
__global__ void __launch_bounds__(256) k_compact1d(K1D P, const uint8_t* __restrict__ mask) {
  __shared__ int wsum[4];
  const int4 tl = P.tiles[blockIdx.x];
  const Chan c = P.ch[tl.x];
  const int end = min(tl.y + P.tile, c.n);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int base = P.tile_off[blockIdx.x];
  for (int r0 = tl.y; r0 < end; r0 += blockDim.x) {
    const int i = r0 + threadIdx.x;
    const bool on = (i < end) && mask[c.off + i];
    const unsigned long long bal = __ballot(on);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(bal);
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wv; w++) wbase += wsum[w];
    if (on) {
      const int k = base + wbase + pre;
      P.act_cell[k] = (int)(c.off + i);
      P.act_chan[k] = tl.x;
    }
    base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// elliptic system on the packed rows
// ---------------------------------------------------------------------------
namespace {
struct CellNH {
  double D, al, phi;
};
struct FaceNH {
  double K, a, b, qp, fd;
};

struct Local {
  const K1D* P;
  const Chan* c;
  const double *ht, *mt, *kt;
  Motion M;
  double dt, dx;

  __device__ double depth(int s) const {
    const double x = (s + 0.5) * dx;
    return P->ds[c->off + s] - body_shape(*c, x - M.X, 0.0).B;
  }
  // d_x, 4 + d_x^2 and phi (Eq. 5) at channel cell s (0 <= s < n)
  __device__ CellNH cell(int s) const {
    const int n = c->n;
    const int l = reflect(s - 1, n), r = reflect(s + 1, n);
    const double dl = depth(l), d0 = depth(s), dr = depth(r);
    const double D = (dr - dl) / (2.0 * dx);
    const double dxx = (dr - 2.0 * d0 + dl) / (dx * dx);
    const int64_t o = c->off;
    const double ex = ((ht[o + r] - dr) - (ht[o + l] - dl)) / (2.0 * dx);
    const double hs = ht[o + s];
    const double u = mt[o + s] / hs;
    const double x = (s + 0.5) * dx;
    const BedRate br = bed_rate(M, body_shape(*c, x - M.X, 0.0));
    CellNH q;
    q.D = D;
    q.al = 4.0 + D * D;
    q.phi = P->rho * hs / q.al * (P->g * D * ex - br.d_tt - 2.0 * u * br.d_xt - u * u * dxx);
    return q;
  }
  // face f between cells f-1 and f (0 <= f <= n), given phi of both sides
  __device__ FaceNH face(int f, double phil, double phir) const {
    const int n = c->n;
    const int l = reflect(f - 1, n), r = reflect(f, n);
    const int64_t o = c->off;
    const double hf = 0.5 * (ht[o + l] + ht[o + r]);
    const double Df = (depth(r) - depth(l)) / dx;
    const double hx = (ht[o + r] - ht[o + l]) / dx;
    const double ml = (l == f - 1 ? 1.0 : -1.0) * mt[o + l];
    const double mr = (r == f ? 1.0 : -1.0) * mt[o + r];
    const double af = 4.0 + Df * Df;
    const double s11 = (2.0 * hx - 3.0 * Df) / (2.0 * hf);
    FaceNH q;
    q.K = 4.0 * dt * hf / (P->rho * af);
    q.a = -1.0 / dx + 0.5 * s11;
    q.b = 1.0 / dx + 0.5 * s11;
    q.fd = dt / P->rho * (0.5 * (phil + phir)) * Df;
    q.qp = 0.5 * (ml + mr) + q.fd;
    return q;
  }
};
}  // namespace

__global__ void __launch_bounds__(256) k_assemble1d(K1D P, const double* __restrict__ ht,
                                                    const double* __restrict__ mt,
                                                    const double* __restrict__ kt,
                                                    const uint8_t* __restrict__ mask,
                                                    const double* t_in, const double* dt_in,
                                                    double* __restrict__ dg, double* __restrict__ up,
                                                    double* __restrict__ rh) {
  const int na = *P.n_act;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < na; k += gridDim.x * blockDim.x) {
    const int gi = P.act_cell[k], ci = P.act_chan[k];
    const Chan c = P.ch[ci];
    const int i = (int)(gi - c.off), n = c.n;
    Local L{&P, &c, ht, mt, kt, body_motion(c, t_in[ci] + dt_in[ci]), dt_in[ci], P.dx};
    const CellNH cm = L.cell(reflect(i - 1, n)), c0 = L.cell(i), cp = L.cell(reflect(i + 1, n));
    const FaceNH fl = L.face(i, cm.phi, c0.phi), fr = L.face(i + 1, c0.phi, cp.phi);
    const double hs = ht[gi];
    const double s22 = 3.0 * L.dt / (P.rho * hs);
    const double xx = (i + 0.5) * P.dx;
    const BedRate br = bed_rate(L.M, body_shape(c, xx - L.M.X, 0.0));
    const double f2 = -2.0 * br.d_t - 2.0 * kt[gi] / hs - c0.D * mt[gi] / (2.0 * hs) -
                      L.dt * c0.al * c0.phi / (2.0 * P.rho * hs);
    dg[k] = s22 + fl.K * fl.b * fl.b + fr.K * fr.a * fr.a;
    up[k] = (i + 1 < n && mask[gi + 1]) ? fr.K * fr.a * fr.b : 0.0;
    rh[k] = f2 + fl.b * fl.qp + fr.a * fr.qp;
  }
}

// projection on the packed rows: x = packed pressure
__global__ void __launch_bounds__(256) k_correct1d(K1D P, const double* __restrict__ ht,
                                                   const double* __restrict__ mt,
                                                   const double* __restrict__ kt,
                                                   const uint8_t* __restrict__ mask,
                                                   const double* t_in, const double* dt_in,
                                                   const double* __restrict__ x, double* hu,
                                                   double* hw, double* p) {
  const int na = *P.n_act;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < na; k += gridDim.x * blockDim.x) {
    const int gi = P.act_cell[k], ci = P.act_chan[k];
    const Chan c = P.ch[ci];
    const int i = (int)(gi - c.off), n = c.n;
    Local L{&P, &c, ht, mt, kt, body_motion(c, t_in[ci] + dt_in[ci]), dt_in[ci], P.dx};
    const CellNH cm = L.cell(reflect(i - 1, n)), c0 = L.cell(i), cp = L.cell(reflect(i + 1, n));
    const FaceNH fl = L.face(i, cm.phi, c0.phi), fr = L.face(i + 1, c0.phi, cp.phi);
    const double pc = x[k];
    const double pl = (i > 0 && mask[gi - 1]) ? x[k - 1] : 0.0;
    const double pr = (i + 1 < n && mask[gi + 1]) ? x[k + 1] : 0.0;
    const double dql = fl.fd - fl.K * (fl.a * pl + fl.b * pc);
    const double dqr = fr.fd - fr.K * (fr.a * pc + fr.b * pr);
    const double dm = 0.5 * (dql + dqr);
    const double Pb = 1.5 * pc - P.rho * c0.D * dm / (4.0 * L.dt) + c0.al * c0.phi / 4.0;
    hu[gi] = mt[gi] + dm;
    hw[gi] = kt[gi] + L.dt * Pb / P.rho;
    if (p) p[gi] = pc;
  }
}

// ---------------------------------------------------------------------------
// fused FP64 step
// ---------------------------------------------------------------------------
// One kernel per tile runs both Heun stages on an LDS window that extends the
// tile by e + 2 cells on each side (e = enlargement), so that the criterion,
// its enlargement and the elliptic coefficients of the tile's cells and faces
// all read Q~ from LDS; Q~ never goes to HBM.  The new state goes to a second
// buffer (the caller's arrays and the workspace alternate), because
// neighbouring tiles still read Q^n.
//
// The marked rows of a tile are consecutive rows of the packed system in cell
// order.  The tile eliminates its interior rows (pinned first and last row,
// parallel cyclic reduction for three right-hand sides), which leaves two
// rows per tile: the level-1 system, tridiagonal over all tiles of all
// channels.  Its solution gives every row as x = z + u x_first + v x_last.
// A tile with one marked row keeps it as the first row, or as the last row
// when it couples to the next tile.  Tiles without marked rows give identity
// rows.
namespace {
constexpr int EMAXF = 8;          // largest enlargement of the fused step
constexpr int HMAXF = EMAXF + 2;  // Q~ beyond the tile: criterion stencil + enlargement
constexpr int L1MAX = 1024;       // level-1 rows solved inside the projection kernel

// checks one cell of the final state and folds its wave speed into s
__device__ __forceinline__ void final_state(double g, double hh, double mm, double kk, double& s,
                                            int& flags) {
  if (!isfinite(hh) || !isfinite(mm) || !isfinite(kk)) {
    flags |= ST_NAN;
  } else if (!(hh > 0.0)) {
    flags |= ST_DRY;
  } else {
    s = fmax(s, fabs(mm * rcp64(hh)) + sqrt64(g * hh));
  }
}

// block max of s and OR of flags -> next step's speed buffer and status
template <int NT>
__device__ void flush_speed(const K1D& P, int chan, int par, double s, int flags) {
  __shared__ double red[NT / 64];
  __shared__ int fl;
  if (threadIdx.x == 0) fl = 0;
  s = wave_max(s);
  __syncthreads();
  if (flags) atomicOr(&fl, flags);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < NT / 64; w++) m = fmax(m, red[w]);
    atomicMax(&P.smax[speed_at((par ^ 1) * P.nch + chan, blockIdx.x & (P.nslot - 1), P.nslot)],
              pos_bits(m));
    if (fl) atomicOr(P.status, fl);
  }
}

// rank (in cell order) of the marked cells of a tile: thread t handles the
// tile cells k = 1 + t + NT q; rank[q] is valid where the cell is marked.
// Returns the number of marked cells.
template <int T, int NT, typename On>
__device__ int tile_ranks(On on_of, int (&rank)[T / NT], bool (&on)[T / NT]) {
  __shared__ int wcnt[NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int base = 0;
#pragma unroll
  for (int q = 0; q < T / NT; q++) {
    on[q] = on_of(1 + (int)threadIdx.x + NT * q);
    const unsigned long long bal = __ballot(on[q]);
    if (lane == 0) wcnt[wv] = __popcll(bal);
    __syncthreads();
    int wb = 0, tot = 0;
    for (int w = 0; w < NT / 64; w++) {
      if (w < wv) wb += wcnt[w];
      tot += wcnt[w];
    }
    rank[q] = base + wb + __popcll(bal & ((1ull << lane) - 1ull));
    base += tot;
    __syncthreads();
  }
  return base;
}

template <int T, int NT>
struct StepSmem {
  static constexpr int WMAX = T + 2 * (4 + HMAXF);  // predictor window
  static constexpr int RW = T > NT ? T : NT;        // rows of the in-LDS tile system
  // two buffers let each reduction level end with one barrier instead of two;
  // they fit beside the other members only for the 128-cell window (larger
  // windows would lose blocks per CU)
  static constexpr int NB = T <= 128 ? 2 : 1;
  // eta (then h~ after the predictor), hu, hw; depth at t^n and t^{n+1}
  double e[WMAX], m[WMAX], k[WMAX], d0[WMAX], d1[WMAX];
  union {
    struct {
      double Fh[WMAX], AL[WMAX], AR[WMAX], Fk[WMAX];  // face fluxes
    } f;  // a predictor stage
    struct {
      CellNH cq[T + 2];  // cells start-1 .. end
      FaceNH fq[T + 1];  // faces start .. end
    } q;
    struct {
      double a[RW], b[RW], c[RW], d[3][RW], r[RW];  // r = 1 / b
    } s[NB];  // tile system (the reduction alternates between NB buffers)
    struct {
      float a[RW], b[RW], c[RW], r[RW];  // FP32 tile system, r = 1 / b
      float d[2][3][RW];                 // right-hand sides, alternating by level
      double x[3][RW];                   // FP64 solution, by row
      double ends[8];                    // FP64 first and last rows before pinning
      double red[1][NT / 64];            // block maxima
      double red6[6][NT / 64];
    } g;  // FP32 reduction with FP64 refinement
  } u;
  uint8_t raw[T + 2 + 2 * EMAXF];
  uint8_t mk[T + 2];
  short cell_of[RW];  // tile system row -> tile cell
};

// face fluxes of one predictor stage on faces [f0, f1) of the window (face f
// between window cells f-1 and f) from the minmod slopes of eta, hu, hw and
// the depth in the two cells beside the face (each face takes them from the
// four cells f-2 .. f+1 itself: recomputing a slope per face is cheaper than
// a pass that stores them and the barrier after it); the
// momentum fluxes carry the centred bed source of the cell on each side,
// g h (d_x) / 2 with the reconstructed depth at this face, so that a cell's
// momentum update is the difference of two face values.  Dry faces touching
// channel cells of [lo_cell, hi_cell) raise the flag.
template <typename SM>
__device__ __forceinline__ void step_faces(SM& S, const double* d, double g, int f0, int f1,
                                           int lo_cell, int hi_cell, int base, int& flags) {
  for (int f = f0 + threadIdx.x; f < f1; f += blockDim.x) {
    const int l = f - 1, r = f;
    const double e0 = S.e[l - 1], e1 = S.e[l], e2 = S.e[r], e3 = S.e[r + 1];
    const double m0 = S.m[l - 1], m1 = S.m[l], m2 = S.m[r], m3 = S.m[r + 1];
    const double k0 = S.k[l - 1], k1 = S.k[l], k2 = S.k[r], k3 = S.k[r + 1];
    const double d0 = d[l - 1], d1 = d[l], d2 = d[r], d3 = d[r + 1];
    const double sdl = minmod(d1 - d0, d2 - d1), sdr = minmod(d2 - d1, d3 - d2);
    const Flux F = rusanov1d(g, e1 + 0.5 * minmod(e1 - e0, e2 - e1),
                             m1 + 0.5 * minmod(m1 - m0, m2 - m1),
                             k1 + 0.5 * minmod(k1 - k0, k2 - k1), d1 + 0.5 * sdl,
                             e2 - 0.5 * minmod(e2 - e1, e3 - e2),
                             m2 - 0.5 * minmod(m2 - m1, m3 - m2),
                             k2 - 0.5 * minmod(k2 - k1, k3 - k2), d2 - 0.5 * sdr);
    S.u.f.Fh[f] = F.Fh;
    S.u.f.AL[f] = F.FmL - 0.5 * g * F.hL * sdl;
    S.u.f.AR[f] = F.FmR + 0.5 * g * F.hR * sdr;
    S.u.f.Fk[f] = F.Fk;
    const int il = base + l, ir = base + r;
    const bool used = (il >= lo_cell && il < hi_cell) || (ir >= lo_cell && ir < hi_cell);
    if (F.dry && used) flags |= ST_DRY;
  }
}

template <typename SM>
__device__ __forceinline__ void step_cell(const SM& S, double idx, int e, double& Lh, double& Lm,
                                          double& Lk) {
  Lh = -(S.u.f.Fh[e + 1] - S.u.f.Fh[e]) * idx;
  Lm = -(S.u.f.AL[e + 1] - S.u.f.AR[e]) * idx;
  Lk = -(S.u.f.Fk[e + 1] - S.u.f.Fk[e]) * idx;
}

// Q~ and the depth at t^{n+1} of channel cells, read from the window
struct WinQ {
  const double *h, *m, *k, *d;  // window arrays
  int lo, n;
  double dx, idx, i2dx;  // dx, 1 / dx, 1 / (2 dx)
  __device__ double H(int i) const { return h[reflect(i, n) - lo]; }
  __device__ double D(int i) const { return d[reflect(i, n) - lo]; }
  // momentum of cell i, odd under the wall reflection
  __device__ double Mo(int i) const {
    const int s = reflect(i, n);
    return (s == i ? 1.0 : -1.0) * m[s - lo];
  }
  __device__ double K(int i) const { return k[reflect(i, n) - lo]; }
};

// criterion of Sec. 5.1 at channel cell i from the window
__device__ double indicator_win(const WinQ& Q, int i, int crit) {
  switch (crit) {
    case SWE_NH_CRIT_ETA_D: {
      const double d = Q.D(i);
      return fabs((Q.H(i) - d) / d);
    }
    case SWE_NH_CRIT_ETA_X:
      return fabs(((Q.H(i + 1) - Q.D(i + 1)) - (Q.H(i - 1) - Q.D(i - 1))) * Q.i2dx);
    case SWE_NH_CRIT_U:
      return fabs(Q.Mo(i) / Q.H(i));
    case SWE_NH_CRIT_U_X:
      return fabs((Q.Mo(i + 1) / Q.H(i + 1) - Q.Mo(i - 1) / Q.H(i - 1)) * Q.i2dx);
    case SWE_NH_CRIT_W:
      return fabs(Q.K(i) / Q.H(i));
    default:  // SWE_NH_CRIT_W_X
      return fabs((Q.K(i + 1) / Q.H(i + 1) - Q.K(i - 1) / Q.H(i - 1)) * Q.i2dx);
  }
}

// d_x, 4 + d_x^2 and phi (Eq. 5) at channel cell s from the window
__device__ CellNH cell_win(const WinQ& Q, const K1D& P, const Chan& c, const Motion& M, int s) {
  const double dl = Q.D(s - 1), d0 = Q.D(s), dr = Q.D(s + 1);
  const double D = (dr - dl) * Q.i2dx;
  const double dxx = (dr - 2.0 * d0 + dl) * (Q.idx * Q.idx);
  const double ex = ((Q.H(s + 1) - dr) - (Q.H(s - 1) - dl)) * Q.i2dx;
  const double hs = Q.H(s);
  const double u = Q.Mo(s) * rcp64(hs);
  const BedRate br = bed_rate(M, body_shape(c, (s + 0.5) * Q.dx - M.X, 0.0));
  CellNH q;
  q.D = D;
  q.al = 4.0 + D * D;
  q.phi = P.rho * hs * rcp64(q.al) * (P.g * D * ex - br.d_tt - 2.0 * u * br.d_xt - u * u * dxx);
  return q;
}

// face f between cells f-1 and f (0 <= f <= n) from the window
__device__ FaceNH face_win(const WinQ& Q, const K1D& P, double dt, int f, double phil,
                           double phir) {
  const double hl = Q.H(f - 1), hr = Q.H(f);
  const double hf = 0.5 * (hl + hr);
  const double Df = (Q.D(f) - Q.D(f - 1)) * Q.idx;
  const double hx = (hr - hl) * Q.idx;
  const double af = 4.0 + Df * Df;
  const double rhf = rcp64(hf);
  const double s11 = (hx - 1.5 * Df) * rhf;
  FaceNH q;
  q.K = 4.0 * dt * hf * rcp64(P.rho * af);
  q.a = -Q.idx + 0.5 * s11;
  q.b = Q.idx + 0.5 * s11;
  q.fd = dt / P.rho * (0.5 * (phil + phir)) * Df;
  q.qp = 0.5 * (Q.Mo(f - 1) + Q.Mo(f)) + q.fd;
  return q;
}

// parallel cyclic reduction of the first m rows of the tile system (rows
// m..RW are identity), three right-hand sides, starting in buffer 0; returns
// the buffer that holds the result
template <int T, int NT>
__device__ int pcr_tile(StepSmem<T, NT>& S, int m) {
  constexpr int RW = StepSmem<T, NT>::RW, RPT = RW / NT, NB = StepSmem<T, NT>::NB;
  int cur = 0;
  for (int s = 1; s < m; s <<= 1) {
    const auto& Y = S.u.s[cur];
    double na[RPT], nb[RPT], nc[RPT], nd[RPT][3];
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      const int i = RPT * threadIdx.x + j;
      const int im = i - s, ip = i + s;
      double bi = Y.b[i], ai = 0.0, ci = 0.0;
      double di[3] = {Y.d[0][i], Y.d[1][i], Y.d[2][i]};
      if (im >= 0) {
        const double k1 = Y.a[i] * Y.r[im];
        ai = -Y.a[im] * k1;
        bi -= Y.c[im] * k1;
#pragma unroll
        for (int r = 0; r < 3; r++) di[r] -= Y.d[r][im] * k1;
      }
      if (ip < RW) {
        const double k2 = Y.c[i] * Y.r[ip];
        ci = -Y.c[ip] * k2;
        bi -= Y.a[ip] * k2;
#pragma unroll
        for (int r = 0; r < 3; r++) di[r] -= Y.d[r][ip] * k2;
      }
      na[j] = ai;
      nb[j] = bi;
      nc[j] = ci;
#pragma unroll
      for (int r = 0; r < 3; r++) nd[j][r] = di[r];
    }
    // one buffer: everyone has read before anyone writes; two: the level
    // writes the other buffer, whose last readers finished a barrier ago
    if (NB == 1) __syncthreads();
    const int nxt = (NB == 2) ? cur ^ 1 : cur;
    auto& Z = S.u.s[nxt];
#pragma unroll
    for (int j = 0; j < RPT; j++) {
      const int i = RPT * threadIdx.x + j;
      Z.a[i] = na[j];
      Z.b[i] = nb[j];
      Z.c[i] = nc[j];
      Z.r[i] = rcp64(nb[j]);
#pragma unroll
      for (int r = 0; r < 3; r++) Z.d[r][i] = nd[j][r];
    }
    __syncthreads();
    cur = nxt;
  }
  return cur;
}
// ---- FP32 tile reduction with FP64 refinement ----
// The pinned tile system M X = D (three right-hand sides: the tile's rows and
// unit vectors at its first and last row) is reduced in FP32 by the parallel
// cyclic reduction of pcr_tile, which keeps each level's two elimination
// factors of every row in registers, so that a later right-hand side needs
// only two products per level and column.  Classical iterative refinement
// follows: R = D - M X from the FP64 rows, E = M^-1 R with the FP32 factors,
// X += E in FP64, until the normwise backward error of every column,
// max_j |R_j| / max_j (|M| |X| + |D|)_j over the unpinned rows (the pinned
// rows' residuals are zero), is at most tol (the measure of
// Rigal and Gaches 1967; a backward-stable solve reaches the unit roundoff,
// whatever the condition number).  The tile's own column is refined scaled
// by the power of two that brings its largest right-hand side to [1, 2)
// (exact, and undone at the end), and every residual goes to FP32 scaled the
// same way: far from the slide the right-hand sides can lie below FP32's
// range, and even in FP64's subnormal range, where no residual could be
// computed to a relative accuracy.  In the reduction thread t
// owns rows RPT t .. RPT t + RPT - 1; in the residual, the rows of its marked
// cells (rank[q]).  On return u.g.x holds the FP64 basis columns z, u, v by
// row and u.g.ends the FP64 first row (b, c, d) and last row (a, b, c, d)
// before pinning; returns the sweeps taken, or -1 - sweeps when tol was not
// reached in max_sweeps.
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

template <int RW>
constexpr int levels_of() {
  int l = 0;
  while ((1 << l) < RW) l++;
  return l;
}

// exponent e with 2^e <= v < 2^(e+1) (0 for v == 0)
__device__ __forceinline__ int exp2_of(double v) { return v > 0.0 ? ilogb(v) : 0; }

// block maxima of the thread's values v[0..N) (all threads get them; one barrier)
template <int NT, int N>
__device__ __forceinline__ void block_max(double (&v)[N], double (*red)[NT / 64]) {
#pragma unroll
  for (int k = 0; k < N; k++) v[k] = wave_max(v[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < N; k++) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; k++) {
    v[k] = red[k][0];
#pragma unroll
    for (int w = 1; w < NT / 64; w++) v[k] = fmax(v[k], red[k][w]);
  }
}

template <int T, int NT>
__device__ int refine_tile32(StepSmem<T, NT>& S, int m, const double (&ra)[T / NT],
                             const double (&rb)[T / NT], const double (&rc)[T / NT],
                             const double (&rd)[T / NT], const int (&rank)[T / NT],
                             const bool (&on)[T / NT], double tol, int max_sweeps,
                             double& berr_out) {
  constexpr int RW = StepSmem<T, NT>::RW, RPT = RW / NT, LV = levels_of<RW>(), QN = T / NT;
  auto& G = S.u.g;
  // identity rows, and the largest right-hand side of the tile's own rows
  double dmax[1] = {0.0};
#pragma unroll
  for (int q = 0; q < QN; q++)
    if (on[q] && rank[q] != 0 && rank[q] != m - 1) dmax[0] = fmax(dmax[0], fabs(rd[q]));
  for (int j = threadIdx.x; j < RW; j += NT) {
    G.a[j] = 0.0f;
    G.b[j] = 1.0f;
    G.c[j] = 0.0f;
    G.r[j] = 1.0f;
    G.d[0][0][j] = 0.0f;
    G.d[0][1][j] = j == 0 ? 1.0f : 0.0f;
    G.d[0][2][j] = j == m - 1 ? 1.0f : 0.0f;
  }
  block_max<NT, 1>(dmax, G.red);  // its barrier also orders the identity rows
  const int e0 = exp2_of(dmax[0]);
#pragma unroll
  for (int q = 0; q < QN; q++) {
    if (!on[q]) continue;
    const int j = rank[q];
    if (j == 0) {
      G.ends[0] = rb[q];
      G.ends[1] = rc[q];
      G.ends[2] = rd[q];
    } else if (j == m - 1) {
      G.ends[3] = ra[q];
      G.ends[4] = rb[q];
      G.ends[5] = rc[q];
      G.ends[6] = rd[q];
    } else {
      const float bj = (float)rb[q];
      G.a[j] = (float)ra[q];
      G.b[j] = bj;
      G.c[j] = (float)rc[q];
      G.r[j] = rcp32(bj);
      G.d[0][0][j] = (float)ldexp(rd[q], -e0);  // exact while the scaled value is normal
    }
  }
  __syncthreads();
  // FP32 reduction of the matrix and the three columns, factors kept
  float k1[RPT][LV], k2[RPT][LV];
  int cur = 0;
#pragma unroll
  for (int lv = 0; lv < LV; lv++) {
    const int s = 1 << lv;
#pragma unroll
    for (int jj = 0; jj < RPT; jj++) k1[jj][lv] = k2[jj][lv] = 0.0f;
    if (s >= m) continue;  // m is the same for the whole block
    float na[RPT], nb[RPT], nc[RPT], nd[RPT][3];
#pragma unroll
    for (int jj = 0; jj < RPT; jj++) {
      const int i = RPT * threadIdx.x + jj, im = i - s, ip = i + s;
      float bi = G.b[i], ai = 0.0f, ci = 0.0f;
      float di[3] = {G.d[cur][0][i], G.d[cur][1][i], G.d[cur][2][i]};
      if (im >= 0) {
        const float f = G.a[i] * G.r[im];
        k1[jj][lv] = f;
        ai = -G.a[im] * f;
        bi -= G.c[im] * f;
#pragma unroll
        for (int r = 0; r < 3; r++) di[r] -= G.d[cur][r][im] * f;
      }
      if (ip < RW) {
        const float f = G.c[i] * G.r[ip];
        k2[jj][lv] = f;
        ci = -G.c[ip] * f;
        bi -= G.a[ip] * f;
#pragma unroll
        for (int r = 0; r < 3; r++) di[r] -= G.d[cur][r][ip] * f;
      }
      na[jj] = ai;
      nb[jj] = bi;
      nc[jj] = ci;
#pragma unroll
      for (int r = 0; r < 3; r++) nd[jj][r] = di[r];
    }
    __syncthreads();  // the matrix is reduced in place: all reads before any write
#pragma unroll
    for (int jj = 0; jj < RPT; jj++) {
      const int i = RPT * threadIdx.x + jj;
      G.a[i] = na[jj];
      G.b[i] = nb[jj];
      G.c[i] = nc[jj];
      G.r[i] = rcp32(nb[jj]);
#pragma unroll
      for (int r = 0; r < 3; r++) G.d[cur ^ 1][r][i] = nd[jj][r];
    }
    __syncthreads();
    cur ^= 1;
  }
  float rbf[RPT];
  double X[RPT][3];
#pragma unroll
  for (int jj = 0; jj < RPT; jj++) {
    const int i = RPT * threadIdx.x + jj;
    rbf[jj] = G.r[i];
#pragma unroll
    for (int r = 0; r < 3; r++) X[jj][r] = (double)(G.d[cur][r][i] * rbf[jj]);  // column 0 scaled
  }
  int sweeps = 0;
  double berr = 0.0;
  for (;;) {
#pragma unroll
    for (int jj = 0; jj < RPT; jj++)
#pragma unroll
      for (int r = 0; r < 3; r++) G.x[r][RPT * threadIdx.x + jj] = X[jj][r];
    __syncthreads();
    // FP64 residual of the thread's marked rows (per column the largest |R_j|
    // and (|M| |X| + |D|)_j), computed again after the reduction, when it
    // goes to FP32 scaled, rather than kept in registers across it
    auto resid = [&](int q, int r, double& den) {
      const int j = rank[q];
      const double dj = j == 0 ? (r == 1 ? 1.0 : 0.0)
                               : j == m - 1 ? (r == 2 ? 1.0 : 0.0)
                                            : (r == 0 ? ldexp(rd[q], -e0) : 0.0);
      if (j == 0 || j == m - 1) {
        den = 0.0;  // the pinned rows' scale is arbitrary (and their residual zero)
        return dj - G.x[r][j];
      }
      const double t0 = ra[q] * G.x[r][j - 1], t1 = rb[q] * G.x[r][j], t2 = rc[q] * G.x[r][j + 1];
      den = fabs(t0) + fabs(t1) + fabs(t2) + fabs(dj);
      return dj - t0 - t1 - t2;
    };
    double mx[6];
#pragma unroll
    for (int k = 0; k < 6; k++) mx[k] = 0.0;
#pragma unroll
    for (int q = 0; q < QN; q++) {
      if (!on[q]) continue;
#pragma unroll
      for (int r = 0; r < 3; r++) {
        double den;
        const double rv = resid(q, r, den);
        mx[r] = fmax(mx[r], fabs(rv));
        mx[3 + r] = fmax(mx[3 + r], den);
      }
    }
    block_max<NT, 6>(mx, G.red6);
    berr = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++)
      if (mx[r] > 0.0) berr = fmax(berr, mx[r] / mx[3 + r]);
    if (berr <= tol || sweeps >= max_sweeps) break;
    // the residuals, scaled per column, as FP32 right-hand sides
    int er[3];
#pragma unroll
    for (int r = 0; r < 3; r++) er[r] = exp2_of(mx[r]);
#pragma unroll
    for (int q = 0; q < QN; q++) {
      if (!on[q]) continue;
#pragma unroll
      for (int r = 0; r < 3; r++) {
        double den;
        G.d[cur][r][rank[q]] = (float)ldexp(resid(q, r, den), -er[r]);
      }
    }
    __syncthreads();
    // E = M^-1 R with the kept factors (the pinned rows' residuals are zero)
#pragma unroll
    for (int lv = 0; lv < LV; lv++) {
      const int s = 1 << lv;
      if (s >= m) continue;
      float nd[RPT][3];
#pragma unroll
      for (int jj = 0; jj < RPT; jj++) {
        const int i = RPT * threadIdx.x + jj, im = i - s, ip = i + s;
#pragma unroll
        for (int r = 0; r < 3; r++) {
          float v = G.d[cur][r][i];
          if (im >= 0) v -= G.d[cur][r][im] * k1[jj][lv];
          if (ip < RW) v -= G.d[cur][r][ip] * k2[jj][lv];
          nd[jj][r] = v;
        }
      }
#pragma unroll
      for (int jj = 0; jj < RPT; jj++)
#pragma unroll
        for (int r = 0; r < 3; r++) G.d[cur ^ 1][r][RPT * threadIdx.x + jj] = nd[jj][r];
      __syncthreads();
      cur ^= 1;
    }
#pragma unroll
    for (int jj = 0; jj < RPT; jj++)
#pragma unroll
      for (int r = 0; r < 3; r++)
        X[jj][r] += ldexp((double)(G.d[cur][r][RPT * threadIdx.x + jj] * rbf[jj]), er[r]);
    sweeps++;
  }
  // the tile's own column back to its scale (the caller reads u.g.x after a
  // barrier of its own)
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < RPT; jj++) G.x[0][RPT * threadIdx.x + jj] = ldexp(X[jj][0], e0);
  __syncthreads();
  berr_out = berr;
  return berr <= tol ? sweeps : -1 - sweeps;
}

// Tridiagonal solve of n <= 64 rows held one per lane of the calling
// wavefront (a: sub-, b: main, c: super-diagonal, d: right-hand side; lanes
// at or beyond n hold identity rows): parallel cyclic reduction with
// cross-lane shuffles, no block barrier.  Returns x of the lane's row.
__device__ __forceinline__ double wave_pcr(double a, double b, double c, double d, int n) {
  const int lane = threadIdx.x & 63;
  for (int s = 1; s < n; s <<= 1) {
    const double am = __shfl_up(a, s), bm = __shfl_up(b, s), cm = __shfl_up(c, s),
                 dm = __shfl_up(d, s);
    const double ap = __shfl_down(a, s), bp = __shfl_down(b, s), cp = __shfl_down(c, s),
                 dp = __shfl_down(d, s);
    double na = 0.0, nb = b, nc = 0.0, nd = d;
    if (lane >= s) {
      const double k1 = a * rcp64(bm);
      na = -am * k1;
      nb -= cm * k1;
      nd -= dm * k1;
    }
    if (lane + s < 64) {
      const double k2 = c * rcp64(bp);
      nc = -cp * k2;
      nb -= ap * k2;
      nd -= dp * k2;
    }
    a = na;
    b = nb;
    c = nc;
    d = nd;
  }
  return d * rcp64(b);
}

// polls the 6 level-1 row values of tile t (12 words) in one loop, so their
// loads overlap; false when the wait timed out or the step aborted
__device__ bool poll_rows6(const unsigned long long* rw, int t, unsigned tag, double (&v)[6],
                           int* status) {
  unsigned need = 0x3fu;
  const unsigned long long t0 = wall_clock64();
  unsigned polls = 0;
  for (;;) {
#pragma unroll
    for (int k = 0; k < 6; k++)
      if ((need & (1u << k)) && try_tagged(rw + ((size_t)t * 6 + k) * 2, tag, v[k]))
        need &= ~(1u << k);
    if (!need) return true;
    if ((++polls & 255u) == 0u) {
      if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_ABORT)
        return false;
      if (wall_clock64() - t0 > POLL_TICKS) {
        atomicOr(status, ST_ABORT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// One-kernel step, level-1 part.  Every tile publishes its marked count (and,
// when marked, its F and L rows: dg, up, rh) as tagged words.  Block 0 and
// every marked block then poll all counts and list the marked tiles in tile
// order (onepass_counts).  Up to 64 marked tiles, each marked block solves
// the level-1 system itself (onepass_solve_local: the rows coupled like the
// packed system, F-L within a tile and L to the next tile's F when the two
// tiles are neighbours; two rows per lane of one wavefront, one
// cyclic-reduction level, then wave_pcr), which saves a round of
// publishing; beyond, block 0 runs a Thomas sweep and publishes the solution
// (onepass_solve_publish).  Once block 0 has every count, every block has
// read the speed buffer of the step: block 0 clears it and records the tag.

constexpr int ONEPASS_NI = ONEPASS_TILES / 64;  // count words per lane of wavefront 0

// loads of the count words, issued early (wavefront 0, lane l: tiles l + 64 i)
// and checked only in onepass_counts: the round trip overlaps the caller's
// own work in between
__device__ __forceinline__ void onepass_prefetch(const K1D& P,
                                                 unsigned long long (&pre)[ONEPASS_NI]) {
#pragma unroll
  for (int i = 0; i < ONEPASS_NI; i++) {
    const int t = (int)threadIdx.x + 64 * i;
    pre[i] = (threadIdx.x < 64 && t < P.ntiles) ? load_word(P.tw + t) : 0ull;
  }
}

// the marked tiles in tile order -> tl (LDS); returns their number, or -1
// when a poll timed out or the step aborted (all threads of the block call;
// pre: the words of onepass_prefetch, or 0 to poll them all)
__device__ int onepass_counts(const K1D& P, unsigned tag, int* tl,
                              const unsigned long long (&pre)[ONEPASS_NI]) {
  __shared__ int s_nm;
  const unsigned long long* cw = P.tw;
  __syncthreads();  // the block's own tile data in LDS is consumed
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    // all the lane's counts (tiles lane + 64 i): those already in the
    // prefetched words, the rest polled in one loop
    constexpr int NI = ONEPASS_NI;
    unsigned cnt[NI];
    unsigned need = 0;
#pragma unroll
    for (int i = 0; i < NI; i++) {
      cnt[i] = (unsigned)pre[i];
      if (lane + 64 * i < P.ntiles && (unsigned)(pre[i] >> 32) != tag) need |= 1u << i;
    }
    bool ok = true;
    const unsigned long long c0 = wall_clock64();
    unsigned polls = 0;
    while (need) {
#pragma unroll
      for (int i = 0; i < NI; i++)
        if ((need & (1u << i)) && try_tagged(cw + lane + 64 * i, tag, cnt[i])) need &= ~(1u << i);
      if (!need) break;
      if ((++polls & 255u) == 0u) {
        if ((__hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_ABORT) ||
            wall_clock64() - c0 > POLL_TICKS) {
          atomicOr(P.status, ST_ABORT);
          ok = false;
          break;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
    int base = 0;
#pragma unroll
    for (int i = 0; i < NI; i++) {
      const int t = lane + 64 * i;
      const bool mt = t < P.ntiles && cnt[i] > 0;
      const unsigned long long bal = __ballot(mt);
      if (mt) tl[base + __popcll(bal & ((1ull << lane) - 1ull))] = t;
      base += __popcll(bal);
    }
    const unsigned long long bad = __ballot(!ok);
    if (lane == 0) s_nm = bad ? -1 : base;
  }
  __syncthreads();
  return s_nm;
}

// nm <= 64 marked tiles: the level-1 system solved by wavefront 0 of the
// calling block; xv = x of this tile's F and L rows, of the previous tile's L
// row (when nb_l) and of the next tile's F row (when nb_r).  False when a
// poll failed.  All threads of the block call.
__device__ bool onepass_solve_local(const K1D& P, unsigned tag, const int* tl, int nm, bool nb_l,
                                    bool nb_r, double* xv) {
  __shared__ int s_ok;
  const unsigned long long* rw = P.tw + P.ntiles;
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // F: dg, up, rh; L: dg, up, rh
    bool ok = true;
    const int t = l < nm ? tl[l] : -2;
    if (l < nm) ok = poll_rows6(rw, t, tag, v, P.status);
    const double upLprev = __shfl_up(v[4], 1);
    double a0 = 0.0, b0 = 1.0, c0 = 0.0, d0 = 0.0, a1 = 0.0, b1 = 1.0, c1 = 0.0, d1 = 0.0;
    if (l < nm) {
      a0 = (l > 0 && tl[l - 1] == t - 1) ? upLprev : 0.0;
      b0 = v[0];
      c0 = v[1];
      d0 = v[2];
      a1 = v[1];
      b1 = v[3];
      c1 = (l + 1 < nm && tl[l + 1] == t + 1) ? v[4] : 0.0;
      d1 = v[5];
    }
    // rows 2l (F) and 2l + 1 (L): the odd rows eliminated from the even ones
    const double am = __shfl_up(a1, 1), bm = __shfl_up(b1, 1), cm = __shfl_up(c1, 1),
                 dm = __shfl_up(d1, 1);  // row 2l - 1
    double na = 0.0, nb = b0, nd = d0;
    if (l > 0) {
      const double k1 = a0 * rcp64(bm);
      na = -am * k1;
      nb -= cm * k1;
      nd -= dm * k1;
    }
    const double r1 = rcp64(b1), k2 = c0 * r1;
    const double nc = -c1 * k2;
    nb -= a1 * k2;
    nd -= d1 * k2;
    const double xe = wave_pcr(na, nb, nc, nd, nm);
    const double xn = __shfl_down(xe, 1);  // x of row 2l + 2
    const double xo = (d1 - a1 * xe - (l < 63 ? c1 * xn : 0.0)) * r1;
    // this tile's compact position r: its neighbours, when marked, are r -+ 1
    const unsigned long long me = __ballot(l < nm && t == (int)blockIdx.x);
    const int r = me ? __ffsll((long long)me) - 1 : 0;
    const double xF = __shfl(xe, r), xL = __shfl(xo, r);
    const double xP = __shfl(xo, r > 0 ? r - 1 : 0), xN = __shfl(xe, r + 1 < 64 ? r + 1 : r);
    const unsigned long long bad = __ballot(!ok);
    if (l == 0) {
      xv[0] = xF;
      xv[1] = xL;
      xv[2] = nb_l ? xP : 0.0;
      xv[3] = nb_r ? xN : 0.0;
      s_ok = bad ? 0 : 1;
    }
  }
  __syncthreads();
  return s_ok != 0;
}

// nm > 64 marked tiles: block 0 solves by a Thomas sweep (one thread) over
// rows staged in LDS (st: 64 tiles x 6 values), recurrences in P.l1s, and
// publishes x per marked tile (F, L) as tagged words.  All threads of block 0
// call; false when a poll failed.
__device__ bool onepass_solve_publish(const K1D& P, unsigned tag, const int* tl, int nm,
                                      double (*st)[6]) {
  __shared__ int s_ok;
  const unsigned long long* rw = P.tw + P.ntiles;
  unsigned long long* xw = P.tw + 13 * (size_t)P.ntiles;
  double* cps = P.l1s;
  double* dps = P.l1s + 2 * (size_t)P.ntiles;
  double cp = 0.0, dp = 0.0, upLprev = 0.0;
  int tprev = -2;
  if (threadIdx.x == 0) s_ok = 1;
  for (int r0 = 0; r0 < nm; r0 += 64) {
    __syncthreads();
    if (threadIdx.x < 64) {
      const int r = r0 + threadIdx.x;
      bool ok = true;
      if (r < nm) {
        double v[6];
        ok = poll_rows6(rw, tl[r], tag, v, P.status);
#pragma unroll
        for (int k = 0; k < 6; k++) st[threadIdx.x][k] = v[k];
      }
      const unsigned long long bad = __ballot(!ok);
      if (threadIdx.x == 0 && bad) s_ok = 0;
    }
    __syncthreads();
    if (!s_ok) return false;
    if (threadIdx.x == 0) {
      const int r1 = min(nm, r0 + 64);
      for (int r = r0; r < r1; r++) {
        const int t = tl[r];
        const double* v = st[r - r0];
        // row F of tile t
        double a = tprev == t - 1 ? upLprev : 0.0;
        double rd = rcp64(v[0] - a * cp);
        cp = v[1] * rd;
        dp = (v[2] - a * dp) * rd;
        cps[2 * r] = cp;
        dps[2 * r] = dp;
        // row L
        a = v[1];
        rd = rcp64(v[3] - a * cp);
        const double c = (r + 1 < nm && tl[r + 1] == t + 1) ? v[4] : 0.0;
        cp = c * rd;
        dp = (v[5] - a * dp) * rd;
        cps[2 * r + 1] = cp;
        dps[2 * r + 1] = dp;
        tprev = t;
        upLprev = v[4];
      }
    }
  }
  if (threadIdx.x == 0) {
    double x = 0.0;
    for (int j = 2 * nm - 1; j >= 0; j--) {
      x = dps[j] - cps[j] * x;
      put_tagged(xw + (size_t)tl[j >> 1] * 4 + 2 * (j & 1), x, tag);
    }
  }
  __syncthreads();
  return true;
}

// block 0, once it has every count: every block has read the speed buffer
// `par`, which is cleared for the step after next, and the tag is recorded
__device__ void onepass_block0(const K1D& P, int par, unsigned tag) {
  if (!P.keep_speed)
    for (int i = threadIdx.x; i < P.nch * P.nslot; i += blockDim.x)
      P.smax[((size_t)par * P.nch * P.nslot + i) * SPEED_PAD] = 0ull;
  if (threadIdx.x == 0) *P.tag1 = tag;
}

}  // namespace

// Whole step of a tile up to the level-1 rows: dt from the speed of Q^n, both
// Heun stages (Eqs. 8-9), criterion and enlargement (Secs. 5.1-5.2), the new
// state's defaults (h = h~, hu = hu~, hw = hw~, p = 0 off the marked area),
// the speed of the unmarked cells' new state, assembly of the marked rows
// (Eqs. 10-17) and their reduction to the two level-1 rows.  ONE: the
// one-kernel step, which goes on to the level-1 solve and the
// projection of the marked cells (Eqs. 10-11), as the projection kernel does.
template <int T, int NT, bool ONE, bool F32R>
__global__ void __launch_bounds__(NT, 5) k_step1d(K1D P, const double* __restrict__ h,
                                               const double* __restrict__ hu,
                                               const double* __restrict__ hw,
                                               double* __restrict__ hn, double* __restrict__ hun,
                                               double* __restrict__ hwn, uint8_t* __restrict__ mask,
                                               double* __restrict__ p, int par) {
  static_assert(NT >= 128, "the step kernel needs two wavefronts for its time step and motions");
  using SM = StepSmem<T, NT>;
  constexpr int WMAX = SM::WMAX, RW = SM::RW;
  constexpr int Q = (WMAX - 4 + NT - 1) / NT;  // window cells per thread
  __shared__ SM S;
  __shared__ int sflags;
  const int4 tl = P.tiles[blockIdx.x];
  const Chan c = P.ch[tl.x];  // body parameters, needed after the first loads
  const int n = tl.w, start = tl.y, end = min(start + P.tile, n), len = end - start;
  const int64_t off = tl.z;
  const int step = P.step[par];
  const double t0 = P.t[par * P.nch + tl.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.step[par ^ 1] = step + 1;
    P.n_acc[par ^ 1] = 0;  // counts the next step
    if constexpr (F32R) {
      P.sweeps[par ^ 1] = 0;
      P.berr[par ^ 1] = 0ull;
    }
  }
  const int ee = P.enlarge, HL = 6 + ee, W = P.tile + 2 * HL;
  const int lo = start - HL;  // window cell w <-> channel cell lo + w
  const double idx = 1.0 / P.dx;
  if (threadIdx.x == 0) sflags = 0;
  int flags = 0;

  // ---- predictor ----
  // Q^n and d_s of the window into registers; meanwhile the body's motion at
  // t^n and t^{n+1}, one wavefront each (the same for every cell of the tile)
  constexpr int QL = (SM::WMAX + NT - 1) / NT;
  double vh[QL], vm[QL], vk[QL], vd[QL];
#pragma unroll
  for (int q = 0; q < QL; q++) {
    const int w = threadIdx.x + NT * q;
    if (w >= W) continue;
    const int i = lo + w;
    const int s = reflect(max(-n, min(i, 2 * n - 1)), n);
    const int64_t gi = off + s;
    vh[q] = h[gi];
    vm[q] = (s == i ? 1.0 : -1.0) * hu[gi];
    vk[q] = hw[gi];
    vd[q] = P.ds[gi];
  }
  Motion M0, M1;
  double dt;
  if constexpr (ONE) {
    block_step_motions(P, par, tl.x, c, t0, dt, M0, M1);
    if (start == 0 && threadIdx.x == 0) {  // the channel's first tile
      P.dt[tl.x] = dt;
      P.t[(par ^ 1) * P.nch + tl.x] = t0 + dt;  // the next step's start time
    }
  } else {  // from the channel's step table
    const double* ct = P.ctab + (size_t)tl.x * CTAB_N;
    dt = ct[CT_DT];
    M0 = Motion{ct[CT_X0], ct[CT_V0], ct[CT_A0]};
    M1 = Motion{ct[CT_X1], ct[CT_V1], ct[CT_A1]};
  }
  const double t1 = t0 + dt;
#pragma unroll
  for (int q = 0; q < QL; q++) {
    const int w = threadIdx.x + NT * q;
    if (w >= W) continue;
    const int s = reflect(max(-n, min(lo + w, 2 * n - 1)), n);
    const double x = (s + 0.5) * P.dx;
    const double dA = vd[q] - body_shape(c, x - M0.X, 0.0).B;
    S.e[w] = vh[q] - dA;
    S.m[w] = vm[q];
    S.k[w] = vk[q];
    S.d0[w] = dA;
    S.d1[w] = vd[q] - body_shape(c, x - M1.X, 0.0).B;
  }
  __syncthreads();
  double Qn[Q][3], L1[Q][3];
  step_faces(S, S.d0, P.g, 2, W - 1, max(0, start - 2), min(n, start + P.tile + 2), lo, flags);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const int e = 2 + threadIdx.x + NT * q;
    Qn[q][0] = Qn[q][1] = Qn[q][2] = 0.0;
    L1[q][0] = L1[q][1] = L1[q][2] = 0.0;
    if (e < W - 2) {
      step_cell(S, idx, e, L1[q][0], L1[q][1], L1[q][2]);
      Qn[q][0] = S.e[e] + S.d0[e];
      Qn[q][1] = S.m[e];
      Qn[q][2] = S.k[e];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; q++) {  // Q* on the channel cells
    const int e = 2 + threadIdx.x + NT * q;
    const int i = lo + e;
    if (e < W - 2 && i >= 0 && i < n) {
      S.e[e] = Qn[q][0] + dt * L1[q][0] - S.d1[e];
      S.m[e] = Qn[q][1] + dt * L1[q][1];
      S.k[e] = Qn[q][2] + dt * L1[q][2];
    }
  }
  __syncthreads();
  for (int w = threadIdx.x; w < W; w += NT) {  // ghosts of Q*: reflections
    const int i = lo + w;
    if (i >= 0 && i < n) continue;
    const int es = reflect(max(-n, min(i, 2 * n - 1)), n) - lo;
    double ev = 0.0, mv = 0.0, kv = 0.0;
    if (es >= 2 && es < W - 2) {
      ev = S.e[es];
      mv = -S.m[es];
      kv = S.k[es];
    }
    S.e[w] = ev;
    S.m[w] = mv;
    S.k[w] = kv;
  }
  __syncthreads();
  // stage 2 on window cells [4, W - 4): the tile and e + 2 cells beyond
  step_faces(S, S.d1, P.g, 4, W - 3, start, end, lo, flags);
  __syncthreads();
  double Qt[Q][3];
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const int e = 2 + threadIdx.x + NT * q;
    Qt[q][0] = Qt[q][1] = Qt[q][2] = 0.0;
    if (e < 4 || e >= W - 4) continue;
    double a, b, k2;
    step_cell(S, idx, e, a, b, k2);
    Qt[q][0] = Qn[q][0] + 0.5 * dt * (L1[q][0] + a);
    Qt[q][1] = Qn[q][1] + 0.5 * dt * (L1[q][1] + b);
    Qt[q][2] = Qn[q][2] + 0.5 * dt * (L1[q][2] + k2);
  }
  if (flags) atomicOr(&sflags, flags);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; q++) {  // the window now holds h~, hu~, hw~
    const int e = 2 + threadIdx.x + NT * q;
    if (e < 4 || e >= W - 4) continue;
    S.e[e] = Qt[q][0];
    S.m[e] = Qt[q][1];
    S.k[e] = Qt[q][2];
  }
  if (threadIdx.x == 0 && sflags) atomicOr(P.status, sflags);
  __syncthreads();

  // ---- criterion, enlargement ----
  const WinQ QW{S.e, S.m, S.k, S.d1, lo, n, P.dx, idx, 0.5 * idx};
  int mode;
  {
    const bool wcrit = (P.crit == SWE_NH_CRIT_W || P.crit == SWE_NH_CRIT_W_X);
    if (P.crit == SWE_NH_CRIT_GLOBAL || (wcrit && P.first_global && step == 0))
      mode = 1;
    else if (P.crit == SWE_NH_CRIT_NONE)
      mode = 2;
    else
      mode = 0;
  }
  if (mode == 0) {
    for (int w = threadIdx.x; w < len + 2 + 2 * ee; w += NT) {
      const int i = start - 1 - ee + w;
      uint8_t r = 0;
      if (i >= 0 && i < n) r = indicator_win(QW, i, P.crit) > P.k_nh;
      S.raw[w] = r;
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < len + 2; k += NT) {
    const int i = start - 1 + k;
    uint8_t v = 0;
    if (i >= 0 && i < n) {
      if (mode == 1) {
        v = 1;
      } else if (mode == 0) {
        for (int j = 0; j <= 2 * ee; j++) v |= S.raw[k + j];
      }
    }
    S.mk[k] = v;
  }
  __syncthreads();
  // ---- new state defaults, speed where no projection follows ----
  double smax = 0.0;
  int fl2 = 0;
#pragma unroll
  for (int q = 0; q < T / NT; q++) {
    const int k = 1 + threadIdx.x + NT * q;
    if (k > len) continue;
    const int i = start + k - 1, w = i - lo;
    const int64_t gi = off + i;
    const bool on = S.mk[k] != 0;
    const double hh = S.e[w], mm = S.m[w], kk = S.k[w];
    mask[gi] = on;
    hn[gi] = hh;
    hun[gi] = mm;
    hwn[gi] = kk;
    if (!on) {
      p[gi] = 0.0;
      final_state(P.g, hh, mm, kk, smax, fl2);
    }
  }
  int rank[T / NT];
  bool on[T / NT];
  const int m = tile_ranks<T, NT>([&](int k) { return k <= len && S.mk[k] != 0; }, rank, on);
  // the one-kernel step's marked tiles fold these speeds into their
  // projection's flush (one flush, after the critical path's polls)
  if (!ONE || m == 0) flush_speed<NT>(P, tl.x, par, smax, fl2);
  const int F = 2 * blockIdx.x, L = F + 1;
  if (threadIdx.x == 0) {
    P.tile_cnt[blockIdx.x] = m;
    if (m) {
      atomicAdd(&P.n_acc[par], m);
      if (!ONE) P.mlist[atomicAdd(P.mcount, 1)] = blockIdx.x;  // for the projection
    }
  }
  // one-kernel step: the tag of this step's words; the level-1 scratch (the
  // marked tiles' list, staged rows) lives in the LDS union once the block's
  // own tile is done
  const unsigned tag = ONE ? *P.tag1 + 1u : 0u;
  // the count goes out as soon as it is known, so that it is visible long
  // before the marked tiles finish their elliptic rows and poll the counts
  if (ONE && threadIdx.x == 0) put_tagged(P.tw + blockIdx.x, (unsigned)m, tag);
  unsigned long long pre[ONEPASS_NI];  // ONE: the count words, loaded before the tile reduction
  int* l1tl = reinterpret_cast<int*>(&S.u);
  double(*l1st)[6] = reinterpret_cast<double(*)[6]>(reinterpret_cast<char*>(&S.u) +
                                                     sizeof(int) * ONEPASS_TILES);
  if (m == 0) {
    if constexpr (ONE) {
      if (blockIdx.x == 0) {
        unsigned long long pre[ONEPASS_NI];
#pragma unroll
        for (int i = 0; i < ONEPASS_NI; i++) pre[i] = 0ull;
        const int nm = onepass_counts(P, tag, l1tl, pre);
        if (nm >= 0) {
          onepass_block0(P, par, tag);
          if (nm > 64) onepass_solve_publish(P, tag, l1tl, nm, l1st);
        }
      }
    } else {
      if (threadIdx.x == 0) {
        P.dg1[F] = 1.0;
        P.up1[F] = 0.0;
        P.rh1[F] = 0.0;
        P.dg1[L] = 1.0;
        P.up1[L] = 0.0;
        P.rh1[L] = 0.0;
      }
    }
    return;
  }
  // ---- elliptic rows of the marked cells (Eqs. 10-17 at t^{n+1}) ----
  for (int k = threadIdx.x; k < len + 2; k += NT)
    S.u.q.cq[k] = cell_win(QW, P, c, M1, reflect(start - 1 + k, n));
  __syncthreads();
  for (int f = threadIdx.x; f <= len; f += NT)
    S.u.q.fq[f] = face_win(QW, P, dt, start + f, S.u.q.cq[f].phi, S.u.q.cq[f + 1].phi);
  __syncthreads();
  const int64_t zs = (int64_t)P.ntiles * T;  // stride of the zw planes
  const int64_t pb = (int64_t)blockIdx.x * T;
  double ra[T / NT], rb[T / NT], rc[T / NT], rd[T / NT];
  double zr[T / NT][ZW_N];  // ONE: the projection data of the thread's cells, kept in registers
#pragma unroll
  for (int q = 0; q < T / NT; q++) {
    if (!on[q]) continue;
    const int k = 1 + threadIdx.x + NT * q;
    const int i = start + k - 1, w = i - lo;
    const FaceNH fl = S.u.q.fq[k - 1], fr = S.u.q.fq[k];
    const CellNH c0 = S.u.q.cq[k];
    const double hs = S.e[w], ms = S.m[w], ks = S.k[w];
    const double rh = rcp64(hs), dtr = dt / P.rho;
    const double s22 = 3.0 * dtr * rh;
    const BedRate br = bed_rate(M1, body_shape(c, (i + 0.5) * P.dx - M1.X, 0.0));
    const double f2 = -2.0 * br.d_t - (2.0 * ks + 0.5 * c0.D * ms + 0.5 * dtr * c0.al * c0.phi) * rh;
    ra[q] = (i > 0 && S.mk[k - 1]) ? fl.K * fl.a * fl.b : 0.0;
    rb[q] = s22 + fl.K * fl.b * fl.b + fr.K * fr.a * fr.a;
    rc[q] = (i + 1 < n && S.mk[k + 1]) ? fr.K * fr.a * fr.b : 0.0;
    rd[q] = f2 + fl.b * fl.qp + fr.a * fr.qp;
    S.cell_of[rank[q]] = (short)(k - 1);
    if constexpr (ONE) {
      zr[q][ZW_KL] = fl.K;
      zr[q][ZW_AL] = fl.a;
      zr[q][ZW_BL] = fl.b;
      zr[q][ZW_FL] = fl.fd;
      zr[q][ZW_KR] = fr.K;
      zr[q][ZW_AR] = fr.a;
      zr[q][ZW_BR] = fr.b;
      zr[q][ZW_FR] = fr.fd;
      zr[q][ZW_D] = c0.D;
      zr[q][ZW_P] = c0.al * c0.phi / 4.0;
      zr[q][ZW_HT] = hs;
      zr[q][ZW_MT] = ms;
      zr[q][ZW_KT] = ks;
    } else {
      double* z = P.zw + pb + (k - 1);  // in cell order: the projection needs no ranks
      z[ZW_KL * zs] = fl.K;
      z[ZW_AL * zs] = fl.a;
      z[ZW_BL * zs] = fl.b;
      z[ZW_FL * zs] = fl.fd;
      z[ZW_KR * zs] = fr.K;
      z[ZW_AR * zs] = fr.a;
      z[ZW_BR * zs] = fr.b;
      z[ZW_FR * zs] = fr.fd;
      z[ZW_D * zs] = c0.D;
      z[ZW_P * zs] = c0.al * c0.phi / 4.0;
      z[ZW_HT * zs] = hs;
      z[ZW_MT * zs] = ms;
      z[ZW_KT * zs] = ks;
    }
  }
  // a marked tile needs every count once its rows are out: load them now, so
  // that the loads return during the tile reduction; the counts of the
  // slowest tiles are not out yet and are polled again after it
  if constexpr (ONE) onepass_prefetch(P, pre);
  __syncthreads();  // cq, fq dead: the tile system takes their place
  auto& Y = S.u.s[0];
  for (int j = threadIdx.x; j < RW; j += NT) {
    Y.a[j] = 0.0;
    Y.b[j] = 1.0;
    Y.c[j] = 0.0;
    Y.d[0][j] = 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < T / NT; q++) {
    if (!on[q]) continue;
    const int j = rank[q];
    Y.a[j] = ra[q];
    Y.b[j] = rb[q];
    Y.c[j] = rc[q];
    Y.d[0][j] = rd[q];
  }
  __syncthreads();
  double l1v[6];  // thread 0: the tile's level-1 rows (F: dg, up, rh; L: dg, up, rh)
  if (m == 1) {
    const bool asL = Y.c[0] != 0.0;  // couples to the next tile's first row
    if (threadIdx.x == 0) {
      l1v[0] = asL ? 1.0 : Y.b[0];
      l1v[1] = 0.0;
      l1v[2] = asL ? 0.0 : Y.d[0][0];
      l1v[3] = asL ? Y.b[0] : 1.0;
      l1v[4] = asL ? Y.c[0] : 0.0;
      l1v[5] = asL ? Y.d[0][0] : 0.0;
    }
    if constexpr (ONE) {
#pragma unroll
      for (int q = 0; q < T / NT; q++) {
        zr[q][ZW_Z] = 0.0;
        zr[q][ZW_U] = asL ? 0.0 : 1.0;
        zr[q][ZW_V] = asL ? 1.0 : 0.0;
      }
    } else if (threadIdx.x == 0) {
      const int64_t cz = pb + S.cell_of[0];
      P.zw[cz + ZW_Z * zs] = 0.0;
      P.zw[cz + ZW_U * zs] = asL ? 0.0 : 1.0;
      P.zw[cz + ZW_V * zs] = asL ? 1.0 : 0.0;
    }
  } else if constexpr (F32R) {
    double berr;
    const int sw = refine_tile32<T, NT>(S, m, ra, rb, rc, rd, rank, on, P.tol, P.max_sweeps, berr);
    if (threadIdx.x == 0) {
      atomicMax(&P.sweeps[par], sw < 0 ? -1 - sw : sw);
      atomicMax(&P.berr[par], pos_bits(berr));
      if (sw < 0) atomicOr(P.status, ST_NOCONV);
    }
    const auto& GX = S.u.g.x;
    if constexpr (ONE) {
#pragma unroll
      for (int q = 0; q < T / NT; q++) {
        if (!on[q]) continue;
        const int j = rank[q];
        zr[q][ZW_Z] = GX[0][j];
        zr[q][ZW_U] = GX[1][j];
        zr[q][ZW_V] = GX[2][j];
      }
    } else {
      for (int j = threadIdx.x; j < m; j += NT) {
        const int64_t cz = pb + S.cell_of[j];
        P.zw[cz + ZW_Z * zs] = GX[0][j];
        P.zw[cz + ZW_U * zs] = GX[1][j];
        P.zw[cz + ZW_V * zs] = GX[2][j];
      }
    }
    if (threadIdx.x == 0) {
      const double* E = S.u.g.ends;
      l1v[0] = E[0] + E[1] * GX[1][1];
      l1v[1] = E[1] * GX[2][1];
      l1v[2] = E[2] - E[1] * GX[0][1];
      l1v[3] = E[4] + E[3] * GX[2][m - 2];
      l1v[4] = E[5];
      l1v[5] = E[6] - E[3] * GX[0][m - 2];
    }
  } else {
    // keep the end rows, then pin them: x_first and x_last become parameters
    const double b0 = Y.b[0], c0 = Y.c[0], d0 = Y.d[0][0];
    const double aL = Y.a[m - 1], bL = Y.b[m - 1], cL = Y.c[m - 1], dL = Y.d[0][m - 1];
    __syncthreads();
    for (int j = threadIdx.x; j < RW; j += NT) {
      const bool first = j == 0, last = j == m - 1;
      if (first || last) {
        Y.a[j] = 0.0;
        Y.c[j] = 0.0;
        Y.b[j] = 1.0;
        Y.d[0][j] = 0.0;
      }
      Y.d[1][j] = first ? 1.0 : 0.0;
      Y.d[2][j] = last ? 1.0 : 0.0;
      Y.r[j] = rcp64(Y.b[j]);
    }
    __syncthreads();
    const auto& X = S.u.s[pcr_tile<T, NT>(S, m)];
    if constexpr (ONE) {
#pragma unroll
      for (int q = 0; q < T / NT; q++) {
        if (!on[q]) continue;
        const int j = rank[q];
        const double ib = X.r[j];
        zr[q][ZW_Z] = X.d[0][j] * ib;
        zr[q][ZW_U] = X.d[1][j] * ib;
        zr[q][ZW_V] = X.d[2][j] * ib;
      }
    } else {
      for (int j = threadIdx.x; j < m; j += NT) {
        const double ib = X.r[j];
        const int64_t cz = pb + S.cell_of[j];
        P.zw[cz + ZW_Z * zs] = X.d[0][j] * ib;
        P.zw[cz + ZW_U * zs] = X.d[1][j] * ib;
        P.zw[cz + ZW_V * zs] = X.d[2][j] * ib;
      }
    }
    if (threadIdx.x == 0) {
      const double z1 = X.d[0][1] * X.r[1], u1 = X.d[1][1] * X.r[1], v1 = X.d[2][1] * X.r[1];
      const double zL = X.d[0][m - 2] * X.r[m - 2], vL = X.d[2][m - 2] * X.r[m - 2];
      l1v[0] = b0 + c0 * u1;
      l1v[1] = c0 * v1;
      l1v[2] = d0 - c0 * z1;
      l1v[3] = bL + aL * vL;
      l1v[4] = cL;
      l1v[5] = dL - aL * zL;
    }
  }
  if constexpr (!ONE) {
    if (threadIdx.x == 0) {
      P.dg1[F] = l1v[0];
      P.up1[F] = l1v[1];
      P.rh1[F] = l1v[2];
      P.dg1[L] = l1v[3];
      P.up1[L] = l1v[4];
      P.rh1[L] = l1v[5];
    }
  } else {
    // ---- one-kernel step: publish the rows, gather every marked tile's
    // rows and solve the level-1 system here (up to 64 marked tiles; beyond,
    // block 0 solves and publishes), then project the marked cells ----
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < 6; k++)
        put_tagged(P.tw + P.ntiles + ((size_t)blockIdx.x * 6 + k) * 2, l1v[k], tag);
    }
    const int nm = onepass_counts(P, tag, l1tl, pre);
    if (nm < 0) return;
    if (blockIdx.x == 0) onepass_block0(P, par, tag);
    const bool nb_l = start > 0 && S.mk[0] != 0, nb_r = end < n && S.mk[len + 1] != 0;
    __shared__ double xv[4];  // x of the tile's F and L rows, of the previous L, of the next F
    __shared__ int xok;
    if (nm <= 64) {
      if (!onepass_solve_local(P, tag, l1tl, nm, nb_l, nb_r, xv)) return;
    } else {
      bool ok = true;
      if (blockIdx.x == 0) ok = onepass_solve_publish(P, tag, l1tl, nm, l1st);
      if (threadIdx.x < 64) {
        const unsigned long long* xw = P.tw + 13 * (size_t)P.ntiles;
        const int j = threadIdx.x;
        double v = 0.0;
        bool good = ok;
        if (j < 4 && ok && (j < 2 || (j == 2 && nb_l) || (j == 3 && nb_r))) {
          const int64_t tt = j == 2 ? (int64_t)blockIdx.x - 1 : j == 3 ? (int64_t)blockIdx.x + 1
                                                                        : (int64_t)blockIdx.x;
          good = poll_tagged(xw + tt * 4 + (j == 1 || j == 2 ? 2 : 0), tag, v, P.status);
        }
        if (j < 4) xv[j] = v;
        const unsigned long long bad = __ballot(!good);
        if (j == 0) xok = bad ? 0 : 1;
      }
      __syncthreads();
      if (!xok) return;
    }
    double* xs = reinterpret_cast<double*>(&S.u);  // p on tile cells 0 .. len + 1
#pragma unroll
    for (int q = 0; q < T / NT; q++) {
      const int k = 1 + threadIdx.x + NT * q;
      if (k > len) continue;
      xs[k] = on[q] ? zr[q][ZW_Z] + zr[q][ZW_U] * xv[0] + zr[q][ZW_V] * xv[1] : 0.0;
    }
    if (threadIdx.x == 0) {
      xs[0] = nb_l ? xv[2] : 0.0;
      xs[len + 1] = nb_r ? xv[3] : 0.0;
    }
    __syncthreads();
    const double rdt4 = P.rho / (4.0 * dt), dtr = dt / P.rho;
    double sp = smax;  // the unmarked cells' speed and flags from above
    int fl3 = fl2;
#pragma unroll
    for (int q = 0; q < T / NT; q++) {
      if (!on[q]) continue;
      const int k = 1 + threadIdx.x + NT * q;
      const int64_t gi = off + start + k - 1;
      const double* z = zr[q];
      const double pc = xs[k], pl = xs[k - 1], pr = xs[k + 1];
      const double dql = z[ZW_FL] - z[ZW_KL] * (z[ZW_AL] * pl + z[ZW_BL] * pc);
      const double dqr = z[ZW_FR] - z[ZW_KR] * (z[ZW_AR] * pc + z[ZW_BR] * pr);
      const double dm = 0.5 * (dql + dqr);
      const double Pb = 1.5 * pc - rdt4 * z[ZW_D] * dm + z[ZW_P];
      const double mn = z[ZW_MT] + dm, kn = z[ZW_KT] + dtr * Pb;
      hun[gi] = mn;
      hwn[gi] = kn;
      p[gi] = pc;
      final_state(P.g, z[ZW_HT], mn, kn, sp, fl3);
    }
    flush_speed<NT>(P, tl.x, par, sp, fl3);
  }
}



// LDS of the level-1 solve of one channel (rows of its marked tiles)
template <int NT>
struct L1Smem {
  double la[L1MAX], lb[L1MAX], lc[L1MAX], ld[L1MAX], lr[L1MAX];
  double rdg[L1MAX], rup[L1MAX], rrh[L1MAX];  // level-1 rows as stored (2 per tile)
  int rcnt[L1MAX / 2];
  int tpos[L1MAX / 2], tlist[L1MAX / 2];  // tile <-> compact level-1 tile
  int wc[NT / 64];
};

// The level-1 system of the tiles [t_lo, t_lo + ntc) (one channel, at most
// L1MAX / 2 tiles: the channels' systems are decoupled) restricted to its
// marked tiles (an unmarked tile's two identity rows are decoupled from
// everything), in tile order, solved in LDS by the whole block: after it,
// row k of local tile t (marked) has x = ld[r] lr[r], r = 2 tpos[t] + k.
// Parallel cyclic reduction (lr holds 1 / lb); up to 64 rows on one
// wavefront, up to 128 with one elimination level before that.
template <int NT>
__device__ void level1_solve_lds(const K1D& P, int t_lo, int ntc, L1Smem<NT>& S) {
  // the channel's level-1 rows and tile counts in one round of loads
  for (int g = threadIdx.x; g < 2 * ntc; g += NT) {
    S.rdg[g] = P.dg1[2 * t_lo + g];
    S.rup[g] = P.up1[2 * t_lo + g];
    S.rrh[g] = P.rh1[2 * t_lo + g];
  }
  for (int t = threadIdx.x; t < ntc; t += NT) S.rcnt[t] = P.tile_cnt[t_lo + t];
  __syncthreads();
  int base = 0;
  for (int t0 = 0; t0 < ntc; t0 += NT) {
    const int t = t0 + threadIdx.x;
    const bool mt = t < ntc && S.rcnt[t] > 0;
    const unsigned long long bal = __ballot(mt);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) S.wc[wv] = __popcll(bal);
    __syncthreads();
    int wb = 0, tot = 0;
    for (int w = 0; w < NT / 64; w++) {
      if (w < wv) wb += S.wc[w];
      tot += S.wc[w];
    }
    const int r = base + wb + __popcll(bal & ((1ull << lane) - 1ull));
    if (t < ntc) S.tpos[t] = mt ? r : -1;
    if (mt) S.tlist[r] = t;
    base += tot;
    __syncthreads();
  }
  const int n1 = 2 * base;
  // coupling of compact row j to row j + 1
  auto up_c = [&](int j) {
    const int t = S.tlist[j >> 1];
    if ((j & 1) == 0) return S.rup[2 * t];
    return (j + 1 < n1 && S.tlist[(j >> 1) + 1] == t + 1) ? S.rup[2 * t + 1] : 0.0;
  };
  if (n1 <= 64) {
    // one wavefront solves it in registers; the others wait
    if (threadIdx.x < 64) {
      const int j = threadIdx.x;
      double a = 0.0, b = 1.0, c = 0.0, d = 0.0;
      if (j < n1) {
        const int g = 2 * S.tlist[j >> 1] + (j & 1);
        a = j > 0 ? up_c(j - 1) : 0.0;
        b = S.rdg[g];
        c = up_c(j);
        d = S.rrh[g];
      }
      S.ld[j] = wave_pcr(a, b, c, d, n1);
      S.lr[j] = 1.0;
    }
    __syncthreads();
  } else if (n1 <= 128) {
    // two rows per lane (2l, 2l + 1): one cyclic-reduction level
    // eliminates the odd rows, one wavefront solves the even rows as
    // above, and each odd row follows from its two even neighbours
    if (threadIdx.x < 64) {
      const int l = threadIdx.x, j0 = 2 * l, j1 = j0 + 1;
      double a0 = 0.0, b0 = 1.0, c0 = 0.0, d0 = 0.0;
      double a1 = 0.0, b1 = 1.0, c1 = 0.0, d1 = 0.0;
      if (j0 < n1) {
        const int g = 2 * S.tlist[j0 >> 1];
        a0 = j0 > 0 ? up_c(j0 - 1) : 0.0;
        b0 = S.rdg[g];
        c0 = up_c(j0);
        d0 = S.rrh[g];
      }
      if (j1 < n1) {
        const int g = 2 * S.tlist[j1 >> 1] + 1;
        a1 = up_c(j0);
        b1 = S.rdg[g];
        c1 = up_c(j1);
        d1 = S.rrh[g];
      }
      const double am = __shfl_up(a1, 1), bm = __shfl_up(b1, 1), cm = __shfl_up(c1, 1),
                   dm = __shfl_up(d1, 1);  // row 2l - 1
      double na = 0.0, nb = b0, nd = d0;
      if (l > 0) {
        const double k1 = a0 * rcp64(bm);
        na = -am * k1;
        nb -= cm * k1;
        nd -= dm * k1;
      }
      const double r1 = rcp64(b1), k2 = c0 * r1;
      const double nc = -c1 * k2;
      nb -= a1 * k2;
      nd -= d1 * k2;
      const double xe = wave_pcr(na, nb, nc, nd, (n1 + 1) >> 1);
      const double xn = __shfl_down(xe, 1);  // x of row 2l + 2
      S.ld[j0] = xe;
      S.ld[j1] = (d1 - a1 * xe - (l < 63 ? c1 * xn : 0.0)) * r1;
      S.lr[j0] = 1.0;
      S.lr[j1] = 1.0;
    }
    __syncthreads();
  } else {
    for (int j = threadIdx.x; j < L1MAX; j += NT) {
      if (j < n1) {
        const int g = 2 * S.tlist[j >> 1] + (j & 1);
        S.la[j] = j > 0 ? up_c(j - 1) : 0.0;
        S.lb[j] = S.rdg[g];
        S.lc[j] = up_c(j);
        S.ld[j] = S.rrh[g];
      } else {
        S.la[j] = 0.0;
        S.lb[j] = 1.0;
        S.lc[j] = 0.0;
        S.ld[j] = 0.0;
      }
      S.lr[j] = rcp64(S.lb[j]);
    }
    __syncthreads();
    for (int s = 1; s < n1; s <<= 1) {
      double na[(L1MAX / NT)], nb[(L1MAX / NT)], nc[(L1MAX / NT)], nd[(L1MAX / NT)];
#pragma unroll
      for (int r = 0; r < (L1MAX / NT); r++) {
        const int i = threadIdx.x + NT * r;
        if (i >= n1) continue;
        const int im = i - s, ip = i + s;
        double ai = 0.0, bi = S.lb[i], ci = 0.0, di = S.ld[i];
        if (im >= 0) {
          const double k1 = S.la[i] * S.lr[im];
          ai = -S.la[im] * k1;
          bi -= S.lc[im] * k1;
          di -= S.ld[im] * k1;
        }
        if (ip < L1MAX) {
          const double k2 = S.lc[i] * S.lr[ip];
          ci = -S.lc[ip] * k2;
          bi -= S.la[ip] * k2;
          di -= S.ld[ip] * k2;
        }
        na[r] = ai;
        nb[r] = bi;
        nc[r] = ci;
        nd[r] = di;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < (L1MAX / NT); r++) {
        const int i = threadIdx.x + NT * r;
        if (i >= n1) continue;
        S.la[i] = na[r];
        S.lb[i] = nb[r];
        S.lc[i] = nc[r];
        S.ld[i] = nd[r];
        S.lr[i] = rcp64(nb[r]);
      }
      __syncthreads();
    }
  }
}

// the projection of tile b (nothing for a tile without marked cells)
template <int T, int NT, bool L1LOCAL>
__device__ __forceinline__ void apply_tile(const K1D& P, int b, const uint8_t* __restrict__ mask,
                                           double* hun, double* hwn, double* p, int par,
                                           double* xs, L1Smem<NT>* L1S) {
  const int4 tl = P.tiles[b];
  const int n = tl.w, start = tl.y, end = min(start + P.tile, n), len = end - start;
  const int64_t off = tl.z;
  const double dt = P.dt[tl.x];
  const int m = P.tile_cnt[b];
  if (m == 0) return;  // no marked cell: the step kernel already took this tile's speed
  double smax = 0.0;
  int flags = 0;
  {
    // the tile's marked cells and their stored data (cell order) first, in
    // one round of loads (the data of unmarked cells is read and ignored):
    // they are in flight while the level-1 system is solved
    bool on[T / NT];
    const int64_t m0 = off + start - 1;  // mask[m0 + k]: tile-local cell k
    const int64_t zs = (int64_t)P.ntiles * T;
    const int64_t pb = (int64_t)b * T;
    double zr[T / NT][ZW_N];
#pragma unroll
    for (int q = 0; q < T / NT; q++) {
      const int k = 1 + threadIdx.x + NT * q;
      on[q] = false;
      if (k > len) continue;
      on[q] = mask[m0 + k] != 0;
      const double* z = P.zw + pb + (k - 1);
#pragma unroll
      for (int v = 0; v < ZW_N; v++) zr[q][v] = z[v * zs];
    }
    const bool nb_l = start > 0 && mask[m0], nb_r = end < n && mask[m0 + len + 1];
    // the channel's tiles [t_lo, t_lo + ntc): local tile t <-> tile t_lo + t
    const int t_lo = L1LOCAL ? P.first_tile[tl.x] : 0;
    const int ntc = L1LOCAL ? (tl.x + 1 < P.nch ? P.first_tile[tl.x + 1] : P.ntiles) - t_lo : 0;
    // level-1 solution of row j (= 2 tile + 0 first / 1 last)
    auto x1 = [&](int j) {
      if (!L1LOCAL) return P.x1[j];
      const int jl = j - 2 * t_lo;
      const int r = 2 * L1S->tpos[jl >> 1] + (jl & 1);
      return L1S->ld[r] * L1S->lr[r];
    };
    if (L1LOCAL) level1_solve_lds<NT>(P, t_lo, ntc, *L1S);
    const double xF = x1(2 * b), xL = x1(2 * b + 1);
#pragma unroll
    for (int q = 0; q < T / NT; q++) {
      const int k = 1 + threadIdx.x + NT * q;
      if (k > len) continue;
      xs[k] = on[q] ? zr[q][ZW_Z] + zr[q][ZW_U] * xF + zr[q][ZW_V] * xL : 0.0;
    }
    if (threadIdx.x == 0) {
      xs[0] = nb_l ? x1(2 * b - 1) : 0.0;
      xs[len + 1] = nb_r ? x1(2 * b + 2) : 0.0;
    }
    __syncthreads();
    const double rdt4 = P.rho / (4.0 * dt), dtr = dt / P.rho;
#pragma unroll
    for (int q = 0; q < T / NT; q++) {
      if (!on[q]) continue;
      const int k = 1 + threadIdx.x + NT * q;
      const int64_t gi = off + start + k - 1;
      const double* z = zr[q];
      const double pc = xs[k], pl = xs[k - 1], pr = xs[k + 1];
      const double dql = z[ZW_FL] - z[ZW_KL] * (z[ZW_AL] * pl + z[ZW_BL] * pc);
      const double dqr = z[ZW_FR] - z[ZW_KR] * (z[ZW_AR] * pc + z[ZW_BR] * pr);
      const double dm = 0.5 * (dql + dqr);
      const double Pb = 1.5 * pc - rdt4 * z[ZW_D] * dm + z[ZW_P];
      const double mn = z[ZW_MT] + dm, kn = z[ZW_KT] + dtr * Pb;
      hun[gi] = mn;
      hwn[gi] = kn;
      p[gi] = pc;
      final_state(P.g, z[ZW_HT], mn, kn, smax, flags);
    }
  }
  flush_speed<NT>(P, tl.x, par, smax, flags);
}

// Projection of the marked cells (a6) from the level-1 solution -- solved
// here, redundantly by every tile that needs it, when the whole level-1
// system has at most L1MAX rows (L1LOCAL: one block per tile, each solving
// its channel's part; the channels' systems are decoupled), else read from
// P.x1 (a grid of at most APPLY_GRID blocks walks the list of marked tiles
// the step kernel appended: on the ensemble most tiles have no marked cell,
// and a block per tile spent some 30 us launching blocks that exit at once)
// -- and the speed of their new state.  par: parity of the step within the
// run (the time, step counter, marked count and speed buffers alternate with
// it).
constexpr int APPLY_GRID = 2048;
template <int T, int NT, bool L1LOCAL>
__global__ void __launch_bounds__(NT) k_apply1d(K1D P, const uint8_t* __restrict__ mask,
                                                double* hun, double* hwn, double* p,
                                                int par) {
  __shared__ double xs[T + 2];
  // the level-1 solve's LDS only where this kernel solves it
  __shared__ typename std::conditional<L1LOCAL, L1Smem<NT>, char>::type l1s;
  if constexpr (L1LOCAL) {
    apply_tile<T, NT, true>(P, blockIdx.x, mask, hun, hwn, p, par, xs, &l1s);
  } else {
    const int nm = *P.mcount;
    for (int k = blockIdx.x; k < nm; k += gridDim.x) {
      __syncthreads();  // the previous tile's last reads of xs
      apply_tile<T, NT, false>(P, P.mlist[k], mask, hun, hwn, p, par, xs, nullptr);
    }
  }
}

// The level-1 systems of the channels when the whole system is too large
// for the projection kernel but each channel's part fits (at most L1MAX
// rows), one block per channel: the marked tiles' solution into P.x1 (an
// unmarked tile's rows are identity rows with a zero right-hand side: 0)
template <int NT>
__global__ void __launch_bounds__(NT) k_level1_chan(K1D P) {
  __shared__ L1Smem<NT> S;
  const int ch = blockIdx.x;
  const int t_lo = P.first_tile[ch];
  const int ntc = (ch + 1 < P.nch ? P.first_tile[ch + 1] : P.ntiles) - t_lo;
  level1_solve_lds<NT>(P, t_lo, ntc, S);
  for (int g = threadIdx.x; g < 2 * ntc; g += NT) {
    const int r = S.tpos[g >> 1], k = 2 * r + (g & 1);
    P.x1[2 * t_lo + g] = r >= 0 ? S.ld[k] * S.lr[k] : 0.0;
  }
}

// the two-kernel step's table: per channel (one wavefront each), dt from the
// speed slots of buffer `par` (their maximum, read by one lane each as
// read_speed does, then cleared) and the body's motion at both ends of the
// step (lanes 0 and 1); the step's dt and the next step's start time go to
// P.dt and P.t[par ^ 1] here, so the step kernel's blocks only read them
__global__ void __launch_bounds__(256) k_chan_step(K1D P, int par) {
  const int ch = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0) *P.mcount = 0;  // the step's marked-tile list
  if (ch >= P.nch) return;
  const double dt = (P.cfl > 0.0) ? P.cfl * P.dx / read_speed(P, par, ch) : P.dt_fixed;
  // the slots just read collect the speed of the step after next (stage
  // timing replays the step and keeps them)
  if (!P.keep_speed && lane < P.nslot)
    P.smax[speed_at(par * P.nch + ch, lane, P.nslot)] = 0ull;
  const double t0 = P.t[par * P.nch + ch];
  if (lane < 2) {
    const Motion M = body_motion(P.ch[ch], lane == 0 ? t0 : t0 + dt);
    double* ct = P.ctab + (size_t)ch * CTAB_N + (lane == 0 ? CT_X0 : CT_X1);
    ct[0] = M.X;
    ct[1] = M.V;
    ct[2] = M.A;
    if (lane == 0) {
      P.ctab[(size_t)ch * CTAB_N + CT_DT] = dt;
      P.dt[ch] = dt;
      P.t[(par ^ 1) * P.nch + ch] = t0 + dt;
    }
  }
}

// prologue of a run of fused steps: both speed buffers and the first marked
// count cleared (buffer 0 then collects the speed of the caller's state)
__global__ void k_run_begin(K1D P) {
  for (int i = threadIdx.x; i < 2 * P.nch * P.nslot; i += blockDim.x)
    P.smax[(size_t)i * SPEED_PAD] = 0ull;
  if (threadIdx.x == 0) {
    P.n_acc[0] = 0;
    if (P.refine) {
      P.sweeps[0] = 0;
      P.berr[0] = 0ull;
    }
  }
}

// end of a run of fused steps: time, step counter and the speed of the new
// state back in slot 0, the last step's marked count published
__global__ void k_run_end(K1D P, int last_par) {
  if (last_par) {
    for (int ch = threadIdx.x; ch < P.nch; ch += blockDim.x) P.t[ch] = P.t[P.nch + ch];
    const int ns = P.nch * P.nslot;
    for (int i = threadIdx.x; i < ns; i += blockDim.x)
      P.smax[(size_t)i * SPEED_PAD] = P.smax[(size_t)(ns + i) * SPEED_PAD];
  }
  if (threadIdx.x == 0) {
    if (last_par) P.step[0] = P.step[1];
    *P.n_act = P.n_acc[last_par ^ 1];
    if (P.refine) {  // the last step's refinement: most sweeps, largest backward error
      *P.iters_out = P.sweeps[last_par ^ 1];
      *P.rel_out = __longlong_as_double((long long)P.berr[last_par ^ 1]);
    }
  }
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_f64(double* a, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
// p (packed rows) -> full array
__global__ void k_gather_packed(const int* __restrict__ act_cell, const int* n_act,
                                const double* __restrict__ full, double* __restrict__ packed) {
  const int na = *n_act;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < na; k += gridDim.x * blockDim.x)
    packed[k] = full[act_cell[k]];
}
__global__ void k_scatter_packed(const int* __restrict__ act_cell, const int* n_act,
                                 const double* __restrict__ packed, double* __restrict__ full) {
  const int na = *n_act;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < na; k += gridDim.x * blockDim.x)
    full[act_cell[k]] = packed[k];
}

// end of a step: t += dt, speed reset, step counter
__global__ void k_advance(K1D P, int nch) {
  for (int c = threadIdx.x; c < nch; c += blockDim.x) P.t[c] += P.dt[c];
  for (int i = threadIdx.x; i < nch * P.nslot; i += blockDim.x) P.smax[(size_t)i * SPEED_PAD] = 0ull;
  if (threadIdx.x == 0) *P.step += 1;
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }
// grid of the kernels that walk the marked rows with a grid-stride loop: the
// row count lives on the device, and a grid sized by the host bound (every
// cell) spent most of its time in blocks that only load the count and exit
static inline int rows_grid(int64_t max_rows) {
  const int b = blocks_for(max_rows, 256);
  return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}

void launch_speed1d(const K1D& P, const double* h, const double* hu, const double* hw,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_speed1d, dim3(P.ntiles), dim3(256), 0, s, P, h, hu, hw);
}
void launch_pred1d(const K1D& P, const double* h, const double* hu, const double* hw, double* ht,
                   double* mt, double* kt, const double* t_in, const double* dt_in,
                   int dt_from_speed, hipStream_t s) {
  if (P.cap == 128)
    hipLaunchKernelGGL((k_pred1d<128, 128>), dim3(P.ntiles), dim3(128), 0, s, P, h, hu, hw, ht, mt,
                       kt, t_in, dt_in, dt_from_speed);
  else if (P.cap == 256)
    hipLaunchKernelGGL((k_pred1d<256, 256>), dim3(P.ntiles), dim3(256), 0, s, P, h, hu, hw, ht, mt,
                       kt, t_in, dt_in, dt_from_speed);
  else
    hipLaunchKernelGGL((k_pred1d<512, 256>), dim3(P.ntiles), dim3(256), 0, s, P, h, hu, hw, ht, mt,
                       kt, t_in, dt_in, dt_from_speed);
}
void launch_mask1d(const K1D& P, const double* ht, const double* mt, const double* kt,
                   const double* t_in, const double* dt_in, int mode_override, uint8_t* mask,
                   double* h, double* hu, double* hw, double* p, int write_state, hipStream_t s) {
  hipLaunchKernelGGL(k_mask1d, dim3(P.ntiles), dim3(256), 0, s, P, ht, mt, kt, t_in, dt_in,
                     mode_override, mask, h, hu, hw, p, write_state);
}
void launch_count1d(const K1D& P, const uint8_t* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_count1d, dim3(P.ntiles), dim3(256), 0, s, P, mask);
}
void launch_scan(const int* cnt, int* off, int n, int* total, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cnt, off, n, total);
}
void launch_compact1d(const K1D& P, const uint8_t* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_compact1d, dim3(P.ntiles), dim3(256), 0, s, P, mask);
}
void launch_assemble1d(const K1D& P, int64_t max_rows, const double* ht, const double* mt,
                       const double* kt, const uint8_t* mask, const double* t_in,
                       const double* dt_in, double* dg, double* up, double* rh, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble1d, dim3(rows_grid(max_rows)), dim3(256), 0, s, P, ht, mt,
                     kt, mask, t_in, dt_in, dg, up, rh);
}
void launch_correct1d(const K1D& P, int64_t max_rows, const double* ht, const double* mt,
                      const double* kt, const uint8_t* mask, const double* t_in,
                      const double* dt_in, const double* x, double* hu, double* hw, double* p,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_correct1d, dim3(rows_grid(max_rows)), dim3(256), 0, s, P, ht, mt,
                     kt, mask, t_in, dt_in, x, hu, hw, p);
}
void launch_advance(const K1D& P, int nch, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(256), 0, s, P, nch);
}
void launch_fill(double* a, int64_t n, double v, hipStream_t s) {
  int b = blocks_for(n, 256);
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_fill_f64, dim3(b), dim3(256), 0, s, a, n, v);
}
__global__ void k_fill_i32(int* a, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
void launch_fill_i32(int* a, int64_t n, int v, hipStream_t s) {
  int b = blocks_for(n, 256);
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_fill_i32, dim3(b), dim3(256), 0, s, a, n, v);
}
void launch_copy(const double* a, double* b, int64_t n, hipStream_t s) {
  int g = blocks_for(n, 256);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_copy_f64, dim3(g), dim3(256), 0, s, a, b, n);
}
void launch_gather_packed(const int* act_cell, const int* n_act, int64_t max_rows,
                          const double* full, double* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_packed, dim3(rows_grid(max_rows)), dim3(256), 0, s, act_cell,
                     n_act, full, packed);
}
void launch_scatter_packed(const int* act_cell, const int* n_act, int64_t max_rows,
                           const double* packed, double* full, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_packed, dim3(rows_grid(max_rows)), dim3(256), 0, s,
                     act_cell, n_act, packed, full);
}

template <int T, int NT>
static void launch_step_t(const K1D& P, const double* h, const double* hu, const double* hw,
                          double* hn, double* hun, double* hwn, uint8_t* mask, double* p, int par,
                          hipStream_t s) {
  if (P.onepass) {
    if (P.refine)
      hipLaunchKernelGGL((k_step1d<T, NT, true, true>), dim3(P.ntiles), dim3(NT), 0, s, P, h, hu,
                         hw, hn, hun, hwn, mask, p, par);
    else
      hipLaunchKernelGGL((k_step1d<T, NT, true, false>), dim3(P.ntiles), dim3(NT), 0, s, P, h, hu,
                         hw, hn, hun, hwn, mask, p, par);
  } else {
    hipLaunchKernelGGL(k_chan_step, dim3((P.nch + 3) / 4), dim3(256), 0, s, P, par);
    if (P.refine)
      hipLaunchKernelGGL((k_step1d<T, NT, false, true>), dim3(P.ntiles), dim3(NT), 0, s, P, h,
                         hu, hw, hn, hun, hwn, mask, p, par);
    else
      hipLaunchKernelGGL((k_step1d<T, NT, false, false>), dim3(P.ntiles), dim3(NT), 0, s, P, h,
                         hu, hw, hn, hun, hwn, mask, p, par);
  }
}
// blocks of the one-kernel step kernel that fit on the device at once
template <int T, int NT, bool F32R>
static int onepass_resident_t() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step1d<T, NT, true, F32R>, NT, 0) !=
      hipSuccess)
    return 0;
  return cus * per_cu;
}
int onepass_resident(const K1D& P) {
  if (P.refine) {
    if (P.cap == 128) return onepass_resident_t<128, 128, true>();
    if (P.cap == 256) return onepass_resident_t<256, 256, true>();
    return onepass_resident_t<512, 256, true>();
  }
  if (P.cap == 128) return onepass_resident_t<128, 128, false>();
  if (P.cap == 256) return onepass_resident_t<256, 256, false>();
  return onepass_resident_t<512, 256, false>();
}
void launch_step1d(const K1D& P, const double* h, const double* hu, const double* hw, double* hn,
                   double* hun, double* hwn, uint8_t* mask, double* p, int par, hipStream_t s) {
  if (P.cap == 128)
    launch_step_t<128, 128>(P, h, hu, hw, hn, hun, hwn, mask, p, par, s);
  else if (P.cap == 256)
    launch_step_t<256, 256>(P, h, hu, hw, hn, hun, hwn, mask, p, par, s);
  else
    launch_step_t<512, 256>(P, h, hu, hw, hn, hun, hwn, mask, p, par, s);
}
template <int T, int NT>
static void launch_apply_t(const K1D& P, const uint8_t* mask, double* hun, double* hwn, double* p,
                           int par, hipStream_t s) {
  if (level1_local(P))
    hipLaunchKernelGGL((k_apply1d<T, NT, true>), dim3(P.ntiles), dim3(NT), 0, s, P, mask, hun, hwn,
                       p, par);
  else
    hipLaunchKernelGGL((k_apply1d<T, NT, false>), dim3(std::min(P.ntiles, APPLY_GRID)), dim3(NT),
                       0, s, P, mask, hun, hwn, p, par);
}
void launch_apply1d(const K1D& P, const uint8_t* mask, double* hun, double* hwn, double* p,
                    int par, hipStream_t s) {
  if (P.cap == 128)
    launch_apply_t<128, 128>(P, mask, hun, hwn, p, par, s);
  else if (P.cap == 256)
    launch_apply_t<256, 256>(P, mask, hun, hwn, p, par, s);
  else
    launch_apply_t<512, 256>(P, mask, hun, hwn, p, par, s);
}
void launch_run_end(const K1D& P, int last_par, hipStream_t s) {
  hipLaunchKernelGGL(k_run_end, dim3(1), dim3(256), 0, s, P, last_par);
}
bool level1_local(const K1D& P) { return 2 * P.ntiles <= L1MAX; }
bool level1_per_channel(const K1D& P) { return 2 * P.max_ch_tiles <= L1MAX; }
void launch_level1_chan(const K1D& P, hipStream_t s) {
  hipLaunchKernelGGL(k_level1_chan<256>, dim3(P.nch), dim3(256), 0, s, P);
}
int fused_max_enlarge() { return EMAXF; }
void launch_speed_prologue(const K1D& P, const double* h, const double* hu, const double* hw,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_run_begin, dim3(1), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_speed1d, dim3(P.ntiles), dim3(256), 0, s, P, h, hu, hw);
}

}  // namespace swenh
