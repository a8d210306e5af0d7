// swe_nh_cnn.hip -- the warm-start network on matrix cores (gfx950).
//
// Six 3x3 convolutions with zero padding, channels 16 -> 32 -> 32 -> 32 ->
// 32 -> 32 -> 1, ReLU between layers.  Activations are BF16 in NHWC layout,
// weights are kept in FP32 (master copy, [Cout][3][3][Cin] per layer followed
// by the biases) and packed to BF16 per launch; every product accumulates in
// FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16 where a layer has 32
// input channels, v_mfma_f32_16x16x16_bf16 for the first layer's 16).
//
// A convolution is an implicit GEMM: M = 16 pixels of an image row, N = 16
// output channels, K = the input channels of one tap (32, or 16).  A block owns a 16 x 16
// pixel tile (4 waves x 4 rows), with the input patch (tile + 1-pixel halo)
// and the packed weights in LDS.  The input-gradient pass is the same kernel
// on the output gradient with the weights transposed and the taps flipped,
// times the ReLU derivative of the layer's input.  The weight gradient is a
// GEMM over pixels (M = output channel, N = (tap, input channel)) with one
// partial sum per block, reduced in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "swe_nh.h"
#include "swe_nh_cnn.h"
#include "swe_nh_common.h"

namespace swenh {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int CT = 16;       // tile edge (pixels)
constexpr int PW = CT + 2;   // patch edge
constexpr int CPAD = 8;      // channel padding of LDS rows (halves)
constexpr int NTC = 256;
constexpr int NL = 6;
constexpr int CINL[NL] = {16, 32, 32, 32, 32, 32};
constexpr int COUTL[NL] = {32, 32, 32, 32, 32, 1};

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest, ties to even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__host__ __device__ constexpr int cpad16(int c) { return c < 16 ? 16 : c; }

// ---------------------------------------------------------------------------
// weight packing: FP32 master -> BF16 LDS image [N][9][K + CPAD]
// mode 0 (forward): N = Cout (padded to 16), K = Cin, B[n][t][k] = W[n][t][k]
// mode 1 (input gradient): N = Cin, K = Cout (padded to 16),
//                          B[n][t][k] = W[k][8 - t][n]
// ---------------------------------------------------------------------------
__global__ void k_pack_w(const float* __restrict__ W, int cin, int cout, int mode,
                         uint16_t* __restrict__ out) {
  const int N = mode == 0 ? cpad16(cout) : cin;
  const int K = mode == 0 ? cin : cpad16(cout);
  const int total = N * 9 * (K + CPAD);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int k = e % (K + CPAD), t = (e / (K + CPAD)) % 9, n = e / ((K + CPAD) * 9);
    float v = 0.0f;
    if (k < K) {
      if (mode == 0) {
        if (n < cout) v = W[((int64_t)n * 9 + t) * cin + k];
      } else {
        if (k < cout) v = W[((int64_t)k * 9 + (8 - t)) * cin + n];
      }
    }
    out[e] = f2bf(v);
  }
}

// ---------------------------------------------------------------------------
// convolution as implicit GEMM (forward, or input gradient with mode 1)
//   in  : BF16 NHWC with CI channels
//   out : mode 0 relu: BF16 NHWC CO channels, max(0, acc + bias)
//         mode 0 last: FP32 [n][h][w], channel 0 of acc + bias
//         mode 1     : BF16 NHWC CO channels, acc * (gate > 0), gate NHWC CO
// ---------------------------------------------------------------------------
enum { EPI_RELU = 0, EPI_LAST = 1, EPI_GATE = 2 };

template <int CI, int CO, int EPI>
__global__ void __launch_bounds__(NTC) k_conv(const uint16_t* __restrict__ in,
                                              const uint16_t* __restrict__ wpk,
                                              const float* __restrict__ bias, int H, int W,
                                              uint16_t* __restrict__ out_bf,
                                              float* __restrict__ out_f,
                                              const uint16_t* __restrict__ gate,
                                              const int* box) {
  constexpr int RS = CI + CPAD;  // LDS row stride (halves) of a pixel / of a weight row
  __shared__ __attribute__((aligned(16))) uint16_t patch[PW * PW * RS];
  __shared__ __attribute__((aligned(16))) uint16_t wts[CO * 9 * RS];
  const int tiles_x = W / CT;
  const int tx0 = (blockIdx.x % tiles_x) * CT, ty0 = (blockIdx.x / tiles_x) * CT;
  // only the pixel tiles that meet box = [x0, x1) x [y0, y1) (null: all)
  if (box && (tx0 + CT <= box[0] || tx0 >= box[2] || ty0 + CT <= box[1] || ty0 >= box[3])) return;
  const int img = blockIdx.y;
  const int64_t ibase = (int64_t)img * H * W;
  // stage the input patch (zero outside the image) and the packed weights
  constexpr int CH4 = CI / 4;  // 8-byte chunks per pixel
  for (int e = threadIdx.x; e < PW * PW * CH4; e += NTC) {
    const int q = e % CH4, pix = e / CH4;
    const int py = pix / PW, px = pix % PW;
    const int gy = ty0 + py - 1, gx = tx0 + px - 1;
    uint2 v = make_uint2(0u, 0u);
    if (gy >= 0 && gy < H && gx >= 0 && gx < W)
      v = *reinterpret_cast<const uint2*>(in + (ibase + (int64_t)gy * W + gx) * CI + 4 * q);
    *reinterpret_cast<uint2*>(patch + pix * RS + 4 * q) = v;
  }
  for (int e = threadIdx.x; e < CO * 9 * RS / 4; e += NTC)
    reinterpret_cast<uint2*>(wts)[e] = reinterpret_cast<const uint2*>(wpk)[e];
  __syncthreads();

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int xr = lane & 15, kq = (lane >> 4) * 4;
  constexpr int NB = CO / 16;
  f4 acc[4][NB];
#pragma unroll
  for (int r = 0; r < 4; r++)
#pragma unroll
    for (int nb = 0; nb < NB; nb++) acc[r][nb] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (CI % 32 == 0) {
    // K = 32 input channels per product (gfx950's 16x16x32 BF16 form: lane
    // holds 8 consecutive k of row / column lane % 16, k0 = 8 (lane / 16))
    const int kq8 = (lane >> 4) * 8;
#pragma unroll 1
    for (int t = 0; t < 9; t++) {
      const int ky = t / 3, kx = t % 3;
#pragma unroll
      for (int c0 = 0; c0 < CI; c0 += 32) {
        bf8 b[NB];
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
          b[nb] = *reinterpret_cast<const bf8*>(wts + ((nb * 16 + xr) * 9 + t) * RS + c0 + kq8);
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int y = wv * 4 + r;
          const bf8 a =
              *reinterpret_cast<const bf8*>(patch + ((y + ky) * PW + xr + kx) * RS + c0 + kq8);
#pragma unroll
          for (int nb = 0; nb < NB; nb++)
            acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[r][nb], 0, 0, 0);
        }
      }
    }
  } else {
    // K = 16 (the first layer's 16 input channels)
#pragma unroll 1
    for (int t = 0; t < 9; t++) {
      const int ky = t / 3, kx = t % 3;
#pragma unroll
      for (int c0 = 0; c0 < CI; c0 += 16) {
        s4 b[NB];
#pragma unroll
        for (int nb = 0; nb < NB; nb++)
          b[nb] = *reinterpret_cast<const s4*>(wts + ((nb * 16 + xr) * 9 + t) * RS + c0 + kq);
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int y = wv * 4 + r;
          const s4 a =
              *reinterpret_cast<const s4*>(patch + ((y + ky) * PW + xr + kx) * RS + c0 + kq);
#pragma unroll
          for (int nb = 0; nb < NB; nb++)
            acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[nb], acc[r][nb], 0, 0, 0);
        }
      }
    }
  }
  // D[row = pixel x][col = channel]: lane holds x = kq + i, channel = nb * 16 + xr
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int gy = ty0 + wv * 4 + r;
#pragma unroll
    for (int nb = 0; nb < NB; nb++) {
      const int ch = nb * 16 + xr;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int gx = tx0 + kq + i;
        const int64_t pix = ibase + (int64_t)gy * W + gx;
        const float v = acc[r][nb][i];
        if (EPI == EPI_RELU) {
          out_bf[pix * CO + ch] = f2bf(fmaxf(v + bias[ch], 0.0f));
        } else if (EPI == EPI_LAST) {
          if (ch == 0) out_f[pix] = v + bias[0];
        } else {
          const float g = bf2f(gate[pix * CO + ch]);
          out_bf[pix * CO + ch] = f2bf(g > 0.0f ? v : 0.0f);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: part[block][co][t][ci] = sum over the block's pixels of
// dY[p][co] X[p + off(t)][ci]; part_b[block][co] = sum dY[p][co]
// ---------------------------------------------------------------------------
template <int CI, int CO>
__global__ void __launch_bounds__(NTC) k_conv_bwdw(const uint16_t* __restrict__ X,
                                                   const uint16_t* __restrict__ dY, int N, int H,
                                                   int W, float* __restrict__ part,
                                                   float* __restrict__ part_b) {
  constexpr int RX = CI + CPAD, RY = CO + CPAD;
  __shared__ __attribute__((aligned(16))) uint16_t patch[PW * PW * RX];
  __shared__ __attribute__((aligned(16))) uint16_t gy_t[CT * CT * RY];
  constexpr int MB = CO / 16, NBK = 9 * CI / 16, NOB = MB * NBK;
  constexpr int PER = (NOB + 3) / 4;
  const int tiles_x = W / CT, tiles_img = tiles_x * (H / CT), ntiles = tiles_img * N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int xr = lane & 15, kq = (lane >> 4) * 4;
  f4 acc[PER];
#pragma unroll
  for (int j = 0; j < PER; j++) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int img = tile / tiles_img, tt = tile % tiles_img;
    const int tx0 = (tt % tiles_x) * CT, ty0 = (tt / tiles_x) * CT;
    const int64_t ibase = (int64_t)img * H * W;
    __syncthreads();
    for (int e = threadIdx.x; e < PW * PW * (CI / 4); e += NTC) {
      const int q = e % (CI / 4), pix = e / (CI / 4);
      const int py = pix / PW, px = pix % PW;
      const int gyy = ty0 + py - 1, gxx = tx0 + px - 1;
      uint2 v = make_uint2(0u, 0u);
      if (gyy >= 0 && gyy < H && gxx >= 0 && gxx < W)
        v = *reinterpret_cast<const uint2*>(X + (ibase + (int64_t)gyy * W + gxx) * CI + 4 * q);
      *reinterpret_cast<uint2*>(patch + pix * RX + 4 * q) = v;
    }
    for (int e = threadIdx.x; e < CT * CT * (CO / 4); e += NTC) {
      const int q = e % (CO / 4), p = e / (CO / 4);
      const int py = p / CT, px = p % CT;
      const uint2 v = *reinterpret_cast<const uint2*>(
          dY + (ibase + (int64_t)(ty0 + py) * W + tx0 + px) * CO + 4 * q);
      *reinterpret_cast<uint2*>(gy_t + p * RY + 4 * q) = v;
    }
    __syncthreads();
    if (threadIdx.x < CO)
      for (int p = 0; p < CT * CT; p++) bsum += bf2f(gy_t[p * RY + threadIdx.x]);
#pragma unroll 1
    for (int kc = 0; kc < CT; kc++) {  // 16 pixels (one tile row) per K step
      s4 a[MB];
#pragma unroll
      for (int mb = 0; mb < MB; mb++) {
        const int co = mb * 16 + xr;
        s4 v;
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = (short)gy_t[(kc * CT + kq + j) * RY + co];
        a[mb] = v;
      }
#pragma unroll
      for (int j2 = 0; j2 < PER; j2++) {
        const int ob = wv + 4 * j2;
        if (ob < NOB) {
          const int mb = ob / NBK, nb = ob % NBK;
          const int n = nb * 16 + xr, t = n / CI, ci = n % CI;
          const int ky = t / 3, kx = t % 3;
          s4 b;
#pragma unroll
          for (int j = 0; j < 4; j++)
            b[j] = (short)patch[((kc + ky) * PW + kq + j + kx) * RX + ci];
          acc[j2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mb], b, acc[j2], 0, 0, 0);
        }
      }
    }
  }
  const int64_t pb = (int64_t)blockIdx.x * CO * 9 * CI;
#pragma unroll
  for (int j2 = 0; j2 < PER; j2++) {
    const int ob = wv + 4 * j2;
    if (ob < NOB) {
      const int mb = ob / NBK, nb = ob % NBK;
      const int n = nb * 16 + xr;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int co = mb * 16 + kq + i;
        part[pb + (int64_t)co * 9 * CI + n] = acc[j2][i];
      }
    }
  }
  if (threadIdx.x < CO) part_b[(int64_t)blockIdx.x * CO + threadIdx.x] = bsum;
}

// grad[layer] = sum over blocks of the partials, in a fixed order: 64
// gradient entries per block, each of its 8 wavefronts sums a contiguous
// eighth of the partials, wavefront 0 adds the eight sums in order (one
// thread per entry walking every partial left most CUs idle)
constexpr int RW_WAVES = 8;
__global__ void __launch_bounds__(64 * RW_WAVES) k_reduce_w(const float* __restrict__ part,
                                                            const float* __restrict__ part_b,
                                                            int nblk, int cin, int co_real,
                                                            int co_pad, float* __restrict__ gw,
                                                            float* __restrict__ gb) {
  __shared__ float red[RW_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = co_real * 9 * cin, e = blockIdx.x * 64 + lane;
  const int per = (nblk + RW_WAVES - 1) / RW_WAVES;
  const int b0 = min(nblk, wv * per), b1 = min(nblk, b0 + per);
  float s = 0.0f;
  if (e < nw) {
    for (int b = b0; b < b1; b++) s += part[(int64_t)b * co_pad * 9 * cin + e];
  } else if (e < nw + co_real) {
    for (int b = b0; b < b1; b++) s += part_b[(int64_t)b * co_pad + (e - nw)];
  }
  red[wv][lane] = s;
  __syncthreads();
  if (wv != 0 || e >= nw + co_real) return;
  float t = red[0][lane];
  for (int k = 1; k < RW_WAVES; k++) t += red[k][lane];
  if (e < nw)
    gw[e] = t;
  else
    gb[e - nw] = t;
}

// FP32 output gradient of the last layer -> BF16 NHWC with 16 channels
__global__ void k_pad_dout(const float* __restrict__ d, int64_t npix, uint16_t* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npix * 16;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (e % 16 == 0) ? f2bf(d[e / 16]) : (uint16_t)0;
}

// masked mean squared error: loss = sum w (o - t)^2 / sum w, dout = 2 w (o - t) / sum w
__global__ void k_mse_part(const float* __restrict__ o, const float* __restrict__ t,
                           const float* __restrict__ w, int64_t n, double* part) {
  double se = 0.0, sw = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)o[e] - (double)t[e];
    se += (double)w[e] * d * d;
    sw += (double)w[e];
  }
  __shared__ double sh[2][NTC / 64];
  se = wave_sum(se);
  sw = wave_sum(sw);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = se;
    sh[1][threadIdx.x >> 6] = sw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < NTC / 64; k++) {
      a += sh[0][k];
      b += sh[1][k];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// the loss from the block partials: one block, a fixed order (each thread a
// strided subset, then the wavefronts' sums in order)
constexpr int MF_NT = 1024;
__global__ void __launch_bounds__(MF_NT) k_mse_final(const double* part, int nb, float* loss,
                                                     double* wsum) {
  __shared__ double sh[2][MF_NT / 64];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += MF_NT) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = a;
    sh[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  a = 0.0;
  b = 0.0;
  for (int k = 0; k < MF_NT / 64; k++) {
    a += sh[0][k];
    b += sh[1][k];
  }
  *wsum = b;
  *loss = b > 0.0 ? (float)(a / b) : 0.0f;
}

__global__ void k_mse_grad(const float* __restrict__ o, const float* __restrict__ t,
                           const float* __restrict__ w, int64_t n, const double* wsum,
                           float* __restrict__ dout) {
  const double s = *wsum;
  const float sc = s > 0.0 ? (float)(2.0 / s) : 0.0f;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dout[e] = sc * w[e] * (o[e] - t[e]);
}

// weighted binary cross-entropy of logits (the mask proposal): loss =
// sum w l / sum w, l = max(o, 0) - o t + log(1 + exp(-|o|)) (the logistic
// cross-entropy without overflow), dout = w (s(o) - t) / sum w with s the
// logistic function; the partial sums in FP64 like the MSE's
__global__ void k_bce_part(const float* __restrict__ o, const float* __restrict__ t,
                           const float* __restrict__ w, int64_t n, double* part) {
  double se = 0.0, sw = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)o[e];
    const double l = fmax(x, 0.0) - x * (double)t[e] + log1p(exp(-fabs(x)));
    se += (double)w[e] * l;
    sw += (double)w[e];
  }
  __shared__ double sh[2][NTC / 64];
  se = wave_sum(se);
  sw = wave_sum(sw);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = se;
    sh[1][threadIdx.x >> 6] = sw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < NTC / 64; k++) {
      a += sh[0][k];
      b += sh[1][k];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

__global__ void k_bce_grad(const float* __restrict__ o, const float* __restrict__ t,
                           const float* __restrict__ w, int64_t n, const double* wsum,
                           float* __restrict__ dout) {
  const double s = *wsum;
  const float sc = s > 0.0 ? (float)(1.0 / s) : 0.0f;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float sg = 1.0f / (1.0f + expf(-o[e]));
    dout[e] = sc * w[e] * (sg - t[e]);
  }
}

// Adam (Kingma & Ba 2015, Algorithm 1) on FP32 master weights
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// network input from a 2D predictor state: eta / s0, hu / s1, hv / s2,
// -d_t / s3, mask, then 11 zero channels
struct FScale {
  double s[4];
};

// over the window of w x h cells at org = (i0, j0) of the grid (org null: the
// whole grid, w = nx, h = ny); out is the window's image
__global__ void k_features(const Chan* ch, const double* __restrict__ ds, int nx, int ny,
                           double dx, double dy, FScale F, const double* t, const double* dt_,
                           const double* __restrict__ ht, const double* __restrict__ mt,
                           const double* __restrict__ nt, const uint8_t* __restrict__ mask,
                           uint16_t* __restrict__ out, const int* org, int w, int h) {
  const Chan c = ch[0];
  const Motion M = body_motion(c, t[0] + dt_[0]);
  const int i0 = org ? org[0] : 0, j0 = org ? org[1] : 0;
  const int64_t n = (int64_t)w * h;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int i = i0 + (int)(o % w), j = j0 + (int)(o / w);
    const int64_t g = (int64_t)j * nx + i;
    const double x = (i + 0.5) * dx, y = (j + 0.5) * dy;
    const Shape S = body_shape(c, x - M.X, y - c.y0);
    const double d = ds[g] - S.B;
    const double dt = bed_rate(M, S).d_t;
    uint32_t v[5];
    v[0] = f2bf((float)((ht[g] - d) / F.s[0]));
    v[1] = f2bf((float)(mt[g] / F.s[1]));
    v[2] = f2bf((float)(nt[g] / F.s[2]));
    v[3] = f2bf((float)(-dt / F.s[3]));
    v[4] = f2bf(mask[g] ? 1.0f : 0.0f);
    uint4* dst = reinterpret_cast<uint4*>(out + o * 16);
    dst[0] = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4], 0u);
    dst[1] = make_uint4(0u, 0u, 0u, 0u);
  }
}

int blocks_of(int64_t n) {
  int64_t b = (n + NTC - 1) / NTC;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
int64_t cnn_param_count() {
  int64_t n = 0;
  for (int l = 0; l < NL; l++) n += (int64_t)COUTL[l] * 9 * CINL[l] + COUTL[l];
  return n;
}

static int64_t layer_off(int l) {
  int64_t n = 0;
  for (int k = 0; k < l; k++) n += (int64_t)COUTL[k] * 9 * CINL[k] + COUTL[k];
  return n;
}

static int64_t packed_elems(int l, int mode) {
  const int N = mode == 0 ? cpad16(COUTL[l]) : CINL[l];
  const int K = mode == 0 ? CINL[l] : cpad16(COUTL[l]);
  return (int64_t)N * 9 * (K + CPAD);
}

CnnLayout cnn_layout(int n, int h, int w) {
  CnnLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += bytes ? bytes : 1;
    return o;
  };
  const int64_t npix = (int64_t)n * h * w;
  for (int l = 0; l < NL; l++) {
    L.wpk[l] = take(2 * packed_elems(l, 0));
    L.wpk_t[l] = take(2 * packed_elems(l, 1));
  }
  for (int l = 0; l < NL - 1; l++) L.act[l] = take(2 * npix * 32);
  L.out = take(4 * npix);
  L.dy_a = take(2 * npix * 32);
  L.dy_b = take(2 * npix * 32);
  L.dy16 = take(2 * npix * 16);
  const int ntiles = (int)(npix / (CT * CT));
  L.nblk_w = ntiles < 256 ? (ntiles > 0 ? ntiles : 1) : 256;
  L.part = take(4 * (size_t)L.nblk_w * 32 * 9 * 32);
  L.part_b = take(4 * (size_t)L.nblk_w * 32);
  L.mse_part = take(8 * 2 * 1024);
  L.mse_w = take(8);
  L.bytes = off + 256;
  return L;
}

void cnn_pack_weights(const float* params, char* ws, const CnnLayout& L, bool with_transposed,
                      hipStream_t s) {
  for (int l = 0; l < NL; l++) {
    const float* W = params + layer_off(l);
    hipLaunchKernelGGL(k_pack_w, dim3(blocks_of(packed_elems(l, 0))), dim3(NTC), 0, s, W, CINL[l],
                       COUTL[l], 0, reinterpret_cast<uint16_t*>(ws + L.wpk[l]));
    if (with_transposed && l > 0)
      hipLaunchKernelGGL(k_pack_w, dim3(blocks_of(packed_elems(l, 1))), dim3(NTC), 0, s, W,
                         CINL[l], COUTL[l], 1, reinterpret_cast<uint16_t*>(ws + L.wpk_t[l]));
  }
}

void cnn_forward(const float* params, const uint16_t* x, int n, int h, int w, char* ws,
                 const CnnLayout& L, float* out, hipStream_t s, const int* box) {
  const dim3 grid((w / CT) * (h / CT), n);
  const uint16_t* in = x;
  for (int l = 0; l < NL; l++) {
    const float* b = params + layer_off(l) + (int64_t)COUTL[l] * 9 * CINL[l];
    const uint16_t* wp = reinterpret_cast<const uint16_t*>(ws + L.wpk[l]);
    if (l == 0) {
      uint16_t* o = reinterpret_cast<uint16_t*>(ws + L.act[0]);
      hipLaunchKernelGGL((k_conv<16, 32, EPI_RELU>), grid, dim3(NTC), 0, s, in, wp, b, h, w, o,
                         (float*)nullptr, (const uint16_t*)nullptr, box);
      in = o;
    } else if (l < NL - 1) {
      uint16_t* o = reinterpret_cast<uint16_t*>(ws + L.act[l]);
      hipLaunchKernelGGL((k_conv<32, 32, EPI_RELU>), grid, dim3(NTC), 0, s, in, wp, b, h, w, o,
                         (float*)nullptr, (const uint16_t*)nullptr, box);
      in = o;
    } else {
      hipLaunchKernelGGL((k_conv<32, 16, EPI_LAST>), grid, dim3(NTC), 0, s, in, wp, b, h, w,
                         (uint16_t*)nullptr, out, (const uint16_t*)nullptr, box);
    }
  }
}

void cnn_backward(const float* params, const uint16_t* x, const float* dout, int n, int h, int w,
                  char* ws, const CnnLayout& L, float* grad, hipStream_t s) {
  const dim3 grid((w / CT) * (h / CT), n);
  const int64_t npix = (int64_t)n * h * w;
  uint16_t* dy16 = reinterpret_cast<uint16_t*>(ws + L.dy16);
  hipLaunchKernelGGL(k_pad_dout, dim3(blocks_of(npix * 16)), dim3(NTC), 0, s, dout, npix, dy16);
  float* part = reinterpret_cast<float*>(ws + L.part);
  float* part_b = reinterpret_cast<float*>(ws + L.part_b);
  const uint16_t* dy = dy16;
  uint16_t* bufs[2] = {reinterpret_cast<uint16_t*>(ws + L.dy_a), reinterpret_cast<uint16_t*>(ws + L.dy_b)};
  for (int l = NL - 1; l >= 0; l--) {
    const uint16_t* xin = l == 0 ? x : reinterpret_cast<const uint16_t*>(ws + L.act[l - 1]);
    float* gw = grad + layer_off(l);
    float* gb = gw + (int64_t)COUTL[l] * 9 * CINL[l];
    if (l == NL - 1)
      hipLaunchKernelGGL((k_conv_bwdw<32, 16>), dim3(L.nblk_w), dim3(NTC), 0, s, xin, dy, n, h, w,
                         part, part_b);
    else if (l > 0)
      hipLaunchKernelGGL((k_conv_bwdw<32, 32>), dim3(L.nblk_w), dim3(NTC), 0, s, xin, dy, n, h, w,
                         part, part_b);
    else
      hipLaunchKernelGGL((k_conv_bwdw<16, 32>), dim3(L.nblk_w), dim3(NTC), 0, s, xin, dy, n, h, w,
                         part, part_b);
    const int nw = COUTL[l] * 9 * CINL[l] + COUTL[l];
    hipLaunchKernelGGL(k_reduce_w, dim3((nw + 63) / 64), dim3(64 * RW_WAVES), 0, s, part, part_b,
                       L.nblk_w, CINL[l], COUTL[l], cpad16(COUTL[l]), gw, gb);
    if (l > 0) {
      uint16_t* dx = bufs[l & 1];
      const uint16_t* wt = reinterpret_cast<const uint16_t*>(ws + L.wpk_t[l]);
      const uint16_t* gate = reinterpret_cast<const uint16_t*>(ws + L.act[l - 1]);
      if (l == NL - 1)
        hipLaunchKernelGGL((k_conv<16, 32, EPI_GATE>), grid, dim3(NTC), 0, s, dy, wt,
                           (const float*)nullptr, h, w, dx, (float*)nullptr, gate,
                           (const int*)nullptr);
      else
        hipLaunchKernelGGL((k_conv<32, 32, EPI_GATE>), grid, dim3(NTC), 0, s, dy, wt,
                           (const float*)nullptr, h, w, dx, (float*)nullptr, gate,
                           (const int*)nullptr);
      dy = dx;
    }
  }
}

void cnn_mse(const float* o, const float* t, const float* wgt, int64_t n, char* ws,
             const CnnLayout& L, float* dout, float* loss, hipStream_t s) {
  double* part = reinterpret_cast<double*>(ws + L.mse_part);
  double* wsum = reinterpret_cast<double*>(ws + L.mse_w);
  const int nb = blocks_of(n) < 1024 ? blocks_of(n) : 1024;
  hipLaunchKernelGGL(k_mse_part, dim3(nb), dim3(NTC), 0, s, o, t, wgt, n, part);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(MF_NT), 0, s, (const double*)part, nb, loss, wsum);
  hipLaunchKernelGGL(k_mse_grad, dim3(blocks_of(n)), dim3(NTC), 0, s, o, t, wgt, n,
                     (const double*)wsum, dout);
}

void cnn_bce(const float* o, const float* t, const float* wgt, int64_t n, char* ws,
             const CnnLayout& L, float* dout, float* loss, hipStream_t s) {
  double* part = reinterpret_cast<double*>(ws + L.mse_part);
  double* wsum = reinterpret_cast<double*>(ws + L.mse_w);
  const int nb = blocks_of(n) < 1024 ? blocks_of(n) : 1024;
  hipLaunchKernelGGL(k_bce_part, dim3(nb), dim3(NTC), 0, s, o, t, wgt, n, part);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(MF_NT), 0, s, (const double*)part, nb, loss, wsum);
  hipLaunchKernelGGL(k_bce_grad, dim3(blocks_of(n)), dim3(NTC), 0, s, o, t, wgt, n,
                     (const double*)wsum, dout);
}

void cnn_adam(float* p, float* m, float* v, const float* g, int64_t n, int step, float lr,
              float b1, float b2, float eps, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_of(n)), dim3(NTC), 0, s, p, m, v, g, n, lr, b1, b2, eps,
                     c1, c2);
}

void cnn_features(const Chan* ch, const double* ds, int nx, int ny, double dx, double dy,
                  const double* scale, const double* t, const double* dt, const double* ht,
                  const double* mt, const double* nt, const uint8_t* mask, uint16_t* out,
                  hipStream_t s, const int* org, int w, int h) {
  FScale F;
  for (int k = 0; k < 4; k++) F.s[k] = scale[k];
  if (!org) {
    w = nx;
    h = ny;
  }
  hipLaunchKernelGGL(k_features, dim3(blocks_of((int64_t)w * h)), dim3(NTC), 0, s, ch, ds, nx,
                     ny, dx, dy, F, t, dt, ht, mt, nt, mask, out, org, w, h);
}


// Inference-only layout: the packed forward weights and two activation
// buffers that the layers use in turn (layer l reads one, writes the other).
CnnLayout cnn_layout_infer(int n, int h, int w) {
  CnnLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += bytes ? bytes : 1;
    return o;
  };
  const int64_t npix = (int64_t)n * h * w;
  for (int l = 0; l < NL; l++) L.wpk[l] = take(2 * packed_elems(l, 0));
  const size_t a = take(2 * npix * 32), b = take(2 * npix * 32);
  for (int l = 0; l < NL - 1; l++) L.act[l] = (l & 1) ? b : a;
  L.bytes = off;
  return L;
}

// Scratch of the allocation-free inference entry point.  Each device holds
// its own copy from module load until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for that device.
static __device__ __align__(256) unsigned char scratch[SWE_NH_CNN_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];  // per device ordinal, set on the first call on that device

// device address of `scratch` on device dev (which must be current), or null
static void* scratch_on(int dev) {
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace swenh

// ---------------------------------------------------------------------------
// C ABI of the network (training and inference on caller-owned buffers)
// ---------------------------------------------------------------------------
using namespace swenh;

extern "C" {

size_t swe_nh_cnn_param_count(void) { return (size_t)cnn_param_count(); }

size_t swe_nh_cnn_workspace_bytes(int32_t n, int32_t h, int32_t w) {
  if (n < 1 || h < 16 || w < 16 || h % 16 || w % 16) return 0;
  return cnn_layout(n, h, w).bytes;
}

static int cnn_args_ok(int32_t n, int32_t h, int32_t w, size_t bytes) {
  const size_t need = swe_nh_cnn_workspace_bytes(n, h, w);
  if (!need) return SWE_NH_EINVAL;
  if (bytes < need) return SWE_NH_ENOMEM;
  return SWE_NH_OK;
}

int swe_nh_cnn_forward(const float* params, const uint16_t* x, int32_t n, int32_t h, int32_t w,
                       float* out, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !x || !out || !ws) return SWE_NH_EINVAL;
  const int rc = cnn_args_ok(n, h, w, ws_bytes);
  if (rc) return rc;
  const CnnLayout L = cnn_layout(n, h, w);
  hipStream_t s = (hipStream_t)stream;
  cnn_pack_weights(params, (char*)ws, L, true, s);
  cnn_forward(params, x, n, h, w, (char*)ws, L, out, s);
  return hipGetLastError() == hipSuccess ? SWE_NH_OK : SWE_NH_EHIP;
}

int swe_nh_cnn_forward_noalloc(const float* params, const uint16_t* x, int32_t n, int32_t h,
                               int32_t w, float* out, void* stream) {
  if (!params || !x || !out) return SWE_NH_EINVAL;
  if (n < 1 || h < 16 || w < 16 || h % 16 || w % 16) return SWE_NH_EINVAL;
  if ((int64_t)n * h * w > SWE_NH_CNN_NOALLOC_MAX_PIXELS) return SWE_NH_ENOMEM;
  const CnnLayout L = cnn_layout_infer(n, h, w);
  if (L.bytes > SWE_NH_CNN_NOALLOC_SCRATCH_BYTES) return SWE_NH_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SWE_NH_EHIP;
  if (s) {  // the scratch address is per device: the stream must be the current device's
    int sdev = -1;
    if (hipStreamGetDevice(s, &sdev) != hipSuccess) return SWE_NH_EHIP;
    if (sdev != dev) return SWE_NH_EINVAL;
  }
  char* ws = static_cast<char*>(scratch_on(dev));
  if (!ws) return SWE_NH_EHIP;
  cnn_pack_weights(params, ws, L, false, s);
  cnn_forward(params, x, n, h, w, ws, L, out, s);
  return hipGetLastError() == hipSuccess ? SWE_NH_OK : SWE_NH_EHIP;
}

int swe_nh_cnn_backward(const float* params, const uint16_t* x, const float* dout, int32_t n,
                        int32_t h, int32_t w, float* grad, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!params || !x || !dout || !grad || !ws) return SWE_NH_EINVAL;
  const int rc = cnn_args_ok(n, h, w, ws_bytes);
  if (rc) return rc;
  const CnnLayout L = cnn_layout(n, h, w);
  cnn_backward(params, x, dout, n, h, w, (char*)ws, L, grad, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SWE_NH_OK : SWE_NH_EHIP;
}

int swe_nh_cnn_mse(const float* out, const float* target, const float* weight, int32_t n,
                   int32_t h, int32_t w, float* dout, float* loss, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!out || !target || !weight || !dout || !loss || !ws) return SWE_NH_EINVAL;
  const int rc = cnn_args_ok(n, h, w, ws_bytes);
  if (rc) return rc;
  const CnnLayout L = cnn_layout(n, h, w);
  cnn_mse(out, target, weight, (int64_t)n * h * w, (char*)ws, L, dout, loss, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SWE_NH_OK : SWE_NH_EHIP;
}

int swe_nh_cnn_bce(const float* out, const float* target, const float* weight, int32_t n,
                   int32_t h, int32_t w, float* dout, float* loss, void* ws, size_t ws_bytes,
                   void* stream) {
  if (!out || !target || !weight || !dout || !loss || !ws) return SWE_NH_EINVAL;
  const int rc = cnn_args_ok(n, h, w, ws_bytes);
  if (rc) return rc;
  const CnnLayout L = cnn_layout(n, h, w);
  cnn_bce(out, target, weight, (int64_t)n * h * w, (char*)ws, L, dout, loss, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SWE_NH_OK : SWE_NH_EHIP;
}

int swe_nh_cnn_adam(float* params, float* m, float* v, const float* grad, int64_t count,
                    int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!params || !m || !v || !grad || count < 1 || step < 1) return SWE_NH_EINVAL;
  cnn_adam(params, m, v, grad, count, step, lr, beta1, beta2, eps, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SWE_NH_OK : SWE_NH_EHIP;
}

}  // extern "C"
