// swe_nh_common.h -- device-side types and helpers shared by the HIP kernels
// of the non-hydrostatic SWE hot path (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swe_nh.h"

namespace swenh {

constexpr double kPi = 3.14159265358979323846;

// status bits accumulated on the device during a step
enum : int32_t { ST_DRY = 1, ST_NAN = 2, ST_NOCONV = 4, ST_ABORT = 8 };

// one independent 1D channel (or the single 2D domain)
struct Chan {
  int64_t off;      // first packed cell
  int32_t n;        // cells
  int32_t kind;     // body shape
  int32_t law;      // body travel law
  int32_t pad;
  double amp, len, x0, y0, dir;
  double q[5];
};

// position, velocity and acceleration of the body centre along x
struct Motion {
  double X, V, A;
};

__device__ __forceinline__ Motion body_motion(const Chan& c, double t) {
  double s = 0.0, v = 0.0, a = 0.0;
  switch (c.law) {
    case SWE_NH_LAW_CONST_VEL:
      s = c.q[0] * t;
      v = c.q[0];
      break;
    case SWE_NH_LAW_SIN_RAMP: {
      // ramp of length q1 over the distance q0, half a cosine period
      const double L = c.q[0], T = c.q[1];
      if (t <= T) {
        const double w = kPi / T;
        double sn, cs;
        sincos(w * t, &sn, &cs);
        s = 0.5 * L * (1.0 - cs);
        v = 0.5 * L * w * sn;
        a = 0.5 * L * w * w * cs;
      } else {
        s = L;
      }
    } break;
    case SWE_NH_LAW_PIECEWISE: {
      // Eq. 21: accelerate (a0) to t1, coast at u_t to t2, decelerate to t3
      const double a0 = c.q[0], ut = c.q[1], t1 = c.q[2], t2 = c.q[3], t3 = c.q[4];
      const double s1 = 0.5 * a0 * t1 * t1;
      if (t <= t1) {
        s = 0.5 * a0 * t * t;
        v = a0 * t;
        a = a0;
      } else if (t <= t2) {
        s = s1 + ut * (t - t1);
        v = ut;
      } else if (t <= t3) {
        const double r = t - t2;
        s = s1 + ut * (t - t1) - 0.5 * a0 * r * r;
        v = ut - a0 * r;
        a = -a0;
      } else {
        const double r = t3 - t2;
        s = s1 + ut * (t3 - t1) - 0.5 * a0 * r * r;
      }
    } break;
    default:
      break;
  }
  Motion m;
  m.X = c.x0 + c.dir * s;
  m.V = c.dir * v;
  m.A = c.dir * a;
  return m;
}

// body thickness B at (xi, zeta) relative to its centre, with dB/dxi,
// d2B/dxi2 and d2B/dxi dzeta
struct Shape {
  double B, Bx, Bxx, Bxy;
};

__device__ __forceinline__ Shape body_shape(const Chan& c, double xi, double zeta) {
  Shape s{0.0, 0.0, 0.0, 0.0};
  if (c.kind == SWE_NH_BODY_QUARTIC) {
    // Eq. 20 with z = 2 xi / L: B = H (1 - z^4) on |z| < 1
    const double r = 2.0 / c.len;
    const double z = xi * r;
    if (fabs(xi) < 0.5 * c.len) {
      const double z2 = z * z;
      s.B = c.amp * (1.0 - z2 * z2);
      s.Bx = -4.0 * c.amp * r * z2 * z;
      s.Bxx = -12.0 * c.amp * r * r * z2;
    }
  } else if (c.kind == SWE_NH_BODY_GAUSS) {
    const double iw2 = 1.0 / (c.len * c.len);
    const double e = c.amp * exp(-(xi * xi + zeta * zeta) * iw2);
    s.B = e;
    s.Bx = -2.0 * xi * iw2 * e;
    s.Bxx = (4.0 * xi * xi * iw2 * iw2 - 2.0 * iw2) * e;
    s.Bxy = 4.0 * xi * zeta * iw2 * iw2 * e;
  }
  return s;
}

// B alone (the depth needs nothing else), with the arithmetic of body_shape.
// Far from the Gaussian mound the exponential is not evaluated: beyond
// (xi^2 + zeta^2) / len^2 > 80 it is below amp e^-80 ~ 2e-35 amp, which no
// depth of a wet cell registers.
__device__ __forceinline__ double body_B(const Chan& c, double xi, double zeta) {
  if (c.kind == SWE_NH_BODY_QUARTIC) {
    if (!(fabs(xi) < 0.5 * c.len)) return 0.0;
    const double z = xi * (2.0 / c.len), z2 = z * z;
    return c.amp * (1.0 - z2 * z2);
  }
  if (c.kind == SWE_NH_BODY_GAUSS) {
    const double q = (xi * xi + zeta * zeta) * (1.0 / (c.len * c.len));
    return q > 80.0 ? 0.0 : c.amp * exp(-q);
  }
  return 0.0;
}

// time derivatives of the moving bottom d = d_s - B(x - X(t), y - y0)
struct BedRate {
  double d_t, d_tt, d_xt, d_yt;
};

__device__ __forceinline__ BedRate bed_rate(const Motion& m, const Shape& s) {
  BedRate r;
  r.d_t = m.V * s.Bx;
  r.d_tt = m.A * s.Bx - m.V * m.V * s.Bxx;
  r.d_xt = m.V * s.Bxx;
  r.d_yt = m.V * s.Bxy;
  return r;
}

// 1 / x for finite nonzero x whose reciprocal is a normal number: the
// hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r), each of which squares the relative error.  Within an
// ulp or so of the correctly rounded quotient; used where the state is divided
// by a depth in the stencil sweeps.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(x) for x = 0 or x >= 2^-960 (a wave speed squared, g times a depth):
// the hardware estimate y of 1/sqrt(x), one coupled Newton step on s = x y
// ~ sqrt(x) and t = y / 2 ~ 1 / (2 sqrt(x)) (with e = 1/2 - s t both become
// s (1 + e) and t (1 + e), squaring the relative error), then one correction
// s + t (x - s^2).  No scaling of tiny or huge arguments and no special cases
// beyond 0, which is what the library square root spends most of its
// instructions on; within an ulp of the correctly rounded root.
__device__ __forceinline__ double sqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, t = 0.5 * y;
  const double e = fma(-s, t, 0.5);
  s = fma(s, e, s);
  t = fma(t, e, t);
  s = fma(fma(-s, s, x), t, s);
  return x > 0.0 ? s : 0.0;
}

// minmod(a, b): the argument of smaller magnitude when both have one sign,
// else zero, as max(min(a, b), 0) + min(max(a, b), 0) (one of the two terms
// is always zero, so the sum is exact): five instructions, no compare and
// select chains
__device__ __forceinline__ double minmod(double a, double b) {
  return fmax(fmin(a, b), 0.0) + fmin(fmax(a, b), 0.0);
}

// reflect a channel-local cell index into [0, n)
__device__ __forceinline__ int reflect(int i, int n) {
  return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}

// order-preserving bit pattern of a non-negative double (for atomicMax)
__device__ __forceinline__ unsigned long long pos_bits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

// wave64 reductions
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Tagged words: a value published with a tag in the upper half of a 64-bit
// word (agent-scope relaxed atomic stores; an FP64 value takes two words,
// each with the tag).  A reader polls with agent-scope relaxed atomic loads
// until each word carries the tag it expects: single-copy atomicity makes a
// word's value and tag consistent, so no ordering between words (no fence)
// is needed.
__device__ __forceinline__ void put_tagged(unsigned long long* w, float v, unsigned tag) {
  __hip_atomic_store(w, ((unsigned long long)tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_tagged(unsigned long long* w, unsigned v, unsigned tag) {
  __hip_atomic_store(w, ((unsigned long long)tag << 32) | v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_tagged(unsigned long long* w, double v, unsigned tag) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  __hip_atomic_store(w, ((unsigned long long)tag << 32) | (b & 0xffffffffull), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, ((unsigned long long)tag << 32) | (b >> 32), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_word(const unsigned long long* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// one poll: true (and the value) when the words carry the tag
__device__ __forceinline__ bool try_tagged(const unsigned long long* w, unsigned tag, float& v) {
  const unsigned long long a = load_word(w);
  if ((unsigned)(a >> 32) != tag) return false;
  v = __uint_as_float((unsigned)a);
  return true;
}
__device__ __forceinline__ bool try_tagged(const unsigned long long* w, unsigned tag, unsigned& v) {
  const unsigned long long a = load_word(w);
  if ((unsigned)(a >> 32) != tag) return false;
  v = (unsigned)a;
  return true;
}
__device__ __forceinline__ bool try_tagged(const unsigned long long* w, unsigned tag, double& v) {
  const unsigned long long a = load_word(w), b = load_word(w + 1);
  if ((unsigned)(a >> 32) != tag || (unsigned)(b >> 32) != tag) return false;
  v = __longlong_as_double((long long)((b << 32) | (a & 0xffffffffull)));
  return true;
}
// bounded polls: a wait longer than POLL_TICKS (wall_clock64 ticks at 100 MHz)
// or another wait's abort (ST_ABORT in *status) ends it with false
constexpr unsigned long long POLL_TICKS = 50000000ull;
template <typename V>
__device__ bool poll_tagged(const unsigned long long* w, unsigned tag, V& v, int* status) {
  const unsigned long long t0 = wall_clock64();
  unsigned polls = 0;
  while (!try_tagged(w, tag, v)) {
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
  return true;
}

}  // namespace swenh
