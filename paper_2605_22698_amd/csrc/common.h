// Shared device helpers of the e3mi HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace e3mi {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// Per-edge radial weights R and their adjoint dR are stored as FP32, or as
// BF16 (rounded to nearest even) in the BF16 mode; arithmetic is FP32.
__device__ __forceinline__ float ldr(const float* p) { return *p; }
__device__ __forceinline__ float ldr(const __bf16* p) { return (float)*p; }
__device__ __forceinline__ void str(float* p, float v) { *p = v; }
__device__ __forceinline__ void str(__bf16* p, float v) { *p = (__bf16)v; }
// n consecutive stored values (n = 1, 2, 4 or 8) as floats, one vector load
template <int n>
__device__ __forceinline__ void ldr_n(const float* p, float* v) {
  if constexpr (n == 1) {
    v[0] = p[0];
  } else if constexpr (n == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    v[0] = t.x;
    v[1] = t.y;
  } else {
#pragma unroll
    for (int q = 0; q < n; q += 4) {
      const float4 t = *reinterpret_cast<const float4*>(p + q);
      v[q] = t.x;
      v[q + 1] = t.y;
      v[q + 2] = t.z;
      v[q + 3] = t.w;
    }
  }
}
template <int n>
__device__ __forceinline__ void ldr_n(const __bf16* p, float* v) {
  typedef __bf16 bvec __attribute__((ext_vector_type(n)));
  const bvec t = *reinterpret_cast<const bvec*>(p);
#pragma unroll
  for (int q = 0; q < n; ++q) v[q] = (float)t[q];
}
template <int n>
__device__ __forceinline__ void str_n(float* p, const float* v) {
  if constexpr (n == 1) {
    p[0] = v[0];
  } else if constexpr (n == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  } else {
#pragma unroll
    for (int q = 0; q < n; q += 4) *reinterpret_cast<float4*>(p + q) = make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]);
  }
}
template <int n>
__device__ __forceinline__ void str_n(__bf16* p, const float* v) {
  typedef __bf16 bvec __attribute__((ext_vector_type(n)));
  bvec t;
#pragma unroll
  for (int q = 0; q < n; ++q) t[q] = (__bf16)v[q];
  *reinterpret_cast<bvec*>(p) = t;
}

// logistic function with the hardware reciprocal (v_rcp_f32, 1 ulp) in place
// of a correctly rounded division: 1 + exp(-x) >= 1, so no denormal input
__device__ __forceinline__ float sigmoidf(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ __forceinline__ float siluf(float x) { return x * sigmoidf(x); }
// d silu / dx = s + x s (1 - s)
__device__ __forceinline__ float silu_grad(float x) {
  const float s = sigmoidf(x);
  return s * (1.0f + x * (1.0f - s));
}

// Workgroups are handed to the 8 XCDs (each with its own L2) in round-robin
// order of the block index. For receiver-centric kernels, map block b so that
// XCD b % 8 walks a contiguous range of receivers: neighbouring receivers
// share senders, so their gathers hit the same L2. A bijection on [0, n).
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sums of NV <= 16 per-lane values over the 64 lanes of a wave, by recursive
// halving: each exchange over lane bits 5, 4, 3, 2 hands the partner the half
// of the values this lane does not keep, so lane L ends with a partial of
// value q = L >> 2, which the exchanges over bits 1 and 0 complete (17 lane
// exchanges where 16 butterfly reductions take 96). Returns the total of
// value lane >> 2 (zero for q >= NV).
template <int NV>
__device__ __forceinline__ float wave_sum_scatter16(const float* v) {
  static_assert(NV <= 16, "at most 16 values");
  const int lane = threadIdx.x & 63;
  float a[8], b[4], c[2];
  bool hi = lane & 32;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float lo_v = q < NV ? v[q] : 0.0f, hi_v = q + 8 < NV ? v[q + 8] : 0.0f;
    a[q] = (hi ? hi_v : lo_v) + __shfl_xor(hi ? lo_v : hi_v, 32);
  }
  hi = lane & 16;
#pragma unroll
  for (int q = 0; q < 4; ++q) b[q] = (hi ? a[q + 4] : a[q]) + __shfl_xor(hi ? a[q] : a[q + 4], 16);
  hi = lane & 8;
#pragma unroll
  for (int q = 0; q < 2; ++q) c[q] = (hi ? b[q + 2] : b[q]) + __shfl_xor(hi ? b[q] : b[q + 2], 8);
  hi = lane & 4;
  float d = (hi ? c[1] : c[0]) + __shfl_xor(hi ? c[0] : c[1], 4);
  d += __shfl_xor(d, 2);
  d += __shfl_xor(d, 1);
  return d;
}

// Real spherical harmonics of a unit vector, component normalised
// (sum_m Y_lm^2 = 2l + 1), index l*l + m + l. Only orders <= LMAX are written.
template <int LMAX>
__device__ __forceinline__ void real_sh(float x, float y, float z, float* Y) {
  Y[0] = 1.0f;
  if constexpr (LMAX >= 1) {
    constexpr float s3 = 1.7320508075688772f;
    Y[1] = s3 * y;
    Y[2] = s3 * z;
    Y[3] = s3 * x;
  }
  if constexpr (LMAX >= 2) {
    constexpr float s15 = 3.872983346207417f, s5h = 1.118033988749895f;
    Y[4] = s15 * x * y;
    Y[5] = s15 * y * z;
    Y[6] = s5h * (3.0f * z * z - 1.0f);
    Y[7] = s15 * x * z;
    Y[8] = 0.5f * s15 * (x * x - y * y);
  }
  if constexpr (LMAX >= 3) {
    constexpr float a358 = 2.091650066335189f, s105 = 10.246950765959598f;
    constexpr float a218 = 1.620185174601965f, s7h = 1.3228756555322954f;
    Y[9] = a358 * y * (3.0f * x * x - y * y);
    Y[10] = s105 * x * y * z;
    Y[11] = a218 * y * (5.0f * z * z - 1.0f);
    Y[12] = s7h * z * (5.0f * z * z - 3.0f);
    Y[13] = a218 * x * (5.0f * z * z - 1.0f);
    Y[14] = 0.5f * s105 * z * (x * x - y * y);
    Y[15] = a358 * x * (x * x - 3.0f * y * y);
  }
}

// G = sum_c dY[c] * grad P_c(x, y, z), where P_c is the polynomial above
// (the caller projects out the radial part).
template <int LMAX>
__device__ __forceinline__ void real_sh_vjp(float x, float y, float z, const float* dY, float& gx,
                                            float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if constexpr (LMAX >= 1) {
    constexpr float s3 = 1.7320508075688772f;
    gy += s3 * dY[1];
    gz += s3 * dY[2];
    gx += s3 * dY[3];
  }
  if constexpr (LMAX >= 2) {
    constexpr float s15 = 3.872983346207417f, s5h = 1.118033988749895f;
    gx += s15 * (y * dY[4] + z * dY[7] + x * dY[8]);
    gy += s15 * (x * dY[4] + z * dY[5] - y * dY[8]);
    gz += s15 * (y * dY[5] + x * dY[7]) + 6.0f * s5h * z * dY[6];
  }
  if constexpr (LMAX >= 3) {
    constexpr float a358 = 2.091650066335189f, s105 = 10.246950765959598f;
    constexpr float a218 = 1.620185174601965f, s7h = 1.3228756555322954f;
    gx += a358 * (6.0f * x * y * dY[9] + 3.0f * (x * x - y * y) * dY[15]) + s105 * (y * z * dY[10] + x * z * dY[14]) +
          a218 * (5.0f * z * z - 1.0f) * dY[13];
    gy += a358 * (3.0f * (x * x - y * y) * dY[9] - 6.0f * x * y * dY[15]) + s105 * (x * z * dY[10] - y * z * dY[14]) +
          a218 * (5.0f * z * z - 1.0f) * dY[11];
    gz += s105 * x * y * dY[10] + 10.0f * a218 * z * (y * dY[11] + x * dY[13]) +
          s7h * (15.0f * z * z - 3.0f) * dY[12] + 0.5f * s105 * (x * x - y * y) * dY[14];
  }
}


// Directional derivative of real_sh_vjp along u: H u with H = sum_c dY[c]
// times the Hessian of the polynomial P_c at (x, y, z).
template <int LMAX>
__device__ __forceinline__ void real_sh_vjp_jvp(float x, float y, float z, float ux, float uy, float uz,
                                                const float* dY, float& hx, float& hy, float& hz) {
  hx = hy = hz = 0.0f;
  if constexpr (LMAX >= 2) {
    constexpr float s15 = 3.872983346207417f, s5h = 1.118033988749895f;
    hx += s15 * (uy * dY[4] + uz * dY[7] + ux * dY[8]);
    hy += s15 * (ux * dY[4] + uz * dY[5] - uy * dY[8]);
    hz += s15 * (uy * dY[5] + ux * dY[7]) + 6.0f * s5h * uz * dY[6];
  }
  if constexpr (LMAX >= 3) {
    constexpr float a358 = 2.091650066335189f, s105 = 10.246950765959598f;
    constexpr float a218 = 1.620185174601965f, s7h = 1.3228756555322954f;
    const float xy_d = ux * y + x * uy, xx_yy_d = 2.0f * (x * ux - y * uy);
    hx += a358 * (6.0f * xy_d * dY[9] + 3.0f * xx_yy_d * dY[15]) +
          s105 * ((uy * z + y * uz) * dY[10] + (ux * z + x * uz) * dY[14]) + a218 * 10.0f * z * uz * dY[13];
    hy += a358 * (3.0f * xx_yy_d * dY[9] - 6.0f * xy_d * dY[15]) +
          s105 * ((ux * z + x * uz) * dY[10] - (uy * z + y * uz) * dY[14]) + a218 * 10.0f * z * uz * dY[11];
    hz += s105 * xy_d * dY[10] + 10.0f * a218 * (uz * (y * dY[11] + x * dY[13]) + z * (uy * dY[11] + ux * dY[13])) +
          s7h * 30.0f * z * uz * dY[12] + 0.5f * s105 * xx_yy_d * dY[14];
  }
}

// Directional derivative of every harmonic polynomial along u:
// Yd[c] = grad P_c(x, y, z) . u (the caller passes the tangential part of the
// direction change, u = (I - n n^T) d_dot / r).
template <int LMAX>
__device__ __forceinline__ void real_sh_jvp(float x, float y, float z, float ux, float uy, float uz, float* Yd) {
  Yd[0] = 0.0f;
  if constexpr (LMAX >= 1) {
    constexpr float s3 = 1.7320508075688772f;
    Yd[1] = s3 * uy;
    Yd[2] = s3 * uz;
    Yd[3] = s3 * ux;
  }
  if constexpr (LMAX >= 2) {
    constexpr float s15 = 3.872983346207417f, s5h = 1.118033988749895f;
    Yd[4] = s15 * (y * ux + x * uy);
    Yd[5] = s15 * (z * uy + y * uz);
    Yd[6] = 6.0f * s5h * z * uz;
    Yd[7] = s15 * (z * ux + x * uz);
    Yd[8] = s15 * (x * ux - y * uy);
  }
  if constexpr (LMAX >= 3) {
    constexpr float a358 = 2.091650066335189f, s105 = 10.246950765959598f;
    constexpr float a218 = 1.620185174601965f, s7h = 1.3228756555322954f;
    Yd[9] = a358 * (6.0f * x * y * ux + 3.0f * (x * x - y * y) * uy);
    Yd[10] = s105 * (y * z * ux + x * z * uy + x * y * uz);
    Yd[11] = a218 * ((5.0f * z * z - 1.0f) * uy + 10.0f * y * z * uz);
    Yd[12] = s7h * (15.0f * z * z - 3.0f) * uz;
    Yd[13] = a218 * ((5.0f * z * z - 1.0f) * ux + 10.0f * x * z * uz);
    Yd[14] = s105 * (x * z * ux - y * z * uy) + 0.5f * s105 * (x * x - y * y) * uz;
    Yd[15] = a358 * (3.0f * (x * x - y * y) * ux - 6.0f * x * y * uy);
  }
}

// Harmonics and their directional derivatives for an edge vector d (length
// r) moving with velocity dd: n = d / r, u = (I - n n^T) dd / r.
template <int LMAX>
__device__ __forceinline__ void real_sh_dual(float4 d, float4 dd, float* Y, float* Yd) {
  const float ir = 1.0f / d.w;
  const float x = d.x * ir, y = d.y * ir, z = d.z * ir;
  real_sh<LMAX>(x, y, z, Y);
  const float dot = x * dd.x + y * dd.y + z * dd.z;
  real_sh_jvp<LMAX>(x, y, z, (dd.x - dot * x) * ir, (dd.y - dot * y) * ir, (dd.z - dot * z) * ir, Yd);
}

// silu'' = s (1 - s) (2 + x (1 - 2 s))
__device__ __forceinline__ float silu_grad2(float x) {
  const float s = sigmoidf(x);
  return s * (1.0f - s) * (2.0f + x * (1.0f - 2.0f * s));
}

// Bessel x polynomial-envelope radial basis B_n(r), n = 1..NB, and optionally
// its derivative dB_n/dr. Zero for r >= rc.
template <int NB>
__device__ __forceinline__ void radial_basis(float r, float rc, int p, float* B, float* dB) {
  const float x = r / rc;
  if (!(x < 1.0f)) {
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      B[n] = 0.0f;
      if (dB) dB[n] = 0.0f;
    }
    return;
  }
  // u(x) = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2)
  // u'(x) = -p(p+1)(p+2)/2 x^(p-1) (1-x)^2
  float xp1 = 1.0f;  // x^(p-1)
  for (int k = 0; k < p - 1; ++k) xp1 *= x;
  const float xp = xp1 * x;
  const float fp = (float)p;
  const float u = 1.0f - 0.5f * (fp + 1.0f) * (fp + 2.0f) * xp + fp * (fp + 2.0f) * xp * x -
                  0.5f * fp * (fp + 1.0f) * xp * x * x;
  const float du_dr = -0.5f * fp * (fp + 1.0f) * (fp + 2.0f) * xp1 * (1.0f - x) * (1.0f - x) / rc;
  const float pref = sqrtf(2.0f / rc);
  const float inv_r = 1.0f / r;
  const float w = 3.14159265358979f / rc;
  // sin and cos of (n + 1) w r by angle addition from those of w r (one
  // sincosf per edge instead of one per basis function)
  float s1, c1;
  sincosf(w * r, &s1, &c1);
  float s = s1, c = c1;
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    if (n > 0) {
      const float sn = s * c1 + c * s1;
      c = c * c1 - s * s1;
      s = sn;
    }
    const float b = pref * s * inv_r;
    B[n] = b * u;
    if (dB) {
      const float db = pref * ((n + 1) * w * c * inv_r - s * inv_r * inv_r);
      dB[n] = db * u + b * du_dr;
    }
  }
}

}  // namespace e3mi
