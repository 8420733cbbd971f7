// First interaction layer, factorised by species.
//
// The first layer's input features are the embedding h0_j = W_emb[z_j] (a
// function of the sender's species only), and its paths are (0, l, l). The
// neighbour sum then factorises exactly:
//   A_i[l, k, m] = nu^-1 sum_e R_e[l, k] W_emb[z_j, k] (C Y_e)[l m]
//                = nu^-1 sum_{s, q} W3[q, l C + k] W_emb[s, k] G_i[s, q, l m],
//   G_i[s, q, l m] = sum_{e in in(i), z_j = s} H2_e[q] (C Y_e)[l m],
// with H2 the radial MLP's second hidden layer. Folding in the channel mix,
//   h~_l = G_l U_l (+ h0 S_0 for l = 0),   U_l = nu^-1 (W3_l o W_emb) W_mix_l,
// so the per-edge output layer of the radial MLP (64 x P C multiply-adds and
// 4 P C bytes of R per edge) is never formed: per edge only the 8 -> 64 -> 64
// hidden layers and a 64 x 16 outer product remain, and U_l is a weight
// computed once per model.
//
// Kernels (one workgroup per receiver, its CSR row in tiles of 64 edges):
//   k_first_fwd  G_i [N, (L3+1)^2, S*64]
//   k_first_bwd  from dG = dh~_l U_l^T: dH2_e = sum_c dG[c, z_j] (CY)_e[c],
//                d(CY)_e = sum_q dG[c, z_j, q] H2_e[q], back through the MLP and
//                the harmonics to g_e = dE/dd_e (added to the other layers').
#include "common.h"
#include "paths.h"
#include "runtime.h"

namespace e3mi {
namespace {

constexpr int kTile = 64;
constexpr int kH = 64;
constexpr int kLd = 65;
constexpr int kMaxS64 = 512;  // species x hidden width held in LDS

__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ f32x16 block_64(const float (*X)[kLd], int rb, const float* __restrict__ W, int ldw,
                                           int cb) {
  const int lane = threadIdx.x & 63;
  f32x16 acc = {};
#pragma unroll 8
  for (int kk = 0; kk < kH; kk += 2)
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(X[rb + (lane & 31)][kk + (lane >> 5)],
                                                W[(kk + (lane >> 5)) * ldw + cb + (lane & 31)], acc, 0, 0, 0);
  return acc;
}

// (C Y)[l m3] = sum_m2 C^{(0,l,l)}[0, m2, m3] Y[l m2] for l <= L3 (and its transpose).
template <int L3>
__device__ __forceinline__ void cg_apply(const float* Y, float* CY) {
  static_for<L3 + 1>([&](auto l) {
    constexpr int lv = decltype(l)::value;
    constexpr int g = [] {
      for (int q = 0; q < kNumPaths; ++q)
        if (kL1[q] == 0 && kL2[q] == lv && kL3[q] == lv) return q;
      return -1;
    }();
    static_assert(g >= 0, "path (0,l,l) missing from the table");
#pragma unroll
    for (int m = 0; m < 2 * lv + 1; ++m) CY[lv * lv + m] = 0.0f;
    static_for<kNzBegin[g + 1] - kNzBegin[g]>([&](auto z) {
      constexpr int q = kNzBegin[g] + z;
      CY[lv * lv + kM3[q]] += kC[q] * Y[lv * lv + kM2[q]];
    });
  });
}
template <int L3>
__device__ __forceinline__ void cg_apply_t(const float* dCY, float* dY) {
  static_for<L3 + 1>([&](auto l) {
    constexpr int lv = decltype(l)::value;
    constexpr int g = [] {
      for (int q = 0; q < kNumPaths; ++q)
        if (kL1[q] == 0 && kL2[q] == lv && kL3[q] == lv) return q;
      return -1;
    }();
#pragma unroll
    for (int m = 0; m < 2 * lv + 1; ++m) dY[lv * lv + m] = 0.0f;
    static_for<kNzBegin[g + 1] - kNzBegin[g]>([&](auto z) {
      constexpr int q = kNzBegin[g] + z;
      dY[lv * lv + kM2[q]] += kC[q] * dCY[lv * lv + kM3[q]];
    });
  });
}

// B (and dB/dr) and the CG-weighted harmonics of one tile; padded rows get zeros.
template <int LMAX, int L3, int NB>
__device__ __forceinline__ void tile_geometry(const float4* __restrict__ dvec, const int* __restrict__ src,
                                              const int* __restrict__ species, int e0, int e1, float rc, int p,
                                              float (*Bs)[NB + 1], float (*dBs)[NB + 1],
                                              float (*Ys)[(L3 + 1) * (L3 + 1) + 1], int* sp) {
  constexpr int NC3 = (L3 + 1) * (L3 + 1);
  const int t = threadIdx.x;
  if (t < kTile) {
    const int e = e0 + t;
    const bool valid = e < e1;
    const float4 d = valid ? dvec[e] : make_float4(0.f, 0.f, 1.f, rc);
    float b[NB], db[NB];
    radial_basis<NB>(d.w, rc, p, b, dBs ? db : nullptr);
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      Bs[t][n] = b[n];
      if (dBs) dBs[t][n] = db[n];
    }
    float Y[(LMAX + 1) * (LMAX + 1)], CY[NC3];
    const float ir = 1.0f / d.w;
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    cg_apply<L3>(Y, CY);
#pragma unroll
    for (int c = 0; c < NC3; ++c) Ys[t][c] = valid ? CY[c] : 0.0f;
    sp[t] = valid ? species[src[e]] : 0;
  }
}

template <int NB>
__device__ __forceinline__ void hidden1(const float (*Bs)[NB + 1], const float* __restrict__ W1, float (*P1)[kLd],
                                        float (*H1)[kLd]) {
  const int t = threadIdx.x;
  const int row = t >> 2, cb = (t & 3) * 16;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    float s = 0.0f;
#pragma unroll
    for (int n = 0; n < NB; ++n) s += Bs[row][n] * W1[n * kH + cb + j];
    if (P1) P1[row][cb + j] = s;
    H1[row][cb + j] = siluf(s);
  }
}

template <int LMAX, int L3>
__global__ void __launch_bounds__(256) k_first_fwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                   const float4* __restrict__ dvec, const int* __restrict__ species,
                                                   int S64, const float* __restrict__ W1, const float* __restrict__ W2,
                                                   float rc, int p, float* __restrict__ G) {
  constexpr int NB = 8;
  constexpr int NC3 = (L3 + 1) * (L3 + 1);
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float X[kTile][kLd];
  __shared__ float Ys[kTile][NC3 + 1];
  __shared__ int sp[kTile];
  extern __shared__ float Gs[];  // [NC3][S64]
  const int i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int k = t; k < NC3 * S64; k += 256) Gs[k] = 0.0f;
  const int e1 = row_ptr[i + 1];
  for (int e0 = row_ptr[i]; e0 < e1; e0 += kTile) {
    __syncthreads();
    tile_geometry<LMAX, L3, NB>(dvec, src, species, e0, e1, rc, p, Bs, nullptr, Ys, sp);
    __syncthreads();
    hidden1<NB>(Bs, W1, nullptr, X);
    __syncthreads();
    {
      const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
      const f32x16 acc = block_64(X, rb, W2, kH, cb);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) X[rb + acc_row(r, lane)][cb + (lane & 31)] = siluf(acc[r]);
    }
    __syncthreads();
    const int n_e = min(kTile, e1 - e0);
    for (int e = 0; e < n_e; ++e) {
      const float h = X[e][lane];
      const int base = sp[e] * kH + lane;
      for (int c = w; c < NC3; c += 4) Gs[c * S64 + base] += h * Ys[e][c];
    }
  }
  __syncthreads();
  float* Gi = G + (long)i * NC3 * S64;
  for (int k = t; k < NC3 * S64; k += 256) Gi[k] = Gs[k];
}

template <int LMAX, int L3>
__global__ void __launch_bounds__(256) k_first_bwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                   const float4* __restrict__ dvec, const int* __restrict__ species,
                                                   int S64, const float* __restrict__ W1, const float* __restrict__ W2,
                                                   const float* __restrict__ W2T, const float* __restrict__ dG,
                                                   float4* __restrict__ g, int accumulate, float rc, int p) {
  constexpr int NB = 8;
  constexpr int NC3 = (L3 + 1) * (L3 + 1);
  // LDS kept under 64 KB (static + the receiver's dG): the first hidden
  // layer's pre-activation is recomputed where its derivative is needed.
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float dBs[kTile][NB + 1];
  __shared__ float P2[kTile][kLd];
  __shared__ float X[kTile][kLd];
  __shared__ float Ys[kTile][NC3 + 1];
  __shared__ float dYs[kTile][NC3 + 1];
  __shared__ int sp[kTile];
  extern __shared__ float Gs[];  // [NC3][S64], the receiver's dG
  const int i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
  const float* dGi = dG + (long)i * NC3 * S64;
  for (int k = t; k < NC3 * S64; k += 256) Gs[k] = dGi[k];
  const int e1 = row_ptr[i + 1];
  for (int e0 = row_ptr[i]; e0 < e1; e0 += kTile) {
    __syncthreads();
    tile_geometry<LMAX, L3, NB>(dvec, src, species, e0, e1, rc, p, Bs, dBs, Ys, sp);
    __syncthreads();
    hidden1<NB>(Bs, W1, nullptr, X);
    __syncthreads();
    {
      const f32x16 acc = block_64(X, rb, W2, kH, cb);
#pragma unroll
      for (int r = 0; r < 16; ++r) P2[rb + acc_row(r, lane)][cb + (lane & 31)] = acc[r];
    }
    __syncthreads();
    for (int e = w; e < kTile; e += 4) X[e][lane] = siluf(P2[e][lane]);  // H2
    __syncthreads();
    // d(CY)_e[c] = sum_q dG[c, s_e, q] H2_e[q]
    {
      const int e = t >> 2;
      const int base = sp[e] * kH;
      for (int c = t & 3; c < NC3; c += 4) {
        float s = 0.0f;
#pragma unroll 8
        for (int q = 0; q < kH; ++q) s += Gs[c * S64 + base + q] * X[e][q];
        dYs[e][c] = s;
      }
    }
    __syncthreads();
    // dH2[e, q] = sum_c dG[c, s_e, q] (CY)_e[c]  ->  dP2 = dH2 silu'(P2)  (into X)
    for (int e = w; e < kTile; e += 4) {
      const int base = sp[e] * kH + lane;
      float s = 0.0f;
#pragma unroll
      for (int c = 0; c < NC3; ++c) s += Gs[c * S64 + base] * Ys[e][c];
      X[e][lane] = s * silu_grad(P2[e][lane]);
    }
    __syncthreads();
    {
      // dH1 = dP2 W2^T, dP1 = dH1 silu'(P1) -> P2, with P1 = B W1 recomputed
      const f32x16 a2 = block_64(X, rb, W2T, kH, cb);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = rb + acc_row(r, lane), col = cb + (lane & 31);
        float p1 = 0.0f;
#pragma unroll
        for (int n = 0; n < NB; ++n) p1 += Bs[row][n] * W1[n * kH + col];
        P2[row][col] = a2[r] * silu_grad(p1);
      }
    }
    __syncthreads();
    if (t < kTile && e0 + t < e1) {
      const int e = e0 + t;
      float dr = 0.0f;
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        float s = 0.0f;
        for (int q = 0; q < kH; ++q) s += P2[t][q] * W1[n * kH + q];
        dr += s * dBs[t][n];
      }
      const float4 d = dvec[e];
      const float ir = 1.0f / d.w;
      const float nx = d.x * ir, ny = d.y * ir, nz = d.z * ir;
      float dcy[NC3], dy[16];
#pragma unroll
      for (int c = 0; c < NC3; ++c) dcy[c] = dYs[t][c];
#pragma unroll
      for (int c = 0; c < 16; ++c) dy[c] = 0.0f;
      cg_apply_t<L3>(dcy, dy);
      float Gx, Gy, Gz;
      real_sh_vjp<LMAX>(nx, ny, nz, dy, Gx, Gy, Gz);
      const float dot = Gx * nx + Gy * ny + Gz * nz;
      const float gx = dr * nx + (Gx - dot * nx) * ir;
      const float gy = dr * ny + (Gy - dot * ny) * ir;
      const float gz = dr * nz + (Gz - dot * nz) * ir;
      if (accumulate) {
        const float4 o = g[e];
        g[e] = make_float4(o.x + gx, o.y + gy, o.z + gz, 0.0f);
      } else {
        g[e] = make_float4(gx, gy, gz, 0.0f);
      }
    }
  }
}

}  // namespace

template <int LMAX, int L3>
static void first_launch(bool fwd, const int* row_ptr, const int* src, const float4* dvec, const int* species, int N,
                         int S64, const float* W1, const float* W2, const float* W2T, float* G, const float* dG,
                         float4* g, int accumulate, float rc, int p, hipStream_t st) {
  const size_t lds = sizeof(float) * (size_t)(L3 + 1) * (L3 + 1) * S64;
  if (fwd)
    k_first_fwd<LMAX, L3><<<N, 256, lds, st>>>(row_ptr, src, dvec, species, S64, W1, W2, rc, p, G);
  else
    k_first_bwd<LMAX, L3><<<N, 256, lds, st>>>(row_ptr, src, dvec, species, S64, W1, W2, W2T, dG, g, accumulate, rc,
                                               p);
}

// LDS a first-layer workgroup needs (the larger, adjoint kernel): static
// arrays plus the receiver's [(l3+1)^2, S*64] block. Kept within 64 KB.
size_t first_lds_bytes(int l3max, int S64) {
  const size_t nc3 = (size_t)(l3max + 1) * (l3max + 1);
  const size_t fixed = 2 * kTile * 9 * 4 + 2 * kTile * kLd * 4 + 2 * kTile * (nc3 + 1) * 4 + kTile * 4;
  return fixed + nc3 * S64 * 4;
}

void launch_first(bool fwd, int lmax, int l3max, const int* row_ptr, const int* src, const float4* dvec,
                  const int* species, int N, int S64, const float* W1, const float* W2, const float* W2T, float* G,
                  const float* dG, float4* g, int accumulate, float rc, int p, hipStream_t st) {
  if (N == 0) return;
  if (S64 > kMaxS64 || first_lds_bytes(l3max, S64) > 65536)
    throw Error(E3MI_EUNSUPPORTED, "first-layer factorisation: too many species for the LDS budget");
  if (lmax == 3 && l3max == 3)
    first_launch<3, 3>(fwd, row_ptr, src, dvec, species, N, S64, W1, W2, W2T, G, dG, g, accumulate, rc, p, st);
  else if (lmax == 3 && l3max == 0)
    first_launch<3, 0>(fwd, row_ptr, src, dvec, species, N, S64, W1, W2, W2T, G, dG, g, accumulate, rc, p, st);
  else if (lmax == 2 && l3max == 2)
    first_launch<2, 2>(fwd, row_ptr, src, dvec, species, N, S64, W1, W2, W2T, G, dG, g, accumulate, rc, p, st);
  else if (lmax == 2 && l3max == 0)
    first_launch<2, 0>(fwd, row_ptr, src, dvec, species, N, S64, W1, W2, W2T, G, dG, g, accumulate, rc, p, st);
  else
    throw Error(E3MI_EUNSUPPORTED, "first-layer factorisation: unsupported orders");
}

}  // namespace e3mi
