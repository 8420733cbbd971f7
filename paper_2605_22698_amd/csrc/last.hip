// Last interaction layer, fused: radial MLP, tensor product and neighbour sum
// in one kernel per direction, with no per-edge radial tensor in memory.
//
// The last layer only feeds the energy through its scalar outputs, so its
// paths are (l, l, 0) for l = 0..L and, per edge e = (i <- j),
//   s_e[l, c]  = sum_m h_j[l m, c] V_e[l m],   V_e = C^{(l,l,0)} folded with Y_e
//   A_i[l, c]  = nu^-1 sum_e R_e[l, c] s_e[l, c],   R_e = W3^T H2_e,
// H2_e the radial MLP's second hidden layer (8 -> 64 -> 64). Writing R out as
// W3^T H2 gives
//   A_i[l, c]  = nu^-1 sum_q W3[q, l C + c] T_i[q, (l, c)],
//   T_i[q, (l, c)] = sum_e H2_e[q] s_e[l, c],
// a 64 x (L+1)C matrix per receiver that is a product over the receiver's
// edges (matrix cores), so the forward pass never forms R.
//
// The adjoint of the same layer, given dA (and dA-hat = nu^-1 dA):
//   dR_e = dA-hat_i o s_e         -> dH2_e = W3 dR_e  (matrix cores, K = (L+1)C)
//   R_e  = W3^T H2_e              (matrix cores, recomputed per tile)
//   dV_e[l m]    = sum_c dA-hat_i[l, c] R_e[l, c] h_j[l m, c]
//   dh_i[l m, c] += (-1)^l sum_{e in in(i)} dA-hat_j[l, c] R_e[l, c] V_e[l m]
// The last line is the sender-side term of the reverse edge (j <- i): R is a
// function of |d| only and Y(-d) = (-1)^l Y(d), so it is gathered from the
// receiver's own row. dH2 goes back through the MLP to dr, dV through the CG
// fold and the harmonics to the direction, giving g_e = dE/dd_e.
//
// One workgroup per receiver, C/32 waves; wave w owns channels
// [32w, 32w + 32) for every order l. Edges are processed in tiles of 64.
#include "common.h"
#include "paths.h"
#include "runtime.h"

namespace e3mi {
namespace {

constexpr int kT = 64;   // edges per tile
constexpr int kH = 64;   // hidden width of the radial MLP
constexpr int kLd = 65;  // padded LDS row
constexpr int kNB = 8;   // radial basis size

__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// Hides a per-lane pointer's value from the optimiser where it is formed, so
// that loads through it with constant offsets are not turned into hoisted
// 64-bit addresses (which would not fit in registers).
template <class T>
__device__ __forceinline__ const T* opaque_v(const T* p) {
  asm volatile("" : "+v"(p));
  return p;
}

// Orders the LDS accesses of one wave (lanes exchange data through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ f32x16 mfma(float a, float b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// V[l m1] = sum_{m2} C^{(l,l,0)}[m1, m2, 0] Y[l m2] (the scalar-output paths
// are the first L+1 entries of the table, in order of l).
template <int LMAX>
__device__ __forceinline__ void fold_cg(const float* Y, float* V) {
  static_for<LMAX + 1>([&](auto l) {
    constexpr int lv = decltype(l)::value;
    static_assert(kL1[lv] == lv && kL2[lv] == lv && kL3[lv] == 0, "scalar-output paths lead the table");
#pragma unroll
    for (int m = 0; m < 2 * lv + 1; ++m) V[lv * lv + m] = 0.0f;
    static_for<kNzBegin[lv + 1] - kNzBegin[lv]>([&](auto z) {
      constexpr int q = kNzBegin[lv] + z;
      static_assert(kM3[q] == 0, "scalar output");
      V[lv * lv + kM1[q]] += kC[q] * Y[lv * lv + kM2[q]];
    });
  });
}
template <int LMAX>
__device__ __forceinline__ void fold_cg_t(const float* dV, float* dY) {
  static_for<LMAX + 1>([&](auto l) {
    constexpr int lv = decltype(l)::value;
#pragma unroll
    for (int m = 0; m < 2 * lv + 1; ++m) dY[lv * lv + m] = 0.0f;
    static_for<kNzBegin[lv + 1] - kNzBegin[lv]>([&](auto z) {
      constexpr int q = kNzBegin[lv] + z;
      dY[lv * lv + kM2[q]] += kC[q] * dV[lv * lv + kM1[q]];
    });
  });
}

// Per-tile edge data: basis (and its r-derivative), folded harmonics, sender.
// Padded rows get B = 0 and V = 0, so they contribute nothing anywhere.
template <int LMAX>
__device__ __forceinline__ void tile_edges(const float4* __restrict__ dvec, const int* __restrict__ src, int e0,
                                           int n_e, float rc, int p, float (*Bs)[kNB + 1], float (*dBs)[kNB + 1],
                                           float (*Vs)[(LMAX + 1) * (LMAX + 1) + 1], int* js) {
  constexpr int NY = (LMAX + 1) * (LMAX + 1);
  const int t = threadIdx.x;
  if (t < kT) {
    const bool valid = t < n_e;
    const float4 d = valid ? dvec[e0 + t] : make_float4(0.f, 0.f, 1.f, rc);
    float b[kNB], db[kNB];
    radial_basis<kNB>(d.w, rc, p, b, dBs ? db : nullptr);
#pragma unroll
    for (int n = 0; n < kNB; ++n) {
      Bs[t][n] = b[n];
      if (dBs) dBs[t][n] = db[n];
    }
    float Y[NY], V[NY];
    const float ir = 1.0f / d.w;
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    fold_cg<LMAX>(Y, V);
#pragma unroll
    for (int k = 0; k < NY; ++k) Vs[t][k] = valid ? V[k] : 0.0f;
    js[t] = src[e0 + (valid ? t : 0)];
  }
}

// H1 = silu(B W1) into X (all rows of the tile).
template <int NT>
__device__ __forceinline__ void hidden1(const float (*Bs)[kNB + 1], const float* __restrict__ W1, float (*X)[kLd]) {
  for (int o = threadIdx.x; o < kT * kH; o += NT) {
    const int row = o >> 6, col = o & 63;
    float s = 0.0f;
#pragma unroll
    for (int n = 0; n < kNB; ++n) s += Bs[row][n] * W1[n * kH + col];
    X[row][col] = siluf(s);
  }
}

// One 32 x 32 block of X[64 x 64] . W[64 x 64] (row block rb, column block cb).
__device__ __forceinline__ f32x16 block_64(const float (*X)[kLd], int rb, const float* __restrict__ W, int cb) {
  const int lane = threadIdx.x & 63;
  f32x16 acc = {};
#pragma unroll 8
  for (int kk = 0; kk < kH; kk += 2)
    acc = mfma(X[rb + (lane & 31)][kk + (lane >> 5)], W[(kk + (lane >> 5)) * kH + cb + (lane & 31)], acc);
  return acc;
}

// Orders handled by a forward wave: pair 0 takes l = 0 and l = L, pair 1 the
// orders in between, so both gather about the same number of components.
template <int LMAX, int PAIR>
struct FwdOrders {
  static constexpr int N = PAIR == 0 ? 2 : LMAX - 1;
  static constexpr int l(int k) { return PAIR == 0 ? (k == 0 ? 0 : LMAX) : 1 + k; }
};

template <int LMAX, int NCB, int PAIR>
__device__ __forceinline__ void last_fwd_body(int i, const int* __restrict__ row_ptr, const int* __restrict__ src,
                                              const float4* __restrict__ dvec, const float* __restrict__ h,
                                              const float* __restrict__ W1, const float* __restrict__ W2,
                                              const float* __restrict__ W3, int ldw3, float* __restrict__ A, float rc,
                                              int p, float inv_nu, float (*Bs)[kNB + 1], float (*X)[kLd],
                                              float (*Vs)[(LMAX + 1) * (LMAX + 1) + 1], int* js) {
  using O = FwdOrders<LMAX, PAIR>;
  constexpr int NW = 2 * NCB, NT = 64 * NW, C = 32 * NCB, NL = LMAX + 1, NY = NL * NL;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c = 32 * (w % NCB) + (lane & 31);
  f32x16 T[2][O::N];
#pragma unroll
  for (int k = 0; k < O::N; ++k) T[0][k] = T[1][k] = f32x16{};
  const int e1 = row_ptr[i + 1];
  for (int e0 = row_ptr[i]; e0 < e1; e0 += kT) {
    const int n_e = min(kT, e1 - e0);
    __syncthreads();
    tile_edges<LMAX>(dvec, src, e0, n_e, rc, p, Bs, nullptr, Vs, js);
    __syncthreads();
    hidden1<NT>(Bs, W1, X);
    __syncthreads();
    {
      // the four 32 x 32 blocks of P2 = H1 W2 over the first waves
      f32x16 acc[2] = {f32x16{}, f32x16{}};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int blk = w + k * NW;
        if (blk < 4) acc[k] = block_64(X, (blk >> 1) * 32, W2, (blk & 1) * 32);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int blk = w + k * NW;
        if (blk < 4) {
#pragma unroll
          for (int r = 0; r < 16; ++r) X[(blk >> 1) * 32 + acc_row(r, lane)][(blk & 1) * 32 + (lane & 31)] = siluf(acc[k][r]);
        }
      }
    }
    __syncthreads();
    // T[q, (l, c)] += sum_e H2[e, q] s[e, (l, c)]: A operand H2^T (lane -> q),
    // B operand s (lane -> channel), two edges per step.
    for (int kk = 0; kk < n_e; kk += 2) {
      const int e = kk + (lane >> 5);
      const float a0 = X[e][lane & 31], a1 = X[e][32 + (lane & 31)];
      const float* hj = h + (long)js[e] * NY * C + c;
      static_for<O::N>([&](auto k) {
        constexpr int lv = O::l(decltype(k)::value);
        float sv = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * lv + 1; ++m) sv += hj[(lv * lv + m) * C] * Vs[e][lv * lv + m];
        T[0][k] = mfma(a0, sv, T[0][k]);
        T[1][k] = mfma(a1, sv, T[1][k]);
      });
    }
  }
  // A[i, l, c] = nu^-1 sum_q W3[q, l C + c] T[q, (l, c)]
  static_for<O::N>([&](auto k) {
    constexpr int lv = O::l(decltype(k)::value);
    float part = 0.0f;
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 16; ++r) part += W3[(long)(qb * 32 + acc_row(r, lane)) * ldw3 + lv * C + c] * T[qb][k][r];
    part += __shfl_xor(part, 32);
    if (lane < 32) A[((long)i * NL + lv) * C + c] = part * inv_nu;
  });
}

// NCB = C / 32 channel blocks; 2 NCB waves (channel block x order pair).
template <int LMAX, int NCB>
__global__ void __launch_bounds__(128 * NCB) k_last_fwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                         const float4* __restrict__ dvec, const float* __restrict__ h,
                                                         const float* __restrict__ W1, const float* __restrict__ W2,
                                                         const float* __restrict__ W3, int ldw3,
                                                         float* __restrict__ A, float rc, int p, float inv_nu) {
  constexpr int NY = (LMAX + 1) * (LMAX + 1);
  __shared__ float Bs[kT][kNB + 1];
  __shared__ float X[kT][kLd];
  __shared__ float Vs[kT][NY + 1];
  __shared__ int js[kT];
  const int i = xcd_contiguous(blockIdx.x, gridDim.x);
  if ((threadIdx.x >> 6) / NCB == 0)
    last_fwd_body<LMAX, NCB, 0>(i, row_ptr, src, dvec, h, W1, W2, W3, ldw3, A, rc, p, inv_nu, Bs, X, Vs, js);
  else
    last_fwd_body<LMAX, NCB, 1>(i, row_ptr, src, dvec, h, W1, W2, W3, ldw3, A, rc, p, inv_nu, Bs, X, Vs, js);
}

// Adjoint. Wave w owns channels [32w, 32w + 32). Per order l:
//   1. R^T_l[e, c] on the matrix cores (lane -> channel): the sender-side
//      node gradient sums over the lane's own edges; ds = dA-hat_i o R goes
//      to LDS.
//   2. per edge (lane -> edge, four channels per lane): one pass over
//      h_j[l m, c..c+3] gives s (-> dR, the B operand of dH2 = W3 dR on the
//      matrix cores, K split over the waves) and dV (with ds from LDS).
template <int LMAX, int NW>
__global__ void __launch_bounds__(64 * NW, 2) k_last_bwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                          const float4* __restrict__ dvec, const float* __restrict__ h,
                                                          const float* __restrict__ dA, const float* __restrict__ W1,
                                                          const float* __restrict__ W2, const float* __restrict__ W2T,
                                                          const float* __restrict__ W3,
                                                          const float* __restrict__ W3T, float4* __restrict__ g,
                                                          int accumulate, float* __restrict__ dh, float rc, int p,
                                                          float inv_nu) {
  constexpr int NT = 64 * NW, C = 32 * NW, NL = LMAX + 1, NY = NL * NL;
  __shared__ float Bs[kT][kNB + 1];
  __shared__ float X[kT][kLd];       // H2, then dH2 -> dP2
  __shared__ float G2[kT][kLd];      // P2, then silu'(P2), then dP1
  __shared__ float DS[kT][C + 1];    // ds = dA-hat_i o R for one order
  __shared__ float Vs[kT][NY + 1];
  __shared__ float dVs[kT][NY + 1];  // dV summed over waves in wave order
  __shared__ int js[kT];
  __shared__ float drs[NW][kT];
  const int i = xcd_contiguous(blockIdx.x, gridDim.x);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c = 32 * w + (lane & 31);
  float dhacc[NY];
#pragma unroll
  for (int k = 0; k < NY; ++k) dhacc[k] = 0.0f;
  const float* dAi = dA + (long)i * NL * C;
  const int e1 = row_ptr[i + 1];
  for (int e0 = row_ptr[i]; e0 < e1; e0 += kT) {
    const int n_e = min(kT, e1 - e0);
    __syncthreads();
    tile_edges<LMAX>(dvec, src, e0, n_e, rc, p, Bs, nullptr, Vs, js);
    __syncthreads();
    hidden1<NT>(Bs, W1, X);
    __syncthreads();
    for (int blk = w; blk < 4; blk += NW) {
      const int rb = (blk >> 1) * 32, cb = (blk & 1) * 32;
      const f32x16 acc = block_64(X, rb, W2, cb);
#pragma unroll
      for (int r = 0; r < 16; ++r) G2[rb + acc_row(r, lane)][cb + (lane & 31)] = acc[r];
    }
    __syncthreads();
    for (int o = t; o < kT * kH; o += NT) {
      const int row = o >> 6, col = o & 63;
      const float p2 = G2[row][col];
      X[row][col] = siluf(p2);
      G2[row][col] = silu_grad(p2);
    }
    __syncthreads();

    f32x16 D[2][2];
    D[0][0] = D[0][1] = D[1][0] = D[1][1] = f32x16{};
    float dv[2][NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) dv[0][k] = dv[1][k] = 0.0f;
    static_for<NL>([&](auto l) __attribute__((always_inline)) {
      constexpr int lv = decltype(l)::value;
      constexpr float sgn = (lv & 1) ? -1.0f : 1.0f;
      {
        // R^T_l[e, c] = sum_q H2[e, q] W3[q, l C + c]; the column of W3 is
        // fetched in one batch
        const float* w3l = opaque_v(W3 + (lane >> 5) * (NL * C) + lv * C + c);
        float wB[kH / 2];
#pragma unroll
        for (int k = 0; k < kH / 2; ++k) wB[k] = w3l[2 * k * (NL * C)];
        f32x16 R[2] = {f32x16{}, f32x16{}};
#pragma unroll
        for (int k = 0; k < kH / 2; ++k) {
          const int q = 2 * k + (lane >> 5);
          R[0] = mfma(X[lane & 31][q], wB[k], R[0]);
          R[1] = mfma(X[32 + (lane & 31)][q], wB[k], R[1]);
        }
        const float dai = inv_nu * dAi[lv * C + c];
        const float* dAl = dA + lv * C + c;
#pragma unroll 1
        for (int eb = 0; eb < 2; ++eb)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int e = eb * 32 + acc_row(r, lane);
            const float u = (sgn * inv_nu) * dAl[(long)js[e] * (NL * C)] * R[eb][r];
#pragma unroll
            for (int m = 0; m < 2 * lv + 1; ++m) dhacc[lv * lv + m] += u * Vs[e][lv * lv + m];
            DS[e][c] = dai * R[eb][r];
          }
      }
      // DS columns [32w, 32w + 32) are written and read by wave w only
      wave_sync();
#pragma unroll 1
      for (int g8 = 0; g8 < 4; ++g8) {
        const int c0 = 32 * w + 8 * g8 + 4 * (lane >> 5);
        // every load of the group is issued before any of it is used
        const float* wtp = opaque_v(W3T + (lv * C + c0) * kH + (lane & 31));
        float wt[8];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          wt[2 * tt] = wtp[tt * kH];
          wt[2 * tt + 1] = wtp[tt * kH + 32];
        }
        const float4 da4 = *reinterpret_cast<const float4*>(dAi + lv * C + c0);
        float4 hv4[2][2 * lv + 1];
#pragma unroll
        for (int eb = 0; eb < 2; ++eb) {
          const float* hj = opaque_v(h + (long)js[eb * 32 + (lane & 31)] * NY * C + lv * lv * C + c0);
#pragma unroll
          for (int m = 0; m < 2 * lv + 1; ++m) hv4[eb][m] = *reinterpret_cast<const float4*>(hj + m * C);
        }
        float dr[2][4];
#pragma unroll
        for (int eb = 0; eb < 2; ++eb) {
          const int e = eb * 32 + (lane & 31);
          const float d0 = DS[e][c0], d1 = DS[e][c0 + 1], d2 = DS[e][c0 + 2], d3 = DS[e][c0 + 3];
          float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
          for (int m = 0; m < 2 * lv + 1; ++m) {
            const float4 hv = hv4[eb][m];
            const float vv = Vs[e][lv * lv + m];
            s0 += hv.x * vv;
            s1 += hv.y * vv;
            s2 += hv.z * vv;
            s3 += hv.w * vv;
            dv[eb][lv * lv + m] += d0 * hv.x + d1 * hv.y + d2 * hv.z + d3 * hv.w;
          }
          dr[eb][0] = inv_nu * da4.x * s0;
          dr[eb][1] = inv_nu * da4.y * s1;
          dr[eb][2] = inv_nu * da4.z * s2;
          dr[eb][3] = inv_nu * da4.w * s3;
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const float aq0 = wt[2 * tt], aq1 = wt[2 * tt + 1];
          D[0][0] = mfma(aq0, dr[0][tt], D[0][0]);
          D[0][1] = mfma(aq0, dr[1][tt], D[0][1]);
          D[1][0] = mfma(aq1, dr[0][tt], D[1][0]);
          D[1][1] = mfma(aq1, dr[1][tt], D[1][1]);
        }
      }
      wave_sync();  // DS is rewritten for the next order
    });
    // the two halves of a wave hold disjoint channels of the same edges
#pragma unroll
    for (int eb = 0; eb < 2; ++eb)
#pragma unroll
      for (int k = 0; k < NY; ++k) dv[eb][k] += __shfl_xor(dv[eb][k], 32);
    // sum over waves in wave order: dH2 into X, dV into dVs
    for (int ww = 0; ww < NW; ++ww) {
      if (w == ww) {
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
          for (int eb = 0; eb < 2; ++eb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int q = qb * 32 + acc_row(r, lane), e = eb * 32 + (lane & 31);
              X[e][q] = (ww == 0 ? 0.0f : X[e][q]) + D[qb][eb][r];
            }
        if (lane < 32) {
#pragma unroll
          for (int eb = 0; eb < 2; ++eb)
#pragma unroll
            for (int k = 0; k < NY; ++k)
              dVs[eb * 32 + lane][k] = (ww == 0 ? 0.0f : dVs[eb * 32 + lane][k]) + dv[eb][k];
        }
      }
      __syncthreads();
    }
    // dP2 = dH2 o silu'(P2)
    for (int o = t; o < kT * kH; o += NT) {
      const int row = o >> 6, col = o & 63;
      X[row][col] *= G2[row][col];
    }
    __syncthreads();
    // dH1 = dP2 W2^T, dP1 = dH1 o silu'(B W1) -> G2
    for (int blk = w; blk < 4; blk += NW) {
      const int rb = (blk >> 1) * 32, cb = (blk & 1) * 32;
      const f32x16 acc = block_64(X, rb, W2T, cb);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = rb + acc_row(r, lane), col = cb + (lane & 31);
        float p1 = 0.0f;
#pragma unroll
        for (int n = 0; n < kNB; ++n) p1 += Bs[row][n] * W1[n * kH + col];
        G2[row][col] = acc[r] * silu_grad(p1);
      }
    }
    __syncthreads();
    // dr partials: sum over the basis functions owned by this wave of
    // dB/dr_n (dP1 . W1[n, :]), with dB/dr recomputed
    {
      const int e = lane;
      const float r = e < n_e ? dvec[e0 + e].w : rc;
      float b[kNB], db[kNB];
      radial_basis<kNB>(r, rc, p, b, db);
      float part = 0.0f;
#pragma unroll
      for (int n = 0; n < kNB; ++n) {
        if (n % NW != w) continue;
        float sacc = 0.0f;
#pragma unroll 8
        for (int q = 0; q < kH; ++q) sacc += G2[e][q] * W1[n * kH + q];
        part += sacc * db[n];
      }
      drs[w][e] = part;
    }
    __syncthreads();
    if (t < n_e) {
      float dr = 0.0f;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) dr += drs[ww][t];
      float dV[NY], dY[NY];
#pragma unroll
      for (int k = 0; k < NY; ++k) dV[k] = dVs[t][k];
      fold_cg_t<LMAX>(dV, dY);
      const int e = e0 + t;
      const float4 d = dvec[e];
      const float ir = 1.0f / d.w;
      const float nx = d.x * ir, ny = d.y * ir, nz = d.z * ir;
      float Gx, Gy, Gz;
      real_sh_vjp<LMAX>(nx, ny, nz, dY, Gx, Gy, Gz);
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
  // node gradient of the layer input: both halves of the wave saw half the edges
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const float v = dhacc[k] + __shfl_xor(dhacc[k], 32);
    if (lane < 32) dh[((long)i * NY + k) * C + c] += v;
  }
}

template <int LMAX, int NW>
void last_launch(bool fwd, const LastArgs& a, hipStream_t st) {
  if (fwd)
    k_last_fwd<LMAX, NW><<<a.N, 128 * NW, 0, st>>>(a.row_ptr, a.src, a.dvec, a.h, a.W1, a.W2, a.W3, a.ldw3, a.A, a.rc,
                                                   a.p, a.inv_nu);
  else
    k_last_bwd<LMAX, NW><<<a.N, 64 * NW, 0, st>>>(a.row_ptr, a.src, a.dvec, a.h, a.dA, a.W1, a.W2, a.W2T, a.W3,
                                                   a.W3T, a.g, a.accumulate, a.dh, a.rc, a.p, a.inv_nu);
}

}  // namespace

bool last_supported(int lmax, int C) { return (lmax == 2 || lmax == 3) && (C == 32 || C == 64 || C == 128); }

void launch_last(bool fwd, const LastArgs& a, hipStream_t st) {
  if (a.N == 0) return;
  if (!last_supported(a.lmax, a.C)) throw Error(E3MI_EUNSUPPORTED, "fused last layer: unsupported order or width");
  if (a.ldw3 != (a.lmax + 1) * a.C) throw Error(E3MI_EINVAL, "fused last layer: W3 must hold the used columns only");
  if (a.lmax == 3) {
    if (a.C == 128) last_launch<3, 4>(fwd, a, st);
    else if (a.C == 64) last_launch<3, 2>(fwd, a, st);
    else last_launch<3, 1>(fwd, a, st);
  } else {
    if (a.C == 128) last_launch<2, 4>(fwd, a, st);
    else if (a.C == 64) last_launch<2, 2>(fwd, a, st);
    else last_launch<2, 1>(fwd, a, st);
  }
}

}  // namespace e3mi
