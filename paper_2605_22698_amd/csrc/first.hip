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
// The hidden layers depend on the edge length only, so an edge and its
// reverse share them: k_first_hidden computes the second hidden layer's
// pre-activation P2 = silu(B W1) W2 once per edge pair (tiles of 64 pair
// owners, or of 64 edges without the pair list), and both kernels below read
// it through the edge's pair index.
//
// Kernels (one workgroup per receiver, its CSR row in tiles of 64 edges):
//   k_first_hidden  P2 [pairs, 64]
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
  // three waves in parallel: the basis (wave 0), the harmonics (wave 1) and
  // the senders' species (wave 2) of the tile's 64 edges
  const int t = threadIdx.x, te = t & 63, part = t >> 6;
  const int e = e0 + te;
  const bool valid = e < e1;
  if (part == 0) {
    const float r = valid ? dvec[e].w : rc;
    float b[NB], db[NB];
    radial_basis<NB>(r, rc, p, b, dBs ? db : nullptr);
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      Bs[te][n] = b[n];
      if (dBs) dBs[te][n] = db[n];
    }
  } else if (part == 1) {
    const float4 d = valid ? dvec[e] : make_float4(0.f, 0.f, 1.f, rc);
    float Y[(LMAX + 1) * (LMAX + 1)], CY[NC3];
    const float ir = 1.0f / d.w;
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    cg_apply<L3>(Y, CY);
#pragma unroll
    for (int c = 0; c < NC3; ++c) Ys[te][c] = valid ? CY[c] : 0.0f;
  } else if (part == 2) {
    sp[te] = valid ? species[src[e]] : 0;
  }
}

template <int NB>
__device__ __forceinline__ void hidden1(const float (*Bs)[NB + 1], const float* __restrict__ W1, float (*H1)[kLd]) {
  for (int o = threadIdx.x; o < kTile * kH; o += 256) {
    const int row = o >> 6, col = o & 63;
    float s = 0.0f;
#pragma unroll
    for (int n = 0; n < NB; ++n) s += Bs[row][n] * W1[n * kH + col];
    H1[row][col] = siluf(s);
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// The tile's edges grouped by sender species, a stable counting sort by wave
// 0: rows perm[start[s] .. start[s] + cnt[s]) of the tile have z_j = s.
__device__ __forceinline__ void species_lists(const int* sp, int n_e, int S, int* perm, int* start, int* cnt) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const bool valid = lane < n_e;
    const int z = sp[lane];
    const unsigned long long below = (1ull << lane) - 1ull;
    int base = 0;
    for (int s = 0; s < S; ++s) {
      const unsigned long long m = __ballot(valid && z == s);
      if (valid && z == s) perm[base + __popcll(m & below)] = lane;
      if (lane == 0) {
        start[s] = base;
        cnt[s] = __popcll(m);
      }
      base += __popcll(m);
    }
  }
}

// X[row] = P2 row of the tile's edge e0 + row (its pair's, through pair_of,
// or its own), or silu of it; rows past the tile's n_e edges zero. All 256
// threads, 16-byte loads.
__device__ __forceinline__ void load_p2_rows(const float* __restrict__ P2, const int* __restrict__ pair_of, int e0,
                                             int n_e, float (*X)[kLd], bool silu = false) {
  for (int o = threadIdx.x; o < kTile * (kH / 4); o += 256) {
    const int row = o / (kH / 4), c4 = (o % (kH / 4)) * 4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < n_e) {
      const int e = e0 + row;
      v = *reinterpret_cast<const float4*>(P2 + (long)(pair_of ? pair_of[e] : e) * kH + c4);
      if (silu) v = make_float4(siluf(v.x), siluf(v.y), siluf(v.z), siluf(v.w));
    }
    X[row][c4] = v.x;
    X[row][c4 + 1] = v.y;
    X[row][c4 + 2] = v.z;
    X[row][c4 + 3] = v.w;
  }
}

// P2 = silu(B W1) W2 of 64 pair owners (own: the pair list, P = *n_own) or
// of 64 edges (own NULL: every edge inside the cutoff, row_ptr_x[N]), row q
// of P2 for the tile's row q.
template <int NB>
__global__ void __launch_bounds__(256) k_first_hidden(const float4* __restrict__ dvec, const int* __restrict__ row_ptr_x,
                                                      int N, const int* __restrict__ own,
                                                      const int* __restrict__ n_own, const float* __restrict__ W1,
                                                      const float* __restrict__ W2, float rc, int p,
                                                      float* __restrict__ P2) {
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float X[kTile][kLd];
  const int n = own ? *n_own : row_ptr_x[N];
  const int q0 = blockIdx.x * kTile;
  if (q0 >= n) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t < kTile) {
    const int q = q0 + t;
    const int e = q < n ? (own ? own[q] : q) : -1;
    const float r = e >= 0 ? dvec[e].w : rc;
    float b[NB];
    radial_basis<NB>(r, rc, p, b, nullptr);
#pragma unroll
    for (int k = 0; k < NB; ++k) Bs[t][k] = b[k];
  }
  __syncthreads();
  hidden1<NB>(Bs, W1, X);
  __syncthreads();
  const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
  const f32x16 a = block_64(X, rb, W2, kH, cb);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int q = q0 + rb + acc_row(r, lane);
    if (q < n) P2[(long)q * kH + cb + (lane & 31)] = a[r];
  }
}

// Forward: G_i[n = (c, s), q] = sum_e [z_j(e) = s] (CY)_e[c] H2_e[q]. For each
// species, a 16 (component) x 64 (q) product over that species' edges of the
// tile on the matrix cores (16x16x4 steps over groups of 4 edges), accumulated
// across tiles in registers; wave w takes species w and w + 4.
template <int LMAX, int L3>
__global__ void __launch_bounds__(256) k_first_fwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                   const float4* __restrict__ dvec, const int* __restrict__ species,
                                                   int S, const int* __restrict__ pair_of,
                                                   const float* __restrict__ P2, float rc, int p,
                                                   float* __restrict__ G) {
  constexpr int NB = 8;
  constexpr int NC3 = (L3 + 1) * (L3 + 1);
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float X[kTile][kLd];
  __shared__ float Ys[kTile][NC3 + 1];
  __shared__ int sp[kTile];
  __shared__ int perm[kTile], start[8], cnt[8];
  const int i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int NN = NC3 * S;
  const int c = lane & 15, h = lane >> 4;
  f32x4 acc[2][4];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[j][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int e1 = row_ptr[i + 1];
  for (int e0 = row_ptr[i]; e0 < e1; e0 += kTile) {
    const int n_e = min(kTile, e1 - e0);
    __syncthreads();
    tile_geometry<LMAX, L3, NB>(dvec, src, species, e0, e1, rc, p, Bs, nullptr, Ys, sp);
    __syncthreads();
    species_lists(sp, n_e, S, perm, start, cnt);
    // H2 = silu(P2) of the tile's edges (rows past them zero, never read)
    load_p2_rows(P2, pair_of, e0, n_e, X, true);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int s = w + 4 * j;
      if (s >= S) break;
      const int s0 = start[s], ns = cnt[s];
      for (int kk = 0; kk < ns; kk += 4) {
        const int e = kk + h < ns ? perm[s0 + kk + h] : -1;
        const float a = (e >= 0 && c < NC3) ? Ys[e][c] : 0.0f;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[j][nb] = mfma16(a, e >= 0 ? X[e][nb * 16 + c] : 0.0f, acc[j][nb]);
      }
    }
  }
  float* Gi = G + (long)i * NN * kH;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int s = w + 4 * j;
    if (s >= S) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cc = 4 * h + r;
      if (cc < NC3) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) Gi[(cc * S + s) * kH + nb * 16 + c] = acc[j][nb][r];
      }
    }
  }
}

// Adjoint, from dG (= dh~ U^T) of the receiver, held in LDS as U[n][q]; for
// the edges of each sender species s (blocks of 16, 16x16x4 matrix-core steps):
//   d(CY)_e[c] = sum_q H2[e, q] U[(c, s), q]
//   dH2[e, q]  = sum_c (CY)_e[c] U[(c, s), q]
//   dP2 = dH2 o silu'(P2), dH1 = dP2 W2^T, dP1 = dH1 o silu'(B W1),
//   dr = sum_n (dP1 . W1[n, :]) dB_n/dr, and d(CY) -> dY -> direction,
// giving g_e = dE/dd_e (added to the other layers' contributions).
template <int LMAX, int L3>
__global__ void __launch_bounds__(256) k_first_bwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                   const float4* __restrict__ dvec, const int* __restrict__ species,
                                                   int S, const float* __restrict__ W1,
                                                   const float* __restrict__ W2T, const int* __restrict__ pair_of,
                                                   const float* __restrict__ P2, const float* __restrict__ dG,
                                                   float4* __restrict__ g, int accumulate, float rc, int p) {
  constexpr int NB = 8;
  constexpr int NC3 = (L3 + 1) * (L3 + 1);
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float X[kTile][kLd];   // H1, H2, then dP2
  __shared__ float Ys[kTile][NC3 + 1];
  __shared__ float dYs[kTile][NC3 + 1];
  __shared__ int sp[kTile];
  __shared__ float drs[4][kTile];
  __shared__ int perm[kTile], start[8], cnt[8];
  extern __shared__ float Ub[];     // [max(NN, 64)][kLd]: the receiver's dG, then dP1
  float (*U)[kLd] = reinterpret_cast<float (*)[kLd]>(Ub);
  const int i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int NN = NC3 * S;
  const int c16 = lane & 15, h4 = lane >> 4;
  const float* dGi = dG + (long)i * NN * kH;
  const int e1 = row_ptr[i + 1];
  for (int e0 = row_ptr[i]; e0 < e1; e0 += kTile) {
    const int n_e = min(kTile, e1 - e0);
    __syncthreads();
    {
      const float4* dG4 = reinterpret_cast<const float4*>(dGi);
      for (int o = t; o < NN * kH / 4; o += 256) {
        const float4 v = dG4[o];
        float* u = &U[o >> 4][(o & 15) * 4];
        u[0] = v.x;
        u[1] = v.y;
        u[2] = v.z;
        u[3] = v.w;
      }
    }
    tile_geometry<LMAX, L3, NB>(dvec, src, species, e0, e1, rc, p, Bs, nullptr, Ys, sp);
    __syncthreads();
    species_lists(sp, n_e, S, perm, start, cnt);
    // the tile's P2 rows into LDS (rows past the tile's edges zero), then
    // H2 = silu(P2) in place; silu'(P2) of this wave's block stays in
    // registers (the dH2 block below has the same rows and columns)
    load_p2_rows(P2, pair_of, e0, n_e, X);
    __syncthreads();
    f32x16 sg;
    {
      const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float& x = X[rb + acc_row(r, lane)][cb + (lane & 31)];
        const float pv = x;
        sg[r] = silu_grad(pv);
        x = siluf(pv);
      }
    }
    __syncthreads();
    // Work items (species s, block of 16 of its edges), dealt to the waves in
    // turn; blocks of 16 rows of perm (padded with -1).
    int n_items = 0;
    for (int s = 0; s < S; ++s) n_items += (cnt[s] + 15) >> 4;
    auto item = [&](int it, int& s, int& eb) {
      s = 0;
      for (;; ++s) {
        const int nb = (cnt[s] + 15) >> 4;
        if (it < nb) break;
        it -= nb;
      }
      eb = it;
    };
    // d(CY)_e[c] = sum_q H2[e, q] U[(c, s), q] for the edges of species s
    // (16 edges x 16 components, K = 64 in steps of 4)
    for (int it = w; it < n_items; it += 4) {
      int s, eb;
      item(it, s, eb);
      const int s0 = start[s], ns = cnt[s];
      const int ea = eb * 16 + c16 < ns ? perm[s0 + eb * 16 + c16] : -1;
      f32x4 a = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int kk = 0; kk < kH; kk += 4) {
        const int q = kk + h4;
        a = mfma16(ea >= 0 ? X[ea][q] : 0.0f, c16 < NC3 ? U[c16 * S + s][q] : 0.0f, a);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int el = eb * 16 + 4 * h4 + r;
        if (el < ns && c16 < NC3) dYs[perm[s0 + el]][c16] = a[r];
      }
    }
    __syncthreads();  // H2 no longer read: X takes dH2
    // dH2[e, q] = sum_c (CY)_e[c] U[(c, s), q] (16 edges x 64 q, K = NC3 <= 16)
    for (int it = w; it < n_items; it += 4) {
      int s, eb;
      item(it, s, eb);
      const int s0 = start[s], ns = cnt[s];
      const int ea = eb * 16 + c16 < ns ? perm[s0 + eb * 16 + c16] : -1;
      f32x4 a[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) a[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < NC3; kk += 4) {
        const int cc = kk + h4;
        const bool ok = cc < NC3;
        const float av = (ea >= 0 && ok) ? Ys[ea][cc] : 0.0f;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) a[nb] = mfma16(av, ok ? U[cc * S + s][nb * 16 + c16] : 0.0f, a[nb]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int el = eb * 16 + 4 * h4 + r;
        if (el < ns) {
          const int e = perm[s0 + el];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) X[e][nb * 16 + c16] = a[nb][r];
        }
      }
    }
    __syncthreads();
    {
      // dP2 = dH2 silu'(P2) in the P2 block layout (rows past the tile's edges zeroed)
      const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int e = rb + acc_row(r, lane), q = cb + (lane & 31);
        X[e][q] = e < n_e ? X[e][q] * sg[r] : 0.0f;
      }
    }
    __syncthreads();
    {
      // dH1 = dP2 W2^T, dP1 = dH1 silu'(P1) -> U, with P1 = B W1 recomputed
      const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
      const f32x16 a2 = block_64(X, rb, W2T, kH, cb);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = rb + acc_row(r, lane), col = cb + (lane & 31);
        float p1 = 0.0f;
#pragma unroll
        for (int n = 0; n < NB; ++n) p1 += Bs[row][n] * W1[n * kH + col];
        U[row][col] = a2[r] * silu_grad(p1);
      }
    }
    __syncthreads();
    {
      // dr partials: wave w takes basis functions 2w, 2w+1
      const int e = lane;
      const float r = lane < n_e ? dvec[e0 + lane].w : rc;
      float b[NB], db[NB];
      radial_basis<NB>(r, rc, p, b, db);
      float part = 0.0f;
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        if (n / (NB / 4) != w) continue;
        float s = 0.0f;
#pragma unroll 8
        for (int q = 0; q < kH; ++q) s += U[e][q] * W1[n * kH + q];
        part += s * db[n];
      }
      drs[w][e] = part;
    }
    __syncthreads();
    if (t < n_e) {
      const int e = e0 + t;
      const float dr = drs[0][t] + drs[1][t] + drs[2][t] + drs[3][t];
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
                         int S, const float* W1, const float* W2T, const int* pair_of, const float* P2, float* G,
                         const float* dG, float4* g, int accumulate, float rc, int p, hipStream_t st) {
  constexpr int NC3 = (L3 + 1) * (L3 + 1);
  if (fwd) {
    k_first_fwd<LMAX, L3><<<N, 256, 0, st>>>(row_ptr, src, dvec, species, S, pair_of, P2, rc, p, G);
  } else {
    const size_t lds = sizeof(float) * (size_t)std::max(NC3 * S, kTile) * kLd;
    k_first_bwd<LMAX, L3><<<N, 256, lds, st>>>(row_ptr, src, dvec, species, S, W1, W2T, pair_of, P2, dG, g,
                                               accumulate, rc, p);
  }
}

// LDS a first-layer workgroup needs (the larger, adjoint kernel): static
// arrays plus the receiver's dG block [(l3+1)^2 S, 64] (padded rows, at least
// 64 of them, later reused for dP1). Kept within 64 KB.
size_t first_lds_bytes(int l3max, int S64) {
  const size_t nc3 = (size_t)(l3max + 1) * (l3max + 1), S = (size_t)S64 / kH;
  const size_t fixed = kTile * 9 * 4 + kTile * kLd * 4 + 2 * kTile * (nc3 + 1) * 4 + kTile * 4 + 4 * kTile * 4;
  return fixed + std::max(nc3 * S, (size_t)kTile) * kLd * 4;
}

void launch_first_hidden(const float4* dvec, const int* row_ptr_x, int N, long e_cap, const int* own,
                         const int* n_own, const float* W1, const float* W2, float rc, int p, float* P2,
                         hipStream_t st) {
  if (e_cap == 0) return;
  E3MI_REQUIRE((own == nullptr) == (n_own == nullptr), E3MI_EINVAL, "first layer: pair list without its count");
  k_first_hidden<8><<<(int)((e_cap + kTile - 1) / kTile), 256, 0, st>>>(dvec, row_ptr_x, N, own, n_own, W1, W2, rc,
                                                                         p, P2);
}

void launch_first(bool fwd, int lmax, int l3max, const int* row_ptr, const int* src, const float4* dvec,
                  const int* species, int N, int S64, const float* W1, const float* W2T, const int* pair_of,
                  const float* P2, float* G, const float* dG, float4* g, int accumulate, float rc, int p,
                  hipStream_t st) {
  if (N == 0) return;
  E3MI_REQUIRE(P2, E3MI_EINVAL, "first layer: hidden pre-activations missing");
  if (S64 > kMaxS64 || first_lds_bytes(l3max, S64) > 65536)
    throw Error(E3MI_EUNSUPPORTED, "first-layer factorisation: too many species for the LDS budget");
  if (lmax == 3 && l3max == 3)
    first_launch<3, 3>(fwd, row_ptr, src, dvec, species, N, S64 / kH, W1, W2T, pair_of, P2, G, dG, g, accumulate,
                       rc, p, st);
  else if (lmax == 3 && l3max == 0)
    first_launch<3, 0>(fwd, row_ptr, src, dvec, species, N, S64 / kH, W1, W2T, pair_of, P2, G, dG, g, accumulate,
                       rc, p, st);
  else if (lmax == 2 && l3max == 2)
    first_launch<2, 2>(fwd, row_ptr, src, dvec, species, N, S64 / kH, W1, W2T, pair_of, P2, G, dG, g, accumulate,
                       rc, p, st);
  else if (lmax == 2 && l3max == 0)
    first_launch<2, 0>(fwd, row_ptr, src, dvec, species, N, S64 / kH, W1, W2T, pair_of, P2, G, dG, g, accumulate,
                       rc, p, st);
  else
    throw Error(E3MI_EUNSUPPORTED, "first-layer factorisation: unsupported orders");
}

}  // namespace e3mi
