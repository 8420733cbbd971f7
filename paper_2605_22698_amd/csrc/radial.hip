// Radial MLP per edge (NequIP table of Appendix F: 8 Bessel functions, a
// radial net of two hidden layers of 64 with swish, polynomial envelope; one
// output weight per (path, channel), no biases):
//   B = bessel(r) u(r/rc);  H1 = silu(B W1);  H2 = silu(H1 W2);  R = H2 W3
// and its adjoint, which ends in the geometric gradient of every edge:
//   dr = dR . dR/dr  (through the MLP and the basis),
//   g_e = dE/dd_e = dr d^ + (I - d^ d^T)/r grad_Y(d^) . dY
//
// One workgroup (4 waves) owns a tile of 64 consecutive edges. The 64x64
// hidden layer and the 64 x (P C) output layer are dense contractions and run
// on the FP32 matrix cores (v_mfma_f32_32x32x2f32: each wave owns 32x32
// output blocks). The edge count is read on the device (row_ptr_x[N]); the
// grid is sized for the skin-list capacity and surplus tiles exit at once.
//
// An edge and its reverse have exactly opposite vectors, so equal lengths and
// equal R. With the pair owners of the pruned list given (own[0 .. P), P on
// the device), a tile holds 64 owners instead of 64 edges: the forward pass
// computes R once per pair and stores it in the pair's row p (mode 2; the
// tensor-product kernels find an edge's row through its pair index) or in
// both edges' rows (mode 1), and the adjoint takes dR of the pair's two edges
// summed (E depends on the pair's length through both) through the MLP once;
// the length gradient goes to the owner's g and each edge keeps its own
// harmonics term. F_i sums g_e - g_rev(e) over i's edges, so the forces are
// those of the edge-by-edge adjoint (to rounding). The modes are template
// arguments, so the edge-by-edge instantiations (mode 0) carry none of it.
//
// MFMA 32x32x2 operand layout (wave64): lane l supplies A[l%32][l/32] and
// B[l/32][l%32]; accumulator register r of lane l holds
// D[8 (r/4) + 4 (l/32) + r%4][l%32].
#include <type_traits>

#include "common.h"
#include "runtime.h"

namespace e3mi {
namespace {

constexpr int kTile = 64;
constexpr int kH = 64;  // hidden width
constexpr int kLd = 65; // padded LDS row

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// pre1 = B W1 (K = NB) on the vector ALU; 256 threads x 16 outputs.
template <int NB>
__device__ __forceinline__ void layer1(const float (*Bs)[NB + 1], const float* __restrict__ W1, float (*P1)[kLd],
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

// acc (32x32 block of the wave) = X[rb:rb+32, :] * W[:, cb:cb+32], K = 64,
// X from LDS, W row-major [64][ldw] from global memory, on the FP32 matrix
// cores.
__device__ __forceinline__ f32x16 block_64(const float (*X)[kLd], int rb, const float* __restrict__ W, int ldw, int cb) {
  const int lane = threadIdx.x & 63;
  f32x16 acc = {};
#pragma unroll 8
  for (int kk = 0; kk < kH; kk += 2) {
    const float a = X[rb + (lane & 31)][kk + (lane >> 5)];
    const float b = W[(kk + (lane >> 5)) * ldw + cb + (lane & 31)];
    acc = mfma32(a, b, acc);
  }
  return acc;
}

// Two 32x32 row blocks (rows 0-31 and 32-63 of X) times W[:, cc:cc+32], K = 64.
__device__ __forceinline__ void block_64x2(const float (*X)[kLd], const float* __restrict__ W, int ldw, int cc,
                                           f32x16& a0, f32x16& a1) {
  const int lane = threadIdx.x & 63;
  a0 = f32x16{};
  a1 = f32x16{};
#pragma unroll 8
  for (int kk = 0; kk < kH; kk += 2) {
    const float b = W[(kk + (lane >> 5)) * ldw + cc + (lane & 31)];
    a0 = mfma32(X[lane & 31][kk + (lane >> 5)], b, a0);
    a1 = mfma32(X[32 + (lane & 31)][kk + (lane >> 5)], b, a1);
  }
}

// The BF16 mode's products: operands rounded to BF16 (nearest even) and
// multiplied on v_mfma_f32_32x32x16_bf16 (lane l supplies A[l%32][8 (l/32) ..
// +8] and B[8 (l/32) .. +8][l%32]), FP32 accumulation.
// BF16 operands already rounded and laid out for the 32x32x16 steps: rows of
// X in LDS as BF16 (row stride kLdb, 16-byte aligned), and the weights
// transposed so that each output column's K values are contiguous (WT[col *
// ldk + k]). Lane l then loads its 8 A and 8 B values with one 16-byte read
// each; the values are the ones the conversions at use produce (round to
// nearest even of the same FP32 numbers), so the results are the same.
constexpr int kLdb = 72;
__device__ __forceinline__ f32x16 block_64_bf(const __bf16 (*Xb)[kLdb], int rb, const __bf16* __restrict__ WT, int ldk,
                                              int cb) {
  const int lane = threadIdx.x & 63;
  f32x16 acc = {};
#pragma unroll
  for (int kb = 0; kb < kH; kb += 16) {
    const int k0 = kb + 8 * (lane >> 5);
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&Xb[rb + (lane & 31)][k0]);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(WT + (long)(cb + (lane & 31)) * ldk + k0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// rows 0-31 and 32-63 of Xb times the columns cc .. cc+31 of W (WT = W^T, K = 64)
__device__ __forceinline__ void block_64x2_bf(const __bf16 (*Xb)[kLdb], const __bf16* __restrict__ WT, int cc,
                                              f32x16& a0, f32x16& a1) {
  const int lane = threadIdx.x & 63;
  a0 = f32x16{};
  a1 = f32x16{};
#pragma unroll
  for (int kb = 0; kb < kH; kb += 16) {
    const int k0 = kb + 8 * (lane >> 5);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(WT + (long)(cc + (lane & 31)) * kH + k0);
    const bf16x8 x0 = *reinterpret_cast<const bf16x8*>(&Xb[lane & 31][k0]);
    const bf16x8 x1 = *reinterpret_cast<const bf16x8*>(&Xb[32 + (lane & 31)][k0]);
    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, b, a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, b, a1, 0, 0, 0);
  }
}

// the 64 x 64 floats of X rounded into Xb (all 256 threads)
__device__ __forceinline__ void to_bf16_tile(const float (*X)[kLd], __bf16 (*Xb)[kLdb]) {
  for (int o = threadIdx.x; o < kTile * kH; o += 256) Xb[o >> 6][o & 63] = (__bf16)X[o >> 6][o & 63];
}

template <int NB, bool BF, class RS, int MODE>
__global__ void __launch_bounds__(256) k_radial_fwd(const float4* __restrict__ dvec, const int* __restrict__ row_ptr_x,
                                                    int N, const float* __restrict__ W1, const float* __restrict__ W2,
                                                    const float* __restrict__ W3, int ld3, int PC,
                                                    RS* __restrict__ R, float rc, int p, int e_first, int e_end,
                                                    const __bf16* __restrict__ W2Tb,
                                                    const __bf16* __restrict__ W3Tb, const int* __restrict__ own,
                                                    const int* __restrict__ n_own, const int* __restrict__ rev) {
  // edges [e_first, e_end) (e_end < 0: every edge inside the cutoff); R is
  // indexed from e_first. BF: W2Tb = W2^T and W3Tb = W3^T (used columns) in
  // BF16. MODE 0: the tile's rows are edges; 1: pair owners (e_first = 0,
  // e_end < 0), R written to both edges' rows; 2: pair owners, R written to
  // the pair's row
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float H[kTile][kLd];
  __shared__ __align__(16) __bf16 Hb[BF ? kTile : 1][kLdb];
  __shared__ int Es[MODE == 1 ? kTile : 1], Ps[MODE == 1 ? kTile : 1];  // owners and partners (-1: none)
  const int E = MODE ? *n_own : e_end >= 0 ? e_end : row_ptr_x[N];
  const int e0 = (MODE ? 0 : e_first) + blockIdx.x * kTile;
  if (e0 >= E) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t < kTile) {
    const int q = e0 + t;
    const int e = q < E ? (MODE ? own[q] : q) : -1;
    if constexpr (MODE == 1) {
      Es[t] = e;
      Ps[t] = e >= 0 ? rev[e] : -1;
    }
    const float r = e >= 0 ? dvec[e].w : rc;
    float b[NB];
    radial_basis<NB>(r, rc, p, b, nullptr);
#pragma unroll
    for (int n = 0; n < NB; ++n) Bs[t][n] = b[n];
  }
  __syncthreads();
  layer1<NB>(Bs, W1, nullptr, H);
  __syncthreads();
  if constexpr (BF) {
    to_bf16_tile(H, Hb);
    __syncthreads();
  }
  {
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    f32x16 acc;
    if constexpr (BF)
      acc = block_64_bf(Hb, rb, W2Tb, kH, cb);
    else
      acc = block_64(H, rb, W2, kH, cb);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if constexpr (BF)
        Hb[rb + acc_row(r, lane)][cb + (lane & 31)] = (__bf16)siluf(acc[r]);
      else
        H[rb + acc_row(r, lane)][cb + (lane & 31)] = siluf(acc[r]);
    }
  }
  __syncthreads();
  for (int cc = w * 32; cc < PC; cc += 128) {
    f32x16 a0, a1;
    if constexpr (BF)
      block_64x2_bf(Hb, W3Tb, cc, a0, a1);
    else
      block_64x2(H, W3, ld3, cc, a0, a1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = acc_row(r, lane);
      if constexpr (MODE != 1) {  // rows in order: edges, or pair indices
        const int ea = e0 + row, eb = e0 + 32 + row;
        if (ea < E) str(R + (long)(ea - e_first) * PC + cc + (lane & 31), a0[r]);
        if (eb < E) str(R + (long)(eb - e_first) * PC + cc + (lane & 31), a1[r]);
      } else {
        const int ea = Es[row], eb = Es[32 + row], pa = Ps[row], pb = Ps[32 + row];
        if (ea >= 0) str(R + (long)ea * PC + cc + (lane & 31), a0[r]);
        if (eb >= 0) str(R + (long)eb * PC + cc + (lane & 31), a1[r]);
        if (pa >= 0) str(R + (long)pa * PC + cc + (lane & 31), a0[r]);
        if (pb >= 0) str(R + (long)pb * PC + cc + (lane & 31), a1[r]);
      }
    }
  }
}

template <int NB, int LMAX, bool BF, class RS, bool PAIR>
__global__ void __launch_bounds__(256) k_radial_bwd(const float4* __restrict__ dvec, const int* __restrict__ row_ptr_x,
                                                    int N, const float* __restrict__ W1, const float* __restrict__ W2,
                                                    const float* __restrict__ W2T, const float* __restrict__ W3T,
                                                    int PC, const RS* __restrict__ dR, const float* __restrict__ dY,
                                                    float4* __restrict__ g, int accumulate, float rc, int p,
                                                    int e_first, int e_end, const __bf16* __restrict__ W2Tb,
                                                    const __bf16* __restrict__ W2b,
                                                    const __bf16* __restrict__ W3ub, const int* __restrict__ own,
                                                    const int* __restrict__ n_own, const int* __restrict__ rev) {
  // BF: W2Tb = W2^T, W2b = W2 and W3ub = W3 (used columns) in BF16, W3 in
  // slabs of 32 columns: W3ub[((c / 32) * 64 + q) * 32 + c % 32] = W3[q][c]
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float dBs[kTile][NB + 1];
  __shared__ float P2[kTile][kLd];
  __shared__ float X[kTile][kLd];
  __shared__ float Ds[BF ? 1 : kTile][33];
  __shared__ __align__(16) __bf16 Xb[BF ? kTile : 1][kLdb];
  __shared__ __align__(16) __bf16 Dsb[BF ? kTile : 1][40];
  __shared__ int Es[PAIR ? kTile : 1], Ps[PAIR ? kTile : 1];  // owners and partners (-1: none)
  // edges [e_first, e_end) (e_end < 0: every edge inside the cutoff); dR is
  // indexed from e_first, dY and g by edge. PAIR: the tile's rows are pair
  // owners (e_first = 0, e_end < 0)
  const int E = PAIR ? *n_own : e_end >= 0 ? e_end : row_ptr_x[N];
  const int e0 = (PAIR ? 0 : e_first) + blockIdx.x * kTile;
  if (e0 >= E) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
  // the row's edge and (pair mode) its partner
  auto row_edge = [&](int row) { return PAIR ? Es[row] : (e0 + row < E ? e0 + row : -1); };
  auto row_partner = [&](int row) { return PAIR ? Ps[row] : -1; };
  if (t < kTile) {
    const int q = e0 + t;
    const int e = q < E ? (PAIR ? own[q] : q) : -1;
    if constexpr (PAIR) {
      Es[t] = e;
      Ps[t] = e >= 0 ? rev[e] : -1;
    }
    const float r = e >= 0 ? dvec[e].w : rc;
    float b[NB], db[NB];
    radial_basis<NB>(r, rc, p, b, db);
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      Bs[t][n] = b[n];
      dBs[t][n] = db[n];
    }
  }
  __syncthreads();
  layer1<NB>(Bs, W1, nullptr, X);  // X = H1 (pre1 is recomputed at the end)
  __syncthreads();
  if constexpr (BF) {
    to_bf16_tile(X, Xb);
    __syncthreads();
  }
  {
    f32x16 acc;
    if constexpr (BF)
      acc = block_64_bf(Xb, rb, W2Tb, kH, cb);
    else
      acc = block_64(X, rb, W2, kH, cb);
#pragma unroll
    for (int r = 0; r < 16; ++r) P2[rb + acc_row(r, lane)][cb + (lane & 31)] = acc[r];
  }
  // dH2 = dR W3^T, K = PC, dR staged through LDS in slabs of 32 columns; the
  // next slab (and, in FP32, its W3^T operands) is loaded into registers
  // while the current one is multiplied.
  // In pair mode a row's dR is the sum of its two edges' rows; the partner's
  // slab is loaded beside the owner's and added when the slab is staged.
  f32x16 acc = {};
  const int srow = t >> 2, sc8 = (t & 3) * 8;
  const int se = row_edge(srow), sp = row_partner(srow);
  const bool sval = se >= 0;
  const RS* dRrow = dR + (long)(sval ? se - e_first : 0) * PC + sc8;
  const RS* dRpart = dR + (long)(sp >= 0 ? sp : 0) * PC + sc8;
  float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0, q0 = p0, q1 = p0;
  float wb[16];
  auto load_slab = [&](int kc) {
    if (sval) {
      float v[8];
      ldr_n<8>(dRrow + kc, v);
      p0 = make_float4(v[0], v[1], v[2], v[3]);
      p1 = make_float4(v[4], v[5], v[6], v[7]);
    }
    if (sp >= 0) {
      float v[8];
      ldr_n<8>(dRpart + kc, v);
      q0 = make_float4(v[0], v[1], v[2], v[3]);
      q1 = make_float4(v[4], v[5], v[6], v[7]);
    }
    if constexpr (!BF) {
#pragma unroll
      for (int i = 0; i < 16; ++i) wb[i] = W3T[(kc + 2 * i + (lane >> 5)) * kH + cb + (lane & 31)];
    }
  };
  load_slab(0);
  for (int kc = 0; kc < PC; kc += 32) {
    __syncthreads();
    if (sp >= 0) {
      p0 = make_float4(p0.x + q0.x, p0.y + q0.y, p0.z + q0.z, p0.w + q0.w);
      p1 = make_float4(p1.x + q1.x, p1.y + q1.y, p1.z + q1.z, p1.w + q1.w);
    }
    if constexpr (BF) {
      bf16x8 v;
      v[0] = (__bf16)p0.x;
      v[1] = (__bf16)p0.y;
      v[2] = (__bf16)p0.z;
      v[3] = (__bf16)p0.w;
      v[4] = (__bf16)p1.x;
      v[5] = (__bf16)p1.y;
      v[6] = (__bf16)p1.z;
      v[7] = (__bf16)p1.w;
      *reinterpret_cast<bf16x8*>(&Dsb[srow][sc8]) = v;
    } else {
      Ds[srow][sc8] = p0.x;
      Ds[srow][sc8 + 1] = p0.y;
      Ds[srow][sc8 + 2] = p0.z;
      Ds[srow][sc8 + 3] = p0.w;
      Ds[srow][sc8 + 4] = p1.x;
      Ds[srow][sc8 + 5] = p1.y;
      Ds[srow][sc8 + 6] = p1.z;
      Ds[srow][sc8 + 7] = p1.w;
    }
    float wcur[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) wcur[i] = wb[i];
    __syncthreads();
    if (kc + 32 < PC) load_slab(kc + 32);
    if constexpr (BF) {
#pragma unroll
      for (int kb = 0; kb < 32; kb += 16) {
        const int k0 = kb + 8 * (lane >> 5);
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&Dsb[rb + (lane & 31)][k0]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(W3ub + ((long)(kc >> 5) * kH + cb + (lane & 31)) * 32 + k0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) acc = mfma32(Ds[rb + (lane & 31)][2 * i + (lane >> 5)], wcur[i], acc);
    }
  }
  __syncthreads();
  // dpre2 = dH2 * silu'(pre2) -> X
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = rb + acc_row(r, lane), col = cb + (lane & 31);
    const float v = acc[r] * silu_grad(P2[row][col]);
    if constexpr (BF)
      Xb[row][col] = (__bf16)v;
    else
      X[row][col] = v;
  }
  __syncthreads();
  {
    // dH1 = dpre2 W2^T ; dpre1 = dH1 * silu'(pre1) -> P2
    f32x16 a2;
    if constexpr (BF)
      a2 = block_64_bf(Xb, rb, W2b, kH, cb);
    else
      a2 = block_64(X, rb, W2T, kH, cb);
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
  // threads 0-63: the rows' edges (length gradient and harmonics term);
  // threads 64-127 in pair mode: the partners (their harmonics term only)
  if (t < (PAIR ? 2 : 1) * kTile) {
    const bool partner = t >= kTile;
    const int row = t & (kTile - 1);
    const int e = partner ? row_partner(row) : row_edge(row);
    if (e >= 0) {
      float dr = 0.0f;
      if (!partner) {
#pragma unroll
        for (int n = 0; n < NB; ++n) {
          float s = 0.0f;
          for (int q = 0; q < kH; ++q) s += P2[row][q] * W1[n * kH + q];
          dr += s * dBs[row][n];
        }
      }
      const float4 d = dvec[e];
      const float ir = 1.0f / d.w;
      const float nx = d.x * ir, ny = d.y * ir, nz = d.z * ir;
      float gx = dr * nx, gy = dr * ny, gz = dr * nz;
      if (dY) {
        float dy[16];
#pragma unroll
        for (int q = 0; q < (LMAX + 1) * (LMAX + 1); ++q) dy[q] = dY[(long)e * 16 + q];
        float Gx, Gy, Gz;
        real_sh_vjp<LMAX>(nx, ny, nz, dy, Gx, Gy, Gz);
        const float dot = Gx * nx + Gy * ny + Gz * nz;
        gx += (Gx - dot * nx) * ir;
        gy += (Gy - dot * ny) * ir;
        gz += (Gz - dot * nz) * ir;
      }
      if (accumulate) {
        const float4 o = g[e];
        g[e] = make_float4(o.x + gx, o.y + gy, o.z + gz, 0.0f);
      } else {
        g[e] = make_float4(gx, gy, gz, 0.0f);
      }
    }
  }
}


// ---- second order (parameter gradients of a force-dependent loss) ----------------
// Tangent pass along per-edge (d_dot, r_dot): B_dot = B'(r) r_dot,
// P1_dot = B_dot W1, H1_dot = silu'(P1) P1_dot, P2_dot = H1_dot W2,
// H2_dot = silu'(P2) P2_dot, R_dot = H2_dot W3. Stores, per edge, [B | B_dot],
// [P1 | P1_dot], [H1 | H1_dot], [P2 | P2_dot], [H2 | H2_dot] for the reverse
// pass and the weight-gradient reductions.
template <int NB>
__global__ void __launch_bounds__(256) k_radial_dual_fwd(const float4* __restrict__ dvec, const float4* __restrict__ dd,
                                                         const int* __restrict__ row_ptr_x, int N,
                                                         const float* __restrict__ W1, const float* __restrict__ W2,
                                                         const float* __restrict__ W3, int ld3, int PC,
                                                         float* __restrict__ Rd, float* __restrict__ Bd,
                                                         float* __restrict__ P1d, float* __restrict__ H1d,
                                                         float* __restrict__ P2d, float* __restrict__ H2d, float rc,
                                                         int p) {
  __shared__ float Bs[kTile][NB + 1];
  __shared__ float Bts[kTile][NB + 1];
  __shared__ float X[kTile][kLd];
  __shared__ float Xt[kTile][kLd];
  const int E = row_ptr_x[N];
  const int e0 = blockIdx.x * kTile;
  if (e0 >= E) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t < kTile) {
    const int e = e0 + t;
    const float r = e < E ? dvec[e].w : rc;
    const float rdot = e < E ? dd[e].w : 0.0f;
    float b[NB], db[NB];
    radial_basis<NB>(r, rc, p, b, db);
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      Bs[t][n] = b[n];
      Bts[t][n] = db[n] * rdot;
      if (e < E) {
        Bd[(long)e * 16 + n] = b[n];
        Bd[(long)e * 16 + 8 + n] = db[n] * rdot;
      }
    }
  }
  __syncthreads();
  {
    const int row = t >> 2, cb = (t & 3) * 16;
    const int e = e0 + row;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      float s = 0.0f, sd = 0.0f;
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        s += Bs[row][n] * W1[n * kH + cb + j];
        sd += Bts[row][n] * W1[n * kH + cb + j];
      }
      const float h = siluf(s), hd = silu_grad(s) * sd;
      X[row][cb + j] = h;
      Xt[row][cb + j] = hd;
      if (e < E) {
        P1d[(long)e * 128 + cb + j] = s;
        P1d[(long)e * 128 + 64 + cb + j] = sd;
        H1d[(long)e * 128 + cb + j] = h;
        H1d[(long)e * 128 + 64 + cb + j] = hd;
      }
    }
  }
  __syncthreads();
  {
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    const f32x16 a = block_64(X, rb, W2, kH, cb);
    const f32x16 ad = block_64(Xt, rb, W2, kH, cb);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = rb + acc_row(r, lane), col = cb + (lane & 31);
      const float h = siluf(a[r]), hd = silu_grad(a[r]) * ad[r];
      X[row][col] = h;
      Xt[row][col] = hd;
      const int e = e0 + row;
      if (e < E) {
        P2d[(long)e * 128 + col] = a[r];
        P2d[(long)e * 128 + 64 + col] = ad[r];
        H2d[(long)e * 128 + col] = h;
        H2d[(long)e * 128 + 64 + col] = hd;
      }
    }
  }
  __syncthreads();
  for (int cc = w * 32; cc < PC; cc += 128) {
    f32x16 a0 = {}, a1 = {};
#pragma unroll 8
    for (int kk = 0; kk < kH; kk += 2) {
      const float b = W3[(kk + (lane >> 5)) * ld3 + cc + (lane & 31)];
      a0 = mfma32(Xt[lane & 31][kk + (lane >> 5)], b, a0);
      a1 = mfma32(Xt[32 + (lane & 31)][kk + (lane >> 5)], b, a1);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = acc_row(r, lane);
      const int ea = e0 + row, eb = e0 + 32 + row;
      if (ea < E) Rd[(long)ea * PC + cc + (lane & 31)] = a0[r];
      if (eb < E) Rd[(long)eb * PC + cc + (lane & 31)] = a1[r];
    }
  }
}

// Reverse of the tangent pass: from the adjoints of R and R_dot (Rb, Rc) to
// the adjoints of the pre-activations, [P2b | P2c] and [P1b | P1c]:
//   H2b = Rb W3^T, H2c = Rc W3^T
//   P2b = H2b silu'(P2) + H2c silu''(P2) P2_dot,  P2c = H2c silu'(P2)
//   H1b = P2b W2^T, H1c = P2c W2^T
//   P1b = H1b silu'(P1) + H1c silu''(P1) P1_dot,  P1c = H1c silu'(P1)
__global__ void __launch_bounds__(256) k_radial_dual_bwd(const int* __restrict__ row_ptr_x, int N,
                                                         const float* __restrict__ W2T, const float* __restrict__ W3T,
                                                         int PC, const float* __restrict__ Rb,
                                                         const float* __restrict__ Rc, const float* __restrict__ P1d,
                                                         const float* __restrict__ P2d, float* __restrict__ P1g,
                                                         float* __restrict__ P2g) {
  __shared__ float Ds[kTile][33];
  __shared__ float Dc[kTile][33];
  __shared__ float X[kTile][kLd];
  __shared__ float Xc[kTile][kLd];
  const int E = row_ptr_x[N];
  const int e0 = blockIdx.x * kTile;
  if (e0 >= E) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
  f32x16 ab = {}, ac = {};
  for (int kc = 0; kc < PC; kc += 32) {
    __syncthreads();
    {
      const int row = t >> 2, c8 = (t & 3) * 8;
      const int e = e0 + row;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        Ds[row][c8 + q] = e < E ? Rb[(long)e * PC + kc + c8 + q] : 0.0f;
        Dc[row][c8 + q] = e < E ? Rc[(long)e * PC + kc + c8 + q] : 0.0f;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 32; kk += 2) {
      const float b = W3T[(kc + kk + (lane >> 5)) * kH + cb + (lane & 31)];
      ab = mfma32(Ds[rb + (lane & 31)][kk + (lane >> 5)], b, ab);
      ac = mfma32(Dc[rb + (lane & 31)][kk + (lane >> 5)], b, ac);
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = rb + acc_row(r, lane), col = cb + (lane & 31);
    const int e = e0 + row;
    float pb = 0.0f, pc = 0.0f;
    if (e < E) {
      const float x = P2d[(long)e * 128 + col], xd = P2d[(long)e * 128 + 64 + col];
      const float g1 = silu_grad(x);
      pb = ab[r] * g1 + ac[r] * silu_grad2(x) * xd;
      pc = ac[r] * g1;
      P2g[(long)e * 128 + col] = pb;
      P2g[(long)e * 128 + 64 + col] = pc;
    }
    X[row][col] = pb;
    Xc[row][col] = pc;
  }
  __syncthreads();
  const f32x16 hb = block_64(X, rb, W2T, kH, cb);
  const f32x16 hc = block_64(Xc, rb, W2T, kH, cb);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = rb + acc_row(r, lane), col = cb + (lane & 31);
    const int e = e0 + row;
    if (e < E) {
      const float x = P1d[(long)e * 128 + col], xd = P1d[(long)e * 128 + 64 + col];
      const float g1 = silu_grad(x);
      P1g[(long)e * 128 + col] = hb[r] * g1 + hc[r] * silu_grad2(x) * xd;
      P1g[(long)e * 128 + 64 + col] = hc[r] * g1;
    }
  }
}

inline int tiles(long n) { return (int)((n + kTile - 1) / kTile); }



}  // namespace

void launch_radial_fwd(int n_basis, const float4* dvec, const int* row_ptr_x, int N, long e_cap, const float* W1,
                       const float* W2, const float* W3, int ld3, int PC, void* R, bool r_bf16, float rc, int p,
                       bool bf16, hipStream_t st, int e_first, int e_end, const RadialBf16* wb,
                       const EdgePairs* pairs) {
  if (e_cap == 0) return;
  if (n_basis != 8) throw Error(E3MI_EUNSUPPORTED, "n_basis must be 8");
  if (PC % 32) throw Error(E3MI_EUNSUPPORTED, "paths x channels must be a multiple of 32");
  if (r_bf16 && !bf16) throw Error(E3MI_EINVAL, "BF16 radial weights need the BF16 mode");
  if (bf16 && !(wb && wb->W2T && wb->W3T)) throw Error(E3MI_EINVAL, "BF16 mode: BF16 radial weights missing");
  if (pairs && (e_first != 0 || e_end >= 0 || !pairs->own || !pairs->n_own || !pairs->rev))
    throw Error(E3MI_EINVAL, "radial MLP per edge pair: needs the whole edge list and the pair owners");
  const int grid = tiles(e_end >= 0 ? (long)e_end - e_first : e_cap);
  if (grid == 0) return;
  const int mode = pairs ? (pairs->compact ? 2 : 1) : 0;
  const int* own = pairs ? pairs->own : nullptr;
  const int* n_own = pairs ? pairs->n_own : nullptr;
  const int* rev = pairs ? pairs->rev : nullptr;
  auto go = [&](auto mc) {
    constexpr int MODE = decltype(mc)::value;
    if (r_bf16)
      k_radial_fwd<8, true, __bf16, MODE><<<grid, 256, 0, st>>>(dvec, row_ptr_x, N, W1, W2, W3, ld3, PC,
                                                                static_cast<__bf16*>(R), rc, p, e_first, e_end,
                                                                wb->W2T, wb->W3T, own, n_own, rev);
    else if (bf16)
      k_radial_fwd<8, true, float, MODE><<<grid, 256, 0, st>>>(dvec, row_ptr_x, N, W1, W2, W3, ld3, PC,
                                                               static_cast<float*>(R), rc, p, e_first, e_end,
                                                               wb->W2T, wb->W3T, own, n_own, rev);
    else
      k_radial_fwd<8, false, float, MODE><<<grid, 256, 0, st>>>(dvec, row_ptr_x, N, W1, W2, W3, ld3, PC,
                                                                static_cast<float*>(R), rc, p, e_first, e_end,
                                                                nullptr, nullptr, own, n_own, rev);
  };
  if (mode == 0) go(std::integral_constant<int, 0>{});
  else if (mode == 1) go(std::integral_constant<int, 1>{});
  else go(std::integral_constant<int, 2>{});
}

template <int LMAX>
static void radial_bwd_l(bool bf16, bool r_bf16, long e_cap, const float4* dvec, const int* row_ptr_x, int N,
                         const float* W1, const float* W2, const float* W2T, const float* W3T, int PC, const void* dR,
                         const float* dY, float4* g, int accumulate, float rc, int p, hipStream_t st, int e_first,
                         int e_end, const RadialBf16* wb, const int* own, const int* n_own, const int* rev) {
  const int grid = tiles(e_end >= 0 ? (long)e_end - e_first : e_cap);
  if (grid == 0) return;
  auto go = [&](auto pc) {
    constexpr bool PAIR = decltype(pc)::value;
    if (r_bf16)
      k_radial_bwd<8, LMAX, true, __bf16, PAIR><<<grid, 256, 0, st>>>(
          dvec, row_ptr_x, N, W1, W2, W2T, W3T, PC, static_cast<const __bf16*>(dR), dY, g, accumulate, rc, p,
          e_first, e_end, wb->W2T, wb->W2, wb->W3u, own, n_own, rev);
    else if (bf16)
      k_radial_bwd<8, LMAX, true, float, PAIR><<<grid, 256, 0, st>>>(
          dvec, row_ptr_x, N, W1, W2, W2T, W3T, PC, static_cast<const float*>(dR), dY, g, accumulate, rc, p,
          e_first, e_end, wb->W2T, wb->W2, wb->W3u, own, n_own, rev);
    else
      k_radial_bwd<8, LMAX, false, float, PAIR><<<grid, 256, 0, st>>>(
          dvec, row_ptr_x, N, W1, W2, W2T, W3T, PC, static_cast<const float*>(dR), dY, g, accumulate, rc, p,
          e_first, e_end, nullptr, nullptr, nullptr, own, n_own, rev);
  };
  if (own) go(std::true_type{});
  else go(std::false_type{});
}

void launch_radial_bwd(int n_basis, int lmax, const float4* dvec, const int* row_ptr_x, int N, long e_cap,
                       const float* W1, const float* W2, const float* W2T, const float* W3T, int PC, const void* dR,
                       bool r_bf16, const float* dY, float4* g, int accumulate, float rc, int p, bool bf16,
                       hipStream_t st, int e_first, int e_end, const RadialBf16* wb, const EdgePairs* pairs) {
  if (e_cap == 0) return;
  if (n_basis != 8) throw Error(E3MI_EUNSUPPORTED, "n_basis must be 8");
  if (r_bf16 && !bf16) throw Error(E3MI_EINVAL, "BF16 radial weights need the BF16 mode");
  if (bf16 && !(wb && wb->W2T && wb->W2 && wb->W3u))
    throw Error(E3MI_EINVAL, "BF16 mode: BF16 radial weights missing");
  if (pairs && (e_first != 0 || e_end >= 0 || !pairs->own || !pairs->n_own || !pairs->rev))
    throw Error(E3MI_EINVAL, "radial adjoint per edge pair: needs the whole edge list and the pair owners");
  const int* own = pairs ? pairs->own : nullptr;
  const int* n_own = pairs ? pairs->n_own : nullptr;
  const int* rev = pairs ? pairs->rev : nullptr;
  if (lmax == 3)
    radial_bwd_l<3>(bf16, r_bf16, e_cap, dvec, row_ptr_x, N, W1, W2, W2T, W3T, PC, dR, dY, g, accumulate, rc, p, st,
                    e_first, e_end, wb, own, n_own, rev);
  else if (lmax == 2)
    radial_bwd_l<2>(bf16, r_bf16, e_cap, dvec, row_ptr_x, N, W1, W2, W2T, W3T, PC, dR, dY, g, accumulate, rc, p, st,
                    e_first, e_end, wb, own, n_own, rev);
  else
    throw Error(E3MI_EUNSUPPORTED, "lmax must be 2 or 3");
}

}  // namespace e3mi

namespace e3mi {
void launch_radial_dual_fwd(int n_basis, const float4* dvec, const float4* dd, const int* row_ptr_x, int N, long e_cap,
                            const float* W1, const float* W2, const float* W3, int ld3, int PC, float* Rd, float* Bd,
                            float* P1d, float* H1d, float* P2d, float* H2d, float rc, int p, hipStream_t st) {
  if (e_cap == 0) return;
  if (n_basis != 8) throw Error(E3MI_EUNSUPPORTED, "n_basis must be 8");
  k_radial_dual_fwd<8><<<tiles(e_cap), 256, 0, st>>>(dvec, dd, row_ptr_x, N, W1, W2, W3, ld3, PC, Rd, Bd, P1d, H1d,
                                                     P2d, H2d, rc, p);
}
void launch_radial_dual_bwd(const int* row_ptr_x, int N, long e_cap, const float* W2T, const float* W3T, int PC,
                            const float* Rb, const float* Rc, const float* P1d, const float* P2d, float* P1g,
                            float* P2g, hipStream_t st) {
  if (e_cap == 0) return;
  k_radial_dual_bwd<<<tiles(e_cap), 256, 0, st>>>(row_ptr_x, N, W2T, W3T, PC, Rb, Rc, P1d, P2d, P1g, P2g);
}
}  // namespace e3mi
