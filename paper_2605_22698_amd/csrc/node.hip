// Per-atom stages of the interaction:
//   channel mix + self connection (dense contractions on the FP32 matrix cores)
//     h~[l3] = A[l3] W[l3] + h[l3] S[l3]        rows (atom, m), columns channels
//   gate (MACE table of Appendix F: gate_nodes):
//     h[0] = silu(h~[0]),  h[l>0] = h~[l] sigmoid(h~[0])
//   embedding h0 = W_emb[z];  readout E_i = w2 . silu(W_r^T h[0]) + E0[z_i]
//   (Section 5.3 readout with one head), fused with its adjoint dE/dh[0]
//   energy reduction per structure in FP64, fixed summation order
//   force assembly F_i = sum_{e in in(i)} (g_e - g_rev(e))
#include "common.h"
#include "runtime.h"

namespace e3mi {

namespace {

__device__ __forceinline__ long row_off(const RowMap& m, int r) {
  return (long)(r / m.g) * m.s_atom + (long)(r % m.g) * m.s_m;
}
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// 64x64 output tile per workgroup, each wave a 32x32 block on
// v_mfma_f32_32x32x2f32 (FP32), or with both operands rounded to BF16 on
// v_mfma_f32_32x32x16_bf16 (BF), FP32 accumulation. K runs over the two
// operand pairs in slabs of 32 staged through LDS; the next slab is fetched
// into registers while the current one is multiplied.
constexpr int kSlab = 32;
constexpr int kPer = kSlab / 16;  // float4 of each operand per thread and slab
constexpr int kRowQ = kSlab / 4;  // float4 per row of an A slab

struct Slab {
  float4 a[kPer], b[kPer];
};

// Slab s of the K loop (products 0 then 1) into registers: A through the row
// pointers of the rows this thread stages (null past M), B row-major.
__device__ __forceinline__ void gemm_load_slab(const GemmArgs& a, const float* const* ap0, const float* const* ap1,
                                               int s, int s0, int bn, Slab& r) {
  const int t = threadIdx.x;
  const int op = s >= s0;
  const float* __restrict__ B = op ? a.b1 : a.b0;
  const int ldb = op ? a.ldb1 : a.ldb0;
  const int K = op ? a.k1 : a.k0;
  const int k0 = (op ? s - s0 : s) * kSlab;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int idx = t + 256 * i;
    const int kq = (idx % kRowQ) * 4;
    const float* p = op ? ap1[i] : ap0[i];
    r.a[i] = (p && k0 + kq < K) ? *reinterpret_cast<const float4*>(p + k0 + kq) : make_float4(0.f, 0.f, 0.f, 0.f);
    const int kr = idx >> 4, c4 = (idx & 15) * 4, gk = k0 + kr, gc = bn + c4;
    r.b[i] = (gk < K && gc < a.Nc) ? *reinterpret_cast<const float4*>(B + (long)gk * ldb + gc)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// Independent products of one group share a launch: workgroup b (after the
// XCD-contiguous remapping, so that the column blocks of a row tile and
// neighbouring row tiles meet in one L2) takes tile b - tile0[k] of product k,
// column blocks fastest.
struct GemmGroup {
  GemmArgs g[kMaxGemmGroup];
  int tile0[kMaxGemmGroup + 1];
  int ncb[kMaxGemmGroup];
  int n;
};

template <bool BF>
__global__ void __launch_bounds__(256) k_gemm(GemmGroup gg) {
  __shared__ float As[64][kSlab + 1];
  __shared__ float Bs[kSlab][65];
  __shared__ long coff[64];  // offsets of the tile's output rows (-1 past M)
  const int b = xcd_contiguous(blockIdx.x, gridDim.x);
  int gi = 0;
  while (gi + 1 < gg.n && b >= gg.tile0[gi + 1]) ++gi;
  const GemmArgs& a = gg.g[gi];
  const int local = b - gg.tile0[gi];
  const int bm = (local / gg.ncb[gi]) * 64, bn = (local % gg.ncb[gi]) * 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
  const int s0 = (a.k0 + kSlab - 1) / kSlab, ns = s0 + (a.k1 + kSlab - 1) / kSlab;
  // row offsets (a division by the rows per atom each) once per tile, not per slab
  if (t < 64) {
    const int r = bm + t;
    coff[t] = r < a.M ? row_off(a.c, r) : -1;
  }
  const float* ap0[kPer];
  const float* ap1[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int gr = bm + (t + 256 * i) / kRowQ;
    const bool in = gr < a.M;
    ap0[i] = in ? a.a0.base + row_off(a.a0, gr) : nullptr;
    ap1[i] = (in && a.k1 > 0) ? a.a1.base + row_off(a.a1, gr) : nullptr;
  }
  f32x16 acc = {};
  Slab cur;
  if (ns > 0) gemm_load_slab(a, ap0, ap1, 0, s0, bn, cur);
  else __syncthreads();
  for (int s = 0; s < ns; ++s) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int idx = t + 256 * i;
      const int row = idx / kRowQ, kq = (idx % kRowQ) * 4;
      As[row][kq] = cur.a[i].x;
      As[row][kq + 1] = cur.a[i].y;
      As[row][kq + 2] = cur.a[i].z;
      As[row][kq + 3] = cur.a[i].w;
      const int kr = idx >> 4, c4 = (idx & 15) * 4;
      Bs[kr][c4] = cur.b[i].x;
      Bs[kr][c4 + 1] = cur.b[i].y;
      Bs[kr][c4 + 2] = cur.b[i].z;
      Bs[kr][c4 + 3] = cur.b[i].w;
    }
    __syncthreads();
    if (s + 1 < ns) gemm_load_slab(a, ap0, ap1, s + 1, s0, bn, cur);
    if constexpr (BF) {
#pragma unroll
      for (int kb = 0; kb < kSlab; kb += 16) {
        const int k0 = kb + 8 * (lane >> 5);
        bf16x8 x, y;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          x[q] = (__bf16)As[rb + (lane & 31)][k0 + q];
          y[q] = (__bf16)Bs[k0 + q][cb + (lane & 31)];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < kSlab; kk += 2)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[rb + (lane & 31)][kk + (lane >> 5)],
                                                    Bs[kk + (lane >> 5)][cb + (lane & 31)], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = bn + cb + (lane & 31);
  if (col < a.Nc) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long o = coff[rb + acc_row(r, lane)];
      if (o >= 0) {
        float* p = a.c.base + o + col;
        *p = a.accumulate ? *p + acc[r] : acc[r];
      }
    }
  }
}

__global__ void k_gate_fwd(const float* __restrict__ ht, float* __restrict__ h, int N, int nc, int C) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)N * C) return;
  const long i = idx / C;
  const int k = (int)(idx % C);
  const float* src = ht + i * nc * C + k;
  float* dst = h + i * nc * C + k;
  const float s0 = src[0];
  const float s = sigmoidf(s0);
  dst[0] = s0 * s;
  for (int c = 1; c < nc; ++c) dst[(long)c * C] = src[(long)c * C] * s;
}

// Scalar-only layer whose channel mix was split over K: h~ = the sum of the
// partial products in order, then h = silu(h~).
__global__ void k_gate_fwd_sum(const float* __restrict__ part, int n_parts, float* __restrict__ ht,
                               float* __restrict__ h, long NC) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NC) return;
  float s0 = part[idx];
  for (int p = 1; p < n_parts; ++p) s0 += part[p * NC + idx];
  ht[idx] = s0;
  h[idx] = s0 * sigmoidf(s0);
}

__global__ void k_gate_bwd(const float* __restrict__ ht, const float* __restrict__ dh, float* __restrict__ dht,
                           int N, int nc, int C) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)N * C) return;
  const long i = idx / C;
  const int k = (int)(idx % C);
  const float* x = ht + i * nc * C + k;
  const float* g = dh + i * nc * C + k;
  float* o = dht + i * nc * C + k;
  const float s0 = x[0];
  const float s = sigmoidf(s0);
  float acc = 0.0f;
  for (int c = 1; c < nc; ++c) {
    acc += g[(long)c * C] * x[(long)c * C];
    o[(long)c * C] = g[(long)c * C] * s;
  }
  o[0] = g[0] * silu_grad(s0) + acc * s * (1.0f - s);
}

__global__ void k_embed(const int* __restrict__ species, const float* __restrict__ emb, float* __restrict__ h0, int N,
                        int C) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)N * C) return;
  const long i = idx / C;
  const int k = (int)(idx % C);
  h0[idx] = emb[(long)species[i] * C + k];
}

// One wave per atom; readout_hidden = 16.
__global__ void __launch_bounds__(256) k_readout(const float* __restrict__ h, int nc, const int* __restrict__ species,
                                                 const float* __restrict__ Wr, const float* __restrict__ w2,
                                                 const float* __restrict__ e0, int N, int C,
                                                 double* __restrict__ e_atom, float* __restrict__ dh,
                                                 const float* __restrict__ wq, const float* __restrict__ bq,
                                                 float* __restrict__ q_raw) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const float* hi = h + (long)i * nc * C;
  float pre[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) pre[q] = 0.0f;
  float qa = 0.0f;
  for (int k = lane; k < C; k += 64) {
    const float x = hi[k];
#pragma unroll
    for (int q = 0; q < 16; ++q) pre[q] += x * Wr[k * 16 + q];
    if (wq) qa += x * wq[k];
  }
  if (wq) {
    qa = wave_sum(qa);
    if (lane == 0) q_raw[i] = qa + bq[species[i]];
  }
  float e = 0.0f;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    pre[q] = wave_sum(pre[q]);
    e += w2[q] * siluf(pre[q]);
  }
  if (lane == 0) e_atom[i] = (double)e + (double)e0[species[i]];
  float gq[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) gq[q] = w2[q] * silu_grad(pre[q]);
  for (int k = lane; k < C; k += 64) {
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += Wr[k * 16 + q] * gq[q];
    dh[(long)i * C + k] = s;
  }
}

// Readout of a scalar-only last layer straight from its pre-gate values x (the
// sum of n_parts partial products [n_parts, N, C], or h~ itself when n_parts
// is 0), with the gate and its adjoint folded in: h = silu(x),
// E_i = w2 . silu(W_r^T h) + E0[z_i], dh~ = (W_r g) o silu'(x).
__global__ void __launch_bounds__(256) k_readout_gated(const float* __restrict__ xt, int n_parts,
                                                       const int* __restrict__ species, const float* __restrict__ Wr,
                                                       const float* __restrict__ w2, const float* __restrict__ e0,
                                                       int N, int C, double* __restrict__ e_atom,
                                                       float* __restrict__ dht) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const long NC = (long)N * C;
  auto x_of = [&](int k) {
    float x = xt[(long)i * C + k];
    for (int p = 1; p < n_parts; ++p) x += xt[p * NC + (long)i * C + k];
    return x;
  };
  float pre[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) pre[q] = 0.0f;
  for (int k = lane; k < C; k += 64) {
    const float x = x_of(k);
    const float hv = x * sigmoidf(x);
#pragma unroll
    for (int q = 0; q < 16; ++q) pre[q] += hv * Wr[k * 16 + q];
  }
  // lane L holds the pre-activation of hidden unit L / 4
  const float pq = wave_sum_scatter16<16>(pre);
  const int q0 = lane >> 2;
  float e = (lane & 3) == 0 ? w2[q0] * siluf(pq) : 0.0f;
#pragma unroll
  for (int off = 4; off < 64; off <<= 1) e += __shfl_xor(e, off);
  if (lane == 0) e_atom[i] = (double)e + (double)e0[species[i]];
  const float gl = w2[q0] * silu_grad(pq);
  float gq[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) gq[q] = __shfl(gl, 4 * q);
  for (int k = lane; k < C; k += 64) {
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += Wr[k * 16 + q] * gq[q];
    dht[(long)i * C + k] = s * silu_grad(x_of(k));
  }
}

__global__ void __launch_bounds__(256) k_energy(const double* __restrict__ e_atom, const int64_t* __restrict__ off,
                                                double* __restrict__ energy) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  const int64_t a = off[s], b = off[s + 1];
  double acc = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) acc += e_atom[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) energy[s] = red[0];
}

// One wave per atom: the lanes take the row's edges in turn, then a fixed
// reduction tree over the wave (bitwise repeatable).
__global__ void __launch_bounds__(256) k_forces(const int* __restrict__ row_ptr, const int* __restrict__ rev,
                                                const float4* __restrict__ g, int N, const float* __restrict__ extra,
                                                float* __restrict__ F) {
  const int i = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int b = row_ptr[i + 1];
  for (int e = row_ptr[i] + lane; e < b; e += 64) {
    const int re = rev[e];
    const float4 a = g[e];
    const float4 r = re >= 0 ? g[re] : make_float4(0.f, 0.f, 0.f, 0.f);
    fx += a.x - r.x;
    fy += a.y - r.y;
    fz += a.z - r.z;
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  if (extra) {
    fx += extra[3 * i];
    fy += extra[3 * i + 1];
    fz += extra[3 * i + 2];
  }
  if (lane == 0) {
    F[3 * i] = fx;
    F[3 * i + 1] = fy;
    F[3 * i + 2] = fz;
  }
}

inline int blocks(long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_gemm(const GemmArgs& a, hipStream_t st, bool bf16) { launch_gemm_group(&a, 1, st, bf16); }

void launch_gemm_group(const GemmArgs* a, int n, hipStream_t st, bool bf16) {
  if (n < 1 || n > kMaxGemmGroup) throw Error(E3MI_EINVAL, "GEMM group size out of range");
  GemmGroup gg{};
  int tiles = 0, m = 0;
  for (int k = 0; k < n; ++k) {
    if (a[k].M == 0 || a[k].Nc == 0) continue;
    if ((a[k].k0 % 4) || (a[k].k1 % 4) || (a[k].Nc % 4) || (a[k].ldb0 % 4) || (a[k].k1 && (a[k].ldb1 % 4)))
      throw Error(E3MI_EUNSUPPORTED, "GEMM dimensions must be multiples of 4");
    gg.g[m] = a[k];
    gg.tile0[m] = tiles;
    gg.ncb[m] = (int)blocks(a[k].Nc, 64);
    tiles += (int)blocks(a[k].M, 64) * gg.ncb[m];
    ++m;
  }
  if (m == 0) return;
  gg.tile0[m] = tiles;
  gg.n = m;
  if (bf16)
    k_gemm<true><<<tiles, 256, 0, st>>>(gg);
  else
    k_gemm<false><<<tiles, 256, 0, st>>>(gg);
}
void launch_gate_fwd(const float* ht, float* h, int N, int nc, int C, hipStream_t st) {
  if (N == 0) return;
  k_gate_fwd<<<blocks((long)N * C, 256), 256, 0, st>>>(ht, h, N, nc, C);
}
void launch_gate_fwd_sum(const float* part, int n_parts, float* ht, float* h, int N, int C, hipStream_t st) {
  if (N == 0) return;
  k_gate_fwd_sum<<<blocks((long)N * C, 256), 256, 0, st>>>(part, n_parts, ht, h, (long)N * C);
}
void launch_gate_bwd(const float* ht, const float* dh, float* dht, int N, int nc, int C, hipStream_t st) {
  if (N == 0) return;
  k_gate_bwd<<<blocks((long)N * C, 256), 256, 0, st>>>(ht, dh, dht, N, nc, C);
}
void launch_embed(const int* species, const float* emb, float* h0, int N, int C, hipStream_t st) {
  if (N == 0) return;
  k_embed<<<blocks((long)N * C, 256), 256, 0, st>>>(species, emb, h0, N, C);
}
void launch_readout(const float* h, int nc, const int* species, const float* Wr, const float* w2, const float* e0,
                    int N, int C, double* e_atom, float* dh, hipStream_t st, const float* wq, const float* bq,
                    float* q_raw) {
  if (N == 0) return;
  k_readout<<<blocks((long)N * 64, 256), 256, 0, st>>>(h, nc, species, Wr, w2, e0, N, C, e_atom, dh, wq, bq, q_raw);
}
void launch_readout_gated(const float* xt, int n_parts, const int* species, const float* Wr, const float* w2,
                          const float* e0, int N, int C, double* e_atom, float* dht, hipStream_t st) {
  if (N == 0) return;
  k_readout_gated<<<blocks((long)N * 64, 256), 256, 0, st>>>(xt, n_parts, species, Wr, w2, e0, N, C, e_atom, dht);
}
void launch_energy(const double* e_atom, const int64_t* off, int S, double* energy, hipStream_t st) {
  k_energy<<<S, 256, 0, st>>>(e_atom, off, energy);
}
void launch_forces(const int* row_ptr, const int* rev, const float4* g, int N, float* F, hipStream_t st,
                   const float* extra) {
  if (N == 0) return;
  k_forces<<<blocks((long)N * 64, 256), 256, 0, st>>>(row_ptr, rev, g, N, extra, F);
}

}  // namespace e3mi
