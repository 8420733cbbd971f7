// Parameter gradients of a loss that depends on energies and forces.
//
// For upstream gradients gE (per structure) and gF (per atom), the gradient
// with respect to the weights theta is
//   dL/dtheta = d/dtheta [ sum_s gE_s E_s  -  D_v E ],   v = gF,
// where D_v E = sum_i v_i . dE/dr_i is the change of E when the atoms move
// along v (forces are -dE/dr; the paper trains on force labels and, in §5.2,
// on Hessian rows obtained by differentiating forces). D_v E is computed by a
// tangent (forward-mode) pass through the interaction and the whole scalar by
// a reverse pass over both the primal and the tangent values. This file holds
// the per-atom and per-edge kernels of those passes that are not tensor
// products or radial MLPs, and the reductions over edges and atoms that give
// the weight gradients, in a fixed order (no atomics).
#include <algorithm>

#include "common.h"
#include "runtime.h"

namespace e3mi {
namespace {

inline int blocks(long n, int t) { return (int)((n + t - 1) / t); }

// d_dot = v_j - v_i for edge e = (i <- j); r_dot = n . d_dot. One wave per row.
__global__ void __launch_bounds__(256) k_edge_tangent(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                      const float4* __restrict__ dvec, const float* __restrict__ v,
                                                      int N, float4* __restrict__ dd) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const float vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
  const int b = row_ptr[i + 1];
  for (int e = row_ptr[i] + lane; e < b; e += 64) {
    const int j = src[e];
    const float4 d = dvec[e];
    const float x = v[3 * j] - vx, y = v[3 * j + 1] - vy, z = v[3 * j + 2] - vz;
    dd[e] = make_float4(x, y, z, (d.x * x + d.y * y + d.z * z) / d.w);
  }
}

// h_dot = gate'(h~) h~_dot
__global__ void k_gate_dual_fwd(const float* __restrict__ x, const float* __restrict__ xd, float* __restrict__ hd,
                                int N, int nc, int C) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)N * C) return;
  const long base = (idx / C) * nc * C + idx % C;
  const float x0 = x[base], xd0 = xd[base];
  const float s = sigmoidf(x0), s1 = s * (1.0f - s);
  hd[base] = silu_grad(x0) * xd0;
  for (int c = 1; c < nc; ++c) {
    const long o = base + (long)c * C;
    hd[o] = xd[o] * s + x[o] * s1 * xd0;
  }
}

// Reverse of (h, h_dot) = gate(h~), gate'(h~) h~_dot:
//   xc_l = hc_l s                       xc_0 = hc_0 silu'(x0) + sum_l hc_l x_l s'
//   xb_l = hb_l s + hc_l s' xd0          xb_0 = hb_0 silu'(x0) + hc_0 silu''(x0) xd0
//                                              + sum_l [hb_l x_l s' + hc_l (xd_l s' + x_l s'' xd0)]
__global__ void k_gate_dual_bwd(const float* __restrict__ x, const float* __restrict__ xd, const float* __restrict__ hb,
                                const float* __restrict__ hc, float* __restrict__ xb, float* __restrict__ xc, int N,
                                int nc, int C) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)N * C) return;
  const long base = (idx / C) * nc * C + idx % C;
  const float x0 = x[base], xd0 = xd[base];
  const float s = sigmoidf(x0), s1 = s * (1.0f - s), s2 = s1 * (1.0f - 2.0f * s);
  float b0 = hb[base] * silu_grad(x0) + hc[base] * silu_grad2(x0) * xd0;
  float c0 = hc[base] * silu_grad(x0);
  for (int c = 1; c < nc; ++c) {
    const long o = base + (long)c * C;
    const float xl = x[o], xdl = xd[o], hbl = hb[o], hcl = hc[o];
    xc[o] = hcl * s;
    xb[o] = hbl * s + hcl * s1 * xd0;
    c0 += hcl * xl * s1;
    b0 += hbl * xl * s1 + hcl * (xdl * s1 + xl * s2 * xd0);
  }
  xb[base] = b0;
  xc[base] = c0;
}

// Readout E_i = w2 . silu(P), P = h0 W_r, with tangent E_dot_i = w2 . (silu'(P) P_dot),
// P_dot = h0_dot W_r, reversed for the scalar sum_i [gE_{s(i)} E_i - E_dot_i].
// One wave per atom. Writes the adjoints of P and P_dot ([N,16] each), the
// per-atom terms of the w2 gradient ([N,16]), the adjoints of h0 and h0_dot
// ([N, nc, C], component 0) and gE_{s(i)} per atom (for the E0 gradient).
__global__ void __launch_bounds__(256) k_readout_dual(const float* __restrict__ h, const float* __restrict__ hd, int nc,
                                                      const int* __restrict__ owner, const double* __restrict__ gE,
                                                      const float* __restrict__ Wr, const float* __restrict__ w2,
                                                      int N, int C, float* __restrict__ Pb, float* __restrict__ Pc,
                                                      float* __restrict__ w2c, float* __restrict__ hb,
                                                      float* __restrict__ hc, float* __restrict__ eb) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  float P[16], Pd[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) P[q] = Pd[q] = 0.0f;
  for (int k = lane; k < C; k += 64) {
    const float a = h[(long)i * nc * C + k], ad = hd[(long)i * nc * C + k];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      P[q] += a * Wr[k * 16 + q];
      Pd[q] += ad * Wr[k * 16 + q];
    }
  }
  const float Eb = (float)gE[owner[i]];
  const float Ec = -1.0f;
  float pb[16], pc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    P[q] = wave_sum(P[q]);
    Pd[q] = wave_sum(Pd[q]);
    const float s1 = silu_grad(P[q]), s2 = silu_grad2(P[q]);
    pc[q] = Ec * w2[q] * s1;
    pb[q] = Eb * w2[q] * s1 + Ec * w2[q] * s2 * Pd[q];
    if (lane == q) {
      Pb[(long)i * 16 + q] = pb[q];
      Pc[(long)i * 16 + q] = pc[q];
      w2c[(long)i * 16 + q] = Eb * siluf(P[q]) + Ec * s1 * Pd[q];
    }
  }
  if (lane == 0) eb[i] = Eb;
  for (int k = lane; k < C; k += 64) {
    float sb = 0.0f, sc = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      sb += Wr[k * 16 + q] * pb[q];
      sc += Wr[k * 16 + q] * pc[q];
    }
    hb[(long)i * nc * C + k] = sb;
    hc[(long)i * nc * C + k] = sc;
  }
}

// out[g, c] = sum over atoms i with species[i] == g (all atoms when species is
// NULL) of X[i * ld + c], in atom order, accumulated in FP64.
__global__ void k_group_sum(const float* __restrict__ X, long ld, const int* __restrict__ species, int n_groups, int N,
                            int ncols, double* __restrict__ out, long ld_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_groups * ncols) return;
  const int g = t / ncols, c = t % ncols;
  double acc = 0.0;
  for (int i = 0; i < N; ++i)
    if (!species || species[i] == g) acc += (double)X[(long)i * ld + c];
  out[(long)g * ld_out + c] = acc;
}

// Partial sums over a chunk of rows of X1^T Y1 + X2^T Y2 (X: [rows, mo],
// Y: [rows, no], rows addressed through RowMaps), 64x64 output tiles on the
// FP32 matrix cores; grid.z enumerates the row chunks.
__global__ void __launch_bounds__(256) k_gemm_tn(RowMap x1, RowMap y1, RowMap x2, RowMap y2, int rows,
                                                 const int* __restrict__ rows_dev, int mo, int no, int chunk_rows,
                                                 float* __restrict__ partial) {
  __shared__ float Xs[16][65];
  __shared__ float Ys[16][65];
  int R = rows;
  if (rows_dev) R = min(R, *rows_dev);
  const int bm = blockIdx.x * 64, bn = blockIdx.y * 64;
  const int r0 = blockIdx.z * chunk_rows, r1 = min(R, r0 + chunk_rows);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
  f32x16 acc = {};
  for (int term = 0; term < 2; ++term) {
    const RowMap X = term ? x2 : x1, Y = term ? y2 : y1;
    if (!X.base) continue;
    for (int r = r0; r < r1; r += 16) {
      {
        const int kr = t >> 4, c4 = (t & 15) * 4;
        const int gr = r + kr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int cm = bm + c4 + q, cn = bn + c4 + q;
          float xv = 0.0f, yv = 0.0f;
          if (gr < r1) {
            const long ro_x = (long)(gr / X.g) * X.s_atom + (long)(gr % X.g) * X.s_m;
            const long ro_y = (long)(gr / Y.g) * Y.s_atom + (long)(gr % Y.g) * Y.s_m;
            if (cm < mo) xv = X.base[ro_x + cm];
            if (cn < no) yv = Y.base[ro_y + cn];
          }
          Xs[kr][c4 + q] = xv;
          Ys[kr][c4 + q] = yv;
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; kk += 2)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(Xs[kk + (lane >> 5)][rb + (lane & 31)],
                                                    Ys[kk + (lane >> 5)][cb + (lane & 31)], acc, 0, 0, 0);
      __syncthreads();
    }
  }
  float* P = partial + (long)blockIdx.z * mo * no;
  const int col = bn + cb + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = bm + rb + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row < mo && col < no) P[(long)row * no + col] = acc[r];
  }
}

// out[i * ld_out + j] = sum over chunks of partial[c][i][j], chunks in order, FP64.
__global__ void k_reduce_partials(const float* __restrict__ partial, int chunks, int mo, int no,
                                  double* __restrict__ out, long ld_out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)mo * no) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += (double)partial[(long)c * mo * no + idx];
  out[(idx / no) * ld_out + idx % no] = s;
}

// Bessel x envelope basis with its first and second radial derivatives
// (r inside the cutoff).
template <int NB>
__device__ __forceinline__ void radial_basis_d2(float r, float rc, int p, float* B, float* dB, float* d2B) {
  const float x = r / rc;
  float xp2 = 1.0f;  // x^(p-2)
  for (int k = 0; k < p - 2; ++k) xp2 *= x;
  const float xp1 = xp2 * x, xp = xp1 * x;
  const float fp = (float)p, c3 = 0.5f * fp * (fp + 1.0f) * (fp + 2.0f);
  const float u = 1.0f - 0.5f * (fp + 1.0f) * (fp + 2.0f) * xp + fp * (fp + 2.0f) * xp * x -
                  0.5f * fp * (fp + 1.0f) * xp * x * x;
  const float om = 1.0f - x;
  const float du = -c3 * xp1 * om * om / rc;
  const float d2u = -c3 * ((fp - 1.0f) * xp2 * om * om - 2.0f * xp1 * om) / (rc * rc);
  const float pref = sqrtf(2.0f / rc);
  const float ir = 1.0f / r;
  const float w = 3.14159265358979f / rc;
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    const float kk = (n + 1) * w;
    float s, c;
    sincosf(kk * r, &s, &c);
    const float b = pref * s * ir;
    const float b1 = pref * (kk * c * ir - s * ir * ir);
    const float b2 = pref * (-kk * kk * s * ir - 2.0f * kk * c * ir * ir + 2.0f * s * ir * ir * ir);
    B[n] = b * u;
    dB[n] = b1 * u + b * du;
    d2B[n] = b2 * u + 2.0f * b1 * du + b * d2u;
  }
}

// Per-edge position adjoint of the second-order scalar s (the Hessian-vector
// pass: s = -D_v E) through the edge geometry of one layer. With n = d/r,
// the tangent d_dot, r_dot = n . d_dot, P = I - n n^T and u = P d_dot / r:
//   harmonics  Y = P_c(n), Y_dot = grad P_c(n) . u, adjoints Yb, Yc:
//     g += P G1 / r + P (H u) / r - r_dot/r^2 P G2 - (G2 . n)/r^2 P d_dot - (G2 . P d_dot)/r^2 n
//     G1 = sum Yb grad P, G2 = sum Yc grad P, H = sum Yc hess P
//   basis      B(r), B_dot = B'(r) r_dot, adjoints Bb = W1 P1b, Bc = W1 P1c:
//     g += (Bb . B' + r_dot Bc . B'') n + (Bc . B') P d_dot / r
// One thread per edge; g accumulates over the layers.
template <int LMAX>
__global__ void __launch_bounds__(256) k_hvp_geo(const int* __restrict__ row_ptr_x, int N,
                                                 const float4* __restrict__ dvec, const float4* __restrict__ dd,
                                                 const float* __restrict__ Yb, const float* __restrict__ Yc,
                                                 const float* __restrict__ P1g, const float* __restrict__ W1,
                                                 float rc, int p, int accumulate, float4* __restrict__ g) {
  __shared__ float w1s[8 * 64];
  for (int q = threadIdx.x; q < 8 * 64; q += blockDim.x) w1s[q] = W1[q];
  __syncthreads();
  const int E = row_ptr_x[N];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  constexpr int NY = (LMAX + 1) * (LMAX + 1);
  const float4 d = dvec[e], t = dd[e];
  const float r = d.w, ir = 1.0f / r;
  const float nx = d.x * ir, ny = d.y * ir, nz = d.z * ir;
  const float rd = t.w;
  const float px = t.x - nx * rd, py = t.y - ny * rd, pz = t.z - nz * rd;  // P d_dot
  float yb[NY], yc[NY];
#pragma unroll
  for (int q = 0; q < NY; ++q) {
    yb[q] = Yb[(long)e * 16 + q];
    yc[q] = Yc[(long)e * 16 + q];
  }
  float g1x, g1y, g1z, g2x, g2y, g2z, hx, hy, hz;
  real_sh_vjp<LMAX>(nx, ny, nz, yb, g1x, g1y, g1z);
  real_sh_vjp<LMAX>(nx, ny, nz, yc, g2x, g2y, g2z);
  real_sh_vjp_jvp<LMAX>(nx, ny, nz, px * ir, py * ir, pz * ir, yc, hx, hy, hz);
  // P applied to (G1 + H u) / r - r_dot / r^2 G2
  const float ax = (g1x + hx) * ir - rd * ir * ir * g2x;
  const float ay = (g1y + hy) * ir - rd * ir * ir * g2y;
  const float az = (g1z + hz) * ir - rd * ir * ir * g2z;
  const float an = ax * nx + ay * ny + az * nz;
  const float g2n = g2x * nx + g2y * ny + g2z * nz;
  const float g2p = g2x * px + g2y * py + g2z * pz;
  float gx = ax - an * nx - g2n * ir * ir * px - g2p * ir * ir * nx;
  float gy = ay - an * ny - g2n * ir * ir * py - g2p * ir * ir * ny;
  float gz = az - an * nz - g2n * ir * ir * pz - g2p * ir * ir * nz;
  // radial basis
  float B[8], dB[8], d2B[8];
  radial_basis_d2<8>(r, rc, p, B, dB, d2B);
  const float* pb = P1g + (long)e * 128;
  float sr = 0.0f, sd = 0.0f;  // coefficients of n and of P d_dot / r
  for (int n = 0; n < 8; ++n) {
    float bb = 0.0f, bc = 0.0f;
#pragma unroll 8
    for (int q = 0; q < 64; ++q) {
      bb += w1s[n * 64 + q] * pb[q];
      bc += w1s[n * 64 + q] * pb[64 + q];
    }
    sr += bb * dB[n] + rd * bc * d2B[n];
    sd += bc * dB[n];
  }
  gx += sr * nx + sd * px * ir;
  gy += sr * ny + sd * py * ir;
  gz += sr * nz + sd * pz * ir;
  if (accumulate) {
    const float4 o = g[e];
    gx += o.x;
    gy += o.y;
    gz += o.z;
  }
  g[e] = make_float4(gx, gy, gz, 0.0f);
}

}  // namespace

void launch_edge_tangent(const int* row_ptr, const int* src, const float4* dvec, const float* v, int N, float4* dd,
                         hipStream_t st) {
  if (N == 0) return;
  k_edge_tangent<<<blocks((long)N * 64, 256), 256, 0, st>>>(row_ptr, src, dvec, v, N, dd);
}
void launch_gate_dual_fwd(const float* x, const float* xd, float* hd, int N, int nc, int C, hipStream_t st) {
  if (N == 0) return;
  k_gate_dual_fwd<<<blocks((long)N * C, 256), 256, 0, st>>>(x, xd, hd, N, nc, C);
}
void launch_gate_dual_bwd(const float* x, const float* xd, const float* hb, const float* hc, float* xb, float* xc,
                          int N, int nc, int C, hipStream_t st) {
  if (N == 0) return;
  k_gate_dual_bwd<<<blocks((long)N * C, 256), 256, 0, st>>>(x, xd, hb, hc, xb, xc, N, nc, C);
}
void launch_readout_dual(const float* h, const float* hd, int nc, const int* owner, const double* gE, const float* Wr,
                         const float* w2, int N, int C, float* Pb, float* Pc, float* w2c, float* hb, float* hc,
                         float* eb, hipStream_t st) {
  if (N == 0) return;
  k_readout_dual<<<blocks((long)N * 64, 256), 256, 0, st>>>(h, hd, nc, owner, gE, Wr, w2, N, C, Pb, Pc, w2c, hb, hc,
                                                             eb);
}
void launch_group_sum(const float* X, long ld, const int* species, int n_groups, int N, int ncols, double* out,
                      long ld_out, hipStream_t st) {
  k_group_sum<<<blocks((long)n_groups * ncols, 64), 64, 0, st>>>(X, ld, species, n_groups, N, ncols, out, ld_out);
}
// out (FP64, row stride ld_out) = X1^T Y1 + X2^T Y2 over `rows` rows (capped
// at *rows_dev when given); `partial` must hold chunks(rows) * mo * no floats.
int tn_chunks(long rows) {
  const long c = (rows + 1023) / 1024;
  return (int)std::max<long>(1, std::min<long>(c, 256));
}
static int tn_chunks_for(long rows, int mo, int no) {
  // cap the partial buffer at 16 M floats
  const long cap = std::max<long>(1, (16L << 20) / ((long)mo * no));
  return (int)std::min<long>(tn_chunks(rows), cap);
}
void launch_gemm_tn(RowMap x1, RowMap y1, RowMap x2, RowMap y2, long rows, const int* rows_dev, int mo, int no,
                    float* partial, double* out, long ld_out, hipStream_t st) {
  if (mo == 0 || no == 0) return;
  const int chunks = tn_chunks_for(rows, mo, no);
  const int chunk_rows = (int)((rows + chunks - 1) / chunks);
  dim3 grid(blocks(mo, 64), blocks(no, 64), chunks);
  if (rows > 0) {
    k_gemm_tn<<<grid, 256, 0, st>>>(x1, y1, x2, y2, (int)rows, rows_dev, mo, no, chunk_rows, partial);
    k_reduce_partials<<<blocks((long)mo * no, 256), 256, 0, st>>>(partial, chunks, mo, no, out, ld_out);
  }
}

void launch_hvp_geo(int lmax, const int* row_ptr_x, int N, long e_cap, const float4* dvec, const float4* dd,
                    const float* Yb, const float* Yc, const float* P1g, const float* W1, float rc, int p,
                    int accumulate, float4* g, hipStream_t st) {
  if (e_cap == 0) return;
  const int grid = blocks(e_cap, 256);
  if (lmax == 3)
    k_hvp_geo<3><<<grid, 256, 0, st>>>(row_ptr_x, N, dvec, dd, Yb, Yc, P1g, W1, rc, p, accumulate, g);
  else if (lmax == 2)
    k_hvp_geo<2><<<grid, 256, 0, st>>>(row_ptr_x, N, dvec, dd, Yb, Yc, P1g, W1, rc, p, accumulate, g);
  else
    throw Error(E3MI_EUNSUPPORTED, "lmax must be 2 or 3");
}

}  // namespace e3mi
