// Clebsch-Gordan tensor product + neighbour sum (the operation the paper's
// backend accelerates, Section 4), and its two adjoints.
//
// Receiver-centric: one workgroup owns one receiver atom i and walks its CSR
// row of edges e = (i <- j), so the neighbour sum accumulates in registers and
// needs no global atomics. Threads map to channels (channel-contiguous h, R and
// A make every load and store coalesced); each thread handles CPT channels.
//
//   forward   A[i,p,k,m3]  = nu^-1 sum_e R[e,p,k] sum_{m1 m2} C^p[m1,m2,m3] h[j,k,l1 m1] Y_e[l2 m2]
//   edge adj  dR[e,p,k]    = nu^-1 sum_m3 dA[i,p,k,m3] T[e,p,k,m3]   (T = the inner CG sum)
//             dY[e,l2 m2]  = nu^-1 sum_{p,k,m1,m3} C R dA h           (reduced over channels)
//   node adj  dh[j,k,l1 m1] = nu^-1 sum_{e: src(e) = j} sum_p R sum C Y_e dA[dst(e)]
//             computed for atom j from its own incoming edges e' via the reverse
//             edge: dst(rev e') = src(e'), R is a function of |d| only, and
//             Y(-d) = (-1)^l Y(d), so no other row is read except dA[src(e')].
//
// A layout (consumed by the channel-mix GEMM): for each output order l3 a
// block [N, 2 l3 + 1, P_l3, C].
#include "common.h"
#include "paths.h"
#include "runtime.h"

namespace e3mi {
namespace {

template <int W>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

// The scalar-output layer's forward is compiled for at most three waves per
// SIMD: the compiler then schedules its edge loop with 88 registers instead
// of 72 (the hardware still holds five waves) and it runs faster (0.134 ms
// against 0.141 on the 3,000-atom step). Holding residency at three or two
// waves for real, by reserving LDS, is slower (0.167, 0.196 ms).
template <int LMAX, int KIND, int CPT, class RS, bool IDX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, KIND == kLast ? 3 : 10))) k_tp_fwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                const float4* __restrict__ dvec, const RS* __restrict__ R,
                                                int r_stride, const float* __restrict__ h, int h_nc,
                                                float* __restrict__ A, int N, int C, float inv_nu, int i0,
                                                int e_first, const int* __restrict__ r_row) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NOUT = PS::NOUT, NIN = PS::NIN, NY = PS::NY;
  const int i = i0 + xcd_contiguous(blockIdx.x, gridDim.x);
  const int tpr = blockDim.x;
  float acc[CPT][NOUT];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int o = 0; o < NOUT; ++o) acc[c][o] = 0.0f;
  const int e1 = row_ptr[i + 1];
  for (int e = row_ptr[i]; e < e1; ++e) {
    const int j = src[e];
    const float4 d = dvec[e];
    const float ir = 1.0f / d.w;
    float Y[NY];
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    const RS* Re = R + (long)(IDX ? r_row[e] : e - e_first) * r_stride;
    const float* hj = h + (long)j * h_nc * C;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      float hv[NIN], rv[NP];
#pragma unroll
      for (int q = 0; q < NIN; ++q) hv[q] = hj[q * C + k];
      // every path's weight of the edge in one batch of loads
#pragma unroll
      for (int q = 0; q < NP; ++q) rv[q] = ldr(Re + q * C + k);
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int off = PS::T.off[pi];
        const float rp = rv[pi];
        float tm[2 * l3 + 1];
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) tm[m] = 0.0f;
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          tm[kM3[q]] += hv[l1 * l1 + kM1[q]] * (kC[q] * Y[l2 * l2 + kM2[q]]);
        });
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) acc[c][off + m] += rp * tm[m];
      });
    }
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = threadIdx.x + c * tpr;
    static_for<NP>([&](auto pi) {
      constexpr int g = PS::T.id[pi];
      constexpr int l3 = kL3[g];
      constexpr int off = PS::T.off[pi], rank = PS::T.rank[pi];
      constexpr int P3 = PS::T.np_l3[l3];
      float* base = A + a_group_base<PS>(l3, N, C);
#pragma unroll
      for (int m = 0; m < 2 * l3 + 1; ++m)
        base[(((long)i * (2 * l3 + 1) + m) * P3 + rank) * C + k] = acc[c][off + m] * inv_nu;
    });
  }
}

// MSG: also write each edge's share of its sender's gradient,
//   msg[e, l1 m1, k] = nu^-1 sum_p R[e,p,k] sum_{m2 m3} C^p Y_e[l2 m2] dA[i,p,k,m3],
// at row e - e_first, for k_tp_msg_node to add up per sender.
// Layers with every path hold 99 adjoint values per channel: the compiler is
// asked for two waves per SIMD (at most 256 registers); one wave per SIMD
// halves the kernel's speed.
template <int LMAX, int KIND, int CPT, bool MSG, class RS, bool IDX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KIND == kFull ? 2 : 1, 10))) k_tp_bwd_edge(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                     const float4* __restrict__ dvec, const RS* __restrict__ R,
                                                     int r_stride, const float* __restrict__ h, int h_nc,
                                                     const float* __restrict__ dA, RS* __restrict__ dR,
                                                     float* __restrict__ dY, int N, int C, float inv_nu, int i0,
                                                     int e_first, float* __restrict__ msg, int* __restrict__ touched,
                                                     int tag, const int* __restrict__ r_row) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NOUT = PS::NOUT, NIN = PS::NIN, NY = PS::NY;
  __shared__ float red[4][16];
  const int i = i0 + xcd_contiguous(blockIdx.x, gridDim.x);
  const int tpr = blockDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float dai[CPT][NOUT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = threadIdx.x + c * tpr;
    static_for<NP>([&](auto pi) {
      constexpr int g = PS::T.id[pi];
      constexpr int l3 = kL3[g];
      constexpr int off = PS::T.off[pi], rank = PS::T.rank[pi];
      constexpr int P3 = PS::T.np_l3[l3];
      const float* base = dA + a_group_base<PS>(l3, N, C);
#pragma unroll
      for (int m = 0; m < 2 * l3 + 1; ++m)
        dai[c][off + m] = base[(((long)i * (2 * l3 + 1) + m) * P3 + rank) * C + k] * inv_nu;
    });
  }
  const int e1 = row_ptr[i + 1];
  for (int e = row_ptr[i]; e < e1; ++e) {
    const int j = src[e];
    if (MSG && threadIdx.x == 0) touched[j] = tag;  // j receives a message from this chunk
    const float4 d = dvec[e];
    const float ir = 1.0f / d.w;
    float Y[NY];
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    const RS* Re = R + (long)(IDX ? r_row[e] : e - e_first) * r_stride;
    RS* dRe = dR + (long)(e - e_first) * r_stride;
    const float* hj = h + (long)j * h_nc * C;
    float dyp[NY];
#pragma unroll
    for (int q = 0; q < NY; ++q) dyp[q] = 0.0f;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      float hv[NIN], mv[MSG ? NIN : 1], rv[NP];
#pragma unroll
      for (int q = 0; q < NIN; ++q) hv[q] = hj[q * C + k];
#pragma unroll
      for (int q = 0; q < NP; ++q) rv[q] = ldr(Re + q * C + k);
#pragma unroll
      for (int q = 0; q < (MSG ? NIN : 1); ++q) mv[q] = 0.0f;
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int off = PS::T.off[pi];
        const float rp = rv[pi];
        float tm[2 * l3 + 1];
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) tm[m] = 0.0f;
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          const float cy = kC[q] * Y[l2 * l2 + kM2[q]];
          const float rd = rp * dai[c][off + kM3[q]];
          tm[kM3[q]] += hv[l1 * l1 + kM1[q]] * cy;
          dyp[l2 * l2 + kM2[q]] += kC[q] * (hv[l1 * l1 + kM1[q]] * rd);
          if constexpr (MSG) mv[l1 * l1 + kM1[q]] += rd * cy;
        });
        float s = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) s += dai[c][off + m] * tm[m];
        str(dRe + pi * C + k, s);
      });
      if constexpr (MSG) {
        float* me = msg + (long)(e - e_first) * NIN * C + k;
#pragma unroll
        for (int q = 0; q < NIN; ++q) me[q * C] = mv[q];
      }
    }
    // reduce dY over the channels of the workgroup
    if (tpr >= 64) {
      const float tot = wave_sum_scatter16<NY>(dyp);
      const int q = lane >> 2;
      if (tpr == 64) {
        if ((lane & 3) == 0 && q < NY) dY[(long)e * 16 + q] = tot;
      } else {
        if ((lane & 3) == 0) red[wave][q] = tot;
        __syncthreads();
        if (threadIdx.x < NY) {
          float v = 0.0f;
          for (int w = 0; w < tpr / 64; ++w) v += red[w][threadIdx.x];
          dY[(long)e * 16 + threadIdx.x] = v;
        }
        __syncthreads();
      }
    } else {
#pragma unroll
      for (int q = 0; q < NY; ++q) dyp[q] = group_sum<32>(dyp[q]);
      if (lane < NY) {
        float v = 0.0f;
#pragma unroll
        for (int q = 0; q < NY; ++q) v = lane == q ? dyp[q] : v;
        dY[(long)e * 16 + lane] = v;
      }
    }
  }
}

template <int LMAX, int KIND, int CPT, class RS, bool IDX>
__global__ void __launch_bounds__(256) k_tp_bwd_node(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                     const float4* __restrict__ dvec, const RS* __restrict__ R,
                                                     int r_stride, const float* __restrict__ dA,
                                                     float* __restrict__ dh, int dh_nc, int N, int C, float inv_nu,
                                                     int i0, int e_first, int dh_acc, const int* __restrict__ r_row) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NIN = PS::NIN, NY = PS::NY;
  const int j = i0 + xcd_contiguous(blockIdx.x, gridDim.x);
  const int tpr = blockDim.x;
  float acc[CPT][NIN];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int q = 0; q < NIN; ++q) acc[c][q] = 0.0f;
  const int e1 = row_ptr[j + 1];
  for (int e = row_ptr[j]; e < e1; ++e) {
    const int i2 = src[e];  // receiver of the reverse edge
    const float4 d = dvec[e];
    const float ir = -1.0f / d.w;  // direction of the reverse edge
    float Y[NY];
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    const RS* Re = R + (long)(IDX ? r_row[e] : e - e_first) * r_stride;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int rank = PS::T.rank[pi];
        constexpr int P3 = PS::T.np_l3[l3];
        const float rp = ldr(Re + pi * C + k);
        const float* base = dA + a_group_base<PS>(l3, N, C);
        float dav[2 * l3 + 1];
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m)
          dav[m] = rp * base[(((long)i2 * (2 * l3 + 1) + m) * P3 + rank) * C + k];
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          acc[c][l1 * l1 + kM1[q]] += dav[kM3[q]] * (kC[q] * Y[l2 * l2 + kM2[q]]);
        });
      });
    }
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = threadIdx.x + c * tpr;
    // components below dh_acc (all when dh_acc <= 0) are added to, the others
    // written (zero past the paths' inputs)
#pragma unroll
    for (int q = 0; q < NIN; ++q) {
      float* o = dh + ((long)j * dh_nc + q) * C + k;
      *o = (dh_acc <= 0 || q < dh_acc) ? *o + acc[c][q] * inv_nu : acc[c][q] * inv_nu;
    }
    if (dh_acc > 0)
      for (int q = NIN; q < dh_nc; ++q)
        if (q >= dh_acc) dh[((long)j * dh_nc + q) * C + k] = 0.0f;
  }
}

// Sender gradient from the edges' messages: dh[j] continues from its stored
// value (from init, the first chunk, or the previous chunk) and adds msg of
// j's outgoing edges e = rev(e2), e2 over the run of j's row whose senders
// (the receivers of e) lie in this chunk's receivers [c0, c1), in row order.
// Rows are sorted by sender, so the runs of successive chunks follow each
// other along the row and every sender's sum is the same sequence of
// additions whatever the chunking. init: components below dh_acc (all when
// dh_acc <= 0) start from dh, the others from zero (components NIN..dh_nc-1
// past dh_acc are zeroed). Block b is sender b (no XCD remapping): the
// senders a chunk touches are a compact index range (atoms are spatially
// sorted), and consecutive blocks go to different XCDs, so that range
// spreads over the whole chip. Messages are read four edges at a time (64
// loads in flight per lane) and added in row order.
template <int NIN>
__global__ void __launch_bounds__(256) k_tp_msg_node(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                     const int* __restrict__ rev, const float* __restrict__ msg,
                                                     float* __restrict__ dh, int dh_nc, int C, int c0, int c1,
                                                     int e_first, int init, int dh_acc,
                                                     const int* __restrict__ touched, int tag) {
  const int j = blockIdx.x;
  // after the first chunk, only senders this chunk's edge adjoint sent to
  // (touched carries the chunk's tag; another value can only add an empty run)
  if (!init && touched[j] != tag) return;
  const int a = row_ptr[j], b = row_ptr[j + 1];
  // the run: first entry with src >= c0 .. first entry with src >= c1
  auto lower = [&](int v) {
    int lo = a, hi = b;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (src[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  const int r0 = lower(c0), r1 = lower(c1);
  for (int k = threadIdx.x; k < C; k += blockDim.x) {
    float acc[NIN];
#pragma unroll
    for (int q = 0; q < NIN; ++q) {
      const bool keep = !init || dh_acc <= 0 || q < dh_acc;
      acc[q] = keep ? dh[((long)j * dh_nc + q) * C + k] : 0.0f;
    }
    int e2 = r0;
    for (; e2 + 4 <= r1; e2 += 4) {
      int ev[4];
      float mv[4][NIN];
#pragma unroll
      for (int u = 0; u < 4; ++u) ev[u] = rev[e2 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // an edge without a reverse reads the chunk's first message, unused
        const float* me = msg + (ev[u] >= 0 ? (long)(ev[u] - e_first) : 0L) * NIN * C + k;
#pragma unroll
        for (int q = 0; q < NIN; ++q) mv[u][q] = me[q * C];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NIN; ++q)
          if (ev[u] >= 0) acc[q] += mv[u][q];
    }
    for (; e2 < r1; ++e2) {
      const int e = rev[e2];
      if (e < 0) continue;
      const float* me = msg + (long)(e - e_first) * NIN * C + k;
#pragma unroll
      for (int q = 0; q < NIN; ++q) acc[q] += me[q * C];
    }
#pragma unroll
    for (int q = 0; q < NIN; ++q) dh[((long)j * dh_nc + q) * C + k] = acc[q];
    if (init && dh_acc > 0)
      for (int q = NIN; q < dh_nc; ++q)
        if (q >= dh_acc) dh[((long)j * dh_nc + q) * C + k] = 0.0f;
  }
}

// ---- second order: reverse over the tangent along a position direction v ----
//   A_dot = TP(h_dot, Y, R) + TP(h, Y_dot, R) + TP(h, Y, R_dot)
// with Y_dot, R_dot the changes of the edge harmonics and radial weights when
// every atom moves along v (d_dot = v_j - v_i). The reverse pass only needs the
// adjoints of R, R_dot, h and h_dot (Y has no parameters).

template <int LMAX, int KIND, int CPT>
__global__ void __launch_bounds__(256) k_tp_dual_fwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                     const float4* __restrict__ dvec, const float4* __restrict__ dd,
                                                     const float* __restrict__ R, const float* __restrict__ Rd,
                                                     int r_stride, const float* __restrict__ h,
                                                     const float* __restrict__ hd, int h_nc, float* __restrict__ Ad,
                                                     int N, int C, float inv_nu) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NOUT = PS::NOUT, NIN = PS::NIN, NY = PS::NY;
  const int i = xcd_contiguous(blockIdx.x, gridDim.x);
  const int tpr = blockDim.x;
  float acc[CPT][NOUT];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int o = 0; o < NOUT; ++o) acc[c][o] = 0.0f;
  const int e1 = row_ptr[i + 1];
  for (int e = row_ptr[i]; e < e1; ++e) {
    const int j = src[e];
    float Y[NY], Yd[NY];
    real_sh_dual<LMAX>(dvec[e], dd[e], Y, Yd);
    const float* Re = R + (long)e * r_stride;
    const float* Rde = Rd + (long)e * r_stride;
    const float* hj = h + (long)j * h_nc * C;
    const float* hdj = hd ? hd + (long)j * h_nc * C : nullptr;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      float hv[NIN], hdv[NIN];
#pragma unroll
      for (int q = 0; q < NIN; ++q) {
        hv[q] = hj[q * C + k];
        hdv[q] = hdj ? hdj[q * C + k] : 0.0f;
      }
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int off = PS::T.off[pi];
        const float rp = Re[pi * C + k], rdp = Rde[pi * C + k];
        float tm[2 * l3 + 1], td[2 * l3 + 1];
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) tm[m] = td[m] = 0.0f;
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          const float a = hv[l1 * l1 + kM1[q]], ad = hdv[l1 * l1 + kM1[q]];
          tm[kM3[q]] += a * (kC[q] * Y[l2 * l2 + kM2[q]]);
          td[kM3[q]] += kC[q] * (ad * Y[l2 * l2 + kM2[q]] + a * Yd[l2 * l2 + kM2[q]]);
        });
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) acc[c][off + m] += rdp * tm[m] + rp * td[m];
      });
    }
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = threadIdx.x + c * tpr;
    static_for<NP>([&](auto pi) {
      constexpr int g = PS::T.id[pi];
      constexpr int l3 = kL3[g];
      constexpr int off = PS::T.off[pi], rank = PS::T.rank[pi];
      constexpr int P3 = PS::T.np_l3[l3];
      float* base = Ad + a_group_base<PS>(l3, N, C);
#pragma unroll
      for (int m = 0; m < 2 * l3 + 1; ++m)
        base[(((long)i * (2 * l3 + 1) + m) * P3 + rank) * C + k] = acc[c][off + m] * inv_nu;
    });
  }
}

template <int LMAX, int KIND, int CPT>
__global__ void __launch_bounds__(256) k_tp_dual_bwd_edge(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                          const float4* __restrict__ dvec, const float4* __restrict__ dd,
                                                          int r_stride, const float* __restrict__ h,
                                                          const float* __restrict__ hd, int h_nc,
                                                          const float* __restrict__ Ab, const float* __restrict__ Ac,
                                                          float* __restrict__ Rb, float* __restrict__ Rc, int N, int C,
                                                          float inv_nu) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NOUT = PS::NOUT, NIN = PS::NIN, NY = PS::NY;
  const int i = xcd_contiguous(blockIdx.x, gridDim.x);
  const int tpr = blockDim.x;
  float ab[CPT][NOUT], ac[CPT][NOUT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = threadIdx.x + c * tpr;
    static_for<NP>([&](auto pi) {
      constexpr int g = PS::T.id[pi];
      constexpr int l3 = kL3[g];
      constexpr int off = PS::T.off[pi], rank = PS::T.rank[pi];
      constexpr int P3 = PS::T.np_l3[l3];
      const long gb = a_group_base<PS>(l3, N, C);
#pragma unroll
      for (int m = 0; m < 2 * l3 + 1; ++m) {
        const long idx = gb + (((long)i * (2 * l3 + 1) + m) * P3 + rank) * C + k;
        ab[c][off + m] = Ab[idx] * inv_nu;
        ac[c][off + m] = Ac[idx] * inv_nu;
      }
    });
  }
  const int e1 = row_ptr[i + 1];
  for (int e = row_ptr[i]; e < e1; ++e) {
    const int j = src[e];
    float Y[NY], Yd[NY];
    real_sh_dual<LMAX>(dvec[e], dd[e], Y, Yd);
    const float* hj = h + (long)j * h_nc * C;
    const float* hdj = hd ? hd + (long)j * h_nc * C : nullptr;
    float* Rbe = Rb + (long)e * r_stride;
    float* Rce = Rc + (long)e * r_stride;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      float hv[NIN], hdv[NIN];
#pragma unroll
      for (int q = 0; q < NIN; ++q) {
        hv[q] = hj[q * C + k];
        hdv[q] = hdj ? hdj[q * C + k] : 0.0f;
      }
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int off = PS::T.off[pi];
        float tm[2 * l3 + 1], td[2 * l3 + 1];
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) tm[m] = td[m] = 0.0f;
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          const float a = hv[l1 * l1 + kM1[q]], ad = hdv[l1 * l1 + kM1[q]];
          tm[kM3[q]] += a * (kC[q] * Y[l2 * l2 + kM2[q]]);
          td[kM3[q]] += kC[q] * (ad * Y[l2 * l2 + kM2[q]] + a * Yd[l2 * l2 + kM2[q]]);
        });
        float sb = 0.0f, sc = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) {
          sb += ab[c][off + m] * tm[m] + ac[c][off + m] * td[m];
          sc += ac[c][off + m] * tm[m];
        }
        Rbe[pi * C + k] = sb;
        Rce[pi * C + k] = sc;
      });
    }
  }
}

template <int LMAX, int KIND, int CPT>
__global__ void __launch_bounds__(256) k_tp_dual_bwd_node(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                          const float4* __restrict__ dvec, const float4* __restrict__ dd,
                                                          const float* __restrict__ R, const float* __restrict__ Rd,
                                                          int r_stride, const float* __restrict__ Ab,
                                                          const float* __restrict__ Ac, float* __restrict__ hb,
                                                          float* __restrict__ hc, int dh_nc, int N, int C,
                                                          float inv_nu) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NIN = PS::NIN, NY = PS::NY;
  const int j = xcd_contiguous(blockIdx.x, gridDim.x);
  const int tpr = blockDim.x;
  float accb[CPT][NIN], accc[CPT][NIN];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int q = 0; q < NIN; ++q) accb[c][q] = accc[c][q] = 0.0f;
  const int e1 = row_ptr[j + 1];
  for (int e = row_ptr[j]; e < e1; ++e) {
    const int i2 = src[e];  // receiver of the reverse edge
    const float4 d = dvec[e], v = dd[e];
    float Y[NY], Yd[NY];
    // the reverse edge has vector -d and tangent -d_dot
    real_sh_dual<LMAX>(make_float4(-d.x, -d.y, -d.z, d.w), make_float4(-v.x, -v.y, -v.z, v.w), Y, Yd);
    const float* Re = R + (long)e * r_stride;
    const float* Rde = Rd + (long)e * r_stride;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int rank = PS::T.rank[pi];
        constexpr int P3 = PS::T.np_l3[l3];
        const float rp = Re[pi * C + k], rdp = Rde[pi * C + k];
        const long gb = a_group_base<PS>(l3, N, C);
        float u[2 * l3 + 1], w[2 * l3 + 1];
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) {
          const long idx = gb + (((long)i2 * (2 * l3 + 1) + m) * P3 + rank) * C + k;
          const float ab = Ab[idx], ac = Ac[idx];
          u[m] = rp * ab + rdp * ac;  // multiplies Y
          w[m] = rp * ac;             // multiplies Y_dot (h adjoint) and Y (h_dot adjoint)
        }
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          const float y = kC[q] * Y[l2 * l2 + kM2[q]], yd = kC[q] * Yd[l2 * l2 + kM2[q]];
          accb[c][l1 * l1 + kM1[q]] += y * u[kM3[q]] + yd * w[kM3[q]];
          accc[c][l1 * l1 + kM1[q]] += y * w[kM3[q]];
        });
      });
    }
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = threadIdx.x + c * tpr;
#pragma unroll
    for (int q = 0; q < NIN; ++q) {
      hb[((long)j * dh_nc + q) * C + k] += accb[c][q] * inv_nu;
      if (hc) hc[((long)j * dh_nc + q) * C + k] += accc[c][q] * inv_nu;
    }
  }
}

// Adjoints of the harmonics and of their tangent for the Hessian-vector
// product: with eb = ab R + ac R_dot and ec = ac R per (path, output, channel),
//   Yb[l2 m2] = sum C (eb h[l1 m1] + ec h_dot[l1 m1]),  Yc[l2 m2] = sum C ec h[l1 m1]
// summed over paths, CG entries and the channels of the workgroup; one row
// [16] of each per edge.
template <int LMAX, int KIND, int CPT>
__global__ void __launch_bounds__(256) k_tp_dual_geo(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                     const float* __restrict__ R, const float* __restrict__ Rd,
                                                     int r_stride, const float* __restrict__ h,
                                                     const float* __restrict__ hd, int h_nc,
                                                     const float* __restrict__ Ab, const float* __restrict__ Ac,
                                                     float* __restrict__ Yb, float* __restrict__ Yc, int N, int C,
                                                     float inv_nu) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NOUT = PS::NOUT, NIN = PS::NIN, NY = PS::NY;
  __shared__ float red[4][2 * 16];
  const int i = xcd_contiguous(blockIdx.x, gridDim.x);
  const int tpr = blockDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float ab[CPT][NOUT], ac[CPT][NOUT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = threadIdx.x + c * tpr;
    static_for<NP>([&](auto pi) {
      constexpr int g = PS::T.id[pi];
      constexpr int l3 = kL3[g];
      constexpr int off = PS::T.off[pi], rank = PS::T.rank[pi];
      constexpr int P3 = PS::T.np_l3[l3];
      const long gb = a_group_base<PS>(l3, N, C);
#pragma unroll
      for (int m = 0; m < 2 * l3 + 1; ++m) {
        const long idx = gb + (((long)i * (2 * l3 + 1) + m) * P3 + rank) * C + k;
        ab[c][off + m] = Ab[idx] * inv_nu;
        ac[c][off + m] = Ac[idx] * inv_nu;
      }
    });
  }
  const int e1 = row_ptr[i + 1];
  for (int e = row_ptr[i]; e < e1; ++e) {
    const int j = src[e];
    const float* Re = R + (long)e * r_stride;
    const float* Rde = Rd + (long)e * r_stride;
    const float* hj = h + (long)j * h_nc * C;
    const float* hdj = hd ? hd + (long)j * h_nc * C : nullptr;
    float yb[NY], yc[NY];
#pragma unroll
    for (int q = 0; q < NY; ++q) yb[q] = yc[q] = 0.0f;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      float hv[NIN], hdv[NIN];
#pragma unroll
      for (int q = 0; q < NIN; ++q) {
        hv[q] = hj[q * C + k];
        hdv[q] = hdj ? hdj[q * C + k] : 0.0f;
      }
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int off = PS::T.off[pi];
        const float rp = Re[pi * C + k], rdp = Rde[pi * C + k];
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          const float eb = kC[q] * (ab[c][off + kM3[q]] * rp + ac[c][off + kM3[q]] * rdp);
          const float ec = kC[q] * (ac[c][off + kM3[q]] * rp);
          yb[l2 * l2 + kM2[q]] += eb * hv[l1 * l1 + kM1[q]] + ec * hdv[l1 * l1 + kM1[q]];
          yc[l2 * l2 + kM2[q]] += ec * hv[l1 * l1 + kM1[q]];
        });
      });
    }
    // reduce over the channels of the workgroup
    if (tpr >= 64) {
      const float tb = wave_sum_scatter16<NY>(yb), tc = wave_sum_scatter16<NY>(yc);
      if ((lane & 3) == 0) {
        red[wave][lane >> 2] = tb;
        red[wave][16 + (lane >> 2)] = tc;
      }
    } else {
#pragma unroll
      for (int q = 0; q < NY; ++q) {
        yb[q] = group_sum<32>(yb[q]);
        yc[q] = group_sum<32>(yc[q]);
      }
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NY; ++q) {
          red[0][q] = yb[q];
          red[0][16 + q] = yc[q];
        }
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * 16) {
      const int q = threadIdx.x & 15;
      float v = 0.0f;
      if (q < NY)
        for (int w = 0; w < (tpr + 63) / 64; ++w) v += red[w][threadIdx.x];
      (threadIdx.x < 16 ? Yb : Yc)[(long)e * 16 + q] = v;
    }
    __syncthreads();
  }
}

}  // namespace

// ---- dispatch ---------------------------------------------------------------

// the first-order passes (0 forward, 1 edge adjoint, 2 node adjoint); IDX:
// R rows through the edges' pair indices
template <int LMAX, int KIND, int CPT, bool IDX>
static void first_order_launch(int which, const TpArgs& a, int nr, int tpr, hipStream_t st) {
  const __bf16* Rb = reinterpret_cast<const __bf16*>(a.R);
  __bf16* dRb = reinterpret_cast<__bf16*>(a.dR);
  if (which == 0 && a.r_bf16)
    k_tp_fwd<LMAX, KIND, CPT, __bf16, IDX><<<nr, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, Rb, a.r_stride, a.h, a.h_nc,
                                                                a.A, a.N, a.C, a.inv_nu, a.i0, a.e_first, a.r_row);
  else if (which == 0)
    k_tp_fwd<LMAX, KIND, CPT, float, IDX><<<nr, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.R, a.r_stride, a.h, a.h_nc,
                                                               a.A, a.N, a.C, a.inv_nu, a.i0, a.e_first, a.r_row);
  else if (which == 1 && a.r_bf16 && a.msg)
    k_tp_bwd_edge<LMAX, KIND, CPT, true, __bf16, IDX><<<nr, tpr, 0, st>>>(
        a.row_ptr, a.src, a.dvec, Rb, a.r_stride, a.h, a.h_nc, a.dA, dRb, a.dY, a.N, a.C, a.inv_nu, a.i0, a.e_first,
        a.msg, a.touched, a.tag, a.r_row);
  else if (which == 1 && a.r_bf16)
    k_tp_bwd_edge<LMAX, KIND, CPT, false, __bf16, IDX><<<nr, tpr, 0, st>>>(
        a.row_ptr, a.src, a.dvec, Rb, a.r_stride, a.h, a.h_nc, a.dA, dRb, a.dY, a.N, a.C, a.inv_nu, a.i0, a.e_first,
        nullptr, nullptr, 0, a.r_row);
  else if (which == 1 && a.msg)
    k_tp_bwd_edge<LMAX, KIND, CPT, true, float, IDX><<<nr, tpr, 0, st>>>(
        a.row_ptr, a.src, a.dvec, a.R, a.r_stride, a.h, a.h_nc, a.dA, a.dR, a.dY, a.N, a.C, a.inv_nu, a.i0, a.e_first,
        a.msg, a.touched, a.tag, a.r_row);
  else if (which == 1)
    k_tp_bwd_edge<LMAX, KIND, CPT, false, float, IDX><<<nr, tpr, 0, st>>>(
        a.row_ptr, a.src, a.dvec, a.R, a.r_stride, a.h, a.h_nc, a.dA, a.dR, a.dY, a.N, a.C, a.inv_nu, a.i0, a.e_first,
        nullptr, nullptr, 0, a.r_row);
  else if (which == 2 && a.r_bf16)
    k_tp_bwd_node<LMAX, KIND, CPT, __bf16, IDX><<<nr, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, Rb, a.r_stride, a.dA,
                                                                     a.dh, a.dh_nc, a.N, a.C, a.inv_nu, a.i0,
                                                                     a.e_first, a.dh_acc, a.r_row);
  else if (which == 2)
    k_tp_bwd_node<LMAX, KIND, CPT, float, IDX><<<nr, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.R, a.r_stride, a.dA,
                                                                    a.dh, a.dh_nc, a.N, a.C, a.inv_nu, a.i0,
                                                                    a.e_first, a.dh_acc, a.r_row);
}

template <int LMAX, int KIND, int CPT>
static void tp_launch(int which, const TpArgs& a, hipStream_t st) {
  const int tpr = a.C / CPT;
  if (a.N == 0) return;
  const int nr = a.n_recv > 0 ? a.n_recv : a.N;  // receivers of this launch
  if (which <= 2 && a.n_recv == 0 && (a.i0 != 0 || a.e_first != 0))
    throw Error(E3MI_EINVAL, "tensor product: receiver offset without a receiver count");
  if (a.r_bf16 && which > 2 && which != 7)
    throw Error(E3MI_EINVAL, "tensor product: BF16 radial weights only in the first-order passes");
  if (a.r_row && which > 2 && which != 7)
    throw Error(E3MI_EINVAL, "tensor product: R rows per edge pair only in the first-order passes");
  if (which <= 2) {
    if (a.r_row)
      first_order_launch<LMAX, KIND, CPT, true>(which, a, nr, tpr, st);
    else
      first_order_launch<LMAX, KIND, CPT, false>(which, a, nr, tpr, st);
  }
  else if (which == 7) {
    using PS = PathSet<LMAX, KIND>;
    const int c1 = a.n_recv > 0 ? a.i0 + a.n_recv : a.N;
    k_tp_msg_node<PS::NIN><<<a.N, 128, 0, st>>>(a.row_ptr, a.src, a.rev, a.msg, a.dh, a.dh_nc, a.C, a.i0, c1,
                                                 a.e_first, a.i0 == 0 ? 1 : 0, a.dh_acc, a.touched, a.tag);
  }
  else if (which == 3)
    k_tp_dual_fwd<LMAX, KIND, CPT><<<a.N, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.dd, a.R, a.Rd, a.r_stride, a.h,
                                                         a.hd, a.h_nc, a.Ad, a.N, a.C, a.inv_nu);
  else if (which == 4)
    k_tp_dual_bwd_edge<LMAX, KIND, CPT><<<a.N, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.dd, a.r_stride, a.h, a.hd,
                                                              a.h_nc, a.Ab, a.Ac, a.Rb, a.Rc, a.N, a.C, a.inv_nu);
  else if (which == 5)
    k_tp_dual_bwd_node<LMAX, KIND, CPT><<<a.N, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.dd, a.R, a.Rd, a.r_stride,
                                                              a.Ab, a.Ac, a.hb, a.hc, a.dh_nc, a.N, a.C, a.inv_nu);
  else
    k_tp_dual_geo<LMAX, KIND, CPT><<<a.N, tpr, 0, st>>>(a.row_ptr, a.src, a.R, a.Rd, a.r_stride, a.h, a.hd, a.h_nc,
                                                         a.Ab, a.Ac, a.Yb, a.Yc, a.N, a.C, a.inv_nu);
}

template <int LMAX, int KIND>
static void tp_cpt(int which, const TpArgs& a, hipStream_t st) {
  // Layers with every path keep one channel per thread (the accumulators of
  // 99 outputs already fill the register file). The others run one channel
  // per thread too (twice the workgroups: one receiver per workgroup leaves
  // few waves per SIMD) except in the kernels that reduce over the
  // workgroup's channels once per edge (the first-order edge adjoint's dY and
  // the harmonic adjoints), which take the requested two.
  if constexpr (KIND == kFull) {
    if (a.cpt == 1) return tp_launch<LMAX, KIND, 1>(which, a, st);
  } else {
    const bool reduces_per_edge = which == 1 || which == 6;
    if (a.cpt == 1 || (a.cpt == 2 && !reduces_per_edge)) return tp_launch<LMAX, KIND, 1>(which, a, st);
    if (a.cpt == 2) return tp_launch<LMAX, KIND, 2>(which, a, st);
  }
  throw Error(E3MI_EUNSUPPORTED, "channels per thread not supported for this layer");
}

template <int LMAX>
static void tp_kind(int which, const TpArgs& a, hipStream_t st) {
  switch (a.kind) {
    case kFirst: return tp_cpt<LMAX, kFirst>(which, a, st);
    case kFull: return tp_cpt<LMAX, kFull>(which, a, st);
    case kLast: return tp_cpt<LMAX, kLast>(which, a, st);
    case kFirstLast: return tp_cpt<LMAX, kFirstLast>(which, a, st);
    default: throw Error(E3MI_EINVAL, "bad layer kind");
  }
}

void launch_tp(int which, const TpArgs& a, hipStream_t st) {
  switch (a.lmax) {
    case 2: return tp_kind<2>(which, a, st);
    case 3: return tp_kind<3>(which, a, st);
    default: throw Error(E3MI_EUNSUPPORTED, "lmax must be 2 or 3");
  }
}

}  // namespace e3mi
