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

template <int LMAX, int KIND, int CPT>
__global__ void __launch_bounds__(256) k_tp_fwd(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                const float4* __restrict__ dvec, const float* __restrict__ R,
                                                int r_stride, const float* __restrict__ h, int h_nc,
                                                float* __restrict__ A, int N, int C, float inv_nu) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NOUT = PS::NOUT, NIN = PS::NIN, NY = PS::NY;
  const int i = blockIdx.x;
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
    const float* Re = R + (long)e * r_stride;
    const float* hj = h + (long)j * h_nc * C;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      float hv[NIN];
#pragma unroll
      for (int q = 0; q < NIN; ++q) hv[q] = hj[q * C + k];
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int off = PS::T.off[pi];
        const float rp = Re[pi * C + k];
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

template <int LMAX, int KIND, int CPT>
__global__ void __launch_bounds__(256) k_tp_bwd_edge(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                     const float4* __restrict__ dvec, const float* __restrict__ R,
                                                     int r_stride, const float* __restrict__ h, int h_nc,
                                                     const float* __restrict__ dA, float* __restrict__ dR,
                                                     float* __restrict__ dY, int N, int C, float inv_nu) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NOUT = PS::NOUT, NIN = PS::NIN, NY = PS::NY;
  __shared__ float red[4][16];
  const int i = blockIdx.x;
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
    const float4 d = dvec[e];
    const float ir = 1.0f / d.w;
    float Y[NY];
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    const float* Re = R + (long)e * r_stride;
    float* dRe = dR + (long)e * r_stride;
    const float* hj = h + (long)j * h_nc * C;
    float dyp[NY];
#pragma unroll
    for (int q = 0; q < NY; ++q) dyp[q] = 0.0f;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      float hv[NIN];
#pragma unroll
      for (int q = 0; q < NIN; ++q) hv[q] = hj[q * C + k];
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int off = PS::T.off[pi];
        const float rp = Re[pi * C + k];
        float tm[2 * l3 + 1];
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) tm[m] = 0.0f;
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          tm[kM3[q]] += hv[l1 * l1 + kM1[q]] * (kC[q] * Y[l2 * l2 + kM2[q]]);
          dyp[l2 * l2 + kM2[q]] += kC[q] * (hv[l1 * l1 + kM1[q]] * (rp * dai[c][off + kM3[q]]));
        });
        float s = 0.0f;
#pragma unroll
        for (int m = 0; m < 2 * l3 + 1; ++m) s += dai[c][off + m] * tm[m];
        dRe[pi * C + k] = s;
      });
    }
    // reduce dY over the channels of the workgroup
    if (tpr >= 64) {
#pragma unroll
      for (int q = 0; q < NY; ++q) dyp[q] = group_sum<64>(dyp[q]);
      if (tpr == 64) {
        if (lane < NY) {
          float v = 0.0f;
#pragma unroll
          for (int q = 0; q < NY; ++q) v = lane == q ? dyp[q] : v;
          dY[(long)e * 16 + lane] = v;
        }
      } else {
        if (lane == 0) {
#pragma unroll
          for (int q = 0; q < NY; ++q) red[wave][q] = dyp[q];
        }
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

template <int LMAX, int KIND, int CPT>
__global__ void __launch_bounds__(256) k_tp_bwd_node(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                     const float4* __restrict__ dvec, const float* __restrict__ R,
                                                     int r_stride, const float* __restrict__ dA,
                                                     float* __restrict__ dh, int dh_nc, int N, int C, float inv_nu) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NIN = PS::NIN, NY = PS::NY;
  const int j = blockIdx.x;
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
    const float* Re = R + (long)e * r_stride;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = threadIdx.x + c * tpr;
      static_for<NP>([&](auto pi) {
        constexpr int g = PS::T.id[pi];
        constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
        constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
        constexpr int rank = PS::T.rank[pi];
        constexpr int P3 = PS::T.np_l3[l3];
        const float rp = Re[pi * C + k];
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
#pragma unroll
    for (int q = 0; q < NIN; ++q) dh[((long)j * dh_nc + q) * C + k] += acc[c][q] * inv_nu;
  }
}

}  // namespace

// ---- dispatch ---------------------------------------------------------------

template <int LMAX, int KIND, int CPT>
static void tp_launch(int which, const TpArgs& a, hipStream_t st) {
  const int tpr = a.C / CPT;
  if (a.N == 0) return;
  if (which == 0)
    k_tp_fwd<LMAX, KIND, CPT><<<a.N, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.R, a.r_stride, a.h, a.h_nc, a.A, a.N,
                                                    a.C, a.inv_nu);
  else if (which == 1)
    k_tp_bwd_edge<LMAX, KIND, CPT><<<a.N, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.R, a.r_stride, a.h, a.h_nc, a.dA,
                                                         a.dR, a.dY, a.N, a.C, a.inv_nu);
  else
    k_tp_bwd_node<LMAX, KIND, CPT><<<a.N, tpr, 0, st>>>(a.row_ptr, a.src, a.dvec, a.R, a.r_stride, a.dA, a.dh,
                                                         a.dh_nc, a.N, a.C, a.inv_nu);
}

template <int LMAX, int KIND>
static void tp_cpt(int which, const TpArgs& a, hipStream_t st) {
  switch (a.cpt) {
    case 1: return tp_launch<LMAX, KIND, 1>(which, a, st);
    case 2: return tp_launch<LMAX, KIND, 2>(which, a, st);
    case 4:
      if constexpr (KIND != kFull) return tp_launch<LMAX, KIND, 4>(which, a, st);
      [[fallthrough]];
    default: throw Error(E3MI_EUNSUPPORTED, "channels per thread not supported for this layer");
  }
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
