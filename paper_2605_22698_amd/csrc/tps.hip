// Adjoint of the tensor product + neighbour sum of a scalar-output layer
// (only the paths (l, l, 0): the last layer, whose outputs only the readout
// reads), from the senders' side, for 64 x CH channels (CH adjacent channels
// per lane, loaded as one vector).
//
// For an edge e = (i <- j) with direction d_e the forward gives
//   A[i,p,k] = nu^-1 sum_e R[e,p,k] T[e,p,k],  T[e,p,k] = sum_m C^p[m,m,0] h[j,k,l m] Y_e[l m],
// so the adjoint needs, per edge,
//   dR[e,p,k]  = nu^-1 dA[i,p,k] T[e,p,k]
//   dY[e,l m]  = nu^-1 sum_{p,k} C^p R[e,p,k] dA[i,p,k] h[j,k,l m]
// and per sender
//   dh[j,k,l m] = nu^-1 sum_{e: src(e) = j} C^p R[e,p,k] dA[i,p,k] Y_e[l m].
// A wave owns a sender j, holds h_j in registers and walks j's own incoming
// edges e' = (j <- i): each stands for j's outgoing edge e = rev(e') = (i <- j),
// with d_e = -d_e', R_e = R_e' (R depends on |d| only) and dA_i gathered
// (NP x C values, where a receiver-side pass gathers h_j, (L+1)^2 x C, per
// edge). dh_j is summed in registers in the order of j's row, so the result
// does not depend on other structures in the batch.
//
// dR_e and dY_e are stored in the slot of e' (j's own row, contiguous, and
// inside a receiver chunk when j is), dY_e with the sign (-1)^l: it is then the
// adjoint of the harmonics of e''s own direction (Y_l(-n) = (-1)^l Y_l(n)),
// and the radial adjoint of slot e' yields the gradient with respect to d_e'
// = -d_e, i.e. minus e's. Forces F_i = sum_{e in in(i)} (g_e - g_rev(e)) take
// each edge with both signs, so the forces are the same. An edge inside the
// cutoff whose reverse is not (its FP64 length within rounding of r_c, where
// the envelope and its derivatives vanish) gets zeros.
#include "common.h"
#include "paths.h"
#include "runtime.h"

namespace e3mi {
namespace {

// dR and dY are streamed out with non-temporal stores (not kept in the
// caches), so that they do not evict the R rows this pass still has to read
template <int n>
__device__ __forceinline__ void str_nt(float* p, const float* v) {
  if constexpr (n == 1) {
    __builtin_nontemporal_store(v[0], p);
  } else if constexpr (n == 2) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(f2{v[0], v[1]}, reinterpret_cast<f2*>(p));
  } else {
    typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < n; q += 4)
      __builtin_nontemporal_store(f4{v[q], v[q + 1], v[q + 2], v[q + 3]}, reinterpret_cast<f4*>(p + q));
  }
}
template <int n>
__device__ __forceinline__ void str_nt(__bf16* p, const float* v) {
  typedef __bf16 bvec __attribute__((ext_vector_type(n)));
  bvec t;
#pragma unroll
  for (int q = 0; q < n; ++q) t[q] = (__bf16)v[q];
  __builtin_nontemporal_store(t, reinterpret_cast<bvec*>(p));
}

template <int LMAX, int KIND, int CH, bool DH, class RS>
__global__ void __launch_bounds__(64) k_tps_bwd_sender(const int* __restrict__ row_ptr, const int* __restrict__ src,
                                                       const int* __restrict__ rev, const float4* __restrict__ dvec,
                                                       const RS* __restrict__ R, int r_stride,
                                                       const float* __restrict__ h, int h_nc,
                                                       const float* __restrict__ dA, RS* __restrict__ dR,
                                                       float* __restrict__ dY, float* __restrict__ dh, int dh_nc,
                                                       int dh_acc, int C, float inv_nu, int i0, int e_first,
                                                       const int* __restrict__ r_row) {
  using PS = PathSet<LMAX, KIND>;
  constexpr int NP = PS::NP, NIN = PS::NIN, NY = PS::NY;
  constexpr int NA = DH ? NIN : 1;
  static_assert(PS::NOUT == NP, "scalar outputs only");
  const int j = i0 + xcd_contiguous(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x;
  const int k0 = lane * CH;
  float hv[NIN][CH];
  {
    const float* hj = h + (long)j * h_nc * C + k0;
#pragma unroll
    for (int q = 0; q < NIN; ++q) ldr_n<CH>(hj + q * C, hv[q]);
  }
  float acc[NA][CH];
#pragma unroll
  for (int q = 0; q < NA; ++q)
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[q][c] = 0.0f;
  // Software pipeline over j's row (up to 128 channels): the indices of edge
  // e2 + 2 and the R and dA rows of edge e2 + 1 are in flight while edge e2
  // is processed (the rows of consecutive edges lie far apart, and a wave
  // owns one sender). With 256 channels the prefetched rows would halve the
  // waves per SIMD: each edge's rows are loaded when it is processed.
  constexpr bool kPipe = CH <= 2;
  const int eb = row_ptr[j], e1 = row_ptr[j + 1];
  struct Idx {
    int rev, i, row;
    float4 d;
  };
  auto load_idx = [&](int e) {
    Idx x;
    x.rev = rev[e];
    x.i = src[e];
    x.row = r_row ? r_row[e] : e - e_first;
    x.d = dvec[e];
    return x;
  };
  auto load_rows = [&](const Idx& x, float (&oR)[NP][CH], float (&oA)[NP][CH]) {
    if (x.rev < 0) return;
    const RS* Re = R + (long)x.row * r_stride + k0;
    const float* dAi = dA + (long)x.i * NP * C + k0;
    static_for<NP>([&](auto pi) {
      ldr_n<CH>(Re + pi * C, oR[pi]);
      ldr_n<CH>(dAi + PS::T.rank[pi] * C, oA[pi]);
    });
  };
  float nR[kPipe ? NP : 1][CH], nA[kPipe ? NP : 1][CH];
  Idx nx{-1, 0, 0, make_float4(0.f, 0.f, 1.f, 1.f)}, nnx = nx;
  if constexpr (kPipe) {
    if (eb < e1) {
      nx = load_idx(eb);
      load_rows(nx, nR, nA);
    }
    if (eb + 1 < e1) nnx = load_idx(eb + 1);
  }
  for (int e2 = eb; e2 < e1; ++e2) {
    Idx cx;
    float cR[NP][CH], cA[NP][CH];
    if constexpr (kPipe) {
      cx = nx;
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          cR[p][c] = nR[p][c];
          cA[p][c] = nA[p][c];
        }
      if (e2 + 1 < e1) {
        nx = nnx;
        load_rows(nx, nR, nA);
        if (e2 + 2 < e1) nnx = load_idx(e2 + 2);
      }
    } else {
      cx = load_idx(e2);
      load_rows(cx, cR, cA);
    }
    RS* dRe = dR + (long)(e2 - e_first) * r_stride + k0;
    if (cx.rev < 0) {  // the edge i <- j is not in i's list
      const float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      static_for<NP>([&](auto pi) { str_nt<CH>(dRe + pi * C, z); });
      if (lane < 16) __builtin_nontemporal_store(0.0f, dY + (long)e2 * 16 + lane);
      continue;
    }
    const float4 d = cx.d;
    const float ir = -1.0f / d.w;  // d_e = -d_e2
    float Y[NY];
    real_sh<LMAX>(d.x * ir, d.y * ir, d.z * ir, Y);
    float dyp[NY];
#pragma unroll
    for (int q = 0; q < NY; ++q) dyp[q] = 0.0f;
    static_for<NP>([&](auto pi) {
      constexpr int g = PS::T.id[pi];
      constexpr int l1 = kL1[g], l2 = kL2[g];
      constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
      float s[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const float dai = cA[pi][c] * inv_nu;
        const float u = cR[pi][c] * dai;
        float t = 0.0f;
        static_for<nz>([&](auto z) {
          constexpr int q = z0 + z;
          const float cy = kC[q] * Y[l2 * l2 + kM2[q]];
          t += hv[l1 * l1 + kM1[q]][c] * cy;
          dyp[l2 * l2 + kM2[q]] += kC[q] * (hv[l1 * l1 + kM1[q]][c] * u);
          if constexpr (DH) acc[l1 * l1 + kM1[q]][c] += u * cy;
        });
        s[c] = dai * t;
      }
      str_nt<CH>(dRe + pi * C, s);
    });
    const float tot = wave_sum_scatter16<NY>(dyp);
    const int q = lane >> 2;
    // (-1)^l for component q = l^2 + m + l: odd for q in 1..3 and 9..15
    const bool odd = (q >= 1 && q <= 3) || q >= 9;
    if ((lane & 3) == 0 && q < NY) __builtin_nontemporal_store(odd ? -tot : tot, dY + (long)e2 * 16 + q);
  }
  if constexpr (DH) {
    // components below dh_acc (all when dh_acc <= 0) are added to, the others
    // written (zero past the paths' inputs)
#pragma unroll
    for (int q = 0; q < NIN; ++q) {
      float* o = dh + ((long)j * dh_nc + q) * C + k0;
      float v[CH];
      const bool add = dh_acc <= 0 || q < dh_acc;
      if (add) ldr_n<CH>(o, v);
#pragma unroll
      for (int c = 0; c < CH; ++c) v[c] = (add ? v[c] : 0.0f) + acc[q][c];
      str_n<CH>(o, v);
    }
    if (dh_acc > 0)
      for (int q = NIN; q < dh_nc; ++q)
        if (q >= dh_acc) {
          const float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
          str_n<CH>(dh + ((long)j * dh_nc + q) * C + k0, z);
        }
  }
}

template <int LMAX, int KIND, int CH, class RS>
void sender_launch_rs(const TpArgs& a, int nr, hipStream_t st) {
  const RS* R = reinterpret_cast<const RS*>(a.R);
  RS* dR = reinterpret_cast<RS*>(a.dR);
  if (a.dh)
    k_tps_bwd_sender<LMAX, KIND, CH, true, RS><<<nr, 64, 0, st>>>(a.row_ptr, a.src, a.rev, a.dvec, R, a.r_stride, a.h,
                                                                  a.h_nc, a.dA, dR, a.dY, a.dh, a.dh_nc, a.dh_acc, a.C,
                                                                  a.inv_nu, a.i0, a.e_first, a.r_row);
  else
    k_tps_bwd_sender<LMAX, KIND, CH, false, RS><<<nr, 64, 0, st>>>(a.row_ptr, a.src, a.rev, a.dvec, R, a.r_stride,
                                                                   a.h, a.h_nc, a.dA, dR, a.dY, nullptr, 0, 0, a.C,
                                                                   a.inv_nu, a.i0, a.e_first, a.r_row);
}

template <int LMAX, int KIND, int CH>
void sender_launch(const TpArgs& a, int nr, hipStream_t st) {
  if (a.r_bf16) return sender_launch_rs<LMAX, KIND, CH, __bf16>(a, nr, st);
  sender_launch_rs<LMAX, KIND, CH, float>(a, nr, st);
}

template <int LMAX, int KIND>
void tps_kind(const TpArgs& a, int nr, hipStream_t st) {
  switch (a.C) {
    case 64: return sender_launch<LMAX, KIND, 1>(a, nr, st);
    case 128: return sender_launch<LMAX, KIND, 2>(a, nr, st);
    case 256: return sender_launch<LMAX, KIND, 4>(a, nr, st);
    default: throw Error(E3MI_EUNSUPPORTED, "scalar-output tensor product: channels must be 64, 128 or 256");
  }
}

}  // namespace

bool tps_supported(const TpArgs& a) {
  return (a.kind == kLast || a.kind == kFirstLast) && (a.C == 64 || a.C == 128 || a.C == 256) &&
         (a.lmax == 2 || a.lmax == 3);
}

void launch_tps_sender(const TpArgs& a, hipStream_t st) {
  if (a.N == 0) return;
  E3MI_REQUIRE(tps_supported(a), E3MI_EUNSUPPORTED, "sender-side adjoint: unsupported layer");
  E3MI_REQUIRE(a.rev, E3MI_EINVAL, "sender-side adjoint: needs the reverse edges");
  // senders i0 .. i0 + nr - 1: their rows hold the chunk's R and dR
  const int nr = a.n_recv > 0 ? a.n_recv : a.N;
  if (a.n_recv == 0 && (a.i0 != 0 || a.e_first != 0))
    throw Error(E3MI_EINVAL, "tensor product: receiver offset without a receiver count");
  if (a.lmax == 2) {
    if (a.kind == kLast) return tps_kind<2, kLast>(a, nr, st);
    return tps_kind<2, kFirstLast>(a, nr, st);
  }
  if (a.kind == kLast) return tps_kind<3, kLast>(a, nr, st);
  return tps_kind<3, kFirstLast>(a, nr, st);
}

}  // namespace e3mi
