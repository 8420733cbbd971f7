// MACE-style product block between the channel mix and the gate (the
// symmetric contraction of body order 2; the paper's MACE models use
// correlation 2, Appendix F). For atom i of species z and channel k:
//   B^L_k = w1[z, L, k] A~^L_k + sum_p w2[z, p, k] sum C^{l1 l2 L}_{m1 m2 M} A~^{l1}_{m1,k} A~^{l2}_{m2,k}
// over the couplings p = (l1 <= l2, L) of the Clebsch-Gordan table with
// L <= LOUT, in table order (by L, then l1, then l2). The block is
// per-channel and per-atom (no dense contraction), so it runs on the vector
// ALU with one thread per (atom, channel): loads and stores are coalesced
// over channels and the coefficients are immediates. Its adjoint:
//   dA~^L += w1 dB^L,  dA~^{l1} += w2 C dB^L A~^{l2},  dA~^{l2} += w2 C dB^L A~^{l1}.
#include "common.h"
#include "paths.h"
#include "runtime.h"

namespace e3mi {
namespace {

template <int LMAX, int LOUT>
struct ProductSet {
  static constexpr int NA = (LMAX + 1) * (LMAX + 1);  // components of A~
  static constexpr int NB = (LOUT + 1) * (LOUT + 1);  // components of B
  static constexpr bool keep(int g) { return kL1[g] <= kL2[g] && kL2[g] <= LMAX && kL3[g] <= LOUT; }
  static constexpr int count() {
    int c = 0;
    for (int g = 0; g < kNumPaths; ++g) c += keep(g) ? 1 : 0;
    return c;
  }
  static constexpr int NP = count();
  struct Table {
    int id[NP];
  };
  static constexpr Table make() {
    Table t{};
    int c = 0;
    for (int g = 0; g < kNumPaths; ++g)
      if (keep(g)) t.id[c++] = g;
    return t;
  }
  static constexpr Table T = make();
};

template <int LMAX, int LOUT>
__global__ void __launch_bounds__(256) k_product_fwd(const float* __restrict__ at, const int* __restrict__ species,
                                                     const float* __restrict__ w1, const float* __restrict__ w2,
                                                     int N, int lg_c, float* __restrict__ B) {
  using PS = ProductSet<LMAX, LOUT>;
  const int C = 1 << lg_c;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= ((long)N << lg_c)) return;
  const int i = (int)(e >> lg_c), k = (int)(e & (C - 1));
  const int z = species[i];
  float a[PS::NA];
#pragma unroll
  for (int q = 0; q < PS::NA; ++q) a[q] = at[((long)i * PS::NA + q) * C + k];
  const float* w1z = w1 + (long)z * (LOUT + 1) * C + k;
  const float* w2z = w2 + (long)z * PS::NP * C + k;
  float b[PS::NB];
#pragma unroll
  for (int L = 0; L <= LOUT; ++L) {
    const float wl = w1z[L * C];
#pragma unroll
    for (int m = 0; m < 2 * L + 1; ++m) b[L * L + m] = wl * a[L * L + m];
  }
  static_for<PS::NP>([&](auto p) {
    constexpr int g = PS::T.id[p];
    constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
    constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
    float t[2 * l3 + 1];
#pragma unroll
    for (int m = 0; m < 2 * l3 + 1; ++m) t[m] = 0.0f;
    static_for<nz>([&](auto zz) {
      constexpr int q = z0 + zz;
      t[kM3[q]] += kC[q] * (a[l1 * l1 + kM1[q]] * a[l2 * l2 + kM2[q]]);
    });
    const float wp = w2z[(int)p * C];
#pragma unroll
    for (int m = 0; m < 2 * l3 + 1; ++m) b[l3 * l3 + m] += wp * t[m];
  });
#pragma unroll
  for (int q = 0; q < PS::NB; ++q) B[((long)i * PS::NB + q) * C + k] = b[q];
}

template <int LMAX, int LOUT>
__global__ void __launch_bounds__(256) k_product_bwd(const float* __restrict__ at, const int* __restrict__ species,
                                                     const float* __restrict__ w1, const float* __restrict__ w2,
                                                     const float* __restrict__ dB, int N, int lg_c,
                                                     float* __restrict__ dat) {
  using PS = ProductSet<LMAX, LOUT>;
  const int C = 1 << lg_c;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= ((long)N << lg_c)) return;
  const int i = (int)(e >> lg_c), k = (int)(e & (C - 1));
  const int z = species[i];
  float a[PS::NA], da[PS::NA], db[PS::NB];
#pragma unroll
  for (int q = 0; q < PS::NA; ++q) {
    a[q] = at[((long)i * PS::NA + q) * C + k];
    da[q] = 0.0f;
  }
#pragma unroll
  for (int q = 0; q < PS::NB; ++q) db[q] = dB[((long)i * PS::NB + q) * C + k];
  const float* w1z = w1 + (long)z * (LOUT + 1) * C + k;
  const float* w2z = w2 + (long)z * PS::NP * C + k;
#pragma unroll
  for (int L = 0; L <= LOUT; ++L) {
    const float wl = w1z[L * C];
#pragma unroll
    for (int m = 0; m < 2 * L + 1; ++m) da[L * L + m] = wl * db[L * L + m];
  }
  static_for<PS::NP>([&](auto p) {
    constexpr int g = PS::T.id[p];
    constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
    constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
    const float wp = w2z[(int)p * C];
    float s[2 * l3 + 1];
#pragma unroll
    for (int m = 0; m < 2 * l3 + 1; ++m) s[m] = wp * db[l3 * l3 + m];
    static_for<nz>([&](auto zz) {
      constexpr int q = z0 + zz;
      const float c = kC[q] * s[kM3[q]];
      da[l1 * l1 + kM1[q]] += c * a[l2 * l2 + kM2[q]];
      da[l2 * l2 + kM2[q]] += c * a[l1 * l1 + kM1[q]];
    });
  });
#pragma unroll
  for (int q = 0; q < PS::NA; ++q) dat[((long)i * PS::NA + q) * C + k] = da[q];
}

// Tangent of the block along A~_dot (second-order pass):
//   B_dot^L = w1 A~_dot^L + sum_p w2_p sum C (A~_dot^{l1} A~^{l2} + A~^{l1} A~_dot^{l2}).
template <int LMAX, int LOUT>
__global__ void __launch_bounds__(256) k_product_jvp(const float* __restrict__ at, const float* __restrict__ atd,
                                                     const int* __restrict__ species, const float* __restrict__ w1,
                                                     const float* __restrict__ w2, int N, int lg_c,
                                                     float* __restrict__ Bd) {
  using PS = ProductSet<LMAX, LOUT>;
  const int C = 1 << lg_c;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= ((long)N << lg_c)) return;
  const int i = (int)(e >> lg_c), k = (int)(e & (C - 1));
  const int z = species[i];
  float a[PS::NA], ad[PS::NA];
#pragma unroll
  for (int q = 0; q < PS::NA; ++q) {
    a[q] = at[((long)i * PS::NA + q) * C + k];
    ad[q] = atd[((long)i * PS::NA + q) * C + k];
  }
  const float* w1z = w1 + (long)z * (LOUT + 1) * C + k;
  const float* w2z = w2 + (long)z * PS::NP * C + k;
  float b[PS::NB];
#pragma unroll
  for (int L = 0; L <= LOUT; ++L) {
    const float wl = w1z[L * C];
#pragma unroll
    for (int m = 0; m < 2 * L + 1; ++m) b[L * L + m] = wl * ad[L * L + m];
  }
  static_for<PS::NP>([&](auto p) {
    constexpr int g = PS::T.id[p];
    constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
    constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
    float t[2 * l3 + 1];
#pragma unroll
    for (int m = 0; m < 2 * l3 + 1; ++m) t[m] = 0.0f;
    static_for<nz>([&](auto zz) {
      constexpr int q = z0 + zz;
      const int q1 = l1 * l1 + kM1[q], q2 = l2 * l2 + kM2[q];
      t[kM3[q]] += kC[q] * (ad[q1] * a[q2] + a[q1] * ad[q2]);
    });
    const float wp = w2z[(int)p * C];
#pragma unroll
    for (int m = 0; m < 2 * l3 + 1; ++m) b[l3 * l3 + m] += wp * t[m];
  });
#pragma unroll
  for (int q = 0; q < PS::NB; ++q) Bd[((long)i * PS::NB + q) * C + k] = b[q];
}

// Reverse of (B, B_dot) = (f(A~), f'(A~) A~_dot) for adjoints Bb of B and Bc
// of B_dot, f the block above:
//   A~_bar     = f'(A~)^T Bb + (d/dA~ of f'(A~) A~_dot)^T Bc,
//   A~_dot_bar = f'(A~)^T Bc,
// where the second term of A~_bar is the bilinear part alone: w2 C Bc^L
// A~_dot^{l2} into component l1 and w2 C Bc^L A~_dot^{l1} into l2. With DW,
// atom i's share of the weight gradients:
//   d/dw1[L]  = sum_m (Bb^L_m A~^L_m + Bc^L_m A~_dot^L_m),
//   d/dw2[p]  = sum_M (Bb^L_M T_p,M + Bc^L_M T_dot_p,M), T_p = sum C A~^{l1} A~^{l2}.
template <int LMAX, int LOUT, bool DW>
__global__ void __launch_bounds__(256) k_product_dual_bwd(const float* __restrict__ at, const float* __restrict__ atd,
                                                          const int* __restrict__ species,
                                                          const float* __restrict__ w1, const float* __restrict__ w2,
                                                          const float* __restrict__ Bb, const float* __restrict__ Bc,
                                                          int N, int lg_c, float* __restrict__ atb,
                                                          float* __restrict__ atc, float* __restrict__ dw) {
  using PS = ProductSet<LMAX, LOUT>;
  const int C = 1 << lg_c;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= ((long)N << lg_c)) return;
  const int i = (int)(e >> lg_c), k = (int)(e & (C - 1));
  const int z = species[i];
  float a[PS::NA], ad[PS::NA], ga[PS::NA], gc[PS::NA], bb[PS::NB], bc[PS::NB];
#pragma unroll
  for (int q = 0; q < PS::NA; ++q) {
    a[q] = at[((long)i * PS::NA + q) * C + k];
    ad[q] = atd[((long)i * PS::NA + q) * C + k];
    ga[q] = 0.0f;
    gc[q] = 0.0f;
  }
#pragma unroll
  for (int q = 0; q < PS::NB; ++q) {
    bb[q] = Bb[((long)i * PS::NB + q) * C + k];
    bc[q] = Bc[((long)i * PS::NB + q) * C + k];
  }
  const float* w1z = w1 + (long)z * (LOUT + 1) * C + k;
  const float* w2z = w2 + (long)z * PS::NP * C + k;
  float* dwi = DW ? dw + (long)i * (LOUT + 1 + PS::NP) * C + k : nullptr;
#pragma unroll
  for (int L = 0; L <= LOUT; ++L) {
    const float wl = w1z[L * C];
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < 2 * L + 1; ++m) {
      const int q = L * L + m;
      ga[q] = wl * bb[q];
      gc[q] = wl * bc[q];
      s += bb[q] * a[q] + bc[q] * ad[q];
    }
    if constexpr (DW) dwi[L * C] = s;
  }
  static_for<PS::NP>([&](auto p) {
    constexpr int g = PS::T.id[p];
    constexpr int l1 = kL1[g], l2 = kL2[g], l3 = kL3[g];
    constexpr int z0 = kNzBegin[g], nz = kNzBegin[g + 1] - kNzBegin[g];
    const float wp = w2z[(int)p * C];
    float s = 0.0f;
    static_for<nz>([&](auto zz) {
      constexpr int q = z0 + zz;
      const int q1 = l1 * l1 + kM1[q], q2 = l2 * l2 + kM2[q], q3 = l3 * l3 + kM3[q];
      const float cb = kC[q] * wp * bb[q3], cc = kC[q] * wp * bc[q3];
      ga[q1] += cb * a[q2] + cc * ad[q2];
      ga[q2] += cb * a[q1] + cc * ad[q1];
      gc[q1] += cc * a[q2];
      gc[q2] += cc * a[q1];
      if constexpr (DW) s += kC[q] * (bb[q3] * (a[q1] * a[q2]) + bc[q3] * (ad[q1] * a[q2] + a[q1] * ad[q2]));
    });
    if constexpr (DW) dwi[(LOUT + 1 + (int)p) * C] = s;
  });
#pragma unroll
  for (int q = 0; q < PS::NA; ++q) {
    atb[((long)i * PS::NA + q) * C + k] = ga[q];
    atc[((long)i * PS::NA + q) * C + k] = gc[q];
  }
}

int log2_channels(int C) {
  int lg = 0;
  while ((1 << lg) < C) ++lg;
  if ((1 << lg) != C) throw Error(E3MI_EUNSUPPORTED, "product block: channels must be a power of two");
  return lg;
}

template <int LMAX, int LOUT>
void product_l(bool fwd, const ProductArgs& p, int lg, int grid, hipStream_t st) {
  if (fwd)
    k_product_fwd<LMAX, LOUT><<<grid, 256, 0, st>>>(p.at, p.species, p.w1, p.w2, p.N, lg, p.B);
  else
    k_product_bwd<LMAX, LOUT><<<grid, 256, 0, st>>>(p.at, p.species, p.w1, p.w2, p.dB, p.N, lg, p.dat);
}

template <int LMAX, int LOUT>
void product_dual_l(bool jvp, const ProductArgs& p, int lg, int grid, hipStream_t st) {
  if (jvp)
    k_product_jvp<LMAX, LOUT><<<grid, 256, 0, st>>>(p.at, p.atd, p.species, p.w1, p.w2, p.N, lg, p.Bd);
  else if (p.dw)
    k_product_dual_bwd<LMAX, LOUT, true><<<grid, 256, 0, st>>>(p.at, p.atd, p.species, p.w1, p.w2, p.Bb, p.Bc, p.N,
                                                               lg, p.atb, p.atc, p.dw);
  else
    k_product_dual_bwd<LMAX, LOUT, false><<<grid, 256, 0, st>>>(p.at, p.atd, p.species, p.w1, p.w2, p.Bb, p.Bc,
                                                                p.N, lg, p.atb, p.atc, nullptr);
}

template <class F>
void product_dispatch(const ProductArgs& p, F&& f) {
  if (p.lmax == 3 && p.lout == 3)
    f(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{});
  else if (p.lmax == 3 && p.lout == 0)
    f(std::integral_constant<int, 3>{}, std::integral_constant<int, 0>{});
  else if (p.lmax == 2 && p.lout == 2)
    f(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
  else if (p.lmax == 2 && p.lout == 0)
    f(std::integral_constant<int, 2>{}, std::integral_constant<int, 0>{});
  else
    throw Error(E3MI_EUNSUPPORTED, "product block: unsupported (lmax, output order)");
}

}  // namespace

int product_pair_count(int lmax, int lout) {
  int c = 0;
  for (int g = 0; g < kNumPaths; ++g) c += (kL1[g] <= kL2[g] && kL2[g] <= lmax && kL3[g] <= lout) ? 1 : 0;
  return c;
}

void launch_product(bool fwd, const ProductArgs& p, hipStream_t st) {
  if (p.N == 0) return;
  const int lg = log2_channels(p.C);
  const long n = (long)p.N * p.C;
  const int grid = (int)((n + 255) / 256);
  product_dispatch(p, [&](auto lm, auto lo) { product_l<lm, lo>(fwd, p, lg, grid, st); });
}

void launch_product_jvp(const ProductArgs& p, hipStream_t st) {
  if (p.N == 0) return;
  E3MI_REQUIRE(p.at && p.atd && p.Bd, E3MI_EINVAL, "product block tangent: null argument");
  const int lg = log2_channels(p.C);
  const int grid = (int)(((long)p.N * p.C + 255) / 256);
  product_dispatch(p, [&](auto lm, auto lo) { product_dual_l<lm, lo>(true, p, lg, grid, st); });
}

void launch_product_dual_bwd(const ProductArgs& p, hipStream_t st) {
  if (p.N == 0) return;
  E3MI_REQUIRE(p.at && p.atd && p.Bb && p.Bc && p.atb && p.atc, E3MI_EINVAL,
               "product block second-order adjoint: null argument");
  const int lg = log2_channels(p.C);
  const int grid = (int)(((long)p.N * p.C + 255) / 256);
  product_dispatch(p, [&](auto lm, auto lo) { product_dual_l<lm, lo>(false, p, lg, grid, st); });
}

}  // namespace e3mi
