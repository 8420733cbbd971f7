// Compile-time description of the Clebsch-Gordan paths one interaction layer
// uses, built from the generated coefficient table (cg_tables.inc), plus a
// static_for that unrolls loops with constant indices so that every
// coefficient becomes an immediate and every accumulator a register.
#pragma once

#include <type_traits>
#include <utility>

#include "cg_tables.inc"

namespace e3mi {

using namespace e3mi_cg;

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Layer kinds: which orders enter (l1) and leave (l3) the layer.
enum LayerKind : int {
  kFirst = 0,      // scalar input (the embedding), all output orders
  kFull = 1,       // all input orders, all output orders
  kLast = 2,       // all input orders, scalar output only (the only part the energy reads)
  kFirstLast = 3,  // a single layer: scalar in, scalar out
};

template <int LMAX, int KIND>
struct PathSet {
  static constexpr int L1MAX = (KIND == kFirst || KIND == kFirstLast) ? 0 : LMAX;
  static constexpr int L3MAX = (KIND == kLast || KIND == kFirstLast) ? 0 : LMAX;
  static constexpr int NY = (LMAX + 1) * (LMAX + 1);      // harmonics used
  static constexpr int NIN = (L1MAX + 1) * (L1MAX + 1);   // input components read
  static constexpr int NCOUT = (L3MAX + 1) * (L3MAX + 1); // output components of h~
  static constexpr bool keep(int g) { return kL1[g] <= L1MAX && kL2[g] <= LMAX && kL3[g] <= L3MAX; }
  static constexpr int count() {
    int c = 0;
    for (int g = 0; g < kNumPaths; ++g) c += keep(g) ? 1 : 0;
    return c;
  }
  static constexpr int NP = count();
  struct Table {
    int id[NP];     // global path id
    int off[NP];    // offset of the path's (2 l3 + 1) outputs in a per-channel accumulator
    int rank[NP];   // rank among the layer's paths with the same l3
    int np_l3[4];   // paths per output order
    int nout;       // sum_p (2 l3 + 1)
  };
  static constexpr Table make() {
    Table t{};
    int c = 0, o = 0;
    for (int l = 0; l < 4; ++l) t.np_l3[l] = 0;
    for (int g = 0; g < kNumPaths; ++g)
      if (keep(g)) {
        t.id[c] = g;
        t.off[c] = o;
        t.rank[c] = t.np_l3[kL3[g]]++;
        o += 2 * kL3[g] + 1;
        ++c;
      }
    t.nout = o;
    return t;
  }
  static constexpr Table T = make();
  static constexpr int NOUT = T.nout;
};

// Element offset of A[i, p, m3, k] in the grouped layout used between the
// tensor product and the channel mix: for each output order l3 a block
// [N, 2 l3 + 1, P_l3, C], blocks consecutive in l3.
template <class PS>
__device__ __forceinline__ long a_group_base(int l3, long N, int C) {
  long b = 0;
  for (int l = 0; l < l3; ++l) b += N * (2 * l + 1) * PS::T.np_l3[l] * (long)C;
  return b;
}

}  // namespace e3mi
