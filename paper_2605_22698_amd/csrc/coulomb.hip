// Long-range electrostatics of open structures (Section 5.1, the
// charge-correction and long-range-interaction equations):
//   raw charges   q_i = w_q . h_i[0] + b_q[z_i]      (written by the readout)
//   correction    q~_i = q_i - (sum_{j in s} q_j - Q_s) / N_s
//   energy        E_i += 1/2 k_e q~_i phi_i,   phi_i = sum_{j != i in s} q~_j kappa(r_ij)
//   kappa(r) = 1/chi(r) = f(r/r0) / sqrt(r^2 + 1) + (1 - f(r/r0)) / r,
//   f(x) = 1 - 6x^5 + 15x^4 - 10x^3 for x < 1, else 0   (PhysNet's soft core)
// and its adjoint:
//   F_i  += k_e q~_i sum_j q~_j kappa'(r_ij) (r_j - r_i) / r_ij
//   dE/dq_i = k_e (phi_i - mean_{k in s} phi_k)          (through the correction)
//   dE/dh_i[0] += dE/dq_i w_q                            (into the readout's adjoint)
// All pairs of a structure, no cutoff: O(N_s^2) per structure. One workgroup
// per tile of 64 receivers of one structure, its waves splitting the senders
// (more waves for larger structures, to fill the chip); sender positions and charges are
// staged through LDS, so each sender is read from HBM once per tile. Pairs
// beyond the soft-core radius (the soft-core weight is 0 there) take the
// plain 1/r form whenever no lane of the wave has a closer pair. Positions are taken relative to the structure's first
// atom in FP64 before rounding to FP32; the potential sum is kept in FP64.
#include "common.h"
#include "runtime.h"

namespace e3mi {
namespace {

constexpr float kCoulombK = 14.399645478425668f;  // e^2 / (4 pi eps0) in eV angstrom

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

constexpr int kRedThreads = 1024;

// One block per structure: q~ = q - (sum q - Q_s) / N_s.
__global__ void __launch_bounds__(kRedThreads) k_charge_fix(const float* __restrict__ q_raw,
                                                            const int64_t* __restrict__ off,
                                                            const double* __restrict__ Q, float* __restrict__ q) {
  __shared__ double red[kRedThreads];
  const int s = blockIdx.x;
  const int64_t a = off[s], b = off[s + 1];
  if (b == a) return;
  double acc = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += kRedThreads) acc += (double)q_raw[i];
  const double tot = block_sum<kRedThreads>(acc, red);
  const double shift = (tot - Q[s]) / (double)(b - a);
  for (int64_t i = a + threadIdx.x; i < b; i += kRedThreads) q[i] = (float)((double)q_raw[i] - shift);
}

// The hardware reciprocal square root (about 1 ulp). Its arguments here are
// squared distances of distinct atoms, far from the denormal range that
// rsqrtf guards with extra scaling instructions.
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Pair terms for squared distance r2 (rinv = 1/r) and sender charge qj: the
// potential qj kappa(r) and the force factor qj kappa'(r) / r. FULL takes the
// soft-core form; otherwise kappa = 1/r, exact for r >= r0.
template <bool FULL>
__device__ __forceinline__ void pair_terms(float r2, float rinv, float qj, float inv_r0, float& pot, float& fr) {
  if (!FULL) {
    pot = qj * rinv;
    fr = -pot * rinv * rinv;
    return;
  }
  const float r = r2 * rinv;
  const float x = fminf(r * inv_r0, 1.0f);
  const float om = 1.0f - x;
  const float f = 1.0f + x * x * x * (-10.0f + x * (15.0f - 6.0f * x));
  const float df = -30.0f * inv_r0 * x * x * om * om;
  const float sr = rsq(r2 + 1.0f);
  const float kap = rinv + f * (sr - rinv);
  const float dkap = df * (sr - rinv) - f * r * sr * sr * sr - (1.0f - f) * rinv * rinv;
  pot = qj * kap;
  fr = qj * dkap * rinv;
}

// Senders xw[0 .. m4) against this lane's receiver (xi, yi, zi), four at a
// time; slot self_slot (-1: none) is the receiver itself and carries no term.
// (A separate loop for the one chunk that holds the receivers measured slower
// than the per-pair select.)
__device__ __forceinline__ void sender_block(const float4* xw, int m4, int self_slot, float xi, float yi, float zi,
                                             float inv_r0, float r02, float& ps, float& fx, float& fy, float& fz) {
  for (int k = 0; k < m4; k += 4) {
    float dx[4], dy[4], dz[4], r2[4], qj[4];
    bool near = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float4 sj = xw[k + u];
      dx[u] = sj.x - xi;
      dy[u] = sj.y - yi;
      dz[u] = sj.z - zi;
      const float d2 = dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u];
      const bool self = k + u == self_slot;
      r2[u] = self ? 1.0f : d2;
      qj[u] = self ? 0.0f : sj.w;
      near |= !self && d2 < r02;
    }
    float pk[4], fr[4];
    if (__ballot(near)) {
#pragma unroll
      for (int u = 0; u < 4; ++u) pair_terms<true>(r2[u], rsq(r2[u]), qj[u], inv_r0, pk[u], fr[u]);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) pair_terms<false>(r2[u], rsq(r2[u]), qj[u], inv_r0, pk[u], fr[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ps += pk[u];
      fx += fr[u] * dx[u];
      fy += fr[u] * dy[u];
      fz += fr[u] * dz[u];
    }
  }
}

// Tile t covers receivers tiles[t].y .. +63 of structure tiles[t].x. The
// structure's size alone fixes how many waves split its senders (nw: enough
// to cover it in one round, at most NW), so a structure gets the same sums
// alone and packed with others; waves beyond nw only join the barriers. Each
// round stages 64 nw senders in LDS (one per thread; past the structure's end
// a zero charge far away) and wave w takes senders 64w .. 64w+63 of the
// round, four at a time, with one vote per four on whether any lane has a
// pair inside r0. The partial sums are added in wave order at the end.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_coulomb(const int2* __restrict__ tiles, const int64_t* __restrict__ off,
                                                     const double* __restrict__ pos, const float* __restrict__ q,
                                                     float inv_r0, double* __restrict__ e_atom,
                                                     float* __restrict__ pot, float* __restrict__ fc) {
  constexpr int NT = 64 * NW;
  __shared__ float4 xs[NT];
  __shared__ double red_phi[NW][64];
  __shared__ float red_f[NW][3][64];
  const int2 tl = tiles[blockIdx.x];
  const int64_t a = off[tl.x], b = off[tl.x + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)tl.y + lane;
  const bool live = i < b;
  const double ox = pos[3 * a], oy = pos[3 * a + 1], oz = pos[3 * a + 2];
  float xi = 1e18f, yi = 1e18f, zi = 1e18f;  // an idle lane sits far from every sender
  if (live) {
    xi = (float)(pos[3 * i] - ox);
    yi = (float)(pos[3 * i + 1] - oy);
    zi = (float)(pos[3 * i + 2] - oz);
  }
  const float r02 = 1.0f / (inv_r0 * inv_r0);
  int nw = 1;
  while (nw < NW && 64 * (int64_t)nw < b - a) nw *= 2;
  const int R = 64 * nw;  // senders per round
  double phi = 0.0;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  for (int64_t j0 = a; j0 < b; j0 += R) {  // block-uniform trip count
    const int64_t j = j0 + threadIdx.x;
    float4 v = make_float4(-1e18f, -1e18f, -1e18f, 0.f);
    if (j < b && (int)threadIdx.x < R)
      v = make_float4((float)(pos[3 * j] - ox), (float)(pos[3 * j + 1] - oy), (float)(pos[3 * j + 2] - oz), q[j]);
    __syncthreads();
    xs[threadIdx.x] = v;
    __syncthreads();
    const int64_t base = j0 + 64 * w;
    const int m = w < nw ? (int)max((int64_t)0, min((int64_t)64, b - base)) : 0;
    const int m4 = (m + 3) & ~3;  // padded slots hold zero charges
    const float4* xw = xs + 64 * w;
    float ps = 0.f;
    // tiles and rounds start at multiples of 64 from the structure's first
    // atom, so a sender slot is a lane's own atom only when base is the tile
    sender_block(xw, m4, base == (int64_t)tl.y ? lane : -1, xi, yi, zi, inv_r0, r02, ps, fx, fy, fz);
    phi += (double)ps;
  }
  red_phi[w][lane] = phi;
  red_f[w][0][lane] = fx;
  red_f[w][1][lane] = fy;
  red_f[w][2][lane] = fz;
  __syncthreads();
  if (w > 0 || !live) return;
  for (int u = 1; u < nw; ++u) {
    phi += red_phi[u][lane];
    fx += red_f[u][0][lane];
    fy += red_f[u][1][lane];
    fz += red_f[u][2][lane];
  }
  const float qi = q[i];
  e_atom[i] += 0.5 * (double)kCoulombK * (double)qi * phi;
  pot[i] = (float)((double)kCoulombK * phi);
  const float c = kCoulombK * qi;
  fc[3 * i] = c * fx;
  fc[3 * i + 1] = c * fy;
  fc[3 * i + 2] = c * fz;
}

// One block per structure: the structure's mean potential.
__global__ void __launch_bounds__(kRedThreads) k_pot_mean(const int64_t* __restrict__ off,
                                                          const float* __restrict__ pot, float* __restrict__ mean) {
  __shared__ double red[kRedThreads];
  const int s = blockIdx.x;
  const int64_t a = off[s], b = off[s + 1];
  double acc = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += kRedThreads) acc += (double)pot[i];
  const double tot = block_sum<kRedThreads>(acc, red);
  if (threadIdx.x == 0) mean[s] = b > a ? (float)(tot / (double)(b - a)) : 0.0f;
}

// dh[i, k] += (pot_i - mean pot of i's structure) w_q[k], one thread per element (C = 2^lg_c).
__global__ void __launch_bounds__(256) k_coulomb_dq(const int* __restrict__ owner, const float* __restrict__ pot,
                                                    const float* __restrict__ mean, const float* __restrict__ wq,
                                                    int lg_c, long n, float* __restrict__ dh) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int i = (int)(e >> lg_c);
  const int k = (int)(e & ((1 << lg_c) - 1));
  dh[e] += (pot[i] - mean[owner[i]]) * wq[k];
}

}  // namespace

void launch_charge_fix(const float* q_raw, const int64_t* off, const double* Q, int S, float* q, hipStream_t st) {
  if (S == 0) return;
  k_charge_fix<<<S, kRedThreads, 0, st>>>(q_raw, off, Q, q);
}

void launch_coulomb(const int2* tiles, int n_tiles, int waves, const int64_t* off, const double* pos, const float* q,
                    float r0, double* e_atom, float* pot, float* fc, hipStream_t st) {
  if (n_tiles == 0) return;
  const float ir = 1.0f / r0;
  switch (waves) {
    case 1: k_coulomb<1><<<n_tiles, 64, 0, st>>>(tiles, off, pos, q, ir, e_atom, pot, fc); break;
    case 2: k_coulomb<2><<<n_tiles, 128, 0, st>>>(tiles, off, pos, q, ir, e_atom, pot, fc); break;
    case 4: k_coulomb<4><<<n_tiles, 256, 0, st>>>(tiles, off, pos, q, ir, e_atom, pot, fc); break;
    case 8: k_coulomb<8><<<n_tiles, 512, 0, st>>>(tiles, off, pos, q, ir, e_atom, pot, fc); break;
    case 16: k_coulomb<16><<<n_tiles, 1024, 0, st>>>(tiles, off, pos, q, ir, e_atom, pot, fc); break;
    default: throw Error(E3MI_EINVAL, "coulomb: waves per tile must be 1, 2, 4, 8 or 16");
  }
}

void launch_coulomb_dq(const int64_t* off, const int* owner, int S, int N, const float* pot, float* mean,
                       const float* wq, int C, float* dh, hipStream_t st) {
  if (S == 0 || N == 0) return;
  int lg = 0;
  while ((1 << lg) < C) ++lg;
  if ((1 << lg) != C) throw Error(E3MI_EUNSUPPORTED, "coulomb: channels must be a power of two");
  k_pot_mean<<<S, kRedThreads, 0, st>>>(off, pot, mean);
  const long n = (long)N * C;
  k_coulomb_dq<<<(int)((n + 255) / 256), 256, 0, st>>>(owner, pot, mean, wq, lg, n, dh);
}

}  // namespace e3mi
